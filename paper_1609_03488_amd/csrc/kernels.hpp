// Launchers of the HIP kernels of the solver engine (implemented in kernels.hip).
//
// Every launcher enqueues on `st` and takes the tile tables of the current
// instance set; `prec` is 0 (FP64) or 1 (FP32) and selects the element type of
// the X/Y vectors and operator data.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace cgs {

struct ConvLaunch {
    const ConvTile* tiles;
    const ConvBlock* blocks;
    int ntiles;
};
struct DenseLaunch {
    const DenseTile* tiles;
    const DenseBlock* blocks;
    int ntiles;
};

// out[i] = base[i] (or 0) + sigma * sum over identity blocks; out/in/base are
// vector kinds; adj = 0: out is Y, in is X; adj = 1: out is X, in is Y.
void launch_apply_init(int prec, const Tables& t, int adj, int out, int in, int base,
                       double sigma, int gate, hipStream_t st);
// out += sigma * scale * conv(in) for every conv tile (adj selects A or A^T).
void launch_conv(int prec, const Tables& t, const ConvLaunch& c, int adj, int out, int in,
                 double sigma, int gate, hipStream_t st);
// out += sigma * scale * a (or a^T) * in for every dense tile.
void launch_gemv(int prec, const Tables& t, const DenseLaunch& d, int adj, int out, int in,
                 double sigma, int gate, hipStream_t st);

// CG (Section IV-B listing) on (I + A^T A) z = h with kinds z, r, p, q, h.
// init: r = h - q (q = K z, or q = 0 when have_q = 0), p = r, rr = ||r||^2,
//       tol = ||h|| * max(floor, zeta / (k+1)^rate), CG active iff ||r|| > tol.
void launch_cg_init(int prec, const Tables& t, int z, int r, int p, int q, int h, int have_q,
                    double zeta, double rate, double floor, int cg_max, int gate, hipStream_t st);
// alpha = rr / <p, q>
void launch_cg_dot(int prec, const Tables& t, int p, int q, int gate, hipStream_t st);
// z += alpha p; r -= alpha q; rr' = ||r||^2; beta = rr'/rr; stop test
void launch_cg_update(int prec, const Tables& t, int z, int r, int p, int q, int cg_max,
                      int gate, hipStream_t st);
// p = r + beta p
void launch_cg_dir(int prec, const Tables& t, int r, int p, int gate, hipStream_t st);

// ---- ADMM step pieces (Section V-B: subspace projection, then cone projection)
// w_y = u_y + v_s
void launch_wy(int prec, const Tables& t, int gate, hipStream_t st);
// u~_tau = (tau + kappa + c^T z_x + b^T z_y) / eta, then tau, kappa updates
void launch_tau_dots(int prec, const Tables& t, double alpha, hipStream_t st);
// head value and tail sum of squares of (u_bar_y - v_s) per second-order cone
void launch_soc_prep(int prec, const Tables& t, double alpha, hipStream_t st);
// relaxation, projection onto K, dual update of every X/Y entry
void launch_project(int prec, const Tables& t, double alpha, hipStream_t st);
// termination quantities from A u_x (in YT) and A^T u_y (in XT)
void launch_resid(int prec, const Tables& t, double eps, int max_iters, hipStream_t st);

// ---- setup
// u = v = (0,0,1), z = g = 0, scalars cleared; only >= 0 restricts to one instance
void launch_reset(int prec, const Tables& t, int only, hipStream_t st);
void launch_norms(int prec, const Tables& t, int gate, hipStream_t st);  // ||b||, ||c||
void launch_eta(int prec, const Tables& t, hipStream_t st);            // eta, phase -> 1
void launch_fill(int prec, const Tables& t, int is_y, int kind, double v, int gate,
                 hipStream_t st);
void launch_copy(int prec, const Tables& t, int is_y, int dst, int src, int gate, hipStream_t st);
// point extraction: out64 = vec / tau (kind of vector chosen by `what`)
//   what: 0 x = u_x/tau, 1 y = u_y/tau, 2 s = v_s/tau, 3 raw u_x, 4 raw u_y, 5 raw v_s
//   with certificates: status INFEASIBLE scales y by 1/(-b^T u_y); UNBOUNDED
//   scales x, s by 1/(-c^T u_x).
void launch_extract(int prec, const InstDesc* inst_dev, int inst, int what, int64_t off,
                    int64_t len, double* out64, hipStream_t st);
// generic conversion of a contiguous FP64 buffer into the working precision
void launch_cast(int prec, const double* src, void* dst, int64_t n, hipStream_t st);
// dst (rows x ld, working precision) <- src (rows x cols FP64, row-major), zero pad
void launch_cast_pad(int prec, const double* src, int64_t rows, int64_t cols, void* dst,
                     int64_t ld, hipStream_t st);
// dst^T: dst[c * ldt + r0 + r] <- src[r * cols + c] (rows of a chunk)
void launch_cast_transpose(int prec, const double* src, int64_t rows, int64_t cols, void* dst,
                           int64_t ldt, int64_t r0, hipStream_t st);
// dst (FP64) <- src (working precision)
void launch_cast_back(int prec, const void* src, double* dst, int64_t n, hipStream_t st);
// out[i * NSC + j] = scalar j of instance i
void launch_gather_scalars(const InstDesc* insts, int ninst, double* out, hipStream_t st);
void launch_set_scalar(const InstDesc* insts, int inst, int slot, double v, hipStream_t st);
// BF16 copies (round to nearest even) of a working-precision FP32 matrix
void launch_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t st);

}  // namespace cgs
