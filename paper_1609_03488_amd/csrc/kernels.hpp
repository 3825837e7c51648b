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
    int kc;          // taps per LDS staging pass: min(max kpad of the launch, CONV_KC_MAX)
    // output-initialisation tiles run by workgroups ntiles.. of the same launch
    // (only when every convolution owns its output range in this direction, so
    // that the two kinds of workgroups write disjoint elements)
    const VecTile* init;
    int ninit;
    // the same outputs as tiles of the FFT engine (two windows of FFT_L - k + 1
    // outputs each); fft = 1 when every block of the launch has spectra
    const ConvTile* ftiles;
    int nftiles;
    int fft;
    // CG steps folded into an A^T launch of the FFT engine that writes every X
    // element of every instance (fold != 0; partials in part[4 b + j] of
    // workgroup b):
    //   1 (CG start): the output is h; r = h - q (and p = r when fp >= 0) is
    //     written instead of h (kinds fr, fp, fq), partials ||r||^2, ||h||^2;
    //   2 (CG products): the output is q = p + A^T A p; partials <p, q>,
    //     ||r||^2, <r, q>, ||q||^2 (kinds fr, fp), and the iteration mark
    //     fit in the instance's scalars (the role of k_cg_dot)
    int fold;
    int fr, fp, fq, fit;
    double* part;
    // FFT engine, fold = 0: pair = 1 runs a second apply of the same direction
    // in the same launch, on kinds (out2, in2, base2) with the same sigma
    int pair;
    int out2, in2, base2;
    // fold = 1: idrows = k + 1 also writes, for each identity block of A, the
    // rows of Y kind k that A p has there for p = r: (T)(scale * r), the value
    // the A launch's initialisation workgroups would write (0: none)
    int idrows;
};
// dynamic LDS bytes of the convolution kernel for a staging pass of kc taps
size_t conv_smem_bytes(int prec, int kc);
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
void launch_conv(int prec, const Tables& t, const ConvLaunch& c, int adj, int out, int in, int base,
                 double sigma, int gate, hipStream_t st);
// FP32 only: the same convolution tiles on the matrix cores (conv_mfma.hip)
void launch_conv_mfma(const Tables& t, const ConvLaunch& c, int adj, int out, int in, int base,
                      double sigma,
                      int gate, hipStream_t st);
size_t conv_mfma_smem_bytes(int kc);
// FP32 only: the same convolution by FFT (overlap-save; conv_fft.hip), and the
// conj(DFT) of k taps zero-padded to FFT_L points that it multiplies by
void launch_conv_fft(const Tables& t, const ConvLaunch& c, int adj, int out, int in, int base,
                     double sigma, int gate, hipStream_t st);
void launch_conv_spectrum(const void* w, int64_t k, void* spec, hipStream_t st);
// out += sigma * scale * a (or a^T) * in for every dense tile.
void launch_gemv(int prec, const Tables& t, const DenseLaunch& d, int adj, int out, int in,
                 double sigma, int gate, hipStream_t st);

// CG (Section IV-B listing) on (I + A^T A) z = h with kinds z, r, p, q, h.
// init: r = h - q (q = K z, or q = 0 when have_q = 0), p = r, rr = ||r||^2,
//       tol = ||h|| * max(floor, zeta / (k+1)^rate), CG active iff ||r|| > tol.
void launch_cg_init(int prec, const Tables& t, int z, int r, int p, int q, int h, int have_q,
                    double zeta, double rate, double floor, int cg_max, int gate, hipStream_t st);
// partials of <p, q>, ||r||^2, <r, q>, ||q||^2; marks iteration `it` as in progress
void launch_cg_dot(int prec, const Tables& t, int p, int q, int r, int it, int gate, hipStream_t st);
// alpha = ||r||^2 / <p, q>; z += alpha p; r -= alpha q; beta = ||r'||^2 / ||r||^2
// (from the dot partials); stop test (||r'|| <= tol or it + 1 = cg_max);
// p = r' + beta p while CG goes on.
// track = 1: also K z += alpha q and A z += alpha (A p) (carried products)
// `it`: CG iteration of the current loop (must match the preceding launch_cg_dot)
// The CG start test evaluated by the first update of a step (folded path: the
// right-hand side's partials are in Tables::spart and the first iteration's
// products ran ungated)
struct CgStart {
    double zeta, rate, floor_;
    int on;
    // 1: the update in which an instance's CG ends also does the work of
    // launch_tau_dots on the final z and A z (folded ADMM path,
    // where some update of the loop always runs)
    int tau;
    // with tau: that update also forms the cone terms of the projection that
    // follows (launch_project): relative to
    // the expansion point e = the previous step's u~_tau, every second-order
    // cone row has u_bar - v = a - (u~_tau - e) b with
    //   a = alpha z_y + (1 - alpha) u_y - v_s - alpha e g_y,   b = alpha g_y,
    // so the cone's tail norm is sum a^2 - 2 (u~_tau - e) sum a b
    // + (u~_tau - e)^2 sum b^2; the tau products go to slot 0 and the sums over
    // the tail to slots 1..3 of Tables::tpart, the head's a and b to seg_val,
    // and the first X tile's workgroup stores e and tau + kappa in its X
    // partial slots 1 and 2
    int cone;
    double alpha;
    // where the next direction p' = r' + beta p is written (-1: over p).  The
    // first CG iteration of a folded ADMM step reads p = r from r's vector
    // (the right-hand side launch does not copy it) and writes p' to XP.
    int pn = -1;
};
void launch_cg_update(int prec, const Tables& t, int z, int r, int p, int q, int it, int cg_max,
                      int gate, int track, hipStream_t st, int folded = 0, int last = 0,
                      CgStart cs = CgStart{0.0, 0.0, 0.0, 0, 0, 0, 0.0});
// (folded = 1: the partials come from the A^T launch of ConvLaunch::fold = 2;
// last = 1: the step's last CG launch of a round run from a snapshot; when CG
// would go on the instance is suspended, phase 3, for the host to run the
// round again with more launches)
// copy of the carried state of the instances on the one-launch-per-kernel path
// (InstDesc::snap); restore = 1 copies it back
void launch_snapshot(int prec, const Tables& t, int restore, hipStream_t st);

// ---- ADMM step pieces (Section V-B: subspace projection, then cone projection)
// w_y = u_y + v_s
void launch_wy(int prec, const Tables& t, int gate, hipStream_t st);
// after CG on the one-launch-per-kernel path: the partials of c^T z_x and
// b^T z_y, z_y = w_y + (carried A z) formed and not stored, and the cone terms
// of CgStart::cone (the work the update that ends CG does on the folded path)
void launch_tau_dots(int prec, const Tables& t, double alpha, hipStream_t st);
// relaxation, projection onto K, dual update of every X/Y entry: every
// workgroup forms u~_tau = (tau + kappa + c^T z_x + b^T z_y) / eta from the tau
// products' partials and the cone norms from the cone terms (CgStart::cone)
void launch_project(int prec, const Tables& t, double alpha, hipStream_t st);
// termination quantities from A u_x (in YT) and A^T u_y (in XT)
void launch_resid(int prec, const Tables& t, double eps, int max_iters, int gate, hipStream_t st);

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
// dst (rows x ld, working precision) <- src (rows x cols, row stride lds,
// FP64 when src_dtype = 0, FP32 when 1), zero pad
void launch_cast_pad(int prec, const void* src, int src_dtype, int64_t lds, int64_t rows, int64_t cols,
                     void* dst, int64_t ld, hipStream_t st);
// dst^T: dst[c * ldt + r0 + r] <- src[r * lds + c] (rows of a chunk)
void launch_cast_transpose(int prec, const void* src, int src_dtype, int64_t lds, int64_t rows,
                           int64_t cols, void* dst, int64_t ldt, int64_t r0, hipStream_t st);
// Sum of squares of a device matrix (rows x cols, row stride lda, FP64 when
// dtype = 0, FP32 when 1), in the order the host forms it for a copied block:
// each row's squares summed in column order, then the row sums in row order.
// Returns CGS_OK, CGS_EINVAL when an entry is not finite, CGS_EHIP.
int dense_frob2_device(const void* a, int dtype, int64_t rows, int64_t cols, int64_t lda, double* frob2);
// dst (FP64) <- src (working precision)
void launch_cast_back(int prec, const void* src, double* dst, int64_t n, hipStream_t st);
// out[i * NSC + j] = scalar j of instance i
void launch_gather_scalars(const InstDesc* insts, int ninst, double* out, hipStream_t st);
void launch_set_scalar(const InstDesc* insts, int inst, int slot, double v, hipStream_t st);
// BF16 copies (round to nearest even) of a working-precision FP32 matrix: hi =
// bf16(x), lo = bf16(x - hi)

// ---- fused small-instance steps (fused.hip): one workgroup per instance runs
// nsteps ADMM steps and, with check, the termination test and the exact
// recomputation of the carried warm-start products.
struct FusedArgs {
    int nsteps;
    int check;
    int refresh;     // 1: only recompute the carried A z and (I + A^T A) z, then return
    double alpha, eps, zeta, rate, floor_;
    int cg_max;
    int max_iters;
    int kc;          // taps per LDS staging pass (as ConvLaunch::kc)
    // set by launch_fused: LDS bytes of the convolution's staging area, and
    // the bytes after it that hold an instance's most used vectors
    int64_t lds_conv, lds_res;
    int64_t res_want;   // bytes those vectors of the largest instance take (0: none)
};
size_t fused_smem_bytes(int prec, int kc);
// bytes that every resident-vector candidate of an instance with n variables
// and m rows takes in LDS (16-byte aligned each)
int64_t fused_resident_bytes(int prec, int64_t n, int64_t m);
// queries the device's LDS per workgroup and lets the fused kernels take it
// (once per device, outside any stream capture); returns that limit
int fused_prepare();
void launch_fused(int prec, const Tables& t, FusedArgs fa, hipStream_t st);

// ---- batched dense applies as BF16 MFMA GEMMs (gemm.hip)
struct GemmPlan {
    int mpad;               // instances padded to the 64-row M tile
    int ntiles;             // 128-column N tiles
    int ksteps_per_split;   // 16-wide K steps per split
    int nsplit;             // K splits (partials reduced in fixed order)
    int64_t npad;
};
// W (rows x kpad FP32, row-major) -> BF16 hi / lo in the GEMM's packed operand layout
void launch_gemm_pack_w(const float* w, int64_t rows, int64_t kpad, uint16_t* hi, uint16_t* lo,
                        hipStream_t st);
// target_wgs: workgroups to aim for (K splits = target / (N tiles x M tiles), >= 1, <= 64)
GemmPlan gemm_plan(int64_t N, int64_t kpad, int ninst, int target_wgs);
constexpr int GEMM_TARGET_MAX = 1024;   // largest target the autotuner tries (sizes the partials)
size_t gemm_part_bytes(const GemmPlan& g);
// out_b += sigma * scale * W x_b for every instance b of the tables (W = A, or
// A^T when adj), W in BF16 (plus refinement products when corr); panel holds
// three mpad x kpad BF16 panels, part the split-K partials.  With init the
// packing launch also writes the output's initial value (base + identity
// blocks, as launch_apply_init) before the products are added.
void launch_gemm_apply(const Tables& tb, const DenseBlock& db, int adj, int out, int in, double sigma,
                       int gate, int corr, uint16_t* panel, size_t panel_stride, float* part,
                       int target_wgs, hipStream_t st, bool init = false, int base = -1);

}  // namespace cgs
