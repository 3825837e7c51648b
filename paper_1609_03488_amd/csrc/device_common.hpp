// Device helpers shared by the HIP sources of the engine.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.hpp"

namespace cgs {

#define DEVI __device__ __forceinline__

// Pointers into instance regions and operator data are loaded from tables, so
// the compiler cannot infer their address space; they are declared global
// (address space 1) to get global (not flat) memory instructions.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- helpers
template <typename T>
DEVI gptr<T> xvec(const InstDesc& d, int k) {
    return (gptr<T>)(d.base + REGION_HDR) + (int64_t)k * d.nxs;
}
template <typename T>
DEVI gptr<T> yvec(const InstDesc& d, int k) {
    return (gptr<T>)(d.base + REGION_HDR) + (int64_t)NXV * d.nxs + (int64_t)k * d.nys;
}
DEVI gptr<double> scal(const InstDesc& d) { return (gptr<double>)d.base; }
DEVI int* counters(const InstDesc& d) { return reinterpret_cast<int*>(d.base + NSC * 8); }

DEVI bool gate_ok(gptr<const double> sc, int gate) {
    // the three flags are loaded together (short-circuit tests would issue
    // each load only after the previous one returned)
    const double act = sc[SC_ACTIVE], ph = sc[SC_PHASE], cg = sc[SC_CGACT];
    const bool on = act != 0.0;
    switch (gate) {
        case G_ALL: return true;
        case G_SETUP: return on & (ph == 0.0);
        case G_SETUP_CG: return on & (ph == 0.0) & (cg != 0.0);
        case G_ADMM:
        case G_CHECK: return on & (ph == 1.0);
        case G_ADMM_CG: return on & (ph == 1.0) & (cg != 0.0);
        case G_ANY_CG: return cg != 0.0;
        case G_CHECK_ANY: return on & (ph >= 1.0);
        default: return false;
    }
}

DEVI double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup in a fixed order; the result is valid in thread 0.
template <int NT>
DEVI double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) r += sh[i];
    }
    return r;
}

// Four sums over the workgroup in a fixed order, returned to every thread
// (sh: 4 * NT / 64 doubles).
template <int NT>
DEVI void block_sum4(double (&s)[4], double* sh) {
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = wave_sum(s[j]);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) sh[j * (NT / 64) + w] = s[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) r += sh[j * (NT / 64) + i];
        s[j] = r;
    }
    __syncthreads();
}

// N sums at once, each in the order of block_sum4 (sh: N * NT / 64 doubles):
// one barrier pair for all of them.
template <int NT, int N>
DEVI void block_sumN(double (&s)[N], double* sh) {
#pragma unroll
    for (int j = 0; j < N; ++j) s[j] = wave_sum(s[j]);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) sh[j * (NT / 64) + w] = s[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) r += sh[j * (NT / 64) + i];
        s[j] = r;
    }
    __syncthreads();
}

// A thread's share of a fixed-order sum of p[stride i], i in [t0, t1): the
// elements t0 + threadIdx.x + NT r in increasing r, loaded U at a time so that
// U loads are in flight together (one at a time, each load of the loop would
// wait for the previous one's add).  An index past t1 loads p[stride t0] and
// is not added.
template <int NT, int U>
DEVI double thread_sum(const double* p, int64_t t0, int64_t t1, int64_t stride) {
    double s = 0.0;
    for (int64_t b = t0; b < t1; b += (int64_t)NT * U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = b + (int64_t)u * NT + threadIdx.x;
            v[u] = p[stride * (i < t1 ? i : t0)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (b + (int64_t)u * NT + threadIdx.x < t1) s += v[u];
    }
    return s;
}

// Fixed-order sum of partial slot j over tiles [t0, t1) (partials of the
// previous kernel: the kernel boundary makes them visible).
template <int NT>
DEVI double sum_parts(const double* part, int t0, int t1, int j, double* sh) {
    const double s = thread_sum<NT, 4>(part + j, t0, t1, 4);
    return block_sum<NT>(s, sh);
}

// All four X-tile partial slots of the instance at once (sh: 4 * VEC_NT / 64).
DEVI void inst_xsum4(const Tables& tb, const InstDesc& d, double (&s)[4], double* sh) {
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = thread_sum<VEC_NT, 4>(tb.xpart + j, d.xt0, d.xt1, 4);
    block_sum4<VEC_NT>(s, sh);
}

// The same over the partials of a CG step folded into the instance's A^T
// convolution launch (Tables::cpart): its transform workgroups, then its
// initialisation ones; with start, also slots 0 and 1 of the right-hand side
// launch's partials (Tables::spart: ||r||^2, ||h||^2 of the CG start), all
// loaded in the same pass (sh: 12 * VEC_NT / 64 doubles).
DEVI void inst_csum4(const Tables& tb, const InstDesc& d, double (&s)[4], bool start, double& h0, double& h1,
                     double* sh) {
    double a[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) a[j] = 0.0;
    // each thread's records of a range, U at a time, loaded before any is
    // added (a record past the range's end loads its first one, not added)
    auto range = [&](int lo, int hi, double* acc) {
        constexpr int U = 2;
        for (int b0 = lo; b0 < hi; b0 += U * VEC_NT) {
            f64x2 c[U][2], q[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = b0 + u * VEC_NT + (int)threadIdx.x;
                const int k = i < hi ? i : lo;
                const f64x2* pc = reinterpret_cast<const f64x2*>(tb.cpart + 4 * (int64_t)k);
                c[u][0] = pc[0];
                c[u][1] = pc[1];
                if (start) q[u] = *reinterpret_cast<const f64x2*>(tb.spart + 4 * (int64_t)k);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (b0 + u * VEC_NT + (int)threadIdx.x >= hi) continue;
                acc[0] += c[u][0][0];
                acc[1] += c[u][0][1];
                acc[2] += c[u][1][0];
                acc[3] += c[u][1][1];
                if (start) {
                    acc[4] += q[u][0];
                    acc[5] += q[u][1];
                }
            }
        }
    };
    range(d.cp0, d.cp1, a);
    range(d.ip0, d.ip1, a + 6);
    block_sumN<VEC_NT, 12>(a, sh);
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = a[j] + a[6 + j];
    h0 = a[4] + a[10];
    h1 = a[5] + a[11];
}

// CG stop threshold at ADMM step k (k = 0 in the setup solve):
// ||h|| max(floor, zeta / (k+1)^rate)
DEVI double cg_tolerance(double k, double hh, double zeta, double rate, double floor_) {
    double rel = zeta > 0.0 ? zeta / pow(k + 1.0, rate) : 0.0;
    rel = rel > floor_ ? rel : floor_;
    return sqrt(hh) * rel;
}

// Tile of a kernel that walks the X tiles and then the Y tiles.
struct XYTile {
    VecTile t;
    bool is_y;
    int index;   // index in its own table
};
DEVI XYTile xy_tile(const Tables& tb) {
    XYTile r;
    const int b = blockIdx.x;
    if (b < tb.nx_tiles) {
        r.t = tb.xt[b];
        r.is_y = false;
        r.index = b;
    } else {
        r.t = tb.yt[b - tb.nx_tiles];
        r.is_y = true;
        r.index = b - tb.nx_tiles;
    }
    return r;
}

// 16-byte vector access helpers (native clang vector types: f32x4, f64x2 above)
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = f32x4; static constexpr int W = 4; };
template <> struct Vec16<double> { using type = f64x2; static constexpr int W = 2; };

template <typename T>
DEVI void vec_get(const typename Vec16<T>::type& v, T* o) {
#pragma unroll
    for (int e = 0; e < Vec16<T>::W; ++e) o[e] = v[e];
}

// ---------------------------------------------------------------- vector chunks
// A thread's elements of a vector tile [lo, hi): NCH chunks of four
// consecutive elements, chunk j starting at c0 + 4 (threadIdx.x + VEC_NT j)
// with c0 = lo rounded down to 4.  The tile builder keeps every tile within
// NCH * VEC_NT chunks (a tile that starts off the 4-element grid is shortened
// by the offset), and vectors are padded to XY_ALIGN elements, so a chunk that
// holds an element of the tile lies inside its vector.  A chunk without one is
// loaded at c0 (its values are never used) and not stored.
template <typename T> using v4 = T __attribute__((ext_vector_type(4)));
constexpr int NCH = VEC_TILE / (4 * VEC_NT);
static_assert(NCH * 4 * VEC_NT == VEC_TILE, "chunks per thread");
struct Chunks {
    int64_t lo, hi, c0;
    DEVI Chunks(int64_t lo_, int64_t hi_) : lo(lo_), hi(hi_), c0(lo_ & ~int64_t(3)) {}
    DEVI int64_t at(int j) const { return c0 + 4 * ((int64_t)threadIdx.x + (int64_t)VEC_NT * j); }
    DEVI bool any(int j) const { return at(j) < hi; }   // (at(j) + 4 > lo always)
    DEVI int64_t ld_at(int j) const { return any(j) ? at(j) : c0; }
    DEVI bool full(int j) const { const int64_t i = at(j); return i >= lo && i + 4 <= hi; }
    DEVI bool has(int j, int e) const { const int64_t i = at(j) + e; return i >= lo && i < hi; }
};
template <typename T>
DEVI v4<T> ld4(gptr<const T> p, int64_t i) {
    return *(gptr<const v4<T>>)(p + i);
}
template <typename T>
DEVI void st4(gptr<T> p, const Chunks& c, int j, const v4<T>& v) {
    if (!c.any(j)) return;
    const int64_t i = c.at(j);
    if (c.full(j)) {
        *(gptr<v4<T>>)(p + i) = v;
        return;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (c.has(j, e)) p[i + e] = v[e];
}

// ---------------------------------------------------------------- operator: convolution
// Direct full convolution and its adjoint (valid correlation) in one
// correlation form:  out[o] += s * sum_t w[t] * in[o + off + t]  with
//   A x : w = reversed taps, off = -(k-1), in = x (zero outside [0, n_in));
//   A^T y: w = taps,          off = 0,      in = y.
// One wave computes a tile of CONV_NT * R consecutive outputs; each lane keeps
// R outputs in registers and slides a 2R-wide register window over an LDS copy
// of the tile's input window (TILE + kc - 1 values, staged with batched
// loads); the taps of the chunk sit in LDS and are read as broadcasts.  The
// LDS size follows the kernel length (dynamic shared memory), so kernels up to
// CONV_KC_MAX taps need a single staging pass.
constexpr int CONV_NT = 64;
template <typename T> struct ConvCfg;
template <> struct ConvCfg<float> { static constexpr int R = 8; };
template <> struct ConvCfg<double> { static constexpr int R = 4; };
static_assert(CONV_NT * ConvCfg<float>::R == CONV_TILE_F32 && ConvCfg<float>::R == CONV_R_F32, "conv tile");
static_assert(CONV_NT * ConvCfg<double>::R == CONV_TILE_F64 && ConvCfg<double>::R == CONV_R_F64, "conv tile");

template <typename T, int R>
DEVI void lds_vec(T (&v)[R], const T* p) {   // 16-byte aligned LDS reads
    using V = typename Vec16<T>::type;
    constexpr int VW = Vec16<T>::W;
#pragma unroll
    for (int j = 0; j < R / VW; ++j) {
        const V q = reinterpret_cast<const V*>(p)[j];
        vec_get<T>(q, v + j * VW);
    }
}

template <typename T, int R>
DEVI void conv_step(T (&acc)[R], const T (&lo)[R], const T (&hi)[R], const T (&tw)[R]) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const T xv = (r + u < R) ? lo[r + u] : hi[r + u - R];
            acc[r] = fma(tw[u], xv, acc[r]);
        }
    }
}

// Termination test from the six sums of a check on the scaled iterate
// (u^, v^) with A^ = D A E, b^ = sb D b, c^ = sc E c:
//   y0 = ||(A^ u^_x + v^_s - tau b^) / D||^2   y1 = ||(A^ u^_x + v^_s) / D||^2   y2 = b^T u^_y
//   x0 = ||(A^T u^_y + tau c^) / E||^2          x1 = ||A^T u^_y / E||^2           x2 = c^T u^_x
// The original problem's point is x = E u^_x / (sb tau), y = D u^_y / (sc tau),
// s = v^_s / (D sb tau), so its relative residuals are sqrt(y0) / (sb tau (1 + ||b||))
// and sqrt(x0) / (sc tau (1 + ||c||)), and c^T x = x2 / (sb sc tau); the
// certificate rays (the same points without the 1 / tau) are tested the same way.
struct CheckOut {
    double rp, rd, gap, cx, by;   // residuals, gap, c^T x, b^T y (tau > 0)
    double cux, buy;              // c^T x_ray, b^T y_ray
    double status;                // 0: continue, else the CGS_* outcome
};
DEVI CheckOut check_outcome(gptr<const double> sc, double tau, double kap, double iter, double y0,
                            double y1, double y2, double x0, double x1, double x2, double eps,
                            int max_iters) {
    CheckOut o;
    const double sb = sc[SC_SB], scc = sc[SC_SC];
    o.cux = x2 / (sb * scc);
    o.buy = y2 / (sb * scc);
    o.rp = o.rd = o.gap = INFINITY;
    o.cx = o.by = NAN;
    o.status = 0.0;
    const bool finite = std::isfinite(y0) && std::isfinite(y1) && std::isfinite(y2) &&
                        std::isfinite(x0) && std::isfinite(x1) && std::isfinite(x2) &&
                        std::isfinite(tau) && std::isfinite(kap);
    if (!finite) {
        o.status = 5.0;   // CGS_NUMERICAL
        return o;
    }
    if (tau > 0.0) {
        o.rp = sqrt(y0) / (sb * tau) / (1.0 + sc[SC_NB]);
        o.rd = sqrt(x0) / (scc * tau) / (1.0 + sc[SC_NC]);
        o.cx = o.cux / tau;
        o.by = o.buy / tau;
        o.gap = fabs(o.cx + o.by) / (1.0 + fabs(o.cx) + fabs(o.by));
        if (o.rp <= eps && o.rd <= eps && o.gap <= eps) o.status = 1.0;   // CGS_SOLVED
    }
    if (o.status == 0.0 && tau < kap) {
        // ||A^T y_ray|| = sqrt(x1) / sc,  ||A x_ray + s_ray|| = sqrt(y1) / sb
        if (o.buy < 0.0 && sqrt(x1) / scc <= eps * (-o.buy)) o.status = 3.0;        // INFEASIBLE
        else if (o.cux < 0.0 && sqrt(y1) / sb <= eps * (-o.cux)) o.status = 4.0;   // UNBOUNDED
    }
    if (o.status == 0.0 && iter >= (double)max_iters) o.status = 2.0;   // MAX_ITERS
    return o;
}

// The part of an apply's output element g (index in the output vector) that
// does not come from convolution or dense blocks: base[g] (base >= 0) plus the
// identity blocks of the instance that cover g.
template <typename T>
DEVI double owned_init(const InstDesc& d, const IdBlock* ids, int adj, int out, int in, int base,
                       double sigma, int64_t g) {
    (void)out;
    gptr<const T> src = adj ? yvec<T>(d, in) : xvec<T>(d, in);
    double v = base >= 0 ? (double)(adj ? xvec<T>(d, base) : yvec<T>(d, base))[g] : 0.0;
    for (int b = d.id0; b < d.id1; ++b) {
        const IdBlock ib = ids[b];
        const int64_t r0 = adj ? ib.col0 : ib.row0;
        const int64_t c0 = adj ? ib.row0 : ib.col0;
        if (g >= r0 && g < r0 + ib.len) v += sigma * ib.scale * (double)src[g - r0 + c0];
    }
    return v;
}

// Initialisation of an apply's output tile: base plus identity blocks, for the
// elements that no owning convolution writes (the tile's ends are trimmed
// against owned ranges; an owned range inside the tile is skipped element by
// element).  Convolution and dense blocks that do not own their range then
// accumulate into these values.
// Four partial sums of a CG step folded into an A^T launch.
struct Fold4 {
    double a, b, c, d;
};

// The CG work folded into an A^T launch for X element g whose apply output is
// v (the arithmetic of k_cg_init and k_cg_dot):
//   mode 1: h = v; r = h - x_fq (and p = r when fp >= 0) written (not h); a += r^2, b += h^2
//   mode 2: q = v is written to `out`; a += p q, b += r^2, c += r q, d += q^2
template <typename T>
DEVI void fold_elem(const Tables& tb, const InstDesc& d, int mode, int fr, int fp, int fq, int out,
                    int64_t g, double v, Fold4& f, int idrows) {
    if (mode == 1) {
        const T h = (T)v;
        const double hd = (double)h;
        const T r = (T)(hd - (double)xvec<T>(d, fq)[g]);
        xvec<T>(d, fr)[g] = r;
        if (fp >= 0) xvec<T>(d, fp)[g] = r;
        f.a += (double)r * (double)r;
        f.b += hd * hd;
        if (idrows) {
            // A p's identity rows for p = r (ConvLaunch::idrows)
            for (int b = d.id0; b < d.id1; ++b) {
                const IdBlock ib = tb.ids[b];
                if (g >= ib.col0 && g < ib.col0 + ib.len)
                    yvec<T>(d, idrows - 1)[ib.row0 + g - ib.col0] = (T)(0.0 + ib.scale * (double)r);
            }
        }
    } else {
        const T q = (T)v;
        xvec<T>(d, out)[g] = q;
        const double pd = (double)xvec<T>(d, fp)[g], rd = (double)xvec<T>(d, fr)[g], qd = (double)q;
        f.a = fma(pd, qd, f.a);
        f.b = fma(rd, rd, f.b);
        f.c = fma(rd, qd, f.c);
        f.d = fma(qd, qd, f.d);
    }
}

// BATCH: loads of several elements in flight (a kernel of its own); without
// it the element loop, for initialisation tiles riding on long kernels, where
// the batched loop's code and registers would cost the kernel's main path.
template <typename T, bool BATCH = true>
DEVI void init_tile(const Tables& tb, const InstDesc& d, const VecTile& tl, int adj, int out, int in,
                    int base, double sigma, int fold, int fr, int fp, int fq, Fold4& f, int idrows = 0) {
    gptr<T> o = adj ? xvec<T>(d, out) : yvec<T>(d, out);
    gptr<const T> src = adj ? yvec<T>(d, in) : xvec<T>(d, in);
    gptr<const T> bs = base >= 0 ? (adj ? xvec<T>(d, base) : yvec<T>(d, base)) : nullptr;
    int64_t lo = tl.start, hi = tl.start + tl.len;
    int64_t olo[4], ohi[4];
    int nown = 0;
    for (int b = d.cb0; b < d.cb1 && nown < 4; ++b) {
        const ConvBlock cb = tb.cblk[b];
        if (!((cb.own >> adj) & 1)) continue;
        olo[nown] = adj ? cb.col0 : cb.row0;
        ohi[nown] = olo[nown] + (adj ? cb.n_in : cb.n_in + cb.k - 1);
        ++nown;
    }
    for (int j = 0; j < nown; ++j) {
        if (olo[j] <= lo && ohi[j] > lo) lo = ohi[j] < hi ? ohi[j] : hi;
        if (olo[j] < hi && ohi[j] >= hi) hi = olo[j] > lo ? olo[j] : lo;
    }
    // The identity blocks that reach [lo, hi) (at most IB of them; more take
    // the element-by-element loop).  Each thread then handles U elements at a
    // time with all their loads issued before the first addition: element by
    // element, every load would wait for the previous element's store.  The
    // additions keep the order of the plain form, base first, then the blocks
    // in table order.
    constexpr int IB = 4, U = 8;
    int64_t br0[IB], bc0[IB], bhi[IB];
    double bw[IB];
    int nb = 0;
    bool many = false;
    for (int b = d.id0; BATCH && b < d.id1; ++b) {
        const IdBlock ib = tb.ids[b];
        const int64_t r0 = adj ? ib.col0 : ib.row0;
        if (ib.len <= 0 || r0 >= hi || r0 + ib.len <= lo) continue;
        if (nb == IB) {
            many = true;
            break;
        }
        br0[nb] = r0;
        bc0[nb] = adj ? ib.row0 : ib.col0;
        bhi[nb] = r0 + ib.len;
        bw[nb] = sigma * ib.scale;
        ++nb;
    }
    if (many || !BATCH) {
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            bool owned = false;
            for (int j = 0; j < nown; ++j) owned = owned || (i >= olo[j] && i < ohi[j]);
            if (owned) continue;
            double v = bs ? (double)bs[i] : 0.0;
            for (int b = d.id0; b < d.id1; ++b) {
                const IdBlock ib = tb.ids[b];
                const int64_t r0 = adj ? ib.col0 : ib.row0;
                const int64_t c0 = adj ? ib.row0 : ib.col0;
                if (i >= r0 && i < r0 + ib.len) v += sigma * ib.scale * (double)src[i - r0 + c0];
            }
            if (fold) fold_elem<T>(tb, d, fold, fr, fp, fq, out, i, v, f, idrows);
            else o[i] = (T)v;
        }
        return;
    }
    const int64_t step = (int64_t)blockDim.x;
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += U * step) {
        T bv[U], sv[IB][U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * step;
            bv[u] = bs ? bs[i < hi ? i : lo] : (T)0;
        }
#pragma unroll
        for (int j = 0; j < IB; ++j) {
            if (j >= nb) break;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = i0 + u * step;
                const bool in_b = i < hi && i >= br0[j] && i < bhi[j];
                sv[j][u] = src[in_b ? i - br0[j] + bc0[j] : bc0[j]];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * step;
            if (i >= hi) break;
            bool owned = false;
            for (int j = 0; j < nown; ++j) owned = owned || (i >= olo[j] && i < ohi[j]);
            if (owned) continue;
            double v = bs ? (double)bv[u] : 0.0;
#pragma unroll
            for (int j = 0; j < IB; ++j)
                if (j < nb && i >= br0[j] && i < bhi[j]) v += bw[j] * (double)sv[j][u];
            if (fold) fold_elem<T>(tb, d, fold, fr, fp, fq, out, i, v, f, idrows);
            else o[i] = (T)v;
        }
    }
}
template <typename T>
DEVI void init_tile(const Tables& tb, const InstDesc& d, const VecTile& tl, int adj, int out, int in,
                    int base, double sigma) {
    Fold4 f{0.0, 0.0, 0.0, 0.0};
    init_tile<T>(tb, d, tl, adj, out, in, base, sigma, 0, 0, 0, 0, f);
}

// z_y = w_y + A z in working precision, with w_y = u_y + v_s formed as the
// projection stores it (the same two roundings as the update that ends CG,
// which forms z_y for the tau products and does not store it)
template <typename T>
DEVI T z_y(T u, T v, T az) {
    return (T)((double)(T)((double)u + (double)v) + (double)az);
}

// relaxed point minus v for a Y entry
template <typename T>
DEVI double ybar_minus_v(const InstDesc& d, int64_t i, double ut, double alpha, double& ubar) {
    const T u = yvec<T>(d, YU)[i];
    const double uy = (double)u;
    const double ut_y = (double)z_y<T>(u, yvec<T>(d, YV)[i], yvec<T>(d, YA)[i]) - ut * (double)yvec<T>(d, YG)[i];
    ubar = alpha * ut_y + (1.0 - alpha) * uy;
    return ubar - (double)yvec<T>(d, YV)[i];
}

// The sums of one tile of NT * R consecutive outputs (from `ot`) of a
// convolution block (adj = 0: A, adj = 1: A^T): acc[r] = the unscaled sum for
// output ot + R threadIdx.x + r.  src points at the block's first input (any
// address space).  smem: (NT * R + 2 * KC + 2R) elements of T.  Called by every
// thread of the workgroup; each chunk of taps starts with a workgroup barrier.
template <typename T, int NT, typename PC>
DEVI void conv_sums(const ConvBlock& cb, int adj, PC src, int64_t ot, int KC, unsigned char* smem,
                    T (&acc)[ConvCfg<T>::R]) {
    constexpr int R = ConvCfg<T>::R, TILE = NT * R;
    T* win = reinterpret_cast<T*>(smem);        // TILE + KC + 2R entries
    T* taps = win + TILE + KC + 2 * R;          // KC entries
    const int64_t n_out = adj ? cb.n_in : cb.n_in + cb.k - 1;
    const int64_t n_in = adj ? cb.n_in + cb.k - 1 : cb.n_in;
    const int64_t off = adj ? 0 : -(cb.k - 1);
    gptr<const T> w = (gptr<const T>)(adj ? cb.w_adj : cb.w_fwd);
    const int tid = threadIdx.x;
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = T(0);

    for (int64_t t0 = 0; t0 < cb.kpad; t0 += KC) {
        const int kc = (int)((cb.kpad - t0) < KC ? (cb.kpad - t0) : KC);
        __syncthreads();
        // stage the input window and the taps, 8 entries of each per lane
        // with all their loads in flight together (nwin > kc)
        const int64_t w0 = ot + off + t0;
        const int nwin = TILE + kc + 2 * R;
        for (int base = 0; base < nwin; base += 8 * NT) {
            T v[8], tv[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = base + j * NT + tid;
                const int64_t g = w0 + i;
                v[j] = (i < nwin && g >= 0 && g < n_in) ? src[g] : T(0);
                tv[j] = i < kc ? w[t0 + i] : T(0);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = base + j * NT + tid;
                if (i < nwin) win[i] = v[j];
                if (i < kc) taps[i] = tv[j];
            }
        }
        __syncthreads();
        // a wave whose outputs all lie past the block's end skips the sums
        if (ot + (int64_t)(tid & ~63) * R >= n_out) continue;
        const T* wp = win + tid * R;
        T a[R], b[R], tw[R];
        lds_vec<T, R>(a, wp);
        int tt = 0;
        for (; tt + 2 * R <= kc; tt += 2 * R) {
            lds_vec<T, R>(b, wp + tt + R);
            lds_vec<T, R>(tw, taps + tt);
            conv_step<T, R>(acc, a, b, tw);
            lds_vec<T, R>(a, wp + tt + 2 * R);
            lds_vec<T, R>(tw, taps + tt + R);
            conv_step<T, R>(acc, b, a, tw);
        }
        if (tt < kc) {
            lds_vec<T, R>(b, wp + tt + R);
            lds_vec<T, R>(tw, taps + tt);
            conv_step<T, R>(acc, a, b, tw);
        }
    }
}

// One tile of NT * R consecutive outputs (from `ot`) of a convolution block
// (adj = 0: A, out is Y; adj = 1: A^T, out is X), out += sigma * scale * (...),
// or, when ids is given and the block owns its output range, out = the
// element's base and identity-block terms + sigma * scale * (...).
// smem: (NT * R + 2 * KC + 2R) elements of T.  Called by every thread of the
// workgroup; starts and ends with a workgroup barrier.
template <typename T, int NT>
DEVI void conv_tile(const InstDesc& d, const ConvBlock& cb, int adj, int out, int in, double sigma,
                    int64_t ot, int KC, unsigned char* smem, const IdBlock* ids = nullptr,
                    int base = -1) {
    constexpr int R = ConvCfg<T>::R;
    const int64_t n_out = adj ? cb.n_in : cb.n_in + cb.k - 1;
    gptr<T> o = adj ? xvec<T>(d, out) + cb.col0 : yvec<T>(d, out) + cb.row0;
    gptr<const T> src = adj ? yvec<T>(d, in) + cb.row0 : xvec<T>(d, in) + cb.col0;
    const int tid = threadIdx.x;
    T acc[R];
    conv_sums<T, NT>(cb, adj, src, ot, KC, smem, acc);
    const double s = sigma * cb.scale;
    if (ids && (cb.own >> adj) & 1) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t oi = ot + (int64_t)tid * R + r;
            if (oi < n_out) o[oi] = (T)(owned_init<T>(d, ids, adj, out, in, base, sigma,
                                                      (adj ? cb.col0 : cb.row0) + oi) +
                                        s * (double)acc[r]);
        }
    } else {
        T ov[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t oi = ot + (int64_t)tid * R + r;
            ov[r] = oi < n_out ? o[oi] : T(0);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t oi = ot + (int64_t)tid * R + r;
            if (oi < n_out) o[oi] = (T)((double)ov[r] + s * (double)acc[r]);
        }
    }
    __syncthreads();
}


}  // namespace cgs
