// Fused ADMM steps for small instances: one workgroup per instance.
//
// A workgroup runs `nsteps` whole HSDE ADMM steps of its instance -- w_y, the
// right-hand side A^T w_y, the conjugate-gradient loop (Section IV-B listing,
// with its data-dependent trip count), the u~_tau solve, relaxation, cone
// projection and dual update (Section V-B) -- and then the termination test,
// with only workgroup barriers: no grid-wide synchronisation and no launch per
// step.  Reductions are fixed-order workgroup sums, so an instance's numbers do
// not depend on the other instances of the launch.  Arithmetic per element is
// the same as in the multi-kernel path; only the reduction trees differ.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>

#include "kernels.hpp"
#include "device_common.hpp"

namespace cgs {

constexpr int FNT = 512;   // threads per instance workgroup
constexpr int FU = 2;      // elements per thread whose loads are issued together

// Workgroup sum in a fixed order; every thread receives the result.
DEVI double bsum(double v, double* sh) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < FNT / 64; ++i) r += sh[i];
    return r;
}

// Elementwise pass over [0, len): the thread's elements tid + FNT j, FU at a
// time, with all FU elements' loads (ld) issued before any of their stores
// (st).  Element by element, every load would wait for the previous
// element's stores (the compiler cannot tell the vectors apart), one memory
// round trip each; more than two at a time measured slower (code size).
// Elements are visited in increasing j, so sums that st accumulates keep the
// order of a plain loop.  Indices are 32-bit: an instance on this path has
// n + m <= fused_max.
template <typename R, typename L, typename S>
DEVI void ew(int len, L ld, S st) {
    for (int i0 = threadIdx.x; i0 < len; i0 += FNT * FU) {
        R rg[FU];
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            const int i = i0 + u * FNT;
            if (i < len) ld(rg[u], i);
        }
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            const int i = i0 + u * FNT;
            if (i < len) st(rg[u], i);
        }
    }
}

// Where an instance's vectors live during a fused launch.  Every vector
// starts in the instance's region of global memory; the ones the CG loop and
// the step's other passes touch most are moved into the workgroup's LDS for the
// launch when they fit (a flat pointer reaches either), in the order of
// kResident, and written back at its end.  Only where the values sit changes:
// the arithmetic is the same.
template <typename T>
struct FVecs {
    T* x[NXV];
    T* y[NYV];
    unsigned res;   // bit j: kResident[j] is in LDS
};
// (X vectors below NXV, Y vectors as NXV + their index)
constexpr int kResident[] = {XP, XQ, XR, XZ, XK, NXV + YT, NXV + YA, XH, NXV + YW, NXV + YZ};
constexpr int kNumResident = sizeof(kResident) / sizeof(kResident[0]);
// carried from one launch to the next (the others are written before they are read)
constexpr bool resident_live(int v) { return v == XZ || v == XK || v == NXV + YA; }

template <typename T>
DEVI T*& fv_slot(FVecs<T>& fv, int v) { return v < NXV ? fv.x[v] : fv.y[v - NXV]; }

// Copy every resident vector between LDS and the instance's region: to LDS
// (in = true: only the vectors that hold live values) or back (in = false).
template <typename T>
DEVI void fv_copy(const InstDesc& d, FVecs<T>& fv, bool in) {
#pragma unroll
    for (int j = 0; j < kNumResident; ++j) {
        if (!((fv.res >> j) & 1u)) continue;
        const int v = kResident[j];
        if (in && !resident_live(v)) continue;
        T* lds = fv_slot(fv, v);
        T* glb = v < NXV ? (T*)xvec<T>(d, v) : (T*)yvec<T>(d, v - NXV);
        const int64_t len = v < NXV ? d.n : d.m;
        T* dst = in ? lds : glb;
        const T* src = in ? glb : lds;
        for (int64_t i0 = threadIdx.x; i0 < len; i0 += (int64_t)FNT * 8) {
            T t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = i0 + (int64_t)u * FNT;
                if (i < len) t[u] = src[i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = i0 + (int64_t)u * FNT;
                if (i < len) dst[i] = t[u];
            }
        }
    }
    __syncthreads();
}

// out_rows += sigma * scale * W in (W = A or its stored transpose); a wave per row.
template <typename T>
DEVI void dense_rows(const DenseBlock& db, int adj, T* out, const T* in, double sigma) {
    gptr<const T> a = (gptr<const T>)(adj ? db.at : db.a);
    const int64_t ld = adj ? db.ldt : db.ld;
    const int64_t nrows = adj ? db.cols : db.rows, ncols = adj ? db.rows : db.cols;
    T* o = out + (adj ? db.col0 : db.row0);
    const T* x = in + (adj ? db.row0 : db.col0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double s = sigma * db.scale;
    for (int64_t r = wave; r < nrows; r += FNT / 64) {
        double acc = 0.0;
        for (int64_t j = lane; j < ncols; j += 64) acc = fma((double)a[r * ld + j], (double)x[j], acc);
        acc = wave_sum(acc);
        if (lane == 0) o[r] = (T)((double)o[r] + s * acc);
    }
}

// out = base (or 0) + the identity blocks' terms, every entry of out: FU
// elements at a time, their base and the inputs of up to four identity blocks
// loaded together, then added block by block in the blocks' order.
template <typename T>
DEVI void f_identity(const Tables& tb, const InstDesc& d, int adj, T* o, const T* src, const T* bs,
                     int64_t len64, double sigma) {
    constexpr int NB = 4;
    const int len = (int)len64;
    for (int i0 = threadIdx.x; i0 < len; i0 += FNT * FU) {
        double v[FU];
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            const int i = i0 + u * FNT;
            v[u] = (bs && i < len) ? (double)bs[i] : 0.0;
        }
        for (int b0 = d.id0; b0 < d.id1; b0 += NB) {
            int r0[NB], c0[NB], ln[NB];
            double sb[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (b0 + b < d.id1) {
                    const IdBlock ib = tb.ids[b0 + b];
                    r0[b] = (int)(adj ? ib.col0 : ib.row0);
                    c0[b] = (int)(adj ? ib.row0 : ib.col0);
                    ln[b] = (int)ib.len;
                    sb[b] = ib.scale;
                } else {
                    r0[b] = c0[b] = ln[b] = 0;
                    sb[b] = 0.0;
                }
            }
            T x[NB][FU];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int u = 0; u < FU; ++u) {
                    const int i = i0 + u * FNT;
                    x[b][u] = (i < len && i >= r0[b] && i < r0[b] + ln[b]) ? src[i - r0[b] + c0[b]] : T(0);
                }
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int u = 0; u < FU; ++u) {
                    const int i = i0 + u * FNT;
                    if (i >= r0[b] && i < r0[b] + ln[b]) v[u] += sigma * sb[b] * (double)x[b][u];
                }
        }
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            const int i = i0 + u * FNT;
            if (i < len) o[i] = (T)v[u];
        }
    }
}

// out = base (or 0) + sigma * (A in) (adj = 0) or sigma * (A^T in) (adj = 1).
template <typename T>
DEVI void f_apply(const Tables& tb, const InstDesc& d, int adj, T* o, const T* src, const T* bs,
                  double sigma, int kc, unsigned char* smem) {
    f_identity<T>(tb, d, adj, o, src, bs, adj ? d.n : d.m, sigma);
    constexpr int R = ConvCfg<T>::R;
    const int tid = threadIdx.x;
    for (int c = d.cb0; c < d.cb1; ++c) {
        const ConvBlock cb = tb.cblk[c];
        const int64_t n_out = adj ? cb.n_in : cb.n_in + cb.k - 1;
        T* ob = o + (adj ? cb.col0 : cb.row0);
        const T* ib = src + (adj ? cb.row0 : cb.col0);
        const double s = sigma * cb.scale;
        for (int64_t ot = 0; ot < n_out; ot += (int64_t)FNT * R) {
            T acc[R];
            conv_sums<T, FNT>(cb, adj, ib, ot, kc, smem, acc);   // (its first barrier orders o's writes)
            T ov[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t oi = ot + (int64_t)tid * R + r;
                ov[r] = oi < n_out ? ob[oi] : T(0);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t oi = ot + (int64_t)tid * R + r;
                if (oi < n_out) ob[oi] = (T)((double)ov[r] + s * (double)acc[r]);
            }
        }
    }
    __syncthreads();
    for (int q = d.db0; q < d.db1; ++q) {
        dense_rows<T>(tb.dblk[q], adj, o, src, sigma);
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(FNT) void k_fused(Tables tb, FusedArgs fa) {
    extern __shared__ __align__(16) unsigned char fsmem[];
    __shared__ double sh[6 * (FNT / 64)];
    const InstDesc d = tb.inst[blockIdx.x];
    gptr<double> sc = scal(d);
    if (!(sc[SC_ACTIVE] != 0.0 && sc[SC_PHASE] == 2.0)) return;
    FVecs<T> fv;
#pragma unroll
    for (int k = 0; k < NXV; ++k) fv.x[k] = (T*)xvec<T>(d, k);
#pragma unroll
    for (int k = 0; k < NYV; ++k) fv.y[k] = (T*)yvec<T>(d, k);
    fv.res = 0u;
    if (fa.refresh) {
        // the same applies as the exact recomputation at a check, so that a
        // refresh between checks leaves the carried products bitwise unchanged
        f_apply<T>(tb, d, 0, fv.y[YA], fv.x[XZ], nullptr, 1.0, fa.kc, fsmem);
        f_apply<T>(tb, d, 1, fv.x[XK], fv.y[YA], fv.x[XZ], 1.0, fa.kc, fsmem);
        return;
    }
    {
        // LDS past the convolution's staging area, vector by vector in the
        // order of kResident while they fit
        unsigned char* p = fsmem + fa.lds_conv;
        int64_t left = fa.lds_res;
#pragma unroll
        for (int j = 0; j < kNumResident; ++j) {
            const int v = kResident[j];
            const int64_t bytes = (((v < NXV ? d.n : d.m) * (int64_t)sizeof(T)) + 15) & ~int64_t(15);
            if (bytes <= left) {
                fv_slot(fv, v) = reinterpret_cast<T*>(p);
                p += bytes;
                left -= bytes;
                fv.res |= 1u << j;
            }
        }
        fv_copy<T>(d, fv, true);
    }
    const int tid = threadIdx.x;
    const int64_t n = d.n, m = d.m;
    double tau = sc[SC_TAU], kap = sc[SC_KAPPA], ut = sc[SC_UT];
    const double eta = sc[SC_ETA];
    double iter = sc[SC_ITER], cgtot = sc[SC_CGTOT], cgmax = sc[SC_CGMAX];
    T *ux = fv.x[XU], *zx = fv.x[XZ], *rx = fv.x[XR], *px = fv.x[XP];
    T *qx = fv.x[XQ], *hx = fv.x[XH], *kz = fv.x[XK];
    const T *gx = fv.x[XG], *cx = fv.x[XC];
    T *uy = fv.y[YU], *vs = fv.y[YV], *wy = fv.y[YW], *zy = fv.y[YZ];
    T *ty = fv.y[YT], *az = fv.y[YA];
    const T *by = fv.y[YB], *gy = fv.y[YG];
    const double al = fa.alpha;

    for (int step = 0; step < fa.nsteps; ++step) {
        // w_y = u_y + v_s; h = u_x - A^T w_y
        struct V2 { T a, b; };
        ew<V2>(m, [&](V2& r, int i) { r.a = uy[i]; r.b = vs[i]; },
               [&](V2& r, int i) { wy[i] = (T)((double)r.a + (double)r.b); });
        __syncthreads();
        f_apply<T>(tb, d, 1, hx, wy, ux, -1.0, fa.kc, fsmem);
        // CG on (I + A^T A) z = h from the warm start (carried K z, A z)
        double s2[2] = {0.0, 0.0};   // ||r||^2, ||h||^2
        ew<V2>(n, [&](V2& r, int i) { r.a = hx[i]; r.b = kz[i]; },
               [&](V2& r, int i) {
                   const double hi = (double)r.a;
                   const T ri = (T)(hi - (double)r.b);
                   rx[i] = ri;
                   px[i] = ri;
                   s2[0] = fma((double)ri, (double)ri, s2[0]);
                   s2[1] = fma(hi, hi, s2[1]);
               });
        block_sumN<FNT, 2>(s2, sh);
        double rr = s2[0];
        const double hh = s2[1];
        double rel = fa.zeta > 0.0 ? fa.zeta / pow(iter + 1.0, fa.rate) : 0.0;
        rel = rel > fa.floor_ ? rel : fa.floor_;
        const double tol = sqrt(hh) * rel;
        int cgit = 0;
        bool act = fa.cg_max > 0 && std::isfinite(rr) && sqrt(rr) > tol;
        while (act) {
            f_apply<T>(tb, d, 0, ty, px, nullptr, 1.0, fa.kc, fsmem);   // A p
            f_apply<T>(tb, d, 1, qx, ty, px, 1.0, fa.kc, fsmem);        // q = p + A^T A p
            double pq = 0.0;
            ew<V2>(n, [&](V2& r, int i) { r.a = px[i]; r.b = qx[i]; },
                   [&](V2& r, int i) { pq = fma((double)r.a, (double)r.b, pq); });
            pq = bsum(pq, sh);
            const double a = rr / pq;
            if (!(pq > 0.0 && std::isfinite(a))) break;
            double rn = 0.0;
            struct V5 { T q, p, z, r, k; };
            ew<V5>(n, [&](V5& r, int i) { r.q = qx[i]; r.p = px[i]; r.z = zx[i]; r.r = rx[i]; r.k = kz[i]; },
                   [&](V5& r, int i) {
                       const double qi = (double)r.q;
                       zx[i] = (T)fma(a, (double)r.p, (double)r.z);
                       const T ri = (T)fma(-a, qi, (double)r.r);
                       rx[i] = ri;
                       kz[i] = (T)fma(a, qi, (double)r.k);
                       rn = fma((double)ri, (double)ri, rn);
                   });
            ew<V2>(m, [&](V2& r, int i) { r.a = ty[i]; r.b = az[i]; },
                   [&](V2& r, int i) { az[i] = (T)fma(a, (double)r.a, (double)r.b); });
            rn = bsum(rn, sh);
            const double be = rr > 0.0 ? rn / rr : 0.0;
            rr = rn;
            ++cgit;
            cgtot += 1.0;
            act = std::isfinite(rr) && sqrt(rr) > tol && cgit < fa.cg_max;
            if (act)
                ew<V2>(n, [&](V2& r, int i) { r.a = px[i]; r.b = rx[i]; },
                       [&](V2& r, int i) { px[i] = (T)fma(be, (double)r.a, (double)r.b); });
            __syncthreads();
        }
        if (cgit > cgmax) cgmax = cgit;
        // z_y = w_y + A z; u~_tau = (tau + kappa + c^T z_x + b^T z_y) / eta
        double s3[2] = {0.0, 0.0};   // c^T z_x, b^T z_y
        ew<V2>(n, [&](V2& r, int i) { r.a = cx[i]; r.b = zx[i]; },
               [&](V2& r, int i) { s3[0] = fma((double)r.a, (double)r.b, s3[0]); });
        struct V3 { T w, a, b; };
        ew<V3>(m, [&](V3& r, int i) { r.w = wy[i]; r.a = az[i]; r.b = by[i]; },
               [&](V3& r, int i) {
                   const T zv = (T)((double)r.w + (double)r.a);
                   zy[i] = zv;
                   s3[1] = fma((double)r.b, (double)zv, s3[1]);
               });
        block_sumN<FNT, 2>(s3, sh);
        const double cz = s3[0], bz = s3[1];
        ut = (tau + kap + cz + bz) / eta;
        const double ubar = al * ut + (1.0 - al) * tau;
        const double tnew = ubar - kap > 0.0 ? ubar - kap : 0.0;
        kap = kap - ubar + tnew;
        tau = tnew;
        iter += 1.0;
        // relaxed point minus v_s of Y entry i, from its u_y, z_y, g_y, v_s
        struct V4 { T u, z, g, v; };
        auto ld4y = [&](V4& r, int i) { r.u = uy[i]; r.z = zy[i]; r.g = gy[i]; r.v = vs[i]; };
        auto pv_of = [&](const V4& r) {
            const double ut_y = (double)r.z - ut * (double)r.g;
            const double ub = al * ut_y + (1.0 - al) * (double)r.u;
            return ub - (double)r.v;
        };
        // second-order cones: head and tail norm of u_bar_y - v_s
        for (int sgi = d.sg0; sgi < d.sg1; ++sgi) {
            const SocSeg sg = tb.seg[sgi];
            double ss = 0.0;
            ew<V4>(sg.len - 1, [&](V4& r, int i) { ld4y(r, sg.start + 1 + i); },
                   [&](V4& r, int) {
                       const double pv = pv_of(r);
                       ss = fma(pv, pv, ss);
                   });
            ss = bsum(ss, sh);
            if (tid == 0) {
                V4 r;
                ld4y(r, sg.start);
                tb.seg_val[2 * sgi] = pv_of(r);
                tb.seg_val[2 * sgi + 1] = ss;
            }
        }
        __syncthreads();
        // relaxation, projection, dual update
        struct V3x { T z, g, u; };
        ew<V3x>(n, [&](V3x& r, int i) { r.z = zx[i]; r.g = gx[i]; r.u = ux[i]; },
                [&](V3x& r, int i) {
                    ux[i] = (T)(al * ((double)r.z - ut * (double)r.g) + (1.0 - al) * (double)r.u);
                });
        ew<V4>(d.l, ld4y, [&](V4& r, int i) {
            const double pv = pv_of(r);
            const double pr = pv > 0.0 ? pv : 0.0;
            uy[i] = (T)pr;
            vs[i] = (T)(pr - pv);
        });
        for (int sgi = d.sg0; sgi < d.sg1; ++sgi) {
            const SocSeg sg = tb.seg[sgi];
            const double t = tb.seg_val[2 * sgi];
            const double nz = sqrt(tb.seg_val[2 * sgi + 1]);
            int mode;
            double aa = 0.0;
            if (nz <= t) mode = 0;
            else if (nz <= -t) mode = 1;
            else {
                mode = 2;
                aa = 0.5 * (t + nz);
            }
            ew<V4>(sg.len, [&](V4& r, int i) { ld4y(r, sg.start + i); },
                   [&](V4& r, int i) {
                       const double pv = pv_of(r);
                       double pr;
                       if (mode == 0) pr = pv;
                       else if (mode == 1) pr = 0.0;
                       else pr = (i == 0) ? aa : (aa / nz) * pv;
                       uy[sg.start + i] = (T)pr;
                       vs[sg.start + i] = (T)(pr - pv);
                   });
        }
        __syncthreads();
    }

    double status = 0.0;
    if (fa.check) {
        f_apply<T>(tb, d, 0, ty, ux, nullptr, 1.0, fa.kc, fsmem);          // A u_x
        f_apply<T>(tb, d, 1, fv.x[XT], uy, nullptr, 1.0, fa.kc, fsmem);    // A^T u_y
        const T* aty = fv.x[XT];
        const T* dr = fv.y[YD];
        const T* ec = fv.x[XE];
        double r6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // Y: 0-2, X: 3-5
        struct V5y { T d, t, v, b, u; };
        ew<V5y>(m, [&](V5y& r, int i) { r.d = dr[i]; r.t = ty[i]; r.v = vs[i]; r.b = by[i]; r.u = uy[i]; },
                [&](V5y& r, int) {
                    const double w = 1.0 / (double)r.d;
                    const double e = ((double)r.t + (double)r.v) * w;
                    const double rp = e - tau * (double)r.b * w;
                    r6[0] = fma(rp, rp, r6[0]);
                    r6[1] = fma(e, e, r6[1]);
                    r6[2] = fma((double)r.b, (double)r.u, r6[2]);
                });
        struct V4x { T e, a, c, u; };
        ew<V4x>(n, [&](V4x& r, int i) { r.e = ec[i]; r.a = aty[i]; r.c = cx[i]; r.u = ux[i]; },
                [&](V4x& r, int) {
                    const double w = 1.0 / (double)r.e;
                    const double e = (double)r.a * w;
                    const double rd = e + tau * (double)r.c * w;
                    r6[3] = fma(rd, rd, r6[3]);
                    r6[4] = fma(e, e, r6[4]);
                    r6[5] = fma((double)r.c, (double)r.u, r6[5]);
                });
        block_sumN<FNT, 6>(r6, sh);
        const double y0 = r6[0], y1 = r6[1], y2 = r6[2], x0 = r6[3], x1 = r6[4], x2 = r6[5];
        const CheckOut co = check_outcome(sc, tau, kap, iter, y0, y1, y2, x0, x1, x2, fa.eps,
                                          fa.max_iters);
        status = co.status;
        if (tid == 0) {
            sc[SC_CUX] = co.cux;
            sc[SC_BUY] = co.buy;
            sc[SC_RP] = co.rp;
            sc[SC_RD] = co.rd;
            sc[SC_GAP] = co.gap;
            sc[SC_CX] = co.cx;
            sc[SC_BY] = co.by;
        }
        if (status == 0.0) {
            // exact recomputation of the carried products of the warm start
            f_apply<T>(tb, d, 0, az, zx, nullptr, 1.0, fa.kc, fsmem);
            f_apply<T>(tb, d, 1, kz, az, zx, 1.0, fa.kc, fsmem);
        }
    }
    __syncthreads();
    fv_copy<T>(d, fv, false);
    if (tid == 0) {
        sc[SC_TAU] = tau;
        sc[SC_KAPPA] = kap;
        sc[SC_UT] = ut;
        sc[SC_ITER] = iter;
        sc[SC_CGTOT] = cgtot;
        if (fa.check) {
            sc[SC_CGMAXLAST] = cgmax;
            sc[SC_CGMAX] = 0.0;
        } else {
            sc[SC_CGMAX] = cgmax;
        }
        if (status != 0.0) {
            sc[SC_STATUS] = status;
            sc[SC_ACTIVE] = 0.0;
        }
    }
}

size_t fused_smem_bytes(int prec, int kc) {
    const int R = prec == 0 ? CONV_R_F64 : CONV_R_F32;
    return (size_t)(FNT * R + 2 * kc + 2 * R) * (prec == 0 ? 8 : 4);
}

int64_t fused_resident_bytes(int prec, int64_t n, int64_t m) {
    const int64_t es = prec == 0 ? 8 : 4;
    int64_t b = 0;
    for (int j = 0; j < kNumResident; ++j)
        b += (((kResident[j] < NXV ? n : m) * es) + 15) & ~int64_t(15);
    return b;
}

// Dynamic LDS per workgroup that the fused kernels may take on each device
// (0: not yet queried; then what fits in the 64 KB that needs no attribute)
static std::atomic<int> g_fused_lds[64];   // (zero-initialised: static storage)

static int fused_static_lds() {
    int b = 0;
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, (const void*)k_fused<double>) == hipSuccess) b = std::max(b, (int)a.sharedSizeBytes);
    if (hipFuncGetAttributes(&a, (const void*)k_fused<float>) == hipSuccess) b = std::max(b, (int)a.sharedSizeBytes);
    return b > 0 ? b : 1024;
}

int fused_prepare() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536 - 1024;
    if (g_fused_lds[dev].load() == 0) {
        const int fixed = fused_static_lds();   // the kernels' own __shared__ arrays
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        int dyn = v - fixed;
        if (dyn > 65536 - fixed &&
            (hipFuncSetAttribute((const void*)k_fused<double>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) !=
                 hipSuccess ||
             hipFuncSetAttribute((const void*)k_fused<float>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) !=
                 hipSuccess))
            dyn = 65536 - fixed;
        g_fused_lds[dev].store(dyn);   // (two threads that get here store the same value)
    }
    return g_fused_lds[dev].load();
}

void launch_fused(int prec, const Tables& t, FusedArgs fa, hipStream_t st) {
    if (t.ninst <= 0) return;
    int dev = 0;
    const int known = (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) ? g_fused_lds[dev].load() : 0;
    const int cap = known > 0 ? known : 65536 - 1024;
    fa.lds_conv = ((int64_t)fused_smem_bytes(prec, fa.kc) + 15) & ~int64_t(15);
    fa.lds_res = std::max<int64_t>(0, std::min<int64_t>(fa.res_want, (int64_t)cap - fa.lds_conv));
    const size_t lds = (size_t)(fa.lds_conv + fa.lds_res);
    if (prec == 0) k_fused<double><<<t.ninst, FNT, lds, st>>>(t, fa);
    else k_fused<float><<<t.ninst, FNT, lds, st>>>(t, fa);
}

}  // namespace cgs
