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

#include <cmath>
#include <cstdint>

#include "kernels.hpp"
#include "device_common.hpp"

namespace cgs {

constexpr int FNT = 512;   // threads per instance workgroup

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

// out_rows += sigma * scale * W in (W = A or its stored transpose); a wave per row.
template <typename T>
DEVI void dense_rows(const InstDesc& d, const DenseBlock& db, int adj, int out, int in, double sigma) {
    gptr<const T> a = (gptr<const T>)(adj ? db.at : db.a);
    const int64_t ld = adj ? db.ldt : db.ld;
    const int64_t nrows = adj ? db.cols : db.rows, ncols = adj ? db.rows : db.cols;
    gptr<T> o = adj ? xvec<T>(d, out) + db.col0 : yvec<T>(d, out) + db.row0;
    gptr<const T> x = adj ? yvec<T>(d, in) + db.row0 : xvec<T>(d, in) + db.col0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double s = sigma * db.scale;
    for (int64_t r = wave; r < nrows; r += FNT / 64) {
        double acc = 0.0;
        for (int64_t j = lane; j < ncols; j += 64) acc = fma((double)a[r * ld + j], (double)x[j], acc);
        acc = wave_sum(acc);
        if (lane == 0) o[r] = (T)((double)o[r] + s * acc);
    }
}

// out = base (or 0) + sigma * (A in) (adj = 0) or sigma * (A^T in) (adj = 1).
template <typename T>
DEVI void f_apply(const Tables& tb, const InstDesc& d, int adj, int out, int in, int base,
                  double sigma, int kc, unsigned char* smem) {
    gptr<T> o = adj ? xvec<T>(d, out) : yvec<T>(d, out);
    gptr<const T> src = adj ? yvec<T>(d, in) : xvec<T>(d, in);
    gptr<const T> bs = base >= 0 ? (adj ? xvec<T>(d, base) : yvec<T>(d, base)) : nullptr;
    const int64_t len = adj ? d.n : d.m;
    for (int64_t i = threadIdx.x; i < len; i += FNT) {
        double v = bs ? (double)bs[i] : 0.0;
        for (int b = d.id0; b < d.id1; ++b) {
            const IdBlock ib = tb.ids[b];
            const int64_t r0 = adj ? ib.col0 : ib.row0;
            const int64_t c0 = adj ? ib.row0 : ib.col0;
            if (i >= r0 && i < r0 + ib.len) v += sigma * ib.scale * (double)src[i - r0 + c0];
        }
        o[i] = (T)v;
    }
    __syncthreads();
    constexpr int R = ConvCfg<T>::R;
    for (int c = d.cb0; c < d.cb1; ++c) {
        const ConvBlock cb = tb.cblk[c];
        const int64_t n_out = adj ? cb.n_in : cb.n_in + cb.k - 1;
        for (int64_t ot = 0; ot < n_out; ot += (int64_t)FNT * R)
            conv_tile<T, FNT>(d, cb, adj, out, in, sigma, ot, kc, smem);
    }
    for (int q = d.db0; q < d.db1; ++q) {
        const DenseBlock db = tb.dblk[q];
        dense_rows<T>(d, db, adj, out, in, sigma);
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(FNT) void k_fused(Tables tb, FusedArgs fa) {
    extern __shared__ __align__(16) unsigned char fsmem[];
    __shared__ double sh[FNT / 64];
    const InstDesc d = tb.inst[blockIdx.x];
    gptr<double> sc = scal(d);
    if (!(sc[SC_ACTIVE] != 0.0 && sc[SC_PHASE] == 2.0)) return;
    if (fa.refresh) {
        // the same applies as the exact recomputation at a check, so that a
        // refresh between checks leaves the carried products bitwise unchanged
        f_apply<T>(tb, d, 0, YA, XZ, -1, 1.0, fa.kc, fsmem);
        f_apply<T>(tb, d, 1, XK, YA, XZ, 1.0, fa.kc, fsmem);
        return;
    }
    const int tid = threadIdx.x;
    const int64_t n = d.n, m = d.m;
    double tau = sc[SC_TAU], kap = sc[SC_KAPPA], ut = sc[SC_UT];
    const double eta = sc[SC_ETA];
    double iter = sc[SC_ITER], cgtot = sc[SC_CGTOT], cgmax = sc[SC_CGMAX];
    gptr<T> ux = xvec<T>(d, XU), zx = xvec<T>(d, XZ), rx = xvec<T>(d, XR), px = xvec<T>(d, XP);
    gptr<T> qx = xvec<T>(d, XQ), hx = xvec<T>(d, XH), kz = xvec<T>(d, XK);
    gptr<const T> gx = xvec<T>(d, XG), cx = xvec<T>(d, XC);
    gptr<T> uy = yvec<T>(d, YU), vs = yvec<T>(d, YV), wy = yvec<T>(d, YW), zy = yvec<T>(d, YZ);
    gptr<T> ty = yvec<T>(d, YT), az = yvec<T>(d, YA);
    gptr<const T> by = yvec<T>(d, YB);
    const double al = fa.alpha;

    for (int step = 0; step < fa.nsteps; ++step) {
        // w_y = u_y + v_s; h = u_x - A^T w_y
        for (int64_t i = tid; i < m; i += FNT) wy[i] = (T)((double)uy[i] + (double)vs[i]);
        __syncthreads();
        f_apply<T>(tb, d, 1, XH, YW, XU, -1.0, fa.kc, fsmem);
        // CG on (I + A^T A) z = h from the warm start (carried K z, A z)
        double rr = 0.0, hh = 0.0;
        for (int64_t i = tid; i < n; i += FNT) {
            const double hi = (double)hx[i];
            const T ri = (T)(hi - (double)kz[i]);
            rx[i] = ri;
            px[i] = ri;
            rr = fma((double)ri, (double)ri, rr);
            hh = fma(hi, hi, hh);
        }
        rr = bsum(rr, sh);
        hh = bsum(hh, sh);
        double rel = fa.zeta > 0.0 ? fa.zeta / pow(iter + 1.0, fa.rate) : 0.0;
        rel = rel > fa.floor_ ? rel : fa.floor_;
        const double tol = sqrt(hh) * rel;
        int cgit = 0;
        bool act = fa.cg_max > 0 && std::isfinite(rr) && sqrt(rr) > tol;
        while (act) {
            f_apply<T>(tb, d, 0, YT, XP, -1, 1.0, fa.kc, fsmem);       // A p
            f_apply<T>(tb, d, 1, XQ, YT, XP, 1.0, fa.kc, fsmem);       // q = p + A^T A p
            double pq = 0.0;
            for (int64_t i = tid; i < n; i += FNT) pq = fma((double)px[i], (double)qx[i], pq);
            pq = bsum(pq, sh);
            const double a = rr / pq;
            if (!(pq > 0.0 && std::isfinite(a))) break;
            double rn = 0.0;
            for (int64_t i = tid; i < n; i += FNT) {
                const double qi = (double)qx[i];
                zx[i] = (T)fma(a, (double)px[i], (double)zx[i]);
                const T ri = (T)fma(-a, qi, (double)rx[i]);
                rx[i] = ri;
                kz[i] = (T)fma(a, qi, (double)kz[i]);
                rn = fma((double)ri, (double)ri, rn);
            }
            for (int64_t i = tid; i < m; i += FNT) az[i] = (T)fma(a, (double)ty[i], (double)az[i]);
            rn = bsum(rn, sh);
            const double be = rr > 0.0 ? rn / rr : 0.0;
            rr = rn;
            ++cgit;
            cgtot += 1.0;
            act = std::isfinite(rr) && sqrt(rr) > tol && cgit < fa.cg_max;
            if (act)
                for (int64_t i = tid; i < n; i += FNT) px[i] = (T)fma(be, (double)px[i], (double)rx[i]);
            __syncthreads();
        }
        if (cgit > cgmax) cgmax = cgit;
        // z_y = w_y + A z; u~_tau = (tau + kappa + c^T z_x + b^T z_y) / eta
        double cz = 0.0, bz = 0.0;
        for (int64_t i = tid; i < n; i += FNT) cz = fma((double)cx[i], (double)zx[i], cz);
        for (int64_t i = tid; i < m; i += FNT) {
            const T zv = (T)((double)wy[i] + (double)az[i]);
            zy[i] = zv;
            bz = fma((double)by[i], (double)zv, bz);
        }
        cz = bsum(cz, sh);
        bz = bsum(bz, sh);
        ut = (tau + kap + cz + bz) / eta;
        const double ubar = al * ut + (1.0 - al) * tau;
        const double tnew = ubar - kap > 0.0 ? ubar - kap : 0.0;
        kap = kap - ubar + tnew;
        tau = tnew;
        iter += 1.0;
        // second-order cones: head and tail norm of u_bar_y - v_s
        for (int sgi = d.sg0; sgi < d.sg1; ++sgi) {
            const SocSeg sg = tb.seg[sgi];
            double ss = 0.0;
            for (int64_t i = sg.start + 1 + tid; i < sg.start + sg.len; i += FNT) {
                double ub;
                const double pv = ybar_minus_v<T>(d, i, ut, al, ub);
                ss = fma(pv, pv, ss);
            }
            ss = bsum(ss, sh);
            if (tid == 0) {
                double ub;
                tb.seg_val[2 * sgi] = ybar_minus_v<T>(d, sg.start, ut, al, ub);
                tb.seg_val[2 * sgi + 1] = ss;
            }
        }
        __syncthreads();
        // relaxation, projection, dual update
        for (int64_t i = tid; i < n; i += FNT)
            ux[i] = (T)(al * ((double)zx[i] - ut * (double)gx[i]) + (1.0 - al) * (double)ux[i]);
        for (int64_t i = tid; i < d.l; i += FNT) {
            double ub;
            const double pv = ybar_minus_v<T>(d, i, ut, al, ub);
            const double pr = pv > 0.0 ? pv : 0.0;
            uy[i] = (T)pr;
            vs[i] = (T)(pr - pv);
        }
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
            for (int64_t i = sg.start + tid; i < sg.start + sg.len; i += FNT) {
                double ub;
                const double pv = ybar_minus_v<T>(d, i, ut, al, ub);
                double pr;
                if (mode == 0) pr = pv;
                else if (mode == 1) pr = 0.0;
                else pr = (i == sg.start) ? aa : (aa / nz) * pv;
                uy[i] = (T)pr;
                vs[i] = (T)(pr - pv);
            }
        }
        __syncthreads();
    }

    double status = 0.0;
    if (fa.check) {
        f_apply<T>(tb, d, 0, YT, XU, -1, 1.0, fa.kc, fsmem);   // A u_x
        f_apply<T>(tb, d, 1, XT, YU, -1, 1.0, fa.kc, fsmem);   // A^T u_y
        double y0 = 0, y1 = 0, y2 = 0, x0 = 0, x1 = 0, x2 = 0;
        gptr<const T> aty = xvec<T>(d, XT);
        gptr<const T> dr = yvec<T>(d, YD);
        gptr<const T> ec = xvec<T>(d, XE);
        for (int64_t i = tid; i < m; i += FNT) {
            const double w = 1.0 / (double)dr[i];
            const double e = ((double)ty[i] + (double)vs[i]) * w;
            const double rp = e - tau * (double)by[i] * w;
            y0 = fma(rp, rp, y0);
            y1 = fma(e, e, y1);
            y2 = fma((double)by[i], (double)uy[i], y2);
        }
        for (int64_t i = tid; i < n; i += FNT) {
            const double w = 1.0 / (double)ec[i];
            const double e = (double)aty[i] * w;
            const double rd = e + tau * (double)cx[i] * w;
            x0 = fma(rd, rd, x0);
            x1 = fma(e, e, x1);
            x2 = fma((double)cx[i], (double)ux[i], x2);
        }
        y0 = bsum(y0, sh); y1 = bsum(y1, sh); y2 = bsum(y2, sh);
        x0 = bsum(x0, sh); x1 = bsum(x1, sh); x2 = bsum(x2, sh);
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
            f_apply<T>(tb, d, 0, YA, XZ, -1, 1.0, fa.kc, fsmem);
            f_apply<T>(tb, d, 1, XK, YA, XZ, 1.0, fa.kc, fsmem);
        }
    }
    __syncthreads();
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

void launch_fused(int prec, const Tables& t, const FusedArgs& fa, hipStream_t st) {
    if (t.ninst <= 0) return;
    const size_t lds = fused_smem_bytes(prec, fa.kc);
    if (prec == 0) k_fused<double><<<t.ninst, FNT, lds, st>>>(t, fa);
    else k_fused<float><<<t.ninst, FNT, lds, st>>>(t, fa);
}

}  // namespace cgs
