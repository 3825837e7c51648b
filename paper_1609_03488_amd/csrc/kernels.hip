// HIP kernels of the structured-operator conic solver (gfx950 / CDNA4).
//
// Conventions
//  * One workgroup per tile of a tile table (see common.hpp).  Every tile lies
//    in one instance; a workgroup first reads its instance's gate flags and
//    leaves at once when the instance does not take part in this step.
//  * Reductions (dot products, norms) are deterministic: each workgroup folds
//    its tile in a fixed thread/wave order into FP64 partials, and a finalize
//    kernel (one workgroup per instance) sums the instance's partials in tile
//    order and finishes the scalar work (CG alpha and beta, tau/kappa,
//    residuals).  No atomics and no device-wide fences are used inside a
//    kernel (on a multi-XCD part a device-scope fence writes back and
//    invalidates the XCD's L2), so an instance's numbers do not depend on the
//    other instances of a launch.
//  * Vectors are in the working precision T (float or double); every scalar of
//    the method (tau, kappa, eta, CG alpha/beta, norms, residuals) is FP64.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "cgs.h"

#include <cmath>
#include <cstdint>

#include "kernels.hpp"
#include "device_common.hpp"

namespace cgs {

// ---------------------------------------------------------------- operator: identity part + base
template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_apply_init(Tables tb, int adj, int out, int in, int base,
                                                       double sigma, int gate) {
    const VecTile tl = adj ? tb.xt[blockIdx.x] : tb.yt[blockIdx.x];
    const InstDesc d = tb.inst[tl.inst];
    if (!gate_ok(scal(d), gate)) return;
    init_tile<T>(tb, d, tl, adj, out, in, base, sigma);
}

template <typename T>
__global__ __launch_bounds__(CONV_NT) void k_conv(Tables tb, ConvLaunch cl, int adj, int out, int in,
                                                  int base, double sigma, int gate) {
    extern __shared__ __align__(16) unsigned char conv_smem[];
    if ((int)blockIdx.x >= cl.ntiles) {   // initialisation tiles riding on the launch
        const VecTile it = cl.init[blockIdx.x - cl.ntiles];
        const InstDesc di = tb.inst[it.inst];
        if (gate_ok(scal(di), gate)) init_tile<T>(tb, di, it, adj, out, in, base, sigma);
        return;
    }
    const ConvTile tl = cl.tiles[blockIdx.x];
    const InstDesc d = tb.inst[tl.inst];
    if (!gate_ok(scal(d), gate)) return;
    const ConvBlock cb = cl.blocks[tl.blk];
    conv_tile<T, CONV_NT>(d, cb, adj, out, in, sigma, tl.start, cl.kc, conv_smem, tb.ids, base);
}

size_t conv_smem_bytes(int prec, int kc) {
    const int R = prec == 0 ? CONV_R_F64 : CONV_R_F32;
    const int tile = prec == 0 ? CONV_TILE_F64 : CONV_TILE_F32;
    return (size_t)(tile + 2 * kc + 2 * R) * (prec == 0 ? 8 : 4);
}

// ---------------------------------------------------------------- operator: dense block
// out[row] += s * dot(a[row, :], in) for GEMV_RB rows per workgroup; all
// threads stride over the columns with 16-byte loads of the (padded,
// 16-byte aligned) rows; FP64 accumulation.  The adjoint walks the stored
// transpose, so both directions read rows contiguously.
constexpr int GEMV_NT = 256;
constexpr int GEMV_RB = DENSE_ROWS;

template <typename T>
__global__ __launch_bounds__(GEMV_NT) void k_gemv(Tables tb, DenseLaunch dl, int adj, int out, int in,
                                                  double sigma, int gate) {
    using V = typename Vec16<T>::type;
    constexpr int VW = Vec16<T>::W;
    __shared__ double sh[GEMV_RB][GEMV_NT / 64];
    const DenseTile tl = dl.tiles[blockIdx.x];
    const InstDesc d = tb.inst[tl.inst];
    if (!gate_ok(scal(d), gate)) return;
    const DenseBlock db = dl.blocks[tl.blk];
    gptr<const T> a;
    int64_t ld, ncols;
    gptr<T> o;
    gptr<const T> x;
    if (!adj) {
        a = (gptr<const T>)db.a;
        ld = db.ld;
        ncols = db.cols;
        o = yvec<T>(d, out) + db.row0;
        x = xvec<T>(d, in) + db.col0;
    } else {
        a = (gptr<const T>)db.at;
        ld = db.ldt;
        ncols = db.rows;
        o = xvec<T>(d, out) + db.col0;
        x = yvec<T>(d, in) + db.row0;
    }
    const int nr = tl.nr;
    gptr<const T> arow = a + tl.r0 * ld;
    double acc[GEMV_RB];
#pragma unroll
    for (int r = 0; r < GEMV_RB; ++r) acc[r] = 0.0;
    const int64_t nvec = ncols / VW;
    for (int64_t v = threadIdx.x; v < nvec; v += GEMV_NT) {
        T xv[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) xv[e] = x[v * VW + e];
#pragma unroll
        for (int r = 0; r < GEMV_RB; ++r) {
            if (r < nr) {
                const V av = *(gptr<const V>)(arow + r * ld + v * VW);
                T ae[VW];
                vec_get<T>(av, ae);
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[r] = fma((double)ae[e], (double)xv[e], acc[r]);
            }
        }
    }
    for (int64_t j = nvec * VW + threadIdx.x; j < ncols; j += GEMV_NT) {
        const double xj = (double)x[j];
#pragma unroll
        for (int r = 0; r < GEMV_RB; ++r)
            if (r < nr) acc[r] = fma((double)arow[r * ld + j], xj, acc[r]);
    }
    const double s = sigma * db.scale;
#pragma unroll
    for (int r = 0; r < GEMV_RB; ++r) {
        const double tot = block_sum<GEMV_NT>(acc[r], sh[r]);
        if (threadIdx.x == 0 && r < nr) {
            gptr<T> op = o + tl.r0 + r;
            *op = (T)((double)*op + s * tot);
        }
    }
}

// ---------------------------------------------------------------- CG
template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_cg_init(Tables tb, int z, int r, int p, int q, int h,
                                                    int have_q, double zeta, double rate,
                                                    double floor_, int cg_max, int gate) {
    __shared__ double sh[VEC_NT / 64];
    const VecTile tl = tb.xt[blockIdx.x];
    const InstDesc d = tb.inst[tl.inst];
    gptr<double> sc = scal(d);
    if (!gate_ok(sc, gate)) return;
    gptr<T> rv = xvec<T>(d, r);
    gptr<T> pv = xvec<T>(d, p);
    gptr<const T> qv = xvec<T>(d, q);
    gptr<const T> hv = xvec<T>(d, h);
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = tl.start + threadIdx.x; i < tl.start + tl.len; i += VEC_NT) {
        const double hi = (double)hv[i];
        const T ri = (T)(have_q ? hi - (double)qv[i] : hi);
        rv[i] = ri;
        pv[i] = ri;
        s0 += (double)ri * (double)ri;
        s1 += hi * hi;
    }
    s0 = block_sum<VEC_NT>(s0, sh);
    s1 = block_sum<VEC_NT>(s1, sh);
    double* part = tb.xpart + 4 * (int64_t)blockIdx.x;
    if (threadIdx.x == 0) {
        part[0] = s0;
        part[1] = s1;
    }
}

// Partials of <p, q>, ||r||^2, <r, q> and ||q||^2 (slots 0..3).  The first
// tile's workgroup records the iteration whose products are now in place: the
// update of that iteration runs only if it finds this mark, so the update can
// clear the run flag without racing its own workgroups' gate tests.
template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_cg_dot(Tables tb, int p, int q, int r, int it, int gate) {
    __shared__ double sh[4 * (VEC_NT / 64)];
    const VecTile tl = tb.xt[blockIdx.x];
    const InstDesc d = tb.inst[tl.inst];
    gptr<double> sc = scal(d);
    if (!gate_ok(sc, gate)) return;
    if ((int)blockIdx.x == d.xt0 && threadIdx.x == 0) sc[SC_CGRUN] = (double)it;
    gptr<const T> pv = xvec<T>(d, p);
    gptr<const T> qv = xvec<T>(d, q);
    gptr<const T> rv = xvec<T>(d, r);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = tl.start + threadIdx.x; i < tl.start + tl.len; i += VEC_NT) {
        const double pi = (double)pv[i], qi = (double)qv[i], ri = (double)rv[i];
        s[0] = fma(pi, qi, s[0]);
        s[1] = fma(ri, ri, s[1]);
        s[2] = fma(ri, qi, s[2]);
        s[3] = fma(qi, qi, s[3]);
    }
    block_sum4<VEC_NT>(s, sh);
    if (threadIdx.x == 0) {
        double* part = tb.xpart + 4 * (int64_t)blockIdx.x;
        part[0] = s[0];
        part[1] = s[1];
        part[2] = s[2];
        part[3] = s[3];
    }
}

// The scalar products of u~_tau for one tile (Section V-B: the tau component
// of the subspace projection): c^T z_x over an X tile, or b^T z_y over a Y
// tile with z_y = w_y + A z (the carried product) formed, not stored; FP64 partial in
// slot 0 of the tile's X or Y partials.  With CgStart::cone the cone terms of
// the projection that follows are formed as well (see CgStart).
//
// The element work of the update that ends an instance's CG, and of a CG
// update that goes on, in one routine: `upd` = 0 leaves z and A z as they are
// (a step whose CG ran no update) and only does the tau (and cone) work.
// Every thread loads its chunks of every vector it needs before the first
// arithmetic, then stores.
template <typename T>
DEVI void cg_elems(const Tables& tb, const InstDesc& d, const XYTile& xt, gptr<const double> sc,
                   const CgStart& cs, bool upd, double al, double be, bool more, bool track, bool tw,
                   int z, int r, int p, int q, double* sh) {
    // One chunk at a time (all its loads, then the arithmetic, then its
    // stores): holding every chunk of every vector at once needs more
    // registers than let all of a launch's workgroups be resident together.
    const Chunks ck(xt.t.start, xt.t.start + xt.t.len);
    if (!xt.is_y) {
        gptr<T> zp = xvec<T>(d, z);
        gptr<T> rp = xvec<T>(d, r);
        gptr<const T> pp = xvec<T>(d, p);
        gptr<T> pw = xvec<T>(d, cs.pn >= 0 ? cs.pn : p);
        gptr<const T> qp = xvec<T>(d, q);
        gptr<T> kp = xvec<T>(d, XK);
        gptr<const T> cp = xvec<T>(d, XC);
        double s0 = 0.0;
#pragma unroll 1
        for (int j = 0; j < NCH; ++j) {
            if (!ck.any(j)) break;
            const int64_t i = ck.at(j);
            v4<T> zv = ld4<T>(zp, i), qv, pv, rv, kv, cv;
            if (upd) {
                qv = ld4<T>(qp, i);
                pv = ld4<T>(pp, i);
                if (more) rv = ld4<T>(rp, i);
                if (track) kv = ld4<T>(kp, i);
            }
            if (tw) cv = ld4<T>(cp, i);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (upd) {
                    const double qi = (double)qv[e], pi = (double)pv[e];
                    zv[e] = (T)fma(al, pi, (double)zv[e]);
                    if (more) {
                        const T ri = (T)fma(-al, qi, (double)rv[e]);
                        rv[e] = ri;
                        pv[e] = (T)fma(be, pi, (double)ri);
                    }
                    if (track) kv[e] = (T)fma(al, qi, (double)kv[e]);
                }
                if (tw && ck.has(j, e)) s0 = fma((double)cv[e], (double)zv[e], s0);
            }
            if (upd) {
                // (once CG has ended, r is dead: the next solve forms it afresh)
                st4<T>(zp, ck, j, zv);
                if (more) {
                    st4<T>(rp, ck, j, rv);
                    st4<T>(pw, ck, j, pv);
                }
                if (track) st4<T>(kp, ck, j, kv);
            }
        }
        if (tw) {
            s0 = block_sum<VEC_NT>(s0, sh);
            if (threadIdx.x == 0) {
                double* part = tb.xpart + 4 * (int64_t)xt.index;
                if (cs.cone) tb.tpart[xt.index] = s0;
                else part[0] = s0;
                if (cs.cone && xt.index == d.xt0) {
                    // for the projection: the expansion point and tau + kappa
                    // (it rewrites tau and kappa while its workgroups run)
                    const double ex = sc[SC_UT];
                    part[1] = std::isfinite(ex) ? ex : 0.0;
                    part[2] = sc[SC_TAU] + sc[SC_KAPPA];
                }
            }
        }
        return;
    }
    gptr<T> azp = yvec<T>(d, YA);
    gptr<const T> app = yvec<T>(d, YT);
    gptr<const T> wyp = yvec<T>(d, YW);
    gptr<const T> bp = yvec<T>(d, YB);
    gptr<const T> uyp = yvec<T>(d, YU);
    gptr<const T> vsp = yvec<T>(d, YV);
    gptr<const T> gyp = yvec<T>(d, YG);
    const bool cone = tw && cs.cone && xt.t.seg >= 0;
    double e_pt = 0.0;
    int64_t head = -1;
    if (cone) {
        const double ex = sc[SC_UT];
        e_pt = std::isfinite(ex) ? ex : 0.0;
        head = tb.seg[xt.t.seg].start;
    }
    const double alpha = cs.alpha;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int j = 0; j < NCH; ++j) {
        if (!ck.any(j)) break;
        const int64_t i = ck.at(j);
        v4<T> av = ld4<T>(azp, i), apv, wv, bv, uv, vv, gv;
        if (upd) apv = ld4<T>(app, i);
        if (tw) bv = ld4<T>(bp, i);
        if (cone) {
            // w_y = u_y + v_s as the projection (or k_wy) formed it from
            // these stored values: recomputed instead of loaded
            uv = ld4<T>(uyp, i);
            vv = ld4<T>(vsp, i);
            gv = ld4<T>(gyp, i);
#pragma unroll
            for (int e = 0; e < 4; ++e) wv[e] = (T)((double)uv[e] + (double)vv[e]);
        } else if (tw) {
            wv = ld4<T>(wyp, i);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (upd) av[e] = (T)fma(al, (double)apv[e], (double)av[e]);
            if (!tw) continue;
            const T zy = (T)((double)wv[e] + (double)av[e]);
            wv[e] = zy;   // (w_y is not needed again: the register holds z_y)
            if (!ck.has(j, e)) continue;
            s[0] = fma((double)bv[e], (double)zy, s[0]);
            if (cone) {
                const double g = (double)gv[e];
                const double a = alpha * (double)zy + (1.0 - alpha) * (double)uv[e] - (double)vv[e] -
                                 alpha * e_pt * g;
                const double b = alpha * g;
                if (i + e == head) {
                    tb.seg_val[2 * xt.t.seg] = a;
                    tb.seg_val[2 * xt.t.seg + 1] = b;
                } else {
                    s[1] = fma(a, a, s[1]);
                    s[2] = fma(a, b, s[2]);
                    s[3] = fma(b, b, s[3]);
                }
            }
        }
        if (upd) st4<T>(azp, ck, j, av);
        // (z_y is not stored: the projection forms it again from u_y, v_s and A z)
    }
    if (!tw) return;
    const int64_t ntl = (int64_t)tb.nx_tiles + tb.ny_tiles, b = (int64_t)tb.nx_tiles + xt.index;
    if (cone) {
        block_sum4<VEC_NT>(s, sh);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) tb.tpart[j * ntl + b] = s[j];
        }
    } else {
        s[0] = block_sum<VEC_NT>(s[0], sh);
        if (threadIdx.x == 0) {
            if (cs.cone) tb.tpart[b] = s[0];
            else tb.ypart[4 * (int64_t)xt.index] = s[0];
        }
    }
}

// One CG step after the products: alpha = ||r||^2 / <p, q>; z += alpha p;
// r' = r - alpha q (and the carried K z, A z when tracking); then the next
// direction p = r' + beta p in the same pass.  beta needs ||r'||^2 before r'
// exists anywhere but in this kernel, so it is taken from the expansion
// ||r - alpha q||^2 = ||r||^2 - 2 alpha <r, q> + alpha^2 ||q||^2 of the FP64
// partials of k_cg_dot (the same quantity the method defines, evaluated
// without a second reduction pass); the stop test uses the same value.  Every
// workgroup sums the partials in the same fixed order.  The first tile's
// workgroup records alpha, beta, the counters and the run flag.
template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_cg_update(Tables tb, int z, int r, int p, int q, int it,
                                                      int cg_max, int gate, int track, int folded,
                                                      int last, CgStart cs) {
    __shared__ double sh[12 * (VEC_NT / 64)];
    const XYTile xt = xy_tile(tb);
    const InstDesc d = tb.inst[xt.t.inst];
    gptr<double> sc = scal(d);
    if (!gate_ok(sc, gate) || sc[SC_CGRUN] != (double)it) return;
    const bool rec = !xt.is_y && xt.index == d.xt0 && threadIdx.x == 0;
    double s[4];
    double h0 = 0.0, h1 = 0.0;
    if (folded) inst_csum4(tb, d, s, cs.on != 0, h0, h1, sh);   // partials of the A^T launch(es)
    else inst_xsum4(tb, d, s, sh);                              // partials of k_cg_dot
    double tol;
    if (cs.on) {
        // the step's CG start test, from the right-hand side launch's partials
        // ||r||^2, ||h||^2 (the products of this first iteration ran whatever
        // its outcome); every workgroup evaluates it
        tol = cg_tolerance(sc[SC_ITER], h1, cs.zeta, cs.rate, cs.floor_);
        const bool act = cg_max > 0 && sqrt(h0) > tol && std::isfinite(h0);
        if (rec) {
            sc[SC_RR] = h0;
            sc[SC_HN] = sqrt(h1);
            sc[SC_CGTOL] = tol;
            sc[SC_CGIT] = 0.0;
            sc[SC_CGACT] = act ? 1.0 : 0.0;
        }
        if (!act) {
            if (cs.tau) cg_elems<T>(tb, d, xt, sc, cs, false, 0.0, 0.0, false, false, true, z, r, p, q, sh);
            return;
        }
    } else {
        tol = sc[SC_CGTOL];
    }
    const double pq = s[0], rr = s[1], rq = s[2], qq = s[3];
    const double al = rr / pq;
    const bool ok = pq > 0.0 && std::isfinite(al);
    const double rr1 = fma(al * al, qq, fma(-2.0 * al, rq, rr));
    const double be = rr > 0.0 ? rr1 / rr : 0.0;
    const bool more = ok && std::isfinite(rr1) && sqrt(rr1) > tol && it + 1 < cg_max;
    if (rec) {
        sc[SC_PQ] = pq;
        sc[SC_ALPHA] = ok ? al : 0.0;
        sc[SC_RR] = ok ? rr1 : rr;
        sc[SC_BETA] = be;
        if (ok) {
            sc[SC_CGIT] += 1.0;
            sc[SC_CGTOT] += 1.0;
            if (sc[SC_CGIT] > sc[SC_CGMAX]) sc[SC_CGMAX] = sc[SC_CGIT];
            if (gate == G_SETUP) sc[SC_SETUPIT] += 1.0;
        }
        // the step's last CG launch, and CG would go on: the step needs more
        // launches than the interval has.  The instance is suspended (phase 3:
        // every later kernel of the interval skips it) until the host restores
        // the interval's snapshot and runs the interval again.
        if (last && more) sc[SC_PHASE] = 3.0;
        sc[SC_CGACT] = more ? 1.0 : 0.0;
    }
    // the step's last CG update also does the work of k_tau_dots on the final
    // z and A z (cs.tau: every instance's CG ends in an update of this loop)
    const bool tw = cs.tau && !more;
    if ((!ok || (xt.is_y && !track)) && !tw) return;
    cg_elems<T>(tb, d, xt, sc, cs, ok, al, be, more, track != 0, tw, z, r, p, q, sh);
}

template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_wy(Tables tb, int gate) {
    const VecTile tl = tb.yt[blockIdx.x];
    const InstDesc d = tb.inst[tl.inst];
    if (!gate_ok(scal(d), gate)) return;
    gptr<const T> u = yvec<T>(d, YU);
    gptr<const T> v = yvec<T>(d, YV);
    gptr<T> w = yvec<T>(d, YW);
    for (int64_t i = tl.start + threadIdx.x; i < tl.start + tl.len; i += VEC_NT)
        w[i] = (T)((double)u[i] + (double)v[i]);
}

// The products of u~_tau = (w_tau + c^T z_x + b^T z_y) / eta (exact solve of
// (I+Q) u~ = w, last row) after CG, on the one-launch-per-kernel path: the
// partials of c^T z_x and b^T z_y (z_y = w_y + carried A z), and the cone terms
// of the projection (the work the update that ends CG does on the folded path,
// with z and A z as CG left them; CgStart::cone)
template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_tau_dots(Tables tb, double alpha) {
    __shared__ double sh[4 * (VEC_NT / 64)];
    const XYTile xt = xy_tile(tb);
    const InstDesc d = tb.inst[xt.t.inst];
    gptr<double> sc = scal(d);
    if (!gate_ok(sc, G_ADMM)) return;
    const CgStart cs{0.0, 0.0, 0.0, 0, 1, 1, alpha};
    cg_elems<T>(tb, d, xt, sc, cs, false, 0.0, 0.0, false, false, true, XZ, XR, XP, XQ, sh);
}

// A thread's elements of a Y tile of u_y, A z, g_y, v_s, loaded at once
// (ahead of a reduction, and ahead of stores into the same vectors, which
// element by element would order each load after the previous stores);
// pv() is ybar_minus_v on them.
template <typename T>
struct YbarTile {
    static constexpr int R = VEC_TILE / VEC_NT;
    T u[R], a[R], g[R], v[R];
    DEVI void load(const InstDesc& d, const VecTile& tl) {
        gptr<const T> pu = yvec<T>(d, YU), pa = yvec<T>(d, YA), pg = yvec<T>(d, YG), pvv = yvec<T>(d, YV);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t o = threadIdx.x + (int64_t)j * VEC_NT;
            const int64_t i = tl.start + (o < tl.len ? o : 0);
            u[j] = pu[i];
            a[j] = pa[i];
            g[j] = pg[i];
            v[j] = pvv[i];
        }
    }
    DEVI bool has(const VecTile& tl, int j) const { return threadIdx.x + (int64_t)j * VEC_NT < tl.len; }
    DEVI int64_t at(const VecTile& tl, int j) const { return tl.start + threadIdx.x + (int64_t)j * VEC_NT; }
    DEVI double pv(int j, double ut, double alpha) const {
        const double uy = (double)u[j];
        const double ut_y = (double)z_y<T>(u[j], v[j], a[j]) - ut * (double)g[j];
        const double ub = alpha * ut_y + (1.0 - alpha) * uy;
        return ub - (double)v[j];
    }
};

template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_project(Tables tb, double alpha) {
    __shared__ double sh[4 * (VEC_NT / 64)];
    const XYTile xt = xy_tile(tb);
    const InstDesc d = tb.inst[xt.t.inst];
    gptr<double> sc = scal(d);
    if (!gate_ok(sc, G_ADMM)) return;
    const int seg = xt.is_y ? xt.t.seg : -1;
    YbarTile<T> yb;
    double ut, t = 0.0, nz = 0.0;
    {
        // u~_tau = (tau + kappa + c^T z_x + b^T z_y) / eta from the slot-0
        // partials (Tables::tpart) of every X and Y tile of the instance, and the cone's head
        // value and tail norm from the cone terms (CgStart::cone), all summed
        // in one fixed order by every workgroup
        const double* xp0 = tb.xpart + 4 * (int64_t)d.xt0;
        const double e_pt = xp0[1], wtau = xp0[2];
        const int64_t ntl = (int64_t)tb.nx_tiles + tb.ny_tiles;
        const double* ty = tb.tpart + tb.nx_tiles;   // slot 0 of the Y tiles
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        s[0] = thread_sum<VEC_NT, 4>(tb.tpart, d.xt0, d.xt1, 1) + thread_sum<VEC_NT, 4>(ty, d.yt0, d.yt1, 1);
        double ah = 0.0, bh = 0.0;
        if (seg >= 0) {
            const SocSeg sg = tb.seg[seg];
            ah = tb.seg_val[2 * seg];
            bh = tb.seg_val[2 * seg + 1];
#pragma unroll
            for (int j = 1; j < 4; ++j)
                s[j] = thread_sum<VEC_NT, 4>(ty + j * ntl, sg.yt0, sg.yt0 + sg.ntiles, 1);
        }
        block_sum4<VEC_NT>(s, sh);
        ut = (wtau + s[0]) / sc[SC_ETA];
        if (seg >= 0) {
            const double dl = ut - e_pt;
            t = ah - dl * bh;
            const double n2 = s[1] - 2.0 * dl * s[2] + dl * dl * s[3];
            nz = sqrt(n2 > 0.0 ? n2 : 0.0);
        }
    }
    if (!xt.is_y && xt.index == d.xt0 && threadIdx.x == 0) {
        // tau, kappa of the step (no other workgroup of this kernel reads them)
        sc[SC_UT] = ut;
        const double tau = sc[SC_TAU], kap = sc[SC_KAPPA];
        const double ubar = alpha * ut + (1.0 - alpha) * tau;
        const double tnew = ubar - kap > 0.0 ? ubar - kap : 0.0;
        sc[SC_KAPPA] = kap - ubar + tnew;
        sc[SC_TAU] = tnew;
        sc[SC_ITER] += 1.0;
    }
    const int64_t lo = xt.t.start, hi = xt.t.start + xt.t.len;
    if (!xt.is_y) {
        gptr<T> ux = xvec<T>(d, XU);
        gptr<const T> zx = xvec<T>(d, XZ);
        gptr<const T> gx = xvec<T>(d, XG);
        for (int64_t i = lo + threadIdx.x; i < hi; i += VEC_NT) {
            const double utx = (double)zx[i] - ut * (double)gx[i];
            ux[i] = (T)(alpha * utx + (1.0 - alpha) * (double)ux[i]);
        }
        return;
    }
    gptr<T> uy = yvec<T>(d, YU);
    gptr<T> vs = yvec<T>(d, YV);
    gptr<T> wy = yvec<T>(d, YW);
    if (seg < 0) {
        for (int64_t i = lo + threadIdx.x; i < hi; i += VEC_NT) {
            double ub;
            const double pv = ybar_minus_v<T>(d, i, ut, alpha, ub);
            const double pr = pv > 0.0 ? pv : 0.0;
            const T u = (T)pr, v = (T)(pr - pv);
            uy[i] = u;
            vs[i] = v;
            wy[i] = (T)((double)u + (double)v);
        }
        return;
    }
    const SocSeg sg = tb.seg[seg];
    yb.load(d, xt.t);
    // Pi(t, z): (t, z) if ||z|| <= t; 0 if ||z|| <= -t; ((t+||z||)/2)(1, z/||z||) otherwise
    int mode;
    double a = 0.0;
    if (nz <= t) mode = 0;
    else if (nz <= -t) mode = 1;
    else {
        mode = 2;
        a = 0.5 * (t + nz);
    }
#pragma unroll
    for (int j = 0; j < YbarTile<T>::R; ++j) {
        if (!yb.has(xt.t, j)) continue;
        const int64_t i = yb.at(xt.t, j);
        const double pv = yb.pv(j, ut, alpha);
        double pr;
        if (mode == 0) pr = pv;
        else if (mode == 1) pr = 0.0;
        else pr = (i == sg.start) ? a : (a / nz) * pv;
        const T u = (T)pr, v = (T)(pr - pv);
        uy[i] = u;
        vs[i] = v;
        wy[i] = (T)((double)u + (double)v);   // w_y of the next step
    }
}

// Termination test (relative 2-norm criteria, or the HSDE certificates), in
// the original problem's units: the row sums are divided by D, the column sums
// by E (sums listed at check_outcome).  YT holds A u_x and XT holds A^T u_y on entry.
template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_resid(Tables tb, double eps, int max_iters, int gate) {
    __shared__ double sh[VEC_NT / 64];
    const XYTile xt = xy_tile(tb);
    const InstDesc d = tb.inst[xt.t.inst];
    gptr<double> sc = scal(d);
    if (!gate_ok(sc, gate)) return;
    const double tau = sc[SC_TAU];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const int64_t lo = xt.t.start, hi = xt.t.start + xt.t.len;
    if (xt.is_y) {
        gptr<const T> au = yvec<T>(d, YT);
        gptr<const T> vs = yvec<T>(d, YV);
        gptr<const T> b = yvec<T>(d, YB);
        gptr<const T> uy = yvec<T>(d, YU);
        gptr<const T> dr = yvec<T>(d, YD);
        for (int64_t i = lo + threadIdx.x; i < hi; i += VEC_NT) {
            const double w = 1.0 / (double)dr[i];
            const double e = ((double)au[i] + (double)vs[i]) * w;
            const double rp = e - tau * (double)b[i] * w;
            s0 = fma(rp, rp, s0);
            s1 = fma(e, e, s1);
            s2 = fma((double)b[i], (double)uy[i], s2);
        }
    } else {
        gptr<const T> aty = xvec<T>(d, XT);
        gptr<const T> c = xvec<T>(d, XC);
        gptr<const T> ux = xvec<T>(d, XU);
        gptr<const T> ec = xvec<T>(d, XE);
        for (int64_t i = lo + threadIdx.x; i < hi; i += VEC_NT) {
            const double w = 1.0 / (double)ec[i];
            const double e = (double)aty[i] * w;
            const double rd = e + tau * (double)c[i] * w;
            s0 = fma(rd, rd, s0);
            s1 = fma(e, e, s1);
            s2 = fma((double)c[i], (double)ux[i], s2);
        }
    }
    s0 = block_sum<VEC_NT>(s0, sh);
    s1 = block_sum<VEC_NT>(s1, sh);
    s2 = block_sum<VEC_NT>(s2, sh);
    double* part = (xt.is_y ? tb.ypart : tb.xpart) + 4 * (int64_t)xt.index;
    if (threadIdx.x == 0) {
        part[0] = s0;
        part[1] = s1;
        part[2] = s2;
    }
}


// ---------------------------------------------------------------- per-instance finalize
// One workgroup per instance sums the partials of the kernel just before it in
// tile order and finishes the scalar work of the method.
enum FinMode : int {
    FIN_CG_INIT = 0,   // rr = ||r||^2, ||h||; CG tolerance and start flag
    FIN_RESID,         // residuals, gap, certificates, status
    FIN_NORMS,         // ||b||, ||c||
    FIN_ETA            // eta = 1 + c^T g_x + b^T g_y; phase -> iterating
};
struct FinArgs {
    double a0, a1, a2;
    int i0, i1;
};

__global__ __launch_bounds__(VEC_NT) void k_finalize(Tables tb, int mode, int gate, FinArgs fa) {
    __shared__ double sh[VEC_NT / 64];
    const InstDesc d = tb.inst[blockIdx.x];
    gptr<double> sc = scal(d);
    if (!gate_ok(sc, gate)) return;
    double x0 = 0, x1 = 0, x2 = 0, y0 = 0, y1 = 0, y2 = 0;
    const bool use_x = true;
    const bool use_y = mode == FIN_RESID || mode == FIN_NORMS || mode == FIN_ETA;
    const int nslot = (mode == FIN_RESID) ? 3 : (mode == FIN_CG_INIT ? 2 : 1);
    if (use_x) {
        x0 = sum_parts<VEC_NT>(tb.xpart, d.xt0, d.xt1, 0, sh);
        if (nslot > 1) x1 = sum_parts<VEC_NT>(tb.xpart, d.xt0, d.xt1, 1, sh);
        if (nslot > 2) x2 = sum_parts<VEC_NT>(tb.xpart, d.xt0, d.xt1, 2, sh);
    }
    if (use_y) {
        y0 = sum_parts<VEC_NT>(tb.ypart, d.yt0, d.yt1, 0, sh);
        if (nslot > 1) y1 = sum_parts<VEC_NT>(tb.ypart, d.yt0, d.yt1, 1, sh);
        if (nslot > 2) y2 = sum_parts<VEC_NT>(tb.ypart, d.yt0, d.yt1, 2, sh);
    }
    if (threadIdx.x != 0) return;
    switch (mode) {
        case FIN_CG_INIT: {
            const int cg_max = fa.i0;
            const double k = (gate == G_SETUP || gate == G_SETUP_CG) ? 0.0 : sc[SC_ITER];
            const double tol = cg_tolerance(k, x1, fa.a0, fa.a1, fa.a2);
            sc[SC_RR] = x0;
            sc[SC_HN] = sqrt(x1);
            sc[SC_CGTOL] = tol;
            sc[SC_CGIT] = 0.0;
            sc[SC_CGRUN] = -1.0;
            sc[SC_CGACT] = (cg_max > 0 && sqrt(x0) > tol && std::isfinite(x0)) ? 1.0 : 0.0;
            break;
        }
        case FIN_RESID: {
            const CheckOut co = check_outcome(sc, sc[SC_TAU], sc[SC_KAPPA], sc[SC_ITER], y0, y1, y2,
                                              x0, x1, x2, fa.a0, fa.i0);
            sc[SC_CUX] = co.cux;
            sc[SC_BUY] = co.buy;
            sc[SC_CGMAXLAST] = sc[SC_CGMAX];
            sc[SC_CGMAX] = 0.0;
            sc[SC_RP] = co.rp;
            sc[SC_RD] = co.rd;
            sc[SC_GAP] = co.gap;
            sc[SC_CX] = co.cx;
            sc[SC_BY] = co.by;
            if (co.status != 0.0) {
                sc[SC_STATUS] = co.status;
                sc[SC_ACTIVE] = 0.0;
            }
            break;
        }
        case FIN_NORMS:   // of the original b = b^ / (sb D) and c = c^ / (sc E)
            sc[SC_NB] = sqrt(y0) / sc[SC_SB];
            sc[SC_NC] = sqrt(x0) / sc[SC_SC];
            break;
        case FIN_ETA:
            sc[SC_ETA] = 1.0 + x0 + y0;
            sc[SC_PHASE] = d.fused ? 2.0 : 1.0;
            sc[SC_CGACT] = 0.0;
            break;
        default:
            break;
    }
}


// ---------------------------------------------------------------- setup
template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_reset(Tables tb, int only) {
    const XYTile xt = xy_tile(tb);
    if (only >= 0 && xt.t.inst != only) return;
    const InstDesc d = tb.inst[xt.t.inst];
    const int64_t lo = xt.t.start, hi = xt.t.start + xt.t.len;
    if (xt.is_y) {
        gptr<T> uy = yvec<T>(d, YU);
        gptr<T> vs = yvec<T>(d, YV);
        gptr<T> az = yvec<T>(d, YA);
        for (int64_t i = lo + threadIdx.x; i < hi; i += VEC_NT) {
            uy[i] = T(0);
            vs[i] = T(0);
            az[i] = T(0);
        }
    } else {
        gptr<T> ux = xvec<T>(d, XU);
        gptr<T> zx = xvec<T>(d, XZ);
        gptr<T> gx = xvec<T>(d, XG);
        gptr<T> kz = xvec<T>(d, XK);
        for (int64_t i = lo + threadIdx.x; i < hi; i += VEC_NT) {
            ux[i] = T(0);
            zx[i] = T(0);
            gx[i] = T(0);
            kz[i] = T(0);
        }
        if (xt.index == d.xt0 && threadIdx.x == 0) {
            gptr<double> sc = scal(d);
            const double sb = sc[SC_SB], scc = sc[SC_SC];   // data, like b and c
            for (int j = 0; j < NSC; ++j) sc[j] = 0.0;
            sc[SC_SB] = sb;
            sc[SC_SC] = scc;
            sc[SC_TAU] = 1.0;
            sc[SC_KAPPA] = 1.0;
            sc[SC_ACTIVE] = 1.0;
            sc[SC_PHASE] = 0.0;
            int* cn = counters(d);
            for (int j = 0; j < NCNT; ++j) cn[j] = 0;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_norms(Tables tb, int gate) {
    __shared__ double sh[VEC_NT / 64];
    const XYTile xt = xy_tile(tb);
    const InstDesc d = tb.inst[xt.t.inst];
    gptr<double> sc = scal(d);
    if (!gate_ok(sc, gate)) return;
    gptr<const T> v = xt.is_y ? yvec<T>(d, YB) : xvec<T>(d, XC);
    gptr<const T> w = xt.is_y ? yvec<T>(d, YD) : xvec<T>(d, XE);
    double s0 = 0.0;
    for (int64_t i = xt.t.start + threadIdx.x; i < xt.t.start + xt.t.len; i += VEC_NT) {
        const double e = (double)v[i] / (double)w[i];
        s0 = fma(e, e, s0);
    }
    s0 = block_sum<VEC_NT>(s0, sh);
    double* part = (xt.is_y ? tb.ypart : tb.xpart) + 4 * (int64_t)xt.index;
    if (threadIdx.x == 0) part[0] = s0;
}

// eta = 1 + c^T g_x + b^T g_y; the instance then starts iterating.
template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_eta(Tables tb) {
    __shared__ double sh[VEC_NT / 64];
    const XYTile xt = xy_tile(tb);
    const InstDesc d = tb.inst[xt.t.inst];
    gptr<double> sc = scal(d);
    if (!gate_ok(sc, G_SETUP)) return;
    gptr<const T> a = xt.is_y ? yvec<T>(d, YB) : xvec<T>(d, XC);
    gptr<const T> g = xt.is_y ? yvec<T>(d, YG) : xvec<T>(d, XG);
    double s0 = 0.0;
    for (int64_t i = xt.t.start + threadIdx.x; i < xt.t.start + xt.t.len; i += VEC_NT)
        s0 = fma((double)a[i], (double)g[i], s0);
    s0 = block_sum<VEC_NT>(s0, sh);
    double* part = (xt.is_y ? tb.ypart : tb.xpart) + 4 * (int64_t)xt.index;
    if (threadIdx.x == 0) part[0] = s0;
}

template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_fill(Tables tb, int is_y, int kind, double v, int gate) {
    const VecTile tl = is_y ? tb.yt[blockIdx.x] : tb.xt[blockIdx.x];
    const InstDesc d = tb.inst[tl.inst];
    if (!gate_ok(scal(d), gate)) return;
    gptr<T> o = is_y ? yvec<T>(d, kind) : xvec<T>(d, kind);
    for (int64_t i = tl.start + threadIdx.x; i < tl.start + tl.len; i += VEC_NT) o[i] = (T)v;
}

template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_copy(Tables tb, int is_y, int dst, int src, int gate) {
    const VecTile tl = is_y ? tb.yt[blockIdx.x] : tb.xt[blockIdx.x];
    const InstDesc d = tb.inst[tl.inst];
    if (!gate_ok(scal(d), gate)) return;
    gptr<T> o = is_y ? yvec<T>(d, dst) : xvec<T>(d, dst);
    gptr<const T> s = is_y ? yvec<T>(d, src) : xvec<T>(d, src);
    for (int64_t i = tl.start + threadIdx.x; i < tl.start + tl.len; i += VEC_NT) o[i] = s[i];
}

// Copy of the carried state of every instance that runs one launch per kernel
// (restore = 0: region -> copy; 1: copy -> region).  X tiles copy u_x, z, K z,
// Y tiles u_y, v_s, w_y, A z; the first X tile's workgroup also copies the
// header (scalars and counters).  Instances of the fused path, which runs
// concurrently on another stream, and instances without a copy are left alone.
template <typename T>
__global__ __launch_bounds__(VEC_NT) void k_snapshot(Tables tb, int restore) {
    const XYTile xt = xy_tile(tb);
    const InstDesc d = tb.inst[xt.t.inst];
    if (d.fused || d.snap == nullptr) return;
    gptr<char> region = (gptr<char>)d.base;
    gptr<char> copy = (gptr<char>)d.snap;
    if (!xt.is_y && xt.index == d.xt0) {
        gptr<const int64_t> hs = (gptr<const int64_t>)(restore ? copy : region);
        gptr<int64_t> hd = (gptr<int64_t>)(restore ? region : copy);
        for (int i = threadIdx.x; i < REGION_HDR / 8; i += VEC_NT) hd[i] = hs[i];
    }
    gptr<T> cx = (gptr<T>)(copy + REGION_HDR);
    gptr<T> cy = cx + (int64_t)SNAP_X * d.nxs;
    const int64_t lo = xt.t.start, hi = xt.t.start + xt.t.len;
    const int nv = xt.is_y ? SNAP_Y : SNAP_X;
    for (int v = 0; v < nv; ++v) {
        gptr<T> live = xt.is_y ? yvec<T>(d, v == 0 ? YU : YV) : xvec<T>(d, v == 0 ? XU : XZ);
        gptr<T> kept = xt.is_y ? cy + (int64_t)v * d.nys : cx + (int64_t)v * d.nxs;
        gptr<T> dst = restore ? live : kept;
        gptr<const T> src = restore ? kept : live;
        for (int64_t i = lo + threadIdx.x; i < hi; i += VEC_NT) dst[i] = src[i];
    }
}

// Points of the original problem (what 0: x, 1: y, 2: s; rays scaled by
// -c^T x_ray or -b^T y_ray for certificates) or the raw iterate (3: u_x,
// 4: u_y, 5: v_s) of the scaled problem.
template <typename T>
__global__ void k_extract(const InstDesc* insts, int inst, int what, int64_t off, int64_t len,
                          double* out) {
    const InstDesc d = insts[inst];
    gptr<const double> sc = scal(d);
    const double status = sc[SC_STATUS];
    double scale = 1.0;
    gptr<const T> v;
    gptr<const T> w = nullptr;
    bool divide = false;
    if (what == 0 || what == 3) v = xvec<T>(d, XU);
    else if (what == 1 || what == 4) v = yvec<T>(d, YU);
    else v = yvec<T>(d, YV);
    if (what <= 2) {
        double ray = sc[SC_TAU];   // x = x_ray / tau, ...
        if (status == 3.0) ray = (what == 1) ? -sc[SC_BUY] : NAN;
        else if (status == 4.0) ray = (what == 1) ? NAN : -sc[SC_CUX];
        if (what == 0) {          // x_ray = E u_x / sb
            w = xvec<T>(d, XE);
            scale = 1.0 / (sc[SC_SB] * ray);
        } else if (what == 1) {   // y_ray = D u_y / sc
            w = yvec<T>(d, YD);
            scale = 1.0 / (sc[SC_SC] * ray);
        } else {                  // s_ray = v_s / (D sb)
            w = yvec<T>(d, YD);
            divide = true;
            scale = 1.0 / (sc[SC_SB] * ray);
        }
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        double e = (double)v[off + i];
        if (w) e = divide ? e / (double)w[off + i] : e * (double)w[off + i];
        out[i] = e * scale;
    }
}

template <typename T>
__global__ void k_cast(const double* src, T* dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (T)src[i];
}

template <typename S, typename T>
__global__ void k_cast_pad(const S* src, int64_t lds, int64_t rows, int64_t cols, T* dst, int64_t ld) {
    const int64_t total = rows * ld;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / ld, c = i - r * ld;
        dst[i] = c < cols ? (T)(double)src[r * lds + c] : T(0);
    }
}

// 32x32 LDS-tiled transpose of a row chunk: dst[c * ldt + r0 + r] = src[r * lds + c]
template <typename S, typename T>
__global__ __launch_bounds__(256) void k_cast_transpose(const S* src, int64_t lds, int64_t rows,
                                                        int64_t cols, T* dst, int64_t ldt,
                                                        int64_t r0) {
    __shared__ double tile[32][33];
    const int64_t c_base = (int64_t)blockIdx.x * 32, r_base = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int j = ty; j < 32; j += 8) {
        const int64_t r = r_base + j, c = c_base + tx;
        tile[j][tx] = (r < rows && c < cols) ? (double)src[r * lds + c] : 0.0;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int64_t c = c_base + j, r = r_base + tx;
        if (c < cols && r < rows) dst[c * ldt + r0 + r] = (T)tile[tx][j];
    }
}

// Row sums of squares of a device matrix, one thread per row, each summed in
// column order (the host's order for a copied block); a non-finite entry
// raises *bad.  Rows [r0, r0 + nr) into out[0, nr).
template <typename S>
__global__ __launch_bounds__(256) void k_dense_rowsq(const S* a, int64_t lda, int64_t r0, int64_t nr,
                                                     int64_t cols, double* out, int* bad) {
    // products and sums rounded separately, as the host's (which has no FMA)
#pragma clang fp contract(off)
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const S* row = a + (r0 + r) * lda;
    double s = 0.0;
    bool fin = true;
    for (int64_t c = 0; c < cols; ++c) {
        const double v = (double)row[c];
        fin = fin && isfinite(v);
        s += v * v;
    }
    out[r] = s;
    if (!fin) atomicOr(bad, 1);
}

template <typename T>
__global__ void k_cast_back(const T* src, double* dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

// Gather every instance's scalar block into one contiguous array.
__global__ void k_gather_scalars(const InstDesc* insts, int ninst, double* out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ninst * NSC; i += gridDim.x * blockDim.x) {
        const int a = i / NSC, j = i - a * NSC;
        out[i] = reinterpret_cast<const double*>(insts[a].base)[j];
    }
}

// Write one scalar of one instance (host-side state changes).
__global__ void k_set_scalar(const InstDesc* insts, int inst, int slot, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) reinterpret_cast<double*>(insts[inst].base)[slot] = v;
}

// ---------------------------------------------------------------- launchers
#define CGS_DISPATCH(prec, KERNEL, grid, block, st, ...)                                 \
    do {                                                                                \
        if ((grid) > 0) {                                                               \
            if ((prec) == 0) KERNEL<double><<<(grid), (block), 0, (st)>>>(__VA_ARGS__);  \
            else KERNEL<float><<<(grid), (block), 0, (st)>>>(__VA_ARGS__);               \
        }                                                                               \
    } while (0)

static int flat_grid(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65535) g = 65535;
    return g < 1 ? 1 : (int)g;
}

void launch_apply_init(int prec, const Tables& t, int adj, int out, int in, int base,
                       double sigma, int gate, hipStream_t st) {
    CGS_DISPATCH(prec, k_apply_init, adj ? t.nx_tiles : t.ny_tiles, VEC_NT, st, t, adj, out, in,
                 base, sigma, gate);
}
void launch_conv(int prec, const Tables& t, const ConvLaunch& c, int adj, int out, int in, int base,
                 double sigma, int gate, hipStream_t st) {
    const int grid = c.ntiles + c.ninit;
    if (grid <= 0) return;
    const size_t lds = conv_smem_bytes(prec, c.kc);
    if (prec == 0) k_conv<double><<<grid, CONV_NT, lds, st>>>(t, c, adj, out, in, base, sigma, gate);
    else k_conv<float><<<grid, CONV_NT, lds, st>>>(t, c, adj, out, in, base, sigma, gate);
}
void launch_gemv(int prec, const Tables& t, const DenseLaunch& d, int adj, int out, int in,
                 double sigma, int gate, hipStream_t st) {
    CGS_DISPATCH(prec, k_gemv, d.ntiles, GEMV_NT, st, t, d, adj, out, in, sigma, gate);
}
void launch_cg_init(int prec, const Tables& t, int z, int r, int p, int q, int h, int have_q,
                    double zeta, double rate, double floor_, int cg_max, int gate, hipStream_t st) {
    CGS_DISPATCH(prec, k_cg_init, t.nx_tiles, VEC_NT, st, t, z, r, p, q, h, have_q, zeta, rate,
                 floor_, cg_max, gate);
    k_finalize<<<t.ninst, VEC_NT, 0, st>>>(t, FIN_CG_INIT, gate, FinArgs{zeta, rate, floor_, cg_max, 0});
}
void launch_cg_dot(int prec, const Tables& t, int p, int q, int r, int it, int gate, hipStream_t st) {
    CGS_DISPATCH(prec, k_cg_dot, t.nx_tiles, VEC_NT, st, t, p, q, r, it, gate);
}
void launch_cg_update(int prec, const Tables& t, int z, int r, int p, int q, int it, int cg_max,
                      int gate, int track, hipStream_t st, int folded, int last, CgStart cs) {
    // the update's own gate is the phase test of the CG gate plus the mark of k_cg_dot
    const int g = gate == G_ADMM_CG ? G_ADMM : gate == G_SETUP_CG ? G_SETUP : G_ALL;
    CGS_DISPATCH(prec, k_cg_update, t.nx_tiles + (track ? t.ny_tiles : 0), VEC_NT, st, t, z, r, p, q,
                 it, cg_max, g, track, folded, last, cs);
}
void launch_snapshot(int prec, const Tables& t, int restore, hipStream_t st) {
    CGS_DISPATCH(prec, k_snapshot, t.nx_tiles + t.ny_tiles, VEC_NT, st, t, restore);
}
void launch_wy(int prec, const Tables& t, int gate, hipStream_t st) {
    CGS_DISPATCH(prec, k_wy, t.ny_tiles, VEC_NT, st, t, gate);
}
void launch_tau_dots(int prec, const Tables& t, double alpha, hipStream_t st) {
    CGS_DISPATCH(prec, k_tau_dots, t.nx_tiles + t.ny_tiles, VEC_NT, st, t, alpha);
}
void launch_project(int prec, const Tables& t, double alpha, hipStream_t st) {
    CGS_DISPATCH(prec, k_project, t.nx_tiles + t.ny_tiles, VEC_NT, st, t, alpha);
}
void launch_resid(int prec, const Tables& t, double eps, int max_iters, int gate, hipStream_t st) {
    CGS_DISPATCH(prec, k_resid, t.nx_tiles + t.ny_tiles, VEC_NT, st, t, eps, max_iters, gate);
    k_finalize<<<t.ninst, VEC_NT, 0, st>>>(t, FIN_RESID, gate, FinArgs{eps, 0, 0, max_iters, 0});
}
void launch_reset(int prec, const Tables& t, int only, hipStream_t st) {
    CGS_DISPATCH(prec, k_reset, t.nx_tiles + t.ny_tiles, VEC_NT, st, t, only);
}
void launch_norms(int prec, const Tables& t, int gate, hipStream_t st) {
    CGS_DISPATCH(prec, k_norms, t.nx_tiles + t.ny_tiles, VEC_NT, st, t, gate);
    k_finalize<<<t.ninst, VEC_NT, 0, st>>>(t, FIN_NORMS, gate, FinArgs{0, 0, 0, 0, 0});
}
void launch_eta(int prec, const Tables& t, hipStream_t st) {
    CGS_DISPATCH(prec, k_eta, t.nx_tiles + t.ny_tiles, VEC_NT, st, t);
    k_finalize<<<t.ninst, VEC_NT, 0, st>>>(t, FIN_ETA, G_SETUP, FinArgs{0, 0, 0, 0, 0});
}
void launch_fill(int prec, const Tables& t, int is_y, int kind, double v, int gate,
                 hipStream_t st) {
    CGS_DISPATCH(prec, k_fill, is_y ? t.ny_tiles : t.nx_tiles, VEC_NT, st, t, is_y, kind, v, gate);
}
void launch_copy(int prec, const Tables& t, int is_y, int dst, int src, int gate, hipStream_t st) {
    CGS_DISPATCH(prec, k_copy, is_y ? t.ny_tiles : t.nx_tiles, VEC_NT, st, t, is_y, dst, src, gate);
}
void launch_extract(int prec, const InstDesc* inst_dev, int inst, int what, int64_t off,
                    int64_t len, double* out64, hipStream_t st) {
    CGS_DISPATCH(prec, k_extract, flat_grid(len, 256), 256, st, inst_dev, inst, what, off, len,
                 out64);
}
void launch_cast(int prec, const double* src, void* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    if (prec == 0) k_cast<double><<<flat_grid(n, 256), 256, 0, st>>>(src, (double*)dst, n);
    else k_cast<float><<<flat_grid(n, 256), 256, 0, st>>>(src, (float*)dst, n);
}
void launch_cast_pad(int prec, const void* src, int src_dtype, int64_t lds, int64_t rows, int64_t cols,
                     void* dst, int64_t ld, hipStream_t st) {
    if (rows <= 0) return;
    const unsigned g = flat_grid(rows * ld, 256);
    if (src_dtype == 0) {
        const double* s = (const double*)src;
        if (prec == 0) k_cast_pad<double, double><<<g, 256, 0, st>>>(s, lds, rows, cols, (double*)dst, ld);
        else k_cast_pad<double, float><<<g, 256, 0, st>>>(s, lds, rows, cols, (float*)dst, ld);
    } else {
        const float* s = (const float*)src;
        if (prec == 0) k_cast_pad<float, double><<<g, 256, 0, st>>>(s, lds, rows, cols, (double*)dst, ld);
        else k_cast_pad<float, float><<<g, 256, 0, st>>>(s, lds, rows, cols, (float*)dst, ld);
    }
}
void launch_cast_transpose(int prec, const void* src, int src_dtype, int64_t lds, int64_t rows,
                           int64_t cols, void* dst, int64_t ldt, int64_t r0, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return;
    dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    if (src_dtype == 0) {
        const double* s = (const double*)src;
        if (prec == 0) k_cast_transpose<double, double><<<grid, 256, 0, st>>>(s, lds, rows, cols, (double*)dst, ldt, r0);
        else k_cast_transpose<double, float><<<grid, 256, 0, st>>>(s, lds, rows, cols, (float*)dst, ldt, r0);
    } else {
        const float* s = (const float*)src;
        if (prec == 0) k_cast_transpose<float, double><<<grid, 256, 0, st>>>(s, lds, rows, cols, (double*)dst, ldt, r0);
        else k_cast_transpose<float, float><<<grid, 256, 0, st>>>(s, lds, rows, cols, (float*)dst, ldt, r0);
    }
}

int fail(int code, const char* fmt, ...);

// Output of k_dense_rowsq: a fixed device array (no allocation call), one
// user at a time per process (the mutex), addressed through
// hipGetSymbolAddress on the current device.
namespace {
constexpr int64_t ROWSQ_CHUNK = 65536;
__device__ double g_rowsq[ROWSQ_CHUNK];
__device__ int g_rowsq_bad;
std::mutex g_rowsq_mu;
}  // namespace

int dense_frob2_device(const void* a, int dtype, int64_t rows, int64_t cols, int64_t lda, double* frob2) {
    std::lock_guard<std::mutex> lock(g_rowsq_mu);
    double* out = nullptr;
    int* bad = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&out, HIP_SYMBOL(g_rowsq));
    if (e == hipSuccess) e = hipGetSymbolAddress((void**)&bad, HIP_SYMBOL(g_rowsq_bad));
    if (e != hipSuccess) return fail(CGS_EHIP, "hipGetSymbolAddress failed: %s", hipGetErrorString(e));
    std::vector<double> host((size_t)std::min<int64_t>(rows, ROWSQ_CHUNK));
    int flag = 0;
    e = hipMemcpy(bad, &flag, sizeof(int), hipMemcpyHostToDevice);
    double s = 0.0;
    for (int64_t r0 = 0; e == hipSuccess && r0 < rows; r0 += ROWSQ_CHUNK) {
        const int64_t nr = std::min(ROWSQ_CHUNK, rows - r0);
        const unsigned g = (unsigned)((nr + 255) / 256);
        if (dtype == 0) k_dense_rowsq<double><<<g, 256, 0, 0>>>((const double*)a, lda, r0, nr, cols, out, bad);
        else k_dense_rowsq<float><<<g, 256, 0, 0>>>((const float*)a, lda, r0, nr, cols, out, bad);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpy(host.data(), out, (size_t)nr * sizeof(double), hipMemcpyDeviceToHost);
        for (int64_t i = 0; e == hipSuccess && i < nr; ++i) s += host[(size_t)i];
    }
    if (e == hipSuccess) e = hipMemcpy(&flag, bad, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(CGS_EHIP, "dense block check failed: %s", hipGetErrorString(e));
    if (flag) return fail(CGS_EINVAL, "the dense block has a non-finite entry");
    *frob2 = s;
    return CGS_OK;
}
void launch_cast_back(int prec, const void* src, double* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    if (prec == 0) k_cast_back<double><<<flat_grid(n, 256), 256, 0, st>>>((const double*)src, dst, n);
    else k_cast_back<float><<<flat_grid(n, 256), 256, 0, st>>>((const float*)src, dst, n);
}
void launch_gather_scalars(const InstDesc* insts, int ninst, double* out, hipStream_t st) {
    if (ninst > 0) k_gather_scalars<<<flat_grid((int64_t)ninst * NSC, 256), 256, 0, st>>>(insts, ninst, out);
}
void launch_set_scalar(const InstDesc* insts, int inst, int slot, double v, hipStream_t st) {
    k_set_scalar<<<1, 64, 0, st>>>(insts, inst, slot, v);
}

}  // namespace cgs
