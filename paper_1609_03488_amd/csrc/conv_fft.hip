// FP32 convolution tiles by FFT (overlap-save), for kernels of up to FFT_KMAX taps.
//
// The correlation form out[o] = sum_t w[t] in[o + off + t] of A x and A^T y
// (taps w of length k, zero beyond) is, for a window u[p] = in[o0 + off + p]
// of FFT_L = L inputs, the circular correlation of u with w at the positions
// p < B = L - k + 1, where no product wraps around.  The circular correlation
// is IDFT(DFT(u) . conj(DFT(w))); conj(DFT(w)) is computed once per block and
// direction when the operator is uploaded.  w is real, so the correlation maps
// real inputs to real outputs: two windows (outputs o0.. and o0 + B..) travel
// as the real and imaginary parts of one complex transform, and the real and
// imaginary parts of the result are their outputs.  The inverse transform is a
// forward one on the conjugate.
//
// Transforms: L = 2048 points in LDS, 256 threads, Stockham self-sorting
// stages of radix 8, 8, 8 and 4 (Govindaraju et al., "High performance
// discrete Fourier transforms on graphics processors", SC 2008); each thread
// keeps the 8 values of its butterflies in registers; the twiddles come from a
// table of the 2048 roots of unity (sincospi) that each workgroup builds in LDS
// first.  One workgroup per two output blocks (2B outputs).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.hpp"
#include "device_common.hpp"

namespace cgs {

namespace {

constexpr int FT = 256;   // threads per transform
static_assert(FFT_L == 2048 && FT * 8 == FFT_L, "transform shape");

struct cf {
    float x, y;
};
DEVI cf cmul(cf a, cf b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
DEVI cf cadd(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
DEVI cf csub(cf a, cf b) { return {a.x - b.x, a.y - b.y}; }
DEVI cf mul_mi(cf a) { return {a.y, -a.x}; }   // times -i

// 4- and 8-point DFTs (e^{-2 pi i n k / R}) in place, natural order
DEVI void dft4(cf* v) {
    const cf a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const cf a2 = cadd(v[1], v[3]), a3 = mul_mi(csub(v[1], v[3]));
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = cadd(a1, a3);
    v[3] = csub(a1, a3);
}
DEVI void dft8(cf* v) {
    cf e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft4(e);
    dft4(o);
    const float h = 0.70710678118654752f;
    const cf w1 = {h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};   // o1 e^{-i pi/4}
    const cf w2 = mul_mi(o[2]);                                     // o2 e^{-i pi/2}
    const cf w3 = {h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};  // o3 e^{-3i pi/4}
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], w1);
    v[5] = csub(e[1], w1);
    v[2] = cadd(e[2], w2);
    v[6] = csub(e[2], w2);
    v[3] = cadd(e[3], w3);
    v[7] = csub(e[3], w3);
}
// The transform's LDS array is padded by one entry per 32: the radix-8
// stores of a stage hit addresses 8 or 64 entries apart across the lanes of a
// wave, which without padding fall into the same few LDS banks.
constexpr int LDS_L = FFT_L + FFT_L / 32;
DEVI int lp(int i) { return i + (i >> 5); }

// Twiddle factors e^{-2 pi i m / FFT_L}, stored per stage in the order the
// lanes read them: entry (r - 1) * Ns + k holds the factor of butterfly input
// r for k = thread % Ns, so the lanes of a wave read consecutive entries (a
// table indexed by m would put the lanes of one stage 32 or 256 bytes apart,
// in the same few LDS banks).  Stages Ns = 8 and 64 (radix 8, m = r k FFT_L /
// (8 Ns)) and the radix-4 stage (m = r j, j < 512); every entry is the value
// the m-indexed table would hold.
constexpr int TW8 = 0, TW64 = 7 * 8, TW512 = TW64 + 7 * 64, TW_N = TW512 + 3 * 512;
DEVI int tw_index(int e) {   // entry -> m
    if (e < TW64) return ((e / 8 + 1) * (e % 8) * (FFT_L / 64)) & (FFT_L - 1);
    if (e < TW512) return (((e - TW64) / 64 + 1) * ((e - TW64) % 64) * (FFT_L / 512)) & (FFT_L - 1);
    return (((e - TW512) / 512 + 1) * ((e - TW512) % 512)) & (FFT_L - 1);
}
// filled by every workgroup (8 values per thread)
DEVI void fill_twiddles(cf* tw) {
#pragma unroll
    for (int r = 0; r < (TW_N + FT - 1) / FT; ++r) {
        const int e = threadIdx.x + FT * r;
        if (e >= TW_N) break;
        float s, c;
        sincospif(-2.0f * (float)tw_index(e) / (float)FFT_L, &s, &c);
        tw[e] = {c, s};
    }
}
// v[r] *= factor (r - 1) of the stage table `t` (stride n), r = 1 .. R-1
template <int R>
DEVI void twiddle(cf* v, const cf* t, int n) {
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], t[(r - 1) * n]);
}

// Forward DFT of the 2048 values x[t + 256 r] that thread t holds in v[r].
// On return thread t holds X[j + 512 r] (r = 0..3) in v[0..3] for j = t and
// in v[4..7] for j = t + 256.  lds: LDS_L entries (padded, lp); tw: the twiddle table (filled
// before a barrier the first stage passes); ends with a barrier.
DEVI void fft2048(cf* v, cf* lds, const cf* tw) {
    const int t = threadIdx.x;
    dft8(v);   // stage Ns = 1: outputs to 8 t + r
#pragma unroll
    for (int r = 0; r < 8; ++r) lds[lp(8 * t + r)] = v[r];
    __syncthreads();
#pragma unroll
    for (int Ns = 8; Ns <= 64; Ns *= 8) {
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = lds[lp(t + FT * r)];
        const int k = t % Ns;
        twiddle<8>(v, tw + (Ns == 8 ? TW8 : TW64) + k, Ns);
        dft8(v);
        __syncthreads();
        const int base = (t / Ns) * Ns * 8 + k;
#pragma unroll
        for (int r = 0; r < 8; ++r) lds[lp(base + r * Ns)] = v[r];
        __syncthreads();
    }
    // stage Ns = 512, radix 4: butterflies t and t + 256
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = t + FT * h;
        cf* w = v + 4 * h;
#pragma unroll
        for (int r = 0; r < 4; ++r) w[r] = lds[lp(j + 512 * r)];
        twiddle<4>(w, tw + TW512 + j, 512);
        dft4(w);
    }
    __syncthreads();
}

// The workgroup's partials of a folded CG step (every thread calls this).
DEVI void fold_partials(double* part, const Fold4& f, double* red) {
    double v[4] = {f.a, f.b, f.c, f.d};
    block_sum4<FT>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) part[4 * (int64_t)blockIdx.x + j] = v[j];
    }
}

}  // namespace

// conj(DFT(w zero-padded to FFT_L)) of k correlation-order taps
__global__ __launch_bounds__(FT) void k_conv_spectrum(const float* w, int k, float2* spec) {
    __shared__ cf lds[LDS_L];
    __shared__ cf tw[TW_N];
    const int t = threadIdx.x;
    fill_twiddles(tw);
    cf v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int i = t + FT * r;
        v[r] = {i < k ? w[i] : 0.0f, 0.0f};
    }
    fft2048(v, lds, tw);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) spec[t + FT * h + 512 * r] = make_float2(v[4 * h + r].x, -v[4 * h + r].y);
}

template <int FOLD>
__global__ __launch_bounds__(FT) void k_conv_fft(Tables tb, ConvLaunch cl, int adj, int out, int in, int base,
                                                 double sigma, int gate) {
    __shared__ cf lds[LDS_L];
    __shared__ cf tw[TW_N];
    __shared__ double red[4 * (FT / 64)];
    Fold4 f{0.0, 0.0, 0.0, 0.0};
    int bid = (int)blockIdx.x;
    if (FOLD == 0 && cl.pair) {
        // two applies in one launch: the second operand set's transform
        // workgroups follow the first set's, then both sets' initialisation
        // tiles in the same order
        bool second;
        if (bid < 2 * cl.nftiles) {
            second = bid >= cl.nftiles;
            bid -= second ? cl.nftiles : 0;
        } else {
            int w = bid - 2 * cl.nftiles;
            second = w >= cl.ninit;
            w -= second ? cl.ninit : 0;
            bid = cl.nftiles + w;
        }
        if (second) {
            out = cl.out2;
            in = cl.in2;
            base = cl.base2;
        }
    }
    if (bid >= cl.nftiles) {   // initialisation tiles riding on the launch
        const VecTile it = cl.init[bid - cl.nftiles];
        const InstDesc di = tb.inst[it.inst];
        if (!gate_ok(scal(di), gate)) return;
        init_tile<float, false>(tb, di, it, adj, out, in, base, sigma, FOLD, cl.fr, cl.fp, cl.fq, f,
                                FOLD == 1 ? cl.idrows : 0);
        if (FOLD) fold_partials(cl.part, f, red);
        return;
    }
    const ConvTile tl = cl.ftiles[bid];
    const InstDesc d = tb.inst[tl.inst];
    const ConvBlock cb = cl.blocks[tl.blk];   // (loaded beside the instance, ahead of the gate)
    if (!gate_ok(scal(d), gate)) return;
    if (FOLD == 2 && (int)blockIdx.x == d.cp0 && threadIdx.x == 0) scal(d)[SC_CGRUN] = (double)cl.fit;
    int64_t n_out, n_in, off;
    gptr<float> o;
    gptr<const float> src;
    const float2* spec;
    if (!adj) {
        n_out = cb.n_in + cb.k - 1;
        n_in = cb.n_in;
        off = -(cb.k - 1);
        spec = (const float2*)cb.s_fwd;
        o = yvec<float>(d, out) + cb.row0;
        src = xvec<float>(d, in) + cb.col0;
    } else {
        n_out = cb.n_in;
        n_in = cb.n_in + cb.k - 1;
        off = 0;
        spec = (const float2*)cb.s_adj;
        o = xvec<float>(d, out) + cb.col0;
        src = yvec<float>(d, in) + cb.row0;
    }
    const int t = threadIdx.x;
    const int B = FFT_L - (int)cb.k + 1;   // outputs per window
    const int64_t oa = tl.start;
    // the pair's inputs as 32-bit offsets q = p (window a) and B + p (window b)
    // from input position oa + off; valid offsets [qlo, qhi)
    const int64_t i0 = oa + off;
    const int qlo = i0 < 0 ? (int)-i0 : 0;
    const int qhi = n_in - i0 < FFT_L + B ? (int)(n_in - i0) : FFT_L + B;
    gptr<const float> sw = src + i0;
    cf v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int p = t + FT * r;
        v[r] = {(p >= qlo && p < qhi) ? sw[p] : 0.0f, (B + p >= qlo && B + p < qhi) ? sw[B + p] : 0.0f};
    }
    fill_twiddles(tw);
    fft2048(v, lds, tw);
    // product with conj(DFT(w)), conjugated: the inverse is a forward transform.
    // The thread holds X[t + 256 (h + 2 r)] in v[4 h + r], which is exactly
    // the set x[t + 256 r'] the next transform's first stage takes from it:
    // the products only change register, v'[r'] = p[4 (r' % 2) + r' / 2]
    // (no exchange through LDS; the transform ended with a barrier).
    gptr<const float> sp = (gptr<const float>)spec;   // interleaved (re, im)
    cf pr[8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = t + FT * h + 512 * r;
            const cf p = cmul(v[4 * h + r], cf{sp[2 * j], sp[2 * j + 1]});
            pr[h + 2 * r] = {p.x, -p.y};
        }
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = pr[r];
    fft2048(v, lds, tw);
    // conj(result) / L: real part = window a, imaginary part = window b.
    // Epilogue: every load of the thread's outputs (base, identity blocks,
    // folded operands) is issued before its first store; element by element
    // each load would wait for the previous element's stores, since they may
    // alias as far as the compiler knows.  The additions keep the order of the
    // element-wise form: (base + identity terms) + sum, then the fold.
    const double s = sigma * cb.scale / (double)FFT_L;
    const bool own = (cb.own >> adj) & 1;
    const int64_t g0 = adj ? cb.col0 : cb.row0;
    bool id_hit = false;     // an identity block adds to the workgroup's outputs
    for (int b = d.id0; b < d.id1; ++b) {
        const IdBlock ib = tb.ids[b];
        const int64_t r0 = adj ? ib.col0 : ib.row0;
        id_hit = id_hit || (ib.len > 0 && r0 < g0 + oa + 2 * (int64_t)B && r0 + ib.len > g0 + oa);
    }
    // Output positions as 32-bit offsets from the pair's first output oa
    // (window a: j, window b: B + j); offsets below nlim exist.  The block's
    // outputs start at g0 in the output vector.
    const int nlim = n_out - oa < 2 * (int64_t)B ? (int)(n_out - oa) : 2 * B;
    gptr<float> ow = o + oa;
    if (FOLD == 0 && own && base < 0 && !id_hit) {
        // nothing to load: the outputs are the sums alone
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = t + FT * h + 512 * r;
                if (j >= B) continue;
                if (j < nlim) ow[j] = (float)(0.0 + s * (double)v[4 * h + r].x);
                if (B + j < nlim) ow[B + j] = (float)(0.0 + s * -(double)v[4 * h + r].y);
            }
        return;
    }
    constexpr int NE = 16;   // two windows x 8 values
    // (-1: no output)
    int li[NE];
    double res[NE];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = 4 * h + r;
            const int j = t + FT * h + 512 * r;
            li[2 * e] = (j < B && j < nlim) ? j : -1;
            li[2 * e + 1] = (j < B && B + j < nlim) ? B + j : -1;
            res[2 * e] = (double)v[e].x;
            res[2 * e + 1] = -(double)v[e].y;
        }
    if (!own) {
        double old[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) old[e] = (double)ow[li[e] >= 0 ? li[e] : 0];
#pragma unroll
        for (int e = 0; e < NE; ++e)
            if (li[e] >= 0) ow[li[e]] = (float)(old[e] + s * res[e]);
        return;
    }
    const int64_t gw = g0 + oa;   // output vector position of offset 0
    // base + identity blocks of the owned range
    double bv[NE];
    float bl[NE];   // the base values as loaded (FOLD 2: the base is p)
    {
        // (loads are unconditional, at the pair's first output where the
        // thread has no output, so that none sits behind a branch)
        if (base >= 0) {
            gptr<const float> bp = (adj ? xvec<float>(d, base) : yvec<float>(d, base)) + gw;
#pragma unroll
            for (int e = 0; e < NE; ++e) bl[e] = bp[li[e] >= 0 ? li[e] : 0];
#pragma unroll
            for (int e = 0; e < NE; ++e) bv[e] = li[e] >= 0 ? (double)bl[e] : 0.0;
        } else {
#pragma unroll
            for (int e = 0; e < NE; ++e) bv[e] = 0.0;
        }
        gptr<const float> isrc = adj ? yvec<float>(d, in) : xvec<float>(d, in);
        for (int b = d.id0; b < d.id1; ++b) {
            const IdBlock ib = tb.ids[b];
            const int64_t r0 = adj ? ib.col0 : ib.row0;
            // blocks that miss the workgroup's outputs [oa, oa + 2B) issue no load
            if (ib.len <= 0 || r0 >= gw + 2 * (int64_t)B || r0 + ib.len <= gw) continue;
            const int64_t c0 = adj ? ib.row0 : ib.col0;
            const double w = sigma * ib.scale;
            // the block's rows as offsets, clamped to [0, 2B]
            const int64_t rl = r0 - gw, rh = r0 + ib.len - gw;
            const int lo = rl < 0 ? 0 : (int)rl;
            const int hi = rh > 2 * (int64_t)B ? 2 * B : (int)rh;
            gptr<const float> iw = isrc + (c0 - r0 + gw);
            float l[NE];
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const bool in_r = li[e] >= lo && li[e] < hi;
                l[e] = in_r ? iw[li[e]] : isrc[c0];
            }
#pragma unroll
            for (int e = 0; e < NE; ++e)
                if (li[e] >= lo && li[e] < hi) bv[e] += w * (double)l[e];
        }
    }
    if (FOLD == 0) {
#pragma unroll
        for (int e = 0; e < NE; ++e)
            if (li[e] >= 0) ow[li[e]] = (float)(bv[e] + s * res[e]);
        return;
    }
    // (a folded launch owns every X element)
    if (FOLD == 1) {
        // h = value; r = h - K z (and p = r when fp >= 0) written instead of h
        gptr<const float> kz = xvec<float>(d, cl.fq) + gw;
        float kv[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) kv[e] = kz[li[e] >= 0 ? li[e] : 0];
        gptr<float> rv = xvec<float>(d, cl.fr) + gw;
        gptr<float> pv = xvec<float>(d, cl.fp >= 0 ? cl.fp : cl.fr) + gw;   // (fp < 0: p is not written)
        float rrv[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            rrv[e] = 0.0f;
            if (li[e] < 0) continue;
            const float hv = (float)(bv[e] + s * res[e]);
            const double hd = (double)hv;
            const float rr = (float)(hd - (double)kv[e]);
            rrv[e] = rr;
            rv[li[e]] = rr;
            if (cl.fp >= 0) pv[li[e]] = rr;
            f.a += (double)rr * (double)rr;
            f.b += hd * hd;
        }
        if (cl.idrows) {
            // A p's identity rows for p = r: A's block maps X column col0 + i
            // to Y row row0 + i (ConvLaunch::idrows)
            gptr<float> yt = yvec<float>(d, cl.idrows - 1);
            for (int b = d.id0; b < d.id1; ++b) {
                const IdBlock ib = tb.ids[b];
                const int64_t rl = ib.col0 - gw, rh = ib.col0 + ib.len - gw;
                if (ib.len <= 0 || rh <= 0 || rl >= 2 * (int64_t)B) continue;
                const int lo = rl < 0 ? 0 : (int)rl;
                const int hi = rh > 2 * (int64_t)B ? 2 * B : (int)rh;
                gptr<float> yw = yt + (ib.row0 - ib.col0 + gw);
#pragma unroll
                for (int e = 0; e < NE; ++e)
                    if (li[e] >= lo && li[e] < hi) yw[li[e]] = (float)(0.0 + ib.scale * (double)rrv[e]);
            }
        }
    } else {
        // q = value; partials <p, q>, ||r||^2, <r, q>, ||q||^2.  p is the
        // launch's base (q = p + A^T A p), already loaded; r is p's vector in
        // a step's first iteration (p = r)
        const bool p_base = base == cl.fp, r_p = cl.fr == cl.fp;
        gptr<const float> pp = xvec<float>(d, cl.fp) + gw;
        gptr<const float> rp = xvec<float>(d, cl.fr) + gw;
        float pvv[NE], rvv[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) pvv[e] = p_base ? bl[e] : pp[li[e] >= 0 ? li[e] : 0];
        if (r_p) {
#pragma unroll
            for (int e = 0; e < NE; ++e) rvv[e] = pvv[e];
        } else {
#pragma unroll
            for (int e = 0; e < NE; ++e) rvv[e] = rp[li[e] >= 0 ? li[e] : 0];
        }
        gptr<float> qo = xvec<float>(d, out) + gw;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            if (li[e] < 0) continue;
            const float q = (float)(bv[e] + s * res[e]);
            qo[li[e]] = q;
            const double pd = (double)pvv[e], rd = (double)rvv[e], qd = (double)q;
            f.a = fma(pd, qd, f.a);
            f.b = fma(rd, rd, f.b);
            f.c = fma(rd, qd, f.c);
            f.d = fma(qd, qd, f.d);
        }
    }
    if (FOLD) fold_partials(cl.part, f, red);
}

void launch_conv_spectrum(const void* w, int64_t k, void* spec, hipStream_t st) {
    k_conv_spectrum<<<1, FT, 0, st>>>((const float*)w, (int)k, (float2*)spec);
}

void launch_conv_fft(const Tables& t, const ConvLaunch& c, int adj, int out, int in, int base, double sigma,
                     int gate, hipStream_t st) {
    const int grid = (c.nftiles + c.ninit) * (c.pair && c.fold == 0 ? 2 : 1);
    if (grid <= 0) return;
    if (c.fold == 1) k_conv_fft<1><<<grid, FT, 0, st>>>(t, c, adj, out, in, base, sigma, gate);
    else if (c.fold == 2) k_conv_fft<2><<<grid, FT, 0, st>>>(t, c, adj, out, in, base, sigma, gate);
    else k_conv_fft<0><<<grid, FT, 0, st>>>(t, c, adj, out, in, base, sigma, gate);
}

}  // namespace cgs
