// Batched dense-block applies as BF16 MFMA GEMMs (gfx950 v_mfma_f32_32x32x16_bf16).
//
// For B instances sharing one dense block W (N x K, row-major, K padded to a
// multiple of 16 with zeros) the apply out_b += s * W x_b of every instance is
// the product  C = X W^T  with X the B x K panel of the instances' input
// vectors.  Three kernels:
//   pack   : X as three BF16 panels (round to nearest even): hi, the BF16
//            rounding of the remainder (mid) and of what is left (lo), so that
//            hi + mid + lo carries the FP32 input to about 24 bits; rows padded
//            to a multiple of 64;
//   gemm   : split-K MFMA product, FP32 accumulation, FP32 partials per K split:
//            (X_hi + X_mid + X_lo) W_hi, a fixed linear map (the BF16 matrix) of
//            the FP32 input; with `corr` the products (X_hi + X_mid) W_lo are
//            added (matrix to about 16 bits);
//   reduce : out_b[n] += s * sum over K splits (fixed order), gated per instance.
// The order of the K terms inside a dot product is irrelevant to the result's
// definition, so each lane feeds the A (panel) and B (W) operands the same
// k indices: k0 + 8 * (lane / 32) + e, e = 0..7.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device_common.hpp"

namespace cgs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

DEVI uint16_t f32_to_bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
DEVI float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------- packed layouts
// Operands are stored in the order a wave feeds them to the MFMA: for a tile of
// 32 rows and a step of 16 k, lane l holds row (l % 32), k = 8 (l / 32) + e,
// e = 0..7, as one 16-byte vector; the 64 lanes' vectors of a (tile, step)
// are contiguous (1 KB), tiles are ksteps blocks apart.  Every operand load
// of a wave is then one fully coalesced 1 KB read.
DEVI int64_t packed_index(int64_t row, int64_t k, int64_t ksteps) {
    const int64_t t = row >> 5, ks = k >> 4, kk = k & 15;
    const int64_t lane = (row & 31) + 32 * (kk >> 3);
    return ((t * ksteps + ks) * 64 + lane) * 8 + (kk & 7);
}

// ---------------------------------------------------------------- pack
// Panels for b < mpad, k < kpad; instance b's input is its vector `in`
// (X when !adj, Y when adj) starting at `off`, K valid entries; zeros beyond.
// Blocks past the kblocks * mpad packing blocks are the output's
// initialisation tiles (base + identity blocks, as k_apply_init), which the
// apply's reduce then adds to: the output is not an input of the pack.
__global__ __launch_bounds__(256) void k_gemm_pack(Tables tb, int ninst, int adj, int in, int64_t off,
                                                    int64_t K, int64_t kpad, int kblocks, int mpad,
                                                    uint16_t* hi, uint16_t* mid, uint16_t* lo, int out,
                                                    int base, double sigma, int gate) {
    const int npack = kblocks * mpad;
    if ((int)blockIdx.x >= npack) {
        const int t = (int)blockIdx.x - npack;
        const VecTile tl = adj ? tb.xt[t] : tb.yt[t];
        const InstDesc d = tb.inst[tl.inst];
        if (gate_ok(scal(d), gate)) init_tile<float>(tb, d, tl, adj, out, in, base, sigma);
        return;
    }
    const int b = (int)blockIdx.x / kblocks;
    const int64_t k = (int64_t)((int)blockIdx.x % kblocks) * 256 + threadIdx.x;
    if (k >= kpad) return;
    float v = 0.0f;
    if (b < ninst && k < K) {
        const InstDesc d = tb.inst[b];
        gptr<const float> src = adj ? yvec<const float>(d, in) : xvec<const float>(d, in);
        v = src[off + k];
    }
    const uint16_t h = f32_to_bf16_rne(v);
    const float r1 = v - bf16_to_f32(h);           // exact in FP32
    const uint16_t md = f32_to_bf16_rne(r1);
    const int64_t i = packed_index(b, k, kpad / 16);
    hi[i] = h;
    mid[i] = md;
    lo[i] = f32_to_bf16_rne(r1 - bf16_to_f32(md));
}

// W (rows x ld FP32, row-major, ld = kpad) -> packed BF16 hi and lo (BF16
// rounding of the remainder), rows padded with zeros to a multiple of 32.
__global__ __launch_bounds__(256) void k_gemm_pack_w(const float* w, int64_t rows, int64_t kpad,
                                                      uint16_t* hi, uint16_t* lo) {
    const int64_t rpad = (rows + 31) / 32 * 32;
    const int64_t total = rpad * kpad;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / kpad, k = i - r * kpad;
        const float v = r < rows ? w[r * kpad + k] : 0.0f;
        const uint16_t h = f32_to_bf16_rne(v);
        const int64_t j = packed_index(r, k, kpad / 16);
        hi[j] = h;
        lo[j] = f32_to_bf16_rne(v - bf16_to_f32(h));
    }
}

// ---------------------------------------------------------------- gemm
// grid: (N tiles of 128, K splits, M tiles of 64); 4 waves, wave w owns the
// 32-column tile 4 blockIdx.x + w and both 32-row halves of the 64-row M tile.
// The six panel blocks of a K step (hi, mid, lo x two halves, 6 KB) are the
// same for the four waves: the workgroup stages them in LDS, GEMM_KC steps at
// a time in two buffers, loading chunk c + 1 (and each wave its W blocks of
// chunk c + 1) while the matrix cores work on chunk c.  Every wave reads W
// once; the panels cross from L2 once per workgroup instead of once per wave.
constexpr int GEMM_NT = 256;
constexpr int GEMM_TN = 128;
constexpr int GEMM_TM = 64;
constexpr int GEMM_KC = 4;
constexpr int GEMM_NPAN = 6;                          // (hi, mid, lo) x (rows 0-31, 32-63)
constexpr int GEMM_XCH = GEMM_KC * GEMM_NPAN * 64;    // 16-byte entries per chunk
static_assert(GEMM_XCH % GEMM_NT == 0, "chunk staging");

template <int CORR>
__global__ __launch_bounds__(GEMM_NT) void k_gemm_bf16(const uint16_t* __restrict__ w_hi,
                                                       const uint16_t* __restrict__ w_lo,
                                                       int64_t N, int64_t kpad,
                                                       const uint16_t* __restrict__ x_hi,
                                                       const uint16_t* __restrict__ x_mid,
                                                       const uint16_t* __restrict__ x_lo,
                                                       int ksteps_per_split,
                                                       float* __restrict__ part, int64_t npad,
                                                       int mpad) {
    __shared__ u16x8 xs[2][GEMM_XCH];   // [buffer][(kk * 6 + panel) * 64 + lane]
    constexpr int PER = GEMM_XCH / GEMM_NT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nt = (int64_t)blockIdx.x * (GEMM_TN / 32) + wave;
    const int s = blockIdx.y;
    const int mt0 = blockIdx.z * (GEMM_TM / 32);
    const int64_t ksteps = kpad / 16;
    const int64_t kstep0 = (int64_t)s * ksteps_per_split;
    int64_t kend = kstep0 + ksteps_per_split;
    if (kend > ksteps) kend = ksteps;
    const int nk = (int)(kend - kstep0);   // >= 1 (gemm_plan)
    const int nch = (nk + GEMM_KC - 1) / GEMM_KC;
    // tiles of W past the padded rows do not exist: clamp (their columns are
    // never reduced)
    const int64_t ntw = nt < (N + 31) / 32 ? nt : (N + 31) / 32 - 1;
    const u16x8* wh = reinterpret_cast<const u16x8*>(w_hi) + (ntw * ksteps + kstep0) * 64 + lane;
    const u16x8* wl = reinterpret_cast<const u16x8*>(w_lo) + (ntw * ksteps + kstep0) * 64 + lane;
    const u16x8* xsrc[3] = {reinterpret_cast<const u16x8*>(x_hi), reinterpret_cast<const u16x8*>(x_mid),
                            reinterpret_cast<const u16x8*>(x_lo)};
    // the entries this thread stages: chunk step kk, panel p, lane ln
    int64_t xoff[PER];
    int xkk[PER], xpn[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + GEMM_NT * i;
        xkk[i] = e / (GEMM_NPAN * 64);
        xpn[i] = (e / 64) % GEMM_NPAN;
        xoff[i] = ((int64_t)(mt0 + (xpn[i] & 1)) * ksteps + kstep0 + xkk[i]) * 64 + (e & 63);
    }
    u16x8 xr[PER], wc[GEMM_KC], wn[GEMM_KC], lc[GEMM_KC], ln[GEMM_KC];
    const u16x8 zero = {};
    auto load_chunk = [&](int c, u16x8* w, u16x8* l) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const bool ok = c * GEMM_KC + xkk[i] < nk;
            xr[i] = ok ? xsrc[xpn[i] >> 1][xoff[i] + (int64_t)c * GEMM_KC * 64] : zero;
        }
#pragma unroll
        for (int kk = 0; kk < GEMM_KC; ++kk) {
            const bool ok = c * GEMM_KC + kk < nk;
            const int64_t o = (int64_t)(c * GEMM_KC + kk) * 64;
            w[kk] = ok ? wh[o] : zero;
            if (CORR) l[kk] = ok ? wl[o] : zero;
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int i = 0; i < PER; ++i) xs[buf][threadIdx.x + GEMM_NT * i] = xr[i];
    };
    f32x16 acc0 = {}, acc1 = {};
    load_chunk(0, wc, lc);
    stage(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const bool more = c + 1 < nch;
        if (more) load_chunk(c + 1, wn, ln);
        const u16x8* xb = xs[c & 1];
#pragma unroll
        for (int kk = 0; kk < GEMM_KC; ++kk) {
            if (c * GEMM_KC + kk >= nk) break;
            const u16x8* q = xb + kk * GEMM_NPAN * 64 + lane;
            const bf16x8 h0 = __builtin_bit_cast(bf16x8, q[0 * 64]);
            const bf16x8 h1 = __builtin_bit_cast(bf16x8, q[1 * 64]);
            const bf16x8 m0 = __builtin_bit_cast(bf16x8, q[2 * 64]);
            const bf16x8 m1 = __builtin_bit_cast(bf16x8, q[3 * 64]);
            const bf16x8 l0 = __builtin_bit_cast(bf16x8, q[4 * 64]);
            const bf16x8 l1 = __builtin_bit_cast(bf16x8, q[5 * 64]);
            const bf16x8 bw = __builtin_bit_cast(bf16x8, wc[kk]);
            // smallest terms first
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(l0, bw, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(l1, bw, acc1, 0, 0, 0);
            if (CORR) {
                const bf16x8 bwl = __builtin_bit_cast(bf16x8, lc[kk]);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(m0, bwl, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(m1, bwl, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h0, bwl, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h1, bwl, acc1, 0, 0, 0);
            }
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(m0, bw, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(m1, bw, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h0, bw, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h1, bw, acc1, 0, 0, 0);
        }
        if (more) {
            stage((c + 1) & 1);
#pragma unroll
            for (int kk = 0; kk < GEMM_KC; ++kk) {
                wc[kk] = wn[kk];
                if (CORR) lc[kk] = ln[kk];
            }
        }
        // chunk c + 1 visible to every wave, and every wave done with the
        // buffer that chunk c + 2 overwrites
        __syncthreads();
    }
    // D layout of a 32x32 MFMA: column = lane % 32, row = 8 (v / 4) + 4 (lane / 32) + v % 4
    const int row = lane & 31, half = lane >> 5;
    const int64_t col = nt * 32 + row;
    const int m0r = mt0 * 32;
    float* p = part + (int64_t)s * mpad * npad;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int r = 8 * (v / 4) + 4 * half + (v % 4);
        p[(int64_t)(m0r + r) * npad + col] = acc0[v];
        p[(int64_t)(m0r + 32 + r) * npad + col] = acc1[v];
    }
}

// ---------------------------------------------------------------- reduce
__global__ __launch_bounds__(256) void k_gemm_reduce(const InstDesc* insts, int ninst, int adj, int out,
                                                      int64_t off, int64_t N, const float* part,
                                                      int nsplit, int64_t npad, int mpad, double s,
                                                      int gate_kind) {
    const int b = blockIdx.y;
    if (b >= ninst) return;
    const InstDesc d = insts[b];
    gptr<const double> sc = (gptr<const double>)d.base;
    bool on;
    switch (gate_kind) {
        case G_ALL: on = true; break;
        case G_SETUP: on = sc[SC_ACTIVE] != 0.0 && sc[SC_PHASE] == 0.0; break;
        case G_SETUP_CG: on = sc[SC_ACTIVE] != 0.0 && sc[SC_PHASE] == 0.0 && sc[SC_CGACT] != 0.0; break;
        case G_ADMM:
        case G_CHECK: on = sc[SC_ACTIVE] != 0.0 && sc[SC_PHASE] == 1.0; break;
        case G_ADMM_CG: on = sc[SC_ACTIVE] != 0.0 && sc[SC_PHASE] == 1.0 && sc[SC_CGACT] != 0.0; break;
        case G_ANY_CG: on = sc[SC_CGACT] != 0.0; break;
        case G_CHECK_ANY: on = sc[SC_ACTIVE] != 0.0 && sc[SC_PHASE] >= 1.0; break;
        default: on = false;
    }
    if (!on) return;
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    float acc = 0.0f;
    for (int q = 0; q < nsplit; ++q) acc += part[((int64_t)q * mpad + b) * npad + n];
    gptr<float> o = adj ? xvec<float>(d, out) : yvec<float>(d, out);
    o[off + n] = (float)((double)o[off + n] + s * (double)acc);
}

// ---------------------------------------------------------------- launchers
GemmPlan gemm_plan(int64_t N, int64_t kpad, int ninst, int target_wgs) {
    GemmPlan g{};
    g.mpad = (int)((ninst + GEMM_TM - 1) / GEMM_TM * GEMM_TM);
    g.ntiles = (int)((N + GEMM_TN - 1) / GEMM_TN);
    g.npad = (int64_t)g.ntiles * GEMM_TN;
    const int64_t ksteps = kpad / 16;
    const int mtiles = g.mpad / GEMM_TM;
    int64_t want = (int64_t)target_wgs / ((int64_t)g.ntiles * mtiles);
    if (want < 1) want = 1;
    if (want > ksteps) want = ksteps;
    if (want > 64) want = 64;
    g.ksteps_per_split = (int)((ksteps + want - 1) / want);
    g.nsplit = (int)((ksteps + g.ksteps_per_split - 1) / g.ksteps_per_split);
    return g;
}

size_t gemm_part_bytes(const GemmPlan& g) { return (size_t)g.nsplit * g.mpad * g.npad * sizeof(float); }

void launch_gemm_pack_w(const float* w, int64_t rows, int64_t kpad, uint16_t* hi, uint16_t* lo,
                        hipStream_t st) {
    const int64_t total = (rows + 31) / 32 * 32 * kpad;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    if (blocks > 0) k_gemm_pack_w<<<(unsigned)blocks, 256, 0, st>>>(w, rows, kpad, hi, lo);
}

void launch_gemm_apply(const Tables& tb, const DenseBlock& db, int adj, int out, int in, double sigma,
                       int gate, int corr, uint16_t* panel, size_t panel_stride, float* part,
                       int target_wgs, hipStream_t st, bool init, int base) {
    const InstDesc* insts = tb.inst;
    const int ninst = tb.ninst;
    uint16_t* panel_hi = panel;
    uint16_t* panel_mid = panel + panel_stride;
    uint16_t* panel_lo = panel + 2 * panel_stride;
    const int64_t N = adj ? db.cols : db.rows;        // outputs
    const int64_t K = adj ? db.rows : db.cols;        // inputs
    const int64_t kpad = adj ? db.ldt : db.ld;
    const uint16_t* w_hi = (const uint16_t*)(adj ? db.at16 : db.a16);
    const uint16_t* w_lo = (const uint16_t*)(adj ? db.at16lo : db.a16lo);
    const int64_t off_in = adj ? db.row0 : db.col0;
    const int64_t off_out = adj ? db.col0 : db.row0;
    const GemmPlan g = gemm_plan(N, kpad, ninst, target_wgs);
    const int kblocks = (int)((kpad + 255) / 256);
    const int ninit = init ? (adj ? tb.nx_tiles : tb.ny_tiles) : 0;
    k_gemm_pack<<<(unsigned)(kblocks * g.mpad + ninit), 256, 0, st>>>(
        tb, ninst, adj, in, off_in, K, kpad, kblocks, g.mpad, panel_hi, panel_mid, panel_lo, out, base,
        sigma, gate);
    dim3 gg((unsigned)g.ntiles, (unsigned)g.nsplit, (unsigned)(g.mpad / GEMM_TM));
    if (corr)
        k_gemm_bf16<1><<<gg, GEMM_NT, 0, st>>>(w_hi, w_lo, N, kpad, panel_hi, panel_mid, panel_lo,
                                               g.ksteps_per_split, part, g.npad, g.mpad);
    else
        k_gemm_bf16<0><<<gg, GEMM_NT, 0, st>>>(w_hi, w_lo, N, kpad, panel_hi, panel_mid, panel_lo,
                                               g.ksteps_per_split, part, g.npad, g.mpad);
    dim3 rg((unsigned)((N + 255) / 256), (unsigned)ninst);
    k_gemm_reduce<<<rg, 256, 0, st>>>(insts, ninst, adj, out, off_out, N, part, g.nsplit, g.npad, g.mpad,
                                      sigma * db.scale, gate);
}

}  // namespace cgs
