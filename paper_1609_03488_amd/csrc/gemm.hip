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

#include "kernels.hpp"

namespace cgs {

#define DEVI __device__ __forceinline__
template <typename T> using gptr = __attribute__((address_space(1))) T*;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

DEVI uint16_t f32_to_bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
DEVI float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename T>
DEVI gptr<T> xvec_g(const InstDesc& d, int k) {
    return (gptr<T>)(d.base + REGION_HDR) + (int64_t)k * d.nxs;
}
template <typename T>
DEVI gptr<T> yvec_g(const InstDesc& d, int k) {
    return (gptr<T>)(d.base + REGION_HDR) + (int64_t)NXV * d.nxs + (int64_t)k * d.nys;
}

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
__global__ __launch_bounds__(256) void k_gemm_pack(const InstDesc* insts, int ninst, int adj, int in,
                                                    int64_t off, int64_t K, int64_t kpad, int mpad,
                                                    uint16_t* hi, uint16_t* mid, uint16_t* lo) {
    const int b = blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= kpad) return;
    float v = 0.0f;
    if (b < ninst && k < K) {
        const InstDesc d = insts[b];
        gptr<const float> src = adj ? yvec_g<const float>(d, in) : xvec_g<const float>(d, in);
        v = src[off + k];
    }
    const uint16_t h = f32_to_bf16_rne(v);
    const float r1 = v - bf16_to_f32(h);           // exact in FP32
    const uint16_t md = f32_to_bf16_rne(r1);
    const int64_t i = packed_index(b, k, kpad / 16);
    hi[i] = h;
    mid[i] = md;
    lo[i] = f32_to_bf16_rne(r1 - bf16_to_f32(md));
    (void)mpad;
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
// Four K steps are loaded (1 KB per operand and step, coalesced) before their
// products are issued, so that 16-28 loads per lane are in flight.
constexpr int GEMM_NT = 256;
constexpr int GEMM_TN = 128;
constexpr int GEMM_TM = 64;
constexpr int GEMM_U = 4;

__global__ __launch_bounds__(GEMM_NT) void k_gemm_bf16(const uint16_t* __restrict__ w_hi,
                                                       const uint16_t* __restrict__ w_lo,
                                                       int64_t N, int64_t kpad,
                                                       const uint16_t* __restrict__ x_hi,
                                                       const uint16_t* __restrict__ x_mid,
                                                       const uint16_t* __restrict__ x_lo,
                                                       int ksteps_per_split, int corr,
                                                       float* __restrict__ part, int64_t npad,
                                                       int mpad) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nt = (int64_t)blockIdx.x * (GEMM_TN / 32) + wave;
    if (nt * 32 >= npad) return;
    const int s = blockIdx.y;
    const int mt0 = blockIdx.z * (GEMM_TM / 32);
    const int64_t ksteps = kpad / 16;
    const int64_t kstep0 = (int64_t)s * ksteps_per_split;
    int64_t kend = kstep0 + ksteps_per_split;
    if (kend > ksteps) kend = ksteps;
    // tiles of W past the padded rows do not exist: clamp (their columns are
    // never reduced)
    const int64_t ntw = nt < (N + 31) / 32 ? nt : (N + 31) / 32 - 1;
    const u16x8* wh = reinterpret_cast<const u16x8*>(w_hi) + ntw * ksteps * 64 + lane;
    const u16x8* wl = reinterpret_cast<const u16x8*>(w_lo) + ntw * ksteps * 64 + lane;
    const u16x8* xh0 = reinterpret_cast<const u16x8*>(x_hi) + (int64_t)mt0 * ksteps * 64 + lane;
    const u16x8* xm0 = reinterpret_cast<const u16x8*>(x_mid) + (int64_t)mt0 * ksteps * 64 + lane;
    const u16x8* xl0 = reinterpret_cast<const u16x8*>(x_lo) + (int64_t)mt0 * ksteps * 64 + lane;
    const int64_t mstride = ksteps * 64;   // next 32-row M tile
    f32x16 acc0 = {}, acc1 = {};
    int64_t ks = kstep0;
    for (; ks + GEMM_U <= kend; ks += GEMM_U) {
        u16x8 w[GEMM_U], wlo[GEMM_U], h0[GEMM_U], h1[GEMM_U], m0[GEMM_U], m1[GEMM_U], l0[GEMM_U],
            l1[GEMM_U];
#pragma unroll
        for (int u = 0; u < GEMM_U; ++u) {
            const int64_t o = (ks + u) * 64;
            w[u] = wh[o];
            if (corr) wlo[u] = wl[o];
            h0[u] = xh0[o];
            h1[u] = xh0[o + mstride];
            m0[u] = xm0[o];
            m1[u] = xm0[o + mstride];
            l0[u] = xl0[o];
            l1[u] = xl0[o + mstride];
        }
#pragma unroll
        for (int u = 0; u < GEMM_U; ++u) {
            const bf16x8 bw = __builtin_bit_cast(bf16x8, w[u]);
            // smallest terms first
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, l0[u]), bw, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, l1[u]), bw, acc1, 0, 0, 0);
            if (corr) {
                const bf16x8 bwl = __builtin_bit_cast(bf16x8, wlo[u]);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, m0[u]), bwl, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, m1[u]), bwl, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, h0[u]), bwl, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, h1[u]), bwl, acc1, 0, 0, 0);
            }
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, m0[u]), bw, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, m1[u]), bw, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, h0[u]), bw, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, h1[u]), bw, acc1, 0, 0, 0);
        }
    }
    for (; ks < kend; ++ks) {
        const int64_t o = ks * 64;
        const bf16x8 bw = __builtin_bit_cast(bf16x8, wh[o]);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xl0[o]), bw, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xl0[o + mstride]), bw, acc1, 0, 0, 0);
        if (corr) {
            const bf16x8 bwl = __builtin_bit_cast(bf16x8, wl[o]);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xm0[o]), bwl, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xm0[o + mstride]), bwl, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xh0[o]), bwl, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xh0[o + mstride]), bwl, acc1, 0, 0, 0);
        }
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xm0[o]), bw, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xm0[o + mstride]), bw, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xh0[o]), bw, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xh0[o + mstride]), bw, acc1, 0, 0, 0);
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
    gptr<float> o = adj ? xvec_g<float>(d, out) : yvec_g<float>(d, out);
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

void launch_gemm_apply(const InstDesc* insts, int ninst, const DenseBlock& db, int adj, int out, int in,
                       double sigma, int gate, int corr, uint16_t* panel, size_t panel_stride,
                       float* part, int target_wgs, hipStream_t st) {
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
    dim3 pg((unsigned)((kpad + 255) / 256), (unsigned)g.mpad);
    k_gemm_pack<<<pg, 256, 0, st>>>(insts, ninst, adj, in, off_in, K, kpad, g.mpad, panel_hi, panel_mid,
                                    panel_lo);
    dim3 gg((unsigned)g.ntiles, (unsigned)g.nsplit, (unsigned)(g.mpad / GEMM_TM));
    k_gemm_bf16<<<gg, GEMM_NT, 0, st>>>(w_hi, w_lo, N, kpad, panel_hi, panel_mid, panel_lo,
                                        g.ksteps_per_split, corr, part, g.npad, g.mpad);
    dim3 rg((unsigned)((N + 255) / 256), (unsigned)ninst);
    k_gemm_reduce<<<rg, 256, 0, st>>>(insts, ninst, adj, out, off_out, N, part, g.nsplit, g.npad, g.mpad,
                                      sigma * db.scale, gate);
}

}  // namespace cgs
