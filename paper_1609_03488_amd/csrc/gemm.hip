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

// ---------------------------------------------------------------- pack
// panel[b][k] for b < mpad, k < kpad; instance b's input is its vector `in`
// (X when !adj, Y when adj) starting at `off`, K valid entries.
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
    hi[(int64_t)b * kpad + k] = h;
    mid[(int64_t)b * kpad + k] = md;
    lo[(int64_t)b * kpad + k] = f32_to_bf16_rne(r1 - bf16_to_f32(md));
    (void)mpad;
}

// ---------------------------------------------------------------- gemm
// grid: (N tiles of 128, K splits, M tiles of 64); 4 waves, wave w owns columns
// [n0 + 32w, n0 + 32w + 32) and both 32-row halves of the 64-row M tile.
constexpr int GEMM_NT = 256;
constexpr int GEMM_TN = 128;
constexpr int GEMM_TM = 64;

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
    const int64_t n0 = (int64_t)blockIdx.x * GEMM_TN + wave * 32;
    const int s = blockIdx.y;
    const int m0 = blockIdx.z * GEMM_TM;
    const int64_t kstep0 = (int64_t)s * ksteps_per_split;
    const int64_t ksteps = kpad / 16;
    int64_t kend = kstep0 + ksteps_per_split;
    if (kend > ksteps) kend = ksteps;
    const int row = lane & 31, half = lane >> 5;
    // lanes past the last row of W read a valid row; their columns (>= N) are
    // never reduced
    const int64_t wn = (n0 + row < N) ? (n0 + row) : (N - 1);
    const u16x8* wh = reinterpret_cast<const u16x8*>(w_hi + wn * kpad) + half;
    const u16x8* wl = reinterpret_cast<const u16x8*>(w_lo + wn * kpad) + half;
    const u16x8* xh0 = reinterpret_cast<const u16x8*>(x_hi + (int64_t)(m0 + row) * kpad) + half;
    const u16x8* xh1 = reinterpret_cast<const u16x8*>(x_hi + (int64_t)(m0 + 32 + row) * kpad) + half;
    const u16x8* xm0 = reinterpret_cast<const u16x8*>(x_mid + (int64_t)(m0 + row) * kpad) + half;
    const u16x8* xm1 = reinterpret_cast<const u16x8*>(x_mid + (int64_t)(m0 + 32 + row) * kpad) + half;
    const u16x8* xl0 = reinterpret_cast<const u16x8*>(x_lo + (int64_t)(m0 + row) * kpad) + half;
    const u16x8* xl1 = reinterpret_cast<const u16x8*>(x_lo + (int64_t)(m0 + 32 + row) * kpad) + half;
    f32x16 acc0 = {}, acc1 = {};
    for (int64_t ks = kstep0; ks < kend; ++ks) {
        const int64_t o = ks * 2;   // 16 bf16 per step = two 8-element vectors
        const bf16x8 bw = __builtin_bit_cast(bf16x8, wh[o]);
        const bf16x8 a0 = __builtin_bit_cast(bf16x8, xh0[o]);
        const bf16x8 a1 = __builtin_bit_cast(bf16x8, xh1[o]);
        const bf16x8 a0m = __builtin_bit_cast(bf16x8, xm0[o]);
        const bf16x8 a1m = __builtin_bit_cast(bf16x8, xm1[o]);
        const bf16x8 a0l = __builtin_bit_cast(bf16x8, xl0[o]);
        const bf16x8 a1l = __builtin_bit_cast(bf16x8, xl1[o]);
        // smallest terms first
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0l, bw, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1l, bw, acc1, 0, 0, 0);
        if (corr) {
            const bf16x8 bwl = __builtin_bit_cast(bf16x8, wl[o]);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0m, bwl, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1m, bwl, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, bwl, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bwl, acc1, 0, 0, 0);
        }
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0m, bw, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1m, bw, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, bw, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bw, acc1, 0, 0, 0);
    }
    // D layout of a 32x32 MFMA: column = lane % 32, row = 8 (v / 4) + 4 (lane / 32) + v % 4
    const int64_t col = n0 + row;
    float* p = part + (int64_t)s * mpad * npad;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int r = 8 * (v / 4) + 4 * half + (v % 4);
        if (col < npad) {
            p[(int64_t)(m0 + r) * npad + col] = acc0[v];
            p[(int64_t)(m0 + 32 + r) * npad + col] = acc1[v];
        }
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
