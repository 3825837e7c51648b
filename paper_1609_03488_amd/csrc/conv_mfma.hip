// FP32 convolution tiles on the matrix cores (v_mfma_f32_16x16x4_f32).
//
// The correlation form out[o] = sum_t w[t] in[o + off + t] of A x and A^T y is
// a dense contraction once the outputs are grouped in blocks of 16: with
// o = o0 + 16 b + a and the input offset s = a + t = 16 J + r (a, r < 16),
//
//     out[o0 + 16 b + a] = sum_J sum_r  w[16 J + r - a] * in[o0 + off + 16 (b + J) + r],
//
// i.e. C = sum_J T_J X_J with T_J[a][r] = w[16 J + r - a] (16 x 16 Toeplitz
// blocks of the taps, zero outside [0, k)) and X_J[r][b] the input shifted by
// J blocks.  A wave computes a 16 x 16 tile of C (256 consecutive outputs) with
// one 16x16x4 MFMA per (J, 4 values of r): K = 16 * (number of J) taps, about
// k + 30, so the extra work over the direct sum is a few percent for large k.
// A workgroup of two waves covers a 512-output tile (the tile tables of the
// VALU kernel); the input window is staged once per tap pass in LDS, stored
// with the 16 residues of an index in separate rows (row stride odd) so that the
// 16 lanes of a group read 16 consecutive words.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.hpp"
#include "device_common.hpp"

namespace cgs {

typedef float mf32x4 __attribute__((ext_vector_type(4)));

constexpr int CM_NT = 128;          // two waves
constexpr int CM_SUB = 256;         // outputs per wave
static_assert(CM_NT / 64 * CM_SUB == CONV_TILE_F32, "tile tables");

DEVI int cm_nj(int kc) { return (kc + 14) / 16 + 1; }          // J blocks of a pass of kc taps
DEVI int cm_stride(int nj) { const int q = nj + 31; return q | 1; }   // odd row stride

__global__ __launch_bounds__(CM_NT) void k_conv_mfma(Tables tb, ConvLaunch cl, int adj, int out, int in,
                                                     int base, double sigma, int gate) {
    extern __shared__ __align__(16) unsigned char cm_smem[];
    if ((int)blockIdx.x >= cl.ntiles) {   // initialisation tiles riding on the launch
        const VecTile it = cl.init[blockIdx.x - cl.ntiles];
        const InstDesc di = tb.inst[it.inst];
        if (gate_ok(scal(di), gate)) init_tile<float>(tb, di, it, adj, out, in, base, sigma);
        return;
    }
    const ConvTile tl = cl.tiles[blockIdx.x];
    const InstDesc d = tb.inst[tl.inst];
    if (!gate_ok(scal(d), gate)) return;
    const ConvBlock cb = cl.blocks[tl.blk];
    int64_t n_out, n_in, off;
    gptr<const float> w;
    gptr<float> o;
    gptr<const float> src;
    if (!adj) {
        n_out = cb.n_in + cb.k - 1;
        n_in = cb.n_in;
        off = -(cb.k - 1);
        w = (gptr<const float>)cb.w_fwd;
        o = yvec<float>(d, out) + cb.row0;
        src = xvec<float>(d, in) + cb.col0;
    } else {
        n_out = cb.n_in;
        n_in = cb.n_in + cb.k - 1;
        off = 0;
        w = (gptr<const float>)cb.w_adj;
        o = xvec<float>(d, out) + cb.col0;
        src = yvec<float>(d, in) + cb.row0;
    }
    const int tid = threadIdx.x, lane = tid & 63, sub = tid >> 6;
    const int g = lane >> 4, col = lane & 15;
    const int KC = cl.kc;
    const int njmax = cm_nj(KC);
    float* win = reinterpret_cast<float*>(cm_smem);          // 16 rows x stride
    float* tbuf = win + 16 * cm_stride(njmax);               // 16 * njmax + 32
    const int64_t ot = tl.start;
    mf32x4 acc0 = {}, acc1 = {};
    for (int64_t t0 = 0; t0 < cb.kpad; t0 += KC) {
        const int kc = (int)((cb.kpad - t0) < KC ? (cb.kpad - t0) : KC);
        const int nj = cm_nj(kc);
        const int S = cm_stride(nj);
        const int W = 16 * (nj + 31);
        const int TB = 16 * nj + 32;
        __syncthreads();
        const int64_t ws = ot + off + t0;
        for (int base = 0; base < W; base += 8 * CM_NT) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int p = base + j * CM_NT + tid;
                const int64_t gi = ws + p;
                v[j] = (p < W && gi >= 0 && gi < n_in) ? src[gi] : 0.0f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int p = base + j * CM_NT + tid;
                if (p < W) win[(p & 15) * S + (p >> 4)] = v[j];
            }
        }
        for (int base = 0; base < TB; base += 8 * CM_NT) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = base + j * CM_NT + tid;
                const int t = i - 16;
                v[j] = (i < TB && t >= 0 && t < kc) ? w[t0 + t] : 0.0f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = base + j * CM_NT + tid;
                if (i < TB) tbuf[i] = v[j];
            }
        }
        __syncthreads();
        // lane: A = T_J[a = col][r = r0 + g] = w[16 J + r0 + g - col];
        //       B = X_J[r = r0 + g][b = col]  = window[16 (16 sub + col + J) + r0 + g]
        const float* ta = tbuf + 16 + g - col;
        const float* xb = win + g * S + 16 * sub + col;
        int J = 0;
        for (; J + 1 < nj; J += 2) {
#pragma unroll
            for (int r0 = 0; r0 < 16; r0 += 4) {
                const float a0 = ta[16 * J + r0];
                const float b0 = xb[r0 * S + J];
                const float a1 = ta[16 * (J + 1) + r0];
                const float b1 = xb[r0 * S + J + 1];
                acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc1, 0, 0, 0);
            }
        }
        if (J < nj) {
#pragma unroll
            for (int r0 = 0; r0 < 16; r0 += 4)
                acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ta[16 * J + r0], xb[r0 * S + J], acc0, 0, 0, 0);
        }
    }
    // D[a][b]: a = 4 (lane / 16) + v, b = lane % 16 -> output o0 + 16 b + a
    const double s = sigma * cb.scale;
    const int64_t o0 = ot + CM_SUB * sub + 16 * col + 4 * g;
    if ((cb.own >> adj) & 1) {   // this block alone writes its outputs: final values
        const int64_t g0 = adj ? cb.col0 : cb.row0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t oi = o0 + v;
            if (oi < n_out)
                o[oi] = (float)(owned_init<float>(d, tb.ids, adj, out, in, base, sigma, g0 + oi) +
                                s * (double)(acc0[v] + acc1[v]));
        }
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t oi = o0 + v;
            if (oi < n_out) o[oi] = (float)((double)o[oi] + s * (double)(acc0[v] + acc1[v]));
        }
    }
}

size_t conv_mfma_smem_bytes(int kc) {
    const int nj = (kc + 14) / 16 + 1;
    const int S = (nj + 31) | 1;
    return (size_t)(16 * S + 16 * nj + 32) * sizeof(float);
}

void launch_conv_mfma(const Tables& t, const ConvLaunch& c, int adj, int out, int in, int base,
                      double sigma, int gate, hipStream_t st) {
    const int grid = c.ntiles + c.ninit;
    if (grid <= 0) return;
    k_conv_mfma<<<grid, CM_NT, conv_mfma_smem_bytes(c.kc), st>>>(t, c, adj, out, in, base, sigma, gate);
}

}  // namespace cgs
