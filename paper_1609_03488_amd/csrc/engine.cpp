// Host orchestration of the solver engine.
#include "engine.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace cgs {

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
const char* last_error() { return g_err.c_str(); }

// ---------------------------------------------------------------- validation
int validate_cone(int64_t m, int64_t l, const int64_t* q, int64_t nq) {
    if (l < 0 || nq < 0) return fail(CGS_ECONE, "negative cone count (l=%lld, nq=%lld)", (long long)l, (long long)nq);
    if (nq > 0 && q == nullptr) return fail(CGS_EINVAL, "q is null with nq=%lld", (long long)nq);
    int64_t tot = l;
    for (int64_t i = 0; i < nq; ++i) {
        if (q[i] < 1) return fail(CGS_ECONE, "second-order cone %lld has size %lld < 1", (long long)i, (long long)q[i]);
        tot += q[i];
    }
    if (tot != m)
        return fail(CGS_ECONE, "cones cover %lld rows but the operator has m=%lld", (long long)tot, (long long)m);
    return CGS_OK;
}

int validate_settings(const cgs_settings* s) {
    if (!s) return fail(CGS_EINVAL, "settings is null");
    if (!(s->eps > 0.0) || !std::isfinite(s->eps)) return fail(CGS_EINVAL, "eps must be finite and > 0");
    if (!(s->alpha > 0.0 && s->alpha < 2.0)) return fail(CGS_EINVAL, "alpha must lie in (0, 2)");
    if (s->max_iters < 1) return fail(CGS_EINVAL, "max_iters must be >= 1");
    if (s->check_every < 1) return fail(CGS_EINVAL, "check_every must be >= 1");
    if (s->precision < CGS_FP64 || s->precision > CGS_BF16) return fail(CGS_EINVAL, "unknown precision %d", s->precision);
    if (s->cg_max_iters < 1 || s->cg_max_iters > 10000) return fail(CGS_EINVAL, "cg_max_iters must be in [1, 10000]");
    if (!(s->cg_tol >= 0.0) || !(s->cg_rate >= 0.0) || !(s->cg_floor >= 0.0) ||
        !std::isfinite(s->cg_tol) || !std::isfinite(s->cg_rate) || !std::isfinite(s->cg_floor))
        return fail(CGS_EINVAL, "cg_tol, cg_rate, cg_floor must be finite and >= 0");
    if (!(s->setup_tol > 0.0) || !std::isfinite(s->setup_tol)) return fail(CGS_EINVAL, "setup_tol must be finite and > 0");
    if (s->setup_max_iters < 1) return fail(CGS_EINVAL, "setup_max_iters must be >= 1");
    if (s->bf16_phase1_digits < 0 || s->bf16_phase1_digits > 15)
        return fail(CGS_EINVAL, "bf16_phase1_digits must be in [0, 15]");
    if (s->normalize < 0 || s->normalize > 2) return fail(CGS_EINVAL, "normalize must be 0, 1 or 2");
    if (s->fused_max < 0 || s->fused_lone_max < 0) return fail(CGS_EINVAL, "fused_max, fused_lone_max must be >= 0");
    if (s->conv_mfma < 0 || s->conv_mfma > 2) return fail(CGS_EINVAL, "conv_mfma must be 0, 1 or 2");
    if (s->intervals_per_sync < 1 || s->intervals_per_sync > 64)
        return fail(CGS_EINVAL, "intervals_per_sync must be in [1, 64]");
    if (s->vec_tile != 0 && s->vec_tile != VEC_TILE_MIN && s->vec_tile != VEC_TILE)
        return fail(CGS_EINVAL, "vec_tile must be 0, %d or %d", VEC_TILE_MIN, VEC_TILE);
    return CGS_OK;
}

// ---------------------------------------------------------------- layouts
static int64_t conv_r(int precision) { return precision == CGS_FP64 ? CONV_R_F64 : CONV_R_F32; }
static int64_t conv_tile(int precision) { return precision == CGS_FP64 ? CONV_TILE_F64 : CONV_TILE_F32; }
static int64_t dense_ld(int64_t cols) { return round_up(cols, 16); }   // K of the MFMA steps

int64_t staging_doubles(const cgs_op& op, int64_t max_vec) {
    int64_t need = std::max<int64_t>(max_vec, int64_t(1) << 16);
    for (const auto& b : op.blocks) {
        if (b.kind == CGS_BLOCK_CONV) need = std::max<int64_t>(need, 2 * round_up(b.k, 8));
        if (b.kind == CGS_BLOCK_DENSE && b.dev == nullptr) {   // (a borrowed block needs none)
            need = std::max<int64_t>(need, std::min<int64_t>(b.rows * b.cols, int64_t(4) << 20));
            need = std::max<int64_t>(need, b.cols);
        }
    }
    return need;
}

size_t region_bytes(int64_t n, int64_t m, int precision) {
    const size_t sz = elem_bytes(precision);
    return align256(REGION_HDR + (size_t)NXV * round_up(n, XY_ALIGN) * sz +
                    (size_t)NYV * round_up(m, XY_ALIGN) * sz);
}

size_t snap_bytes(int64_t n, int64_t m, int precision) {
    const size_t sz = elem_bytes(precision);
    return align256(REGION_HDR + (size_t)SNAP_X * round_up(n, XY_ALIGN) * sz +
                    (size_t)SNAP_Y * round_up(m, XY_ALIGN) * sz);
}

size_t op_dev_bytes(const cgs_op& op, int precision) {
    const size_t sz = elem_bytes(precision);
    size_t tot = 0;
    for (const auto& b : op.blocks) {
        if (b.kind == CGS_BLOCK_CONV) {
            tot += 2 * align256(round_up(b.k, conv_r(precision)) * sz);
            if (work_prec(precision) == 1 && b.k <= FFT_KMAX) tot += 2 * align256((size_t)FFT_L * 8);
        }
        if (b.kind == CGS_BLOCK_DENSE) {
            const size_t ld = dense_ld(b.cols), ldt = dense_ld(b.rows);
            tot += align256(b.rows * ld * sz) + align256(b.cols * ldt * sz);
            if (precision == CGS_BF16)   // packed MFMA operands, rows padded to 32
                tot += 2 * (align256(round_up(b.rows, 32) * ld * 2) + align256(round_up(b.cols, 32) * ldt * 2));
        }
    }
    return tot;
}

// ---------------------------------------------------------------- equilibration
namespace {
// Contiguous groups of [0, len): intervals that share a position merge;
// uncovered runs are groups of their own.  Returns the group starts (+ len).
std::vector<int64_t> partition(int64_t len, std::vector<std::pair<int64_t, int64_t>> iv) {
    std::sort(iv.begin(), iv.end());
    std::vector<std::pair<int64_t, int64_t>> merged;
    for (const auto& p : iv) {
        if (p.second <= p.first) continue;
        if (!merged.empty() && p.first < merged.back().second)
            merged.back().second = std::max(merged.back().second, p.second);
        else
            merged.push_back(p);
    }
    std::vector<int64_t> lo;
    int64_t pos = 0;
    for (const auto& p : merged) {
        if (p.first > pos) lo.push_back(pos);
        lo.push_back(p.first);
        pos = p.second;
    }
    if (pos < len || lo.empty()) lo.push_back(pos);
    lo.push_back(len);
    return lo;
}
int group_of(const std::vector<int64_t>& lo, int64_t i) {
    return (int)(std::upper_bound(lo.begin(), lo.end(), i) - lo.begin()) - 1;
}
}  // namespace

void compute_scaling(const cgs_op& op, int64_t l, const int64_t* q, int64_t nq, int level,
                     Scaling* out) {
    const int kPasses = level >= 2 ? 20 : 0;
    const bool on = level >= 1;
    constexpr double kMin = 1e-4, kMax = 1e4;
    std::vector<std::pair<int64_t, int64_t>> rows, cols;
    for (const auto& b : op.blocks) {
        rows.emplace_back(b.row0, b.row0 + b.rows);
        cols.emplace_back(b.col0, b.col0 + b.cols);
    }
    int64_t start = l;
    for (int64_t i = 0; i < nq; ++i) {
        rows.emplace_back(start, start + q[i]);
        start += q[i];
    }
    out->row_lo = partition(op.m, rows);
    out->col_lo = partition(op.n, cols);
    const int p = (int)out->row_lo.size() - 1, r = (int)out->col_lo.size() - 1;
    out->d.assign(p, 1.0);
    out->e.assign(r, 1.0);
    out->blk.assign(op.blocks.size(), 1.0);
    out->mean_row = out->mean_col = 1.0;
    out->on = on;
    if (!on) return;
    std::vector<int> bg(op.blocks.size()), bh(op.blocks.size());
    std::vector<double> F((size_t)p * r, 0.0), R(p), Cn(r);
    for (size_t k = 0; k < op.blocks.size(); ++k) {
        const HostBlock& b = op.blocks[k];
        bg[k] = group_of(out->row_lo, b.row0);
        bh[k] = group_of(out->col_lo, b.col0);
        F[(size_t)bg[k] * r + bh[k]] += b.frob2 * b.scale * b.scale;
    }
    for (int g = 0; g < p; ++g) R[g] = (double)(out->row_lo[g + 1] - out->row_lo[g]);
    for (int h = 0; h < r; ++h) Cn[h] = (double)(out->col_lo[h + 1] - out->col_lo[h]);
    std::vector<double>& D = out->d;
    std::vector<double>& E = out->e;
    auto row_rms = [&](int g) {
        double s = 0.0;
        for (int h = 0; h < r; ++h) s += F[(size_t)g * r + h] * E[h] * E[h];
        return std::sqrt(D[g] * D[g] * s / R[g]);
    };
    auto col_rms = [&](int h) {
        double s = 0.0;
        for (int g = 0; g < p; ++g) s += F[(size_t)g * r + h] * D[g] * D[g];
        return std::sqrt(E[h] * E[h] * s / Cn[h]);
    };
    for (int pass = 0; pass < kPasses; ++pass) {
        std::vector<double> rho(p), gam(r);
        for (int g = 0; g < p; ++g) rho[g] = row_rms(g);
        for (int g = 0; g < p; ++g)
            if (rho[g] > 0.0) D[g] /= std::sqrt(std::min(std::max(rho[g], kMin), kMax));
        for (int h = 0; h < r; ++h) gam[h] = col_rms(h);
        for (int h = 0; h < r; ++h)
            if (gam[h] > 0.0) E[h] /= std::sqrt(std::min(std::max(gam[h], kMin), kMax));
    }
    double mr = 0.0, mc = 0.0;
    for (int g = 0; g < p; ++g) mr += R[g] * row_rms(g);
    for (int h = 0; h < r; ++h) mc += Cn[h] * col_rms(h);
    out->mean_row = mr / (double)op.m;
    out->mean_col = mc / (double)op.n;
    for (size_t k = 0; k < op.blocks.size(); ++k) out->blk[k] = D[bg[k]] * E[bh[k]];
}

void scale_data(const Scaling& s, int64_t m, int64_t n, const double* b, const double* c,
                double* dv, double* ev, double* bh, double* ch, double* sb, double* sc) {
    for (size_t g = 0; g + 1 < s.row_lo.size(); ++g)
        for (int64_t i = s.row_lo[g]; i < s.row_lo[g + 1]; ++i) dv[i] = s.d[g];
    for (size_t h = 0; h + 1 < s.col_lo.size(); ++h)
        for (int64_t j = s.col_lo[h]; j < s.col_lo[h + 1]; ++j) ev[j] = s.e[h];
    double nb = 0.0, nc = 0.0;
    for (int64_t i = 0; i < m; ++i) nb += (dv[i] * b[i]) * (dv[i] * b[i]);
    for (int64_t j = 0; j < n; ++j) nc += (ev[j] * c[j]) * (ev[j] * c[j]);
    constexpr double kDataMin = 1e-4;
    *sb = s.on ? s.mean_row / std::max(std::sqrt(nb), kDataMin) : 1.0;
    *sc = s.on ? s.mean_col / std::max(std::sqrt(nc), kDataMin) : 1.0;
    for (int64_t i = 0; i < m; ++i) bh[i] = *sb * dv[i] * b[i];
    for (int64_t j = 0; j < n; ++j) ch[j] = *sc * ev[j] * c[j];
}

void op_dev_shape(const cgs_op& op, int precision, OpDev* out, const double* mult) {
    out->ids.clear();
    out->convs.clear();
    out->dense.clear();
    size_t bi = 0;
    for (const auto& b : op.blocks) {
        const double scale = b.scale * (mult ? mult[bi] : 1.0);
        ++bi;
        if (b.kind == CGS_BLOCK_IDENTITY) {
            out->ids.push_back(IdBlock{b.row0, b.col0, b.rows, scale});
        } else if (b.kind == CGS_BLOCK_CONV) {
            ConvBlock cb{};
            cb.row0 = b.row0;
            cb.col0 = b.col0;
            cb.n_in = b.n_in;
            cb.k = b.k;
            cb.kpad = round_up(b.k, conv_r(precision));
            cb.scale = scale;
            out->convs.push_back(cb);
        } else {
            DenseBlock db{};
            db.row0 = b.row0;
            db.col0 = b.col0;
            db.rows = b.rows;
            db.cols = b.cols;
            db.ld = dense_ld(b.cols);
            db.ldt = dense_ld(b.rows);
            db.scale = scale;
            out->dense.push_back(db);
        }
    }
    // a convolution owns its output range in a direction when no other
    // convolution or dense block writes into it (identity blocks may)
    auto overlap = [](int64_t a0, int64_t a1, int64_t b0, int64_t b1) { return a0 < b1 && b0 < a1; };
    for (size_t i = 0; i < out->convs.size(); ++i) {
        ConvBlock& c = out->convs[i];
        const int64_t r0 = c.row0, r1 = c.row0 + c.n_in + c.k - 1, c0 = c.col0, c1 = c.col0 + c.n_in;
        bool fwd = true, adj = true;
        for (size_t j = 0; j < out->convs.size(); ++j) {
            if (j == i) continue;
            const ConvBlock& o = out->convs[j];
            if (overlap(r0, r1, o.row0, o.row0 + o.n_in + o.k - 1)) fwd = false;
            if (overlap(c0, c1, o.col0, o.col0 + o.n_in)) adj = false;
        }
        for (const DenseBlock& o : out->dense) {
            if (overlap(r0, r1, o.row0, o.row0 + o.rows)) fwd = false;
            if (overlap(c0, c1, o.col0, o.col0 + o.cols)) adj = false;
        }
        c.own = (fwd ? 1 : 0) | (adj ? 2 : 0);
    }
}

int op_upload(const cgs_op& op, int precision, char* dst, const Staging& stg, hipStream_t st,
              OpDev* out, const double* mult) {
    op_dev_shape(op, precision, out, mult);
    const int prec = work_prec(precision);
    const size_t sz = elem_bytes(precision);
    char* p = dst;
    size_t ci = 0, di = 0;
    for (const auto& b : op.blocks) {
        if (b.kind == CGS_BLOCK_CONV) {
            ConvBlock& cb = out->convs[ci++];
            const int64_t kpad = cb.kpad, k = cb.k;
            if (2 * kpad > stg.cap) return fail(CGS_ENOMEM, "staging too small for %lld taps", (long long)k);
            for (int64_t t = 0; t < kpad; ++t) {
                stg.host[t] = t < k ? b.data[k - 1 - t] : 0.0;   // correlation order of A x
                stg.host[kpad + t] = t < k ? b.data[t] : 0.0;    // correlation order of A^T y
            }
            CGS_HIP(hipMemcpyAsync(stg.dev, stg.host, 2 * kpad * sizeof(double), hipMemcpyHostToDevice, st));
            cb.w_fwd = p;
            launch_cast(prec, stg.dev, p, kpad, st);
            p += align256(kpad * sz);
            cb.w_adj = p;
            launch_cast(prec, stg.dev + kpad, p, kpad, st);
            p += align256(kpad * sz);
            if (prec == 1 && k <= FFT_KMAX) {   // spectra for the FFT engine
                cb.s_fwd = p;
                launch_conv_spectrum(cb.w_fwd, k, p, st);
                p += align256((size_t)FFT_L * 8);
                cb.s_adj = p;
                launch_conv_spectrum(cb.w_adj, k, p, st);
                p += align256((size_t)FFT_L * 8);
            }
            CGS_HIP(hipStreamSynchronize(st));
        } else if (b.kind == CGS_BLOCK_DENSE) {
            DenseBlock& db = out->dense[di++];
            const int64_t rows = db.rows, cols = db.cols, ld = db.ld, ldt = db.ldt;
            db.a = p;
            p += align256(rows * ld * sz);
            db.at = p;
            p += align256(cols * ldt * sz);
            CGS_HIP(hipMemsetAsync(const_cast<void*>(db.at), 0, cols * ldt * sz, st));
            if (b.dev != nullptr) {
                // borrowed device memory: converted in place, no host round trip
                int cur = -1;
                CGS_HIP(hipGetDevice(&cur));
                if (cur != b.dev_id)
                    return fail(CGS_EINVAL, "a borrowed dense block lives on device %d, the solver on %d",
                                b.dev_id, cur);
                launch_cast_pad(prec, b.dev, b.dev_dtype, b.dev_ld, rows, cols, const_cast<void*>(db.a), ld, st);
                launch_cast_transpose(prec, b.dev, b.dev_dtype, b.dev_ld, rows, cols, const_cast<void*>(db.at),
                                      ldt, 0, st);
                CGS_HIP(hipStreamSynchronize(st));
            }
            const int64_t rpc = std::max<int64_t>(1, stg.cap / cols);
            for (int64_t r0 = 0; b.dev == nullptr && r0 < rows; r0 += rpc) {
                const int64_t nr = std::min(rpc, rows - r0);
                std::memcpy(stg.host, b.data.data() + r0 * cols, (size_t)(nr * cols) * sizeof(double));
                CGS_HIP(hipMemcpyAsync(stg.dev, stg.host, (size_t)(nr * cols) * sizeof(double),
                                       hipMemcpyHostToDevice, st));
                launch_cast_pad(prec, stg.dev, 0, cols, nr, cols, (char*)db.a + r0 * ld * sz, ld, st);
                launch_cast_transpose(prec, stg.dev, 0, cols, nr, cols, const_cast<void*>(db.at), ldt, r0, st);
                CGS_HIP(hipStreamSynchronize(st));
            }
            if (precision == CGS_BF16) {
                db.a16 = p;
                p += align256(round_up(rows, 32) * ld * 2);
                db.a16lo = p;
                p += align256(round_up(rows, 32) * ld * 2);
                db.at16 = p;
                p += align256(round_up(cols, 32) * ldt * 2);
                db.at16lo = p;
                p += align256(round_up(cols, 32) * ldt * 2);
                launch_gemm_pack_w((const float*)db.a, rows, ld, (uint16_t*)db.a16, (uint16_t*)db.a16lo, st);
                launch_gemm_pack_w((const float*)db.at, cols, ldt, (uint16_t*)db.at16, (uint16_t*)db.at16lo, st);
            }
        }
    }
    CGS_HIP(hipGetLastError());
    CGS_HIP(hipStreamSynchronize(st));
    return CGS_OK;
}

int upload_f64(const Staging& stg, hipStream_t st, const double* src, int64_t n, int prec, void* dst) {
    const size_t sz = prec == 0 ? 8 : 4;
    for (int64_t off = 0; off < n; off += stg.cap) {
        const int64_t c = std::min(stg.cap, n - off);
        std::memcpy(stg.host, src + off, (size_t)c * sizeof(double));
        CGS_HIP(hipMemcpyAsync(stg.dev, stg.host, (size_t)c * sizeof(double), hipMemcpyHostToDevice, st));
        launch_cast(prec, stg.dev, (char*)dst + off * sz, c, st);
        CGS_HIP(hipGetLastError());
        CGS_HIP(hipStreamSynchronize(st));
    }
    return CGS_OK;
}

int upload_raw(const Staging& stg, hipStream_t st, const void* src, size_t bytes, void* dst) {
    if (bytes > (size_t)stg.cap * sizeof(double)) return fail(CGS_ENOMEM, "staging too small");
    std::memcpy(stg.host, src, bytes);
    CGS_HIP(hipMemcpyAsync(dst, stg.host, bytes, hipMemcpyHostToDevice, st));
    CGS_HIP(hipStreamSynchronize(st));
    return CGS_OK;
}

int download_f64(const Staging& stg, hipStream_t st, int prec, const void* src, int64_t n, double* dst) {
    const size_t sz = prec == 0 ? 8 : 4;
    for (int64_t off = 0; off < n; off += stg.cap) {
        const int64_t c = std::min(stg.cap, n - off);
        launch_cast_back(prec, (const char*)src + off * sz, stg.dev, c, st);
        CGS_HIP(hipGetLastError());
        CGS_HIP(hipMemcpyAsync(stg.host, stg.dev, (size_t)c * sizeof(double), hipMemcpyDeviceToHost, st));
        CGS_HIP(hipStreamSynchronize(st));
        std::memcpy(dst + off, stg.host, (size_t)c * sizeof(double));
    }
    return CGS_OK;
}

// ---------------------------------------------------------------- tables
void build_image(const std::vector<InstRec>& recs, int precision, TableImage& im, int vec_tile) {
    im = TableImage{};
    const int64_t ct = conv_tile(precision);
    for (size_t i = 0; i < recs.size(); ++i) {
        const InstRec& r = recs[i];
        const int ii = (int)i;
        InstDesc d{};
        d.base = r.base;
        d.n = r.n;
        d.m = r.m;
        d.nxs = round_up(r.n, XY_ALIGN);
        d.nys = round_up(r.m, XY_ALIGN);
        d.l = r.l;
        d.xt0 = (int32_t)im.xt.size();
        for (int64_t s = 0; s < r.n; s += vec_tile)
            im.xt.push_back(VecTile{ii, -1, s, (int32_t)std::min<int64_t>(vec_tile, r.n - s), 0});
        d.xt1 = (int32_t)im.xt.size();
        d.yt0 = (int32_t)im.yt.size();
        for (int64_t s = 0; s < r.l; s += vec_tile)
            im.yt.push_back(VecTile{ii, -1, s, (int32_t)std::min<int64_t>(vec_tile, r.l - s), 0});
        d.sg0 = (int32_t)im.seg.size();
        int64_t off = r.l;
        for (int64_t qj : r.q) {
            SocSeg sg{};
            sg.inst = ii;
            sg.yt0 = (int32_t)im.yt.size();
            sg.start = off;
            sg.len = qj;
            const int32_t sid = (int32_t)im.seg.size();
            // a tile spans at most VEC_TILE elements of the 4-element grid
            // (vector kernels walk tiles in aligned chunks of four)
            for (int64_t s = 0; s < qj;) {
                const int64_t len = std::min<int64_t>(vec_tile - ((off + s) & 3), qj - s);
                im.yt.push_back(VecTile{ii, sid, off + s, (int32_t)len, 0});
                s += len;
            }
            sg.ntiles = (int32_t)im.yt.size() - sg.yt0;
            im.seg.push_back(sg);
            off += qj;
        }
        d.sg1 = (int32_t)im.seg.size();
        d.yt1 = (int32_t)im.yt.size();
        d.id0 = (int32_t)im.ids.size();
        for (const IdBlock& b : r.op->ids) im.ids.push_back(b);
        d.id1 = (int32_t)im.ids.size();
        d.cb0 = (int32_t)im.cblk.size();
        d.cb1 = d.cb0 + (int32_t)r.op->convs.size();
        d.db0 = (int32_t)im.dblk.size();
        d.db1 = d.db0 + (int32_t)r.op->dense.size();
        for (size_t j = 0; j < r.op->convs.size(); ++j) {
            if (im.cfwd.size() <= j) {
                im.cfwd.resize(j + 1);
                im.cadj.resize(j + 1);
                im.ffwd.resize(j + 1);
                im.fadj.resize(j + 1);
            }
            const ConvBlock& cb = r.op->convs[j];
            const int32_t bi = (int32_t)im.cblk.size();
            im.cblk.push_back(cb);
            const int64_t n_out = cb.n_in + cb.k - 1;
            for (int64_t s = 0; s < n_out; s += ct) im.cfwd[j].push_back(ConvTile{ii, bi, s});
            for (int64_t s = 0; s < cb.n_in; s += ct) im.cadj[j].push_back(ConvTile{ii, bi, s});
            if (work_prec(precision) == 1 && cb.k <= FFT_KMAX) {
                // FFT-engine tiles (the blocks that get spectra at upload): two
                // windows of FFT_L - k + 1 outputs each
                const int64_t w2 = 2 * (FFT_L - cb.k + 1);
                for (int64_t s = 0; s < n_out; s += w2) im.ffwd[j].push_back(ConvTile{ii, bi, s});
                for (int64_t s = 0; s < cb.n_in; s += w2) im.fadj[j].push_back(ConvTile{ii, bi, s});
            }
        }
        for (size_t j = 0; j < r.op->dense.size(); ++j) {
            if (im.dfwd.size() <= j) {
                im.dfwd.resize(j + 1);
                im.dadj.resize(j + 1);
            }
            const DenseBlock& db = r.op->dense[j];
            const int32_t bi = (int32_t)im.dblk.size();
            im.dblk.push_back(db);
            for (int64_t s = 0; s < db.rows; s += DENSE_ROWS)
                im.dfwd[j].push_back(DenseTile{ii, bi, s, (int32_t)std::min<int64_t>(DENSE_ROWS, db.rows - s), 0});
            for (int64_t s = 0; s < db.cols; s += DENSE_ROWS)
                im.dadj[j].push_back(DenseTile{ii, bi, s, (int32_t)std::min<int64_t>(DENSE_ROWS, db.cols - s), 0});
        }
        im.inst.push_back(d);
    }
}

template <typename V>
static size_t vbytes(const std::vector<V>& v) { return align256(v.size() * sizeof(V)); }

size_t image_table_bytes(const TableImage& im) {
    size_t t = vbytes(im.inst) + vbytes(im.xt) + vbytes(im.yt) + vbytes(im.seg) + vbytes(im.ids) +
               vbytes(im.cblk) + vbytes(im.dblk);
    for (const auto& v : im.cfwd) t += vbytes(v);
    for (const auto& v : im.cadj) t += vbytes(v);
    for (const auto& v : im.ffwd) t += vbytes(v);
    for (const auto& v : im.fadj) t += vbytes(v);
    for (const auto& v : im.dfwd) t += vbytes(v);
    for (const auto& v : im.dadj) t += vbytes(v);
    t += vbytes(im.xt) + vbytes(im.yt);   // initialisation tiles folded into convolution launches
    return t + 256;
}

size_t image_work_bytes(const TableImage& im) {
    const size_t nfa = im.fadj.empty() ? 0 : im.fadj[0].size();
    return align256(4 * im.xt.size() * 8) + align256(4 * im.yt.size() * 8) +
           align256(2 * im.seg.size() * 8) + align256(im.seg.size() * 4) +
           2 * align256(4 * (nfa + im.xt.size()) * 8) + align256(4 * (im.xt.size() + im.yt.size()) * 8) +
           align256(im.inst.size() * NSC * 8) + 256;
}

// ---------------------------------------------------------------- engine
Engine::~Engine() {
    drop_graph();
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
    if (!pageable) {
        if (tab_host) (void)hipHostFree(tab_host);
        if (scal_host) (void)hipHostFree(scal_host);
        if (stg.host) (void)hipHostFree(stg.host);
    }
}

void Engine::drop_graph() {
    for (CachedGraph& g : graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    graphs.clear();
}

// CG launches per step for the next check interval: the most CG iterations any
// running instance used in a step of the last interval (cg_max_iters for an
// instance's first interval), within [1, cg_max_iters]; fixed at cg_max_iters
// when adaptation is off.  An interval
// whose steps needed more is run again from its snapshot (Engine::rollback).
void Engine::adapt_cg() {
    if (!st.cg_adaptive || !snap_ok) {
        // (without a copy to run an interval again from, no prediction)
        cg_launch = st.cg_max_iters;
        return;
    }
    double need = 0.0;
    for (int i = 0; i < T.ninst; ++i) {
        const double* sc = scalars(i);
        if (sc[SC_ACTIVE] == 0.0 || sc[SC_PHASE] != 1.0) continue;
        // an instance's first interval has nothing to predict from (and its
        // cold-started CG solves take the most iterations of the solve)
        need = std::max(need, sc[SC_ITER] == 0.0 ? (double)st.cg_max_iters : sc[SC_CGMAXLAST]);
    }
    cg_launch = std::max(1, std::min(st.cg_max_iters, (int)need));
}

int Engine::init_host_buffers(size_t tab_bytes, int max_inst, int64_t stg_doubles) {
    const size_t tb = std::max<size_t>(tab_bytes, 256);
    const size_t sb = std::max<size_t>(1, (size_t)max_inst) * NSC * sizeof(double);
    const size_t gb = (size_t)stg_doubles * sizeof(double);
    if (pageable) {
        const size_t tw = (tb + 7) / 8, sw = sb / 8, gw = gb / 8;
        try {
            host_store.assign(tw + sw + gw, 0.0);
        } catch (...) {
            return fail(CGS_ENOMEM, "host allocation failed");
        }
        tab_host = reinterpret_cast<char*>(host_store.data());
        scal_host = host_store.data() + tw;
        stg.host = host_store.data() + tw + sw;
    } else {
        CGS_HIP(hipHostMalloc((void**)&tab_host, tb, hipHostMallocDefault));
        CGS_HIP(hipHostMalloc((void**)&scal_host, sb, hipHostMallocDefault));
        CGS_HIP(hipHostMalloc((void**)&stg.host, gb, hipHostMallocDefault));
    }
    tab_host_cap = tab_bytes;
    scal_host_cap = max_inst;
    stg.cap = stg_doubles;
    return CGS_OK;
}

int Engine::build(const std::vector<InstRec>& r) {
    recs = r;
    rounds_since_build = 0;
    build_image(recs, precision, im, vec_tile);
    // each instance's path depends on its own size only (never on the mix);
    // a solver's single instance has the whole chip to itself on the other path
    n_fused = n_multi = 0;
    const int64_t lim = (lone && st.fused_lone_max > 0) ? std::min(st.fused_max, st.fused_lone_max)
                                                        : (int64_t)st.fused_max;
    for (InstDesc& d : im.inst) {
        int64_t dense = 0;
        for (int b = d.db0; b < d.db1; ++b) dense += im.dblk[b].rows * im.dblk[b].cols;
        d.fused = (st.fused_max > 0 && !use_gemm && d.n + d.m <= lim && dense <= FUSED_DENSE_MAX) ? 1 : 0;
        (d.fused ? n_fused : n_multi) += 1;
    }
    fused_res = 0;
    for (const InstDesc& d : im.inst)
        if (d.fused) fused_res = std::max(fused_res, fused_resident_bytes(prec, d.n, d.m));
    if (n_fused) fused_prepare();
    // When every convolution owns its output range in a direction, the output
    // initialisation rides on the first convolution launch as extra
    // workgroups (one launch fewer per apply); tiles wholly inside an owned
    // range need no initialisation at all.
    std::vector<VecTile> init_tiles[2];
    for (int adj = 0; adj < 2; ++adj) {
        fold_init[adj] = 0;
        if ((adj ? im.cadj : im.cfwd).empty()) continue;
        bool all = true;
        for (const ConvBlock& cb : im.cblk) all = all && ((cb.own >> adj) & 1);
        if (!all) continue;
        for (const VecTile& t : adj ? im.xt : im.yt) {
            const InstDesc& d = im.inst[t.inst];
            bool covered = false;
            for (int b = d.cb0; b < d.cb1 && !covered; ++b) {
                const ConvBlock& cb = im.cblk[b];
                const int64_t lo = adj ? cb.col0 : cb.row0;
                const int64_t hi = lo + (adj ? cb.n_in : cb.n_in + cb.k - 1);
                covered = lo <= t.start && t.start + t.len <= hi;
            }
            if (!covered) init_tiles[adj].push_back(t);
        }
        fold_init[adj] = 1;
    }
    // CG steps fold into the FFT engine's A^T launch when that launch (its
    // transform workgroups and its initialisation workgroups) writes every X
    // element: one convolution slot, all blocks owned and with spectra, no
    // dense block.  Each instance's partials are then those of its transform
    // workgroups and of its initialisation workgroups.
    fold_cg = 0;
    if (fold_init[1] && im.cadj.size() == 1 && im.dadj.empty() && !use_gemm && work_prec(precision) == 1) {
        bool fft = !im.cadj[0].empty();
        for (const ConvTile& t : im.cadj[0]) fft = fft && im.cblk[t.blk].k <= FFT_KMAX;
        fold_cg = fft && !im.fadj.empty() ? 1 : 0;
    }
    // The right-hand side launch can also write the identity rows of A p (the
    // first CG product, p = r): possible when, in every instance on this
    // path, the convolution rows and rows reached by exactly one identity
    // block cover the Y vector; the step's first A p launch then needs no
    // initialisation workgroups.
    idrows = 0;
    if (fold_cg) {
        bool ok = true;
        for (const InstDesc& d : im.inst) {
            if (d.fused) continue;
            std::vector<std::pair<int64_t, int64_t>> iv;
            for (int b = d.cb0; b < d.cb1; ++b)
                iv.emplace_back(im.cblk[b].row0, im.cblk[b].row0 + im.cblk[b].n_in + im.cblk[b].k - 1);
            for (int b = d.id0; b < d.id1; ++b)
                if (im.ids[b].len > 0) iv.emplace_back(im.ids[b].row0, im.ids[b].row0 + im.ids[b].len);
            std::sort(iv.begin(), iv.end());
            int64_t pos = 0;
            for (const auto& r : iv) {
                ok = ok && r.first == pos;
                pos = r.second;
            }
            ok = ok && pos == d.m && d.db0 == d.db1;
        }
        idrows = ok ? 1 : 0;
    }
    for (InstDesc& d : im.inst) d.cp0 = d.cp1 = d.ip0 = d.ip1 = 0;
    if (fold_cg) {
        const int nft = (int)im.fadj[0].size();
        for (int i = 0; i < nft; ++i) {
            InstDesc& d = im.inst[im.fadj[0][i].inst];
            if (d.cp1 == 0) d.cp0 = i;
            d.cp1 = i + 1;
        }
        for (int i = 0; i < (int)init_tiles[1].size(); ++i) {
            InstDesc& d = im.inst[init_tiles[1][i].inst];
            if (d.ip1 == 0) d.ip0 = nft + i;
            d.ip1 = nft + i + 1;
        }
    }
    // copies of the carried state for check intervals run with fewer CG
    // launches per step than the iteration limit: one per instance of the
    // one-launch-per-kernel path, packed into the snapshot area (none when
    // they do not all fit)
    {
        size_t need = 0;
        for (const InstDesc& d : im.inst)
            if (!d.fused) need += snap_bytes(d.n, d.m, precision);
        const bool fit = snap_dev != nullptr && need <= snap_cap;
        size_t o = 0;
        for (InstDesc& d : im.inst) {
            d.snap = nullptr;
            if (fit && !d.fused) {
                d.snap = snap_dev + o;
                o += snap_bytes(d.n, d.m, precision);
            }
        }
        snap_ok = fit && n_multi > 0 ? 1 : 0;
    }
    spec_launch = 0;
    const size_t tb = image_table_bytes(im), wb = image_work_bytes(im);
    if (tb > tab_cap || tb > tab_host_cap || wb > work_cap || (int)im.inst.size() > scal_host_cap)
        return fail(CGS_ENOMEM, "tile tables need %zu + %zu bytes (have %zu + %zu)", tb, wb, tab_cap, work_cap);
    CGS_HIP(hipStreamSynchronize(stream));
    size_t off = 0;
    auto put = [&](const void* src, size_t bytes) -> char* {
        if (bytes) std::memcpy(tab_host + off, src, bytes);
        char* d = tab_dev + off;
        off += align256(bytes);
        return d;
    };
    inst_dev = (InstDesc*)put(im.inst.data(), im.inst.size() * sizeof(InstDesc));
    T.inst = inst_dev;
    T.xt = (const VecTile*)put(im.xt.data(), im.xt.size() * sizeof(VecTile));
    T.yt = (const VecTile*)put(im.yt.data(), im.yt.size() * sizeof(VecTile));
    T.seg = (const SocSeg*)put(im.seg.data(), im.seg.size() * sizeof(SocSeg));
    T.ids = (const IdBlock*)put(im.ids.data(), im.ids.size() * sizeof(IdBlock));
    const ConvBlock* cbd = (const ConvBlock*)put(im.cblk.data(), im.cblk.size() * sizeof(ConvBlock));
    const DenseBlock* dbd = (const DenseBlock*)put(im.dblk.data(), im.dblk.size() * sizeof(DenseBlock));
    T.cblk = cbd;
    T.dblk = dbd;
    cf.clear(); ca.clear(); df.clear(); da.clear();
    const int64_t kcmax = precision == CGS_FP64 ? CONV_KC_MAX_F64 : CONV_KC_MAX_F32;
    auto slot_kc = [&](const std::vector<ConvTile>& v) {
        int64_t kc = conv_r(precision);
        for (const ConvTile& t : v) kc = std::max(kc, std::min(kcmax, im.cblk[t.blk].kpad));
        return (int)kc;
    };
    // the FFT engine can take a slot when every block in it has spectra
    auto slot_fft = [&](const std::vector<ConvTile>& v) {
        bool ok = !v.empty();
        for (const ConvTile& t : v) ok = ok && im.cblk[t.blk].s_fwd != nullptr;
        return ok ? 1 : 0;
    };
    for (size_t j = 0; j < im.cfwd.size(); ++j) {
        const auto& v = im.cfwd[j];
        const int fft = slot_fft(v);
        const auto& fv = im.ffwd[j];
        cf.push_back(ConvLaunch{(const ConvTile*)put(v.data(), v.size() * sizeof(ConvTile)), cbd, (int)v.size(),
                                slot_kc(v), nullptr, 0,
                                fft ? (const ConvTile*)put(fv.data(), fv.size() * sizeof(ConvTile)) : nullptr,
                                fft ? (int)fv.size() : 0, fft});
    }
    for (size_t j = 0; j < im.cadj.size(); ++j) {
        const auto& v = im.cadj[j];
        const int fft = slot_fft(v);
        const auto& fv = im.fadj[j];
        ca.push_back(ConvLaunch{(const ConvTile*)put(v.data(), v.size() * sizeof(ConvTile)), cbd, (int)v.size(),
                                slot_kc(v), nullptr, 0,
                                fft ? (const ConvTile*)put(fv.data(), fv.size() * sizeof(ConvTile)) : nullptr,
                                fft ? (int)fv.size() : 0, fft});
    }
    for (int adj = 0; adj < 2; ++adj) {
        std::vector<ConvLaunch>& cl = adj ? ca : cf;
        if (!fold_init[adj] || cl.empty()) continue;
        cl[0].init = (const VecTile*)put(init_tiles[adj].data(), init_tiles[adj].size() * sizeof(VecTile));
        cl[0].ninit = (int)init_tiles[adj].size();
    }
    for (const auto& v : im.dfwd) df.push_back(DenseLaunch{(const DenseTile*)put(v.data(), v.size() * sizeof(DenseTile)), dbd, (int)v.size()});
    for (const auto& v : im.dadj) da.push_back(DenseLaunch{(const DenseTile*)put(v.data(), v.size() * sizeof(DenseTile)), dbd, (int)v.size()});
    if (off > tab_cap) return fail(CGS_ENOMEM, "table overflow");
    CGS_HIP(hipMemcpyAsync(tab_dev, tab_host, off, hipMemcpyHostToDevice, stream));
    char* w = work_dev;
    T.xpart = (double*)w; w += align256(4 * im.xt.size() * 8);
    T.ypart = (double*)w; w += align256(4 * im.yt.size() * 8);
    T.seg_val = (double*)w; w += align256(2 * im.seg.size() * 8);
    T.seg_cnt = (int*)w; w += align256(im.seg.size() * 4);
    T.cpart = (double*)w; w += align256(4 * ((im.fadj.empty() ? 0 : im.fadj[0].size()) + im.xt.size()) * 8);
    T.spart = (double*)w; w += align256(4 * ((im.fadj.empty() ? 0 : im.fadj[0].size()) + im.xt.size()) * 8);
    T.tpart = (double*)w; w += align256(4 * (im.xt.size() + im.yt.size()) * 8);
    gather_dev = (double*)w;
    if (!im.seg.empty()) CGS_HIP(hipMemsetAsync(T.seg_cnt, 0, im.seg.size() * 4, stream));
    T.nx_tiles = (int)im.xt.size();
    T.ny_tiles = (int)im.yt.size();
    T.nseg = (int)im.seg.size();
    T.ninst = (int)im.inst.size();
    fused_kc = (int)conv_r(precision);
    for (const ConvBlock& cb : im.cblk) fused_kc = std::max<int>(fused_kc, (int)std::min(kcmax, cb.kpad));
    CGS_HIP(hipStreamSynchronize(stream));
    drop_graph();
    return CGS_OK;
}

char* Engine::xptr(int i, int kind) const {
    const InstDesc& d = im.inst[i];
    return d.base + REGION_HDR + (size_t)kind * d.nxs * elem_bytes(precision);
}
char* Engine::yptr(int i, int kind) const {
    const InstDesc& d = im.inst[i];
    return d.base + REGION_HDR + ((size_t)NXV * d.nxs + (size_t)kind * d.nys) * elem_bytes(precision);
}

// Convolution engine for FP32 (conv_mfma): 1 matrix cores, 2 FFT (slots whose
// blocks all have spectra; the matrix cores otherwise), 0 vector ALU; FP64
// always on the vector ALU.
void Engine::conv(const ConvLaunch& c, int adj, int out, int in, int base, double sigma, int gate) {
    if (prec == 1 && st.conv_mfma == 2 && c.fft) launch_conv_fft(T, c, adj, out, in, base, sigma, gate, stream);
    else if (prec == 1 && st.conv_mfma) launch_conv_mfma(T, c, adj, out, in, base, sigma, gate, stream);
    else launch_conv(prec, T, c, adj, out, in, base, sigma, gate, stream);
}

void Engine::apply(int adj, int out, int in, int base, double sigma, int gate) {
    const auto& cl = adj ? ca : cf;
    // with no convolution launch in between, the first GEMM's packing launch
    // also writes the output's initial value
    const bool init_in_pack = use_gemm && cl.empty() && !fold_init[adj] && !recs[0].op->dense.empty();
    if (!fold_init[adj] && !init_in_pack) launch_apply_init(prec, T, adj, out, in, base, sigma, gate, stream);
    for (const auto& c : cl) conv(c, adj, out, in, base, sigma, gate);
    if (use_gemm) {
        // every instance shares the dense blocks: one MFMA GEMM per block
        bool first = true;
        for (const DenseBlock& db : recs[0].op->dense) {
            launch_gemm_apply(T, db, adj, out, in, sigma, gate, gemm_corr, panel, panel_stride, gemm_part,
                              gemm_target, stream, first && init_in_pack, base);
            first = false;
        }
    } else {
        for (const auto& d : adj ? da : df) launch_gemv(prec, T, d, adj, out, in, sigma, gate, stream);
    }
}

// One CG iteration of the Section IV-B listing on (I + A^T A):
// q = p + A^T (A p); alpha = rr/<p,q>; z += alpha p; r -= alpha q; beta; p = r + beta p.
void Engine::cg_iter(int z, int gate, int cg_max, int track, int it, int last, int start) {
    if (start) {
        // first iteration of an ADMM step on the folded path: the products run
        // whatever the CG start test says (a step without CG iterations is
        // rare) and the update evaluates the test from the right-hand side's
        // partials, so no launch separates the right-hand side from A p
        // p = r: this iteration reads the direction from r's vector (the
        // right-hand side launch wrote r only) and its update writes the next
        // direction to XP
        if (idrows) {
            // (the identity rows of A p came with r from the right-hand side launch)
            for (ConvLaunch a : cf) {
                a.ninit = 0;
                conv(a, 0, YT, XR, -1, 1.0, G_ADMM);
            }
        } else {
            apply(0, YT, XR, -1, 1.0, G_ADMM);
        }
        ConvLaunch c = ca[0];
        c.fold = 2;
        c.fr = XR;
        c.fp = XR;
        c.fit = it;
        c.part = T.cpart;
        conv(c, 1, XQ, YT, XR, 1.0, G_ADMM);
        CgStart cs{st.cg_tol, st.cg_rate, cg_floor(), 1, 1, 1, st.alpha};
        cs.pn = XP;
        launch_cg_update(prec, T, z, XR, XR, XQ, it, cg_max, gate, track, stream, 1, last, cs);
        return;
    }
    apply(0, YT, XP, -1, 1.0, gate);
    if (folded_cg()) {
        // q = p + A^T (A p) with the dot partials and the iteration mark formed
        // as each element of q is written (the work of k_cg_dot)
        ConvLaunch c = ca[0];
        c.fold = 2;
        c.fr = XR;
        c.fp = XP;
        c.fit = it;
        c.part = T.cpart;
        conv(c, 1, XQ, YT, XP, 1.0, gate);
        // (on the ADMM path the update that ends CG also takes the tau products)
        const int tau = gate == G_ADMM_CG && track ? 1 : 0;
        launch_cg_update(prec, T, z, XR, XP, XQ, it, cg_max, gate, track, stream, 1, last,
                         CgStart{0.0, 0.0, 0.0, 0, tau, tau, st.alpha});
        return;
    }
    apply(1, XQ, YT, XP, 1.0, gate);
    launch_cg_dot(prec, T, XP, XQ, XR, it, gate, stream);
    launch_cg_update(prec, T, z, XR, XP, XQ, it, cg_max, gate, track, stream, 0, last);
}

// One ADMM step of the homogeneous self-dual embedding.  The CG warm start z
// carries A z (YA) and (I + A^T A) z (XK), updated with every CG step and
// recomputed exactly at every termination check, so a step applies the
// operator 1 + 2 * (CG iterations) times.
void Engine::admm_step() {
    // w_y = u_y + v_s was written by the previous step's projection (or refresh)
    if (folded_cg()) {
        // h = u_x - A^T w_y formed in the launch's epilogue, which writes
        // r = h - K z (not h) and the CG start partials; the first CG
        // update takes the start test
        ConvLaunch c = ca[0];
        c.fold = 1;
        c.fr = XR;
        c.fp = -1;   // (the first iteration reads p = r from XR)
        c.fq = XK;
        c.part = T.spart;
        c.idrows = idrows ? YT + 1 : 0;
        conv(c, 1, XH, YW, XU, -1.0, G_ADMM);
        const int nl = std::max(1, cg_launch);
        for (int i = 0; i < nl; ++i)
            cg_iter(XZ, G_ADMM_CG, st.cg_max_iters, 1, i, spec_now && i == nl - 1, i == 0);
    } else {
        apply(1, XH, YW, XU, -1.0, G_ADMM);                      // h = u_x - A^T w_y
        launch_cg_init(prec, T, XZ, XR, XP, XK, XH, 1, st.cg_tol, st.cg_rate, cg_floor(),
                       st.cg_max_iters, G_ADMM, stream);         // r = h - K z
        for (int i = 0; i < cg_launch; ++i)
            cg_iter(XZ, G_ADMM_CG, st.cg_max_iters, 1, i, spec_now && i == cg_launch - 1);
    }
    if (folded_cg()) {
        // z_y, the tau products and the cone terms came from the last CG update
        launch_project(prec, T, st.alpha, stream);               // relax, project, dual update
        return;
    }
    // z_y = w_y + A z; c^T z_x + b^T z_y; the cone terms of u_bar - v (CgStart::cone)
    launch_tau_dots(prec, T, st.alpha, stream);
    launch_project(prec, T, st.alpha, stream);                   // relax, project, dual update
}

// Two applies of one direction; one launch where the FFT engine alone serves
// that direction (its transform workgroups and initialisation tiles for both).
void Engine::apply_pair(int adj, int out1, int in1, int base1, int out2, int in2, int base2, double sigma,
                        int gate) {
    const auto& cl = adj ? ca : cf;
    if (prec == 1 && st.conv_mfma == 2 && fold_init[adj] && cl.size() == 1 && cl[0].fft &&
        (adj ? da : df).empty() && !use_gemm) {
        ConvLaunch c = cl[0];
        c.pair = 1;
        c.out2 = out2;
        c.in2 = in2;
        c.base2 = base2;
        launch_conv_fft(T, c, adj, out1, in1, base1, sigma, gate, stream);
        return;
    }
    apply(adj, out1, in1, base1, sigma, gate);
    apply(adj, out2, in2, base2, sigma, gate);
}

void Engine::check(int gate) {
    if (gate == G_CHECK) {
        // with the exact A z and z + A^T A z for the next interval (the gates
        // G_CHECK and G_ADMM select the same instances)
        apply_pair(0, YT, XU, -1, YA, XZ, -1, 1.0, gate);       // A u_x, A z
        apply_pair(1, XT, YU, -1, XK, YA, XZ, 1.0, gate);       // A^T u_y, z + A^T A z
        launch_resid(prec, T, st.eps, st.max_iters, gate, stream);
        return;
    }
    apply(0, YT, XU, -1, 1.0, gate);                             // A u_x
    apply(1, XT, YU, -1, 1.0, gate);                             // A^T u_y
    launch_resid(prec, T, st.eps, st.max_iters, gate, stream);
}

// Exact recomputation of the carried products of the CG warm start.
void Engine::refresh() {
    if (n_fused) {
        // instances that run fused steps keep their products in that kernel's
        // arithmetic (a result must not depend on when the host refreshes)
        FusedArgs fa{};
        fa.refresh = 1;
        fa.kc = fused_kc;
        launch_fused(prec, T, fa, stream);
    }
    if (n_multi) {
        launch_wy(prec, T, G_ADMM, stream);                      // w_y = u_y + v_s
        apply(0, YA, XZ, -1, 1.0, G_ADMM);                       // A z
        apply(1, XK, YA, XZ, 1.0, G_ADMM);                       // z + A^T (A z)
    }
}

void Engine::fused_steps(int nsteps, int check) {
    FusedArgs fa{};
    fa.nsteps = nsteps;
    fa.check = check;
    fa.alpha = st.alpha;
    fa.eps = st.eps;
    fa.zeta = st.cg_tol;
    fa.rate = st.cg_rate;
    fa.floor_ = cg_floor();
    fa.cg_max = st.cg_max_iters;
    fa.max_iters = st.max_iters;
    fa.kc = fused_kc;
    fa.res_want = fused_res;
    launch_fused(prec, T, fa, stream);
}

void Engine::steps_with_checks(int nsteps) {
    for (int i = 0; i < nsteps; ++i) {
        admm_step();
        if ((i + 1) % st.check_every == 0 || i + 1 == nsteps) check();
    }
}

int Engine::round(int nsteps, bool multi_only) {
    bool forked = false;
    if (multi_only) {
        // the fused instances' interval already ran
    } else if (n_fused && n_multi && stream != nullptr) {
        // both paths in the round: the fused launch runs on the side stream
        // beside the other instances' kernels (they touch disjoint instance
        // regions and partial buffers) and the main stream waits for it
        if (!side) {
            CGS_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
            CGS_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
            CGS_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
        }
        CGS_HIP(hipEventRecord(ev_fork, stream));
        CGS_HIP(hipStreamWaitEvent(side, ev_fork, 0));
        hipStream_t main_stream = stream;
        stream = side;
        for (int done = 0; done < nsteps; done += st.check_every)
            fused_steps(std::min(st.check_every, nsteps - done), 1);
        stream = main_stream;
        CGS_HIP(hipGetLastError());
        CGS_HIP(hipEventRecord(ev_join, side));
        forked = true;
    } else if (n_fused) {
        for (int done = 0; done < nsteps; done += st.check_every)
            fused_steps(std::min(st.check_every, nsteps - done), 1);
    }
    if (!n_multi) {
        CGS_HIP(hipGetLastError());
        return CGS_OK;
    }
    // Fewer CG launches per step than the iteration limit: the interval starts
    // with a copy of the carried state, kept until the host has seen whether
    // some step's CG would have gone on after its last launch.
    const bool spec = st.cg_adaptive && snap_ok && cg_launch < st.cg_max_iters;
    if (!multi_only && spec) {
        spec_live.assign((size_t)T.ninst, 0);
        for (int i = 0; i < T.ninst; ++i) {
            const double* sc = scalars(i);
            spec_live[(size_t)i] = !im.inst[(size_t)i].fused && sc[SC_ACTIVE] != 0.0 && sc[SC_PHASE] == 1.0;
        }
    }
    spec_launch = spec ? cg_launch : 0;
    spec_nsteps = nsteps;
    spec_now = spec;
    ++n_rounds;
    // Capture and instantiation cost more than launching one round directly,
    // so a graph is captured only for tables that have already served a round
    // (a server rebuilds them whenever requests arrive or leave).
    const bool use_g = st.use_graph && stream != nullptr && nsteps == round_steps() &&
                       (!graphs.empty() || rounds_since_build >= 1);
    ++rounds_since_build;
    if (use_g) {
        CachedGraph* hit = nullptr;
        for (CachedGraph& g : graphs)
            if (g.steps == nsteps && g.cg == cg_launch && g.spec == (int)spec) hit = &g;
        if (!hit) {
            if (graphs.size() >= GRAPH_CACHE) {
                size_t old = 0;
                for (size_t j = 1; j < graphs.size(); ++j)
                    if (graphs[j].used < graphs[old].used) old = j;
                (void)hipGraphExecDestroy(graphs[old].exec);
                (void)hipGraphDestroy(graphs[old].graph);
                graphs.erase(graphs.begin() + (std::ptrdiff_t)old);
            }
            CGS_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            if (spec) launch_snapshot(prec, T, 0, stream);
            steps_with_checks(nsteps);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(stream, &g);
            if (e != hipSuccess) return fail(CGS_EHIP, "graph capture failed: %s", hipGetErrorString(e));
            hipGraphExec_t x = nullptr;
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                return fail(CGS_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
            }
            graphs.push_back(CachedGraph{nsteps, cg_launch, (int)spec, g, x, 0});
            hit = &graphs.back();
        }
        hit->used = n_rounds;
        CGS_HIP(hipGraphLaunch(hit->exec, stream));
    } else {
        if (spec) launch_snapshot(prec, T, 0, stream);
        steps_with_checks(nsteps);
    }
    spec_now = false;
    if (forked) CGS_HIP(hipStreamWaitEvent(stream, ev_join, 0));
    CGS_HIP(hipGetLastError());
    return CGS_OK;
}

bool Engine::truncated() const {
    if (spec_launch <= 0) return false;
    for (int i = 0; i < T.ninst; ++i)
        if (spec_live[(size_t)i] && scalars(i)[SC_PHASE] == 3.0) return true;
    return false;
}

int Engine::rollback() {
    launch_snapshot(prec, T, 1, stream);
    // w_y, A z and z + A^T A z as the check before the interval formed them
    launch_wy(prec, T, G_ADMM, stream);
    apply(0, YA, XZ, -1, 1.0, G_ADMM);
    apply(1, XK, YA, XZ, 1.0, G_ADMM);
    CGS_HIP(hipGetLastError());
    ++n_reruns;
    cg_launch = std::min(st.cg_max_iters, 2 * spec_launch + 1);
    return round(spec_nsteps, true);
}

int Engine::fetch_scalars() {
    launch_gather_scalars(inst_dev, T.ninst, gather_dev, stream);
    CGS_HIP(hipGetLastError());
    CGS_HIP(hipMemcpyAsync(scal_host, gather_dev, (size_t)T.ninst * NSC * sizeof(double),
                           hipMemcpyDeviceToHost, stream));
    CGS_HIP(hipStreamSynchronize(stream));
    return CGS_OK;
}

int Engine::setup() {
    launch_norms(prec, T, G_SETUP, stream);
    apply(1, XH, YB, XC, -1.0, G_SETUP);                          // h = c - A^T b
    // CG from the current g_x (0 after a reset; the previous operator's
    // embedding vector when a refined operator restarts the setup)
    apply(0, YT, XG, -1, 1.0, G_SETUP);                           // A g_x
    apply(1, XQ, YT, XG, 1.0, G_SETUP);                           // (I + A^T A) g_x
    launch_cg_init(prec, T, XG, XR, XP, XQ, XH, 1, 0.0, 0.0, setup_tol(), st.setup_max_iters,
                   G_SETUP, stream);
    int it = 0;
    while (it < st.setup_max_iters) {
        const int nb = std::min(8, st.setup_max_iters - it);
        for (int j = 0; j < nb; ++j) cg_iter(XG, G_SETUP_CG, st.setup_max_iters, 0, it + j);
        it += nb;
        CGS_TRY(fetch_scalars());
        bool any = false;
        for (int i = 0; i < T.ninst; ++i) {
            const double* sc = scalars(i);
            if (sc[SC_ACTIVE] != 0.0 && sc[SC_PHASE] == 0.0 && sc[SC_CGACT] != 0.0) any = true;
        }
        if (!any) break;
    }
    apply(0, YG, XG, YB, 1.0, G_SETUP);                           // g_y = b + A g_x
    launch_eta(prec, T, stream);                                  // eta; phase -> 1
    CGS_HIP(hipGetLastError());
    return CGS_OK;
}

int Engine::reset(int inst) {
    launch_reset(prec, T, inst, stream);
    CGS_HIP(hipGetLastError());
    return CGS_OK;
}

int Engine::set_scalar(int inst, int slot, double v) {
    launch_set_scalar(inst_dev, inst, slot, v, stream);
    CGS_HIP(hipGetLastError());
    return CGS_OK;
}

void Engine::fill_info(int i, cgs_info* info) const {
    const double* sc = scalars(i);
    info->status = (int32_t)sc[SC_STATUS];
    info->iters = (int32_t)sc[SC_ITER];
    info->cg_iters = (int64_t)sc[SC_CGTOT];
    info->tau = sc[SC_TAU];
    info->kappa = sc[SC_KAPPA];
    const double tau = sc[SC_TAU];
    info->pobj = tau > 0.0 ? sc[SC_CUX] / tau : NAN;
    info->dobj = tau > 0.0 ? -sc[SC_BUY] / tau : NAN;
    info->res_pri = sc[SC_RP];
    info->res_dual = sc[SC_RD];
    info->gap = sc[SC_GAP];
    info->cert_precision = precision;
    info->reserved_ = 0;
}

}  // namespace cgs
