// extern "C" entry points of libcgs.so (declared in include/cgs.h).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "engine.hpp"

using cgs::fail;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool all_finite(const double* p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int check_block(const cgs_op* op, int64_t row0, int64_t col0, int64_t rows, int64_t cols, double scale) {
    if (!op) return fail(CGS_EINVAL, "operator is null");
    if (rows < 1 || cols < 1) return fail(CGS_EDIM, "block size %lld x %lld", (long long)rows, (long long)cols);
    if (row0 < 0 || col0 < 0 || row0 + rows > op->m || col0 + cols > op->n)
        return fail(CGS_EDIM, "block [%lld,%lld)x[%lld,%lld) outside the %lld x %lld operator",
                    (long long)row0, (long long)(row0 + rows), (long long)col0, (long long)(col0 + cols),
                    (long long)op->m, (long long)op->n);
    if (!std::isfinite(scale)) return fail(CGS_EINVAL, "scale is not finite");
    return CGS_OK;
}

// Device bytes of the solver: tables, reduction scratch, staging, operator data, regions.
struct SolverLayout {
    size_t tab = 0, work = 0, stg = 0, opb = 0, region = 0, snap = 0, total = 0;
    size_t panel = 0, part = 0;          // BF16 GEMM panel (hi and lo) and split-K partials
    int64_t stg_doubles = 0;
};

int solver_layout(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq, const cgs_settings* st,
                  int64_t batch, SolverLayout* L) {
    if (!op) return fail(CGS_EINVAL, "operator is null");
    CGS_TRY(cgs::validate_settings(st));
    CGS_TRY(cgs::validate_cone(op->m, l, q, nq));
    if (batch < 1 || batch > 1000000) return fail(CGS_EINVAL, "batch must be in [1, 1e6]");
    cgs::OpDev shape;
    cgs::op_dev_shape(*op, st->precision, &shape);
    std::vector<cgs::InstRec> recs((size_t)batch);
    for (auto& r : recs) {
        r.n = op->n;
        r.m = op->m;
        r.l = l;
        r.q.assign(q, q + nq);
        r.op = &shape;
    }
    cgs::TableImage im;
    cgs::build_image(recs, st->precision, im, cgs::VEC_TILE_MIN);   // (the most tiles a tuning can ask for)
    L->tab = cgs::align256(cgs::image_table_bytes(im));
    L->work = cgs::align256(cgs::image_work_bytes(im));
    L->stg_doubles = cgs::staging_doubles(*op, std::max(op->n, op->m));
    L->stg = cgs::align256((size_t)L->stg_doubles * sizeof(double));
    L->opb = cgs::align256(cgs::op_dev_bytes(*op, st->precision));
    L->region = cgs::region_bytes(op->n, op->m, st->precision);
    L->snap = st->cg_adaptive ? cgs::snap_bytes(op->n, op->m, st->precision) : 0;
    if (st->precision == CGS_BF16) {
        for (const cgs::DenseBlock& db : shape.dense) {
            for (int adj = 0; adj < 2; ++adj) {
                const int64_t N = adj ? db.cols : db.rows, kpad = adj ? db.ldt : db.ld;
                for (int target = 128; target <= cgs::GEMM_TARGET_MAX; target *= 2) {
                    const cgs::GemmPlan g = cgs::gemm_plan(N, kpad, (int)batch, target);
                    L->panel = std::max(L->panel, cgs::align256((size_t)g.mpad * kpad * 2));
                    L->part = std::max(L->part, cgs::align256(cgs::gemm_part_bytes(g)));
                }
            }
        }
    }
    L->total = L->tab + L->work + L->stg + L->opb + 3 * L->panel + L->part +
               (size_t)batch * (L->region + L->snap);
    return CGS_OK;
}

}  // namespace

struct cgs_solver {
    cgs::Engine eng;
    cgs::OpDev opdev;
    cgs::Scaling scl;
    int64_t n = 0, m = 0, batch = 0;
    std::vector<char> has_data;
    // CGS_BF16 batches: arithmetic of the operator whose residual test gave
    // each instance's outcome in the last solve
    std::vector<int> cert;
};

struct ServerReq {
    int64_t ticket = 0;
    size_t off = 0, bytes = 0;
    int64_t n = 0, m = 0, l = 0;
    std::vector<int64_t> q;
    cgs::OpDev opdev;
    bool fresh = true;        // reset + setup pending
    int eng_index = -1;       // index in the engine's tables at the last rebuild
    bool finished = false;
    cgs_info info{};
    double t_submit = 0.0;
};

struct cgs_server {
    cgs::Engine eng;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    int64_t max_slots = 0;
    int64_t next_ticket = 1;
    std::map<size_t, size_t> free_list;              // offset -> size
    std::vector<std::unique_ptr<ServerReq>> live;    // admitted, in engine order
    bool dirty = false;
    int64_t stg_doubles = 0;
};

extern "C" {

const char* cgs_last_error(void) { return cgs::last_error(); }
const char* cgs_version(void) { return "cgs 0.1 (gfx950)"; }

// ---------------------------------------------------------------- operator
int cgs_op_create(int64_t m, int64_t n, cgs_op** out) {
    if (!out) return fail(CGS_EINVAL, "out is null");
    *out = nullptr;
    if (m < 1 || n < 1) return fail(CGS_EDIM, "operator size %lld x %lld", (long long)m, (long long)n);
    cgs_op* op = new (std::nothrow) cgs_op;
    if (!op) return fail(CGS_ENOMEM, "host allocation failed");
    op->m = m;
    op->n = n;
    *out = op;
    return CGS_OK;
}

int cgs_op_add_identity(cgs_op* op, int64_t row0, int64_t col0, int64_t len, double scale) {
    CGS_TRY(check_block(op, row0, col0, len, len, scale));
    cgs::HostBlock b{};
    b.kind = CGS_BLOCK_IDENTITY;
    b.row0 = row0;
    b.col0 = col0;
    b.rows = b.cols = len;
    b.scale = scale;
    b.frob2 = (double)len;
    op->blocks.push_back(std::move(b));
    return CGS_OK;
}

int cgs_op_add_conv(cgs_op* op, int64_t row0, int64_t col0, const double* taps, int64_t k,
                    int64_t n_in, double scale) {
    if (!taps) return fail(CGS_EINVAL, "taps is null");
    if (k < 1 || k > (int64_t(1) << 24)) return fail(CGS_EDIM, "kernel length %lld", (long long)k);
    if (n_in < 1) return fail(CGS_EDIM, "n_in %lld", (long long)n_in);
    CGS_TRY(check_block(op, row0, col0, n_in + k - 1, n_in, scale));
    if (!all_finite(taps, k)) return fail(CGS_EINVAL, "taps contain a non-finite value");
    cgs::HostBlock b{};
    b.kind = CGS_BLOCK_CONV;
    b.row0 = row0;
    b.col0 = col0;
    b.rows = n_in + k - 1;
    b.cols = n_in;
    b.k = k;
    b.n_in = n_in;
    b.scale = scale;
    b.data.assign(taps, taps + k);
    b.frob2 = 0.0;   // full convolution: every column holds all k taps
    for (int64_t t = 0; t < k; ++t) b.frob2 += taps[t] * taps[t];
    b.frob2 *= (double)n_in;
    op->blocks.push_back(std::move(b));
    return CGS_OK;
}

int cgs_op_add_dense(cgs_op* op, int64_t row0, int64_t col0, int64_t rows, int64_t cols,
                     const double* a, int64_t lda, double scale) {
    return cgs_op_add_dense_ex(op, row0, col0, rows, cols, a, lda, CGS_DTYPE_F64, CGS_MEM_HOST_COPY, scale);
}

int cgs_op_add_dense_ex(cgs_op* op, int64_t row0, int64_t col0, int64_t rows, int64_t cols,
                        const void* a, int64_t lda, int32_t dtype, int32_t mem, double scale) {
    if (!a) return fail(CGS_EINVAL, "matrix is null");
    if (dtype != CGS_DTYPE_F64 && dtype != CGS_DTYPE_F32) return fail(CGS_EINVAL, "unknown dtype %d", dtype);
    if (mem != CGS_MEM_HOST_COPY && mem != CGS_MEM_DEVICE_BORROW)
        return fail(CGS_EINVAL, "unknown memory kind %d", mem);
    CGS_TRY(check_block(op, row0, col0, rows, cols, scale));
    if (lda < cols) return fail(CGS_EDIM, "lda %lld < cols %lld", (long long)lda, (long long)cols);
    cgs::HostBlock b{};
    b.kind = CGS_BLOCK_DENSE;
    b.row0 = row0;
    b.col0 = col0;
    b.rows = rows;
    b.cols = cols;
    b.scale = scale;
    if (mem == CGS_MEM_DEVICE_BORROW) {
        hipPointerAttribute_t at{};
        int cur = -1;
        CGS_HIP(hipGetDevice(&cur));
        if (hipPointerGetAttributes(&at, a) != hipSuccess || at.type != hipMemoryTypeDevice || at.device != cur) {
            (void)hipGetLastError();
            return fail(CGS_EINVAL, "a borrowed dense block must be device memory of the current device");
        }
        CGS_TRY(cgs::dense_frob2_device(a, dtype, rows, cols, lda, &b.frob2));
        b.dev = a;
        b.dev_dtype = dtype;
        b.dev_ld = lda;
        b.dev_id = cur;
        op->blocks.push_back(std::move(b));
        return CGS_OK;
    }
    try {
        b.data.resize((size_t)(rows * cols));
    } catch (...) {
        return fail(CGS_ENOMEM, "host allocation of %lld doubles failed", (long long)(rows * cols));
    }
    // each row's squares in column order, then the row sums in row order (the
    // order the device forms it in for a borrowed block)
    b.frob2 = 0.0;
    for (int64_t i = 0; i < rows; ++i) {
        double* dst = b.data.data() + i * cols;
        if (dtype == CGS_DTYPE_F64) {
            const double* src = (const double*)a + i * lda;
            if (!all_finite(src, cols)) return fail(CGS_EINVAL, "matrix row %lld has a non-finite value", (long long)i);
            std::memcpy(dst, src, (size_t)cols * sizeof(double));
        } else {
            const float* src = (const float*)a + i * lda;
            for (int64_t j = 0; j < cols; ++j) {
                if (!std::isfinite(src[j]))
                    return fail(CGS_EINVAL, "matrix row %lld has a non-finite value", (long long)i);
                dst[j] = (double)src[j];
            }
        }
        double rs = 0.0;
        for (int64_t j = 0; j < cols; ++j) rs += dst[j] * dst[j];
        b.frob2 += rs;
    }
    op->blocks.push_back(std::move(b));
    return CGS_OK;
}

int cgs_op_info(const cgs_op* op, int64_t* m, int64_t* n, int64_t* nblocks) {
    if (!op) return fail(CGS_EINVAL, "operator is null");
    if (m) *m = op->m;
    if (n) *n = op->n;
    if (nblocks) *nblocks = (int64_t)op->blocks.size();
    return CGS_OK;
}

int cgs_op_equilibrate(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq, int32_t level,
                       const double* b, const double* c, double* d, double* e, double* sigma) {
    if (!op) return fail(CGS_EINVAL, "operator is null");
    CGS_TRY(cgs::validate_cone(op->m, l, q, nq));
    if (level < 0 || level > 2) return fail(CGS_EINVAL, "level must be 0, 1 or 2");
    if ((b == nullptr) != (c == nullptr)) return fail(CGS_EINVAL, "give both b and c, or neither");
    cgs::Scaling scl;
    cgs::compute_scaling(*op, l, q, nq, level, &scl);
    std::vector<double> dv((size_t)op->m), ev((size_t)op->n), bh((size_t)op->m), ch((size_t)op->n);
    std::vector<double> zb((size_t)op->m, 0.0), zc((size_t)op->n, 0.0);
    double sb = 1.0, sc = 1.0;
    cgs::scale_data(scl, op->m, op->n, b ? b : zb.data(), c ? c : zc.data(), dv.data(), ev.data(),
                    bh.data(), ch.data(), &sb, &sc);
    if (d) std::memcpy(d, dv.data(), dv.size() * sizeof(double));
    if (e) std::memcpy(e, ev.data(), ev.size() * sizeof(double));
    if (sigma && b) {
        sigma[0] = sb;
        sigma[1] = sc;
    }
    return CGS_OK;
}

void cgs_op_destroy(cgs_op* op) { delete op; }

// ---------------------------------------------------------------- settings
void cgs_settings_default(cgs_settings* st) {
    if (!st) return;
    std::memset(st, 0, sizeof *st);
    st->eps = 1e-4;
    st->alpha = 1.5;
    st->max_iters = 100000;
    st->check_every = 10;
    st->precision = CGS_FP32;
    st->cg_max_iters = 10;
    st->cg_tol = 0.1;
    st->cg_rate = 1.5;
    st->cg_floor = 1e-6;
    st->setup_tol = 1e-7;
    st->setup_max_iters = 500;
    st->use_graph = 1;
    st->bf16_phase1_digits = 3;
    st->cg_adaptive = 1;
    st->fused_max = 16384;
    st->fused_lone_max = 8192;
    st->conv_mfma = 2;
    st->normalize = 1;
    st->intervals_per_sync = 2;
}

// Equilibrated data of one instance written into its region (layout of
// common.hpp): b^ = sb D b and c^ = sc E c, the scaling vectors D and E, and
// the data scales sb, sc.
static int upload_instance_data(cgs::Engine& e, const cgs::Scaling& scl, char* base, int64_t n,
                                int64_t m, const double* b, const double* c) {
    std::vector<double> dv, ev, bh, ch;
    try {
        dv.resize((size_t)m); bh.resize((size_t)m);
        ev.resize((size_t)n); ch.resize((size_t)n);
    } catch (...) {
        return fail(CGS_ENOMEM, "host allocation failed");
    }
    double sc2[2];
    cgs::scale_data(scl, m, n, b, c, dv.data(), ev.data(), bh.data(), ch.data(), &sc2[0], &sc2[1]);
    const size_t sz = cgs::elem_bytes(e.precision);
    const int64_t nxs = cgs::round_up(n, cgs::XY_ALIGN), nys = cgs::round_up(m, cgs::XY_ALIGN);
    auto xv = [&](int k) { return base + cgs::REGION_HDR + (size_t)k * nxs * sz; };
    auto yv = [&](int k) { return base + cgs::REGION_HDR + ((size_t)cgs::NXV * nxs + (size_t)k * nys) * sz; };
    CGS_TRY(cgs::upload_f64(e.stg, e.stream, bh.data(), m, e.prec, yv(cgs::YB)));
    CGS_TRY(cgs::upload_f64(e.stg, e.stream, dv.data(), m, e.prec, yv(cgs::YD)));
    CGS_TRY(cgs::upload_f64(e.stg, e.stream, ch.data(), n, e.prec, xv(cgs::XC)));
    CGS_TRY(cgs::upload_f64(e.stg, e.stream, ev.data(), n, e.prec, xv(cgs::XE)));
    CGS_TRY(cgs::upload_raw(e.stg, e.stream, sc2, sizeof sc2, base + cgs::SC_SB * sizeof(double)));
    return CGS_OK;
}

// ---------------------------------------------------------------- solver
int cgs_workspace_bytes(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq,
                        const cgs_settings* st, int64_t batch, size_t* bytes) {
    if (!bytes) return fail(CGS_EINVAL, "bytes is null");
    SolverLayout L;
    CGS_TRY(solver_layout(op, l, q, nq, st, batch, &L));
    *bytes = L.total;
    return CGS_OK;
}

int cgs_solver_create(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq,
                      const cgs_settings* st, int64_t batch, void* workspace, size_t ws_bytes,
                      void* stream, cgs_solver** out) {
    return cgs::solver_create(op, l, q, nq, st, batch, workspace, ws_bytes, stream, false, out);
}

}  // extern "C"

int cgs::solver_create(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq, const cgs_settings* st,
                       int64_t batch, void* workspace, size_t ws_bytes, void* stream, bool pageable,
                       cgs_solver** out) {
    if (!out) return fail(CGS_EINVAL, "out is null");
    *out = nullptr;
    SolverLayout L;
    CGS_TRY(solver_layout(op, l, q, nq, st, batch, &L));
    if (!workspace) return fail(CGS_EINVAL, "workspace is null");
    if ((uintptr_t)workspace % 256) return fail(CGS_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total) return fail(CGS_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    std::unique_ptr<cgs_solver> s(new (std::nothrow) cgs_solver);
    if (!s) return fail(CGS_ENOMEM, "host allocation failed");
    cgs::Engine& e = s->eng;
    e.precision = st->precision;
    e.prec = cgs::work_prec(st->precision);
    e.st = *st;
    e.stream = (hipStream_t)stream;
    e.cg_launch = st->cg_max_iters;
    e.vec_tile = st->vec_tile ? st->vec_tile : cgs::VEC_TILE;
    e.lone = batch == 1 ? 1 : 0;
    e.pageable = pageable;
    char* p = (char*)workspace;
    e.tab_dev = p; e.tab_cap = L.tab; p += L.tab;
    e.work_dev = p; e.work_cap = L.work; p += L.work;
    CGS_TRY(e.init_host_buffers(L.tab, (int)batch, L.stg_doubles));
    e.stg.dev = (double*)p; p += L.stg;
    char* opdata = p; p += L.opb;
    if (st->precision == CGS_BF16 && L.part > 0) {
        e.use_gemm = 1;
        e.panel = (uint16_t*)p; p += 3 * L.panel;
        e.panel_stride = L.panel / sizeof(uint16_t);
        e.gemm_part = (float*)p; p += L.part;
    }
    e.snap_dev = L.snap ? p : nullptr;
    e.snap_cap = (size_t)batch * L.snap;
    p += e.snap_cap;
    cgs::compute_scaling(*op, l, q, nq, st->normalize, &s->scl);
    CGS_TRY(cgs::op_upload(*op, st->precision, opdata, e.stg, e.stream, &s->opdev, s->scl.blk.data()));
    std::vector<cgs::InstRec> recs((size_t)batch);
    for (int64_t i = 0; i < batch; ++i) {
        recs[i].base = p + (size_t)i * L.region;
        recs[i].n = op->n;
        recs[i].m = op->m;
        recs[i].l = l;
        recs[i].q.assign(q, q + nq);
        recs[i].op = &s->opdev;
    }
    CGS_TRY(e.build(recs));
    CGS_TRY(e.reset(-1));
    // every instance stays inactive until its data arrive
    for (int64_t i = 0; i < batch; ++i) CGS_TRY(e.set_scalar((int)i, cgs::SC_ACTIVE, 0.0));
    CGS_HIP(hipStreamSynchronize(e.stream));
    s->n = op->n;
    s->m = op->m;
    s->batch = batch;
    s->has_data.assign((size_t)batch, 0);
    s->cert.assign((size_t)batch, st->precision);
    *out = s.release();
    return CGS_OK;
}

extern "C" {

int cgs_solver_set_data(cgs_solver* s, int64_t inst, const double* b, const double* c) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    if (inst < 0 || inst >= s->batch) return fail(CGS_ENOTFOUND, "instance %lld of %lld", (long long)inst, (long long)s->batch);
    if (!b || !c) return fail(CGS_EINVAL, "b or c is null");
    if (!all_finite(b, s->m)) return fail(CGS_EINVAL, "b has a non-finite entry");
    if (!all_finite(c, s->n)) return fail(CGS_EINVAL, "c has a non-finite entry");
    cgs::Engine& e = s->eng;
    CGS_TRY(e.reset((int)inst));
    CGS_TRY(upload_instance_data(e, s->scl, e.recs[(size_t)inst].base, s->n, s->m, b, c));
    CGS_HIP(hipStreamSynchronize(e.stream));
    s->has_data[(size_t)inst] = 1;
    return CGS_OK;
}

int cgs_solver_reset(cgs_solver* s, int64_t inst) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    if (inst >= s->batch) return fail(CGS_ENOTFOUND, "instance %lld", (long long)inst);
    cgs::Engine& e = s->eng;
    CGS_TRY(e.reset(inst < 0 ? -1 : (int)inst));
    for (int64_t i = 0; i < s->batch; ++i)
        if ((inst < 0 || i == inst) && !s->has_data[(size_t)i]) CGS_TRY(e.set_scalar((int)i, cgs::SC_ACTIVE, 0.0));
    CGS_HIP(hipStreamSynchronize(e.stream));
    return CGS_OK;
}

int cgs_solver_kernel_time(cgs_solver* s, int32_t kernel, int32_t reps, double* avg_ms) {
    if (!s || !avg_ms) return fail(CGS_EINVAL, "null argument");
    if (reps < 1 || kernel < 0 || kernel > 4) return fail(CGS_EINVAL, "bad kernel / reps");
    cgs::Engine& e = s->eng;
    const std::vector<cgs::ConvLaunch>& cl = kernel == 1 ? e.ca : e.cf;
    const std::vector<cgs::DenseLaunch>& dl = kernel == 3 ? e.da : e.df;
    if ((kernel <= 1 && cl.empty()) || ((kernel == 2 || kernel == 3) && dl.empty()))
        return fail(CGS_ENOTFOUND, "the operator has no block of that kind");
    hipEvent_t a, b;
    CGS_HIP(hipEventCreate(&a));
    CGS_HIP(hipEventCreate(&b));
    CGS_HIP(hipEventRecord(a, e.stream));
    int launches = 0;
    for (int r = 0; r < reps; ++r) {
        if (kernel <= 1) {
            // A u_x into the scratch Y vector, A^T u_y into the scratch X vector
            for (const auto& c : cl)
                e.conv(c, kernel, kernel ? cgs::XT : cgs::YT, kernel ? cgs::YU : cgs::XU, -1, 1.0, cgs::G_ALL),
                    ++launches;
        } else if (kernel <= 3) {
            const int adj = kernel == 3;
            if (e.use_gemm) {
                // the batch's dense applies: pack + BF16 MFMA GEMM + reduce
                for (const cgs::DenseBlock& db : s->opdev.dense)
                    cgs::launch_gemm_apply(e.T, db, adj, adj ? cgs::XT : cgs::YT, adj ? cgs::YU : cgs::XU, 1.0,
                                           cgs::G_ALL, e.gemm_corr, e.panel, e.panel_stride, e.gemm_part,
                                           e.gemm_target, e.stream),
                        ++launches;
            } else {
                for (const auto& d : dl)
                    cgs::launch_gemv(e.prec, e.T, d, adj, adj ? cgs::XT : cgs::YT, adj ? cgs::YU : cgs::XU,
                                     1.0, cgs::G_ALL, e.stream), ++launches;
            }
        } else {
            e.apply(0, cgs::YT, cgs::XP, -1, 1.0, cgs::G_ALL);
            e.apply(1, cgs::XT, cgs::YT, cgs::XP, 1.0, cgs::G_ALL);
            ++launches;
        }
    }
    CGS_HIP(hipEventRecord(b, e.stream));
    CGS_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    CGS_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    CGS_HIP(hipGetLastError());
    *avg_ms = (double)ms / launches;
    return CGS_OK;
}

static int run_setup_if_needed(cgs_solver* s, bool* did);

// Every instance back to u = v = (0, 0, 1) with its data kept; instances
// without data stay inactive (cgs_solver_reset).
static int restart_all(cgs_solver* s) {
    cgs::Engine& e = s->eng;
    CGS_TRY(e.reset(-1));
    for (int64_t i = 0; i < s->batch; ++i)
        if (!s->has_data[(size_t)i]) CGS_TRY(e.set_scalar((int)i, cgs::SC_ACTIVE, 0.0));
    CGS_HIP(hipStreamSynchronize(e.stream));
    return CGS_OK;
}

// Device time of one ADMM step of every instance with the current kernel
// choices, from a fresh start: setup, three untimed steps, then `reps` steps
// between HIP events (one CG launch per step, the count the solve settles on
// once its first steps are past); the instances restart afterwards.
static int time_steps(cgs_solver* s, int reps, double* ms_per_step) {
    cgs::Engine& e = s->eng;
    CGS_TRY(restart_all(s));
    CGS_TRY(run_setup_if_needed(s, nullptr));
    e.refresh();
    const int keep = e.cg_launch;
    e.cg_launch = 1;
    for (int i = 0; i < 3; ++i) e.admm_step();
    hipEvent_t a, b;
    CGS_HIP(hipEventCreate(&a));
    CGS_HIP(hipEventCreate(&b));
    CGS_HIP(hipEventRecord(a, e.stream));
    for (int i = 0; i < reps; ++i) e.admm_step();
    CGS_HIP(hipEventRecord(b, e.stream));
    CGS_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    CGS_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    e.cg_launch = keep;
    CGS_HIP(hipGetLastError());
    *ms_per_step = (double)ms / reps;
    return restart_all(s);
}

int cgs_solver_autotune(cgs_solver* s, int32_t reps, int32_t* choice) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    if (reps < 1) return fail(CGS_EINVAL, "reps must be >= 1");
    cgs::Engine& e = s->eng;
    bool have_data = true;
    for (int64_t i = 0; i < s->batch; ++i) have_data = have_data && s->has_data[(size_t)i];
    bool fft = false;
    for (const auto& c : e.cf) fft = fft || c.fft;
    std::vector<int> engines, tiles, targets;
    if (!e.cf.empty() && e.prec == 1) {
        engines = {0, 1};
        if (fft) engines.push_back(2);
    } else {
        engines = {e.st.conv_mfma};
    }
    if (e.use_gemm) {
        for (int t = 128; t <= cgs::GEMM_TARGET_MAX; t *= 2) targets.push_back(t);
    } else {
        targets = {e.gemm_target};
    }
    // vector tiles only matter on the one-launch-per-kernel path
    if (have_data && e.n_multi > 0) tiles = {cgs::VEC_TILE_MIN, cgs::VEC_TILE};
    else tiles = {e.vec_tile};
    int best_m = e.st.conv_mfma, best_t = e.gemm_target, best_v = e.vec_tile;
    // BF16 products are timed with their refinement terms (the hi/lo phase,
    // where a BF16 solve spends most of its applies)
    const int keep_corr = e.gemm_corr;
    if (e.use_gemm) e.gemm_corr = 1;
    if (have_data && e.n_multi > 0) {
        // every combination timed on whole ADMM steps of the solver's own
        // instances: the launches the solve runs, folded ones included
        double best = 0.0;
        bool first = true;
        for (int v : tiles) {
            if (v != e.vec_tile) {
                e.vec_tile = v;
                CGS_TRY(e.build(e.recs));
            }
            for (int m : engines) {
                for (int t : targets) {
                    e.st.conv_mfma = m;
                    e.gemm_target = t;
                    double ms = 0.0;
                    CGS_TRY(time_steps(s, reps, &ms));
                    if (first || ms < best) {
                        best = ms;
                        best_m = m;
                        best_t = t;
                        best_v = v;
                        first = false;
                    }
                }
            }
        }
        e.st.conv_mfma = best_m;
        e.gemm_target = best_t;
        if (best_v != e.vec_tile) {
            e.vec_tile = best_v;
            CGS_TRY(e.build(e.recs));
        }
        CGS_TRY(restart_all(s));
    } else {
        // no data yet (or every instance on the fused path): the operator's
        // launches alone, A and A^T
        if (engines.size() > 1) {
            double best = 0.0;
            for (int m : engines) {
                e.st.conv_mfma = m;
                double a = 0.0, b = 0.0;
                // untimed first launches: the runtime loads a kernel's code on its
                // first launch, which the events would otherwise count
                CGS_TRY(cgs_solver_kernel_time(s, 0, 1, &a));
                CGS_TRY(cgs_solver_kernel_time(s, 1, 1, &b));
                CGS_TRY(cgs_solver_kernel_time(s, 0, reps, &a));
                CGS_TRY(cgs_solver_kernel_time(s, 1, reps, &b));
                if (m == engines[0] || a + b < best) {
                    best = a + b;
                    best_m = m;
                }
            }
            e.st.conv_mfma = best_m;
        }
        if (e.use_gemm) {
            double best = 0.0;
            for (int target : targets) {
                e.gemm_target = target;
                double a = 0.0, b = 0.0;
                CGS_TRY(cgs_solver_kernel_time(s, 2, 1, &a));
                CGS_TRY(cgs_solver_kernel_time(s, 3, 1, &b));
                CGS_TRY(cgs_solver_kernel_time(s, 2, reps, &a));
                CGS_TRY(cgs_solver_kernel_time(s, 3, reps, &b));
                if (target == targets[0] || a + b < best) {
                    best = a + b;
                    best_t = target;
                }
            }
            e.gemm_target = best_t;
        }
    }
    e.gemm_corr = keep_corr;
    e.drop_graph();
    if (choice) {
        choice[0] = (!e.cf.empty() && e.prec == 1) ? e.st.conv_mfma : -1;
        choice[1] = e.use_gemm ? e.gemm_target : -1;
        choice[2] = e.vec_tile;
        choice[3] = -1;
    }
    return CGS_OK;
}

static int ensure_data(cgs_solver* s) {
    for (int64_t i = 0; i < s->batch; ++i)
        if (!s->has_data[(size_t)i]) return fail(CGS_ESTATE, "instance %lld has no data", (long long)i);
    return CGS_OK;
}

static int run_setup_if_needed(cgs_solver* s, bool* did) {
    cgs::Engine& e = s->eng;
    CGS_TRY(e.fetch_scalars());
    bool need = false;
    for (int i = 0; i < e.T.ninst; ++i) {
        const double* sc = e.scalars(i);
        if (sc[cgs::SC_ACTIVE] != 0.0 && sc[cgs::SC_PHASE] == 0.0) need = true;
    }
    if (need) CGS_TRY(e.setup());
    if (did) *did = need;
    return CGS_OK;
}

static int solve_rounds(cgs_solver* s);

int cgs_solve(cgs_solver* s, cgs_info* info) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    CGS_TRY(ensure_data(s));
    cgs::Engine& e = s->eng;
    const double t0 = now_s();
    double t1 = t0;
    if (e.use_gemm) {
        // Phase 1: BF16 products, to max(eps, 10^-digits).  Phase 2: the
        // refinement operator (hi/lo products) from phase 1's state, with the
        // embedding vector recomputed for that operator, to eps * kPhase2Margin.
        // Phase 3: the FP32 operator (dense products on the vector ALU from the
        // FP32 copy of the blocks): the residual test runs on it at phase 2's
        // point, and an instance that fails it iterates on that operator (with
        // its own embedding vector) until it passes.  The reported status is
        // always that of the FP32 operator's test (cgs_info.cert_precision).
        constexpr double kPhase2Margin = 0.5;
        const double eps = e.st.eps;
        const double eps1 = std::max(eps, std::pow(10.0, -(double)e.st.bf16_phase1_digits));
        const double eps2 = eps * kPhase2Margin;
        std::fill(s->cert.begin(), s->cert.end(), CGS_BF16);
        e.gemm_corr = 0;
        e.st.eps = std::max(eps1, eps2);
        e.drop_graph();
        CGS_TRY(run_setup_if_needed(s, nullptr));
        e.refresh();
        t1 = now_s();
        int rc = solve_rounds(s);
        e.st.eps = eps;
        if (rc != CGS_OK) return rc;
        auto reopen = [&](double phase) -> int {
            // instances the last phase solved run again (the others keep their outcome)
            CGS_TRY(e.fetch_scalars());
            int n = 0;
            for (int i = 0; i < e.T.ninst; ++i) {
                if (e.scalars(i)[cgs::SC_STATUS] != (double)CGS_SOLVED) continue;
                CGS_TRY(e.set_scalar(i, cgs::SC_STATUS, 0.0));
                CGS_TRY(e.set_scalar(i, cgs::SC_ACTIVE, 1.0));
                CGS_TRY(e.set_scalar(i, cgs::SC_PHASE, phase));
                ++n;
            }
            return n;
        };
        if (eps1 > eps2) {
            const int r = reopen(0.0);
            if (r < 0) return r;
            e.gemm_corr = 1;
            e.st.eps = eps2;
            e.drop_graph();
            CGS_TRY(run_setup_if_needed(s, nullptr));
            e.refresh();
            rc = solve_rounds(s);
            e.st.eps = eps;
            if (rc != CGS_OK) return rc;
        }
        // phase 3
        const int nre = reopen(1.0);
        if (nre < 0) return nre;
        e.use_gemm = 0;
        e.gemm_corr = 0;
        e.drop_graph();
        rc = CGS_OK;
        if (nre > 0) {
            e.check(cgs::G_CHECK_ANY);   // the test alone: no step, no carried products
            rc = e.fetch_scalars();
            for (int i = 0; rc == CGS_OK && i < e.T.ninst; ++i) {
                const double* sc = e.scalars(i);
                s->cert[(size_t)i] = CGS_FP32;
                if (sc[cgs::SC_ACTIVE] != 0.0 && sc[cgs::SC_PHASE] == 1.0)
                    rc = e.set_scalar(i, cgs::SC_PHASE, 0.0);   // iterate: setup for this operator
            }
            if (rc == CGS_OK) rc = run_setup_if_needed(s, nullptr);
            if (rc == CGS_OK) {
                e.refresh();
                rc = solve_rounds(s);
            }
        }
        e.use_gemm = 1;
        e.drop_graph();
        if (rc != CGS_OK) return rc;
    } else {
        CGS_TRY(run_setup_if_needed(s, nullptr));
        e.refresh();   // carried A z, (I + A^T A) z of the warm start
        t1 = now_s();
        CGS_TRY(solve_rounds(s));
    }
    const double t2 = now_s();
    if (info) {
        for (int i = 0; i < e.T.ninst; ++i) {
            e.fill_info(i, &info[i]);
            info[i].setup_s = t1 - t0;
            info[i].solve_s = t2 - t1;
            info[i].cert_precision = e.use_gemm ? s->cert[(size_t)i] : e.precision;
        }
    }
    return CGS_OK;
}

// ADMM rounds (check_every steps + termination test) until no instance runs.
static int solve_rounds(cgs_solver* s) {
    cgs::Engine& e = s->eng;
    for (;;) {
        CGS_TRY(e.fetch_scalars());
        if (e.truncated()) {
            // a step of the last interval needed more CG launches than it had
            CGS_TRY(e.rollback());
            continue;
        }
        e.spec_launch = 0;
        bool any = false;
        double min_it = 1e300;
        for (int i = 0; i < e.T.ninst; ++i) {
            const double* sc = e.scalars(i);
            if (sc[cgs::SC_ACTIVE] != 0.0 && sc[cgs::SC_PHASE] >= 1.0) {
                any = true;
                min_it = std::min(min_it, sc[cgs::SC_ITER]);
            }
        }
        if (!any) break;
        const int64_t rem = (int64_t)e.st.max_iters - (int64_t)min_it;
        const int nsteps = (int)std::max<int64_t>(1, std::min<int64_t>(e.round_steps(), rem));
        e.adapt_cg();
        CGS_TRY(e.round(nsteps));
    }
    return CGS_OK;
}

int cgs_solver_iterate(cgs_solver* s, int32_t iters) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    if (iters < 0) return fail(CGS_EINVAL, "iters < 0");
    CGS_TRY(ensure_data(s));
    cgs::Engine& e = s->eng;
    CGS_TRY(run_setup_if_needed(s, nullptr));
    e.cg_launch = e.st.cg_max_iters;
    e.refresh();
    if (e.n_fused) e.fused_steps(iters, 0);
    if (e.n_multi)
        for (int i = 0; i < iters; ++i) e.admm_step();
    CGS_HIP(hipGetLastError());
    CGS_HIP(hipStreamSynchronize(e.stream));
    return CGS_OK;
}

int cgs_solver_rounds(cgs_solver* s, int64_t* rounds, int64_t* reruns) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    if (rounds) *rounds = s->eng.n_rounds;
    if (reruns) *reruns = s->eng.n_reruns;
    return CGS_OK;
}

int cgs_solver_get_solution(cgs_solver* s, int64_t inst, double* x, double* y, double* sl) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    if (inst < 0 || inst >= s->batch) return fail(CGS_ENOTFOUND, "instance %lld", (long long)inst);
    cgs::Engine& e = s->eng;
    double* outs[3] = {x, y, sl};
    const int64_t lens[3] = {s->n, s->m, s->m};
    for (int w = 0; w < 3; ++w) {
        if (!outs[w]) continue;
        for (int64_t off = 0; off < lens[w]; off += e.stg.cap) {
            const int64_t c = std::min(e.stg.cap, lens[w] - off);
            cgs::launch_extract(e.prec, e.inst_dev, (int)inst, w, off, c, e.stg.dev, e.stream);
            CGS_HIP(hipGetLastError());
            CGS_HIP(hipMemcpyAsync(e.stg.host, e.stg.dev, c * sizeof(double), hipMemcpyDeviceToHost, e.stream));
            CGS_HIP(hipStreamSynchronize(e.stream));
            std::memcpy(outs[w] + off, e.stg.host, c * sizeof(double));
        }
    }
    return CGS_OK;
}

int cgs_solver_get_state(cgs_solver* s, int64_t inst, double* ux, double* uy, double* vs, double* scal) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    if (inst < 0 || inst >= s->batch) return fail(CGS_ENOTFOUND, "instance %lld", (long long)inst);
    cgs::Engine& e = s->eng;
    const int i = (int)inst;
    if (ux) CGS_TRY(cgs::download_f64(e.stg, e.stream, e.prec, e.xptr(i, cgs::XU), s->n, ux));
    if (uy) CGS_TRY(cgs::download_f64(e.stg, e.stream, e.prec, e.yptr(i, cgs::YU), s->m, uy));
    if (vs) CGS_TRY(cgs::download_f64(e.stg, e.stream, e.prec, e.yptr(i, cgs::YV), s->m, vs));
    if (scal) {
        CGS_TRY(e.fetch_scalars());
        scal[0] = e.scalars(i)[cgs::SC_TAU];
        scal[1] = e.scalars(i)[cgs::SC_KAPPA];
    }
    return CGS_OK;
}

int cgs_solver_set_state(cgs_solver* s, int64_t inst, const double* ux, const double* uy,
                         const double* vs, const double* scal) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    if (inst < 0 || inst >= s->batch) return fail(CGS_ENOTFOUND, "instance %lld", (long long)inst);
    if (!ux || !uy || !vs || !scal) return fail(CGS_EINVAL, "state pointer is null");
    if (!all_finite(ux, s->n) || !all_finite(uy, s->m) || !all_finite(vs, s->m) || !all_finite(scal, 2))
        return fail(CGS_EINVAL, "state has a non-finite entry");
    if (scal[0] < 0.0 || scal[1] < 0.0) return fail(CGS_EINVAL, "tau and kappa must be >= 0");
    cgs::Engine& e = s->eng;
    const int i = (int)inst;
    CGS_TRY(cgs::upload_f64(e.stg, e.stream, ux, s->n, e.prec, e.xptr(i, cgs::XU)));
    CGS_TRY(cgs::upload_f64(e.stg, e.stream, uy, s->m, e.prec, e.yptr(i, cgs::YU)));
    CGS_TRY(cgs::upload_f64(e.stg, e.stream, vs, s->m, e.prec, e.yptr(i, cgs::YV)));
    CGS_TRY(e.set_scalar(i, cgs::SC_TAU, scal[0]));
    CGS_TRY(e.set_scalar(i, cgs::SC_KAPPA, scal[1]));
    CGS_TRY(e.set_scalar(i, cgs::SC_STATUS, 0.0));
    CGS_TRY(e.set_scalar(i, cgs::SC_ACTIVE, s->has_data[(size_t)i] ? 1.0 : 0.0));
    CGS_HIP(hipStreamSynchronize(e.stream));
    return CGS_OK;
}

int cgs_solver_residuals(cgs_solver* s, cgs_info* info) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    CGS_TRY(ensure_data(s));
    cgs::Engine& e = s->eng;
    CGS_TRY(run_setup_if_needed(s, nullptr));
    e.check(cgs::G_CHECK_ANY);   // every iterating instance, whichever path it runs on
    CGS_HIP(hipGetLastError());
    CGS_TRY(e.fetch_scalars());
    if (info)
        for (int i = 0; i < e.T.ninst; ++i) {
            e.fill_info(i, &info[i]);
            info[i].setup_s = info[i].solve_s = 0.0;
        }
    return CGS_OK;
}

int cgs_solver_apply(cgs_solver* s, int32_t transpose, const double* in, double* out) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    if (!in || !out) return fail(CGS_EINVAL, "in/out is null");
    cgs::Engine& e = s->eng;
    const int64_t nin = transpose ? s->m : s->n, nout = transpose ? s->n : s->m;
    if (!all_finite(in, nin)) return fail(CGS_EINVAL, "input has a non-finite entry");
    if (!transpose) {
        CGS_TRY(cgs::upload_f64(e.stg, e.stream, in, nin, e.prec, e.xptr(0, cgs::XT)));
        e.apply(0, cgs::YT, cgs::XT, -1, 1.0, cgs::G_ALL);
        CGS_HIP(hipGetLastError());
        CGS_TRY(cgs::download_f64(e.stg, e.stream, e.prec, e.yptr(0, cgs::YT), nout, out));
    } else {
        CGS_TRY(cgs::upload_f64(e.stg, e.stream, in, nin, e.prec, e.yptr(0, cgs::YT)));
        e.apply(1, cgs::XT, cgs::YT, -1, 1.0, cgs::G_ALL);
        CGS_HIP(hipGetLastError());
        CGS_TRY(cgs::download_f64(e.stg, e.stream, e.prec, e.xptr(0, cgs::XT), nout, out));
    }
    return CGS_OK;
}

int cgs_solver_normal_solve(cgs_solver* s, const double* rhs, const double* z0, double* z,
                            double tol, int32_t max_iters, int32_t* iters) {
    if (!s) return fail(CGS_EINVAL, "solver is null");
    if (!rhs || !z) return fail(CGS_EINVAL, "rhs/z is null");
    if (!(tol >= 0.0) || max_iters < 0) return fail(CGS_EINVAL, "bad tol / max_iters");
    if (!all_finite(rhs, s->n) || (z0 && !all_finite(z0, s->n))) return fail(CGS_EINVAL, "non-finite input");
    cgs::Engine& e = s->eng;
    CGS_TRY(cgs::upload_f64(e.stg, e.stream, rhs, s->n, e.prec, e.xptr(0, cgs::XH)));
    if (z0) CGS_TRY(cgs::upload_f64(e.stg, e.stream, z0, s->n, e.prec, e.xptr(0, cgs::XZ)));
    else cgs::launch_fill(e.prec, e.T, 0, cgs::XZ, 0.0, cgs::G_ALL, e.stream);
    e.apply(0, cgs::YT, cgs::XZ, -1, 1.0, cgs::G_ALL);
    e.apply(1, cgs::XQ, cgs::YT, cgs::XZ, 1.0, cgs::G_ALL);
    cgs::launch_cg_init(e.prec, e.T, cgs::XZ, cgs::XR, cgs::XP, cgs::XQ, cgs::XH, 1, 0.0, 0.0, tol,
                        max_iters, cgs::G_ALL, e.stream);
    int done = 0;
    while (done < max_iters) {
        const int nb = std::min(8, max_iters - done);
        for (int j = 0; j < nb; ++j) e.cg_iter(cgs::XZ, cgs::G_ANY_CG, max_iters, 0, done + j);
        done += nb;
        CGS_TRY(e.fetch_scalars());
        if (e.scalars(0)[cgs::SC_CGACT] == 0.0) break;
    }
    CGS_TRY(e.fetch_scalars());
    if (iters) *iters = (int32_t)e.scalars(0)[cgs::SC_CGIT];
    CGS_TRY(cgs::download_f64(e.stg, e.stream, e.prec, e.xptr(0, cgs::XZ), s->n, z));
    return CGS_OK;
}

void cgs_solver_destroy(cgs_solver* s) {
    if (s) (void)hipStreamSynchronize(s->eng.stream);
    delete s;
}

// ---------------------------------------------------------------- server
int cgs_server_request_bytes(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq,
                             int32_t precision, size_t* bytes) {
    if (!op || !bytes) return fail(CGS_EINVAL, "null argument");
    if (precision < CGS_FP64 || precision > CGS_FP32) return fail(CGS_EINVAL, "server precision must be FP64 or FP32");
    CGS_TRY(cgs::validate_cone(op->m, l, q, nq));
    *bytes = cgs::region_bytes(op->n, op->m, precision) + cgs::align256(cgs::op_dev_bytes(*op, precision));
    return CGS_OK;
}

int cgs_server_create(int64_t max_slots, const cgs_settings* st, void* workspace, size_t ws_bytes,
                      void* stream, cgs_server** out) {
    if (!out) return fail(CGS_EINVAL, "out is null");
    *out = nullptr;
    CGS_TRY(cgs::validate_settings(st));
    if (st->precision == CGS_BF16) return fail(CGS_EINVAL, "server precision must be FP64 or FP32");
    if (max_slots < 1 || max_slots > 100000) return fail(CGS_EINVAL, "max_slots must be in [1, 1e5]");
    if (!workspace || (uintptr_t)workspace % 256) return fail(CGS_EINVAL, "workspace must be non-null and 256-byte aligned");
    std::unique_ptr<cgs_server> sv(new (std::nothrow) cgs_server);
    if (!sv) return fail(CGS_ENOMEM, "host allocation failed");
    cgs::Engine& e = sv->eng;
    e.precision = st->precision;
    e.prec = cgs::work_prec(st->precision);
    e.st = *st;
    e.stream = (hipStream_t)stream;
    e.st.cg_adaptive = 0;     // results must not depend on the other requests in the mix
    e.st.intervals_per_sync = 1;   // requests arrive and leave at every check
    e.cg_launch = st->cg_max_iters;
    // tables and reduction scratch: a fixed slice of the workspace
    const size_t tab = cgs::align256(std::max<size_t>(size_t(1) << 20, ws_bytes / 64));
    const size_t work = tab;
    sv->stg_doubles = int64_t(1) << 20;
    const size_t stg = cgs::align256((size_t)sv->stg_doubles * sizeof(double));
    if (ws_bytes < tab + work + stg + (size_t(1) << 20))
        return fail(CGS_ENOMEM, "server workspace too small (%zu bytes)", ws_bytes);
    char* p = (char*)workspace;
    e.tab_dev = p; e.tab_cap = tab; p += tab;
    e.work_dev = p; e.work_cap = work; p += work;
    e.stg.dev = (double*)p; p += stg;
    CGS_TRY(e.init_host_buffers(tab, (int)max_slots, sv->stg_doubles));
    sv->arena = p;
    sv->arena_bytes = ws_bytes - (size_t)(p - (char*)workspace);
    sv->arena_bytes &= ~size_t(255);
    sv->free_list[0] = sv->arena_bytes;
    sv->max_slots = max_slots;
    *out = sv.release();
    return CGS_OK;
}

static bool arena_alloc(cgs_server* sv, size_t bytes, size_t* off) {
    for (auto it = sv->free_list.begin(); it != sv->free_list.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t noff = it->first + bytes;
            sv->free_list.erase(it);
            if (rest) sv->free_list[noff] = rest;
            return true;
        }
    }
    return false;
}

static void arena_free(cgs_server* sv, size_t off, size_t bytes) {
    auto it = sv->free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != sv->free_list.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        sv->free_list.erase(nx);
    }
    if (it != sv->free_list.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            sv->free_list.erase(it);
        }
    }
}

int cgs_server_submit(cgs_server* sv, const cgs_op* op, int64_t l, const int64_t* q, int64_t nq,
                      const double* b, const double* c, int64_t* ticket) {
    if (!sv || !op || !b || !c || !ticket) return fail(CGS_EINVAL, "null argument");
    CGS_TRY(cgs::validate_cone(op->m, l, q, nq));
    if (!all_finite(b, op->m) || !all_finite(c, op->n)) return fail(CGS_EINVAL, "b or c has a non-finite entry");
    if ((int64_t)sv->live.size() >= sv->max_slots) return fail(CGS_EBUSY, "no free slot");
    cgs::Engine& e = sv->eng;
    if (cgs::staging_doubles(*op, std::max(op->n, op->m)) > e.stg.cap)
        return fail(CGS_ENOMEM, "request too large for the server staging buffer");
    const size_t region = cgs::region_bytes(op->n, op->m, e.precision);
    const size_t bytes = region + cgs::align256(cgs::op_dev_bytes(*op, e.precision));
    size_t off = 0;
    if (!arena_alloc(sv, bytes, &off)) return fail(CGS_EBUSY, "not enough free device memory (%zu bytes)", bytes);
    std::unique_ptr<ServerReq> r(new ServerReq);
    r->ticket = sv->next_ticket++;
    r->off = off;
    r->bytes = bytes;
    r->n = op->n;
    r->m = op->m;
    r->l = l;
    r->q.assign(q, q + nq);
    r->t_submit = now_s();
    char* base = sv->arena + off;
    cgs::Scaling scl;
    cgs::compute_scaling(*op, l, q, nq, e.st.normalize, &scl);
    int rc = cgs::op_upload(*op, e.precision, base + region, e.stg, e.stream, &r->opdev, scl.blk.data());
    if (rc != CGS_OK) {
        arena_free(sv, off, bytes);
        return rc;
    }
    // the equilibrated b and c go straight into the region
    rc = upload_instance_data(e, scl, base, op->n, op->m, b, c);
    if (rc != CGS_OK) {
        arena_free(sv, off, bytes);
        return rc;
    }
    *ticket = r->ticket;
    sv->live.push_back(std::move(r));
    sv->dirty = true;
    return CGS_OK;
}

static int server_rebuild(cgs_server* sv) {
    cgs::Engine& e = sv->eng;
    std::vector<cgs::InstRec> recs;
    for (auto& r : sv->live) {
        cgs::InstRec rec;
        rec.base = sv->arena + r->off;
        rec.n = r->n;
        rec.m = r->m;
        rec.l = r->l;
        rec.q = r->q;
        rec.op = &r->opdev;
        recs.push_back(std::move(rec));
    }
    if (recs.empty()) {
        e.recs.clear();
        e.T = cgs::Tables{};
        sv->dirty = false;
        return CGS_OK;
    }
    CGS_TRY(e.build(recs));
    for (size_t i = 0; i < sv->live.size(); ++i) {
        sv->live[i]->eng_index = (int)i;
        if (sv->live[i]->fresh) {
            CGS_TRY(e.reset((int)i));
            sv->live[i]->fresh = false;
        }
    }
    sv->dirty = false;
    return CGS_OK;
}

static void server_collect(cgs_server* sv) {
    cgs::Engine& e = sv->eng;
    const double t = now_s();
    for (size_t i = 0; i < sv->live.size(); ++i) {
        ServerReq& r = *sv->live[i];
        if (r.finished) continue;
        const double* sc = e.scalars((int)i);
        if (sc[cgs::SC_ACTIVE] == 0.0) {
            r.finished = true;
            e.fill_info((int)i, &r.info);
            r.info.setup_s = 0.0;
            r.info.solve_s = t - r.t_submit;
        }
    }
}

int cgs_server_step(cgs_server* sv, int32_t steps, int64_t* n_running) {
    if (!sv) return fail(CGS_EINVAL, "server is null");
    if (steps < 0) return fail(CGS_EINVAL, "steps < 0");
    cgs::Engine& e = sv->eng;
    if (sv->dirty) CGS_TRY(server_rebuild(sv));
    if (!sv->live.empty()) {
        CGS_TRY(e.fetch_scalars());
        bool need_setup = false;
        for (size_t i = 0; i < sv->live.size(); ++i) {
            const double* sc = e.scalars((int)i);
            if (sc[cgs::SC_ACTIVE] != 0.0 && sc[cgs::SC_PHASE] == 0.0) need_setup = true;
        }
        if (need_setup) CGS_TRY(e.setup());
        e.refresh();
        const int rounds = (steps + e.st.check_every - 1) / e.st.check_every;
        for (int r = 0; r < rounds; ++r) {
            CGS_TRY(e.round(e.st.check_every));
            CGS_TRY(e.fetch_scalars());
            server_collect(sv);
            bool any = false;
            for (auto& q : sv->live) any = any || !q->finished;
            if (!any) break;
        }
    }
    if (n_running) {
        int64_t k = 0;
        for (auto& q : sv->live) k += q->finished ? 0 : 1;
        *n_running = k;
    }
    return CGS_OK;
}

static int find_req(cgs_server* sv, int64_t ticket) {
    for (size_t i = 0; i < sv->live.size(); ++i)
        if (sv->live[i]->ticket == ticket) return (int)i;
    return -1;
}

int cgs_server_poll(cgs_server* sv, int64_t ticket, int32_t* status) {
    if (!sv || !status) return fail(CGS_EINVAL, "null argument");
    const int i = find_req(sv, ticket);
    if (i < 0) return fail(CGS_ENOTFOUND, "ticket %lld", (long long)ticket);
    *status = sv->live[i]->finished ? sv->live[i]->info.status : CGS_RUNNING;
    return CGS_OK;
}

int cgs_server_finished(const cgs_server* sv, int64_t* tickets, int64_t cap, int64_t* count) {
    if (!sv || !count) return fail(CGS_EINVAL, "null argument");
    if (cap < 0 || (cap > 0 && !tickets)) return fail(CGS_EINVAL, "bad ticket buffer");
    int64_t k = 0;
    for (const auto& r : sv->live)
        if (r->finished) {
            if (k < cap) tickets[k] = r->ticket;
            ++k;
        }
    *count = k;
    return CGS_OK;
}

int cgs_server_fetch(cgs_server* sv, int64_t ticket, double* x, double* y, double* sl, cgs_info* info) {
    if (!sv) return fail(CGS_EINVAL, "server is null");
    const int i = find_req(sv, ticket);
    if (i < 0) return fail(CGS_ENOTFOUND, "ticket %lld", (long long)ticket);
    ServerReq& r = *sv->live[i];
    if (!r.finished || r.eng_index < 0) return fail(CGS_ESTATE, "ticket %lld is still running", (long long)ticket);
    cgs::Engine& e = sv->eng;
    const int ei = r.eng_index;   // finished requests keep their slot in the current tables
    double* outs[3] = {x, y, sl};
    const int64_t lens[3] = {r.n, r.m, r.m};
    for (int w = 0; w < 3; ++w) {
        if (!outs[w]) continue;
        for (int64_t off = 0; off < lens[w]; off += e.stg.cap) {
            const int64_t c = std::min(e.stg.cap, lens[w] - off);
            cgs::launch_extract(e.prec, e.inst_dev, ei, w, off, c, e.stg.dev, e.stream);
            CGS_HIP(hipGetLastError());
            CGS_HIP(hipMemcpyAsync(e.stg.host, e.stg.dev, c * sizeof(double), hipMemcpyDeviceToHost, e.stream));
            CGS_HIP(hipStreamSynchronize(e.stream));
            std::memcpy(outs[w] + off, e.stg.host, c * sizeof(double));
        }
    }
    if (info) *info = r.info;
    return cgs_server_cancel(sv, ticket);
}

int cgs_server_cancel(cgs_server* sv, int64_t ticket) {
    if (!sv) return fail(CGS_EINVAL, "server is null");
    const int i = find_req(sv, ticket);
    if (i < 0) return fail(CGS_ENOTFOUND, "ticket %lld", (long long)ticket);
    CGS_HIP(hipStreamSynchronize(sv->eng.stream));
    arena_free(sv, sv->live[i]->off, sv->live[i]->bytes);
    sv->live.erase(sv->live.begin() + i);
    sv->dirty = true;
    return CGS_OK;
}

int cgs_server_usage(const cgs_server* sv, int64_t* slots_used, size_t* bytes_free) {
    if (!sv) return fail(CGS_EINVAL, "server is null");
    if (slots_used) *slots_used = (int64_t)sv->live.size();
    if (bytes_free) {
        size_t f = 0;
        for (const auto& kv : sv->free_list) f += kv.second;
        *bytes_free = f;
    }
    return CGS_OK;
}

void cgs_server_destroy(cgs_server* sv) {
    if (sv) (void)hipStreamSynchronize(sv->eng.stream);
    delete sv;
}

}  // extern "C"
