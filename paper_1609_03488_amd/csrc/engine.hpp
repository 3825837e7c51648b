// Host side of the solver engine: operator descriptions, device layouts, tile
// tables and the orchestration of the ADMM iteration on a HIP stream.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "cgs.h"
#include "common.hpp"
#include "kernels.hpp"

namespace cgs {

// ---------------------------------------------------------------- errors
int fail(int code, const char* fmt, ...);
const char* last_error();

#define CGS_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::cgs::fail(CGS_EHIP, "%s failed: %s (%s:%d)", #call,                 \
                               hipGetErrorString(e_), __FILE__, __LINE__);              \
    } while (0)
#define CGS_TRY(expr)              \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ != CGS_OK) return rc_; \
    } while (0)

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
inline int work_prec(int precision) { return precision == CGS_FP64 ? 0 : 1; }
inline size_t elem_bytes(int precision) { return precision == CGS_FP64 ? 8 : 4; }

// ---------------------------------------------------------------- host operator
struct HostBlock {
    int kind;
    int64_t row0, col0, rows, cols;
    int64_t k, n_in;          // conv
    double scale;
    double frob2;             // sum of squares of the entries, scale excluded
    std::vector<double> data; // taps (k) or dense rows x cols (packed)
    // a dense block borrowed from device memory (data empty): rows x cols
    // entries of type dev_dtype, row stride dev_ld, on device dev_id
    const void* dev = nullptr;
    int dev_dtype = 0;
    int64_t dev_ld = 0;
    int dev_id = -1;
};

}  // namespace cgs

struct cgs_op {
    int64_t m, n;
    std::vector<cgs::HostBlock> blocks;
};

namespace cgs {

int validate_cone(int64_t m, int64_t l, const int64_t* q, int64_t nq);
// cgs_solver_create with the choice of host buffers: pageable = true keeps the
// solver's host-side staging in ordinary host memory (no HIP allocation call)
int solver_create(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq, const cgs_settings* st,
                  int64_t batch, void* workspace, size_t ws_bytes, void* stream, bool pageable,
                  cgs_solver** out);
int validate_settings(const cgs_settings* st);

// ---------------------------------------------------------------- staging
// FP64 transfers go through a pinned host buffer and a device buffer of `cap`
// doubles; conversion to the working precision happens on the device.
struct Staging {
    double* dev = nullptr;
    double* host = nullptr;
    int64_t cap = 0;
};
int64_t staging_doubles(const cgs_op& op, int64_t max_vec);

// ---------------------------------------------------------------- equilibration
// Diagonal scaling D (rows) and E (columns), constant on groups: the coarsest
// contiguous partitions in which every block and every second-order cone (rows)
// or every block (columns) lies inside one group.  Ruiz passes on the group
// matrix F[g][h] = sum of squared entries of the blocks in row group g and
// column group h; b and c are then scaled to the mean row / column norm.
struct Scaling {
    std::vector<int64_t> row_lo;   // group g: rows [row_lo[g], row_lo[g + 1])
    std::vector<double> d;
    std::vector<int64_t> col_lo;
    std::vector<double> e;
    std::vector<double> blk;       // D_g E_h of every operator block
    double mean_row = 1.0, mean_col = 1.0;
    bool on = false;
};
// level 0: none; 1: b and c only (D = E = I); 2: Ruiz passes on the blocks, then b and c
void compute_scaling(const cgs_op& op, int64_t l, const int64_t* q, int64_t nq, int level,
                     Scaling* out);
// Expanded D (m), E (n), b^ = sb D b, c^ = sc E c; returns {sb, sc}.
void scale_data(const Scaling& s, int64_t m, int64_t n, const double* b, const double* c,
                double* dv, double* ev, double* bh, double* ch, double* sb, double* sc);

// ---------------------------------------------------------------- device operator data
struct OpDev {
    std::vector<IdBlock> ids;
    std::vector<ConvBlock> convs;
    std::vector<DenseBlock> dense;
};
size_t op_dev_bytes(const cgs_op& op, int precision);
// Metadata only (null data pointers): used to size tables.  `mult` (nullable):
// per-block factor applied to the block's scale (the equilibration).
void op_dev_shape(const cgs_op& op, int precision, OpDev* out, const double* mult = nullptr);
int op_upload(const cgs_op& op, int precision, char* dst, const Staging& stg, hipStream_t st,
              OpDev* out, const double* mult = nullptr);
// Raw byte copy host -> device through the pinned staging buffer (synchronises).
int upload_raw(const Staging& stg, hipStream_t st, const void* src, size_t bytes, void* dst);

// Bytes of one instance's region (scalars, counters, X and Y vectors).
size_t region_bytes(int64_t n, int64_t m, int precision);
// copy of an instance's carried state (InstDesc::snap)
size_t snap_bytes(int64_t n, int64_t m, int precision);

int upload_f64(const Staging& stg, hipStream_t st, const double* src, int64_t n, int prec,
               void* dst);
int download_f64(const Staging& stg, hipStream_t st, int prec, const void* src, int64_t n,
                 double* dst);

// ---------------------------------------------------------------- instances and tables
struct InstRec {
    char* base = nullptr;
    int64_t n = 0, m = 0, l = 0;
    std::vector<int64_t> q;
    const OpDev* op = nullptr;
};

struct TableImage {
    std::vector<InstDesc> inst;
    std::vector<VecTile> xt, yt;
    std::vector<SocSeg> seg;
    std::vector<IdBlock> ids;
    std::vector<ConvBlock> cblk;
    std::vector<std::vector<ConvTile>> cfwd, cadj;   // per conv slot
    std::vector<std::vector<ConvTile>> ffwd, fadj;   // the same slots as FFT-engine tiles
    std::vector<DenseBlock> dblk;
    std::vector<std::vector<DenseTile>> dfwd, dadj;  // per dense slot
};
// vec_tile: elements per X/Y vector tile, VEC_TILE_MIN..VEC_TILE
void build_image(const std::vector<InstRec>& recs, int precision, TableImage& im, int vec_tile = VEC_TILE);
size_t image_table_bytes(const TableImage& im);
size_t image_work_bytes(const TableImage& im);
// dense entries above which an instance never takes the fused path (a dense
// product on one workgroup is 20-80x slower than spread over the chip)
constexpr int64_t FUSED_DENSE_MAX = 65536;

// ---------------------------------------------------------------- engine
class Engine {
  public:
    int precision = CGS_FP32;
    int prec = 1;                 // element type selector of the kernels
    cgs_settings st{};
    hipStream_t stream = nullptr;

    char* tab_dev = nullptr;  size_t tab_cap = 0;
    char* work_dev = nullptr; size_t work_cap = 0;
    char* tab_host = nullptr; size_t tab_host_cap = 0;   // pinned (pageable: host_store)
    double* scal_host = nullptr; int scal_host_cap = 0;   // pinned (pageable: host_store)
    Staging stg;
    // host buffers in ordinary (pageable) host memory instead of pinned memory,
    // for a solver that must not call any HIP allocation routine
    bool pageable = false;
    std::vector<double> host_store;

    std::vector<InstRec> recs;
    TableImage im;
    Tables T{};
    InstDesc* inst_dev = nullptr;
    double* gather_dev = nullptr;
    std::vector<ConvLaunch> cf, ca;
    int fold_init[2] = {0, 0};   // output initialisation rides on the first convolution launch
    // CG start and CG products folded into the FFT engine's A^T launch: when
    // that one launch writes every X element of every instance
    int fold_cg = 0;
    std::vector<DenseLaunch> df, da;
    int cg_launch = 1;
    // snapshot area for check intervals run with fewer CG launches per step
    // than the iteration limit (InstDesc::snap), and the last such interval:
    // its launches (0: the last round was not one), steps and the instances
    // that were iterating when it began
    char* snap_dev = nullptr; size_t snap_cap = 0;
    int snap_ok = 0;
    int spec_launch = 0, spec_nsteps = 0;
    std::vector<char> spec_live;
    int64_t n_rounds = 0, n_reruns = 0;
    // fused path: one workgroup per instance runs whole steps (instances with
    // n + m <= fused_max); the others take one launch per kernel
    int n_fused = 0, n_multi = 0;
    int lone = 0;                // a solver with a single instance (fused_lone_max applies)
    int fused_kc = 8;
    int64_t fused_res = 0;        // LDS bytes of the largest fused instance's resident vectors
    // batched BF16 MFMA path for dense blocks shared by every instance
    int use_gemm = 0;
    int gemm_corr = 0;           // 1: add the refinement products (hi x lo)
    uint16_t* panel = nullptr;   // three BF16 panels (hi, mid, lo) of panel_stride elements
    size_t panel_stride = 0;
    float* gemm_part = nullptr;
    int gemm_target = 256;       // GEMM workgroups aimed for (autotuned; 256 its usual choice)
    int vec_tile = VEC_TILE;     // elements per X/Y vector tile (autotuned)

    // side stream for the fused launch, overlapped with the one-launch-per-kernel
    // round of the other instances (disjoint memory); default priority
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    // instantiated check-interval graphs, by (steps, CG launches per step); the
    // launch count moves between a few values over a solve
    struct CachedGraph {
        int steps, cg, spec;
        hipGraph_t graph;
        hipGraphExec_t exec;
        int64_t used;
    };
    std::vector<CachedGraph> graphs;
    static constexpr size_t GRAPH_CACHE = 4;
    bool spec_now = false;        // the round being enqueued records a step that needs more CG launches
    int rounds_since_build = 0;   // a graph is captured only once the tables have held a round

    ~Engine();
    int init_host_buffers(size_t tab_bytes, int max_inst, int64_t stg_doubles);
    // Build and upload the tile tables of `recs`.
    int build(const std::vector<InstRec>& r);
    void drop_graph();

    // ---- device work (enqueue only)
    void apply(int adj, int out, int in, int base, double sigma, int gate);
    void conv(const ConvLaunch& c, int adj, int out, int in, int base, double sigma, int gate);
    // last = 1: the step's last CG launch (records a step that needed more);
    // start = 1: the first iteration of a step on the folded path (ungated
    // products, the update takes the CG start test)
    void cg_iter(int z, int gate, int cg_max, int track, int it, int last = 0, int start = 0);
    // CG steps run folded into the A^T launch (FFT engine chosen and the tables allow it)
    int idrows = 0;   // the right-hand side launch writes A p's identity rows (build)
    bool folded_cg() const { return fold_cg && prec == 1 && st.conv_mfma == 2 && !ca.empty() && ca[0].fft; }
    // relative floor of the ADMM steps' CG tolerance: cg_floor, and in FP64 at
    // most eps / 100 (subspace solves well below the target tolerance; FP32
    // CG cannot go much below its default 1e-6)
    double cg_floor() const { return precision == CGS_FP64 ? std::min(st.cg_floor, 1e-2 * st.eps) : st.cg_floor; }
    // relative tolerance of the embedding-vector solve: setup_tol, and in FP64
    // at most 1e-10 (in FP32 the vector g itself carries about 7 digits)
    double setup_tol() const { return precision == CGS_FP64 ? std::min(st.setup_tol, 1e-10) : st.setup_tol; }
    void admm_step();
    void fused_steps(int nsteps, int check);
    // steps of a round: intervals_per_sync check intervals
    int round_steps() const { return st.check_every * std::max(1, st.intervals_per_sync); }
    // nsteps ADMM steps with the termination test after every check_every of them
    void steps_with_checks(int nsteps);
    void check(int gate = G_CHECK);
    void apply_pair(int adj, int out1, int in1, int base1, int out2, int in2, int base2, double sigma,
                    int gate);
    void refresh();
    void adapt_cg();
    // ---- host loops
    int setup();                  // instances with phase 0 (synchronises)
    // nsteps ADMM steps, a termination test after every check_every of them and
    // at the end (enqueue); reads scal_host, so it
    // follows fetch_scalars.  multi_only: the one-launch-per-kernel instances only
    int round(int nsteps, bool multi_only = false);
    // after fetch_scalars: the last round ran fewer CG launches per step than
    // some step of an instance needed
    bool truncated() const;
    // restore the snapshot of that round and run it again with more launches
    int rollback();
    int fetch_scalars();          // gather per-instance scalars into scal_host (synchronises)
    const double* scalars(int i) const { return scal_host + (size_t)i * NSC; }
    int reset(int inst);          // inst < 0: all
    int set_scalar(int inst, int slot, double v);
    char* xptr(int inst, int kind) const;
    char* yptr(int inst, int kind) const;
    void fill_info(int i, cgs_info* info) const;
};

}  // namespace cgs
