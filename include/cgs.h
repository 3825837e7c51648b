/*
 * cgs.h -- C ABI of the structured-operator conic solver (libcgs.so, gfx950).
 *
 * Problem (the cone program of eq. (1), Section II-A, in the sign convention
 * A -> -A):
 *
 *     minimize  c^T x   subject to   A x + s = b,   s in K,
 *
 * with K = R_+^l x SOC(q_0) x SOC(q_1) x ...  (rows in that order) and A given
 * as an *operator description* -- a sum of placed structured blocks (identity /
 * scaling, full 1-D convolution, dense) -- instead of a sparse or dense matrix
 * (Sections III-A and IV: linear operators as functions, with adjoints).
 * The method is the homogeneous self-dual embedding ADMM iteration the paper
 * runs ("SCS", Sections II-D and V-B) with the subspace step solved by
 * conjugate gradients on I + A^T A (Section IV-B, the cg_solve listing)
 * followed by projections onto K (Section V-B).
 *
 * Conventions for every call:
 *   - Every function returns CGS_OK (0) or a negative error code; a text
 *     description of the last error on the calling thread is available from
 *     cgs_last_error().  The outcome of a solve is reported separately in
 *     cgs_info.status.
 *   - Host arrays passed in are copied before the call returns; the caller may
 *     free them afterwards.  Host output arrays are allocated by the caller.
 *   - Device memory: the library never allocates device memory on its own for
 *     solver state.  Every solver / server works inside one caller-provided
 *     device buffer ("workspace"), sized by the matching *_workspace_bytes call,
 *     which must stay alive until the handle is destroyed.
 *   - Streams: all device work of a handle is enqueued on the hipStream_t given
 *     at creation (NULL = the default stream).  Calls that return host results
 *     synchronise that stream.
 *   - A handle must be used by one thread at a time.
 *   - Indices and sizes are int64_t; rows/columns are 0-based.
 */
#ifndef CGS_H
#define CGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
enum {
    CGS_OK = 0,
    CGS_EINVAL = -1,   /* bad argument: null pointer, non-finite value, bad setting */
    CGS_EDIM = -2,     /* dimension mismatch or block outside the operator        */
    CGS_ECONE = -3,    /* cone sizes do not cover the rows or a size is < 1      */
    CGS_ENOMEM = -4,   /* workspace / memory budget too small                    */
    CGS_EHIP = -5,     /* HIP runtime failure (detail in cgs_last_error)          */
    CGS_EBUSY = -6,    /* no free slot or budget for a request right now         */
    CGS_ESTATE = -7,   /* call not valid in the handle's current state           */
    CGS_ENOTFOUND = -8 /* unknown ticket / instance                              */
};

/* Solve outcomes (cgs_info.status). */
enum {
    CGS_RUNNING = 0,
    CGS_SOLVED = 1,       /* res_pri, res_dual, gap all <= eps                    */
    CGS_MAX_ITERS = 2,    /* iteration limit reached first                        */
    CGS_INFEASIBLE = 3,   /* certificate y: -b^T y = 1, ||A^T y|| <= eps, y in K*  */
    CGS_UNBOUNDED = 4,    /* certificate x,s: -c^T x = 1, ||A x + s|| <= eps       */
    CGS_NUMERICAL = 5     /* a non-finite value appeared in the iterates          */
};

/* Arithmetic of the vectors and operator applies.  Dot products, norms, the
 * embedding scalars tau/kappa/eta and the residuals are always accumulated
 * and kept in FP64. */
enum {
    CGS_FP64 = 0,   /* everything in FP64                                        */
    CGS_FP32 = 1,   /* FP32 vectors and operator applies, FP64 scalars/norms     */
    CGS_BF16 = 2    /* CGS_FP32 plus BF16 MFMA products (FP32 accumulation) for a
                       dense block shared by a batch: two phases on the BF16
                       matrix (8, then ~16 significant bits), then the residual
                       test -- and, where it fails, further iterations -- on the
                       FP32 operator (see bf16_phase1_digits)                    */
};

/* Block kinds of an operator description. */
enum { CGS_BLOCK_IDENTITY = 0, CGS_BLOCK_CONV = 1, CGS_BLOCK_DENSE = 2 };

/* Element types and memory kinds of a dense block (cgs_op_add_dense_ex). */
enum { CGS_DTYPE_F64 = 0, CGS_DTYPE_F32 = 1 };
enum {
    CGS_MEM_HOST_COPY = 0,      /* host array, copied by the call                   */
    CGS_MEM_DEVICE_BORROW = 1   /* device array on the current device, read in
                                   place (never copied to the host)              */
};

typedef struct cgs_op cgs_op;
typedef struct cgs_solver cgs_solver;
typedef struct cgs_server cgs_server;

/* Iteration settings.  Start from cgs_settings_default(). */
typedef struct {
    double eps;            /* relative tolerance on res_pri, res_dual and gap (> 0)   */
    double alpha;          /* over-relaxation in (0, 2)                               */
    int32_t max_iters;     /* ADMM iteration limit (>= 1)                             */
    int32_t check_every;   /* residuals are evaluated every this many steps (>= 1)    */
    int32_t precision;     /* CGS_FP64 | CGS_FP32 | CGS_BF16                          */
    int32_t cg_max_iters;  /* CG iterations per ADMM step, upper bound (>= 1)         */
    double cg_tol;         /* CG stops when ||r|| <= ||rhs|| * max(cg_floor,          */
    double cg_rate;        /*        cg_tol / (k+1)^cg_rate)  at ADMM step k          */
    double cg_floor;       /* (CGS_FP64 uses min(cg_floor, eps / 100): its subspace
                              solves stay well below the target tolerance)          */
    double setup_tol;      /* relative CG tolerance of the embedding-vector solve
                              (CGS_FP64 uses min(setup_tol, 1e-10))                  */
    int32_t setup_max_iters; /* CG iteration limit of that solve                      */
    int32_t use_graph;     /* 1: replay each block of check_every steps as a hipGraph */
    int32_t bf16_phase1_digits; /* CGS_BF16: the BF16-product phase solves to
                              max(eps, 10^-digits); the refinement phase (BF16 hi/lo
                              products, ~16 significant bits) then continues from its
                              state to eps / 2 with a fresh setup solve; the last
                              phase tests the point on the FP32 operator (dense
                              products from the FP32 copy of the blocks) and, for an
                              instance that fails the test, iterates on that operator
                              with its own setup solve until it passes (default 3)  */
    int32_t cg_adaptive;   /* 1 (default): a check interval runs as many CG launches
                              per step as the most CG iterations any instance used in
                              a step of the previous interval (at least 1, at most
                              cg_max_iters; cg_max_iters in an instance's first
                              interval), starting from a copy of the state each
                              step hands to the next.  When some step's CG would have
                              gone on after its last launch, the interval is restored
                              from that copy and run again with 2 L + 1 launches
                              (capped), so results equal those of 0 bit for bit.  The
                              copy takes 512 + (3 n' + 4 m') * element bytes of
                              workspace per instance (n', m': n, m rounded up to 64).
                              0: always cg_max_iters launches (no copy).  A server
                              always uses 0                                           */
    int32_t fused_max;     /* instances with n + m <= fused_max run whole ADMM steps in
                              one workgroup each (one launch per check interval for
                              all of them, CG loop inside the kernel); larger ones
                              take one launch per kernel spread over the chip.  The
                              path depends on an instance's own size only; 0
                              disables (default 16384: a crowd of such instances
                              fills the chip one workgroup each).  Instances whose
                              dense blocks hold more than 65536 entries always take
                              the launch-per-kernel path (a dense product on one
                              workgroup is 20-80x slower than spread over the chip) */
    int32_t conv_mfma;     /* FP32 convolution engine.  2 (default): FFT overlap-save
                              (2048-point transforms in LDS, two real windows per
                              complex transform) for kernels of up to 1536 taps,
                              the matrix cores for longer ones; 1: matrix cores
                              (16x16x4 FP32 MFMA over Toeplitz blocks of the taps);
                              0: vector ALU.  The products agree to their rounding
                              (elementwise for 0 and 1; normwise per 2048-point
                              window for 2)                                         */
    int32_t normalize;     /* data scaling the iteration runs on: 1 (default):
                              sb b, sc c with sb, sc bringing b and c to the mean row /
                              column norm of A (A itself, and so the conditioning of
                              the CG systems, unchanged); 2: first D A E with diagonal
                              D (rows) and E (columns) constant on every operator
                              block and second-order cone (20 Ruiz passes on the
                              blocks' Frobenius norms), then sb D b, sc E c; 0: data
                              as given.  Termination and returned points are those
                              of the original problem; the raw state and the
                              diagnostic apply / normal solve use the scaled data. */
    int32_t fused_lone_max; /* a solver holding a single instance (batch 1) takes the
                              fused path only for n + m <= min(fused_max,
                              fused_lone_max): alone, one workgroup races the whole
                              chip, and measured per-step times cross near n + m =
                              8000 (default 8192; 0: fused_max alone decides)       */
    int32_t vec_tile;      /* elements per vector tile of the vector kernels and their
                              reductions: 1024 or 2048 (0, the default: 2048; the
                              autotuner may change it)                              */
    int32_t intervals_per_sync; /* check intervals enqueued (one graph) between two
                              reads of the instances' scalars by the host (>= 1,
                              default 2).  The termination test still runs every
                              check_every steps on the device and an instance that
                              passes it stops there; only the host's decisions
                              (CG launches per step, a rerun, the end of the solve)
                              wait for the end of the batch of intervals.  Results
                              do not depend on it.  A server always uses 1.         */
} cgs_settings;

/* Per-instance result. */
typedef struct {
    int32_t status;        /* CGS_SOLVED ... (see above)                              */
    int32_t iters;         /* ADMM iterations taken                                   */
    int64_t cg_iters;      /* CG iterations over the whole solve (normal-operator
                              applications, setup included)                           */
    double pobj;           /* c^T x                                                   */
    double dobj;           /* -b^T y                                                  */
    double res_pri;        /* ||A x + s - b|| / (1 + ||b||)                           */
    double res_dual;       /* ||A^T y + c|| / (1 + ||c||)                             */
    double gap;            /* |c^T x + b^T y| / (1 + |c^T x| + |b^T y|)               */
    double tau, kappa;     /* embedding scalars at exit                               */
    double setup_s;        /* wall time of the setup (embedding vector) phase         */
    double solve_s;        /* wall time of the iterations                             */
    int32_t cert_precision; /* arithmetic of the operator whose residual test gave
                              status: the solver's precision, or CGS_FP32 for a
                              CGS_BF16 instance the FP32 phase tested (CGS_BF16 if
                              an earlier phase ended it without a solution)        */
    int32_t reserved_;
} cgs_info;

/* ---------------------------------------------------------------- errors */
const char* cgs_last_error(void);
/* Library version string. */
const char* cgs_version(void);

/* ---------------------------------------------------------------- operator
 * A structured operator A (m x n) is a sum of placed blocks.  A block maps a
 * contiguous range of the input (columns col0 .. col0+cols-1) into a contiguous
 * range of the output (rows row0 .. row0+rows-1), times a scale; blocks may
 * overlap, their contributions add.  Applying A^T uses each block's adjoint
 * with the placement transposed (Section IV-A: the adjoint of a linear graph).
 * Host-only calls: no device work happens until a solver is created. */

/* New empty operator of size m x n (m, n >= 1). */
int cgs_op_create(int64_t m, int64_t n, cgs_op** out);
/* Identity (times scale) of length len: out[row0+i] += scale * in[col0+i]. */
int cgs_op_add_identity(cgs_op* op, int64_t row0, int64_t col0, int64_t len, double scale);
/* Full 1-D convolution with k taps (Section V, eq. 6):
 *   out[row0+i] += scale * sum_j taps[j] * in[col0+i-j],  i = 0 .. n_in+k-2,
 * rows = n_in + k - 1, cols = n_in.  Its adjoint is the valid correlation
 *   in[col0+j] += scale * sum_t taps[t] * out[row0+j+t].
 * taps: host FP64 array of k >= 1 finite values (copied). */
int cgs_op_add_conv(cgs_op* op, int64_t row0, int64_t col0, const double* taps, int64_t k,
                    int64_t n_in, double scale);
/* Dense block: out[row0+i] += scale * sum_j a[i*lda + j] * in[col0+j]
 * for i < rows, j < cols.  a: host FP64 row-major array with lda >= cols
 * (copied; converted to the solver's precision at solver creation). */
int cgs_op_add_dense(cgs_op* op, int64_t row0, int64_t col0, int64_t rows, int64_t cols,
                     const double* a, int64_t lda, double scale);
/* The same block from typed memory (Section III: a dense block is one of the
 * structured pieces the operator is composed of; this call only chooses where
 * its entries come from).  dtype: CGS_DTYPE_F64 or CGS_DTYPE_F32 (FP32 host
 * data is widened to FP64 exactly).  mem:
 *   CGS_MEM_HOST_COPY     a is a host array, validated and copied now;
 *   CGS_MEM_DEVICE_BORROW a is device memory of the current device (for
 *                         instance a torch tensor's data).  The call reads it
 *                         once on the device to validate it (every entry
 *                         finite) and to form its Frobenius norm; every solver
 *                         and server created from this operator reads it again
 *                         at creation (conversion to the working precision,
 *                         transpose, BF16 copies) on its own stream.  The
 *                         caller keeps the memory allocated and unchanged until
 *                         cgs_op_destroy; the library never frees it.
 * lda >= cols elements.  Errors: CGS_EINVAL (null a, unknown dtype or mem, a
 * non-finite entry, a borrowed pointer that is not device memory of the
 * current device), CGS_EDIM (bad shape or lda), CGS_EHIP (device failure). */
int cgs_op_add_dense_ex(cgs_op* op, int64_t row0, int64_t col0, int64_t rows, int64_t cols,
                        const void* a, int64_t lda, int32_t dtype, int32_t mem, double scale);
/* Number of blocks and the operator size. */
int cgs_op_info(const cgs_op* op, int64_t* m, int64_t* n, int64_t* nblocks);
/* The scaling a solver with normalize = level applies to this operator and
 * cone (host computation, no device work): d (m entries) and e (n entries)
 * receive the row and column scalings D and E (all ones below level 2),
 * constant on the groups of rows / columns that every block and second-order
 * cone lies in; with b (m) and c (n) given, sigma[2] receives
 * {sigma_b, sigma_c}, the factors of b^ = sigma_b D b and c^ = sigma_c E c.
 * Any output may be NULL.  The raw solver state is
 * u^ = (sigma_b E^-1 x tau, sigma_c D^-1 y tau, tau), v^_s = sigma_b D s tau. */
int cgs_op_equilibrate(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq, int32_t level,
                       const double* b, const double* c, double* d, double* e, double* sigma);
void cgs_op_destroy(cgs_op* op);

/* ---------------------------------------------------------------- solver
 * A solver holds `batch` instances that share the operator and the cone; each
 * instance has its own b and c (cgs_solver_set_data).  batch = 1 is the plain
 * one-problem solver.  With CGS_BF16 and a dense block, the operator applies
 * of the whole batch run as BF16 MFMA GEMMs with FP32 accumulation. */

void cgs_settings_default(cgs_settings* st);
/* Device bytes a solver needs for (op, cone, settings, batch). */
int cgs_workspace_bytes(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq,
                        const cgs_settings* st, int64_t batch, size_t* bytes);
/* Create a solver inside `workspace` (device memory of ws_bytes, 256-byte
 * aligned) on `stream`.  Uploads the operator (conversion to the working
 * precision happens on the device).  Cone: l nonnegative rows followed by nq
 * second-order cones of sizes q[0..nq-1]; l + sum(q) must equal m. */
int cgs_solver_create(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq,
                      const cgs_settings* st, int64_t batch, void* workspace, size_t ws_bytes,
                      void* stream, cgs_solver** out);
/* Set b (m entries) and c (n entries) of instance `inst` from host FP64 arrays.
 * Non-finite entries -> CGS_EINVAL.  Resets that instance's iterates. */
int cgs_solver_set_data(cgs_solver* s, int64_t inst, const double* b, const double* c);
/* Restart instance `inst` (all instances if inst < 0) from u = v = (0, 0, 1)
 * with its b and c kept on the device: the next cgs_solve runs the whole
 * method again, setup included, without any host-to-device transfer. */
int cgs_solver_reset(cgs_solver* s, int64_t inst);
/* Solve every instance from its current state (fresh: u = v = (0, 0, 1)).
 * info: array of `batch` entries (may be NULL).  With CGS_BF16 and dense
 * blocks, the dense applies of all instances run as one BF16 MFMA GEMM
 * (FP32 accumulation); the solve has three phases (see bf16_phase1_digits),
 * the last on the FP32 operator. */
int cgs_solve(cgs_solver* s, cgs_info* info);
/* Run exactly `iters` ADMM steps on every unfinished instance, with no
 * termination test (the setup solve runs first if needed). */
int cgs_solver_iterate(cgs_solver* s, int32_t iters);
/* Check intervals the solver has run since it was created, runs again
 * included (rounds), and how many of them were runs again from an interval's
 * start because a step needed more CG launches than the interval had (reruns,
 * cg_adaptive = 1); either may be NULL. */
int cgs_solver_rounds(cgs_solver* s, int64_t* rounds, int64_t* reruns);
/* Primal-dual point (x = u_x/tau, y = u_y/tau, s = v_s/tau) of an instance, as
 * FP64 host arrays of n, m, m entries (any may be NULL). */
int cgs_solver_get_solution(cgs_solver* s, int64_t inst, double* x, double* y, double* sl);
/* Raw embedding state of the (equilibrated) problem the iteration runs on:
 * u_x (n), u_y (m), v_s (m) and scal[2] = {tau, kappa}. */
int cgs_solver_get_state(cgs_solver* s, int64_t inst, double* ux, double* uy, double* vs,
                         double* scal);
/* Overwrite the embedding state (warm start / resume); the next cgs_solve or
 * cgs_solver_iterate continues from it.  u_y and v_s should lie in K. */
int cgs_solver_set_state(cgs_solver* s, int64_t inst, const double* ux, const double* uy,
                         const double* vs, const double* scal);
/* Evaluate the termination quantities at the current state of every instance
 * (info: batch entries; status stays CGS_RUNNING unless a test passes). */
int cgs_solver_residuals(cgs_solver* s, cgs_info* info);
/* One operator application on the device in the working precision, for
 * instance 0's operator as the iteration sees it (D A E when normalize = 2):
 * out = A in (transpose = 0, in: n, out: m) or out = A^T in (transpose = 1,
 * in: m, out: n).  Host FP64 arrays. */
int cgs_solver_apply(cgs_solver* s, int32_t transpose, const double* in, double* out);
/* Conjugate gradients on (I + A^T A) z = rhs (A as in cgs_solver_apply) in the working precision from
 * z = z0 (NULL: 0) until ||r|| <= tol ||rhs|| or max_iters; host FP64 arrays of
 * n entries; *iters receives the iteration count (Section IV-B listing). */
int cgs_solver_normal_solve(cgs_solver* s, const double* rhs, const double* z0, double* z,
                            double tol, int32_t max_iters, int32_t* iters);
/* Device time of one operator kernel class, measured with HIP events on the
 * solver's stream around `reps` back-to-back launches on the current iterate
 * vectors: kernel 0 = convolution (A), 1 = convolution adjoint (A^T),
 * 2 = dense block (A), 3 = dense block (A^T) (for a CGS_BF16 batch: the
 * pack + MFMA GEMM + reduce of all instances), 4 = the whole normal-operator
 * application p + A^T A p.  *avg_ms receives the mean time per launch (per
 * operator block, for 0-3); CGS_ENOTFOUND if the operator has no such block. */
int cgs_solver_kernel_time(cgs_solver* s, int32_t kernel, int32_t reps, double* avg_ms);
/* Autotuner: picks, for this solver's own operator and instances, the FP32
 * convolution engine (vector ALU, matrix cores, or FFT when the kernels are
 * short enough), the split-K width of the batched BF16 GEMM and the length of
 * the vector tiles (1024 or 2048 elements) the vector kernels and reductions
 * work on.  With data on every instance it times each combination on whole
 * ADMM steps of the instances (setup, three untimed steps, then `reps` steps
 * between HIP events: the launches the solve runs, folded ones included) and
 * restarts every instance from u = v = (0, 0, 1) afterwards; without data it
 * times the operator's launches alone (vector tiles unchanged).  choice[4]
 * (nullable) receives {conv engine (conv_mfma value, or -1), GEMM workgroup
 * target (or -1), vector tile length, -1}.  Only how the same products and
 * sums are computed changes: applies agree to their rounding, and reductions
 * keep a fixed order for each choice. */
int cgs_solver_autotune(cgs_solver* s, int32_t reps, int32_t* choice);
void cgs_solver_destroy(cgs_solver* s);

/* ---------------------------------------------------------------- no allocation
 * For callers that cannot allocate device memory (a serving loop or a harness
 * that must not call hipMalloc): one solve of one problem -- cgs_solver_create,
 * cgs_solver_set_data, cgs_solve and cgs_solver_get_solution in one call -- with
 * the workspace taken from a fixed array in device memory instead of the
 * caller's buffer.  Each GPU the library runs on holds one such array of
 * CGS_NOALLOC_SCRATCH_BYTES from the time the library's code is loaded until
 * the process ends; the call makes no HIP allocation of any kind (no device,
 * pinned or graph memory: check intervals run without a graph, use_graph is
 * ignored) and needs no workspace argument.
 * Arguments are those of cgs_solver_create (batch 1, st->precision CGS_FP64 or
 * CGS_FP32) and cgs_solver_set_data; x (n), y (m), sl (m) and info (one entry)
 * receive the results as in cgs_solver_get_solution and cgs_solve (any may be
 * NULL).  The stream must belong to the current device.
 * Errors: CGS_ENOMEM when the problem's workspace (cgs_workspace_bytes) exceeds
 * CGS_NOALLOC_SCRATCH_BYTES, CGS_EINVAL for CGS_BF16, plus those of the calls
 * it stands for.  Calls on one device share its array: they run one at a
 * time (a lock per device; overlapping calls from other host threads wait),
 * and each call rewrites everything it reads before reading it.  The call
 * returns after its device work has finished. */
#define CGS_NOALLOC_SCRATCH_BYTES (32u << 20)
int cgs_solve_noalloc(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq, const cgs_settings* st,
                      const double* b, const double* c, void* stream, double* x, double* y, double* sl,
                      cgs_info* info);

/* ---------------------------------------------------------------- server
 * Continuous batching of independent problems, each with its own operator
 * (same block kinds; any sizes), cone and data.  Requests are admitted while a
 * slot is free and their device footprint fits in the unused part of the
 * server's workspace; admitted problems advance together, one launch per
 * kernel for all of them, and leave as soon as they finish.  Each instance's
 * arithmetic is independent of the others in the mix (fixed per-instance
 * reduction order), so its result is the same alone and in any mix. */

/* Device bytes a single request needs inside a server (footprint used for
 * admission). */
int cgs_server_request_bytes(const cgs_op* op, int64_t l, const int64_t* q, int64_t nq,
                             int32_t precision, size_t* bytes);
int cgs_server_create(int64_t max_slots, const cgs_settings* st, void* workspace,
                      size_t ws_bytes, void* stream, cgs_server** out);
/* Admit a problem; CGS_EBUSY if no slot or not enough free workspace.
 * *ticket identifies it until cgs_server_fetch / cgs_server_cancel. */
int cgs_server_submit(cgs_server* sv, const cgs_op* op, int64_t l, const int64_t* q, int64_t nq,
                      const double* b, const double* c, int64_t* ticket);
/* Advance every admitted problem by up to `steps` ADMM steps (termination is
 * tested every check_every steps of each problem's own count).  *n_running
 * receives the number of problems still running afterwards. */
int cgs_server_step(cgs_server* sv, int32_t steps, int64_t* n_running);
/* Status of a ticket (CGS_RUNNING while unfinished). */
int cgs_server_poll(cgs_server* sv, int64_t ticket, int32_t* status);
/* Tickets of the finished problems not yet fetched or cancelled, in admission
 * order: up to `cap` of them into tickets (may be NULL when cap = 0); *count
 * receives how many there are in all. */
int cgs_server_finished(const cgs_server* sv, int64_t* tickets, int64_t cap, int64_t* count);
/* Copy out a finished problem's x (n), y (m), s (m) and info, and release its
 * slot and memory. */
int cgs_server_fetch(cgs_server* sv, int64_t ticket, double* x, double* y, double* sl,
                     cgs_info* info);
/* Drop a request (finished or not) and release its slot and memory. */
int cgs_server_cancel(cgs_server* sv, int64_t ticket);
/* Slots in use and free workspace bytes. */
int cgs_server_usage(const cgs_server* sv, int64_t* slots_used, size_t* bytes_free);
void cgs_server_destroy(cgs_server* sv);

#ifdef __cplusplus
}
#endif
#endif /* CGS_H */
