// Shared host/device definitions of the solver engine.
//
// An *engine* advances a set of problem instances together.  Every instance
// owns one contiguous region of device memory:
//
//   [ scalars: NSC doubles | counters: NCNT ints | X vectors (NXV x nxs) | Y vectors (NYV x nys) ]
//
// X vectors have the length n of the variable, Y vectors the length m of the
// constraint rows; nxs / nys are those lengths rounded up to XY_ALIGN elements.
// The iteration runs on the equilibrated data (D A E, sb D b, sc E c); the
// termination test and the returned points are those of the original problem.
// Kernels walk *tile tables*: every tile lies inside one instance, so a single
// launch covers all instances, and the per-instance arithmetic (including the
// fixed-order reductions) does not depend on which other instances are in it.
#pragma once
#include <cstdint>

namespace cgs {

// ---------------------------------------------------------------- vectors
// X-space vectors (length n)
enum XVec : int {
    XU = 0,   // u_x
    XG,       // g_x  (embedding vector, x part)
    XC,       // c
    XZ,       // CG iterate: z_x = (I + A^T A)^{-1} (u_x - A^T w_y); warm start
    XR,       // CG residual
    XP,       // CG direction
    XQ,       // (I + A^T A) p
    XH,       // CG right-hand side
    XT,       // scratch (A^T y for residuals / diagnostics)
    XK,       // (I + A^T A) z, carried through the CG updates
    XE,       // column scaling E of the equilibrated operator D A E
    NXV
};
// Y-space vectors (length m)
enum YVec : int {
    YU = 0,   // u_y
    YV,       // v_s (the y-block of v)
    YG,       // g_y
    YB,       // b
    YW,       // w_y = u_y + v_s
    YZ,       // z_y = w_y + A z_x (stored by the fused kernel only; the other
              // kernels form it from u_y, v_s and A z where they need it)
    YT,       // scratch (A p, A u_x)
    YA,       // A z, carried through the CG updates
    YD,       // row scaling D of the equilibrated operator D A E
    NYV
};

// ---------------------------------------------------------------- scalars
// per-instance FP64 scalars
enum Scal : int {
    SC_TAU = 0, SC_KAPPA, SC_ETA, SC_UT,        // tau, kappa, eta, u~_tau
    SC_RR, SC_PQ, SC_ALPHA, SC_BETA,           // CG: ||r||^2, <p,q>, alpha, beta
    SC_CGTOL, SC_HN,                           // CG stop threshold on ||r||, ||rhs||
    SC_NB, SC_NC,                              // ||b||, ||c||
    SC_CX, SC_BY,                              // c^T x, b^T y at the last check
    SC_RP, SC_RD, SC_GAP,                      // residuals at the last check
    SC_ACTIVE,                                 // 1 while the instance runs
    SC_PHASE,                                  // 0: setup pending, 1: iterating (one launch
                                               // per kernel), 2: iterating (fused steps),
                                               // 3: suspended (a step needed more CG
                                               // launches than its round had)
    SC_CGACT,                                  // 1 while CG of the instance runs
    SC_CGIT,                                   // CG iterations in the current solve
    SC_CGTOT,                                  // CG iterations since set_data
    SC_ITER,                                   // ADMM iterations done
    SC_STATUS,                                 // CGS_* outcome
    SC_SETUPIT,                                // CG iterations of the setup solve
    SC_CUX, SC_BUY,                            // raw c^T u_x, b^T u_y at the last check
    SC_CGMAX,                                  // most CG iterations of a step since the last check
    SC_CGMAXLAST,                              // ... over the previous check interval
    SC_SB, SC_SC,                              // data scales: b^ = sb D b, c^ = sc E c
    SC_CGRUN,                                  // CG iteration whose products are in place
                                               // (set by the dot kernel, -1 at CG start)
    NSC_USED
};
constexpr int NSC = 32;      // doubles reserved per instance (256 bytes)
static_assert(NSC_USED <= NSC, "scalar slots");
constexpr int NCNT = 64;     // int counters reserved per instance (256 bytes)
constexpr int XY_ALIGN = 64; // elements
constexpr int REGION_HDR = NSC * 8 + NCNT * 4;  // 512 bytes
// vectors of that copy: u_x, z, K z and u_y, v_s, w_y, A z (every other vector
// is either constant during the iteration or written before it is read in a step)
constexpr int SNAP_X = 2;   // u_x, z (the CG warm start)
constexpr int SNAP_Y = 2;   // u_y, v_s

// ---------------------------------------------------------------- gates
enum Gate : int {
    G_ALL = 0,        // every instance
    G_SETUP = 1,      // active and setup pending
    G_SETUP_CG = 2,   // ... and CG running
    G_ADMM = 3,       // active and iterating
    G_ADMM_CG = 4,    // ... and CG running
    G_CHECK = 5,      // active and iterating (termination test)
    G_ANY_CG = 6,     // CG running, whatever the phase (diagnostic solves)
    G_CHECK_ANY = 7   // active and iterating on either path (diagnostic residuals)
};

// ---------------------------------------------------------------- tables
struct InstDesc {
    char* base;          // region base (device address)
    int64_t n, m;        // variables, constraint rows
    int64_t nxs, nys;    // padded vector strides (elements)
    int64_t l;           // nonnegative rows
    int32_t xt0, xt1;    // X-tile range
    int32_t yt0, yt1;    // Y-tile range
    int32_t sg0, sg1;    // SOC segment range
    int32_t id0, id1;    // identity-block range
    int32_t cb0, cb1;    // convolution-block range (Tables::cblk)
    int32_t db0, db1;    // dense-block range (Tables::dblk)
    int32_t fused;       // 1: whole ADMM steps run in one workgroup (k_fused)
    int32_t pad_;
    // partials of CG steps folded into the A^T convolution launch (Tables::cpart
    // and Tables::spart indices): the instance's transform workgroups [cp0, cp1) and
    // initialisation workgroups [ip0, ip1) of that launch
    int32_t cp0, cp1, ip0, ip1;
    // copy of the state carried from one ADMM step to the next, taken at the
    // start of a check interval run with fewer CG launches per step than the
    // iteration limit (null: none): [header | SNAP_X vectors of nxs | SNAP_Y of nys].
    // The rest of the carried state (w_y = u_y + v_s, A z and (I + A^T A) z)
    // is a function of these, formed exactly by the check that precedes every
    // such interval, and is formed again the same way on a restore.
    char* snap;
};

// A tile of an X or Y vector: `len` elements from instance-local `start`.
// seg >= 0: the rows belong to second-order cone `seg` (Y tiles only).
struct VecTile {
    int32_t inst;
    int32_t seg;
    int64_t start;
    int32_t len;
    int32_t pad;
};

struct SocSeg {
    int32_t inst;
    int32_t ntiles;      // Y tiles covering the segment
    int32_t yt0;         // first of those tiles
    int32_t pad;
    int64_t start;       // instance-local row of the cone's first entry (t)
    int64_t len;
};

struct IdBlock {         // out[row0+i] += scale * in[col0+i], i < len
    int64_t row0, col0, len;
    double scale;
};

struct ConvBlock {       // full convolution of n_in inputs with k taps
    int64_t row0, col0, n_in, k, kpad;
    const void* w_fwd;   // taps reversed (correlation order for A x), kpad entries
    const void* w_adj;   // taps in order (correlation order for A^T y), kpad entries
    // conj(DFT) of w_fwd / w_adj zero-padded to FFT_L points (float2), for the
    // FFT engine (FP32 working precision and k <= FFT_KMAX), else null
    const void* s_fwd;
    const void* s_adj;
    double scale;
    // bit 0 (A x) / bit 1 (A^T y): no other convolution or dense block writes
    // into this block's output range, so the convolution writes the final
    // value there (base + identity blocks + its own sum) and the separate
    // initialisation pass skips the range
    int32_t own;
    int32_t pad_;
};

struct ConvTile {        // CONV_TILE outputs starting at block-local `start`
    int32_t inst;
    int32_t blk;
    int64_t start;
};

struct DenseBlock {      // rows x cols block
    int64_t row0, col0, rows, cols;
    int64_t ld, ldt;     // leading dimensions of a (rows x ld) and at (cols x ldt)
    const void* a;       // working precision, row-major
    const void* at;      // its transpose, row-major
    const void* a16;     // BF16 (round to nearest even) copies in the GEMM's packed
                         // operand layout (rows padded to 32), CGS_BF16 only, or null
    const void* at16;
    const void* a16lo;   // BF16 rounding of the remainder a - a16 (refinement products)
    const void* at16lo;
    double scale;
};

struct DenseTile {       // `nr` rows of the (possibly transposed) block from r0
    int32_t inst;
    int32_t blk;
    int64_t r0;
    int32_t nr;
    int32_t pad;
};

struct Tables {
    const InstDesc* inst;
    const VecTile* xt;
    const VecTile* yt;
    const SocSeg* seg;
    double* seg_val;     // 2 per segment: head value, tail sum of squares
    int* seg_cnt;        // 1 per segment
    const IdBlock* ids;
    const struct ConvBlock* cblk;
    const struct DenseBlock* dblk;
    double* xpart;       // 4 per X tile
    double* ypart;       // 4 per Y tile
    double* cpart;       // 4 per workgroup of the A^T convolution launch (folded CG products)
    double* spart;       // the same for the right-hand side's A^T launch (folded CG start)
    // slot-major partials of the update that ends CG for the projection that
    // follows (CgStart::cone): tpart[j * (nx_tiles + ny_tiles) + b] for the
    // workgroup b of an X-then-Y tile launch, slots 0 (tau products) to 3
    double* tpart;
    int nx_tiles, ny_tiles, nseg, ninst;
};

constexpr int VEC_TILE = 2048;     // most elements per X/Y tile (the kernels' per-thread share)
constexpr int VEC_TILE_MIN = 1024; // smallest tile length the autotuner tries (sizes the tables)
constexpr int VEC_NT = 256;        // threads per vector-kernel block
constexpr int CONV_TILE_F32 = 512;   // outputs per convolution tile (64 lanes x 8)
constexpr int CONV_TILE_F64 = 256;   // (64 lanes x 4)
constexpr int CONV_KC_MAX_F32 = 2048;  // taps staged per pass (LDS: (512 + 2*2048 + 16) * 4 B)
constexpr int CONV_KC_MAX_F64 = 1024;
constexpr int CONV_R_F32 = 8;        // taps are padded to a multiple of this
constexpr int CONV_R_F64 = 4;
constexpr int DENSE_ROWS = 4;        // rows per dense-GEMV tile
constexpr int FFT_L = 2048;          // points per transform of the FFT convolution engine
constexpr int FFT_KMAX = 1536;       // longest kernel it takes (>= 513 outputs per window)

}  // namespace cgs
