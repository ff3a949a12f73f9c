// Internal definitions shared by the planner (host) and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qgt {

constexpr int kTile = 64;          // Cholesky tile (complex entries)
constexpr int kGramTile = 128;     // Gram output tile; matrices are padded to a multiple of it
constexpr int kMaxProblems = 64;   // problems batched in one plan
constexpr int kPackRowsS = 8;      // sample-form pack: 64-row strips per workgroup

enum Prec : int32_t { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16 = 2 };
enum Form : int32_t { FORM_P = 1, FORM_S = 2 };

// k-group length of the packed Gram operand: the contraction index k is stored
// in groups of G consecutive values per output column, G * element size = 16
// bytes, so that one lane reads its MFMA inputs for a group with one 16-byte
// load.
__host__ __device__ constexpr int pack_group(int prec) { return prec == PREC_FP64 ? 2 : (prec == PREC_FP32 ? 4 : 8); }
// k-extent of one LDS stage of the Gram kernel: four k-groups.
__host__ __device__ constexpr int gram_stage_k(int prec) { return 4 * pack_group(prec); }
__host__ __device__ constexpr int prec_bytes(int prec) { return prec == PREC_FP64 ? 8 : (prec == PREC_FP32 ? 4 : 2); }
// The stored block matrix (the shifted Gram, then its Cholesky factor) and the
// inverses of the factor's diagonal tiles are complex FP64 by default.  A plan
// may ask for complex FP32 storage and an FP32 factorisation on blocks whose
// Gram is accumulated in BF16 (BlockDev::fact32): such a Gram is itself only
// good to about 1e-3 relative, far above what an FP32 factorisation adds, and
// the FP64 CG iteration on the exact operator removes both.
__host__ __device__ constexpr int factor_bytes(bool fp32) { return fp32 ? 8 : 16; }

// One layer block of one problem.  All *_off are byte offsets into the
// caller's workspace.
struct BlockDev {
  int32_t prob;      // problem index
  int32_t form;      // FORM_P or FORM_S
  int32_t prec;      // Gram precision
  int32_t ntiles;    // m_pad / kTile
  int32_t fact32;    // 1: the matrix is stored and factored in complex FP32, 0: complex FP64
  int32_t chunk;     // panels per trailing-update task of the Cholesky (tile DAG)
  int32_t tile_state;  // first entry of the block's tile counters in the Cholesky state array
  int32_t pad0;
  int64_t col_off;   // first column of the block in O (and in delta)
  int64_t n_b;       // block size
  int64_t m;         // matrix order: n_b (P) or n_s (S)
  int64_t m_pad;     // m rounded up to kTile
  int64_t K;         // contraction length: n_s (P) or n_b (S)
  int64_t K_pad;     // K rounded up to the Gram stage
  int64_t pack_off;  // packed operand: Re plane then Im plane, K_pad x m_pad each
  int64_t mat_off;   // shifted Gram / Cholesky factor: m_pad x m_pad complex (fact32 ? FP32 : FP64) row-major
  int64_t linv_off;  // inverses of the diagonal Cholesky tiles: ntiles x 64 x 64, same element type
  int64_t x_off;     // solution vector (delta_b or z_b): m_pad complex128
  int64_t r_off;     // right-hand side, then residual of the CG iteration: m_pad complex128
  int64_t y_off;     // triangular-solve intermediate: m_pad complex128
  int64_t z_off;     // preconditioned residual M^{-1} r: m_pad complex128
  int64_t p_off;     // CG search direction: m_pad complex128
  int64_t q_off;     // operator applied to the search direction: m_pad complex128
  int64_t u_off;     // per-sample vector of the block: n_s complex128
  int64_t tr_off;    // trace of the block QGT (one double, written by the column pass)
  int64_t cg_off;    // this block's CG scalars (CgScal)
  double lambda;
  double inv_ns;
};

struct ProbDev {
  int64_t n_s;
  int64_t n_p;
  int32_t first_block;
  int32_t n_blocks;
  int64_t dE_off;    // centred local energies, n_s complex128
  int64_t mu_off;    // column means, n_p complex128
  int64_t F_off;     // force, n_p complex128
  int64_t v_off;     // column-pass result used by the sample-space operator, n_p complex128
  int64_t sd_off;    // diagonal of the QGT, sum_x |O[x,k]|^2 / n_s - |mu_k|^2, n_p double
  int64_t scal_off;  // scalars: [0] sum of dE (complex128)
  int32_t rc;        // row chunks of the column pass (depends on n_s only)
  int32_t pad;
  double lambda;
  double inv_ns;
};

// Pointers bound per call, stored in the workspace by a bind kernel so that
// every other kernel reads them from device memory.
struct ProbPtrs {
  const void* O;
  int64_t ldo;
  const double2* e_loc;
  double2* delta;
};

struct BindArgs {
  ProbPtrs p[kMaxProblems];
};

// Column-pass tile: up to 64 columns of one block.
struct ColTile {
  int32_t g;     // global block
  int32_t c0;    // first column within the block
  int32_t nc;    // number of columns (<= 64)
  int32_t pad;
};

// Gram work item: output tile (ti, tj), ti >= tj, of block g over the stage
// range [s0, s1) of the contraction; slot >= 0 marks a split-K partial.
struct GramItem {
  int32_t g, ti, tj, s0, s1, slot;
};

// Split-K reduction item: output tile of block g summing nsplit consecutive
// partial slots starting at slot0.
struct SplitItem {
  int32_t g, ti, tj, slot0, nsplit, pad;
};

// Row-pass item: up to 16 rows of one block.
struct RowItem {
  int32_t g, r0, pad0, pad1;
};

enum ColPhase : int32_t { COL_FORCE = 0, COL_APPLY = 1, COL_BACKPROJ = 2 };
enum RowPhase : int32_t { ROW_P_U = 0, ROW_S_APPLY = 1 };
enum CgPhase : int32_t { CG_START = 0, CG_ALPHA = 1, CG_BETA = 2, CG_FINAL = 3 };

// ---------------------------------------------------------------------------
// Cholesky as one persistent launch over a DAG of 64x64 tile tasks.
//
// Tile (i, j), i >= j, of a block receives, in order, the trailing updates from
// the panels k < j, grouped in chunks (chol_chunk_bounds), then its final
// operation: POTRF when i == j, TRSM when i > j.  A counter per tile
// (tri_index) counts the completed operations, kCholWaves per operation (each
// wave of the workgroup publishes its own stores); a task waits until its
// tile's counter shows every earlier operation on the tile and the counters of
// the tiles it reads show them final.
// ---------------------------------------------------------------------------
constexpr int kCholWaves = 4;
constexpr int kCholCtl = 16;   // control words: [0, 8) ticket counters of the XCD queues, [8] abort flag
// XCD that performs every operation on tile (i, j) of block g (nq XCDs).
__host__ __device__ inline int chol_owner(int g, int i, int j, int nq) { return (i + 2 * j + g) % nq; }
enum CholOp : int16_t { CHOL_POTRF = 0, CHOL_TRSM = 1, CHOL_UPD = 2 };
struct CholTask {
  int32_t g;                     // global block
  int16_t type;                  // CholOp
  int16_t i, j;                  // tile (i, j); TRSM: tile (i, k) with j = k; POTRF: i == j == k
  int16_t k0, k1;                // UPD: panels [k0, k1)
  int16_t seq;                   // index of this operation in the tile's sequence
};
__host__ __device__ inline int tri_index(int i, int j) { return i * (i + 1) / 2 + j; }
// Update chunks of tile column j with chunk length c: the panels [0, j - 1)
// in chunks of c, then the last panel j - 1 alone (it is the one the column
// waits for, so its update is kept short).
__host__ __device__ inline int chol_nchunks(int j, int c) { return j == 0 ? 0 : 1 + (j - 1 + c - 1) / c; }
__host__ __device__ inline void chol_chunk_bounds(int j, int c, int u, int& k0, int& k1) {
  const int n = chol_nchunks(j, c);
  if (u == n - 1) {
    k0 = j - 1;
    k1 = j;
  } else {
    k0 = u * c;
    k1 = (u + 1) * c < j - 1 ? (u + 1) * c : j - 1;
  }
}

// Per-block scalars of the preconditioned CG iteration (in the workspace).
struct CgScal {
  double rho;    // r^H z of the current iterate
  double est;    // relative size of the last correction, ||z|| / ||x + z||
  int32_t done;  // the block met the convergence test: later iterations skip it
  int32_t iters; // operator applications (CG iterations) the block has run
};


// ---------------------------------------------------------------------------
// Device formation of O (per-sample log-derivatives of the network).
// ---------------------------------------------------------------------------
constexpr int kJacMaxLayers = 8;   // dense layers of a network
constexpr int kJacMaxSegs = 10;    // column segments of one row of O
constexpr int kJacTaskElems = 4096;  // target columns of one row of O per workgroup
constexpr int kJacMaxTaskRows = 1024;  // product rows of one task (their derivatives are staged in LDS)

// Dense-layer product C[s, o] = sum_k A[s, k] B(k, o), s < n_s, o < n_o,
// k < n_k, with B(k, o) = W[k * wk + o * wo].  A is the int8 spin matrix x
// (row stride lda) or a complex128 activation matrix.  FWD: z = C + bias,
// tg = tanh(z) * (scale ? scale[o] : 1), h = logcosh(z) when h is set.  BWD:
// tg *= C (the derivative reaching the layer's output times tanh of its
// pre-activation).
struct DenseArgs {
  const int8_t* x;      // A when the layer reads the spins
  const double2* a;     // A otherwise
  int64_t lda;
  const double2* W;
  int64_t wk, wo;
  const double2* bias;  // FWD: n_o entries
  const double2* scale; // FWD: readout weights, or null
  double2* tg;          // n_s x n_o, row stride ldt
  double2* h;           // FWD: logcosh(z), or null
  int64_t ldt;
  int64_t n_s;
  int32_t n_o, n_k;
};

// One column segment of a row of O.  OUTER: n_out x n_in outer product
// g[j] * v[i] (row-major), then the n_out entries g[j] (the layer's bias
// derivatives).  COPY: the n_in entries v[i], then a constant 1 when tail_one.
// v is the spin row (v_layer = 0) or the activation h^{v_layer}; g is the
// derivative array of layer g_layer.  A row of O is cut into tasks (one
// workgroup each): an OUTER segment into blocks of jrows product rows (the
// last block also writes the bias part), a COPY segment into one task.
enum JacKind : int32_t { JAC_OUTER = 0, JAC_COPY = 1 };
struct JacSeg {
  int64_t off;          // first column in the row of O
  int32_t kind, n_out, n_in, g_layer, v_layer, tail_one;
  int32_t task0;        // first task of the segment within a row
  int32_t jrows;        // OUTER: product rows per task
  int32_t rpi;          // OUTER with n_in < 256: product rows per 256-lane pass (256 / n_in), else 1
  int32_t pad;
};

struct JacArgs {
  JacSeg seg[kJacMaxSegs];
  const double2* g[kJacMaxLayers + 1];  // derivative arrays by layer (index 1..L)
  const double2* v[kJacMaxLayers + 1];  // activation arrays by layer (index 1..L); index 0 unused
  int64_t ld[kJacMaxLayers + 1];        // row stride of both arrays of a layer
  const int8_t* x;
  int64_t ldx;
  void* O;
  int64_t ldo;
  int64_t n_s;
  int32_t nseg;
  int32_t tasks;                        // workgroups per row
};

// Periodic 3x3 convolution layer over all samples: rows r = sample * S + site
// (S = side^2 sites, row-major), C[r, o] = sum_k A(r, k) B(k, o) with
// k = (input channel, offset) = c * 9 + 3 dy + dx.  FWD: A(r, k) =
// h[sample][c][site shifted by (dy - 1, dx - 1)] (the spins for the first
// layer), B(k, o) = K[o][c][dy][dx], output channels o < cout; epilogue as
// for a dense layer.  BWD: A(r, k) = g[sample][c][site shifted by
// (1 - dy, 1 - dx)], B(k, o) = K[c][o][dy][dx], o < cin; tg *= C.
// Activations are stored channel-major per sample: [sample][channel][site].
struct ConvArgs {
  const int8_t* x;      // spins (first layer, FWD)
  int64_t ldx;
  const double2* a;     // input activations (FWD) or derivatives (BWD)
  const double2* K;     // the layer's kernel, [cout][cin][3][3]
  const double2* bias;  // FWD
  double2* tg;          // FWD: tanh(z) (= d log psi / d z on the last layer); BWD: multiplied in place
  double2* h;           // FWD: logcosh(z), or null
  int64_t n_s;
  int32_t side, cin, cout;
  int32_t n_o, n_k;     // outputs (cout FWD, cin BWD) and contraction length (9 cin FWD, 9 cout BWD)
};

// Kernel derivatives of every layer: one workgroup per (sample, layer).
struct ConvDkLayer {
  const double2* g;     // d log psi / d z of the layer, [sample][cout][site]
  const double2* hin;   // input activations [sample][cin][site], null for the spins
  int64_t off;          // first column of the layer's block in a row of O
  int32_t cin, pad;
};
struct ConvDkArgs {
  ConvDkLayer layer[kJacMaxLayers];
  const int8_t* x;
  int64_t ldx;
  void* O;
  int64_t ldo;
  int64_t n_s;
  int32_t side, cout;
};

}  // namespace qgt
