// Internal declarations of libspaqr: host plan, runtime state, kernel
// descriptors and launchers.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <set>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/spaqr.h"

namespace spaqr {
struct KernelTimer;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SPAQR_HIP(call)                                                                 \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::spaqr::Error(SPAQR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Analysis (host only)
// ---------------------------------------------------------------------------

struct NDNode {
  int level = 0;
  int64_t path = 0;
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  int axis = -1;  // -1: leaf
  int t = -1;     // first separator plane
  int child[2] = {-1, -1};
  int parent = -1;
  int rank = 0;
  // cluster ids of the pieces at granularity level + i
  std::vector<std::vector<int>> pieces;
  bool leaf() const { return axis < 0; }
};

struct Cluster {
  int64_t key0 = 0, key1 = 0;  // (separator elimination rank, lower-corner cell)
  int sep = -1;                // ND node index (rank)
  int gran = 0;
  int lo[3], hi[3];
  int parent = -1;
  std::vector<int> children;   // cluster ids at gran + 1, in id order
  std::vector<int> cells;      // finest clusters: cells ascending
  int finest_index = -1;
};

struct InitGroup {
  int owner;                   // cluster id
  std::vector<int> rows;       // ascending
  std::vector<int> clus;       // touched clusters, id order
  int64_t offset;              // element offset inside the initial-group region
  int64_t ld;
  int width;
};

struct Plan {
  int64_t M = 0, N = 0, nnz = 0;
  int grid[3] = {1, 1, 1};
  int depth = 0, skip = 0, w = 2;
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col_idx;
  std::vector<double> vals, D, ahat;
  std::vector<NDNode> nodes;        // indexed by elimination rank
  std::vector<Cluster> clusters;    // every granularity; id order == key order
  std::vector<int> finest;          // finest cluster ids, id order
  std::vector<int> col_cluster;     // finest cluster id of each column
  std::vector<int> row_owner;       // finest cluster id of each row
  std::vector<InitGroup> init_groups;
  std::vector<int64_t> init_dst;    // per CSR entry: element offset of its slot in the initial groups
  int64_t init_elems = 0;
  // A^T in CSR (column-major view of A) for the transposed products
  std::vector<int64_t> at_ptr;
  std::vector<int32_t> at_idx;
  std::vector<int64_t> at_src;      // CSR entry index of each A^T entry
  // Independent problems held by the plan (a batch is the block-diagonal
  // union): problem g owns columns [seg_col[g], seg_col[g+1]) and rows
  // [seg_row[g], seg_row[g+1]).
  int count = 1;
  std::vector<int64_t> seg_col, seg_row;
  std::vector<int> seg_depth;
};

void analyze_plan(Plan& P, const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                  int64_t M, int64_t N, const spaqr_options& opt);
// Block-diagonal union of independently analysed plans.  Tree levels are
// aligned from the leaves (a problem of depth d sits at levels
// depth_max - d + 1 .. depth_max), so one level of the union holds the
// same-level fronts of every problem.  All parts must share the
// sparsification skip.
void union_plans(Plan& U, std::vector<Plan>& parts);
void rescale_values(Plan& P, const double* vals);
// Graph nested dissection, interfaces and hierarchy for a plan without a
// grid (fills nodes, clusters, finest, col_cluster); graph_nd.cpp.
void graph_partition(Plan& P);
// Row matched to every column: the assignment of largest product of |a_ij|.
std::vector<int64_t> max_product_matching(const Plan& P);
// Checks, row ownership (matched rows to their column's cluster, the others
// by the max-norm rule), initial groups and the transposed pattern.
void finish_plan(Plan& P, const std::vector<int64_t>& match);

// ---------------------------------------------------------------------------
// Device memory
// ---------------------------------------------------------------------------

// Bump allocator over large device chunks; reset() keeps the chunks.
class Arena {
 public:
  ~Arena();
  void* alloc(size_t bytes);
  void reset();
  void release();
  size_t capacity() const;
  size_t used() const { return used_total_; }

 private:
  struct Chunk {
    char* ptr;
    size_t size;
    size_t off;
  };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0;
  size_t used_total_ = 0;
};

// Bump allocator over pinned host memory, used to stage descriptor uploads.
class Staging {
 public:
  ~Staging();
  void* alloc(size_t bytes);
  void reset();
  void release();

 private:
  struct Chunk {
    char* ptr;
    size_t size;
    size_t off;
  };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0;
};

// ---------------------------------------------------------------------------
// Kernel descriptors (plain structs copied to the device)
// ---------------------------------------------------------------------------

// dst[(row0 + r) + (col0 + c) * dst_ld] = colmap[c] >= 0 ? src[r + colmap[c] * src_ld] : 0
// (transpose == 1: dst[c + (col0 + r) * dst_ld] instead).
struct GatherDesc {
  const void* src;
  void* dst;
  const int* colmap;
  int64_t src_ld, dst_ld, row0, col0;
  int nrows, ncols, transpose, pad_;
};

// Column map of a gather built on the device from the group's side: out[c]
// = i where fpos[i] = c (fpos: front column of each of the group's nslots
// columns, -1 where the front has none), -1 for the other c < n.
struct ExpandDesc {
  const int* fpos;
  int* out;
  int nslots, n;
};

// Householder QR of the leading k columns of A (m x n, ld lda); the
// reflectors are applied to all n columns.  tau[min(m,k)].
struct QRDesc {
  void* A;
  void* tau;
  int64_t lda;
  int m, n, k, pad_;
};

// Column-pivoted QR of A (m x n), in place, columns not swapped; first
// `rank` rows of A become the first rows of Q^T A with zeros below the
// diagonal of pivot columns.  V (ld m) and tau receive the reflectors when
// non-null.  rank_out[0] receives the rank.
// Rank rule: stop at the first step i with |R_ii| <= noise * ||A||_F (the
// numerical rank), then at |R_ii| < eps |R_00| unless `exact` is set, or at
// i == forced when forced >= 0.
struct PQRDesc {
  void* A;
  void* V;
  void* tau;
  double* work;      // 3 * n doubles (norms, reference norms, done flags)
  int* rank_out;
  int* piv_out;      // pivot column per step (min(m,n))
  int64_t lda;
  double noise;
  int m, n, forced;
  int blk0, nblk;    // this matrix's column chunks in the launch (set by the launcher)
  int cw;            // columns per chunk (set by the launcher)
  int g0;            // first 8-column group of this matrix (persistent form)
  int exact;         // 1: the eps rule is off (only the numerical-rank floor stops)
};
static_assert(sizeof(PQRDesc) == 96, "one pivot-step work-group reads one 96-byte descriptor");

// Per-matrix state of the step-synchronous pivoted QR, double-buffered by
// step parity (step i reads slot i&1 and writes slot (i+1)&1).
struct PQRState {
  double r00, floor, beta;
  int pivot, pstep, rank, stopped;
};
// chunk argmax of one step (one 16-byte load per chunk when scanned)
struct alignas(16) PQRPart {
  double val;
  int idx, pad_;
};

// B <- B R^-1 on the columns colmap[0..c) of a group block (nrows x ., ld).
struct TrsmDesc {
  void* B;
  const void* R;
  const int* colmap;
  int64_t ldb, ldr;
  int nrows, c;
};

// owner[i] = argmax over clusters q of sum_{c in q} A[i, colmap[c]]^2 for
// i < nrows, cluster q owning colmap entries [cl_off[q], cl_off[q+1]);
// first maximum wins.  nrows_dev (when set) holds the row count on the
// device, e.g. the rank just chosen by a rank-revealing QR; nrows is then
// its upper bound.
struct OwnerDesc {
  const void* A;
  const int* colmap;
  const int* cl_off;
  int* owner;
  const int* nrows_dev;
  int64_t lda;
  int nrows, ncl;
};

// dst[i + c * dst_ld] = src[rows[i] + c * src_ld] for c < ncols, zeroed where
// c < rows[i] - tri_base when tri != 0 (upper-trapezoidal rows).
struct RowCopyDesc {
  const void* src;
  void* dst;
  const int* rows;
  int64_t src_ld, dst_ld;
  int nrows, ncols, tri, tri_base;
};

// Copy upper triangle of A (c x c, lda) to R (ldr), then set the block to I.
// flag[0] = 1 if min |R_ii| <= 64 u ||R||_F.
struct ExtractDesc {
  void* A;
  void* R;
  int* flag;
  int64_t lda, ldr;
  int c, pad_;
};

// Step-2 write-back.  For transposed pieces: dst[r + colmap[i] * ld] =
// C[i + (col0 + r) * ldc] for i < rank, r < nrows.  For the scaled rows
// (transpose == 0): dst[i + colmap[c] * ld] = C[i + (col0 + c) * ldc] for
// i < rank, c < ncols; identity == 1 writes delta_ij on colmap instead.
struct ScatterDesc {
  const void* C;
  void* dst;
  const int* colmap;
  const int* rank;
  int64_t ldc, ld, col0;
  int nrows, ncols, transpose, identity;
};

// ---------------------------------------------------------------------------
// Apply descriptors (W^-1 / W^-T sweeps)
// ---------------------------------------------------------------------------

struct ApplyOp {
  const void* R;       // eliminate / scale: triangular factor; sparsify: reflectors
  const void* tau;     // sparsify
  const int* s1;       // slots of the cluster
  const int* s2;       // slots of the neighbours (eliminate)
  int64_t ld;
  int n1, n2;          // eliminate: c_s, c_N; scale: c_p, 0; sparsify: c_p, r
  int kind;
  int nstage;          // eliminate, W^-T: offset of R_sN^T x_s in the staging buffer
  int64_t poff;        // eliminate: offset of its vectors in the work buffer (see below)
  int nchunk, pad_;    // eliminate: column chunks of R_sN (APPLY_CHUNK columns each)
};
// Neighbour products of the eliminations are split over column chunks of
// R_sN, one work-group per (op, chunk):
//  W^-1: work[poff + k * n1 + i] = sum over chunk k of R_sN[i, c] x_N[c], then
//        the op's work-group uses x_s - sum_k work[poff + k * n1 ..];
//  W^-T: the op's work-group writes t = R_ss^-T x_s to work[poff ..], then
//        stage[nstage + c] = R_sN[:, c]^T t per chunk.
constexpr int APPLY_CHUNK = 256;

// ---------------------------------------------------------------------------
// Launchers (kernels.hip, apply.hip)
// ---------------------------------------------------------------------------

template <typename T>
void launch_gather(const GatherDesc* d_desc, int n, int max_cols, hipStream_t s);
void launch_expand_maps(const ExpandDesc* d_desc, int n, hipStream_t s);
template <typename T>
void launch_scatter_csr(T* base, const int64_t* dst, const double* ahat, int64_t nnz, hipStream_t s);
// Blocked Householder QR of a batch.  Panels of QR_NB columns; a tall panel
// is split over row segments of QR_RS rows (two launches per column), the
// trailing update over (front, column tile, row segment) blocks with a
// deterministic two-stage reduction of V^T C.
constexpr int QR_NB = 32;
constexpr int QR_TN = 64;
constexpr int QR_RS = 1024;
struct QRWork {
  double* tbuf;   // nfront * NB * NB        compact-WY T factors
  double* betas;  // nfront                  last diagonal of a row-split panel
  double* normp;  // nfront * MS             norm partials
  double* dp;     // 2 * nfront * MS * NB    dot partials (two column parities in the cooperative panel)
  double* gp;     // nfront * MS * NB * NB   Gram partials
  double* wp;     // nfront * MT * MS * NB * TN  partial V^T C
  double* w;      // nfront * MT * NB * TN        reduced T^T V^T C
  int MS, MT;     // max row segments, max column tiles
};
void qr_work_dims(const std::vector<QRDesc>& h, int* MS, int* MT);
template <typename T>
// kt (may be null): the handle's kernel timer; family "qrp_coop" brackets
// every cooperative tall-panel launch with events.
// allow_coop: tall FP32 panels may use the cooperative one-launch form.
void launch_qr(const QRDesc* d_desc, const std::vector<QRDesc>& h_desc, const QRWork& ws, hipStream_t s,
               int* launches, KernelTimer* kt, bool allow_coop);
// Column-pivoted QR of a batch, one launch per pivot step (columns split in
// chunks of PQR_CW; the columns stay in registers while the step's 64-aligned
// row window is at most reg_rows rows, 1024 at most)
// chunks of PQR_CW over work-groups).  The caller provides device scratch:
// states (2 per matrix), parts (2 per chunk), frop (squared Frobenius norm
// per chunk, one per chunk), bmap (one int2 per chunk) and an `active`
// counter; h_desc must already carry blk0/nblk.  The step launch takes one
// descriptor per work-group (d_blk[b] = the descriptor of matrix bmap[b].x),
// so a work-group finds its matrix without a dependent load.
constexpr int PQR_CW = 8;
// self-timing stamps of one timed launch: STAMP_SLOTS slots of STAMP_STRIDE
// words (complement of the earliest start, latest end, padding)
constexpr int STAMP_SLOTS = 32;
constexpr int STAMP_STRIDE = 8;
template <typename T>
void launch_pqr_init(const PQRDesc* d_desc, int nblocks, PQRState* states, PQRPart* parts, double* frop,
                     const int2* bmap, hipStream_t s);
template <typename T>
void launch_pqr_step(const PQRDesc* d_blk, int nblocks, int total_parts, PQRState* states,
                     PQRPart* parts, const double* frop, const int2* bmap, int* active, int i, double eps,
                     int max_m, int cw, int reg_rows, unsigned long long* stamp, unsigned long long* report,
                     unsigned tag, bool check_first, hipStream_t s);
template <typename T>
void launch_pqr_finish(const PQRDesc* d_desc, int nmat, PQRState* states, int steps, hipStream_t s);
// Persistent form: all pivot steps of a batch in one cooperative launch of
// one-wave work-groups (chunks of the matrices' columns) that exchange, per
// step, their chunk argmax and candidate pivot column through the buffers
// below, as 64-bit words tagged with the step number.  Only for batches whose
// tallest matrix has at most PQR_RUN_ROWS rows; the factors are bit-identical
// to the one-launch-per-step form.  The buffers must be zeroed before the
// launch.
constexpr int PQR_RUN_ROWS = 256;
struct PQRXch {
  unsigned long long* part;  // [2][G][3] chunk argmax (value halves, column), by step parity
  unsigned long long* pub;   // [2][G][rows][sizeof(T) / 4] candidate columns
  unsigned long long* frop;  // [groups][2] squared Frobenius norm per 8-column group
  int* err;                  // set (and every wave exits) when a wait exceeds its spin limit
  int G;                     // work-groups (chunks) in the launch
  int rows;                  // rows per candidate column (64 PQ)
};
// 64-bit words of the exchange buffers of a launch
inline size_t pqr_xch_words(int G, int rows, int groups, size_t tsize) {
  return 6 * (size_t)G + 2 * (size_t)G * rows * (tsize / 4) + 2 * (size_t)groups;
}
// Chooses the chunk width for a batch (columns per work-group), or returns 0
// when the persistent form does not apply (too tall, or more work-groups than
// can be co-resident).  ns: column counts of the matrices.
template <typename T>
int pqr_run_width(int max_m, const std::vector<int>& ns, int* rows);
template <typename T>
void launch_pqr_run(const PQRDesc* d_desc, int nblocks, const int2* bmap, const PQRXch& xc, double eps, int cw,
                    unsigned long long* stamp, hipStream_t s);
// rowblocks: (descriptor, block) for every TRSM_ROWS-row block of every
// descriptor with rows (the LDS form launches one work-group per entry)
constexpr int TRSM_ROWS = 64;
template <typename T>
void launch_trsm(const TrsmDesc* d_desc, int n, int max_rows, int max_c, const int2* d_rowblocks,
                 int n_rowblocks, hipStream_t s);
template <typename T>
void launch_owner(const OwnerDesc* d_desc, int n, int max_rows, hipStream_t s);
template <typename T>
void launch_rowcopy(const RowCopyDesc* d_desc, int n, int max_cols, hipStream_t s);
template <typename T>
void launch_extract(const ExtractDesc* d_desc, int n, hipStream_t s);
template <typename T>
void launch_scatter(const ScatterDesc* d_desc, int n, hipStream_t s);

// One round of W^-1 or W^-T ops.  In W^-T an elimination writes
// R_sN^T x_s to stage + nstage instead of updating x; launch_apply_nsum then
// subtracts, per neighbour slot, its contributions summed in op order
// (deterministic, no atomics).
template <typename T>
void launch_apply_batch(const ApplyOp* d_ops, int n, int max_n1, bool transpose, double* x,
                        double* stage, double* work, hipStream_t s);
// chunk work-groups of the eliminations of a batch: chunks[k] = (op, chunk)
template <typename T>
void launch_apply_gemv(const ApplyOp* d_ops, const int2* chunks, int nchunks, bool transpose, const double* x,
                       double* stage, double* work, hipStream_t s);
void launch_apply_nsum(const int* nslots, const int* nptr, const int* noff, int n, const double* stage,
                       double* x, hipStream_t s);

void launch_spmv(const int64_t* ptr, const int32_t* idx, const double* val, const double* x,
                 double* y, int64_t rows, hipStream_t s);
void launch_spmv_at(const int64_t* ptr, const int32_t* idx, const int64_t* src, const double* val,
                    const double* x, double* y, int64_t cols, hipStream_t s);

}  // namespace spaqr
