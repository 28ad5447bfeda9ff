// Internal declarations shared by the kernel and driver translation units of
// the MI355X k-means library.  Not part of the public ABI (include/kmeans.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace km {

constexpr int kSelDigitBits = 12;
constexpr int kSelBins = 1 << kSelDigitBits;
constexpr int64_t kSelChunk = 8192;   // indices per block in the ordered compaction
constexpr int kThreads = 256;          // threads per block of the point kernels
constexpr int kSlots = 32;             // rows of 64-bit cluster-sum slots blocks add into
// Bias of the sums of the paired-tile pass: each term is added as the bits of
// 1.5 2^52 + q (q = rint(x 2^F)), so the finalize subtracts N of these (mod 2^64).
constexpr unsigned long long kSumBias = 0x4338000000000000ull;
constexpr int kMaxBlocks = 4096;       // upper bound of an assignment kernel's grid
constexpr int kHistLds = 16384;        // labels up to this count are sorted with LDS counters
constexpr int kScreenRows = 256;       // BF16 center rows are padded to a multiple of this

// Rows of the BF16 screen's center copy: k padded with zero rows whose bias is huge.
inline int64_t bf16_rows(int32_t k) {
  return ((int64_t)k + kScreenRows - 1) / kScreenRows * kScreenRows;
}
// Position of entry (row j, dim t) in the BF16 screen's center copy (kd16 dims
// per row).  The copy is tiled: tiles of 32 rows; in a tile, the 16-byte chunks
// (8 dims) of all 32 rows for chunk 0, then chunk 1, and so on.  A stage of
// tiles is then one contiguous range, and the rows of one chunk are contiguous
// for the MFMA operand reads.
__host__ __device__ inline int64_t cb16_at(int64_t j, int t, int kd16) {
  return (((j >> 5) * (kd16 >> 3) + (t >> 3)) * 32 + (j & 31)) * 8 + (t & 7);
}

// Progress of one radix selection of the r smallest 64-bit keys.  When done,
// a key is selected iff its top `bits` bits are <= prefix (keys are distinct).
struct SelState {
  uint64_t prefix;
  int64_t need;       // still to take from the bin `prefix`
  int64_t bin_count;  // elements in the bin `prefix`
  int32_t bits;
  int32_t done;
};

// Device-resident state of one stage's Lloyd loop.
struct PassState {
  int32_t done;        // stage finished: kernels of later passes return at once
  int32_t iter;        // passes run in this stage
  int32_t max_iter;
  int32_t F;           // cluster sums add rint(x * 2^F) as 64-bit integers
  float scale;         // 2^F
  float cmax;          // upper bound of max_j ||c_j||, for the FP32 error bound
  uint32_t maxabs_bits;  // bits of max |x| over the stage's rows (NaN/Inf -> >= 0x7f800000)
  uint32_t xn2max_bits;  // bits of max ||x||^2 over the stage's rows
  uint32_t ticket;     // blocks of the finalize kernel that are done (last one concludes)
  uint32_t qcount;     // points queued for the BF16 re-screen in this pass
  int32_t FJ;          // the sorted update adds J in units of 2^-FJ (exact integer limbs)
  float B;             // score offset >= max ||x||^2 of the BF16 screen (keeps scores >= 0)
  int32_t nonfinite;
  int32_t empty;
  int32_t converged;
  double tol;
  double J;
  double shift;
  int64_t uncertain;   // labels settled by the FP64 check over all centers, cumulative
  int64_t pairs;       // labels settled by FP64 between the best two candidates, cumulative
  int64_t rows;
  // BF16 screen: dcn >= max_j ||bf16(-2 c_j) + 2 c_j|| for the current centers
  // (the exact rounding error of the screen's center copy); dcn_bits gathers
  // the maximum over the blocks of the kernel that writes the copy.
  float dcn;
  uint32_t dcn_bits;
  // Empty-cluster re-seeding (opt-in): reseed = 1 turns it on for the stage;
  // reseed_j is the empty cluster the current pass re-seeds (-1: none).
  int32_t reseed;
  int32_t reseed_j;
};

// One instance of a batched pass: many independent k-means problems advance
// together, one launch per kernel for all of them (device-resident; filled by
// the host).  Work units are tiles of points; finalize entries are centers.
struct BatchInst {
  const void* X;
  int64_t n;
  int32_t d, k;
  int32_t dtype;     // 0 FP32, 1 BF16
  int32_t mode;      // 0 idle, 1 Lloyd pass (assign + update), 2 labelling pass
  int32_t lds_sums;  // 1: cluster sums privatised in LDS, 0: atomics into the slot rows
  int32_t ktile;     // centers per LDS tile of the assignment
  int64_t unit0, units;  // its work units in the assignment grid (tiles of tile_pts points)
  int64_t tile_pts;
  int64_t center0;       // its first entry in the finalize grid (k entries)
  double* c64; float* cw; float* cn; double* cnorm; double* shiftj; int32_t* emptyj;
  PassState* st;
  long long* slots;      // [kSlots][k][d+1]
  int32_t* labels;       // [n]
  double* Jpart;         // [units]
  long long* upart;      // [2 * units]
  double* J_hist; double* shift_hist;  // optional, indexed by the pass
  // BF16 screen instances (k_batch_screen): the tiled BF16 copy of -2c as
  // hi + lo (bf16_rows(k) rows of kd16 dims each) and ||c||^2 + B; NULL for
  // the FP32 kernel
  uint16_t* cb16; float* cnB; int32_t kd16;
  uint16_t* cb16lo;
  // Lloyd passes whose sums do not fit in LDS: units of k_batch_sums (ranges of
  // kBatchSumPts points x skc centers), 0 when the assignment adds the sums
  int32_t skc;
  int64_t sunit0, sunits;
  // slot rows the pass adds into (a power of two <= kSlots; the finalize reads
  // only these)
  int32_t nslots;
};
struct BatchHead {
  int32_t ninst;
  int32_t pad;
  int64_t units;    // sum of the instances' units (assignment) ...
  int64_t centers;  // ... and of their k (finalize)
};
// Compact per-instance status after a batched pass, for the host scheduler.
struct BatchStatus {
  int32_t done, iter, converged, empty, nonfinite, pad;
  double J, shift;
  int64_t uncertain;
};

// Launch helpers (kernels.hip).  All return hipSuccess or the launch error.
hipError_t sel_run(const int64_t* idx_arr, int64_t count, uint64_t seed, int64_t r,
                   SelState* st, unsigned long long* hist, int64_t* blk, int64_t* out,
                   hipStream_t s);
hipError_t rank_by_key(const int64_t* sel, int32_t k, uint64_t seed, int64_t* out,
                       hipStream_t s);
hipError_t gather_rows(const void* X, int64_t nrows, int dtype, int32_t d, const int64_t* idx,
                       int64_t m, void* out, hipStream_t s);
hipError_t centers_from_rows(const void* X, int64_t nrows, int dtype, int32_t d,
                             const int64_t* idx, int32_t k, double* c64, hipStream_t s);
hipError_t stage_reset(PassState* st, hipStream_t s);
hipError_t row_stats(const void* X, int dtype, int64_t rows, int32_t d, bool norms,
                     PassState* st, hipStream_t s);
hipError_t zero_i64(long long* p, int64_t count, hipStream_t s);
// cb16lo: when given, -2c is kept as hi + lo (the rest rounded to BF16 again)
hipError_t prep_bf16(const double* c64, int32_t k, int32_t d, int kd16, PassState* st,
                     uint16_t* cb16, float* cnB, hipStream_t s, uint16_t* cb16lo = nullptr);
hipError_t prep_centers(const double* c64, int32_t k, int32_t d, float* cw, float* cn,
                        double* cnorm, hipStream_t s);
hipError_t stage_begin(PassState* st, int32_t max_iter, double tol, int64_t rows,
                       const double* cnorm, int32_t k, int32_t d, int64_t pg, hipStream_t s,
                       int reseed = 0);

struct PassBufs {
  const void* X; int dtype; int64_t n; int32_t d; int32_t k;
  double* c64; float* cw; float* cn; double* cnorm;
  double* shiftj; int32_t* emptyj;
  long long* slots;    // [kSlots][k][d+1] exact cluster sums (counts last); zero between passes
  long long* jslots;   // [kSlots][2] J of the sorted update as limbs of 2^-FJ, 2^(40-FJ); zeroed
  uint32_t* perm;      // [n] point indices in label order (sorted update)
  long long* scnt;     // [k * sort_chunks] label counts per chunk, then their offsets
  long long* stot;     // [scan tiles + 1] tile totals of the offset scan
  long long* rstart;   // [k + 1] first position of every label's run
  uint16_t* cb16;      // bf16_rows(k) x ks*16 BF16 (-2 c) of the BF16 screen, tiled (cb16_at)
  float* cnB;          // [bf16_rows(k)] ||c||^2 + B of the BF16 screen (+inf on padding rows)
  uint32_t* queue;     // [n] points of the BF16 screen with more than 4 candidates (n < 2^32)
  int4* rq_c;          // [n] candidates of the points the BF16 screen marks for the FP64
                       //   re-rank (label -1): up to four center indices, -1 = none
  float* qthr;         // [n] their score thresholds
  double* Jpart; long long* upart;
  int32_t* labels;     // labels of the rows (required by the split path)
  PassState* st;
  double* J_hist; double* shift_hist;
  double* S_out; int64_t* N_out;   // optional exact sums / counts of the pass
  // optional per-pass trace, indexed by the stage's pass: the centers a pass
  // starts from ([pass][k][d]) and its cluster sizes ([pass][k])
  double* trace_c; long long* trace_n;
  // re-seeding: per-block farthest-point partials of k_farthest (kFarBlocks)
  double* fpart; long long* fidx;
};
constexpr int kFarBlocks = 1024;       // grid of the farthest-point search

// Geometry chosen once per (rows, d, k): fused or split path and block counts.
struct PassPlan {
  bool bf16;         // split pass with the BF16 MFMA screen (x.c^T as 32x32x16 tiles)
  bool fscreen;      // fused pass on the BF16 MFMA screen (d <= 16, k <= 128)
  bool fsplit;       // ... with -2c and FP32 points as BF16 hi + lo parts (auto precision)
  int ks;            // 16-dim K steps of the BF16 screen
  bool mfma;         // fused pass on FP32 MFMA (x.c^T as 32x32x2 tiles)
  int kd, nt;        // padded dims and 32-center tiles of the MFMA kernels
  int d;             // dims of the rows (the fused screen has a kernel for d == kd)
  bool fused;
  int dmax;          // register tile of a row (0: generic)
  int ppt;           // points per thread
  int64_t blocks;    // blocks of the assign kernel (= partial rows in the fused path)
  int64_t sort_chunk;   // points per chunk of the label sort (split path)
  int64_t sort_chunks;
  int64_t pg;           // positions per lane group of the run sums
  size_t lds_assign;
  int ktile;         // centers per LDS tile (split assign)
  int64_t rr_blocks = 0;  // resident blocks of the re-rank kernel (BF16 screen path)
};

// The pass keeps a BF16 copy of the centers (prep_bf16, then the finalize).
inline bool copy16(const PassPlan& p) { return p.bf16 || p.fscreen; }
// The stage statistics include max ||x||^2 (split paths and the BF16 screens).
inline bool wants_norms(const PassPlan& p) { return !p.fused || p.fscreen; }

// Batched passes (kernels.hip).  A group shares the element type and the
// register tile (dmax, points per thread); bi/hd are device pointers.
struct BatchShape {
  int dtype, dmax, ppt;
  size_t lds;   // dynamic LDS of the assignment launch
  int blocks;   // persistent grid
  int screen;   // K steps of the BF16 screen kernel (0: the FP32 kernel)
};
// The batched BF16 screen takes BF16 data with 16 < d <= 128 and k <= 256;
// returns its K steps (2, 4 or 8), or 0.
int batch_screen_ks(int dtype, int32_t d, int32_t k);
int batch_dmax(int32_t d);                       // 0: d too large for the batched path
int64_t batch_resident_blocks(int dtype, int dmax, int ppt, size_t lds, int cus,
                              int screen = 0);
hipError_t batch_assign(const BatchHead* hd, const BatchInst* bi, const BatchShape& sh,
                        hipStream_t s);
// Cluster sums of the instances with sum units (after the assignment launches).
constexpr int64_t kBatchSumPts = 8192;
constexpr size_t kBatchSumLds = 65536;
hipError_t batch_sums(const BatchHead* hd, const BatchInst* bi, int blocks, hipStream_t s);
hipError_t batch_finalize(const BatchHead* hd, const BatchInst* bi, int blocks, hipStream_t s);
hipError_t batch_status(const BatchHead* hd, const BatchInst* bi, BatchStatus* out,
                        hipStream_t s);
// uniform [-1, 1) values: kind 0 FP32, 1 BF16 bits, 2 FP64
hipError_t fill_uniform(void* p, int kind, int64_t count, uint64_t seed, hipStream_t s);

PassPlan plan_pass(int64_t rows, int32_t d, int32_t k, int dtype, int precision,
                   size_t lds_limit, int cus);
hipError_t lloyd_pass(const PassBufs& b, const PassPlan& p, bool update, hipStream_t s);
// the assignment kernel of a pass (for the BF16 path, its screen of all points), and
// everything after it (re-screen, update, reduction, stop test)
hipError_t pass_assign(const PassBufs& b, const PassPlan& p, bool update, hipStream_t s);
hipError_t pass_rest(const PassBufs& b, const PassPlan& p, bool update, hipStream_t s);
hipError_t assign_only(const PassBufs& b, const PassPlan& p, hipStream_t s);

}  // namespace km
