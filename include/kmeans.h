/*
 * kmeans.h -- C ABI of the MI355X two-stage (fast/slow) k-means library.
 *
 * Method: Salman, Kecman, Li, Strack and Test, "Fast k-means algorithm
 * clustering" (arXiv 1108.1351), section 2 (Algorithm): Lloyd passes
 * (squared distance, nearest center, cluster averages) first on a random
 * fraction of the data starting from centers sampled from that fraction (the
 * fast stage), then on the whole data starting from the fast stage's centers
 * (the slow stage).  Readings of what the paper leaves open:
 *   - distance is the squared Euclidean distance ("modified distance" of the
 *     Algorithm, eq. (1) without the root); ties go to the lowest center index;
 *   - J is eq. (3) taken as a sum over the points of the squared distance to
 *     the nearest center;
 *   - a stage stops after the pass whose largest center movement (Euclidean)
 *     is below tol, or after max_iter passes (sections 5 and 6 stop on center
 *     movement); that last pass is counted, as in Table 1;
 *   - a cluster left without points keeps its center;
 *   - the fast-stage subset holds m = min(n, max(k, floor(f*n + 0.5))) points,
 *     those with the smallest keys key_i = SplitMix64 output i+1 for the seed
 *     (Steele, Lea and Flood 2014); the initial centers are the k points with the
 *     smallest keys, center j being the point with the j-th smallest key;
 *   - labels and J are returned at the returned centers (one extra pass).
 *
 * Pointers.  X, centers and labels are DEVICE pointers (HIP, this process's
 * current device), owned by the caller; the library never frees or keeps them
 * after a call returns.  Info structs are HOST memory.  Rows are row-major,
 * 64-bit indexed.
 *
 * Errors.  Every entry point returns a km_status and never aborts or throws.
 * On a non-OK status the outputs are unspecified and kmeans_last_error()
 * returns a message (thread-local, valid until the next call on that thread).
 * Not converging within max_iter is not an error (converged[s] = 0).
 *
 * Determinism.  Cluster sums are exact 64-bit fixed-point integer sums and J
 * is reduced in a fixed order, so a call repeated on the same inputs returns
 * identical bits.
 */
#ifndef KMEANS_MI355X_H
#define KMEANS_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KM_OK = 0,
  KM_EINVAL = 1,      /* invalid argument (bad size, null pointer, NaN/Inf in X, ...) */
  KM_ENOMEM = 2,      /* device allocation failed or the workspace is too small */
  KM_EDEVICE = 3,     /* a HIP call failed; the message carries hipGetErrorString */
  KM_EBUSY = 4,       /* resource in use (serving: queue full) */
  KM_ECANCELLED = 5,  /* serving: the job was cancelled or the server destroyed */
  KM_ETIMEOUT = 6,    /* serving: the wait timed out */
  KM_ENOTFOUND = 7    /* serving: unknown ticket */
} km_status;

typedef enum { KM_F32 = 0, KM_BF16 = 1 } km_dtype;

typedef enum {
  KM_PREC_AUTO = 0,        /* d <= 16 and k <= 128: split BF16 MFMA screen (-2c and FP32 points as
                              BF16 high + low parts, FP32 accumulation); BF16 data with d >= 32:
                              BF16 MFMA + re-rank; otherwise FP32.  Every screen is certified:
                              points its error band cannot decide get FP64 decisions */
  KM_PREC_FP32 = 1,        /* FP32 distances, FP64 check of uncertain points */
  KM_PREC_BF16_RERANK = 2  /* BF16 MFMA x.c^T, FP32 re-rank of the top 4, FP64 check */
} km_precision;

typedef struct {
  int32_t iters[2];      /* passes run in the fast and slow stage, incl. the one that met tol */
  int32_t converged[2];  /* 1 if the stage stopped on shift < tol */
  int32_t empty[2];      /* clusters with no member in the last pass of each stage */
  int64_t m;             /* fast-stage subset size */
  double J;              /* sum over all n points of the squared distance to the nearest returned center */
  double J_stage1;       /* J of the last fast-stage pass (over the subset, at that pass's centers) */
  int64_t dist_evals;    /* k*(m*iters[0] + n*iters[1]) + k*n: point-center distances the method needs */
  double shift[2];       /* last largest center movement of each stage */
  int64_t uncertain;     /* labels the screen could not settle among its best candidates, summed
                            over passes: the FP64 check over all centers (FP32 and small-d
                            paths); on the BF16 screen path the points queued for the
                            re-screen, plus those it sends to the FP64 check */
  double seconds[3];     /* wall time of sampling, fast stage, slow stage + final labels */
  int64_t fp64_pairs;    /* labels decided among a short candidate list, summed over passes:
                            FP64 distances to the best two (FP32 and small-d paths); on the
                            BF16 screen path the points re-ranked among two to four
                            candidates, plus re-screened points decided in FP64 */
} km_info;

typedef struct {
  km_dtype dtype;              /* element type of X */
  km_precision precision;
  int32_t max_iter[2];         /* per stage (fast, slow), >= 1 */
  double tol[2];               /* per stage, >= 0 (0: run exactly max_iter passes) */
  const double* init_centers;  /* optional HOST k*d FP64: replaces the sampled initial centers */
  int32_t skip_stage1;         /* 1: slow stage only ("normal" k-means, or resume from init_centers) */
  void* stream;                /* hipStream_t to run on; NULL = the null stream */
  double* centers64_out;       /* optional DEVICE k*d FP64 copy of the returned centers */
  double* J_hist;              /* optional HOST arrays of max_iter[0] + max_iter[1] entries: */
  double* shift_hist;          /*   J and shift of every pass, fast stage first */
  /* Optional caller-provided DEVICE scratch (256-byte aligned).  With workspace
     != NULL the call takes all its device memory from it and allocates none;
     it returns KM_ENOMEM when workspace_bytes is below kmeans_workspace_bytes()
     for the same sizes and options.  The library keeps nothing in it after the
     call returns; calls that share one workspace must not overlap. */
  void* workspace;
  size_t workspace_bytes;
  /* 1: scan all of X for NaN/Inf before any pass (one extra read of X), so bad
     data fails before the fast stage; 0: each stage's statistics pass finds it
     (the same KM_EINVAL, after the fast stage when the bad rows lie outside the
     subset). */
  int32_t check_finite;
  /* Empty clusters.  0 (the paper is silent; the default): an empty cluster keeps
     its center.  1: after the update of a pass that left clusters empty, the
     lowest-index empty cluster takes as its new center the point farthest (FP64
     squared distance) from its nearest updated center, lowest point index on
     equal distances; that movement counts in the pass's largest movement.  One
     cluster per pass (section 3 warns of blank clusters from small subsets). */
  int32_t reseed;
  /* Optional HOST per-pass trace in the form of Table 1 (section 5), fast stage
     first, pass p of stage s at row max_iter[0]*s + p (rows past the passes
     run are zero):
       trace_centers: (max_iter[0] + max_iter[1]) * k * d FP64, the centers the
                      pass starts from (a pass's new centers start the next pass
                      of its stage, the fast stage's last ones start the slow
                      stage, the slow stage's last ones are returned);
       trace_counts:  (max_iter[0] + max_iter[1]) * k, the cluster sizes the
                      pass found. */
  double* trace_centers;
  int64_t* trace_counts;
} km_options;

/*
 * The two-stage method on FP32 data.  X: device n*d FP32.  centers_out: device
 * k*d FP32.  labels_out: device n int32 (may be NULL).  info: host (may be NULL).
 * Requires 1 <= k <= n, d >= 1, 0 < subset_frac <= 1, max_iter >= 1, tol >= 0.
 * Runs on the null stream and returns when the result is in place.
 */
km_status kmeans_fit(const float* X, int64_t n, int32_t d, int32_t k, double subset_frac,
                     uint64_t seed, int32_t max_iter, double tol, float* centers_out,
                     int32_t* labels_out, km_info* info);

/* As kmeans_fit with per-stage limits, BF16 data, a stream and a resume point.
   opt may not be NULL (fill it with kmeans_default_options). */
km_status kmeans_fit_ex(const void* X, int64_t n, int32_t d, int32_t k, double subset_frac,
                        uint64_t seed, const km_options* opt, float* centers_out,
                        int32_t* labels_out, km_info* info);

/*
 * kmeans_fit_ex for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * call's scratch is a fixed device array of KM_STATIC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends, and the call
 * allocates nothing (no device, pinned or event allocation; profiling with
 * kmeans_profile_begin does not record it).  opt->workspace must be NULL.
 * KM_ENOMEM when kmeans_workspace_bytes() for the sizes and options exceeds
 * KM_STATIC_SCRATCH_BYTES.  Every call on a GPU uses that GPU's one array:
 * calls that overlap in time on the same GPU (other threads or streams) race
 * and must not be made.  Results are those of kmeans_fit_ex.
 */
#define KM_STATIC_SCRATCH_BYTES (64u << 20)
km_status kmeans_fit_static(const void* X, int64_t n, int32_t d, int32_t k,
                            double subset_frac, uint64_t seed, const km_options* opt,
                            float* centers_out, int32_t* labels_out, km_info* info);

/* Options equivalent to kmeans_fit(max_iter, tol) on FP32 data. */
void kmeans_default_options(km_options* opt, int32_t max_iter, double tol);

/* Device bytes kmeans_fit_ex allocates for these sizes and options (0 on
   invalid sizes): the smallest workspace_bytes a caller workspace may have. */
size_t kmeans_workspace_bytes(int64_t n, int32_t d, int32_t k, double subset_frac,
                              const km_options* opt);

/*
 * Fast-stage sampling (Algorithm: "%per of S_n", "Select X_c from S_n
 * randomly").  subset_idx: device m int64, ascending point indices of the
 * subset; init_idx: device k int64, the initial centers' point indices in key
 * order.  m must equal min(n, max(k, floor(f*n + 0.5))) for some f; any
 * 1 <= k <= m <= n is accepted.  stream: hipStream_t or NULL.
 */
km_status km_sample(int64_t n, int64_t m, int32_t k, uint64_t seed, int64_t* subset_idx,
                    int64_t* init_idx, void* stream);

/*
 * One Lloyd pass (Algorithm, one iteration of a While loop): nearest centers of
 * the n rows of X (device, dtype) from centers C (device k*d FP64), cluster
 * sums S (device k*d FP64, exact sums rounded once), counts N (device k int64),
 * new centers C_new (device k*d FP64; an empty cluster keeps its center) and,
 * in host memory, J, the largest center movement and the number of empty
 * clusters.  labels (device n int32) may be NULL.
 */
km_status km_step(const void* X, km_dtype dtype, int64_t n, int32_t d, const double* C,
                  int32_t k, km_precision precision, int32_t* labels, double* S, int64_t* N,
                  double* C_new, double* J, double* shift, int32_t* empty, int64_t* uncertain,
                  void* stream);

/*
 * Nearest center of every row (the Algorithm's assignment step, at fixed
 * centers): labels (device n int32) and, in host memory, J = sum of the
 * squared distances to those centers (eq. (3) as a sum).
 */
km_status km_assign(const void* X, km_dtype dtype, int64_t n, int32_t d, const double* C,
                    int32_t k, km_precision precision, int32_t* labels, double* J,
                    int64_t* uncertain, void* stream);

/*
 * Pass timing, for measuring the library against the roofline.  Between
 * kmeans_profile_begin() and kmeans_profile_end(), every fit records HIP events
 * on its stream around each Lloyd pass and around the pass's assignment kernel
 * (the dominant kernel); only passes that ran are counted.  Process-wide;
 * fits that overlap in time are all counted.  out may be NULL.
 */
typedef struct {
  int64_t fits;          /* fits completed while profiling */
  int64_t passes[2];     /* Lloyd passes run, fast and slow stage */
  int64_t rows[2];       /* rows processed by those passes' assignment kernels */
  double assign_ms[2];   /* summed duration of the assignment kernels */
  double pass_ms[2];     /* summed duration of whole passes (assign through stop decision) */
} km_prof;

km_status kmeans_profile_begin(void);
km_status kmeans_profile_end(km_prof* out);

/*
 * Measured roofline denominators (beside the datasheet peaks), timed with HIP
 * events on `stream` (hipStream_t or NULL) after one untimed launch:
 *   km_probe_stream_read: read `bytes` (>= 16) of the 16-byte aligned DEVICE
 *     buffer `buf` `reps` times with 16-byte loads; *gbps = bytes read per
 *     second / 1e9;
 *   km_probe_mfma_bf16: two waves per SIMD on every CU, each `iters` rounds of
 *     four independent 32x32x16 BF16 MFMAs (FP32 accumulation), no memory
 *     traffic; *tflops = 2 * 32 * 32 * 16 flops per MFMA per second / 1e12.
 */
km_status km_probe_stream_read(const void* buf, size_t bytes, int32_t reps, double* gbps,
                               void* stream);
km_status km_probe_mfma_bf16(int32_t iters, double* tflops, void* stream);

/* ---------------------------------------------------------------------------
 * Many independent problems at once.  Each request is the two-stage method of
 * kmeans_fit on its own data; the passes of all requests advance together,
 * one launch per kernel for all of them (a batched pass), so that many small
 * problems share the GPU instead of each paying its own launches.  FP32 data,
 * and BF16 data with d <= 16, are scored in FP32 with the same certified error
 * bound and FP64 check as kmeans_fit's FP32 kernels; BF16 data with
 * 16 < d <= 128 and k <= 256 on BF16 matrix cores against -2c kept as two BF16
 * parts, with a certified band and FP64 decisions among the candidates inside
 * it.  Labels equal the FP64 argmin except at FP64 ties.  Cluster sums are
 * exact 64-bit integers; d <= 128.  The FP32 kernel's register tile (points
 * per thread, centers per LDS tile) comes from a built-in autotuner, measured
 * once per (dtype, d bucket, k bucket) and cached for the process.
 * ------------------------------------------------------------------------- */
typedef struct {
  const void* X;          /* n*d elements, row-major: device memory, or host memory with */
  int32_t x_on_host;      /*   x_on_host = 1 (serving only; the server copies it)         */
  km_dtype dtype;
  int64_t n;
  int32_t d;
  int32_t k;
  double subset_frac;     /* as kmeans_fit */
  uint64_t seed;
  int32_t max_iter[2];    /* fast, slow stage */
  double tol[2];
  float* centers_out;     /* DEVICE k*d FP32, written when the problem completes */
  int32_t* labels_out;    /* DEVICE n int32, or NULL */
} km_request;

typedef struct {
  km_status status;       /* KM_OK, or the problem's own error (others still complete) */
  km_info info;           /* seconds[] and fp64_pairs are not filled by the batched path */
  double queue_seconds;   /* serving: submit -> admission */
  double run_seconds;     /* admission (or call start) -> results in place */
} km_result;

/* Fits count problems.  X, centers_out and labels_out are device pointers
   (x_on_host must be 0).  results: host, count entries.  Returns KM_OK when
   every problem was attempted; per-problem errors are in results[i].status.
   Blocks until all results are in place.  stream: hipStream_t or NULL.
   Passes run in chunks of up to 8 between host synchronisations, as in the
   server (passes_per_sync below). */
km_status kmeans_fit_batch(const km_request* reqs, int32_t count, km_result* results,
                           void* stream);

/* The autotuner's choice for a problem shape: points per thread of the
   batched assignment and centers per LDS tile (a problem with fewer centers
   uses k of them).  Tunes on first use of the (dtype, d, k) bucket. */
km_status km_tune_query(km_dtype dtype, int32_t d, int32_t k, int32_t* points_per_thread,
                        int32_t* centers_per_tile);

/* ---------------------------------------------------------------------------
 * Serving.  A server owns a scheduler thread and a HIP stream on the device
 * current at creation.  Submitted problems wait in a queue until their device
 * footprint (a copy of X, centers, labels, sums and sampling buffers) fits in
 * the budget next to the admitted ones; admitted problems advance together in
 * batched passes, and problems that arrive while others run join at the next
 * pass (continuous batching).  Results are bit-identical to the same request
 * run alone (exact sums, fixed-order J).
 * ------------------------------------------------------------------------- */
typedef struct {
  size_t hbm_budget_bytes;  /* device memory for admitted problems (0: 3/4 of free memory) */
  int32_t max_active;       /* problems advanced together, <= 8192 (0: 4096) */
  int32_t max_pending;      /* submitted, not yet admitted (0: 1 << 20); beyond: KM_EBUSY */
  int32_t use_graphs;       /* 1: replay captured HIP graphs of the batched pass */
  /* Batched passes run back to back between two host synchronisations (0: 4,
     at most 16).  A chunk never holds more passes than any admitted problem
     may still need to reach its stage's max_iter; a problem whose stage stops
     earlier (tol) is skipped by the device for the rest of the chunk.  New
     problems join, and finished ones leave, between chunks. */
  int32_t passes_per_sync;
} km_server_cfg;

typedef struct {
  int64_t submitted, admitted, completed, failed;
  int64_t rounds;              /* batched passes launched */
  int64_t active, pending;     /* now */
  size_t bytes_in_use, peak_bytes;
  int64_t peak_active;
  int64_t syncs;               /* host synchronisations: chunks of passes run */
} km_server_counters;

typedef struct km_server km_server;

km_status km_server_create(const km_server_cfg* cfg, km_server** out);
/* Queues a copy of the request and returns at once with a ticket.  The server
   copies X into its own device buffer when it admits the problem, so X (host or
   device) and the output pointers must stay valid until km_server_wait returns
   for the ticket. */
km_status km_server_submit(km_server* srv, const km_request* req, uint64_t* ticket);
/* Waits up to timeout_us (< 0: forever) for the ticket's result; KM_ETIMEOUT
   leaves it pending, KM_ENOTFOUND for an unknown or already collected ticket.
   Admission goes by arrival order, except that a problem which does not fit
   yet lets later ones that fit go first, at most 64 admission rounds in a
   row; then the queue waits for it. */
km_status km_server_wait(km_server* srv, uint64_t ticket, km_result* out, int64_t timeout_us);
km_status km_server_stats(km_server* srv, km_server_counters* out);
/* Stops the scheduler; unfinished problems (waiting or running) complete with
   KM_ECANCELLED, and threads blocked in km_server_wait return that status.
   Returns after every such thread has left km_server_wait; the handle is then
   freed, so no call on it may start once destroy has begun. */
km_status km_server_destroy(km_server* srv);

/* Return the device memory the library keeps for reuse between calls. */
km_status kmeans_release_memory(void);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* kmeans_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KMEANS_MI355X_H */
