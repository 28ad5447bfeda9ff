/*
 * FP64 CPU oracle for the two-stage (fast/slow) k-means of Salman, Kecman, Li,
 * Strack and Test, "Fast k-means algorithm clustering" (arXiv 1108.1351).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU library: not a header, not a kernel, not a constant table.
 *
 * Data X is n x d row-major; dtype 0 = FP32, 1 = BF16 bit patterns (uint16),
 * 2 = FP64.  Every element is widened exactly to FP64 and all arithmetic is
 * FP64 in the plain order the method states.
 */
#ifndef KMEANS_ORACLE_H
#define KMEANS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t iters[2];     /* assign+update passes per stage (fast, slow), incl. the pass that met tol */
  int32_t converged[2]; /* 1 if the stage stopped on shift < tol */
  int32_t empty[2];     /* clusters with no member in the last pass of each stage */
  int64_t m;            /* fast-stage subset size */
  double J;             /* sum over all n points of the squared distance to the nearest returned center */
  double J_stage1;      /* J of the last fast-stage pass, over the subset */
  int64_t dist_evals;   /* k*(m*iters[0] + n*iters[1]) + k*n */
  double shift[2];      /* last max center shift of each stage */
} oracle_info;

/* SplitMix64 output number i+1 for a generator seeded with `seed`: the key of point i. */
uint64_t oracle_key(uint64_t seed, int64_t i);

/* m = min(n, max(k, floor(f*n + 0.5))). */
int64_t oracle_subset_size(int64_t n, int32_t k, double f);

/* The m points with the smallest (key, index) pairs, ascending by index, and the k
   smallest of them ordered by (key, index): the initial centers' rows. */
int oracle_select(int64_t n, int64_t m, int32_t k, uint64_t seed, int64_t* subset_idx,
                  int64_t* init_idx);

/* Nearest center (lowest index on ties), best and second-best squared distance. */
int oracle_assign(const void* X, int32_t dtype, int64_t n, int32_t d, const double* C, int32_t k,
                  int32_t* labels, double* D1, double* D2);

/* One Lloyd pass over n rows from centers C: labels, per-cluster sums S (k*d) and
   counts N (k), J (sum of nearest squared distances), new centers, max shift,
   number of empty clusters (which keep their previous center). */
int oracle_step(const void* Y, int32_t dtype, int64_t n, int32_t d, const double* C, int32_t k,
                int32_t* labels, double* S, int64_t* N, double* J, double* Cnew, double* shift,
                int32_t* empty);

/* The whole two-stage method.  max_iter and tol are per stage (fast, slow).
   init_centers (optional, k*d FP64) replaces the sampled initial centers;
   skip_stage1 = 1 runs the slow stage only ("normal" k-means).  Histories
   (optional, max_iter[s] entries each) receive J and shift of every pass. */
int oracle_fit(const void* X, int32_t dtype, int64_t n, int32_t d, int32_t k, double subset_frac,
               uint64_t seed, const int32_t* max_iter, const double* tol,
               const double* init_centers, int32_t skip_stage1, double* centers_out,
               int32_t* labels_out, oracle_info* info, double* J_hist0, double* shift_hist0,
               double* J_hist1, double* shift_hist1);

/* oracle_step with the optional empty-cluster re-seeding (reseed = 1): after
   the update, the lowest-index empty cluster moves to the point farthest from
   its nearest updated center (lowest index on ties); its movement counts in
   shift.  reseed = 0 is oracle_step. */
int oracle_step_ex(const void* Y, int32_t dtype, int64_t n, int32_t d, const double* C,
                   int32_t k, int32_t reseed, int32_t* labels, double* S, int64_t* N, double* J,
                   double* Cnew, double* shift, int32_t* empty);

/* oracle_fit with re-seeding and the optional per-pass trace of each stage:
   trace_c<s> (max_iter[s] * k * d) receives the centers every pass starts from,
   trace_n<s> (max_iter[s] * k) the cluster sizes the pass finds. */
int oracle_fit_ex(const void* X, int32_t dtype, int64_t n, int32_t d, int32_t k,
                  double subset_frac, uint64_t seed, const int32_t* max_iter, const double* tol,
                  const double* init_centers, int32_t skip_stage1, int32_t reseed,
                  double* centers_out, int32_t* labels_out, oracle_info* info, double* J_hist0,
                  double* shift_hist0, double* J_hist1, double* shift_hist1, double* trace_c0,
                  int64_t* trace_n0, double* trace_c1, int64_t* trace_n1);

void oracle_set_threads(int32_t nthreads);
int32_t oracle_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
