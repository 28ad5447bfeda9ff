/*
 * FP64 CPU oracle for the two-stage (fast/slow) k-means of Salman et al.,
 * "Fast k-means algorithm clustering" (arXiv 1108.1351).
 *
 * TEST INFRASTRUCTURE: plain, slow and meant to be read against the paper.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * What the paper fixes and how it is read here:
 *  - distance: the "modified distance" of the Algorithm (section 2), i.e. the
 *    squared Euclidean distance (x - c)^T (x - c) of eq. (1) without the root;
 *  - assignment: each point gets the cluster of the nearest center (Algorithm);
 *    on equal distances the lowest center index wins (the paper is silent);
 *  - update: new centers are the averages of the points of each cluster
 *    (Algorithm, "Calculate the average"), done after every pass as in Lloyd's
 *    method (section 4.1) and as Table 1 shows row by row; a cluster with no
 *    point keeps its center (the paper only assumes clusters are not empty);
 *  - objective: J of eq. (3), taken as the sum over the points of the squared
 *    distance to the nearest center (the sample form of the expectation);
 *  - stopping: the paper stops a stage on a required accuracy measured as the
 *    movement of the centers (sections 5 and 6); here a stage stops after the
 *    pass whose largest center movement (Euclidean) is below tol, or after
 *    max_iter passes.  The pass that meets tol is counted, as in Table 1 where
 *    the last pass of each stage shows unchanged centers;
 *  - fast stage: a random fraction of the data (Algorithm, "%per of S_n";
 *    section 6 "randomly selected"), m = floor(f*n + 0.5) points clamped to
 *    [k, n], drawn without replacement as the m smallest SplitMix64 keys;
 *    initial centers are k random points of that subset (section 2 and the
 *    Algorithm): the k smallest keys, in key order;
 *  - slow stage: the whole data set starting from the fast stage's centers
 *    (Algorithm, "Use the whole dataset"; corollary of section 4.1);
 *  - output: labels and J over all points at the returned centers;
 *  - optional variant for empty clusters (section 3 names blank clusters as
 *    the risk of small subsets; the paper gives no rule): after the update of
 *    a pass that left clusters empty, the lowest-index empty cluster takes as
 *    its new center the point farthest from its nearest updated center (the
 *    lowest point index among equally far points), and that movement joins the
 *    pass's largest movement.  One cluster per pass;
 *  - optional trace in the form of Table 1 (section 5): for every pass, the
 *    centers it starts from and the number of points of each cluster.
 */
#include "kmeans_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) ---------------------- */
uint64_t oracle_key(uint64_t seed, int64_t i) {
  uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

int64_t oracle_subset_size(int64_t n, int32_t k, double f) {
  int64_t m = (int64_t)floor(f * (double)n + 0.5);
  if (m < k) m = k;
  if (m > n) m = n;
  return m;
}

typedef struct { uint64_t key; int64_t idx; } kpair;

static int kpair_less(kpair a, kpair b) {
  return a.key < b.key || (a.key == b.key && a.idx < b.idx);
}

static int cmp_kpair(const void* a, const void* b) {
  kpair x = *(const kpair*)a, y = *(const kpair*)b;
  return kpair_less(x, y) ? -1 : (kpair_less(y, x) ? 1 : 0);
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* max-heap on (key, idx): the root is the largest of the m kept pairs */
static void heap_sift_down(kpair* h, int64_t m, int64_t p) {
  for (;;) {
    int64_t l = 2 * p + 1, r = l + 1, big = p;
    if (l < m && kpair_less(h[big], h[l])) big = l;
    if (r < m && kpair_less(h[big], h[r])) big = r;
    if (big == p) return;
    kpair t = h[p]; h[p] = h[big]; h[big] = t;
    p = big;
  }
}

static void heap_sift_up(kpair* h, int64_t p) {
  while (p > 0) {
    int64_t q = (p - 1) / 2;
    if (!kpair_less(h[q], h[p])) return;
    kpair t = h[p]; h[p] = h[q]; h[q] = t;
    p = q;
  }
}

int oracle_select(int64_t n, int64_t m, int32_t k, uint64_t seed, int64_t* subset_idx,
                  int64_t* init_idx) {
  if (n < 1 || m < 1 || m > n || k < 1 || k > m) return 1;
  kpair* h = (kpair*)malloc((size_t)m * sizeof(kpair));
  if (!h) return 2;
  int64_t sz = 0;
  for (int64_t i = 0; i < n; ++i) {
    kpair p = {oracle_key(seed, i), i};
    if (sz < m) {
      h[sz] = p;
      heap_sift_up(h, sz);
      ++sz;
    } else if (kpair_less(p, h[0])) {
      h[0] = p;
      heap_sift_down(h, m, 0);
    }
  }
  qsort(h, (size_t)m, sizeof(kpair), cmp_kpair);
  if (init_idx)
    for (int32_t j = 0; j < k; ++j) init_idx[j] = h[j].idx;
  if (subset_idx) {
    for (int64_t r = 0; r < m; ++r) subset_idx[r] = h[r].idx;
    qsort(subset_idx, (size_t)m, sizeof(int64_t), cmp_i64);
  }
  free(h);
  return 0;
}

/* ---- one element of X, widened exactly ---------------------------------- */
static inline double xval(const void* X, int32_t dtype, int64_t e) {
  if (dtype == 0) return (double)((const float*)X)[e];
  if (dtype == 1) {
    uint32_t b = (uint32_t)((const uint16_t*)X)[e] << 16;
    float f;
    memcpy(&f, &b, 4);
    return (double)f;
  }
  return ((const double*)X)[e];
}

/* ---- nearest center ------------------------------------------------------ */
int oracle_assign(const void* X, int32_t dtype, int64_t n, int32_t d, const double* C, int32_t k,
                  int32_t* labels, double* D1, double* D2) {
  if (!X || !C || n < 0 || d < 1 || k < 1 || dtype < 0 || dtype > 2) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double best = INFINITY, second = INFINITY;
    int32_t bi = 0;
    for (int32_t j = 0; j < k; ++j) {
      double D = 0.0;
      for (int32_t t = 0; t < d; ++t) {
        double diff = xval(X, dtype, i * d + t) - C[(int64_t)j * d + t];
        D += diff * diff;
      }
      if (D < best) {
        second = best;
        best = D;
        bi = j;
      } else if (D < second) {
        second = D;
      }
    }
    if (labels) labels[i] = bi;
    if (D1) D1[i] = best;
    if (D2) D2[i] = second;
  }
  return 0;
}

/* ---- one Lloyd pass -------------------------------------------------------- */
/* Re-seeding of one empty cluster j: the point farthest from its nearest
   center of Cn (squared distance, direct form; lowest index on ties) becomes
   center j.  Returns the center's movement. */
static double reseed_farthest(const void* Y, int32_t dtype, int64_t n, int32_t d, double* Cn,
                              int32_t k, int32_t j) {
  double far = -1.0;
  int64_t fi = 0;
  for (int64_t i = 0; i < n; ++i) {
    double m = INFINITY;
    for (int32_t l = 0; l < k; ++l) {
      double D = 0.0;
      for (int32_t t = 0; t < d; ++t) {
        double diff = xval(Y, dtype, i * d + t) - Cn[(int64_t)l * d + t];
        D += diff * diff;
      }
      if (D < m) m = D;
    }
    if (m > far) {  /* strictly farther: the lowest index wins among equals */
      far = m;
      fi = i;
    }
  }
  double mv = 0.0;
  for (int32_t t = 0; t < d; ++t) {
    double x = xval(Y, dtype, fi * d + t);
    double diff = x - Cn[(int64_t)j * d + t];
    mv += diff * diff;
    Cn[(int64_t)j * d + t] = x;
  }
  return sqrt(mv);
}

int oracle_step(const void* Y, int32_t dtype, int64_t n, int32_t d, const double* C, int32_t k,
                int32_t* labels, double* S, int64_t* N, double* J, double* Cnew, double* shift,
                int32_t* empty) {
  return oracle_step_ex(Y, dtype, n, d, C, k, 0, labels, S, N, J, Cnew, shift, empty);
}

int oracle_step_ex(const void* Y, int32_t dtype, int64_t n, int32_t d, const double* C,
                   int32_t k, int32_t reseed, int32_t* labels, double* S, int64_t* N, double* J,
                   double* Cnew, double* shift, int32_t* empty) {
  if (!Y || !C || n < 1 || d < 1 || k < 1) return 1;
  int32_t* lab = labels ? labels : (int32_t*)malloc((size_t)n * sizeof(int32_t));
  double* D1 = (double*)malloc((size_t)n * sizeof(double));
  double* Sl = S ? S : (double*)malloc((size_t)k * d * sizeof(double));
  int64_t* Nl = N ? N : (int64_t*)malloc((size_t)k * sizeof(int64_t));
  double* Cn = Cnew ? Cnew : (double*)malloc((size_t)k * d * sizeof(double));
  if (!lab || !D1 || !Sl || !Nl || !Cn) return 2;
  oracle_assign(Y, dtype, n, d, C, k, lab, D1, NULL);

  /* sums in point-index order */
  memset(Sl, 0, (size_t)k * d * sizeof(double));
  memset(Nl, 0, (size_t)k * sizeof(int64_t));
  double Jsum = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t j = lab[i];
    Nl[j] += 1;
    for (int32_t t = 0; t < d; ++t) Sl[(int64_t)j * d + t] += xval(Y, dtype, i * d + t);
    Jsum += D1[i];
  }
  /* averages; an empty cluster keeps its center */
  double mx = 0.0;
  int32_t ne = 0;
  for (int32_t j = 0; j < k; ++j) {
    double mv = 0.0;
    for (int32_t t = 0; t < d; ++t) {
      int64_t e = (int64_t)j * d + t;
      double c = Nl[j] > 0 ? Sl[e] / (double)Nl[j] : C[e];
      double diff = c - C[e];
      mv += diff * diff;
      Cn[e] = c;
    }
    if (Nl[j] == 0) ++ne;
    double mvr = sqrt(mv);
    if (mvr > mx) mx = mvr;
  }
  if (reseed && ne > 0) {
    int32_t je = 0;
    while (Nl[je] != 0) ++je;
    double mvr = reseed_farthest(Y, dtype, n, d, Cn, k, je);
    if (mvr > mx) mx = mvr;
  }
  if (J) *J = Jsum;
  if (shift) *shift = mx;
  if (empty) *empty = ne;
  if (!labels) free(lab);
  free(D1);
  if (!S) free(Sl);
  if (!N) free(Nl);
  if (!Cnew) free(Cn);
  return 0;
}

/* One stage: passes until the largest center movement is below tol or max_iter. */
static int run_stage(const void* Y, int32_t dtype, int64_t n, int32_t d, int32_t k, double* C,
                     int32_t max_iter, double tol, int32_t reseed, int32_t* iters,
                     int32_t* converged, int32_t* empty, double* Jlast, double* shlast,
                     double* Jh, double* Sh, double* Tc, int64_t* Tn) {
  double* Cn = (double*)malloc((size_t)k * d * sizeof(double));
  int64_t* Nv = (int64_t*)malloc((size_t)k * sizeof(int64_t));
  if (!Cn || !Nv) return 2;
  int32_t t = 0, conv = 0, ne = 0;
  double Jv = 0.0, sh = 0.0;
  while (t < max_iter) {
    if (Tc) memcpy(Tc + (size_t)t * k * d, C, (size_t)k * d * sizeof(double));
    int rc = oracle_step_ex(Y, dtype, n, d, C, k, reseed, NULL, NULL, Nv, &Jv, Cn, &sh, &ne);
    if (rc) { free(Cn); free(Nv); return rc; }
    if (Tn) memcpy(Tn + (size_t)t * k, Nv, (size_t)k * sizeof(int64_t));
    memcpy(C, Cn, (size_t)k * d * sizeof(double));
    if (Jh) Jh[t] = Jv;
    if (Sh) Sh[t] = sh;
    ++t;
    if (sh < tol) { conv = 1; break; }
  }
  *iters = t;
  *converged = conv;
  *empty = ne;
  *Jlast = Jv;
  *shlast = sh;
  free(Cn);
  free(Nv);
  return 0;
}

int oracle_fit(const void* X, int32_t dtype, int64_t n, int32_t d, int32_t k, double subset_frac,
               uint64_t seed, const int32_t* max_iter, const double* tol,
               const double* init_centers, int32_t skip_stage1, double* centers_out,
               int32_t* labels_out, oracle_info* info, double* J_hist0, double* shift_hist0,
               double* J_hist1, double* shift_hist1) {
  return oracle_fit_ex(X, dtype, n, d, k, subset_frac, seed, max_iter, tol, init_centers,
                       skip_stage1, 0, centers_out, labels_out, info, J_hist0, shift_hist0,
                       J_hist1, shift_hist1, NULL, NULL, NULL, NULL);
}

int oracle_fit_ex(const void* X, int32_t dtype, int64_t n, int32_t d, int32_t k,
                  double subset_frac, uint64_t seed, const int32_t* max_iter, const double* tol,
                  const double* init_centers, int32_t skip_stage1, int32_t reseed,
                  double* centers_out, int32_t* labels_out, oracle_info* info, double* J_hist0,
                  double* shift_hist0, double* J_hist1, double* shift_hist1, double* trace_c0,
                  int64_t* trace_n0, double* trace_c1, int64_t* trace_n1) {
  if (!X || !max_iter || !tol || !centers_out || !info) return 1;
  if (n < 1 || d < 1 || k < 1 || k > n || dtype < 0 || dtype > 2) return 1;
  if (!(subset_frac > 0.0 && subset_frac <= 1.0)) return 1;
  if (max_iter[0] < 1 || max_iter[1] < 1 || !(tol[0] >= 0.0) || !(tol[1] >= 0.0)) return 1;
  memset(info, 0, sizeof(*info));
  int64_t m = oracle_subset_size(n, k, subset_frac);
  info->m = m;
  int64_t* sub = (int64_t*)malloc((size_t)m * sizeof(int64_t));
  int64_t* ini = (int64_t*)malloc((size_t)k * sizeof(int64_t));
  double* C = (double*)malloc((size_t)k * d * sizeof(double));
  if (!sub || !ini || !C) return 2;
  int rc = oracle_select(n, m, k, seed, sub, ini);
  if (rc) return rc;
  for (int32_t j = 0; j < k; ++j)
    for (int32_t t = 0; t < d; ++t)
      C[(int64_t)j * d + t] = init_centers ? init_centers[(int64_t)j * d + t]
                                           : xval(X, dtype, ini[j] * d + t);
  double Jv, sh;
  if (!skip_stage1) {
    /* fast stage on the subset rows, gathered in index order */
    double* Y = (double*)malloc((size_t)m * d * sizeof(double));
    if (!Y) return 2;
    for (int64_t r = 0; r < m; ++r)
      for (int32_t t = 0; t < d; ++t) Y[r * d + t] = xval(X, dtype, sub[r] * d + t);
    rc = run_stage(Y, 2, m, d, k, C, max_iter[0], tol[0], reseed, &info->iters[0],
                   &info->converged[0], &info->empty[0], &Jv, &sh, J_hist0, shift_hist0,
                   trace_c0, trace_n0);
    free(Y);
    if (rc) return rc;
    info->J_stage1 = Jv;
    info->shift[0] = sh;
  }
  /* slow stage on the whole data, from the fast stage's centers */
  rc = run_stage(X, dtype, n, d, k, C, max_iter[1], tol[1], reseed, &info->iters[1],
                 &info->converged[1], &info->empty[1], &Jv, &sh, J_hist1, shift_hist1, trace_c1,
                 trace_n1);
  if (rc) return rc;
  info->shift[1] = sh;
  /* labels and J at the returned centers */
  int32_t* lab = labels_out ? labels_out : (int32_t*)malloc((size_t)n * sizeof(int32_t));
  double* D1 = (double*)malloc((size_t)n * sizeof(double));
  if (!lab || !D1) return 2;
  oracle_assign(X, dtype, n, d, C, k, lab, D1, NULL);
  double Jsum = 0.0;
  for (int64_t i = 0; i < n; ++i) Jsum += D1[i];
  info->J = Jsum;
  info->dist_evals = (int64_t)k * (m * info->iters[0] + n * info->iters[1]) + (int64_t)k * n;
  memcpy(centers_out, C, (size_t)k * d * sizeof(double));
  if (!labels_out) free(lab);
  free(D1);
  free(sub);
  free(ini);
  free(C);
  return 0;
}

void oracle_set_threads(int32_t nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int32_t oracle_get_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}
