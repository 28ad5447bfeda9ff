/*
 * Seeded synthetic Gaussian-mixture generator.
 *
 * Input fixture for the k-means library and for its FP64 oracle: it produces the
 * data matrix X only and holds none of the clustering arithmetic.  Every value
 * is a pure function of (seed, stream, counter), so any row range can be
 * generated on its own, by any number of threads, with identical bits.
 *
 * Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used as a counter-based hash:
 * the value for counter c of a stream is the SplitMix64 finaliser applied to
 * base(stream) + (c + 1) * golden.  Uniforms take the top 53 bits; normals use
 * the Box-Muller transform on pairs of uniforms (both halves are used).
 *
 * The mixture follows the paper's description of its synthetic validation
 * data (random clusters, section 4): component means and spreads are drawn
 * once per seed, then each point picks a component and adds isotropic
 * Gaussian noise.  Points are generated in FP64 and rounded once to the
 * output type (FP32 or BF16, round-to-nearest-even, no double rounding).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define SYNTH_GOLDEN 0x9E3779B97F4A7C15ULL

typedef struct {
  int32_t d;           /* dimension */
  int32_t ncomp;       /* mixture components */
  int32_t mean_kind;   /* 0: means uniform in [mean_lo, mean_hi]^d; 1: means ~ N(0, mean_sd^2 I) */
  int32_t weight_kind; /* 0: equal weights; 1: Dirichlet(1) weights */
  double mean_lo, mean_hi, mean_sd;
  double sigma_lo, sigma_hi; /* per-component sigma ~ U[sigma_lo, sigma_hi] */
} synth_spec;

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_base(uint64_t seed, uint64_t stream) {
  return sm_mix(seed ^ sm_mix(stream * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL));
}

static inline uint64_t draw_u64(uint64_t base, uint64_t ctr) {
  return sm_mix(base + (ctr + 1ULL) * SYNTH_GOLDEN);
}

/* uniform in the open interval (0, 1) */
static inline double draw_unif(uint64_t base, uint64_t ctr) {
  return ((double)(draw_u64(base, ctr) >> 11) + 0.5) * 0x1.0p-53;
}

static inline double draw_normal(uint64_t base, uint64_t ctr) {
  uint64_t pair = ctr >> 1;
  double u1 = draw_unif(base, 2 * pair), u2 = draw_unif(base, 2 * pair + 1);
  double r = sqrt(-2.0 * log(u1));
  double th = 6.283185307179586476925286766559 * u2;
  return (ctr & 1) ? r * sin(th) : r * cos(th);
}

enum { ST_MEAN = 10, ST_MEAN_N = 11, ST_SIGMA = 12, ST_WEIGHT = 13, ST_COMP = 1, ST_NOISE = 2 };

/* Exported raw stream access, for the generator's own statistical tests. */
uint64_t synth_u64(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return draw_u64(stream_base(seed, stream), ctr);
}
double synth_uniform(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return draw_unif(stream_base(seed, stream), ctr);
}
double synth_normal(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return draw_normal(stream_base(seed, stream), ctr);
}

/* Component parameters: means (ncomp*d), sigmas (ncomp), cumulative weights (ncomp, last == 1). */
int synth_params(const synth_spec* s, uint64_t seed, double* means, double* sigmas, double* cumw) {
  if (!s || s->d < 1 || s->ncomp < 1 || !means || !sigmas || !cumw) return 1;
  uint64_t bm = stream_base(seed, ST_MEAN), bmn = stream_base(seed, ST_MEAN_N);
  uint64_t bs = stream_base(seed, ST_SIGMA), bw = stream_base(seed, ST_WEIGHT);
  for (int64_t c = 0; c < s->ncomp; ++c) {
    for (int64_t t = 0; t < s->d; ++t) {
      uint64_t ctr = (uint64_t)(c * s->d + t);
      means[c * s->d + t] = s->mean_kind == 0
                                ? s->mean_lo + (s->mean_hi - s->mean_lo) * draw_unif(bm, ctr)
                                : s->mean_sd * draw_normal(bmn, ctr);
    }
    sigmas[c] = s->sigma_lo + (s->sigma_hi - s->sigma_lo) * draw_unif(bs, (uint64_t)c);
  }
  double tot = 0.0;
  for (int64_t c = 0; c < s->ncomp; ++c) {
    double w = s->weight_kind == 0 ? 1.0 : -log(draw_unif(bw, (uint64_t)c)); /* Exp(1) */
    tot += w;
    cumw[c] = tot;
  }
  for (int64_t c = 0; c < s->ncomp; ++c) cumw[c] /= tot;
  cumw[s->ncomp - 1] = 1.0;
  return 0;
}

/* Round an FP64 value to the nearest BF16 (ties to even), returning its bits. */
static uint16_t f64_to_bf16(double v) {
  if (v != v) return 0x7FC0;
  if (v == 0.0) return signbit(v) ? 0x8000 : 0x0000;
  int e;
  double m = frexp(fabs(v), &e);        /* |v| = m * 2^e, m in [0.5, 1) */
  double q = nearbyint(ldexp(m, 8));    /* 8 significant bits, RNE */
  float f = (float)ldexp(q, e - 8);     /* exact */
  uint32_t b;
  memcpy(&b, &f, 4);
  uint16_t h = (uint16_t)(b >> 16);
  return (uint16_t)(v < 0 ? (h | 0x8000) : h);
}

/*
 * Rows [row0, row0 + nrows) of X.  dtype: 0 = FP32, 1 = BF16 (uint16 bits), 2 = FP64.
 * comp_out (optional, nrows int32): the component each row was drawn from.
 */
int synth_points(const synth_spec* s, uint64_t seed, const double* means, const double* sigmas,
                 const double* cumw, int64_t row0, int64_t nrows, int32_t dtype, void* out,
                 int32_t* comp_out) {
  if (!s || !means || !sigmas || !cumw || !out || nrows < 0 || row0 < 0) return 1;
  if (dtype < 0 || dtype > 2) return 1;
  const int64_t d = s->d, nc = s->ncomp;
  const uint64_t bc = stream_base(seed, ST_COMP), bn = stream_base(seed, ST_NOISE);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t i = row0 + r;
    double u = draw_unif(bc, (uint64_t)i);
    int64_t lo = 0, hi = nc - 1; /* first c with u < cumw[c] */
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if (u < cumw[mid]) hi = mid; else lo = mid + 1;
    }
    if (comp_out) comp_out[r] = (int32_t)lo;
    const double* mu = means + lo * d;
    double sg = sigmas[lo];
    for (int64_t t = 0; t < d; ++t) {
      double v = mu[t] + sg * draw_normal(bn, (uint64_t)(i * d + t));
      if (dtype == 0) ((float*)out)[r * d + t] = (float)v;
      else if (dtype == 1) ((uint16_t*)out)[r * d + t] = f64_to_bf16(v);
      else ((double*)out)[r * d + t] = v;
    }
  }
  return 0;
}
