// Host driver and C ABI (include/kmeans.h) of the two-stage k-means library.
//
// The two-stage loop follows the Algorithm of section 2 of Salman et al.
// (arXiv 1108.1351): sample the fast-stage subset and the initial centers,
// run Lloyd passes on the subset, then on the whole data from the subset's
// centers, then label every point at the returned centers.  Each stage's pass
// loop is enqueued in chunks of passes whose kernels return at once when the
// device-side state says the stage has stopped; the host reads that state
// after each chunk (one small copy), so it never waits on every pass.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kmeans.h"
#include "host_common.h"
#include "km_internal.h"

using namespace km;

namespace {

struct Layout {
  size_t sel, hist, blk, sub, init_sel, init_key, xs, c64, cw, cn, cnorm, shiftj, emptyj, st,
      jh, sh, slots, jslots, cb16, cnb, queue, qthr, jpart, upart, labels, perm, scnt, stot,
      rstart, tc, tn, fpart, fidx, rqc;
  size_t bytes;
  bool labels_ws;
};

struct Sizes {
  int64_t n, m;
  int32_t d, k;
  int elt;
  bool stage1, sample;
  int32_t hist_len;
  PassPlan p1, p2;
  bool need_labels_ws;
  bool trace, reseed;
};

// per-block partials: the BF16 screen's re-screen kernel has a second set
int64_t blocks_max(const Sizes& z) {
  auto nb = [](const PassPlan& p) { return p.bf16 ? 2 * p.blocks : p.blocks; };
  return std::max(z.stage1 ? nb(z.p1) : 0, nb(z.p2));
}

bool any_bf16(const Sizes& z) { return (z.stage1 && z.p1.bf16) || z.p2.bf16; }
bool any_copy16(const Sizes& z) { return (z.stage1 && copy16(z.p1)) || copy16(z.p2); }
int ks_max(const Sizes& z) { return std::max(z.stage1 ? z.p1.ks : 0, z.p2.ks); }

// Buffers of the sorted update (split paths), sized for the larger stage.
struct SortSizes {
  size_t perm, cnt, tiles, starts;
};

SortSizes sort_sizes(const PassPlan* p1, const PassPlan* p2, int64_t m, int64_t n, int32_t k) {
  SortSizes o{0, 0, 0, 0};
  auto add = [&](const PassPlan* p, int64_t rows) {
    if (!p || p->fused) return;
    const size_t cn = (size_t)k * (size_t)p->sort_chunks;
    o.perm = std::max(o.perm, (size_t)rows);
    o.cnt = std::max(o.cnt, cn);
    o.tiles = std::max(o.tiles, (cn + 2047) / 2048 + 1);
    o.starts = std::max(o.starts, (size_t)k + 1);
  };
  add(p1, m);
  add(p2, n);
  return o;
}

Layout make_layout(const Sizes& z) {
  Layout L{};
  Carver c;
  const int64_t nmax = std::max<int64_t>(z.n, 1);
  L.sel = c.take<SelState>(1);
  L.hist = c.take<unsigned long long>(kSelBins);
  L.blk = c.take<int64_t>((size_t)((nmax + kSelChunk - 1) / kSelChunk + 1));
  L.sub = c.take<int64_t>((size_t)z.m);
  L.init_sel = c.take<int64_t>((size_t)z.k);
  L.init_key = c.take<int64_t>((size_t)z.k);
  L.xs = c.take<unsigned char>(z.stage1 ? (size_t)z.m * z.d * z.elt : 0);
  L.c64 = c.take<double>((size_t)z.k * z.d);
  L.cw = c.take<float>((size_t)z.k * z.d);
  L.cn = c.take<float>((size_t)z.k);
  L.cnorm = c.take<double>((size_t)z.k);
  L.shiftj = c.take<double>((size_t)z.k);
  L.emptyj = c.take<int32_t>((size_t)z.k);
  L.st = c.take<PassState>(1);
  L.jh = c.take<double>((size_t)z.hist_len);
  L.sh = c.take<double>((size_t)z.hist_len);
  const size_t C = (size_t)z.k * (z.d + 1);
  L.slots = c.take<long long>((size_t)kSlots * C);
  L.jslots = c.take<long long>((size_t)kSlots * 2);
  L.cb16 = c.take<uint16_t>(any_copy16(z) ? (size_t)bf16_rows(z.k) * 16 * ks_max(z) : 0);
  L.cnb = c.take<float>((size_t)bf16_rows(z.k));
  L.queue = c.take<uint32_t>(any_bf16(z) ? (size_t)z.n : 0);
  L.qthr = c.take<float>(any_bf16(z) ? (size_t)z.n : 0);
  L.rqc = c.take<int4>(any_bf16(z) ? (size_t)z.n : 0);
  L.jpart = c.take<double>((size_t)blocks_max(z));
  L.upart = c.take<long long>((size_t)blocks_max(z) * 2);
  L.labels_ws = z.need_labels_ws;
  L.labels = c.take<int32_t>(z.need_labels_ws ? (size_t)z.n : 0);
  const SortSizes so = sort_sizes(z.stage1 ? &z.p1 : nullptr, &z.p2, z.m, z.n, z.k);
  L.perm = c.take<uint32_t>(so.perm);
  L.scnt = c.take<long long>(so.cnt);
  L.stot = c.take<long long>(so.tiles);
  L.rstart = c.take<long long>(so.starts);
  // per-pass trace (device copy, brought back at the end) and re-seeding partials
  L.tc = c.take<double>(z.trace ? (size_t)z.hist_len * z.k * z.d : 0);
  L.tn = c.take<long long>(z.trace ? (size_t)z.hist_len * z.k : 0);
  L.fpart = c.take<double>(z.reseed ? (size_t)kFarBlocks : 0);
  L.fidx = c.take<long long>(z.reseed ? (size_t)kFarBlocks : 0);
  L.bytes = c.off;
  return L;
}

// Event timing of the passes (kmeans_profile_begin / _end).
struct Prof {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> free_events;
  km_prof acc;
};
Prof g_prof;

hipEvent_t take_event() {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (!g_prof.free_events.empty()) {
    hipEvent_t e = g_prof.free_events.back();
    g_prof.free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void give_events(std::vector<hipEvent_t>& evs) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (hipEvent_t e : evs)
    if (e) g_prof.free_events.push_back(e);
  evs.clear();
}

bool prof_on() {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  return g_prof.on;
}

// Per thread: two pass-state copies in pinned host memory and an event behind
// each, for reading a chunk's state while the next chunk runs (kept for the
// life of the thread, recreated if the thread moves to another device).
struct StageSync {
  PassState* h = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int dev = -1;
};

StageSync* stage_sync() {
  thread_local StageSync ss;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  if (ss.dev != dev) {
    if (!ss.h && hipHostMalloc(reinterpret_cast<void**>(&ss.h), 2 * sizeof(PassState)) != hipSuccess) {
      ss.h = nullptr;
      return nullptr;
    }
    for (hipEvent_t& e : ss.ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    ss.dev = dev;
  }
  return &ss;
}

struct StageResult {
  int32_t iters = 0, converged = 0, empty = 0;
  double J = 0.0, shift = 0.0;
  int64_t uncertain = 0, pairs = 0;
};

// One stage's Lloyd loop on `rows` rows of Y.  noalloc: the host reads the
// pass state into its own (pageable) memory after each chunk and waits for
// it, with no pinned buffer, event or profiler event to create.
km_status run_stage(PassBufs b, const PassPlan& plan, int32_t max_iter, double tol,
                    hipStream_t s, StageResult* out, int stage, int reseed, bool noalloc) {
  km_status rc = KM_OK;
  PassState hs;
  int32_t launched = 0, chunk = 2;
  const int64_t rows = b.n;
  const bool prof = !noalloc && prof_on();
  StageSync* ss = noalloc ? nullptr : stage_sync();
  int slot = 0, in_flight = 0;
  auto drain = [&]() {  // the copies still in flight land before the buffers are reused
    for (; in_flight > 0; --in_flight) {
      const int old = (slot - in_flight) & 1;
      (void)hipEventSynchronize(ss->ev[old]);
    }
  };
  if (!ss && !noalloc) return fail(KM_EDEVICE, "pinned pass-state buffer or events unavailable");
  std::vector<hipEvent_t> ev;
  if (prof)
    for (int32_t i = 0; i < 3 * max_iter; ++i) ev.push_back(take_event());
  HIP_TRY(stage_reset(b.st, s));
  HIP_TRY(row_stats(b.X, b.dtype, rows, b.d, wants_norms(plan), b.st, s));
  HIP_TRY(stage_begin(b.st, max_iter, tol, rows, b.cnorm, b.k, b.d, plan.fused ? 0 : plan.pg, s,
                      reseed));
  if (copy16(plan)) HIP_TRY(prep_bf16(b.c64, b.k, b.d, plan.ks * 16, b.st, b.cb16, b.cnB, s));
  HIP_TRY(zero_i64(b.slots, (int64_t)kSlots * b.k * (b.d + 1), s));
  HIP_TRY(zero_i64(b.jslots, (int64_t)kSlots * 2, s));
  // Passes go out in chunks (2, 4, 8, then 16), each followed by a copy of the
  // pass state.  One more chunk is queued before the host waits for a chunk's
  // state, so the device does not idle while the host reads it; passes queued
  // after the stop are gated and return at once.
  while (true) {
    if (launched < max_iter && in_flight < 2) {
      const int32_t q = std::min(chunk, max_iter - launched);
      for (int32_t i = 0; i < q; ++i) {
        const int32_t t = launched + i;
        if (prof && ev[3 * t]) HIP_TRY(hipEventRecord(ev[3 * t], s));
        HIP_TRY(pass_assign(b, plan, true, s));
        if (prof && ev[3 * t + 1]) HIP_TRY(hipEventRecord(ev[3 * t + 1], s));
        HIP_TRY(pass_rest(b, plan, true, s));
        if (prof && ev[3 * t + 2]) HIP_TRY(hipEventRecord(ev[3 * t + 2], s));
      }
      launched += q;
      chunk = std::min(chunk * 2, 16);
      if (noalloc) {
        HIP_TRY(hipMemcpyAsync(&hs, b.st, sizeof(PassState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hs.nonfinite) {
          rc = fail(KM_EINVAL, "X contains NaN or Inf");
          goto done;
        }
        if (hs.done || launched >= max_iter) break;
        continue;
      }
      HIP_TRY(hipMemcpyAsync(&ss->h[slot], b.st, sizeof(PassState), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipEventRecord(ss->ev[slot], s));
      slot ^= 1;
      ++in_flight;
      continue;
    }
    if (in_flight == 0) break;  // every pass ran and its state was read
    const int old = (slot - in_flight) & 1;
    const hipError_t e = hipEventSynchronize(ss->ev[old]);
    --in_flight;
    if (e != hipSuccess) {
      rc = fail(KM_EDEVICE, "hipEventSynchronize failed: %s", hipGetErrorString(e));
      goto done;
    }
    hs = ss->h[old];
    if (hs.nonfinite) {
      rc = fail(KM_EINVAL, "X contains NaN or Inf");
      goto done;
    }
    if (hs.done) break;
  }
  drain();
  out->iters = hs.iter;
  out->converged = hs.converged;
  out->empty = hs.empty;
  out->J = hs.J;
  out->shift = hs.shift;
  out->uncertain = hs.uncertain;
  out->pairs = hs.pairs;
  if (prof) {
    // only the first hs.iter passes ran; later ones returned at once
    double a = 0.0, p = 0.0;
    bool ok = true;
    for (int32_t t = 0; t < hs.iter && ok; ++t) {
      float ea = 0.f, ep = 0.f;
      ok = ev[3 * t] && ev[3 * t + 1] && ev[3 * t + 2] &&
           hipEventElapsedTime(&ea, ev[3 * t], ev[3 * t + 1]) == hipSuccess &&
           hipEventElapsedTime(&ep, ev[3 * t], ev[3 * t + 2]) == hipSuccess;
      a += ea;
      p += ep;
    }
    if (ok) {
      std::lock_guard<std::mutex> lk(g_prof.mu);
      g_prof.acc.passes[stage] += hs.iter;
      g_prof.acc.rows[stage] += (int64_t)hs.iter * rows;
      g_prof.acc.assign_ms[stage] += a;
      g_prof.acc.pass_ms[stage] += p;
    }
  }
done:
  drain();
  if (!ev.empty()) give_events(ev);
  return rc;
}

}  // namespace

extern "C" {

const char* kmeans_last_error(void) { return g_err.c_str(); }

km_status kmeans_profile_begin(void) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  memset(&g_prof.acc, 0, sizeof g_prof.acc);
  g_prof.on = true;
  return KM_OK;
}

km_status kmeans_profile_end(km_prof* out) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = false;
  if (out) *out = g_prof.acc;
  return KM_OK;
}

km_status kmeans_release_memory(void) {
  g_err.clear();
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (hipMemPool_t p : g_pools)
    if (p) {
      hipError_t e = hipMemPoolTrimTo(p, 0);
      if (e != hipSuccess)
        return fail(KM_EDEVICE, "hipMemPoolTrimTo failed: %s", hipGetErrorString(e));
    }
  return KM_OK;
}

void kmeans_default_options(km_options* opt, int32_t max_iter, double tol) {
  if (!opt) return;
  memset(opt, 0, sizeof *opt);
  opt->dtype = KM_F32;
  opt->precision = KM_PREC_AUTO;
  opt->max_iter[0] = opt->max_iter[1] = max_iter;
  opt->tol[0] = opt->tol[1] = tol;
}

static bool fit_sizes(int64_t n, int32_t d, int32_t k, double f, const km_options* opt,
                      bool labels_given, Sizes* z) {
  if (!valid_common(n, d, k)) return false;
  if (k > n) return !fail(KM_EINVAL, "k (%d) must not exceed n (%lld)", k, (long long)n);
  if (!(f > 0.0 && f <= 1.0)) return !fail(KM_EINVAL, "subset_frac must be in (0, 1]");
  if (opt->dtype != KM_F32 && opt->dtype != KM_BF16) return !fail(KM_EINVAL, "unknown dtype");
  if (opt->precision < KM_PREC_AUTO || opt->precision > KM_PREC_BF16_RERANK)
    return !fail(KM_EINVAL, "unknown precision");
  for (int s = 0; s < 2; ++s) {
    if (opt->max_iter[s] < 1) return !fail(KM_EINVAL, "max_iter must be >= 1");
    if (!(opt->tol[s] >= 0.0)) return !fail(KM_EINVAL, "tol must be >= 0 and not NaN");
  }
  z->n = n;
  z->d = d;
  z->k = k;
  z->m = subset_size(n, k, f);
  z->elt = opt->dtype == KM_F32 ? 4 : 2;
  z->stage1 = !opt->skip_stage1;
  z->sample = !(opt->skip_stage1 && opt->init_centers);
  z->hist_len = opt->max_iter[0] + opt->max_iter[1];
  const size_t lds = device_lds_limit();
  const int dt = opt->dtype == KM_F32 ? 0 : 1;
  z->p1 = plan_pass(z->m, d, k, dt, (int)opt->precision, lds, device_cus());
  z->p2 = plan_pass(n, d, k, dt, (int)opt->precision, lds, device_cus());
  z->need_labels_ws = !labels_given && ((z->stage1 && !z->p1.fused) || !z->p2.fused);
  z->trace = opt->trace_centers || opt->trace_counts;
  z->reseed = opt->reseed != 0;
  if (opt->reseed != 0 && opt->reseed != 1) return !fail(KM_EINVAL, "reseed must be 0 or 1");
  if (!z->p2.fused && n > (int64_t)UINT32_MAX)
    return !fail(KM_EINVAL, "n = %lld rows need the sorted update, which takes n < 2^32",
                 (long long)n);
  return true;
}

size_t kmeans_workspace_bytes(int64_t n, int32_t d, int32_t k, double subset_frac,
                              const km_options* opt) {
  km_options o;
  if (!opt) {
    kmeans_default_options(&o, 1, 0.0);
    opt = &o;
  }
  Sizes z;
  // sized for labels_out == NULL (the larger case)
  if (!fit_sizes(n, d, k, subset_frac, opt, false, &z)) return 0;
  return make_layout(z).bytes;
}

}  // extern "C"

namespace km {

km_status fit_impl(const void* X, int64_t n, int32_t d, int32_t k, double subset_frac,
                   uint64_t seed, const km_options* opt, float* centers_out, int32_t* labels_out,
                   km_info* info, bool noalloc) {
  if (!opt) return fail(KM_EINVAL, "opt must not be NULL");
  if (!X || !centers_out) return fail(KM_EINVAL, "X and centers_out must not be NULL");
  Sizes z;
  if (!fit_sizes(n, d, k, subset_frac, opt, labels_out != nullptr, &z)) return KM_EINVAL;
  if (opt->init_centers)
    for (int64_t e = 0; e < (int64_t)k * d; ++e)
      if (!std::isfinite(opt->init_centers[e])) return fail(KM_EINVAL, "init_centers not finite");
  hipStream_t s = (hipStream_t)opt->stream;
  const Layout L = make_layout(z);
  if (opt->workspace) {
    // a caller workspace must hold what kmeans_workspace_bytes() asks for (sized
    // without labels_out), whatever this call's own layout needs
    Sizes zmax;
    (void)fit_sizes(n, d, k, subset_frac, opt, false, &zmax);
    const size_t need = make_layout(zmax).bytes;
    if (opt->workspace_bytes < need)
      return fail(KM_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed",
                  opt->workspace_bytes, need);
  }
  DevMem mem;
  km_status rc = mem.get(L.bytes, opt->workspace, opt->workspace_bytes, s);
  if (rc != KM_OK) return rc;
  void* base = mem.ptr;
  SelState* sel = at<SelState>(base, L.sel);
  unsigned long long* hist = at<unsigned long long>(base, L.hist);
  int64_t* blk = at<int64_t>(base, L.blk);
  int64_t* sub = at<int64_t>(base, L.sub);
  int64_t* init_sel = at<int64_t>(base, L.init_sel);
  int64_t* init_key = at<int64_t>(base, L.init_key);
  PassState* st = at<PassState>(base, L.st);
  int32_t* lab_scratch = labels_out ? labels_out : (L.labels_ws ? at<int32_t>(base, L.labels) : nullptr);
  StageResult r1, r2;
  PassState hs;
  std::vector<double> jh(z.hist_len), shh(z.hist_len);
  const int dt = opt->dtype == KM_F32 ? 0 : 1;
  const double t0 = now_s();
  double t1 = t0, t2 = t0, t3 = t0;
  PassBufs b{};
  b.dtype = dt;
  b.d = d;
  b.k = k;
  b.c64 = at<double>(base, L.c64);
  b.cw = at<float>(base, L.cw);
  b.cn = at<float>(base, L.cn);
  b.cnorm = at<double>(base, L.cnorm);
  b.shiftj = at<double>(base, L.shiftj);
  b.emptyj = at<int32_t>(base, L.emptyj);
  b.slots = at<long long>(base, L.slots);
  b.jslots = at<long long>(base, L.jslots);
  b.cb16 = at<uint16_t>(base, L.cb16);
  b.cnB = at<float>(base, L.cnb);
  b.queue = at<uint32_t>(base, L.queue);
  b.qthr = at<float>(base, L.qthr);
  b.rq_c = at<int4>(base, L.rqc);
  b.Jpart = at<double>(base, L.jpart);
  b.upart = at<long long>(base, L.upart);
  b.perm = at<uint32_t>(base, L.perm);
  b.scnt = at<long long>(base, L.scnt);
  b.stot = at<long long>(base, L.stot);
  b.rstart = at<long long>(base, L.rstart);
  b.st = st;
  if (z.reseed) {
    b.fpart = at<double>(base, L.fpart);
    b.fidx = at<long long>(base, L.fidx);
  }
  if (opt->check_finite) {
    // all of X, before any pass: the same scan the stage statistics make
    HIP_TRY(stage_reset(st, s));
    HIP_TRY(row_stats(X, dt, n, d, false, st, s));
    HIP_TRY(hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hs.maxabs_bits >= 0x7f800000u) {
      rc = fail(KM_EINVAL, "X contains NaN or Inf");
      goto done;
    }
  }
  HIP_TRY(hipMemsetAsync(hist, 0, sizeof(unsigned long long) * kSelBins, s));

  // ---- fast-stage subset and initial centers ("%per of S_n", "Select X_c")
  if (z.sample) {
    if (z.stage1) {
      HIP_TRY(sel_run(nullptr, n, seed, z.m, sel, hist, blk, sub, s));
      HIP_TRY(sel_run(sub, z.m, seed, k, sel, hist, blk, init_sel, s));
    } else {
      // the k smallest keys overall are the k smallest keys of the subset
      HIP_TRY(sel_run(nullptr, n, seed, k, sel, hist, blk, init_sel, s));
    }
    HIP_TRY(rank_by_key(init_sel, k, seed, init_key, s));
  } else if (z.stage1) {
    HIP_TRY(sel_run(nullptr, n, seed, z.m, sel, hist, blk, sub, s));
  }
  if (opt->init_centers) {
    HIP_TRY(hipMemcpyAsync(b.c64, opt->init_centers, sizeof(double) * k * d,
                           hipMemcpyHostToDevice, s));
  } else {
    HIP_TRY(centers_from_rows(X, n, dt, d, init_key, k, b.c64, s));
  }
  if (z.stage1) HIP_TRY(gather_rows(X, n, dt, d, sub, z.m, at<unsigned char>(base, L.xs), s));
  HIP_TRY(prep_centers(b.c64, k, d, b.cw, b.cn, b.cnorm, s));
  HIP_TRY(hipStreamSynchronize(s));
  t1 = now_s();

  // ---- fast stage on the subset
  if (z.stage1) {
    PassBufs b1 = b;
    b1.X = at<unsigned char>(base, L.xs);
    b1.n = z.m;
    b1.labels = z.p1.fused ? nullptr : lab_scratch;
    b1.J_hist = at<double>(base, L.jh);
    b1.shift_hist = at<double>(base, L.sh);
    if (z.trace) {
      b1.trace_c = at<double>(base, L.tc);
      b1.trace_n = at<long long>(base, L.tn);
    }
    rc = run_stage(b1, z.p1, opt->max_iter[0], opt->tol[0], s, &r1, 0, opt->reseed, noalloc);
    if (rc != KM_OK) goto done;
  }
  t2 = now_s();

  // ---- slow stage on all points, from the fast stage's centers
  {
    PassBufs b2 = b;
    b2.X = X;
    b2.n = n;
    b2.labels = z.p2.fused ? nullptr : lab_scratch;
    b2.J_hist = at<double>(base, L.jh) + opt->max_iter[0];
    b2.shift_hist = at<double>(base, L.sh) + opt->max_iter[0];
    if (z.trace) {
      b2.trace_c = at<double>(base, L.tc) + (size_t)opt->max_iter[0] * k * d;
      b2.trace_n = at<long long>(base, L.tn) + (size_t)opt->max_iter[0] * k;
    }
    rc = run_stage(b2, z.p2, opt->max_iter[1], opt->tol[1], s, &r2, 1, opt->reseed, noalloc);
    if (rc != KM_OK) goto done;
    // ---- labels and J at the returned centers
    b2.labels = z.p2.fused ? labels_out : lab_scratch;
    HIP_TRY(assign_only(b2, z.p2, s));
  }
  HIP_TRY(hipMemcpyAsync(centers_out, b.cw, sizeof(float) * k * d, hipMemcpyDeviceToDevice, s));
  if (opt->centers64_out)
    HIP_TRY(hipMemcpyAsync(opt->centers64_out, b.c64, sizeof(double) * k * d,
                           hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(jh.data(), at<double>(base, L.jh), sizeof(double) * z.hist_len,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(shh.data(), at<double>(base, L.sh), sizeof(double) * z.hist_len,
                         hipMemcpyDeviceToHost, s));
  if (z.trace) {
    // only the rows of passes that ran hold data; the rest are zeroed
    const int run[2] = {r1.iters, r2.iters};
    const size_t kd = (size_t)k * d;
    for (int s2 = 0; s2 < 2; ++s2) {
      const size_t off = s2 == 0 ? 0 : (size_t)opt->max_iter[0];
      const size_t lim = (size_t)opt->max_iter[s2];
      if (opt->trace_centers) {
        if (run[s2] > 0)
          HIP_TRY(hipMemcpyAsync(opt->trace_centers + off * kd, at<double>(base, L.tc) + off * kd,
                                 sizeof(double) * kd * run[s2], hipMemcpyDeviceToHost, s));
        memset(opt->trace_centers + (off + run[s2]) * kd, 0,
               sizeof(double) * kd * (lim - (size_t)run[s2]));
      }
      if (opt->trace_counts) {
        if (run[s2] > 0)
          HIP_TRY(hipMemcpyAsync(opt->trace_counts + off * k, at<long long>(base, L.tn) + off * k,
                                 sizeof(int64_t) * k * run[s2], hipMemcpyDeviceToHost, s));
        memset(opt->trace_counts + (off + run[s2]) * k, 0,
               sizeof(int64_t) * k * (lim - (size_t)run[s2]));
      }
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  t3 = now_s();
  if (!noalloc && prof_on()) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.acc.fits += 1;
  }
  if (info) {
    memset(info, 0, sizeof *info);
    info->iters[0] = r1.iters;
    info->iters[1] = r2.iters;
    info->converged[0] = r1.converged;
    info->converged[1] = r2.converged;
    info->empty[0] = r1.empty;
    info->empty[1] = r2.empty;
    info->m = z.m;
    info->J = hs.J;
    info->J_stage1 = r1.J;
    info->shift[0] = r1.shift;
    info->shift[1] = r2.shift;
    info->dist_evals = (int64_t)k * (z.m * r1.iters + n * r2.iters) + (int64_t)k * n;
    info->uncertain = r1.uncertain + hs.uncertain;
    info->fp64_pairs = r1.pairs + hs.pairs;
    info->seconds[0] = t1 - t0;
    info->seconds[1] = t2 - t1;
    info->seconds[2] = t3 - t2;
  }
  if (opt->J_hist || opt->shift_hist) {
    for (int s2 = 0; s2 < 2; ++s2) {
      const int off = s2 == 0 ? 0 : opt->max_iter[0];
      const int cnt = s2 == 0 ? r1.iters : r2.iters;
      const int lim = s2 == 0 ? opt->max_iter[0] : opt->max_iter[1];
      for (int i = 0; i < lim; ++i) {
        if (opt->J_hist) opt->J_hist[off + i] = i < cnt ? jh[off + i] : 0.0;
        if (opt->shift_hist) opt->shift_hist[off + i] = i < cnt ? shh[off + i] : 0.0;
      }
    }
  }
done:
  if (rc != KM_OK) (void)hipStreamSynchronize(s);
  return rc;
}

}  // namespace km

extern "C" {

km_status kmeans_fit_ex(const void* X, int64_t n, int32_t d, int32_t k, double subset_frac,
                        uint64_t seed, const km_options* opt, float* centers_out,
                        int32_t* labels_out, km_info* info) {
  g_err.clear();
  return fit_impl(X, n, d, k, subset_frac, seed, opt, centers_out, labels_out, info, false);
}

km_status kmeans_fit(const float* X, int64_t n, int32_t d, int32_t k, double subset_frac,
                     uint64_t seed, int32_t max_iter, double tol, float* centers_out,
                     int32_t* labels_out, km_info* info) {
  km_options o;
  kmeans_default_options(&o, max_iter, tol);
  return kmeans_fit_ex(X, n, d, k, subset_frac, seed, &o, centers_out, labels_out, info);
}

km_status km_sample(int64_t n, int64_t m, int32_t k, uint64_t seed, int64_t* subset_idx,
                    int64_t* init_idx, void* stream) {
  g_err.clear();
  if (n < 1 || k < 1 || m < k || m > n)
    return fail(KM_EINVAL, "need 1 <= k <= m <= n (n=%lld m=%lld k=%d)", (long long)n,
                (long long)m, k);
  if (!subset_idx || !init_idx) return fail(KM_EINVAL, "null output pointer");
  hipStream_t s = (hipStream_t)stream;
  Carver c;
  const size_t o_sel = c.take<SelState>(1), o_hist = c.take<unsigned long long>(kSelBins),
               o_blk = c.take<int64_t>((size_t)((n + kSelChunk - 1) / kSelChunk + 1)),
               o_is = c.take<int64_t>((size_t)k);
  DevMem mem;
  km_status rc = mem.get(c.off, nullptr, 0, s);
  if (rc != KM_OK) return rc;
  void* base = mem.ptr;
  HIP_TRY(hipMemsetAsync(at<unsigned char>(base, o_hist), 0, sizeof(unsigned long long) * kSelBins, s));
  HIP_TRY(sel_run(nullptr, n, seed, m, at<SelState>(base, o_sel),
                  at<unsigned long long>(base, o_hist), at<int64_t>(base, o_blk), subset_idx, s));
  HIP_TRY(sel_run(subset_idx, m, seed, k, at<SelState>(base, o_sel),
                  at<unsigned long long>(base, o_hist), at<int64_t>(base, o_blk),
                  at<int64_t>(base, o_is), s));
  HIP_TRY(rank_by_key(at<int64_t>(base, o_is), k, seed, init_idx, s));
  HIP_TRY(hipStreamSynchronize(s));
done:
  return rc;
}

// One pass (update) or a labelling (no update) at centers C.
static km_status one_pass(const void* X, km_dtype dtype, int64_t n, int32_t d, const double* C,
                          int32_t k, km_precision precision, int32_t* labels, double* S,
                          int64_t* N, double* C_new, double* J, double* shift, int32_t* empty,
                          int64_t* uncertain, void* stream, bool update) {
  g_err.clear();
  if (!valid_common(n, d, k)) return KM_EINVAL;
  if (!X || !C) return fail(KM_EINVAL, "X and C must not be NULL");
  if (dtype != KM_F32 && dtype != KM_BF16) return fail(KM_EINVAL, "unknown dtype");
  if (precision < KM_PREC_AUTO || precision > KM_PREC_BF16_RERANK)
    return fail(KM_EINVAL, "unknown precision");
  hipStream_t s = (hipStream_t)stream;
  const PassPlan p = plan_pass(n, d, k, dtype == KM_F32 ? 0 : 1, (int)precision,
                               device_lds_limit(), device_cus());
  const bool lab_ws = !labels && !p.fused;
  if (!p.fused && n > (int64_t)UINT32_MAX)
    return fail(KM_EINVAL, "n = %lld rows need the sorted update, which takes n < 2^32",
                (long long)n);
  Carver c;
  const size_t C_ = (size_t)k * (d + 1);
  const size_t o_c64 = c.take<double>((size_t)k * d), o_cw = c.take<float>((size_t)k * d),
               o_cn = c.take<float>(k), o_cnorm = c.take<double>(k),
               o_sh = c.take<double>(k), o_em = c.take<int32_t>(k),
               o_st = c.take<PassState>(1), o_slots = c.take<long long>((size_t)kSlots * C_),
               o_qs = c.take<long long>((size_t)kSlots * 2),
               o_cb = c.take<uint16_t>(copy16(p) ? (size_t)bf16_rows(k) * 16 * p.ks : 0),
               o_cnb = c.take<float>((size_t)bf16_rows(k)), o_q = c.take<uint32_t>(p.bf16 ? (size_t)n : 0),
               o_qt = c.take<float>(p.bf16 ? (size_t)n : 0),
               o_rqc = c.take<int4>(p.bf16 ? (size_t)n : 0),
               o_jp = c.take<double>((size_t)p.blocks * 2),
               o_up = c.take<long long>((size_t)p.blocks * 4),
               o_lab = c.take<int32_t>(lab_ws ? (size_t)n : 0);
  const SortSizes so = sort_sizes(nullptr, &p, 0, n, k);
  const size_t o_perm = c.take<uint32_t>(so.perm), o_scnt = c.take<long long>(so.cnt),
               o_stot = c.take<long long>(so.tiles), o_rst = c.take<long long>(so.starts);
  DevMem mem;
  km_status rc = mem.get(c.off, nullptr, 0, s);
  if (rc != KM_OK) return rc;
  void* base = mem.ptr;
  PassState hs;
  PassBufs b{};
  b.X = X;
  b.dtype = dtype == KM_F32 ? 0 : 1;
  b.n = n;
  b.d = d;
  b.k = k;
  b.c64 = at<double>(base, o_c64);
  b.cw = at<float>(base, o_cw);
  b.cn = at<float>(base, o_cn);
  b.cnorm = at<double>(base, o_cnorm);
  b.shiftj = at<double>(base, o_sh);
  b.emptyj = at<int32_t>(base, o_em);
  b.slots = at<long long>(base, o_slots);
  b.jslots = at<long long>(base, o_qs);
  b.cb16 = at<uint16_t>(base, o_cb);
  b.cnB = at<float>(base, o_cnb);
  b.queue = at<uint32_t>(base, o_q);
  b.qthr = at<float>(base, o_qt);
  b.rq_c = at<int4>(base, o_rqc);
  b.Jpart = at<double>(base, o_jp);
  b.upart = at<long long>(base, o_up);
  b.labels = labels ? labels : (lab_ws ? at<int32_t>(base, o_lab) : nullptr);
  b.perm = at<uint32_t>(base, o_perm);
  b.scnt = at<long long>(base, o_scnt);
  b.stot = at<long long>(base, o_stot);
  b.rstart = at<long long>(base, o_rst);
  b.st = at<PassState>(base, o_st);
  b.S_out = S;
  b.N_out = N;
  HIP_TRY(hipMemcpyAsync(b.c64, C, sizeof(double) * k * d, hipMemcpyDeviceToDevice, s));
  HIP_TRY(prep_centers(b.c64, k, d, b.cw, b.cn, b.cnorm, s));
  HIP_TRY(stage_reset(b.st, s));
  HIP_TRY(row_stats(X, b.dtype, n, d, wants_norms(p), b.st, s));
  HIP_TRY(stage_begin(b.st, 1, 0.0, n, b.cnorm, k, d, p.fused ? 0 : p.pg, s));
  if (copy16(p)) HIP_TRY(prep_bf16(b.c64, k, d, p.ks * 16, b.st, b.cb16, b.cnB, s));
  HIP_TRY(zero_i64(b.slots, (int64_t)kSlots * k * (d + 1), s));
  HIP_TRY(zero_i64(b.jslots, (int64_t)kSlots * 2, s));
  HIP_TRY(hipMemcpyAsync(&hs, b.st, sizeof hs, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hs.nonfinite) return fail(KM_EINVAL, "X contains NaN or Inf");
  HIP_TRY(lloyd_pass(b, p, update, s));
  if (update && C_new)
    HIP_TRY(hipMemcpyAsync(C_new, b.c64, sizeof(double) * k * d, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(&hs, b.st, sizeof hs, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (J) *J = hs.J;
  if (shift) *shift = hs.shift;
  if (empty) *empty = hs.empty;
  if (uncertain) *uncertain = hs.uncertain;
done:
  return rc;
}

km_status km_step(const void* X, km_dtype dtype, int64_t n, int32_t d, const double* C,
                  int32_t k, km_precision precision, int32_t* labels, double* S, int64_t* N,
                  double* C_new, double* J, double* shift, int32_t* empty, int64_t* uncertain,
                  void* stream) {
  return one_pass(X, dtype, n, d, C, k, precision, labels, S, N, C_new, J, shift, empty,
                  uncertain, stream, true);
}

km_status km_assign(const void* X, km_dtype dtype, int64_t n, int32_t d, const double* C,
                    int32_t k, km_precision precision, int32_t* labels, double* J,
                    int64_t* uncertain, void* stream) {
  return one_pass(X, dtype, n, d, C, k, precision, labels, nullptr, nullptr, nullptr, J, nullptr,
                  nullptr, uncertain, stream, false);
}

}  // extern "C"
