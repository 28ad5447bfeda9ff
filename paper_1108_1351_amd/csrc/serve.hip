// Many independent two-stage k-means problems at once: the batched pass
// engine, its autotuner, kmeans_fit_batch and the serving loop (km_server_*).
//
// Every admitted problem runs the method of section 2 of Salman et al.
// (arXiv 1108.1351) on its own data -- sampling, Lloyd passes on the subset,
// Lloyd passes on all points, final labels -- but the passes of all problems
// advance together: one batched pass is a launch of the assignment kernel per
// shape (the FP32 kernel per register tile, the BF16 screen per K-step count),
// one cluster-sum launch and one finalize launch for every problem.  Chunks of
// such passes are replayed from captured HIP graphs; problems move between
// stages on the host between chunks, from a compact status array copied back
// per chunk (a problem whose stage ends inside a chunk is skipped by the
// device until the chunk ends).
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>

#include "host_common.h"

using namespace km;

namespace {

constexpr int kMaxShapes = 16;        // register-tile shapes live in one engine
constexpr int kTableCap = 8192;       // problems advanced together
constexpr size_t kSumsLds = 32768;    // LDS for privatised cluster sums in the batched kernel
constexpr int kFinalizeBlocks = 1024;
constexpr int kMaxChunk = 16;         // passes between two host synchronisations

// ------------------------------------------------------------------ autotuner
struct TuneKey {
  int dtype, dmax, kb;
  bool operator<(const TuneKey& o) const {
    return std::tie(dtype, dmax, kb) < std::tie(o.dtype, o.dmax, o.kb);
  }
};
struct TuneVal {
  int ppt = 1, ktile = 64;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

int k_bucket(int32_t k) {
  int b = 8;
  while (b < k && b < (1 << 20)) b <<= 1;
  return b;
}

std::vector<int> ppt_choices(int dmax) {
  if (dmax <= 8) return {2, 4};
  if (dmax == 16) return {1, 2};
  return {1};
}

size_t batch_lds(int dmax, int ktile) {
  return ((size_t)ktile * (dmax + 1) * 4 + 15) / 16 * 16 + kSumsLds;
}

// Times the batched assignment of one synthetic problem (uniform data, d =
// dmax, k = the bucket) for each candidate tile and keeps the fastest.
km_status tune(int dtype, int dmax, int kb, hipStream_t s, TuneVal* out) {
  km_status rc = KM_OK;
  const int64_t n = 1 << 16;
  const int d = dmax, k = kb;
  std::vector<std::pair<int, int>> cands;
  for (int ppt : ppt_choices(dmax))
    for (int kt : {32, 64, 128, 256}) {
      if (kt > std::max(32, k)) continue;
      if (batch_lds(dmax, kt) > device_lds_limit()) continue;
      cands.push_back({ppt, kt});
    }
  if (cands.empty()) cands.push_back({ppt_choices(dmax)[0], 32});
  Carver c;
  const size_t oX = c.take<float>((size_t)n * d), oC = c.take<double>((size_t)k * d),
               oCw = c.take<float>((size_t)k * d), oCn = c.take<float>(k),
               oCnorm = c.take<double>(k), oSt = c.take<PassState>(1),
               oLab = c.take<int32_t>(n), oJ = c.take<double>(n), oU = c.take<long long>(2 * n),
               oHd = c.take<BatchHead>(1), oBi = c.take<BatchInst>(1);
  DevMem mem;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float best = INFINITY;
  TuneVal bestv{cands[0].first, cands[0].second};
  rc = mem.get(c.off, nullptr, 0, s);
  if (rc != KM_OK) return rc;
  {
    void* base = mem.ptr;
    float* Xf = at<float>(base, oX);
    double* c64 = at<double>(base, oC);
    PassState* st = at<PassState>(base, oSt);
    HIP_TRY(fill_uniform(Xf, dtype, n * d, 17, s));  // the problem's element type
    HIP_TRY(fill_uniform(c64, 2, (int64_t)k * d, 29, s));
    HIP_TRY(prep_centers(c64, k, d, at<float>(base, oCw), at<float>(base, oCn),
                         at<double>(base, oCnorm), s));
    HIP_TRY(stage_reset(st, s));
    HIP_TRY(row_stats(Xf, dtype, n, d, false, st, s));
    HIP_TRY(stage_begin(st, 1, 0.0, n, at<double>(base, oCnorm), k, d, 0, s));
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    for (auto [ppt, kt] : cands) {
      const int64_t tp = 256LL * ppt;
      BatchHead hh{1, 0, (n + tp - 1) / tp, k};
      BatchInst bb{};
      bb.X = Xf;
      bb.n = n;
      bb.d = d;
      bb.k = k;
      bb.dtype = dtype;
      bb.mode = 2;
      bb.lds_sums = 0;
      bb.nslots = 1;
      bb.ktile = kt;
      bb.unit0 = 0;
      bb.units = hh.units;
      bb.tile_pts = tp;
      bb.center0 = 0;
      bb.c64 = c64;
      bb.cw = at<float>(base, oCw);
      bb.cn = at<float>(base, oCn);
      bb.cnorm = at<double>(base, oCnorm);
      bb.st = st;
      bb.labels = at<int32_t>(base, oLab);
      bb.Jpart = at<double>(base, oJ);
      bb.upart = at<long long>(base, oU);
      HIP_TRY(hipMemcpyAsync(at<BatchHead>(base, oHd), &hh, sizeof hh, hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(at<BatchInst>(base, oBi), &bb, sizeof bb, hipMemcpyHostToDevice, s));
      BatchShape sh{dtype, dmax, ppt, batch_lds(dmax, kt), 0};
      sh.blocks = (int)std::max<int64_t>(
          1, std::min<int64_t>(hh.units, batch_resident_blocks(dtype, dmax, ppt, sh.lds,
                                                                device_cus())));
      HIP_TRY(batch_assign(at<BatchHead>(base, oHd), at<BatchInst>(base, oBi), sh, s));  // warm
      HIP_TRY(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r)
        HIP_TRY(batch_assign(at<BatchHead>(base, oHd), at<BatchInst>(base, oBi), sh, s));
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        bestv = {ppt, kt};
      }
    }
  }
  *out = bestv;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  return rc;
}

km_status tuned(int dtype, int dmax, int32_t k, hipStream_t s, TuneVal* out) {
  const TuneKey key{dtype, dmax, k_bucket(k)};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      *out = it->second;
      return KM_OK;
    }
  }
  TuneVal v;
  km_status rc = tune(dtype, dmax, key.kb, s, &v);
  if (rc != KM_OK) return rc;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = v;
  *out = v;
  return KM_OK;
}

// ------------------------------------------------------------------ problems
struct Job {
  km_request rq{};
  uint64_t ticket = 0;
  int phase = 0;  // 0 waiting, 1 fast stage, 2 slow stage, 3 labelling, 4 finished
  km_status status = KM_OK;
  std::string err;
  km_info info{};
  int64_t m = 0;
  int dmax = 0, shape = -1;
  TuneVal tv;
  size_t bytes = 0;
  DevMem mem;
  bool copy_x = false;
  const void* X = nullptr;  // the data the passes read (the caller's or the copy)
  // workspace
  SelState* sel = nullptr;
  unsigned long long* hist = nullptr;
  int64_t *blk = nullptr, *sub = nullptr, *init_sel = nullptr, *init_key = nullptr;
  void* xs = nullptr;
  double *c64 = nullptr, *cnorm = nullptr, *shiftj = nullptr;
  float *cw = nullptr, *cn = nullptr;
  int32_t *emptyj = nullptr, *labels = nullptr;
  PassState* st = nullptr;
  long long* slots = nullptr;
  double* jpart = nullptr;
  long long* upart = nullptr;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int64_t unc2 = 0;  // FP64 checks counted by the slow stage's passes
  int64_t passed_over = 0;  // admission rounds in which later problems went ahead
  int32_t iter_now = 0;     // passes run in the current stage, from the last status
  // BF16 data with 16 < d <= 128 and k <= 256: the batched BF16 screen (its K
  // steps), with the tiled BF16 copy of -2c and ||c||^2 + B
  int screen = 0;
  uint16_t* cb16 = nullptr;
  uint16_t* cb16lo = nullptr;
  float* cnB = nullptr;
};

// Admission rounds a waiting problem may be passed by later, smaller ones;
// beyond this the queue holds behind it until it fits (no starvation).
constexpr int64_t kMaxPassOver = 64;

int elt_size(km_dtype t) { return t == KM_F32 ? 4 : 2; }

bool valid_request(const km_request& r, bool serving) {
  if (!valid_common(r.n, r.d, r.k)) return false;
  if (r.dtype != KM_F32 && r.dtype != KM_BF16) return !fail(KM_EINVAL, "unknown dtype");
  if (!r.X || !r.centers_out) return !fail(KM_EINVAL, "X and centers_out must not be NULL");
  if (r.x_on_host && !serving) return !fail(KM_EINVAL, "x_on_host is for serving only");
  if (r.k > r.n) return !fail(KM_EINVAL, "k = %d exceeds n = %lld", r.k, (long long)r.n);
  if (!(r.subset_frac > 0.0 && r.subset_frac <= 1.0))
    return !fail(KM_EINVAL, "subset_frac must lie in (0, 1]");
  for (int s = 0; s < 2; ++s) {
    if (r.max_iter[s] < 1) return !fail(KM_EINVAL, "max_iter must be >= 1");
    if (!(r.tol[s] >= 0.0)) return !fail(KM_EINVAL, "tol must be >= 0 and not NaN");
  }
  if (batch_dmax(r.d) == 0) return !fail(KM_EINVAL, "the batched path takes d <= 128 (got %d)", r.d);
  if ((int64_t)r.k * (r.d + 1) > (1 << 24)) return !fail(KM_EINVAL, "k*(d+1) too large for batching");
  return true;
}

// Device bytes of a problem: sampling, subset copy, centers, sums, labels,
// partials, and (serving) its copy of X.
size_t job_layout(Job& j, void* base) {
  const km_request& r = j.rq;
  const int64_t n = r.n, m = j.m;
  const int32_t d = r.d, k = r.k;
  const int64_t units = (n + 255) / 256;  // tiles of >= 256 points
  Carver c;
  const size_t o_sel = c.take<SelState>(1), o_hist = c.take<unsigned long long>(kSelBins),
               o_blk = c.take<int64_t>((size_t)((n + kSelChunk - 1) / kSelChunk + 1)),
               o_sub = c.take<int64_t>((size_t)m), o_is = c.take<int64_t>(k),
               o_ik = c.take<int64_t>(k), o_xs = c.take<unsigned char>((size_t)m * d * elt_size(r.dtype)),
               o_c64 = c.take<double>((size_t)k * d), o_cw = c.take<float>((size_t)k * d),
               o_cn = c.take<float>(k), o_cnorm = c.take<double>(k), o_sh = c.take<double>(k),
               o_em = c.take<int32_t>(k), o_st = c.take<PassState>(1),
               o_slots = c.take<long long>((size_t)kSlots * k * (d + 1)),
               o_lab = c.take<int32_t>(r.labels_out ? 0 : (size_t)n),
               o_jp = c.take<double>((size_t)units), o_up = c.take<long long>((size_t)units * 2),
               o_x = c.take<unsigned char>(j.copy_x ? (size_t)n * d * elt_size(r.dtype) : 0),
               o_cb = c.take<uint16_t>(j.screen ? (size_t)bf16_rows(k) * 16 * j.screen * 2 : 0),
               o_cnb = c.take<float>(j.screen ? (size_t)bf16_rows(k) : 0);
  if (base) {
    j.sel = at<SelState>(base, o_sel);
    j.hist = at<unsigned long long>(base, o_hist);
    j.blk = at<int64_t>(base, o_blk);
    j.sub = at<int64_t>(base, o_sub);
    j.init_sel = at<int64_t>(base, o_is);
    j.init_key = at<int64_t>(base, o_ik);
    j.xs = at<unsigned char>(base, o_xs);
    j.c64 = at<double>(base, o_c64);
    j.cw = at<float>(base, o_cw);
    j.cn = at<float>(base, o_cn);
    j.cnorm = at<double>(base, o_cnorm);
    j.shiftj = at<double>(base, o_sh);
    j.emptyj = at<int32_t>(base, o_em);
    j.st = at<PassState>(base, o_st);
    j.slots = at<long long>(base, o_slots);
    j.labels = r.labels_out ? r.labels_out : at<int32_t>(base, o_lab);
    j.jpart = at<double>(base, o_jp);
    j.upart = at<long long>(base, o_up);
    j.X = j.copy_x ? (const void*)at<unsigned char>(base, o_x) : r.X;
    j.cb16 = j.screen ? at<uint16_t>(base, o_cb) : nullptr;
    j.cb16lo = j.screen ? j.cb16 + (size_t)bf16_rows(k) * 16 * j.screen : nullptr;
    j.cnB = j.screen ? at<float>(base, o_cnb) : nullptr;
  }
  return c.off;
}

// Puts a problem's stage on the device: row statistics of its data, the stop
// rule, zeroed sums.  stage 1: the subset, stage 2: all points.
km_status begin_stage(Job& j, int stage, hipStream_t s) {
  km_status rc = KM_OK;
  const km_request& r = j.rq;
  const int dt = r.dtype == KM_F32 ? 0 : 1;
  const void* X = stage == 1 ? j.xs : j.X;
  const int64_t rows = stage == 1 ? j.m : r.n;
  HIP_TRY(stage_reset(j.st, s));
  // the screen's score offset needs max ||x||^2 of the stage's rows
  HIP_TRY(row_stats(X, dt, rows, r.d, j.screen != 0, j.st, s));
  HIP_TRY(stage_begin(j.st, r.max_iter[stage - 1], r.tol[stage - 1], rows, j.cnorm, r.k, r.d, 0,
                      s));
  if (j.screen)
    HIP_TRY(prep_bf16(j.c64, r.k, r.d, 16 * j.screen, j.st, j.cb16, j.cnB, s, j.cb16lo));
  HIP_TRY(zero_i64(j.slots, (int64_t)kSlots * r.k * (r.d + 1), s));
  j.phase = stage;
  j.iter_now = 0;
done:
  return rc;
}

// Sampling, initial centers, the subset copy and the first stage.
km_status start_job(Job& j, hipStream_t s) {
  km_status rc = KM_OK;
  const km_request& r = j.rq;
  const int dt = r.dtype == KM_F32 ? 0 : 1;
  if (j.copy_x)
    HIP_TRY(hipMemcpyAsync(const_cast<void*>(j.X), r.X, (size_t)r.n * r.d * elt_size(r.dtype),
                           r.x_on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemsetAsync(j.hist, 0, sizeof(unsigned long long) * kSelBins, s));
  HIP_TRY(sel_run(nullptr, r.n, r.seed, j.m, j.sel, j.hist, j.blk, j.sub, s));
  HIP_TRY(sel_run(j.sub, j.m, r.seed, r.k, j.sel, j.hist, j.blk, j.init_sel, s));
  HIP_TRY(rank_by_key(j.init_sel, r.k, r.seed, j.init_key, s));
  HIP_TRY(centers_from_rows(j.X, r.n, dt, r.d, j.init_key, r.k, j.c64, s));
  HIP_TRY(gather_rows(j.X, r.n, dt, r.d, j.sub, j.m, j.xs, s));
  HIP_TRY(prep_centers(j.c64, r.k, r.d, j.cw, j.cn, j.cnorm, s));
  rc = begin_stage(j, 1, s);
done:
  return rc;
}

// ------------------------------------------------------------------ engine
// The batched pass: per round, the descriptors of the active problems go to
// fixed device tables (one per register-tile shape, one for the finalize and
// status kernels), then the captured launches run and the statuses come back.
class Engine {
 public:
  struct Shape {
    int dtype, dmax, ppt, ktile;
    size_t lds;
    int blocks;
    int screen;  // K steps of the batched BF16 screen, 0 for the FP32 kernel
  };

  explicit Engine(hipStream_t s) : s_(s) {}
  ~Engine() { release(); }

  km_status init() {
    km_status rc = KM_OK;
    const size_t heads = sizeof(BatchHead) * (kMaxShapes + 2);
    const size_t insts = sizeof(BatchInst) * (size_t)kTableCap * (kMaxShapes + 1);
    const size_t stat = sizeof(BatchStatus) * kTableCap;
    bytes_ = heads + insts + stat;
    HIP_TRY(hipMalloc(&dev_, bytes_));
    HIP_TRY(hipHostMalloc(&host_, heads + insts, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(&hstat_, stat, hipHostMallocDefault));
    d_heads_ = static_cast<BatchHead*>(dev_);
    d_insts_ = reinterpret_cast<BatchInst*>(static_cast<char*>(dev_) + heads);
    d_stat_ = reinterpret_cast<BatchStatus*>(static_cast<char*>(dev_) + heads + insts);
    h_heads_ = static_cast<BatchHead*>(host_);
    h_insts_ = reinterpret_cast<BatchInst*>(static_cast<char*>(host_) + heads);
  done:
    return rc;
  }

  // Shape slot for a register tile and LDS center tile (created on first use).
  int shape_of(int dtype, int dmax, int ppt, int ktile, int screen = 0) {
    for (int i = 0; i < (int)shapes_.size(); ++i)
      if (shapes_[i].dtype == dtype && shapes_[i].dmax == dmax && shapes_[i].ppt == ppt &&
          shapes_[i].ktile == ktile && shapes_[i].screen == screen)
        return i;
    if ((int)shapes_.size() >= kMaxShapes) return -1;
    // the screen's LDS is static (center tiles, candidate lists)
    Shape sh{dtype, dmax, ppt, ktile, screen ? 0 : batch_lds(dmax, ktile), 0, screen};
    sh.blocks = (int)std::max<int64_t>(
        1, batch_resident_blocks(dtype, dmax, ppt, sh.lds, device_cus(), screen));
    shapes_.push_back(sh);
    return (int)shapes_.size() - 1;
  }

  // `passes` batched passes for the given problems (each in phase 1, 2 or 3),
  // then their statuses.  A problem whose stage stops inside the chunk keeps its
  // done flag, and the kernels of the later passes skip it.
  km_status round(const std::vector<Job*>& act, bool graphs, int passes,
                  std::vector<BatchStatus>& st) {
    km_status rc = KM_OK;
    const int na = (int)act.size();
    if (na > kTableCap) return fail(KM_EINVAL, "more than %d active problems", kTableCap);
    const int ns = (int)shapes_.size();
    std::vector<int> cnt(ns, 0);
    std::vector<int64_t> units(ns, 0);
    int64_t centers = 0, sunits = 0;
    unsigned mask = 0;
    for (int a = 0; a < na; ++a) {
      Job& j = *act[a];
      const int g = j.shape;
      BatchInst b{};
      b.X = j.phase == 1 ? j.xs : j.X;
      b.n = j.phase == 1 ? j.m : j.rq.n;
      b.d = j.rq.d;
      b.k = j.rq.k;
      b.dtype = j.rq.dtype == KM_F32 ? 0 : 1;
      b.mode = j.phase == 3 ? 2 : 1;
      // the BF16 screen keeps its LDS for the center tiles: its sums always
      // go through k_batch_sums
      b.lds_sums = !j.screen && (size_t)j.rq.k * (j.rq.d + 1) * 8 <= kSumsLds ? 1 : 0;
      b.cb16 = j.cb16;
      b.cb16lo = j.cb16lo;
      b.cnB = j.cnB;
      b.kd16 = 16 * j.screen;
      b.ktile = j.tv.ktile;
      b.tile_pts = 256LL * shapes_[g].ppt;
      b.unit0 = units[g];
      b.units = (b.n + b.tile_pts - 1) / b.tile_pts;
      b.center0 = centers;
      b.c64 = j.c64;
      b.cw = j.cw;
      b.cn = j.cn;
      b.cnorm = j.cnorm;
      b.shiftj = j.shiftj;
      b.emptyj = j.emptyj;
      b.st = j.st;
      b.slots = j.slots;
      b.labels = j.labels;
      b.Jpart = j.jpart;
      b.upart = j.upart;
      // sums too large for the assignment's LDS: ranges of points x centers
      b.skc = (int32_t)std::min<int64_t>(b.k, kBatchSumLds / ((size_t)(b.d + 1) * 8));
      b.sunit0 = sunits;
      b.sunits = b.mode == 1 && !b.lds_sums
                     ? (b.n + kBatchSumPts - 1) / kBatchSumPts * ((b.k + b.skc - 1) / b.skc)
                     : 0;
      sunits += b.sunits;
      {
        // one slot row per writer (tile flushes or point ranges), at most kSlots
        const int64_t writers = b.sunits ? (b.n + kBatchSumPts - 1) / kBatchSumPts : b.units;
        int ns = 1;
        while (ns < kSlots && ns < writers) ns <<= 1;
        b.nslots = ns;
      }
      units[g] += b.units;
      centers += b.k;
      h_insts_[(size_t)g * kTableCap + cnt[g]++] = b;
      h_insts_[(size_t)kMaxShapes * kTableCap + a] = b;
      mask |= 1u << g;
    }
    for (int g = 0; g < ns; ++g) h_heads_[g] = BatchHead{cnt[g], 0, units[g], 0};
    h_heads_[kMaxShapes] = BatchHead{na, 0, 0, centers};
    h_heads_[kMaxShapes + 1] = BatchHead{na, 0, sunits, 0};
    // descriptors: only the used prefix of each table travels
    for (int g = 0; g < ns; ++g)
      if (cnt[g])
        HIP_TRY(hipMemcpyAsync(d_insts_ + (size_t)g * kTableCap, h_insts_ + (size_t)g * kTableCap,
                               sizeof(BatchInst) * cnt[g], hipMemcpyHostToDevice, s_));
    HIP_TRY(hipMemcpyAsync(d_insts_ + (size_t)kMaxShapes * kTableCap,
                           h_insts_ + (size_t)kMaxShapes * kTableCap, sizeof(BatchInst) * na,
                           hipMemcpyHostToDevice, s_));
    HIP_TRY(hipMemcpyAsync(d_heads_, h_heads_, sizeof(BatchHead) * (kMaxShapes + 2),
                           hipMemcpyHostToDevice, s_));
    if (graphs) {
      hipGraphExec_t ex = nullptr;
      rc = graph_for(mask, passes, &ex);
      if (rc != KM_OK) goto done;
      HIP_TRY(hipGraphLaunch(ex, s_));
    } else {
      for (int p = 0; p < passes && rc == KM_OK; ++p) rc = launch(mask);
      if (rc != KM_OK) goto done;
    }
    HIP_TRY(hipMemcpyAsync(hstat_, d_stat_, sizeof(BatchStatus) * na, hipMemcpyDeviceToHost, s_));
    HIP_TRY(hipStreamSynchronize(s_));
    st.assign(hstat_, hstat_ + na);
    rounds_ += passes;
    ++syncs_;
  done:
    return rc;
  }

  int64_t rounds() const { return rounds_; }
  int64_t syncs() const { return syncs_; }
  hipStream_t stream() const { return s_; }

 private:
  km_status launch(unsigned mask) {
    km_status rc = KM_OK;
    for (int g = 0; g < (int)shapes_.size(); ++g) {
      if (!(mask & (1u << g))) continue;
      const Shape& sh = shapes_[g];
      BatchShape bs{sh.dtype, sh.dmax, sh.ppt, sh.lds, sh.blocks, sh.screen};
      HIP_TRY(batch_assign(d_heads_ + g, d_insts_ + (size_t)g * kTableCap, bs, s_));
    }
    HIP_TRY(batch_sums(d_heads_ + kMaxShapes + 1, d_insts_ + (size_t)kMaxShapes * kTableCap,
                       2 * device_cus(), s_));
    HIP_TRY(batch_finalize(d_heads_ + kMaxShapes, d_insts_ + (size_t)kMaxShapes * kTableCap,
                           kFinalizeBlocks, s_));
    HIP_TRY(batch_status(d_heads_ + kMaxShapes, d_insts_ + (size_t)kMaxShapes * kTableCap, d_stat_,
                         s_));
  done:
    return rc;
  }

  // The launches of `passes` rounds for a set of shapes, captured once and replayed.
  km_status graph_for(unsigned mask, int passes, hipGraphExec_t* out) {
    km_status rc = KM_OK;
    const uint64_t key = (uint64_t)mask << 8 | (uint64_t)passes;
    auto it = graphs_.find(key);
    if (it != graphs_.end()) {
      *out = it->second;
      return KM_OK;
    }
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    HIP_TRY(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
    for (int p = 0; p < passes && rc == KM_OK; ++p) rc = launch(mask);
    {
      const hipError_t e = hipStreamEndCapture(s_, &g);
      if (rc != KM_OK) goto done;
      if (e != hipSuccess) {
        rc = fail(KM_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
        goto done;
      }
    }
    HIP_TRY(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    graphs_[key] = ex;
    *out = ex;
  done:
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }

  void release() {
    for (auto& kv : graphs_) (void)hipGraphExecDestroy(kv.second);
    graphs_.clear();
    if (dev_) (void)hipFree(dev_);
    if (host_) (void)hipHostFree(host_);
    if (hstat_) (void)hipHostFree(hstat_);
    dev_ = host_ = nullptr;
    hstat_ = nullptr;
  }

  hipStream_t s_;
  size_t bytes_ = 0;
  void* dev_ = nullptr;
  void* host_ = nullptr;
  BatchStatus* hstat_ = nullptr;
  BatchHead *d_heads_ = nullptr, *h_heads_ = nullptr;
  BatchInst *d_insts_ = nullptr, *h_insts_ = nullptr;
  BatchStatus* d_stat_ = nullptr;
  std::vector<Shape> shapes_;
  std::unordered_map<uint64_t, hipGraphExec_t> graphs_;
  int64_t rounds_ = 0, syncs_ = 0;
};

// Admission of a problem: shape from the autotuner, workspace, the first stage.
km_status admit(Engine& eng, Job& j, hipStream_t s) {
  km_status rc = KM_OK;
  const km_request& r = j.rq;
  const int dt = r.dtype == KM_F32 ? 0 : 1;
  j.dmax = batch_dmax(r.d);
  if (j.screen) {
    // the BF16 screen: 256-point units, no register-tile choice to tune
    j.tv.ppt = 1;
    j.tv.ktile = 32;
  } else {
    rc = tuned(dt, j.dmax, r.k, s, &j.tv);
    if (rc != KM_OK) return rc;
  }
  j.shape = eng.shape_of(dt, j.dmax, j.tv.ppt, j.tv.ktile, j.screen);
  if (j.shape < 0) return fail(KM_EBUSY, "too many register-tile shapes at once");
  rc = j.mem.get(j.bytes, nullptr, 0, s);
  if (rc != KM_OK) return rc;
  job_layout(j, j.mem.ptr);
  return start_job(j, s);
}

// After a round: stage changes and completion.  Returns true when finished.
bool advance(Job& j, const BatchStatus& b, hipStream_t s) {
  const km_request& r = j.rq;
  j.iter_now = b.iter;
  if (b.nonfinite) {
    j.status = fail(KM_EINVAL, "X contains NaN or Inf");
    j.err = g_err;
    j.phase = 4;
    return true;
  }
  if (j.phase == 1 && b.done == 1) {
    j.info.iters[0] = b.iter;
    j.info.converged[0] = b.converged;
    j.info.empty[0] = b.empty;
    j.info.shift[0] = b.shift;
    j.info.J_stage1 = b.J;
    j.info.uncertain += b.uncertain;
    km_status rc = begin_stage(j, 2, s);
    if (rc != KM_OK) {
      j.status = rc;
      j.err = g_err;
      j.phase = 4;
      return true;
    }
  } else if (j.phase == 2 && b.done == 1) {
    j.info.iters[1] = b.iter;
    j.info.converged[1] = b.converged;
    j.info.empty[1] = b.empty;
    j.info.shift[1] = b.shift;
    j.info.uncertain += b.uncertain;
    j.unc2 = b.uncertain;
    j.phase = 3;
  } else if (j.phase == 3 && b.done == 2) {
    j.info.J = b.J;
    j.info.uncertain += b.uncertain - j.unc2;  // the labelling pass adds to the stage's count
    j.info.m = j.m;
    j.info.dist_evals =
        (int64_t)r.k * (j.m * (int64_t)j.info.iters[0] + r.n * (int64_t)j.info.iters[1]) +
        (int64_t)r.k * r.n;
    const hipError_t e = hipMemcpyAsync(r.centers_out, j.cw, sizeof(float) * r.k * r.d,
                                        hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
      j.status = fail(KM_EDEVICE, "copy of the centers failed: %s", hipGetErrorString(e));
      j.err = g_err;
    }
    j.phase = 4;
    return true;
  }
  return false;
}

// Passes for the next chunk: at most `cap`, and no more than any problem may
// still need before its stage reaches max_iter (one for a labelling pass), so
// a problem waits past its stage's end only when tol stops it early.
int chunk_passes(const std::vector<Job*>& act, int cap) {
  int r = std::max(1, std::min(cap, kMaxChunk));
  for (const Job* j : act) {
    const int rem = j->phase == 3 ? 1 : j->rq.max_iter[j->phase - 1] - j->iter_now;
    r = std::min(r, std::max(1, rem));
  }
  return r;
}

void fill_result(const Job& j, km_result* out) {
  memset(out, 0, sizeof *out);
  out->status = j.status;
  out->info = j.info;
  out->queue_seconds = j.t_admit > 0 ? j.t_admit - j.t_submit : 0.0;
  out->run_seconds = j.t_done > 0 && j.t_admit > 0 ? j.t_done - j.t_admit : 0.0;
}

}  // namespace

// ------------------------------------------------------------------ server
struct km_server {
  km_server_cfg cfg{};
  int device = 0;
  hipStream_t s = nullptr;
  std::unique_ptr<Engine> eng;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<Job>> pending;
  std::vector<std::unique_ptr<Job>> active;
  std::unordered_map<uint64_t, std::unique_ptr<Job>> finished;
  std::unordered_map<uint64_t, int> where;  // 0 pending, 1 active, 2 finished
  uint64_t next_ticket = 1;
  bool stop = false;
  size_t in_use = 0, budget = 0;
  km_server_counters ctr{};
  std::thread th;
  // threads inside km_server_wait; km_server_destroy frees the server only
  // after the last one has left
  int waiters = 0;
  std::condition_variable cv_left;

  void loop();
};

void km_server::loop() {
  (void)hipSetDevice(device);
  std::vector<BatchStatus> stat;
  for (;;) {
    std::vector<std::unique_ptr<Job>> admitted_now;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !pending.empty() || !active.empty(); });
      if (stop) break;
      // admission by footprint, in arrival order; a problem that does not fit
      // yet lets smaller later ones pass, until it has been passed over
      // kMaxPassOver times: then nothing behind it is admitted before it
      Job* blocked = nullptr;
      for (auto it = pending.begin(); it != pending.end() &&
                                      (int)(active.size() + admitted_now.size()) < cfg.max_active;) {
        if (in_use + (*it)->bytes <= budget) {
          in_use += (*it)->bytes;
          where[(*it)->ticket] = 1;
          admitted_now.push_back(std::move(*it));
          it = pending.erase(it);
        } else {
          if (!blocked) blocked = it->get();
          if ((*it)->passed_over >= kMaxPassOver) break;
          ++it;
        }
      }
      if (blocked && !admitted_now.empty()) ++blocked->passed_over;
      ctr.pending = (int64_t)pending.size();
    }
    std::vector<std::unique_ptr<Job>> failed_now;
    for (auto& jp : admitted_now) {
      jp->t_admit = now_s();
      const km_status rc = admit(*eng, *jp, s);
      if (rc != KM_OK) {
        jp->status = rc;
        jp->err = g_err;
        jp->phase = 4;
        failed_now.push_back(std::move(jp));
      } else {
        active.push_back(std::move(jp));
      }
    }
    std::vector<std::unique_ptr<Job>> done_now = std::move(failed_now);
    if (!active.empty()) {
      std::vector<Job*> act;
      for (auto& jp : active) act.push_back(jp.get());
      const int passes = chunk_passes(act, cfg.passes_per_sync);
      const km_status rc = eng->round(act, cfg.use_graphs != 0, passes, stat);
      std::vector<std::unique_ptr<Job>> keep;
      for (size_t a = 0; a < active.size(); ++a) {
        bool fin;
        if (rc != KM_OK) {
          active[a]->status = rc;
          active[a]->err = g_err;
          fin = true;
        } else {
          fin = advance(*active[a], stat[a], s);
        }
        if (fin) done_now.push_back(std::move(active[a]));
        else keep.push_back(std::move(active[a]));
      }
      active = std::move(keep);
      if (!done_now.empty()) (void)hipStreamSynchronize(s);
    }
    if (!done_now.empty() || !admitted_now.empty()) {
      std::lock_guard<std::mutex> lk(mu);
      for (auto& jp : done_now) {
        jp->t_done = now_s();
        in_use -= std::min(in_use, jp->bytes);
        if (jp->status == KM_OK) ++ctr.completed;
        else ++ctr.failed;
        where[jp->ticket] = 2;
        jp->mem.release();  // back to the pool, stream-ordered
        finished[jp->ticket] = std::move(jp);
      }
      ctr.admitted += (int64_t)admitted_now.size();
      ctr.active = (int64_t)active.size();  // written here, under mu, read by km_server_stats
      ctr.peak_active = std::max(ctr.peak_active, ctr.active);
      ctr.bytes_in_use = in_use;
      ctr.peak_bytes = std::max(ctr.peak_bytes, in_use);
      ctr.rounds = eng->rounds();
      ctr.syncs = eng->syncs();
    }
    if (!done_now.empty()) cv_done.notify_all();
  }
  // cancel what is left
  std::lock_guard<std::mutex> lk(mu);
  (void)hipStreamSynchronize(s);
  auto cancel = [&](std::unique_ptr<Job>& jp) {
    jp->status = KM_ECANCELLED;
    jp->phase = 4;
    jp->mem.release();
    where[jp->ticket] = 2;
    finished[jp->ticket] = std::move(jp);
  };
  for (auto& jp : active) cancel(jp);
  for (auto& jp : pending) cancel(jp);
  active.clear();
  pending.clear();
  cv_done.notify_all();
}

extern "C" {

km_status km_tune_query(km_dtype dtype, int32_t d, int32_t k, int32_t* points_per_thread,
                        int32_t* centers_per_tile) {
  g_err.clear();
  if (dtype != KM_F32 && dtype != KM_BF16) return fail(KM_EINVAL, "unknown dtype");
  if (d < 1 || k < 1) return fail(KM_EINVAL, "d and k must be >= 1");
  const int dmax = batch_dmax(d);
  if (!dmax) return fail(KM_EINVAL, "the batched path takes d <= 128 (got %d)", d);
  TuneVal v;
  const km_status rc = tuned(dtype == KM_F32 ? 0 : 1, dmax, k, nullptr, &v);
  if (rc != KM_OK) return rc;
  if (points_per_thread) *points_per_thread = v.ppt;
  if (centers_per_tile) *centers_per_tile = v.ktile;
  return KM_OK;
}

}  // extern "C"

namespace {

// The batch on a private stream (graph capture needs one that is not the null stream).
km_status fit_batch_on(const km_request* reqs, int32_t count, km_result* results, hipStream_t s) {
  const double t0 = now_s();
  Engine eng(s);
  km_status rc = eng.init();
  if (rc != KM_OK) return rc;
  std::vector<std::unique_ptr<Job>> jobs(count);
  std::vector<Job*> act;
  for (int32_t i = 0; i < count; ++i) {
    jobs[i] = std::make_unique<Job>();
    Job& j = *jobs[i];
    j.rq = reqs[i];
    j.t_submit = j.t_admit = t0;
    if (!valid_request(j.rq, false)) {
      j.status = KM_EINVAL;
      j.err = g_err;
      j.phase = 4;
      continue;
    }
    j.m = subset_size(j.rq.n, j.rq.k, j.rq.subset_frac);
    j.screen = batch_screen_ks(j.rq.dtype == KM_F32 ? 0 : 1, j.rq.d, j.rq.k);
    j.bytes = job_layout(j, nullptr);
    const km_status ra = admit(eng, j, s);
    if (ra != KM_OK) {
      j.status = ra;
      j.err = g_err;
      j.phase = 4;
      continue;
    }
    act.push_back(&j);
  }
  std::vector<BatchStatus> stat;
  // problems beyond the table capacity wait for earlier ones to finish
  std::vector<Job*> run, waiting;
  for (Job* j : act) (run.size() < (size_t)kTableCap ? run : waiting).push_back(j);
  while (!run.empty()) {
    rc = eng.round(run, true, chunk_passes(run, 8), stat);
    if (rc != KM_OK) break;
    std::vector<Job*> keep;
    for (size_t a = 0; a < run.size(); ++a)
      if (!advance(*run[a], stat[a], s)) keep.push_back(run[a]);
    run = std::move(keep);
    while (!waiting.empty() && run.size() < (size_t)kTableCap) {
      run.push_back(waiting.back());
      waiting.pop_back();
    }
  }
  const hipError_t e = hipStreamSynchronize(s);
  if (rc == KM_OK && e != hipSuccess)
    rc = fail(KM_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
  const double t1 = now_s();
  for (int32_t i = 0; i < count; ++i) {
    Job& j = *jobs[i];
    if (rc != KM_OK && j.phase != 4) j.status = rc;
    j.t_done = t1;
    fill_result(j, &results[i]);
  }
  return rc;
}

}  // namespace

extern "C" {

km_status kmeans_fit_batch(const km_request* reqs, int32_t count, km_result* results,
                           void* stream) {
  g_err.clear();
  if (count < 0 || (count > 0 && (!reqs || !results)))
    return fail(KM_EINVAL, "reqs and results must hold count entries");
  // work the caller queued before the call (e.g. filling X) is complete first
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return fail(KM_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
  hipStream_t s = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return fail(KM_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
  const km_status rc = fit_batch_on(reqs, count, results, s);
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  return rc;
}

km_status km_server_create(const km_server_cfg* cfg, km_server** out) {
  g_err.clear();
  if (!out) return fail(KM_EINVAL, "out must not be NULL");
  *out = nullptr;
  auto srv = std::make_unique<km_server>();
  if (cfg) srv->cfg = *cfg;
  if (srv->cfg.max_active <= 0) srv->cfg.max_active = 4096;
  srv->cfg.max_active = std::min(srv->cfg.max_active, kTableCap);
  if (srv->cfg.max_pending <= 0) srv->cfg.max_pending = 1 << 20;
  if (srv->cfg.passes_per_sync <= 0) srv->cfg.passes_per_sync = 4;
  srv->cfg.passes_per_sync = std::min(srv->cfg.passes_per_sync, kMaxChunk);
  if (hipGetDevice(&srv->device) != hipSuccess) return fail(KM_EDEVICE, "no HIP device");
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(KM_EDEVICE, "hipMemGetInfo failed");
  srv->budget = srv->cfg.hbm_budget_bytes ? srv->cfg.hbm_budget_bytes : fr / 4 * 3;
  if (hipStreamCreateWithFlags(&srv->s, hipStreamNonBlocking) != hipSuccess)
    return fail(KM_EDEVICE, "hipStreamCreate failed");
  srv->eng = std::make_unique<Engine>(srv->s);
  const km_status rc = srv->eng->init();
  if (rc != KM_OK) {
    (void)hipStreamDestroy(srv->s);
    return rc;
  }
  km_server* p = srv.release();
  p->th = std::thread([p] { p->loop(); });
  *out = p;
  return KM_OK;
}

km_status km_server_submit(km_server* srv, const km_request* req, uint64_t* ticket) {
  g_err.clear();
  if (!srv || !req || !ticket) return fail(KM_EINVAL, "srv, req and ticket must not be NULL");
  auto j = std::make_unique<Job>();
  j->rq = *req;
  if (!valid_request(j->rq, true)) return KM_EINVAL;
  j->copy_x = true;
  j->m = subset_size(j->rq.n, j->rq.k, j->rq.subset_frac);
  j->screen = batch_screen_ks(j->rq.dtype == KM_F32 ? 0 : 1, j->rq.d, j->rq.k);
  j->bytes = job_layout(*j, nullptr);
  j->t_submit = now_s();
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) return fail(KM_ECANCELLED, "the server is shutting down");
  if (j->bytes > srv->budget)
    return fail(KM_ENOMEM, "the problem needs %zu device bytes, the budget is %zu", j->bytes,
                srv->budget);
  if ((int64_t)srv->pending.size() >= srv->cfg.max_pending)
    return fail(KM_EBUSY, "%d problems are already waiting", srv->cfg.max_pending);
  j->ticket = srv->next_ticket++;
  *ticket = j->ticket;
  srv->where[j->ticket] = 0;
  srv->pending.push_back(std::move(j));
  ++srv->ctr.submitted;
  srv->ctr.pending = (int64_t)srv->pending.size();
  srv->cv_work.notify_one();
  return KM_OK;
}

km_status km_server_wait(km_server* srv, uint64_t ticket, km_result* out, int64_t timeout_us) {
  g_err.clear();
  if (!srv || !out) return fail(KM_EINVAL, "srv and out must not be NULL");
  std::unique_lock<std::mutex> lk(srv->mu);
  if (!srv->where.count(ticket)) return fail(KM_ENOTFOUND, "unknown ticket %llu",
                                             (unsigned long long)ticket);
  // registered as a waiter until return, so that km_server_destroy does not
  // free the server under this thread
  ++srv->waiters;
  struct Leave {
    km_server* s;
    ~Leave() {
      if (--s->waiters == 0) s->cv_left.notify_all();
    }
  } leave{srv};
  auto ready = [&] { return srv->finished.count(ticket) > 0; };
  if (timeout_us < 0) {
    srv->cv_done.wait(lk, ready);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return fail(KM_ETIMEOUT, "ticket %llu not finished", (unsigned long long)ticket);
  }
  auto it = srv->finished.find(ticket);
  fill_result(*it->second, out);
  if (it->second->status != KM_OK && !it->second->err.empty()) g_err = it->second->err;
  const km_status st = it->second->status;
  srv->finished.erase(it);
  srv->where.erase(ticket);
  return st == KM_OK ? KM_OK : st;
}

km_status km_server_stats(km_server* srv, km_server_counters* out) {
  g_err.clear();
  if (!srv || !out) return fail(KM_EINVAL, "srv and out must not be NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->ctr;  // the scheduler thread owns `active`; ctr.active is its count
  out->pending = (int64_t)srv->pending.size();
  return KM_OK;
}

km_status km_server_destroy(km_server* srv) {
  g_err.clear();
  if (!srv) return fail(KM_EINVAL, "srv must not be NULL");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->th.joinable()) srv->th.join();
  // the scheduler has cancelled every unfinished problem (KM_ECANCELLED) and
  // woken the waiters; they collect their results before the server goes
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_left.wait(lk, [&] { return srv->waiters == 0; });
  }
  srv->eng.reset();
  (void)hipStreamDestroy(srv->s);
  delete srv;
  return KM_OK;
}

}  // extern "C"
