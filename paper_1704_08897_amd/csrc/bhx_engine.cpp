// Serving engine: continuous batching of extension requests on one device.
//
// Requests are admitted at submit time against an HBM budget (their
// workspace is carved from one device arena) and a slot limit.  A worker
// thread owns the stream: at every iteration-chunk boundary it sets up the
// requests admitted since the last boundary (mask, right-hand side, first
// preconditioner application - as a batch of their own), then runs one
// captured chunk of PCG iterations over every active request, checks the
// true residual of the requests that stopped, restarts those that miss the
// target and retires the rest, returning their workspace to the arena.  New
// requests therefore join while others are mid-solve, and their work shares
// the same launches.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "bhx_runtime.h"

namespace bhx {
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Req {
  uint64_t id;
  InstSpec spec;
  size_t off = 0, bytes = 0;
  int slot = -1;
  double t_submit = 0;
  Inst inst;
  bool active = false;
  bool finished = false;
  int status = BHX_OK;
  bhx_stats st;
};

// A device-resident batch header with its own instance and work-item arrays.
struct DevBatch {
  Batch* hdr = nullptr;
  Inst* inst = nullptr;
  int* items[kNumPass] = {nullptr, nullptr, nullptr};
  int inst_cap = 0;
  int items_cap[kNumPass] = {0, 0, 0};
  int count = 0;
  int n_items[kNumPass] = {0, 0, 0};
};

}  // namespace
}  // namespace bhx

struct bhx_engine {
  bhx_handle* hd = nullptr;
  bhx::Resolved R;
  size_t budget = 0, committed = 0;
  int max_slots = 0;
  char* arena_base = nullptr;
  bhx::Arena arena;
  bhx::Ctl* ctl_d = nullptr;
  bhx::Ctl* ctl_h = nullptr;
  int* flag_d = nullptr;            // per-request flags of a setup round [max_slots]
  bhx::DevBatch run, aux;
  std::vector<int> free_slots;
  std::deque<bhx::Req*> incoming;
  std::vector<bhx::Req*> active;
  std::deque<bhx::Req*> completed;
  std::map<std::pair<int, int>, int> plan_idx;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  std::atomic<int> inflight{0};
  uint64_t next_id = 1;
  std::thread worker;
  int device = 0;
  // kernel timing of the iteration passes (engines created with a profile mask)
  double prof_ms[4] = {0, 0, 0, 0};
  long long prof_launches[4] = {0, 0, 0, 0};
  double prof_unknown[4] = {0, 0, 0, 0}, prof_nodes[4] = {0, 0, 0, 0};
};

namespace bhx {
namespace {

#define ENG_CHECK(x)                                          \
  do {                                                        \
    hipError_t _e = (x);                                      \
    if (_e != hipSuccess) {                                   \
      set_last_error(#x, __LINE__, _e);                       \
      return BHX_ERR_HIP;                                     \
    }                                                         \
  } while (0)

template <typename T>
hipError_t ensure(T** p, int* cap, int need) {
  if (need <= *cap && *p) return hipSuccess;
  if (*p) {
    hipError_t e = hipFree(*p);
    if (e != hipSuccess) return e;
    *p = nullptr;
  }
  const int c = std::max(need, 2 * *cap);
  hipError_t e = hipMalloc((void**)p, (size_t)c * sizeof(T));
  *cap = e == hipSuccess ? c : 0;
  return e;
}

// Upload a batch of requests into `db` (descriptor copies + work lists).
int upload_batch(bhx_engine* E, DevBatch& db, const std::vector<Req*>& reqs, hipStream_t st) {
  const int n = (int)reqs.size();
  std::vector<Inst> inst(n);
  std::vector<int> items[kNumPass];
  for (int i = 0; i < n; ++i) {
    inst[i] = reqs[i]->inst;
    for (int p = 0; p < kNumPass; ++p)
      for (int k = 0; k < list_items(inst[i], p); ++k) items[p].push_back((i << kItemShift) | k);
  }
  if (!db.hdr) ENG_CHECK(hipMalloc((void**)&db.hdr, sizeof(Batch)));
  ENG_CHECK(ensure(&db.inst, &db.inst_cap, std::max(n, 1)));
  for (int p = 0; p < kNumPass; ++p)
    ENG_CHECK(ensure(&db.items[p], &db.items_cap[p], std::max<int>(1, (int)items[p].size())));
  Batch B;
  std::memset(&B, 0, sizeof(B));
  B.count = n;
  for (int p = 0; p < kNumPass; ++p) {
    B.n_items[p] = (int)items[p].size();
    B.items[p] = (std::remove_reference_t<decltype(B.items[p])>)db.items[p];
    db.n_items[p] = B.n_items[p];
  }
  B.inst = (decltype(B.inst))db.inst;
  B.plans = (decltype(B.plans))E->hd->plans.plans_d();
  for (int p = 0; p < 2; ++p) {
    B.ctab[p] = (std::remove_reference_t<decltype(B.ctab[p])>)E->hd->plans.ctab(p);
    B.rtab[p] = (std::remove_reference_t<decltype(B.rtab[p])>)E->hd->plans.rtab(p);
  }
  db.count = n;
  // previous launches reading this header have completed; the copies are
  // stream-ordered before the launches that follow on st
  ENG_CHECK(hipStreamSynchronize(st));
  Upload u[2 + kNumPass] = {{db.inst, inst.data(), n * sizeof(Inst)},
                            {db.hdr, &B, sizeof(Batch)}};
  for (int p = 0; p < kNumPass; ++p)
    u[2 + p] = {db.items[p], items[p].data(), items[p].size() * sizeof(int)};
  ENG_CHECK(upload_ordered(E->hd, st, u, 2 + kNumPass));
  return BHX_OK;
}

// Packed rows per transform work item of the engine's requests: the
// caller's bhx_opts.rows, else the fullest items (-1): every launch is
// shared with other requests, so none has to fill the GPU alone.  A request
// equals its solo solve with the same bhx_opts.rows bit for bit.
int engine_rows(const bhx_engine* E) {
  return E->R.sched.rows_cap != 0 ? E->R.sched.rows_cap : -1;
}

// Launch geometry for a set of requests: persistent grids of fixed size (so
// captured graphs survive changes of the active set) and LDS from the
// largest transform among the requests.
Grids engine_grids(bhx_engine* E, const std::vector<Req*>& reqs) {
  Grids g;
  const int cu = E->hd->num_cu;
  g.s = cu * 8;
  g.r = cu * 2;
  g.c = cu * 2;
  const int csize = E->R.precision == 0 ? 16 : 8;
  int buf_r = 0, buf_c = 0;
  int any_dense = 0;
  g.count = (int)reqs.size();
  for (Req* q : reqs) {
    g.reduce |= q->inst.reduce;
    if (q->inst.dense) {                         // no FFT pass works on it
      any_dense = 1;
      continue;
    }
    const AxisPlan& PX = E->hd->plans.plan(q->inst.planx);
    const AxisPlan& PY = E->hd->plans.plan(q->inst.plany);
    plan_family(PX, q->inst.G / 2, &g.shape_r);  // plan-table kernel families
    plan_family(PY, q->inst.Gc / 2, &g.shape_c);
    buf_r = std::max(buf_r, (q->inst.G / 2) * row_slots(PX.m));
    buf_c = std::max(buf_c, (q->inst.Gc / 2) * row_slots(PY.m));
  }
  // the engine runs the plan-table kernels, which read their tables from
  // global memory: LDS for the packed rows alone, rounded up to 4 KiB steps
  // so graphs are reused across batches (two 4096-point FP64 rows' blocks
  // still fit one CU)
  auto up = [](int b) { return (b + 4095) / 4096 * 4096; };
  g.tw_r = buf_r;
  g.lds_r = std::min(kLdsDynMax, up(buf_r * csize));
  g.tw_c = buf_c;
  g.lds_c = std::min(kLdsDynMax, up(buf_c * csize));
  // the FFT family launches every iteration (with no request on it it
  // returns at once); the dense passes, sized for the longest dense axis,
  // only while a dense request is active.  The captured graphs depend on the
  // active set through these few fields alone.
  g.fft = 1;
  g.dense = any_dense;
  if (any_dense) dense_grids(E->R.precision, kDenseMax, kDenseMax, cu * 2, cu * 2, cu, 2, &g);
  return g;
}

void finish_req(bhx_engine* E, Req* q, double t) {
  q->finished = true;
  q->st.seconds = t - q->t_submit;
  std::lock_guard<std::mutex> lk(E->mu);
  E->arena.release(q->off, q->bytes);
  E->committed -= q->bytes;
  E->free_slots.push_back(q->slot);
  E->completed.push_back(q);
}

// Setup of newly admitted requests (as their own batch), then the first
// preconditioner application; requests that end here (nothing unknown,
// singular, non-finite, zero right-hand side) complete at once.
int setup_new(bhx_engine* E, std::vector<Req*>& news, hipStream_t st) {
  bhx_handle* hd = E->hd;
  for (Req* q : news) {
    const InstSpec& S = q->spec;
    const int px = hd->plans.get(S.nx, S.bcx), py = hd->plans.get(S.ny, S.bcy);
    Layout L;
    const bool dense = use_dense(E->R, hd->plans.plan(px), hd->plans.plan(py));
    make_layout(S.nx, S.ny, E->R.precision, hd->plans.plan(px).m, hd->plans.plan(py).m,
                engine_rows(E), &L, dense);
    Inst& I = q->inst;
    std::memset(&I, 0, sizeof(I));
    I.nx = S.nx; I.ny = S.ny; I.nz = 1; I.nrows = S.ny;
    I.bcx = S.bcx; I.bcy = S.bcy;
    I.planx = px; I.plany = py;
    I.G = L.G; I.Gc = L.Gc; I.tiles_x = L.tiles_x; I.tiles_y = L.tiles_y; I.tiles_z = 1;
    for (int p = 0; p < kNumPass; ++p) I.n_items[p] = L.n_items[p];
    I.maxit = E->R.maxit_user > 0 ? E->R.maxit_user : 50 * std::max(S.nx, S.ny);
    I.flexible = E->R.flexible;
    I.warm = E->R.warm;
    I.reduce = L.n_items[kPassS] + 3 * L.n_items[kPassR] > kReduceMin;
    I.dense = dense;
    I.phi = (decltype(I.phi))S.phi;
    I.F = (decltype(I.F))S.F;
    char* b = E->arena_base + q->off;
    const size_t Np = vec_stride(S.nx, S.ny);
    I.mask = (decltype(I.mask))(b + L.off_mask);
    double* v = (double*)(b + L.off_vec);
    I.r = (decltype(I.r))v;
    I.p[0] = (decltype(I.r))(v + Np);
    I.p[1] = (decltype(I.r))(v + 2 * Np);
    I.q = (decltype(I.r))(v + 3 * Np);
    I.z = (decltype(I.r))(v + 4 * Np);
    I.t = (decltype(I.t))(b + L.off_t);
    I.part = (decltype(I.part))(b + L.off_part);
    I.ctl = (decltype(I.ctl))(E->ctl_d + q->slot);
    Ctl C;
    std::memset(&C, 0, sizeof(C));
    C.tol2 = S.tol * S.tol;
    C.tol_inner2 = E->R.tol_inner * E->R.tol_inner;
    C.accurate = E->R.accurate;
    C.max_restarts = E->R.accurate ? 12 : 8;
    E->ctl_h[q->slot] = C;
    ENG_CHECK(hipMemcpyAsync(E->ctl_d + q->slot, &E->ctl_h[q->slot], sizeof(Ctl),
                             hipMemcpyHostToDevice, st));
  }
  ENG_CHECK(hd->plans.sync_device(st));
  int rc = upload_batch(E, E->aux, news, st);
  if (rc != BHX_OK) return rc;
  const Grids g = engine_grids(E, news);
  const int n = (int)news.size();
  ENG_CHECK(launch_setup(E->aux.hdr, 2, g.s, st));
  ENG_CHECK(launch_setup_rows(E->aux.hdr, std::max(g.r, g.rd), st));
  ENG_CHECK(launch_stencil(E->aux.hdr, 2, kModeRhs, g.s, 0, st));
  ENG_CHECK(launch_finalize(E->aux.hdr, n, kFinSetupH, st));
  ENG_CHECK(hipMemcpyAsync(E->ctl_h, E->ctl_d, E->max_slots * sizeof(Ctl), hipMemcpyDeviceToHost,
                           st));
  ENG_CHECK(hipStreamSynchronize(st));
  std::vector<int> zero_flag(n, 0);
  bool any_zero = false;
  std::vector<Req*> keep, done_now;
  for (int i = 0; i < n; ++i) {
    Req* q = news[i];
    Ctl& C = E->ctl_h[q->slot];
    const double N = (double)q->spec.nx * q->spec.ny;
    int s = BHX_OK;
    bool fin = true;
    if (C.n_unknown == 0) s = BHX_OK;
    else if (C.n_unknown == N && q->spec.bcx != kDirichlet && q->spec.bcy != kDirichlet)
      s = BHX_ERR_SINGULAR;
    else if (!std::isfinite(C.bb)) s = BHX_ERR_NONFINITE;
    else if (C.bb == 0.0) { zero_flag[i] = 1; any_zero = true; }
    else fin = false;
    if (fin) {
      C.done = kSkip;
      ENG_CHECK(hipMemcpyAsync(E->ctl_d + q->slot, &C, sizeof(Ctl), hipMemcpyHostToDevice, st));
      std::memset(&q->st, 0, sizeof(q->st));
      q->st.status = s;
      q->st.n_unknown = (int)C.n_unknown;
      done_now.push_back(q);
    } else {
      keep.push_back(q);
    }
  }
  if (any_zero) {
    // flag_d holds max_slots entries (allocated with the engine); a setup
    // round never has more new requests than slots
    const Upload u{E->flag_d, zero_flag.data(), n * sizeof(int)};
    ENG_CHECK(upload_ordered(E->hd, st, &u, 1));
    ENG_CHECK(launch_zero_unknown(E->aux.hdr, 2, E->flag_d, g.s, st));
    ENG_CHECK(hipStreamSynchronize(st));
  }
  if (E->R.warm && !keep.empty()) {
    // warm start: r0 = b - A x0; requests whose start already meets the
    // tolerance, or whose residual is not finite, end here with F untouched
    ENG_CHECK(launch_stencil(E->aux.hdr, 2, kModeWarm, g.s, 0, st));
    ENG_CHECK(launch_finalize(E->aux.hdr, n, kFinWarmH, st));
    ENG_CHECK(hipMemcpyAsync(E->ctl_h, E->ctl_d, E->max_slots * sizeof(Ctl),
                             hipMemcpyDeviceToHost, st));
    ENG_CHECK(hipStreamSynchronize(st));
    std::vector<Req*> still;
    for (Req* q : keep) {
      Ctl& C = E->ctl_h[q->slot];
      const int w = warm_start_outcome(C);
      if (w == 0) {
        still.push_back(q);
        continue;
      }
      C.done = kSkip;
      ENG_CHECK(hipMemcpyAsync(E->ctl_d + q->slot, &C, sizeof(Ctl), hipMemcpyHostToDevice, st));
      std::memset(&q->st, 0, sizeof(q->st));
      q->st.status = w == 1 ? BHX_OK : BHX_ERR_NONFINITE;
      q->st.n_unknown = (int)C.n_unknown;
      if (C.bb0 > 0) q->st.rel_residual = q->st.true_rel_residual = std::sqrt(C.rr / C.bb0);
      done_now.push_back(q);
    }
    keep.swap(still);
  }
  if (!keep.empty()) {
    // preconditioner of r0 for the requests that iterate (skipped ones are
    // marked done and ignored by the kernels)
    ENG_CHECK(launch_precond(E->aux.hdr, E->R, g, st));
  }
  ENG_CHECK(hipStreamSynchronize(st));
  const double t = now_s();
  for (Req* q : done_now) finish_req(E, q, t);
  for (Req* q : keep) {
    q->active = true;
    E->active.push_back(q);
  }
  return BHX_OK;
}

// One chunk of iterations over all active requests; retire the finished.
int step_active(bhx_engine* E, hipStream_t st) {
  int rc = upload_batch(E, E->run, E->active, st);
  if (rc != BHX_OK) return rc;
  const Grids g = engine_grids(E, E->active);
  const int n = (int)E->active.size();
  std::vector<int> iter_before(n);
  for (int i = 0; i < n; ++i) iter_before[i] = E->ctl_h[E->active[i]->slot].iter;
  Graph* used = nullptr;
  ENG_CHECK(run_chunk(E->hd, E->run.hdr, n, E->R, g, st, &used));
  ENG_CHECK(hipMemcpyAsync(E->ctl_h, E->ctl_d, E->max_slots * sizeof(Ctl), hipMemcpyDeviceToHost,
                           st));
  ENG_CHECK(hipStreamSynchronize(st));
  if (E->R.profile && used && !used->ev.empty()) {
    // launch c of a pass worked on the requests that ran more than c
    // iterations of this chunk; their node counts go with its time
    int worked = 0;
    double iu = 0, in = 0;
    for (int i = 0; i < n; ++i) {
      const Req* q = E->active[i];
      const int it = E->ctl_h[q->slot].iter - iter_before[i];
      worked = std::max(worked, it);
      iu += (double)it * E->ctl_h[q->slot].n_unknown;
      in += (double)it * q->spec.nx * q->spec.ny;
    }
    for (int p = 0; p < 4; ++p) {
      if (!(E->R.profile & (1 << p))) continue;
      double sum = 0;
      for (int c = 0; c < worked && c < E->R.chunk; ++c) {
        float ms = 0;
        ENG_CHECK(hipEventElapsedTime(&ms, used->ev[((size_t)p * E->R.chunk + c) * 2],
                                      used->ev[((size_t)p * E->R.chunk + c) * 2 + 1]));
        sum += ms;
      }
      std::lock_guard<std::mutex> lk(E->mu);   // read by bhx_engine_profile
      E->prof_ms[p] += sum;
      E->prof_launches[p] += std::min(worked, E->R.chunk);
      E->prof_unknown[p] += iu;
      E->prof_nodes[p] += in;
    }
  }
  bool any_done = false;
  for (Req* q : E->active)
    if (E->ctl_h[q->slot].done != kRunning) any_done = true;
  if (!any_done) return BHX_OK;
  ENG_CHECK(launch_resid(E->run.hdr, 2, g.s, st));
  ENG_CHECK(launch_finalize(E->run.hdr, n, kFinResidH, st));
  ENG_CHECK(launch_restart(E->run.hdr, n, st));
  ENG_CHECK(hipMemcpyAsync(E->ctl_h, E->ctl_d, E->max_slots * sizeof(Ctl), hipMemcpyDeviceToHost,
                           st));
  ENG_CHECK(hipStreamSynchronize(st));
  std::vector<Req*> restarted, still, finished;
  for (Req* q : E->active) {
    const Ctl& C = E->ctl_h[q->slot];
    if (C.done == kRunning) {
      still.push_back(q);
      if (C.restart_iter == C.iter && C.restarts > 0 && C.iter > 0) restarted.push_back(q);
    } else {
      finished.push_back(q);
    }
  }
  if (!restarted.empty()) {
    // restarted requests need z = M r of their new residual (only them)
    rc = upload_batch(E, E->aux, restarted, st);
    if (rc != BHX_OK) return rc;
    ENG_CHECK(launch_precond(E->aux.hdr, E->R, engine_grids(E, restarted), st));
    ENG_CHECK(hipStreamSynchronize(st));
  }
  const double t = now_s();
  for (Req* q : finished) {
    const Ctl& C = E->ctl_h[q->slot];
    bhx_stats& o = q->st;
    std::memset(&o, 0, sizeof(o));
    switch (C.done) {
      case kConverged: o.status = C.true_rr <= C.accept ? BHX_OK : BHX_NOT_CONVERGED; break;
      case kMaxIt: o.status = BHX_NOT_CONVERGED; break;
      default: o.status = BHX_ERR_BREAKDOWN; break;
    }
    o.iterations = C.iter;
    o.restarts = C.restarts;
    o.n_unknown = (int)C.n_unknown;
    o.rel_residual = C.bb0 > 0 ? std::sqrt(C.rr / C.bb0) : 0.0;
    o.true_rel_residual = C.bb0 > 0 ? std::sqrt(C.true_rr / C.bb0) : 0.0;
    q->active = false;
    finish_req(E, q, t);
  }
  E->active = still;
  return BHX_OK;
}

void worker_main(bhx_engine* E) {
  (void)hipSetDevice(E->device);
  hipStream_t st = E->hd->own_stream;
  for (;;) {
    std::vector<Req*> news;
    {
      std::unique_lock<std::mutex> lk(E->mu);
      E->cv.wait(lk, [&] { return E->stop || !E->incoming.empty() || !E->active.empty(); });
      if (E->stop && E->incoming.empty() && E->active.empty()) break;
      while (!E->incoming.empty()) {
        news.push_back(E->incoming.front());
        E->incoming.pop_front();
      }
    }
    int rc = BHX_OK;
    if (!news.empty()) rc = setup_new(E, news, st);
    if (rc == BHX_OK && !E->active.empty()) rc = step_active(E, st);
    if (rc != BHX_OK) {
      // fail every request in flight with the error and keep serving
      const double t = now_s();
      std::vector<Req*> all = E->active;
      for (Req* q : news)
        if (!q->active && !q->finished) all.push_back(q);
      E->active.clear();
      for (Req* q : all) {
        std::memset(&q->st, 0, sizeof(q->st));
        q->st.status = rc;
        finish_req(E, q, t);
      }
      (void)hipStreamSynchronize(st);
    }
  }
}

}  // namespace
}  // namespace bhx

extern "C" {

int bhx_engine_create(bhx_engine** out, int device, size_t hbm_budget, int max_slots,
                      const bhx_opts* o) {
  if (!out) return BHX_ERR_ARG;
  *out = nullptr;
  if (max_slots < 1 || max_slots > (1 << (31 - bhx::kItemShift)) || hbm_budget < (1u << 20))
    return BHX_ERR_ARG;
  bhx::Resolved R = bhx::resolve_opts(o);
  static const double dummy = 0;
  if (bhx::validate(&dummy, (double*)&dummy, 8, 8, 1.0, 0, 0.5, R) != BHX_OK || R.solver != 0)
    return BHX_ERR_ARG;
  bhx_engine* E = new (std::nothrow) bhx_engine();
  if (!E) return BHX_ERR_NOMEM;
  int s = bhx_create(&E->hd, device);
  if (s != BHX_OK) {
    delete E;
    return s;
  }
  E->device = device;
  E->R = R;
  E->R.chunk = o && o->chunk > 0 ? o->chunk : 16;   // short chunks: new requests join quickly
  E->R.chunk += E->R.chunk & 1;                       // even (buffer parity restarts each chunk)
  // profile mask: the chunks launch directly with dispatch events around the
  // selected passes (slower than the captured graphs; for measurement runs)
  E->R.profile = o ? o->profile : 0;
  E->budget = hbm_budget;
  E->max_slots = max_slots;
  if (hipMalloc((void**)&E->arena_base, hbm_budget) != hipSuccess ||
      hipMalloc((void**)&E->ctl_d, max_slots * sizeof(bhx::Ctl)) != hipSuccess ||
      hipMalloc((void**)&E->flag_d, max_slots * sizeof(int)) != hipSuccess ||
      hipHostMalloc((void**)&E->ctl_h, max_slots * sizeof(bhx::Ctl)) != hipSuccess) {
    bhx_engine_destroy(E);
    return BHX_ERR_NOMEM;
  }
  std::memset(E->ctl_h, 0, max_slots * sizeof(bhx::Ctl));
  E->arena.reset(hbm_budget);
  for (int i = max_slots - 1; i >= 0; --i) E->free_slots.push_back(i);
  E->worker = std::thread(bhx::worker_main, E);
  *out = E;
  return BHX_OK;
}

int bhx_engine_submit(bhx_engine* E, const double* phi, double* F, int nx, int ny, double h,
                      int bc, double tol, uint64_t* id) {
  if (!E || !id) return BHX_ERR_ARG;
  int v = bhx::validate(phi, F, nx, ny, h, bc, tol, E->R);
  if (v != BHX_OK) return v;
  const size_t bytes =
      bhx::instance_bytes(nx, ny, bc & 15, (bc >> 4) & 15, E->R.precision, bhx::engine_rows(E));
  if (bytes == 0 || bytes > E->budget) return BHX_ERR_ARG;      // can never fit
  bhx::Req* q = new (std::nothrow) bhx::Req();
  if (!q) return BHX_ERR_NOMEM;
  {
    std::lock_guard<std::mutex> lk(E->mu);
    if (E->stop || E->free_slots.empty() || E->committed + bytes > E->budget ||
        !E->arena.alloc(bytes, &q->off)) {
      delete q;
      return BHX_BUSY;
    }
    q->slot = E->free_slots.back();
    E->free_slots.pop_back();
    q->bytes = bytes;
    E->committed += bytes;
    q->id = E->next_id++;
    q->spec = bhx::InstSpec{phi, F, nx, ny, bc & 15, (bc >> 4) & 15, tol};
    q->t_submit = bhx::now_s();
    E->incoming.push_back(q);
    *id = q->id;
    E->inflight++;
  }
  E->cv.notify_one();
  return BHX_OK;
}

int bhx_engine_poll(bhx_engine* E, uint64_t* ids, bhx_stats* st, int max, int* n_done) {
  if (!E || !n_done || max < 0 || (max > 0 && (!ids || !st))) return BHX_ERR_ARG;
  std::lock_guard<std::mutex> lk(E->mu);
  int n = 0;
  while (n < max && !E->completed.empty()) {
    bhx::Req* q = E->completed.front();
    E->completed.pop_front();
    ids[n] = q->id;
    st[n] = q->st;
    ++n;
    delete q;
    E->inflight--;
  }
  *n_done = n;
  return BHX_OK;
}

int bhx_engine_inflight(bhx_engine* E) { return E ? E->inflight.load() : 0; }

int bhx_engine_profile(bhx_engine* E, double* ms, long long* launches, double* unknown_nodes,
                       double* nodes, int reset) {
  if (!E || !ms || !launches || !unknown_nodes || !nodes) return BHX_ERR_ARG;
  std::lock_guard<std::mutex> lk(E->mu);
  for (int p = 0; p < 4; ++p) {
    ms[p] = E->prof_ms[p];
    launches[p] = E->prof_launches[p];
    unknown_nodes[p] = E->prof_unknown[p];
    nodes[p] = E->prof_nodes[p];
    if (reset) {
      E->prof_ms[p] = 0;
      E->prof_launches[p] = 0;
      E->prof_unknown[p] = E->prof_nodes[p] = 0;
    }
  }
  return BHX_OK;
}

void bhx_engine_destroy(bhx_engine* E) {
  if (!E) return;
  {
    std::lock_guard<std::mutex> lk(E->mu);
    E->stop = true;
  }
  E->cv.notify_all();
  if (E->worker.joinable()) E->worker.join();
  for (bhx::Req* q : E->completed) delete q;
  (void)hipSetDevice(E->device);
  auto free_db = [](bhx::DevBatch& d) {
    if (d.hdr) (void)hipFree(d.hdr);
    if (d.inst) (void)hipFree(d.inst);
    for (int p = 0; p < bhx::kNumPass; ++p)
      if (d.items[p]) (void)hipFree(d.items[p]);
  };
  free_db(E->run);
  free_db(E->aux);
  if (E->arena_base) (void)hipFree(E->arena_base);
  if (E->ctl_d) (void)hipFree(E->ctl_d);
  if (E->flag_d) (void)hipFree(E->flag_d);
  if (E->ctl_h) (void)hipHostFree(E->ctl_h);
  if (E->hd) bhx_destroy(E->hd);
  delete E;
}

}  // extern "C"
