// C ABI of libfcgno, serving: the continuous-batching engine (requests of
// any grid size admitted by device-pool footprint, grouped by N, advanced in
// steps of check_every iterations on per-group streams).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "common.h"
#include "fcgno.h"
#include "host.h"
#include "prof.h"
#include "train.h"

using namespace fcgno;
using namespace fcgno_host;

namespace fcgno_host {

struct EngReq {
  int64_t id = 0;
  int N = 0, max_iter = 0;
  double rtol = 0.0;
  const double* k = nullptr;
  const double* f = nullptr;
  double* u = nullptr;
  size_t off = 0, bytes = 0;
  Plan p;
  SysDev sd{};
};

struct EngGroup {
  int N = 0;
  size_t off = 0, bytes = 0;
  size_t E64 = 0, Eacc = 0, T = 0, TT = 0, FA = 0, SA = 0, RD = 0, EX = 0, table = 0, ftable = 0, flags = 0, tres = 0;
  std::vector<int64_t> members;
  bool dirty = true;
  size_t hoff = 0;           // this step's range in the engine's pinned export buffers
  hipStream_t s = nullptr;   // the engine lane this group's work runs on
};

}  // namespace fcgno_host

struct fcgno_engine {
  const fcgno_model* m = nullptr;
  fcgno_engine_desc d{};
  hipStream_t s = nullptr;
  char* pool = nullptr;
  std::map<size_t, size_t> free_;       // offset -> size of free blocks
  std::deque<EngReq> queue;
  std::map<int64_t, EngReq> active;
  std::map<int, EngGroup> groups;
  std::vector<fcgno_engine_result> done;
  int64_t next_id = 1;
  int* hflags = nullptr;     // pinned host copies of the exported state, max_slots entries
  double* htres = nullptr;   // two per slot: relative to ||r_0|| and to ||f||
  // Groups of different N run on separate streams (default priority), so a
  // large group's bandwidth-bound launches and a small group's latency-bound
  // ones overlap on the device; every step first waits for the caller's stream.
  std::vector<hipStream_t> lanes;
  hipEvent_t ready = nullptr;
  int next_lane = 0;
};

namespace fcgno_host {

bool pool_alloc(fcgno_engine* e, size_t bytes, size_t* off) {
  bytes = align256(bytes);
  for (auto it = e->free_.begin(); it != e->free_.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t roff = it->first + bytes;
      e->free_.erase(it);
      if (rest) e->free_[roff] = rest;
      return true;
    }
  }
  return false;
}

void pool_free(fcgno_engine* e, size_t off, size_t bytes) {
  bytes = align256(bytes);
  auto it = e->free_.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != e->free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    e->free_.erase(nx);
  }
  if (it != e->free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      e->free_.erase(it);
    }
  }
}

size_t request_bytes(const fcgno_model* m, int op, int m_max, int N, int max_iter) {
  return make_plan(op == PID ? nullptr : m, N, 1, m_max, max_iter, op, KIND_SOLVE).total;
}

size_t group_bytes(const fcgno_model* m, int op, int N, int slots, EngGroup* g) {
  Carver cv;
  const int MP = m && op != PID ? round16(2 * m->arch.modes) : 16, NP = round16(N);
  const int esz = op_esize(op == PID ? P64 : op), asz = acc_esize(op == PID ? P64 : op);
  EngGroup t;
  t.E64 = cv.take((size_t)tw_period(m ? m->arch.basis : B_FOURIER, N) * 16);
  t.Eacc = cv.take((size_t)tw_period(m ? m->arch.basis : B_FOURIER, N) * 2 * asz);
  t.T = cv.take((size_t)NP * MP * esz);
  t.TT = cv.take((size_t)MP * NP * esz);
  t.RD = cv.take((size_t)NP * 32 * 8);
  if (op == PBF) {   // split-bfloat16 twiddle operands of the matrix-core x transforms
    t.FA = cv.take((size_t)2 * 32 * 2 * NP * 2);
    t.SA = cv.take((size_t)2 * NP * 64 * 2);
    t.EX = cv.take((size_t)NP * 32 * 8);
  }
  t.table = cv.take((size_t)slots * sizeof(SysDev));
  t.ftable = cv.take((size_t)slots * sizeof(SysDev));
  t.flags = cv.take((size_t)slots * 3 * sizeof(int));
  t.tres = cv.take((size_t)slots * 2 * sizeof(double));
  if (g) {
    g->E64 = t.E64; g->Eacc = t.Eacc; g->T = t.T; g->TT = t.TT; g->FA = t.FA; g->SA = t.SA; g->RD = t.RD; g->EX = t.EX;
    g->table = t.table; g->ftable = t.ftable; g->flags = t.flags; g->tres = t.tres;
  }
  return cv.n;
}

NOLaunch group_no(const fcgno_engine* e, const EngGroup& g, const SysDev* table, int nsys) {
  const fcgno_model* m = e->m;
  const int op = e->d.op;
  char* base = e->pool + g.off;
  NOLaunch L{};
  L.sys = table;
  L.nsys = nsys;
  L.N = g.N;
  L.C = m->arch.width;
  L.M = m->arch.modes;
  L.MP = round16(2 * L.M);
  L.L = m->arch.layers;
  // groups of few requests run one row segment per wave (the same bits)
  L.S = seg_count(g.N);
  L.spw = nsys > 0 && nsys <= LOW_ACTIVE ? 1 : SPW_HIGH;
  L.prec = op;
  L.basis = m->arch.basis;
  L.tab.E64 = (const double*)(base + g.E64);
  L.tab.Eacc = base + g.Eacc;
  L.tab.T = base + g.T;
  L.tab.TT = base + g.TT;
  L.tab.FA = op == PBF ? base + g.FA : nullptr;
  L.tab.SA = op == PBF ? base + g.SA : nullptr;
  L.tab.RD = (const double*)(base + g.RD);
  L.tab.EX = op == PBF ? base + g.EX : nullptr;
  L.Wfrag = m->Wfrag[op].data();
  L.bias = m->bias[op].data();
  L.Rmix = m->Rmix[op].data();
  L.WP = m->WP[op];
  L.bP = dev_bP(m);
  L.WL0 = m->WL0[op];
  L.WL = dev_WL(m);
  L.bL = dev_bL(m);
  L.stream = g.s;
  L.op_bytes = op_esize(op);
  L.acc_bytes = acc_esize(op);
  return L;
}

// Lay out a new group of grid N and reserve its pool block; nothing is queued
// on the device yet, so a failed admission can hand the block back at once.
bool group_reserve(fcgno_engine* e, int N, EngGroup* g) {
  g->N = N;
  g->bytes = group_bytes(e->d.op == PID ? nullptr : e->m, e->d.op, N, e->d.max_slots, g);
  return pool_alloc(e, g->bytes, &g->off);
}

// Register a reserved group: pick its lane and queue its twiddle tables there.
EngGroup* group_commit(fcgno_engine* e, EngGroup g) {
  g.s = e->lanes[e->next_lane];
  e->next_lane = (e->next_lane + 1) % (int)e->lanes.size();
  if (e->d.op != PID) {
    const NOLaunch NL = group_no(e, g, nullptr, 0);
    char* base = e->pool + g.off;
    const bool bf = e->d.op == PBF;
    launch_tables(NL, (double*)(base + g.E64), base + g.Eacc, base + g.T, base + g.TT, (double*)(base + g.RD),
                  bf ? base + g.FA : nullptr, bf ? base + g.SA : nullptr, bf ? base + g.EX : nullptr);
  }
  return &e->groups.emplace(g.N, g).first->second;
}

void group_close(fcgno_engine* e, int N) {
  auto it = e->groups.find(N);
  if (it == e->groups.end()) return;
  pool_free(e, it->second.off, it->second.bytes);
  e->groups.erase(it);
}

// Set up one admitted request: state, operator inputs, r0 (all stream-ordered).
fcgno_status admit(fcgno_engine* e, EngReq& q, EngGroup& g) {
  const fcgno_model* m = e->d.op == PID ? nullptr : e->m;
  const int N = q.N, op = e->d.op;
  char* base = e->pool + q.off;
  const size_t n = (size_t)N * N;
  const Plan& p = q.p;
  SysDev& sd = q.sd;
  std::memset(&sd, 0, sizeof(SysDev));
  sd.k = (decltype(sd.k))q.k;
  sd.f = (decltype(sd.f))q.f;
  sd.u = (decltype(sd.u))q.u;
  sd.r = (decltype(sd.r))(base + p.r);
  sd.w = op == PID ? sd.r : (decltype(sd.w))(base + p.w);
  sd.P = (decltype(sd.P))(base + p.P);
  sd.S = (decltype(sd.S))(base + p.S);
  sd.st = (decltype(sd.st))(base + p.state);
  sd.hist = (decltype(sd.hist))(base + p.hist);
  sd.part = (decltype(sd.part))(base + p.part);
  sd.n_active = (decltype(sd.n_active))(base + p.counter);
  if (op != PID) {
    std::vector<SysDev> h(1, sd);
    fill_no(m, p, base, N, 1, op, h.data());
    sd = h[0];
  }
  const SysDev* own = (const SysDev*)(base + p.sysdev);
  HIPCHK(hipMemcpyAsync(base + p.sysdev, &sd, sizeof(SysDev), hipMemcpyHostToDevice, g.s));
  KrylovLaunch KL{own, 1, N, e->d.m_max, g.s};
  launch_init_state(KL, q.max_iter, q.rtol);
  if (op != PID) {
    launch_zero(base + p.Hc, (size_t)N * m->arch.width * p.MP * op_esize(op), g.s);
    launch_zero(base + p.Wh, p.wh_bytes_per_sys, g.s);
    NOLaunch NL = group_no(e, g, own, 1);
    launch_no_setup(NL, (double*)(base + p.Gp));
  }
  launch_residual(KL, 0);
  (void)n;
  HIPCHK(hipGetLastError());
  return FCGNO_OK;
}

fcgno_status upload_table(fcgno_engine* e, EngGroup& g, size_t where, const std::vector<int64_t>& ids) {
  std::vector<SysDev> h;
  h.reserve(ids.size());
  for (int64_t id : ids) h.push_back(e->active.at(id).sd);
  HIPCHK(hipMemcpyAsync(e->pool + g.off + where, h.data(), h.size() * sizeof(SysDev), hipMemcpyHostToDevice, g.s));
  // the records' copies of each request's state (a request may have stopped
  // at set-up, which the host has not seen yet)
  launch_sync_records((const SysDev*)(e->pool + g.off + where), (int)h.size(), g.s);
  return FCGNO_OK;
}

}  // namespace fcgno_host

extern "C" size_t fcgno_engine_request_bytes(const fcgno_model* m, const fcgno_engine_desc* d, int32_t n,
                                             int32_t max_iter) {
  if (!d || !sizes_ok(n, 1) || max_iter < 1 || d->m_max < 1 || d->m_max > MAXW) return 0;
  if (d->op != PID && (!m || !arch_ok_for(m, n))) return 0;
  return align256(request_bytes(m, d->op, d->m_max, n, max_iter));
}

extern "C" fcgno_status fcgno_engine_create(const fcgno_model* m, const fcgno_engine_desc* d, void* stream,
                                            fcgno_engine** out) {
  if (!d || !out) return fail(FCGNO_E_INVALID, "null argument");
  if (d->op < 0 || d->op > PID) return fail(FCGNO_E_INVALID, "the engine takes FP64, FP32, BF16 or IDENTITY");
  if (d->op != PID && !m) return fail(FCGNO_E_INVALID, "operator precision needs a model");
  if (d->m_max < 1 || d->m_max > MAXW) return fail(FCGNO_E_INVALID, "m_max must be in 1..32");
  if (d->max_slots < 1 || d->max_slots > MAX_BATCH || d->budget_bytes < 4096)
    return fail(FCGNO_E_INVALID, "need max_slots in 1..65535 and a budget");
  fcgno_engine* e = new fcgno_engine();
  e->m = m;
  e->d = *d;
  if (e->d.check_every <= 0) e->d.check_every = 8;
  e->s = (hipStream_t)stream;
  bool ok = hipEventCreateWithFlags(&e->ready, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < 4; ++i) {
    hipStream_t ls = nullptr;
    ok = hipStreamCreateWithFlags(&ls, hipStreamNonBlocking) == hipSuccess;
    if (ok) e->lanes.push_back(ls);
  }
  if (!ok) {
    for (hipStream_t ls : e->lanes) (void)hipStreamDestroy(ls);
    if (e->ready) (void)hipEventDestroy(e->ready);
    delete e;
    return fail(FCGNO_E_HIP, "cannot create the engine's streams");
  }
  const size_t bytes = d->budget_bytes & ~(size_t)255;
  fcgno_status st = FCGNO_OK;
  if (hipMalloc((void**)&e->pool, bytes) != hipSuccess) {
    e->pool = nullptr;
    st = fail(FCGNO_E_NOMEM, "cannot allocate the engine pool");
  } else if (hipHostMalloc((void**)&e->hflags, (size_t)d->max_slots * 3 * sizeof(int), 0) != hipSuccess ||
             hipHostMalloc((void**)&e->htres, (size_t)d->max_slots * 2 * sizeof(double), 0) != hipSuccess) {
    st = fail(FCGNO_E_HIP, "hipHostMalloc failed");
  }
  if (st != FCGNO_OK) {
    if (e->hflags) (void)hipHostFree(e->hflags);
    if (e->pool) (void)hipFree(e->pool);
    for (hipStream_t ls : e->lanes) (void)hipStreamDestroy(ls);
    (void)hipEventDestroy(e->ready);
    delete e;
    return st;
  }
  e->free_[0] = bytes;
  *out = e;
  return FCGNO_OK;
}

extern "C" fcgno_status fcgno_engine_submit(fcgno_engine* e, int32_t N, const double* k, const double* f, double* u,
                                            double rtol, int32_t max_iter, int64_t* id_out) {
  if (!e || !k || !f || !u || !id_out) return fail(FCGNO_E_INVALID, "null argument");
  if (check_sizes(N, 1) != FCGNO_OK) return FCGNO_E_INVALID;
  if (max_iter < 1 || !(rtol > 0.0) || !std::isfinite(rtol)) return fail(FCGNO_E_INVALID, "bad request");
  if (e->d.op != PID && !arch_ok_for(e->m, N)) return fail(FCGNO_E_INVALID, "need 2*modes <= n");
  EngReq q;
  q.id = e->next_id++;
  q.N = N;
  q.max_iter = max_iter;
  q.rtol = rtol;
  q.k = k;
  q.f = f;
  q.u = u;
  q.p = make_plan(e->d.op == PID ? nullptr : e->m, N, 1, e->d.m_max, max_iter, e->d.op, KIND_SOLVE);
  q.bytes = q.p.total;
  const size_t gb = group_bytes(e->d.op == PID ? nullptr : e->m, e->d.op, N, e->d.max_slots, nullptr);
  if (align256(q.bytes) + align256(gb) > (e->d.budget_bytes & ~(size_t)255))
    return fail(FCGNO_E_NOMEM, "request larger than the engine's HBM budget");
  *id_out = q.id;
  e->queue.push_back(q);
  return FCGNO_OK;
}

extern "C" fcgno_status fcgno_engine_step(fcgno_engine* e, int32_t* n_active, int32_t* n_queued) {
  if (!e) return fail(FCGNO_E_INVALID, "null engine");
  // the caller's prior work on its stream (inputs of new requests) comes first
  HIPCHK(hipEventRecord(e->ready, e->s));
  for (hipStream_t ls : e->lanes) HIPCHK(hipStreamWaitEvent(ls, e->ready, 0));
  // 1. admission: scan the queue in arrival order, admit what fits now
  // A request needs its own pool block and, for a grid size with no group
  // yet, the group's block too.  Both are reserved before any work is queued:
  // a block handed back after queuing work on one lane could be reused at
  // once by a request on another lane while that work is still pending.
  for (auto it = e->queue.begin(); it != e->queue.end();) {
    if ((int)e->active.size() >= e->d.max_slots) break;
    auto git = e->groups.find(it->N);
    const bool new_group = git == e->groups.end();
    EngGroup ng;
    if (new_group && !group_reserve(e, it->N, &ng)) { ++it; continue; }
    size_t off = 0;
    if (!pool_alloc(e, it->bytes, &off)) {
      if (new_group) pool_free(e, ng.off, ng.bytes);
      ++it;
      continue;
    }
    EngGroup* g = new_group ? group_commit(e, ng) : &git->second;
    EngReq q = *it;
    q.off = off;
    it = e->queue.erase(it);
    auto ins = e->active.emplace(q.id, q).first;
    fcgno_status st = admit(e, ins->second, *g);
    if (st != FCGNO_OK) return st;
    g->members.push_back(q.id);
    g->dirty = true;
  }
  // 2. advance every group by K iterations, then export the state summaries
  const int K = e->d.check_every;
  size_t ho = 0;
  for (auto& kv : e->groups) {
    EngGroup& g = kv.second;
    const int G = (int)g.members.size();
    if (G == 0) continue;
    char* base = e->pool + g.off;
    if (g.dirty) {
      fcgno_status st = upload_table(e, g, g.table, g.members);
      if (st != FCGNO_OK) return st;
      g.dirty = false;
    }
    const SysDev* table = (const SysDev*)(base + g.table);
    KrylovLaunch KL{table, G, g.N, e->d.m_max, g.s};
    NOLaunch NL{};
    // the projection layer forms the window sums (no window-sum launch)
    const bool pwd = e->d.op != PID && proj_wdots(g.N, e->d.m_max);
    if (e->d.op != PID) NL = group_no(e, g, table, G);
    NL.wdots = pwd ? 1 : 0;
    KL.wslots = pwd ? proj_wslots(g.N) : 0;
    for (int i = 0; i < K; ++i) {
      if (e->d.op != PID) launch_no_apply(NL);
      if (!pwd) launch_wdots(KL);
      launch_dir(KL);
      launch_update(KL);
    }
    launch_export(table, G, (int*)(base + g.flags), (double*)(base + g.tres), g.s);
    g.hoff = ho;
    HIPCHK(hipMemcpyAsync(e->hflags + 3 * ho, base + g.flags, (size_t)G * 3 * sizeof(int), hipMemcpyDeviceToHost,
                          g.s));
    ho += G;
  }
  HIPCHK(hipGetLastError());
  for (hipStream_t ls : e->lanes) HIPCHK(hipStreamSynchronize(ls));
  // 3. true residual of the requests that stopped, then release them
  bool any = false;
  std::map<int, std::vector<int64_t>> fin;
  for (auto& kv : e->groups) {
    EngGroup& g = kv.second;
    for (size_t b = 0; b < g.members.size(); ++b)
      if (e->hflags[3 * (g.hoff + b)] == 0) fin[kv.first].push_back(g.members[b]);
  }
  ho = 0;
  for (auto& kv : fin) {
    EngGroup& g = e->groups.at(kv.first);
    char* base = e->pool + g.off;
    const int F = (int)kv.second.size();
    g.hoff = ho;
    fcgno_status st = upload_table(e, g, g.ftable, kv.second);
    if (st != FCGNO_OK) return st;
    const SysDev* ft = (const SysDev*)(base + g.ftable);
    KrylovLaunch KF{ft, F, g.N, e->d.m_max, g.s};
    launch_residual(KF, 1);
    launch_export(ft, F, (int*)(base + g.flags), (double*)(base + g.tres), g.s);
    HIPCHK(hipMemcpyAsync(e->hflags + 3 * ho, base + g.flags, (size_t)F * 3 * sizeof(int), hipMemcpyDeviceToHost,
                          g.s));
    HIPCHK(hipMemcpyAsync(e->htres + 2 * ho, base + g.tres, (size_t)F * 2 * sizeof(double), hipMemcpyDeviceToHost,
                          g.s));
    ho += F;
    any = true;
  }
  if (any) {
    HIPCHK(hipGetLastError());
    for (hipStream_t ls : e->lanes) HIPCHK(hipStreamSynchronize(ls));
    for (auto& kv : fin) {
      EngGroup& g = e->groups.at(kv.first);
      for (size_t b = 0; b < kv.second.size(); ++b) {
        const int64_t id = kv.second[b];
        fcgno_engine_result r{};
        r.id = id;
        r.status = e->hflags[3 * (g.hoff + b) + 1];
        r.iters = e->hflags[3 * (g.hoff + b) + 2];
        r.true_rel_res = e->htres[2 * (g.hoff + b)];
        r.true_rel_res_f = e->htres[2 * (g.hoff + b) + 1];
        e->done.push_back(r);
        EngReq& q = e->active.at(id);
        pool_free(e, q.off, q.bytes);
        e->active.erase(id);
        g.members.erase(std::find(g.members.begin(), g.members.end(), id));
        g.dirty = true;
      }
      if (g.members.empty()) group_close(e, kv.first);
    }
  }
  if (n_active) *n_active = (int32_t)e->active.size();
  if (n_queued) *n_queued = (int32_t)e->queue.size();
  return FCGNO_OK;
}

extern "C" int32_t fcgno_engine_poll(fcgno_engine* e, fcgno_engine_result* out, int32_t max_results) {
  if (!e || !out || max_results < 1) return 0;
  const int32_t n = (int32_t)std::min<size_t>(e->done.size(), (size_t)max_results);
  std::copy(e->done.begin(), e->done.begin() + n, out);
  e->done.erase(e->done.begin(), e->done.begin() + n);
  return n;
}

extern "C" void fcgno_engine_destroy(fcgno_engine* e) {
  if (!e) return;
  for (hipStream_t ls : e->lanes) {
    (void)hipStreamSynchronize(ls);
    (void)hipStreamDestroy(ls);
  }
  if (e->ready) (void)hipEventDestroy(e->ready);
  (void)hipHostFree(e->hflags);
  (void)hipHostFree(e->htres);
  (void)hipFree(e->pool);
  delete e;
}

