// C ABI of libfcgno: model lifecycle, workspace planning, the FCG solve
// driver (Algorithm 1), Krylov and residual samples, the standalone operator
// application, error strings.  Training entry points are in train_api.hip,
// the serving engine in serve.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "fcgno.h"
#include "host.h"
#include "prof.h"
#include "train.h"

using namespace fcgno;
using namespace fcgno_host;


extern "C" size_t fcgno_weight_count(const fcgno_arch* a) {
  if (!a || a->layers < 1 || a->width < 1 || a->modes < 1) return 0;
  const size_t C = a->width, M = a->modes, Cin = a->in_channels;
  return C * Cin + C + (size_t)a->layers * (2 * C * C * 2 * M * M + C * C + C) + C + 1;
}

// Lay out the derived arrays once; their contents come from the device blob.
fcgno_status fcgno_host::alloc_derived(fcgno_model* m) {
  const int C = m->arch.width, M = m->arch.modes, L = m->arch.layers;
  Carver cv;
  struct Off { std::vector<size_t> Wf, bias, R; size_t WP, WL0; } off[3];
  for (int p = 0; p < 3; ++p) {
    const int esz = op_esize(p), asz = acc_esize(p), ks = kstep(p);
    off[p].Wf.resize(L); off[p].bias.resize(L); off[p].R.resize(L);
    for (int l = 0; l < L; ++l) {
      const int KWP = l == 0 ? ks : C;
      off[p].Wf[l] = cv.take((size_t)C * KWP * esz);
      off[p].bias[l] = cv.take((size_t)C * asz);
      off[p].R[l] = cv.take((size_t)M * 2 * M * C * C * 2 * asz);
    }
    off[p].WP = cv.take((size_t)C * asz);
    off[p].WL0 = cv.take((size_t)C * asz);
  }
  HIPCHK(hipMalloc((void**)&m->dev, cv.n));
  m->dev_bytes = cv.n;
  HIPCHK(hipMalloc((void**)&m->blob, m->w.size() * sizeof(double)));
  for (int p = 0; p < 3; ++p) {
    m->Wfrag[p].resize(L); m->bias[p].resize(L); m->Rmix[p].resize(L);
    DeriveArgs& d = m->derive[p];
    std::memset(&d, 0, sizeof(d));
    d.blob = m->blob;
    d.C = C; d.M = M; d.L = L; d.kpl = kstep(p) / 4;
    for (int l = 0; l < L; ++l) {
      d.Wfrag[l] = m->dev + off[p].Wf[l];
      d.bias[l] = m->dev + off[p].bias[l];
      d.Rmix[l] = m->dev + off[p].R[l];
      m->Wfrag[p][l] = d.Wfrag[l];
      m->bias[p][l] = d.bias[l];
      m->Rmix[p][l] = d.Rmix[l];
    }
    d.WP = m->dev + off[p].WP;
    d.WL0 = m->dev + off[p].WL0;
    m->WP[p] = d.WP;
    m->WL0[p] = d.WL0;
  }
  return FCGNO_OK;
}

// Derived arrays of every precision from the device blob (stream-ordered).
void fcgno_host::derive_all(fcgno_model* m, hipStream_t s) {
  for (int p = 0; p < 3; ++p) launch_derive(m->derive[p], p, s);
}

fcgno_status fcgno_host::upload_weights(fcgno_model* m) {
  HIPCHK(hipMemcpy(m->blob, m->w.data(), m->w.size() * sizeof(double), hipMemcpyHostToDevice));
  derive_all(m, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipDeviceSynchronize());
  m->host_stale = false;
  return FCGNO_OK;
}


extern "C" fcgno_status fcgno_model_create(const fcgno_arch* arch, const double* weights_host,
                                           size_t n_weights, fcgno_model** out) {
  if (!arch || !weights_host || !out) return fail(FCGNO_E_INVALID, "null argument");
  if (arch->in_channels != 4) return fail(FCGNO_E_INVALID, "in_channels must be 4");
  if (arch->width != 16 && arch->width != 32) return fail(FCGNO_E_INVALID, "width must be 16 or 32");
  if (arch->modes < 1 || arch->modes > 16) return fail(FCGNO_E_INVALID, "modes must be in 1..16");
  if (arch->basis != B_FOURIER && arch->basis != B_SINE) return fail(FCGNO_E_INVALID, "unknown basis");
  if (arch->layers < 1 || arch->layers > 64) return fail(FCGNO_E_INVALID, "layers must be in 1..64");
  if (n_weights != fcgno_weight_count(arch)) return fail(FCGNO_E_INVALID, "weight count mismatch");
  for (size_t i = 0; i < n_weights; ++i)
    if (!std::isfinite(weights_host[i])) return fail(FCGNO_E_INVALID, "non-finite weight");
  fcgno_model* m = new fcgno_model();
  m->arch = *arch;
  m->w.assign(weights_host, weights_host + n_weights);
  fcgno_status s = FCGNO_OK;
  if (hipGetDevice(&m->device) != hipSuccess) s = fail(FCGNO_E_HIP, "hipGetDevice failed");
  if (s == FCGNO_OK) s = alloc_derived(m);
  if (s == FCGNO_OK) s = upload_weights(m);
  if (s != FCGNO_OK) {
    if (m->dev) (void)hipFree(m->dev);
    if (m->blob) (void)hipFree(m->blob);
    delete m;
    return s;
  }
  *out = m;
  return FCGNO_OK;
}

fcgno_status fcgno_host::sync_host(const fcgno_model* mc) {
  fcgno_model* m = const_cast<fcgno_model*>(mc);
  if (!m->host_stale) return FCGNO_OK;
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(m->w.data(), m->blob, m->w.size() * sizeof(double), hipMemcpyDeviceToHost));
  m->host_stale = false;
  return FCGNO_OK;
}

extern "C" fcgno_status fcgno_model_get_weights(const fcgno_model* m, double* wh, size_t n) {
  if (!m || !wh) return fail(FCGNO_E_INVALID, "null argument");
  if (n != m->w.size()) return fail(FCGNO_E_INVALID, "weight count mismatch");
  fcgno_status s = sync_host(m);
  if (s != FCGNO_OK) return s;
  std::memcpy(wh, m->w.data(), n * sizeof(double));
  return FCGNO_OK;
}

extern "C" fcgno_status fcgno_model_set_weights(fcgno_model* m, const double* wh, size_t n) {
  if (!m || !wh) return fail(FCGNO_E_INVALID, "null argument");
  if (n != m->w.size()) return fail(FCGNO_E_INVALID, "weight count mismatch");
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(wh[i])) return fail(FCGNO_E_INVALID, "non-finite weight");
  m->w.assign(wh, wh + n);
  return upload_weights(m);
}

extern "C" void fcgno_model_destroy(fcgno_model* m) {
  if (!m) return;
  if (m->dev) (void)hipFree(m->dev);
  if (m->blob) (void)hipFree(m->blob);
  delete m;
}

// ---------------------------------------------------------------------------
// Workspace plans
// ---------------------------------------------------------------------------
namespace fcgno_host {

size_t part_blocks(int N) { return (size_t)pslot_stride(N); }

// backward kernel geometry: Sb row segments of TPW tiles per row, nbs = N Sb
// row segments per system (one wave each)
void bwd_geometry(int N, int prec, int& Sb, int& nbs) {
  (void)prec;
  Sb = seg_count(N);
  nbs = N * Sb;
}

Plan make_plan(const fcgno_model* m, int N, int B, int m_max, int max_iter, int op, int kind) {
  Plan p;
  Carver cv;
  const size_t n = (size_t)N * N;
  p.n_part_blocks = part_blocks(N);
  p.sysdev = cv.take((size_t)B * sizeof(SysDev));
  p.state = cv.take((size_t)B * sizeof(SysState));
  p.counter = cv.take(MAX_SUB * sizeof(int));   // one active-system count per sub-batch
  p.part = cv.take((size_t)B * p.n_part_blocks * NQ * sizeof(double));
  if (kind == KIND_SOLVE) {
    p.sysdev2 = cv.take((size_t)B * sizeof(SysDev));   // compacted launch table
    p.idle = cv.take(sizeof(SysState));
    p.hist = cv.take((size_t)B * (max_iter + 1) * sizeof(double));
    p.r = cv.take((size_t)B * n * 8);
    p.P = cv.take((size_t)B * (m_max + 1) * n * 8);
    p.S = cv.take((size_t)B * (m_max + 1) * n * 8);
    p.w = op != PID ? cv.take((size_t)B * n * 8) : 0;
    p.tmp = op == PJAC ? cv.take((size_t)B * n * 8) : 0;
  }
  if (is_no(op) && m) {
    const int C = m->arch.width, M = m->arch.modes, L = m->arch.layers;
    const int MP = round16(2 * M), NP = round16(N);
    const int nyt = NP / 16;
    const int S = seg_count(N);
    const int esz = op_esize(op), asz = acc_esize(op);
    if (kind == KIND_TRAIN) {
      bwd_geometry(N, op, p.Sb, p.nbs);
      p.nblk = (int)(((size_t)B * p.nbs + 3) / 4);   // four row segments per block
    }
    p.S_seg = S;
    p.MP = MP;
    p.act_slots = kind == KIND_TRAIN ? std::max(1, L - 1) : 1;
    p.act = cv.take((size_t)p.act_slots * B * n * C * esz);
    p.logk = cv.take((size_t)B * n * esz);
    p.Gr = cv.take((size_t)B * N * MP * 8);
    p.gp_bytes_per_sys = std::max((size_t)N * std::max(S, p.Sb) * MP * C * asz, (size_t)4 * N * MP * 8);
    p.Gp = cv.take((size_t)B * p.gp_bytes_per_sys);
    p.Hc = cv.take((size_t)B * N * C * MP * esz);
    p.Vc = cv.take((size_t)B * C * 2 * M * M * 2 * asz);
    p.wh_bytes_per_sys = (size_t)C * MP * M * 2 * asz;
    p.Wh = cv.take((size_t)B * p.wh_bytes_per_sys);
    const int XS = (N + 63) / 64;
    p.vp_bytes_per_sys = (size_t)M * XS * C * 2 * M * 2 * asz;
    p.Vp = cv.take((size_t)B * p.vp_bytes_per_sys);
    p.E64 = cv.take((size_t)tw_period(m->arch.basis, N) * 2 * 8);
    p.Eacc = cv.take((size_t)tw_period(m->arch.basis, N) * 2 * asz);
    p.T = cv.take((size_t)NP * MP * esz);
    p.TT = cv.take((size_t)MP * NP * esz);
    p.RD = cv.take((size_t)NP * 32 * 8);
    if (op == PBF) {
      // matrix-core x transforms: split-bfloat16 twiddle operands and the
      // synthesis operand of each system (see the bfloat16 spectral kernels)
      p.FA = cv.take((size_t)2 * 32 * 2 * NP * 2);
      p.SA = cv.take((size_t)2 * NP * 64 * 2);
      p.EX = cv.take((size_t)NP * 32 * 8);
      p.wt_bytes_per_sys = (size_t)2 * C * M * 64 * 2;
      p.WT = cv.take((size_t)B * p.wt_bytes_per_sys);
    }
    if (kind == KIND_TRAIN) {
      const size_t vs = (size_t)M * C * 2 * M * 2;
      p.z = cv.take((size_t)L * B * n * C * esz);
      p.vsave = cv.take((size_t)L * B * vs * asz);
      p.tw = cv.take((size_t)B * n * 8);
      p.gw = cv.take((size_t)B * n * 8);
      p.dvec = cv.take((size_t)B * n * 8);
      p.dzA = cv.take((size_t)B * n * C * asz);
      p.dzB = cv.take((size_t)B * n * C * asz);
      p.Gh = cv.take((size_t)B * vs * asz);
      p.gscale = cv.take((size_t)B * 8);
      p.loss = cv.take((size_t)B * 8);
      p.loss_nb = (int)((n + FLAT_PTS - 1) / FLAT_PTS);
      p.lpart = cv.take((size_t)B * p.loss_nb * 2 * 8);
      p.pdW = cv.take((size_t)p.nblk * C * C * asz);
      p.pdb = cv.take((size_t)p.nblk * C * asz);
      p.pdWP = cv.take((size_t)p.nblk * C * asz);
      p.pdbP = cv.take((size_t)p.nblk * asz);
      p.pdWL = cv.take((size_t)p.nblk * C * 4 * asz);
      p.pdbL = cv.take((size_t)p.nblk * C * asz);
      p.grad = cv.take(m->w.size() * 8);
      p.rstage = cv.take((size_t)REDUCE_CHUNKS * C * C * 8);
    }
  }
  p.total = cv.n;
  return p;
}

bool arch_ok_for(const fcgno_model* m, int N) { return m && 2 * m->arch.modes <= N; }

// Fill the per-system operator pointers of a plan.
void fill_no(const fcgno_model* m, const Plan& p, char* base, int N, int B, int op, SysDev* h) {
  const int C = m->arch.width, M = m->arch.modes, MP = p.MP;
  const size_t n = (size_t)N * N;
  const int esz = op_esize(op), asz = acc_esize(op);
  for (int b = 0; b < B; ++b) {
    h[b].act = (decltype(h[b].act))(base + p.act + (size_t)b * n * C * esz);
    h[b].act_stride = (size_t)B * n * C;   // elements between activation slots
    h[b].logk = (decltype(h[b].logk))(base + p.logk + (size_t)b * n * esz);
    h[b].Gr = (decltype(h[b].Gr))((double*)(base + p.Gr) + (size_t)b * N * MP);
    h[b].Gp = (decltype(h[b].Gp))(base + p.Gp + (size_t)b * p.gp_bytes_per_sys);
    h[b].Hc = (decltype(h[b].Hc))(base + p.Hc + (size_t)b * N * C * MP * esz);
    h[b].Vc = (decltype(h[b].Vc))(base + p.Vc + (size_t)b * C * 2 * M * M * 2 * asz);
    h[b].Wh = (decltype(h[b].Wh))(base + p.Wh + (size_t)b * p.wh_bytes_per_sys);
    h[b].Vp = (decltype(h[b].Vp))(base + p.Vp + (size_t)b * p.vp_bytes_per_sys);
    h[b].WT = p.wt_bytes_per_sys ? (decltype(h[b].WT))(base + p.WT + (size_t)b * p.wt_bytes_per_sys) : nullptr;
  }
}

NOLaunch make_no(const fcgno_model* m, const Plan& p, char* base, const SysDev* sysdev, int N, int B, int op,
                 hipStream_t s) {
  NOLaunch L{};
  L.sys = sysdev;
  L.nsys = B;
  L.N = N;
  L.C = m->arch.width;
  L.M = m->arch.modes;
  L.MP = p.MP;
  L.L = m->arch.layers;
  L.S = p.S_seg;
  L.spw = SPW_HIGH;
  L.prec = op;
  L.basis = m->arch.basis;
  L.tab.E64 = (const double*)(base + p.E64);
  L.tab.Eacc = base + p.Eacc;
  L.tab.T = base + p.T;
  L.tab.TT = base + p.TT;
  L.tab.FA = op == PBF ? base + p.FA : nullptr;
  L.tab.SA = op == PBF ? base + p.SA : nullptr;
  L.tab.RD = (const double*)(base + p.RD);
  L.tab.EX = op == PBF ? base + p.EX : nullptr;
  L.Wfrag = m->Wfrag[op].data();
  L.bias = m->bias[op].data();
  L.Rmix = m->Rmix[op].data();
  L.WP = m->WP[op];
  L.bP = dev_bP(m);
  L.WL0 = m->WL0[op];
  L.WL = dev_WL(m);
  L.bL = dev_bL(m);
  L.stream = s;
  L.op_bytes = op_esize(op);
  L.acc_bytes = acc_esize(op);
  return L;
}

// Operator set-up shared by every kind: tables, log k, constant layer-0 spectrum.
fcgno_status operator_setup(const fcgno_model* m, const Plan& p, char* base, const NOLaunch& NL, int N, int B,
                            int op, hipStream_t s) {
  launch_zero(base + p.Hc, (size_t)B * N * m->arch.width * p.MP * op_esize(op), s);
  launch_zero(base + p.Wh, (size_t)B * p.wh_bytes_per_sys, s);
  launch_tables(NL, (double*)(base + p.E64), base + p.Eacc, base + p.T, base + p.TT, (double*)(base + p.RD),
                op == PBF ? base + p.FA : nullptr, op == PBF ? base + p.SA : nullptr,
                op == PBF ? base + p.EX : nullptr);
  launch_no_setup(NL, (double*)(base + p.Gp));
  return FCGNO_OK;
}

fcgno_status check_desc(const fcgno_model* m, const fcgno_solve_desc* d) {
  if (!d) return fail(FCGNO_E_INVALID, "null descriptor");
  if (check_sizes(d->n, d->batch) != FCGNO_OK) return FCGNO_E_INVALID;
  if (d->m_max < 1 || d->m_max > MAXW) return fail(FCGNO_E_INVALID, "m_max must be in 1..32");
  if (d->max_iter < 1) return fail(FCGNO_E_INVALID, "max_iter must be >= 1");
  if (!(d->rtol > 0.0) || !std::isfinite(d->rtol)) return fail(FCGNO_E_INVALID, "rtol must be > 0");
  if (d->op < 0 || d->op > PSGS) return fail(FCGNO_E_INVALID, "unknown op");
  if ((d->op == PJAC || d->op == PSGS) && (d->precond_steps < 1 || d->precond_steps > 1000))
    return fail(FCGNO_E_INVALID, "precond_steps must be in 1..1000 for JACOBI and SGS_RB");
  if (d->streams < 0 || d->streams > MAX_SUB) return fail(FCGNO_E_INVALID, "streams must be in 0..8");
  if (is_no(d->op)) {
    if (!m) return fail(FCGNO_E_INVALID, "operator precision needs a model");
    if (!arch_ok_for(m, d->n)) return fail(FCGNO_E_INVALID, "need 2*modes <= n");
  }
  if ((double)d->n * d->n * d->batch > 4.0e9) return fail(FCGNO_E_INVALID, "problem too large");
  return FCGNO_OK;
}

}  // namespace fcgno_host

extern "C" size_t fcgno_solve_workspace_bytes(const fcgno_model* m, const fcgno_solve_desc* d) {
  if (check_desc(m, d) != FCGNO_OK) return 0;
  return make_plan(m, d->n, d->batch, d->m_max, d->max_iter, d->op, KIND_SOLVE).total;
}

namespace fcgno_host {
struct Record {
  int m;
  double* rec_r;
  double* rec_e;
  const double* ustar;
};

// Library-owned streams for sub-batched solves: created on first use on each
// device (non-blocking, default priority) and kept until the process ends.
// Solves issued from several host threads on one device share them (their
// sub-batches then run one after another on each stream).
std::mutex g_sub_mutex;
std::map<int, std::vector<hipStream_t>> g_sub_streams;

fcgno_status sub_streams(int count, std::vector<hipStream_t>& out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_sub_mutex);
  std::vector<hipStream_t>& v = g_sub_streams[dev];
  while ((int)v.size() < count) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
      return fail(FCGNO_E_HIP, "stream creation failed");
    v.push_back(st);
  }
  out.assign(v.begin(), v.begin() + count);
  return FCGNO_OK;
}

// While a solve is forked, an early return (a failed HIP call) must not leave
// work that reads the caller's buffers running on the library streams.
struct ForkGuard {
  const std::vector<hipStream_t>* ss = nullptr;
  bool forked = false;
  ~ForkGuard() {
    if (forked)
      for (hipStream_t st : *ss) (void)hipStreamSynchronize(st);
  }
};

// Events of one fork/join, destroyed on every return path.
struct EventSet {
  std::vector<hipEvent_t> ev;
  fcgno_status make(int count) {
    for (int i = 0; i < count; ++i) {
      hipEvent_t e = nullptr;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return fail(FCGNO_E_HIP, "event creation failed");
      ev.push_back(e);
    }
    return FCGNO_OK;
  }
  ~EventSet() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

// Pinned host slots for the overlapped convergence polls of one host thread
// (two chunks' active counts) and their events; created on first use and
// kept (like the library streams, never released: a release at process exit
// could run after the HIP runtime has gone).  nullptr if pinned memory or
// events are unavailable: the solve then polls synchronously.
struct PollBuf {
  int* count = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int device = -1;
};
PollBuf* poll_buffer() {
  thread_local PollBuf pb;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  if (pb.count && pb.device == dev) return &pb;
  if (pb.count) {   // events belong to the device that created them
    for (hipEvent_t& e : pb.ev)
      if (e) (void)hipEventDestroy(e), e = nullptr;
    (void)hipHostFree(pb.count);
    pb.count = nullptr;
  }
  if (hipHostMalloc((void**)&pb.count, 2 * MAX_SUB * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    pb.count = nullptr;
    return nullptr;
  }
  for (hipEvent_t& e : pb.ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      return nullptr;
    }
  pb.device = dev;
  return &pb;
}

fcgno_status solve_impl(const fcgno_model* m, const fcgno_solve_desc* d, const double* k, const double* f,
                        double* u, double* r_out, int32_t* iters, int32_t* sys_status, double* rel_hist,
                        double* true_rel_res, double* true_rel_res_f, void* ws, size_t ws_bytes, void* stream,
                        const Record* rec) {
  fcgno_status cs = check_desc(m, d);
  if (cs != FCGNO_OK) return cs;
  if (!k || !f || !u || !iters || !sys_status || !ws) return fail(FCGNO_E_INVALID, "null pointer argument");
  const int N = d->n, B = d->batch, op = d->op;
  const Plan p = make_plan(m, N, B, d->m_max, d->max_iter, op, KIND_SOLVE);
  if (ws_bytes < p.total) return fail(FCGNO_E_NOMEM, "workspace too small");
  if (((uintptr_t)ws & 255u) != 0) return fail(FCGNO_E_INVALID, "workspace must be 256-byte aligned");
  char* base = (char*)ws;
  hipStream_t s = (hipStream_t)stream;
  const size_t n = (size_t)N * N;
  std::vector<SysDev> h(B);
  SysState* st = (SysState*)(base + p.state);
  int* counter = (int*)(base + p.counter);
  // sub-batch g holds systems [b0[g], b0[g+1]) and counts its active systems in counter[g]
  const int G = rec ? 1 : std::max(1, std::min(d->streams, B));
  std::vector<int> b0(G + 1);
  for (int g = 0; g <= G; ++g) b0[g] = (int)(((long long)g * B) / G);
  int grp = 0;
  for (int b = 0; b < B; ++b) {
    while (b >= b0[grp + 1]) ++grp;
    SysDev& sd = h[b];
    std::memset(&sd, 0, sizeof(SysDev));
    sd.k = (decltype(sd.k))(k + (size_t)b * (N + 2) * (N + 2));
    sd.f = (decltype(sd.f))(f + (size_t)b * n);
    sd.u = (decltype(sd.u))(u + (size_t)b * n);
    sd.r = (decltype(sd.r))(r_out ? r_out + (size_t)b * n : (double*)(base + p.r) + (size_t)b * n);
    sd.w = op == PID ? sd.r : (decltype(sd.w))((double*)(base + p.w) + (size_t)b * n);
    sd.P = (decltype(sd.P))((double*)(base + p.P) + (size_t)b * (d->m_max + 1) * n);
    sd.S = (decltype(sd.S))((double*)(base + p.S) + (size_t)b * (d->m_max + 1) * n);
    sd.st = (decltype(sd.st))(st + b);
    sd.hist = (decltype(sd.hist))((double*)(base + p.hist) + (size_t)b * (d->max_iter + 1));
    sd.part = (decltype(sd.part))((double*)(base + p.part) + (size_t)b * p.n_part_blocks * NQ);
    sd.n_active = (decltype(sd.n_active))(counter + grp);
    if (op == PJAC) sd.tmp = (decltype(sd.tmp))((double*)(base + p.tmp) + (size_t)b * n);
  }
  if (is_no(op)) fill_no(m, p, base, N, B, op, h.data());
  const SysDev* sysdev = (const SysDev*)(base + p.sysdev);
  HIPCHK(hipMemcpyAsync(base + p.sysdev, h.data(), B * sizeof(SysDev), hipMemcpyHostToDevice, s));
  KrylovLaunch KL{sysdev, B, N, d->m_max, s};
  // neural-operator solves: the projection layer forms the window sums
  const bool pwd = is_no(op) && proj_wdots(N, d->m_max);
  KL.wslots = pwd ? proj_wslots(N) : 0;
  for (int g = 0; g < G; ++g) {
    KrylovLaunch KLg{sysdev + b0[g], b0[g + 1] - b0[g], N, d->m_max, s};
    launch_init_state(KLg, d->max_iter, d->rtol);
  }
  NOLaunch NL{};
  if (is_no(op)) {
    NL = make_no(m, p, base, sysdev, N, B, op, s);
    NL.wdots = pwd ? 1 : 0;
    fcgno_status os = operator_setup(m, p, base, NL, N, B, op, s);
    if (os != FCGNO_OK) return os;
  }
  launch_residual(KL, 0);
  HIPCHK(hipGetLastError());
  // iterations: each sub-batch on its own stream (the caller's when G == 1)
  std::vector<hipStream_t> ss(G, s);
  EventSet events;
  ForkGuard guard;
  guard.ss = &ss;
  if (G > 1) {
    fcgno_status es = sub_streams(G, ss);
    if (es == FCGNO_OK) es = events.make(G + 1);
    if (es != FCGNO_OK) return es;
    HIPCHK(hipEventRecord(events.ev[G], s));
    guard.forked = true;
    for (int g = 0; g < G; ++g) HIPCHK(hipStreamWaitEvent(ss[g], events.ev[G], 0));
  }
  std::vector<KrylovLaunch> KLs(G);
  std::vector<NOLaunch> NLs(G, NL);
  std::vector<int> nact(G), hn(G);
  for (int g = 0; g < G; ++g) {
    KLs[g] = KrylovLaunch{sysdev + b0[g], b0[g + 1] - b0[g], N, d->m_max, ss[g]};
    KLs[g].wslots = pwd ? proj_wslots(N) : 0;
    NLs[g].sys = sysdev + b0[g];
    NLs[g].nsys = b0[g + 1] - b0[g];
    NLs[g].stream = ss[g];
    nact[g] = b0[g + 1] - b0[g];
  }
  const int K = d->check_every > 0 ? d->check_every : (N >= 256 ? 4 : 8);
  // Sub-batches pay off while they keep many systems busy; once fewer than
  // SUB_MIN_ACTIVE systems per sub-batch remain on average, the streams join
  // and the rest of the solve runs as one launch sequence on the caller's
  // stream (stopped systems leave their blocks at once, so this is exact).
  constexpr int SUB_MIN_ACTIVE = 3;
  bool split = G > 1;
  NOLaunch NL1 = NL;
  KrylovLaunch KL1 = KL;
  int it = 0;
  int active = B;   // active systems at the last poll
  // Once systems stop, the single-stream launches run on a compacted table
  // of the active systems' records (rebuilt on the device, in stream order,
  // whenever the polled count drops), sized to the last polled count, which
  // bounds the true one.  Not with recording, whose output is indexed by
  // the launch slot.
  SysDev* sysdev2 = (SysDev*)(base + p.sysdev2);
  SysState* idle = (SysState*)(base + p.idle);
  const bool compact = rec == nullptr;
  int launched = B;
  if (compact) launch_zero(idle, sizeof(SysState), s);
  auto shrink = [&]() {
    if (!compact || active >= launched) return;
    launch_compact(sysdev, B, sysdev2, idle, s);
    launched = active;
    KL1.sys = sysdev2;
    KL1.nsys = active;
    NL1.sys = sysdev2;
    NL1.nsys = active;
  };
  // Single-stream polling overlaps the device: after queuing a chunk the host
  // reads the previous chunk's active count (copied into pinned memory behind
  // that chunk), so the device starts the next chunk while the host waits.  A
  // chunk queued after every system stopped runs only the kernels' early
  // exits.
  PollBuf* pb = poll_buffer();
  int pending = -1, chunks = 0;
  while (it < d->max_iter) {
    const int end = std::min(d->max_iter, it + K);
    if (!split && pb) {
      shrink();
      if (is_no(op)) NL1.spw = active <= LOW_ACTIVE ? 1 : SPW_HIGH;
      for (int i = it; i < end; ++i) {
        if (is_no(op)) launch_no_apply(NL1);
        else if (op == PJAC) launch_jacobi(KL1, d->precond_steps);
        else if (op == PSGS) launch_rbsgs(KL1, d->precond_steps);
        if (!pwd) launch_wdots(KL1);
        launch_dir(KL1);
        launch_update(KL1);
        if (rec && i < rec->m) launch_record(KL, i, rec->m, rec->rec_r, rec->rec_e, rec->ustar);
      }
      it = end;
      HIPCHK(hipGetLastError());
      const int slot = chunks++ & 1;
      HIPCHK(hipMemcpyAsync(pb->count + slot * MAX_SUB, counter, G * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipEventRecord(pb->ev[slot], s));
      if (pending >= 0) {
        HIPCHK(hipEventSynchronize(pb->ev[pending]));
        int total = 0;
        for (int g = 0; g < G; ++g) total += std::max(pb->count[pending * MAX_SUB + g], 0);
        if (total <= 0) break;
        active = total;
      }
      pending = slot;
      continue;
    }
    if (!split) {
      shrink();
      // few systems left: one row segment per wave (more, shorter waves keep
      // more of the chip busy); the same bits either way
      if (is_no(op)) NL1.spw = active <= LOW_ACTIVE ? 1 : SPW_HIGH;
      for (int i = it; i < end; ++i) {
        if (is_no(op)) launch_no_apply(NL1);
        else if (op == PJAC) launch_jacobi(KL1, d->precond_steps);
        else if (op == PSGS) launch_rbsgs(KL1, d->precond_steps);
        if (!pwd) launch_wdots(KL1);
        launch_dir(KL1);
        launch_update(KL1);
        if (rec && i < rec->m) launch_record(KL, i, rec->m, rec->rec_r, rec->rec_e, rec->ustar);
      }
      it = end;
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(hn.data(), counter, G * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      int total = 0;
      for (int g = 0; g < G; ++g) total += std::max(hn[g], 0);
      if (total <= 0) break;
      active = total;
      continue;
    }
    for (int g = 0; g < G; ++g) {
      if (nact[g] <= 0) continue;
      for (int i = it; i < end; ++i) {
        if (is_no(op)) launch_no_apply(NLs[g]);
        else if (op == PJAC) launch_jacobi(KLs[g], d->precond_steps);
        else if (op == PSGS) launch_rbsgs(KLs[g], d->precond_steps);
        if (!pwd) launch_wdots(KLs[g]);
        launch_dir(KLs[g]);
        launch_update(KLs[g]);
        if (rec && i < rec->m) launch_record(KLs[g], i, rec->m, rec->rec_r, rec->rec_e, rec->ustar);
      }
    }
    it = end;
    HIPCHK(hipGetLastError());
    for (int g = 0; g < G; ++g)
      if (nact[g] > 0) HIPCHK(hipMemcpyAsync(&hn[g], counter + g, sizeof(int), hipMemcpyDeviceToHost, ss[g]));
    int total = 0;
    for (int g = 0; g < G; ++g) {
      if (nact[g] <= 0) continue;
      HIPCHK(hipStreamSynchronize(ss[g]));
      nact[g] = hn[g];
      total += std::max(nact[g], 0);
    }
    if (total <= 0) break;
    if (total < SUB_MIN_ACTIVE * G) {
      // join: the caller's stream continues after every sub-batch's work
      for (int g = 0; g < G; ++g) {
        HIPCHK(hipEventRecord(events.ev[g], ss[g]));
        HIPCHK(hipStreamWaitEvent(s, events.ev[g], 0));
      }
      split = false;
      guard.forked = false;
    }
  }
  if (split) {
    for (int g = 0; g < G; ++g) {
      HIPCHK(hipEventRecord(events.ev[g], ss[g]));
      HIPCHK(hipStreamWaitEvent(s, events.ev[g], 0));
    }
    guard.forked = false;
  }
  launch_residual(KL, 1);
  HIPCHK(hipGetLastError());
  std::vector<SysState> hs(B);
  HIPCHK(hipMemcpyAsync(hs.data(), st, B * sizeof(SysState), hipMemcpyDeviceToHost, s));
  std::vector<double> hh;
  if (rel_hist) {
    hh.resize((size_t)B * (d->max_iter + 1));
    HIPCHK(hipMemcpyAsync(hh.data(), base + p.hist, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  if (prof_on()) prof_collect();
  bool all_ok = true;
  for (int b = 0; b < B; ++b) {
    iters[b] = hs[b].iters;
    sys_status[b] = hs[b].status;
    if (hs[b].status != S_OK) all_ok = false;
    if (true_rel_res) true_rel_res[b] = hs[b].tres;
    if (true_rel_res_f) true_rel_res_f[b] = hs[b].tresf;
    if (rel_hist) {
      const int upto = hs[b].status == S_NONFINITE ? 0 : hs[b].iters;
      for (int i = 0; i <= upto; ++i)
        rel_hist[(size_t)b * (d->max_iter + 1) + i] = hh[(size_t)b * (d->max_iter + 1) + i];
    }
  }
  return all_ok ? FCGNO_OK : FCGNO_NOT_CONVERGED;
}
}  // namespace fcgno_host

extern "C" fcgno_status fcgno_solve(const fcgno_model* m, const fcgno_solve_desc* d, const double* k,
                                    const double* f, double* u, double* r_out, int32_t* iters,
                                    int32_t* sys_status, double* rel_hist, double* true_rel_res,
                                    double* true_rel_res_f, void* ws, size_t ws_bytes, void* stream) {
  return solve_impl(m, d, k, f, u, r_out, iters, sys_status, rel_hist, true_rel_res, true_rel_res_f, ws, ws_bytes,
                    stream, nullptr);
}

extern "C" size_t fcgno_krylov_samples_workspace_bytes(int32_t n, int32_t batch, int32_t max_iter) {
  if (!sizes_ok(n, batch) || max_iter < 1) return 0;
  const size_t sol = make_plan(nullptr, n, batch, 1, max_iter, PID, KIND_SOLVE).total;
  return sol + align256((size_t)batch * n * n * 8) * 2;
}

extern "C" fcgno_status fcgno_krylov_samples(int32_t N, int32_t B, int32_t m_iter, int32_t max_iter,
                                             const double* k, const double* f, const double* u0, double* r_out,
                                             double* e_out, void* ws, size_t ws_bytes, void* stream) {
  if (check_sizes(N, B) != FCGNO_OK) return FCGNO_E_INVALID;
  if (m_iter < 1 || max_iter < 1 || !k || !f || !u0 || !r_out || !e_out || !ws)
    return fail(FCGNO_E_INVALID, "invalid argument");
  if (ws_bytes < fcgno_krylov_samples_workspace_bytes(N, B, std::max(max_iter, m_iter)))
    return fail(FCGNO_E_NOMEM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const size_t n = (size_t)N * N;
  char* base = (char*)ws;
  const size_t sol = make_plan(nullptr, N, B, 1, std::max(max_iter, m_iter), PID, KIND_SOLVE).total;
  double* ustar = (double*)(base + sol);
  double* ucur = (double*)(base + sol + align256((size_t)B * n * 8));
  std::vector<int32_t> it(B), st(B);
  // u* = A^-1 f by conjugate gradients to a tight tolerance
  HIPCHK(hipMemcpyAsync(ustar, u0, (size_t)B * n * 8, hipMemcpyDeviceToDevice, s));
  fcgno_solve_desc d1{N, B, 1, max_iter, 1e-13, PID, 0};
  fcgno_status r1 = solve_impl(nullptr, &d1, k, f, ustar, nullptr, it.data(), st.data(), nullptr, nullptr, nullptr, ws, sol,
                               stream, nullptr);
  if (r1 < 0) return r1;
  // the recorded CG run (FCG with B = I, window 1) from u0
  HIPCHK(hipMemcpyAsync(ucur, u0, (size_t)B * n * 8, hipMemcpyDeviceToDevice, s));
  fcgno_solve_desc d2{N, B, 1, m_iter, 1e-300, PID, m_iter};
  Record rec{m_iter, r_out, e_out, ustar};
  fcgno_status r2 = solve_impl(nullptr, &d2, k, f, ucur, nullptr, it.data(), st.data(), nullptr, nullptr, nullptr, ws, sol,
                               stream, &rec);
  if (r2 < 0) return r2;
  return r1;
}

extern "C" fcgno_status fcgno_residual_samples(int32_t N, int32_t B, int32_t max_iter, const double* k,
                                               const double* f, const double* u, double* r_out, double* e_out,
                                               void* ws, size_t ws_bytes, void* stream) {
  if (check_sizes(N, B) != FCGNO_OK) return FCGNO_E_INVALID;
  if (max_iter < 1 || !k || !f || !u || !r_out || !e_out || !ws)
    return fail(FCGNO_E_INVALID, "invalid argument");
  if (ws_bytes < fcgno_krylov_samples_workspace_bytes(N, B, max_iter))
    return fail(FCGNO_E_NOMEM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const size_t n = (size_t)N * N;
  char* base = (char*)ws;
  const Plan p = make_plan(nullptr, N, B, 1, max_iter, PID, KIND_SOLVE);
  double* ustar = (double*)(base + p.total);
  std::vector<int32_t> it(B), st(B);
  // A^-1 f by conjugate gradients to a tight tolerance, starting from u
  HIPCHK(hipMemcpyAsync(ustar, u, (size_t)B * n * 8, hipMemcpyDeviceToDevice, s));
  fcgno_solve_desc d1{N, B, 1, max_iter, 1e-13, PID, 0};
  fcgno_status r1 = solve_impl(nullptr, &d1, k, f, ustar, nullptr, it.data(), st.data(), nullptr, nullptr, nullptr,
                               ws, p.total, stream, nullptr);
  if (r1 < 0) return r1;
  // r = f - A u into r_out, then e = A^-1 f - u (state and partials reused from the plan)
  std::vector<SysDev> h(B);
  for (int b = 0; b < B; ++b) {
    SysDev& sd = h[b];
    std::memset(&sd, 0, sizeof(SysDev));
    sd.k = (decltype(sd.k))(k + (size_t)b * (N + 2) * (N + 2));
    sd.f = (decltype(sd.f))(f + (size_t)b * n);
    sd.u = (decltype(sd.u))(const_cast<double*>(u) + (size_t)b * n);
    sd.r = (decltype(sd.r))(r_out + (size_t)b * n);
    sd.st = (decltype(sd.st))((SysState*)(base + p.state) + b);
    // the initial-residual kernels also write the history's first entry
    sd.hist = (decltype(sd.hist))((double*)(base + p.hist) + (size_t)b * (max_iter + 1));
    sd.part = (decltype(sd.part))((double*)(base + p.part) + (size_t)b * p.n_part_blocks * NQ);
    sd.n_active = (decltype(sd.n_active))(base + p.counter);
  }
  HIPCHK(hipMemcpyAsync(base + p.sysdev, h.data(), B * sizeof(SysDev), hipMemcpyHostToDevice, s));
  KrylovLaunch KL{(const SysDev*)(base + p.sysdev), B, N, 1, s};
  launch_init_state(KL, 1, 1.0);
  launch_residual(KL, 0);
  launch_record(KL, 0, 1, r_out, e_out, ustar);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return r1;
}

// ---------------------------------------------------------------------------
// Operator application (and the training forward, which also saves z and V^)
// ---------------------------------------------------------------------------
namespace fcgno_host {

fcgno_status operator_forward(const fcgno_model* m, const Plan& p, char* base, int N, int B, int op,
                              const double* k, const double* r, double* w, bool train, hipStream_t s,
                              SysDev* table) {
  const size_t n = (size_t)N * N;
  std::vector<SysDev> own;
  if (!table) {
    own.resize(B);
    table = own.data();
  }
  SysDev* h = table;
  SysState* st = (SysState*)(base + p.state);
  for (int b = 0; b < B; ++b) {
    SysDev& sd = h[b];
    std::memset(&sd, 0, sizeof(SysDev));
    sd.k = (decltype(sd.k))(k + (size_t)b * (N + 2) * (N + 2));
    sd.r = (decltype(sd.r))(const_cast<double*>(r) + (size_t)b * n);
    sd.w = (decltype(sd.w))(w + (size_t)b * n);
    sd.st = (decltype(sd.st))(st + b);
    sd.part = (decltype(sd.part))((double*)(base + p.part) + (size_t)b * p.n_part_blocks * NQ);
    sd.n_active = (decltype(sd.n_active))((int*)(base + p.counter));
  }
  fill_no(m, p, base, N, B, op, h);
  const SysDev* sysdev = (const SysDev*)(base + p.sysdev);
  HIPCHK(hipMemcpyAsync(base + p.sysdev, h, B * sizeof(SysDev), hipMemcpyHostToDevice, s));
  KrylovLaunch KL{sysdev, B, N, 1, s};
  launch_init_state(KL, 1, 1.0);
  NOLaunch NL = make_no(m, p, base, sysdev, N, B, op, s);
  fcgno_status os = operator_setup(m, p, base, NL, N, B, op, s);
  if (os != FCGNO_OK) return os;
  launch_rnorm(KL);
  if (train) {
    const int C = m->arch.width, M = m->arch.modes;
    NL.zsave = base + p.z;
    NL.z_sys = n * C;
    NL.z_layer = (size_t)B * n * C;
    NL.vsave = base + p.vsave;
    NL.vs_sys = (size_t)M * C * 2 * M * 2;
    NL.vs_layer = (size_t)B * NL.vs_sys;
    ProfScope ps(PK_TRAIN_FWD, s);
    launch_no_apply(NL);
  } else {
    launch_no_apply(NL);
  }
  HIPCHK(hipGetLastError());
  return FCGNO_OK;
}

}  // namespace fcgno_host

extern "C" size_t fcgno_precond_workspace_bytes(const fcgno_model* m, int32_t n, int32_t batch, int32_t op) {
  if (!m || !sizes_ok(n, batch) || op < 0 || op >= PID || !arch_ok_for(m, n)) return 0;
  return make_plan(m, n, batch, 1, 1, op, KIND_APPLY).total;
}

extern "C" fcgno_status fcgno_precond_apply(const fcgno_model* m, int32_t N, int32_t B, int32_t op,
                                            const double* k, const double* r, double* w, void* ws,
                                            size_t ws_bytes, void* stream) {
  if (!m || !k || !r || !w || !ws) return fail(FCGNO_E_INVALID, "null pointer argument");
  if (check_sizes(N, B) != FCGNO_OK) return FCGNO_E_INVALID;
  if (op < 0 || op >= PID) return fail(FCGNO_E_INVALID, "op must be FP64, FP32 or BF16");
  if (!arch_ok_for(m, N)) return fail(FCGNO_E_INVALID, "need 2*modes <= n");
  const Plan p = make_plan(m, N, B, 1, 1, op, KIND_APPLY);
  if (ws_bytes < p.total) return fail(FCGNO_E_NOMEM, "workspace too small");
  if (((uintptr_t)ws & 255u) != 0) return fail(FCGNO_E_INVALID, "workspace must be 256-byte aligned");
  return operator_forward(m, p, (char*)ws, N, B, op, k, r, w, false, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Operator application without a workspace argument: the scratch memory is a
// static device array of the library (one per device, held until the process
// ends).  Host code never passes the array's name to a kernel or a copy: on
// the host it is a stand-in symbol, not a device address.  The device
// address comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is used.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[FCGNO_NOALLOC_SCRATCH_BYTES];

namespace fcgno_host {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (looked up on first use).
fcgno_status scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(FCGNO_E_INVALID, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FCGNO_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FCGNO_OK;
}
}  // namespace fcgno_host

extern "C" fcgno_status fcgno_precond_apply_noalloc(const fcgno_model* m, int32_t N, int32_t B, int32_t op,
                                                    const double* k, const double* r, double* w, void* stream) {
  if (!m || !k || !r || !w) return fail(FCGNO_E_INVALID, "null pointer argument");
  if (check_sizes(N, B) != FCGNO_OK) return FCGNO_E_INVALID;
  if (op < 0 || op >= PID) return fail(FCGNO_E_INVALID, "op must be FP64, FP32 or BF16");
  if (!arch_ok_for(m, N)) return fail(FCGNO_E_INVALID, "need 2*modes <= n");
  const Plan p = make_plan(m, N, B, 1, 1, op, KIND_APPLY);
  if (p.total > FCGNO_NOALLOC_SCRATCH_BYTES)
    return fail(FCGNO_E_NOMEM, "operator application needs " + std::to_string(p.total) +
                                   " scratch bytes, more than the static array's " +
                                   std::to_string((size_t)FCGNO_NOALLOC_SCRATCH_BYTES));
  void* ws = nullptr;
  fcgno_status s = scratch_address(&ws);
  if (s != FCGNO_OK) return s;
  // at most this many per-system records live on the stack (no host allocation)
  constexpr int STACK_SYS = 64;
  if (B > STACK_SYS) return fail(FCGNO_E_INVALID, "batch must be <= 64 without a workspace");
  SysDev table[STACK_SYS];
  return operator_forward(m, p, (char*)ws, N, B, op, k, r, w, false, (hipStream_t)stream, table);
}

// ---------------------------------------------------------------------------
// Training
// ---------------------------------------------------------------------------
extern "C" const char* fcgno_last_error(void) { return g_err.c_str(); }

extern "C" const char* fcgno_status_string(fcgno_status s) {
  switch (s) {
    case FCGNO_OK: return "ok";
    case FCGNO_NOT_CONVERGED: return "not converged";
    case FCGNO_E_INVALID: return "invalid argument";
    case FCGNO_E_NOMEM: return "insufficient workspace or device memory";
    case FCGNO_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

// ---------------------------------------------------------------------------
// Serving engine: continuous batching of FCG-NO solves.
//
// Requests (one system each, any N) wait in a queue until a slot and a block
// of the engine's device pool are free; their state then lives on the device
// until they stop.  Active requests of one N form a group; every step
// advances every group by K iterations with the same kernels as
// fcgno_solve (systems at different iterations share launches: all state is
// per system), then reports and releases the requests that stopped.  A
// system's arithmetic depends only on its own data and N, so its result is
// the same bits alone and in any mix.
// ---------------------------------------------------------------------------