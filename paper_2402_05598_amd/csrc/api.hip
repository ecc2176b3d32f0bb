// C ABI of libfcgno: model lifecycle, workspace planning, the FCG solve
// driver (Algorithm 1), the standalone operator application and the training
// entry points (forward with saved activations, hand-written backward, energy
// loss, AdamW step).
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
#include "prof.h"
#include "train.h"

using namespace fcgno;

namespace {

thread_local std::string g_err;

fcgno_status fail(fcgno_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(x)                                                                                    \
  do {                                                                                               \
    hipError_t e_ = (x);                                                                             \
    if (e_ != hipSuccess) return fail(FCGNO_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline int round16(int v) { return (v + 15) & ~15; }
inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int op_esize(int prec) { return prec == P64 ? 8 : (prec == P32 ? 4 : 2); }
int acc_esize(int prec) { return prec == P64 ? 8 : 4; }
int kstep(int prec) { return prec == PBF ? 16 : 4; }

struct Carver {
  size_t n = 0;
  size_t take(size_t bytes) {
    size_t o = n;
    n += align256(bytes);
    return o;
  }
};

// Offsets of the parameter groups in the float64 blob.
struct BlobLayout {
  size_t WL, bL, WP, bP, nR;
  std::vector<size_t> Rre, Rim, W, b;
  BlobLayout(int C, int M, int L) : Rre(L), Rim(L), W(L), b(L) {
    nR = (size_t)C * C * 2 * M * M;
    size_t o = 0;
    WL = o; o += (size_t)C * 4;
    bL = o; o += C;
    for (int l = 0; l < L; ++l) {
      Rre[l] = o; o += nR;
      Rim[l] = o; o += nR;
      W[l] = o; o += (size_t)C * C;
      b[l] = o; o += C;
    }
    WP = o; o += C;
    bP = o;
  }
};

}  // namespace

struct fcgno_model {
  fcgno_arch arch{};
  std::vector<double> w;       // host copy of the weights (refreshed lazily after training)
  bool host_stale = false;
  double* blob = nullptr;      // device float64 master weights, blob order
  char* dev = nullptr;         // derived device arrays of every precision
  size_t dev_bytes = 0;
  int device = 0;
  std::vector<const void*> Wfrag[3], bias[3], Rmix[3];
  const void* WP[3] = {nullptr, nullptr, nullptr};
  const void* WL0[3] = {nullptr, nullptr, nullptr};
  DeriveArgs derive[3];
};

struct fcgno_optim {
  size_t n = 0;
  double lr = 1e-3, wd = 1e-2, b1 = 0.9, b2 = 0.999, eps = 1e-8;
  long long t = 0;
  double* m = nullptr;
  double* v = nullptr;
};

extern "C" size_t fcgno_weight_count(const fcgno_arch* a) {
  if (!a || a->layers < 1 || a->width < 1 || a->modes < 1) return 0;
  const size_t C = a->width, M = a->modes, Cin = a->in_channels;
  return C * Cin + C + (size_t)a->layers * (2 * C * C * 2 * M * M + C * C + C) + C + 1;
}

// Lay out the derived arrays once; their contents come from the device blob.
static fcgno_status alloc_derived(fcgno_model* m) {
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
static void derive_all(fcgno_model* m, hipStream_t s) {
  for (int p = 0; p < 3; ++p) launch_derive(m->derive[p], p, s);
}

static fcgno_status upload_weights(fcgno_model* m) {
  HIPCHK(hipMemcpy(m->blob, m->w.data(), m->w.size() * sizeof(double), hipMemcpyHostToDevice));
  derive_all(m, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipDeviceSynchronize());
  m->host_stale = false;
  return FCGNO_OK;
}

static const double* dev_WL(const fcgno_model* m) { return m->blob; }
static const double* dev_bL(const fcgno_model* m) { return m->blob + (size_t)m->arch.width * 4; }
static const double* dev_bP(const fcgno_model* m) { return m->blob + m->w.size() - 1; }

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

static fcgno_status sync_host(const fcgno_model* mc) {
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
namespace {

constexpr int KIND_SOLVE = 0, KIND_APPLY = 1, KIND_TRAIN = 2;

constexpr int MAX_SUB = 8;   // sub-batches (streams) of one solve

struct Plan {
  size_t total = 0;
  size_t sysdev = 0, state = 0, counter = 0, hist = 0, part = 0;
  size_t r = 0, w = 0, P = 0, S = 0, tmp = 0;
  size_t act = 0, logk = 0, Gr = 0, Gp = 0, Hc = 0, Vc = 0, Wh = 0, Vp = 0;
  size_t E64 = 0, Eacc = 0, T = 0, TT = 0;
  size_t n_part_blocks = 0, gp_bytes_per_sys = 0, vp_bytes_per_sys = 0, wh_bytes_per_sys = 0;
  int S_seg = 1, MP = 16, act_slots = 1;
  // training
  size_t z = 0, vsave = 0, tw = 0, gw = 0, dvec = 0, dzA = 0, dzB = 0, Gh = 0, gscale = 0, loss = 0, lpart = 0;
  size_t pdW = 0, pdb = 0, pdWP = 0, pdbP = 0, pdWL = 0, pdbL = 0, grad = 0, rstage = 0;
  int Sb = 1, nbs = 1, nblk = 1, loss_nb = 1;
};

size_t part_blocks(int N) {
  const size_t flat = ((size_t)N * N + FLAT_PTS - 1) / FLAT_PTS;
  const size_t tile = (size_t)((N + TILE_I - 1) / TILE_I) * ((N + TILE_J - 1) / TILE_J);
  return std::max(flat, tile);
}

// backward row-kernel geometry for N points per row
void bwd_geometry(int N, int prec, int& Sb, int& nbs) {
  const int PB = prec == P64 ? PtsPerBlock<double>::value : PtsPerBlock<float>::value;
  if (N <= PB) {
    const int RB = PB / N;
    Sb = 1;
    nbs = (N + RB - 1) / RB;
  } else {
    Sb = (N + PB - 1) / PB;
    nbs = N * Sb;
  }
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
    const int S = (nyt + TPW - 1) / TPW;
    const int esz = op_esize(op), asz = acc_esize(op);
    if (kind == KIND_TRAIN) {
      bwd_geometry(N, op, p.Sb, p.nbs);
      p.nblk = B * p.nbs;
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
void fill_no(const fcgno_model* m, const Plan& p, char* base, int N, int B, int op, std::vector<SysDev>& h) {
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
  L.prec = op;
  L.basis = m->arch.basis;
  L.tab.E64 = (const double*)(base + p.E64);
  L.tab.Eacc = base + p.Eacc;
  L.tab.T = base + p.T;
  L.tab.TT = base + p.TT;
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
  HIPCHK(hipMemsetAsync(base + p.Hc, 0, (size_t)B * N * m->arch.width * p.MP * op_esize(op), s));
  HIPCHK(hipMemsetAsync(base + p.Wh, 0, (size_t)B * p.wh_bytes_per_sys, s));
  launch_tables(NL, (double*)(base + p.E64), base + p.Eacc, base + p.T, base + p.TT);
  launch_no_setup(NL, (double*)(base + p.Gp));
  return FCGNO_OK;
}

fcgno_status check_desc(const fcgno_model* m, const fcgno_solve_desc* d) {
  if (!d) return fail(FCGNO_E_INVALID, "null descriptor");
  if (d->n < 1 || d->batch < 1) return fail(FCGNO_E_INVALID, "n and batch must be >= 1");
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

}  // namespace

extern "C" size_t fcgno_solve_workspace_bytes(const fcgno_model* m, const fcgno_solve_desc* d) {
  if (check_desc(m, d) != FCGNO_OK) return 0;
  return make_plan(m, d->n, d->batch, d->m_max, d->max_iter, d->op, KIND_SOLVE).total;
}

namespace {
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

fcgno_status solve_impl(const fcgno_model* m, const fcgno_solve_desc* d, const double* k, const double* f,
                        double* u, double* r_out, int32_t* iters, int32_t* sys_status, double* rel_hist,
                        double* true_rel_res, void* ws, size_t ws_bytes, void* stream, const Record* rec) {
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
  if (is_no(op)) fill_no(m, p, base, N, B, op, h);
  const SysDev* sysdev = (const SysDev*)(base + p.sysdev);
  HIPCHK(hipMemcpyAsync(base + p.sysdev, h.data(), B * sizeof(SysDev), hipMemcpyHostToDevice, s));
  KrylovLaunch KL{sysdev, B, N, d->m_max, s};
  for (int g = 0; g < G; ++g) {
    KrylovLaunch KLg{sysdev + b0[g], b0[g + 1] - b0[g], N, d->m_max, s};
    launch_init_state(KLg, d->max_iter, d->rtol);
  }
  NOLaunch NL{};
  if (is_no(op)) {
    NL = make_no(m, p, base, sysdev, N, B, op, s);
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
  int it = 0;
  while (it < d->max_iter) {
    const int end = std::min(d->max_iter, it + K);
    if (!split) {
      for (int i = it; i < end; ++i) {
        if (is_no(op)) launch_no_apply(NL1);
        else if (op == PJAC) launch_jacobi(KL, d->precond_steps);
        else if (op == PSGS) launch_rbsgs(KL, d->precond_steps);
        launch_wdots(KL);
        launch_dir(KL);
        launch_update(KL);
        if (rec && i < rec->m) launch_record(KL, i, rec->m, rec->rec_r, rec->rec_e, rec->ustar);
      }
      it = end;
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(hn.data(), counter, G * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      int total = 0;
      for (int g = 0; g < G; ++g) total += std::max(hn[g], 0);
      if (total <= 0) break;
      continue;
    }
    for (int g = 0; g < G; ++g) {
      if (nact[g] <= 0) continue;
      for (int i = it; i < end; ++i) {
        if (is_no(op)) launch_no_apply(NLs[g]);
        else if (op == PJAC) launch_jacobi(KLs[g], d->precond_steps);
        else if (op == PSGS) launch_rbsgs(KLs[g], d->precond_steps);
        launch_wdots(KLs[g]);
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
    if (rel_hist) {
      const int upto = hs[b].status == S_NONFINITE ? 0 : hs[b].iters;
      for (int i = 0; i <= upto; ++i)
        rel_hist[(size_t)b * (d->max_iter + 1) + i] = hh[(size_t)b * (d->max_iter + 1) + i];
    }
  }
  return all_ok ? FCGNO_OK : FCGNO_NOT_CONVERGED;
}
}  // namespace

extern "C" fcgno_status fcgno_solve(const fcgno_model* m, const fcgno_solve_desc* d, const double* k,
                                    const double* f, double* u, double* r_out, int32_t* iters,
                                    int32_t* sys_status, double* rel_hist, double* true_rel_res, void* ws,
                                    size_t ws_bytes, void* stream) {
  return solve_impl(m, d, k, f, u, r_out, iters, sys_status, rel_hist, true_rel_res, ws, ws_bytes, stream,
                    nullptr);
}

extern "C" size_t fcgno_krylov_samples_workspace_bytes(int32_t n, int32_t batch, int32_t max_iter) {
  if (n < 1 || batch < 1 || max_iter < 1) return 0;
  const size_t sol = make_plan(nullptr, n, batch, 1, max_iter, PID, KIND_SOLVE).total;
  return sol + align256((size_t)batch * n * n * 8) * 2;
}

extern "C" fcgno_status fcgno_krylov_samples(int32_t N, int32_t B, int32_t m_iter, int32_t max_iter,
                                             const double* k, const double* f, const double* u0, double* r_out,
                                             double* e_out, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || B < 1 || m_iter < 1 || max_iter < 1 || !k || !f || !u0 || !r_out || !e_out || !ws)
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
  fcgno_status r1 = solve_impl(nullptr, &d1, k, f, ustar, nullptr, it.data(), st.data(), nullptr, nullptr, ws, sol,
                               stream, nullptr);
  if (r1 < 0) return r1;
  // the recorded CG run (FCG with B = I, window 1) from u0
  HIPCHK(hipMemcpyAsync(ucur, u0, (size_t)B * n * 8, hipMemcpyDeviceToDevice, s));
  fcgno_solve_desc d2{N, B, 1, m_iter, 1e-300, PID, m_iter};
  Record rec{m_iter, r_out, e_out, ustar};
  fcgno_status r2 = solve_impl(nullptr, &d2, k, f, ucur, nullptr, it.data(), st.data(), nullptr, nullptr, ws, sol,
                               stream, &rec);
  if (r2 < 0) return r2;
  return r1;
}

extern "C" fcgno_status fcgno_residual_samples(int32_t N, int32_t B, int32_t max_iter, const double* k,
                                               const double* f, const double* u, double* r_out, double* e_out,
                                               void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || B < 1 || max_iter < 1 || !k || !f || !u || !r_out || !e_out || !ws)
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
  fcgno_status r1 = solve_impl(nullptr, &d1, k, f, ustar, nullptr, it.data(), st.data(), nullptr, nullptr, ws,
                               p.total, stream, nullptr);
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
namespace {

fcgno_status operator_forward(const fcgno_model* m, const Plan& p, char* base, int N, int B, int op,
                              const double* k, const double* r, double* w, bool train, hipStream_t s) {
  const size_t n = (size_t)N * N;
  std::vector<SysDev> h(B);
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
  HIPCHK(hipMemcpyAsync(base + p.sysdev, h.data(), B * sizeof(SysDev), hipMemcpyHostToDevice, s));
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

}  // namespace

extern "C" size_t fcgno_precond_workspace_bytes(const fcgno_model* m, int32_t n, int32_t batch, int32_t op) {
  if (!m || n < 1 || batch < 1 || op < 0 || op >= PID || !arch_ok_for(m, n)) return 0;
  return make_plan(m, n, batch, 1, 1, op, KIND_APPLY).total;
}

extern "C" fcgno_status fcgno_precond_apply(const fcgno_model* m, int32_t N, int32_t B, int32_t op,
                                            const double* k, const double* r, double* w, void* ws,
                                            size_t ws_bytes, void* stream) {
  if (!m || !k || !r || !w || !ws) return fail(FCGNO_E_INVALID, "null pointer argument");
  if (N < 1 || B < 1) return fail(FCGNO_E_INVALID, "n and batch must be >= 1");
  if (op < 0 || op >= PID) return fail(FCGNO_E_INVALID, "op must be FP64, FP32 or BF16");
  if (!arch_ok_for(m, N)) return fail(FCGNO_E_INVALID, "need 2*modes <= n");
  const Plan p = make_plan(m, N, B, 1, 1, op, KIND_APPLY);
  if (ws_bytes < p.total) return fail(FCGNO_E_NOMEM, "workspace too small");
  if (((uintptr_t)ws & 255u) != 0) return fail(FCGNO_E_INVALID, "workspace must be 256-byte aligned");
  return operator_forward(m, p, (char*)ws, N, B, op, k, r, w, false, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Training
// ---------------------------------------------------------------------------
namespace {

fcgno_status check_train(const fcgno_model* m, int N, int B, int op) {
  if (!m) return fail(FCGNO_E_INVALID, "null model");
  if (N < 1 || B < 1) return fail(FCGNO_E_INVALID, "n and batch must be >= 1");
  if (op != P64 && op != P32) return fail(FCGNO_E_INVALID, "training runs in FP64 or FP32");
  if (!arch_ok_for(m, N)) return fail(FCGNO_E_INVALID, "need 2*modes <= n");
  return FCGNO_OK;
}

// Backward of the operator: upstream gradient gw [B][N^2] scaled per system by
// gscale, with the forward state saved in the plan -> grad (float64 blob).
fcgno_status operator_backward(const fcgno_model* m, const Plan& p, char* base, int N, int B, int op,
                               const double* k, const double* r, const double* gw, const double* gscale,
                               double* grad, hipStream_t s) {
  const int C = m->arch.width, M = m->arch.modes, L = m->arch.layers, MP = p.MP;
  const size_t n = (size_t)N * N;
  const BlobLayout bl(C, M, L);
  const SysDev* sysdev = (const SysDev*)(base + p.sysdev);
  NOLaunch NL = make_no(m, p, base, sysdev, N, B, op, s);
  NL.S = p.Sb;
  const int asz = acc_esize(op);
  BwdArgs a{};
  a.N = N; a.M = M; a.MP = MP; a.L = L; a.nbs = p.nbs; a.S = p.Sb;
  a.st = (const SysState*)(base + p.state);
  a.gscale = gscale;
  a.gw = gw;
  a.r = r;
  a.k = k;
  a.z = base + p.z;
  a.z_sys = n * C;
  a.z_layer = (size_t)B * n * C;
  a.act = base + p.act;
  a.act_sys = n * C;
  a.act_slot = (size_t)B * n * C;
  a.Hcb = base + p.Hc;
  a.hc_sys = (size_t)N * C * MP;
  a.T = base + p.T;
  a.blob = m->blob;
  a.off_WP = bl.WP;
  a.off_WL = bl.WL;
  a.off_bL = bl.bL;
  a.Gb = base + p.Gp;
  a.gb_sys = p.gp_bytes_per_sys / asz;
  a.pdW = base + p.pdW; a.pdb = base + p.pdb; a.pdWP = base + p.pdWP; a.pdbP = base + p.pdbP;
  a.pdWL = base + p.pdWL; a.pdbL = base + p.pdbL;
  void* dz[2] = {base + p.dzA, base + p.dzB};
  double* rst = (double*)(base + p.rstage);
  int cur = 0;
  // start: projection, then the target layer L-1
  a.mode = 0;
  a.l = 0;
  a.dz_in = nullptr;
  a.dz_out = dz[cur];
  launch_bwd(a, op, C, p.nblk, s);
  launch_reduce(base + p.pdWP, op, p.nblk, C, grad + bl.WP, rst, s);
  launch_reduce(base + p.pdbP, op, p.nblk, 1, grad + bl.bP, rst, s);
  launch_reduce(base + p.pdW, op, p.nblk, C * C, grad + bl.W[L - 1], rst, s);
  launch_reduce(base + p.pdb, op, p.nblk, C, grad + bl.b[L - 1], rst, s);
  const int XS = (N + 63) / 64;
  for (int l = L - 1; l >= 0; --l) {
    // spectral adjoint of layer l from the row partials of dz_l
    SpecArgs sa{sysdev, N, p.Sb, M, 0, XS, B, NL.tab.Eacc, NL.tab.E64, m->Rmix[op][l], m->WL0[op], nullptr, 0, 1,
                NL.basis};
    launch_spec_fwd(NL, sa);
    BSpecArgs ba{};
    ba.N = N; ba.M = M; ba.B = B; ba.XS = XS; ba.basis = NL.basis;
    ba.Vp = base + p.Vp;
    ba.vp_sys = p.vp_bytes_per_sys / asz;
    ba.R = m->Rmix[op][l];
    ba.Gh = base + p.Gh;
    ba.gh_sys = (size_t)M * C * 2 * M * 2;
    ba.Wh = base + p.Wh;
    ba.wh_sys = p.wh_bytes_per_sys / asz;
    ba.Vsave = base + p.vsave + (size_t)l * B * ba.gh_sys * asz;
    ba.vs_sys = ba.gh_sys;
    launch_bspec_mix(ba, op, C, s);
    launch_dR(ba, op, C, grad + bl.Rre[l], grad + bl.Rim[l], s);
    launch_spec_inv(NL, sa);
    // dv_l, then the next target layer (or the lift)
    a.mode = 1;
    a.l = l;
    a.off_W = bl.W[l];
    a.dz_in = dz[cur];
    a.dz_out = dz[1 - cur];
    launch_bwd(a, op, C, p.nblk, s);
    if (l >= 1) {
      launch_reduce(base + p.pdW, op, p.nblk, C * C, grad + bl.W[l - 1], rst, s);
      launch_reduce(base + p.pdb, op, p.nblk, C, grad + bl.b[l - 1], rst, s);
    } else {
      launch_reduce(base + p.pdWL, op, p.nblk, C * 4, grad + bl.WL, rst, s);
      launch_reduce(base + p.pdbL, op, p.nblk, C, grad + bl.bL, rst, s);
    }
    cur = 1 - cur;
  }
  HIPCHK(hipGetLastError());
  return FCGNO_OK;
}

}  // namespace

extern "C" fcgno_status fcgno_optim_create(const fcgno_model* m, double lr, double weight_decay, double beta1,
                                           double beta2, double eps, fcgno_optim** out) {
  if (!m || !out) return fail(FCGNO_E_INVALID, "null argument");
  if (!(lr > 0.0) || !(weight_decay >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0))
    return fail(FCGNO_E_INVALID, "invalid optimiser hyper-parameters");
  fcgno_optim* o = new fcgno_optim();
  o->n = m->w.size();
  o->lr = lr; o->wd = weight_decay; o->b1 = beta1; o->b2 = beta2; o->eps = eps;
  if (hipMalloc((void**)&o->m, o->n * 8) != hipSuccess || hipMalloc((void**)&o->v, o->n * 8) != hipSuccess ||
      hipMemset(o->m, 0, o->n * 8) != hipSuccess || hipMemset(o->v, 0, o->n * 8) != hipSuccess) {
    if (o->m) (void)hipFree(o->m);
    if (o->v) (void)hipFree(o->v);
    delete o;
    return fail(FCGNO_E_HIP, "optimiser state allocation failed");
  }
  *out = o;
  return FCGNO_OK;
}

extern "C" fcgno_status fcgno_optim_set_lr(fcgno_optim* o, double lr) {
  if (!o || !(lr > 0.0)) return fail(FCGNO_E_INVALID, "invalid learning rate");
  o->lr = lr;
  return FCGNO_OK;
}

extern "C" void fcgno_optim_destroy(fcgno_optim* o) {
  if (!o) return;
  if (o->m) (void)hipFree(o->m);
  if (o->v) (void)hipFree(o->v);
  delete o;
}

extern "C" size_t fcgno_train_workspace_bytes(const fcgno_model* m, int32_t n, int32_t batch, int32_t op) {
  if (check_train(m, n, batch, op) != FCGNO_OK) return 0;
  return make_plan(m, n, batch, 1, 1, op, KIND_TRAIN).total;
}

extern "C" fcgno_status fcgno_op_forward(const fcgno_model* m, int32_t N, int32_t B, int32_t op, const double* k,
                                         const double* r, double* w, void* ws, size_t ws_bytes, void* stream) {
  fcgno_status cs = check_train(m, N, B, op);
  if (cs != FCGNO_OK) return cs;
  if (!k || !r || !w || !ws) return fail(FCGNO_E_INVALID, "null pointer argument");
  const Plan p = make_plan(m, N, B, 1, 1, op, KIND_TRAIN);
  if (ws_bytes < p.total) return fail(FCGNO_E_NOMEM, "workspace too small");
  if (((uintptr_t)ws & 255u) != 0) return fail(FCGNO_E_INVALID, "workspace must be 256-byte aligned");
  return operator_forward(m, p, (char*)ws, N, B, op, k, r, w, true, (hipStream_t)stream);
}

extern "C" fcgno_status fcgno_op_backward(const fcgno_model* m, int32_t N, int32_t B, int32_t op,
                                          const double* k, const double* r, const double* grad_w,
                                          double* grad_params, void* ws, size_t ws_bytes, void* stream) {
  fcgno_status cs = check_train(m, N, B, op);
  if (cs != FCGNO_OK) return cs;
  if (!k || !r || !grad_w || !grad_params || !ws) return fail(FCGNO_E_INVALID, "null pointer argument");
  const Plan p = make_plan(m, N, B, 1, 1, op, KIND_TRAIN);
  if (ws_bytes < p.total) return fail(FCGNO_E_NOMEM, "workspace too small");
  if (((uintptr_t)ws & 255u) != 0) return fail(FCGNO_E_INVALID, "workspace must be 256-byte aligned");
  char* base = (char*)ws;
  hipStream_t s = (hipStream_t)stream;
  std::vector<double> ones(B, 1.0);
  HIPCHK(hipMemcpyAsync(base + p.gscale, ones.data(), B * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return operator_backward(m, p, base, N, B, op, k, r, grad_w, (const double*)(base + p.gscale), grad_params, s);
}

namespace {
struct LossPlan {
  size_t total, dvec, gw, part, gscale;
  int nb;
};
LossPlan loss_plan(int N, int B) {
  LossPlan lp{};
  const size_t n = (size_t)N * N;
  lp.nb = (int)((n + FLAT_PTS - 1) / FLAT_PTS);
  Carver cv;
  lp.dvec = cv.take(B * n * 8);
  lp.gw = cv.take(B * n * 8);
  lp.part = cv.take((size_t)B * lp.nb * 16);
  lp.gscale = cv.take(B * 8);
  lp.total = cv.n;
  return lp;
}
}  // namespace

extern "C" size_t fcgno_energy_loss_workspace_bytes(int32_t N, int32_t B) {
  if (N < 1 || B < 1) return 0;
  return loss_plan(N, B).total;
}

extern "C" fcgno_status fcgno_loss(int32_t kind, int32_t N, int32_t B, const double* k, const double* w,
                                   const double* e, double* loss_dev, double* grad_w, void* ws, size_t ws_bytes,
                                   void* stream) {
  if (kind != FCGNO_LOSS_ENERGY && kind != FCGNO_LOSS_L2) return fail(FCGNO_E_INVALID, "unknown loss");
  if (N < 1 || B < 1 || !k || !w || !e || !loss_dev || !ws) return fail(FCGNO_E_INVALID, "invalid argument");
  const LossPlan lp = loss_plan(N, B);
  if (ws_bytes < lp.total) return fail(FCGNO_E_NOMEM, "workspace too small");
  if (((uintptr_t)ws & 255u) != 0) return fail(FCGNO_E_INVALID, "workspace must be 256-byte aligned");
  char* base = (char*)ws;
  hipStream_t s = (hipStream_t)stream;
  double* gwbuf = grad_w ? grad_w : (double*)(base + lp.gw);
  LossArgs la{N, B, lp.nb, k, w, e, (double*)(base + lp.dvec), gwbuf, (double*)(base + lp.part), loss_dev,
              (double*)(base + lp.gscale), kind};
  launch_loss(la, s);
  if (grad_w) launch_scale_rows(grad_w, (const double*)(base + lp.gscale), B, (size_t)N * N, s);
  HIPCHK(hipGetLastError());
  return FCGNO_OK;
}

extern "C" fcgno_status fcgno_energy_loss(int32_t N, int32_t B, const double* k, const double* w, const double* e,
                                          double* loss_dev, double* grad_w, void* ws, size_t ws_bytes,
                                          void* stream) {
  return fcgno_loss(FCGNO_LOSS_ENERGY, N, B, k, w, e, loss_dev, grad_w, ws, ws_bytes, stream);
}

extern "C" fcgno_status fcgno_train_step_loss(fcgno_model* m, fcgno_optim* opt, int32_t N, int32_t B, int32_t op,
                                              int32_t loss_kind, const double* k, const double* r, const double* e,
                                              double* loss_host, void* ws, size_t ws_bytes, void* stream) {
  if (loss_kind != FCGNO_LOSS_ENERGY && loss_kind != FCGNO_LOSS_L2) return fail(FCGNO_E_INVALID, "unknown loss");
  fcgno_status cs = check_train(m, N, B, op);
  if (cs != FCGNO_OK) return cs;
  if (!opt || !k || !r || !e || !ws) return fail(FCGNO_E_INVALID, "null pointer argument");
  if (opt->n != m->w.size()) return fail(FCGNO_E_INVALID, "optimiser belongs to another architecture");
  const Plan p = make_plan(m, N, B, 1, 1, op, KIND_TRAIN);
  if (ws_bytes < p.total) return fail(FCGNO_E_NOMEM, "workspace too small");
  if (((uintptr_t)ws & 255u) != 0) return fail(FCGNO_E_INVALID, "workspace must be 256-byte aligned");
  char* base = (char*)ws;
  hipStream_t s = (hipStream_t)stream;
  double* w = (double*)(base + p.tw);
  fcgno_status fs = operator_forward(m, p, base, N, B, op, k, r, w, true, s);
  if (fs != FCGNO_OK) return fs;
  LossArgs la{N, B, p.loss_nb, k, w, e, (double*)(base + p.dvec), (double*)(base + p.gw),
              (double*)(base + p.lpart), (double*)(base + p.loss), (double*)(base + p.gscale), loss_kind};
  launch_loss(la, s);
  double* grad = (double*)(base + p.grad);
  fs = operator_backward(m, p, base, N, B, op, k, r, (const double*)(base + p.gw),
                         (const double*)(base + p.gscale), grad, s);
  if (fs != FCGNO_OK) return fs;
  opt->t += 1;
  launch_adamw(m->blob, grad, opt->m, opt->v, opt->n, opt->lr, opt->wd, opt->b1, opt->b2, opt->eps, opt->t, s);
  derive_all(m, s);
  m->host_stale = true;
  HIPCHK(hipGetLastError());
  if (loss_host) {
    std::vector<double> lb(B);
    HIPCHK(hipMemcpyAsync(lb.data(), base + p.loss, B * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double sum = 0.0;
    for (int b = 0; b < B; ++b) sum += lb[b];
    *loss_host = sum / B;
  }
  return FCGNO_OK;
}

extern "C" fcgno_status fcgno_train_step(fcgno_model* m, fcgno_optim* opt, int32_t N, int32_t B, int32_t op,
                                         const double* k, const double* r, const double* e, double* loss_host,
                                         void* ws, size_t ws_bytes, void* stream) {
  return fcgno_train_step_loss(m, opt, N, B, op, FCGNO_LOSS_ENERGY, k, r, e, loss_host, ws, ws_bytes, stream);
}

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
namespace {

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
  size_t E64 = 0, Eacc = 0, T = 0, TT = 0, table = 0, ftable = 0, flags = 0, tres = 0;
  std::vector<int64_t> members;
  bool dirty = true;
  size_t hoff = 0;           // this step's range in the engine's pinned export buffers
  hipStream_t s = nullptr;   // the engine lane this group's work runs on
};

}  // namespace

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
  double* htres = nullptr;
  // Groups of different N run on separate streams (default priority), so a
  // large group's bandwidth-bound launches and a small group's latency-bound
  // ones overlap on the device; every step first waits for the caller's stream.
  std::vector<hipStream_t> lanes;
  hipEvent_t ready = nullptr;
  int next_lane = 0;
};

namespace {

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
  t.table = cv.take((size_t)slots * sizeof(SysDev));
  t.ftable = cv.take((size_t)slots * sizeof(SysDev));
  t.flags = cv.take((size_t)slots * 3 * sizeof(int));
  t.tres = cv.take((size_t)slots * sizeof(double));
  if (g) {
    g->E64 = t.E64; g->Eacc = t.Eacc; g->T = t.T; g->TT = t.TT;
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
  L.S = ((round16(g.N) / 16) + TPW - 1) / TPW;
  L.prec = op;
  L.basis = m->arch.basis;
  L.tab.E64 = (const double*)(base + g.E64);
  L.tab.Eacc = base + g.Eacc;
  L.tab.T = base + g.T;
  L.tab.TT = base + g.TT;
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

fcgno_status group_open(fcgno_engine* e, int N, EngGroup** out) {
  auto it = e->groups.find(N);
  if (it != e->groups.end()) {
    *out = &it->second;
    return FCGNO_OK;
  }
  EngGroup g;
  g.N = N;
  g.s = e->lanes[e->next_lane];
  g.bytes = group_bytes(e->d.op == PID ? nullptr : e->m, e->d.op, N, e->d.max_slots, &g);
  if (!pool_alloc(e, g.bytes, &g.off)) return FCGNO_E_NOMEM;
  if (e->d.op != PID) {
    const NOLaunch NL = group_no(e, g, nullptr, 0);
    char* base = e->pool + g.off;
    launch_tables(NL, (double*)(base + g.E64), base + g.Eacc, base + g.T, base + g.TT);
  }
  e->next_lane = (e->next_lane + 1) % (int)e->lanes.size();
  auto res = e->groups.emplace(N, g);
  *out = &res.first->second;
  return FCGNO_OK;
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
    fill_no(m, p, base, N, 1, op, h);
    sd = h[0];
  }
  const SysDev* own = (const SysDev*)(base + p.sysdev);
  HIPCHK(hipMemcpyAsync(base + p.sysdev, &sd, sizeof(SysDev), hipMemcpyHostToDevice, g.s));
  KrylovLaunch KL{own, 1, N, e->d.m_max, g.s};
  launch_init_state(KL, q.max_iter, q.rtol);
  if (op != PID) {
    HIPCHK(hipMemsetAsync(base + p.Hc, 0, (size_t)N * m->arch.width * p.MP * op_esize(op), g.s));
    HIPCHK(hipMemsetAsync(base + p.Wh, 0, p.wh_bytes_per_sys, g.s));
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
  return FCGNO_OK;
}

}  // namespace

extern "C" size_t fcgno_engine_request_bytes(const fcgno_model* m, const fcgno_engine_desc* d, int32_t n,
                                             int32_t max_iter) {
  if (!d || n < 1 || max_iter < 1 || d->m_max < 1 || d->m_max > MAXW) return 0;
  if (d->op != PID && (!m || !arch_ok_for(m, n))) return 0;
  return align256(request_bytes(m, d->op, d->m_max, n, max_iter));
}

extern "C" fcgno_status fcgno_engine_create(const fcgno_model* m, const fcgno_engine_desc* d, void* stream,
                                            fcgno_engine** out) {
  if (!d || !out) return fail(FCGNO_E_INVALID, "null argument");
  if (d->op < 0 || d->op > PID) return fail(FCGNO_E_INVALID, "the engine takes FP64, FP32, BF16 or IDENTITY");
  if (d->op != PID && !m) return fail(FCGNO_E_INVALID, "operator precision needs a model");
  if (d->m_max < 1 || d->m_max > MAXW) return fail(FCGNO_E_INVALID, "m_max must be in 1..32");
  if (d->max_slots < 1 || d->budget_bytes < 4096) return fail(FCGNO_E_INVALID, "need max_slots >= 1 and a budget");
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
             hipHostMalloc((void**)&e->htres, (size_t)d->max_slots * sizeof(double), 0) != hipSuccess) {
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
  if (N < 1 || max_iter < 1 || !(rtol > 0.0) || !std::isfinite(rtol)) return fail(FCGNO_E_INVALID, "bad request");
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
  for (auto it = e->queue.begin(); it != e->queue.end();) {
    if ((int)e->active.size() >= e->d.max_slots) break;
    EngGroup* g = nullptr;
    const bool had_group = e->groups.count(it->N) != 0;
    if (group_open(e, it->N, &g) != FCGNO_OK) { ++it; continue; }
    size_t off = 0;
    if (!pool_alloc(e, it->bytes, &off)) {
      if (!had_group && g->members.empty()) group_close(e, it->N);
      ++it;
      continue;
    }
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
    if (e->d.op != PID) NL = group_no(e, g, table, G);
    for (int i = 0; i < K; ++i) {
      if (e->d.op != PID) launch_no_apply(NL);
      launch_wdots(KL);
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
    HIPCHK(hipMemcpyAsync(e->htres + ho, base + g.tres, (size_t)F * sizeof(double), hipMemcpyDeviceToHost, g.s));
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
        r.true_rel_res = e->htres[g.hoff + b];
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
