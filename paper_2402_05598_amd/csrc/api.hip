// C ABI of libfcgno: model lifecycle, workspace planning, the FCG solve
// driver (Algorithm 1) and the standalone operator application.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "fcgno.h"
#include "prof.h"

using namespace fcgno;

namespace {

thread_local std::string g_err;

fcgno_status fail(fcgno_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) return fail(FCGNO_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline int round16(int v) { return (v + 15) & ~15; }
inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

uint16_t host_f2bf(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  if ((b & 0x7f800000u) == 0x7f800000u) return (uint16_t)((b >> 16) | ((b & 0xffffu) ? 0x40u : 0u));
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

int op_esize(int prec) { return prec == P64 ? 8 : (prec == P32 ? 4 : 2); }
int acc_esize(int prec) { return prec == P64 ? 8 : 4; }
int kstep(int prec) { return prec == PBF ? 16 : 4; }

// Append value v in element type of size esz (8: f64, 4: f32, 2: bf16).
void put(std::vector<char>& buf, size_t off, int esz, double v) {
  if (esz == 8) std::memcpy(buf.data() + off, &v, 8);
  else if (esz == 4) { float f = (float)v; std::memcpy(buf.data() + off, &f, 4); }
  else { uint16_t h = host_f2bf((float)v); std::memcpy(buf.data() + off, &h, 2); }
}

struct Carver {
  size_t n = 0;
  size_t take(size_t bytes) {
    size_t o = n;
    n += align256(bytes);
    return o;
  }
};

}  // namespace

struct fcgno_model {
  fcgno_arch arch{};
  std::vector<double> w;       // float64 master copy (host)
  char* dev = nullptr;         // one device allocation for every derived array
  size_t dev_bytes = 0;
  int device = 0;
  // per precision (P64, P32, PBF)
  std::vector<const void*> Wfrag[3], bias[3], Rmix[3];
  const void* WP[3] = {nullptr, nullptr, nullptr};
  const void* WL0[3] = {nullptr, nullptr, nullptr};
  const double* WL = nullptr;  // float64 [C][4]
  const double* bL = nullptr;  // float64 [C]
  double bP = 0.0;
};

extern "C" size_t fcgno_weight_count(const fcgno_arch* a) {
  if (!a || a->layers < 1 || a->width < 1 || a->modes < 1) return 0;
  const size_t C = a->width, M = a->modes, Cin = a->in_channels;
  return C * Cin + C + (size_t)a->layers * (2 * C * C * 2 * M * M + C * C + C) + C + 1;
}

static fcgno_status upload_weights(fcgno_model* m) {
  const int C = m->arch.width, M = m->arch.modes, L = m->arch.layers, Cin = 4;
  const double* w = m->w.data();
  // unpack the blob
  size_t o = 0;
  const double* WL = w + o; o += (size_t)C * Cin;
  const double* bL = w + o; o += C;
  std::vector<const double*> Rre(L), Rim(L), W(L), b(L);
  const size_t nR = (size_t)C * C * 2 * M * M;
  for (int l = 0; l < L; ++l) {
    Rre[l] = w + o; o += nR;
    Rim[l] = w + o; o += nR;
    W[l] = w + o; o += (size_t)C * C;
    b[l] = w + o; o += C;
  }
  const double* WP = w + o; o += C;
  const double bP = w[o];
  m->bP = bP;
  // composed layer-0 bypass on the features: (W_0 W_L), W_0 b_L + b_0
  std::vector<double> W0L((size_t)C * 4), b0c(C);
  for (int oc = 0; oc < C; ++oc) {
    for (int f = 0; f < 4; ++f) {
      double s = 0.0;
      for (int c = 0; c < C; ++c) s += W[0][oc * C + c] * WL[c * Cin + f];
      W0L[oc * 4 + f] = s;
    }
    double s = b[0][oc];
    for (int c = 0; c < C; ++c) s += W[0][oc * C + c] * bL[c];
    b0c[oc] = s;
  }
  // plan the device buffer
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
  const size_t offWL = cv.take((size_t)C * 4 * 8), offbL = cv.take((size_t)C * 8);
  std::vector<char> hb(cv.n, 0);
  for (int p = 0; p < 3; ++p) {
    const int esz = op_esize(p), asz = acc_esize(p), ks = kstep(p);
    for (int l = 0; l < L; ++l) {
      const int KWP = l == 0 ? ks : C;
      for (int oc = 0; oc < C; ++oc) {
        for (int kw = 0; kw < KWP; ++kw) {
          double v = 0.0;
          if (l == 0) {
            v = kw < 4 ? W0L[oc * 4 + kw] : 0.0;
          } else {
            // input K index kw = ks*KSTEP + g*KPL + e carries channel g*(C/4) + ks*KPL + e
            const int kpl = ks / 4, kss = kw / ks, rem = kw % ks, g = rem / kpl, e = rem % kpl;
            v = W[l][oc * C + g * (C / 4) + kss * kpl + e];
          }
          put(hb, off[p].Wf[l] + ((size_t)oc * KWP + kw) * esz, esz, v);
        }
        put(hb, off[p].bias[l] + (size_t)oc * asz, asz, l == 0 ? b0c[oc] : b[l][oc]);
      }
      // Rmix[ky][a][c][o] (re, im) from R[c][o][a][ky]
      for (int ky = 0; ky < M; ++ky)
        for (int a = 0; a < 2 * M; ++a)
          for (int c = 0; c < C; ++c)
            for (int oc = 0; oc < C; ++oc) {
              const size_t src = (((size_t)c * C + oc) * 2 * M + a) * M + ky;
              const size_t dst = ((((size_t)ky * 2 * M + a) * C + c) * C + oc) * 2;
              put(hb, off[p].R[l] + dst * asz, asz, Rre[l][src]);
              put(hb, off[p].R[l] + (dst + 1) * asz, asz, Rim[l][src]);
            }
    }
    for (int oc = 0; oc < C; ++oc) {
      put(hb, off[p].WP + (size_t)oc * asz, asz, WP[oc]);
      put(hb, off[p].WL0 + (size_t)oc * asz, asz, WL[oc * Cin + 0]);
    }
  }
  std::memcpy(hb.data() + offWL, WL, (size_t)C * 4 * 8);
  std::memcpy(hb.data() + offbL, bL, (size_t)C * 8);
  if (m->dev && m->dev_bytes != cv.n) {
    HIPCHK(hipFree(m->dev));
    m->dev = nullptr;
  }
  if (!m->dev) {
    HIPCHK(hipMalloc((void**)&m->dev, cv.n));
    m->dev_bytes = cv.n;
  }
  HIPCHK(hipMemcpy(m->dev, hb.data(), cv.n, hipMemcpyHostToDevice));
  for (int p = 0; p < 3; ++p) {
    m->Wfrag[p].resize(L); m->bias[p].resize(L); m->Rmix[p].resize(L);
    for (int l = 0; l < L; ++l) {
      m->Wfrag[p][l] = m->dev + off[p].Wf[l];
      m->bias[p][l] = m->dev + off[p].bias[l];
      m->Rmix[p][l] = m->dev + off[p].R[l];
    }
    m->WP[p] = m->dev + off[p].WP;
    m->WL0[p] = m->dev + off[p].WL0;
  }
  m->WL = (const double*)(m->dev + offWL);
  m->bL = (const double*)(m->dev + offbL);
  return FCGNO_OK;
}

extern "C" fcgno_status fcgno_model_create(const fcgno_arch* arch, const double* weights_host,
                                           size_t n_weights, fcgno_model** out) {
  if (!arch || !weights_host || !out) return fail(FCGNO_E_INVALID, "null argument");
  if (arch->in_channels != 4) return fail(FCGNO_E_INVALID, "in_channels must be 4");
  if (arch->width != 16 && arch->width != 32) return fail(FCGNO_E_INVALID, "width must be 16 or 32");
  if (arch->modes < 1 || arch->modes > 16) return fail(FCGNO_E_INVALID, "modes must be in 1..16");
  if (arch->layers < 1 || arch->layers > 64) return fail(FCGNO_E_INVALID, "layers must be in 1..64");
  if (n_weights != fcgno_weight_count(arch)) return fail(FCGNO_E_INVALID, "weight count mismatch");
  for (size_t i = 0; i < n_weights; ++i)
    if (!std::isfinite(weights_host[i])) return fail(FCGNO_E_INVALID, "non-finite weight");
  fcgno_model* m = new fcgno_model();
  m->arch = *arch;
  m->w.assign(weights_host, weights_host + n_weights);
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return fail(FCGNO_E_HIP, "hipGetDevice failed");
  }
  fcgno_status s = upload_weights(m);
  if (s != FCGNO_OK) {
    if (m->dev) (void)hipFree(m->dev);
    delete m;
    return s;
  }
  *out = m;
  return FCGNO_OK;
}

extern "C" fcgno_status fcgno_model_get_weights(const fcgno_model* m, double* wh, size_t n) {
  if (!m || !wh) return fail(FCGNO_E_INVALID, "null argument");
  if (n != m->w.size()) return fail(FCGNO_E_INVALID, "weight count mismatch");
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
  delete m;
}

// ---------------------------------------------------------------------------
// Workspace plan
// ---------------------------------------------------------------------------
namespace {

struct Plan {
  size_t total = 0;
  size_t sysdev, state, counter, hist, part;
  size_t r, w, P, S;
  size_t act, logk, Gr, Gp, Hc, Vc, Wh, Vp;
  size_t vp_bytes_per_sys;
  size_t E64, Eacc, T, TT;
  size_t n_part_blocks;
  size_t gp_bytes_per_sys;
  int S_seg, MP;
};

size_t part_blocks(int N) {
  const size_t flat = ((size_t)N * N + FLAT_PTS - 1) / FLAT_PTS;
  const size_t tile = (size_t)((N + TILE_I - 1) / TILE_I) * ((N + TILE_J - 1) / TILE_J);
  return std::max(flat, tile);
}

// kind 0: solve, 1: operator application
Plan make_plan(const fcgno_model* m, int N, int B, int m_max, int max_iter, int op, int kind) {
  Plan p{};
  Carver cv;
  const size_t n = (size_t)N * N;
  p.n_part_blocks = part_blocks(N);
  p.sysdev = cv.take((size_t)B * sizeof(SysDev));
  p.state = cv.take((size_t)B * sizeof(SysState));
  p.counter = cv.take(sizeof(int));
  p.part = cv.take((size_t)B * p.n_part_blocks * NQ * sizeof(double));
  if (kind == 0) {
    p.hist = cv.take((size_t)B * (max_iter + 1) * sizeof(double));
    p.r = cv.take((size_t)B * n * 8);
    p.P = cv.take((size_t)B * (m_max + 1) * n * 8);
    p.S = cv.take((size_t)B * (m_max + 1) * n * 8);
    p.w = op != PID ? cv.take((size_t)B * n * 8) : 0;
  }
  if (op != PID && m) {
    const int C = m->arch.width, M = m->arch.modes;
    const int MP = round16(2 * M), NP = round16(N);
    const int nyt = NP / 16;
    const int S = (nyt + TPW - 1) / TPW;
    const int esz = op_esize(op), asz = acc_esize(op);
    p.S_seg = S;
    p.MP = MP;
    p.act = cv.take((size_t)B * n * C * esz);
    p.logk = cv.take((size_t)B * n * esz);
    p.Gr = cv.take((size_t)B * N * MP * 8);
    p.gp_bytes_per_sys = std::max((size_t)N * S * MP * C * asz, (size_t)4 * N * MP * 8);
    p.Gp = cv.take((size_t)B * p.gp_bytes_per_sys);
    p.Hc = cv.take((size_t)B * N * C * MP * esz);
    p.Vc = cv.take((size_t)B * C * 2 * M * M * 2 * asz);
    p.Wh = cv.take((size_t)B * C * MP * M * 2 * asz);
    const int XS = (N + 63) / 64;
    p.vp_bytes_per_sys = (size_t)M * XS * C * 2 * M * 2 * asz;
    p.Vp = cv.take((size_t)B * p.vp_bytes_per_sys);
    p.E64 = cv.take((size_t)N * 2 * 8);
    p.Eacc = cv.take((size_t)N * 2 * asz);
    p.T = cv.take((size_t)NP * MP * esz);
    p.TT = cv.take((size_t)MP * NP * esz);
  }
  p.total = cv.n;
  return p;
}

bool arch_ok_for(const fcgno_model* m, int N) { return m && 2 * m->arch.modes <= N; }

// Fill the per-system operator pointers and the NOLaunch of a plan.
void fill_no(const fcgno_model* m, const Plan& p, char* base, int N, int B, int op,
             std::vector<SysDev>& h) {
  const int C = m->arch.width, M = m->arch.modes, MP = p.MP;
  const size_t n = (size_t)N * N;
  const int esz = op_esize(op), asz = acc_esize(op);
  for (int b = 0; b < B; ++b) {
    h[b].act = base + p.act + (size_t)b * n * C * esz;
    h[b].act_stride = n * C;
    h[b].logk = base + p.logk + (size_t)b * n * esz;
    h[b].Gr = (double*)(base + p.Gr) + (size_t)b * N * MP;
    h[b].Gp = base + p.Gp + (size_t)b * p.gp_bytes_per_sys;
    h[b].Hc = base + p.Hc + (size_t)b * N * C * MP * esz;
    h[b].Vc = base + p.Vc + (size_t)b * C * 2 * M * M * 2 * asz;
    h[b].Wh = base + p.Wh + (size_t)b * C * MP * M * 2 * asz;
    h[b].Vp = base + p.Vp + (size_t)b * p.vp_bytes_per_sys;
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
  L.tab.E64 = (const double*)(base + p.E64);
  L.tab.Eacc = base + p.Eacc;
  L.tab.T = base + p.T;
  L.tab.TT = base + p.TT;
  L.Wfrag = m->Wfrag[op].data();
  L.bias = m->bias[op].data();
  L.Rmix = m->Rmix[op].data();
  L.WP = m->WP[op];
  L.bP = m->bP;
  L.WL0 = m->WL0[op];
  L.WL = m->WL;
  L.bL = m->bL;
  L.stream = s;
  return L;
}

fcgno_status check_desc(const fcgno_model* m, const fcgno_solve_desc* d) {
  if (!d) return fail(FCGNO_E_INVALID, "null descriptor");
  if (d->n < 1 || d->batch < 1) return fail(FCGNO_E_INVALID, "n and batch must be >= 1");
  if (d->m_max < 1 || d->m_max > MAXW) return fail(FCGNO_E_INVALID, "m_max must be in 1..32");
  if (d->max_iter < 1) return fail(FCGNO_E_INVALID, "max_iter must be >= 1");
  if (!(d->rtol > 0.0) || !std::isfinite(d->rtol)) return fail(FCGNO_E_INVALID, "rtol must be > 0");
  if (d->op < 0 || d->op > PID) return fail(FCGNO_E_INVALID, "unknown op precision");
  if (d->op != PID) {
    if (!m) return fail(FCGNO_E_INVALID, "operator precision needs a model");
    if (!arch_ok_for(m, d->n)) return fail(FCGNO_E_INVALID, "need 2*modes <= n");
  }
  if ((double)d->n * d->n * d->batch > 4.0e9) return fail(FCGNO_E_INVALID, "problem too large");
  return FCGNO_OK;
}

}  // namespace

extern "C" size_t fcgno_solve_workspace_bytes(const fcgno_model* m, const fcgno_solve_desc* d) {
  if (check_desc(m, d) != FCGNO_OK) return 0;
  return make_plan(m, d->n, d->batch, d->m_max, d->max_iter, d->op, 0).total;
}

extern "C" fcgno_status fcgno_solve(const fcgno_model* m, const fcgno_solve_desc* d, const double* k,
                                    const double* f, double* u, double* r_out, int32_t* iters,
                                    int32_t* sys_status, double* rel_hist, double* true_rel_res, void* ws,
                                    size_t ws_bytes, void* stream) {
  fcgno_status cs = check_desc(m, d);
  if (cs != FCGNO_OK) return cs;
  if (!k || !f || !u || !iters || !sys_status || !ws) return fail(FCGNO_E_INVALID, "null pointer argument");
  const int N = d->n, B = d->batch, op = d->op;
  const Plan p = make_plan(m, N, B, d->m_max, d->max_iter, op, 0);
  if (ws_bytes < p.total) return fail(FCGNO_E_NOMEM, "workspace too small");
  if (((uintptr_t)ws & 255u) != 0) return fail(FCGNO_E_INVALID, "workspace must be 256-byte aligned");
  char* base = (char*)ws;
  hipStream_t s = (hipStream_t)stream;
  const size_t n = (size_t)N * N;
  std::vector<SysDev> h(B);
  SysState* st = (SysState*)(base + p.state);
  int* counter = (int*)(base + p.counter);
  for (int b = 0; b < B; ++b) {
    SysDev& sd = h[b];
    std::memset(&sd, 0, sizeof(SysDev));
    sd.k = k + (size_t)b * (N + 2) * (N + 2);
    sd.f = f + (size_t)b * n;
    sd.u = u + (size_t)b * n;
    sd.r = r_out ? r_out + (size_t)b * n : (double*)(base + p.r) + (size_t)b * n;
    sd.w = op == PID ? sd.r : (double*)(base + p.w) + (size_t)b * n;
    sd.P = (double*)(base + p.P) + (size_t)b * (d->m_max + 1) * n;
    sd.S = (double*)(base + p.S) + (size_t)b * (d->m_max + 1) * n;
    sd.st = st + b;
    sd.hist = (double*)(base + p.hist) + (size_t)b * (d->max_iter + 1);
    sd.part = (double*)(base + p.part) + (size_t)b * p.n_part_blocks * NQ;
    sd.n_active = counter;
  }
  if (op != PID) fill_no(m, p, base, N, B, op, h);
  const SysDev* sysdev = (const SysDev*)(base + p.sysdev);
  HIPCHK(hipMemcpyAsync(base + p.sysdev, h.data(), B * sizeof(SysDev), hipMemcpyHostToDevice, s));
  KrylovLaunch KL{sysdev, B, N, d->m_max, s};
  launch_init_state(KL, d->max_iter, d->rtol);
  NOLaunch NL{};
  if (op != PID) {
    NL = make_no(m, p, base, sysdev, N, B, op, s);
    HIPCHK(hipMemsetAsync(base + p.Hc, 0, (size_t)B * N * m->arch.width * p.MP * op_esize(op), s));
    HIPCHK(hipMemsetAsync(base + p.Wh, 0, (size_t)B * m->arch.width * p.MP * m->arch.modes * 2 * acc_esize(op), s));
    launch_tables(NL, (double*)(base + p.E64), base + p.Eacc, base + p.T, base + p.TT);
    launch_no_setup(NL, (double*)(base + p.Gp));
  }
  launch_residual(KL, 0);
  HIPCHK(hipGetLastError());
  const int K = d->check_every > 0 ? d->check_every : (N >= 256 ? 4 : 8);
  int it = 0, nact = B;
  while (it < d->max_iter) {
    const int end = std::min(d->max_iter, it + K);
    for (; it < end; ++it) {
      if (op != PID) launch_no_apply(NL);
      launch_wdots(KL);
      launch_dir(KL);
      launch_update(KL);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&nact, counter, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (nact <= 0) break;
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

extern "C" size_t fcgno_precond_workspace_bytes(const fcgno_model* m, int32_t n, int32_t batch, int32_t op) {
  if (!m || n < 1 || batch < 1 || op < 0 || op >= PID || !arch_ok_for(m, n)) return 0;
  return make_plan(m, n, batch, 1, 1, op, 1).total;
}

extern "C" fcgno_status fcgno_precond_apply(const fcgno_model* m, int32_t N, int32_t B, int32_t op,
                                            const double* k, const double* r, double* w, void* ws,
                                            size_t ws_bytes, void* stream) {
  if (!m || !k || !r || !w || !ws) return fail(FCGNO_E_INVALID, "null pointer argument");
  if (N < 1 || B < 1) return fail(FCGNO_E_INVALID, "n and batch must be >= 1");
  if (op < 0 || op >= PID) return fail(FCGNO_E_INVALID, "op must be FP64, FP32 or BF16");
  if (!arch_ok_for(m, N)) return fail(FCGNO_E_INVALID, "need 2*modes <= n");
  const Plan p = make_plan(m, N, B, 1, 1, op, 1);
  if (ws_bytes < p.total) return fail(FCGNO_E_NOMEM, "workspace too small");
  if (((uintptr_t)ws & 255u) != 0) return fail(FCGNO_E_INVALID, "workspace must be 256-byte aligned");
  char* base = (char*)ws;
  hipStream_t s = (hipStream_t)stream;
  const size_t n = (size_t)N * N;
  std::vector<SysDev> h(B);
  SysState* st = (SysState*)(base + p.state);
  for (int b = 0; b < B; ++b) {
    SysDev& sd = h[b];
    std::memset(&sd, 0, sizeof(SysDev));
    sd.k = k + (size_t)b * (N + 2) * (N + 2);
    sd.r = const_cast<double*>(r) + (size_t)b * n;
    sd.w = w + (size_t)b * n;
    sd.st = st + b;
    sd.part = (double*)(base + p.part) + (size_t)b * p.n_part_blocks * NQ;
    sd.n_active = (int*)(base + p.counter);
  }
  fill_no(m, p, base, N, B, op, h);
  const SysDev* sysdev = (const SysDev*)(base + p.sysdev);
  HIPCHK(hipMemcpyAsync(base + p.sysdev, h.data(), B * sizeof(SysDev), hipMemcpyHostToDevice, s));
  KrylovLaunch KL{sysdev, B, N, 1, s};
  launch_init_state(KL, 1, 1.0);
  NOLaunch NL = make_no(m, p, base, sysdev, N, B, op, s);
  HIPCHK(hipMemsetAsync(base + p.Hc, 0, (size_t)B * N * m->arch.width * p.MP * op_esize(op), s));
  HIPCHK(hipMemsetAsync(base + p.Wh, 0, (size_t)B * m->arch.width * p.MP * m->arch.modes * 2 * acc_esize(op), s));
  launch_tables(NL, (double*)(base + p.E64), base + p.Eacc, base + p.T, base + p.TT);
  launch_no_setup(NL, (double*)(base + p.Gp));
  launch_rnorm(KL);
  launch_no_apply(NL);
  HIPCHK(hipGetLastError());
  return FCGNO_OK;
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
