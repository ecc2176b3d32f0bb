// Host-side internals shared by the C ABI sources (api.hip: models, plans,
// the solve driver, operator application; train_api.hip: training entry
// points; serve.hip: the serving engine).  Not part of the public interface.
#pragma once

#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "common.h"
#include "fcgno.h"
#include "train.h"

namespace fcgno_host {

using namespace fcgno;

inline thread_local std::string g_err;

inline fcgno_status fail(fcgno_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(x)                                                                                    \
  do {                                                                                               \
    hipError_t e_ = (x);                                                                             \
    if (e_ != hipSuccess) return fail(FCGNO_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline int round16(int v) { return (v + 15) & ~15; }

// Size limits shared by every entry point: a system's grid indices are 32-bit
// (N^2 < 2^31), twiddle-index products assume N <= 2^15, and the batch is a
// grid dimension of the launches (at most 65535).
constexpr int MAX_N = 32768;
constexpr int MAX_BATCH = 65535;
inline bool sizes_ok(long long N, long long B) { return N >= 1 && N <= MAX_N && B >= 1 && B <= MAX_BATCH; }
inline fcgno_status check_sizes(long long N, long long B) {
  if (!sizes_ok(N, B)) return fail(FCGNO_E_INVALID, "n must be in 1..32768 and batch in 1..65535");
  return FCGNO_OK;
}
inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

inline int op_esize(int prec) { return prec == P64 ? 8 : (prec == P32 ? 4 : 2); }
inline int acc_esize(int prec) { return prec == P64 ? 8 : 4; }
inline int kstep(int prec) { return prec == PBF ? 16 : 4; }

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


constexpr int KIND_SOLVE = 0, KIND_APPLY = 1, KIND_TRAIN = 2;

constexpr int MAX_SUB = 8;   // sub-batches (streams) of one solve

struct Plan {
  size_t total = 0;
  size_t sysdev = 0, state = 0, counter = 0, hist = 0, part = 0, sysdev2 = 0, idle = 0;
  size_t r = 0, w = 0, P = 0, S = 0, tmp = 0;
  size_t act = 0, logk = 0, Gr = 0, Gp = 0, Hc = 0, Vc = 0, Wh = 0, Vp = 0;
  size_t E64 = 0, Eacc = 0, T = 0, TT = 0, FA = 0, SA = 0, WT = 0, wt_bytes_per_sys = 0, RD = 0, EX = 0;
  size_t n_part_blocks = 0, gp_bytes_per_sys = 0, vp_bytes_per_sys = 0, wh_bytes_per_sys = 0;
  int S_seg = 1, MP = 16, act_slots = 1;
  // training
  size_t z = 0, vsave = 0, tw = 0, gw = 0, dvec = 0, dzA = 0, dzB = 0, Gh = 0, gscale = 0, loss = 0, lpart = 0;
  size_t pdW = 0, pdb = 0, pdWP = 0, pdbP = 0, pdWL = 0, pdbL = 0, grad = 0, rstage = 0;
  int Sb = 1, nbs = 1, nblk = 1, loss_nb = 1;
};


// Workspace plans and operator set-up (api.hip).
size_t part_blocks(int N);
void bwd_geometry(int N, int prec, int& Sb, int& nbs);
Plan make_plan(const fcgno_model* m, int N, int B, int m_max, int max_iter, int op, int kind);
bool arch_ok_for(const fcgno_model* m, int N);
void fill_no(const fcgno_model* m, const Plan& p, char* base, int N, int B, int op, SysDev* h);
NOLaunch make_no(const fcgno_model* m, const Plan& p, char* base, const SysDev* sysdev, int N, int B, int op,
                 hipStream_t s);
fcgno_status operator_setup(const fcgno_model* m, const Plan& p, char* base, const NOLaunch& NL, int N, int B,
                            int op, hipStream_t s);
// table: host storage for the B per-system pointer records (NULL: a vector of
// its own); it must stay valid until the call returns.
fcgno_status operator_forward(const fcgno_model* m, const Plan& p, char* base, int N, int B, int op,
                              const double* k, const double* r, double* w, bool train, hipStream_t s,
                              SysDev* table = nullptr);
// Model weights (api.hip).
fcgno_status alloc_derived(fcgno_model* m);
void derive_all(fcgno_model* m, hipStream_t s);
fcgno_status upload_weights(fcgno_model* m);
fcgno_status sync_host(const fcgno_model* mc);

}  // namespace fcgno_host

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
  fcgno::DeriveArgs derive[3];
};

struct fcgno_optim {
  size_t n = 0;
  double lr = 1e-3, wd = 1e-2, b1 = 0.9, b2 = 0.999, eps = 1e-8;
  long long t = 0;
  double* m = nullptr;
  double* v = nullptr;
};

namespace fcgno_host {
// Device float64 lift weights, lift bias and projection bias inside the blob.
inline const double* dev_WL(const fcgno_model* m) { return m->blob; }
inline const double* dev_bL(const fcgno_model* m) { return m->blob + (size_t)m->arch.width * 4; }
inline const double* dev_bP(const fcgno_model* m) { return m->blob + m->w.size() - 1; }
}  // namespace fcgno_host
