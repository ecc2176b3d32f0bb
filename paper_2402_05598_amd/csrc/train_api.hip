// C ABI of libfcgno, training: the operator forward with saved activations,
// the hand-written backward, the energy-norm and Euclidean losses, AdamW.
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

fcgno_status check_train(const fcgno_model* m, int N, int B, int op) {
  if (!m) return fail(FCGNO_E_INVALID, "null model");
  if (check_sizes(N, B) != FCGNO_OK) return FCGNO_E_INVALID;
  if (op != P64 && op != P32) return fail(FCGNO_E_INVALID, "training runs in FP64 or FP32");
  if (!arch_ok_for(m, N)) return fail(FCGNO_E_INVALID, "need 2*modes <= n");
  return FCGNO_OK;
}

// Backward of the operator: upstream gradient gw [B][N^2] scaled per system by
// gscale, with the forward state saved in the plan -> grad (float64 blob);
// with grad_r (gscale = 1, forward output saved in the plan's tw region) also
// the gradient with respect to r.
fcgno_status operator_backward(const fcgno_model* m, const Plan& p, char* base, int N, int B, int op,
                               const double* k, const double* r, const double* gw, const double* gscale,
                               double* grad, hipStream_t s, double* grad_r = nullptr) {
  const int C = m->arch.width, M = m->arch.modes, L = m->arch.layers, MP = p.MP;
  const size_t n = (size_t)N * N;
  const BlobLayout bl(C, M, L);
  const SysDev* sysdev = (const SysDev*)(base + p.sysdev);
  NOLaunch NL = make_no(m, p, base, sysdev, N, B, op, s);
  NL.S = p.Sb;
  const int asz = acc_esize(op);
  BwdArgs a{};
  a.N = N; a.M = M; a.MP = MP; a.L = L; a.nbs = p.nbs; a.S = p.Sb; a.B = B;
  a.st = (const SysState*)(base + p.state);
  a.gscale = gscale;
  a.dphi0 = grad_r ? (double*)(base + p.dvec) : nullptr;
  a.gw = gw;
  a.r = r;
  a.k = k;
  a.logk = base + p.logk;
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
  if (grad_r)
    launch_grad_r(N, B, (const SysState*)(base + p.state), r, gw, (const double*)(base + p.tw),
                  (const double*)(base + p.dvec), grad_r, s);
  HIPCHK(hipGetLastError());
  return FCGNO_OK;
}

}  // namespace fcgno_host

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
  fcgno_status fs = operator_forward(m, p, (char*)ws, N, B, op, k, r, w, true, (hipStream_t)stream);
  if (fs != FCGNO_OK) return fs;
  // keep w for the input gradient of fcgno_op_backward
  HIPCHK(hipMemcpyAsync((char*)ws + p.tw, w, (size_t)B * N * N * sizeof(double), hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  return FCGNO_OK;
}

extern "C" fcgno_status fcgno_op_backward(const fcgno_model* m, int32_t N, int32_t B, int32_t op,
                                          const double* k, const double* r, const double* grad_w,
                                          double* grad_params, double* grad_r, void* ws, size_t ws_bytes,
                                          void* stream) {
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
  return operator_backward(m, p, base, N, B, op, k, r, grad_w, (const double*)(base + p.gscale), grad_params, s,
                           grad_r);
}

namespace fcgno_host {
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
}  // namespace fcgno_host

extern "C" size_t fcgno_energy_loss_workspace_bytes(int32_t N, int32_t B) {
  if (!sizes_ok(N, B)) return 0;
  return loss_plan(N, B).total;
}

extern "C" fcgno_status fcgno_loss(int32_t kind, int32_t N, int32_t B, const double* k, const double* w,
                                   const double* e, double* loss_dev, double* grad_w, void* ws, size_t ws_bytes,
                                   void* stream) {
  if (kind != FCGNO_LOSS_ENERGY && kind != FCGNO_LOSS_L2) return fail(FCGNO_E_INVALID, "unknown loss");
  if (check_sizes(N, B) != FCGNO_OK) return FCGNO_E_INVALID;
  if (!k || !w || !e || !loss_dev || !ws) return fail(FCGNO_E_INVALID, "invalid argument");
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

