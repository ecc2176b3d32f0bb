// Internal declarations of the training kernels.
#pragma once
#include "common.h"

namespace fcgno {

__host__ __device__ inline int round16_t(int v) { return (v + 15) & ~15; }


struct LossArgs {
  int N, B, nb;            // nb: flat blocks per system
  const double* k;         // [B][N+2][N+2]
  const double* w;         // [B][N][N]
  const double* e;         // [B][N][N]
  double* dvec;            // [B][N][N] scratch: w - e
  double* gw;              // [B][N][N] out: A (w - e)
  double* part;            // [B][nb][2]
  double* loss;            // [B] out: ||w-e||_A / ||e||_A
  double* gscale;          // [B] out: 1 / (B ||w-e|| ||e||)
  int kind;                // 0: energy norm (Notay), 1: Euclidean (L2)
};

struct BwdArgs {
  int N, M, MP, L, mode, l, nbs, S;   // S: row segments of TPW tiles; nbs = N S row segments per system
  int B;                              // systems
  const SysState* st;                 // per system: snorm
  const double* gscale;               // [B]
  const double* gw;                   // [B][N^2] upstream gradient of w (before gscale)
  const double* r;                    // [B][N^2]
  const double* k;                    // [B][N+2]^2
  const void* logk;                   // [B][N^2] log k in the op precision (forward set-up)
  const void* z;                      // saved pre-activations [L][B][N^2][C]
  size_t z_sys, z_layer;
  const void* act;                    // saved activations, slot s = v_{s+1}
  size_t act_sys, act_slot;
  const void* dz_in;                  // [B][N^2][C] accumulate precision: dz of layer l
  void* dz_out;                       // [B][N^2][C] accumulate precision: dz of the target layer
  const void* Hcb;                    // [B][N][C][MP] adjoint synthesis rows
  size_t hc_sys;
  const void* T;                      // [NP][MP]
  const double* blob;                 // float64 weights
  size_t off_W, off_WP, off_WL, off_bL;
  void* Gb;                           // [B][N][S][MP][C] row partials of dz (accumulate precision)
  size_t gb_sys;
  // partial gradients, one set per block of four row segments (accumulate precision)
  void* pdW; void* pdb; void* pdWP; void* pdbP; void* pdWL; void* pdbL;
  double* dphi0;                      // nullable [B][N^2]: gradient w.r.t. the feature r/s (float64)
};

struct BSpecArgs {
  int N, M, B, XS;
  const void* Vp;      // [B] per-system chunk spectra (forward kernel output)
  size_t vp_sys;
  const void* R;       // [M][2M][C][C] complex, this layer
  void* Gh;            // [M][2M][B][C] complex: G^ of every system, mode-major
  size_t gh_sys;
  void* Wh;            // [B][M][C][MP] complex: G^_V for the synthesis
  size_t wh_sys;
  const void* Vsave;   // [M][2M][B][C] complex: V^ of this layer, mode-major
  size_t vs_sys;
  int basis;           // B_FOURIER or B_SINE
};

struct DeriveArgs {
  const double* blob;
  int C, M, L, kpl;
  void* Wfrag[64];
  void* bias[64];
  void* Rmix[64];
  void* WP;
  void* WL0;
};

void launch_loss(const LossArgs& a, hipStream_t s);
void launch_bwd(const BwdArgs& a, int prec, int C, int nblk, hipStream_t s);
void launch_bspec_mix(const BSpecArgs& a, int prec, int C, hipStream_t s);
void launch_dR(const BSpecArgs& a, int prec, int C, double* gre, double* gim, hipStream_t s);
// Gradient with respect to the input residual of L = sum_b <g_b, B(r_b)>,
// from the feature gradient dphi0 (see k_grad_r).
void launch_grad_r(int N, int B, const SysState* st, const double* r, const double* g, const double* w,
                   const double* dphi0, double* grad_r, hipStream_t s);
// stage: REDUCE_CHUNKS * count doubles of scratch
constexpr int REDUCE_CHUNKS = 64;
void launch_reduce(const void* part, int prec, int nblk, int count, double* out, double* stage, hipStream_t s);
void launch_adamw(double* theta, const double* g, double* m, double* v, size_t n, double lr, double wd, double b1,
                  double b2, double eps, long long t, hipStream_t s);
void launch_derive(const DeriveArgs& a, int prec, hipStream_t s);
// g[b][p] *= scale[b]
void launch_scale_rows(double* g, const double* scale, int B, size_t n, hipStream_t s);

}  // namespace fcgno
