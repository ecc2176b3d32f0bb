// Training of the operator on the energy-norm loss (the error form of the
// Notay loss, Sec. 3.1): loss, hand-written backward of every layer, AdamW and
// the device-side re-layout of the updated weights.
//
// Adjoint of one Fourier layer z = S(W^) + W v + b, v' = GELU(z), with
// V^ = F(v) the truncated forward DFT, W^ = V^ R per mode and S the synthesis
// N^-2 Re sum g_ky W^ e^{+i phi}:
//   dz   = dv' * GELU'(z)
//   db   = sum dz,  dW = sum dz (x) v
//   G^   = N^-2 g_ky F(dz)                 (the same truncated forward DFT)
//   dR   = sum_batch G^ conj(V^)           (packed d/dRe + i d/dIm)
//   G^_V = sum_o G^[o] conj(R[c][o])
//   dv   = W^T dz + Re sum G^_V e^{+i phi}  (synthesis with unit scale)
// The y-direction halves of F and of the synthesis run in the row kernel
// below; the x-direction halves reuse the forward spectral kernels.
#include <algorithm>

#include "common.h"
#include "prof.h"
#include "train.h"

namespace fcgno {

template <typename T> struct Acc;
template <> struct Acc<float> {
  static __device__ __forceinline__ float erfv(float x) { return erf_as(x); }
  static __device__ __forceinline__ float expv(float x) { return __expf(x); }
};
template <> struct Acc<double> {
  static __device__ __forceinline__ double erfv(double x) { return erf(x); }
  static __device__ __forceinline__ double expv(double x) { return exp(x); }
};

// GELU and its derivative Phi(z) + z phi(z)
template <typename T>
__device__ __forceinline__ T gelu_t(T z) {
  return (T)0.5 * z * ((T)1 + Acc<T>::erfv(z * (T)0.70710678118654752440));
}
template <typename T>
__device__ __forceinline__ T dgelu_t(T z) {
  const T cdf = (T)0.5 * ((T)1 + Acc<T>::erfv(z * (T)0.70710678118654752440));
  const T pdf = (T)0.39894228040143267794 * Acc<T>::expv((T)-0.5 * z * z);
  return cdf + z * pdf;
}

// ---------------------------------------------------------------------------
// Loss: d = w - e, partial (d, A d), (e, A e); A d kept for the gradient.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double apply_A(const double* __restrict__ k, const double* __restrict__ u, int N, int i,
                                          int j) {
  const int K = N + 2;
  const int p = i * N + j;
  const double c = u[p];
  const double e = (i + 1 < N) ? u[p + N] : 0.0;
  const double w = (i > 0) ? u[p - N] : 0.0;
  const double n = (j + 1 < N) ? u[p + 1] : 0.0;
  const double s = (j > 0) ? u[p - 1] : 0.0;
  const double kc = k[(i + 1) * K + (j + 1)];
  const double kE = 0.5 * (kc + k[(i + 2) * K + (j + 1)]);
  const double kW = 0.5 * (kc + k[i * K + (j + 1)]);
  const double kN = 0.5 * (kc + k[(i + 1) * K + (j + 2)]);
  const double kS = 0.5 * (kc + k[(i + 1) * K + j]);
  const double h1 = (double)(N + 1);
  return ((kE + kW + kN + kS) * c - kE * e - kW * w - kN * n - kS * s) * (h1 * h1);
}

// pass 0: dvec = w - e;  pass 1: gw <- A (w - e), partials (d, Ad), (e, Ae)
// (kind 1, the Euclidean loss: gw <- w - e, partials (d, d), (e, e))
__global__ __launch_bounds__(256) void k_loss(LossArgs a, int pass) {
  __shared__ double lds[4];
  const int b = blockIdx.y;
  const int N = a.N, n = N * N;
  const double* k = a.k + (size_t)b * (N + 2) * (N + 2);
  const double* w = a.w + (size_t)b * n;
  const double* e = a.e + (size_t)b * n;
  double* gw = a.gw + (size_t)b * n;
  double* dv = a.dvec + (size_t)b * n;
  double s0 = 0.0, s1 = 0.0;
  for (int q = 0; q < FLAT_PTS / 256; ++q) {
    const int p = blockIdx.x * FLAT_PTS + q * 256 + threadIdx.x;
    if (p >= n) break;
    if (pass == 0) {
      dv[p] = w[p] - e[p];
    } else if (a.kind == 1) {
      const double d = dv[p];
      gw[p] = d;
      s0 += d * d;
      s1 += e[p] * e[p];
    } else {
      const int i = p / N, j = p - i * N;
      const double ad = apply_A(k, dv, N, i, j);
      const double ae = apply_A(k, e, N, i, j);
      gw[p] = ad;
      s0 += dv[p] * ad;
      s1 += e[p] * ae;
    }
  }
  if (pass == 0) return;
  s0 = block_sum(s0, lds);
  s1 = block_sum(s1, lds);
  if (threadIdx.x == 0) {
    a.part[((size_t)b * a.nb + blockIdx.x) * 2 + 0] = s0;
    a.part[((size_t)b * a.nb + blockIdx.x) * 2 + 1] = s1;
  }
}

// per system: loss_b = ||d|| / ||e||, scale_b = 1 / (B ||d|| ||e||) in the loss's norm
__global__ __launch_bounds__(256) void k_loss_fin(LossArgs a) {
  __shared__ double lds[4];
  const int b = blockIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int q = threadIdx.x; q < a.nb; q += 256) {
    s0 += a.part[((size_t)b * a.nb + q) * 2 + 0];
    s1 += a.part[((size_t)b * a.nb + q) * 2 + 1];
  }
  s0 = block_sum(s0, lds);
  s1 = block_sum(s1, lds);
  if (threadIdx.x == 0) {
    const double dn = sqrt(fmax(s0, 0.0)), en = sqrt(fmax(s1, 0.0));
    a.loss[b] = en > 0.0 ? dn / en : 0.0;
    a.gscale[b] = (dn > 0.0 && en > 0.0) ? 1.0 / ((double)a.B * dn * en) : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Backward row kernel.  One thread per point; a block covers RB whole rows
// (N <= PB) or one PB-point segment of a row (N > PB).
//   mode 0 (start):  dv = s * scale * A(w-e) * W_P, plus dW_P, db_P
//   mode 1 (layer l): dv = W_l^T dz_l + sum_j T[y][j] Hc_b[x][c][j]
// then for the target layer tl = (start ? L-1 : l-1):
//   tl >= 0: dz_tl = dv * GELU'(z_tl), dW_tl, db_tl, row DFT partials of dz_tl
//   tl < 0 : dW_L, db_L of the lift (features phi)
// ---------------------------------------------------------------------------
template <typename acc_t, int C>
__global__ void k_bwd(BwdArgs a) {
  constexpr int PB = PtsPerBlock<acc_t>::value;
  __shared__ acc_t sA[PB][C + 1];     // dz (or dv, or s*g*v_L)
  __shared__ acc_t sV[PB][C + 1];     // v_tl (or features)
  __shared__ acc_t sW[C][C + 1];      // W_l (row o, col c)
  __shared__ acc_t sg[PB];
  const int N = a.N, n = N * N, MP = a.MP, twoM = 2 * a.M;
  const int b = blockIdx.x / a.nbs, ub = blockIdx.x - b * a.nbs;
  const int t = threadIdx.x;
  int x, y;
  bool valid;
  if (N <= PB) {
    const int RB = PB / N;
    x = ub * RB + t / N;
    y = t % N;
    valid = (t < RB * N) && x < N;
  } else {
    x = ub / a.S;
    y = (ub - x * a.S) * PB + t;
    valid = y < N;
  }
  // tail threads keep in-range indices so that no load can leave the buffers
  if (!valid) { x = 0; y = 0; }
  const size_t p = (size_t)x * N + y;
  const int tl = a.mode == 0 ? a.L - 1 : a.l - 1;
  const double* blob = a.blob;
  acc_t* pdW = (acc_t*)a.pdW;
  acc_t* pdb = (acc_t*)a.pdb;
  acc_t* pdWP = (acc_t*)a.pdWP;
  acc_t* pdbP = (acc_t*)a.pdbP;
  acc_t* pdWL = (acc_t*)a.pdWL;
  acc_t* pdbL = (acc_t*)a.pdbL;
  // --- dv ---
  acc_t dv[C];
  if (a.mode == 0) {
    const double snorm = a.st[b].snorm;
    const acc_t gws = valid ? (acc_t)(snorm * a.gscale[b] * a.gw[(size_t)b * n + p]) : (acc_t)0;
    const acc_t* z = (const acc_t*)a.z + (size_t)(a.L - 1) * a.z_layer + (size_t)b * a.z_sys + p * C;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      dv[c] = gws * (acc_t)blob[a.off_WP + c];
      sA[t][c] = valid ? gws * gelu_t<acc_t>(z[c]) : (acc_t)0;   // for dW_P
    }
    sg[t] = gws;
    __syncthreads();
    if (t < C) {
      acc_t s = 0;
      for (int q = 0; q < PB; ++q) s += sA[q][t];
      pdWP[(size_t)blockIdx.x * C + t] = s;
    }
    if (t == 0) {
      acc_t s = 0;
      for (int q = 0; q < PB; ++q) s += sg[q];
      pdbP[blockIdx.x] = s;
    }
    __syncthreads();
  } else {
    for (int q = t; q < C * C; q += PB) sW[q / C][q % C] = (acc_t)blob[a.off_W + q];
    __syncthreads();
    const acc_t* dzl = (const acc_t*)a.dz_in + (size_t)b * n * C + p * C;
    acc_t dzv[C];
#pragma unroll
    for (int o = 0; o < C; ++o) dzv[o] = valid ? dzl[o] : (acc_t)0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      acc_t s = 0;
#pragma unroll
      for (int o = 0; o < C; ++o) s += sW[o][c] * dzv[o];
      dv[c] = s;
    }
    if (valid) {
      const acc_t* Tr = (const acc_t*)a.T + (size_t)y * MP;
      const acc_t* Hc = (const acc_t*)a.Hcb + (size_t)b * a.hc_sys + (size_t)x * C * MP;
      for (int j = 0; j < twoM; ++j) {
        const acc_t tj = Tr[j];
#pragma unroll
        for (int c = 0; c < C; ++c) dv[c] += tj * Hc[c * MP + j];
      }
    }
  }
  // --- target layer ---
  const double hstep = 1.0 / (double)(N + 1);
  if (tl >= 0) {
    const acc_t* z = (const acc_t*)a.z + (size_t)tl * a.z_layer + (size_t)b * a.z_sys + p * C;
    acc_t* dzo = (acc_t*)a.dz_out + (size_t)b * n * C + p * C;
    // input v_tl of layer tl
    if (tl >= 1) {
      const acc_t* v = (const acc_t*)a.act + (size_t)(tl - 1) * a.act_slot + (size_t)b * a.act_sys + p * C;
#pragma unroll
      for (int c = 0; c < C; ++c) sV[t][c] = valid ? v[c] : (acc_t)0;
    } else {
      double phi[4] = {0.0, 0.0, 0.0, 0.0};
      if (valid) {
        const double snorm = a.st[b].snorm;
        const double inv_s = snorm > 0.0 ? 1.0 / snorm : 0.0;
        phi[0] = a.r[(size_t)b * n + p] * inv_s;
        phi[1] = log(a.k[(size_t)b * (N + 2) * (N + 2) + (size_t)(x + 1) * (N + 2) + y + 1]);
        phi[2] = (double)(x + 1) * hstep;
        phi[3] = (double)(y + 1) * hstep;
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double v0 = blob[a.off_bL + c];
        for (int f = 0; f < 4; ++f) v0 += blob[a.off_WL + c * 4 + f] * phi[f];
        sV[t][c] = valid ? (acc_t)v0 : (acc_t)0;
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const acc_t d = valid ? dv[c] * dgelu_t<acc_t>(z[c]) : (acc_t)0;
      sA[t][c] = d;
      if (valid) dzo[c] = d;
    }
    __syncthreads();
    // dW_tl[o][c] = sum dz[o] v[c], db_tl[o] = sum dz[o]
    for (int q = t; q < C * C; q += PB) {
      const int o = q / C, c = q - o * C;
      acc_t s = 0;
      for (int u = 0; u < PB; ++u) s += sA[u][o] * sV[u][c];
      pdW[(size_t)blockIdx.x * C * C + q] = s;
    }
    for (int o = t; o < C; o += PB) {
      acc_t s = 0;
      for (int u = 0; u < PB; ++u) s += sA[u][o];
      pdb[(size_t)blockIdx.x * C + o] = s;
    }
    // row partials of the y-direction DFT of dz: Gb[x][seg][j][o] = sum_y T[y][j] dz[y][o]
    acc_t* Gb = (acc_t*)a.Gb;
    if (N <= PB) {
      const int RB = PB / N;
      for (int q = t; q < RB * MP * C; q += PB) {
        const int xr = q / (MP * C), rem = q - xr * (MP * C), j = rem / C, o = rem - j * C;
        const int xx = ub * RB + xr;
        if (xx >= N) continue;
        acc_t s = 0;
        if (j < twoM)
          for (int yy = 0; yy < N; ++yy) s += ((const acc_t*)a.T)[(size_t)yy * MP + j] * sA[xr * N + yy][o];
        Gb[(size_t)b * a.gb_sys + (size_t)xx * MP * C + rem] = s;
      }
    } else {
      const int xb = ub / a.S, seg = ub - xb * a.S;   // block-uniform row and segment
      const int y0 = seg * PB;
      for (int q = t; q < MP * C; q += PB) {
        const int j = q / C, o = q - j * C;
        acc_t s = 0;
        if (j < twoM)
          for (int u = 0; u < PB && y0 + u < N; ++u) s += ((const acc_t*)a.T)[(size_t)(y0 + u) * MP + j] * sA[u][o];
        Gb[(size_t)b * a.gb_sys + ((size_t)xb * a.S + seg) * MP * C + q] = s;
      }
    }
  } else {
    // lift: v_0 = W_L phi + b_L
    if (valid) {
      const double snorm = a.st[b].snorm;
      const double inv_s = snorm > 0.0 ? 1.0 / snorm : 0.0;
      sV[t][0] = (acc_t)(a.r[(size_t)b * n + p] * inv_s);
      sV[t][1] = (acc_t)log(a.k[(size_t)b * (N + 2) * (N + 2) + (size_t)(x + 1) * (N + 2) + y + 1]);
      sV[t][2] = (acc_t)((double)(x + 1) * hstep);
      sV[t][3] = (acc_t)((double)(y + 1) * hstep);
    } else {
      sV[t][0] = sV[t][1] = sV[t][2] = sV[t][3] = (acc_t)0;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) sA[t][c] = valid ? dv[c] : (acc_t)0;
    if (a.dphi0 && valid) {
      // gradient w.r.t. the first feature r/s: W_L[:, 0]^T dv0
      double d = 0.0;
#pragma unroll
      for (int c = 0; c < C; ++c) d += blob[a.off_WL + c * 4] * (double)dv[c];
      a.dphi0[(size_t)b * n + p] = d;
    }
    __syncthreads();
    for (int q = t; q < C * 4; q += PB) {
      const int c = q / 4, f = q - c * 4;
      acc_t s = 0;
      for (int u = 0; u < PB; ++u) s += sA[u][c] * sV[u][f];
      pdWL[(size_t)blockIdx.x * C * 4 + q] = s;
    }
    for (int c = t; c < C; c += PB) {
      acc_t s = 0;
      for (int u = 0; u < PB; ++u) s += sA[u][c];
      pdbL[(size_t)blockIdx.x * C + c] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Spectral adjoint mixing for one ky: G^ = N^-2 g_ky sum_chunks Vp (kept per
// system for dR) and G^_V[c][a] = sum_o G^[o][a] conj(R[c][o][a][ky]), written
// to Wh for the unit-scale synthesis.
// ---------------------------------------------------------------------------
template <typename acc_t, int C>
__global__ __launch_bounds__(256) void k_bspec_mix(BSpecArgs a) {
  __shared__ acc_t Gr_[C][33], Gi_[C][33];
  const int ky = blockIdx.x, b = blockIdx.y;
  const int M = a.M, twoM = 2 * M, MP = round16_t(twoM);
  const int t = threadIdx.x;
  const acc_t* Vp = (const acc_t*)a.Vp + (size_t)b * a.vp_sys + (size_t)ky * a.XS * C * twoM * 2;
  // adjoint of the synthesis normalisation: Fourier N^-2 g_ky, sine (2/(N+1))^2
  const acc_t sc = a.basis == B_SINE ? (acc_t)(4.0 / ((double)(a.N + 1) * (double)(a.N + 1)))
                                     : (acc_t)((ky == 0 ? 1.0 : 2.0) / ((double)a.N * (double)a.N));
  acc_t* Gh = (acc_t*)a.Gh + (size_t)b * a.gh_sys + (size_t)ky * C * twoM * 2;
  for (int q = t; q < C * twoM; q += 256) {
    const int o = q / twoM, kx = q - o * twoM;
    acc_t gr = 0, gi = 0;
    for (int xs = 0; xs < a.XS; ++xs) {
      gr += Vp[(size_t)xs * C * twoM * 2 + 2 * q];
      gi += Vp[(size_t)xs * C * twoM * 2 + 2 * q + 1];
    }
    gr *= sc;
    gi *= sc;
    Gr_[o][kx] = gr;
    Gi_[o][kx] = gi;
    Gh[2 * q] = gr;
    Gh[2 * q + 1] = gi;
  }
  __syncthreads();
  // R layout [ky][a][c][o] complex
  const acc_t* R = (const acc_t*)a.R + (size_t)ky * twoM * C * C * 2;
  acc_t* Wh = (acc_t*)a.Wh + (size_t)b * a.wh_sys + (size_t)ky * C * MP * 2;
  for (int q = t; q < C * twoM; q += 256) {
    const int c = q / twoM, kx = q - c * twoM;
    const acc_t* Rk = R + (size_t)kx * C * C * 2 + (size_t)c * C * 2;
    acc_t sr = 0, si = 0;
    for (int o = 0; o < C; ++o) {
      const acc_t rr = Rk[2 * o], ri = Rk[2 * o + 1];
      // G^[o] * conj(R[c][o])
      sr += Gr_[o][kx] * rr + Gi_[o][kx] * ri;
      si += Gi_[o][kx] * rr - Gr_[o][kx] * ri;
    }
    Wh[2 * (c * MP + kx)] = sr;
    Wh[2 * (c * MP + kx) + 1] = si;
  }
}

// dR[c][o][a][ky] = sum_b G^_b[o][a][ky] conj(V^_b[c][a][ky]), into the float64
// gradient blob (Re block, then Im block).  Grid: (ky, a).
template <typename acc_t, int C>
__global__ __launch_bounds__(256) void k_dR(BSpecArgs a, double* grad_re, double* grad_im) {
  const int ky = blockIdx.x, kx = blockIdx.y;
  const int M = a.M, twoM = 2 * M;
  const int t = threadIdx.x;
  for (int q = t; q < C * C; q += 256) {
    const int c = q / C, o = q - c * C;
    double sr = 0.0, si = 0.0;
#pragma unroll 8
    for (int b = 0; b < a.B; ++b) {
      const acc_t* G = (const acc_t*)a.Gh + (size_t)b * a.gh_sys + (size_t)ky * C * twoM * 2;
      const acc_t* V = (const acc_t*)a.Vsave + (size_t)b * a.vs_sys + (size_t)ky * C * twoM * 2;
      const acc_t gr = G[2 * (o * twoM + kx)], gi = G[2 * (o * twoM + kx) + 1];
      const acc_t vr = V[2 * (c * twoM + kx)], vi = V[2 * (c * twoM + kx) + 1];
      sr += (double)(gr * vr + gi * vi);
      si += (double)(gi * vr - gr * vi);
    }
    const size_t idx = (((size_t)c * C + o) * twoM + kx) * M + ky;
    grad_re[idx] = sr;
    grad_im[idx] = si;
  }
}

// Gradient of L = sum_p g_p w_p, w = B(r) = s NO(r/s), s = ||r||_2 / N, with
// respect to r.  With D = dL/d(r/s) at fixed s (dphi0, from the backward
// pass) and ds/dr = r / (N^2 s):
//   dL/dr = D / s + r (sum_p g_p w_p / s - sum_p D_p r_p / s^2) / (N^2 s),
// zero where s = 0 (B(0) = 0).  One block per system, fixed-order sums.
__global__ __launch_bounds__(256) void k_grad_r(int N, const SysState* st, const double* r, const double* g,
                                                 const double* w, const double* dphi0, double* grad_r) {
  __shared__ double lds[4];
  const size_t n = (size_t)N * N;
  const size_t o = (size_t)blockIdx.x * n;
  const double s = st[blockIdx.x].snorm;
  double gw = 0.0, dr = 0.0;
  for (size_t p = threadIdx.x; p < n; p += 256) {
    gw += g[o + p] * w[o + p];
    dr += dphi0[o + p] * r[o + p];
  }
  gw = block_sum(gw, lds);
  dr = block_sum(dr, lds);
  if (!(s > 0.0)) {
    for (size_t p = threadIdx.x; p < n; p += 256) grad_r[o + p] = 0.0;
    return;
  }
  const double coef = (gw / s - dr / (s * s)) / ((double)n * s);
  for (size_t p = threadIdx.x; p < n; p += 256) grad_r[o + p] = dphi0[o + p] / s + r[o + p] * coef;
}

void launch_grad_r(int N, int B, const SysState* st, const double* r, const double* g, const double* w,
                   const double* dphi0, double* grad_r, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_r, dim3(B), dim3(256), 0, s, N, st, r, g, w, dphi0, grad_r);
}

// Fixed-order reduction of per-block partials, out[i] = sum_blk part[blk][i],
// in two stages: stage 1 sums chunks of consecutive blocks (64 columns per
// workgroup, four interleaved block sequences combined in a fixed order),
// stage 2 sums the chunk results in chunk order.
template <typename acc_t>
__global__ __launch_bounds__(256) void k_reduce1(const acc_t* part, int nblk, int count, int qchunk,
                                                 double* stage) {
  __shared__ double lds[4][64];
  const int cl = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  const int q0 = blockIdx.y * qchunk, q1 = min(nblk, q0 + qchunk);
  double s = 0.0;
  // unrolled so that the loads issue together; the sum keeps its order
  if (c < count)
#pragma unroll 8
    for (int q = q0 + rg; q < q1; q += 4) s += (double)part[(size_t)q * count + c];
  lds[rg][cl] = s;
  __syncthreads();
  if (rg == 0 && c < count)
    stage[(size_t)blockIdx.y * count + c] = (lds[0][cl] + lds[1][cl]) + (lds[2][cl] + lds[3][cl]);
}

__global__ __launch_bounds__(256) void k_reduce2(const double* stage, int nq, int count, double* out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  double s = 0.0;
#pragma unroll 16
  for (int q = 0; q < nq; ++q) s += stage[(size_t)q * count + i];
  out[i] = s;
}

// AdamW with decoupled weight decay on the float64 master weights.
__global__ __launch_bounds__(256) void k_adamw(double* theta, const double* g, double* m, double* v, size_t n,
                                               double lr, double wd, double b1, double b2, double eps, double bc1,
                                               double bc2) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double th = theta[i] * (1.0 - lr * wd);
  const double gi = g[i];
  const double mi = b1 * m[i] + (1.0 - b1) * gi;
  const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th -= lr * (mi / bc1) / (sqrt(vi / bc2) + eps);
  theta[i] = th;
}

// ---------------------------------------------------------------------------
// Device re-layout of the float64 blob into the arrays the kernels read.
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ void store_as(void* p, size_t i, double v);
template <> __device__ __forceinline__ void store_as<double>(void* p, size_t i, double v) { ((double*)p)[i] = v; }
template <> __device__ __forceinline__ void store_as<float>(void* p, size_t i, double v) { ((float*)p)[i] = (float)v; }
template <> __device__ __forceinline__ void store_as<uint16_t>(void* p, size_t i, double v) {
  ((uint16_t*)p)[i] = f2bf((float)v);
}

template <typename in_t, typename acc_t>
__global__ __launch_bounds__(256) void k_derive(DeriveArgs a) {
  const int C = a.C, M = a.M, twoM = 2 * M, KPL = a.kpl, KSTEP = 4 * KPL;
  const int l = blockIdx.z, region = blockIdx.y;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  const double* w = a.blob;
  const size_t nR = (size_t)C * C * twoM * M;
  const size_t offl = (size_t)C * 4 + C + (size_t)l * (2 * nR + (size_t)C * C + C);
  const double* Rre = w + offl;
  const double* Rim = Rre + nR;
  const double* W = Rim + nR;
  const double* bl = W + (size_t)C * C;
  const double* WL = w;
  const double* bL = w + (size_t)C * 4;
  if (region == 0) {
    const int KWP = l == 0 ? KSTEP : C;
    if (i >= (size_t)C * KWP) return;
    const int oc = (int)(i / KWP), kw = (int)(i % KWP);
    double v = 0.0;
    if (l == 0) {
      if (kw < 4)
        for (int c = 0; c < C; ++c) v += W[oc * C + c] * WL[c * 4 + kw];
    } else {
      const int kss = kw / KSTEP, rem = kw % KSTEP, g = rem / KPL, e = rem % KPL;
      v = W[oc * C + g * (C / 4) + kss * KPL + e];
    }
    store_as<in_t>(a.Wfrag[l], i, v);
  } else if (region == 1) {
    if (i >= (size_t)C) return;
    double v = bl[i];
    if (l == 0)
      for (int c = 0; c < C; ++c) v += W[i * C + c] * bL[c];
    store_as<acc_t>(a.bias[l], i, v);
  } else if (region == 2) {
    if (i >= nR) return;
    // destination [ky][a][c][o]; source R[c][o][a][ky]
    const size_t oc = i % C, c = (i / C) % C, kx = (i / ((size_t)C * C)) % twoM, ky = i / ((size_t)C * C * twoM);
    const size_t src = ((c * C + oc) * twoM + kx) * M + ky;
    store_as<acc_t>(a.Rmix[l], 2 * i, Rre[src]);
    store_as<acc_t>(a.Rmix[l], 2 * i + 1, Rim[src]);
  } else if (l == 0) {
    if (i >= (size_t)C) return;
    const size_t offP = (size_t)C * 4 + C + (size_t)a.L * (2 * nR + (size_t)C * C + C);
    store_as<acc_t>(a.WP, i, w[offP + i]);
    store_as<acc_t>(a.WL0, i, WL[i * 4]);
  }
}

__global__ __launch_bounds__(256) void k_scale_rows(double* g, const double* scale, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  g[(size_t)blockIdx.y * n + i] *= scale[blockIdx.y];
}

// ---- launchers ------------------------------------------------------------

void launch_scale_rows(double* g, const double* scale, int B, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)((n + 255) / 256), B), dim3(256), 0, s, g, scale, n);
}

void launch_loss(const LossArgs& a, hipStream_t s) {
  const int n = a.N * a.N;
  const dim3 g((n + FLAT_PTS - 1) / FLAT_PTS, a.B);
  hipLaunchKernelGGL(k_loss, g, dim3(256), 0, s, a, 0);
  hipLaunchKernelGGL(k_loss, g, dim3(256), 0, s, a, 1);
  hipLaunchKernelGGL(k_loss_fin, dim3(a.B), dim3(256), 0, s, a);
}

template <typename acc_t>
static void bwd_c(const BwdArgs& a, int C, int nblk, hipStream_t s) {
  constexpr int PB = PtsPerBlock<acc_t>::value;
  if (C == 16) hipLaunchKernelGGL((k_bwd<acc_t, 16>), dim3(nblk), dim3(PB), 0, s, a);
  else hipLaunchKernelGGL((k_bwd<acc_t, 32>), dim3(nblk), dim3(PB), 0, s, a);
}

void launch_bwd(const BwdArgs& a, int prec, int C, int nblk, hipStream_t s) {
  ProfScope ps(PK_TRAIN_BWD, s);
  if (prec == P64) bwd_c<double>(a, C, nblk, s);
  else bwd_c<float>(a, C, nblk, s);
}

void launch_bspec_mix(const BSpecArgs& a, int prec, int C, hipStream_t s) {
  const dim3 g(a.M, a.B);
  if (prec == P64) {
    if (C == 16) hipLaunchKernelGGL((k_bspec_mix<double, 16>), g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_bspec_mix<double, 32>), g, dim3(256), 0, s, a);
  } else {
    if (C == 16) hipLaunchKernelGGL((k_bspec_mix<float, 16>), g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_bspec_mix<float, 32>), g, dim3(256), 0, s, a);
  }
}

void launch_dR(const BSpecArgs& a, int prec, int C, double* gre, double* gim, hipStream_t s) {
  const dim3 g(a.M, 2 * a.M);
  if (prec == P64) {
    if (C == 16) hipLaunchKernelGGL((k_dR<double, 16>), g, dim3(256), 0, s, a, gre, gim);
    else hipLaunchKernelGGL((k_dR<double, 32>), g, dim3(256), 0, s, a, gre, gim);
  } else {
    if (C == 16) hipLaunchKernelGGL((k_dR<float, 16>), g, dim3(256), 0, s, a, gre, gim);
    else hipLaunchKernelGGL((k_dR<float, 32>), g, dim3(256), 0, s, a, gre, gim);
  }
}

void launch_reduce(const void* part, int prec, int nblk, int count, double* out, double* stage,
                   hipStream_t s) {
  const int nq = std::min(REDUCE_CHUNKS, nblk);
  const int qchunk = (nblk + nq - 1) / nq;
  const int nqe = (nblk + qchunk - 1) / qchunk;   // chunks actually holding blocks
  const dim3 g1((count + 63) / 64, nqe);
  if (prec == P64)
    hipLaunchKernelGGL(k_reduce1<double>, g1, dim3(256), 0, s, (const double*)part, nblk, count, qchunk, stage);
  else
    hipLaunchKernelGGL(k_reduce1<float>, g1, dim3(256), 0, s, (const float*)part, nblk, count, qchunk, stage);
  hipLaunchKernelGGL(k_reduce2, dim3((count + 255) / 256), dim3(256), 0, s, (const double*)stage, nqe, count, out);
}

void launch_adamw(double* theta, const double* g, double* m, double* v, size_t n, double lr, double wd, double b1,
                  double b2, double eps, long long t, hipStream_t s) {
  const double bc1 = 1.0 - pow(b1, (double)t), bc2 = 1.0 - pow(b2, (double)t);
  hipLaunchKernelGGL(k_adamw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, g, m, v, n, lr, wd, b1, b2,
                     eps, bc1, bc2);
}

void launch_derive(const DeriveArgs& a, int prec, hipStream_t s) {
  const size_t nR = (size_t)a.C * a.C * 2 * a.M * a.M;
  const dim3 g((unsigned)((nR + 255) / 256), 4, a.L);
  if (prec == P64) hipLaunchKernelGGL((k_derive<double, double>), g, dim3(256), 0, s, a);
  else if (prec == P32) hipLaunchKernelGGL((k_derive<float, float>), g, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_derive<uint16_t, float>), g, dim3(256), 0, s, a);
}

}  // namespace fcgno
