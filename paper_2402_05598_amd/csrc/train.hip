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
#include "mfma.h"
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
// Backward layer kernel (matrix cores).  One wave per row segment of TPW
// 16-point tiles (x = row, y = column, p = x N + y), four waves per block:
//   mode 0 (start):  dv = s * scale_b * gw * W_P            (outer product)
//   mode 1 (layer l): dv = W_l^T dz_l + sum_j T[y][j] Hc_b[x][c][j]
//       per tile [16 y] x [C]: A operands dz_l and T rows, B operands W_l and
//       the row's adjoint synthesis Hc_b[x] (held for the whole segment)
// then for the target layer tl = (mode 0 ? L-1 : l-1):
//   tl >= 0: dz_tl = dv * GELU'(z_tl), stored; dW_tl += dz_tl^T v_tl and
//       the row partials Gb[j][c] += sum_y T[y][j] dz_tl[y][c] (both products
//       contract over the tile's points, read from the accumulator layout);
//       db_tl += sum dz_tl
//   tl < 0 (lift): dW_L += dv^T phi, db_L += sum dv, and the feature
//       gradient dphi0[p] = W_L[:, 0] . dv
// The four waves' partial weight gradients are added in a fixed order and
// written once per block.  Contraction order of the channel products: step
// ks, lane group g takes channel g KC + ks (KC = C / 4), so that each lane's
// A operand of a tile is one contiguous run of its point's channels; the
// same for the synthesis index j (KJ = MP / 4).
// ---------------------------------------------------------------------------
// SRC: 0 start (dv from the projection), 1 layer l.  TGT: 0 target layer
// tl >= 1 (input from the saved activations), 1 target layer 0 (input
// recomputed from the lift), 2 the lift itself (tl < 0).
template <int PREC, int C, int MP, int SRC, int TGT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PREC == P32 && TGT != 1 ? 3 : 1))) void k_bwd(BwdArgs a) {
  using M_ = Mf<PREC>;
  using acc_t = typename M_::acc_t;
  using accv_t = typename M_::accv_t;
  constexpr int NOB = C / 16, KC = C / 4, KJ = MP / 4, MB = MP / 16;
  constexpr int NW = 4;
  static_assert(M_::KPL == 1, "FP32 / FP64 only");
  __shared__ acc_t red[NW][C * C];
  __shared__ acc_t red2[NW][4][2 * C + 1];   // [wave][lane group][per-channel sums, db_P]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n16 = lane & 15, g = lane >> 4;
  const int N = a.N, n = N * N;
  const int tl = SRC == 0 ? a.L - 1 : a.l - 1;
  const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * NW + w);
  const bool live = item < a.B * a.nbs;
  const int b = live ? item / a.nbs : 0;
  const int rem = item - b * a.nbs;
  const int x = live ? rem / a.S : 0, seg = live ? rem - (rem / a.S) * a.S : 0;
  const int nyt = (N + 15) >> 4;
  const int t0 = seg * TPW, t1 = live ? min(nyt, t0 + TPW) : t0;
  const double* blob = a.blob;
  const double hstep = 1.0 / (double)(N + 1);
  const double snorm = a.st[b].snorm;
  const double inv_s = snorm > 0.0 ? 1.0 / snorm : 0.0;
  const acc_t* T = (const acc_t*)a.T;
  const size_t rowp = (size_t)x * N;   // first point of the row
  const acc_t* zt = (const acc_t*)a.z + (size_t)(TGT == 2 ? 0 : tl) * a.z_layer + (size_t)b * a.z_sys + rowp * C;
  const acc_t* vt = (const acc_t*)a.act + (size_t)(TGT == 0 ? tl - 1 : 0) * a.act_slot + (size_t)b * a.act_sys + rowp * C;
  const acc_t* dzl = (const acc_t*)a.dz_in + (size_t)b * n * C + rowp * C;
  acc_t* dzo = (acc_t*)a.dz_out + (size_t)b * n * C + rowp * C;
  const acc_t* lk = (const acc_t*)a.logk + (size_t)b * n + rowp;   // log k of the forward's set-up
  const double* rr = a.r + (size_t)b * n + rowp;

  // B operands of the layer products: W_l[o = g KC + ks][c], Hc_b[x][c][j = g KJ + ks]
  acc_t BW[SRC == 1 ? KC : 1][NOB], BH[SRC == 1 ? KJ : 1][NOB], wpc[NOB];
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob) {
    const int c = ob * 16 + n16;
    if constexpr (SRC == 1) {
#pragma unroll
      for (int ks = 0; ks < KC; ++ks) BW[ks][ob] = (acc_t)blob[a.off_W + (size_t)(g * KC + ks) * C + c];
      const acc_t* Hc = (const acc_t*)a.Hcb + (size_t)b * a.hc_sys + ((size_t)x * C + c) * MP + g * KJ;
#pragma unroll
      for (int ks = 0; ks < KJ; ++ks) BH[ks][ob] = Hc[ks];
    } else {
      wpc[ob] = (acc_t)blob[a.off_WP + c];
    }
  }
  accv_t dW[NOB][NOB], G2[MB][NOB];
#pragma unroll
  for (int i = 0; i < NOB; ++i)
#pragma unroll
    for (int j = 0; j < NOB; ++j) dW[i][j] = accv_t{0, 0, 0, 0};
#pragma unroll
  for (int jb = 0; jb < MB; ++jb)
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) G2[jb][ob] = accv_t{0, 0, 0, 0};
  acc_t s1[NOB], s2[NOB];   // db (or db_L) and dW_P per channel; dW_L through dW
  acc_t dbp = 0;
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob) s1[ob] = s2[ob] = 0;

  // A operands of GEMM1 for one tile (this lane's point y0 + n, contiguous
  // channel and twiddle runs), two tiles in flight; rows past N read row
  // N - 1 (zero in T) and are masked
  struct TileA {
    acc_t dz[SRC == 1 ? KC : 1], tw[SRC == 1 ? KJ : 1];
  };
  auto load_a = [&](int t, TileA& ta) __attribute__((always_inline)) {
    if constexpr (SRC == 1) {
      const int ya = t * 16 + n16;
      const int yc = ya < N ? ya : N - 1;
      const acc_t* dzr = dzl + (size_t)yc * C + g * KC;
      const acc_t* tr = T + (size_t)ya * MP + g * KJ;   // T has NP >= ya + 1 rows
#pragma unroll
      for (int ks = 0; ks < KC; ++ks) ta.dz[ks] = dzr[ks];
#pragma unroll
      for (int ks = 0; ks < KJ; ++ks) ta.tw[ks] = tr[ks];
    }
  };
  TileA ring[2];
  if (t0 < t1) {
    load_a(t0, ring[0]);
    load_a(min(t0 + 1, t1 - 1), ring[1]);
  }
  auto tile = [&](int t, TileA& ta) __attribute__((always_inline)) {
    const int y0 = t * 16;
    int yr[4];
    bool vr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int y = y0 + M_::row(g, i);
      vr[i] = y < N;
      yr[i] = vr[i] ? y : N - 1;
    }
    // loads of the accumulator-layout operands first: their latency runs
    // under GEMM1
    acc_t zv[NOB][4], vv[NOB][4], gws[4], A2[4][MB];
    double ph0[4], ph1[4];
    if constexpr (SRC == 0) {
      const double sc = snorm * a.gscale[b];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        gws[i] = vr[i] ? (acc_t)(sc * a.gw[(size_t)b * n + rowp + yr[i]]) : (acc_t)0;
    }
    if constexpr (TGT <= 1) {
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) zv[ob][i] = zt[(size_t)yr[i] * C + ob * 16 + n16];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jb = 0; jb < MB; ++jb) A2[i][jb] = T[(size_t)(y0 + M_::row(g, i)) * MP + jb * 16 + n16];
    }
    if constexpr (TGT == 0) {
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) vv[ob][i] = vt[(size_t)yr[i] * C + ob * 16 + n16];
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ph0[i] = rr[yr[i]] * inv_s;
        ph1[i] = (double)lk[yr[i]];
      }
    }
    // --- dv in the accumulator layout: item i of lane (c, g) is dv[y0 + row(g, i)][c]
    accv_t dv[NOB];
    if constexpr (SRC == 0) {
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) dv[ob][i] = gws[i] * wpc[ob];
    } else {
      const bool va = y0 + n16 < N;
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob) {
        accv_t acc = accv_t{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KC; ++ks) acc = M_::mma(va ? ta.dz[ks] : (acc_t)0, BW[ks][ob], acc);
#pragma unroll
        for (int ks = 0; ks < KJ; ++ks) acc = M_::mma(ta.tw[ks], BH[ks][ob], acc);
        dv[ob] = acc;
      }
    }
    if constexpr (TGT <= 1) {
      // --- dz_tl = dv GELU'(z_tl), its store, db, dW_P
      accv_t dz[NOB];
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const acc_t d = vr[i] ? dv[ob][i] * dgelu_t<acc_t>(zv[ob][i]) : (acc_t)0;
          dz[ob][i] = d;
          if (vr[i]) dzo[(size_t)yr[i] * C + ob * 16 + n16] = d;
          s1[ob] += d;
          if constexpr (SRC == 0) s2[ob] += vr[i] ? gws[i] * gelu_t<acc_t>(zv[ob][i]) : (acc_t)0;
        }
      if constexpr (SRC == 0) {
        if (n16 == 0) {
#pragma unroll
          for (int i = 0; i < 4; ++i) dbp += gws[i];
        }
      }
      // --- input v_tl of layer tl in the accumulator layout
      accv_t v[NOB];
      if constexpr (TGT == 0) {
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
          for (int i = 0; i < 4; ++i) v[ob][i] = vr[i] ? vv[ob][i] : (acc_t)0;
      } else {
        // v_0 = W_L phi + b_L
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob) {
          const int c = ob * 16 + n16;
          const double bl = blob[a.off_bL + c], w0 = blob[a.off_WL + c * 4], w1 = blob[a.off_WL + c * 4 + 1],
                       w2 = blob[a.off_WL + c * 4 + 2], w3 = blob[a.off_WL + c * 4 + 3];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double v0 = bl + w0 * ph0[i] + w1 * ph1[i] + w2 * ((double)(x + 1) * hstep) +
                              w3 * ((double)(yr[i] + 1) * hstep);
            v[ob][i] = vr[i] ? (acc_t)v0 : (acc_t)0;
          }
        }
      }
      // --- dW_tl[o][c] += sum_y dz[y][o] v[y][c]: K-step i takes the rows
      // row(g, i) of both accumulator layouts
#pragma unroll
      for (int oo = 0; oo < NOB; ++oo)
#pragma unroll
        for (int oc = 0; oc < NOB; ++oc)
#pragma unroll
          for (int i = 0; i < 4; ++i) dW[oo][oc] = M_::mma(dz[oo][i], v[oc][i], dW[oo][oc]);
      // --- row partials Gb[j][c] += sum_y T[y][j] dz[y][c]
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jb = 0; jb < MB; ++jb)
#pragma unroll
          for (int ob = 0; ob < NOB; ++ob) G2[jb][ob] = M_::mma(A2[i][jb], dz[ob][i], G2[jb][ob]);
    } else {
      // --- lift: dW_L[c][f] += dv[y][c] phi[y][f] (in dW[0][0] .. as
      // [c][f] sums per lane), db_L, dphi0
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double phi[4] = {ph0[i], ph1[i], (double)(x + 1) * hstep, (double)(yr[i] + 1) * hstep};
        double d0 = 0.0;
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob) {
          const acc_t d = vr[i] ? dv[ob][i] : (acc_t)0;
          s1[ob] += d;
#pragma unroll
          for (int f = 0; f < 4; ++f) dW[ob][0][f] += d * (acc_t)phi[f];
          d0 += blob[a.off_WL + (ob * 16 + n16) * 4] * (double)d;
        }
        if (a.dphi0) {
          // W_L[:, 0] . dv over the C channels: lanes n of this group, then blocks ob
          d0 += __shfl_xor(d0, 1, 64);
          d0 += __shfl_xor(d0, 2, 64);
          d0 += __shfl_xor(d0, 4, 64);
          d0 += __shfl_xor(d0, 8, 64);
          if (n16 == 0 && vr[i]) a.dphi0[(size_t)b * n + rowp + yr[i]] = d0;
        }
      }
    }
  };
  for (int t = t0; t < t1; t += 2) {
    tile(t, ring[0]);
    load_a(min(t + 2, t1 - 1), ring[0]);
    if (t + 1 < t1) {
      tile(t + 1, ring[1]);
      load_a(min(t + 3, t1 - 1), ring[1]);
    }
  }
  // --- the segment's row partial spectrum
  if constexpr (TGT <= 1) {
    if (live) {
      acc_t* Gb = (acc_t*)a.Gb + (size_t)b * a.gb_sys + ((size_t)x * a.S + seg) * MP * C;
#pragma unroll
      for (int jb = 0; jb < MB; ++jb)
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
          for (int i = 0; i < 4; ++i) Gb[(jb * 16 + M_::row(g, i)) * C + ob * 16 + n16] = G2[jb][ob][i];
    }
  }

  // --- the block's partial gradients: four waves in a fixed order
  if constexpr (TGT <= 1) {
    // accumulator item i of lane (c, g) in tile (oo, oc) holds dW[oo 16 + row(g, i)][oc 16 + c]
#pragma unroll
    for (int oo = 0; oo < NOB; ++oo)
#pragma unroll
      for (int oc = 0; oc < NOB; ++oc)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[w][(oo * 16 + M_::row(g, i)) * C + oc * 16 + n16] = dW[oo][oc][i];
  } else {
    // dW_L[c][f] per lane (group g) in dW[ob][0][f]
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
      for (int f = 0; f < 4; ++f) red[w][(g * C + ob * 16 + n16) * 4 + f] = dW[ob][0][f];
  }
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob) {
    red2[w][g][ob * 16 + n16] = s1[ob];
    red2[w][g][C + ob * 16 + n16] = s2[ob];
  }
  if (n16 == 0) red2[w][g][2 * C] = dbp;
  __syncthreads();
  const size_t blk = blockIdx.x;
  if constexpr (TGT <= 1) {
    for (int q = threadIdx.x; q < C * C; q += 256) {
      acc_t sum = 0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) sum += red[ww][q];
      ((acc_t*)a.pdW)[blk * C * C + q] = sum;
    }
  } else {
    for (int q = threadIdx.x; q < C * 4; q += 256) {
      acc_t sum = 0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww)
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) sum += red[ww][gg * C * 4 + q];
      ((acc_t*)a.pdWL)[blk * C * 4 + q] = sum;
    }
  }
  for (int c = threadIdx.x; c < C; c += 256) {
    acc_t u0 = 0, u1 = 0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww)
#pragma unroll
      for (int gg = 0; gg < 4; ++gg) {
        u0 += red2[ww][gg][c];
        u1 += red2[ww][gg][C + c];
      }
    ((acc_t*)(TGT <= 1 ? a.pdb : a.pdbL))[blk * C + c] = u0;
    if constexpr (SRC == 0) ((acc_t*)a.pdWP)[blk * C + c] = u1;
  }
  if constexpr (SRC == 0) {
    if (threadIdx.x == 0) {
      acc_t u = 0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww)
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) u += red2[ww][gg][2 * C];
      ((acc_t*)a.pdbP)[blk] = u;
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
  // G^ mode-major, [ky][a][system][o] complex, for the weight gradient's products
  acc_t* Gh = (acc_t*)a.Gh + (size_t)ky * twoM * a.B * C * 2;
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
    const size_t e = (((size_t)kx * a.B + b) * C + o) * 2;
    Gh[e] = gr;
    Gh[e + 1] = gi;
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
// gradient blob (Re block, then Im block).  One block per mode (ky, a); per
// mode a [C x B] by [B x C] complex product on the matrix cores (16x16x4,
// accumulate precision) over the systems b, from the mode-major spectra
// V^ and G^ ([ky][a][b][c] complex):
//   Re = Vr^T Gr + Vi^T Gi,  Im = Vr^T Gi - Vi^T Gr.
// The four waves split the (c, o) tiles and, at C = 16, the systems; the
// split sums are added in a fixed order.
template <int PREC, int C>
__global__ __launch_bounds__(256) void k_dR(BSpecArgs a, double* grad_re, double* grad_im) {
  using M_ = Mf<PREC>;
  using acc_t = typename M_::acc_t;
  using accv_t = typename M_::accv_t;
  constexpr int NOB = C / 16, NT = NOB * NOB, NKS = 4 / NT, KB = 8;
  __shared__ acc_t red[4][2][256];
  const int ky = blockIdx.x, kx = blockIdx.y;
  const int M = a.M, twoM = 2 * M, B = a.B;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, n16 = lane & 15, g = lane >> 4;
  const int tile = w % NT, part = w / NT, cb = tile / NOB, ob = tile % NOB;
  const size_t mode = ((size_t)ky * twoM + kx) * B * C * 2;
  const acc_t* V = (const acc_t*)a.Vsave + mode + (size_t)(cb * 16 + n16) * 2;
  const acc_t* G = (const acc_t*)a.Gh + mode + (size_t)(ob * 16 + n16) * 2;
  // this wave's systems: [b0, b1) in K-steps of four (lane group g takes b + g)
  const int per = (B + NKS - 1) / NKS;
  const int b0 = part * per, b1 = min(B, b0 + per);
  accv_t re = accv_t{0, 0, 0, 0}, im = accv_t{0, 0, 0, 0};
  for (int bs = b0; bs < b1; bs += 4 * KB) {
    // loads of KB K-steps before their products; systems past b1 read b0
    // and are zeroed
    acc_t vr[KB], vi[KB], gr[KB], gi[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int b = bs + 4 * u + g;
      const size_t o = (size_t)(b < b1 ? b : b0) * C * 2;
      vr[u] = V[o];
      vi[u] = V[o + 1];
      gr[u] = G[o];
      gi[u] = G[o + 1];
    }
    // every load above is issued before the first product (the compiler
    // would otherwise wait for each step's loads in turn)
#pragma unroll
    for (int u = 0; u < KB; ++u) asm volatile("" : "+v"(vr[u]), "+v"(vi[u]), "+v"(gr[u]), "+v"(gi[u]));
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const bool ok = bs + 4 * u + g < b1;
      const acc_t xr = ok ? vr[u] : (acc_t)0, xi = ok ? vi[u] : (acc_t)0;
      re = M_::mma(xr, gr[u], re);
      re = M_::mma(xi, gi[u], re);
      im = M_::mma(xr, gi[u], im);
      im = M_::mma(-xi, gr[u], im);
    }
  }
  if constexpr (NKS > 1) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      red[w][0][i * 64 + lane] = re[i];
      red[w][1][i * 64 + lane] = im[i];
    }
    __syncthreads();
    if (part != 0) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc_t sr = 0, si = 0;
      for (int pp = 0; pp < NKS; ++pp) {
        sr += red[pp * NT + tile][0][i * 64 + lane];
        si += red[pp * NT + tile][1][i * 64 + lane];
      }
      re[i] = sr;
      im[i] = si;
    }
  }
  // item i of lane (o, g): c = 16 cb + row(g, i), o = 16 ob + n
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = cb * 16 + M_::row(g, i), o = ob * 16 + n16;
    const size_t idx = (((size_t)c * C + o) * twoM + kx) * M + ky;
    grad_re[idx] = (double)re[i];
    grad_im[idx] = (double)im[i];
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

template <int PREC, int C, int MP>
static void bwd_t(const BwdArgs& a, int nblk, hipStream_t s) {
  const int tl = a.mode == 0 ? a.L - 1 : a.l - 1;
  const dim3 gr(nblk), bl(256);
  if (a.mode == 0) {
    if (tl >= 1) hipLaunchKernelGGL((k_bwd<PREC, C, MP, 0, 0>), gr, bl, 0, s, a);
    else hipLaunchKernelGGL((k_bwd<PREC, C, MP, 0, 1>), gr, bl, 0, s, a);
  } else {
    if (tl >= 1) hipLaunchKernelGGL((k_bwd<PREC, C, MP, 1, 0>), gr, bl, 0, s, a);
    else if (tl == 0) hipLaunchKernelGGL((k_bwd<PREC, C, MP, 1, 1>), gr, bl, 0, s, a);
    else hipLaunchKernelGGL((k_bwd<PREC, C, MP, 1, 2>), gr, bl, 0, s, a);
  }
}

template <int PREC>
static void bwd_c(const BwdArgs& a, int C, int nblk, hipStream_t s) {
  if (C == 16 && a.MP == 16) bwd_t<PREC, 16, 16>(a, nblk, s);
  else if (C == 16) bwd_t<PREC, 16, 32>(a, nblk, s);
  else if (a.MP == 16) bwd_t<PREC, 32, 16>(a, nblk, s);
  else bwd_t<PREC, 32, 32>(a, nblk, s);
}

void launch_bwd(const BwdArgs& a, int prec, int C, int nblk, hipStream_t s) {
  ProfScope ps(PK_TRAIN_BWD, s);
  if (prec == P64) bwd_c<P64>(a, C, nblk, s);
  else bwd_c<P32>(a, C, nblk, s);
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
    if (C == 16) hipLaunchKernelGGL((k_dR<P64, 16>), g, dim3(256), 0, s, a, gre, gim);
    else hipLaunchKernelGGL((k_dR<P64, 32>), g, dim3(256), 0, s, a, gre, gim);
  } else {
    if (C == 16) hipLaunchKernelGGL((k_dR<P32, 16>), g, dim3(256), 0, s, a, gre, gim);
    else hipLaunchKernelGGL((k_dR<P32, 32>), g, dim3(256), 0, s, a, gre, gim);
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
