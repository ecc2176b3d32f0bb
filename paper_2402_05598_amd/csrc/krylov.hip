// Krylov part of flexible conjugate gradients (Algorithm 1), float64.
//
// Per iteration i and system b (after w_i = B(r_i) is available):
//   k_wdots   partial (w_i, s_k) over the window k = i-m_i .. i-1
//   k_dir     c_k = (w_i, s_k) / (p_k, s_k) (formed in every block),
//             p_i = w_i - sum_k c_k p_k (recomputed on a halo in LDS),
//             s_i = A p_i, partial (p_i, r_i), (p_i, s_i)
//   k_update  alpha_i = (p_i, r_i)/(p_i, s_i) or breakdown (every block),
//             u += alpha p_i, r -= alpha s_i, partial ||r_{i+1}||^2
//   k_fin(2)  ||r_{i+1}|| / ||r_0||, stopping test, i <- i+1
// Reductions are two-level and deterministic: every block writes its partial
// sums to a fixed slot, and either a one-block-per-system kernel or every
// block of the consuming kernel sums the slots in block order (the kernel
// boundary makes the slots visible, so no device-wide fences are needed).
// The block -> points mapping depends only on N, so a system gives the same
// bits alone and inside any batch.
#include <algorithm>

#include "common.h"
#include "prof.h"

namespace fcgno {

constexpr int PPT = FLAT_PTS / 256;   // points per thread in the flat kernels


// 5-point operator at interior point (i, j) with neighbour values supplied.
__device__ __forceinline__ double stencil_at(const double* __restrict__ k, int N, int i, int j,
                                             double c, double e, double wv, double nv, double sv) {
  const int K = N + 2;
  const double kc = k[(i + 1) * K + (j + 1)];
  const double kE = 0.5 * (kc + k[(i + 2) * K + (j + 1)]);
  const double kW = 0.5 * (kc + k[(i)*K + (j + 1)]);
  const double kN = 0.5 * (kc + k[(i + 1) * K + (j + 2)]);
  const double kS = 0.5 * (kc + k[(i + 1) * K + (j)]);
  const double h1 = (double)(N + 1);
  return ((kE + kW + kN + kS) * c - kE * e - kW * wv - kN * nv - kS * sv) * (h1 * h1);
}

__global__ __launch_bounds__(64) void k_init_state(const SysDev* sys, int nsys, int max_iter,
                                                   int m_max, double rtol) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= nsys) return;
  GLOBAL SysState* st = sys[b].st;
  st->i = 0;
  st->active = 1;
  SysDev* rec = (SysDev*)(sys + b);
  rec->active = 1;
  rec->it = 0;
  rec->mmax = m_max;
  st->status = S_NOTCONV;
  st->iters = 0;
  for (int q = 0; q < 4; ++q) st->tick[q] = 0u;
  st->m = 0;
  st->max_iter = max_iter;
  st->m_max = m_max;
  st->rr0 = 0.0;
  st->rr = 0.0;
  st->alpha = 0.0;
  st->snorm = 0.0;
  st->tres = 0.0;
  st->tresf = 0.0;
  st->ff = 0.0;
  st->rtol = rtol;
  for (int q = 0; q <= MAXW; ++q) st->ps_ring[q] = 0.0;
  for (int q = 0; q < MAXW; ++q) st->coef[q] = 0.0;
  if (b == 0) *sys[0].n_active = nsys;
}

// mode 0: r = f - A u, partial ||r_0||^2, ||f||^2 and input checks (k > 0
//         and finite, f and u finite).  mode 1: partial ||f - A u||^2 only,
//         every system.
__global__ __launch_bounds__(256) void k_residual(const SysDev* sys, int N, int mode) {
  __shared__ double lds[4];
  const SysDev sd = sys[blockIdx.y];
  if (mode == 0 && !sd.active) return;
  const int n = N * N;
  const int K = N + 2;
  double acc = 0.0, bad = 0.0, ff = 0.0;
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int p = blockIdx.x * FLAT_PTS + e * 256 + threadIdx.x;
    if (p < n) {
      const int i = p / N, j = p - i * N;
      const double c = sd.u[p];
      const double ue = (i + 1 < N) ? sd.u[p + N] : 0.0;
      const double uw = (i > 0) ? sd.u[p - N] : 0.0;
      const double un = (j + 1 < N) ? sd.u[p + 1] : 0.0;
      const double us = (j > 0) ? sd.u[p - 1] : 0.0;
      const double fv = sd.f[p];
      const double rv = fv - stencil_at(sd.k, N, i, j, c, ue, uw, un, us);
      if (mode == 0) {
        // every node except the four corners is read by some interior point
        const double kc = sd.k[(i + 1) * K + j + 1];
        bool ok = (kc > 0.0) && isfinite(kc) && isfinite(fv) && isfinite(c);
        if (i == 0) { double t = sd.k[j + 1]; ok = ok && t > 0.0 && isfinite(t); }
        if (i == N - 1) { double t = sd.k[(N + 1) * K + j + 1]; ok = ok && t > 0.0 && isfinite(t); }
        if (j == 0) { double t = sd.k[(i + 1) * K]; ok = ok && t > 0.0 && isfinite(t); }
        if (j == N - 1) { double t = sd.k[(i + 1) * K + N + 1]; ok = ok && t > 0.0 && isfinite(t); }
        if (!ok) bad += 1.0;
        sd.r[p] = rv;
        ff += fv * fv;
      }
      acc += rv * rv;
    }
  }
  acc = block_sum(acc, lds);
  if (mode == 0) {
    bad = block_sum(bad, lds);
    ff = block_sum(ff, lds);
  }
  if (threadIdx.x == 0) {
    sd.part[pslot(N, 0, blockIdx.x)] = acc;
    sd.part[pslot(N, 1, blockIdx.x)] = bad;
    sd.part[pslot(N, 2, blockIdx.x)] = ff;
  }
}

// partial ||r||^2 for a standalone operator application.
__global__ __launch_bounds__(256) void k_rnorm(const SysDev* sys, int N) {
  __shared__ double lds[4];
  const SysDev sd = sys[blockIdx.y];
  const int n = N * N;
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int p = blockIdx.x * FLAT_PTS + e * 256 + threadIdx.x;
    if (p < n) {
      const double v = sd.r[p];
      acc += v * v;
    }
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) sd.part[pslot(N, 0, blockIdx.x)] = acc;
}

// Loads in these kernels are unconditional, at clamped indices, with the
// values of out-of-range points masked afterwards: a load under a per-lane
// condition becomes a branch, and the compiler then waits for each such load
// before the next one instead of keeping them in flight together.

// Partial-slot slots of the two folded reductions: the direction kernel's
// (p_i, r_i), (p_i, s_i) and the update kernel's ||r_{i+1}||^2 go to slots
// that no kernel reading the previous kernel's slots overwrites.
constexpr int SL_PR = MAXW, SL_PS = MAXW + 1, SL_RR = MAXW + 2;

// Sum of slot q over nb partial blocks in a fixed order (the same in every
// block that forms it, so every block holds the same bits); all threads
// return the sum.
__device__ __forceinline__ double slot_sum(const GLOBAL double* part, int N, int nb, int q, double* lds) {
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) v += part[pslot(N, q, b)];
  return block_sum(v, lds);
}

// slot_sum of the nq <= QN consecutive slots q0 .. q0 + nq - 1 at once: the
// same per-thread partials, wave sums and four-wave combine (the same bits),
// with every slot's loads in flight together (one memory round trip instead
// of nq).  out[q] is valid in every thread; lds holds >= 4 QN values.
template <int QN>
__device__ __forceinline__ void slot_sums(const GLOBAL double* part, int N, int nb, int q0, int nq, double (&out)[QN],
                                          double* lds) {
  double v[QN];
#pragma unroll
  for (int q = 0; q < QN; ++q) v[q] = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    double t[QN];
    // slots past nq read the last one (unconditional loads) and are not added
#pragma unroll
    for (int q = 0; q < QN; ++q) t[q] = part[pslot(N, q0 + min(q, nq - 1), b)];
#pragma unroll
    for (int q = 0; q < QN; ++q)
      if (q < nq) v[q] += t[q];
  }
#pragma unroll
  for (int q = 0; q < QN; ++q) v[q] = wave_sum(v[q]);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < QN; ++q) lds[4 * q + w] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < QN; ++q) out[q] = (lds[4 * q] + lds[4 * q + 1]) + (lds[4 * q + 2] + lds[4 * q + 3]);
}

// Window sums over NV (a compile-time count) window vectors for this
// thread's points.
template <int NV>
__device__ __forceinline__ void wdots_pass(const double* __restrict__ S, size_t n, int slot0, int ring,
                                           const int (&pc)[PPT], const bool (&ok)[PPT], const double (&wv)[PPT],
                                           double (&acc)[8]) {
  double sv[NV][PPT];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double* __restrict__ Sv = S + (size_t)((slot0 + q) % ring) * n;
#pragma unroll
    for (int e = 0; e < PPT; ++e) sv[q][e] = Sv[pc[e]];
  }
#pragma unroll
  for (int q = 0; q < NV; ++q)
#pragma unroll
    for (int e = 0; e < PPT; ++e)
      if (ok[e]) acc[q] += wv[e] * sv[q][e];
}

// Window dot products (w_i, s_k), in passes of up to 8 window vectors.
__global__ __launch_bounds__(256) void k_wdots(const SysDev* sys, int N) {
  const SysDev sd = sys[blockIdx.y];
  if (!sd.active) return;
  const int i = sd.it, mm = sd.mmax;
  const int m = window_size(i, mm);
  if (m == 0) return;
  const int n = N * N;
  const int ring = mm + 1;
  const double* __restrict__ w = sd.w;
  int pc[PPT];
  bool ok[PPT];
  double wv[PPT];
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int p = blockIdx.x * FLAT_PTS + e * 256 + threadIdx.x;
    ok[e] = p < n;
    pc[e] = ok[e] ? p : n - 1;
  }
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const double t = w[pc[e]];
    wv[e] = ok[e] ? t : 0.0;
  }
  __shared__ double red[8][4];
  for (int q0 = 0; q0 < m; q0 += 8) {
    const int nq = min(8, m - q0);
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    const int slot0 = i - m + q0;
    switch (nq) {
      case 1: wdots_pass<1>(sd.S, n, slot0, ring, pc, ok, wv, acc); break;
      case 2: wdots_pass<2>(sd.S, n, slot0, ring, pc, ok, wv, acc); break;
      case 3: wdots_pass<3>(sd.S, n, slot0, ring, pc, ok, wv, acc); break;
      case 4: wdots_pass<4>(sd.S, n, slot0, ring, pc, ok, wv, acc); break;
      case 5: wdots_pass<5>(sd.S, n, slot0, ring, pc, ok, wv, acc); break;
      case 6: wdots_pass<6>(sd.S, n, slot0, ring, pc, ok, wv, acc); break;
      case 7: wdots_pass<7>(sd.S, n, slot0, ring, pc, ok, wv, acc); break;
      default: wdots_pass<8>(sd.S, n, slot0, ring, pc, ok, wv, acc); break;
    }
    // all window sums through LDS at once: wave sums, then lane q of the
    // first wave adds the four waves' values in a fixed order
    const int wv_ = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q < nq) {
        const double v = wave_sum(acc[q]);
        if ((threadIdx.x & 63) == 0) red[q][wv_] = v;
      }
    }
    __syncthreads();
    if (threadIdx.x < nq) {
      const int q = threadIdx.x;
      sd.part[pslot(N, q0 + q, blockIdx.x)] = (red[q][0] + red[q][1]) + (red[q][2] + red[q][3]);
    }
    __syncthreads();
  }
}

constexpr int DIR_HW = TILE_J + 2, DIR_HN = (TILE_I + 2) * (TILE_J + 2);
constexpr int DIR_HR = (DIR_HN + 255) / 256;   // halo slots per thread

// p -= sum_q c_q P_q on this thread's halo slots, NV window vectors at once
// (their loads in flight together).
constexpr int DIR_PV = 4;   // window vectors per pass (more would cost occupancy)
template <int NV>
__device__ __forceinline__ void dir_pass(const double* __restrict__ P, size_t n, int slot0, int ring,
                                         const double* cf, const int (&hc)[DIR_HR], const bool (&hok)[DIR_HR],
                                         double (&hv)[DIR_HR]) {
  double pv[NV][DIR_HR];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double* __restrict__ Pq = P + (size_t)((slot0 + q) % ring) * n;
#pragma unroll
    for (int e = 0; e < DIR_HR; ++e) pv[q][e] = Pq[hc[e]];
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double c = cf[q];
#pragma unroll
    for (int e = 0; e < DIR_HR; ++e)
      if (hok[e]) hv[e] -= c * pv[q][e];
  }
}

// Window coefficients c_k = (w_i, s_k)/(p_k, s_k) from the window-sum
// partials, then p_i on the tile and a one-point halo, s_i = A p_i, partial
// (p_i, r_i), (p_i, s_i).  Every block forms the coefficients itself (the same
// fixed-order sums) instead of a one-block pass between the two kernels.
// wslots: partial slots of the window sums (the window-sum kernel's blocks,
// or the projection layer's row segments when it formed them).
__global__ __launch_bounds__(256) void k_dir(const SysDev* sys, int N, int wslots) {
  constexpr int HW = DIR_HW, HN = DIR_HN, HR = DIR_HR;
  __shared__ double pl[HN];
  __shared__ double cf[MAXW];
  __shared__ double lds[4 * 8];
  const SysDev sd = sys[blockIdx.y];
  GLOBAL SysState* st = sd.st;
  if (!sd.active) return;
  const int i = sd.it, mm = sd.mmax, ring = mm + 1;
  const int m = window_size(i, mm);
  const int n = N * N;
  const int tj = (N + TILE_J - 1) / TILE_J;
  const int bi = blockIdx.x / tj, bj = blockIdx.x - bi * tj;
  const int i0 = bi * TILE_I, j0 = bj * TILE_J;
  int hc[HR];
  bool hok[HR];
  double hv[HR];
#pragma unroll
  for (int e = 0; e < HR; ++e) {
    const int t = threadIdx.x + 256 * e;
    const int a = t / HW, c = t - a * HW;
    const int gi = i0 - 1 + a, gj = j0 - 1 + c;
    hok[e] = t < HN && gi >= 0 && gi < N && gj >= 0 && gj < N;
    hc[e] = hok[e] ? gi * N + gj : 0;
  }
#pragma unroll
  for (int e = 0; e < HR; ++e) {
    const double t = sd.w[hc[e]];
    hv[e] = hok[e] ? t : 0.0;
  }
  // the residual at the interior points and (p_k, s_k) of the window, loaded
  // before the coefficient sums so that their latencies overlap
  constexpr int IR = TILE_I * TILE_J / 256;
  bool ok[IR];
  int gic[IR], gjc[IR];
  double rv[IR];
#pragma unroll
  for (int e = 0; e < IR; ++e) {
    const int t = threadIdx.x + 256 * e;
    const int a = t / TILE_J, c = t - a * TILE_J;
    ok[e] = i0 + a < N && j0 + c < N;
    gic[e] = ok[e] ? i0 + a : 0;
    gjc[e] = ok[e] ? j0 + c : 0;
    rv[e] = sd.r[gic[e] * N + gjc[e]];
  }
  const double psq = (int)threadIdx.x < m ? st->ps_ring[(i - m + (int)threadIdx.x) % ring] : 1.0;
  // coefficients (thread q forms c_q), then passes of at most DIR_PV window vectors
  const int nbw = wslots;
  for (int q0 = 0; q0 < m; q0 += 8) {
    double d[8];
    slot_sums<8>(sd.part, N, nbw, q0, min(8, m - q0), d, lds);
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if ((int)threadIdx.x == q0 + q && q0 + q < m) cf[q0 + q] = d[q] / psq;
    __syncthreads();   // lds is reused by the next group
  }
  if (blockIdx.x == 0 && threadIdx.x < m) st->coef[threadIdx.x] = cf[threadIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) st->m = m;
  for (int q0 = 0; q0 < m; q0 += DIR_PV) {
    const int nq = min(DIR_PV, m - q0);
    const int slot0 = i - m + q0;
    switch (nq) {
      case 1: dir_pass<1>(sd.P, n, slot0, ring, cf + q0, hc, hok, hv); break;
      case 2: dir_pass<2>(sd.P, n, slot0, ring, cf + q0, hc, hok, hv); break;
      case 3: dir_pass<3>(sd.P, n, slot0, ring, cf + q0, hc, hok, hv); break;
      default: dir_pass<4>(sd.P, n, slot0, ring, cf + q0, hc, hok, hv); break;
    }
  }
#pragma unroll
  for (int e = 0; e < HR; ++e) {
    const int t = threadIdx.x + 256 * e;
    if (t < HN) pl[t] = hv[e];
  }
  __syncthreads();
  double* __restrict__ Pi = sd.P + (size_t)(i % ring) * n;
  double* __restrict__ Si = sd.S + (size_t)(i % ring) * n;
  // interior points: the stencil, the stores and the two sums
  double pr = 0.0, ps = 0.0;
#pragma unroll
  for (int e = 0; e < IR; ++e) {
    const int t = threadIdx.x + 256 * e;
    const int a = t / TILE_J, c = t - a * TILE_J;
    const int h = (a + 1) * HW + (c + 1);
    const double pc = pl[h];
    const double s = stencil_at(sd.k, N, gic[e], gjc[e], pc, pl[h + HW], pl[h - HW], pl[h + 1], pl[h - 1]);
    if (ok[e]) {
      const int p = gic[e] * N + gjc[e];
      Pi[p] = pc;
      Si[p] = s;
      pr += pc * rv[e];
      ps += pc * s;
    }
  }
  // both sums through LDS at once (wave sums, then a fixed-order add)
  __shared__ double red[2][4];
  pr = wave_sum(pr);
  ps = wave_sum(ps);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = pr;
    red[1][threadIdx.x >> 6] = ps;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int q = threadIdx.x;
    sd.part[pslot(N, q == 0 ? SL_PR : SL_PS, blockIdx.x)] = (red[q][0] + red[q][1]) + (red[q][2] + red[q][3]);
  }
}

// u += alpha p_i, r -= alpha s_i, partial ||r_{i+1}||^2.  Two points per
// thread: measured the fastest streaming shape for four reads and two writes
// per point (more blocks in flight beat more loads per thread here).
//
// The step length alpha_i = (p_i, r_i)/(p_i, s_i) (or the breakdown test) is
// formed in every block from the direction kernel's partials, the same fixed-
// order sums, after this block's vector loads are in flight; block 0 records
// it.  On breakdown no block updates and block 0 stops the system.
__global__ __launch_bounds__(256) void k_update(const SysDev* sys, int N) {
  constexpr int UPT = UPD_PTS / 256;
  __shared__ double lds[4], lds8[8];
  const SysDev sd = sys[blockIdx.y];
  GLOBAL SysState* st = sd.st;
  if (!sd.active) return;
  const int i = sd.it, ring = sd.mmax + 1;
  const int n = N * N;
  const double* __restrict__ Pi = sd.P + (size_t)(i % ring) * n;
  const double* __restrict__ Si = sd.S + (size_t)(i % ring) * n;
  double* __restrict__ u = sd.u;
  double* __restrict__ r = sd.r;
  double uv[UPT], pv[UPT], rv[UPT], sv[UPT];
#pragma unroll
  for (int e = 0; e < UPT; ++e) {
    const int p = blockIdx.x * UPD_PTS + e * 256 + threadIdx.x;
    if (p < n) {
      uv[e] = u[p];
      pv[e] = Pi[p];
      rv[e] = r[p];
      sv[e] = Si[p];
    }
  }
  const int nbd = tile_blocks(N);
  double prs[2];
  slot_sums<2>(sd.part, N, nbd, SL_PR, 2, prs, lds8);
  const double PR = prs[0], PS = prs[1];
  if (!(isfinite(PS) && isfinite(PR)) || !(PS > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->alpha = 0.0;
      deactivate(st, sd.n_active, S_BREAK, i, sys + blockIdx.y);
    }
    return;
  }
  const double alpha = PR / PS;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->alpha = alpha;
    st->ps_ring[i % ring] = PS;
  }
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < UPT; ++e) {
    const int p = blockIdx.x * UPD_PTS + e * 256 + threadIdx.x;
    if (p < n) {
      const double rn = rv[e] - alpha * sv[e];
      u[p] = uv[e] + alpha * pv[e];
      r[p] = rn;
      acc += rn * rn;
    }
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) sd.part[pslot(N, SL_RR, blockIdx.x)] = acc;
}

// One block per system: fixed-order sums of the partial slots and the scalar
// steps of Algorithm 1 that follow them.
//   mode 2: rho_{i+1}, stopping test, i+1  (after k_update)
// (the window coefficients and the step length are formed inside k_dir and
// k_update)
//   mode 3: ||r_0||, input status          (after k_residual mode 0)
//   mode 4: true relative residual         (after k_residual mode 1)
//   mode 5: operator input scale           (after k_rnorm)
__global__ __launch_bounds__(256) void k_fin(const SysDev* sys, int N, int mode) {
  __shared__ double lds[4];
  const SysDev sd = sys[blockIdx.x];
  GLOBAL SysState* st = sd.st;
  if (mode != 4 && mode != 5 && !sd.active) return;
  const int nb = mode == 2 ? upd_blocks(N * N) : flat_blocks(N * N);
  auto fsum = [&](int q) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) v += sd.part[pslot(N, q, b)];
    return block_sum(v, lds);
  };
  const int i = st->i, ring = st->m_max + 1;
  (void)ring;
  if (mode == 2) {
    const double rr = fsum(SL_RR);
    if (threadIdx.x == 0) {
      const double rho = sqrt(rr / st->rr0);
      st->rr = rr;
      st->snorm = sqrt(rr) / (double)N;
      sd.hist[i + 1] = rho;
      st->i = i + 1;
      ((SysDev*)(sys + blockIdx.x))->it = i + 1;
      st->iters = i + 1;
      if (!isfinite(rho)) deactivate(st, sd.n_active, S_BREAK, i + 1, sys + blockIdx.x);
      else if (rho <= st->rtol) deactivate(st, sd.n_active, S_OK, i + 1, sys + blockIdx.x);
      else if (i + 1 >= st->max_iter) deactivate(st, sd.n_active, S_NOTCONV, i + 1, sys + blockIdx.x);
    }
  } else if (mode == 3) {
    const double rr = fsum(0), nbad = fsum(1), ff = fsum(2);
    if (threadIdx.x == 0) {
      st->rr0 = rr;
      st->ff = ff;
      st->rr = rr;
      st->snorm = sqrt(rr) / (double)N;
      if (nbad > 0.0 || !isfinite(rr)) {
        sd.hist[0] = __longlong_as_double(0x7ff8000000000000ll);
        deactivate(st, sd.n_active, S_NONFINITE, 0, sys + blockIdx.x);
      } else {
        sd.hist[0] = 1.0;
        if (rr == 0.0) deactivate(st, sd.n_active, S_OK, 0, sys + blockIdx.x);
      }
    }
  } else if (mode == 4) {
    const double rr = fsum(0);
    if (threadIdx.x == 0) {
      st->tres = st->rr0 > 0.0 ? sqrt(rr / st->rr0) : 0.0;
      // f = 0: zero when u solves A u = 0 exactly, else not defined (+inf)
      st->tresf = st->ff > 0.0 ? sqrt(rr / st->ff) : (rr > 0.0 ? __longlong_as_double(0x7ff0000000000000ll) : 0.0);
    }
  } else {
    const double rr = fsum(0);
    if (threadIdx.x == 0) {
      st->snorm = sqrt(rr) / (double)N;
      st->active = 1;
      ((SysDev*)(sys + blockIdx.x))->active = 1;
    }
  }
}

// Record r_{i+1} and u* - u_{i+1} of every system after iteration it.
__global__ __launch_bounds__(256) void k_record(const SysDev* sys, int N, int it, int m, double* rec_r,
                                                double* rec_e, const double* ustar) {
  const SysDev sd = sys[blockIdx.y];
  const size_t n = (size_t)N * N;
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const size_t o = ((size_t)blockIdx.y * m + it) * n + p;
  rec_r[o] = sd.r[p];
  rec_e[o] = ustar[(size_t)blockIdx.y * n + p] - sd.u[p];
}

// ---- classical preconditioners (the comparison of Table 1) ----------------

// sum of the off-diagonal couplings of point (i, j) times x, and the
// diagonal of A there (zero Dirichlet values outside)
__device__ __forceinline__ void offsum_diag(const GLOBAL double* __restrict__ k, const GLOBAL double* __restrict__ x,
                                            int N, int i, int j, bool use_x, double& off, double& diag) {
  const int K = N + 2;
  const double kc = k[(i + 1) * K + (j + 1)];
  const double kE = 0.5 * (kc + k[(i + 2) * K + (j + 1)]);
  const double kW = 0.5 * (kc + k[(i)*K + (j + 1)]);
  const double kN = 0.5 * (kc + k[(i + 1) * K + (j + 2)]);
  const double kS = 0.5 * (kc + k[(i + 1) * K + (j)]);
  const double h1 = (double)(N + 1);
  diag = (kE + kW + kN + kS) * (h1 * h1);
  off = 0.0;
  if (use_x) {
    const int p = i * N + j;
    const double e = (i + 1 < N) ? x[p + N] : 0.0;
    const double wv = (i > 0) ? x[p - N] : 0.0;
    const double n = (j + 1 < N) ? x[p + 1] : 0.0;
    const double sv = (j > 0) ? x[p - 1] : 0.0;
    off = (kE * e + kW * wv + kN * n + kS * sv) * (h1 * h1);
  }
}

// One Jacobi sweep x_out = x_in + D^-1 (r - A x_in) = D^-1 (r + offsum(x_in));
// first: x_in = 0.  to_w: write w (else the second iterate tmp).
__global__ __launch_bounds__(256) void k_jacobi(const SysDev* sys, int N, int to_w, int first) {
  const SysDev sd = sys[blockIdx.y];
  if (!sd.active) return;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= N * N) return;
  const int i = p / N, j = p - i * N;
  const GLOBAL double* xin = to_w ? sd.tmp : sd.w;
  GLOBAL double* xout = to_w ? sd.w : sd.tmp;
  double off, diag;
  offsum_diag(sd.k, xin, N, i, j, !first, off, diag);
  xout[p] = (sd.r[p] + off) / diag;
}

// Half sweep of red-black Gauss-Seidel in place on w: the points of one
// colour ((i + j) & 1 == color) get D^-1 (r + offsum(w)), their neighbours
// being of the other colour; first: the other colour is x_0 = 0.  One thread
// per point of the colour: row i, pair q covers columns 2q and 2q + 1.
__global__ __launch_bounds__(256) void k_rbgs(const SysDev* sys, int N, int color, int first) {
  const SysDev sd = sys[blockIdx.y];
  if (!sd.active) return;
  const int H = (N + 1) >> 1;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= N * H) return;
  const int i = t / H;
  const int j = 2 * (t - i * H) + ((i + color) & 1);
  if (j >= N) return;
  const int p = i * N + j;
  double off, diag;
  offsum_diag(sd.k, sd.w, N, i, j, !first, off, diag);
  sd.w[p] = (sd.r[p] + off) / diag;
}

// Zero bytes [0, nbytes) of a buffer (16-byte body, byte tail).  A kernel
// rather than a memset so that work a caller captures into a graph holds
// no memset node.
__global__ __launch_bounds__(256) void k_zero(char* p, size_t nbytes) {
  const size_t n16 = nbytes >> 4;
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n16; q += stride) ((uint4*)p)[q] = uint4{0, 0, 0, 0};
  const size_t t = (n16 << 4) + (size_t)blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x == 0 && t < nbytes) p[t] = 0;
}

// Order-preserving compaction of a launch table: the records of the systems
// still iterating first (their copies of the state refreshed from it), then,
// up to nsys slots, records whose state is never active (the first record
// pointing at an idle state).  Kernels find their system by block index and
// leave at once when it has stopped, so launches sized to the active count
// skip the stopped systems' blocks; a system's arithmetic does not depend on
// its slot.  (Pointer parameters stay in the generic address space: the
// host registers a kernel under the name its own signature mangles to.)
__global__ __launch_bounds__(256) void k_compact(const SysDev* sys, int nsys, SysDev* out, SysState* idle_state) {
  constexpr int WORDS = sizeof(SysDev) / 8;
  static_assert(sizeof(SysDev) % 8 == 0, "records copy as 8-byte words");
  GLOBAL SysState* idle = (GLOBAL SysState*)idle_state;
  __shared__ int off[257];
  const int t = threadIdx.x;
  const int per = (nsys + 255) / 256;
  const int b0 = min(nsys, t * per), b1 = min(nsys, b0 + per);
  int c = 0;
  for (int b = b0; b < b1; ++b) c += sys[b].st->active ? 1 : 0;
  off[t + 1] = c;
  __syncthreads();
  if (t == 0) {
    off[0] = 0;
    for (int q = 1; q <= 256; ++q) off[q] += off[q - 1];
  }
  __syncthreads();
  int j = off[t];
  for (int b = b0; b < b1; ++b) {
    const GLOBAL SysState* st = sys[b].st;
    if (!st->active) continue;
    const unsigned long long* src = (const unsigned long long*)(sys + b);
    unsigned long long* dst = (unsigned long long*)(out + j);
    for (int w = 0; w < WORDS; ++w) dst[w] = src[w];
    out[j].active = 1;
    out[j].it = st->i;
    out[j].mmax = st->m_max;
    ++j;
  }
  for (int q = off[256] + t; q < nsys; q += 256) {
    const unsigned long long* src = (const unsigned long long*)sys;
    unsigned long long* dst = (unsigned long long*)(out + q);
    for (int w = 0; w < WORDS; ++w) dst[w] = src[w];
    out[q].st = idle;
    out[q].active = 0;
  }
}

// Refresh the launch table's copies of the state (after the host uploaded
// the table: the host does not know which systems stopped at set-up).
__global__ __launch_bounds__(64) void k_sync_records(const SysDev* sys, int nsys) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= nsys) return;
  const GLOBAL SysState* st = sys[b].st;
  SysDev* rec = (SysDev*)(sys + b);
  rec->active = st->active;
  rec->it = st->i;
  rec->mmax = st->m_max;
}

// Per-system summary for the host: {active, status, iters} and the true residual.
__global__ __launch_bounds__(64) void k_export(const SysDev* sys, int nsys, int* flags, double* tres) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= nsys) return;
  const GLOBAL SysState* st = sys[b].st;
  flags[3 * b] = st->active;
  flags[3 * b + 1] = st->status;
  flags[3 * b + 2] = st->iters;
  tres[2 * b] = st->tres;
  tres[2 * b + 1] = st->tresf;
}

// ---- launchers ------------------------------------------------------------

void launch_jacobi(const KrylovLaunch& L, int steps) {
  const dim3 g((L.N * L.N + 255) / 256, L.nsys);
  // steps alternate between w and tmp so that the last one lands in w
  for (int s = 1; s <= steps; ++s)
    hipLaunchKernelGGL(k_jacobi, g, dim3(256), 0, L.stream, L.sys, L.N, ((steps - s) % 2) == 0 ? 1 : 0,
                       s == 1 ? 1 : 0);
}

void launch_rbsgs(const KrylovLaunch& L, int steps) {
  const int H = (L.N + 1) >> 1;
  const dim3 g((L.N * H + 255) / 256, L.nsys);
  // A symmetric step sweeps red, black, black, red.  Points of one colour
  // couple only to the other, so the repeated black sweep and the next step's
  // first red sweep recompute identical values: k steps are the 2k + 1
  // alternating half sweeps red, black, ..., red.
  for (int h = 0; h < 2 * steps + 1; ++h)
    hipLaunchKernelGGL(k_rbgs, g, dim3(256), 0, L.stream, L.sys, L.N, h & 1, h == 0 ? 1 : 0);
}

void launch_zero(void* p, size_t nbytes, hipStream_t s) {
  if (nbytes == 0) return;
  const size_t n16 = (nbytes >> 4) + 1;
  const unsigned nb = (unsigned)std::min<size_t>((n16 + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero, dim3(nb), dim3(256), 0, s, (char*)p, nbytes);
}

void launch_compact(const SysDev* sys, int nsys, SysDev* out, SysState* idle, hipStream_t s) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(256), 0, s, sys, nsys, out, idle);
}

void launch_sync_records(const SysDev* sys, int nsys, hipStream_t s) {
  hipLaunchKernelGGL(k_sync_records, dim3((nsys + 63) / 64), dim3(64), 0, s, sys, nsys);
}

void launch_export(const SysDev* sys, int nsys, int* flags, double* tres, hipStream_t s) {
  hipLaunchKernelGGL(k_export, dim3((nsys + 63) / 64), dim3(64), 0, s, sys, nsys, flags, tres);
}

void launch_record(const KrylovLaunch& L, int it, int m, double* rec_r, double* rec_e, const double* ustar) {
  const size_t n = (size_t)L.N * L.N;
  hipLaunchKernelGGL(k_record, dim3((unsigned)((n + 255) / 256), L.nsys), dim3(256), 0, L.stream, L.sys, L.N, it, m,
                     rec_r, rec_e, ustar);
}

static inline int flat_nb(int N) { return (N * N + FLAT_PTS - 1) / FLAT_PTS; }

static void fin(const KrylovLaunch& L, int mode) {
  hipLaunchKernelGGL(k_fin, dim3(L.nsys), dim3(256), 0, L.stream, L.sys, L.N, mode);
}

void launch_init_state(const KrylovLaunch& L, int max_iter, double rtol) {
  hipLaunchKernelGGL(k_init_state, dim3((L.nsys + 63) / 64), dim3(64), 0, L.stream, L.sys, L.nsys,
                     max_iter, L.m_max, rtol);
}
void launch_residual(const KrylovLaunch& L, int mode) {
  hipLaunchKernelGGL(k_residual, dim3(flat_nb(L.N), L.nsys), dim3(256), 0, L.stream, L.sys, L.N, mode);
  fin(L, mode == 0 ? 3 : 4);
}
void launch_rnorm(const KrylovLaunch& L) {
  hipLaunchKernelGGL(k_rnorm, dim3(flat_nb(L.N), L.nsys), dim3(256), 0, L.stream, L.sys, L.N);
  fin(L, 5);
}
void launch_wdots(const KrylovLaunch& L) {
  {
    ProfScope ps(PK_WDOTS, L.stream);
    hipLaunchKernelGGL(k_wdots, dim3(flat_nb(L.N), L.nsys), dim3(256), 0, L.stream, L.sys, L.N);
  }
}
void launch_dir(const KrylovLaunch& L) {
  const int nb = ((L.N + TILE_I - 1) / TILE_I) * ((L.N + TILE_J - 1) / TILE_J);
  {
    ProfScope ps(PK_DIR, L.stream);
    hipLaunchKernelGGL(k_dir, dim3(nb, L.nsys), dim3(256), 0, L.stream, L.sys, L.N,
                       L.wslots > 0 ? L.wslots : (L.N * L.N + FLAT_PTS - 1) / FLAT_PTS);
  }
}
void launch_update(const KrylovLaunch& L) {
  {
    ProfScope ps(PK_UPDATE, L.stream);
    hipLaunchKernelGGL(k_update, dim3((L.N * L.N + UPD_PTS - 1) / UPD_PTS, L.nsys), dim3(256), 0, L.stream, L.sys,
                       L.N);
  }
  fin(L, 2);
}

}  // namespace fcgno
