// Forward pass of the Fourier neural-operator preconditioner B(r; theta)
// (Sec. 2.4.2: layers u <- S L A u with the FFT as analysis and synthesis,
// here a truncated DFT done as twiddle products).
//
// Shapes: N x N grid, C channels, M modes, kept kx in {0..M-1} U {N-M..N-1}
// (index a < 2M), ky in {0..M-1}; MP = 2M rounded up to 16; NP = N rounded up
// to 16.
//
// Per layer l the work splits in two launches:
//   k_spectral (grid M x systems, VALU): for one ky, the x-direction forward
//     DFT of the row partials G[x][c] -> V^[c][a], the per-mode complex
//     mixing W^[o][a] = sum_c V^[c][a] R[c][o][a][ky], and the x-direction
//     inverse DFT H[x][o] = sum_a W^[o][a] e^{+2 pi i kx x/N}, written as the
//     rows Hc[x][o][2ky], Hc[x][o][2ky+1] that the layer kernel consumes.
//   k_layer (one wave per row segment, matrix cores): for 16 points of a row
//     at a time, z = [T(y) | v(y)] . [Hc(x) ; W^T] + b (the y-direction
//     inverse DFT and the 1x1 bypass in one product), v' = GELU(z), then
//     either store v' and accumulate the y-direction forward DFT of v'
//     (T^T . v', the next layer's row partials), or project to w.
// Layer 0 never materialises the lifted field: its bypass uses the composed
// weights W_0 W_L on the four features, and its spectrum is
// (W_L[:,0]/s) DFT(r) + (a per-solve constant from log k, x1, x2, 1).
#include <algorithm>

#include <type_traits>

#include <hip/hip_ext.h>

#include "common.h"
#include "mfma.h"
#include "prof.h"

namespace fcgno {

__host__ __device__ inline int round16(int v) { return (v + 15) & ~15; }

// CB contiguous elements of type T as one vector access.
template <typename T, int CB>
struct Vec {
  typedef T type __attribute__((ext_vector_type(CB)));
};

// ---------------------------------------------------------------------------
// Tables.  Fourier: E64/Eacc[m] = (cos, sin)(2 pi m / N); T[y][2q], T[y][2q+1]
// = cos, sin of 2 pi q y / N for q < M.  Sine: E64/Eacc[m] = (sin(pi m/(N+1)),
// 0) for m < 2N + 2; T[y][2q] = sin(pi (q+1)(y+1)/(N+1)), T[y][2q+1] = 0.
// Zero elsewhere (and for y >= N); TT = T^T.  BF16 stores both in the layer
// kernel's fragment order (below).
// ---------------------------------------------------------------------------
template <int PREC>
__global__ void k_tables(int N, int M, int basis, double* E64, void* Eacc, void* T, void* TT) {
  using M_ = Mf<PREC>;
  using in_t = typename M_::in_t;
  using acc_t = typename M_::acc_t;
  const int MP = round16(2 * M), NP = round16(N);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tw_period(basis, N)) {
    double s, c;
    if (basis == B_SINE) {
      sincospi((double)t / (double)(N + 1), &c, &s);   // c = sin(pi t/(N+1)) in the cosine slot
      s = 0.0;
    } else {
      sincospi(2.0 * (double)t / (double)N, &s, &c);
    }
    E64[2 * t] = c;
    E64[2 * t + 1] = s;
    ((acc_t*)Eacc)[2 * t] = (acc_t)c;
    ((acc_t*)Eacc)[2 * t + 1] = (acc_t)s;
  }
  if (t < NP * MP) {
    const int y = t / MP, k = t - y * MP;
    double v = 0.0;
    if (y < N && k < 2 * M) {
      const int q = k >> 1;
      double s, c;
      if (basis == B_SINE) {
        const int m = (int)(((long long)(q + 1) * (y + 1)) % (2 * N + 2));
        sincospi((double)m / (double)(N + 1), &s, &c);
        v = (k & 1) ? 0.0 : s;
      } else {
        const int m = (int)(((long long)q * y) % N);
        sincospi(2.0 * (double)m / (double)N, &s, &c);
        v = (k & 1) ? s : c;
      }
    }
    if constexpr (PREC == PBF) {
      // Fragment order of the layer kernel's two products, so that a wave
      // reads each 16-point tile's operands as one contiguous block: lane
      // (n, g) = 16 g + n of tile y / 16 holds, for GEMM1 fragment ks,
      // T[16 tile + n][16 ks + 4 g + e] at T[((tile * 64 + lane) * KT + ks) * 4 + e]
      // and, for GEMM2 fragment jb, T[16 tile + 4 g + e][16 jb + n] at
      // TT[((tile * 64 + lane) * KT + jb) * 4 + e]  (KT = MP / 16).
      const int KT = MP >> 4, tile = y >> 4, yr = y & 15, kb = k >> 4, kr = k & 15;
      const int l1 = 16 * (kr >> 2) + yr, l2 = 16 * (yr >> 2) + kr;
      ((in_t*)T)[((tile * 64 + l1) * KT + kb) * 4 + (kr & 3)] = M_::cvt((acc_t)v);
      ((in_t*)TT)[((tile * 64 + l2) * KT + kb) * 4 + (yr & 3)] = M_::cvt((acc_t)v);
    } else {
      ((in_t*)T)[y * MP + k] = M_::cvt((acc_t)v);
      ((in_t*)TT)[k * NP + y] = M_::cvt((acc_t)v);
    }
  }
}

// log k at the interior nodes in op precision.
template <int PREC>
__global__ void k_logk(const SysDev* sys, int N) {
  using M_ = Mf<PREC>;
  using in_t = typename M_::in_t;
  using acc_t = typename M_::acc_t;
  const SysDev sd = sys[blockIdx.y];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N * N) return;
  const int i = p / N, j = p - i * N;
  ((in_t*)sd.logk)[p] = M_::cvt((acc_t)log(sd.k[(i + 1) * (N + 2) + j + 1]));
}

// y-direction DFT of one row of a per-solve feature, float64 (set-up only):
// out[j] = sum_y field(y) T(y, j) for j < 2M, one wave per row.  FIELD 1..4:
// log k, x1, x2, 1.
template <int FIELD>
__device__ __forceinline__ double row_field(const SysDev& sd, int N, int x, int y) {
  if (FIELD == 1) return log(sd.k[(x + 1) * (N + 2) + y + 1]);
  if (FIELD == 2) return (double)(x + 1) / (double)(N + 1);
  if (FIELD == 3) return (double)(y + 1) / (double)(N + 1);
  return 1.0;
}

template <int FIELD>
__global__ __launch_bounds__(256) void k_rowdft(const SysDev* sys, int N, int M, int basis, const double* E64,
                                               double* out_base, size_t out_sys_stride) {
  const SysDev sd = sys[blockIdx.y];
  const int x = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (x >= N) return;
  const int lane = threadIdx.x & 63;
  const int MP = round16(2 * M);
  double acc[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) acc[q] = 0.0;
  if (basis == B_SINE) {
    // sin(pi (q+1)(y+1)/(N+1)), q = 0..15, by the same rotation recurrence
    // started at the first harmonic; the odd (imaginary) columns stay zero
    for (int y = lane; y < N; y += 64) {
      const double v = row_field<FIELD>(sd, N, x, y);
      double s1, c1;
      sincospi((double)(y + 1) / (double)(N + 1), &s1, &c1);
      double c = c1, sn = s1;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        acc[2 * q] += v * sn;
        const double cn = c * c1 - sn * s1;
        sn = sn * c1 + c * s1;
        c = cn;
      }
    }
  } else {
    // harmonics q = 0..15 of e^{2 pi i y / N} by complex-multiplication recurrence
    for (int y = lane; y < N; y += 64) {
      const double v = row_field<FIELD>(sd, N, x, y);
      const double c1 = E64[2 * y], s1 = E64[2 * y + 1];
      double c = 1.0, sn = 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        acc[2 * q] += v * c;
        acc[2 * q + 1] += v * sn;
        const double cn = c * c1 - sn * s1;
        sn = sn * c1 + c * s1;
        c = cn;
      }
    }
  }
  double* out = out_base + out_sys_stride * blockIdx.y + (size_t)x * MP;
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    const double s = wave_sum(acc[q]);
    if (lane == 0 && q < 2 * M) out[q] = s;
  }
}

// The row transform of r on the matrix cores, float64: Gr[x][k] =
// sum_y r[x][y] T(y, k) for k < 2M, T as in the tables above.  A block covers
// 16 rows; each of its eight waves takes an eighth of y (a 16 x 32 x Q product
// in 16x16x4 steps) and the eight partial tiles are added through LDS in a
// fixed order, so a system's result does not depend on the batch.  A wave
// issues all loads of a 64-point chunk of y before its products, since the
// launch is too small to hide memory latency by occupancy.  The B operands
// come from RD, stored in the products' fragment order: one contiguous 512-byte
// read per step and column tile (a gather from E64 would cost a cache access
// per lane).
constexpr int RD_WAVES = 8;   // the combine below adds eight partials; 512 threads = 16 rows x 32 columns
__global__ __launch_bounds__(64 * RD_WAVES) void k_rowdft_r(const SysDev* sys, int N, int M, const double* RD) {
  __shared__ double part[RD_WAVES][16][33];
  const SysDev sd = sys[blockIdx.y];
  if (!sd.active) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n16 = lane & 15, g = lane >> 4;
  const int x0 = blockIdx.x * 16;
  const int MP = round16(2 * M);
  const int Q = (((N + RD_WAVES - 1) / RD_WAVES) + 3) & ~3;
  const int ybeg = w * Q, yend = min(N, ybeg + Q);
  const int xr = x0 + n16;
  const bool rowok = xr < N;
  const double* rrow = sd.r + (size_t)(rowok ? xr : 0) * N;
  const int last = (round16(N) >> 2) - 1;   // last step of RD
  const double* RDl = RD + lane;
  double4_t acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  constexpr int CH = 16;   // steps of 4 points per chunk
  for (int yc = ybeg; yc < yend; yc += 4 * CH) {
    double av[CH], bv[CH][2];
#pragma unroll
    for (int s = 0; s < CH; ++s) {
      const int y = yc + 4 * s + g;
      av[s] = (rowok && y < yend) ? rrow[y] : 0.0;
      // steps past the table (points past N, whose r is zero above) read its last step
      const int st = min((yc >> 2) + s, last);
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) bv[s][cb] = RDl[(size_t)(st * 2 + cb) * 64];
    }
#pragma unroll
    for (int s = 0; s < CH; ++s)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s][cb], acc[cb], 0, 0, 0);
  }
  // accumulator item i of lane (n16, g) holds row 4 i + g, column n16
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int i = 0; i < 4; ++i) part[w][4 * i + g][cb * 16 + n16] = acc[cb][i];
  __syncthreads();
  const int row = threadIdx.x >> 5, col = threadIdx.x & 31;
  if (col < 2 * M && x0 + row < N) {
    double v[RD_WAVES];
#pragma unroll
    for (int j = 0; j < RD_WAVES; ++j) v[j] = part[j][row][col];
    sd.Gr[(size_t)(x0 + row) * MP + col] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  }
}

// Per-solve constant part of the layer-0 spectrum:
// Vc[c][a][ky] = sum_{f=1..3} W_L[c][f] DFT(phi_f) + b_L[c] DFT(1).
template <int PREC>
__global__ __launch_bounds__(256) void k_vconst(const SysDev* sys, int N, int M, int C, int basis,
                                               const double* E64, const double* Gf, size_t gf_sys_stride,
                                               const double* WL, const double* bL) {
  using acc_t = typename Mf<PREC>::acc_t;
  __shared__ double Fr[4][32], Fi[4][32];
  const SysDev sd = sys[blockIdx.y];
  const int ky = blockIdx.x;
  const int twoM = 2 * M, MP = round16(twoM);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double* G = Gf + gf_sys_stride * blockIdx.y;
  for (int job = wv; job < 4 * twoM; job += 4) {
    const int f = job / twoM, a = job - f * twoM;
    // twiddle index tw_index(basis, N, M, a, x), stepped by 64 rows at a time
    const int P = tw_period(basis, N);
    const int kv = basis == B_SINE ? a + 1 : (a < M ? a : N - twoM + a);
    const int xo = basis == B_SINE ? 1 : 0;
    double sr = 0.0, si = 0.0;
    int idx = (int)(((long long)kv * (lane + xo)) % P);
    const int step = (int)(((long long)kv * 64) % P);
    for (int x = lane; x < N; x += 64) {
      const double gc = G[((size_t)f * N + x) * MP + 2 * ky];
      const double gs = G[((size_t)f * N + x) * MP + 2 * ky + 1];
      const double c = E64[2 * idx], s = E64[2 * idx + 1];
      sr += gc * c - gs * s;
      si -= gc * s + gs * c;
      idx += step;
      if (idx >= P) idx -= P;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
      Fr[f][a] = sr;
      Fi[f][a] = si;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < C * twoM; t += 256) {
    const int c = t / twoM, a = t - c * twoM;
    double vr = bL[c] * Fr[3][a], vi = bL[c] * Fi[3][a];
    for (int f = 0; f < 3; ++f) {
      vr += WL[c * 4 + f + 1] * Fr[f][a];
      vi += WL[c * 4 + f + 1] * Fi[f][a];
    }
    acc_t* o = (acc_t*)sd.Vc + 2 * ((size_t)(c * twoM + a) * M + ky);
    o[0] = (acc_t)vr;
    o[1] = (acc_t)vi;
  }
}

// ---------------------------------------------------------------------------
// Spectral part of one layer, two launches.
//   k_spec_fwd (grid M x systems): for one ky, the x-direction forward DFT of
//     the row partials, V^[c][a] = sum_x (Gc - i Gs)[x][c] e^{-2 pi i kx_a x/N}
//     (rows staged through LDS in chunks of 64), then the per-mode mixing
//     W^[o][a] = sum_c V^[c][a] R[c][o][a][ky], written to Wh[ky][o][a].
//     Layer 0 builds V^ from the DFT of r and the per-solve constant part.
//   k_spec_inv (grid N/16 x systems): the x-direction synthesis
//     H[x][o][ky] = sum_a W^[o][a][ky] e^{+2 pi i kx_a x/N}, written as the
//     complete rows Hc[x][o][.] = (N^-2 g_ky Re H, -N^-2 g_ky Im H), g_0 = 1,
//     g_ky = 2 otherwise.
// ---------------------------------------------------------------------------
constexpr int SX = 64;   // rows per chunk in the forward transform

// Partial forward x-DFT over one chunk of SX rows for one ky:
// Vp[ky][xs][c][a] = sum_{x in chunk} (Gc - i Gs)[x][c] e^{-2 pi i kx_a x / N}.
// Layer 0 transforms the single channel of r's row partials instead.
template <int PREC, int C>
__global__ __launch_bounds__(256) void k_spec_fwd(SpecArgs a) {
  using M_ = Mf<PREC>;
  using acc_t = typename M_::acc_t;
  constexpr int CH = C;                        // channels per chunk row
  constexpr int LPT = SX * CH / 256;           // loads per thread
  __shared__ acc_t Gr_[SX][CH + 1], Gi_[SX][CH + 1];
  __shared__ acc_t Er_[32][SX + 1], Ei_[32][SX + 1];
  const int ky = blockIdx.x, xs = blockIdx.y;
  const SysDev sd = a.sys[blockIdx.z];
  if (!sd.active) return;
  const int N = a.N, M = a.M, twoM = 2 * M, MP = round16(twoM);
  const int x0 = xs * SX, nx = min(SX, N - x0);
  const acc_t* E = (const acc_t*)a.Eacc;
  const int t = threadIdx.x;
  acc_t* Vp = (acc_t*)sd.Vp + ((size_t)(ky * a.XS + xs) * C) * twoM * 2;
  // a fixed trip count (2M <= 32) so that every thread's table loads are in
  // flight together rather than one round trip per pass
#pragma unroll
  for (int i = 0; i < 32 * SX / 256; ++i) {
    const int q = t + 256 * i;
    const int kx = q / SX, xl = q - kx * SX;
    if (kx < twoM) {
      const int idx = (int)tw_index(a.basis, N, M, kx, x0 + xl);
      Er_[kx][xl] = E[2 * idx];
      Ei_[kx][xl] = -E[2 * idx + 1];
    } else {   // rows past 2M feed only output rows that are not stored
      Er_[kx][xl] = 0;
      Ei_[kx][xl] = 0;
    }
  }
  if (a.layer0) {
    if (t < SX) {
      const bool v = t < nx;
      Gr_[t][0] = v ? (acc_t)sd.Gr[(size_t)(x0 + t) * MP + 2 * ky] : (acc_t)0;
      Gi_[t][0] = v ? (acc_t)(-sd.Gr[(size_t)(x0 + t) * MP + 2 * ky + 1]) : (acc_t)0;
    }
    __syncthreads();
    if (t < twoM) {
      acc_t sr = 0, si = 0;
      for (int xl = 0; xl < nx; ++xl) {
        const acc_t gr = Gr_[xl][0], gi = Gi_[xl][0], er = Er_[t][xl], ei = Ei_[t][xl];
        sr += gr * er - gi * ei;
        si += gr * ei + gi * er;
      }
      Vp[2 * t] = sr;
      Vp[2 * t + 1] = si;
    }
    return;
  }
  const acc_t* Gp = (const acc_t*)sd.Gp;
  acc_t gc[LPT], gs[LPT];
#pragma unroll
  for (int u = 0; u < LPT; ++u) {
    gc[u] = 0;
    gs[u] = 0;
  }
  // segments outermost: the LPT points' loads of one segment are independent
  // and issue together (the per-point sums keep their segment order)
  for (int sg = 0; sg < a.S; ++sg) {
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int q = t + 256 * u;
      const int xl = q / CH, c = q - xl * CH;
      if (xl < nx) {
        const acc_t* row = Gp + (size_t)((x0 + xl) * a.S + sg) * MP * C;
        gc[u] += row[(2 * ky) * C + c];
        gs[u] += row[(2 * ky + 1) * C + c];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < LPT; ++u) {
    const int q = t + 256 * u;
    const int xl = q / CH, c = q - xl * CH;
    Gr_[xl][c] = gc[u];
    Gi_[xl][c] = -gs[u];
  }
  __syncthreads();
  // V^[kx][c] on the matrix cores in the accumulate precision, as real
  // products over the SX rows of the chunk (rows past nx hold zeros):
  // Re = Er Gr - Ei Gi, Im = Er Gi + Ei Gr.  Wave w takes the (16 x-modes,
  // 16 channels) output tiles w, w + 4, ...
  using MM = Mf<sizeof(acc_t) == 8 ? P64 : P32>;
  using vec_t = typename MM::accv_t;
  const int lane = t & 63, w = t >> 6, n16 = lane & 15, g = lane >> 4;
  const int nkt = (twoM + 15) >> 4;
  for (int pr = w; pr < nkt * (C / 16); pr += 4) {
    const int kt = pr % nkt, ct = pr / nkt;
    const int ka = kt * 16 + n16, cb = ct * 16 + n16;
    vec_t vr = {0, 0, 0, 0}, vi = {0, 0, 0, 0};
#pragma unroll 4
    for (int xb = 0; xb < SX; xb += 4) {
      const int xl = xb + g;
      const acc_t er = Er_[ka][xl], ei = Ei_[ka][xl];
      const acc_t gr = Gr_[xl][cb], gi = Gi_[xl][cb];
      vr = MM::mma(er, gr, vr);
      vr = MM::mma(-ei, gi, vr);
      vi = MM::mma(er, gi, vi);
      vi = MM::mma(ei, gr, vi);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kx = kt * 16 + MM::row(g, i);
      if (kx < twoM) {
        Vp[2 * (cb * twoM + kx)] = vr[i];
        Vp[2 * (cb * twoM + kx) + 1] = vi[i];
      }
    }
  }
}

// Sum of the chunk partials in chunk order and the per-mode mixing
// W^[o][a] = sum_c V^[c][a] R[c][o][a][ky], written to Wh[ky][o][a].
template <int PREC, int C>
__global__ __launch_bounds__(256) void k_spec_mix(SpecArgs a) {
  using M_ = Mf<PREC>;
  using acc_t = typename M_::acc_t;
  // one block per (ky, chunk of KXB kept x-modes, system); thread t owns
  // channel t % C of mode kx0 + t / C in both phases
  constexpr int KXB = 256 / C;
  __shared__ acc_t Vr[C][KXB + 1], Vi[C][KXB + 1];
  const int ky = blockIdx.x;
  const SysDev sd = a.sys[blockIdx.z];
  if (!sd.active) return;
  const int M = a.M, twoM = 2 * M;
  const int t = threadIdx.x;
  const int ch = t % C, kl = t / C, kx = blockIdx.y * KXB + kl;
  const bool live = kx < twoM;
  const acc_t* Vp = (const acc_t*)sd.Vp + (size_t)ky * a.XS * C * twoM * 2;
  // phase 1: this thread's V[c = ch][kx], the sum of the XS chunk partials
  if (live) {
    const size_t e = a.layer0 ? (size_t)2 * kx : (size_t)2 * (ch * twoM + kx);
    acc_t vr = 0, vi = 0;
    for (int xs = 0; xs < a.XS; ++xs) {
      vr += Vp[(size_t)xs * C * twoM * 2 + e];
      vi += Vp[(size_t)xs * C * twoM * 2 + e + 1];
    }
    if (a.layer0) {
      const double snorm = sd.st->snorm;
      const double inv_s = snorm > 0.0 ? 1.0 / snorm : 0.0;
      const double wl = (double)((const acc_t*)a.WL0)[ch] * inv_s;
      const acc_t* vc = (const acc_t*)sd.Vc + 2 * ((size_t)(ch * twoM + kx) * M + ky);
      vr = (acc_t)(wl * (double)vr) + vc[0];
      vi = (acc_t)(wl * (double)vi) + vc[1];
    }
    Vr[ch][kl] = vr;
    Vi[ch][kl] = vi;
    if (a.Vsave) {
      // mode-major, [ky][kx][system][c] complex (the weight gradient's operand)
      acc_t* vs = (acc_t*)a.Vsave + ((((size_t)ky * twoM + kx) * a.nsys + blockIdx.z) * C + ch) * 2;
      vs[0] = vr;
      vs[1] = vi;
    }
  }
  __syncthreads();
  if (!live) return;
  // phase 2: output channel o = ch of mode kx, all C weight pairs in flight
  const int o = ch, MP = round16(twoM);
  const acc_t* Rk = (const acc_t*)a.R + ((size_t)ky * twoM + kx) * C * C * 2;
  acc_t rr[C], ri[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    rr[c] = Rk[2 * (c * C + o)];
    ri[c] = Rk[2 * (c * C + o) + 1];
  }
  acc_t sr = 0, si = 0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    sr += Vr[c][kl] * rr[c] - Vi[c][kl] * ri[c];
    si += Vr[c][kl] * ri[c] + Vi[c][kl] * rr[c];
  }
  acc_t* Wh = (acc_t*)sd.Wh + (size_t)ky * C * MP * 2;
  Wh[2 * (o * MP + kx)] = sr;
  Wh[2 * (o * MP + kx) + 1] = si;
}

// x-direction synthesis for SR rows: H[x][o][ky] = sum_a W^[ky][o][a]
// e^{+2 pi i kx_a x/N}, staged in LDS as complete rows Hc[x][o][0..MP) and
// written out contiguously.
// One thread per (o, ky) pair: the block has C*M threads rounded up to whole
// waves (at most 512).
template <int PREC> struct SynthRows { static constexpr int SR = 8; };
template <> struct SynthRows<P64> { static constexpr int SR = 8; };
__host__ __device__ inline int synth_threads(int C, int M) { return ((C * M + 63) / 64) * 64; }

template <int PREC, int C, int MP>
__global__ __launch_bounds__(512) void k_spec_inv(SpecArgs a) {
  using M_ = Mf<PREC>;
  using in_t = typename M_::in_t;
  using acc_t = typename M_::acc_t;
  constexpr int SR = SynthRows<PREC>::SR;
  __shared__ acc_t Er_[SR][MP], Ei_[SR][MP];   // zero for kx >= 2M
  __shared__ __attribute__((aligned(16))) in_t tile[SR * C * MP];
  const SysDev sd = a.sys[blockIdx.y];
  if (!sd.active) return;
  const int N = a.N, M = a.M, twoM = 2 * M;
  const int x0 = blockIdx.x * SR;
  const int nx = min(SR, N - x0);
  const acc_t* E = (const acc_t*)a.Eacc;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int q = t; q < SR * MP; q += nt) {
    const int xl = q / MP, kx = q - xl * MP;
    const int idx = kx < twoM ? (int)tw_index(a.basis, N, M, kx, x0 + xl) : 0;
    Er_[xl][kx] = kx < twoM ? E[2 * idx] : (acc_t)0;
    Ei_[xl][kx] = kx < twoM ? E[2 * idx + 1] : (acc_t)0;
  }
  for (int q = t; q < SR * C * MP; q += nt) tile[q] = M_::cvt((acc_t)0);
  __syncthreads();
  const double scale = 1.0 / ((double)N * (double)N);
  for (int q = t; q < C * M; q += nt) {
    const int o = q / M, ky = q - o * M;
    const acc_t* Wh = (const acc_t*)sd.Wh + ((size_t)ky * C + o) * MP * 2;   // zero past 2M
    acc_t wr[MP], wi[MP];
#pragma unroll
    for (int kx = 0; kx < MP; ++kx) {
      wr[kx] = Wh[2 * kx];
      wi[kx] = Wh[2 * kx + 1];
    }
    // inverse normalisation: Fourier N^-2 g_ky (g_0 = 1, else 2), sine (2/(N+1))^2
    const acc_t sc = a.unit_scale ? (acc_t)1
                     : a.basis == B_SINE ? (acc_t)(4.0 / ((double)(N + 1) * (double)(N + 1)))
                                         : (acc_t)((ky == 0 ? 1.0 : 2.0) * scale);
    for (int xl = 0; xl < nx; ++xl) {
      acc_t hr = 0, hi = 0;
#pragma unroll
      for (int kx = 0; kx < MP; ++kx) {
        hr += wr[kx] * Er_[xl][kx] - wi[kx] * Ei_[xl][kx];
        hi += wr[kx] * Ei_[xl][kx] + wi[kx] * Er_[xl][kx];
      }
      tile[(xl * C + o) * MP + 2 * ky] = M_::cvt(sc * hr);
      tile[(xl * C + o) * MP + 2 * ky + 1] = M_::cvt(-sc * hi);
    }
  }
  __syncthreads();
  // contiguous copy of rows x0 .. x0+nx-1 (nx*C*MP elements, a multiple of 16 bytes)
  const int nbytes = nx * C * MP * (int)sizeof(in_t);
  const uint4* src = (const uint4*)tile;
  uint4* dst = (uint4*)((char*)sd.Hc + (size_t)x0 * C * MP * sizeof(in_t));
  for (int q = t; q < nbytes / 16; q += nt) dst[q] = src[q];
}

// ---------------------------------------------------------------------------
// bfloat16 operator: the x-direction transforms on the matrix cores
// (16x16x32 bfloat16 products with float32 accumulation).  Every operand
// value v travels as a bfloat16 pair hi = bf16(v), lo = bf16(v - hi), and a
// product is accumulated as hi*hi + hi*lo + lo*hi (the dropped lo*lo term is
// below 2^-16 of it), so the spectra keep close to float32 accuracy while the
// contraction runs at the bfloat16 rate.
//
// Interleaving real and imaginary parts along the contraction index k makes
// the complex sums real products:
//   forward, k = (x, t):   V~r[a][c] = sum_k Ar[a][k] G[k][c], V~i likewise
//       with Ai, where G[(x,0)][c] = Gc[x][c], G[(x,1)][c] = Gs[x][c],
//       Ar[a][(x,0)] = cos, Ar[a][(x,1)] = -sin and Ai = (-sin, -cos) per
//       pair (V^ = sum_x (cos - i sin)(Gc - i Gs) with the angle of mode a at
//       row x);
//   synthesis, k = (a, t): Hr[x][j] = sum_k Sr[x][k] W[k][j], Hi likewise
//       with Si, where W[(a,0)][j] = Re W^[a][j], W[(a,1)][j] = Im W^[a][j],
//       Sr[x][(a,0)] = cos, Sr[x][(a,1)] = -sin and Si = (sin, cos) per pair
//       (H = sum_a W^ (cos + i sin)).
// Ai and Si pairs are Ar and Sr pairs swapped with one sign flipped, so
// only Ar (table FA) and Sr (table SA) are stored; both hold the same values
// in two layouts.  For the sine basis the "cos" slot holds the sine mode and
// the "sin" slot zero, as in the other tables.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short short8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float4_t mfma_bf32(bf16x8_t a, bf16x8_t b, float4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// hi*hi + hi*lo + lo*hi
__device__ __forceinline__ float4_t mfma_bf3(bf16x8_t ah, bf16x8_t al, bf16x8_t bh, bf16x8_t bl, float4_t c) {
  c = mfma_bf32(ah, bh, c);
  c = mfma_bf32(ah, bl, c);
  return mfma_bf32(al, bh, c);
}
// pairs (e0, e1) -> (e1, -e0): forward Ai from Ar
__device__ __forceinline__ bf16x8_t pairs_fwd(bf16x8_t v) {
  const short8_t s = __builtin_bit_cast(short8_t, v);
  short8_t o;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    o[2 * p] = s[2 * p + 1];
    o[2 * p + 1] = (short)(s[2 * p] ^ (short)0x8000);
  }
  return __builtin_bit_cast(bf16x8_t, o);
}
// pairs (e0, e1) -> (-e1, e0): synthesis Si from Sr
__device__ __forceinline__ bf16x8_t pairs_inv(bf16x8_t v) {
  const short8_t s = __builtin_bit_cast(short8_t, v);
  short8_t o;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    o[2 * p] = (short)(s[2 * p + 1] ^ (short)0x8000);
    o[2 * p + 1] = s[2 * p];
  }
  return __builtin_bit_cast(bf16x8_t, o);
}
__device__ __forceinline__ void split_bf(float v, __bf16& hi, __bf16& lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

// Twiddle A operands of the x-direction products, value (h, a, x, t) = part h
// (0 hi, 1 lo) of t = 0: cos, t = 1: -sin of mode a < 32 at row x < NP (zero
// for a >= 2M or x >= N), each in the fragment order of its product so that
// a wave reads one contiguous kilobyte per fragment:
//   FA (forward, lane (n, g) of row step s and mode group kg holds a = 16 kg
//       + n, x = 16 s + 4 g + e / 2, t = e % 2, e < 8):
//       FA[(((h * 2 + kg) * NP / 16 + s) * 64 + 16 g + n) * 8 + e]
//   SA (synthesis, lane (n, g) of row tile xt and step ks holds x = 16 xt + n,
//       2a + t = 32 ks + 8 g + e):
//       SA[(((h * NP / 16 + xt) * 2 + ks) * 64 + 16 g + n) * 8 + e]
__global__ __launch_bounds__(256) void k_tables_bfx(int N, int M, int basis, const double* E64, __bf16* FA,
                                                   __bf16* SA) {
  const int NP = round16(N);
  const int q = blockIdx.x * 256 + threadIdx.x;   // (x, a, t), a fastest after t
  if (q >= NP * 64) return;
  const int x = q >> 6, a = (q >> 1) & 31, t = q & 1;
  double v = 0.0;
  if (a < 2 * M && x < N) {
    const unsigned idx = tw_index(basis, N, M, a, x);
    v = t == 0 ? E64[2 * idx] : -E64[2 * idx + 1];
  }
  const __bf16 hi = (__bf16)(float)v;
  const __bf16 lo = (__bf16)(float)(v - (double)(float)hi);
  const int ns = NP >> 4;
  const size_t fa = ((size_t)((a >> 4) * ns + (x >> 4)) * 64 + 16 * ((x & 15) >> 2) + (a & 15)) * 8 + 2 * (x & 3) + t;
  const int col = 2 * a + t;
  const size_t sa = ((size_t)((x >> 4) * 2 + (col >> 5)) * 64 + 16 * ((col & 31) >> 3) + (x & 15)) * 8 + (col & 7);
  FA[fa] = hi;
  FA[(size_t)2 * ns * 512 + fa] = lo;
  SA[sa] = hi;
  SA[(size_t)ns * 1024 + sa] = lo;
}

// Gather-free twiddles, copied from E64 / Eacc (the same values the index
// walks over those tables would fetch):
//   RD (every operator): the row transform of r, entry (s, cb, 16 g + n) =
//       T(4 s + g, 16 cb + n), the B operand of step s, column tile cb
//   EX (bfloat16 operator): the first layer's x transform, EX[x][a] =
//       (Eacc cos, -Eacc sin) at tw_index(a, x)
__global__ __launch_bounds__(256) void k_tables_rx(int N, int M, int basis, const double* E64, const float* Eacc,
                                                  double* RD, float2* EX) {
  const int NP = round16(N);
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= NP * 32) return;
  {
    const int st = q >> 7, cb = (q >> 6) & 1, n = q & 15, g = (q >> 4) & 3;
    const int y = 4 * st + g, k = cb * 16 + n, h = k >> 1;
    const bool sine = basis == B_SINE;
    double v = 0.0;
    if (y < N && k < 2 * M && !(sine && (k & 1))) {
      const unsigned P = (unsigned)tw_period(basis, N);
      const unsigned idx = sine ? ((unsigned)(h + 1) * (unsigned)(y + 1)) % P : ((unsigned)h * (unsigned)y) % P;
      v = E64[2 * idx + (sine ? 0 : (k & 1))];
    }
    RD[q] = v;
  }
  if (EX) {
    const int x = q >> 5, a = q & 31;
    float2 e = {0.f, 0.f};
    if (x < N && a < 2 * M) {
      const unsigned idx = tw_index(basis, N, M, a, x);
      e = float2{Eacc[2 * idx], -Eacc[2 * idx + 1]};
    }
    EX[q] = e;
  }
}

// Synthesis operand WT[h] of the mixed spectrum, value (j = o M + ky,
// column 2a + t) in the fragment order of the synthesis product: lane
// (n, g) of column tile jt and step ks holds j = 16 jt + n, column 32 ks +
// 8 g + e.
__device__ __forceinline__ size_t wt_index(int j, int col) {
  return ((size_t)((j >> 4) * 2 + (col >> 5)) * 64 + 16 * ((col & 31) >> 3) + (j & 15)) * 8 + (col & 7);
}

// Row partial spectra of the bfloat16 layer kernel, Gp[ky][x][seg][c][t]
// (t = 0: the cos part, 1: the sin part of mode ky; modes ky < M only):
// the forward transform of mode ky reads one contiguous block.
__device__ __forceinline__ size_t gp_index(int N, int S, int C, int ky, int x, int seg, int c) {
  return ((((size_t)ky * N + x) * S + seg) * C + c) * 2;
}

// Forward transform along x and mode mixing of one layer, one block per
// (ky, group of 16 kept x-modes, system), bfloat16 operator:
//   V^[c][a] = sum_x (Gc - i Gs)[x][c] e^{-2 pi i kx_a x / N}   (matrix cores)
//   W^[o][a] = sum_c V^[c][a] R[c][o][a][ky]                      (vector ALU)
// The mixing of mode a needs V^ of that mode only, so the blocks of one
// (ky, system) split the modes and need no exchange.  The mixed spectrum is
// written as the synthesis operand WT (zero for a >= 2M).  Eight waves split the 16-row steps of x; each issues the loads
// of its steps before their products, and the eight partial tiles are added
// in a fixed order through LDS.  Layer 0 transforms the single channel of
// r's row partials instead and adds the per-solve constant part.
// SEG: the row-segment count a.S as a compile-time constant (1, 2 or 4, so
// that the loads of every segment issue together), or 0 for any count.
// KGN: groups of 16 modes per block, 1 or 2 (two: the block reads its rows
// once for both groups; used while many systems fill the chip, the same
// sums either way).
constexpr int XFM_THREADS = 512;
constexpr int XFM_CUS = 256;   // compute units of the MI355X
template <int C, int SEG, int KGN>
__global__ __launch_bounds__(XFM_THREADS) void k_xfm_bf(SpecArgs a, const __bf16* FA) {
  constexpr int NW = XFM_THREADS / 64, NCT = C / 16, SPW = SEG == 4 ? 2 : 4;
  constexpr int SEG0 = SEG > 0 ? SEG : 1;   // segments summed in the first pass
  constexpr int NK = 16 * KGN;              // modes of the block
  __shared__ float red[NW][KGN * 2 * NCT][256];   // [wave][(group, re/im, ct)][element]
  __shared__ float Vr_[C][NK + 1], Vi_[C][NK + 1];
  const int ky = blockIdx.x, kg = blockIdx.y * KGN;   // modes a = 16 kg .. 16 kg + NK - 1
  const SysDev sd = a.sys[blockIdx.z];
  if (!sd.active) return;
  const int N = a.N, M = a.M, twoM = 2 * M, MP = round16(twoM), NP = round16(N);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, n16 = lane & 15, g = lane >> 4;
  const int nkt = (twoM + 15) >> 4;
  if (KGN == 1 && a.layer0) {
    // S[a] = sum_x (Gr - i Gi)[x] e^{-i theta}, float32, 32 row parts per mode
    constexpr int XR = XFM_THREADS / 16, CHR = 8;
    __shared__ float pr_[XR][17], pi_[XR][17];
    const float2* EX = (const float2*)a.EX;   // [NP][32]: 16 modes of a row in 128 contiguous bytes
    const int kl = t & 15, ka = kg * 16 + kl, part = t >> 4;
    float sr = 0.f, si = 0.f;
    if (ka < twoM) {
      // chunks of eight rows per thread: every load of a chunk is issued
      // before its sums (a runtime loop would wait on each load in turn)
      for (int x0 = part; x0 < N; x0 += XR * CHR) {
        double g0[CHR], g1[CHR];
        float er[CHR], ei[CHR];
#pragma unroll
        for (int e = 0; e < CHR; ++e) {
          // rows past N read row 0 (unconditional loads, no branches) and
          // are zeroed below
          const int x = x0 + e * XR;
          const int xc = x < N ? x : 0;
          g0[e] = sd.Gr[(size_t)xc * MP + 2 * ky];
          g1[e] = sd.Gr[(size_t)xc * MP + 2 * ky + 1];
          const float2 ex = EX[(size_t)xc * 32 + ka];
          er[e] = ex.x;
          ei[e] = ex.y;
        }
#pragma unroll
        for (int e = 0; e < CHR; ++e) {
          const bool v = x0 + e * XR < N;
          const float gr = v ? (float)g0[e] : 0.f, gi = v ? -(float)g1[e] : 0.f;
          sr += gr * er[e] - gi * ei[e];
          si += gr * ei[e] + gi * er[e];
        }
      }
    }
    pr_[part][kl] = sr;
    pi_[part][kl] = si;
    __syncthreads();
    const double snorm = sd.st->snorm;
    const double inv_s = snorm > 0.0 ? 1.0 / snorm : 0.0;
    for (int q = t; q < C * 16; q += XFM_THREADS) {
      const int c = q >> 4, k2 = q & 15, kx = kg * 16 + k2;
      if (kx >= twoM) continue;
      float vr = 0.f, vi = 0.f;
#pragma unroll
      for (int p = 0; p < XR; ++p) {
        vr += pr_[p][k2];
        vi += pi_[p][k2];
      }
      const double wl = (double)((const float*)a.WL0)[c] * inv_s;
      const float* vc = (const float*)sd.Vc + 2 * ((size_t)(c * twoM + kx) * M + ky);
      Vr_[c][k2] = (float)(wl * (double)vr) + vc[0];
      Vi_[c][k2] = (float)(wl * (double)vi) + vc[1];
    }
  } else {
    const float* Gp = (const float*)sd.Gp;
    const int ns = NP >> 4;
    const __bf16* FAh = FA + ((size_t)kg * ns * 64 + lane) * 8;
    const __bf16* FAl = FAh + (size_t)2 * ns * 512;
    float4_t acc[KGN][2][NCT];
#pragma unroll
    for (int kq = 0; kq < KGN; ++kq)
#pragma unroll
      for (int ri = 0; ri < 2; ++ri)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[kq][ri][ct] = float4_t{0.f, 0.f, 0.f, 0.f};
    const int nsteps = NP >> 4;
    for (int s0 = w; s0 < nsteps; s0 += NW * SPW) {
      // loads of up to SPW steps (s0, s0 + NW, ...) before any product: the
      // first SEG0 segments of every (step, channel, row, Gc/Gs); rows past
      // N and dead steps read row 0 and are zeroed after
      float raw[SPW][NCT][8][SEG0];
      bf16x8_t ah[SPW][KGN], al[SPW][KGN];
#pragma unroll
      for (int u = 0; u < SPW; ++u) {
        const int st = s0 + u * NW;
        const int stc = st < nsteps ? st : 0;
        const int x0 = stc * 16 + 4 * g;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const int c = ct * 16 + n16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int x = x0 + r < N ? x0 + r : 0;
#pragma unroll
            for (int sg = 0; sg < SEG0; ++sg) {
              const float2 v = *(const float2*)(Gp + gp_index(N, a.S, C, ky, x, sg, c));
              raw[u][ct][2 * r][sg] = v.x;
              raw[u][ct][2 * r + 1][sg] = v.y;
            }
          }
        }
#pragma unroll
        for (int kq = 0; kq < KGN; ++kq) {
          ah[u][kq] = *(const bf16x8_t*)(FAh + ((size_t)kq * ns + stc) * 512);
          al[u][kq] = *(const bf16x8_t*)(FAl + ((size_t)kq * ns + stc) * 512);
        }
      }
      // every load above completes here, before any sum or product (the
      // compiler would otherwise issue each step's loads after the previous
      // step's products, one round trip per step)
#pragma unroll
      for (int u = 0; u < SPW; ++u) {
#pragma unroll
        for (int kq = 0; kq < KGN; ++kq) asm volatile("" : "+v"(ah[u][kq]), "+v"(al[u][kq]));
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
          for (int e = 0; e < 8; ++e)
#pragma unroll
            for (int sg = 0; sg < SEG0; ++sg) asm volatile("" : "+v"(raw[u][ct][e][sg]));
      }
      float gv[SPW][NCT][8];
#pragma unroll
      for (int u = 0; u < SPW; ++u) {
        const int st = s0 + u * NW;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            float v = 0.f;
#pragma unroll
            for (int sg = 0; sg < SEG0; ++sg) v += raw[u][ct][e][sg];
            const bool ok = st < nsteps && st * 16 + 4 * g + (e >> 1) < N;
            gv[u][ct][e] = ok ? v : 0.f;
          }
      }
      for (int sg = SEG0; SEG == 0 && sg < a.S; ++sg) {
#pragma unroll
        for (int u = 0; u < SPW; ++u) {
          const int st = s0 + u * NW;
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            const int c = ct * 16 + n16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int x = st * 16 + 4 * g + r;
              const bool v = st < nsteps && x < N;
              const float2 gcs = *(const float2*)(Gp + gp_index(N, a.S, C, ky, v ? x : 0, sg, c));
              gv[u][ct][2 * r] += v ? gcs.x : 0.f;
              gv[u][ct][2 * r + 1] += v ? gcs.y : 0.f;
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < SPW; ++u) {
        if (s0 + u * NW >= nsteps) break;
        bf16x8_t bh[NCT], bl[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            __bf16 h, l;
            split_bf(gv[u][ct][e], h, l);
            bh[ct][e] = h;
            bl[ct][e] = l;
          }
#pragma unroll
        for (int kq = 0; kq < KGN; ++kq) {
          const bf16x8_t aih = pairs_fwd(ah[u][kq]), ail = pairs_fwd(al[u][kq]);
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            acc[kq][0][ct] = mfma_bf3(ah[u][kq], al[u][kq], bh[ct], bl[ct], acc[kq][0][ct]);
            acc[kq][1][ct] = mfma_bf3(aih, ail, bh[ct], bl[ct], acc[kq][1][ct]);
          }
        }
      }
    }
    // partial tiles -> LDS; element index i * 64 + lane (row 4 g + i, column n16)
#pragma unroll
    for (int kq = 0; kq < KGN; ++kq)
#pragma unroll
      for (int ri = 0; ri < 2; ++ri)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
          for (int i = 0; i < 4; ++i) red[w][(kq * 2 + ri) * NCT + ct][i * 64 + lane] = acc[kq][ri][ct][i];
    __syncthreads();
    // fixed-order sum over the waves, then V^[c][a] of this block's modes
    for (int q = t; q < KGN * 2 * NCT * 256; q += XFM_THREADS) {
      const int tile = q >> 8, el = q & 255;
      float v = 0.f;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) v += red[ww][tile][el];
      const int ct = tile % NCT, ri = (tile / NCT) & 1, kq = tile / (2 * NCT);
      const int i = el >> 6, ln = el & 63;
      const int k2 = kq * 16 + 4 * (ln >> 4) + i, c = ct * 16 + (ln & 15);
      if (ri == 0) Vr_[c][k2] = v;
      else Vi_[c][k2] = v;
    }
  }
  __syncthreads();
  // mixing: output (a, o) per thread, all C weight pairs of it loaded together
  const float* Rk0 = (const float*)a.R + (size_t)ky * twoM * C * C * 2;
  __bf16* WTh = (__bf16*)sd.WT;
  __bf16* WTl = WTh + (size_t)C * M * 64;
  // this block's modes; the last group also clears the slots 16 nkt .. 31
  const int kend = kg + KGN - 1 == nkt - 1 ? 32 : kg * 16 + NK;
  // mixed values staged per output channel o: word k2 holds the bfloat16
  // pair of local mode k2 (33 words per row: no bank conflicts)
  __shared__ uint32_t wst[2][C][33];
  for (int q = t; q < (kend - kg * 16) * C; q += XFM_THREADS) {
    const int kx = kg * 16 + q / C, o = q % C, k2 = kx - kg * 16;
    float sr = 0.f, si = 0.f;
    if (kx < twoM) {
      const float* Rk = Rk0 + (size_t)kx * C * C * 2;
      float rr[C], rim[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        rr[c] = Rk[2 * (c * C + o)];
        rim[c] = Rk[2 * (c * C + o) + 1];
      }
      // each term's rounding is written out (one product rounded, the other
      // fused), so that every variant of the kernel forms the same bits
#pragma unroll
      for (int c = 0; c < C; ++c) {
        sr += __builtin_fmaf(Vr_[c][k2], rr[c], -(Vi_[c][k2] * rim[c]));
        si += __builtin_fmaf(Vi_[c][k2], rr[c], Vr_[c][k2] * rim[c]);
      }
    }
    __bf16 h0, l0, h1, l1;
    split_bf(sr, h0, l0);
    split_bf(si, h1, l1);
    // columns 2 kx (Re) and 2 kx + 1 (Im), one 32-bit word per part
    wst[0][o][k2] = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
    wst[1][o][k2] = (uint32_t)__builtin_bit_cast(uint16_t, l0) | ((uint32_t)__builtin_bit_cast(uint16_t, l1) << 16);
  }
  __syncthreads();
  // each (part, output channel, group of 8 columns) leaves as one 16-byte
  // store: the 8 columns 32 kg + 8 cg .. + 7 of row o M + ky are contiguous
  const int ncg = (kend - kg * 16) >> 2;
  for (int q = t; q < 2 * C * ncg; q += XFM_THREADS) {
    const int part = q / (C * ncg), o = (q / ncg) % C, cg = q % ncg;
    const uint32_t* src = &wst[part][o][4 * cg];
    uint4 v;
    v.x = src[0];
    v.y = src[1];
    v.z = src[2];
    v.w = src[3];
    *(uint4*)((part ? WTl : WTh) + wt_index(o * M + ky, 32 * kg + 8 * cg)) = v;
  }
}

// x-direction synthesis, bfloat16 operator, one block per (16 rows, group of
// output channels: the grid's y dimension splits the channels into equal
// groups whose column tiles split evenly):
// H[x][j] = sum_a W^[a][j] e^{+2 pi i kx_a x / N}, j = o*M + ky, on the matrix
// cores, written as the rows Hc[x][o][.] = (s Re H, -s Im H) of the block's
// channels with the inverse normalisation s of the basis (Fourier N^-2 g_ky,
// g_0 = 1 else 2; sine (2/(N+1))^2), zero past 2M.  Column tile jt covers
// j = 16 jt .. 16 jt + 15, so group y of the tiles holds exactly the
// channels y C/nh .. (y + 1) C/nh - 1.  Waves take the block's tiles in turn;
// the rows pass through LDS for contiguous stores.
template <int C, int MP, int TPWV>
__global__ __launch_bounds__(256) void k_xinv_bf(SpecArgs a, const __bf16* SA) {
  __shared__ __attribute__((aligned(16))) uint16_t tile[16 * C * MP];
  const SysDev sd = a.sys[blockIdx.z];
  if (!sd.active) return;
  const int N = a.N, M = a.M, NP = round16(N);
  const int x0 = blockIdx.x * 16;
  const int nx = min(16, N - x0);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, n16 = lane & 15, g = lane >> 4;
  const int ntile = C * M / 16;   // at most 32 (C, M <= 32, 16)
  const int nh = gridDim.y;       // channel groups: C and ntile divisible by nh
  const int jt0 = blockIdx.y * (ntile / nh), jt1 = jt0 + ntile / nh;
  const int o0 = blockIdx.y * (C / nh), o1 = o0 + C / nh;
  for (int q = t; q < 16 * C * MP / 8; q += 256) ((uint4*)tile)[q] = uint4{0u, 0u, 0u, 0u};
  // A operands of this lane's row x0 + n16, both contraction steps (k = 32 ks + 8 g ..)
  const __bf16* SAl = SA + (size_t)NP * 64;
  bf16x8_t sh[2], sl[2], ih[2], il[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    const size_t o = ((size_t)(blockIdx.x * 2 + ks) * 64 + lane) * 8;
    sh[ks] = *(const bf16x8_t*)(SA + o);
    sl[ks] = *(const bf16x8_t*)(SAl + o);
    ih[ks] = pairs_inv(sh[ks]);
    il[ks] = pairs_inv(sl[ks]);
  }
  __syncthreads();
  const __bf16* WTh = (const __bf16*)sd.WT;
  const __bf16* WTl = WTh + (size_t)C * M * 64;
  const float scale0 = a.basis == B_SINE ? (float)(4.0 / ((double)(N + 1) * (double)(N + 1)))
                                         : (float)(1.0 / ((double)N * (double)N));
  // a wave takes tiles jt0 + w, jt0 + w + 4, ... (at most TPWV of them)
  bf16x8_t bh[TPWV][2], bl[TPWV][2];
#pragma unroll
  for (int u = 0; u < TPWV; ++u) {
    const int jt = jt0 + w + 4 * u;
    const int jc = jt < jt1 ? jt : jt0;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const size_t o = ((size_t)(jc * 2 + ks) * 64 + lane) * 8;
      bh[u][ks] = *(const bf16x8_t*)(WTh + o);
      bl[u][ks] = *(const bf16x8_t*)(WTl + o);
    }
  }
#pragma unroll
  for (int u = 0; u < TPWV; ++u) {
    const int jt = jt0 + w + 4 * u;
    if (jt >= jt1) break;
    const int j = jt * 16 + n16;
    float4_t hr = {0.f, 0.f, 0.f, 0.f}, hi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      hr = mfma_bf3(sh[ks], sl[ks], bh[u][ks], bl[u][ks], hr);
      hi = mfma_bf3(ih[ks], il[ks], bh[u][ks], bl[u][ks], hi);
    }
    // lane holds rows 4 g + i of column j
    const int o = j / M, ky = j - o * M;
    const float sc = a.basis == B_SINE ? scale0 : (ky == 0 ? scale0 : 2.f * scale0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int xl = 4 * g + i;
      tile[(xl * C + o) * MP + 2 * ky] = f2bf(sc * hr[i]);
      tile[(xl * C + o) * MP + 2 * ky + 1] = f2bf(-sc * hi[i]);
    }
  }
  __syncthreads();
  // rows x0 .. x0 + nx - 1, channels o0 .. o1 - 1: one contiguous run per row
  const int nrow = (o1 - o0) * MP / 8;   // 16-byte chunks per row
  for (int q = t; q < nx * nrow; q += 256) {
    const int xl = q / nrow, c = q - xl * nrow;
    const size_t e = (size_t)(xl * C + o0) * MP + (size_t)c * 8;
    *(uint4*)((uint16_t*)sd.Hc + (size_t)x0 * C * MP + e) = *(const uint4*)(tile + e);
  }
}

// ---------------------------------------------------------------------------
// Layer kernel: synthesis along y + bypass + bias + GELU, then either the
// next layer's y-direction analysis or the projection.
// ---------------------------------------------------------------------------
// Layer activation in the accumulate precision: erf-form GELU for the float64
// and float32 operators, the cheaper fitted form for the bfloat16 operator.
template <int PREC, typename T>
__device__ __forceinline__ T act(T z) {
  if constexpr (PREC == PBF) return gelu_bf(z);
  else return gelu(z);
}

struct LayerArgs {
  const SysDev* sys;
  int N, S, twoM, slot_in, slot_out;
  const void* T;    // [NP][MP]
  const void* TT;   // [MP][NP]
  const void* Wf;   // [C][KWP] op precision
  const void* bias; // [C] accumulate precision
  const void* WP;   // [C] accumulate precision
  const double* bP; // float64 projection bias (device)
  void* zout;       // training: pre-activation z of this layer, [sys][N^2][C] op precision (nullable)
  size_t z_sys;     // elements per system in zout
  int spw;          // row segments (of TPW tiles) per wave
  int wdots = 0;    // projection layer in a solve: also form the window sums (w_i, s_k)
};

template <int PREC, int C, int MP, bool FEAT, bool PROJ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PREC == PBF ? (FEAT ? 4 : 3) : 1))) void k_layer(LayerArgs a) {
  using M_ = Mf<PREC>;
  using in_t = typename M_::in_t;
  using acc_t = typename M_::acc_t;
  using frag_t = typename M_::frag_t;
  using accv_t = typename M_::accv_t;
  constexpr int KPL = M_::KPL, KSTEP = 4 * KPL;
  constexpr int NOB = C / 16;
  constexpr int KT = MP / KSTEP;
  constexpr int KIN = FEAT ? 1 : C / KSTEP;
  constexpr int KWP = KIN * KSTEP;
  constexpr int MB = MP / 16;
  // Activations are stored [point][C] in channel order.  Lane group g loads the
  // CB = C/4 contiguous channels [g*CB, (g+1)*CB) of its point with one vector
  // access; input K-step ks, element e then carries channel g*CB + ks*KPL + e
  // (the host lays out the bypass weights in that order).
  constexpr int CB = C / 4;
  constexpr int PADE = 16 / (int)sizeof(in_t);   // LDS row padding, 16 bytes
  __shared__ __attribute__((aligned(16))) in_t otile[4][16 * (C + PADE)];
  const int lane = threadIdx.x & 63;
  const int n16 = lane & 15, g = lane >> 4;
  const SysDev sd = a.sys[blockIdx.y];
  if (!sd.active) return;
  const int N = a.N, NP = round16(N);
  // A wave takes a.spw consecutive row segments of TPW tiles each and writes
  // one partial spectrum per segment, so the results do not depend on spw.
  const int ngrp = (a.S + a.spw - 1) / a.spw;
  // wave-uniform: kept in scalar registers, with every index derived from it
  const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (item >= N * ngrp) return;
  const int x = item / ngrp, grp = item - x * ngrp;
  const int nyt = NP >> 4;
  const int sg0 = grp * a.spw, sg1 = min(a.S, sg0 + a.spw);
  const double snorm = sd.st->snorm;
  const int twoM = a.twoM;
  // Projection layer in a solve: the window sums (w_i, s_k) of Algorithm 1
  // over the window k = i - m_i .. i - 1, formed from w_i as it is written
  // (the separate window-sum pass would read w_i back).  Lane group g takes
  // the window slots g and g + 4 (m_i <= 8).  One partial per 4/S rows
  // (S <= 2): each wave adds its segments' sums in segment order, the block
  // adds its waves' values per row and the rows per partial in order, so the
  // partials do not depend on spw.
  constexpr int WJ = 2;
  int wm = 0;
  const double* svp[WJ] = {nullptr, nullptr};
  if (PROJ && a.wdots) {
    const int it = sd.it, mmax = sd.mmax, ring = mmax + 1;
    wm = window_size(it, mmax);
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      const int q = min(g + 4 * j, max(wm - 1, 0));
      svp[j] = sd.S + (size_t)((it - wm + q) % ring) * N * N + (size_t)x * N;
    }
  }
  const bool wd = wm > 0;
  double wacc[WJ] = {0.0, 0.0}, wrow[WJ] = {0.0, 0.0};

  frag_t Bf[KT + KIN][NOB];
  const in_t* Hc = (const in_t*)sd.Hc + (size_t)x * C * MP;
  const in_t* Wf = (const in_t*)a.Wf;
  // bias and projection weights by accumulator item: the projection layer
  // computes its product transposed (item i of lane (n, g) holds channel
  // 16 ob + row(g, i) of point y0 + n), the others item-independent
  acc_t bias[NOB][4], wp[NOB][4];
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob) {
    const int o = ob * 16 + n16;
#pragma unroll
    for (int ks = 0; ks < KT; ++ks) Bf[ks][ob] = M_::ld(Hc + o * MP + ks * KSTEP + g * KPL);
#pragma unroll
    for (int ks = 0; ks < KIN; ++ks) Bf[KT + ks][ob] = M_::ld(Wf + o * KWP + ks * KSTEP + g * KPL);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int oi = PROJ ? ob * 16 + M_::row(g, i) : o;
      bias[ob][i] = ((const acc_t*)a.bias)[oi];
      wp[ob][i] = PROJ ? ((const acc_t*)a.WP)[oi] : (acc_t)0;
    }
  }
  accv_t G2[MB][NOB];
#pragma unroll
  for (int jb = 0; jb < MB; ++jb)
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) G2[jb][ob] = accv_t{0, 0, 0, 0};
  // bfloat16: a wave that holds every segment of its row (spw >= S) adds the
  // segment partials itself, from zero and in segment order as the x
  // transform would, and writes the one sum (the x transform then reads a
  // single segment): half the partial-spectrum traffic, the same bits
  const bool whole = PREC == PBF && ngrp == 1 && a.S > 1;
  accv_t Gs[PREC == PBF ? MB : 1][NOB];

  const in_t* T = (const in_t*)a.T;
  const in_t* TT = (const in_t*)a.TT;
  const in_t* act_in = (const in_t*)sd.act + (size_t)a.slot_in * sd.act_stride + (size_t)x * N * C;
  in_t* act_out = (in_t*)sd.act + (size_t)a.slot_out * sd.act_stride + (size_t)x * N * C;
  const double inv_s = snorm > 0.0 ? 1.0 / snorm : 0.0;
  const double h = 1.0 / (double)(N + 1);
  const double bP = PROJ ? *a.bP : 0.0;

  // Lane-constant parts of every per-tile address; a tile adds the uniform
  // offset of its first point y0.
  // A operands of GEMM1 and GEMM2 (bfloat16: this lane's fragments, KT of
  // each per tile, contiguous; tile t's start at 16 t MP)
  const in_t* Tl = KPL == 4 ? T + lane * KT * 4 : T + n16 * MP + g * KPL;
  const in_t* TTl = KPL == 4 ? TT + lane * KT * 4 : TT;
  const in_t* act_l = act_in + n16 * C + g * CB;                  // this lane's input channels
  constexpr int CPR = C * (int)sizeof(in_t) / 16;                 // 16-byte chunks per point
  static_assert(16 * CPR <= 64 || (16 * CPR) % 64 == 0, "store chunks per lane");
  // Operands of one 16-point tile: A fragments (twiddles and inputs); for the
  // feature layer the raw features.  FULL: all 16 points lie inside the row.
  // GEMM2's twiddle operand is part of the prefetch too: loading it at its
  // use would make the wave wait for every older memory operation (the
  // counter drains in order), stores and prefetches included.
  constexpr int NA2 = PROJ ? 1 : (KPL == 4 ? MB : 4 * MB);
  struct TileIn {
    frag_t Af[KT + KIN];
    frag_t A2[NA2];
    double rr;
    acc_t lk;
    double sv[PROJ ? WJ : 1];   // window vectors s_k at this lane's point
  };
  using full_t = std::integral_constant<bool, true>;
  using part_t = std::integral_constant<bool, false>;
  // A operands of GEMM1 (twiddle rows and inputs, or the raw features) ...
  auto load_a = [&](int t, TileIn& ti, auto fullc) __attribute__((always_inline)) {
    constexpr bool FULL = decltype(fullc)::value;
    const int y0 = t * 16;
    const int ya = y0 + n16;
    const bool va = FULL || ya < N;
    if constexpr (KPL == 4) {
      const in_t* tp = Tl + y0 * MP;
      if constexpr (KT % 2 == 0) {
#pragma unroll
        for (int ks = 0; ks < KT; ks += 2) {
          const short8_t v = *(const short8_t*)(tp + ks * 4);
          ti.Af[ks] = short4_t{v[0], v[1], v[2], v[3]};
          ti.Af[ks + 1] = short4_t{v[4], v[5], v[6], v[7]};
        }
      } else {
#pragma unroll
        for (int ks = 0; ks < KT; ++ks) ti.Af[ks] = M_::ld(tp + ks * 4);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < KT; ++ks) ti.Af[ks] = M_::ld(Tl + y0 * MP + ks * KSTEP);
    }
    if constexpr (FEAT) {
      ti.rr = va ? sd.r[(size_t)x * N + ya] : 0.0;
      ti.lk = va ? M_::up(((const in_t*)sd.logk)[(size_t)x * N + ya]) : (acc_t)0;
    } else {
      typedef typename Vec<in_t, CB>::type vec_t;
      vec_t vv = {};
      if (va) vv = *(const vec_t*)(act_l + y0 * C);
#pragma unroll
      for (int ks = 0; ks < KIN; ++ks) {
        if constexpr (KPL == 4) {
          ti.Af[KT + ks] = short4_t{(short)vv[ks * 4 + 0], (short)vv[ks * 4 + 1], (short)vv[ks * 4 + 2],
                                    (short)vv[ks * 4 + 3]};
        } else {
          ti.Af[KT + ks] = vv[ks];
        }
      }
    }
  };
  // ... and the twiddle operand of GEMM2
  auto load_b = [&](int t, TileIn& ti) __attribute__((always_inline)) {
    const int y0 = t * 16;
    // the window vectors at this lane's point (projection layer): refilled
    // with GEMM2's operand, after the epilogue that reads them
    if constexpr (PROJ) {
      if (wd) {
        const int yc = min(y0 + n16, N - 1);
#pragma unroll
        for (int j = 0; j < WJ; ++j) ti.sv[j] = g + 4 * j < wm ? svp[j][yc] : 0.0;
      }
    }
    if constexpr (!PROJ) {
      if constexpr (KPL == 4) {
        const in_t* tp = TTl + y0 * MP;
        if constexpr (MB % 2 == 0) {
#pragma unroll
          for (int jb = 0; jb < MB; jb += 2) {
            const short8_t v = *(const short8_t*)(tp + jb * 4);
            ti.A2[jb] = short4_t{v[0], v[1], v[2], v[3]};
            ti.A2[jb + 1] = short4_t{v[4], v[5], v[6], v[7]};
          }
        } else {
#pragma unroll
          for (int jb = 0; jb < MB; ++jb) ti.A2[jb] = M_::ld(tp + jb * 4);
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int jb = 0; jb < MB; ++jb) ti.A2[i * MB + jb] = T[(y0 + M_::row(g, i)) * MP + jb * 16 + n16];
      }
    }
  };
  // One 16-point tile: GEMM1, GELU, store, GEMM2 (or the projection).  With
  // RELOAD, each operand set of the slot is refilled with tile tn's right
  // after its last use, into the same registers: a refill issued before that
  // use would need a second register set and a copy of the in-flight load,
  // and the copy waits for it (and, the counter draining in order, for every
  // memory operation issued before it).
  auto process = [&](int t, TileIn& cur, int tn, auto fullc, auto reloadc) __attribute__((always_inline)) {
    constexpr bool FULL = decltype(fullc)::value;
    constexpr bool RELOAD = decltype(reloadc)::value;
    const int y0 = t * 16;
    const int ya = y0 + n16;
    const bool va = FULL || ya < N;
    frag_t Af[KT + KIN];
#pragma unroll
    for (int ks = 0; ks < KT + KIN; ++ks) Af[ks] = cur.Af[ks];
    if constexpr (FEAT) {
      acc_t f0 = 0, f1 = 0, f2 = 0, f3 = 0;
      if (va) {
        f0 = (acc_t)(cur.rr * inv_s);
        f1 = cur.lk;
        f2 = (acc_t)((double)(x + 1) * h);
        f3 = (acc_t)((double)(ya + 1) * h);
      }
      if constexpr (KPL == 4) {
        Af[KT] = (g == 0) ? short4_t{(short)f2bf(f0), (short)f2bf(f1), (short)f2bf(f2), (short)f2bf(f3)}
                          : M_::zero();
      } else {
        const acc_t fv = g == 0 ? f0 : (g == 1 ? f1 : (g == 2 ? f2 : f3));
        Af[KT] = (frag_t)fv;
      }
    }
    accv_t acc[NOB];
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) {
      acc[ob] = accv_t{bias[ob][0], bias[ob][1], bias[ob][2], bias[ob][3]};
      // twiddle columns past 2M are zero in T and Hc, so every K-step runs.
      // The projection layer swaps the operands: the A-operand layout of
      // [T | v] is the B-operand layout of its transpose, so z^T comes out
      // with the point along the lane and its channels along the items.
#pragma unroll
      for (int ks = 0; ks < KT + KIN; ++ks)
        acc[ob] = PROJ ? M_::mma(Bf[ks][ob], Af[ks], acc[ob]) : M_::mma(Af[ks], Bf[ks][ob], acc[ob]);
    }
    if constexpr (RELOAD) load_a(tn, cur, full_t{});
    // lane holds z[y0 + row(g, i)][ob*16 + n16] (projection: z[y0 + n16][ob*16 + row(g, i)])
    if (a.zout) {
      // training: keep the pre-activation (same LDS transpose as the activations)
      in_t* ot = otile[threadIdx.x >> 6];
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if constexpr (PROJ) ot[n16 * (C + PADE) + ob * 16 + M_::row(g, i)] = M_::cvt(acc[ob][i]);
          else ot[M_::row(g, i) * (C + PADE) + ob * 16 + n16] = M_::cvt(acc[ob][i]);
          // float32, width 16: the compiler merges these four stores into a
          // paired LDS store with a wrong offset for the second row (seen in
          // the generated assembly); a compiler barrier keeps them apart
          if constexpr (PREC == P32 && C == 16) asm volatile("" ::: "memory");
        }
      // compiler-only barrier: LDS operations of one wave complete in order,
      // so the reads below see the writes above without a wait instruction
      asm volatile("" ::: "memory");
      in_t* zo = (in_t*)a.zout + a.z_sys * blockIdx.y + (size_t)x * N * C;
      for (int q = lane; q < 16 * CPR; q += 64) {
        const int pt = q / CPR, ch = q - pt * CPR;
        if (FULL || y0 + pt < N) {
          const uint4 val = *(const uint4*)((const char*)ot + pt * (C + PADE) * sizeof(in_t) + ch * 16);
          *(uint4*)((char*)zo + ((size_t)(y0 + pt) * C) * sizeof(in_t) + ch * 16) = val;
        }
      }
      asm volatile("" ::: "memory");
    }
    if constexpr (PROJ) {
      // w[y] = sum_o W_P[o] GELU(z[y][o]): this lane's channels, then the
      // four lane groups of point y0 + n16
      acc_t part = 0;
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) part += wp[ob][i] * act<PREC>(acc[ob][i]);
      part += __shfl_xor(part, 16, 64);
      part += __shfl_xor(part, 32, 64);
      const double wv = snorm * ((double)part + bP);
      if (g == 0 && va) sd.w[(size_t)x * N + ya] = wv;
      if (wd && va) {
#pragma unroll
        for (int j = 0; j < WJ; ++j)
          if (g + 4 * j < wm) wacc[j] += wv * cur.sv[j];
      }
      if constexpr (RELOAD) load_b(tn, cur);
    } else {
      // v' = GELU(z) rounded once to the op precision; rows past N are zero
      in_t hv[NOB][4];
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const acc_t gv = act<PREC>(acc[ob][i]);
          hv[ob][i] = M_::cvt((FULL || y0 + M_::row(g, i) < N) ? gv : (acc_t)0);
        }
      // transpose the 16 x C tile through LDS, then 16-byte coalesced stores
      in_t* ot = otile[threadIdx.x >> 6];
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) ot[M_::row(g, i) * (C + PADE) + ob * 16 + n16] = hv[ob][i];
      // compiler-only barrier: LDS operations of one wave complete in order,
      // so the reads below see the writes above without a wait instruction
      asm volatile("" ::: "memory");
#pragma unroll
      for (int q0 = 0; q0 < 16 * CPR; q0 += 64) {
        const int q = q0 + lane;
        const int pt = q / CPR, ch = q - pt * CPR;
        if ((16 * CPR) % 64 == 0 || q < 16 * CPR) {
          if (FULL || y0 + pt < N) {
            const uint4 val = *(const uint4*)((const char*)ot + pt * (C + PADE) * sizeof(in_t) + ch * 16);
            *(uint4*)((char*)(act_out + (size_t)y0 * C) + pt * C * sizeof(in_t) + ch * 16) = val;
          }
        }
      }
      // next layer's y-direction analysis: G2[j][o] += sum_y T[y][j] v'[y][o]
      if constexpr (KPL == 4) {
#pragma unroll
        for (int jb = 0; jb < MB; ++jb) {
          const frag_t A2 = cur.A2[jb];
#pragma unroll
          for (int ob = 0; ob < NOB; ++ob) {
            const frag_t B2 = short4_t{(short)hv[ob][0], (short)hv[ob][1], (short)hv[ob][2], (short)hv[ob][3]};
            G2[jb][ob] = M_::mma(A2, B2, G2[jb][ob]);
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
          for (int jb = 0; jb < MB; ++jb) {
            const frag_t A2 = cur.A2[i * MB + jb];
#pragma unroll
            for (int ob = 0; ob < NOB; ++ob) G2[jb][ob] = M_::mma(A2, (frag_t)hv[ob][i], G2[jb][ob]);
          }
        }
      }
      if constexpr (RELOAD) load_b(tn, cur);
    }
  };
  // Tiles t0 .. tf-1 hold 16 points each; at most one partial tile (the
  // row's last, when 16 does not divide N) follows.  Full tiles rotate
  // through DEPTH register sets, each refilled, after its use, with the tile
  // DEPTH places later: four for the inner bfloat16 layer, two elsewhere.
  constexpr int DEPTH = (PREC == PBF && !FEAT && !PROJ) ? 4 : 2;
  // the wave's tiles T0 .. T1-1 run through one ring across its segments; at
  // the end of each segment its partial spectrum is written and restarted
  const int T0 = sg0 * TPW, T1 = min(nyt, sg1 * TPW);
  const int tf = min(T1, N >> 4);
  static_assert(TPW % DEPTH == 0, "segments must hold whole ring passes");
  auto seg_done = [&](int t) __attribute__((always_inline)) {
    if constexpr (PROJ) {
      if (wd && ((t + 1) % TPW == 0 || t + 1 == T1)) {
        // this segment's window sums over the 16 points of each lane group
        // (a fixed order), added to the wave's from zero in segment order
        const bool first = t / TPW == sg0;
#pragma unroll
        for (int j = 0; j < WJ; ++j) {
          double v = wacc[j];
          v += __shfl_xor(v, 1, 64);
          v += __shfl_xor(v, 2, 64);
          v += __shfl_xor(v, 4, 64);
          v += __shfl_xor(v, 8, 64);
          wrow[j] = (first ? 0.0 : wrow[j]) + v;
          wacc[j] = 0.0;
        }
      }
    } else {
      if ((t + 1) % TPW == 0 || t + 1 == T1) {
        if constexpr (PREC == PBF) {
          const int seg = t / TPW;
          if (whole) {
#pragma unroll
            for (int jb = 0; jb < MB; ++jb)
#pragma unroll
              for (int ob = 0; ob < NOB; ++ob) {
                Gs[jb][ob] = (seg == 0 ? accv_t{0, 0, 0, 0} : Gs[jb][ob]) + G2[jb][ob];
                G2[jb][ob] = accv_t{0, 0, 0, 0};
              }
            if (t + 1 != T1) return;
          }
          // lane holds j = 16 jb + 4 g + i, i.e. mode 8 jb + 2 g + i / 2, part i % 2
          float* Gp = (float*)sd.Gp;
#pragma unroll
          for (int jb = 0; jb < MB; ++jb)
#pragma unroll
            for (int ob = 0; ob < NOB; ++ob) {
              const accv_t v = whole ? Gs[jb][ob] : G2[jb][ob];
#pragma unroll
              for (int ip = 0; ip < 2; ++ip) {
                const int ky = 8 * jb + 2 * g + ip;
                if (2 * ky < twoM)
                  *(float2*)(Gp + gp_index(N, whole ? 1 : a.S, C, ky, x, whole ? 0 : seg, ob * 16 + n16)) =
                      float2{v[2 * ip], v[2 * ip + 1]};
              }
              G2[jb][ob] = accv_t{0, 0, 0, 0};
            }
        } else {
          acc_t* Gp = (acc_t*)sd.Gp + (size_t)(x * a.S + t / TPW) * MP * C;
#pragma unroll
          for (int jb = 0; jb < MB; ++jb)
#pragma unroll
            for (int ob = 0; ob < NOB; ++ob) {
#pragma unroll
              for (int i = 0; i < 4; ++i) Gp[(jb * 16 + M_::row(g, i)) * C + ob * 16 + n16] = G2[jb][ob][i];
              G2[jb][ob] = accv_t{0, 0, 0, 0};
            }
        }
      }
    }
  };
  if (T0 < tf) {
    // refills past the wave's last full tile read that tile again (in
    // bounds, unused), so that no refill is conditional
    TileIn ring[DEPTH];
#pragma unroll
    for (int i = 0; i < DEPTH; ++i) {
      load_a(min(T0 + i, tf - 1), ring[i], full_t{});
      load_b(min(T0 + i, tf - 1), ring[i]);
    }
    // whole ring passes, then the wave's last few full tiles
    int t = T0;
    for (; t + DEPTH <= tf; t += DEPTH) {
#pragma unroll
      for (int i = 0; i < DEPTH; ++i) process(t + i, ring[i], min(t + i + DEPTH, tf - 1), full_t{}, std::true_type{});
      // DEPTH divides TPW and T0 is a segment start, so a segment can end
      // only after a whole ring pass (or at the wave's last full tile)
      seg_done(t + DEPTH - 1);
    }
    if (t < tf) {
#pragma unroll
      for (int i = 0; i < DEPTH - 1; ++i)
        if (t + i < tf) process(t + i, ring[i], 0, full_t{}, std::false_type{});
      seg_done(tf - 1);
    }
  }
  if (tf < T1) {
    TileIn tl;
    load_a(tf, tl, part_t{});
    load_b(tf, tl);
    process(tf, tl, 0, part_t{}, std::false_type{});
    seg_done(tf);
  }
  if constexpr (PROJ) {
    // window-sum partials: a block holds 4 / ngrp whole rows (S <= 2, so
    // ngrp is 1 or 2), i.e. spw partials of 4 / S rows.  Waves past the last
    // row have left; the barrier waits for the others only.
    __shared__ double wl[4][WJ][4];
    if (wd) {
      const int w = threadIdx.x >> 6;
      if (n16 == 0) {
#pragma unroll
        for (int j = 0; j < WJ; ++j) wl[w][j][g] = wrow[j];
      }
      __syncthreads();
      if (w == 0) {
        const int sl = lane >> 3, j = (lane >> 2) & 1, gg = lane & 3, q = gg + 4 * j;
        const int rps = 4 / a.S, xb = (int)(blockIdx.x * 4) / ngrp, rows = 4 / ngrp;
        if (sl < rows / rps && q < wm) {
          const int sidx = xb / rps + sl;
          double val = 0.0;
          for (int r = 0; r < rps; ++r) {
            const int row = sidx * rps + r;
            if (row >= N) break;
            double rv = 0.0;
            for (int gp = 0; gp < ngrp; ++gp) rv += wl[(row - xb) * ngrp + gp][j][gg];
            val += rv;
          }
          sd.part[pslot(N, q, sidx)] = val;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int PREC>
static void tables_p(const NOLaunch& L, double* E64, void* Eacc, void* T, void* TT) {
  const int n = std::max(tw_period(L.basis, L.N), round16(L.N) * L.MP);
  hipLaunchKernelGGL(k_tables<PREC>, dim3((n + 255) / 256), dim3(256), 0, L.stream, L.N, L.M, L.basis, E64, Eacc,
                     T, TT);
}

void launch_tables(const NOLaunch& L, double* E64, void* Eacc, void* T, void* TT, double* RD, void* FA, void* SA,
                   void* EX) {
  if (L.prec == P64) tables_p<P64>(L, E64, Eacc, T, TT);
  else if (L.prec == P32) tables_p<P32>(L, E64, Eacc, T, TT);
  else {
    tables_p<PBF>(L, E64, Eacc, T, TT);
    // after E64 on the same stream
    const int n = round16(L.N) * 64;
    hipLaunchKernelGGL(k_tables_bfx, dim3((n + 255) / 256), dim3(256), 0, L.stream, L.N, L.M, L.basis, E64,
                       (__bf16*)FA, (__bf16*)SA);
  }
  const int n = round16(L.N) * 32;
  hipLaunchKernelGGL(k_tables_rx, dim3((n + 255) / 256), dim3(256), 0, L.stream, L.N, L.M, L.basis, E64,
                     L.prec == PBF ? (const float*)Eacc : nullptr, RD, L.prec == PBF ? (float2*)EX : nullptr);
}

template <int PREC>
static void setup_p(const NOLaunch& L, double* scratch) {
  const int n = L.N * L.N;
  const size_t stride = (size_t)4 * L.N * L.MP;
  hipLaunchKernelGGL(k_logk<PREC>, dim3((n + 255) / 256, L.nsys), dim3(256), 0, L.stream, L.sys, L.N);
  const dim3 rg((L.N + 3) / 4, L.nsys);
  const size_t fs = (size_t)L.N * L.MP;
  hipLaunchKernelGGL(k_rowdft<1>, rg, dim3(256), 0, L.stream, L.sys, L.N, L.M, L.basis, L.tab.E64, scratch + 0 * fs, stride);
  hipLaunchKernelGGL(k_rowdft<2>, rg, dim3(256), 0, L.stream, L.sys, L.N, L.M, L.basis, L.tab.E64, scratch + 1 * fs, stride);
  hipLaunchKernelGGL(k_rowdft<3>, rg, dim3(256), 0, L.stream, L.sys, L.N, L.M, L.basis, L.tab.E64, scratch + 2 * fs, stride);
  hipLaunchKernelGGL(k_rowdft<4>, rg, dim3(256), 0, L.stream, L.sys, L.N, L.M, L.basis, L.tab.E64, scratch + 3 * fs, stride);
  hipLaunchKernelGGL(k_vconst<PREC>, dim3(L.M, L.nsys), dim3(256), 0, L.stream, L.sys, L.N, L.M, L.C, L.basis,
                     L.tab.E64, scratch, stride, L.WL, L.bL);
}

void launch_no_setup(const NOLaunch& L, double* scratch) {
  if (L.prec == P64) setup_p<P64>(L, scratch);
  else if (L.prec == P32) setup_p<P32>(L, scratch);
  else setup_p<PBF>(L, scratch);
}

// With the layer family's timing on, the launch carries its own event pair
// (hipExtLaunchKernelGGL) rather than events recorded around it.
template <int PREC, int C, int MP, bool FEAT, bool PROJ>
static void layer_launch(const NOLaunch& L, const LayerArgs& la, int pk) {
  const dim3 grid((L.N * ((L.S + L.spw - 1) / L.spw) + 3) / 4, L.nsys);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof_kernel_events(pk, &e0, &e1)) {
    hipExtLaunchKernelGGL((k_layer<PREC, C, MP, FEAT, PROJ>), grid, dim3(256), 0, L.stream, e0, e1, 0, la);
    prof_kernel_done(pk, e0, e1);
  } else {
    hipLaunchKernelGGL((k_layer<PREC, C, MP, FEAT, PROJ>), grid, dim3(256), 0, L.stream, la);
  }
}

template <int PREC, int C, int MP>
static void layer_dispatch(const NOLaunch& L, const LayerArgs& la, bool feat, bool proj) {
  const int pk = feat ? PK_LAYER_FEAT : (proj ? PK_LAYER_PROJ : PK_LAYER);
  if (feat && proj) layer_launch<PREC, C, MP, true, true>(L, la, pk);
  else if (feat) layer_launch<PREC, C, MP, true, false>(L, la, pk);
  else if (proj) layer_launch<PREC, C, MP, false, true>(L, la, pk);
  else layer_launch<PREC, C, MP, false, false>(L, la, pk);
}

template <int PREC, int C>
static void spec_fwd_pc(const NOLaunch& L, const SpecArgs& sa) {
  hipLaunchKernelGGL((k_spec_fwd<PREC, C>), dim3(L.M, sa.XS, L.nsys), dim3(256), 0, L.stream, sa);
}
template <int PREC, int C>
static void spec_inv_pc(const NOLaunch& L, const SpecArgs& sa) {
  constexpr int SR = SynthRows<PREC>::SR;
  if (L.MP == 16)
    hipLaunchKernelGGL((k_spec_inv<PREC, C, 16>), dim3((L.N + SR - 1) / SR, L.nsys), dim3(synth_threads(C, L.M)), 0,
                       L.stream, sa);
  else
    hipLaunchKernelGGL((k_spec_inv<PREC, C, 32>), dim3((L.N + SR - 1) / SR, L.nsys), dim3(synth_threads(C, L.M)), 0,
                       L.stream, sa);
}

void launch_spec_fwd(const NOLaunch& L, const SpecArgs& a) {
  if (L.prec == P64) { if (L.C == 16) spec_fwd_pc<P64, 16>(L, a); else spec_fwd_pc<P64, 32>(L, a); }
  else if (L.prec == P32) { if (L.C == 16) spec_fwd_pc<P32, 16>(L, a); else spec_fwd_pc<P32, 32>(L, a); }
  else { if (L.C == 16) spec_fwd_pc<PBF, 16>(L, a); else spec_fwd_pc<PBF, 32>(L, a); }
}
void launch_spec_inv(const NOLaunch& L, const SpecArgs& a) {
  if (L.prec == P64) { if (L.C == 16) spec_inv_pc<P64, 16>(L, a); else spec_inv_pc<P64, 32>(L, a); }
  else if (L.prec == P32) { if (L.C == 16) spec_inv_pc<P32, 16>(L, a); else spec_inv_pc<P32, 32>(L, a); }
  else { if (L.C == 16) spec_inv_pc<PBF, 16>(L, a); else spec_inv_pc<PBF, 32>(L, a); }
}

template <int PREC, int C>
static void apply_pc(const NOLaunch& L) {
  {
    ProfScope ps(PK_ROWDFT, L.stream);
    hipLaunchKernelGGL(k_rowdft_r, dim3((L.N + 15) / 16, L.nsys), dim3(64 * RD_WAVES), 0, L.stream, L.sys, L.N, L.M,
                       L.tab.RD);
  }
  for (int l = 0; l < L.L; ++l) {
    const int XS = (L.N + SX - 1) / SX;
    SpecArgs sa{L.sys, L.N, L.S, L.M, l == 0 ? 1 : 0, XS, L.nsys, L.tab.Eacc, L.tab.E64, L.Rmix[l], L.WL0,
                L.vsave ? (char*)L.vsave + L.vs_layer * l * L.acc_bytes : nullptr, L.vs_sys, 0, L.basis,
                L.tab.EX};
    if constexpr (PREC == PBF) {
      // matrix-core x transforms (inference only: training runs FP32/FP64).
      // With spw >= S the layer kernel wrote each row's segment partials
      // already summed, as one segment.
      ProfScope ps(PK_SPECTRAL, L.stream);
      const int Sx = L.spw >= L.S ? 1 : L.S;
      sa.S = Sx;
      const int nkt = (2 * L.M + 15) / 16;
      const __bf16* FA = (const __bf16*)L.tab.FA;
      auto xfm = [&](auto segc, auto kgnc) {
        constexpr int SEG = decltype(segc)::value, KGN = decltype(kgnc)::value;
        hipLaunchKernelGGL((k_xfm_bf<C, SEG, KGN>), dim3(L.M, nkt / KGN, L.nsys), dim3(XFM_THREADS), 0, L.stream, sa,
                           FA);
      };
      using I1 = std::integral_constant<int, 1>;
      using I2 = std::integral_constant<int, 2>;
      // both mode groups per block once one group per block would need more
      // blocks than the chip has compute units (measured at 512^2, M = 12:
      // one group is faster up to 10 systems, two from 12 on); the first
      // layer transforms r's row spectrum and always takes one group
      if (Sx == 1 && nkt == 2 && l > 0 && L.spw > 1 && L.nsys * L.M * nkt > XFM_CUS) xfm(I1{}, I2{});
      else if (Sx == 1) xfm(I1{}, I1{});
      else if (Sx == 2) xfm(I2{}, I1{});
      else if (Sx == 4) xfm(std::integral_constant<int, 4>{}, I1{});
      else xfm(std::integral_constant<int, 0>{}, I1{});
      // output-channel groups per 16 rows: halves when the column tiles split
      // evenly, then quarters and eighths while the blocks stay within four
      // per compute unit (measured at 512^2, M = 12: eighths are fastest for
      // one to three systems, quarters for six, halves from 16 on)
      const int ntile = C * L.M / 16;
      int halves = ntile % 2 == 0 ? 2 : 1;
      while (halves < 8 && ntile % (2 * halves) == 0 && C % (2 * halves) == 0 &&
             (long)(round16(L.N) / 16) * 2 * halves * L.nsys <= 4 * XFM_CUS)
        halves *= 2;
      // column tiles per wave (four waves), rounded up to a power of two
      const int tpw = (ntile / halves + 3) / 4;
      const dim3 xg(round16(L.N) / 16, halves, L.nsys);
      auto xinv = [&](auto mpc) {
        constexpr int MPC = decltype(mpc)::value;
        if (tpw <= 1) hipLaunchKernelGGL((k_xinv_bf<C, MPC, 1>), xg, dim3(256), 0, L.stream, sa, (const __bf16*)L.tab.SA);
        else if (tpw <= 2) hipLaunchKernelGGL((k_xinv_bf<C, MPC, 2>), xg, dim3(256), 0, L.stream, sa, (const __bf16*)L.tab.SA);
        else if (tpw <= 4) hipLaunchKernelGGL((k_xinv_bf<C, MPC, 4>), xg, dim3(256), 0, L.stream, sa, (const __bf16*)L.tab.SA);
        else hipLaunchKernelGGL((k_xinv_bf<C, MPC, 8>), xg, dim3(256), 0, L.stream, sa, (const __bf16*)L.tab.SA);
      };
      if (L.MP == 16) xinv(std::integral_constant<int, 16>{});
      else xinv(std::integral_constant<int, 32>{});
    } else {
      ProfScope ps(PK_SPECTRAL, L.stream);
      constexpr int SR = SynthRows<PREC>::SR;
      hipLaunchKernelGGL((k_spec_fwd<PREC, C>), dim3(L.M, XS, L.nsys), dim3(256), 0, L.stream, sa);
      hipLaunchKernelGGL((k_spec_mix<PREC, C>), dim3(L.M, (2 * L.M + 256 / C - 1) / (256 / C), L.nsys), dim3(256), 0,
                         L.stream, sa);
      if (L.MP == 16)
        hipLaunchKernelGGL((k_spec_inv<PREC, C, 16>), dim3((L.N + SR - 1) / SR, L.nsys), dim3(synth_threads(C, L.M)), 0,
                       L.stream, sa);
      else
        hipLaunchKernelGGL((k_spec_inv<PREC, C, 32>), dim3((L.N + SR - 1) / SR, L.nsys), dim3(synth_threads(C, L.M)), 0,
                       L.stream, sa);
    }
    // inference updates the activation in place (slot 0); training keeps
    // v_{l+1} in slot l so the backward pass can read every layer's input
    const int sin = L.zsave ? (l > 0 ? l - 1 : 0) : 0, sout = L.zsave ? l : 0;
    LayerArgs la{L.sys, L.N, L.S, 2 * L.M, sin, sout, L.tab.T, L.tab.TT, L.Wfrag[l], L.bias[l], L.WP, L.bP,
                 L.zsave ? (char*)L.zsave + L.z_layer * l * L.op_bytes : nullptr, L.z_sys, L.spw};
    const bool feat = l == 0, proj = l == L.L - 1;
    la.wdots = proj ? L.wdots : 0;
    if (L.MP == 16) layer_dispatch<PREC, C, 16>(L, la, feat, proj);
    else layer_dispatch<PREC, C, 32>(L, la, feat, proj);
  }
}

void launch_no_apply(const NOLaunch& L) {
  if (L.prec == P64) { if (L.C == 16) apply_pc<P64, 16>(L); else apply_pc<P64, 32>(L); }
  else if (L.prec == P32) { if (L.C == 16) apply_pc<P32, 16>(L); else apply_pc<P32, 32>(L); }
  else { if (L.C == 16) apply_pc<PBF, 16>(L); else apply_pc<PBF, 32>(L); }
}

}  // namespace fcgno
