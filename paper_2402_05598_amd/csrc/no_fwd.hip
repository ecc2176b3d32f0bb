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

#include "common.h"

namespace fcgno {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));

template <int PREC> struct Mf;

template <> struct Mf<P64> {
  using in_t = double;
  using acc_t = double;
  using frag_t = double;
  using accv_t = double4_t;
  static constexpr int KPL = 1;
  // accumulator item i of lane (n, g) holds row 4*i + g (rows interleaved)
  static __device__ __forceinline__ int row(int g, int i) { return 4 * i + g; }
  static __device__ __forceinline__ accv_t mma(frag_t a, frag_t b, accv_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ in_t cvt(acc_t v) { return v; }
  static __device__ __forceinline__ acc_t up(in_t v) { return v; }
  static __device__ __forceinline__ frag_t ld(const in_t* p) { return *p; }
  static __device__ __forceinline__ frag_t zero() { return 0.0; }
};

template <> struct Mf<P32> {
  using in_t = float;
  using acc_t = float;
  using frag_t = float;
  using accv_t = float4_t;
  static constexpr int KPL = 1;
  // accumulator item i of lane (n, g) holds row 4*g + i
  static __device__ __forceinline__ int row(int g, int i) { return 4 * g + i; }
  static __device__ __forceinline__ accv_t mma(frag_t a, frag_t b, accv_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ in_t cvt(acc_t v) { return v; }
  static __device__ __forceinline__ acc_t up(in_t v) { return v; }
  static __device__ __forceinline__ frag_t ld(const in_t* p) { return *p; }
  static __device__ __forceinline__ frag_t zero() { return 0.0f; }
};

template <> struct Mf<PBF> {
  using in_t = uint16_t;
  using acc_t = float;
  using frag_t = short4_t;
  using accv_t = float4_t;
  static constexpr int KPL = 4;
  // accumulator item i of lane (n, g) holds row 4*g + i
  static __device__ __forceinline__ int row(int g, int i) { return 4 * g + i; }
  static __device__ __forceinline__ accv_t mma(frag_t a, frag_t b, accv_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ in_t cvt(acc_t v) { return f2bf(v); }
  static __device__ __forceinline__ acc_t up(in_t v) { return bf2f(v); }
  static __device__ __forceinline__ frag_t ld(const in_t* p) { return *(const short4_t*)p; }
  static __device__ __forceinline__ frag_t zero() { return short4_t{0, 0, 0, 0}; }
};

__host__ __device__ inline int round16(int v) { return (v + 15) & ~15; }

// ---------------------------------------------------------------------------
// Tables: E64/Eacc[m] = (cos, sin)(2 pi m / N); T[y][2q], T[y][2q+1] = cos, sin
// of 2 pi q y / N for q < M, zero elsewhere (and for y >= N); TT = T^T.
// ---------------------------------------------------------------------------
template <int PREC>
__global__ void k_tables(int N, int M, double* E64, void* Eacc, void* T, void* TT) {
  using M_ = Mf<PREC>;
  using in_t = typename M_::in_t;
  using acc_t = typename M_::acc_t;
  const int MP = round16(2 * M), NP = round16(N);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) {
    double s, c;
    sincospi(2.0 * (double)t / (double)N, &s, &c);
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
      const int m = (int)(((long long)q * y) % N);
      double s, c;
      sincospi(2.0 * (double)m / (double)N, &s, &c);
      v = (k & 1) ? s : c;
    }
    ((in_t*)T)[y * MP + k] = M_::cvt((acc_t)v);
    ((in_t*)TT)[k * NP + y] = M_::cvt((acc_t)v);
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

// y-direction DFT of one row, float64: out[j] = sum_y field(y) T64[j](y) for
// j < 2M, one wave per row.  FIELD 0: r.  FIELD 1..4: log k, x1, x2, 1.
template <int FIELD>
__device__ __forceinline__ double row_field(const SysDev& sd, int N, int x, int y) {
  if (FIELD == 0) return sd.r[x * N + y];
  if (FIELD == 1) return log(sd.k[(x + 1) * (N + 2) + y + 1]);
  if (FIELD == 2) return (double)(x + 1) / (double)(N + 1);
  if (FIELD == 3) return (double)(y + 1) / (double)(N + 1);
  return 1.0;
}

template <int FIELD>
__global__ __launch_bounds__(256) void k_rowdft(const SysDev* sys, int N, int M, const double* E64,
                                               double* out_base, size_t out_sys_stride) {
  const SysDev sd = sys[blockIdx.y];
  if (FIELD == 0 && !sd.st->active) return;
  const int x = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (x >= N) return;
  const int lane = threadIdx.x & 63;
  const int MP = round16(2 * M);
  double acc[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) acc[q] = 0.0;
  for (int y = lane; y < N; y += 64) {
    const double v = row_field<FIELD>(sd, N, x, y);
    int idx = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (q < M) {
        acc[2 * q] += v * E64[2 * idx];
        acc[2 * q + 1] += v * E64[2 * idx + 1];
        idx += y;
        if (idx >= N) idx -= N;
      }
    }
  }
  double* out = (FIELD == 0 ? sd.Gr : out_base + out_sys_stride * blockIdx.y) + (size_t)x * MP;
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    if (q < 2 * M) {
      const double s = wave_sum(acc[q]);
      if (lane == 0) out[q] = s;
    }
  }
}

// Per-solve constant part of the layer-0 spectrum:
// Vc[c][a][ky] = sum_{f=1..3} W_L[c][f] DFT(phi_f) + b_L[c] DFT(1).
template <int PREC>
__global__ __launch_bounds__(256) void k_vconst(const SysDev* sys, int N, int M, int C, const double* E64,
                                               const double* Gf, size_t gf_sys_stride,
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
    const int kv = a < M ? a : N - twoM + a;
    double sr = 0.0, si = 0.0;
    int idx = (int)(((long long)kv * lane) % N);
    const int step = (int)(((long long)kv * 64) % N);
    for (int x = lane; x < N; x += 64) {
      const double gc = G[((size_t)f * N + x) * MP + 2 * ky];
      const double gs = G[((size_t)f * N + x) * MP + 2 * ky + 1];
      const double c = E64[2 * idx], s = E64[2 * idx + 1];
      sr += gc * c - gs * s;
      si -= gc * s + gs * c;
      idx += step;
      if (idx >= N) idx -= N;
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
// Spectral part of one layer for one ky.
// ---------------------------------------------------------------------------
struct SpecArgs {
  const SysDev* sys;
  int N, S, M, layer0;
  const void* Eacc;
  const double* E64;
  const void* R;     // [M][2M][C][C] complex, accumulate precision
  const void* WL0;   // [C] accumulate precision
};

template <int PREC, int C>
__global__ __launch_bounds__(256) void k_spectral(SpecArgs a) {
  using M_ = Mf<PREC>;
  using in_t = typename M_::in_t;
  using acc_t = typename M_::acc_t;
  __shared__ acc_t Vr[C][33], Vi[C][33], Wr[C][33], Wi[C][33];
  __shared__ double Rr[32], Ri[32];
  const int ky = blockIdx.x;
  const SysDev sd = a.sys[blockIdx.y];
  if (!sd.st->active) return;
  const int N = a.N, M = a.M, twoM = 2 * M, MP = round16(twoM);
  const acc_t* E = (const acc_t*)a.Eacc;
  if (a.layer0) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int kx = wv; kx < twoM; kx += 4) {
      const int kv = kx < M ? kx : N - twoM + kx;
      double sr = 0.0, si = 0.0;
      int idx = (int)(((long long)kv * lane) % N);
      const int step = (int)(((long long)kv * 64) % N);
      for (int x = lane; x < N; x += 64) {
        const double gc = sd.Gr[(size_t)x * MP + 2 * ky], gs = sd.Gr[(size_t)x * MP + 2 * ky + 1];
        const double c = a.E64[2 * idx], s = a.E64[2 * idx + 1];
        sr += gc * c - gs * s;
        si -= gc * s + gs * c;
        idx += step;
        if (idx >= N) idx -= N;
      }
      sr = wave_sum(sr);
      si = wave_sum(si);
      if (lane == 0) {
        Rr[kx] = sr;
        Ri[kx] = si;
      }
    }
    __syncthreads();
    const double snorm = sd.st->snorm;
    const double inv_s = snorm > 0.0 ? 1.0 / snorm : 0.0;
    for (int t = threadIdx.x; t < C * twoM; t += 256) {
      const int c = t / twoM, kx = t - c * twoM;
      const double wl = (double)((const acc_t*)a.WL0)[c] * inv_s;
      const acc_t* vc = (const acc_t*)sd.Vc + 2 * ((size_t)(c * twoM + kx) * M + ky);
      Vr[c][kx] = (acc_t)(wl * Rr[kx]) + vc[0];
      Vi[c][kx] = (acc_t)(wl * Ri[kx]) + vc[1];
    }
  } else {
    const acc_t* Gp = (const acc_t*)sd.Gp;
    for (int t = threadIdx.x; t < C * twoM; t += 256) {
      const int c = t % C, kx = t / C;
      const int kv = kx < M ? kx : N - twoM + kx;
      acc_t sr = 0, si = 0;
      int idx = 0;
      for (int x = 0; x < N; ++x) {
        acc_t gc = 0, gs = 0;
        for (int sg = 0; sg < a.S; ++sg) {
          const acc_t* row = Gp + (size_t)(x * a.S + sg) * MP * C;
          gc += row[(2 * ky) * C + c];
          gs += row[(2 * ky + 1) * C + c];
        }
        const acc_t cs = E[2 * idx], sn = E[2 * idx + 1];
        sr += gc * cs - gs * sn;
        si -= gc * sn + gs * cs;
        idx += kv;
        if (idx >= N) idx -= N;
      }
      Vr[c][kx] = sr;
      Vi[c][kx] = si;
    }
  }
  __syncthreads();
  const acc_t* R = (const acc_t*)a.R + (size_t)ky * twoM * C * C * 2;
  for (int t = threadIdx.x; t < C * twoM; t += 256) {
    const int o = t % C, kx = t / C;
    const acc_t* Rk = R + (size_t)kx * C * C * 2;
    acc_t sr = 0, si = 0;
    for (int c = 0; c < C; ++c) {
      const acc_t rr = Rk[2 * (c * C + o)], ri = Rk[2 * (c * C + o) + 1];
      sr += Vr[c][kx] * rr - Vi[c][kx] * ri;
      si += Vr[c][kx] * ri + Vi[c][kx] * rr;
    }
    Wr[o][kx] = sr;
    Wi[o][kx] = si;
  }
  __syncthreads();
  const acc_t sc = (acc_t)((ky == 0 ? 1.0 : 2.0) / ((double)N * (double)N));
  in_t* Hc = (in_t*)sd.Hc;
  for (int t = threadIdx.x; t < N * C; t += 256) {
    const int x = t / C, o = t - x * C;
    acc_t hr = 0, hi = 0;
    int idx = 0;
    for (int kx = 0; kx < twoM; ++kx) {
      if (kx == M) idx = (int)(((long long)(N - M) * x) % N);
      const acc_t cs = E[2 * idx], sn = E[2 * idx + 1];
      hr += Wr[o][kx] * cs - Wi[o][kx] * sn;
      hi += Wr[o][kx] * sn + Wi[o][kx] * cs;
      idx += x;
      if (idx >= N) idx -= N;
    }
    Hc[((size_t)x * C + o) * MP + 2 * ky] = M_::cvt(sc * hr);
    Hc[((size_t)x * C + o) * MP + 2 * ky + 1] = M_::cvt(-sc * hi);
  }
}

// ---------------------------------------------------------------------------
// Layer kernel: synthesis along y + bypass + bias + GELU, then either the
// next layer's y-direction analysis or the projection.
// ---------------------------------------------------------------------------
struct LayerArgs {
  const SysDev* sys;
  int N, S, twoM, slot_in, slot_out;
  const void* T;    // [NP][MP]
  const void* TT;   // [MP][NP]
  const void* Wf;   // [C][KWP] op precision
  const void* bias; // [C] accumulate precision
  const void* WP;   // [C] accumulate precision
  double bP;
};

template <int PREC, int C, int MP, bool FEAT, bool PROJ>
__global__ __launch_bounds__(256) void k_layer(LayerArgs a) {
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
  const int lane = threadIdx.x & 63;
  const int n16 = lane & 15, g = lane >> 4;
  const SysDev sd = a.sys[blockIdx.y];
  if (!sd.st->active) return;
  const int N = a.N, NP = round16(N);
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= N * a.S) return;
  const int x = item / a.S, seg = item - x * a.S;
  const int nyt = NP >> 4;
  const int t0 = seg * TPW, t1 = min(nyt, t0 + TPW);
  const double snorm = sd.st->snorm;
  const int twoM = a.twoM;

  frag_t Bf[KT + KIN][NOB];
  const in_t* Hc = (const in_t*)sd.Hc + (size_t)x * C * MP;
  const in_t* Wf = (const in_t*)a.Wf;
  acc_t bias[NOB], wp[NOB];
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob) {
    const int o = ob * 16 + n16;
#pragma unroll
    for (int ks = 0; ks < KT; ++ks) Bf[ks][ob] = M_::ld(Hc + o * MP + ks * KSTEP + g * KPL);
#pragma unroll
    for (int ks = 0; ks < KIN; ++ks) Bf[KT + ks][ob] = M_::ld(Wf + o * KWP + ks * KSTEP + g * KPL);
    bias[ob] = ((const acc_t*)a.bias)[o];
    wp[ob] = PROJ ? ((const acc_t*)a.WP)[o] : (acc_t)0;
  }
  accv_t G2[MB][NOB];
#pragma unroll
  for (int jb = 0; jb < MB; ++jb)
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) G2[jb][ob] = accv_t{0, 0, 0, 0};

  const in_t* T = (const in_t*)a.T;
  const in_t* TT = (const in_t*)a.TT;
  const in_t* act_in = (const in_t*)sd.act + (size_t)a.slot_in * sd.act_stride + (size_t)x * N * C;
  in_t* act_out = (in_t*)sd.act + (size_t)a.slot_out * sd.act_stride + (size_t)x * N * C;
  const double inv_s = snorm > 0.0 ? 1.0 / snorm : 0.0;
  const double h = 1.0 / (double)(N + 1);

  for (int t = t0; t < t1; ++t) {
    const int y0 = t * 16;
    const int ya = y0 + n16;
    const bool va = ya < N;
    frag_t Af[KT + KIN];
#pragma unroll
    for (int ks = 0; ks < KT; ++ks) Af[ks] = M_::ld(T + ya * MP + ks * KSTEP + g * KPL);
    if constexpr (FEAT) {
      acc_t f0 = 0, f1 = 0, f2 = 0, f3 = 0;
      if (va) {
        f0 = (acc_t)(sd.r[(size_t)x * N + ya] * inv_s);
        f1 = M_::up(((const in_t*)sd.logk)[(size_t)x * N + ya]);
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
    } else {
#pragma unroll
      for (int ks = 0; ks < KIN; ++ks)
        Af[KT + ks] = va ? M_::ld(act_in + (size_t)ya * C + ks * KSTEP + g * KPL) : M_::zero();
    }
    accv_t acc[NOB];
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) {
      acc[ob] = accv_t{bias[ob], bias[ob], bias[ob], bias[ob]};
#pragma unroll
      for (int ks = 0; ks < KT; ++ks)
        if (ks * KSTEP < twoM) acc[ob] = M_::mma(Af[ks], Bf[ks][ob], acc[ob]);
#pragma unroll
      for (int ks = 0; ks < KIN; ++ks) acc[ob] = M_::mma(Af[KT + ks], Bf[KT + ks][ob], acc[ob]);
    }
    // lane holds z[y0 + row(g, i)][ob*16 + n16]
    acc_t v[NOB][4];
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int yv = y0 + M_::row(g, i);
        const acc_t gv = gelu(acc[ob][i]);
        v[ob][i] = yv < N ? (PROJ ? gv : M_::up(M_::cvt(gv))) : (acc_t)0;
      }
    if constexpr (PROJ) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc_t part = 0;
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob) part += wp[ob] * v[ob][i];
        part += __shfl_xor(part, 1, 64);
        part += __shfl_xor(part, 2, 64);
        part += __shfl_xor(part, 4, 64);
        part += __shfl_xor(part, 8, 64);
        const int yv = y0 + M_::row(g, i);
        if (n16 == i && yv < N) sd.w[(size_t)x * N + yv] = snorm * ((double)part + a.bP);
      }
    } else {
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int yv = y0 + M_::row(g, i);
          if (yv < N) act_out[(size_t)yv * C + ob * 16 + n16] = M_::cvt(v[ob][i]);
        }
      if constexpr (KPL == 4) {
        frag_t B2[NOB];
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob)
          B2[ob] = short4_t{(short)f2bf(v[ob][0]), (short)f2bf(v[ob][1]), (short)f2bf(v[ob][2]),
                            (short)f2bf(v[ob][3])};
#pragma unroll
        for (int jb = 0; jb < MB; ++jb) {
          if (jb * 16 < twoM) {
            const frag_t A2 = M_::ld(TT + (jb * 16 + n16) * NP + y0 + 4 * g);
#pragma unroll
            for (int ob = 0; ob < NOB; ++ob) G2[jb][ob] = M_::mma(A2, B2[ob], G2[jb][ob]);
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int yv = y0 + M_::row(g, i);
#pragma unroll
          for (int jb = 0; jb < MB; ++jb) {
            if (jb * 16 < twoM) {
              const frag_t A2 = T[yv * MP + jb * 16 + n16];
#pragma unroll
              for (int ob = 0; ob < NOB; ++ob) G2[jb][ob] = M_::mma(A2, (frag_t)v[ob][i], G2[jb][ob]);
            }
          }
        }
      }
    }
  }
  if constexpr (!PROJ) {
    acc_t* Gp = (acc_t*)sd.Gp + (size_t)(x * a.S + seg) * MP * C;
#pragma unroll
    for (int jb = 0; jb < MB; ++jb)
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) Gp[(jb * 16 + M_::row(g, i)) * C + ob * 16 + n16] = G2[jb][ob][i];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int PREC>
static void tables_p(const NOLaunch& L, double* E64, void* Eacc, void* T, void* TT) {
  const int n = std::max(L.N, round16(L.N) * L.MP);
  hipLaunchKernelGGL(k_tables<PREC>, dim3((n + 255) / 256), dim3(256), 0, L.stream, L.N, L.M, E64, Eacc, T, TT);
}

void launch_tables(const NOLaunch& L, double* E64, void* Eacc, void* T, void* TT) {
  if (L.prec == P64) tables_p<P64>(L, E64, Eacc, T, TT);
  else if (L.prec == P32) tables_p<P32>(L, E64, Eacc, T, TT);
  else tables_p<PBF>(L, E64, Eacc, T, TT);
}

template <int PREC>
static void setup_p(const NOLaunch& L, double* scratch) {
  const int n = L.N * L.N;
  const size_t stride = (size_t)4 * L.N * L.MP;
  hipLaunchKernelGGL(k_logk<PREC>, dim3((n + 255) / 256, L.nsys), dim3(256), 0, L.stream, L.sys, L.N);
  const dim3 rg((L.N + 3) / 4, L.nsys);
  const size_t fs = (size_t)L.N * L.MP;
  hipLaunchKernelGGL(k_rowdft<1>, rg, dim3(256), 0, L.stream, L.sys, L.N, L.M, L.tab.E64, scratch + 0 * fs, stride);
  hipLaunchKernelGGL(k_rowdft<2>, rg, dim3(256), 0, L.stream, L.sys, L.N, L.M, L.tab.E64, scratch + 1 * fs, stride);
  hipLaunchKernelGGL(k_rowdft<3>, rg, dim3(256), 0, L.stream, L.sys, L.N, L.M, L.tab.E64, scratch + 2 * fs, stride);
  hipLaunchKernelGGL(k_rowdft<4>, rg, dim3(256), 0, L.stream, L.sys, L.N, L.M, L.tab.E64, scratch + 3 * fs, stride);
  hipLaunchKernelGGL(k_vconst<PREC>, dim3(L.M, L.nsys), dim3(256), 0, L.stream, L.sys, L.N, L.M, L.C,
                     L.tab.E64, scratch, stride, L.WL, L.bL);
}

void launch_no_setup(const NOLaunch& L, double* scratch) {
  if (L.prec == P64) setup_p<P64>(L, scratch);
  else if (L.prec == P32) setup_p<P32>(L, scratch);
  else setup_p<PBF>(L, scratch);
}

template <int PREC, int C, int MP>
static void layer_dispatch(const NOLaunch& L, const LayerArgs& la, bool feat, bool proj) {
  const dim3 grid((L.N * L.S + 3) / 4, L.nsys);
  if (feat && proj) hipLaunchKernelGGL((k_layer<PREC, C, MP, true, true>), grid, dim3(256), 0, L.stream, la);
  else if (feat) hipLaunchKernelGGL((k_layer<PREC, C, MP, true, false>), grid, dim3(256), 0, L.stream, la);
  else if (proj) hipLaunchKernelGGL((k_layer<PREC, C, MP, false, true>), grid, dim3(256), 0, L.stream, la);
  else hipLaunchKernelGGL((k_layer<PREC, C, MP, false, false>), grid, dim3(256), 0, L.stream, la);
}

template <int PREC, int C>
static void apply_pc(const NOLaunch& L) {
  hipLaunchKernelGGL(k_rowdft<0>, dim3((L.N + 3) / 4, L.nsys), dim3(256), 0, L.stream, L.sys, L.N, L.M,
                     L.tab.E64, (double*)nullptr, (size_t)0);
  for (int l = 0; l < L.L; ++l) {
    SpecArgs sa{L.sys, L.N, L.S, L.M, l == 0 ? 1 : 0, L.tab.Eacc, L.tab.E64, L.Rmix[l], L.WL0};
    hipLaunchKernelGGL((k_spectral<PREC, C>), dim3(L.M, L.nsys), dim3(256), 0, L.stream, sa);
    LayerArgs la{L.sys, L.N, L.S, 2 * L.M, 0, 0, L.tab.T, L.tab.TT, L.Wfrag[l], L.bias[l], L.WP, L.bP};
    const bool feat = l == 0, proj = l == L.L - 1;
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
