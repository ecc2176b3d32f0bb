// Internal declarations shared by the HIP translation units of libfcgno.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fcgno {

constexpr int MAXW = 32;        // largest truncation window m_max
constexpr int NQ = MAXW + 4;    // partial-sum slots per block
constexpr int FLAT_PTS = 2048;  // points per workgroup in the flat Krylov kernels
constexpr int UPD_PTS = 512;    // points per workgroup of the update kernel (two per thread)
constexpr int TILE_I = 16;      // stencil tile rows (x1)
constexpr int TILE_J = 64;      // stencil tile columns (x2, contiguous)
constexpr int TPW = 16;         // 16-point column tiles per row segment in the layer kernel
constexpr int SPW_HIGH = 2;     // row segments per wave while many systems are active
constexpr int LOW_ACTIVE = 4;   // active systems at or below which a wave takes one segment
// row segments of the layer kernel for N points per row
__host__ __device__ inline int seg_count(int N) { return ((N + 15) / 16 + TPW - 1) / TPW; }

enum Prec { P64 = 0, P32 = 1, PBF = 2, PID = 3, PJAC = 4, PSGS = 5 };

// neural-operator precisions (the others are identity and classical sweeps)
__host__ __device__ inline bool is_no(int op) { return op == P64 || op == P32 || op == PBF; }

// Device memory reached through pointers that the kernels read from memory
// (the per-system tables) is declared in the global address space for the
// device compiler, so that accesses compile to global_* rather than flat_*
// instructions (flat accesses also count against the LDS wait counter, which
// makes every LDS wait drain outstanding memory loads).  Host code sees plain
// pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__)
#define GLOBAL __attribute__((address_space(1)))
#else
#define GLOBAL
#endif

enum SysStatus { S_OK = 0, S_NOTCONV = 1, S_BREAK = 2, S_NONFINITE = 3 };

// Scalar state of one system, resident on the device.
struct SysState {
  int i;          // next iteration index
  int active;     // 1 while iterating
  int status;     // SysStatus
  int iters;      // iteration count reported
  unsigned tick[4];
  int m;          // window size m_i of the current iteration
  int max_iter;
  int m_max;
  int pad0;
  double rr0;     // ||r_0||^2
  double rr;      // ||r_i||^2
  double alpha;
  double snorm;   // ||r_i||_2 / N, the operator's input scale
  double tres;    // ||f - A u||_2 / ||r_0||_2 (final check)
  double tresf;   // ||f - A u||_2 / ||f||_2 (final check)
  double ff;      // ||f||_2^2
  double rtol;
  double ps_ring[MAXW + 1];   // (p_k, A p_k) by ring slot k mod (m_max+1)
  double coef[MAXW];          // (w_i, s_k)/(p_k, s_k) of the current window
};

// Per-system device pointers.  All systems of one launch share N.
struct SysDev {
  const GLOBAL double* k;   // [(N+2)^2]
  const GLOBAL double* f;   // [N^2]
  GLOBAL double* u;
  GLOBAL double* r;
  GLOBAL double* w;         // == r for the identity operator
  GLOBAL double* P;         // ring [(m_max+1)][N^2]
  GLOBAL double* S;         // ring
  GLOBAL SysState* st;
  GLOBAL double* hist;      // [max_iter+1]
  GLOBAL double* part;      // [blocks][NQ]
  GLOBAL int* n_active;     // batch counter of active systems
  // operator buffers (op precision unless noted)
  GLOBAL void* act;         // [slots][N^2][C]
  size_t act_stride;        // elements per activation slot
  GLOBAL void* logk;        // [N^2]
  GLOBAL double* Gr;        // [N][MP] row DFT partials of r, float64
  GLOBAL void* Gp;          // row DFT partials of activations, accumulate precision: [N][S][MP][C]
                            // (bfloat16 operator: [M][N][S][C][2], see gp_index)
  GLOBAL void* Hc;          // [N][C][MP] synthesis rows for the layer kernel
  GLOBAL void* Vc;          // [C][2M][M] complex, accumulate precision: constant part of layer-0 spectrum
  GLOBAL void* Wh;          // [M][C][MP] complex, accumulate precision: mixed spectrum of the current layer (zero past 2M)
  GLOBAL void* Vp;          // [M][XS][C][2M] complex, accumulate precision: per-chunk forward spectra
  GLOBAL double* tmp;       // [N^2] second iterate of the Jacobi sweeps
  GLOBAL void* WT;          // bfloat16 operator: mixed spectrum as the synthesis operand,
                            // [2 (hi, lo)][C*M][64] bfloat16 (see k_xfm_bf)
  // copies of the state's active flag, iteration index and window size in
  // the launch table itself, kept by the kernels that change the state:
  // a kernel reads them with its record instead of behind the state pointer
  int active, it, mmax;
};

// Per-N tables shared by the systems of one launch.
// Spectral bases of the operator layers.
enum Basis { B_FOURIER = 0, B_SINE = 1 };

// Entries of the x-direction twiddle table: N (Fourier, angles 2 pi m / N) or
// 2N + 2 (sine, angles pi m / (N + 1)).
__host__ __device__ inline int tw_period(int basis, int N) { return basis == B_SINE ? 2 * N + 2 : N; }

// Twiddle-table index of kept x-mode a (< 2M) at row x.  Fourier: kx_a x mod N
// with kx_a = a for a < M, N - 2M + a otherwise.  Sine: (a + 1)(x + 1) mod
// (2N + 2), whose table entry holds sin(pi (a+1)(x+1)/(N+1)) in the cosine
// slot and zero in the sine slot, so that the complex transforms reduce to
// real DST-I sums.  All products stay below 2^32 for N <= 2^15.
__device__ __forceinline__ unsigned tw_index(int basis, int N, int M, int a, int x) {
  if (basis == B_SINE) return ((unsigned)(a + 1) * (unsigned)(x + 1)) % (unsigned)(2 * N + 2);
  const int kv = a < M ? a : N - 2 * M + a;
  return ((unsigned)kv * (unsigned)x) % (unsigned)N;
}

struct Tables {
  const double* E64;  // [tw_period] Fourier: (cos, sin)(2 pi m / N); sine: (sin(pi m/(N+1)), 0)
  const void* Eacc;   // same in accumulate precision
  const void* T;      // [N][MP] op precision: Fourier T[y][2q] = cos(2 pi q y/N), T[y][2q+1] = sin(...);
                      // sine T[y][2q] = sin(pi (q+1)(y+1)/(N+1)), T[y][2q+1] = 0
  const void* TT;     // [MP][N] transpose of T
  // bfloat16 operator only: the x-direction transforms as matrix-core
  // operands, each value split into a bfloat16 pair hi + lo
  const void* FA;     // [2][32][2 NP] forward: FA[h][a][2x] = cos, FA[h][a][2x+1] = -sin
  const void* SA;     // [2][NP][64]   synthesis: SA[h][x][2a] = cos, SA[h][x][2a+1] = -sin
  // float64 twiddles of the row transform of r, as the B operand of its
  // 16x16x4 products: RD[(s * 2 + cb) * 64 + 16 g + n] = T(4 s + g, 16 cb + n)
  // (T as above, zero for y >= N and columns >= 2M); NP / 4 steps of 4 rows
  const double* RD;
  // bfloat16 operator: the first layer's x transform, EX[x][a] = (cos, -sin)
  // of kept x-mode a at row x in float32 (zero for a >= 2M or x >= N), [NP][32]
  const void* EX;
};

__host__ __device__ inline int flat_blocks(int n) { return (n + FLAT_PTS - 1) / FLAT_PTS; }
__host__ __device__ inline int upd_blocks(int n) { return (n + UPD_PTS - 1) / UPD_PTS; }
__host__ __device__ inline int tile_blocks(int N) {
  return ((N + TILE_I - 1) / TILE_I) * ((N + TILE_J - 1) / TILE_J);
}
// Partial-sum slots of a system: slot-major, [NQ][stride], so that one slot's
// values from every writer are contiguous (the kernels that sum them in every
// block read whole lines).  stride = the most partials of any writer: blocks
// of the flat and tiled Krylov kernels (FLAT_PTS >= UPD_PTS), or the
// projection layer's window sums (one per 4/S rows).
__host__ __device__ inline int proj_wslots(int N) { return (N * seg_count(N) + 3) / 4; }
__host__ __device__ inline int pslot_stride(int N) {
  const int a = upd_blocks(N * N), b = tile_blocks(N), c = proj_wslots(N);
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}
__device__ __forceinline__ size_t pslot(int N, int q, int b) { return (size_t)q * pslot_stride(N) + b; }

__device__ __forceinline__ int window_size(int i, int m_max) {
  int r = i % (m_max + 1);
  int a = r > 1 ? r : 1;
  return i < a ? i : a;
}

// ---- deterministic reductions ------------------------------------------

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a 256-thread block in a fixed order; result valid in every thread.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* lds /* >= 4 */) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  T s = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  return s;
}

__device__ __forceinline__ void deactivate(GLOBAL SysState* st, GLOBAL int* n_active, int status, int iters,
                                           const SysDev* rec) {
  st->status = status;
  st->iters = iters;
  st->active = 0;
  ((SysDev*)rec)->active = 0;
  atomicSub(n_active, 1);
}

// ---- bfloat16 helpers ----------------------------------------------------

// float -> bfloat16 bits, round to nearest even (one hardware conversion)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
// two floats -> packed bfloat16 pair (a in the low half)
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
  bf2_t v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}

// ---- GELU ----------------------------------------------------------------

// erf(x) by Abramowitz & Stegun, Handbook of Mathematical Functions, formula
// 7.1.26: 1 - (a1 t + ... + a5 t^5) exp(-x^2), t = 1/(1 + p|x|), odd in x,
// absolute error <= 1.5e-7.  Branch-free; used by the float32 and bfloat16
// operators (below float32 resolution of GELU's output scale).
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
  float q = 1.061405429f;
  q = fmaf(q, t, -1.453152027f);
  q = fmaf(q, t, 1.421413741f);
  q = fmaf(q, t, -0.284496736f);
  q = fmaf(q, t, 0.254829592f);
  q *= t;
  const float r = 1.0f - q * __expf(-ax * ax);
  return copysignf(r, x);
}

// GELU(z) = z/2 (1 + erf(z / sqrt 2))
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f)); }
__device__ __forceinline__ double gelu(double z) { return 0.5 * z * (1.0 + erf(z * 0.70710678118654752440)); }

// GELU of the bfloat16 operator: z * sigmoid(P(z)), P(z) = z (c1 + c3 z^2 +
// c5 z^4 + c7 z^6) fitted for the smallest maximum deviation from the erf
// form on [-6, 6] (argument clamped there): |error| <= 1.3e-5 in float32,
// below the bfloat16 rounding of the result wherever |GELU(z)| > 3e-3.  Two
// transcendental and eight plain operations against twenty-odd for erf_as.
// The coefficients below are -c_k log2(e), so sigmoid(P) = 1 / (1 + 2^(poly)).
__device__ __forceinline__ float gelu_bf(float z) {
  const float zc = __builtin_amdgcn_fmed3f(z, -6.0f, 6.0f);
  const float u = zc * zc;
  float q = fmaf(u, 2.481038791302126e-05f, 7.364328484982252e-04f);
  q = fmaf(q, u, -1.0598407685756683e-01f);
  q = fmaf(q, u, -2.3016459941864014f);
  const float e = __builtin_amdgcn_exp2f(q * zc);
  return z * __builtin_amdgcn_rcpf(1.0f + e);
}

// ---- host-side launchers (defined in the .hip files) ---------------------

struct KrylovLaunch {
  const SysDev* sys;   // device table
  int nsys;
  int N;
  int m_max;
  hipStream_t stream;
  int wslots = 0;      // partial slots of the window sums (0: the window-sum kernel's)
};

void launch_init_state(const KrylovLaunch& L, int max_iter, double rtol);
void launch_residual(const KrylovLaunch& L, int mode);   // 0: r0 setup, 1: final true residual
void launch_rnorm(const KrylovLaunch& L);                 // snorm from r (operator only)
void launch_wdots(const KrylovLaunch& L);
// The projection layer forms the window sums itself (no window-sum launch)
// when the window holds at most 8 vectors (two per lane group) and a row has
// at most two segments (N <= 512), proj_wslots(N) partials.
constexpr int PROJ_WDOTS_MAX_M = 8;
inline bool proj_wdots(int N, int m_max) { return m_max <= PROJ_WDOTS_MAX_M && seg_count(N) <= 2; }
void launch_dir(const KrylovLaunch& L);
void launch_update(const KrylovLaunch& L);
// classical preconditioners: w = x_steps of Jacobi / red-black symmetric
// Gauss-Seidel on A x = r from x_0 = 0 (active systems)
void launch_jacobi(const KrylovLaunch& L, int steps);
void launch_rbsgs(const KrylovLaunch& L, int steps);
void launch_record(const KrylovLaunch& L, int it, int m, double* rec_r, double* rec_e, const double* ustar);
// flags[3b..3b+2] = {active, status, iters}; tres[2b], tres[2b+1] = true
// residual relative to ||r_0|| and to ||f||
void launch_export(const SysDev* sys, int nsys, int* flags, double* tres, hipStream_t s);
// the launch table's copies of active flag, iteration index and window size
// from each system's state (after a host upload of the table)
void launch_sync_records(const SysDev* sys, int nsys, hipStream_t s);
// out[0 .. nsys): the records of sys[0 .. nsys) whose systems are active, in
// order, then records pointing at idle (whose active flag must be zero)
void launch_compact(const SysDev* sys, int nsys, SysDev* out, SysState* idle, hipStream_t s);
void launch_zero(void* p, size_t nbytes, hipStream_t s);      // bytes [0, nbytes) = 0

struct NOLaunch {
  const SysDev* sys;
  int nsys;
  int N, C, M, MP, L;   // MP = 2M rounded up to 16
  int S;                // row segments (of TPW tiles) per row in the layer kernel
  int spw;              // row segments per wave (1 or SPW_HIGH): the results do not depend on it
  int prec;             // P64, P32, PBF
  int basis;            // B_FOURIER or B_SINE
  Tables tab;
  // model weights in the op / accumulate precisions
  const void* const* Wfrag;   // [L] op precision [C][KWP_l]
  const void* const* bias;    // [L] accumulate precision [C]
  const void* const* Rmix;    // [L] accumulate precision [M][2M][C][C] complex
  const void* WP;             // accumulate precision [C]
  const double* bP;           // float64 projection bias (device)
  const void* WL0;            // accumulate precision [C]: lift weights of the r/s feature
  const double* WL;           // float64 [C][4]
  const double* bL;           // float64 [C]
  hipStream_t stream;
  // training forward (all nullable / zero in inference)
  void* zsave;                // pre-activations, [L][sys][N^2][C] op precision
  size_t z_sys, z_layer;      // element strides
  void* vsave;                // spectra V^, [L][sys][M][C][2M] complex accumulate precision
  size_t vs_sys, vs_layer;    // element strides
  int op_bytes, acc_bytes;
  // solve: the projection layer also forms the window sums (w_i, s_k) of
  // Algorithm 1 (one partial per row segment; the window-sum kernel is skipped)
  int wdots = 0;
};

struct SpecArgs {
  const SysDev* sys;
  int N, S, M, layer0, XS;   // XS: x-chunks of 64 rows in the forward transform
  int nsys;                  // systems in the table (the mixing kernel groups them)
  const void* Eacc;
  const double* E64;
  const void* R;     // [M][2M][C][C] complex, accumulate precision
  const void* WL0;   // [C] accumulate precision
  void* Vsave;       // training: V^ of this layer, [M][2M][nsys][C] complex (nullable)
  size_t vs_sys;     // elements per system in Vsave
  int unit_scale;    // synthesis without the normalisation factor (backward pass)
  int basis;         // B_FOURIER or B_SINE (set from NOLaunch::basis)
  const void* EX = nullptr;   // bfloat16 first layer: Tables::EX
};

// FA, SA, EX: bfloat16 operator only (nullptr otherwise); RD: every operator
void launch_tables(const NOLaunch& L, double* E64, void* Eacc, void* T, void* TT, double* RD, void* FA = nullptr,
                   void* SA = nullptr, void* EX = nullptr);
// single stages of the spectral part (used by the backward pass)
void launch_spec_fwd(const NOLaunch& L, const SpecArgs& a);
void launch_spec_inv(const NOLaunch& L, const SpecArgs& a);
void launch_no_setup(const NOLaunch& L, double* scratch);   // logk, Vc
void launch_no_apply(const NOLaunch& L);                    // w = B(r) for active systems

}  // namespace fcgno
