// Matrix-core operand traits shared by the layer kernels and the backward:
// element types, the 16 x 16 MFMA of each precision and its accumulator
// layout.  Operand layout of every 16 x 16 x K product used here: lane
// (n, g) = 16 g + n holds A[n][k] and B[k][n] for the KPL contraction
// indices k of group g; accumulator item i of lane (n, g) holds D[row(g, i)][n].
#pragma once

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

}  // namespace fcgno
