// Device helpers for the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qgt_internal.h"

namespace qgt {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// a * b
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// conj(a) * b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -a.y * b.x));
}
// acc + a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
// acc + conj(a) * b
__device__ __forceinline__ double2 cfmac(double2 a, double2 b, double2 acc) {
  return make_double2(fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y)));
}

// Native two-component vectors (the HIP double2 struct can make the compiler
// serialise independent loads) and global-address-space pointers (pointers
// read from memory would otherwise be accessed with flat instructions).
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));
#define QGT_GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ dv2 to_dv2(double2 v) { return dv2{v.x, v.y}; }
__device__ __forceinline__ double2 to_d2(dv2 v) { return make_double2(v.x, v.y); }
// acc + a * b (complex)
__device__ __forceinline__ dv2 vfma(dv2 a, dv2 b, dv2 acc) {
  return dv2{fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y))};
}
// acc + conj(a) * b
__device__ __forceinline__ dv2 vfmac(dv2 a, dv2 b, dv2 acc) {
  return dv2{fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y))};
}

// Element idx of O as complex double; DT 0 = complex64, 1 = complex128.
template <int DT>
__device__ __forceinline__ dv2 load_ov(const void* O, int64_t idx) {
  if constexpr (DT == 0) {
    const fv2 v = ((const QGT_GLOBAL fv2*)O)[idx];
    return dv2{(double)v.x, (double)v.y};
  } else {
    return ((const QGT_GLOBAL dv2*)O)[idx];
  }
}
template <int DT>
__device__ __forceinline__ double2 load_o(const void* O, int64_t idx) {
  return to_d2(load_ov<DT>(O, idx));
}

// Round a double to bfloat16, nearest-even, with a single rounding: truncate to
// float, keep a sticky bit for the discarded part (round to odd), then round
// the float to nearest-even at bfloat16 precision.  Finite inputs only.
__device__ __forceinline__ uint16_t f64_to_bf16_rne(double d) {
  float f = __double2float_rz(d);
  uint32_t u = __float_as_uint(f);
  if ((double)f != d) u |= 1u;
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

template <int PREC> struct PackT;
template <> struct PackT<PREC_FP64> { typedef double T; };
template <> struct PackT<PREC_FP32> { typedef float T; };
template <> struct PackT<PREC_BF16> { typedef uint16_t T; };

template <int PREC>
__device__ __forceinline__ typename PackT<PREC>::T to_pack(double v) {
  if constexpr (PREC == PREC_FP64) return v;
  else if constexpr (PREC == PREC_FP32) return (float)v;  // round to nearest even
  else return f64_to_bf16_rne(v);
}

// True once block B has met the CG convergence test: the remaining iterations
// skip it (its solution and last correction are kept for the final step).
__device__ __forceinline__ bool cg_done(const BlockDev& B, const char* ws) {
  return reinterpret_cast<const CgScal*>(ws + B.cg_off)->done != 0;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ const T* ws_at(const char* ws, int64_t off) { return reinterpret_cast<const T*>(ws + off); }
template <typename T>
__device__ __forceinline__ T* ws_at(char* ws, int64_t off) { return reinterpret_cast<T*>(ws + off); }

}  // namespace qgt
