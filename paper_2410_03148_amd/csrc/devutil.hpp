// Device helpers shared by the operator kernels (ops.hip, elem.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace phz {
namespace dev {

// Workgroups are handed to the eight XCDs round-robin (workgroup b runs on
// XCD b % 8), and each XCD has its own L2.  A gather whose neighbours sit in
// the neighbouring workgroups (the rows y +- 1) would therefore fetch every
// row into three L2s.  This maps the hardware workgroup id to a logical one
// so that each XCD owns one contiguous range of logical workgroups (a slab
// of whole rows and planes): a bijection on [0, nb) for any nb.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  constexpr unsigned X = 8;
  const unsigned q = nb / X, r = nb % X, x = b % X, i = b / X;
  return x * q + (x < r ? x : r) + i;
}

// y = beta*yin + alpha*acc, optional Chebyshev epilogue (FO == FI) or first
// Chebyshev step on y (a.d1), for the KK load columns k0 .. k0+KK-1 of a node
// (column (f, k) at (f*K + k)*nn)
template <typename T, int FO, int K, int KK, bool CHEBY>
__device__ __forceinline__ void epilogue_cols(unsigned n, unsigned nn, int k0, const T* acc, const OpArgs<T>& a) {
  T out[FO * KK];
  if (a.beta == T(0)) {
#pragma unroll
    for (int f = 0; f < FO; ++f)
#pragma unroll
      for (int j = 0; j < KK; ++j) out[f * KK + j] = a.alpha * acc[f * KK + j];
  } else {
#pragma unroll
    for (int f = 0; f < FO; ++f)
#pragma unroll
      for (int j = 0; j < KK; ++j)
        out[f * KK + j] = a.beta * a.yin[(size_t)(f * K + k0 + j) * nn + n] + a.alpha * acc[f * KK + j];
  }
#pragma unroll
  for (int f = 0; f < FO; ++f)
#pragma unroll
    for (int j = 0; j < KK; ++j) a.y[(size_t)(f * K + k0 + j) * nn + n] = out[f * KK + j];
  if constexpr (CHEBY) {
    const T ca = a.cab[0], cb = a.cab[1];
    T Di[FO * FO];
#pragma unroll
    for (int t = 0; t < FO * FO; ++t) Di[t] = a.dinv[(size_t)t * nn + n];
#pragma unroll
    for (int j = 0; j < KK; ++j)
#pragma unroll
      for (int f = 0; f < FO; ++f) {
        T z = T(0);
#pragma unroll
        for (int g = 0; g < FO; ++g) z += Di[f * FO + g] * out[g * KK + j];
        const size_t o = (size_t)(f * K + k0 + j) * nn + n;
        const T dold = a.dold[o];
        const T dv = ca * dold + cb * z;
        a.dnew[o] = dv;
        T xo = dv;
        if (a.fold_dold) xo += dold;
        if (a.xin) xo += a.xin[o];
        a.x[o] = xo;
      }
  } else {
    if (a.d1) {
      const T c0 = a.cab[0];
      T Di[FO * FO];
#pragma unroll
      for (int t = 0; t < FO * FO; ++t) Di[t] = a.dinv[(size_t)t * nn + n];
#pragma unroll
      for (int j = 0; j < KK; ++j)
#pragma unroll
        for (int f = 0; f < FO; ++f) {
          T z = T(0);
#pragma unroll
          for (int g = 0; g < FO; ++g) z += Di[f * FO + g] * out[g * KK + j];
          a.d1[(size_t)(f * K + k0 + j) * nn + n] = c0 * z;
        }
    }
  }
}

template <typename T, int FO, int K, bool CHEBY>
__device__ __forceinline__ void epilogue(unsigned n, unsigned nn, const T* acc, const OpArgs<T>& a) {
  epilogue_cols<T, FO, K, K, CHEBY>(n, nn, 0, acc, a);
}

// Raw buffer loads: one scalar resource per array, the column offset in a
// scalar register and the node offset in a 32-bit vector register (no
// per-load 64-bit address arithmetic).  Arrays must span < 4 GiB.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

}  // namespace dev
}  // namespace phz
