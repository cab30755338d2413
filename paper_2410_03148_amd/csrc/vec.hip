// Vector, reduction, GMRES and per-element physics kernels (gfx950).
//
// Internal vectors are structure of arrays: column f*K + k (field f, load
// column k) holds nn contiguous node values.  Reductions are two-stage and
// deterministic: blocks of a (slice, column) grid write partial sums, then
// one block per output adds them in a fixed order.  Krylov vectors may be
// float or double; every inner product accumulates in double.
#include <algorithm>
#include <array>
#include <cmath>
#include <limits>
#include <utility>

#include "common.hpp"
#include "devutil.hpp"

namespace phz {

namespace {

inline unsigned blocks_for(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

constexpr int kMaxPartBlocks = 2048;

// slices per column so that the reduction grid has ~2048 blocks
inline unsigned slices_for(size_t nn, int ncol) {
  size_t g = kMaxPartBlocks / (size_t)ncol;
  const size_t cap = (nn + 255) / 256;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum over a 256-thread block; result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* lds4) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) lds4[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = lds4[0] + lds4[1] + lds4[2] + lds4[3];
  __syncthreads();
  return r;
}

// out[o] (o = (i - i0)*K + k) = sum_{f < F} sum_{b < G} part[((f*K + k)*G + b)*J + i];
// one block per output, fixed summation order
__global__ __launch_bounds__(256) void k_reduce_cols(int G, int F, int K, int J, int i0,
                                                     const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double lds[256];
  const int o = blockIdx.x;
  const int i = i0 + o / K, k = o % K;
  double s = 0.0;
  for (int q = threadIdx.x; q < F * G; q += 256) {
    const int f = q / G, b = q % G;
    s += part[((size_t)(f * K + k) * G + b) * J + i];
  }
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[o] = lds[0];
}

void reduce_cols(int G, int F, int K, int J, int i0, int nout_i, const double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_cols, dim3(nout_i * K), dim3(256), 0, st, G, F, K, J, i0, part, out);
}

// per-column sums (or sums of squares) of column blockIdx.y over slice blockIdx.x
template <typename T, bool SQ>
__global__ __launch_bounds__(256) void k_col_sums(unsigned nn, const T* __restrict__ v, double* __restrict__ part) {
  __shared__ double lds4[4];
  const T* col = v + (size_t)blockIdx.y * nn;
  double acc = 0.0;
  for (unsigned n = blockIdx.x * 256 + threadIdx.x; n < nn; n += gridDim.x * 256) {
    const double x = (double)col[n];
    acc += SQ ? x * x : x;
  }
  acc = block_sum(acc, lds4);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

// per-column dot products a.b of column blockIdx.y over slice blockIdx.x
template <typename T>
__global__ __launch_bounds__(256) void k_col_dots(unsigned nn, const T* __restrict__ a, const T* __restrict__ b,
                                                  double* __restrict__ part) {
  __shared__ double lds4[4];
  const size_t co = (size_t)blockIdx.y * nn;
  double acc = 0.0;
  for (unsigned n = blockIdx.x * 256 + threadIdx.x; n < nn; n += gridDim.x * 256)
    acc += (double)a[co + n] * (double)b[co + n];
  acc = block_sum(acc, lds4);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

template <typename T, bool SQ>
void col_reduce(size_t nn, int F, int K, const T* v, double* out, double* work, hipStream_t st) {
  const unsigned G = slices_for(nn, F * K);
  hipLaunchKernelGGL((k_col_sums<T, SQ>), dim3(G, F * K), dim3(256), 0, st, (unsigned)nn, v, work);
  reduce_cols((int)G, F, K, 1, 0, 1, work, out, st);
  PHZ_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- Arnoldi
// J = j + 1 basis vectors, a compile-time count so that every load of the
// unrolled loops is unconditional and independent (memory-level
// parallelism).  Grid (slices, F*K): each block stays on one column, so the
// load column k = blockIdx.y % K and its coefficients are block-uniform.
template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

// Four consecutive values per thread as 16-byte accesses (one float4, or two
// double2), widened to double; the pointer must be 16-byte aligned.
__device__ __forceinline__ void ld4(const float* p, double (&v)[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}
__device__ __forceinline__ void ld4(const double* p, double (&v)[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void st4(float* p, const double (&v)[4]) {
  *reinterpret_cast<float4*>(p) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
}
__device__ __forceinline__ void st4(double* p, const double (&v)[4]) {
  reinterpret_cast<double2*>(p)[0] = double2{v[0], v[1]};
  reinterpret_cast<double2*>(p)[1] = double2{v[2], v[3]};
}

// Four consecutive nodes per thread and load (nn is a multiple of 8: N is
// even), 16-byte accesses.
template <typename T, int J>
__global__ __launch_bounds__(256) void k_arnoldi_dots(unsigned nn, const T* __restrict__ V, size_t vstride,
                                                      const T* __restrict__ w, double* __restrict__ part) {
  __shared__ double lds4[4];
  const size_t co = (size_t)blockIdx.y * nn;
  const unsigned nq = nn / 4;
  double acc[J];
#pragma unroll
  for (int i = 0; i < J; ++i) acc[i] = 0.0;
  for (unsigned h = blockIdx.x * 256 + threadIdx.x; h < nq; h += gridDim.x * 256) {
    double wv[4];
    ld4(w + co + 4 * (size_t)h, wv);
#pragma unroll
    for (int i = 0; i < J; ++i) {
      double v[4];
      ld4(V + i * vstride + co + 4 * (size_t)h, v);
      acc[i] += v[0] * wv[0] + v[1] * wv[1] + v[2] * wv[2] + v[3] * wv[3];
    }
  }
  const size_t base = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * J;
#pragma unroll
  for (int i = 0; i < J; ++i) {
    const double s = block_sum(acc[i], lds4);
    if (threadIdx.x == 0) part[base + i] = s;
  }
}

// w -= sum_i V_i h[i][k]; then (DOTS) V^T w_new, and ||w_new||^2 (last slot).
// flags (may be null): a load whose flag is 0 is left as it is (its blocks
// only write zero partial sums).
template <typename T, int J, bool DOTS>
__global__ __launch_bounds__(256) void k_arnoldi_update(unsigned nn, int K, const T* __restrict__ V, size_t vstride,
                                                        T* __restrict__ w, const double* __restrict__ hin,
                                                        double* __restrict__ part, const int* __restrict__ flags) {
  __shared__ double lds4[4];
  const int kk = blockIdx.y % K;
  const size_t co = (size_t)blockIdx.y * nn;
  const unsigned nq = nn / 4;
  constexpr int NV = (DOTS ? J : 0) + 1;
  if (flags && !flags[kk]) {   // block-uniform
    if (threadIdx.x < NV) part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * NV + threadIdx.x] = 0.0;
    return;
  }
  double h[J];
#pragma unroll
  for (int i = 0; i < J; ++i) h[i] = hin[i * K + kk];
  double acc[DOTS ? J : 1];
#pragma unroll
  for (int i = 0; i < (DOTS ? J : 1); ++i) acc[i] = 0.0;
  double nrm = 0.0;
  for (unsigned hh = blockIdx.x * 256 + threadIdx.x; hh < nq; hh += gridDim.x * 256) {
    T* wp = w + co + 4 * (size_t)hh;
    double vv[DOTS ? J : 1][4];
    double wv[4];
    ld4(wp, wv);
#pragma unroll
    for (int i = 0; i < J; ++i) {
      double v[4];
      ld4(V + i * vstride + co + 4 * (size_t)hh, v);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if constexpr (DOTS) vv[i][c] = v[c];
        wv[c] -= h[i] * v[c];
      }
    }
    // round to the vector's type once, and use the rounded values below
#pragma unroll
    for (int c = 0; c < 4; ++c) wv[c] = (double)(T)wv[c];
    st4(wp, wv);
#pragma unroll
    for (int c = 0; c < 4; ++c) nrm += wv[c] * wv[c];
    if constexpr (DOTS) {
#pragma unroll
      for (int i = 0; i < J; ++i) acc[i] += vv[i][0] * wv[0] + vv[i][1] * wv[1] + vv[i][2] * wv[2] + vv[i][3] * wv[3];
    }
  }
  const size_t base = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * NV;
  if constexpr (DOTS) {
#pragma unroll
    for (int i = 0; i < J; ++i) {
      const double s = block_sum(acc[i], lds4);
      if (threadIdx.x == 0) part[base + i] = s;
    }
  }
  const double s = block_sum(nrm, lds4);
  if (threadIdx.x == 0) part[base + NV - 1] = s;
}

constexpr int kFusedMaxJ = 12;

template <typename T, int J>
void launch_dots_J(dim3 g, hipStream_t st, unsigned nn, const T* V, size_t vs, const T* w, double* part) {
  hipLaunchKernelGGL((k_arnoldi_dots<T, J>), g, dim3(256), 0, st, nn, V, vs, w, part);
}
template <typename T, int J>
void launch_update_J(dim3 g, hipStream_t st, unsigned nn, int K, const T* V, size_t vs, T* w, const double* hin,
                     int want, double* part, const int* flags) {
  if constexpr (J <= kFusedMaxJ) {
    if (want) {
      hipLaunchKernelGGL((k_arnoldi_update<T, J, true>), g, dim3(256), 0, st, nn, K, V, vs, w, hin, part, flags);
      return;
    }
  }
  hipLaunchKernelGGL((k_arnoldi_update<T, J, false>), g, dim3(256), 0, st, nn, K, V, vs, w, hin, part, flags);
}
template <typename T>
using DotsFn = void (*)(dim3, hipStream_t, unsigned, const T*, size_t, const T*, double*);
template <typename T>
using UpdFn = void (*)(dim3, hipStream_t, unsigned, int, const T*, size_t, T*, const double*, int, double*,
                       const int*);
template <typename T, int... Js>
constexpr std::array<DotsFn<T>, sizeof...(Js)> dots_table(std::integer_sequence<int, Js...>) {
  return {&launch_dots_J<T, Js + 1>...};
}
template <typename T, int... Js>
constexpr std::array<UpdFn<T>, sizeof...(Js)> upd_table(std::integer_sequence<int, Js...>) {
  return {&launch_update_J<T, Js + 1>...};
}

// ------------------------------------------------------------- elementwise
template <typename T>
__global__ void k_scale_cols(unsigned nn, int K, const T* __restrict__ w, const double* __restrict__ scale,
                             T* __restrict__ v) {
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const size_t o = (size_t)blockIdx.y * nn + n;
  v[o] = (T)((double)w[o] * scale[blockIdx.y % K]);
}

// four-wide forms of the column kernels below (nn a multiple of 4)
template <typename T>
__global__ void k_scale_cols4(unsigned nn, int K, const T* __restrict__ w, const double* __restrict__ scale,
                              T* __restrict__ v) {
  const unsigned n = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (n >= nn) return;
  const size_t o = (size_t)blockIdx.y * nn + n;
  const double sc = scale[blockIdx.y % K];
  double a[4];
  ld4(w + o, a);
#pragma unroll
  for (int c = 0; c < 4; ++c) a[c] *= sc;
  st4(v + o, a);
}
template <typename T>
__global__ void k_combine4(unsigned nn, int K, const T* __restrict__ V, size_t vstride, const double* __restrict__ y,
                           const int* __restrict__ kused, T* __restrict__ t) {
  const unsigned n = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (n >= nn) return;
  const int kk = blockIdx.y % K;
  const int ku = kused[kk];
  const size_t o = (size_t)blockIdx.y * nn + n;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < ku; ++i) {
    double v[4];
    ld4(V + i * vstride + o, v);
    const double yi = y[i * K + kk];
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] += yi * v[c];
  }
  st4(t + o, s);
}
template <typename Tx, typename Tz>
__global__ void k_axpy_cols4(unsigned nn, int K, const double* __restrict__ a, const Tz* __restrict__ z,
                             Tx* __restrict__ x) {
  const unsigned n = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (n >= nn) return;
  const size_t o = (size_t)blockIdx.y * nn + n;
  const double av = a ? a[blockIdx.y % K] : 1.0;
  double xv[4], zv[4];
  ld4(x + o, xv);
  ld4(z + o, zv);
#pragma unroll
  for (int c = 0; c < 4; ++c) xv[c] += av * zv[c];
  st4(x + o, xv);
}
template <typename T>
__global__ void k_xpby_cols4(unsigned nn, int K, const double* __restrict__ beta, const T* __restrict__ z,
                             T* __restrict__ p) {
  const unsigned n = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (n >= nn) return;
  const size_t o = (size_t)blockIdx.y * nn + n;
  const double b = beta[blockIdx.y % K];
  double zv[4], pv[4];
  ld4(z + o, zv);
  ld4(p + o, pv);
#pragma unroll
  for (int c = 0; c < 4; ++c) pv[c] = zv[c] + b * pv[c];
  st4(p + o, pv);
}

template <typename T>
__global__ void k_combine(unsigned nn, int K, const T* __restrict__ V, size_t vstride, const double* __restrict__ y,
                          const int* __restrict__ kused, T* __restrict__ t) {
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int kk = blockIdx.y % K;
  const int ku = kused[kk];
  const size_t o = (size_t)blockIdx.y * nn + n;
  double s = 0.0;
  for (int i = 0; i < ku; ++i) s += y[i * K + kk] * (double)V[i * vstride + o];
  t[o] = (T)s;
}

template <typename Tx, typename Tz>
__global__ void k_axpy_cols(unsigned nn, int K, const double* __restrict__ a, const Tz* __restrict__ z,
                            Tx* __restrict__ x) {
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const size_t o = (size_t)blockIdx.y * nn + n;
  const double av = a ? a[blockIdx.y % K] : 1.0;
  x[o] = (Tx)((double)x[o] + av * (double)z[o]);
}

// p = z + beta_k p (per load column k)
template <typename T>
__global__ void k_xpby_cols(unsigned nn, int K, const double* __restrict__ beta, const T* __restrict__ z,
                            T* __restrict__ p) {
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const size_t o = (size_t)blockIdx.y * nn + n;
  p[o] = (T)((double)z[o] + beta[blockIdx.y % K] * (double)p[o]);
}

template <typename Ts, typename Td>
__global__ void k_convert(size_t count, const Ts* __restrict__ s, Td* __restrict__ d) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    d[i] = (Td)s[i];
}

template <typename T>
__global__ void k_fill(size_t count, T v, T* __restrict__ d) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    d[i] = v;
}

template <typename T>
__global__ void k_subtract_mean(unsigned nn, const double* __restrict__ sums, T* __restrict__ v) {
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const size_t o = (size_t)blockIdx.y * nn + n;
  v[o] = (T)((double)v[o] - sums[blockIdx.y] / (double)nn);
}

// column f of a 4-field single-load vector <-> column f*9 + load of a 9-load block
__global__ void k_extract_col(unsigned nn, int load, const double* __restrict__ block, double* __restrict__ col) {
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  col[(size_t)blockIdx.y * nn + n] = block[(size_t)(blockIdx.y * 9 + load) * nn + n];
}
__global__ void k_insert_col(unsigned nn, int load, const double* __restrict__ col, double* __restrict__ block) {
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  block[(size_t)(blockIdx.y * 9 + load) * nn + n] = col[(size_t)blockIdx.y * nn + n];
}

// dst[n*ncol + c] = src[c*nn + n] (and back)
__global__ void k_soa_to_aos(unsigned nn, int ncol, const double* __restrict__ src, double* __restrict__ dst) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)nn * ncol) return;
  const unsigned n = (unsigned)(i / ncol);
  const int c = (int)(i - (size_t)n * ncol);
  dst[i] = src[(size_t)c * nn + n];
}
__global__ void k_aos_to_soa(unsigned nn, int ncol, const double* __restrict__ src, double* __restrict__ dst) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)nn * ncol) return;
  const unsigned n = (unsigned)(i / ncol);
  const int c = (int)(i - (size_t)n * ncol);
  dst[(size_t)c * nn + n] = src[i];
}

// --------------------------------------------------------------- GMRES small
__global__ void k_gmres_start(int K, const double* __restrict__ nrm2, double rtol, GmresState s) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const int k = threadIdx.x;
  if (k < K) {
    const double beta = sqrt(nrm2[k]);
    s.g[k] = beta;
    const double bn = s.bnorm[k];
    const double tk = s.tol ? s.tol[k] : rtol;
    const int act = (bn > 0.0) && (beta > tk * bn) && isfinite(beta);
    s.active[k] = act;
    s.kused[k] = 0;
    s.scale[k] = act ? 1.0 / beta : 0.0;
    if (act) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) s.nactive[0] = cnt;
}

// Selective reorthogonalisation.  After one classical Gram-Schmidt pass
// w' = w - V h1, h2 = V^T w' are w''s remaining components along the basis,
// so |h2| / |w'| is exactly how far v = w' / |w'| is from orthogonal to it.
// A load needs the second pass only where |h2|^2 > tau2 |w'|^2; elsewhere
// its h2 is zeroed (the Hessenberg column is then h1 and |w'|, which is the
// Arnoldi relation of the vector actually kept) and flag[k] = 0.  tau2 < 0:
// every active load takes the second pass (plain CGS2); inactive (converged)
// loads never do.  count[k] accumulates the second passes taken.
__global__ void k_reorth_decide(int K, int J, double tau2, double* __restrict__ h2, const double* __restrict__ na2,
                                const int* __restrict__ active, int* __restrict__ flag, int* __restrict__ count) {
  const int k = threadIdx.x;
  if (k >= K) return;
  double q = 0.0;
  for (int i = 0; i < J; ++i) q += h2[i * K + k] * h2[i * K + k];
  const int need = active[k] && (tau2 < 0.0 || q > tau2 * na2[k]) ? 1 : 0;
  flag[k] = need;
  count[k] += need;
  if (!need)
    for (int i = 0; i < J; ++i) h2[i * K + k] = 0.0;
}

// nrm2 is |w|^2 after the second pass where flag[k] (or flag is null), else
// na2[k], the norm after the first
__global__ void k_gmres_givens(int K, int m, int j, const double* __restrict__ h1, const double* __restrict__ h2,
                               const double* __restrict__ nrm2, double rtol, double stall, GmresState s,
                               const int* __restrict__ flag, const double* __restrict__ na2) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const int k = threadIdx.x;
  if (k < K && s.active[k]) {
    double col[kMaxRestart + 1];
    for (int i = 0; i <= j; ++i) col[i] = h1[i * K + k] + (h2 ? h2[i * K + k] : 0.0);
    const double hn = sqrt(flag && !flag[k] ? na2[k] : nrm2[k]);
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double c = s.cs[i * K + k], sn = s.sn[i * K + k];
      const double a = c * col[i] + sn * col[i + 1];
      col[i + 1] = -sn * col[i] + c * col[i + 1];
      col[i] = a;
    }
    double den = hypot(col[j], col[j + 1]);
    double c = 1.0, sn = 0.0;
    if (den > 0.0) {
      c = col[j] / den;
      sn = col[j + 1] / den;
    }
    s.cs[j * K + k] = c;
    s.sn[j * K + k] = sn;
    col[j] = den;
    for (int i = 0; i <= j; ++i) s.H[((size_t)i * m + j) * K + k] = col[i];
    const double gj = s.g[j * K + k];
    s.g[(j + 1) * K + k] = -sn * gj;
    s.g[j * K + k] = c * gj;
    const double est = fabs(s.g[(j + 1) * K + k]) / s.bnorm[k];
    s.est[j * K + k] = est;
    // stall: the estimate fell by less than the factor `stall` over two steps
    const bool stalled = stall > 0.0 && j >= 2 && est > stall * s.est[(j - 2) * K + k];
    const double tk = s.tol ? s.tol[k] : rtol;
    const bool stop = !(est > tk) || !(hn > 0.0) || (j + 1 == m) || !isfinite(est) || stalled;
    s.kused[k] = j + 1;
    if (stop) {
      s.active[k] = 0;
      s.scale[k] = 0.0;
    } else {
      s.scale[k] = 1.0 / hn;
      atomicAdd(&cnt, 1);
    }
  } else if (k < K) {
    s.scale[k] = 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) s.nactive[0] = cnt;
}

__global__ void k_gmres_solve_y(int K, int m, GmresState s) {
  const int k = threadIdx.x;
  if (k >= K) return;
  const int ku = s.kused[k];
  for (int i = ku - 1; i >= 0; --i) {
    double v = s.g[i * K + k];
    for (int c = i + 1; c < ku; ++c) v -= s.H[((size_t)i * m + c) * K + k] * s.y[c * K + k];
    const double d = s.H[((size_t)i * m + i) * K + k];
    s.y[i * K + k] = d != 0.0 ? v / d : 0.0;
  }
}

// ---------------------------------------------------------------- physics
struct Nb {
  unsigned i, j, k, im, jm, km, ip, jp, kp;
};
__device__ __forceinline__ Nb nbr(unsigned n, unsigned N) {
  Nb r;
  const unsigned t = n / N;
  r.i = n - t * N;
  r.k = t / N;
  r.j = t - r.k * N;
  r.im = r.i ? r.i - 1 : N - 1;
  r.jm = r.j ? r.j - 1 : N - 1;
  r.km = r.k ? r.k - 1 : N - 1;
  r.ip = r.i + 1 < N ? r.i + 1 : 0;
  r.jp = r.j + 1 < N ? r.j + 1 : 0;
  r.kp = r.k + 1 < N ? r.k + 1 : 0;
  return r;
}
__device__ __forceinline__ unsigned at(unsigned N, unsigned i, unsigned j, unsigned k) { return i + N * (j + N * k); }

// element e with origin (i,j,k): corner c is node (i + cx, j + cy, k + cz)
__device__ __forceinline__ unsigned corner_node(const Nb& q, unsigned N, int c) {
  return at(N, (c & 1) ? q.ip : q.i, (c & 2) ? q.jp : q.j, (c & 4) ? q.kp : q.k);
}
// node n is corner c of element with origin n - c
__device__ __forceinline__ unsigned elem_of_corner(const Nb& q, unsigned N, int c) {
  return at(N, (c & 1) ? q.im : q.i, (c & 2) ? q.jm : q.j, (c & 4) ? q.km : q.k);
}

__device__ __forceinline__ double sheaviside(double t, double eta) {
  if (t < -eta) return 0.0;
  if (t > eta) return 1.0;
  return 0.5 * (1.0 + t / eta + sin(M_PI * t / eta) / M_PI);
}
__device__ __forceinline__ double sheaviside_d(double t, double eta) {
  if (t < -eta || t > eta) return 0.0;
  return (1.0 + cos(M_PI * t / eta)) / (2.0 * eta);
}

__global__ void k_levelset_to_scale(unsigned N, const double* __restrict__ phi, double eta, double ev,
                                    double* __restrict__ rho, double* __restrict__ s, float* __restrict__ s32) {
  const unsigned nn = N * N * N;
  const unsigned e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const Nb q = nbr(e, N);
  double m = 0.0;
  for (int c = 0; c < 8; ++c) m += phi[corner_node(q, N, c)];
  m *= 0.125;
  const double r = 1.0 - sheaviside(m, eta);
  const double sv = ev + (1.0 - ev) * r;
  rho[e] = r;
  s[e] = sv;
  s32[e] = (float)sv;
}

// Quadrature-point smoothing: the level set interpolated trilinearly at the
// element's eight Gauss points p = i + 2j + 4k (points (g_i, g_j, g_k)),
// smoothed there; sq[8e + p] the point scales, s and rho their element means.
__global__ void k_levelset_to_scale_qp(unsigned N, const double* __restrict__ phi, double eta, double ev,
                                       double* __restrict__ rho, double* __restrict__ s, float* __restrict__ s32,
                                       double* __restrict__ sq, float* __restrict__ sq32) {
  const unsigned nn = N * N * N;
  const unsigned e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const Nb q = nbr(e, N);
  double pc[8];
  for (int c = 0; c < 8; ++c) pc[c] = phi[corner_node(q, N, c)];
  const double g[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  double rsum = 0.0, ssum = 0.0;
  for (int p = 0; p < 8; ++p) {
    const double xi = g[p & 1], yi = g[(p >> 1) & 1], zi = g[(p >> 2) & 1];
    double v = 0.0;
    for (int c = 0; c < 8; ++c)
      v += ((c & 1) ? xi : 1.0 - xi) * ((c & 2) ? yi : 1.0 - yi) * ((c & 4) ? zi : 1.0 - zi) * pc[c];
    const double r = 1.0 - sheaviside(v, eta);
    const double sv = ev + (1.0 - ev) * r;
    sq[(size_t)e * 8 + p] = sv;
    sq32[(size_t)e * 8 + p] = (float)sv;
    rsum += r;
    ssum += sv;
  }
  rho[e] = 0.125 * rsum;
  s[e] = 0.125 * ssum;
  s32[e] = (float)(0.125 * ssum);
}

// point scales equal to the element scale (a cell given by its densities)
__global__ void k_point_scales(unsigned nn, const double* __restrict__ s, double* __restrict__ sq,
                               float* __restrict__ sq32) {
  const unsigned e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  for (int p = 0; p < 8; ++p) {
    sq[(size_t)e * 8 + p] = s[e];
    sq32[(size_t)e * 8 + p] = (float)s[e];
  }
}

__global__ void k_density_to_scale(unsigned nn, const double* __restrict__ rho, double ev, double* __restrict__ s,
                                   float* __restrict__ s32) {
  const unsigned e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const double sv = ev + (1.0 - ev) * rho[e];
  s[e] = sv;
  s32[e] = (float)sv;
}

// b[(f*9 + L)][n] = -sum_c s_{n-c} F0[4c + f][L]   (absval: sum_c s |F0|)
__global__ __launch_bounds__(128) void k_build_rhs(unsigned N, const double* __restrict__ s,
                                                   const double* __restrict__ F0, double* __restrict__ b, int absval) {
  const unsigned nn = N * N * N;
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const Nb q = nbr(n, N);
  double se[8];
  for (int c = 0; c < 8; ++c) se[c] = s[elem_of_corner(q, N, c)];
  for (int f = 0; f < 4; ++f)
    for (int L = 0; L < 9; ++L) {
      double acc = 0.0;
      for (int c = 0; c < 8; ++c) {
        const double v = F0[(4 * c + f) * 9 + L];
        acc -= se[c] * (absval ? -fabs(v) : v);
      }
      b[(size_t)(f * 9 + L) * nn + n] = acc;
    }
}

// b[(f*9 + L)][n] = -sum_c sum_p sq[8 e_c + p] F0q[p][4c + f][L], e_c the
// element whose corner c is n (absval: the magnitudes of the terms)
__global__ __launch_bounds__(128) void k_build_rhs_qp(unsigned N, const double* __restrict__ sq,
                                                      const double* __restrict__ F0q, double* __restrict__ b,
                                                      int absval) {
  const unsigned nn = N * N * N;
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const Nb q = nbr(n, N);
  unsigned ec[8];
  for (int c = 0; c < 8; ++c) ec[c] = elem_of_corner(q, N, c);
  for (int f = 0; f < 4; ++f)
    for (int L = 0; L < 9; ++L) {
      double acc = 0.0;
      for (int c = 0; c < 8; ++c)
        for (int p = 0; p < 8; ++p) {
          const double v = F0q[p * 288 + (4 * c + f) * 9 + L];
          acc -= sq[(size_t)ec[c] * 8 + p] * (absval ? -fabs(v) : v);
        }
      b[(size_t)(f * 9 + L) * nn + n] = acc;
    }
}

// partial Y[(l, col)] = sum_n s_{n - c(l)} X[col][n] for column blockIdx.y,
// the scale of element e read at s[stride e + off]
__global__ __launch_bounds__(256) void k_reduce_effective(unsigned N, const double* __restrict__ s, int stride,
                                                          int off, const double* __restrict__ X,
                                                          double* __restrict__ part) {
  __shared__ double lds4[4];
  const unsigned nn = N * N * N;
  const double* col = X + (size_t)blockIdx.y * nn;
  double acc[8];
  for (int l = 0; l < 8; ++l) acc[l] = 0.0;
  for (unsigned n = blockIdx.x * 256 + threadIdx.x; n < nn; n += gridDim.x * 256) {
    const Nb q = nbr(n, N);
    const double xv = col[n];
    for (int l = 0; l < 8; ++l) acc[l] += s[(size_t)elem_of_corner(q, N, l) * stride + off] * xv;
  }
  const size_t base = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 8;
  for (int l = 0; l < 8; ++l) {
    const double v = block_sum(acc[l], lds4);
    if (threadIdx.x == 0) part[base + l] = v;
  }
}

// U = X W per node: U[(f*9 + L)*nn + n] = sum_L' X[(f*9 + L')*nn + n] W[L'*9 + L]
__global__ __launch_bounds__(256) void k_mix_cols(unsigned nn, const double* __restrict__ X,
                                                  const double* __restrict__ W, double* __restrict__ U) {
  __shared__ double ws[81];
  for (int t = threadIdx.x; t < 81; t += blockDim.x) ws[t] = W[t];
  __syncthreads();
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (n >= nn) return;
  double xv[9];
  for (int L = 0; L < 9; ++L) xv[L] = X[(size_t)(f * 9 + L) * nn + n];
  for (int L = 0; L < 9; ++L) {
    double v = 0.0;
    for (int Lp = 0; Lp < 9; ++Lp) v += xv[Lp] * ws[Lp * 9 + L];
    U[(size_t)(f * 9 + L) * nn + n] = v;
  }
}

typedef __attribute__((ext_vector_type(4))) double f64x4;

// dJ/drho_e = factor * ( cterm + <X_e, FW> + sum_L U_e[:, L]^T K0 X_e[:, L] ), U = X W
// (the bilinear term <K0 X_e, X_e W> taken column by column).  X_e[:, L] is
// the element's 32 inputs of load column L (row 4 c + f: corner c, field f).
// A workgroup takes a 16 x 4 x 4 block of elements (masked past N on ragged
// blocks) and, per load column, stages the block's 17 x 5 x 5 nodes of X and U
// in LDS.  Each wave contracts four rows of 16 elements on the matrix cores:
// D = K0 X_e for the 16 elements of a row is two row tiles (rows 0..15 and
// 16..31 of K0) times eight k-steps of v_mfma_f64_16x16x4f64, k-step s being
// corner s with its four fields; a lane then dots its eight rows of D (one
// field of eight corners) with the element's U, and the four lanes of an
// element add their sums at the end.
__global__ __launch_bounds__(256) void k_backward_mfma(unsigned N, const double* __restrict__ X,
                                                       const double* __restrict__ U, const double* __restrict__ K0,
                                                       const double* __restrict__ FW, double cterm, double factor,
                                                       int stride, int off, double* __restrict__ grad) {
  constexpr int TX = 16, TY = 4, TZ = 4, NX = TX + 1, NY = TY + 1, NZ = TZ + 1, NB = NX * NY * NZ;
  constexpr int NS = 4 * NB, PF = (NS + 255) / 256;  // staged values per array, per thread
  __shared__ double xs[NS];  // [node][field]
  __shared__ double us[NS];
  __shared__ double fws[32 * 9];
  const unsigned nn = N * N * N;
  const unsigned ntx = (N + TX - 1) / TX, nty = (N + TY - 1) / TY;
  const unsigned b = dev::xcd_block(blockIdx.x, gridDim.x);
  const unsigned x0 = (b % ntx) * TX, y0 = ((b / ntx) % nty) * TY, z0 = (b / (ntx * nty)) * TZ;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int t = tid; t < 32 * 9; t += 256) fws[t] = FW[t];
  // A operands: K0 rows 16 t + (lane & 15), column 4 s + (lane >> 4)
  double ak[2][8];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int s8 = 0; s8 < 8; ++s8) ak[t][s8] = K0[(16 * t + (lane & 15)) * 32 + 4 * s8 + (lane >> 4)];
  // staged values of this thread: slot q = tid + 256 p is field q / NB of
  // block node q % NB (x fastest); its global offset without the column
  size_t go[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    const int q = tid + 256 * p;
    const int f = q / NB, m = q % NB;
    const unsigned gx = (x0 + m % NX) % N, gy = (y0 + (m / NX) % NY) % N, gz = (z0 + m / (NX * NY)) % N;
    go[p] = q < NS ? (size_t)(f * 9) * nn + gx + N * (gy + (size_t)N * gz) : 0;
  }
  double px[PF], pu[PF];
  auto fetch = [&](int L) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      px[p] = X[go[p] + (size_t)L * nn];
      pu[p] = U[go[p] + (size_t)L * nn];
    }
  };
  const int xl = lane & 15, g = lane >> 4;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  fetch(0);
  for (int L = 0; L < 9; ++L) {
    __syncthreads();  // the previous column's LDS reads are complete
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int q = tid + 256 * p;
      if (q < NS) {
        const int f = q / NB, m = q % NB;
        xs[m * 4 + f] = px[p];
        us[m * 4 + f] = pu[p];
      }
    }
    if (L + 1 < 9) fetch(L + 1);  // in flight during this column's products
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wave + 4 * i, ey = r % TY, ez = r / TY;
      f64x4 d0 = {0.0, 0.0, 0.0, 0.0}, d1 = {0.0, 0.0, 0.0, 0.0};
      double fw = 0.0;
#pragma unroll
      for (int s8 = 0; s8 < 8; ++s8) {
        const int m = (xl + (s8 & 1)) + NX * ((ey + ((s8 >> 1) & 1)) + NY * (ez + (s8 >> 2)));
        const double bv = xs[m * 4 + g];  // X_e row 4 s + g (corner s, field g)
        fw += bv * fws[(4 * s8 + g) * 9 + L];
        d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ak[0][s8], bv, d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ak[1][s8], bv, d1, 0, 0, 0);
      }
      // register j of row tile t holds row 16 t + 4 j + g of D (the f64
      // product's output layout): corner 4 t + j, field g
      double dot = fw;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const f64x4 dd = t == 0 ? d0 : d1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = 4 * t + j;
          const int m = (xl + (c & 1)) + NX * ((ey + ((c >> 1) & 1)) + NY * (ez + (c >> 2)));
          const double dj = dd[j];
          dot += dj * us[m * 4 + g];
        }
      }
      acc[i] += dot;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double v = acc[i];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    const int r = wave + 4 * i;
    const unsigned ex = x0 + xl, ey = y0 + r % TY, ez = z0 + r / TY;
    if (g == 0 && ex < N && ey < N && ez < N)
      grad[(ex + N * (ey + (size_t)N * ez)) * stride + off] = factor * (cterm + v);
  }
}

// Chain rule of the point densities rho_ep = 1 - H(phi(x_p)) to the nodes:
// dJ/dphi_n = -sum over the 8 elements e with n = corner c of e, and their
// Gauss points p, of H'(phi(x_p)) N_c(xi_p) g_ep, with g_ep = g[8e + p]
// (stride 8) or g[e] / 8 (stride 1: an element gradient spread evenly)
__global__ void k_grad_phi_qp(unsigned N, const double* __restrict__ phi, double eta, const double* __restrict__ g,
                              int stride, double* __restrict__ out) {
  const unsigned nn = N * N * N;
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const Nb q = nbr(n, N);
  const double gq[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  double acc = 0.0;
  for (int c = 0; c < 8; ++c) {
    const unsigned e = elem_of_corner(q, N, c);
    const Nb qe = nbr(e, N);
    double pc[8];
    for (int cc = 0; cc < 8; ++cc) pc[cc] = phi[corner_node(qe, N, cc)];
    for (int p = 0; p < 8; ++p) {
      const double xi = gq[p & 1], yi = gq[(p >> 1) & 1], zi = gq[(p >> 2) & 1];
      double v = 0.0, nc = 0.0;
      for (int cc = 0; cc < 8; ++cc) {
        const double w = ((cc & 1) ? xi : 1.0 - xi) * ((cc & 2) ? yi : 1.0 - yi) * ((cc & 4) ? zi : 1.0 - zi);
        v += w * pc[cc];
        if (cc == c) nc = w;
      }
      const double ge = stride == 8 ? g[(size_t)e * 8 + p] : 0.125 * g[e];
      acc -= sheaviside_d(v, eta) * nc * ge;
    }
  }
  out[n] = acc;
}

// per element, the sum of its eight point values
__global__ void k_sum_points(unsigned nn, const double* __restrict__ gq, double* __restrict__ ge) {
  const unsigned e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  double v = 0.0;
  for (int p = 0; p < 8; ++p) v += gq[(size_t)e * 8 + p];
  ge[e] = v;
}

// partial cross products sum_n X[(f, a)][n] * Y[(f, b)][n] for (f, a) = blockIdx.y
__global__ __launch_bounds__(256) void k_cross_dots(unsigned nn, const double* __restrict__ X,
                                                    const double* __restrict__ Y, double* __restrict__ part) {
  __shared__ double lds4[4];
  const int f = blockIdx.y / 9;
  const double* xc = X + (size_t)blockIdx.y * nn;
  double acc[9];
  for (int b = 0; b < 9; ++b) acc[b] = 0.0;
  for (unsigned n = blockIdx.x * 256 + threadIdx.x; n < nn; n += gridDim.x * 256) {
    const double xv = xc[n];
    for (int b = 0; b < 9; ++b) acc[b] += xv * Y[(size_t)(f * 9 + b) * nn + n];
  }
  const size_t base = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 9;
  for (int b = 0; b < 9; ++b) {
    const double v = block_sum(acc[b], lds4);
    if (threadIdx.x == 0) part[base + b] = v;
  }
}

__global__ void k_grad_phi(unsigned N, const double* __restrict__ phi, double eta, const double* __restrict__ grho,
                           double* __restrict__ out) {
  const unsigned nn = N * N * N;
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const Nb q = nbr(n, N);
  double acc = 0.0;
  for (int c = 0; c < 8; ++c) {
    const unsigned e = elem_of_corner(q, N, c);
    const Nb qe = nbr(e, N);
    double m = 0.0;
    for (int cc = 0; cc < 8; ++cc) m += phi[corner_node(qe, N, cc)];
    m *= 0.125;
    acc -= sheaviside_d(m, eta) * grho[e];
  }
  out[n] = acc * 0.125;
}

__global__ void k_nodal_mean(unsigned N, const double* __restrict__ ge, double* __restrict__ vn) {
  const unsigned nn = N * N * N;
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const Nb q = nbr(n, N);
  double acc = 0.0;
  for (int c = 0; c < 8; ++c) acc += ge[elem_of_corner(q, N, c)];
  vn[n] = acc * 0.125;
}

__global__ void k_max_abs(size_t count, const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double lds[256];
  double m = 0.0;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < count; idx += (size_t)gridDim.x * 256)
    m = fmax(m, fabs(v[idx]));
  lds[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = lds[0];
}

__global__ void k_max_partials(int nb, const double* __restrict__ part, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int b = 0; b < nb; ++b) m = fmax(m, part[b]);
    out[0] = m;
  }
}

// values that are not finite or lie outside [lo, hi]
__global__ void k_count_outside(size_t count, const double* __restrict__ v, double lo, double hi,
                                double* __restrict__ part) {
  __shared__ double lds4[4];
  double c = 0.0;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < count; idx += (size_t)gridDim.x * 256) {
    const double x = v[idx];
    c += (isfinite(x) && x >= lo && x <= hi) ? 0.0 : 1.0;
  }
  c = block_sum(c, lds4);
  if (threadIdx.x == 0) part[blockIdx.x] = c;
}

__global__ void k_hj_step(unsigned N, const double* __restrict__ phi, const double* __restrict__ v,
                          const double* __restrict__ vmax, double dt, double* __restrict__ out) {
  const unsigned nn = N * N * N;
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const Nb q = nbr(n, N);
  const double h = 1.0 / N;
  const double f0 = phi[n];
  const double fx[2] = {phi[at(N, q.im, q.j, q.k)], phi[at(N, q.ip, q.j, q.k)]};
  const double fy[2] = {phi[at(N, q.i, q.jm, q.k)], phi[at(N, q.i, q.jp, q.k)]};
  const double fz[2] = {phi[at(N, q.i, q.j, q.km)], phi[at(N, q.i, q.j, q.kp)]};
  const double* nb[3] = {fx, fy, fz};
  double gp = 0.0, gm = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double dm = (f0 - nb[a][0]) / h, dp = (nb[a][1] - f0) / h;
    gp += fmax(dm, 0.0) * fmax(dm, 0.0) + fmin(dp, 0.0) * fmin(dp, 0.0);
    gm += fmin(dm, 0.0) * fmin(dm, 0.0) + fmax(dp, 0.0) * fmax(dp, 0.0);
  }
  const double vm = vmax ? vmax[0] : 1.0;
  const double vv = vm > 0.0 ? v[n] / vm : 0.0;
  out[n] = f0 - dt * (fmax(vv, 0.0) * sqrt(gp) + fmin(vv, 0.0) * sqrt(gm));
}

// One pseudo-time step of the reinitialisation equation
// phi_t + S(phi0) (|grad phi| - 1) = 0, S = phi0 / sqrt(phi0^2 + h^2), with the
// first-order Godunov upwinding of the HJ step
__global__ void k_reinit_step(unsigned N, const double* __restrict__ phi, const double* __restrict__ phi0, double dt,
                              int subcell, double* __restrict__ out) {
  const unsigned nn = N * N * N;
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const Nb q = nbr(n, N);
  const double h = 1.0 / N;
  const double f0 = phi[n];
  const double p0 = phi0[n];
  double S;
  if (subcell) {
    // subcell fix: a node with a sign change of phi0 towards a neighbour
    // relaxes towards its distance estimate phi0 / |grad phi0|
    const double gx[2] = {phi0[at(N, q.im, q.j, q.k)], phi0[at(N, q.ip, q.j, q.k)]};
    const double gy[2] = {phi0[at(N, q.i, q.jm, q.k)], phi0[at(N, q.i, q.jp, q.k)]};
    const double gz[2] = {phi0[at(N, q.i, q.j, q.km)], phi0[at(N, q.i, q.j, q.kp)]};
    const double* g[3] = {gx, gy, gz};
    bool iface = p0 == 0.0;
    double grad2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      iface = iface || p0 * g[a][0] < 0.0 || p0 * g[a][1] < 0.0;
      const double d = fmax(fabs(g[a][1] - g[a][0]) / 2.0, fmax(fabs(g[a][1] - p0), fabs(p0 - g[a][0])));
      grad2 += d * d;
    }
    S = p0 > 0.0 ? 1.0 : (p0 < 0.0 ? -1.0 : 0.0);
    if (iface) {
      const double D = grad2 > 0.0 ? h * p0 / sqrt(grad2) : 0.0;
      out[n] = f0 - (dt / h) * (S * fabs(f0) - D);
      return;
    }
  } else {
    S = p0 / sqrt(p0 * p0 + h * h);
  }
  const double fx[2] = {phi[at(N, q.im, q.j, q.k)], phi[at(N, q.ip, q.j, q.k)]};
  const double fy[2] = {phi[at(N, q.i, q.jm, q.k)], phi[at(N, q.i, q.jp, q.k)]};
  const double fz[2] = {phi[at(N, q.i, q.j, q.km)], phi[at(N, q.i, q.j, q.kp)]};
  const double* nb[3] = {fx, fy, fz};
  double gp = 0.0, gm = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double dm = (f0 - nb[a][0]) / h, dp = (nb[a][1] - f0) / h;
    gp += fmax(dm, 0.0) * fmax(dm, 0.0) + fmin(dp, 0.0) * fmin(dp, 0.0);
    gm += fmin(dm, 0.0) * fmin(dm, 0.0) + fmax(dp, 0.0) * fmax(dp, 0.0);
  }
  out[n] = f0 - dt * (fmax(S, 0.0) * sqrt(gp) + fmin(S, 0.0) * sqrt(gm) - S);
}

// One Chebyshev step on K columns for a constant 27-point node stencil w[d]
// (d = dx + 3 dy + 9 dz, offsets -1..1): q = W d at the node, then
// x += d, r -= q, dn = c1 d + c2 r.  dn is a separate buffer because the
// stencil reads d at the neighbours.
__global__ __launch_bounds__(256) void k_stencil_cheb(unsigned N, const double* __restrict__ w,
                                                      const double* __restrict__ d, double* __restrict__ x,
                                                      double* __restrict__ r, double* __restrict__ dn, double c1,
                                                      double c2) {
  const unsigned nn = N * N * N;
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const size_t co = (size_t)blockIdx.y * nn;
  const Nb q = nbr(n, N);
  const unsigned xs[3] = {q.im, q.i, q.ip}, ys[3] = {q.jm, q.j, q.jp}, zs[3] = {q.km, q.k, q.kp};
  double acc = 0.0;
  for (int e = 0; e < 27; ++e) acc += w[e] * d[co + at(N, xs[e % 3], ys[(e / 3) % 3], zs[e / 9])];
  const double dv = d[co + n];
  const double rv = r[co + n] - acc;
  x[co + n] += dv;
  r[co + n] = rv;
  dn[co + n] = c1 * dv + c2 * rv;
}

// TriCG direction and iterate update on one block (F fields, K loads,
// column f K + k): with the load's coefficients cf[6k..6k+5] =
// (L00, L01, L10, L11, z0, z1) and the block's basis vector w entering the
// first (side 0) or the second (side 1) direction column,
//   g1 <- [side 0] w - (L00 g1 + L01 g2),  g2 <- [side 1] w - (L10 g1 + L11 g2),
//   x  += z0 g1 + z1 g2.
__global__ void k_tricg_update(size_t nn, size_t count, int K, const double* __restrict__ cf,
                               const double* __restrict__ w, int side, double* __restrict__ g1,
                               double* __restrict__ g2, double* __restrict__ x) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const double* c = cf + 6 * ((idx / nn) % K);
  const double o1 = g1[idx], o2 = g2[idx], wv = w[idx];
  const double n1 = (side == 0 ? wv : 0.0) - (c[0] * o1 + c[1] * o2);
  const double n2 = (side == 1 ? wv : 0.0) - (c[2] * o1 + c[3] * o2);
  g1[idx] = n1;
  g2[idx] = n2;
  x[idx] += c[4] * n1 + c[5] * n2;
}

template <typename T>
__global__ void k_normalize_by(size_t count, const double* __restrict__ nrm2, const T* __restrict__ w,
                               T* __restrict__ v) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const double nr = sqrt(nrm2[0]);
  v[idx] = (T)(nr > 0.0 ? (double)w[idx] / nr : 0.0);
}

__global__ void k_hash_fill(size_t count, unsigned seed, double* __restrict__ v) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  unsigned long long z = (unsigned long long)idx * 0x9E3779B97F4A7C15ULL + seed;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  v[idx] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

}  // namespace

size_t reduce_work_size() { return (size_t)kMaxPartBlocks * (kMaxRestart + 2) + 4096; }

template <typename Ts, typename Td>
void convert(long count, const Ts* src, Td* dst, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_convert<Ts, Td>), dim3(std::min<size_t>(blocks_for(count, 256), 65536)), dim3(256), 0, st,
                     (size_t)count, src, dst);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void fill(long count, T value, T* dst, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_fill<T>), dim3(std::min<size_t>(blocks_for(count, 256), 65536)), dim3(256), 0, st,
                     (size_t)count, value, dst);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void col_norm2(long nn, int F, int K, const T* v, double* out, double* work, hipStream_t st) {
  col_reduce<T, true>((size_t)nn, F, K, v, out, work, st);
}

template <typename T>
void col_dot(long nn, int F, int K, const T* a, const T* b, double* out, double* work, hipStream_t st) {
  const unsigned G = slices_for((size_t)nn, F * K);
  hipLaunchKernelGGL((k_col_dots<T>), dim3(G, F * K), dim3(256), 0, st, (unsigned)nn, a, b, work);
  reduce_cols((int)G, F, K, 1, 0, 1, work, out, st);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void xpby_cols(long nn, int F, int K, const double* beta, const T* z, T* p, hipStream_t st) {
  if (nn % 4 == 0)
    hipLaunchKernelGGL((k_xpby_cols4<T>), dim3(blocks_for(nn / 4, 256), F * K), dim3(256), 0, st, (unsigned)nn, K,
                       beta, z, p);
  else
    hipLaunchKernelGGL((k_xpby_cols<T>), dim3(blocks_for(nn, 256), F * K), dim3(256), 0, st, (unsigned)nn, K, beta,
                       z, p);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void field_sums(long nn, int F, int K, const T* v, double* out, double* work, hipStream_t st) {
  col_reduce<T, false>((size_t)nn, 1, F * K, v, out, work, st);
}

template <typename T>
void subtract_mean(long nn, int F, int K, const double* sums, T* v, hipStream_t st) {
  hipLaunchKernelGGL((k_subtract_mean<T>), dim3(blocks_for(nn, 256), F * K), dim3(256), 0, st, (unsigned)nn, sums, v);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void arnoldi_dots(long nn, int F, int K, int j, const T* V, long vstride, const T* w, double* hout, double* work,
                  hipStream_t st) {
  static constexpr auto table = dots_table<T>(std::make_integer_sequence<int, kMaxRestart + 1>{});
  if (nn % 4 != 0 || vstride % 4 != 0) throw std::logic_error("Arnoldi vectors: length and stride multiples of 4");
  const unsigned G = slices_for((size_t)nn, F * K);
  table[j](dim3(G, F * K), st, (unsigned)nn, V, (size_t)vstride, w, work);
  reduce_cols((int)G, F, K, j + 1, 0, j + 1, work, hout, st);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void arnoldi_update(long nn, int F, int K, int j, const T* V, long vstride, T* w, const double* hin, double* hout,
                    double* nrm2out, double* work, hipStream_t st, const int* flags) {
  static constexpr auto table = upd_table<T>(std::make_integer_sequence<int, kMaxRestart + 1>{});
  if (nn % 4 != 0 || vstride % 4 != 0) throw std::logic_error("Arnoldi vectors: length and stride multiples of 4");
  if (flags && hout) throw std::logic_error("Arnoldi update: flags only on a pass without inner products");
  const unsigned G = slices_for((size_t)nn, F * K);
  const bool fused = hout && j + 1 <= kFusedMaxJ;
  const int NV = (fused ? j + 1 : 0) + 1;
  table[j](dim3(G, F * K), st, (unsigned)nn, K, V, (size_t)vstride, w, hin, fused ? 1 : 0, work, flags);
  if (fused) reduce_cols((int)G, F, K, NV, 0, j + 1, work, hout, st);
  if (nrm2out) reduce_cols((int)G, F, K, NV, NV - 1, 1, work, nrm2out, st);
  PHZ_LAUNCH_CHECK();
  if (hout && !fused) arnoldi_dots<T>(nn, F, K, j, V, vstride, w, hout, work, st);
}

template <typename T>
void scale_cols(long nn, int F, int K, const T* w, const double* scale, T* v, hipStream_t st) {
  if (nn % 4 == 0)
    hipLaunchKernelGGL((k_scale_cols4<T>), dim3(blocks_for(nn / 4, 256), F * K), dim3(256), 0, st, (unsigned)nn, K,
                       w, scale, v);
  else
    hipLaunchKernelGGL((k_scale_cols<T>), dim3(blocks_for(nn, 256), F * K), dim3(256), 0, st, (unsigned)nn, K, w,
                       scale, v);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void combine(long nn, int F, int K, const T* V, long vstride, const double* y, const int* kused, T* t, hipStream_t st) {
  if (nn % 4 == 0 && vstride % 4 == 0)
    hipLaunchKernelGGL((k_combine4<T>), dim3(blocks_for(nn / 4, 256), F * K), dim3(256), 0, st, (unsigned)nn, K, V,
                       (size_t)vstride, y, kused, t);
  else
    hipLaunchKernelGGL((k_combine<T>), dim3(blocks_for(nn, 256), F * K), dim3(256), 0, st, (unsigned)nn, K, V,
                       (size_t)vstride, y, kused, t);
  PHZ_LAUNCH_CHECK();
}

template <typename Tx, typename Tz>
void axpy_cols(long nn, int F, int K, const double* a, const Tz* z, Tx* x, hipStream_t st) {
  if (nn % 4 == 0)
    hipLaunchKernelGGL((k_axpy_cols4<Tx, Tz>), dim3(blocks_for(nn / 4, 256), F * K), dim3(256), 0, st, (unsigned)nn,
                       K, a, z, x);
  else
    hipLaunchKernelGGL((k_axpy_cols<Tx, Tz>), dim3(blocks_for(nn, 256), F * K), dim3(256), 0, st, (unsigned)nn, K, a,
                       z, x);
  PHZ_LAUNCH_CHECK();
}

void extract_column(long nn, int load, const double* block, double* col, hipStream_t st) {
  hipLaunchKernelGGL(k_extract_col, dim3(blocks_for(nn, 256), 4), dim3(256), 0, st, (unsigned)nn, load, block, col);
  PHZ_LAUNCH_CHECK();
}
void insert_column(long nn, int load, const double* col, double* block, hipStream_t st) {
  hipLaunchKernelGGL(k_insert_col, dim3(blocks_for(nn, 256), 4), dim3(256), 0, st, (unsigned)nn, load, col, block);
  PHZ_LAUNCH_CHECK();
}
void soa_to_aos(long nn, int ncol, const double* src, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_soa_to_aos, dim3(blocks_for((size_t)nn * ncol, 256)), dim3(256), 0, st, (unsigned)nn, ncol, src,
                     dst);
  PHZ_LAUNCH_CHECK();
}
void aos_to_soa(long nn, int ncol, const double* src, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_aos_to_soa, dim3(blocks_for((size_t)nn * ncol, 256)), dim3(256), 0, st, (unsigned)nn, ncol, src,
                     dst);
  PHZ_LAUNCH_CHECK();
}

void gmres_start(int nrhs, const double* nrm2, double rtol, GmresState s, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_start, dim3(1), dim3(64), 0, st, nrhs, nrm2, rtol, s);
  PHZ_LAUNCH_CHECK();
}
void gmres_givens(int nrhs, int m, int j, const double* h1, const double* h2, const double* nrm2, double rtol,
                  double stall, GmresState s, hipStream_t st, const int* flag, const double* na2) {
  hipLaunchKernelGGL(k_gmres_givens, dim3(1), dim3(64), 0, st, nrhs, m, j, h1, h2, nrm2, rtol, stall, s, flag, na2);
  PHZ_LAUNCH_CHECK();
}
void reorth_decide(int K, int J, double tau2, double* h2, const double* na2, const int* active, int* flag, int* count,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_reorth_decide, dim3(1), dim3(64), 0, st, K, J, tau2, h2, na2, active, flag, count);
  PHZ_LAUNCH_CHECK();
}
void gmres_solve_y(int nrhs, int m, GmresState s, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_solve_y, dim3(1), dim3(64), 0, st, nrhs, m, s);
  PHZ_LAUNCH_CHECK();
}

void levelset_to_scale(int N, const double* phi, double eta, double void_scale, double* rho, double* s, float* s32,
                       hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  hipLaunchKernelGGL(k_levelset_to_scale, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)N, phi, eta,
                     void_scale, rho, s, s32);
  PHZ_LAUNCH_CHECK();
}
void density_to_scale(long nn, const double* rho, double void_scale, double* s, float* s32, hipStream_t st) {
  hipLaunchKernelGGL(k_density_to_scale, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)nn, rho, void_scale, s,
                     s32);
  PHZ_LAUNCH_CHECK();
}
void levelset_to_scale_qp(int N, const double* phi, double eta, double void_scale, double* rho, double* s,
                          float* s32, double* sq, float* sq32, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  hipLaunchKernelGGL(k_levelset_to_scale_qp, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)N, phi, eta,
                     void_scale, rho, s, s32, sq, sq32);
  PHZ_LAUNCH_CHECK();
}
void point_scales(long nn, const double* s, double* sq, float* sq32, hipStream_t st) {
  hipLaunchKernelGGL(k_point_scales, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)nn, s, sq, sq32);
  PHZ_LAUNCH_CHECK();
}
void build_rhs_qp(int N, const double* sq, const double* F0q, double* b, hipStream_t st, bool absval) {
  const size_t nn = (size_t)N * N * N;
  hipLaunchKernelGGL(k_build_rhs_qp, dim3(blocks_for(nn, 128)), dim3(128), 0, st, (unsigned)N, sq, F0q, b,
                     (int)absval);
  PHZ_LAUNCH_CHECK();
}
void build_rhs(int N, const double* s, const double* F0, double* b, hipStream_t st, bool absval) {
  const size_t nn = (size_t)N * N * N;
  hipLaunchKernelGGL(k_build_rhs, dim3(blocks_for(nn, 128)), dim3(128), 0, st, (unsigned)N, s, F0, b, (int)absval);
  PHZ_LAUNCH_CHECK();
}
void reduce_effective(int N, const double* s, const double* X, double* out, double* work, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  const unsigned G = slices_for(nn, 36);
  hipLaunchKernelGGL(k_reduce_effective, dim3(G, 36), dim3(256), 0, st, (unsigned)N, s, 1, 0, X, work);
  // out[l*36 + col] = sum over slices
  reduce_cols((int)G, 1, 36, 8, 0, 8, work, out, st);
  // out[288] = sum_e s_e
  col_reduce<double, false>(nn, 1, 1, s, out + 288, work, st);
}
void reduce_effective_point(int N, const double* sq, int p, const double* X, double* out, double* work,
                            hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  const unsigned G = slices_for(nn, 36);
  hipLaunchKernelGGL(k_reduce_effective, dim3(G, 36), dim3(256), 0, st, (unsigned)N, sq, 8, p, X, work);
  reduce_cols((int)G, 1, 36, 8, 0, 8, work, out, st);
}
void cross_dots(long nn, const double* X, const double* Y, double* out, double* work, hipStream_t st) {
  const unsigned G = slices_for((size_t)nn, 36);
  hipLaunchKernelGGL(k_cross_dots, dim3(G, 36), dim3(256), 0, st, (unsigned)nn, X, Y, work);
  // out[b*9 + a] = sum_{f, slices} part[((f*9 + a)*G + slice)*9 + b]
  reduce_cols((int)G, 4, 9, 9, 0, 9, work, out, st);
  PHZ_LAUNCH_CHECK();
}
void mix_cols(long nn, const double* X, const double* W, double* U, hipStream_t st) {
  hipLaunchKernelGGL(k_mix_cols, dim3(blocks_for((size_t)nn, 256), 4), dim3(256), 0, st, (unsigned)nn, X, W, U);
  PHZ_LAUNCH_CHECK();
}
void backward_elem(int N, const double* X, const double* U, const double* K0, const double* FW, double cterm,
                   double factor, double* grad, hipStream_t st, int stride, int off) {
  const unsigned nb = ((N + 15) / 16) * ((N + 3) / 4) * ((N + 3) / 4);
  hipLaunchKernelGGL(k_backward_mfma, dim3(nb), dim3(256), 0, st, (unsigned)N, X, U, K0, FW, cterm, factor, stride,
                     off, grad);
  PHZ_LAUNCH_CHECK();
}
void grad_phi_qp(int N, const double* phi, double eta, const double* g, int stride, double* out, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  hipLaunchKernelGGL(k_grad_phi_qp, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)N, phi, eta, g, stride,
                     out);
  PHZ_LAUNCH_CHECK();
}
void sum_points(long nn, const double* gq, double* ge, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_points, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)nn, gq, ge);
  PHZ_LAUNCH_CHECK();
}
void grad_phi(int N, const double* phi, double eta, const double* grad_rho, double* out, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  hipLaunchKernelGGL(k_grad_phi, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)N, phi, eta, grad_rho, out);
  PHZ_LAUNCH_CHECK();
}
void nodal_mean_of_elements(int N, const double* ge, double* vn, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  hipLaunchKernelGGL(k_nodal_mean, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)N, ge, vn);
  PHZ_LAUNCH_CHECK();
}
void max_abs(long count, const double* v, double* out, double* work, hipStream_t st) {
  unsigned g = blocks_for(count, 256);
  if (g > 512) g = 512;
  hipLaunchKernelGGL(k_max_abs, dim3(g), dim3(256), 0, st, (size_t)count, v, work);
  hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(64), 0, st, (int)g, work, out);
  PHZ_LAUNCH_CHECK();
}
int count_nonfinite(long count, const double* v, double* work, hipStream_t st) {
  return count_outside(count, v, -std::numeric_limits<double>::max(), std::numeric_limits<double>::max(), work, st);
}
int count_outside(long count, const double* v, double lo, double hi, double* work, hipStream_t st) {
  unsigned g = blocks_for(count, 256);
  if (g > 512) g = 512;
  hipLaunchKernelGGL(k_count_outside, dim3(g), dim3(256), 0, st, (size_t)count, v, lo, hi, work);
  reduce_cols((int)g, 1, 1, 1, 0, 1, work, work + 1024, st);
  PHZ_LAUNCH_CHECK();
  double h = 0.0;
  PHZ_HIP(hipMemcpyAsync(&h, work + 1024, sizeof(double), hipMemcpyDeviceToHost, st));
  PHZ_HIP(hipStreamSynchronize(st));
  return (int)h;
}
void reinit_step(int N, const double* phi, const double* phi0, double dt, int subcell, double* out, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  hipLaunchKernelGGL(k_reinit_step, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)N, phi, phi0, dt, subcell, out);
  PHZ_LAUNCH_CHECK();
}

void tricg_update(long nn, int F, int K, const double* cf, const double* w, int side, double* g1, double* g2,
                  double* x, hipStream_t st) {
  const size_t count = (size_t)nn * F * K;
  hipLaunchKernelGGL(k_tricg_update, dim3(blocks_for(count, 256)), dim3(256), 0, st, (size_t)nn, count, K, cf, w,
                     side, g1, g2, x);
  PHZ_LAUNCH_CHECK();
}

void stencil_cheb_step(int N, int K, const double* w, const double* d, double* x, double* r, double* dn, double c1,
                       double c2, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  hipLaunchKernelGGL(k_stencil_cheb, dim3(blocks_for(nn, 256), K), dim3(256), 0, st, (unsigned)N, w, d, x, r, dn,
                     c1, c2);
  PHZ_LAUNCH_CHECK();
}

void hj_step(int N, const double* phi, const double* v, const double* vmax, double dt, double* out, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  hipLaunchKernelGGL(k_hj_step, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)N, phi, v, vmax, dt, out);
  PHZ_LAUNCH_CHECK();
}
template <typename T>
void normalize_by(long count, const double* nrm2, const T* w, T* v, hipStream_t st) {
  hipLaunchKernelGGL((k_normalize_by<T>), dim3(blocks_for(count, 256)), dim3(256), 0, st, (size_t)count, nrm2, w, v);
  PHZ_LAUNCH_CHECK();
}
void hash_fill(long count, unsigned seed, double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_hash_fill, dim3(blocks_for(count, 256)), dim3(256), 0, st, (size_t)count, seed, v);
  PHZ_LAUNCH_CHECK();
}

#define PHZ_VINST(T)                                                                                          \
  template void fill<T>(long, T, T*, hipStream_t);                                                            \
  template void col_norm2<T>(long, int, int, const T*, double*, double*, hipStream_t);                       \
  template void col_dot<T>(long, int, int, const T*, const T*, double*, double*, hipStream_t);               \
  template void xpby_cols<T>(long, int, int, const double*, const T*, T*, hipStream_t);                      \
  template void field_sums<T>(long, int, int, const T*, double*, double*, hipStream_t);                      \
  template void subtract_mean<T>(long, int, int, const double*, T*, hipStream_t);                            \
  template void arnoldi_dots<T>(long, int, int, int, const T*, long, const T*, double*, double*, hipStream_t); \
  template void arnoldi_update<T>(long, int, int, int, const T*, long, T*, const double*, double*, double*,   \
                                  double*, hipStream_t, const int*);                                          \
  template void scale_cols<T>(long, int, int, const T*, const double*, T*, hipStream_t);                     \
  template void combine<T>(long, int, int, const T*, long, const double*, const int*, T*, hipStream_t);      \
  template void normalize_by<T>(long, const double*, const T*, T*, hipStream_t);
PHZ_VINST(double)
PHZ_VINST(float)
#undef PHZ_VINST
template void convert<double, float>(long, const double*, float*, hipStream_t);
template void convert<float, double>(long, const float*, double*, hipStream_t);
template void convert<double, double>(long, const double*, double*, hipStream_t);
template void axpy_cols<double, double>(long, int, int, const double*, const double*, double*, hipStream_t);
template void axpy_cols<double, float>(long, int, int, const double*, const float*, double*, hipStream_t);
template void axpy_cols<float, float>(long, int, int, const double*, const float*, float*, hipStream_t);

}  // namespace phz
