// Vector, reduction, GMRES and per-element physics kernels (gfx950).
//
// Reductions are two-stage and deterministic: every block writes its partial
// sums, one block adds the partials in a fixed order.  Krylov vectors may be
// float or double; every inner product accumulates in double.
#include <cmath>

#include "common.hpp"

namespace phz {

namespace {

constexpr int kRedBlocks = 512;

inline unsigned blocks_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }
inline unsigned red_grid(long n, int bs) {
  long g = (n + bs - 1) / bs;
  if (g > kRedBlocks) g = kRedBlocks;
  if (g < 1) g = 1;
  return (unsigned)g;
}
// block size that is a multiple of `slots` (<= 1024)
inline int slot_block(int slots) { return slots * (1024 / slots); }

__global__ void k_sum_partials(int nblocks, int nvals, const double* __restrict__ part,
                               double* __restrict__ out) {
  for (int v = threadIdx.x; v < nvals; v += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(long)b * nvals + v];
    out[v] = s;
  }
}

// sum (or sum of squares) of a flat array per slot = index % slots
template <typename T, bool SQ>
__global__ void k_flat_sums(long count, int slots, const T* __restrict__ v, double* __restrict__ part) {
  extern __shared__ double lds[];
  const int bs = blockDim.x;
  const int t = threadIdx.x;
  double acc = 0.0;
  for (long idx = (long)blockIdx.x * bs + t; idx < count; idx += (long)gridDim.x * bs) {
    const double x = (double)v[idx];
    acc += SQ ? x * x : x;
  }
  lds[t] = acc;
  __syncthreads();
  if (t < slots) {
    double s = 0.0;
    for (int u = t; u < bs; u += slots) s += lds[u];
    part[(long)blockIdx.x * slots + t] = s;
  }
}

template <typename T, bool SQ>
void flat_sums(long count, int slots, const T* v, double* out, double* work, hipStream_t st) {
  const int bs = slot_block(slots);
  const unsigned g = red_grid(count, bs);
  hipLaunchKernelGGL((k_flat_sums<T, SQ>), dim3(g), dim3(bs), bs * sizeof(double), st, count, slots, v, work);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (int)g, slots, work, out);
  PHZ_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- Arnoldi
template <typename T>
__global__ __launch_bounds__(576) void k_arnoldi_dots(long count, int K, int j, const T* __restrict__ V, long vstride,
                               const T* __restrict__ w, double* __restrict__ part) {
  extern __shared__ double lds[];
  const int bs = blockDim.x, t = threadIdx.x;
  double acc[kMaxRestart + 1];
#pragma unroll
  for (int i = 0; i <= kMaxRestart; ++i) acc[i] = 0.0;
  for (long idx = (long)blockIdx.x * bs + t; idx < count; idx += (long)gridDim.x * bs) {
    const double wv = (double)w[idx];
#pragma unroll
    for (int i = 0; i <= kMaxRestart; ++i)
      if (i <= j) acc[i] += (double)V[(long)i * vstride + idx] * wv;
  }
  const int nv = (j + 1) * K;
  for (int i = 0; i <= j; ++i) {
    double a = 0.0;
#pragma unroll
    for (int u = 0; u <= kMaxRestart; ++u)
      if (u == i) a = acc[u];
    lds[t] = a;
    __syncthreads();
    if (t < K) {
      double s = 0.0;
      for (int u = t; u < bs; u += K) s += lds[u];
      part[(long)blockIdx.x * nv + i * K + t] = s;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(576) void k_arnoldi_update(long count, int K, int j, const T* __restrict__ V, long vstride,
                                 T* __restrict__ w, const double* __restrict__ hin, int want_dots,
                                 double* __restrict__ part) {
  extern __shared__ double lds[];
  const int bs = blockDim.x, t = threadIdx.x;
  const int kk = t % K;  // block size and grid stride are multiples of K
  __shared__ double hs[(kMaxRestart + 1) * 9];
  for (int u = t; u < (j + 1) * K; u += bs) hs[u] = hin[u];
  __syncthreads();
  double acc[kMaxRestart + 1];
#pragma unroll
  for (int i = 0; i <= kMaxRestart; ++i) acc[i] = 0.0;
  double nrm = 0.0;
  for (long idx = (long)blockIdx.x * bs + t; idx < count; idx += (long)gridDim.x * bs) {
    double wv = (double)w[idx];
#pragma unroll
    for (int i = 0; i <= kMaxRestart; ++i)
      if (i <= j) wv -= hs[i * K + kk] * (double)V[(long)i * vstride + idx];
    const T wt = (T)wv;
    w[idx] = wt;
    const double wr = (double)wt;
    nrm += wr * wr;
    if (want_dots) {
#pragma unroll
      for (int i = 0; i <= kMaxRestart; ++i)
        if (i <= j) acc[i] += (double)V[(long)i * vstride + idx] * wr;
    }
  }
  const int nv = (want_dots ? (j + 1) : 0) * K + K;
  const int nloop = want_dots ? j + 1 : 0;
  for (int i = 0; i <= nloop; ++i) {
    double a = 0.0;
    if (i == nloop) a = nrm;
    else {
#pragma unroll
      for (int u = 0; u <= kMaxRestart; ++u)
        if (u == i) a = acc[u];
    }
    lds[t] = a;
    __syncthreads();
    if (t < K) {
      double s = 0.0;
      for (int u = t; u < bs; u += K) s += lds[u];
      part[(long)blockIdx.x * nv + i * K + t] = s;
    }
    __syncthreads();
  }
}

__global__ void k_split_partials(int nblocks, int nv, int ndots, const double* __restrict__ part,
                                 double* __restrict__ hout, double* __restrict__ nrmout) {
  for (int v = threadIdx.x; v < nv; v += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(long)b * nv + v];
    if (v < ndots) {
      if (hout) hout[v] = s;
    } else if (nrmout) {
      nrmout[v - ndots] = s;
    }
  }
}

template <typename T>
__global__ void k_scale_cols(long count, int K, const T* __restrict__ w, const double* __restrict__ scale,
                             T* __restrict__ v) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  v[idx] = (T)((double)w[idx] * scale[idx % K]);
}

template <typename T>
__global__ void k_combine(long count, int K, int m, const T* __restrict__ V, long vstride,
                          const double* __restrict__ y, const int* __restrict__ kused, T* __restrict__ t) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const int kk = (int)(idx % K);
  const int ku = kused[kk];
  double s = 0.0;
  for (int i = 0; i < ku; ++i) s += y[i * K + kk] * (double)V[(long)i * vstride + idx];
  t[idx] = (T)s;
}

template <typename Tx, typename Tz>
__global__ void k_axpy_cols(long count, int K, const double* __restrict__ a, const Tz* __restrict__ z,
                            Tx* __restrict__ x) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const double av = a ? a[idx % K] : 1.0;
  x[idx] = (Tx)((double)x[idx] + av * (double)z[idx]);
}

template <typename Ts, typename Td>
__global__ void k_convert(long count, const Ts* __restrict__ s, Td* __restrict__ d) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) d[idx] = (Td)s[idx];
}

template <typename T>
__global__ void k_fill(long count, T v, T* __restrict__ d) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) d[idx] = v;
}

template <typename T>
__global__ void k_subtract_mean(long nn, int FK, const double* __restrict__ sums, T* __restrict__ v) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn * FK) return;
  v[idx] = (T)((double)v[idx] - sums[idx % FK] / (double)nn);
}

template <typename T>
__global__ void k_split(long nn, int K, const T* __restrict__ full, T* __restrict__ u, T* __restrict__ p) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn * 4 * K) return;
  const long n = idx / (4 * K);
  const int r = (int)(idx % (4 * K));
  const int f = r / K, kk = r % K;
  if (f < 3) u[n * 3 * K + f * K + kk] = full[idx];
  else p[n * K + kk] = full[idx];
}

template <typename T>
__global__ void k_merge(long nn, int K, const T* __restrict__ u, const T* __restrict__ p, T* __restrict__ full) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn * 4 * K) return;
  const long n = idx / (4 * K);
  const int r = (int)(idx % (4 * K));
  const int f = r / K, kk = r % K;
  full[idx] = f < 3 ? u[n * 3 * K + f * K + kk] : p[n * K + kk];
}

__global__ void k_extract_col(long nn, int load, const double* __restrict__ block, double* __restrict__ col) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn * 4) return;
  col[idx] = block[idx * 9 + load];
}

__global__ void k_insert_col(long nn, int load, const double* __restrict__ col, double* __restrict__ block) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn * 4) return;
  block[idx * 9 + load] = col[idx];
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
    const int act = (bn > 0.0) && (beta > rtol * bn) && isfinite(beta);
    s.active[k] = act;
    s.kused[k] = 0;
    s.scale[k] = act ? 1.0 / beta : 0.0;
    if (act) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) s.nactive[0] = cnt;
}

__global__ void k_gmres_givens(int K, int m, int j, const double* __restrict__ h1, const double* __restrict__ h2,
                               const double* __restrict__ nrm2, double rtol, GmresState s) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const int k = threadIdx.x;
  if (k < K && s.active[k]) {
    double col[kMaxRestart + 1];
    for (int i = 0; i <= j; ++i) col[i] = h1[i * K + k] + (h2 ? h2[i * K + k] : 0.0);
    const double hn = sqrt(nrm2[k]);
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
    for (int i = 0; i <= j; ++i) s.H[((long)i * m + j) * K + k] = col[i];
    const double gj = s.g[j * K + k];
    s.g[(j + 1) * K + k] = -sn * gj;
    s.g[j * K + k] = c * gj;
    const double est = fabs(s.g[(j + 1) * K + k]) / s.bnorm[k];
    s.est[j * K + k] = est;
    const bool stop = !(est > rtol) || !(hn > 1e-300 * den) || (j + 1 == m) || !isfinite(est);
    if (stop) {
      s.active[k] = 0;
      s.kused[k] = j + 1;
      s.scale[k] = 0.0;
    } else {
      s.kused[k] = j + 1;
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
    for (int c = i + 1; c < ku; ++c) v -= s.H[((long)i * m + c) * K + k] * s.y[c * K + k];
    const double d = s.H[((long)i * m + i) * K + k];
    s.y[i * K + k] = d != 0.0 ? v / d : 0.0;
  }
}

// ---------------------------------------------------------------- physics
struct Nb {
  int i, j, k, im, jm, km, ip, jp, kp;
};
__device__ __forceinline__ Nb nbr(long n, int N) {
  Nb r;
  r.i = (int)(n % N);
  r.j = (int)((n / N) % N);
  r.k = (int)(n / ((long)N * N));
  r.im = r.i ? r.i - 1 : N - 1;
  r.jm = r.j ? r.j - 1 : N - 1;
  r.km = r.k ? r.k - 1 : N - 1;
  r.ip = r.i + 1 < N ? r.i + 1 : 0;
  r.jp = r.j + 1 < N ? r.j + 1 : 0;
  r.kp = r.k + 1 < N ? r.k + 1 : 0;
  return r;
}
__device__ __forceinline__ long at(int N, int i, int j, int k) { return (long)i + (long)N * (j + (long)N * k); }

// element e with origin (i,j,k): corner c is node (i + cx, j + cy, k + cz)
__device__ __forceinline__ long corner_node(const Nb& q, int N, int c) {
  return at(N, (c & 1) ? q.ip : q.i, (c & 2) ? q.jp : q.j, (c & 4) ? q.kp : q.k);
}
// node n is corner c of element with origin n - c
__device__ __forceinline__ long elem_of_corner(const Nb& q, int N, int c) {
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

__global__ void k_levelset_to_scale(int N, const double* __restrict__ phi, double eta, double ev,
                                    double* __restrict__ rho, double* __restrict__ s, float* __restrict__ s32) {
  const long nn = (long)N * N * N;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
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

__global__ void k_density_to_scale(long nn, const double* __restrict__ rho, double ev, double* __restrict__ s,
                                   float* __restrict__ s32) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const double sv = ev + (1.0 - ev) * rho[e];
  s[e] = sv;
  s32[e] = (float)sv;
}

__global__ void k_build_rhs(int N, const double* __restrict__ s, const double* __restrict__ F0,
                            double* __restrict__ b, int absval) {
  const long nn = (long)N * N * N;
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const Nb q = nbr(n, N);
  double acc[36];
  for (int t = 0; t < 36; ++t) acc[t] = 0.0;
  for (int c = 0; c < 8; ++c) {
    const double se = s[elem_of_corner(q, N, c)];
    for (int f = 0; f < 4; ++f)
      for (int L = 0; L < 9; ++L) {
        const double v = F0[(4 * c + f) * 9 + L];
        acc[f * 9 + L] -= se * (absval ? -fabs(v) : v);
      }
  }
  for (int t = 0; t < 36; ++t) b[n * 36 + t] = acc[t];
}

// Y[(l, p)] = sum_n s_{n - c(l)} X[n][p], p = f*9 + L; plus sum_e s_e
__global__ void k_reduce_effective(int N, const double* __restrict__ s, const double* __restrict__ X,
                                   double* __restrict__ part) {
  __shared__ double lds[576 * 9];
  const long nn = (long)N * N * N;
  const int t = threadIdx.x;  // 576 = 16 nodes x 36 values
  const int p = t % 36, qo = t / 36;
  double acc[9];
  for (int u = 0; u < 9; ++u) acc[u] = 0.0;
  for (long n = (long)blockIdx.x * 16 + qo; n < nn; n += (long)gridDim.x * 16) {
    const Nb q = nbr(n, N);
    const double xv = X[n * 36 + p];
    for (int l = 0; l < 8; ++l) acc[l] += s[elem_of_corner(q, N, l)] * xv;
    if (p == 0) acc[8] += s[n];
  }
  for (int u = 0; u < 9; ++u) lds[u * 576 + t] = acc[u];
  __syncthreads();
  for (int v = t; v < 289; v += blockDim.x) {
    double sum = 0.0;
    if (v < 288) {
      const int l = v / 36, pp = v % 36;
      for (int qq = 0; qq < 16; ++qq) sum += lds[l * 576 + qq * 36 + pp];
    } else {
      for (int qq = 0; qq < 16; ++qq) sum += lds[8 * 576 + qq * 36];
    }
    part[(long)blockIdx.x * 289 + v] = sum;
  }
}

// dJ/drho_e = factor * ( cterm + <X_e, FW> + sum_{l,l'} <K0[l,l'], (x_l W) x_l'^T> )
__global__ __launch_bounds__(128) void k_backward(int N, const double* __restrict__ X, const double* __restrict__ K0,
                                                  const double* __restrict__ FW, const double* __restrict__ W,
                                                  double cterm, double factor, double* __restrict__ grad) {
  const long nn = (long)N * N * N;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const Nb q = nbr(e, N);
  double total = cterm;
  for (int l = 0; l < 8; ++l) {
    const double* xl = X + corner_node(q, N, l) * 36;
    double u[36];  // u = x_l W  (4 x 9)
    for (int f = 0; f < 4; ++f) {
      for (int L = 0; L < 9; ++L) {
        double v = 0.0;
        for (int Kk = 0; Kk < 9; ++Kk) v += xl[f * 9 + Kk] * W[Kk * 9 + L];
        u[f * 9 + L] = v;
      }
    }
    for (int f = 0; f < 4; ++f)
      for (int L = 0; L < 9; ++L) total += xl[f * 9 + L] * FW[(4 * l + f) * 9 + L];
    for (int lp = 0; lp < 8; ++lp) {
      const double* xm = X + corner_node(q, N, lp) * 36;
      for (int f = 0; f < 4; ++f)
        for (int fp = 0; fp < 4; ++fp) {
          double v = 0.0;
          for (int L = 0; L < 9; ++L) v += u[f * 9 + L] * xm[fp * 9 + L];
          total += K0[(4 * l + f) * 32 + 4 * lp + fp] * v;
        }
    }
  }
  grad[e] = factor * total;
}

__global__ void k_grad_phi(int N, const double* __restrict__ phi, double eta, const double* __restrict__ grho,
                           double* __restrict__ out) {
  const long nn = (long)N * N * N;
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const Nb q = nbr(n, N);
  double acc = 0.0;
  for (int c = 0; c < 8; ++c) {
    const long e = elem_of_corner(q, N, c);
    const Nb qe = nbr(e, N);
    double m = 0.0;
    for (int cc = 0; cc < 8; ++cc) m += phi[corner_node(qe, N, cc)];
    m *= 0.125;
    acc -= sheaviside_d(m, eta) * grho[e];
  }
  out[n] = acc * 0.125;
}

__global__ void k_nodal_mean(int N, const double* __restrict__ ge, double* __restrict__ vn) {
  const long nn = (long)N * N * N;
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const Nb q = nbr(n, N);
  double acc = 0.0;
  for (int c = 0; c < 8; ++c) acc += ge[elem_of_corner(q, N, c)];
  vn[n] = acc * 0.125;
}

__global__ void k_max_abs(long count, const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double lds[256];
  double m = 0.0;
  for (long idx = (long)blockIdx.x * 256 + threadIdx.x; idx < count; idx += (long)gridDim.x * 256)
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

__global__ void k_count_nonfinite(long count, const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double lds[256];
  double c = 0.0;
  for (long idx = (long)blockIdx.x * 256 + threadIdx.x; idx < count; idx += (long)gridDim.x * 256)
    c += isfinite(v[idx]) ? 0.0 : 1.0;
  lds[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = lds[0];
}

__global__ void k_hj_step(int N, const double* __restrict__ phi, const double* __restrict__ v,
                          const double* __restrict__ vmax, double dt, double* __restrict__ out) {
  const long nn = (long)N * N * N;
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
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

template <typename T>
__global__ void k_normalize_by(long count, const double* __restrict__ nrm2, const T* __restrict__ w, T* __restrict__ v) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const double nr = sqrt(nrm2[0]);
  v[idx] = (T)(nr > 0.0 ? (double)w[idx] / nr : 0.0);
}

__global__ void k_hash_fill(long count, unsigned seed, double* __restrict__ v) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  unsigned long long z = (unsigned long long)idx * 0x9E3779B97F4A7C15ULL + seed;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  v[idx] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

}  // namespace

size_t reduce_work_size(int nvals) { return (size_t)kRedBlocks * (size_t)nvals; }

template <typename Ts, typename Td>
void convert(long count, const Ts* src, Td* dst, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_convert<Ts, Td>), dim3(blocks_for(count, 256)), dim3(256), 0, st, count, src, dst);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void fill(long count, T value, T* dst, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_fill<T>), dim3(blocks_for(count, 256)), dim3(256), 0, st, count, value, dst);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void col_norm2(long rows, int nrhs, const T* v, double* out, double* work, hipStream_t st) {
  flat_sums<T, true>(rows * nrhs, nrhs, v, out, work, st);
}

template <typename T>
void field_sums(long nn, int F, int nrhs, const T* v, double* out, double* work, hipStream_t st) {
  flat_sums<T, false>(nn * F * nrhs, F * nrhs, v, out, work, st);
}

template <typename T>
void subtract_mean(long nn, int F, int nrhs, const double* sums, T* v, hipStream_t st) {
  const long count = nn * F * nrhs;
  hipLaunchKernelGGL((k_subtract_mean<T>), dim3(blocks_for(count, 256)), dim3(256), 0, st, nn, F * nrhs, sums, v);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void arnoldi_dots(long rows, int nrhs, int j, const T* V, long vstride, const T* w, double* hout, double* work,
                  hipStream_t st) {
  const long count = rows * nrhs;
  const int bs = nrhs == 1 ? 256 : 64 * nrhs;
  const unsigned g = red_grid(count, bs);
  const int nv = (j + 1) * nrhs;
  hipLaunchKernelGGL((k_arnoldi_dots<T>), dim3(g), dim3(bs), bs * sizeof(double), st, count, nrhs, j, V, vstride, w,
                     work);
  hipLaunchKernelGGL(k_split_partials, dim3(1), dim3(256), 0, st, (int)g, nv, nv, work, hout, (double*)nullptr);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void arnoldi_update(long rows, int nrhs, int j, const T* V, long vstride, T* w, const double* hin, double* hout,
                    double* nrm2out, double* work, hipStream_t st) {
  const long count = rows * nrhs;
  const int bs = nrhs == 1 ? 256 : 64 * nrhs;
  const unsigned g = red_grid(count, bs);
  const int want = hout ? 1 : 0;
  const int nd = want * (j + 1) * nrhs;
  const int nv = nd + nrhs;
  hipLaunchKernelGGL((k_arnoldi_update<T>), dim3(g), dim3(bs), bs * sizeof(double), st, count, nrhs, j, V, vstride, w,
                     hin, want, work);
  hipLaunchKernelGGL(k_split_partials, dim3(1), dim3(256), 0, st, (int)g, nv, nd, work, hout, nrm2out);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void scale_cols(long rows, int nrhs, const T* w, const double* scale, T* v, hipStream_t st) {
  const long count = rows * nrhs;
  hipLaunchKernelGGL((k_scale_cols<T>), dim3(blocks_for(count, 256)), dim3(256), 0, st, count, nrhs, w, scale, v);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void combine(long rows, int nrhs, int m, const T* V, long vstride, const double* y, const int* kused, T* t,
             hipStream_t st) {
  const long count = rows * nrhs;
  hipLaunchKernelGGL((k_combine<T>), dim3(blocks_for(count, 256)), dim3(256), 0, st, count, nrhs, m, V, vstride, y,
                     kused, t);
  PHZ_LAUNCH_CHECK();
}

template <typename Tx, typename Tz>
void axpy_cols(long rows, int nrhs, const double* a, const Tz* z, Tx* x, hipStream_t st) {
  const long count = rows * nrhs;
  hipLaunchKernelGGL((k_axpy_cols<Tx, Tz>), dim3(blocks_for(count, 256)), dim3(256), 0, st, count, nrhs, a, z, x);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void split_fields(long nn, int nrhs, const T* full, T* u, T* p, hipStream_t st) {
  const long count = nn * 4 * nrhs;
  hipLaunchKernelGGL((k_split<T>), dim3(blocks_for(count, 256)), dim3(256), 0, st, nn, nrhs, full, u, p);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void merge_fields(long nn, int nrhs, const T* u, const T* p, T* full, hipStream_t st) {
  const long count = nn * 4 * nrhs;
  hipLaunchKernelGGL((k_merge<T>), dim3(blocks_for(count, 256)), dim3(256), 0, st, nn, nrhs, u, p, full);
  PHZ_LAUNCH_CHECK();
}

void extract_column(long nn, int load, const double* block, double* col, hipStream_t st) {
  hipLaunchKernelGGL(k_extract_col, dim3(blocks_for(nn * 4, 256)), dim3(256), 0, st, nn, load, block, col);
  PHZ_LAUNCH_CHECK();
}
void insert_column(long nn, int load, const double* col, double* block, hipStream_t st) {
  hipLaunchKernelGGL(k_insert_col, dim3(blocks_for(nn * 4, 256)), dim3(256), 0, st, nn, load, col, block);
  PHZ_LAUNCH_CHECK();
}

void gmres_start(int nrhs, const double* nrm2, double rtol, GmresState s, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_start, dim3(1), dim3(64), 0, st, nrhs, nrm2, rtol, s);
  PHZ_LAUNCH_CHECK();
}
void gmres_givens(int nrhs, int m, int j, const double* h1, const double* h2, const double* nrm2, double rtol,
                  GmresState s, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_givens, dim3(1), dim3(64), 0, st, nrhs, m, j, h1, h2, nrm2, rtol, s);
  PHZ_LAUNCH_CHECK();
}
void gmres_solve_y(int nrhs, int m, GmresState s, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_solve_y, dim3(1), dim3(64), 0, st, nrhs, m, s);
  PHZ_LAUNCH_CHECK();
}

void levelset_to_scale(int N, const double* phi, double eta, double void_scale, double* rho, double* s, float* s32,
                       hipStream_t st) {
  const long nn = (long)N * N * N;
  hipLaunchKernelGGL(k_levelset_to_scale, dim3(blocks_for(nn, 256)), dim3(256), 0, st, N, phi, eta, void_scale, rho,
                     s, s32);
  PHZ_LAUNCH_CHECK();
}
void density_to_scale(long nn, const double* rho, double void_scale, double* s, float* s32, hipStream_t st) {
  hipLaunchKernelGGL(k_density_to_scale, dim3(blocks_for(nn, 256)), dim3(256), 0, st, nn, rho, void_scale, s, s32);
  PHZ_LAUNCH_CHECK();
}
void build_rhs(int N, const double* s, const double* F0, double* b, hipStream_t st, bool absval) {
  const long nn = (long)N * N * N;
  hipLaunchKernelGGL(k_build_rhs, dim3(blocks_for(nn, 128)), dim3(128), 0, st, N, s, F0, b, (int)absval);
  PHZ_LAUNCH_CHECK();
}
void reduce_effective(int N, const double* s, const double* X, double* out, double* work, hipStream_t st) {
  const long nn = (long)N * N * N;
  unsigned g = (unsigned)((nn + 15) / 16);
  if (g > (unsigned)kRedBlocks) g = kRedBlocks;
  hipLaunchKernelGGL(k_reduce_effective, dim3(g), dim3(576), 0, st, N, s, X, work);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(320), 0, st, (int)g, 289, work, out);
  PHZ_LAUNCH_CHECK();
}
void backward_elem(int N, const double* X, const double* K0, const double* FW, double cterm, double factor,
                   double* grad, hipStream_t st) {
  // W (9x9) is stored right after FW (32x9) in the same buffer
  const long nn = (long)N * N * N;
  hipLaunchKernelGGL(k_backward, dim3(blocks_for(nn, 128)), dim3(128), 0, st, N, X, K0, FW, FW + 288, cterm, factor,
                     grad);
  PHZ_LAUNCH_CHECK();
}
void grad_phi(int N, const double* phi, double eta, const double* grad_rho, double* out, hipStream_t st) {
  const long nn = (long)N * N * N;
  hipLaunchKernelGGL(k_grad_phi, dim3(blocks_for(nn, 256)), dim3(256), 0, st, N, phi, eta, grad_rho, out);
  PHZ_LAUNCH_CHECK();
}
void nodal_mean_of_elements(int N, const double* ge, double* vn, hipStream_t st) {
  const long nn = (long)N * N * N;
  hipLaunchKernelGGL(k_nodal_mean, dim3(blocks_for(nn, 256)), dim3(256), 0, st, N, ge, vn);
  PHZ_LAUNCH_CHECK();
}
void max_abs(long count, const double* v, double* out, double* work, hipStream_t st) {
  const unsigned g = red_grid(count, 256);
  hipLaunchKernelGGL(k_max_abs, dim3(g), dim3(256), 0, st, count, v, work);
  hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(64), 0, st, (int)g, work, out);
  PHZ_LAUNCH_CHECK();
}
int count_nonfinite(long count, const double* v, double* work, hipStream_t st) {
  const unsigned g = red_grid(count, 256);
  hipLaunchKernelGGL(k_count_nonfinite, dim3(g), dim3(256), 0, st, count, v, work);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, (int)g, 1, work, work + kRedBlocks);
  PHZ_LAUNCH_CHECK();
  double h = 0.0;
  PHZ_HIP(hipMemcpyAsync(&h, work + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, st));
  PHZ_HIP(hipStreamSynchronize(st));
  return (int)h;
}
void hj_step(int N, const double* phi, const double* v, const double* vmax, double dt, double* out, hipStream_t st) {
  const long nn = (long)N * N * N;
  hipLaunchKernelGGL(k_hj_step, dim3(blocks_for(nn, 256)), dim3(256), 0, st, N, phi, v, vmax, dt, out);
  PHZ_LAUNCH_CHECK();
}
template <typename T>
void normalize_by(long count, const double* nrm2, const T* w, T* v, hipStream_t st) {
  hipLaunchKernelGGL((k_normalize_by<T>), dim3(blocks_for(count, 256)), dim3(256), 0, st, count, nrm2, w, v);
  PHZ_LAUNCH_CHECK();
}
void hash_fill(long count, unsigned seed, double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_hash_fill, dim3(blocks_for(count, 256)), dim3(256), 0, st, count, seed, v);
  PHZ_LAUNCH_CHECK();
}

#define PHZ_VINST(T)                                                                                          \
  template void fill<T>(long, T, T*, hipStream_t);                                                            \
  template void col_norm2<T>(long, int, const T*, double*, double*, hipStream_t);                             \
  template void field_sums<T>(long, int, int, const T*, double*, double*, hipStream_t);                      \
  template void subtract_mean<T>(long, int, int, const double*, T*, hipStream_t);                            \
  template void arnoldi_dots<T>(long, int, int, const T*, long, const T*, double*, double*, hipStream_t);     \
  template void arnoldi_update<T>(long, int, int, const T*, long, T*, const double*, double*, double*,        \
                                  double*, hipStream_t);                                                      \
  template void scale_cols<T>(long, int, const T*, const double*, T*, hipStream_t);                          \
  template void combine<T>(long, int, int, const T*, long, const double*, const int*, T*, hipStream_t);      \
  template void split_fields<T>(long, int, const T*, T*, T*, hipStream_t);                                   \
  template void merge_fields<T>(long, int, const T*, const T*, T*, hipStream_t);                             \
  template void normalize_by<T>(long, const double*, const T*, T*, hipStream_t);
PHZ_VINST(double)
PHZ_VINST(float)
#undef PHZ_VINST
template void convert<double, float>(long, const double*, float*, hipStream_t);
template void convert<float, double>(long, const float*, double*, hipStream_t);
template void convert<double, double>(long, const double*, double*, hipStream_t);
template void axpy_cols<double, double>(long, int, const double*, const double*, double*, hipStream_t);
template void axpy_cols<double, float>(long, int, const double*, const float*, double*, hipStream_t);
template void axpy_cols<float, float>(long, int, const double*, const float*, float*, hipStream_t);

}  // namespace phz
