// Operator and multigrid kernels for the periodic hex8 cell (gfx950).
//
// Fine level (matrix-free): the assembled operator of Sec. 2.5 is
// sum_e s_e K0 with the reference element matrix K0.  One thread owns one
// output node n and gathers its 27 neighbours m = n + d: the 4x4 (or
// sub-block) coupling between n and m is
//     K_nm = sum_{elements e containing n and m} s_e K0[corner(n, e), corner(m, e)],
// built in registers from the eight element scales around n and applied to
// all load columns of x[m].  Every output is written by exactly one thread:
// no scatter, no atomics, deterministic.  The block build costs 64*FO*FI
// FMAs per node independent of the number of load columns, the apply
// 27*FO*FI*K, so batching the nine loads halves the work of the element-wise
// product (which would cost 64*FO*FI*K).
//
// Coarse levels: Galerkin element matrices (R A P assembled per coarse
// element from its eight children) stored as [corner][element][F][8F] and
// applied with the same owner-computes gather.
#include "common.hpp"

namespace phz {

namespace {

struct NodeIdx {
  int i, j, k;
  int im, ip, jm, jp, km, kp;
};

__device__ __forceinline__ NodeIdx node_idx(long n, int N) {
  NodeIdx r;
  r.i = (int)(n % N);
  long t = n / N;
  r.j = (int)(t % N);
  r.k = (int)(t / N);
  r.im = r.i == 0 ? N - 1 : r.i - 1;
  r.ip = r.i + 1 == N ? 0 : r.i + 1;
  r.jm = r.j == 0 ? N - 1 : r.j - 1;
  r.jp = r.j + 1 == N ? 0 : r.j + 1;
  r.km = r.k == 0 ? N - 1 : r.k - 1;
  r.kp = r.k + 1 == N ? 0 : r.k + 1;
  return r;
}

__device__ __forceinline__ int pick(int d, int m, int c, int p) { return d < 0 ? m : (d > 0 ? p : c); }

__device__ __forceinline__ long nb_node(const NodeIdx& q, int N, int dx, int dy, int dz) {
  return (long)pick(dx, q.im, q.i, q.ip) +
         (long)N * ((long)pick(dy, q.jm, q.j, q.jp) + (long)N * pick(dz, q.km, q.k, q.kp));
}

template <int OP> struct OpFields;
template <> struct OpFields<0> { static constexpr int FO = 4, FI = 4; };
template <> struct OpFields<1> { static constexpr int FO = 3, FI = 3; };
template <> struct OpFields<2> { static constexpr int FO = 1, FI = 3; };
template <> struct OpFields<3> { static constexpr int FO = 1, FI = 1; };

template <typename T, int FO, int FI, int K>
__global__ __launch_bounds__(256) void k_fine_apply(int N, const T* __restrict__ s,
                                                    const T* __restrict__ kref,
                                                    const T* __restrict__ x,
                                                    const T* __restrict__ yin,
                                                    T* __restrict__ y, T alpha, T beta) {
  const long nn = (long)N * N * N;
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const NodeIdx q = node_idx(n, N);
  // scale of the element whose corner c is this node (origin n - c)
  T se[8];
#pragma unroll
  for (int c = 0; c < 8; ++c)
    se[c] = s[nb_node(q, N, -(c & 1), -((c >> 1) & 1), -((c >> 2) & 1))];

  T acc[FO * K];
#pragma unroll
  for (int t = 0; t < FO * K; ++t) acc[t] = T(0);

#pragma unroll
  for (int d = 0; d < 27; ++d) {
    const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
    T blk[FO * FI];
#pragma unroll
    for (int t = 0; t < FO * FI; ++t) blk[t] = T(0);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int mx = (c & 1) + dx, my = ((c >> 1) & 1) + dy, mz = ((c >> 2) & 1) + dz;
      if (mx < 0 || mx > 1 || my < 0 || my > 1 || mz < 0 || mz > 1) continue;
      const int lm = mx + 2 * my + 4 * mz;
#pragma unroll
      for (int fo = 0; fo < FO; ++fo)
#pragma unroll
        for (int fi = 0; fi < FI; ++fi)
          blk[fo * FI + fi] += se[c] * kref[(c * FO + fo) * (8 * FI) + lm * FI + fi];
    }
    const T* xm = x + nb_node(q, N, dx, dy, dz) * (FI * K);
#pragma unroll
    for (int fi = 0; fi < FI; ++fi)
#pragma unroll
      for (int kk = 0; kk < K; ++kk) {
        const T xv = xm[fi * K + kk];
#pragma unroll
        for (int fo = 0; fo < FO; ++fo) acc[fo * K + kk] += blk[fo * FI + fi] * xv;
      }
  }
  T* yo = y + n * (FO * K);
  if (beta == T(0)) {
#pragma unroll
    for (int t = 0; t < FO * K; ++t) yo[t] = alpha * acc[t];
  } else {
    const T* yi = yin + n * (FO * K);
#pragma unroll
    for (int t = 0; t < FO * K; ++t) yo[t] = beta * yi[t] + alpha * acc[t];
  }
}

template <typename T, int F, int K>
__global__ __launch_bounds__(256) void k_coarse_apply(int N, const T* __restrict__ Ae,
                                                      const T* __restrict__ x,
                                                      const T* __restrict__ yin,
                                                      T* __restrict__ y, T alpha, T beta) {
  constexpr int S = 8 * F;
  const long nn = (long)N * N * N;
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const NodeIdx q = node_idx(n, N);
  T acc[F * K];
#pragma unroll
  for (int t = 0; t < F * K; ++t) acc[t] = T(0);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
    const long e = nb_node(q, N, -cx, -cy, -cz);
    const T* rows = Ae + ((long)c * nn + e) * (F * S);
#pragma unroll
    for (int lp = 0; lp < 8; ++lp) {
      const int dx = (lp & 1) - cx, dy = ((lp >> 1) & 1) - cy, dz = ((lp >> 2) & 1) - cz;
      const T* xm = x + nb_node(q, N, dx, dy, dz) * (F * K);
#pragma unroll
      for (int fi = 0; fi < F; ++fi)
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
          const T xv = xm[fi * K + kk];
#pragma unroll
          for (int fo = 0; fo < F; ++fo) acc[fo * K + kk] += rows[fo * S + lp * F + fi] * xv;
        }
    }
  }
  T* yo = y + n * (F * K);
  if (beta == T(0)) {
#pragma unroll
    for (int t = 0; t < F * K; ++t) yo[t] = alpha * acc[t];
  } else {
    const T* yi = yin + n * (F * K);
#pragma unroll
    for (int t = 0; t < F * K; ++t) yo[t] = beta * yi[t] + alpha * acc[t];
  }
}

// trilinear weight of coarse local node L at fine local node l of child cp
__device__ __forceinline__ double qweight(int cp, int l, int L) {
  double w = 1.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double xi = 0.5 * (double)(((cp >> d) & 1) + ((l >> d) & 1));
    w *= ((L >> d) & 1) ? xi : 1.0 - xi;
  }
  return w;
}

template <int F>
__global__ void k_galerkin(int Nf, const double* __restrict__ s, const double* __restrict__ kref,
                           const double* __restrict__ Afine, double* __restrict__ Acoarse) {
  constexpr int S = 8 * F;
  __shared__ double Kc[S * S];
  __shared__ double T1[S * S];
  const int Nc = Nf / 2;
  const long nec = (long)Nc * Nc * Nc;
  const long nef = (long)Nf * Nf * Nf;
  const long E = blockIdx.x;
  const int I = (int)(E % Nc), J = (int)((E / Nc) % Nc), Kk = (int)(E / ((long)Nc * Nc));
  double acc[(S * S + 63) / 64];
  const int per = (S * S + blockDim.x - 1) / blockDim.x;
  for (int u = 0; u < per; ++u) acc[u] = 0.0;
  for (int cp = 0; cp < 8; ++cp) {
    const long ef = (long)(2 * I + (cp & 1)) +
                    (long)Nf * ((2 * J + ((cp >> 1) & 1)) + (long)Nf * (2 * Kk + ((cp >> 2) & 1)));
    for (int t = threadIdx.x; t < S * S; t += blockDim.x) {
      const int r = t / S, col = t % S;
      if (s) {
        Kc[t] = s[ef] * kref[t];
      } else {
        const int l = r / F, f = r % F;
        Kc[t] = Afine[(((long)l * nef + ef) * F + f) * S + col];
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < S * S; t += blockDim.x) {
      const int r = t / S, col = t % S;
      const int Lp = col / F, g = col % F;
      double v = 0.0;
      for (int lp = 0; lp < 8; ++lp) v += Kc[r * S + lp * F + g] * qweight(cp, lp, Lp);
      T1[t] = v;
    }
    __syncthreads();
    int u = 0;
    for (int t = threadIdx.x; t < S * S; t += blockDim.x, ++u) {
      const int r = t / S, col = t % S;
      const int L = r / F, f = r % F;
      double v = 0.0;
      for (int l = 0; l < 8; ++l) v += qweight(cp, l, L) * T1[(l * F + f) * S + col];
      acc[u] += v;
    }
    __syncthreads();
  }
  int u = 0;
  for (int t = threadIdx.x; t < S * S; t += blockDim.x, ++u) {
    const int r = t / S, col = t % S;
    const int L = r / F, f = r % F;
    Acoarse[(((long)L * nec + E) * F + f) * S + col] = acc[u];
  }
}

__device__ __forceinline__ void inv3(const double* a, double* o) {
  const double c00 = a[4] * a[8] - a[5] * a[7];
  const double c01 = a[5] * a[6] - a[3] * a[8];
  const double c02 = a[3] * a[7] - a[4] * a[6];
  const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  const double id = 1.0 / det;
  o[0] = c00 * id;
  o[1] = (a[2] * a[7] - a[1] * a[8]) * id;
  o[2] = (a[1] * a[5] - a[2] * a[4]) * id;
  o[3] = c01 * id;
  o[4] = (a[0] * a[8] - a[2] * a[6]) * id;
  o[5] = (a[2] * a[3] - a[0] * a[5]) * id;
  o[6] = c02 * id;
  o[7] = (a[1] * a[6] - a[0] * a[7]) * id;
  o[8] = (a[0] * a[4] - a[1] * a[3]) * id;
}

template <int F>
__global__ void k_diag_fine(int N, const double* __restrict__ s, const double* __restrict__ kref,
                            double* __restrict__ Dinv) {
  const long nn = (long)N * N * N;
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const NodeIdx q = node_idx(n, N);
  double D[F * F];
  for (int t = 0; t < F * F; ++t) D[t] = 0.0;
  for (int c = 0; c < 8; ++c) {
    const double sc = s[nb_node(q, N, -(c & 1), -((c >> 1) & 1), -((c >> 2) & 1))];
    for (int f = 0; f < F; ++f)
      for (int g = 0; g < F; ++g) D[f * F + g] += sc * kref[(c * F + f) * (8 * F) + c * F + g];
  }
  if (F == 1) {
    Dinv[n] = 1.0 / D[0];
  } else {
    double o[9];
    inv3(D, o);
    for (int t = 0; t < 9; ++t) Dinv[n * 9 + t] = o[t];
  }
}

template <int F>
__global__ void k_diag_coarse(int N, const double* __restrict__ Ae, double* __restrict__ Dinv) {
  constexpr int S = 8 * F;
  const long nn = (long)N * N * N;
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const NodeIdx q = node_idx(n, N);
  double D[F * F];
  for (int t = 0; t < F * F; ++t) D[t] = 0.0;
  for (int c = 0; c < 8; ++c) {
    const long e = nb_node(q, N, -(c & 1), -((c >> 1) & 1), -((c >> 2) & 1));
    const double* rows = Ae + ((long)c * nn + e) * (F * S);
    for (int f = 0; f < F; ++f)
      for (int g = 0; g < F; ++g) D[f * F + g] += rows[f * S + c * F + g];
  }
  if (F == 1) {
    Dinv[n] = 1.0 / D[0];
  } else {
    double o[9];
    inv3(D, o);
    for (int t = 0; t < 9; ++t) Dinv[n * 9 + t] = o[t];
  }
}

template <typename T, int F, int K>
__global__ __launch_bounds__(256) void k_cheby(long nn, const T* __restrict__ Dinv,
                                               const T* __restrict__ r, T* __restrict__ d,
                                               T* __restrict__ x, T a, T b, int xzero) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const T* rn = r + n * (F * K);
  T* dn = d + n * (F * K);
  T* xn = x + n * (F * K);
  T Di[F * F];
#pragma unroll
  for (int t = 0; t < F * F; ++t) Di[t] = Dinv[n * (F * F) + t];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    T rv[F];
#pragma unroll
    for (int f = 0; f < F; ++f) rv[f] = rn[f * K + kk];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      T z = T(0);
#pragma unroll
      for (int g = 0; g < F; ++g) z += Di[f * F + g] * rv[g];
      T dv = b * z;
      if (a != T(0)) dv += a * dn[f * K + kk];
      dn[f * K + kk] = dv;
      if (xzero) xn[f * K + kk] = dv;
      else xn[f * K + kk] += dv;
    }
  }
}

// rc[I] = sum_{d in {-1,0,1}^3} prod(1 - |d|/2) rf[2I + d]
template <typename T, int F, int K>
__global__ void k_restrict(int Nc, const T* __restrict__ rf, T* __restrict__ rc) {
  const int Nf = 2 * Nc;
  const long nc = (long)Nc * Nc * Nc;
  const long I = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int ic = (int)(I % Nc), jc = (int)((I / Nc) % Nc), kc = (int)(I / ((long)Nc * Nc));
  T acc[F * K];
#pragma unroll
  for (int t = 0; t < F * K; ++t) acc[t] = T(0);
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const T w = T((dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0));
        const int fi = (2 * ic + dx + Nf) % Nf, fj = (2 * jc + dy + Nf) % Nf,
                  fk = (2 * kc + dz + Nf) % Nf;
        const T* src = rf + ((long)fi + (long)Nf * (fj + (long)Nf * fk)) * (F * K);
#pragma unroll
        for (int t = 0; t < F * K; ++t) acc[t] += w * src[t];
      }
  T* dst = rc + I * (F * K);
#pragma unroll
  for (int t = 0; t < F * K; ++t) dst[t] = acc[t];
}

// xf[i] += sum_I P[i, I] xc[I], fine node i = 2I + c with c in {0,1}^3
template <typename T, int F, int K>
__global__ void k_prolong(int Nc, const T* __restrict__ xc, T* __restrict__ xf) {
  const int Nf = 2 * Nc;
  const long nf = (long)Nf * Nf * Nf;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const int fi = (int)(i % Nf), fj = (int)((i / Nf) % Nf), fk = (int)(i / ((long)Nf * Nf));
  const int bi = fi >> 1, bj = fj >> 1, bk = fk >> 1;
  const int oi = fi & 1, oj = fj & 1, ok = fk & 1;
  T acc[F * K];
#pragma unroll
  for (int t = 0; t < F * K; ++t) acc[t] = T(0);
  for (int c = 0; c < 8; ++c) {
    const int ax = c & 1, ay = (c >> 1) & 1, az = (c >> 2) & 1;
    if ((ax && !oi) || (ay && !oj) || (az && !ok)) continue;
    const T w = T((oi ? 0.5 : 1.0) * (oj ? 0.5 : 1.0) * (ok ? 0.5 : 1.0));
    const long I = (long)((bi + ax) % Nc) + (long)Nc * (((bj + ay) % Nc) + (long)Nc * ((bk + az) % Nc));
    const T* src = xc + I * (F * K);
#pragma unroll
    for (int t = 0; t < F * K; ++t) acc[t] += w * src[t];
  }
  T* dst = xf + i * (F * K);
#pragma unroll
  for (int t = 0; t < F * K; ++t) dst[t] += acc[t];
}

template <typename T>
__global__ void k_dense_apply(int rows, int K, const double* __restrict__ Minv,
                              const T* __restrict__ r, T* __restrict__ z) {
  const int row = blockIdx.x;
  const int kk = threadIdx.y;
  __shared__ double part[9][64];
  double v = 0.0;
  for (int c = threadIdx.x; c < rows; c += 64) v += Minv[(long)row * rows + c] * (double)r[(long)c * K + kk];
  part[kk][threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int t = 0; t < 64; ++t) sum += part[kk][t];
    z[(long)row * K + kk] = (T)sum;
  }
}

inline unsigned blocks_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

template <typename T>
void fine_apply(int op, int nrhs, int N, const T* s, const T* kref, const T* x, const T* yin,
                T* y, T alpha, T beta, hipStream_t st) {
  const long nn = (long)N * N * N;
  const int bs = 128;
  const unsigned g = blocks_for(nn, bs);
#define PHZ_FA(OPV, KV)                                                                    \
  hipLaunchKernelGGL((k_fine_apply<T, OpFields<OPV>::FO, OpFields<OPV>::FI, KV>), dim3(g),  \
                     dim3(bs), 0, st, N, s, kref, x, yin, y, alpha, beta)
  if (nrhs == 1) {
    switch (op) {
      case 0: PHZ_FA(0, 1); break;
      case 1: PHZ_FA(1, 1); break;
      case 2: PHZ_FA(2, 1); break;
      case 3: PHZ_FA(3, 1); break;
      default: throw std::invalid_argument("fine_apply op");
    }
  } else if (nrhs == 9) {
    switch (op) {
      case 0: PHZ_FA(0, 9); break;
      case 1: PHZ_FA(1, 9); break;
      case 2: PHZ_FA(2, 9); break;
      case 3: PHZ_FA(3, 9); break;
      default: throw std::invalid_argument("fine_apply op");
    }
  } else {
    throw std::invalid_argument("fine_apply nrhs");
  }
#undef PHZ_FA
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void coarse_apply(int F, int nrhs, int N, const T* Ae, const T* x, const T* yin, T* y, T alpha,
                  T beta, hipStream_t st) {
  const long nn = (long)N * N * N;
  const int bs = 128;
  const unsigned g = blocks_for(nn, bs);
#define PHZ_CA(FV, KV) \
  hipLaunchKernelGGL((k_coarse_apply<T, FV, KV>), dim3(g), dim3(bs), 0, st, N, Ae, x, yin, y, alpha, beta)
  if (F == 3 && nrhs == 1) PHZ_CA(3, 1);
  else if (F == 3 && nrhs == 9) PHZ_CA(3, 9);
  else if (F == 1 && nrhs == 1) PHZ_CA(1, 1);
  else if (F == 1 && nrhs == 9) PHZ_CA(1, 9);
  else throw std::invalid_argument("coarse_apply");
#undef PHZ_CA
  PHZ_LAUNCH_CHECK();
}

void galerkin_build(int F, int Nf, const double* s, const double* kref, const double* Afine,
                    double* Acoarse, hipStream_t st) {
  const long nec = (long)(Nf / 2) * (Nf / 2) * (Nf / 2);
  if (F == 3) hipLaunchKernelGGL(k_galerkin<3>, dim3((unsigned)nec), dim3(576), 0, st, Nf, s, kref, Afine, Acoarse);
  else if (F == 1) hipLaunchKernelGGL(k_galerkin<1>, dim3((unsigned)nec), dim3(64), 0, st, Nf, s, kref, Afine, Acoarse);
  else throw std::invalid_argument("galerkin F");
  PHZ_LAUNCH_CHECK();
}

void diag_inv_fine(int F, int N, const double* s, const double* kref, double* Dinv, hipStream_t st) {
  const long nn = (long)N * N * N;
  if (F == 3) hipLaunchKernelGGL(k_diag_fine<3>, dim3(blocks_for(nn, 256)), dim3(256), 0, st, N, s, kref, Dinv);
  else hipLaunchKernelGGL(k_diag_fine<1>, dim3(blocks_for(nn, 256)), dim3(256), 0, st, N, s, kref, Dinv);
  PHZ_LAUNCH_CHECK();
}

void diag_inv_coarse(int F, int N, const double* Ae, double* Dinv, hipStream_t st) {
  const long nn = (long)N * N * N;
  if (F == 3) hipLaunchKernelGGL(k_diag_coarse<3>, dim3(blocks_for(nn, 256)), dim3(256), 0, st, N, Ae, Dinv);
  else hipLaunchKernelGGL(k_diag_coarse<1>, dim3(blocks_for(nn, 256)), dim3(256), 0, st, N, Ae, Dinv);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void cheby_step(int F, int nrhs, long nn, const T* Dinv, const T* r, T* d, T* x, T a, T b, bool xzero,
                hipStream_t st) {
  const unsigned g = blocks_for(nn, 256);
#define PHZ_CH(FV, KV) \
  hipLaunchKernelGGL((k_cheby<T, FV, KV>), dim3(g), dim3(256), 0, st, nn, Dinv, r, d, x, a, b, (int)xzero)
  if (F == 3 && nrhs == 1) PHZ_CH(3, 1);
  else if (F == 3 && nrhs == 9) PHZ_CH(3, 9);
  else if (F == 1 && nrhs == 1) PHZ_CH(1, 1);
  else if (F == 1 && nrhs == 9) PHZ_CH(1, 9);
  else throw std::invalid_argument("cheby_step");
#undef PHZ_CH
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void restrict_fw(int F, int nrhs, int Nc, const T* rf, T* rc, hipStream_t st) {
  const long nc = (long)Nc * Nc * Nc;
  const unsigned g = blocks_for(nc, 128);
#define PHZ_RS(FV, KV) hipLaunchKernelGGL((k_restrict<T, FV, KV>), dim3(g), dim3(128), 0, st, Nc, rf, rc)
  if (F == 3 && nrhs == 1) PHZ_RS(3, 1);
  else if (F == 3 && nrhs == 9) PHZ_RS(3, 9);
  else if (F == 1 && nrhs == 1) PHZ_RS(1, 1);
  else if (F == 1 && nrhs == 9) PHZ_RS(1, 9);
  else throw std::invalid_argument("restrict");
#undef PHZ_RS
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void prolong_add(int F, int nrhs, int Nc, const T* xc, T* xf, hipStream_t st) {
  const long nf = 8L * Nc * Nc * Nc;
  const unsigned g = blocks_for(nf, 128);
#define PHZ_PR(FV, KV) hipLaunchKernelGGL((k_prolong<T, FV, KV>), dim3(g), dim3(128), 0, st, Nc, xc, xf)
  if (F == 3 && nrhs == 1) PHZ_PR(3, 1);
  else if (F == 3 && nrhs == 9) PHZ_PR(3, 9);
  else if (F == 1 && nrhs == 1) PHZ_PR(1, 1);
  else if (F == 1 && nrhs == 9) PHZ_PR(1, 9);
  else throw std::invalid_argument("prolong");
#undef PHZ_PR
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void dense_apply(int rows, int nrhs, const double* Minv, const T* r, T* z, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_apply<T>, dim3(rows), dim3(64, nrhs), 0, st, rows, nrhs, Minv, r, z);
  PHZ_LAUNCH_CHECK();
}

#define PHZ_INST(T)                                                                                 \
  template void fine_apply<T>(int, int, int, const T*, const T*, const T*, const T*, T*, T, T,      \
                              hipStream_t);                                                         \
  template void coarse_apply<T>(int, int, int, const T*, const T*, const T*, T*, T, T, hipStream_t); \
  template void cheby_step<T>(int, int, long, const T*, const T*, T*, T*, T, T, bool, hipStream_t); \
  template void restrict_fw<T>(int, int, int, const T*, T*, hipStream_t);                          \
  template void prolong_add<T>(int, int, int, const T*, T*, hipStream_t);                          \
  template void dense_apply<T>(int, int, const double*, const T*, T*, hipStream_t);
PHZ_INST(double)
PHZ_INST(float)
#undef PHZ_INST

}  // namespace phz
