// Operator and multigrid kernels for the periodic hex8 cell (gfx950).
//
// Vector layout (device, internal): structure of arrays, one contiguous
// column of nn node values per (field f, load column k), column index
// f*K + k.  Consecutive threads own consecutive nodes, so every load and
// store below is a unit-stride wavefront access.
//
// Fine level (matrix-free): the assembled operator of Sec. 2.5 is
// sum_e s_e K0 with the reference element matrix K0.  One thread owns one
// output node n and gathers its 27 neighbours m = n + d: the FO x FI coupling
// between n and m is
//     K_nm = sum_{elements e containing n and m} s_e K0[corner(n, e), corner(m, e)],
// built in registers from the eight element scales around n and applied to
// all load columns of x[m].  Every output is written by exactly one thread:
// no scatter, no atomics, deterministic.  The block build costs 64*FO*FI
// FMAs per node independent of the number of load columns, the apply
// 27*FO*FI*K, so batching the nine loads roughly halves the work of the
// element-wise product (64*FO*FI*K).
//
// Coarse levels: Galerkin element matrices (R A P assembled per coarse
// element from its eight children), stored structure-of-arrays as
// [corner L][row f][col][element], applied with the same owner-computes
// gather.
//
// Every square-block operator kernel takes an optional Chebyshev epilogue:
// with r_new = yin - A d_old of a node in registers it also forms
// d_new = ca d_old + cb Dinv r_new and x += d_new for that node, which saves
// a separate pass over r, d and x per smoothing step.
#include "common.hpp"
#include "devutil.hpp"

namespace phz {

namespace {
using namespace dev;

struct NodeIdx {
  unsigned i, j, k, im, ip, jm, jp, km, kp;
};

__device__ __forceinline__ NodeIdx node_idx(unsigned n, unsigned N) {
  NodeIdx r;
  const unsigned t = n / N;
  r.i = n - t * N;
  r.k = t / N;
  r.j = t - r.k * N;
  r.im = r.i == 0 ? N - 1 : r.i - 1;
  r.ip = r.i + 1 == N ? 0 : r.i + 1;
  r.jm = r.j == 0 ? N - 1 : r.j - 1;
  r.jp = r.j + 1 == N ? 0 : r.j + 1;
  r.km = r.k == 0 ? N - 1 : r.k - 1;
  r.kp = r.k + 1 == N ? 0 : r.k + 1;
  return r;
}

__device__ __forceinline__ unsigned pick(int d, unsigned m, unsigned c, unsigned p) {
  return d < 0 ? m : (d > 0 ? p : c);
}

__device__ __forceinline__ unsigned nb_node(const NodeIdx& q, unsigned N, int dx, int dy, int dz) {
  return pick(dx, q.im, q.i, q.ip) + N * (pick(dy, q.jm, q.j, q.jp) + N * pick(dz, q.km, q.k, q.kp));
}

template <int OP> struct OpFields;
template <> struct OpFields<0> { static constexpr int FO = 4, FI = 4; };
template <> struct OpFields<1> { static constexpr int FO = 3, FI = 3; };
template <> struct OpFields<2> { static constexpr int FO = 1, FI = 3; };
template <> struct OpFields<3> { static constexpr int FO = 1, FI = 1; };
template <> struct OpFields<5> { static constexpr int FO = 3, FI = 1; };  // B^T

// Contribution of the neighbour m = n + (dx, dy, dz) to the FO x K outputs of
// node n: its FO x FI stencil block (the reference element blocks of the
// elements shared by n and m, weighted by their scales) times its FI x K
// input columns.
template <typename T, int FO, int FI, int K, bool BUF>
__device__ __forceinline__ void fine_neighbour(unsigned m, int dx, int dy, int dz, unsigned nn, const T* se,
                                               const T* kr, __amdgpu_buffer_rsrc_t xr, const T* __restrict__ x,
                                               T* acc) {
  T xv[FI * K];
#pragma unroll
  for (int col = 0; col < FI * K; ++col) {
    if constexpr (BUF)
      xv[col] = buf_load<T>(xr, m * (unsigned)sizeof(T), (unsigned)(col * nn * sizeof(T)));
    else
      xv[col] = x[(size_t)col * nn + m];
  }
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
      for (int fi = 0; fi < FI; ++fi) blk[fo * FI + fi] += se[c] * kr[(c * FO + fo) * (8 * FI) + lm * FI + fi];
  }
#pragma unroll
  for (int fi = 0; fi < FI; ++fi)
#pragma unroll
    for (int kk = 0; kk < K; ++kk)
#pragma unroll
      for (int fo = 0; fo < FO; ++fo) acc[fo * K + kk] += blk[fo * FI + fi] * xv[fi * K + kk];
}

// Whether the 9 (dy, dz) rows of neighbours run as a runtime loop: that keeps
// the compiler from holding the loads of many neighbours live at once, which
// lowers register use (raising occupancy) for the FP32 A and S blocks; the
// other variants use fewer registers fully unrolled.
template <typename T, int FO, int FI>
constexpr bool fine_row_loop() { return sizeof(T) == 4 && FO == FI && FO != 4; }

// One thread per output node.  The reference block sits in LDS (a broadcast
// read per coefficient, no scalar-register pressure); the 27 neighbour
// records are read with buffer loads, all FI*K columns of a neighbour issued
// before the block build so their latency overlaps it.
template <typename T, int FO, int FI, int K, bool CHEBY, bool BUF>
__global__ __launch_bounds__(128) void k_fine_apply(unsigned N, const T* __restrict__ s,
                                                    const T* __restrict__ kref,
                                                    const T* __restrict__ x, OpArgs<T> a) {
  constexpr int NK = 64 * FO * FI;
  __shared__ T kr[NK];
  for (int t = threadIdx.x; t < NK; t += blockDim.x) kr[t] = kref[t];
  __syncthreads();
  const unsigned nn = N * N * N;
  const unsigned n = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const NodeIdx q = node_idx(n, N);
  // scale of the element whose corner c is this node (origin n - c)
  T se[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) se[c] = s[nb_node(q, N, -(c & 1), -((c >> 1) & 1), -((c >> 2) & 1))];

  __amdgpu_buffer_rsrc_t xr;
  if constexpr (BUF) xr = make_rsrc(x, (unsigned)((size_t)FI * K * nn * sizeof(T)));

  T acc[FO * K];
#pragma unroll
  for (int t = 0; t < FO * K; ++t) acc[t] = T(0);

  if constexpr (fine_row_loop<T, FO, FI>()) {
#pragma unroll 1
    for (int r = 0; r < 9; ++r) {
      const int dy = r % 3 - 1, dz = r / 3 - 1;
      const unsigned ry = dy < 0 ? q.jm : (dy > 0 ? q.jp : q.j);
      const unsigned rz = dz < 0 ? q.km : (dz > 0 ? q.kp : q.k);
      const unsigned rowbase = N * (ry + N * rz);
      fine_neighbour<T, FO, FI, K, BUF>(rowbase + q.im, -1, dy, dz, nn, se, kr, xr, x, acc);
      fine_neighbour<T, FO, FI, K, BUF>(rowbase + q.i, 0, dy, dz, nn, se, kr, xr, x, acc);
      fine_neighbour<T, FO, FI, K, BUF>(rowbase + q.ip, 1, dy, dz, nn, se, kr, xr, x, acc);
    }
  } else {
#pragma unroll
    for (int d = 0; d < 27; ++d) {
      const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
      fine_neighbour<T, FO, FI, K, BUF>(nb_node(q, N, dx, dy, dz), dx, dy, dz, nn, se, kr, xr, x, acc);
    }
  }
  epilogue<T, FO, K, CHEBY>(n, nn, acc, a);
}

// The full operator with the material interpolated at the quadrature points:
// the block of neighbour m sums, over the elements shared with node n and
// their eight Gauss points p, sq[8 e + p] K0q[p] (the per-point reference
// terms, read through the caches: every lane reads the same coefficient).
template <typename T, int K>
__global__ __launch_bounds__(128) void k_fine_apply_qp(unsigned N, const T* __restrict__ sq, const T* __restrict__ kq,
                                                       const T* __restrict__ x, OpArgs<T> a) {
  const unsigned nn = N * N * N;
  const unsigned n = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const NodeIdx q = node_idx(n, N);
  unsigned ec[8];  // element whose corner c is this node (origin n - c)
#pragma unroll
  for (int c = 0; c < 8; ++c) ec[c] = nb_node(q, N, -(c & 1), -((c >> 1) & 1), -((c >> 2) & 1));
  T acc[4 * K];
#pragma unroll
  for (int t = 0; t < 4 * K; ++t) acc[t] = T(0);
#pragma unroll 1
  for (int d = 0; d < 27; ++d) {
    const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
    const unsigned m = nb_node(q, N, dx, dy, dz);
    T xv[4 * K];
#pragma unroll
    for (int col = 0; col < 4 * K; ++col) xv[col] = x[(size_t)col * nn + m];
    T blk[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) blk[t] = T(0);
#pragma unroll 1
    for (int c = 0; c < 8; ++c) {
      const int mx = (c & 1) + dx, my = ((c >> 1) & 1) + dy, mz = ((c >> 2) & 1) + dz;
      if (mx < 0 || mx > 1 || my < 0 || my > 1 || mz < 0 || mz > 1) continue;
      const int lm = mx + 2 * my + 4 * mz;
      const T* sp = sq + (size_t)ec[c] * 8;
#pragma unroll 1
      for (int p = 0; p < 8; ++p) {
        const T sv = sp[p];
        const T* kr = kq + p * 1024 + (c * 4) * 32 + lm * 4;
#pragma unroll
        for (int fo = 0; fo < 4; ++fo)
#pragma unroll
          for (int fi = 0; fi < 4; ++fi) blk[fo * 4 + fi] += sv * kr[fo * 32 + fi];
      }
    }
#pragma unroll
    for (int fi = 0; fi < 4; ++fi)
#pragma unroll
      for (int kk = 0; kk < K; ++kk)
#pragma unroll
        for (int fo = 0; fo < 4; ++fo) acc[fo * K + kk] += blk[fo * 4 + fi] * xv[fi * K + kk];
  }
  epilogue<T, 4, K, false>(n, nn, acc, a);
}

// ---------------------------------------------------------------------------
// LDS-tiled variant of the float32 gather (nine load columns).  A workgroup
// owns a GTX x GTY x GTZ tile of 256 output nodes (one per thread) and first
// stages the tile's input nodes plus a one-node halo, all FI*K columns of
// each, in LDS as rows of CP floats (CP = FI*K rounded up to a multiple of 4,
// so a row is whole 16-byte words and eight consecutive rows of a wave's
// ds_read_b128 phase fall on disjoint banks for CP = 12, 28 and 36).  The 27
// neighbour records of every node are then LDS reads instead of global
// loads; the block build and the epilogue are those of the direct gather.
constexpr int GTX = 16, GTY = 4, GTZ = 4;
constexpr int GNX = GTX + 2, GNY = GTY + 2, GNZ = GTZ + 2, GNI = GNX * GNY * GNZ;

__device__ __forceinline__ unsigned wrap1(int v, unsigned N) {
  return v < 0 ? (unsigned)(v + (int)N) : ((unsigned)v >= N ? (unsigned)v - N : (unsigned)v);
}

// Stage the workgroup's input tile plus a one-node halo (GNI nodes, C
// columns each) in LDS as rows of CP floats.  Every global load of the
// thread's (at most three) staged nodes is issued before the first LDS
// write, so the loads' latencies overlap instead of adding up node by node.
template <int C, int CP>
__device__ __forceinline__ void stage_tile(float4* xs, const float* __restrict__ x, unsigned N, unsigned nn, int x0,
                                           int y0, int z0, int tid) {
  constexpr int PF = (GNI + 255) / 256;
  float v[PF][CP];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    const int q = tid + 256 * p;
    const int li = q % GNX, lj = (q / GNX) % GNY, lk = q / (GNX * GNY);
    const unsigned m = wrap1(x0 - 1 + li, N) + N * (wrap1(y0 - 1 + lj, N) + N * wrap1(z0 - 1 + lk, N));
#pragma unroll
    for (int col = 0; col < CP; ++col) v[p][col] = (q < GNI && col < C) ? x[(size_t)col * nn + m] : 0.f;
  }
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    const int q = tid + 256 * p;
    if (q < GNI) {
#pragma unroll
      for (int c4 = 0; c4 < CP / 4; ++c4)
        xs[q * (CP / 4) + c4] = make_float4(v[p][4 * c4], v[p][4 * c4 + 1], v[p][4 * c4 + 2], v[p][4 * c4 + 3]);
    }
  }
}

template <int FO, int FI, int K, int CP>
__device__ __forceinline__ void tiled_neighbour(const float4* __restrict__ row, int dx, int dy, int dz,
                                                const float* se, const float* kr, float* acc) {
  float xv[CP];
#pragma unroll
  for (int c4 = 0; c4 < CP / 4; ++c4) {
    const float4 v = row[c4];
    xv[4 * c4] = v.x;
    xv[4 * c4 + 1] = v.y;
    xv[4 * c4 + 2] = v.z;
    xv[4 * c4 + 3] = v.w;
  }
  float blk[FO * FI];
#pragma unroll
  for (int t = 0; t < FO * FI; ++t) blk[t] = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int mx = (c & 1) + dx, my = ((c >> 1) & 1) + dy, mz = ((c >> 2) & 1) + dz;
    if (mx < 0 || mx > 1 || my < 0 || my > 1 || mz < 0 || mz > 1) continue;
    const int lm = mx + 2 * my + 4 * mz;
#pragma unroll
    for (int fo = 0; fo < FO; ++fo)
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) blk[fo * FI + fi] += se[c] * kr[(c * FO + fo) * (8 * FI) + lm * FI + fi];
  }
#pragma unroll
  for (int fi = 0; fi < FI; ++fi)
#pragma unroll
    for (int kk = 0; kk < K; ++kk)
#pragma unroll
      for (int fo = 0; fo < FO; ++fo) acc[fo * K + kk] += blk[fo * FI + fi] * xv[fi * K + kk];
}

template <int FO, int FI, int K, bool CHEBY>
__global__ __launch_bounds__(256) void k_fine_tiled(unsigned N, const float* __restrict__ s,
                                                    const float* __restrict__ kref, const float* __restrict__ x,
                                                    OpArgs<float> a) {
  constexpr int C = FI * K, CP = (C + 3) / 4 * 4, NK = 64 * FO * FI;
  __shared__ float kr[NK];
  __shared__ float4 xs[GNI * (CP / 4)];
  const unsigned nn = N * N * N;
  const unsigned ntx = N / GTX, nty = N / GTY;
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int x0 = (int)((b % ntx) * GTX), y0 = (int)(((b / ntx) % nty) * GTY), z0 = (int)((b / (ntx * nty)) * GTZ);
  const int tid = threadIdx.x;
  for (int t = tid; t < NK; t += 256) kr[t] = kref[t];
  stage_tile<C, CP>(xs, x, N, nn, x0, y0, z0, tid);
  const int ti = tid % GTX, tj = (tid / GTX) % GTY, tk = tid / (GTX * GTY);
  const unsigned n = (unsigned)(x0 + ti) + N * ((unsigned)(y0 + tj) + N * (unsigned)(z0 + tk));
  // scale of the element whose corner c is this node (origin n - c)
  float se[8];
#pragma unroll
  for (int c = 0; c < 8; ++c)
    se[c] = s[wrap1(x0 + ti - (c & 1), N) + N * (wrap1(y0 + tj - ((c >> 1) & 1), N) + N * wrap1(z0 + tk - (c >> 2), N))];
  float acc[FO * K];
#pragma unroll
  for (int t = 0; t < FO * K; ++t) acc[t] = 0.f;
  __syncthreads();
  const int qc = (ti + 1) + GNX * ((tj + 1) + GNY * (tk + 1));
  if constexpr (fine_row_loop<float, FO, FI>()) {
#pragma unroll 1
    for (int r = 0; r < 9; ++r) {
      const int dy = r % 3 - 1, dz = r / 3 - 1;
      const float4* row = xs + (qc + GNX * (dy + GNY * dz)) * (CP / 4);
      tiled_neighbour<FO, FI, K, CP>(row - CP / 4, -1, dy, dz, se, kr, acc);
      tiled_neighbour<FO, FI, K, CP>(row, 0, dy, dz, se, kr, acc);
      tiled_neighbour<FO, FI, K, CP>(row + CP / 4, 1, dy, dz, se, kr, acc);
    }
  } else {
#pragma unroll
    for (int d = 0; d < 27; ++d) {
      const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
      tiled_neighbour<FO, FI, K, CP>(xs + (qc + dx + GNX * (dy + GNY * dz)) * (CP / 4), dx, dy, dz, se, kr, acc);
    }
  }
  epilogue<float, FO, K, CHEBY>(n, nn, acc, a);
}

template <int OPV>
void launch_tiled(unsigned N, const float* s, const float* kref, const float* x, const OpArgs<float>& a, bool cheby,
                  hipStream_t st) {
  constexpr int FO = OpFields<OPV>::FO, FI = OpFields<OPV>::FI;
  const unsigned g = (N / GTX) * (N / GTY) * (N / GTZ);
  if constexpr (FO == FI) {
    if (cheby) {
      hipLaunchKernelGGL((k_fine_tiled<FO, FI, 9, true>), dim3(g), dim3(256), 0, st, N, s, kref, x, a);
      return;
    }
  }
  if (cheby) throw std::invalid_argument("Chebyshev epilogue needs a square block");
  hipLaunchKernelGGL((k_fine_tiled<FO, FI, 9, false>), dim3(g), dim3(256), 0, st, N, s, kref, x, a);
}

// LDS-tiled variant of the coarse-level stencil apply (float32, nine load
// columns, one thread per node of a GTX x GTY x GTZ tile).  The direct kernel
// below reads every input value 27 times through the caches, which at 64^3
// and nine columns is more traffic than the L2 delivers at HBM speed; here
// the tile's input nodes plus a one-node halo are staged once in LDS (rows of
// CP floats as in the tiled fine gather) and each node's 27 stencil blocks
// are streamed from HBM once.
//
// COMPACT: the 26 off-centre blocks come as bf16 (S16, [d'][fo][fi][n] with
// d' = d, or d - 1 past the centre d = 13) and the centre block as float32
// minus their sum (Sc, [fo][fi][n]).  A Galerkin operator annihilates
// constants per field pair (every block row sums to zero), and so does the
// stored one, to float32 rounding: the apply equals
// sum_{d != centre} S_d (x_{n+d} - x_n), whose bf16 coefficient error
// (2^-9 relative) scales with the differences across the stencil rather than
// with the values.  About half the stencil bytes per node.
template <int F, bool CHEBY, bool BUF, bool COMPACT>
__global__ __launch_bounds__(256) void k_stencil_tiled(unsigned N, const float* __restrict__ S,
                                                       const unsigned short* __restrict__ S16,
                                                       const float* __restrict__ Sc,
                                                       const float* __restrict__ x, OpArgs<float> a) {
  constexpr int K = 9, C = F * K, CP = (C + 3) / 4 * 4;
  __shared__ float4 xs[GNI * (CP / 4)];
  const unsigned nn = N * N * N;
  const unsigned ntx = N / GTX, nty = N / GTY;
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int x0 = (int)((b % ntx) * GTX), y0 = (int)(((b / ntx) % nty) * GTY), z0 = (int)((b / (ntx * nty)) * GTZ);
  const int tid = threadIdx.x;
  stage_tile<C, CP>(xs, x, N, nn, x0, y0, z0, tid);
  const int ti = tid % GTX, tj = (tid / GTX) % GTY, tk = tid / (GTX * GTY);
  const unsigned n = (unsigned)(x0 + ti) + N * ((unsigned)(y0 + tj) + N * (unsigned)(z0 + tk));
  __amdgpu_buffer_rsrc_t sr;
  if constexpr (BUF) sr = make_rsrc(S, (unsigned)((size_t)27 * F * F * nn * sizeof(float)));
  float acc[F * K];
#pragma unroll
  for (int t = 0; t < F * K; ++t) acc[t] = 0.f;
  __syncthreads();
  const int qc = (ti + 1) + GNX * ((tj + 1) + GNY * (tk + 1));
  // the stencil blocks stream from HBM two neighbours ahead of their use
  auto load_block = [&](int d, float* sv) {
#pragma unroll
    for (int t = 0; t < F * F; ++t) {
      if constexpr (COMPACT) {
        if (d == 13) {
          sv[t] = Sc[(size_t)t * nn + n];
        } else {
          const int dd = d < 13 ? d : d - 1;
          sv[t] = __builtin_bit_cast(float, (unsigned)S16[(size_t)(dd * F * F + t) * nn + n] << 16);
        }
      } else if constexpr (BUF) {
        sv[t] = buf_load<float>(sr, n * (unsigned)sizeof(float), (unsigned)((d * F * F + t) * nn * sizeof(float)));
      } else {
        sv[t] = S[(size_t)(d * F * F + t) * nn + n];
      }
    }
  };
  float sq[3][F * F];
  load_block(0, sq[0]);
  load_block(1, sq[1]);
#pragma unroll
  for (int d = 0; d < 27; ++d) {
    const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
    if (d + 2 < 27) load_block(d + 2, sq[(d + 2) % 3]);
    const float* sv = sq[d % 3];
    const float4* row = xs + (qc + dx + GNX * (dy + GNY * dz)) * (CP / 4);
    float xv[CP];
#pragma unroll
    for (int c4 = 0; c4 < CP / 4; ++c4) {
      const float4 v = row[c4];
      xv[4 * c4] = v.x;
      xv[4 * c4 + 1] = v.y;
      xv[4 * c4 + 2] = v.z;
      xv[4 * c4 + 3] = v.w;
    }
#pragma unroll
    for (int fi = 0; fi < F; ++fi)
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int fo = 0; fo < F; ++fo) acc[fo * K + j] += sv[fo * F + fi] * xv[fi * K + j];
  }
  epilogue_cols<float, F, K, K, CHEBY>(n, nn, 0, acc, a);
}

template <int F>
void launch_stencil_tiled(unsigned N, const float* S, const float* x, const OpArgs<float>& a, bool cheby,
                          hipStream_t st) {
  const unsigned g = (N / GTX) * (N / GTY) * (N / GTZ);
  const bool buf = (size_t)N * N * N * 27 * F * F * sizeof(float) < (size_t(1) << 32);
#define PHZ_ST(CH, BUF) \
  hipLaunchKernelGGL((k_stencil_tiled<F, CH, BUF, false>), dim3(g), dim3(256), 0, st, N, S, nullptr, nullptr, x, a)
  if (cheby) { if (buf) PHZ_ST(true, true); else PHZ_ST(true, false); }
  else { if (buf) PHZ_ST(false, true); else PHZ_ST(false, false); }
#undef PHZ_ST
}

template <int F>
void launch_stencil_tiled_compact(unsigned N, const unsigned short* S16, const float* Sc, const float* x,
                                  const OpArgs<float>& a, bool cheby, hipStream_t st) {
  const unsigned g = (N / GTX) * (N / GTY) * (N / GTZ);
  if (cheby)
    hipLaunchKernelGGL((k_stencil_tiled<F, true, false, true>), dim3(g), dim3(256), 0, st, N, nullptr, S16, Sc, x, a);
  else
    hipLaunchKernelGGL((k_stencil_tiled<F, false, false, true>), dim3(g), dim3(256), 0, st, N, nullptr, S16, Sc, x, a);
}

// Compact form of a level's stencils: the off-centre blocks rounded to bf16
// (nearest even), the centre block minus their rounded sum (accumulated in
// float64, then rounded to float32).
template <int F>
__global__ void k_compact_stencil(unsigned nn, const double* __restrict__ S, unsigned short* __restrict__ S16,
                                  float* __restrict__ Sc) {
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  for (int t = 0; t < F * F; ++t) {
    double sum = 0.0;
    for (int d = 0; d < 27; ++d) {
      if (d == 13) continue;
      const __bf16 h = (__bf16)(float)S[(size_t)(d * F * F + t) * nn + n];
      const unsigned short hb = __builtin_bit_cast(unsigned short, h);
      S16[(size_t)((d < 13 ? d : d - 1) * F * F + t) * nn + n] = hb;
      sum += (double)__builtin_bit_cast(float, (unsigned)hb << 16);
    }
    Sc[(size_t)t * nn + n] = (float)(-sum);
  }
}

// Coarse levels: assembled 27-point node stencils S[(d*F + fo)*F + fi][n]
// (block coupling node n to neighbour d).  KK = K: one thread per node and
// all load columns (large levels: each stencil coefficient read once);
// KK = 1: one thread per (node, load column k = blockIdx.y) for small levels
// where one thread per node would leave most of the chip idle.
template <typename T, int F, int K, int KK, bool CHEBY, bool BUF>
__global__ __launch_bounds__(256) void k_stencil_apply(unsigned N, const T* __restrict__ S,
                                                       const T* __restrict__ x, OpArgs<T> a) {
  const unsigned nn = N * N * N;
  const unsigned n = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int k0 = KK == K ? 0 : (int)blockIdx.y;
  const NodeIdx q = node_idx(n, N);
  __amdgpu_buffer_rsrc_t sr, xr;
  if constexpr (BUF) {
    sr = make_rsrc(S, (unsigned)((size_t)27 * F * F * nn * sizeof(T)));
    xr = make_rsrc(x, (unsigned)((size_t)F * K * nn * sizeof(T)));
  }
  T acc[F * KK];
#pragma unroll
  for (int t = 0; t < F * KK; ++t) acc[t] = T(0);
#pragma unroll
  for (int d = 0; d < 27; ++d) {
    const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
    const unsigned m = nb_node(q, N, dx, dy, dz);
    T sv[F * F], xv[F * KK];
#pragma unroll
    for (int t = 0; t < F * F; ++t) {
      if constexpr (BUF) sv[t] = buf_load<T>(sr, n * (unsigned)sizeof(T), (unsigned)((d * F * F + t) * nn * sizeof(T)));
      else sv[t] = S[(size_t)(d * F * F + t) * nn + n];
    }
#pragma unroll
    for (int fi = 0; fi < F; ++fi)
#pragma unroll
      for (int j = 0; j < KK; ++j) {
        const unsigned col = fi * K + k0 + j;
        if constexpr (BUF) xv[fi * KK + j] = buf_load<T>(xr, m * (unsigned)sizeof(T), col * nn * (unsigned)sizeof(T));
        else xv[fi * KK + j] = x[(size_t)col * nn + m];
      }
#pragma unroll
    for (int fi = 0; fi < F; ++fi)
#pragma unroll
      for (int j = 0; j < KK; ++j)
#pragma unroll
        for (int fo = 0; fo < F; ++fo) acc[fo * KK + j] += sv[fo * F + fi] * xv[fi * KK + j];
  }
  epilogue_cols<T, F, K, KK, CHEBY>(n, nn, k0, acc, a);
}

// S[(d*F + fo)*F + fi][n] = sum over elements e containing n and n + d of
// the element block coupling them (element matrices Ae, structure of arrays)
template <int F>
__global__ void k_build_stencil(unsigned N, const double* __restrict__ Ae, double* __restrict__ S) {
  constexpr int SZ = 8 * F;
  const unsigned nn = N * N * N;
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const NodeIdx q = node_idx(n, N);
  for (int d = 0; d < 27; ++d) {
    const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
    double blk[F * F];
    for (int t = 0; t < F * F; ++t) blk[t] = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int mx = (c & 1) + dx, my = ((c >> 1) & 1) + dy, mz = ((c >> 2) & 1) + dz;
      if (mx < 0 || mx > 1 || my < 0 || my > 1 || mz < 0 || mz > 1) continue;
      const int lm = mx + 2 * my + 4 * mz;
      const unsigned e = nb_node(q, N, -(c & 1), -((c >> 1) & 1), -((c >> 2) & 1));
      for (int fo = 0; fo < F; ++fo)
        for (int fi = 0; fi < F; ++fi) blk[fo * F + fi] += Ae[((size_t)((c * F + fo) * SZ + lm * F + fi)) * nn + e];
    }
    for (int t = 0; t < F * F; ++t) S[(size_t)(d * F * F + t) * nn + n] = blk[t];
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

// One workgroup per coarse element E: K_E = sum_children Q_c^T K_c Q_c.
template <int F>
__global__ __launch_bounds__(576) void k_galerkin(unsigned Nf, const double* __restrict__ s,
                                                  const double* __restrict__ kref,
                                                  const double* __restrict__ Afine, double* __restrict__ Acoarse) {
  constexpr int S = 8 * F;
  __shared__ double Kc[S * S];
  __shared__ double T1[S * S];
  const unsigned Nc = Nf / 2;
  const unsigned nec = Nc * Nc * Nc;
  const unsigned nef = Nf * Nf * Nf;
  const unsigned E = blockIdx.x;
  const unsigned I = E % Nc, J = (E / Nc) % Nc, Kk = E / (Nc * Nc);
  const int t = threadIdx.x;  // blockDim == S*S
  const int r = t / S, col = t % S;
  double acc = 0.0;
  for (int cp = 0; cp < 8; ++cp) {
    const unsigned ef = (2 * I + (cp & 1)) + Nf * ((2 * J + ((cp >> 1) & 1)) + Nf * (2 * Kk + ((cp >> 2) & 1)));
    if (s) {
      Kc[t] = s[ef] * kref[t];
    } else {
      const int l = r / F, f = r % F;
      Kc[t] = Afine[((size_t)((l * F + f) * S + col)) * nef + ef];
    }
    __syncthreads();
    {
      const int Lp = col / F, g = col % F;
      double v = 0.0;
      for (int lp = 0; lp < 8; ++lp) v += Kc[r * S + lp * F + g] * qweight(cp, lp, Lp);
      T1[t] = v;
    }
    __syncthreads();
    {
      const int L = r / F, f = r % F;
      double v = 0.0;
      for (int l = 0; l < 8; ++l) v += qweight(cp, l, L) * T1[(l * F + f) * S + col];
      acc += v;
    }
    __syncthreads();
  }
  const int L = r / F, f = r % F;
  Acoarse[((size_t)((L * F + f) * S + col)) * nec + E] = acc;
}

// Coarsening of stored element matrices, G coarse elements per workgroup
// (consecutive in x; Nc a multiple of G): the children of neighbouring
// coarse elements sit two elements apart, so a thread's G reads of one
// entry share cache lines, where one element per workgroup read one line
// per value.
template <int F, int G>
__global__ __launch_bounds__(64 * F * F) void k_galerkin_stored(unsigned Nf, const double* __restrict__ Afine,
                                                                double* __restrict__ Acoarse) {
  constexpr int S = 8 * F;
  __shared__ double Kc[G][S * S];
  __shared__ double T1[G][S * S];
  const unsigned Nc = Nf / 2;
  const unsigned nec = Nc * Nc * Nc;
  const unsigned nef = Nf * Nf * Nf;
  const unsigned E0 = blockIdx.x * G;  // G consecutive coarse elements along x
  const unsigned I0 = E0 % Nc, J = (E0 / Nc) % Nc, Kk = E0 / (Nc * Nc);
  const int t = threadIdx.x;  // blockDim == S*S
  const int r = t / S, col = t % S;
  const int L = r / F, f = r % F, Lp = col / F, gq = col % F;
  double acc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g] = 0.0;
  for (int cp = 0; cp < 8; ++cp) {
    const unsigned ef0 = (2 * I0 + (cp & 1)) + Nf * ((2 * J + ((cp >> 1) & 1)) + Nf * (2 * Kk + ((cp >> 2) & 1)));
    const int l0 = r / F, f0 = r % F;
#pragma unroll
    for (int g = 0; g < G; ++g) Kc[g][t] = Afine[((size_t)((l0 * F + f0) * S + col)) * nef + ef0 + 2 * g];
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
      double v = 0.0;
      for (int lp = 0; lp < 8; ++lp) v += Kc[g][r * S + lp * F + gq] * qweight(cp, lp, Lp);
      T1[g][t] = v;
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
      double v = 0.0;
      for (int l = 0; l < 8; ++l) v += qweight(cp, l, L) * T1[g][(l * F + f) * S + col];
      acc[g] += v;
    }
    __syncthreads();
  }
#pragma unroll
  for (int g = 0; g < G; ++g) Acoarse[((size_t)((L * F + f) * S + col)) * nec + E0 + g] = acc[g];
}

// The eight fixed blocks of the first coarsening, M_c = Q_c^T kref Q_c
// (block c: child c of a coarse element), mq[c][r][col] with r, col in
// (corner, field) order.  One workgroup per child, one thread per entry.
template <int F>
__global__ void k_galerkin_ref(const double* __restrict__ kref, double* __restrict__ mq) {
  constexpr int S = 8 * F;
  const int cp = blockIdx.x, t = threadIdx.x;
  const int r = t / S, col = t % S;
  const int L = r / F, f = r % F, Lp = col / F, g = col % F;
  double v = 0.0;
  for (int l = 0; l < 8; ++l) {
    const double wl = qweight(cp, l, L);
    for (int lp = 0; lp < 8; ++lp) v += wl * kref[(l * F + f) * S + lp * F + g] * qweight(cp, lp, Lp);
  }
  mq[cp * S * S + t] = v;
}

// First coarsening, one thread per coarse element E: K_E = sum_c s_c M_c
// over its eight children, written entry by entry (coalesced over E).
template <int F>
__global__ __launch_bounds__(256) void k_galerkin_first(unsigned Nf, const double* __restrict__ s,
                                                        const double* __restrict__ mq,
                                                        double* __restrict__ Acoarse) {
  constexpr int S = 8 * F;
  const unsigned Nc = Nf / 2, nec = Nc * Nc * Nc;
  const unsigned E = blockIdx.x * blockDim.x + threadIdx.x;
  if (E >= nec) return;
  const unsigned I = E % Nc, J = (E / Nc) % Nc, Kk = E / (Nc * Nc);
  double sc[8];
#pragma unroll
  for (int cp = 0; cp < 8; ++cp)
    sc[cp] = s[(2 * I + (cp & 1)) + Nf * ((2 * J + ((cp >> 1) & 1)) + Nf * (2 * Kk + ((cp >> 2) & 1)))];
  for (int t = 0; t < S * S; ++t) {
    double v = 0.0;
#pragma unroll
    for (int cp = 0; cp < 8; ++cp) v += sc[cp] * mq[cp * S * S + t];
    Acoarse[(size_t)t * nec + E] = v;
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

// Dinv stored [F*F][nn] (entry (f, g) of node n at (f*F + g)*nn + n)
template <int F>
__device__ __forceinline__ void store_inv(unsigned n, unsigned nn, const double* D, double* Dinv) {
  if (F == 1) {
    Dinv[n] = 1.0 / D[0];
  } else {
    double o[9];
    inv3(D, o);
    for (int t = 0; t < 9; ++t) Dinv[(size_t)t * nn + n] = o[t];
  }
}

template <int F>
__global__ void k_diag_fine(unsigned N, const double* __restrict__ s, const double* __restrict__ kref,
                            double* __restrict__ Dinv) {
  const unsigned nn = N * N * N;
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const NodeIdx q = node_idx(n, N);
  double D[F * F];
  for (int t = 0; t < F * F; ++t) D[t] = 0.0;
  for (int c = 0; c < 8; ++c) {
    const double sc = s[nb_node(q, N, -(c & 1), -((c >> 1) & 1), -((c >> 2) & 1))];
    for (int f = 0; f < F; ++f)
      for (int g = 0; g < F; ++g) D[f * F + g] += sc * kref[(c * F + f) * (8 * F) + c * F + g];
  }
  store_inv<F>(n, nn, D, Dinv);
}

template <int F>
__global__ void k_diag_coarse(unsigned N, const double* __restrict__ Ae, double* __restrict__ Dinv) {
  constexpr int S = 8 * F;
  const unsigned nn = N * N * N;
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const NodeIdx q = node_idx(n, N);
  double D[F * F];
  for (int t = 0; t < F * F; ++t) D[t] = 0.0;
  for (int c = 0; c < 8; ++c) {
    const unsigned e = nb_node(q, N, -(c & 1), -((c >> 1) & 1), -((c >> 2) & 1));
    for (int f = 0; f < F; ++f)
      for (int g = 0; g < F; ++g) D[f * F + g] += Ae[((size_t)((c * F + f) * S + c * F + g)) * nn + e];
  }
  store_inv<F>(n, nn, D, Dinv);
}

// First Chebyshev step for (node, column k = blockIdx.y): d = cf Dinv r; x
// untouched, x = d or x += d (xmode)
template <typename T, int F>
__global__ __launch_bounds__(256) void k_cheby_first(unsigned nn, int K, const T* __restrict__ Dinv,
                                                     const T* r, T* d, T* x, const T* __restrict__ cfp,
                                                     int xmode) {
  const unsigned n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int kk = blockIdx.y;
  const T cf = cfp[0];
  T rv[F];
#pragma unroll
  for (int f = 0; f < F; ++f) rv[f] = r[(size_t)(f * K + kk) * nn + n];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    T z = T(0);
#pragma unroll
    for (int g = 0; g < F; ++g) z += Dinv[(size_t)(f * F + g) * nn + n] * rv[g];
    const T dv = cf * z;
    const size_t o = (size_t)(f * K + kk) * nn + n;
    d[o] = dv;
    if (xmode == kChebyXSet) x[o] = dv;
    else if (xmode == kChebyXAdd) x[o] += dv;
  }
}

// Two consecutive values of one column (the pair at an even index: 8- or
// 16-byte aligned, one load or store instruction).
template <typename T> struct Pair;
template <> struct Pair<float> { using type = float2; };
template <> struct Pair<double> { using type = double2; };

// rc[I] = sum_{d in {-1,0,1}^3} prod(1 - |d|/2) rf[2I + d]: one thread per
// (coarse node, chunk of CPT columns starting at CPT * blockIdx.y); the index
// arithmetic is shared by the chunk, whose loads are independent
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_restrict(unsigned Nc, const T* __restrict__ rf, T* __restrict__ rc) {
  const unsigned Nf = 2 * Nc;
  const unsigned nc = Nc * Nc * Nc, nf = Nf * Nf * Nf;
  const unsigned I = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const unsigned ic = I % Nc, jc = (I / Nc) % Nc, kc = I / (Nc * Nc);
  const unsigned xs[3] = {(2 * ic + Nf - 1) % Nf, 2 * ic, 2 * ic + 1};
  const unsigned ys[3] = {(2 * jc + Nf - 1) % Nf, 2 * jc, 2 * jc + 1};
  const unsigned zs[3] = {(2 * kc + Nf - 1) % Nf, 2 * kc, 2 * kc + 1};
  const T* src = rf + (size_t)blockIdx.y * CPT * nf;
  T acc[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) acc[q] = T(0);
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    const int dx = t % 3, dy = (t / 3) % 3, dz = t / 9;
    const T w = T((dx == 1 ? 1.0 : 0.5) * (dy == 1 ? 1.0 : 0.5) * (dz == 1 ? 1.0 : 0.5));
    const unsigned o = xs[dx] + Nf * (ys[dy] + Nf * zs[dz]);
#pragma unroll
    for (int q = 0; q < CPT; ++q) acc[q] += w * src[(size_t)q * nf + o];
  }
#pragma unroll
  for (int q = 0; q < CPT; ++q) rc[((size_t)blockIdx.y * CPT + q) * nc + I] = acc[q];
}

// xf[i] += sum_I P[i, I] xc[I] (trilinear, periodic): one thread per (coarse
// cell, chunk of CPT columns starting at CPT * blockIdx.y).  The cell's eight
// coarse corners give its 2 x 2 x 2 fine nodes by averaging along each axis
// where the fine node is odd; each fine row pair is read and written as one
// access.
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_prolong(unsigned Nc, const T* __restrict__ xc, T* __restrict__ xf) {
  using P2 = typename Pair<T>::type;
  const unsigned Nf = 2 * Nc;
  const unsigned nc = Nc * Nc * Nc, nf = Nf * Nf * Nf;
  const unsigned i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const unsigned bi = i % Nc, bj = (i / Nc) % Nc, bk = i / (Nc * Nc);
  const unsigned bi1 = bi + 1 == Nc ? 0 : bi + 1, bj1 = bj + 1 == Nc ? 0 : bj + 1, bk1 = bk + 1 == Nc ? 0 : bk + 1;
  unsigned ci[8];
#pragma unroll
  for (int c = 0; c < 8; ++c)
    ci[c] = ((c & 1) ? bi1 : bi) + Nc * (((c >> 1) & 1 ? bj1 : bj) + Nc * ((c >> 2) ? bk1 : bk));
  const unsigned f0 = 2 * bi + Nf * (2 * bj + Nf * 2 * bk);
  const size_t c0 = (size_t)blockIdx.y * CPT;
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const T* src = xc + (c0 + q) * nc;
    T v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = src[ci[c]];
    T* dst = xf + (c0 + q) * nf + f0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {   // fine row (oj, ok) = (r & 1, r >> 1)
      const int oj = r & 1, ok = r >> 1;
      // coarse values of this row at x = bi and bi + 1
      T e[2];
#pragma unroll
      for (int ax = 0; ax < 2; ++ax) {
        const T z0 = oj ? T(0.5) * (v[ax] + v[ax + 2]) : v[ax];
        const T z1 = oj ? T(0.5) * (v[ax + 4] + v[ax + 6]) : v[ax + 4];
        e[ax] = ok ? T(0.5) * (z0 + z1) : z0;
      }
      P2* p = reinterpret_cast<P2*>(dst + Nf * (oj + Nf * ok));
      P2 cur = *p;
      cur.x += e[0];
      cur.y += T(0.5) * (e[0] + e[1]);
      *p = cur;
    }
  }
}

// z[(f, k, n)] = sum_{(g, m)} Minv[(f*nc + n), (g*nc + m)] r[(g, k, m)]
template <typename T>
__global__ void k_dense_apply(int F, int nc, int K, const double* __restrict__ Minv, const T* __restrict__ r,
                              T* __restrict__ z) {
  const int row = blockIdx.x;  // f*nc + n
  const int kk = threadIdx.y;
  const int rows = F * nc;
  const int f = row / nc, n = row % nc;
  __shared__ double part[9][64];
  double v = 0.0;
  for (int c = threadIdx.x; c < rows; c += 64) {
    const int g = c / nc, m = c % nc;
    v += Minv[(size_t)row * rows + c] * (double)r[(size_t)(g * K + kk) * nc + m];
  }
  part[kk][threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int t = 0; t < 64; ++t) sum += part[kk][t];
    z[(size_t)(f * K + kk) * nc + n] = (T)sum;
  }
}

inline unsigned blocks_for(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T, int OPV, int KV>
void launch_fine(unsigned N, const T* s, const T* kref, const T* x, const OpArgs<T>& a, bool cheby,
                 hipStream_t st) {
  constexpr int FO = OpFields<OPV>::FO, FI = OpFields<OPV>::FI;
  const size_t nn = (size_t)N * N * N;
  const unsigned g = blocks_for(nn, 128);
  const bool buf = nn * FI * KV * sizeof(T) < (size_t(1) << 32);
#define PHZ_FK(CH, BUF) \
  hipLaunchKernelGGL((k_fine_apply<T, FO, FI, KV, CH, BUF>), dim3(g), dim3(128), 0, st, N, s, kref, x, a)
  if constexpr (FO == FI) {
    if (cheby) {
      if (buf) PHZ_FK(true, true);
      else PHZ_FK(true, false);
      return;
    }
  }
  if (cheby) throw std::invalid_argument("Chebyshev epilogue needs a square block");
  if (buf) PHZ_FK(false, true);
  else PHZ_FK(false, false);
#undef PHZ_FK
}

template <typename T, int FV, int KV>
void launch_coarse(unsigned N, const T* S, const T* x, const OpArgs<T>& a, bool cheby, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  const bool buf = nn * 27 * FV * FV * sizeof(T) < (size_t(1) << 32) && nn * FV * KV * sizeof(T) < (size_t(1) << 32);
  // one thread per node when that already fills the chip, else per (node, column)
  const bool per_node = KV == 1 || nn >= 131072;
  const unsigned g = blocks_for(nn, 256);
#define PHZ_CK(KK, CH, BUF, GY) \
  hipLaunchKernelGGL((k_stencil_apply<T, FV, KV, KK, CH, BUF>), dim3(g, GY), dim3(256), 0, st, N, S, x, a)
  if (per_node) {
    if (cheby) { if (buf) PHZ_CK(KV, true, true, 1); else PHZ_CK(KV, true, false, 1); }
    else { if (buf) PHZ_CK(KV, false, true, 1); else PHZ_CK(KV, false, false, 1); }
  } else {
    if (cheby) { if (buf) PHZ_CK(1, true, true, KV); else PHZ_CK(1, true, false, KV); }
    else { if (buf) PHZ_CK(1, false, true, KV); else PHZ_CK(1, false, false, KV); }
  }
#undef PHZ_CK
}

}  // namespace

template <typename T>
void fine_apply(int op, int nrhs, int N, const T* s, const T* kref, const T* x, const OpArgs<T>& a, bool cheby,
                hipStream_t st) {
#define PHZ_FA(OPV, KV) launch_fine<T, OPV, KV>((unsigned)N, s, kref, x, a, cheby, st)
  if (nrhs == 1) {
    switch (op) {
      case 0: PHZ_FA(0, 1); break;
      case 1: PHZ_FA(1, 1); break;
      case 2: PHZ_FA(2, 1); break;
      case 3: PHZ_FA(3, 1); break;
      case 5: PHZ_FA(5, 1); break;
      default: throw std::invalid_argument("fine_apply op");
    }
  } else if (nrhs == 9) {
    switch (op) {
      case 0: PHZ_FA(0, 9); break;
      case 1: PHZ_FA(1, 9); break;
      case 2: PHZ_FA(2, 9); break;
      case 3: PHZ_FA(3, 9); break;
      case 5: PHZ_FA(5, 9); break;
      default: throw std::invalid_argument("fine_apply op");
    }
  } else {
    throw std::invalid_argument("fine_apply nrhs");
  }
#undef PHZ_FA
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void fine_apply_qp(int nrhs, int N, const T* sq, const T* kq, const T* x, const OpArgs<T>& a, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  const unsigned g = blocks_for(nn, 128);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_fine_apply_qp<T, 1>), dim3(g), dim3(128), 0, st, (unsigned)N, sq, kq, x, a);
  else if (nrhs == 9)
    hipLaunchKernelGGL((k_fine_apply_qp<T, 9>), dim3(g), dim3(128), 0, st, (unsigned)N, sq, kq, x, a);
  else
    throw std::invalid_argument("fine_apply_qp nrhs");
  PHZ_LAUNCH_CHECK();
}

bool fine_tiled_fits(int N) { return N >= GTX && N % GTX == 0 && N % GTY == 0 && N % GTZ == 0; }

void fine_apply_tiled(int op, int nrhs, int N, const float* s, const float* kref, const float* x,
                      const OpArgs<float>& a, bool cheby, hipStream_t st) {
  if (nrhs != 9 || !fine_tiled_fits(N)) throw std::invalid_argument("fine_apply_tiled: nine columns, N a multiple of 16");
  switch (op) {
    case 0: launch_tiled<0>((unsigned)N, s, kref, x, a, cheby, st); break;
    case 1: launch_tiled<1>((unsigned)N, s, kref, x, a, cheby, st); break;
    case 2: launch_tiled<2>((unsigned)N, s, kref, x, a, cheby, st); break;
    case 3: launch_tiled<3>((unsigned)N, s, kref, x, a, cheby, st); break;
    default: throw std::invalid_argument("fine_apply_tiled op");
  }
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void coarse_apply(int F, int nrhs, int N, const T* Ae, const T* x, const OpArgs<T>& a, bool cheby, hipStream_t st) {
  if (F == 3 && nrhs == 1) launch_coarse<T, 3, 1>((unsigned)N, Ae, x, a, cheby, st);
  else if (F == 3 && nrhs == 9) launch_coarse<T, 3, 9>((unsigned)N, Ae, x, a, cheby, st);
  else if (F == 1 && nrhs == 1) launch_coarse<T, 1, 1>((unsigned)N, Ae, x, a, cheby, st);
  else if (F == 1 && nrhs == 9) launch_coarse<T, 1, 9>((unsigned)N, Ae, x, a, cheby, st);
  else throw std::invalid_argument("coarse_apply");
  PHZ_LAUNCH_CHECK();
}

bool coarse_tiled_fits(int N) { return fine_tiled_fits(N); }

void coarse_apply_tiled(int F, int N, const float* S, const float* x, const OpArgs<float>& a, bool cheby,
                        hipStream_t st) {
  if (!coarse_tiled_fits(N)) throw std::invalid_argument("coarse_apply_tiled: N must be a multiple of 16");
  if (F == 3) launch_stencil_tiled<3>((unsigned)N, S, x, a, cheby, st);
  else if (F == 1) launch_stencil_tiled<1>((unsigned)N, S, x, a, cheby, st);
  else throw std::invalid_argument("coarse_apply_tiled F");
  PHZ_LAUNCH_CHECK();
}

void coarse_apply_tiled_compact(int F, int N, const unsigned short* S16, const float* Sc, const float* x,
                                const OpArgs<float>& a, bool cheby, hipStream_t st) {
  if (!coarse_tiled_fits(N)) throw std::invalid_argument("coarse_apply_tiled_compact: N must be a multiple of 16");
  if (F == 3) launch_stencil_tiled_compact<3>((unsigned)N, S16, Sc, x, a, cheby, st);
  else if (F == 1) launch_stencil_tiled_compact<1>((unsigned)N, S16, Sc, x, a, cheby, st);
  else throw std::invalid_argument("coarse_apply_tiled_compact F");
  PHZ_LAUNCH_CHECK();
}

void compact_stencil(int F, long nn, const double* S, unsigned short* S16, float* Sc, hipStream_t st) {
  const unsigned g = (unsigned)((nn + 255) / 256);
  if (F == 3) hipLaunchKernelGGL((k_compact_stencil<3>), dim3(g), dim3(256), 0, st, (unsigned)nn, S, S16, Sc);
  else if (F == 1) hipLaunchKernelGGL((k_compact_stencil<1>), dim3(g), dim3(256), 0, st, (unsigned)nn, S, S16, Sc);
  else throw std::invalid_argument("compact_stencil F");
  PHZ_LAUNCH_CHECK();
}

void galerkin_build(int F, int Nf, const double* s, const double* kref, const double* Afine, double* Acoarse,
                    double* mq, hipStream_t st) {
  const unsigned nec = (unsigned)(Nf / 2) * (Nf / 2) * (Nf / 2);
  if (s) {
    // from the fine level: the children's blocks are s_c kref, so
    // K_E = sum_c s_c M_c with the eight fixed M_c = Q_c^T kref Q_c
    const unsigned g = (nec + 255) / 256;
    if (F == 3) {
      hipLaunchKernelGGL(k_galerkin_ref<3>, dim3(8), dim3(576), 0, st, kref, mq);
      hipLaunchKernelGGL(k_galerkin_first<3>, dim3(g), dim3(256), 0, st, (unsigned)Nf, s, mq, Acoarse);
    } else if (F == 1) {
      hipLaunchKernelGGL(k_galerkin_ref<1>, dim3(8), dim3(64), 0, st, kref, mq);
      hipLaunchKernelGGL(k_galerkin_first<1>, dim3(g), dim3(256), 0, st, (unsigned)Nf, s, mq, Acoarse);
    } else {
      throw std::invalid_argument("galerkin F");
    }
  } else if ((Nf / 2) % 4 == 0) {
    if (F == 3)
      hipLaunchKernelGGL((k_galerkin_stored<3, 4>), dim3(nec / 4), dim3(576), 0, st, (unsigned)Nf, Afine, Acoarse);
    else if (F == 1)
      hipLaunchKernelGGL((k_galerkin_stored<1, 4>), dim3(nec / 4), dim3(64), 0, st, (unsigned)Nf, Afine, Acoarse);
    else
      throw std::invalid_argument("galerkin F");
  } else if (F == 3) {
    hipLaunchKernelGGL(k_galerkin<3>, dim3(nec), dim3(576), 0, st, (unsigned)Nf, s, kref, Afine, Acoarse);
  } else if (F == 1) {
    hipLaunchKernelGGL(k_galerkin<1>, dim3(nec), dim3(64), 0, st, (unsigned)Nf, s, kref, Afine, Acoarse);
  } else {
    throw std::invalid_argument("galerkin F");
  }
  PHZ_LAUNCH_CHECK();
}

void diag_inv_fine(int F, int N, const double* s, const double* kref, double* Dinv, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  if (F == 3) hipLaunchKernelGGL(k_diag_fine<3>, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)N, s, kref, Dinv);
  else hipLaunchKernelGGL(k_diag_fine<1>, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)N, s, kref, Dinv);
  PHZ_LAUNCH_CHECK();
}

void diag_inv_coarse(int F, int N, const double* Ae, double* Dinv, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  if (F == 3) hipLaunchKernelGGL(k_diag_coarse<3>, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)N, Ae, Dinv);
  else hipLaunchKernelGGL(k_diag_coarse<1>, dim3(blocks_for(nn, 256)), dim3(256), 0, st, (unsigned)N, Ae, Dinv);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void cheby_first(int F, int nrhs, long nn, const T* Dinv, const T* r, T* d, T* x, const T* cf, int xmode,
                 hipStream_t st) {
  const dim3 g(blocks_for((size_t)nn, 256), nrhs);
  if (F == 3)
    hipLaunchKernelGGL((k_cheby_first<T, 3>), g, dim3(256), 0, st, (unsigned)nn, nrhs, Dinv, r, d, x, cf, xmode);
  else if (F == 1)
    hipLaunchKernelGGL((k_cheby_first<T, 1>), g, dim3(256), 0, st, (unsigned)nn, nrhs, Dinv, r, d, x, cf, xmode);
  else
    throw std::invalid_argument("cheby_first");
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void restrict_fw(int F, int nrhs, int Nc, const T* rf, T* rc, hipStream_t st) {
  const int ncol = F * nrhs;
  const unsigned g = blocks_for((size_t)Nc * Nc * Nc, 256);
  if (ncol % 9 == 0) hipLaunchKernelGGL((k_restrict<T, 9>), dim3(g, ncol / 9), dim3(256), 0, st, (unsigned)Nc, rf, rc);
  else if (ncol % 3 == 0) hipLaunchKernelGGL((k_restrict<T, 3>), dim3(g, ncol / 3), dim3(256), 0, st, (unsigned)Nc, rf, rc);
  else hipLaunchKernelGGL((k_restrict<T, 1>), dim3(g, ncol), dim3(256), 0, st, (unsigned)Nc, rf, rc);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void prolong_add(int F, int nrhs, int Nc, const T* xc, T* xf, hipStream_t st) {
  const int ncol = F * nrhs;
  const unsigned g = blocks_for((size_t)Nc * Nc * Nc, 256);
  if (ncol % 9 == 0) hipLaunchKernelGGL((k_prolong<T, 9>), dim3(g, ncol / 9), dim3(256), 0, st, (unsigned)Nc, xc, xf);
  else if (ncol % 3 == 0) hipLaunchKernelGGL((k_prolong<T, 3>), dim3(g, ncol / 3), dim3(256), 0, st, (unsigned)Nc, xc, xf);
  else hipLaunchKernelGGL((k_prolong<T, 1>), dim3(g, ncol), dim3(256), 0, st, (unsigned)Nc, xc, xf);
  PHZ_LAUNCH_CHECK();
}

void build_stencil(int F, int N, const double* Ae, double* S, hipStream_t st) {
  const size_t nn = (size_t)N * N * N;
  if (F == 3) hipLaunchKernelGGL(k_build_stencil<3>, dim3(blocks_for(nn, 128)), dim3(128), 0, st, (unsigned)N, Ae, S);
  else hipLaunchKernelGGL(k_build_stencil<1>, dim3(blocks_for(nn, 128)), dim3(128), 0, st, (unsigned)N, Ae, S);
  PHZ_LAUNCH_CHECK();
}

template <typename T>
void dense_apply(int F, int nc, int nrhs, const double* Minv, const T* r, T* z, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_apply<T>, dim3(F * nc), dim3(64, nrhs), 0, st, F, nc, nrhs, Minv, r, z);
  PHZ_LAUNCH_CHECK();
}

#define PHZ_INST(T)                                                                                            \
  template void fine_apply<T>(int, int, int, const T*, const T*, const T*, const OpArgs<T>&, bool, hipStream_t); \
  template void fine_apply_qp<T>(int, int, const T*, const T*, const T*, const OpArgs<T>&, hipStream_t); \
  template void coarse_apply<T>(int, int, int, const T*, const T*, const OpArgs<T>&, bool, hipStream_t);         \
  template void cheby_first<T>(int, int, long, const T*, const T*, T*, T*, const T*, int, hipStream_t);               \
  template void restrict_fw<T>(int, int, int, const T*, T*, hipStream_t);                                     \
  template void prolong_add<T>(int, int, int, const T*, T*, hipStream_t);                                     \
  template void dense_apply<T>(int, int, int, const double*, const T*, T*, hipStream_t);
PHZ_INST(double)
PHZ_INST(float)
#undef PHZ_INST

}  // namespace phz
