// Fine-level operator as an element contraction on the matrix cores (gfx950),
// in split-BF16 arithmetic with FP32 accumulation.
//
// The fine operator of Sec. 2.5 is y = sum_e s_e P_e^T Kref P_e x: per element
// the product Y_e = Kref X_e of the reference block with the element's
// gathered inputs (one column per load).  Kref is padded to 32 x 32 with the
// (corner c, field f) index 4c + f on both sides (four field slots per
// corner; slots beyond the block's fields are zero), so every block of the
// operator (full 4 -> 4, A 3 -> 3, B 3 -> 1, S_bar 1 -> 1) is the same MFMA
// shape.  A workgroup owns a TX x TY x TZ tile of 256 output nodes, one per
// thread, and for each load column
//   1. stages the tile's input nodes plus a one-node halo in LDS (float32;
//      the next column's global loads are issued before this column's
//      contraction so their latency is hidden);
//   2. contracts every element with a corner in the tile, (TX+1)(TY+1)(TZ+1)
//      of them, 16 elements per v_mfma_f32_16x16x32_bf16 (elements are the
//      MFMA columns, Kref rows the MFMA rows).  Kref annihilates per-field
//      constants, so the element's inputs enter as differences to its corner
//      0, d = x - x_0, split into bf16 pairs hi = rne(d), lo = rne(d - hi)
//      (d = hi + lo to 2^-18 relative):
//      Y = lo(K) hi(D) + hi(K) lo(D) + hi(K) hi(D) accumulated in FP32 (the
//      dropped lo*lo term is about 2^-18 relative); the error then scales
//      with the differences across an element, not with the nodal values,
//      which keeps the residuals of smooth fields accurate.  The element
//      outputs are stored in LDS by (corner, element);
//   3. sums, for its node, the outputs of the eight elements around it times
//      their scales s_e in a fixed corner order (deterministic, no atomics),
//      then runs the same
//      output epilogue as the gather kernels (residual form and the fused
//      Chebyshev step).
// Elements on the tile's halo are contracted by every tile that touches
// them: the price of the owner-computes sum.
#include <cstring>

#include "common.hpp"
#include "devutil.hpp"

namespace phz {

namespace {
using namespace dev;

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) unsigned u32x4;

template <int OP> struct ElemFields;
template <> struct ElemFields<0> { static constexpr int FO = 4, FI = 4; };
template <> struct ElemFields<1> { static constexpr int FO = 3, FI = 3; };
template <> struct ElemFields<2> { static constexpr int FO = 1, FI = 3; };
template <> struct ElemFields<3> { static constexpr int FO = 1, FI = 1; };

template <int TX, int TY, int TZ>
struct ElemTile {
  static_assert(TX * TY * TZ == 256, "one output node per thread");
  static constexpr int NX = TX + 2, NY = TY + 2, NZ = TZ + 2, NI = NX * NY * NZ;  // input nodes
  static constexpr int EX = TX + 1, EY = TY + 1, EZ = TZ + 1, NE = EX * EY * EZ;  // elements
  static constexpr int CT = (NE + 15) / 16;                                        // MFMA column tiles
  static constexpr int NEP = 16 * CT;          // elements padded to whole column tiles
  static constexpr int MT = (CT + 3) / 4;      // column tiles per wave (at most)
  // LDS of a workgroup (staged nodes, element outputs, element scales) and
  // the waves per SIMD to ask the register allocator for: three where three
  // workgroups' LDS fits in a CU's 160 KiB (the three-field blocks on the
  // 8x8x4 and 16x4x4 tiles), else two
  static constexpr int lds_bytes(int fo) { return (NI + 3) * 16 + 8 * NEP * fo * 4 + NEP * 4; }
  static constexpr int waves(int fo) { return fo == 3 && 3 * lds_bytes(fo) <= 160 * 1024 ? 3 : 2; }
};

// periodic wrap of a coordinate in [-1, N]
__device__ __forceinline__ unsigned wrapc(int v, unsigned N) {
  return v < 0 ? (unsigned)(v + (int)N) : ((unsigned)v >= N ? (unsigned)v - N : (unsigned)v);
}

typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) float f32x2;

// Split of two float32 values into packed bf16 hi and lo halves:
// hi = rne(v), lo = rne(v - hi), two values per conversion instruction.
__device__ __forceinline__ void split2(float a, float b, unsigned& hi, unsigned& lo) {
  const unsigned h = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a, b}, bf16x2));
  const float ha = __builtin_bit_cast(float, h << 16), hb = __builtin_bit_cast(float, h & 0xffff0000u);
  hi = h;
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a - ha, b - hb}, bf16x2));
}

// Differences of two corners' four field slots to a base corner, split into
// the hi and lo B operands of one MFMA column (8 bf16 each).
__device__ __forceinline__ void split_corners(float4 p, float4 q, float4 base, bf16x8& bh, bf16x8& bl) {
  unsigned h0, h1, h2, h3, l0, l1, l2, l3;
  split2(p.x - base.x, p.y - base.y, h0, l0);
  split2(p.z - base.z, p.w - base.w, h1, l1);
  split2(q.x - base.x, q.y - base.y, h2, l2);
  split2(q.z - base.z, q.w - base.w, h3, l3);
  bh = __builtin_bit_cast(bf16x8, u32x4{h0, h1, h2, h3});
  bl = __builtin_bit_cast(bf16x8, u32x4{l0, l1, l2, l3});
}

template <int FO, int FI, int K, int TERMS, bool CHEBY, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ElemTile<TX, TY, TZ>::waves(FO)))) void k_elem_mfma(unsigned N, const float* __restrict__ s,
                                                   const bf16x8* __restrict__ kop,
                                                   const float* __restrict__ x, OpArgs<float> a) {
  using TL = ElemTile<TX, TY, TZ>;
  constexpr int NX = TL::NX, NY = TL::NY, NI = TL::NI;
  constexpr int EX = TL::EX, EY = TL::EY, NE = TL::NE, CT = TL::CT, NEP = TL::NEP, MT = TL::MT;
  constexpr int PF = (NI + 255) / 256;  // staged input nodes per thread
  __shared__ float4 xs[NI + 3];         // input node values, field slots 0..3; two zero pads, a spill slot
  __shared__ float zs[8 * NEP * FO];    // element outputs [corner][element][field]
  __shared__ float se[NEP];

  const unsigned nn = N * N * N;
  const unsigned ntx = N / TX, nty = N / TY;
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int x0 = (int)((b % ntx) * TX), y0 = (int)(((b / ntx) % nty) * TY), z0 = (int)((b / (ntx * nty)) * TZ);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // scales of the elements touching the tile (element origin = tile origin - 1
  // + local); the padding columns get scale 0 and read the zero pad nodes
  for (int e = tid; e < NEP; e += 256) {
    const int ex = e % EX, ey = (e / EX) % EY, ez = e / (EX * EY);
    se[e] = e < NE ? s[wrapc(x0 - 1 + ex, N) + N * (wrapc(y0 - 1 + ey, N) + N * wrapc(z0 - 1 + ez, N))] : 0.f;
  }
  if (tid < 2) xs[NI + tid] = float4{0.f, 0.f, 0.f, 0.f};
  // global node of each staged input node of this thread
  unsigned gm[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    const int t = tid + 256 * p;
    const int li = t % NX, lj = (t / NX) % NY, lk = t / (NX * NY);
    gm[p] = t < NI ? wrapc(x0 - 1 + li, N) + N * (wrapc(y0 - 1 + lj, N) + N * wrapc(z0 - 1 + lk, N)) : 0u;
  }
  // reference block, MFMA A operand: row tile t (rows 16t .. 16t+15), hi and lo
  bf16x8 ah[2], al[2];
  ah[0] = kop[0 * 64 + lane];
  ah[1] = kop[1 * 64 + lane];
  if constexpr (TERMS == 3) {
    al[0] = kop[2 * 64 + lane];
    al[1] = kop[3 * 64 + lane];
  }

  // this thread's output node
  const int ti = tid % TX, tj = (tid / TX) % TY, tk = tid / (TX * TY);
  const unsigned n = (unsigned)(x0 + ti) + N * ((unsigned)(y0 + tj) + N * (unsigned)(z0 + tk));
  // MFMA lane roles: column (element) lane & 15; k-slice g = lane >> 4 covers
  // corners 2g (cx = 0) and 2g + 1 (cx = 1), both with cy = g & 1, cz = g >> 1;
  // output rows of row tile t are corner 4t + g, fields 0..3
  const int g = lane >> 4, gy = g & 1, gz = g >> 1;
  // per column tile of this wave: LDS index of the element's corner 0 and of
  // corner 2g (corner 2g + 1 follows it), the same for every load column
  int tb[MT], t0[MT];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    const int e = (wave + 4 * i) * 16 + (lane & 15);
    if (e < NE) {
      const int ex = e % EX, ey = (e / EX) % EY, ez = e / (EX * EY);
      tb[i] = ex + NX * (ey + NY * ez);
      t0[i] = ex + NX * ((ey + gy) + NY * (ez + gz));
    } else {
      tb[i] = NI;
      t0[i] = NI;
    }
  }

  // input values of column k for the staged nodes and this node's residual
  // input of column k, fetched one column ahead so their latency overlaps a
  // column of work
  float pv[PF][FI];
  float eyin[FO];
  const bool has_yin = a.beta != 0.f;
  auto fetch = [&](int k) {
#pragma unroll
    for (int p = 0; p < PF; ++p)
#pragma unroll
      for (int f = 0; f < FI; ++f)
        pv[p][f] = (tid + 256 * p < NI) ? x[(size_t)(f * K + k) * nn + gm[p]] : 0.f;
#pragma unroll
    for (int f = 0; f < FO; ++f) eyin[f] = has_yin ? a.yin[(size_t)(f * K + k) * nn + n] : 0.f;
  };
  // the node's Jacobi block and the step's coefficients, the same for every
  // column (Chebyshev epilogue, or the first step on the output, a.d1)
  float Di[FO * FO];
  float ca = 0.f, cb = 0.f;
  const bool with_d1 = !CHEBY && a.d1 != nullptr;
  if (CHEBY || with_d1) {
    ca = a.cab[0];
    if constexpr (CHEBY) cb = a.cab[1];
#pragma unroll
    for (int t = 0; t < FO * FO; ++t) Di[t] = a.dinv[(size_t)t * nn + n];
  }
  fetch(0);

  // scales of the eight elements around this thread's node (the same for
  // every column)
  __syncthreads();
  float sg[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
    sg[c] = se[(ti + 1 - cx) + EX * ((tj + 1 - cy) + EY * (tk + 1 - cz))];
  }

  // a column's outputs (y; with the Chebyshev step d_new and x; or d1) are
  // stored once the next column's inputs are staged: the wait for those
  // loads then does not also wait for the stores
  float so[3][FO];
  auto store_outputs = [&](int k) {
#pragma unroll
    for (int f = 0; f < FO; ++f) {
      const size_t o = (size_t)(f * K + k) * nn + n;
      a.y[o] = so[0][f];
      if constexpr (CHEBY) {
        a.dnew[o] = so[1][f];
        a.x[o] = so[2][f];
      } else {
        if (with_d1) a.d1[o] = so[1][f];
      }
    }
  };

  for (int k = 0; k < K; ++k) {
    __syncthreads();  // the previous column's LDS reads are complete
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      // threads past the staged nodes write the spill slot, so the staging
      // writes need no branch
      const int t = tid + 256 * p;
      float4 v = {0.f, 0.f, 0.f, 0.f};
      v.x = pv[p][0];
      if constexpr (FI > 1) { v.y = pv[p][1]; v.z = pv[p][2]; }
      if constexpr (FI > 3) v.w = pv[p][3];
      xs[t < NI ? t : NI + 2] = v;
    }
    if (k > 0) store_outputs(k - 1);
    // the Chebyshev step's operands of column k (previous correction,
    // iterate) are issued now, in flight during the contraction: fetching
    // them a column ahead too would hold more registers than three waves
    // per SIMD allow
    float cyin[FO], cdold[FO], cxit[FO];
#pragma unroll
    for (int f = 0; f < FO; ++f) {
      const size_t o = (size_t)(f * K + k) * nn + n;
      cyin[f] = eyin[f];
      cdold[f] = 0.f;
      cxit[f] = 0.f;
      if constexpr (CHEBY) {
        cdold[f] = a.dold[o];
        if (a.xin) cxit[f] = a.xin[o];
      }
    }
    if (k + 1 < K) fetch(k + 1);  // in flight during this column's contraction
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const int ct = wave + 4 * i;
      if (ct < CT) {
        const int e = ct * 16 + (lane & 15);
        // Kref annihilates per-field constants (rigid translations, constant
        // potential), so Kref X_e = Kref (X_e - x_corner0): contracting the
        // differences makes the split error scale with them, not the values
        bf16x8 bh, bl;
        split_corners(xs[t0[i]], xs[t0[i] + 1], xs[tb[i]], bh, bl);
        f32x4 d0 = {0.f, 0.f, 0.f, 0.f}, d1 = {0.f, 0.f, 0.f, 0.f};
        if constexpr (TERMS == 3) {
          d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[0], bh, d0, 0, 0, 0);
          d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[1], bh, d1, 0, 0, 0);
          d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[0], bl, d0, 0, 0, 0);
          d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[1], bl, d1, 0, 0, 0);
        }
        d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[0], bh, d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[1], bh, d1, 0, 0, 0);
        // rows of row tile t: corner 4t + g, field slots 0..3 (unscaled: the
        // gather applies s_e)
        if constexpr (FO == 4) {
          *reinterpret_cast<float4*>(&zs[(g * NEP + e) * 4]) = float4{d0[0], d0[1], d0[2], d0[3]};
          *reinterpret_cast<float4*>(&zs[((4 + g) * NEP + e) * 4]) = float4{d1[0], d1[1], d1[2], d1[3]};
        } else {
#pragma unroll
          for (int fo = 0; fo < FO; ++fo) {
            zs[(g * NEP + e) * FO + fo] = d0[fo];
            zs[((4 + g) * NEP + e) * FO + fo] = d1[fo];
          }
        }
      }
    }
    __syncthreads();
    float acc[FO];
#pragma unroll
    for (int fo = 0; fo < FO; ++fo) acc[fo] = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
      const int ee = (ti + 1 - cx) + EX * ((tj + 1 - cy) + EY * (tk + 1 - cz));
#pragma unroll
      for (int fo = 0; fo < FO; ++fo) acc[fo] += sg[c] * zs[(c * NEP + ee) * FO + fo];
    }
    // y = beta y_in + alpha acc; with the Chebyshev step also
    // d_new = ca d_old + cb Dinv y and x += d_new; or d1 = ca Dinv y.  Kept
    // in registers and stored during the next column
    float* out = so[0];
#pragma unroll
    for (int f = 0; f < FO; ++f) out[f] = has_yin ? a.beta * cyin[f] + a.alpha * acc[f] : a.alpha * acc[f];
    if constexpr (CHEBY) {
#pragma unroll
      for (int f = 0; f < FO; ++f) {
        float z = 0.f;
#pragma unroll
        for (int q = 0; q < FO; ++q) z += Di[f * FO + q] * out[q];
        const float dv = ca * cdold[f] + cb * z;
        so[1][f] = dv;
        so[2][f] = (a.fold_dold ? dv + cdold[f] : dv) + cxit[f];
      }
    } else {
      if (with_d1) {
#pragma unroll
        for (int f = 0; f < FO; ++f) {
          float z = 0.f;
#pragma unroll
          for (int q = 0; q < FO; ++q) z += Di[f * FO + q] * out[q];
          so[1][f] = ca * z;
        }
      }
    }
  }
  store_outputs(K - 1);
}

struct TileShape {
  int tx, ty, tz;
};
constexpr TileShape kTiles[] = {{8, 8, 4}, {16, 4, 4}, {16, 8, 2}};
constexpr int kNumTiles = (int)(sizeof(kTiles) / sizeof(kTiles[0]));

template <int OPV, int TERMS, int TX, int TY, int TZ>
void launch_elem_tile(unsigned N, const float* s, const void* kop, const float* x, const OpArgs<float>& a,
                      bool cheby, hipStream_t st) {
  constexpr int FO = ElemFields<OPV>::FO, FI = ElemFields<OPV>::FI;
  const unsigned blocks = (N / TX) * (N / TY) * (N / TZ);
  const bf16x8* kp = static_cast<const bf16x8*>(kop);
  if constexpr (FO == FI) {
    if (cheby) {
      hipLaunchKernelGGL((k_elem_mfma<FO, FI, 9, TERMS, true, TX, TY, TZ>), dim3(blocks), dim3(256), 0, st, N, s,
                         kp, x, a);
      return;
    }
  }
  if (cheby) throw std::invalid_argument("Chebyshev epilogue needs a square block");
  hipLaunchKernelGGL((k_elem_mfma<FO, FI, 9, TERMS, false, TX, TY, TZ>), dim3(blocks), dim3(256), 0, st, N, s, kp,
                     x, a);
}

template <int OPV, int TERMS>
void launch_elem(int tile, unsigned N, const float* s, const void* kop, const float* x, const OpArgs<float>& a,
                 bool cheby, hipStream_t st) {
  switch (tile) {
    case 0: launch_elem_tile<OPV, TERMS, 8, 8, 4>(N, s, kop, x, a, cheby, st); break;
    case 1: launch_elem_tile<OPV, TERMS, 16, 4, 4>(N, s, kop, x, a, cheby, st); break;
    case 2: launch_elem_tile<OPV, TERMS, 16, 8, 2>(N, s, kop, x, a, cheby, st); break;
    default: throw std::invalid_argument("elem tile");
  }
}

int op_fields_out(int op) { return op == 0 ? 4 : op == 1 ? 3 : 1; }
int op_fields_in(int op) { return op == 0 ? 4 : op == 3 ? 1 : 3; }

unsigned short rne_bf16_host(float v) {
  unsigned u;
  std::memcpy(&u, &v, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan unchanged
  const unsigned lsb = (u >> 16) & 1u;
  return (unsigned short)((u + 0x7fffu + lsb) >> 16);
}
float bf16_to_float_host(unsigned short h) {
  const unsigned u = (unsigned)h << 16;
  float v;
  std::memcpy(&v, &u, 4);
  return v;
}

}  // namespace

int elem_tile_count() { return kNumTiles; }

bool elem_tile_fits(int N, int tile) {
  if (tile < 0 || tile >= kNumTiles) return false;
  const TileShape t = kTiles[tile];
  return N >= t.tx && N >= t.ty && N >= t.tz && N % t.tx == 0 && N % t.ty == 0 && N % t.tz == 0;
}

void elem_operand_host(int op, const double* kref, unsigned short* out) {
  const int FO = op_fields_out(op), FI = op_fields_in(op);
  // padded block M[4c + fo][4c' + fi]
  double M[32][32];
  for (int r = 0; r < 32; ++r)
    for (int q = 0; q < 32; ++q) M[r][q] = 0.0;
  for (int c = 0; c < 8; ++c)
    for (int fo = 0; fo < FO; ++fo)
      for (int cp = 0; cp < 8; ++cp)
        for (int fi = 0; fi < FI; ++fi) M[4 * c + fo][4 * cp + fi] = kref[(c * FO + fo) * (8 * FI) + cp * FI + fi];
  // A operand of row tile t for lane l: row 16t + l % 16, columns 8 (l / 16) + j
  for (int t = 0; t < 2; ++t)
    for (int l = 0; l < 64; ++l)
      for (int j = 0; j < 8; ++j) {
        const float v = (float)M[16 * t + l % 16][8 * (l / 16) + j];
        const unsigned short h = rne_bf16_host(v);
        const unsigned short lo = rne_bf16_host(v - bf16_to_float_host(h));
        out[(t * 64 + l) * 8 + j] = h;
        out[((2 + t) * 64 + l) * 8 + j] = lo;
      }
}

void elem_apply(int op, int nrhs, int N, int terms, int tile, const float* s, const void* kop, const float* x,
                const OpArgs<float>& a, bool cheby, hipStream_t st) {
  if (nrhs != 9) throw std::invalid_argument("elem_apply: nine load columns");
  if (!elem_tile_fits(N, tile)) throw std::invalid_argument("elem_apply: tile does not divide N");
  const unsigned n = (unsigned)N;
#define PHZ_EA(OPV)                                                    \
  do {                                                                 \
    if (terms == 3) launch_elem<OPV, 3>(tile, n, s, kop, x, a, cheby, st); \
    else if (terms == 1) launch_elem<OPV, 1>(tile, n, s, kop, x, a, cheby, st); \
    else throw std::invalid_argument("elem_apply: terms");             \
  } while (0)
  switch (op) {
    case 0: PHZ_EA(0); break;
    case 1: PHZ_EA(1); break;
    case 2: PHZ_EA(2); break;
    case 3: PHZ_EA(3); break;
    default: throw std::invalid_argument("elem_apply op");
  }
#undef PHZ_EA
  PHZ_LAUNCH_CHECK();
}

}  // namespace phz
