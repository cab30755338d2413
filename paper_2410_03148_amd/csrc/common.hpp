// Shared declarations of the HIP kernels' host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace phz {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define PHZ_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::phz::HipError(std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define PHZ_LAUNCH_CHECK() PHZ_HIP(hipGetLastError())

// Maximum GMRES restart length supported by the fused Arnoldi kernels.
constexpr int kMaxRestart = 32;

// ---- operators (ops.hip) -----------------------------------------------------
// Output side of an operator launch: y = beta*yin + alpha*(A x), and with the
// Chebyshev epilogue (square blocks only) also, per node and column,
// dnew = ca*dold + cb*Dinv*y and x = xin + dnew (+ dold if fold_dold; xin
// null reads as zero), with (ca, cb) = (cab[0], cab[1]) read on the device.
// y may alias yin and x may alias xin; dnew must not alias the operator input.
template <typename T>
struct OpArgs {
  const T* yin = nullptr;
  T* y = nullptr;
  T alpha = T(1), beta = T(0);
  const T* dinv = nullptr;
  const T* dold = nullptr;
  T* dnew = nullptr;
  const T* xin = nullptr;
  T* x = nullptr;
  const T* cab = nullptr;
  int fold_dold = 0;
  // plain (non-Chebyshev) epilogue of a square block: when set, also the
  // first Chebyshev step on the output, d1 = cab[0] * dinv y (no iterate
  // update), so that a residual and the next smoothing step's first
  // correction come out of one pass
  T* d1 = nullptr;
};

// Fine-level matrix-free block operator on sum_e s_e Kref.
// op: 0 full (4->4), 1 A (3->3), 2 B (3->1), 3 S_bar (1->1).  nrhs in {1, 9}.
// kref is the op's reference block in (l*FO + fo, l'*FI + fi) layout.
template <typename T>
void fine_apply(int op, int nrhs, int N, const T* s, const T* kref, const T* x, const OpArgs<T>& a,
                bool cheby, hipStream_t st);

// The full operator (4 x 4 fields) with the material interpolated at the
// quadrature points: point scales sq[8 e + p], per-point reference terms
// kq[p][32 x 32]; nrhs in {1, 9}
template <typename T>
void fine_apply_qp(int nrhs, int N, const T* sq, const T* kq, const T* x, const OpArgs<T>& a, hipStream_t st);

// The float32 fine-level gather with the workgroup's input tile (16 x 4 x 4
// nodes and a one-node halo, all columns) staged in LDS; nine columns, N a
// multiple of 16 (fine_tiled_fits).
bool fine_tiled_fits(int N);
void fine_apply_tiled(int op, int nrhs, int N, const float* s, const float* kref, const float* x,
                      const OpArgs<float>& a, bool cheby, hipStream_t st);

// Fine-level operator as an element contraction on MFMA in split-BF16
// arithmetic (elem.hip), FP32 vectors, nine load columns.  kop holds the op's
// reference block padded to 32 x 32 and split into bf16 hi and lo in MFMA
// operand order (2048 values from elem_operand_host).  terms: 3 (hi*hi +
// hi*lo + lo*hi) or 1 (hi*hi).  tile: a tile-shape index < elem_tile_count()
// with elem_tile_fits(N, tile).
int elem_tile_count();
bool elem_tile_fits(int N, int tile);
void elem_operand_host(int op, const double* kref, unsigned short* out);
void elem_apply(int op, int nrhs, int N, int terms, int tile, const float* s, const void* kop, const float* x,
                const OpArgs<float>& a, bool cheby, hipStream_t st);

// Coarse-level apply with assembled 27-point node stencils S laid out
// structure-of-arrays [(d*F + fo)*F + fi][node].
template <typename T>
void coarse_apply(int F, int nrhs, int N, const T* S, const T* x, const OpArgs<T>& a, bool cheby,
                  hipStream_t st);
// The float32 nine-column coarse apply with the workgroup's input tile
// (16 x 4 x 4 nodes and a one-node halo) staged in LDS; N a multiple of 16
// (coarse_tiled_fits).
bool coarse_tiled_fits(int N);
void coarse_apply_tiled(int F, int N, const float* S, const float* x, const OpArgs<float>& a, bool cheby,
                        hipStream_t st);
// The same with the compact stencil form (compact_stencil): the 26
// off-centre blocks in bf16 (S16, [d'][fo][fi][n], centre skipped) and the
// centre block in float32 as minus their sum (Sc, [fo][fi][n]).
void coarse_apply_tiled_compact(int F, int N, const unsigned short* S16, const float* Sc, const float* x,
                                const OpArgs<float>& a, bool cheby, hipStream_t st);
void compact_stencil(int F, long nn, const double* S, unsigned short* S16, float* Sc, hipStream_t st);
// Node stencils of a coarse level from its Galerkin element matrices
// (structure-of-arrays [corner L][row f][col][element]).
void build_stencil(int F, int N, const double* Ae, double* S, hipStream_t st);

// Galerkin coarsening of element matrices: coarse element E gets
// sum_children Q_c^T K_c Q_c with trilinear Q_c.  From the fine level
// (s != nullptr: K_c = s_c kref, so K_E = sum_c s_c M_c with the eight fixed
// M_c = Q_c^T kref Q_c, built into mq: 8 (8F)^2 doubles of device memory) or
// from stored matrices Afine (mq unused).
void galerkin_build(int F, int Nf, const double* s, const double* kref, const double* Afine,
                    double* Acoarse, double* mq, hipStream_t st);

// Inverse node-block diagonal (F x F per node), fine or coarse level.
void diag_inv_fine(int F, int N, const double* s, const double* kref, double* Dinv,
                   hipStream_t st);
void diag_inv_coarse(int F, int N, const double* Ae, double* Dinv, hipStream_t st);

// First Chebyshev-Jacobi step: d = cf[0] Dinv r (cf on the device), and x
// per xmode: untouched (kChebyXNone: the next step folds d into x), x = d
// (kChebyXSet) or x += d (kChebyXAdd).  r, d and x may alias (per-node
// in-place).
enum { kChebyXNone = 0, kChebyXSet = 1, kChebyXAdd = 2 };
template <typename T>
void cheby_first(int F, int nrhs, long nn, const T* Dinv, const T* r, T* d, T* x, const T* cf, int xmode,
                 hipStream_t st);

// Full-weighting restriction rc = P^T rf and prolongation xf += P xc (periodic,
// trilinear).  Nc = coarse N.
template <typename T>
void restrict_fw(int F, int nrhs, int Nc, const T* rf, T* rc, hipStream_t st);
template <typename T>
void prolong_add(int F, int nrhs, int Nc, const T* xc, T* xf, hipStream_t st);

// z = Minv r on the coarsest level: dense float64 matrix over rows (f*nc + n).
template <typename T>
void dense_apply(int F, int nc, int nrhs, const double* Minv, const T* r, T* z, hipStream_t st);

// ---- vectors / reductions / physics (vec.hip) --------------------------------
// Vectors are structure of arrays: F*K columns (field f, load k -> column
// f*K + k) of nn contiguous node values.
template <typename Ts, typename Td>
void convert(long count, const Ts* src, Td* dst, hipStream_t st);
template <typename T>
void fill(long count, T value, T* dst, hipStream_t st);

// scratch (doubles) needed by every reduction below
size_t reduce_work_size();
// out[k] = sum over fields and nodes of v^2, per load column k (double)
template <typename T>
void col_norm2(long nn, int F, int K, const T* v, double* out, double* work, hipStream_t st);
// out[k] = sum over the F fields of column k of a . b (float64 accumulation)
template <typename T>
void col_dot(long nn, int F, int K, const T* a, const T* b, double* out, double* work, hipStream_t st);
// p = z + beta[k] p, per load column k
template <typename T>
void xpby_cols(long nn, int F, int K, const double* beta, const T* z, T* p, hipStream_t st);
// out[f*K + k] = sum over nodes of column (f, k)
template <typename T>
void field_sums(long nn, int F, int K, const T* v, double* out, double* work, hipStream_t st);
// v[(f, k)][n] -= sums[f*K + k] / nn
template <typename T>
void subtract_mean(long nn, int F, int K, const double* sums, T* v, hipStream_t st);

// Arnoldi passes with the basis V_i = V + i*vstride:
//   dots:    hout[i*K + k] = <V_i, w>_k for i <= j
//   update:  w -= sum_i V_i hin[i*K + k]; then (if hout) hout = V^T w_new and
//            (if nrm2out) nrm2out[k] = ||w_new||_k^2
template <typename T>
void arnoldi_dots(long nn, int F, int K, int j, const T* V, long vstride, const T* w, double* hout,
                  double* work, hipStream_t st);
template <typename T>
void arnoldi_update(long nn, int F, int K, int j, const T* V, long vstride, T* w, const double* hin,
                    double* hout, double* nrm2out, double* work, hipStream_t st, const int* flags = nullptr);
// selective reorthogonalisation: flag[k] = active[k] and |h2_k|^2 > tau2
// na2[k] (a second Gram-Schmidt pass is needed), h2 zeroed where not;
// count[k] += flag[k]
void reorth_decide(int K, int J, double tau2, double* h2, const double* na2, const int* active, int* flag,
                   int* count, hipStream_t st);
// v = w * scale[k] (in place allowed)
template <typename T>
void scale_cols(long nn, int F, int K, const T* w, const double* scale, T* v, hipStream_t st);
// t = sum_{i < kused[k]} V_i y[i*K + k]
template <typename T>
void combine(long nn, int F, int K, const T* V, long vstride, const double* y, const int* kused, T* t,
             hipStream_t st);
// x += a[k] * z (a may be null -> 1), mixed precision source allowed
template <typename Tx, typename Tz>
void axpy_cols(long nn, int F, int K, const double* a, const Tz* z, Tx* x, hipStream_t st);
// one load of a 9-load block <-> a single-load vector (4 fields)
void extract_column(long nn, int load, const double* block, double* col, hipStream_t st);
void insert_column(long nn, int load, const double* col, double* block, hipStream_t st);
// structure of arrays [ncol][nn] <-> node-major [nn][ncol]
void soa_to_aos(long nn, int ncol, const double* src, double* dst, hipStream_t st);
void aos_to_soa(long nn, int ncol, const double* src, double* dst, hipStream_t st);

// GMRES small-matrix kernels (one workgroup; state arrays in device memory).
struct GmresState {
  double* H;        // [(m+1)][m][K]
  double* cs;       // [m][K]
  double* sn;       // [m][K]
  double* g;        // [(m+1)][K]
  double* y;        // [m][K]
  double* est;      // [m][K] relative residual estimates
  double* bnorm;    // [K]
  double* scale;    // [K] 1/h_{j+1,j} or 0
  int* active;      // [K]
  int* kused;       // [K]
  int* nactive;     // [1]
  const double* tol = nullptr;  // [K] per-column relative tolerance, or nullptr: the scalar one
};
// start of a cycle: beta = sqrt(nrm2); g[0] = beta; active if beta > tol*bnorm;
// scale = 1/beta or 0.
void gmres_start(int nrhs, const double* nrm2, double rtol, GmresState s, hipStream_t st);
// Givens step j: a column stops at its tolerance, at the restart length, and,
// with stall > 0, once its estimate fell by less than the factor `stall` over
// two steps (a float cycle whose operator error floors it).
// flag, na2 (may be null): where flag[k] = 0 the new vector's norm^2 is
// na2[k] (no second Gram-Schmidt pass) instead of nrm2[k].
void gmres_givens(int nrhs, int m, int j, const double* h1, const double* h2,
                  const double* nrm2, double rtol, double stall, GmresState s, hipStream_t st,
                  const int* flag = nullptr, const double* na2 = nullptr);
void gmres_solve_y(int nrhs, int m, GmresState s, hipStream_t st);

// physics
void levelset_to_scale(int N, const double* phi, double eta, double void_scale, double* rho,
                       double* s, float* s32, hipStream_t st);
void density_to_scale(long nn, const double* rho, double void_scale, double* s, float* s32,
                      hipStream_t st);
// b[(f*9 + L)][n] = -sum_e s_e F0 e_L; absval: sum_e s_e |F0| (a magnitude reference)
void build_rhs(int N, const double* s, const double* F0, double* b, hipStream_t st, bool absval = false);
// quadrature-point smoothing: point scales sq[8 e + p] (p = i + 2j + 4k) and
// their element means; point scales from element scales; the load vectors
// from point scales and the per-point terms F0q[p][32 x 9]
void levelset_to_scale_qp(int N, const double* phi, double eta, double void_scale, double* rho, double* s,
                          float* s32, double* sq, float* sq32, hipStream_t st);
void point_scales(long nn, const double* s, double* sq, float* sq32, hipStream_t st);
void build_rhs_qp(int N, const double* sq, const double* F0q, double* b, hipStream_t st, bool absval = false);
// as reduce_effective (out[l*36 + col] only) with the scales of point p
void reduce_effective_point(int N, const double* sq, int p, const double* X, double* out, double* work,
                            hipStream_t st);
// out[l*36 + f*9 + L] = sum_e s_e x_{node(e,l)}[f][L]; out[288] = sum_e s_e
void reduce_effective(int N, const double* s, const double* X, double* out, double* work,
                      hipStream_t st);
// out[b*9 + a] = sum_{f, n} X[(f, a)][n] Y[(f, b)][n]  (9-load blocks)
void cross_dots(long nn, const double* X, const double* Y, double* out, double* work, hipStream_t st);
// U = X W per node (W 9 x 9 over the load columns, X and U [4][9][nn])
void mix_cols(long nn, const double* X, const double* W, double* U, hipStream_t st);
// grad[stride e + off] = factor (cterm + <X_e, FW> + sum_L U_e[:, L]^T K0 X_e[:, L]), U = X W
void backward_elem(int N, const double* X, const double* U, const double* K0, const double* FW, double cterm,
                   double factor, double* grad, hipStream_t st, int stride = 1, int off = 0);
void grad_phi(int N, const double* phi, double eta, const double* grad_rho, double* out,
              hipStream_t st);
// chain rule of the point densities to the nodes: g per point (stride 8) or
// per element spread evenly over its points (stride 1)
void grad_phi_qp(int N, const double* phi, double eta, const double* g, int stride, double* out, hipStream_t st);
// ge[e] = sum_p gq[8 e + p]
void sum_points(long nn, const double* gq, double* ge, hipStream_t st);
void nodal_mean_of_elements(int N, const double* ge, double* vn, hipStream_t st);
void max_abs(long count, const double* v, double* out, double* work, hipStream_t st);
void hj_step(int N, const double* phi, const double* v, const double* vmax, double dt,
             double* out, hipStream_t st);
// one pseudo-time step of the reinitialisation equation towards a signed
// distance, smoothed sign taken from phi0
void reinit_step(int N, const double* phi, const double* phi0, double dt, int subcell, double* out,
                 hipStream_t st);
// y = W x, a constant 27-point stencil w[dx + 3 dy + 9 dz] (offsets -1..1), K node columns
// TriCG update of one block (F fields, K loads) with per-load coefficients
// cf[6k..6k+5] = (L00, L01, L10, L11, z0, z1): g1 <- [side 0] w - (L00 g1 +
// L01 g2), g2 <- [side 1] w - (L10 g1 + L11 g2), x += z0 g1 + z1 g2
void tricg_update(long nn, int F, int K, const double* cf, const double* w, int side, double* g1, double* g2,
                  double* x, hipStream_t st);
// one Chebyshev step for a constant 27-point stencil (K columns):
// x += d, r -= W d, dn = c1 d + c2 r
void stencil_cheb_step(int N, int K, const double* w, const double* d, double* x, double* r, double* dn, double c1,
                       double c2, hipStream_t st);
int count_nonfinite(long count, const double* v, double* work, hipStream_t st);
// number of values that are not finite or lie outside [lo, hi]
int count_outside(long count, const double* v, double lo, double hi, double* work, hipStream_t st);
// power iteration helper: v = w / sqrt(nrm2[0])
template <typename T>
void normalize_by(long count, const double* nrm2, const T* w, T* v, hipStream_t st);
void hash_fill(long count, unsigned seed, double* v, hipStream_t st);

}  // namespace phz
