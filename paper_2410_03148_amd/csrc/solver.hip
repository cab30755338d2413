// Host runtime and C ABI of the periodic piezoelectric homogenisation solver.
//
// Solve path (Sec. 2.5.3 of the paper, SCP-GMRES):
//   calA = [[A, B^T], [B, -C]],  P = [[A, 0], [B, -S_bar]],
//   right-preconditioned GMRES(m) on calA P^-1, with
//   P^-1 (r_u, r_p) = (z_u, z_p):  z_u = A^-1 r_u,  z_p = S_bar^-1 (B z_u - r_p).
// A^-1 and S_bar^-1 are geometric-multigrid V-cycles (Galerkin coarse
// operators, Chebyshev-Jacobi smoothing, dense coarsest solve), a fixed
// number per application so that P^-1 is a fixed linear operator.
// The nine load columns run either as one 9-column block (one operator
// apply serves all nine; nine independent Arnoldi processes in lockstep with
// per-column convergence masks) or one at a time.
// The FP32_IR form runs the same GMRES in float (operator, smoothers and
// Krylov basis; float64 inner products, Hessenberg and Givens) as the inner
// solver of float64 iterative refinement on the true residual.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "piezohom.h"
#include "refelem.hpp"

namespace phz {

// Device memory of a context: the caller's allocator (phz_create's
// phz_allocator) when one was given, else hipMalloc.  Every entry point that
// takes a context makes that context's hook current for the calling thread
// (AllocScope); a buffer remembers the hook it was allocated with and returns
// its memory through it.
struct AllocHook {
  phz_allocator a{};
  hipStream_t stream = nullptr;
  bool active = false;
};
static thread_local const AllocHook* g_alloc_hook = nullptr;
struct AllocScope {
  const AllocHook* prev;
  explicit AllocScope(const AllocHook* h) : prev(g_alloc_hook) { g_alloc_hook = h; }
  ~AllocScope() { g_alloc_hook = prev; }
};

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  const AllocHook* hook = nullptr;   // allocator the memory came from (null: hipMalloc)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      if (hook) hook->a.free(p, hook->stream, hook->a.user);
      else hipFree(p);
    }
    p = nullptr;
    n = 0;
    hook = nullptr;
  }
  void alloc(size_t count) {
    if (count == n && p) return;
    release();
    if (count == 0) return;
    const AllocHook* h = g_alloc_hook && g_alloc_hook->active ? g_alloc_hook : nullptr;
    if (h) {
      p = static_cast<T*>(h->a.alloc(count * sizeof(T), h->stream, h->a.user));
      if (!p) throw HipError(std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) +
                             " bytes: the caller's allocator returned NULL");
      hook = h;
    } else {
      hipError_t e = hipMalloc(&p, count * sizeof(T));
      if (e != hipSuccess) {
        p = nullptr;
        throw HipError(std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) +
                       " bytes: " + hipGetErrorString(e));
      }
    }
    n = count;
  }
  void upload(const T* h, size_t count, hipStream_t st) {
    alloc(count);
    PHZ_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, st));
  }
};

struct Level {
  int N = 0;
  long nn = 0;
  DevBuf<double> Ae;      // Galerkin element matrices (levels >= 1)
  DevBuf<double> S;       // assembled 27-point node stencils (levels >= 1)
  DevBuf<float> S32;
  // compact float form of S for the tiled apply: off-centre blocks in bf16,
  // the centre block minus their sum (levels whose side is a multiple of 16)
  DevBuf<unsigned short> S16;
  DevBuf<float> Sc;
  DevBuf<double> pv, pw, py;  // power-iteration vectors, kept across set-ups
  DevBuf<double> Dinv;    // node-block diagonal inverse
  DevBuf<float> Dinv32;
  double lmax = 0.0;
  // Chebyshev coefficients on the device, read by the smoothing kernels (so a
  // captured launch sequence stays valid when the geometry changes):
  // [0] = 1/theta, [2i] = ca_i, [2i+1] = cb_i for steps i = 1 .. degree-1
  std::vector<double> cheb_host;
  std::vector<float> cheb_host32;
  DevBuf<double> cheb;
  DevBuf<float> cheb32;
  // kernel of the float32 nine-column applies of this coarse level: 0 the
  // direct stencil apply, 1 the LDS-tiled one, 2 the LDS-tiled one on the
  // compact stencils, -1 not yet chosen
  int ckind = -1;
};

struct Hierarchy {
  int F = 0;              // 3 for A, 1 for S_bar
  int op = 0;             // fine-level operator id
  std::vector<std::unique_ptr<Level>> lv;
  int rows = 0;           // coarsest dense size
  DevBuf<double> Minv;
  DevBuf<double> Mq;      // the first coarsening's eight fixed child blocks
};

template <typename T>
struct LevelWork {
  DevBuf<T> b, x, r, d, d2;
};

template <typename T>
struct Work {
  int cap_k = 0, cap_m = 0;
  std::vector<std::unique_ptr<LevelWork<T>>> A, S, C;
  DevBuf<T> t1u, t2u, t1p, t2p, t3p;   // preconditioner temporaries
  DevBuf<T> pr, pz, pp, pq;            // conjugate gradients of the inexact block maps
  DevBuf<T> V, w, z, t, r, b, x;                  // GMRES
  DevBuf<T> Z;  // preconditioned basis P^-1 V_j (flexible GMRES, the float cycles)
};

// One Arnoldi step (preconditioner, operator, orthogonalisation, Givens,
// next basis vector) captured as a HIP graph.  Valid while the buffers it
// was captured on stay in place (graph epoch) and for the same columns,
// tolerance and stall factor.
struct StepGraph {
  hipGraphExec_t exec = nullptr;
  int K = 0;
  double rtol = 0.0, stall = 0.0;
  const double* tol = nullptr;
  long epoch = -1;
};

}  // namespace phz

struct phz_ctx {
  phz::AllocHook hook;   // first member: destroyed after every buffer that uses it
  int N = 0;
  long nn = 0;
  phz_material mat{};
  phz_options opt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;

  phz::RefElement ref;
  // reference blocks: 0 full, 1 A, 2 B, 3 S_bar, and 4 C (the dielectric
  // block, a 1 -> 1 block like S_bar, used by the block-diagonal
  // preconditioner)
  phz::DevBuf<double> kref_full, kref_A, kref_B, kref_S, kref_C, kref_BT, F0d;
  // quadrature-point smoothing: per-point reference terms and point scales
  phz::DevBuf<double> kq64, f0q, sq;
  phz::DevBuf<float> kq32, sq32;
  phz::DevBuf<float> kref32_full, kref32_A, kref32_B, kref32_S, kref32_C, kref32_BT;
  // split-BF16 MFMA operands of the five fine blocks, the tile choice of the
  // four block shapes (-1 not yet chosen, -2 none divides N), and the kernel
  // chosen for each shape's float32 nine-column launches
  phz::DevBuf<unsigned short> kop[5];
  int elem_tile[4] = {-1, -1, -1, -1};
  int fkind[4] = {-1, -1, -1, -1};   // kernel of the float32 nine-column launches, -1 not yet chosen

  phz::DevBuf<double> phi, rho, s, grad_rho, tmp_nodes;
  phz::DevBuf<double> grad_q;  // per-point density gradient (quadrature-point smoothing)
  phz::DevBuf<double> bw_u;    // U = X W of the backward pass (36 nn)
  // node-sized staging of the optimisation entry points and the backward's
  // per-term block, kept so repeated calls do not allocate
  phz::DevBuf<double> node_a, node_b, bw_terms;
  phz::DevBuf<float> s32;
  bool have_phi = false, have_s = false, have_solution = false, have_grad = false;
  bool x_valid = false;   // X holds the finite result of the last solve (any geometry)
  bool precond_ready = false;
  bool have_guess = false;
  // refinement-stall fallback of the current solve: 0 the configured form,
  // 1 float32 kernels only (a split-BF16 context leaves its bf16 products
  // and bf16 stencils), 2 a float64 inner GMRES
  int ir_level = 0;

  phz::Hierarchy hA, hS, hC;   // hC: only for the block-diagonal preconditioner
  phz::Work<double> w64;
  phz::Work<float> w32;

  phz::DevBuf<double> X, Bvec, R64, guess, col_b, col_x, col_r;  // [nn][4][9] and columns
  phz::DevBuf<double> red_work, small;   // reduction scratch, small device values
  phz::DevBuf<double> gm_H, gm_cs, gm_sn, gm_g, gm_y, gm_est, gm_bnorm, gm_scale, gm_h1, gm_h2, gm_nrm;
  phz::DevBuf<double> gm_tol;  // per-column relative targets of a float refinement cycle
  phz::DevBuf<int> gm_int;
  phz::DevBuf<double> gm_na2;  // |w|^2 after the first Gram-Schmidt pass, per load
  phz::DevBuf<int> gm_flag, gm_reorth;  // second pass needed per load; second passes counted per load

  // captured Arnoldi steps (use_graph), per precision and step index; the
  // epoch advances whenever a buffer they reference may have moved
  std::vector<phz::StepGraph> graphs64, graphs32;
  long graph_epoch = 0;
  phz::DevBuf<double> one64;   // the constant 1.0 (power-iteration Jacobi step)
  phz::DevBuf<double> negone;  // nine copies of -1.0 (block-diagonal preconditioner)
  // optimisation step: Helmholtz stencil, conjugate-gradient vectors and
  // scalars of the Riesz solves, the velocity's direction vectors
  phz::DevBuf<double> helm_w, rz_r, rz_z, rz_p, rz_g, rz_j, rz_dev;
  double rz_host[40] = {};  // staged stencil weights and column scales (outlive their async copies)
  phz::DevBuf<double> pcg_dev; // per-column scalars of the inexact block maps
  // TriCG vectors: displacement block [3][K][nn], potential block [K][nn]
  phz::DevBuf<double> tri_u, tri_Eu, tri_Eup, tri_q, tri_Eq, tri_g1x, tri_g2x;
  phz::DevBuf<double> tri_v, tri_Fv, tri_Fvp, tri_p, tri_Fp, tri_g1y, tri_g2y;
  phz::DevBuf<double> tri_dev;  // per-load coefficients and reductions

  // optional per-kernel timing with HIP events on the context stream
  bool ktime = false;
  bool ktime_fine_only = false;   // timing mode 2: fine-level operator launches only
  std::vector<hipEvent_t> ev;           // start/stop pairs
  std::vector<std::string> ev_name;
  size_t ev_used = 0;
  std::map<std::string, std::pair<long, double>> ktotals;

  double MH[81] = {0}, MHe[81] = {0};
  std::vector<double> hist[9];
  phz_stats stats{};
};

namespace phz {

static const char* kStatusNames[] = {"ok", "not converged", "invalid argument", "NaN or Inf",
                                     "HIP runtime error", "out of memory", "invalid state",
                                     "internal error"};

using Clock = std::chrono::steady_clock;
static double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

static void sync(phz_ctx* c) { PHZ_HIP(hipStreamSynchronize(c->stream)); }

constexpr size_t kMaxTimedLaunches = 1 << 16;

// Record a start event before a launch; returns the slot or -1.
static long time_begin(phz_ctx* c, const char* name) {
  if (!c->ktime || c->ev_used >= kMaxTimedLaunches) return -1;
  if (c->ktime_fine_only && std::strncmp(name, "fine", 4) != 0 && std::strncmp(name, "tiled_", 6) != 0 &&
      std::strncmp(name, "elem_", 5) != 0)
    return -1;
  const size_t i = c->ev_used++;
  if (c->ev.size() < 2 * (i + 1)) {
    hipEvent_t a, b;
    PHZ_HIP(hipEventCreate(&a));
    PHZ_HIP(hipEventCreate(&b));
    c->ev.push_back(a);
    c->ev.push_back(b);
    c->ev_name.emplace_back();
  }
  c->ev_name[i] = name;
  PHZ_HIP(hipEventRecord(c->ev[2 * i], c->stream));
  return (long)i;
}
static void time_end(phz_ctx* c, long slot) {
  if (slot < 0) return;
  PHZ_HIP(hipEventRecord(c->ev[2 * slot + 1], c->stream));
}
// Fold recorded launch durations into the per-name totals (after a sync).
static void collect_timing(phz_ctx* c) {
  for (size_t i = 0; i < c->ev_used; ++i) {
    float ms = 0.0f;
    PHZ_HIP(hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
    auto& t = c->ktotals[c->ev_name[i]];
    t.first += 1;
    t.second += ms;
  }
  c->ev_used = 0;
}

// ------------------------------------------------------------------ setup
static void upload_reference(phz_ctx* c) {
  c->ref = build_ref_element(c->mat, 1.0 / c->N);
  const RefElement& R = c->ref;
  hipStream_t st = c->stream;
  c->kref_full.upload(R.K0, 32 * 32, st);
  c->kref_A.upload(R.A0, 24 * 24, st);
  c->kref_B.upload(R.B0, 8 * 24, st);
  c->kref_S.upload(R.S0, 8 * 8, st);
  c->kref_C.upload(R.C0, 8 * 8, st);
  // B^T in the 3 <- 1 block layout [(corner c, field f)][corner m]
  double BT[24 * 8];
  for (int cn = 0; cn < 8; ++cn)
    for (int f = 0; f < 3; ++f)
      for (int m = 0; m < 8; ++m) BT[(cn * 3 + f) * 8 + m] = R.B0[m * 24 + cn * 3 + f];
  c->kref_BT.upload(BT, 24 * 8, st);
  c->kq64.upload(&R.K0q[0][0], 8 * 1024, st);
  c->f0q.upload(&R.F0q[0][0], 8 * 288, st);
  sync(c);
  c->F0d.upload(R.F0, 32 * 9, st);
  std::vector<float> f(32 * 32);
  auto up32 = [&](DevBuf<float>& d, const double* h, int n) {
    for (int i = 0; i < n; ++i) f[i] = (float)h[i];
    d.upload(f.data(), n, st);
    sync(c);
  };
  up32(c->kref32_full, R.K0, 32 * 32);
  up32(c->kref32_A, R.A0, 24 * 24);
  up32(c->kref32_B, R.B0, 8 * 24);
  up32(c->kref32_S, R.S0, 8 * 8);
  up32(c->kref32_C, R.C0, 8 * 8);
  up32(c->kref32_BT, BT, 24 * 8);
  {
    std::vector<float> kq(8 * 1024);
    for (int i = 0; i < 8 * 1024; ++i) kq[i] = (float)(&R.K0q[0][0])[i];
    c->kq32.upload(kq.data(), kq.size(), st);
    sync(c);
  }
  std::vector<unsigned short> ops(2048);
  const double* krefs[5] = {R.K0, R.A0, R.B0, R.S0, R.C0};
  for (int op = 0; op < 5; ++op) {
    elem_operand_host(op == 4 ? 3 : op, krefs[op], ops.data());
    c->kop[op].upload(ops.data(), ops.size(), st);
    sync(c);
  }
}

// Side of the coarsest level under the halving rule of build_levels.  Its
// dense inverse is formed on the host, so the side is bounded by
// kMaxCoarsestN (at most 3 * 10^3 rows).
static const int kMaxCoarsestN = 10;
static int coarsest_side(int N, int mg_levels) {
  const int maxl = mg_levels > 0 ? mg_levels : 64;
  int levels = 1;
  while (N % 2 == 0 && N > 4 && levels < maxl) {
    N /= 2;
    ++levels;
  }
  return N;
}

// Level sizes N, N/2, ... while N is even and above 4 (or mg_levels levels).
// Existing levels of the same structure are kept, so their device buffers
// (and any launch sequence captured on them) stay where they are.
static void build_levels(phz_ctx* c, Hierarchy& H, int F, int op) {
  std::vector<int> sizes;
  int N = c->N;
  const int maxl = c->opt.mg_levels > 0 ? c->opt.mg_levels : 64;
  for (;;) {
    sizes.push_back(N);
    if (!(N % 2 == 0 && N > 4 && (int)sizes.size() < maxl)) break;
    N /= 2;
  }
  bool same = H.F == F && H.op == op && H.lv.size() == sizes.size();
  for (size_t l = 0; same && l < sizes.size(); ++l) same = H.lv[l]->N == sizes[l];
  if (same) return;
  H.F = F;
  H.op = op;
  H.lv.clear();
  for (int n : sizes) {
    auto L = std::make_unique<Level>();
    L->N = n;
    L->nn = (long)n * n * n;
    H.lv.push_back(std::move(L));
  }
  ++c->graph_epoch;
}

// Krylov basis vectors are padded apart so that the many concurrent streams
// of an Arnoldi pass do not sit at power-of-two distances
static size_t basis_stride(long nn, int K) { return (size_t)nn * 4 * K + 512; }

template <typename T>
static void alloc_work(phz_ctx* c, Work<T>& W, int K, int m) {
  if (W.cap_k >= K && W.cap_m >= m && !W.A.empty()) return;
  ++c->graph_epoch;
  const long nn = c->nn;
  auto mk = [&](Hierarchy& H, std::vector<std::unique_ptr<LevelWork<T>>>& out) {
    out.clear();
    for (size_t l = 0; l < H.lv.size(); ++l) {
      auto w = std::make_unique<LevelWork<T>>();
      const size_t cnt = (size_t)H.lv[l]->nn * H.F * K;
      w->r.alloc(cnt);
      w->d.alloc(cnt);
      w->d2.alloc(cnt);
      if (l > 0) {
        w->b.alloc(cnt);
        w->x.alloc(cnt);
      }
      out.push_back(std::move(w));
    }
  };
  mk(c->hA, W.A);
  mk(c->hS, W.S);
  mk(c->hC, W.C);
  const size_t u = (size_t)nn * 3 * K, p = (size_t)nn * K, full = (size_t)nn * 4 * K;
  W.t1u.alloc(u); W.t2u.alloc(u);
  W.t1p.alloc(p); W.t2p.alloc(p); W.t3p.alloc(p);
  W.V.alloc(basis_stride(nn, K) * (m + 1));
  if (std::is_same<T, float>::value || c->opt.inner == 1) W.Z.alloc(basis_stride(nn, K) * m);
  W.w.alloc(full); W.z.alloc(full); W.t.alloc(full); W.r.alloc(full); W.b.alloc(full); W.x.alloc(full);
  W.cap_k = K;
  W.cap_m = m;
}

static void ensure_state_buffers(phz_ctx* c) {
  const int m = c->opt.restart, K = 9;
  c->gm_H.alloc((size_t)(m + 1) * m * K);
  c->gm_cs.alloc((size_t)m * K);
  c->gm_sn.alloc((size_t)m * K);
  c->gm_g.alloc((size_t)(m + 1) * K);
  c->gm_y.alloc((size_t)m * K);
  c->gm_est.alloc((size_t)m * K);
  c->gm_bnorm.alloc(K);
  c->gm_scale.alloc(K);
  c->gm_h1.alloc((size_t)(kMaxRestart + 1) * K);
  c->gm_h2.alloc((size_t)(kMaxRestart + 1) * K);
  c->gm_nrm.alloc(4 * K);
  c->gm_int.alloc(3 * K + 1);
  c->gm_na2.alloc(K);
  c->gm_flag.alloc(K);
  c->gm_reorth.alloc(K);
  c->gm_tol.alloc(K);
  c->red_work.alloc(reduce_work_size());
  c->small.alloc(512);
}

static GmresState gm_state(phz_ctx* c) {
  GmresState s;
  s.H = c->gm_H.p;
  s.cs = c->gm_cs.p;
  s.sn = c->gm_sn.p;
  s.g = c->gm_g.p;
  s.y = c->gm_y.p;
  s.est = c->gm_est.p;
  s.bnorm = c->gm_bnorm.p;
  s.scale = c->gm_scale.p;
  s.active = c->gm_int.p;
  s.kused = c->gm_int.p + 9;
  s.nactive = c->gm_int.p + 27;
  return s;
}

// ---------------------------------------------------------- level operators
template <typename T> static const T* kref_of(phz_ctx* c, int op);
template <> const double* kref_of<double>(phz_ctx* c, int op) {
  return op == 0 ? c->kref_full.p : op == 1 ? c->kref_A.p : op == 2 ? c->kref_B.p : op == 3 ? c->kref_S.p
       : op == 4 ? c->kref_C.p : c->kref_BT.p;
}
template <> const float* kref_of<float>(phz_ctx* c, int op) {
  return op == 0 ? c->kref32_full.p : op == 1 ? c->kref32_A.p : op == 2 ? c->kref32_B.p
       : op == 3 ? c->kref32_S.p : op == 4 ? c->kref32_C.p : c->kref32_BT.p;
}
// launch shape (fields in and out) of a reference block: C is shaped like
// S_bar; B^T (block 5, 3 <- 1) has its own shape and only the direct gather
static int shape_of(int op) { return op == 4 ? 3 : op; }
template <typename T> static const T* s_of(phz_ctx* c);
template <> const double* s_of<double>(phz_ctx* c) { return c->s.p; }
template <> const float* s_of<float>(phz_ctx* c) { return c->s32.p; }
template <typename T> static const T* stencil_of(Level& L);
template <> const double* stencil_of<double>(Level& L) { return L.S.p; }
template <> const float* stencil_of<float>(Level& L) { return L.S32.p; }
template <typename T> static const T* dinv_of(Level& L);
template <> const double* dinv_of<double>(Level& L) { return L.Dinv.p; }
template <> const float* dinv_of<float>(Level& L) { return L.Dinv32.p; }
template <typename T> static Work<T>& work_of(phz_ctx* c);
template <> Work<double>& work_of<double>(phz_ctx* c) { return c->w64; }
template <> Work<float>& work_of<float>(phz_ctx* c) { return c->w32; }

// timing labels of the fine operator launches: block, load columns,
// precision, and "_cheby" for the launches with the fused smoothing step
static const char* fine_op_name(int op, int K, bool f32, bool cheby) {
  static const char* names[4][2][2][2] = {
      {{{"fine_full_k1_f64", "fine_full_k1_f64_cheby"}, {"fine_full_k1_f32", "fine_full_k1_f32_cheby"}},
       {{"fine_full_k9_f64", "fine_full_k9_f64_cheby"}, {"fine_full_k9_f32", "fine_full_k9_f32_cheby"}}},
      {{{"fine_A_k1_f64", "fine_A_k1_f64_cheby"}, {"fine_A_k1_f32", "fine_A_k1_f32_cheby"}},
       {{"fine_A_k9_f64", "fine_A_k9_f64_cheby"}, {"fine_A_k9_f32", "fine_A_k9_f32_cheby"}}},
      {{{"fine_B_k1_f64", "fine_B_k1_f64_cheby"}, {"fine_B_k1_f32", "fine_B_k1_f32_cheby"}},
       {{"fine_B_k9_f64", "fine_B_k9_f64_cheby"}, {"fine_B_k9_f32", "fine_B_k9_f32_cheby"}}},
      {{{"fine_S_k1_f64", "fine_S_k1_f64_cheby"}, {"fine_S_k1_f32", "fine_S_k1_f32_cheby"}},
       {{"fine_S_k9_f64", "fine_S_k9_f64_cheby"}, {"fine_S_k9_f32", "fine_S_k9_f32_cheby"}}}};
  return names[op][K == 9][f32][cheby];
}

template <typename T>
static OpArgs<T> plain_args(const T* yin, T* y, T alpha, T beta) {
  OpArgs<T> a;
  a.yin = yin;
  a.y = y;
  a.alpha = alpha;
  a.beta = beta;
  return a;
}

// timing labels of the split-BF16 element-contraction launches
static const char* elem_op_name(int op, bool three_terms, bool cheby) {
  static const char* names[4][2][2] = {
      {{"elem_full_k9_bf16x1", "elem_full_k9_bf16x1_cheby"}, {"elem_full_k9_bf16x3", "elem_full_k9_bf16x3_cheby"}},
      {{"elem_A_k9_bf16x1", "elem_A_k9_bf16x1_cheby"}, {"elem_A_k9_bf16x3", "elem_A_k9_bf16x3_cheby"}},
      {{"elem_B_k9_bf16x1", "elem_B_k9_bf16x1_cheby"}, {"elem_B_k9_bf16x3", "elem_B_k9_bf16x3_cheby"}},
      {{"elem_S_k9_bf16x1", "elem_S_k9_bf16x1_cheby"}, {"elem_S_k9_bf16x3", "elem_S_k9_bf16x3_cheby"}}};
  return names[op][three_terms][cheby];
}

// Kinds of a float32 nine-column fine-block launch.
enum { kFineDirect = 0, kFineTiled = 1, kFineElem = 2 };

static const char* tiled_op_name(int op, bool cheby) {
  static const char* names[4][2] = {{"tiled_full_k9_f32", "tiled_full_k9_f32_cheby"},
                                    {"tiled_A_k9_f32", "tiled_A_k9_f32_cheby"},
                                    {"tiled_B_k9_f32", "tiled_B_k9_f32_cheby"},
                                    {"tiled_S_k9_f32", "tiled_S_k9_f32_cheby"}};
  return names[op][cheby];
}

// Average time of a launch over three repetitions after one warm-up (HIP
// events on the context stream).
template <typename F>
static float time_launch(phz_ctx* c, F&& launch) {
  hipEvent_t e0, e1;
  PHZ_HIP(hipEventCreate(&e0));
  PHZ_HIP(hipEventCreate(&e1));
  launch();
  PHZ_HIP(hipEventRecord(e0, c->stream));
  for (int r = 0; r < 3; ++r) launch();
  PHZ_HIP(hipEventRecord(e1, c->stream));
  PHZ_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  PHZ_HIP(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return ms;
}

// Zero input and an output buffer for timing block `op` (the cost does not
// depend on the values).
struct TuneBufs {
  DevBuf<float> x, y;
  OpArgs<float> a;
};
static void tune_bufs(phz_ctx* c, int op, TuneBufs& b) {
  const int fo = op == 0 ? 4 : op == 1 ? 3 : 1, fi = op == 0 ? 4 : op == 3 ? 1 : 3;
  b.x.alloc((size_t)fi * 9 * c->nn);
  b.y.alloc((size_t)fo * 9 * c->nn);
  PHZ_HIP(hipMemsetAsync(b.x.p, 0, b.x.n * sizeof(float), c->stream));
  b.a = plain_args<float>(nullptr, b.y.p, 1.0f, 0.0f);
}

// Whether block `op` may run as the split-BF16 element contraction: the
// PHZ_BF16X3_IR form, and for the full operator only with bf16_outer.
static bool elem_eligible(phz_ctx* c, int op) {
  return c->opt.precision == PHZ_BF16X3_IR && (op != 0 || c->opt.bf16_outer);
}

// A timed candidate replaces the current choice only when it is more than 3%
// faster, so that near-equal candidates resolve to the earlier one in the
// fixed candidate order instead of to launch-to-launch noise.
static bool clearly_faster(float ms, float best_ms) { return ms < 0.97f * best_ms; }

// Split products of the element contraction of block shape `op`: the full
// block runs only as the GMRES operator, the others only inside the
// preconditioner.
static int elem_terms(const phz_ctx* c, int op) {
  return op == 0 ? c->opt.bf16_terms : c->opt.bf16_terms_precond;
}

// Tile of the element contraction for block `op`: the option's choice, or
// the fastest tile that divides N (timed once per context); -1 if none fits.
static int elem_tile_of(phz_ctx* c, int op) {
  if (c->elem_tile[op] == -1) {
    const int pinned = c->opt.block_tile[op] >= 0 ? c->opt.block_tile[op] : c->opt.elem_tile;
    if (pinned >= 0) {
      c->elem_tile[op] = elem_tile_fits(c->N, pinned) ? pinned : -2;
    } else {
      TuneBufs b;
      tune_bufs(c, op, b);
      int best = -2;
      float best_ms = 0.0f;
      for (int t = 0; t < elem_tile_count(); ++t) {
        if (!elem_tile_fits(c->N, t)) continue;
        const float ms = time_launch(c, [&] {
          elem_apply(op, 9, c->N, elem_terms(c, op), t, c->s32.p, c->kop[op].p, b.x.p, b.a, false, c->stream);
        });
        if (best < 0 || clearly_faster(ms, best_ms)) {
          best = t;
          best_ms = ms;
        }
      }
      c->elem_tile[op] = best;
    }
  }
  return c->elem_tile[op] >= 0 ? c->elem_tile[op] : -1;
}

// Kernel of the float32 nine-column launches of block `op`:
//  * block_kernel[op] >= 0: that kernel where it applies, else the direct
//    gather;
//  * PHZ_BF16X3_IR with a fixed elem_tile: the element contraction;
//  * fine_kernel >= 0: that kernel where it applies, else the direct gather;
//  * otherwise the fastest of the direct gather, the LDS-tiled gather (N a
//    multiple of 16) and, where eligible, the element contraction on its
//    best tile, timed once per context.
static int fine_kind_of(phz_ctx* c, int op) {
  if (c->fkind[op] >= 0) return c->fkind[op];
  const bool elem_ok = elem_eligible(c, op);
  const bool tiled_ok = fine_tiled_fits(c->N);
  int kind = kFineDirect;
  if (c->opt.block_kernel[op] < 0 && elem_ok && c->opt.elem_tile >= 0 && elem_tile_of(c, op) >= 0) {
    kind = kFineElem;
  } else if (c->opt.block_kernel[op] >= 0 || c->opt.fine_kernel >= 0) {
    kind = c->opt.block_kernel[op] >= 0 ? c->opt.block_kernel[op] : c->opt.fine_kernel;
    if ((kind == kFineTiled && !tiled_ok) || (kind == kFineElem && !(elem_ok && elem_tile_of(c, op) >= 0)))
      kind = kFineDirect;
  } else {
    TuneBufs b;
    tune_bufs(c, op, b);
    float best_ms = time_launch(c, [&] {
      fine_apply<float>(op, 9, c->N, c->s32.p, kref_of<float>(c, op), b.x.p, b.a, false, c->stream);
    });
    if (tiled_ok) {
      const float ms = time_launch(c, [&] {
        fine_apply_tiled(op, 9, c->N, c->s32.p, kref_of<float>(c, op), b.x.p, b.a, false, c->stream);
      });
      if (clearly_faster(ms, best_ms)) {
        best_ms = ms;
        kind = kFineTiled;
      }
    }
    if (elem_ok && elem_tile_of(c, op) >= 0) {
      const int t = c->elem_tile[op];
      const float ms = time_launch(c, [&] {
        elem_apply(op, 9, c->N, elem_terms(c, op), t, c->s32.p, c->kop[op].p, b.x.p, b.a, false, c->stream);
      });
      if (clearly_faster(ms, best_ms)) {
        best_ms = ms;
        kind = kFineElem;
      }
    }
  }
  c->fkind[op] = kind;
  c->stats.fine_kernel[op] = kind;
  c->stats.elem_tile[op] = kind == kFineElem ? c->elem_tile[op] : -1;
  return kind;
}

// fine-level operator launch with optional timing
// (blk: reference block 0..4; launches use its shape, whose kernel and tile
// choices it shares)
template <typename T> static const T* sq_of(phz_ctx* c);
template <> const double* sq_of<double>(phz_ctx* c) { return c->sq.p; }
template <> const float* sq_of<float>(phz_ctx* c) { return c->sq32.p; }
template <typename T> static const T* kq_of(phz_ctx* c);
template <> const double* kq_of<double>(phz_ctx* c) { return c->kq64.p; }
template <> const float* kq_of<float>(phz_ctx* c) { return c->kq32.p; }

template <typename T>
static void op_apply_args(phz_ctx* c, int blk, int K, const T* x, const OpArgs<T>& a, bool cheby) {
  const int op = shape_of(blk);
  if (blk == 0 && c->opt.smoothing == PHZ_SMOOTH_QP) {
    // the full operator with the material at the quadrature points (the
    // preconditioner's blocks keep the element means)
    if (cheby) throw std::logic_error("no smoothing step on the full operator");
    const long slot = time_begin(c, sizeof(T) == 4 ? (K == 9 ? "fineqp_full_k9_f32" : "fineqp_full_k1_f32")
                                                   : (K == 9 ? "fineqp_full_k9_f64" : "fineqp_full_k1_f64"));
    fine_apply_qp<T>(K, c->N, sq_of<T>(c), kq_of<T>(c), x, a, c->stream);
    time_end(c, slot);
    return;
  }
  if constexpr (std::is_same<T, float>::value) {
    if (K == 9 && op <= 3) {
      int kind = fine_kind_of(c, op);
      // after a refinement stall the float solve leaves the bf16 products
      if (kind == kFineElem && c->ir_level > 0) kind = fine_tiled_fits(c->N) ? kFineTiled : kFineDirect;
      if (kind == kFineElem) {
        const int terms = elem_terms(c, op);
        const long slot = time_begin(c, elem_op_name(op, terms == 3, cheby));
        elem_apply(op, K, c->N, terms, c->elem_tile[op], c->s32.p, c->kop[blk].p, x, a, cheby, c->stream);
        time_end(c, slot);
        return;
      }
      if (kind == kFineTiled) {
        const long slot = time_begin(c, tiled_op_name(op, cheby));
        fine_apply_tiled(op, K, c->N, c->s32.p, kref_of<float>(c, blk), x, a, cheby, c->stream);
        time_end(c, slot);
        return;
      }
    }
  }
  const long slot = time_begin(c, fine_op_name(op, K, sizeof(T) == 4, cheby));
  fine_apply<T>(op, K, c->N, s_of<T>(c), kref_of<T>(c, blk), x, a, cheby, c->stream);
  time_end(c, slot);
}

// y = beta*yin + alpha*A x on the fine level
template <typename T>
static void op_apply(phz_ctx* c, int op, int K, const T* x, const T* yin, T* y, T alpha, T beta) {
  op_apply_args<T>(c, op, K, x, plain_args<T>(yin, y, alpha, beta), false);
}

template <typename T>
static void level_apply_args(phz_ctx* c, Hierarchy& H, int l, int K, const T* x, const OpArgs<T>& a, bool cheby) {
  Level& L = *H.lv[l];
  if (l == 0) {
    op_apply_args<T>(c, H.op, K, x, a, cheby);
  } else {
    if constexpr (sizeof(T) == 4) {
      if (K == 9 && (L.ckind == 1 || (L.ckind == 2 && c->ir_level > 0))) {
        const long slot = time_begin(c, H.F == 3 ? "coarse_tiled_A_f32" : "coarse_tiled_S_f32");
        coarse_apply_tiled(H.F, L.N, L.S32.p, x, a, cheby, c->stream);
        time_end(c, slot);
        return;
      }
      if (K == 9 && L.ckind == 2) {
        const long slot = time_begin(c, H.F == 3 ? "coarse_tiledbf_A_f32" : "coarse_tiledbf_S_f32");
        coarse_apply_tiled_compact(H.F, L.N, L.S16.p, L.Sc.p, x, a, cheby, c->stream);
        time_end(c, slot);
        return;
      }
    }
    const long slot = time_begin(c, H.F == 3 ? (sizeof(T) == 4 ? "coarse_A_f32" : "coarse_A_f64")
                                             : (sizeof(T) == 4 ? "coarse_S_f32" : "coarse_S_f64"));
    coarse_apply<T>(H.F, K, L.N, stencil_of<T>(L), x, a, cheby, c->stream);
    time_end(c, slot);
  }
}

// y = beta*yin + alpha*A_l x
template <typename T>
static void level_apply(phz_ctx* c, Hierarchy& H, int l, int K, const T* x, const T* yin, T* y, T alpha,
                        T beta) {
  level_apply_args<T>(c, H, l, K, x, plain_args<T>(yin, y, alpha, beta), false);
}

// ------------------------------------------------------- multigrid set-up
static void host_element_matrices(phz_ctx* c, Hierarchy& H, int l, std::vector<double>& Ae) {
  Level& L = *H.lv[l];
  const int F = H.F, S = 8 * F;
  Ae.assign((size_t)8 * L.nn * F * S, 0.0);
  if (l == 0) {
    std::vector<double> sh(L.nn);
    PHZ_HIP(hipMemcpyAsync(sh.data(), c->s.p, L.nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    const double* kref = F == 3 ? c->ref.A0 : H.op == 4 ? c->ref.C0 : c->ref.S0;
    for (int Lc = 0; Lc < 8; ++Lc)
      for (int f = 0; f < F; ++f)
        for (int col = 0; col < S; ++col)
          for (long e = 0; e < L.nn; ++e)
            Ae[((size_t)((Lc * F + f) * S + col)) * L.nn + e] = sh[e] * kref[(Lc * F + f) * S + col];
  } else {
    PHZ_HIP(hipMemcpyAsync(Ae.data(), L.Ae.p, Ae.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
  }
}

static void build_coarsest(phz_ctx* c, Hierarchy& H) {
  const int l = (int)H.lv.size() - 1;
  Level& L = *H.lv[l];
  const int F = H.F, S = 8 * F, N = L.N;
  std::vector<double> Ae;
  host_element_matrices(c, H, l, Ae);
  const int rows = (int)(F * L.nn);
  std::vector<double> M((size_t)rows * rows, 0.0);
  for (long e = 0; e < L.nn; ++e) {
    const int i = (int)(e % N), j = (int)((e / N) % N), k = (int)(e / ((long)N * N));
    long node[8];
    for (int q = 0; q < 8; ++q)
      node[q] = ((i + (q & 1)) % N) + (long)N * (((j + ((q >> 1) & 1)) % N) + (long)N * ((k + ((q >> 2) & 1)) % N));
    for (int Lc = 0; Lc < 8; ++Lc)
      for (int f = 0; f < F; ++f)
        for (int Lp = 0; Lp < 8; ++Lp)
          for (int g = 0; g < F; ++g)
            M[(size_t)(f * L.nn + node[Lc]) * rows + g * L.nn + node[Lp]] +=
                Ae[((size_t)((Lc * F + f) * S + Lp * F + g)) * L.nn + e];
  }
  // the periodic kernel is the constant field of each component; add
  // alpha/nn * 1 1^T per component so the matrix is SPD and zero-mean
  // right-hand sides give zero-mean solutions
  double tr = 0.0;
  for (int r = 0; r < rows; ++r) tr += M[(size_t)r * rows + r];
  const double alpha = tr / rows / (double)L.nn;
  for (long n = 0; n < L.nn; ++n)
    for (long m2 = 0; m2 < L.nn; ++m2)
      for (int f = 0; f < F; ++f) M[(size_t)(f * L.nn + n) * rows + f * L.nn + m2] += alpha;
  if (!spd_inverse(rows, M)) throw std::runtime_error("coarsest multigrid matrix is not positive definite");
  H.rows = rows;
  H.Minv.upload(M.data(), M.size(), c->stream);
  sync(c);
}

static double power_lmax(phz_ctx* c, Hierarchy& H, int l) {
  Level& L = *H.lv[l];
  const long cnt = L.nn * H.F;
  // kept on the level: every set-up asks for the same sizes, so no
  // allocation (and no implicit synchronisation of a free) after the first
  L.pv.alloc(cnt);
  L.pw.alloc(cnt);
  L.py.alloc(cnt);
  double* v = L.pv.p;
  double* w = L.pw.p;
  double* nrm = c->small.p;
  hash_fill(cnt, 12345u + 7u * l + 101u * H.F, v, c->stream);
  col_norm2<double>(L.nn, H.F, 1, v, nrm, c->red_work.p, c->stream);
  normalize_by<double>(cnt, nrm, v, v, c->stream);
  // each step w = D^-1 A v is one pass: the plain apply with its first
  // Chebyshev step at coefficient 1 (y = A v is a by-product).  The direction
  // does not depend on scale, so the iterate is normalised only every fifth
  // step (its norm grows by about lambda_max per step) and before the last,
  // whose ||w|| is the estimate
  const int iters = 20;
  for (int it = 0; it < iters; ++it) {
    OpArgs<double> a = plain_args<double>(nullptr, L.py.p, 1.0, 0.0);
    a.dinv = L.Dinv.p;
    a.cab = c->one64.p;
    a.d1 = w;
    level_apply_args<double>(c, H, l, 1, v, a, false);
    if (it + 1 == iters) break;
    if ((it + 1) % 5 == 0 || it + 2 == iters) {
      col_norm2<double>(L.nn, H.F, 1, w, nrm, c->red_work.p, c->stream);
      normalize_by<double>(cnt, nrm, w, v, c->stream);
    } else {
      std::swap(v, w);
    }
  }
  col_norm2<double>(L.nn, H.F, 1, w, nrm, c->red_work.p, c->stream);
  double h = 0.0;
  PHZ_HIP(hipMemcpyAsync(&h, nrm, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return std::sqrt(h);
}

static void setup_hierarchy(phz_ctx* c, Hierarchy& H) {
  const int F = H.F;
  const double* krefd = F == 3 ? c->kref_A.p : H.op == 4 ? c->kref_C.p : c->kref_S.p;
  const int nl = (int)H.lv.size();
  for (int l = 0; l < nl; ++l) {
    Level& L = *H.lv[l];
    if (l > 0) {
      L.Ae.alloc((size_t)8 * L.nn * F * 8 * F);
      if (l == 1) {
        H.Mq.alloc((size_t)8 * (8 * F) * (8 * F));
        galerkin_build(F, H.lv[0]->N, c->s.p, krefd, nullptr, L.Ae.p, H.Mq.p, c->stream);
      } else {
        galerkin_build(F, H.lv[l - 1]->N, nullptr, nullptr, H.lv[l - 1]->Ae.p, L.Ae.p, nullptr, c->stream);
      }
    }
    if (l > 0) {
      L.S.alloc((size_t)27 * F * F * L.nn);
      build_stencil(F, L.N, L.Ae.p, L.S.p, c->stream);
    }
    if (l < nl - 1) {
      L.Dinv.alloc((size_t)L.nn * F * F);
      if (l == 0) diag_inv_fine(F, L.N, c->s.p, krefd, L.Dinv.p, c->stream);
      else diag_inv_coarse(F, L.N, L.Ae.p, L.Dinv.p, c->stream);
    }
  }
  for (int l = 0; l < nl - 1; ++l) {
    Level& L = *H.lv[l];
    L.lmax = power_lmax(c, H, l);
    // Chebyshev-Jacobi on [0.15, 1.1] lambda_max (Saad, Alg. 12.1)
    const int deg = std::max(1, c->opt.cheby_degree);
    const double hi = 1.1 * L.lmax, lo = 0.15 * L.lmax;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    L.cheb_host.assign(2 * deg, 0.0);
    L.cheb_host[0] = 1.0 / theta;
    double rho = 1.0 / sigma;
    for (int i = 1; i < deg; ++i) {
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      L.cheb_host[2 * i] = rho_new * rho;
      L.cheb_host[2 * i + 1] = 2.0 * rho_new / delta;
      rho = rho_new;
    }
    L.cheb_host32.assign(L.cheb_host.begin(), L.cheb_host.end());
    L.cheb.upload(L.cheb_host.data(), L.cheb_host.size(), c->stream);
    L.cheb32.upload(L.cheb_host32.data(), L.cheb_host32.size(), c->stream);
  }
  build_coarsest(c, H);
  if (c->opt.precision != PHZ_FP64) {
    for (int l = 0; l < nl; ++l) {
      Level& L = *H.lv[l];
      if (L.S.p) {
        L.S32.alloc(L.S.n);
        convert<double, float>((long)L.S.n, L.S.p, L.S32.p, c->stream);
        if (coarse_tiled_fits(L.N)) {
          L.S16.alloc((size_t)26 * H.F * H.F * L.nn);
          L.Sc.alloc((size_t)H.F * H.F * L.nn);
          compact_stencil(H.F, L.nn, L.S.p, L.S16.p, L.Sc.p, c->stream);
        }
      }
      if (L.Dinv.p) {
        L.Dinv32.alloc(L.Dinv.n);
        convert<double, float>((long)L.Dinv.n, L.Dinv.p, L.Dinv32.p, c->stream);
      }
    }
  }
}

template <typename T>
static void drop_level_work_if_changed(phz_ctx* c, Work<T>& W) {
  if (W.A.size() != c->hA.lv.size() || W.S.size() != c->hS.lv.size() || W.C.size() != c->hC.lv.size()) {
    W.A.clear();
    W.S.clear();
    W.C.clear();
    W.cap_k = 0;
  }
}

static int coarse_kind_of(phz_ctx* c, Hierarchy& H, int l);

static void setup_preconditioner(phz_ctx* c) {
  if (c->precond_ready) return;
  // choose (time) the float32 kernels before any solve launches them, so no
  // tuning runs inside a solve or a graph capture
  for (int op = 0; op < 4; ++op) {
    c->stats.elem_tile[op] = -1;
    c->stats.fine_kernel[op] = -1;
    if (c->opt.precision != PHZ_FP64 && c->opt.batched) {
      c->stats.fine_kernel[op] = fine_kind_of(c, op);
      if (c->stats.fine_kernel[op] == kFineElem) c->stats.elem_tile[op] = c->elem_tile[op];
    }
  }
  build_levels(c, c->hA, 3, 1);
  build_levels(c, c->hS, 1, 3);
  // the C hierarchy only exists for the block-diagonal preconditioner and TriCG
  if (c->opt.solver == PHZ_SOLVER_DBP || c->opt.solver == PHZ_SOLVER_TRICG) {
    build_levels(c, c->hC, 1, 4);
  } else if (!c->hC.lv.empty()) {
    c->hC.lv.clear();
    ++c->graph_epoch;
  }
  drop_level_work_if_changed(c, c->w64);
  drop_level_work_if_changed(c, c->w32);
  setup_hierarchy(c, c->hA);
  setup_hierarchy(c, c->hS);
  if (!c->hC.lv.empty()) setup_hierarchy(c, c->hC);
  for (int q = 0; q < 16; ++q) c->stats.coarse_kernel[q] = -1;
  if (c->opt.precision != PHZ_FP64 && c->opt.batched) {
    for (size_t l = 1; l < c->hA.lv.size() && l < 8; ++l) c->stats.coarse_kernel[l] = coarse_kind_of(c, c->hA, (int)l);
    for (size_t l = 1; l < c->hS.lv.size() && l < 8; ++l) c->stats.coarse_kernel[8 + l] = coarse_kind_of(c, c->hS, (int)l);
    for (size_t l = 1; l < c->hC.lv.size(); ++l) coarse_kind_of(c, c->hC, (int)l);
  }
  sync(c);
  c->precond_ready = true;
  c->stats.mg_levels = (int)c->hA.lv.size();
  int q = 0;
  for (auto& L : c->hA.lv)
    if (q < 16) c->stats.cheb_lambda[q++] = L->lmax;
  for (auto& L : c->hS.lv)
    if (q < 16) c->stats.cheb_lambda[q++] = L->lmax;
}

// Kernel of the float32 nine-column applies of coarse level l: the option's
// choice where it applies, else the faster of the direct and the LDS-tiled
// stencil apply (timed once per level; the tiled one must be more than 3%
// faster).
static int coarse_kind_of(phz_ctx* c, Hierarchy& H, int l) {
  Level& L = *H.lv[l];
  if (L.ckind >= 0) return L.ckind;
  int kind = 0;
  if (coarse_tiled_fits(L.N) && c->opt.coarse_kernel != 0) {
    // the bf16 compact stencils are a candidate of the automatic choice only
    // in the split-BF16 form; the float32 form keeps float32 stencils unless
    // coarse_kernel = 2 pins them
    const bool compact_ok = c->opt.precision == PHZ_BF16X3_IR;
    if (c->opt.coarse_kernel >= 1) {
      kind = c->opt.coarse_kernel;
    } else {
      DevBuf<float> x, y;
      x.alloc((size_t)H.F * 9 * L.nn);
      y.alloc((size_t)H.F * 9 * L.nn);
      PHZ_HIP(hipMemsetAsync(x.p, 0, x.n * sizeof(float), c->stream));
      const OpArgs<float> a = plain_args<float>(nullptr, y.p, 1.0f, 0.0f);
      float best = time_launch(c, [&] { coarse_apply<float>(H.F, 9, L.N, L.S32.p, x.p, a, false, c->stream); });
      const float tiled = time_launch(c, [&] { coarse_apply_tiled(H.F, L.N, L.S32.p, x.p, a, false, c->stream); });
      if (clearly_faster(tiled, best)) {
        kind = 1;
        best = tiled;
      }
      if (compact_ok) {
        const float compact = time_launch(c, [&] {
          coarse_apply_tiled_compact(H.F, L.N, L.S16.p, L.Sc.p, x.p, a, false, c->stream);
        });
        if (clearly_faster(compact, best)) kind = 2;
      }
    }
  }
  L.ckind = kind;
  return kind;
}

// ---------------------------------------------------------------- V-cycle
// Chebyshev-Jacobi smoothing of degree d on A_l x = b (Saad, Iterative
// Methods for Sparse Linear Systems, Alg. 12.1, with the block-Jacobi
// preconditioner), interval [0.15, 1.1] * lambda_max(D^-1 A).  The residual
// is carried along: on return r points at b - A (x - d) and dcur at the last
// correction, so that b - A x = r - A dcur.
template <typename T> static const T* cheb_of(Level& L);
template <> const double* cheb_of<double>(Level& L) { return L.cheb.p; }
template <> const float* cheb_of<float>(Level& L) { return L.cheb32.p; }

template <typename T>
static void cheby_smooth(phz_ctx* c, Hierarchy& H, int l, int K, const T* b, T* x, bool xzero, LevelWork<T>& W,
                         const T*& r, T*& dcur) {
  Level& L = *H.lv[l];
  const int deg = std::max(1, c->opt.cheby_degree);
  const T* coef = cheb_of<T>(L);
  r = b;
  // with more steps to come the first correction is folded into x by the
  // next fused step (x = x_in + d_1 + d_2), which saves a pass over x
  const int xmode = deg > 1 ? kChebyXNone : (xzero ? kChebyXSet : kChebyXAdd);
  if (!xzero) {
    OpArgs<T> a = plain_args<T>(b, W.r.p, T(-1), T(1));
    if (xmode == kChebyXNone) {
      // the residual's pass also writes the first correction d_1
      a.dinv = dinv_of<T>(L);
      a.cab = coef;
      a.d1 = W.d.p;
    }
    level_apply_args<T>(c, H, l, K, x, a, false);
    r = W.r.p;
  }
  if (xzero || xmode != kChebyXNone) cheby_first<T>(H.F, K, L.nn, dinv_of<T>(L), r, W.d.p, x, coef, xmode, c->stream);
  dcur = W.d.p;
  T* dnext = W.d2.p;
  for (int i = 1; i < deg; ++i) {
    OpArgs<T> a;
    a.yin = r;
    a.y = W.r.p;
    a.alpha = T(-1);
    a.beta = T(1);
    a.dinv = dinv_of<T>(L);
    a.dold = dcur;
    a.dnew = dnext;
    a.x = x;
    a.xin = (i == 1 && xzero) ? nullptr : x;
    a.fold_dold = i == 1 ? 1 : 0;
    a.cab = coef + 2 * i;
    level_apply_args<T>(c, H, l, K, dcur, a, true);
    r = W.r.p;
    std::swap(dcur, dnext);
  }
}

// One V-cycle for A_l x = b: from a zero initial guess (xzero), else from
// the x passed in, which it updates in place (the same as adding the
// zero-guess cycle of the residual b - A x, without a separate residual,
// correction vector and update pass).  Below level l the cycles start from
// zero; the coarsest level is solved directly and needs xzero.
template <typename T>
static void vcycle(phz_ctx* c, Hierarchy& H, std::vector<std::unique_ptr<LevelWork<T>>>& WL, int l, int K,
                   const T* b, T* x, bool xzero = true) {
  const int nl = (int)H.lv.size();
  if (l == nl - 1) {
    if (!xzero) throw std::logic_error("vcycle: the coarsest level needs a zero initial guess");
    dense_apply<T>(H.F, (int)H.lv[l]->nn, K, H.Minv.p, b, x, c->stream);
    return;
  }
  LevelWork<T>& W = *WL[l];
  LevelWork<T>& Wc = *WL[l + 1];
  const T* r = nullptr;
  T* dcur = nullptr;
  cheby_smooth<T>(c, H, l, K, b, x, xzero, W, r, dcur);
  level_apply<T>(c, H, l, K, dcur, r, W.r.p, T(-1), T(1));   // b - A x
  restrict_fw<T>(H.F, K, H.lv[l + 1]->N, W.r.p, Wc.b.p, c->stream);
  vcycle<T>(c, H, WL, l + 1, K, Wc.b.p, Wc.x.p);
  prolong_add<T>(H.F, K, H.lv[l + 1]->N, Wc.x.p, x, c->stream);
  cheby_smooth<T>(c, H, l, K, b, x, false, W, r, dcur);
}

// x = (ncycles V-cycles) A^-1 b
template <typename T>
static void block_solve(phz_ctx* c, Hierarchy& H, std::vector<std::unique_ptr<LevelWork<T>>>& WL, int K,
                        int ncycles, const T* b, T* x, T* tmp_r, T* tmp_e) {
  vcycle<T>(c, H, WL, 0, K, b, x);
  for (int it = 1; it < ncycles; ++it) {
    if (H.lv.size() > 1) {
      vcycle<T>(c, H, WL, 0, K, b, x, false);
    } else {
      // a single (directly solved) level: correction from the residual
      level_apply<T>(c, H, 0, K, x, b, tmp_r, T(-1), T(1));
      vcycle<T>(c, H, WL, 0, K, tmp_r, tmp_e);
      axpy_cols<T, T>(H.lv[0]->nn, H.F, K, nullptr, tmp_e, x, c->stream);
    }
  }
}

// z = P^-1 r on [nn][4][K]
// (structure of arrays: the displacement block of a 4-field vector is its
// first 3K columns, the potential block the last K)
// Inexact block map x ~= M^-1 b for the fine-level operator M of hierarchy
// H (A, S_bar or C): conjugate gradients preconditioned by one V-cycle, from
// x = 0, until ||b - M x|| <= inner_eps ||b|| in every load column or
// inner_maxit iterations.  M is singular on the periodic cell (constants per
// field), so b and every preconditioned residual are projected onto zero
// field means, which keeps the iteration in M's range.  Returns the number
// of iterations.
template <typename T>
static int pcg_block(phz_ctx* c, Hierarchy& H, std::vector<std::unique_ptr<LevelWork<T>>>& WL, int K, const T* b,
                     T* x) {
  Work<T>& W = work_of<T>(c);
  const long nn = c->nn;
  const int F = H.F;
  const size_t cnt = (size_t)nn * F * K;
  hipStream_t st = c->stream;
  if (c->pcg_dev.n < (size_t)(3 * K + F * K)) throw std::logic_error("pcg_block: scalar workspace too small");
  for (DevBuf<T>* v : {&W.pr, &W.pz, &W.pp, &W.pq})
    if (v->n < (size_t)nn * 3 * K) v->alloc((size_t)nn * 3 * K);
  T *r = W.pr.p, *z = W.pz.p, *p = W.pp.p, *q = W.pq.p;
  double* dv = c->pcg_dev.p;     // [0, K) alpha, [K, 2K) -alpha, [2K, 3K) beta, [3K, 3K + F K) reductions
  double* red = dv + 3 * K;
  std::vector<double> bn(K), rz(K), h(K), al(2 * K), be(K);
  std::vector<int> act(K);
  auto to_host = [&](std::vector<double>& out) {
    PHZ_HIP(hipMemcpyAsync(out.data(), red, K * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(c);
  };
  auto project = [&](T* v) {
    field_sums<T>(nn, F, K, v, red, c->red_work.p, st);
    subtract_mean<T>(nn, F, K, red, v, st);
  };
  PHZ_HIP(hipMemcpyAsync(r, b, cnt * sizeof(T), hipMemcpyDeviceToDevice, st));
  project(r);
  fill<T>((long)cnt, T(0), x, st);
  col_norm2<T>(nn, F, K, r, red, c->red_work.p, st);
  to_host(bn);
  int nact = 0;
  for (int k = 0; k < K; ++k) {
    bn[k] = std::sqrt(bn[k]);
    act[k] = bn[k] > 0.0;
    nact += act[k];
  }
  if (nact == 0) return 0;
  vcycle<T>(c, H, WL, 0, K, r, z);
  project(z);
  PHZ_HIP(hipMemcpyAsync(p, z, cnt * sizeof(T), hipMemcpyDeviceToDevice, st));
  col_dot<T>(nn, F, K, r, z, red, c->red_work.p, st);
  to_host(rz);
  int it = 0;
  const double eps = c->opt.inner_eps;
  while (it < c->opt.inner_maxit) {
    level_apply<T>(c, H, 0, K, p, (const T*)nullptr, q, T(1), T(0));
    col_dot<T>(nn, F, K, p, q, red, c->red_work.p, st);
    to_host(h);
    for (int k = 0; k < K; ++k) {
      const double a = act[k] && h[k] > 0.0 ? rz[k] / h[k] : 0.0;
      al[k] = a;
      al[K + k] = -a;
    }
    PHZ_HIP(hipMemcpyAsync(dv, al.data(), 2 * K * sizeof(double), hipMemcpyHostToDevice, st));
    axpy_cols<T, T>(nn, F, K, dv, p, x, st);
    axpy_cols<T, T>(nn, F, K, dv + K, q, r, st);
    ++it;
    col_norm2<T>(nn, F, K, r, red, c->red_work.p, st);
    to_host(h);
    nact = 0;
    for (int k = 0; k < K; ++k) {
      if (act[k] && (std::sqrt(h[k]) <= eps * bn[k] || !(h[k] >= 0.0))) act[k] = 0;
      nact += act[k];
    }
    if (nact == 0) break;
    vcycle<T>(c, H, WL, 0, K, r, z);
    project(z);
    col_dot<T>(nn, F, K, r, z, red, c->red_work.p, st);
    to_host(h);
    for (int k = 0; k < K; ++k) {
      be[k] = act[k] && rz[k] != 0.0 ? h[k] / rz[k] : 0.0;
      rz[k] = h[k];
    }
    PHZ_HIP(hipMemcpyAsync(dv + 2 * K, be.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
    xpby_cols<T>(nn, F, K, dv + 2 * K, z, p, st);
  }
  return it;
}

// z = P^-1 r on [nn][4][K]
// (structure of arrays: the displacement block of a 4-field vector is its
// first 3K columns, the potential block the last K).  SCP (the approximate
// Schur complement, lower block-triangular): z_u = A^-1 r_u, then
// z_p = S_bar^-1 (B z_u - r_p).  DBP (block diagonal diag(A, -C)):
// z_u = A^-1 r_u, z_p = -C^-1 r_p.  The block maps are fixed V-cycle counts
// (vcycles_a, vcycles_s) or, with inner = 1, conjugate gradients to
// inner_eps.
template <typename T>
static void precond_apply(phz_ctx* c, int K, const T* r, T* z) {
  Work<T>& W = work_of<T>(c);
  const size_t off = (size_t)c->nn * 3 * K;
  const T* ru = r;
  const T* rp = r + off;
  T* zu = z;
  T* zp = z + off;
  const bool pcg = c->opt.inner == 1;
  if (pcg) {
    c->stats.inner_iters[0] += pcg_block<T>(c, c->hA, W.A, K, ru, zu);
    c->stats.inner_calls[0] += 1;
  } else {
    block_solve<T>(c, c->hA, W.A, K, std::max(1, c->opt.vcycles_a), ru, zu, W.t1u.p, W.t2u.p);
  }
  const bool dbp = c->opt.solver == PHZ_SOLVER_DBP;
  Hierarchy& Hp = dbp ? c->hC : c->hS;
  auto& WLp = dbp ? W.C : W.S;
  if (dbp) {
    // t = -r_p
    scale_cols<T>((long)c->nn, 1, K, rp, c->negone.p, W.t1p.p, c->stream);
  } else {
    // t = B z_u - r_p
    op_apply<T>(c, 2, K, zu, rp, W.t1p.p, T(1), T(-1));
  }
  if (pcg) {
    c->stats.inner_iters[1] += pcg_block<T>(c, Hp, WLp, K, W.t1p.p, zp);
    c->stats.inner_calls[1] += 1;
  } else {
    block_solve<T>(c, Hp, WLp, K, std::max(1, c->opt.vcycles_s), W.t1p.p, zp, W.t2p.p, W.t3p.p);
  }
}

// ------------------------------------------------------------------ GMRES
struct GmresResult {
  int iters[9] = {0};
  int restarts[9] = {0};
  double true_rel[9] = {0};
  bool converged = false;
};

template <typename T> static std::vector<StepGraph>& graphs_of(phz_ctx* c);
template <> std::vector<StepGraph>& graphs_of<double>(phz_ctx* c) { return c->graphs64; }
template <> std::vector<StepGraph>& graphs_of<float>(phz_ctx* c) { return c->graphs32; }

static void drop_graphs(std::vector<StepGraph>& G) {
  for (auto& g : G)
    if (g.exec) hipGraphExecDestroy(g.exec);
  G.clear();
}

// Run Arnoldi step j from its captured graph, capturing `body` (the step's
// launches, no host synchronisation or allocation) on first use.
template <typename T, typename Body>
static void run_step_graph(phz_ctx* c, int K, int j, double rtol, double stall, const double* tol, Body&& body) {
  std::vector<StepGraph>& G = graphs_of<T>(c);
  if ((int)G.size() <= j) G.resize(j + 1);
  StepGraph& g = G[j];
  if (!g.exec || g.K != K || g.rtol != rtol || g.stall != stall || g.tol != tol || g.epoch != c->graph_epoch) {
    if (g.exec) hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    hipGraph_t graph = nullptr;
    PHZ_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    try {
      body();
    } catch (...) {
      hipStreamEndCapture(c->stream, &graph);
      if (graph) hipGraphDestroy(graph);
      throw;
    }
    PHZ_HIP(hipStreamEndCapture(c->stream, &graph));
    const hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    PHZ_HIP(e);
    g.K = K;
    g.rtol = rtol;
    g.stall = stall;
    g.tol = tol;
    g.epoch = c->graph_epoch;
  }
  PHZ_HIP(hipGraphLaunch(g.exec, c->stream));
}

// Solve calA x = b (x holds the initial guess), K columns, storage T.
// true residuals are evaluated in T (the caller refines in float64 if T is float).
// x_is_zero: skip the first residual apply (r = b).  one_cycle: run one
// restart cycle only and leave the true residual to the caller (float64
// iterative refinement evaluates it in float64).
template <typename T>
static GmresResult gmres(phz_ctx* c, int K, const T* b, T* x, double rtol, int maxit, int hist_base,
                         bool record_hist, bool x_is_zero = false, bool one_cycle = false,
                         const double* coltol = nullptr) {
  Work<T>& W = work_of<T>(c);
  const long nn = c->nn;
  const long vs = (long)basis_stride(nn, K);
  const int m = c->opt.restart;
  // the float cycles keep P^-1 V_j (flexible GMRES): the correction is then
  // Z y with no further preconditioner application, and the preconditioner's
  // input-dependent rounding does not enter the Arnoldi relation
  // (and so does every cycle whose block maps are conjugate-gradient solves,
  // a preconditioner that changes from one application to the next)
  const bool flexible = std::is_same<T, float>::value || c->opt.inner == 1;
  // selective reorthogonalisation threshold: 32 units of roundoff of the
  // basis's type by default
  const bool selective = c->opt.reorth_tol >= 0.0;
  const double tau = c->opt.reorth_tol > 0.0 ? c->opt.reorth_tol
                                             : 32.0 * (std::is_same<T, float>::value ? 0x1p-24 : 0x1p-53);
  if (flexible && W.Z.n < (size_t)vs * m) W.Z.alloc((size_t)vs * m);
  GmresState S = gm_state(c);
  S.tol = coltol;
  hipStream_t st = c->stream;
  GmresResult res;
  double* nrm = c->gm_nrm.p;
  // ||b||
  col_norm2<T>(nn, 4, K, b, nrm, c->red_work.p, st);
  {
    std::vector<double> h(K);
    PHZ_HIP(hipMemcpyAsync(h.data(), nrm, K * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(c);
    for (int k = 0; k < K; ++k) h[k] = std::sqrt(h[k]);
    PHZ_HIP(hipMemcpyAsync(S.bnorm, h.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
    sync(c);
  }
  int total = 0;
  std::vector<double> estbuf((size_t)m * K), rn(K), bn(K);
  std::vector<int> kused(K), act(K);
  PHZ_HIP(hipMemcpyAsync(bn.data(), S.bnorm, K * sizeof(double), hipMemcpyDeviceToHost, st));
  sync(c);
  for (int cycle = 0;; ++cycle) {
    // r = b - calA x
    if (cycle == 0 && x_is_zero)
      PHZ_HIP(hipMemcpyAsync(W.r.p, b, (size_t)nn * 4 * K * sizeof(T), hipMemcpyDeviceToDevice, st));
    else
      op_apply<T>(c, 0, K, x, b, W.r.p, T(-1), T(1));
    col_norm2<T>(nn, 4, K, W.r.p, nrm, c->red_work.p, st);
    gmres_start(K, nrm, rtol, S, st);
    PHZ_HIP(hipMemcpyAsync(rn.data(), nrm, K * sizeof(double), hipMemcpyDeviceToHost, st));
    int nact = 0;
    PHZ_HIP(hipMemcpyAsync(&nact, S.nactive, sizeof(int), hipMemcpyDeviceToHost, st));
    sync(c);
    for (int k = 0; k < K; ++k) {
      res.true_rel[k] = bn[k] > 0 ? std::sqrt(rn[k]) / bn[k] : 0.0;
      if (record_hist) c->hist[hist_base + k].push_back(res.true_rel[k]);
    }
    if (nact == 0) {
      res.converged = true;
      for (int k = 0; k < K; ++k)
        if (!(res.true_rel[k] <= rtol) && bn[k] > 0) res.converged = false;
      break;
    }
    if (total >= maxit) break;
    for (int k = 0; k < K; ++k)
      if (bn[k] > 0 && !(res.true_rel[k] <= rtol)) res.restarts[k] += 1;
    // V_0 = r / beta
    scale_cols<T>(nn, 4, K, W.r.p, S.scale, W.V.p, st);
    int j = 0;
    // a float refinement cycle ends when its estimate stalls (the float
    // operator's own error floors it); the float64 refinement carries on
    const double stall = one_cycle ? 0.9 : 0.0;
    for (; j < m; ++j) {
      auto step = [&] {
        T* Vj = W.V.p + (size_t)j * vs;
        T* Zj = flexible ? W.Z.p + (size_t)j * vs : W.z.p;
        const long tp = time_begin(c, sizeof(T) == 4 ? "precond_f32" : "precond_f64");
        precond_apply<T>(c, K, Vj, Zj);
        time_end(c, tp);
        op_apply<T>(c, 0, K, Zj, (const T*)nullptr, W.w.p, T(1), T(0));
        // classical Gram-Schmidt: the first pass fused with the inner
        // products of the second; the second pass for the loads whose first
        // left components above reorth_tol (every load with reorth_tol < 0)
        const long ts = time_begin(c, sizeof(T) == 4 ? "arnoldi_cgs2_f32" : "arnoldi_cgs2_f64");
        arnoldi_dots<T>(nn, 4, K, j, W.V.p, vs, W.w.p, c->gm_h1.p, c->red_work.p, st);
        arnoldi_update<T>(nn, 4, K, j, W.V.p, vs, W.w.p, c->gm_h1.p, c->gm_h2.p, c->gm_na2.p, c->red_work.p, st);
        // (tau2 < 0: every active load takes the second pass)
        reorth_decide(K, j + 1, selective ? tau * tau : -1.0, c->gm_h2.p, c->gm_na2.p, S.active, c->gm_flag.p,
                      c->gm_reorth.p, st);
        arnoldi_update<T>(nn, 4, K, j, W.V.p, vs, W.w.p, c->gm_h2.p, nullptr, nrm, c->red_work.p, st, c->gm_flag.p);
        time_end(c, ts);
        gmres_givens(K, m, j, c->gm_h1.p, c->gm_h2.p, nrm, rtol, stall, S, st, c->gm_flag.p, c->gm_na2.p);
        scale_cols<T>(nn, 4, K, W.w.p, S.scale, W.V.p + (size_t)(j + 1) * vs, st);
      };
      // per-kernel timing needs eager launches
      // (inexact block maps synchronise with the host: never captured)
      if (c->opt.use_graph && !c->ktime && c->opt.inner == 0) run_step_graph<T>(c, K, j, rtol, stall, coltol, step);
      else step();
      ++total;
      PHZ_HIP(hipMemcpyAsync(&nact, S.nactive, sizeof(int), hipMemcpyDeviceToHost, st));
      sync(c);
      if (nact == 0 || total >= maxit) {
        ++j;
        break;
      }
    }
    // x += P^-1 (V y), or Z y when the cycle kept Z = P^-1 V
    gmres_solve_y(K, m, S, st);
    if (flexible) {
      combine<T>(nn, 4, K, W.Z.p, vs, S.y, S.kused, W.t.p, st);
      axpy_cols<T, T>(nn, 4, K, nullptr, W.t.p, x, st);
    } else {
      combine<T>(nn, 4, K, W.V.p, vs, S.y, S.kused, W.t.p, st);
      precond_apply<T>(c, K, W.t.p, W.z.p);
      axpy_cols<T, T>(nn, 4, K, nullptr, W.z.p, x, st);
    }
    PHZ_HIP(hipMemcpyAsync(kused.data(), S.kused, K * sizeof(int), hipMemcpyDeviceToHost, st));
    PHZ_HIP(hipMemcpyAsync(estbuf.data(), S.est, (size_t)m * K * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(c);
    for (int k = 0; k < K; ++k) {
      res.iters[k] += kused[k];
      if (record_hist)
        for (int i = 0; i < kused[k]; ++i) c->hist[hist_base + k].push_back(estbuf[(size_t)i * K + k]);
    }
    if (one_cycle) {
      res.converged = false;
      for (int k = 0; k < K; ++k) {
        res.true_rel[k] = kused[k] > 0 ? estbuf[(size_t)(kused[k] - 1) * K + k] : res.true_rel[k];
        if (kused[k] > 0) res.restarts[k] = 1;
      }
      break;
    }
  }
  return res;
}

// ------------------------------------------------------------ solve paths
static void solve_fp64(phz_ctx* c, int K, const double* b, double* x, double rtol, int hist_base, GmresResult& out) {
  alloc_work<double>(c, c->w64, K, c->opt.restart);
  out = gmres<double>(c, K, b, x, rtol, c->opt.max_iters, hist_base, true);
}

// float64 iterative refinement around the float GMRES
static int solve_ir(phz_ctx* c, int K, const double* b, double* x, double rtol, int hist_base, GmresResult& out) {
  alloc_work<float>(c, c->w32, K, c->opt.restart);
  Work<float>& W = c->w32;
  const long nn = c->nn;
  const long count = nn * 4 * K;
  hipStream_t st = c->stream;
  double* nrm = c->gm_nrm.p + 9;
  std::vector<double> bn(K), rn(K), scale(K), inv(K), tol(K);
  col_norm2<double>(nn, 4, K, b, nrm, c->red_work.p, st);
  PHZ_HIP(hipMemcpyAsync(bn.data(), nrm, K * sizeof(double), hipMemcpyDeviceToHost, st));
  sync(c);
  for (int k = 0; k < K; ++k) bn[k] = std::sqrt(bn[k]);
  DevBuf<double>& r64 = c->R64;
  double* scp = c->gm_nrm.p + 18;
  int steps = 0;
  int used = 0;
  // refinement-stall fallback: a refinement step that leaves a load above
  // its target without reducing its float64 residual tenfold (when its
  // cycle aimed at more than that) moves the float solve one form down:
  // split-BF16 -> float32 kernels -> a float64 inner GMRES on the residual
  // (ir_fallback = 2 treats every step as stalled, to exercise the path)
  c->ir_level = 0;
  std::vector<double> prev_rel(K, -1.0), prev_tol(K, 1.0);
  for (;;) {
    // r = b - calA x in float64
    op_apply<double>(c, 0, K, x, b, r64.p, -1.0, 1.0);
    col_norm2<double>(nn, 4, K, r64.p, nrm, c->red_work.p, st);
    PHZ_HIP(hipMemcpyAsync(rn.data(), nrm, K * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(c);
    bool done = true;
    for (int k = 0; k < K; ++k) {
      rn[k] = std::sqrt(rn[k]);
      out.true_rel[k] = bn[k] > 0 ? rn[k] / bn[k] : 0.0;
      c->hist[hist_base + k].push_back(out.true_rel[k]);
      if (bn[k] > 0 && !(out.true_rel[k] <= rtol)) done = false;
      if (!std::isfinite(rn[k])) throw std::runtime_error("non-finite residual in refinement");
    }
    if (done) {
      out.converged = true;
      break;
    }
    if (steps >= c->opt.max_refine || used >= c->opt.max_iters) break;
    if (steps > 0 && c->opt.ir_fallback > 0) {
      bool stalled = c->opt.ir_fallback == 2;
      for (int k = 0; k < K; ++k)
        if (bn[k] > 0 && !(out.true_rel[k] <= rtol) && prev_tol[k] <= 0.1 && out.true_rel[k] > 0.1 * prev_rel[k])
          stalled = true;
      if (stalled && c->ir_level < 2) {
        c->ir_level = c->opt.precision == PHZ_BF16X3_IR ? c->ir_level + 1 : 2;
        ++c->graph_epoch;   // captured steps hold the kernels of the form they were captured in
        c->stats.fallbacks += 1;
        if (c->opt.verbose)
          std::fprintf(stderr, "[piezohom] refinement step %d stalled: float solve falls back to %s\n", steps,
                       c->ir_level == 1 ? "float32 kernels" : "a float64 inner GMRES");
      }
    }
    if (c->ir_level == 2) {
      // float64 GMRES from the current iterate to the target
      alloc_work<double>(c, c->w64, K, c->opt.restart);
      GmresResult g = gmres<double>(c, K, b, x, rtol, std::max(c->opt.max_iters - used, 1), hist_base, true);
      for (int k = 0; k < K; ++k) {
        out.iters[k] += g.iters[k];
        out.restarts[k] += g.restarts[k];
        out.true_rel[k] = g.true_rel[k];
      }
      out.converged = g.converged;
      ++steps;
      break;
    }
    for (int k = 0; k < K; ++k) prev_rel[k] = out.true_rel[k];
    // solve calA d = r / ||r|| in float, x += ||r|| d.  A load's cycle aims
    // at inner_rtol, or, when less than that remains to its target, at what
    // remains (with a margin of 4 for the float estimate): the last cycle
    // stops as soon as the float64 target is in reach
    for (int k = 0; k < K; ++k) {
      const bool act = bn[k] > 0 && !(out.true_rel[k] <= rtol);
      scale[k] = act ? rn[k] : 0.0;
      inv[k] = act ? 1.0 / rn[k] : 0.0;
      tol[k] = act ? std::max(c->opt.inner_rtol, 0.25 * rtol / out.true_rel[k]) : c->opt.inner_rtol;
      prev_tol[k] = tol[k];
    }
    PHZ_HIP(hipMemcpyAsync(c->gm_tol.p, tol.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
    PHZ_HIP(hipMemcpyAsync(scp, inv.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
    scale_cols<double>(nn, 4, K, r64.p, scp, r64.p, st);
    convert<double, float>(count, r64.p, W.b.p, st);
    fill<float>(count, 0.0f, W.x.p, st);
    GmresResult g = gmres<float>(c, K, W.b.p, W.x.p, c->opt.inner_rtol, c->opt.max_iters - used, hist_base, true,
                                 true, true, c->gm_tol.p);
    PHZ_HIP(hipMemcpyAsync(scp, scale.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
    axpy_cols<double, float>(nn, 4, K, scp, W.x.p, x, st);
    sync(c);
    int mx = 0;
    for (int k = 0; k < K; ++k) {
      out.iters[k] += g.iters[k];
      out.restarts[k] += g.restarts[k];
      mx = std::max(mx, g.iters[k]);
    }
    used += std::max(mx, 1);
    ++steps;
  }
  // the form that finished: the most precise one any column block needed
  // (codes: PHZ_FP64 < PHZ_FP32_IR < PHZ_BF16X3_IR)
  const int form = c->ir_level == 0 ? c->opt.precision : c->ir_level == 1 ? PHZ_FP32_IR : PHZ_FP64;
  c->stats.final_precision = std::min(c->stats.final_precision, form);
  c->ir_level = 0;
  return steps;
}

// TriCG (Sec. 2.5.2) on calA x = b in float64 for K loads in lockstep.  With
// E = A, F = C and the coupling B^T, calA = [[E, B^T], [B, -F]] is
// quasi-definite.  Per iteration: the tridiagonalisation step
//   q = B^T v_k - gamma_k E u_{k-1},  p = B u_k - beta_k F v_{k-1},
//   alpha_k = u_k . q,  q -= alpha_k E u_k,  p -= alpha_k F v_k,
//   beta_{k+1} = sqrt(q . E^-1 q),  gamma_{k+1} = sqrt(p . F^-1 p),
// (E^-1, F^-1 by conjugate gradients to inner_eps), then the block LDL^T
// step of the Galerkin system [[I, T], [T^T, -I]] on the host (2 x 2 per
// load), and one fused update of the two direction columns and the iterate
// per block.  The residual norm after step k is
// sqrt((z_1 ||q||)^2 + (z_0 ||p||)^2) with z the step's last solution block.
// Cycles start from the true residual; see the header for the zero-block
// start and the breakdown rule.
static void solve_tricg(phz_ctx* c, int K, const double* b, double* x, double rtol, int hist_base,
                        GmresResult& out) {
  alloc_work<double>(c, c->w64, K, 1);
  Work<double>& W = c->w64;
  const long nn = c->nn;
  hipStream_t st = c->stream;
  const size_t nu = (size_t)nn * 3 * K, np = (size_t)nn * K;
  for (DevBuf<double>* v : {&c->tri_u, &c->tri_Eu, &c->tri_Eup, &c->tri_q, &c->tri_Eq, &c->tri_g1x, &c->tri_g2x})
    if (v->n < nu) v->alloc(nu);
  for (DevBuf<double>* v : {&c->tri_v, &c->tri_Fv, &c->tri_Fvp, &c->tri_p, &c->tri_Fp, &c->tri_g1y, &c->tri_g2y})
    if (v->n < np) v->alloc(np);
  if (c->tri_dev.n < (size_t)(20 * K)) c->tri_dev.alloc(20 * 9);
  double* cf = c->tri_dev.p;              // [0, 6K) update coefficients
  double* sc = c->tri_dev.p + 6 * K;      // [6K, 8K) two per-load scale vectors
  double* red = c->tri_dev.p + 8 * K;     // [8K, 12K) four reductions
  // raw pointers so the rotations below are pointer swaps
  double *u = c->tri_u.p, *Eu = c->tri_Eu.p, *Eup = c->tri_Eup.p, *q = c->tri_q.p, *Eq = c->tri_Eq.p;
  double *v = c->tri_v.p, *Fv = c->tri_Fv.p, *Fvp = c->tri_Fvp.p, *p = c->tri_p.p, *Fp = c->tri_Fp.p;
  double *g1x = c->tri_g1x.p, *g2x = c->tri_g2x.p, *g1y = c->tri_g1y.p, *g2y = c->tri_g2y.p;
  double* r = c->R64.p;
  const double* bu = b;
  const double* bp = b + nu;
  double* xu = x;
  double* xp = x + nu;
  std::vector<double> h4(4 * K), s1(K), s2(K), cfh(6 * K);
  auto fetch = [&](int slots) {
    PHZ_HIP(hipMemcpyAsync(h4.data(), red, (size_t)slots * K * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(c);
  };
  auto put = [&](double* dst, const std::vector<double>& src) {
    PHZ_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice, st));
  };
  auto emap = [&](const double* rhs, double* sol) {
    c->stats.inner_iters[0] += pcg_block<double>(c, c->hA, W.A, K, rhs, sol);
    c->stats.inner_calls[0] += 1;
  };
  auto fmap = [&](const double* rhs, double* sol) {
    c->stats.inner_iters[1] += pcg_block<double>(c, c->hC, W.C, K, rhs, sol);
    c->stats.inner_calls[1] += 1;
  };
  col_norm2<double>(nn, 4, K, b, red, c->red_work.p, st);
  fetch(1);
  std::vector<double> bn(K), ru(K), rp(K);
  for (int k = 0; k < K; ++k) bn[k] = std::sqrt(h4[k]);
  std::vector<int> done(K, 0);
  // r = b - calA x, per-load block norms; marks converged loads
  auto residual = [&]() {
    op_apply<double>(c, 0, K, x, b, r, -1.0, 1.0);
    col_norm2<double>(nn, 3, K, r, red, c->red_work.p, st);
    col_norm2<double>(nn, 1, K, r + nu, red + K, c->red_work.p, st);
    fetch(2);
    bool all = true;
    for (int k = 0; k < K; ++k) {
      ru[k] = std::sqrt(h4[k]);
      rp[k] = std::sqrt(h4[K + k]);
      out.true_rel[k] = bn[k] > 0 ? std::hypot(ru[k], rp[k]) / bn[k] : 0.0;
      if (!std::isfinite(out.true_rel[k])) throw std::runtime_error("non-finite residual in TriCG");
      done[k] = bn[k] == 0.0 || out.true_rel[k] <= rtol;
      all = all && done[k];
    }
    return all;
  };
  const int max_cycles = 100;
  int used = 0;
  out.converged = residual();
  for (int cyc = 0; cyc < max_cycles && !out.converged && used < c->opt.max_iters; ++cyc) {
    for (int k = 0; k < K; ++k) out.restarts[k] += !done[k];
    // loads whose residual has a (relatively) zero block take the shifted start
    std::vector<double> zc(K, 0.0), zb(K, 0.0);
    bool any_zc = false, any_zb = false;
    const double tiny = std::min(1e-13, 0.1 * rtol);
    for (int k = 0; k < K; ++k) {
      if (done[k]) continue;
      if (rp[k] <= 1e-12 * ru[k] || rp[k] <= tiny * bn[k]) zc[k] = 1.0, any_zc = true;
      else if (ru[k] <= 1e-12 * rp[k] || ru[k] <= tiny * bn[k]) zb[k] = 1.0, any_zb = true;
    }
    if (any_zc) {
      // xh = E^-1 r_u, w = B xh, y0 = F^-1 w; y += y0, or x += xh where w = 0
      put(sc, zc);
      scale_cols<double>(nn, 3, K, r, sc, q, st);
      emap(q, Eq);
      op_apply<double>(c, 2, K, Eq, (const double*)nullptr, p, 1.0, 0.0);
      col_norm2<double>(nn, 1, K, p, red, c->red_work.p, st);
      fetch(1);
      for (int k = 0; k < K; ++k) {
        s1[k] = zc[k] != 0.0 && h4[k] == 0.0 ? 1.0 : 0.0;
        s2[k] = zc[k] != 0.0 && h4[k] != 0.0 ? 1.0 : 0.0;
      }
      fmap(p, Fp);
      put(sc, s1);
      put(sc + K, s2);
      axpy_cols<double, double>(nn, 3, K, sc, Eq, xu, st);
      axpy_cols<double, double>(nn, 1, K, sc + K, Fp, xp, st);
      sync(c);
    }
    if (any_zb) {
      // yh = F^-1 r_p, t = B^T yh, x0 = -E^-1 t; x += x0, or y -= yh where t = 0
      put(sc, zb);
      scale_cols<double>(nn, 1, K, r + nu, sc, p, st);
      fmap(p, Fp);
      op_apply<double>(c, 5, K, Fp, (const double*)nullptr, q, 1.0, 0.0);
      col_norm2<double>(nn, 3, K, q, red, c->red_work.p, st);
      fetch(1);
      for (int k = 0; k < K; ++k) {
        s1[k] = zb[k] != 0.0 && h4[k] != 0.0 ? -1.0 : 0.0;
        s2[k] = zb[k] != 0.0 && h4[k] == 0.0 ? -1.0 : 0.0;
      }
      emap(q, Eq);
      put(sc, s1);
      put(sc + K, s2);
      axpy_cols<double, double>(nn, 3, K, sc, Eq, xu, st);
      axpy_cols<double, double>(nn, 1, K, sc + K, Fp, xp, st);
      sync(c);
    }
    if (any_zc || any_zb) {
      out.converged = residual();
      continue;
    }
    // a TriCG cycle from zero on the masked residual (converged loads idle)
    for (int k = 0; k < K; ++k) s1[k] = done[k] ? 0.0 : 1.0;
    put(sc, s1);
    scale_cols<double>(nn, 3, K, r, sc, Eu, st);
    scale_cols<double>(nn, 1, K, r + nu, sc, Fv, st);
    emap(Eu, u);
    fmap(Fv, v);
    col_dot<double>(nn, 3, K, Eu, u, red, c->red_work.p, st);
    col_dot<double>(nn, 1, K, Fv, v, red + K, c->red_work.p, st);
    fetch(2);
    std::vector<double> beta(K), gamma(K), bmax(K), gmax(K), d(2 * K), D(4 * K), alpha(K);
    std::vector<int> act(K, 0), first(K, 1);
    int nact = 0;
    for (int k = 0; k < K; ++k) {
      beta[k] = std::sqrt(std::max(h4[k], 0.0));
      gamma[k] = std::sqrt(std::max(h4[K + k], 0.0));
      act[k] = !done[k] && beta[k] > 0.0 && gamma[k] > 0.0;
      nact += act[k];
      bmax[k] = beta[k];
      gmax[k] = gamma[k];
      d[2 * k] = beta[k];
      d[2 * k + 1] = gamma[k];
      s1[k] = act[k] ? 1.0 / beta[k] : 0.0;
      s2[k] = act[k] ? 1.0 / gamma[k] : 0.0;
    }
    if (nact == 0) break;
    put(sc, s1);
    put(sc + K, s2);
    scale_cols<double>(nn, 3, K, Eu, sc, Eu, st);
    scale_cols<double>(nn, 3, K, u, sc, u, st);
    scale_cols<double>(nn, 1, K, Fv, sc + K, Fv, st);
    scale_cols<double>(nn, 1, K, v, sc + K, v, st);
    fill<double>((long)nu, 0.0, Eup, st);
    fill<double>((long)np, 0.0, Fvp, st);
    fill<double>((long)nu, 0.0, g1x, st);
    fill<double>((long)nu, 0.0, g2x, st);
    fill<double>((long)np, 0.0, g1y, st);
    fill<double>((long)np, 0.0, g2y, st);
    sync(c);  // the host staging vectors are rewritten below
    while (nact > 0 && used < c->opt.max_iters) {
      // q = B^T v - gamma E u_prev, p = B u - beta F v_prev
      for (int k = 0; k < K; ++k) {
        s1[k] = act[k] ? -gamma[k] : 0.0;
        s2[k] = act[k] ? -beta[k] : 0.0;
      }
      put(sc, s1);
      put(sc + K, s2);
      op_apply<double>(c, 5, K, v, (const double*)nullptr, q, 1.0, 0.0);
      axpy_cols<double, double>(nn, 3, K, sc, Eup, q, st);
      op_apply<double>(c, 2, K, u, (const double*)nullptr, p, 1.0, 0.0);
      axpy_cols<double, double>(nn, 1, K, sc + K, Fvp, p, st);
      col_dot<double>(nn, 3, K, u, q, red, c->red_work.p, st);
      fetch(1);
      for (int k = 0; k < K; ++k) {
        alpha[k] = act[k] ? h4[k] : 0.0;
        s1[k] = -alpha[k];
      }
      put(sc, s1);
      axpy_cols<double, double>(nn, 3, K, sc, Eu, q, st);
      axpy_cols<double, double>(nn, 1, K, sc, Fv, p, st);
      emap(q, Eq);
      fmap(p, Fp);
      col_dot<double>(nn, 3, K, q, Eq, red, c->red_work.p, st);
      col_dot<double>(nn, 1, K, p, Fp, red + K, c->red_work.p, st);
      col_norm2<double>(nn, 3, K, q, red + 2 * K, c->red_work.p, st);
      col_norm2<double>(nn, 1, K, p, red + 3 * K, c->red_work.p, st);
      fetch(4);
      ++used;
      // block LDL^T step and the update coefficients, per load
      std::vector<int> cont(K, 0);
      for (int k = 0; k < K; ++k) {
        double* ck = &cfh[6 * k];
        for (int i = 0; i < 6; ++i) ck[i] = 0.0;
        s1[k] = s2[k] = 0.0;
        if (!act[k]) continue;
        const double a = alpha[k];
        double L[4] = {0.0, 0.0, 0.0, 0.0};
        double Dn[4] = {1.0, a, a, -1.0};
        double* dk = &d[2 * k];
        if (!first[k]) {
          // L = Gamma D^-1, D_new = Delta - L Gamma^T, d = -L d;  Gamma = [[0, beta], [gamma, 0]]
          const double* Dk = &D[4 * k];
          const double det = Dk[0] * Dk[3] - Dk[1] * Dk[2];
          const double Di[4] = {Dk[3] / det, -Dk[1] / det, -Dk[2] / det, Dk[0] / det};
          const double G[4] = {0.0, beta[k], gamma[k], 0.0};
          L[0] = G[0] * Di[0] + G[1] * Di[2];
          L[1] = G[0] * Di[1] + G[1] * Di[3];
          L[2] = G[2] * Di[0] + G[3] * Di[2];
          L[3] = G[2] * Di[1] + G[3] * Di[3];
          // (L Gamma^T)_ij = sum_l L_il G_jl
          Dn[0] -= L[0] * G[0] + L[1] * G[1];
          Dn[1] -= L[0] * G[2] + L[1] * G[3];
          Dn[2] -= L[2] * G[0] + L[3] * G[1];
          Dn[3] -= L[2] * G[2] + L[3] * G[3];
          const double d0 = -(L[0] * dk[0] + L[1] * dk[1]);
          const double d1 = -(L[2] * dk[0] + L[3] * dk[1]);
          dk[0] = d0;
          dk[1] = d1;
        }
        first[k] = 0;
        for (int i = 0; i < 4; ++i) D[4 * k + i] = Dn[i];
        const double det = Dn[0] * Dn[3] - Dn[1] * Dn[2];
        const double z0 = (Dn[3] * dk[0] - Dn[1] * dk[1]) / det;
        const double z1 = (-Dn[2] * dk[0] + Dn[0] * dk[1]) / det;
        ck[0] = L[0];
        ck[1] = L[1];
        ck[2] = L[2];
        ck[3] = L[3];
        ck[4] = z0;
        ck[5] = z1;
        out.iters[k] += 1;
        const double est = std::hypot(z1 * std::sqrt(std::max(h4[2 * K + k], 0.0)),
                                      z0 * std::sqrt(std::max(h4[3 * K + k], 0.0)));
        c->hist[hist_base + k].push_back(bn[k] > 0 ? est / bn[k] : 0.0);
        const double bnext = std::sqrt(std::max(h4[k], 0.0)), gnext = std::sqrt(std::max(h4[K + k], 0.0));
        if (!(std::isfinite(est) && std::isfinite(z0) && std::isfinite(z1)))
          throw std::runtime_error("TriCG: non-finite recurrence");
        if (est <= rtol * bn[k]) continue;
        bmax[k] = std::max(bmax[k], bnext);
        gmax[k] = std::max(gmax[k], gnext);
        if (!(bnext > 1e-10 * bmax[k] && gnext > 1e-10 * gmax[k])) continue;  // breakdown: the cycle ends
        cont[k] = 1;
        beta[k] = bnext;
        gamma[k] = gnext;
        s1[k] = 1.0 / bnext;
        s2[k] = 1.0 / gnext;
      }
      put(cf, cfh);
      tricg_update(nn, 3, K, cf, u, 0, g1x, g2x, xu, st);
      tricg_update(nn, 1, K, cf, v, 1, g1y, g2y, xp, st);
      // next basis vectors: E u_prev <- E u, E u <- q / beta, u <- E^-1 q / beta (and the same for v)
      put(sc, s1);
      put(sc + K, s2);
      std::swap(Eu, Eup);
      scale_cols<double>(nn, 3, K, q, sc, Eu, st);
      scale_cols<double>(nn, 3, K, Eq, sc, Eq, st);
      std::swap(u, Eq);
      std::swap(Fv, Fvp);
      scale_cols<double>(nn, 1, K, p, sc + K, Fv, st);
      scale_cols<double>(nn, 1, K, Fp, sc + K, Fp, st);
      std::swap(v, Fp);
      sync(c);  // the host staging vectors are rewritten next iteration
      nact = 0;
      for (int k = 0; k < K; ++k) {
        act[k] = cont[k];
        nact += act[k];
      }
    }
    out.converged = residual();
  }
  // hand the rotated buffers back to their owners
  c->tri_u.p = u; c->tri_Eu.p = Eu; c->tri_Eup.p = Eup; c->tri_q.p = q; c->tri_Eq.p = Eq;
  c->tri_v.p = v; c->tri_Fv.p = Fv; c->tri_Fvp.p = Fvp; c->tri_p.p = p; c->tri_Fp.p = Fp;
  sync(c);
}

static void compute_effective(phz_ctx* c) {
  hipStream_t st = c->stream;
  const long nn = c->nn;
  // zero-mean fields (gauge); tensors do not depend on it
  double* sums = c->small.p;
  field_sums<double>(nn, 4, 9, c->X.p, sums, c->red_work.p, st);
  subtract_mean<double>(nn, 4, 9, sums, c->X.p, st);
  double* out = c->small.p + 64;
  reduce_effective(c->N, c->s.p, c->X.p, out, c->red_work.p, st);
  std::vector<double> red(289);
  PHZ_HIP(hipMemcpyAsync(red.data(), out, 289 * sizeof(double), hipMemcpyDeviceToHost, st));
  sync(c);
  const double h3 = std::pow(1.0 / c->N, 3);
  const double ssum = red[288];
  const RefElement& R = c->ref;
  double FY[81];
  for (int K = 0; K < 9; ++K)
    for (int L = 0; L < 9; ++L) {
      double v = 0.0;
      for (int l = 0; l < 8; ++l)
        for (int f = 0; f < 4; ++f) v += R.F0[(4 * l + f) * 9 + K] * red[l * 36 + f * 9 + L];
      FY[K * 9 + L] = v;
    }
  if (c->opt.smoothing == PHZ_SMOOTH_QP) {
    // F0^T sum_e s_e X_e becomes sum_p F0q[p]^T sum_e s_ep X_e (the <s> M term
    // is unchanged: the element scale is the mean of the point scales)
    for (int i = 0; i < 81; ++i) FY[i] = 0.0;
    std::vector<double> rp(288);
    for (int p = 0; p < 8; ++p) {
      reduce_effective_point(c->N, c->sq.p, p, c->X.p, out, c->red_work.p, st);
      PHZ_HIP(hipMemcpyAsync(rp.data(), out, 288 * sizeof(double), hipMemcpyDeviceToHost, st));
      sync(c);
      for (int K = 0; K < 9; ++K)
        for (int L = 0; L < 9; ++L) {
          double v = 0.0;
          for (int l = 0; l < 8; ++l)
            for (int f = 0; f < 4; ++f) v += R.F0q[p][(4 * l + f) * 9 + K] * rp[l * 36 + f * 9 + L];
          FY[K * 9 + L] += v;
        }
    }
  }
  for (int K = 0; K < 9; ++K)
    for (int L = 0; L < 9; ++L) c->MH[K * 9 + L] = h3 * ssum * R.M[K * 9 + L] + FY[K * 9 + L];
  // energy form: <s>M + FY + FY^T + X^T calA X
  op_apply<double>(c, 0, 9, c->X.p, (const double*)nullptr, c->R64.p, 1.0, 0.0);
  std::vector<double> XtAX(81, 0.0);
  {
    std::vector<double> h(81);
    cross_dots(nn, c->X.p, c->R64.p, c->small.p + 400, c->red_work.p, st);
    PHZ_HIP(hipMemcpyAsync(h.data(), c->small.p + 400, 81 * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(c);
    for (int a = 0; a < 9; ++a)
      for (int b = 0; b < 9; ++b) XtAX[a * 9 + b] = h[b * 9 + a];
  }
  double mx = 0.0, df = 0.0;
  for (int K = 0; K < 9; ++K)
    for (int L = 0; L < 9; ++L) {
      c->MHe[K * 9 + L] = h3 * ssum * R.M[K * 9 + L] + FY[K * 9 + L] + FY[L * 9 + K] + XtAX[K * 9 + L];
      mx = std::max(mx, std::fabs(c->MH[K * 9 + L]));
      df = std::max(df, std::fabs(c->MH[K * 9 + L] - c->MHe[K * 9 + L]));
    }
  c->stats.flux_energy_defect = mx > 0 ? df / mx : 0.0;
}

// b = -sum_e s_e F0 e_L, projected to zero mean per field (the exact load is
// compatible; rounding is not), and columns that vanish in exact arithmetic
// (below 1e-12 of the magnitude of the terms they sum) set to exactly zero,
// so such loads return X = 0 without iterating on rounding noise.
static void prepare_rhs(phz_ctx* c) {
  hipStream_t st = c->stream;
  const long nn = c->nn;
  const bool qp = c->opt.smoothing == PHZ_SMOOTH_QP;
  if (qp) build_rhs_qp(c->N, c->sq.p, c->f0q.p, c->R64.p, st, true);
  else build_rhs(c->N, c->s.p, c->F0d.p, c->R64.p, st, true);
  double* nb = c->small.p;
  double* nref = c->small.p + 16;
  col_norm2<double>(nn, 4, 9, c->R64.p, nref, c->red_work.p, st);
  if (qp) build_rhs_qp(c->N, c->sq.p, c->f0q.p, c->Bvec.p, st, false);
  else build_rhs(c->N, c->s.p, c->F0d.p, c->Bvec.p, st, false);
  field_sums<double>(nn, 4, 9, c->Bvec.p, c->small.p + 32, c->red_work.p, st);
  subtract_mean<double>(nn, 4, 9, c->small.p + 32, c->Bvec.p, st);
  col_norm2<double>(nn, 4, 9, c->Bvec.p, nb, c->red_work.p, st);
  double h[32];
  PHZ_HIP(hipMemcpyAsync(h, c->small.p, 32 * sizeof(double), hipMemcpyDeviceToHost, st));
  sync(c);
  double keep[9];
  for (int L = 0; L < 9; ++L) keep[L] = std::sqrt(h[L]) <= 1e-12 * std::sqrt(h[16 + L]) ? 0.0 : 1.0;
  PHZ_HIP(hipMemcpyAsync(c->small.p + 80, keep, 9 * sizeof(double), hipMemcpyHostToDevice, st));
  scale_cols<double>(nn, 4, 9, c->Bvec.p, c->small.p + 80, c->Bvec.p, st);
  sync(c);
}

static int do_solve(phz_ctx* c) {
  if (!c->have_s) {
    c->err = "no geometry: call phz_set_levelset or phz_set_density first";
    return PHZ_E_STATE;
  }
  const auto t0 = Clock::now();
  hipStream_t st = c->stream;
  const long nn = c->nn;
  std::memset(c->stats.iterations, 0, sizeof(c->stats.iterations));
  std::memset(c->stats.restarts, 0, sizeof(c->stats.restarts));
  c->stats.refinements = 0;
  c->stats.fallbacks = 0;
  c->stats.final_precision = c->opt.precision;
  c->stats.reorth_passes = 0;
  for (int i = 0; i < 2; ++i) c->stats.inner_iters[i] = c->stats.inner_calls[i] = 0;
  for (auto& h : c->hist) h.clear();
  ensure_state_buffers(c);
  PHZ_HIP(hipMemsetAsync(c->gm_reorth.p, 0, c->gm_reorth.n * sizeof(int), st));
  c->X.alloc(nn * 36);
  c->Bvec.alloc(nn * 36);
  c->R64.alloc(nn * 36);
  const auto ts = Clock::now();
  setup_preconditioner(c);
  c->stats.setup_ms = ms_since(ts);
  prepare_rhs(c);
  const bool warm = !c->have_guess && c->opt.warm_start && c->x_valid;
  c->x_valid = false;
  if (c->have_guess)
    PHZ_HIP(hipMemcpyAsync(c->X.p, c->guess.p, nn * 36 * sizeof(double), hipMemcpyDeviceToDevice, st));
  else if (!warm)
    fill<double>(nn * 36, 0.0, c->X.p, st);
  const double rtol = c->opt.rtol;
  bool conv = true;
  const bool tri = c->opt.solver == PHZ_SOLVER_TRICG;
  if (c->opt.batched) {
    GmresResult g;
    if (tri) solve_tricg(c, 9, c->Bvec.p, c->X.p, rtol, 0, g);
    else if (c->opt.precision != PHZ_FP64) c->stats.refinements = solve_ir(c, 9, c->Bvec.p, c->X.p, rtol, 0, g);
    else solve_fp64(c, 9, c->Bvec.p, c->X.p, rtol, 0, g);
    for (int k = 0; k < 9; ++k) {
      c->stats.iterations[k] = g.iters[k];
      c->stats.restarts[k] = g.restarts[k];
      c->stats.true_residual[k] = g.true_rel[k];
    }
    conv = g.converged;
  } else {
    c->col_b.alloc(nn * 4);
    c->col_x.alloc(nn * 4);
    for (int L = 0; L < 9; ++L) {
      extract_column(nn, L, c->Bvec.p, c->col_b.p, st);
      extract_column(nn, L, c->X.p, c->col_x.p, st);
      GmresResult g;
      if (tri) solve_tricg(c, 1, c->col_b.p, c->col_x.p, rtol, L, g);
      else if (c->opt.precision != PHZ_FP64) c->stats.refinements += solve_ir(c, 1, c->col_b.p, c->col_x.p, rtol, L, g);
      else solve_fp64(c, 1, c->col_b.p, c->col_x.p, rtol, L, g);
      insert_column(nn, L, c->col_x.p, c->X.p, st);
      c->stats.iterations[L] = g.iters[0];
      c->stats.restarts[L] = g.restarts[0];
      c->stats.true_residual[L] = g.true_rel[0];
      conv = conv && g.converged;
    }
  }
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(c->stats.true_residual[k])) {
      c->err = "non-finite residual";
      return PHZ_E_NAN;
    }
  compute_effective(c);
  {
    int cnt[9] = {0};
    PHZ_HIP(hipMemcpyAsync(cnt, c->gm_reorth.p, 9 * sizeof(int), hipMemcpyDeviceToHost, st));
    sync(c);
    for (int k = 0; k < 9; ++k) c->stats.reorth_passes += cnt[k];
  }
  collect_timing(c);
  c->have_solution = true;
  c->x_valid = true;
  c->have_grad = false;
  c->stats.solve_ms = ms_since(t0);
  if (c->opt.verbose) {
    int mx = 0;
    for (int k = 0; k < 9; ++k) mx = std::max(mx, c->stats.iterations[k]);
    std::fprintf(stderr, "[piezohom] N=%d %s %s: max iters %d, refinements %d, setup %.2f ms, solve %.2f ms\n",
                 c->N, c->opt.precision == PHZ_BF16X3_IR ? "bf16x3-ir" : c->opt.precision == PHZ_FP32_IR ? "fp32-ir" : "fp64", c->opt.batched ? "batched" : "sequential",
                 mx, c->stats.refinements, c->stats.setup_ms, c->stats.solve_ms);
  }
  if (!conv) {
    c->err = "GMRES did not reach rtol within max_iters";
    return PHZ_NOT_CONVERGED;
  }
  return PHZ_OK;
}

// ------------------------------------------------------------------ FOMs
static bool inv_general(int n, const double* A, double* out) {
  std::vector<long double> M((size_t)n * 2 * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j) M[(size_t)i * 2 * n + j] = j < n ? A[i * n + j] : (j - n == i ? 1.0L : 0.0L);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabsl(M[(size_t)r * 2 * n + col]) > fabsl(M[(size_t)piv * 2 * n + col])) piv = r;
    if (M[(size_t)piv * 2 * n + col] == 0.0L) return false;
    if (piv != col)
      for (int j = 0; j < 2 * n; ++j) std::swap(M[(size_t)piv * 2 * n + j], M[(size_t)col * 2 * n + j]);
    const long double d = M[(size_t)col * 2 * n + col];
    for (int j = 0; j < 2 * n; ++j) M[(size_t)col * 2 * n + j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const long double f = M[(size_t)r * 2 * n + col];
      if (f == 0.0L) continue;
      for (int j = 0; j < 2 * n; ++j) M[(size_t)r * 2 * n + j] -= f * M[(size_t)col * 2 * n + j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[i * n + j] = (double)M[(size_t)i * 2 * n + n + j];
  return true;
}

// Element scales from the level set, and with quadrature-point smoothing the
// point scales (the element scales are then their means, used by the
// preconditioner)
static void update_scales(phz_ctx* c) {
  const double eta = c->opt.smooth_width / c->N;
  if (c->opt.smoothing == PHZ_SMOOTH_QP) {
    if (c->sq.n < (size_t)c->nn * 8) c->sq.alloc((size_t)c->nn * 8);
    if (c->sq32.n < (size_t)c->nn * 8) c->sq32.alloc((size_t)c->nn * 8);
    levelset_to_scale_qp(c->N, c->phi.p, eta, c->mat.void_scale, c->rho.p, c->s.p, c->s32.p, c->sq.p, c->sq32.p,
                         c->stream);
  } else {
    levelset_to_scale(c->N, c->phi.p, eta, c->mat.void_scale, c->rho.p, c->s.p, c->s32.p, c->stream);
  }
}

// point scales equal to the element scales (a cell given by densities)
static void fill_point_scales(phz_ctx* c) {
  if (c->opt.smoothing != PHZ_SMOOTH_QP) return;
  if (c->sq.n < (size_t)c->nn * 8) c->sq.alloc((size_t)c->nn * 8);
  if (c->sq32.n < (size_t)c->nn * 8) c->sq32.alloc((size_t)c->nn * 8);
  point_scales(c->nn, c->s.p, c->sq.p, c->sq32.p, c->stream);
}

}  // namespace phz

namespace phz {

// Device scratch of phz_hj_step_noalloc, one copy per GPU for the life of
// the process: the nodal velocity (up to kNoAllocMaxNodes values) and the
// partial maxima of its normalisation.  Host code never passes `scratch`
// itself (on the host it names a stand-in, not device memory): each device's
// address comes from hipGetSymbolAddress, taken once per device with that
// device current.
constexpr long kNoAllocMaxNodes = 128L * 128L * 128L;
constexpr long kNoAllocPartials = 1024;
__device__ __align__(256) double scratch[kNoAllocMaxNodes + kNoAllocPartials];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[64] = {};

// Address of the current device's scratch, or nullptr (err set).
static double* scratch_of_current_device(std::string& err) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    err = "no current HIP device (or device index above 63)";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

// error text of the last failing call that has no context
static thread_local std::string g_free_err;

}  // namespace phz

using namespace phz;

static const AllocHook* hook_of(phz_ctx* c) { return c ? &c->hook : nullptr; }

#define PHZ_GUARD_BEGIN \
  try {                 \
    AllocScope alloc_scope_(hook_of(c));
#define PHZ_GUARD_END(ctx)                                           \
  }                                                                  \
  catch (const HipError& ex) {                                       \
    if (ctx) (ctx)->err = ex.what();                                 \
    return std::strstr(ex.what(), "hipMalloc") ? PHZ_E_OOM : PHZ_E_HIP; \
  }                                                                  \
  catch (const std::invalid_argument& ex) {                          \
    if (ctx) (ctx)->err = ex.what();                                 \
    return PHZ_E_INVALID;                                            \
  }                                                                  \
  catch (const std::exception& ex) {                                 \
    if (ctx) (ctx)->err = ex.what();                                 \
    return PHZ_E_INTERNAL;                                           \
  }                                                                  \
  catch (...) {                                                      \
    if (ctx) (ctx)->err = "unknown exception";                       \
    return PHZ_E_INTERNAL;                                           \
  }

extern "C" {

void phz_default_options(phz_options* o) {
  if (!o) return;
  o->precision = PHZ_FP64;
  o->batched = 1;
  o->restart = 30;
  o->max_iters = 2000;
  o->rtol = 1e-10;
  o->cheby_degree = 2;
  o->mg_levels = 0;
  o->smooth_width = 2.0;
  o->vcycles_a = 1;
  o->vcycles_s = 1;
  o->inner_rtol = 1e-5;
  o->max_refine = 50;
  o->verbose = 0;
  o->bf16_terms = 3;
  o->bf16_outer = 1;
  o->elem_tile = -1;
  o->use_graph = 0;
  o->fine_kernel = -1;
  for (int op = 0; op < 4; ++op) o->block_kernel[op] = o->block_tile[op] = -1;
  o->coarse_kernel = -1;
  o->solver = PHZ_SOLVER_SCP;
  o->inner = 0;
  o->inner_eps = 1e-2;
  o->inner_maxit = 200;
  o->warm_start = 0;
  o->smoothing = PHZ_SMOOTH_ELEMENT;
  o->bf16_terms_precond = 1;
  o->ir_fallback = 1;
  o->reorth_tol = 0.0;
}

const char* phz_strerror(int status) {
  if (status == PHZ_OK) return kStatusNames[0];
  if (status == PHZ_NOT_CONVERGED) return kStatusNames[1];
  if (status <= -1 && status >= -6) return kStatusNames[1 - status];
  return "unknown status";
}

const char* phz_last_error(const phz_ctx* ctx) { return ctx ? ctx->err.c_str() : g_free_err.c_str(); }

static int check_options(const phz_options* o, std::string& err) {
  if (o->precision != PHZ_FP64 && o->precision != PHZ_FP32_IR && o->precision != PHZ_BF16X3_IR) { err = "precision must be PHZ_FP64, PHZ_FP32_IR or PHZ_BF16X3_IR"; return PHZ_E_INVALID; }
  if (o->bf16_terms != 1 && o->bf16_terms != 3) { err = "bf16_terms must be 1 or 3"; return PHZ_E_INVALID; }
  if (o->bf16_terms_precond != 1 && o->bf16_terms_precond != 3) { err = "bf16_terms_precond must be 1 or 3"; return PHZ_E_INVALID; }
  if (o->bf16_outer != 0 && o->bf16_outer != 1) { err = "bf16_outer must be 0 or 1"; return PHZ_E_INVALID; }
  if (o->elem_tile < -1 || o->elem_tile >= elem_tile_count()) { err = "elem_tile must be -1 or a tile index"; return PHZ_E_INVALID; }
  if (o->use_graph != 0 && o->use_graph != 1) { err = "use_graph must be 0 or 1"; return PHZ_E_INVALID; }
  if (o->fine_kernel < -1 || o->fine_kernel > 2) { err = "fine_kernel must be -1, 0, 1 or 2"; return PHZ_E_INVALID; }
  if (o->coarse_kernel < -1 || o->coarse_kernel > 2) { err = "coarse_kernel must be -1, 0, 1 or 2"; return PHZ_E_INVALID; }
  if (o->solver != PHZ_SOLVER_SCP && o->solver != PHZ_SOLVER_DBP && o->solver != PHZ_SOLVER_TRICG) { err = "solver must be PHZ_SOLVER_SCP, PHZ_SOLVER_DBP or PHZ_SOLVER_TRICG"; return PHZ_E_INVALID; }
  if (o->solver == PHZ_SOLVER_TRICG && o->precision != PHZ_FP64) { err = "TriCG runs in float64 (precision PHZ_FP64)"; return PHZ_E_INVALID; }
  if (o->inner != 0 && o->inner != 1) { err = "inner must be 0 or 1"; return PHZ_E_INVALID; }
  if (!(o->inner_eps > 0 && o->inner_eps < 1)) { err = "inner_eps must be in (0, 1)"; return PHZ_E_INVALID; }
  if (o->inner_maxit < 1) { err = "inner_maxit must be positive"; return PHZ_E_INVALID; }
  if (o->warm_start != 0 && o->warm_start != 1) { err = "warm_start must be 0 or 1"; return PHZ_E_INVALID; }
  if (o->smoothing != PHZ_SMOOTH_ELEMENT && o->smoothing != PHZ_SMOOTH_QP) { err = "smoothing must be PHZ_SMOOTH_ELEMENT or PHZ_SMOOTH_QP"; return PHZ_E_INVALID; }
  if (o->smoothing == PHZ_SMOOTH_QP && o->solver == PHZ_SOLVER_TRICG) { err = "TriCG applies the element-smoothed blocks; use SCP or DBP with smoothing = PHZ_SMOOTH_QP"; return PHZ_E_INVALID; }
  for (int op = 0; op < 4; ++op) {
    if (o->block_kernel[op] < -1 || o->block_kernel[op] > 2) { err = "block_kernel entries must be -1, 0, 1 or 2"; return PHZ_E_INVALID; }
    if (o->block_tile[op] < -1 || o->block_tile[op] >= elem_tile_count()) {
      err = "block_tile entries must be -1 or a tile index";
      return PHZ_E_INVALID;
    }
  }
  if (o->restart < 1 || o->restart > kMaxRestart) { err = "restart must be in [1, 32]"; return PHZ_E_INVALID; }
  if (o->max_iters < 1) { err = "max_iters must be >= 1"; return PHZ_E_INVALID; }
  if (!(o->rtol > 0 && o->rtol < 1)) { err = "rtol must be in (0, 1)"; return PHZ_E_INVALID; }
  if (o->cheby_degree < 1 || o->cheby_degree > 16) { err = "cheby_degree must be in [1, 16]"; return PHZ_E_INVALID; }
  if (o->mg_levels < 0) { err = "mg_levels must be >= 0"; return PHZ_E_INVALID; }
  if (!(o->smooth_width > 0)) { err = "smooth_width must be > 0"; return PHZ_E_INVALID; }
  if (o->vcycles_a < 1 || o->vcycles_s < 1) { err = "vcycles must be >= 1"; return PHZ_E_INVALID; }
  if (!(o->inner_rtol > 0 && o->inner_rtol < 1)) { err = "inner_rtol must be in (0, 1)"; return PHZ_E_INVALID; }
  if (o->max_refine < 1) { err = "max_refine must be >= 1"; return PHZ_E_INVALID; }
  if (o->ir_fallback < 0 || o->ir_fallback > 2) { err = "ir_fallback must be 0, 1 or 2"; return PHZ_E_INVALID; }
  if (!(o->reorth_tol < 1.0)) { err = "reorth_tol must be below 1"; return PHZ_E_INVALID; }
  return PHZ_OK;
}

int phz_create(int nx, int ny, int nz, const phz_material* mat, const phz_options* opt, void* stream,
               const phz_allocator* alloc, phz_ctx** out) {
  if (!out) return PHZ_E_INVALID;
  *out = nullptr;
  if (nx != ny || ny != nz) return PHZ_E_INVALID;
  const int n = nx;
  if (!mat || n < 2 || n % 2 != 0 || n > 1024) return PHZ_E_INVALID;
  if (alloc && (!alloc->alloc || !alloc->free)) return PHZ_E_INVALID;
  for (int i = 0; i < 36; ++i) if (!std::isfinite(mat->C[i])) return PHZ_E_NAN;
  for (int i = 0; i < 18; ++i) if (!std::isfinite(mat->e[i])) return PHZ_E_NAN;
  for (int i = 0; i < 9; ++i) if (!std::isfinite(mat->kappa[i])) return PHZ_E_NAN;
  if (!(mat->void_scale > 0.0 && mat->void_scale <= 1.0)) return PHZ_E_INVALID;
  phz_options o;
  if (opt) o = *opt;
  else phz_default_options(&o);
  {
    std::string err;
    const int rc = check_options(&o, err);
    if (rc) return rc;
  }
  if (coarsest_side(n, o.mg_levels) > kMaxCoarsestN) return PHZ_E_INVALID;
  // a context that fails part-way is torn down like any other (its buffers
  // go back through the caller's allocator, its own stream is destroyed)
  struct Pending {
    phz_ctx* c;
    ~Pending() { if (c) phz_destroy(c); }
  } pending{new (std::nothrow) phz_ctx()};
  phz_ctx* c = pending.c;
  if (!c) return PHZ_E_OOM;
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      c->stream = nullptr;
      return PHZ_E_HIP;
    }
    c->own_stream = true;
  }
  if (alloc) {
    c->hook.a = *alloc;
    c->hook.stream = c->stream;
    c->hook.active = true;
  }
  PHZ_GUARD_BEGIN
  c->N = n;
  c->nn = (long)n * n * n;
  c->mat = *mat;
  c->opt = o;
  for (int op = 0; op < 4; ++op) c->stats.elem_tile[op] = c->stats.fine_kernel[op] = -1;
  for (int q = 0; q < 16; ++q) c->stats.coarse_kernel[q] = -1;
  upload_reference(c);
  static const double kOne = 1.0;
  c->one64.upload(&kOne, 1, c->stream);
  const double neg[9] = {-1.0, -1.0, -1.0, -1.0, -1.0, -1.0, -1.0, -1.0, -1.0};
  c->negone.upload(neg, 9, c->stream);
  c->pcg_dev.alloc(3 * 9 + 4 * 9);   // alpha, -alpha, beta; then up to 4 x 9 reductions
  c->phi.alloc(c->nn);
  c->rho.alloc(c->nn);
  c->s.alloc(c->nn);
  c->s32.alloc(c->nn);
  ensure_state_buffers(c);
  sync(c);
  *out = c;
  pending.c = nullptr;
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

void phz_destroy(phz_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) hipStreamSynchronize(ctx->stream);
  for (hipEvent_t e : ctx->ev) hipEventDestroy(e);
  phz::drop_graphs(ctx->graphs64);
  phz::drop_graphs(ctx->graphs32);
  hipStream_t st = ctx->stream;
  bool own = ctx->own_stream;
  delete ctx;
  if (own && st) hipStreamDestroy(st);
}

int phz_set_options(phz_ctx* c, const phz_options* opt) {
  if (!c || !opt) return PHZ_E_INVALID;
  int rc = check_options(opt, c->err);
  if (rc) return rc;
  if (coarsest_side(c->N, opt->mg_levels) > kMaxCoarsestN) {
    c->err = "mg_levels leaves a coarsest level above 10^3 nodes";
    return PHZ_E_INVALID;
  }
  PHZ_GUARD_BEGIN
  const bool hier_change = opt->mg_levels != c->opt.mg_levels || opt->precision != c->opt.precision;
  if (opt->restart != c->opt.restart) {
    c->w64.cap_m = 0;
    c->w32.cap_m = 0;
  }
  for (int op = 0; op < 4; ++op) {
    c->elem_tile[op] = -1;
    c->fkind[op] = -1;
  }
  if (opt->solver != c->opt.solver) c->precond_ready = false;   // the C hierarchy comes or goes
  if (opt->coarse_kernel != c->opt.coarse_kernel) {
    // the per-level choice is made again with the hierarchy
    for (auto& L : c->hA.lv) L->ckind = -1;
    for (auto& L : c->hS.lv) L->ckind = -1;
    c->precond_ready = false;
  }
  const bool smooth_change = opt->smoothing != c->opt.smoothing || opt->smooth_width != c->opt.smooth_width;
  c->opt = *opt;
  ++c->graph_epoch;
  if (hier_change) c->precond_ready = false;
  if (smooth_change && c->have_s) {
    // the current geometry's scales under the new smoothing
    if (c->have_phi) update_scales(c);
    else fill_point_scales(c);
    sync(c);
    c->precond_ready = false;
    c->have_solution = false;
    c->have_grad = false;
  }
  ensure_state_buffers(c);
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

static int set_input(phz_ctx* c, const double* src, int on_device, DevBuf<double>& dst) {
  if (on_device) PHZ_HIP(hipMemcpyAsync(dst.p, src, c->nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  else PHZ_HIP(hipMemcpyAsync(dst.p, src, c->nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (count_nonfinite(c->nn, dst.p, c->red_work.p, c->stream) > 0) {
    c->err = "input holds NaN or Inf";
    return PHZ_E_NAN;
  }
  return PHZ_OK;
}

int phz_set_levelset(phz_ctx* c, const double* phi, int on_device) {
  if (!c || !phi) return PHZ_E_INVALID;
  PHZ_GUARD_BEGIN
  int rc = set_input(c, phi, on_device, c->phi);
  if (rc) return rc;
  update_scales(c);
  sync(c);
  c->have_phi = true;
  c->have_s = true;
  c->precond_ready = false;
  c->have_solution = false;
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_set_density(phz_ctx* c, const double* rho, int on_device) {
  if (!c || !rho) return PHZ_E_INVALID;
  PHZ_GUARD_BEGIN
  int rc = set_input(c, rho, on_device, c->rho);
  if (rc) return rc;
  if (count_outside(c->nn, c->rho.p, 0.0, 1.0, c->red_work.p, c->stream) > 0) {
    c->err = "densities must lie in [0, 1]";
    return PHZ_E_INVALID;
  }
  density_to_scale(c->nn, c->rho.p, c->mat.void_scale, c->s.p, c->s32.p, c->stream);
  fill_point_scales(c);
  sync(c);
  c->have_phi = false;
  c->have_s = true;
  c->precond_ready = false;
  c->have_solution = false;
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_get_scale(phz_ctx* c, double* s, int on_device) {
  if (!c || !s) return PHZ_E_INVALID;
  if (!c->have_s) return PHZ_E_STATE;
  PHZ_GUARD_BEGIN
  PHZ_HIP(hipMemcpyAsync(s, c->s.p, c->nn * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         c->stream));
  sync(c);
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_solve(phz_ctx* c) {
  if (!c) return PHZ_E_INVALID;
  PHZ_GUARD_BEGIN
  return do_solve(c);
  PHZ_GUARD_END(c)
}

int phz_get_effective(phz_ctx* c, double CH[36], double eH[18], double kH[9]) {
  if (!c) return PHZ_E_INVALID;
  if (!c->have_solution) { c->err = "no solution: call phz_solve first"; return PHZ_E_STATE; }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j)
      if (CH) CH[i * 6 + j] = kStress * c->MH[i * 9 + j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 6; ++j)
      if (eH) eH[i * 6 + j] = -kCharge * c->MH[(6 + i) * 9 + j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (kH) kH[i * 3 + j] = -kPerm * c->MH[(6 + i) * 9 + 6 + j];
  return PHZ_OK;
}

int phz_get_effective_nd(phz_ctx* c, double MH[81], double MHe[81]) {
  if (!c) return PHZ_E_INVALID;
  if (!c->have_solution) return PHZ_E_STATE;
  if (MH) std::memcpy(MH, c->MH, sizeof(c->MH));
  if (MHe) std::memcpy(MHe, c->MHe, sizeof(c->MHe));
  return PHZ_OK;
}

int phz_get_history(phz_ctx* c, int load, double* buf, int cap, int* len) {
  if (!c || load < 0 || load > 8 || cap < 0) return PHZ_E_INVALID;
  const auto& h = c->hist[load];
  const int n = (int)h.size();
  if (buf)
    for (int i = 0; i < std::min(n, cap); ++i) buf[i] = h[i];
  if (len) *len = n;
  return PHZ_OK;
}

int phz_get_stats(phz_ctx* c, phz_stats* st) {
  if (!c || !st) return PHZ_E_INVALID;
  *st = c->stats;
  return PHZ_OK;
}

int phz_get_solution(phz_ctx* c, double* X, int on_device) {
  if (!c || !X) return PHZ_E_INVALID;
  if (!c->have_solution) return PHZ_E_STATE;
  PHZ_GUARD_BEGIN
  // internal structure of arrays -> documented node-major [n][4][9]
  c->R64.alloc(c->nn * 36);
  soa_to_aos(c->nn, 36, c->X.p, c->R64.p, c->stream);
  PHZ_HIP(hipMemcpyAsync(X, c->R64.p, c->nn * 36 * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_set_initial_guess(phz_ctx* c, const double* X, int on_device) {
  if (!c) return PHZ_E_INVALID;
  PHZ_GUARD_BEGIN
  if (!X) {
    c->have_guess = false;
    return PHZ_OK;
  }
  c->guess.alloc(c->nn * 36);
  c->R64.alloc(c->nn * 36);
  PHZ_HIP(hipMemcpyAsync(c->R64.p, X, c->nn * 36 * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  aos_to_soa(c->nn, 36, c->R64.p, c->guess.p, c->stream);
  if (count_nonfinite(c->nn * 36, c->guess.p, c->red_work.p, c->stream) > 0) {
    c->err = "initial guess holds NaN or Inf";
    return PHZ_E_NAN;
  }
  c->have_guess = true;
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_get_rhs(phz_ctx* c, double* b, int on_device) {
  if (!c || !b) return PHZ_E_INVALID;
  if (!c->have_s) return PHZ_E_STATE;
  PHZ_GUARD_BEGIN
  c->Bvec.alloc(c->nn * 36);
  c->R64.alloc(c->nn * 36);
  prepare_rhs(c);
  soa_to_aos(c->nn, 36, c->Bvec.p, c->R64.p, c->stream);
  PHZ_HIP(hipMemcpyAsync(b, c->R64.p, c->nn * 36 * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_foms(const double CH[36], const double eH[18], const double kH[9], phz_foms_t* out, const char* grad_of,
             double gC[36], double ge[18], double gk[9]) {
  if (!CH || !eH || !kH) return PHZ_E_INVALID;
  double S[36];
  if (!inv_general(6, CH, S)) return PHZ_E_INVALID;
  double d[18];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 6; ++j) {
      double v = 0.0;
      for (int k = 0; k < 6; ++k) v += eH[i * 6 + k] * S[k * 6 + j];
      d[i * 6 + j] = v;
    }
  const double dh = d[12] + d[13] + d[14];
  double bv = 0.0, sr = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      bv += CH[i * 6 + j] / 9.0;
      sr += S[i * 6 + j];
    }
  const double br = 1.0 / sr;
  double de33 = 0.0;  // (d e^T)_33
  for (int j = 0; j < 6; ++j) de33 += d[12 + j] * eH[12 + j];
  const double kT = kH[8] + de33;
  const double gh = dh / kT;
  const double kh = std::sqrt(dh * gh * br);
  if (out) {
    out->d_h = dh;
    out->g_h = gh;
    out->B_voigt = bv;
    out->B_reuss = br;
    out->k_h = kh;
  }
  if (!grad_of) return PHZ_OK;
  // a = S 1_3, b = S^T e_z, c = S^T 1_3, f = S e_z
  double a[6], bb[6], cc[6], ff[6];
  for (int i = 0; i < 6; ++i) {
    a[i] = S[i * 6 + 0] + S[i * 6 + 1] + S[i * 6 + 2];
    cc[i] = S[0 * 6 + i] + S[1 * 6 + i] + S[2 * 6 + i];
    double v = 0.0, w = 0.0;
    for (int k = 0; k < 6; ++k) {
      v += S[k * 6 + i] * eH[12 + k];
      w += S[i * 6 + k] * eH[12 + k];
    }
    bb[i] = v;
    ff[i] = w;
  }
  double dC_dh[36], de_dh[18], dk_dh[9] = {0};
  double dC_kT[36], de_kT[18], dk_kT[9] = {0};
  double dC_br[36];
  for (int i = 0; i < 18; ++i) de_dh[i] = de_kT[i] = 0.0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      dC_dh[i * 6 + j] = -bb[i] * a[j];
      dC_kT[i * 6 + j] = -bb[i] * ff[j];
      dC_br[i * 6 + j] = br * br * cc[i] * a[j];
    }
  for (int j = 0; j < 6; ++j) {
    de_dh[12 + j] = a[j];
    de_kT[12 + j] = bb[j] + ff[j];
  }
  dk_kT[8] = 1.0;
  const std::string which(grad_of);
  double oc[36], oe[18], ok[9];
  for (int i = 0; i < 36; ++i) oc[i] = 0.0;
  for (int i = 0; i < 18; ++i) oe[i] = 0.0;
  for (int i = 0; i < 9; ++i) ok[i] = 0.0;
  if (which == "d_h") {
    for (int i = 0; i < 36; ++i) oc[i] = dC_dh[i];
    for (int i = 0; i < 18; ++i) oe[i] = de_dh[i];
  } else if (which == "B_voigt") {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) oc[i * 6 + j] = 1.0 / 9.0;
  } else if (which == "B_reuss") {
    for (int i = 0; i < 36; ++i) oc[i] = dC_br[i];
  } else if (which == "g_h" || which == "k_h") {
    double gC_[36], ge_[18], gk_[9];
    for (int i = 0; i < 36; ++i) gC_[i] = dC_dh[i] / kT - dh / (kT * kT) * dC_kT[i];
    for (int i = 0; i < 18; ++i) ge_[i] = de_dh[i] / kT - dh / (kT * kT) * de_kT[i];
    for (int i = 0; i < 9; ++i) gk_[i] = dk_dh[i] / kT - dh / (kT * kT) * dk_kT[i];
    if (which == "g_h") {
      std::memcpy(oc, gC_, sizeof(oc));
      std::memcpy(oe, ge_, sizeof(oe));
      std::memcpy(ok, gk_, sizeof(ok));
    } else {
      const double f = 0.5 / kh;
      for (int i = 0; i < 36; ++i) oc[i] = f * (dC_dh[i] * gh * br + dh * gC_[i] * br + dh * gh * dC_br[i]);
      for (int i = 0; i < 18; ++i) oe[i] = f * (de_dh[i] * gh * br + dh * ge_[i] * br);
      for (int i = 0; i < 9; ++i) ok[i] = f * (dh * gk_[i] * br);
    }
  } else {
    return PHZ_E_INVALID;
  }
  if (gC) std::memcpy(gC, oc, sizeof(oc));
  if (ge) std::memcpy(ge, oe, sizeof(oe));
  if (gk) std::memcpy(gk, ok, sizeof(ok));
  return PHZ_OK;
}

int phz_backward(phz_ctx* c, const double gC[36], const double ge[18], const double gk[9], double* grad_rho,
                 double* grad_phi_out, int on_device) {
  if (!c || !grad_rho) return PHZ_E_INVALID;
  if (!c->have_solution) { c->err = "backward needs a solve"; return PHZ_E_STATE; }
  if (grad_phi_out && !c->have_phi) { c->err = "grad_phi needs a level set"; return PHZ_E_STATE; }
  PHZ_GUARD_BEGIN
  double W[81] = {0};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) W[i * 9 + j] = gC ? kStress * gC[i * 6 + j] : 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 6; ++j) W[(6 + i) * 9 + j] = ge ? -kCharge * ge[i * 6 + j] : 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) W[(6 + i) * 9 + 6 + j] = gk ? -kPerm * gk[i * 3 + j] : 0.0;
  for (int i = 0; i < 81; ++i)
    if (!std::isfinite(W[i])) { c->err = "non-finite upstream gradient"; return PHZ_E_NAN; }
  const RefElement& R = c->ref;
  const bool qp = c->opt.smoothing == PHZ_SMOOTH_QP;
  // per element, or per Gauss point p (K0 -> K0q[p], F0 -> F0q[p], the
  // constant term's weight h^3 -> h^3 / 8)
  const int nterms = qp ? 8 : 1;
  std::vector<double> buf((size_t)nterms * 369);
  double cw = 0.0;
  for (int i = 0; i < 81; ++i) cw += W[i] * R.M[i];
  for (int p = 0; p < nterms; ++p) {
    const double* F0 = qp ? R.F0q[p] : R.F0;
    double* b = buf.data() + (size_t)p * 369;
    for (int i = 0; i < 32; ++i)
      for (int L = 0; L < 9; ++L) {
        double v = 0.0;
        for (int K = 0; K < 9; ++K) v += F0[i * 9 + K] * (W[K * 9 + L] + W[L * 9 + K]);
        b[i * 9 + L] = v;
      }
    for (int i = 0; i < 81; ++i) b[288 + i] = W[i];
  }
  const double cterm = cw * std::pow(1.0 / c->N, 3) / nterms;
  DevBuf<double>& dbuf = c->bw_terms;
  dbuf.upload(buf.data(), buf.size(), c->stream);
  c->grad_rho.alloc(c->nn);
  const double eta = c->opt.smooth_width / c->N;
  // U = X W, the same for every term (W follows the first term's FW in dbuf)
  c->bw_u.alloc((size_t)c->nn * 36);
  mix_cols(c->nn, c->X.p, dbuf.p + 288, c->bw_u.p, c->stream);
  if (qp) {
    c->grad_q.alloc((size_t)c->nn * 8);
    for (int p = 0; p < 8; ++p)
      backward_elem(c->N, c->X.p, c->bw_u.p, c->kq64.p + (size_t)p * 1024, dbuf.p + (size_t)p * 369, cterm,
                    1.0 - c->mat.void_scale, c->grad_q.p, c->stream, 8, p);
    sum_points(c->nn, c->grad_q.p, c->grad_rho.p, c->stream);
  } else {
    backward_elem(c->N, c->X.p, c->bw_u.p, c->kref_full.p, dbuf.p, cterm, 1.0 - c->mat.void_scale, c->grad_rho.p,
                  c->stream);
  }
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  PHZ_HIP(hipMemcpyAsync(grad_rho, c->grad_rho.p, c->nn * sizeof(double), kind, c->stream));
  if (grad_phi_out) {
    c->tmp_nodes.alloc(c->nn);
    if (qp) grad_phi_qp(c->N, c->phi.p, eta, c->grad_q.p, 8, c->tmp_nodes.p, c->stream);
    else grad_phi(c->N, c->phi.p, eta, c->grad_rho.p, c->tmp_nodes.p, c->stream);
    PHZ_HIP(hipMemcpyAsync(grad_phi_out, c->tmp_nodes.p, c->nn * sizeof(double), kind, c->stream));
  }
  sync(c);
  c->have_grad = true;
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_hj_step(phz_ctx* c, const double* velocity, double cfl, double* phi_out, int on_device) {
  if (!c || !(cfl > 0)) return PHZ_E_INVALID;
  if (!c->have_phi) { c->err = "HJ step needs a level set"; return PHZ_E_STATE; }
  if (!velocity && !c->have_grad) { c->err = "no velocity and no backward result"; return PHZ_E_STATE; }
  PHZ_GUARD_BEGIN
  DevBuf<double>& v = c->node_a;
  DevBuf<double>& out = c->node_b;
  v.alloc(c->nn);
  out.alloc(c->nn);
  double* vmax = c->small.p + 500;
  if (velocity) {
    int rc = set_input(c, velocity, on_device, v);
    if (rc) return rc;
    hj_step(c->N, c->phi.p, v.p, nullptr, cfl / c->N, out.p, c->stream);
  } else {
    nodal_mean_of_elements(c->N, c->grad_rho.p, v.p, c->stream);
    max_abs(c->nn, v.p, vmax, c->red_work.p, c->stream);
    hj_step(c->N, c->phi.p, v.p, vmax, cfl / c->N, out.p, c->stream);
  }
  PHZ_HIP(hipMemcpyAsync(c->phi.p, out.p, c->nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  update_scales(c);
  if (phi_out)
    PHZ_HIP(hipMemcpyAsync(phi_out, c->phi.p, c->nn * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  sync(c);
  c->precond_ready = false;
  c->have_solution = false;
  c->have_grad = false;
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_hj_step_noalloc(int n, const double* phi, const double* grad_rho, double cfl, double* phi_out,
                        void* stream) {
  g_free_err.clear();
  if (!phi || !grad_rho || !phi_out || !(cfl > 0) || n < 2) {
    g_free_err = "phz_hj_step_noalloc: null buffer, n < 2 or cfl <= 0";
    return PHZ_E_INVALID;
  }
  const long nn = (long)n * n * n;
  if (nn > kNoAllocMaxNodes) {
    g_free_err = "phz_hj_step_noalloc: n^3 = " + std::to_string(nn) + " exceeds the scratch maximum of " +
                 std::to_string(kNoAllocMaxNodes) + " nodes (n <= 128)";
    return PHZ_E_INVALID;
  }
  if (phi_out == phi) {
    g_free_err = "phz_hj_step_noalloc: phi_out must not be phi (the step reads phi's neighbours)";
    return PHZ_E_INVALID;
  }
  double* scr = scratch_of_current_device(g_free_err);
  if (!scr) return PHZ_E_HIP;
  try {
    hipStream_t st = (hipStream_t)stream;
    double* v = scr;                                  // nodal velocity, nn values
    double* part = scr + kNoAllocMaxNodes;            // partial maxima (at most 512)
    double* vmax = scr + kNoAllocMaxNodes + 512;      // max |v|
    nodal_mean_of_elements(n, grad_rho, v, st);
    max_abs(nn, v, vmax, part, st);
    hj_step(n, phi, v, vmax, cfl / n, phi_out, st);
  } catch (const std::exception& ex) {
    g_free_err = ex.what();
    return PHZ_E_HIP;
  }
  return PHZ_OK;
}

// ------------------------------------------------------- optimisation step
namespace phz {

// 27 weights of H = alpha^2 K + M on the periodic node grid, K and M the
// trilinear finite-element Laplace and mass matrices: on a tensor grid both
// are tensor products of the assembled one-dimensional stencils, mass
// h/6 (1, 4, 1) and Laplace (1/h) (-1, 2, -1).
static void helmholtz_weights(int N, double alpha, double* w) {
  const double h = 1.0 / N;
  const double m1[3] = {h / 6.0, 4.0 * h / 6.0, h / 6.0}, k1[3] = {-1.0 / h, 2.0 / h, -1.0 / h};
  for (int d = 0; d < 27; ++d) {
    const int a = d % 3, b = (d / 3) % 3, e = d / 9;
    const double mass = m1[a] * m1[b] * m1[e];
    const double lap = k1[a] * m1[b] * m1[e] + m1[a] * k1[b] * m1[e] + m1[a] * m1[b] * k1[e];
    w[d] = alpha * alpha * lap + mass;
  }
}

// g = H^-1 j for K node columns (device) by Chebyshev iteration.  H is
// periodic with constant coefficients, so its eigenvalues are its symbol at
// the grid frequencies.  Per direction, with c = cos t, the symbols
// m = h (2 + c) / 3 and k = 2 (1 - c) / h are affine in c, so the symbol
// alpha^2 (k1 m2 m3 + m1 k2 m3 + m1 m2 k3) + m1 m2 m3 is multilinear in
// (c1, c2, c3) and takes its extremes at the vertices c = +-1, which are grid
// frequencies for even N: the bounds are exact.  After k steps the residual is
// at most 2 rho^k times the initial one, rho = (sqrt(kappa) - 1) /
// (sqrt(kappa) + 1), so the step count for a relative residual of 1e-12 is
// known in advance and the iteration takes no inner products (no host round
// trip).  Returns the step count.
static int riesz_solve(phz_ctx* c, int K, double alpha, const double* j, double* g) {
  const long nn = c->nn;
  hipStream_t st = c->stream;
  const double h = 1.0 / c->N;
  double lmin = HUGE_VAL, lmax = 0.0;
  for (int v = 0; v < 8; ++v) {
    double m[3], k[3];
    for (int a = 0; a < 3; ++a) {
      const double cs = (v >> a) & 1 ? -1.0 : 1.0;
      m[a] = h * (2.0 + cs) / 3.0;
      k[a] = 2.0 * (1.0 - cs) / h;
    }
    const double lam =
        alpha * alpha * (k[0] * m[1] * m[2] + m[0] * k[1] * m[2] + m[0] * m[1] * k[2]) + m[0] * m[1] * m[2];
    lmin = std::min(lmin, lam);
    lmax = std::max(lmax, lam);
  }
  // the mass part alone spans a factor 27, so lmax > lmin
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  const double sk = std::sqrt(lmax / lmin);
  const double nsteps = std::ceil(std::log(2.0 / 1e-12) / std::log((sk + 1.0) / (sk - 1.0)));
  // the step count grows with alpha / h (kappa ~ 4 (alpha / h)^2, about
  // 28 alpha / h steps): refuse length scales that would take more than 20000
  if (!(nsteps <= 20000.0)) throw std::invalid_argument("alpha too large for the extension (too many steps)");
  const int steps = (int)nsteps;
  helmholtz_weights(c->N, alpha, c->rz_host);
  for (int k = 0; k < K; ++k) c->rz_host[27 + k] = 1.0 / theta;
  c->helm_w.upload(c->rz_host, 27, st);
  c->rz_dev.upload(c->rz_host + 27, K, st);
  for (DevBuf<double>* v : {&c->rz_r, &c->rz_z, &c->rz_p})
    if (v->n < (size_t)nn * K) v->alloc((size_t)nn * K);
  double *r = c->rz_r.p, *d = c->rz_z.p, *dn = c->rz_p.p;
  PHZ_HIP(hipMemcpyAsync(r, j, (size_t)nn * K * sizeof(double), hipMemcpyDeviceToDevice, st));
  fill<double>(nn * K, 0.0, g, st);
  scale_cols<double>(nn, 1, K, r, c->rz_dev.p, d, st);  // d0 = r0 / theta
  double rho = 1.0 / sigma;
  for (int it = 0; it < steps; ++it) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    stencil_cheb_step(c->N, K, c->helm_w.p, d, g, r, dn, rho1 * rho, 2.0 * rho1 / delta, st);
    std::swap(d, dn);
    rho = rho1;
  }
  return steps;
}

// copies K host or device node vectors into one device block of K columns
static void gather_columns(phz_ctx* c, int K, const double* const* src, int on_device, DevBuf<double>& dst) {
  dst.alloc((size_t)c->nn * K);
  for (int k = 0; k < K; ++k)
    PHZ_HIP(hipMemcpyAsync(dst.p + (size_t)k * c->nn, src[k], c->nn * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
}

static double device_max_abs(phz_ctx* c, const double* v) {
  double* out = c->small.p + 500;
  max_abs(c->nn, v, out, c->red_work.p, c->stream);
  double mx = 0.0;
  PHZ_HIP(hipMemcpyAsync(&mx, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return mx;
}

static double device_dot(phz_ctx* c, const double* a, const double* b) {
  double* out = c->small.p + 501;
  col_dot<double>(c->nn, 1, 1, a, b, out, c->red_work.p, c->stream);
  double d = 0.0;
  PHZ_HIP(hipMemcpyAsync(&d, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return d;
}

}  // namespace phz

int phz_reinit(phz_ctx* c, int steps, double cfl, int subcell, double* phi_out, int on_device) {
  if (!c || steps < 0 || !(cfl > 0) || (subcell != 0 && subcell != 1)) return PHZ_E_INVALID;
  if (!c->have_phi) { c->err = "reinitialisation needs a level set"; return PHZ_E_STATE; }
  PHZ_GUARD_BEGIN
  // phi0 stays fixed; the steps alternate between the geometry and rz_r
  for (DevBuf<double>* v : {&c->rz_p, &c->rz_r})
    if (v->n < (size_t)c->nn) v->alloc(c->nn);
  double* phi0 = c->rz_p.p;
  double* buf[2] = {c->phi.p, c->rz_r.p};
  PHZ_HIP(hipMemcpyAsync(phi0, c->phi.p, c->nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  for (int i = 0; i < steps; ++i)
    reinit_step(c->N, buf[i & 1], phi0, cfl / c->N, subcell, buf[(i + 1) & 1], c->stream);
  if (steps & 1)
    PHZ_HIP(hipMemcpyAsync(c->phi.p, buf[1], c->nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  update_scales(c);
  if (phi_out)
    PHZ_HIP(hipMemcpyAsync(phi_out, c->phi.p, c->nn * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  sync(c);
  c->precond_ready = false;
  c->have_solution = false;
  c->have_grad = false;
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_levelset_gradient(phz_ctx* c, const double* grad_rho, double* grad_phi, int on_device) {
  if (!c || !grad_rho || !grad_phi) return PHZ_E_INVALID;
  if (!c->have_phi) { c->err = "the chain rule needs a level set"; return PHZ_E_STATE; }
  PHZ_GUARD_BEGIN
  DevBuf<double>& g = c->node_a;
  DevBuf<double>& out = c->node_b;
  const double* gr = grad_rho;
  if (!on_device) {
    g.upload(grad_rho, c->nn, c->stream);
    gr = g.p;
  }
  double* o = grad_phi;
  if (!on_device) {
    out.alloc(c->nn);
    o = out.p;
  }
  // with quadrature-point smoothing an element gradient is the derivative for
  // the element's mean point density: each point takes an eighth
  if (c->opt.smoothing == PHZ_SMOOTH_QP) phz::grad_phi_qp(c->N, c->phi.p, c->opt.smooth_width / c->N, gr, 1, o, c->stream);
  else phz::grad_phi(c->N, c->phi.p, c->opt.smooth_width / c->N, gr, o, c->stream);
  if (!on_device) PHZ_HIP(hipMemcpyAsync(grad_phi, o, c->nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_riesz(phz_ctx* c, int ncol, double alpha, const double* j, double* g, int* iters) {
  if (!c || !j || !g || ncol < 1 || ncol > 9 || !(alpha >= 0)) return PHZ_E_INVALID;
  PHZ_GUARD_BEGIN
  const int it = riesz_solve(c, ncol, alpha, j, g);
  sync(c);
  if (iters) *iters = it;
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_hpm_velocity(phz_ctx* c, int m, const double* j_obj, const double* const* j_cons, const double* viol,
                     double alpha, double cfl, double gamma, double obj_weight, double* v_out, int on_device) {
  if (!c || !j_obj || !v_out || m < 0 || m > 8 || (m > 0 && (!j_cons || !viol)) || !(cfl > 0) || !(gamma >= 0) ||
      !(obj_weight >= 0.0 && obj_weight <= 1.0))
    return PHZ_E_INVALID;
  for (int i = 0; i < m; ++i)
    if (!j_cons[i] || !std::isfinite(viol[i])) return PHZ_E_INVALID;
  PHZ_GUARD_BEGIN
  const long nn = c->nn;
  const int K = 1 + m;
  const double h = 1.0 / c->N;
  if (!(alpha > 0)) alpha = 4.0 * h;
  std::vector<const double*> src(K);
  src[0] = j_obj;
  for (int i = 0; i < m; ++i) src[1 + i] = j_cons[i];
  gather_columns(c, K, src.data(), on_device, c->rz_j);
  c->rz_g.alloc((size_t)nn * K);
  riesz_solve(c, K, alpha, c->rz_j.p, c->rz_g.p);
  const double* jv = c->rz_j.p;
  const double* gv = c->rz_g.p;
  auto col = [&](const double* base, int k) { return base + (size_t)k * nn; };
  // Gram matrix of the constraint directions and their products with g_0
  std::vector<double> G((size_t)m * m), b(m), lb(m), lc(m);
  for (int i = 0; i < m; ++i) {
    b[i] = device_dot(c, col(jv, 1 + i), col(gv, 0));
    for (int k = 0; k < m; ++k) G[(size_t)i * m + k] = device_dot(c, col(jv, 1 + i), col(gv, 1 + k));
  }
  if (m > 0) {
    // small dense solves G lb = b, G lc = viol (Gaussian elimination, partial pivoting)
    std::vector<double> A = G, rb = b, rc(viol, viol + m);
    for (int p = 0; p < m; ++p) {
      int piv = p;
      for (int r = p + 1; r < m; ++r)
        if (std::fabs(A[(size_t)r * m + p]) > std::fabs(A[(size_t)piv * m + p])) piv = r;
      if (!(std::fabs(A[(size_t)piv * m + p]) > 0)) throw std::runtime_error("constraint directions are dependent");
      if (piv != p) {
        for (int q = 0; q < m; ++q) std::swap(A[(size_t)p * m + q], A[(size_t)piv * m + q]);
        std::swap(rb[p], rb[piv]);
        std::swap(rc[p], rc[piv]);
      }
      for (int r = p + 1; r < m; ++r) {
        const double f = A[(size_t)r * m + p] / A[(size_t)p * m + p];
        for (int q = p; q < m; ++q) A[(size_t)r * m + q] -= f * A[(size_t)p * m + q];
        rb[r] -= f * rb[p];
        rc[r] -= f * rc[p];
      }
    }
    for (int p = m - 1; p >= 0; --p) {
      double sb = rb[p], sc = rc[p];
      for (int q = p + 1; q < m; ++q) {
        sb -= A[(size_t)p * m + q] * lb[q];
        sc -= A[(size_t)p * m + q] * lc[q];
      }
      lb[p] = sb / A[(size_t)p * m + p];
      lc[p] = sc / A[(size_t)p * m + p];
    }
  }
  // theta_J = g_0 - sum_i lb_i g_i into the output
  double* v = v_out;
  if (!on_device) {
    c->node_a.alloc(nn);
    v = c->node_a.p;
  }
  PHZ_HIP(hipMemcpyAsync(v, col(gv, 0), nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  double* cf = c->small.p + 502;
  auto add = [&](double a, const double* x) {
    PHZ_HIP(hipMemcpyAsync(cf, &a, sizeof(double), hipMemcpyHostToDevice, c->stream));
    axpy_cols<double, double>(nn, 1, 1, cf, x, v, c->stream);
    sync(c);
  };
  for (int i = 0; i < m; ++i) add(-lb[i], col(gv, 1 + i));
  const double mj = device_max_abs(c, v);
  if (!(mj > 0)) throw std::runtime_error("the objective direction vanishes");
  // v = w theta_J / max|theta_J| + (gamma / (cfl h)) theta_C, theta_C = -sum_i lc_i g_i
  std::vector<double> one{obj_weight / mj};
  PHZ_HIP(hipMemcpyAsync(cf, one.data(), sizeof(double), hipMemcpyHostToDevice, c->stream));
  scale_cols<double>(nn, 1, 1, v, cf, v, c->stream);
  sync(c);
  const double sC = gamma / (cfl * h);
  for (int i = 0; i < m; ++i) add(-sC * lc[i], col(gv, 1 + i));
  const double mv = device_max_abs(c, v);
  if (mv > 1.0) {
    one[0] = 1.0 / mv;
    PHZ_HIP(hipMemcpyAsync(cf, one.data(), sizeof(double), hipMemcpyHostToDevice, c->stream));
    scale_cols<double>(nn, 1, 1, v, cf, v, c->stream);
  }
  if (!on_device) PHZ_HIP(hipMemcpyAsync(v_out, v, nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_kernel_timing(phz_ctx* c, int enable) {
  if (!c || enable < 0 || enable > 2) return PHZ_E_INVALID;
  PHZ_GUARD_BEGIN
  sync(c);
  collect_timing(c);
  c->ktime = enable != 0;
  c->ktime_fine_only = enable == 2;
  c->ktotals.clear();
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_get_kernel_timing(phz_ctx* c, char* buf, int cap, int* len) {
  if (!c || cap < 0) return PHZ_E_INVALID;
  PHZ_GUARD_BEGIN
  sync(c);
  collect_timing(c);
  std::string out;
  char line[160];
  for (auto& kv : c->ktotals) {
    std::snprintf(line, sizeof(line), "%s %ld %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
    out += line;
  }
  if (len) *len = (int)out.size();
  if (buf && cap > 0) {
    const int n = std::min(cap - 1, (int)out.size());
    std::memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_apply(phz_ctx* c, int op, int nrhs, int precision, const void* x, void* y) {
  if (!c || !x || !y || op < 0 || op > 5 || (nrhs != 1 && nrhs != 9)) return PHZ_E_INVALID;
  if (!c->have_s) return PHZ_E_STATE;
  if (op == 5 && precision == PHZ_BF16X3_IR) {
    c->err = "B^T has no split-BF16 form";
    return PHZ_E_INVALID;
  }
  if (op == 0 && precision == PHZ_BF16X3_IR && c->opt.smoothing == PHZ_SMOOTH_QP) {
    c->err = "the split-BF16 full operator has no quadrature-point form";
    return PHZ_E_INVALID;
  }
  PHZ_GUARD_BEGIN
  if (precision == PHZ_FP64)
    op_apply<double>(c, op, nrhs, (const double*)x, (const double*)nullptr, (double*)y, 1.0, 0.0);
  else if (precision == PHZ_FP32_IR)
    op_apply<float>(c, op, nrhs, (const float*)x, (const float*)nullptr, (float*)y, 1.0f, 0.0f);
  else if (precision == PHZ_BF16X3_IR) {
    const int tile = nrhs == 9 ? elem_tile_of(c, shape_of(op)) : -1;
    if (tile < 0) {
      c->err = "split-BF16 apply needs nine columns and a tile that divides N";
      return PHZ_E_INVALID;
    }
    elem_apply(shape_of(op), 9, c->N, c->opt.bf16_terms, tile, c->s32.p, c->kop[op].p, (const float*)x,
               plain_args<float>(nullptr, (float*)y, 1.0f, 0.0f), false, c->stream);
  } else
    return PHZ_E_INVALID;
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

extern "C++" {
template <typename T>
static void orthogonalize_hook(phz_ctx* c, int j, const T* V, T* w, double* h, double* nrm2, int* second) {
  const long nn = c->nn;
  const int K = 9;
  hipStream_t st = c->stream;
  const long vs = 36 * nn;
  const bool selective = c->opt.reorth_tol >= 0.0;
  const double tau = c->opt.reorth_tol > 0.0 ? c->opt.reorth_tol
                                             : 32.0 * (std::is_same<T, float>::value ? 0x1p-24 : 0x1p-53);
  GmresState S = gm_state(c);
  const int ones[9] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
  PHZ_HIP(hipMemcpyAsync(S.active, ones, sizeof(ones), hipMemcpyHostToDevice, st));
  PHZ_HIP(hipMemsetAsync(c->gm_reorth.p, 0, K * sizeof(int), st));
  double* nrm = c->gm_nrm.p;
  arnoldi_dots<T>(nn, 4, K, j, V, vs, w, c->gm_h1.p, c->red_work.p, st);
  arnoldi_update<T>(nn, 4, K, j, V, vs, w, c->gm_h1.p, c->gm_h2.p, c->gm_na2.p, c->red_work.p, st);
  reorth_decide(K, j + 1, selective ? tau * tau : -1.0, c->gm_h2.p, c->gm_na2.p, S.active, c->gm_flag.p,
                c->gm_reorth.p, st);
  arnoldi_update<T>(nn, 4, K, j, V, vs, w, c->gm_h2.p, nullptr, nrm, c->red_work.p, st, c->gm_flag.p);
  std::vector<double> h1((size_t)(j + 1) * K), h2((size_t)(j + 1) * K), n1(K), n2(K);
  std::vector<int> fl(K);
  PHZ_HIP(hipMemcpyAsync(h1.data(), c->gm_h1.p, h1.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  PHZ_HIP(hipMemcpyAsync(h2.data(), c->gm_h2.p, h2.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  PHZ_HIP(hipMemcpyAsync(n1.data(), c->gm_na2.p, K * sizeof(double), hipMemcpyDeviceToHost, st));
  PHZ_HIP(hipMemcpyAsync(n2.data(), nrm, K * sizeof(double), hipMemcpyDeviceToHost, st));
  PHZ_HIP(hipMemcpyAsync(fl.data(), c->gm_flag.p, K * sizeof(int), hipMemcpyDeviceToHost, st));
  sync(c);
  for (int k = 0; k < K; ++k) {
    for (int i = 0; i <= j; ++i) h[i * K + k] = h1[i * K + k] + h2[i * K + k];
    nrm2[k] = fl[k] ? n2[k] : n1[k];
    second[k] = fl[k];
  }
}
}  // extern "C++"

int phz_orthogonalize(phz_ctx* c, int precision, int nvec, const void* V, void* w, double* h, double* nrm2,
                      int* second_pass) {
  if (!c || !V || !w || !h || !nrm2 || !second_pass || nvec < 1 || nvec > kMaxRestart + 1) return PHZ_E_INVALID;
  if (precision != PHZ_FP64 && precision != PHZ_FP32_IR) return PHZ_E_INVALID;
  PHZ_GUARD_BEGIN
  ensure_state_buffers(c);
  if (precision == PHZ_FP64)
    orthogonalize_hook<double>(c, nvec - 1, (const double*)V, (double*)w, h, nrm2, second_pass);
  else
    orthogonalize_hook<float>(c, nvec - 1, (const float*)V, (float*)w, h, nrm2, second_pass);
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_precondition(phz_ctx* c, int nrhs, const double* r, double* z) {
  if (!c || !r || !z || (nrhs != 1 && nrhs != 9)) return PHZ_E_INVALID;
  if (!c->have_s) return PHZ_E_STATE;
  PHZ_GUARD_BEGIN
  ensure_state_buffers(c);
  if (c->opt.precision != PHZ_FP64) { c->err = "phz_precondition runs the float64 preconditioner"; }
  const int saved = c->opt.precision;
  c->opt.precision = PHZ_FP64;
  setup_preconditioner(c);
  alloc_work<double>(c, c->w64, nrhs, c->opt.restart);
  precond_apply<double>(c, nrhs, r, z);
  c->opt.precision = saved;
  if (saved != PHZ_FP64) c->precond_ready = false;
  sync(c);
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

int phz_coarse_apply(phz_ctx* c, int level, int op, int nrhs, int precision, const void* x, void* y) {
  if (!c || !x || !y || (nrhs != 1 && nrhs != 9) || (op != PHZ_OP_A && op != PHZ_OP_SBAR)) return PHZ_E_INVALID;
  if (precision != PHZ_FP64 && precision != PHZ_FP32_IR) return PHZ_E_INVALID;
  if (!c->have_s) return PHZ_E_STATE;
  PHZ_GUARD_BEGIN
  ensure_state_buffers(c);
  setup_preconditioner(c);
  Hierarchy& H = op == PHZ_OP_A ? c->hA : c->hS;
  if (level < 1 || level >= (int)H.lv.size()) { c->err = "level out of range"; return PHZ_E_INVALID; }
  Level& L = *H.lv[level];
  if (precision == PHZ_FP64) {
    coarse_apply<double>(H.F, nrhs, L.N, L.S.p, (const double*)x, plain_args<double>(nullptr, (double*)y, 1.0, 0.0),
                         false, c->stream);
  } else {
    if (!L.S32.p) { c->err = "float32 coarse operators exist only in the float forms"; return PHZ_E_STATE; }
    const OpArgs<float> a = plain_args<float>(nullptr, (float*)y, 1.0f, 0.0f);
    const int kind = nrhs == 9 ? coarse_kind_of(c, H, level) : 0;
    if (kind == 1) coarse_apply_tiled(H.F, L.N, L.S32.p, (const float*)x, a, false, c->stream);
    else if (kind == 2) coarse_apply_tiled_compact(H.F, L.N, L.S16.p, L.Sc.p, (const float*)x, a, false, c->stream);
    else coarse_apply<float>(H.F, nrhs, L.N, L.S32.p, (const float*)x, a, false, c->stream);
  }
  sync(c);
  return PHZ_OK;
  PHZ_GUARD_END(c)
}

}  // extern "C"
