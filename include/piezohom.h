/*
 * piezohom — periodic piezoelectric homogenisation on one AMD MI355X (gfx950).
 *
 * The library computes the effective (homogenised) tensors of a periodic
 * piezoelectric unit cell, following Wegert, Roberts & Challis, "Level
 * set-based inverse homogenisation of three-dimensional piezoelectric
 * materials":
 *
 *   Sec. 2.1   the cell geometry is a level set phi (phi < 0 solid, phi > 0
 *              void) or a per-element density rho in [0, 1];
 *   Sec. 2.2   the nine cell problems (six unit macroscopic strains, three
 *              unit macroscopic electric fields) of linear piezoelectricity
 *              are solved on a periodic N^3 mesh of trilinear hexahedra with
 *              4 dofs per node (u_x, u_y, u_z, phi); the effective C^H, e^H,
 *              kappa^H are the cell averages of stress and electric
 *              displacement (the paper's homogenisation formulas);
 *   Sec. 2.5   the saddle-point system [[A, B^T], [B, -C]] is solved by
 *              right-preconditioned GMRES with the block lower-triangular
 *              approximate-Schur preconditioner of Sec. 2.5.3, whose Schur
 *              block is the element-wise S_bar = sum_e C_e + B_e A_e^-1 B_e^T;
 *              the inner maps v -> A\v and u -> S_bar\u are geometric
 *              multigrid V-cycles with Chebyshev-Jacobi smoothing;
 *   Sec. 2.3   figures of merit d_h, g_h, B_Voigt, B_Reuss, k_h;
 *   Sec. 2.1   one Hamilton-Jacobi upwind step of the level set.
 *
 * Material interpolation: every element carries the ersatz scale
 * s_e = eps_v + (1 - eps_v) rho_e applied to C, e and kappa alike, with
 * rho_e = 1 - H_eta(mean of the element's 8 nodal phi), H_eta the sinusoidal
 * smoothed Heaviside of half-width eta = smooth_width * h (Sec. 2.6: the
 * interface is smoothed over about two elements).
 *
 * Grid and layouts (all arrays are C order, float64 unless stated):
 *   node n = i + N*(j + N*k), x fastest, coordinates (i, j, k)/N, periodic;
 *   element (i, j, k) has corner nodes ((i+a)%N, (j+b)%N, (k+c)%N) and shares
 *   the node numbering (element e "starts" at node e);
 *   solution X: [node][field 0..3][load 0..8], fields (u_x, u_y, u_z, phi),
 *   loads in Voigt order (xx, yy, zz, yz, xz, xy) then (E_x, E_y, E_z);
 *   tensors are SI, Voigt order (xx, yy, zz, yz, xz, xy), engineering shear:
 *   C[6*6] Pa, e[3*6] C/m^2, kappa[3*3] F/m, all row-major.
 *
 * Ownership: the caller owns every buffer it passes.  Host pointers are
 * read or written before the call returns.  Device pointers (on_device = 1)
 * must be device memory of the context's device; the library reads and
 * writes them on the context's stream, and the caller orders later work on
 * that stream.  The library owns its workspaces until phz_destroy.
 *
 * Errors: every call returns an int status.  PHZ_OK = 0;
 * PHZ_NOT_CONVERGED = 1 is a warning (outputs and histories are written);
 * negative values are errors, after which phz_last_error(ctx) describes the
 * cause.  Nothing throws, aborts or exits across this interface.  A context
 * is used by one host thread at a time.
 */
#ifndef PIEZOHOM_H
#define PIEZOHOM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PHZ_OK 0
#define PHZ_NOT_CONVERGED 1
#define PHZ_E_INVALID (-1)
#define PHZ_E_NAN (-2)
#define PHZ_E_HIP (-3)
#define PHZ_E_OOM (-4)
#define PHZ_E_STATE (-5)
#define PHZ_E_INTERNAL (-6)

/* precision forms of phz_options.precision */
#define PHZ_FP64 0       /* every kernel and vector in float64 */
#define PHZ_FP32_IR 1    /* float32 operator, smoothers and Krylov basis inside
                            float64 iterative refinement; float64 residuals,
                            Hessenberg/Givens, coarse solve and reductions */
#define PHZ_BF16X3_IR 2  /* as PHZ_FP32_IR, with the fine-level operators of
                            the float solve computed as element contractions
                            on the matrix cores in split-BF16 arithmetic: each
                            float32 value x = hi + lo with hi, lo bfloat16, and
                            products hi*hi + hi*lo + lo*hi accumulated in
                            float32 (about 2^-16 relative per product).  The
                            preconditioner's fine blocks always, the float
                            GMRES operator if bf16_outer.  Float vectors stay
                            float32; refinement, residuals, Hessenberg/Givens,
                            coarse solve and reductions stay float64. */

/* solvers of phz_options.solver (Sec. 2.5): the first two right-precondition
 * GMRES on calA */
#define PHZ_SOLVER_SCP 0 /* approximate Schur complement, lower block-triangular
                            [[A, 0], [-B, S_bar]] (SCP-GMRES, the default)   */
#define PHZ_SOLVER_DBP 1 /* block diagonal [[A, 0], [0, -C]] (DBP-GMRES)     */
#define PHZ_SOLVER_TRICG 2 /* TriCG (Sec. 2.5.2) on the quasi-definite calA:
                            orthogonal tridiagonalisation in the A- and
                            C-inner products, block LDL^T short recurrences;
                            A^-1 and C^-1 by conjugate gradients to inner_eps
                            (one V-cycle per iteration).  PHZ_FP64 only.
                            Each cycle starts from the true residual; a
                            residual block below 1e-12 of the other, or
                            below min(1e-13, rtol / 10) of ||b||, starts
                            from a shifted point (c = 0: y0 = C^-1 B A^-1 b;
                            b = 0: x0 = -A^-1 B^T C^-1 c), and a breakdown
                            (beta or gamma below 1e-10 of its largest value)
                            ends the cycle.  stats: iterations = TriCG
                            iterations, restarts = cycles                    */

/* smoothing of the material near the interface (phz_options.smoothing;
 * Sec. 2.6: within two elements of the zero level set) */
#define PHZ_SMOOTH_ELEMENT 0 /* once per element, at the mean of its 8 nodal
                                phi (default)                               */
#define PHZ_SMOOTH_QP 1      /* at each of the element's 8 Gauss points, on
                                the trilinear interpolation of phi: the
                                operator, loads and tensors use the point
                                scales; the preconditioner (multigrid, S_bar,
                                the split-BF16 blocks) their element means.
                                Not with TriCG.  phz_backward
                                differentiates the point densities (its
                                grad_rho[e] is their sum over the element,
                                the derivative for a uniform change of the
                                element's points); phz_levelset_gradient
                                spreads an element gradient evenly over its
                                points.  A cell given by densities has equal
                                point scales (the element form)             */

/* operator blocks for phz_apply (Sec. 2.5 block structure) */
#define PHZ_OP_FULL 0    /* calA = [[A, B^T], [B, -C]] on [n][4][k]        */
#define PHZ_OP_A 1       /* A (elasticity) on [n][3][k]                    */
#define PHZ_OP_B 2       /* B (coupling) [n][3][k] -> [n][1][k]            */
#define PHZ_OP_SBAR 3    /* element-wise approximate Schur S_bar on [n][1][k] */
#define PHZ_OP_C 4       /* C (dielectric; calA's (phi, phi) block is -C) on
                            [n][1][k]                                       */
#define PHZ_OP_BT 5      /* B^T [n][1][k] -> [n][3][k] (PHZ_FP64 and
                            PHZ_FP32_IR only)                                */

typedef struct phz_ctx phz_ctx;

/* Base material, SI units (Sec. 2.3 layout).  void_scale = eps_v. */
typedef struct {
    double C[36];
    double e[18];
    double kappa[9];
    double void_scale;
} phz_material;

typedef struct {
    int precision;          /* PHZ_FP64, PHZ_FP32_IR or PHZ_BF16X3_IR (default
                               PHZ_FP64)                                        */
    int batched;            /* 1: the nine loads as one 9-column block;
                               0: one load at a time                            */
    int restart;            /* GMRES restart length m (default 30)              */
    int max_iters;          /* cap on GMRES iterations per load (default 2000)  */
    double rtol;            /* true relative residual target (default 1e-10)    */
    int cheby_degree;       /* Chebyshev smoothing degree per sweep (default 2) */
    int mg_levels;          /* 0 = coarsen while N even and N > 4               */
    double smooth_width;    /* eta / h of the smoothed Heaviside (default 2)    */
    int vcycles_a;          /* V-cycles per application of A^-1 (default 1)     */
    int vcycles_s;          /* V-cycles per application of S_bar^-1 (default 1) */
    double inner_rtol;      /* FP32_IR: relative residual reduction at which one
                               float GMRES cycle stops early (default 1e-5)     */
    int max_refine;         /* FP32_IR: cap on refinement steps, each one float
                               GMRES cycle of at most `restart` steps (default 50) */
    int verbose;            /* 0 silent; 1 per-solve summary on stderr          */
    int bf16_terms;         /* PHZ_BF16X3_IR: split products of the float GMRES
                               operator's element contraction (bf16_outer) and
                               of phz_apply: 3 (default) or 1 (hi*hi only,
                               about 2^-8 relative)                            */
    int bf16_outer;         /* PHZ_BF16X3_IR: 1 (default) also runs the float
                               GMRES operator on the matrix cores, 0 only the
                               preconditioner's fine blocks                    */
    int elem_tile;          /* PHZ_BF16X3_IR: workgroup tile of the element
                               contraction, -1 (default) = the fastest tile
                               that divides N, timed per block (and the block
                               runs on whichever kernel, fine_kernel, timed
                               fastest; in both choices a later candidate
                               must be more than 3% faster to replace an
                               earlier one), else an index in [0, 3): 8x8x4,
                               16x4x4, 16x8x2 nodes, used for every block    */
    int use_graph;          /* 1: each GMRES Arnoldi step (preconditioner,
                               operator, orthogonalisation, Givens update) is
                               captured once as a HIP graph and replayed; the
                               graphs survive geometry changes and are
                               re-captured when options or workspaces change.
                               Per-kernel timing (phz_kernel_timing) runs the
                               steps eagerly.  Default 0                      */
    int fine_kernel;        /* float32 nine-column fine blocks: -1 (default)
                               the fastest of those that apply, timed once per
                               context; 0 the direct gather; 1 the gather with
                               the input tile staged in LDS (N a multiple of
                               16); 2 the element contraction (PHZ_BF16X3_IR).
                               A kernel that does not apply falls back to 0.
                               In PHZ_BF16X3_IR a fixed elem_tile selects 2. */
    int block_kernel[4];    /* per fine block (full, A, B, S_bar): -1 (default)
                               follows elem_tile / fine_kernel above, else pins
                               that block's float32 nine-column kernel (0, 1, 2
                               as in fine_kernel; one that does not apply falls
                               back to 0).  For reproducible profiling: pin
                               the choice that phz_get_stats reported        */
    int block_tile[4];      /* per fine block: -1 (default) follows elem_tile,
                               else pins the element-contraction tile index  */
    int coarse_kernel;      /* float32 nine-column applies of the coarse
                               multigrid levels: -1 (default) per level the
                               fastest (timed once, in the order 0, 1, 2; a
                               later one must be more than 3% faster) of
                               0 the direct stencil apply, 1 the apply with
                               the input tile staged in LDS, and 2 the same on
                               compact stencils: the 26 off-centre blocks in
                               bf16 and the centre block as minus their sum,
                               so that rows still annihilate constants and
                               the bf16 error scales with the differences
                               across the stencil (1 and 2: levels with N a
                               multiple of 16); 0, 1 or 2 forces that kernel
                               where it applies.  The coarse operators serve
                               the preconditioner only                        */
    int solver;             /* PHZ_SOLVER_SCP (default), PHZ_SOLVER_DBP or
                               PHZ_SOLVER_TRICG                               */
    int inner;              /* block maps v -> A^-1 v and the potential block's
                               inverse (S_bar or C): 0 (default) fixed V-cycle
                               counts (vcycles_a, vcycles_s), a fixed linear
                               preconditioner; 1 conjugate gradients with one
                               V-cycle per iteration to the relative tolerance
                               inner_eps (inexact inner solves, Sec. 2.5; the
                               GMRES cycles are then flexible, keeping the
                               preconditioned basis, and are not captured in
                               graphs)                                        */
    double inner_eps;       /* inner = 1: relative tolerance, default 1e-2     */
    int inner_maxit;        /* inner = 1: iterations per map, default 200      */
    int warm_start;         /* 1: a solve with no phz_set_initial_guess guess
                               starts from the last successful solve's
                               solution, kept on the device across geometry
                               changes (an optimisation loop's next cell is
                               close to the last); 0 (default) from zero     */
    int smoothing;          /* PHZ_SMOOTH_ELEMENT (default) or PHZ_SMOOTH_QP;
                               a change recomputes the current geometry's
                               scales                                        */
    int bf16_terms_precond; /* PHZ_BF16X3_IR: split products of the element
                               contractions inside the preconditioner (the A,
                               B and S_bar blocks' smoothing steps and
                               residuals): 1 (default) or 3.  The
                               preconditioner's own accuracy sets only how
                               fast GMRES converges; the operator and the FP64
                               refinement set the result                     */
    int ir_fallback;        /* PHZ_FP32_IR and PHZ_BF16X3_IR: 1 (default) when
                               a refinement step leaves a load above rtol
                               without reducing its float64 residual tenfold
                               (its float cycle having aimed at more), the
                               float solve moves one form down for the rest
                               of the solve: split-BF16 -> float32 kernels
                               (float32 gathers and stencils) -> a float64
                               GMRES from the current iterate to rtol; 0 never;
                               2 treats every refinement step as stalled (a
                               host-side switch that exercises the path).
                               phz_stats reports the form that finished     */
    double reorth_tol;      /* Arnoldi orthogonalisation: classical
                               Gram-Schmidt, whose first pass also computes
                               h2 = V^T w' of the projected vector w'; a load
                               takes the second pass only where
                               |h2| > reorth_tol |w'| (|h2| / |w'| is the new
                               basis vector's departure from orthogonality).
                               0 (default): 32 units of roundoff of the
                               basis's type; > 0 that tolerance; < 0 the
                               second pass always (CGS2)                      */
} phz_options;

typedef struct {
    int iterations[9];      /* total GMRES iterations per load (inner, for IR) */
    int restarts[9];        /* restart cycles per load                          */
    int refinements;        /* FP64 refinement steps (FP32_IR), else 0          */
    double true_residual[9];/* final ||b - calA x|| / ||b|| in float64          */
    double flux_energy_defect; /* max |MH_flux - MH_energy| / max |MH|          */
    double setup_ms;        /* preconditioner setup (last phz_solve)            */
    double solve_ms;        /* whole phz_solve wall time                        */
    int mg_levels;          /* levels used                                      */
    double cheb_lambda[16]; /* lambda_max estimates, A then S_bar per level     */
    int elem_tile[4];       /* PHZ_BF16X3_IR: tile used per fine block (full, A,
                               B, S_bar), -1 where the block is not on MFMA
                               (bf16_outer = 0, no tile divides N, or another
                               kernel timed faster)                           */
    int fine_kernel[4];     /* kernel of each fine block's float32 nine-column
                               launches (fine_kernel codes), -1 if the solve
                               has none (FP64, or loads one at a time)        */
    int coarse_kernel[16];  /* kernel of the float32 nine-column applies per
                               coarse level (coarse_kernel codes): [l] for the
                               A hierarchy, [8 + l] for S_bar, l >= 1; -1 for
                               level 0, absent levels, FP64 and single-load
                               solves                                          */
    long inner_iters[2];    /* inner = 1: conjugate-gradient iterations summed
                               over the solve, [0] the A maps, [1] the
                               potential block's maps                          */
    long inner_calls[2];    /* inner = 1: number of those maps                 */
    int final_precision;    /* form that finished the last solve: the option's
                               precision, or after refinement-stall fallbacks
                               PHZ_FP32_IR or PHZ_FP64 (ir_fallback)          */
    int fallbacks;          /* refinement-stall fallbacks in the last solve   */
    long reorth_passes;     /* second Gram-Schmidt passes taken, summed over
                               loads and Arnoldi steps (reorth_tol)           */
} phz_stats;

typedef struct {
    double d_h, g_h, B_voigt, B_reuss, k_h;
} phz_foms_t;

/* Device memory supplied by the caller (for instance a framework's caching
 * allocator).  alloc(bytes, stream, user) returns device memory of the
 * context's device usable on `stream` (the context's stream), or NULL on
 * failure (the calling entry point then returns PHZ_E_OOM);
 * free(ptr, stream, user) takes back a pointer alloc returned, after all work
 * the library queued on `stream` that reads or writes it (the library calls
 * free only for memory whose last use is ordered before the call on that
 * stream).  The callbacks run on the thread that called the entry point, only
 * during calls on the context that was created with them, and must not call
 * back into the library. */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*free)(void* ptr, void* stream, void* user);
    void* user;
} phz_allocator;

/* Fill *o with the defaults documented in phz_options. */
void phz_default_options(phz_options* o);

/* Create a context for a periodic cell of nx x ny x nz elements (the cell
 * resolution of Sec. 2.6; Sec. 2.2's cell problems on the unit cube).  The
 * cell must be cubic (nx = ny = nz = N, else PHZ_E_INVALID).  N must be even
 * and >= 2 (multigrid halves N), and halving N while it is even and above 4
 * (at most mg_levels - 1 times when mg_levels > 0) must end at a side of at
 * most 10: the coarsest level is inverted densely on the host.  So N = m 2^k
 * with m <= 10 (96 and 128 qualify, 100 does not); otherwise PHZ_E_INVALID.
 * phz_set_options applies the same rule to a new mg_levels.  mat: base
 * material (Sec. 2.3), copied.  opt: NULL for the defaults, copied.  stream
 * is a hipStream_t (NULL: the library creates its own and destroys it in
 * phz_destroy).  alloc (may be NULL: hipMalloc and hipFree) supplies every
 * device workspace of the context, copied; the callbacks' user pointer must
 * stay valid until phz_destroy returns.  On success *out owns device
 * workspaces sized for N, nine loads and the chosen restart length; on
 * failure *out is NULL and everything allocated is returned. */
int phz_create(int nx, int ny, int nz, const phz_material* mat, const phz_options* opt,
               void* stream, const phz_allocator* alloc, phz_ctx** out);
/* Wait for the context's stream, return every workspace (through the
 * allocator given to phz_create, if any) and free the context.  NULL is a
 * no-op. */
void phz_destroy(phz_ctx* ctx);
/* Text of the last error on ctx (owned by ctx, valid until its next call);
 * with ctx = NULL, of the calling thread's last failing call that takes no
 * context (phz_hj_step_noalloc). */
const char* phz_last_error(const phz_ctx* ctx);
/* Static name of a status code. */
const char* phz_strerror(int status);
/* Replace the options of an existing context (workspaces are re-sized). */
int phz_set_options(phz_ctx* ctx, const phz_options* opt);

/* Geometry.  phi: [N^3] nodal level set (Sec. 2.1: phi < 0 solid, phi > 0
 * void); the element densities follow by the smoothed Heaviside of Sec. 2.6
 * (header comment).  rho: [N^3] per-element density in [0, 1] (Sec. 2.6's
 * smoothed density given directly).  Host, or (on_device) device memory of
 * the context's device; read before the call returns.  NaN/Inf ->
 * PHZ_E_NAN; a density outside [0, 1] -> PHZ_E_INVALID. */
int phz_set_levelset(phz_ctx* ctx, const double* phi, int on_device);
int phz_set_density(phz_ctx* ctx, const double* rho, int on_device);
/* Per-element ersatz scale s_e = eps_v + (1 - eps_v) rho_e currently in use,
 * [N^3], host or device as above. */
int phz_get_scale(phz_ctx* ctx, double* s, int on_device);

/* Solve the nine cell problems of Sec. 2.2 for the current geometry with
 * the configured solver (Sec. 2.5, default SCP-GMRES of Sec. 2.5.3) and
 * precision form, and reduce to the effective tensors.  PHZ_NOT_CONVERGED:
 * max_iters (or max_refine) ran out before every load reached rtol; the
 * tensors, histories and stats are still written.  PHZ_E_STATE without a
 * geometry. */
int phz_solve(phz_ctx* ctx);

/* Effective tensors of the last solve (Sec. 2.2's homogenised C^H, e^H,
 * kappa^H: cell averages of stress and electric displacement over the nine
 * cell solutions), SI, host buffers.  Any pointer may be NULL.  PHZ_E_STATE
 * before a solve. */
int phz_get_effective(phz_ctx* ctx, double CH[36], double eH[18], double kH[9]);
/* The same as the non-dimensional 9x9 matrix M^H = [[C, -e^T], [-e, -kappa]]
 * (row-major, host): flux form (cell average, Sec. 2.2) and energy form
 * (the solutions' energy pairing, equal at convergence). */
int phz_get_effective_nd(phz_ctx* ctx, double MH[81], double MH_energy[81]);
/* Per-load convergence history of the last solve (the residual histories
 * behind the iteration counts of Table 1): relative residual estimates of
 * every GMRES iteration, with the true relative residual ||b - calA x|| /
 * ||b|| at each restart and at exit.  load in [0, 9) (Voigt order, then the
 * electric fields).  Writes min(cap, available) values to buf (host; may be
 * NULL when cap = 0) and the available count to *len. */
int phz_get_history(phz_ctx* ctx, int load, double* buf, int cap, int* len);
/* Solver statistics of the last solve (Table 1's quantities: outer
 * iterations, restarts, refinement steps, inner iterations of inexact block
 * maps; final true residuals; set-up and solve times; the kernels chosen).
 * st: host. */
int phz_get_stats(phz_ctx* ctx, phz_stats* st);
/* Fluctuation solution X of the nine cell problems of Sec. 2.2 (the
 * periodic parts of displacement and potential), [N^3][4][9]
 * non-dimensional, zero mean per field.  X: host or (on_device) device
 * memory of 36 N^3 doubles, written (device: on the context's stream, then
 * synchronised).  PHZ_E_STATE before a solve. */
int phz_get_solution(phz_ctx* ctx, double* X, int on_device);
/* Warm start for the next solve, same layout as phz_get_solution (read
 * before the call returns); NULL clears it. */
int phz_set_initial_guess(phz_ctx* ctx, const double* X, int on_device);
/* Load vectors of the nine cell problems (Sec. 2.2: the weak form's
 * right-hand side for unit macroscopic strains and fields)
 * b = -sum_e s_e F0 e_L (with PHZ_SMOOTH_QP -sum_e sum_p s_ep F0_p e_L),
 * [N^3][4][9] non-dimensional, host or device as phz_get_solution.
 * PHZ_E_STATE without a geometry. */
int phz_get_rhs(phz_ctx* ctx, double* b, int on_device);

/* Figures of merit (Sec. 2.3) of SI tensors and their gradients with respect
 * to every entry of C (36), e (18), kappa (9).  Gradient pointers may be
 * NULL.  Pure function: no context. */
int phz_foms(const double CH[36], const double eH[18], const double kH[9],
             phz_foms_t* out, const char* grad_of,
             double gC[36], double ge[18], double gk[9]);

/* Sensitivities of J with respect to the per-element density, given
 * gC = dJ/dC^H, ge = dJ/de^H, gk = dJ/dkappa^H (SI).  Uses the last solve:
 * dJ/drho_e = (1 - eps_v) <W, G_e>, G_e[K, L] = element energy of the
 * fields e_K + B x^K and e_L + B x^L.  grad_rho: [N^3].  grad_phi (may be
 * NULL): [N^3] chain rule through the smoothed Heaviside (requires a level
 * set given by phz_set_levelset).  With PHZ_SMOOTH_QP the same per Gauss
 * point (G_ep, the point's share of the element energy): grad_rho[e] is the
 * sum over the element's points, grad_phi goes through the point densities. */
int phz_backward(phz_ctx* ctx, const double gC[36], const double ge[18],
                 const double gk[9], double* grad_rho, double* grad_phi,
                 int on_device);

/* One first-order Godunov step of phi_t + v |grad phi| = 0 (Sec. 2.1) on
 * the context's level set, dt = cfl * h.  velocity: [N^3] nodal values, or
 * NULL to use the nodal mean of the last phz_backward's dJ/drho normalised
 * to max |v| = 1.  The stepped level set becomes the context's geometry and
 * is written to phi_out ([N^3], may be NULL). */
int phz_hj_step(phz_ctx* ctx, const double* velocity, double cfl,
                double* phi_out, int on_device);

/* phz_hj_step's step from the last backward, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): no context, nothing allocated, nothing
 * synchronised.  phi (device, [N^3] nodal level set), grad_rho (device,
 * [N^3], an element density gradient such as phz_backward's), phi_out
 * (device, [N^3], not phi): phi_out = one Godunov step of phi with the nodal
 * velocity v_n = mean of grad_rho over the 8 elements around node n,
 * normalised to max |v| = 1, dt = cfl / n; the same kernels as phz_hj_step.
 * Enqueued on `stream` (a hipStream_t, NULL the default stream) of the
 * current device; the caller orders later work on it.  Working memory is a
 * fixed per-device scratch array of the library (16 MiB plus 8 KiB, held
 * until the process ends), so n is at most 128 (larger: PHZ_E_INVALID,
 * described by phz_last_error(NULL)); calls that overlap on one GPU (other
 * streams or threads) race on that scratch and must be serialised by the
 * caller. */
int phz_hj_step_noalloc(int n, const double* phi, const double* grad_rho, double cfl, double* phi_out,
                        void* stream);

/* ---- the optimisation loop around the solve (Sec. 2.1, Sec. 2.6) ---- */

/* Reinitialise the context's level set towards a signed distance (Sec. 2.6:
 * a standard first-order scheme): `steps` pseudo-time steps of
 * phi_t + S(phi0) (|grad phi| - 1) = 0 with the HJ step's first-order Godunov
 * upwinding, dtau = cfl * h.  subcell = 0: S = phi0 / sqrt(phi0^2 + h^2)
 * everywhere.  subcell = 1: the subcell fix of Russo and Smereka (J. Comput.
 * Phys. 163, 2000): S = sign(phi0), and a node whose phi0 changes sign towards
 * one of its six neighbours (or is 0) relaxes towards D = phi0 / |grad phi0|,
 * phi <- phi - (dtau / h)(sign(phi0) |phi| - D), |grad phi0| taking per
 * direction the largest of the central and one-sided differences; the zero
 * level set then stays in place instead of moving by a fraction of h per call.
 * The result becomes the geometry and is written to phi_out ([N^3], may be
 * NULL).  steps < 0, cfl <= 0 or subcell outside {0, 1}: PHZ_E_INVALID. */
int phz_reinit(phz_ctx* ctx, int steps, double cfl, int subcell, double* phi_out, int on_device);
/* Chain rule of the density map rho_e = 1 - H(mean of phi over element e)
 * (Sec. 2.1, Sec. 2.6 smoothing): grad_phi[N^3] = dJ/dphi from any element
 * gradient grad_rho[N^3] (e.g. 1/N^3 for the volume). */
int phz_levelset_gradient(phz_ctx* ctx, const double* grad_rho, double* grad_phi, int on_device);
/* Riesz representatives in the Hilbert space of the velocity extension:
 * g = H^-1 j for ncol (<= 9) device node columns [ncol][N^3], with
 * H = alpha^2 K + M the trilinear finite-element Laplace and mass matrices of
 * the periodic grid (alpha: length scale, cell units).  Chebyshev iteration
 * on H's exact extreme eigenvalues (constant coefficients: the extremes of its
 * symbol over the grid frequencies), run for the step count whose bound
 * 2 rho^k reaches a relative residual of 1e-12, with no host synchronisation
 * inside; *iters (may be NULL) gets the count (114 for alpha = 4h; about
 * 28 alpha / h for large alpha).  An alpha needing more than 20000 steps
 * (alpha above about 700 h) returns PHZ_E_INVALID.  j and g must not
 * overlap. */
int phz_riesz(phz_ctx* ctx, int ncol, double alpha, const double* j, double* g, int* iters);
/* Velocity of one constrained optimisation step by projection in that
 * Hilbert space (the paper uses a Hilbertian projection method for its
 * equality constraints).  j_obj[N^3] = -dJ/dphi (J to be increased),
 * j_cons[i][N^3] = -dC_i/dphi, viol[i] = current relative violations
 * (host), i < m <= 8.  With g = H^-1 j, G_ik = j_i . g_k:
 *   theta_J = g_0 - sum_i g_i (G^-1 b)_i,  b_k = j_k . g_0,
 *   theta_C = -sum_i g_i (G^-1 viol)_i,
 *   v = w theta_J / max|theta_J| + gamma / (cfl h) theta_C, scaled to
 *   max|v| <= 1,
 * so that an HJ step of cfl moves the boundary by up to w cfl h along the
 * objective's direction with the constraints' first-order changes removed,
 * and removes a fraction gamma of each violation to first order.  w =
 * obj_weight in [0, 1] (1: the full step; a step control may lower it).
 * alpha <= 0 selects 4h.  Vectors on the host or (on_device) the device. */
int phz_hpm_velocity(phz_ctx* ctx, int m, const double* j_obj, const double* const* j_cons,
                     const double* viol, double alpha, double cfl, double gamma, double obj_weight,
                     double* v_out, int on_device);

/* Low-level operator apply on the current geometry: y = calA_block x for
 * nrhs in {1, 9} columns, device pointers.  These low-level entry points use
 * the library's internal structure-of-arrays layout [field][load][N^3]
 * (one contiguous column of node values per (field, load)).
 * precision PHZ_FP64 (double buffers), PHZ_FP32_IR (float buffers, float32
 * gather kernel) or PHZ_BF16X3_IR (float buffers, nrhs = 9, the split-BF16
 * element contraction with the context's bf16_terms and elem_tile; N must be
 * a multiple of the tile). */
int phz_apply(phz_ctx* ctx, int op, int nrhs, int precision,
              const void* x, void* y);
/* Apply the SCP preconditioner z = P^-1 r (device, [4][nrhs][N^3], float64),
 * building it for the current geometry if needed. */
int phz_precondition(phz_ctx* ctx, int nrhs, const double* r, double* z);
/* One Arnoldi orthogonalisation of the GMRES step (Sec. 2.5's GMRES, its
 * Gram-Schmidt kernels and the reorth_tol rule) on caller data: w (device,
 * [4][9][N^3], float64 for PHZ_FP64, float32 for PHZ_FP32_IR) is
 * orthogonalised in place against the nvec (1 .. 33) vectors of V (device,
 * nvec x [4][9][N^3], contiguous), column by column of the nine loads.  h
 * (host, [nvec][9]) gets the projection coefficients (both passes summed),
 * nrm2 (host, [9]) |w|^2 of the result, second_pass (host, [9]) 1 where the
 * second pass ran.  w is not normalised.  A test hook of the solver's
 * internals. */
int phz_orthogonalize(phz_ctx* ctx, int precision, int nvec, const void* V, void* w, double* h,
                      double* nrm2, int* second_pass);
/* Galerkin coarse operator of multigrid level >= 1 applied to x (device):
 * block PHZ_OP_A ([3][nrhs][nc]) or PHZ_OP_SBAR ([nrhs][nc]).  precision
 * PHZ_FP64 (double buffers, the FP64 stencils) or PHZ_FP32_IR (float buffers,
 * the float32 stencils of a context in a float form, and for nrhs = 9 the
 * kernel the context chose for that level, coarse_kernel); PHZ_E_STATE if a
 * float apply is asked of an FP64 context. */
int phz_coarse_apply(phz_ctx* ctx, int level, int op, int nrhs, int precision,
                     const void* x, void* y);

/* Per-kernel timing (measurement support, not part of the method).  With
 * timing enabled (enable = 1), every operator launch (fine
 * blocks, coarse levels), every SCP preconditioner application and every
 * Arnoldi orthogonalisation of later calls is bracketed by HIP events on the
 * context's stream; enable = 2 brackets the fine-level operator launches
 * only (fewer events, so less drain between launches).  Each bracket drains
 * the stream between launches, so timed runs are a few per cent slower.
 * Enabling (or disabling, enable = 0) clears the totals.
 * phz_get_kernel_timing writes one line "name count total_ms" per kernel
 * class into buf (NUL-terminated, truncated to cap) and the full length to
 * *len.  Names: fine_{full,A,B,S}_k{1,9}_f{64,32} (suffix _cheby for the
 * launches that fuse a Chebyshev smoothing step), coarse_{A,S}_f{64,32},
 * coarse_tiled_{A,S}_f32 (the LDS-tiled coarse apply),
 * precond_f{64,32}, arnoldi_cgs2_f{64,32}. */
int phz_kernel_timing(phz_ctx* ctx, int enable);
int phz_get_kernel_timing(phz_ctx* ctx, char* buf, int cap, int* len);

#ifdef __cplusplus
}
#endif
#endif /* PIEZOHOM_H */
