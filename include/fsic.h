/*
 * fsic.h -- C ABI of the MI355X (gfx950) library for the real-space FLOSIC
 * self-interaction-correction path of Diaz, Suryanarayana, Xu, Baruah, Pask
 * and Zope, "Implementation of Perdew-Zunger self-interaction correction in
 * real space using Fermi-Loewdin orbitals" (arXiv 2108.01186).
 *
 * Given Kohn-Sham orbitals on a uniform grid and Fermi-orbital descriptors
 * (FODs), the library computes per spin channel
 *   (a) the Fermi orbitals F_i = sum_a psi_a(a_i) psi_a / sqrt(rho(a_i))
 *       (Eq. 6-8; psi at the FODs by cubic interpolation, Sec. II.B),
 *   (b) their Loewdin orthonormalisation phi = S^{-1/2} F, S = dV F F^T
 *       (Sec. I.B),
 *   (c) one finite-difference Poisson solve per FLO density rho_i = phi_i^2
 *       (high-order centred Laplacian, Dirichlet values from a multipole
 *       expansion, Sec. II.A), solved by conjugate gradients,
 *   (d) the LSDA (Slater exchange + PW92 correlation) energy and potential
 *       of each rho_i at full spin polarisation (Eq. 1, Sec. III),
 *   (e) the generalised-Slater average of the orbital SIC potentials
 *       V_SIC = s sum_i rho_i V_i / sum_i rho_i, V_i = -(v_H[rho_i] +
 *       v_xc[rho_i, 0]) (Eq. 5, 13; scaled variant of Sec. II.C), and the
 *       energy E_SIC = -sum_i (U[rho_i] + E_xc[rho_i, 0]) (Eq. 1),
 * and, on request, the exact gradient dE_SIC/da_i of the discrete energy
 * (the FOD forces of Eq. 9-11 are its negative).
 *
 * Units: Hartree atomic units (Bohr, Hartree).  Grids: node (i, j, k) sits
 * at origin + h (i, j, k); fields are C-order with x fastest,
 * index = (k n[1] + j) n[0] + i, M = n[0] n[1] n[2].  Integrals use the
 * trapezoid weight dV = h^3 on every node.  All floating-point data are
 * IEEE binary64 unless a function says otherwise.
 *
 * Ownership: the caller owns every buffer it passes.  Device pointers must
 * be device memory of the GPU current when the context was created; host
 * pointers are ordinary host memory.  Nothing is retained after a call
 * returns, except that the forward pass keeps (inside the context) what the
 * backward pass needs until the next forward pass or fsic_destroy.
 *
 * Errors: every entry point returns an fsic_status; nothing is thrown
 * across the ABI.  Arguments are validated on the host before anything is
 * launched.  Conditions found on the device (an FOD in vacuum, a singular
 * overlap, no convergence) are reported when the call returns.
 * fsic_last_error() gives a human-readable detail of the last failure.
 *
 * Calls on one context are serialised by the caller; a context is bound to
 * the HIP stream given at creation (NULL = the default stream) and every
 * entry point returns only after its work on that stream has completed.
 */
#ifndef FSIC_H
#define FSIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsic_ctx fsic_ctx;

typedef enum {
    FSIC_OK = 0,
    FSIC_EINVAL = 1,      /* bad argument, size, option or non-finite input */
    FSIC_ENOMEM = 2,      /* device or host allocation failed */
    FSIC_EHIP = 3,        /* a HIP runtime call failed (detail in fsic_last_error) */
    FSIC_ENONORTHO = 4,   /* input orbitals not orthonormal: max|dV psi psi^T - I| > 1e-8 */
    FSIC_EVACUUM = 5,     /* rho(a_i) <= rho_floor: the division of Eq. 8 is undefined */
    FSIC_EBOUNDARY = 6,   /* an FOD's 4-node interpolation stencil leaves the grid */
    FSIC_ESINGULAR = 7,   /* smallest eigenvalue of S below s_eig_floor (linear dependence) */
    FSIC_ENOCONV = 8,     /* a Poisson solve missed tol within max_iter (results still written) */
    FSIC_ENOTAPE = 9      /* backward without a forward pass run with FSIC_KEEP_TAPE */
} fsic_status;

/* Precision of the Poisson solves (c).  FSIC_FP64: FP64 conjugate
 * gradients.  FSIC_MIXED: FP32 stencil and CG sweeps whose accumulated
 * solution is corrected in FP64 against the FP64 residual until the same
 * FP64 relative-residual tolerance is met; overlap, S^{-1/2}, residuals and
 * energies stay FP64. */
enum { FSIC_FP64 = 0, FSIC_MIXED = 1 };

/* Poisson solver (c) for -L v = 4 pi rho + boundary term:
 *   FSIC_CG   plain conjugate gradients;
 *   FSIC_PCG  conjugate gradients preconditioned by the inverse of the same
 *             stencil with odd-reflection faces, applied with type-I sine
 *             transforms along each axis (a few iterations instead of
 *             hundreds); a batch with a grid axis above 256 nodes is solved
 *             with plain CG instead.  The default.
 *   FSIC_AAR  alternating Anderson-Richardson (the solver of the paper's
 *             real-space code, Sec. II.A) with the same preconditioner:
 *             Richardson steps x += f, f = M^{-1}(b + L x), and every third
 *             iteration an Anderson extrapolation over the last 7
 *             differences of x and f (weights 1 and 1).  Needs precision
 *             FSIC_FP64 (the iterate and residual are FP64, f is FP32) and
 *             12 extra bytes per orbital node per history column (84 B).
 *             Batches with an axis above 256 nodes use plain CG.
 * All stop on the same FP64 relative residual. */
enum { FSIC_CG = 0, FSIC_PCG = 1, FSIC_AAR = 2 };

/* option flags */
#define FSIC_WANT_VSIC       1u  /* write V_SIC into fsic_system.vsic[] */
#define FSIC_KEEP_TAPE       2u  /* keep what fsic_backward needs */
#define FSIC_ALLOW_NONORTHO  4u  /* accept non-orthonormal psi (S = T G T^T is exact anyway) */
#define FSIC_PROFILE         8u  /* time sampled CG launches with HIP events (fsic_stats.sweep_*) */
#define FSIC_GRAPHS         32u  /* FSIC_PCG with FSIC_MIXED: capture each restart cycle (its CG
                                    iterations and the FP64 residual check) as a HIP graph once per
                                    batch layout and buffers, and replay it; ignored with FSIC_PROFILE */
#define FSIC_FP32_ORBITALS  16u  /* Fermi-Loewdin orbitals phi = (Z T) psi from an fp32 GEMM on the
                                    matrix cores (fp32 operands and accumulation); costs about 1e-7
                                    relative in phi, more than the 1e-8 Ha energy budget allows */
#define FSIC_PAPER_GRADIENT 64u  /* forward pass: grad psi at each FOD by interpolating per-node first
                                    differences (central inside, one-sided at the first and last node),
                                    as Sec. II.B does, instead of differentiating the cubic interpolant;
                                    the gradient is then no longer that of the discrete E_SIC(a) */
#define FSIC_EQ9_FORCES    128u  /* backward pass: the FOD gradient in the form of Eq. 9 with
                                    eps_kl = <phi_l|V_k|phi_k>, V_k = -(v_k + vxc_k) (Eq. 5); it treats
                                    the Poisson map as symmetric, so no adjoint Poisson solves run
                                    (the boundary part of the map is the only difference) */
#define FSIC_DIRECT_BC     256u  /* forward pass with FSIC_KEEP_TAPE: solve each orbital's problem with
                                    its multipole boundary values directly.  Without it the forward
                                    pass solves the zero-boundary problems K w_i = 4 pi rho_i (the
                                    adjoint fields the FOD gradient needs, so fsic_backward runs no
                                    Poisson solve) and forms v_i = w_i + sum_lm Q_lm,i U_lm from the
                                    moments and a per-grid basis U of unit-moment boundary solutions
                                    (the map is linear in the boundary values); the basis is solved
                                    once per grid and context in FP64 to relative residual 1e-13 */

typedef struct {
    int32_t n[3];       /* nodes per axis, 8..4096, fewer than 2^29 nodes in all */
    double h;           /* spacing (Bohr), > 0 */
    double origin[3];   /* position of node (0, 0, 0) */
} fsic_grid;

typedef struct {
    int32_t fd_order;   /* even, 2..12: order of the central second difference; radius p = fd_order/2 */
    int32_t lmax;       /* multipole order of the Dirichlet values, 0..8 */
    int32_t solver;     /* FSIC_CG | FSIC_PCG | FSIC_AAR */
    int32_t precision;  /* FSIC_FP64 | FSIC_MIXED */
    double  tol;        /* relative FP64 residual ||b + L v|| / ||b|| to reach, (0, 1) */
    int32_t max_iter;   /* CG iteration cap per solve, >= 1 */
    double  vsic_scale; /* s: scales V_SIC only, never E_SIC or the gradient */
    double  rho_floor;  /* densities <= floor give zero XC and zero V_SIC; FOD vacuum test */
    double  s_eig_floor;/* smallest admissible eigenvalue of the FO overlap S */
    uint32_t flags;     /* FSIC_WANT_VSIC | FSIC_KEEP_TAPE | FSIC_ALLOW_NONORTHO | FSIC_PROFILE |
                           FSIC_FP32_ORBITALS | FSIC_GRAPHS | FSIC_PAPER_GRADIENT | FSIC_EQ9_FORCES */
} fsic_opts;

/* One system: up to two spin channels on one grid. */
typedef struct {
    fsic_grid grid;
    int32_t nspin;            /* 1 or 2 */
    int32_t nocc[2];          /* orbitals (= FODs) per spin, 1..128 */
    const double *psi[2];     /* DEVICE, [nocc[s]][M]: occupied KS orbitals of spin s */
    const double *fod[2];     /* HOST, [nocc[s]][3]: FOD positions (Bohr) */
    double *vsic[2];          /* DEVICE, [M] or NULL: output V_SIC of spin s */
} fsic_system;

typedef struct {
    int32_t nsolves;          /* Poisson solves in the call (forward: sum of nocc) */
    int32_t max_iters;        /* largest number of CG sweeps that did work for one solve */
    int64_t total_iters;      /* CG sweeps that did work, summed over solves */
    int32_t outer_refinements;/* mixed precision: rounds of FP64 residual checks (each
                                 folds the FP32 correction into the FP64 solution) */
    double  max_relres;       /* largest final FP64 relative residual */
    double  cond_S_max;       /* largest condition number of any FO overlap S */
    double  min_rho_fod;      /* smallest rho(a_i) */
    double  max_nonortho;     /* max |dV psi psi^T - I| over channels */
    double  ms_phase[8];      /* host wall time per phase: 0 setup, 1 FO+Loewdin,
                                 2 boundary+RHS, 3 CG, 4 XC+average, 5 adjoint CG,
                                 6 adjoint rest, 7 total */
    /* with FSIC_PROFILE: HIP-event time, on the context's stream, of the CG
     * launches of every 16th iteration (k % 16 == 15; the environment
     * variable FSIC_PROFILE_EVERY changes the period, 1 = every launch), and
     * the algorithmic HBM bytes of exactly those launches (each array of an
     * active orbital read or written once per launch).  Sampling keeps the
     * events' own cost (a few microseconds per recorded launch) out of the
     * timed work. */
    int32_t sweep_launches;   /* sampled stencil sweeps (p = r + beta p, q = -L p) */
    int32_t update_launches;  /* sampled pointwise updates (x += alpha p, r -= alpha q) */
    double  sweep_ms, sweep_bytes;
    double  update_ms, update_bytes;
    /* FSIC_PCG with FSIC_PROFILE: iterations are sampled every other one, and
     * each sampled preconditioner application (three transform passes with
     * the in-plane pair fused, else five) is timed as one unit with its
     * algorithmic bytes (each array of an active orbital read or written
     * once per pass) and flops */
    int32_t precond_launches;
    double  precond_ms, precond_bytes, precond_flops;
    /* stencil shape of the CG sweeps: tiles of 32 x 8*stencil_cpt columns,
     * stencil_depth planes fetched ahead, z-chunks halved until a launch has
     * stencil_blocks blocks.  The first call for a given (device, precision,
     * order, grid sizes and orbital counts) times the candidate shapes on
     * the batch and keeps the fastest for the rest of the process (tune_ms:
     * time that took, 0 when the shape came from that cache or from
     * FSIC_STENCIL_CPT / FSIC_STENCIL_DEPTH / FSIC_STENCIL_BLOCKS, or
     * defaults under FSIC_AUTOTUNE=0). */
    int32_t stencil_cpt, stencil_depth;
    int64_t stencil_blocks;
    double  tune_ms;
    /* FSIC_PCG in FSIC_MIXED with FSIC_PROFILE: the FP64 residual pass that
     * closes each restart cycle (every cycle but the first is sampled) */
    int32_t resid_launches;
    double  resid_ms, resid_bytes;
    /* FSIC_GRAPHS: restart-cycle graphs captured so far by this context
     * (a replayed graph is not counted again) */
    int32_t graph_captures;
    /* FSIC_PCG / FSIC_AAR: layout of the sine-transform preconditioner, bits
     * 1 fused in-plane passes (else five per-axis passes), 2 two fused-pass
     * blocks per compute unit, 4 two-block z pass, 8 inverse pass reads p_old
     * before its products, plus 16 x the transform variant (1-3; 0: solved
     * without the preconditioner).  The first call for a given (device,
     * precision, order, solver, grid sizes and orbital counts) times every
     * combination of the open choices on the batch and keeps the fastest for
     * the process (precond_tune_ms: time that took, 0 when cached, when
     * nothing was open, or under FSIC_AUTOTUNE=0). */
    int32_t precond_layout;
    double  precond_tune_ms;
    /* Poisson problems whose solutions this call produced: the CG solves
     * (nsolves) plus, on a forward pass that formed the multipole-boundary
     * potentials from the zero-boundary (adjoint) solutions and the boundary
     * basis (FSIC_KEEP_TAPE without FSIC_DIRECT_BC or FSIC_EQ9_FORCES), those
     * potentials too; fsic_backward then reports 0 for both.  basis_solves,
     * basis_ms: unit-moment boundary solutions solved in this call for grids
     * new to the context, and the time they took */
    int32_t npoisson;
    int32_t basis_solves;
    double  basis_ms;
} fsic_stats;

/* Fills *o with the defaults: fd_order 12, lmax 6, FSIC_PCG, FP64, tol 1e-10,
 * max_iter 20000, vsic_scale 1, rho_floor 1e-30, s_eig_floor 1e-12,
 * flags FSIC_WANT_VSIC. */
fsic_status fsic_default_opts(fsic_opts *o);

/* Creates a context bound to hip_stream (a hipStream_t, NULL = default
 * stream) on the current device.  *ctx receives the context. */
fsic_status fsic_create(fsic_ctx **ctx, const fsic_opts *opts, void *hip_stream);

/* Changes the options of an existing context (same validation as create). */
fsic_status fsic_set_opts(fsic_ctx *ctx, const fsic_opts *opts);

/* Forward pass over nsys systems (Eq. 1, 5-8, 13; Sec. I.B, II.A-C).
 *   e_sic: HOST [nsys], E_SIC of each system summed over its spins (Hartree).
 *   U, X:  HOST or NULL, [sum over systems and spins of nocc]: the Hartree
 *          self-energy U[rho_i] and E_xc[rho_i, 0] of every FLO density, in
 *          system, spin, orbital order.
 *   st:    HOST or NULL, statistics of the call.
 * V_SIC is written to sys[k].vsic[s] when FSIC_WANT_VSIC is set and the
 * pointer is non-NULL.  Returns FSIC_ENOCONV (with every output written)
 * when some solve missed tol. */
fsic_status fsic_forward(fsic_ctx *ctx, int32_t nsys, const fsic_system *sys,
                         double *e_sic, double *U, double *X, fsic_stats *st);

/* Backward pass of the last forward pass (which needs FSIC_KEEP_TAPE):
 * dE_da[k] (HOST, [nspin][nocc][3] of system k) receives
 * grad_e[k] * dE_SIC/da for system k (Eq. 9-11 in exact discrete form:
 * one adjoint Poisson solve per orbital, reverse mode through the Loewdin
 * step, the Fermi-orbital construction and the cubic interpolation).
 * With FSIC_EQ9_FORCES set at this call, Eq. 9 with the orbital SIC
 * potentials instead (no adjoint solves); with FSIC_PAPER_GRADIENT set at
 * the forward call, grad psi at the FODs comes from per-node differences.
 * grad_e: HOST [nsys], NULL means all ones.  The input orbitals of the
 * forward pass must still be valid and unchanged. */
fsic_status fsic_backward(fsic_ctx *ctx, const double *grad_e, double *const *dE_da,
                          fsic_stats *st);

/* fsic_forward and then fsic_backward in one call, for callers that want
 * E_SIC and the FOD gradient of the same FODs (the step of an FOD
 * optimisation).  Needs FSIC_KEEP_TAPE.  Without FSIC_EQ9_FORCES and
 * FSIC_DIRECT_BC the backward pass's device work (it runs no Poisson solve:
 * the forward pass solved the adjoint problems) is enqueued behind the
 * forward pass's before the host waits, so the two share one
 * synchronisation; otherwise the two run one after the other.  Arguments
 * as in the two calls (grad_e may be NULL: 1 per system; st_fwd and st_bwd
 * may be NULL); the results and the tape left behind are those of the two
 * calls.  An error of the forward pass is returned before any gradient is
 * written. */
fsic_status fsic_forward_backward(fsic_ctx *ctx, int32_t nsys, const fsic_system *sys, double *e_sic,
                                  double *U, double *X, const double *grad_e, double *const *dE_da,
                                  fsic_stats *st_fwd, fsic_stats *st_bwd);

const char *fsic_status_string(fsic_status s);
const char *fsic_last_error(const fsic_ctx *ctx);
void fsic_destroy(fsic_ctx *ctx);

/* ----------------------------------------------------------------------
 * Operator-level entry points (the same kernels the path runs), for
 * component checks.  All pointers are DEVICE memory unless stated; each
 * call is synchronous on the given stream (NULL = default stream).
 * -------------------------------------------------------------------- */

/* Lu[f] = L u[f] for count fields on grid n with spacing h: the
 * fd_order-th order centred star Laplacian (Sec. II.A), zero Dirichlet
 * ghosts.  u, Lu: [count][M] FP64; u and Lu must not overlap. */
fsic_status fsic_op_laplacian(const int32_t *n /* HOST [3] */, double h, int32_t fd_order,
                              int32_t count, const double *u, double *Lu, void *hip_stream);

/* FP32 variant of fsic_op_laplacian (the mixed-precision inner operator). */
fsic_status fsic_op_laplacian_f32(const int32_t *n, double h, int32_t fd_order,
                                  int32_t count, const float *u, float *Lu, void *hip_stream);

/* Pointwise fully polarised LSDA (Sec. III): for each of count densities,
 * eps_x, eps_c (energy per particle) and v_x, v_c (potentials); zero where
 * rho <= rho_floor.  Any output pointer may be NULL. */
fsic_status fsic_op_xc(int64_t count, const double *rho, double rho_floor, double *ex,
                       double *ec, double *vx, double *vc, void *hip_stream);

/* Kohn-Sham Hamiltonian applied to count orbitals (the step after this
 * path in the self-consistent cycle, Sec. II.C, where V_SIC enters the
 * local potential): out[f] = -1/2 L psi[f] + v psi[f], L the fd_order-th
 * order star Laplacian with zero Dirichlet values (Sec. II.A), v one [M]
 * potential (for instance v_KS + V_SIC of the orbitals' spin channel).
 * psi, out: [count][M] FP64, not overlapping; v: [M] FP64.  FSIC_EINVAL on
 * bad sizes. */
fsic_status fsic_op_hamiltonian(const int32_t *n /* HOST [3] */, double h, int32_t fd_order,
                                int32_t count, const double *psi, const double *v, double *out,
                                void *hip_stream);

/* Hartree potentials v[f] of count densities rho[f] on one grid: -L v =
 * 4 pi rho with multipole Dirichlet values of order lmax about the box
 * centre (Sec. II.A), solved to tol.  iters, relres: HOST [count] or NULL.
 * precision: FSIC_FP64 or FSIC_MIXED; solver: FSIC_CG or FSIC_PCG. */
fsic_status fsic_op_poisson(const fsic_grid *grid, int32_t fd_order, int32_t lmax,
                            int32_t count, const double *rho, double *v, double tol,
                            int32_t max_iter, int32_t precision, int32_t solver,
                            int32_t *iters, double *relres, void *hip_stream);

/* Inverse square root of count symmetric positive definite N x N matrices
 * (row-major, N <= 128) by parallel cyclic Jacobi on the device: Z =
 * U diag(lam)^{-1/2} U^T.  S, Z: [count][N][N]; lam: [count][N] or NULL. */
fsic_status fsic_op_invsqrt(int32_t N, int32_t count, const double *S, double *Z, double *lam,
                            void *hip_stream);

/* Cubic interpolation of N orbitals at K points (Sec. II.B): psi DEVICE
 * [N][M], pts HOST [K][3] (Bohr); u DEVICE [K][N] receives psi_a(p_k) and
 * du DEVICE [K][N][3] its gradient: fd_gradient = 0, the derivative of the
 * tensor cubic interpolant (4 nodes per axis); fd_gradient = 1, the same
 * interpolation applied to per-node first differences (central inside,
 * one-sided at the first and last node; 6 nodes per axis).  N <= 128.
 * FSIC_EBOUNDARY when a point's 4-node stencil leaves the grid (its cell
 * index floor((p - origin)/h) must lie in [1, n-3] on every axis). */
fsic_status fsic_op_interp(const fsic_grid *grid, int32_t N, int32_t K, const double *psi,
                           const double *pts, int32_t fd_gradient, double *u, double *du,
                           void *hip_stream);

/* Fermi-Loewdin orbitals of one spin channel (Eq. 6-8, Sec. I.B, II.B):
 * psi (DEVICE [N][M]) and FODs (HOST [N][3]) give, for every non-NULL
 * DEVICE output, T ([N][N], Eq. 8), G = dV psi psi^T ([N][N]), S = T G T^T
 * ([N][N], the FO overlap), Z = S^{-1/2} ([N][N]) and phi = Z T psi
 * ([N][M]).  Same validation and status codes as fsic_forward. */
fsic_status fsic_op_flo(const fsic_grid *grid, int32_t N, const double *psi, const double *fod,
                        double rho_floor, double *T, double *G, double *S, double *Z, double *phi,
                        void *hip_stream);

/* fsic_op_flo without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, outputs, validation
 * and status codes as fsic_op_flo.  Every intermediate (interpolated
 * values, the Gram partial tiles, the N x N matrices, the Jacobi work
 * space, the device status word) lives in one file-scope device array of
 * about 18 MiB that each GPU the library runs on holds until the process
 * ends; N <= 128 and any grid fit in it (larger N is rejected with
 * FSIC_EINVAL before any launch).  The call itself allocates nothing: no
 * hipMalloc, hipFree or allocating library routine.  All calls on one GPU
 * share that GPU's array and it keeps the last call's contents (the status
 * word is cleared at the start of each call), so calls that overlap on one
 * GPU race; serialise them.  Synchronous on the given stream. */
fsic_status fsic_op_flo_noalloc(const fsic_grid *grid, int32_t N, const double *psi,
                                const double *fod, double rho_floor, double *T, double *G,
                                double *S, double *Z, double *phi, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* FSIC_H */
