/*
 * fsic_oracle.h -- plain FP64 CPU oracle for the real-space FLOSIC
 * self-interaction-correction path (Diaz et al., arXiv 2108.01186).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a slow, obviously correct definition.  Only the test suite, the
 * package smoke check and the CPU-baseline leg of the benchmark may load or
 * call it.  It shares no code, header, table or constant generator with the
 * HIP path, and the HIP path never links or calls it.
 *
 * Conventions (all functions):
 *   - Hartree atomic units (Bohr, Hartree).
 *   - A grid is n[0] x n[1] x n[2] nodes (x, y, z); node (i, j, k) sits at
 *     origin + h*(i, j, k).  Fields are stored C-order with x fastest:
 *     index = (k*n[1] + j)*n[0] + i.  M = n[0]*n[1]*n[2].
 *   - Integrals use the trapezoid weight dV = h^3 on every node (boundary
 *     values live in ghost layers outside the box).
 *   - Every pointer is host memory owned by the caller.
 *   - Functions return 0 on success and a negative code on bad arguments
 *     (-1), an FOD whose interpolation stencil leaves the grid (-2), an FOD
 *     in vacuum (-3), a singular overlap matrix (-4), or no CG convergence
 *     (-5, results are still written).
 */
#ifndef FSIC_ORACLE_H
#define FSIC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* 2p-th order central second-derivative coefficients c[0..p] on unit
 * spacing: f''(x) ~ sum_{k=-p..p} c[|k|] f(x + k). */
int orc_fd_coeffs(int p, double *c);

/* Lu = L u with the 2p-th order star Laplacian and zero Dirichlet ghosts. */
int orc_apply_laplacian(const int *n, double h, int p, const double *u, double *Lu);

/* Kohn-Sham Hamiltonian of count orbitals: out = -1/2 L psi + v psi (L as
 * above, zero Dirichlet values; v: one [M] potential for all orbitals). */
int orc_hamiltonian(const int *n, double h, int p, int count, const double *psi,
                    const double *v, double *out);

/* Real orthonormal spherical harmonics times r^l ("regular solid
 * harmonics") at (x, y, z): out[l*l + l + m] = r^l Y_lm, m = -l..l. */
int orc_solid_harmonics(int lmax, double x, double y, double z, double *out);

/* Multipole moments Q_lm = dV sum_r rho(r) |r-c|^l Y_lm about the box
 * centre c; Q has (lmax+1)^2 entries. */
int orc_multipole_moments(const int *n, double h, const double *origin, int lmax,
                          const double *rho, double *Q);

/* Exterior multipole potential sum_lm 4pi/(2l+1) Q_lm Y_lm / |r-c|^(l+1) at one point. */
double orc_multipole_potential(const int *n, double h, const double *origin, int lmax,
                               const double *Q, double x, double y, double z);

/* Hartree potential of rho: -L v = 4 pi rho with Dirichlet values from the
 * multipole expansion on the p ghost layers of each face; CG from v = 0 to
 * ||b + L v|| / ||b|| <= tol.  iters / relres may be NULL. */
int orc_poisson(const int *n, double h, const double *origin, int p, int lmax,
                const double *rho, double tol, int maxit, double *v,
                int *iters, double *relres);

/* Transpose of the map rho -> v above, applied to rho: out = A^T rho. */
int orc_poisson_transpose(const int *n, double h, const double *origin, int p, int lmax,
                          const double *rho, double tol, int maxit, double *out,
                          int *iters, double *relres);

/* Fully spin-polarised LSDA at one density: Slater exchange and PW92
 * correlation energy per particle and potential (zeta = 1). */
void orc_xc_pol(double rho, double rho_floor, double *ex, double *ec, double *vx, double *vc);

/* Tensor cubic (4-point Lagrange) interpolation of N fields at point a:
 * u[N] values, du[N*3] gradient of the interpolant (du may be NULL). */
int orc_interp(const int *n, double h, const double *origin, int N, const double *psi,
               const double *a, double *u, double *du);

/* Per-node gradient of one field by first differences along each axis
 * (Sec. II.B): central inside, forward at the first node, backward at the
 * last.  g[3*M] = x, y, z components; every n[d] >= 2. */
int orc_grid_gradient(const int *n, double h, const double *f, double *g);

/* Values u[N] by cubic interpolation and gradients du[N*3] by interpolating
 * orc_grid_gradient's per-node gradient with the same cubic scheme
 * (Sec. II.B's construction of grad psi at the FODs). */
int orc_interp_fdgrad(const int *n, double h, const double *origin, int N, const double *psi,
                      const double *a, double *u, double *du);

/* Cyclic Jacobi eigen-decomposition of a symmetric N x N matrix:
 * A = U diag(lam) U^T, U column j = eigenvector j (row-major U[i*N+j]). */
int orc_jacobi_eig(int N, const double *A, double *lam, double *U);

/* Energy terms of one orbital density rho[M] (Eq. 1): U = 1/2 dV rho.v_H[rho]
 * (Poisson problem as in orc_poisson) and X = dV sum rho (eps_x + eps_c) at
 * full spin polarisation.  iters / relres may be NULL. */
int orc_orbital_terms(const int *n, double h, const double *origin, int p, int lmax,
                      double tol, int maxit, double rho_floor, const double *rho,
                      double *U, double *X, int *iters, double *relres);

/* One spin channel of the SIC path (Fermi orbitals, Loewdin, Poisson,
 * LSDA, Slater average).  Outputs other than e_spin may be NULL.
 *   e_spin = -sum_i (U_i + X_i)
 *   vsic[M] = s * sum_i rho_i V_i / sum_i rho_i, V_i = -(v_i + vxc_i)
 * T, S, Z are N x N; phi and v are N x M; iters, relres are N. */
int orc_sic_spin(const int *n, double h, const double *origin, int p, int lmax,
                 double tol, int maxit, double vscale, double rho_floor,
                 int N, const double *psi, const double *fod,
                 double *e_spin, double *U, double *X, double *vsic,
                 double *T, double *S, double *Z, double *phi, double *v,
                 int *iters, double *relres);

/* Gradient dE_SIC/da (N x 3) of one spin channel's SIC energy, tangent
 * mode over the 3N FOD coordinates. */
int orc_sic_grad_spin(const int *n, double h, const double *origin, int p, int lmax,
                      double tol, int maxit, double rho_floor,
                      int N, const double *psi, const double *fod, double *dEda);

/* Same gradient with a choice of ingredients:
 *   gmode 0: grad psi(a_i) = derivative of the cubic interpolant;
 *   gmode 1: grad psi(a_i) = interpolated per-node differences (Sec. II.B);
 *   form 0:  exact derivative of the discrete E_SIC (adjoint Poisson solves);
 *   form 1:  Eq. 9 with eps_kl = <phi_l|V_k|phi_k>, V_k = -(v_k + vxc_k) (Eq. 5),
 *            which treats the Poisson map as symmetric (no adjoint solves). */
int orc_sic_grad_spin_mode(const int *n, double h, const double *origin, int p, int lmax,
                           double tol, int maxit, double rho_floor,
                           int N, const double *psi, const double *fod, int gmode, int form,
                           double *dEda);

/* Fermi-Loewdin orbitals only (steps (a) and (b) of orc_sic_spin):
 * phi[N*M]; T, S, Z may be NULL. */
int orc_flo_spin(const int *n, double h, const double *origin, double rho_floor, int N,
                 const double *psi, const double *fod, double *phi, double *T, double *S,
                 double *Z);

/* OpenMP threads the oracle uses. */
int orc_num_threads(void);
/* threads of the parallel loops from here on (n > 0; the default is OpenMP's) */
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
