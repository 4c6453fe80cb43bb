/*
 * fsic_oracle.c -- plain FP64 CPU oracle for the real-space FLOSIC
 * self-interaction correction (Diaz, Suryanarayana, Xu, Baruah, Pask, Zope,
 * "Implementation of Perdew-Zunger self-interaction correction in real space
 * using Fermi-Loewdin orbitals", arXiv 2108.01186).
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg are the only callers.  Nothing here is shared
 * with the HIP path, and the HIP path never calls it.
 *
 * Every routine is the plain definition, written for a reader to check
 * against the paper by eye: no blocking, no fusion, no reordering beyond what
 * the definition states.  OpenMP only splits independent loops.
 *
 * Readings taken where the paper is silent (each listed in the design notes):
 *   - trapezoid weight h^3 on every node; all n^3 nodes are unknowns and the
 *     Dirichlet values sit in p ghost layers outside each face;
 *   - multipole expansion about the box centre, real orthonormal Y_lm;
 *   - "cubic interpolation" = tensor 4-point Lagrange cubic on nodes
 *     i0-1..i0+2, gradient = exact derivative of that interpolant;
 *   - occupations f = 1, spin-resolved FOD density;
 *   - LSDA at full polarisation: Slater exchange + PW92 correlation
 *     (original published parameter set for zeta = 1);
 *   - orbital SIC potential V_i = -(v_H[rho_i] + v_xc[rho_i, 0]), Slater
 *     average over sum_i rho_i, the scale factor applies to the potential
 *     only.
 *
 * Pins: every routine is checked by the CPU tests against closed forms,
 * invariants or brute force.  One partial exception: the PW92 fit constants
 * alpha1, beta3, beta4 (zeta = 1) are pinned only to the 0.5 % accuracy of
 * two other published fits of the same Monte Carlo data; their digits below
 * that are parity unpinned.
 */
#include "fsic_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EBADARG   (-1)
#define ORC_EBOUNDARY (-2)
#define ORC_EVACUUM   (-3)
#define ORC_ESINGULAR (-4)
#define ORC_ENOCONV   (-5)

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Grid helpers (Sec. II.A: uniform grid, trapezoidal rule)                  */
/* ------------------------------------------------------------------------ */

static long grid_size(const int *n) { return (long)n[0] * n[1] * n[2]; }

static void box_centre(const int *n, double h, const double *origin, double *c)
{
    for (int d = 0; d < 3; ++d) c[d] = origin[d] + 0.5 * h * (n[d] - 1);
}

/* ------------------------------------------------------------------------ */
/* Finite-difference Laplacian (Sec. II.A: high-order centred differences;   */
/* the Kronecker-sum Laplacian D(x)I(x)I + I(x)D(x)I + I(x)I(x)D)             */
/* ------------------------------------------------------------------------ */

/* Closed form of the 2p-th order central second derivative (Fornberg):
 *   c_k = 2 (-1)^(k+1) (p!)^2 / (k^2 (p-k)! (p+k)!),  c_0 = -2 sum_k c_k. */
int orc_fd_coeffs(int p, double *c)
{
    if (p < 1 || p > 16 || !c) return ORC_EBADARG;
    double sum = 0.0;
    for (int k = 1; k <= p; ++k) {
        /* (p!)^2 / ((p-k)! (p+k)!) = prod_{j=1..k} (p-k+j) / (p+j) */
        double ratio = 1.0;
        for (int j = 1; j <= k; ++j) ratio *= (double)(p - k + j) / (double)(p + j);
        double sign = (k % 2 == 1) ? 1.0 : -1.0;
        c[k] = 2.0 * sign * ratio / ((double)k * (double)k);
        sum += c[k];
    }
    c[0] = -2.0 * sum;
    return 0;
}

/* Padded field: n[d] + 2p per axis, interior node (i,j,k) at padded (i+p, j+p, k+p). */
typedef struct {
    int n[3], p, P[3];
} padded_t;

static padded_t make_padded(const int *n, int p)
{
    padded_t g;
    for (int d = 0; d < 3; ++d) { g.n[d] = n[d]; g.P[d] = n[d] + 2 * p; }
    g.p = p;
    return g;
}

static long pad_size(const padded_t *g) { return (long)g->P[0] * g->P[1] * g->P[2]; }

/* padded index of node (i,j,k) given in interior coordinates (may be negative) */
static long pidx(const padded_t *g, int i, int j, int k)
{
    return ((long)(k + g->p) * g->P[1] + (j + g->p)) * g->P[0] + (i + g->p);
}

/* out(node) = sum over the three axes of sum_{k=-p..p} c_|k| / h^2 * u(node + k e_axis),
 * evaluated at interior node (i,j,k); u is a padded field. */
static double lap_at(const padded_t *g, const double *c, double h, const double *u,
                     int i, int j, int k)
{
    double acc = 3.0 * c[0] * u[pidx(g, i, j, k)];
    for (int s = 1; s <= g->p; ++s) {
        acc += c[s] * (u[pidx(g, i + s, j, k)] + u[pidx(g, i - s, j, k)]);
        acc += c[s] * (u[pidx(g, i, j + s, k)] + u[pidx(g, i, j - s, k)]);
        acc += c[s] * (u[pidx(g, i, j, k + s)] + u[pidx(g, i, j, k - s)]);
    }
    return acc / (h * h);
}

/* Lu over the interior for a padded field u */
static void lap_padded(const padded_t *g, const double *c, double h, const double *u, double *Lu)
{
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                Lu[((long)k * ny + j) * nx + i] = lap_at(g, c, h, u, i, j, k);
}

static void scatter_interior(const padded_t *g, const double *u, double *up)
{
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                up[pidx(g, i, j, k)] = u[((long)k * ny + j) * nx + i];
}

int orc_apply_laplacian(const int *n, double h, int p, const double *u, double *Lu)
{
    if (!n || !u || !Lu || h <= 0 || n[0] < 1 || n[1] < 1 || n[2] < 1) return ORC_EBADARG;
    double c[17];
    if (orc_fd_coeffs(p, c)) return ORC_EBADARG;
    padded_t g = make_padded(n, p);
    double *up = calloc(pad_size(&g), sizeof(double));
    if (!up) return ORC_EBADARG;
    scatter_interior(&g, u, up);
    lap_padded(&g, c, h, up, Lu);
    free(up);
    return 0;
}

/* Kohn-Sham Hamiltonian applied to count orbitals (Sec. II.C: the SIC
 * potential enters the KS equations as a local term): out = -1/2 L psi +
 * v psi, zero Dirichlet values, v one field for all orbitals. */
int orc_hamiltonian(const int *n, double h, int p, int count, const double *psi,
                    const double *v, double *out)
{
    if (!n || !psi || !v || !out || count < 1) return ORC_EBADARG;
    const long M = grid_size(n);
    for (int f = 0; f < count; ++f) {
        int st = orc_apply_laplacian(n, h, p, psi + (long)f * M, out + (long)f * M);
        if (st) return st;
        for (long m = 0; m < M; ++m)
            out[(long)f * M + m] = -0.5 * out[(long)f * M + m] + v[m] * psi[(long)f * M + m];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Multipole expansion for the Dirichlet values (Sec. II.A, isolated case)   */
/* ------------------------------------------------------------------------ */

/* associated Legendre P_l^m(x), m >= 0, without the Condon-Shortley phase,
 * by the textbook three-term recurrence in l. */
static double assoc_legendre(int l, int m, double x)
{
    double somx2 = sqrt(fmax(0.0, (1.0 - x) * (1.0 + x)));
    double pmm = 1.0;
    for (int i = 1; i <= m; ++i) pmm *= (2.0 * i - 1.0) * somx2;
    if (l == m) return pmm;
    double pmmp1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pmmp1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pll = ((2.0 * ll - 1.0) * x * pmmp1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pmmp1;
        pmmp1 = pll;
    }
    return pll;
}

/* real orthonormal Y_lm times r^l, from spherical angles */
int orc_solid_harmonics(int lmax, double x, double y, double z, double *out)
{
    if (lmax < 0 || lmax > 20 || !out) return ORC_EBADARG;
    double r = sqrt(x * x + y * y + z * z);
    double ct = (r > 0.0) ? z / r : 1.0;
    double ph = (r > 0.0) ? atan2(y, x) : 0.0;
    for (int l = 0; l <= lmax; ++l) {
        double rl = pow(r, (double)l);
        if (l == 0) rl = 1.0;
        for (int m = 0; m <= l; ++m) {
            /* N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) */
            double fr = 1.0;
            for (int j = l - m + 1; j <= l + m; ++j) fr /= (double)j;
            double nlm = sqrt((2.0 * l + 1.0) / (4.0 * PI) * fr);
            double plm = assoc_legendre(l, m, ct);
            if (m == 0) {
                out[l * l + l] = rl * nlm * plm;
            } else {
                out[l * l + l + m] = rl * sqrt(2.0) * nlm * plm * cos(m * ph);
                out[l * l + l - m] = rl * sqrt(2.0) * nlm * plm * sin(m * ph);
            }
        }
    }
    return 0;
}

int orc_multipole_moments(const int *n, double h, const double *origin, int lmax,
                          const double *rho, double *Q)
{
    if (!n || !origin || !rho || !Q || lmax < 0 || lmax > 20) return ORC_EBADARG;
    const int nlm = (lmax + 1) * (lmax + 1);
    double c[3];
    box_centre(n, h, origin, c);
    const double dV = h * h * h;
    const int nz = n[2];
    double *part = calloc((size_t)nz * nlm, sizeof(double));
    if (!part) return ORC_EBADARG;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        double R[441];
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                double x = origin[0] + h * i - c[0];
                double y = origin[1] + h * j - c[1];
                double z = origin[2] + h * k - c[2];
                orc_solid_harmonics(lmax, x, y, z, R);
                double rv = rho[((long)k * n[1] + j) * n[0] + i];
                for (int q = 0; q < nlm; ++q) part[(long)k * nlm + q] += rv * R[q];
            }
    }
    for (int q = 0; q < nlm; ++q) {
        double s = 0.0;
        for (int k = 0; k < nz; ++k) s += part[(long)k * nlm + q];
        Q[q] = dV * s;
    }
    free(part);
    return 0;
}

/* 1/|r - r'| = sum_l 4pi/(2l+1) r'^l / r^(l+1) sum_m Y_lm(r^) Y_lm(r'^), |r'| < |r|:
 * the exterior potential of a charge with moments Q_lm about c. */
double orc_multipole_potential(const int *n, double h, const double *origin, int lmax,
                               const double *Q, double x, double y, double z)
{
    double c[3], R[441];
    box_centre(n, h, origin, c);
    double dx = x - c[0], dy = y - c[1], dz = z - c[2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    orc_solid_harmonics(lmax, dx, dy, dz, R);
    double v = 0.0;
    for (int l = 0; l <= lmax; ++l) {
        double inv = 1.0 / pow(r, 2.0 * l + 1.0); /* r^l Y_lm / r^(2l+1) = Y_lm / r^(l+1) */
        for (int m = -l; m <= l; ++m)
            v += 4.0 * PI / (2.0 * l + 1.0) * Q[l * l + l + m] * R[l * l + l + m] * inv;
    }
    return v;
}

/* is padded node (i,j,k) (interior coordinates) inside one of the six face
 * slabs: exactly one coordinate outside [0, n) and by at most p */
static int in_face_slab(const padded_t *g, int i, int j, int k)
{
    int idx[3] = {i, j, k}, outside = 0;
    for (int d = 0; d < 3; ++d) {
        if (idx[d] < 0 || idx[d] >= g->n[d]) {
            ++outside;
            if (idx[d] < -g->p || idx[d] >= g->n[d] + g->p) return 0;
        }
    }
    return outside == 1;
}

/* ------------------------------------------------------------------------ */
/* Conjugate gradients on K = -L (zero Dirichlet ghosts)                      */
/* ------------------------------------------------------------------------ */

static double dot(long M, const double *a, const double *b)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long q = 0; q < M; ++q) s += a[q] * b[q];
    return s;
}

/* K x = b, K = -L with zero ghosts; x starts at 0.  Plain CG (Hestenes-
 * Stiefel); when the recursive residual meets tol the true residual is
 * recomputed and CG restarts from x if it does not. */
static int cg_solve(const padded_t *g, const double *c, double h, const double *b,
                    double tol, int maxit, double *x, int *iters, double *relres)
{
    const long M = (long)g->n[0] * g->n[1] * g->n[2];
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    double *r = malloc(M * sizeof(double));
    double *q = malloc(M * sizeof(double));
    double *pp = calloc(pad_size(g), sizeof(double)); /* search direction, padded, zero ghosts */
    double *xp = calloc(pad_size(g), sizeof(double));
    if (!r || !q || !pp || !xp) { free(r); free(q); free(pp); free(xp); return ORC_EBADARG; }
    const double bnorm = sqrt(dot(M, b, b));
    int it = 0, status = ORC_ENOCONV;
    memset(x, 0, M * sizeof(double));
    double rel = 0.0;
    if (bnorm == 0.0) { status = 0; goto done; }

    for (int restart = 0; restart < 8 && it < maxit; ++restart) {
        /* r = b - K x = b + L x */
        scatter_interior(g, x, xp);
        lap_padded(g, c, h, xp, q);
        for (long m = 0; m < M; ++m) r[m] = b[m] + q[m];
        double rr = dot(M, r, r);
        if (sqrt(rr) / bnorm <= tol) { status = 0; break; }
        scatter_interior(g, r, pp);
        while (it < maxit) {
            lap_padded(g, c, h, pp, q);              /* q = L p */
            for (long m = 0; m < M; ++m) q[m] = -q[m]; /* q = K p */
            double pq = 0.0;
#pragma omp parallel for reduction(+ : pq) schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i)
                        pq += pp[pidx(g, i, j, k)] * q[((long)k * ny + j) * nx + i];
            const double alpha = rr / pq;
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        long m = ((long)k * ny + j) * nx + i;
                        x[m] += alpha * pp[pidx(g, i, j, k)];
                        r[m] -= alpha * q[m];
                    }
            ++it;
            const double rr_new = dot(M, r, r);
            if (sqrt(rr_new) / bnorm <= tol) break;
            const double beta = rr_new / rr;
            rr = rr_new;
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        long pi = pidx(g, i, j, k);
                        pp[pi] = r[((long)k * ny + j) * nx + i] + beta * pp[pi];
                    }
        }
    }
done:
    /* true residual */
    if (bnorm > 0.0) {
        scatter_interior(g, x, xp);
        lap_padded(g, c, h, xp, q);
        for (long m = 0; m < M; ++m) r[m] = b[m] + q[m];
        rel = sqrt(dot(M, r, r)) / bnorm;
        status = (rel <= tol) ? 0 : ORC_ENOCONV;
    }
    if (iters) *iters = it;
    if (relres) *relres = rel;
    free(r); free(q); free(pp); free(xp);
    return status;
}

/* ghost values of the multipole expansion of rho on the face slabs, written
 * into a padded field whose interior is zero */
static int fill_ghosts(const padded_t *g, double h, const double *origin, int lmax,
                       const double *Q, double *gp)
{
    const int p = g->p;
    memset(gp, 0, pad_size(g) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = -p; k < g->n[2] + p; ++k)
        for (int j = -p; j < g->n[1] + p; ++j)
            for (int i = -p; i < g->n[0] + p; ++i) {
                if (!in_face_slab(g, i, j, k)) continue;
                gp[pidx(g, i, j, k)] = orc_multipole_potential(
                    g->n, h, origin, lmax, Q, origin[0] + h * i, origin[1] + h * j, origin[2] + h * k);
            }
    return 0;
}

int orc_poisson(const int *n, double h, const double *origin, int p, int lmax,
                const double *rho, double tol, int maxit, double *v,
                int *iters, double *relres)
{
    if (!n || !origin || !rho || !v || h <= 0 || lmax < 0 || lmax > 20) return ORC_EBADARG;
    double c[17];
    if (orc_fd_coeffs(p, c)) return ORC_EBADARG;
    padded_t g = make_padded(n, p);
    const long M = grid_size(n);
    const int nlm = (lmax + 1) * (lmax + 1);
    double Q[441];
    orc_multipole_moments(n, h, origin, lmax, rho, Q);
    double *gp = malloc(pad_size(&g) * sizeof(double));
    double *b = malloc(M * sizeof(double));
    if (!gp || !b) { free(gp); free(b); return ORC_EBADARG; }
    (void)nlm;
    fill_ghosts(&g, h, origin, lmax, Q, gp);
    /* -L_full v = 4 pi rho  =>  -L_int v = 4 pi rho + (L g)|interior */
    lap_padded(&g, c, h, gp, b);
    for (long m = 0; m < M; ++m) b[m] += 4.0 * PI * rho[m];
    int st = cg_solve(&g, c, h, b, tol, maxit, v, iters, relres);
    free(gp); free(b);
    return st;
}

/* v = A rho with A = K^{-1} (4 pi I + C E_g P):  P takes moments, E_g maps
 * moments to ghost values, C maps ghost values into the right-hand side.
 * Its transpose is A^T = (4 pi I + P^T E_g^T C^T) K^{-1} (K symmetric). */
int orc_poisson_transpose(const int *n, double h, const double *origin, int p, int lmax,
                          const double *rho, double tol, int maxit, double *out,
                          int *iters, double *relres)
{
    if (!n || !origin || !rho || !out || h <= 0 || lmax < 0 || lmax > 20) return ORC_EBADARG;
    double c[17];
    if (orc_fd_coeffs(p, c)) return ORC_EBADARG;
    padded_t g = make_padded(n, p);
    const long M = grid_size(n);
    const int nlm = (lmax + 1) * (lmax + 1);
    double *w = malloc(M * sizeof(double));
    double *wp = calloc(pad_size(&g), sizeof(double));
    if (!w || !wp) { free(w); free(wp); return ORC_EBADARG; }
    /* w = K^{-1} rho */
    int st = cg_solve(&g, c, h, rho, tol, maxit, w, iters, relres);
    scatter_interior(&g, w, wp);
    /* z = C^T w: the stencil of the zero-extended w evaluated at each ghost
     * node (C_ij = L_ij for interior i and ghost j, and L is symmetric);
     * then E_g^T z: Q'_lm = sum_ghost 4pi/(2l+1) Y_lm / r^(l+1) z */
    double cen[3];
    box_centre(n, h, origin, cen);
    double Qt[441];
    memset(Qt, 0, sizeof(Qt));
    for (int k = -p; k < n[2] + p; ++k) {
        for (int j = -p; j < n[1] + p; ++j)
            for (int i = -p; i < n[0] + p; ++i) {
                if (!in_face_slab(&g, i, j, k)) continue;
                /* stencil at the ghost node; taps outside the padded box are zero
                 * for a zero-extended field, so clip them */
                double z = 0.0;
                int idx[3] = {i, j, k};
                for (int d = 0; d < 3; ++d)
                    for (int s = -p; s <= p; ++s) {
                        int t[3] = {idx[0], idx[1], idx[2]};
                        t[d] += s;
                        if (t[0] < 0 || t[0] >= n[0] || t[1] < 0 || t[1] >= n[1] ||
                            t[2] < 0 || t[2] >= n[2])
                            continue;
                        z += c[abs(s)] / (h * h) * w[((long)t[2] * n[1] + t[1]) * n[0] + t[0]];
                    }
                if (z == 0.0) continue;
                double R[441];
                double x = origin[0] + h * i - cen[0];
                double y = origin[1] + h * j - cen[1];
                double zz = origin[2] + h * k - cen[2];
                double r = sqrt(x * x + y * y + zz * zz);
                orc_solid_harmonics(lmax, x, y, zz, R);
                for (int l = 0; l <= lmax; ++l)
                    for (int m = -l; m <= l; ++m)
                        Qt[l * l + l + m] += 4.0 * PI / (2.0 * l + 1.0) * R[l * l + l + m] /
                                             pow(r, 2.0 * l + 1.0) * z;
            }
    }
    /* out = 4 pi w + P^T Q' with (P^T Q')(r) = dV sum_lm Q'_lm r^l Y_lm */
    const double dV = h * h * h;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n[2]; ++k) {
        double R[441];
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                orc_solid_harmonics(lmax, origin[0] + h * i - cen[0], origin[1] + h * j - cen[1],
                                    origin[2] + h * k - cen[2], R);
                double f = 0.0;
                for (int q = 0; q < nlm; ++q) f += Qt[q] * R[q];
                long m = ((long)k * n[1] + j) * n[0] + i;
                out[m] = 4.0 * PI * w[m] + dV * f;
            }
    }
    free(w); free(wp);
    return st;
}

/* ------------------------------------------------------------------------ */
/* LSDA exchange-correlation at full spin polarisation (Sec. III: LSDA       */
/* exchange with PW92 correlation; E_xc[rho_i, 0] of Eq. 1)                  */
/* ------------------------------------------------------------------------ */

void orc_xc_pol(double rho, double rho_floor, double *ex, double *ec, double *vx, double *vc)
{
    if (!(rho > rho_floor)) { *ex = *ec = *vx = *vc = 0.0; return; }
    /* Slater exchange of a density carried by one spin:
     * E_x[rho, 0] = (1/2) E_x^unpol[2 rho] = -(3/4)(6/pi)^(1/3) int rho^(4/3) */
    const double c6pi = cbrt(6.0 / PI);
    const double r13 = cbrt(rho);
    *ex = -0.75 * c6pi * r13;
    *vx = -c6pi * r13; /* d(rho ex)/d rho = (4/3) ex */

    /* PW92 interpolation G(rs; A, a1, b1..b4, p = 1), fully polarised set */
    const double A = 0.015545, a1 = 0.20548;
    const double b1 = 14.1189, b2 = 6.1977, b3 = 3.3662, b4 = 0.62517;
    const double rs = cbrt(3.0 / (4.0 * PI * rho));
    const double srs = sqrt(rs);
    const double den = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs);
    const double dden = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs);
    const double lg = log1p(1.0 / den);
    const double pre = -2.0 * A * (1.0 + a1 * rs);
    *ec = pre * lg;
    /* d eps_c / d rs */
    const double dec = -2.0 * A * a1 * lg + pre * (-dden / (den * den + den));
    /* v_c = eps_c - (rs/3) d eps_c / d rs; the zeta-derivative term vanishes at zeta = 1 */
    *vc = *ec - rs / 3.0 * dec;
}

/* ------------------------------------------------------------------------ */
/* Cubic interpolation at the FODs (Sec. II.B)                               */
/* ------------------------------------------------------------------------ */

/* Lagrange basis on nodes {-1, 0, 1, 2}: value and derivative at t */
static void lagrange4(double t, double *w, double *dw)
{
    const double tn[4] = {-1.0, 0.0, 1.0, 2.0};
    for (int j = 0; j < 4; ++j) {
        double val = 1.0;
        for (int k = 0; k < 4; ++k)
            if (k != j) val *= (t - tn[k]) / (tn[j] - tn[k]);
        w[j] = val;
        double der = 0.0;
        for (int m = 0; m < 4; ++m) {
            if (m == j) continue;
            double prod = 1.0 / (tn[j] - tn[m]);
            for (int k = 0; k < 4; ++k)
                if (k != j && k != m) prod *= (t - tn[k]) / (tn[j] - tn[k]);
            der += prod;
        }
        dw[j] = der;
    }
}

int orc_interp(const int *n, double h, const double *origin, int N, const double *psi,
               const double *a, double *u, double *du)
{
    if (!n || !origin || !psi || !a || !u || N < 0) return ORC_EBADARG;
    int i0[3];
    double w[3][4], dw[3][4];
    for (int d = 0; d < 3; ++d) {
        double s = (a[d] - origin[d]) / h;
        if (!isfinite(s)) return ORC_EBADARG;
        i0[d] = (int)floor(s);
        if (i0[d] < 1 || i0[d] > n[d] - 3) return ORC_EBOUNDARY;
        lagrange4(s - i0[d], w[d], dw[d]);
    }
    const long M = grid_size(n);
    for (int al = 0; al < N; ++al) {
        const double *f = psi + (long)al * M;
        double val = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        for (int c = 0; c < 4; ++c)
            for (int b = 0; b < 4; ++b)
                for (int q = 0; q < 4; ++q) {
                    double fv = f[((long)(i0[2] - 1 + c) * n[1] + (i0[1] - 1 + b)) * n[0] + (i0[0] - 1 + q)];
                    val += w[0][q] * w[1][b] * w[2][c] * fv;
                    gx += dw[0][q] * w[1][b] * w[2][c] * fv;
                    gy += w[0][q] * dw[1][b] * w[2][c] * fv;
                    gz += w[0][q] * w[1][b] * dw[2][c] * fv;
                }
        u[al] = val;
        if (du) {
            du[al * 3 + 0] = gx / h;
            du[al * 3 + 1] = gy / h;
            du[al * 3 + 2] = gz / h;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Symmetric eigenproblem: cyclic Jacobi (Golub & Van Loan, Alg. 8.4.3)      */

/* Per-node gradient of one grid field by first differences along each axis,
 * the scheme of Sec. II.B: central (f[i+1] - f[i-1]) / 2h at inner nodes,
 * forward (f[1] - f[0]) / h at the first node and backward
 * (f[n-1] - f[n-2]) / h at the last.  g[3*M] holds the x, y and z
 * components one after another. */
int orc_grid_gradient(const int *n, double h, const double *f, double *g)
{
    if (!n || !f || !g || !(h > 0)) return ORC_EBADARG;
    for (int d = 0; d < 3; ++d)
        if (n[d] < 2) return ORC_EBADARG;
    const long M = grid_size(n);
    const long stride[3] = {1, n[0], (long)n[0] * n[1]};
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < n[2]; ++k)
            for (int j = 0; j < n[1]; ++j)
                for (int i = 0; i < n[0]; ++i) {
                    const long m = ((long)k * n[1] + j) * n[0] + i;
                    const int q = (d == 0) ? i : (d == 1) ? j : k;
                    const long s = stride[d];
                    double v;
                    if (q == 0)
                        v = (f[m + s] - f[m]) / h;
                    else if (q == n[d] - 1)
                        v = (f[m] - f[m - s]) / h;
                    else
                        v = (f[m + s] - f[m - s]) / (2.0 * h);
                    g[d * M + m] = v;
                }
    return 0;
}

/* psi_alpha(a) and grad psi_alpha(a) the way Sec. II.B builds them: the
 * value by cubic interpolation, the gradient by first forming the per-node
 * difference gradient of each orbital (orc_grid_gradient) and interpolating
 * its three components at a with the same cubic scheme. */
int orc_interp_fdgrad(const int *n, double h, const double *origin, int N, const double *psi,
                      const double *a, double *u, double *du)
{
    if (!n || !origin || !psi || !a || !u || !du || N < 0) return ORC_EBADARG;
    const long M = grid_size(n);
    double *g = malloc(3 * M * sizeof(double));
    if (!g) return ORC_EBADARG;
    int st = 0;
    for (int al = 0; al < N && !st; ++al) {
        st = orc_interp(n, h, origin, 1, psi + (long)al * M, a, u + al, NULL);
        if (!st) st = orc_grid_gradient(n, h, psi + (long)al * M, g);
        if (!st) st = orc_interp(n, h, origin, 3, g, a, du + 3 * al, NULL);
    }
    free(g);
    return st;
}

/* ------------------------------------------------------------------------ */

int orc_jacobi_eig(int N, const double *A, double *lam, double *U)
{
    if (N < 1 || !A || !lam || !U) return ORC_EBADARG;
    double *a = malloc((size_t)N * N * sizeof(double));
    if (!a) return ORC_EBADARG;
    memcpy(a, A, (size_t)N * N * sizeof(double));
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) U[i * N + j] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (int i = 0; i < N * N; ++i) fro += a[i] * a[i];
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j) off += a[i * N + j] * a[i * N + j];
        if (off <= 1e-34 * fro) break;
        for (int p = 0; p < N - 1; ++p)
            for (int q = p + 1; q < N; ++q) {
                double apq = a[p * N + q];
                if (apq == 0.0) continue;
                double tau = (a[q * N + q] - a[p * N + p]) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
                for (int k = 0; k < N; ++k) { /* A <- A J */
                    double akp = a[k * N + p], akq = a[k * N + q];
                    a[k * N + p] = cs * akp - sn * akq;
                    a[k * N + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < N; ++k) { /* A <- J^T A */
                    double apk = a[p * N + k], aqk = a[q * N + k];
                    a[p * N + k] = cs * apk - sn * aqk;
                    a[q * N + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < N; ++k) { /* U <- U J */
                    double ukp = U[k * N + p], ukq = U[k * N + q];
                    U[k * N + p] = cs * ukp - sn * ukq;
                    U[k * N + q] = sn * ukp + cs * ukq;
                }
            }
    }
    for (int i = 0; i < N; ++i) lam[i] = a[i * N + i];
    /* ascending order */
    for (int i = 0; i < N; ++i) {
        int mn = i;
        for (int j = i + 1; j < N; ++j)
            if (lam[j] < lam[mn]) mn = j;
        if (mn != i) {
            double t = lam[i]; lam[i] = lam[mn]; lam[mn] = t;
            for (int k = 0; k < N; ++k) {
                double u0 = U[k * N + i]; U[k * N + i] = U[k * N + mn]; U[k * N + mn] = u0;
            }
        }
    }
    free(a);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One spin channel of the SIC path                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int N;
    long M;
    double *u, *du;   /* N x N values psi_alpha(a_i); N x N x 3 gradients */
    double *rhoa;     /* N  FOD densities */
    double *T;        /* N x N  T_i,alpha = psi_alpha(a_i)/sqrt(rho(a_i))  (Eq. 8) */
    double *F;        /* N x M  Fermi orbitals (Eq. 6-7) */
    double *S;        /* N x N  overlap dV F F^T */
    double *lam, *Us; /* eigen-decomposition of S */
    double *Z;        /* S^{-1/2} */
    double *phi;      /* N x M  FLOs (Loewdin) */
    double *v;        /* N x M  Hartree potentials of rho_i = phi_i^2 */
    double *U, *X;    /* N  Hartree and XC energies of each FLO density */
    int *iters;
    double *relres;
} fwd_t;

static void fwd_free(fwd_t *f)
{
    free(f->u); free(f->du); free(f->rhoa); free(f->T); free(f->F); free(f->S);
    free(f->lam); free(f->Us); free(f->Z); free(f->phi); free(f->v); free(f->U);
    free(f->X); free(f->iters); free(f->relres);
}

static int forward_impl(const int *n, double h, const double *origin, int p, int lmax,
                        double tol, int maxit, double rho_floor, int N, const double *psi,
                        const double *fod, fwd_t *f, int flo_only, int gmode)
{
    memset(f, 0, sizeof(*f));
    if (!n || !origin || !psi || !fod || N < 1 || h <= 0) return ORC_EBADARG;
    const long M = grid_size(n);
    const double dV = h * h * h;
    f->N = N;
    f->M = M;
    f->u = malloc((size_t)N * N * sizeof(double));
    f->du = malloc((size_t)N * N * 3 * sizeof(double));
    f->rhoa = malloc(N * sizeof(double));
    f->T = malloc((size_t)N * N * sizeof(double));
    f->F = malloc((size_t)N * M * sizeof(double));
    f->S = malloc((size_t)N * N * sizeof(double));
    f->lam = malloc(N * sizeof(double));
    f->Us = malloc((size_t)N * N * sizeof(double));
    f->Z = malloc((size_t)N * N * sizeof(double));
    f->phi = malloc((size_t)N * M * sizeof(double));
    f->v = malloc((size_t)N * M * sizeof(double));
    f->U = malloc(N * sizeof(double));
    f->X = malloc(N * sizeof(double));
    f->iters = malloc(N * sizeof(int));
    f->relres = malloc(N * sizeof(double));
    if (!f->u || !f->du || !f->rhoa || !f->T || !f->F || !f->S || !f->lam || !f->Us || !f->Z ||
        !f->phi || !f->v || !f->U || !f->X || !f->iters || !f->relres)
        return ORC_EBADARG;

    /* (a) psi_alpha(a_i) by cubic interpolation; rho(a_i) = sum_alpha f_alpha |psi_alpha(a_i)|^2
     * with f = 1; T_i,alpha = psi_alpha(a_i) / sqrt(rho(a_i))  (Sec. II.B, Eq. 8) */
    for (int i = 0; i < N; ++i) {
        int st = orc_interp(n, h, origin, N, psi, fod + 3 * i, f->u + (long)i * N,
                            gmode ? NULL : f->du + (long)i * N * 3);
        if (st) return st;
        double s = 0.0;
        for (int al = 0; al < N; ++al) s += f->u[i * N + al] * f->u[i * N + al];
        if (!(s > rho_floor)) return ORC_EVACUUM;
        f->rhoa[i] = s;
        for (int al = 0; al < N; ++al) f->T[i * N + al] = f->u[i * N + al] / sqrt(s);
    }
    if (gmode) {
        /* grad psi_alpha(a_i) as Sec. II.B builds it: per-node differences of
         * each orbital, interpolated at the FODs like the values */
        double *g = malloc(3 * M * sizeof(double));
        if (!g) return ORC_EBADARG;
        for (int al = 0; al < N; ++al) {
            orc_grid_gradient(n, h, psi + (long)al * M, g);
            for (int i = 0; i < N; ++i)
                orc_interp(n, h, origin, 3, g, fod + 3 * i, f->du + ((long)i * N + al) * 3, NULL);
        }
        free(g);
    }
    /* Fermi orbitals F_i = sum_alpha T_i,alpha psi_alpha  (Eq. 6-7) */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (long m = 0; m < M; ++m) {
            double s = 0.0;
            for (int al = 0; al < N; ++al) s += f->T[i * N + al] * psi[(long)al * M + m];
            f->F[(long)i * M + m] = s;
        }
    /* (b) overlap S_ij = dV sum_r F_i F_j and Loewdin orthonormalisation
     * phi = S^{-1/2} F (Sec. I.B: Fermi orbitals are normalised, not mutually orthogonal) */
    for (int i = 0; i < N; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = dV * dot(M, f->F + (long)i * M, f->F + (long)j * M);
            f->S[i * N + j] = f->S[j * N + i] = s;
        }
    orc_jacobi_eig(N, f->S, f->lam, f->Us);
    if (!(f->lam[0] > 1e-12)) return ORC_ESINGULAR;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int k = 0; k < N; ++k) s += f->Us[i * N + k] / sqrt(f->lam[k]) * f->Us[j * N + k];
            f->Z[i * N + j] = s;
        }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (long m = 0; m < M; ++m) {
            double s = 0.0;
            for (int j = 0; j < N; ++j) s += f->Z[i * N + j] * f->F[(long)j * M + m];
            f->phi[(long)i * M + m] = s;
        }
    if (flo_only) return 0;
    /* (c) Hartree potential of each FLO density, (d) its XC energy */
    int status = 0;
    double *rho = malloc((size_t)N * M * sizeof(double));
    if (!rho) return ORC_EBADARG;
    for (long q = 0; q < (long)N * M; ++q) rho[q] = f->phi[q] * f->phi[q];
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < N; ++i) {
        const double *ri = rho + (long)i * M;
        int st = orc_poisson(n, h, origin, p, lmax, ri, tol, maxit, f->v + (long)i * M,
                             f->iters + i, f->relres + i);
        if (st) {
#pragma omp critical
            status = st;
        }
        double u = 0.0, x = 0.0;
        for (long m = 0; m < M; ++m) {
            double ex, ec, vx, vc;
            u += ri[m] * f->v[(long)i * M + m];
            orc_xc_pol(ri[m], rho_floor, &ex, &ec, &vx, &vc);
            x += ri[m] * (ex + ec);
        }
        f->U[i] = 0.5 * dV * u;
        f->X[i] = dV * x;
    }
    free(rho);
    return status;
}

static int forward(const int *n, double h, const double *origin, int p, int lmax, double tol,
                   int maxit, double rho_floor, int N, const double *psi, const double *fod,
                   fwd_t *f)
{
    return forward_impl(n, h, origin, p, lmax, tol, maxit, rho_floor, N, psi, fod, f, 0, 0);
}

int orc_flo_spin(const int *n, double h, const double *origin, double rho_floor, int N,
                 const double *psi, const double *fod, double *phi, double *T, double *S,
                 double *Z)
{
    fwd_t f;
    int st = forward_impl(n, h, origin, 1, 0, 1e-10, 1, rho_floor, N, psi, fod, &f, 1, 0);
    if (st == 0) {
        const long M = grid_size(n);
        if (phi) memcpy(phi, f.phi, (size_t)N * M * sizeof(double));
        if (T) memcpy(T, f.T, (size_t)N * N * sizeof(double));
        if (S) memcpy(S, f.S, (size_t)N * N * sizeof(double));
        if (Z) memcpy(Z, f.Z, (size_t)N * N * sizeof(double));
    }
    fwd_free(&f);
    return st;
}

int orc_num_threads(void) { return omp_get_max_threads(); }

void orc_set_num_threads(int n) { if (n > 0) omp_set_num_threads(n); }

int orc_sic_spin(const int *n, double h, const double *origin, int p, int lmax,
                 double tol, int maxit, double vscale, double rho_floor,
                 int N, const double *psi, const double *fod,
                 double *e_spin, double *U, double *X, double *vsic,
                 double *T, double *S, double *Z, double *phi, double *v,
                 int *iters, double *relres)
{
    fwd_t f;
    int st = forward(n, h, origin, p, lmax, tol, maxit, rho_floor, N, psi, fod, &f);
    if (st && st != ORC_ENOCONV) { fwd_free(&f); return st; }
    const long M = f.M;
    /* E_SIC = -sum_i (U[rho_i] + E_xc[rho_i, 0])  (Eq. 1) */
    double e = 0.0;
    for (int i = 0; i < N; ++i) e -= f.U[i] + f.X[i];
    if (e_spin) *e_spin = e;
    if (U) memcpy(U, f.U, N * sizeof(double));
    if (X) memcpy(X, f.X, N * sizeof(double));
    if (T) memcpy(T, f.T, (size_t)N * N * sizeof(double));
    if (S) memcpy(S, f.S, (size_t)N * N * sizeof(double));
    if (Z) memcpy(Z, f.Z, (size_t)N * N * sizeof(double));
    if (phi) memcpy(phi, f.phi, (size_t)N * M * sizeof(double));
    if (v) memcpy(v, f.v, (size_t)N * M * sizeof(double));
    if (iters) memcpy(iters, f.iters, N * sizeof(int));
    if (relres) memcpy(relres, f.relres, N * sizeof(double));
    /* (e) generalised Slater average of the orbital SIC potentials
     * V_i = -(v_H[rho_i] + v_xc[rho_i, 0]), weighted by the FLO densities (Eq. 5, 13),
     * times the scale factor s */
    if (vsic) {
#pragma omp parallel for schedule(static)
        for (long m = 0; m < M; ++m) {
            double num = 0.0, den = 0.0;
            for (int i = 0; i < N; ++i) {
                double r = f.phi[(long)i * M + m] * f.phi[(long)i * M + m];
                double ex, ec, vx, vc;
                orc_xc_pol(r, rho_floor, &ex, &ec, &vx, &vc);
                double Vi = -(f.v[(long)i * M + m] + vx + vc);
                num += r * Vi;
                den += r;
            }
            vsic[m] = (den > rho_floor) ? vscale * num / den : 0.0;
        }
    }
    fwd_free(&f);
    return st;
}

/* The two energy terms of one orbital density (Eq. 1): the Hartree energy
 * U = 1/2 dV sum_r rho v_H[rho] and the fully polarised LSDA energy
 * X = dV sum_r rho (eps_x + eps_c), for sampled checks on large grids. */
int orc_orbital_terms(const int *n, double h, const double *origin, int p, int lmax,
                      double tol, int maxit, double rho_floor, const double *rho,
                      double *U, double *X, int *iters, double *relres)
{
    if (!n || !origin || !rho || !U || !X || h <= 0) return ORC_EBADARG;
    const long M = grid_size(n);
    const double dV = h * h * h;
    double *v = malloc((size_t)M * sizeof(double));
    if (!v) return ORC_EBADARG;
    int st = orc_poisson(n, h, origin, p, lmax, rho, tol, maxit, v, iters, relres);
    double u = 0.0, x = 0.0;
    for (long m = 0; m < M; ++m) {
        double ex, ec, vx, vc;
        u += rho[m] * v[m];
        orc_xc_pol(rho[m], rho_floor, &ex, &ec, &vx, &vc);
        x += rho[m] * (ex + ec);
    }
    *U = 0.5 * dV * u;
    *X = dV * x;
    free(v);
    return st;
}

/* ------------------------------------------------------------------------ */
/* FOD gradient (Eq. 9-11), tangent mode                                     */
/* ------------------------------------------------------------------------ */

/* C = A B with A (r x k), B (k x c), all row-major */
static void matmul(int r, int k, int c, const double *A, const double *B, double *C)
{
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) {
            double s = 0.0;
            for (int q = 0; q < k; ++q) s += A[i * k + q] * B[q * c + j];
            C[i * c + j] = s;
        }
}

/* Tangent of Q = Z T (phi = Q psi) along FOD coordinate (mi, d):
 * row mi of T moves as T_m = u_m / |u_m| (Eq. 8, and Eq. 11 in a form free of
 * 1/psi), S = T G T^T moves as dS = dT G T^T + T G dT^T, Z = S^{-1/2} moves by
 * the Frechet derivative dZ = U [(U^T dS U) o K] U^T, and dQ = dZ T + Z dT. */
typedef struct {
    int N;
    const fwd_t *f;
    double *K, *TG, *UT, *dT, *dS, *dZ, *tmp, *tmp2;
} tangent_t;

static int tangent_init(tangent_t *t, const fwd_t *f, const double *G)
{
    const int N = f->N;
    const size_t bytes = (size_t)N * N * sizeof(double);
    t->N = N;
    t->f = f;
    t->K = malloc(bytes); t->TG = malloc(bytes); t->UT = malloc(bytes); t->dT = malloc(bytes);
    t->dS = malloc(bytes); t->dZ = malloc(bytes); t->tmp = malloc(bytes); t->tmp2 = malloc(bytes);
    if (!t->K || !t->TG || !t->UT || !t->dT || !t->dS || !t->dZ || !t->tmp || !t->tmp2)
        return ORC_EBADARG;
    /* K_jk = (lam_j^{-1/2} - lam_k^{-1/2}) / (lam_j - lam_k) in its stable form */
    for (int j = 0; j < N; ++j)
        for (int k = 0; k < N; ++k) {
            double sj = sqrt(f->lam[j]), sk = sqrt(f->lam[k]);
            t->K[j * N + k] = -1.0 / (sj * sk * (sj + sk));
        }
    matmul(N, N, N, f->T, G, t->TG); /* T G */
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) t->UT[i * N + j] = f->Us[j * N + i];
    return 0;
}

static void tangent_free(tangent_t *t)
{
    free(t->K); free(t->TG); free(t->UT); free(t->dT); free(t->dS); free(t->dZ);
    free(t->tmp); free(t->tmp2);
}

static void tangent_dQ(tangent_t *t, int mi, int d, double *dQ)
{
    const int N = t->N;
    const fwd_t *f = t->f;
    const double norm = sqrt(f->rhoa[mi]);
    double *dT = t->dT, *dS = t->dS, *dZ = t->dZ, *tmp = t->tmp, *tmp2 = t->tmp2;
    memset(dT, 0, (size_t)N * N * sizeof(double));
    double tdu = 0.0;
    for (int al = 0; al < N; ++al) tdu += f->T[mi * N + al] * f->du[((long)mi * N + al) * 3 + d];
    for (int al = 0; al < N; ++al)
        dT[mi * N + al] = (f->du[((long)mi * N + al) * 3 + d] - tdu * f->T[mi * N + al]) / norm;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int q = 0; q < N; ++q)
                s += dT[i * N + q] * t->TG[j * N + q] + t->TG[i * N + q] * dT[j * N + q];
            dS[i * N + j] = s;
        }
    matmul(N, N, N, t->UT, dS, tmp);
    matmul(N, N, N, tmp, f->Us, tmp2);
    for (int q = 0; q < N * N; ++q) tmp2[q] *= t->K[q];
    matmul(N, N, N, f->Us, tmp2, tmp);
    matmul(N, N, N, tmp, t->UT, dZ);
    matmul(N, N, N, dZ, f->T, tmp);
    matmul(N, N, N, f->Z, dT, tmp2);
    for (int q = 0; q < N * N; ++q) dQ[q] = tmp[q] + tmp2[q];
}

int orc_sic_grad_spin_mode(const int *n, double h, const double *origin, int p, int lmax,
                           double tol, int maxit, double rho_floor,
                           int N, const double *psi, const double *fod, int gmode, int form,
                           double *dEda)
{
    if (!dEda || gmode < 0 || gmode > 1 || form < 0 || form > 1) return ORC_EBADARG;
    fwd_t f;
    int st = forward_impl(n, h, origin, p, lmax, tol, maxit, rho_floor, N, psi, fod, &f, 0, gmode);
    if (st && st != ORC_ENOCONV) { fwd_free(&f); return st; }
    const long M = f.M;
    const double dV = h * h * h;
    double *G = malloc((size_t)N * N * sizeof(double));
    double *dQ = malloc((size_t)N * N * sizeof(double));
    tangent_t tg;
    memset(&tg, 0, sizeof(tg));
    int st2 = (!G || !dQ) ? ORC_EBADARG : 0;
    if (!st2) {
        for (int i = 0; i < N; ++i)
            for (int al = 0; al < N; ++al)
                G[i * N + al] = dV * dot(M, psi + (long)i * M, psi + (long)al * M);
        st2 = tangent_init(&tg, &f, G);
    }
    if (!st2 && form == 0) {
        /* exact derivative of the discrete E_SIC.  With respect to phi_i(r):
         *   dE/dphi_i = 2 dV phi_i omega_i,
         *   omega_i = -( (1/2)(v_i + A^T rho_i) + v_xc(rho_i) ),
         * because U_i = (1/2) dV rho_i^T A rho_i and dE_xc/drho = dV v_xc.
         * phi = Q psi, so dE = sum_{i,alpha} dQ_i,alpha B_i,alpha, B = Gam psi^T. */
        double *Gam = malloc((size_t)N * M * sizeof(double));
        double *B = malloc((size_t)N * N * sizeof(double));
        if (!Gam || !B) st2 = ORC_EBADARG;
        const int nrun = st2 ? 0 : N;
#pragma omp parallel for schedule(dynamic, 1)
        for (int i = 0; i < nrun; ++i) {
            double *rho = malloc(M * sizeof(double));
            double *at = malloc(M * sizeof(double));
            const double *ph = f.phi + (long)i * M;
            for (long m = 0; m < M; ++m) rho[m] = ph[m] * ph[m];
            int s = orc_poisson_transpose(n, h, origin, p, lmax, rho, tol, maxit, at, NULL, NULL);
            if (s) {
#pragma omp critical
                st2 = s;
            }
            for (long m = 0; m < M; ++m) {
                double ex, ec, vx, vc;
                orc_xc_pol(rho[m], rho_floor, &ex, &ec, &vx, &vc);
                double om = -(0.5 * (f.v[(long)i * M + m] + at[m]) + vx + vc);
                Gam[(long)i * M + m] = 2.0 * dV * ph[m] * om;
            }
            free(rho); free(at);
        }
        if (B && Gam)
            for (int i = 0; i < N; ++i)
                for (int al = 0; al < N; ++al) B[i * N + al] = dot(M, Gam + (long)i * M, psi + (long)al * M);
        for (int mi = 0; mi < N && B && Gam; ++mi)
            for (int d = 0; d < 3; ++d) {
                tangent_dQ(&tg, mi, d, dQ);
                double dE = 0.0;
                for (int q = 0; q < N * N; ++q) dE += dQ[q] * B[q];
                dEda[mi * 3 + d] = dE;
            }
        free(Gam); free(B);
    } else if (!st2) {
        /* Eq. 9: dE/da_m = sum_kl eps_kl ( <dphi_k/da_m|phi_l> - <dphi_l/da_m|phi_k> )
         * with eps_kl = <phi_l| V_k |phi_k> and the orbital SIC potential
         * V_k = -(v_k + v_xc(rho_k)) of Eq. 5 */
        double *eps = malloc((size_t)N * N * sizeof(double));
        double *Vphi = malloc((size_t)N * M * sizeof(double));
        double *dphi = malloc((size_t)N * M * sizeof(double));
        double *A = malloc((size_t)N * N * sizeof(double));
        if (!eps || !Vphi || !dphi || !A) st2 = ORC_EBADARG;
        const int nrun = st2 ? 0 : N;
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nrun; ++k)
            for (long m = 0; m < M; ++m) {
                const double ph = f.phi[(long)k * M + m];
                double ex, ec, vx, vc;
                orc_xc_pol(ph * ph, rho_floor, &ex, &ec, &vx, &vc);
                Vphi[(long)k * M + m] = -(f.v[(long)k * M + m] + vx + vc) * ph;
            }
        for (int k = 0; k < nrun; ++k)
            for (int l = 0; l < N; ++l) eps[k * N + l] = dV * dot(M, f.phi + (long)l * M, Vphi + (long)k * M);
        for (int mi = 0; mi < nrun; ++mi)
            for (int d = 0; d < 3; ++d) {
                tangent_dQ(&tg, mi, d, dQ);
                /* dphi_k = sum_alpha dQ_k,alpha psi_alpha; A_kl = <dphi_k | phi_l> */
#pragma omp parallel for schedule(static)
                for (int k = 0; k < N; ++k)
                    for (long m = 0; m < M; ++m) {
                        double sacc = 0.0;
                        for (int al = 0; al < N; ++al) sacc += dQ[k * N + al] * psi[(long)al * M + m];
                        dphi[(long)k * M + m] = sacc;
                    }
                for (int k = 0; k < N; ++k)
                    for (int l = 0; l < N; ++l) A[k * N + l] = dV * dot(M, dphi + (long)k * M, f.phi + (long)l * M);
                double dE = 0.0;
                for (int k = 0; k < N; ++k)
                    for (int l = 0; l < N; ++l) dE += eps[k * N + l] * (A[k * N + l] - A[l * N + k]);
                dEda[mi * 3 + d] = dE;
            }
        free(eps); free(Vphi); free(dphi); free(A);
    }
    tangent_free(&tg);
    free(G); free(dQ);
    fwd_free(&f);
    return st2 ? st2 : st;
}

int orc_sic_grad_spin(const int *n, double h, const double *origin, int p, int lmax,
                      double tol, int maxit, double rho_floor,
                      int N, const double *psi, const double *fod, double *dEda)
{
    return orc_sic_grad_spin_mode(n, h, origin, p, lmax, tol, maxit, rho_floor, N, psi, fod, 0, 0,
                                  dEda);
}
