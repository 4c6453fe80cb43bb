// Dirichlet boundary values of the Hartree problem for isolated systems from
// a multipole expansion of each FLO density about the box centre (Sec. II.A),
// the right-hand side -L v = 4 pi rho + (boundary term), and the transpose of
// that boundary map for the adjoint (FOD-gradient) solves.
//
// Real solid harmonics r^l Y_lm are built without trigonometry: the
// azimuthal factor is (x + i y)^m and the polar factor r^(l-m) d^m P_l/dx^m
// (z / r) obeys the three-term recurrence in l, so one node costs a few
// hundred flops and no transcendental calls.
#include "kernels.h"

namespace fsic {

// Calls f(q, l, r^l Y_lm(x, y, z)) for q = l*l + l + m, every l <= L, in the
// order the recurrence produces the values (real, orthonormal, no
// Condon-Shortley phase).  Consuming each value at once keeps few of them
// live, so accumulating kernels need no harmonic array in registers.
template <int L, class F>
__device__ __forceinline__ void visit_regular_harmonics(double x, double y, double z, const double *norm,
                                                        F &&f) {
    const double r2 = x * x + y * y + z * z;
    double cm = 1.0, sm = 0.0;  // Re, Im of (x + i y)^m
    double dfact = 1.0;         // (2m - 1)!!
#pragma unroll
    for (int m = 0; m <= L; ++m) {
        if (m > 0) {
            const double c2 = cm * x - sm * y;
            sm = cm * y + sm * x;
            cm = c2;
            dfact *= (double)(2 * m - 1);
        }
        double pm2 = 0.0, pm1 = 0.0;
#pragma unroll
        for (int l = m; l <= L; ++l) {
            double pl;
            if (l == m)
                pl = dfact;
            else if (l == m + 1)
                pl = (double)(2 * m + 1) * z * pm1;
            else
                pl = ((double)(2 * l - 1) * z * pm1 - (double)(l + m - 1) * r2 * pm2) *
                     (1.0 / (double)(l - m));  // compile-time reciprocal: no FP64 divide
            pm2 = pm1;
            pm1 = pl;
            if (m == 0) {
                f(l * l + l, l, norm[l * l + l] * pl);
            } else {
                f(l * l + l + m, l, norm[l * l + l + m] * cm * pl);
                f(l * l + l - m, l, norm[l * l + l - m] * sm * pl);
            }
        }
    }
}

// R[l*l + l + m] = r^l Y_lm(x, y, z)
template <int L>
__device__ __forceinline__ void regular_harmonics(double x, double y, double z, const double *norm,
                                                  double *R) {
    visit_regular_harmonics<L>(x, y, z, norm, [&](int q, int, double v) { R[q] = v; });
}

// ---------------------------------------------------------------------------
// moments Q_lm = dV sum_r rho(r) R_lm(r - c)
// ---------------------------------------------------------------------------

template <int L>
__global__ __launch_bounds__(256) void k_moments(HarmTables ht, const OrbDesc *orb,
                                                 const Item *items, const double *src, int square,
                                                 double *partQ) {
    constexpr int NLM = (L + 1) * (L + 1);
    __shared__ double sw[4][NLM];
    const Item it = items[blockIdx.x];
    if (it.orb < 0) return;
    const OrbDesc od = orb[it.orb];
    const long long M = (long long)od.nx * od.ny * od.nz;
    double acc[NLM];
#pragma unroll
    for (int q = 0; q < NLM; ++q) acc[q] = 0.0;
    const long long base = (long long)it.tile * kPW;
    for (int e = 0; e < kPW / 256; ++e) {
        const long long i = base + e * 256 + threadIdx.x;
        if (i < M) {
            // node indices in 32 bits (at most 2^29 nodes per orbital)
            const int ii = (int)i, pxy = od.nx * od.ny;
            const int iz = ii / pxy, rem = ii - iz * pxy;
            const int iy = rem / od.nx, ix = rem - iy * od.nx;
            const double sv = src[od.off + i];
            const double rho = square ? sv * sv : sv;
            visit_regular_harmonics<L>(od.origin[0] + od.h * ix - od.centre[0],
                                       od.origin[1] + od.h * iy - od.centre[1],
                                       od.origin[2] + od.h * iz - od.centre[2], ht.norm,
                                       [&](int q, int, double v) { acc[q] += rho * v; });
        }
    }
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
        const double v = wave_sum(acc[q]);
        if ((threadIdx.x & 63) == 0) sw[w][q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NLM; q += 256)
        partQ[(size_t)(od.base8 + it.tile) * NLM + q] = (sw[0][q] + sw[1][q]) + (sw[2][q] + sw[3][q]);
}

__global__ __launch_bounds__(256) void k_moments_final(int nlm, const OrbDesc *orb,
                                                       const double *partQ, double *Q) {
    const int o = blockIdx.x;
    const OrbDesc od = orb[o];
    const double dV = od.h * od.h * od.h;
    for (int q = threadIdx.x; q < nlm; q += 256) {
        double s = 0.0;
        for (int t = 0; t < od.nt8; ++t) s += partQ[(size_t)(od.base8 + t) * nlm + q];
        Q[(size_t)o * nlm + q] = dV * s;
    }
}

// ---------------------------------------------------------------------------
// ghost nodes: six face slabs of depth P; per orbital, in the order
// x-, x+, y-, y+, z-, z+; layer d = 1..P; then the face's 2-D index.
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool ghost_decode(const OrbDesc &od, int P, long long g, int &gi, int &gj,
                                             int &gk, int &face, int &d) {
    const long long Fx = (long long)od.ny * od.nz, Fy = (long long)od.nx * od.nz,
                    Fz = (long long)od.nx * od.ny;
    const long long sz[3] = {P * Fx, P * Fy, P * Fz};
    const long long Fs[3] = {Fx, Fy, Fz};
    long long rem = g;
    for (int ax = 0; ax < 3; ++ax) {
        for (int side = 0; side < 2; ++side) {
            if (rem < sz[ax]) {
                d = (int)(rem / Fs[ax]) + 1;
                const long long f2 = rem % Fs[ax];
                face = 2 * ax + side;
                if (ax == 0) {
                    gj = (int)(f2 % od.ny);
                    gk = (int)(f2 / od.ny);
                    gi = side ? od.nx - 1 + d : -d;
                } else if (ax == 1) {
                    gi = (int)(f2 % od.nx);
                    gk = (int)(f2 / od.nx);
                    gj = side ? od.ny - 1 + d : -d;
                } else {
                    gi = (int)(f2 % od.nx);
                    gj = (int)(f2 / od.nx);
                    gk = side ? od.nz - 1 + d : -d;
                }
                return true;
            }
            rem -= sz[ax];
        }
    }
    return false;
}

template <int L>
__global__ __launch_bounds__(256) void k_ghosts(int P, HarmTables ht, const OrbDesc *orb,
                                                const long long *gcount, const double *Q,
                                                double *G) {
    constexpr int NLM = (L + 1) * (L + 1);
    const int o = blockIdx.y;
    const OrbDesc od = orb[o];
    const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
    if (g >= gcount[o]) return;
    int gi, gj, gk, face, d;
    if (!ghost_decode(od, P, g, gi, gj, gk, face, d)) return;
    const double x = od.origin[0] + od.h * gi - od.centre[0];
    const double y = od.origin[1] + od.h * gj - od.centre[1];
    const double z = od.origin[2] + od.h * gk - od.centre[2];
    double R[NLM];
    regular_harmonics<L>(x, y, z, ht.norm, R);
    const double r2 = x * x + y * y + z * z;
    const double ir2 = 1.0 / r2;
    const double ir = sqrt(ir2);
    double v = 0.0;
    double pw = ir;  // r^-(2l+1)
#pragma unroll
    for (int l = 0; l <= L; ++l) {
        double s = 0.0;
#pragma unroll
        for (int m = -l; m <= l; ++m) s += ht.gfac[l * l + l + m] * Q[(size_t)o * NLM + l * l + l + m] * R[l * l + l + m];
        v += s * pw;
        pw *= ir2;
    }
    G[od.goff + g] = v;
}

// ---------------------------------------------------------------------------
// right-hand side b = scale * rho + (L g)|interior
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_rhs(int P, Coeffs cf, const OrbDesc *orb,
                                             const Item *items, const double *src, int square,
                                             double scale, const double *G, double *B,
                                             double *R64, float *R32, double *X64zero,
                                             double *part8) {
    __shared__ double sred[4];
    const Item it = items[blockIdx.x];
    if (it.orb < 0) return;
    const OrbDesc od = orb[it.orb];
    const int nx = od.nx, ny = od.ny, nz = od.nz;
    const long long M = (long long)nx * ny * nz;
    const long long Fx = (long long)ny * nz, Fy = (long long)nx * nz, Fz = (long long)nx * ny;
    const long long oxm = 0, oxp = P * Fx, oym = 2 * P * Fx, oyp = oym + P * Fy,
                    ozm = oym + 2 * P * Fy, ozp = ozm + P * Fz;
    const long long base = (long long)it.tile * kPW;
    double acc = 0.0;
    for (int e = 0; e < kPW / 256; ++e) {
        const long long i = base + e * 256 + threadIdx.x;
        if (i >= M) continue;
        // node indices in 32 bits (at most 2^29 nodes per orbital)
        const int ii = (int)i, pxy = nx * ny;
        const int iz = ii / pxy, rem = ii - iz * pxy;
        const int iy = rem / nx, ix = rem - iy * nx;
        const double sv = src[od.off + i];
        double b = scale * (square ? sv * sv : sv);
        if (G) {
            const double *g = G + od.goff;
            double bt = 0.0;
            // taps that reach the ghost layers of each face: node at distance e
            // from the face sees ghost layer d with weight c_{e+d}, e + d <= P
            int e0 = ix;
            for (int d = 1; d <= P - e0; ++d) bt += cf.c[e0 + d] * g[oxm + (d - 1) * Fx + iy + (long long)ny * iz];
            e0 = nx - 1 - ix;
            for (int d = 1; d <= P - e0; ++d) bt += cf.c[e0 + d] * g[oxp + (d - 1) * Fx + iy + (long long)ny * iz];
            e0 = iy;
            for (int d = 1; d <= P - e0; ++d) bt += cf.c[e0 + d] * g[oym + (d - 1) * Fy + ix + (long long)nx * iz];
            e0 = ny - 1 - iy;
            for (int d = 1; d <= P - e0; ++d) bt += cf.c[e0 + d] * g[oyp + (d - 1) * Fy + ix + (long long)nx * iz];
            e0 = iz;
            for (int d = 1; d <= P - e0; ++d) bt += cf.c[e0 + d] * g[ozm + (d - 1) * Fz + ix + (long long)nx * iy];
            e0 = nz - 1 - iz;
            for (int d = 1; d <= P - e0; ++d) bt += cf.c[e0 + d] * g[ozp + (d - 1) * Fz + ix + (long long)nx * iy];
            b += bt * od.inv_h2;
        }
        const long long gi = od.off + i;
        if (B) B[gi] = b;
        if (R64) R64[gi] = b;
        if (R32) R32[gi] = (float)b;
        if (X64zero) X64zero[gi] = 0.0;
        acc += b * b;
    }
    const double s = block_sum256(acc, sred);
    if (threadIdx.x == 0) part8[od.base8 + it.tile] = s;
}

// ---------------------------------------------------------------------------
// adjoint boundary: zt_lm = sum_ghost gfac_lm Y_lm / r^(l+1) (C^T w)_ghost,
// (C^T w)_ghost = sum over interior taps c_k / h^2 w
// ---------------------------------------------------------------------------

template <int L>
__global__ __launch_bounds__(256) void k_adj_boundary(int P, HarmTables ht, Coeffs cf,
                                                      const OrbDesc *orb, const long long *gcount,
                                                      const double *W, double *partZ,
                                                      int zchunks) {
    constexpr int NLM = (L + 1) * (L + 1);
    __shared__ double sw[4][NLM];
    const int o = blockIdx.y;
    const OrbDesc od = orb[o];
    const long long G = gcount[o];
    double acc[NLM];
#pragma unroll
    for (int q = 0; q < NLM; ++q) acc[q] = 0.0;
    const long long per = (G + zchunks - 1) / zchunks;
    const long long g0 = per * blockIdx.x, g1 = min(G, g0 + per);
    const double *w = W + od.off;
    for (long long g = g0 + threadIdx.x; g < g1; g += 256) {
        int gi, gj, gk, face, d;
        if (!ghost_decode(od, P, g, gi, gj, gk, face, d)) continue;
        // taps from the ghost node into the interior, along the face normal
        double zsum = 0.0;
        const int ax = face >> 1, side = face & 1;
        for (int t = 0; t + d <= P; ++t) {
            int ii = gi, jj = gj, kk = gk;  // interior node at distance t from the face
            if (ax == 0) ii = side ? od.nx - 1 - t : t;
            if (ax == 1) jj = side ? od.ny - 1 - t : t;
            if (ax == 2) kk = side ? od.nz - 1 - t : t;
            zsum += cf.c[t + d] * w[((long long)kk * od.ny + jj) * od.nx + ii];
        }
        zsum *= od.inv_h2;
        const double x = od.origin[0] + od.h * gi - od.centre[0];
        const double y = od.origin[1] + od.h * gj - od.centre[1];
        const double z = od.origin[2] + od.h * gk - od.centre[2];
        double R[NLM];
        regular_harmonics<L>(x, y, z, ht.norm, R);
        const double ir2 = 1.0 / (x * x + y * y + z * z);
        double pw = sqrt(ir2) * zsum;
#pragma unroll
        for (int l = 0; l <= L; ++l) {
#pragma unroll
            for (int m = -l; m <= l; ++m) acc[l * l + l + m] += ht.gfac[l * l + l + m] * R[l * l + l + m] * pw;
            pw *= ir2;
        }
    }
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NLM; ++q) {
        const double v = wave_sum(acc[q]);
        if ((threadIdx.x & 63) == 0) sw[wv][q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NLM; q += 256)
        partZ[((size_t)o * zchunks + blockIdx.x) * NLM + q] = (sw[0][q] + sw[1][q]) + (sw[2][q] + sw[3][q]);
}

__global__ void k_adj_boundary_final(int nlm, int zchunks, const double *partZ, double *Zt) {
    const int o = blockIdx.x;
    for (int q = threadIdx.x; q < nlm; q += blockDim.x) {
        double s = 0.0;
        for (int t = 0; t < zchunks; ++t) s += partZ[((size_t)o * zchunks + t) * nlm + q];
        Zt[(size_t)o * nlm + q] = s;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define FSIC_L_SWITCH(lmax, CALL)   \
    switch (lmax) {                 \
        case 0: CALL(0); break;     \
        case 1: CALL(1); break;     \
        case 2: CALL(2); break;     \
        case 3: CALL(3); break;     \
        case 4: CALL(4); break;     \
        case 5: CALL(5); break;     \
        case 6: CALL(6); break;     \
        case 7: CALL(7); break;     \
        case 8: CALL(8); break;     \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_moments(int lmax, const HarmTables &ht, int norb, const OrbDesc *orb,
                          const Item *items8, int nitems8, const double *src, int square,
                          double *partQ, int tot8, double *Q, hipStream_t s) {
    (void)tot8;
    if (nitems8 <= 0 || norb <= 0) return hipSuccess;
#define CALL(L) hipLaunchKernelGGL(k_moments<L>, dim3(nitems8), dim3(256), 0, s, ht, orb, items8, src, square, partQ)
    FSIC_L_SWITCH(lmax, CALL)
#undef CALL
    hipLaunchKernelGGL(k_moments_final, dim3(norb), dim3(256), 0, s, (lmax + 1) * (lmax + 1), orb,
                       partQ, Q);
    return hipGetLastError();
}

hipError_t launch_ghosts(int radius, int lmax, const HarmTables &ht, int norb,
                         const OrbDesc *orb, const long long *ghost_count, const double *Q,
                         double *G, long long max_ghost, hipStream_t s) {
    if (norb <= 0) return hipSuccess;
    dim3 grid((unsigned)((max_ghost + 255) / 256), (unsigned)norb);
#define CALL(L) hipLaunchKernelGGL(k_ghosts<L>, grid, dim3(256), 0, s, radius, ht, orb, ghost_count, Q, G)
    FSIC_L_SWITCH(lmax, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_rhs(int radius, const Coeffs &c, const Item *items8, int nitems8,
                      const OrbDesc *orb, const double *src, int square, double scale,
                      const double *G, double *B, double *R64, float *R32, double *X64zero,
                      double *part8, hipStream_t s) {
    if (nitems8 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rhs, dim3(nitems8), dim3(256), 0, s, radius, c, orb, items8, src, square,
                       scale, G, B, R64, R32, X64zero, part8);
    return hipGetLastError();
}

hipError_t launch_adjoint_boundary(int radius, int lmax, const HarmTables &ht, const Coeffs &c,
                                   int norb, const OrbDesc *orb, const long long *ghost_count,
                                   const double *W, double *partZ, int zchunks, double *Zt,
                                   long long max_ghost, hipStream_t s) {
    (void)max_ghost;
    if (norb <= 0) return hipSuccess;
    dim3 grid((unsigned)zchunks, (unsigned)norb);
#define CALL(L) hipLaunchKernelGGL(k_adj_boundary<L>, grid, dim3(256), 0, s, radius, ht, c, orb, ghost_count, W, partZ, zchunks)
    FSIC_L_SWITCH(lmax, CALL)
#undef CALL
    hipLaunchKernelGGL(k_adj_boundary_final, dim3(norb), dim3(128), 0, s, (lmax + 1) * (lmax + 1),
                       zchunks, partZ, Zt);
    return hipGetLastError();
}

}  // namespace fsic
