// Fermi orbitals and their Loewdin orthonormalisation (Eq. 6-8, Sec. I.B),
// the cubic interpolation of the KS orbitals at the FODs (Sec. II.B), and the
// reverse-mode derivative of that chain for the FOD gradient (Eq. 9-11).
//
// The two grid-sized contractions run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64):
//   * the Gram matrix G = dV psi psi^T, from which the FO overlap follows
//     exactly as S = dV F F^T = T G T^T (F = T psi), so F is never stored;
//   * the Fermi-Loewdin orbitals phi = Q psi with Q = S^{-1/2} T.
// Everything N x N (N <= 128) runs in one workgroup: S = T G T^T, a parallel
// cyclic Jacobi eigen-decomposition (round-robin pairing), S^{-1/2}, Q.
#include <algorithm>
#include <cstdint>

#include "kernels.h"
#include "tsgemm.h"

namespace fsic {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// MFMA f64 16x16x4 fragment layout (64 lanes):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[l / 16 + 4 j][l % 16], j = 0..3 (rows interleaved)
__device__ __forceinline__ dbl4 mfma16x16x4(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// cubic interpolation at the FODs, T = u / |u|
// ---------------------------------------------------------------------------

__device__ __forceinline__ void cubic_weights(double t, double *w, double *dw) {
    // Lagrange basis on the nodes -1, 0, 1, 2 and its derivative in t
    const double tm1 = t - 1.0, tm2 = t - 2.0, tp1 = t + 1.0;
    w[0] = -t * tm1 * tm2 * (1.0 / 6.0);
    w[1] = tp1 * tm1 * tm2 * 0.5;
    w[2] = -tp1 * t * tm2 * 0.5;
    w[3] = tp1 * t * tm1 * (1.0 / 6.0);
    const double t2 = t * t;
    dw[0] = -(3.0 * t2 - 6.0 * t + 2.0) * (1.0 / 6.0);
    dw[1] = (3.0 * t2 - 4.0 * t - 1.0) * 0.5;
    dw[2] = -(3.0 * t2 - 2.0 * t - 2.0) * 0.5;
    dw[3] = (3.0 * t2 - 1.0) * (1.0 / 6.0);
}

// Weights, over the six nodes i0-2 .. i0+3 of one axis, that turn grid
// values into the cubic interpolant (at offset t from node i0) of the
// per-node first differences: central (f[j+1] - f[j-1]) / 2 inside, forward
// at node 0, backward at node n-1 (in units of 1/h).  Sec. II.B builds
// grad psi at an FOD this way.  Entries 0 and 5 stay zero whenever their
// node lies outside the grid (i0 is in [1, n-3]).
__device__ __forceinline__ void fd_interp_weights(const double *w, int i0, int n, double *e) {
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = i0 - 1 + q;  // node carrying weight w[q]; its slot is q + 1
        if (j == 0) {
            e[q + 2] += w[q];
            e[q + 1] -= w[q];
        } else if (j == n - 1) {
            e[q + 1] += w[q];
            e[q] -= w[q];
        } else {
            e[q + 2] += 0.5 * w[q];
            e[q] -= 0.5 * w[q];
        }
    }
}

// One block per FOD (or query point) i, one thread per orbital a < N (N <=
// 128): u = psi_a(a_i), du = grad psi_a(a_i), and, for the FOD path,
// rho(a_i) and T_i,a = u / sqrt(rho).  FD = false: du is the derivative of
// the cubic interpolant (the exact derivative of the discrete u); FD = true:
// du interpolates the per-node difference gradient.
template <bool FD>
__global__ __launch_bounds__(128) void k_interp(int N, int nx, int ny, int nz, double h,
                                                const double *psi, const FodCell *cells,
                                                double floor, double *u, double *du,
                                                double *rhoa, double *T, int *status) {
    __shared__ double sred[2];
    const int i = blockIdx.x;  // FOD
    const FodCell cl = cells[i];
    double wx[4], wy[4], wz[4], dx[4], dy[4], dz[4];
    cubic_weights(cl.t[0], wx, dx);
    cubic_weights(cl.t[1], wy, dy);
    cubic_weights(cl.t[2], wz, dz);
    const long long M = (long long)nx * ny * nz;
    const int a = threadIdx.x;
    double val = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    if (a < N && !FD) {
        const double *f = psi + (long long)a * M;
        for (int c = 0; c < 4; ++c) {
            for (int b = 0; b < 4; ++b) {
                const double *row = f + ((long long)(cl.i0[2] - 1 + c) * ny + (cl.i0[1] - 1 + b)) * nx + (cl.i0[0] - 1);
                double sx = 0.0, sdx = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    sx += wx[q] * row[q];
                    sdx += dx[q] * row[q];
                }
                val += wz[c] * wy[b] * sx;
                gx += wz[c] * wy[b] * sdx;
                gy += wz[c] * dy[b] * sx;
                gz += dz[c] * wy[b] * sx;
            }
        }
    } else if (a < N) {
        // six-node windows: value weights padded with zeros, difference weights
        double vx6[6] = {0.0, wx[0], wx[1], wx[2], wx[3], 0.0};
        double vy6[6] = {0.0, wy[0], wy[1], wy[2], wy[3], 0.0};
        double vz6[6] = {0.0, wz[0], wz[1], wz[2], wz[3], 0.0};
        double ex[6], ey[6], ez[6];
        fd_interp_weights(wx, cl.i0[0], nx, ex);
        fd_interp_weights(wy, cl.i0[1], ny, ey);
        fd_interp_weights(wz, cl.i0[2], nz, ez);
        int xs[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) xs[q] = min(max(cl.i0[0] - 2 + q, 0), nx - 1);
        const double *f = psi + (long long)a * M;
        for (int c = 0; c < 6; ++c) {
            const int kz = min(max(cl.i0[2] - 2 + c, 0), nz - 1);
            for (int b = 0; b < 6; ++b) {
                const int jy = min(max(cl.i0[1] - 2 + b, 0), ny - 1);
                const double *row = f + ((long long)kz * ny + jy) * nx;
                double sx = 0.0, sdx = 0.0;
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    const double fv = row[xs[q]];
                    sx += vx6[q] * fv;
                    sdx += ex[q] * fv;
                }
                val += vz6[c] * vy6[b] * sx;
                gx += vz6[c] * vy6[b] * sdx;
                gy += vz6[c] * ey[b] * sx;
                gz += ez[c] * vy6[b] * sx;
            }
        }
    }
    if (a < N) {
        const double ih = 1.0 / h;
        u[(size_t)i * N + a] = val;
        du[((size_t)i * N + a) * 3 + 0] = gx * ih;
        du[((size_t)i * N + a) * 3 + 1] = gy * ih;
        du[((size_t)i * N + a) * 3 + 2] = gz * ih;
    }
    // rho(a_i) = sum_a psi_a(a_i)^2 (occupations 1), fixed-order reduction
    double sq = (a < N) ? val * val : 0.0;
    sq = wave_sum(sq);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = sq;
    __syncthreads();
    const double rho = sred[0] + sred[1];
    if (a == 0) {
        rhoa[i] = rho;
        if (!(rho > floor)) atomicOr(status, kStVacuum);
        if (!isfinite(rho)) atomicOr(status, kStNonFinite);
    }
    if (a < N) T[(size_t)i * N + a] = (rho > floor) ? val / sqrt(rho) : 0.0;
}

hipError_t launch_interp(int K, int N, int nx, int ny, int nz, double h, const double *psi,
                         const FodCell *cells, double floor, double *u, double *du,
                         double *rhoa, double *T, int *status, bool fd_gradient, hipStream_t s) {
    if (K < 1 || N < 1 || N > 128) return hipErrorInvalidValue;
    if (fd_gradient)
        hipLaunchKernelGGL(k_interp<true>, dim3(K), dim3(128), 0, s, N, nx, ny, nz, h, psi, cells,
                           floor, u, du, rhoa, T, status);
    else
        hipLaunchKernelGGL(k_interp<false>, dim3(K), dim3(128), 0, s, N, nx, ny, nz, h, psi, cells,
                           floor, u, du, rhoa, T, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gram matrix G = dV psi psi^T on the matrix cores: k_tsg_nt<true>
// (tsgemm.h) for more than 32 orbitals, below for at most 32
// ---------------------------------------------------------------------------

// Small N (at most two 16-row tiles): the tile pairs t1 <= t2 of
// psi psi^T over the node range [b chunk, (b+1) chunk) of block b (chunk a
// multiple of 64).  Every wave forms all pairs over its own 16-node groups;
// lane (row r = l % 16, q = l / 16) holds nodes g + 4q .. g + 4q + 3 of row r
// (32 contiguous bytes: the four lanes of a row read one 128-byte line) and
// k-step j contracts node g + 4q + j; the four waves' tiles are added in
// LDS.  partG[b] holds the block's sums.
__global__ __launch_bounds__(256) void k_gram_small(int N, long long M, long long chunk, const double *psi,
                                                    int vec, double *partG) {
    const int Nt = (N + 15) >> 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row = lane & 15, kk = lane >> 4;
    const int np = Nt == 1 ? 1 : 3;  // pairs (0,0) [, (0,1), (1,1)]
    dbl4 acc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[q] = dbl4{0.0, 0.0, 0.0, 0.0};
    const long long m0 = (long long)blockIdx.x * chunk;
    const long long m1 = min(M, m0 + chunk);
    for (long long g = m0 + 16 * w; g < m1; g += 64) {
        const long long mb = g + 4 * kk;
        double f[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int r = 16 * t + row;
            const double *src = psi + (long long)r * M + mb;
            if (t < Nt && r < N && mb < m1) {
                if (vec && mb + 4 <= m1) {
                    const double2 lo = *reinterpret_cast<const double2 *>(src);
                    const double2 hi = *reinterpret_cast<const double2 *>(src + 2);
                    f[t][0] = lo.x; f[t][1] = lo.y; f[t][2] = hi.x; f[t][3] = hi.y;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) f[t][j] = mb + j < m1 ? src[j] : 0.0;
                }
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) f[t][j] = 0.0;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[0] = mfma16x16x4(f[0][j], f[0][j], acc[0]);
            if (np == 3) {
                acc[1] = mfma16x16x4(f[0][j], f[1][j], acc[1]);
                acc[2] = mfma16x16x4(f[1][j], f[1][j], acc[2]);
            }
        }
    }
    const int NP = Nt * 16;
    double *out = partG + (size_t)blockIdx.x * NP * NP;
    __shared__ double sacc[4][3][4][64];
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (q < np)
#pragma unroll
            for (int j = 0; j < 4; ++j) sacc[w][q][j][lane] = acc[q][j];
    __syncthreads();
    if (w != 0) return;
    const int pt1[3] = {0, 0, 1}, pt2[3] = {0, 1, 1};
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (q < np)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                // D lane l, item j: row l / 16 + 4 j, column l % 16
                const int r = 16 * pt1[q] + kk + 4 * j;
                const int c = 16 * pt2[q] + row;
                out[(size_t)r * NP + c] = (sacc[0][q][j][lane] + sacc[1][q][j][lane]) +
                                          (sacc[2][q][j][lane] + sacc[3][q][j][lane]);
            }
}


// G[i][j] = dV * sum over the blocks' partial tiles (the upper block triangle
// holds the tile pairs); one 256-thread block per element, fixed order
__global__ __launch_bounds__(256) void k_gram_final(int N, int nblk, double dV, const double *partG,
                                                    double *G) {
    __shared__ double sred[4];
    const int NP = ((N + 15) >> 4) * 16;
    const int e = blockIdx.x;
    int i = e / N, j = e % N;
    if ((i >> 4) > (j >> 4)) { const int t = i; i = j; j = t; }
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += partG[(size_t)b * NP * NP + (size_t)i * NP + j];
    s = block_sum256(s, sred);
    if (threadIdx.x == 0) G[e] = dV * s;
}

// partial-sum blocks for a node range split within the partial buffer (cap
// doubles): for the staged kernels four per compute unit (at most 1024) of
// at least four 32-node tiles; for the small-N ones up to 4096 of 64 nodes
int grid_blocks(int N, long long M, size_t cap) {
    const size_t NP = (size_t)((N + 15) >> 4) * 16;
    const bool small = NP <= 32;
    long long nb = (long long)std::min<size_t>(small ? 4096 : 1024, cap / (NP * NP));
    nb = std::min(nb, small ? (M + 63) / 64 : (M + 4 * kTK - 1) / (4 * kTK));
    return (int)std::max(1LL, nb);
}

hipError_t launch_gram(int N, long long M, double dV, const double *psi, double *partG, size_t cap,
                       double *G, hipStream_t s) {
    if (N < 1 || N > kMaxOrb) return hipErrorInvalidValue;
    const int nblk = grid_blocks(N, M, cap);
    long long chunk = (M + nblk - 1) / nblk;
    if (N <= 32) {
        chunk = (chunk + 63) & ~63LL;
        // 16-byte loads where every row start is 16-byte aligned
        const int vec = ((M & 1) == 0 && (reinterpret_cast<uintptr_t>(psi) & 15) == 0) ? 1 : 0;
        hipLaunchKernelGGL(k_gram_small, dim3(nblk), dim3(256), 0, s, N, M, chunk, psi, vec, partG);
    } else {
        chunk = (chunk + kTK - 1) / kTK * kTK;
        const size_t lds = tsg_lds_bytes(N, 1);
        if (lds > 65536)
            hipFuncSetAttribute((const void *)k_tsg_nt<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_tsg_nt<true>, dim3(nblk), dim3(256), lds, s, N, M, chunk, psi, psi, partG);
    }
    hipLaunchKernelGGL(k_gram_final, dim3(N * N), dim3(256), 0, s, N, nblk, dV, partG, G);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Loewdin: S = T G T^T, Jacobi, Z = S^{-1/2}, Q = Z T (one workgroup)
// ---------------------------------------------------------------------------

// C = A B (+ transposes) for N x N row-major matrices held anywhere (flat).
__device__ void small_gemm(int N, const double *A, int ta, const double *B, int tb, double *C,
                           double alpha) {
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        double s = 0.0;
        for (int k = 0; k < N; ++k) {
            const double a = ta ? A[k * N + i] : A[i * N + k];
            const double b = tb ? B[j * N + k] : B[k * N + j];
            s += a * b;
        }
        C[e] = alpha * s;
    }
}

__device__ __forceinline__ void lowdin_one(int N, int Ne, const double *T, const double *G,
                                           double *S, double *lam, double *U, double *Z,
                                           double *Qm, double *work, int lds_mode,
                                           double eig_floor, int *status, double *info) {
    extern __shared__ double dsm[];
    __shared__ double rc[kMaxOrb / 2], rs_[kMaxOrb / 2];
    __shared__ int rp[kMaxOrb / 2], rq[kMaxOrb / 2];
    __shared__ double sred[4];
    __shared__ int sflag;
    // A (Ne x Ne) and V (Ne x Ne) in LDS or in work
    double *A = (lds_mode >= 1) ? dsm : work;
    double *V = (lds_mode >= 2) ? dsm + Ne * Ne : work + Ne * Ne;
    double *TG = work + 2 * Ne * Ne;  // N x N scratch
    // TG = T G
    small_gemm(N, T, 0, G, 0, TG, 1.0);
    __syncthreads();
    // S = TG T^T, exactly symmetric, padded to Ne with the identity
    for (int e = threadIdx.x; e < Ne * Ne; e += 256) {
        const int i = e / Ne, j = e % Ne;
        double v;
        if (i < N && j < N) {
            const int a = min(i, j), b = max(i, j);
            double s = 0.0;
            for (int k = 0; k < N; ++k) s += TG[a * N + k] * T[b * N + k];
            v = s;
            S[i * N + j] = v;
        } else {
            v = (i == j) ? 1.0 : 0.0;
        }
        A[e] = v;
        V[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int half = Ne / 2;
    for (int sweep = 0; sweep < 40; ++sweep) {
        // convergence: off-diagonal vs diagonal mass
        double off = 0.0, dg = 0.0;
        for (int e = threadIdx.x; e < Ne * Ne; e += 256) {
            const int i = e / Ne, j = e % Ne;
            const double a = A[e];
            if (i == j) dg += a * a; else off += a * a;
        }
        off = block_sum256(off, sred);
        dg = block_sum256(dg, sred);
        if (off <= 1e-30 * dg) break;
        for (int r = 0; r < Ne - 1; ++r) {
            // round-robin pairing: position 0 holds index 0, positions 1..Ne-1
            // hold 1..Ne-1 rotated by r; pair position j with Ne-1-j
            if (threadIdx.x < half) {
                const int j = threadIdx.x;
                auto at = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + r) % (Ne - 1)) + 1; };
                int p = at(j), q = at(Ne - 1 - j);
                if (p > q) { const int t = p; p = q; q = t; }
                const double apq = A[p * Ne + q], app = A[p * Ne + p], aqq = A[q * Ne + q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0 && fabs(apq) > 1e-300) {
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                rp[j] = p; rq[j] = q; rc[j] = c; rs_[j] = s;
            }
            __syncthreads();
            // A <- J^T A J by 2 x 2 blocks (rows of pair i, columns of pair
            // j: the blocks are disjoint, so each updates in place; rows
            // first, then columns), the rotated pair's own entry set to
            // zero; V <- V J by rows
            const int nA = half * half;
            for (int e = threadIdx.x; e < nA + Ne * half; e += 256) {
                if (e < nA) {
                    const int bi = e / half, bj = e - bi * half;
                    const int pi = rp[bi], qi = rq[bi], pj = rp[bj], qj = rq[bj];
                    const double ci = rc[bi], si = rs_[bi], cj = rc[bj], sj = rs_[bj];
                    const double a_pp = A[pi * Ne + pj], a_pq = A[pi * Ne + qj];
                    const double a_qp = A[qi * Ne + pj], a_qq = A[qi * Ne + qj];
                    const double r_pp = ci * a_pp - si * a_qp, r_pq = ci * a_pq - si * a_qq;
                    const double r_qp = si * a_pp + ci * a_qp, r_qq = si * a_pq + ci * a_qq;
                    double o_pq = sj * r_pp + cj * r_pq, o_qp = cj * r_qp - sj * r_qq;
                    if (bi == bj && si != 0.0) o_pq = o_qp = 0.0;
                    A[pi * Ne + pj] = cj * r_pp - sj * r_pq;
                    A[pi * Ne + qj] = o_pq;
                    A[qi * Ne + pj] = o_qp;
                    A[qi * Ne + qj] = sj * r_qp + cj * r_qq;
                } else {
                    const int e2 = e - nA, rw = e2 / half, j = e2 - rw * half;
                    const int p = rp[j], q = rq[j];
                    const double c = rc[j], s = rs_[j];
                    const double vp = V[rw * Ne + p], vq = V[rw * Ne + q];
                    V[rw * Ne + p] = c * vp - s * vq;
                    V[rw * Ne + q] = s * vp + c * vq;
                }
            }
            __syncthreads();
        }
    }
    // eigenvalues, condition number, singularity test
    if (threadIdx.x == 0) sflag = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += 256) lam[i] = A[i * Ne + i];
    for (int e = threadIdx.x; e < N * N; e += 256) U[e] = V[(e / N) * Ne + (e % N)];
    __syncthreads();
    if (threadIdx.x == 0) {
        double mn = lam[0], mx = lam[0];
        for (int i = 1; i < N; ++i) { mn = fmin(mn, lam[i]); mx = fmax(mx, lam[i]); }
        info[0] = mx / mn;
        info[1] = mn;
        if (!(mn > eig_floor)) { atomicOr(status, kStSingular); sflag = 1; }
    }
    __syncthreads();
    if (sflag) return;
    // Z = U diag(lam^{-1/2}) U^T ; Q = Z T
    double *W = work + 2 * Ne * Ne;
    for (int e = threadIdx.x; e < N * N; e += 256) W[e] = U[e] / sqrt(lam[e % N]);
    __syncthreads();
    small_gemm(N, W, 0, U, 1, Z, 1.0);
    __syncthreads();
    small_gemm(N, Z, 0, T, 0, Qm, 1.0);
}

__global__ __launch_bounds__(256) void k_lowdin(int N, int Ne, const double *T, const double *G,
                                                double *S, double *lam, double *U, double *Z,
                                                double *Qm, double *work, int lds_mode,
                                                double eig_floor, int *status, double *info) {
    lowdin_one(N, Ne, T, G, S, lam, U, Z, Qm, work, lds_mode, eig_floor, status, info);
}

// one workgroup per channel: channel b's arrays sit at small + so[b] + the
// given offsets, its scratch at work + b * wstride
__global__ __launch_bounds__(256) void k_lowdin_batch(LowdinBatch lb, double *small, LowdinOffsets off,
                                                      double *work, long long wstride, int lds_mode,
                                                      double eig_floor, int *status) {
    const int b = blockIdx.x;
    const int N = lb.N[b], Ne = N + (N & 1);
    double *sm = small + lb.so[b];
    lowdin_one(N, Ne, sm + off.T, sm + off.G, sm + off.S, sm + off.lam, sm + off.U, sm + off.Z,
               sm + off.Q, work + (size_t)b * wstride, lds_mode, eig_floor, status, sm + off.info);
}

// LDS mode of the Loewdin kernels for channels of up to N orbitals: 2 keeps
// A and V in LDS, 1 only A, 0 neither (then both live in the scratch)
static int lowdin_lds(int N, size_t &dyn) {
    const int Ne = N + (N & 1);
    int dev = 0;
    hipGetDevice(&dev);
    int maxsh = 0;
    hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    const size_t static_bytes = 4 * 64 * 8 + 64;  // rotation tables, reductions
    const size_t need1 = (size_t)Ne * Ne * sizeof(double);
    dyn = 0;
    if (2 * need1 + static_bytes <= (size_t)maxsh) { dyn = 2 * need1; return 2; }
    if (need1 + static_bytes <= (size_t)maxsh) { dyn = need1; return 1; }
    return 0;
}

hipError_t launch_lowdin(int N, const double *T, const double *G, double *S, double *lam,
                         double *U, double *Z, double *Qm, double *work, double eig_floor,
                         int *status, double *info, hipStream_t s) {
    const int Ne = N + (N & 1);
    size_t dyn = 0;
    const int mode = lowdin_lds(N, dyn);
    if (dyn > 65536) hipFuncSetAttribute((const void *)k_lowdin, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    hipLaunchKernelGGL(k_lowdin, dim3(1), dim3(256), dyn, s, N, Ne, T, G, S, lam, U, Z, Qm, work,
                       mode, eig_floor, status, info);
    return hipGetLastError();
}

hipError_t launch_lowdin_batch(const LowdinBatch &lb, double *small, const LowdinOffsets &off,
                               double *work, long long wstride, double eig_floor, int *status,
                               hipStream_t s) {
    if (lb.n <= 0 || lb.n > kLowdinBatch) return hipErrorInvalidValue;
    int nmax = 1;
    for (int b = 0; b < lb.n; ++b) nmax = std::max(nmax, lb.N[b]);
    size_t dyn = 0;
    const int mode = lowdin_lds(nmax, dyn);
    if (dyn > 65536)
        hipFuncSetAttribute((const void *)k_lowdin_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    hipLaunchKernelGGL(k_lowdin_batch, dim3(lb.n), dim3(256), dyn, s, lb, small, off, work, wstride, mode,
                       eig_floor, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// out = A psi  (N x N times N x M) on the matrix cores: k_tsg_nn (tsgemm.h)
// for more than 32 orbitals; for at most 32 each wave takes 16-node strips
// and all output rows, A read through the cache
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_orb_gemm(int N, long long M, const double *A,
                                                  const double *psi, double *out) {
    const int Nt = (N + 15) >> 4;
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kk = lane >> 4;
    const long long nstrip = (M + 15) >> 4;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwave = ((long long)gridDim.x * blockDim.x) >> 6;
    // N <= 16: the 16-row A fragments stay in registers and each pass takes
    // two strips, whose psi loads are all issued before the products
    if (Nt == 1) {
        double af[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int a = 4 * q + kk;
            af[q] = (row < N && a < N) ? A[row * N + a] : 0.0;
        }
        for (long long st = wave; st < nstrip; st += 2 * nwave) {
            const long long ms[2] = {st * 16 + row, (st + nwave) * 16 + row};
            double b[2][4];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int a = 4 * q + kk;
                    b[u][q] = (a < N && ms[u] < M) ? psi[(long long)a * M + ms[u]] : 0.0;
                }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < 4; ++q) acc = mfma16x16x4(af[q], b[u][q], acc);
                if (ms[u] < M)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int i = kk + 4 * j;
                        if (i < N) out[(long long)i * M + ms[u]] = acc[j];
                    }
            }
        }
        return;
    }
    for (long long st = wave; st < nstrip; st += nwave) {
        const long long m = st * 16 + row;
        dbl4 acc[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
        for (int a0 = 0; a0 < N; a0 += 4) {
            const int a = a0 + kk;
            const double b = (a < N && m < M) ? psi[(long long)a * M + m] : 0.0;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (t < Nt) {
                    const int i = 16 * t + row;
                    const double av = (i < N && a < N) ? A[i * N + a] : 0.0;
                    acc[t] = mfma16x16x4(av, b, acc[t]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (t < Nt && m < M) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i = 16 * t + kk + 4 * j;
                    if (i < N) out[(long long)i * M + m] = acc[t][j];
                }
            }
        }
    }
}

// fp32 variant: A and psi rounded to fp32, products accumulated in fp32 on
// v_mfma_f32_16x16x4f32 (D lane l, item j: row 4 (l/16) + j), out in fp64
typedef float flt4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_orb_gemm32(int N, long long M, const double *A,
                                                    const double *psi, double *out) {
    const int Nt = (N + 15) >> 4;
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kk = lane >> 4;
    const long long nstrip = (M + 15) >> 4;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwave = ((long long)gridDim.x * blockDim.x) >> 6;
    for (long long st = wave; st < nstrip; st += nwave) {
        const long long m = st * 16 + row;
        flt4 acc[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = flt4{0.f, 0.f, 0.f, 0.f};
        for (int a0 = 0; a0 < N; a0 += 4) {
            const int a = a0 + kk;
            const float b = (a < N && m < M) ? (float)psi[(long long)a * M + m] : 0.f;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (t < Nt) {
                    const int i = 16 * t + row;
                    const float av = (i < N && a < N) ? (float)A[i * N + a] : 0.f;
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b, acc[t], 0, 0, 0);
                }
            }
        }
        const long long mo = st * 16 + row;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (t < Nt && mo < M) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i = 16 * t + 4 * kk + j;
                    if (i < N) out[(long long)i * M + mo] = (double)acc[t][j];
                }
            }
        }
    }
}

hipError_t launch_orb_gemm32(int N, long long M, const double *A, const double *psi, double *out,
                             hipStream_t s) {
    const long long nstrip = (M + 15) / 16;
    long long nblk = (nstrip + 3) / 4;
    if (nblk > 8192) nblk = 8192;
    hipLaunchKernelGGL(k_orb_gemm32, dim3((unsigned)nblk), dim3(256), 0, s, N, M, A, psi, out);
    return hipGetLastError();
}

hipError_t launch_orb_gemm(int N, long long M, const double *A, const double *psi, double *out,
                           hipStream_t s) {
    if (N < 1 || N > kMaxOrb) return hipErrorInvalidValue;
    if (N <= 32) {
        const long long nstrip = (M + 15) / 16;
        const long long nblk = std::max(1LL, std::min((nstrip + 3) / 4, 8192LL));
        hipLaunchKernelGGL(k_orb_gemm, dim3((unsigned)nblk), dim3(256), 0, s, N, M, A, psi, out);
        return hipGetLastError();
    }
    const long long ntile = (M + kTK - 1) / kTK;
    const long long nblk = std::max(1LL, std::min(ntile, 512LL));  // two per compute unit
    const size_t lds = (size_t)16 * ((N + 15) / 16) * kTKS * sizeof(double);  // at most 33 KiB
    if (N <= 64)
        hipLaunchKernelGGL((k_tsg_nn<1, 16>), dim3((unsigned)nblk), dim3(256), lds, s, N, M, A, psi, out);
    else
        hipLaunchKernelGGL((k_tsg_nn<2, 32>), dim3((unsigned)nblk), dim3(256), lds, s, N, M, A, psi, out);
    return hipGetLastError();
}

}  // namespace fsic
