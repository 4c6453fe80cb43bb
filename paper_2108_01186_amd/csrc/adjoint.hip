// Reverse-mode FOD gradient of the discrete SIC energy (the FOD forces of
// Eq. 9-11, in exact form for this discretisation).
//
// With v_i = A rho_i, A = K^{-1} (4 pi I + C E_g P) (K = -L, C: ghost values
// into the right-hand side, E_g: moments to ghost values, P: density to
// moments), U_i = dV/2 rho_i^T A rho_i and dE_xc/drho = dV v_xc:
//   dE/dphi_i = Gam_i = 2 dV phi_i omega_i,
//   omega_i = -( (v_i + A^T rho_i) / 2 + v_xc(rho_i) ),
//   A^T rho = w' + dV sum_lm zt_lm r^l Y_lm,  K w' = 4 pi rho,
//   zt_lm = (1 / 4 pi) sum_ghost 4 pi/(2l+1) Y_lm / r^(l+1) (C^T w')_ghost.
// phi = Q psi gives B = Gam psi^T (one grid-sized contraction on the FP64
// matrix cores); the rest is N x N: Q = Z T, Z = S^{-1/2} (Daleckii-Krein
// form of the derivative of the inverse square root), S = T G T^T,
// T_i = u_i / |u_i|, u_i,a = psi_a(a_i) (cubic interpolant).
#include <algorithm>
#include <cstdint>

#include "kernels.h"
#include "lsda.h"
#include "tsgemm.h"

namespace fsic {


// Small N (at most two 16-row tiles): B[i][a] = sum_m Gam_i(m) psi_a(m),
// Gam formed on the fly; block b sums the node range [b chunk, (b+1) chunk)
// (chunk a multiple of 64).  Every wave forms all the tiles over its own
// 16-node groups; lane (row r = l % 16, q = l / 16) holds nodes g + 4q ..
// g + 4q + 3 of row r (32 contiguous bytes: the four lanes of a row read one
// 128-byte line), and k-step j of a group contracts node g + 4q + j (any
// assignment of nodes to k-steps splits the sum, as long as both operands
// use the same one).  The four waves' tiles are added in LDS at the end.
__global__ __launch_bounds__(256) void k_adj_contract_small(int N, long long M, long long chunk, double dV,
                                                            const double *PHI, const double *V,
                                                            const double *W, const double *psi,
                                                            double floor, int vec, double *partB) {
    const int Nt = (N + 15) >> 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row = lane & 15, kk = lane >> 4;
    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[a][t] = dbl4{0.0, 0.0, 0.0, 0.0};
    const long long m0 = (long long)blockIdx.x * chunk;
    const long long m1 = min(M, m0 + chunk);
    // four consecutive values of row i from node mb (zero past m1)
    auto load4 = [&](const double *X, int i, long long mb, double (&v)[4]) {
        const double *src = X + (long long)i * M + mb;
        if (vec && mb + 4 <= m1) {
            const double2 lo = *reinterpret_cast<const double2 *>(src);
            const double2 hi = *reinterpret_cast<const double2 *>(src + 2);
            v[0] = lo.x; v[1] = lo.y; v[2] = hi.x; v[3] = hi.y;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = mb + j < m1 ? src[j] : 0.0;
        }
    };
    for (long long g = m0 + 16 * w; g < m1; g += 64) {
        const long long mb = g + 4 * kk;
        double gam[2][4], f[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int i = 16 * a + row;
#pragma unroll
            for (int j = 0; j < 4; ++j) gam[a][j] = 0.0;
            if (a < Nt && i < N && mb < m1) {
                double ph[4], vv[4], ww[4];
                load4(PHI, i, mb, ph);
                load4(V, i, mb, vv);
                load4(W, i, mb, ww);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double om = -(0.5 * (vv[j] + ww[j]) + vxc_pol(ph[j] * ph[j], floor));
                    gam[a][j] = 2.0 * dV * ph[j] * om;  // zero past m1 (ph = 0 there)
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int r = 16 * t + row;
            if (t < Nt && r < N && mb < m1) load4(psi, r, mb, f[t]);
            else
#pragma unroll
                for (int j = 0; j < 4; ++j) f[t][j] = 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                if (a < Nt)
#pragma unroll
                    for (int t = 0; t < 2; ++t)
                        if (t < Nt) acc[a][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(gam[a][j], f[t][j], acc[a][t], 0, 0, 0);
    }
    const int NP = Nt * 16;
    double *out = partB + (size_t)blockIdx.x * NP * NP;
    __shared__ double sacc[4][4][4][64];  // wave, tile (a, t), item, lane
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int t = 0; t < 2; ++t)
            if (a < Nt && t < Nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) sacc[w][2 * a + t][j][lane] = acc[a][t][j];
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int t = 0; t < 2; ++t)
            if (a < Nt && t < Nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // D layout of the f64 16x16x4 MFMA: lane l, item j -> row l/16 + 4 j, col l % 16
                    const int r = 16 * a + kk + 4 * j;
                    const int c = 16 * t + row;
                    out[(size_t)r * NP + c] = (sacc[0][2 * a + t][j][lane] + sacc[1][2 * a + t][j][lane]) +
                                              (sacc[2][2 * a + t][j][lane] + sacc[3][2 * a + t][j][lane]);
                }
}

// Gam_i(m) = 2 dV phi_i omega_i, omega_i = -((v_i + w_i) / 2 + vxc(phi_i^2)),
// over the channel's N x M values (Gam may be W: each value is read before
// it is written, by the same thread)
__global__ __launch_bounds__(256) void k_gamma(long long count, double dV, const double *PHI,
                                               const double *V, const double *W, double floor,
                                               double *Gam) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long long)gridDim.x * 256) {
        const double ph = PHI[i];
        const double om = -(0.5 * (V[i] + W[i]) + vxc_pol(ph * ph, floor));
        Gam[i] = 2.0 * dV * ph * om;
    }
}

// Bm[i][j] = sum of the blocks' partial tiles; one 256-thread block per element
__global__ __launch_bounds__(256) void k_adj_contract_final(int N, int nblk, const double *partB,
                                                            double *Bm) {
    __shared__ double sred[4];
    const int NP = ((N + 15) >> 4) * 16;
    const int e = blockIdx.x;
    const int i = e / N, j = e % N;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += partB[(size_t)b * NP * NP + (size_t)i * NP + j];
    s = block_sum256(s, sred);
    if (threadIdx.x == 0) Bm[e] = s;
}

// C = op(A) op(B) for N x N row-major matrices (flat pointers)
__device__ void nn_gemm(int N, const double *A, int ta, const double *B, int tb, double *C) {
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        double s = 0.0;
        for (int k = 0; k < N; ++k) {
            const double a = ta ? A[k * N + i] : A[i * N + k];
            const double b = tb ? B[j * N + k] : B[k * N + j];
            s += a * b;
        }
        C[e] = s;
    }
}

// Reverse mode through Q = Z T, Z = S^{-1/2}, S = T G T^T, T_i = u_i/|u_i|.
//   Gam_T  = Z^T B + 2 Gam_S T G          (Gam_Q = B)
//   Gam_Z  = B T^T
//   Gam_S  = U [(U^T sym(Gam_Z) U) o K] U^T,
//            K_jk = -1 / (sqrt(l_j) sqrt(l_k) (sqrt(l_j) + sqrt(l_k)))
//   Gam_u_i = (Gam_T_i - (Gam_T_i . T_i) T_i) / |u_i|
//   dE/da_i = sum_a Gam_u_i,a grad psi_a(a_i)
__device__ __forceinline__ void lowdin_backward_one(int N, const double *Bm, const double *T,
                                                       const double *G, const double *lam,
                                                       const double *U, const double *Z,
                                                       const double *rhoa, const double *du,
                                                       double *work, double *dEda) {
    const size_t NN = (size_t)N * N;
    double *GT = work;            // Gam_T
    double *T1 = work + NN;
    double *T2 = work + 2 * NN;
    double *T3 = work + 3 * NN;
    // Gam_Z = B T^T, symmetrised
    nn_gemm(N, Bm, 0, T, 1, T1);
    __syncthreads();
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        T2[e] = 0.5 * (T1[i * N + j] + T1[j * N + i]);
    }
    __syncthreads();
    // U^T sym U, times K
    nn_gemm(N, U, 1, T2, 0, T1);
    __syncthreads();
    nn_gemm(N, T1, 0, U, 0, T3);
    __syncthreads();
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int j = e / N, k = e % N;
        const double sj = sqrt(lam[j]), sk = sqrt(lam[k]);
        T3[e] *= -1.0 / (sj * sk * (sj + sk));
    }
    __syncthreads();
    // Gam_S = U T3 U^T
    nn_gemm(N, U, 0, T3, 0, T1);
    __syncthreads();
    nn_gemm(N, T1, 0, U, 1, T2);  // T2 = Gam_S
    __syncthreads();
    // Gam_T = Z^T B + 2 Gam_S T G
    nn_gemm(N, Z, 1, Bm, 0, GT);
    __syncthreads();
    nn_gemm(N, T2, 0, T, 0, T1);
    __syncthreads();
    nn_gemm(N, T1, 0, G, 0, T3);
    __syncthreads();
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) GT[e] += 2.0 * T3[e];
    __syncthreads();
    // Gam_u and dE/da
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double dot = 0.0;
        for (int a = 0; a < N; ++a) dot += GT[i * N + a] * T[i * N + a];
        const double inv = 1.0 / sqrt(rhoa[i]);
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int a = 0; a < N; ++a) {
            const double gu = (GT[i * N + a] - dot * T[i * N + a]) * inv;
            gx += gu * du[((size_t)i * N + a) * 3 + 0];
            gy += gu * du[((size_t)i * N + a) * 3 + 1];
            gz += gu * du[((size_t)i * N + a) * 3 + 2];
        }
        dEda[3 * i + 0] = gx;
        dEda[3 * i + 1] = gy;
        dEda[3 * i + 2] = gz;
    }
}

// the reverse Loewdin step of up to kLowdinBatch channels in one launch, one
// workgroup each: channel b's B at Bm + b N_max^2 stride, its small arrays at
// small + so[b], scratch at work + b wstride; dE/da to its small block and to
// packed + go[b] (all channels' gradients in one block for one copy)
__global__ __launch_bounds__(256) void k_lowdin_backward_batch(LowdinBwdBatch lb, const double *Bm, long long bstride,
                                                               double *small, LowdinBwdOffsets off, double *work,
                                                               long long wstride, double *packed) {
    const int b = blockIdx.x;
    const int N = lb.N[b];
    double *sm = small + lb.so[b];
    double *dEda = sm + off.dEda;
    lowdin_backward_one(N, Bm + (size_t)b * bstride, sm + off.T, sm + off.G, sm + off.lam, sm + off.U,
                           sm + off.Z, sm + off.rhoa, sm + off.du, work + (size_t)b * wstride, dEda);
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) packed[lb.go[b] + e] = dEda[e];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_lowdin_backward_batch(const LowdinBwdBatch &lb, const double *Bm, long long bstride, double *small,
                                        const LowdinBwdOffsets &off, double *work, long long wstride, double *packed,
                                        hipStream_t s) {
    if (lb.n <= 0 || lb.n > kLowdinBatch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lowdin_backward_batch, dim3(lb.n), dim3(256), 0, s, lb, Bm, bstride, small, off, work,
                       wstride, packed);
    return hipGetLastError();
}

hipError_t launch_adjoint_contract(int N, long long M, double dV, const double *PHI, const double *V,
                                    const double *W, const double *psi, double floor, double *partB,
                                    size_t cap, double *Bm, double *Gam, hipStream_t s) {
    if (N < 1 || N > kMaxOrb) return hipErrorInvalidValue;
    const int nblk = grid_blocks(N, M, cap);
    long long chunk = (M + nblk - 1) / nblk;
    if (N <= 32) {  // Gam built on the fly
        chunk = (chunk + 63) & ~63LL;
        // 16-byte loads where every row start is 16-byte aligned
        const int vec = ((M & 1) == 0 && ((reinterpret_cast<uintptr_t>(PHI) | reinterpret_cast<uintptr_t>(V) |
                                           reinterpret_cast<uintptr_t>(W) | reinterpret_cast<uintptr_t>(psi)) &
                                          15) == 0)
                            ? 1
                            : 0;
        hipLaunchKernelGGL(k_adj_contract_small, dim3(nblk), dim3(256), 0, s, N, M, chunk, dV, PHI, V, W, psi,
                           floor, vec, partB);
        hipLaunchKernelGGL(k_adj_contract_final, dim3(N * N), dim3(256), 0, s, N, nblk, partB, Bm);
        return hipGetLastError();
    }
    const long long count = (long long)N * M;
    const long long gblk = std::max(1LL, std::min((count + 255) / 256, 4096LL));
    hipLaunchKernelGGL(k_gamma, dim3((unsigned)gblk), dim3(256), 0, s, count, dV, PHI, V, W, floor, Gam);
    chunk = (chunk + kTK - 1) / kTK * kTK;
    const size_t lds = tsg_lds_bytes(N, 2);
    if (lds > 65536) hipFuncSetAttribute((const void *)k_tsg_nt<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_tsg_nt<false>, dim3(nblk), dim3(256), lds, s, N, M, chunk, Gam, psi, partB);
    hipLaunchKernelGGL(k_adj_contract_final, dim3(N * N), dim3(256), 0, s, N, nblk, partB, Bm);
    return hipGetLastError();
}

}  // namespace fsic
