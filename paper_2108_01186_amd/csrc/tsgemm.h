// Tall-skinny FP64 products over the grid on the matrix cores: the overlap
// Gram matrix G = dV psi psi^T and the adjoint contraction B = Gam psi^T
// (N x M times M x N, a reduction over the M grid nodes), and the orbital
// transform phi = Q psi (N x N times N x M).  Eq. 6-8 and Sec. I.B give the
// products; N <= 128 orbitals of one spin channel, M up to 2^29 nodes.
//
// Design (gfx950, v_mfma_f64_16x16x4f64): a block stages 32-node tiles of
// its operands in LDS with coalesced row loads (one 256-byte run per
// orbital row); the loads of the next tile are in flight in registers while
// the four waves multiply the current one.  Reductions write one partial
// N x N tile per block, added afterwards in block order (bitwise
// reproducible).
#pragma once

#include "kernels.h"

namespace fsic {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kTK = 32;       // nodes per staged tile
constexpr int kTKS = kTK + 1;  // LDS row stride (odd: conflict-free column reads)

// this thread's share of a [NP][kTK] tile of rows r < N of X (row stride M),
// nodes [n0, n1): element e = threadIdx.x + 256 i is row e / kTK, node e % kTK
template <int RI>
__device__ __forceinline__ void tsg_load(const double *__restrict__ X, int N, int NP, long long M, long long n0,
                                         long long n1, double (&reg)[RI]) {
#pragma unroll
    for (int i = 0; i < RI; ++i) {
        const int e = threadIdx.x + 256 * i;
        const int r = e / kTK;
        const long long m = n0 + (e % kTK);
        reg[i] = (r < NP && r < N && m < n1) ? X[(long long)r * M + m] : 0.0;
    }
}

template <int RI>
__device__ __forceinline__ void tsg_store(double *S, int NP, const double (&reg)[RI]) {
#pragma unroll
    for (int i = 0; i < RI; ++i) {
        const int e = threadIdx.x + 256 * i;
        const int r = e / kTK;
        if (r < NP) S[r * kTKS + (e % kTK)] = reg[i];
    }
}

// part[b] = sum over the nodes [b chunk, (b+1) chunk) of X_i(m) Y_j(m) as an
// NP x NP tile (NP = 16 ceil(N / 16)).  SYM: Y = X and only the tile pairs
// t1 <= t2 are formed (the reader mirrors the rest).  Wave w owns row tiles
// t1 = w and (SYM) NT-1-w when that is above 3, or (else) w + 4, each against
// every column tile;
// with at most two row tiles every wave forms all of them over a quarter of
// the k-steps instead and the four partial tiles are added in LDS.
// Dynamic LDS: NP x kTKS doubles (SYM) or twice that.
template <bool SYM>
__global__ __launch_bounds__(256) void k_tsg_nt(int N, long long M, long long chunk, const double *X,
                                                const double *Y, double *part) {
    extern __shared__ double lds[];
    const int NT = (N + 15) >> 4, NP = 16 * NT;
    double *Xs = lds;
    double *Ys = SYM ? lds : lds + NP * kTKS;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    const bool ksplit = NT <= 2;
    int t1[2];
    if (ksplit) {
        t1[0] = 0;
        t1[1] = NT > 1 ? 1 : 8;
    } else if (SYM) {
        // rows w and (beyond the four primary rows) NT - 1 - w: the longer
        // and the shorter row of the tile triangle
        t1[0] = w < NT ? w : 8;
        t1[1] = (NT - 1 - w >= 4) ? NT - 1 - w : 8;
    } else {
        t1[0] = w < NT ? w : 8;
        t1[1] = w + 4 < NT ? w + 4 : 8;
    }
    dbl4 acc[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[a][t] = dbl4{0.0, 0.0, 0.0, 0.0};
    const long long m0 = (long long)blockIdx.x * chunk;
    const long long m1 = min(M, m0 + chunk);
    double xr[16], yr[SYM ? 1 : 16];
    if (m0 < m1) {
        tsg_load(X, N, NP, M, m0, m1, xr);
        if constexpr (!SYM) tsg_load(Y, N, NP, M, m0, m1, yr);
    }
    for (long long n0 = m0; n0 < m1; n0 += kTK) {
        tsg_store(Xs, NP, xr);
        if constexpr (!SYM) tsg_store(Ys, NP, yr);
        __syncthreads();
        if (n0 + kTK < m1) {  // next tile in flight during the products
            tsg_load(X, N, NP, M, n0 + kTK, m1, xr);
            if constexpr (!SYM) tsg_load(Y, N, NP, M, n0 + kTK, m1, yr);
        }
#pragma unroll
        for (int ks = 0; ks < kTK / 4; ++ks) {
            if (ksplit && (ks & 3) != w) continue;  // uniform
            const int k = 4 * ks + lk;
            double fy[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) fy[t] = t < NT ? Ys[(16 * t + lr) * kTKS + k] : 0.0;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                if (t1[a] < NT) {  // uniform
                    const double fx = Xs[(16 * t1[a] + lr) * kTKS + k];
#pragma unroll
                    for (int t = 0; t < 8; ++t)
                        if (t < NT && (!SYM || t >= t1[a]))
                            acc[a][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(fx, fy[t], acc[a][t], 0, 0, 0);
                }
            }
        }
        __syncthreads();  // products done with the tile
    }
    double *out = part + (size_t)blockIdx.x * NP * NP;
    if (ksplit) {
        // the four waves' tiles (at most 2 x 2 of them) added in LDS, wave order
        double *sacc = lds;  // [4 waves][4 tiles][4 items][64 lanes], fits NP x kTKS
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) sacc[((w * 4 + 2 * a + t) * 4 + j) * 64 + lane] = acc[a][t][j];
        __syncthreads();
        if (w != 0) return;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    double s = 0.0;
#pragma unroll
                    for (int v = 0; v < 4; ++v) s += sacc[((v * 4 + 2 * a + t) * 4 + j) * 64 + lane];
                    acc[a][t][j] = s;
                }
    }
    // D lane l, item j: row 16 t1 + l / 16 + 4 j, column 16 t + l % 16
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        if (t1[a] >= NT) continue;
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (t < NT && (!SYM || t >= t1[a]))
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    out[(size_t)(16 * t1[a] + lk + 4 * j) * NP + 16 * t + lr] = acc[a][t][j];
    }
}

// out[i][m] = sum_a A[i][a] X[a][m] (A: N x N row-major).  Wave w owns row
// tiles w and (RT = 2) w + 4 and holds their A fragments (KSM k-steps of 4)
// in registers for the whole launch; a block stages 32-node tiles of X in
// LDS (next tile in flight) and writes 16 x 16 result tiles straight from
// the accumulators.  Grid-stride over the node tiles.  RT = 1, KSM = 16
// serves N <= 64, RT = 2, KSM = 32 N <= 128.  Dynamic LDS: NP x kTKS doubles.
template <int RT, int KSM>
__global__ __launch_bounds__(256) void k_tsg_nn(int N, long long M, const double *A, const double *X,
                                                double *out) {
    extern __shared__ double lds[];
    const int NT = (N + 15) >> 4, NP = 16 * NT;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    int t1[RT];
#pragma unroll
    for (int a = 0; a < RT; ++a) t1[a] = w + 4 * a < NT ? w + 4 * a : 8;
    // A fragment of k-step ks: A[16 t1 + lr][4 ks + lk]
    double fa[RT][KSM];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int ks = 0; ks < KSM; ++ks) {
            const int i = 16 * t1[a] + lr, c = 4 * ks + lk;
            fa[a][ks] = (t1[a] < NT && i < N && c < N) ? A[i * N + c] : 0.0;
        }
    const long long ntile = (M + kTK - 1) / kTK;
    double xr[16];
    long long tile = blockIdx.x;
    if (tile < ntile) tsg_load(X, N, NP, M, tile * kTK, min(M, (tile + 1) * kTK), xr);
    for (; tile < ntile; tile += gridDim.x) {
        const long long n0 = tile * kTK;
        tsg_store(lds, NP, xr);
        __syncthreads();
        const long long nt = tile + gridDim.x;
        if (nt < ntile) tsg_load(X, N, NP, M, nt * kTK, min(M, (nt + 1) * kTK), xr);
        dbl4 acc[RT][2];
#pragma unroll
        for (int a = 0; a < RT; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) acc[a][c] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KSM; ++ks) {
            if (4 * ks >= NP) break;  // uniform
            double fb[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) fb[c] = lds[(4 * ks + lk) * kTKS + 16 * c + lr];
#pragma unroll
            for (int a = 0; a < RT; ++a)
                if (t1[a] < NT)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a][ks], fb[c], acc[a][c], 0, 0, 0);
        }
        // D lane l, item j: row 16 t1 + l / 16 + 4 j, node n0 + 16 c + l % 16
#pragma unroll
        for (int a = 0; a < RT; ++a) {
            if (t1[a] >= NT) continue;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const long long m = n0 + 16 * c + lr;
                if (m >= M) continue;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i = 16 * t1[a] + lk + 4 * j;
                    if (i < N) out[(long long)i * M + m] = acc[a][c][j];
                }
            }
        }
        __syncthreads();  // products done with the tile
    }
}

// dynamic LDS bytes of the kernels above for N orbitals (two operands: x2);
// k_tsg_nt with at most two row tiles also adds the waves' tiles in it
inline size_t tsg_lds_bytes(int N, int operands) {
    const size_t nt = (size_t)(N + 15) / 16;
    const size_t d = (size_t)operands * 16 * nt * kTKS;
    return (nt <= 2 && d < 4096 ? 4096 : d) * sizeof(double);
}

}  // namespace fsic
