// Alternating Anderson-Richardson (AAR) iteration for the per-orbital
// Poisson problems -L v = b, the solver the paper's real-space code uses
// (Sec. II.A).  With f_k = M^{-1} (b + L x_k) (M^{-1}: the sine-transform
// preconditioner) and the last m differences
//   X_k = [x_{i+1} - x_i],  F_k = [f_{i+1} - f_i],  i = k-m .. k-1,
// every p-th iteration is an Anderson extrapolation
//   x_{k+1} = x_k + beta f_k - (X_k + beta F_k) gamma,
//   gamma = argmin || f_k - F_k gamma ||  (normal equations, m x m),
// and the others are Richardson steps x_{k+1} = x_k + omega f_k.
// The history is kept as ring buffers of m columns (column i in slot i % m).
// All orbitals of a batch advance together; converged ones are skipped.
#include "kernels.h"

namespace fsic {

namespace {

// slot of the Gram entry (i, j), i <= j < nh, then nh right-hand sides
__device__ __forceinline__ int gram_slot(int i, int j, int nh) {
    return i * nh - i * (i - 1) / 2 + (j - i);
}

}  // namespace

// History of the newest difference column and, at Anderson steps, the
// per-tile partial sums of F^T F and F^T f.
//   hist: f_k - f_{k-1} goes into slot (k-1) % m (needs k >= 1);
//   fprev := f_k.
__global__ __launch_bounds__(256) void k_aar_dots(AarBufs a, int k, int nh, int hist, int dots) {
    __shared__ double swave[4][kAarD];
    const Item it = a.items8[blockIdx.x];
    if (it.orb < 0) return;
    if (a.done[it.orb] == 1) return;
    const OrbDesc od = a.orb[it.orb];
    const long long M = (long long)od.nx * od.ny * od.nz;
    const long long base = (long long)it.tile * kPW;
    const int hs = (k + a.m - 1) % a.m;
    double acc[kAarD];
#pragma unroll
    for (int q = 0; q < kAarD; ++q) acc[q] = 0.0;
    for (int e = 0; e < kPW / 256; ++e) {
        const long long i = base + e * 256 + threadIdx.x;
        if (i >= M) continue;
        const long long g = od.off + i;
        const float f = a.F[g];
        if (hist) {
            a.Fh[(size_t)hs * a.fields + g] = f - a.Fprev[g];
            a.Fprev[g] = f;
        }
        if (dots) {
            float col[kAarM];
#pragma unroll
            for (int j = 0; j < kAarM; ++j) col[j] = (j < nh) ? a.Fh[(size_t)j * a.fields + g] : 0.f;
#pragma unroll
            for (int ii = 0; ii < kAarM; ++ii)
#pragma unroll
                for (int jj = ii; jj < kAarM; ++jj)
                    if (jj < nh) acc[gram_slot(ii, jj, kAarM)] += (double)col[ii] * (double)col[jj];
#pragma unroll
            for (int ii = 0; ii < kAarM; ++ii)
                if (ii < nh) acc[kAarG + ii] += (double)col[ii] * (double)f;
        }
    }
    if (!dots) return;
    // every accumulator index is a compile-time constant (a runtime index
    // would put the array in scratch memory): wave sums into LDS, one
    // barrier, then thread q adds the four wave sums of entry q in fixed order
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kAarD; ++q) {
        const double t = wave_sum(acc[q]);
        if ((threadIdx.x & 63) == 0) swave[w][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < kAarD) {
        const int q = threadIdx.x;
        a.partD[(size_t)(od.base8 + it.tile) * kAarD + q] = (swave[0][q] + swave[1][q]) + (swave[2][q] + swave[3][q]);
    }
}

// Per orbital: sum the tile partials (fixed order) and solve the nh x nh
// normal equations for gamma by Gaussian elimination with partial pivoting;
// a tiny multiple of the largest diagonal entry is added to the diagonal so
// nearly dependent history columns give a bounded gamma.
__global__ __launch_bounds__(256) void k_aar_solve(AarBufs a, int nh) {
    __shared__ double sred[4];
    __shared__ double d[kAarD];
    const int o = blockIdx.x;
    if (a.done[o] == 1) return;
    const OrbDesc od = a.orb[o];
    for (int q = 0; q < kAarD; ++q) {
        double s = 0.0;
        for (int t = threadIdx.x; t < od.nt8; t += 256) s += a.partD[(size_t)(od.base8 + t) * kAarD + q];
        s = block_sum256(s, sred);
        if (threadIdx.x == 0) d[q] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double G[kAarM][kAarM + 1];
    double dmax = 0.0;
    for (int i = 0; i < nh; ++i) {
        for (int j = i; j < nh; ++j) G[i][j] = G[j][i] = d[gram_slot(i, j, kAarM)];
        G[i][nh] = d[kAarG + i];
        dmax = fmax(dmax, G[i][i]);
    }
    for (int i = 0; i < nh; ++i) G[i][i] += 1e-13 * dmax;
    for (int col = 0; col < nh; ++col) {
        int piv = col;
        for (int r = col + 1; r < nh; ++r)
            if (fabs(G[r][col]) > fabs(G[piv][col])) piv = r;
        if (piv != col)
            for (int j = 0; j <= nh; ++j) {
                const double tmp = G[col][j];
                G[col][j] = G[piv][j];
                G[piv][j] = tmp;
            }
        const double pv = G[col][col];
        for (int r = col + 1; r < nh; ++r) {
            const double fct = (pv != 0.0) ? G[r][col] / pv : 0.0;
            for (int j = col; j <= nh; ++j) G[r][j] -= fct * G[col][j];
        }
    }
    double gam[kAarM];
    for (int i = nh - 1; i >= 0; --i) {
        double s = G[i][nh];
        for (int j = i + 1; j < nh; ++j) s -= G[i][j] * gam[j];
        gam[i] = (G[i][i] != 0.0) ? s / G[i][i] : 0.0;
    }
    for (int i = 0; i < kAarM; ++i) a.gamma[(size_t)o * kAarM + i] = (i < nh && isfinite(gam[i])) ? gam[i] : 0.0;
}

// The step: Richardson (omega f) or Anderson (beta f - sum_j gamma_j (X_j +
// beta F_j)); x += step and the step becomes history column k (slot k % m).
// hist: 1 also records f_k - f_{k-1} and f_k first, 2 only f_k (the first
// iteration), 0 neither (Anderson steps did both in k_aar_dots).
template <bool AND>
__global__ __launch_bounds__(256) void k_aar_step(AarBufs a, int k, int nh, double omega, double beta,
                                                  int hist) {
    const Item it = a.items8[blockIdx.x];
    if (it.orb < 0) return;
    if (a.done[it.orb] == 1) return;
    const OrbDesc od = a.orb[it.orb];
    const long long M = (long long)od.nx * od.ny * od.nz;
    const long long base = (long long)it.tile * kPW;
    const int hs = (k + a.m - 1) % a.m, xs = k % a.m;
    double gam[kAarM];
#pragma unroll
    for (int j = 0; j < kAarM; ++j) gam[j] = (AND && j < nh) ? a.gamma[(size_t)it.orb * kAarM + j] : 0.0;
    for (int e = 0; e < kPW / 256; ++e) {
        const long long i = base + e * 256 + threadIdx.x;
        if (i >= M) continue;
        const long long g = od.off + i;
        const float f = a.F[g];
        if (hist == 1) a.Fh[(size_t)hs * a.fields + g] = f - a.Fprev[g];
        if (hist) a.Fprev[g] = f;
        double step;
        if (AND) {
            step = beta * (double)f;
#pragma unroll
            for (int j = 0; j < kAarM; ++j)
                if (j < nh)
                    step -= gam[j] * (a.Xh[(size_t)j * a.fields + g] + beta * (double)a.Fh[(size_t)j * a.fields + g]);
        } else {
            step = omega * (double)f;
        }
        a.X[g] += step;
        a.Xh[(size_t)xs * a.fields + g] = step;
    }
}

hipError_t launch_aar_dots(const AarBufs &a, int nitems8, int k, int nh, int hist, int dots,
                           hipStream_t s) {
    if (nitems8 <= 0 || nh > kAarM || a.m != kAarM) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_aar_dots, dim3(nitems8), dim3(256), 0, s, a, k, nh, hist, dots);
    return hipGetLastError();
}

hipError_t launch_aar_solve(const AarBufs &a, int norb, int nh, hipStream_t s) {
    if (norb <= 0 || nh < 1 || nh > kAarM) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_aar_solve, dim3(norb), dim3(256), 0, s, a, nh);
    return hipGetLastError();
}

hipError_t launch_aar_step(const AarBufs &a, int nitems8, int k, int nh, double omega, double beta,
                           bool anderson, int hist, hipStream_t s) {
    if (nitems8 <= 0 || nh > kAarM || a.m != kAarM) return hipErrorInvalidValue;
    if (anderson)
        hipLaunchKernelGGL(k_aar_step<true>, dim3(nitems8), dim3(256), 0, s, a, k, nh, omega, beta, hist);
    else
        hipLaunchKernelGGL(k_aar_step<false>, dim3(nitems8), dim3(256), 0, s, a, k, nh, omega, beta, hist);
    return hipGetLastError();
}

}  // namespace fsic
