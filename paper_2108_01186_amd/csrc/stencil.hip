// Star-stencil Laplacian and conjugate-gradient sweeps for the per-orbital
// Poisson problems of the SIC path (Sec. II.A: high-order centred finite
// differences on a uniform grid; the Laplacian is the Kronecker sum of 1-D
// second differences applied matrix-free).
//
// Design (gfx950): one 256-thread block owns a 32 x 16 column tile of an
// orbital's grid and marches through a z-chunk.  Each thread keeps the
// 2p + 1 z-neighbours of its two columns in registers; the current xy plane
// with its p-deep cross-shaped halo is staged in LDS.  The operand of the
// stencil is produced on the fly by a policy (p = r + beta p_old for CG,
// x64 + x32 for the FP64 residual), so every CG iteration is two HBM
// passes: this sweep and one pointwise update.  Dot products accumulate in
// FP64 into per-block partial sums that later blocks add up in a fixed
// order, so results are bitwise reproducible.
#include "kernels.h"

namespace fsic {

// ---------------------------------------------------------------------------
// z-marching stencil driver
// ---------------------------------------------------------------------------

template <typename T, int P, class Pol>
__global__ __launch_bounds__(256) void k_zmarch(Pol pol, Coeffs cf) {
    __shared__ T sm[kTY + 2 * P][kTX + 2 * P];
    __shared__ double sred[4];
    const Item it = pol.items[blockIdx.x];
    if (it.orb < 0) return;
    const OrbDesc od = pol.orb[it.orb];
    Pol p = pol;
    if (!p.setup(it.orb, od, sred)) return;  // uniform across the block

    const int nx = od.nx, ny = od.ny, nz = od.nz;
    const int bx = it.tile % od.tiles_x;
    const int by = (it.tile / od.tiles_x) % od.tiles_y;
    const int bz = it.tile / (od.tiles_x * od.tiles_y);
    const int tx = threadIdx.x & (kTX - 1);
    const int ty = threadIdx.x >> 5;  // 0..7
    const int x = bx * kTX + tx;
    const int y0 = by * kTY + ty;
    const int y1 = y0 + 8;
    const int z0 = bz * od.zc;
    const int z1 = min(nz, z0 + od.zc);

    T c[P + 1];
#pragma unroll
    for (int k = 0; k <= P; ++k) c[k] = (T)cf.c[k];
    const T c0x3 = T(3) * c[0];
    const T ih2 = (T)od.inv_h2;

    auto ld = [&](int xx, int yy, int zz) -> T {
        if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) return T(0);
        return p.load(od, ((long long)zz * ny + yy) * nx + xx);
    };

    T qa[2 * P + 1], qb[2 * P + 1];
#pragma unroll
    for (int j = 0; j < 2 * P; ++j) {
        qa[j] = ld(x, y0, z0 - P + j);
        qb[j] = ld(x, y1, z0 - P + j);
    }
    double dot = 0.0;
    for (int z = z0; z < z1; ++z) {
        qa[2 * P] = ld(x, y0, z + P);
        qb[2 * P] = ld(x, y1, z + P);
        sm[ty + P][tx + P] = qa[P];
        sm[ty + 8 + P][tx + P] = qb[P];
        for (int hh = threadIdx.x; hh < 2 * P * (kTX + kTY); hh += 256) {
            int hx, hy;
            if (hh < 2 * P * kTY) {
                const int side = hh / (P * kTY);
                const int rem = hh - side * P * kTY;
                hy = rem / P;
                hx = rem - hy * P;
                hx = side ? kTX + hx : hx - P;
            } else {
                const int h2 = hh - 2 * P * kTY;
                const int side = h2 / (P * kTX);
                const int rem = h2 - side * P * kTX;
                const int yy = rem / kTX;
                hx = rem - yy * kTX;
                hy = side ? kTY + yy : yy - P;
            }
            sm[hy + P][hx + P] = ld(bx * kTX + hx, by * kTY + hy, z);
        }
        __syncthreads();
        T la = c0x3 * qa[P], lb = c0x3 * qb[P];
#pragma unroll
        for (int k = 1; k <= P; ++k) {
            la += c[k] * ((sm[ty + P][tx + P + k] + sm[ty + P][tx + P - k]) +
                          (sm[ty + P + k][tx + P] + sm[ty + P - k][tx + P]) +
                          (qa[P + k] + qa[P - k]));
            lb += c[k] * ((sm[ty + 8 + P][tx + P + k] + sm[ty + 8 + P][tx + P - k]) +
                          (sm[ty + 8 + P + k][tx + P] + sm[ty + 8 + P - k][tx + P]) +
                          (qb[P + k] + qb[P - k]));
        }
        la *= ih2;
        lb *= ih2;
        if (x < nx) {
            if (y0 < ny) dot += p.epilogue(od, ((long long)z * ny + y0) * nx + x, qa[P], la);
            if (y1 < ny) dot += p.epilogue(od, ((long long)z * ny + y1) * nx + x, qb[P], lb);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2 * P; ++j) {
            qa[j] = qa[j + 1];
            qb[j] = qb[j + 1];
        }
    }
    if (p.wants_dot()) {
        const double s = block_sum256(dot, sred);
        if (threadIdx.x == 0) p.finish(it, od, s);
    }
}

// ---------------------------------------------------------------------------
// policies
// ---------------------------------------------------------------------------

template <typename T>
struct PolApply {  // Lu = L u
    const Item *items;
    const OrbDesc *orb;
    const T *u;
    T *out;
    __device__ bool setup(int, const OrbDesc &, double *) { return true; }
    __device__ T load(const OrbDesc &od, long long i) const { return u[od.off + i]; }
    __device__ double epilogue(const OrbDesc &od, long long i, T, T lap) const {
        out[od.off + i] = lap;
        return 0.0;
    }
    __device__ bool wants_dot() const { return false; }
    __device__ void finish(const Item &, const OrbDesc &, double) const {}
};

template <typename T>
__device__ __forceinline__ double rr_of(const CGIter<T> &a, const OrbDesc &od, int j,
                                        int from_ru, double *sbuf) {
    if (from_ru) return sum_partials(a.partRU + od.base7, od.nt7, sbuf);
    return sum_partials(a.part8 + (size_t)(j & 1) * a.tot8 + od.base8, od.nt8, sbuf);
}

template <typename T>
struct PolCG {  // p_k = r_k + beta p_{k-1}; q = K p_k = -L p_k
    const Item *items;
    const OrbDesc *orb;
    CGIter<T> a;
    int k, cur_ru, prev_ru, check;
    double beta;
    __device__ bool setup(int o, const OrbDesc &od, double *sbuf) {
        // other blocks of this orbital may set done[o] during this launch:
        // read it once and broadcast so the whole block takes one branch
        if (threadIdx.x == 0) sbuf[0] = (double)a.done[o];
        __syncthreads();
        const bool dn = sbuf[0] != 0.0;
        __syncthreads();
        if (dn) return false;
        const double rr = rr_of(a, od, k, cur_ru, sbuf);
        if (check && rr <= a.tol2 * a.bb[o]) {
            if (threadIdx.x == 0) {
                a.done[o] = 1;
                a.iters[o] = k;
                a.rrfin[o] = rr;
            }
            return false;
        }
        if (k == 0) {
            beta = 0.0;
        } else {
            const double rp = rr_of(a, od, k - 1, prev_ru, sbuf);
            beta = rr / rp;
        }
        return true;
    }
    __device__ T load(const OrbDesc &od, long long i) const {
        const long long g = od.off + i;
        if (k == 0) return a.R[g];
        return a.R[g] + (T)beta * a.Pold[g];
    }
    __device__ double epilogue(const OrbDesc &od, long long i, T c, T lap) const {
        const long long g = od.off + i;
        const T q = -lap;
        a.Pnew[g] = c;
        a.Q[g] = q;
        return (double)c * (double)q;
    }
    __device__ bool wants_dot() const { return true; }
    __device__ void finish(const Item &it, const OrbDesc &od, double s) const {
        a.part7[od.base7 + it.tile] = s;
    }
};

struct PolRes {  // res = b + L x, x = x64 (+ x32)
    const Item *items;
    const OrbDesc *orb;
    const int *done;
    const double *X64;
    const float *X32;
    const double *B;
    double *X64new;
    float *R32;
    double *partRU;
    __device__ bool setup(int o, const OrbDesc &, double *) { return done == nullptr || !done[o]; }
    __device__ double load(const OrbDesc &od, long long i) const {
        const long long g = od.off + i;
        return X32 ? X64[g] + (double)X32[g] : X64[g];
    }
    __device__ double epilogue(const OrbDesc &od, long long i, double c, double lap) const {
        const long long g = od.off + i;
        const double res = B[g] + lap;
        if (X64new) X64new[g] = c;
        if (R32) R32[g] = (float)res;
        return res * res;
    }
    __device__ bool wants_dot() const { return true; }
    __device__ void finish(const Item &it, const OrbDesc &od, double s) const {
        partRU[od.base7 + it.tile] = s;
    }
};

// ---------------------------------------------------------------------------
// pointwise CG update
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_cg_update(CGIter<T> a, int k, int cur_ru, int x_first) {
    __shared__ double sred[4];
    const Item it = a.items8[blockIdx.x];
    if (it.orb < 0) return;
    if (a.done[it.orb]) return;
    const OrbDesc od = a.orb[it.orb];
    const double rr = rr_of(a, od, k, cur_ru, sred);
    const double pq = sum_partials(a.part7 + od.base7, od.nt7, sred);
    const double alpha = rr / pq;
    const T al = (T)alpha;
    const long long M = (long long)od.nx * od.ny * od.nz;
    const long long base = (long long)it.tile * kPW;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < kPW / 256; ++e) {
        const long long i = base + e * 256 + threadIdx.x;
        if (i < M) {
            const long long g = od.off + i;
            const T pv = a.Pnew[g];
            const T xv = x_first ? al * pv : a.X[g] + al * pv;
            const T rv = a.R[g] - al * a.Q[g];
            a.X[g] = xv;
            a.R[g] = rv;
            acc += (double)rv * (double)rv;
        }
    }
    const double s = block_sum256(acc, sred);
    if (threadIdx.x == 0) a.part8[(size_t)((k + 1) & 1) * a.tot8 + od.base8 + it.tile] = s;
}

__global__ __launch_bounds__(256) void k_reduce_partials(int norb, const OrbDesc *orb,
                                                         const double *part, int stencil,
                                                         double *out) {
    __shared__ double sred[4];
    const int o = blockIdx.x;
    if (o >= norb) return;
    const OrbDesc od = orb[o];
    const double s = stencil ? sum_partials(part + od.base7, od.nt7, sred)
                             : sum_partials(part + od.base8, od.nt8, sred);
    if (threadIdx.x == 0) out[o] = s;
}


// x64 += x32 after a reliable update (mixed precision)
__global__ __launch_bounds__(256) void k_mixed_accumulate(const Item *items8, const OrbDesc *orb,
                                                          const int *done, double *X64,
                                                          const float *X32) {
    const Item it = items8[blockIdx.x];
    if (it.orb < 0 || done[it.orb]) return;
    const OrbDesc od = orb[it.orb];
    const long long M = (long long)od.nx * od.ny * od.nz;
    const long long base = (long long)it.tile * kPW;
#pragma unroll
    for (int e = 0; e < kPW / 256; ++e) {
        const long long i = base + e * 256 + threadIdx.x;
        if (i < M) X64[od.off + i] += (double)X32[od.off + i];
    }
}

// convergence on the FP64 residual of the last reliable update
__global__ __launch_bounds__(256) void k_ru_check(const OrbDesc *orb, const double *partRU,
                                                  const double *bb, double tol2, int k, int *done,
                                                  int *iters, double *rrfin) {
    __shared__ double sred[4];
    const int o = blockIdx.x;
    if (done[o]) return;
    const OrbDesc od = orb[o];
    const double rr = sum_partials(partRU + od.base7, od.nt7, sred);
    if (threadIdx.x == 0 && rr <= tol2 * bb[o]) {
        done[o] = 1;
        iters[o] = k;
        rrfin[o] = rr;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define FSIC_RADIUS_SWITCH(radius, CALL) \
    switch (radius) {                    \
        case 1: CALL(1); break;          \
        case 2: CALL(2); break;          \
        case 3: CALL(3); break;          \
        case 4: CALL(4); break;          \
        case 5: CALL(5); break;          \
        case 6: CALL(6); break;          \
        default: return hipErrorInvalidValue; \
    }

template <typename T>
hipError_t launch_apply(int radius, const Coeffs &c, const Item *items, int nitems,
                        const OrbDesc *orb, const T *u, T *Lu, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    PolApply<T> pol{items, orb, u, Lu};
#define CALL(P) hipLaunchKernelGGL((k_zmarch<T, P, PolApply<T>>), dim3(nitems), dim3(256), 0, s, pol, c)
    FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_stencil(int radius, const Coeffs &c, const CGIter<T> &a, int k,
                             int cur_from_ru, int prev_from_ru, int check, hipStream_t s) {
    if (a.nitems7 <= 0) return hipSuccess;
    PolCG<T> pol{a.items7, a.orb, a, k, cur_from_ru, prev_from_ru, check, 0.0};
#define CALL(P) hipLaunchKernelGGL((k_zmarch<T, P, PolCG<T>>), dim3(a.nitems7), dim3(256), 0, s, pol, c)
    FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_update(const CGIter<T> &a, int k, int cur_from_ru, int x_first,
                            hipStream_t s) {
    if (a.nitems8 <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_cg_update<T>), dim3(a.nitems8), dim3(256), 0, s, a, k, cur_from_ru,
                       x_first);
    return hipGetLastError();
}

hipError_t launch_true_residual(int radius, const Coeffs &c, const Item *items7, int nitems7,
                                const OrbDesc *orb, const int *done, const double *X64,
                                const float *X32, const double *B, double *X64new, float *R32,
                                double *partRU, hipStream_t s) {
    if (nitems7 <= 0) return hipSuccess;
    PolRes pol{items7, orb, done, X64, X32, B, X64new, R32, partRU};
#define CALL(P) hipLaunchKernelGGL((k_zmarch<double, P, PolRes>), dim3(nitems7), dim3(256), 0, s, pol, c)
    FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_reduce_partials(int norb, const OrbDesc *orb, const double *part,
                                  int stencil_layout, double *out, hipStream_t s) {
    if (norb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_partials, dim3(norb), dim3(256), 0, s, norb, orb, part,
                       stencil_layout, out);
    return hipGetLastError();
}


hipError_t launch_mixed_accumulate(int nitems8, const Item *items8, const OrbDesc *orb,
                                   const int *done, double *X64, const float *X32, hipStream_t s) {
    if (nitems8 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mixed_accumulate, dim3(nitems8), dim3(256), 0, s, items8, orb, done, X64, X32);
    return hipGetLastError();
}

hipError_t launch_ru_check(int norb, const OrbDesc *orb, const double *partRU, const double *bb,
                           double tol2, int k, int *done, int *iters, double *rrfin, hipStream_t s) {
    if (norb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ru_check, dim3(norb), dim3(256), 0, s, orb, partRU, bb, tol2, k, done, iters, rrfin);
    return hipGetLastError();
}

template hipError_t launch_apply<double>(int, const Coeffs &, const Item *, int, const OrbDesc *,
                                         const double *, double *, hipStream_t);
template hipError_t launch_apply<float>(int, const Coeffs &, const Item *, int, const OrbDesc *,
                                        const float *, float *, hipStream_t);
template hipError_t launch_cg_stencil<double>(int, const Coeffs &, const CGIter<double> &, int, int,
                                              int, int, hipStream_t);
template hipError_t launch_cg_stencil<float>(int, const Coeffs &, const CGIter<float> &, int, int,
                                             int, int, hipStream_t);
template hipError_t launch_cg_update<double>(const CGIter<double> &, int, int, int, hipStream_t);
template hipError_t launch_cg_update<float>(const CGIter<float> &, int, int, int, hipStream_t);

}  // namespace fsic
