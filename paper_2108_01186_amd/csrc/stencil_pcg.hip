// Preconditioned conjugate gradients (Sec. II.A; preconditioner in dst.hip):
// the sweep p = z + beta p_old, q = -L p, and the update of x and r.
#include <algorithm>

#include "zmarch.h"

namespace fsic {

template <typename T>
__global__ __launch_bounds__(256) void k_pcg_update(CGIter<T> a, int k, int x_first) {
    using V = typename Vec16<T>::V;
    constexpr int VN = Vec16<T>::n;
    __shared__ double sred[4];
    const Item it = a.items8[blockIdx.x];
    if (it.orb < 0) return;
    if (a.done[it.orb]) return;
    const OrbDesc od = a.orb[it.orb];
    const double rz = rz_of(a, od, k, sred);
    const double pq = sum_partials(a.part7 + od.base7, od.nt7, sred);
    const T al = (T)(rz / pq);
    const long long M = (long long)od.nx * od.ny * od.nz;
    const long long base = (long long)it.tile * kPW;
    double acc = 0.0;
    if (((od.off | M) % VN) == 0) {
#pragma unroll
        for (int e = 0; e < kPW / (256 * VN); ++e) {
            const long long i = base + (long long)(e * 256 + threadIdx.x) * VN;
            if (i < M) {
                const long long g = od.off + i;
                V pv = *reinterpret_cast<const V *>(a.P + g);
                V qv = *reinterpret_cast<const V *>(a.Q + g);
                V rv = *reinterpret_cast<const V *>(a.R + g);
                V xv = x_first ? V{} : *reinterpret_cast<const V *>(a.X + g);
                T *px = reinterpret_cast<T *>(&xv), *pr = reinterpret_cast<T *>(&rv);
                const T *pp = reinterpret_cast<const T *>(&pv), *pqv = reinterpret_cast<const T *>(&qv);
#pragma unroll
                for (int j = 0; j < VN; ++j) {
                    px[j] = x_first ? al * pp[j] : px[j] + al * pp[j];
                    pr[j] = pr[j] - al * pqv[j];
                    acc += (double)pr[j] * (double)pr[j];
                }
                *reinterpret_cast<V *>(a.X + g) = xv;
                *reinterpret_cast<V *>(a.R + g) = rv;
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < kPW / 256; ++e) {
            const long long i = base + e * 256 + threadIdx.x;
            if (i < M) {
                const long long g = od.off + i;
                const T pv = a.P[g];
                const T xv = x_first ? al * pv : a.X[g] + al * pv;
                const T rv = a.R[g] - al * a.Q[g];
                a.X[g] = xv;
                a.R[g] = rv;
                acc += (double)rv * (double)rv;
            }
        }
    }
    const double s = block_sum256(acc, sred);
    if (threadIdx.x == 0) {
        a.part8[(size_t)((k + 1) & 1) * a.tot8 + od.base8 + it.tile] = s;
        if (it.tile == 0) {
            a.nact[a.norb + it.orb] += 1;
            if (a.nsamp) a.nsamp[a.norb + it.orb] += 1;
        }
    }
}

template <typename T>
hipError_t launch_pcg_stencil(int radius, const Coeffs &c, const CGIter<T> &a, int k,
                              int cur_from_ru, int restart, int pause, hipStream_t s) {
    if (a.nitems7 <= 0) return hipSuccess;
    PolPCG<T> pol{a.items7, a.orb, a, k, cur_from_ru, restart, pause, 0.0, false};
    if (k == 0 || restart) pol.a.Pold = a.R;  // beta = 0: any finite p_old will do
#define CALL(P, C, DD) hipLaunchKernelGGL((k_zmarch<T, P, C, DD, PolPCG<T>>), dim3(a.nitems7), dim3(256), 0, s, pol, c)
    FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_update(const CGIter<T> &a, int k, int x_first, hipStream_t s) {
    if (a.nitems8 <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_pcg_update<T>), dim3(a.nitems8), dim3(256), 0, s, a, k, x_first);
    return hipGetLastError();
}

template hipError_t launch_pcg_stencil<double>(int, const Coeffs &, const CGIter<double> &, int, int,
                                               int, int, hipStream_t);
template hipError_t launch_pcg_stencil<float>(int, const Coeffs &, const CGIter<float> &, int, int,
                                              int, int, hipStream_t);
template hipError_t launch_pcg_update<double>(const CGIter<double> &, int, int, hipStream_t);
template hipError_t launch_pcg_update<float>(const CGIter<float> &, int, int, hipStream_t);

// mixed restart cycles: r -= alpha q with the new r.r partials (and the x
// modes of launch_pcg_rupdate)
__global__ __launch_bounds__(256) void k_pcg_rupd(CGIter<float> a, int k, int xmode, const int *pz, int li) {
    __shared__ double sred[4];
    const Item it = a.items8[blockIdx.x];
    if (it.orb < 0) return;
    if (a.done[it.orb] || (pz && pz[it.orb] < li)) return;
    const OrbDesc od = a.orb[it.orb];
    const float al = (float)alpha_of(a, od, k, sred);
    const long long M = (long long)od.nx * od.ny * od.nz;
    const long long base = (long long)it.tile * kPW;
    double acc = 0.0;
    if (((od.off | M) & 3) == 0) {
#pragma unroll
        for (int e = 0; e < kPW / 1024; ++e) {
            const long long i = base + (long long)(e * 256 + threadIdx.x) * 4;
            if (i < M) {
                const long long g = od.off + i;
                float4 rv = *reinterpret_cast<const float4 *>(a.R + g);
                const float4 qv = *reinterpret_cast<const float4 *>(a.Q + g);
                rv.x -= al * qv.x; rv.y -= al * qv.y; rv.z -= al * qv.z; rv.w -= al * qv.w;
                acc += (double)rv.x * rv.x + (double)rv.y * rv.y + (double)rv.z * rv.z + (double)rv.w * rv.w;
                *reinterpret_cast<float4 *>(a.R + g) = rv;
                if (xmode) {
                    const float4 pv = *reinterpret_cast<const float4 *>(a.P + g);
                    float4 xv = xmode == 2 ? *reinterpret_cast<const float4 *>(a.X + g)
                                           : float4{0.f, 0.f, 0.f, 0.f};
                    xv.x += al * pv.x; xv.y += al * pv.y; xv.z += al * pv.z; xv.w += al * pv.w;
                    *reinterpret_cast<float4 *>(a.X + g) = xv;
                }
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < kPW / 256; ++e) {
            const long long i = base + e * 256 + threadIdx.x;
            if (i < M) {
                const long long g = od.off + i;
                const float rv = a.R[g] - al * a.Q[g];
                a.R[g] = rv;
                acc += (double)rv * rv;
                if (xmode) a.X[g] = (xmode == 2 ? a.X[g] : 0.f) + al * a.P[g];
            }
        }
    }
    const double ssum = block_sum256(acc, sred);
    if (threadIdx.x == 0) {
        a.part8[(size_t)((k + 1) & 1) * a.tot8 + od.base8 + it.tile] = ssum;
        if (it.tile == 0) {
            a.nact[a.norb + it.orb] += 1;
            if (a.nsamp) a.nsamp[a.norb + it.orb] += 1;
        }
    }
}

// pause check: one block per orbital
__global__ __launch_bounds__(256) void k_pause_check(CGIter<float> a, int k, double ftol2, int *pz, int li) {
    __shared__ double sred[4];
    const int o = blockIdx.x;
    if (a.done[o] || pz[o] < li) return;  // converged, or paused before this update ran
    const OrbDesc od = a.orb[o];
    const double rr = sum_partials(a.part8 + (size_t)((k + 1) & 1) * a.tot8 + od.base8, od.nt8, sred);
    if (threadIdx.x == 0 && rr <= ftol2 * a.bb[o]) pz[o] = li;
}

__global__ void k_fill_int(int *p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_pcg_sweep(int radius, const Coeffs &c, const CGIter<float> &a, int k, const int *pz,
                            int li, hipStream_t s) {
    if (a.nitems7 <= 0) return hipSuccess;
    PolPQ pol{a.items7, a.orb, a, k, pz, li, false};
#define CALL(P, C, DD) hipLaunchKernelGGL((k_zmarch<float, P, C, DD, PolPQ>), dim3(a.nitems7), dim3(256), 0, s, pol, c)
    FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_pcg_rupdate(const CGIter<float> &a, int k, int xmode, const int *pz, int li,
                              hipStream_t s) {
    if (a.nitems8 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pcg_rupd, dim3(a.nitems8), dim3(256), 0, s, a, k, xmode, pz, li);
    return hipGetLastError();
}

hipError_t launch_pause_check(const CGIter<float> &a, int k, double ftol2, int *pz, int li, hipStream_t s) {
    if (a.norb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pause_check, dim3(a.norb), dim3(256), 0, s, a, k, ftol2, pz, li);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_ints(IntFills f) {
    const int e = blockIdx.y;
    int *const p = f.p[e];
    const int n = f.n[e], v = f.v[e];
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = v;
}

hipError_t launch_fill_ints(const IntFills &f, hipStream_t s) {
    if (f.count <= 0 || f.count > kIntFills) return f.count == 0 ? hipSuccess : hipErrorInvalidValue;
    int nmax = 1;
    for (int e = 0; e < f.count; ++e) nmax = std::max(nmax, f.n[e]);
    const unsigned gx = (unsigned)std::min(64, (nmax + 255) / 256);
    hipLaunchKernelGGL(k_fill_ints, dim3(gx, (unsigned)f.count), dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int n, int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace fsic
