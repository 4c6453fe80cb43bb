// Plain conjugate gradients for the per-orbital Poisson problems (Sec. II.A):
// the stencil sweep q = -L p with the p.q, r.q, q.q partials, and the pointwise
// update that also forms the next search direction.
#include "zmarch.h"

namespace fsic {

// x += alpha p; r -= alpha q; p = r + beta p (one node)
template <typename T>
__device__ __forceinline__ double upd_elem(T &x, T &r, T &p, T qv, T al, T be, int x_first) {
    x = x_first ? al * p : x + al * p;
    r = r - al * qv;
    p = r + be * p;
    return (double)r * (double)r;
}

template <typename T>
__global__ __launch_bounds__(256) void k_cg_update(CGIter<T> a, int k, int cur_ru, int x_first) {
    using V = typename Vec16<T>::V;
    constexpr int VN = Vec16<T>::n;
    __shared__ double sred[4];
    const Item it = a.items8[blockIdx.x];
    if (it.orb < 0) return;
    if (a.done[it.orb]) return;
    const OrbDesc od = a.orb[it.orb];
    const bool restart = a.rs_iter && a.rs_iter[it.orb] == k;
    const double rr = rr_of(a, od, k, cur_ru || restart, sred);
    const double pq = sum_partials(a.part7 + od.base7, od.nt7, sred);
    const double rq = sum_partials(a.part7 + (size_t)a.tot7 + od.base7, od.nt7, sred);
    const double qq = sum_partials(a.part7 + 2 * (size_t)a.tot7 + od.base7, od.nt7, sred);
    const double alpha = rr / pq;
    // |r_{k+1}|^2 = |r_k|^2 - 2 alpha r_k.q_k + alpha^2 |q_k|^2, so the next
    // direction is formed here; the direct r.r of this pass (below) decides
    // alpha and convergence of the next iteration
    const double rn = rr - 2.0 * alpha * rq + alpha * alpha * qq;
    const double beta = rn > 0.0 ? rn / rr : 0.0;
    const T al = (T)alpha, be = (T)beta;
    const T *Pin = ((k == 0) || restart) ? a.R : a.P;  // p_k = r_k at a (re)start
    const long long M = (long long)od.nx * od.ny * od.nz;
    const long long base = (long long)it.tile * kPW;
    double acc = 0.0;
    if (((od.off | M) % VN) == 0) {
        // 16-byte vector path: each thread owns VN consecutive nodes per pass
#pragma unroll
        for (int e = 0; e < kPW / (256 * VN); ++e) {
            const long long i = base + (long long)(e * 256 + threadIdx.x) * VN;
            if (i < M) {
                const long long g = od.off + i;
                V pv = *reinterpret_cast<const V *>(Pin + g);
                V qv = *reinterpret_cast<const V *>(a.Q + g);
                V rv = *reinterpret_cast<const V *>(a.R + g);
                V xv = x_first ? V{} : *reinterpret_cast<const V *>(a.X + g);
                T *px = reinterpret_cast<T *>(&xv), *pr = reinterpret_cast<T *>(&rv);
                T *pp = reinterpret_cast<T *>(&pv);
                const T *pqv = reinterpret_cast<const T *>(&qv);
#pragma unroll
                for (int j = 0; j < VN; ++j)
                    acc += upd_elem(px[j], pr[j], pp[j], pqv[j], al, be, x_first);
                *reinterpret_cast<V *>(a.X + g) = xv;
                *reinterpret_cast<V *>(a.R + g) = rv;
                *reinterpret_cast<V *>(a.P + g) = pv;
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < kPW / 256; ++e) {
            const long long i = base + e * 256 + threadIdx.x;
            if (i < M) {
                const long long g = od.off + i;
                T xv = x_first ? T(0) : a.X[g];
                T rv = a.R[g];
                T pv = Pin[g];
                acc += upd_elem(xv, rv, pv, a.Q[g], al, be, x_first);
                a.X[g] = xv;
                a.R[g] = rv;
                a.P[g] = pv;
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

// preconditioned CG: x += alpha p; r -= alpha q; alpha = r.z / p.q

template <typename T>
hipError_t launch_cg_stencil(int radius, const Coeffs &c, const CGIter<T> &a, int k,
                             int cur_from_ru, int check, hipStream_t s) {
    if (a.nitems7 <= 0) return hipSuccess;
    PolCG<T> pol{a.items7, a.orb, a, k, cur_from_ru, check, false, false};
#define CALL(P, C, DD) hipLaunchKernelGGL((k_zmarch<T, P, C, DD, PolCG<T>>), dim3(a.nitems7), dim3(256), 0, s, pol, c)
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

template hipError_t launch_cg_stencil<double>(int, const Coeffs &, const CGIter<double> &, int, int,
                                              int, hipStream_t);
template hipError_t launch_cg_stencil<float>(int, const Coeffs &, const CGIter<float> &, int, int,
                                             int, hipStream_t);
template hipError_t launch_cg_update<double>(const CGIter<double> &, int, int, int, hipStream_t);
template hipError_t launch_cg_update<float>(const CGIter<float> &, int, int, int, hipStream_t);

}  // namespace fsic
