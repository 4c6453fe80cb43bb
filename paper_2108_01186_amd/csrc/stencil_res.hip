// FP64 residual b + L x of a batch (the defect-correction check of the
// mixed-precision solves and the final residual report), and the small
// per-orbital kernels around it.
#include <algorithm>

#include "zmarch.h"

namespace fsic {

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
    if (it.orb < 0 || done[it.orb] == 1) return;
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
                                                  int *iters, double *rrfin, int *rs_iter, int *ndone,
                                                  int *fin, int xfin, int *pz, int cyc) {
    __shared__ double sred[4];
    const int o = blockIdx.x;
    if (done[o] == 1) return;
    const OrbDesc od = orb[o];
    const double rr = sum_partials(partRU + od.base7, od.nt7, sred);
    if (threadIdx.x == 0) {
        if (rr <= tol2 * bb[o]) {
            done[o] = 1;
            iters[o] = k;
            rrfin[o] = rr;
            if (ndone) atomicAdd(ndone, 1);
            if (fin) fin[o] = xfin;
        } else if (pz) {
            pz[o] = cyc;  // not confirmed: the next cycle runs in full
        } else if (done[o] == 2) {
            // the FP32 recursion met tol but the FP64 residual did not:
            // resume with a restart from the FP64 residual
            done[o] = 0;
            rs_iter[o] = k;
        }
    }
}

hipError_t launch_true_residual(int radius, const Coeffs &c, const Item *items7, int nitems7,
                                const OrbDesc *orb, const int *done, const double *X64,
                                const float *X32, const double *B, double *X64new, float *R32,
                                double *partRU, hipStream_t s) {
    if (nitems7 <= 0) return hipSuccess;
    if (X32) {
        PolRes<true> pol{items7, orb, done, X64, X32, B, X64new, R32, partRU, false};
#define CALL(P, C, DD) hipLaunchKernelGGL((k_zmarch<double, P, C, DD, PolRes<true>>), dim3(nitems7), dim3(256), 0, s, pol, c)
        FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    } else {
        PolRes<false> pol{items7, orb, done, X64, X32, B, X64new, R32, partRU, false};
#define CALL(P, C, DD) hipLaunchKernelGGL((k_zmarch<double, P, C, DD, PolRes<false>>), dim3(nitems7), dim3(256), 0, s, pol, c)
        FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    }
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
                           double tol2, int k, int *done, int *iters, double *rrfin, int *rs_iter,
                           int *ndone, int *fin, int xfin, int *pz, int cyc, hipStream_t s) {
    if (norb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ru_check, dim3(norb), dim3(256), 0, s, orb, partRU, bb, tol2, k, done,
                       iters, rrfin, rs_iter, ndone, fin, xfin, pz, cyc);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_stage_stats(int norb, const int *iters, const int *nact,
                                                     const int *done, const double *ptrue,
                                                     const double *bb, double *stage) {
    int *si = reinterpret_cast<int *>(stage);
    double *sd = stage + 4 * (size_t)norb;
    const int stride = gridDim.x * 256;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < 8 * norb; i += stride)
        si[i] = i < norb ? iters[i] : (i < 7 * norb ? nact[i - norb] : done[i - 7 * norb]);
    for (int i = blockIdx.x * 256 + threadIdx.x; i < 2 * norb; i += stride)
        sd[i] = i < norb ? ptrue[i] : bb[i - norb];
}

hipError_t launch_stage_stats(int norb, const int *iters, const int *nact, const int *done,
                              const double *ptrue, const double *bb, double *stage, hipStream_t s) {
    if (norb <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min(16, (8 * norb + 255) / 256);
    hipLaunchKernelGGL(k_stage_stats, dim3(g), dim3(256), 0, s, norb, iters, nact, done, ptrue, bb, stage);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_pack_checks(ChkPack p, const double *small, double *out) {
    const int e = blockIdx.x;
    const int N = p.N[e], NN = N * N;
    const double *sm = small + p.so[e];
    double *o = out + p.q[e];
    for (int i = threadIdx.x; i < NN + 2 + N; i += 256)
        o[i] = i < NN ? sm[p.oG + i] : (i < NN + 2 ? sm[p.oI + (i - NN)] : sm[p.oR + (i - NN - 2)]);
}

hipError_t launch_pack_checks(const ChkPack &p, const double *small, double *out, hipStream_t s) {
    if (p.n <= 0) return hipSuccess;
    if (p.n > kChkPack) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pack_checks, dim3(p.n), dim3(256), 0, s, p, small, out);
    return hipGetLastError();
}

// the final x of each orbital: copied from the second x64 buffer where the
// restart cycle that converged it (fin[o], or fallback for an unconverged
// orbital) wrote it there
__global__ __launch_bounds__(256) void k_take_x(const Item *items8, const OrbDesc *orb, const int *fin,
                                                int fallback, double *X, const double *Xb) {
    const Item it = items8[blockIdx.x];
    if (it.orb < 0) return;
    const int f = fin[it.orb];
    if ((f >= 0 ? f : fallback) != 1) return;
    const OrbDesc od = orb[it.orb];
    const long long M = (long long)od.nx * od.ny * od.nz;
    const long long base = (long long)it.tile * kPW;
#pragma unroll
    for (int e = 0; e < kPW / 256; ++e) {
        const long long i = base + e * 256 + threadIdx.x;
        if (i < M) X[od.off + i] = Xb[od.off + i];
    }
}

hipError_t launch_take_x(int nitems8, const Item *items8, const OrbDesc *orb, const int *fin, int fallback,
                         double *X, const double *Xb, hipStream_t s) {
    if (nitems8 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_take_x, dim3(nitems8), dim3(256), 0, s, items8, orb, fin, fallback, X, Xb);
    return hipGetLastError();
}

// end of a mixed solve in one launch: blocks [0, nitems8) move the final x
// as k_take_x; block nitems8 + o finishes orbital o: its FP64 residual from
// the residual pass's partials (as k_reduce_partials), iters = the
// iterations that did work, and its statistics staged as k_stage_stats
__global__ __launch_bounds__(256) void k_mixed_finish(int nitems8, const Item *items8, const OrbDesc *orb,
                                                      const int *fin, int fallback, double *X, const double *Xb,
                                                      int norb, const double *partRU, const int *nact,
                                                      const int *done, const double *bb, int *iters,
                                                      double *ptrue, double *stage) {
    __shared__ double sred[4];
    if ((int)blockIdx.x < nitems8) {
        const Item it = items8[blockIdx.x];
        if (it.orb < 0) return;
        const int f = fin[it.orb];
        if ((f >= 0 ? f : fallback) != 1) return;
        const OrbDesc od = orb[it.orb];
        const long long M = (long long)od.nx * od.ny * od.nz;
        const long long base = (long long)it.tile * kPW;
#pragma unroll
        for (int e = 0; e < kPW / 256; ++e) {
            const long long i = base + e * 256 + threadIdx.x;
            if (i < M) X[od.off + i] = Xb[od.off + i];
        }
        return;
    }
    const int o = (int)blockIdx.x - nitems8;
    const OrbDesc od = orb[o];
    const double rr = sum_partials(partRU + od.base7, od.nt7, sred);
    if (threadIdx.x == 0) {
        ptrue[o] = rr;
        iters[o] = nact[o];
        int *si = reinterpret_cast<int *>(stage);
        double *sd = stage + 4 * (size_t)norb;
        si[o] = nact[o];
        for (int q = 0; q < 6; ++q) si[norb + q * norb + o] = nact[q * norb + o];
        si[7 * norb + o] = done[o];
        sd[o] = rr;
        sd[norb + o] = bb[o];
    }
}

hipError_t launch_mixed_finish(int nitems8, const Item *items8, const OrbDesc *orb, const int *fin, int fallback,
                               double *X, const double *Xb, int norb, const double *partRU, const int *nact,
                               const int *done, const double *bb, int *iters, double *ptrue, double *stage,
                               hipStream_t s) {
    if (nitems8 < 0 || norb <= 0) return norb == 0 ? hipSuccess : hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mixed_finish, dim3((unsigned)(nitems8 + norb)), dim3(256), 0, s, nitems8, items8, orb,
                       fin, fallback, X, Xb, norb, partRU, nact, done, bb, iters, ptrue, stage);
    return hipGetLastError();
}

hipError_t launch_res_steps(int radius, const Coeffs &c, const CGIter<float> &a, const ResStep &rs,
                            hipStream_t s) {
    if (a.nitems7 <= 0) return hipSuccess;
    // x64 absent in the first cycle (x starts at 0), x32 only in cycles of
    // more than two iterations
    if (rs.X32 && rs.X64) {
        PolResP<true> pol{a.items7, a.orb, a, rs, false, 0.0, 0.0};
#define CALL(P, C, DD) hipLaunchKernelGGL((k_zmarch<double, P, C, DD, PolResP<true>>), dim3(a.nitems7), dim3(256), 0, s, pol, c)
        FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    } else if (rs.X32) {
        PolResP<true, false> pol{a.items7, a.orb, a, rs, false, 0.0, 0.0};
#define CALL(P, C, DD) hipLaunchKernelGGL((k_zmarch<double, P, C, DD, PolResP<true, false>>), dim3(a.nitems7), dim3(256), 0, s, pol, c)
        FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    } else if (rs.X64) {
        PolResP<false> pol{a.items7, a.orb, a, rs, false, 0.0, 0.0};
#define CALL(P, C, DD) hipLaunchKernelGGL((k_zmarch<double, P, C, DD, PolResP<false>>), dim3(a.nitems7), dim3(256), 0, s, pol, c)
        FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    } else {
        PolResP<false, false> pol{a.items7, a.orb, a, rs, false, 0.0, 0.0};
#define CALL(P, C, DD) hipLaunchKernelGGL((k_zmarch<double, P, C, DD, PolResP<false, false>>), dim3(a.nitems7), dim3(256), 0, s, pol, c)
        FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    }
    return hipGetLastError();
}

}  // namespace fsic
