// LSDA exchange-correlation of each FLO density at full spin polarisation
// (E_xc[rho_i, 0] of Eq. 1; LSDA exchange and PW92 correlation, Sec. III),
// the orbital SIC potentials V_i = -(v_H[rho_i] + v_xc[rho_i, 0]) (Eq. 5),
// their generalised-Slater average weighted by the FLO densities (Eq. 13,
// optionally scaled), and the per-orbital Hartree and XC energies.
//
// One fused pass per spin channel: each thread owns nodes and walks the
// orbitals, so phi_i and v_i are read once and V_SIC is written once.
#include "kernels.h"
#include "lsda.h"

namespace fsic {

__global__ __launch_bounds__(256) void k_xc_pointwise(long long count, const double *rho,
                                                      double floor, double *ex, double *ec,
                                                      double *vx, double *vc) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    double a, b, c, d;
    lsda_pol(rho[i], floor, a, b, c, d);
    if (ex) ex[i] = a;
    if (ec) ec[i] = b;
    if (vx) vx[i] = c;
    if (vc) vc[i] = d;
}

hipError_t launch_xc_pointwise(long long count, const double *rho, double floor, double *ex,
                               double *ec, double *vx, double *vc, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_xc_pointwise, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       count, rho, floor, ex, ec, vx, vc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Slater average and energy partial sums
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_sic_average(const ChanDesc *chans, const int *blk_chan,
                                                     const double *PHI, const double *V,
                                                     double floor, double *partU, double *partX) {
    __shared__ double su[4][kMaxOrb], sx[4][kMaxOrb];
    const int c = blk_chan[blockIdx.x];
    const ChanDesc ch = chans[c];
    const int tile = blockIdx.x - ch.blk_base;
    const long long base = (long long)tile * kSicTile;
    double num[kSicTile / 256], den[kSicTile / 256];
#pragma unroll
    for (int e = 0; e < kSicTile / 256; ++e) num[e] = den[e] = 0.0;
    const int w = threadIdx.x >> 6;
    // the next orbital's phi and v are loaded while this one's are used
    constexpr int E = kSicTile / 256;
    double pn[E], vn[E];
    auto load = [&](int i) {
        const double *ph = PHI + ch.off + (long long)i * ch.M;
        const double *vh = V + ch.off + (long long)i * ch.M;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const long long m = base + e * 256 + threadIdx.x;
            pn[e] = m < ch.M ? ph[m] : 0.0;
            vn[e] = m < ch.M ? vh[m] : 0.0;
        }
    };
    if (ch.N > 0) load(0);
    for (int i = 0; i < ch.N; ++i) {
        double pc[E], vc_[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            pc[e] = pn[e];
            vc_[e] = vn[e];
        }
        if (i + 1 < ch.N) load(i + 1);
        double u = 0.0, x = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const long long m = base + e * 256 + threadIdx.x;
            if (m < ch.M) {
                const double p = pc[e];
                const double r = p * p;
                const double v = vc_[e];
                double ex, ec, vx, vc;
                lsda_pol(r, floor, ex, ec, vx, vc);
                u += r * v;
                x += r * (ex + ec);
                const double Vi = -(v + vx + vc);
                num[e] += r * Vi;
                den[e] += r;
            }
        }
        u = wave_sum(u);
        x = wave_sum(x);
        if ((threadIdx.x & 63) == 0) {
            su[w][i] = u;
            sx[w][i] = x;
        }
    }
    if (ch.vsic) {
#pragma unroll
        for (int e = 0; e < kSicTile / 256; ++e) {
            const long long m = base + e * 256 + threadIdx.x;
            if (m < ch.M) ch.vsic[m] = (den[e] > floor) ? ch.vscale * num[e] / den[e] : 0.0;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ch.N; i += 256) {
        partU[(size_t)blockIdx.x * kMaxOrb + i] = (su[0][i] + su[1][i]) + (su[2][i] + su[3][i]);
        partX[(size_t)blockIdx.x * kMaxOrb + i] = (sx[0][i] + sx[1][i]) + (sx[2][i] + sx[3][i]);
    }
}

// U_i and X_i: one block per (channel, orbital) sums the partials of the
// channel's blocks in a fixed order
__global__ __launch_bounds__(256) void k_sic_energy(const ChanDesc *chans, const double *partU,
                                                    const double *partX, double *U, double *X) {
    __shared__ double sred[4];
    const ChanDesc ch = chans[blockIdx.y];
    const int i = blockIdx.x;
    if (i >= ch.N) return;  // uniform
    const double dV = ch.h * ch.h * ch.h;
    double su = 0.0, sx = 0.0;
    for (int t = threadIdx.x; t < ch.nblk; t += 256) {
        su += partU[(size_t)(ch.blk_base + t) * kMaxOrb + i];
        sx += partX[(size_t)(ch.blk_base + t) * kMaxOrb + i];
    }
    su = block_sum256(su, sred);
    sx = block_sum256(sx, sred);
    if (threadIdx.x == 0) {
        U[ch.first_orb + i] = 0.5 * dV * su;
        X[ch.first_orb + i] = dV * sx;
    }
}

// E_SIC of each channel: -sum_i (U_i + X_i) in orbital order
__global__ void k_sic_echan(const ChanDesc *chans, const double *U, const double *X, double *Echan) {
    const ChanDesc ch = chans[blockIdx.x];
    if (threadIdx.x != 0) return;
    double e = 0.0;
    for (int i = 0; i < ch.N; ++i) e -= U[ch.first_orb + i] + X[ch.first_orb + i];
    Echan[blockIdx.x] = e;
}

hipError_t launch_sic_average(int nchan, const ChanDesc *chan, int nblk_total,
                              const int *blk_chan, const double *PHI, const double *V,
                              double floor, double *partU, double *partX, hipStream_t s) {
    (void)nchan;
    if (nblk_total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sic_average, dim3(nblk_total), dim3(256), 0, s, chan, blk_chan, PHI, V,
                       floor, partU, partX);
    return hipGetLastError();
}

hipError_t launch_sic_energy(int nchan, const ChanDesc *chan, const double *partU,
                             const double *partX, double *U, double *X, double *Echan,
                             hipStream_t s) {
    if (nchan <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sic_energy, dim3(kMaxOrb, nchan), dim3(256), 0, s, chan, partU, partX, U, X);
    hipLaunchKernelGGL(k_sic_echan, dim3(nchan), dim3(64), 0, s, chan, U, X, Echan);
    return hipGetLastError();
}

}  // namespace fsic
