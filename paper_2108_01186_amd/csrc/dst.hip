// Spectral preconditioner of the per-orbital Poisson problems.
//
// The star Laplacian with zero values outside the box (Sec. II.A, the
// operator the CG solves with) differs from its odd reflection at the faces
// only in the few rows whose taps reach past the first ghost.  The
// reflected operator is diagonalised by the type-I discrete sine transform
// along each axis, S_n[m][k] = sin(pi (m+1)(k+1) / (n+1)), with eigenvalues
//   lambda(j, k, l) = (s_x(j) + s_y(k) + s_z(l)) / h^2,
//   s_n(j) = -(c_0 + 2 sum_m c_m cos(m theta_j)), theta_j = pi (j+1) / (n+1),
// so M^{-1} r = (prod_d 2 / (n_d + 1)) S_x S_y S_z diag(1/lambda) S_z S_y S_x r
// is an SPD preconditioner that leaves only the face corrections for CG.
//
// An application is a sequence of batched passes over a float work array,
// each multiplying panels of the field by n x n sine matrices on the matrix
// cores:
//   * k_dst_xy (in-plane axes up to 128 nodes): the x and y transforms of
//     one z plane in one visit, forward (reads r) and inverse (writes z);
//   * k_dst_fast<2, 1>: the z transform, the 1/lambda scaling and the
//     inverse z transform, with the r.z partial sums;
//   * otherwise five per-axis passes of k_dst_fast (x, y, z with the 1/lambda
//     scaling and the r.z partial sums, y, x).
// The last pass writes z, or directly the next CG search direction
// p = z + beta p_old (PcgOut).  The kernels split each fp32 operand into
// bf16 hi + lo (see below).
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <set>
#include <tuple>

#include "kernels.h"

namespace fsic {

typedef float flt4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ int axis_n(const OrbDesc &od, int ax) {
    return ax == 0 ? od.nx : (ax == 1 ? od.ny : od.nz);
}

}  // namespace

// ---------------------------------------------------------------------------
// fast pass (axes of at most 128 nodes): bf16 matrix cores with split operands
// ---------------------------------------------------------------------------
//
// Each fp32 operand is split into bf16 hi + lo (lo = x - hi), and
// S X ~ S_hi X_hi + S_hi X_lo + S_lo X_hi on v_mfma_f32_16x16x32_bf16 with
// fp32 accumulation, which keeps about 16 significant bits (the dropped
// S_lo X_lo term is ~2^-16 relative): the preconditioner then behaves as in
// fp32 while the matrix cores do five times less work.  A persistent
// 512-thread block streams a contiguous range of (orbital, 128-column panel)
// units: S (hi, lo) of the current axis length stays in LDS (restaged only
// when the length changes) and the next unit's loads are in flight while the
// current panel is multiplied (two register buffers: the loads of the unit
// after next are issued once the current unit's values are in LDS).
// Operand layouts: A lane l holds S[m0 + l%16][k0 + 8(l/16) .. +7], B lane l
// holds X[k0 + 8(l/16) .. +7][c0 + l%16] (the panel is stored transposed,
// Xt[c][k], so both are one 16-byte LDS read), and D lane l, item j is
// C[m0 + 4(l/16) + j][c0 + l%16].

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

constexpr int kFT = 512;   // threads per block (8 waves)
constexpr int kFV = 32;    // panel values per thread and buffer: np * PC / kFT <= 32
constexpr int kNV2 = 20;   // fused x-y pass with two blocks per compute unit: plane <= kNV2 * kFT
constexpr int kNVZ = 12;   // z pass with two blocks per compute unit: np * 64 <= kNVZ * kFT (np <= 96)

__device__ __forceinline__ void bsplit(float x, __bf16 &hi, __bf16 &lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// fixed-order sum over the waves of a kFT-thread block (all threads get it);
// the barriers order LDS only, so global loads and stores stay in flight
__device__ __forceinline__ double block_sum_fast(double v, double *sbuf) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    lds_barrier();
    if ((threadIdx.x & 63) == 0) sbuf[w] = v;
    lds_barrier();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kFT / 64; ++i) s += sbuf[i];
    return s;
}

size_t dst_fast_lds(int np, int pc, bool slo) {
    const int sw = np + 8;
    return (size_t)(slo ? 2 : 1) * np * sw * 2 + (size_t)2 * pc * sw * 2 + 16 * sizeof(double) +
           (size_t)np * sizeof(float);
}

// 16-byte loads of four consecutive values as floats
__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ float4 ld4(const double *p) {
    const double2 a = *reinterpret_cast<const double2 *>(p);
    const double2 b = *reinterpret_cast<const double2 *>(p + 2);
    return float4{(float)a.x, (float)a.y, (float)b.x, (float)b.y};
}

// TR (the solve's residual type) only names the instantiation per precision.
// RZ (z pass): r.z partial sums from the spectral coefficients.  PO (last
// pass): write p = z + beta p_old as described by po.  NPM (one block per
// compute unit): the longest padded axis the instantiation serves; it sizes
// the register buffers and accumulator tiles.
template <int AX, int MODE, typename TIN, typename TR, bool RZ, int PC, bool SLO, bool OCC2 = false,
          bool PO = false, int NPM = (PC == 128 ? 128 : 256)>
__global__ __launch_bounds__(kFT, OCC2 ? 4 : 2) void k_dst_fast(const Item *units, int nunits, int npmax,
                                                  const OrbDesc *orb, const int *done,
                                                  const float *tab, const TIN *in, float *out,
                                                  double *rz, PcgOut po, int *cnt) {
    static_assert(!RZ || MODE == 1, "r.z comes from the z pass");
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    // persistent: block b streams the units [u0, u1) (unit = orbital, panel);
    // the LDS layout is sized for the largest axis of the batch
    const int sw = npmax + 8;  // LDS row stride (bf16): 16-byte rows
    constexpr int G = kFT / PC;  // threads per panel column in the loads
    __bf16 *Shi = reinterpret_cast<__bf16 *>(smem);
    __bf16 *Slo = Shi + (size_t)npmax * sw;  // only with SLO
    __bf16 *Xhi = Slo + (SLO ? (size_t)npmax * sw : 0);
    __bf16 *Xlo = Xhi + (size_t)PC * sw;
    double *sred = reinterpret_cast<double *>(Xlo + (size_t)PC * sw);  // kFT / 64 doubles
    const int t = threadIdx.x;
    const int u0 = (int)((long long)blockIdx.x * nunits / gridDim.x);
    const int u1 = (int)((long long)(blockIdx.x + 1) * nunits / gridDim.x);
    auto next_active = [&](int u) {  // done[] and pz[] do not change during this launch: uniform
        while (u < u1 && (units[u].orb < 0 || done[units[u].orb] || (po.pz && po.pz[units[u].orb] <= po.li)))
            ++u;
        return u;
    };

    // matrix view of an orbital's field along AX: column cg of ncol,
    // element k at eoff(cg) + k * kstr
    auto ncol_of = [&](const OrbDesc &od) -> long long {
        return AX == 0 ? (long long)od.ny * od.nz
                       : (AX == 1 ? (long long)od.nx * od.nz : (long long)od.nx * od.ny);
    };
    auto kstr_of = [&](const OrbDesc &od) -> long long {
        return AX == 0 ? 1 : (AX == 1 ? (long long)od.nx : (long long)od.nx * od.ny);
    };
    auto eoff = [&](const OrbDesc &od, long long cg) -> long long {
        if (AX == 0) return cg * od.nx;
        if (AX == 1) {
            const long long z = cg / od.nx;
            return z * ((long long)od.nx * od.ny) + (cg - z * od.nx);
        }
        return cg;
    };

    // x axis with nx and the orbital offset multiples of 4: rows go in and out
    // as 16-byte vectors
    auto xvec = [&](const OrbDesc &od) -> bool {
        return AX == 0 && (od.nx & 3) == 0 && (od.off & 3) == 0;
    };
    // OCC2 (two blocks per compute unit, np * PC <= kNVZ * kFT): one register
    // buffer and no prefetch inside the block; the other resident block
    // overlaps its memory traffic with this one's products
    constexpr int NV = OCC2 ? kNVZ : NPM * PC / kFT;
    static_assert(OCC2 || (NPM * PC % (4 * kFT) == 0 && NV <= kFV), "panel values per thread");
    // panel loads into v[NV]: thread t holds column c_ld and, per i, either
    // rows k = 2 kg + 2 G i, k + 1 (pairs) or k = 4 kg + 4 G i .. + 3 (x vectors)
    const int c_ld = AX == 0 ? (t / G) : (t % PC);
    const int kg = AX == 0 ? (t % G) : (t / PC);
    auto load = [&](float (&v)[NV], const OrbDesc &od, int pnl) {
        const int n = axis_n(od, AX);
        const int np = (n + 31) & ~31;
        const long long cg = (long long)pnl * PC + c_ld;
        const bool cv = cg < ncol_of(od);
        const long long base = od.off + (cv ? eoff(od, cg) : 0);
        if (xvec(od)) {
#pragma unroll
            for (int i = 0; i < NV / 4; ++i) {
                const int k = 4 * kg + 4 * G * i;
                const float4 q = (k < np && cv && k < n) ? ld4(in + base + k) : float4{0.f, 0.f, 0.f, 0.f};
                v[4 * i] = q.x; v[4 * i + 1] = q.y; v[4 * i + 2] = q.z; v[4 * i + 3] = q.w;
            }
            return;
        }
        const long long ks = kstr_of(od);
        const int npair = np / (2 * G);
#pragma unroll
        for (int i = 0; i < NV / 2; ++i) {
            const int k = 2 * kg + 2 * G * i;
            v[2 * i] = (i < npair && cv && k < n) ? (float)in[base + (long long)k * ks] : 0.f;
            v[2 * i + 1] = (i < npair && cv && k + 1 < n) ? (float)in[base + (long long)(k + 1) * ks] : 0.f;
        }
    };
    auto to_lds = [&](const float (&v)[NV], const OrbDesc &od) {
        const int np = (axis_n(od, AX) + 31) & ~31;
        if (xvec(od)) {
#pragma unroll
            for (int i = 0; i < NV / 4; ++i) {
                const int k = 4 * kg + 4 * G * i;
                if (k < np) {
                    __bf16 h[4], l[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) bsplit(v[4 * i + j], h[j], l[j]);
                    *reinterpret_cast<bf4 *>(Xhi + c_ld * sw + k) = bf4{h[0], h[1], h[2], h[3]};
                    *reinterpret_cast<bf4 *>(Xlo + c_ld * sw + k) = bf4{l[0], l[1], l[2], l[3]};
                }
            }
            return;
        }
        const int npair = np / (2 * G);
#pragma unroll
        for (int i = 0; i < NV / 2; ++i) {
            if (i < npair) {
                const int k = 2 * kg + 2 * G * i;
                __bf16 h0, l0, h1, l1;
                bsplit(v[2 * i], h0, l0);
                bsplit(v[2 * i + 1], h1, l1);
                *reinterpret_cast<bf2 *>(Xhi + c_ld * sw + k) = bf2{h0, h1};
                *reinterpret_cast<bf2 *>(Xlo + c_ld * sw + k) = bf2{l0, l1};
            }
        }
    };

    // wave tiling: PC / 16 column tiles; the waves of a column tile split its
    // row tiles (stride RS)
    const int lane = t & 63, w = t >> 6;
    constexpr int NCT = PC / 16;
    constexpr int RS = (kFT / 64) / NCT;
    const int ct = w % NCT, r0 = w / NCT;
    constexpr int MT = OCC2 ? 3 : NPM / 16 / RS;  // row tiles per wave: np / 16 / RS <= MT (OCC2: np <= 96)
    const int lr = lane & 15, lq = lane >> 4;
    flt4 acc[MT];
    auto gemm = [&](int np) {
        const int nrt = np >> 4;
#pragma unroll
        for (int i = 0; i < MT; ++i) acc[i] = flt4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < np; k0 += 32) {
            const int kb = k0 + 8 * lq;
            const bf8 bh = *reinterpret_cast<const bf8 *>(Xhi + (ct * 16 + lr) * sw + kb);
            const bf8 bl = *reinterpret_cast<const bf8 *>(Xlo + (ct * 16 + lr) * sw + kb);
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const int rt = r0 + RS * i;
                if (rt < nrt) {
                    const bf8 ah = *reinterpret_cast<const bf8 *>(Shi + (rt * 16 + lr) * sw + kb);
                    if constexpr (SLO) {
                        const bf8 al = *reinterpret_cast<const bf8 *>(Slo + (rt * 16 + lr) * sw + kb);
                        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[i], 0, 0, 0);
                    }
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[i], 0, 0, 0);
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[i], 0, 0, 0);
                }
            }
        }
    };

    float *gzs = reinterpret_cast<float *>(sred + 16);  // eigenvalue symbol of the staged z length
    int staged = -1;  // axis length whose sine matrix is in LDS
    int borb = -1;    // orbital whose beta is in `beta` (PO)
    float beta = 0.f;
    // one unit: products of the panel held in v; the unit `pf` (or u1: none)
    // is loaded into v once its values are in LDS
    auto unit = [&](float (&v)[NV], int u, OrbDesc &od, int pf) {
        const Item cur = units[u];
        const OrbDesc oc = od;
        const int n = axis_n(oc, AX);
        const int np = (n + 31) & ~31;
        if (cnt && cur.tile == 0 && t == 0) cnt[cur.orb] += 1;
        lds_barrier();  // the previous unit's products are done with S and Xt
        if constexpr (PO) {
            if (!po.first && cur.orb != borb) {  // uniform: the whole block takes it
                double a = 0.0, b = 0.0;
                for (int i = t; i < oc.nt9; i += kFT) {
                    a += po.rzc[oc.base9 + i];
                    b += po.rzp[oc.base9 + i];
                }
                a = block_sum_fast(a, sred);
                b = block_sum_fast(b, sred);
                beta = b != 0.0 ? (float)(a / b) : 0.f;
                borb = cur.orb;
            }
        }
        if (n != staged) {
            const float *S = tab + oc.dst_s[AX];  // np x np, zero beyond n
            for (int e = t; e < np * np; e += kFT) {
                const int m = e / np, k = e - m * np;
                __bf16 hi, lo;
                bsplit(S[e], hi, lo);
                Shi[m * sw + k] = hi;
                if constexpr (SLO) Slo[m * sw + k] = lo;
            }
            if (MODE == 1)
                for (int m = t; m < n; m += kFT) gzs[m] = tab[oc.dst_g[2] + m];
            staged = n;
        }
        to_lds(v, oc);
        lds_barrier();
        if (pf < u1) {  // two units ahead: in flight during this unit and the next
            od = orb[units[pf].orb];
            load(v, od, units[pf].tile);
        }
        gemm(np);
        const int nrt = np >> 4;
        const int c = ct * 16 + lr;
        const long long cg = (long long)cur.tile * PC + c;
        const bool cv = cg < ncol_of(oc);
        double part = 0.0;
        if (MODE == 1) {
            // scale by norm / lambda(jx, jy, m) and transform again
            const float *gx = tab + oc.dst_g[0], *gy = tab + oc.dst_g[1];
            const float norm = 8.f / ((float)(oc.nx + 1) * (float)(oc.ny + 1) * (float)(oc.nz + 1));
            const float ih2 = (float)oc.inv_h2;
            const int jy = cv ? (int)(cg / oc.nx) : 0, jx = cv ? (int)(cg - (long long)jy * oc.nx) : 0;
            const float gxy = cv ? gx[jx] + gy[jy] : 1.f;
            lds_barrier();  // every wave is done reading Xt
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const int rt = r0 + RS * i;
                if (rt < nrt) {
                    const int m0 = rt * 16 + 4 * lq;
                    __bf16 hh[4], ll[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int m = m0 + j;
                        const float vv = (cv && m < n) ? acc[i][j] * (norm / ((gxy + gzs[m]) * ih2)) : 0.f;
                        // r.z = c sum_k rhat_k^2 / lambda_k (rhat = S r, S^2 = I / c)
                        if (RZ) part += (double)acc[i][j] * (double)vv;
                        bsplit(vv, hh[j], ll[j]);
                    }
                    *reinterpret_cast<bf4 *>(Xhi + c * sw + m0) = bf4{hh[0], hh[1], hh[2], hh[3]};
                    *reinterpret_cast<bf4 *>(Xlo + c * sw + m0) = bf4{ll[0], ll[1], ll[2], ll[3]};
                }
            }
            lds_barrier();
            gemm(np);
        }
        if (cv) {
            const long long eo = oc.off + eoff(oc, cg);
            const long long ks = kstr_of(oc);
            const bool vec = xvec(oc);
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const int rt = r0 + RS * i;
                if (rt < nrt) {
                    const int m0 = rt * 16 + 4 * lq;
                    if (vec) {
                        if (m0 < n) {  // n % 4 == 0: all four rows are in range
                            float4 q = float4{acc[i][0], acc[i][1], acc[i][2], acc[i][3]};
                            if (PO && !po.first) {
                                const float4 o = ld4(po.pold + eo + m0);
                                q = float4{q.x + beta * o.x, q.y + beta * o.y, q.z + beta * o.z,
                                           q.w + beta * o.w};
                            }
                            *reinterpret_cast<float4 *>(out + eo + m0) = q;
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int m = m0 + j;
                            if (m < n) {
                                const long long a = eo + (long long)m * ks;
                                out[a] = (PO && !po.first) ? acc[i][j] + beta * po.pold[a] : acc[i][j];
                            }
                        }
                    }
                }
            }
        }
        if (RZ) {
            const double sum = block_sum_fast(part, sred);
            if (t == 0) rz[oc.base9 + cur.tile] = sum;
        }
    };

    if constexpr (OCC2) {
        // one register buffer: once a unit's values are in LDS the next
        // unit's loads go into it, in flight during this unit's products
        float v[NV];
        int q = next_active(u0);
        if (q >= u1) return;
        OrbDesc o = orb[units[q].orb];
        load(v, o, units[q].tile);
        while (q < u1) {
            const int qn = next_active(q + 1);
            unit(v, q, o, qn);  // o becomes unit qn's descriptor
            q = qn;
        }
        return;
    }
    // two register buffers: va holds unit q0, vb unit q1 (u1: none)
    float va[NV], vb[NV];
    int q0 = next_active(u0);
    if (q0 >= u1) return;
    int q1 = next_active(q0 + 1);
    OrbDesc o0 = orb[units[q0].orb], o1;
    load(va, o0, units[q0].tile);
    if (q1 < u1) {
        o1 = orb[units[q1].orb];
        load(vb, o1, units[q1].tile);
    }
    while (true) {
        const int q2 = q1 < u1 ? next_active(q1 + 1) : u1;
        unit(va, q0, o0, q2);
        q0 = q2;
        if (q1 >= u1) break;
        const int q3 = q0 < u1 ? next_active(q0 + 1) : u1;
        unit(vb, q1, o1, q3);
        q1 = q3;
        if (q0 >= u1) break;
    }
}

// ---------------------------------------------------------------------------
// fused x-y pass: both in-plane transforms of one z plane in one visit
// ---------------------------------------------------------------------------
//
// Unit = (orbital, z plane).  The plane P (ny x nx) is staged in LDS as
// split bf16 (rows y, stride sw), then
//   C1 = P Sx      (x transform of every row; Sx symmetric),
//   C2 = Sy C1     (y transform of every column),
// with C1 written back transposed (C1t[x][y]) over P so that both products
// read their B operand as one 16-byte LDS row segment.  The transforms along
// different axes commute, so the same kernel serves the forward pass (reads
// the CG residual) and the inverse pass (writes z).  Each application of the
// preconditioner then moves the field through HBM three times (xy, z, xy)
// instead of five, and the z pass between them forms r.z from the spectral
// coefficients it already holds (r.z = c sum_k rhat_k^2 / lambda_k), so the
// inverse pass does not read r.
// VEC (every nx and orbital offset of the batch a multiple of 4) moves the
// planes as 16-byte vectors; otherwise as single values.
// Wave w computes the 32 x (npx / 2) block of C at rows 32 (w / 2) and
// columns (w % 2) npx / 2: two row tiles times npx / 32 column tiles, so each
// A fragment is reused over the column tiles and each B fragment over both
// row tiles.  Waves w >= npy / 16 only move data.
// two fused x-y blocks fit one compute unit: the plane (<= 96 x 96) fits the
// single register buffer and two blocks' LDS fit 160 KB
bool dst_xy_occ2(int np, bool two) {
    return np <= 96 && (size_t)np * np <= (size_t)kNV2 * kFT && 2 * dst_xy_lds(np, two) <= 160 * 1024;
}

// two z-pass blocks (64-column panels with S_lo) fit one compute unit
bool dst_z_occ2(int np) {
    return np <= 96 && np * 64 <= kNVZ * kFT && 2 * dst_fast_lds(np, 64, true) <= 160 * 1024;
}

size_t dst_xy_lds(int np, bool two) {
    const int sw = np + 8;
    return (size_t)2 * np * sw * 2 + (size_t)(two ? 2 : 1) * 2 * np * sw * 2 + 16 * sizeof(double);
}

// TR (the solve's residual type) only names the instantiation per precision.
// PO: write p = z + beta p_old as described by po (the inverse pass).  PV
// (with PO): load this lane's p_old values before the products instead of at
// the store.
template <bool VEC, typename TIN, typename TR, bool OCC2, bool PO = false, bool PV = false>
__global__ __launch_bounds__(kFT, OCC2 ? 4 : 2) void k_dst_xy(const Item *units, int nunits, int npmax, int two,
                                                               const OrbDesc *orb, const int *done,
                                                               const float *tab, const TIN *in, float *out,
                                                               PcgOut po, int *cnt) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int sw = npmax + 8;  // LDS row stride (bf16): 16-byte rows
    __bf16 *Xhi = reinterpret_cast<__bf16 *>(smem);
    __bf16 *Xlo = Xhi + (size_t)npmax * sw;
    __bf16 *Sxh = Xlo + (size_t)npmax * sw;
    __bf16 *Sxl = Sxh + (size_t)npmax * sw;
    __bf16 *Syh = two ? Sxl + (size_t)npmax * sw : Sxh;
    __bf16 *Syl = two ? Syh + (size_t)npmax * sw : Sxl;
    double *sred = reinterpret_cast<double *>(Syl + (size_t)npmax * sw);  // kFT / 64 doubles
    const int t = threadIdx.x;
    const int u0 = (int)((long long)blockIdx.x * nunits / gridDim.x);
    const int u1 = (int)((long long)(blockIdx.x + 1) * nunits / gridDim.x);
    auto next_active = [&](int u) {  // done[] and pz[] do not change during this launch: uniform
        while (u < u1 && (units[u].orb < 0 || done[units[u].orb] || (po.pz && po.pz[units[u].orb] <= po.li)))
            ++u;
        return u;
    };
    // VEC (every nx and orbital offset a multiple of 4): planes move as
    // 16-byte vectors
    // OCC2 (planes up to kNV2 * kFT nodes, two blocks per compute unit): one
    // register buffer, no prefetch inside the block; the other resident block
    // overlaps its memory traffic with this one's products
    constexpr int NV = OCC2 ? kNV2 : kFV;
    // plane loads into v[NV]: vector group g = t + kFT i (elements 4g .. 4g+3)
    // or element e = t + kFT i, in row-major (y, x) order
    auto load = [&](float (&v)[NV], const OrbDesc &od, int z) {
        const int pl = od.nx * od.ny;
        const long long base = od.off + (long long)z * pl;
        if (VEC) {
#pragma unroll
            for (int i = 0; i < NV / 4; ++i) {
                const int g = t + kFT * i;
                const float4 q = (4 * g < pl) ? ld4(in + base + 4 * g) : float4{0.f, 0.f, 0.f, 0.f};
                v[4 * i] = q.x; v[4 * i + 1] = q.y; v[4 * i + 2] = q.z; v[4 * i + 3] = q.w;
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int e = t + kFT * i;
            v[i] = (e < pl) ? (float)in[base + e] : 0.f;
        }
    };
    auto to_lds = [&](const float (&v)[NV], const OrbDesc &od) {
        const int nx = od.nx, pl = od.nx * od.ny;
        if (VEC) {
#pragma unroll
            for (int i = 0; i < NV / 4; ++i) {
                const int g = t + kFT * i;
                if (4 * g < pl) {
                    const int y = (4 * g) / nx, x = 4 * g - y * nx;
                    __bf16 h[4], l[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) bsplit(v[4 * i + j], h[j], l[j]);
                    *reinterpret_cast<bf4 *>(Xhi + y * sw + x) = bf4{h[0], h[1], h[2], h[3]};
                    *reinterpret_cast<bf4 *>(Xlo + y * sw + x) = bf4{l[0], l[1], l[2], l[3]};
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int e = t + kFT * i;
                if (e < pl) {
                    const int y = e / nx, x = e - y * nx;
                    __bf16 h, l;
                    bsplit(v[i], h, l);
                    Xhi[y * sw + x] = h;
                    Xlo[y * sw + x] = l;
                }
            }
        }
        // zero the padding the products read: columns nx .. npx-1, rows ny .. npy-1
        const int npx = (od.nx + 31) & ~31, npy = (od.ny + 31) & ~31;
        if (npx != od.nx || npy != od.ny)
            for (int e = t; e < npy * npx; e += kFT) {
                const int y = e / npx, x = e - y * npx;
                if (y >= od.ny || x >= od.nx) {
                    Xhi[y * sw + x] = (__bf16)0.f;
                    Xlo[y * sw + x] = (__bf16)0.f;
                }
            }
    };

    const int lane = t & 63, w = t >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    const int rb = w >> 1, cb = w & 1;
    constexpr int BC = OCC2 ? 3 : 4;  // column tiles per wave: npx / 32 <= BC
    flt4 acc[2][BC];
    // acc = A B over k < npk for the wave's block; A rows from Ah/Al
    // (row-major, stride sw), B as Bt[col][k] from Bh/Bl
    auto gemm = [&](const __bf16 *Ah, const __bf16 *Al, const __bf16 *Bh, const __bf16 *Bl, int npk,
                    int bc) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < BC; ++c) acc[r][c] = flt4{0.f, 0.f, 0.f, 0.f};
        const int row0 = 32 * rb, col0 = cb * 16 * bc;
#pragma unroll 1
        for (int k0 = 0; k0 < npk; k0 += 32) {
            const int kb = k0 + 8 * lq;
            bf8 ah[2], al[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                ah[r] = *reinterpret_cast<const bf8 *>(Ah + (row0 + 16 * r + lr) * sw + kb);
                al[r] = *reinterpret_cast<const bf8 *>(Al + (row0 + 16 * r + lr) * sw + kb);
            }
#pragma unroll
            for (int c = 0; c < BC; ++c) {
                if (c < bc) {
                    const bf8 bh = *reinterpret_cast<const bf8 *>(Bh + (col0 + 16 * c + lr) * sw + kb);
                    const bf8 bl = *reinterpret_cast<const bf8 *>(Bl + (col0 + 16 * c + lr) * sw + kb);
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[r], bh, acc[r][c], 0, 0, 0);
                        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bl, acc[r][c], 0, 0, 0);
                        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bh, acc[r][c], 0, 0, 0);
                    }
                }
            }
        }
    };

    int sx_n = -1, sy_n = -1;  // axis lengths whose sine matrices are in LDS
    int borb = -1;             // orbital whose beta is in `beta` (PO)
    float beta = 0.f;
    auto stage_s = [&](__bf16 *Sh, __bf16 *Sl, const float *S, int np) {
        for (int e = t; e < np * np; e += kFT) {
            const int m = e / np, k = e - m * np;
            __bf16 hi, lo;
            bsplit(S[e], hi, lo);
            Sh[m * sw + k] = hi;
            Sl[m * sw + k] = lo;
        }
    };
    auto unit = [&](float (&v)[NV], int u, OrbDesc &od, int pf) {
        const Item cur = units[u];
        const OrbDesc oc = od;
        const int nx = oc.nx, ny = oc.ny;
        const int npx = (nx + 31) & ~31, npy = (ny + 31) & ~31;
        const int bc = npx >> 5;
        const bool act = rb < (npy >> 5);
        if (cnt && cur.tile == 0 && t == 0) cnt[cur.orb] += 1;
        lds_barrier();  // the previous unit's products are done with S and X
        if constexpr (PO) {
            if (!po.first && cur.orb != borb) {  // uniform: the whole block takes it
                double a = 0.0, b = 0.0;
                for (int i = t; i < oc.nt9; i += kFT) {
                    a += po.rzc[oc.base9 + i];
                    b += po.rzp[oc.base9 + i];
                }
                a = block_sum_fast(a, sred);
                b = block_sum_fast(b, sred);
                beta = b != 0.0 ? (float)(a / b) : 0.f;
                borb = cur.orb;
            }
        }
        if (nx != sx_n || (two && ny != sy_n)) {
            stage_s(Sxh, Sxl, tab + oc.dst_s[0], npx);
            if (two) stage_s(Syh, Syl, tab + oc.dst_s[1], npy);
            sx_n = nx;
            sy_n = ny;
        }
        to_lds(v, oc);
        lds_barrier();
        if (pf < u1) {  // two units ahead: in flight during this unit and the next
            od = orb[units[pf].orb];
            load(v, od, units[pf].tile);
        }
        const long long base = oc.off + (long long)cur.tile * nx * ny;
        // PO: p_old at this lane's output nodes, loaded now so the loads are
        // in flight during both products
        float pv[2][BC][4];
        if (PO && PV && !po.first && act) {
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < BC; ++c)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int x = cb * 16 * bc + 16 * c + lr;
                        const int y = 32 * rb + 16 * r + 4 * lq + j;
                        pv[r][c][j] = (c < bc && x < nx && y < ny) ? po.pold[base + (long long)y * nx + x] : 0.f;
                    }
        }
        // C1 = P Sx: rows y, columns x
        if (act) gemm(Xhi, Xlo, Sxh, Sxl, npx, bc);
        lds_barrier();  // every wave is done reading P
        if (act) {
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < BC; ++c) {
                    if (c < bc) {
                        const int x = cb * 16 * bc + 16 * c + lr;
                        const int y0 = 32 * rb + 16 * r + 4 * lq;
                        __bf16 hh[4], ll[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) bsplit(acc[r][c][j], hh[j], ll[j]);
                        *reinterpret_cast<bf4 *>(Xhi + x * sw + y0) = bf4{hh[0], hh[1], hh[2], hh[3]};
                        *reinterpret_cast<bf4 *>(Xlo + x * sw + y0) = bf4{ll[0], ll[1], ll[2], ll[3]};
                    }
                }
        }
        lds_barrier();
        // C2 = Sy C1: rows y, columns x (B = C1t)
        if (act) gemm(Syh, Syl, Xhi, Xlo, npy, bc);
        if (act) {
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < BC; ++c) {
                    const int x = cb * 16 * bc + 16 * c + lr;
                    if (c < bc && x < nx) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int y = 32 * rb + 16 * r + 4 * lq + j;
                            if (y < ny) {
                                const long long a = base + (long long)y * nx + x;
                                float o = 0.f;
                                if (PO && !po.first) o = PV ? pv[r][c][j] : po.pold[a];  // (PV: loaded early)
                                out[a] = (PO && !po.first) ? acc[r][c][j] + beta * o : acc[r][c][j];
                            }
                        }
                    }
                }
        }
    };

    if constexpr (OCC2) {
        // one register buffer; the other resident block overlaps its memory
        // traffic with this one's products (a prefetch into this buffer
        // during the products measured no faster and spills)
        float v[NV];
        for (int q = next_active(u0); q < u1; q = next_active(q + 1)) {
            OrbDesc o = orb[units[q].orb];
            load(v, o, units[q].tile);
            unit(v, q, o, u1);
        }
        return;
    }
    float va[NV], vb[NV];
    int q0 = next_active(u0);
    if (q0 >= u1) return;
    int q1 = next_active(q0 + 1);
    OrbDesc o0 = orb[units[q0].orb], o1;
    load(va, o0, units[q0].tile);
    if (q1 < u1) {
        o1 = orb[units[q1].orb];
        load(vb, o1, units[q1].tile);
    }
    while (true) {
        const int q2 = q1 < u1 ? next_active(q1 + 1) : u1;
        unit(va, q0, o0, q2);
        q0 = q2;
        if (q1 >= u1) break;
        const int q3 = q0 < u1 ? next_active(q0 + 1) : u1;
        unit(vb, q1, o1, q3);
        q1 = q3;
        if (q0 >= u1) break;
    }
}

template <class K>
void set_lds_limit(K kern, size_t bytes) {
    if (bytes > 65536) hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

namespace {

// The passes of one preconditioner application.  T: type of r; PO: the last
// pass writes p = z + beta p_old (po) into `out` instead of z.
template <typename T, bool PO>
hipError_t dst_apply(const DstItems &di, const OrbDesc *orb, const int *done, const float *tab,
                     const T *r, float *work, float *out, double *rz, const PcgOut &po, int *cnt,
                     hipStream_t s) {
    if (di.nx <= 0 && di.nxy <= 0) return hipSuccess;
    if (!di.fast) return hipErrorInvalidValue;  // the host solves such batches without it
    const float *wk = work;
    int *nc = nullptr;
    // forward and middle passes: no p output, but the pause state of po
    const PcgOut none{nullptr, nullptr, nullptr, 1, po.pz, po.li};
    const bool pv = di.pv != 0;
    auto grid = [&](int units) { return dim3((unsigned)std::min(units, di.blocks)); };
#define FSIC_DST_FAST(PC_, SLO_, NPM_)                                                                \
    do {                                                                                              \
        const size_t lds = dst_fast_lds(di.np, PC_, SLO_);                                            \
        const size_t lz = dst_fast_lds(di.np, 64, SLO_);                                              \
        hipLaunchKernelGGL((k_dst_fast<0, 0, T, T, false, PC_, SLO_, false, false, NPM_>), grid(di.nx), \
                           dim3(kFT), lds, s, di.x, di.nx, di.np, orb, done, tab, r, work, nullptr,    \
                           none, cnt);                                                                 \
        hipLaunchKernelGGL((k_dst_fast<1, 0, float, T, false, PC_, SLO_, false, false, NPM_>),          \
                           grid(di.ny), dim3(kFT), lds, s, di.y, di.ny, di.np, orb, done, tab, wk,     \
                           work, nullptr, none, nc);                                                   \
        hipLaunchKernelGGL((k_dst_fast<2, 1, float, T, true, 64, SLO_, false, false, NPM_>),            \
                           grid(di.nz), dim3(kFT), lz, s, di.z, di.nz, di.np, orb, done, tab, wk, work, \
                           rz, none, nc);                                                              \
        hipLaunchKernelGGL((k_dst_fast<1, 0, float, T, false, PC_, SLO_, false, false, NPM_>),          \
                           grid(di.ny), dim3(kFT), lds, s, di.y, di.ny, di.np, orb, done, tab, wk,     \
                           work, nullptr, none, nc);                                                   \
        hipLaunchKernelGGL((k_dst_fast<0, 0, float, T, false, PC_, SLO_, false, PO, NPM_>), grid(di.nx), \
                           dim3(kFT), lds, s, di.x, di.nx, di.np, orb, done, tab, wk, out, nullptr,    \
                           po, nc);                                                                    \
    } while (0)
#define FSIC_DST_XY(SLO_, NPM_)                                                                       \
    do {                                                                                              \
        const size_t lxy = dst_xy_lds(di.npxy, di.two != 0);                                          \
        const size_t lz = dst_fast_lds(di.np, 64, SLO_);                                              \
        const bool o2 = di.xyvec && di.xyocc2 && dst_xy_occ2(di.npxy, di.two != 0);                   \
        const dim3 gxy = o2 ? dim3((unsigned)std::min(di.nxy, 2 * di.blocks)) : grid(di.nxy);         \
        if (o2)                                                                                       \
            hipLaunchKernelGGL((k_dst_xy<true, T, T, true>), gxy, dim3(kFT), lxy, s, di.xy, di.nxy,   \
                               di.npxy, di.two, orb, done, tab, r, work, none, cnt);                  \
        else if (di.xyvec)                                                                            \
            hipLaunchKernelGGL((k_dst_xy<true, T, T, false>), gxy, dim3(kFT), lxy, s, di.xy, di.nxy,  \
                               di.npxy, di.two, orb, done, tab, r, work, none, cnt);                  \
        else                                                                                          \
            hipLaunchKernelGGL((k_dst_xy<false, T, T, false>), gxy, dim3(kFT), lxy, s, di.xy, di.nxy, \
                               di.npxy, di.two, orb, done, tab, r, work, none, cnt);                  \
        if (di.zocc2)                                                                                 \
            hipLaunchKernelGGL((k_dst_fast<2, 1, float, T, true, 64, true, true>),                    \
                               dim3((unsigned)std::min(di.nz, 2 * di.blocks)), dim3(kFT),              \
                               dst_fast_lds(di.np, 64, true), s, di.z, di.nz, di.np, orb, done, tab,   \
                               wk, work, rz, none, nc);                                                \
        else                                                                                          \
            hipLaunchKernelGGL((k_dst_fast<2, 1, float, T, true, 64, SLO_, false, false, NPM_>),       \
                               grid(di.nz), dim3(kFT), lz, s, di.z, di.nz, di.np, orb, done, tab, wk,  \
                               work, rz, none, nc);                                                    \
        if (o2 && pv)                                                                                 \
            hipLaunchKernelGGL((k_dst_xy<true, float, T, true, PO, PO>), gxy, dim3(kFT), lxy, s, di.xy, \
                               di.nxy, di.npxy, di.two, orb, done, tab, wk, out, po, nc);             \
        else if (o2)                                                                                  \
            hipLaunchKernelGGL((k_dst_xy<true, float, T, true, PO>), gxy, dim3(kFT), lxy, s, di.xy,   \
                               di.nxy, di.npxy, di.two, orb, done, tab, wk, out, po, nc);             \
        else if (di.xyvec)                                                                            \
            hipLaunchKernelGGL((k_dst_xy<true, float, T, false, PO, PO>), gxy, dim3(kFT), lxy, s,     \
                               di.xy, di.nxy, di.npxy, di.two, orb, done, tab, wk, out, po, nc);      \
        else                                                                                          \
            hipLaunchKernelGGL((k_dst_xy<false, float, T, false, PO>), gxy, dim3(kFT), lxy, s, di.xy, \
                               di.nxy, di.npxy, di.two, orb, done, tab, wk, out, po, nc);             \
    } while (0)
    // the longest padded axis of each variant (kDstNpm) sizes its kernels
    if (di.nxy > 0) {
        if (di.fast == 1) FSIC_DST_XY(true, 128);
        else if (di.fast == 2) FSIC_DST_XY(true, 160);
        else FSIC_DST_XY(false, 192);
    } else if (di.fast == 1) FSIC_DST_FAST(128, true, 128);
    else if (di.fast == 2) FSIC_DST_FAST(64, true, 160);
    else FSIC_DST_FAST(64, false, 192);
#undef FSIC_DST_FAST
#undef FSIC_DST_XY
    return hipGetLastError();
}

}  // namespace

// z = M^{-1} r for the orbitals of the batch, with r.z partial sums.
template <typename T>
hipError_t launch_dst_precond(const DstItems &di, const OrbDesc *orb, const int *done,
                              const float *tab, const T *r, float *work, float *z, double *rz,
                              int *cnt, hipStream_t s) {
    return dst_apply<T, false>(di, orb, done, tab, r, work, z, rz,
                               PcgOut{nullptr, nullptr, nullptr, 1, nullptr, 0}, cnt, s);
}

// p = M^{-1} r + beta p_old for the orbitals of the batch, with r.z partial sums.
hipError_t launch_dst_pcg(const DstItems &di, const OrbDesc *orb, const int *done, const float *tab,
                          const float *r, float *work, float *p, double *rz, const PcgOut &po, int *cnt,
                          hipStream_t s) {
    return dst_apply<float, true>(di, orb, done, tab, r, work, p, rz, po, cnt, s);
}

// raise the dynamic-LDS limit of the fast transform kernels (once per batch,
// outside any stream capture)
hipError_t dst_setup(int np, int variant, int npxy, bool two) {
    // the limits are set once per (device, shape): a later batch of the same
    // shape finds them in place
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    const auto key = std::make_tuple(dev, np, variant, npxy, two);
    static std::mutex mu;
    static std::set<std::tuple<int, int, int, int, bool>> done;
    std::lock_guard<std::mutex> lk(mu);
    if (done.count(key)) return hipSuccess;
    if (npxy > 0) {
        const size_t lxy = dst_xy_lds(npxy, two);
        set_lds_limit(k_dst_xy<true, float, float, false>, lxy);
        set_lds_limit(k_dst_xy<true, double, double, false>, lxy);
        set_lds_limit(k_dst_xy<true, float, double, false>, lxy);
        set_lds_limit(k_dst_xy<false, float, float, false>, lxy);
        set_lds_limit(k_dst_xy<false, double, double, false>, lxy);
        set_lds_limit(k_dst_xy<false, float, double, false>, lxy);
        set_lds_limit(k_dst_xy<true, float, float, false, true, true>, lxy);
        set_lds_limit(k_dst_xy<true, float, float, false, true, false>, lxy);
        set_lds_limit(k_dst_xy<false, float, float, false, true>, lxy);
        if (dst_xy_occ2(npxy, two)) {
            set_lds_limit(k_dst_xy<true, float, float, true>, lxy);
            set_lds_limit(k_dst_xy<true, double, double, true>, lxy);
            set_lds_limit(k_dst_xy<true, float, double, true>, lxy);
            set_lds_limit(k_dst_xy<true, float, float, true, true>, lxy);
            set_lds_limit(k_dst_xy<true, float, float, true, true, true>, lxy);
        }
        if (dst_z_occ2(np)) {
            set_lds_limit(k_dst_fast<2, 1, float, float, true, 64, true, true>, dst_fast_lds(np, 64, true));
            set_lds_limit(k_dst_fast<2, 1, float, double, true, 64, true, true>, dst_fast_lds(np, 64, true));
        }
    }
#define FSIC_DST_LIMITS(PC_, SLO_, NPM_)                                                                  \
    do {                                                                                                  \
        const size_t lds = dst_fast_lds(np, PC_, SLO_), lz = dst_fast_lds(np, 64, SLO_);                  \
        set_lds_limit(k_dst_fast<0, 0, float, float, false, PC_, SLO_, false, false, NPM_>, lds);         \
        set_lds_limit(k_dst_fast<0, 0, double, double, false, PC_, SLO_, false, false, NPM_>, lds);       \
        set_lds_limit(k_dst_fast<1, 0, float, float, false, PC_, SLO_, false, false, NPM_>, lds);         \
        set_lds_limit(k_dst_fast<1, 0, float, double, false, PC_, SLO_, false, false, NPM_>, lds);        \
        set_lds_limit(k_dst_fast<2, 1, float, float, true, 64, SLO_, false, false, NPM_>, lz);            \
        set_lds_limit(k_dst_fast<2, 1, float, double, true, 64, SLO_, false, false, NPM_>, lz);           \
        set_lds_limit(k_dst_fast<0, 0, float, float, false, PC_, SLO_, false, true, NPM_>, lds);          \
        set_lds_limit(k_dst_fast<0, 0, float, double, false, PC_, SLO_, false, false, NPM_>, lds);        \
    } while (0)
    if (variant == 1) FSIC_DST_LIMITS(128, true, 128);
    else if (variant == 2) FSIC_DST_LIMITS(64, true, 160);
    else if (variant == 3) FSIC_DST_LIMITS(64, false, 192);
#undef FSIC_DST_LIMITS
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) done.insert(key);
    return e;
}

template hipError_t launch_dst_precond<float>(const DstItems &, const OrbDesc *, const int *,
                                              const float *, const float *, float *, float *,
                                              double *, int *, hipStream_t);
template hipError_t launch_dst_precond<double>(const DstItems &, const OrbDesc *, const int *,
                                               const float *, const double *, float *, float *,
                                               double *, int *, hipStream_t);

}  // namespace fsic
