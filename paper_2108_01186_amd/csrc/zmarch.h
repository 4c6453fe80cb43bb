// Star-stencil Laplacian driver and its policies for the per-orbital
// Poisson problems of the SIC path (Sec. II.A: high-order centred finite
// differences on a uniform grid; the Laplacian is the Kronecker sum of 1-D
// second differences applied matrix-free).
//
// Design (gfx950): one 256-thread block owns a 32 x 8*cpt column tile of an
// orbital's grid and marches through a z-chunk.  Each thread keeps the
// 2p + 1 z-neighbours of its cpt columns in registers; the current xy plane
// with its p-deep cross-shaped halo is staged in double-buffered LDS, and the
// next plane is fetched into registers while the current one is computed,
// so one barrier per plane separates the stages.  A policy supplies the
// operand (p for CG, x64 + x32 for the FP64 residual), one extra value per
// column node fetched with the plane (r for CG, b for the residual) and the
// epilogue.  Every CG iteration is two HBM passes: this sweep, whose halo
// carries the single operand array, and one pointwise update that also forms
// the next search direction.  Dot products accumulate in FP64 into per-block
// partial sums that later blocks add up in a fixed order, so results are
// bitwise reproducible.
#pragma once

#include <type_traits>

#include "kernels.h"

namespace fsic {

// ---------------------------------------------------------------------------
// z-marching stencil driver
// ---------------------------------------------------------------------------

// Raw buffer access: a uniform resource (base, size) plus a 32-bit vector
// byte offset and a 32-bit scalar byte offset, so no per-lane 64-bit address
// arithmetic is needed.  Every access here is in range by construction.
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc make_rsrc(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
template <class X> __device__ __forceinline__ X bld(Rsrc r, unsigned vidx, int sidx);
template <> __device__ __forceinline__ float bld<float>(Rsrc r, unsigned vidx, int sidx) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vidx * 4u, sidx * 4, 0));
}
template <> __device__ __forceinline__ double bld<double>(Rsrc r, unsigned vidx, int sidx) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vidx * 8u, sidx * 8, 0));
}
__device__ __forceinline__ void bst(Rsrc r, unsigned vidx, int sidx, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vidx * 4u, sidx * 4, 0);
}
__device__ __forceinline__ void bst(Rsrc r, unsigned vidx, int sidx, double v) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, vidx * 8u, sidx * 8, 0);
}

// calls f(integral_constant<int, U>, arg) for U = 0..N-1 (forced unrolling)
template <int N, int U = 0>
struct Unroller {
    template <class F, class A>
    __device__ __forceinline__ static void run(F &f, A arg) {
        if constexpr (U < N) {
            f(std::integral_constant<int, U>{}, arg);
            Unroller<N, U + 1>::run(f, arg);
        }
    }
};
template <int N, class F, class A>
__device__ __forceinline__ void unroll_steps(F &f, A arg) {
    Unroller<N>::run(f, arg);
}

template <typename T, int P, int CPT, int D, class Pol>
__global__ __launch_bounds__(256) void k_zmarch(Pol pol, Coeffs cf) {
    using Raw = typename Pol::Raw;  // operand load (columns and halo)
    using Ext = typename Pol::Ext;  // per-column value at the current plane
    using Acc = typename Pol::Acc;  // epilogue accumulators
    constexpr int TY = 8 * CPT;              // tile rows (each thread owns CPT columns)
    // LDS row stride 64 elements (>= kTX + 2P): the +-k-row neighbours are
    // then multiples of 64 elements apart and fit the ds_read2st64 offsets
    constexpr int W = 64;
    constexpr int H = TY + 2 * P;            // LDS rows
    constexpr int NH = 2 * P * (kTX + TY);   // cross-shaped halo values per plane
    constexpr int HS = (NH + 255) / 256;     // halo slots per thread
    constexpr int NW = 2 * P + 1;            // z window
    __shared__ T sm[2][H * W + 1];           // double-buffered plane (+1 dump slot)
    __shared__ double sred[4];
    const Item it = pol.items[blockIdx.x];
    if (it.orb < 0) return;
    const OrbDesc od = pol.orb[it.orb];
    Pol p = pol;
    p.tile0 = (it.tile == 0);
    if (!p.setup(it.orb, od, sred)) return;  // uniform across the block
    p.init(od);

    const int nx = od.nx, ny = od.ny, nz = od.nz;
    const int plane = nx * ny;
    const int bx = it.tile % od.tiles_x;
    const int by = (it.tile / od.tiles_x) % od.tiles_y;
    const int bz = it.tile / (od.tiles_x * od.tiles_y);
    const int tx = threadIdx.x & (kTX - 1);
    const int ty = threadIdx.x >> 5;  // 0..7
    const int x = bx * kTX + tx;
    const int z0 = bz * od.zc;
    const int z1 = min(nz, z0 + od.zc);
    const int len = z1 - z0;
    // odd z-chunks march downwards: the two chunks beside a chunk boundary
    // then reach it at the same time (both at their start or both at their
    // end), so the halo planes one of them fetches are still in L2 for the
    // other (their blocks are adjacent in the item table, on one XCD)
    const bool down = (bz & 1) != 0;
    auto zat = [&](int s) -> int { return down ? z1 - 1 - s : z0 + s; };  // plane at march step s

    T c[P + 1];
#pragma unroll
    for (int k = 0; k <= P; ++k) c[k] = (T)cf.c[k];
    const T c0x3 = T(3) * c[0];
    const T ih2 = (T)od.inv_h2;

    // z-invariant 32-bit in-plane offsets; addresses are a uniform plane base
    // plus these.  Invalid positions read a clamped in-grid node and are
    // zeroed by select, so no load is predicated.
    unsigned coff[CPT];
    bool cval[CPT];
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
        const int y = by * TY + ty + 8 * cc;
        cval[cc] = (x < nx) && (y < ny);
        coff[cc] = (unsigned)(min(y, ny - 1) * nx + min(x, nx - 1));
    }
    unsigned hoff[HS];
    int hlds[HS];
    bool hval[HS];
#pragma unroll
    for (int sl = 0; sl < HS; ++sl) {
        const int hh = threadIdx.x + 256 * sl;
        int hx = 0, hy = 0;
        if (hh < 2 * P * TY) {
            const int side = hh / (P * TY);
            const int rem = hh - side * P * TY;
            hy = rem / P;
            hx = rem - hy * P;
            hx = side ? kTX + hx : hx - P;
        } else {
            const int h2 = hh - 2 * P * TY;
            const int side = h2 / (P * kTX);
            const int rem = h2 - side * P * kTX;
            const int yy = rem / kTX;
            hx = rem - yy * kTX;
            hy = side ? TY + yy : yy - P;
        }
        const int gx = bx * kTX + hx, gy = by * TY + hy;
        hlds[sl] = (hh < NH) ? (hy + P) * W + (hx + P) : H * W;  // spare threads write the dump slot
        hval[sl] = (hh < NH) && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        hoff[sl] = (unsigned)(min(max(gy, 0), ny - 1) * nx + min(max(gx, 0), nx - 1));
    }
    auto zoff = [&](int z) -> int {  // uniform element offset of plane z (clamped)
        return min(max(z, 0), nz - 1) * plane;
    };
    auto use = [&](const Raw &r, bool valid) -> T { return valid ? p.combine(r) : T(0); };

    // z window of each column in registers, rotated by unrolling (no moves):
    // the plane of march step s - P + j lives in slot (s + j) % NW (the
    // stencil is symmetric in z, so the direction does not matter)
    T q[CPT][NW];
#pragma unroll
    for (int j = 0; j < 2 * P; ++j) {
        const int z = zat(j - P);
        const int pz = zoff(z);
        const bool zin = z >= 0 && z < nz;
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) q[cc][j] = use(p.raw(coff[cc], pz), cval[cc] && zin);
    }
    // prefetch ring: stage d holds the raw loads of march step d (+ P for the
    // columns' operand)
    Raw sc[D][CPT], sh[D][HS];
    Ext se[D][CPT];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int pc = zoff(zat(d + P)), ph = zoff(zat(d));
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            sc[d][cc] = p.raw(coff[cc], pc);
            se[d][cc] = p.ext(coff[cc], ph);
        }
#pragma unroll
        for (int sl = 0; sl < HS; ++sl) sh[d][sl] = p.raw(hoff[sl], ph);
    }

    Acc acc{};
    // one z step; U is the compile-time position in the unrolled block of NW*D
    auto step = [&](auto uc, int sb) {
        constexpr int u = decltype(uc)::value;
        constexpr int d = u % D;
        constexpr int sl0 = u % NW;  // slot of march step s - P
        const int s = sb + u;
        if (s >= len) return;
        const int z = zat(s);
        // buffer parity follows the step index (NW*D is odd, so u & 1 would
        // reuse a buffer across the boundary of two unrolled blocks)
        T *S = sm[s & 1];
        const int zt = zat(s + P);
        const bool ztop = zt >= 0 && zt < nz;
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            q[cc][(sl0 + 2 * P) % NW] = use(sc[d][cc], cval[cc] && ztop);
            S[(ty + 8 * cc + P) * W + tx + P] = q[cc][(sl0 + P) % NW];
        }
#pragma unroll
        for (int sl = 0; sl < HS; ++sl) S[hlds[sl]] = use(sh[d][sl], hval[sl]);
        lds_barrier();
        Ext ecur[CPT];
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) ecur[cc] = se[d][cc];
        if (s + D < len) {  // refill this stage with march step s + D
            const int pc = zoff(zat(s + D + P)), ph = zoff(zat(s + D));
#pragma unroll
            for (int cc = 0; cc < CPT; ++cc) {
                sc[d][cc] = p.raw(coff[cc], pc);
                se[d][cc] = p.ext(coff[cc], ph);
            }
#pragma unroll
            for (int sl = 0; sl < HS; ++sl) sh[d][sl] = p.raw(hoff[sl], ph);
        }
        const int pz = z * plane;
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            // xb: this row from x - P; yb: this column from row - P (stride W)
            const T *xb = S + (ty + 8 * cc + P) * W + tx;
            const T *yb = S + (ty + 8 * cc) * W + tx + P;
            T lap = c0x3 * q[cc][(sl0 + P) % NW];
#pragma unroll
            for (int k = 1; k <= P; ++k)
                lap += c[k] * ((xb[P + k] + xb[P - k]) + (yb[(P + k) * W] + yb[(P - k) * W]) +
                               (q[cc][(sl0 + P + k) % NW] + q[cc][(sl0 + P - k) % NW]));
            lap *= ih2;
            if (cval[cc]) p.epilogue(coff[cc], pz, q[cc][(sl0 + P) % NW], lap, ecur[cc], acc);
        }
    };
    for (int sb = 0; sb < len; sb += NW * D) unroll_steps<NW * D>(step, sb);
    p.finish(it, od, acc, sred);  // every thread (block reductions)
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
    struct Raw { T a; };
    struct Ext {};
    struct Acc {};
    bool tile0;
    Rsrc ru, ro;
    __device__ bool setup(int, const OrbDesc &, double *) { return true; }
    __device__ void init(const OrbDesc &od) {
        const unsigned bytes = (unsigned)((long long)od.nx * od.ny * od.nz * sizeof(T));
        ru = make_rsrc(u + od.off, bytes);
        ro = make_rsrc(out + od.off, bytes);
    }
    __device__ Raw raw(unsigned i, int zo) const { return Raw{bld<T>(ru, i, zo)}; }
    __device__ Ext ext(unsigned, int) const { return Ext{}; }
    __device__ T combine(const Raw &r) const { return r.a; }
    __device__ void epilogue(unsigned i, int zo, T, T lap, const Ext &, Acc &) const {
        bst(ro, i, zo, lap);
    }
    __device__ void finish(const Item &, const OrbDesc &, const Acc &, double *) const {}
};

template <typename T>
struct PolHam {  // out = -1/2 L psi + v psi (v: one field shared by the orbitals)
    const Item *items;
    const OrbDesc *orb;
    const T *psi;
    const T *v;
    T *out;
    struct Raw { T a; };
    typedef T Ext;
    struct Acc {};
    bool tile0;
    Rsrc ru, rv, ro;
    __device__ bool setup(int, const OrbDesc &, double *) { return true; }
    __device__ void init(const OrbDesc &od) {
        const unsigned bytes = (unsigned)((long long)od.nx * od.ny * od.nz * sizeof(T));
        ru = make_rsrc(psi + od.off, bytes);
        rv = make_rsrc(v, bytes);
        ro = make_rsrc(out + od.off, bytes);
    }
    __device__ Raw raw(unsigned i, int zo) const { return Raw{bld<T>(ru, i, zo)}; }
    __device__ Ext ext(unsigned i, int zo) const { return bld<T>(rv, i, zo); }
    __device__ T combine(const Raw &r) const { return r.a; }
    __device__ void epilogue(unsigned i, int zo, T c, T lap, const Ext &vv, Acc &) const {
        bst(ro, i, zo, T(-0.5) * lap + vv * c);
    }
    __device__ void finish(const Item &, const OrbDesc &, const Acc &, double *) const {}
};

// r_j.r_j of an orbital: the CG recursion's partial sums (by iteration
// parity) or those of the last FP64 residual, added in a fixed order
template <typename T>
__device__ __forceinline__ double rr_of(const CGIter<T> &a, const OrbDesc &od, int j, int from_ru,
                                        double *sbuf) {
    if (from_ru) return sum_partials(a.partRU + od.base7, od.nt7, sbuf);
    return sum_partials(a.part8 + (size_t)(j & 1) * a.tot8 + od.base8, od.nt8, sbuf);
}

template <typename T>
struct PolCG {  // q = K p_k = -L p_k; partial sums of p.q, r.q, q.q
    const Item *items;
    const OrbDesc *orb;
    CGIter<T> a;
    int k, cur_ru, check;
    bool p_from_r;  // the recursion (re)starts here: p_k = r_k
    bool tile0;
    __device__ bool setup(int o, const OrbDesc &od, double *sbuf) {
        // other blocks of this orbital may change done[o] during this launch:
        // read it once and broadcast so the whole block takes one branch
        if (threadIdx.x == 0) sbuf[0] = (double)a.done[o];
        __syncthreads();
        const bool dn = sbuf[0] != 0.0;
        __syncthreads();
        if (dn) return false;
        // restart (beta = 0) from the FP64 residual after an unconfirmed pause
        const bool restart = a.rs_iter && a.rs_iter[o] == k;
        const double rr = rr_of(a, od, k, cur_ru || restart, sbuf);
        if (check && rr <= a.tol2 * a.bb[o]) {
            if (threadIdx.x == 0) {
                if (a.rs_iter) {
                    a.done[o] = 2;  // mixed: confirm on the FP64 residual first
                } else {
                    a.done[o] = 1;
                    a.iters[o] = k;
                    a.rrfin[o] = rr;
                }
            }
            return false;
        }
        p_from_r = (k == 0) || restart;
        if (threadIdx.x == 0 && tile0) {  // one count per orbital and launch
            a.nact[o] += 1;
            if (a.nsamp) a.nsamp[o] += 1;
        }
        return true;
    }
    struct Raw { T p; };
    typedef T Ext;
    struct Acc { double pq, rq, qq; };
    Rsrc rr_, rp, rq;
    __device__ void init(const OrbDesc &od) {
        const unsigned bytes = (unsigned)((long long)od.nx * od.ny * od.nz * sizeof(T));
        rr_ = make_rsrc(a.R + od.off, bytes);
        rp = make_rsrc((p_from_r ? a.R : a.P) + od.off, bytes);
        rq = make_rsrc(a.Q + od.off, bytes);
    }
    __device__ Raw raw(unsigned i, int zo) const { return Raw{bld<T>(rp, i, zo)}; }
    __device__ Ext ext(unsigned i, int zo) const { return bld<T>(rr_, i, zo); }
    __device__ T combine(const Raw &v) const { return v.p; }
    __device__ void epilogue(unsigned i, int zo, T pv, T lap, const Ext &rv, Acc &s) const {
        const T qv = -lap;
        bst(rq, i, zo, qv);
        const double qd = (double)qv;
        s.pq += (double)pv * qd;
        s.rq += (double)rv * qd;
        s.qq += qd * qd;
    }
    __device__ void finish(const Item &it, const OrbDesc &od, const Acc &s, double *sred) const {
        const double pq = block_sum256(s.pq, sred);
        const double rq = block_sum256(s.rq, sred);
        const double qq = block_sum256(s.qq, sred);
        if (threadIdx.x == 0) {
            const size_t j = (size_t)od.base7 + it.tile;
            a.part7[j] = pq;
            a.part7[(size_t)a.tot7 + j] = rq;
            a.part7[2 * (size_t)a.tot7 + j] = qq;
        }
    }
};

// r_j.z_j of an orbital (preconditioned CG), by iteration parity
template <typename T>
__device__ __forceinline__ double rz_of(const CGIter<T> &a, const OrbDesc &od, int j, double *sbuf) {
    return sum_partials(a.partRZ + (size_t)(j & 1) * a.tot9 + od.base9, od.nt9, sbuf);
}

template <typename T>
struct PolPCG {  // p_k = z_k + beta p_{k-1}; q = K p_k = -L p_k; p.q partials
    const Item *items;
    const OrbDesc *orb;
    CGIter<T> a;
    int k, cur_ru, restart, pause;
    double beta;
    bool tile0;
    __device__ bool setup(int o, const OrbDesc &od, double *sbuf) {
        if (threadIdx.x == 0) sbuf[0] = (double)a.done[o];
        __syncthreads();
        const bool dn = sbuf[0] != 0.0;
        __syncthreads();
        if (dn) return false;
        const double rr = rr_of(a, od, k, cur_ru, sbuf);
        if (rr <= a.tol2 * a.bb[o]) {
            if (threadIdx.x == 0) {
                if (pause) {
                    a.done[o] = 2;  // mixed: confirm on the FP64 residual first
                } else if (atomicCAS(a.done + o, 0, 1) == 0) {  // first block of o to see it
                    a.iters[o] = k;
                    a.rrfin[o] = rr;
                    if (a.ndone) atomicAdd(a.ndone, 1);
                }
            }
            return false;
        }
        if (k == 0 || restart) {
            beta = 0.0;
        } else {
            beta = rz_of(a, od, k, sbuf) / rz_of(a, od, k - 1, sbuf);
        }
        if (threadIdx.x == 0 && tile0) {
            a.nact[o] += 1;
            if (a.nsamp) a.nsamp[o] += 1;
        }
        return true;
    }
    struct Raw { float z; T p; };
    struct Ext {};
    typedef double Acc;
    Rsrc rz_, rpo, rpn, rq;
    __device__ void init(const OrbDesc &od) {
        const long long M = (long long)od.nx * od.ny * od.nz;
        rz_ = make_rsrc(a.Z + od.off, (unsigned)(M * 4));
        rpo = make_rsrc(a.Pold + od.off, (unsigned)(M * sizeof(T)));
        rpn = make_rsrc(a.P + od.off, (unsigned)(M * sizeof(T)));
        rq = make_rsrc(a.Q + od.off, (unsigned)(M * sizeof(T)));
    }
    __device__ Raw raw(unsigned i, int zo) const {
        // beta = 0 at a (re)start and the host points p_old at finite data
        return Raw{bld<float>(rz_, i, zo), bld<T>(rpo, i, zo)};
    }
    __device__ Ext ext(unsigned, int) const { return Ext{}; }
    __device__ T combine(const Raw &v) const { return (T)v.z + (T)beta * v.p; }
    __device__ void epilogue(unsigned i, int zo, T c, T lap, const Ext &, Acc &s) const {
        const T qv = -lap;
        bst(rpn, i, zo, c);
        bst(rq, i, zo, qv);
        s += (double)c * (double)qv;
    }
    __device__ void finish(const Item &it, const OrbDesc &od, const Acc &s, double *sred) const {
        const double t = block_sum256(s, sred);
        if (threadIdx.x == 0) a.part7[od.base7 + it.tile] = t;
    }
};

// sweep of the mixed restart cycles: q_k = -L p_k, p_k.q_k partials by parity
struct PolPQ {
    const Item *items;
    const OrbDesc *orb;
    CGIter<float> a;
    int k;
    const int *pz;  // paused orbitals (pz[o] <= li) are skipped
    int li;
    bool tile0;
    __device__ bool setup(int o, const OrbDesc &, double *sbuf) {
        if (threadIdx.x == 0) sbuf[0] = (double)(a.done[o] || (pz && pz[o] <= li));
        __syncthreads();
        const bool dn = sbuf[0] != 0.0;
        __syncthreads();
        if (dn) return false;
        if (threadIdx.x == 0 && tile0) {
            a.nact[o] += 1;
            if (a.nsamp) a.nsamp[o] += 1;
        }
        return true;
    }
    struct Raw { float p; };
    struct Ext {};
    typedef double Acc;
    Rsrc rp, rq;
    __device__ void init(const OrbDesc &od) {
        const unsigned bytes = (unsigned)((long long)od.nx * od.ny * od.nz * 4);
        rp = make_rsrc(a.P + od.off, bytes);
        rq = make_rsrc(a.Q + od.off, bytes);
    }
    __device__ Raw raw(unsigned i, int zo) const { return Raw{bld<float>(rp, i, zo)}; }
    __device__ Ext ext(unsigned, int) const { return Ext{}; }
    __device__ float combine(const Raw &v) const { return v.p; }
    __device__ void epilogue(unsigned i, int zo, float c, float lap, const Ext &, Acc &s) const {
        const float qv = -lap;
        bst(rq, i, zo, qv);
        s += (double)c * (double)qv;
    }
    __device__ void finish(const Item &it, const OrbDesc &od, const Acc &s, double *sred) const {
        const double t = block_sum256(s, sred);
        if (threadIdx.x == 0) a.part7[(size_t)(k & 1) * a.tot7 + od.base7 + it.tile] = t;
    }
};

// alpha_j = r_j.z_j / p_j.q_j of an orbital (mixed restart cycles)
__device__ __forceinline__ double alpha_of(const CGIter<float> &a, const OrbDesc &od, int j, double *sbuf) {
    const double rz = rz_of(a, od, j, sbuf);
    const double pq = sum_partials(a.part7 + (size_t)(j & 1) * a.tot7 + od.base7, od.nt7, sbuf);
    return pq != 0.0 ? rz / pq : 0.0;  // p = 0 only for a zero right-hand side
}

// end of a mixed restart cycle: res = b + L x, x = x64 + x32 + alpha_a p_a + alpha_b p_b
// HAS32: x32 present (cycles of more than two iterations); HAS64: x64
// present (every cycle but the first, which starts from x = 0)
template <bool HAS32, bool HAS64 = true>
struct PolResP {
    const Item *items;
    const OrbDesc *orb;
    CGIter<float> a;
    ResStep r;
    bool tile0;
    double aa, ab;
    struct Raw { double x; float x32, pa, pb; };
    typedef double Ext;
    typedef double Acc;
    Rsrc rx, rx32, rpa, rpb, rb, rxn, rr32;
    __device__ bool setup(int o, const OrbDesc &od, double *sbuf) {
        if (a.done[o] == 1) return false;  // not changed during this launch: uniform
        // steps of iterations at or after the pause of o did not run
        const int p = r.pz ? r.pz[o] : (1 << 30);
        aa = r.la < p ? alpha_of(a, od, r.ka, sbuf) : 0.0;
        ab = r.lb < p ? alpha_of(a, od, r.kb, sbuf) : 0.0;
        if (threadIdx.x == 0 && tile0 && a.nsamp) a.nsamp[3 * a.norb + o] += 1;
        return true;
    }
    __device__ void init(const OrbDesc &od) {
        const long long M = (long long)od.nx * od.ny * od.nz;
        if (HAS64) rx = make_rsrc(r.X64 + od.off, (unsigned)(M * 8));
        if (HAS32) rx32 = make_rsrc(r.X32 + od.off, (unsigned)(M * 4));
        rpa = make_rsrc(r.Pa + od.off, (unsigned)(M * 4));
        rpb = make_rsrc(r.Pb + od.off, (unsigned)(M * 4));
        rb = make_rsrc(a.B64 + od.off, (unsigned)(M * 8));
        rxn = make_rsrc(r.X64new + od.off, (unsigned)(M * 8));
        rr32 = make_rsrc(r.R32 + od.off, (unsigned)(M * 4));
    }
    __device__ Raw raw(unsigned i, int zo) const {
        return Raw{HAS64 ? bld<double>(rx, i, zo) : 0.0, HAS32 ? bld<float>(rx32, i, zo) : 0.0f,
                   bld<float>(rpa, i, zo), bld<float>(rpb, i, zo)};
    }
    __device__ Ext ext(unsigned i, int zo) const { return bld<double>(rb, i, zo); }
    __device__ double combine(const Raw &v) const {
        return v.x + ((double)v.x32 + (aa * (double)v.pa + ab * (double)v.pb));
    }
    __device__ void epilogue(unsigned i, int zo, double c, double lap, const Ext &b, Acc &s) const {
        const double res = b + lap;
        bst(rxn, i, zo, c);
        bst(rr32, i, zo, (float)res);
        s += res * res;
    }
    __device__ void finish(const Item &it, const OrbDesc &od, const Acc &s, double *sred) const {
        const double t = block_sum256(s, sred);
        if (threadIdx.x == 0) a.partRU[od.base7 + it.tile] = t;
    }
};

template <bool HAS32>
struct PolRes {  // res = b + L x, x = x64 (+ x32); X64 null (with x32): x64 = 0
    const Item *items;
    const OrbDesc *orb;
    const int *done;
    const double *X64;
    const float *X32;
    const double *B;
    double *X64new;
    float *R32;
    double *partRU;
    struct Raw { double a; float b; };
    typedef double Ext;
    typedef double Acc;
    bool tile0;
    Rsrc rx, rx32, rb, rxn, rr32;
    __device__ bool setup(int o, const OrbDesc &, double *) { return done == nullptr || done[o] != 1; }
    __device__ void init(const OrbDesc &od) {
        const long long M = (long long)od.nx * od.ny * od.nz;
        if (X64) rx = make_rsrc(X64 + od.off, (unsigned)(M * 8));
        rb = make_rsrc(B + od.off, (unsigned)(M * 8));
        if constexpr (HAS32) rx32 = make_rsrc(X32 + od.off, (unsigned)(M * 4));
        if (X64new) rxn = make_rsrc(X64new + od.off, (unsigned)(M * 8));
        if (R32) rr32 = make_rsrc(R32 + od.off, (unsigned)(M * 4));
    }
    __device__ Raw raw(unsigned i, int zo) const {
        if constexpr (HAS32) return Raw{X64 ? bld<double>(rx, i, zo) : 0.0, bld<float>(rx32, i, zo)};
        return Raw{bld<double>(rx, i, zo), 0.0f};
    }
    __device__ Ext ext(unsigned i, int zo) const { return bld<double>(rb, i, zo); }
    __device__ double combine(const Raw &v) const { return v.a + (double)v.b; }
    __device__ void epilogue(unsigned i, int zo, double c, double lap, const Ext &b, Acc &s) const {
        const double res = b + lap;
        if (X64new) bst(rxn, i, zo, c);
        if (R32) bst(rr32, i, zo, (float)res);
        s += res * res;
    }
    __device__ void finish(const Item &it, const OrbDesc &od, const Acc &s, double *sred) const {
        const double t = block_sum256(s, sred);
        if (threadIdx.x == 0) partRU[od.base7 + it.tile] = t;
    }
};

// ---------------------------------------------------------------------------
// pointwise CG update
// ---------------------------------------------------------------------------

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 V; static constexpr int n = 4; };
template <> struct Vec16<double> { typedef double2 V; static constexpr int n = 2; };

#define FSIC_RADIUS_SWITCH(radius, CALL)                           \
    switch (radius * 64 + c.cpt * 8 + c.depth) {                   \
        case 1 * 64 + 2 * 8 + 2: CALL(1, 2, 2); break;             \
        case 2 * 64 + 2 * 8 + 2: CALL(2, 2, 2); break;             \
        case 3 * 64 + 2 * 8 + 2: CALL(3, 2, 2); break;             \
        case 4 * 64 + 2 * 8 + 2: CALL(4, 2, 2); break;             \
        case 5 * 64 + 2 * 8 + 2: CALL(5, 2, 2); break;             \
        case 6 * 64 + 2 * 8 + 2: CALL(6, 2, 2); break;             \
        case 6 * 64 + 1 * 8 + 2: CALL(6, 1, 2); break;             \
        case 6 * 64 + 4 * 8 + 1: CALL(6, 4, 1); break;             \
        case 6 * 64 + 1 * 8 + 1: CALL(6, 1, 1); break;             \
        case 6 * 64 + 2 * 8 + 1: CALL(6, 2, 1); break;             \
        default: return hipErrorInvalidValue;                      \
    }


}  // namespace fsic
