// Dirichlet boundary values of the Hartree problem for isolated systems from
// a multipole expansion of each FLO density about the box centre (Sec. II.A),
// the right-hand side -L v = 4 pi rho + (boundary term), and the transpose of
// that boundary map for the adjoint (FOD-gradient) solves.
//
// Real solid harmonics r^l Y_lm are built without trigonometry: the
// azimuthal factor is (x + i y)^m and the polar factor r^(l-m) d^m P_l/dx^m
// (z / r) obeys the three-term recurrence in l, so one node costs a few
// hundred flops and no transcendental calls.
#include <array>
#include <map>
#include <mutex>
#include <type_traits>

#include "kernels.h"

namespace fsic {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// right-hand side b = scale * rho + (L g)|interior
// ---------------------------------------------------------------------------

// Boundary term of the interior nodes within reach of each face, computed in
// place of the ghost values: a face column's layer e (0-based; the interior
// node at distance e from the face) becomes
//   t_e = sum_{d = 1}^{P - e} c_(e+d) g_d / h^2,
// the taps of that node into the column's ghost layers d = 1..P.  One thread
// per face column; grid.y: orbital.
__global__ __launch_bounds__(256) void k_bterm(int P, Coeffs cf, const OrbDesc *orb, double *G) {
    const OrbDesc od = orb[blockIdx.y];
    const long long F[3] = {(long long)od.ny * od.nz, (long long)od.nx * od.nz, (long long)od.nx * od.ny};
    long long col = (long long)blockIdx.x * 256 + threadIdx.x;
    long long base = od.goff;
    int face = 0;
    for (; face < 6; ++face) {
        const long long Fa = F[face >> 1];
        if (col < Fa) break;
        col -= Fa;
        base += P * Fa;
    }
    if (face == 6) return;
    const long long Fa = F[face >> 1];
    double *gc = G + base + col;
    double g[kMaxRadius];
#pragma unroll
    for (int d = 0; d < kMaxRadius; ++d) g[d] = d < P ? gc[d * Fa] : 0.0;
#pragma unroll
    for (int e = 0; e < kMaxRadius; ++e) {
        if (e < P) {
            double t = 0.0;
#pragma unroll
            for (int d = 1; d <= kMaxRadius; ++d)
                if (d <= P - e) t += cf.c[e + d] * g[d - 1];
            gc[e * Fa] = t * od.inv_h2;
        }
    }
}

constexpr int kRhsU = 4;  // nodes per thread whose loads are issued together

__global__ __launch_bounds__(256) void k_rhs(int P, Coeffs cf, const OrbDesc *orb,
                                             const Item *items, const double *__restrict__ src, int square,
                                             double scale, const double *__restrict__ G,
                                             double *__restrict__ B, double *__restrict__ R64,
                                             float *__restrict__ R32, double *__restrict__ X64zero,
                                             double *part8) {
    __shared__ double sred[4];
    const Item it = items[blockIdx.x];
    if (it.orb < 0) return;
    const OrbDesc od = orb[it.orb];
    const int nx = od.nx, ny = od.ny, nz = od.nz;
    const long long M = (long long)nx * ny * nz;
    const long long Fx = (long long)ny * nz, Fy = (long long)nx * nz, Fz = (long long)nx * ny;
    const long long oxm = 0, oxp = P * Fx, oym = 2 * P * Fx, oyp = oym + P * Fy,
                    ozm = oym + 2 * P * Fy, ozp = ozm + P * Fz;
    const long long base = (long long)it.tile * kPW;
    const double *g = G ? G + od.goff : nullptr;
    // node indices of the thread's first node (32 bits: at most 2^29 nodes
    // per orbital), then advanced by 256 nodes per step without dividing
    const int pxy = nx * ny;
    const int i0 = (int)base + threadIdx.x;
    int iz = i0 / pxy;
    int iy = (i0 - iz * pxy) / nx;
    int ix = i0 - iz * pxy - iy * nx;
    const int sx = 256 % nx, sy = (256 / nx) % ny, sz = 256 / pxy;
    double acc = 0.0;
    for (int e0 = 0; e0 < kPW / 256; e0 += kRhsU) {
        double sv[kRhsU];
#pragma unroll
        for (int u = 0; u < kRhsU; ++u) {
            const long long i = base + (e0 + u) * 256 + threadIdx.x;
            sv[u] = (src && i < M) ? src[od.off + i] : 0.0;  // no source: boundary values only
        }
#pragma unroll
        for (int u = 0; u < kRhsU; ++u) {
            const long long i = base + (e0 + u) * 256 + threadIdx.x;
            if (i < M) {
                double b = scale * (square ? sv[u] * sv[u] : sv[u]);
                if (g) {
                    // boundary term (k_bterm): layer e of the column of each face
                    // within reach, faces in the order x-, x+, y-, y+, z-, z+
                    const long long fx = iy + (long long)ny * iz, fy = ix + (long long)nx * iz,
                                    fz = ix + (long long)nx * iy;
                    double bt = 0.0;
                    if (ix < P) bt += g[oxm + ix * Fx + fx];
                    if (nx - 1 - ix < P) bt += g[oxp + (nx - 1 - ix) * Fx + fx];
                    if (iy < P) bt += g[oym + iy * Fy + fy];
                    if (ny - 1 - iy < P) bt += g[oyp + (ny - 1 - iy) * Fy + fy];
                    if (iz < P) bt += g[ozm + iz * Fz + fz];
                    if (nz - 1 - iz < P) bt += g[ozp + (nz - 1 - iz) * Fz + fz];
                    b += bt;
                }
                const long long gi = od.off + i;
                if (B) B[gi] = b;
                if (R64) R64[gi] = b;
                if (R32) R32[gi] = (float)b;
                if (X64zero) X64zero[gi] = 0.0;
                acc += b * b;
            }
            // next node of this thread: + 256 (sy < ny, so one carry at most per axis)
            ix += sx;
            const int cy = ix >= nx;
            ix -= cy ? nx : 0;
            iy += sy + cy;
            const int cz = iy >= ny;
            iy -= cz ? ny : 0;
            iz += sz + cz;
        }
    }
    const double s = block_sum256(acc, sred);
    if (threadIdx.x == 0) part8[od.base8 + it.tile] = s;
}

// ---------------------------------------------------------------------------
// harmonic contractions on the matrix cores: out[o][q] = scale sum_n
// H_q(n) f_o(n) over the nodes n of one channel's grid, with H built once per
// node for all orbitals of the channel
//   MODE 0 (moments): n = grid nodes, H_q = r^l Y_lm, f_o = rho_o (src^2 if
//          square), scale dV;
//   MODE 1 (adjoint boundary): n = ghost nodes, H_q = gfac_q Y_lm / r^(l+1),
//          f_o = (C^T w_o)(n) = sum_t c_(t+d) w_o(t) / h^2 over the interior
//          taps along the face normal, scale 1.
// A block takes a contiguous range of 64-node chunks.  Per chunk the four
// waves build H in LDS (wave w the azimuthal orders m = w mod 4), then per
// tile of 16 orbitals they stage f in LDS and each wave multiplies its
// 16-row H tiles against it (v_mfma_f64_16x16x4f64).  The loads of the next
// tile's f are issued before the products of the current one.  Each block
// writes one partial tile; a second kernel adds a channel's tiles in item
// order.
// ---------------------------------------------------------------------------

constexpr int kHc = 64;  // nodes per chunk

// f(q, l, r^l Y_lm / norm_lm) for the one azimuthal order MM (m = +MM and
// -MM): the recurrence of visit_regular_harmonics without the normalisation,
// which the contractions apply to their (much smaller) other operand or
// result; no table is read while the harmonics are built
template <int L, int MM, class F>
__device__ __forceinline__ void visit_harmonics_m(double x, double y, double z, F &&f) {
    if constexpr (MM <= L) {
        const double r2 = x * x + y * y + z * z;
        double cm = 1.0, sm = 0.0, dfact = 1.0;
#pragma unroll
        for (int m = 1; m <= MM; ++m) {
            const double c2 = cm * x - sm * y;
            sm = cm * y + sm * x;
            cm = c2;
            dfact *= (double)(2 * m - 1);
        }
        double pm2 = 0.0, pm1 = 0.0;
#pragma unroll
        for (int l = MM; l <= L; ++l) {
            double pl;
            if (l == MM)
                pl = dfact;
            else if (l == MM + 1)
                pl = (double)(2 * MM + 1) * z * pm1;
            else
                pl = ((double)(2 * l - 1) * z * pm1 - (double)(l + MM - 1) * r2 * pm2) * (1.0 / (double)(l - MM));
            pm2 = pm1;
            pm1 = pl;
            if (MM == 0) {
                f(l * l + l, l, pl);
            } else {
                f(l * l + l + MM, l, cm * pl);
                f(l * l + l - MM, l, sm * pl);
            }
        }
    }
}

// the orders m = W, W + 4, W + 8 (kMaxL = 8)
template <int L, int W, class F>
__device__ __forceinline__ void visit_harmonics_set(double x, double y, double z, F &&f) {
    visit_harmonics_m<L, W>(x, y, z, f);
    visit_harmonics_m<L, W + 4>(x, y, z, f);
    visit_harmonics_m<L, W + 8>(x, y, z, f);
}

// column `lane` of the chunk's harmonic rows (unnormalised), wave w the
// orders m = w mod 4; KIND 0: r^l P_lm, KIND 1: the same / r^(2l+1)
template <int L, int KIND>
__device__ __forceinline__ void hc_build(double x, double y, double z, bool valid, int w, int lane,
                                         double (*Hs)[65]) {
    double pw[L + 1];
    if constexpr (KIND == 1) {
        const double ir2 = 1.0 / (x * x + y * y + z * z);
        pw[0] = sqrt(ir2);
#pragma unroll
        for (int l = 1; l <= L; ++l) pw[l] = pw[l - 1] * ir2;
    }
    auto put = [&](int q, int l, double h) {
        if constexpr (KIND == 1) h *= pw[l];
        Hs[q][lane] = valid ? h : 0.0;
    };
    switch (w) {
        case 0: visit_harmonics_set<L, 0>(x, y, z, put); break;
        case 1: visit_harmonics_set<L, 1>(x, y, z, put); break;
        case 2: visit_harmonics_set<L, 2>(x, y, z, put); break;
        default: visit_harmonics_set<L, 3>(x, y, z, put); break;
    }
}

// one node of a chunk: position relative to the centre; MODE 1: the interior
// node next to the face (base), the step inward along the normal, the depth d
struct HcNode {
    double x, y, z;
    int base, st, d;
    bool valid;
};

template <int MODE>
__device__ __forceinline__ HcNode hc_decode(const OrbDesc &od, int P, long long nn, long long n) {
    HcNode nd{1.0, 1.0, 1.0, 0, 0, 0, n < nn};
    if (!nd.valid) return nd;
    int gi, gj, gk;
    if constexpr (MODE == 0) {
        // node indices in 32 bits (at most 2^29 nodes per orbital)
        const int ii = (int)n, pxy = od.nx * od.ny;
        gk = ii / pxy;
        const int rem = ii - gk * pxy;
        gj = rem / od.nx;
        gi = rem - gj * od.nx;
        nd.base = ii;
    } else {
        // ghost index in 32 bits: a slab holds at most P * 4096^2 nodes and
        // all of an orbital's ghosts fewer than 2^31
        const int F[3] = {od.ny * od.nz, od.nx * od.nz, od.nx * od.ny};
        int rem = (int)n, face = 0;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            const int sz = P * F[f >> 1];
            if (face == f && rem >= sz) {
                rem -= sz;
                face = f + 1;
            }
        }
        const int ax = face >> 1, side = face & 1;
        const int Fa = ax == 0 ? F[0] : (ax == 1 ? F[1] : F[2]);
        const int d = rem / Fa + 1, f2 = rem - (d - 1) * Fa;
        const int nu = ax == 0 ? od.ny : od.nx;  // fastest in-face axis
        const int a = f2 % nu, b2 = f2 / nu;
        const int pxy = od.nx * od.ny;
        if (ax == 0) {
            gi = side ? od.nx - 1 + d : -d; gj = a; gk = b2;
            nd.base = (gk * od.ny + gj) * od.nx + (side ? od.nx - 1 : 0);
            nd.st = side ? -1 : 1;
        } else if (ax == 1) {
            gi = a; gj = side ? od.ny - 1 + d : -d; gk = b2;
            nd.base = (gk * od.ny + (side ? od.ny - 1 : 0)) * od.nx + gi;
            nd.st = side ? -od.nx : od.nx;
        } else {
            gi = a; gj = b2; gk = side ? od.nz - 1 + d : -d;
            nd.base = (side ? od.nz - 1 : 0) * pxy + gj * od.nx + gi;
            nd.st = side ? -pxy : pxy;
        }
        nd.d = d;
    }
    nd.x = od.origin[0] + od.h * gi - od.centre[0];
    nd.y = od.origin[1] + od.h * gj - od.centre[1];
    nd.z = od.origin[2] + od.h * gk - od.centre[2];
    return nd;
}

template <int L, int MODE>
__global__ __launch_bounds__(256) void k_harm_contract(Coeffs cf, int P, const OrbDesc *orb,
                                                       const long long *gcount, const HcItem *items,
                                                       const double *src, int square, double *part) {
    constexpr int NLM = (L + 1) * (L + 1);
    constexpr int QT = (NLM + 15) / 16;                // 16-row tiles of H
    constexpr int SL = (QT + 3) / 4;                   // tiles per wave
    constexpr int R = MODE == 0 ? 1 : kMaxRadius;      // loads per f value
    constexpr int D = MODE == 0 ? 3 : 1;               // steps whose loads are in flight
    static_assert(kHc == 64, "hc_build assumes 65-double rows");
    __shared__ double Hs[QT * 16][kHc + 1];  // odd row stride: conflict-free column reads
    __shared__ double Fs[16][kHc + 1];
    __shared__ double cs[2 * kMaxRadius + 2];  // c_k, zero beyond P
    const HcItem it = items[blockIdx.x];
    const OrbDesc od = orb[it.first];  // every orbital of the channel shares this grid
    const int N = it.count;
    const int OT = (N + 15) >> 4;
    const long long M = (long long)od.nx * od.ny * od.nz;
    const long long nn = MODE == 0 ? M : gcount[it.first];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    if (threadIdx.x < 2 * kMaxRadius + 2)
        cs[threadIdx.x] = threadIdx.x <= P && threadIdx.x <= kMaxRadius ? cf.c[threadIdx.x] : 0.0;
    for (int e = threadIdx.x; e < (QT * 16 - NLM) * kHc; e += 256) Hs[NLM + e / kHc][e % kHc] = 0.0;
    dbl4 acc[SL][8];
#pragma unroll
    for (int sl = 0; sl < SL; ++sl)
#pragma unroll
        for (int ot = 0; ot < 8; ++ot) acc[sl][ot] = dbl4{0.0, 0.0, 0.0, 0.0};
    // steps s = (chunk t0 + s / OT, orbital tile s % OT); step s stages f of
    // orbitals 16 ot + w + 4 k (k < 4) at the thread's node from the raw
    // loads of ring slot s % D, issued D steps ahead
    const int nsteps = (it.t1 - it.t0) * OT;
    double raw[D][4][R];
    auto issue = [&](int st, double (&rw)[4][R]) {
        const int tq = st / OT, ot = st - tq * OT;
        const HcNode nd = hc_decode<MODE>(od, P, nn, (long long)(it.t0 + tq) * kHc + lane);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int o = 16 * ot + w + 4 * k;
            const bool ok = nd.valid && o < N;
            const double *fo = src + od.off + (long long)(ok ? o : 0) * M;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const bool tap = ok && (MODE == 0 || q + nd.d <= P);
                rw[k][q] = tap ? fo[nd.base + q * nd.st] : 0.0;
            }
        }
    };
    // products of the staged tile with this wave's harmonic tiles into the
    // accumulators of orbital tile OC
    auto products = [&](auto oc) {
        constexpr int o = decltype(oc)::value;
#pragma unroll
        for (int sl = 0; sl < SL; ++sl) {
            const int qt = w + 4 * sl;
            if (qt < QT) {
#pragma unroll
                for (int k0 = 0; k0 < kHc; k0 += 4)
                    acc[sl][o] = __builtin_amdgcn_mfma_f64_16x16x4f64(Hs[16 * qt + lr][k0 + lk], Fs[lr][k0 + lk],
                                                                      acc[sl][o], 0, 0, 0);
            }
        }
    };
#pragma unroll
    for (int j = 0; j < D; ++j)
        if (j < nsteps) issue(j, raw[j]);
    __syncthreads();  // cs and the zero rows
    HcNode ndc{};
    for (int s0 = 0; s0 < nsteps; s0 += D) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int st = s0 + j;
            if (st >= nsteps) break;  // uniform
            const int tq = st / OT, ot = st - tq * OT;
            if (ot == 0) {
                // this wave's rows of H for the chunk (the previous step's
                // products are done: barrier at the end of every step)
                ndc = hc_decode<MODE>(od, P, nn, (long long)(it.t0 + tq) * kHc + lane);
                hc_build<L, MODE>(ndc.x, ndc.y, ndc.z, ndc.valid, w, lane, Hs);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double f;
                if constexpr (MODE == 0) {
                    f = square ? raw[j][k][0] * raw[j][k][0] : raw[j][k][0];
                } else {
                    f = 0.0;
#pragma unroll
                    for (int q = 0; q < R; ++q) f += cs[q + ndc.d] * raw[j][k][q];
                    f *= od.inv_h2;
                }
                Fs[w + 4 * k][lane] = f;
            }
            if (st + D < nsteps) issue(st + D, raw[j]);  // in flight during the next D steps
            __syncthreads();  // H and f staged
            switch (ot) {
                case 0: products(std::integral_constant<int, 0>{}); break;
                case 1: products(std::integral_constant<int, 1>{}); break;
                case 2: products(std::integral_constant<int, 2>{}); break;
                case 3: products(std::integral_constant<int, 3>{}); break;
                case 4: products(std::integral_constant<int, 4>{}); break;
                case 5: products(std::integral_constant<int, 5>{}); break;
                case 6: products(std::integral_constant<int, 6>{}); break;
                default: products(std::integral_constant<int, 7>{}); break;
            }
            __syncthreads();  // products done with Fs (and, at a chunk's last tile, Hs)
        }
    }
    // partial tile: rows q, columns o (16 * OT of them); D lane l, item j is
    // (row l / 16 + 4 j, column l % 16) of a 16 x 16 tile
    const int np = 16 * OT;
    double *out = part + it.poff;
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
        const int qt = w + 4 * sl;
        if (qt < QT) {
#pragma unroll
            for (int ot = 0; ot < 8; ++ot)
                if (ot < OT)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
                        out[(size_t)(16 * qt + lk + 4 * jj) * np + 16 * ot + lr] = acc[sl][ot][jj];
        }
    }
}

// out[first + o][q] = scale_q * (sum of the channel's partial tiles), scale_q
// = dV norm_q (moments) or gfac_q norm_q (adjoint boundary); one wave per
// output value, the tiles in item order (lane-strided, then a fixed butterfly)
template <int L>
__global__ __launch_bounds__(256) void k_harm_final(HarmTables ht, const HcChan *chans, const OrbDesc *orb,
                                                    int mode, const double *part, double *out) {
    constexpr int NLM = (L + 1) * (L + 1);
    const HcChan ch = chans[blockIdx.y];
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (e >= ch.count * NLM) return;  // wave-uniform
    const int o = e / NLM, q = e - o * NLM;
    const int np = 16 * ((ch.count + 15) >> 4);
    const size_t tile = (size_t)kHcRows * np;  // tiles are kHcRows rows apart
    const double *pp = part + ch.poff + (size_t)q * np + o;
    double sum = 0.0;
    for (int p = lane; p < ch.nparts; p += 64) sum += pp[p * tile];
    sum = wave_sum(sum);
    if (lane == 0) {
        const OrbDesc od = orb[ch.first];
        const double scale = mode == 0 ? od.h * od.h * od.h * ht.norm[q] : ht.gfac[q] * ht.norm[q];
        out[(size_t)(ch.first + o) * NLM + q] = scale * sum;
    }
}

// ---------------------------------------------------------------------------
// harmonic expansions on the matrix cores: out_o(n) (+)= sum_q C'[o][q] H_q(n)
// over the nodes n of one channel
//   MODE 0 (ghost values, Sec. II.A): n = ghosts, H_q = r^l P_lm / r^(2l+1),
//          C' = gfac_q norm_q Q[o][q], out = G (written);
//   MODE 1 (multipole part of the adjoint field): n = grid nodes,
//          H_q = r^l P_lm, C' = dV norm_q zt[o][q], out = W (added to).
// A block takes a range of 64-node chunks and at most kHcExpandTiles tiles
// of 16 orbitals (so their coefficient rows C' in LDS leave room for several
// blocks per compute unit); per chunk the four waves build H as in the
// contraction, then wave w forms the 16 x 16 result tiles of nodes
// 16 w .. 16 w + 15 for each of the block's orbital tiles.
// ---------------------------------------------------------------------------

template <int L, int MODE>
__global__ __launch_bounds__(256) void k_harm_expand(HarmTables ht, int P, const OrbDesc *orb,
                                                     const long long *gcount, const HcItem *items,
                                                     const double *C, double *out) {
    constexpr int NLM = (L + 1) * (L + 1);
    constexpr int KQ = (NLM + 15) / 16 * 16;  // harmonic rows, padded
    constexpr int CST = KQ + 1;                // odd row stride of C'
    static_assert(kHc == 64, "hc_build assumes 65-double rows");
    __shared__ double Hs[KQ][kHc + 1];
    extern __shared__ double Cs[];  // [16 (ot1 - ot0)][CST]
    const HcItem it = items[blockIdx.x];
    const OrbDesc od = orb[it.first];  // every orbital of the channel shares this grid
    const int N = it.count;
    const int OT = it.ot1 - it.ot0;  // this block's orbital tiles, from it.ot0
    const long long M = (long long)od.nx * od.ny * od.nz;
    const long long nn = MODE == 0 ? gcount[it.first] : M;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    const double dV = od.h * od.h * od.h;
    for (int e = threadIdx.x; e < 16 * OT * KQ; e += 256) {
        const int r = e / KQ, q = e - r * KQ;
        const int o = 16 * it.ot0 + r;
        double v = 0.0;
        if (o < N && q < NLM)
            v = C[(size_t)(it.first + o) * NLM + q] * ht.norm[q] * (MODE == 0 ? ht.gfac[q] : dV);
        Cs[r * CST + q] = v;
    }
    for (int e = threadIdx.x; e < (KQ - NLM) * kHc; e += 256) Hs[NLM + e / kHc][e % kHc] = 0.0;
    __syncthreads();
    // steps s = (chunk t0 + s / OT, orbital tile s % OT); MODE 1 reads the W
    // values a step updates D steps ahead, so the read-modify-write does not
    // wait on memory at every chunk
    constexpr int D = MODE == 1 ? 3 : 1;
    const int nsteps = (it.t1 - it.t0) * OT;
    double wv[D][4];
    auto wload = [&](int st, double (&wr)[4]) {
        const int tq = st / OT, ot = st - tq * OT;
        const long long nout = (long long)(it.t0 + tq) * kHc + 16 * w + lr;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = 16 * (it.ot0 + ot) + lk + 4 * j;
            wr[j] = o < N && nout < nn ? out[od.off + (long long)o * M + nout] : 0.0;
        }
    };
    if constexpr (MODE == 1) {
#pragma unroll
        for (int j = 0; j < D; ++j)
            if (j < nsteps) wload(j, wv[j]);
    }
    for (int s0 = 0; s0 < nsteps; s0 += D) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int st = s0 + j;
            if (st >= nsteps) break;  // uniform
            const int tq = st / OT, ot = st - tq * OT;
            const long long n0 = (long long)(it.t0 + tq) * kHc;
            if (ot == 0) {
                if (st > 0) __syncthreads();  // the previous chunk's products are done with H
                const HcNode nd = hc_decode<MODE == 0 ? 1 : 0>(od, P, nn, n0 + lane);
                hc_build<L, MODE == 0 ? 1 : 0>(nd.x, nd.y, nd.z, nd.valid, w, lane, Hs);
                __syncthreads();  // H staged
            }
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k0 = 0; k0 < KQ; k0 += 4)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Cs[(16 * ot + lr) * CST + k0 + lk],
                                                           Hs[k0 + lk][16 * w + lr], acc, 0, 0, 0);
            // D lane l, item j: orbital 16 (ot0 + ot) + l / 16 + 4 j, node 16 w + l % 16
            const long long nout = n0 + 16 * w + lr;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int o = 16 * (it.ot0 + ot) + lk + 4 * jj;
                if (o < N && nout < nn) {
                    if constexpr (MODE == 0)
                        out[od.goff + (long long)o * nn + nout] = acc[jj];
                    else
                        out[od.off + (long long)o * M + nout] = wv[j][jj] + acc[jj];
                }
            }
            // steps st + 1 .. st + D - 1 touch other (orbital, node) pairs
            if constexpr (MODE == 1)
                if (st + D < nsteps) wload(st + D, wv[j]);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define FSIC_L_SWITCH(lmax, CALL)   \
    switch (lmax) {                 \
        case 0: CALL(0); break;     \
        case 1: CALL(1); break;     \
        case 2: CALL(2); break;     \
        case 3: CALL(3); break;     \
        case 4: CALL(4); break;     \
        case 5: CALL(5); break;     \
        case 6: CALL(6); break;     \
        case 7: CALL(7); break;     \
        case 8: CALL(8); break;     \
        default: return hipErrorInvalidValue; \
    }

int harm_slots(int kind, int lmax) {
    static std::mutex mu;
    static std::map<std::array<int, 3>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (kind < 0 || kind > 3 || lmax < 0 || lmax > kMaxL) return 1;
    std::lock_guard<std::mutex> lock(mu);
    const std::array<int, 3> key{dev, kind, lmax};
    const auto f = cache.find(key);
    if (f != cache.end()) return f->second;
    const int kq = ((lmax + 1) * (lmax + 1) + 15) / 16 * 16;
    const size_t lds = kind >= 2 ? (size_t)16 * kHcExpandTiles * (kq + 1) * sizeof(double) : 0;
    const void *fn = nullptr;
#define FN(L)                                                                                  \
    fn = kind == 0 ? (const void *)k_harm_contract<L, 0>                                       \
                   : kind == 1 ? (const void *)k_harm_contract<L, 1>                           \
                               : kind == 2 ? (const void *)k_harm_expand<L, 0> : (const void *)k_harm_expand<L, 1>
    switch (lmax) {
        case 0: FN(0); break;
        case 1: FN(1); break;
        case 2: FN(2); break;
        case 3: FN(3); break;
        case 4: FN(4); break;
        case 5: FN(5); break;
        case 6: FN(6); break;
        case 7: FN(7); break;
        default: FN(8); break;
    }
#undef FN
    if (lds > 32768) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, lds) != hipSuccess || per < 1) per = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    (void)hipGetLastError();  // a failed query leaves no error behind for the next launch
    const int slots = per * cus;
    cache[key] = slots;
    return slots;
}

hipError_t launch_harm_contract(int mode, int lmax, const HarmTables &ht, const Coeffs &c, int radius,
                                const OrbDesc *orb, const long long *ghost_count, const HcItem *items,
                                int nitems, const HcChan *chans, int nchans, int max_count,
                                const double *src, int square, double *part, double *out, hipStream_t s) {
    if (nitems <= 0 || nchans <= 0) return hipSuccess;
    if (radius < 1 || radius > kMaxRadius || max_count < 1 || max_count > kMaxOrb) return hipErrorInvalidValue;
    const int nlm = (lmax + 1) * (lmax + 1);
    const dim3 fgrid((unsigned)((max_count * nlm + 3) / 4), (unsigned)nchans);
#define CALL(L)                                                                                        \
    do {                                                                                               \
        if (mode == 0)                                                                                 \
            hipLaunchKernelGGL((k_harm_contract<L, 0>), dim3(nitems), dim3(256), 0, s, c, radius,      \
                               orb, ghost_count, items, src, square, part);                            \
        else                                                                                           \
            hipLaunchKernelGGL((k_harm_contract<L, 1>), dim3(nitems), dim3(256), 0, s, c, radius,      \
                               orb, ghost_count, items, src, square, part);                            \
        hipLaunchKernelGGL(k_harm_final<L>, fgrid, dim3(256), 0, s, ht, chans, orb, mode, part, out);  \
    } while (0)
    FSIC_L_SWITCH(lmax, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_harm_expand(int mode, int lmax, const HarmTables &ht, int radius, const OrbDesc *orb,
                              const long long *ghost_count, const HcItem *items, int nitems,
                              const double *C, double *out, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (radius < 1 || radius > kMaxRadius) return hipErrorInvalidValue;
    const int kq = ((lmax + 1) * (lmax + 1) + 15) / 16 * 16;
    const size_t lds = (size_t)16 * kHcExpandTiles * (kq + 1) * sizeof(double);
#define CALL(L)                                                                                        \
    do {                                                                                               \
        const void *fn = mode == 0 ? (const void *)k_harm_expand<L, 0> : (const void *)k_harm_expand<L, 1>; \
        if (lds > 32768) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        if (mode == 0)                                                                                 \
            hipLaunchKernelGGL((k_harm_expand<L, 0>), dim3(nitems), dim3(256), lds, s, ht, radius, orb, \
                               ghost_count, items, C, out);                                            \
        else                                                                                           \
            hipLaunchKernelGGL((k_harm_expand<L, 1>), dim3(nitems), dim3(256), lds, s, ht, radius, orb, \
                               ghost_count, items, C, out);                                            \
    } while (0)
    FSIC_L_SWITCH(lmax, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_bterm(int radius, const Coeffs &c, int norb, const OrbDesc *orb, long long max_cols,
                        double *G, hipStream_t s) {
    if (norb <= 0 || max_cols <= 0) return hipSuccess;
    if (radius < 1 || radius > kMaxRadius) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bterm, dim3((unsigned)((max_cols + 255) / 256), (unsigned)norb), dim3(256), 0, s, radius,
                       c, orb, G);
    return hipGetLastError();
}

// v_o = w_o + sum_q Q[first + o][q] U_q for N orbitals on one grid (the
// channels of a system, which share it and lie next to each other): the
// multipole-boundary solution from the zero-boundary one and the basis U of
// unit-moment boundary solutions (the Poisson map is linear in the boundary
// values, which are linear in the moments).  Block (node tile, group of up to
// 32 orbitals): each thread one node, the group's moment rows in LDS, so U is
// read once per node for up to 32 orbitals.
constexpr int kBcGroup = 32;
// The grid is symmetric about the expansion centre (the box centre) and the
// discrete operator, the boundary term and each solid harmonic keep or flip
// sign under the reflection of an axis, so each unit-moment solution U_q
// does too: only its first octant (i < ceil(nx/2), likewise j, k) is kept.
// Parity bits of harmonic q = l^2 + l + mq (mq >= 0: Re (x + iy)^m, mq < 0:
// Im (x + iy)^m, m = |mq|, times a polynomial in z and r^2 of z-parity l - m):
// bit 0 odd in x, bit 1 odd in y, bit 2 odd in z.
__device__ __forceinline__ unsigned harm_parity(int q) {
    int l = 0;
    while ((l + 1) * (l + 1) <= q) ++l;
    const int mq = q - l * l - l, m = mq < 0 ? -mq : mq;
    const unsigned px = mq >= 0 ? (unsigned)(m & 1) : (unsigned)((m + 1) & 1);
    const unsigned py = mq >= 0 ? 0u : 1u;
    const unsigned pz = (unsigned)((l + m) & 1);
    return px | (py << 1) | (pz << 2);
}

// Uc[q][octant node] = U[q][the same node of the full grid]
__global__ __launch_bounds__(256) void k_octant_pack(int nlm, int nx, int ny, int nz, const double *U, double *Uc) {
    const int hx = (nx + 1) / 2, hy = (ny + 1) / 2, hz = (nz + 1) / 2;
    const long long Mo = (long long)hx * hy * hz, M = (long long)nx * ny * nz;
    const long long n = (long long)nlm * Mo;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const long long q = e / Mo, o = e - q * Mo;
        const int i = (int)(o % hx), j = (int)((o / hx) % hy), k = (int)(o / ((long long)hx * hy));
        Uc[e] = U[q * M + ((long long)k * ny + j) * nx + i];
    }
}

hipError_t launch_octant_pack(int nlm, const int *n, const double *U, double *Uc, hipStream_t s) {
    if (nlm < 1 || nlm > kMaxLM || n[0] < 1 || n[1] < 1 || n[2] < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_octant_pack, dim3(1024), dim3(256), 0, s, nlm, n[0], n[1], n[2], U, Uc);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_bc_combine(int N, int nx, int ny, int nz, int nlm, const double *Q,
                                                    int first, const double *__restrict__ U,
                                                    const double *__restrict__ W, double *__restrict__ V) {
    __shared__ double Qs[kMaxLM * kBcGroup];  // [q][j]: one broadcast row per q
    __shared__ unsigned char par[kMaxLM];
    const int o0 = kBcGroup * blockIdx.y;
    const int no = min(kBcGroup, N - o0);
    for (int e = threadIdx.x; e < kBcGroup * nlm; e += 256) {
        const int q = e / kBcGroup, j = e - q * kBcGroup;
        Qs[e] = j < no ? Q[(size_t)(first + o0 + j) * nlm + q] : 0.0;
    }
    for (int q = threadIdx.x; q < nlm; q += 256) par[q] = (unsigned char)harm_parity(q);
    __syncthreads();
    const long long M = (long long)nx * ny * nz;
    const long long m = (long long)blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    // the node's octant image and which axes it mirrors
    const int i = (int)(m % nx), j = (int)((m / nx) % ny), k = (int)(m / ((long long)nx * ny));
    const int hx = (nx + 1) / 2, hy = (ny + 1) / 2, hz = (nz + 1) / 2;
    const int mi = min(i, nx - 1 - i), mj = min(j, ny - 1 - j), mk = min(k, nz - 1 - k);
    const unsigned flip = (i != mi ? 1u : 0u) | (j != mj ? 2u : 0u) | (k != mk ? 4u : 0u);
    const long long Mo = (long long)hx * hy * hz;
    const long long mo = ((long long)mk * hy + mj) * hx + mi;
    double acc[kBcGroup];
#pragma unroll
    for (int jj = 0; jj < kBcGroup; ++jj) acc[jj] = 0.0;
    // eight basis values in flight, then their products
    for (int q0 = 0; q0 < nlm; q0 += 8) {
        double u[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) u[kk] = q0 + kk < nlm ? U[(size_t)(q0 + kk) * Mo + mo] : 0.0;
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            if (q0 + kk >= nlm) break;
            const double uk = (__builtin_popcount(flip & par[q0 + kk]) & 1) ? -u[kk] : u[kk];
            const double *qr = Qs + (q0 + kk) * kBcGroup;
#pragma unroll
            for (int jj = 0; jj < kBcGroup; ++jj) acc[jj] += qr[jj] * uk;
        }
    }
#pragma unroll
    for (int jj = 0; jj < kBcGroup; ++jj)
        if (jj < no) {
            const size_t a = (size_t)(o0 + jj) * M + m;
            V[a] = W[a] + acc[jj];
        }
}

hipError_t launch_bc_combine(int N, const int *n, int lmax, const double *Q, int first, const double *U,
                             const double *W, double *V, hipStream_t s) {
    if (N < 1 || n[0] < 1 || n[1] < 1 || n[2] < 1 || lmax < 0 || lmax > kMaxL) return hipErrorInvalidValue;
    const long long M = (long long)n[0] * n[1] * n[2];
    const int nlm = (lmax + 1) * (lmax + 1);
    const dim3 grid((unsigned)((M + 255) / 256), (unsigned)((N + kBcGroup - 1) / kBcGroup));
    hipLaunchKernelGGL(k_bc_combine, grid, dim3(256), 0, s, N, n[0], n[1], n[2], nlm, Q, first, U, W, V);
    return hipGetLastError();
}

hipError_t launch_rhs(int radius, const Coeffs &c, const Item *items8, int nitems8,
                      const OrbDesc *orb, const double *src, int square, double scale,
                      const double *G, double *B, double *R64, float *R32, double *X64zero,
                      double *part8, hipStream_t s) {
    if (nitems8 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rhs, dim3(nitems8), dim3(256), 0, s, radius, c, orb, items8, src, square,
                       scale, G, B, R64, R32, X64zero, part8);
    return hipGetLastError();
}

}  // namespace fsic
