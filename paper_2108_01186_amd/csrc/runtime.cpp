// Host runtime of the FLOSIC SIC library: argument validation, batched work
// plans (one Poisson problem per orbital, all orbitals of all spin channels
// and systems in the same CG launches), workspace management, the forward
// and backward passes and the operator-level entry points of fsic.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fsic.h"
#include "kernels.h"

using namespace fsic;

namespace {

// ---------------------------------------------------------------------------
// small device buffer that only grows
// ---------------------------------------------------------------------------
template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n) {
        if (n <= cap) return hipSuccess;
        if (p) hipFree(p);
        p = nullptr;
        cap = 0;
        hipError_t e = hipMalloc((void **)&p, std::max<size_t>(n, 1) * sizeof(T));
        if (e == hipSuccess) cap = n;
        return e;
    }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// 2p-th order central second-difference weights on unit spacing, from the
// moment conditions sum_k c_k k^(2j) = delta_{j1} (j = 1..p, c_-k = c_k)
// solved by Gaussian elimination in extended precision.
Coeffs fd_weights(int p) {
    long double A[kMaxRadius][kMaxRadius + 1];
    for (int j = 1; j <= p; ++j) {
        for (int k = 1; k <= p; ++k) {
            long double v = 1.0L;
            for (int e = 0; e < 2 * j; ++e) v *= (long double)k;
            A[j - 1][k - 1] = 2.0L * v;
        }
        A[j - 1][p] = (j == 1) ? 2.0L : 0.0L;  // second derivative of x^2 is 2
    }
    for (int col = 0; col < p; ++col) {
        int piv = col;
        for (int r = col + 1; r < p; ++r)
            if (fabsl(A[r][col]) > fabsl(A[piv][col])) piv = r;
        if (piv != col)
            for (int c = 0; c <= p; ++c) std::swap(A[col][c], A[piv][c]);
        for (int r = 0; r < p; ++r) {
            if (r == col) continue;
            const long double f = A[r][col] / A[col][col];
            for (int c = col; c <= p; ++c) A[r][c] -= f * A[col][c];
        }
    }
    Coeffs cf{};
    long double s = 0.0L;
    for (int k = 1; k <= p; ++k) {
        const long double ck = A[k - 1][p] / A[k - 1][k - 1];
        cf.c[k] = (double)ck;
        s += ck;
    }
    cf.c[0] = (double)(-2.0L * s);
    cf.cpt = 2;
    cf.depth = 2;
    return cf;
}

HarmTables harm_tables(int lmax) {
    HarmTables t{};
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int l = 0; l <= lmax; ++l) {
        for (int m = -l; m <= l; ++m) {
            const int am = m < 0 ? -m : m;
            long double ratio = 1.0L;  // (l - |m|)! / (l + |m|)!
            for (int k = l - am + 1; k <= l + am; ++k) ratio /= (long double)k;
            long double nv = sqrtl((2.0L * l + 1.0L) / (4.0L * pi) * ratio);
            if (m != 0) nv *= sqrtl(2.0L);
            t.norm[l * l + l + m] = (double)nv;
            t.gfac[l * l + l + m] = (double)(4.0L * pi / (2.0L * l + 1.0L));
        }
    }
    return t;
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Chan {
    int sys, spin, N;
    int n[3];
    double h, origin[3];
    long long M;
    const double *psi;
    std::vector<double> fod;   // host copy, N x 3
    int first_orb;
    long long off;             // field offset of orbital 0
    std::vector<FodCell> cells;
    int nblk;                  // pointwise blocks (sic average)
    int blk_base;
    // per-channel device small arrays (offsets into the small arena)
    size_t so;                 // offset in doubles of this channel's small block
};

// small per-channel arrays, N <= kMaxOrb: u, du(3), rhoa, T, G, S, lam, U, Z, Qm, info(2), dEda(3)
constexpr size_t kSmallPerChan = (size_t)kMaxOrb * kMaxOrb * 8 + (size_t)kMaxOrb * 8 + 64;
enum SmallSlot { sU_ = 0, sDU, sRHOA, sT, sG, sS, sLAM, sEV, sZ, sQ, sINFO, sDEDA };
size_t small_off(SmallSlot s) {
    const size_t NN = (size_t)kMaxOrb * kMaxOrb;
    switch (s) {
        case sU_: return 0;
        case sDU: return NN;                 // 3 NN
        case sT: return 4 * NN;
        case sG: return 5 * NN;
        case sS: return 6 * NN;
        case sEV: return 7 * NN;
        case sZ: return 8 * NN;
        case sQ: return 9 * NN;
        case sRHOA: return 10 * NN;          // N
        case sLAM: return 10 * NN + kMaxOrb;
        case sINFO: return 10 * NN + 2 * kMaxOrb;
        case sDEDA: return 10 * NN + 2 * kMaxOrb + 8;  // 3N
    }
    return 0;
}
constexpr size_t kSmallStride = (size_t)kMaxOrb * kMaxOrb * 10 + 2 * kMaxOrb + 8 + 3 * kMaxOrb + 8;

// A batch of Poisson problems sharing one launch sequence.
struct Batch {
    std::vector<OrbDesc> orb;
    std::vector<Item> items7, items8;
    std::vector<long long> gcount;
    long long fields = 0;  // total elements
    long long ghosts = 0;
    long long max_ghost = 0;
    int tot7 = 0, tot8 = 0;
    // spectral preconditioner: panel work lists, sine matrices and symbols
    std::vector<Item> dx, dy, dz;
    std::vector<Item> dxy;  // fused x-y units (orbital, z plane) when dst_xy
    std::vector<float> dtab;
    int tot9 = 0;
    int max_n = 0;
    int dst_fast = 0;      // transform variant (see DstItems)
    bool dst_xy = false;   // in-plane transforms fused per z plane
    bool dst_two = false;  // some orbital has nx != ny
    bool dst_vec = true;   // every nx and orbital offset is a multiple of 4
    int npxy = 0;          // largest in-plane axis, padded to 32
    bool dst_zocc2 = false;  // z pass in 64-column panels, two blocks per compute unit
    bool dst_xyocc2 = true;  // fused x-y passes two blocks per compute unit where the plane fits
    bool dst_pv = true;      // inverse pass reads p_old before its products
    int max_group = 0;  // most orbitals in one channel
    // harmonic contractions over grid nodes (moments) and ghosts (adjoint
    // boundary): block items, channel ranges, partial-tile elements
    std::vector<HcItem> hcN, hcG;
    std::vector<HcItem> hcNx, hcGx;  // the same split by orbital tile groups (expansions)
    std::vector<HcChan> hchN, hchG;
    long long hc_elems = 0;
};

// Splits every channel's 64-node chunks into contiguous ranges, nblocks
// blocks in all (the blocks the device holds at once: one round, no tail),
// per channel in proportion to its work (chunks x orbital tiles).
void build_hc_items(const std::vector<std::array<long long, 3>> &chans, std::vector<HcItem> &items,
                    std::vector<HcChan> &out, long long &elems, int nblocks) {
    items.clear();
    out.clear();
    elems = 0;
    double total = 0.0;
    for (const auto &ch : chans) total += (double)((ch[2] + 63) / 64) * (double)((ch[1] + 15) / 16);
    for (const auto &ch : chans) {
        const int first = (int)ch[0], count = (int)ch[1];
        const long long chunks = (ch[2] + 63) / 64;
        if (count <= 0 || chunks <= 0) continue;
        const double work = (double)chunks * (double)((count + 15) / 16);
        long long nb = (long long)std::llround(nblocks * work / std::max(total, 1.0));
        nb = std::max(1LL, std::min(nb, chunks));
        const long long tile = (long long)kHcRows * 16 * ((count + 15) / 16);
        HcChan hc{first, count, (int)nb, elems};
        for (long long i = 0; i < nb; ++i) {
            items.push_back(HcItem{first, count, (int)(chunks * i / nb), (int)(chunks * (i + 1) / nb), elems, 0,
                                   (count + 15) / 16});
            elems += tile;
        }
        out.push_back(hc);
    }
}


void build_items(const std::vector<std::pair<int, int>> &natural, std::vector<Item> &out) {
    const int n = (int)natural.size();
    const int nb = ((n + 7) / 8) * 8;
    out.assign(nb, Item{-1, 0});
    const int per = nb / 8;
    for (int b = 0; b < nb; ++b) {
        const int idx = xcd_item_of_block(b, nb);
        (void)per;
        if (idx < n) out[b] = Item{natural[idx].first, natural[idx].second};
    }
}

// one sampled launch (FSIC_PROFILE): kind 0 sweep, 1 update, 2 preconditioner,
// 3 residual pass; HIP events around it
struct ProfRec {
    int kind, k, flag;
    hipEvent_t a, b;
};

// what a pinned-memory upload cache remembers of the last upload of a table
struct UpCache {
    const void *dev = nullptr;
    std::vector<char> bytes;
};

}  // namespace

struct fsic_ctx {
    fsic_opts opts{};
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;

    // field buffers
    DBuf<double> PHI, V, W, B, R, P0, P1, Q, X64b;
    DBuf<float> R32, P32a, P32b, Q32, X32;
    DBuf<float> Z32, T32, dtab;     // preconditioned CG: z, transform work array, spectral table
    DBuf<double> partRZ;
    DBuf<float> Fprev, Fh;               // AAR: previous f, f-difference history
    DBuf<double> Xh, aar_gamma, partD;  // AAR: step history, weights, Gram partials
    DBuf<Item> d_dx, d_dy, d_dz, d_dxy;
    DBuf<double> Gh;  // ghost values
    DBuf<double> part7, part8, partRU, partH;  // partH: harmonic-contraction partial tiles
    DBuf<HcItem> d_hcN, d_hcG, d_hcNx, d_hcGx;
    DBuf<HcChan> d_hchN, d_hchG;
    DBuf<double> bb, rrfin, relres, Qlm, Zt, ptrue;
    DBuf<int> done, iters, rs_iter, nact;
    DBuf<OrbDesc> d_orb;
    DBuf<Item> d_items7, d_items8;
    DBuf<long long> d_gcount;
    DBuf<double> small;   // per-channel small arrays
    DBuf<double> work;    // Jacobi / N x N scratch
    DBuf<double> partG;
    DBuf<FodCell> d_cells;
    DBuf<ChanDesc> d_chan;
    DBuf<int> d_blkchan;
    DBuf<double> partU, partX;
    DBuf<double> eux;  // U_i, X_i of every orbital, then E_SIC of every channel (one copy out)
    DBuf<int> status;
    DBuf<double> bmat;
    int *h_done = nullptr;  // pinned
    DBuf<int> ndone, fin;   // converged-orbital counter; buffer holding each final x (mixed PCG)
    DBuf<int> pz;           // mixed PCG: local iteration from which an orbital pauses in its cycle
    int *h_nd = nullptr;    // pinned: two copies of the counter, one per cycle parity
    hipEvent_t evc[2] = {nullptr, nullptr};
    int pred_cycles = 0;    // restart cycles the last mixed solve needed (host checks skipped before)
    // statistics of the last solve, copied to pinned memory and read after
    // the caller's synchronisation (finish_solve)
    // pinned copy of the last solve's statistics (one transfer from
    // d_stage): [8 norb ints: iters, the six nact blocks, done][2 norb
    // doubles: final residual^2, ||b||^2]; h_si and h_sd point into it
    double *h_stage = nullptr;
    int *h_si = nullptr;
    double *h_sd = nullptr;
    size_t h_s_cap = 0;
    DBuf<double> d_stage;
    DBuf<double> d_chk;  // the host checks' inputs, packed (forward pass)
    DBuf<double> d_grad;  // dE/da of every channel, packed (backward pass)
    std::vector<ProfRec> recs;
    bool pend_prof = false, pend_aar = false, pend_pcg = false, pend_mixed = false;
    bool pend_dst_xy = false;
    int pend_dst_fast = 0;
    // device status word of the forward pass, copied once the Loewdin step
    // has run; a solve stops early when it shows an error
    int *h_stat = nullptr;
    bool watch_status = false;
    // pinned staging of the per-channel host checks (G, info, rho(a))
    double *h_chk = nullptr;
    size_t h_chk_cap = 0;
    double *h_eux = nullptr;  // pinned host copy of eux
    size_t h_eux_cap = 0;
    double *h_grad = nullptr;  // pinned host copy of the channels' dE/da
    size_t h_grad_cap = 0;
    std::map<const void *, UpCache> upcache;  // last upload per device table
    // profiling (FSIC_PROFILE): events around every CG launch
    std::vector<hipEvent_t> ev;
    int32_t sweep_launches = 0, update_launches = 0, precond_launches = 0;
    double sweep_ms = 0, sweep_bytes = 0, update_ms = 0, update_bytes = 0;
    double precond_ms = 0, precond_bytes = 0, precond_flops = 0;
    int32_t resid_launches = 0;
    double resid_ms = 0, resid_bytes = 0;
    size_t h_done_cap = 0;

    // plan of the last forward pass (the tape)
    std::vector<Chan> chans;
    Batch batch;
    int nsys = 0;
    bool tape = false;
    // W holds the zero-boundary solutions of the last forward pass (the
    // adjoint fields), until a backward pass overwrites it
    bool w_ready = false;
    // unit-moment boundary solutions per grid (n, h bits, lmax, radius):
    // (lmax + 1)^2 fields of the grid's size, solved once
    std::map<std::array<long long, 6>, DBuf<double>> bbasis;
    DBuf<double> qident;  // identity moments of the basis solves
    int basis_solves = 0;
    double basis_ms = 0.0;
    int radius = 6;
    Coeffs cf{};
    // stencil shape of the last batch and the time its tuning took (0: cached)
    int shape_cpt = 2, shape_depth = 1;
    long long shape_target = 0;
    double tune_ms = 0.0;
    // preconditioner layout of the last batch (fsic_stats.precond_layout) and
    // the time its tuning took (0: cached or not tuned)
    int dst_layout = 0;
    double dst_tune_ms = 0.0;
    // FSIC_GRAPHS: captured CG chunks, and the stream they are captured on
    std::map<std::vector<uint64_t>, hipGraphExec_t> graphs;
    int graph_captures = 0;  // graphs captured over the context's life (FSIC_GRAPHS)
    hipStream_t cap_stream = nullptr;
    HarmTables ht{};

    bool fail(fsic_status, const std::string &m) {
        err = m;
        return false;
    }
};

namespace {

fsic_status set_err(fsic_ctx *c, fsic_status s, const std::string &m) {
    if (c) c->err = m;
    return s;
}

#define HIPCHK(ctx, call)                                                               \
    do {                                                                                \
        hipError_t _e = (call);                                                         \
        if (_e != hipSuccess)                                                           \
            return set_err(ctx, _e == hipErrorOutOfMemory ? FSIC_ENOMEM : FSIC_EHIP,    \
                           std::string(#call) + ": " + hipGetErrorString(_e));          \
    } while (0)

fsic_status validate_opts(const fsic_opts *o, std::string &why) {
    if (!o) { why = "opts is NULL"; return FSIC_EINVAL; }
    if (o->fd_order < 2 || o->fd_order > 12 || (o->fd_order & 1)) { why = "fd_order must be even in [2, 12]"; return FSIC_EINVAL; }
    if (o->lmax < 0 || o->lmax > kMaxL) { why = "lmax must be in [0, 8]"; return FSIC_EINVAL; }
    if (o->solver != FSIC_CG && o->solver != FSIC_PCG && o->solver != FSIC_AAR) { why = "solver must be FSIC_CG, FSIC_PCG or FSIC_AAR"; return FSIC_EINVAL; }
    if (o->solver == FSIC_AAR && o->precision != FSIC_FP64) { why = "FSIC_AAR runs in FSIC_FP64"; return FSIC_EINVAL; }
    if (o->precision != FSIC_FP64 && o->precision != FSIC_MIXED) { why = "precision must be FSIC_FP64 or FSIC_MIXED"; return FSIC_EINVAL; }
    if (!(o->tol > 0.0 && o->tol < 1.0)) { why = "tol must be in (0, 1)"; return FSIC_EINVAL; }
    if (o->max_iter < 1) { why = "max_iter must be >= 1"; return FSIC_EINVAL; }
    if (!std::isfinite(o->vsic_scale)) { why = "vsic_scale must be finite"; return FSIC_EINVAL; }
    if (!(o->rho_floor >= 0.0) || !std::isfinite(o->rho_floor)) { why = "rho_floor must be finite and >= 0"; return FSIC_EINVAL; }
    if (!(o->s_eig_floor > 0.0) || !std::isfinite(o->s_eig_floor)) { why = "s_eig_floor must be finite and > 0"; return FSIC_EINVAL; }
    if (o->flags & ~(FSIC_WANT_VSIC | FSIC_KEEP_TAPE | FSIC_ALLOW_NONORTHO | FSIC_PROFILE | FSIC_FP32_ORBITALS |
                     FSIC_GRAPHS | FSIC_PAPER_GRADIENT | FSIC_EQ9_FORCES | FSIC_DIRECT_BC)) {
        why = "unknown flag bits";
        return FSIC_EINVAL;
    }
    return FSIC_OK;
}

fsic_status validate_grid(const fsic_grid &g, std::string &why) {
    for (int d = 0; d < 3; ++d) {
        if (g.n[d] < 8 || g.n[d] > 4096) { why = "grid n must be in [8, 4096] on every axis"; return FSIC_EINVAL; }
        if (!std::isfinite(g.origin[d])) { why = "grid origin must be finite"; return FSIC_EINVAL; }
    }
    if (!(g.h > 0.0) || !std::isfinite(g.h)) { why = "grid spacing h must be finite and > 0"; return FSIC_EINVAL; }
    // one orbital's FP64 field must stay below 4 GiB (32-bit buffer ranges and node indices)
    if ((long long)g.n[0] * g.n[1] * g.n[2] >= (1LL << 29)) { why = "grid must have fewer than 2^29 nodes"; return FSIC_EINVAL; }
    return FSIC_OK;
}

// Stencil shape: tile height (32 x 8*cpt columns per block), planes
// prefetched ahead (depth), and the number of blocks a launch should reach
// (z-chunks are halved until it does, so a launch fills the 256 compute
// units several times over).
struct Shape {
    int cpt, depth;
    long long target;
};

// preconditioned mixed-precision CG: FP32 iterations between FP64 residual
// checks (each restarts the FP32 recursion).  The FP32 recursion stops
// gaining after a few iterations of a strong preconditioner (measured on
// 40^3-192^3 workloads: two iterations per restart need no more iterations
// in total than FP64 CG with the split-bf16 transforms; three suit the
// weaker ones).  FSIC_PCG_CHUNK overrides.
int pcg_chunk(int variant) {
    static int v = [] {
        const char *e = getenv("FSIC_PCG_CHUNK");
        return e ? std::max(1, atoi(e)) : 0;
    }();
    if (v) return v;
    return (variant == 1 || variant == 2) ? 2 : 3;
}

// iterations of the first restart cycle (from x = 0); FSIC_PCG_FIRST
// overrides
int pcg_first_chunk(int variant) {
    static int v = [] {
        const char *e = getenv("FSIC_PCG_FIRST");
        return e ? std::max(1, atoi(e)) : 0;
    }();
    if (v) return v;
    return pcg_chunk(variant);
}

// AAR parameters (the paper does not state them): Richardson weight omega,
// Anderson mixing beta, an Anderson step every kAarPeriod iterations over
// the last kAarM differences; with the sine-transform preconditioner these
// reach 1e-11 in about as many iterations as preconditioned CG.  The host
// reads the convergence flags every kAarCheck iterations.
constexpr double kAarOmega = 1.0;
constexpr double kAarBeta = 1.0;
constexpr int kAarPeriod = 3;
constexpr int kAarCheck = 4;

// CG iterations between profiled ones (FSIC_PROFILE); FSIC_PROFILE_EVERY
// overrides the default 16
int profile_period() {
    static int v = [] {
        const char *e = getenv("FSIC_PROFILE_EVERY");
        return e ? std::max(1, atoi(e)) : 16;
    }();
    return v;
}

void tile_orbital(OrbDesc &od, int radius, int cpt, long long total_cols_blocks, long long target) {
    od.tiles_x = (od.nx + kTX - 1) / kTX;
    od.tiles_y = (od.ny + 8 * cpt - 1) / (8 * cpt);
    int zc = od.nz;
    long long blocks = total_cols_blocks;
    while (blocks < target && zc >= 4 * radius && zc >= 16) {
        zc = (zc + 1) / 2;
        blocks *= 2;
    }
    od.zc = zc;
    od.tiles_z = (od.nz + zc - 1) / zc;
}

// Build the batch of Poisson problems for a list of (grid, count) groups.
struct Group {
    int n[3];
    double h, origin[3];
    int count;
    long long off;  // field offset of the first orbital
    int chan;
};

// blocks of the persistent transform kernels: one per compute unit, or
// FSIC_DST_BLOCKS
int dst_blocks(const fsic_ctx *c) {
    if (const char *e = getenv("FSIC_DST_BLOCKS")) return std::max(1, atoi(e));
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || v < 1)
        v = 256;
    return v;
}

// Spectral-table block of an axis of n nodes (cached per process): the
// np x np sine matrix sin(pi (m+1)(k+1) / (n+1)) (zero beyond n, np = n
// rounded up to 32), then the n symbols -(c_0 + 2 sum_q c_q cos(q theta_j)).
const std::vector<float> &dst_block(int n, int radius) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, std::vector<float>> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto f = cache.find({n, radius});
    if (f != cache.end()) return f->second;
    const int np = (n + 31) & ~31;
    std::vector<float> v((size_t)np * np, 0.f);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int m = 0; m < n; ++m)
        for (int k = 0; k < n; ++k) {
            // argument reduced exactly in integers
            const long long a = ((long long)(m + 1) * (k + 1)) % (2LL * (n + 1));
            v[(size_t)m * np + k] = (float)sinl(pi * (long double)a / (long double)(n + 1));
        }
    const Coeffs cw = fd_weights(radius);
    for (int j = 0; j < n; ++j) {
        const long double th = pi * (long double)(j + 1) / (long double)(n + 1);
        long double sg = cw.c[0];
        for (int q = 1; q <= radius; ++q) sg += 2.0L * cw.c[q] * cosl(q * th);
        v.push_back((float)(-sg));
    }
    return cache.emplace(std::make_pair(n, radius), std::move(v)).first->second;
}

// LDS bytes one workgroup may use on the current device
size_t device_lds_limit() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
    return (size_t)v;
}

// Layout choices of the spectral preconditioner that LDS fit leaves open;
// each takes effect only where the kernels it names fit (see build_batch):
// fused x-y passes (else five per-axis passes), two fused-pass blocks per
// compute unit, the two-block z pass, and the inverse pass reading p_old
// before its products.  Defaults: all on; choose_dst times the others.
struct DstTune {
    bool xy = true, xyocc2 = true, zocc2 = true, pv = true;
};

void build_batch(const std::vector<Group> &groups, int radius, const Shape &sh, Batch &b,
                 const DstTune &dt = DstTune{}, int lmax = 6) {
    const int cpt = sh.cpt;
    b = Batch{};
    long long cols = 0;
    for (const Group &g : groups)
        cols += (long long)g.count * ((g.n[0] + kTX - 1) / kTX) * ((g.n[1] + 8 * cpt - 1) / (8 * cpt));
    for (const Group &g : groups)
        for (int d = 0; d < 3; ++d) b.max_n = std::max(b.max_n, g.n[d]);
    // fastest transform variant whose LDS fits the device
    const int npx = (b.max_n + 31) & ~31;
    const size_t ldsmax = device_lds_limit();
    int variant = 0;
    if (npx <= dst_variant_npmax(1) && dst_fast_lds(npx, 128, true) <= ldsmax) variant = 1;
    else if (npx <= dst_variant_npmax(2) && dst_fast_lds(npx, 64, true) <= ldsmax) variant = 2;
    else if (npx <= dst_variant_npmax(3) && dst_fast_lds(npx, 64, false) <= ldsmax) variant = 3;
    const bool fast = variant != 0;
    b.dst_fast = variant;
    // fused x-y passes: in-plane axes of at most 128 nodes and LDS for the
    // plane plus one sine matrix (two when some grid has nx != ny);
    // FSIC_DST_XY=0 keeps five separate passes
    for (const Group &g : groups) b.dst_two = b.dst_two || g.n[0] != g.n[1];
    for (const Group &g : groups) b.npxy = std::max(b.npxy, std::max(g.n[0], g.n[1]));
    b.npxy = (b.npxy + 31) & ~31;
    {
        const char *env = std::getenv("FSIC_DST_XY");
        b.dst_xy = fast && b.npxy <= 128 && dst_xy_lds(b.npxy, b.dst_two) <= ldsmax &&
                   !(env && std::atoi(env) == 0) && dt.xy;
        b.dst_zocc2 = b.dst_xy && variant == 1 && dst_z_occ2(npx) && dt.zocc2;
        b.dst_xyocc2 = dt.xyocc2;
        const char *epv = std::getenv("FSIC_DST_PV");
        b.dst_pv = dt.pv && !(epv && std::atoi(epv) == 0);
    }
    std::vector<std::pair<int, int>> nat7, nat8, natx, naty, natz;
    std::map<int, std::pair<int, int>> dst_done;  // n -> (sine offset, symbol offset)
    auto dst_entry = [&](Batch &bb, int n, int radius_) -> const std::pair<int, int> & {
        auto f = dst_done.find(n);
        if (f != dst_done.end()) return f->second;
        const int np = (n + 31) & ~31;
        const std::vector<float> &blk = dst_block(n, radius_);  // np x np sines, then n symbols
        const int so = (int)bb.dtab.size();
        bb.dtab.insert(bb.dtab.end(), blk.begin(), blk.end());
        const int go = so + np * np;
        // pad the table to a multiple of 4 floats
        while (bb.dtab.size() % 4) bb.dtab.push_back(0.f);
        return dst_done[n] = {so, go};
    };
    // harmonic contractions and expansions: one group per run of
    // consecutive groups on one grid whose fields follow each other (the two
    // spins of a system), at most kMaxOrb orbitals, so the harmonics of a
    // node chunk are built once for all of them
    std::vector<std::array<long long, 3>> hcn, hcg;  // (first, count, nodes / ghosts)
    const Group *hprev = nullptr;
    for (const Group &g : groups) {
        const long long M = (long long)g.n[0] * g.n[1] * g.n[2];
        if (g.count > 0) {
            const int first = (int)b.orb.size();
            const long long G = 2LL * radius * ((long long)g.n[1] * g.n[2] + (long long)g.n[0] * g.n[2] +
                                                (long long)g.n[0] * g.n[1]);
            const bool join = hprev && !hcn.empty() && hprev->n[0] == g.n[0] && hprev->n[1] == g.n[1] &&
                              hprev->n[2] == g.n[2] && hprev->h == g.h && hprev->origin[0] == g.origin[0] &&
                              hprev->origin[1] == g.origin[1] && hprev->origin[2] == g.origin[2] &&
                              hcn.back()[0] + hcn.back()[1] == first &&
                              hprev->off + (long long)hprev->count * M == g.off &&
                              hcn.back()[1] + g.count <= kMaxOrb;
            if (join) {
                hcn.back()[1] += g.count;
                hcg.back()[1] += g.count;
            } else {
                hcn.push_back({first, g.count, M});
                hcg.push_back({first, g.count, G});
            }
            b.max_group = std::max(b.max_group, (int)hcn.back()[1]);
            hprev = &g;
        }
        for (int i = 0; i < g.count; ++i) {
            OrbDesc od{};
            od.nx = g.n[0]; od.ny = g.n[1]; od.nz = g.n[2];
            tile_orbital(od, radius, cpt, cols, sh.target);
            od.nt7 = od.tiles_x * od.tiles_y * od.tiles_z;
            od.base7 = b.tot7;
            b.tot7 += od.nt7;
            od.nt8 = (int)((M + kPW - 1) / kPW);
            od.base8 = b.tot8;
            b.tot8 += od.nt8;
            od.off = g.off + (long long)i * M;
            b.dst_vec = b.dst_vec && (g.n[0] % 4 == 0) && (od.off % 4 == 0);
            const long long G = 2LL * radius * ((long long)g.n[1] * g.n[2] + (long long)g.n[0] * g.n[2] + (long long)g.n[0] * g.n[1]);
            od.goff = b.ghosts;
            b.ghosts += G;
            b.max_ghost = std::max(b.max_ghost, G);
            b.gcount.push_back(G);
            od.h = g.h;
            od.inv_h2 = 1.0 / (g.h * g.h);
            for (int d = 0; d < 3; ++d) {
                od.origin[d] = g.origin[d];
                od.centre[d] = g.origin[d] + 0.5 * g.h * (g.n[d] - 1);
            }
            od.chan = g.chan;
            // preconditioner units: panels of 128 columns (fast) or 32
            auto nitem = [&](long long ncol) {
                const int pc = dst_panel_cols(variant);
                return (int)((ncol + pc - 1) / pc);
            };
            // r.z partial slots: one per z-pass panel (the z pass forms r.z
            // from the spectral coefficients)
            const int zpc = 64;  // z-pass panel columns (every variant)
            od.nt9 = (int)(((long long)g.n[0] * g.n[1] + zpc - 1) / zpc);
            od.base9 = b.tot9;
            b.tot9 += od.nt9;
            for (int d = 0; d < 3; ++d) {
                const auto &e = dst_entry(b, g.n[d], radius);
                od.dst_s[d] = e.first;
                od.dst_g[d] = e.second;
            }
            const int o = (int)b.orb.size();
            b.orb.push_back(od);
            // the z-chunks of one column tile next to each other: their
            // blocks share an XCD and run together, so the planes beside a
            // chunk boundary (reached by both at once, the odd chunks marching
            // downwards) are fetched once into that XCD's L2
            for (int by = 0; by < od.tiles_y; ++by)
                for (int bx = 0; bx < od.tiles_x; ++bx)
                    for (int bz = 0; bz < od.tiles_z; ++bz)
                        nat7.push_back({o, bx + od.tiles_x * (by + od.tiles_y * bz)});
            for (int t = 0; t < od.nt8; ++t) nat8.push_back({o, t});
            if (b.dst_xy) {
                for (int z = 0; z < g.n[2]; ++z) b.dxy.push_back(Item{o, z});
            } else {
                const int nx_t = nitem((long long)g.n[1] * g.n[2]);  // x-pass panels
                for (int t = 0; t < nx_t; ++t) natx.push_back({o, t});
                const int ny_t = nitem((long long)g.n[0] * g.n[2]);
                for (int t = 0; t < ny_t; ++t) naty.push_back({o, t});
            }
            const int nz_t = (int)(((long long)g.n[0] * g.n[1] + zpc - 1) / zpc);
            for (int t = 0; t < nz_t; ++t) natz.push_back({o, t});
            b.fields = std::max(b.fields, od.off + M);
        }
    }
    build_items(nat7, b.items7);
    build_items(nat8, b.items8);
    long long en = 0, eg = 0;
    build_hc_items(hcn, b.hcN, b.hchN, en, harm_slots(0, lmax));
    // (a ghost chunk's work falls with its depth, and a block takes
    // consecutive chunks: half again as many blocks as fit at once lets
    // the dispatcher even out the blocks of shallow and deep layers)
    build_hc_items(hcg, b.hcG, b.hchG, eg, harm_slots(1, lmax) * 3 / 2);
    b.hc_elems = std::max(en, eg);
    // expansions: their own ranges (a block takes at most kHcExpandTiles
    // orbital tiles), about as many blocks as the device holds at once
    int tgroups = 1;
    for (const auto &h : hcn) tgroups = std::max(tgroups, (int)((h[1] + 15) / 16 + kHcExpandTiles - 1) / kHcExpandTiles);
    for (int kind = 0; kind < 2; ++kind) {
        std::vector<HcItem> ranges;
        std::vector<HcChan> rch;
        long long rel = 0;
        build_hc_items(kind ? hcn : hcg, ranges, rch, rel, std::max(1, harm_slots(kind ? 3 : 2, lmax) / tgroups));
        std::vector<HcItem> &dst = kind ? b.hcNx : b.hcGx;
        dst.clear();
        for (const HcItem &it : ranges)
            for (int o0 = 0; o0 < it.ot1; o0 += kHcExpandTiles) {
                HcItem e = it;
                e.ot0 = o0;
                e.ot1 = std::min(it.ot1, o0 + kHcExpandTiles);
                dst.push_back(e);
            }
    }
    // persistent kernels take contiguous unit ranges: keep orbital order so
    // one sine matrix serves a whole range
    for (auto *pr : {&natx, &naty, &natz}) {
        std::vector<Item> &dst = pr == &natx ? b.dx : (pr == &naty ? b.dy : b.dz);
        dst.clear();
        for (const auto &q : *pr) dst.push_back(Item{q.first, q.second});
    }
}

template <typename T>
fsic_status upload(fsic_ctx *c, DBuf<T> &d, const std::vector<T> &h) {
    HIPCHK(c, d.ensure(h.size()));
    if (h.empty()) return FSIC_OK;
    // skip the copy when the device table already holds these bytes
    UpCache &uc = c->upcache[&d];
    const size_t nb = h.size() * sizeof(T);
    if (uc.dev == d.p && uc.bytes.size() == nb && std::memcmp(uc.bytes.data(), h.data(), nb) == 0)
        return FSIC_OK;
    HIPCHK(c, hipMemcpyAsync(d.p, h.data(), nb, hipMemcpyHostToDevice, c->stream));
    uc.dev = d.p;
    uc.bytes.assign(reinterpret_cast<const char *>(h.data()), reinterpret_cast<const char *>(h.data()) + nb);
    return FSIC_OK;
}

// The spectral preconditioner serves batches whose longest axis fits one of
// the transform variants (about 208 nodes); larger batches are solved with
// plain CG.
bool use_pcg(const fsic_ctx *c, const Batch &b) {
    return c->opts.solver == FSIC_PCG && b.dst_fast != 0;
}

// AAR uses the same preconditioner, so the same limit (larger batches: plain CG)
bool use_aar(const fsic_ctx *c, const Batch &b) {
    return c->opts.solver == FSIC_AAR && b.dst_fast != 0;
}

// Upload a batch's tables and size the solver buffers.
fsic_status prepare_batch(fsic_ctx *c, const Batch &b, int precision) {
    const size_t F = (size_t)b.fields;
    fsic_status st;
    if ((st = upload(c, c->d_orb, b.orb))) return st;
    if ((st = upload(c, c->d_items7, b.items7))) return st;
    if ((st = upload(c, c->d_items8, b.items8))) return st;
    if ((st = upload(c, c->d_gcount, b.gcount))) return st;
    if ((st = upload(c, c->d_hcN, b.hcN))) return st;
    if ((st = upload(c, c->d_hcG, b.hcG))) return st;
    if ((st = upload(c, c->d_hcNx, b.hcNx))) return st;
    if ((st = upload(c, c->d_hcGx, b.hcGx))) return st;
    if ((st = upload(c, c->d_hchN, b.hchN))) return st;
    if ((st = upload(c, c->d_hchG, b.hchG))) return st;
    if (use_pcg(c, b) || use_aar(c, b)) {
        if ((st = upload(c, c->d_dx, b.dx))) return st;
        if ((st = upload(c, c->d_dy, b.dy))) return st;
        if ((st = upload(c, c->d_dz, b.dz))) return st;
        if (b.dst_xy && (st = upload(c, c->d_dxy, b.dxy))) return st;
        if ((st = upload(c, c->dtab, b.dtab))) return st;
        if (b.dst_fast) HIPCHK(c, dst_setup((b.max_n + 31) & ~31, b.dst_fast, b.dst_xy ? b.npxy : 0, b.dst_two));
        HIPCHK(c, c->Z32.ensure(F));
        HIPCHK(c, c->T32.ensure(F));
        HIPCHK(c, c->partRZ.ensure(2 * (size_t)b.tot9));
        if (precision == FSIC_FP64) HIPCHK(c, c->P1.ensure(F));
        else HIPCHK(c, c->P32b.ensure(F));
    }
    if (use_aar(c, b)) {
        HIPCHK(c, c->R32.ensure(F));
        HIPCHK(c, c->Fprev.ensure(F));
        HIPCHK(c, c->Fh.ensure((size_t)kAarM * F));
        HIPCHK(c, c->Xh.ensure((size_t)kAarM * F));
        HIPCHK(c, c->aar_gamma.ensure((size_t)b.orb.size() * kAarM));
        HIPCHK(c, c->partD.ensure((size_t)b.tot8 * kAarD));
    }
    HIPCHK(c, c->B.ensure(F));
    if (precision == FSIC_FP64) {
        HIPCHK(c, c->R.ensure(F));
        HIPCHK(c, c->P0.ensure(F));
        HIPCHK(c, c->Q.ensure(F));
    } else {
        HIPCHK(c, c->R32.ensure(F));
        HIPCHK(c, c->P32a.ensure(F));
        HIPCHK(c, c->Q32.ensure(F));
        HIPCHK(c, c->X32.ensure(F));
    }
    const int norb = (int)b.orb.size();
    const int nlm = (c->opts.lmax + 1) * (c->opts.lmax + 1);
    HIPCHK(c, c->Gh.ensure((size_t)b.ghosts));
    HIPCHK(c, c->part7.ensure(3 * (size_t)b.tot7));
    HIPCHK(c, c->partRU.ensure((size_t)b.tot7));
    HIPCHK(c, c->part8.ensure(2 * (size_t)b.tot8));
    HIPCHK(c, c->partH.ensure((size_t)b.hc_elems));
    HIPCHK(c, c->bb.ensure(norb));
    HIPCHK(c, c->rrfin.ensure(norb));
    HIPCHK(c, c->relres.ensure(norb));
    HIPCHK(c, c->ptrue.ensure(norb));
    HIPCHK(c, c->Qlm.ensure((size_t)norb * nlm));
    HIPCHK(c, c->Zt.ensure((size_t)norb * nlm));
    HIPCHK(c, c->done.ensure(norb));
    HIPCHK(c, c->iters.ensure(norb));
    HIPCHK(c, c->rs_iter.ensure(norb));
    HIPCHK(c, c->nact.ensure(6 * (size_t)norb));
    HIPCHK(c, c->ndone.ensure(1));
    HIPCHK(c, c->fin.ensure(norb));
    HIPCHK(c, c->pz.ensure(norb));
    if (!c->h_nd) HIPCHK(c, hipHostMalloc((void **)&c->h_nd, 2 * sizeof(int)));
    for (hipEvent_t &e : c->evc)
        if (!e) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (c->h_done_cap < (size_t)norb) {
        if (c->h_done) hipHostFree(c->h_done);
        c->h_done = nullptr;
        HIPCHK(c, hipHostMalloc((void **)&c->h_done, std::max(norb, 1) * sizeof(int)));
        c->h_done_cap = norb;
    }
    if (c->h_s_cap < (size_t)norb) {
        if (c->h_stage) hipHostFree(c->h_stage);
        c->h_stage = nullptr;
        c->h_si = nullptr;
        c->h_sd = nullptr;
        HIPCHK(c, hipHostMalloc((void **)&c->h_stage, 6 * (size_t)std::max(norb, 1) * sizeof(double)));
        c->h_s_cap = norb;
    }
    if (!c->h_stat) {
        HIPCHK(c, hipHostMalloc((void **)&c->h_stat, sizeof(int)));
        *c->h_stat = 0;
    }
    return FSIC_OK;
}

// The forward pass's device status (copied asynchronously once the
// Loewdin step has run) shows an error: its solves need not finish.
bool status_error(const fsic_ctx *c) { return c->watch_status && c->h_stat && *c->h_stat != 0; }

struct SolveReport {
    int max_iters = 0;
    long long total_iters = 0;
    int refinements = 0;
    double max_relres = 0.0;
    bool converged = true;
};

// ---------------------------------------------------------------------------
// stencil autotuner
// ---------------------------------------------------------------------------

Shape default_shape(int radius, int precision) {
    if (radius != 6) return Shape{2, 2, 4096};
    return precision == FSIC_MIXED ? Shape{2, 1, 1024} : Shape{1, 1, 1024};
}

std::vector<Shape> shape_candidates(int radius) {
    std::vector<Shape> v;
    const long long targets[] = {1024, 2048, 4096, 8192};
    if (radius != 6) {
        for (long long t : targets) v.push_back(Shape{2, 2, t});
        return v;
    }
    const int cd[][2] = {{1, 1}, {1, 2}, {2, 1}, {2, 2}, {4, 1}};
    for (auto &x : cd)
        for (long long t : targets) v.push_back(Shape{x[0], x[1], t});
    return v;
}

// A shape fixed by the environment (FSIC_STENCIL_CPT / _DEPTH / _BLOCKS), or
// the default when FSIC_AUTOTUNE=0; false: tune.
bool fixed_shape(int radius, int precision, Shape &sh) {
    const char *ec = getenv("FSIC_STENCIL_CPT"), *ed = getenv("FSIC_STENCIL_DEPTH");
    const char *eb = getenv("FSIC_STENCIL_BLOCKS"), *ea = getenv("FSIC_AUTOTUNE");
    sh = default_shape(radius, precision);
    if (!ec && !ed && !eb) return ea && atoi(ea) == 0;
    if (ec) {
        const int v = atoi(ec);
        if (v == 2 || (radius == 6 && (v == 1 || v == 4))) sh.cpt = v;
    }
    if (ed) {
        const int v = atoi(ed);
        if (radius == 6 && (v == 1 || (v == 2 && sh.cpt <= 2))) sh.depth = v;
    }
    if (sh.cpt == 4) sh.depth = 1;
    if (eb) sh.target = std::max(1LL, atoll(eb));
    return true;
}

// Time the CG sweep (k = 0, no convergence test) of every candidate shape on
// the batch's own buffers, in mixed precision plus half the FP64 residual
// pass (one per restart cycle of two sweeps), and keep the fastest.  The
// solve that follows rewrites everything these launches touch (q, the p.q
// and residual partials, the second x64 buffer and the activity counters).
template <typename T>
fsic_status time_shapes(fsic_ctx *c, const std::vector<Group> &groups, int precision,
                        const std::vector<Shape> &cands, Shape &best) {
    hipStream_t s = c->stream;
    Batch b0;
    build_batch(groups, c->radius, cands[0], b0);
    fsic_status st = prepare_batch(c, b0, precision);
    if (st) return st;
    const bool mixed = precision == FSIC_MIXED;
    const size_t F = (size_t)b0.fields;
    T *R = mixed ? (T *)(void *)c->R32.p : (T *)(void *)c->R.p;
    T *P = mixed ? (T *)(void *)c->P32a.p : (T *)(void *)c->P0.p;
    T *Q = mixed ? (T *)(void *)c->Q32.p : (T *)(void *)c->Q.p;
    HIPCHK(c, hipMemsetAsync(R, 0, F * sizeof(T), s));
    HIPCHK(c, hipMemsetAsync(P, 0, F * sizeof(T), s));
    const int norb = (int)b0.orb.size();
    HIPCHK(c, hipMemsetAsync(c->done.p, 0, norb * sizeof(int), s));
    HIPCHK(c, hipMemsetAsync(c->part8.p, 0, 2 * (size_t)b0.tot8 * sizeof(double), s));
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return set_err(c, FSIC_EHIP, "hipEventCreate failed");
    }
    float best_ms = 0.f;
    fsic_status res = FSIC_OK;
    for (const Shape &sh : cands) {
        Batch b;
        build_batch(groups, c->radius, sh, b);
        if ((res = upload(c, c->d_orb, b.orb))) break;
        if ((res = upload(c, c->d_items7, b.items7))) break;
        if (c->part7.ensure(3 * (size_t)b.tot7) != hipSuccess) { res = FSIC_ENOMEM; break; }
        Coeffs cf = c->cf;
        cf.cpt = sh.cpt;
        cf.depth = sh.depth;
        CGIter<T> a{};
        a.items7 = c->d_items7.p; a.nitems7 = (int)b.items7.size();
        a.orb = c->d_orb.p;
        a.R = R; a.P = P; a.Q = Q;
        a.part7 = c->part7.p; a.tot7 = b.tot7; a.part8 = c->part8.p; a.tot8 = b.tot8;
        a.partRU = c->partRU.p; a.done = c->done.p; a.iters = c->iters.p; a.rrfin = c->rrfin.p;
        a.bb = c->bb.p; a.nact = c->nact.p; a.norb = norb; a.tol2 = 0.0;
        hipError_t he = launch_cg_stencil<T>(c->radius, cf, a, 0, 0, 0, s);
        if (he == hipSuccess) he = hipEventRecord(e0, s);
        for (int r = 0; r < 3 && he == hipSuccess; ++r) he = launch_cg_stencil<T>(c->radius, cf, a, 0, 0, 0, s);
        if (he == hipSuccess) he = hipEventRecord(e1, s);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he == hipSuccess && mixed) {
            // the FP64 residual pass that closes each mixed restart cycle of
            // two FP32 sweeps (three operand arrays: its best shape differs);
            // it reads B and the FP32 field and writes scratch buffers the
            // solve rewrites before reading
            if (c->partRU.ensure((size_t)b.tot7) != hipSuccess || c->X64b.ensure(F) != hipSuccess) {
                res = FSIC_ENOMEM;
                break;
            }
            auto resid = [&]() {
                return launch_true_residual(c->radius, cf, c->d_items7.p, (int)b.items7.size(), c->d_orb.p,
                                            c->done.p, c->B.p, (const float *)(void *)R, c->B.p, c->X64b.p,
                                            (float *)(void *)Q, c->partRU.p, s);
            };
            he = resid();
            if (he == hipSuccess) he = hipEventRecord(e0, s);
            for (int r = 0; r < 3 && he == hipSuccess; ++r) he = resid();
            if (he == hipSuccess) he = hipEventRecord(e1, s);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            float mr = 0.f;
            if (he == hipSuccess) he = hipEventElapsedTime(&mr, e0, e1);
            ms += 0.5f * mr;
        }
        if (he != hipSuccess) { res = set_err(c, FSIC_EHIP, hipGetErrorString(he)); break; }
        if (&sh == &cands[0] || ms < best_ms) {
            best_ms = ms;
            best = sh;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return res;
}

// The stencil shape for a batch: fixed by the environment, else the fastest
// candidate for this (device, precision, order, grids), tuned once per
// process and then reused, so repeated calls are bitwise reproducible.
fsic_status choose_shape(fsic_ctx *c, const std::vector<Group> &groups, int precision, Shape &sh) {
    c->tune_ms = 0.0;
    if (fixed_shape(c->radius, precision, sh)) return FSIC_OK;
    std::string key = std::to_string(c->device) + ":" + std::to_string(precision) + ":" +
                      std::to_string(c->radius);
    for (const Group &g : groups)
        key += ":" + std::to_string(g.n[0]) + "x" + std::to_string(g.n[1]) + "x" +
               std::to_string(g.n[2]) + "*" + std::to_string(g.count);
    static std::mutex mu;
    static std::map<std::string, Shape> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto f = cache.find(key);
        if (f != cache.end()) {
            sh = f->second;
            return FSIC_OK;
        }
    }
    const double t0 = now_ms();
    const std::vector<Shape> cands = shape_candidates(c->radius);
    fsic_status st = precision == FSIC_MIXED ? time_shapes<float>(c, groups, precision, cands, sh)
                                             : time_shapes<double>(c, groups, precision, cands, sh);
    if (st) return st;
    c->tune_ms = now_ms() - t0;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = sh;
    return FSIC_OK;
}


// Time one preconditioner application of a candidate layout on the batch's
// own buffers (the solve that follows rewrites everything it touches):
// one application to warm up, then three timed ones.
fsic_status time_dst_layout(fsic_ctx *c, const std::vector<Group> &groups, int precision, const Shape &sh,
                            const DstTune &dt, hipEvent_t e0, hipEvent_t e1, float &ms) {
    hipStream_t s = c->stream;
    Batch b;
    build_batch(groups, c->radius, sh, b, dt);
    fsic_status st = prepare_batch(c, b, precision);
    if (st) return st;
    const bool mixed = precision == FSIC_MIXED;
    const size_t F = (size_t)b.fields;
    const int norb = (int)b.orb.size();
    HIPCHK(c, hipMemsetAsync(c->done.p, 0, norb * sizeof(int), s));
    // r = 0 and r.z partials of a nonzero pattern (beta finite): the transform
    // passes take the same time for any values
    if (mixed) HIPCHK(c, hipMemsetAsync(c->R32.p, 0, F * sizeof(float), s));
    else HIPCHK(c, hipMemsetAsync(c->R.p, 0, F * sizeof(double), s));
    HIPCHK(c, hipMemsetAsync(c->partRZ.p, 0x3f, 2 * (size_t)b.tot9 * sizeof(double), s));
    const DstItems di{c->d_dx.p, c->d_dy.p, c->d_dz.p, (int)b.dx.size(), (int)b.dy.size(),
                      (int)b.dz.size(), b.dst_fast, (b.max_n + 31) & ~31, dst_blocks(c),
                      b.dst_xy ? c->d_dxy.p : nullptr, b.dst_xy ? (int)b.dxy.size() : 0, b.dst_two ? 1 : 0,
                      b.dst_vec ? 1 : 0, b.npxy, b.dst_zocc2 ? 1 : 0, b.dst_xyocc2 ? 1 : 0, b.dst_pv ? 1 : 0};
    auto apply = [&]() -> hipError_t {
        if (mixed) {
            // the mixed solve's form: the inverse pass writes p = z + beta p_old
            const PcgOut po{c->P32a.p, c->partRZ.p, c->partRZ.p + b.tot9, 0, nullptr, 0};
            return launch_dst_pcg(di, c->d_orb.p, c->done.p, c->dtab.p, c->R32.p, c->T32.p, c->P32b.p,
                                  c->partRZ.p, po, nullptr, s);
        }
        return launch_dst_precond<double>(di, c->d_orb.p, c->done.p, c->dtab.p, c->R.p, c->T32.p, c->Z32.p,
                                          c->partRZ.p, nullptr, s);
    };
    hipError_t he = apply();
    if (he == hipSuccess) he = hipEventRecord(e0, s);
    for (int r = 0; r < 3 && he == hipSuccess; ++r) he = apply();
    if (he == hipSuccess) he = hipEventRecord(e1, s);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) return set_err(c, FSIC_EHIP, hipGetErrorString(he));
    return FSIC_OK;
}

// fsic_stats.precond_layout bits of a built batch: 1 fused x-y passes,
// 2 two fused-pass blocks per compute unit, 4 two-block z pass, 8 early
// p_old read, and the transform variant (1-3) times 16
int dst_layout_bits(const Batch &b) {
    const bool o2 = b.dst_xy && b.dst_vec && b.dst_xyocc2 && dst_xy_occ2(b.npxy, b.dst_two);
    return (b.dst_xy ? 1 : 0) | (o2 ? 2 : 0) | (b.dst_zocc2 ? 4 : 0) | (b.dst_xy && b.dst_pv ? 8 : 0) |
           16 * b.dst_fast;
}

// Preconditioner layout for a batch: the first call for a (device,
// precision, order, grid sizes and orbital counts) times every combination
// of the choices in DstTune that changes the launches on this batch and
// keeps the fastest for the process; FSIC_AUTOTUNE=0 keeps the defaults,
// FSIC_DST_XY=0 / FSIC_DST_PV=0 fix their choice.
fsic_status choose_dst(fsic_ctx *c, const std::vector<Group> &groups, int precision, const Shape &sh,
                       DstTune &dt) {
    dt = DstTune{};
    c->dst_tune_ms = 0.0;
    if (c->opts.solver != FSIC_PCG && c->opts.solver != FSIC_AAR) return FSIC_OK;
    if (const char *ea = getenv("FSIC_AUTOTUNE"))
        if (atoi(ea) == 0) return FSIC_OK;
    Batch b0;
    build_batch(groups, c->radius, sh, b0, dt);
    if (!b0.dst_fast) return FSIC_OK;  // solved without the preconditioner
    // which choices change anything here
    const bool can_xy = b0.dst_xy;
    const bool can_xyocc2 = can_xy && b0.dst_vec && dst_xy_occ2(b0.npxy, b0.dst_two);
    const bool can_zocc2 = b0.dst_zocc2;
    const bool can_pv = can_xy && b0.dst_pv && precision == FSIC_MIXED && c->opts.solver == FSIC_PCG;
    std::vector<DstTune> cands;
    for (int xy = can_xy ? 1 : 0; xy >= 0; --xy)
        for (int o2 = (xy && can_xyocc2) ? 1 : 0; o2 >= 0; --o2)
            for (int z2 = (xy && can_zocc2) ? 1 : 0; z2 >= 0; --z2)
                for (int pv = (xy && can_pv) ? 1 : 0; pv >= 0; --pv) {
                    DstTune t;
                    t.xy = xy; t.xyocc2 = o2; t.zocc2 = z2; t.pv = pv;
                    cands.push_back(t);
                }
    if (cands.size() <= 1) return FSIC_OK;
    std::string key = std::to_string(c->device) + ":" + std::to_string(precision) + ":" +
                      std::to_string(c->radius) + ":" + std::to_string(c->opts.solver);
    for (const char *ev : {"FSIC_DST_XY", "FSIC_DST_PV", "FSIC_DST_BLOCKS"}) {
        const char *e = getenv(ev);
        key += std::string(":") + (e ? e : "-");
    }
    for (const Group &g : groups)
        key += ":" + std::to_string(g.n[0]) + "x" + std::to_string(g.n[1]) + "x" +
               std::to_string(g.n[2]) + "*" + std::to_string(g.count);
    static std::mutex mu;
    static std::map<std::string, DstTune> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto f = cache.find(key);
        if (f != cache.end()) {
            dt = f->second;
            return FSIC_OK;
        }
    }
    const double t0 = now_ms();
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return set_err(c, FSIC_EHIP, "hipEventCreate failed");
    }
    float best = 0.f;
    fsic_status res = FSIC_OK;
    for (size_t i = 0; i < cands.size(); ++i) {
        float ms = 0.f;
        if ((res = time_dst_layout(c, groups, precision, sh, cands[i], e0, e1, ms))) break;
        if (i == 0 || ms < best) {
            best = ms;
            dt = cands[i];
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (res) return res;
    c->dst_tune_ms = now_ms() - t0;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = dt;
    return FSIC_OK;
}

// Solve -L x = scale * rho (+ boundary term) for every orbital of batch b.
//   src: densities (square = 0) or orbitals (square = 1), field layout of b;
//   with_bc: Dirichlet values from the multipole expansion (else zero);
//   X: solution (field layout of b).
// Key of a captured restart cycle: every kernel argument and launch shape
// of its launches, field by field (no struct bytes, so no padding enters).
struct GraphKey {
    std::vector<uint64_t> v;
    void add(const void *p) { v.push_back((uint64_t)(uintptr_t)p); }
    void add(long long x) { v.push_back((uint64_t)x); }
    void add(double x) {
        uint64_t u;
        std::memcpy(&u, &x, sizeof(u));
        v.push_back(u);
    }
};

// Enqueue `body` on stream s: directly, or (graphs) replay its graph,
// captured on the context's capture stream the first time `key` is seen.
template <class Body>
fsic_status run_captured(fsic_ctx *c, bool graphs, const GraphKey &key, Body &body, hipStream_t s) {
    if (!graphs) return body(s);
    auto f = c->graphs.find(key.v);
    if (f == c->graphs.end()) {
        if (c->graphs.size() >= 64) {  // bound the cache (buffers reallocated, other batches)
            for (auto &e : c->graphs) hipGraphExecDestroy(e.second);
            c->graphs.clear();
        }
        if (!c->cap_stream) HIPCHK(c, hipStreamCreate(&c->cap_stream));
        HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
        const fsic_status st = body(c->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (st) {
            if (g) hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return set_err(c, FSIC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (ei != hipSuccess) return set_err(c, FSIC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        f = c->graphs.emplace(key.v, ex).first;
        c->graph_captures += 1;
    }
    HIPCHK(c, hipGraphLaunch(f->second, s));
    return FSIC_OK;
}

fsic_status solve_batch(fsic_ctx *c, const Batch &b, const double *src, int square, double scale,
                        bool with_bc, double *X, int precision, double tol, int max_iter,
                        SolveReport &rep, const double *qlm_in = nullptr) {
    hipStream_t s = c->stream;
    const int norb = (int)b.orb.size();
    const int nlm = (c->opts.lmax + 1) * (c->opts.lmax + 1);
    const int nit7 = (int)b.items7.size(), nit8 = (int)b.items8.size();
    const bool mixed = precision == FSIC_MIXED;
    bool staged = false;  // statistics staged by the solve's own last launch
    if (with_bc) {
        // boundary values from the moments of the source, or (qlm_in) from
        // given moments (the unit-moment basis solves, src null)
        if (!qlm_in)
            HIPCHK(c, launch_harm_contract(0, c->opts.lmax, c->ht, c->cf, c->radius, c->d_orb.p, c->d_gcount.p,
                                           c->d_hcN.p, (int)b.hcN.size(), c->d_hchN.p, (int)b.hchN.size(),
                                           b.max_group, src, square, c->partH.p, c->Qlm.p, s));
        HIPCHK(c, launch_harm_expand(0, c->opts.lmax, c->ht, c->radius, c->d_orb.p, c->d_gcount.p, c->d_hcGx.p,
                                     (int)b.hcGx.size(), qlm_in ? qlm_in : c->Qlm.p, c->Gh.p, s));
        HIPCHK(c, launch_bterm(c->radius, c->cf, norb, c->d_orb.p, b.max_ghost / c->radius, c->Gh.p, s));
    }
    (void)nlm;
    // b, r0 = b, x64 = 0 (mixed), ||b||^2 partials in part8 slot 0
    HIPCHK(c, launch_rhs(c->radius, c->cf, c->d_items8.p, nit8, c->d_orb.p, src, square, scale,
                         with_bc ? c->Gh.p : nullptr, c->B.p, mixed ? nullptr : c->R.p,
                         mixed ? c->R32.p : nullptr,
                         // the mixed preconditioned solve starts x64 at 0 without storing it
                         (mixed && !use_pcg(c, b)) ? X : nullptr, c->part8.p, s));
    HIPCHK(c, launch_reduce_partials(norb, c->d_orb.p, c->part8.p, 0, c->bb.p, s));
    {
        // done = 0, iters = 0, rs_iter = -1 (no restart), activity counters 0
        const IntFills f{{c->done.p, c->iters.p, c->rs_iter.p, c->nact.p},
                         {norb, norb, norb, 6 * norb},
                         {0, 0, -1, 0},
                         4};
        HIPCHK(c, launch_fill_ints(f, s));
    }
    const double tol2 = tol * tol;
    const int chunk = 32;
    int k = 0;
    bool all_done = false;
    // profiling: one event pair per launch of every prof_every-th iteration,
    // recorded on the context's stream; nact[2 norb..] counts what those
    // launches did
    const bool prof = (c->opts.flags & FSIC_PROFILE) != 0;
    // preconditioned solves take a few iterations: sample every other one
    const int prof_every = use_pcg(c, b) ? 2 : profile_period();
    auto sampled = [&](int kk) { return prof && kk % prof_every == prof_every - 1; };
    int *const nsamp = c->nact.p + 2 * norb;  // sampled sweeps, updates, preconditioner passes
    std::vector<ProfRec> &recs = c->recs;
    recs.clear();
    size_t evn = 0;
    auto ev_pair = [&](hipEvent_t &a, hipEvent_t &b) -> hipError_t {
        while (c->ev.size() < evn + 2) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            c->ev.push_back(e);
        }
        a = c->ev[evn];
        b = c->ev[evn + 1];
        evn += 2;
        return hipSuccess;
    };
#define PROF_BEGIN(kind_, k_, flag_)                                   \
    hipEvent_t _ea = nullptr, _eb = nullptr;                            \
    const bool _sp = sampled(k_);                                       \
    a.nsamp = _sp ? nsamp : nullptr;                                    \
    if (_sp) {                                                          \
        HIPCHK(c, ev_pair(_ea, _eb));                                   \
        HIPCHK(c, hipEventRecord(_ea, s));                              \
        recs.push_back(ProfRec{kind_, k_, flag_, _ea, _eb});                \
    }
#define PROF_END() \
    if (_sp) HIPCHK(c, hipEventRecord(_eb, s));
    const bool pcg = use_pcg(c, b);
    const bool graphs = (c->opts.flags & FSIC_GRAPHS) && !prof;
    DstItems di{c->d_dx.p, c->d_dy.p, c->d_dz.p, (int)b.dx.size(), (int)b.dy.size(),
                (int)b.dz.size(), b.dst_fast, (b.max_n + 31) & ~31, dst_blocks(c),
                b.dst_xy ? c->d_dxy.p : nullptr, b.dst_xy ? (int)b.dxy.size() : 0, b.dst_two ? 1 : 0,
                b.dst_vec ? 1 : 0, b.npxy, b.dst_zocc2 ? 1 : 0, b.dst_xyocc2 ? 1 : 0, b.dst_pv ? 1 : 0};
    if (pcg && !mixed) {
        // FP64 CG preconditioned by the FP32 sine-transform inverse.  The host
        // enqueues two iterations at a time and then reads the converged-
        // orbital counter of the pair before (one pair stays in flight), so
        // the device never waits for the host and at most one pair of
        // launches finds every orbital converged.
        CGIter<double> a{};
        a.items7 = c->d_items7.p; a.nitems7 = nit7;
        a.items8 = c->d_items8.p; a.nitems8 = nit8;
        a.orb = c->d_orb.p;
        a.R = c->R.p; a.Q = c->Q.p; a.X = X; a.Z = c->Z32.p;
        a.part7 = c->part7.p; a.part8 = c->part8.p; a.partRU = c->partRU.p; a.partRZ = c->partRZ.p;
        a.tot7 = b.tot7; a.tot8 = b.tot8; a.tot9 = b.tot9;
        a.done = c->done.p; a.iters = c->iters.p; a.rrfin = c->rrfin.p; a.bb = c->bb.p;
        a.rs_iter = nullptr; a.nact = c->nact.p; a.norb = norb; a.ndone = c->ndone.p;
        a.tol2 = tol2;
        const CGIter<double> a0 = a;
        HIPCHK(c, hipMemsetAsync(c->ndone.p, 0, sizeof(int), s));
        HIPCHK(c, launch_dst_precond<double>(di, c->d_orb.p, c->done.p, c->dtab.p, a.R, c->T32.p,
                                             a.Z, a.partRZ, nullptr, s));
        const int pair = 2;
        const int npairs = (max_iter + 1 + pair - 1) / pair;
        auto issue = [&](int j) -> fsic_status {
            CGIter<double> a = a0;
            const int kend = std::min((j + 1) * pair, max_iter + 1);
            for (int k = j * pair; k < kend; ++k) {
                a.P = (k & 1) ? c->P1.p : c->P0.p;
                a.Pold = (k & 1) ? c->P0.p : c->P1.p;
                {
                    PROF_BEGIN(0, k, k == 0)
                    HIPCHK(c, launch_pcg_stencil<double>(c->radius, c->cf, a, k, 0, 0, 0, s));
                    PROF_END()
                }
                if (k < max_iter) {
                    {
                        PROF_BEGIN(1, k, k == 0)
                        HIPCHK(c, launch_pcg_update<double>(a, k, k == 0, s));
                        PROF_END()
                    }
                    PROF_BEGIN(2, k + 1, 0)  // z of iteration k + 1
                    HIPCHK(c, launch_dst_precond<double>(di, c->d_orb.p, c->done.p, c->dtab.p, a.R,
                                                         c->T32.p, a.Z,
                                                         a.partRZ + (size_t)((k + 1) & 1) * b.tot9,
                                                         _sp ? nsamp + 2 * norb : nullptr, s));
                    PROF_END()
                }
            }
            HIPCHK(c, hipMemcpyAsync(c->h_nd + (j & 1), c->ndone.p, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipEventRecord(c->evc[j & 1], s));
            return FSIC_OK;
        };
        fsic_status ist = issue(0);
        if (ist) return ist;
        for (int j = 0;; ++j) {
            const bool more = j + 1 < npairs;
            if (more && (ist = issue(j + 1))) return ist;
            HIPCHK(c, hipEventSynchronize(c->evc[j & 1]));
            if (c->h_nd[j & 1] >= norb || !more || status_error(c)) break;
        }
        HIPCHK(c, launch_true_residual(c->radius, c->cf, c->d_items7.p, nit7, c->d_orb.p, nullptr,
                                       X, nullptr, c->B.p, nullptr, nullptr, c->partRU.p, s));
        HIPCHK(c, launch_reduce_partials(norb, c->d_orb.p, c->partRU.p, 1, c->ptrue.p, s));
    } else if (use_aar(c, b)) {
        // alternating Anderson-Richardson: FP64 iterate and residual, FP32
        // preconditioned residual f = M^{-1} r
        AarBufs aa{c->d_items8.p, c->d_orb.p, c->done.p, c->Z32.p, c->Fprev.p, c->Fh.p, c->Xh.p, X,
                   c->aar_gamma.p, c->partD.p, b.fields, kAarM};
        HIPCHK(c, hipMemsetAsync(X, 0, (size_t)b.fields * sizeof(double), s));
        for (; k <= max_iter && !all_done; ++k) {
            HIPCHK(c, launch_true_residual(c->radius, c->cf, c->d_items7.p, nit7, c->d_orb.p, c->done.p,
                                           X, nullptr, c->B.p, nullptr, c->R32.p, c->partRU.p, s));
            HIPCHK(c, launch_ru_check(norb, c->d_orb.p, c->partRU.p, c->bb.p, tol2, k, c->done.p,
                                      c->iters.p, c->rrfin.p, c->rs_iter.p, nullptr, nullptr, 0, nullptr, 0, s));
            if (k % kAarCheck == kAarCheck - 1 || k == max_iter) {
                HIPCHK(c, hipMemcpyAsync(c->h_done, c->done.p, norb * sizeof(int), hipMemcpyDeviceToHost, s));
                HIPCHK(c, hipStreamSynchronize(s));
                all_done = true;
                for (int o = 0; o < norb; ++o) all_done = all_done && c->h_done[o] == 1;
                if (all_done || k == max_iter || status_error(c)) break;
            }
            HIPCHK(c, launch_dst_precond<float>(di, c->d_orb.p, c->done.p, c->dtab.p, c->R32.p, c->T32.p,
                                                c->Z32.p, c->partRZ.p, nullptr, s));
            const int nh = std::min(k, kAarM);  // history columns after this iteration's f difference
            if ((k + 1) % kAarPeriod == 0 && nh > 0) {
                HIPCHK(c, launch_aar_dots(aa, nit8, k, nh, 1, 1, s));
                HIPCHK(c, launch_aar_solve(aa, norb, nh, s));
                HIPCHK(c, launch_aar_step(aa, nit8, k, nh, kAarOmega, kAarBeta, true, 0, s));
            } else {
                HIPCHK(c, launch_aar_step(aa, nit8, k, nh, kAarOmega, kAarBeta, false, k > 0 ? 1 : 2, s));
            }
        }
        HIPCHK(c, launch_true_residual(c->radius, c->cf, c->d_items7.p, nit7, c->d_orb.p, nullptr,
                                       X, nullptr, c->B.p, nullptr, nullptr, c->partRU.p, s));
        HIPCHK(c, launch_reduce_partials(norb, c->d_orb.p, c->partRU.p, 1, c->ptrue.p, s));
    } else if (pcg) {
        // FP32 preconditioned CG in restart cycles of `cyc` iterations, each
        // closed by the FP64 residual of x64 plus the cycle's steps (defect
        // correction).  Per iteration: the preconditioner's last pass forms
        // p_k = z_k + beta p_{k-1}, the sweep q_k = -L p_k, and (between
        // iterations) r -= alpha q; the last two steps of a cycle go straight
        // into the residual pass, x32 holds the earlier ones (cycles of three
        // or more).  x64 lives in two buffers: cycle j reads xs[j & 1] and
        // writes xs[(j + 1) & 1]; an orbital's final x is in the buffer of the
        // cycle that converged it (fin).  Convergence is decided on the FP64
        // residual only.
        CGIter<float> a{};
        a.items7 = c->d_items7.p; a.nitems7 = nit7;
        a.items8 = c->d_items8.p; a.nitems8 = nit8;
        a.orb = c->d_orb.p;
        a.R = c->R32.p; a.Q = c->Q32.p; a.X = c->X32.p; a.Z = nullptr; a.B64 = c->B.p;
        a.part7 = c->part7.p; a.part8 = c->part8.p; a.partRU = c->partRU.p; a.partRZ = c->partRZ.p;
        a.tot7 = b.tot7; a.tot8 = b.tot8; a.tot9 = b.tot9;
        a.done = c->done.p; a.iters = c->iters.p; a.rrfin = c->rrfin.p; a.bb = c->bb.p;
        a.rs_iter = nullptr; a.nact = c->nact.p; a.norb = norb; a.ndone = c->ndone.p;
        a.tol2 = tol2;
        const CGIter<float> a0 = a;
        // the first cycle (from x = 0) runs cyc0 iterations, the others cyc
        const int cyc = std::max(2, pcg_chunk(b.dst_fast));
        const int cyc0 = std::max(2, pcg_first_chunk(b.dst_fast));
        const int cycmax = std::max(cyc, cyc0);
        const int ncyc = 1 + std::max(0, (max_iter - cyc0) / cyc);
        HIPCHK(c, c->X64b.ensure((size_t)b.fields));
        if (cycmax > 2) HIPCHK(c, c->X32.ensure((size_t)b.fields));
        double *const xs[2] = {X, c->X64b.p};
        float *const P2[2] = {c->P32a.p, c->P32b.p};
        {
            // converged count 0, no final x buffer yet (-1), no pause
            const IntFills f{{c->ndone.p, c->fin.p, c->pz.p}, {1, norb, norb}, {0, -1, cycmax}, 3};
            HIPCHK(c, launch_fill_ints(f, s));
        }
        // an orbital whose FP32 recursion has reached half the tolerance
        // pauses for the rest of its cycle (its residual pass decides)
        const double ftol2 = 0.25 * tol2;
        // cycle variant v: 0 the first (x64 = 0), 1 odd, 2 even (>= 2); the
        // launches depend on v only (iteration indices enter by parity)
        auto cycle = [&](hipStream_t s, int v) -> fsic_status {
            CGIter<float> a = a0;
            const int L = v == 0 ? cyc0 : cyc;  // iterations of this cycle
            // parity of the cycle's first iteration: cycle j >= 1 starts at
            // iteration cyc0 + (j - 1) cyc
            const int ks = v == 0 ? 0 : (v == 1 ? cyc0 & 1 : (cyc0 + cyc) & 1);
            double *const Xc = v == 0 ? nullptr : xs[v == 1 ? 1 : 0];
            double *const Xn = xs[v == 1 ? 0 : 1];
            const bool samp = prof && v != 0;
            for (int i = 0; i < L; ++i) {
                const int k = ks + i;
                const bool last = i == L - 1;
                PcgOut po{nullptr, a.partRZ + (size_t)(k & 1) * b.tot9,
                          a.partRZ + (size_t)((k + 1) & 1) * b.tot9, 1, c->pz.p, i};
                if (i > 0) {
                    const int m = i - 1;  // x32 takes the steps of iterations 0 .. L - 3
                    const int xmode = m <= L - 3 ? (m == 0 ? 1 : 2) : 0;
                    a.P = P2[(k - 1) & 1];
                    {
                        PROF_BEGIN(1, last && samp ? 1 : 0, 0)
                        HIPCHK(c, launch_pcg_rupdate(a, k - 1, xmode, c->pz.p, i, s));
                        PROF_END()
                    }
                    HIPCHK(c, launch_pause_check(a, k - 1, ftol2, c->pz.p, i, s));
                    po.pold = P2[(k - 1) & 1];
                    po.first = 0;
                }
                {
                    PROF_BEGIN(2, last && samp ? 1 : 0, 0)
                    HIPCHK(c, launch_dst_pcg(di, c->d_orb.p, c->done.p, c->dtab.p, a.R, c->T32.p,
                                             P2[k & 1], a.partRZ + (size_t)(k & 1) * b.tot9, po,
                                             _sp ? nsamp + 2 * norb : nullptr, s));
                    PROF_END()
                }
                a.P = P2[k & 1];
                {
                    PROF_BEGIN(0, last && samp ? 1 : 0, 0)
                    HIPCHK(c, launch_pcg_sweep(c->radius, c->cf, a, k, c->pz.p, i, s));
                    PROF_END()
                }
            }
            const int ka = ks + L - 2, kb = ks + L - 1;
            ResStep rs{Xc, L > 2 ? c->X32.p : nullptr, P2[ka & 1], P2[kb & 1], ka, kb, Xn, c->R32.p,
                       c->pz.p, L - 2, L - 1};
            {
                PROF_BEGIN(3, samp ? 1 : 0, 0)
                HIPCHK(c, launch_res_steps(c->radius, c->cf, a, rs, s));
                PROF_END()
            }
            HIPCHK(c, launch_ru_check(norb, c->d_orb.p, c->partRU.p, c->bb.p, tol2, 0, c->done.p,
                                      c->iters.p, c->rrfin.p, nullptr, c->ndone.p, c->fin.p,
                                      Xn == xs[1] ? 1 : 0, c->pz.p, cycmax, s));
            return FSIC_OK;
        };
        auto issue = [&](int j) -> fsic_status {
            const int v = j == 0 ? 0 : ((j & 1) ? 1 : 2);
            auto body = [&](hipStream_t ss) { return cycle(ss, v); };
            GraphKey key;
            if (graphs) {
                key.add((long long)v);
                key.add((long long)cyc);
                key.add((long long)cyc0);
                key.add((long long)c->radius);
                key.add((long long)c->cf.cpt);
                key.add((long long)c->cf.depth);
                for (int q = 0; q <= kMaxRadius; ++q) key.add(c->cf.c[q]);
                key.add(tol2);
                for (const void *ptr : {(const void *)a0.items7, (const void *)a0.items8, (const void *)a0.orb,
                                        (const void *)a0.R, (const void *)a0.Q, (const void *)a0.X,
                                        (const void *)a0.B64, (const void *)a0.part7, (const void *)a0.part8,
                                        (const void *)a0.partRU, (const void *)a0.partRZ,
                                        (const void *)a0.done, (const void *)a0.iters, (const void *)a0.rrfin,
                                        (const void *)a0.bb, (const void *)a0.nact, (const void *)a0.ndone,
                                        (const void *)c->fin.p, (const void *)c->pz.p,
                                        (const void *)xs[0], (const void *)xs[1],
                                        (const void *)P2[0], (const void *)P2[1], (const void *)c->T32.p,
                                        (const void *)c->dtab.p, (const void *)di.x, (const void *)di.y,
                                        (const void *)di.z, (const void *)di.xy})
                    key.add(ptr);
                for (long long q : {(long long)a0.nitems7, (long long)a0.nitems8, (long long)a0.tot7,
                                    (long long)a0.tot8, (long long)a0.tot9, (long long)a0.norb,
                                    (long long)di.nx, (long long)di.ny, (long long)di.nz, (long long)di.fast,
                                    (long long)di.np, (long long)di.blocks, (long long)di.nxy,
                                    (long long)di.two, (long long)di.xyvec, (long long)di.npxy,
                                    (long long)di.zocc2})
                    key.add(q);
            }
            fsic_status st = run_captured(c, graphs, key, body, s);
            if (st) return st;
            HIPCHK(c, hipMemcpyAsync(c->h_nd + (j & 1), c->ndone.p, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipEventRecord(c->evc[j & 1], s));
            return FSIC_OK;
        };
        // one cycle stays in flight while the host reads the counter of the
        // one before; the first pred_cycles - 1 cycles (the last solve's
        // count) are not checked at all, and the cycle the last solve ended
        // with is checked before another is issued (a solve like the last
        // one then runs no cycle beyond its last)
        int used = 0, issued = 1;
        fsic_status ist = issue(0);
        if (ist) return ist;
        for (int j = 0;; ++j) {
            const bool more = j + 1 < ncyc;
            const bool hold = j + 1 == c->pred_cycles;
            if (more && !hold && issued == j + 1) {
                if ((ist = issue(j + 1))) return ist;
                issued = j + 2;
            }
            if (more && j + 1 < c->pred_cycles) continue;
            HIPCHK(c, hipEventSynchronize(c->evc[j & 1]));
            if (c->h_nd[j & 1] >= norb || !more || status_error(c)) {
                used = j + 1;
                break;
            }
            if (issued == j + 1) {
                if ((ist = issue(j + 1))) return ist;
                issued = j + 2;
            }
        }
        c->pred_cycles = used;
        rep.refinements += used;
        // move x from the second buffer where the converging cycle left it
        // there; an unconverged orbital's latest x is where the last cycle
        // that ran wrote it (cycle j writes buffer (j + 1) & 1; cycles up to
        // `issued` - 1 ran)
        // ... in one launch with the per-orbital end: iterations that did
        // work (the restart cycles report no index), the final FP64 residual
        // (the residual pass of the cycle that produced each orbital's x left
        // its partial sums in partRU; later cycles skip it) and the
        // statistics stage
        HIPCHK(c, c->d_stage.ensure(6 * (size_t)std::max(norb, 1)));
        HIPCHK(c, launch_mixed_finish(nit8, c->d_items8.p, c->d_orb.p, c->fin.p, (issued & 1) ? 1 : 0, X,
                                      c->X64b.p, norb, c->partRU.p, c->nact.p, c->done.p, c->bb.p, c->iters.p,
                                      c->ptrue.p, c->d_stage.p, s));
        staged = true;
    } else if (!mixed) {
        CGIter<double> a{};
        a.items7 = c->d_items7.p; a.nitems7 = nit7;
        a.items8 = c->d_items8.p; a.nitems8 = nit8;
        a.orb = c->d_orb.p;
        a.R = c->R.p; a.Q = c->Q.p; a.X = X;
        a.P = c->P0.p;
        a.part7 = c->part7.p; a.part8 = c->part8.p; a.partRU = c->partRU.p;
        a.tot7 = b.tot7; a.tot8 = b.tot8;
        a.done = c->done.p; a.iters = c->iters.p; a.rrfin = c->rrfin.p; a.bb = c->bb.p;
        a.rs_iter = nullptr; a.nact = c->nact.p; a.norb = norb;
        a.tol2 = tol2;
        while (k < max_iter + 1 && !all_done) {
            const int kend = std::min(k + chunk, max_iter + 1);
            for (; k < kend; ++k) {
                {
                    PROF_BEGIN(0, k, k == 0)
                    HIPCHK(c, launch_cg_stencil<double>(c->radius, c->cf, a, k, 0, 1, s));
                    PROF_END()
                }
                if (k < max_iter) {
                    PROF_BEGIN(1, k, k == 0)
                    HIPCHK(c, launch_cg_update<double>(a, k, 0, k == 0, s));
                    PROF_END()
                }
            }
            HIPCHK(c, hipMemcpyAsync(c->h_done, c->done.p, norb * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
            all_done = true;
            for (int o = 0; o < norb; ++o) all_done = all_done && c->h_done[o];
            if (status_error(c)) break;
        }
        // true FP64 residual of the final iterate
        HIPCHK(c, launch_true_residual(c->radius, c->cf, c->d_items7.p, nit7, c->d_orb.p, nullptr,
                                       X, nullptr, c->B.p, nullptr, nullptr, c->partRU.p, s));
        HIPCHK(c, launch_reduce_partials(norb, c->d_orb.p, c->partRU.p, 1, c->ptrue.p, s));
    } else {
        CGIter<float> a{};
        a.items7 = c->d_items7.p; a.nitems7 = nit7;
        a.items8 = c->d_items8.p; a.nitems8 = nit8;
        a.orb = c->d_orb.p;
        a.R = c->R32.p; a.Q = c->Q32.p; a.X = c->X32.p;
        a.P = c->P32a.p;
        a.part7 = c->part7.p; a.part8 = c->part8.p; a.partRU = c->partRU.p;
        a.tot7 = b.tot7; a.tot8 = b.tot8;
        a.done = c->done.p; a.iters = c->iters.p; a.rrfin = c->rrfin.p; a.bb = c->bb.p;
        a.rs_iter = c->rs_iter.p; a.nact = c->nact.p; a.norb = norb;
        a.tol2 = tol2;
        int nref = 0;
        while (k < max_iter && !all_done) {
            const int kstart = k;
            const int kend = std::min(k + chunk, max_iter);
            for (; k < kend; ++k) {
                const int j = k - kstart;
                const int cur_ru = (j == 0 && k > 0);
                {
                    PROF_BEGIN(0, k, k == 0)
                    HIPCHK(c, launch_cg_stencil<float>(c->radius, c->cf, a, k, cur_ru, 1, s));
                    PROF_END()
                }
                {
                    PROF_BEGIN(1, k, j == 0)
                    HIPCHK(c, launch_cg_update<float>(a, k, cur_ru, j == 0, s));
                    PROF_END()
                }
            }
            // reliable update: FP64 residual of x64 + x32, then x64 += x32
            HIPCHK(c, launch_true_residual(c->radius, c->cf, c->d_items7.p, nit7, c->d_orb.p,
                                           c->done.p, X, c->X32.p, c->B.p, nullptr, c->R32.p,
                                           c->partRU.p, s));
            HIPCHK(c, launch_mixed_accumulate(nit8, c->d_items8.p, c->d_orb.p, c->done.p, X, c->X32.p, s));
            HIPCHK(c, launch_ru_check(norb, c->d_orb.p, c->partRU.p, c->bb.p, tol2, k, c->done.p,
                                      c->iters.p, c->rrfin.p, c->rs_iter.p, nullptr, nullptr, 0, nullptr, 0, s));
            ++nref;
            HIPCHK(c, hipMemcpyAsync(c->h_done, c->done.p, norb * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
            all_done = true;
            for (int o = 0; o < norb; ++o) all_done = all_done && c->h_done[o] == 1;
            if (status_error(c)) break;
        }
        rep.refinements += nref;
        // final report: FP64 residual of x64 (x32 already folded in)
        HIPCHK(c, launch_true_residual(c->radius, c->cf, c->d_items7.p, nit7, c->d_orb.p, nullptr,
                                       X, nullptr, c->B.p, nullptr, nullptr, c->partRU.p, s));
        HIPCHK(c, launch_reduce_partials(norb, c->d_orb.p, c->partRU.p, 1, c->ptrue.p, s));
    }
    // statistics: copied now, read by finish_solve after the caller's sync
    HIPCHK(c, c->d_stage.ensure(6 * (size_t)std::max(norb, 1)));
    if (!staged)
        HIPCHK(c, launch_stage_stats(norb, c->iters.p, c->nact.p, c->done.p, c->ptrue.p, c->bb.p, c->d_stage.p, s));
    HIPCHK(c, hipMemcpyAsync(c->h_stage, c->d_stage.p, 6 * (size_t)norb * sizeof(double), hipMemcpyDeviceToHost, s));
    c->h_si = reinterpret_cast<int *>(c->h_stage);
    c->h_sd = c->h_stage + 4 * (size_t)norb;
    c->pend_prof = prof;
    c->pend_aar = use_aar(c, b);
    c->pend_pcg = pcg;
    c->pend_mixed = mixed;
    c->pend_dst_xy = b.dst_xy;
    c->pend_dst_fast = b.dst_fast;
#undef PROF_BEGIN
#undef PROF_END
    return FSIC_OK;
}

// Read the statistics of the last solve_batch (the caller has synchronised
// the context's stream since) into rep, and the sampled launch times.
fsic_status finish_solve(fsic_ctx *c, const Batch &b, SolveReport &rep) {
    const int norb = (int)b.orb.size();
    const int *it = c->h_si, *na = c->h_si + norb;
    const double *pt = c->h_sd, *bbh = c->h_sd + norb;
    const bool prof = c->pend_prof, pcg = c->pend_pcg, mixed = c->pend_mixed;
    for (int o = 0; o < norb; ++o) {
        // stencil sweeps that did work for this orbital (AAR: residual
        // evaluations before convergence)
        const int itv = c->pend_aar ? it[o] : na[o];
        rep.max_iters = std::max(rep.max_iters, itv);
        rep.total_iters += itv;
        const double rr = bbh[o] > 0 ? std::sqrt(pt[o] / bbh[o]) : 0.0;
        rep.max_relres = std::max(rep.max_relres, rr);
        if (it[7 * norb + o] != 1) rep.converged = false;  // done
    }
    if (prof) {
        // algorithmic bytes of the sampled launches: each array of each
        // orbital that did work in a launch, read or written once (sweep: p,
        // r read, q written; update: x, p, r, q read, x, r, p written).
        // Sampled launches are never the first of a solve or of a restart of
        // x from zero.
        const double esz = mixed ? 4.0 : 8.0;
        for (const ProfRec &r : c->recs) {
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, r.a, r.b));
            if (r.kind == 0) { c->sweep_launches += 1; c->sweep_ms += ms; }
            else if (r.kind == 1) { c->update_launches += 1; c->update_ms += ms; }
            else if (r.kind == 2) { c->precond_launches += 1; c->precond_ms += ms; }
            else { c->resid_launches += 1; c->resid_ms += ms; }
        }
        // preconditioned CG: sweep reads z (float) and p_old, writes p, q;
        // update reads x, p, r, q, writes x, r; the preconditioner reads r
        // and passes the float work array through its transform passes (each
        // reads and writes it once) until the last writes z: three passes
        // with the in-plane pair fused (r.z from the spectral coefficients of
        // the z pass), else five, the last reading r again for r.z; its flops
        // are 2 n per value per transform along an axis of n nodes
        for (int o = 0; o < norb; ++o) {
            const OrbDesc &od = b.orb[o];
            const double Mo = (double)od.nx * od.ny * od.nz;
            const double ns = na[2 * (size_t)norb + o], nu = na[3 * (size_t)norb + o];
            if (pcg && mixed) {
                // restart cycles (sampled: the last iteration of every cycle
                // but the first, and its residual pass): the sweep reads p and
                // writes q; the update reads r, q and writes r; the
                // preconditioner reads r, passes the work array through its
                // passes and its last pass reads p_old and writes p; the
                // residual pass reads x64, b, the last two p (and x32) and
                // writes x64 and r (FP64, FP64, FP32)
                const double npc = na[4 * (size_t)norb + o], nr = na[5 * (size_t)norb + o];
                const int cyc = std::max(2, pcg_chunk(c->pend_dst_fast));
                c->sweep_bytes += Mo * 8.0 * ns;
                c->update_bytes += Mo * 12.0 * nu;
                c->precond_bytes += Mo * (c->pend_dst_xy ? 28.0 : 44.0) * npc;
                c->precond_flops += Mo * 4.0 * (od.nx + od.ny + od.nz) * npc;
                c->resid_bytes += Mo * (36.0 + (cyc > 2 ? 4.0 : 0.0)) * nr;
            } else if (pcg) {
                const double npc = na[4 * (size_t)norb + o];
                c->sweep_bytes += Mo * (4.0 + 3.0 * esz) * ns;
                c->update_bytes += Mo * esz * 6.0 * nu;
                c->precond_bytes += Mo * (c->pend_dst_xy ? 20.0 + esz : 36.0 + esz) * npc;
                c->precond_flops += Mo * 4.0 * (od.nx + od.ny + od.nz) * npc;
            } else {
                c->sweep_bytes += Mo * esz * 3.0 * ns;
                c->update_bytes += Mo * esz * 7.0 * nu;
            }
        }
    }
    return FSIC_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

fsic_status fsic_default_opts(fsic_opts *o) {
    if (!o) return FSIC_EINVAL;
    o->fd_order = 12;
    o->lmax = 6;
    o->solver = FSIC_PCG;
    o->precision = FSIC_FP64;
    o->tol = 1e-10;
    o->max_iter = 20000;
    o->vsic_scale = 1.0;
    o->rho_floor = 1e-30;
    o->s_eig_floor = 1e-12;
    o->flags = FSIC_WANT_VSIC;
    return FSIC_OK;
}

const char *fsic_status_string(fsic_status s) {
    switch (s) {
        case FSIC_OK: return "ok";
        case FSIC_EINVAL: return "invalid argument";
        case FSIC_ENOMEM: return "out of memory";
        case FSIC_EHIP: return "HIP runtime error";
        case FSIC_ENONORTHO: return "input orbitals are not orthonormal on the grid";
        case FSIC_EVACUUM: return "FOD in vacuum: rho(a_i) <= rho_floor";
        case FSIC_EBOUNDARY: return "FOD interpolation stencil leaves the grid";
        case FSIC_ESINGULAR: return "Fermi-orbital overlap is singular";
        case FSIC_ENOCONV: return "Poisson solve did not converge";
        case FSIC_ENOTAPE: return "no forward tape for backward";
    }
    return "unknown status";
}

const char *fsic_last_error(const fsic_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// Stencil weights for a radius, with the default tile of 32 x 16 columns.
static void set_stencil_defaults(fsic_ctx *c, int radius) {
    c->radius = radius;
    c->cf = fd_weights(radius);
    c->cf.cpt = 2;
    c->cf.depth = (radius == 6) ? 1 : 2;
}

fsic_status fsic_create(fsic_ctx **ctx, const fsic_opts *opts, void *hip_stream) {
    if (!ctx) return FSIC_EINVAL;
    *ctx = nullptr;
    std::string why;
    fsic_status st = validate_opts(opts, why);
    if (st) return st;
    fsic_ctx *c = new (std::nothrow) fsic_ctx();
    if (!c) return FSIC_ENOMEM;
    c->opts = *opts;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return FSIC_EHIP; }
    set_stencil_defaults(c, opts->fd_order / 2);
    c->ht = harm_tables(opts->lmax);
    if (c->status.ensure(1) != hipSuccess) { delete c; return FSIC_ENOMEM; }
    *ctx = c;
    return FSIC_OK;
}

fsic_status fsic_set_opts(fsic_ctx *c, const fsic_opts *opts) {
    if (!c) return FSIC_EINVAL;
    std::string why;
    fsic_status st = validate_opts(opts, why);
    if (st) return set_err(c, st, why);
    c->opts = *opts;
    set_stencil_defaults(c, opts->fd_order / 2);
    c->ht = harm_tables(opts->lmax);
    c->tape = false;
    return FSIC_OK;
}

void fsic_destroy(fsic_ctx *c) {
    if (!c) return;
    hipStreamSynchronize(c->stream);
    for (auto &kv : c->bbasis) kv.second.release();
    c->bbasis.clear();
    c->qident.release();
    c->PHI.release(); c->V.release(); c->W.release(); c->B.release(); c->R.release();
    c->P0.release(); c->P1.release(); c->Q.release(); c->X64b.release();
    c->R32.release(); c->P32a.release(); c->P32b.release(); c->Q32.release(); c->X32.release();
    c->Z32.release(); c->T32.release(); c->dtab.release(); c->partRZ.release();
    c->Fprev.release(); c->Fh.release(); c->Xh.release(); c->aar_gamma.release(); c->partD.release();
    c->d_dx.release(); c->d_dy.release(); c->d_dz.release(); c->d_dxy.release();
    c->Gh.release(); c->part7.release(); c->part8.release(); c->partRU.release();
    c->partH.release(); c->d_hcN.release(); c->d_hcG.release(); c->d_hcNx.release(); c->d_hcGx.release(); c->d_hchN.release(); c->d_hchG.release();
    c->bb.release(); c->rrfin.release();
    c->relres.release(); c->Qlm.release(); c->Zt.release(); c->ptrue.release(); c->d_stage.release(); c->d_chk.release(); c->d_grad.release();
    c->done.release(); c->iters.release(); c->rs_iter.release(); c->nact.release(); c->d_orb.release(); c->d_items7.release();
    c->d_items8.release(); c->d_gcount.release(); c->small.release(); c->work.release();
    c->partG.release(); c->d_cells.release(); c->d_chan.release(); c->d_blkchan.release();
    c->partU.release(); c->partX.release(); c->eux.release();
    c->status.release(); c->bmat.release();
    for (hipEvent_t e : c->ev) hipEventDestroy(e);
    for (auto &g : c->graphs) hipGraphExecDestroy(g.second);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    if (c->h_done) hipHostFree(c->h_done);
    if (c->h_nd) hipHostFree(c->h_nd);
    if (c->h_stage) hipHostFree(c->h_stage);
    if (c->h_stat) hipHostFree(c->h_stat);
    if (c->h_chk) hipHostFree(c->h_chk);
    if (c->h_eux) hipHostFree(c->h_eux);
    if (c->h_grad) hipHostFree(c->h_grad);
    for (hipEvent_t e : c->evc)
        if (e) hipEventDestroy(e);
    c->ndone.release(); c->fin.release(); c->pz.release();
    delete c;
}

// The unit-moment boundary solutions U_q (q < (lmax + 1)^2) of a grid:
// K U_q = the boundary term of the ghost values of moment vector e_q (no
// source), solved in FP64 to relative residual 1e-13 with the batch's stencil
// shape and preconditioner layout, once per grid for the context.  Since the
// map from moments to ghost values to right-hand side is linear, the
// multipole-boundary solution of any source is its zero-boundary solution
// plus sum_q Q_q U_q.  Uses the context's solve buffers (the caller prepares
// its own batch afterwards).
static fsic_status boundary_basis(fsic_ctx *c, const Chan &ch, const Shape &sh, const DstTune &dt,
                                  const double **U) {
    const int lmax = c->opts.lmax, nlm = (lmax + 1) * (lmax + 1);
    long long hb = 0;
    std::memcpy(&hb, &ch.h, sizeof(hb));
    const std::array<long long, 6> key{ch.n[0], ch.n[1], ch.n[2], hb, lmax, c->radius};
    auto f = c->bbasis.find(key);
    if (f != c->bbasis.end()) {
        *U = f->second.p;
        return FSIC_OK;
    }
    const double t0 = now_ms();
    Group g{};
    for (int d = 0; d < 3; ++d) { g.n[d] = ch.n[d]; g.origin[d] = ch.origin[d]; }
    g.h = ch.h; g.count = nlm; g.off = 0; g.chan = 0;
    Batch bb;
    build_batch({g}, c->radius, sh, bb, dt, c->opts.lmax);
    fsic_status st = prepare_batch(c, bb, FSIC_FP64);
    if (st) return st;
    std::vector<double> ident((size_t)nlm * nlm, 0.0);
    for (int q = 0; q < nlm; ++q) ident[(size_t)q * nlm + q] = 1.0;
    if ((st = upload(c, c->qident, ident))) return st;
    DBuf<double> Ub;
    HIPCHK(c, Ub.ensure((size_t)nlm * ch.M));
    SolveReport rep;
    st = solve_batch(c, bb, nullptr, 0, 0.0, true, Ub.p, FSIC_FP64, 1e-13, c->opts.max_iter, rep, c->qident.p);
    if (!st) {
        const hipError_t e = hipStreamSynchronize(c->stream);
        st = e != hipSuccess ? set_err(c, FSIC_EHIP, hipGetErrorString(e)) : finish_solve(c, bb, rep);
    }
    if (!st && !rep.converged) st = set_err(c, FSIC_ENOCONV, "boundary basis solve did not converge");
    if (st) {
        Ub.release();
        return st;
    }
    // kept: the first octant (the solutions' reflection parities give the rest)
    DBuf<double> Uc;
    const size_t Mo = (size_t)((ch.n[0] + 1) / 2) * ((ch.n[1] + 1) / 2) * ((ch.n[2] + 1) / 2);
    hipError_t he = Uc.ensure((size_t)nlm * Mo);
    if (he == hipSuccess) he = launch_octant_pack(nlm, ch.n, Ub.p, Uc.p, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    Ub.release();
    if (he != hipSuccess) {
        Uc.release();
        return set_err(c, FSIC_EHIP, hipGetErrorString(he));
    }
    c->basis_solves += nlm;
    c->basis_ms += now_ms() - t0;
    DBuf<double> &slot = c->bbasis[key];
    std::swap(slot, Uc);
    *U = slot.p;
    return FSIC_OK;
}

// The backward pass in two parts: everything up to the gradient copies is
// enqueued (backward_enqueue), then, after the caller's wait on the stream,
// backward_finish reads the copies back.  fused: behind a forward pass in
// the same call (fsic_forward_backward), which prepared the batch and has
// not yet read its own statistics.
struct BwdState {
    double t0 = 0.0, t1 = 0.0;
    SolveReport rep;
    bool eq9 = false, reuse_w = false;
    std::vector<size_t> goff;
    std::vector<int> spin0;
};

static fsic_status backward_enqueue(fsic_ctx *c, bool fused, BwdState &bs);
static fsic_status backward_finish(fsic_ctx *c, bool fused, const double *grad_e, double *const *dE_da,
                                   fsic_stats *st, BwdState &bs);

// The forward pass; with dE_da (fsic_forward_backward) the backward pass's
// device work is enqueued behind it before the host waits, and read back
// after the forward pass's own checks.
static fsic_status forward_impl(fsic_ctx *c, int32_t nsys, const fsic_system *sys, double *e_sic,
                                double *Uout, double *Xout, fsic_stats *st, const double *grad_e,
                                double *const *dE_da, fsic_stats *bst) {
    if (!c) return FSIC_EINVAL;
    const double t0 = now_ms();
    if (nsys < 1 || !sys || !e_sic) return set_err(c, FSIC_EINVAL, "nsys >= 1, sys and e_sic are required");
    c->tape = false;
    const fsic_opts &o = c->opts;
    const int P = c->radius;
    std::string why;
    // ---- validation and plan (host) ----
    std::vector<Chan> chans;
    long long off = 0;
    int first = 0;
    for (int k = 0; k < nsys; ++k) {
        const fsic_system &sy = sys[k];
        fsic_status vs = validate_grid(sy.grid, why);
        if (vs) return set_err(c, vs, "system " + std::to_string(k) + ": " + why);
        if (sy.nspin < 1 || sy.nspin > 2) return set_err(c, FSIC_EINVAL, "nspin must be 1 or 2");
        const long long M = (long long)sy.grid.n[0] * sy.grid.n[1] * sy.grid.n[2];
        for (int s = 0; s < sy.nspin; ++s) {
            const int N = sy.nocc[s];
            if (N < 1 || N > kMaxOrb) return set_err(c, FSIC_EINVAL, "nocc must be in [1, 128]");
            if (!sy.psi[s] || !sy.fod[s]) return set_err(c, FSIC_EINVAL, "psi and fod are required");
            Chan ch{};
            ch.sys = k; ch.spin = s; ch.N = N;
            for (int d = 0; d < 3; ++d) { ch.n[d] = sy.grid.n[d]; ch.origin[d] = sy.grid.origin[d]; }
            ch.h = sy.grid.h;
            ch.M = M;
            ch.psi = sy.psi[s];
            ch.fod.assign(sy.fod[s], sy.fod[s] + 3 * N);
            ch.first_orb = first;
            ch.off = off;
            ch.cells.resize(N);
            for (int i = 0; i < N; ++i) {
                FodCell cl{};
                for (int d = 0; d < 3; ++d) {
                    const double a = ch.fod[3 * i + d];
                    if (!std::isfinite(a)) return set_err(c, FSIC_EINVAL, "non-finite FOD coordinate");
                    const double sc = (a - ch.origin[d]) / ch.h;
                    const double fl = std::floor(sc);
                    if (fl < 1.0 || fl > (double)(ch.n[d] - 3))
                        return set_err(c, FSIC_EBOUNDARY, "system " + std::to_string(k) + " spin " + std::to_string(s) +
                                                              " FOD " + std::to_string(i) + ": interpolation stencil leaves the grid");
                    cl.i0[d] = (int)fl;
                    cl.t[d] = sc - fl;
                }
                ch.cells[i] = cl;
            }
            off += (long long)N * M;
            first += N;
            chans.push_back(std::move(ch));
        }
    }
    const size_t F = (size_t)off;
    const int nchan = (int)chans.size();
    const int norb = first;
    std::vector<Group> groups;
    for (int ci = 0; ci < nchan; ++ci) {
        const Chan &ch = chans[ci];
        Group g{};
        for (int d = 0; d < 3; ++d) { g.n[d] = ch.n[d]; g.origin[d] = ch.origin[d]; }
        g.h = ch.h; g.count = ch.N; g.off = ch.off; g.chan = ci;
        groups.push_back(g);
    }
    Batch b;
    // zero-boundary solves plus the boundary basis when a backward pass will
    // need the zero-boundary (adjoint) solutions anyway
    const bool use_basis = (o.flags & FSIC_KEEP_TAPE) && !(o.flags & (FSIC_EQ9_FORCES | FSIC_DIRECT_BC));
    std::vector<const double *> basisU(nchan, nullptr);
    c->basis_solves = 0;
    c->basis_ms = 0.0;
    {
        Shape sh;
        fsic_status tst = choose_shape(c, groups, o.precision, sh);
        if (tst) return tst;
        c->cf.cpt = sh.cpt;
        c->cf.depth = sh.depth;
        c->shape_cpt = sh.cpt;
        c->shape_depth = sh.depth;
        c->shape_target = sh.target;
        DstTune dt;
        if ((tst = choose_dst(c, groups, o.precision, sh, dt))) return tst;
        if (use_basis)
            for (int ci = 0; ci < nchan; ++ci)
                if ((tst = boundary_basis(c, chans[ci], sh, dt, &basisU[ci]))) return tst;
        build_batch(groups, P, sh, b, dt, o.lmax);
        c->dst_layout = dst_layout_bits(b);
    }
    // channel descriptors for the average pass
    std::vector<ChanDesc> cd(nchan);
    std::vector<int> blkchan;
    int nblk_total = 0;
    for (int ci = 0; ci < nchan; ++ci) {
        Chan &ch = chans[ci];
        ch.nblk = (int)((ch.M + kSicTile - 1) / kSicTile);
        ch.blk_base = nblk_total;
        nblk_total += ch.nblk;
        for (int t = 0; t < ch.nblk; ++t) blkchan.push_back(ci);
        ChanDesc &d = cd[ci];
        d.N = ch.N; d.first_orb = ch.first_orb; d.M = ch.M; d.off = ch.off;
        d.nx = ch.n[0]; d.ny = ch.n[1]; d.nz = ch.n[2];
        d.nblk = ch.nblk; d.blk_base = ch.blk_base; d.h = ch.h; d.vscale = o.vsic_scale;
        d.vsic = (o.flags & FSIC_WANT_VSIC) ? sys[ch.sys].vsic[ch.spin] : nullptr;
        ch.so = (size_t)ci * kSmallStride;
    }
    // ---- buffers ----
    hipStream_t s = c->stream;
    HIPCHK(c, c->PHI.ensure(F));
    HIPCHK(c, c->V.ensure(F));
    fsic_status pst = prepare_batch(c, b, o.precision);
    if (pst) return pst;
    HIPCHK(c, c->small.ensure((size_t)nchan * kSmallStride));
    const long long lw = 3LL * kMaxOrb * kMaxOrb;  // Loewdin scratch per channel of a batched launch
    // (sized for the backward pass's 4 kMaxOrb^2 per channel, so it does not grow then)
    HIPCHK(c, c->work.ensure((size_t)std::min(nchan, kLowdinBatch) * 4 * (size_t)kMaxOrb * kMaxOrb));
    const int gram_blk = 1024;  // partial tiles of the orbital GEMMs: up to four blocks per compute unit
    c->sweep_launches = c->update_launches = c->precond_launches = 0;
    c->sweep_ms = c->sweep_bytes = c->update_ms = c->update_bytes = 0.0;
    c->precond_ms = c->precond_bytes = c->precond_flops = 0.0;
    c->resid_launches = 0;
    c->resid_ms = c->resid_bytes = 0.0;
    HIPCHK(c, c->partG.ensure((size_t)gram_blk * kMaxOrb * kMaxOrb));
    std::vector<FodCell> cells;
    for (const Chan &ch : chans) cells.insert(cells.end(), ch.cells.begin(), ch.cells.end());
    fsic_status ust;
    if ((ust = upload(c, c->d_cells, cells))) return ust;
    if ((ust = upload(c, c->d_chan, cd))) return ust;
    if ((ust = upload(c, c->d_blkchan, blkchan))) return ust;
    HIPCHK(c, c->partU.ensure((size_t)nblk_total * kMaxOrb));
    HIPCHK(c, c->partX.ensure((size_t)nblk_total * kMaxOrb));
    const size_t neux = 2 * (size_t)norb + nchan;
    HIPCHK(c, c->eux.ensure(neux));
    if (c->h_eux_cap < neux) {
        if (c->h_eux) hipHostFree(c->h_eux);
        c->h_eux = nullptr;
        c->h_eux_cap = 0;
        HIPCHK(c, hipHostMalloc((void **)&c->h_eux, neux * sizeof(double)));
        c->h_eux_cap = neux;
    }
    HIPCHK(c, hipMemsetAsync(c->status.p, 0, sizeof(int), s));
    const double t1 = now_ms();

    // ---- (a) Fermi orbitals, (b) Loewdin: per channel ----
    int cell_base = 0;
    for (int ci = 0; ci < nchan; ++ci) {
        const Chan &ch = chans[ci];
        double *sm = c->small.p + ch.so;
        const double dV = ch.h * ch.h * ch.h;
        HIPCHK(c, launch_interp(ch.N, ch.N, ch.n[0], ch.n[1], ch.n[2], ch.h, ch.psi, c->d_cells.p + cell_base,
                                o.rho_floor, sm + small_off(sU_), sm + small_off(sDU),
                                sm + small_off(sRHOA), sm + small_off(sT), c->status.p,
                                (o.flags & FSIC_PAPER_GRADIENT) != 0, s));
        HIPCHK(c, launch_gram(ch.N, ch.M, dV, ch.psi, c->partG.p, c->partG.cap, sm + small_off(sG), s));
        cell_base += ch.N;
    }
    // Loewdin steps of all channels, kLowdinBatch per launch (one workgroup each)
    const LowdinOffsets loff{(long long)small_off(sT), (long long)small_off(sG), (long long)small_off(sS),
                             (long long)small_off(sLAM), (long long)small_off(sEV), (long long)small_off(sZ),
                             (long long)small_off(sQ), (long long)small_off(sINFO)};
    for (int c0 = 0; c0 < nchan; c0 += kLowdinBatch) {
        LowdinBatch lb{};
        lb.n = std::min(kLowdinBatch, nchan - c0);
        for (int q = 0; q < lb.n; ++q) {
            lb.N[q] = chans[c0 + q].N;
            lb.so[q] = (long long)chans[c0 + q].so;
        }
        HIPCHK(c, launch_lowdin_batch(lb, c->small.p, loff, c->work.p, lw, o.s_eig_floor, c->status.p, s));
    }
    // device status and the per-channel overlap data for the host checks:
    // copied now, read after the pass (a solve stops early when the status
    // shows an error); stage layout per channel: G (N^2), info (2), rho(a) (N)
    size_t chk_n = 0;
    for (const Chan &ch : chans) chk_n += (size_t)ch.N * ch.N + 2 + ch.N;
    if (c->h_chk_cap < chk_n) {
        if (c->h_chk) hipHostFree(c->h_chk);
        c->h_chk = nullptr;
        c->h_chk_cap = 0;
        HIPCHK(c, hipHostMalloc((void **)&c->h_chk, chk_n * sizeof(double)));
        c->h_chk_cap = chk_n;
    }
    HIPCHK(c, hipMemcpyAsync(c->h_stat, c->status.p, sizeof(int), hipMemcpyDeviceToHost, s));
    {
        // packed on the device, one copy
        HIPCHK(c, c->d_chk.ensure(chk_n));
        ChkPack pk{};
        pk.oG = (long long)small_off(sG);
        pk.oI = (long long)small_off(sINFO);
        pk.oR = (long long)small_off(sRHOA);
        size_t q = 0;
        for (size_t ci = 0; ci < chans.size(); ++ci) {
            const Chan &ch = chans[ci];
            pk.N[pk.n] = ch.N;
            pk.so[pk.n] = (long long)ch.so;
            pk.q[pk.n] = (long long)q;
            ++pk.n;
            q += (size_t)ch.N * ch.N + 2 + ch.N;
            if (pk.n == kChkPack || ci + 1 == chans.size()) {
                HIPCHK(c, launch_pack_checks(pk, c->small.p, c->d_chk.p, s));
                pk.n = 0;
            }
        }
        HIPCHK(c, hipMemcpyAsync(c->h_chk, c->d_chk.p, chk_n * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    // phi = Q psi on the matrix cores
    for (int ci = 0; ci < nchan; ++ci) {
        const Chan &ch = chans[ci];
        if (o.flags & FSIC_FP32_ORBITALS)
            HIPCHK(c, launch_orb_gemm32(ch.N, ch.M, c->small.p + ch.so + small_off(sQ), ch.psi, c->PHI.p + ch.off, s));
        else
            HIPCHK(c, launch_orb_gemm(ch.N, ch.M, c->small.p + ch.so + small_off(sQ), ch.psi, c->PHI.p + ch.off, s));
    }
    const double t2 = now_ms();

    // ---- (c) Poisson solves for all orbitals at once ----
    SolveReport rep;
    c->watch_status = true;
    c->w_ready = false;
    fsic_status sst;
    if (use_basis) {
        // moments of rho_i, zero-boundary solves into W, then
        // v_i = w_i + sum_q Q_q,i U_q
        HIPCHK(c, c->W.ensure(F));
        HIPCHK(c, launch_harm_contract(0, o.lmax, c->ht, c->cf, c->radius, c->d_orb.p, c->d_gcount.p, c->d_hcN.p,
                                       (int)b.hcN.size(), c->d_hchN.p, (int)b.hchN.size(), b.max_group, c->PHI.p,
                                       1, c->partH.p, c->Qlm.p, s));
        sst = solve_batch(c, b, c->PHI.p, 1, 4.0 * M_PI, false, c->W.p, o.precision, o.tol, o.max_iter, rep);
        // one launch per run of consecutive channels on one grid (a system's
        // spins: their orbitals are contiguous), so the basis is read once
        for (int ci = 0; !sst && ci < nchan;) {
            const Chan &ch = chans[ci];
            int cj = ci + 1, n = ch.N;
            while (cj < nchan && basisU[cj] == basisU[ci] && chans[cj].off == ch.off + (long long)n * ch.M &&
                   chans[cj].first_orb == ch.first_orb + n) {
                n += chans[cj].N;
                ++cj;
            }
            HIPCHK(c, launch_bc_combine(n, ch.n, o.lmax, c->Qlm.p, ch.first_orb, basisU[ci], c->W.p + ch.off,
                                        c->V.p + ch.off, s));
            ci = cj;
        }
    } else {
        sst = solve_batch(c, b, c->PHI.p, 1, 4.0 * M_PI, true, c->V.p, o.precision, o.tol, o.max_iter, rep);
    }
    c->watch_status = false;
    if (sst) return sst;
    const double t3 = now_ms();

    // ---- (d) XC, (e) Slater average and energies ----
    HIPCHK(c, launch_sic_average(nchan, c->d_chan.p, nblk_total, c->d_blkchan.p, c->PHI.p, c->V.p,
                                 o.rho_floor, c->partU.p, c->partX.p, s));
    double *const dU = c->eux.p, *const dX = dU + norb, *const dE = dX + norb;
    HIPCHK(c, launch_sic_energy(nchan, c->d_chan.p, c->partU.p, c->partX.p, dU, dX, dE, s));
    HIPCHK(c, hipMemcpyAsync(c->h_eux, c->eux.p, (2 * (size_t)norb + nchan) * sizeof(double),
                             hipMemcpyDeviceToHost, s));
    // the plan becomes the tape (its flag is set once the checks below pass)
    c->chans = std::move(chans);
    c->batch = std::move(b);
    c->nsys = nsys;
    const std::vector<Chan> &chs = c->chans;
    const Batch &bt = c->batch;
    // fused backward pass: enqueued now, behind the forward pass's work
    const bool fused = dE_da != nullptr && use_basis;
    BwdState bws;
    if (fused) {
        c->w_ready = true;
        fsic_status bs = backward_enqueue(c, true, bws);
        c->w_ready = false;  // the enqueued work turns W into Gam
        if (bs) return bs;
    }
    HIPCHK(c, hipStreamSynchronize(s));
    const double *const uo = c->h_eux, *const xo = uo + norb, *const ech = xo + norb;

    // ---- host checks of the inputs (Sec. I.B: normalised, linearly
    // independent Fermi orbitals; Eq. 8: nonzero density at every FOD) ----
    const int hstatus = *c->h_stat;
    if (hstatus & kStNonFinite) return set_err(c, FSIC_EINVAL, "non-finite orbital values at an FOD");
    if (hstatus & kStVacuum) return set_err(c, FSIC_EVACUUM, "an FOD lies where rho(a_i) <= rho_floor");
    double nonortho = 0.0, condmax = 0.0, minrho = 1e300, minlam = 0.0;
    {
        size_t q = 0;
        for (const Chan &ch : chs) {
            const size_t NN = (size_t)ch.N * ch.N;
            const double *G = c->h_chk + q, *info = c->h_chk + q + NN, *rhoa = c->h_chk + q + NN + 2;
            for (int i = 0; i < ch.N; ++i) {
                for (int j = 0; j < ch.N; ++j) {
                    const double g = G[(size_t)i * ch.N + j];
                    if (!std::isfinite(g)) return set_err(c, FSIC_EINVAL, "non-finite values in psi");
                    nonortho = std::max(nonortho, std::fabs(g - (i == j ? 1.0 : 0.0)));
                }
                minrho = std::min(minrho, rhoa[i]);
            }
            condmax = std::max(condmax, info[0]);
            if (minlam == 0.0 || info[1] < minlam) minlam = info[1];
            q += NN + 2 + ch.N;
        }
    }
    if (hstatus & kStSingular)
        return set_err(c, FSIC_ESINGULAR, "smallest eigenvalue of S = " + std::to_string(minlam) +
                                              " below s_eig_floor");
    if (!(o.flags & FSIC_ALLOW_NONORTHO) && nonortho > 1e-8)
        return set_err(c, FSIC_ENONORTHO, "max |dV psi psi^T - I| = " + std::to_string(nonortho));
    fsic_status fst = finish_solve(c, bt, rep);
    if (fst) return fst;
    for (int k = 0; k < nsys; ++k) e_sic[k] = 0.0;
    for (int ci = 0; ci < nchan; ++ci) e_sic[chs[ci].sys] += ech[ci];
    if (Uout) std::memcpy(Uout, uo, norb * sizeof(double));
    if (Xout) std::memcpy(Xout, xo, norb * sizeof(double));
    const double t4 = now_ms();
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->nsolves = norb;
        st->max_iters = rep.max_iters;
        st->total_iters = rep.total_iters;
        st->outer_refinements = rep.refinements;
        st->max_relres = rep.max_relres;
        st->cond_S_max = condmax;
        st->min_rho_fod = minrho;
        st->max_nonortho = nonortho;
        st->ms_phase[0] = t1 - t0;
        st->ms_phase[1] = t2 - t1;
        st->ms_phase[3] = t3 - t2;
        st->ms_phase[4] = t4 - t3;
        st->ms_phase[7] = t4 - t0;
        st->sweep_launches = c->sweep_launches;
        st->update_launches = c->update_launches;
        st->sweep_ms = c->sweep_ms;
        st->sweep_bytes = c->sweep_bytes;
        st->update_ms = c->update_ms;
        st->update_bytes = c->update_bytes;
        st->precond_launches = c->precond_launches;
        st->precond_ms = c->precond_ms;
        st->precond_bytes = c->precond_bytes;
        st->precond_flops = c->precond_flops;
        st->resid_launches = c->resid_launches;
        st->resid_ms = c->resid_ms;
        st->resid_bytes = c->resid_bytes;
        st->graph_captures = c->graph_captures;
        st->precond_layout = c->dst_layout;
        st->precond_tune_ms = c->dst_tune_ms;
        st->stencil_cpt = c->shape_cpt;
        st->stencil_depth = c->shape_depth;
        st->stencil_blocks = c->shape_target;
        st->tune_ms = c->tune_ms;
        st->npoisson = use_basis ? 2 * norb : norb;
        st->basis_solves = c->basis_solves;
        st->basis_ms = c->basis_ms;
    }
    c->tape = (o.flags & FSIC_KEEP_TAPE) != 0;
    c->w_ready = use_basis && rep.converged && !fused;
    if (!rep.converged) return set_err(c, FSIC_ENOCONV, "a Poisson solve missed tol within max_iter");
    if (fused) return backward_finish(c, true, grad_e, dE_da, bst, bws);
    return FSIC_OK;
}

fsic_status fsic_forward(fsic_ctx *c, int32_t nsys, const fsic_system *sys, double *e_sic,
                         double *Uout, double *Xout, fsic_stats *st) {
    return forward_impl(c, nsys, sys, e_sic, Uout, Xout, st, nullptr, nullptr, nullptr);
}

fsic_status fsic_forward_backward(fsic_ctx *c, int32_t nsys, const fsic_system *sys, double *e_sic,
                                  double *Uout, double *Xout, const double *grad_e, double *const *dE_da,
                                  fsic_stats *st_fwd, fsic_stats *st_bwd) {
    if (!c) return FSIC_EINVAL;
    if (!(c->opts.flags & FSIC_KEEP_TAPE))
        return set_err(c, FSIC_ENOTAPE, "fsic_forward_backward needs FSIC_KEEP_TAPE");
    if (!dE_da) return set_err(c, FSIC_EINVAL, "dE_da is required");
    if (nsys < 1 || !sys) return set_err(c, FSIC_EINVAL, "nsys >= 1, sys and e_sic are required");
    for (int k = 0; k < nsys; ++k)
        if (!dE_da[k]) return set_err(c, FSIC_EINVAL, "dE_da[k] is required for every system");
    const bool basis = !(c->opts.flags & (FSIC_EQ9_FORCES | FSIC_DIRECT_BC));
    if (basis) return forward_impl(c, nsys, sys, e_sic, Uout, Xout, st_fwd, grad_e, dE_da, st_bwd);
    // the backward pass solves its own adjoint problems: one after the other
    fsic_status e = forward_impl(c, nsys, sys, e_sic, Uout, Xout, st_fwd, nullptr, nullptr, nullptr);
    if (e) return e;
    return fsic_backward(c, grad_e, dE_da, st_bwd);
}

// ---------------------------------------------------------------------------
// operator-level entry points
// ---------------------------------------------------------------------------

namespace {
struct OpCtx {
    fsic_ctx *c = nullptr;
    ~OpCtx() { fsic_destroy(c); }
};
}  // namespace

fsic_status fsic_op_laplacian(const int32_t *n, double h, int32_t fd_order, int32_t count,
                              const double *u, double *Lu, void *hip_stream) {
    if (!n || !u || !Lu || count < 1 || fd_order < 2 || fd_order > 12 || (fd_order & 1))
        return FSIC_EINVAL;
    fsic_grid g{{n[0], n[1], n[2]}, h, {0, 0, 0}};
    std::string why;
    if (validate_grid(g, why)) return FSIC_EINVAL;
    const int P = fd_order / 2;
    std::vector<Group> groups(1);
    for (int d = 0; d < 3; ++d) { groups[0].n[d] = n[d]; groups[0].origin[d] = 0.0; }
    groups[0].h = h; groups[0].count = count; groups[0].off = 0; groups[0].chan = 0;
    Batch b;
    build_batch(groups, P, Shape{2, 2, 4096}, b);  // fd_weights: cpt 2, depth 2
    hipStream_t s = (hipStream_t)hip_stream;
    DBuf<OrbDesc> dorb;
    DBuf<Item> dit;
    if (dorb.ensure(b.orb.size()) || dit.ensure(b.items7.size())) return FSIC_ENOMEM;
    hipMemcpyAsync(dorb.p, b.orb.data(), b.orb.size() * sizeof(OrbDesc), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dit.p, b.items7.data(), b.items7.size() * sizeof(Item), hipMemcpyHostToDevice, s);
    hipError_t e = launch_apply<double>(P, fd_weights(P), dit.p, (int)b.items7.size(), dorb.p, u, Lu, s);
    hipError_t e2 = hipStreamSynchronize(s);
    dorb.release();
    dit.release();
    return (e || e2) ? FSIC_EHIP : FSIC_OK;
}

fsic_status fsic_op_hamiltonian(const int32_t *n, double h, int32_t fd_order, int32_t count,
                                const double *psi, const double *v, double *out, void *hip_stream) {
    if (!n || !psi || !v || !out || count < 1 || fd_order < 2 || fd_order > 12 || (fd_order & 1))
        return FSIC_EINVAL;
    fsic_grid g{{n[0], n[1], n[2]}, h, {0, 0, 0}};
    std::string why;
    if (validate_grid(g, why)) return FSIC_EINVAL;
    const int P = fd_order / 2;
    std::vector<Group> groups(1);
    for (int d = 0; d < 3; ++d) { groups[0].n[d] = n[d]; groups[0].origin[d] = 0.0; }
    groups[0].h = h; groups[0].count = count; groups[0].off = 0; groups[0].chan = 0;
    Batch b;
    build_batch(groups, P, Shape{2, 2, 4096}, b);  // fd_weights: cpt 2, depth 2
    hipStream_t s = (hipStream_t)hip_stream;
    DBuf<OrbDesc> dorb;
    DBuf<Item> dit;
    if (dorb.ensure(b.orb.size()) || dit.ensure(b.items7.size())) return FSIC_ENOMEM;
    hipError_t e = hipMemcpyAsync(dorb.p, b.orb.data(), b.orb.size() * sizeof(OrbDesc), hipMemcpyHostToDevice, s);
    if (!e) e = hipMemcpyAsync(dit.p, b.items7.data(), b.items7.size() * sizeof(Item), hipMemcpyHostToDevice, s);
    if (!e) e = launch_hamiltonian(P, fd_weights(P), dit.p, (int)b.items7.size(), dorb.p, psi, v, out, s);
    hipError_t e2 = hipStreamSynchronize(s);
    dorb.release();
    dit.release();
    return (e || e2) ? FSIC_EHIP : FSIC_OK;
}

fsic_status fsic_op_laplacian_f32(const int32_t *n, double h, int32_t fd_order, int32_t count,
                                  const float *u, float *Lu, void *hip_stream) {
    if (!n || !u || !Lu || count < 1 || fd_order < 2 || fd_order > 12 || (fd_order & 1))
        return FSIC_EINVAL;
    fsic_grid g{{n[0], n[1], n[2]}, h, {0, 0, 0}};
    std::string why;
    if (validate_grid(g, why)) return FSIC_EINVAL;
    const int P = fd_order / 2;
    std::vector<Group> groups(1);
    for (int d = 0; d < 3; ++d) { groups[0].n[d] = n[d]; groups[0].origin[d] = 0.0; }
    groups[0].h = h; groups[0].count = count; groups[0].off = 0; groups[0].chan = 0;
    Batch b;
    build_batch(groups, P, Shape{2, 2, 4096}, b);  // fd_weights: cpt 2, depth 2
    hipStream_t s = (hipStream_t)hip_stream;
    DBuf<OrbDesc> dorb;
    DBuf<Item> dit;
    if (dorb.ensure(b.orb.size()) || dit.ensure(b.items7.size())) return FSIC_ENOMEM;
    hipMemcpyAsync(dorb.p, b.orb.data(), b.orb.size() * sizeof(OrbDesc), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dit.p, b.items7.data(), b.items7.size() * sizeof(Item), hipMemcpyHostToDevice, s);
    hipError_t e = launch_apply<float>(P, fd_weights(P), dit.p, (int)b.items7.size(), dorb.p, u, Lu, s);
    hipError_t e2 = hipStreamSynchronize(s);
    dorb.release();
    dit.release();
    return (e || e2) ? FSIC_EHIP : FSIC_OK;
}

fsic_status fsic_op_xc(int64_t count, const double *rho, double rho_floor, double *ex, double *ec,
                       double *vx, double *vc, void *hip_stream) {
    if (count < 0 || (count > 0 && !rho) || !(rho_floor >= 0.0)) return FSIC_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = launch_xc_pointwise(count, rho, rho_floor, ex, ec, vx, vc, s);
    hipError_t e2 = hipStreamSynchronize(s);
    return (e || e2) ? FSIC_EHIP : FSIC_OK;
}

fsic_status fsic_op_poisson(const fsic_grid *grid, int32_t fd_order, int32_t lmax, int32_t count,
                            const double *rho, double *v, double tol, int32_t max_iter,
                            int32_t precision, int32_t solver, int32_t *iters, double *relres,
                            void *hip_stream) {
    if (!grid || !rho || !v || count < 1) return FSIC_EINVAL;
    fsic_opts o;
    fsic_default_opts(&o);
    o.fd_order = fd_order;
    o.lmax = lmax;
    o.tol = tol;
    o.max_iter = max_iter;
    o.precision = precision;
    o.solver = solver;
    std::string why;
    if (validate_opts(&o, why) || validate_grid(*grid, why)) return FSIC_EINVAL;
    OpCtx oc;
    fsic_status st = fsic_create(&oc.c, &o, hip_stream);
    if (st) return st;
    fsic_ctx *c = oc.c;
    std::vector<Group> groups(1);
    for (int d = 0; d < 3; ++d) { groups[0].n[d] = grid->n[d]; groups[0].origin[d] = grid->origin[d]; }
    groups[0].h = grid->h; groups[0].count = count; groups[0].off = 0; groups[0].chan = 0;
    Batch b;
    Shape sh;
    st = choose_shape(c, groups, precision, sh);
    if (st) return st;
    c->cf.cpt = sh.cpt;
    c->cf.depth = sh.depth;
    DstTune dt;
    if ((st = choose_dst(c, groups, precision, sh, dt))) return st;
    build_batch(groups, c->radius, sh, b, dt, lmax);
    st = prepare_batch(c, b, precision);
    if (st) return st;
    SolveReport rep;
    st = solve_batch(c, b, rho, 0, 4.0 * M_PI, true, v, precision, tol, max_iter, rep);
    if (st) return st;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return FSIC_EHIP;
    st = finish_solve(c, b, rep);
    if (st) return st;
    std::vector<int> it(count);
    std::vector<double> pt(count), bbh(count);
    hipMemcpy(it.data(), c->iters.p, count * sizeof(int), hipMemcpyDeviceToHost);
    hipMemcpy(pt.data(), c->ptrue.p, count * sizeof(double), hipMemcpyDeviceToHost);
    hipMemcpy(bbh.data(), c->bb.p, count * sizeof(double), hipMemcpyDeviceToHost);
    std::vector<int> dn(count);
    hipMemcpy(dn.data(), c->done.p, count * sizeof(int), hipMemcpyDeviceToHost);
    for (int f = 0; f < count; ++f) {
        if (iters) iters[f] = dn[f] ? it[f] : max_iter;
        if (relres) relres[f] = bbh[f] > 0 ? std::sqrt(pt[f] / bbh[f]) : 0.0;
    }
    return rep.converged ? FSIC_OK : FSIC_ENOCONV;
}

fsic_status fsic_op_invsqrt(int32_t N, int32_t count, const double *S, double *Z, double *lam,
                            void *hip_stream) {
    if (N < 1 || N > kMaxOrb || count < 1 || !S || !Z) return FSIC_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t NN = (size_t)N * N;
    DBuf<double> T, tmp, work, info;
    DBuf<int> status;
    if (T.ensure(NN) || tmp.ensure(5 * NN) || work.ensure(3 * (size_t)kMaxOrb * kMaxOrb) ||
        info.ensure(2) || status.ensure(1))
        return FSIC_ENOMEM;
    std::vector<double> eye(NN, 0.0);
    for (int i = 0; i < N; ++i) eye[(size_t)i * N + i] = 1.0;
    hipMemcpyAsync(T.p, eye.data(), NN * sizeof(double), hipMemcpyHostToDevice, s);
    hipMemsetAsync(status.p, 0, sizeof(int), s);
    hipError_t e = hipSuccess;
    for (int k = 0; k < count && e == hipSuccess; ++k) {
        double *lamk = lam ? lam + (size_t)k * N : tmp.p + 4 * NN;
        e = launch_lowdin(N, T.p, S + k * NN, tmp.p, lamk, tmp.p + NN, Z + k * NN, tmp.p + 2 * NN,
                          work.p, 0.0, status.p, info.p, s);
    }
    hipError_t e2 = hipStreamSynchronize(s);
    int hs = 0;
    hipMemcpy(&hs, status.p, sizeof(int), hipMemcpyDeviceToHost);
    T.release(); tmp.release(); work.release(); info.release(); status.release();
    if (e || e2) return FSIC_EHIP;
    return (hs & kStSingular) ? FSIC_ESINGULAR : FSIC_OK;
}

fsic_status fsic_op_interp(const fsic_grid *grid, int32_t N, int32_t K, const double *psi,
                           const double *pts, int32_t fd_gradient, double *u, double *du,
                           void *hip_stream) {
    if (!grid || !psi || !pts || !u || !du || N < 1 || N > kMaxOrb || K < 1 ||
        (fd_gradient != 0 && fd_gradient != 1))
        return FSIC_EINVAL;
    std::string why;
    if (validate_grid(*grid, why)) return FSIC_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<FodCell> cells(K);
    for (int i = 0; i < K; ++i)
        for (int d = 0; d < 3; ++d) {
            const double a = pts[3 * i + d];
            if (!std::isfinite(a)) return FSIC_EINVAL;
            const double sc = (a - grid->origin[d]) / grid->h;
            const double fl = std::floor(sc);
            if (fl < 1.0 || fl > (double)(grid->n[d] - 3)) return FSIC_EBOUNDARY;
            cells[i].i0[d] = (int)fl;
            cells[i].t[d] = sc - fl;
        }
    DBuf<double> rhoa, T;
    DBuf<FodCell> dc;
    DBuf<int> status;
    if (rhoa.ensure(K) || T.ensure((size_t)K * N) || dc.ensure(K) || status.ensure(1)) return FSIC_ENOMEM;
    hipError_t e = hipMemcpyAsync(dc.p, cells.data(), K * sizeof(FodCell), hipMemcpyHostToDevice, s);
    if (!e) e = hipMemsetAsync(status.p, 0, sizeof(int), s);
    if (!e) e = launch_interp(K, N, grid->n[0], grid->n[1], grid->n[2], grid->h, psi, dc.p, -1.0, u, du,
                              rhoa.p, T.p, status.p, fd_gradient != 0, s);
    hipError_t e2 = hipStreamSynchronize(s);
    rhoa.release(); T.release(); dc.release(); status.release();
    return (e || e2) ? FSIC_EHIP : FSIC_OK;
}

}  // extern "C"

namespace {
// Interpolation cells of N FODs on a grid (host validation shared by the
// Fermi-Loewdin entry points): FSIC_EINVAL for a non-finite coordinate,
// FSIC_EBOUNDARY when a 4-node stencil leaves the grid.
fsic_status fod_cells(const fsic_grid &g, int N, const double *fod, FodCell *cells) {
    for (int i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) {
            const double a = fod[3 * i + d];
            if (!std::isfinite(a)) return FSIC_EINVAL;
            const double sc = (a - g.origin[d]) / g.h;
            const double fl = std::floor(sc);
            if (fl < 1.0 || fl > (double)(g.n[d] - 3)) return FSIC_EBOUNDARY;
            cells[i].i0[d] = (int)fl;
            cells[i].pad = 0;
            cells[i].t[d] = sc - fl;
        }
    return FSIC_OK;
}
}  // namespace

extern "C" {

fsic_status fsic_op_flo_noalloc(const fsic_grid *grid, int32_t N, const double *psi, const double *fod,
                                double rho_floor, double *T, double *G, double *S, double *Z,
                                double *phi, void *hip_stream) {
    if (!grid || !psi || !fod || N < 1 || N > kMaxOrb || !(rho_floor >= 0.0)) return FSIC_EINVAL;
    std::string why;
    if (validate_grid(*grid, why)) return FSIC_EINVAL;
    FodCell cells[kMaxOrb];
    const fsic_status cs = fod_cells(*grid, N, fod, cells);
    if (cs) return cs;
    int hs = 0;
    const hipError_t e = noalloc_flo(N, grid->n, grid->h, psi, cells, rho_floor, T, G, S, Z, phi, &hs,
                                     (hipStream_t)hip_stream);
    if (e != hipSuccess) return FSIC_EHIP;
    if (hs & kStVacuum) return FSIC_EVACUUM;
    if (hs & kStSingular) return FSIC_ESINGULAR;
    return FSIC_OK;
}

fsic_status fsic_op_flo(const fsic_grid *grid, int32_t N, const double *psi, const double *fod,
                        double rho_floor, double *T, double *G, double *S, double *Z, double *phi,
                        void *hip_stream) {
    if (!grid || !psi || !fod || N < 1 || N > kMaxOrb || !(rho_floor >= 0.0)) return FSIC_EINVAL;
    std::string why;
    if (validate_grid(*grid, why)) return FSIC_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<FodCell> cells(N);
    {
        const fsic_status cs = fod_cells(*grid, N, fod, cells.data());
        if (cs) return cs;
    }
    const long long M = (long long)grid->n[0] * grid->n[1] * grid->n[2];
    const double dV = grid->h * grid->h * grid->h;
    DBuf<double> sm, work, partG;
    DBuf<FodCell> dc;
    DBuf<int> status;
    if (sm.ensure(kSmallStride) || work.ensure(3 * (size_t)kMaxOrb * kMaxOrb) ||
        partG.ensure(256 * (size_t)kMaxOrb * kMaxOrb) || dc.ensure(N) || status.ensure(1))
        return FSIC_ENOMEM;
    hipError_t e = hipMemcpyAsync(dc.p, cells.data(), N * sizeof(FodCell), hipMemcpyHostToDevice, s);
    if (!e) e = hipMemsetAsync(status.p, 0, sizeof(int), s);
    double *b = sm.p;
    if (!e) e = launch_interp(N, N, grid->n[0], grid->n[1], grid->n[2], grid->h, psi, dc.p, rho_floor,
                              b + small_off(sU_), b + small_off(sDU), b + small_off(sRHOA),
                              b + small_off(sT), status.p, false, s);
    if (!e) e = launch_gram(N, M, dV, psi, partG.p, partG.cap, b + small_off(sG), s);
    if (!e) e = launch_lowdin(N, b + small_off(sT), b + small_off(sG), b + small_off(sS),
                              b + small_off(sLAM), b + small_off(sEV), b + small_off(sZ),
                              b + small_off(sQ), work.p, 0.0, status.p, b + small_off(sINFO), s);
    if (!e && phi) e = launch_orb_gemm(N, M, b + small_off(sQ), psi, phi, s);
    const size_t NN = (size_t)N * N * sizeof(double);
    if (!e && T) e = hipMemcpyAsync(T, b + small_off(sT), NN, hipMemcpyDeviceToDevice, s);
    if (!e && G) e = hipMemcpyAsync(G, b + small_off(sG), NN, hipMemcpyDeviceToDevice, s);
    if (!e && S) e = hipMemcpyAsync(S, b + small_off(sS), NN, hipMemcpyDeviceToDevice, s);
    if (!e && Z) e = hipMemcpyAsync(Z, b + small_off(sZ), NN, hipMemcpyDeviceToDevice, s);
    int hs = 0;
    if (!e) e = hipMemcpyAsync(&hs, status.p, sizeof(int), hipMemcpyDeviceToHost, s);
    hipError_t e2 = hipStreamSynchronize(s);
    sm.release(); work.release(); partG.release(); dc.release(); status.release();
    if (e || e2) return FSIC_EHIP;
    if (hs & kStVacuum) return FSIC_EVACUUM;
    if (hs & kStSingular) return FSIC_ESINGULAR;
    return FSIC_OK;
}

static fsic_status backward_enqueue(fsic_ctx *c, bool fused, BwdState &bs) {
    bs.t0 = now_ms();
    const double t0 = bs.t0;
    (void)t0;
    const fsic_opts &o = c->opts;
    const Batch &b = c->batch;
    hipStream_t s = c->stream;
    if (!fused) {
        c->tune_ms = 0.0;  // the backward pass reuses the forward pass's stencil shape and
        c->dst_tune_ms = 0.0;  // preconditioner layout
        c->sweep_launches = c->update_launches = c->precond_launches = 0;
        c->sweep_ms = c->sweep_bytes = c->update_ms = c->update_bytes = 0.0;
        c->precond_ms = c->precond_bytes = c->precond_flops = 0.0;
        c->resid_launches = 0;
        c->resid_ms = c->resid_bytes = 0.0;
        // (fused: the forward pass prepared this batch and its statistics
        // are still to be read)
        fsic_status pst = prepare_batch(c, b, o.precision);
        if (pst) return pst;
    }
    SolveReport &rep = bs.rep;
    rep = SolveReport{};
    rep.converged = true;
    // Eq. 9 form: the orbital SIC potential -(v_i + vxc_i) in place of the
    // exact -((v_i + A^T rho_i)/2 + vxc_i), so A^T rho_i is taken as v_i
    const bool eq9 = (o.flags & FSIC_EQ9_FORCES) != 0;
    bs.eq9 = eq9;
    const double *Wt = c->V.p;
    // the forward pass left the adjoint fields in W (zero-boundary solves)
    const bool reuse_w = !eq9 && c->w_ready;
    bs.reuse_w = reuse_w;
    if (!eq9) {
        HIPCHK(c, c->W.ensure((size_t)b.fields));
        if (!reuse_w) {
            // adjoint solves: K w' = 4 pi rho_i with zero Dirichlet values
            fsic_status sst = solve_batch(c, b, c->PHI.p, 1, 4.0 * M_PI, false, c->W.p, o.precision, o.tol,
                                          o.max_iter, rep);
            if (sst) return sst;
        }
        // boundary part of A^T rho: zt = E_g^T C^T w' / (4 pi), then W += P^T zt
        HarmTables hta = c->ht;
        for (int q = 0; q < kMaxLM; ++q) hta.gfac[q] /= 4.0 * M_PI;
        HIPCHK(c, launch_harm_contract(1, o.lmax, hta, c->cf, c->radius, c->d_orb.p, c->d_gcount.p,
                                       c->d_hcG.p, (int)b.hcG.size(), c->d_hchG.p, (int)b.hchG.size(),
                                       b.max_group, c->W.p, 0, c->partH.p, c->Zt.p, s));
        HIPCHK(c, launch_harm_expand(1, o.lmax, c->ht, c->radius, c->d_orb.p, c->d_gcount.p, c->d_hcNx.p,
                                     (int)b.hcNx.size(), c->Zt.p, c->W.p, s));
        Wt = c->W.p;
    }
    bs.t1 = now_ms();
    HIPCHK(c, c->W.ensure((size_t)b.fields));  // Gam (the Eq. 9 form has no adjoint field)
    // per channel: B = Gam psi^T, then the N x N reverse chain
    std::vector<int> &spin0 = bs.spin0;
    spin0.assign(c->nsys, 0);
    for (const Chan &ch : c->chans)
        if (ch.spin == 0) spin0[ch.sys] = ch.N;
    // dE/da of every channel lands in one pinned host block (asynchronous
    // copies, one wait at the end)
    std::vector<size_t> &goff = bs.goff;
    goff.assign(c->chans.size() + 1, 0);
    for (size_t ci = 0; ci < c->chans.size(); ++ci) goff[ci + 1] = goff[ci] + 3 * (size_t)c->chans[ci].N;
    if (c->h_grad_cap < goff.back()) {
        if (c->h_grad) hipHostFree(c->h_grad);
        c->h_grad = nullptr;
        c->h_grad_cap = 0;
        HIPCHK(c, hipHostMalloc((void **)&c->h_grad, std::max<size_t>(goff.back(), 1) * sizeof(double)));
        c->h_grad_cap = goff.back();
    }
    // per channel B = Gam psi^T into its own block of bmat, then the reverse
    // Loewdin steps of up to kLowdinBatch channels in one launch, which also
    // packs every dE/da for one copy
    const int nch = (int)c->chans.size();
    const long long bstride = (long long)kMaxOrb * kMaxOrb, wstride = 4LL * kMaxOrb * kMaxOrb;
    HIPCHK(c, c->bmat.ensure((size_t)bstride * std::min(nch, kLowdinBatch)));
    HIPCHK(c, c->work.ensure((size_t)wstride * std::min(nch, kLowdinBatch)));
    HIPCHK(c, c->d_grad.ensure(std::max<size_t>(goff.back(), 1)));
    const LowdinBwdOffsets lo{(long long)small_off(sT),   (long long)small_off(sG),   (long long)small_off(sLAM),
                              (long long)small_off(sEV),  (long long)small_off(sZ),   (long long)small_off(sRHOA),
                              (long long)small_off(sDU),  (long long)small_off(sDEDA)};
    for (int c0 = 0; c0 < nch; c0 += kLowdinBatch) {
        LowdinBwdBatch lb{};
        lb.n = std::min(kLowdinBatch, nch - c0);
        for (int q = 0; q < lb.n; ++q) {
            const Chan &ch = c->chans[c0 + q];
            const double dV = ch.h * ch.h * ch.h;
            // Gam overwrites W (the adjoint field is not needed after it)
            HIPCHK(c, launch_adjoint_contract(ch.N, ch.M, dV, c->PHI.p + ch.off, c->V.p + ch.off,
                                              Wt + ch.off, ch.psi, o.rho_floor, c->partG.p, c->partG.cap,
                                              c->bmat.p + (size_t)q * bstride, c->W.p + ch.off, s));
            lb.N[q] = ch.N;
            lb.so[q] = (long long)ch.so;
            lb.go[q] = (long long)goff[c0 + q];
        }
        HIPCHK(c, launch_lowdin_backward_batch(lb, c->bmat.p, bstride, c->small.p, lo, c->work.p, wstride,
                                               c->d_grad.p, s));
    }
    HIPCHK(c, hipMemcpyAsync(c->h_grad, c->d_grad.p, goff.back() * sizeof(double), hipMemcpyDeviceToHost, s));
    return FSIC_OK;
}

static fsic_status backward_finish(fsic_ctx *c, bool fused, const double *grad_e, double *const *dE_da,
                                   fsic_stats *st, BwdState &bs) {
    const fsic_opts &o = c->opts;
    (void)o;
    const Batch &b = c->batch;
    const int norb = (int)b.orb.size();
    const double t0 = bs.t0, t1 = bs.t1;
    SolveReport &rep = bs.rep;
    const bool eq9 = bs.eq9, reuse_w = bs.reuse_w;
    const std::vector<size_t> &goff = bs.goff;
    const std::vector<int> &spin0 = bs.spin0;
    c->w_ready = false;  // W now holds Gam
    if (!eq9 && !reuse_w) {
        fsic_status fst = finish_solve(c, b, rep);
        if (fst) return fst;
    }
    for (size_t ci = 0; ci < c->chans.size(); ++ci) {
        const Chan &ch = c->chans[ci];
        const double ge = grad_e ? grad_e[ch.sys] : 1.0;
        double *dst = dE_da[ch.sys] + 3 * (ch.spin == 0 ? 0 : spin0[ch.sys]);
        for (int q = 0; q < 3 * ch.N; ++q) dst[q] = ge * c->h_grad[goff[ci] + q];
    }
    const double t2 = now_ms();
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->nsolves = (eq9 || reuse_w) ? 0 : norb;
        st->npoisson = st->nsolves;
        st->max_iters = rep.max_iters;
        st->total_iters = rep.total_iters;
        st->outer_refinements = rep.refinements;
        st->max_relres = rep.max_relres;
        st->ms_phase[5] = t1 - t0;
        st->ms_phase[6] = t2 - t1;
        st->ms_phase[7] = t2 - t0;
        st->sweep_launches = c->sweep_launches;
        st->update_launches = c->update_launches;
        st->sweep_ms = c->sweep_ms;
        st->sweep_bytes = c->sweep_bytes;
        st->update_ms = c->update_ms;
        st->update_bytes = c->update_bytes;
        st->precond_launches = c->precond_launches;
        st->precond_ms = c->precond_ms;
        st->precond_bytes = c->precond_bytes;
        st->precond_flops = c->precond_flops;
        st->resid_launches = c->resid_launches;
        st->resid_ms = c->resid_ms;
        st->resid_bytes = c->resid_bytes;
        st->graph_captures = c->graph_captures;
        st->precond_layout = c->dst_layout;
        st->precond_tune_ms = c->dst_tune_ms;
        st->stencil_cpt = c->shape_cpt;
        st->stencil_depth = c->shape_depth;
        st->stencil_blocks = c->shape_target;
        st->tune_ms = c->tune_ms;
        if (fused) {
            // no solve ran here: the launch statistics and phase times in
            // the context are the forward pass's
            const int32_t layout = st->precond_layout, cpt = st->stencil_cpt, depth = st->stencil_depth;
            const int64_t blocks = st->stencil_blocks;
            std::memset(st, 0, sizeof(*st));
            st->precond_layout = layout;
            st->stencil_cpt = cpt;
            st->stencil_depth = depth;
            st->stencil_blocks = blocks;
            st->graph_captures = c->graph_captures;
            st->max_relres = rep.max_relres;
        }
    }
    if (!rep.converged) return set_err(c, FSIC_ENOCONV, "an adjoint Poisson solve missed tol within max_iter");
    return FSIC_OK;
}


fsic_status fsic_backward(fsic_ctx *c, const double *grad_e, double *const *dE_da, fsic_stats *st) {
    if (!c) return FSIC_EINVAL;
    if (!c->tape) return set_err(c, FSIC_ENOTAPE, "backward needs a forward pass with FSIC_KEEP_TAPE");
    if (!dE_da) return set_err(c, FSIC_EINVAL, "dE_da is required");
    for (int k = 0; k < c->nsys; ++k)
        if (!dE_da[k]) return set_err(c, FSIC_EINVAL, "dE_da[k] is required for every system");
    BwdState bs;
    fsic_status e = backward_enqueue(c, false, bs);
    if (e) return e;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return backward_finish(c, false, grad_e, dE_da, st, bs);
}

}  // extern "C"
