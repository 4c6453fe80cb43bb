// Internal declarations shared by the HIP kernels and the host runtime of
// the FLOSIC SIC library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsic {

constexpr int kMaxRadius = 6;    // fd_order <= 12
constexpr int kMaxOrb = 128;     // orbitals per spin channel
constexpr int kMaxL = 8;         // multipole order
constexpr int kMaxLM = (kMaxL + 1) * (kMaxL + 1);

// Stencil tile: 32 (x) by 8*cpt (y) columns per 256-thread block, marching in z.
constexpr int kTX = 32;
// Pointwise tile: 256 threads x 16 nodes (few partial sums per orbital, so
// the blocks that re-add them stay cheap).
constexpr int kPW = 4096;

// Device status bits (first error wins in the host's reading order).
enum : int {
    kStVacuum = 1,
    kStSingular = 2,
    kStNonFinite = 4,
};

// One Poisson problem (one orbital density) in a batched solve.
struct OrbDesc {
    int nx, ny, nz;
    int tiles_x, tiles_y, tiles_z, zc;  // stencil tiling (zc: planes per z-chunk)
    int nt7, base7;                     // stencil partial-sum slots
    int nt8, base8;                     // pointwise partial-sum slots
    long long off;                      // element offset of this orbital's fields
    long long goff;                     // element offset of its ghost values
    double inv_h2;
    double h;
    double origin[3];
    double centre[3];
    int chan;                           // spin channel (for the moment tables)
    int nt9, base9;                     // spectral-preconditioner partial-sum slots (x-pass panels)
    int dst_s[3];                       // sine-matrix offsets (x, y, z) in the spectral table
    int dst_g[3];                       // eigenvalue-symbol offsets (x, y, z) in the spectral table
    int pad;
};


// Work item of a block: orbital and tile index; orb < 0 means idle block.
struct Item {
    int orb, tile;
};
// Work lists of the spectral-preconditioner passes (see dst.hip); fast: 1
// persistent split-bf16 kernels with 128-column panels; 2 the same with
// 64-column panels; 3 64-column panels with the sine matrix rounded to bf16
// (no S_lo term), for axes whose split sine matrix does not fit the LDS
// (0: no variant fits; such batches are solved without the preconditioner).
// np: largest axis padded to 32; blocks: persistent blocks per pass.
struct DstItems {
    const Item *x, *y, *z;
    int nx, ny, nz;
    int fast, np, blocks;
    const Item *xy;  // fused x-y units (orbital, z plane), or null
    int nxy, two;    // their count; two: separate x and y sine matrices in LDS
    int xyvec;       // every nx and orbital offset is a multiple of 4
    int npxy;        // largest padded in-plane axis (LDS layout of the fused kernel)
    int zocc2;       // z pass: 64-column panels, two blocks per compute unit
    int xyocc2;      // fused x-y passes two blocks per compute unit (where the plane fits)
    int pv;          // the inverse pass reads p_old before its products (else at the store)
};

// Output of the last transform pass when it forms the next search
// direction of preconditioned CG directly: p_k = z_k + beta p_{k-1},
// beta = r_k.z_k / r_{k-1}.z_{k-1} per orbital from the z pass's partial
// sums (slots base9 .. base9 + nt9 of each orbital), or p_k = z_k when first.
struct PcgOut {
    const float *pold;   // p_{k-1} (not read when first)
    const double *rzc;   // r_k.z_k partial sums
    const double *rzp;   // r_{k-1}.z_{k-1} partial sums
    int first;           // 1: beta = 0 (first iteration of a restart cycle)
    // mixed restart cycles: an orbital with pz[o] <= li (the cycle's local
    // iteration of this application) is paused for the rest of the cycle
    // and skipped like a converged one (pz null: none)
    const int *pz;
    int li;
};

// panel columns of a fast transform variant's x and y passes (the z pass
// uses 64-column panels in every variant)
inline int dst_panel_cols(int variant) { return variant == 1 ? 128 : 64; }
// longest padded axis a variant's kernels are sized for
inline int dst_variant_npmax(int variant) { return variant == 1 ? 128 : (variant == 2 ? 160 : 192); }

struct Coeffs {
    double c[kMaxRadius + 1];  // unit-spacing second-difference weights
    int cpt;                   // stencil tile: 32 x 8*cpt columns (1, 2 or 4; 1 and 4 only for p = 6)
    int depth;                 // planes fetched ahead in the z march (2; 1, 3, 4 only for p = 6)
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// Workgroup barrier that orders LDS traffic only: this wave's LDS operations
// complete (lgkmcnt(0)), then s_barrier.  Unlike __syncthreads() it does not
// wait for outstanding global loads, so the next plane's prefetch stays in
// flight across the barrier.
__device__ __forceinline__ void lds_barrier() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt/expcnt: no wait; lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the 256 threads of a block; every thread gets the same value, in
// a fixed order (bitwise reproducible).  sbuf: 4 doubles of shared memory.
__device__ __forceinline__ double block_sum256(double v, double *sbuf) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sbuf[w] = v;
    __syncthreads();
    double s = (sbuf[0] + sbuf[1]) + (sbuf[2] + sbuf[3]);
    return s;
}

// Fixed-order sum of n partial sums (n arbitrary) by a 256-thread block.
__device__ __forceinline__ double sum_partials(const double *p, int n, double *sbuf) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += p[i];
    return block_sum256(v, sbuf);
}

// Block-to-item table order: block b runs on XCD b % 8; items are split in 8
// contiguous ranges so that neighbouring tiles share an XCD (and its L2).
inline int xcd_item_of_block(int b, int nblocks) {
    const int per = nblocks / 8;
    return (b % 8) * per + b / 8;
}

}  // namespace fsic
