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
// Work lists of the three spectral-preconditioner passes (see dst.hip);
// fast: 0 fp32 kernels (32-column panels); 1 persistent split-bf16 kernels
// with 128-column panels; 2 the same with 64-column panels; 3 64-column
// panels with the sine matrix rounded to bf16 (no S_lo term), for axes whose
// split sine matrix does not fit the LDS.  np: largest axis padded to 32;
// blocks: persistent blocks per pass.
struct DstItems {
    const Item *x, *y, *z;
    int nx, ny, nz;
    int fast, np, blocks;
    const Item *xy;  // fused x-y units (orbital, z plane), or null
    int nxy, two;    // their count; two: separate x and y sine matrices in LDS
    int xyvec;       // every nx and orbital offset is a multiple of 4
    int npxy;        // largest padded in-plane axis (LDS layout of the fused kernel)
    int zocc2;       // z pass: 64-column panels, two blocks per compute unit
};

// panel columns of a fast transform variant
inline int dst_panel_cols(int variant) { return variant == 1 ? 128 : (variant ? 64 : 32); }

struct Coeffs {
    double c[kMaxRadius + 1];  // unit-spacing second-difference weights
    int cpt;                   // stencil tile: 32 x 8*cpt columns (1, 2 or 4; 1 and 4 only for p = 6)
    int depth;                 // planes fetched ahead in the z march (2; 1, 3, 4 only for p = 6)
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

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
