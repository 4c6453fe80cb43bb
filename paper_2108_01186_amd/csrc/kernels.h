// Host-side launchers of the HIP kernels (internal to the library).
#pragma once

#include "common.h"

namespace fsic {

// ----------------------------------------------------------------------------
// stencil.hip: z-marching star stencil and conjugate-gradient sweeps
// ----------------------------------------------------------------------------

// Lu = L u (zero ghosts) for the orbitals of an item table.
template <typename T>
hipError_t launch_apply(int radius, const Coeffs &c, const Item *items, int nitems,
                        const OrbDesc *orb, const T *u, T *Lu, hipStream_t s);

// out = -1/2 L psi + v psi for the orbitals of an item table (v: [M], shared).
hipError_t launch_hamiltonian(int radius, const Coeffs &c, const Item *items, int nitems,
                              const OrbDesc *orb, const double *psi, const double *v, double *out,
                              hipStream_t s);

// Arguments of one CG iteration over a batch of orbitals.
template <typename T>
struct CGIter {
    const Item *items7;  // stencil items
    int nitems7;
    const Item *items8;  // pointwise items
    int nitems8;
    const OrbDesc *orb;
    T *R;               // residual
    T *P;               // search direction: p_k before the update of iteration k, p_{k+1} after
                        // (preconditioned CG: p_k written by the sweep of iteration k)
    T *Pold;            // preconditioned CG: p_{k-1}
    float *Z;           // preconditioned CG: z_k = M^{-1} r_k
    double *partRZ;     // preconditioned CG: [2*tot9] r.z partial sums, by iteration parity
    int tot9;
    T *Q;               // K p
    T *X;               // solution (FP64 path) or FP32 correction (mixed path)
    const double *B64;  // right-hand side (mixed restart cycles' residual pass)
    double *part7;      // [3*tot7] p.q, r.q and q.q partial sums of the sweep (three blocks of tot7)
    int tot7;
    double *part8;      // [2*tot8] r.r partial sums, by iteration parity
    double *partRU;     // [tot7]   FP64-residual partial sums
    int tot8;
    int *done;          // per orbital: 0 iterating, 1 converged, 2 paused until the next FP64 check
    int *iters;         // per orbital: iterations at convergence
    int *rs_iter;       // per orbital: iteration that restarts CG from the FP64 residual (or null)
    int *nact;          // per orbital: active sweeps [norb] then active updates [norb]
    int *nsamp;         // same layout for the profiled launches only (null: not profiled)
    int *ndone;         // orbitals marked converged (counted once each), or null
    int norb;
    double *rrfin;      // per orbital: residual norm^2 at convergence
    const double *bb;   // per orbital: ||b||^2
    double tol2;        // tol^2
};

// One stencil sweep: q = K p_k = -L p_k with partial sums of p.q, r.q, q.q.
//   k: iteration; cur_from_ru: r_k.r_k is in partRU rather than part8;
//   check: test convergence on r_k.r_k first.  p_k is read from R when the
//   recursion (re)starts at k (k == 0 or a restart after a pause).
template <typename T>
hipError_t launch_cg_stencil(int radius, const Coeffs &c, const CGIter<T> &a, int k,
                             int cur_from_ru, int check, hipStream_t s);

// One pointwise update: x += alpha p; r -= alpha q; r.r partials; and the
// next search direction p = r + beta p with beta from the sweep's partials
// (|r - alpha q|^2 = r.r - 2 alpha r.q + alpha^2 q.q).
//   x_first: x is not read (x = alpha p).
template <typename T>
hipError_t launch_cg_update(const CGIter<T> &a, int k, int cur_from_ru, int x_first,
                            hipStream_t s);

// Preconditioned CG sweep: p_k = z_k + beta p_{k-1} (beta = r_k.z_k /
// r_{k-1}.z_{k-1}; 0 when k == 0 or restart), q = -L p_k, p.q partials.
//   cur_from_ru: r_k.r_k is in partRU; pause: a converged FP32 recursion
//   waits for the FP64 check (done = 2) instead of finishing.
template <typename T>
hipError_t launch_pcg_stencil(int radius, const Coeffs &c, const CGIter<T> &a, int k,
                              int cur_from_ru, int restart, int pause, hipStream_t s);

// Preconditioned CG update: alpha = r_k.z_k / p.q; x += alpha p; r -= alpha q;
// r.r partials.  x_first: x is not read (x = alpha p).
template <typename T>
hipError_t launch_pcg_update(const CGIter<T> &a, int k, int x_first, hipStream_t s);

// Mixed-precision preconditioned CG (restart cycles of FP32 iterations
// checked on the FP64 residual).  Sweep of iteration k: q_k = -L p_k with the
// p_k.q_k partials in part7 slice (k & 1); p_k was formed by the last
// preconditioner pass.
hipError_t launch_pcg_sweep(int radius, const Coeffs &c, const CGIter<float> &a, int k, const int *pz,
                            int li, hipStream_t s);

// Update after the sweep of iteration k: alpha_k = r_k.z_k / p_k.q_k,
// r_{k+1} = r_k - alpha_k q_k with its r.r partials (part8 slice (k+1) & 1);
// xmode 1: x = alpha_k p_k, 2: x += alpha_k p_k (0: x untouched; the residual
// pass adds the last steps itself).  li: the cycle's local index of
// iteration k + 1; orbitals paused before it (pz[o] < li) are skipped.
hipError_t launch_pcg_rupdate(const CGIter<float> &a, int k, int xmode, const int *pz, int li,
                              hipStream_t s);

// Pause check after that update: an orbital not paused before local
// iteration li whose r_{k+1}.r_{k+1} <= ftol2 ||b||^2 is paused from li on
// (pz[o] = li) for the rest of the cycle; the residual pass that closes the
// cycle decides its convergence.
hipError_t launch_pause_check(const CGIter<float> &a, int k, double ftol2, int *pz, int li, hipStream_t s);

// p[i] = v for n ints (a fill kernel, usable inside a captured graph)
hipError_t launch_fill_int(int *p, int n, int v, hipStream_t s);
// up to kIntFills integer arrays set to one value each, in one launch
constexpr int kIntFills = 8;
struct IntFills {
    int *p[kIntFills];
    int n[kIntFills];
    int v[kIntFills];
    int count;
};
hipError_t launch_fill_ints(const IntFills &f, hipStream_t s);

// FP64 residual of x = x64 + x32 + alpha_a p_a + alpha_b p_b at the end of a
// restart cycle (alpha_j = r_j.z_j / p_j.q_j from the partials of
// iterations ka and kb, p_a and p_b the FP32 directions of those
// iterations): res = b + L x; writes xnew = x, r32 = (float) res and the
// res.res partials.  Null x64 (x32) stands for zero.  Orbitals with
// done == 1 are skipped.
struct ResStep {
    const double *X64;
    const float *X32;
    const float *Pa, *Pb;
    int ka, kb;
    double *X64new;
    float *R32;
    const int *pz;  // paused orbitals: a step of local iteration >= pz[o] did not run
    int la, lb;     // local iterations of ka and kb
};
hipError_t launch_res_steps(int radius, const Coeffs &c, const CGIter<float> &a, const ResStep &rs,
                            hipStream_t s);

// v_o = w_o + sum_q Q[first + o][q] U_q (q < (lmax + 1)^2) for N
// consecutive orbitals on one grid of n[0] x n[1] x n[2] nodes: U holds the
// first octant of the grid's unit-moment boundary solutions (q-major,
// ceil(n/2) per axis, x fastest; the rest follows from their parities under
// the axis reflections); W and V point at the first orbital
hipError_t launch_bc_combine(int N, const int *n, int lmax, const double *Q, int first, const double *U,
                             const double *W, double *V, hipStream_t s);
// Uc = the first octant of nlm full-grid fields U (the layout launch_bc_combine reads)
hipError_t launch_octant_pack(int nlm, const int *n, const double *U, double *Uc, hipStream_t s);
// The host checks' inputs of up to kChkPack channels, packed one after the
// other for one copy to the host: channel e's G (N x N), info (2) and
// rho(a) (N) from small + so[e] (+ oG, oI, oR) to out + q[e].
constexpr int kChkPack = 32;
struct ChkPack {
    int n;
    long long oG, oI, oR;
    int N[kChkPack];
    long long so[kChkPack], q[kChkPack];
};
hipError_t launch_pack_checks(const ChkPack &p, const double *small, double *out, hipStream_t s);
// The end of a mixed solve in one launch: the final x as launch_take_x, then
// per orbital the final FP64 residual (partRU partials), iters = nact[0..norb)
// and the statistics stage of launch_stage_stats.
hipError_t launch_mixed_finish(int nitems8, const Item *items8, const OrbDesc *orb, const int *fin, int fallback,
                               double *X, const double *Xb, int norb, const double *partRU, const int *nact,
                               const int *done, const double *bb, int *iters, double *ptrue, double *stage,
                               hipStream_t s);
// the statistics of a solve gathered for one transfer: stage holds 8 norb
// ints (iters, nact[6 norb], done) and then 2 norb doubles (ptrue, bb)
hipError_t launch_stage_stats(int norb, const int *iters, const int *nact, const int *done,
                              const double *ptrue, const double *bb, double *stage, hipStream_t s);
// Final x of the mixed restart cycles: X[o] = Xb[o] for the orbitals whose
// result is in the second buffer (fin[o] == 1, or fallback == 1 where
// fin[o] < 0: not converged).
hipError_t launch_take_x(int nitems8, const Item *items8, const OrbDesc *orb, const int *fin, int fallback,
                         double *X, const double *Xb, hipStream_t s);

// FP64 residual of x64 (+ x32): res = b + L (x64 + x32); writes x64new =
// x64 + x32, r32 = (float) res (if r32 != null), res.res partials.  With
// x32, a null x64 stands for x64 = 0 (the first restart of a mixed solve).
hipError_t launch_true_residual(int radius, const Coeffs &c, const Item *items7, int nitems7,
                                const OrbDesc *orb, const int *done, const double *X64,
                                const float *X32, const double *B, double *X64new, float *R32,
                                double *partRU, hipStream_t s);

// mixed precision: x64 += x32 (orbitals not yet converged)
hipError_t launch_mixed_accumulate(int nitems8, const Item *items8, const OrbDesc *orb,
                                   const int *done, double *X64, const float *X32, hipStream_t s);

// mixed precision: mark orbitals whose FP64 residual (partRU) meets tol;
// counts them in *ndone (if not null), stores xfin in fin[o] (if not null)
// and resets the pause of the others (pz[o] = cyc, if pz is not null)
hipError_t launch_ru_check(int norb, const OrbDesc *orb, const double *partRU, const double *bb,
                           double tol2, int k, int *done, int *iters, double *rrfin, int *rs_iter,
                           int *ndone, int *fin, int xfin, int *pz, int cyc, hipStream_t s);

// per orbital: out[o] = sum of partials (stencil layout if stencil_layout,
// else pointwise slot range starting at the parity-0 block)
hipError_t launch_reduce_partials(int norb, const OrbDesc *orb, const double *part,
                                  int stencil_layout, double *out, hipStream_t s);

// ----------------------------------------------------------------------------
// aar.hip: alternating Anderson-Richardson iteration
// ----------------------------------------------------------------------------

constexpr int kAarM = 7;                        // history columns
constexpr int kAarG = kAarM * (kAarM + 1) / 2;  // Gram entries (upper triangle)
constexpr int kAarD = kAarG + kAarM;            // plus right-hand sides

struct AarBufs {
    const Item *items8;
    const OrbDesc *orb;
    const int *done;
    const float *F;       // f = M^{-1} r of the current iterate
    float *Fprev;         // f of the previous iterate
    float *Fh;            // [m][fields] f differences (ring)
    double *Xh;           // [m][fields] x steps (ring)
    double *X;            // iterate
    double *gamma;        // [norb][kAarM] extrapolation weights
    double *partD;        // [tot8][kAarD] per-tile Gram partials
    long long fields;     // elements per history column
    int m;                // history length (kAarM)
};

// Records f_k - f_{k-1} (hist) and, with dots, the per-tile partials of
// F^T F and F^T f over the nh valid columns.
hipError_t launch_aar_dots(const AarBufs &a, int nitems8, int k, int nh, int hist, int dots,
                           hipStream_t s);
// gamma of every unconverged orbital from the partials.
hipError_t launch_aar_solve(const AarBufs &a, int norb, int nh, hipStream_t s);
// x += Richardson or Anderson step; the step becomes history column k.
hipError_t launch_aar_step(const AarBufs &a, int nitems8, int k, int nh, double omega, double beta,
                           bool anderson, int hist, hipStream_t s);

// ----------------------------------------------------------------------------
// dst.hip: spectral (type-I sine transform) preconditioner
// ----------------------------------------------------------------------------

// LDS bytes of a fast transform block for axes padded to np nodes, panels
// of pc columns, with (slo) or without the sine matrix's low bf16 part.
size_t dst_fast_lds(int np, int pc, bool slo);

// LDS bytes of the fused x-y transform block for in-plane axes padded to np
// nodes; two: the x and y sine matrices differ somewhere in the batch.
size_t dst_xy_lds(int np, bool two);

// The z pass of a fused-plane batch with all axes padded to np can run two
// 64-column blocks per compute unit.
bool dst_z_occ2(int np);
// The fused in-plane passes of planes padded to np (two: separate x and y
// sine matrices) can run two blocks per compute unit.
bool dst_xy_occ2(int np, bool two);

// Allows the fast transform kernels of a variant (1..3, see DstItems) their
// dynamic LDS for axes up to np, and the fused x-y kernel (npxy > 0: in-plane
// axes up to npxy) its own.
hipError_t dst_setup(int np, int variant, int npxy, bool two);

// z = M^{-1} r (float) for the orbitals of the work lists with done == 0,
// through the float work array; r.z partial sums into rz[base9 + panel].
// tab: sine matrices and eigenvalue symbols (offsets in OrbDesc); cnt (may
// be null): per orbital, applications that did work.
template <typename T>
hipError_t launch_dst_precond(const DstItems &di, const OrbDesc *orb, const int *done,
                              const float *tab, const T *r, float *work, float *z, double *rz,
                              int *cnt, hipStream_t s);

// The same application for the mixed CG, whose last pass writes the next
// search direction p = M^{-1} r + beta p_old (po) instead of z.
hipError_t launch_dst_pcg(const DstItems &di, const OrbDesc *orb, const int *done, const float *tab,
                          const float *r, float *work, float *p, double *rz, const PcgOut &po, int *cnt,
                          hipStream_t s);

// ----------------------------------------------------------------------------
// multipole.hip: Dirichlet values from a multipole expansion, right-hand side
// ----------------------------------------------------------------------------

struct HarmTables {
    double norm[kMaxLM];   // real orthonormal Y_lm normalisation (incl. sqrt 2 for m != 0)
    double gfac[kMaxLM];   // 4 pi / (2l + 1)
};

// Harmonic contractions of one channel's orbitals on the matrix cores (the
// harmonics built once per node for all of them): mode 0, the moments
// Q[o][lm] = dV sum_r rho_o(r) r^l Y_lm (rho = src^2 if square); mode 1, the
// adjoint boundary term zt[o][lm] = sum_ghost gfac_lm Y_lm / r^(l+1)
// (C^T w_o)_ghost with src = w (square 0).  Work items: per block a
// contiguous range of 64-node chunks of one channel and the offset of its
// partial tile; per channel its partial tiles, which the second kernel adds
// in item order (a fixed order: the result does not depend on timing).
struct HcItem {
    int first, count;  // orbitals of the channel
    int t0, t1;        // chunks [t0, t1) of 64 nodes (grid nodes or ghosts)
    long long poff;    // element offset of this block's partial tile
    int ot0, ot1;      // 16-orbital tiles [ot0, ot1) of the channel (expansions; contractions take all)
};
// 16-orbital tiles per expansion block (its coefficient rows in LDS)
constexpr int kHcExpandTiles = 2;
struct HcChan {
    int first, count;  // orbitals of the channel
    int nparts;        // its partial tiles, consecutive from poff
    long long poff;
};
// rows of a partial tile: (kMaxL + 1)^2 harmonics padded to 16; columns: the
// channel's orbitals padded to 16
constexpr int kHcRows = (kMaxLM + 15) / 16 * 16;
// Blocks of a harmonic kernel the current device holds at once (blocks per
// compute unit from the occupancy query, times the compute units): kind 0
// the contraction over grid nodes, 1 over ghosts, 2 the expansion over
// ghosts, 3 over grid nodes.  Cached per device; at least 1.
int harm_slots(int kind, int lmax);
hipError_t launch_harm_contract(int mode, int lmax, const HarmTables &ht, const Coeffs &c, int radius,
                                const OrbDesc *orb, const long long *ghost_count, const HcItem *items,
                                int nitems, const HcChan *chans, int nchans, int max_count,
                                const double *src, int square, double *part, double *out, hipStream_t s);

// Harmonic expansions of one channel's orbitals on the matrix cores: mode 0,
// the ghost values g_o = sum_lm gfac_lm Q[o][lm] Y_lm / r^(l+1) on the face
// slabs (written to out = G); mode 1, the multipole part of the adjoint
// field, W_o += dV sum_lm zt[o][lm] r^l Y_lm on the grid.  items: ghost
// chunks (mode 0) or node chunks (mode 1), each with at most
// kHcExpandTiles orbital tiles.
hipError_t launch_harm_expand(int mode, int lmax, const HarmTables &ht, int radius, const OrbDesc *orb,
                              const long long *ghost_count, const HcItem *items, int nitems,
                              const double *C, double *out, hipStream_t s);

// In place of the ghost values G, the boundary term of the interior nodes
// within reach of each face: layer e of a face column becomes
// sum_{d=1}^{P-e} c_(e+d) g_d / h^2 (the right-hand side then adds one value
// per face in reach).  max_cols: most face columns of one orbital,
// 2 (nx ny + ny nz + nx nz).
hipError_t launch_bterm(int radius, const Coeffs &c, int norb, const OrbDesc *orb, long long max_cols,
                        double *G, hipStream_t s);

// b = scale * rho + (boundary term from launch_bterm, if G != null); writes B,
// R64 or R32 = b, optionally X64 = 0, and b.b partials into part8 slot 0.
hipError_t launch_rhs(int radius, const Coeffs &c, const Item *items8, int nitems8,
                      const OrbDesc *orb, const double *src, int square, double scale,
                      const double *G, double *B, double *R64, float *R32, double *X64zero,
                      double *part8, hipStream_t s);

// ----------------------------------------------------------------------------
// xc.hip: LSDA at full polarisation, Slater average, energies, adjoint source
// ----------------------------------------------------------------------------

hipError_t launch_xc_pointwise(long long count, const double *rho, double floor, double *ex,
                               double *ec, double *vx, double *vc, hipStream_t s);

struct ChanDesc {
    int N;                 // orbitals
    int first_orb;         // index of orbital 0 in the batch
    long long M;
    long long off;         // element offset of orbital 0's fields (phi, v)
    int nx, ny, nz;
    int nblk;              // blocks of the channel's pointwise passes
    int blk_base;          // first partial slot (per orbital: [N][nblk])
    int pad;
    double h;
    double vscale;
    double *vsic;          // output V_SIC or null
};

// U and X partials per block and orbital, V_SIC
hipError_t launch_sic_average(int nchan, const ChanDesc *chan, int nblk_total,
                              const int *blk_chan, const double *PHI, const double *V,
                              double floor, double *partU, double *partX, hipStream_t s);

// per orbital U = dV/2 sum partU, X = dV sum partX; per channel E = -sum(U + X)
hipError_t launch_sic_energy(int nchan, const ChanDesc *chan, const double *partU,
                             const double *partX, double *U, double *X, double *Echan,
                             hipStream_t s);

// ----------------------------------------------------------------------------
// fo.hip: FOD interpolation, Gram matrix, Loewdin, Fermi-Loewdin GEMM
// ----------------------------------------------------------------------------

struct FodCell {
    int i0[3];    // lower-left node of the 4-node stencil is i0 - 1
    int pad;
    double t[3];  // fractional position in [0, 1)
};

// u[i][a] = psi_a(a_i), du[i][a][3]; rhoa[i]; T[i][a]; sets status on vacuum
hipError_t launch_interp(int K, int N, int nx, int ny, int nz, double h, const double *psi,
                         const FodCell *cells, double floor, double *u, double *du,
                         double *rhoa, double *T, int *status, bool fd_gradient, hipStream_t s);

// G = dV psi psi^T (MFMA FP64), partial sums then reduction; nonortho = max|G - I|
// blocks of a node-range split whose N x N partial tiles fit in cap doubles
int grid_blocks(int N, long long M, size_t cap);

hipError_t launch_gram(int N, long long M, double dV, const double *psi, double *partG, size_t cap,
                       double *G, hipStream_t s);

// Loewdin step on one block: S = T G T^T; S = U diag(lam) U^T (parallel
// Jacobi); Z = S^{-1/2}; Q = Z T.  work: device scratch of >= 2 N^2 doubles.
hipError_t launch_lowdin(int N, const double *T, const double *G, double *S, double *lam,
                         double *U, double *Z, double *Qm, double *work, double eig_floor,
                         int *status, double *info, hipStream_t s);

// Loewdin step of up to kLowdinBatch channels in one launch (one workgroup
// each): channel b has N[b] orbitals and its small arrays at small + so[b]
// plus the offsets below; scratch of wstride >= 3 N^2 doubles per channel.
constexpr int kLowdinBatch = 64;
struct LowdinBatch {
    int n;
    int N[kLowdinBatch];
    long long so[kLowdinBatch];
};
struct LowdinOffsets {
    long long T, G, S, lam, U, Z, Q, info;
};
hipError_t launch_lowdin_batch(const LowdinBatch &lb, double *small, const LowdinOffsets &off,
                               double *work, long long wstride, double eig_floor, int *status,
                               hipStream_t s);

// out[i][m] = sum_a A[i][a] psi[a][m]  (MFMA FP64), N <= 128
hipError_t launch_orb_gemm(int N, long long M, const double *A, const double *psi, double *out,
                           hipStream_t s);
// the same with fp32 operands and fp32 accumulation on the matrix cores
hipError_t launch_orb_gemm32(int N, long long M, const double *A, const double *psi, double *out,
                             hipStream_t s);

// Nodes of one channel per block of the Slater average (its partial sums
// come one per such block).
constexpr int kSicTile = 1024;

// B[i][a] = sum_m Gam_i(m) psi_a(m) with Gam_i = 2 dV phi_i omega_i,
// omega_i = -((v_i + w_i) / 2 + vxc(phi_i^2)), contracted on the matrix cores
// (FP64); for more than 32 orbitals Gam is first written to Gam (N x M; may
// be W) by an elementwise pass, for at most 32 it is built on the fly
hipError_t launch_adjoint_contract(int N, long long M, double dV, const double *PHI, const double *V,
                                    const double *W, const double *psi, double floor, double *partB,
                                    size_t cap, double *Bm, double *Gam, hipStream_t s);

// reverse mode through Q = S^{-1/2} T, S = T G T^T, T = u/|u|, u = psi(a):
// dEda[i][d] = gscale * sum_a Gam_u[i][a] dpsi_a(a_i)/da_d
// the reverse Loewdin step of up to kLowdinBatch channels, one workgroup
// each (channel b: N[b] orbitals, small arrays at small + so[b] plus the
// offsets, B at Bm + b bstride, scratch of wstride >= 4 N^2 doubles at
// work + b wstride); dE/da also to packed + go[b]
struct LowdinBwdBatch {
    int n;
    int N[kLowdinBatch];
    long long so[kLowdinBatch], go[kLowdinBatch];
};
struct LowdinBwdOffsets {
    long long T, G, lam, U, Z, rhoa, du, dEda;
};
hipError_t launch_lowdin_backward_batch(const LowdinBwdBatch &lb, const double *Bm, long long bstride, double *small,
                                        const LowdinBwdOffsets &off, double *work, long long wstride, double *packed,
                                        hipStream_t s);
// ----------------------------------------------------------------------------
// noalloc.hip: the Fermi-Loewdin step on a file-scope scratch array
// ----------------------------------------------------------------------------

// Device address and size (doubles) of the current device's scratch array.
hipError_t noalloc_scratch(double **ptr, size_t *doubles);

// interpolation, Gram matrix, Loewdin step and phi = Z T psi of one channel
// with every intermediate in the scratch array (synchronous on s); *hstatus
// receives the device status bits
hipError_t noalloc_flo(int N, const int n[3], double h, const double *psi, const FodCell *cells,
                       double rho_floor, double *T, double *G, double *S, double *Z, double *phi,
                       int *hstatus, hipStream_t s);

}  // namespace fsic
