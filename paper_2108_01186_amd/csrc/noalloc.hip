// Fermi-Loewdin orbitals of one spin channel without any allocation: the
// same kernels as fsic_op_flo (cubic interpolation at the FODs, Eq. 6-8 and
// Sec. II.B; Gram matrix, overlap and S^{-1/2}, Sec. I.B; phi = Z T psi),
// with every intermediate in one file-scope device array instead of memory
// the library allocates.  For callers that cannot allocate device memory.
//
// Every call on a GPU shares that GPU's copy of the array, and the array
// keeps the last call's contents: the status word is cleared at the start of
// each call (everything else is written before it is read), and calls that
// overlap on one GPU race.
#include <mutex>

#include "../../include/fsic.h"
#include "kernels.h"

namespace fsic {

namespace {

// layout of the scratch array, in doubles
constexpr size_t kNaSmall = (size_t)kMaxOrb * kMaxOrb * 10 + 2 * kMaxOrb + 8 + 3 * kMaxOrb + 8;
constexpr size_t kNaWork = 3 * (size_t)kMaxOrb * kMaxOrb;
constexpr size_t kNaCells = (size_t)kMaxOrb * sizeof(FodCell) / sizeof(double);
constexpr size_t kNaStatus = 8;
constexpr size_t kNaPartG = (size_t)1 << 21;  // Gram partial tiles: 16 MiB
constexpr size_t kNaDoubles = kNaSmall + kNaWork + kNaCells + kNaStatus + kNaPartG;

}  // namespace

// the scratch array (about 18 MiB per GPU, held until the process ends)
static __device__ __align__(256) double scratch[kNaDoubles];

namespace {

constexpr int kNaMaxDevices = 64;
std::mutex na_mu;
double *na_ptr[kNaMaxDevices] = {};

__global__ void k_clear_status(int *status) {
    if (threadIdx.x == 0) *status = 0;
}

// offsets of the small per-channel arrays (the layout fsic_op_flo uses)
constexpr size_t kNN = (size_t)kMaxOrb * kMaxOrb;
constexpr size_t oU = 0, oDU = kNN, oT = 4 * kNN, oG = 5 * kNN, oS = 6 * kNN, oEV = 7 * kNN,
                 oZ = 8 * kNN, oQ = 9 * kNN, oRHOA = 10 * kNN, oLAM = 10 * kNN + kMaxOrb,
                 oINFO = 10 * kNN + 2 * kMaxOrb;

}  // namespace

// Device address of the current device's scratch array, looked up once per
// device (with that device current); the host-side name of the array is not
// a device address.
hipError_t noalloc_scratch(double **ptr, size_t *doubles) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(na_mu);
    if (!na_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        na_ptr[dev] = static_cast<double *>(p);
    }
    *ptr = na_ptr[dev];
    *doubles = kNaDoubles;
    return hipSuccess;
}

// The no-allocation Fermi-Loewdin step: cells are the host-validated FOD
// cells (N of them), every output pointer may be null except that nothing
// useful happens without one.  Returns the device status bits in *hstatus.
hipError_t noalloc_flo(int N, const int n[3], double h, const double *psi, const FodCell *cells,
                       double rho_floor, double *T, double *G, double *S, double *Z, double *phi,
                       int *hstatus, hipStream_t s) {
    double *base = nullptr;
    size_t cap = 0;
    hipError_t e = noalloc_scratch(&base, &cap);
    if (e != hipSuccess) return e;
    double *small = base;
    double *work = small + kNaSmall;
    FodCell *dcells = reinterpret_cast<FodCell *>(work + kNaWork);
    int *status = reinterpret_cast<int *>(work + kNaWork + kNaCells);
    double *partG = work + kNaWork + kNaCells + kNaStatus;
    const long long M = (long long)n[0] * n[1] * n[2];
    const double dV = h * h * h;
    e = hipMemcpyAsync(dcells, cells, (size_t)N * sizeof(FodCell), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, status);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = launch_interp(N, N, n[0], n[1], n[2], h, psi, dcells, rho_floor, small + oU, small + oDU,
                          small + oRHOA, small + oT, status, false, s);
    if (e == hipSuccess) e = launch_gram(N, M, dV, psi, partG, kNaPartG, small + oG, s);
    if (e == hipSuccess)
        e = launch_lowdin(N, small + oT, small + oG, small + oS, small + oLAM, small + oEV, small + oZ,
                          small + oQ, work, 0.0, status, small + oINFO, s);
    if (e == hipSuccess && phi) e = launch_orb_gemm(N, M, small + oQ, psi, phi, s);
    const size_t NN = (size_t)N * N * sizeof(double);
    if (e == hipSuccess && T) e = hipMemcpyAsync(T, small + oT, NN, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && G) e = hipMemcpyAsync(G, small + oG, NN, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && S) e = hipMemcpyAsync(S, small + oS, NN, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && Z) e = hipMemcpyAsync(Z, small + oZ, NN, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hstatus, status, sizeof(int), hipMemcpyDeviceToHost, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    return e != hipSuccess ? e : e2;
}

}  // namespace fsic
