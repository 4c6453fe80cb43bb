// Operator applications on the z-marching stencil: L u and the Kohn-Sham
// Hamiltonian -1/2 L psi + v psi (Sec. II.A, Sec. II.C).
#include "zmarch.h"

namespace fsic {

template <typename T>
hipError_t launch_apply(int radius, const Coeffs &c, const Item *items, int nitems,
                        const OrbDesc *orb, const T *u, T *Lu, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    PolApply<T> pol{items, orb, u, Lu, false};
#define CALL(P, C, DD) hipLaunchKernelGGL((k_zmarch<T, P, C, DD, PolApply<T>>), dim3(nitems), dim3(256), 0, s, pol, c)
    FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_hamiltonian(int radius, const Coeffs &c, const Item *items, int nitems,
                              const OrbDesc *orb, const double *psi, const double *v, double *out,
                              hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    PolHam<double> pol{items, orb, psi, v, out, false};
#define CALL(P, C, DD) hipLaunchKernelGGL((k_zmarch<double, P, C, DD, PolHam<double>>), dim3(nitems), dim3(256), 0, s, pol, c)
    FSIC_RADIUS_SWITCH(radius, CALL)
#undef CALL
    return hipGetLastError();
}

template hipError_t launch_apply<double>(int, const Coeffs &, const Item *, int, const OrbDesc *,
                                         const double *, double *, hipStream_t);
template hipError_t launch_apply<float>(int, const Coeffs &, const Item *, int, const OrbDesc *,
                                        const float *, float *, hipStream_t);

}  // namespace fsic
