// Fully polarised LSDA of one FLO density, E_xc[rho_i, 0] of Eq. 1 (Sec. III):
// Slater exchange and the PW92 correlation interpolation at zeta = 1.
//   exchange: eps_x = -(3/4)(6/pi)^(1/3) rho^(1/3), v_x = (4/3) eps_x
//   correlation: G(rs) = -2A (1 + alpha1 rs) ln(1 + 1 / q1(rs)),
//     q1 = 2A (beta1 rs^(1/2) + beta2 rs + beta3 rs^(3/2) + beta4 rs^2),
//     A = 0.015545, alpha1 = 0.20548, beta1..4 = 14.1189, 6.1977, 3.3662, 0.62517;
//     v_c = eps_c - (rs/3) d eps_c / d rs (no zeta term at zeta = 1).
// The powers rho^(-1/3), rs^(-1/2) and the reciprocals are formed by Newton's
// method from single-precision starting values (two steps from a relative
// error of about 1e-7 reach double precision), so the only double-precision
// library call per density is the logarithm.
#pragma once

#include "kernels.h"

namespace fsic {

// (6/pi)^(1/3) and (3/(4 pi))^(1/3)
constexpr double kSixOverPiCbrt = 1.2407009817988000333;
constexpr double kRsCoef = 0.62035049089940001667;

// x^(-1/3), x > 0 in single-precision range: Newton's method for y^-3 = x,
// y <- y (4 - x y^3) / 3
__device__ __forceinline__ double newton_inv_cbrt(double x) {
    double y = (double)__builtin_amdgcn_exp2f(-(1.0f / 3.0f) * __builtin_amdgcn_logf((float)x));
#pragma unroll
    for (int k = 0; k < 2; ++k) y = y * (4.0 - x * (y * y * y)) * (1.0 / 3.0);
    return y;
}

// x^(-1/2): Newton's method for y^-2 = x, y <- y (3 - x y^2) / 2
__device__ __forceinline__ double newton_inv_sqrt(double x) {
    double y = (double)__builtin_amdgcn_rsqf((float)x);
#pragma unroll
    for (int k = 0; k < 2; ++k) y = y * (1.5 - 0.5 * x * (y * y));
    return y;
}

// 1/x: Newton's method for 1/y = x, y <- y + y (1 - x y)
__device__ __forceinline__ double newton_recip(double x) {
    double y = (double)__builtin_amdgcn_rcpf((float)x);
#pragma unroll
    for (int k = 0; k < 2; ++k) y = fma(y, fma(-x, y, 1.0), y);
    return y;
}

// energies per particle and potentials at one density; rho <= floor: all zero
__device__ __forceinline__ void lsda_pol(double rho, double floor, double &ex, double &ec, double &vx,
                                         double &vc) {
    if (!(rho > floor)) {
        ex = ec = vx = vc = 0.0;
        return;
    }
    constexpr double A = 0.015545, a1 = 0.20548;
    constexpr double b1 = 14.1189, b2 = 6.1977, b3 = 3.3662, b4 = 0.62517;
    const double y = newton_inv_cbrt(rho);  // rho^(-1/3)
    const double r13 = rho * (y * y);       // rho^(1/3)
    ex = -0.75 * kSixOverPiCbrt * r13;
    vx = -kSixOverPiCbrt * r13;
    const double rs = kRsCoef * y;
    const double is = newton_inv_sqrt(rs);  // rs^(-1/2)
    const double s = rs * is;               // rs^(1/2)
    const double q1 = 2.0 * A * (s * (b1 + s * (b2 + s * (b3 + s * b4))));
    const double q1p = A * (b1 * is + 2.0 * b2 + 3.0 * b3 * s + 4.0 * b4 * rs);  // d q1 / d rs
    const double u = newton_recip(q1);
    const double lg = log1p(u);
    const double q0 = -2.0 * A * (1.0 + a1 * rs);
    ec = q0 * lg;
    // q0 q1p / (q1 (q1 + 1)) with 1 / (q1 (q1 + 1)) = u^2 / (1 + u)
    const double dec = -2.0 * A * a1 * lg - q0 * q1p * (u * u) * newton_recip(1.0 + u);
    vc = ec - rs * dec * (1.0 / 3.0);
}

// v_x + v_c at one density
__device__ __forceinline__ double vxc_pol(double rho, double floor) {
    double ex, ec, vx, vc;
    lsda_pol(rho, floor, ex, ec, vx, vc);
    return vx + vc;
}

}  // namespace fsic
