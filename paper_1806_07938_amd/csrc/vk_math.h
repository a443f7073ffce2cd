// von Karman structure function in float64 (App. A.2), usable on host and device.
//
//   D(r) = c_D (L0/r0)^(5/3) B(x),  x = 2 pi r / L0,
//   B(x) = 1 - (2^(1/6) / Gamma(5/6)) x^(5/6) K_{5/6}(x),
//   c_D  = Gamma(11/6) Gamma(5/6) pi^(-8/3) (24/5 Gamma(6/5))^(5/6),
//
// with the readings (r/L0)^(5/6) for the printed (r0/L0)^(5/6) (the bracket must
// vanish at r = 0) and the exact constant for the printed 0.17253.
//
// B is evaluated without cancellation at small x from the ascending series of
// K_nu = pi/(2 sin nu pi) (I_-nu - I_nu) (DLMF 10.27.4, 10.25.2): with
// nu = 5/6, y = x^2/4, Gamma(nu) Gamma(1-nu) = pi / sin(nu pi),
//
//   B(x) = x^(2 nu) sum_{k>=0} b_k y^k - sum_{k>=1} a_k y^k,
//   a_0 = 1,  a_k = a_{k-1} / (k (k - nu)),
//   b_0 = Gamma(1-nu) 2^(-2 nu) / Gamma(1+nu),  b_k = b_{k-1} / (k (k + nu)),
//
// (the a_0 term cancels the leading 1 exactly) for x <= 2, and for x > 2 from
// the integral K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt (DLMF 10.32.9)
// by the trapezoidal rule with step h = 1/8, which converges geometrically for
// this analytic integrand:
//
//   x^nu K_nu(x) = exp(nu ln x - x) h [1/2 + sum_m exp(-x (cosh(mh) - 1)) cosh(nu m h)].
#pragma once

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

#include <cmath>

namespace vk {

constexpr double NU = 5.0 / 6.0;
constexpr double TRAP_H = 0.125;
constexpr int NTRAP = 48;            // cosh(6) - 1 = 200: exp(-400) for x > 2
constexpr int NSERIES = 26;          // y <= 1: a_k y^k < 1e-50 by k = 26

struct Params {
    double Dscale;     // c_D (L0/r0)^(5/3)
    double xscale;     // 2 pi / L0
    double b0;         // Gamma(1-nu) 2^(-2 nu) / Gamma(1+nu)
    double cK;         // 2^(1-nu) / Gamma(nu)
};

struct Trap {
    double a[NTRAP];   // cosh(m h) - 1
    double b[NTRAP];   // cosh(nu m h)
};

inline Params make_params(double r0, double L0) {
    Params p;
    const double cD = std::tgamma(11.0 / 6.0) * std::tgamma(5.0 / 6.0) * std::pow(M_PI, -8.0 / 3.0)
                      * std::pow(24.0 / 5.0 * std::tgamma(6.0 / 5.0), 5.0 / 6.0);
    p.Dscale = cD * std::pow(L0 / r0, 5.0 / 3.0);
    p.xscale = 2.0 * M_PI / L0;
    p.b0 = std::tgamma(1.0 - NU) * std::pow(2.0, -2.0 * NU) / std::tgamma(1.0 + NU);
    p.cK = std::pow(2.0, 1.0 - NU) / std::tgamma(NU);
    return p;
}

inline Trap make_trap() {
    Trap t;
    for (int m = 0; m < NTRAP; ++m) {
        const double u = m * TRAP_H;
        const double sh = std::sinh(0.5 * u);
        t.a[m] = 2.0 * sh * sh;          // cosh(u) - 1 without cancellation
        t.b[m] = std::cosh(NU * u);
    }
    return t;
}

__host__ __device__ inline double bracket(double x, const Params& p, const double* ta, const double* tb) {
    if (!(x > 0.0)) return 0.0;
    if (x <= 2.0) {
        const double y = 0.25 * x * x;
        double ak = 1.0, bk = p.b0, yk = 1.0, sa = 0.0, sb = p.b0;
        for (int k = 1; k < NSERIES; ++k) {
            yk *= y;
            ak /= (k * (k - NU));
            bk /= (k * (k + NU));
            sa += ak * yk;
            sb += bk * yk;
        }
        return exp(2.0 * NU * log(x)) * sb - sa;
    }
    double s = 0.5;
    for (int m = 1; m < NTRAP; ++m) s += exp(-x * ta[m]) * tb[m];
    return 1.0 - p.cK * exp(NU * log(x) - x) * TRAP_H * s;
}

__host__ __device__ inline double structure(double dx, double dy, const Params& p, const double* ta,
                                            const double* tb) {
    return p.Dscale * bracket(p.xscale * sqrt(dx * dx + dy * dy), p, ta, tb);
}

}  // namespace vk
