// host_math.h -- host-side quantities of the run set-up shared by the 1D and
// 2D libraries: the speed-mixture weights of the g-particle loader and the
// mean of 1/beta over a Maxwellian (the weight factor Z of Eq. 5).
#pragma once

#include <cmath>

#include "slpic.h"

namespace slpic {

// <1/beta> over the Maxwell speed density sqrt(2/pi) s^2 exp(-s^2/2), speeds
// in thermal units, ut = v0/vt.  Eq. (11b): closed form of the split at ut.
// Eq. (11a): composite five-point Gauss-Legendre quadrature on [0, 40].
inline void step_mixture(double ut, double& Ps, double& Pf) {
    const double c = 0.7978845608028654;  // sqrt(2/pi)
    double e = std::exp(-0.5 * ut * ut);
    Ps = std::erf(ut / std::sqrt(2.0)) - c * ut * e;
    Pf = c * (ut * ut + 2.0) * e / ut;
}

inline double mean_inv_beta(int kind, double ut) {
    if (std::isinf(ut)) return 1.0;
    if (kind == SLPIC_BETA_STEP) {
        double Ps, Pf;
        step_mixture(ut, Ps, Pf);
        return Ps + Pf;
    }
    static const double xg[5] = {-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831,
                                 0.9061798459386640};
    static const double wg[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                                 0.4786286704993665, 0.2369268850561891};
    const int panels = 4000;
    const double L = 40.0, h = L / panels;
    double sum = 0.0;
    for (int p = 0; p < panels; ++p) {
        double mid = (p + 0.5) * h;
        for (int k = 0; k < 5; ++k) {
            double s = mid + 0.5 * h * xg[k];
            double f = 0.7978845608028654 * s * s * std::exp(-0.5 * s * s) * std::sqrt(1.0 + (s / ut) * (s / ut));
            sum += 0.5 * h * wg[k] * f;
        }
    }
    return sum;
}

}  // namespace slpic
