// Uniform-z cosmology tables shared by the particle pastes: comoving distance chi(z) [Mpc/h] and
// the optical depth tau(z) of a fully ionised universe (Sec. 3.4), tabulated on a uniform z grid by
// k_cosmo_table and read back by cubic Lagrange interpolation.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "bp_device.hpp"

namespace bp {

constexpr int kNZ = 16384;
constexpr double kZmax = 16.0;

// cubic Lagrange interpolation on the uniform table
__device__ inline double table_interp(const double *__restrict__ t, double z) {
    double s = z * ((kNZ - 1) / kZmax);
    int i = (int)floor(s);
    i = min(max(i, 1), kNZ - 3);
    double f = s - i;
    double w0 = -f * (f - 1.0) * (f - 2.0) / 6.0, w1 = (f + 1.0) * (f - 1.0) * (f - 2.0) * 0.5;
    double w2 = -(f + 1.0) * f * (f - 2.0) * 0.5, w3 = (f + 1.0) * f * (f - 1.0) / 6.0;
    return w0 * t[i - 1] + w1 * t[i] + w2 * t[i + 1] + w3 * t[i + 2];
}

}  // namespace bp
