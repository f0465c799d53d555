// D2Q9 lattice of the solver library (c = 1, c_s^2 = 1/3): velocity order
// (0,0), (1,0), (0,1), (-1,0), (0,-1), (1,1), (-1,1), (-1,-1), (1,-1).
#pragma once

#include <hip/hip_runtime.h>

namespace sdg {

__device__ constexpr double kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr double kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// Second-order Hermite truncation of the Maxwellian (Eq. Feq of the paper
// written for the discrete velocity set): w rho (1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u).
__device__ __forceinline__ double feq_one(double w, double ex, double ey, double rho, double ux, double uy)
{
    const double eu = ex * ux + ey * uy;
    const double uu = ux * ux + uy * uy;
    return w * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

}  // namespace sdg
