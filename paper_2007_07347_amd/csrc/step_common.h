// Device helpers shared by the fused step kernels (general tiles and the
// structured step): compile-time lattice arithmetic, global-address-space
// pointers, lane exchanges and sums, and the boundary states of Section III.
#pragma once

#include <type_traits>
#include <utility>

#include "device.h"

namespace sdg {
namespace {

// ---- compile-time lattice arithmetic.  Velocity loops are unrolled with the
// index as a constant, so products with the lattice components 0 and +-1
// are written as what they are (IEEE rules forbid the compiler to drop
// x * 0 on its own).
constexpr int cEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int cEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr double cW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Device-global memory, said so explicitly.  Pointers that the compiler
// cannot trace to a kernel argument (a batched launch reads its members'
// pointers from their records) would otherwise be accessed with flat
// instructions, whose outstanding loads also hold up every wait on LDS and
// scalar results.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gmem = __attribute__((address_space(1))) T;
#else
template <typename T>
using gmem = T;   // the host pass only parses device code
#endif
template <typename T>
__device__ __forceinline__ const gmem<T> *gin(const T *p)
{
    return (const gmem<T> *)p;
}
template <typename T>
__device__ __forceinline__ gmem<T> *gout(T *p)
{
    return (gmem<T> *)p;
}

// c x for c in {-1, 0, 1}
template <int C, typename T>
__device__ __forceinline__ T cmul(T x)
{
    if constexpr (C == 0) return T(0);
    else if constexpr (C > 0) return x;
    else return -x;
}
// a x + b y for a, b in {-1, 0, 1}, one rounding at most
template <int A, int B, typename T>
__device__ __forceinline__ T cdot(T x, T y)
{
    if constexpr (A == 0) return cmul<B>(y);
    else if constexpr (B == 0) return cmul<A>(x);
    else if constexpr (A > 0 && B > 0) return x + y;
    else if constexpr (A > 0) return x - y;
    else if constexpr (B > 0) return y - x;
    else return -(x + y);
}
// x - c d for c in {-1, 0, 1}
template <int C, typename T>
__device__ __forceinline__ T csub(T x, T d)
{
    if constexpr (C == 0) return x;
    else if constexpr (C > 0) return x - d;
    else return x + d;
}
// Second-order equilibrium of velocity (EX, EY) with weight w, uu = u.u.
template <int EX, int EY, typename T>
__device__ __forceinline__ T feq_c(T w, T rho, T ux, T uy, T uu)
{
    const T eu = cdot<EX, EY>(ux, uy);
    return w * rho * ((T)1 + (T)3 * eu + (T)4.5 * eu * eu - (T)1.5 * uu);
}

// Quad-lane exchange by DPP (no LDS traffic): lane l reads lane l ^ 1 (0xB1)
// or l ^ 2 (0x4E) of its group of four.
template <int CTRL>
__device__ __forceinline__ double qx(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float qx(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the four lanes of a cell, butterfly order: (a + b) + (c + d) on
// every lane, so all four end with the same bits.
__device__ __forceinline__ double lane_sum4(double v)
{
    v += qx<0xB1>(v);
    v += qx<0x4E>(v);
    return v;
}

// Compensated sum over the four lanes of a cell: TwoSum at each butterfly
// level (its error term is exact whatever the operand order, so every lane
// ends with the same bits), errors added at the end.
__device__ __forceinline__ float lane_sum4_comp(float v)
{
    float e = 0.0f;
    static_for<2>([&](auto L) {
        constexpr int CTRL = L == 0 ? 0xB1 : 0x4E;
        const float b = qx<CTRL>(v), eb = qx<CTRL>(e);
        const float sum = v + b;
        const float bb = sum - v;
        const float err = (v - (sum - bb)) + (b - bb);
        e = (e + eb) + err;
        v = sum;
    });
    return v + e;
}

// Boundary state of entry e of the LDS table (type, rho, u, v) seen from a
// cell with macros (rho, ux, uy).
__device__ __forceinline__ void boundary_state_t(const double *sbc, int e, double rho, double ux, double uy,
                                                 double &rb, double &ub, double &vb)
{
    const double type = sbc[4 * e], brho = sbc[4 * e + 1], bu = sbc[4 * e + 2], bv = sbc[4 * e + 3];
    if (type == 2.0) { rb = brho; ub = bu; vb = bv; }                // inlet / far field
    else if (type == 3.0) { rb = rho; ub = ux; vb = uy; }            // outlet
    else if (type == 5.0) {                                          // symmetry: (bu, bv) = unit normal
        const double un = ux * bu + uy * bv;
        rb = rho; ub = ux - un * bu; vb = uy - un * bv;
    }
    else { rb = rho; ub = bu; vb = bv; }                             // wall
}


}  // namespace
}  // namespace sdg
