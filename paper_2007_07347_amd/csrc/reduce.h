// Deterministic reduction bodies of the residual, mass and finiteness check
// (per-block partial sums in a fixed order, then one block adding the
// partials in a fixed order), shared by every kernel that reduces an
// instance, so a member's residual is bitwise the same whichever call
// computes it.
#pragma once

#include "device.h"

namespace sdg {

// Block blk of the per-instance partial sums over [lo, hi) of the cells:
// {sum |u - u_snap|^2, sum |u_snap|^2, sum V rho, non-finite count}.
__device__ __forceinline__ void reduce_block(int nc, int np, const double *__restrict__ W,
                                             const double *__restrict__ area, double *snap, int update,
                                             double *partials, int blk)
{
    __shared__ double red[4][256];
    const int chunk = (nc + kReduceBlocks - 1) / kReduceBlocks;
    const int lo = blk * chunk, hi = min(nc, lo + chunk);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int c = lo + threadIdx.x; c < hi; c += blockDim.x) {
        const double r = W[c];
        const double U = W[np + c] / r, V = W[2 * np + c] / r;
        const double su = snap[c], sv = snap[np + c];
        a0 += (U - su) * (U - su) + (V - sv) * (V - sv);
        a1 += su * su + sv * sv;
        a2 += area[c] * r;
        a3 += (isfinite(r) && isfinite(U) && isfinite(V)) ? 0.0 : 1.0;
        if (update) { snap[c] = U; snap[np + c] = V; }
    }
    red[0][threadIdx.x] = a0; red[1][threadIdx.x] = a1; red[2][threadIdx.x] = a2; red[3][threadIdx.x] = a3;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 4; k++) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) partials[threadIdx.x * kReduceBlocks + blk] = red[threadIdx.x][0];
}

__device__ __forceinline__ void reduce_final(const double *partials, double *out4)
{
    __shared__ double red[4][kReduceBlocks];
    for (int k = 0; k < 4; k++) red[k][threadIdx.x] = partials[k * kReduceBlocks + threadIdx.x];
    __syncthreads();
    for (int w = kReduceBlocks / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 4; k++) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) out4[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace sdg
