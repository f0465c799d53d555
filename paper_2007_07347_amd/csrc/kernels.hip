// gfx950 kernels of one sDUGKS time step (Zhong et al., arXiv:2007.07347,
// Section II, eleven-step summary), FP64 storage.
//
//   k_grad          steps 2-3: fbar+ = a f + b feq(W) at every centre and its
//                   least-squares gradient (normal equations of the LLSR fit,
//                   boundary states as points at the face midpoints);
//                   one thread per (cell, velocity).
//   k_flux_update   steps 1, 3-11: per face the upwind reconstruction at the
//                   foot point x_f - e_i dt (Eq. fbpsource), the face macros
//                   and equilibrium, f at the face (Eq. f_t_n+1), the
//                   mesoscopic and macroscopic fluxes (Eqs. MesoFlux,
//                   MacroFlux); per cell the conservative update of W
//                   (Eq. MacroUpdate), feq^{n+1} and f^{n+1} (Eq. fn+1).
//                   Four lanes per cell, one face each; the per-cell flux
//                   sums are formed with lane shuffles in a fixed order.
//   k_reduce*       residual of the cavity case, total mass, finiteness (one
//                   instance, or every member of a batch in one launch).
//   k_set_equilibrium  f = feq of given macros (initial states).
//
// Every face is evaluated by both of its cells from bit-identical operands
// (the mesh builder stores mirrored copies), so the two evaluations agree
// exactly and each face flux leaves one cell exactly as it enters the other.
#include "device.h"

#include "d2q9.h"
#include "reduce.h"

namespace sdg {

namespace {

// Boundary state (rho_b, u_b) of Section III for a face of the given tag,
// seen from the adjacent cell with macros (rho, ux, uy).
__device__ __forceinline__ void boundary_state(const DevBC &bc, double rho, double ux, double uy,
                                               double &rb, double &ub, double &vb)
{
    if (bc.type == 2) { rb = bc.rho; ub = bc.u; vb = bc.v; }          // inlet / far field
    else if (bc.type == 3) { rb = rho; ub = ux; vb = uy; }            // outlet
    else if (bc.type == 5) {                                          // symmetry: (u, v) = unit normal
        const double un = ux * bc.u + uy * bc.v;
        rb = rho; ub = ux - un * bc.u; vb = uy - un * bc.v;
    }
    else { rb = rho; ub = bc.u; vb = bc.v; }                          // wall (moving or at rest)
}

__global__ void __launch_bounds__(256) k_grad(DevMesh m, DevState s, DevScratch x)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (c >= m.nc) return;
    const int np = m.np;
    const double exi = kEx[i], eyi = kEy[i], wi = kW[i];
    const double rho = s.W[c];
    const double ux = s.W[np + c] / rho, uy = s.W[2 * np + c] / rho;
    const double fe = feq_one(wi, exi, eyi, rho, ux, uy);
    const double fc = s.f[(size_t)i * np + c];
    const double fb = m.a * fc + m.b * fe;
    double ax = 0.0, ay = 0.0;
    for (int sl = 0; sl < m.D; sl++) {
        const int q = sl * np + c;
        const int nb = m.nbr[q];
        if (nb == INT32_MIN) continue;
        double val, dx, dy;
        if (nb >= 0) {
            const double rk = s.W[nb];
            const double uk = s.W[np + nb] / rk, vk = s.W[2 * np + nb] / rk;
            val = m.a * s.f[(size_t)i * np + nb] + m.b * feq_one(wi, exi, eyi, rk, uk, vk);
            dx = m.rs[q].x - m.ro[q].x;
            dy = m.rs[q].y - m.ro[q].y;
        } else {
            const DevBC bc = m.bcs[m.bf_tag[-1 - nb]];
            double rb, ub, vb;
            boundary_state(bc, rho, ux, uy, rb, ub, vb);
            val = feq_one(wi, exi, eyi, rb, ub, vb) + m.a * (fc - fe);
            dx = m.rs[q].x;
            dy = m.rs[q].y;
        }
        const double df = val - fb;
        ax += dx * df;
        ay += dy * df;
    }
    const double i0 = m.ainv[c], i1 = m.ainv[np + c], i2 = m.ainv[2 * np + c];
    x.fbp[(size_t)i * np + c] = fb;
    x.sg[(size_t)i * np + c] = i0 * ax + i1 * ay;
    x.sg[(size_t)(9 + i) * np + c] = i1 * ax + i2 * ay;
}

// Sum over the L lanes of a cell, butterfly order (every lane gets the same bits).
template <int L>
__device__ __forceinline__ double lane_sum(double v)
{
#pragma unroll
    for (int off = 1; off < L; off <<= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int L>
__global__ void __launch_bounds__(256) k_flux_update(DevMesh m, DevState s, DevScratch x, int lagged)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = t / L;
    const int sl = t % L;
    const bool valid = c < m.nc;
    const int np = m.np;
    double phi[9], g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
    for (int i = 0; i < 9; i++) phi[i] = 0.0;
    const int nb = (valid && sl < m.D) ? m.nbr[sl * np + c] : INT32_MIN;
    if (nb != INT32_MIN) {
        const int q = sl * np + c;
        const double2 ln = m.ln[q], rsv = m.rs[q];
        const double lnx = ln.x, lny = ln.y;
        const double rsx = rsv.x, rsy = rsv.y;
        double fbar[9];
        if (nb >= 0) {
            const double2 rov = m.ro[q];
            const double rox = rov.x, roy = rov.y;
#pragma unroll
            for (int i = 0; i < 9; i++) {
                const double sn = kEx[i] * lnx + kEy[i] * lny;
                double rs = 0.0, ro = 0.0;
                if (sn >= 0.0)
                    rs = x.fbp[(size_t)i * np + c] + (rsx - m.dt * kEx[i]) * x.sg[(size_t)i * np + c]
                         + (rsy - m.dt * kEy[i]) * x.sg[(size_t)(9 + i) * np + c];
                if (sn <= 0.0)
                    ro = x.fbp[(size_t)i * np + nb] + (rox - m.dt * kEx[i]) * x.sg[(size_t)i * np + nb]
                         + (roy - m.dt * kEy[i]) * x.sg[(size_t)(9 + i) * np + nb];
                fbar[i] = sn > 0.0 ? rs : (sn < 0.0 ? ro : 0.5 * (rs + ro));
            }
        } else {
            const double rho = s.W[c];
            const double ux = s.W[np + c] / rho, uy = s.W[2 * np + c] / rho;
            const DevBC bc = m.bcs[m.bf_tag[-1 - nb]];
            double rb, ub, vb;
            boundary_state(bc, rho, ux, uy, rb, ub, vb);
#pragma unroll
            for (int i = 0; i < 9; i++) {
                const double sn = kEx[i] * lnx + kEy[i] * lny;
                const double sx = x.sg[(size_t)i * np + c], sy = x.sg[(size_t)(9 + i) * np + c];
                if (sn >= 0.0) {
                    fbar[i] = x.fbp[(size_t)i * np + c] + (rsx - m.dt * kEx[i]) * sx + (rsy - m.dt * kEy[i]) * sy;
                } else {
                    // incoming: the boundary state's fbar+ carried to the foot point
                    const double fe = feq_one(kW[i], kEx[i], kEy[i], rho, ux, uy);
                    const double gb = feq_one(kW[i], kEx[i], kEy[i], rb, ub, vb) + m.a * (s.f[(size_t)i * np + c] - fe);
                    fbar[i] = gb - m.dt * (kEx[i] * sx + kEy[i] * sy);
                }
            }
        }
        // face macros (step 5), face equilibrium (6), face f (7), fluxes (8, 1)
        double rf = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
        for (int i = 0; i < 9; i++) { rf += fbar[i]; mx += kEx[i] * fbar[i]; my += kEy[i] * fbar[i]; }
        const double uf = mx / rf, vf = my / rf;
#pragma unroll
        for (int i = 0; i < 9; i++) {
            const double sn = kEx[i] * lnx + kEy[i] * lny;
            const double ff = m.c1 * (fbar[i] + m.b * feq_one(kW[i], kEx[i], kEy[i], rf, uf, vf));
            phi[i] = sn * ff;
            g0 += phi[i];
            g1 += kEx[i] * phi[i];
            g2 += kEy[i] * phi[i];
        }
    }
#pragma unroll
    for (int i = 0; i < 9; i++) phi[i] = lane_sum<L>(phi[i]);
    g0 = lane_sum<L>(g0);
    g1 = lane_sum<L>(g1);
    g2 = lane_sum<L>(g2);
    if (!valid) return;
    // steps 9-11
    const double dtv = m.dtv[c];
    double G0 = g0, G1 = g1, G2 = g2;
    if (lagged) { G0 = s.G[c]; G1 = s.G[np + c]; G2 = s.G[2 * np + c]; }
    const double rn = s.W[c] - dtv * G0;
    const double mxn = s.W[np + c] - dtv * G1;
    const double myn = s.W[2 * np + c] - dtv * G2;
    if (sl == 0) s.Wo[c] = rn;
    if (sl == 1 % L) s.Wo[np + c] = mxn;
    if (sl == 2 % L) s.Wo[2 * np + c] = myn;
    if (lagged) {
        if (sl == 0) s.Go[c] = g0;
        if (sl == 1 % L) s.Go[np + c] = g1;
        if (sl == 2 % L) s.Go[2 * np + c] = g2;
    }
    const double un = mxn / rn, vn = myn / rn;
    const double inv = m.inv1l;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        if (i % L != sl) continue;
        const double fe = feq_one(kW[i], kEx[i], kEy[i], rn, un, vn);
        s.fo[(size_t)i * np + c] = (s.f[(size_t)i * np + c] - dtv * phi[i] + m.lam * fe) * inv;
    }
}

__global__ void __launch_bounds__(256) k_reduce(int nc, int np, const double *__restrict__ W,
                                               const double *__restrict__ area, double *snap, int update,
                                               double *partials)
{
    reduce_block(nc, np, W, area, snap, update, partials, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_reduce_final(const double *partials, double *out4)
{
    reduce_final(partials, out4);
}

// Batched residual: blockIdx.y selects the member.
__global__ void __launch_bounds__(256) k_reduce_batch(const ReduceJob *jobs)
{
    const ReduceJob j = jobs[blockIdx.y];
    reduce_block(j.nc, j.np, j.W, j.area, j.snap, 1, j.partials, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_reduce_final_batch(const ReduceJob *jobs, double *out)
{
    reduce_final(jobs[blockIdx.x].partials, out + 4 * (size_t)blockIdx.x);
}

// Equilibrium state from per-cell macros m3 = [3][np] (rho, u, v): f = feq
// (Eq. Feq; its moments are the macros, Eq. Macro), stored as f or, with f32,
// as the deviation feq - w_i rho0 in FP32 (rho0 < 0: the non-equilibrium
// part, zero); W = (rho, rho u, rho v); G = 0;
// the residual snapshot = the velocity of W.
__global__ void __launch_bounds__(256) k_set_equilibrium(int nc, int np, const double *m3, double *f, float *f32,
                                                        double rho0, double *W, double *G, double *snap)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double r = m3[c], ux = m3[np + c], uy = m3[2 * np + c];
#pragma unroll
    for (int i = 0; i < 9; i++) {
        const double fe = feq_one(kW[i], kEx[i], kEy[i], r, ux, uy);
        if (f32) f32[(size_t)i * np + c] = rho0 < 0.0 ? 0.0f : (float)(fe - kW[i] * rho0);
        else f[(size_t)i * np + c] = fe;
    }
    const double mx = r * ux, my = r * uy;
    W[c] = r;
    W[np + c] = mx;
    W[2 * np + c] = my;
    G[c] = 0.0;
    G[np + c] = 0.0;
    G[2 * np + c] = 0.0;
    // the velocity exactly as the residual reduction derives it from W
    snap[c] = mx / r;
    snap[np + c] = my / r;
}

__global__ void k_poke_nan(void *p, int bytes)
{
    if (bytes == 8) *reinterpret_cast<double *>(p) = __builtin_nan("");
    else *reinterpret_cast<float *>(p) = __builtin_nanf("");
}

}  // namespace

hipError_t launch_grad(const DevMesh &m, const DevState &s, const DevScratch &x, hipStream_t st, GraphChain *gc)
{
    return emit(&k_grad, dim3((m.nc + 255) / 256, 9), dim3(256), 0, st, gc, m, s, x);
}

hipError_t launch_flux_update(const DevMesh &m, const DevState &s, const DevScratch &x, int lagged, hipStream_t st,
                              GraphChain *gc)
{
    if (m.D <= 4) {
        const long threads = (long)m.nc * 4;
        return emit(&k_flux_update<4>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, gc, m, s, x, lagged);
    }
    const long threads = (long)m.nc * 8;
    return emit(&k_flux_update<8>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, gc, m, s, x, lagged);
}

hipError_t launch_reduce(const DevMesh &m, const double *W, double *snap, int update_snap, double *partials,
                         double *out4, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce, dim3(kReduceBlocks), dim3(256), 0, st, m.nc, m.np, W, m.area, snap, update_snap, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kReduceBlocks), 0, st, partials, out4);
    return hipGetLastError();
}

hipError_t launch_reduce_batch(const ReduceJob *jobs, int n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_batch, dim3(kReduceBlocks, n), dim3(256), 0, st, jobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final_batch, dim3(n), dim3(kReduceBlocks), 0, st, jobs, out);
    return hipGetLastError();
}

hipError_t launch_set_equilibrium(int nc, int np, const double *m3, double *f, float *f32, double rho0, double *W,
                                  double *G, double *snap, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_equilibrium, dim3((nc + 255) / 256), dim3(256), 0, st, nc, np, m3, f, f32, rho0, W, G,
                       snap);
    return hipGetLastError();
}

hipError_t launch_poke_nan(void *p, int bytes, hipStream_t st)
{
    hipLaunchKernelGGL(k_poke_nan, dim3(1), dim3(1), 0, st, p, bytes);
    return hipGetLastError();
}

}  // namespace sdg
