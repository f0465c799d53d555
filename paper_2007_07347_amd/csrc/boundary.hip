// Fluxes through the boundary faces on the current state, for wall forces and
// surface pressure (not part of the time step).
//
// For each plain boundary face the adjacent cell's fbar+ and its least-squares
// gradient are rebuilt from the state (Eq. fbarplus and the LLSR normal
// equations through the stored weights, boundary states as points at the face
// midpoints), the face value of fbar follows the boundary rule of Section III
// (interior reconstruction for e_i . N >= 0, the boundary state's fbar+ carried
// to the foot point otherwise), and the face distribution of Eq. f_t_n+1 gives
// the fluxes of Eqs. MesoFlux and MacroFlux.  N points out of the fluid, so the
// momentum that leaves through a wall face is the force the fluid exerts on it.
// The arithmetic is the face pass of the step in FP64 (for the deviation form,
// f = stored deviation + w_i rho0).
#include "d2q9.h"
#include "device.h"

namespace sdg {

namespace {

// f of cell c in FP64 whatever the storage (mode: 0 FP64 f; 1 FP32 f - w_i
// rho0; 2 FP32 f - feq(W)), and its macros.
__device__ void load_cell(const DevMesh &m, const DevState &s, int mode, int c, double *f, double &r, double &ux,
                          double &uy)
{
    const int np = m.np;
    r = s.W[c];
    ux = s.W[np + c] / r;
    uy = s.W[2 * np + c] / r;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        if (mode == 0) f[i] = s.f[(size_t)i * np + c];
        else if (mode == 1) f[i] = (double)s.f32[(size_t)i * np + c] + kW[i] * m.rho0;
        else f[i] = (double)s.f32[(size_t)i * np + c] + feq_one(kW[i], kEx[i], kEy[i], r, ux, uy);
    }
}

// Boundary state (rho_b, u_b) of a table entry seen from a cell with macros (r, ux, uy).
__device__ void bstate(const DevBC &bc, double r, double ux, double uy, double &rb, double &ub, double &vb)
{
    if (bc.type == 2) { rb = bc.rho; ub = bc.u; vb = bc.v; }          // inlet / far field
    else if (bc.type == 3) { rb = r; ub = ux; vb = uy; }              // outlet
    else if (bc.type == 5) {                                          // symmetry: (u, v) = unit normal
        const double un = ux * bc.u + uy * bc.v;
        rb = r; ub = ux - un * bc.u; vb = uy - un * bc.v;
    }
    else { rb = r; ub = bc.u; vb = bc.v; }                            // wall
}

__global__ void __launch_bounds__(64) k_boundary_flux(DevMesh m, DevState s, DevBnd q, int mode)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= q.n) return;
    const int4 h = q.hdr[b];
    const int c = h.x, tag = h.z, D = m.D;
    double fc[9], r, ux, uy;
    load_cell(m, s, mode, c, fc, r, ux, uy);
    double fe[9], fbp[9], sx[9], sy[9];
#pragma unroll
    for (int i = 0; i < 9; i++) {
        fe[i] = feq_one(kW[i], kEx[i], kEy[i], r, ux, uy);
        fbp[i] = m.a * fc[i] + m.b * fe[i];
        sx[i] = 0.0;
        sy[i] = 0.0;
    }
    // gradient of fbar+ at the cell: sum over its stencil of w (value - fbar+_c)
    for (int j = 0; j < D; j++) {
        const int v = q.nb[(size_t)b * D + j];
        if (v == -1) continue;
        const double2 w = q.w[(size_t)b * D + j];
        if (v >= 0) {
            double fk[9], rk, uk, vk;
            load_cell(m, s, mode, v, fk, rk, uk, vk);
#pragma unroll
            for (int i = 0; i < 9; i++) {
                const double d = (m.a * fk[i] + m.b * feq_one(kW[i], kEx[i], kEy[i], rk, uk, vk)) - fbp[i];
                sx[i] += w.x * d;
                sy[i] += w.y * d;
            }
        } else {
            double rb, ub, vb;
            bstate(m.bcs[-2 - v], r, ux, uy, rb, ub, vb);
#pragma unroll
            for (int i = 0; i < 9; i++) {
                const double d = feq_one(kW[i], kEx[i], kEy[i], rb, ub, vb) - fe[i];
                sx[i] += w.x * d;
                sy[i] += w.y * d;
            }
        }
    }
    // the face: fbar by the boundary rule, face macros, face f, fluxes
    const double2 ln = q.geo[2 * (size_t)b], rs = q.geo[2 * (size_t)b + 1];
    double rb, ub, vb;
    bstate(m.bcs[tag], r, ux, uy, rb, ub, vb);
    double fbar[9], rf = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        const double sn = kEx[i] * ln.x + kEy[i] * ln.y;
        const double inner = fbp[i] + (rs.x - m.dtr * kEx[i]) * sx[i] + (rs.y - m.dtr * kEy[i]) * sy[i];
        const double gb = (feq_one(kW[i], kEx[i], kEy[i], rb, ub, vb) - fe[i]) + fbp[i];
        fbar[i] = sn >= 0.0 ? inner : gb - m.dtr * (kEx[i] * sx[i] + kEy[i] * sy[i]);
        rf += fbar[i];
        mx += kEx[i] * fbar[i];
        my += kEy[i] * fbar[i];
    }
    const double uf = mx / rf, vf = my / rf;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        const double sn = kEx[i] * ln.x + kEy[i] * ln.y;
        const double phi = sn * (m.fc1 * (fbar[i] + m.fb * feq_one(kW[i], kEx[i], kEy[i], rf, uf, vf)));
        g0 += phi;
        g1 += kEx[i] * phi;
        g2 += kEy[i] * phi;
    }
    double *o = q.out + 4 * (size_t)b;
    o[0] = g0;
    o[1] = g1;
    o[2] = g2;
    o[3] = rf;
}

// Sums of the three fluxes over the faces of one tag (all when tag < 0), in a
// fixed order: strided partial sums per thread, then a tree.
__global__ void __launch_bounds__(256) k_boundary_sum(DevBnd q, int tag)
{
    __shared__ double red[3][256];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int b = threadIdx.x; b < q.n; b += blockDim.x) {
        if (tag >= 0 && q.hdr[b].z != tag) continue;
        a0 += q.out[4 * (size_t)b];
        a1 += q.out[4 * (size_t)b + 1];
        a2 += q.out[4 * (size_t)b + 2];
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    red[2][threadIdx.x] = a2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; k++) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) q.sum[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace

hipError_t launch_boundary_flux(const DevMesh &m, const DevState &s, const DevBnd &q, int mode, int tag, hipStream_t st)
{
    if (q.n > 0) {
        hipLaunchKernelGGL(k_boundary_flux, dim3((unsigned)((q.n + 63) / 64)), dim3(64), 0, st, m, s, q, mode);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_boundary_sum, dim3(1), dim3(256), 0, st, q, tag);
    return hipGetLastError();
}

}  // namespace sdg
