// Fused sDUGKS time step (Zhong et al., arXiv:2007.07347, Section II, the
// eleven-step summary) in one kernel: one workgroup per tile of cells.
//
//   phase 1  fbar+ = a f + b feq(W) (Eq. fbarplus) and W for the tile and its
//            two halo rings, into LDS (halo values are recomputed by every
//            tile that needs them instead of being stored to memory);
//   phase 2  least-squares gradient of fbar+ (LLSR normal equations, boundary
//            states as points at the face midpoints) for the tile and its
//            first ring, into LDS;
//   phase 3  four lanes per tile cell, one face each: upwind reconstruction at
//            the foot point (Eq. fbpsource), face macros and equilibrium,
//            f at the face (Eq. f_t_n+1), mesoscopic and macroscopic fluxes
//            (Eqs. MesoFlux, MacroFlux); per-cell sums by lane shuffles in a
//            fixed order; then W^{n+1} (Eq. MacroUpdate), feq^{n+1} and
//            f^{n+1} (Eq. fn+1) written once.
//
// f and W of each cell are read from memory by the tile that owns it and by
// the tiles whose halos contain it (mostly cache hits: neighbouring tiles run
// close together), and written once.  A face shared by two tiles is evaluated
// by both from identical operands, so the flux that leaves one cell enters the
// other exactly.
#include "d2q9.h"
#include "device.h"

namespace sdg {

namespace {

__device__ __forceinline__ void boundary_state_t(const DevBC &bc, double rho, double ux, double uy,
                                                 double &rb, double &ub, double &vb)
{
    if (bc.type == 2) { rb = bc.rho; ub = bc.u; vb = bc.v; }          // inlet / far field
    else if (bc.type == 3) { rb = rho; ub = ux; vb = uy; }            // outlet
    else { rb = rho; ub = bc.u; vb = bc.v; }                          // wall
}

__device__ __forceinline__ double lane_sum4(double v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    return v;
}

template <int D>
__global__ void __launch_bounds__(256) k_step_tiled(DevMesh m, DevTiles tl, DevState s, int lagged)
{
    extern __shared__ double smem[];
    const int t = blockIdx.x;
    const int *hd = tl.hdr + 8 * t;
    const int g0 = hd[0], nt = hd[1], n1 = hd[2], n2 = hd[3], hoff = hd[4], aoff = hd[5];
    const int na = nt + n1, nl = na + n2;
    const int P = tl.nl_max, P1 = tl.na_max;
    const int np = m.np;
    double *sfbp = smem;               // [9][P]
    double *sW = smem + 9 * P;         // [3][P]   raw W
    double *ssg = smem + 12 * P;       // [18][P1] gradient (x rows 0..8, y rows 9..17)
    const int16_t *ladj = tl.ladj + aoff;

    // ---- phase 1: fbar+ and W of every local cell
    for (int lc = threadIdx.x; lc < nl; lc += blockDim.x) {
        const int g = lc < nt ? g0 + lc : tl.hlist[hoff + lc - nt];
        const double r = s.W[g], mu = s.W[np + g], mv = s.W[2 * np + g];
        sW[lc] = r;
        sW[P + lc] = mu;
        sW[2 * P + lc] = mv;
        const double ux = mu / r, uy = mv / r;
#pragma unroll
        for (int i = 0; i < 9; i++)
            sfbp[i * P + lc] = m.a * s.f[(size_t)i * np + g] + m.b * feq_one(kW[i], kEx[i], kEy[i], r, ux, uy);
    }
    __syncthreads();

    // ---- phase 2: gradients of the tile and its first ring
    for (int lc = threadIdx.x; lc < na; lc += blockDim.x) {
        const int g = lc < nt ? g0 + lc : tl.hlist[hoff + lc - nt];
        double ax[9], ay[9], fc[9];
#pragma unroll
        for (int i = 0; i < 9; i++) { ax[i] = 0.0; ay[i] = 0.0; fc[i] = sfbp[i * P + lc]; }
#pragma unroll
        for (int sl = 0; sl < D; sl++) {
            const int la = ladj[sl * na + lc];
            if (la == -2) continue;
            const int q = sl * np + g;
            if (la >= 0) {
                const double dx = m.rsx[q] - m.rox[q], dy = m.rsy[q] - m.roy[q];
#pragma unroll
                for (int i = 0; i < 9; i++) {
                    const double df = sfbp[i * P + la] - fc[i];
                    ax[i] += dx * df;
                    ay[i] += dy * df;
                }
            } else {
                // boundary point: fbar+_b - fbar+_c = feq(rho_b, u_b) - feq(W_c)
                const DevBC bc = m.bcs[m.bf_tag[-1 - m.nbr[q]]];
                const double r = sW[lc], ux = sW[P + lc] / r, uy = sW[2 * P + lc] / r;
                double rb, ub, vb;
                boundary_state_t(bc, r, ux, uy, rb, ub, vb);
                const double dx = m.rsx[q], dy = m.rsy[q];
#pragma unroll
                for (int i = 0; i < 9; i++) {
                    const double df = feq_one(kW[i], kEx[i], kEy[i], rb, ub, vb) - feq_one(kW[i], kEx[i], kEy[i], r, ux, uy);
                    ax[i] += dx * df;
                    ay[i] += dy * df;
                }
            }
        }
        const double i0 = m.ainv[g], i1 = m.ainv[np + g], i2 = m.ainv[2 * np + g];
#pragma unroll
        for (int i = 0; i < 9; i++) {
            ssg[i * P1 + lc] = i0 * ax[i] + i1 * ay[i];
            ssg[(9 + i) * P1 + lc] = i1 * ax[i] + i2 * ay[i];
        }
    }
    __syncthreads();

    // ---- phase 3: faces of the tile cells (4 lanes per cell) and the update
    const double inv = 1.0 / (1.0 + m.lam);
    for (int base = 0; base < 4 * nt; base += blockDim.x) {
        const int lane = base + threadIdx.x;
        const int lc = lane >> 2, sl = lane & 3;
        const bool valid = lc < nt;
        double phi[9], g0s = 0.0, g1s = 0.0, g2s = 0.0;
#pragma unroll
        for (int i = 0; i < 9; i++) phi[i] = 0.0;
        const int la = (valid && sl < D) ? ladj[sl * na + lc] : -2;
        if (la != -2) {
            const int g = g0 + lc;
            const int q = sl * np + g;
            const double lnx = m.lnx[q], lny = m.lny[q], rsx = m.rsx[q], rsy = m.rsy[q];
            double fbar[9];
            if (la >= 0) {
                const double rox = m.rox[q], roy = m.roy[q];
#pragma unroll
                for (int i = 0; i < 9; i++) {
                    const double sn = kEx[i] * lnx + kEy[i] * lny;
                    double rs = 0.0, ro = 0.0;
                    if (sn >= 0.0)
                        rs = sfbp[i * P + lc] + (rsx - m.dt * kEx[i]) * ssg[i * P1 + lc]
                             + (rsy - m.dt * kEy[i]) * ssg[(9 + i) * P1 + lc];
                    if (sn <= 0.0)
                        ro = sfbp[i * P + la] + (rox - m.dt * kEx[i]) * ssg[i * P1 + la]
                             + (roy - m.dt * kEy[i]) * ssg[(9 + i) * P1 + la];
                    fbar[i] = sn > 0.0 ? rs : (sn < 0.0 ? ro : 0.5 * (rs + ro));
                }
            } else {
                const DevBC bc = m.bcs[m.bf_tag[-1 - m.nbr[q]]];
                const double r = sW[lc], ux = sW[P + lc] / r, uy = sW[2 * P + lc] / r;
                double rb, ub, vb;
                boundary_state_t(bc, r, ux, uy, rb, ub, vb);
#pragma unroll
                for (int i = 0; i < 9; i++) {
                    const double sn = kEx[i] * lnx + kEy[i] * lny;
                    const double sx = ssg[i * P1 + lc], sy = ssg[(9 + i) * P1 + lc];
                    const double fb = sfbp[i * P + lc];
                    if (sn >= 0.0) {
                        fbar[i] = fb + (rsx - m.dt * kEx[i]) * sx + (rsy - m.dt * kEy[i]) * sy;
                    } else {
                        // incoming: the boundary state's fbar+ carried to the foot point
                        const double gb = feq_one(kW[i], kEx[i], kEy[i], rb, ub, vb) + fb
                                          - feq_one(kW[i], kEx[i], kEy[i], r, ux, uy);
                        fbar[i] = gb - m.dt * (kEx[i] * sx + kEy[i] * sy);
                    }
                }
            }
            double rf = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
            for (int i = 0; i < 9; i++) { rf += fbar[i]; mx += kEx[i] * fbar[i]; my += kEy[i] * fbar[i]; }
            const double uf = mx / rf, vf = my / rf;
#pragma unroll
            for (int i = 0; i < 9; i++) {
                const double sn = kEx[i] * lnx + kEy[i] * lny;
                const double ff = m.c1 * (fbar[i] + m.b * feq_one(kW[i], kEx[i], kEy[i], rf, uf, vf));
                phi[i] = sn * ff;
                g0s += phi[i];
                g1s += kEx[i] * phi[i];
                g2s += kEy[i] * phi[i];
            }
        }
#pragma unroll
        for (int i = 0; i < 9; i++) phi[i] = lane_sum4(phi[i]);
        g0s = lane_sum4(g0s);
        g1s = lane_sum4(g1s);
        g2s = lane_sum4(g2s);
        if (valid) {
            const int g = g0 + lc;
            const double dtv = m.dtv[g];
            double G0 = g0s, G1 = g1s, G2 = g2s;
            if (lagged) { G0 = s.G[g]; G1 = s.G[np + g]; G2 = s.G[2 * np + g]; }
            const double rn = sW[lc] - dtv * G0;
            const double mxn = sW[P + lc] - dtv * G1;
            const double myn = sW[2 * P + lc] - dtv * G2;
            if (sl == 0) s.Wo[g] = rn;
            if (sl == 1) s.Wo[np + g] = mxn;
            if (sl == 2) s.Wo[2 * np + g] = myn;
            if (lagged) {
                if (sl == 0) s.Go[g] = g0s;
                if (sl == 1) s.Go[np + g] = g1s;
                if (sl == 2) s.Go[2 * np + g] = g2s;
            }
            const double un = mxn / rn, vn = myn / rn;
#pragma unroll
            for (int i = 0; i < 9; i++) {
                if ((i & 3) != sl) continue;
                const double fe = feq_one(kW[i], kEx[i], kEy[i], rn, un, vn);
                s.fo[(size_t)i * np + g] = (s.f[(size_t)i * np + g] - dtv * phi[i] + m.lam * fe) * inv;
            }
        }
    }
}

}  // namespace

size_t step_tiled_lds_bytes(const DevTiles &t) { return (12 * (size_t)t.nl_max + 18 * (size_t)t.na_max) * sizeof(double); }

hipError_t launch_step_tiled(const DevMesh &m, const DevTiles &t, const DevState &s, int lagged, int block,
                             hipStream_t st)
{
    const size_t lds = step_tiled_lds_bytes(t);
    if (m.D <= 3)
        hipLaunchKernelGGL(k_step_tiled<3>, dim3(t.n_tiles), dim3(block), lds, st, m, t, s, lagged);
    else
        hipLaunchKernelGGL(k_step_tiled<4>, dim3(t.n_tiles), dim3(block), lds, st, m, t, s, lagged);
    return hipGetLastError();
}

}  // namespace sdg
