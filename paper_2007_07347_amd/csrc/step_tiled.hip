// Fused sDUGKS time step (Zhong et al., arXiv:2007.07347, Section II, the
// eleven-step summary) in one kernel: one workgroup per tile of cells, at
// most one work item per thread in every phase.
//
//   phase 1  fbar+ = a f + b feq(W) (Eq. fbarplus) of the tile and its two
//            halo rings into LDS, with the macros later phases read (rho and
//            u of the tile and first ring, the momentum of the tile); halo
//            values are recomputed by every tile that needs them instead of
//            being stored to memory;
//   phase 2  least-squares gradient of fbar+ (the LLSR normal equations solved
//            through precomputed weights A^-1 d; boundary states are points at
//            the face midpoints) for the tile and its first ring, into LDS (in
//            FP64 the two halves of the workgroup take velocities 0..4 and
//            5..8 of the same cells when those fit in one half);
//   phase 3  four lanes per tile cell, one face each: upwind reconstruction at
//            the foot point (Eq. fbpsource), face macros and equilibrium,
//            f at the face (Eq. f_t_n+1), mesoscopic and macroscopic fluxes
//            (Eqs. MesoFlux, MacroFlux); per-cell sums by lane shuffles in a
//            fixed order; then W^{n+1} (Eq. MacroUpdate), feq^{n+1} and
//            f^{n+1} (Eq. fn+1), each lane writing two or three velocities.
//
// Three forms share the code (template parameter PM), all with FP64 density
// and momentum, their update and the macroscopic fluxes:
//   PM = 0  f stored and computed in FP64;
//   PM = 1  the deviation f - w_i rho0 stored in FP32 with FP32 face records
//           and least-squares weights, fbar+, gradients and face fluxes
//           computed in FP32 on deviations (the constant parts cancel
//           exactly: sum_i w_i e_i = 0 and the scaled normals of a closed cell
//           sum to zero), per-cell flux sums compensated (TwoSum);
//   PM = 2  the non-equilibrium part f - feq(W) stored in FP32 (FP32 tables),
//           every operation in FP64: f = feq(W) + stored part on load, and
//           f^{n+1} - feq(W^{n+1}) rounded to FP32 on store.
//
// Every global input of phases 2 and 3 (adjacency, least-squares weights,
// face records) is requested at kernel start, so its latency overlaps phase 1.
// The faces of a tile's cells are one table of records per tile: a face
// between two tile cells is read once and used by both cells, mirrored.  Each
// XCD sweeps a contiguous range of bisection tiles, those with boundary faces
// first, so the halo cells a tile reads are mostly L2 hits and the slower
// tiles start earliest.  A face shared by two tiles is evaluated by both from
// identical operands: the flux that leaves one cell enters the other exactly.
#include <type_traits>
#include <utility>

#include "d2q9.h"
#include "device.h"
#include "mesh.h"
#include "step_common.h"

namespace sdg {

namespace {

// Least-squares gradient of fbar+ for velocities [I0, I1) of local cell c:
// sum over its stencil of w (value - fbar+_c), boundary points carrying
// fbar+_b - fbar+_c = feq(rho_b, u_b) - feq(W_c).
template <int I0, int I1, int D, typename R>
__device__ __forceinline__ void gradient_cell(const R *sfbp, R *ssg, const double *sW, const double *sbc, int P1, int c,
                                              const int *la2, const R *wx2, const R *wy2)
{
    constexpr int N = I1 - I0, SG = kGradStride;
    R ax[N], ay[N], fc[N];
    static_for<N>([&](auto K) {
        ax[K] = 0;
        ay[K] = 0;
        fc[K] = sfbp[c * 9 + I0 + K];
    });
#pragma unroll
    for (int sl = 0; sl < D; sl++) {
        const int la = la2[sl];
        if (la == -1) continue;
        if (la >= 0) {
            static_for<N>([&](auto K) {
                const R df = sfbp[la * 9 + I0 + K] - fc[K];
                ax[K] += wx2[sl] * df;
                ay[K] += wy2[sl] * df;
            });
        } else {
            const double r = sW[c], ux = sW[P1 + c], uy = sW[2 * P1 + c];
            double rb, ub, vb;
            boundary_state_t(sbc, -2 - la, r, ux, uy, rb, ub, vb);
            const double uu = ux * ux + uy * uy, uub = ub * ub + vb * vb;
            static_for<N>([&](auto K) {
                constexpr int i = I0 + K;
                const R df = (R)(feq_c<cEx[i], cEy[i]>(cW[i], rb, ub, vb, uub) -
                                 feq_c<cEx[i], cEy[i]>(cW[i], r, ux, uy, uu));
                ax[K] += wx2[sl] * df;
                ay[K] += wy2[sl] * df;
            });
        }
    }
    static_for<N>([&](auto K) {
        ssg[c * SG + I0 + K] = ax[K];
        ssg[c * SG + 9 + I0 + K] = ay[K];
    });
}

// One time step of tile t of one instance (the whole workgroup takes part).
template <int D, int PM>
__device__ __forceinline__ void step_tile(const DevMesh &m, const DevTiles &tl, const DevState &s, int lagged, int t)
{
    constexpr bool S32 = PM != 0;    // f and the tables stored in FP32
    constexpr bool DEV = PM == 1;    // FP32 arithmetic on deviations from the rest state w_i rho0
    constexpr bool NEQ = PM == 2;    // stored: f - feq(W); arithmetic in FP64
    using R = typename std::conditional<DEV, float, double>::type;   // arithmetic of fbar+, gradients, faces
    extern __shared__ double smem[];
    const int P = tl.nl_max, P1 = tl.na_max, PT = tl.nt_max;
    const int np = m.np;
    const int tid = threadIdx.x;
    // macros: rho, u, v of the tile and first-ring cells [3][P1] (the
    // boundary states need them), rho u, rho v of the tile cells [2][PT] (the
    // update needs them); nothing for the second ring
    double *sW = smem;
    double *sM = smem + 3 * P1;
    // per cell: fbar+ [P][9] (deviation in DEV) and its gradient [P1][SG]
    // (x components 0..8, y components 9..17, one pad); cell-major, so the
    // velocity and component are constant offsets of one per-cell address
    R *sfbp = reinterpret_cast<R *>(smem + 3 * P1 + 2 * PT);
    R *ssg = sfbp + 9 * P;
    // boundary-condition table [n_bc][4]: type, rho, u, v (16-byte aligned after the gradient)
    constexpr int SG = kGradStride;
    double *sbc = smem + (((3 * P1 + 2 * PT) * 8 + (9 * P + SG * P1) * (int)sizeof(R) + 15) / 16 * 16) / 8;
    const gmem<int16_t> *ladj = gin(tl.ladj + (size_t)t * D * P1);
    const gmem<int16_t> *lfc = gin(tl.lfc + (size_t)t * D * PT);
    using T2 = typename std::conditional<S32, float2, double2>::type;   // tables
    const gmem<T2> *lw, *frt;
    if constexpr (S32) {
        lw = gin(tl.lw32 + (size_t)t * D * P1);
        frt = gin(tl.fr32 + (size_t)t * tl.nf_max * 3);
    } else {
        lw = gin(tl.lw + (size_t)t * D * P1);
        frt = gin(tl.fr + (size_t)t * tl.nf_max * 3);
    }
    const int PF = tl.nf_max;
    // fbar+ from the cell variable (phase 1); the face step: reconstruction
    // time and the coefficients of the face distribution (phase 3)
    const R ra = (R)m.a, rb_ = (R)m.b, rc1 = (R)m.fc1, rbf = (R)m.fb, rdt = (R)m.dtr;
    // ---- requests of all phases, in this order: the local cell ids and the
    // face codes of the lanes; the adjacency, least-squares weights and
    // boundary table, which need nothing loaded first; the phase-1 state at
    // the cell ids; then the face records at the face codes.  Indices are
    // clamped with the tables' pitches, not the tile's own counts: every
    // padded entry is a valid filler (cell 0, no neighbour, zero weight, empty
    // face), so no request waits for the tile header, whose counts only mask
    // what lanes without work read.
    const unsigned g1 = (unsigned)gin(tl.lgid)[(size_t)t * P + (tid < P ? tid : 0)];
    const int lc3 = tid >> 2, sl3 = tid & 3;
    const int sl3c = sl3 < D ? sl3 : D - 1;
    const int lc3c = lc3 < PT ? lc3 : 0;
    const int fc3 = lfc[sl3c * PT + lc3c];
    __builtin_amdgcn_sched_barrier(0);
    // phase 2 cell of this thread: in FP64, with two waves or more and at
    // least twice as many threads as tile and first-ring cells, the two halves
    // of the workgroup take the same cells, velocities 0..4 and 5..8 (in the
    // deviation form the gradient is cheap enough that one half does it all)
    const int half = (int)blockDim.x >> 1;
    const bool split = !DEV && half >= 64 && P1 <= half;
    const int c2 = split && tid >= half ? tid - half : tid;
    const int t2 = c2 < P1 ? c2 : 0;
    int la2[D];
    R wx2[D], wy2[D];
#pragma unroll
    for (int sl = 0; sl < D; sl++) {
        la2[sl] = ladj[sl * P1 + t2];
        const T2 w = lw[sl * P1 + t2];
        wx2[sl] = (R)w.x;
        wy2[sl] = (R)w.y;
    }
    const int a3 = ladj[sl3c * P1 + lc3c];
    const bool pb = tid < m.n_bc;
    const DevBC bcl = gin(m.bcs)[pb ? tid : 0];
    __builtin_amdgcn_sched_barrier(0);
    const double r = gin(s.W)[g1], mu = gin(s.W)[(size_t)np + g1], mv = gin(s.W)[2 * (size_t)np + g1];
    R fv[9];
#pragma unroll
    for (int i = 0; i < 9; i++) {
        if constexpr (S32) fv[i] = gin(s.f32)[(size_t)i * np + g1];
        else fv[i] = gin(s.f)[(size_t)i * np + g1];
    }
    __builtin_amdgcn_sched_barrier(0);
    // the tile header: first cell and the counts of tile, first-ring and
    // second-ring cells, for the masks of each phase
    const gmem<int> *hd = gin(tl.hdr + 8 * t);
    const int g0 = hd[0], nt = hd[1], na = nt + hd[2], nl = na + hd[3];
    const bool p1 = tid < nl, p2 = c2 < na, p3 = lc3 < nt;
#pragma unroll
    for (int sl = 0; sl < D; sl++) la2[sl] = p2 ? la2[sl] : -1;
    const int g3 = g0 + (p3 ? lc3 : 0);
    const int la3 = (p3 && sl3 < D) ? a3 : -1;
    // the lane's face: the record as seen from the lane's cell (l n, r_self,
    // r_other), or from the other cell (-l n, r_other, r_self)
    const int rec = fc3 >= 0 ? fc3 >> 1 : 0;
    const T2 lnv = frt[rec], rav = frt[PF + rec], rbv = frt[2 * PF + rec];
    const bool flip = (fc3 & 1) != 0;
    const R lnx = flip ? -(R)lnv.x : (R)lnv.x, lny = flip ? -(R)lnv.y : (R)lnv.y;
    const R rsx = (R)(flip ? rbv.x : rav.x), rsy = (R)(flip ? rbv.y : rav.y);
    const R rox = (R)(flip ? rav.x : rbv.x), roy = (R)(flip ? rav.y : rbv.y);

    // ---- phase 1: macros and fbar+ of every local cell
    if (pb) {
        sbc[4 * tid] = (double)bcl.type;
        sbc[4 * tid + 1] = bcl.rho;
        sbc[4 * tid + 2] = bcl.u;
        sbc[4 * tid + 3] = bcl.v;
    }
    if (p1) {
        const double ir = 1.0 / r;
        const double ux = mu * ir, uy = mv * ir, uu = ux * ux + uy * uy;
        if (tid < na) {
            sW[tid] = r;
            sW[P1 + tid] = ux;
            sW[2 * P1 + tid] = uy;
        }
        if (tid < nt) {
            sM[tid] = mu;
            sM[PT + tid] = mv;
        }
        static_for<9>([&](auto I) {
            constexpr int i = I;
            const double fe = feq_c<cEx[i], cEy[i]>(cW[i], r, ux, uy, uu) - (DEV ? cW[i] * m.rho0 : 0.0);
            // NEQ: fv is f - feq, and a + b = 1 (both schemes)
            if constexpr (NEQ) sfbp[tid * 9 + i] = fe + ra * fv[i];
            else sfbp[tid * 9 + i] = ra * fv[i] + rb_ * (R)fe;
        });
    }
    __syncthreads();

    // ---- phase 2: gradients of the tile and its first ring
    if (p2) {
        if (!split) gradient_cell<0, 9, D>(sfbp, ssg, sW, sbc, P1, c2, la2, wx2, wy2);
        else if (tid < half) gradient_cell<0, 5, D>(sfbp, ssg, sW, sbc, P1, c2, la2, wx2, wy2);
        else gradient_cell<5, 9, D>(sfbp, ssg, sW, sbc, P1, c2, la2, wx2, wy2);
    }
    __syncthreads();

    // ---- phase 3: the face of each lane, per-cell sums, update
    // the lane's velocities in the update: sl3, sl3 + 4 and, on lane 0, 8
    // (the tile's own cells, just read in phase 1: cache hits)
    double fo0, fo1, fo2;
    if constexpr (S32) {
        fo0 = gin(s.f32)[(size_t)sl3 * np + g3];
        fo1 = gin(s.f32)[(size_t)(sl3 + 4) * np + g3];
        fo2 = gin(s.f32)[(size_t)8 * np + g3];
    } else {
        fo0 = gin(s.f)[(size_t)sl3 * np + g3];
        fo1 = gin(s.f)[(size_t)(sl3 + 4) * np + g3];
        fo2 = gin(s.f)[(size_t)8 * np + g3];
    }
    const double dtv = gin(m.dtv)[g3];
    R phi[9];
    double g0s = 0.0, g1s = 0.0, g2s = 0.0;
#pragma unroll
    for (int i = 0; i < 9; i++) phi[i] = 0;
    if (la3 != -1) {
        const int lc = lc3;
        R fbar[9];
        if (la3 >= 0) {
            // upwind side by the sign of e.n; exact tie: mean of both sides
            const int la = la3;
            static_for<9>([&](auto I) {
                constexpr int i = I, EX = cEx[i], EY = cEy[i];
                const R sn = cdot<EX, EY>(lnx, lny);
                const R rs = sfbp[lc * 9 + i] + csub<EX>(rsx, rdt) * ssg[lc * SG + i]
                             + csub<EY>(rsy, rdt) * ssg[lc * SG + 9 + i];
                const R ro = sfbp[la * 9 + i] + csub<EX>(rox, rdt) * ssg[la * SG + i]
                             + csub<EY>(roy, rdt) * ssg[la * SG + 9 + i];
                const R up = sn > (R)0 ? rs : ro;
                fbar[i] = sn == (R)0 ? (R)0.5 * (rs + ro) : up;
            });
        } else {
            const double r = sW[lc], ux = sW[P1 + lc], uy = sW[2 * P1 + lc];
            double rb, ub, vb;
            boundary_state_t(sbc, -2 - la3, r, ux, uy, rb, ub, vb);
            const double uu = ux * ux + uy * uy, uub = ub * ub + vb * vb;
            static_for<9>([&](auto I) {
                constexpr int i = I, EX = cEx[i], EY = cEy[i];
                const R sn = cdot<EX, EY>(lnx, lny);
                const R sx = ssg[lc * SG + i], sy = ssg[lc * SG + 9 + i];
                const R fb = sfbp[lc * 9 + i];
                const R inner = fb + csub<EX>(rsx, rdt) * sx + csub<EY>(rsy, rdt) * sy;
                // incoming: the boundary state's fbar+ carried to the foot point
                const R gb = (R)(feq_c<EX, EY>(cW[i], rb, ub, vb, uub) - feq_c<EX, EY>(cW[i], r, ux, uy, uu)) + fb;
                fbar[i] = sn >= (R)0 ? inner : gb - rdt * cdot<EX, EY>(sx, sy);
            });
        }
        // face macros (deviations in DEV: rho_f = rho0 + sum, momentum unchanged)
        R rsum = fbar[0], mx = 0, my = 0;
        static_for<9>([&](auto I) {
            constexpr int i = I;
            if constexpr (i > 0) rsum += fbar[i];
            if constexpr (cEx[i] != 0) mx += cmul<cEx[i]>(fbar[i]);
            if constexpr (cEy[i] != 0) my += cmul<cEy[i]>(fbar[i]);
        });
        const R rf = DEV ? (R)m.rho0 + rsum : rsum;
        const R irf = (R)1 / rf;
        const R uf = mx * irf, vf = my * irf;
        const R uu = uf * uf + vf * vf;
        static_for<9>([&](auto I) {
            constexpr int i = I, EX = cEx[i], EY = cEy[i];
            const R sn = cdot<EX, EY>(lnx, lny);
            R fe;
            if constexpr (DEV) {
                const R eu = cdot<EX, EY>(uf, vf);
                fe = (R)cW[i] * (rsum + rf * ((R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * uu));
            } else {
                fe = feq_c<EX, EY>((R)cW[i], rf, uf, vf, uu);
            }
            phi[i] = sn * (rc1 * (fbar[i] + rbf * fe));
            g0s += (double)phi[i];
            if constexpr (EX != 0) g1s += cmul<EX>((double)phi[i]);
            if constexpr (EY != 0) g2s += cmul<EY>((double)phi[i]);
        });
    }
#pragma unroll
    for (int i = 0; i < 9; i++) {
        if constexpr (PM == 1) phi[i] = lane_sum4_comp(phi[i]);
        else phi[i] = lane_sum4(phi[i]);
    }
    g0s = lane_sum4(g0s);
    g1s = lane_sum4(g1s);
    g2s = lane_sum4(g2s);
    if (p3) {
        const int lc = lc3, g = g3;
        double G0 = g0s, G1 = g1s, G2 = g2s;
        if (lagged) { G0 = gin(s.G)[g]; G1 = gin(s.G)[np + g]; G2 = gin(s.G)[2 * np + g]; }
        const double rn = sW[lc] - dtv * G0;
        const double mxn = sM[lc] - dtv * G1;
        const double myn = sM[PT + lc] - dtv * G2;
        if (sl3 == 0) gout(s.Wo)[g] = rn;
        if (sl3 == 1) gout(s.Wo)[np + g] = mxn;
        if (sl3 == 2) gout(s.Wo)[2 * np + g] = myn;
        if (lagged) {
            if (sl3 == 0) gout(s.Go)[g] = g0s;
            if (sl3 == 1) gout(s.Go)[np + g] = g1s;
            if (sl3 == 2) gout(s.Go)[2 * np + g] = g2s;
        }
        const double irn = 1.0 / rn;
        const double un = mxn * irn, vn = myn * irn, uun = un * un + vn * vn;
        const double inv = m.inv1l, lam = m.lam;
        // this lane's velocities: i0 = sl3 (rest, +x, +y, -x) and i1 = sl3 + 4
        // (-y, (1,1), (-1,1), (-1,-1)); their e.u, weights and fluxes
        const double eu0 = sl3 == 0 ? 0.0 : (sl3 == 1 ? un : (sl3 == 2 ? vn : -un));
        const double eu1 = sl3 == 0 ? -vn : (sl3 == 1 ? un + vn : (sl3 == 2 ? vn - un : -(un + vn)));
        const double w0 = sl3 == 0 ? cW[0] : cW[1], w1 = sl3 == 0 ? cW[4] : cW[5];
        const double F0 = sl3 == 0 ? phi[0] : (sl3 == 1 ? phi[1] : (sl3 == 2 ? phi[2] : phi[3]));
        const double F1 = sl3 == 0 ? phi[4] : (sl3 == 1 ? phi[5] : (sl3 == 2 ? phi[6] : phi[7]));
        const double base = 1.0 - 1.5 * uun;
        const int i0 = sl3, i1 = sl3 + 4;
        if constexpr (NEQ) {
            // f^n of this lane's velocities = feq(W^n) + the stored part
            const double ro = sW[lc], uo = sW[P1 + lc], vo = sW[2 * P1 + lc];
            const double bo = 1.0 - 1.5 * (uo * uo + vo * vo);
            const double e0 = sl3 == 0 ? 0.0 : (sl3 == 1 ? uo : (sl3 == 2 ? vo : -uo));
            const double e1 = sl3 == 0 ? -vo : (sl3 == 1 ? uo + vo : (sl3 == 2 ? vo - uo : -(uo + vo)));
            fo0 += w0 * ro * (bo + e0 * (3.0 + 4.5 * e0));
            fo1 += w1 * ro * (bo + e1 * (3.0 + 4.5 * e1));
            if (sl3 == 0) fo2 += feq_c<cEx[8], cEy[8]>(cW[8], ro, uo, vo, uo * uo + vo * vo);
        }
        const double fe0 = w0 * rn * (base + eu0 * (3.0 + 4.5 * eu0)) - (DEV ? w0 * m.rho0 : 0.0);
        const double fe1 = w1 * rn * (base + eu1 * (3.0 + 4.5 * eu1)) - (DEV ? w1 * m.rho0 : 0.0);
        double v0, v1;
        if (m.scheme == 0) {
            v0 = (fo0 - dtv * F0 + lam * fe0) * inv;
            v1 = (fo1 - dtv * F1 + lam * fe1) * inv;
        } else {
            // the original scheme: ft^{n+1} = (4/3) fbar+ - (1/3) ft - dt/V F
            v0 = (4.0 / 3.0) * (double)sfbp[lc * 9 + i0] - (1.0 / 3.0) * fo0 - dtv * F0;
            v1 = (4.0 / 3.0) * (double)sfbp[lc * 9 + i1] - (1.0 / 3.0) * fo1 - dtv * F1;
        }
        if constexpr (NEQ) { v0 -= fe0; v1 -= fe1; }          // store f^{n+1} - feq(W^{n+1})
        if constexpr (S32) { gout(s.fo32)[(size_t)i0 * np + g] = (float)v0; gout(s.fo32)[(size_t)i1 * np + g] = (float)v1; }
        else { gout(s.fo)[(size_t)i0 * np + g] = v0; gout(s.fo)[(size_t)i1 * np + g] = v1; }
        if (sl3 == 0) {
            const double fe2 = feq_c<cEx[8], cEy[8]>(cW[8], rn, un, vn, uun) - (DEV ? cW[8] * m.rho0 : 0.0);
            double v2;
            if (m.scheme == 0) {
                v2 = (fo2 - dtv * (double)phi[8] + lam * fe2) * inv;
            } else {
                v2 = (4.0 / 3.0) * (double)sfbp[lc * 9 + 8] - (1.0 / 3.0) * fo2 - dtv * (double)phi[8];
            }
            if constexpr (NEQ) v2 -= fe2;
            if constexpr (S32) gout(s.fo32)[(size_t)8 * np + g] = (float)v2;
            else gout(s.fo)[(size_t)8 * np + g] = v2;
        }
    }
}

// Workgroups are dealt round-robin to the XCDs: block b runs on XCD b % 8.
// Give XCD x the contiguous range [x * per, (x + 1) * per) of a sequence of
// slots (the grid a multiple of 8).
__device__ __forceinline__ int xcd_tile(int n)
{
    const int per = (n + kXcds - 1) / kXcds;
    return (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
}

// One block per tile: the tile of this block, XCD by XCD in contiguous ranges
// (xcd_range_start).  It follows from the block index and the grid size
// alone, so the first requests wait for nothing but the table pointers.
template <int D, int PM>
__global__ void __launch_bounds__(256) k_step_tiled(DevMesh m, DevTiles tl, DevState s, int lagged)
{
    const int x = (int)(blockIdx.x % kXcds);
    const int t = xcd_range_start((int)gridDim.x, x) + (int)(blockIdx.x / kXcds);
    step_tile<D, PM>(m, tl, s, lagged, t);
}

// Batched step: the tiles of all instances form one sequence; the grid covers
// a fixed capacity and each block reads its member and local tile from the
// device map (one load; member -1 past the live tiles), so the table can
// change between launches of a captured graph.  parity selects each
// instance's ping-pong buffers: it reads buffer (parity0 ^ parity).  Global
// memory is reached through global-address-space pointers (gin, gout in
// step_tile): the members' pointers come from their records, not from
// kernel arguments.
template <int D, int PM>
__global__ void __launch_bounds__(256) k_step_batch(BatchTable tab, int parity)
{
    // the slot's (member, tile) as one 8-byte load, so that the tile index
    // does not wait for the exit test on the member
    const unsigned long long slot = reinterpret_cast<const unsigned long long *>(tab.tmap)[xcd_tile((int)gridDim.x)];
    const int member = (int)(unsigned)slot, tile = (int)(unsigned)(slot >> 32);
    // the member's record copied once: its fields are then requested together
    // (no address depends on another field) and stay in scalar registers
    // across the barriers instead of being reloaded from memory.  A slot past
    // the live tiles (member -1) leaves without stepping (the compiler may
    // take that exit before the record is requested).
    const BatchInst &in = tab.inst[member < 0 ? 0 : member];
    const DevMesh m = in.m;
    const DevTiles tl = in.t;
    const bool sw = ((in.parity0 ^ parity) & 1) != 0;
    void *const f0 = in.f[0], *const f1 = in.f[1];
    double *const W0 = in.W[0], *const W1 = in.W[1], *const G0 = in.G[0], *const G1 = in.G[1];
    DevState s;
    s.W = sw ? W1 : W0; s.G = sw ? G1 : G0; s.Wo = sw ? W0 : W1; s.Go = sw ? G0 : G1;
    void *const fi = sw ? f1 : f0, *const fo = sw ? f0 : f1;
    s.f = reinterpret_cast<const double *>(fi);
    s.fo = reinterpret_cast<double *>(fo);
    s.f32 = reinterpret_cast<const float *>(fi);
    s.fo32 = reinterpret_cast<float *>(fo);
    if (member < 0) return;
    step_tile<D, PM>(m, tl, s, in.lagged, tile);
}

}  // namespace

size_t step_tiled_lds_bytes(const DevTiles &t, int mode, int n_bc)
{
    return tile_lds_bytes(t.nl_max, t.na_max, t.nt_max, n_bc, mode == 1 ? sizeof(float) : sizeof(double));
}

static unsigned step_tiled_grid(const DevTiles &t) { return (unsigned)t.n_tiles; }

// mode: 0 FP64, 1 FP32 deviation with FP32 face arithmetic, 2 FP32
// storage of f - feq(W) with FP64 arithmetic (the SDUGKS_FP64 / FP32DEV / FP32NEQ values)
hipError_t launch_step_tiled(const DevMesh &m, const DevTiles &t, const DevState &s, int lagged, int mode,
                             int block, hipStream_t st, GraphChain *gc)
{
    const size_t lds = step_tiled_lds_bytes(t, mode, m.n_bc);
    const dim3 grid(step_tiled_grid(t)), blk(block);
#define SDG_TILED(DD, PP) return emit(&k_step_tiled<DD, PP>, grid, blk, lds, st, gc, m, t, s, lagged)
    if (m.D <= 3) {
        if (mode == 1) SDG_TILED(3, 1);
        if (mode == 2) SDG_TILED(3, 2);
        SDG_TILED(3, 0);
    }
    if (mode == 1) SDG_TILED(4, 1);
    if (mode == 2) SDG_TILED(4, 2);
    SDG_TILED(4, 0);
#undef SDG_TILED
}

hipError_t launch_step_batch(const BatchTable &tab, int D, int mode, int parity, int cap_tiles, size_t lds,
                             int block, hipStream_t st, GraphChain *gc)
{
    const dim3 grid((unsigned)batch_grid(cap_tiles)), blk(block);
#define SDG_BATCH(DD, PP) return emit(&k_step_batch<DD, PP>, grid, blk, lds, st, gc, tab, parity)
    if (D <= 3) {
        if (mode == 1) SDG_BATCH(3, 1);
        if (mode == 2) SDG_BATCH(3, 2);
        SDG_BATCH(3, 0);
    }
    if (mode == 1) SDG_BATCH(4, 1);
    if (mode == 2) SDG_BATCH(4, 2);
    SDG_BATCH(4, 0);
#undef SDG_BATCH
}

}  // namespace sdg
