// Structured sDUGKS time step (Zhong et al., arXiv:2007.07347, Section II,
// the eleven-step summary) for tensor-product quad meshes: the cells are the
// rectangles of two coordinate arrays, so every face is normal to x or to y,
// each cell's least-squares stencil is its four face neighbours (or the wall
// face midpoints), and nothing about the geometry needs a table beyond one
// record per column and per row.  One workgroup of 256 threads per tile of
// 16 x 7 cells:
//
//   phase 1   fbar+ = a f + b feq(W) (Eq. fbarplus) of the tile and its two
//             halo rings (the cells within Manhattan distance 2) into LDS;
//   phase 2   the least-squares gradient (the LLSR normal equations, which
//             are diagonal on this stencil) of the tile and its first ring;
//   phase 3a  one lane per face: the tile's 17 x 7 faces normal to x on
//             threads 0..118 and its 16 x 8 faces normal to y on threads
//             128..255, each evaluated once: upwind reconstruction at the
//             foot point (Eq. fbpsource; the upwind side is known per velocity
//             at compile time), face macros and equilibrium, f at the face
//             (Eq. f_t_n+1), the six mesoscopic fluxes that cross a face
//             normal to that axis (Eq. MesoFlux) and the macroscopic flux
//             (Eq. MacroFlux, FP64); then into LDS over the fbar+ area;
//   phase 3b  one thread per tile cell: the fluxes of its four faces summed
//             in a fixed order, W^{n+1} (Eq. MacroUpdate), feq^{n+1}, f^{n+1}
//             (Eq. fn+1).
//
// A face on a tile edge is evaluated by both tiles from identical operands
// (the same cells, column and row records), so the flux that leaves one cell
// enters the other exactly.  Boundary faces follow Section III as in the
// general step: velocities entering the fluid take the boundary state's
// fbar+ carried to the foot point with the adjacent cell's gradient, the
// others the adjacent cell's reconstruction; the boundary state is a
// least-squares point at the face midpoint.  The three precision forms (PM)
// are those of the general step.
#include <type_traits>
#include <utility>

#include "d2q9.h"
#include "device.h"
#include "mesh.h"
#include "step_common.h"

namespace sdg {

namespace {

constexpr int TX = kCartTX, TY = kCartTY;      // tile cells
constexpr int BX = TX + 4, BY = TY + 4;        // box of the tile and both halo rings
constexpr int NB = BX * BY;
constexpr int NXF = (TX + 1) * TY;             // faces normal to x
constexpr int NYF = TX * (TY + 1);             // faces normal to y
constexpr int YF0 = 128;                       // first thread of the y faces
constexpr int NT = TX * TY;
constexpr int SG = kGradStride;
static_assert(NB <= 256 && NXF <= YF0 && YF0 + NYF <= 256 && NT <= 256, "tile does not fit 256 threads");

// the six velocities with a non-zero component along an axis, in order
constexpr int cXv[6] = {1, 3, 5, 6, 7, 8};
constexpr int cYv[6] = {2, 4, 5, 6, 7, 8};
// position of velocity i among them (-1: none)
constexpr int cXk[9] = {-1, 0, -1, 1, -1, 2, 3, 4, 5};
constexpr int cYk[9] = {-1, -1, 0, -1, 1, 2, 3, 4, 5};

// LDS layout (doubles first): rho, u, v of every box cell [3][NB]; momentum of
// the tile cells [2][NT]; then fbar+ [NB][9] and the gradient [NB][SG] of the
// storage type R (the face fluxes replace them after phase 3a: G of the x and
// y faces [3][NXF], [3][NYF] in FP64, then phi [6][NXF], [6][NYF] in R); then
// the boundary table [n_bc][4].
template <typename R>
__host__ __device__ constexpr size_t cart_head_bytes()
{
    return (3 * (size_t)NB + 2 * (size_t)NT) * 8 + ((9 + (size_t)SG) * NB * sizeof(R) + 15) / 16 * 16;
}

// Face of the tile along axis AX (0: normal +x, between the lower cell Lo =
// (i - 1, j) and the upper cell Hi = (i, j); 1: normal +y, between (i, j - 1)
// and (i, j)).  lo, hi: box indices (equal on a wall face, pointing at the
// fluid cell); hlo, hhi: the face offset from the lower and upper centres
// along the axis; len: face length; wall: 0 none, -1 the lower side is
// outside the fluid, +1 the upper side is; tag: its boundary entry.
// Writes the six fluxes phi of the velocities crossing the face (flux along
// +axis) and the macroscopic flux (mass, x- and y-momentum) in FP64.
template <int AX, int PM, typename R>
__device__ __forceinline__ void face_flux(const DevMesh &m, const R *sfbp, const R *ssg, const double *sW,
                                          const double *sbc, int lo, int hi, double hlo, double hhi, double len,
                                          int wall, int tag, R *phi, double &g0, double &g1, double &g2)
{
    constexpr bool DEV = PM == 1;
    const R rdt = (R)m.dtr, rc1 = (R)m.fc1, rbf = (R)m.fb;
    const R hl = (R)hlo, hh = (R)hhi;
    // boundary state of a wall face, seen from its fluid cell
    double rb = 0, ub = 0, vb = 0, rin = 0, uin = 0, vin = 0;
    const int in = wall < 0 ? hi : lo;
    if (wall != 0) {
        rin = sW[in];
        uin = sW[NB + in];
        vin = sW[2 * NB + in];
        boundary_state_t(sbc, tag, rin, uin, vin, rb, ub, vb);
    }
    R fbar[9];
    static_for<9>([&](auto I) {
        constexpr int i = I;
        constexpr int EN = AX == 0 ? cEx[i] : cEy[i];   // component along the face normal
        constexpr int ET = AX == 0 ? cEy[i] : cEx[i];   // tangential component
        constexpr int NO = AX == 0 ? 0 : 9, TO = AX == 0 ? 9 : 0;   // gradient rows: normal, tangential
        // reconstructions of the two sides at the foot point x_f - e_i dt
        // (the face midpoint lies on the row / column of both centres)
        R rlo = 0, rhi = 0;
        if constexpr (EN >= 0) {
            rlo = sfbp[lo * 9 + i] + csub<EN>(hl, rdt) * ssg[lo * SG + NO + i];
            if constexpr (ET != 0) rlo = csub<ET>(rlo, rdt * ssg[lo * SG + TO + i]);
        }
        if constexpr (EN <= 0) {
            rhi = sfbp[hi * 9 + i] + csub<EN>(hh, rdt) * ssg[hi * SG + NO + i];
            if constexpr (ET != 0) rhi = csub<ET>(rhi, rdt * ssg[hi * SG + TO + i]);
        }
        R v;
        if constexpr (EN > 0) v = rlo;
        else if constexpr (EN < 0) v = rhi;
        else v = wall < 0 ? rhi : (wall > 0 ? rlo : (R)0.5 * (rlo + rhi));
        // a velocity entering the fluid through a wall face: the boundary
        // state's fbar+ = feq_b + (fbar+_in - feq_in), carried to the foot point
        if constexpr (EN != 0) {
            if ((EN > 0 && wall < 0) || (EN < 0 && wall > 0)) {
                const double uu = uin * uin + vin * vin, uub = ub * ub + vb * vb;
                constexpr int EX = cEx[i], EY = cEy[i];
                const R gb = (R)(feq_c<EX, EY>(cW[i], rb, ub, vb, uub) - feq_c<EX, EY>(cW[i], rin, uin, vin, uu)) +
                             sfbp[in * 9 + i];
                v = gb - rdt * cdot<EX, EY>(ssg[in * SG + i], ssg[in * SG + 9 + i]);
            }
        }
        fbar[i] = v;
    });
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
    const R sl = (R)len;
    g0 = 0.0; g1 = 0.0; g2 = 0.0;
    static_for<6>([&](auto K) {
        constexpr int i = AX == 0 ? cXv[K] : cYv[K];
        constexpr int EX = cEx[i], EY = cEy[i], EN = AX == 0 ? EX : EY;
        R fe;
        if constexpr (DEV) {
            const R eu = cdot<EX, EY>(uf, vf);
            fe = (R)cW[i] * (rsum + rf * ((R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * uu));
        } else {
            fe = feq_c<EX, EY>((R)cW[i], rf, uf, vf, uu);
        }
        const R p = cmul<EN>(sl) * (rc1 * (fbar[i] + rbf * fe));
        phi[K] = p;
        g0 += (double)p;
        if constexpr (EX != 0) g1 += cmul<EX>((double)p);
        if constexpr (EY != 0) g2 += cmul<EY>((double)p);
    });
}

// Compensated sum a - b + c - d (TwoSum at each addition, errors added last).
__device__ __forceinline__ float sum4_comp(float a, float b, float c, float d)
{
    float s = a, e = 0.0f;
    const float t[3] = {-b, c, -d};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const float x = t[k], r = s + x, bb = r - s;
        e += (s - (r - bb)) + (x - bb);
        s = r;
    }
    return s + e;
}
__device__ __forceinline__ float sum2_comp(float a, float b)
{
    const float r = a - b, bb = r - a;
    return r + ((a - (r - bb)) + (-b - bb));
}

// One time step of tile t of a structured instance (the whole workgroup).
template <int PM>
__device__ __forceinline__ void cart_tile(const DevMesh &m, const DevCart &cg, const DevState &s, int lagged, int t)
{
    constexpr bool S32 = PM != 0;    // f stored in FP32
    constexpr bool DEV = PM == 1;    // FP32 arithmetic on deviations from w_i rho0
    constexpr bool NEQ = PM == 2;    // stored: f - feq(W); FP64 arithmetic
    using R = typename std::conditional<DEV, float, double>::type;
    extern __shared__ double smem[];
    double *sW = smem;                           // [3][NB]
    double *sM = smem + 3 * NB;                  // [2][NT]
    R *sfbp = reinterpret_cast<R *>(smem + 3 * NB + 2 * NT);
    R *ssg = sfbp + 9 * NB;
    double *sbc = reinterpret_cast<double *>(reinterpret_cast<char *>(smem) + cart_head_bytes<R>());
    // face fluxes, over fbar+ and the gradient once phase 3a has read them
    double *gxf = reinterpret_cast<double *>(sfbp);   // [3][NXF]
    double *gyf = gxf + 3 * NXF;                      // [3][NYF]
    R *pxf = reinterpret_cast<R *>(gyf + 3 * NYF);    // [6][NXF]
    R *pyf = pxf + 6 * NXF;                           // [6][NYF]

    const int tid = threadIdx.x;
    const int nx = cg.nx, ny = cg.ny, np = m.np;
    const int tx = t % cg.ntx, ty = t / cg.ntx;
    const int i0 = tx * TX, j0 = ty * TY;
    const int w = nx - i0 < TX ? nx - i0 : TX, h = ny - j0 < TY ? ny - j0 : TY;

    // ---- phase 1 cell: box cell tid, needed when within distance 2 of the tile
    const int bx = tid % BX, by = tid / BX;
    const int li = bx - 2, lj = by - 2;
    const int ddx = li < 0 ? -li : (li >= w ? li - w + 1 : 0);
    const int ddy = lj < 0 ? -lj : (lj >= h ? lj - h + 1 : 0);
    int gi = i0 + li, gj = j0 + lj;
    if (cg.per_x) gi = gi < 0 ? gi + nx : (gi >= nx ? gi - nx : gi);
    if (cg.per_y) gj = gj < 0 ? gj + ny : (gj >= ny ? gj - ny : gj);
    const bool inside = gi >= 0 && gi < nx && gj >= 0 && gj < ny;
    const bool p1 = tid < NB && ddx + ddy <= 2 && inside;
    const bool p2 = p1 && ddx + ddy <= 1;
    const int g1 = p1 ? cart_index(gi, gj, nx, ny) : 0;
    // requests of every phase at kernel start: the state of the box cell, the
    // column and row records phase 2 needs, the boundary table
    const double r = gin(s.W)[g1], mu = gin(s.W)[(size_t)np + g1], mv = gin(s.W)[2 * (size_t)np + g1];
    R fv[9];
#pragma unroll
    for (int i = 0; i < 9; i++) {
        if constexpr (S32) fv[i] = gin(s.f32)[(size_t)i * np + g1];
        else fv[i] = gin(s.f)[(size_t)i * np + g1];
    }
    const int ci = p1 ? gi : 0, cj = p1 ? gj : 0;
    const double wxl = gin(cg.col)[ci * kCartVals + 3], wxr = gin(cg.col)[ci * kCartVals + 4];
    const double wyl = gin(cg.row)[cj * kCartVals + 3], wyr = gin(cg.row)[cj * kCartVals + 4];
    const bool pb = tid < m.n_bc;
    const DevBC bcl = gin(m.bcs)[pb ? tid : 0];
    if (pb) {
        sbc[4 * tid] = (double)bcl.type;
        sbc[4 * tid + 1] = bcl.rho;
        sbc[4 * tid + 2] = bcl.u;
        sbc[4 * tid + 3] = bcl.v;
    }
    const R ra = (R)m.a, rb_ = (R)m.b;
    if (tid < NB) {
        if (p1) {
            const double ir = 1.0 / r;
            const double ux = mu * ir, uy = mv * ir, uu = ux * ux + uy * uy;
            sW[tid] = r;
            sW[NB + tid] = ux;
            sW[2 * NB + tid] = uy;
            if (ddx + ddy == 0) {
                sM[lj * TX + li] = mu;
                sM[NT + lj * TX + li] = mv;
            }
            static_for<9>([&](auto I) {
                constexpr int i = I;
                const double fe = feq_c<cEx[i], cEy[i]>(cW[i], r, ux, uy, uu) - (DEV ? cW[i] * m.rho0 : 0.0);
                if constexpr (NEQ) sfbp[tid * 9 + i] = fe + ra * fv[i];
                else sfbp[tid * 9 + i] = ra * fv[i] + rb_ * (R)fe;
            });
        } else {
            // cells outside the fluid or not needed: zeros, never selected
            sW[tid] = 1.0;
            sW[NB + tid] = 0.0;
            sW[2 * NB + tid] = 0.0;
#pragma unroll
            for (int i = 0; i < 9; i++) sfbp[tid * 9 + i] = 0;
        }
    }
    __syncthreads();

    // ---- phase 2: gradients of the tile and its first ring; a stencil point
    // outside the fluid is the wall face midpoint with fbar+_b - fbar+_c =
    // feq(rho_b, u_b) - feq(W_c)
    if (tid < NB) {
        R ax[9], ay[9];
#pragma unroll
        for (int i = 0; i < 9; i++) { ax[i] = 0; ay[i] = 0; }
        if (p2) {
            const int c = tid;
            const double rc = sW[c], uc = sW[NB + c], vc = sW[2 * NB + c];
            // the four stencil points: left, right, below, above
            static_for<4>([&](auto Q) {
                constexpr int q = Q;
                constexpr bool ax_x = q < 2;
                constexpr int di = q == 0 ? -1 : (q == 1 ? 1 : 0), dj = q == 2 ? -1 : (q == 3 ? 1 : 0);
                const int ni = gi + di, nj = gj + dj;
                bool out;
                int tag = 0;
                if constexpr (ax_x) {
                    out = !cg.per_x && (ni < 0 || ni >= nx);
                    if (out) tag = gin(cg.side)[2 * nx + (q == 0 ? 0 : ny) + gj];
                } else {
                    out = !cg.per_y && (nj < 0 || nj >= ny);
                    if (out) tag = gin(cg.side)[(q == 2 ? 0 : nx) + gi];
                }
                const R wq = (R)(q == 0 ? wxl : (q == 1 ? wxr : (q == 2 ? wyl : wyr)));
                const int nb = c + di + dj * BX;
                if (!out) {
                    static_for<9>([&](auto I) {
                        constexpr int i = I;
                        const R df = sfbp[nb * 9 + i] - sfbp[c * 9 + i];
                        if constexpr (ax_x) ax[i] += wq * df;
                        else ay[i] += wq * df;
                    });
                } else {
                    double rbq, ubq, vbq;
                    boundary_state_t(sbc, tag, rc, uc, vc, rbq, ubq, vbq);
                    const double uu = uc * uc + vc * vc, uub = ubq * ubq + vbq * vbq;
                    static_for<9>([&](auto I) {
                        constexpr int i = I;
                        const R df = (R)(feq_c<cEx[i], cEy[i]>(cW[i], rbq, ubq, vbq, uub) -
                                         feq_c<cEx[i], cEy[i]>(cW[i], rc, uc, vc, uu));
                        if constexpr (ax_x) ax[i] += wq * df;
                        else ay[i] += wq * df;
                    });
                }
            });
        }
#pragma unroll
        for (int i = 0; i < 9; i++) {
            ssg[tid * SG + i] = ax[i];
            ssg[tid * SG + 9 + i] = ay[i];
        }
    }
    __syncthreads();

    // ---- phase 3a: one lane per face
    R phi[6];
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    bool pf = false;
    int fidx = 0;
    if (tid < YF0) {
        // face normal to x at x_{i0 + fx}, row j0 + fy: lower cell box (fx + 1, fy + 2)
        const int fx = tid % (TX + 1), fy = tid / (TX + 1);
        pf = tid < NXF && fx <= w && fy < h;
        fidx = tid;
        if (pf) {
            const int ig = i0 + fx, jg = j0 + fy;
            const int wall = cg.per_x ? 0 : (ig == 0 ? -1 : (ig == nx ? 1 : 0));
            int lo = (fy + 2) * BX + fx + 1, hi = lo + 1;
            if (wall < 0) lo = hi;
            if (wall > 0) hi = lo;
            const int il = ig == 0 ? nx - 1 : ig - 1, ih = ig == nx ? 0 : ig;
            const double hlo = gin(cg.col)[il * kCartVals + 2], hhi = gin(cg.col)[ih * kCartVals + 1];
            const double len = gin(cg.row)[jg * kCartVals];
            const int tag = wall < 0 ? gin(cg.side)[2 * nx + jg] : (wall > 0 ? gin(cg.side)[2 * nx + ny + jg] : 0);
            face_flux<0, PM>(m, sfbp, ssg, sW, sbc, lo, hi, hlo, hhi, len, wall, tag, phi, q0, q1, q2);
        }
    } else {
        // face normal to y at y_{j0 + fy}, column i0 + fx: lower cell box (fx + 2, fy + 1)
        const int k = tid - YF0;
        const int fx = k % TX, fy = k / TX;
        pf = k < NYF && fx < w && fy <= h;
        fidx = k;
        if (pf) {
            const int ig = i0 + fx, jg = j0 + fy;
            const int wall = cg.per_y ? 0 : (jg == 0 ? -1 : (jg == ny ? 1 : 0));
            int lo = (fy + 1) * BX + fx + 2, hi = lo + BX;
            if (wall < 0) lo = hi;
            if (wall > 0) hi = lo;
            const int jl = jg == 0 ? ny - 1 : jg - 1, jh = jg == ny ? 0 : jg;
            const double hlo = gin(cg.row)[jl * kCartVals + 2], hhi = gin(cg.row)[jh * kCartVals + 1];
            const double len = gin(cg.col)[ig * kCartVals];
            const int tag = wall < 0 ? gin(cg.side)[ig] : (wall > 0 ? gin(cg.side)[nx + ig] : 0);
            face_flux<1, PM>(m, sfbp, ssg, sW, sbc, lo, hi, hlo, hhi, len, wall, tag, phi, q0, q1, q2);
        }
    }
    // the update's own-cell inputs, requested before the barriers
    const int lx = tid % TX, ly = tid / TX;
    const bool p3 = tid < NT && lx < w && ly < h;
    const int ui = i0 + (p3 ? lx : 0), uj = j0 + (p3 ? ly : 0);
    const int g3 = cart_index(ui, uj, nx, ny);
    double fo[9];
#pragma unroll
    for (int i = 0; i < 9; i++) {
        if constexpr (S32) fo[i] = gin(s.f32)[(size_t)i * np + g3];
        else fo[i] = gin(s.f)[(size_t)i * np + g3];
    }
    const double dtv = m.dt * (gin(cg.col)[ui * kCartVals + 5] * gin(cg.row)[uj * kCartVals + 5]);
    __syncthreads();
    if (pf) {
        if (tid < YF0) {
            gxf[fidx] = q0; gxf[NXF + fidx] = q1; gxf[2 * NXF + fidx] = q2;
#pragma unroll
            for (int k = 0; k < 6; k++) pxf[k * NXF + fidx] = phi[k];
        } else {
            gyf[fidx] = q0; gyf[NYF + fidx] = q1; gyf[2 * NYF + fidx] = q2;
#pragma unroll
            for (int k = 0; k < 6; k++) pyf[k * NYF + fidx] = phi[k];
        }
    }
    __syncthreads();

    // ---- phase 3b: the cell update
    if (!p3) return;
    const int xl = ly * (TX + 1) + lx, xr = xl + 1;    // x faces left and right of the cell
    const int yb = ly * TX + lx, yt = yb + TX;          // y faces below and above
    const int bc = (ly + 2) * BX + lx + 2;              // box index of the cell
    double G0 = (gxf[xr] - gxf[xl]) + (gyf[yt] - gyf[yb]);
    double G1 = (gxf[NXF + xr] - gxf[NXF + xl]) + (gyf[NYF + yt] - gyf[NYF + yb]);
    double G2 = (gxf[2 * NXF + xr] - gxf[2 * NXF + xl]) + (gyf[2 * NYF + yt] - gyf[2 * NYF + yb]);
    const double gs0 = G0, gs1 = G1, gs2 = G2;
    const int g = g3;
    if (lagged) { G0 = gin(s.G)[g]; G1 = gin(s.G)[np + g]; G2 = gin(s.G)[2 * np + g]; }
    const double ro = sW[bc], uo = sW[NB + bc], vo = sW[2 * NB + bc];
    const double rn = ro - dtv * G0;
    const double mxn = sM[ly * TX + lx] - dtv * G1;
    const double myn = sM[NT + ly * TX + lx] - dtv * G2;
    gout(s.Wo)[g] = rn;
    gout(s.Wo)[np + g] = mxn;
    gout(s.Wo)[2 * np + g] = myn;
    if (lagged) {
        gout(s.Go)[g] = gs0;
        gout(s.Go)[np + g] = gs1;
        gout(s.Go)[2 * np + g] = gs2;
    }
    const double irn = 1.0 / rn;
    const double un = mxn * irn, vn = myn * irn, uun = un * un + vn * vn;
    const double uuo = uo * uo + vo * vo;
    const double inv = m.inv1l, lam = m.lam;
    static_for<9>([&](auto I) {
        constexpr int i = I;
        constexpr int KX = cXk[i], KY = cYk[i];
        // mesoscopic flux of the cell: out through the right and top faces,
        // in through the left and bottom ones
        double F;
        if constexpr (DEV) {
            if constexpr (KX >= 0 && KY >= 0)
                F = (double)sum4_comp(pxf[KX * NXF + xr], pxf[KX * NXF + xl], pyf[KY * NYF + yt], pyf[KY * NYF + yb]);
            else if constexpr (KX >= 0) F = (double)sum2_comp(pxf[KX * NXF + xr], pxf[KX * NXF + xl]);
            else if constexpr (KY >= 0) F = (double)sum2_comp(pyf[KY * NYF + yt], pyf[KY * NYF + yb]);
            else F = 0.0;
        } else {
            if constexpr (KX >= 0 && KY >= 0)
                F = (pxf[KX * NXF + xr] - pxf[KX * NXF + xl]) + (pyf[KY * NYF + yt] - pyf[KY * NYF + yb]);
            else if constexpr (KX >= 0) F = pxf[KX * NXF + xr] - pxf[KX * NXF + xl];
            else if constexpr (KY >= 0) F = pyf[KY * NYF + yt] - pyf[KY * NYF + yb];
            else F = 0.0;
        }
        // f^n (FP32DEV: its deviation) and, for the original scheme, fbar+ of
        // the cell recomputed from it (the LDS copy now holds face fluxes)
        double f0 = fo[i];
        const double feo = feq_c<cEx[i], cEy[i]>(cW[i], ro, uo, vo, uuo) - (DEV ? cW[i] * m.rho0 : 0.0);
        if constexpr (NEQ) f0 += feo;
        const double fe = feq_c<cEx[i], cEy[i]>(cW[i], rn, un, vn, uun) - (DEV ? cW[i] * m.rho0 : 0.0);
        double v;
        if (m.scheme == 0) v = (f0 - dtv * F + lam * fe) * inv;
        else v = (4.0 / 3.0) * (m.a * f0 + m.b * feo) - (1.0 / 3.0) * f0 - dtv * F;
        if constexpr (NEQ) v -= fe;
        if constexpr (S32) gout(s.fo32)[(size_t)i * np + g] = (float)v;
        else gout(s.fo)[(size_t)i * np + g] = v;
    });
}

// One workgroup per tile, XCD by XCD in contiguous ranges of the row-major
// tile order.
template <int PM>
__global__ void __launch_bounds__(256) k_step_cart(DevMesh m, DevCart c, DevState s, int lagged)
{
    const int x = (int)(blockIdx.x % kXcds);
    const int t = xcd_range_start((int)gridDim.x, x) + (int)(blockIdx.x / kXcds);
    cart_tile<PM>(m, c, s, lagged, t);
}

// Batched structured step: as the batched general step, the slot map gives
// each workgroup its member and tile.
template <int PM>
__global__ void __launch_bounds__(256) k_step_batch_cart(BatchTable tab, int parity)
{
    const int x = (int)(blockIdx.x % kXcds);
    const int per = (int)gridDim.x / kXcds;
    const unsigned long long slot = reinterpret_cast<const unsigned long long *>(tab.tmap)[x * per + (int)(blockIdx.x / kXcds)];
    const int member = (int)(unsigned)slot, tile = (int)(unsigned)(slot >> 32);
    const BatchInst &in = tab.inst[member < 0 ? 0 : member];
    const DevMesh m = in.m;
    const DevCart cg = in.c;
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
    cart_tile<PM>(m, cg, s, in.lagged, tile);
}

}  // namespace

size_t step_cart_lds_bytes(int mode, int n_bc)
{
    return (mode == 1 ? cart_head_bytes<float>() : cart_head_bytes<double>()) + 32 * (size_t)n_bc;
}

hipError_t launch_step_cart(const DevMesh &m, const DevCart &c, const DevState &s, int lagged, int mode,
                            hipStream_t st, GraphChain *gc)
{
    const size_t lds = step_cart_lds_bytes(mode, m.n_bc);
    const dim3 grid((unsigned)(c.ntx * c.nty)), blk(256);
    if (mode == 1) return emit(&k_step_cart<1>, grid, blk, lds, st, gc, m, c, s, lagged);
    if (mode == 2) return emit(&k_step_cart<2>, grid, blk, lds, st, gc, m, c, s, lagged);
    return emit(&k_step_cart<0>, grid, blk, lds, st, gc, m, c, s, lagged);
}

hipError_t launch_step_batch_cart(const BatchTable &tab, int mode, int parity, int cap_tiles, size_t lds,
                                  hipStream_t st, GraphChain *gc)
{
    const dim3 grid((unsigned)batch_grid(cap_tiles)), blk(256);
    if (mode == 1) return emit(&k_step_batch_cart<1>, grid, blk, lds, st, gc, tab, parity);
    if (mode == 2) return emit(&k_step_batch_cart<2>, grid, blk, lds, st, gc, tab, parity);
    return emit(&k_step_batch_cart<0>, grid, blk, lds, st, gc, tab, parity);
}

}  // namespace sdg
