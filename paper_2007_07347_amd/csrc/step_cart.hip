// Structured sDUGKS time step (Zhong et al., arXiv:2007.07347, Section II,
// the eleven-step summary) for tensor-product quad meshes: the cells are the
// rectangles of two coordinate arrays, so every face is normal to x or to y,
// each cell's least-squares stencil is its four face neighbours (or the wall
// face midpoints), and nothing about the geometry needs a table beyond one
// record per column and per row.  One workgroup per tile of 16 x TY cells
// (TY = 14 on 512 threads for FP32 deviations, 7 on 256 threads for the forms
// with FP64 face arithmetic, whose LDS values are twice as wide):
//
//   phase 1   fbar+ = a f + b feq(W) (Eq. fbarplus) of the tile and its two
//             halo rings (the cells within Manhattan distance 2) into LDS;
//   phase 2   the least-squares gradient (the LLSR normal equations, which
//             are diagonal on this stencil) of the tile and its first ring;
//   phase 3a  one lane per face: the tile's 17 x TY faces normal to x on the
//             first half of the threads and its 16 x (TY + 1) faces normal to
//             y on the second, each evaluated once: upwind reconstruction at
//             the foot point (Eq. fbpsource; the upwind side is known per
//             velocity at compile time), face macros and equilibrium, f at the
//             face (Eq. f_t_n+1), the six mesoscopic fluxes that cross a face
//             normal to that axis (Eq. MesoFlux) and the macroscopic flux
//             (Eq. MacroFlux), both kept in FP64 in LDS over the fbar+ area;
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
#include <cstdint>
#include <type_traits>
#include <utility>

#include "d2q9.h"
#include "device.h"
#include "mesh.h"
#include "step_common.h"

namespace sdg {

namespace {

constexpr int SG = kGradStride;

// Tile of step form PM.
template <int PM>
struct Shape {
    static constexpr int TX = kCartTX, TY = cart_tile_rows(PM);
    static constexpr int NTHR = PM == SDUGKS_FP32DEV ? 512 : 256;
    static constexpr int BX = TX + 4, BY = TY + 4, NB = BX * BY;      // tile and both halo rings
    static constexpr int IX = TX + 2, IY = TY + 2, NI = IX * IY;      // tile and its first ring
    static constexpr int NXF = (TX + 1) * TY, NYF = TX * (TY + 1);    // faces normal to x, to y
    static constexpr int YF0 = NTHR / 2;                               // first thread of the y faces
    static constexpr int NT = TX * TY;
    using R = typename std::conditional<PM == SDUGKS_FP32DEV, float, double>::type;
    // LDS (doubles first): rho, u, v of every box cell [3][NB]; momentum of
    // the tile cells [2][NT]; then, in R, fbar+ [NB][9] and the gradient of
    // the inner box [NI][SG]; after phase 3a the same area holds, in FP64, G
    // of the x and y faces [3][NXF], [3][NYF] and phi [6][NXF], [6][NYF];
    // then the boundary table [n_bc][4].
    static constexpr size_t AREA = (9 * (size_t)NB + (size_t)SG * NI) * sizeof(R);
    static constexpr size_t HEAD = (3 * (size_t)NB + 2 * (size_t)NT) * 8 + (AREA + 15) / 16 * 16;
    static_assert(NB <= NTHR && NI <= NTHR && NXF <= YF0 && NYF <= NTHR - YF0 && NT <= NTHR,
                  "tile does not fit its workgroup");
    static_assert(9 * (size_t)(NXF + NYF) * 8 <= AREA, "face fluxes do not fit the fbar+ area");
};

// the six velocities with a non-zero component along an axis, in order
constexpr int cXv[6] = {1, 3, 5, 6, 7, 8};
constexpr int cYv[6] = {2, 4, 5, 6, 7, 8};
// position of velocity i among them (-1: none)
constexpr int cXk[9] = {-1, 0, -1, 1, -1, 2, 3, 4, 5};
constexpr int cYk[9] = {-1, -1, 0, -1, 1, 2, 3, 4, 5};
constexpr bool positions_match()
{
    for (int k = 0; k < 6; k++)
        if (cXk[cXv[k]] != k || cYk[cYv[k]] != k || cEx[cXv[k]] == 0 || cEy[cYv[k]] == 0) return false;
    return true;
}
static_assert(positions_match(), "velocity positions along the axes");

// Element i of a row that starts at base, addressed as base + a 32-bit byte
// offset: the base stays a scalar and the lanes add one unsigned offset (the
// mesh build keeps every row of a structured instance under 4 GiB).
template <typename T>
__device__ __forceinline__ T ld_at(const T *base, uint32_t i)
{
    return *(const gmem<T> *)((const gmem<char> *)gin(base) + i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st_at(T *base, uint32_t i, T v)
{
    *(gmem<T> *)((gmem<char> *)gout(base) + i * (uint32_t)sizeof(T)) = v;
}

// The nine equilibria of Eq. Feq (its second-order discrete form) minus
// w_i off, grouped by opposite velocities: for a lattice direction d with
// weight w_d, f(+d) = w_d (S_d + 3 d.m) and f(-d) = w_d (S_d - 3 d.m), where
// S_d = B + 4.5 (d.m)(d.u), B = (rho - off) - 1.5 rho u.u and m = rho u.
template <typename T>
__device__ __forceinline__ void feq9(T rho, T mx, T my, T ux, T uy, T off, T fe[9])
{
    const T B = (rho - off) - (T)1.5 * rho * (ux * ux + uy * uy);
    fe[0] = (T)(4.0 / 9.0) * B;
    auto pair = [&](int ip, int im, T w, T dm, T du) {
        const T S = B + (T)4.5 * dm * du, A = (T)3 * dm;
        fe[ip] = w * (S + A);
        fe[im] = w * (S - A);
    };
    pair(1, 3, (T)(1.0 / 9.0), mx, ux);
    pair(2, 4, (T)(1.0 / 9.0), my, uy);
    pair(5, 7, (T)(1.0 / 36.0), mx + my, ux + uy);
    pair(6, 8, (T)(1.0 / 36.0), my - mx, uy - ux);
}

// Face of the tile along axis AX (0: normal +x, between the lower cell (i - 1,
// j) and the upper cell (i, j); 1: normal +y, between (i, j - 1) and (i, j)).
// lob, hib: box indices of the two cells, loi, hii: their inner-box indices
// (equal on a wall face, pointing at the fluid cell); hlo, hhi: the face
// offset from the lower and upper centres along the axis; len: face length;
// wall: 0 none, -1 the lower side is outside the fluid, +1 the upper side is;
// tag: its boundary entry.  Writes the six fluxes phi of the velocities
// crossing the face (flux along +axis, in the order of cXv / cYv) and the
// macroscopic flux (mass, x- and y-momentum), all in FP64.
template <int AX, int PM>
__device__ __forceinline__ void face_flux(const DevMesh &m, const typename Shape<PM>::R *sfbp,
                                          const typename Shape<PM>::R *ssg, const double *sW, const double *sbc,
                                          int lob, int hib, int loi, int hii, double hlo, double hhi, double len,
                                          int wall, int tag, double *phi, double &g0, double &g1, double &g2)
{
    using S = Shape<PM>;
    using R = typename S::R;
    constexpr bool DEV = PM == SDUGKS_FP32DEV;
    const R rdt = (R)m.dtr, rc1 = (R)m.fc1, rbf = (R)m.fb;
    // reconstruction offsets along the normal from the upwind centre: h - e_n dt
    const R lom = (R)hlo - rdt, hip = (R)hhi + rdt;
    // boundary state of a wall face, seen from its fluid cell
    double rb = 0, ub = 0, vb = 0, rin = 0, uin = 0, vin = 0;
    const int inb = wall < 0 ? hib : lob, ini = wall < 0 ? hii : loi;
    if (wall != 0) {
        rin = sW[inb];
        uin = sW[S::NB + inb];
        vin = sW[2 * S::NB + inb];
        boundary_state_t(sbc, tag, rin, uin, vin, rb, ub, vb);
    }
    R fbar[9];
    static_for<9>([&](auto I) {
        constexpr int i = I;
        constexpr int EN = AX == 0 ? cEx[i] : cEy[i];   // component along the face normal
        constexpr int ET = AX == 0 ? cEy[i] : cEx[i];   // tangential component
        constexpr int NO = AX == 0 ? 0 : 9, TO = AX == 0 ? 9 : 0;   // gradient rows: normal, tangential
        // reconstructions of the two sides at the foot point x_f - e_i dt
        // (the face midpoint lies on the row / column of both centres); on a
        // wall face both sides are the fluid cell with the same offset, so
        // the average of a tangential velocity is that cell's value
        R rlo = 0, rhi = 0;
        if constexpr (EN >= 0) {
            rlo = sfbp[lob * 9 + i] + (EN > 0 ? lom : (R)hlo) * ssg[loi * SG + NO + i];
            if constexpr (ET != 0) rlo = csub<ET>(rlo, rdt * ssg[loi * SG + TO + i]);
        }
        if constexpr (EN <= 0) {
            rhi = sfbp[hib * 9 + i] + (EN < 0 ? hip : (R)hhi) * ssg[hii * SG + NO + i];
            if constexpr (ET != 0) rhi = csub<ET>(rhi, rdt * ssg[hii * SG + TO + i]);
        }
        if constexpr (EN > 0) fbar[i] = rlo;
        else if constexpr (EN < 0) fbar[i] = rhi;
        else fbar[i] = (R)0.5 * (rlo + rhi);
    });
    if (wall != 0) {
        // a velocity entering the fluid through a wall face: the boundary
        // state's fbar+ = feq_b + (fbar+_in - feq_in), carried to the foot point
        const double uu = uin * uin + vin * vin, uub = ub * ub + vb * vb;
        static_for<9>([&](auto I) {
            constexpr int i = I;
            constexpr int EN = AX == 0 ? cEx[i] : cEy[i];
            if constexpr (EN != 0) {
                if ((EN > 0 && wall < 0) || (EN < 0 && wall > 0)) {
                    constexpr int EX = cEx[i], EY = cEy[i];
                    const R gb = (R)(feq_c<EX, EY>(cW[i], rb, ub, vb, uub) -
                                     feq_c<EX, EY>(cW[i], rin, uin, vin, uu)) + sfbp[inb * 9 + i];
                    fbar[i] = gb - rdt * cdot<EX, EY>(ssg[ini * SG + i], ssg[ini * SG + 9 + i]);
                }
            }
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
    R irf;
    if constexpr (DEV) irf = __builtin_amdgcn_rcpf(rf);
    else irf = (R)1 / rf;
    const R uf = mx * irf, vf = my * irf;
    // the equilibria by opposite pairs (as feq9; DEV: B from the deviation sum)
    const R B = (DEV ? rsum : rf) - (R)1.5 * rf * (uf * uf + vf * vf);
    const R C = (R)len * rc1, K1 = C * rbf * (R)(1.0 / 9.0), K5 = C * rbf * (R)(1.0 / 36.0);
    // phi(+d) = C (fbar(+d) + fb feq(+d)), phi(-d) = -C (fbar(-d) + fb feq(-d)),
    // d the member of the pair that points along +axis
    auto pr = [&](int kp, int km, int ip, int im, R K, R dm, R du) {
        const R Sd = B + (R)4.5 * dm * du, A = (R)3 * dm;
        phi[kp] = (double)(C * fbar[ip] + K * (Sd + A));
        phi[km] = (double)(-(C * fbar[im] + K * (Sd - A)));
    };
    if constexpr (AX == 0) {
        pr(0, 1, 1, 3, K1, mx, uf);              // (1, 0) and (-1, 0)
        pr(2, 4, 5, 7, K5, mx + my, uf + vf);    // (1, 1) and (-1, -1)
        pr(5, 3, 8, 6, K5, mx - my, uf - vf);    // (1, -1) and (-1, 1)
        const double s0 = phi[0] + phi[1], s1 = phi[2] + phi[4], s2 = phi[5] + phi[3];
        const double d0 = phi[0] - phi[1], d1 = phi[2] - phi[4], d2 = phi[5] - phi[3];
        g0 = (s0 + s1) + s2;
        g1 = (d0 + d1) + d2;
        g2 = d1 - d2;
    } else {
        pr(0, 1, 2, 4, K1, my, vf);              // (0, 1) and (0, -1)
        pr(2, 4, 5, 7, K5, mx + my, uf + vf);    // (1, 1) and (-1, -1)
        pr(3, 5, 6, 8, K5, my - mx, vf - uf);    // (-1, 1) and (1, -1)
        const double s0 = phi[0] + phi[1], s1 = phi[2] + phi[4], s2 = phi[3] + phi[5];
        const double d0 = phi[0] - phi[1], d1 = phi[2] - phi[4], d2 = phi[3] - phi[5];
        g0 = (s0 + s1) + s2;
        g1 = d1 - d2;
        g2 = (d0 + d1) + d2;
    }
}

// Cell (i, j) of the box around the tile at (i0, j0) with w x h cells: its
// global column and row after periodic wrapping, whether it is a fluid cell,
// and its Manhattan distance from the tile.
struct BoxCell {
    int gi, gj, dist;
    bool inside;
};
__device__ __forceinline__ BoxCell box_cell(const DevCart &cg, int i0, int j0, int w, int h, int li, int lj)
{
    BoxCell b;
    const int ddx = li < 0 ? -li : (li >= w ? li - w + 1 : 0);
    const int ddy = lj < 0 ? -lj : (lj >= h ? lj - h + 1 : 0);
    b.dist = ddx + ddy;
    int gi = i0 + li, gj = j0 + lj;
    if (cg.per_x) gi = gi < 0 ? gi + cg.nx : (gi >= cg.nx ? gi - cg.nx : gi);
    if (cg.per_y) gj = gj < 0 ? gj + cg.ny : (gj >= cg.ny ? gj - cg.ny : gj);
    b.inside = gi >= 0 && gi < cg.nx && gj >= 0 && gj < cg.ny;
    b.gi = gi;
    b.gj = gj;
    return b;
}

// One time step of tile t of a structured instance (the whole workgroup).
template <int PM>
__device__ __forceinline__ void cart_tile(const DevMesh &m, const DevCart &cg, const DevState &s, int lagged, int t)
{
    using S = Shape<PM>;
    using R = typename S::R;
    constexpr int TX = S::TX, TY = S::TY, BX = S::BX, NB = S::NB, IX = S::IX, NI = S::NI;
    constexpr int NXF = S::NXF, NYF = S::NYF, YF0 = S::YF0, NT = S::NT;
    constexpr bool S32 = PM != SDUGKS_FP64;        // f stored in FP32
    constexpr bool DEV = PM == SDUGKS_FP32DEV;     // FP32 arithmetic on deviations from w_i rho0
    constexpr bool NEQ = PM == SDUGKS_FP32NEQ;     // stored: f - feq(W); FP64 arithmetic
    extern __shared__ double smem[];
    double *sW = smem;                           // [3][NB]
    double *sM = smem + 3 * NB;                  // [2][NT]
    R *sfbp = reinterpret_cast<R *>(smem + 3 * NB + 2 * NT);
    R *ssg = sfbp + 9 * NB;
    double *sbc = reinterpret_cast<double *>(reinterpret_cast<char *>(smem) + S::HEAD);
    // face fluxes, over fbar+ and the gradient once phase 3a has read them
    double *gxf = reinterpret_cast<double *>(sfbp);   // [3][NXF]
    double *gyf = gxf + 3 * NXF;                      // [3][NYF]
    double *pxf = gyf + 3 * NYF;                      // [6][NXF]
    double *pyf = pxf + 6 * NXF;                      // [6][NYF]

    const int tid = threadIdx.x;
    const int nx = cg.nx, ny = cg.ny, np = m.np;
    const int tx = t % cg.ntx, ty = t / cg.ntx;
    const int i0 = tx * TX, j0 = ty * TY;
    const int w = nx - i0 < TX ? nx - i0 : TX, h = ny - j0 < TY ? ny - j0 : TY;
    const double *W0 = s.W, *W1 = s.W + np, *W2 = s.W + 2 * (size_t)np;

    // ---- requests of every phase at kernel start
    // phase 1: box cell tid, needed when within distance 2 of the tile
    const int bx = tid % BX, by = tid / BX;
    const BoxCell c1 = box_cell(cg, i0, j0, w, h, bx - 2, by - 2);
    const bool p1 = tid < NB && c1.dist <= 2 && c1.inside;
    const uint32_t g1 = p1 ? (uint32_t)cart_index(c1.gi, c1.gj, nx, ny) : 0u;
    const double r = ld_at(W0, g1), mu = ld_at(W1, g1), mv = ld_at(W2, g1);
    R fv[9];
#pragma unroll
    for (int i = 0; i < 9; i++) {
        if constexpr (S32) fv[i] = ld_at(s.f32 + (size_t)i * np, g1);
        else fv[i] = ld_at(s.f + (size_t)i * np, g1);
    }
    // phase 2: inner-box cell tid, needed within distance 1; its column and
    // row least-squares weights
    const int ix = tid % IX, iy = tid / IX;
    const BoxCell c2 = box_cell(cg, i0, j0, w, h, ix - 1, iy - 1);
    const bool p2 = tid < NI && c2.dist <= 1 && c2.inside;
    const int ci = p2 ? c2.gi : 0, cj = p2 ? c2.gj : 0;
    const double wxl = ld_at(cg.col, (uint32_t)(ci * kCartVals + 3)), wxr = ld_at(cg.col, (uint32_t)(ci * kCartVals + 4));
    const double wyl = ld_at(cg.row, (uint32_t)(cj * kCartVals + 3)), wyr = ld_at(cg.row, (uint32_t)(cj * kCartVals + 4));
    // the boundary table
    const bool pb = tid < m.n_bc;
    const DevBC bcl = gin(m.bcs)[pb ? tid : 0];
    if (pb) {
        sbc[4 * tid] = (double)bcl.type;
        sbc[4 * tid + 1] = bcl.rho;
        sbc[4 * tid + 2] = bcl.u;
        sbc[4 * tid + 3] = bcl.v;
    }

    // ---- phase 1
    const R ra = (R)m.a, rb_ = (R)m.b;
    if (tid < NB) {
        if (p1) {
            const double ir = 1.0 / r;
            const double ux = mu * ir, uy = mv * ir;
            sW[tid] = r;
            sW[NB + tid] = ux;
            sW[2 * NB + tid] = uy;
            if (c1.dist == 0) {
                sM[(by - 2) * TX + bx - 2] = mu;
                sM[NT + (by - 2) * TX + bx - 2] = mv;
            }
            double fe[9];
            feq9(r, mu, mv, ux, uy, DEV ? m.rho0 : 0.0, fe);
#pragma unroll
            for (int i = 0; i < 9; i++) {
                if constexpr (NEQ) sfbp[tid * 9 + i] = fe[i] + ra * fv[i];
                else sfbp[tid * 9 + i] = ra * fv[i] + rb_ * (R)fe[i];
            }
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
    if (tid < NI) {
        R ax[9], ay[9];
#pragma unroll
        for (int i = 0; i < 9; i++) { ax[i] = 0; ay[i] = 0; }
        if (p2) {
            const int c = (iy + 1) * BX + ix + 1;   // box index
            // the four stencil points: left, right, below, above
            static_for<4>([&](auto Q) {
                constexpr int q = Q;
                constexpr bool ax_x = q < 2;
                constexpr int di = q == 0 ? -1 : (q == 1 ? 1 : 0), dj = q == 2 ? -1 : (q == 3 ? 1 : 0);
                const int ni = c2.gi + di, nj = c2.gj + dj;
                bool out;
                int tag = 0;
                if constexpr (ax_x) {
                    out = !cg.per_x && (ni < 0 || ni >= nx);
                    if (out) tag = gin(cg.side)[2 * nx + (q == 0 ? 0 : ny) + c2.gj];
                } else {
                    out = !cg.per_y && (nj < 0 || nj >= ny);
                    if (out) tag = gin(cg.side)[(q == 2 ? 0 : nx) + c2.gi];
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
                    const double rc = sW[c], uc = sW[NB + c], vc = sW[2 * NB + c];
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
    double phi[6];
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    bool pf = false;
    int fidx = 0;
    if (tid < YF0) {
        // face normal to x at x_{i0 + fx}, row j0 + fy: lower cell box (fx + 1,
        // fy + 2), inner box (fx, fy + 1)
        const int fx = tid % (TX + 1), fy = tid / (TX + 1);
        pf = tid < NXF && fx <= w && fy < h;
        fidx = tid;
        if (pf) {
            const int ig = i0 + fx, jg = j0 + fy;
            const int wall = cg.per_x ? 0 : (ig == 0 ? -1 : (ig == nx ? 1 : 0));
            int lob = (fy + 2) * BX + fx + 1, hib = lob + 1, loi = (fy + 1) * IX + fx, hii = loi + 1;
            const int il = ig == 0 ? nx - 1 : ig - 1, ih = ig == nx ? 0 : ig;
            double hlo = ld_at(cg.col, (uint32_t)(il * kCartVals + 2));
            double hhi = ld_at(cg.col, (uint32_t)(ih * kCartVals + 1));
            if (wall < 0) { lob = hib; loi = hii; hlo = hhi; }
            if (wall > 0) { hib = lob; hii = loi; hhi = hlo; }
            const double len = ld_at(cg.row, (uint32_t)(jg * kCartVals));
            const int tag = wall < 0 ? gin(cg.side)[2 * nx + jg] : (wall > 0 ? gin(cg.side)[2 * nx + ny + jg] : 0);
            face_flux<0, PM>(m, sfbp, ssg, sW, sbc, lob, hib, loi, hii, hlo, hhi, len, wall, tag, phi, q0, q1, q2);
        }
    } else {
        // face normal to y at y_{j0 + fy}, column i0 + fx: lower cell box (fx + 2,
        // fy + 1), inner box (fx + 1, fy)
        const int k = tid - YF0;
        const int fx = k % TX, fy = k / TX;
        pf = k < NYF && fx < w && fy <= h;
        fidx = k;
        if (pf) {
            const int ig = i0 + fx, jg = j0 + fy;
            const int wall = cg.per_y ? 0 : (jg == 0 ? -1 : (jg == ny ? 1 : 0));
            int lob = (fy + 1) * BX + fx + 2, hib = lob + BX, loi = fy * IX + fx + 1, hii = loi + IX;
            const int jl = jg == 0 ? ny - 1 : jg - 1, jh = jg == ny ? 0 : jg;
            double hlo = ld_at(cg.row, (uint32_t)(jl * kCartVals + 2));
            double hhi = ld_at(cg.row, (uint32_t)(jh * kCartVals + 1));
            if (wall < 0) { lob = hib; loi = hii; hlo = hhi; }
            if (wall > 0) { hib = lob; hii = loi; hhi = hlo; }
            const double len = ld_at(cg.col, (uint32_t)(ig * kCartVals));
            const int tag = wall < 0 ? gin(cg.side)[ig] : (wall > 0 ? gin(cg.side)[nx + ig] : 0);
            face_flux<1, PM>(m, sfbp, ssg, sW, sbc, lob, hib, loi, hii, hlo, hhi, len, wall, tag, phi, q0, q1, q2);
        }
    }
    // the update's own-cell inputs, requested before the barriers
    const int lx = tid % TX, ly = tid / TX;
    const bool p3 = tid < NT && lx < w && ly < h;
    uint32_t g = 0;
    typename std::conditional<S32, float, double>::type fo[9];
    double dtv = 0.0;
    if (p3) {
        g = (uint32_t)cart_index(i0 + lx, j0 + ly, nx, ny);
#pragma unroll
        for (int i = 0; i < 9; i++) {
            if constexpr (S32) fo[i] = ld_at(s.f32 + (size_t)i * np, g);
            else fo[i] = ld_at(s.f + (size_t)i * np, g);
        }
        dtv = m.dt * (ld_at(cg.col, (uint32_t)((i0 + lx) * kCartVals + 5)) *
                      ld_at(cg.row, (uint32_t)((j0 + ly) * kCartVals + 5)));
    }
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
    const double ro = sW[bc], uo = sW[NB + bc], vo = sW[2 * NB + bc];
    const double mxo = sM[ly * TX + lx], myo = sM[NT + ly * TX + lx];
    if (lagged) {
        G0 = ld_at(s.G, g);
        G1 = ld_at(s.G + np, g);
        G2 = ld_at(s.G + 2 * (size_t)np, g);
    }
    const double rn = ro - dtv * G0;
    const double mxn = mxo - dtv * G1;
    const double myn = myo - dtv * G2;
    st_at(s.Wo, g, rn);
    st_at(s.Wo + np, g, mxn);
    st_at(s.Wo + 2 * (size_t)np, g, myn);
    if (lagged) {
        st_at(s.Go, g, gs0);
        st_at(s.Go + np, g, gs1);
        st_at(s.Go + 2 * (size_t)np, g, gs2);
    }
    const double irn = 1.0 / rn;
    const double off = DEV ? m.rho0 : 0.0;
    double fe[9], feo[9];
    feq9(rn, mxn, myn, mxn * irn, myn * irn, off, fe);
    // f^n from its stored form, and feq(W^n) where the form or the original
    // scheme needs it (the LDS copy of fbar+ now holds face fluxes)
    if (NEQ || m.scheme != 0) feq9(ro, mxo, myo, uo, vo, off, feo);
    const double inv = m.inv1l, lam = m.lam;
    static_for<9>([&](auto I) {
        constexpr int i = I;
        constexpr int KX = cXk[i], KY = cYk[i];
        // mesoscopic flux of the cell: out through the right and top faces,
        // in through the left and bottom ones
        double F;
        if constexpr (KX >= 0 && KY >= 0)
            F = (pxf[KX * NXF + xr] - pxf[KX * NXF + xl]) + (pyf[KY * NYF + yt] - pyf[KY * NYF + yb]);
        else if constexpr (KX >= 0) F = pxf[KX * NXF + xr] - pxf[KX * NXF + xl];
        else if constexpr (KY >= 0) F = pyf[KY * NYF + yt] - pyf[KY * NYF + yb];
        else F = 0.0;
        double f0 = (double)fo[i];
        if constexpr (NEQ) f0 += feo[i];
        double v;
        if (m.scheme == 0) v = (f0 - dtv * F + lam * fe[i]) * inv;
        else v = (4.0 / 3.0) * (m.a * f0 + m.b * feo[i]) - (1.0 / 3.0) * f0 - dtv * F;
        if constexpr (NEQ) v -= fe[i];
        if constexpr (S32) st_at(s.fo32 + (size_t)i * np, g, (float)v);
        else st_at(s.fo + (size_t)i * np, g, v);
    });
}

// One workgroup per tile, XCD by XCD in contiguous ranges of the row-major
// tile order.
template <int PM>
__global__ void __launch_bounds__(Shape<PM>::NTHR) k_step_cart(DevMesh m, DevCart c, DevState s, int lagged)
{
    const int x = (int)(blockIdx.x % kXcds);
    const int t = xcd_range_start((int)gridDim.x, x) + (int)(blockIdx.x / kXcds);
    cart_tile<PM>(m, c, s, lagged, t);
}

// Batched structured step: as the batched general step, the slot map gives
// each workgroup its member and tile.
template <int PM>
__global__ void __launch_bounds__(Shape<PM>::NTHR) k_step_batch_cart(BatchTable tab, int parity)
{
    const int x = (int)(blockIdx.x % kXcds);
    const int per = (int)gridDim.x / kXcds;
    const unsigned long long slot = reinterpret_cast<const unsigned long long *>(tab.tmap)[x * per + (int)(blockIdx.x / kXcds)];
    const int member = (int)(unsigned)slot, tile = (int)(unsigned)(slot >> 32);
    if (member < 0) return;
    const BatchInst &in = tab.inst[member];
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
    cart_tile<PM>(m, cg, s, in.lagged, tile);
}

}  // namespace

size_t step_cart_lds_bytes(int mode, int n_bc)
{
    const size_t head = mode == SDUGKS_FP32DEV ? Shape<SDUGKS_FP32DEV>::HEAD
                                               : (mode == SDUGKS_FP32NEQ ? Shape<SDUGKS_FP32NEQ>::HEAD
                                                                         : Shape<SDUGKS_FP64>::HEAD);
    return head + 32 * (size_t)n_bc;
}

int step_cart_threads(int mode)
{
    return mode == SDUGKS_FP32DEV ? Shape<SDUGKS_FP32DEV>::NTHR : Shape<SDUGKS_FP64>::NTHR;
}

hipError_t launch_step_cart(const DevMesh &m, const DevCart &c, const DevState &s, int lagged, int mode,
                            hipStream_t st, GraphChain *gc)
{
    const size_t lds = step_cart_lds_bytes(mode, m.n_bc);
    const dim3 grid((unsigned)(c.ntx * c.nty)), blk((unsigned)step_cart_threads(mode));
    if (mode == SDUGKS_FP32DEV) return emit(&k_step_cart<SDUGKS_FP32DEV>, grid, blk, lds, st, gc, m, c, s, lagged);
    if (mode == SDUGKS_FP32NEQ) return emit(&k_step_cart<SDUGKS_FP32NEQ>, grid, blk, lds, st, gc, m, c, s, lagged);
    return emit(&k_step_cart<SDUGKS_FP64>, grid, blk, lds, st, gc, m, c, s, lagged);
}

hipError_t launch_step_batch_cart(const BatchTable &tab, int mode, int parity, int cap_tiles, size_t lds,
                                  hipStream_t st, GraphChain *gc)
{
    const dim3 grid((unsigned)batch_grid(cap_tiles)), blk((unsigned)step_cart_threads(mode));
    if (mode == SDUGKS_FP32DEV) return emit(&k_step_batch_cart<SDUGKS_FP32DEV>, grid, blk, lds, st, gc, tab, parity);
    if (mode == SDUGKS_FP32NEQ) return emit(&k_step_batch_cart<SDUGKS_FP32NEQ>, grid, blk, lds, st, gc, tab, parity);
    return emit(&k_step_batch_cart<SDUGKS_FP64>, grid, blk, lds, st, gc, tab, parity);
}

}  // namespace sdg
