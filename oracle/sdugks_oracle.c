/*
 * sdugks_oracle.c -- plain, slow, FP64 reference of the sDUGKS step (D2Q9).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark; never by the solver library.  Compiled with
 * -O2 -ffp-contract=off (no fused multiply-add, IEEE FP64 throughout).
 *
 * Method (Zhong et al., arXiv:2007.07347, Section II, the eleven-step summary):
 *   1. macroscopic flux G^n from the face distribution at t_n (Eq. MacroFlux);
 *   2. fbar+ = (2tau-dt)/(2tau) f + dt/(2tau) feq at cell centres (Eq. fbarplus);
 *   3. fbar+ at the foot point x_f - e_i dt by the linear Taylor expansion
 *      (Eq. fbpsource) with the gradient from the unweighted linear
 *      least-squares normal equations over the adjacent cells;
 *   4. fbar(x_f, t_{n+1}) = fbar+(x_f - e_i dt, t_n) (Eq. fbar);
 *   5. face macros = moments of fbar (Eq. Macro);
 *   6. face equilibrium from the face macros;
 *   7. f(x_f, t_{n+1}) = 2tau/(2tau+dt) (fbar + dt/(2tau) feq_f) (Eq. f_t_n+1);
 *   8. mesoscopic flux F = sum over faces of l (e_i . n) f_face (Eq. MesoFlux,
 *      one midpoint per face);
 *   9. W^{n+1} = W^n - dt/V G (Eq. MacroUpdate);
 *  10. feq^{n+1} from W^{n+1};
 *  11. f^{n+1} = [f^n - dt/V F + (dt/tau) feq^{n+1}] / (1 + dt/tau) (Eq. fn+1).
 * Boundary conditions (Section III): for e_i . N < 0 (N outward) the face value
 * of fbar comes from the boundary state f_b = feq(rho_b, u_b) + (f_in - feq_in)
 * with (rho_b, u_b) = (rho_in, u_wall) on walls, (rho_inf, u_inf) on inlets,
 * (rho_in, u_in) on outlets; for e_i . N >= 0 it comes from the interior
 * reconstruction.  Symmetry faces (ghost cells mirrored about the boundary):
 * (rho_b, u_b) = (rho_in, u_in - (u_in . N) N), the mean of the inner cell and
 * its mirror image, in the same construction.  Periodic sides are glued into interior faces with a
 * translation (the ghost cells of the periodic condition carry the partner
 * cell's state, so gluing is the same thing).
 *
 * Readings where the paper is silent, ambiguous or garbled:
 *  - velocity model D2Q9 (c = 1, c_s^2 = 1/3, weights 4/9, 1/9, 1/36) with the
 *    second-order Hermite truncation of the Maxwellian (Eq. Feq prints the
 *    exponent without its factor 2; the discrete form does not need it);
 *  - isothermal: W = (rho, rho u, rho v), the energy row of Eq. Macro dropped;
 *  - tau = nu / c_s^2 = 3 nu;  dt = CFL * h_min / sqrt(2) where h_j is twice the
 *    smallest distance from the centroid of cell j to the lines of its faces;
 *  - time level of the macroscopic flux: the summary computes it first from the
 *    face distribution at t_n, while the conclusion speaks of the flux on the
 *    current step and the paper claims stability up to dt >= 10 tau.  "current"
 *    mode (the default) takes the moments of this step's face fluxes, so W stays
 *    the moment of f; "lagged" mode takes the previous step's (G^0 = 0 unless
 *    set) and is unstable on generic data once dt exceeds about 3 tau;
 *  - upwind tie (e_i . n == 0 exactly) on an interior face: the mean of the two
 *    one-sided reconstructions; on a boundary face: the interior side;
 *  - least-squares stencil: the face neighbours (periodic images translated)
 *    plus, for each boundary face of the cell, the boundary state as a point at
 *    the face midpoint with value fbar+_b (below) -- the ghost-point treatment
 *    the paper gives for its symmetry boundary, applied to every boundary.
 *    Without these points a triangle with one wall edge extrapolates to the
 *    wall from two neighbours only, and the step is linearly unstable there.
 *    A singular 2x2 system gives a zero gradient;
 *  - boundary value of fbar for incoming velocities: fbar+ of the boundary
 *    state, fbar+_b = feq(rho_b,u_b) + (2tau-dt)/(2tau) (f_in - feq_in), carried
 *    from the face midpoint to the foot point x_f - e_i dt with the gradient of
 *    the adjacent cell: fbar = fbar+_b - dt e_i . sigma_in (Eq. fbpsource about
 *    the face; without the shift the wall slips at O(dt) and Couette flow
 *    converges at first order only);
 *  - cell centre = polygon area centroid; one midpoint per face.
 *
 * Scheme ORC_DUGKS (an A/B of what the paper simplifies, not the paper's own
 * step): the original discrete unified gas kinetic scheme.  The cell carries
 * ft = f - (dt/2) Omega; fbar+ = f + (h/2) Omega with h = dt/2 is
 * (2tau-h)/(2tau+dt) ft + 3h/(2tau+dt) feq; faces are reconstructed at
 * x_f - e_i h and f_face = 2tau/(2tau+h) (fbar + h/(2tau) feq_f); the cell
 * update is ft^{n+1} = (4/3) fbar+ - (1/3) ft - dt/V F (ft+ = f + (dt/2) Omega),
 * W^{n+1} = W^n - dt/V G.  The boundary states keep their non-equilibrium
 * extrapolation, applied to ft (which carries the same f - feq up to the
 * factor of the fbar+ coefficients, so fbar+_b - fbar+_c = feq_b - feq_c
 * as in the simplified scheme).
 */
#include "sdugks_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 lattice: rest, four axis velocities, four diagonals (c = 1). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

struct orc_case {
    int nc, nf, nb, nsing;
    /* cells */
    double *area, *cx, *cy, *h;
    int *cf_ptr, *cf;           /* faces of each cell, in polygon edge order */
    double *wx, *wy;            /* least-squares weights per (cell, face slot) */
    /* faces */
    int *fo, *fn, *fbc;
    double *lnx, *lny, *xm, *ym, *tx, *ty;
    /* boundary conditions */
    int nbc;
    int *bct;
    double *bcv;                /* rho, u, v, sx, sy */
    /* parameters */
    double dt, tau, hmin, a, b, c1, lam;
    double dtr, fb_b, fb_c1;    /* face step: reconstruction time, dt/(2tau) and 2tau/(2tau+dt) of Eq. f_t_n+1 */
    int macro_mode, assembly, scheme;
    /* state */
    double *f, *W, *G;          /* [nc][9], [nc][3], [nc][3] */
    double *snapU, *snapV;
    /* scratch */
    double *fbp, *sig, *F, *Gn, *phi, *gam, *ghost;
};

void orc_feq(double rho, double ux, double uy, double *out)
{
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; i++) {
        double eu = EX[i] * ux + EY[i] * uy;
        out[i] = WT[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

static void feq_of_W(const double *W, double *out)
{
    orc_feq(W[0], W[1] / W[0], W[2] / W[0], out);
}

/* ---------------------------------------------------------------- geometry */

typedef struct { int lo, hi, cell, a, b, k; } half_edge;

static int cmp_he(const void *p, const void *q)
{
    const half_edge *x = p, *y = q;
    if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
    if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
    return x->cell < y->cell ? -1 : (x->cell > y->cell);
}

typedef struct { int lo, hi, idx; } bedge_key;

static int cmp_bk(const void *p, const void *q)
{
    const bedge_key *x = p, *y = q;
    if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
    if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
    return 0;
}

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }

orc_case *orc_create(int n_nodes, const double *xy, int nc, const int *cptr, const int *cnodes,
                     int nbe, const int *bnodes, const int *btag, int nbc, const int *bct,
                     const double *bcv, const int *bcpart, const double *prm, const int *iprm, char *err)
{
#define FAIL(...) do { snprintf(err, 256, __VA_ARGS__); goto fail; } while (0)
    orc_case *o = xcalloc(1, sizeof *o);
    half_edge *he = NULL;
    bedge_key *bk = NULL;
    int *bpair = NULL, *bcell = NULL, *bha = NULL, *bhb = NULL, *bslot = NULL;
    err[0] = 0;
    if (nc <= 0 || n_nodes <= 0) FAIL("empty mesh");
    o->nc = nc;
    o->nbc = nbc;
    o->bct = xcalloc(nbc, sizeof(int));
    o->bcv = xcalloc((size_t)nbc * 5, sizeof(double));
    memcpy(o->bct, bct, sizeof(int) * nbc);
    memcpy(o->bcv, bcv, sizeof(double) * 5 * nbc);

    /* cell areas and centroids (shoelace, relative to the first vertex) */
    o->area = xcalloc(nc, 8); o->cx = xcalloc(nc, 8); o->cy = xcalloc(nc, 8); o->h = xcalloc(nc, 8);
    int nhe = cptr[nc];
    for (int c = 0; c < nc; c++) {
        int p0 = cptr[c], m = cptr[c + 1] - p0;
        if (m < 3) FAIL("cell %d has %d nodes", c, m);
        double x0 = xy[2 * cnodes[p0]], y0 = xy[2 * cnodes[p0] + 1];
        double A = 0, Sx = 0, Sy = 0;
        for (int k = 0; k < m; k++) {
            int na = cnodes[p0 + k], nb2 = cnodes[p0 + (k + 1) % m];
            if (na < 0 || na >= n_nodes || nb2 < 0 || nb2 >= n_nodes) FAIL("cell %d: node out of range", c);
            double xa = xy[2 * na] - x0, ya = xy[2 * na + 1] - y0;
            double xb = xy[2 * nb2] - x0, yb = xy[2 * nb2 + 1] - y0;
            double cr = xa * yb - xb * ya;
            A += cr;
            Sx += (xa + xb) * cr;
            Sy += (ya + yb) * cr;
        }
        A *= 0.5;
        if (!(A > 0)) FAIL("cell %d is not counter-clockwise or has zero area", c);
        o->area[c] = A;
        o->cx[c] = x0 + Sx / (6.0 * A);
        o->cy[c] = y0 + Sy / (6.0 * A);
    }

    /* half edges, matched by unordered node pair */
    he = xcalloc(nhe, sizeof *he);
    for (int c = 0, q = 0; c < nc; c++) {
        int p0 = cptr[c], m = cptr[c + 1] - p0;
        for (int k = 0; k < m; k++, q++) {
            int na = cnodes[p0 + k], nb2 = cnodes[p0 + (k + 1) % m];
            he[q].a = na; he[q].b = nb2; he[q].cell = c; he[q].k = k;
            he[q].lo = na < nb2 ? na : nb2; he[q].hi = na < nb2 ? nb2 : na;
        }
    }
    qsort(he, nhe, sizeof *he, cmp_he);
    bk = xcalloc(nbe, sizeof *bk);
    for (int e = 0; e < nbe; e++) {
        int na = bnodes[2 * e], nb2 = bnodes[2 * e + 1];
        bk[e].lo = na < nb2 ? na : nb2; bk[e].hi = na < nb2 ? nb2 : na; bk[e].idx = e;
        if (btag[e] < 0 || btag[e] >= nbc) FAIL("boundary edge %d: tag %d out of range", e, btag[e]);
    }
    qsort(bk, nbe, sizeof *bk, cmp_bk);

    /* Count faces: interior pairs + boundary singles (periodic singles pair up). */
    int maxf = nhe;
    o->fo = xcalloc(maxf, 4); o->fn = xcalloc(maxf, 4); o->fbc = xcalloc(maxf, 4);
    o->lnx = xcalloc(maxf, 8); o->lny = xcalloc(maxf, 8); o->xm = xcalloc(maxf, 8); o->ym = xcalloc(maxf, 8);
    o->tx = xcalloc(maxf, 8); o->ty = xcalloc(maxf, 8);
    o->cf_ptr = xcalloc(nc + 1, 4); o->cf = xcalloc(nhe, 4);
    for (int c = 0; c <= nc; c++) o->cf_ptr[c] = cptr[c];
    for (int q = 0; q < nhe; q++) o->cf[q] = -1;
    /* boundary half edge bookkeeping, indexed by boundary edge id */
    bcell = xcalloc(nbe, 4); bha = xcalloc(nbe, 4); bhb = xcalloc(nbe, 4); bslot = xcalloc(nbe, 4);
    bpair = xcalloc(nbe, 4);
    for (int e = 0; e < nbe; e++) { bcell[e] = -1; bpair[e] = -1; }

    int nf = 0;
    for (int q = 0; q < nhe;) {
        int r = q + 1;
        while (r < nhe && he[r].lo == he[q].lo && he[r].hi == he[q].hi) r++;
        if (r - q > 2) FAIL("edge (%d,%d) shared by %d cells", he[q].lo, he[q].hi, r - q);
        if (r - q == 2) {
            const half_edge *ow = &he[q], *nb2 = &he[q + 1];   /* sorted: lower cell owns */
            if (ow->cell == nb2->cell) FAIL("cell %d repeats an edge", ow->cell);
            int f = nf++;
            double xa = xy[2 * ow->a], ya = xy[2 * ow->a + 1], xb = xy[2 * ow->b], yb = xy[2 * ow->b + 1];
            o->fo[f] = ow->cell; o->fn[f] = nb2->cell; o->fbc[f] = -1;
            o->lnx[f] = yb - ya; o->lny[f] = -(xb - xa);
            o->xm[f] = 0.5 * (xa + xb); o->ym[f] = 0.5 * (ya + yb);
            o->tx[f] = 0; o->ty[f] = 0;
            o->cf[cptr[ow->cell] + ow->k] = f;
            o->cf[cptr[nb2->cell] + nb2->k] = f;
        } else {
            bedge_key key = {he[q].lo, he[q].hi, 0};
            bedge_key *hit = bsearch(&key, bk, nbe, sizeof *bk, cmp_bk);
            if (!hit) FAIL("edge (%d,%d) of cell %d is on the boundary but not tagged", he[q].lo, he[q].hi, he[q].cell);
            int e = hit->idx;
            if (bcell[e] >= 0) FAIL("boundary edge %d listed twice", e);
            bcell[e] = he[q].cell; bha[e] = he[q].a; bhb[e] = he[q].b; bslot[e] = cptr[he[q].cell] + he[q].k;
        }
        q = r;
    }
    for (int e = 0; e < nbe; e++)
        if (bcell[e] < 0) FAIL("boundary edge %d is not an edge of any cell", e);

    /* plain boundary faces */
    for (int e = 0; e < nbe; e++) {
        int t = btag[e];
        if (bct[t] == ORC_PERIODIC) continue;
        if (bct[t] != ORC_WALL && bct[t] != ORC_INLET && bct[t] != ORC_OUTLET && bct[t] != ORC_SYMMETRY)
            FAIL("bc %d: unknown type %d", t, bct[t]);
        int f = nf++;
        double xa = xy[2 * bha[e]], ya = xy[2 * bha[e] + 1], xb = xy[2 * bhb[e]], yb = xy[2 * bhb[e] + 1];
        o->fo[f] = bcell[e]; o->fn[f] = -1; o->fbc[f] = t;
        o->lnx[f] = yb - ya; o->lny[f] = -(xb - xa);
        o->xm[f] = 0.5 * (xa + xb); o->ym[f] = 0.5 * (ya + yb);
        o->tx[f] = 0; o->ty[f] = 0;
        o->cf[bslot[e]] = f;
    }
    o->nb = nf;
    /* periodic sides: brute-force matching of midpoints under the translation */
    for (int e = 0; e < nbe; e++) {
        int t = btag[e];
        if (bct[t] != ORC_PERIODIC || bpair[e] >= 0) continue;
        int pt = bcpart[t];
        if (pt < 0 || pt >= nbc || bct[pt] != ORC_PERIODIC || bcpart[pt] != t) FAIL("bc %d: bad periodic partner", t);
        double sx = bcv[5 * t + 3], sy = bcv[5 * t + 4];
        if (fabs(sx + bcv[5 * pt + 3]) > 1e-12 * (1 + fabs(sx)) || fabs(sy + bcv[5 * pt + 4]) > 1e-12 * (1 + fabs(sy)))
            FAIL("bc %d: partner shift is not the opposite translation", t);
        double mx = 0.5 * (xy[2 * bha[e]] + xy[2 * bhb[e]]) + sx;
        double my = 0.5 * (xy[2 * bha[e] + 1] + xy[2 * bhb[e] + 1]) + sy;
        double scale = 1.0 + fabs(mx) + fabs(my);
        int best = -1;
        for (int g = 0; g < nbe; g++) {
            if (btag[g] != pt || bpair[g] >= 0 || g == e) continue;
            double gx = 0.5 * (xy[2 * bha[g]] + xy[2 * bhb[g]]);
            double gy = 0.5 * (xy[2 * bha[g] + 1] + xy[2 * bhb[g] + 1]);
            if (fabs(gx - mx) <= 1e-9 * scale && fabs(gy - my) <= 1e-9 * scale) { best = g; break; }
        }
        if (best < 0) FAIL("periodic edge %d has no partner", e);
        bpair[e] = best; bpair[best] = e;
        int eo = e, en = best;
        if (bcell[en] < bcell[eo]) { eo = best; en = e; }
        int f = nf++;
        int to = btag[eo];
        double xa = xy[2 * bha[eo]], ya = xy[2 * bha[eo] + 1], xb = xy[2 * bhb[eo]], yb = xy[2 * bhb[eo] + 1];
        o->fo[f] = bcell[eo]; o->fn[f] = bcell[en]; o->fbc[f] = to;
        o->lnx[f] = yb - ya; o->lny[f] = -(xb - xa);
        o->xm[f] = 0.5 * (xa + xb); o->ym[f] = 0.5 * (ya + yb);
        o->tx[f] = bcv[5 * to + 3]; o->ty[f] = bcv[5 * to + 4];
        o->cf[bslot[eo]] = f;
        o->cf[bslot[en]] = f;
    }
    o->nf = nf;
    o->nb = 0;
    for (int f = 0; f < nf; f++) o->nb += (o->fn[f] < 0);

    /* h_j = 2 * min distance from the centroid to the lines of the cell's faces */
    for (int c = 0; c < nc; c++) {
        double hm = INFINITY;
        for (int q = o->cf_ptr[c]; q < o->cf_ptr[c + 1]; q++) {
            int f = o->cf[q];
            double px, py;
            if (o->fo[f] == c) { px = o->xm[f]; py = o->ym[f]; }
            else { px = o->xm[f] + o->tx[f]; py = o->ym[f] + o->ty[f]; }
            double l = sqrt(o->lnx[f] * o->lnx[f] + o->lny[f] * o->lny[f]);
            double d = fabs((px - o->cx[c]) * o->lnx[f] + (py - o->cy[c]) * o->lny[f]) / l;
            if (2.0 * d < hm) hm = 2.0 * d;
        }
        o->h[c] = hm;
    }
    o->hmin = INFINITY;
    for (int c = 0; c < nc; c++) if (o->h[c] < o->hmin) o->hmin = o->h[c];

    /* least-squares weights w_jk = A_j^{-1} d_jk (assembled mode) */
    o->wx = xcalloc(nhe, 8); o->wy = xcalloc(nhe, 8);
    o->nsing = 0;
    for (int c = 0; c < nc; c++) {
        double sxx = 0, sxy = 0, syy = 0;
        double dxs[16], dys[16];
        int m = o->cf_ptr[c + 1] - o->cf_ptr[c];
        if (m > 16) FAIL("cell %d has more than 16 faces", c);
        for (int q = o->cf_ptr[c], s = 0; q < o->cf_ptr[c + 1]; q++, s++) {
            int f = o->cf[q];
            double kx, ky;
            if (o->fn[f] < 0) { kx = o->xm[f]; ky = o->ym[f]; }        /* boundary point */
            else {
                int k = (o->fo[f] == c) ? o->fn[f] : o->fo[f];
                kx = o->cx[k]; ky = o->cy[k];
                if (o->fo[f] == c) { kx -= o->tx[f]; ky -= o->ty[f]; }
                else { kx += o->tx[f]; ky += o->ty[f]; }
            }
            dxs[s] = kx - o->cx[c]; dys[s] = ky - o->cy[c];
            sxx += dxs[s] * dxs[s]; sxy += dxs[s] * dys[s]; syy += dys[s] * dys[s];
        }
        double det = sxx * syy - sxy * sxy;
        int sing = !(fabs(det) > 1e-12 * (sxx + syy) * (sxx + syy));
        o->nsing += sing;
        for (int q = o->cf_ptr[c], s = 0; q < o->cf_ptr[c + 1]; q++, s++) {
            o->wx[q] = sing ? 0.0 : (syy * dxs[s] - sxy * dys[s]) / det;
            o->wy[q] = sing ? 0.0 : (sxx * dys[s] - sxy * dxs[s]) / det;
        }
    }

    /* parameters */
    double nu = prm[0], tau = prm[1], cfl = prm[2], dt = prm[3];
    if (tau <= 0) tau = 3.0 * nu;
    if (!(tau > 0)) FAIL("need nu > 0 or tau > 0");
    if (dt <= 0) dt = cfl * o->hmin / sqrt(2.0);
    if (!(dt > 0)) FAIL("need dt > 0 or cfl > 0");
    o->tau = tau; o->dt = dt;
    o->a = (2.0 * tau - dt) / (2.0 * tau);
    o->b = dt / (2.0 * tau);
    o->c1 = 2.0 * tau / (2.0 * tau + dt);
    o->lam = dt / tau;
    o->dtr = dt; o->fb_b = o->b; o->fb_c1 = o->c1;
    o->macro_mode = iprm[0];
    o->assembly = iprm[1];
    o->scheme = iprm[2];
    if (o->scheme == ORC_DUGKS) {
        /* the original scheme: faces at half a step, h = dt/2, and the cell
         * variable ft = f - (dt/2) Omega; fbar+ = f + (h/2) Omega written in ft */
        double h = 0.5 * dt;
        if (o->macro_mode != ORC_CURRENT) FAIL("the original scheme has no lagged macroscopic flux");
        o->a = (2.0 * tau - h) / (2.0 * tau + dt);
        o->b = 3.0 * h / (2.0 * tau + dt);
        o->dtr = h; o->fb_b = h / (2.0 * tau); o->fb_c1 = 2.0 * tau / (2.0 * tau + h);
    } else if (o->scheme != ORC_SDUGKS) FAIL("unknown scheme %d", o->scheme);

    /* state: uniform equilibrium (rho0, u0, v0), G = 0 */
    o->f = xcalloc((size_t)nc * 9, 8); o->W = xcalloc((size_t)nc * 3, 8); o->G = xcalloc((size_t)nc * 3, 8);
    o->snapU = xcalloc(nc, 8); o->snapV = xcalloc(nc, 8);
    double fe[9];
    orc_feq(prm[4], prm[5], prm[6], fe);
    for (int c = 0; c < nc; c++) {
        for (int i = 0; i < 9; i++) o->f[9 * c + i] = fe[i];
        o->W[3 * c] = prm[4]; o->W[3 * c + 1] = prm[4] * prm[5]; o->W[3 * c + 2] = prm[4] * prm[6];
        o->snapU[c] = prm[5]; o->snapV[c] = prm[6];
    }
    o->fbp = xcalloc((size_t)nc * 9, 8); o->sig = xcalloc((size_t)nc * 18, 8);
    o->F = xcalloc((size_t)nc * 9, 8); o->Gn = xcalloc((size_t)nc * 3, 8);
    o->phi = xcalloc((size_t)nf * 9, 8); o->gam = xcalloc((size_t)nf * 3, 8);
    o->ghost = xcalloc((size_t)nf * 9, 8);

    free(he); free(bk); free(bpair); free(bcell); free(bha); free(bhb); free(bslot);
    return o;
fail:
    free(he); free(bk); free(bpair); free(bcell); free(bha); free(bhb); free(bslot);
    orc_free(o);
    return NULL;
#undef FAIL
}

void orc_free(orc_case *o)
{
    if (!o) return;
    void *p[] = {o->area, o->cx, o->cy, o->h, o->cf_ptr, o->cf, o->wx, o->wy, o->fo, o->fn, o->fbc,
                 o->lnx, o->lny, o->xm, o->ym, o->tx, o->ty, o->bct, o->bcv, o->f, o->W, o->G,
                 o->snapU, o->snapV, o->fbp, o->sig, o->F, o->Gn, o->phi, o->gam, o->ghost};
    for (size_t k = 0; k < sizeof p / sizeof p[0]; k++) free(p[k]);
    free(o);
}

void orc_info(const orc_case *o, double *d, int *iv)
{
    d[0] = o->dt; d[1] = o->tau; d[2] = o->hmin; d[3] = o->a; d[4] = o->b; d[5] = o->c1; d[6] = o->lam;
    iv[0] = o->nc; iv[1] = o->nf; iv[2] = o->nb; iv[3] = o->nsing;
}

void orc_geometry(const orc_case *o, double *area, double *cx, double *cy, double *h)
{
    for (int c = 0; c < o->nc; c++) { area[c] = o->area[c]; cx[c] = o->cx[c]; cy[c] = o->cy[c]; h[c] = o->h[c]; }
}

void orc_faces(const orc_case *o, int *ow, int *nb, int *bcid, double *lnx, double *lny, double *xm, double *ym,
               double *tx, double *ty)
{
    for (int f = 0; f < o->nf; f++) {
        ow[f] = o->fo[f]; nb[f] = o->fn[f]; bcid[f] = o->fbc[f];
        lnx[f] = o->lnx[f]; lny[f] = o->lny[f]; xm[f] = o->xm[f]; ym[f] = o->ym[f]; tx[f] = o->tx[f]; ty[f] = o->ty[f];
    }
}

/* the original scheme keeps ft = f - (dt/2) Omega = (1 + dt/2tau) f - (dt/2tau) feq(W) per cell */
static void to_tilde(const orc_case *o, const double *f, const double *W, double *ft, int inverse)
{
    double k = o->dt / (2.0 * o->tau), fe[9];
    for (int c = 0; c < o->nc; c++) {
        feq_of_W(&W[3 * c], fe);
        for (int i = 0; i < 9; i++)
            ft[9 * c + i] = inverse ? (f[9 * c + i] + k * fe[i]) / (1.0 + k) : (1.0 + k) * f[9 * c + i] - k * fe[i];
    }
}

void orc_set_state(orc_case *o, const double *f, const double *W, const double *G)
{
    if (o->scheme == ORC_DUGKS) to_tilde(o, f, W, o->f, 0);
    else memcpy(o->f, f, sizeof(double) * 9 * o->nc);
    memcpy(o->W, W, sizeof(double) * 3 * o->nc);
    memcpy(o->G, G, sizeof(double) * 3 * o->nc);
    for (int c = 0; c < o->nc; c++) { o->snapU[c] = W[3 * c + 1] / W[3 * c]; o->snapV[c] = W[3 * c + 2] / W[3 * c]; }
}

void orc_get_state(const orc_case *o, double *f, double *W, double *G)
{
    if (f) {
        if (o->scheme == ORC_DUGKS) to_tilde(o, o->f, o->W, f, 1);
        else memcpy(f, o->f, sizeof(double) * 9 * o->nc);
    }
    if (W) memcpy(W, o->W, sizeof(double) * 3 * o->nc);
    if (G) memcpy(G, o->G, sizeof(double) * 3 * o->nc);
}

/* ------------------------------------------------------------ the scheme */

/* neighbour of cell c across face f, and the position of its image seen from c */
static int other_side(const orc_case *o, int f, int c, double *kx, double *ky)
{
    int k;
    if (o->fo[f] == c) { k = o->fn[f]; *kx = o->cx[k] - o->tx[f]; *ky = o->cy[k] - o->ty[f]; }
    else { k = o->fo[f]; *kx = o->cx[k] + o->tx[f]; *ky = o->cy[k] + o->ty[f]; }
    return k;
}

/* Stencil value seen by cell c across slot q: the neighbour's value (its
 * periodic image carries the same value) or, on a boundary face, the value of
 * the boundary state at the face midpoint. */
static double stencil_value(const orc_case *o, const double *fld, const double *bval, int stride, int i, int c,
                            int f, double *kx, double *ky)
{
    if (o->fn[f] < 0) { *kx = o->xm[f]; *ky = o->ym[f]; return bval[stride * f + i]; }
    int k = other_side(o, f, c, kx, ky);
    return fld[stride * k + i];
}

/* gradient of fld[.][i] at cell c from the normal equations, Cramer's rule */
static void lsq_cramer(const orc_case *o, const double *fld, const double *bval, int stride, int i, int c,
                       double *gx, double *gy)
{
    double sxx = 0, sxy = 0, syy = 0, bx = 0, by = 0;
    for (int q = o->cf_ptr[c]; q < o->cf_ptr[c + 1]; q++) {
        double kx, ky;
        double vk = stencil_value(o, fld, bval, stride, i, c, o->cf[q], &kx, &ky);
        double dx = kx - o->cx[c], dy = ky - o->cy[c];
        double df = vk - fld[stride * c + i];
        sxx += dx * dx; sxy += dx * dy; syy += dy * dy;
        bx += dx * df; by += dy * df;
    }
    double det = sxx * syy - sxy * sxy;
    if (!(fabs(det) > 1e-12 * (sxx + syy) * (sxx + syy))) { *gx = 0; *gy = 0; return; }
    *gx = (syy * bx - sxy * by) / det;
    *gy = (sxx * by - sxy * bx) / det;
}

/* gradient from the precomputed weights: sum_k w_jk (fld_k - fld_j) */
static void lsq_weights(const orc_case *o, const double *fld, const double *bval, int stride, int i, int c,
                        double *gx, double *gy)
{
    double sx = 0, sy = 0;
    for (int q = o->cf_ptr[c]; q < o->cf_ptr[c + 1]; q++) {
        double kx, ky;
        double df = stencil_value(o, fld, bval, stride, i, c, o->cf[q], &kx, &ky) - fld[stride * c + i];
        sx += o->wx[q] * df;
        sy += o->wy[q] * df;
    }
    *gx = sx; *gy = sy;
}

void orc_lsq_gradient(const orc_case *o, const double *field, const double *bfield, double *grad, int mode)
{
    for (int c = 0; c < o->nc; c++) {
        if (mode == 0) lsq_weights(o, field, bfield, 1, 0, c, &grad[2 * c], &grad[2 * c + 1]);
        else lsq_cramer(o, field, bfield, 1, 0, c, &grad[2 * c], &grad[2 * c + 1]);
    }
}

/* steps 2 and 3: fbar+ at every centre, the boundary states, the gradients */
static void prepare(orc_case *o, int cramer)
{
    #pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; c++) {
        double fe[9];
        feq_of_W(&o->W[3 * c], fe);
        for (int i = 0; i < 9; i++) o->fbp[9 * c + i] = o->a * o->f[9 * c + i] + o->b * fe[i];
    }
    #pragma omp parallel for schedule(static)
    for (int f = 0; f < o->nf; f++) {
        if (o->fn[f] >= 0) continue;
        int c = o->fo[f], t = o->fbc[f];
        double rho_in = o->W[3 * c], u_in = o->W[3 * c + 1] / rho_in, v_in = o->W[3 * c + 2] / rho_in;
        double rb, ub, vb;
        if (o->bct[t] == ORC_WALL) { rb = rho_in; ub = o->bcv[5 * t + 1]; vb = o->bcv[5 * t + 2]; }
        else if (o->bct[t] == ORC_INLET) { rb = o->bcv[5 * t]; ub = o->bcv[5 * t + 1]; vb = o->bcv[5 * t + 2]; }
        else if (o->bct[t] == ORC_SYMMETRY) {
            /* the mean of the inner cell and its mirror image about the face:
             * same density, normal velocity removed, tangential velocity kept */
            double l = sqrt(o->lnx[f] * o->lnx[f] + o->lny[f] * o->lny[f]);
            double nx = o->lnx[f] / l, ny = o->lny[f] / l, un = u_in * nx + v_in * ny;
            rb = rho_in; ub = u_in - un * nx; vb = v_in - un * ny;
        }
        else { rb = rho_in; ub = u_in; vb = v_in; }
        double feb[9], fein[9];
        orc_feq(rb, ub, vb, feb);
        orc_feq(rho_in, u_in, v_in, fein);
        for (int i = 0; i < 9; i++) {
            double fb = feb[i] + (o->f[9 * c + i] - fein[i]);           /* boundary state at t_n */
            o->ghost[9 * f + i] = o->a * fb + o->b * feb[i];            /* its fbar+ */
        }
    }
    #pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; c++)
        for (int i = 0; i < 9; i++) {
            if (cramer) lsq_cramer(o, o->fbp, o->ghost, 9, i, c, &o->sig[18 * c + 2 * i], &o->sig[18 * c + 2 * i + 1]);
            else lsq_weights(o, o->fbp, o->ghost, 9, i, c, &o->sig[18 * c + 2 * i], &o->sig[18 * c + 2 * i + 1]);
        }
}

/* fbar+ of cell c reconstructed at the foot point (px,py) - e_i dt, where
 * (px,py) is the face midpoint in c's frame */
static double reconstruct(const orc_case *o, int c, int i, double px, double py)
{
    double rx = px - EX[i] * o->dtr - o->cx[c];
    double ry = py - EY[i] * o->dtr - o->cy[c];
    return o->fbp[9 * c + i] + rx * o->sig[18 * c + 2 * i] + ry * o->sig[18 * c + 2 * i + 1];
}

/* steps 3-8 for one face: fills fbar, fface, phi (9 each) and gamma (3) */
static void face_flux(const orc_case *o, int f, double *fbar, double *fface, double *phi, double *gam)
{
    int co = o->fo[f], cn = o->fn[f];
    for (int i = 0; i < 9; i++) {
        double s = EX[i] * o->lnx[f] + EY[i] * o->lny[f];
        if (cn < 0) {
            /* incoming: the boundary state's fbar+ carried to the foot point x_f - e_i dt
             * with the adjacent cell's gradient (Eq. fbpsource about the face) */
            fbar[i] = (s >= 0) ? reconstruct(o, co, i, o->xm[f], o->ym[f])
                               : o->ghost[9 * f + i] - o->dtr * (EX[i] * o->sig[18 * co + 2 * i]
                                                                + EY[i] * o->sig[18 * co + 2 * i + 1]);
        } else {
            double ro = reconstruct(o, co, i, o->xm[f], o->ym[f]);
            double rn = reconstruct(o, cn, i, o->xm[f] + o->tx[f], o->ym[f] + o->ty[f]);
            fbar[i] = s > 0 ? ro : (s < 0 ? rn : 0.5 * (ro + rn));
        }
    }
    double rho = 0, mx = 0, my = 0;
    for (int i = 0; i < 9; i++) { rho += fbar[i]; mx += EX[i] * fbar[i]; my += EY[i] * fbar[i]; }
    double fe[9];
    orc_feq(rho, mx / rho, my / rho, fe);
    gam[0] = gam[1] = gam[2] = 0;
    for (int i = 0; i < 9; i++) {
        double s = EX[i] * o->lnx[f] + EY[i] * o->lny[f];
        fface[i] = o->fb_c1 * (fbar[i] + o->fb_b * fe[i]);
        phi[i] = s * fface[i];
        gam[0] += phi[i]; gam[1] += EX[i] * phi[i]; gam[2] += EY[i] * phi[i];
    }
}

void orc_face_states(const orc_case *o0, double *fbar, double *fface, double *phi)
{
    orc_case *o = (orc_case *)o0;   /* scratch arrays only */
    prepare(o, o->assembly == ORC_BRUTE);
    double g[3];
    for (int f = 0; f < o->nf; f++) face_flux(o, f, &fbar[9 * f], &fface[9 * f], &phi[9 * f], g);
}

static void one_step(orc_case *o)
{
    int brute = (o->assembly == ORC_BRUTE);
    prepare(o, brute);
    #pragma omp parallel for schedule(static)
    for (int f = 0; f < o->nf; f++) {
        double fb[9], ff[9];
        face_flux(o, f, fb, ff, &o->phi[9 * f], &o->gam[3 * f]);
    }
    if (brute) {
        /* scatter in face order */
        memset(o->F, 0, sizeof(double) * 9 * o->nc);
        memset(o->Gn, 0, sizeof(double) * 3 * o->nc);
        for (int f = 0; f < o->nf; f++) {
            int co = o->fo[f], cn = o->fn[f];
            for (int i = 0; i < 9; i++) o->F[9 * co + i] += o->phi[9 * f + i];
            for (int m = 0; m < 3; m++) o->Gn[3 * co + m] += o->gam[3 * f + m];
            if (cn >= 0) {
                for (int i = 0; i < 9; i++) o->F[9 * cn + i] -= o->phi[9 * f + i];
                for (int m = 0; m < 3; m++) o->Gn[3 * cn + m] -= o->gam[3 * f + m];
            }
        }
    } else {
        /* gather in each cell's polygon edge order */
        #pragma omp parallel for schedule(static)
        for (int c = 0; c < o->nc; c++) {
            double Fc[9] = {0}, Gc[3] = {0};
            for (int q = o->cf_ptr[c]; q < o->cf_ptr[c + 1]; q++) {
                int f = o->cf[q];
                double sg = (o->fo[f] == c) ? 1.0 : -1.0;
                if (o->fo[f] == c && o->fn[f] == c) sg = 0.0;   /* a cell glued to itself */
                for (int i = 0; i < 9; i++) Fc[i] += sg * o->phi[9 * f + i];
                for (int m = 0; m < 3; m++) Gc[m] += sg * o->gam[3 * f + m];
            }
            memcpy(&o->F[9 * c], Fc, sizeof Fc);
            memcpy(&o->Gn[3 * c], Gc, sizeof Gc);
        }
    }
    /* steps 9-11 */
    #pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; c++) {
        double fe[9];
        double k = o->dt / o->area[c];
        const double *Gs = (o->macro_mode == ORC_LAGGED) ? &o->G[3 * c] : &o->Gn[3 * c];
        for (int m = 0; m < 3; m++) o->W[3 * c + m] = o->W[3 * c + m] - k * Gs[m];
        if (o->scheme == ORC_DUGKS) {
            /* ft^{n+1} = ft+ - dt/V F with ft+ = f + (dt/2) Omega = (4/3) fbar+ - (1/3) ft */
            for (int i = 0; i < 9; i++)
                o->f[9 * c + i] = (4.0 / 3.0) * o->fbp[9 * c + i] - (1.0 / 3.0) * o->f[9 * c + i] - k * o->F[9 * c + i];
            for (int m = 0; m < 3; m++) o->G[3 * c + m] = o->Gn[3 * c + m];
            continue;
        }
        feq_of_W(&o->W[3 * c], fe);
        for (int i = 0; i < 9; i++)
            o->f[9 * c + i] = (o->f[9 * c + i] - k * o->F[9 * c + i] + o->lam * fe[i]) / (1.0 + o->lam);
        for (int m = 0; m < 3; m++) o->G[3 * c + m] = o->Gn[3 * c + m];
    }
}

/* Threads of the per-cell and per-face loops (OpenMP when compiled with it):
 * every iteration computes the same operations on the same operands whatever
 * thread runs it, so the results do not depend on the thread count.  The
 * scatter of the brute-force assembly stays serial, in face order. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_step(orc_case *o, int n)
{
    for (int s = 0; s < n; s++) one_step(o);
}

double orc_residual(orc_case *o)
{
    double num = 0, den = 0;
    for (int c = 0; c < o->nc; c++) {
        double U = o->W[3 * c + 1] / o->W[3 * c], V = o->W[3 * c + 2] / o->W[3 * c];
        double dU = U - o->snapU[c], dV = V - o->snapV[c];
        num += dU * dU + dV * dV;
        den += o->snapU[c] * o->snapU[c] + o->snapV[c] * o->snapV[c];
        o->snapU[c] = U; o->snapV[c] = V;
    }
    return den > 0 ? sqrt(num) / sqrt(den) : INFINITY;
}

double orc_mass(const orc_case *o)
{
    double m = 0;
    for (int c = 0; c < o->nc; c++) m += o->area[c] * o->W[3 * c];
    return m;
}
