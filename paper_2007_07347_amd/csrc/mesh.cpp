// Host mesh builder: geometry of Section II of Zhong et al. (arXiv:2007.07347)
// -- control volumes V_j and their centres, face normals and midpoints (one
// quadrature point per face for the contour integrals of Eqs. MacroFlux and
// MesoFlux), the linear least-squares normal matrix of the LLSR gradient, the
// periodic gluing of Section III -- laid out for the device.
//
// Layout decisions (not the paper's): every cell carries D face slots
// (structure of arrays, padded), each slot holding the face seen from the
// cell.  Both cells of an interior face store bit-identical copies of the
// face data (mirrored), so the two evaluate the face flux from identical
// operands and the flux leaves one cell exactly as it enters the other.
// Boundary states enter the least-squares system as points at the face
// midpoints.  Cells are renumbered for locality: into compact tiles by
// recursive coordinate bisection for the fused one-kernel step (each tile
// with its two halo rings and a local adjacency table), or by reverse
// Cuthill-McKee for the two-kernel step.
#include "mesh.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <deque>
#include <unordered_map>

namespace sdg {

namespace {

struct HalfEdge {
    int32_t cell, slot, a, b;
};

inline uint64_t edge_key(int32_t p, int32_t q)
{
    uint32_t lo = (uint32_t)std::min(p, q), hi = (uint32_t)std::max(p, q);
    return ((uint64_t)lo << 32) | hi;
}

// Reverse Cuthill-McKee on the cell adjacency graph (CSR adj).
std::vector<int32_t> rcm_order(int32_t n, const std::vector<int32_t> &ptr, const std::vector<int32_t> &adj)
{
    std::vector<int32_t> deg(n), order;
    order.reserve(n);
    for (int32_t c = 0; c < n; c++) deg[c] = ptr[c + 1] - ptr[c];
    std::vector<char> seen(n, 0);
    std::vector<int32_t> level(n, -1);
    auto bfs_last = [&](int32_t s) {   // farthest node of a BFS from s (pseudo-peripheral search)
        std::deque<int32_t> q{s};
        std::vector<int32_t> touched{s};
        level[s] = 0;
        int32_t last = s;
        while (!q.empty()) {
            int32_t c = q.front();
            q.pop_front();
            last = c;
            for (int32_t e = ptr[c]; e < ptr[c + 1]; e++) {
                int32_t k = adj[e];
                if (level[k] < 0) { level[k] = level[c] + 1; q.push_back(k); touched.push_back(k); }
            }
        }
        int32_t depth = level[last];
        for (int32_t t : touched) level[t] = -1;
        return std::make_pair(last, depth);
    };
    for (int32_t start = 0; start < n; start++) {
        if (seen[start]) continue;
        // pseudo-peripheral start: repeat BFS from the farthest node while the depth grows
        int32_t s = start;
        auto r = bfs_last(s);
        for (int it = 0; it < 4; it++) {
            auto r2 = bfs_last(r.first);
            if (r2.second <= r.second) break;
            s = r.first;
            r = r2;
        }
        std::deque<int32_t> q{s};
        seen[s] = 1;
        std::vector<int32_t> nb;
        while (!q.empty()) {
            int32_t c = q.front();
            q.pop_front();
            order.push_back(c);
            nb.clear();
            for (int32_t e = ptr[c]; e < ptr[c + 1]; e++)
                if (!seen[adj[e]]) { nb.push_back(adj[e]); seen[adj[e]] = 1; }
            std::sort(nb.begin(), nb.end(), [&](int32_t x, int32_t y) { return deg[x] != deg[y] ? deg[x] < deg[y] : x < y; });
            for (int32_t k : nb) q.push_back(k);
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// Recursive coordinate bisection of ids[lo, hi) into k parts of near-equal
// size, split across the longer side of the bounding box of the centroids.
void rcb(std::vector<int32_t> &ids, size_t lo, size_t hi, int64_t k, const std::vector<double> &cx,
         const std::vector<double> &cy, std::vector<std::pair<size_t, size_t>> &parts)
{
    if (k <= 1 || hi - lo <= 1) { parts.emplace_back(lo, hi); return; }
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (size_t j = lo; j < hi; j++) {
        x0 = std::min(x0, cx[ids[j]]); x1 = std::max(x1, cx[ids[j]]);
        y0 = std::min(y0, cy[ids[j]]); y1 = std::max(y1, cy[ids[j]]);
    }
    const bool by_x = (x1 - x0) >= (y1 - y0);
    const int64_t kl = k / 2;
    const size_t n = hi - lo, nl = (size_t)((int64_t)n * kl / k);
    auto key = [&](int32_t c) { return by_x ? std::make_tuple(cx[c], cy[c], c) : std::make_tuple(cy[c], cx[c], c); };
    std::nth_element(ids.begin() + lo, ids.begin() + lo + nl, ids.begin() + hi,
                     [&](int32_t a, int32_t b) { return key(a) < key(b); });
    rcb(ids, lo, lo + nl, kl, cx, cy, parts);
    rcb(ids, lo + nl, hi, k - kl, cx, cy, parts);
}

// Tiles of the fused step over the internal order (tile-major already).
// Every per-tile table is padded to the largest tile so tile t's block starts
// at t times a fixed pitch.  False if the two views of some face are not exact
// mirrors (they always are: both are built from one face record below).
bool build_tiles(MeshBuild &out, std::vector<std::pair<size_t, size_t>> parts)
{
    const int32_t nc = out.nc, D = out.D;
    out.n_tiles = (int32_t)parts.size();
    // Tiles with a boundary face do more work (boundary states in phases 2 and
    // 3).  Each XCD takes a contiguous range of tiles (xcd_range_start) and
    // starts them in order, so within each range those tiles go first.
    {
        auto at_boundary = [&](const std::pair<size_t, size_t> &p) {
            for (size_t c = p.first; c < p.second; c++)
                for (int32_t s = 0; s < D; s++) {
                    const int32_t nb = out.nbr[(size_t)s * nc + c];
                    if (nb < 0 && nb != kEmptySlot) return true;
                }
            return false;
        };
        const int32_t n = (int32_t)parts.size();
        for (int32_t x = 0; x < kXcds; x++)
            std::stable_partition(parts.begin() + xcd_range_start(n, x), parts.begin() + xcd_range_start(n, x + 1),
                                  at_boundary);
    }
    out.tile_hdr.assign((size_t)out.n_tiles * 8, 0);
    std::vector<std::vector<int32_t>> locals(out.n_tiles);
    std::vector<int32_t> stamp(nc, -1), h1, h2;
    out.nl_max = out.na_max = 0;
    // pass 1: halo rings of every tile
    for (int32_t t = 0; t < out.n_tiles; t++) {
        const int32_t g0 = (int32_t)parts[t].first, nt = (int32_t)(parts[t].second - parts[t].first);
        for (int32_t k = 0; k < nt; k++) stamp[g0 + k] = t;
        h1.clear(); h2.clear();
        // cells stamped t are already local; a ring collects the unstamped
        // face neighbours of a set of cells and stamps them
        auto ring = [&](int32_t c, std::vector<int32_t> &dst) {
            for (int32_t s = 0; s < D; s++) {
                const int32_t nb = out.nbr[(size_t)s * nc + c];
                if (nb >= 0 && stamp[nb] != t) { stamp[nb] = t; dst.push_back(nb); }
            }
        };
        // each ring in rows (centroid y, then x), like the tile's own cells
        auto rows = [&](std::vector<int32_t> &v) {
            std::sort(v.begin(), v.end(), [&](int32_t a, int32_t b) {
                return std::make_tuple(out.cy[a], out.cx[a], a) < std::make_tuple(out.cy[b], out.cx[b], b);
            });
        };
        for (int32_t k = 0; k < nt; k++) ring(g0 + k, h1);
        rows(h1);
        for (int32_t c : h1) ring(c, h2);
        rows(h2);
        std::vector<int32_t> &L = locals[t];
        for (int32_t k = 0; k < nt; k++) L.push_back(g0 + k);
        L.insert(L.end(), h1.begin(), h1.end());
        L.insert(L.end(), h2.begin(), h2.end());
        int32_t *h = &out.tile_hdr[(size_t)t * 8];
        h[0] = g0; h[1] = nt; h[2] = (int32_t)h1.size(); h[3] = (int32_t)h2.size();
        out.nl_max = std::max(out.nl_max, (int32_t)L.size());
        out.na_max = std::max(out.na_max, nt + h[2]);
    }
    // pass 2: padded tables
    const size_t PL = out.nl_max, PA = out.na_max;
    out.lgid.assign((size_t)out.n_tiles * PL, 0);
    out.ladj.assign((size_t)out.n_tiles * D * PA, -1);
    out.lw.assign((size_t)out.n_tiles * D * PA * 2, 0.0);
    std::vector<int32_t> loc(nc, -1);
    for (int32_t t = 0; t < out.n_tiles; t++) {
        const std::vector<int32_t> &L = locals[t];
        const int32_t na = out.tile_hdr[(size_t)t * 8 + 1] + out.tile_hdr[(size_t)t * 8 + 2];
        for (size_t k = 0; k < L.size(); k++) { loc[L[k]] = (int32_t)k; out.lgid[t * PL + k] = L[k]; }
        for (int32_t k = 0; k < na; k++) {
            const int32_t c = L[k];
            for (int32_t s = 0; s < D; s++) {
                const size_t q = (size_t)s * nc + c;
                const int32_t nb = out.nbr[q];
                int16_t v;
                if (nb == kEmptySlot) v = -1;
                else if (nb < 0) v = (int16_t)(-2 - out.bf_tag[-1 - nb]);
                else v = (int16_t)loc[nb];
                out.ladj[((size_t)t * D + s) * PA + k] = v;
                out.lw[(((size_t)t * D + s) * PA + k) * 2 + 0] = out.wx[q];
                out.lw[(((size_t)t * D + s) * PA + k) * 2 + 1] = out.wy[q];
            }
        }
        for (int32_t c : L) loc[c] = -1;
    }
    // pass 3: one face record per face of the tile cells, and each slot's code
    int32_t n_face_ids = 0;
    for (int32_t f : out.fid) n_face_ids = std::max(n_face_ids, f + 1);
    std::vector<int32_t> rec_of(n_face_ids, -1);
    std::vector<std::vector<double>> recs(out.n_tiles);
    std::vector<std::vector<int16_t>> codes(out.n_tiles);
    out.nt_max = out.nf_max = 0;
    for (int32_t t = 0; t < out.n_tiles; t++) out.nt_max = std::max(out.nt_max, out.tile_hdr[(size_t)t * 8 + 1]);
    const size_t PT = out.nt_max;
    for (int32_t t = 0; t < out.n_tiles; t++) {
        const int32_t g0 = out.tile_hdr[(size_t)t * 8], nt = out.tile_hdr[(size_t)t * 8 + 1];
        std::vector<double> &R = recs[t];
        codes[t].assign((size_t)D * PT, -1);
        std::vector<int32_t> used;
        for (int32_t k = 0; k < nt; k++)
            for (int32_t s = 0; s < D; s++) {
                const size_t q = (size_t)s * nc + g0 + k;
                const int32_t f = out.fid[q];
                if (f < 0) continue;
                const double v[6] = {out.lnx[q], out.lny[q], out.rsx[q], out.rsy[q], out.rox[q], out.roy[q]};
                int32_t code;
                if (rec_of[f] < 0) {
                    rec_of[f] = (int32_t)(R.size() / 6);
                    used.push_back(f);
                    R.insert(R.end(), v, v + 6);
                    code = 2 * rec_of[f];
                } else {
                    const double *r = &R[(size_t)rec_of[f] * 6];
                    if (!(v[0] == -r[0] && v[1] == -r[1] && v[2] == r[4] && v[3] == r[5] && v[4] == r[2] && v[5] == r[3]))
                        return false;
                    code = 2 * rec_of[f] + 1;
                }
                codes[t][(size_t)s * PT + k] = (int16_t)code;
            }
        for (int32_t f : used) rec_of[f] = -1;
        out.nf_max = std::max(out.nf_max, (int32_t)(R.size() / 6));
    }
    const size_t PF = std::max<int32_t>(1, out.nf_max);
    out.lfc.assign((size_t)out.n_tiles * D * PT, -1);
    out.frec.assign((size_t)out.n_tiles * 3 * PF * 2, 0.0);
    for (int32_t t = 0; t < out.n_tiles; t++) {
        std::copy(codes[t].begin(), codes[t].end(), out.lfc.begin() + (size_t)t * D * PT);
        const std::vector<double> &R = recs[t];
        for (size_t r = 0; r < R.size() / 6; r++)
            for (size_t k = 0; k < 3; k++)
                for (size_t e = 0; e < 2; e++)
                    out.frec[(((size_t)t * 3 + k) * PF + r) * 2 + e] = R[r * 6 + 2 * k + e];
    }
    return true;
}

}  // namespace

int build_mesh(const sdugks_mesh *m, const sdugks_bc *bc, int32_t n_bc, const sdugks_params *prm,
               MeshBuild &out, std::string &err)
{
    char buf[256];
#define BAD(...) do { std::snprintf(buf, sizeof buf, __VA_ARGS__); err = buf; return SDUGKS_EINVAL; } while (0)
    if (!m || !prm) BAD("null mesh or params");
    const int32_t nc = m->n_cells, nn = m->n_nodes;
    if (nc <= 0 || nn <= 0 || !m->node_xy || !m->cell_ptr || !m->cell_nodes) BAD("empty mesh");
    if (m->n_bedges < 0 || (m->n_bedges > 0 && (!m->bedge_nodes || !m->bedge_tag))) BAD("bad boundary edge arrays");
    if (n_bc < 0 || (n_bc > 0 && !bc)) BAD("bad boundary-condition table");
    if (m->cell_ptr[0] != 0) BAD("cell_ptr[0] must be 0");
    const double *xy = m->node_xy;

    // ---- per-cell geometry in caller order: fan triangulation about the vertex mean
    std::vector<double> area(nc), cx(nc), cy(nc);
    int32_t D = 0;
    for (int32_t c = 0; c < nc; c++) {
        int32_t p0 = m->cell_ptr[c], deg = m->cell_ptr[c + 1] - p0;
        if (deg < 3 || deg > 8) BAD("cell %d has %d nodes (3..8 supported)", c, deg);
        D = std::max(D, deg);
        double mx = 0, my = 0;
        for (int32_t k = 0; k < deg; k++) {
            int32_t v = m->cell_nodes[p0 + k];
            if (v < 0 || v >= nn) BAD("cell %d references node %d", c, v);
            mx += xy[2 * v];
            my += xy[2 * v + 1];
        }
        mx /= deg;
        my /= deg;
        double A = 0, Sx = 0, Sy = 0;
        for (int32_t k = 0; k < deg; k++) {
            int32_t v = m->cell_nodes[p0 + k], w = m->cell_nodes[p0 + (k + 1) % deg];
            double ax = xy[2 * v] - mx, ay = xy[2 * v + 1] - my, bx = xy[2 * w] - mx, by = xy[2 * w + 1] - my;
            double t = 0.5 * (ax * by - ay * bx);      // signed area of (mean, v, w)
            A += t;
            Sx += t * (ax + bx) / 3.0;
            Sy += t * (ay + by) / 3.0;
        }
        if (!(A > 0)) BAD("cell %d is not counter-clockwise (signed area %g)", c, A);
        area[c] = A;
        cx[c] = mx + Sx / A;
        cy[c] = my + Sy / A;
    }

    // ---- match edges
    std::unordered_map<uint64_t, int32_t> first;   // edge -> half edge index awaiting its twin
    std::vector<HalfEdge> he;
    he.reserve(m->cell_ptr[nc]);
    struct Face { int32_t o, n, os, ns, tag; double lnx, lny, xm, ym, tx, ty; };
    std::vector<Face> faces;
    faces.reserve(m->cell_ptr[nc]);
    std::vector<int32_t> slot_face((size_t)nc * D, -1);   // caller order [c*D + s]
    auto make_face = [&](const HalfEdge &o, int32_t n, int32_t ns, int32_t tag, double tx, double ty) {
        Face f;
        f.o = o.cell; f.os = o.slot; f.n = n; f.ns = ns; f.tag = tag;
        double xa = xy[2 * o.a], ya = xy[2 * o.a + 1], xb = xy[2 * o.b], yb = xy[2 * o.b + 1];
        f.lnx = yb - ya;
        f.lny = xa - xb;
        f.xm = 0.5 * (xa + xb);
        f.ym = 0.5 * (ya + yb);
        f.tx = tx; f.ty = ty;
        faces.push_back(f);
        int32_t id = (int32_t)faces.size() - 1;
        slot_face[(size_t)o.cell * D + o.slot] = id;
        if (n >= 0) slot_face[(size_t)n * D + ns] = id;
    };
    for (int32_t c = 0; c < nc; c++) {
        int32_t p0 = m->cell_ptr[c], deg = m->cell_ptr[c + 1] - p0;
        for (int32_t k = 0; k < deg; k++) {
            HalfEdge h{c, k, m->cell_nodes[p0 + k], m->cell_nodes[p0 + (k + 1) % deg]};
            if (h.a == h.b) BAD("cell %d has a repeated node", c);
            uint64_t key = edge_key(h.a, h.b);
            auto it = first.find(key);
            if (it == first.end()) { first.emplace(key, (int32_t)he.size()); he.push_back(h); continue; }
            int32_t j = it->second;
            if (j < 0) BAD("edge (%d,%d) is shared by more than two cells", h.a, h.b);
            const HalfEdge &g = he[j];
            if (g.a != h.b || g.b != h.a) BAD("cells %d and %d traverse edge (%d,%d) the same way", g.cell, c, h.a, h.b);
            if (g.cell == c) BAD("cell %d uses edge (%d,%d) twice", c, h.a, h.b);
            make_face(g, c, k, -1, 0.0, 0.0);
            it->second = -1;
        }
    }
    // boundary edges: each must close an unmatched half edge
    struct BEdge { int32_t he, tag; double mx, my; };
    std::vector<BEdge> bed(m->n_bedges);
    std::unordered_map<uint64_t, int32_t> bseen;
    for (int32_t e = 0; e < m->n_bedges; e++) {
        int32_t p = m->bedge_nodes[2 * e], q = m->bedge_nodes[2 * e + 1], t = m->bedge_tag[e];
        if (t < 0 || t >= n_bc) BAD("boundary edge %d has tag %d (table has %d)", e, t, n_bc);
        uint64_t key = edge_key(p, q);
        auto it = first.find(key);
        if (it == first.end() || it->second < 0) BAD("boundary edge %d (%d,%d) is not a free cell edge", e, p, q);
        if (!bseen.emplace(key, e).second) BAD("boundary edge %d listed twice", e);
        const HalfEdge &h = he[it->second];
        bed[e] = {it->second, t, 0.5 * (xy[2 * h.a] + xy[2 * h.b]), 0.5 * (xy[2 * h.a + 1] + xy[2 * h.b + 1])};
    }
    if ((size_t)m->n_bedges != bseen.size()) BAD("duplicate boundary edges");
    for (auto &kv : first)
        if (kv.second >= 0 && !bseen.count(kv.first)) BAD("cell %d has an untagged free edge", he[kv.second].cell);
    for (int32_t t = 0; t < n_bc; t++) {
        int32_t ty = bc[t].type;
        if (ty < SDUGKS_BC_WALL || ty > SDUGKS_BC_SYMMETRY) BAD("bc %d: unknown type %d", t, ty);
        if (ty == SDUGKS_BC_INLET && !(bc[t].rho > 0)) BAD("bc %d: inlet density must be positive", t);
        if (ty == SDUGKS_BC_PERIODIC) {
            int32_t p = bc[t].partner;
            if (p < 0 || p >= n_bc || p == t || bc[p].type != SDUGKS_BC_PERIODIC || bc[p].partner != t) BAD("bc %d: bad periodic partner", t);
            double tol = 1e-12 * (1.0 + std::fabs(bc[t].shift_x) + std::fabs(bc[t].shift_y));
            if (std::fabs(bc[t].shift_x + bc[p].shift_x) > tol || std::fabs(bc[t].shift_y + bc[p].shift_y) > tol)
                BAD("bc %d: partner shift is not the opposite translation", t);
        }
    }
    // symmetry sides: one straight line per tag; its unit outward normal
    std::vector<double> sym_nx(n_bc, 0.0), sym_ny(n_bc, 0.0);
    {
        double ext = 0;
        for (int32_t v = 0; v < nn; v++) ext = std::max(ext, std::fabs(xy[2 * v]) + std::fabs(xy[2 * v + 1]));
        std::vector<double> sx(n_bc, 0.0), sy(n_bc, 0.0);
        for (int32_t e = 0; e < m->n_bedges; e++) {
            const int32_t t = bed[e].tag;
            if (bc[t].type != SDUGKS_BC_SYMMETRY) continue;
            const HalfEdge &h = he[bed[e].he];
            sx[t] += xy[2 * h.b + 1] - xy[2 * h.a + 1];
            sy[t] += xy[2 * h.a] - xy[2 * h.b];
        }
        for (int32_t t = 0; t < n_bc; t++) {
            if (bc[t].type != SDUGKS_BC_SYMMETRY) continue;
            const double l = std::sqrt(sx[t] * sx[t] + sy[t] * sy[t]);
            if (!(l > 0)) BAD("bc %d: symmetry side has no edges", t);
            sym_nx[t] = sx[t] / l;
            sym_ny[t] = sy[t] / l;
        }
        std::vector<double> off(n_bc, NAN);
        for (int32_t e = 0; e < m->n_bedges; e++) {
            const int32_t t = bed[e].tag;
            if (bc[t].type != SDUGKS_BC_SYMMETRY) continue;
            const HalfEdge &h = he[bed[e].he];
            const double ex = xy[2 * h.b + 1] - xy[2 * h.a + 1], ey = xy[2 * h.a] - xy[2 * h.b];
            const double le = std::sqrt(ex * ex + ey * ey);
            const double d = sym_nx[t] * bed[e].mx + sym_ny[t] * bed[e].my;
            if (std::isnan(off[t])) off[t] = d;
            if (std::fabs(ex / le - sym_nx[t]) > 1e-9 || std::fabs(ey / le - sym_ny[t]) > 1e-9 ||
                std::fabs(d - off[t]) > 1e-9 * (1.0 + ext))
                BAD("bc %d: symmetry edges must lie on one straight line (edge %d)", t, e);
        }
    }
    // plain boundary faces
    std::vector<int32_t> bf_cell_c, bf_tag_c;   // caller order of cells
    for (int32_t e = 0; e < m->n_bedges; e++) {
        if (bc[bed[e].tag].type == SDUGKS_BC_PERIODIC) continue;
        make_face(he[bed[e].he], -1, -1, bed[e].tag, 0.0, 0.0);
    }
    // periodic gluing: sort each partner side by midpoint, look targets up with a tolerance
    double ext = 0;
    for (int32_t v = 0; v < nn; v++) ext = std::max(ext, std::fabs(xy[2 * v]) + std::fabs(xy[2 * v + 1]));
    const double tol = 1e-9 * (1.0 + ext);
    std::vector<char> glued(m->n_bedges, 0);
    for (int32_t t = 0; t < n_bc; t++) {
        if (bc[t].type != SDUGKS_BC_PERIODIC || bc[t].partner < t) continue;
        int32_t p = bc[t].partner;
        std::vector<int32_t> side_p;
        for (int32_t e = 0; e < m->n_bedges; e++) if (bed[e].tag == p) side_p.push_back(e);
        std::sort(side_p.begin(), side_p.end(), [&](int32_t x, int32_t y) { return bed[x].mx < bed[y].mx; });
        for (int32_t e = 0; e < m->n_bedges; e++) {
            if (bed[e].tag != t) continue;
            double gx = bed[e].mx + bc[t].shift_x, gy = bed[e].my + bc[t].shift_y;
            auto lo = std::lower_bound(side_p.begin(), side_p.end(), gx - tol,
                                       [&](int32_t x, double v) { return bed[x].mx < v; });
            int32_t hit = -1;
            for (auto it = lo; it != side_p.end() && bed[*it].mx <= gx + tol; ++it)
                if (!glued[*it] && std::fabs(bed[*it].my - gy) <= tol) { hit = *it; break; }
            if (hit < 0) BAD("periodic edge %d (tag %d) has no partner on tag %d", e, t, p);
            glued[e] = glued[hit] = 1;
            const HalfEdge &ht = he[bed[e].he], &hp = he[bed[hit].he];
            // the edge of tag t owns the face; its neighbour sits at x - shift_t seen from it
            make_face(ht, hp.cell, hp.slot, t, bc[t].shift_x, bc[t].shift_y);
        }
    }
    for (int32_t e = 0; e < m->n_bedges; e++)
        if (bc[bed[e].tag].type == SDUGKS_BC_PERIODIC && !glued[e]) BAD("periodic edge %d left unglued", e);

    // ---- structured (tensor-product) quad meshes: the cells are the
    // rectangles of two sorted coordinate arrays, every plain boundary face on
    // one of the four sides, periodic gluing (if any) between opposite sides
    // of the same row or column
    bool cart = false;
    std::vector<int32_t> cart_cell;   // (i + nx j) -> caller cell
    std::vector<double> cxs, cys;
    int32_t cnx = 0, cny = 0, cper_x = 0, cper_y = 0;
    std::vector<int32_t> cside;
    if (prm->structured < 0 || prm->structured > 2) BAD("structured must be 0, 1 or 2");
    if (prm->structured != 1 && (prm->structured == 2 || prm->tile_cells == 0) && D == 4 && n_bc <= kMaxTileBcs) {
        auto detect = [&]() -> bool {
            for (int32_t c = 0; c < nc; c++)
                if (m->cell_ptr[c + 1] - m->cell_ptr[c] != 4) return false;
            for (int32_t v = 0; v < nn; v++) { cxs.push_back(xy[2 * v]); cys.push_back(xy[2 * v + 1]); }
            std::sort(cxs.begin(), cxs.end());
            cxs.erase(std::unique(cxs.begin(), cxs.end()), cxs.end());
            std::sort(cys.begin(), cys.end());
            cys.erase(std::unique(cys.begin(), cys.end()), cys.end());
            cnx = (int32_t)cxs.size() - 1;
            cny = (int32_t)cys.size() - 1;
            if (cnx < 2 || cny < 2 || (int64_t)cnx * cny != nc) return false;
            // the step addresses each velocity's row of f with 32-bit byte offsets
            if ((int64_t)nc > (1LL << 29) - 4096) return false;
            cart_cell.assign((size_t)nc, -1);
            std::vector<int32_t> ci(nc), cj(nc);
            for (int32_t c = 0; c < nc; c++) {
                int32_t ii[4], jj[4], k0 = 0;
                for (int32_t k = 0; k < 4; k++) {
                    const int32_t v = m->cell_nodes[m->cell_ptr[c] + k];
                    ii[k] = (int32_t)(std::lower_bound(cxs.begin(), cxs.end(), xy[2 * v]) - cxs.begin());
                    jj[k] = (int32_t)(std::lower_bound(cys.begin(), cys.end(), xy[2 * v + 1]) - cys.begin());
                    if (ii[k] < ii[k0] || (ii[k] == ii[k0] && jj[k] < jj[k0])) k0 = k;
                }
                const int32_t i = ii[k0], j = jj[k0];
                const int32_t di[4] = {0, 1, 1, 0}, dj[4] = {0, 0, 1, 1};   // counter-clockwise from the lower left
                for (int32_t k = 0; k < 4; k++)
                    if (ii[(k0 + k) % 4] != i + di[k] || jj[(k0 + k) % 4] != j + dj[k]) return false;
                if (i >= cnx || j >= cny || cart_cell[i + (size_t)cnx * j] >= 0) return false;
                cart_cell[i + (size_t)cnx * j] = c;
                ci[c] = i;
                cj[c] = j;
            }
            cside.assign(2 * (size_t)cnx + 2 * (size_t)cny, -2);
            int32_t glued_x = 0, glued_y = 0;
            for (const Face &f : faces) {
                const int32_t i = ci[f.o], j = cj[f.o];
                if (f.n < 0) {
                    if (f.lny == 0 && f.lnx < 0 && i == 0) cside[2 * cnx + j] = f.tag;
                    else if (f.lny == 0 && f.lnx > 0 && i == cnx - 1) cside[2 * cnx + cny + j] = f.tag;
                    else if (f.lnx == 0 && f.lny < 0 && j == 0) cside[i] = f.tag;
                    else if (f.lnx == 0 && f.lny > 0 && j == cny - 1) cside[cnx + i] = f.tag;
                    else return false;
                    continue;
                }
                const int32_t in = ci[f.n], jn = cj[f.n];
                if (f.tx == 0 && f.ty == 0) {
                    if (std::abs(in - i) + std::abs(jn - j) != 1) return false;
                    continue;
                }
                // glued across a periodic pair of sides
                if (j == jn && f.ty == 0 && ((i == 0 && in == cnx - 1) || (i == cnx - 1 && in == 0))) glued_x++;
                else if (i == in && f.tx == 0 && ((j == 0 && jn == cny - 1) || (j == cny - 1 && jn == 0))) glued_y++;
                else return false;
            }
            if (glued_x && glued_x != cny) return false;
            if (glued_y && glued_y != cnx) return false;
            cper_x = glued_x > 0;
            cper_y = glued_y > 0;
            for (int32_t k = 0; k < 2 * cnx + 2 * cny; k++) {
                const bool periodic = k < 2 * cnx ? cper_y : cper_x;
                if (periodic) {
                    if (cside[k] != -2) return false;
                    cside[k] = -1;
                } else if (cside[k] < 0) {
                    return false;
                }
            }
            return true;
        };
        cart = detect();
    }
    if (!cart && prm->structured == 2)
        BAD("the structured step needs a tensor-product quad mesh (cells the rectangles of two coordinate arrays, "
            "at least two along each axis, at most 2^29 - 4096 cells) and at most %d boundary-condition entries",
            kMaxTileBcs);

    // ---- cell order: tile-major (fused step) or reverse Cuthill-McKee
    std::vector<int32_t> perm(nc), iperm(nc);
    const bool tiled = prm->tile_cells >= 0 && D <= 4 && n_bc <= kMaxTileBcs;
    const int32_t B = prm->block_threads > 0 ? prm->block_threads : kDefaultBlock;
    int32_t T = prm->tile_cells > 0 ? std::min(prm->tile_cells, B / 4) : B / 4;
    if (tiled && T < 4) BAD("tile_cells must be at least 4 (or 0 / -1)");
    std::vector<std::pair<size_t, size_t>> parts;
    if (cart) {
        for (int32_t j = 0; j < cny; j++)
            for (int32_t i = 0; i < cnx; i++) perm[cart_index(i, j, cnx, cny)] = cart_cell[i + (size_t)cnx * j];
    } else if (tiled) {
        for (int32_t c = 0; c < nc; c++) perm[c] = c;
        rcb(perm, 0, nc, ((int64_t)nc + T - 1) / T, cx, cy, parts);
        // rows of cells inside each tile (by centroid y, then x): the local
        // indices of face neighbours then differ by near-constant offsets, so
        // a wave's LDS gathers of neighbour data spread over the banks
        for (const auto &p : parts)
            std::sort(perm.begin() + p.first, perm.begin() + p.second, [&](int32_t a, int32_t b) {
                return std::make_tuple(cy[a], cx[a], a) < std::make_tuple(cy[b], cx[b], b);
            });
    } else if (prm->reorder) {
        std::vector<int32_t> ptr(nc + 1, 0), adj;
        for (const Face &f : faces)
            if (f.n >= 0 && f.n != f.o) { ptr[f.o + 1]++; ptr[f.n + 1]++; }
        for (int32_t c = 0; c < nc; c++) ptr[c + 1] += ptr[c];
        adj.resize(ptr[nc]);
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (const Face &f : faces)
            if (f.n >= 0 && f.n != f.o) { adj[fill[f.o]++] = f.n; adj[fill[f.n]++] = f.o; }
        perm = rcm_order(nc, ptr, adj);
    } else {
        for (int32_t c = 0; c < nc; c++) perm[c] = c;
    }
    for (int32_t k = 0; k < nc; k++) iperm[perm[k]] = k;

    // ---- slot arrays in internal order
    out.nc = nc; out.D = D; out.n_faces = (int32_t)faces.size();
    out.perm = perm; out.iperm = iperm;
    out.area.resize(nc); out.cx.resize(nc); out.cy.resize(nc); out.ainv.assign(3 * (size_t)nc, 0.0);
    size_t ns = (size_t)D * nc;
    out.nbr.assign(ns, kEmptySlot);
    out.lnx.assign(ns, 0); out.lny.assign(ns, 0); out.rsx.assign(ns, 0); out.rsy.assign(ns, 0);
    out.rox.assign(ns, 0); out.roy.assign(ns, 0);
    out.wx.assign(ns, 0); out.wy.assign(ns, 0);
    out.fid.assign(ns, -1);
    out.bf_cell.clear(); out.bf_tag.clear();
    std::vector<int32_t> bf_index(faces.size(), -1);
    for (size_t fi = 0; fi < faces.size(); fi++)
        if (faces[fi].n < 0) {
            bf_index[fi] = (int32_t)out.bf_cell.size();
            out.bf_cell.push_back(iperm[faces[fi].o]);
            out.bf_tag.push_back(faces[fi].tag);
        }
    out.n_bfaces = (int32_t)out.bf_cell.size();
    double hmin = INFINITY;
    out.n_singular = 0;
    for (int32_t k = 0; k < nc; k++) {
        int32_t c = perm[k];
        out.area[k] = area[c]; out.cx[k] = cx[c]; out.cy[k] = cy[c];
        int32_t deg = m->cell_ptr[c + 1] - m->cell_ptr[c];
        double sxx = 0, sxy = 0, syy = 0, hc = INFINITY;
        for (int32_t s = 0; s < deg; s++) {
            const Face &f = faces[slot_face[(size_t)c * D + s]];
            size_t q = (size_t)s * nc + k;
            out.fid[q] = slot_face[(size_t)c * D + s];
            bool own = (f.o == c && f.os == s);
            // face data from the owner's side: midpoint, its image on the neighbour side
            double ro_x = f.xm - cx[f.o], ro_y = f.ym - cy[f.o];
            double rn_x = 0, rn_y = 0;
            if (f.n >= 0) { rn_x = (f.xm + f.tx) - cx[f.n]; rn_y = (f.ym + f.ty) - cy[f.n]; }
            double dx, dy;
            if (f.n < 0) {
                out.nbr[q] = -(1 + bf_index[slot_face[(size_t)c * D + s]]);
                out.lnx[q] = f.lnx; out.lny[q] = f.lny;
                out.rsx[q] = ro_x; out.rsy[q] = ro_y;
                dx = ro_x; dy = ro_y;                         // boundary point at the face midpoint
            } else if (own) {
                out.nbr[q] = iperm[f.n];
                out.lnx[q] = f.lnx; out.lny[q] = f.lny;
                out.rsx[q] = ro_x; out.rsy[q] = ro_y; out.rox[q] = rn_x; out.roy[q] = rn_y;
                dx = ro_x - rn_x; dy = ro_y - rn_y;
            } else {
                out.nbr[q] = iperm[f.o];
                out.lnx[q] = -f.lnx; out.lny[q] = -f.lny;
                out.rsx[q] = rn_x; out.rsy[q] = rn_y; out.rox[q] = ro_x; out.roy[q] = ro_y;
                dx = rn_x - ro_x; dy = rn_y - ro_y;
            }
            sxx += dx * dx; sxy += dx * dy; syy += dy * dy;
            double l = std::sqrt(out.lnx[q] * out.lnx[q] + out.lny[q] * out.lny[q]);
            double dist = std::fabs(out.rsx[q] * out.lnx[q] + out.rsy[q] * out.lny[q]) / l;
            hc = std::min(hc, 2.0 * dist);
        }
        hmin = std::min(hmin, hc);
        double det = sxx * syy - sxy * sxy, tr = sxx + syy;
        if (std::fabs(det) > 1e-12 * tr * tr) {
            const double i0 = syy / det, i1 = -sxy / det, i2 = sxx / det;
            out.ainv[k] = i0;
            out.ainv[(size_t)nc + k] = i1;
            out.ainv[2 * (size_t)nc + k] = i2;
            // least-squares weights A^-1 d of every stencil point
            for (int32_t s = 0; s < deg; s++) {
                const size_t q = (size_t)s * nc + k;
                const double dx = out.nbr[q] < 0 ? out.rsx[q] : out.rsx[q] - out.rox[q];
                const double dy = out.nbr[q] < 0 ? out.rsy[q] : out.rsy[q] - out.roy[q];
                out.wx[q] = i0 * dx + i1 * dy;
                out.wy[q] = i1 * dx + i2 * dy;
            }
        } else {
            out.n_singular++;
        }
    }
    out.bcs.resize(n_bc);
    for (int32_t t = 0; t < n_bc; t++) {
        out.bcs[t] = {bc[t].type, bc[t].rho, bc[t].u, bc[t].v};
        if (bc[t].type == SDUGKS_BC_SYMMETRY) { out.bcs[t].u = sym_nx[t]; out.bcs[t].v = sym_ny[t]; }   // the line's normal
    }
    out.tile_T = 0; out.n_tiles = 0;
    out.tile_hdr.clear(); out.lgid.clear(); out.ladj.clear(); out.lfc.clear(); out.frec.clear(); out.lw.clear();
    out.cart = cart;
    if (cart) {
        // per column / row: width, face offsets, least-squares weights of the
        // two stencil points along that axis (the neighbour centre, its
        // periodic image, or the wall face midpoint), inverse width
        auto axis = [](const std::vector<double> &xs, int32_t n, bool periodic, std::vector<double> &v) {
            v.assign((size_t)n * kCartVals, 0.0);
            const double L = xs[n] - xs[0];
            auto ctr = [&](int32_t i) { return 0.5 * (xs[i] + xs[i + 1]); };
            for (int32_t i = 0; i < n; i++) {
                const double c = ctr(i), w = xs[i + 1] - xs[i];
                const double hl = xs[i] - c, hr = xs[i + 1] - c;
                double dm, dp;   // distances to the left and right stencil points
                if (i > 0) dm = c - ctr(i - 1);
                else dm = periodic ? c - (ctr(n - 1) - L) : -hl;
                if (i < n - 1) dp = ctr(i + 1) - c;
                else dp = periodic ? (ctr(0) + L) - c : hr;
                const double den = dp * dp + dm * dm;
                double *r = &v[(size_t)i * kCartVals];
                r[0] = w; r[1] = hl; r[2] = hr; r[3] = -dm / den; r[4] = dp / den; r[5] = 1.0 / w;
            }
        };
        axis(cxs, cnx, cper_x, out.col);
        axis(cys, cny, cper_y, out.row);
        out.nx = cnx; out.ny = cny; out.per_x = cper_x; out.per_y = cper_y;
        const int32_t rows = cart_tile_rows(prm->precision);
        out.ntx = (cnx + kCartTX - 1) / kCartTX;
        out.nty = (cny + rows - 1) / rows;
        out.side = cside;
        out.n_tiles = out.ntx * out.nty;
        out.tile_T = kCartTX * rows;
    } else if (tiled) {
        if (!build_tiles(out, parts)) BAD("internal: the two views of a face are not exact mirrors");
        if (tile_lds_bytes(out.nl_max, out.na_max, out.nt_max, n_bc) > kTileLdsLimit || out.nl_max > B) {
            // one thread per local cell and LDS for all of them: bisect into smaller tiles
            if (T <= 4) BAD("mesh too irregular for the fused step's tiles");
            sdugks_params smaller = *prm;
            smaller.tile_cells = T / 2;
            return build_mesh(m, bc, n_bc, &smaller, out, err);
        }
        out.tile_T = T;
    }

    // ---- time scales
    out.h_min = hmin;
    double tau = prm->tau > 0 ? prm->tau : prm->nu / (1.0 / 3.0);
    if (!(tau > 0) || !std::isfinite(tau)) BAD("need tau > 0 or nu > 0");
    double dt = prm->dt > 0 ? prm->dt : prm->cfl * hmin / std::sqrt(2.0);
    if (!(dt > 0) || !std::isfinite(dt)) BAD("need dt > 0 or cfl > 0");
    out.tau = tau;
    out.dt = dt;
    return SDUGKS_OK;
#undef BAD
}

}  // namespace sdg
