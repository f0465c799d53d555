// C ABI of libsdugks.so: handles, device memory, step driver, reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sdugks.h"
#include "device.h"
#include "mesh.h"

using namespace sdg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail(SDUGKS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
// Steps per replay of the long step graphs, in pairs (each pair returns every
// instance to its buffer index).
constexpr int64_t kGraphPairs = 16;
constexpr int kBatchGraphs = 5;   // 2^(kBatchGraphs - 1) = kGraphPairs
static_assert((int64_t)1 << (kBatchGraphs - 1) == kGraphPairs, "batch graph lengths");

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Byte layout of one handle's device memory.  Everything is carved from one
// block: per-cell rows are pitched to np = nc rounded up to 64, plus 64 when
// that is a multiple of 2048 (rows a large power of two apart start at the
// same offset modulo the memory channel interleave, so the nine rows of one
// cell would be read from the same channels).
struct Layout {
    size_t np = 0;
    size_t off_f[2]{}, off_W[2]{}, off_G[2]{}, off_fbp = 0, off_sg = 0, off_snap = 0;
    size_t off_nbr = 0, off_geo = 0, off_ainv = 0, off_dtv = 0, off_area = 0, off_bft = 0, off_bcs = 0;
    size_t off_part = 0, off_out = 0, total = 0;
    size_t off_thdr = 0, off_lgid = 0, off_ladj = 0, off_lfc = 0, off_frec = 0, off_lw = 0;
    size_t off_bq_hdr = 0, off_bq_nb = 0, off_bq_w = 0, off_bq_geo = 0, off_bq_out = 0, off_bq_sum = 0;
    size_t off_ccol = 0, off_crow = 0, off_cside = 0;
};

// What the three step forms need: the two-kernel step keeps fbar+ and its
// gradient in memory with per-cell neighbour lists, inverse normal matrices
// and per-slot face geometry; the fused step keeps its tile tables (with the
// face records) instead; the deviation form stores f, the face records and
// the least-squares weights in FP32.
Layout make_layout(const MeshBuild &mb, int precision)
{
    Layout L;
    L.np = ((size_t)mb.nc + 63) / 64 * 64;
    if (L.np % 2048 == 0) L.np += 64;
    const bool dev = precision != SDUGKS_FP64;
    const size_t row = L.np * sizeof(double), rowf = L.np * (dev ? sizeof(float) : sizeof(double));
    size_t p = 0;
    auto take = [&](size_t bytes) { size_t o = p; p += align_up(bytes); return o; };
    for (int k = 0; k < 2; k++) {
        L.off_f[k] = take(9 * rowf);
        L.off_W[k] = take(3 * row);
        L.off_G[k] = take(3 * row);
    }
    if (mb.cart) {
        // structured step: one record per column and per row, the side tags
        L.off_ccol = take(mb.col.size() * sizeof(double));
        L.off_crow = take(mb.row.size() * sizeof(double));
        L.off_cside = take(mb.side.size() * sizeof(int32_t));
    } else if (mb.n_tiles > 0) {
        // fused step: fbar+ and its gradient live in LDS only
        L.off_thdr = take(mb.tile_hdr.size() * sizeof(int32_t));
        L.off_lgid = take(mb.lgid.size() * sizeof(int32_t));
        L.off_ladj = take(mb.ladj.size() * sizeof(int16_t));
        L.off_lfc = take(mb.lfc.size() * sizeof(int16_t));
        L.off_frec = take(mb.frec.size() * (dev ? sizeof(float) : sizeof(double)));
        L.off_lw = take(mb.lw.size() * (dev ? sizeof(float) : sizeof(double)));
    } else {
        L.off_fbp = take(9 * row);
        L.off_sg = take(18 * row);
        L.off_nbr = take((size_t)mb.D * L.np * sizeof(int32_t));
        L.off_ainv = take(3 * row);
        L.off_bft = take(std::max<size_t>(1, mb.n_bfaces) * sizeof(int32_t));
    }
    L.off_snap = take(2 * row);
    if (mb.n_tiles == 0) L.off_geo = take(6 * (size_t)mb.D * row);   // two-kernel step: FP64 only
    L.off_dtv = take(row);
    L.off_area = take(row);
    L.off_bcs = take(std::max<size_t>(1, mb.bcs.size()) * sizeof(DevBC));
    L.off_part = take(4 * kReduceBlocks * sizeof(double));
    L.off_out = take(4 * sizeof(double));
    // boundary-face table of the flux diagnostic
    const size_t nbq = std::max<int32_t>(1, mb.n_bfaces);
    L.off_bq_hdr = take(nbq * sizeof(int4));
    L.off_bq_nb = take(nbq * mb.D * sizeof(int32_t));
    L.off_bq_w = take(nbq * mb.D * sizeof(double2));
    L.off_bq_geo = take(nbq * 2 * sizeof(double2));
    L.off_bq_out = take(nbq * 4 * sizeof(double));
    L.off_bq_sum = take(4 * sizeof(double));
    L.total = p;
    return L;
}

}  // namespace

struct sdugks_s {
    MeshBuild mb;
    Layout L;
    int device = 0;
    hipStream_t stream = nullptr;
    char *base = nullptr;
    bool own = false;
    int cur = 0;                 // index of the current (input) state buffers
    int64_t step = 0;
    bool diverged = false;
    int precision = SDUGKS_FP64, macro = SDUGKS_MACRO_CURRENT, scheme = SDUGKS_SCHEME_SIMPLIFIED;
    double rho0 = 1.0;
    int block = 256;
    DevMesh dm{};
    DevTiles dt{};
    DevCart dc{};
    DevBnd bq{};
    double *host4 = nullptr;     // pinned, 4 doubles
    // steps replayed from graphs: [buffer index at launch][one pair,
    // kGraphPairs pairs], launched on `stream`
    hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};

    template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(base + off); }
    // buffers of a step that reads buffer index c and writes c ^ 1
    DevState state_at(int c) const
    {
        DevState s;
        s.f = at<double>(L.off_f[c]); s.W = at<double>(L.off_W[c]); s.G = at<double>(L.off_G[c]);
        s.fo = at<double>(L.off_f[c ^ 1]); s.Wo = at<double>(L.off_W[c ^ 1]); s.Go = at<double>(L.off_G[c ^ 1]);
        s.f32 = at<float>(L.off_f[c]);
        s.fo32 = at<float>(L.off_f[c ^ 1]);
        return s;
    }
    DevState state() const { return state_at(cur); }
    bool dev32() const { return precision != SDUGKS_FP64; }   // f stored as the FP32 deviation
    DevScratch scratch() const { return {at<double>(L.off_fbp), at<double>(L.off_sg)}; }
};

// Members of one launch: same face class (three or four slots) and precision mode.
struct BatchGroup {
    int D = 4, mode = 0, block = 64;
    bool cart = false;
    size_t lds = 0;
    int n_inst = 0, n_tiles = 0, cap_inst = 0, cap_tiles = 0;
    BatchInst *d_inst = nullptr;      // device table, capacity cap_inst
    int2 *d_tmap = nullptr;           // batch_grid(cap_tiles) slots: member, local tile
    std::vector<int> members;         // indices into the batch's member list
};

struct sdugks_batch_s {
    std::vector<sdugks_t *> members;
    std::vector<BatchGroup> groups;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t ev = nullptr;
    // graphs of 1, 2, 4, .. kGraphPairs pairs of steps: a step count is
    // replayed as runs of the longest plus one graph per set bit of the rest
    hipGraph_t graph[kBatchGraphs] = {};
    hipGraphExec_t exec[kBatchGraphs] = {};
    int device = 0;
    std::vector<int> cur_at_fill;     // members' buffer indices when the tables were filled
    bool failed = false;              // a table rebuild failed: no members until set_members succeeds
    bool fail_next_build = false;     // failure injection for tests
    // batched residual: job table (pinned host copy and device) and results
    int cap_jobs = 0;
    ReduceJob *h_jobs = nullptr, *d_jobs = nullptr;
    double *h_out = nullptr, *d_out = nullptr;
};

namespace {

int check_prm(const sdugks_params *prm)
{
    if (!prm) return fail(SDUGKS_EINVAL, "null params");
    if (prm->precision != SDUGKS_FP64 && prm->precision != SDUGKS_FP32DEV && prm->precision != SDUGKS_FP32NEQ)
        return fail(SDUGKS_EINVAL, "precision must be SDUGKS_FP64, SDUGKS_FP32DEV or SDUGKS_FP32NEQ");
    if (prm->macro_flux != SDUGKS_MACRO_CURRENT && prm->macro_flux != SDUGKS_MACRO_LAGGED)
        return fail(SDUGKS_EINVAL, "macro_flux must be SDUGKS_MACRO_CURRENT or SDUGKS_MACRO_LAGGED");
    if (prm->scheme != SDUGKS_SCHEME_SIMPLIFIED && prm->scheme != SDUGKS_SCHEME_ORIGINAL)
        return fail(SDUGKS_EINVAL, "scheme must be SDUGKS_SCHEME_SIMPLIFIED or SDUGKS_SCHEME_ORIGINAL");
    if (prm->scheme == SDUGKS_SCHEME_ORIGINAL && prm->macro_flux != SDUGKS_MACRO_CURRENT)
        return fail(SDUGKS_EINVAL, "the original scheme has no lagged macroscopic flux");
    if (!(prm->rho0 > 0)) return fail(SDUGKS_EINVAL, "rho0 must be positive");
    if (prm->block_threads != 0 && prm->block_threads != 64 && prm->block_threads != 128 && prm->block_threads != 256)
        return fail(SDUGKS_EINVAL, "block_threads must be 0, 64, 128 or 256");
    return SDUGKS_OK;
}

int build(const sdugks_mesh *mesh, const sdugks_bc *bc, int32_t n_bc, const sdugks_params *prm, MeshBuild &mb)
{
    int rc = check_prm(prm);
    if (rc) return rc;
    std::string err;
    rc = build_mesh(mesh, bc, n_bc, prm, mb, err);
    if (rc) return fail(rc, "mesh: " + err);
    if (prm->precision != SDUGKS_FP64 && mb.n_tiles == 0)
        return fail(SDUGKS_EINVAL, "FP32 storage needs the fused step (polygons of at most four faces, at most 64 boundary-condition entries, tile_cells >= 0)");
    if (prm->scheme == SDUGKS_SCHEME_ORIGINAL && mb.n_tiles == 0)
        return fail(SDUGKS_EINVAL, "SDUGKS_SCHEME_ORIGINAL needs the fused step (polygons of at most four faces, at most 64 boundary-condition entries, tile_cells >= 0)");
    return SDUGKS_OK;
}

// Upload helper: host vector into a pitched [rows][np] device block.
template <typename T>
int upload_rows(T *dst, const std::vector<T> &src, size_t rows, size_t nc, size_t np, hipStream_t st)
{
    std::vector<T> tmp(rows * np, T(0));
    for (size_t r = 0; r < rows; r++) std::copy(src.begin() + r * nc, src.begin() + (r + 1) * nc, tmp.begin() + r * np);
    HIPCHK(hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return SDUGKS_OK;
}

double feq_host(int i, double rho, double ux, double uy)
{
    static const double ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    const double eu = ex[i] * ux + ey[i] * uy, uu = ux * ux + uy * uy;
    return w[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

int sync_check(sdugks_t *h)
{
    HIPCHK(hipStreamSynchronize(h->stream));
    return SDUGKS_OK;
}

// Run the reduction kernel and fetch {num, den, mass, nonfinite}.
int reduce(sdugks_t *h, int update_snap, double out[4])
{
    HIPCHK(hipSetDevice(h->device));
    DevState s = h->state();
    HIPCHK(launch_reduce(h->dm, s.W, h->at<double>(h->L.off_snap), update_snap, h->at<double>(h->L.off_part),
                         h->at<double>(h->L.off_out), h->stream));
    HIPCHK(hipMemcpyAsync(h->host4, h->at<double>(h->L.off_out), 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    std::memcpy(out, h->host4, 4 * sizeof(double));
    if (out[3] != 0.0) h->diverged = true;
    return SDUGKS_OK;
}

// One step that reads buffer index c, on stream st, or appended to a graph
// chain (no bookkeeping).
int launch_step_at(sdugks_t *h, int c, hipStream_t st, GraphChain *gc = nullptr)
{
    DevState s = h->state_at(c);
    const int lagged = h->macro == SDUGKS_MACRO_LAGGED;
    if (h->mb.cart) {
        HIPCHK(launch_step_cart(h->dm, h->dc, s, lagged, h->precision, st, gc));
    } else if (h->mb.n_tiles > 0) {
        HIPCHK(launch_step_tiled(h->dm, h->dt, s, lagged, h->precision, h->block, st, gc));
    } else {
        DevScratch x = h->scratch();
        HIPCHK(launch_grad(h->dm, s, x, st, gc));
        HIPCHK(launch_flux_update(h->dm, s, x, lagged, st, gc));
    }
    return SDUGKS_OK;
}

int enqueue_step(sdugks_t *h)
{
    int rc = launch_step_at(h, h->cur, h->stream);
    if (rc) return rc;
    h->cur ^= 1;
    h->step++;
    return SDUGKS_OK;
}

void release_step_graphs(sdugks_t *h)
{
    for (int c = 0; c < 2; c++)
        for (int k = 0; k < 2; k++) {
            if (h->exec[c][k]) (void)hipGraphExecDestroy(h->exec[c][k]);
            if (h->graph[c][k]) (void)hipGraphDestroy(h->graph[c][k]);
            h->exec[c][k] = nullptr;
            h->graph[c][k] = nullptr;
        }
}

// `pairs` pairs of steps starting from buffer index c as one graph, built
// node by node (no stream capture: nothing another thread does can
// invalidate it); launched on the handle's stream.
int capture_step_graph(sdugks_t *h, int c, int64_t pairs, hipGraph_t &graph, hipGraphExec_t &exec)
{
    hipGraph_t gr = nullptr;
    HIPCHK(hipGraphCreate(&gr, 0));
    GraphChain gc;
    gc.graph = gr;
    int rc = 0;
    for (int64_t k = 0; k < pairs && !rc; k++) {
        rc = launch_step_at(h, c, h->stream, &gc);
        if (!rc) rc = launch_step_at(h, c ^ 1, h->stream, &gc);
    }
    if (rc) { (void)hipGraphDestroy(gr); return rc; }
    const hipError_t ie = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(gr);
        exec = nullptr;
        return fail(SDUGKS_EHIP, std::string("graph instantiation: ") + hipGetErrorString(ie));
    }
    graph = gr;
    return SDUGKS_OK;
}

}  // namespace

extern "C" {

const char *sdugks_last_error(void) { return g_err.c_str(); }

int sdugks_geometry(const sdugks_mesh *mesh, const sdugks_bc *bc, int32_t n_bc, const sdugks_params *prm,
                    double *dt, double *tau, double *h_min, int32_t *n_faces, double *area, double *cx, double *cy,
                    int32_t *perm)
{
    MeshBuild mb;
    int rc = build(mesh, bc, n_bc, prm, mb);
    if (rc) return rc;
    if (dt) *dt = mb.dt;
    if (tau) *tau = mb.tau;
    if (h_min) *h_min = mb.h_min;
    if (n_faces) *n_faces = mb.n_faces;
    for (int32_t k = 0; k < mb.nc; k++) {
        int32_t c = mb.perm[k];
        if (area) area[c] = mb.area[k];
        if (cx) cx[c] = mb.cx[k];
        if (cy) cy[c] = mb.cy[k];
        if (perm) perm[k] = c;
    }
    return SDUGKS_OK;
}

int sdugks_tiling(const sdugks_mesh *mesh, const sdugks_bc *bc, int32_t n_bc, const sdugks_params *prm,
                  int32_t *tile_cells, int32_t *n_tiles, int32_t *max_local, int32_t *max_ring1, int32_t *structured)
{
    MeshBuild mb;
    int rc = build(mesh, bc, n_bc, prm, mb);
    if (rc) return rc;
    if (tile_cells) *tile_cells = mb.tile_T;
    if (n_tiles) *n_tiles = mb.n_tiles;
    const int32_t rows = cart_tile_rows(prm->precision);
    if (max_local) *max_local = mb.cart ? (kCartTX + 4) * (rows + 4) : mb.nl_max;
    if (max_ring1) *max_ring1 = mb.cart ? (kCartTX + 2) * (rows + 2) : mb.na_max;
    if (structured) *structured = mb.cart ? 1 : 0;
    return SDUGKS_OK;
}

int sdugks_state_bytes(const sdugks_mesh *mesh, const sdugks_bc *bc, int32_t n_bc, const sdugks_params *prm,
                       size_t *bytes)
{
    if (!bytes) return fail(SDUGKS_EINVAL, "null bytes");
    MeshBuild mb;
    int rc = build(mesh, bc, n_bc, prm, mb);
    if (rc) return rc;
    *bytes = make_layout(mb, prm->precision).total;
    return SDUGKS_OK;
}

int sdugks_create(const sdugks_mesh *mesh, const sdugks_bc *bc, int32_t n_bc, const sdugks_params *prm,
                  void *stream, void *workspace, size_t workspace_bytes, sdugks_t **out)
{
    if (!out) return fail(SDUGKS_EINVAL, "null out");
    *out = nullptr;
    sdugks_t *h = new (std::nothrow) sdugks_t();
    if (!h) return fail(SDUGKS_ENOMEM, "host allocation failed");
    int rc = build(mesh, bc, n_bc, prm, h->mb);
    if (rc) { delete h; return rc; }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) { delete h; return fail(SDUGKS_ENODEV, "no HIP device"); }
    if (hipGetDevice(&h->device) != hipSuccess) { delete h; return fail(SDUGKS_ENODEV, "no current HIP device"); }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) != hipSuccess || std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        delete h;
        return fail(SDUGKS_ENODEV, "the current device is not gfx950");
    }
    h->stream = (hipStream_t)stream;
    h->block = prm->block_threads ? prm->block_threads : 256;
    h->precision = prm->precision;
    h->macro = prm->macro_flux;
    h->scheme = prm->scheme;
    h->rho0 = prm->rho0;
    h->L = make_layout(h->mb, prm->precision);
    const Layout &L = h->L;
    if (workspace) {
        if (workspace_bytes < L.total || ((uintptr_t)workspace % kAlign)) {
            delete h;
            return fail(SDUGKS_ENOMEM, "workspace smaller than sdugks_state_bytes or not 256-byte aligned");
        }
        h->base = (char *)workspace;
    } else {
        if (hipMalloc((void **)&h->base, L.total) != hipSuccess) { delete h; return fail(SDUGKS_ENOMEM, "hipMalloc of the state failed"); }
        h->own = true;
    }
    if (hipHostMalloc((void **)&h->host4, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        if (h->own) (void)hipFree(h->base);
        delete h;
        return fail(SDUGKS_ENOMEM, "pinned host allocation failed");
    }
    const MeshBuild &mb = h->mb;
    const size_t nc = mb.nc, np = L.np;
    auto cleanup = [&](int code) {
        if (h->own) (void)hipFree(h->base);
        (void)hipHostFree(h->host4);
        delete h;
        return code;
    };
    // geometry
    const bool dev = h->dev32(), tiled = mb.n_tiles > 0;
    if (!tiled) {
        // two-kernel step (FP64 only): face geometry as (x, y) pairs, rows [3][D]
        // (l n, r_self, r_other) of np pairs each
        const size_t D = mb.D, n_geo = 3 * D * np * 2;
        std::vector<double> geo(n_geo, 0.0);
        const std::vector<double> *parts[3][2] = {{&mb.lnx, &mb.lny}, {&mb.rsx, &mb.rsy}, {&mb.rox, &mb.roy}};
        for (size_t k = 0; k < 3; k++)
            for (size_t sl = 0; sl < D; sl++)
                for (size_t c = 0; c < nc; c++)
                    for (size_t e = 0; e < 2; e++)
                        geo[((k * D + sl) * np + c) * 2 + e] = (*parts[k][e])[sl * nc + c];
        if (hipMemcpy(h->at<double>(L.off_geo), geo.data(), n_geo * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(SDUGKS_EHIP, "upload of the face geometry failed"));
    }
    if (!tiled) {
        rc = upload_rows(h->at<int32_t>(L.off_nbr), mb.nbr, mb.D, nc, np, h->stream);
        if (rc) return cleanup(rc);
        rc = upload_rows(h->at<double>(L.off_ainv), mb.ainv, 3, nc, np, h->stream);
        if (rc) return cleanup(rc);
        if (mb.n_bfaces &&
            hipMemcpy(h->at<int32_t>(L.off_bft), mb.bf_tag.data(), mb.n_bfaces * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(SDUGKS_EHIP, "upload of boundary tags failed"));
    }
    {
        std::vector<double> dtv(nc);
        for (size_t c = 0; c < nc; c++) dtv[c] = mb.dt / mb.area[c];
        rc = upload_rows(h->at<double>(L.off_dtv), dtv, 1, nc, np, h->stream);
        if (rc) return cleanup(rc);
        rc = upload_rows(h->at<double>(L.off_area), mb.area, 1, nc, np, h->stream);
        if (rc) return cleanup(rc);
    }
    {
        std::vector<DevBC> bcs(mb.bcs.size());
        for (size_t t = 0; t < bcs.size(); t++) bcs[t] = {mb.bcs[t].type, mb.bcs[t].rho, mb.bcs[t].u, mb.bcs[t].v};
        if (!bcs.empty() && hipMemcpy(h->at<DevBC>(L.off_bcs), bcs.data(), bcs.size() * sizeof(DevBC), hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(SDUGKS_EHIP, "upload of the boundary table failed"));
    }
    {
        // boundary-face table: cell, slot and tag of every plain boundary face,
        // the cell's stencil and weights, the face's l n and r_self
        const size_t nbf = mb.n_bfaces, D = mb.D;
        std::vector<int4> hdr(std::max<size_t>(1, nbf), int4{0, 0, 0, 0});
        std::vector<int32_t> nb(std::max<size_t>(1, nbf) * D, -1);
        std::vector<double2> w(std::max<size_t>(1, nbf) * D, double2{0.0, 0.0});
        std::vector<double2> geo(std::max<size_t>(1, nbf) * 2, double2{0.0, 0.0});
        for (size_t k = 0; k < nc; k++)
            for (size_t sl = 0; sl < D; sl++) {
                const int32_t v = mb.nbr[sl * nc + k];
                if (v >= 0 || v == kEmptySlot) continue;
                const size_t b = (size_t)(-1 - v), q = sl * nc + k;
                hdr[b] = int4{(int)k, (int)sl, mb.bf_tag[b], 0};
                geo[2 * b] = double2{mb.lnx[q], mb.lny[q]};
                geo[2 * b + 1] = double2{mb.rsx[q], mb.rsy[q]};
                for (size_t j = 0; j < D; j++) {
                    const size_t qj = j * nc + k;
                    const int32_t u = mb.nbr[qj];
                    nb[b * D + j] = u == kEmptySlot ? -1 : (u >= 0 ? u : -2 - mb.bf_tag[-1 - u]);
                    w[b * D + j] = double2{mb.wx[qj], mb.wy[qj]};
                }
            }
        auto upb = [&](size_t off, const void *src, size_t bytes) {
            return hipMemcpy(h->base + off, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
        };
        if (!upb(L.off_bq_hdr, hdr.data(), hdr.size() * sizeof(int4)) || !upb(L.off_bq_nb, nb.data(), nb.size() * sizeof(int32_t)) ||
            !upb(L.off_bq_w, w.data(), w.size() * sizeof(double2)) || !upb(L.off_bq_geo, geo.data(), geo.size() * sizeof(double2)))
            return cleanup(fail(SDUGKS_EHIP, "upload of the boundary-face table failed"));
        h->bq.n = (int32_t)nbf;
        h->bq.hdr = h->at<int4>(L.off_bq_hdr);
        h->bq.nb = h->at<int32_t>(L.off_bq_nb);
        h->bq.w = h->at<double2>(L.off_bq_w);
        h->bq.geo = h->at<double2>(L.off_bq_geo);
        h->bq.out = h->at<double>(L.off_bq_out);
        h->bq.sum = h->at<double>(L.off_bq_sum);
    }
    if (mb.cart) {
        auto up = [&](size_t off, const void *src, size_t bytes) {
            return hipMemcpy(h->base + off, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
        };
        if (!up(L.off_ccol, mb.col.data(), mb.col.size() * sizeof(double)) ||
            !up(L.off_crow, mb.row.data(), mb.row.size() * sizeof(double)) ||
            !up(L.off_cside, mb.side.data(), mb.side.size() * sizeof(int32_t)))
            return cleanup(fail(SDUGKS_EHIP, "upload of the structured-grid tables failed"));
        h->dc.nx = mb.nx; h->dc.ny = mb.ny; h->dc.ntx = mb.ntx; h->dc.nty = mb.nty;
        h->dc.per_x = mb.per_x; h->dc.per_y = mb.per_y;
        h->dc.col = h->at<double>(L.off_ccol);
        h->dc.row = h->at<double>(L.off_crow);
        h->dc.side = h->at<int32_t>(L.off_cside);
    } else if (tiled) {
        auto up = [&](size_t off, const void *src, size_t bytes) {
            return hipMemcpy(h->base + off, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
        };
        std::vector<float> frec32, lw32;
        if (dev) { frec32.assign(mb.frec.begin(), mb.frec.end()); lw32.assign(mb.lw.begin(), mb.lw.end()); }
        if (!up(L.off_thdr, mb.tile_hdr.data(), mb.tile_hdr.size() * sizeof(int32_t)) ||
            !up(L.off_lgid, mb.lgid.data(), mb.lgid.size() * sizeof(int32_t)) ||
            !up(L.off_ladj, mb.ladj.data(), mb.ladj.size() * sizeof(int16_t)) ||
            !up(L.off_lfc, mb.lfc.data(), mb.lfc.size() * sizeof(int16_t)) ||
            !(dev ? up(L.off_frec, frec32.data(), frec32.size() * sizeof(float))
                  : up(L.off_frec, mb.frec.data(), mb.frec.size() * sizeof(double))) ||
            !(dev ? up(L.off_lw, lw32.data(), lw32.size() * sizeof(float))
                  : up(L.off_lw, mb.lw.data(), mb.lw.size() * sizeof(double))))
            return cleanup(fail(SDUGKS_EHIP, "upload of the tile tables failed"));
        h->dt.n_tiles = mb.n_tiles;
        h->dt.nl_max = mb.nl_max;
        h->dt.na_max = mb.na_max;
        h->dt.nt_max = mb.nt_max;
        h->dt.nf_max = std::max<int32_t>(1, mb.nf_max);
        h->dt.hdr = h->at<int32_t>(L.off_thdr);
        h->dt.lgid = h->at<int32_t>(L.off_lgid);
        h->dt.ladj = h->at<int16_t>(L.off_ladj);
        h->dt.lfc = h->at<int16_t>(L.off_lfc);
        h->dt.fr = dev ? nullptr : h->at<double2>(L.off_frec);
        h->dt.fr32 = dev ? h->at<float2>(L.off_frec) : nullptr;
        h->dt.lw = dev ? nullptr : h->at<double2>(L.off_lw);
        h->dt.lw32 = dev ? h->at<float2>(L.off_lw) : nullptr;
    }
    DevMesh &d = h->dm;
    d.nc = mb.nc; d.np = (int32_t)np; d.D = mb.D; d.n_bfaces = mb.n_bfaces; d.n_bc = (int32_t)mb.bcs.size();
    const size_t blk = (size_t)mb.D * np;
    if (!tiled) {
        const double2 *g = h->at<double2>(L.off_geo);
        d.ln = g; d.rs = g + blk; d.ro = g + 2 * blk;
    }
    if (!tiled) {
        d.nbr = h->at<int32_t>(L.off_nbr);
        d.ainv = h->at<double>(L.off_ainv);
        d.bf_tag = h->at<int32_t>(L.off_bft);
    }
    d.rho0 = prm->rho0;
    d.dtv = h->at<double>(L.off_dtv);
    d.area = h->at<double>(L.off_area);
    d.bcs = h->at<DevBC>(L.off_bcs);
    const double tau = mb.tau, dt = mb.dt;
    d.a = (2.0 * tau - dt) / (2.0 * tau);
    d.b = dt / (2.0 * tau);
    d.c1 = 2.0 * tau / (2.0 * tau + dt);
    d.lam = dt / tau;
    d.inv1l = 1.0 / (1.0 + d.lam);
    d.dtr = dt; d.fb = d.b; d.fc1 = d.c1; d.scheme = h->scheme;
    if (h->scheme == SDUGKS_SCHEME_ORIGINAL) {
        const double hh = 0.5 * dt;
        d.a = (2.0 * tau - hh) / (2.0 * tau + dt);
        d.b = 3.0 * hh / (2.0 * tau + dt);
        d.dtr = hh; d.fb = hh / (2.0 * tau); d.fc1 = 2.0 * tau / (2.0 * tau + hh);
    }
    d.dt = dt;
    // initial state: uniform equilibrium, G = 0, snapshot = initial velocity
    {
        std::vector<double> f(9 * nc), W(3 * nc), G(3 * nc, 0.0);
        for (size_t c = 0; c < nc; c++) {
            for (int i = 0; i < 9; i++) f[c * 9 + i] = feq_host(i, prm->rho0, prm->u0, prm->v0);
            W[3 * c] = prm->rho0; W[3 * c + 1] = prm->rho0 * prm->u0; W[3 * c + 2] = prm->rho0 * prm->v0;
        }
        *out = h;
        // set_state expects caller order; the uniform state is order-free
        rc = sdugks_set_state(h, f.data(), W.data(), G.data());
        if (rc) { *out = nullptr; return cleanup(rc); }
    }
    return SDUGKS_OK;
}

// The original scheme stores ft = f - (dt/2) Omega = (1 + k) f - k feq(W),
// k = dt/(2 tau); inverse f = (ft + k feq(W)) / (1 + k).  Caller order, in place.
static void tilde_convert(double *f, const double *W, size_t nc, double k, bool inverse)
{
    for (size_t c = 0; c < nc; c++) {
        const double r = W[3 * c], u = W[3 * c + 1] / r, v = W[3 * c + 2] / r;
        for (int i = 0; i < 9; i++) {
            const double fe = feq_host(i, r, u, v);
            double &x = f[c * 9 + i];
            x = inverse ? (x + k * fe) / (1.0 + k) : (1.0 + k) * x - k * fe;
        }
    }
}

int sdugks_set_state(sdugks_t *h, const double *f, const double *W, const double *G)
{
    if (!h) return fail(SDUGKS_EINVAL, "null handle");
    HIPCHK(hipSetDevice(h->device));
    const size_t nc = h->mb.nc, np = h->L.np;
    std::vector<double> ft, Wc;
    const bool neq = h->precision == SDUGKS_FP32NEQ;
    if (f && (h->scheme == SDUGKS_SCHEME_ORIGINAL || neq)) {
        // the macros that go with f: the new ones, else the stored ones
        Wc.resize(3 * nc);
        if (W) std::copy(W, W + 3 * nc, Wc.begin());
        else if (int r0 = sdugks_get_state(h, nullptr, Wc.data(), nullptr)) return r0;
    }
    if (f && h->scheme == SDUGKS_SCHEME_ORIGINAL) {
        ft.assign(f, f + 9 * nc);
        tilde_convert(ft.data(), Wc.data(), nc, h->mb.dt / (2.0 * h->mb.tau), false);
        f = ft.data();
    }
    const Layout &L = h->L;
    std::vector<double> buf(9 * np, 0.0);
    auto put = [&](const double *src, int rows, size_t off) -> int {
        std::fill(buf.begin(), buf.end(), 0.0);
        for (size_t k = 0; k < nc; k++) {
            size_t c = h->mb.perm[k];
            for (int r = 0; r < rows; r++) buf[r * np + k] = src[c * rows + r];
        }
        HIPCHK(hipMemcpyAsync(h->base + off, buf.data(), rows * np * sizeof(double), hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        return SDUGKS_OK;
    };
    int rc;
    if (f && h->dev32()) {
        // FP32 storage: f - w_i rho0 (FP32DEV) or f - feq(W) (FP32NEQ)
        static const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
        std::vector<float> b32(9 * np, 0.0f);
        for (size_t k = 0; k < nc; k++) {
            size_t c = h->mb.perm[k];
            for (int i = 0; i < 9; i++) {
                double ref = w[i] * h->rho0;
                if (neq) {
                    const double r = Wc[3 * c];
                    ref = feq_host(i, r, Wc[3 * c + 1] / r, Wc[3 * c + 2] / r);
                }
                b32[i * np + k] = (float)(f[c * 9 + i] - ref);
            }
        }
        HIPCHK(hipMemcpyAsync(h->base + L.off_f[h->cur], b32.data(), 9 * np * sizeof(float), hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    } else if (f && (rc = put(f, 9, L.off_f[h->cur]))) {
        return rc;
    }
    if (W) {
        if ((rc = put(W, 3, L.off_W[h->cur]))) return rc;
        // snapshot of the residual = this velocity field
        std::vector<double> snap(2 * np, 0.0);
        for (size_t k = 0; k < nc; k++) {
            size_t c = h->mb.perm[k];
            snap[k] = W[3 * c + 1] / W[3 * c];
            snap[np + k] = W[3 * c + 2] / W[3 * c];
        }
        HIPCHK(hipMemcpyAsync(h->base + L.off_snap, snap.data(), 2 * np * sizeof(double), hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    if (G && (rc = put(G, 3, L.off_G[h->cur]))) return rc;
    h->diverged = false;
    return SDUGKS_OK;
}

int sdugks_get_state(sdugks_t *h, double *f, double *W, double *G)
{
    if (!h) return fail(SDUGKS_EINVAL, "null handle");
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipStreamSynchronize(h->stream));
    const size_t nc = h->mb.nc, np = h->L.np;
    const Layout &L = h->L;
    std::vector<double> buf(9 * np);
    auto get = [&](double *dst, int rows, size_t off) -> int {
        HIPCHK(hipMemcpyAsync(buf.data(), h->base + off, rows * np * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (size_t k = 0; k < nc; k++) {
            size_t c = h->mb.perm[k];
            for (int r = 0; r < rows; r++) dst[c * rows + r] = buf[r * np + k];
        }
        return SDUGKS_OK;
    };
    int rc;
    const bool neq = h->precision == SDUGKS_FP32NEQ;
    std::vector<double> Wc;
    if (f && (neq || h->scheme == SDUGKS_SCHEME_ORIGINAL)) {
        Wc.resize(3 * nc);
        if ((rc = get(Wc.data(), 3, L.off_W[h->cur]))) return rc;
    }
    if (f && h->dev32()) {
        // FP32 storage: f = w_i rho0 (FP32DEV) or feq(W) (FP32NEQ) + stored part
        static const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
        std::vector<float> b32(9 * np);
        HIPCHK(hipMemcpyAsync(b32.data(), h->base + L.off_f[h->cur], 9 * np * sizeof(float), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (size_t k = 0; k < nc; k++) {
            size_t c = h->mb.perm[k];
            for (int i = 0; i < 9; i++) {
                double ref = w[i] * h->rho0;
                if (neq) {
                    const double r = Wc[3 * c];
                    ref = feq_host(i, r, Wc[3 * c + 1] / r, Wc[3 * c + 2] / r);
                }
                f[c * 9 + i] = ref + (double)b32[i * np + k];
            }
        }
    } else if (f && (rc = get(f, 9, L.off_f[h->cur]))) {
        return rc;
    }
    if (W && (rc = get(W, 3, L.off_W[h->cur]))) return rc;
    if (f && h->scheme == SDUGKS_SCHEME_ORIGINAL) tilde_convert(f, Wc.data(), nc, h->mb.dt / (2.0 * h->mb.tau), true);
    if (G) {
        if (h->macro == SDUGKS_MACRO_LAGGED) { if ((rc = get(G, 3, L.off_G[h->cur]))) return rc; }
        else std::fill(G, G + 3 * nc, 0.0);
    }
    return SDUGKS_OK;
}

int sdugks_set_macros(sdugks_t *h, const double *rho, const double *u, const double *v)
{
    if (!h || !rho || !u || !v) return fail(SDUGKS_EINVAL, "null argument");
    const size_t nc = h->mb.nc, np = h->L.np;
    for (size_t c = 0; c < nc; c++)
        if (!(rho[c] > 0.0) || !std::isfinite(rho[c]) || !std::isfinite(u[c]) || !std::isfinite(v[c]))
            return fail(SDUGKS_EINVAL, "set_macros: rho must be positive and rho, u, v finite (cell " +
                                           std::to_string(c) + ")");
    HIPCHK(hipSetDevice(h->device));
    // the macros staged in the W rows the next step writes, in the internal order
    std::vector<double> m3(3 * nc);
    for (size_t k = 0; k < nc; k++) {
        const size_t c = h->mb.perm[k];
        m3[k] = rho[c];
        m3[nc + k] = u[c];
        m3[2 * nc + k] = v[c];
    }
    double *stage = h->at<double>(h->L.off_W[h->cur ^ 1]);
    int rc = upload_rows(stage, m3, 3, nc, np, h->stream);
    if (rc) return rc;
    const bool dev = h->dev32();
    HIPCHK(launch_set_equilibrium((int)nc, (int)np, stage, dev ? nullptr : h->at<double>(h->L.off_f[h->cur]),
                                  dev ? h->at<float>(h->L.off_f[h->cur]) : nullptr,
                                  h->precision == SDUGKS_FP32NEQ ? -1.0 : h->rho0,
                                  h->at<double>(h->L.off_W[h->cur]), h->at<double>(h->L.off_G[h->cur]),
                                  h->at<double>(h->L.off_snap), h->stream));
    rc = sync_check(h);
    if (rc) return rc;
    h->diverged = false;
    return SDUGKS_OK;
}

int sdugks_macros(sdugks_t *h, double *rho, double *u, double *v)
{
    if (!h) return fail(SDUGKS_EINVAL, "null handle");
    std::vector<double> W(3 * (size_t)h->mb.nc);
    int rc = sdugks_get_state(h, nullptr, W.data(), nullptr);
    if (rc) return rc;
    for (int32_t c = 0; c < h->mb.nc; c++) {
        if (rho) rho[c] = W[3 * c];
        if (u) u[c] = W[3 * c + 1] / W[3 * c];
        if (v) v[c] = W[3 * c + 2] / W[3 * c];
    }
    return SDUGKS_OK;
}

int sdugks_step(sdugks_t *h, int64_t n)
{
    if (!h) return fail(SDUGKS_EINVAL, "null handle");
    if (n < 0) return fail(SDUGKS_EINVAL, "negative step count");
    if (h->diverged) return fail(SDUGKS_EDIVERGED, "state is not finite; reset it with sdugks_set_state");
    HIPCHK(hipSetDevice(h->device));
    // whole runs of kGraphPairs pairs replay the long graph, the remaining
    // pairs the one-pair graph, an odd last step is launched alone
    int64_t pairs = n / 2;
    const int64_t runs = pairs / kGraphPairs;
    pairs -= runs * kGraphPairs;
    const int c = h->cur;
    int rc;
    if (runs > 0) {
        if (!h->exec[c][1] && (rc = capture_step_graph(h, c, kGraphPairs, h->graph[c][1], h->exec[c][1]))) return rc;
        for (int64_t k = 0; k < runs; k++) HIPCHK(hipGraphLaunch(h->exec[c][1], h->stream));
    }
    if (pairs > 0) {
        if (!h->exec[c][0] && (rc = capture_step_graph(h, c, 1, h->graph[c][0], h->exec[c][0]))) return rc;
        for (int64_t k = 0; k < pairs; k++) HIPCHK(hipGraphLaunch(h->exec[c][0], h->stream));
    }
    h->step += 2 * (n / 2);
    if (n & 1) return enqueue_step(h);
    return SDUGKS_OK;
}

int sdugks_step_eager(sdugks_t *h, int64_t n)
{
    if (!h) return fail(SDUGKS_EINVAL, "null handle");
    if (n < 0) return fail(SDUGKS_EINVAL, "negative step count");
    if (h->diverged) return fail(SDUGKS_EDIVERGED, "state is not finite; reset it with sdugks_set_state");
    HIPCHK(hipSetDevice(h->device));
    for (int64_t k = 0; k < n; k++) {
        int rc = enqueue_step(h);
        if (rc) return rc;
    }
    return SDUGKS_OK;
}

int sdugks_step_profiled(sdugks_t *h, int64_t n, double *avg_ms, const char **names, int32_t max_kernels,
                         int32_t *n_kernels)
{
    if (!h || !avg_ms || max_kernels < 2 || !n_kernels || n < 0) return fail(SDUGKS_EINVAL, "bad arguments");
    if (h->diverged) return fail(SDUGKS_EDIVERGED, "state is not finite");
    HIPCHK(hipSetDevice(h->device));
    const bool tiled = h->mb.n_tiles > 0;
    const int nk = tiled ? 1 : 2;
    struct Events {                       // destroyed on every return path
        hipEvent_t e[3] = {nullptr, nullptr, nullptr};
        ~Events() { for (hipEvent_t x : e) if (x) (void)hipEventDestroy(x); }
    } evs;
    hipEvent_t *ev = evs.e;
    for (int k = 0; k < 3; k++) HIPCHK(hipEventCreate(&ev[k]));
    double acc[2] = {0, 0};
    for (int64_t k = 0; k < n; k++) {
        DevState s = h->state();
        const int lagged = h->macro == SDUGKS_MACRO_LAGGED;
        HIPCHK(hipEventRecord(ev[0], h->stream));
        if (h->mb.cart) {
            HIPCHK(launch_step_cart(h->dm, h->dc, s, lagged, h->precision, h->stream));
            HIPCHK(hipEventRecord(ev[1], h->stream));
        } else if (tiled) {
            HIPCHK(launch_step_tiled(h->dm, h->dt, s, lagged, h->precision, h->block, h->stream));
            HIPCHK(hipEventRecord(ev[1], h->stream));
        } else {
            DevScratch x = h->scratch();
            HIPCHK(launch_grad(h->dm, s, x, h->stream));
            HIPCHK(hipEventRecord(ev[1], h->stream));
            HIPCHK(launch_flux_update(h->dm, s, x, lagged, h->stream));
            HIPCHK(hipEventRecord(ev[2], h->stream));
        }
        HIPCHK(hipEventSynchronize(ev[nk]));
        float a = 0, b = 0;
        HIPCHK(hipEventElapsedTime(&a, ev[0], ev[1]));
        if (!tiled) HIPCHK(hipEventElapsedTime(&b, ev[1], ev[2]));
        acc[0] += a; acc[1] += b;
        h->cur ^= 1;
        h->step++;
    }
    for (int k = 0; k < nk; k++) avg_ms[k] = n ? acc[k] / n : 0;
    if (names) {
        if (h->mb.cart) names[0] = "k_step_cart";
        else if (tiled) names[0] = "k_step_tiled";
        else { names[0] = "k_grad"; names[1] = "k_flux_update"; }
    }
    *n_kernels = nk;
    return SDUGKS_OK;
}

int sdugks_residual(sdugks_t *h, double *eps)
{
    if (!h || !eps) return fail(SDUGKS_EINVAL, "null argument");
    double r[4];
    int rc = reduce(h, 1, r);
    if (rc) return rc;
    if (r[3] != 0.0) { *eps = NAN; return fail(SDUGKS_EDIVERGED, "non-finite density or velocity"); }
    *eps = r[1] > 0 ? std::sqrt(r[0]) / std::sqrt(r[1]) : INFINITY;
    return SDUGKS_OK;
}

int sdugks_mass(sdugks_t *h, double *mass)
{
    if (!h || !mass) return fail(SDUGKS_EINVAL, "null argument");
    double r[4];
    int rc = reduce(h, 0, r);
    if (rc) return rc;
    *mass = r[2];
    if (r[3] != 0.0) return fail(SDUGKS_EDIVERGED, "non-finite density or velocity");
    return SDUGKS_OK;
}

int sdugks_boundary_flux(sdugks_t *h, int32_t tag, double *faces, double *sum, int32_t *n_faces)
{
    if (!h) return fail(SDUGKS_EINVAL, "null handle");
    if (tag >= (int32_t)h->mb.bcs.size()) return fail(SDUGKS_EINVAL, "tag beyond the boundary-condition table");
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(launch_boundary_flux(h->dm, h->state(), h->bq, h->precision, tag, h->stream));
    if (faces && h->bq.n > 0)
        HIPCHK(hipMemcpyAsync(faces, h->bq.out, (size_t)h->bq.n * 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(h->host4, h->bq.sum, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (sum) std::memcpy(sum, h->host4, 3 * sizeof(double));
    if (n_faces) *n_faces = h->bq.n;
    return SDUGKS_OK;
}

int sdugks_info(sdugks_t *h, double *dt, double *tau, int64_t *step, int32_t *n_cells)
{
    if (!h) return fail(SDUGKS_EINVAL, "null handle");
    if (dt) *dt = h->mb.dt;
    if (tau) *tau = h->mb.tau;
    if (step) *step = h->step;
    if (n_cells) *n_cells = h->mb.nc;
    return SDUGKS_OK;
}

int sdugks_destroy(sdugks_t *h)
{
    if (!h) return SDUGKS_OK;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    release_step_graphs(h);
    if (h->own) (void)hipFree(h->base);
    (void)hipHostFree(h->host4);
    delete h;
    return SDUGKS_OK;
}

int sdugks_debug_poison(sdugks_t *h, int32_t cell, int32_t i)
{
    if (!h || cell < 0 || cell >= h->mb.nc || i < 0 || i > 8) return fail(SDUGKS_EINVAL, "bad poison target");
    HIPCHK(hipSetDevice(h->device));
    const size_t idx = (size_t)i * h->L.np + h->mb.iperm[cell];
    void *p = h->dev32() ? (void *)(h->at<float>(h->L.off_f[h->cur]) + idx) : (void *)(h->at<double>(h->L.off_f[h->cur]) + idx);
    HIPCHK(launch_poke_nan(p, h->dev32() ? 4 : 8, h->stream));
    return sync_check(h);
}

namespace {

const char *const kBatchFailedMsg =
    "the batch lost its members when a table rebuild failed; set them again with sdugks_batch_set_members";

size_t next_pow2(size_t x)
{
    size_t p = 8;
    while (p < x) p <<= 1;
    return p;
}

void batch_release_graph(sdugks_batch_t *b)
{
    for (int k = 0; k < kBatchGraphs; k++) {
        if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
        if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
        b->exec[k] = nullptr;
        b->graph[k] = nullptr;
    }
}

void batch_release_groups(sdugks_batch_t *b)
{
    for (auto &g : b->groups) {
        (void)hipFree(g.d_inst);
        (void)hipFree(g.d_tmap);
    }
    b->groups.clear();
}

// (Re)build the device tables for the current members.  Existing tables and
// the captured graph are kept when every group still fits their capacity,
// launch shape and LDS; otherwise they are reallocated and the graph dropped.
int batch_build_tables(sdugks_batch_t *b)
{
    std::vector<BatchGroup> want;
    for (size_t k = 0; k < b->members.size(); k++) {
        sdugks_t *h = b->members[k];
        const int D = h->mb.D <= 3 ? 3 : 4, mode = h->precision;
        const bool cart = h->mb.cart;
        BatchGroup *g = nullptr;
        for (auto &x : want) if (x.D == D && x.mode == mode && x.cart == cart) g = &x;
        if (!g) { want.emplace_back(); g = &want.back(); g->D = D; g->mode = mode; g->cart = cart; }
        g->members.push_back((int)k);
        g->block = cart ? step_cart_threads(mode) : std::max(g->block, h->block);
        g->lds = std::max(g->lds, cart ? step_cart_lds_bytes(mode, (int)h->mb.bcs.size())
                                       : step_tiled_lds_bytes(h->dt, mode, (int)h->mb.bcs.size()));
        g->n_inst++;
        g->n_tiles += h->mb.n_tiles;
    }
    bool reuse = want.size() == b->groups.size();
    for (size_t k = 0; reuse && k < want.size(); k++) {
        const BatchGroup &o = b->groups[k], &n = want[k];
        reuse = o.D == n.D && o.mode == n.mode && o.cart == n.cart && o.block >= n.block && o.lds >= n.lds &&
                o.cap_inst >= n.n_inst && o.cap_tiles >= n.n_tiles;
    }
    if (!reuse) {
        batch_release_graph(b);
        batch_release_groups(b);
        for (auto &g : want) {
            // tile slots: the live tiles rounded up to a sixteenth of their
            // power of two (at most 1/8 of the grid empty, room for members
            // that join later without a rebuild)
            const int32_t q = std::max<int32_t>(kXcds, (int32_t)(next_pow2(g.n_tiles) / 16));
            g.cap_inst = (int)next_pow2(g.n_inst);
            g.cap_tiles = std::max(q, (g.n_tiles + q - 1) / q * q);
            // LDS exactly the largest member's: a spare margin for later members
            // would cost resident workgroups per CU on every step (a member that
            // needs more rebuilds the group, like one that exceeds a capacity)
            if (hipMalloc((void **)&g.d_inst, g.cap_inst * sizeof(BatchInst)) != hipSuccess ||
                hipMalloc((void **)&g.d_tmap, batch_grid(g.cap_tiles) * sizeof(int2)) != hipSuccess) {
                for (auto &x : want) {
                    if (x.d_inst) (void)hipFree(x.d_inst);
                    if (x.d_tmap) (void)hipFree(x.d_tmap);
                }
                return fail(SDUGKS_ENOMEM, "hipMalloc of a batch table failed");
            }
        }
        b->groups = want;
        for (auto &g : want) g.d_inst = nullptr, g.d_tmap = nullptr;
    } else {
        for (size_t k = 0; k < want.size(); k++) {
            b->groups[k].members = want[k].members;
            b->groups[k].n_inst = want[k].n_inst;
            b->groups[k].n_tiles = want[k].n_tiles;
        }
    }
    // fill the tables (stream-ordered after any launch still reading them)
    b->cur_at_fill.resize(b->members.size());
    for (size_t k = 0; k < b->members.size(); k++) b->cur_at_fill[k] = b->members[k]->cur;
    for (auto &g : b->groups) {
        std::vector<BatchInst> inst(g.n_inst);
        std::vector<int2> seq;   // live tiles in member order: member, local tile
        seq.reserve(g.n_tiles);
        for (int k = 0; k < g.n_inst; k++) {
            sdugks_t *h = b->members[g.members[k]];
            BatchInst &e = inst[k];
            e.m = h->dm;
            e.t = h->dt;
            e.c = h->dc;
            for (int p = 0; p < 2; p++) {
                e.f[p] = h->base + h->L.off_f[p];
                e.W[p] = h->at<double>(h->L.off_W[p]);
                e.G[p] = h->at<double>(h->L.off_G[p]);
            }
            e.parity0 = h->cur;
            e.lagged = h->macro == SDUGKS_MACRO_LAGGED;
            for (int32_t t = 0; t < h->mb.n_tiles; t++) seq.push_back(make_int2(k, t));
        }
        // each XCD's range of tile slots gets an equal, contiguous share of the
        // live tiles at its start; the remaining slots are empty (-1)
        const int32_t grid = batch_grid(g.cap_tiles), per = grid / kXcds, n = (int32_t)seq.size();
        std::vector<int2> tmap(grid, make_int2(-1, 0));
        for (int32_t x = 0; x < kXcds; x++) {
            const int32_t lo = (int32_t)((int64_t)n * x / kXcds), hi = (int32_t)((int64_t)n * (x + 1) / kXcds);
            for (int32_t j = 0; j < hi - lo; j++) tmap[(size_t)x * per + j] = seq[lo + j];
        }
        HIPCHK(hipMemcpyAsync(g.d_inst, inst.data(), inst.size() * sizeof(BatchInst), hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipMemcpyAsync(g.d_tmap, tmap.data(), tmap.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    }
    return SDUGKS_OK;
}

// batch_build_tables, and on any failure a batch with no members, tables or
// graphs: tables left half filled (or a step with none, which would flip the
// members' buffer index without advancing them) must never be launched
int batch_build(sdugks_batch_t *b)
{
    const int rc = b->fail_next_build ? fail(SDUGKS_ENOMEM, "batch table rebuild failed (injected)")
                                      : batch_build_tables(b);
    b->fail_next_build = false;
    b->failed = rc != SDUGKS_OK;
    if (rc) {
        batch_release_graph(b);
        batch_release_groups(b);
        b->members.clear();
        b->cur_at_fill.clear();
    }
    return rc;
}

// One batched step: a launch per group.  In a graph the groups' nodes of one
// step depend only on the previous step's nodes (their members are disjoint),
// so the runtime may run them side by side.
int batch_launch(sdugks_batch_t *b, int parity, GraphChain *gc = nullptr)
{
    if (gc) gc->begin_fan();
    for (auto &g : b->groups) {
        BatchTable tab{g.d_inst, g.d_tmap};
        if (g.cart) HIPCHK(launch_step_batch_cart(tab, g.mode, parity, g.cap_tiles, g.lds, b->stream, gc));
        else HIPCHK(launch_step_batch(tab, g.D, g.mode, parity, g.cap_tiles, g.lds, g.block, b->stream, gc));
    }
    if (gc) gc->end_fan();
    return SDUGKS_OK;
}

// Order the batch stream after the members' streams (before) or the members'
// streams after the batch stream (after).
int batch_join(sdugks_batch_t *b, bool before)
{
    // each distinct member stream once: members usually share one stream, and
    // a record and a wait per member kept the host busy (and the batch
    // stream idle) for about 13 us per member before the first step
    std::vector<hipStream_t> seen;
    for (sdugks_t *h : b->members) {
        if (h->stream == b->stream || std::find(seen.begin(), seen.end(), h->stream) != seen.end()) continue;
        if (before) {
            HIPCHK(hipEventRecord(b->ev, h->stream));
            HIPCHK(hipStreamWaitEvent(b->stream, b->ev, 0));
        } else {
            if (seen.empty()) HIPCHK(hipEventRecord(b->ev, b->stream));
            HIPCHK(hipStreamWaitEvent(h->stream, b->ev, 0));
        }
        seen.push_back(h->stream);
    }
    return SDUGKS_OK;
}

int batch_check_members(sdugks_t *const *members, int32_t n)
{
    if (!members || n <= 0) return fail(SDUGKS_EINVAL, "bad batch members");
    for (int32_t k = 0; k < n; k++) {
        if (!members[k]) return fail(SDUGKS_EINVAL, "null batch member");
        if (members[k]->mb.n_tiles == 0) return fail(SDUGKS_EINVAL, "batch members need the fused step");
        if (members[k]->diverged) return fail(SDUGKS_EDIVERGED, "a batch member is not finite");
        for (int32_t j = 0; j < k; j++)
            if (members[j] == members[k]) return fail(SDUGKS_EINVAL, "a handle appears twice in a batch");
        if (members[k]->device != members[0]->device) return fail(SDUGKS_EINVAL, "batch members on different devices");
    }
    return SDUGKS_OK;
}

}  // namespace

int sdugks_batch_create(sdugks_t *const *members, int32_t n, void *stream, sdugks_batch_t **out)
{
    if (!out) return fail(SDUGKS_EINVAL, "null out");
    *out = nullptr;
    int rc = batch_check_members(members, n);
    if (rc) return rc;
    sdugks_batch_t *b = new (std::nothrow) sdugks_batch_t();
    if (!b) return fail(SDUGKS_ENOMEM, "host allocation failed");
    b->device = members[0]->device;
    HIPCHK(hipSetDevice(b->device));
    b->members.assign(members, members + n);
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) { delete b; return fail(SDUGKS_EHIP, "stream creation failed"); }
        b->own_stream = true;
    }
    if (hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) {
        sdugks_batch_destroy(b);
        return fail(SDUGKS_EHIP, "event creation failed");
    }
    rc = batch_build(b);
    if (rc) { sdugks_batch_destroy(b); return rc; }
    *out = b;
    return SDUGKS_OK;
}

int sdugks_batch_set_members(sdugks_batch_t *b, sdugks_t *const *members, int32_t n)
{
    if (!b) return fail(SDUGKS_EINVAL, "null batch");
    int rc = batch_check_members(members, n);
    if (rc) return rc;
    HIPCHK(hipSetDevice(b->device));
    HIPCHK(hipStreamSynchronize(b->stream));
    b->members.assign(members, members + n);
    return batch_build(b);
}

namespace {

// `pairs` pairs of batched steps as one graph, built node by node.
int batch_capture(sdugks_batch_t *b, int64_t pairs, hipGraph_t &graph, hipGraphExec_t &exec)
{
    hipGraph_t gr = nullptr;
    HIPCHK(hipGraphCreate(&gr, 0));
    GraphChain gc;
    gc.graph = gr;
    int rc = 0;
    for (int64_t k = 0; k < pairs && !rc; k++) {
        rc = batch_launch(b, 0, &gc);
        if (!rc) rc = batch_launch(b, 1, &gc);
    }
    if (rc) { (void)hipGraphDestroy(gr); return rc; }
    const hipError_t ie = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(gr);
        exec = nullptr;
        return fail(SDUGKS_EHIP, std::string("graph instantiation: ") + hipGetErrorString(ie));
    }
    graph = gr;
    return SDUGKS_OK;
}
}  // namespace

int sdugks_batch_step(sdugks_batch_t *b, int64_t n)
{
    if (!b) return fail(SDUGKS_EINVAL, "null batch");
    if (n < 0) return fail(SDUGKS_EINVAL, "negative step count");
    if (b->failed) return fail(SDUGKS_EINVAL, kBatchFailedMsg);
    for (sdugks_t *h : b->members)
        if (h->diverged) return fail(SDUGKS_EDIVERGED, "a batch member is not finite");
    if (n == 0) return SDUGKS_OK;
    HIPCHK(hipSetDevice(b->device));
    // a member stepped alone since the table was filled: refresh its buffer index
    for (size_t k = 0; k < b->members.size(); k++)
        if (b->members[k]->cur != b->cur_at_fill[k]) {
            int rc = batch_build(b);
            if (rc) return rc;
            break;
        }
    int rc = batch_join(b, true);
    if (rc) return rc;
    // whole runs of kGraphPairs pairs replay the longest graph, the remaining
    // pairs one graph per set bit (the runtime leaves a gap of several us
    // between two graph launches, so few launches matter for short calls),
    // the shortest first so that the device starts while the host submits
    // the longer ones; all lengths are captured together at the first call
    // that needs one
    int64_t pairs = n / 2;
    const int64_t runs = pairs / kGraphPairs;
    pairs -= runs * kGraphPairs;
    if (runs > 0 || pairs > 0)
        for (int k = 0; k < kBatchGraphs; k++)
            if (!b->exec[k] && (rc = batch_capture(b, (int64_t)1 << k, b->graph[k], b->exec[k]))) return rc;
    for (int k = 0; k <= kBatchGraphs - 2; k++)
        if (pairs & ((int64_t)1 << k)) HIPCHK(hipGraphLaunch(b->exec[k], b->stream));
    for (int64_t k = 0; k < runs; k++) HIPCHK(hipGraphLaunch(b->exec[kBatchGraphs - 1], b->stream));
    if (n & 1) {
        rc = batch_launch(b, 0);
        if (rc) return rc;
    }
    rc = batch_join(b, false);
    if (rc) return rc;
    for (sdugks_t *h : b->members) {
        h->cur ^= (int)(n & 1);
        h->step += n;
    }
    if (n & 1) return batch_build(b);          // every member's buffer index flipped
    return SDUGKS_OK;
}

int sdugks_batch_residual(sdugks_batch_t *b, double *eps)
{
    if (!b || !eps) return fail(SDUGKS_EINVAL, "null argument");
    if (b->failed) return fail(SDUGKS_EINVAL, kBatchFailedMsg);
    const int n = (int)b->members.size();
    if (n == 0) return SDUGKS_OK;
    HIPCHK(hipSetDevice(b->device));
    if (n > b->cap_jobs) {
        HIPCHK(hipStreamSynchronize(b->stream));
        (void)hipHostFree(b->h_jobs); (void)hipFree(b->d_jobs); (void)hipHostFree(b->h_out); (void)hipFree(b->d_out);
        b->h_jobs = nullptr; b->d_jobs = nullptr; b->h_out = nullptr; b->d_out = nullptr;
        b->cap_jobs = 0;
        const size_t cap = next_pow2((size_t)n);
        if (hipHostMalloc((void **)&b->h_jobs, cap * sizeof(ReduceJob), hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&b->d_jobs, cap * sizeof(ReduceJob)) != hipSuccess ||
            hipHostMalloc((void **)&b->h_out, cap * 4 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&b->d_out, cap * 4 * sizeof(double)) != hipSuccess)
            return fail(SDUGKS_ENOMEM, "allocation of the batched residual buffers failed");
        b->cap_jobs = (int)cap;
    }
    for (int k = 0; k < n; k++) {
        const sdugks_t *h = b->members[k];
        b->h_jobs[k] = ReduceJob{h->mb.nc, (int32_t)h->L.np, h->at<double>(h->L.off_W[h->cur]),
                                 h->at<double>(h->L.off_area), h->at<double>(h->L.off_snap),
                                 h->at<double>(h->L.off_part)};
    }
    int rc = batch_join(b, true);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(b->d_jobs, b->h_jobs, n * sizeof(ReduceJob), hipMemcpyHostToDevice, b->stream));
    HIPCHK(launch_reduce_batch(b->d_jobs, n, b->d_out, b->stream));
    HIPCHK(hipMemcpyAsync(b->h_out, b->d_out, n * 4 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    bool bad = false;
    for (int k = 0; k < n; k++) {
        const double *r = b->h_out + 4 * k;
        if (r[3] != 0.0) {
            b->members[k]->diverged = true;
            eps[k] = NAN;
            bad = true;
        } else {
            eps[k] = r[1] > 0 ? std::sqrt(r[0]) / std::sqrt(r[1]) : INFINITY;
        }
    }
    return bad ? fail(SDUGKS_EDIVERGED, "non-finite density or velocity in a batch member (its residual is NaN)")
               : SDUGKS_OK;
}

int sdugks_residuals_static(sdugks_t *const *members, int32_t n, double *eps)
{
    if (!members || !eps || n <= 0) return fail(SDUGKS_EINVAL, "bad arguments");
    if (n > kNoAllocMaxMembers)
        return fail(SDUGKS_EINVAL, "sdugks_residuals_static takes at most " + std::to_string(kNoAllocMaxMembers) +
                                       " members");
    for (int32_t k = 0; k < n; k++) {
        if (!members[k]) return fail(SDUGKS_EINVAL, "null member");
        if (members[k]->stream != members[0]->stream || members[k]->device != members[0]->device)
            return fail(SDUGKS_EINVAL, "sdugks_residuals_static: all members must share one device and one stream");
        for (int32_t j = 0; j < k; j++)
            if (members[j] == members[k]) return fail(SDUGKS_EINVAL, "a handle appears twice");
    }
    const int dev = members[0]->device;
    hipStream_t st = members[0]->stream;
    HIPCHK(hipSetDevice(dev));
    double *out = nullptr;
    HIPCHK(noalloc_scratch(dev, &out));
    // the job table on the stack: it is copied into the kernel arguments
    ReduceJob jobs[kNoAllocPack];
    for (int32_t k0 = 0; k0 < n; k0 += kNoAllocPack) {
        const int m = std::min<int32_t>(kNoAllocPack, n - k0);
        for (int k = 0; k < m; k++) {
            const sdugks_t *h = members[k0 + k];
            jobs[k] = ReduceJob{h->mb.nc, (int32_t)h->L.np, h->at<double>(h->L.off_W[h->cur]),
                                h->at<double>(h->L.off_area), h->at<double>(h->L.off_snap),
                                h->at<double>(h->L.off_part)};
        }
        HIPCHK(launch_reduce_packs(jobs, m, out + 4 * (size_t)k0, st));
    }
    double res[4 * kNoAllocMaxMembers];
    HIPCHK(hipMemcpyAsync(res, out, (size_t)n * 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool bad = false;
    for (int32_t k = 0; k < n; k++) {
        const double *r = res + 4 * k;
        if (r[3] != 0.0) {
            members[k]->diverged = true;
            eps[k] = NAN;
            bad = true;
        } else {
            eps[k] = r[1] > 0 ? std::sqrt(r[0]) / std::sqrt(r[1]) : INFINITY;
        }
    }
    return bad ? fail(SDUGKS_EDIVERGED, "non-finite density or velocity in a member (its residual is NaN)")
               : SDUGKS_OK;
}

int sdugks_debug_batch_fail(sdugks_batch_t *b)
{
    if (!b) return fail(SDUGKS_EINVAL, "null batch");
    b->fail_next_build = true;
    return SDUGKS_OK;
}

int sdugks_batch_destroy(sdugks_batch_t *b)
{
    if (!b) return SDUGKS_OK;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    (void)hipHostFree(b->h_jobs);
    (void)hipFree(b->d_jobs);
    (void)hipHostFree(b->h_out);
    (void)hipFree(b->d_out);
    batch_release_graph(b);
    batch_release_groups(b);
    if (b->ev) (void)hipEventDestroy(b->ev);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return SDUGKS_OK;
}

}  // extern "C"
