// Device-side data of one solver instance and the launchers of its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <tuple>
#include <vector>
#include <utility>

namespace sdg {

struct DevBC {
    int32_t type;
    double rho, u, v;
};

// Mesh and constants of one instance, as seen by the kernels.  All per-cell
// arrays are pitched: entry (row r, cell c) at r*np + c.
struct DevMesh {
    int32_t nc, np, D, n_bfaces, n_bc;
    const int32_t *nbr;                 // [D][np]
    // two-kernel step only (the fused step reads per-tile face records):
    const double2 *ln;                  // [D][np] scaled outward normal (x, y)
    const double2 *rs;                  // [D][np] midpoint - own centroid
    const double2 *ro;                  // [D][np] midpoint image - neighbour centroid
    const double *ainv;                 // [3][np] inverse LSQ normal matrix
    const double *dtv;                  // [np] dt / V
    const double *area;                 // [np]
    const int32_t *bf_tag;              // [n_bfaces]
    const DevBC *bcs;                   // [n_bc]
    double a, b, c1, lam, dt;           // (2tau-dt)/2tau, dt/2tau, 2tau/(2tau+dt), dt/tau, dt
    double inv1l;                       // 1 / (1 + dt/tau)
    // face step: reconstruction time, and the coefficients of the face
    // distribution f_face = fc1 (fbar + fb feq_f); (dt, b, c1) for the paper's
    // scheme, (dt/2, dt/4tau, 2tau/(2tau+dt/2)) for the original one
    double dtr, fb, fc1;
    int32_t scheme;                     // 0 the paper's scheme, 1 the original one
    double rho0;                        // offset of the deviation form: f = w_i rho0 + stored value
};

// State buffers of one step: read (in) and write (out).  f is FP64 ([9][np]
// doubles) or, in the deviation form, f - w_i rho0 in FP32 (f32 / fo32).
struct DevState {
    const double *f, *W, *G;            // [9][np], [3][np], [3][np]
    double *fo, *Wo, *Go;
    const float *f32;
    float *fo32;
};

// Tiles of the fused step (see MeshBuild): headers [n_tiles][8] (g0, nt, n1,
// n2), the padded per-tile tables lgid [PL], ladj [D][PA], lfc [D][PT] and the
// face records [3][PF] (rows l n, r_self, r_other of (x, y) pairs) and the
// least-squares weights lw [D][PA] ((x, y) pairs), with PL = nl_max,
// PA = na_max, PT = nt_max, PF = nf_max.
struct DevTiles {
    int32_t n_tiles, nl_max, na_max, nt_max, nf_max;
    const int32_t *hdr;
    const int32_t *lgid;
    const int16_t *ladj;
    const int16_t *lfc;
    const double2 *fr, *lw;             // FP64 form
    const float2 *fr32, *lw32;          // deviation form
};

// Structured step (tensor-product quad meshes): grid and tile counts,
// periodic flags, per-column / per-row records [n][kCartVals] and the
// boundary-condition entry of every boundary face of the four sides (bottom
// [nx], top [nx], left [ny], right [ny]; -1 on periodic sides).
struct DevCart {
    int32_t nx, ny, ntx, nty, per_x, per_y;
    const double *col, *row;
    const int32_t *side;
};

// One member of a batched launch: its mesh, tiles (or structured grid), both
// ping-pong buffers and the buffer index it reads at parity 0.
struct BatchInst {
    DevMesh m;
    DevTiles t;
    DevCart c;
    void *f[2];
    double *W[2];
    double *G[2];
    int32_t parity0, lagged;
};

// Device-side batch table: the members, and for every tile slot of the
// launch grid its member and the tile's index inside that member (member -1
// for the slots past the live tiles).
struct BatchTable {
    const BatchInst *inst;
    const int2 *tmap;
};

// Plain boundary faces for the face-flux diagnostic, in the caller's order of
// its non-periodic boundary edges: the adjacent cell, the face's slot and tag,
// the cell's least-squares stencil (neighbour >= 0, -2 - tag for a boundary
// point, -1 empty) with its weights, and the face's scaled normal l n and
// midpoint offset r_self.  out [n][4]: mass flux, x- and y-momentum flux
// leaving the fluid, face density; sum [3]: the fluxes summed over one tag.
struct DevBnd {
    int32_t n;
    const int4 *hdr;                    // [n]: cell, slot, tag, 0
    const int32_t *nb;                  // [n][D]
    const double2 *w;                   // [n][D]
    const double2 *geo;                 // [n][2]: l n, r_self
    double *out;
    double *sum;
};

struct DevScratch {
    double *fbp;                        // [9][np] fbar+ at the cell centres
    double *sg;                         // [18][np] its least-squares gradient (x rows 0..8, y rows 9..17)
};

// Where a step launcher puts its kernels: on its stream, or, given a chain,
// as the next nodes of a graph under construction (each node depending on the
// previous one).  Graphs are built node by node rather than by stream
// capture, so that another thread's allocations or synchronous copies can
// never invalidate them.
// Kernel nodes appended to a graph.  A node depends on `deps` (the previous
// node, or every node of the previous fan); between begin_fan and end_fan the
// nodes are collected instead, all depending on the same `deps`, so they may
// run concurrently, and end_fan makes the next node wait for all of them.
struct GraphChain {
    hipGraph_t graph = nullptr;
    std::vector<hipGraphNode_t> deps;
    std::vector<hipGraphNode_t> fan;
    bool fanning = false;
    void begin_fan() { fan.clear(); fanning = true; }
    void end_fan()
    {
        fanning = false;
        if (!fan.empty()) deps.swap(fan);
        fan.clear();
    }
};

template <typename Tup, size_t... I>
inline void kernel_arg_ptrs(Tup &t, void **p, std::index_sequence<I...>)
{
    ((p[I] = (void *)&std::get<I>(t)), ...);
}

// Launch fn<<<grid, blk, lds, st>>>(args...), or append it to the chain.
template <typename... P, typename... A>
inline hipError_t emit(void (*fn)(P...), dim3 grid, dim3 blk, size_t lds, hipStream_t st, GraphChain *gc,
                       A &&...args)
{
    std::tuple<P...> vals(std::forward<A>(args)...);
    void *ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1];
    kernel_arg_ptrs(vals, ptrs, std::index_sequence_for<P...>{});
    if (!gc) return hipLaunchKernel(reinterpret_cast<const void *>(fn), grid, blk, ptrs, lds, st);
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void *>(fn);
    kp.gridDim = grid;
    kp.blockDim = blk;
    kp.sharedMemBytes = (unsigned)lds;
    kp.kernelParams = ptrs;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    const hipError_t e = hipGraphAddKernelNode(&node, gc->graph, gc->deps.empty() ? nullptr : gc->deps.data(),
                                               gc->deps.size(), &kp);
    if (e != hipSuccess) return e;
    if (gc->fanning) gc->fan.push_back(node);
    else gc->deps.assign(1, node);
    return e;
}

// Launchers (stream-ordered, no synchronisation).  Return the hipError_t of the launch.
hipError_t launch_grad(const DevMesh &m, const DevState &s, const DevScratch &x, hipStream_t st,
                       GraphChain *gc = nullptr);
hipError_t launch_flux_update(const DevMesh &m, const DevState &s, const DevScratch &x, int lagged, hipStream_t st,
                              GraphChain *gc = nullptr);
// Fused one-kernel step over tiles (D <= 4 slots per cell).
// mode: 0 FP64; 1 FP32 storage of f - w_i rho0, FP32 face arithmetic; 2 FP32
// storage of f - feq(W), FP64 arithmetic.
hipError_t launch_step_tiled(const DevMesh &m, const DevTiles &t, const DevState &s, int lagged, int mode,
                             int block, hipStream_t st, GraphChain *gc = nullptr);
size_t step_tiled_lds_bytes(const DevTiles &t, int mode, int n_bc);
// Structured step over the tiles of a tensor-product quad mesh (one
// workgroup per tile: 16 x 14 cells on 512 threads for FP32 deviations, 16 x 7
// on 256 threads otherwise), and its batched form (members of one mode on the
// structured step).
hipError_t launch_step_cart(const DevMesh &m, const DevCart &c, const DevState &s, int lagged, int mode,
                            hipStream_t st, GraphChain *gc = nullptr);
size_t step_cart_lds_bytes(int mode, int n_bc);
int step_cart_threads(int mode);
hipError_t launch_step_batch_cart(const BatchTable &tab, int mode, int parity, int cap_tiles, size_t lds,
                                  hipStream_t st, GraphChain *gc = nullptr);
// Batched fused step over the tiles of all members (same D class and mode).
hipError_t launch_step_batch(const BatchTable &tab, int D, int mode, int parity, int cap_tiles, size_t lds,
                             int block, hipStream_t st, GraphChain *gc = nullptr);
// Deterministic reductions of the residual / mass / finiteness check: writes
// out4 = {sum |u-u_snap|^2, sum |u_snap|^2, sum V rho, count of non-finite}.
// snap = [2][np] (U, V); update_snap re-snapshots.
hipError_t launch_reduce(const DevMesh &m, const double *W, double *snap, int update_snap, double *partials,
                         double *out4, hipStream_t st);
// Boundary face fluxes on the state s (mode: the storage of f, as for the
// step), then their sums over the faces of `tag` (all when tag < 0).
hipError_t launch_boundary_flux(const DevMesh &m, const DevState &s, const DevBnd &q, int mode, int tag, hipStream_t st);
// One member of a batched residual: its cells, current W, areas, snapshot
// (re-snapshotted) and its own partial sums.
struct ReduceJob {
    int32_t nc, np;
    const double *W;
    const double *area;
    double *snap;
    double *partials;
};
// Residuals of n members at once: out [n][4] as launch_reduce's out4 each.
hipError_t launch_reduce_batch(const ReduceJob *jobs, int n, double *out, hipStream_t st);
// Residuals of n members without any allocation: the per-member results
// [n][4] go to the file-scope scratch array of noalloc.hip (at most
// kNoAllocMaxMembers members), the job table travels in the kernel arguments
// (kNoAllocPack members per launch).
constexpr int kNoAllocMaxMembers = 1024;
constexpr int kNoAllocPack = 32;
constexpr int kNoAllocMaxDevices = 64;
struct ReducePack {
    ReduceJob jobs[kNoAllocPack];
};
// The device address of this device's scratch array ([kNoAllocMaxMembers][4]
// doubles), looked up once per device.
hipError_t noalloc_scratch(int device, double **out);
hipError_t launch_reduce_packs(const ReduceJob *jobs, int n, double *out, hipStream_t st);
// f = feq of the macros m3 = [3][np] (rho, u, v) (FP64 f, or with f32 the
// FP32 deviation from w_i rho0, or zero -- the non-equilibrium part -- when
// rho0 < 0), W, G = 0 and the residual snapshot.
hipError_t launch_set_equilibrium(int nc, int np, const double *m3, double *f, float *f32, double rho0, double *W,
                                  double *G, double *snap, hipStream_t st);
// *p = NaN, p pointing at a double (bytes 8) or a float (bytes 4): failure injection.
hipError_t launch_poke_nan(void *p, int bytes, hipStream_t st);

constexpr int kReduceBlocks = 256;

}  // namespace sdg
