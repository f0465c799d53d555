/*
 * sdugks.h -- C ABI of the MI355X (gfx950) sDUGKS solver library, libsdugks.so.
 *
 * The library advances the D2Q9 BGK distribution of a 2-D finite-volume mesh
 * with the simplified discrete unified gas kinetic scheme of Zhong et al.,
 * "A simplified discrete unified gas kinetic scheme for incompressible flow"
 * (arXiv:2007.07347).  The problem it solves is the one stated in Section II:
 * given control volumes V_j, boundary conditions (Section III), a relaxation
 * time (or viscosity) and a time step, march f, rho and u from t_n to t_{n+1}
 * by the eleven-step summary at the end of Section II, until the velocity
 * residual of the lid-driven cavity case (Section IV) falls below a tolerance.
 *
 * Conventions for every call:
 *  - Return value: 0 (SDUGKS_OK) or a negative SDUGKS_E* code.  Nothing throws
 *    across the ABI.  sdugks_last_error() returns a thread-local message for
 *    the last failing call of the calling thread.
 *  - Ownership: inputs are copied; the caller may free them when the call
 *    returns.  A handle owns the device memory it allocates; with a caller
 *    workspace, the caller owns that memory and must keep it alive and
 *    untouched until sdugks_destroy.
 *  - Cell order: every per-cell array crossing the ABI is in the caller's cell
 *    order (the order of mesh.cell_ptr), whatever internal reordering is used.
 *  - Layout: per-cell arrays are row-major, cell-major: f[n_cells][9] in the
 *    D2Q9 order (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1),
 *    W[n_cells][3] = (rho, rho*u, rho*v).  All host pointers unless stated.
 *  - Streams: device work is enqueued on the hipStream_t given at creation
 *    (NULL = the null stream).  sdugks_step is asynchronous; calls that return
 *    host data synchronise that stream first.
 *  - Threads: one handle must not be used by two threads at once.
 *  - Step forms: the fused step (one kernel per time step over tiles of at
 *    most 64 cells of triangles and quads) and, on tensor-product quad meshes,
 *    the structured step run every precision form, both schemes and the
 *    batched calls.  Meshes with polygons of more than four faces (or more
 *    than 64 boundary-condition entries, or tile_cells = -1) take the
 *    two-kernel step instead, which is limited: FP64 only, the simplified
 *    scheme only, no batching (SDUGKS_EINVAL otherwise), and it writes fbar+
 *    and its gradient to device memory, 432 B per cell per step more.
 */
#ifndef SDUGKS_H
#define SDUGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SDUGKS_OK = 0,
    SDUGKS_EINVAL = -1,     /* bad argument or invalid mesh */
    SDUGKS_ENOMEM = -2,     /* host or device allocation failed, or workspace too small */
    SDUGKS_EHIP = -3,       /* a HIP runtime call failed (message names it) */
    SDUGKS_EDIVERGED = -4,  /* a non-finite density or velocity was found; the handle refuses to step */
    SDUGKS_ENODEV = -5      /* no gfx950 device usable */
};

/* Boundary-condition types, Section III.  WALL: rho from the adjacent cell,
 * u = wall velocity.  INLET: (rho_inf, u_inf).  OUTLET: rho and u of the
 * adjacent cell.  SYMMETRY: rho of the adjacent cell and its velocity without
 * the normal component, u_in - (u_in . N) N (the mean of the cell and its
 * mirror image about the boundary); the tag's edges must lie on one straight
 * line (u, v of the entry are ignored).  These four build the boundary
 * distribution by non-equilibrium extrapolation,
 * f_b = feq(rho_b, u_b) + (f_in - feq_in), and use it for the velocities with
 * e_i . N < 0 (N outward).  PERIODIC: the tag's edges are glued to the partner
 * tag's edges shifted by (shift_x, shift_y). */
enum { SDUGKS_BC_WALL = 1, SDUGKS_BC_INLET = 2, SDUGKS_BC_OUTLET = 3, SDUGKS_BC_PERIODIC = 4, SDUGKS_BC_SYMMETRY = 5 };

/* Precision of f.  FP64: stored and computed in FP64.  FP32DEV: stored in
 * FP32 as the deviation f - w_i rho0 and advected in FP32 (fbar+, gradients,
 * face values and fluxes; per-cell flux sums compensated in the general
 * step, in FP64 in the structured step), with density,
 * momentum, their update, the macroscopic flux, mass and residual in FP64;
 * the rounding of its FP32 arithmetic (fbar+, gradients and face pass
 * alike) keeps the velocity residual from falling below a few 1e-8 on fine
 * meshes.  FP32NEQ: the non-equilibrium
 * part f - feq(rho, u) stored in FP32 (half the bytes of FP64 f), every
 * operation of the step in FP64; converges like FP64. */
enum { SDUGKS_FP64 = 0, SDUGKS_FP32DEV = 1, SDUGKS_FP32NEQ = 2 };

/* Time level of the macroscopic flux of Eq. (MacroFlux) used by
 * Eq. (MacroUpdate): this step's face fluxes (CURRENT, default) or the previous
 * step's (LAGGED; stable only for dt below about 3 tau). */
enum { SDUGKS_MACRO_LAGGED = 0, SDUGKS_MACRO_CURRENT = 1 };

/* SIMPLIFIED: the paper's step (Section II summary).  ORIGINAL: the discrete
 * unified gas kinetic scheme it simplifies, for comparison -- faces at half a
 * step (h = dt/2, reconstruction at x_f - e_i h, f_face = 2tau/(2tau+h)
 * (fbar + h/(2tau) feq_f)), the cell variable ft = f - (dt/2) Omega and the
 * explicit update ft^{n+1} = (4/3) fbar+ - (1/3) ft - dt/V F.  f crossing the
 * ABI is always f.  ORIGINAL needs the fused step and the CURRENT flux. */
enum { SDUGKS_SCHEME_SIMPLIFIED = 0, SDUGKS_SCHEME_ORIGINAL = 1 };

/* Raw mesh: polygons of 3..8 nodes, counter-clockwise.  Every edge of a cell
 * that no other cell shares must appear once in bedge_nodes (either order). */
typedef struct {
    int32_t n_nodes;
    const double *node_xy;        /* [n_nodes][2] */
    int32_t n_cells;
    const int32_t *cell_ptr;      /* [n_cells + 1] offsets into cell_nodes */
    const int32_t *cell_nodes;    /* [cell_ptr[n_cells]] node ids */
    int32_t n_bedges;
    const int32_t *bedge_nodes;   /* [n_bedges][2] */
    const int32_t *bedge_tag;     /* [n_bedges] index into the sdugks_bc table */
} sdugks_mesh;

typedef struct {
    int32_t type;                 /* SDUGKS_BC_* */
    int32_t partner;              /* PERIODIC: tag of the partner side */
    double rho, u, v;             /* INLET: rho_inf, u_inf; WALL: u, v = wall velocity */
    double shift_x, shift_y;      /* PERIODIC: this side + shift = partner side */
} sdugks_bc;

typedef struct {
    double nu;                    /* kinematic viscosity; tau = nu / c_s^2 = 3 nu */
    double tau;                   /* relaxation time; > 0 overrides nu */
    double cfl;                   /* dt = cfl * h_min / sqrt(2) (h_j = 2 * min centroid-to-face distance) */
    double dt;                    /* > 0 overrides cfl */
    double rho0, u0, v0;          /* initial uniform equilibrium; rho0 is also the offset of FP32 storage */
    int32_t precision;            /* SDUGKS_FP64, SDUGKS_FP32DEV or SDUGKS_FP32NEQ */
    int32_t macro_flux;           /* SDUGKS_MACRO_CURRENT (default) or SDUGKS_MACRO_LAGGED */
    int32_t reorder;              /* two-kernel step: 1 = reverse Cuthill-McKee cell order inside the
                                     library (the fused step orders cells tile by tile instead) */
    int32_t residual_interval;    /* steps between residual checks in serving loops (paper: 1000) */
    int32_t tile_cells;           /* fused one-kernel step over tiles of at most this many cells
                                     (0 = library default, -1 = two-kernel step without tiles; meshes with
                                     polygons of more than four faces or more than 64 boundary-condition
                                     entries always take the two-kernel step) */
    int32_t block_threads;        /* threads per workgroup of the fused step: 64, 128 or 256 (0 = default) */
    int32_t scheme;               /* SDUGKS_SCHEME_SIMPLIFIED (default) or SDUGKS_SCHEME_ORIGINAL */
    int32_t structured;           /* structured step for tensor-product quad meshes (the cells are the
                                     rectangles of two coordinate arrays; periodic sides glued row to row
                                     or column to column; at most 2^29 - 4096 cells): 0 = used when the
                                     mesh is one and tile_cells is 0, 1 = never, 2 = required
                                     (SDUGKS_EINVAL otherwise).  It fixes
                                     its own tiles (16 x 14 cells on 512 threads for FP32DEV, 16 x 7 cells on
                                     256 threads otherwise) and ignores block_threads */
} sdugks_params;

typedef struct sdugks_s sdugks_t;

/* Host-only mesh build, no device needed.  Outputs may be NULL.  dt, tau: the
 * values sdugks_create would use; h_min: min_j h_j; n_faces: faces after
 * periodic gluing; area, cx, cy: [n_cells] cell area and centroid in the
 * caller's order; perm: [n_cells], perm[k] = caller index of the k-th cell in
 * the library's internal order. */
int sdugks_geometry(const sdugks_mesh *mesh, const sdugks_bc *bc, int32_t n_bc, const sdugks_params *prm,
                    double *dt, double *tau, double *h_min, int32_t *n_faces,
                    double *area, double *cx, double *cy, int32_t *perm);

/* Host-only: how the fused step would tile this mesh.  tile_cells: the tile
 * size used (0 when the two-kernel step is used: polygons with more than four
 * faces, or tile_cells = -1); n_tiles; max_local: largest tile plus both halo
 * rings; max_ring1: largest tile plus its first ring; structured: 1 when the
 * structured step is used (its tiles are 16 x 14 cells for FP32DEV, 16 x 7 otherwise).  Outputs
 * may be NULL. */
int sdugks_tiling(const sdugks_mesh *mesh, const sdugks_bc *bc, int32_t n_bc, const sdugks_params *prm,
                  int32_t *tile_cells, int32_t *n_tiles, int32_t *max_local, int32_t *max_ring1,
                  int32_t *structured);

/* Device bytes a handle for this problem needs (all state, geometry and
 * scratch); the size of a caller workspace.  Host only. */
int sdugks_state_bytes(const sdugks_mesh *mesh, const sdugks_bc *bc, int32_t n_bc, const sdugks_params *prm,
                       size_t *bytes);

/* Build the mesh, upload it, and set f = feq(rho0, u0, v0), W = (rho0, rho0 u0,
 * rho0 v0), G = 0 on the current HIP device.  stream: a hipStream_t or NULL.
 * workspace: device memory of at least sdugks_state_bytes bytes, 256-byte
 * aligned, or NULL for the library to allocate. */
int sdugks_create(const sdugks_mesh *mesh, const sdugks_bc *bc, int32_t n_bc, const sdugks_params *prm,
                  void *stream, void *workspace, size_t workspace_bytes, sdugks_t **out);

/* Advance n >= 0 time steps (asynchronous).  Fails with SDUGKS_EDIVERGED once a
 * residual, mass or state call has seen a non-finite value.  Pairs of steps
 * are replayed from hipGraphs built on first use (32 steps per replay, then
 * 2; an odd last step is launched alone), node by node rather than by stream
 * capture, and launched on the handle's stream, which may be the null stream.
 * Results are bitwise those of sdugks_step_eager. */
int sdugks_step(sdugks_t *h, int64_t n);

/* The same n steps with one plain kernel launch each (no graph): for callers
 * that capture their own graph around the library, or time single launches. */
int sdugks_step_eager(sdugks_t *h, int64_t n);

/* rho, u, v: [n_cells] host arrays (any may be NULL).  Synchronises. */
int sdugks_macros(sdugks_t *h, double *rho, double *u, double *v);

/* Full state: f [n_cells][9], W [n_cells][3], G [n_cells][3] (the stored
 * macroscopic flux of the lagged mode; zeros otherwise).  Any may be NULL.
 * With FP32 storage f is returned as w_i rho0 + (stored deviation) for FP32DEV
 * and as feq(W) + (stored non-equilibrium part) for FP32NEQ; set_state stores
 * f minus the same reference (FP32NEQ: feq of the W given, else of the
 * stored W). */
int sdugks_get_state(sdugks_t *h, double *f, double *W, double *G);
int sdugks_set_state(sdugks_t *h, const double *f, const double *W, const double *G);

/* Equilibrium state from macroscopic fields: f_i = feq_i(rho, u, v) on the
 * device (the second-order discrete form of Eq. Feq, whose moments are rho
 * and rho u, Eq. Macro), W = (rho, rho u, rho v), G = 0, and the residual
 * snapshot = the velocity (rho u) / rho of that W.  rho, u, v: host arrays [n_cells] in the caller's order,
 * rho > 0 and all finite (SDUGKS_EINVAL otherwise, state untouched).  With the
 * original scheme the stored f~ of an equilibrium is f itself.  Clears the
 * diverged flag.  Synchronises. */
int sdugks_set_macros(sdugks_t *h, const double *rho, const double *u, const double *v);

/* eps = sqrt(sum_j |u_j - u_j^snap|^2) / sqrt(sum_j |u_j^snap|^2) over cells
 * (unweighted), the residual of the paper's cavity case, against the snapshot
 * taken by the previous call (or at create / set_state), then re-snapshots.
 * +inf when the snapshot is all zero.  Deterministic FP64 reduction.
 * Returns SDUGKS_EDIVERGED if any rho or u is not finite.  Synchronises. */
int sdugks_residual(sdugks_t *h, double *eps);

/* mass = sum_j V_j rho_j, deterministic FP64 reduction.  Synchronises. */
int sdugks_mass(sdugks_t *h, double *mass);

/* Fluxes through the plain (not periodic) boundary faces on the current state:
 * the face distribution of Eq. f_t_n+1 (with the boundary rule of Section III)
 * and its flux moments (1, e_x, e_y) of Eqs. MesoFlux / MacroFlux, with the
 * face normal pointing out of the fluid -- so the two momentum fluxes through a
 * wall are the force the fluid exerts on it (drag and lift of the circular
 * cylinder case are these, summed over its wall).  FP64 arithmetic.
 *   faces   host [n_faces][4] or NULL: per face mass flux, x-momentum flux,
 *           y-momentum flux and face density rho_f (pressure rho_f / 3), in
 *           the caller's order of its non-periodic boundary edges;
 *   sum     host [3] or NULL: the three fluxes summed over the faces whose
 *           boundary tag is `tag` (all faces when tag < 0), deterministic;
 *   n_faces host or NULL: number of plain boundary faces.
 * SDUGKS_EINVAL for a tag beyond the boundary-condition table.  Synchronises. */
int sdugks_boundary_flux(sdugks_t *h, int32_t tag, double *faces, double *sum, int32_t *n_faces);

/* Any output may be NULL. */
int sdugks_info(sdugks_t *h, double *dt, double *tau, int64_t *step, int32_t *n_cells);

/* Average device duration (milliseconds) of each kernel of the step over the
 * next n steps, measured with HIP events on the handle's stream around every
 * launch (slower than sdugks_step; for profiling).  names: optional array of
 * max_kernels const char* receiving static kernel names.  *n_kernels: count. */
int sdugks_step_profiled(sdugks_t *h, int64_t n, double *avg_ms, const char **names, int32_t max_kernels,
                         int32_t *n_kernels);

int sdugks_destroy(sdugks_t *h);

const char *sdugks_last_error(void);

/* ---- batched form: many independent instances (uneven meshes, their own tau,
 * dt and boundary tables) advanced by one launch per step over the tiles of
 * all members; members with three-slot and four-slot cells, or with the two
 * storage forms, go to separate launches.  Each XCD takes an equal,
 * contiguous share of the concatenated tile sequence.  Steps are replayed
 * from hipGraphs built node by node (one of 32 steps, one of 2 for the rest;
 * no stream capture, so other threads may allocate meanwhile) that read
 * a device-side table (members, and each tile slot's member and local tile),
 * so changing the membership only rewrites the table unless the tile count
 * or the LDS a member needs outgrows what the launch was built with (it is
 * then rebuilt).
 *  - members: handles using the fused step (n >= 1, no duplicates, same
 *    device); they keep their own state and stay usable individually, and the
 *    batch does not own them: destroy the batch (or change its membership)
 *    before destroying a member.
 *  - stream: a hipStream_t that is not the null stream, or NULL for the batch
 *    to create its own; the batch orders itself after each member's stream
 *    before stepping and each member's stream after itself afterwards.
 * Results are bitwise those of stepping each member alone. */
typedef struct sdugks_batch_s sdugks_batch_t;
int sdugks_batch_create(sdugks_t *const *members, int32_t n, void *stream, sdugks_batch_t **out);
/* Replace the membership (continuous batching): waits for the batch stream.
 * If the new members pass the checks but the device tables cannot be
 * allocated (SDUGKS_ENOMEM) or filled (SDUGKS_EHIP), the batch is left with
 * no members and marked failed: sdugks_batch_step and sdugks_batch_residual
 * then return SDUGKS_EINVAL until a later sdugks_batch_set_members succeeds.
 * The same holds for the table refresh inside sdugks_batch_step. */
int sdugks_batch_set_members(sdugks_batch_t *b, sdugks_t *const *members, int32_t n);
/* Advance every member n >= 0 time steps (asynchronous on the batch stream),
 * one launch per step and step form (structured or general, precision).
 * Pairs of steps are replayed from hipGraphs of 2, 4, 8, 16 and 32 steps,
 * all built at the first call that needs one (again after a membership
 * change that rebuilds the launch): one graph per set bit of the pairs
 * left over after whole runs of 32 steps, the shortest first, then the runs;
 * an odd last step is launched alone.  SDUGKS_EDIVERGED
 * when a member has been seen non-finite; SDUGKS_EINVAL for n < 0 or a
 * failed batch. */
int sdugks_batch_step(sdugks_batch_t *b, int64_t n);

/* Residual of every member (the definition of sdugks_residual, each against
 * its own snapshot, then re-snapshotted) in one batched reduction launch and
 * one synchronisation; bitwise the values sdugks_residual would return.
 * eps: host [n members] in member order.  A member with a non-finite density
 * or velocity gets NaN, refuses further steps, and the call returns
 * SDUGKS_EDIVERGED after filling every entry. */
int sdugks_batch_residual(sdugks_batch_t *b, double *eps);
int sdugks_batch_destroy(sdugks_batch_t *b);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * residuals of sdugks_batch_residual for up to 1024 handles without a batch
 * object and without any allocation -- no hipMalloc, hipFree, events or
 * streams are created; the per-member results go through one file-scope
 * device array of 32 KiB (1024 x 4 doubles), held by each device the library
 * runs on until the process ends, and the job table travels in the kernel
 * arguments.  Same values, bitwise, as sdugks_residual and
 * sdugks_batch_residual (each member re-snapshotted).
 *   members: n distinct handles, 1 <= n <= 1024 (SDUGKS_EINVAL beyond), all
 *            on one device and created with the same stream, on which the
 *            work is enqueued (the call then synchronises that stream);
 *   eps:     host [n], filled as sdugks_batch_residual does (NaN and
 *            SDUGKS_EDIVERGED for a non-finite member).
 * Every call on a device shares that device's array: calls that overlap on
 * one device (from two threads, or on two streams) race and must not be made. */
int sdugks_residuals_static(sdugks_t *const *members, int32_t n, double *eps);

/* Failure injection for tests: writes NaN into f of one cell and velocity
 * (caller cell order). */
int sdugks_debug_poison(sdugks_t *h, int32_t cell, int32_t i);
/* Failure injection for tests: the batch's next table rebuild fails with
 * SDUGKS_ENOMEM (nothing is allocated). */
int sdugks_debug_batch_fail(sdugks_batch_t *b);

#ifdef __cplusplus
}
#endif
#endif
