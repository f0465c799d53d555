/*
 * sdugks_oracle.h -- plain FP64 CPU oracle of one sDUGKS time step (D2Q9).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The solver library
 * never includes, links or calls it, and it shares no code with the solver.
 *
 * What it computes follows Zhong et al., "A simplified discrete unified gas
 * kinetic scheme for incompressible flow" (arXiv:2007.07347), Section II
 * (Eqs. Integration, fn+1, bar_eq_plus, fbar, fbar1, fbarplus, fbpsource, the
 * LLSR normal equations, MacroFlux, MacroUpdate, f_t_n+1, MesoFlux and the
 * eleven-step summary) and Section III (wall, inlet, outlet, periodic
 * boundary conditions).  Readings where the paper is silent are listed in the
 * source file header.
 *
 * All arrays are row-major, cell-major: f[n_cells][9], W[n_cells][3]
 * (rho, rho*u, rho*v), G[n_cells][3]; cells in the caller's order.
 */
#ifndef SDUGKS_ORACLE_H
#define SDUGKS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_case orc_case;

enum { ORC_WALL = 1, ORC_INLET = 2, ORC_OUTLET = 3, ORC_PERIODIC = 4, ORC_SYMMETRY = 5 };
enum { ORC_LAGGED = 0, ORC_CURRENT = 1 };     /* time level of the macroscopic flux */
enum { ORC_ASSEMBLED = 0, ORC_BRUTE = 1 };    /* assembly mode */
enum { ORC_SDUGKS = 0, ORC_DUGKS = 1 };       /* the paper's simplified step, or the original half-step scheme */

/* prm: {nu, tau, cfl, dt, rho0, u0, v0}; nu or tau > 0 (tau wins), dt > 0 overrides cfl.
 * iprm: {macro_mode, assembly_mode, scheme}.
 * bc_val: per BC {rho, u, v, shift_x, shift_y}.
 * Returns NULL on error, with a message in err (256 bytes). */
orc_case *orc_create(int n_nodes, const double *node_xy, int n_cells, const int *cell_ptr,
                     const int *cell_nodes, int n_bedges, const int *bedge_nodes, const int *bedge_tag,
                     int n_bc, const int *bc_type, const double *bc_val, const int *bc_partner,
                     const double *prm, const int *iprm, char *err);
void orc_free(orc_case *o);

/* dout: {dt, tau, h_min, a, b, c1, lambda}; iout: {n_cells, n_faces, n_boundary_faces, n_singular} */
void orc_info(const orc_case *o, double *dout, int *iout);
void orc_geometry(const orc_case *o, double *area, double *cx, double *cy, double *h);
/* faces: owner, neighbour (-1 = boundary), bc index (-1 = plain interior), scaled normal
 * (l*n), midpoint, translation t (neighbour image = x_nbr - t). */
void orc_faces(const orc_case *o, int *owner, int *nbr, int *bcid, double *lnx, double *lny,
               double *xm, double *ym, double *tx, double *ty);

void orc_set_state(orc_case *o, const double *f, const double *W, const double *G);
void orc_get_state(const orc_case *o, double *f, double *W, double *G);
void orc_step(orc_case *o, int n);
/* threads of the per-cell / per-face loops (results independent of it) */
void orc_set_threads(int n);
int orc_max_threads(void);
/* relative L2 change of (U, V) since the last call (or creation), then re-snapshot */
double orc_residual(orc_case *o);
double orc_mass(const orc_case *o);

/* Pins and probes. */
void orc_feq(double rho, double ux, double uy, double *out9);
/* least-squares gradient of an arbitrary cell field (bfield: its values at the
 * boundary face midpoints, indexed by face), both ways:
 * mode 0 = precomputed weights, 1 = normal equations solved by Cramer's rule. */
void orc_lsq_gradient(const orc_case *o, const double *field, const double *bfield, double *grad, int mode);
/* face states of the current state without advancing: fbar[n_faces][9] (the
 * reconstructed transformed distribution), fface[n_faces][9] (the face
 * distribution at t_{n+1}), phi[n_faces][9] (l * (e_i . n) * fface). */
void orc_face_states(const orc_case *o, double *fbar, double *fface, double *phi);

#ifdef __cplusplus
}
#endif
#endif
