/*
 * dugks2p_oracle.h -- plain FP64 CPU oracle of the two-phase DUGKS time step
 * (Zhang, Yang & Guo, "A discrete unified gas-kinetic scheme for immiscible
 * two-phase flows", arXiv:1802.02868).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU baseline leg of the benchmark can check the HIP path
 * against an independent, slow, obviously-staged implementation.  Nothing in
 * the product library links, includes or calls it, and it shares no code,
 * header, table or constant generator with the product.
 *
 * Every array is FP64, host memory, row-major [ny][nx] with x fastest.
 * Populations are stored [18][ny][nx]: q = 0..8 is f~ (pressure/momentum
 * population, Sec. 2.2), q = 9..17 is g~ (order-parameter population).
 * D2Q9 order (eq. D2Q9): 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1)
 * 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1), all times c = sqrt(3 RT).
 */
#ifndef DUGKS2P_ORACLE_H
#define DUGKS2P_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_PERIODIC = 0, ORC_BC_WALL = 1 };
enum { ORC_RECON_CENTRAL = 0, ORC_RECON_UPWIND = 1 };

typedef struct {
  int nx, ny;
  const double *x_faces; /* nx+1 strictly increasing face coordinates */
  const double *y_faces; /* ny+1 */
  int bc_x, bc_y;        /* ORC_BC_* per axis */
  int recon;             /* ORC_RECON_* */
  int phi_clamp;         /* clamp phi into [phi_b, phi_a] inside rho() and mu_d() */
  double cfl, c_max;     /* dt = cfl * min spacing / c_max (eq. cfl); c_max <= 0 -> sqrt(6 RT) */
  double dt;             /* > 0: explicit time step (cfl ignored) */
  double rt;             /* RT = c_s^2 */
  double tau_g;          /* relaxation time of g */
  double mobility;       /* lambda; eta = lambda / (c_s^2 tau_g), eq. kineticandmobility */
  double tau_f;          /* > 0: uniform tau_f; else tau_f = mu_d(phi) / (rho c_s^2) */
  double beta, kappa;
  double phi_a, phi_b, rho_a, rho_b, nu_a, nu_b;
  double gx, gy, rho_ref; /* body force (rho - rho_ref) g */
} orc_params;

typedef struct orc_sim orc_sim;

/* Returns NULL on invalid parameters (message via orc_last_error). */
orc_sim *orc_create(const orc_params *p, const double *phi0, const double *ux0,
                    const double *uy0, const double *p0);
void orc_destroy(orc_sim *s);
const char *orc_last_error(void);

double orc_dt(const orc_sim *s);
long orc_step_count(const orc_sim *s);
void orc_step(orc_sim *s, long nsteps);

/* Cell macroscopic fields at the current time (Step 7); any pointer may be NULL. */
void orc_moments(orc_sim *s, double *phi, double *rho, double *ux, double *uy, double *p,
                 double *mu);
/* out[0..5] = M_phi, E_k, E_free, max|u|, non-finite population count, step */
void orc_monitors(orc_sim *s, double out[6]);

void orc_get_pops(const orc_sim *s, double *out);   /* [18][ny][nx] */
void orc_set_pops(orc_sim *s, const double *in);    /* [18][ny][nx] */

/* ---- pieces exposed for the pins in tests/ ------------------------------ */

/* Cell equilibria and sources at one point (eqs. feq, geq, su, Hi, F, G).
 * in[13] = phi, rho, ux, uy, p, mu, drho_x, drho_y, D, Fx, Fy, dp_x, dp_y
 * (D = div(lambda grad mu)); outputs are 9 values each. */
void orc_point_eq(const orc_sim *s, const double in[13], double feq[9], double geq[9],
                  double ff[9], double fg[9]);

/* App. B first/second derivative of a cell field along one axis
 * (axis 0 = x, 1 = y) with the boundary rule of that axis. */
void orc_deriv(const orc_sim *s, int axis, const double *field, double *d1, double *d2);

/* The cell transforms of Step 2 for the current state: bar+ and tilde+ [18][ny][nx]. */
void orc_cell_transforms(orc_sim *s, double *barp, double *tilp);

/* Step 3 alone: half-step face populations bar(x_b, t+h) from a given bar+ field
 * [18][ny][nx].  xface[18][ny][nfx], yface[18][nfy][nx] with nfx = nx+1 and
 * nfy = ny+1 (face k is the low face of cell k; for a periodic axis face n
 * repeats face 0).  Wall faces use the wall rule. */
void orc_reconstruct(const orc_sim *s, const double *barp, double *xface, double *yface);

/* The face operator of R5 (value, normal derivative, tangential derivative
 * of a cell field at every face; the tangential derivative from the App. B
 * first-derivative stencil along the face) applied to a given cell field F
 * [ny][nx].  Layout as orc_reconstruct: x faces [ny][nx+1], y faces
 * [ny+1][nx]. */
void orc_face_fields(const orc_sim *s, const double *F, double *xv, double *xdn, double *xdt,
                     double *yv, double *ydn, double *ydt);

/* Step 4 face distributions phi(x_b, t+h) of the current state, same layout. */
void orc_face_dists(orc_sim *s, double *xface, double *yface);

#ifdef __cplusplus
}
#endif
#endif
