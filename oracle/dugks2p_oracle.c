/*
 * dugks2p_oracle.c -- plain FP64 CPU oracle of one time step of the two-phase
 * discrete unified gas-kinetic scheme (DUGKS) of Zhang, Yang & Guo
 * (arXiv:1802.02868), Sec. 2.2, "the procedure in one time step".
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline leg of bench.py.  The product library never links, includes or
 * calls this file.  It is written for a reader checking it against the paper:
 * every stage fills whole arrays before the next stage starts (no fusion, no
 * blocking), in the order of the paper's Steps 1-7.
 *
 * Where the paper is silent or garbled, the reading taken is stated at the
 * place it is used (the same readings are listed in the design notes):
 *   R1  c_s^2 = RT; xi_i = c e_i with c = sqrt(3 RT) (eq. D2Q9).
 *   R2  D2Q9 numbering 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1)
 *       6:(-1,1) 7:(-1,-1) 8:(1,-1) (eq. D2Q9), opposites 1-3, 2-4, 5-7, 6-8.
 *   R3  phi = sum g~ literally (eq. phi), not with the dt/2 sum of F^g
 *       (which vanishes analytically, eq. sumG).
 *   R4  face macros use bar-phi and h/2 (eq. conservedVariable with dt -> h,
 *       tilde -> bar; the sentence after eq. fbar_h states it reversed).
 *   R5  face values of mu, grad mu, grad phi, grad p and D come from the
 *       time-n cell fields through the face operator of step 3: distance-
 *       weighted value, two-point normal derivative, weighted tangential
 *       derivative (the paper is silent on them).
 *   R6  2-D derivatives are the App. B three-point formulas per axis.
 *   R7  walls: macro stencils use a mirror ghost (value of the wall cell,
 *       centre reflected across the wall); population gradients are one-sided
 *       at a wall cell; at a wall face the populations leaving the fluid and
 *       the tangential ones are expanded from the wall cell, the ones entering
 *       the fluid are the bounce-back of their opposites, before and after
 *       eq. original-function (the paper names bounce-back, gives no formula).
 *   R8  body force F_b = (rho - rho_ref) g (rising-bubble force form).
 *   R9  tau_f = mu_d(phi) / (rho c_s^2) at cells and faces (eqs.
 *       kineticandmobility, mixvis) unless a uniform tau_f is given.
 *   R10 UPWIND reconstruction (optional): expand from the upwind cell with its
 *       cell gradient; a direction tangential to the face uses CENTRAL.
 *
 * Values that depend on the state are of type `real`: double here, or
 * double _Complex when the file is compiled with ORC_COMPLEX_STEP for
 * complex-step differentiation (derivatives of the FP64 scheme to rounding,
 * used to check adjoints).  Mesh weights and the other parameters stay
 * double; kappa and the body force g are real so that they can be perturbed.
 */
#include "dugks2p_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_COMPLEX_STEP
#include <complex.h>
typedef double _Complex real;
#define RE(x) creal(x)
#else
typedef double real;
#define RE(x) (x)
#endif

/* R2 */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

static __thread char g_err[512];

static void set_err(const char *m) {
  snprintf(g_err, sizeof g_err, "%s", m);
}

const char *orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------ */
/* One mesh axis: faces, centres, App. B stencil weights, face weights.      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n, bc, nf; /* cells, boundary rule, stored faces (n periodic, n+1 wall) */
  double *f, *c, *w;
  double L;
  int *lo, *hi;       /* neighbour cell used by the stencils (wrap or mirror) */
  double *d1, *d2;    /* App. B weights (minus, centre, plus) per cell */
  double *pg;         /* population-gradient weights per cell */
  int *fl, *fr;       /* cells on the low / high side of face k, -1 = wall */
  double *fwl, *fwr, *finv, *foffl, *foffr;
  double *rdt;        /* dt / width */
} axis_t;

static void axis_free(axis_t *a) {
  free(a->f); free(a->c); free(a->w); free(a->lo); free(a->hi);
  free(a->d1); free(a->d2); free(a->pg); free(a->fl); free(a->fr);
  free(a->fwl); free(a->fwr); free(a->finv); free(a->foffl); free(a->foffr);
  free(a->rdt);
}

static int axis_init(axis_t *a, int n, int bc, const double *faces) {
  memset(a, 0, sizeof *a);
  a->n = n; a->bc = bc; a->nf = (bc == ORC_BC_PERIODIC) ? n : n + 1;
  a->f = malloc(sizeof(double) * (n + 1));
  a->c = malloc(sizeof(double) * n);
  a->w = malloc(sizeof(double) * n);
  a->lo = malloc(sizeof(int) * n);
  a->hi = malloc(sizeof(int) * n);
  a->d1 = malloc(sizeof(double) * 3 * n);
  a->d2 = malloc(sizeof(double) * 3 * n);
  a->pg = malloc(sizeof(double) * 3 * n);
  a->fl = malloc(sizeof(int) * (n + 1));
  a->fr = malloc(sizeof(int) * (n + 1));
  a->fwl = calloc(n + 1, sizeof(double));
  a->fwr = calloc(n + 1, sizeof(double));
  a->finv = calloc(n + 1, sizeof(double));
  a->foffl = calloc(n + 1, sizeof(double));
  a->foffr = calloc(n + 1, sizeof(double));
  a->rdt = malloc(sizeof(double) * n);
  if (!a->f || !a->c || !a->w || !a->lo || !a->hi || !a->d1 || !a->d2 || !a->pg ||
      !a->fl || !a->fr || !a->fwl || !a->fwr || !a->finv || !a->foffl || !a->foffr ||
      !a->rdt)
    return -1;
  memcpy(a->f, faces, sizeof(double) * (n + 1));
  for (int k = 0; k < n; ++k) {
    a->c[k] = 0.5 * (a->f[k] + a->f[k + 1]);
    a->w[k] = a->f[k + 1] - a->f[k];
  }
  a->L = a->f[n] - a->f[0];

  for (int k = 0; k < n; ++k) {
    int im, ip;
    double pm, pp;
    /* left neighbour: interior, periodic wrap, or mirror ghost across a wall */
    if (k > 0) { im = k - 1; pm = a->c[k - 1]; }
    else if (bc == ORC_BC_PERIODIC) { im = n - 1; pm = a->c[n - 1] - a->L; }
    else { im = k; pm = 2.0 * a->f[0] - a->c[0]; }
    if (k < n - 1) { ip = k + 1; pp = a->c[k + 1]; }
    else if (bc == ORC_BC_PERIODIC) { ip = 0; pp = a->c[0] + a->L; }
    else { ip = k; pp = 2.0 * a->f[n] - a->c[n - 1]; }
    a->lo[k] = im; a->hi[k] = ip;

    /* App. B, eqs. nonphi/nonphi2 with h_l = theta_l dx, h_r = theta_r dx:
     *   d1 = [h_l^2 F+ + (h_r^2 - h_l^2) F0 - h_r^2 F-] / [h_l h_r (h_l + h_r)]
     *   d2 = 2 [h_l F+ - (h_l + h_r) F0 + h_r F-]      / [h_l h_r (h_l + h_r)] */
    double hl = a->c[k] - pm, hr = pp - a->c[k];
    double hl2 = hl * hl, hr2 = hr * hr, den = hl * hr * (hl + hr);
    a->d1[3 * k + 0] = -hr2 / den;
    a->d1[3 * k + 1] = (hr2 - hl2) / den;
    a->d1[3 * k + 2] = hl2 / den;
    a->d2[3 * k + 0] = 2.0 * hr / den;
    a->d2[3 * k + 1] = -2.0 * (hl + hr) / den;
    a->d2[3 * k + 2] = 2.0 * hl / den;

    /* population gradient: App. B first derivative, one-sided at a wall (R7) */
    if (bc == ORC_BC_WALL && k == 0) {
      double inv = 1.0 / (a->c[1] - a->c[0]);
      a->pg[3 * k + 0] = 0.0; a->pg[3 * k + 1] = -inv; a->pg[3 * k + 2] = inv;
    } else if (bc == ORC_BC_WALL && k == n - 1) {
      double inv = 1.0 / (a->c[n - 1] - a->c[n - 2]);
      a->pg[3 * k + 0] = -inv; a->pg[3 * k + 1] = inv; a->pg[3 * k + 2] = 0.0;
    } else {
      a->pg[3 * k + 0] = a->d1[3 * k + 0];
      a->pg[3 * k + 1] = a->d1[3 * k + 1];
      a->pg[3 * k + 2] = a->d1[3 * k + 2];
    }
  }

  for (int k = 0; k < a->nf; ++k) {
    if (bc == ORC_BC_WALL && (k == 0 || k == n)) {
      a->fl[k] = (k == 0) ? -1 : n - 1;
      a->fr[k] = (k == 0) ? 0 : -1;
      if (k == 0) a->foffr[k] = a->f[0] - a->c[0];
      else a->foffl[k] = a->f[n] - a->c[n - 1];
      continue;
    }
    int il = (k == 0) ? n - 1 : k - 1;
    double xl = (k == 0) ? a->c[n - 1] - a->L : a->c[k - 1];
    double xr = a->c[k], xf = a->f[k];
    double d = xr - xl;
    a->fl[k] = il; a->fr[k] = k;
    a->fwl[k] = (xr - xf) / d;
    a->fwr[k] = (xf - xl) / d;
    a->finv[k] = 1.0 / d;
    a->foffl[k] = xf - xl;
    a->foffr[k] = xf - xr;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
struct orc_sim {
  orc_params P;
  axis_t ax[2];
  int nx, ny;
  long N, nstep;
  double dt, h, hdt, hh, cs2, c, eta, gam, inv_dphi, drho, mumu, c4b, phimid;
  double lo_phi, hi_phi, k1, k2, k3;
  double xi[9][2], w9[9];
  real kappa, gx, gy; /* the parameters of the same names */
  real *pop;
  /* cell work arrays (Steps 2 and 7) */
  real *phi, *rho, *mu, *dphx, *dphy, *dmux, *dmuy, *D, *Fx, *Fy, *ux, *uy, *p;
  real *dpx, *dpy, *tauf;
  real *barp, *tilp, *gbx, *gby;
  real *facex, *facey; /* 18 x ny x nfx, 18 x nfy x nx */
};

static void sim_free(orc_sim *s) {
  if (!s) return;
  axis_free(&s->ax[0]); axis_free(&s->ax[1]);
  free(s->pop); free(s->phi); free(s->rho); free(s->mu); free(s->dphx); free(s->dphy);
  free(s->dmux); free(s->dmuy); free(s->D); free(s->Fx); free(s->Fy); free(s->ux);
  free(s->uy); free(s->p); free(s->dpx); free(s->dpy); free(s->tauf);
  free(s->barp); free(s->tilp); free(s->gbx); free(s->gby); free(s->facex); free(s->facey);
  free(s);
}

void orc_destroy(orc_sim *s) { sim_free(s); }
double orc_dt(const orc_sim *s) { return s->dt; }
long orc_step_count(const orc_sim *s) { return s->nstep; }

/* eq. oderrho, with the optional clamp of phi inside rho() only */
static real clamp_phi(const orc_sim *s, real ph) {
  if (!s->P.phi_clamp) return ph;
  return RE(ph) < s->lo_phi ? s->lo_phi : (RE(ph) > s->hi_phi ? s->hi_phi : ph);
}

static real rho_of(const orc_sim *s, real phi) {
  const real ph = clamp_phi(s, phi);
  return ((ph - s->P.phi_b) * s->P.rho_a + (s->P.phi_a - ph) * s->P.rho_b) * s->inv_dphi;
}

/* eqs. kineticandmobility and mixvis: tau_f = mu_d / (rho c_s^2) (R9) */
static real tauf_of(const orc_sim *s, real phi, real rho) {
  if (s->P.tau_f > 0.0) return s->P.tau_f;
  const real ph = clamp_phi(s, phi);
  double mu_a = s->P.rho_a * s->P.nu_a, mu_b = s->P.rho_b * s->P.nu_b;
  real mud = s->mumu / ((ph - s->P.phi_b) * mu_b + (s->P.phi_a - ph) * mu_a);
  return mud / (rho * s->cs2);
}

/* Macroscopic state at one point, input of the equilibria and sources. */
typedef struct {
  real phi, rho, ux, uy, p, mu, grx, gry, D, Fx, Fy, gpx, gpy, icr;
} macro_t;

/* eqs. feq, geq, su, Hi, F, G at one point. */
static void point_eq(const orc_sim *s, const macro_t *m, real feq[9], real geq[9],
                     real ff[9], real fg[9]) {
  const double cs2 = s->cs2;
  const real uu = m->ux * m->ux + m->uy * m->uy;
  for (int i = 0; i < 9; ++i) {
    const double wi = s->w9[i], xx = s->xi[i][0], xy = s->xi[i][1];
    const real eu = xx * m->ux + xy * m->uy;
    /* eq. su: s_i = w_i [xi.u / cs2 + (xi.u)^2 / (2 cs2^2) - u^2 / (2 cs2)] */
    const real si = wi * (eu * s->k1 + eu * eu * s->k2 - uu * s->k3);
    /* eq. feq */
    feq[i] = wi * m->p + cs2 * m->rho * si;
    /* eqs. geq, Hi */
    const real Hi = (i == 0) ? m->phi - (1.0 - s->w9[0]) * s->eta * m->mu
                             : wi * s->eta * m->mu;
    geq[i] = Hi + m->phi * si;
    /* eqs. F, G with Gamma_i = w_i + s_i */
    const real G = wi + si;
    const real cx = xx - m->ux, cy = xy - m->uy;
    ff[i] = cx * (m->Fx * G + si * cs2 * m->grx) + cy * (m->Fy * G + si * cs2 * m->gry) -
            wi * cs2 * m->rho * s->gam * m->D;
    fg[i] = m->phi * m->icr * (cx * (m->Fx - m->gpx) + cy * (m->Fy - m->gpy)) * G;
  }
}

#ifndef ORC_COMPLEX_STEP
void orc_point_eq(const orc_sim *s, const double in[13], double feq[9], double geq[9],
                  double ff[9], double fg[9]) {
  macro_t m;
  m.phi = in[0]; m.rho = in[1]; m.ux = in[2]; m.uy = in[3]; m.p = in[4]; m.mu = in[5];
  m.grx = in[6]; m.gry = in[7]; m.D = in[8]; m.Fx = in[9]; m.Fy = in[10];
  m.gpx = in[11]; m.gpy = in[12];
  m.icr = 1.0 / (s->cs2 * m.rho);
  point_eq(s, &m, feq, geq, ff, fg);
}
#endif

/* Three-point stencil along x / y of a cell field, weights w (3 per cell). */
static real sx(const orc_sim *s, const double *w3, const real *F, int i, int j) {
  const axis_t *a = &s->ax[0];
  const double *w = w3 + 3 * i;
  const long r = (long)j * s->nx;
  return w[0] * F[r + a->lo[i]] + w[1] * F[r + i] + w[2] * F[r + a->hi[i]];
}
static real sy(const orc_sim *s, const double *w3, const real *F, int i, int j) {
  const axis_t *a = &s->ax[1];
  const double *w = w3 + 3 * j;
  return w[0] * F[(long)a->lo[j] * s->nx + i] + w[1] * F[(long)j * s->nx + i] +
         w[2] * F[(long)a->hi[j] * s->nx + i];
}

/* Steps 7 / 2 prerequisites: cell macroscopic fields from the state,
 * eqs. phi, oderrho, chemicalpotential, u, P in the order that each needs
 * the previous ones: phi -> rho -> mu -> grad mu, lap mu -> F -> u -> p -> grad p. */
static void cell_macros(orc_sim *s) {
  const int nx = s->nx, ny = s->ny;
  const long N = s->N;
  const real *f = s->pop, *g = s->pop + 9 * N;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    real acc = 0.0;
    for (int i = 0; i < 9; ++i) acc += g[i * N + c]; /* eq. phi, R3 */
    s->phi[c] = acc;
    s->rho[c] = rho_of(s, acc);
  }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const long c = (long)j * nx + i;
      const real ph = s->phi[c];
      const real lap = sx(s, s->ax[0].d2, s->phi, i, j) + sy(s, s->ax[1].d2, s->phi, i, j);
      /* eq. chemicalpotential */
      s->mu[c] = s->c4b * (ph - s->P.phi_a) * (ph - s->P.phi_b) * (ph - s->phimid) -
                 s->kappa * lap;
      s->dphx[c] = sx(s, s->ax[0].d1, s->phi, i, j);
      s->dphy[c] = sy(s, s->ax[1].d1, s->phi, i, j);
    }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const long c = (long)j * nx + i;
      s->dmux[c] = sx(s, s->ax[0].d1, s->mu, i, j);
      s->dmuy[c] = sy(s, s->ax[1].d1, s->mu, i, j);
      const real lapmu = sx(s, s->ax[0].d2, s->mu, i, j) + sy(s, s->ax[1].d2, s->mu, i, j);
      s->D[c] = s->P.mobility * lapmu; /* div(lambda grad mu), lambda constant */
      const real ph = s->phi[c], rh = s->rho[c];
      /* F = F_s + F_b, F_s = -phi grad mu (Sec. 2.1), F_b by R8 */
      s->Fx[c] = -ph * s->dmux[c] + (rh - s->P.rho_ref) * s->gx;
      s->Fy[c] = -ph * s->dmuy[c] + (rh - s->P.rho_ref) * s->gy;
      real s0 = 0.0, jx = 0.0, jy = 0.0;
      for (int i2 = 0; i2 < 9; ++i2) s0 += f[i2 * N + c];
      for (int i2 = 0; i2 < 9; ++i2) jx += s->xi[i2][0] * f[i2 * N + c];
      for (int i2 = 0; i2 < 9; ++i2) jy += s->xi[i2][1] * f[i2 * N + c];
      const real icr = 1.0 / (s->cs2 * rh);
      /* eq. u */
      s->ux[c] = (jx + s->hdt * s->cs2 * s->Fx[c]) * icr;
      s->uy[c] = (jy + s->hdt * s->cs2 * s->Fy[c]) * icr;
      /* eq. P, with grad rho = (rho_A - rho_B)/(phi_A - phi_B) grad phi */
      const real grx = s->drho * s->dphx[c], gry = s->drho * s->dphy[c];
      s->p[c] = s0 + s->hdt * s->cs2 * (s->ux[c] * grx + s->uy[c] * gry - s->gam * rh * s->D[c]);
    }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const long c = (long)j * nx + i;
      s->dpx[c] = sx(s, s->ax[0].d1, s->p, i, j);
      s->dpy[c] = sy(s, s->ax[1].d1, s->p, i, j);
      s->tauf[c] = tauf_of(s, s->phi[c], s->rho[c]);
    }
}

static void cell_macro_at(const orc_sim *s, long c, macro_t *m) {
  m->phi = s->phi[c]; m->rho = s->rho[c]; m->ux = s->ux[c]; m->uy = s->uy[c];
  m->p = s->p[c]; m->mu = s->mu[c];
  m->grx = s->drho * s->dphx[c]; m->gry = s->drho * s->dphy[c];
  m->D = s->D[c]; m->Fx = s->Fx[c]; m->Fy = s->Fy[c];
  m->gpx = s->dpx[c]; m->gpy = s->dpy[c];
  m->icr = 1.0 / (s->cs2 * m->rho);
}

/* Step 2: eqs. relations1 and relations2 in every cell. */
static void cell_transforms(orc_sim *s) {
  const long N = s->N;
  const double dt = s->dt, h = s->h;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    macro_t m;
    real feq[9], geq[9], ff[9], fg[9];
    cell_macro_at(s, c, &m);
    point_eq(s, &m, feq, geq, ff, fg);
    for (int half = 0; half < 2; ++half) {
      const real tau = half ? s->P.tau_g : s->tauf[c];
      const real den = 1.0 / (2.0 * tau + dt);
      const real ca = (2.0 * tau - h) * den; /* eq. relations1 */
      const real cb = 3.0 * h * den;
      const real cc = 3.0 * tau * h * den;
      const real *eq = half ? geq : feq, *src = half ? fg : ff;
      for (int i = 0; i < 9; ++i) {
        const long q = (long)(9 * half + i) * N + c;
        const real til = s->pop[q];
        const real bp = ca * til + cb * eq[i] + cc * src[i];
        s->barp[q] = bp;
        s->tilp[q] = (4.0 / 3.0) * bp - (1.0 / 3.0) * til; /* eq. relations2 */
      }
    }
  }
}

/* Cell gradients of bar+ for the face reconstruction (R6, R7). */
static void pop_gradients(const orc_sim *s, const real *barp, real *gbx, real *gby) {
  const int nx = s->nx, ny = s->ny;
  const long N = s->N;
#pragma omp parallel for schedule(static)
  for (int q = 0; q < 18; ++q)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const long c = (long)j * nx + i;
        gbx[q * N + c] = sx(s, s->ax[0].pg, barp + q * N, i, j);
        gby[q * N + c] = sy(s, s->ax[1].pg, barp + q * N, i, j);
      }
}

/* Step 3 at one face: bar(x_b, t+h) for the 18 populations (eqs. fbar, fbar_h).
 * a = axis normal to the face, k = face index along a, t = cell index along
 * the other axis. */
static void face_reconstruct(const orc_sim *s, const real *barp, const real *gbx,
                             const real *gby, int a, int k, int t, real bar[18]) {
  const axis_t *A = &s->ax[a];
  const long N = s->N;
  const double h = s->h;
  const real *gn = a == 0 ? gbx : gby, *gt = a == 0 ? gby : gbx;
  const int cl = A->fl[k], cr = A->fr[k];
#define CELL_ID(ia) (a == 0 ? (long)t * s->nx + (ia) : (long)(ia) * s->nx + t)
  if (cl < 0 || cr < 0) {
    /* wall face (R7): expand leaving and tangential populations from the
     * fluid cell C; the ones entering the fluid bounce back. */
    const int cc = cl < 0 ? cr : cl;
    const double off = cl < 0 ? A->foffr[k] : A->foffl[k];
    const int nout = cl < 0 ? -1 : 1; /* outward normal of C across the wall */
    const long C = CELL_ID(cc);
    for (int q = 0; q < 18; ++q) {
      const int i = q % 9;
      const int en = a == 0 ? EX[i] : EY[i];
      if (en * nout < 0) continue;
      const real Ac = barp[q * N + C], Gn = gn[q * N + C], Gt = gt[q * N + C];
      const real val = Ac + off * Gn;
      const real sgx = a == 0 ? Gn : Gt, sgy = a == 0 ? Gt : Gn;
      bar[q] = val - h * (s->xi[i][0] * sgx + s->xi[i][1] * sgy);
    }
    for (int q = 0; q < 18; ++q) {
      const int i = q % 9;
      const int en = a == 0 ? EX[i] : EY[i];
      if (en * nout < 0) bar[q] = bar[q - i + OPP[i]];
    }
    return;
  }
  const long L = CELL_ID(cl), R = CELL_ID(cr);
  const double wl = A->fwl[k], wr = A->fwr[k], inv = A->finv[k];
  for (int q = 0; q < 18; ++q) {
    const int i = q % 9;
    const int en = a == 0 ? EX[i] : EY[i];
    const real AL = barp[q * N + L], AR = barp[q * N + R];
    real val, sn, st;
    if (s->P.recon == ORC_RECON_UPWIND && en > 0) {
      val = AL + A->foffl[k] * gn[q * N + L];
      sn = gn[q * N + L];
      st = gt[q * N + L];
    } else if (s->P.recon == ORC_RECON_UPWIND && en < 0) {
      val = AR + A->foffr[k] * gn[q * N + R];
      sn = gn[q * N + R];
      st = gt[q * N + R];
    } else {
      /* Step 3: linear interpolation of bar+ and of its gradient */
      val = wl * AL + wr * AR;
      sn = (AR - AL) * inv;
      st = wl * gt[q * N + L] + wr * gt[q * N + R];
    }
    const real sgx = a == 0 ? sn : st, sgy = a == 0 ? st : sn;
    bar[q] = val - h * (s->xi[i][0] * sgx + s->xi[i][1] * sgy);
  }
#undef CELL_ID
}

/* R5: value, normal and tangential derivative of a cell field at a face. */
static void face_field(const orc_sim *s, int a, int k, int t, const real *F,
                       const real *Ft, real *v, real *dn, real *dtn) {
  const axis_t *A = &s->ax[a];
  const int cl = A->fl[k], cr = A->fr[k];
#define CELL_ID(ia) (a == 0 ? (long)t * s->nx + (ia) : (long)(ia) * s->nx + t)
  if (cl < 0 || cr < 0) {
    const long C = CELL_ID(cl < 0 ? cr : cl);
    *v = F[C];
    *dn = 0.0;
    *dtn = Ft[C];
    return;
  }
  const long L = CELL_ID(cl), R = CELL_ID(cr);
  *v = A->fwl[k] * F[L] + A->fwr[k] * F[R];
  *dn = (F[R] - F[L]) * A->finv[k];
  *dtn = A->fwl[k] * Ft[L] + A->fwr[k] * Ft[R];
#undef CELL_ID
}

/* Step 4 at one face: macros from bar (R4), equilibria and sources at the
 * face, then eq. original-function. */
static void face_dist(const orc_sim *s, int a, int k, int t, const real bar[18],
                      real out[18]) {
  const axis_t *A = &s->ax[a];
  const int is_wall = A->fl[k] < 0 || A->fr[k] < 0;
  const real *Tmu = a == 0 ? s->dmuy : s->dmux;
  const real *Tph = a == 0 ? s->dphy : s->dphx;
  const real *Tp = a == 0 ? s->dpy : s->dpx;
  real mu_b, D_b, tmp, gmn, gmt, gfn, gft, gpn, gpt;
  face_field(s, a, k, t, s->mu, Tmu, &mu_b, &gmn, &gmt);
  face_field(s, a, k, t, s->D, s->D, &D_b, &tmp, &tmp);
  face_field(s, a, k, t, s->phi, Tph, &tmp, &gfn, &gft);
  face_field(s, a, k, t, s->p, Tp, &tmp, &gpn, &gpt);
  const real gmx = a == 0 ? gmn : gmt, gmy = a == 0 ? gmt : gmn;
  const real gfx = a == 0 ? gfn : gft, gfy = a == 0 ? gft : gfn;
  const real gpx = a == 0 ? gpn : gpt, gpy = a == 0 ? gpt : gpn;

  macro_t m;
  real phib = 0.0;
  for (int i = 0; i < 9; ++i) phib += bar[9 + i];
  m.phi = phib;
  m.rho = rho_of(s, phib);
  m.mu = mu_b;
  m.D = D_b;
  m.grx = s->drho * gfx;
  m.gry = s->drho * gfy;
  m.gpx = gpx;
  m.gpy = gpy;
  m.Fx = -phib * gmx + (m.rho - s->P.rho_ref) * s->gx;
  m.Fy = -phib * gmy + (m.rho - s->P.rho_ref) * s->gy;
  m.icr = 1.0 / (s->cs2 * m.rho);
  real s0 = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < 9; ++i) s0 += bar[i];
  for (int i = 0; i < 9; ++i) jx += s->xi[i][0] * bar[i];
  for (int i = 0; i < 9; ++i) jy += s->xi[i][1] * bar[i];
  m.ux = (jx + s->hh * s->cs2 * m.Fx) * m.icr;
  m.uy = (jy + s->hh * s->cs2 * m.Fy) * m.icr;
  m.p = s0 + s->hh * s->cs2 * (m.ux * m.grx + m.uy * m.gry - s->gam * m.rho * m.D);

  real feq[9], geq[9], ff[9], fg[9];
  point_eq(s, &m, feq, geq, ff, fg);
  const double h = s->h;
  for (int half = 0; half < 2; ++half) {
    const real tau = half ? s->P.tau_g : tauf_of(s, phib, m.rho);
    const real den = 1.0 / (2.0 * tau + h);
    const real k1 = 2.0 * tau * den, k2 = h * den, k3 = tau * h * den;
    const real *eq = half ? geq : feq, *src = half ? fg : ff;
    for (int i = 0; i < 9; ++i)
      out[9 * half + i] = k1 * bar[9 * half + i] + k2 * eq[i] + k3 * src[i];
  }
  if (is_wall) {
    const int nout = A->fl[k] < 0 ? -1 : 1;
    for (int q = 0; q < 18; ++q) {
      const int i = q % 9;
      const int en = a == 0 ? EX[i] : EY[i];
      if (en * nout < 0) out[q] = out[q - i + OPP[i]];
    }
  }
}

static void all_faces(orc_sim *s) {
  const int nx = s->nx, ny = s->ny, nfx = s->ax[0].nf, nfy = s->ax[1].nf;
  const long NX = (long)ny * nfx, NY = (long)nfy * nx;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int k = 0; k < nfx; ++k) {
      real bar[18], out[18];
      face_reconstruct(s, s->barp, s->gbx, s->gby, 0, k, j, bar);
      face_dist(s, 0, k, j, bar, out);
      for (int q = 0; q < 18; ++q) s->facex[q * NX + (long)j * nfx + k] = out[q];
    }
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nfy; ++k)
    for (int i = 0; i < nx; ++i) {
      real bar[18], out[18];
      face_reconstruct(s, s->barp, s->gbx, s->gby, 1, k, i, bar);
      face_dist(s, 1, k, i, bar, out);
      for (int q = 0; q < 18; ++q) s->facey[q * NY + (long)k * nx + i] = out[q];
    }
}

/* Steps 5-6: eq. updatef with the flux of eq. microfluxf summed over the
 * W, E, S, N faces; for a rectangle (dt/|V|) sum (xi.n)|S| phi_b equals
 * (dt/dx) xi_x (phi_E - phi_W) + (dt/dy) xi_y (phi_N - phi_S). */
static void update(orc_sim *s) {
  const int nx = s->nx, ny = s->ny, nfx = s->ax[0].nf, nfy = s->ax[1].nf;
  const long N = s->N, NX = (long)ny * nfx, NY = (long)nfy * nx;
  const int perx = s->ax[0].bc == ORC_BC_PERIODIC, pery = s->ax[1].bc == ORC_BC_PERIODIC;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const long c = (long)j * nx + i;
      const int ie = (perx && i == nx - 1) ? 0 : i + 1;
      const int jn = (pery && j == ny - 1) ? 0 : j + 1;
      const double rx = s->ax[0].rdt[i], ry = s->ax[1].rdt[j];
      for (int q = 0; q < 18; ++q) {
        const int d = q % 9;
        const real W = s->facex[q * NX + (long)j * nfx + i];
        const real E = s->facex[q * NX + (long)j * nfx + ie];
        const real S = s->facey[q * NY + (long)j * nx + i];
        const real Nn = s->facey[q * NY + (long)jn * nx + i];
        s->pop[q * N + c] =
            s->tilp[q * N + c] - rx * s->xi[d][0] * (E - W) - ry * s->xi[d][1] * (Nn - S);
      }
    }
}

void orc_step(orc_sim *s, long nsteps) {
  for (long n = 0; n < nsteps; ++n) {
    cell_macros(s);                          /* Step 7 of the previous step */
    cell_transforms(s);                      /* Step 2 */
    pop_gradients(s, s->barp, s->gbx, s->gby);
    all_faces(s);                            /* Steps 3-4 */
    update(s);                               /* Steps 5-6 */
    s->nstep++;
  }
}

/* ------------------------------------------------------------------------ */
static int check_faces(const double *f, int n) {
  if (!f) return -1;
  for (int k = 0; k < n; ++k)
    if (!(f[k + 1] > f[k])) return -1;
  return 0;
}

/* Step 1 from phi0 (+ i h dphi0 in the complex-step build), u0, p0 with
 * kappa and g (+ i h dkappa, i h dg). */
static orc_sim *create(const orc_params *P, const double *phi0, const double *ux0,
                       const double *uy0, const double *p0, const double *dphi0,
                       double dkappa, double dgx, double dgy, double hcs) {
  if (!P || !phi0 || !ux0 || !uy0 || !p0) { set_err("null argument"); return NULL; }
  if (P->nx < 1 || P->ny < 1) { set_err("nx, ny must be >= 1"); return NULL; }
  if ((P->bc_x != ORC_BC_PERIODIC && P->bc_x != ORC_BC_WALL) ||
      (P->bc_y != ORC_BC_PERIODIC && P->bc_y != ORC_BC_WALL)) {
    set_err("bad boundary code"); return NULL;
  }
  if ((P->bc_x == ORC_BC_WALL && P->nx < 2) || (P->bc_y == ORC_BC_WALL && P->ny < 2)) {
    set_err("a wall axis needs at least 2 cells"); return NULL;
  }
  if (check_faces(P->x_faces, P->nx) || check_faces(P->y_faces, P->ny)) {
    set_err("faces must be strictly increasing"); return NULL;
  }
  if (!(P->rt > 0.0) || !(P->tau_g > 0.0) || !(P->mobility >= 0.0) || P->phi_a == P->phi_b ||
      !(P->rho_a > 0.0) || !(P->rho_b > 0.0)) {
    set_err("bad physical parameter"); return NULL;
  }
  if (!(P->tau_f > 0.0) && !(P->nu_a > 0.0 && P->nu_b > 0.0)) {
    set_err("need tau_f > 0 or nu_a, nu_b > 0"); return NULL;
  }
  if (!(P->dt > 0.0) && !(P->cfl > 0.0)) { set_err("need dt > 0 or cfl > 0"); return NULL; }
  if (P->recon != ORC_RECON_CENTRAL && P->recon != ORC_RECON_UPWIND) {
    set_err("bad recon"); return NULL;
  }

  orc_sim *s = calloc(1, sizeof *s);
  if (!s) { set_err("out of memory"); return NULL; }
  s->P = *P;
  s->kappa = P->kappa;
  s->gx = P->gx;
  s->gy = P->gy;
#ifdef ORC_COMPLEX_STEP
  s->kappa += I * hcs * dkappa;
  s->gx += I * hcs * dgx;
  s->gy += I * hcs * dgy;
#else
  (void)dphi0; (void)dkappa; (void)dgx; (void)dgy; (void)hcs;
#endif
  s->nx = P->nx; s->ny = P->ny; s->N = (long)P->nx * P->ny;
  if (axis_init(&s->ax[0], P->nx, P->bc_x, P->x_faces) ||
      axis_init(&s->ax[1], P->ny, P->bc_y, P->y_faces)) {
    set_err("out of memory"); sim_free(s); return NULL;
  }
  s->P.x_faces = s->ax[0].f; s->P.y_faces = s->ax[1].f;

  /* eq. cfl: dt = alpha dx_min / C_max, C_max = sqrt(6 RT) unless given */
  if (P->dt > 0.0) {
    s->dt = P->dt;
  } else {
    double dxmin = s->ax[0].w[0];
    for (int k = 0; k < P->nx; ++k) if (s->ax[0].w[k] < dxmin) dxmin = s->ax[0].w[k];
    for (int k = 0; k < P->ny; ++k) if (s->ax[1].w[k] < dxmin) dxmin = s->ax[1].w[k];
    const double cmax = P->c_max > 0.0 ? P->c_max : sqrt(6.0 * P->rt);
    s->dt = P->cfl * dxmin / cmax;
  }
  s->h = 0.5 * s->dt;
  s->hdt = 0.5 * s->dt;
  s->hh = 0.5 * s->h;
  for (int a = 0; a < 2; ++a)
    for (int k = 0; k < s->ax[a].n; ++k) s->ax[a].rdt[k] = s->dt / s->ax[a].w[k];

  s->cs2 = P->rt;
  s->c = sqrt(3.0 * P->rt);
  s->k1 = 1.0 / s->cs2;
  s->k2 = 1.0 / (2.0 * s->cs2 * s->cs2);
  s->k3 = 1.0 / (2.0 * s->cs2);
  s->eta = P->mobility / (s->cs2 * P->tau_g);      /* eq. kineticandmobility */
  const double rr = P->rho_a / P->rho_b;
  s->gam = (rr - 1.0) / (P->phi_a - P->phi_b * rr); /* eq. Gama */
  s->inv_dphi = 1.0 / (P->phi_a - P->phi_b);
  s->drho = (P->rho_a - P->rho_b) * s->inv_dphi;
  s->mumu = (P->rho_a * P->nu_a) * (P->rho_b * P->nu_b) * (P->phi_a - P->phi_b);
  s->c4b = 4.0 * P->beta;
  s->phimid = 0.5 * (P->phi_a + P->phi_b);
  s->lo_phi = P->phi_a < P->phi_b ? P->phi_a : P->phi_b;
  s->hi_phi = P->phi_a < P->phi_b ? P->phi_b : P->phi_a;
  for (int i = 0; i < 9; ++i) {
    s->xi[i][0] = EX[i] * s->c;
    s->xi[i][1] = EY[i] * s->c;
    s->w9[i] = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }

  const long N = s->N;
  const long NX = (long)P->ny * s->ax[0].nf, NY = (long)s->ax[1].nf * P->nx;
  real **cells[] = {&s->phi, &s->rho, &s->mu, &s->dphx, &s->dphy, &s->dmux, &s->dmuy,
                    &s->D, &s->Fx, &s->Fy, &s->ux, &s->uy, &s->p, &s->dpx, &s->dpy,
                    &s->tauf};
  for (size_t k = 0; k < sizeof cells / sizeof cells[0]; ++k) {
    *cells[k] = calloc(N, sizeof(real));
    if (!*cells[k]) { set_err("out of memory"); sim_free(s); return NULL; }
  }
  s->pop = calloc(18 * N, sizeof(real));
  s->barp = calloc(18 * N, sizeof(real));
  s->tilp = calloc(18 * N, sizeof(real));
  s->gbx = calloc(18 * N, sizeof(real));
  s->gby = calloc(18 * N, sizeof(real));
  s->facex = calloc(18 * NX, sizeof(real));
  s->facey = calloc(18 * NY, sizeof(real));
  if (!s->pop || !s->barp || !s->tilp || !s->gbx || !s->gby || !s->facex || !s->facey) {
    set_err("out of memory"); sim_free(s); return NULL;
  }

  /* Step 1: phi0, u0, p0 -> the fields the equilibria need, with p and u
   * given rather than taken from populations; then f = f^eq, g = g^eq and
   * eq. auxf(a) gives tilde = eq - (dt/2) F. */
  const int nx = P->nx, ny = P->ny;
  for (long c = 0; c < N; ++c) {
    s->phi[c] = phi0[c];
#ifdef ORC_COMPLEX_STEP
    if (dphi0) s->phi[c] += I * hcs * dphi0[c];
#endif
    s->ux[c] = ux0[c];
    s->uy[c] = uy0[c];
    s->p[c] = p0[c];
  }
  for (long c = 0; c < N; ++c) s->rho[c] = rho_of(s, s->phi[c]);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const long c = (long)j * nx + i;
      const real ph = s->phi[c];
      const real lap = sx(s, s->ax[0].d2, s->phi, i, j) + sy(s, s->ax[1].d2, s->phi, i, j);
      s->mu[c] = s->c4b * (ph - P->phi_a) * (ph - P->phi_b) * (ph - s->phimid) - s->kappa * lap;
      s->dphx[c] = sx(s, s->ax[0].d1, s->phi, i, j);
      s->dphy[c] = sy(s, s->ax[1].d1, s->phi, i, j);
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const long c = (long)j * nx + i;
      s->dmux[c] = sx(s, s->ax[0].d1, s->mu, i, j);
      s->dmuy[c] = sy(s, s->ax[1].d1, s->mu, i, j);
      const real lapmu = sx(s, s->ax[0].d2, s->mu, i, j) + sy(s, s->ax[1].d2, s->mu, i, j);
      s->D[c] = P->mobility * lapmu;
      s->Fx[c] = -s->phi[c] * s->dmux[c] + (s->rho[c] - P->rho_ref) * s->gx;
      s->Fy[c] = -s->phi[c] * s->dmuy[c] + (s->rho[c] - P->rho_ref) * s->gy;
      s->dpx[c] = sx(s, s->ax[0].d1, s->p, i, j);
      s->dpy[c] = sy(s, s->ax[1].d1, s->p, i, j);
    }
  for (long c = 0; c < N; ++c) {
    macro_t m;
    real feq[9], geq[9], ff[9], fg[9];
    cell_macro_at(s, c, &m);
    point_eq(s, &m, feq, geq, ff, fg);
    for (int i = 0; i < 9; ++i) {
      s->pop[(long)i * N + c] = feq[i] - s->hdt * ff[i];
      s->pop[(long)(9 + i) * N + c] = geq[i] - s->hdt * fg[i];
    }
  }
  return s;
}

#ifdef ORC_COMPLEX_STEP
orc_sim *orc_cs_create(const orc_params *P, const double *phi0, const double *ux0,
                       const double *uy0, const double *p0, const double *dphi0,
                       double dkappa, double dgx, double dgy, double h) {
  return create(P, phi0, ux0, uy0, p0, dphi0, dkappa, dgx, dgy, h);
}

void orc_cs_get_pops(const orc_sim *s, double *re, double *im) {
  for (long k = 0; k < 18 * s->N; ++k) {
    re[k] = creal(s->pop[k]);
    im[k] = cimag(s->pop[k]);
  }
}
#else
orc_sim *orc_create(const orc_params *P, const double *phi0, const double *ux0,
                    const double *uy0, const double *p0) {
  return create(P, phi0, ux0, uy0, p0, NULL, 0.0, 0.0, 0.0, 0.0);
}

void orc_moments(orc_sim *s, double *phi, double *rho, double *ux, double *uy, double *p,
                 double *mu) {
  cell_macros(s);
  const size_t b = sizeof(double) * s->N;
  if (phi) memcpy(phi, s->phi, b);
  if (rho) memcpy(rho, s->rho, b);
  if (ux) memcpy(ux, s->ux, b);
  if (uy) memcpy(uy, s->uy, b);
  if (p) memcpy(p, s->p, b);
  if (mu) memcpy(mu, s->mu, b);
}

/* Neumaier-compensated running sum */
typedef struct { double s, c; } ksum_t;
static void kadd(ksum_t *k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
  else k->c += (x - t) + k->s;
  k->s = t;
}

void orc_monitors(orc_sim *s, double out[6]) {
  cell_macros(s);
  ksum_t M = {0, 0}, Ek = {0, 0}, Ef = {0, 0};
  double umax = 0.0, bad = 0.0;
  for (int j = 0; j < s->ny; ++j)
    for (int i = 0; i < s->nx; ++i) {
      const long c = (long)j * s->nx + i;
      const double V = s->ax[0].w[i] * s->ax[1].w[j];
      const double ph = s->phi[c];
      const double u2 = s->ux[c] * s->ux[c] + s->uy[c] * s->uy[c];
      /* eq. doublewell and eq. freeenergyfunction */
      const double a1 = ph - s->P.phi_a, b1 = ph - s->P.phi_b;
      const double psi = s->P.beta * a1 * a1 * b1 * b1;
      const double g2 = s->dphx[c] * s->dphx[c] + s->dphy[c] * s->dphy[c];
      kadd(&M, ph * V);
      kadd(&Ek, 0.5 * s->rho[c] * u2 * V);
      kadd(&Ef, (psi + 0.5 * s->P.kappa * g2) * V);
      const double um = sqrt(u2);
      if (um > umax) umax = um;
    }
  for (long k = 0; k < 18 * s->N; ++k)
    if (!isfinite(s->pop[k])) bad += 1.0;
  out[0] = M.s + M.c;
  out[1] = Ek.s + Ek.c;
  out[2] = Ef.s + Ef.c;
  out[3] = umax;
  out[4] = bad;
  out[5] = (double)s->nstep;
}

void orc_get_pops(const orc_sim *s, double *out) {
  memcpy(out, s->pop, sizeof(double) * 18 * s->N);
}
void orc_set_pops(orc_sim *s, const double *in) {
  memcpy(s->pop, in, sizeof(double) * 18 * s->N);
}

void orc_deriv(const orc_sim *s, int axis, const double *field, double *d1, double *d2) {
  for (int j = 0; j < s->ny; ++j)
    for (int i = 0; i < s->nx; ++i) {
      const long c = (long)j * s->nx + i;
      if (axis == 0) {
        if (d1) d1[c] = sx(s, s->ax[0].d1, field, i, j);
        if (d2) d2[c] = sx(s, s->ax[0].d2, field, i, j);
      } else {
        if (d1) d1[c] = sy(s, s->ax[1].d1, field, i, j);
        if (d2) d2[c] = sy(s, s->ax[1].d2, field, i, j);
      }
    }
}

void orc_cell_transforms(orc_sim *s, double *barp, double *tilp) {
  cell_macros(s);
  cell_transforms(s);
  if (barp) memcpy(barp, s->barp, sizeof(double) * 18 * s->N);
  if (tilp) memcpy(tilp, s->tilp, sizeof(double) * 18 * s->N);
}

static void copy_faces_out(const orc_sim *s, const double *fx, const double *fy,
                           double *xface, double *yface) {
  const int nx = s->nx, ny = s->ny, nfx = s->ax[0].nf, nfy = s->ax[1].nf;
  const long NX = (long)ny * nfx, NY = (long)nfy * nx;
  const long OX = (long)ny * (nx + 1), OY = (long)(ny + 1) * nx;
  for (int q = 0; q < 18; ++q) {
    for (int j = 0; j < ny; ++j)
      for (int k = 0; k <= nx; ++k) {
        const int kk = k < nfx ? k : 0; /* periodic: face nx repeats face 0 */
        xface[q * OX + (long)j * (nx + 1) + k] = fx[q * NX + (long)j * nfx + kk];
      }
    for (int k = 0; k <= ny; ++k)
      for (int i = 0; i < nx; ++i) {
        const int kk = k < nfy ? k : 0;
        yface[q * OY + (long)k * nx + i] = fy[q * NY + (long)kk * nx + i];
      }
  }
}

void orc_reconstruct(const orc_sim *s, const double *barp, double *xface, double *yface) {
  const int nx = s->nx, ny = s->ny, nfx = s->ax[0].nf, nfy = s->ax[1].nf;
  const long N = s->N, NX = (long)ny * nfx, NY = (long)nfy * nx;
  double *gx = malloc(sizeof(double) * 18 * N), *gy = malloc(sizeof(double) * 18 * N);
  double *fx = malloc(sizeof(double) * 18 * NX), *fy = malloc(sizeof(double) * 18 * NY);
  if (!gx || !gy || !fx || !fy) { free(gx); free(gy); free(fx); free(fy); return; }
  pop_gradients(s, barp, gx, gy);
  double bar[18];
  for (int j = 0; j < ny; ++j)
    for (int k = 0; k < nfx; ++k) {
      face_reconstruct(s, barp, gx, gy, 0, k, j, bar);
      for (int q = 0; q < 18; ++q) fx[q * NX + (long)j * nfx + k] = bar[q];
    }
  for (int k = 0; k < nfy; ++k)
    for (int i = 0; i < nx; ++i) {
      face_reconstruct(s, barp, gx, gy, 1, k, i, bar);
      for (int q = 0; q < 18; ++q) fy[q * NY + (long)k * nx + i] = bar[q];
    }
  copy_faces_out(s, fx, fy, xface, yface);
  free(gx); free(gy); free(fx); free(fy);
}

/* R5 alone: the face operator applied to a given cell field F, with the
 * tangential derivative taken by the App. B first-derivative stencil of the
 * tangential axis, exactly as Step 4 feeds mu, phi and p to it. */
void orc_face_fields(const orc_sim *s, const double *F, double *xv, double *xdn, double *xdt,
                     double *yv, double *ydn, double *ydt) {
  const int nx = s->nx, ny = s->ny, nfx = s->ax[0].nf, nfy = s->ax[1].nf;
  const long N = s->N, NX = (long)ny * nfx, NY = (long)nfy * nx;
  double *dfx = malloc(sizeof(double) * N), *dfy = malloc(sizeof(double) * N);
  double *fx = malloc(sizeof(double) * 18 * NX), *fy = malloc(sizeof(double) * 18 * NY);
  double *ox = malloc(sizeof(double) * 18 * (long)ny * (nx + 1));
  double *oy = malloc(sizeof(double) * 18 * (long)(ny + 1) * nx);
  if (!dfx || !dfy || !fx || !fy || !ox || !oy) {
    free(dfx); free(dfy); free(fx); free(fy); free(ox); free(oy);
    return;
  }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      dfx[(long)j * nx + i] = sx(s, s->ax[0].d1, F, i, j);
      dfy[(long)j * nx + i] = sy(s, s->ax[1].d1, F, i, j);
    }
  /* planes 0..2 of the face layout carry value, normal and tangential
   * derivative; copy_faces_out then maps the stored faces to nx+1 / ny+1 */
  memset(fx, 0, sizeof(double) * 18 * NX);
  memset(fy, 0, sizeof(double) * 18 * NY);
  for (int j = 0; j < ny; ++j)
    for (int k = 0; k < nfx; ++k) {
      const long o = (long)j * nfx + k;
      face_field(s, 0, k, j, F, dfy, &fx[o], &fx[NX + o], &fx[2 * NX + o]);
    }
  for (int k = 0; k < nfy; ++k)
    for (int i = 0; i < nx; ++i) {
      const long o = (long)k * nx + i;
      face_field(s, 1, k, i, F, dfx, &fy[o], &fy[NY + o], &fy[2 * NY + o]);
    }
  copy_faces_out(s, fx, fy, ox, oy);
  const long OX = (long)ny * (nx + 1), OY = (long)(ny + 1) * nx;
  memcpy(xv, ox, sizeof(double) * OX);
  memcpy(xdn, ox + OX, sizeof(double) * OX);
  memcpy(xdt, ox + 2 * OX, sizeof(double) * OX);
  memcpy(yv, oy, sizeof(double) * OY);
  memcpy(ydn, oy + OY, sizeof(double) * OY);
  memcpy(ydt, oy + 2 * OY, sizeof(double) * OY);
  free(dfx); free(dfy); free(fx); free(fy); free(ox); free(oy);
}

void orc_face_dists(orc_sim *s, double *xface, double *yface) {
  cell_macros(s);
  cell_transforms(s);
  pop_gradients(s, s->barp, s->gbx, s->gby);
  all_faces(s);
  copy_faces_out(s, s->facex, s->facey, xface, yface);
}
#endif /* ORC_COMPLEX_STEP */
