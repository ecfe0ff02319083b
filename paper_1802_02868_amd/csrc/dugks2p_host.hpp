// dugks2p_host.hpp -- host-side preparation of a two-phase DUGKS problem:
// parameter validation, App. B mesh tables, derived constants, workspace
// layout, and the stage sequence of one time step (templated on an
// executor so the same sequence drives GPU launches and host test runs).
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/dugks2p.h"
#include "dugks2p_dev.hpp"

namespace DUGKS2P_NS {

// Tables of one axis in host memory (see struct Axis).
struct AxisHost {
  int n = 0, bc = 0, nf = 0;
  double L = 0.0;
  std::vector<double> f, c, w, d1, d2, pg, rdt, fwl, fwr, finv, foffl, foffr;
  std::vector<int> lo, hi, fl, fr;
};

inline bool strictly_increasing(const double *f, int n) {
  for (int k = 0; k < n; ++k)
    if (!(f[k + 1] > f[k])) return false;
  return true;
}

// App. B three-point weights with h_l, h_r the distances to the left and right
// neighbour centres (periodic images or mirror ghosts across walls).
inline void build_axis(AxisHost &a, int n, int bc, const double *faces) {
  a.n = n;
  a.bc = bc;
  a.nf = bc == DUGKS2P_BC_PERIODIC ? n : n + 1;
  a.f.assign(faces, faces + n + 1);
  a.c.resize(n);
  a.w.resize(n);
  for (int k = 0; k < n; ++k) {
    a.c[k] = 0.5 * (a.f[k] + a.f[k + 1]);
    a.w[k] = a.f[k + 1] - a.f[k];
  }
  a.L = a.f[n] - a.f[0];
  a.lo.resize(n);
  a.hi.resize(n);
  a.d1.resize(3 * n);
  a.d2.resize(3 * n);
  a.pg.resize(3 * n);
  a.rdt.resize(n);
  for (int k = 0; k < n; ++k) {
    int im, ip;
    double pm, pp;
    if (k > 0) {
      im = k - 1;
      pm = a.c[k - 1];
    } else if (bc == DUGKS2P_BC_PERIODIC) {
      im = n - 1;
      pm = a.c[n - 1] - a.L;
    } else {
      im = k;
      pm = 2.0 * a.f[0] - a.c[0];
    }
    if (k < n - 1) {
      ip = k + 1;
      pp = a.c[k + 1];
    } else if (bc == DUGKS2P_BC_PERIODIC) {
      ip = 0;
      pp = a.c[0] + a.L;
    } else {
      ip = k;
      pp = 2.0 * a.f[n] - a.c[n - 1];
    }
    a.lo[k] = im;
    a.hi[k] = ip;
    const double hl = a.c[k] - pm, hr = pp - a.c[k];
    const double hl2 = hl * hl, hr2 = hr * hr, den = hl * hr * (hl + hr);
    a.d1[3 * k + 0] = -hr2 / den;
    a.d1[3 * k + 1] = (hr2 - hl2) / den;
    a.d1[3 * k + 2] = hl2 / den;
    a.d2[3 * k + 0] = 2.0 * hr / den;
    a.d2[3 * k + 1] = -2.0 * (hl + hr) / den;
    a.d2[3 * k + 2] = 2.0 * hl / den;
    if (bc == DUGKS2P_BC_WALL && k == 0) {
      const double inv = 1.0 / (a.c[1] - a.c[0]);
      a.pg[3 * k + 0] = 0.0;
      a.pg[3 * k + 1] = -inv;
      a.pg[3 * k + 2] = inv;
    } else if (bc == DUGKS2P_BC_WALL && k == n - 1) {
      const double inv = 1.0 / (a.c[n - 1] - a.c[n - 2]);
      a.pg[3 * k + 0] = -inv;
      a.pg[3 * k + 1] = inv;
      a.pg[3 * k + 2] = 0.0;
    } else {
      for (int m = 0; m < 3; ++m) a.pg[3 * k + m] = a.d1[3 * k + m];
    }
  }
  a.fl.assign(a.nf, 0);
  a.fr.assign(a.nf, 0);
  a.fwl.assign(a.nf, 0.0);
  a.fwr.assign(a.nf, 0.0);
  a.finv.assign(a.nf, 0.0);
  a.foffl.assign(a.nf, 0.0);
  a.foffr.assign(a.nf, 0.0);
  for (int k = 0; k < a.nf; ++k) {
    if (bc == DUGKS2P_BC_WALL && (k == 0 || k == n)) {
      a.fl[k] = k == 0 ? -1 : n - 1;
      a.fr[k] = k == 0 ? 0 : -1;
      if (k == 0)
        a.foffr[k] = a.f[0] - a.c[0];
      else
        a.foffl[k] = a.f[n] - a.c[n - 1];
      continue;
    }
    const double xl = k == 0 ? a.c[n - 1] - a.L : a.c[k - 1];
    const double xr = a.c[k], xf = a.f[k];
    const double d = xr - xl;
    a.fl[k] = k == 0 ? n - 1 : k - 1;
    a.fr[k] = k;
    a.fwl[k] = (xr - xf) / d;
    a.fwr[k] = (xf - xl) / d;
    a.finv[k] = 1.0 / d;
    a.foffl[k] = xf - xl;
    a.foffr[k] = xf - xr;
  }
}

// Returns an empty string if the parameters are valid, else the reason.
inline std::string validate(const dugks2p_params *P) {
  if (!P) return "params is NULL";
  if (P->abi_version != DUGKS2P_ABI_VERSION) return "abi_version mismatch";
  if (P->nx < 1 || P->ny < 1) return "nx and ny must be >= 1";
  if ((P->bc_x != DUGKS2P_BC_PERIODIC && P->bc_x != DUGKS2P_BC_WALL) ||
      (P->bc_y != DUGKS2P_BC_PERIODIC && P->bc_y != DUGKS2P_BC_WALL))
    return "bc_x / bc_y must be DUGKS2P_BC_PERIODIC or DUGKS2P_BC_WALL";
  if ((P->bc_x == DUGKS2P_BC_WALL && P->nx < 2) || (P->bc_y == DUGKS2P_BC_WALL && P->ny < 2))
    return "a wall axis needs at least 2 cells";
  if (P->precision != DUGKS2P_FP64 && P->precision != DUGKS2P_FP32_STATE)
    return "precision must be DUGKS2P_FP64 or DUGKS2P_FP32_STATE";
  if (P->recon != DUGKS2P_RECON_CENTRAL && P->recon != DUGKS2P_RECON_UPWIND)
    return "recon must be DUGKS2P_RECON_CENTRAL or DUGKS2P_RECON_UPWIND";
  if (P->kernel < DUGKS2P_KERNEL_AUTO || P->kernel > DUGKS2P_KERNEL_FUSED_FMA)
    return "kernel must be a DUGKS2P_KERNEL_* value";
  if (P->tile < DUGKS2P_TILE_AUTO || P->tile > DUGKS2P_TILE_TALL)
    return "tile must be a DUGKS2P_TILE_* value";
  if (!P->x_faces || !P->y_faces) return "x_faces / y_faces is NULL";
  if (!strictly_increasing(P->x_faces, P->nx) || !strictly_increasing(P->y_faces, P->ny))
    return "faces must be strictly increasing";
  if (!(P->rt > 0.0)) return "rt must be > 0";
  if (!(P->tau_g > 0.0)) return "tau_g must be > 0";
  if (!(P->mobility >= 0.0)) return "mobility must be >= 0";
  if (!(P->phi_a != P->phi_b)) return "phi_a must differ from phi_b";
  if (!(P->rho_a > 0.0) || !(P->rho_b > 0.0)) return "rho_a and rho_b must be > 0";
  if (!(P->tau_f > 0.0) && !(P->nu_a > 0.0 && P->nu_b > 0.0))
    return "need tau_f > 0, or nu_a > 0 and nu_b > 0";
  if (!(P->dt > 0.0) && !(P->cfl > 0.0)) return "need dt > 0 or cfl > 0";
  const double vals[] = {P->cfl, P->c_max, P->dt, P->rt, P->tau_g, P->mobility, P->tau_f,
                         P->beta, P->kappa, P->phi_a, P->phi_b, P->rho_a, P->rho_b,
                         P->nu_a, P->nu_b, P->gx, P->gy, P->rho_ref};
  for (double v : vals)
    if (!isfinite(v)) return "parameters must be finite";
  if ((int64_t)P->nx * P->ny > (int64_t)1 << 34) return "grid too large";
  return std::string();
}

// Row pitch in elements: rows start on 256-byte boundaries for FP64 grids
// wider than one wave.
inline int row_pitch(int nx) { return nx < 64 ? nx : ((nx + 31) / 32) * 32; }

inline double time_step(const dugks2p_params *P, const AxisHost &ax, const AxisHost &ay) {
  if (P->dt > 0.0) return P->dt;
  double dxmin = ax.w[0];
  for (int k = 0; k < ax.n; ++k)
    if (ax.w[k] < dxmin) dxmin = ax.w[k];
  for (int k = 0; k < ay.n; ++k)
    if (ay.w[k] < dxmin) dxmin = ay.w[k];
  const double cmax = P->c_max > 0.0 ? P->c_max : sqrt(6.0 * P->rt);
  return P->cfl * dxmin / cmax;
}

// Derived constants of the step (device table pointers filled later).
inline Consts make_consts(const dugks2p_params *P, AxisHost &ax, AxisHost &ay) {
  Consts K;
  memset(&K, 0, sizeof K);
  K.nx = P->nx;
  K.ny = P->ny;
  K.ld = row_pitch(P->nx);
  K.nfx = ax.nf;
  K.nfy = ay.nf;
  K.recon = P->recon;
  K.phi_clamp = P->phi_clamp ? 1 : 0;
  K.plane = (i64)K.ny * K.ld;
  K.xplane = (i64)K.ny * K.nfx;
  K.yplane = (i64)K.nfy * K.ld;
  const double dt = time_step(P, ax, ay);
  K.dt = dt;
  K.h = 0.5 * dt;
  K.hdt = 0.5 * dt;
  K.hh = 0.5 * K.h;
  K.cs2 = P->rt;
  const double c = sqrt(3.0 * P->rt);
  K.unit = c == 1.0 ? 1 : 0;
  K.k1 = 1.0 / K.cs2;
  K.k2 = 1.0 / (2.0 * K.cs2 * K.cs2);
  K.k3 = 1.0 / (2.0 * K.cs2);
  K.eta = P->mobility / (K.cs2 * P->tau_g);
  const double rr = P->rho_a / P->rho_b;
  K.gam = (rr - 1.0) / (P->phi_a - P->phi_b * rr);
  K.inv_dphi = 1.0 / (P->phi_a - P->phi_b);
  K.drho = (P->rho_a - P->rho_b) * K.inv_dphi;
  K.mu_a = P->rho_a * P->nu_a;
  K.mu_b = P->rho_b * P->nu_b;
  K.mumu = (P->rho_a * P->nu_a) * (P->rho_b * P->nu_b) * (P->phi_a - P->phi_b);
  K.c4b = 4.0 * P->beta;
  K.phimid = 0.5 * (P->phi_a + P->phi_b);
  K.lo_phi = P->phi_a < P->phi_b ? P->phi_a : P->phi_b;
  K.hi_phi = P->phi_a < P->phi_b ? P->phi_b : P->phi_a;
  K.tau_g = P->tau_g;
  K.tau_f = P->tau_f > 0.0 ? P->tau_f : 0.0;
  K.mobility = P->mobility;
  K.kappa = P->kappa;
  K.beta = P->beta;
  K.phi_a = P->phi_a;
  K.phi_b = P->phi_b;
  K.rho_a = P->rho_a;
  K.rho_b = P->rho_b;
  K.gx = P->gx;
  K.gy = P->gy;
  K.rho_ref = P->rho_ref;
  K.hdtcs2 = K.hdt * K.cs2;
  K.hhcs2 = K.hh * K.cs2;
  static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  for (int i = 0; i < 9; ++i) {
    K.w9[i] = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    K.xi0[i] = EX[i] * c;
    K.xi1[i] = EY[i] * c;
  }
  K.ch0 = (1.0 - K.w9[0]) * K.eta;
  for (int i = 0; i < 9; ++i) {
    K.chi[i] = K.w9[i] * K.eta;
    K.wics2[i] = K.w9[i] * K.cs2;
  }
  const double tg = P->tau_g;
  const double den = 1.0 / (2.0 * tg + dt);
  K.gca = (2.0 * tg - K.h) * den;
  K.gcb = 3.0 * K.h * den;
  K.gcc = 3.0 * tg * K.h * den;
  const double den2 = 1.0 / (2.0 * tg + K.h);
  K.gk1 = 2.0 * tg * den2;
  K.gk2 = K.h * den2;
  K.gk3 = tg * K.h * den2;
  for (int k = 0; k < ax.n; ++k) ax.rdt[k] = dt / ax.w[k];
  for (int k = 0; k < ay.n; ++k) ay.rdt[k] = dt / ay.w[k];
  return K;
}

// ---------------------------------------------------------------------------
// Workspace layout.  Every region starts on a 256-byte boundary.
// ---------------------------------------------------------------------------
// Ping-pong states up to this size (both buffers, bytes) stay in the MALL
// (256 MB) while a step runs, so the square and two-ring tile kernels at unit
// lattice speed keep tilde+ in the output buffer there (with_fused_kernel):
// the store and reload then cost no HBM traffic, and the LDS they free lets
// three workgroups share a CU.  On larger states the reload goes to HBM and
// the LDS form is faster (measured: 6-8 % faster at 159-170 MB, 4 % slower
// at 231 MB, 2 % slower at 302 MB).
constexpr double TILDE_OUT_MAX_STATE_BYTES = 192.0 * 1024.0 * 1024.0;

struct Layout {
  size_t tables[2];  // per-axis table block
  size_t state[2];   // ping-pong population buffers
  size_t work;       // 13 cell fields (+3 for the staged kernels)
  size_t barp, facex, facey;  // staged kernels only
  size_t mon;        // monitor and observable partials (9 per 64 x 4 block)
  size_t centres;    // cell centres of both axes (nx + ny doubles)
  size_t total;
  size_t state_bytes;
  size_t f32_planes;  // byte offset of the FP64 phi plane in an FP32 state
  int nwork;
  size_t mon_blocks;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline size_t axis_table_bytes(const AxisHost &a) {
  // ints: lo, hi (n), fl, fr (nf); doubles: d1, d2, pg (3n), rdt, w (n),
  // fwl, fwr, finv, foffl, foffr (nf)
  size_t b = 0;
  b += align256(sizeof(int) * (2 * a.n + 2 * a.nf));
  b += align256(sizeof(double) * (9 * a.n + 2 * a.n + 5 * a.nf));
  return b;
}

inline Layout make_layout(const Consts &K, const AxisHost &ax, const AxisHost &ay, int precision,
                          bool staged) {
  Layout L;
  size_t off = 0;
  L.tables[0] = off;
  off += align256(axis_table_bytes(ax));
  L.tables[1] = off;
  off += align256(axis_table_bytes(ay));
  // FP64: 18 double planes.  FP32 state: 17 float planes + 1 double plane
  // (layout of IoE32).
  L.f32_planes = align256(17 * sizeof(float) * (size_t)K.plane);
  L.state_bytes = precision == DUGKS2P_FP64 ? 18 * sizeof(double) * (size_t)K.plane
                                            : L.f32_planes + sizeof(double) * (size_t)K.plane;
  L.state[0] = off;
  off += align256(L.state_bytes);
  L.state[1] = off;
  off += align256(L.state_bytes);
  L.nwork = 23;
  L.work = off;
  off += L.nwork * align256(sizeof(double) * (size_t)K.plane);
  if (staged) {
    L.barp = off;
    off += align256(18 * sizeof(double) * (size_t)K.plane);
    L.facex = off;
    off += align256(18 * sizeof(double) * (size_t)K.xplane);
    L.facey = off;
    off += align256(18 * sizeof(double) * (size_t)K.yplane);
  } else {
    L.barp = L.facex = L.facey = 0;
  }
  L.mon_blocks = (size_t)((K.nx + 63) / 64) * ((K.ny + 3) / 4);
  L.mon = off;
  off += align256(sizeof(double) * (9 * L.mon_blocks + 16));
  L.centres = off;
  off += align256(sizeof(double) * ((size_t)K.nx + K.ny));
  L.total = off;
  return L;
}

// Host copy of one axis table block (same layout as on the device).
inline void pack_axis(const AxisHost &a, std::vector<unsigned char> &buf) {
  buf.assign(axis_table_bytes(a), 0);
  int *ip = (int *)buf.data();
  memcpy(ip, a.lo.data(), sizeof(int) * a.n);
  memcpy(ip + a.n, a.hi.data(), sizeof(int) * a.n);
  memcpy(ip + 2 * a.n, a.fl.data(), sizeof(int) * a.nf);
  memcpy(ip + 2 * a.n + a.nf, a.fr.data(), sizeof(int) * a.nf);
  double *dp = (double *)(buf.data() + align256(sizeof(int) * (2 * a.n + 2 * a.nf)));
  size_t o = 0;
  memcpy(dp + o, a.d1.data(), sizeof(double) * 3 * a.n); o += 3 * a.n;
  memcpy(dp + o, a.d2.data(), sizeof(double) * 3 * a.n); o += 3 * a.n;
  memcpy(dp + o, a.pg.data(), sizeof(double) * 3 * a.n); o += 3 * a.n;
  memcpy(dp + o, a.rdt.data(), sizeof(double) * a.n); o += a.n;
  memcpy(dp + o, a.w.data(), sizeof(double) * a.n); o += a.n;
  memcpy(dp + o, a.fwl.data(), sizeof(double) * a.nf); o += a.nf;
  memcpy(dp + o, a.fwr.data(), sizeof(double) * a.nf); o += a.nf;
  memcpy(dp + o, a.finv.data(), sizeof(double) * a.nf); o += a.nf;
  memcpy(dp + o, a.foffl.data(), sizeof(double) * a.nf); o += a.nf;
  memcpy(dp + o, a.foffr.data(), sizeof(double) * a.nf); o += a.nf;
}

// Point an Axis at a table block located at `base` (device or host address).
inline Axis bind_axis(const AxisHost &a, unsigned char *base) {
  Axis x;
  memset(&x, 0, sizeof x);
  x.n = a.n;
  x.bc = a.bc;
  x.nf = a.nf;
  int *ip = (int *)base;
  x.lo = ip;
  x.hi = ip + a.n;
  x.fl = ip + 2 * a.n;
  x.fr = ip + 2 * a.n + a.nf;
  double *dp = (double *)(base + align256(sizeof(int) * (2 * a.n + 2 * a.nf)));
  size_t o = 0;
  x.d1 = dp + o; o += 3 * a.n;
  x.d2 = dp + o; o += 3 * a.n;
  x.pg = dp + o; o += 3 * a.n;
  x.rdt = dp + o; o += a.n;
  x.w = dp + o; o += a.n;
  x.fwl = dp + o; o += a.nf;
  x.fwr = dp + o; o += a.nf;
  x.finv = dp + o; o += a.nf;
  x.foffl = dp + o; o += a.nf;
  x.foffr = dp + o; o += a.nf;
  return x;
}

inline Work bind_work(const Layout &L, const Consts &K, unsigned char *base) {
  Work w;
  memset(&w, 0, sizeof w);
  double **f[23] = {&w.phi, &w.rho, &w.mu,  &w.dphx, &w.dphy, &w.dmux, &w.dmuy, &w.D,
                    &w.Fx,  &w.Fy,  &w.ux,  &w.uy,   &w.p,    &w.dpx,  &w.dpy,  &w.tauf,
                    &w.s0,  &w.jx,  &w.jy,  &w.phin, &w.s0n,  &w.jxn,  &w.jyn};
  const size_t fb = align256(sizeof(double) * (size_t)K.plane);
  for (int k = 0; k < 23; ++k) *f[k] = (double *)(base + L.work + k * fb);
  if (L.barp) {
    w.barp = (double *)(base + L.barp);
    w.facex = (double *)(base + L.facex);
    w.facey = (double *)(base + L.facey);
  }
  return w;
}

// ---------------------------------------------------------------------------
// Stage sequences (Ex provides grid(functor, n0, n1)).
// ---------------------------------------------------------------------------
template <class Ex, class IO>
void seq_init(Ex &ex, const Consts &K, const Work &w, const double *phi0, const double *ux0,
              const double *uy0, const double *p0, const IO &dst) {
  ex.grid(FInit0{K, w, phi0, ux0, uy0, p0}, K.nx, K.ny);
  ex.grid(FMu{K, w}, K.nx, K.ny);
  ex.grid(FInit1{K, w}, K.nx, K.ny);
  ex.grid(FInit2<IO>{K, w, dst}, K.nx, K.ny);
}

inline IoF64 io_f64(void *state, const Consts &K) { return IoF64{(double *)state, K.plane}; }
inline IoE32 io_e32(void *state, const Consts &K, const Layout &L) {
  return IoE32{(float *)state, (double *)((unsigned char *)state + L.f32_planes), K.plane};
}

// Cell macroscopic fields of the current state (Step 7), staged form.
template <class Ex, class T>
void seq_staged_macros(Ex &ex, const Consts &K, const Work &w, const T *src) {
  ex.grid(FPhi<T>{K, w, src}, K.nx, K.ny);
  ex.grid(FMu{K, w}, K.nx, K.ny);
  ex.grid(FMacro<T>{K, w, src}, K.nx, K.ny);
}

// One time step with the staged kernels (one pass per stage).
// R: arithmetic type of Steps 2-6 (double: every form computes in FP64).
template <class Ex, class T, class R = double>
void seq_staged_step(Ex &ex, const Consts &K, const Work &w, const T *src, T *dst) {
  seq_staged_macros(ex, K, w, src);
  ex.grid(FCell<T, R>{K, w, src}, K.nx, K.ny);
  ex.grid(FXFace<R>{K, w}, K.nfx, K.ny);
  ex.grid(FYFace<R>{K, w}, K.nx, K.nfy);
  ex.grid(FUpdate<T, R>{K, w, src, dst}, K.nx, K.ny);
}

}  // namespace DUGKS2P_NS
