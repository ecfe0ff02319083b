// dugks2p_dev.hpp -- device arithmetic of the two-phase DUGKS step
// (Zhang, Yang & Guo, arXiv:1802.02868, Sec. 2.2).
//
// Every function here is __host__ __device__ so that the exact same code runs
// in the gfx950 kernels and in a host build used for testing the kernel logic.
// FP64 arithmetic is written in a fixed evaluation order and compiled without
// FMA contraction, so the FP64 path is reproducible bit for bit across the
// staged and fused kernels.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define DFN __host__ __device__ __forceinline__
#else
#define DFN inline
#endif

// The step's code lives in namespace dg.  The FMA-contracted build of the
// fused step (dugks2p_fma.hip, a translation unit compiled with
// -ffp-contract=fast) defines DUGKS2P_NS as dg_fma before including these
// headers, so that its copies of the same templates and kernels coexist
// with the exact ones in one library.
#ifndef DUGKS2P_NS
#define DUGKS2P_NS dg
#endif

namespace DUGKS2P_NS {

typedef long long i64;

// D2Q9 (eq. D2Q9): 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1)
// 7:(-1,-1) 8:(1,-1); opposites 1-3, 2-4, 5-7, 6-8.
DFN int ex_of(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0); }
DFN int ey_of(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0); }
DFN int opp_of(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5); }

// Unit lattice speed (c = sqrt(3 RT) = 1, i.e. RT = 1/3 as in every test of
// the paper): xi_i = e_i in {-1, 0, 1}^2 and the weights are literals, so the
// per-direction products fold away.  Each helper returns the value the
// general expression yields, with the same association (x * 1 = x, x + 0 =
// x, x * -1 = -x are exact), so both variants agree bit for bit.
DFN double w9_lit(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }

// e_i . (a, b) in the order (e_x a) + (e_y b)
template <class R>
DFN R edot(int i, R a, R b) {
  switch (i) {
    case 0: return (R)0.0;
    case 1: return a;
    case 2: return b;
    case 3: return -a;
    case 4: return -b;
    case 5: return a + b;
    case 6: return -a + b;
    case 7: return -a + -b;
    default: return a + -b;
  }
}

// One mesh axis (App. B tensor-product mesh).  Cell k: neighbours lo/hi
// (periodic wrap, or the cell itself standing for the mirror ghost across a
// wall), three-point weights (minus, centre, plus) of the first and second
// derivative and of the population gradient.  Face k is the low face of cell
// k; fl/fr are the cells on either side (-1 = wall).
struct Axis {
  int n, bc, nf, pad;
  const int *lo, *hi, *fl, *fr;
  const double *d1, *d2, *pg, *rdt, *w;
  const double *fwl, *fwr, *finv, *foffl, *foffr;
};

// Neighbours along an axis are topology only: cell k's stencil neighbours
// are k -+ 1, wrapped on a periodic axis and the cell itself (standing for
// its mirror ghost) at a wall; face k lies between cells k - 1 and k, with
// -1 for the wall side.  These equal the tables lo, hi, fl, fr.
DFN int ax_lo(const Axis &a, int k) { return k > 0 ? k - 1 : (a.bc == 0 ? a.n - 1 : 0); }
DFN int ax_hi(const Axis &a, int k) { return k < a.n - 1 ? k + 1 : (a.bc == 0 ? 0 : k); }
DFN int ax_fl(const Axis &a, int k) { return (a.bc == 0 && k == 0) ? a.n - 1 : k - 1; }
DFN int ax_fr(const Axis &a, int k) { return (a.bc != 0 && k == a.n) ? -1 : k; }

// Geometry of face k of an axis: the cells on either side (-1 = wall), the
// interpolation weights and inverse distance of the central face operator,
// and the offsets from the two cell centres to the face.
struct FaceGeo {
  int cl, cr;
  double wl, wr, inv, offl, offr;
};

DFN FaceGeo face_geo(const Axis &a, int k) {
  FaceGeo g;
  g.cl = ax_fl(a, k);
  g.cr = ax_fr(a, k);
  g.wl = a.fwl[k];
  g.wr = a.fwr[k];
  g.inv = a.finv[k];
  g.offl = a.foffl[k];
  g.offr = a.foffr[k];
  return g;
}

struct Consts {
  int nx, ny, ld, nfx, nfy, recon, phi_clamp, unit;  // unit: c = sqrt(3 RT) == 1
  i64 plane;   // ny * ld: stride between populations / fields
  i64 xplane;  // ny * nfx: stride of x-face arrays
  i64 yplane;  // nfy * ld: stride of y-face arrays
  double dt, h, hdt, hh, cs2, k1, k2, k3, eta, gam, inv_dphi, drho, mumu, mu_a, mu_b;
  double c4b, phimid, lo_phi, hi_phi, tau_g, tau_f, mobility, kappa, beta;
  double phi_a, phi_b, rho_a, rho_b, gx, gy, rho_ref;
  double hdtcs2, hhcs2, ch0;
  double w9[9], chi[9], wics2[9], xi0[9], xi1[9];
  double gca, gcb, gcc, gk1, gk2, gk3;  // transforms of g (constant tau_g)
  Axis ax[2];
};

// Macroscopic state at a point: input of the equilibria and sources.
template <class R>
struct Mac {
  R phi, rho, ux, uy, p, mu, grx, gry, D, Fx, Fy, gpx, gpy, icr;
};

// eq. oderrho (optional clamp of phi inside rho() only)
template <class R>
DFN R rho_of(const Consts &K, R phi) {
  R ph = phi;
  if (K.phi_clamp) ph = ph < (R)K.lo_phi ? (R)K.lo_phi : (ph > (R)K.hi_phi ? (R)K.hi_phi : ph);
  return ((ph - (R)K.phi_b) * (R)K.rho_a + ((R)K.phi_a - ph) * (R)K.rho_b) * (R)K.inv_dphi;
}

// Viscosity model of the f~ relaxation time, as a kernel is compiled for it:
// VIS_ANY reads it from Consts at run time (a given tau_f when K.tau_f > 0,
// else the mixture viscosity); VIS_UNIFORM and VIS_MIXTURE fix one of the
// two, and the host launches them only where K.tau_f agrees.
enum { VIS_ANY = 0, VIS_UNIFORM = 1, VIS_MIXTURE = 2 };

// eqs. kineticandmobility and mixvis: tau_f = mu_d / (rho c_s^2)
template <class R, int V = VIS_ANY>
DFN R tauf_of(const Consts &K, R phi, R rho) {
  if (V == VIS_UNIFORM || (V == VIS_ANY && K.tau_f > 0.0)) return (R)K.tau_f;
  R ph = phi;
  if (K.phi_clamp) ph = ph < (R)K.lo_phi ? (R)K.lo_phi : (ph > (R)K.hi_phi ? (R)K.hi_phi : ph);
  const R mud = (R)K.mumu / ((ph - (R)K.phi_b) * (R)K.mu_b + ((R)K.phi_a - ph) * (R)K.mu_a);
  return mud / (rho * (R)K.cs2);
}

// eqs. feq, geq, su, Hi, F, G at one point, direction i.  U: unit speed.
template <class R, bool U = false>
DFN void point_eq1(const Consts &K, const Mac<R> &m, R uu, int i, R &feq, R &geq, R &ff, R &fg) {
  const R cs2 = (R)K.cs2;
  const R wi = U ? (R)w9_lit(i) : (R)K.w9[i];
  const R xx = U ? (R)ex_of(i) : (R)K.xi0[i], xy = U ? (R)ey_of(i) : (R)K.xi1[i];
  const R eu = U ? edot<R>(i, m.ux, m.uy) : xx * m.ux + xy * m.uy;
  const R si = wi * (eu * (R)K.k1 + eu * eu * (R)K.k2 - uu * (R)K.k3);
  feq = wi * m.p + cs2 * m.rho * si;
  // chi and wics2 take three distinct values (one per weight class)
  const int wc = U ? (i == 0 ? 0 : (i < 5 ? 1 : 5)) : i;
  const R Hi = (i == 0) ? m.phi - (R)K.ch0 * m.mu : (R)K.chi[wc] * m.mu;
  geq = Hi + m.phi * si;
  const R G = wi + si;
  const R cx = xx - m.ux, cy = xy - m.uy;
  ff = cx * (m.Fx * G + si * cs2 * m.grx) + cy * (m.Fy * G + si * cs2 * m.gry) -
       (R)K.wics2[wc] * m.rho * (R)K.gam * m.D;
  fg = m.phi * m.icr * (cx * (m.Fx - m.gpx) + cy * (m.Fy - m.gpy)) * G;
}

// sum_i xi_x,i v_i and sum_i xi_y,i v_i over 9 values, ascending i.
template <class R, bool U>
DFN void xi_sums(const Consts &K, const R v[9], R &jx, R &jy) {
  if (U) {
    jx = ((((v[1] - v[3]) + v[5]) - v[6]) - v[7]) + v[8];
    jy = ((((v[2] - v[4]) + v[5]) + v[6]) - v[7]) - v[8];
    return;
  }
  jx = (R)0.0;
  jy = (R)0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) jx += (R)K.xi0[i] * v[i];
#pragma unroll
  for (int i = 0; i < 9; ++i) jy += (R)K.xi1[i] * v[i];
}

// Three-point stencil along x (axis 0) or y (axis 1) of a cell field with
// row pitch ld.
DFN double stx(const Consts &K, const double *w3, const double *F, int i, int j) {
  const Axis &a = K.ax[0];
  const double *w = w3 + 3 * i;
  const i64 r = (i64)j * K.ld;
  return w[0] * F[r + ax_lo(a, i)] + w[1] * F[r + i] + w[2] * F[r + ax_hi(a, i)];
}
DFN double sty(const Consts &K, const double *w3, const double *F, int i, int j) {
  const Axis &a = K.ax[1];
  const double *w = w3 + 3 * j;
  return w[0] * F[(i64)ax_lo(a, j) * K.ld + i] + w[1] * F[(i64)j * K.ld + i] +
         w[2] * F[(i64)ax_hi(a, j) * K.ld + i];
}

// Scratch fields of the staged step (all FP64, pitch ld, stride plane).
struct Work {
  double *phi, *rho, *mu, *dphx, *dphy, *dmux, *dmuy, *D, *Fx, *Fy, *ux, *uy, *p, *dpx, *dpy,
      *tauf, *s0, *jx, *jy;
  // phi and the f~ sums of the state a fused step writes (NULL: not kept);
  // the host swaps them with phi, s0, jx, jy when the step is committed
  double *phin, *s0n, *jxn, *jyn;
  double *barp;   // 18 x plane
  double *facex;  // 18 x xplane: [q][j][k]
  double *facey;  // 18 x yplane: [q][k][i]
};

// ---------------------------------------------------------------------------
// State storage.  Populations are handled as 18 doubles per cell
// (q = 0..8 f~, 9..17 g~); an IO policy maps them to memory.
// ---------------------------------------------------------------------------

// FP64 state: 18 planes of doubles.
struct IoF64 {
  double *p;
  i64 plane;
  DFN void load(i64 c, double v[18]) const {
#pragma unroll
    for (int q = 0; q < 18; ++q) v[q] = p[q * plane + c];
  }
  DFN void store(i64 c, const double v[18]) const {
#pragma unroll
    for (int q = 0; q < 18; ++q) p[q * plane + c] = v[q];
  }
  DFN void load_f(i64 c, double f[9]) const {
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = p[q * plane + c];
  }
  // what phi() and load_f() return after store(c, v)
  DFN void stored(const double v[18], double &ph, double f[9]) const {
    ph = 0.0;
#pragma unroll
    for (int q = 9; q < 18; ++q) ph += v[q];
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = v[q];
  }
  // v as load() would return it after store(c, v)
  DFN static void roundtrip(double v[18]) { (void)v; }
  // eq. phi: phi = sum_i g~_i, ascending i
  DFN double phi(i64 c) const {
    double a = 0.0;
#pragma unroll
    for (int q = 9; q < 18; ++q) a += p[q * plane + c];
    return a;
  }
};

// FP32 state with an FP64 order-parameter channel: f~ as 9 floats, the cell
// order parameter phi = sum g~ as one double, and g~_i - w_i phi (i = 1..8)
// as floats (the i = 0 deviation is minus the sum of the others).  Storing
// phi exactly keeps the rounding of g~ out of phi and hence out of the
// chemical potential and the surface force.  76 bytes per cell.
struct IoE32 {
  float *f;    // 17 planes: f~_0..8, then g~_i - w_i phi for i = 1..8
  double *ph;  // 1 plane: phi
  i64 plane;
  DFN void load(i64 c, double v[18]) const {
#pragma unroll
    for (int q = 0; q < 9; ++q) v[q] = (double)f[q * plane + c];
    double d[9], s = 0.0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      d[i] = (double)f[(8 + i) * plane + c];
      s += d[i];
    }
    d[0] = -s;
    const double phi = ph[c];
#pragma unroll
    for (int i = 0; i < 9; ++i) v[9 + i] = w9_lit(i) * phi + d[i];
  }
  DFN void store(i64 c, const double v[18]) const {
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q * plane + c] = (float)v[q];
    double phi = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) phi += v[9 + i];
    ph[c] = phi;
#pragma unroll
    for (int i = 1; i < 9; ++i) f[(8 + i) * plane + c] = (float)(v[9 + i] - w9_lit(i) * phi);
  }
  DFN void load_f(i64 c, double fo[9]) const {
#pragma unroll
    for (int q = 0; q < 9; ++q) fo[q] = (double)f[q * plane + c];
  }
  // what phi() and load_f() return after store(c, v)
  DFN void stored(const double v[18], double &phv, double fo[9]) const {
    phv = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) phv += v[9 + i];
#pragma unroll
    for (int q = 0; q < 9; ++q) fo[q] = (double)(float)v[q];
  }
  // v as load() would return it after store(c, v)
  DFN static void roundtrip(double v[18]) {
#pragma unroll
    for (int q = 0; q < 9; ++q) v[q] = (double)(float)v[q];
    double phi = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) phi += v[9 + i];
    double d[9], s = 0.0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      d[i] = (double)(float)(v[9 + i] - w9_lit(i) * phi);
      s += d[i];
    }
    d[0] = -s;
#pragma unroll
    for (int i = 0; i < 9; ++i) v[9 + i] = w9_lit(i) * phi + d[i];
  }
  DFN double phi(i64 c) const { return ph[c]; }
};

// ---------------------------------------------------------------------------
// Staged step: one functor per stage, one call per cell or face.
// ---------------------------------------------------------------------------

// eq. phi and eq. oderrho
template <class T>
struct FPhi {
  Consts K;
  Work w;
  const T *st;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i;
    double acc = 0.0;
#pragma unroll
    for (int q = 9; q < 18; ++q) acc += (double)st[q * K.plane + c];
    w.phi[c] = acc;
    w.rho[c] = rho_of<double>(K, acc);
  }
};

// eq. chemicalpotential with the App. B Laplacian of phi at cell (i, j).
// eq. chemicalpotential from phi at a cell (ph) and at its x neighbours
// (xl, xh) and y neighbours (yl, yh), with the App. B second-derivative
// weights of its column (wx) and row (wy).
DFN double mu_from(const Consts &K, double ph, double xl, double xh, double yl, double yh,
                   const double *wx, const double *wy) {
  const double lap = (wx[0] * xl + wx[1] * ph + wx[2] * xh) + (wy[0] * yl + wy[1] * ph + wy[2] * yh);
  return K.c4b * (ph - K.phi_a) * (ph - K.phi_b) * (ph - K.phimid) - K.kappa * lap;
}

DFN double mu_at(const Consts &K, const double *phi, int i, int j) {
  const Axis &X = K.ax[0], &Y = K.ax[1];
  const i64 r = (i64)j * K.ld;
  return mu_from(K, phi[r + i], phi[r + ax_lo(X, i)], phi[r + ax_hi(X, i)],
                 phi[(i64)ax_lo(Y, j) * K.ld + i], phi[(i64)ax_hi(Y, j) * K.ld + i],
                 X.d2 + 3 * i, Y.d2 + 3 * j);
}

// eq. chemicalpotential; grad phi.
struct FMu {
  Consts K;
  Work w;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i;
    w.mu[c] = mu_at(K, w.phi, i, j);
    w.dphx[c] = stx(K, K.ax[0].d1, w.phi, i, j);
    w.dphy[c] = sty(K, K.ax[1].d1, w.phi, i, j);
  }
};

// grad mu, D = div(lambda grad mu), F, eq. u, eq. P.
template <class T>
struct FMacro {
  Consts K;
  Work w;
  const T *st;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i;
    w.dmux[c] = stx(K, K.ax[0].d1, w.mu, i, j);
    w.dmuy[c] = sty(K, K.ax[1].d1, w.mu, i, j);
    const double lapmu = stx(K, K.ax[0].d2, w.mu, i, j) + sty(K, K.ax[1].d2, w.mu, i, j);
    const double D = K.mobility * lapmu;
    w.D[c] = D;
    const double ph = w.phi[c], rh = w.rho[c];
    const double Fx = -ph * w.dmux[c] + (rh - K.rho_ref) * K.gx;
    const double Fy = -ph * w.dmuy[c] + (rh - K.rho_ref) * K.gy;
    w.Fx[c] = Fx;
    w.Fy[c] = Fy;
    double s0 = 0.0, jx = 0.0, jy = 0.0;
    double f[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = (double)st[q * K.plane + c];
#pragma unroll
    for (int q = 0; q < 9; ++q) s0 += f[q];
#pragma unroll
    for (int q = 0; q < 9; ++q) jx += K.xi0[q] * f[q];
#pragma unroll
    for (int q = 0; q < 9; ++q) jy += K.xi1[q] * f[q];
    const double icr = 1.0 / (K.cs2 * rh);
    const double ux = (jx + K.hdtcs2 * Fx) * icr;
    const double uy = (jy + K.hdtcs2 * Fy) * icr;
    w.ux[c] = ux;
    w.uy[c] = uy;
    const double grx = K.drho * w.dphx[c], gry = K.drho * w.dphy[c];
    w.p[c] = s0 + K.hdtcs2 * (ux * grx + uy * gry - K.gam * rh * D);
  }
};

template <class R>
DFN void cell_mac(const Consts &K, const Work &w, i64 c, Mac<R> &m) {
  m.phi = (R)w.phi[c];
  m.rho = (R)w.rho[c];
  m.ux = (R)w.ux[c];
  m.uy = (R)w.uy[c];
  m.p = (R)w.p[c];
  m.mu = (R)w.mu[c];
  m.grx = (R)(K.drho * w.dphx[c]);
  m.gry = (R)(K.drho * w.dphy[c]);
  m.D = (R)w.D[c];
  m.Fx = (R)w.Fx[c];
  m.Fy = (R)w.Fy[c];
  m.gpx = (R)w.dpx[c];
  m.gpy = (R)w.dpy[c];
  m.icr = (R)1.0 / ((R)K.cs2 * m.rho);
}

// Step 2 at one cell (eqs. relations1, relations2): bar+ of the 18
// populations from tilde, the cell macros and tau_f.
template <class R, bool U = false>
DFN void cell_barp(const Consts &K, const Mac<R> &m, R tf, const R til[18], R out[18]) {
  const R uu = m.ux * m.ux + m.uy * m.uy;
  const R den = (R)1.0 / ((R)2.0 * tf + (R)K.dt);
  const R fca = ((R)2.0 * tf - (R)K.h) * den, fcb = (R)3.0 * (R)K.h * den,
          fcc = (R)3.0 * tf * (R)K.h * den;
#pragma unroll
  for (int i2 = 0; i2 < 9; ++i2) {
    R feq, geq, ff, fg;
    point_eq1<R, U>(K, m, uu, i2, feq, geq, ff, fg);
    out[i2] = fca * til[i2] + fcb * feq + fcc * ff;
    out[9 + i2] = (R)K.gca * til[9 + i2] + (R)K.gcb * geq + (R)K.gcc * fg;
  }
}

// grad p, tau_f, and Step 2: bar+ into w.barp.  R is the arithmetic type of
// the transforms (double in every instantiation the library builds).
template <class T, class R = double>
struct FCell {
  Consts K;
  Work w;
  const T *st;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i;
    w.dpx[c] = stx(K, K.ax[0].d1, w.p, i, j);
    w.dpy[c] = sty(K, K.ax[1].d1, w.p, i, j);
    const R tf = tauf_of<R>(K, (R)w.phi[c], (R)w.rho[c]);
    w.tauf[c] = (double)tf;
    Mac<R> m;
    cell_mac(K, w, c, m);
    R til[18], out[18];
#pragma unroll
    for (int q = 0; q < 18; ++q) til[q] = (R)st[q * K.plane + c];
    cell_barp<R>(K, m, tf, til, out);
#pragma unroll
    for (int q = 0; q < 18; ++q) w.barp[q * K.plane + c] = (double)out[q];
  }
};

// The cell fields FCell writes besides bar+ (grad p and tau_f), for a tape
// whose bar+ comes from the tile kernel.
template <class R>
struct FCellFields {
  Consts K;
  Work w;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i;
    w.dpx[c] = stx(K, K.ax[0].d1, w.p, i, j);
    w.dpy[c] = sty(K, K.ax[1].d1, w.p, i, j);
    w.tauf[c] = (double)tauf_of<R>(K, (R)w.phi[c], (R)w.rho[c]);
  }
};

// R5: value, normal derivative and tangential derivative of a cell field at
// an interior face between cells L and R (weights of the face).
struct FaceW {
  double wl, wr, inv;
};
DFN void face_field(const FaceW &fw, double FL, double FR, double TL, double TR, double &v,
                    double &dn, double &dt) {
  v = fw.wl * FL + fw.wr * FR;
  dn = (FR - FL) * fw.inv;
  dt = fw.wl * TL + fw.wr * TR;
}

// Step 4 at a face: macros from bar (eq. conservedVariable with h), face
// equilibria and sources, eq. original-function.  Inputs are the face fields.
template <class R>
struct FaceFields {
  R mu, D, gmx, gmy, gfx, gfy, gpx, gpy;
};

template <class R, bool U = false, int V = VIS_ANY>
DFN void face_dist(const Consts &K, const FaceFields<R> &fl, const R bar[18], R out[18]) {
  Mac<R> m;
  R phib = (R)0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) phib += bar[9 + i];
  m.phi = phib;
  m.rho = rho_of<R>(K, phib);
  m.mu = fl.mu;
  m.D = fl.D;
  m.grx = (R)K.drho * fl.gfx;
  m.gry = (R)K.drho * fl.gfy;
  m.gpx = fl.gpx;
  m.gpy = fl.gpy;
  m.Fx = -phib * fl.gmx + (m.rho - (R)K.rho_ref) * (R)K.gx;
  m.Fy = -phib * fl.gmy + (m.rho - (R)K.rho_ref) * (R)K.gy;
  m.icr = (R)1.0 / ((R)K.cs2 * m.rho);
  R s0 = (R)0.0, jx = (R)0.0, jy = (R)0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) s0 += bar[i];
#pragma unroll
  for (int i = 0; i < 9; ++i) jx += (R)K.xi0[i] * bar[i];
#pragma unroll
  for (int i = 0; i < 9; ++i) jy += (R)K.xi1[i] * bar[i];
  m.ux = (jx + (R)K.hhcs2 * m.Fx) * m.icr;
  m.uy = (jy + (R)K.hhcs2 * m.Fy) * m.icr;
  m.p = s0 + (R)K.hhcs2 * (m.ux * m.grx + m.uy * m.gry - (R)K.gam * m.rho * m.D);
  const R uu = m.ux * m.ux + m.uy * m.uy;
  const R tf = tauf_of<R, V>(K, phib, m.rho);
  const R den = (R)1.0 / ((R)2.0 * tf + (R)K.h);
  const R fk1 = (R)2.0 * tf * den, fk2 = (R)K.h * den, fk3 = tf * (R)K.h * den;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    R feq, geq, ff, fg;
    point_eq1<R, U>(K, m, uu, i, feq, geq, ff, fg);
    out[i] = fk1 * bar[i] + fk2 * feq + fk3 * ff;
    out[9 + i] = (R)K.gk1 * bar[9 + i] + (R)K.gk2 * geq + (R)K.gk3 * fg;
  }
}

// Steps 3-4 at face k of axis A (0: x-face between cells (k-1, t) and (k, t);
// 1: y-face between (t, k-1) and (t, k)).  Acc provides bar+ (A), the cell
// fields mu, D, phi, p and their derivatives dmu, dphi, dp along an axis.
template <int A, class R, class Acc, bool U = false, int V = VIS_ANY>
DFN void face_core(const Consts &K, const Acc &acc, int k, int t, R out[18]) {
  // reconstruction of interior faces: the accessor's own where it fixes one
  const bool upw = Acc::RECON < 0 ? K.recon == 1 : Acc::RECON == 1;
  const FaceGeo fg = acc.geo(A, k);
  const int cl = fg.cl, cr = fg.cr;
  const R h = (R)K.h;
  const int TA = 1 - A;  // tangential axis
  R bar[18];
  FaceFields<R> fl;
#define CX(ia) (A == 0 ? (ia) : t)
#define CY(ia) (A == 0 ? t : (ia))
  if (cl < 0 || cr < 0) {
    // wall face: expand from the fluid cell C; bounce-back of entering ones
    const int cc = cl < 0 ? cr : cl;
    const double off = cl < 0 ? fg.offr : fg.offl;
    const int nout = cl < 0 ? -1 : 1;
    const typename Acc::H HC = acc.cell(CX(cc), CY(cc));
#pragma unroll
    for (int q = 0; q < 18; ++q) {
      const int i = q % 9;
      const int en = A == 0 ? ex_of(i) : ey_of(i);
      if (en * nout < 0) continue;
      const R Ac = (R)acc.A(q, HC);
      const R gx = (R)acc.pgrad(0, q, HC), gy = (R)acc.pgrad(1, q, HC);
      const R Gn = A == 0 ? gx : gy, Gt = A == 0 ? gy : gx;
      const R val = Ac + (R)off * Gn;
      const R sgx = A == 0 ? Gn : Gt, sgy = A == 0 ? Gt : Gn;
      bar[q] = val - h * (U ? edot<R>(i, sgx, sgy) : (R)K.xi0[i] * sgx + (R)K.xi1[i] * sgy);
    }
#pragma unroll
    for (int q = 0; q < 18; ++q) {
      const int i = q % 9;
      const int en = A == 0 ? ex_of(i) : ey_of(i);
      if (en * nout < 0) bar[q] = bar[q - i + opp_of(i)];
    }
    fl.mu = (R)acc.mu(HC);
    fl.D = (R)acc.D(HC);
    const double tmu = acc.dmu(TA, HC), tph = acc.dphi(TA, HC), tp = acc.dp(TA, HC);
    fl.gmx = A == 0 ? (R)0.0 : (R)tmu;
    fl.gmy = A == 0 ? (R)tmu : (R)0.0;
    fl.gfx = A == 0 ? (R)0.0 : (R)tph;
    fl.gfy = A == 0 ? (R)tph : (R)0.0;
    fl.gpx = A == 0 ? (R)0.0 : (R)tp;
    fl.gpy = A == 0 ? (R)tp : (R)0.0;
    face_dist<R, U, V>(K, fl, bar, out);
#pragma unroll
    for (int q = 0; q < 18; ++q) {
      const int i = q % 9;
      const int en = A == 0 ? ex_of(i) : ey_of(i);
      if (en * nout < 0) out[q] = out[q - i + opp_of(i)];
    }
    return;
  }
  const typename Acc::H HL = acc.cell(CX(cl), CY(cl)), HR = acc.cell(CX(cr), CY(cr));
  FaceW fw;
  fw.wl = fg.wl;
  fw.wr = fg.wr;
  fw.inv = fg.inv;
#pragma unroll
  for (int q = 0; q < 18; ++q) {
    const int i = q % 9;
    const int en = A == 0 ? ex_of(i) : ey_of(i);
    const R AL = (R)acc.A(q, HL), AR = (R)acc.A(q, HR);
    R val, sn, st;
    if (upw && en > 0) {
      const R gx = (R)acc.pgrad(0, q, HL), gy = (R)acc.pgrad(1, q, HL);
      const R Gn = A == 0 ? gx : gy, Gt = A == 0 ? gy : gx;
      val = AL + (R)fg.offl * Gn;
      sn = Gn;
      st = Gt;
    } else if (upw && en < 0) {
      const R gx = (R)acc.pgrad(0, q, HR), gy = (R)acc.pgrad(1, q, HR);
      const R Gn = A == 0 ? gx : gy, Gt = A == 0 ? gy : gx;
      val = AR + (R)fg.offr * Gn;
      sn = Gn;
      st = Gt;
    } else {
      const R GtL = (R)acc.pgrad(TA, q, HL);
      const R GtR = (R)acc.pgrad(TA, q, HR);
      val = (R)fw.wl * AL + (R)fw.wr * AR;
      sn = (AR - AL) * (R)fw.inv;
      st = (R)fw.wl * GtL + (R)fw.wr * GtR;
    }
    const R sgx = A == 0 ? sn : st, sgy = A == 0 ? st : sn;
    bar[q] = val - h * (U ? edot<R>(i, sgx, sgy) : (R)K.xi0[i] * sgx + (R)K.xi1[i] * sgy);
  }
  double v, tmp, gn, gt;
  face_field(fw, acc.mu(HL), acc.mu(HR), acc.dmu(TA, HL), acc.dmu(TA, HR), v, gn, gt);
  fl.mu = (R)v;
  fl.gmx = (R)(A == 0 ? gn : gt);
  fl.gmy = (R)(A == 0 ? gt : gn);
  face_field(fw, acc.D(HL), acc.D(HR), 0.0, 0.0, v, tmp, tmp);
  fl.D = (R)v;
  face_field(fw, acc.phi(HL), acc.phi(HR), acc.dphi(TA, HL), acc.dphi(TA, HR), tmp, gn, gt);
  fl.gfx = (R)(A == 0 ? gn : gt);
  fl.gfy = (R)(A == 0 ? gt : gn);
  face_field(fw, acc.p(HL), acc.p(HR), acc.dp(TA, HL), acc.dp(TA, HR), tmp, gn, gt);
  fl.gpx = (R)(A == 0 ? gn : gt);
  fl.gpy = (R)(A == 0 ? gt : gn);
  face_dist<R, U, V>(K, fl, bar, out);
#undef CX
#undef CY
}

// Accessor over the staged global arrays.  A cell handle is its linear
// index and coordinates; derivatives use the App. B weights of the axis.
struct GAcc {
  static constexpr int RECON = -1;  // K.recon at run time
  const Consts *K;
  const Work *w;
  struct H {
    int x, y;
    i64 c, lo[2], hi[2];
  };
  DFN H cell(int x, int y) const {
    H h;
    h.x = x;
    h.y = y;
    h.c = (i64)y * K->ld + x;
    h.lo[0] = (i64)y * K->ld + ax_lo(K->ax[0], x);
    h.hi[0] = (i64)y * K->ld + ax_hi(K->ax[0], x);
    h.lo[1] = (i64)ax_lo(K->ax[1], y) * K->ld + x;
    h.hi[1] = (i64)ax_hi(K->ax[1], y) * K->ld + x;
    return h;
  }
  DFN FaceGeo geo(int a, int k) const { return face_geo(K->ax[a], k); }
  DFN double A(int q, const H &h) const { return w->barp[q * K->plane + h.c]; }
  DFN double pgrad(int a, int q, const H &h) const {
    const double *wt = K->ax[a].pg + 3 * (a == 0 ? h.x : h.y);
    const double *Aq = w->barp + q * K->plane;
    return wt[0] * Aq[h.lo[a]] + wt[1] * Aq[h.c] + wt[2] * Aq[h.hi[a]];
  }
  DFN double mu(const H &h) const { return w->mu[h.c]; }
  DFN double D(const H &h) const { return w->D[h.c]; }
  DFN double phi(const H &h) const { return w->phi[h.c]; }
  DFN double p(const H &h) const { return w->p[h.c]; }
  DFN double dmu(int a, const H &h) const { return (a == 0 ? w->dmux : w->dmuy)[h.c]; }
  DFN double dphi(int a, const H &h) const { return (a == 0 ? w->dphx : w->dphy)[h.c]; }
  DFN double dp(int a, const H &h) const { return (a == 0 ? w->dpx : w->dpy)[h.c]; }
};

template <class R = double>
struct FXFace {
  Consts K;
  Work w;
  DFN void operator()(int k, int j) const {
    R out[18];
    const GAcc acc{&K, &w};
    face_core<0, R>(K, acc, k, j, out);
#pragma unroll
    for (int q = 0; q < 18; ++q) w.facex[q * K.xplane + (i64)j * K.nfx + k] = (double)out[q];
  }
};
template <class R = double>
struct FYFace {
  Consts K;
  Work w;
  DFN void operator()(int i, int k) const {
    R out[18];
    const GAcc acc{&K, &w};
    face_core<1, R>(K, acc, k, i, out);
#pragma unroll
    for (int q = 0; q < 18; ++q) w.facey[q * K.yplane + (i64)k * K.ld + i] = (double)out[q];
  }
};

// Steps 5-6: eq. updatef with tilde+ = 4/3 bar+ - 1/3 tilde (eq. relations2).
template <class T, class R = double>
struct FUpdate {
  Consts K;
  Work w;
  const T *st;
  T *dst;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i;
    const int ie = (K.ax[0].bc == 0 && i == K.nx - 1) ? 0 : i + 1;
    const int jn = (K.ax[1].bc == 0 && j == K.ny - 1) ? 0 : j + 1;
    const R rx = (R)K.ax[0].rdt[i], ry = (R)K.ax[1].rdt[j];
#pragma unroll
    for (int q = 0; q < 18; ++q) {
      const int d = q % 9;
      const R bp = (R)w.barp[q * K.plane + c];
      const R til = (R)st[q * K.plane + c];
      const R tilp = (R)(4.0 / 3.0) * bp - (R)(1.0 / 3.0) * til;
      const R W = (R)w.facex[q * K.xplane + (i64)j * K.nfx + i];
      const R E = (R)w.facex[q * K.xplane + (i64)j * K.nfx + ie];
      const R S = (R)w.facey[q * K.yplane + (i64)j * K.ld + i];
      const R N = (R)w.facey[q * K.yplane + (i64)jn * K.ld + i];
      dst[q * K.plane + c] =
          (T)(tilp - rx * (R)K.xi0[d] * (E - W) - ry * (R)K.xi1[d] * (N - S));
    }
  }
};

// ---------------------------------------------------------------------------
// Step 1 (initialisation) from phi0, u0, p0.
// ---------------------------------------------------------------------------
struct FInit0 {
  Consts K;
  Work w;
  const double *phi0, *ux0, *uy0, *p0;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i, c0 = (i64)j * K.nx + i;
    w.phi[c] = phi0[c0];
    w.rho[c] = rho_of<double>(K, phi0[c0]);
    w.ux[c] = ux0[c0];
    w.uy[c] = uy0[c0];
    w.p[c] = p0[c0];
  }
};

struct FInit1 {
  Consts K;
  Work w;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i;
    w.dmux[c] = stx(K, K.ax[0].d1, w.mu, i, j);
    w.dmuy[c] = sty(K, K.ax[1].d1, w.mu, i, j);
    const double lapmu = stx(K, K.ax[0].d2, w.mu, i, j) + sty(K, K.ax[1].d2, w.mu, i, j);
    w.D[c] = K.mobility * lapmu;
    w.Fx[c] = -w.phi[c] * w.dmux[c] + (w.rho[c] - K.rho_ref) * K.gx;
    w.Fy[c] = -w.phi[c] * w.dmuy[c] + (w.rho[c] - K.rho_ref) * K.gy;
    w.dpx[c] = stx(K, K.ax[0].d1, w.p, i, j);
    w.dpy[c] = sty(K, K.ax[1].d1, w.p, i, j);
  }
};

template <class IO>
struct FInit2 {
  Consts K;
  Work w;
  IO dst;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i;
    Mac<double> m;
    cell_mac(K, w, c, m);
    const double uu = m.ux * m.ux + m.uy * m.uy;
    double v[18];
#pragma unroll
    for (int i2 = 0; i2 < 9; ++i2) {
      double feq, geq, ff, fg;
      point_eq1(K, m, uu, i2, feq, geq, ff, fg);
      v[i2] = feq - K.hdt * ff;
      v[9 + i2] = geq - K.hdt * fg;
    }
    dst.store(c, v);
  }
};

// ---------------------------------------------------------------------------
// Moments and monitors.
// ---------------------------------------------------------------------------
struct FMoments {
  Consts K;
  Work w;
  double *phi, *rho, *ux, *uy, *p;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i, o = (i64)j * K.nx + i;
    if (phi) phi[o] = w.phi[c];
    if (rho) rho[o] = rho_of<double>(K, w.phi[c]);
    if (ux) ux[o] = w.ux[c];
    if (uy) uy[o] = w.uy[c];
    if (p) p[o] = w.p[c];
  }
};

// Per-cell monitor terms: phi |V|, rho |u|^2 |V| / 2, free-energy density
// (eqs. doublewell, freeenergyfunction) times |V|, |u|, non-finite count.
template <class IO>
DFN void monitor_terms(const Consts &K, const Work &w, const IO &io, int i, int j, double out[5]) {
  const i64 c = (i64)j * K.ld + i;
  const double V = K.ax[0].w[i] * K.ax[1].w[j];
  const double ph = w.phi[c];
  const double rh = rho_of<double>(K, ph);
  const double u2 = w.ux[c] * w.ux[c] + w.uy[c] * w.uy[c];
  const double a1 = ph - K.phi_a, b1 = ph - K.phi_b;
  const double psi = K.beta * a1 * a1 * b1 * b1;
  const double gx = stx(K, K.ax[0].d1, w.phi, i, j), gy = sty(K, K.ax[1].d1, w.phi, i, j);
  const double g2 = gx * gx + gy * gy;
  out[0] = ph * V;
  out[1] = 0.5 * rh * u2 * V;
  out[2] = (psi + 0.5 * K.kappa * g2) * V;
  out[3] = u2;  // max of u2, sqrt at the end
  double v[18], bad = 0.0;
  io.load(c, v);
#pragma unroll
  for (int q = 0; q < 18; ++q)
    if (!(v[q] - v[q] == 0.0)) bad += 1.0;
  out[4] = bad;
}

}  // namespace DUGKS2P_NS
