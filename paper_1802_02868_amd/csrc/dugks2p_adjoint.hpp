// dugks2p_adjoint.hpp -- hand-written reverse mode (vector-Jacobian product)
// of one FP64 DUGKS time step and of the initialisation, in gather form.
//
// Forward quantities are recomputed from the staged forward arrays of the
// same step (phi, rho, mu, grad phi, grad mu, D, F, u, p, grad p, bar+).  The
// reverse sweep mirrors the forward stages:
//   face stage  -> per-face records (adjoint of the face values and fields)
//   gather      -> per-cell sums over the records of the cell's four faces
//   Step 2      -> adjoint of the cell transforms (eqs. relations1/2)
//   macros      -> adjoint of eqs. u, P and of F, D
//   mu          -> adjoint of eq. chemicalpotential
//   phi         -> adjoint of eq. phi, eq. oderrho and the phi stencils
// Stencil transposes are gathers (a cell sums what its stencil readers
// received), so no floating-point atomics are used and the result does not
// depend on thread scheduling.  CENTRAL reconstruction, phi_clamp off.
#pragma once

#include "dugks2p_fused.hpp"
#include "dugks2p_host.hpp"

// The reverse arithmetic below (the vector-Jacobian products) may fuse a
// multiply with the add that consumes it: the derivative is not held to bit
// identity, only to rounding (its tests bound it against central
// differences and complex-step derivatives of the oracle).  The forward
// functions it calls keep the exact evaluation of their own definitions.
#if defined(__clang__)
#pragma clang fp contract(fast)
#endif

namespace DUGKS2P_NS {

// ---------------------------------------------------------------------------
// Pointwise adjoints.
// ---------------------------------------------------------------------------

// Adjoint of point_eq1 (eqs. feq, geq, su, Hi, F, G) for direction i:
// accumulates into mb (same fields as Mac) and uub (d/d u^2).
DFN void point_eq1_vjp(const Consts &K, const Mac<double> &m, double uu, int i, double feqb,
                       double geqb, double ffb, double fgb, Mac<double> &mb, double &uub) {
  const double cs2 = K.cs2;
  const double wi = K.w9[i], xx = K.xi0[i], xy = K.xi1[i];
  const double eu = xx * m.ux + xy * m.uy;
  const double si = wi * (eu * K.k1 + eu * eu * K.k2 - uu * K.k3);
  const double G = wi + si;
  const double cx = xx - m.ux, cy = xy - m.uy;
  const double A1 = m.Fx * G + si * cs2 * m.grx, A2 = m.Fy * G + si * cs2 * m.gry;
  const double Q = cx * (m.Fx - m.gpx) + cy * (m.Fy - m.gpy);
  double sib = 0.0, Gb = 0.0, cxb = 0.0, cyb = 0.0;
  // feq = wi p + cs2 rho si
  mb.p += wi * feqb;
  mb.rho += cs2 * si * feqb;
  sib += cs2 * m.rho * feqb;
  // geq = Hi + phi si
  mb.phi += si * geqb;
  sib += m.phi * geqb;
  if (i == 0) {
    mb.phi += geqb;
    mb.mu += -K.ch0 * geqb;
  } else {
    mb.mu += K.chi[i] * geqb;
  }
  // ff = cx A1 + cy A2 - wics2 rho gam D
  cxb += A1 * ffb;
  cyb += A2 * ffb;
  const double A1b = cx * ffb, A2b = cy * ffb;
  mb.rho += -K.wics2[i] * K.gam * m.D * ffb;
  mb.D += -K.wics2[i] * m.rho * K.gam * ffb;
  mb.Fx += G * A1b;
  Gb += m.Fx * A1b;
  sib += cs2 * m.grx * A1b;
  mb.grx += si * cs2 * A1b;
  mb.Fy += G * A2b;
  Gb += m.Fy * A2b;
  sib += cs2 * m.gry * A2b;
  mb.gry += si * cs2 * A2b;
  // fg = phi icr Q G
  mb.phi += m.icr * Q * G * fgb;
  mb.icr += m.phi * Q * G * fgb;
  const double Qb = m.phi * m.icr * G * fgb;
  Gb += m.phi * m.icr * Q * fgb;
  cxb += (m.Fx - m.gpx) * Qb;
  mb.Fx += cx * Qb;
  mb.gpx += -cx * Qb;
  cyb += (m.Fy - m.gpy) * Qb;
  mb.Fy += cy * Qb;
  mb.gpy += -cy * Qb;
  // G = wi + si ; cx = xx - ux ; cy = xy - uy
  sib += Gb;
  mb.ux += -cxb;
  mb.uy += -cyb;
  // si = wi (eu k1 + eu^2 k2 - uu k3)
  const double eub = wi * (K.k1 + 2.0 * eu * K.k2) * sib;
  uub += -wi * K.k3 * sib;
  mb.ux += xx * eub;
  mb.uy += xy * eub;
}

DFN void mac_zero(Mac<double> &m) {
  m.phi = m.rho = m.ux = m.uy = m.p = m.mu = m.grx = m.gry = m.D = m.Fx = m.Fy = m.gpx =
      m.gpy = m.icr = 0.0;
}

// d tau_f / d phi and d tau_f / d rho of eqs. kineticandmobility, mixvis.
DFN void tauf_grad(const Consts &K, double phi, double rho, double &dphi, double &drho) {
  if (K.tau_f > 0.0) {
    dphi = drho = 0.0;
    return;
  }
  const double den = (phi - K.phi_b) * K.mu_b + (K.phi_a - phi) * K.mu_a;
  const double mud = K.mumu / den;
  const double tf = mud / (rho * K.cs2);
  dphi = -mud / den * (K.mu_b - K.mu_a) / (rho * K.cs2);
  drho = -tf / rho;
}

// ---------------------------------------------------------------------------
// Work arrays of the reverse sweep.
// ---------------------------------------------------------------------------
enum {
  FB_MU, FB_D, FB_PHI, FB_P, FB_DMUX, FB_DMUY, FB_DPHX, FB_DPHY, FB_DPX, FB_DPY, FB_RHO, FB_FX,
  FB_FY, FB_UX, FB_UY, FB_S0, FB_JX, FB_JY, FB_LAPMU, FB_LAPPHI, FB_KAP, FB_GX, FB_GY, NFB
};
// Per-face record of the face stage: adjoint of the 18 reconstructed face
// values bar (after folding the bounce-back copies), of the 8 face fields and
// the body-force partials of the face.
enum {
  FS_B = 0, FS_MU = 18, FS_D, FS_GMX, FS_GMY, FS_GFX, FS_GFY, FS_GPX, FS_GPY, FS_GX, FS_GY, NFS
};

struct AdjWork {
  const double *lam;  // 18 planes: adjoint of the state after the step
  double *out;        // 18 planes: adjoint of the state before the step
  double *xs, *ys;    // face records: NFS planes of xplane / yplane
  double *fb;         // NFB planes of per-cell field adjoints and parameter partials
  double *pacc;       // 3 planes: per-cell sums over steps of the kappa, gx, gy partials
};

// Transpose of a three-point stencil along one axis at one cell: the cells
// whose stencil reads this cell (at most three, each counted once) and the
// summed weight with which each reads it.  Unused entries have weight 0 and
// point at the cell itself.
struct TW {
  i64 id[3];
  double w[3];
};

DFN TW stencil_tw(const Consts &K, int ax, const double *wt3, int i, int j) {
  const Axis &X = K.ax[ax];
  const int c = ax == 0 ? i : j;
  const int cand[3] = {ax_lo(X, c), c, ax_hi(X, c)};
  TW t;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int cp = cand[a];
    bool dup = false;
    for (int b = 0; b < a; ++b) dup |= cand[b] == cp;
    const int tgt[3] = {ax_lo(X, cp), cp, ax_hi(X, cp)};
    const double *w = wt3 + 3 * cp;
    double s = 0.0;
    if (!dup)
      for (int m = 0; m < 3; ++m)
        if (tgt[m] == c) s += w[m];
    t.w[a] = s;
    t.id[a] = ax == 0 ? (i64)j * K.ld + cp : (i64)cp * K.ld + i;
  }
  return t;
}

DFN double tw_apply(const TW &t, const double *B) {
  return t.w[0] * B[t.id[0]] + t.w[1] * B[t.id[1]] + t.w[2] * B[t.id[2]];
}

// ---------------------------------------------------------------------------
// Adjoint of Step 4 at a face (eq. original-function with the face macros
// of eq. conservedVariable at h, the equilibria and the sources).
// ob(q): adjoint of the face distribution q.  Accumulates the face-field
// adjoints into fb and the body-force partials into gxb, gyb; returns what
// the adjoint of bar q needs: bar_b(q) = fk1 ob(q) + s0b + xi_q . (jxb, jyb)
// for q < 9 and gk1 ob(q) + phibb for the g populations.
// ---------------------------------------------------------------------------
struct FaceBack {
  double fk1, s0b, jxb, jyb, phibb;
};

// ob(q): the adjoint of face value q; obpair(i, obf, obg): the same for
// q = i and 9 + i, called with i = 0..8 in order (so that it can load the
// next direction's inputs while this one is computed).
template <class OB, class OBP>
DFN FaceBack face_dist_vjp(const Consts &K, const FaceFields<double> &fl, const double bar[18],
                           const OB &ob, OBP &obpair, FaceFields<double> &fb, double &gxb,
                           double &gyb) {
  Mac<double> m;
  double phib = 0.0;
  for (int i = 0; i < 9; ++i) phib += bar[9 + i];
  m.phi = phib;
  m.rho = rho_of<double>(K, phib);
  m.mu = fl.mu;
  m.D = fl.D;
  m.grx = K.drho * fl.gfx;
  m.gry = K.drho * fl.gfy;
  m.gpx = fl.gpx;
  m.gpy = fl.gpy;
  m.Fx = -phib * fl.gmx + (m.rho - K.rho_ref) * K.gx;
  m.Fy = -phib * fl.gmy + (m.rho - K.rho_ref) * K.gy;
  m.icr = 1.0 / (K.cs2 * m.rho);
  double s0 = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < 9; ++i) s0 += bar[i];
  for (int i = 0; i < 9; ++i) jx += K.xi0[i] * bar[i];
  for (int i = 0; i < 9; ++i) jy += K.xi1[i] * bar[i];
  m.ux = (jx + K.hhcs2 * m.Fx) * m.icr;
  m.uy = (jy + K.hhcs2 * m.Fy) * m.icr;
  m.p = s0 + K.hhcs2 * (m.ux * m.grx + m.uy * m.gry - K.gam * m.rho * m.D);
  const double uu = m.ux * m.ux + m.uy * m.uy;
  const double tf = tauf_of<double>(K, phib, m.rho);
  const double den = 1.0 / (2.0 * tf + K.h);
  const double fk1 = 2.0 * tf * den, fk2 = K.h * den, fk3 = tf * K.h * den;
  Mac<double> mb;
  mac_zero(mb);
  double uub = 0.0, fk1b = 0.0, fk2b = 0.0, fk3b = 0.0;
  // one direction at a time (a rolled loop keeps the register footprint
  // small); bar is indexed only in unrolled loops so it stays in registers
#pragma unroll 1
  for (int i = 0; i < 9; ++i) {
    double feq, geq, ff, fg;
    point_eq1<double>(K, m, uu, i, feq, geq, ff, fg);
    double obf, obg;
    obpair(i, obf, obg);
    fk2b += feq * obf;
    fk3b += ff * obf;
    point_eq1_vjp(K, m, uu, i, fk2 * obf, K.gk2 * obg, fk3 * obf, K.gk3 * obg, mb, uub);
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) fk1b += bar[i] * ob(i);
  // fk1 = 2 tf den, fk2 = h den, fk3 = tf h den, den = 1/(2 tf + h)
  const double denb = 2.0 * tf * fk1b + K.h * fk2b + tf * K.h * fk3b;
  const double tfb = 2.0 * den * fk1b + K.h * den * fk3b - 2.0 * den * den * denb;
  double dtp, dtr;
  tauf_grad(K, phib, m.rho, dtp, dtr);
  double phibb = dtp * tfb, rhob = mb.rho + dtr * tfb;
  mb.ux += 2.0 * m.ux * uub;
  mb.uy += 2.0 * m.uy * uub;
  // p = s0 + hhcs2 (ux grx + uy gry - gam rho D)
  const double pb = mb.p;
  mb.ux += K.hhcs2 * m.grx * pb;
  mb.grx += K.hhcs2 * m.ux * pb;
  mb.uy += K.hhcs2 * m.gry * pb;
  mb.gry += K.hhcs2 * m.uy * pb;
  rhob += -K.hhcs2 * K.gam * m.D * pb;
  mb.D += -K.hhcs2 * K.gam * m.rho * pb;
  // u = (j + hhcs2 F) icr
  FaceBack r;
  r.fk1 = fk1;
  r.s0b = pb;
  r.jxb = m.icr * mb.ux;
  r.jyb = m.icr * mb.uy;
  mb.Fx += K.hhcs2 * m.icr * mb.ux;
  mb.Fy += K.hhcs2 * m.icr * mb.uy;
  mb.icr += (jx + K.hhcs2 * m.Fx) * mb.ux + (jy + K.hhcs2 * m.Fy) * mb.uy;
  // icr = 1/(cs2 rho)
  rhob += -K.cs2 * m.icr * m.icr * mb.icr;
  // F = -phib gm + (rho - rho_ref) g
  phibb += -fl.gmx * mb.Fx - fl.gmy * mb.Fy;
  fb.gmx += -phib * mb.Fx;
  fb.gmy += -phib * mb.Fy;
  rhob += K.gx * mb.Fx + K.gy * mb.Fy;
  gxb += (m.rho - K.rho_ref) * mb.Fx;
  gyb += (m.rho - K.rho_ref) * mb.Fy;
  fb.gfx += K.drho * mb.grx;
  fb.gfy += K.drho * mb.gry;
  fb.gpx += mb.gpx;
  fb.gpy += mb.gpy;
  fb.mu += mb.mu;
  fb.D += mb.D;
  r.phibb = phibb + mb.phi + K.drho * rhob;
  return r;
}

// ---------------------------------------------------------------------------
// Reverse stages.
// ---------------------------------------------------------------------------

// Face stage: adjoint of the face distributions from the update (eq.
// updatef), then of Step 4 and of the bounce-back copies; the adjoint of bar
// and of the face fields go to the face record.
// Face k of axis A at tangential index t (0: x-face between cells (k-1, t)
// and (k, t); 1: y-face between (t, k-1) and (t, k)).  Acc provides the
// tape's bar+ and cell fields with their derivatives (GAcc from the global
// tape, LAcc from a tile window in LDS: the same values).
template <int A, class Acc>
DFN void adj_face(const Consts &K, const Acc &acc, const AdjWork &a, int k, int t) {
  const Axis &ax = K.ax[A];
  const int cl = ax_fl(ax, k), cr = ax_fr(ax, k);
  const int TA = 1 - A;
  const i64 fpl = A == 0 ? K.xplane : K.yplane;
  double *rec = (A == 0 ? a.xs + (i64)t * K.nfx + k : a.ys + (i64)k * K.ld + t);
  const bool wall = cl < 0 || cr < 0;
  const int nout = cl < 0 ? -1 : 1;  // outward normal of the fluid cell (walls)
  const i64 P = K.plane;
  const i64 cL = cl >= 0 ? (A == 0 ? (i64)t * K.ld + cl : (i64)cl * K.ld + t) : 0;
  const i64 cR = cr >= 0 ? (A == 0 ? (i64)t * K.ld + cr : (i64)cr * K.ld + t) : 0;
  const double rL = cl >= 0 ? ax.rdt[cl] : 0.0, rR = cr >= 0 ? ax.rdt[cr] : 0.0;
  const double *lam = a.lam;
  // the face value enters the update of cell L with -r_L xi_n and of
  // cell R with +r_R xi_n; at a wall the entering values are copies of
  // the outgoing opposite ones, so their adjoint folds onto those
  // (cL and cR are valid cells even on the wall side, so the loads need no
  // branch and can all be in flight together)
  auto ob_raw = [&](int q) {
    const double xn = A == 0 ? K.xi0[q % 9] : K.xi1[q % 9];
    const double lL = lam[q * P + cL], lR = lam[q * P + cR];
    double v = 0.0;
    if (cl >= 0) v += -(rL * xn) * lL;
    if (cr >= 0) v += (rR * xn) * lR;
    return v;
  };
  auto en_of = [&](int q) { return A == 0 ? ex_of(q % 9) : ey_of(q % 9); };
  auto ob = [&](int q) {
    const int en = en_of(q);
    if (wall && en * nout < 0) return 0.0;
    double v = ob_raw(q);
    if (wall && en * nout > 0) v += ob_raw(q - q % 9 + opp_of(q % 9));
    return v;
  };
  const double h = K.h;
  double bar[18];
  FaceFields<double> fl, fb;
  fb.mu = fb.D = fb.gmx = fb.gmy = fb.gfx = fb.gfy = fb.gpx = fb.gpy = 0.0;
  double gxb = 0.0, gyb = 0.0;
  if (wall) {
    const int cc = cl < 0 ? cr : cl;
    const double off = cl < 0 ? ax.foffr[k] : ax.foffl[k];
    const typename Acc::H HC = acc.cell(A == 0 ? cc : t, A == 0 ? t : cc);
#pragma unroll
    for (int q = 0; q < 18; ++q) {
      const int i = q % 9;
      if (en_of(q) * nout < 0) continue;
      const double Gn = acc.pgrad(A, q, HC), Gt = acc.pgrad(TA, q, HC);
      const double val = acc.A(q, HC) + off * Gn;
      const double sgx = A == 0 ? Gn : Gt, sgy = A == 0 ? Gt : Gn;
      bar[q] = val - h * (K.xi0[i] * sgx + K.xi1[i] * sgy);
    }
#pragma unroll
    for (int q = 0; q < 18; ++q)
      if (en_of(q) * nout < 0) bar[q] = bar[q - q % 9 + opp_of(q % 9)];
    fl.mu = acc.mu(HC);
    fl.D = acc.D(HC);
    const double tmu = acc.dmu(TA, HC), tph = acc.dphi(TA, HC), tp = acc.dp(TA, HC);
    fl.gmx = A == 0 ? 0.0 : tmu;
    fl.gmy = A == 0 ? tmu : 0.0;
    fl.gfx = A == 0 ? 0.0 : tph;
    fl.gfy = A == 0 ? tph : 0.0;
    fl.gpx = A == 0 ? 0.0 : tp;
    fl.gpy = A == 0 ? tp : 0.0;
  } else {
    const typename Acc::H HL = acc.cell(A == 0 ? cl : t, A == 0 ? t : cl);
    const typename Acc::H HR = acc.cell(A == 0 ? cr : t, A == 0 ? t : cr);
    const FaceW fw{ax.fwl[k], ax.fwr[k], ax.finv[k]};
#pragma unroll
    for (int q = 0; q < 18; ++q) {
      const int i = q % 9;
      const double AL = acc.A(q, HL), AR = acc.A(q, HR);
      const double val = fw.wl * AL + fw.wr * AR;
      const double sn = (AR - AL) * fw.inv;
      const double st = fw.wl * acc.pgrad(TA, q, HL) + fw.wr * acc.pgrad(TA, q, HR);
      const double sgx = A == 0 ? sn : st, sgy = A == 0 ? st : sn;
      bar[q] = val - h * (K.xi0[i] * sgx + K.xi1[i] * sgy);
    }
    double v, tmp, gn, gt;
    face_field(fw, acc.mu(HL), acc.mu(HR), acc.dmu(TA, HL), acc.dmu(TA, HR), v, gn, gt);
    fl.mu = v;
    fl.gmx = A == 0 ? gn : gt;
    fl.gmy = A == 0 ? gt : gn;
    face_field(fw, acc.D(HL), acc.D(HR), 0.0, 0.0, v, tmp, tmp);
    fl.D = v;
    face_field(fw, acc.phi(HL), acc.phi(HR), acc.dphi(TA, HL), acc.dphi(TA, HR), tmp, gn, gt);
    fl.gfx = A == 0 ? gn : gt;
    fl.gfy = A == 0 ? gt : gn;
    face_field(fw, acc.p(HL), acc.p(HR), acc.dp(TA, HL), acc.dp(TA, HR), tmp, gn, gt);
    fl.gpx = A == 0 ? gn : gt;
    fl.gpy = A == 0 ? gt : gn;
  }
  // The VJP's direction loop is rolled (registers), so ob(i) there would
  // wait on its loads once per direction.  obpair loads the lam values of
  // direction i + 1 while direction i is computed, and evaluates ob from
  // them in the same order of operations as ob.
  struct LamDir {
    double v[8];  // f (q = i) then g (q = 9 + i): lam at L, at R, and at L, R of opp(q)
  };
  auto lam_dir = [&](int i) {
    LamDir d;
    const int o = opp_of(i);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int q = 9 * s + i, qo = 9 * s + o;
      d.v[4 * s + 0] = lam[q * P + cL];
      d.v[4 * s + 1] = lam[q * P + cR];
      d.v[4 * s + 2] = (wall && cl >= 0) ? lam[qo * P + cL] : 0.0;
      d.v[4 * s + 3] = (wall && cr >= 0) ? lam[qo * P + cR] : 0.0;
    }
    return d;
  };
  auto ob_from = [&](int q, double lL, double lR) {
    const double xn = A == 0 ? K.xi0[q % 9] : K.xi1[q % 9];
    double v = 0.0;
    if (cl >= 0) v += -(rL * xn) * lL;
    if (cr >= 0) v += (rR * xn) * lR;
    return v;
  };
  auto ob_dir = [&](int q, const LamDir &d, int s) {
    const int en = en_of(q);
    if (wall && en * nout < 0) return 0.0;
    double v = ob_from(q, d.v[4 * s + 0], d.v[4 * s + 1]);
    if (wall && en * nout > 0) v += ob_from(q - q % 9 + opp_of(q % 9), d.v[4 * s + 2], d.v[4 * s + 3]);
    return v;
  };
  auto obpair = [&, nxt = lam_dir(0)](int i, double &obf, double &obg) mutable {
    const LamDir cur = nxt;
    if (i + 1 < 9) nxt = lam_dir(i + 1);
    obf = ob_dir(i, cur, 0);
    obg = ob_dir(9 + i, cur, 1);
  };
  const FaceBack r = face_dist_vjp(K, fl, bar, ob, obpair, fb, gxb, gyb);
  auto barb = [&](int q) {
    const int i = q % 9;
    return q < 9 ? r.fk1 * ob(q) + (r.s0b + K.xi0[i] * r.jxb + K.xi1[i] * r.jyb)
                 : K.gk1 * ob(q) + r.phibb;
  };
#pragma unroll
  for (int q = 0; q < 18; ++q) {
    const int en = en_of(q);
    double v;
    if (wall && en * nout < 0)
      v = 0.0;
    else if (wall && en * nout > 0)
      v = barb(q) + barb(q - q % 9 + opp_of(q % 9));
    else
      v = barb(q);
    rec[(FS_B + q) * fpl] = v;
  }
  rec[FS_MU * fpl] = fb.mu;
  rec[FS_D * fpl] = fb.D;
  rec[FS_GMX * fpl] = fb.gmx;
  rec[FS_GMY * fpl] = fb.gmy;
  rec[FS_GFX * fpl] = fb.gfx;
  rec[FS_GFY * fpl] = fb.gfy;
  rec[FS_GPX * fpl] = fb.gpx;
  rec[FS_GPY * fpl] = fb.gpy;
  rec[FS_GX * fpl] = gxb;
  rec[FS_GY * fpl] = gyb;
}

// The face stage over the forward's tiles.  P0 and the tape's bar+ and D on
// the bar+ window go to LDS (the forward's window layout), then each thread
// takes the x-face west of its column and the y-face south of its row, as
// the forward's P2 does, reading the window through LAcc.  A face between
// two tiles is written once: by the tile whose cells lie east (north) of it,
// or for the far wall face by the last tile.
// LDS of the face stage: the forward tile's bar+, scalar and D windows and
// tables, without tilde+ and the face values (about 49 KB for 14 x 14
// tiles, so three workgroups fit a CU).
template <class S>
struct AdjLds {
  struct {
    double A[18][S::WY][S::WX];
  } u;
  double phi[S::SY][S::SX], mu[S::SY][S::SX], p[S::SY][S::SX];
  double D[S::WY][S::WX];
  double pgw[2][S::SM][3], d1w[2][S::SM][3];
  double fwl[2][S::FM], fwr[2][S::FM], finv[2][S::FM], foffl[2][S::FM], foffr[2][S::FM];
  double rdt[2][S::FM];
};

template <class S>
struct AdjFaceTile {
  static_assert(S::RG == 1, "the face stage reads bar+ on a one-cell ring");
  const Consts &K;
  const Work &w;  // the step's tape
  const AdjWork &a;
  int x0, y0;
  AdjLds<S> *L;
  struct PreA {
    double b[18], D;
  };
  using Win = TileP0<S, AdjLds<S>>;
  DFN Win win() const { return Win{K, w, x0, y0, L}; }
  // window cell of thread tid and its global index, false outside a wall domain
  DFN bool cell_of(int tid, int &lx, int &ly, i64 &c) const {
    lx = tid % S::WX;
    ly = tid / S::WX;
    const Win p = win();
    const int gx = p.gcol(x0 - 1 + lx, K.nx, K.ax[0].bc);
    const int gy = p.gcol(y0 - 1 + ly, K.ny, K.ax[1].bc);
    if (gx < 0 || gy < 0) return false;
    c = (i64)gy * K.ld + gx;
    return true;
  }
  DFN void a_load(int tid, PreA &r) const {
    int lx, ly;
    i64 c;
    if (!cell_of(tid, lx, ly, c)) return;
#pragma unroll
    for (int q = 0; q < 18; ++q) r.b[q] = w.barp[q * K.plane + c];
    r.D = w.D[c];
  }
  DFN void a_store(int tid, const PreA &r) const {
    int lx, ly;
    i64 c;
    if (!cell_of(tid, lx, ly, c)) return;
#pragma unroll
    for (int q = 0; q < 18; ++q) L->u.A[q][ly][lx] = r.b[q];
    L->D[ly][lx] = r.D;
  }
  DFN void faces(int tid) const {
    const int tx = tid % S::WX, ty = tid / S::WX;
    const LAcc<S, AdjLds<S>> acc{&K, &w, L, x0, y0};
    if (tx <= S::TX && ty < S::TY) {
      const int k = x0 + tx, t = y0 + ty;
      if (t < K.ny && k < K.nfx && (tx < S::TX || k == K.nx)) adj_face<0>(K, acc, a, k, t);
    }
    if (tx < S::TX && ty <= S::TY) {
      const int k = y0 + ty, t = x0 + tx;
      if (t < K.nx && k < K.nfy && (ty < S::TY || k == K.ny)) adj_face<1>(K, acc, a, k, t);
    }
  }
};

#if defined(__HIPCC__)
// three waves per SIMD (168 VGPRs, a few spilled), measured 2 % faster for
// the whole reverse step than two waves without spills
template <class S>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(3))) void k_adj_faces(Consts K, Work w, AdjWork a, int ntx,
                                                    int ntiles) {
  __shared__ AdjLds<S> L;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const AdjFaceTile<S> ft{K, w, a, (tile % ntx) * S::TX, (tile / ntx) * S::TY, &L};
  const int tid = threadIdx.x;
  typename AdjFaceTile<S>::Win::Pre0 r0;
  typename AdjFaceTile<S>::PreA ra;
  ft.win().p0_load(tid, r0);
  ft.a_load(tid, ra);
  ft.win().p0_store(tid, r0);
  ft.a_store(tid, ra);
  __syncthreads();
  ft.faces(tid);
}
#endif

// Geometry of one face of axis A as seen from the cell on side s (0: low
// side L, 1: high side R): reverse of the face reconstruction of bar (eq.
// original-function with the central face operator, or the one-sided wall
// expansion) and of the face fields.
struct FaceSide {
  bool wall;
  double wgt, sg, off, wa;  // wa = 1 at a wall face, else 0
};

template <int A>
DFN FaceSide face_side(const Consts &K, int k, int s) {
  const Axis &ax = K.ax[A];
  FaceSide f;
  f.wall = ax_fl(ax, k) < 0 || ax_fr(ax, k) < 0;
  if (f.wall) {
    f.wgt = 1.0;
    f.sg = 0.0;
    f.off = ax_fl(ax, k) < 0 ? ax.foffr[k] : ax.foffl[k];
    f.wa = 1.0;
  } else {
    f.wgt = s == 0 ? ax.fwl[k] : ax.fwr[k];
    f.sg = (s == 0 ? -1.0 : 1.0) * ax.finv[k];
    f.off = 0.0;
    f.wa = 0.0;
  }
  return f;
}

// Contribution of a face's bar adjoint (population q) to the cell's bar+
// adjoint and to the adjoints of its population gradients g[0], g[1].
// Interior face: bar = wl AL + wr AR - h (xn (AR - AL) inv + xt (wl GtL +
// wr GtR)); wall face: bar = A + off Gn - h (xn Gn + xt Gt).  One branch-free
// form covers both (wgt = 1, sg = 0, wa = 1 at a wall).
template <int A>
DFN double face_ab_back(const Consts &K, const FaceSide &f, int q, double bb) {
  const double xn = A == 0 ? K.xi0[q % 9] : K.xi1[q % 9];
  return f.wgt * bb + f.sg * (-K.h * xn * bb);
}
template <int A>
DFN void face_grad_back(const Consts &K, const FaceSide &f, int q, double bb, double g[2]) {
  const int i = q % 9;
  const double xn = A == 0 ? K.xi0[i] : K.xi1[i], xt = A == 0 ? K.xi1[i] : K.xi0[i];
  g[A] += f.wa * ((f.off - K.h * xn) * bb);
  g[1 - A] += f.wgt * (-K.h * xt * bb);
}

// Contribution of a face's field adjoints to the cell fields
// fv = (mu, D, phi, p, dmu x/y, dphi x/y, dp x/y, gx, gy partials).
template <int A>
DFN void face_field_back(const FaceSide &f, int s, const double *rec, i64 fpl, double fv[12]) {
  const int TA = 1 - A;
  const double mub = rec[FS_MU * fpl], Db = rec[FS_D * fpl];
  const double mun = rec[(A == 0 ? FS_GMX : FS_GMY) * fpl];
  const double mut = rec[(A == 0 ? FS_GMY : FS_GMX) * fpl];
  const double phn = rec[(A == 0 ? FS_GFX : FS_GFY) * fpl];
  const double pht = rec[(A == 0 ? FS_GFY : FS_GFX) * fpl];
  const double pn = rec[(A == 0 ? FS_GPX : FS_GPY) * fpl];
  const double pt = rec[(A == 0 ? FS_GPY : FS_GPX) * fpl];
  fv[0] += f.wgt * mub + f.sg * mun;
  fv[1] += f.wgt * Db;
  fv[2] += f.sg * phn;
  fv[3] += f.sg * pn;
  fv[4 + TA] += f.wgt * mut;
  fv[6 + TA] += f.wgt * pht;
  fv[8 + TA] += f.wgt * pt;
  // a face's body-force partials are counted once: on side L, or the fluid side
  if (f.wall || s == 0) {
    fv[10] += rec[FS_GX * fpl];
    fv[11] += rec[FS_GY * fpl];
  }
}

// Faces of cell (i, j): it is side R of its W and S faces and side L of its
// E and N faces (a wall face has only the fluid side).
struct CellFaces {
  int iw, ie, js, jn;
  i64 fw, fe, fs, fn;
};

DFN CellFaces cell_faces(const Consts &K, int i, int j) {
  CellFaces f;
  f.iw = i;
  f.ie = (K.ax[0].bc == 0 && i == K.nx - 1) ? 0 : i + 1;
  f.js = j;
  f.jn = (K.ax[1].bc == 0 && j == K.ny - 1) ? 0 : j + 1;
  f.fw = (i64)j * K.nfx + f.iw;
  f.fe = (i64)j * K.nfx + f.ie;
  f.fs = (i64)f.js * K.ld + i;
  f.fn = (i64)f.jn * K.ld + i;
  return f;
}

// Adjoint of the population gradients and of Step 2 (eqs. relations1 and
// relations2), plus the face-field adjoints of each cell's faces: writes the
// adjoint of tilde (before the macro part) and the cell-field adjoints.
// One workgroup per tile, one thread per cell of the tile and its one-cell
// ring.  For each velocity every thread gathers the adjoints of its cell's
// f and g population gradients from the bar adjoints of the cell's four
// faces into LDS (two buffers alternating by velocity, so one barrier per
// velocity); a tile cell's bar+ adjoint is then the 4/3 bar+ part of tilde+,
// its four faces' reconstruction, and the transposed gradient stencils over
// its neighbours' gathered values.
template <class S>
struct AdjCellLds {
  double g[2][2][2][S::WY][S::WX];  // [buffer][gradient axis][f, g][y][x]
};

template <class S>
struct AdjCellTile {
  static_assert(S::RG == 1, "one thread per cell of the tile and a one-cell ring");
  const Consts &K;
  const Work &w;  // the step's tape
  const AdjWork &a;
  const double *st;  // state before the step (FP64)
  int x0, y0;
  AdjCellLds<S> *L;
  // one thread's registers across the phases
  struct St {
    int i, j, lx, ly;  // global cell (i < 0: outside a wall domain), window position
    bool own;          // a cell of the tile
    CellFaces F;
    FaceSide fs[4];
    double bb[2][4];  // face bar adjoints of the current f and g at W, E, S, N
    double nb[2][4];  // the same for the next velocity (loaded ahead)
    double nnb[2][4];  // and for the one after it
    double lf, lg, sf;  // lam of the current f and g, and the current f~
    int ox[3], oy[3];  // window offsets of the transpose stencils' cells
    double wx[3], wy[3];
    Mac<double> m, mb;
    double tf, uu, den, fca, fcb, fcc, fcab, fcbb, fccb, uub;
  };
  DFN static int chk(int v, int lim) {
#ifdef DUGKS2P_WINDOW_CHECK
    if (v < 0 || v >= lim) {
      printf("adjoint cell window check: %d outside [0, %d)\n", v, lim);
      fflush(stdout);
      abort();
    }
#else
    (void)lim;
#endif
    return v;
  }
  DFN void setup(int tid, St &s) const {
    s.lx = tid % S::WX;
    s.ly = tid / S::WX;
    const TileP0<S, AdjCellLds<S>> p{K, w, x0, y0, L};
    s.i = p.gcol(x0 - 1 + s.lx, K.nx, K.ax[0].bc);
    s.j = p.gcol(y0 - 1 + s.ly, K.ny, K.ax[1].bc);
    s.own = s.lx >= 1 && s.lx <= S::TX && s.ly >= 1 && s.ly <= S::TY &&
            x0 + s.lx - 1 < K.nx && y0 + s.ly - 1 < K.ny;
    if (s.i < 0 || s.j < 0) {
      s.i = -1;
      s.own = false;
      return;
    }
    s.F = cell_faces(K, s.i, s.j);
    s.fs[0] = face_side<0>(K, s.F.iw, 1);
    s.fs[1] = face_side<0>(K, s.F.ie, 0);
    s.fs[2] = face_side<1>(K, s.F.js, 1);
    s.fs[3] = face_side<1>(K, s.F.jn, 0);
    load_bb(s.F, 0, s.bb);
    load_bb(s.F, 1, s.nb);
    if (!s.own) return;
    const i64 c = (i64)s.j * K.ld + s.i;
    // the transpose stencils' cells are lo(c), c, hi(c) along each axis: the
    // window neighbours, or the cell itself where lo or hi is the cell
    const TW tx = stencil_tw(K, 0, K.ax[0].pg, s.i, s.j), ty = stencil_tw(K, 1, K.ax[1].pg, s.i, s.j);
    s.ox[0] = ax_lo(K.ax[0], s.i) == s.i ? 0 : -1;
    s.ox[1] = 0;
    s.ox[2] = ax_hi(K.ax[0], s.i) == s.i ? 0 : 1;
    s.oy[0] = ax_lo(K.ax[1], s.j) == s.j ? 0 : -1;
    s.oy[1] = 0;
    s.oy[2] = ax_hi(K.ax[1], s.j) == s.j ? 0 : 1;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      s.wx[e] = tx.w[e];
      s.wy[e] = ty.w[e];
    }
    cell_mac(K, w, c, s.m);
    mac_zero(s.mb);
    s.tf = w.tauf[c];
    s.uu = s.m.ux * s.m.ux + s.m.uy * s.m.uy;
    s.den = 1.0 / (2.0 * s.tf + K.dt);
    s.fca = (2.0 * s.tf - K.h) * s.den;
    s.fcb = 3.0 * K.h * s.den;
    s.fcc = 3.0 * s.tf * K.h * s.den;
    s.fcab = s.fcbb = s.fccb = s.uub = 0.0;
  }
  // the face bar adjoints of velocity i2's f and g at the cell's four faces
  DFN void load_bb(const CellFaces &F, int i2, double bb[2][4]) const {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int q = 9 * k + i2;
      bb[k][0] = a.xs[(FS_B + q) * K.xplane + F.fw];
      bb[k][1] = a.xs[(FS_B + q) * K.xplane + F.fe];
      bb[k][2] = a.ys[(FS_B + q) * K.yplane + F.fs];
      bb[k][3] = a.ys[(FS_B + q) * K.yplane + F.fn];
    }
  }
  // gradient adjoints of the f and g populations of velocity i2;
  // the cell's own inputs of the cell phase are loaded here, ahead of the
  // barrier
  DFN void gather(int i2, St &s) const {
    if (s.i < 0) return;
    const int b = i2 & 1;
    if (s.own) {
      const i64 c = (i64)s.j * K.ld + s.i;
      s.lf = a.lam[i2 * K.plane + c];
      s.lg = a.lam[(9 + i2) * K.plane + c];
      s.sf = st[i2 * K.plane + c];
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int q = 9 * k + i2;
      double g[2] = {0.0, 0.0};
      face_grad_back<0>(K, s.fs[0], q, s.bb[k][0], g);
      face_grad_back<0>(K, s.fs[1], q, s.bb[k][1], g);
      face_grad_back<1>(K, s.fs[2], q, s.bb[k][2], g);
      face_grad_back<1>(K, s.fs[3], q, s.bb[k][3], g);
      L->g[b][0][k][s.ly][s.lx] = g[0];
      L->g[b][1][k][s.ly][s.lx] = g[1];
    }
  }
  // bar+ adjoint of population k (0: f, 1: g) of velocity i2: tilde+'s 4/3
  // bar+, the four faces' reconstruction, the transposed gradient stencils
  DFN double ob_of(int i2, int k, const St &s) const {
    const int q = 9 * k + i2, b = i2 & 1;
    double ab = (4.0 / 3.0) * (k == 0 ? s.lf : s.lg);
    ab += face_ab_back<0>(K, s.fs[0], q, s.bb[k][0]);
    ab += face_ab_back<0>(K, s.fs[1], q, s.bb[k][1]);
    ab += face_ab_back<1>(K, s.fs[2], q, s.bb[k][2]);
    ab += face_ab_back<1>(K, s.fs[3], q, s.bb[k][3]);
    const double(*gx)[S::WX] = L->g[b][0][k];
    const double(*gy)[S::WX] = L->g[b][1][k];
    const double tx = s.wx[0] * gx[s.ly][chk(s.lx + s.ox[0], S::WX)] +
                      s.wx[1] * gx[s.ly][s.lx] +
                      s.wx[2] * gx[s.ly][chk(s.lx + s.ox[2], S::WX)];
    const double ty = s.wy[0] * gy[chk(s.ly + s.oy[0], S::WY)][s.lx] +
                      s.wy[1] * gy[s.ly][s.lx] +
                      s.wy[2] * gy[chk(s.ly + s.oy[2], S::WY)][s.lx];
    return ab + tx + ty;
  }
  // Step 2 adjoint of velocity i2 at a tile cell; every thread first issues
  // the loads of the face values two velocities ahead
  DFN void cell(int i2, St &s) const {
    if (s.i < 0) return;
    if (i2 < 7) load_bb(s.F, i2 + 2, s.nnb);
    if (s.own) {
      const i64 c = (i64)s.j * K.ld + s.i, P = K.plane;
      const int qf = i2, qg = 9 + i2;
      double feq, geq, ff, fg;
      point_eq1<double>(K, s.m, s.uu, i2, feq, geq, ff, fg);
      const double obf = ob_of(i2, 0, s);
      const double obg = ob_of(i2, 1, s);
      a.out[qf * P + c] = s.fca * obf - (1.0 / 3.0) * s.lf;
      a.out[qg * P + c] = K.gca * obg - (1.0 / 3.0) * s.lg;
      s.fcab += s.sf * obf;
      s.fcbb += feq * obf;
      s.fccb += ff * obf;
      point_eq1_vjp(K, s.m, s.uu, i2, s.fcb * obf, K.gcb * obg, s.fcc * obf, K.gcc * obg, s.mb,
                    s.uub);
    }
    if (i2 < 8) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          s.bb[k][e] = s.nb[k][e];
          s.nb[k][e] = s.nnb[k][e];
        }
    }
  }
  // the cell-field adjoints of a tile cell, after the last velocity
  DFN void finish(St &s) const {
    if (!s.own) return;
    const i64 c = (i64)s.j * K.ld + s.i, P = K.plane;
    Mac<double> &mb = s.mb;
    const Mac<double> &m = s.m;
    const double tf = s.tf, den = s.den;
    mb.ux += 2.0 * m.ux * s.uub;
    mb.uy += 2.0 * m.uy * s.uub;
    const double denb = (2.0 * tf - K.h) * s.fcab + 3.0 * K.h * s.fcbb + 3.0 * tf * K.h * s.fccb;
    const double tfb = 2.0 * den * s.fcab + 3.0 * K.h * den * s.fccb - 2.0 * den * den * denb;
    double dtp, dtr;
    tauf_grad(K, m.phi, m.rho, dtp, dtr);
    double fv[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) fv[e] = 0.0;
    face_field_back<0>(s.fs[0], 1, a.xs + s.F.fw, K.xplane, fv);
    face_field_back<0>(s.fs[1], 0, a.xs + s.F.fe, K.xplane, fv);
    face_field_back<1>(s.fs[2], 1, a.ys + s.F.fs, K.yplane, fv);
    face_field_back<1>(s.fs[3], 0, a.ys + s.F.fn, K.yplane, fv);
    double *fb = a.fb;
    fb[FB_MU * P + c] = fv[0] + mb.mu;
    fb[FB_D * P + c] = fv[1] + mb.D;
    fb[FB_PHI * P + c] = fv[2] + (mb.phi + dtp * tfb);
    fb[FB_P * P + c] = fv[3] + mb.p;
    fb[FB_DMUX * P + c] = fv[4];
    fb[FB_DMUY * P + c] = fv[5];
    fb[FB_DPHX * P + c] = fv[6] + K.drho * mb.grx;
    fb[FB_DPHY * P + c] = fv[7] + K.drho * mb.gry;
    fb[FB_DPX * P + c] = fv[8] + mb.gpx;
    fb[FB_DPY * P + c] = fv[9] + mb.gpy;
    fb[FB_GX * P + c] = fv[10];
    fb[FB_GY * P + c] = fv[11];
    fb[FB_RHO * P + c] = mb.rho + dtr * tfb - K.cs2 * m.icr * m.icr * mb.icr;
    fb[FB_UX * P + c] = mb.ux;
    fb[FB_UY * P + c] = mb.uy;
    fb[FB_FX * P + c] = mb.Fx;
    fb[FB_FY * P + c] = mb.Fy;
  }
};

#if defined(__HIPCC__)
template <class S>
__global__ __launch_bounds__(NTHR) void k_adj_cells(Consts K, Work w, AdjWork a,
                                                    const double *st, int ntx, int ntiles) {
  __shared__ AdjCellLds<S> L;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const AdjCellTile<S> ct{K, w, a, st, (tile % ntx) * S::TX, (tile / ntx) * S::TY, &L};
  typename AdjCellTile<S>::St s;
  ct.setup(threadIdx.x, s);
#pragma unroll 1
  for (int i2 = 0; i2 < 9; ++i2) {
    ct.gather(i2, s);
    __syncthreads();
    ct.cell(i2, s);
  }
  ct.finish(s);
}
#endif

// Adjoint of the cell macros (eqs. u, P; F; D): the p adjoint is completed
// by the transpose of its gradient stencil.  init = 1: Step 1 form (u, p
// given, not differentiated).
struct FAdjMacro {
  Consts K;
  Work w;
  AdjWork a;
  int init;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i, P = K.plane;
    double *fb = a.fb;
    const double ph = w.phi[c], rh = w.rho[c];
    const double dmux = w.dmux[c], dmuy = w.dmuy[c], D = w.D[c];
    double Fxb = fb[FB_FX * P + c], Fyb = fb[FB_FY * P + c], Db = fb[FB_D * P + c];
    double rhob = 0.0, phib = 0.0;
    if (!init) {
      const TW tx = stencil_tw(K, 0, K.ax[0].d1, i, j), ty = stencil_tw(K, 1, K.ax[1].d1, i, j);
      const double pb = fb[FB_P * P + c] + tw_apply(tx, fb + FB_DPX * P) +
                        tw_apply(ty, fb + FB_DPY * P);
      const double ux = w.ux[c], uy = w.uy[c];
      const double grx = K.drho * w.dphx[c], gry = K.drho * w.dphy[c];
      const double uxb = fb[FB_UX * P + c] + K.hdtcs2 * grx * pb;
      const double uyb = fb[FB_UY * P + c] + K.hdtcs2 * gry * pb;
      fb[FB_DPHX * P + c] += K.drho * K.hdtcs2 * ux * pb;
      fb[FB_DPHY * P + c] += K.drho * K.hdtcs2 * uy * pb;
      rhob += -K.hdtcs2 * K.gam * D * pb;
      Db += -K.hdtcs2 * K.gam * rh * pb;
      fb[FB_S0 * P + c] = pb;
      const double icr = 1.0 / (K.cs2 * rh);
      fb[FB_JX * P + c] = icr * uxb;
      fb[FB_JY * P + c] = icr * uyb;
      Fxb += K.hdtcs2 * icr * uxb;
      Fyb += K.hdtcs2 * icr * uyb;
      // u = (j + hdtcs2 F) icr, so j + hdtcs2 F = u / icr = u cs2 rho
      const double icrb = ux * (K.cs2 * rh) * uxb + uy * (K.cs2 * rh) * uyb;
      rhob += -K.cs2 * icr * icr * icrb;
    } else {
      fb[FB_S0 * P + c] = fb[FB_JX * P + c] = fb[FB_JY * P + c] = 0.0;
    }
    // F = -phi grad mu + (rho - rho_ref) g
    phib += -dmux * Fxb - dmuy * Fyb;
    fb[FB_DMUX * P + c] += -ph * Fxb;
    fb[FB_DMUY * P + c] += -ph * Fyb;
    rhob += K.gx * Fxb + K.gy * Fyb;
    fb[FB_GX * P + c] += (rh - K.rho_ref) * Fxb;
    fb[FB_GY * P + c] += (rh - K.rho_ref) * Fyb;
    // D = lambda lap mu
    fb[FB_LAPMU * P + c] = K.mobility * Db;
    fb[FB_PHI * P + c] += phib;
    fb[FB_RHO * P + c] += rhob;
  }
};

// Adjoint of eq. chemicalpotential: the mu adjoint is completed by the
// transposes of grad mu and lap mu; kappa partial (beta fixed).
struct FAdjMu {
  Consts K;
  Work w;
  AdjWork a;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i, P = K.plane;
    double *fb = a.fb;
    const TW t1x = stencil_tw(K, 0, K.ax[0].d1, i, j), t1y = stencil_tw(K, 1, K.ax[1].d1, i, j);
    const TW t2x = stencil_tw(K, 0, K.ax[0].d2, i, j), t2y = stencil_tw(K, 1, K.ax[1].d2, i, j);
    const double mub = fb[FB_MU * P + c] + tw_apply(t1x, fb + FB_DMUX * P) +
                       tw_apply(t1y, fb + FB_DMUY * P) + tw_apply(t2x, fb + FB_LAPMU * P) +
                       tw_apply(t2y, fb + FB_LAPMU * P);
    const double ph = w.phi[c];
    const double a1 = ph - K.phi_a, b1 = ph - K.phi_b, m1 = ph - K.phimid;
    const double lap = stx(K, K.ax[0].d2, w.phi, i, j) + sty(K, K.ax[1].d2, w.phi, i, j);
    fb[FB_PHI * P + c] += K.c4b * (b1 * m1 + a1 * m1 + a1 * b1) * mub;
    fb[FB_LAPPHI * P + c] = -K.kappa * mub;
    fb[FB_KAP * P + c] = -lap * mub;
  }
};

// Adjoint of eq. phi and eq. oderrho with the transposes of grad phi and
// lap phi.  Adds the adjoint of the populations through the cell sums (a
// step) or writes the adjoint of phi0 (Step 1); accumulates the parameter
// partials of the cell.
struct FAdjPhi {
  Consts K;
  AdjWork a;
  double *phi0b;  // Step 1 form: adjoint of phi0 ([ny][nx]); NULL for a step
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i, P = K.plane;
    const double *fb = a.fb;
    const TW t1x = stencil_tw(K, 0, K.ax[0].d1, i, j), t1y = stencil_tw(K, 1, K.ax[1].d1, i, j);
    const TW t2x = stencil_tw(K, 0, K.ax[0].d2, i, j), t2y = stencil_tw(K, 1, K.ax[1].d2, i, j);
    const double phb = fb[FB_PHI * P + c] + K.drho * fb[FB_RHO * P + c] +
                       tw_apply(t1x, fb + FB_DPHX * P) + tw_apply(t1y, fb + FB_DPHY * P) +
                       tw_apply(t2x, fb + FB_LAPPHI * P) + tw_apply(t2y, fb + FB_LAPPHI * P);
    a.pacc[c] += fb[FB_KAP * P + c];
    a.pacc[P + c] += fb[FB_GX * P + c];
    a.pacc[2 * P + c] += fb[FB_GY * P + c];
    if (phi0b) {
      phi0b[(i64)j * K.nx + i] = phb;
      return;
    }
    const double s0b = fb[FB_S0 * P + c], jxb = fb[FB_JX * P + c], jyb = fb[FB_JY * P + c];
#pragma unroll
    for (int q = 0; q < 9; ++q) a.out[q * P + c] += s0b + K.xi0[q] * jxb + K.xi1[q] * jyb;
#pragma unroll
    for (int q = 9; q < 18; ++q) a.out[q * P + c] += phb;
  }
};

// Step 1 adjoint at a cell: tilde = eq - (dt/2) F with u, p given.
struct FAdjInit {
  Consts K;
  Work w;
  AdjWork a;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i, P = K.plane;
    Mac<double> m, mb;
    cell_mac(K, w, c, m);
    mac_zero(mb);
    const double uu = m.ux * m.ux + m.uy * m.uy;
    double uub = 0.0;
    for (int q = 0; q < 9; ++q)
      point_eq1_vjp(K, m, uu, q, a.lam[q * P + c], a.lam[(9 + q) * P + c],
                    -K.hdt * a.lam[q * P + c], -K.hdt * a.lam[(9 + q) * P + c], mb, uub);
    double *fb = a.fb;
    for (int f = 0; f < NFB; ++f) fb[f * P + c] = 0.0;
    fb[FB_PHI * P + c] = mb.phi;
    fb[FB_RHO * P + c] = mb.rho - K.cs2 * m.icr * m.icr * mb.icr;
    fb[FB_MU * P + c] = mb.mu;
    fb[FB_DPHX * P + c] = K.drho * mb.grx;
    fb[FB_DPHY * P + c] = K.drho * mb.gry;
    fb[FB_D * P + c] = mb.D;
    fb[FB_FX * P + c] = mb.Fx;
    fb[FB_FY * P + c] = mb.Fy;
  }
};

// Sequences.  The forward arrays (staged stages up to Step 2) of the step
// must be in w; lam = adjoint after the step, out = adjoint before it.
template <class Ex>
void seq_adjoint_step(Ex &ex, const Consts &K, const Work &w, const AdjWork &a,
                      const double *st) {
  ex.adj_faces(K, w, a);
  ex.adj_cells(K, w, a, st);
  ex.grid(FAdjMacro{K, w, a, 0}, K.nx, K.ny);
  ex.grid(FAdjMu{K, w, a}, K.nx, K.ny);
  ex.grid(FAdjPhi{K, a, nullptr}, K.nx, K.ny);
}

// Step 1 adjoint: forward init fields must be in w; lam = adjoint of the
// initial state; phi0b receives the adjoint of phi0.
template <class Ex>
void seq_adjoint_init(Ex &ex, const Consts &K, const Work &w, const AdjWork &a, double *phi0b) {
  ex.grid(FAdjInit{K, w, a}, K.nx, K.ny);
  ex.grid(FAdjMacro{K, w, a, 1}, K.nx, K.ny);
  ex.grid(FAdjMu{K, w, a}, K.nx, K.ny);
  ex.grid(FAdjPhi{K, a, phi0b}, K.nx, K.ny);
}

// ---------------------------------------------------------------------------
// Reverse sweep over a segment of steps, with the forward tape.
// ---------------------------------------------------------------------------

// Rows without padding: every adjoint-side array has the layout
// [plane][ny][nx] of the population export.
inline void pack_rows(Consts &K) {
  K.ld = K.nx;
  K.plane = (i64)K.ny * K.nx;
  K.yplane = (i64)K.nfy * K.nx;
}

// Per step of a segment the tape holds the 16 cell fields of the staged
// step and bar+ (18 planes); the population state of every step but the
// first is kept too.
enum { TAPE_FIELDS = 16, ADJ_RED_BLOCKS = 256 };

struct AdjLayout {
  size_t tables[2];
  size_t field_bytes;  // one cell plane, padded
  size_t slot_bytes;   // one tape slot: 16 fields + bar+
  size_t state_bytes;  // 18 planes
  size_t states, tape, dummy, facex, facey, fwork, lam[2], xs, ys, fb, pacc, red;
  size_t total;
  int mseg;
};

inline AdjLayout make_adj_layout(const Consts &K, const AxisHost &ax, const AxisHost &ay,
                                 int mseg) {
  AdjLayout L;
  const size_t P = (size_t)K.plane;
  size_t off = 0;
  L.mseg = mseg;
  L.tables[0] = off;
  off += align256(axis_table_bytes(ax));
  L.tables[1] = off;
  off += align256(axis_table_bytes(ay));
  L.field_bytes = align256(sizeof(double) * P);
  L.state_bytes = align256(18 * sizeof(double) * P);
  L.slot_bytes = TAPE_FIELDS * L.field_bytes + L.state_bytes;
  L.states = off;
  off += (size_t)mseg * L.state_bytes;
  L.tape = off;
  off += (size_t)mseg * L.slot_bytes;
  L.dummy = off;
  off += 3 * L.field_bytes;
  L.facex = off;
  off += align256(18 * sizeof(double) * (size_t)K.xplane);
  L.facey = off;
  off += align256(18 * sizeof(double) * (size_t)K.yplane);
  L.fwork = off;  // phi and the f~ sums of the recomputed states (two sets)
  off += 8 * L.field_bytes;
  for (int b = 0; b < 2; ++b) {
    L.lam[b] = off;
    off += L.state_bytes;
  }
  L.xs = off;
  off += align256(NFS * sizeof(double) * (size_t)K.xplane);
  L.ys = off;
  off += align256(NFS * sizeof(double) * (size_t)K.yplane);
  L.fb = off;
  off += align256(NFB * sizeof(double) * P);
  L.pacc = off;
  off += align256(3 * sizeof(double) * P);
  L.red = off;  // per-workgroup partial sums of the parameter reduction
  off += align256(3 * sizeof(double) * ADJ_RED_BLOCKS);
  L.total = off;
  return L;
}

struct AdjBufs {
  AdjLayout L;
  unsigned char *base;
  double *state(int n) const { return (double *)(base + L.states + (size_t)n * L.state_bytes); }
  Work tape(int n) const {
    unsigned char *s = base + L.tape + (size_t)n * L.slot_bytes;
    Work w;
    memset(&w, 0, sizeof w);
    double **f[TAPE_FIELDS] = {&w.phi, &w.rho, &w.mu, &w.dphx, &w.dphy, &w.dmux, &w.dmuy, &w.D,
                               &w.Fx,  &w.Fy,  &w.ux, &w.uy,   &w.p,    &w.dpx,  &w.dpy,  &w.tauf};
    for (int k = 0; k < TAPE_FIELDS; ++k) *f[k] = (double *)(s + k * L.field_bytes);
    w.barp = (double *)(s + TAPE_FIELDS * L.field_bytes);
    w.s0 = (double *)(base + L.dummy);
    w.jx = (double *)(base + L.dummy + L.field_bytes);
    w.jy = (double *)(base + L.dummy + 2 * L.field_bytes);
    w.facex = (double *)(base + L.facex);
    w.facey = (double *)(base + L.facey);
    return w;
  }
  // work fields of the fused step (its own, so the tape is untouched)
  // phi and the f~ sums of the state being recomputed (phi, s0, jx, jy) and
  // of the state the tile kernel writes (phin ..); the other fields are unset
  Work fused_work() const {
    Work w;
    memset(&w, 0, sizeof w);
    double **f[8] = {&w.phi, &w.s0, &w.jx, &w.jy, &w.phin, &w.s0n, &w.jxn, &w.jyn};
    for (int k = 0; k < 8; ++k) *f[k] = (double *)(base + L.fwork + k * L.field_bytes);
    return w;
  }
  double *lam(int b) const { return (double *)(base + L.lam[b]); }
  AdjWork adj(int in) const {
    AdjWork a;
    a.lam = lam(in);
    a.out = lam(1 - in);
    a.xs = (double *)(base + L.xs);
    a.ys = (double *)(base + L.ys);
    a.fb = (double *)(base + L.fb);
    a.pacc = (double *)(base + L.pacc);
    return a;
  }
};

// dst[q][c] = src[q][c] (or 0 if src is NULL) for q < nq, packed planes.
struct FCopyPlanes {
  Consts K;
  const double *src;
  double *dst;
  int nq;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i;
    for (int q = 0; q < nq; ++q) dst[q * K.plane + c] = src ? src[q * K.plane + c] : 0.0;
  }
};

// Reverse sweep of one segment: recompute nsteps steps from pops0 (the
// state at the segment start) into the tape, then carry the adjoint of the
// state after the segment (lam_end) back to its start (lam_begin).  The
// per-cell kappa / g partials of the segment are left in pacc.
template <class Ex>
void seq_adjoint_segment(Ex &ex, const Consts &K, const AdjBufs &B, const double *pops0,
                         int nsteps, const double *lam_end, double *lam_begin) {
  const AdjWork a0 = B.adj(0);
  ex.grid(FCopyPlanes{K, nullptr, a0.pacc, 3}, K.nx, K.ny);
  ex.grid(FCopyPlanes{K, lam_end, B.lam(0), 18}, K.nx, K.ny);
  Work wf = B.fused_work();
  for (int n = 0; n < nsteps; ++n) {
    const Work w = B.tape(n);
    const double *src = n == 0 ? pops0 : B.state(n);
    const IoF64 a{(double *)src, K.plane};
    // phi and the f~ sums of the state: computed for the checkpoint, then
    // kept by the tile kernel for each state it writes
    if (n == 0) {
      if (K.unit)
        ex.grid(FPhiSums<IoF64, true>{K, wf, a}, K.nx, K.ny);
      else
        ex.grid(FPhiSums<IoF64, false>{K, wf, a}, K.nx, K.ny);
    }
    // the tape: every cell field of the step from the macro kernel in tape
    // mode (the arithmetic of the staged stages), then grad p and tau_f, and
    // bar+.  bar+ comes from the tile kernel, which computes it with the
    // same arithmetic (FCell only for the segment's last step, which has no
    // fused step)
    ex.macros_tape(K, wf, w);
    if (n + 1 == nsteps) {
      ex.grid(FCell<double, double>{K, w, src}, K.nx, K.ny);
    } else {
      ex.grid(FCellFields<double>{K, w}, K.nx, K.ny);
      // the next state from the tile kernel (bitwise equal to the staged
      // step), reading the tape's fields; the new state's sums go to the
      // spare planes of wf
      Work wt = w;
      wt.phin = wf.phin;
      wt.s0n = wf.s0n;
      wt.jxn = wf.jxn;
      wt.jyn = wf.jyn;
      const IoF64 b{B.state(n + 1), K.plane};
      // (tilde+ in LDS: the segment's states and tape keep the MALL busy)
      with_fused_kernel(DUGKS2P_TILE_SQUARE, K, false, [&](auto u, auto sh, auto v, auto tg) {
        ex.template tiles<IoF64, double, decltype(u)::value, decltype(sh), decltype(v)::value,
                          decltype(tg)::value>(K, wt, a, b);
      });
      swap_sums(wf);
    }
  }
  int cur = 0;
  for (int n = nsteps - 1; n >= 0; --n) {
    seq_adjoint_step(ex, K, B.tape(n), B.adj(cur), n == 0 ? pops0 : B.state(n));
    cur = 1 - cur;
  }
  ex.grid(FCopyPlanes{K, B.lam(cur), lam_begin, 18}, K.nx, K.ny);
}

// Adjoint of Step 1: recompute the initial cell fields from phi0, u0, p0,
// then carry lam0 (adjoint of the initial populations) to phi0_grad.
template <class Ex>
void seq_adjoint_initial(Ex &ex, const Consts &K, const AdjBufs &B, const double *phi0,
                         const double *ux0, const double *uy0, const double *p0,
                         const double *lam0, double *phi0_grad) {
  const Work w = B.tape(0);
  const AdjWork a = B.adj(0);
  ex.grid(FCopyPlanes{K, nullptr, a.pacc, 3}, K.nx, K.ny);
  ex.grid(FCopyPlanes{K, lam0, B.lam(0), 18}, K.nx, K.ny);
  ex.grid(FInit0{K, w, phi0, ux0, uy0, p0}, K.nx, K.ny);
  ex.grid(FMu{K, w}, K.nx, K.ny);
  ex.grid(FInit1{K, w}, K.nx, K.ny);
  seq_adjoint_init(ex, K, w, a, phi0_grad);
}

}  // namespace DUGKS2P_NS

#if defined(__clang__)
#pragma clang fp contract(off)
#endif
