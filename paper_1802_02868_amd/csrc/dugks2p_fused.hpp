// dugks2p_fused.hpp -- the step as two launches, plus a third after a
// fresh state:
//   0. FPhiSums: phi = sum g~ and the f~ sums (one thread per cell), only
//                when the state did not come from a tile kernel, which
//                writes these sums of the state it stores;
//   1. k_macros: mu, D, F, u, p over 64 x 4 blocks of cells (FMacF is the
//                same arithmetic one thread per cell);
//   2. tile kernel: for a tile (14 x 14 by default), Step 2 (bar+) on the
//                tile and a one-cell ring (two cells for UPWIND) into LDS,
//                Steps 3-4 at every face of the tile (each face once), flux
//                exchange through LDS, Steps 5-6.
// The populations are read once per step from HBM (ring cells from L2) and
// written once.  Arithmetic is the same code as the staged stages, so FP64
// results are bitwise identical to them.
//
// The tile work is written as phases separated by workgroup barriers; each
// phase takes the thread index and a per-thread state, so the host build can
// run the phases thread by thread with the same barrier semantics.
#pragma once

#include <type_traits>

#include "dugks2p_dev.hpp"

// DUGKS2P_WINDOW_CHECK turns every LDS-window access of the tile code into a
// bounds-checked one that aborts the process.  It exists for the host build
// of the kernel logic (tests/emu); a GPU build must never carry it.
#if defined(DUGKS2P_WINDOW_CHECK)
#if defined(__HIP_DEVICE_COMPILE__)
#error "DUGKS2P_WINDOW_CHECK is for the host build of the kernel logic only"
#endif
#include <stdio.h>
#include <stdlib.h>
#endif

namespace DUGKS2P_NS {

enum { NTHR = 256 };  // threads of a tile workgroup

// Tile shape: TX x TY cells, an RG-cell ring for bar+ (the WX x WY window,
// one thread per window cell) and an (RG + 1)-cell ring for the cell scalars
// (the SX x SY window).  SM, FM: lengths of the per-axis weight and face
// tables.
template <int TX_, int TY_, int RG_ = 1>
struct Tile {
  enum {
    TX = TX_, TY = TY_, RG = RG_, WX = TX + 2 * RG, WY = TY + 2 * RG, SX = WX + 2, SY = WY + 2,
    SM = SX > SY ? SX : SY, FM = (TX > TY ? TX : TY) + 1
  };
  static_assert(WX * WY == NTHR, "one thread per bar+ window cell");
};
typedef Tile<14, 14> TileSq;   // square tiles (the default)
typedef Tile<30, 6> TileWide;  // wide tiles (long rows)
typedef Tile<6, 30> TileTall;  // tall tiles (long columns)
// UPWIND reconstruction: a face takes bar+ and both of its gradients at the
// upwind cell, so the bar+ window reaches two cells beyond the tile
typedef Tile<12, 12, 2> TileUpw;

// x-face flux slots: directions with e_x != 0 (1, 3, 5, 6, 7, 8); y-face:
// e_y != 0 (2, 4, 5, 6, 7, 8).  -1 = no flux across that face.
DFN int xslot(int i) { return i == 1 ? 0 : (i == 3 ? 1 : (i >= 5 ? i - 3 : -1)); }
DFN int yslot(int i) { return i == 2 ? 0 : (i == 4 ? 1 : (i >= 5 ? i - 3 : -1)); }

// phi, s0 = sum f~, jx, jy = sum xi f~ (the sums of eq. phi and eq. u, P).
template <class IO, bool U>
DFN void phi_sums_at(const Consts &K, const Work &w, const IO &st, int i, int j) {
  const i64 c = (i64)j * K.ld + i;
  w.phi[c] = st.phi(c);
  double f[9];
  st.load_f(c, f);
  double s0 = 0.0, jx, jy;
#pragma unroll
  for (int q = 0; q < 9; ++q) s0 += f[q];
  xi_sums<double, U>(K, f, jx, jy);
  w.s0[c] = s0;
  w.jx[c] = jx;
  w.jy[c] = jy;
}

template <class IO, bool U = false>
struct FPhiSums {
  Consts K;
  Work w;
  IO st;
  DFN void operator()(int i, int j) const { phi_sums_at<IO, U>(K, w, st, i, j); }
};

// grad mu, D = lambda lap mu, F, eq. u and eq. P at a cell from mu and phi
// at the cell (mc, ph) and its x / y neighbours, the f~ sums s0, jx, jy and
// the App. B first / second derivative weights of its column (a1, a2) and
// row (b1, b2).
struct CellMac {
  double D, Fx, Fy, ux, uy, p;
  double rho, dmux, dmuy, dphx, dphy;  // the intermediates, for the adjoint's tape
};

// F = -phi grad mu + F_b and eq. u at a cell from mu at the cell and its
// neighbours, phi, rho and the f~ sums jx, jy (the part of the cell macros
// that the tile kernel recomputes on its bar+ window).
struct CellFU {
  double dmux, dmuy, Fx, Fy, ux, uy;
};
DFN CellFU force_velocity(const Consts &K, double mc, double mxl, double mxh, double myl,
                          double myh, double ph, double rh, double jx, double jy,
                          const double *a1, const double *b1) {
  CellFU r;
  r.dmux = a1[0] * mxl + a1[1] * mc + a1[2] * mxh;
  r.dmuy = b1[0] * myl + b1[1] * mc + b1[2] * myh;
  r.Fx = -ph * r.dmux + (rh - K.rho_ref) * K.gx;
  r.Fy = -ph * r.dmuy + (rh - K.rho_ref) * K.gy;
  const double icr = 1.0 / (K.cs2 * rh);
  r.ux = (jx + K.hdtcs2 * r.Fx) * icr;
  r.uy = (jy + K.hdtcs2 * r.Fy) * icr;
  return r;
}

DFN CellMac macros_from(const Consts &K, double mc, double mxl, double mxh, double myl,
                        double myh, double ph, double pxl, double pxh, double pyl, double pyh,
                        double s0, double jx, double jy, const double *a1, const double *a2,
                        const double *b1, const double *b2) {
  CellMac r;
  const double lapmu =
      (a2[0] * mxl + a2[1] * mc + a2[2] * mxh) + (b2[0] * myl + b2[1] * mc + b2[2] * myh);
  r.D = K.mobility * lapmu;
  const double rh = rho_of<double>(K, ph);
  r.rho = rh;
  const CellFU fu = force_velocity(K, mc, mxl, mxh, myl, myh, ph, rh, jx, jy, a1, b1);
  r.dmux = fu.dmux;
  r.dmuy = fu.dmuy;
  r.Fx = fu.Fx;
  r.Fy = fu.Fy;
  r.ux = fu.ux;
  r.uy = fu.uy;
  r.dphx = a1[0] * pxl + a1[1] * ph + a1[2] * pxh;
  r.dphy = b1[0] * pyl + b1[1] * ph + b1[2] * pyh;
  const double grx = K.drho * r.dphx;
  const double gry = K.drho * r.dphy;
  r.p = s0 + K.hdtcs2 * (r.ux * grx + r.uy * gry - K.gam * rh * r.D);
  return r;
}

// mu, grad mu, D, F, eq. u and eq. P at a cell (global fields).
DFN void macros_at(const Consts &K, const Work &w, int i, int j) {
  const i64 c = (i64)j * K.ld + i;
  const Axis &X = K.ax[0], &Y = K.ax[1];
  const int il = ax_lo(X, i), ih = ax_hi(X, i), jl = ax_lo(Y, j), jh = ax_hi(Y, j);
  const double mc = mu_at(K, w.phi, i, j);
  const double mxl = mu_at(K, w.phi, il, j), mxh = mu_at(K, w.phi, ih, j);
  const double myl = mu_at(K, w.phi, i, jl), myh = mu_at(K, w.phi, i, jh);
  const i64 r = (i64)j * K.ld;
  const CellMac m = macros_from(K, mc, mxl, mxh, myl, myh, w.phi[c], w.phi[r + il],
                                w.phi[r + ih], w.phi[(i64)jl * K.ld + i],
                                w.phi[(i64)jh * K.ld + i], w.s0[c], w.jx[c], w.jy[c],
                                X.d1 + 3 * i, X.d2 + 3 * i, Y.d1 + 3 * j, Y.d2 + 3 * j);
  w.mu[c] = mc;
  w.D[c] = m.D;
  w.Fx[c] = m.Fx;
  w.Fy[c] = m.Fy;
  w.ux[c] = m.ux;
  w.uy[c] = m.uy;
  w.p[c] = m.p;
}

struct FMacF {
  Consts K;
  Work w;
  DFN void operator()(int i, int j) const { macros_at(K, w, i, j); }
};

DFN int wrapi(int g, int n);
DFN int xcd_tile(int b, int n);

// The same cell macros over a 64 x 4 block of cells, in three phases
// separated by workgroup barriers: P0 stages phi on the block and a two-cell
// ring and the App. B second-derivative weights of the mu window in LDS; P1
// forms mu once on the block and a one-cell ring from them (instead of at
// every cell's four neighbours); P2 forms grad mu, D, F, u and p of the
// block's cells.  The arithmetic and its inputs are those of macros_at.
enum { MBX = 64, MBY = 4 };
struct MacLds {
  double phi[MBY + 4][MBX + 4];
  double mu[MBY + 2][MBX + 2];
  double wx[MBX + 2][3], wy[MBY + 2][3];  // d2 weights of the mu window's columns, rows
};

struct MacBlock {
  const Consts &K;
  const Work &w;
  int x0, y0;
  MacLds *L;
  // tape mode (the adjoint's recomputation): every cell field of the step,
  // phi and rho included, goes to *tape instead of w (phi and the sums are
  // still read from w)
  const Work *tape = nullptr;
  // false (the step): only mu, D and p are written; the tile kernel
  // recomputes F and u of its bar+ window itself.  true: every field
  // (moments, monitors, observables).
  bool fields = true;
  enum { PW = (MBX + 4) * (MBY + 4), NPHI = (PW + MBX * MBY - 1) / (MBX * MBY) };
  static_assert((MBX + 2) + (MBY + 2) <= MBX * MBY, "weight roles exceed the block");
  // global index of window offset g along an axis, or -1 outside a wall domain
  DFN int gcol(int g, int n, int bc) const {
    if (bc == 0) return wrapi(g, n);
    return (g >= 0 && g < n) ? g : -1;
  }
  // P0: phi of the two-ring window (elements tid, tid + 256, ...) and one
  // weight row per thread of the first MBX + MBY + 4, loads first
  DFN void p0(int tid) const {
    double ph[NPHI];
    int at[NPHI];
#pragma unroll
    for (int k = 0; k < NPHI; ++k) {
      const int e = tid + k * MBX * MBY;
      at[k] = -1;
      if (e >= PW) continue;
      const int lx = e % (MBX + 4), ly = e / (MBX + 4);
      const int gx = gcol(x0 - 2 + lx, K.nx, K.ax[0].bc);
      const int gy = gcol(y0 - 2 + ly, K.ny, K.ax[1].bc);
      if (gx < 0 || gy < 0) continue;
      ph[k] = w.phi[(i64)gy * K.ld + gx];
      at[k] = e;
    }
    double wt[3];
    const int a = tid < MBX + 2 ? 0 : 1, pos = a == 0 ? tid : tid - (MBX + 2);
    const int g = tid < (MBX + 2) + (MBY + 2)
                      ? gcol((a == 0 ? x0 : y0) - 1 + pos, K.ax[a].n, K.ax[a].bc)
                      : -1;
    if (g >= 0) {
#pragma unroll
      for (int m = 0; m < 3; ++m) wt[m] = K.ax[a].d2[3 * g + m];
    }
#pragma unroll
    for (int k = 0; k < NPHI; ++k)
      if (at[k] >= 0) L->phi[at[k] / (MBX + 4)][at[k] % (MBX + 4)] = ph[k];
    if (g >= 0) {
#pragma unroll
      for (int m = 0; m < 3; ++m) (a == 0 ? L->wx[pos] : L->wy[pos])[m] = wt[m];
    }
  }
  // P1: mu on the one-ring window; a stencil neighbour is the adjacent
  // window position, or the cell itself at a wall
  DFN void p1(int tid) const {
    const Axis &X = K.ax[0], &Y = K.ax[1];
    for (int e = tid; e < (MBX + 2) * (MBY + 2); e += MBX * MBY) {
      const int mx = e % (MBX + 2), my = e / (MBX + 2);
      const int gx = gcol(x0 - 1 + mx, K.nx, X.bc);
      const int gy = gcol(y0 - 1 + my, K.ny, Y.bc);
      if (gx < 0 || gy < 0) continue;
      const int px = mx + 1, py = my + 1;
      const double ph = L->phi[py][px];
      const double xl = (X.bc != 0 && gx == 0) ? ph : L->phi[py][px - 1];
      const double xh = (X.bc != 0 && gx == X.n - 1) ? ph : L->phi[py][px + 1];
      const double yl = (Y.bc != 0 && gy == 0) ? ph : L->phi[py - 1][px];
      const double yh = (Y.bc != 0 && gy == Y.n - 1) ? ph : L->phi[py + 1][px];
      L->mu[my][mx] = mu_from(K, ph, xl, xh, yl, yh, L->wx[mx], L->wy[my]);
    }
  }
  // P2: the cell macros of the block's cells
  DFN void p2(int tid) const {
    const int tx = tid % MBX, ty = tid / MBX;
    const int i = x0 + tx, j = y0 + ty;
    if (i >= K.nx || j >= K.ny) return;
    const Axis &X = K.ax[0], &Y = K.ax[1];
    // neighbours: the adjacent window positions, or the cell itself at a wall
    const int sxl = (X.bc != 0 && i == 0) ? 0 : 1, sxh = (X.bc != 0 && i == X.n - 1) ? 0 : 1;
    const int syl = (Y.bc != 0 && j == 0) ? 0 : 1, syh = (Y.bc != 0 && j == Y.n - 1) ? 0 : 1;
    const int mx = tx + 1, my = ty + 1, px = tx + 2, py = ty + 2;
    const i64 c = (i64)j * K.ld + i;
    const double mc = L->mu[my][mx];
    const double ph = L->phi[py][px];
    const CellMac m = macros_from(
        K, mc, L->mu[my][mx - sxl], L->mu[my][mx + sxh], L->mu[my - syl][mx],
        L->mu[my + syh][mx], ph, L->phi[py][px - sxl], L->phi[py][px + sxh],
        L->phi[py - syl][px], L->phi[py + syh][px], w.s0[c], w.jx[c], w.jy[c], X.d1 + 3 * i,
        X.d2 + 3 * i, Y.d1 + 3 * j, Y.d2 + 3 * j);
    const Work &o = tape ? *tape : w;
    if (tape) {
      o.phi[c] = ph;
      o.rho[c] = m.rho;
      o.dphx[c] = m.dphx;
      o.dphy[c] = m.dphy;
      o.dmux[c] = m.dmux;
      o.dmuy[c] = m.dmuy;
    }
    o.mu[c] = mc;
    o.D[c] = m.D;
    if (fields || tape) {
      o.Fx[c] = m.Fx;
      o.Fy[c] = m.Fy;
      o.ux[c] = m.ux;
      o.uy[c] = m.uy;
    }
    o.p[c] = m.p;
  }
#if defined(__HIPCC__)
  // the phases in order, a workgroup barrier between them
  __device__ void run(int tid) const {
    p0(tid);
    __syncthreads();
    p1(tid);
    __syncthreads();
    p2(tid);
  }
#endif
};

#if defined(__HIPCC__)
// one-dimensional grid of nb blocks, gx per block row, in the XCD-aware
// order of xcd_tile (an XCD takes a band of rows)
__global__ __launch_bounds__(MBX * MBY) void k_macros(Consts K, Work w, int gx, int nb,
                                                      int fields) {
  __shared__ MacLds L;
  const int b = xcd_tile(blockIdx.x, nb);
  const MacBlock mb{K, w, (b % gx) * MBX, (b / gx) * MBY, &L, nullptr, fields != 0};
  mb.run(threadIdx.y * MBX + threadIdx.x);
}

// the same in tape mode: the cell fields of w's state into the tape slot t
__global__ __launch_bounds__(MBX * MBY) void k_macros_tape(Consts K, Work w, Work t, int gx,
                                                           int nb) {
  __shared__ MacLds L;
  const int b = xcd_tile(blockIdx.x, nb);
  const MacBlock mb{K, w, (b % gx) * MBX, (b / gx) * MBY, &L, &t};
  mb.run(threadIdx.y * MBX + threadIdx.x);
}
#endif

// LDS of one tile.  A (bar+ on the tile and its ring) is dead once the faces
// are computed; the face fluxes then reuse its space.  TG: tilde+ of the
// tile's cells waits in the output buffer instead of T (which then shrinks to
// one element), and the LDS left lets three workgroups share a CU.
template <class S, bool TG = false>
struct TileLds {
  union {
    double A[18][S::WY][S::WX];
    struct {
      double X[12][S::TY][S::TX + 1];
      double Y[12][S::TY + 1][S::TX];
    } f;
  } u;
  double phi[S::SY][S::SX], mu[S::SY][S::SX], p[S::SY][S::SX];
  // tilde+ of the tile's cells (Step 2 output kept for Step 6) and D over the
  // bar+ window
  double T[TG ? 1 : 18][TG ? 1 : S::TY][TG ? 1 : S::TX];
  double D[S::WY][S::WX];
  // App. B weights (population gradient, first derivative) of the tile's
  // columns (axis 0) and rows (axis 1) at the scalar-window positions, and
  // the geometry of the tile's faces (local face 0..TX along x, 0..TY along y)
  double pgw[2][S::SM][3], d1w[2][S::SM][3];
  double fwl[2][S::FM], fwr[2][S::FM], finv[2][S::FM], foffl[2][S::FM], foffr[2][S::FM];
  // dt / |V| factors of the tile's columns and rows
  double rdt[2][S::FM];
};

// Two tile workgroups share a CU (160 KiB of LDS): a tile's LDS must stay
// within half of it, or occupancy halves.
static_assert(sizeof(TileLds<TileSq>) <= 80 * 1024, "square tile LDS above 80 KiB");
static_assert(sizeof(TileLds<TileWide>) <= 80 * 1024, "wide tile LDS above 80 KiB");
static_assert(sizeof(TileLds<TileTall>) <= 80 * 1024, "tall tile LDS above 80 KiB");
static_assert(sizeof(TileLds<TileUpw>) <= 80 * 1024, "two-ring tile LDS above 80 KiB");
// ... and three workgroups when tilde+ goes through the output buffer (the
// allocation granule of LDS is 512 bytes)
static_assert(3 * ((sizeof(TileLds<TileSq, true>) + 511) / 512 * 512) <= 160 * 1024,
              "square tile LDS without tilde+ above a third of a CU");
static_assert(3 * ((sizeof(TileLds<TileUpw, true>) + 511) / 512 * 512) <= 160 * 1024,
              "two-ring tile LDS without tilde+ above a third of a CU");

// Accessor of the face code over the tile's LDS (bar+, phi, mu, p) and the
// global D.  Global cell (x, y) maps to the tile window, periodic images
// folded back; a window position holding another image of the same cell
// holds the same value.  A handle carries the LDS offsets of the cell and of
// its stencil neighbours, computed once per face.
template <class S, class Lds = TileLds<S>>
struct LAcc {
  // interior-face reconstruction: UPWIND needs the two-cell bar+ ring, and
  // the host runs UPWIND on the two-ring tiles only, CENTRAL on the others
  static constexpr int RECON = S::RG == 2 ? 1 : 0;
  const Consts *K;
  const Work *w;
  const Lds *L;
  int x0, y0;
  struct H {
    int x, y;
    int o1, lo1[2], hi1[2];  // offsets in the bar+ window (WX x WY)
    int o2, lo2[2], hi2[2];  // offsets in the scalar window (SX x SY)
    int w2[2];               // scalar-window column and row (weight tables)
  };
  DFN int win(int g, int o, int n, int wd) const {
    int d = g - o;
    if (d < 0) d += n;
    else if (d >= wd) d -= n;
#ifdef DUGKS2P_WINDOW_CHECK
    // outside the window: a poisoned offset, trapped only where it is read
    // (ring cells carry unread offsets of their outer neighbours)
    if (d < 0 || d >= wd) return -(1 << 20);
#endif
    return d;
  }
  // a neighbour's window position, poisoned (under the window check) if it
  // falls outside the window
  DFN static int nbw(int p, int wd) {
#ifdef DUGKS2P_WINDOW_CHECK
    if (p < 0 || p >= wd) return -(1 << 20);
#else
    (void)wd;
#endif
    return p;
  }
  // The neighbours of a cell sit at the adjacent window positions (on a
  // periodic axis these hold the wrapped images), or at the cell itself
  // across a wall (mirror ghost).  The scalar window is the bar+ window
  // shifted by one, so position p there holds the same cell as p - 1 here.
  DFN H cell(int x, int y) const {
    const Axis &X = K->ax[0], &Y = K->ax[1];
    H h;
    h.x = x;
    h.y = y;
    const int px = win(x, x0 - S::RG, K->nx, S::WX), py = win(y, y0 - S::RG, K->ny, S::WY);
    const int sxl = (X.bc != 0 && x == 0) ? 0 : 1, sxh = (X.bc != 0 && x == X.n - 1) ? 0 : 1;
    const int syl = (Y.bc != 0 && y == 0) ? 0 : 1, syh = (Y.bc != 0 && y == Y.n - 1) ? 0 : 1;
    const int lx1 = nbw(px - sxl, S::WX), hx1 = nbw(px + sxh, S::WX);
    const int ly1 = nbw(py - syl, S::WY), hy1 = nbw(py + syh, S::WY);
    h.o1 = py * S::WX + px;
    h.lo1[0] = py * S::WX + lx1;
    h.hi1[0] = py * S::WX + hx1;
    h.lo1[1] = ly1 * S::WX + px;
    h.hi1[1] = hy1 * S::WX + px;
    const int qx = px + 1, qy = py + 1;
    h.w2[0] = qx;
    h.w2[1] = qy;
    h.o2 = qy * S::SX + qx;
    h.lo2[0] = qy * S::SX + (qx - sxl);
    h.hi2[0] = qy * S::SX + (qx + sxh);
    h.lo2[1] = (qy - syl) * S::SX + qx;
    h.hi2[1] = (qy + syh) * S::SX + qx;
    return h;
  }
  DFN static int chk(int off, int lim) {
#ifdef DUGKS2P_WINDOW_CHECK
    if (off < 0 || off >= lim) {
      printf("window check: offset %d outside [0, %d)\n", off, lim);
      fflush(stdout);
      abort();
    }
#else
    (void)lim;
#endif
    return off;
  }
  DFN const double *Aq(int q) const { return &L->u.A[q][0][0]; }
  enum { NW1 = S::WX * S::WY, NW2 = S::SX * S::SY };
  DFN double A(int q, const H &h) const { return Aq(q)[chk(h.o1, NW1)]; }
  DFN double pgrad(int a, int q, const H &h) const {
    const double *wt = L->pgw[a][chk(h.w2[a], a == 0 ? S::SX : S::SY)];
    const double *aq = Aq(q);
    return wt[0] * aq[chk(h.lo1[a], NW1)] + wt[1] * aq[chk(h.o1, NW1)] +
           wt[2] * aq[chk(h.hi1[a], NW1)];
  }
  DFN double d1(int a, const H &h, const double *f) const {
    const double *wt = L->d1w[a][chk(h.w2[a], a == 0 ? S::SX : S::SY)];
    return wt[0] * f[chk(h.lo2[a], NW2)] + wt[1] * f[chk(h.o2, NW2)] +
           wt[2] * f[chk(h.hi2[a], NW2)];
  }
  // face k of axis a (a face of this tile; a periodic axis passes the face
  // at the far end as face 0)
  DFN FaceGeo geo(int a, int k) const {
    const Axis &X = K->ax[a];
    int f = k - (a == 0 ? x0 : y0);
    if (f < 0) f += X.n;
#ifdef DUGKS2P_WINDOW_CHECK
    if (f < 0 || f > (a == 0 ? S::TX : S::TY)) {
      printf("face check: axis %d face %d local %d\n", a, k, f);
      fflush(stdout);
      abort();
    }
#endif
    FaceGeo g;
    g.cl = ax_fl(X, k);
    g.cr = ax_fr(X, k);
    g.wl = L->fwl[a][f];
    g.wr = L->fwr[a][f];
    g.inv = L->finv[a][f];
    g.offl = L->foffl[a][f];
    g.offr = L->foffr[a][f];
    return g;
  }
  DFN double mu(const H &h) const { return (&L->mu[0][0])[chk(h.o2, NW2)]; }
  DFN double phi(const H &h) const { return (&L->phi[0][0])[chk(h.o2, NW2)]; }
  DFN double p(const H &h) const { return (&L->p[0][0])[chk(h.o2, NW2)]; }
  DFN double D(const H &h) const { return (&L->D[0][0])[chk(h.o1, NW1)]; }
  DFN double dmu(int a, const H &h) const { return d1(a, h, &L->mu[0][0]); }
  DFN double dphi(int a, const H &h) const { return d1(a, h, &L->phi[0][0]); }
  DFN double dp(int a, const H &h) const { return d1(a, h, &L->p[0][0]); }
};

// g modulo n in [0, n).  Window offsets lie within one period of the
// domain unless the domain is narrower than a tile window, so the common
// cases take a compare and an add; the remainder (an integer division on
// the GPU) runs only for those narrow domains.
DFN int wrapi(int g, int n) {
  if (g >= 0 && g < n) return g;
  if (g < 0 && g >= -n) return g + n;
  if (g >= n && g < 2 * n) return g - n;
  const int r = g % n;
  return r < 0 ? r + n : r;
}

// P0 of a tile with origin (x0, y0): phi, mu, p on the scalar window (the
// tile and an (RG + 1)-cell ring), the App. B weight rows of the window's columns and rows, and the
// geometry and dt/|V| factors of the tile's faces and cells, into LDS.
template <class S, class Lds = TileLds<S>>
struct TileP0 {
  const Consts &K;
  const Work &w;
  int x0, y0;
  Lds *L;
  // global index along an axis of window offset o, or -1 outside a wall domain
  DFN int gcol(int g, int n, int bc) const {
    if (bc == 0) return wrapi(g, n);
    return (g >= 0 && g < n) ? g : -1;
  }
  // All of the phase's global loads are issued (p0_load) before its first
  // LDS store (p0_store), so that they share one memory round trip.  Roles:
  // every thread loads window elements tid and tid + NTHR; the last SX + SY
  // threads a weight row each, the TX + TY + 2 threads below them a face.
  static_assert(S::SX * S::SY <= 2 * NTHR, "scalar window exceeds two elements per thread");
  static_assert(S::SX + S::SY + S::TX + S::TY + 2 <= NTHR, "table roles exceed the workgroup");
  struct Pre0 {
    double v[2][3];  // phi, mu, p
    double t[6];     // pg and d1 weights, or fwl fwr finv foffl foffr rdt
  };
  // window element e: its global cell c, false outside the window or domain
  DFN bool win_elem(int e, i64 &c) const {
    if (e >= S::SX * S::SY) return false;
    const int gx = gcol(x0 - S::RG - 1 + e % S::SX, K.nx, K.ax[0].bc);
    const int gy = gcol(y0 - S::RG - 1 + e / S::SX, K.ny, K.ax[1].bc);
    if (gx < 0 || gy < 0) return false;
    c = (i64)gy * K.ld + gx;
    return true;
  }
  // weight-row role r: axis a, window position pos, global index g
  DFN bool wt_role(int r, int &a, int &pos, int &g) const {
    if (r < 0 || r >= S::SX + S::SY) return false;
    a = r < S::SX ? 0 : 1;
    pos = a == 0 ? r : r - S::SX;
    const Axis &X = K.ax[a];
    g = gcol((a == 0 ? x0 : y0) - S::RG - 1 + pos, X.n, X.bc);
    return g >= 0;
  }
  // face role r: axis a, local face f, global face k
  DFN bool face_role(int r, int &a, int &f, int &k) const {
    if (r < 0 || r >= S::TX + S::TY + 2) return false;
    a = r <= S::TX ? 0 : 1;
    f = a == 0 ? r : r - S::TX - 1;
    const Axis &X = K.ax[a];
    k = (a == 0 ? x0 : y0) + f;
    if (X.bc == 0 && k == X.n) k = 0;
    return k < X.nf;
  }
  DFN void p0_load(int tid, Pre0 &r) const {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      i64 c;
      if (win_elem(tid + j * NTHR, c)) {
        r.v[j][0] = w.phi[c];
        r.v[j][1] = w.mu[c];
        r.v[j][2] = w.p[c];
      }
    }
    const int rw = NTHR - 1 - tid, rf = rw - (S::SX + S::SY);
    int a, pos, g, f, k;
    if (wt_role(rw, a, pos, g)) {
      const Axis &X = K.ax[a];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        r.t[m] = X.pg[3 * g + m];
        r.t[3 + m] = X.d1[3 * g + m];
      }
    } else if (face_role(rf, a, f, k)) {
      const Axis &X = K.ax[a];
      r.t[0] = X.fwl[k];
      r.t[1] = X.fwr[k];
      r.t[2] = X.finv[k];
      r.t[3] = X.foffl[k];
      r.t[4] = X.foffr[k];
      if (f < (a == 0 ? S::TX : S::TY) && k < X.n) r.t[5] = X.rdt[k];
    }
  }
  DFN void p0_store(int tid, const Pre0 &r) const {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      i64 c;
      const int e = tid + j * NTHR;
      if (win_elem(e, c)) {
        const int lx = e % S::SX, ly = e / S::SX;
        L->phi[ly][lx] = r.v[j][0];
        L->mu[ly][lx] = r.v[j][1];
        L->p[ly][lx] = r.v[j][2];
      }
    }
    const int rw = NTHR - 1 - tid, rf = rw - (S::SX + S::SY);
    int a, pos, g, f, k;
    if (wt_role(rw, a, pos, g)) {
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        L->pgw[a][pos][m] = r.t[m];
        L->d1w[a][pos][m] = r.t[3 + m];
      }
    } else if (face_role(rf, a, f, k)) {
      L->fwl[a][f] = r.t[0];
      L->fwr[a][f] = r.t[1];
      L->finv[a][f] = r.t[2];
      L->foffl[a][f] = r.t[3];
      L->foffr[a][f] = r.t[4];
      if (f < (a == 0 ? S::TX : S::TY) && k < K.ax[a].n) L->rdt[a][f] = r.t[5];
    }
  }
};

// One tile of shape S with origin (x0, y0); V: the viscosity model; TG:
// tilde+ of the tile's cells kept in the output buffer between P1 and P4
// (else in LDS).
template <class IO, class R, bool U = false, class S = TileSq, int V = VIS_ANY, bool TG = false>
struct FusedTile {
  using Lds = TileLds<S, TG>;
  const Consts &K;
  const Work &w;
  IO src;
  IO dst;
  int x0, y0;
  Lds *L;

  struct TS {
    R fx[12], fy[12];
    bool hx, hy;
  };
  // global inputs of a window cell's Step 2, loaded ahead of P0 so that their
  // latency overlaps P0's loads
  struct Pre {
    double tv[18], D;
  };

  // global index along an axis of window offset o, or -1 outside a wall domain
  DFN int gcol(int g, int n, int bc) const {
    if (bc == 0) return wrapi(g, n);
    return (g >= 0 && g < n) ? g : -1;
  }

  // window cell of thread tid: global column and row (-1 outside a wall domain)
  DFN void p1_cell(int tid, int &gx, int &gy) const {
    const int lx = tid % S::WX, ly = tid / S::WX;
    gx = gcol(x0 - S::RG + lx, K.nx, K.ax[0].bc);
    gy = gcol(y0 - S::RG + ly, K.ny, K.ax[1].bc);
  }
  DFN void p1_load(int tid, Pre &pr) const {
    int gx, gy;
    p1_cell(tid, gx, gy);
    if (gx < 0 || gy < 0) return;
    const i64 c = (i64)gy * K.ld + gx;
    src.load(c, pr.tv);
    pr.D = w.D[c];
  }

  // P0 (see TileP0)
  using Pre0 = typename TileP0<S, Lds>::Pre0;
  DFN TileP0<S, Lds> win() const { return TileP0<S, Lds>{K, w, x0, y0, L}; }
  DFN void p0_load(int tid, Pre0 &r) const { win().p0_load(tid, r); }
  DFN void p0_store(int tid, const Pre0 &r) const { win().p0_store(tid, r); }

  // P1: Step 2 on the bar+ window (the tile and its RG-cell ring); tilde+
  // kept for the tile.
  DFN void p1(int tid, const Pre &pr) const {
    const int lx = tid % S::WX, ly = tid / S::WX;
    int gx, gy;
    p1_cell(tid, gx, gy);
    if (gx < 0 || gy < 0) return;
    const LAcc<S, Lds> acc{&K, &w, L, x0, y0};
    const typename LAcc<S, Lds>::H hc = acc.cell(gx, gy);
    const double ph = acc.phi(hc);
    const double rh = rho_of<double>(K, ph);
    // F and u of the macro kernel, recomputed from mu in LDS and the f~ sums
    // of the loaded state (the values and the order of operations of the
    // macro kernel, which then need not store them)
    const double *mu = &L->mu[0][0];
    double f[9], jx, jy;
    {
      double phs;
      src.stored(pr.tv, phs, f);
    }
    xi_sums<double, U>(K, f, jx, jy);
    const CellFU cm = force_velocity(K, mu[hc.o2], mu[hc.lo2[0]], mu[hc.hi2[0]], mu[hc.lo2[1]],
                                     mu[hc.hi2[1]], ph, rh, jx, jy, L->d1w[0][hc.w2[0]],
                                     L->d1w[1][hc.w2[1]]);
    Mac<R> m;
    m.phi = (R)ph;
    m.rho = (R)rh;
    m.ux = (R)cm.ux;
    m.uy = (R)cm.uy;
    m.p = (R)acc.p(hc);
    m.mu = (R)acc.mu(hc);
    m.grx = (R)(K.drho * acc.dphi(0, hc));
    m.gry = (R)(K.drho * acc.dphi(1, hc));
    m.D = (R)pr.D;
    m.Fx = (R)cm.Fx;
    m.Fy = (R)cm.Fy;
    L->D[ly][lx] = pr.D;
    m.gpx = (R)acc.dp(0, hc);
    m.gpy = (R)acc.dp(1, hc);
    m.icr = (R)1.0 / ((R)K.cs2 * m.rho);
    const R tf = tauf_of<R, V>(K, (R)ph, (R)rh);
    R til[18], out[18];
#pragma unroll
    for (int q = 0; q < 18; ++q) til[q] = (R)pr.tv[q];
    cell_barp<R, U>(K, m, tf, til, out);
#pragma unroll
    for (int q = 0; q < 18; ++q) L->u.A[q][ly][lx] = (double)out[q];
    // tilde+ of the tile's own cells waits in LDS for P4, rounded as the
    // state encoding would round it; bar+ of those cells also goes to
    // w.barp when it is set (the adjoint's tape)
    const int cx = lx - S::RG, cy = ly - S::RG;
    if (cx >= 0 && cx < S::TX && cy >= 0 && cy < S::TY && x0 + cx < K.nx && y0 + cy < K.ny) {
      if (w.barp) {
        const i64 c = (i64)gy * K.ld + gx;
#pragma unroll
        for (int q = 0; q < 18; ++q) w.barp[q * K.plane + c] = (double)out[q];
      }
      double tv[18];
#pragma unroll
      for (int q = 0; q < 18; ++q)
        tv[q] = (double)((R)(4.0 / 3.0) * (R)(double)out[q] - (R)(1.0 / 3.0) * til[q]);
      if (TG) {
        // into the cell's slot of the output buffer, which P4 reads back
        // (load after store is the encoding's round trip) and overwrites
        dst.store((i64)gy * K.ld + gx, tv);
      } else {
        IO::roundtrip(tv);
#pragma unroll
        for (int q = 0; q < 18; ++q) L->T[TG ? 0 : q][TG ? 0 : cy][TG ? 0 : cx] = tv[q];
      }
    }
  }

  // P2: Steps 3-4 at the x-face west of tile column tx and the y-face south
  // of tile row ty.
  DFN void p2(int tid, TS &ts) const {
    const int tx = tid % S::WX, ty = tid / S::WX;
    const LAcc<S, Lds> acc{&K, &w, L, x0, y0};
    ts.hx = ts.hy = false;
    R out[18];
    const bool perx = K.ax[0].bc == 0, pery = K.ax[1].bc == 0;
    if (tx <= S::TX && ty < S::TY) {
      const int k = x0 + tx, t = y0 + ty;
      if (t < K.ny && k <= K.nx) {
        face_core<0, R, LAcc<S, Lds>, U, V>(K, acc, (perx && k == K.nx) ? 0 : k, t, out);
#pragma unroll
        for (int q = 0; q < 18; ++q) {
          const int s = xslot(q % 9);
          if (s >= 0) ts.fx[(q / 9) * 6 + s] = out[q];
        }
        ts.hx = true;
      }
    }
    if (tx < S::TX && ty <= S::TY) {
      const int k = y0 + ty, t = x0 + tx;
      if (t < K.nx && k <= K.ny) {
        face_core<1, R, LAcc<S, Lds>, U, V>(K, acc, (pery && k == K.ny) ? 0 : k, t, out);
#pragma unroll
        for (int q = 0; q < 18; ++q) {
          const int s = yslot(q % 9);
          if (s >= 0) ts.fy[(q / 9) * 6 + s] = out[q];
        }
        ts.hy = true;
      }
    }
  }

  // P3: face values into LDS (over the dead bar+).
  DFN void p3(int tid, const TS &ts) const {
    const int tx = tid % S::WX, ty = tid / S::WX;
    if (ts.hx)
#pragma unroll
      for (int s = 0; s < 12; ++s) L->u.f.X[s][ty][tx] = (double)ts.fx[s];
    if (ts.hy)
#pragma unroll
      for (int s = 0; s < 12; ++s) L->u.f.Y[s][ty][tx] = (double)ts.fy[s];
  }

#if defined(__HIPCC__)
  // the phases in order, a workgroup barrier between them
  __device__ void run(int tid) const {
    Pre0 r0;
    Pre pr;
    TS ts;
    p0_load(tid, r0);
    p1_load(tid, pr);
    p0_store(tid, r0);
    __syncthreads();
    p1(tid, pr);
    __syncthreads();
    p2(tid, ts);
    __syncthreads();
    p3(tid, ts);
    __syncthreads();
    p4(tid);
  }
#endif

  // P4: Steps 5-6 (eq. updatef) for the tile's cells.
  DFN void p4(int tid) const {
    const int lx = tid % S::WX, ly = tid / S::WX;
    if (lx < 1 || lx > S::TX || ly < 1 || ly > S::TY) return;
    const int cx = lx - 1, cy = ly - 1;
    const int gx = x0 + cx, gy = y0 + cy;
    if (gx >= K.nx || gy >= K.ny) return;
    const i64 c = (i64)gy * K.ld + gx;
    const R rx = (R)L->rdt[0][cx], ry = (R)L->rdt[1][cy];
    double tv[18];
    if (TG) {
      dst.load(c, tv);
    } else {
#pragma unroll
      for (int q = 0; q < 18; ++q) tv[q] = L->T[TG ? 0 : q][TG ? 0 : cy][TG ? 0 : cx];
    }
#pragma unroll
    for (int q = 0; q < 18; ++q) {
      const int d = q % 9, sx = xslot(d), sy = yslot(d);
      R W = (R)0.0, E = (R)0.0, Sf = (R)0.0, N = (R)0.0;
      if (sx >= 0) {
        W = (R)L->u.f.X[(q / 9) * 6 + sx][cy][cx];
        E = (R)L->u.f.X[(q / 9) * 6 + sx][cy][cx + 1];
      }
      if (sy >= 0) {
        Sf = (R)L->u.f.Y[(q / 9) * 6 + sy][cy][cx];
        N = (R)L->u.f.Y[(q / 9) * 6 + sy][cy + 1][cx];
      }
      const R tilp = (R)tv[q];
      if (U) {
        // (rx * e_x) (E - W) with e_x in {-1, 0, 1}; a zero term leaves tilp
        const R tx = sx >= 0 ? (ex_of(d) > 0 ? rx : -rx) * (E - W) : (R)0.0;
        const R ty = sy >= 0 ? (ey_of(d) > 0 ? ry : -ry) * (N - Sf) : (R)0.0;
        tv[q] = (double)(tilp - tx - ty);
      } else {
        tv[q] = (double)(tilp - rx * (R)K.xi0[d] * (E - W) - ry * (R)K.xi1[d] * (N - Sf));
      }
    }
    // phi and the f~ sums of the new state, as the next step would read them
    if (w.phin) {
      double ph, f[9], s0 = 0.0, jx, jy;
      dst.stored(tv, ph, f);
#pragma unroll
      for (int q = 0; q < 9; ++q) s0 += f[q];
      xi_sums<double, U>(K, f, jx, jy);
      w.phin[c] = ph;
      w.s0n[c] = s0;
      w.jxn[c] = jx;
      w.jyn[c] = jy;
    }
    dst.store(c, tv);
  }
};

template <class S>
DFN int tiles_x(const Consts &K) { return (K.nx + S::TX - 1) / S::TX; }

template <class S>
DFN int tiles_y(const Consts &K) { return (K.ny + S::TY - 1) / S::TY; }

// Workgroups are dealt to the 8 XCDs round robin; give each XCD a contiguous
// run of tiles so that neighbouring tiles share its L2.
DFN int xcd_tile(int b, int n) {
  const int xcd = b % 8, slot = b / 8;
  const int q = n / 8, r = n % 8;
  return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

#if defined(__HIPCC__)
// Registers are held to the waves per SIMD that the LDS allows: two
// workgroups per CU, or three without tilde+ in LDS.
template <class IO, class R, bool U, class S, int V, bool TG>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(TG ? 3 : 2))) void
k_fused_tile(Consts K, Work w, IO src, IO dst, int ntx, int ntiles) {
  __shared__ TileLds<S, TG> L;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  FusedTile<IO, R, U, S, V, TG> ft{K, w, src, dst, (tile % ntx) * S::TX, (tile / ntx) * S::TY, &L};
  ft.run(threadIdx.x);
}
#endif

// One fused time step (Ex: grid(functor, n0, n1) and
// tiles<IO, R, U, S, V, TG>(...)).  U: unit lattice speed (RT = 1/3), S: tile
// shape, V: viscosity model, TG: tilde+ through the output buffer, all chosen
// by the host (with_fused_kernel).  sums_ready: phi and the f~ sums of src
// are already in w (written by the previous step's tile kernel).
template <class Ex, class IO, class R, bool U, class S = TileSq, int V = VIS_ANY, bool TG = false>
void seq_fused_step(Ex &ex, const Consts &K, const Work &w, const IO &src, const IO &dst,
                    bool sums_ready = false) {
  if (!sums_ready) ex.grid(FPhiSums<IO, U>{K, w, src}, K.nx, K.ny);
  ex.macros(K, w, false);
  ex.template tiles<IO, R, U, S, V, TG>(K, w, src, dst);
}

// After a committed fused step the sums written for the new state become
// the current ones.
inline void swap_sums(Work &w) {
  double *t;
  t = w.phi; w.phi = w.phin; w.phin = t;
  t = w.s0; w.s0 = w.s0n; w.s0n = t;
  t = w.jx; w.jx = w.jxn; w.jxn = t;
  t = w.jy; w.jy = w.jyn; w.jyn = t;
}

// Calls f(S{}) with the tile shape of a DUGKS2P_TILE_* value (1 square,
// 2 wide, 3 tall, 4 the two-ring tiles of UPWIND reconstruction).  Wide and
// tall tiles exist for unit lattice speed only; other speeds take square
// tiles for CENTRAL reconstruction.
template <class F>
void with_tile_shape(int shape, bool unit, F &&f) {
  if (shape == 4)
    f(TileUpw{});
  else if (unit && shape == 2)
    f(TileWide{});
  else if (unit && shape == 3)
    f(TileTall{});
  else
    f(TileSq{});
}

// Calls f(u, s, v, tg) with the compile-time choices of the single-handle
// tile kernel for a DUGKS2P_TILE_* shape and the constants K: u the
// unit-speed flag (std::bool_constant), s the tile shape, v the viscosity
// model (std::integral_constant<int, VIS_*>), tg whether tilde+ goes through
// the output buffer (std::bool_constant; taken for square and two-ring tiles
// at unit speed when the caller passes resident, a ping-pong state that
// stays in the MALL; the wide and tall tiles would not fit three to a CU
// even so).  At unit lattice speed every
// shape is compiled for a given tau_f and for the mixture viscosity apart
// (the run-time choice costs the tile kernel about a tenth of its speed);
// other speeds take square or two-ring tiles and read the model at run time.
// Shape 4 (the two-ring tiles) is UPWIND reconstruction and every other
// shape CENTRAL: the caller keeps the two matched.
template <class F>
void with_fused_kernel(int shape, const Consts &K, bool resident, F &&f) {
  using Any = std::integral_constant<int, VIS_ANY>;
  using Uni = std::integral_constant<int, VIS_UNIFORM>;
  using Mix = std::integral_constant<int, VIS_MIXTURE>;
  if (!K.unit) {
    if (shape == 4)
      f(std::false_type{}, TileUpw{}, Any{}, std::false_type{});
    else
      f(std::false_type{}, TileSq{}, Any{}, std::false_type{});
    return;
  }
  auto vis = [&](auto sh, auto tg) {
    if (K.tau_f > 0.0)
      f(std::true_type{}, sh, Uni{}, tg);
    else
      f(std::true_type{}, sh, Mix{}, tg);
  };
  if (shape == 4 && resident)
    vis(TileUpw{}, std::true_type{});
  else if (shape == 4)
    vis(TileUpw{}, std::false_type{});
  else if (shape == 2)
    vis(TileWide{}, std::false_type{});
  else if (shape == 3)
    vis(TileTall{}, std::false_type{});
  else if (resident)
    vis(TileSq{}, std::true_type{});
  else
    vis(TileSq{}, std::false_type{});
}

// Cell fields of the current state for moments and monitors (phi, mu, D, F,
// u, p in the work arrays).
template <class Ex, class IO>
void seq_moments(Ex &ex, const Consts &K, const Work &w, const IO &src) {
  ex.grid(FPhiSums<IO, false>{K, w, src}, K.nx, K.ny);
  ex.macros(K, w, true);
}

}  // namespace DUGKS2P_NS
