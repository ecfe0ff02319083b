// Host build of the HIP path's kernel logic, for CPU tests only.
//
// Runs the same functors and stage sequences as the gfx950 kernels, one
// "thread" at a time on the host, so that index and arithmetic-order
// mistakes in the kernel code show up against the oracle without a GPU.
// Built from paper_1802_02868_amd/csrc with the host compiler; never loaded
// by the product.
#include <stdlib.h>
#include <string.h>

#include <type_traits>
#include <vector>

#include "../../paper_1802_02868_amd/csrc/dugks2p_fused.hpp"
#include "../../paper_1802_02868_amd/csrc/dugks2p_host.hpp"
#include "../../paper_1802_02868_amd/csrc/dugks2p_adjoint.hpp"

using namespace dg;

namespace {
struct CpuEx {
  template <class F>
  void grid(const F &f, int n0, int n1) {
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n0; ++i) f(i, j);
  }
  // Every workgroup of the tile kernel in turn; each phase runs for all 256
  // threads before the next (the barrier between phases).
  // every 64 x 4 block of the macro kernel in turn, phase by phase
  void macros(const Consts &K, const Work &w, bool fields, const Work *tape = nullptr) {
    std::vector<MacLds> L(1);
    for (int by = 0; by < (K.ny + MBY - 1) / MBY; ++by)
      for (int bx = 0; bx < (K.nx + MBX - 1) / MBX; ++bx) {
        memset((void *)L.data(), 0xff, sizeof(MacLds));  // NaN poison
        const MacBlock mb{K, w, bx * MBX, by * MBY, L.data(), tape, fields};
        for (int t = 0; t < MBX * MBY; ++t) mb.p0(t);
        for (int t = 0; t < MBX * MBY; ++t) mb.p1(t);
        for (int t = 0; t < MBX * MBY; ++t) mb.p2(t);
      }
  }
  void macros_tape(const Consts &K, const Work &w, const Work &t) { macros(K, w, true, &t); }
  // the adjoint's face stage: every workgroup in turn, phase by phase
  void adj_faces(const Consts &K, const Work &w, const AdjWork &a) {
    using S = TileSq;
    const int ntx = tiles_x<S>(K), nt = ntx * tiles_y<S>(K);
    std::vector<AdjLds<S>> L(1);
    std::vector<typename AdjFaceTile<S>::Win::Pre0> r0(NTHR);
    std::vector<typename AdjFaceTile<S>::PreA> ra(NTHR);
    for (int b = 0; b < nt; ++b) {
      const int tile = xcd_tile(b, nt);
      memset((void *)L.data(), 0xff, sizeof(AdjLds<S>));  // NaN poison: stray reads show
      memset((void *)r0.data(), 0xff, r0.size() * sizeof(r0[0]));
      memset((void *)ra.data(), 0xff, ra.size() * sizeof(ra[0]));
      const AdjFaceTile<S> ft{K, w, a, (tile % ntx) * S::TX, (tile / ntx) * S::TY, L.data()};
      for (int t = 0; t < NTHR; ++t) ft.win().p0_load(t, r0[t]);
      for (int t = 0; t < NTHR; ++t) ft.a_load(t, ra[t]);
      for (int t = 0; t < NTHR; ++t) ft.win().p0_store(t, r0[t]);
      for (int t = 0; t < NTHR; ++t) ft.a_store(t, ra[t]);
      for (int t = 0; t < NTHR; ++t) ft.faces(t);
    }
  }
  // the adjoint's tiled gather and cell stage: phase by phase, one velocity
  // at a time; each buffer is poisoned again before the gather that fills it
  void adj_cells(const Consts &K, const Work &w, const AdjWork &a, const double *st) {
    using S = TileSq;
    using T = AdjCellTile<S>;
    const int ntx = tiles_x<S>(K), nt = ntx * tiles_y<S>(K);
    std::vector<AdjCellLds<S>> L(1);
    std::vector<typename T::St> s(NTHR);
    for (int b = 0; b < nt; ++b) {
      const int tile = xcd_tile(b, nt);
      memset((void *)s.data(), 0xff, s.size() * sizeof(s[0]));
      const T ct{K, w, a, st, (tile % ntx) * S::TX, (tile / ntx) * S::TY, L.data()};
      for (int t = 0; t < NTHR; ++t) ct.setup(t, s[t]);
      for (int i2 = 0; i2 < 9; ++i2) {
        memset((void *)L[0].g[i2 & 1], 0xff, sizeof(L[0].g[0]));
        for (int t = 0; t < NTHR; ++t) ct.gather(i2, s[t]);
        for (int t = 0; t < NTHR; ++t) ct.cell(i2, s[t]);
      }
      for (int t = 0; t < NTHR; ++t) ct.finish(s[t]);
    }
  }
  template <class IO, class R, bool U, class S, int V, bool TG>
  void tiles(const Consts &K, const Work &w, const IO &src, const IO &dst) {
    using FT = FusedTile<IO, R, U, S, V, TG>;
    const int ntx = tiles_x<S>(K), nt = ntx * tiles_y<S>(K);
    std::vector<typename FT::Lds> L(1);
    std::vector<typename FT::TS> ts(NTHR);
    std::vector<typename FT::Pre> pre(NTHR);
    std::vector<typename FT::Pre0> pre0(NTHR);
    for (int b = 0; b < nt; ++b) {
      const int tile = xcd_tile(b, nt);
      memset((void *)L.data(), 0xff, sizeof(typename FT::Lds));  // NaN poison: stray reads show
      memset((void *)pre.data(), 0xff, pre.size() * sizeof(pre[0]));
      memset((void *)pre0.data(), 0xff, pre0.size() * sizeof(pre0[0]));
      FT ft{K, w, src, dst, (tile % ntx) * S::TX, (tile / ntx) * S::TY, L.data()};
      // the kernel's order: P0 and Step 2 loads, P0 stores, barrier, P1, ... P4
      for (int t = 0; t < NTHR; ++t) ft.p0_load(t, pre0[t]);
      for (int t = 0; t < NTHR; ++t) ft.p1_load(t, pre[t]);
      for (int t = 0; t < NTHR; ++t) ft.p0_store(t, pre0[t]);
      for (int t = 0; t < NTHR; ++t) ft.p1(t, pre[t]);
      for (int t = 0; t < NTHR; ++t) ft.p2(t, ts[t]);
      for (int t = 0; t < NTHR; ++t) ft.p3(t, ts[t]);
      for (int t = 0; t < NTHR; ++t) ft.p4(t);
    }
  }
};
}  // namespace

// Fused steps as the runtime runs them: the sums kernel only before the
// first step, then the tile kernel's own sums of the state it writes.
// resident: the library's choice of tilde+ through the output buffer, or the
// one DUGKS2P_EMU_TILDE names ("lds" or "out"), so that tests run both forms.
template <class IO>
static void run_steps(CpuEx &ex, const Consts &K, Work &w, IO st[2], int &cur, bool fused,
                      long long nsteps, int shape, bool resident) {
  const char *force = getenv("DUGKS2P_EMU_TILDE");
  if (force && !strcmp(force, "lds")) resident = false;
  if (force && !strcmp(force, "out")) resident = true;
  bool ready = false;
  for (long long n = 0; n < nsteps; ++n) {
    if (fused)
      with_fused_kernel(shape, K, resident, [&](auto u, auto sh, auto v, auto tg) {
        seq_fused_step<CpuEx, IO, double, decltype(u)::value, decltype(sh), decltype(v)::value,
                       decltype(tg)::value>(ex, K, w, st[cur], st[1 - cur], ready);
      });
    cur = 1 - cur;
    swap_sums(w);
    ready = true;
  }
}

extern "C" int emu_run(const dugks2p_params *P, const double *phi0, const double *ux0,
                       const double *uy0, const double *p0, long long nsteps, double *pops,
                       double *macros) {
  const std::string err = validate(P);
  if (!err.empty()) return -1;
  AxisHost ax, ay;
  build_axis(ax, P->nx, P->bc_x, P->x_faces);
  build_axis(ay, P->ny, P->bc_y, P->y_faces);
  Consts K = make_consts(P, ax, ay);
  const bool fused = P->kernel == DUGKS2P_KERNEL_FUSED;
  const bool f32 = P->precision == DUGKS2P_FP32_STATE;
  if (f32 && !fused) return -2;
  // the library's choice: UPWIND reconstruction runs on the two-ring tiles
  const int shape = P->recon != DUGKS2P_RECON_CENTRAL ? DUGKS2P_TILE_UPWIND : P->tile;
  Layout L = make_layout(K, ax, ay, P->precision, true);
  const bool resident = 2.0 * (double)L.state_bytes <= TILDE_OUT_MAX_STATE_BYTES;
  std::vector<unsigned char> mem(L.total + 256, 0);
  unsigned char *base = (unsigned char *)(((uintptr_t)mem.data() + 255) & ~(uintptr_t)255);
  std::vector<unsigned char> tb;
  pack_axis(ax, tb);
  memcpy(base + L.tables[0], tb.data(), tb.size());
  pack_axis(ay, tb);
  memcpy(base + L.tables[1], tb.data(), tb.size());
  K.ax[0] = bind_axis(ax, base + L.tables[0]);
  K.ax[1] = bind_axis(ay, base + L.tables[1]);
  Work w = bind_work(L, K, base);
  CpuEx ex;
  int cur = 0;
  double v[18];
  if (!f32) {
    IoF64 st[2] = {io_f64(base + L.state[0], K), io_f64(base + L.state[1], K)};
    seq_init(ex, K, w, phi0, ux0, uy0, p0, st[0]);
    if (fused) {
      run_steps(ex, K, w, st, cur, true, nsteps, shape, resident);
    } else {
      for (long long n = 0; n < nsteps; ++n) {
        seq_staged_step(ex, K, w, (const double *)st[cur].p, st[1 - cur].p);
        cur = 1 - cur;
      }
    }
    for (int j = 0; j < K.ny; ++j)
      for (int i = 0; i < K.nx; ++i) {
        st[cur].load((i64)j * K.ld + i, v);
        for (int q = 0; q < 18; ++q) pops[((size_t)q * K.ny + j) * K.nx + i] = v[q];
      }
    if (macros) seq_moments(ex, K, w, st[cur]);
  } else {
    IoE32 st[2] = {io_e32(base + L.state[0], K, L), io_e32(base + L.state[1], K, L)};
    seq_init(ex, K, w, phi0, ux0, uy0, p0, st[0]);
    run_steps(ex, K, w, st, cur, true, nsteps, shape, resident);
    for (int j = 0; j < K.ny; ++j)
      for (int i = 0; i < K.nx; ++i) {
        st[cur].load((i64)j * K.ld + i, v);
        for (int q = 0; q < 18; ++q) pops[((size_t)q * K.ny + j) * K.nx + i] = v[q];
      }
    if (macros) seq_moments(ex, K, w, st[cur]);
  }
  if (macros) {
    for (int j = 0; j < K.ny; ++j)
      for (int i = 0; i < K.nx; ++i) {
        const i64 c = (i64)j * K.ld + i;
        const double vals[5] = {w.phi[c], rho_of<double>(K, w.phi[c]), w.ux[c], w.uy[c], w.p[c]};
        for (int f = 0; f < 5; ++f) macros[((size_t)f * K.ny + j) * K.nx + i] = vals[f];
      }
  }
  return 0;
}

// Adjoint of a rollout in the host build: initialise, run nsteps staged
// steps keeping a checkpoint every mseg steps, then sweep back segment by
// segment and through Step 1.  lam_T: adjoint of the final populations
// ([18][ny][nx]); outputs the final populations, the adjoint of phi0 and the
// kappa / gx / gy gradients (grad3).
extern "C" int emu_adjoint(const dugks2p_params *P, const double *phi0, const double *ux0,
                           const double *uy0, const double *p0, long long nsteps, int mseg,
                           const double *lam_T, double *pops_T, double *phi0_grad,
                           double *grad3) {
  const std::string err = validate(P);
  if (!err.empty() || mseg < 1) return -1;
  AxisHost ax, ay;
  build_axis(ax, P->nx, P->bc_x, P->x_faces);
  build_axis(ay, P->ny, P->bc_y, P->y_faces);
  Consts K = make_consts(P, ax, ay);
  pack_rows(K);
  const AdjLayout AL = make_adj_layout(K, ax, ay, mseg);
  std::vector<unsigned char> mem(AL.total + 256, 0);
  unsigned char *base = (unsigned char *)(((uintptr_t)mem.data() + 255) & ~(uintptr_t)255);
  memset(base, 0xff, AL.total);  // NaN poison: reads of unwritten scratch show
  std::vector<unsigned char> tb;
  pack_axis(ax, tb);
  memcpy(base + AL.tables[0], tb.data(), tb.size());
  pack_axis(ay, tb);
  memcpy(base + AL.tables[1], tb.data(), tb.size());
  K.ax[0] = bind_axis(ax, base + AL.tables[0]);
  K.ax[1] = bind_axis(ay, base + AL.tables[1]);
  const AdjBufs B{AL, base};
  CpuEx ex;
  const size_t np = 18 * (size_t)K.plane;
  std::vector<double> st[2] = {std::vector<double>(np), std::vector<double>(np)};
  const Work w = B.tape(0);
  seq_init(ex, K, w, phi0, ux0, uy0, p0, IoF64{st[0].data(), K.plane});
  std::vector<std::vector<double>> ck;
  int cur = 0;
  for (long long n = 0; n < nsteps; ++n) {
    if (n % mseg == 0) ck.push_back(st[cur]);
    seq_staged_step(ex, K, w, (const double *)st[cur].data(), st[1 - cur].data());
    cur = 1 - cur;
  }
  memcpy(pops_T, st[cur].data(), np * sizeof(double));
  std::vector<double> lam(lam_T, lam_T + np);
  const double *pacc = B.adj(0).pacc;
  for (int m = 0; m < 3; ++m) grad3[m] = 0.0;
  auto reduce = [&]() {
    for (int m = 0; m < 3; ++m) {
      double s = 0.0;
      for (i64 c = 0; c < K.plane; ++c) s += pacc[m * K.plane + c];
      grad3[m] += s;
    }
  };
  for (long long k = (long long)ck.size() - 1; k >= 0; --k) {
    const long long left = nsteps - k * mseg;
    const int ns = (int)(left < mseg ? left : mseg);
    seq_adjoint_segment(ex, K, B, ck[k].data(), ns, lam.data(), lam.data());
    reduce();
  }
  seq_adjoint_initial(ex, K, B, phi0, ux0, uy0, p0, lam.data(), phi0_grad);
  reduce();
  return 0;
}
