// Host build of the HIP path's kernel logic, for CPU tests only.
//
// Runs the same functors and stage sequences as the gfx950 kernels, one
// "thread" at a time on the host, so that index and arithmetic-order
// mistakes in the kernel code show up against the oracle without a GPU.
// Built from paper_1802_02868_amd/csrc with the host compiler; never loaded
// by the product.
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../paper_1802_02868_amd/csrc/dugks2p_fused.hpp"
#include "../../paper_1802_02868_amd/csrc/dugks2p_host.hpp"

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
  template <class T, class R, bool U>
  void tiles(const Consts &K, const Work &w, const T *src, T *dst) {
    const int ntx = tiles_x(K), nt = ntx * tiles_y(K);
    std::vector<TileLds> L(1);
    std::vector<typename FusedTile<T, R, U>::TS> ts(NTHR);
    for (int b = 0; b < nt; ++b) {
      const int tile = xcd_tile(b, nt);
      memset((void *)L.data(), 0xff, sizeof(TileLds));  // NaN poison: stray reads show
      FusedTile<T, R, U> ft{K, w, src, dst, (tile % ntx) * TT, (tile / ntx) * TT, L.data()};
      for (int t = 0; t < NTHR; ++t) ft.p0(t);
      for (int t = 0; t < NTHR; ++t) ft.p1(t, ts[t]);
      for (int t = 0; t < NTHR; ++t) ft.p2(t, ts[t]);
      for (int t = 0; t < NTHR; ++t) ft.p3(t, ts[t]);
      for (int t = 0; t < NTHR; ++t) ft.p4(t, ts[t]);
    }
  }
};
}  // namespace

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
  Layout L = make_layout(K, ax, ay, DUGKS2P_FP64, true);
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
  double *st[2] = {(double *)(base + L.state[0]), (double *)(base + L.state[1])};
  CpuEx ex;
  seq_init(ex, K, w, phi0, ux0, uy0, p0, st[0]);
  int cur = 0;
  for (long long n = 0; n < nsteps; ++n) {
    if (fused && K.unit)
      seq_fused_step<CpuEx, double, double, true>(ex, K, w, st[cur], st[1 - cur]);
    else if (fused)
      seq_fused_step<CpuEx, double, double, false>(ex, K, w, st[cur], st[1 - cur]);
    else
      seq_staged_step(ex, K, w, st[cur], st[1 - cur]);
    cur = 1 - cur;
  }
  for (int q = 0; q < 18; ++q)
    for (int j = 0; j < K.ny; ++j)
      for (int i = 0; i < K.nx; ++i)
        pops[((size_t)q * K.ny + j) * K.nx + i] = st[cur][q * K.plane + (i64)j * K.ld + i];
  if (macros) {
    seq_macros(ex, K, w, st[cur]);
    const double *src[5] = {w.phi, w.rho, w.ux, w.uy, w.p};
    for (int f = 0; f < 5; ++f)
      for (int j = 0; j < K.ny; ++j)
        for (int i = 0; i < K.nx; ++i)
          macros[((size_t)f * K.ny + j) * K.nx + i] = src[f][(i64)j * K.ld + i];
  }
  return 0;
}
