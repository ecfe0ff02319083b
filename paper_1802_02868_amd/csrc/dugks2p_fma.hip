// dugks2p_fma.hip -- the fused step (cell macros and tile kernel) compiled
// with FMA contraction (-ffp-contract=fast), for DUGKS2P_KERNEL_FUSED_FMA.
//
// The arithmetic is the same source as the exact kernels, in the same
// order; the compiler may fuse a multiply and the add that consumes it into
// one fused multiply-add, which rounds once instead of twice.  Results are
// therefore not bit-identical to the oracle; they stay within the FP64
// parity bar (tests).  The code is compiled into namespace dg_fma so that it
// sits beside the exact instantiations in one library.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <string.h>

#define DUGKS2P_NS dg_fma
#include "dugks2p_fused.hpp"
#include "dugks2p_fma.h"

#include <type_traits>

namespace dg_fma {
namespace {

// One thread per (i, j) in a 64 x 4 block, XCD-aware block order (as the
// exact runtime's per-cell launcher).
template <class F>
__global__ __launch_bounds__(256) void k_grid_fma(F f, int n0, int n1, int gx, int nb) {
  const int b = xcd_tile(blockIdx.x, nb);
  const int i = (b % gx) * 64 + threadIdx.x;
  const int j = (b / gx) * 4 + threadIdx.y;
  if (i < n0 && j < n1) f(i, j);
}

struct FmaEx {
  hipStream_t s;
  hipError_t err;
  hipEvent_t e0, e1;
  void note(hipError_t e) {
    if (e != hipSuccess && err == hipSuccess) err = e;
  }
  template <class F>
  void grid(const F &f, int n0, int n1) {
    if (n0 <= 0 || n1 <= 0) return;
    const int gx = (n0 + 63) / 64, nb = gx * ((n1 + 3) / 4);
    hipLaunchKernelGGL(k_grid_fma<F>, dim3(nb), dim3(64, 4), 0, s, f, n0, n1, gx, nb);
    note(hipGetLastError());
  }
  void macros(const Consts &K, const Work &w, bool fields) {
    const int gx = (K.nx + MBX - 1) / MBX, nb = gx * ((K.ny + MBY - 1) / MBY);
    hipLaunchKernelGGL(k_macros, dim3(nb), dim3(MBX, MBY), 0, s, K, w, gx, nb, fields ? 1 : 0);
    note(hipGetLastError());
  }
  template <class IO, class R, bool U, class S, int V, bool TG>
  void tiles(const Consts &K, const Work &w, const IO &src, const IO &dst) {
    const int ntx = tiles_x<S>(K), nt = ntx * tiles_y<S>(K);
    if (e0)
      hipExtLaunchKernelGGL((k_fused_tile<IO, R, U, S, V, TG>), dim3(nt), dim3(NTHR), 0, s, e0,
                            e1, 0, K, w, src, dst, ntx, nt);
    else
      hipLaunchKernelGGL((k_fused_tile<IO, R, U, S, V, TG>), dim3(nt), dim3(NTHR), 0, s, K, w,
                         src, dst, ntx, nt);
    note(hipGetLastError());
  }
};

template <class IO>
hipError_t step(const FmaStepArgs *a) {
  if (a->io_bytes != sizeof(IO)) return hipErrorInvalidValue;
  Consts K;
  Work w;
  IO src, dst;
  memcpy(&K, a->K, sizeof K);
  memcpy(&w, a->w, sizeof w);
  memcpy(&src, a->src, sizeof src);
  memcpy(&dst, a->dst, sizeof dst);
  FmaEx ex{a->stream, hipSuccess, a->e0, a->e1};
  with_fused_kernel(a->shape, K, a->resident != 0, [&](auto u, auto sh, auto v, auto tg) {
    seq_fused_step<FmaEx, IO, double, decltype(u)::value, decltype(sh), decltype(v)::value,
                   decltype(tg)::value>(ex, K, w, src, dst, a->sums_ready != 0);
  });
  return ex.err;
}

}  // namespace
}  // namespace dg_fma

hipError_t dugks2p_fma_step(const FmaStepArgs *a) {
  if (!a || a->K_bytes != sizeof(dg_fma::Consts) || a->w_bytes != sizeof(dg_fma::Work))
    return hipErrorInvalidValue;
  return a->fp32 ? dg_fma::step<dg_fma::IoE32>(a) : dg_fma::step<dg_fma::IoF64>(a);
}
