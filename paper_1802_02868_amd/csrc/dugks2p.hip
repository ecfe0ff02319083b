// dugks2p.hip -- C-ABI runtime of the MI355X two-phase DUGKS library
// (declarations and argument contracts in include/dugks2p.h).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "dugks2p_adjoint.hpp"
#include "dugks2p_fma.h"
#include "dugks2p_fused.hpp"
#include "dugks2p_host.hpp"

using namespace dg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess)                                                            \
      return fail(DUGKS2P_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));     \
  } while (0)

// One thread per (i, j) in a 64 x 4 block.  The grid is one-dimensional:
// workgroups are dealt to the 8 XCDs round robin, and xcd_tile gives each
// XCD a contiguous run of blocks (a band of rows), so that the rows a
// stencil reads above and below a block sit in the same XCD's L2.  xcd = 0
// keeps the plain row-major block order (measured faster for the staged
// step's face kernels, slower for the adjoint's per-cell stages).
template <class F>
__global__ __launch_bounds__(256) void k_grid(F f, int n0, int n1, int gx, int nb, int xcd) {
  const int b = xcd ? xcd_tile(blockIdx.x, nb) : (int)blockIdx.x;
  const int i = (b % gx) * 64 + threadIdx.x;
  const int j = (b / gx) * 4 + threadIdx.y;
  if (i < n0 && j < n1) f(i, j);
}

// Event pairs of the tile-kernel launches of a handle while timing is
// enabled (dugks2p_profile).  The launch itself sets them to the kernel's
// start and end (hipExtLaunchKernelGGL), so no marker packets are timed.
// Events are created on first use and reused.
struct KernelTimer {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  bool on = false;
  hipError_t pair(hipEvent_t &a, hipEvent_t &b) {
    while (ev.size() < used + 2) {
      hipEvent_t e;
      const hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ev.push_back(e);
    }
    a = ev[used];
    b = ev[used + 1];
    used += 2;
    return hipSuccess;
  }
};

struct GpuEx {
  hipStream_t s;
  hipError_t err;
  KernelTimer *kt = nullptr;
  int xcd = 1;  // block order of the per-cell kernels (see k_grid)
  template <class F>
  void grid(const F &f, int n0, int n1) {
    if (n0 <= 0 || n1 <= 0) return;
    const int gx = (n0 + 63) / 64, nb = gx * ((n1 + 3) / 4);
    hipLaunchKernelGGL(k_grid<F>, dim3(nb), dim3(64, 4), 0, s, f, n0, n1, gx, nb, xcd);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess && err == hipSuccess) err = e;
  }
  void macros(const Consts &K, const Work &w, bool fields) {
    const int gx = (K.nx + MBX - 1) / MBX, nb = gx * ((K.ny + MBY - 1) / MBY);
    hipLaunchKernelGGL(k_macros, dim3(nb), dim3(MBX, MBY), 0, s, K, w, gx, nb, fields ? 1 : 0);
    note(hipGetLastError());
  }
  void macros_tape(const Consts &K, const Work &w, const Work &t) {
    const int gx = (K.nx + MBX - 1) / MBX, nb = gx * ((K.ny + MBY - 1) / MBY);
    hipLaunchKernelGGL(k_macros_tape, dim3(nb), dim3(MBX, MBY), 0, s, K, w, t, gx, nb);
    note(hipGetLastError());
  }
  template <class IO, class R, bool U, class S, int V, bool TG>
  void tiles(const Consts &K, const Work &w, const IO &src, const IO &dst) {
    const int ntx = tiles_x<S>(K), nt = ntx * tiles_y<S>(K);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (kt && kt->on) note(kt->pair(e0, e1));
    if (e0)
      hipExtLaunchKernelGGL((k_fused_tile<IO, R, U, S, V, TG>), dim3(nt), dim3(NTHR), 0, s, e0,
                            e1, 0, K, w, src, dst, ntx, nt);
    else
      hipLaunchKernelGGL((k_fused_tile<IO, R, U, S, V, TG>), dim3(nt), dim3(NTHR), 0, s, K, w,
                         src, dst, ntx, nt);
    note(hipGetLastError());
  }
  // the adjoint's face stage over square tiles
  void adj_faces(const Consts &K, const Work &w, const AdjWork &a) {
    const int ntx = tiles_x<TileSq>(K), nt = ntx * tiles_y<TileSq>(K);
    hipLaunchKernelGGL(k_adj_faces<TileSq>, dim3(nt), dim3(NTHR), 0, s, K, w, a, ntx, nt);
    note(hipGetLastError());
  }
  void adj_cells(const Consts &K, const Work &w, const AdjWork &a, const double *st) {
    const int ntx = tiles_x<TileSq>(K), nt = ntx * tiles_y<TileSq>(K);
    hipLaunchKernelGGL(k_adj_cells<TileSq>, dim3(nt), dim3(NTHR), 0, s, K, w, a, st, ntx, nt);
    note(hipGetLastError());
  }
  void note(hipError_t e) {
    if (e != hipSuccess && err == hipSuccess) err = e;
  }
};

// Monitor partial sums: one 64 x 4 block of cells per workgroup, fixed-order
// tree in LDS, one partial per block.  A single-workgroup pass then adds the
// partials in block order, so the result is deterministic.
template <class IO>
__global__ __launch_bounds__(256) void k_mon_partial(Consts K, Work w, IO st, double *part) {
  __shared__ double sh[5][256];
  const int t = threadIdx.y * 64 + threadIdx.x;
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < K.nx && j < K.ny) monitor_terms(K, w, st, i, j, v);
  for (int m = 0; m < 5; ++m) sh[m][t] = v[m];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      for (int m = 0; m < 5; ++m) {
        if (m == 3)
          sh[m][t] = sh[m][t] > sh[m][t + s] ? sh[m][t] : sh[m][t + s];
        else
          sh[m][t] = sh[m][t] + sh[m][t + s];
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    for (int m = 0; m < 5; ++m) part[5 * b + m] = sh[m][0];
  }
}

__global__ __launch_bounds__(256) void k_mon_final(const double *part, long long nb, double *out) {
  __shared__ double sh[5][256];
  const int t = threadIdx.x;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long b = t; b < nb; b += 256)
    for (int m = 0; m < 5; ++m) {
      const double x = part[5 * b + m];
      if (m == 3)
        v[m] = v[m] > x ? v[m] : x;
      else
        v[m] += x;
    }
  for (int m = 0; m < 5; ++m) sh[m][t] = v[m];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s)
      for (int m = 0; m < 5; ++m) {
        if (m == 3)
          sh[m][t] = sh[m][t] > sh[m][t + s] ? sh[m][t] : sh[m][t + s];
        else
          sh[m][t] = sh[m][t] + sh[m][t + s];
      }
    __syncthreads();
  }
  if (t == 0)
    for (int m = 0; m < 5; ++m) out[m] = sh[m][0];
}

// Monitors into device memory (dugks2p_monitors_noalloc): v[5] as
// k_mon_final leaves them -> out[6] with max |u| = sqrt(max |u|^2) and the
// step count.
__global__ void k_mon_out(const double *v, double step, double *out) {
  out[0] = v[0];
  out[1] = v[1];
  out[2] = v[2];
  out[3] = sqrt(v[3]);
  out[4] = v[4];
  out[5] = step;
}

// Observables (dugks2p_observables): per 64 x 4 block of cells, the sums
// (cells above the median level, their area, c|V|, c|V| x, c|V| y, c|V| u_x,
// c|V| u_y with c = (phi - phi_B)/(phi_A - phi_B)) and the largest and
// smallest y of the median-level crossings between each cell and the cell
// above it; then one workgroup adds the partials in block order (the sums
// are deterministic; max and min are exact).
enum { NOBS = 9 };
__global__ __launch_bounds__(256) void k_obs_partial(Consts K, Work w, const double *xc,
                                                     const double *yc, double *part) {
  __shared__ double sh[NOBS][256];
  const int t = threadIdx.y * 64 + threadIdx.x;
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y;
  double v[NOBS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -INFINITY, INFINITY};
  if (i < K.nx && j < K.ny) {
    const i64 c = (i64)j * K.ld + i;
    const double V = K.ax[0].w[i] * K.ax[1].w[j];
    const double ph = w.phi[c], mid = 0.5 * (K.phi_a + K.phi_b);
    const double cv = (ph - K.phi_b) / (K.phi_a - K.phi_b) * V;
    if (ph > mid) {
      v[0] = 1.0;
      v[1] = V;
    }
    v[2] = cv;
    v[3] = cv * xc[i];
    v[4] = cv * yc[j];
    v[5] = cv * w.ux[c];
    v[6] = cv * w.uy[c];
    if (j + 1 < K.ny) {
      const double p1 = w.phi[c + K.ld];
      if ((ph > mid) != (p1 > mid)) {
        const double y = yc[j] + (mid - ph) / (p1 - ph) * (yc[j + 1] - yc[j]);
        v[7] = y;
        v[8] = y;
      }
    }
  }
  for (int m = 0; m < NOBS; ++m) sh[m][t] = v[m];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      for (int m = 0; m < NOBS; ++m) {
        const double a = sh[m][t], b = sh[m][t + s];
        sh[m][t] = m == 7 ? (a > b ? a : b) : (m == 8 ? (a < b ? a : b) : a + b);
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    for (int m = 0; m < NOBS; ++m) part[NOBS * b + m] = sh[m][0];
  }
}

__global__ __launch_bounds__(256) void k_obs_final(const double *part, long long nb, double *out) {
  __shared__ double sh[NOBS][256];
  const int t = threadIdx.x;
  double v[NOBS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -INFINITY, INFINITY};
  for (long long b = t; b < nb; b += 256)
    for (int m = 0; m < NOBS; ++m) {
      const double x = part[NOBS * b + m];
      v[m] = m == 7 ? (v[m] > x ? v[m] : x) : (m == 8 ? (v[m] < x ? v[m] : x) : v[m] + x);
    }
  for (int m = 0; m < NOBS; ++m) sh[m][t] = v[m];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s)
      for (int m = 0; m < NOBS; ++m) {
        const double a = sh[m][t], b = sh[m][t + s];
        sh[m][t] = m == 7 ? (a > b ? a : b) : (m == 8 ? (a < b ? a : b) : a + b);
      }
    __syncthreads();
  }
  if (t == 0)
    for (int m = 0; m < NOBS; ++m) out[m] = sh[m][0];
}

// The Laplace-test pressure P = p0 - kappa phi lap(phi) + kappa |grad phi|^2 / 2
// + p, p0 = phi dpsi/dphi - psi (Sec. 3.1), in the order the oracle writes
// it, into a dense [ny][nx] field.
struct FLaplaceP {
  Consts K;
  Work w;
  double *P;
  DFN void operator()(int i, int j) const {
    const i64 c = (i64)j * K.ld + i;
    const double ph = w.phi[c], b = K.beta, k = K.kappa, pa = K.phi_a, pb = K.phi_b;
    const double a1 = ph - pa, b1 = ph - pb;
    const double psi = b * (a1 * a1) * (b1 * b1);
    const double dpsi = 2.0 * b * a1 * b1 * (2.0 * ph - pa - pb);
    const double d1x = stx(K, K.ax[0].d1, w.phi, i, j), d2x = stx(K, K.ax[0].d2, w.phi, i, j);
    const double d1y = sty(K, K.ax[1].d1, w.phi, i, j), d2y = sty(K, K.ax[1].d2, w.phi, i, j);
    P[(i64)j * K.nx + i] = ph * dpsi - psi - k * ph * (d2x + d2y) +
                           0.5 * k * (d1x * d1x + d1y * d1y) + w.p[c];
  }
};

// Number of non-finite populations of a state, added into *cnt (a rare
// event, so one atomic per thread that finds any).
template <class IO>
__global__ __launch_bounds__(256) void k_count_nonfinite(Consts K, IO st,
                                                         unsigned long long *cnt) {
  const i64 n = (i64)K.nx * K.ny;
  unsigned int bad = 0;
  for (i64 r = (i64)blockIdx.x * 256 + threadIdx.x; r < n; r += (i64)gridDim.x * 256) {
    const i64 j = r / K.nx, i = r - j * K.nx;
    double v[18];
    st.load(j * K.ld + i, v);
    for (int q = 0; q < 18; ++q)
      if (!(v[q] - v[q] == 0.0)) ++bad;
  }
  if (bad) atomicAdd(cnt, (unsigned long long)bad);
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

// State <-> FP64 [18][ny][nx], one thread per cell.
template <class IO>
__global__ __launch_bounds__(256) void k_pops_out(Consts K, IO st, double *dst) {
  const i64 n = (i64)K.nx * K.ny;
  for (i64 r = (i64)blockIdx.x * 256 + threadIdx.x; r < n; r += (i64)gridDim.x * 256) {
    const i64 j = r / K.nx, i = r - j * K.nx;
    double v[18];
    st.load(j * K.ld + i, v);
    for (int q = 0; q < 18; ++q) dst[q * n + r] = v[q];
  }
}

template <class IO>
__global__ __launch_bounds__(256) void k_pops_in(Consts K, const double *src, IO st) {
  const i64 n = (i64)K.nx * K.ny;
  for (i64 r = (i64)blockIdx.x * 256 + threadIdx.x; r < n; r += (i64)gridDim.x * 256) {
    const i64 j = r / K.nx, i = r - j * K.nx;
    double v[18];
    for (int q = 0; q < 18; ++q) v[q] = src[q * n + r];
    st.store(j * K.ld + i, v);
  }
}

}  // namespace

struct dugks2p {
  Consts K;
  Layout L;
  hipStream_t stream;
  int precision, kernel, tile;
  unsigned char *ws;
  bool own_ws;
  void *state[2];
  int cur;
  Work w;
  double *mon_part, *mon_out;
  double *xc, *yc;  // cell centres (device)
  int64_t nstep;
  KernelTimer kt;
  bool sums_ok;  // w.phi, s0, jx, jy hold the sums of state[cur]
  int64_t check_every;  // dugks2p_set_checks: 0 = no checks in dugks2p_step
  int device;           // HIP device current at creation (holds the workspace)
};

namespace {

// Both reconstructions run on the fused tile kernel (UPWIND with the
// two-ring tiles) unless the staged kernels are asked for.
bool use_staged(const dugks2p_params *P) { return P->kernel == DUGKS2P_KERNEL_STAGED; }
// the fused forms (exact and FMA-contracted) share the tile kernel's host logic
bool is_fused(int kernel) {
  return kernel == DUGKS2P_KERNEL_FUSED || kernel == DUGKS2P_KERNEL_FUSED_FMA;
}

struct Prepared {
  AxisHost ax, ay;
  Consts K;
  Layout L;
};

std::string prepare(const dugks2p_params *P, Prepared &pr) {
  std::string e = validate(P);
  if (!e.empty()) return e;
  build_axis(pr.ax, P->nx, P->bc_x, P->x_faces);
  build_axis(pr.ay, P->ny, P->bc_y, P->y_faces);
  pr.K = make_consts(P, pr.ax, pr.ay);
  if (!(pr.K.dt > 0.0) || !isfinite(pr.K.dt)) return "time step is not positive";
  if (P->precision == DUGKS2P_FP32_STATE && use_staged(P))
    return "the FP32-state form runs on the fused kernel";
  pr.L = make_layout(pr.K, pr.ax, pr.ay, P->precision, use_staged(P));
  return std::string();
}

// Enqueue one time step from state[cur] into state[1 - cur] with tile shape
// `shape` (fused form), without committing it.
int enqueue_step(dugks2p *h, int shape) {
  // the tile code takes interior-face reconstruction from the tile shape
  if (is_fused(h->kernel) &&
      (shape == DUGKS2P_TILE_UPWIND) != (h->K.recon != DUGKS2P_RECON_CENTRAL))
    return fail(DUGKS2P_EINVAL, "tile shape does not match the face reconstruction");
  GpuEx ex{h->stream, hipSuccess, &h->kt};
  // a ping-pong state small enough to stay in the MALL
  const bool resident = 2.0 * (double)h->L.state_bytes <= TILDE_OUT_MAX_STATE_BYTES;
  if (h->kernel == DUGKS2P_KERNEL_FUSED_FMA) {
    // the FMA-contracted build of the same step (dugks2p_fma.hip)
    const bool f32 = h->precision != DUGKS2P_FP64;
    const IoF64 s64 = io_f64(h->state[h->cur], h->K), d64 = io_f64(h->state[1 - h->cur], h->K);
    const IoE32 s32 = io_e32(h->state[h->cur], h->K, h->L);
    const IoE32 d32 = io_e32(h->state[1 - h->cur], h->K, h->L);
    FmaStepArgs a;
    a.K = &h->K;
    a.K_bytes = sizeof h->K;
    a.w = &h->w;
    a.w_bytes = sizeof h->w;
    a.fp32 = f32 ? 1 : 0;
    a.src = f32 ? (const void *)&s32 : (const void *)&s64;
    a.dst = f32 ? (const void *)&d32 : (const void *)&d64;
    a.io_bytes = f32 ? sizeof s32 : sizeof s64;
    a.sums_ready = h->sums_ok ? 1 : 0;
    a.shape = shape;
    a.resident = resident ? 1 : 0;
    a.stream = h->stream;
    a.e0 = a.e1 = nullptr;
    if (h->kt.on) ex.note(h->kt.pair(a.e0, a.e1));
    ex.note(dugks2p_fma_step(&a));
  } else if (h->precision == DUGKS2P_FP64 && h->kernel == DUGKS2P_KERNEL_STAGED) {
    ex.xcd = 0;
    seq_staged_step<GpuEx, double, double>(ex, h->K, h->w, (const double *)h->state[h->cur],
                                           (double *)h->state[1 - h->cur]);
  } else if (h->precision == DUGKS2P_FP64) {
    const IoF64 src = io_f64(h->state[h->cur], h->K), dst = io_f64(h->state[1 - h->cur], h->K);
    with_fused_kernel(shape, h->K, resident, [&](auto u, auto sh, auto v, auto tg) {
      seq_fused_step<GpuEx, IoF64, double, decltype(u)::value, decltype(sh), decltype(v)::value,
                     decltype(tg)::value>(ex, h->K, h->w, src, dst, h->sums_ok);
    });
  } else {
    const IoE32 src = io_e32(h->state[h->cur], h->K, h->L);
    const IoE32 dst = io_e32(h->state[1 - h->cur], h->K, h->L);
    with_fused_kernel(shape, h->K, resident, [&](auto u, auto sh, auto v, auto tg) {
      seq_fused_step<GpuEx, IoE32, double, decltype(u)::value, decltype(sh), decltype(v)::value,
                     decltype(tg)::value>(ex, h->K, h->w, src, dst, h->sums_ok);
    });
  }
  if (ex.err != hipSuccess)
    return fail(DUGKS2P_EHIP, std::string("kernel launch: ") + hipGetErrorString(ex.err));
  // a fused step leaves the sums of state[cur] in w (computed or kept)
  if (is_fused(h->kernel)) h->sums_ok = true;
  return DUGKS2P_OK;
}

// One time step on the handle's stream.
int launch_step(dugks2p *h) {
  const int rc = enqueue_step(h, h->tile);
  if (rc) return rc;
  h->cur = 1 - h->cur;
  h->nstep++;
  // the tile kernel wrote the new state's sums into the spare planes
  if (is_fused(h->kernel)) swap_sums(h->w);
  else h->sums_ok = false;
  return DUGKS2P_OK;
}

// Tile-shape tuner: time a few uncommitted steps with each shape (the step
// writes only the spare ping-pong buffer and the work fields, which the next
// real step rewrites) and keep the fastest.  Results do not depend on the
// shape, only the speed does.
int tune_tile(dugks2p *h) {
  const bool upw = h->K.recon != DUGKS2P_RECON_CENTRAL;
  if (!is_fused(h->kernel) || !h->K.unit || upw) {
    h->tile = is_fused(h->kernel) && upw ? DUGKS2P_TILE_UPWIND : DUGKS2P_TILE_SQUARE;
    return DUGKS2P_OK;
  }
  enum { WARM = 1, REPS = 3 };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = DUGKS2P_OK;
  float best = 0.0f;
  int pick = DUGKS2P_TILE_SQUARE;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = fail(DUGKS2P_EHIP, "tuner events");
  for (int shape = DUGKS2P_TILE_SQUARE; rc == DUGKS2P_OK && shape <= DUGKS2P_TILE_TALL; ++shape) {
    for (int r = 0; r < WARM + REPS && rc == DUGKS2P_OK; ++r) {
      if (r == WARM && hipEventRecord(e0, h->stream) != hipSuccess)
        rc = fail(DUGKS2P_EHIP, "tuner event");
      if (rc == DUGKS2P_OK) rc = enqueue_step(h, shape);
    }
    float ms = 0.0f;
    if (rc == DUGKS2P_OK &&
        (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = fail(DUGKS2P_EHIP, "tuner timing");
    if (rc == DUGKS2P_OK && (shape == DUGKS2P_TILE_SQUARE || ms < best)) {
      best = ms;
      pick = shape;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  h->tile = pick;
  return rc;
}

// Count the non-finite populations of the current state; synchronises the
// stream.  The counter is a spare slot after the monitor partials.
int count_nonfinite(dugks2p *h, unsigned long long &bad) {
  unsigned long long *cnt = (unsigned long long *)(h->mon_out + 12);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, h->stream, cnt);
  HIPCHK(hipGetLastError());
  if (h->precision == DUGKS2P_FP64)
    hipLaunchKernelGGL(k_count_nonfinite<IoF64>, dim3(1024), dim3(256), 0, h->stream, h->K,
                       io_f64(h->state[h->cur], h->K), cnt);
  else
    hipLaunchKernelGGL(k_count_nonfinite<IoE32>, dim3(1024), dim3(256), 0, h->stream, h->K,
                       io_e32(h->state[h->cur], h->K, h->L), cnt);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(&bad, cnt, sizeof bad, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DUGKS2P_OK;
}

// Cell fields of the current state into the work arrays.
int launch_macros(dugks2p *h) {
  GpuEx ex{h->stream, hipSuccess};
  if (h->precision == DUGKS2P_FP64)
    seq_moments(ex, h->K, h->w, io_f64(h->state[h->cur], h->K));
  else
    seq_moments(ex, h->K, h->w, io_e32(h->state[h->cur], h->K, h->L));
  if (ex.err != hipSuccess)
    return fail(DUGKS2P_EHIP, std::string("kernel launch: ") + hipGetErrorString(ex.err));
  return DUGKS2P_OK;
}

}  // namespace

extern "C" {

size_t dugks2p_workspace_bytes(const dugks2p_params *P) {
  Prepared pr;
  if (!prepare(P, pr).empty()) return 0;
  return pr.L.total;
}

int dugks2p_create(const dugks2p_params *P, const double *phi0, const double *ux0,
                   const double *uy0, const double *p0, void *hip_stream, dugks2p **out) {
  if (!out) return fail(DUGKS2P_EINVAL, "out is NULL");
  *out = nullptr;
  if (!phi0 || !ux0 || !uy0 || !p0) return fail(DUGKS2P_EINVAL, "initial field pointer is NULL");
  Prepared pr;
  const std::string e = prepare(P, pr);
  if (!e.empty()) return fail(DUGKS2P_EINVAL, e);
  if (P->workspace && P->workspace_bytes < pr.L.total)
    return fail(DUGKS2P_ENOMEM, "workspace smaller than dugks2p_workspace_bytes()");
  if (P->workspace && ((uintptr_t)P->workspace & 255))
    return fail(DUGKS2P_EINVAL, "workspace must be 256-byte aligned");

  dugks2p *h = new dugks2p();
  h->K = pr.K;
  h->L = pr.L;
  h->stream = (hipStream_t)hip_stream;
  h->precision = P->precision;
  h->kernel = use_staged(P) ? DUGKS2P_KERNEL_STAGED
                            : (P->kernel == DUGKS2P_KERNEL_FUSED_FMA ? DUGKS2P_KERNEL_FUSED_FMA
                                                                     : DUGKS2P_KERNEL_FUSED);
  if (is_fused(h->kernel) && P->recon != DUGKS2P_RECON_CENTRAL)
    h->tile = DUGKS2P_TILE_UPWIND;
  else
    h->tile = (is_fused(h->kernel) && pr.K.unit && P->tile != DUGKS2P_TILE_AUTO)
                  ? P->tile
                  : DUGKS2P_TILE_SQUARE;
  h->cur = 0;
  h->nstep = 0;
  h->check_every = 0;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(DUGKS2P_EHIP, "hipGetDevice");
  }
  h->sums_ok = false;
  if (P->workspace) {
    h->ws = (unsigned char *)P->workspace;
    h->own_ws = false;
  } else {
    void *p = nullptr;
    const hipError_t err = hipMalloc(&p, pr.L.total);
    if (err != hipSuccess) {
      delete h;
      return fail(DUGKS2P_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(err));
    }
    h->ws = (unsigned char *)p;
    h->own_ws = true;
  }
  int rc = DUGKS2P_OK;
  do {
    std::vector<unsigned char> tb;
    pack_axis(pr.ax, tb);
    if (hipMemcpyAsync(h->ws + pr.L.tables[0], tb.data(), tb.size(), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess) { rc = fail(DUGKS2P_EHIP, "table upload"); break; }
    // the staging vector must outlive the copy
    if (hipStreamSynchronize(h->stream) != hipSuccess) { rc = fail(DUGKS2P_EHIP, "sync"); break; }
    pack_axis(pr.ay, tb);
    if (hipMemcpyAsync(h->ws + pr.L.tables[1], tb.data(), tb.size(), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess) { rc = fail(DUGKS2P_EHIP, "table upload"); break; }
    if (hipStreamSynchronize(h->stream) != hipSuccess) { rc = fail(DUGKS2P_EHIP, "sync"); break; }
    h->K.ax[0] = bind_axis(pr.ax, h->ws + pr.L.tables[0]);
    h->K.ax[1] = bind_axis(pr.ay, h->ws + pr.L.tables[1]);
    h->w = bind_work(pr.L, h->K, h->ws);
    h->state[0] = h->ws + pr.L.state[0];
    h->state[1] = h->ws + pr.L.state[1];
    h->mon_part = (double *)(h->ws + pr.L.mon);
    h->mon_out = h->mon_part + NOBS * pr.L.mon_blocks;
    h->xc = (double *)(h->ws + pr.L.centres);
    h->yc = h->xc + pr.K.nx;
    {
      std::vector<double> cc(pr.ax.c);
      cc.insert(cc.end(), pr.ay.c.begin(), pr.ay.c.end());
      if (hipMemcpyAsync(h->xc, cc.data(), sizeof(double) * cc.size(), hipMemcpyHostToDevice,
                         h->stream) != hipSuccess ||
          hipStreamSynchronize(h->stream) != hipSuccess) {
        rc = fail(DUGKS2P_EHIP, "centre upload");
        break;
      }
    }
    if (hipMemsetAsync(h->state[0], 0, pr.L.state_bytes, h->stream) != hipSuccess ||
        hipMemsetAsync(h->state[1], 0, pr.L.state_bytes, h->stream) != hipSuccess) {
      rc = fail(DUGKS2P_EHIP, "state clear");
      break;
    }
    GpuEx ex{h->stream, hipSuccess};
    if (P->precision == DUGKS2P_FP64)
      seq_init(ex, h->K, h->w, phi0, ux0, uy0, p0, io_f64(h->state[0], h->K));
    else
      seq_init(ex, h->K, h->w, phi0, ux0, uy0, p0, io_e32(h->state[0], h->K, h->L));
    if (ex.err != hipSuccess) {
      rc = fail(DUGKS2P_EHIP, std::string("init launch: ") + hipGetErrorString(ex.err));
      break;
    }
    if (P->tile == DUGKS2P_TILE_AUTO) rc = tune_tile(h);
  } while (0);
  if (rc != DUGKS2P_OK) {
    (void)hipStreamSynchronize(h->stream);
    if (h->own_ws) (void)hipFree(h->ws);
    delete h;
    return rc;
  }
  *out = h;
  return DUGKS2P_OK;
}

int dugks2p_step(dugks2p *h, int64_t nsteps) {
  if (!h) return fail(DUGKS2P_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(DUGKS2P_EINVAL, "nsteps must be >= 0");
  for (int64_t n = 0; n < nsteps; ++n) {
    int rc = launch_step(h);
    if (rc) return rc;
    // optional checks (dugks2p_set_checks): after every check_every-th step
    // of the call and after its last step
    if (h->check_every > 0 && ((n + 1) % h->check_every == 0 || n + 1 == nsteps)) {
      unsigned long long bad = 0;
      rc = count_nonfinite(h, bad);
      if (rc) return rc;
      if (bad)
        return fail(DUGKS2P_ENONFINITE, std::to_string(bad) +
                                            " non-finite populations in the state after step " +
                                            std::to_string(h->nstep));
    }
  }
  return DUGKS2P_OK;
}

int dugks2p_set_checks(dugks2p *h, int64_t every) {
  if (!h) return fail(DUGKS2P_EINVAL, "handle is NULL");
  if (every < 0) return fail(DUGKS2P_EINVAL, "every must be >= 0");
  h->check_every = every;
  return DUGKS2P_OK;
}

int dugks2p_moments(dugks2p *h, double *phi, double *rho, double *ux, double *uy, double *p) {
  if (!h) return fail(DUGKS2P_EINVAL, "handle is NULL");
  const int rc = launch_macros(h);
  if (rc) return rc;
  GpuEx ex{h->stream, hipSuccess};
  ex.grid(FMoments{h->K, h->w, phi, rho, ux, uy, p}, h->K.nx, h->K.ny);
  if (ex.err != hipSuccess)
    return fail(DUGKS2P_EHIP, std::string("moments launch: ") + hipGetErrorString(ex.err));
  return DUGKS2P_OK;
}

int dugks2p_monitors(dugks2p *h, double out[6]) {
  if (!h || !out) return fail(DUGKS2P_EINVAL, "NULL argument");
  const int rc = launch_macros(h);
  if (rc) return rc;
  const dim3 b(64, 4), g((h->K.nx + 63) / 64, (h->K.ny + 3) / 4);
  const long long nb = (long long)g.x * g.y;
  if (nb > (long long)h->L.mon_blocks) return fail(DUGKS2P_EHIP, "monitor partial buffer too small");
  if (h->precision == DUGKS2P_FP64)
    hipLaunchKernelGGL(k_mon_partial<IoF64>, g, b, 0, h->stream, h->K, h->w,
                       io_f64(h->state[h->cur], h->K), h->mon_part);
  else
    hipLaunchKernelGGL(k_mon_partial<IoE32>, g, b, 0, h->stream, h->K, h->w,
                       io_e32(h->state[h->cur], h->K, h->L), h->mon_part);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_mon_final, dim3(1), dim3(256), 0, h->stream, h->mon_part, nb, h->mon_out);
  HIPCHK(hipGetLastError());
  double v[5];
  HIPCHK(hipMemcpyAsync(v, h->mon_out, sizeof v, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  out[0] = v[0];
  out[1] = v[1];
  out[2] = v[2];
  out[3] = sqrt(v[3]);
  out[4] = v[4];
  out[5] = (double)h->nstep;
  if (v[4] > 0.0) return fail(DUGKS2P_ENONFINITE, "non-finite populations in the state");
  return DUGKS2P_OK;
}

}  // extern "C"

// Scratch of dugks2p_monitors_noalloc: the per-block monitor partials and
// the five reduced values, in a statically allocated array that every GPU
// the library runs on holds until the process ends.  Host code never uses
// the array's name as an address: the device address of each GPU's copy is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and kept in scratch_dev.
namespace {
enum : long long { SCRATCH_DOUBLES = 2 * 1024 * 1024 };  // 16 MiB
enum { SCRATCH_MAX_DEV = 64 };
}  // namespace
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {
std::mutex scratch_mu;
double *scratch_dev[SCRATCH_MAX_DEV];

// Device address of `scratch` on device dev, which must be current.
int scratch_ptr(int dev, double **out) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEV) return fail(DUGKS2P_EUNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DUGKS2P_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                    hipGetErrorString(e));
    scratch_dev[dev] = (double *)p;
  }
  *out = scratch_dev[dev];
  return DUGKS2P_OK;
}
}  // namespace

extern "C" {

int dugks2p_monitors_noalloc(dugks2p *h, double *out) {
  if (!h || !out) return fail(DUGKS2P_EINVAL, "NULL argument");
  const dim3 b(64, 4), g((h->K.nx + 63) / 64, (h->K.ny + 3) / 4);
  const long long nb = (long long)g.x * g.y;
  if (5 * nb + 8 > SCRATCH_DOUBLES)
    return fail(DUGKS2P_EINVAL, "grid too large for the static monitor scratch: " +
                                    std::to_string(nb) + " blocks of 64 x 4 cells, at most " +
                                    std::to_string((SCRATCH_DOUBLES - 8) / 5));
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != h->device) HIPCHK(hipSetDevice(h->device));
  double *part = nullptr;
  int rc = scratch_ptr(h->device, &part);
  if (rc == DUGKS2P_OK) rc = launch_macros(h);
  if (rc == DUGKS2P_OK) {
    double *v = part + 5 * nb;
    if (h->precision == DUGKS2P_FP64)
      hipLaunchKernelGGL(k_mon_partial<IoF64>, g, b, 0, h->stream, h->K, h->w,
                         io_f64(h->state[h->cur], h->K), part);
    else
      hipLaunchKernelGGL(k_mon_partial<IoE32>, g, b, 0, h->stream, h->K, h->w,
                         io_e32(h->state[h->cur], h->K, h->L), part);
    hipLaunchKernelGGL(k_mon_final, dim3(1), dim3(256), 0, h->stream, (const double *)part, nb,
                       v);
    hipLaunchKernelGGL(k_mon_out, dim3(1), dim3(1), 0, h->stream, (const double *)v,
                       (double)h->nstep, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = fail(DUGKS2P_EHIP, std::string("monitor launch: ") + hipGetErrorString(e));
  }
  if (cur != h->device) (void)hipSetDevice(cur);
  return rc;
}

int dugks2p_laplace_pressure(dugks2p *h, double *P) {
  if (!h || !P) return fail(DUGKS2P_EINVAL, "NULL argument");
  const int rc = launch_macros(h);
  if (rc) return rc;
  GpuEx ex{h->stream, hipSuccess};
  ex.grid(FLaplaceP{h->K, h->w, P}, h->K.nx, h->K.ny);
  if (ex.err != hipSuccess)
    return fail(DUGKS2P_EHIP, std::string("pressure launch: ") + hipGetErrorString(ex.err));
  return DUGKS2P_OK;
}

int dugks2p_observables(dugks2p *h, double out[8]) {
  if (!h || !out) return fail(DUGKS2P_EINVAL, "NULL argument");
  const int rc = launch_macros(h);
  if (rc) return rc;
  const dim3 b(64, 4), g((h->K.nx + 63) / 64, (h->K.ny + 3) / 4);
  const long long nb = (long long)g.x * g.y;
  if (nb > (long long)h->L.mon_blocks) return fail(DUGKS2P_EHIP, "partial buffer too small");
  hipLaunchKernelGGL(k_obs_partial, g, b, 0, h->stream, h->K, h->w, (const double *)h->xc,
                     (const double *)h->yc, h->mon_part);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(256), 0, h->stream, h->mon_part, nb, h->mon_out);
  HIPCHK(hipGetLastError());
  double v[NOBS];
  HIPCHK(hipMemcpyAsync(v, h->mon_out, sizeof v, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  out[0] = v[0];
  out[1] = v[1];
  out[2] = v[3] / v[2];
  out[3] = v[4] / v[2];
  out[4] = v[5] / v[2];
  out[5] = v[6] / v[2];
  out[6] = v[7] == -INFINITY ? NAN : v[7];
  out[7] = v[8] == INFINITY ? NAN : v[8];
  return DUGKS2P_OK;
}

int dugks2p_get_populations(dugks2p *h, double *dst) {
  if (!h || !dst) return fail(DUGKS2P_EINVAL, "NULL argument");
  if (h->precision == DUGKS2P_FP64)
    hipLaunchKernelGGL(k_pops_out<IoF64>, dim3(1024), dim3(256), 0, h->stream, h->K,
                       io_f64(h->state[h->cur], h->K), dst);
  else
    hipLaunchKernelGGL(k_pops_out<IoE32>, dim3(1024), dim3(256), 0, h->stream, h->K,
                       io_e32(h->state[h->cur], h->K, h->L), dst);
  HIPCHK(hipGetLastError());
  return DUGKS2P_OK;
}

int dugks2p_set_populations(dugks2p *h, const double *src) {
  if (!h || !src) return fail(DUGKS2P_EINVAL, "NULL argument");
  h->sums_ok = false;
  if (h->precision == DUGKS2P_FP64)
    hipLaunchKernelGGL(k_pops_in<IoF64>, dim3(1024), dim3(256), 0, h->stream, h->K, src,
                       io_f64(h->state[h->cur], h->K));
  else
    hipLaunchKernelGGL(k_pops_in<IoE32>, dim3(1024), dim3(256), 0, h->stream, h->K, src,
                       io_e32(h->state[h->cur], h->K, h->L));
  HIPCHK(hipGetLastError());
  return DUGKS2P_OK;
}

size_t dugks2p_state_bytes(const dugks2p *h) { return h ? h->L.state_bytes : 0; }

int dugks2p_get_state(dugks2p *h, void *dst) {
  if (!h || !dst) return fail(DUGKS2P_EINVAL, "NULL argument");
  HIPCHK(hipMemcpyAsync(dst, h->state[h->cur], h->L.state_bytes, hipMemcpyDeviceToDevice,
                        h->stream));
  return DUGKS2P_OK;
}

int dugks2p_set_state(dugks2p *h, const void *src) {
  if (!h || !src) return fail(DUGKS2P_EINVAL, "NULL argument");
  h->sums_ok = false;
  HIPCHK(hipMemcpyAsync(h->state[h->cur], src, h->L.state_bytes, hipMemcpyDeviceToDevice,
                        h->stream));
  return DUGKS2P_OK;
}

double dugks2p_dt(const dugks2p *h) { return h ? h->K.dt : 0.0; }
int64_t dugks2p_step_count(const dugks2p *h) { return h ? h->nstep : -1; }
int dugks2p_kernel(const dugks2p *h) { return h ? h->kernel : DUGKS2P_EINVAL; }
int dugks2p_tile(const dugks2p *h) { return h ? h->tile : DUGKS2P_EINVAL; }

int dugks2p_profile(dugks2p *h, int enable) {
  if (!h) return fail(DUGKS2P_EINVAL, "handle is NULL");
  h->kt.on = enable != 0;
  h->kt.used = 0;
  return DUGKS2P_OK;
}

int dugks2p_profile_read(dugks2p *h, double *ms, int64_t *launches) {
  if (!h || !ms || !launches) return fail(DUGKS2P_EINVAL, "NULL argument");
  *ms = 0.0;
  *launches = 0;
  HIPCHK(hipStreamSynchronize(h->stream));
  for (size_t k = 0; k + 1 < h->kt.used; k += 2) {
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, h->kt.ev[k], h->kt.ev[k + 1]));
    *ms += t;
    ++*launches;
  }
  h->kt.used = 0;
  return DUGKS2P_OK;
}

int dugks2p_destroy(dugks2p *h) {
  if (!h) return DUGKS2P_OK;
  (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->kt.ev) (void)hipEventDestroy(e);
  if (h->own_ws) (void)hipFree(h->ws);
  delete h;
  return DUGKS2P_OK;
}

const char *dugks2p_last_error(void) { return g_err.c_str(); }

}  // extern "C"
#include "dugks2p_batch.inc"
#include "dugks2p_adjoint.inc"
