/*
 * dugks2p.h -- C ABI of the MI355X (gfx950) two-phase DUGKS library.
 *
 * The library advances the discrete unified gas-kinetic scheme for
 * immiscible two-phase flows of Zhang, Yang & Guo (arXiv:1802.02868): two
 * D2Q9 populations per cell, f~ for pressure and momentum (eq. bgkf) and g~
 * for the Cahn-Hilliard order parameter (eq. bgkg), on a tensor-product mesh
 * that may be non-uniform in each axis (Sec. 3.2, App. B).  One call of
 * dugks2p_step performs the seven-step procedure at the end of Sec. 2.2 once
 * per time step, entirely in HIP kernels on the caller's stream.
 *
 * Conventions for every entry point:
 *   - return value: DUGKS2P_OK (0) or a negative DUGKS2P_E* code; the
 *     library never aborts or exits.  dugks2p_last_error() returns a
 *     thread-local message describing the last failure of this thread.
 *   - "device" pointers are HIP device allocations on the handle's device
 *     (for instance torch CUDA tensors); "host" pointers are host memory.
 *   - the caller owns every buffer it passes; the library owns the handle
 *     and, unless params.workspace is given, its device workspace.
 *   - fields are FP64, row-major [ny][nx] with x fastest; cell centres are
 *     midpoints of consecutive faces.
 *   - work is enqueued on the stream given at creation; functions that
 *     return host data synchronise that stream.  A handle is not thread safe.
 */
#ifndef DUGKS2P_H
#define DUGKS2P_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DUGKS2P_ABI_VERSION 1

enum {
  DUGKS2P_OK = 0,
  DUGKS2P_EINVAL = -1,      /* invalid argument; nothing was enqueued        */
  DUGKS2P_ENOMEM = -2,      /* device allocation failed or workspace too small */
  DUGKS2P_EHIP = -3,        /* a HIP runtime call failed                     */
  DUGKS2P_ENONFINITE = -4,  /* a population became NaN or infinite            */
  DUGKS2P_EUNSUPPORTED = -5 /* valid request the library cannot perform       */
};

enum { DUGKS2P_BC_PERIODIC = 0, DUGKS2P_BC_WALL = 1 };
enum { DUGKS2P_FP64 = 0, DUGKS2P_FP32_STATE = 1 };
enum { DUGKS2P_RECON_CENTRAL = 0, DUGKS2P_RECON_UPWIND = 1 };
/* Implementation of the step.  AUTO = FUSED.  STAGED: one kernel per stage
 * (FP64 only).  FUSED: cell macros plus one tile kernel, FP64 arithmetic in
 * the oracle's order without FMA contraction (bit-identical results).
 * FUSED_FMA: the same kernels compiled with FMA contraction: a multiply and
 * the add that consumes it may round once, so results differ from the exact
 * form in the last bits and stay within the FP64 parity bar (1e-11 relative
 * max-norm after 1000 steps of the stationary drop); fewer instructions. */
enum {
  DUGKS2P_KERNEL_AUTO = 0,
  DUGKS2P_KERNEL_STAGED = 1,
  DUGKS2P_KERNEL_FUSED = 2,
  DUGKS2P_KERNEL_FUSED_FMA = 3
};
/* Tile shape of the fused kernel: cells per tile (x by y).  AUTO times the
 * shapes on the problem at creation and keeps the fastest.  The wide and
 * tall shapes apply at unit lattice speed (RT = 1/3); otherwise square. */
enum {
  DUGKS2P_TILE_AUTO = 0,
  DUGKS2P_TILE_SQUARE = 1, /* 14 x 14 */
  DUGKS2P_TILE_WIDE = 2,   /* 30 x 6  */
  DUGKS2P_TILE_TALL = 3,   /* 6 x 30  */
  DUGKS2P_TILE_UPWIND = 4  /* 12 x 12 with a two-cell bar+ ring: set by the
                              library for UPWIND reconstruction, whatever
                              tile was asked for */
};

/*
 * Problem statement (Sec. 2 and 3 of the paper).
 *   x_faces, y_faces: host, nx+1 / ny+1 strictly increasing coordinates,
 *                copied at creation (tensor-product mesh, App. B).
 *   bc_x, bc_y:  DUGKS2P_BC_PERIODIC, or DUGKS2P_BC_WALL = bounce-back
 *                no-slip walls at both ends of that axis (needs >= 2 cells).
 *   dt:          > 0 explicit time step; otherwise dt = cfl * h_min / c_max
 *                (eq. cfl) with h_min the smallest cell width of either axis
 *                and c_max = sqrt(6 rt) when c_max <= 0 (Sec. 3).
 *   rt:          RT = c_s^2; discrete speed c = sqrt(3 RT) (eq. D2Q9).
 *   tau_g:       relaxation time of g; mobility lambda gives
 *                eta = lambda / (c_s^2 tau_g) (eq. kineticandmobility).
 *   tau_f:       > 0 uniform relaxation time of f; otherwise
 *                tau_f = mu_d(phi) / (rho c_s^2) with the mixture viscosity
 *                of eq. mixvis built from nu_a, nu_b.
 *   beta, kappa: double-well and gradient coefficients (eqs. doublewell,
 *                chemicalpotential).
 *   phi_a, phi_b, rho_a, rho_b: bulk order parameters and densities
 *                (eqs. oderrho, Gama).
 *   gx, gy, rho_ref: body force F_b = (rho - rho_ref) (gx, gy).
 *   phi_clamp:   nonzero clamps phi into [phi_b, phi_a] inside rho() and
 *                mu_d() only (never in the state).
 *   precision:   DUGKS2P_FP64 (state and arithmetic in double) or
 *                DUGKS2P_FP32_STATE (the populations stored as floats, with
 *                the cell order parameter phi = sum g~ kept in double; every
 *                arithmetic operation of the step still in double).
 *   recon:       face reconstruction of Step 3: CENTRAL = linear
 *                interpolation of value and gradient (the paper's choice);
 *                UPWIND = expansion from the upwind cell.
 *   kernel:      DUGKS2P_KERNEL_* implementation choice (AUTO = fused;
 *                the batched form always runs FUSED).
 *   tile:        DUGKS2P_TILE_* tile shape of the fused kernel (a
 *                performance choice: every shape gives the same results
 *                bit for bit).
 *   workspace:   optional device memory of at least
 *                dugks2p_workspace_bytes(params) bytes, 256-byte aligned,
 *                owned by the caller and used instead of a library allocation.
 */
typedef struct {
  int32_t abi_version; /* DUGKS2P_ABI_VERSION */
  int32_t nx, ny;
  int32_t bc_x, bc_y;
  int32_t precision;
  int32_t recon;
  int32_t phi_clamp;
  int32_t kernel;
  int32_t tile; /* DUGKS2P_TILE_* */
  const double *x_faces;
  const double *y_faces;
  double cfl, c_max, dt, rt;
  double tau_g, mobility, tau_f;
  double beta, kappa;
  double phi_a, phi_b, rho_a, rho_b, nu_a, nu_b;
  double gx, gy, rho_ref;
  void *workspace;
  size_t workspace_bytes;
} dugks2p_params;

typedef struct dugks2p dugks2p;

/* Bytes of device workspace the handle needs for these parameters
 * (0 if the parameters are invalid). */
size_t dugks2p_workspace_bytes(const dugks2p_params *params);

/*
 * Step 1 of Sec. 2.2: validate the parameters, build the mesh tables, and
 * initialise f~, g~ from the initial fields phi0, ux0, uy0, p0 (device, FP64,
 * [ny][nx]) with f = f^eq, g = g^eq, i.e. tilde = eq - (dt/2) F (eq. auxf).
 * hip_stream is a hipStream_t (NULL = default stream).  On success *out
 * holds a new handle; on failure *out is NULL and no work is left enqueued.
 */
int dugks2p_create(const dugks2p_params *params, const double *phi0, const double *ux0,
                   const double *uy0, const double *p0, void *hip_stream, dugks2p **out);

/* Advance nsteps >= 0 time steps (Steps 2-7 of Sec. 2.2) on the handle's
 * stream.  By default the call only enqueues work (asynchronous, no check
 * of the result).  With checks enabled (dugks2p_set_checks), it also counts
 * the non-finite populations after every `every`-th step of the call and
 * after its last step, synchronising the stream for each count, and returns
 * DUGKS2P_ENONFINITE at the first count that is nonzero; the handle then
 * holds that state and dugks2p_step_count() tells how far it ran. */
int dugks2p_step(dugks2p *h, int64_t nsteps);

/* Checks of dugks2p_step: every > 0 enables them (see above), 0 (the
 * default) disables them. */
int dugks2p_set_checks(dugks2p *h, int64_t every);

/* Cell fields at the current time (Step 7: eqs. oderrho, phi, u, P): writes
 * phi, rho, ux, uy, p (device, FP64, [ny][nx]); any pointer may be NULL. */
int dugks2p_moments(dugks2p *h, double *phi, double *rho, double *ux, double *uy, double *p);

/* Monitors at the current time, host out[6]: total order parameter
 * sum phi |V|, kinetic energy sum rho |u|^2 |V| / 2, free energy of eq.
 * freeenergyfunction, max |u|, number of non-finite populations, step
 * count.  Reductions are FP64 with a fixed order (deterministic).  Syncs the
 * stream.  Returns DUGKS2P_ENONFINITE if the count is nonzero (out is still
 * filled). */
int dugks2p_monitors(dugks2p *h, double out[6]);

/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the monitors of dugks2p_monitors, written by kernels on the handle's
 * stream to out (device, 6 doubles, caller-owned) in the same order, with no
 * allocation, no host copy and no synchronisation.  The per-block partials
 * go to a statically allocated 16 MiB device array of the library, one per
 * GPU, held until the process ends: grids of more than 419 428 blocks of
 * 64 x 4 cells (about 107 million cells) return DUGKS2P_EINVAL.  Every call
 * on a GPU shares that GPU's array, so calls that overlap in time on one GPU
 * (on different streams or threads) race and must be ordered by the caller.
 * The non-finite count is out[4]; the return value does not report it. */
int dugks2p_monitors_noalloc(dugks2p *h, double *out);

/* Interface observables at the current time, host out[8]:
 *   out[0]  number of cells with phi above the median level
 *           (phi_A + phi_B)/2: the droplet mass of Sec. 3.1 (Table 1);
 *   out[1]  the area (sum |V|) of those cells;
 *   out[2], out[3]  centroid (x, y) of phase A and
 *   out[4], out[5]  its mean velocity (u_x, u_y), weighted by c |V| with
 *           c = (phi - phi_B)/(phi_A - phi_B) (the rising bubble, Sec. 3.3);
 *   out[6], out[7]  highest and lowest y at which the median level is
 *           crossed between a cell and the cell above it, by linear
 *           interpolation between the two centres: the bubble front and
 *           spike tip of Sec. 3.4 (NaN when the level is not crossed).
 * Positions are in the coordinates of x_faces / y_faces.  Reductions are
 * FP64 with a fixed order (deterministic); the crossings are exact maxima
 * and minima.  Syncs the stream. */
int dugks2p_observables(dugks2p *h, double out[8]);

/* The pressure P of the Laplace test (Sec. 3.1) at the current time:
 * P = p0 - kappa phi lap(phi) + kappa |grad phi|^2 / 2 + p with
 * p0 = phi dpsi/dphi - psi, the derivatives by the App. B stencils; written
 * to P (device, FP64, [ny][nx], caller-owned).  Its jump across a drop's
 * interface is sigma / R for the Laplace law.  Enqueued on the handle's
 * stream. */
int dugks2p_laplace_pressure(dugks2p *h, double *P);

/* The 18 populations (q = 0..8 f~, 9..17 g~) converted to FP64,
 * [18][ny][nx], into / from device memory. */
int dugks2p_get_populations(dugks2p *h, double *dst);
int dugks2p_set_populations(dugks2p *h, const double *src);

/* Raw state snapshot for checkpoint / restart: dugks2p_state_bytes() bytes
 * of device memory; restoring a snapshot reproduces the run bit for bit. */
size_t dugks2p_state_bytes(const dugks2p *h);
int dugks2p_get_state(dugks2p *h, void *dst);
int dugks2p_set_state(dugks2p *h, const void *src);

/* Time step actually used, step counter, and the DUGKS2P_KERNEL_* value
 * the handle runs (AUTO resolved). */
double dugks2p_dt(const dugks2p *h);
int64_t dugks2p_step_count(const dugks2p *h);
int dugks2p_kernel(const dugks2p *h);
/* DUGKS2P_TILE_* shape the handle's fused kernel uses (AUTO resolved;
 * DUGKS2P_TILE_UPWIND for UPWIND reconstruction; the staged form reports
 * DUGKS2P_TILE_SQUARE). */
int dugks2p_tile(const dugks2p *h);

/* Measurement aid.  While enabled, each step's tile kernel (the fused
 * form's Steps 2-6 kernel) is launched with a pair of HIP events that the
 * launch itself sets to the kernel's start and end on the handle's stream
 * (no marker packets between launches).  dugks2p_profile(h, 1)
 * enables and clears the record, (h, 0) disables it.  dugks2p_profile_read
 * synchronises the stream, writes the summed kernel time in milliseconds
 * (host *ms) and the number of timed launches (host *launches; 0 for the
 * staged form, which has no tile kernel), and clears the record. */
int dugks2p_profile(dugks2p *h, int enable);
int dugks2p_profile_read(dugks2p *h, double *ms, int64_t *launches);

/* Release the handle and its device memory (NULL is accepted). */
int dugks2p_destroy(dugks2p *h);

const char *dugks2p_last_error(void);

/* ---- Batched form ------------------------------------------------------
 * n independent simulations of arbitrary, uneven sizes advanced together:
 * each time step is two launches over the concatenated work of all
 * instances (a flattened list of (instance, cell block) and (instance,
 * tile) entries; one more pass forms the population sums after creation),
 * and runs of steps are captured once into HIP graphs and replayed.  Each instance evolves exactly as a single handle with the
 * same parameters would (bit for bit).  All instances must share the
 * precision and the reconstruction (else DUGKS2P_EUNSUPPORTED); one tile
 * shape serves the whole batch
 * (dugks2p_batch_tile; DUGKS2P_TILE_UPWIND for UPWIND reconstruction).
 *   params[n]: per-instance parameters (workspace fields ignored);
 *   phi0[n], ux0[n], uy0[n], p0[n]: device FP64 initial fields, each
 *   [ny_i][nx_i] for instance i.  The batch owns one device allocation. */
typedef struct dugks2p_batch dugks2p_batch;
int dugks2p_batch_create(int32_t n, const dugks2p_params *params, const double *const *phi0,
                         const double *const *ux0, const double *const *uy0,
                         const double *const *p0, void *hip_stream, dugks2p_batch **out);
int dugks2p_batch_step(dugks2p_batch *b, int64_t nsteps);
/* Per-instance access, same contracts as the single-handle calls. */
int dugks2p_batch_moments(dugks2p_batch *b, int32_t i, double *phi, double *rho, double *ux,
                          double *uy, double *p);
int dugks2p_batch_monitors(dugks2p_batch *b, int32_t i, double out[6]);
int dugks2p_batch_get_populations(dugks2p_batch *b, int32_t i, double *dst);
int64_t dugks2p_batch_cells(const dugks2p_batch *b);
/* Tile shape of the batched tile kernel: DUGKS2P_TILE_UPWIND for UPWIND
 * reconstruction; else the shape requested by every instance when they
 * agree on one, else (AUTO) the fastest shape found by timing the batch's
 * own step at creation. */
int dugks2p_batch_tile(const dugks2p_batch *b);
int dugks2p_batch_destroy(dugks2p_batch *b);


/* ---- Adjoint form ------------------------------------------------------
 * Reverse-mode derivative (vector-Jacobian product) of a rollout of the
 * FP64 scheme: Step 1 (initialisation from phi0, eq. auxf) followed by
 * time steps (Steps 2-7 of Sec. 2.2), each step differentiated exactly as
 * the forward computes it (CENTRAL reconstruction, phi_clamp off).  For a
 * scalar J of the final populations, with lam = dJ/d(populations) given,
 * the calls return dJ/d(phi0) and dJ/d(kappa, gx, gy) (kappa at fixed
 * beta; gx, gy of the body force).  The caller keeps checkpoints of the
 * forward populations (dugks2p_get_populations) every m <= max_segment
 * steps and walks the segments backwards; within a segment the library
 * recomputes the steps from the checkpoint and keeps their intermediates
 * (a tape of 52 FP64 values per cell and step) in its workspace.
 * Population-shaped arrays are device FP64 [18][ny][nx]; param_grad is
 * device FP64 [3] = (kappa, gx, gy) and is accumulated into (+=).  The
 * reductions are deterministic; results do not depend on scheduling. */
typedef struct dugks2p_adj dugks2p_adj;

/* Device bytes the adjoint needs for these parameters and segment length
 * (0 if invalid: the adjoint needs precision FP64, CENTRAL, phi_clamp 0,
 * 1 <= max_segment <= 100000). */
size_t dugks2p_adjoint_workspace_bytes(const dugks2p_params *params, int32_t max_segment);

/* New adjoint object (params.workspace, if given, must hold
 * dugks2p_adjoint_workspace_bytes bytes, 256-byte aligned).  Valid forward
 * parameters outside the adjoint's scope (FP32 state, UPWIND, phi_clamp)
 * return DUGKS2P_EUNSUPPORTED; invalid ones DUGKS2P_EINVAL. */
int dugks2p_adjoint_create(const dugks2p_params *params, int32_t max_segment, void *hip_stream,
                           dugks2p_adj **out);

/* One segment backwards: pops0 = populations at the segment start,
 * 0 <= nsteps <= max_segment steps, lam_end = adjoint of the populations
 * after them; writes lam_begin = adjoint of pops0 (lam_begin may equal
 * lam_end) and adds the segment's kappa / gx / gy partials to param_grad. */
int dugks2p_adjoint_segment(dugks2p_adj *a, const double *pops0, int32_t nsteps,
                            const double *lam_end, double *lam_begin, double *param_grad);

/* Adjoint of Step 1: lam0 = adjoint of the initial populations; phi0, ux0,
 * uy0, p0 as given to dugks2p_create ([ny][nx]); writes phi0_grad
 * ([ny][nx]) and adds the kappa / gx / gy partials to param_grad. */
int dugks2p_adjoint_initial(dugks2p_adj *a, const double *phi0, const double *ux0,
                            const double *uy0, const double *p0, const double *lam0,
                            double *phi0_grad, double *param_grad);

int dugks2p_adjoint_destroy(dugks2p_adj *a);

#ifdef __cplusplus
}
#endif
#endif
