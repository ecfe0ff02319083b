"""Python binding of the MI355X two-phase DUGKS library (include/dugks2p.h).

Argument marshalling only: every step runs in the HIP kernels of
libdugks2p.so.  torch supplies device memory (initial fields, outputs,
optional workspace) and the stream.  Importing this module fails loudly if
the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdugks2p.so")

from .dugks2p_params import (ABI_VERSION, BC_PERIODIC, BC_WALL, EHIP, EINVAL,  # noqa: F401
                             ENOMEM, ENONFINITE, EUNSUPPORTED, FP32_STATE, FP64,
                             KERNEL_AUTO, KERNEL_FUSED, KERNEL_FUSED_FMA, KERNEL_STAGED, OK,
                             RECON_CENTRAL,
                             RECON_UPWIND, TILE_AUTO, TILE_SQUARE, TILE_TALL, TILE_UPWIND,
                             TILE_WIDE,
                             Params, make_params)


class DugksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("dugks2p error %d: %s" % (code, msg))
        self.code = code


def _load():
    # torch brings its own HIP runtime; loading it first makes this library
    # bind to the same one, so that torch's device memory and streams are
    # valid handles here whatever the caller imported first
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdugks2p.so is not built (run __graft_entry__.build() or "
                          "python -m paper_1802_02868_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, P = ctypes.c_void_p, ctypes.POINTER
    d = ctypes.c_double
    L.dugks2p_workspace_bytes.restype = ctypes.c_size_t
    L.dugks2p_workspace_bytes.argtypes = [P(Params)]
    L.dugks2p_create.restype = ctypes.c_int
    L.dugks2p_create.argtypes = [P(Params), vp, vp, vp, vp, vp, P(vp)]
    L.dugks2p_step.restype = ctypes.c_int
    L.dugks2p_step.argtypes = [vp, ctypes.c_int64]
    L.dugks2p_set_checks.restype = ctypes.c_int
    L.dugks2p_set_checks.argtypes = [vp, ctypes.c_int64]
    L.dugks2p_moments.restype = ctypes.c_int
    L.dugks2p_moments.argtypes = [vp, vp, vp, vp, vp, vp]
    L.dugks2p_monitors.restype = ctypes.c_int
    L.dugks2p_monitors.argtypes = [vp, P(d)]
    L.dugks2p_monitors_noalloc.restype = ctypes.c_int
    L.dugks2p_monitors_noalloc.argtypes = [vp, vp]
    L.dugks2p_observables.restype = ctypes.c_int
    L.dugks2p_observables.argtypes = [vp, P(d)]
    L.dugks2p_laplace_pressure.restype = ctypes.c_int
    L.dugks2p_laplace_pressure.argtypes = [vp, vp]
    L.dugks2p_get_populations.restype = ctypes.c_int
    L.dugks2p_get_populations.argtypes = [vp, vp]
    L.dugks2p_set_populations.restype = ctypes.c_int
    L.dugks2p_set_populations.argtypes = [vp, vp]
    L.dugks2p_state_bytes.restype = ctypes.c_size_t
    L.dugks2p_state_bytes.argtypes = [vp]
    L.dugks2p_get_state.restype = ctypes.c_int
    L.dugks2p_get_state.argtypes = [vp, vp]
    L.dugks2p_set_state.restype = ctypes.c_int
    L.dugks2p_set_state.argtypes = [vp, vp]
    L.dugks2p_dt.restype = d
    L.dugks2p_dt.argtypes = [vp]
    L.dugks2p_step_count.restype = ctypes.c_int64
    L.dugks2p_step_count.argtypes = [vp]
    L.dugks2p_kernel.restype = ctypes.c_int
    L.dugks2p_kernel.argtypes = [vp]
    L.dugks2p_tile.restype = ctypes.c_int
    L.dugks2p_tile.argtypes = [vp]
    L.dugks2p_destroy.restype = ctypes.c_int
    L.dugks2p_destroy.argtypes = [vp]
    L.dugks2p_profile.restype = ctypes.c_int
    L.dugks2p_profile.argtypes = [vp, ctypes.c_int]
    L.dugks2p_profile_read.restype = ctypes.c_int
    L.dugks2p_profile_read.argtypes = [vp, P(d), P(ctypes.c_int64)]
    L.dugks2p_last_error.restype = ctypes.c_char_p
    L.dugks2p_last_error.argtypes = []
    PP = ctypes.POINTER(ctypes.c_void_p)
    L.dugks2p_batch_create.restype = ctypes.c_int
    L.dugks2p_batch_create.argtypes = [ctypes.c_int32, P(Params), PP, PP, PP, PP, vp, P(vp)]
    L.dugks2p_batch_step.restype = ctypes.c_int
    L.dugks2p_batch_step.argtypes = [vp, ctypes.c_int64]
    L.dugks2p_batch_moments.restype = ctypes.c_int
    L.dugks2p_batch_moments.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp]
    L.dugks2p_batch_monitors.restype = ctypes.c_int
    L.dugks2p_batch_monitors.argtypes = [vp, ctypes.c_int32, P(d)]
    L.dugks2p_batch_get_populations.restype = ctypes.c_int
    L.dugks2p_batch_get_populations.argtypes = [vp, ctypes.c_int32, vp]
    L.dugks2p_batch_cells.restype = ctypes.c_int64
    L.dugks2p_batch_cells.argtypes = [vp]
    L.dugks2p_batch_tile.restype = ctypes.c_int
    L.dugks2p_batch_tile.argtypes = [vp]
    L.dugks2p_batch_destroy.restype = ctypes.c_int
    L.dugks2p_batch_destroy.argtypes = [vp]
    L.dugks2p_adjoint_workspace_bytes.restype = ctypes.c_size_t
    L.dugks2p_adjoint_workspace_bytes.argtypes = [P(Params), ctypes.c_int32]
    L.dugks2p_adjoint_create.restype = ctypes.c_int
    L.dugks2p_adjoint_create.argtypes = [P(Params), ctypes.c_int32, vp, P(vp)]
    L.dugks2p_adjoint_segment.restype = ctypes.c_int
    L.dugks2p_adjoint_segment.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp]
    L.dugks2p_adjoint_initial.restype = ctypes.c_int
    L.dugks2p_adjoint_initial.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.dugks2p_adjoint_destroy.restype = ctypes.c_int
    L.dugks2p_adjoint_destroy.argtypes = [vp]
    return L


lib = _load()

EXPORTED = ("dugks2p_workspace_bytes", "dugks2p_create", "dugks2p_step", "dugks2p_set_checks",
            "dugks2p_moments",
            "dugks2p_monitors", "dugks2p_monitors_noalloc", "dugks2p_observables", "dugks2p_laplace_pressure",
            "dugks2p_get_populations",
            "dugks2p_set_populations",
            "dugks2p_state_bytes", "dugks2p_get_state", "dugks2p_set_state", "dugks2p_dt",
            "dugks2p_step_count", "dugks2p_kernel", "dugks2p_tile", "dugks2p_destroy",
            "dugks2p_last_error",
            "dugks2p_profile", "dugks2p_profile_read",
            "dugks2p_batch_create", "dugks2p_batch_step", "dugks2p_batch_moments",
            "dugks2p_batch_monitors", "dugks2p_batch_get_populations", "dugks2p_batch_cells",
            "dugks2p_batch_tile",
            "dugks2p_batch_destroy", "dugks2p_adjoint_workspace_bytes", "dugks2p_adjoint_create",
            "dugks2p_adjoint_segment", "dugks2p_adjoint_initial", "dugks2p_adjoint_destroy")


def _check(rc):
    if rc != OK:
        raise DugksError(rc, lib.dugks2p_last_error().decode())
    return rc


def workspace_bytes(p: dict, x_faces, y_faces, precision=None, kernel=None) -> int:
    P = make_params(p, x_faces, y_faces, precision, kernel)
    return int(lib.dugks2p_workspace_bytes(ctypes.byref(P)))


class Simulation:
    """One DUGKS simulation on the current CUDA/HIP device.

    phi0, ux0, uy0, p0: torch float64 CUDA tensors (or numpy arrays, copied to
    the device) of shape [ny, nx]."""

    def __init__(self, params: dict, x_faces, y_faces, phi0, ux0, uy0, p0, precision=None,
                 kernel=None, stream=None, torch_workspace=True):
        import torch
        self.torch = torch
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        P = make_params(params, x_faces, y_faces, precision, kernel)
        self._ws = None
        if torch_workspace:
            nb = int(lib.dugks2p_workspace_bytes(ctypes.byref(P)))
            if nb == 0:
                self._create_fail(P)
            self._ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            P.workspace = (base + 255) & ~255
            P.workspace_bytes = nb
        fields = [self._dev(a) for a in (phi0, ux0, uy0, p0)]
        h = ctypes.c_void_p()
        rc = lib.dugks2p_create(ctypes.byref(P), *[f.data_ptr() for f in fields],
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        _check(rc)
        self._h = h
        self._P = P
        self.precision = P.precision
        # keep inputs alive until the init kernels have consumed them
        self.stream.synchronize()

    def _create_fail(self, P):
        h = ctypes.c_void_p()
        z = self.torch.zeros(1, dtype=self.torch.float64, device=self.device)
        rc = lib.dugks2p_create(ctypes.byref(P), z.data_ptr(), z.data_ptr(), z.data_ptr(),
                                z.data_ptr(), None, ctypes.byref(h))
        _check(rc if rc != OK else EINVAL)

    def _dev(self, a):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        a = a.to(device=self.device, dtype=t.float64).contiguous()
        if tuple(a.shape) != (self.ny, self.nx):
            raise ValueError("field shape %s != (%d, %d)" % (tuple(a.shape), self.ny, self.nx))
        return a

    @classmethod
    def from_case(cls, case, **kw):
        return cls(case.params, case.x_faces, case.y_faces, case.phi0, case.ux0, case.uy0,
                   case.p0, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.dugks2p_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dt(self):
        return lib.dugks2p_dt(self._h)

    @property
    def kernel_kind(self):
        return lib.dugks2p_kernel(self._h)

    @property
    def nstep(self):
        return lib.dugks2p_step_count(self._h)

    @property
    def tile(self):
        """TILE_* shape the fused kernel uses (AUTO resolved)."""
        return lib.dugks2p_tile(self._h)

    def step(self, n=1):
        _check(lib.dugks2p_step(self._h, int(n)))

    def set_checks(self, every):
        """every > 0: step() counts the non-finite populations after every
        `every`-th step and after its last step (synchronising) and raises
        DugksError(ENONFINITE) at the first nonzero count; 0 disables."""
        _check(lib.dugks2p_set_checks(self._h, int(every)))

    def time_kernel(self, n):
        """Run n steps with HIP events around the tile kernel; returns
        (total kernel milliseconds, timed launches)."""
        _check(lib.dugks2p_profile(self._h, 1))
        try:
            self.step(n)
            ms, cnt = ctypes.c_double(), ctypes.c_int64()
            _check(lib.dugks2p_profile_read(self._h, ctypes.byref(ms), ctypes.byref(cnt)))
        finally:
            lib.dugks2p_profile(self._h, 0)
        return ms.value, cnt.value

    def moments(self):
        t = self.torch
        out = {k: t.empty((self.ny, self.nx), dtype=t.float64, device=self.device)
               for k in ("phi", "rho", "ux", "uy", "p")}
        _check(lib.dugks2p_moments(self._h, *[out[k].data_ptr()
                                              for k in ("phi", "rho", "ux", "uy", "p")]))
        return out

    def monitors(self, raise_nonfinite=True):
        out = (ctypes.c_double * 6)()
        rc = lib.dugks2p_monitors(self._h, out)
        if rc != OK and (raise_nonfinite or rc != ENONFINITE):
            _check(rc)
        return np.array(out[:])

    def monitors_noalloc(self, out):
        """The monitors into `out` (float64 CUDA tensor of 6 elements, the
        caller's), enqueued on the handle's stream without allocation or
        synchronisation (include/dugks2p.h)."""
        if out.dtype != self.torch.float64 or not out.is_cuda or out.numel() < 6 \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 CUDA tensor of 6 elements")
        _check(lib.dugks2p_monitors_noalloc(self._h, out.data_ptr()))
        return out

    def observables(self):
        """[droplet cells, their area, phase-A centroid x, y, mean u_x, u_y,
        highest and lowest median-level y] (include/dugks2p.h)."""
        out = (ctypes.c_double * 8)()
        _check(lib.dugks2p_observables(self._h, out))
        return np.array(out[:])

    def laplace_pressure(self):
        """The Laplace-test pressure field P [ny, nx] (include/dugks2p.h)."""
        t = self.torch
        out = t.empty((self.ny, self.nx), dtype=t.float64, device=self.device)
        _check(lib.dugks2p_laplace_pressure(self._h, out.data_ptr()))
        return out

    def populations(self):
        t = self.torch
        out = t.empty((18, self.ny, self.nx), dtype=t.float64, device=self.device)
        _check(lib.dugks2p_get_populations(self._h, out.data_ptr()))
        return out

    def set_populations(self, pops):
        pops = pops.to(device=self.device, dtype=self.torch.float64).contiguous()
        _check(lib.dugks2p_set_populations(self._h, pops.data_ptr()))
        self.stream.synchronize()

    def get_state(self):
        t = self.torch
        nb = int(lib.dugks2p_state_bytes(self._h))
        buf = t.empty(nb, dtype=t.uint8, device=self.device)
        _check(lib.dugks2p_get_state(self._h, buf.data_ptr()))
        return buf

    def set_state(self, buf):
        _check(lib.dugks2p_set_state(self._h, buf.data_ptr()))
        self.stream.synchronize()


class BatchSimulation:
    """Independent simulations of uneven sizes advanced together (batched
    launches replayed from HIP graphs).  `cases`: objects with params,
    x_faces, y_faces, phi0, ux0, uy0, p0 (see workloads.Case)."""

    def __init__(self, cases, precision=None, stream=None):
        import torch
        self.torch = torch
        self.cases = list(cases)
        self.n = len(self.cases)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (Params * self.n)()
        self._keep = []
        for i, c in enumerate(self.cases):
            P = make_params(c.params, c.x_faces, c.y_faces, precision, KERNEL_FUSED)
            self._keep.append(P._keep)
            arr[i] = P
        fields = []
        ptrs = [(ctypes.c_void_p * self.n)() for _ in range(4)]
        for i, c in enumerate(self.cases):
            for k, a in enumerate((c.phi0, c.ux0, c.uy0, c.p0)):
                t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)
                fields.append(t)
                ptrs[k][i] = t.data_ptr()
        h = ctypes.c_void_p()
        _check(lib.dugks2p_batch_create(self.n, arr, *ptrs, ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(h)))
        self._h = h
        self.stream.synchronize()
        del fields

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.dugks2p_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def cells(self):
        return int(lib.dugks2p_batch_cells(self._h))

    @property
    def tile(self):
        """TILE_* shape of the batched tile kernel (AUTO resolved)."""
        return lib.dugks2p_batch_tile(self._h)

    def step(self, n=1):
        _check(lib.dugks2p_batch_step(self._h, int(n)))

    def populations(self, i):
        c = self.cases[i]
        t = self.torch
        out = t.empty((18, c.ny, c.nx), dtype=t.float64, device=self.device)
        _check(lib.dugks2p_batch_get_populations(self._h, int(i), out.data_ptr()))
        return out

    def monitors(self, i, raise_nonfinite=True):
        out = (ctypes.c_double * 6)()
        rc = lib.dugks2p_batch_monitors(self._h, int(i), out)
        if rc != OK and (raise_nonfinite or rc != ENONFINITE):
            _check(rc)
        return np.array(out[:])


class Adjoint:
    """Reverse sweep of FP64 rollouts (include/dugks2p.h, "Adjoint form").

    Population-shaped tensors are torch float64 CUDA [18, ny, nx]; the
    parameter gradient is a float64 CUDA tensor [3] = d/d(kappa, gx, gy),
    accumulated in place."""

    def __init__(self, params: dict, x_faces, y_faces, max_segment=50, stream=None):
        import torch
        self.torch = torch
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self.max_segment = int(max_segment)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        P = make_params(params, x_faces, y_faces)
        nb = int(lib.dugks2p_adjoint_workspace_bytes(ctypes.byref(P), self.max_segment))
        self._ws = None
        if nb:
            self._ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            P.workspace = (self._ws.data_ptr() + 255) & ~255
            P.workspace_bytes = nb
        h = ctypes.c_void_p()
        _check(lib.dugks2p_adjoint_create(ctypes.byref(P), self.max_segment,
                                          ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.dugks2p_adjoint_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _pops(self, a):
        a = a.to(device=self.device, dtype=self.torch.float64).contiguous()
        if tuple(a.shape) != (18, self.ny, self.nx):
            raise ValueError("population shape %s != (18, %d, %d)" % (tuple(a.shape), self.ny,
                                                                        self.nx))
        return a

    def _field(self, a):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        a = a.to(device=self.device, dtype=t.float64).contiguous()
        if tuple(a.shape) != (self.ny, self.nx):
            raise ValueError("field shape %s != (%d, %d)" % (tuple(a.shape), self.ny, self.nx))
        return a

    def segment(self, pops0, nsteps, lam_end, param_grad, out=None):
        """Adjoint at the segment start from the adjoint after nsteps steps."""
        pops0, lam_end = self._pops(pops0), self._pops(lam_end)
        out = self.torch.empty_like(lam_end) if out is None else out
        _check(lib.dugks2p_adjoint_segment(self._h, pops0.data_ptr(), int(nsteps),
                                           lam_end.data_ptr(), out.data_ptr(),
                                           param_grad.data_ptr()))
        return out

    def initial(self, phi0, ux0, uy0, p0, lam0, param_grad):
        """Adjoint of the initialisation: returns dJ/d(phi0)."""
        f = [self._field(a) for a in (phi0, ux0, uy0, p0)]
        lam0 = self._pops(lam0)
        out = self.torch.empty((self.ny, self.nx), dtype=self.torch.float64, device=self.device)
        _check(lib.dugks2p_adjoint_initial(self._h, *[a.data_ptr() for a in f], lam0.data_ptr(),
                                           out.data_ptr(), param_grad.data_ptr()))
        return out
