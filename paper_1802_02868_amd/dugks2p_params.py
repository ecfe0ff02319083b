"""ctypes mirror of dugks2p_params (include/dugks2p.h) and the constants of
the C ABI; no library is loaded here."""
from __future__ import annotations

import ctypes

import numpy as np

OK, EINVAL, ENOMEM, EHIP, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
BC_PERIODIC, BC_WALL = 0, 1
FP64, FP32_STATE = 0, 1
RECON_CENTRAL, RECON_UPWIND = 0, 1
KERNEL_AUTO, KERNEL_STAGED, KERNEL_FUSED, KERNEL_FUSED_FMA = 0, 1, 2, 3
TILE_AUTO, TILE_SQUARE, TILE_WIDE, TILE_TALL, TILE_UPWIND = 0, 1, 2, 3, 4
ABI_VERSION = 1

_DOUBLE_FIELDS = ("cfl", "c_max", "dt", "rt", "tau_g", "mobility", "tau_f", "beta", "kappa",
                  "phi_a", "phi_b", "rho_a", "rho_b", "nu_a", "nu_b", "gx", "gy", "rho_ref")
_INT_FIELDS = ("abi_version", "nx", "ny", "bc_x", "bc_y", "precision", "recon", "phi_clamp",
               "kernel", "tile")


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in _INT_FIELDS] + \
               [("x_faces", ctypes.POINTER(ctypes.c_double)),
                ("y_faces", ctypes.POINTER(ctypes.c_double))] + \
               [(n, ctypes.c_double) for n in _DOUBLE_FIELDS] + \
               [("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


def _choose(p: dict, name: str, arg, default: int) -> int:
    """An explicit argument wins; the dictionary's entry is used when the
    argument is None; the two may not disagree."""
    if arg is None:
        return int(p.get(name, default))
    if name in p and int(p[name]) != int(arg):
        raise ValueError("%s=%d conflicts with the parameter dictionary's %s=%d"
                         % (name, int(arg), name, int(p[name])))
    return int(arg)


def make_params(p: dict, x_faces, y_faces, precision=None, kernel=None):
    """Fill a Params struct from the parameter dictionary used by the
    workloads module; keeps the face arrays alive on the struct.
    `precision` and `kernel` given explicitly take effect; None takes the
    dictionary's entry (default FP64 / KERNEL_AUTO); a dictionary entry that
    disagrees with an explicit argument raises ValueError."""
    P = Params()
    P.abi_version = ABI_VERSION
    for n in _INT_FIELDS[1:]:
        if n in p:
            setattr(P, n, int(p[n]))
    P.precision = _choose(p, "precision", precision, FP64)
    P.kernel = _choose(p, "kernel", kernel, KERNEL_AUTO)
    for n in _DOUBLE_FIELDS:
        setattr(P, n, float(p[n]))
    xf = np.ascontiguousarray(x_faces, dtype=np.float64)
    yf = np.ascontiguousarray(y_faces, dtype=np.float64)
    P.x_faces = xf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    P.y_faces = yf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    P._keep = (xf, yf)
    return P


