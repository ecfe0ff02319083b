"""Loader of the host build of the HIP path's kernel logic (tests only)."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emu", "dugks2p_emu.cpp")
LIB = os.path.join(HERE, "emu", "libdugks2p_emu.so")
CSRC = os.path.join(os.path.dirname(HERE), "paper_1802_02868_amd", "csrc")


def build():
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-Wall", "-Wno-unknown-pragmas",
           "-o", "%s.tmp%d" % (LIB, os.getpid()), SRC]
    subprocess.run(cmd, check=True)
    os.replace("%s.tmp%d" % (LIB, os.getpid()), LIB)
    return LIB


def _stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [SRC] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    return any(os.path.getmtime(d) > t for d in deps)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build()
        _lib = ctypes.CDLL(LIB)
    return _lib


def run(case, steps, kernel=1, tilde=None):
    """Initialise + `steps` steps in the host build; returns (pops, macros).
    tilde: "lds" or "out" forces where the square-tile kernel keeps tilde+
    (LDS, or the output buffer); None takes the library's choice by state
    size (the output buffer for every grid of these tests)."""
    from paper_1802_02868_amd.dugks2p_params import make_params  # noqa: E402
    P = make_params(case.params, case.x_faces, case.y_faces, kernel=kernel)
    dp = ctypes.POINTER(ctypes.c_double)
    pops = np.empty((18, case.ny, case.nx))
    mac = np.empty((5, case.ny, case.nx))
    fl = [np.ascontiguousarray(a, dtype=np.float64) for a in (case.phi0, case.ux0, case.uy0, case.p0)]
    old = os.environ.pop("DUGKS2P_EMU_TILDE", None)
    if tilde is not None:
        os.environ["DUGKS2P_EMU_TILDE"] = tilde
    try:
        rc = lib().emu_run(ctypes.byref(P), *[a.ctypes.data_as(dp) for a in fl],
                           ctypes.c_longlong(steps), pops.ctypes.data_as(dp),
                           mac.ctypes.data_as(dp))
    finally:
        os.environ.pop("DUGKS2P_EMU_TILDE", None)
        if old is not None:
            os.environ["DUGKS2P_EMU_TILDE"] = old
    assert rc == 0
    return pops, mac


def adjoint(case, steps, mseg, lam):
    """Rollout adjoint in the host build: returns (pops_T, phi0_grad, grad3)
    for J = <lam, pops_T>, grad3 = dJ/d(kappa, gx, gy)."""
    from paper_1802_02868_amd.dugks2p_params import make_params  # noqa: E402
    P = make_params(case.params, case.x_faces, case.y_faces, kernel=1)
    dp = ctypes.POINTER(ctypes.c_double)
    lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(18, case.ny, case.nx)
    pops = np.empty((18, case.ny, case.nx))
    g0 = np.empty((case.ny, case.nx))
    g3 = np.empty(3)
    fl = [np.ascontiguousarray(a, dtype=np.float64) for a in (case.phi0, case.ux0, case.uy0, case.p0)]
    rc = lib().emu_adjoint(ctypes.byref(P), *[a.ctypes.data_as(dp) for a in fl],
                           ctypes.c_longlong(steps), ctypes.c_int(mseg), lam.ctypes.data_as(dp),
                           pops.ctypes.data_as(dp), g0.ctypes.data_as(dp), g3.ctypes.data_as(dp))
    assert rc == 0
    return pops, g0, g3
