"""The host build of the kernel logic under AddressSanitizer and
UndefinedBehaviorSanitizer, with every LDS-window access bounds-checked
(DUGKS2P_WINDOW_CHECK aborts on an offset outside the tile's window).

The stand-alone program tests/emu/sanitize_main.cpp is compiled with g++ and
run as a child process on fused CENTRAL and UPWIND steps, FP32 state, the
staged kernels and the adjoint, including grids of one and two tiles and
ragged tiles.  A sanitizer report, a window overrun or a non-zero exit fails
the test; the outputs must also equal the plain host build bit for bit.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1802_02868_amd import workloads as W
from paper_1802_02868_amd.dugks2p_params import Params, make_params
from tests import _emu

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emu", "sanitize_main.cpp")


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("san") / "sanitize_main")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-DDUGKS2P_WINDOW_CHECK", "-Wno-unknown-pragmas", "-o", out, SRC]
    subprocess.run(cmd, check=True)
    return out


def _run(exe, tmp, case, steps, kind=0, mseg=0, kernel=2, lam=None, tilde=None):
    P = make_params(case.params, case.x_faces, case.y_faces, kernel=kernel)
    n = case.nx * case.ny
    fin, fout = str(tmp / "case.bin"), str(tmp / "out.bin")
    with open(fin, "wb") as f:
        f.write(np.array([kind, steps, mseg, ctypes.sizeof(Params)], dtype=np.int64).tobytes())
        f.write(bytes(P))
        for a in (case.x_faces, case.y_faces, case.phi0, case.ux0, case.uy0, case.p0):
            f.write(np.ascontiguousarray(a, dtype=np.float64).tobytes())
        if kind == 1:
            f.write(np.ascontiguousarray(lam, dtype=np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("DUGKS2P_EMU_TILDE", None)
    if tilde is not None:
        env["DUGKS2P_EMU_TILDE"] = tilde
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (case.name, r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "window check" not in r.stdout, r.stderr[-2000:]
    out = np.fromfile(fout, dtype=np.float64)
    if kind == 0:
        return out[:18 * n].reshape(18, case.ny, case.nx)
    return (out[:18 * n].reshape(18, case.ny, case.nx), out[18 * n:19 * n].reshape(case.ny, case.nx),
            out[19 * n:])


FORWARD = [
    ("drop13_one_tile", lambda: W.drop_case(n=13, radius=3.0), 2, 3),
    ("drop16x14_two_tiles", lambda: W.tensor_drop_case(16, 14, 1.0, 1.0), 2, 3),
    ("rt_walls_ragged", lambda: W.rt_case(30, ny=50, amp_frac=0.2), 2, 2),
    ("tensor_walls_both", lambda: W.tensor_drop_case(20, 18, 2.5, 0.5, bc_x=1, bc_y=1, gx=2e-5), 2, 2),
    ("upwind_drop13", lambda: W.drop_case(n=13, radius=3.0, recon=1), 2, 2),
    ("upwind_rt_walls", lambda: W.rt_case(26, ny=30, amp_frac=0.2, recon=1), 2, 2),
    ("staged_rt_walls", lambda: W.rt_case(20, ny=24, amp_frac=0.2), 1, 2),
    ("wide_tiles_bubble", lambda: W.bubble_case(32, 40, eo=20.0, mo=1e-3), 2, 2),
]


@pytest.mark.parametrize("tilde", ["out", "lds"])
@pytest.mark.parametrize("name,make,kernel,steps", FORWARD, ids=[f[0] for f in FORWARD])
def test_sanitized_forward(sanitized, tmp_path, name, make, kernel, steps, tilde):
    """tilde: where the square-tile kernel keeps tilde+ (output buffer or LDS)."""
    case = make()
    if name.startswith("wide"):
        case.params["tile"] = 2
    got = _run(sanitized, tmp_path, case, steps, kernel=kernel, tilde=tilde)
    ref, _ = _emu.run(case, steps, kernel=kernel, tilde=tilde)
    assert np.array_equal(got, ref), name


@pytest.mark.parametrize("tilde", ["out", "lds"])
def test_sanitized_fp32_state(sanitized, tmp_path, tilde):
    case = W.rt_case(28, ny=30, amp_frac=0.2)
    case.params["precision"] = 1
    got = _run(sanitized, tmp_path, case, 2, kernel=2, tilde=tilde)
    ref, _ = _emu.run(case, 2, kernel=2, tilde=tilde)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("make,steps,mseg", [
    (lambda: W.drop_case(n=14, radius=3.5, noise=1e-3), 3, 2),
    (lambda: W.rt_case(7, ny=13, amp_frac=0.2), 2, 2),
    (lambda: W.tensor_drop_case(18, 16, 2.0, 0.5, bc_x=1, gx=2e-5), 2, 1),
], ids=["drop14_one_tile", "rt7x13_ragged", "tensor_walls_x"])
def test_sanitized_adjoint(sanitized, tmp_path, make, steps, mseg):
    case = make()
    rng = np.random.Generator(np.random.PCG64(5))
    lam = rng.standard_normal((18, case.ny, case.nx))
    pops, g0, g3 = _run(sanitized, tmp_path, case, steps, kind=1, mseg=mseg, kernel=1, lam=lam)
    rp, rg0, rg3 = _emu.adjoint(case, steps, mseg, lam)
    assert np.array_equal(pops, rp) and np.array_equal(g0, rg0) and np.array_equal(g3, rg3)
