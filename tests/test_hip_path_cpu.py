"""CPU checks of the HIP path: the C-ABI library loads and exports every
declared entry point, host-side validation, and the kernel logic (host
build of the same functors and stage sequences) against the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1802_02868_amd import workloads as W
from tests import _emu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "dugks2p.h")).read()
    return sorted(set(re.findall(r"\b(dugks2p_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1802_02868_amd import dugks2p as D
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(D.lib, n), n
    assert set(D.EXPORTED) <= set(names)


def test_create_rejects_small_or_misaligned_workspace():
    """dugks2p_create checks a caller's workspace before it touches the GPU:
    fewer bytes than dugks2p_workspace_bytes() is ENOMEM, an address that is
    not 256-byte aligned is EINVAL.  The device pointers passed here are
    placeholders that these checks never dereference."""
    import ctypes
    from paper_1802_02868_amd import dugks2p as D
    from paper_1802_02868_amd.dugks2p_params import make_params
    c = W.drop_case(n=16, radius=4.0)
    P = make_params(c.params, c.x_faces, c.y_faces, D.FP64, D.KERNEL_AUTO)
    nb = int(D.lib.dugks2p_workspace_bytes(ctypes.byref(P)))
    assert nb > 0
    fake = ctypes.c_void_p(1 << 20)
    h = ctypes.c_void_p()
    for addr, size, code in [(1 << 20, nb - 1, D.ENOMEM), ((1 << 20) + 8, nb, D.EINVAL)]:
        P.workspace = addr
        P.workspace_bytes = size
        rc = D.lib.dugks2p_create(ctypes.byref(P), fake, fake, fake, fake, None, ctypes.byref(h))
        assert rc == code, (rc, D.lib.dugks2p_last_error())
        assert not h.value


def test_adjoint_create_scope_errors():
    """dugks2p_adjoint_create before any GPU work: valid forward parameters
    outside the adjoint's scope (FP32 state, UPWIND, phi_clamp) are
    EUNSUPPORTED, an invalid segment length is EINVAL."""
    import ctypes
    from paper_1802_02868_amd import dugks2p as D
    from paper_1802_02868_amd.dugks2p_params import make_params
    c = W.drop_case(n=16, radius=4.0)
    h = ctypes.c_void_p()
    for over, mseg, code in [(dict(precision=D.FP32_STATE), 4, D.EUNSUPPORTED),
                             (dict(recon=D.RECON_UPWIND), 4, D.EUNSUPPORTED),
                             (dict(phi_clamp=1), 4, D.EUNSUPPORTED),
                             ({}, 0, D.EINVAL), (dict(tau_g=-1.0), 4, D.EINVAL)]:
        p = dict(c.params, **over)
        P = make_params(p, c.x_faces, c.y_faces, p.get("precision", D.FP64), D.KERNEL_STAGED)
        rc = D.lib.dugks2p_adjoint_create(ctypes.byref(P), mseg, None, ctypes.byref(h))
        assert rc == code, (over, mseg, rc, D.lib.dugks2p_last_error())
        assert not h.value


def test_workspace_query_validates_parameters():
    from paper_1802_02868_amd import dugks2p as D
    c = W.drop_case(n=16, radius=4.0)
    nb = D.workspace_bytes(c.params, c.x_faces, c.y_faces, kernel=D.KERNEL_STAGED)
    assert nb > 18 * 2 * 16 * 16 * 8
    for bad in (dict(tau_g=0.0), dict(phi_a=0.0), dict(nx=0), dict(bc_x=7), dict(recon=3),
                dict(rho_b=-1.0), dict(dt=0.0, cfl=0.0), dict(tau_f=0.0, nu_a=0.0)):
        p = dict(c.params)
        p.update(bad)
        assert D.workspace_bytes(p, c.x_faces, c.y_faces, kernel=D.KERNEL_STAGED) == 0, bad
    xf = c.x_faces.copy()
    xf[3] = xf[2]
    assert D.workspace_bytes(c.params, xf, c.y_faces, kernel=D.KERNEL_STAGED) == 0


def _upwind(case):
    case.params["recon"] = 1
    return case


CASES = {
    "drop": (lambda: W.drop_case(n=32, radius=8.0), 20),
    "rt_walls": (lambda: W.rt_case(16, ny=64, amp_frac=0.2), 20),
    "poiseuille_stretched": (lambda: W.poiseuille_case(nx=4, ny=32), 20),
    "bubble_four_walls": (lambda: W.bubble_case(32, 48, eo=20.0, mo=1e-3), 20),
    "upwind": (lambda: W.drop_case(n=16, radius=5.0, recon=1), 10),
    "upwind_walls": (lambda: W.rt_case(16, ny=32, amp_frac=0.2, recon=1), 10),
    # tensor meshes stretched on both axes: walls in x, in y, on both
    "tensor_walls_x": (lambda: W.tensor_drop_case(), 20),
    "tensor_walls_y": (lambda: W.tensor_drop_case(bc_x=0, bc_y=1, gy=-1e-5), 20),
    "tensor_walls_xy_upwind": (lambda: _upwind(W.tensor_drop_case(bc_x=1, bc_y=1, gx=2e-5)), 10),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_staged_kernel_logic_bitwise_equal_to_oracle(oracle_mod, name):
    make, steps = CASES[name]
    case = make()
    pops, mac = _emu.run(case, steps, kernel=1)
    o = oracle_mod.Oracle.from_case(case)
    o.step(steps)
    assert np.array_equal(pops, o.pops())
    m = o.moments()
    for k, f in enumerate(("phi", "rho", "ux", "uy", "p")):
        assert np.array_equal(mac[k], m[f]), f


FUSED_CASES = {
    "drop": (lambda: W.drop_case(n=32, radius=8.0), 10),
    "rt_walls_ragged": (lambda: W.rt_case(30, ny=50, amp_frac=0.2), 10),
    "poiseuille_stretched": (lambda: W.poiseuille_case(nx=4, ny=32), 10),
    "bubble_four_walls": (lambda: W.bubble_case(32, 48, eo=20.0, mo=1e-3), 10),
    "single_cell": (lambda: W.drop_case(n=1, radius=0.3, noise=1e-3), 3),
    "tile_plus_one": (lambda: W.drop_case(n=15, radius=4.0), 5),
    "tensor_walls_x": (lambda: W.tensor_drop_case(), 10),
    "tensor_walls_y": (lambda: W.tensor_drop_case(bc_x=0, bc_y=1, gy=-1e-5), 10),
    "tensor_strong_stretch": (lambda: W.tensor_drop_case(30, 46, 2.5, 0.5, bc_y=1, gx=2e-5), 10),
}


@pytest.mark.parametrize("tilde", ["out", "lds"])
@pytest.mark.parametrize("name", sorted(FUSED_CASES))
def test_fused_kernel_logic_bitwise_equal_to_oracle(oracle_mod, name, tilde):
    """Host run of the fused tile kernel (phases with barrier semantics, LDS
    poisoned with NaN) against the oracle, with tilde+ kept in the output
    buffer or in LDS."""
    make, steps = FUSED_CASES[name]
    case = make()
    pops, mac = _emu.run(case, steps, kernel=2, tilde=tilde)
    o = oracle_mod.Oracle.from_case(case)
    o.step(steps)
    assert np.array_equal(pops, o.pops())


UPWIND_FUSED_CASES = {
    "drop": (lambda: W.drop_case(n=16, radius=5.0, recon=1), 10),
    "rt_walls_ragged": (lambda: W.rt_case(30, ny=50, amp_frac=0.2, recon=1), 10),
    "bubble_four_walls": (lambda: W.bubble_case(32, 48, eo=20.0, mo=1e-3, recon=1), 10),
    "tile_plus_one": (lambda: W.drop_case(n=13, radius=4.0, recon=1), 5),
    "single_cell": (lambda: W.drop_case(n=1, radius=0.3, noise=1e-3, recon=1), 3),
    "two_cells": (lambda: W.drop_case(n=2, radius=0.7, noise=1e-3, recon=1), 3),
    "tensor_walls_xy": (lambda: _upwind(W.tensor_drop_case(bc_x=1, bc_y=1, gx=2e-5)), 10),
    "tensor_walls_y": (lambda: _upwind(W.tensor_drop_case(bc_x=0, bc_y=1, gy=-1e-5)), 10),
}


@pytest.mark.parametrize("tilde", ["out", "lds"])
@pytest.mark.parametrize("name", sorted(UPWIND_FUSED_CASES))
def test_fused_upwind_kernel_logic_bitwise_equal_to_oracle(oracle_mod, name, tilde):
    """UPWIND reconstruction on the fused kernel's two-ring tiles (12 x 12
    cells, bar+ two cells beyond the tile): host run of the phases against
    the oracle, bit for bit, with tilde+ in the output buffer or in LDS."""
    make, steps = UPWIND_FUSED_CASES[name]
    case = make()
    pops, mac = _emu.run(case, steps, kernel=2, tilde=tilde)
    o = oracle_mod.Oracle.from_case(case)
    o.step(steps)
    assert np.array_equal(pops, o.pops())
    m = o.moments()
    for k, f in enumerate(("phi", "rho", "ux", "uy", "p")):
        assert np.array_equal(mac[k], m[f]), f


@pytest.mark.parametrize("tile", [2, 3], ids=["wide30x6", "tall6x30"])
@pytest.mark.parametrize("name", ["drop", "rt_walls_ragged", "bubble_four_walls",
                                  "single_cell", "tile_plus_one"])
def test_fused_tile_shapes_bitwise_equal_to_oracle(oracle_mod, name, tile):
    """The wide (30 x 6) and tall (6 x 30) tile shapes give the oracle's
    results bit for bit, like the square one (ragged edges, walls, periodic
    wrap inside one tile)."""
    make, steps = FUSED_CASES[name]
    case = make()
    case.params["tile"] = tile
    pops, _ = _emu.run(case, steps, kernel=2)
    o = oracle_mod.Oracle.from_case(case)
    o.step(steps)
    assert np.array_equal(pops, o.pops())


def test_general_lattice_speed_kernel_logic(oracle_mod):
    """RT != 1/3 (c != 1) runs the general-direction code of both kernels."""
    case = W.drop_case(n=20, radius=5.0)
    case.params["rt"] = 0.3
    case.params["c_max"] = 0.0
    case.params["cfl"] = 0.4
    o = oracle_mod.Oracle.from_case(case)
    o.step(8)
    for kernel in (1, 2):
        pops, _ = _emu.run(case, 8, kernel=kernel)
        assert np.array_equal(pops, o.pops()), kernel
    # the same with UPWIND reconstruction (the two-ring tiles' general path)
    case.params["recon"] = 1
    o = oracle_mod.Oracle.from_case(case)
    o.step(8)
    for kernel in (1, 2):
        pops, _ = _emu.run(case, 8, kernel=kernel)
        assert np.array_equal(pops, o.pops()), ("upwind", kernel)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_state"])
def test_tilde_in_lds_or_output_buffer_identical(prec):
    """Where the square-tile kernel keeps tilde+ between Step 2 and the update
    changes nothing: for the FP32 state the output buffer's store and load
    round it exactly as the encoding's round trip does in LDS."""
    for case, steps in [(W.rt_case(30, ny=50, amp_frac=0.2), 40),
                        (W.drop_case(n=33, radius=8.0, tau_f=0.5), 30),
                        (W.rt_case(26, ny=30, amp_frac=0.2, recon=1), 30)]:
        case.params["precision"] = prec
        a, ma = _emu.run(case, steps, kernel=2, tilde="out")
        b, mb = _emu.run(case, steps, kernel=2, tilde="lds")
        assert np.array_equal(a, b) and np.array_equal(ma, mb), case.name


def test_fp32_state_kernel_logic_within_tolerance(oracle_mod):
    """FP32 state (f~ as floats, phi as FP64, g~ as float deviations) keeps
    phi and u within 1e-4 of the FP64 oracle."""
    for case, steps in [(W.rt_case(32, ny=128, amp_frac=0.2), 300),
                        (W.drop_case(n=32, radius=8.0), 400),
                        (W.rt_case(32, ny=128, amp_frac=0.2, recon=1), 300)]:
        case.params["precision"] = 1
        pops, mac = _emu.run(case, steps, kernel=2)
        o = oracle_mod.Oracle.from_case(case)
        o.step(steps)
        m = o.moments()
        for k, f in ((0, "phi"), (2, "ux"), (3, "uy")):
            err = np.abs(mac[k] - m[f]).max() / np.abs(m[f]).max()
            assert err < 1e-4, (case.name, f, err)


@pytest.mark.parametrize("name", sorted(W.PAPER_CASES))
def test_paper_parameter_sets_kernel_logic(oracle_mod, name):
    """The paper's own setups (Secs. 3.1-3.4 as printed there) through the
    fused kernel's host build: the oracle's results bit for bit."""
    case = W.PAPER_CASES[name]()
    pops, _ = _emu.run(case, 2, kernel=2)
    o = oracle_mod.Oracle.from_case(case)
    o.step(2)
    assert np.array_equal(pops, o.pops())


def test_make_params_explicit_arguments_win():
    """An explicit precision or kernel reaches the struct; a dictionary entry
    is used only when the argument is left out, and a disagreement between
    the two is an error rather than a silent switch."""
    from paper_1802_02868_amd import dugks2p_params as DP
    c = W.drop_case(n=8, radius=2.0)
    P = DP.make_params(c.params, c.x_faces, c.y_faces, DP.FP32_STATE, DP.KERNEL_STAGED)
    assert (P.precision, P.kernel) == (DP.FP32_STATE, DP.KERNEL_STAGED)
    P = DP.make_params(c.params, c.x_faces, c.y_faces)
    assert (P.precision, P.kernel) == (DP.FP64, DP.KERNEL_AUTO)
    p = dict(c.params, precision=DP.FP32_STATE, kernel=DP.KERNEL_FUSED)
    P = DP.make_params(p, c.x_faces, c.y_faces)
    assert (P.precision, P.kernel) == (DP.FP32_STATE, DP.KERNEL_FUSED)
    P = DP.make_params(p, c.x_faces, c.y_faces, DP.FP32_STATE, DP.KERNEL_FUSED)
    assert (P.precision, P.kernel) == (DP.FP32_STATE, DP.KERNEL_FUSED)
    with pytest.raises(ValueError):
        DP.make_params(p, c.x_faces, c.y_faces, precision=DP.FP64)
    with pytest.raises(ValueError):
        DP.make_params(p, c.x_faces, c.y_faces, kernel=DP.KERNEL_STAGED)
