"""The oracle's complex-step build, and the adjoint against it.

The complex-step build runs the oracle's own source in complex arithmetic
(phi0 + i h dphi0, kappa + i h dkappa, g + i h dg, h = 1e-30).  Its imaginary
part over h is the directional derivative of the FP64 scheme to rounding:
there is no difference quotient, so no truncation error and no cancellation.

Pins of the build itself: its real part is the real oracle bit for bit, and
its derivative agrees with central differences of the real oracle to the
differences' own accuracy (about 1e-9 here).

With it the adjoint is checked through the dot-product identity
<lam, J d> = <J^T lam, d> to machine precision (1e-13 of the sum of the
terms' magnitudes), where J is the Jacobian of the final populations with
respect to (phi0, kappa, gx, gy).  A dropped term, a sign or a transposed
stencil weight anywhere in the adjoint is an O(1) relative error there.
"""
import dataclasses

import numpy as np
import pytest

from tests import _emu
from tests.test_adjoint_cpu import CASES


def _pops(oracle_mod, case, steps, **over):
    o = oracle_mod.Oracle.from_case(case, **over)
    o.step(steps)
    return o.pops()


@pytest.mark.parametrize("case,steps", [(CASES[0][0], 3), (CASES[3][0], 5), (CASES[4][0], 4)],
                         ids=["drop16", "bubble16x24", "rt7x13"])
def test_complex_step_build_pins(oracle_mod, case, steps):
    rng = np.random.default_rng(17)
    d = rng.standard_normal((case.ny, case.nx))
    re, jv = oracle_mod.complex_step_jvp(case, steps, d)
    assert np.array_equal(re, _pops(oracle_mod, case, steps))
    eps = 1e-6
    fd = (_pops(oracle_mod, dataclasses.replace(case, phi0=case.phi0 + eps * d), steps)
          - _pops(oracle_mod, dataclasses.replace(case, phi0=case.phi0 - eps * d), steps)) / (2 * eps)
    assert np.abs(jv - fd).max() <= 1e-8 * np.abs(jv).max()
    for k, name in enumerate(("kappa", "gx", "gy")):
        dp = np.zeros(3)
        dp[k] = 1.0
        re, jp = oracle_mod.complex_step_jvp(case, steps, None, *dp)
        assert np.array_equal(re, _pops(oracle_mod, case, steps))
        v = case.params[name]
        fd = (_pops(oracle_mod, case, steps, **{name: v + eps})
              - _pops(oracle_mod, case, steps, **{name: v - eps})) / (2 * eps)
        assert np.abs(jp - fd).max() <= 1e-7 * np.abs(jp).max(), name


def test_complex_step_is_linear_in_direction(oracle_mod):
    """The derivative is linear in the direction, and a zero direction gives
    exactly zero (no imaginary part ever appears)."""
    case = CASES[1][0]
    rng = np.random.default_rng(23)
    d1, d2 = rng.standard_normal((2, case.ny, case.nx))
    _, a = oracle_mod.complex_step_jvp(case, 5, d1, 0.3)
    _, b = oracle_mod.complex_step_jvp(case, 5, d2, 0.0, -0.7)
    _, c = oracle_mod.complex_step_jvp(case, 5, 2.0 * d1 - d2, 0.6, 0.7)
    assert np.allclose(c, 2.0 * a - b, rtol=0, atol=1e-13 * np.abs(c).max())
    _, z = oracle_mod.complex_step_jvp(case, 5)
    assert not z.any()


@pytest.mark.parametrize("case,steps,mseg", CASES, ids=[c[0].name for c in CASES])
def test_adjoint_dot_product_exact(oracle_mod, case, steps, mseg):
    rng = np.random.default_rng(21)
    lam = rng.standard_normal((18, case.ny, case.nx))
    _, g0, g3 = _emu.adjoint(case, steps, mseg, lam)
    d = rng.standard_normal((case.ny, case.nx))
    dp = rng.standard_normal(3)
    _, jv = oracle_mod.complex_step_jvp(case, steps, d, *dp)
    lhs = float(np.sum(lam * jv))
    rhs = float(np.sum(g0 * d)) + float(g3 @ dp)
    assert abs(lhs - rhs) <= 1e-13 * float(np.sum(np.abs(lam * jv))), (lhs, rhs)
    # each parameter on its own
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        _, jk = oracle_mod.complex_step_jvp(case, steps, None, *e)
        lk = float(np.sum(lam * jk))
        assert abs(lk - g3[k]) <= 1e-13 * float(np.sum(np.abs(lam * jk))) + 1e-300, (k, lk, g3[k])


def test_adjoint_dot_product_longer_rollout(oracle_mod):
    """Many segments and a few hundred steps on a drop: the identity still
    holds to rounding (the adjoint is of the discrete scheme exactly)."""
    from paper_1802_02868_amd import workloads as W
    case = W.drop_case(24, radius=7.0, width=3.0, noise=1e-3)
    case.params.update(gx=2e-5, gy=-1e-5)
    steps, mseg = 200, 50
    rng = np.random.default_rng(29)
    lam = rng.standard_normal((18, case.ny, case.nx))
    _, g0, g3 = _emu.adjoint(case, steps, mseg, lam)
    d = rng.standard_normal((case.ny, case.nx))
    dp = rng.standard_normal(3)
    _, jv = oracle_mod.complex_step_jvp(case, steps, d, *dp)
    lhs = float(np.sum(lam * jv))
    rhs = float(np.sum(g0 * d)) + float(g3 @ dp)
    assert abs(lhs - rhs) <= 1e-12 * float(np.sum(np.abs(lam * jv))), (lhs, rhs)


def _tile_edge_cases():
    from paper_1802_02868_amd import workloads as W
    out = []
    for case in [W.bubble_case(14, 28, 30.0, 1e-3), W.bubble_case(15, 29, 30.0, 1e-3),
                 W.drop_case(14, radius=4.0), W.drop_case(15, radius=4.0), W.rt_case(28, 42)]:
        case.params.update(phi_clamp=0, gx=1e-5)
        out.append(case)
    return out


@pytest.mark.parametrize("case", _tile_edge_cases(), ids=lambda c: c.name)
def test_adjoint_dot_product_tile_edges(oracle_mod, case):
    """Grids of exactly one or two 14 x 14 tiles, one cell over, walls on one
    or both axes: every face record is written by exactly one tile (a
    missing one would read the host build's NaN-poisoned workspace)."""
    rng = np.random.default_rng(3)
    lam = rng.standard_normal((18, case.ny, case.nx))
    _, g0, g3 = _emu.adjoint(case, 4, 3, lam)
    d = rng.standard_normal((case.ny, case.nx))
    dp = rng.standard_normal(3)
    _, jv = oracle_mod.complex_step_jvp(case, 4, d, *dp)
    lhs = float(np.sum(lam * jv))
    rhs = float(np.sum(g0 * d)) + float(g3 @ dp)
    assert abs(lhs - rhs) <= 1e-13 * float(np.sum(np.abs(lam * jv))), (lhs, rhs)

