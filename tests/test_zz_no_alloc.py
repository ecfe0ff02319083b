"""dugks2p_monitors_noalloc: the monitors written to caller device memory
with the partials in the library's static scratch array (no allocation, no
synchronisation), against dugks2p_monitors on the same handle.

The partial and final reductions are the same kernels in the same order, so
the sums and the non-finite count agree bit for bit; max |u| is a square
root taken on the device here and on the host there (both correctly
rounded), held to one ulp.  Two calls in a row, the second on a smaller
grid, show that the shared scratch carries nothing from one call into the
next."""
import numpy as np
import pytest

from paper_1802_02868_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_02868_amd import dugks2p
    return dugks2p


def _check(D, sim, out):
    import torch
    ref = sim.monitors()
    sim.monitors_noalloc(out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got[[0, 1, 2, 4, 5]], ref[[0, 1, 2, 4, 5]]), (got, ref)
    assert abs(got[3] - ref[3]) <= np.spacing(ref[3]), (got[3], ref[3])
    return got


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_monitors_noalloc_matches_monitors(D, prec):
    import torch
    p = D.FP64 if prec == "fp64" else D.FP32_STATE
    out = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
    big = W.rt_case(130, ny=260, amp_frac=0.1)
    print("noalloc", prec, big.name, flush=True)
    a = D.Simulation.from_case(big, precision=p)
    a.step(40)
    got_a = _check(D, a, out)
    assert got_a[3] > 0.0 and got_a[5] == 40
    small = W.drop_case(n=20, radius=5.0)
    print("noalloc", prec, small.name, flush=True)
    b = D.Simulation.from_case(small, precision=p)
    b.step(7)
    _check(D, b, out)
    # the first handle again, after the smaller one used the scratch
    a.step(3)
    _check(D, a, out)
    a.close()
    b.close()


def test_monitors_noalloc_reports_nonfinite(D):
    import torch
    case = W.drop_case(n=16, radius=4.0)
    sim = D.Simulation.from_case(case, kernel=D.KERNEL_FUSED)
    pops = sim.populations()
    pops[2, 3, 4] = float("inf")
    sim.set_populations(pops)
    out = torch.zeros(6, dtype=torch.float64, device="cuda")
    sim.monitors_noalloc(out)
    torch.cuda.synchronize()
    assert out[4].item() == 1.0
    sim.close()
