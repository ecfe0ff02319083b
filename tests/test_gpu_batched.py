"""Batched form on an MI355X: every instance of a batch evolves bit for bit
as a single handle with the same parameters (including step counts that are
not a multiple of the graph length)."""
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


def _cases():
    return [W.bubble_case(32, 64, eo=20.0, mo=1e-3), W.drop_case(n=40, radius=10.0),
            W.rt_case(30, ny=70, amp_frac=0.2), W.bubble_case(48, 80, eo=60.0, mo=1e-4),
            W.poiseuille_case(nx=4, ny=32)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_instances_bitwise_equal_single(D, prec):
    """Batch instances evolve bit for bit as single handles across graph
    boundaries.  At these sizes a single handle keeps tilde+ in the output
    buffer and the batch kernel keeps it in LDS, so this also holds the two
    forms of the tile kernel to each other."""
    p = D.FP64 if prec == "fp64" else D.FP32_STATE
    cases = _cases()
    b = D.BatchSimulation(cases, precision=p)
    assert b.cells == sum(c.nx * c.ny for c in cases)
    b.step(13)   # one 8-step graph + 5 single steps
    b.step(19)   # graphs from the other buffer parity
    for i, c in enumerate(cases):
        print("batch", prec, i, c.name, flush=True)
        s = D.Simulation.from_case(c, precision=p, kernel=D.KERNEL_FUSED)
        s.step(32)
        assert np.array_equal(b.populations(i).cpu().numpy(), s.populations().cpu().numpy()), i
        assert b.monitors(i)[5] == 32


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_upwind_batch_instances_bitwise_equal_single(D, prec):
    """A batch of UPWIND instances (two-ring tiles) evolves bit for bit as
    single handles, across graph boundaries (tilde+ in LDS against the
    single handles' output buffer)."""
    p = D.FP64 if prec == "fp64" else D.FP32_STATE
    cases = _cases()
    for c in cases:
        c.params["recon"] = D.RECON_UPWIND
    b = D.BatchSimulation(cases, precision=p)
    assert b.tile == D.TILE_UPWIND
    b.step(13)
    b.step(19)
    for i, c in enumerate(cases):
        print("upwind batch", prec, i, c.name, flush=True)
        s = D.Simulation.from_case(c, precision=p, kernel=D.KERNEL_FUSED)
        assert s.tile == D.TILE_UPWIND
        s.step(32)
        assert np.array_equal(b.populations(i).cpu().numpy(), s.populations().cpu().numpy()), i


def test_batch_rejects_mixed_reconstruction(D):
    c = W.drop_case(n=16, radius=4.0)
    c2 = W.drop_case(n=16, radius=4.0, recon=1)
    with pytest.raises(D.DugksError) as e:
        D.BatchSimulation([c, c2])
    assert e.value.code == D.EUNSUPPORTED


def test_batch_rejects_mixed_precision(D):
    c = W.drop_case(n=16, radius=4.0)
    c2 = W.drop_case(n=16, radius=4.0)
    c2.params = dict(c2.params, precision=1)
    with pytest.raises(D.DugksError) as e:
        D.BatchSimulation([c, c2])
    assert e.value.code == D.EUNSUPPORTED


@pytest.mark.parametrize("tile", [0, 2, 3], ids=["tuned", "wide", "tall"])
def test_batch_tile_shapes_bitwise_equal_single(D, tile):
    """A batch run with a fixed or a tuned tile shape matches single handles
    (square tiles) bit for bit."""
    cases = _cases()[:3]
    for c in cases:
        c.params["tile"] = tile
    b = D.BatchSimulation(cases, precision=D.FP32_STATE)
    if tile:
        assert b.tile == tile
    else:
        assert b.tile in (D.TILE_SQUARE, D.TILE_WIDE, D.TILE_TALL)
    b.step(11)
    for i, c in enumerate(cases):
        print("batch tile", tile, i, c.name, flush=True)
        c.params["tile"] = D.TILE_SQUARE
        s = D.Simulation.from_case(c, precision=D.FP32_STATE, kernel=D.KERNEL_FUSED)
        s.step(11)
        assert np.array_equal(b.populations(i).cpu().numpy(), s.populations().cpu().numpy()), i
