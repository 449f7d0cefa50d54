"""The oracle against its frozen golden outputs, and the input generators'
reproducibility and shapes."""
import numpy as np
import pytest

from paper_2110_13368_amd import workloads as W
from tests.golden import make_golden as G


@pytest.mark.parametrize("name", list(G.CASES))
def test_oracle_matches_golden(name):
    import os
    path = os.path.join(os.path.dirname(G.__file__), name + ".txt")
    stored = np.loadtxt(path)
    got = G.run(name).ravel()
    assert stored.shape == got.shape
    assert np.max(np.abs(got - stored)) <= 1e-14 * np.max(np.abs(stored))


def test_generators_are_reproducible():
    a = W.single_large(scale=0.1)
    b = W.single_large(scale=0.1)
    sa, sb = a.sims[0], b.sims[0]
    assert np.array_equal(sa.rho0, sb.rho0)
    assert np.array_equal(sa.cells.pos, sb.cells.pos)
    assert np.array_equal(sa.D, sb.D)


def test_named_config_shapes():
    p = W.plain_fp64()
    s = p.sims[0]
    assert s.shape == (50, 50, 50) and s.n_sub == 1 and s.cells.n == 1000
    assert np.all(s.bc_kind == W.DIRICHLET) and np.all(s.bc_value == 38.0)
    assert np.all(s.cells.S == 0) and np.all(s.cells.U == 10) and np.all(s.cells.V == 2494)
    b = W.batched(n_sims=6)
    for sim in b.sims:
        assert all(32 <= n <= 128 for n in sim.shape)
        assert 1000 <= sim.cells.n <= 20000 and sim.n_sub == 2
        assert sim.rho0.dtype == np.float32
    small = W.single_large(scale=0.1)
    s = small.sims[0]
    assert s.shape == (20, 20, 20) and s.n_sub == 4
    lo, hi = np.array(s.lo), np.array(s.lo) + np.array(s.shape) * np.array(s.h)
    assert np.all((s.cells.pos >= lo) & (s.cells.pos < hi))
    assert np.all((s.D >= 1e3) & (s.D <= 1e5)) and np.all((s.lam >= 1e-3) & (s.lam <= 1.0))


def test_planar_config_is_two_dimensional():
    p = W.planar(n_sims=3)
    assert len(p.sims) == 3 and p.voxel_substrates == 3 * 512 * 512 * 4
    for sim in p.sims:
        assert sim.shape == (512, 512, 1) and sim.n_sub == 4 and sim.cells.n == 10000
        assert np.all(sim.bc_kind == 0)
        lo, hi = np.array(sim.lo), np.array(sim.lo) + np.array(sim.shape) * np.array(sim.h)
        assert np.all((sim.cells.pos >= lo) & (sim.cells.pos < hi))
        # a disc: Gaussian in x and y about the centre, uniform through the thickness
        c = 0.5 * (lo + hi)
        assert abs(np.std(sim.cells.pos[:, 0] - c[0]) - 800.0) < 40.0
        assert abs(np.mean(sim.cells.pos[:, 2] - c[2])) < 0.2
    q = W.planar(n_sims=3)
    assert np.array_equal(p.sims[2].cells.pos, q.sims[2].cells.pos)
    assert not np.array_equal(p.sims[0].cells.pos, p.sims[1].cells.pos)
