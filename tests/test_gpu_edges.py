"""Edge cases against the oracle: the smallest grids (a single level, the
coarsest dense solve only), odd sizes that stop coarsening early, the
adiabatic limit k = 0 (closed faces for T), pure-phase grids (C all 0 or
all 1) and a uniform state (exact solution with zero residual)."""
import dataclasses

import numpy as np
import pytest

import oracle as orc
import workloads as W
from gpu_util import host, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solve(prob, prec, rtol=1e-12):
    import workloads.device as D
    h, b_p, b_T, _ = D.setup(prob, prec)
    p, T = torch.empty_like(b_p), torch.empty_like(b_T)
    info = h.solve(b_p, b_T, p, T, rtol=rtol, max_cycles=60)
    levels = h.num_levels()
    return host(p), host(T), host(b_p), host(b_T), info, levels


GRIDS = [(2, (2, 2)), (2, (3, 5)), (2, (4, 2)), (2, (6, 10)), (2, (66, 2)),
         (3, (2, 2, 2)), (3, (5, 3, 7)), (3, (4, 6, 2)), (3, (10, 6, 14))]


@pytest.mark.parametrize("dim,n", GRIDS, ids=["x".join(map(str, g[1])) for g in GRIDS])
@pytest.mark.parametrize("prec", [0, 1])
def test_small_and_odd_grids(dim, n, prec):
    centre = [0.5] * dim
    prob = W.bubble_problem("e", dim, n, [centre], [0.3], W.P0, 10 * W.P0,
                            div_amp=1e-6, div_seed=3)
    P, T, bp, bT, info, levels = _solve(prob, prec)
    assert info["status"] == 0, info
    op, ob_p, ob_T, p_ref, T_ref = orc.solve(prob, rtol=1e-14)
    assert rel_err(bp, ob_p) <= 1e-13 and rel_err(bT, ob_T) <= 1e-13
    assert rel_err(P, p_ref) <= 1e-8 and rel_err(T, T_ref) <= 1e-8
    assert levels == orc.mg_levels(dim, prob.n)


@pytest.mark.parametrize("prec", [0, 1])
def test_adiabatic_limit_closed_faces(prec):
    """k = 0 in both phases: every T face is closed (harmonic mean of
    zeros); T couples to p only through the block."""
    liq = dataclasses.replace(W.LIQUID, k=0.0)
    gas = dataclasses.replace(W.GAS, k=0.0)
    base = W.bubble_problem("k0", 2, (96, 80), [(0.4, 0.5)], [0.2], W.P0, 10 * W.P0,
                            div_amp=1e-6, div_seed=5)
    prob = dataclasses.replace(base, liquid=liq, gas=gas)
    P, T, bp, bT, info, _ = _solve(prob, prec)
    assert info["status"] == 0, info
    op, ob_p, ob_T, p_ref, T_ref = orc.solve(prob, rtol=1e-14)
    assert rel_err(P, p_ref) <= 1e-8 and rel_err(T, T_ref) <= 1e-8


@pytest.mark.parametrize("c", [0.0, 1.0])
def test_pure_phase_grids(c):
    base = W.bubble_problem("pure", 3, (24, 16, 20), [(0.5, 0.5, 0.5)], [0.2], W.P0, W.P0,
                            div_amp=1e-6, div_seed=6)
    prob = dataclasses.replace(base, C=np.full_like(base.C, c))
    for prec in (0, 1):
        P, T, bp, bT, info, _ = _solve(prob, prec)
        assert info["status"] == 0, info
        op, ob_p, ob_T, p_ref, T_ref = orc.solve(prob, rtol=1e-14)
        assert rel_err(P, p_ref) <= 1e-8 and rel_err(T, T_ref) <= 1e-8


@pytest.mark.parametrize("prec", [0, 1])
def test_uniform_state_is_exact(prec):
    """Uniform provisional state and no velocity divergence: (p_adv, T_adv)
    solves the system exactly.  From a zero guess the solver reaches it;
    started there, it stops at cycle 0 and leaves it unchanged."""
    import workloads.device as D
    prob = W.bubble_problem("u", 2, (64, 48), [(0.5, 0.5)], [0.2], W.P0, W.P0)
    h, b_p, b_T, _ = D.setup(prob, prec)
    p, T = torch.empty_like(b_p), torch.empty_like(b_T)
    info = h.solve(b_p, b_T, p, T, rtol=1e-12, max_cycles=60)
    assert info["status"] == 0, info
    assert np.allclose(host(p), W.P0, rtol=1e-10, atol=0)
    assert np.allclose(host(T), W.T0, rtol=1e-10, atol=0)
    p.fill_(W.P0)
    T.fill_(W.T0)
    info = h.solve(b_p, b_T, p, T, rtol=1e-12, max_cycles=60, zero_guess=False)
    assert info["status"] == 0 and info["cycles"] == 0, info
    assert np.all(host(p) == W.P0) and np.all(host(T) == W.T0)


@pytest.mark.parametrize("prec", [0, 1])
def test_zero_rhs_stops_at_cycle_zero_with_zeros(prec):
    """b = 0 from a zero guess: the solve stops at cycle 0 and writes zeros
    into (p, T) whatever they held, on a fresh handle and after a solve
    that ended on an odd cycle (whose parity the next solve takes for its
    iterates); the zero guess itself is never stored, so this final write
    is the only one."""
    import workloads.device as D
    prob = W.bubble_problem("z", 2, (64, 48), [(0.5, 0.5)], [0.2], W.P0, 5 * W.P0,
                            div_amp=1e-6, div_seed=3)
    h, b_p, b_T, _ = D.setup(prob, prec)
    z = torch.zeros_like(b_p)
    for before in (None, 3):
        if before is not None:
            p, T = torch.empty_like(b_p), torch.empty_like(b_T)
            info = h.solve(b_p, b_T, p, T, rtol=1e-30, max_cycles=before, raise_on_noconv=False)
            assert info["cycles"] == before
        p, T = torch.full_like(b_p, 5.0), torch.full_like(b_T, -5.0)
        info = h.solve(z, z, p, T, rtol=1e-12)
        assert info["status"] == 0 and info["cycles"] == 0, info
        assert torch.all(p == 0) and torch.all(T == 0)
