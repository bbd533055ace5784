"""Parity at the benchmarked sizes, in the launch configuration bench.py
times: a non-null stream, the fused finest-grid kernels, the single-block
tail, and bench.py's smoothing for the workload (its SWEEPS table).

  * 1024^2 bubble, FP64: the oracle's own multigrid solution is cheap
    enough to compare element by element.
  * 256^3 near-wall bubble (FP64 and mixed) and 512^3 collapse (mixed):
    the oracle recomputes the paper-form residual of the GPU solution
    (the certificate that holds at any size), the two precisions agree,
    and a manufactured solution u* (b = L(u*) formed by the oracle) is
    recovered (P8).
"""
import os
import sys

import numpy as np
import pytest

import oracle as orc
import workloads as W
from gpu_util import dev, host, rel_err

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402  (the per-workload smoothing table)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solve(prob, prec, rtol, workload, b=None, stiff=False, method=None):
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    # bench.py: the workload's smoothing; diffusive steps the library's V(2,2)
    nu1, nu2, coarse = (2, 2, 0) if stiff else bench.SWEEPS[workload]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        # the handle and the paper right-hand side as bench.py builds them
        # (div u* from the face velocities where the workload has them)
        h, b_p, b_T, t = D.setup(prob, prec, stream=stream)
        h.set_option(ptmg.PT_OPT_COARSE_SWEEPS, coarse)
        if b is not None:
            b_p, b_T = dev(b[0]), dev(b[1])
        p = torch.empty(prob.ncells, dtype=torch.float64, device="cuda")
        T = torch.empty_like(p)
        kw = {} if method is None else {"method": getattr(ptmg, method)}
        info = h.solve(b_p, b_T, p, T, rtol=rtol, max_cycles=40, nu1=nu1, nu2=nu2, **kw)
        torch.cuda.synchronize()
        out = (host(p), host(T), host(b_p), host(b_T), info)
        h.destroy()
    return out


def _manufactured(prob, op):
    """A smooth state u* near the provisional one, and b = L(u*) in the
    paper form, both from the oracle."""
    N = op.N
    sm = W.smooth_field(prob.dim, prob.n, seed=8).reshape(-1)
    p_base = prob.p_adv.reshape(-1) if prob.p_adv is not None else np.full(N, prob.p_adv_const)
    p_star = p_base + 1e-3 * W.P0 * sm
    T_star = prob.T_adv_const + 1e-2 * sm
    zero = np.zeros(N)
    r_p, r_T = orc.paper_residual(op, zero, zero, p_star, T_star)   # = -L(u*)
    return p_star, T_star, -r_p, -r_T


def test_bubble2d_1024_fp64_matches_oracle():
    prob = W.bubble2d(1024)
    P, T, bp, bT, info = _solve(prob, 0, 1e-12, "bubble2d_1024")
    assert info["status"] == 0 and info["cycles"] <= 6, info
    op = orc.assemble(prob)
    ob_p, ob_T = orc.paper_rhs(op, prob)
    assert rel_err(bp, ob_p) <= 1e-13 and rel_err(bT, ob_T) <= 1e-14
    rel = orc.relres(op, ob_p, ob_T, P, T)
    assert rel.max() <= 2e-12, rel
    p_ref, T_ref, cyc, _ = orc.mg_solve(op, ob_p, ob_T, rtol=1e-14)
    assert cyc > 0
    assert rel_err(P, p_ref) <= 1e-8 and rel_err(T, T_ref) <= 1e-8
    # the perturbation from the provisional state (measured 6e-8 for both)
    assert rel_err(P - W.P0, p_ref - W.P0) <= 1e-6
    assert rel_err(T - W.T0, T_ref - W.T0) <= 1e-6


def test_wall3d_256_certified_by_oracle_residual():
    """FP64 and mixed solves, each certified by the oracle's residual; the
    two precisions agree."""
    prob = W.wall3d(256)
    op = orc.assemble(prob)
    ob_p, ob_T = orc.paper_rhs(op, prob)
    sols = {}
    for prec in (0, 1):
        P, T, bp, bT, info = _solve(prob, prec, 1e-12, "wall3d_256")
        assert info["status"] == 0 and info["cycles"] <= 8, info
        rel = orc.relres(op, ob_p, ob_T, P, T)
        assert rel.max() <= 2e-12, (prec, rel)
        sols[prec] = (P, T)
    assert rel_err(sols[1][0], sols[0][0]) <= 1e-9
    assert rel_err(sols[1][1], sols[0][1]) <= 1e-12


def test_wall3d_256_manufactured_solution():
    prob = W.wall3d(256)
    op = orc.assemble(prob)
    p_star, T_star, b_p, b_T = _manufactured(prob, op)
    P, T, _, _, info = _solve(prob, 1, 1e-13, "wall3d_256", b=(b_p, b_T))
    assert info["status"] == 0, info
    assert rel_err(P, p_star) <= 1e-8 and rel_err(T, T_star) <= 1e-8
    # the perturbation from the provisional state (measured 1e-7 and 8e-11)
    p_adv = prob.p_adv.reshape(-1)
    assert rel_err(P - p_adv, p_star - p_adv) <= 1e-6
    assert rel_err(T - prob.T_adv_const, T_star - prob.T_adv_const) <= 1e-6


def test_collapse3d_512_mixed_certified_and_manufactured():
    prob = W.collapse3d(512)
    P, T, bp, bT, info = _solve(prob, 1, 1e-12, "collapse3d_512")
    assert info["status"] == 0 and info["cycles"] <= 8, info
    op = orc.assemble(prob)
    ob_p, ob_T = orc.paper_rhs(op, prob)
    rel = orc.relres(op, ob_p, ob_T, P, T)
    assert rel.max() <= 2e-12, rel
    del P, T
    p_star, T_star, b_p, b_T = _manufactured(prob, op)
    P, T, _, _, info = _solve(prob, 1, 1e-13, "collapse3d_512", b=(b_p, b_T))
    assert info["status"] == 0, info
    assert rel_err(P, p_star) <= 1e-8 and rel_err(T, T_star) <= 1e-8
    # the perturbation from the provisional state (measured 1.5e-8 and 1.3e-11)
    p_adv = prob.p_adv.reshape(-1)
    assert rel_err(P - p_adv, p_star - p_adv) <= 1e-6
    assert rel_err(T - prob.T_adv_const, T_star - prob.T_adv_const) <= 1e-6


def test_axi2d_1024_fp64_matches_oracle():
    """The r-z bubble near the wall at the benchmarked size and smoothing:
    the oracle's r-z residual certifies the GPU solution, which matches the
    oracle's own multigrid solution."""
    prob = W.axi2d(1024)
    P, T, bp, bT, info = _solve(prob, 0, 1e-12, "axi2d_1024")
    assert info["status"] == 0 and info["cycles"] <= 6, info
    op = orc.assemble(prob)
    assert op.axi == 1
    ob_p, ob_T = orc.paper_rhs(op, prob)
    assert rel_err(bp, ob_p) <= 1e-13 and rel_err(bT, ob_T) <= 1e-14
    rel = orc.relres(op, ob_p, ob_T, P, T)
    assert rel.max() <= 2e-12, rel
    p_ref, T_ref, cyc, _ = orc.mg_solve(op, ob_p, ob_T, rtol=1e-14)
    assert cyc > 0
    assert rel_err(P, p_ref) <= 1e-8 and rel_err(T, T_ref) <= 1e-8
    # the perturbation from the provisional state (measured 8e-10 and 7e-10)
    p_adv = prob.p_adv.reshape(-1)
    assert rel_err(P - p_adv, p_ref - p_adv) <= 1e-6
    assert rel_err(T - W.T0, T_ref - W.T0) <= 1e-6


def test_state2d_1024_certified_by_oracle_residual():
    """The state-mode step at the benchmarked size and smoothing: the GPU's
    own provisional state, div u* of the face velocities and operator; the
    oracle's residual of the GPU solution, with the oracle's right-hand
    side."""
    prob = W.state2d(1024)
    P, T, bp, bT, info = _solve(prob, 0, 1e-12, "state2d_1024")
    assert info["status"] == 0 and info["cycles"] <= 6, info
    op = orc.assemble(prob)
    ob_p, ob_T = orc.paper_rhs(op, prob)
    assert rel_err(bp, ob_p) <= 1e-10
    rel = orc.relres(op, ob_p, ob_T, P, T)
    assert rel.max() <= 1e-11, rel


def test_state3d_256_mixed_certified_by_oracle_residual():
    """The 3-D state-mode step in mixed precision at the benchmarked size
    and smoothing, certified by the oracle's residual."""
    prob = W.state3d(256)
    P, T, bp, bT, info = _solve(prob, 1, 1e-12, "state3d_256")
    assert info["status"] == 0 and info["cycles"] <= 8, info
    op = orc.assemble(prob)
    ob_p, ob_T = orc.paper_rhs(op, prob)
    assert rel_err(bp, ob_p) <= 1e-10
    rel = orc.relres(op, ob_p, ob_T, P, T)
    assert rel.max() <= 1e-11, rel


def test_stiff_bubble2d_1024_certified_by_oracle_residual():
    """The diffusive-CFL step at 1024^2 (bench.py --stiff, defect loop with
    the library's V(2,2)), certified by the oracle's residual."""
    prob = W.bubble2d(1024, stiff=True)
    P, T, bp, bT, info = _solve(prob, 0, 1e-12, "bubble2d_1024", stiff=True)
    assert info["status"] == 0 and 8 <= info["cycles"] <= 40, info
    op = orc.assemble(prob)
    ob_p, ob_T = orc.paper_rhs(op, prob)
    rel = orc.relres(op, ob_p, ob_T, P, T)
    assert rel.max() <= 2e-12, rel


def test_explicit_64_matches_oracle():
    """The 64^2 constant-coefficient case (mean constraint, rtol 1e-10) at
    bench.py's smoothing, against the oracle's sparse direct solution."""
    prob = W.explicit_const(64, 64)
    P, T, bp, bT, info = _solve(prob, 0, 1e-10, "explicit_64")
    assert info["status"] == 0 and info["cycles"] <= 12, info
    op, ob_p, ob_T, p_ref, T_ref = orc.solve(prob)
    assert rel_err(bp, ob_p) == 0.0 and rel_err(bT, ob_T) == 0.0
    rel = orc.relres(op, ob_p, ob_T, P, T)
    assert rel.max() <= 2e-10, rel
    assert rel_err(P, p_ref) <= 1e-8 and rel_err(T, T_ref) <= 1e-8


def test_stiff_wall3d_256_certified_by_oracle_residual():
    """The diffusive-CFL 256^3 step in mixed precision (bench.py --stiff,
    V(2,2)), certified by the oracle's residual."""
    prob = W.wall3d(256, stiff=True)
    P, T, bp, bT, info = _solve(prob, 1, 1e-12, "wall3d_256", stiff=True)
    assert info["status"] == 0, info
    op = orc.assemble(prob)
    ob_p, ob_T = orc.paper_rhs(op, prob)
    rel = orc.relres(op, ob_p, ob_T, P, T)
    assert rel.max() <= 2e-12, rel


def test_stiff_bubble2d_1024_bicgstab_certified_by_oracle_residual():
    """bench.py --stiff --method bicgstab at 1024^2: BiCGStab with the
    V-cycle as preconditioner, certified by the oracle's residual, in fewer
    V-cycles than the defect loop."""
    prob = W.bubble2d(1024, stiff=True)
    P, T, bp, bT, info = _solve(prob, 0, 1e-12, "bubble2d_1024", stiff=True,
                                method="PT_SOLVE_BICGSTAB")
    assert info["status"] == 0, info
    op = orc.assemble(prob)
    ob_p, ob_T = orc.paper_rhs(op, prob)
    rel = orc.relres(op, ob_p, ob_T, P, T)
    assert rel.max() <= 2e-12, rel
    _, _, _, _, idef = _solve(prob, 0, 1e-12, "bubble2d_1024", stiff=True)
    assert info["cycles"] < idef["cycles"], (info["cycles"], idef["cycles"])
