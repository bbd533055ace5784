"""Step-by-step parity of the HIP library against the FP64 oracle: assembly,
paper right-hand side, FP64 residual, coarse hierarchy, smoother,
residual+restriction, prolongation and the coarsest solve, in both
precisions.  Tolerances: FP64 steps agree to a few units of round-off of
the terms involved; FP32 steps to a few FP32 ulps of those terms."""
import numpy as np
import pytest

import oracle as orc
import workloads as W
from gpu_util import dev, host, step_problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PROBS = step_problems()
PRECS = ["fp64", "mixed"]


@pytest.fixture(scope="module", params=list(PROBS))
def case(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import workloads.device as D
    prob = PROBS[request.param]
    op = orc.assemble(prob)
    out = {"name": request.param, "prob": prob, "op": op}
    for prec in PRECS:
        code = 1 if prec == "mixed" else 0
        h, b_p, b_T, t = D.setup(prob, code)
        out[prec] = (h, b_p, b_T, t)
    # oracle hierarchy, same coarsening as the library's
    ops = [op]
    for l in range(1, out["fp64"][0].num_levels()):
        ops.append(orc.coarse_operator(ops[-1]))
    out["ops"] = ops
    # the FP32 hierarchy of the mixed-precision V-cycle, built on the oracle
    # side: each coarse level is the averaging of the level above (summed in
    # FP64) rounded to FP32, level 1 from the FP64 finest operator (the
    # library coarsens level 1 from the finest operator's FP32 copy; the
    # two agree within the FP32 tolerances below)
    ops32 = [None]
    src = op
    for l in range(1, out["fp64"][0].num_levels()):
        c = orc.coarse_operator(src)
        c = orc.Operator(c.dim, c.n, c.h, _f32(c.F), _f32(c.B))
        ops32.append(c)
        src = c
    out["ops32"] = ops32
    return out


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32), dtype=np.float64)


def _close(a, b, rtol_scale, label):
    a, b = np.asarray(a), np.asarray(b)
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max() / scale
    assert err <= rtol_scale, f"{label}: max err {err:.3e} (scale {scale:.3e})"


def test_levels_match_oracle_coarsening(case):
    h = case["fp64"][0]
    for l, op in enumerate(case["ops"]):
        n, hl = h.level_dims(l)
        assert tuple(n) == tuple(op.n)
        assert hl == pytest.approx(op.h, rel=1e-15)


@pytest.mark.parametrize("prec", PRECS)
def test_assembly_and_coarse_operators(case, prec):
    """a1 + a3: finest operator (FP64 in both precisions) and every coarse
    level's faces and blocks."""
    h = case[prec][0]
    tol0 = 1e-14
    tolc = 1e-14 if prec == "fp64" else 2e-7
    for l, op in enumerate(case["ops"]):
        F, B = h.get_operator(l)
        F, B = host(F), host(B)
        tol = tol0 if l == 0 else tolc
        for c in range(2):
            for a in range(op.dim):
                _close(F[c * 3 + a], op.F[c * 3 + a], tol, f"level {l} face c{c} a{a}")
        for q in range(4):
            _close(B[q], op.B[q], tol, f"level {l} block {q}")


def test_paper_rhs(case):
    prob, op = case["prob"], case["op"]
    if prob.mode != "phases":
        pytest.skip("explicit mode takes the canonical right-hand side")
    _, b_p, b_T, _ = case["fp64"]
    rp, rT = orc.paper_rhs(op, prob)
    _close(host(b_p), rp, 1e-13, "b_p")
    _close(host(b_T), rT, 1e-14, "b_T")


@pytest.mark.parametrize("prec", PRECS)
def test_outer_residual(case, prec):
    """a4: FP64 residual of the mode-native form at a perturbed state, and
    its relative norms (fixed-order reduction)."""
    prob, op = case["prob"], case["op"]
    h, b_p, b_T, _ = case[prec]
    rng = np.random.default_rng(11)
    N = op.N
    if prob.mode == "phases":
        p_base = prob.p_adv.reshape(-1) if prob.p_adv is not None else np.full(N, prob.p_adv_const)
        p = p_base * (1 + 1e-3 * rng.standard_normal(N))
        T = prob.T_adv_const * (1 + 1e-4 * rng.standard_normal(N))
    else:
        p, T = rng.standard_normal(N), rng.standard_normal(N)
    # both sides take the oracle's right-hand side as the input
    bp, bT = orc.rhs(op, prob)
    r_p, r_T, rel = h.residual(dev(bp), dev(bT), dev(p), dev(T))
    if prob.mode == "phases":
        op_rp, op_rT = orc.paper_residual(op, bp, bT, p, T)
    else:
        op_rp, op_rT = orc.residual(op, bp, bT, p, T)
    # round-off of the terms: |b| and |operator terms| are ~1e4-1e6 x |res|
    _close(host(r_p), op_rp, 1e-11, "res_p")
    _close(host(r_T), op_rT, 1e-11, "res_T")
    ref_rel = [np.linalg.norm(op_rp) / np.linalg.norm(bp), np.linalg.norm(op_rT) / np.linalg.norm(bT)]
    np.testing.assert_allclose(rel, ref_rel, rtol=1e-10)


@pytest.mark.parametrize("prec", PRECS)
def test_outer_residual_zero_iterate(case, prec):
    """a4: the residual of a zero iterate (the first of every solve from a
    zero guess, a pointwise pass) equals the stencil residual of zero
    arrays bit for bit, norms included, and is b itself."""
    import torch
    prob, op = case["prob"], case["op"]
    h = case[prec][0]
    bp, bT = orc.rhs(op, prob)
    db_p, db_T = dev(bp), dev(bT)
    zero = torch.zeros_like(db_p)
    r_p, r_T, rel = h.residual(db_p, db_T, zero, zero)
    z_p, z_T, zrel = h.residual(db_p, db_T, None, None)
    assert torch.equal(r_p, z_p) and torch.equal(r_T, z_T)
    assert rel == zrel and all(x in (0.0, 1.0) for x in zrel)
    assert torch.equal(z_p, db_p) and torch.equal(z_T, db_T)


def _level_fields(op, seed, scale_u=True):
    rng = np.random.default_rng(seed)
    N = op.N
    f_p, f_T = rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)
    # unknowns on the scale the operator maps f to (diagonal scaling)
    u_p = rng.uniform(-1, 1, N) / np.abs(op.B[0]).max()
    u_T = rng.uniform(-1, 1, N) / np.abs(op.B[3]).max()
    return f_p, f_T, u_p, u_T


@pytest.mark.parametrize("prec", PRECS)
def test_smoother_matches_red_black_sweep(case, prec):
    """a5: one red-black block Gauss-Seidel sweep on every level."""
    h = case[prec][0]
    tol = 1e-12 if prec == "fp64" else 3e-5
    for l, op in enumerate(case["ops"]):
        if prec == "mixed" and l > 0:
            op = case["ops32"][l]         # the FP32 operator the V-cycle uses
        f_p, f_T, u_p, u_T = _level_fields(op, 100 + l)
        gp, gT = dev(u_p), dev(u_T)
        h.smooth(l, dev(f_p), dev(f_T), gp, gT, sweeps=1)
        rp, rT = u_p.copy(), u_T.copy()
        orc.sweep(op, f_p, f_T, rp, rT, "rb")
        _close(host(gp), rp, tol, f"level {l} p")
        _close(host(gT), rT, tol, f"level {l} T")


@pytest.mark.parametrize("prec", PRECS)
def test_restrict_residual(case, prec):
    """a6: coarse RHS = mean of the children's residual f - A u."""
    h = case[prec][0]
    tol = 1e-12 if prec == "fp64" else 3e-5
    ops = case["ops"]
    for l in range(len(ops) - 1):
        op = ops[l]
        if prec == "mixed" and l > 0:
            op = case["ops32"][l]
        f_p, f_T, u_p, u_T = _level_fields(op, 200 + l)
        fc_p, fc_T = h.restrict_residual(l, dev(f_p), dev(f_T), dev(u_p), dev(u_T))
        r_p, r_T = orc.residual(op, f_p, f_T, u_p, u_T)
        ref_p, ref_T = orc.restrict(op.dim, op.n, r_p, r_T)
        _close(host(fc_p), ref_p, tol, f"level {l} p")
        _close(host(fc_T), ref_T, tol, f"level {l} T")


@pytest.mark.parametrize("prec", PRECS)
def test_prolong_add(case, prec):
    """a8: u += P e with cell-centred linear weights."""
    h = case[prec][0]
    tol = 1e-15 if prec == "fp64" else 2e-7
    ops = case["ops"]
    rng = np.random.default_rng(3)
    for l in range(len(ops) - 1):
        op, opc = ops[l], ops[l + 1]
        e_p, e_T = rng.standard_normal(opc.N), rng.standard_normal(opc.N)
        u_p, u_T = rng.standard_normal(op.N), rng.standard_normal(op.N)
        gp, gT = dev(u_p), dev(u_T)
        h.prolong_add(l, dev(e_p), dev(e_T), gp, gT)
        orc.prolong_add(op.dim, op.n, e_p, e_T, u_p, u_T)
        _close(host(gp), u_p, tol, f"level {l} p")
        _close(host(gT), u_T, tol, f"level {l} T")


@pytest.mark.parametrize("prec", PRECS)
def test_coarse_solve(case, prec):
    """a7: exact FP64 solve on the coarsest grid (Gauss-Jordan inverse)
    against LU of the same operator."""
    h = case[prec][0]
    L = h.num_levels() - 1
    op = case["ops"][L]
    # the coarsest operator the library inverts, built on the oracle side
    opg = op if (prec == "fp64" or L == 0) else case["ops32"][L]
    rng = np.random.default_rng(4)
    f_p, f_T = rng.uniform(-1, 1, op.N), rng.uniform(-1, 1, op.N)
    if prec == "mixed":   # the V-cycle hands FP32 values to the coarse solve
        f_p, f_T = f_p.astype(np.float32).astype(np.float64), f_T.astype(np.float32).astype(np.float64)
    u_p, u_T = h.coarse_solve(dev(f_p), dev(f_T))
    M = orc.dense_matrix(opg)
    x = orc.lu_solve_dense(M, np.concatenate([f_p, f_T]))
    tol = 1e-11 if prec == "fp64" else 2e-7
    _close(host(u_p), x[: op.N], tol, "p")
    _close(host(u_T), x[op.N:], tol, "T")


@pytest.mark.parametrize("prec", PRECS)
def test_vcycle_reduces_residual(case, prec):
    """One V-cycle from zero contracts the residual strongly."""
    h = case[prec][0]
    op = case["ops"][0]
    rng = np.random.default_rng(6)
    f_p, f_T = rng.uniform(-1, 1, op.N), rng.uniform(-1, 1, op.N)
    e_p, e_T = h.vcycle(dev(f_p), dev(f_T))
    r_p, r_T = orc.residual(op, f_p, f_T, host(e_p), host(e_T))
    assert np.linalg.norm(r_p) < 0.2 * np.linalg.norm(f_p)
    assert np.linalg.norm(r_T) < 0.2 * np.linalg.norm(f_T)
