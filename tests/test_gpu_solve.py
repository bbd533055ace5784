"""Solve parity of the HIP library (FP64 V-cycle, and FP32 V-cycle under FP64
iterative refinement) against the FP64 oracle, plus error paths and
determinism.  Bar: the oracle's own paper-form relative residual of the
GPU solution <= the requested tolerance (x2 for round-off), and a
relative error <= 1e-8 per component against the oracle's solution.  The
p error is ~1e4 x the paper-form residual for bubble problems (the l4
coupling), so the solves that check the error run to 1e-12."""
import ctypes

import numpy as np
import pytest

import oracle as orc
import workloads as W
from gpu_util import dev, host, rel_err, step_problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_REF = {}


def _reference(name, prob):
    if name not in _REF:
        _REF[name] = orc.solve(prob, rtol=1e-14, direct_max=40000)
    return _REF[name]


@pytest.mark.parametrize("name", list(step_problems()))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_matches_oracle(name, prec):
    import workloads.device as D
    prob = step_problems()[name]
    op, b_p, b_T, p_ref, T_ref = _reference(name, prob)
    h, gb_p, gb_T, _ = D.setup(prob, 1 if prec == "mixed" else 0)
    p, T = torch.empty_like(gb_p), torch.empty_like(gb_T)
    info = h.solve(gb_p, gb_T, p, T, rtol=1e-12, max_cycles=40)
    assert info["status"] == 0, info
    assert info["cycles"] <= 12, info
    P, Tt = host(p), host(T)
    rel = orc.relres(op, b_p, b_T, P, Tt)     # the oracle's own right-hand side
    assert rel.max() <= 2e-12, rel
    assert rel_err(P, p_ref) <= 1e-8
    assert rel_err(Tt, T_ref) <= 1e-8
    if prob.mode == "phases":   # the stricter perturbation measure
        p_adv = prob.p_adv.reshape(-1) if prob.p_adv is not None else prob.p_adv_const
        assert rel_err(P - p_adv, p_ref - p_adv) <= 1e-6
        assert rel_err(Tt - prob.T_adv_const, T_ref - prob.T_adv_const) <= 1e-6


def test_mixed_history_contracts_like_fp64():
    """Iterative refinement with the FP32 V-cycle converges at the same
    rate as the FP64 V-cycle until FP32 limits the correction."""
    import workloads.device as D
    prob = step_problems()["bubble2d_200x136"]
    hist = {}
    for prec in (0, 1):
        h, b_p, b_T, _ = D.setup(prob, prec)
        p, T = torch.empty_like(b_p), torch.empty_like(b_T)
        info = h.solve(b_p, b_T, p, T, rtol=1e-13, max_cycles=30)
        hist[prec] = np.array(info["hist"])
    n = min(len(hist[0]), len(hist[1]), 4)
    for c in range(2):
        assert hist[1][n - 1, c] <= 10 * max(hist[0][n - 1, c], 1e-13)


def test_deterministic_bitwise():
    import workloads.device as D
    prob = step_problems()["bubble3d_40x24x56"]
    h, b_p, b_T, _ = D.setup(prob, 1)
    outs = []
    for _ in range(2):
        p, T = torch.empty_like(b_p), torch.empty_like(b_T)
        h.solve(b_p, b_T, p, T, rtol=1e-10)
        outs.append((p.clone(), T.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_warm_start_and_update():
    """The initial guess is used (paper: a good guess saves work), and an
    update with new fields reuses the handle."""
    import workloads.device as D
    prob = step_problems()["twobubble2d_96x80"]
    h, b_p, b_T, t = D.setup(prob, 1)
    p, T = torch.empty_like(b_p), torch.empty_like(b_T)
    cold = h.solve(b_p, b_T, p, T, rtol=1e-11)
    warm = h.solve(b_p, b_T, p, T, rtol=1e-11, zero_guess=False)
    assert warm["cycles"] == 0 and cold["cycles"] > 0
    prob2 = W.bubble_problem("b4", 2, (96, 80), [(0.35, 0.45)], [0.2], W.P0, 3 * W.P0)
    s2, t2 = D.to_device(prob2)
    h.update(s2)
    b2p, b2T = h.paper_rhs(t2.get("p_adv"), None, None)
    info = h.solve(b2p, b2T, p, T, rtol=1e-12)
    op2, rb_p, rb_T, p2, T2 = orc.solve(prob2, direct_max=40000)
    assert rel_err(host(p), p2) <= 1e-8 and rel_err(host(T), T2) <= 1e-8
    assert info["status"] == 0


def test_stiff_time_step():
    """Diffusive-CFL time step (much larger dt): still converges."""
    import workloads.device as D
    prob = W.bubble_problem("st", 2, (128, 128), [(0.5, 0.5)], [0.1], W.P0, W.P0,
                            div_amp=1e-6, div_seed=2, stiff=True)
    op, b_p, b_T, p_ref, T_ref = orc.solve(prob, direct_max=40000)
    for prec in (0, 1):
        h, gb_p, gb_T, _ = D.setup(prob, prec)
        p, T = torch.empty_like(gb_p), torch.empty_like(gb_T)
        info = h.solve(gb_p, gb_T, p, T, rtol=1e-11, max_cycles=60)
        assert info["status"] == 0, info
        assert rel_err(host(p), p_ref) <= 1e-8 and rel_err(host(T), T_ref) <= 1e-8


def test_mean_constraint_poisson():
    """a11: B = 0 (pure Neumann Poisson in both components): zero-mean
    solution of the projected right-hand side."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    n = (80, 48)
    N = n[0] * n[1]
    rng = np.random.default_rng(1)
    prob = W.Problem(name="poisson", dim=2, n=(80, 48, 1), h=1.0 / 80, mode="explicit",
                     alpha_p=1.0, alpha_T=0.25, B_const=(0.0, 0.0, 0.0, 0.0),
                     f_p=rng.uniform(-1, 1, N), f_T=rng.uniform(-1, 1, N), mean_constraint=True)
    op = orc.assemble(prob)
    fp = prob.f_p - prob.f_p.mean()
    fT = prob.f_T - prob.f_T.mean()
    p_ref, T_ref, cyc, _ = orc.mg_solve(op, fp, fT, rtol=1e-13, pin_mean=True)
    assert cyc > 0
    for prec in (0, 1):
        h, b_p, b_T, _ = D.setup(prob, prec)
        p, T = torch.empty_like(b_p), torch.empty_like(b_T)
        info = h.solve(b_p, b_T, p, T, rtol=1e-11, max_cycles=60)
        assert info["status"] == 0, info
        assert abs(host(p).mean()) < 1e-12 * np.abs(p_ref).max()
        assert rel_err(host(p), p_ref) <= 1e-8 and rel_err(host(T), T_ref) <= 1e-8


def test_error_paths():
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = W.bubble_problem("e", 2, (32, 32), [(0.5, 0.5)], [0.2], W.P0, W.P0)
    # C outside [0, 1]
    bad = prob.C.copy()
    bad.reshape(-1)[7] = 1.5
    prob_bad = W.Problem(**{**prob.__dict__, "C": bad})
    s, t = D.to_device(prob_bad)
    with pytest.raises(ptmg.PtMgError) as e:
        ptmg.PtMg(s, 0)
    assert e.value.status == ptmg.PT_ERR_ARG
    # a block with det < 0
    pe = W.explicit_const(32, 32)
    pe = W.Problem(**{**pe.__dict__, "B_const": (1.0, 3.0, 2.0, 1.0)})
    s, t = D.to_device(pe)
    with pytest.raises(ptmg.PtMgError) as e:
        ptmg.PtMg(s, 0)
    assert e.value.status == ptmg.PT_ERR_SINGULAR
    # max_cycles reached: status returned, iterate finite, handle usable
    h, b_p, b_T, _ = D.setup(prob, 1)
    p, T = torch.empty_like(b_p), torch.empty_like(b_T)
    info = h.solve(b_p, b_T, p, T, rtol=1e-15, max_cycles=1, raise_on_noconv=False)
    assert info["status"] == ptmg.PT_ERR_NOCONV and info["cycles"] == 1
    assert torch.isfinite(p).all() and torch.isfinite(T).all()
    # non-finite right-hand side
    b_nan = b_p.clone()
    b_nan[5] = float("nan")
    info = h.solve(b_nan, b_T, p, T, rtol=1e-9, raise_on_noconv=False)
    assert info["status"] == ptmg.PT_ERR_NOCONV
    info = h.solve(b_p, b_T, p, T, rtol=1e-10)
    assert info["status"] == 0


def test_timing_and_counters():
    import workloads.device as D
    prob = step_problems()["bubble3d_40x24x56"]
    h, b_p, b_T, _ = D.setup(prob, 1)
    p, T = torch.empty_like(b_p), torch.empty_like(b_T)
    from paper_2206_11294_amd import ptmg
    h.set_option(ptmg.PT_OPT_SPECULATE, 0)     # exact launch counts
    h.set_timing(True)
    h.reset_stats()
    info = h.solve(b_p, b_T, p, T, rtol=1e-9)
    st = h.kernel_stats()
    # one fused launch per sweep; V(2,2) in 3-D FP32: the second pre-sweep
    # also restricts its residual (a class of its own)
    assert st["smooth_fine"]["launches"] == 3 * info["cycles"]
    assert st["smooth_fine_transfer"]["launches"] == info["cycles"]
    assert st["outer_residual"]["launches"] == info["cycles"] + 1
    assert st["smooth_fine"]["ms"] > 0 and st["smooth_fine"]["bytes"] > 0
    assert st["smooth_fine_transfer"]["ms"] > 0
    assert h.last_cell_updates() > 0
    ts = h.timed_stats()
    for c in st:      # every run timed: the timed launches are all launches
        assert ts[c]["launches"] == st[c]["launches"] and ts[c]["bytes"] == st[c]["bytes"], c
    # one run in three of the finest-grid smoother: two runs per cycle, of
    # one launch (before the restricting sweep) and two (after the cycle)
    h.set_timing(True, classes=["smooth_fine"])
    h.set_option(ptmg.PT_OPT_TIMING_EVERY, 3)
    assert h.get_option(ptmg.PT_OPT_TIMING_EVERY) == 3
    h.reset_stats()
    info = h.solve(b_p, b_T, p, T, rtol=1e-9)
    st, ts = h.kernel_stats(), h.timed_stats()
    runs = 2 * info["cycles"]
    want = sum(1 if r % 2 == 0 else 2 for r in range(runs) if r % 3 == 0)
    assert ts["smooth_fine"]["launches"] == want
    assert ts["smooth_fine"]["ms"] > 0 and ts["outer_residual"]["launches"] == 0
    assert ts["smooth_fine_transfer"]["launches"] == 0
    assert st["smooth_fine"]["launches"] == 3 * info["cycles"]
    with pytest.raises(ptmg.PtMgError):
        h.set_option(ptmg.PT_OPT_TIMING_EVERY, 0)


@pytest.mark.parametrize("name", ["bubble2d_200x136", "bubble3d_40x24x56"])
def test_graph_replay_matches_direct_launches(name):
    """With PT_OPT_GRAPHS on a non-null stream the coarse-level V-cycle is
    replayed from a HIP graph (several replays per solve, host
    synchronisations in between) and the hierarchy build after an assembly
    from another; every solve must equal the one with direct launches bit
    for bit."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = step_problems()[name]
    outs = {}
    for mode in ("direct", "graph"):
        stream = torch.cuda.Stream() if mode == "graph" else None
        ctx = torch.cuda.stream(stream) if stream is not None else torch.cuda.stream(
            torch.cuda.current_stream())
        with ctx:
            h, b_p, b_T, _ = D.setup(prob, 1, stream=stream)
            assert h.get_option(ptmg.PT_OPT_GRAPHS) == 0
            if mode == "graph":
                h.set_option(ptmg.PT_OPT_GRAPHS, 1)
                s2, t2 = D.to_device(prob)
                for _ in range(2):   # hierarchy build captured, then replayed
                    h.update(s2, keepalive=t2)
            res = []
            for _ in range(3):
                p, T = torch.empty_like(b_p), torch.empty_like(b_T)
                info = h.solve(b_p, b_T, p, T, rtol=1e-12)
                assert info["status"] == 0 and info["cycles"] >= 2
                res.append((p.clone(), T.clone()))
            torch.cuda.synchronize()
        for r in res[1:]:
            assert torch.equal(r[0], res[0][0]) and torch.equal(r[1], res[0][1])
        outs[mode] = res[0]
    assert torch.equal(outs["direct"][0], outs["graph"][0])
    assert torch.equal(outs["direct"][1], outs["graph"][1])


@pytest.mark.parametrize("name", ["bubble2d_200x136", "bubble3d_40x24x56"])
def test_hierarchy_graph_follows_fused_toggle(name):
    """PT_OPT_FUSED switched between two updates of a handle that replays
    its hierarchy build from a graph: the build is captured again with the
    other kernels, and every level's operator and the solve equal those of
    a handle with direct launches bit for bit."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = step_problems()[name]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        hg, b_p, b_T, _ = D.setup(prob, 1, stream=stream)
        hd, _, _, _ = D.setup(prob, 1, stream=stream)
        hg.set_option(ptmg.PT_OPT_GRAPHS, 1)
        s2, t2 = D.to_device(prob)
        for fused in (1, 1, 0, 0, 1):
            for h in (hg, hd):
                h.set_option(ptmg.PT_OPT_FUSED, fused)
                h.update(s2, keepalive=t2)
            for lv in range(hg.num_levels()):
                Fg, Bg = hg.get_operator(lv)
                Fd, Bd = hd.get_operator(lv)
                assert torch.equal(Fg, Fd) and torch.equal(Bg, Bd), (fused, lv)
            sol = []
            for h in (hg, hd):
                p, T = torch.empty_like(b_p), torch.empty_like(b_T)
                info = h.solve(b_p, b_T, p, T, rtol=1e-12)
                assert info["status"] == 0
                sol.append((p, T))
            torch.cuda.synchronize()
            assert torch.equal(sol[0][0], sol[1][0]) and torch.equal(sol[0][1], sol[1][1])


@pytest.mark.parametrize("prec", [0, 1])
def test_level1_coarsening_3d_matches_reference(prec):
    """3-D level 1 coarsened from the finest level by the plane-marching
    kernel (PT_OPT_FUSED on) equals the gather kernel's (off) bit for bit,
    on ragged 64 x 4 tiles and z chunks (40 x 24 x 56 and 160 x 48 x 56),
    and so do every coarser level and the solve."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    probs = [step_problems()["bubble3d_40x24x56"],
             W.bubble_problem("b3c", 3, (160, 48, 56), [(0.4, 0.5, 0.5)], [0.25], W.P0,
                              10 * W.P0, div_amp=1e-6, div_seed=15)]
    for prob in probs:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            h1, b_p, b_T, _ = D.setup(prob, prec, stream=stream)
            h0, _, _, _ = D.setup(prob, prec, stream=stream)
            h0.set_option(ptmg.PT_OPT_FUSED, 0)
            s2, t2 = D.to_device(prob)
            for h in (h1, h0):
                h.update(s2, keepalive=t2)
            for lv in range(1, h1.num_levels()):
                F1, B1 = h1.get_operator(lv)
                F0, B0 = h0.get_operator(lv)
                assert torch.equal(F1, F0) and torch.equal(B1, B0), (prob.name, lv)
            h0.set_option(ptmg.PT_OPT_FUSED, 1)
            sol = []
            for h in (h1, h0):
                p, T = torch.empty_like(b_p), torch.empty_like(b_T)
                info = h.solve(b_p, b_T, p, T, rtol=1e-12)
                assert info["status"] == 0
                sol.append((p, T, info["hist"]))
            torch.cuda.synchronize()
            assert sol[0][2] == sol[1][2]
            assert torch.equal(sol[0][0], sol[1][0]) and torch.equal(sol[0][1], sol[1][1])


@pytest.mark.parametrize("name", ["bubble2d_200x136", "bubble3d_40x24x56"])
def test_hierarchy_graph_follows_time_step(name):
    """A mixed-precision phases handle keeps its finest block compact, with
    constants of dt and the phases that the hierarchy graph holds as kernel
    arguments: updates with another dt (and back) capture it again, and
    every level's operator and the solve equal those of a handle with
    direct launches bit for bit."""
    import dataclasses
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = step_problems()[name]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        hg, b_p, b_T, _ = D.setup(prob, 1, stream=stream)
        hd, _, _, _ = D.setup(prob, 1, stream=stream)
        hg.set_option(ptmg.PT_OPT_GRAPHS, 1)
        for dt in (prob.dt, 0.5 * prob.dt, 0.5 * prob.dt, prob.dt):
            pr = dataclasses.replace(prob, dt=dt)
            s2, t2 = D.to_device(pr)
            for h in (hg, hd):
                h.update(s2, keepalive=t2)
            for lv in range(hg.num_levels()):
                Fg, Bg = hg.get_operator(lv)
                Fd, Bd = hd.get_operator(lv)
                assert torch.equal(Fg, Fd) and torch.equal(Bg, Bd), (dt, lv)
            sol = []
            for h in (hg, hd):
                p, T = torch.empty_like(b_p), torch.empty_like(b_T)
                info = h.solve(b_p, b_T, p, T, rtol=1e-12)
                assert info["status"] == 0
                sol.append((p, T))
            torch.cuda.synchronize()
            assert torch.equal(sol[0][0], sol[1][0]) and torch.equal(sol[0][1], sol[1][1])


@pytest.mark.parametrize("n", [(136, 40, 48), (68, 36, 36)])
def test_fused_restriction_3d_equals_reference(n):
    """The 3-D FP32 finest sweep that also restricts its residual (the last
    pre-sweep of each V-cycle) against the separate sweep and restriction
    kernels (PT_OPT_FUSED off): V-cycles with one to three pre-sweeps (one:
    the fused sweep starts from zero) and a whole solve agree bit for bit,
    on grids of several tiles and z chunks with ragged edges."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = W.bubble_problem("fr", 3, n, [(0.45, 0.5, 0.4)], [0.3], 100 * W.P0, 0.01 * W.P0,
                            div_amp=1e-7, div_seed=6)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, b_p, b_T, _ = D.setup(prob, 1, stream=stream)
        rng = np.random.default_rng(3)
        f_p, f_T = dev(rng.uniform(-1, 1, h.N)), dev(rng.uniform(-1, 1, h.N))
        out = {}
        for fused in (1, 0):
            h.set_option(ptmg.PT_OPT_FUSED, fused)
            res = []
            for nu1 in (1, 2, 3):
                e = h.vcycle(f_p, f_T, nu1=nu1, nu2=1)
                res += [e[0].clone(), e[1].clone()]
            p, T = torch.empty_like(b_p), torch.empty_like(b_T)
            info = h.solve(b_p, b_T, p, T, rtol=1e-12, nu1=3, nu2=2)
            torch.cuda.synchronize()
            assert info["status"] == 0
            res += [p.clone(), T.clone()]
            out[fused] = (res, info["cycles"], info["hist"])
    for a, b in zip(out[1][0], out[0][0]):
        assert torch.equal(a, b), (a - b).abs().max().item()
    assert out[1][1] == out[0][1] and out[1][2] == out[0][2]


@pytest.mark.parametrize("name", ["bubble2d_200x136", "bubble3d_40x24x56", "explicit_64",
                                  "twobubble2d_96x80"])
@pytest.mark.parametrize("prec", [0, 1])
def test_tail_and_graph_paths_agree(name, prec):
    """The fused sweeps, the single-block tail cycle and the graph replay
    run the same per-cell arithmetic as the plain colour passes: solves and
    V-cycles agree with the reference launch path bit for bit."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = step_problems()[name]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, b_p, b_T, _ = D.setup(prob, prec, stream=stream)
        rng = np.random.default_rng(2)
        f_p, f_T = dev(rng.uniform(-1, 1, h.N)), dev(rng.uniform(-1, 1, h.N))
        out = {}
        for opts in ((1, 1, 1), (0, 0, 0)):
            h.set_option(ptmg.PT_OPT_GRAPHS, opts[0])
            h.set_option(ptmg.PT_OPT_TAIL, opts[1])
            h.set_option(ptmg.PT_OPT_FUSED, opts[2])
            p, T = torch.empty_like(b_p), torch.empty_like(b_T)
            h.solve(b_p, b_T, p, T, rtol=1e-12)
            e = h.vcycle(f_p, f_T)
            torch.cuda.synchronize()
            out[opts] = (p.clone(), T.clone(), e[0].clone(), e[1].clone())
        h.set_option(ptmg.PT_OPT_TAIL, 1)
        if name == "explicit_64":   # 32^2 .. 2^2 fit in one block's LDS
            assert h.get_option(ptmg.PT_OPT_TAIL) >= 4
    for a, b in zip(out[(1, 1, 1)], out[(0, 0, 0)]):
        assert torch.equal(a, b), (a - b).abs().max().item()


@pytest.mark.parametrize("prec", [0, 1])
def test_solution_parity_and_rate_hints(prec):
    """A zero-guess solve keeps its odd or even iterates in the caller's
    arrays as the previous solve on the handle ended, and predicts its
    second cycle from the previous solve's last contraction: on one handle,
    solves that end after 3, 2, 2, 1, 4 and 3 cycles (and one that
    converges) equal, bit for bit, the same solves each on a fresh handle."""
    import workloads.device as D
    prob = step_problems()["bubble2d_200x136"]
    op = orc.assemble(prob)
    b_p, b_T = orc.rhs(op, prob)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, gb_p, gb_T, _ = D.setup(prob, prec, stream=stream)
        for m in (3, 2, 2, 1, 4, 3, None):
            kw = dict(rtol=1e-12, max_cycles=40) if m is None else \
                dict(rtol=1e-30, max_cycles=m, raise_on_noconv=False)
            p, T = torch.full_like(gb_p, 7.0), torch.full_like(gb_T, 7.0)
            i1 = h.solve(gb_p, gb_T, p, T, **kw)
            h2, gb_p2, gb_T2, _ = D.setup(prob, prec, stream=stream)
            p2, T2 = torch.full_like(gb_p, -3.0), torch.full_like(gb_T, -3.0)
            i2 = h2.solve(gb_p2, gb_T2, p2, T2, **kw)
            torch.cuda.synchronize()
            h2.destroy()
            assert i1["cycles"] == i2["cycles"] and i1["hist"] == i2["hist"]
            assert i1["status"] == i2["status"]
            if m is not None:
                assert i1["cycles"] == m
            assert torch.equal(p, p2) and torch.equal(T, T2)
        assert max(orc.relres(op, b_p, b_T, host(p), host(T))) <= 2e-12


@pytest.mark.parametrize("nu", [(2, 2), (3, 2), (2, 1), (4, 3), (1, 2)])
@pytest.mark.parametrize("name", ["bubble2d_200x136", "explicit_64", "twobubble2d_96x80"])
def test_fused_solve_matches_reference_per_sweep_count(name, nu):
    """2-D FP64 solves with the fused finest-level sweeps and transfers at
    several (nu1, nu2): solution, cycles and every residual norm equal
    those of the separate kernels (PT_OPT_FUSED off) bit for bit, on a grid
    whose width is no multiple of the 256-column tiles and with the mean
    constraint (explicit_64); the solve meets the tolerance against the
    oracle's own right-hand side."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = step_problems()[name]
    op = orc.assemble(prob)
    b_p, b_T = orc.rhs(op, prob)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, gb_p, gb_T, _ = D.setup(prob, 0, stream=stream)
        out = {}
        for fused in (1, 0):
            h.set_option(ptmg.PT_OPT_FUSED, fused)
            p, T = torch.empty_like(gb_p), torch.empty_like(gb_T)
            info = h.solve(gb_p, gb_T, p, T, rtol=1e-11, nu1=nu[0], nu2=nu[1], max_cycles=60)
            torch.cuda.synchronize()
            out[fused] = (p.clone(), T.clone(), info)
    (p1, T1, i1), (p0, T0, i0) = out[1], out[0]
    assert i1["status"] == i0["status"] == 0
    assert i1["cycles"] == i0["cycles"] and i1["hist"] == i0["hist"]
    assert torch.equal(p1, p0) and torch.equal(T1, T0)
    assert max(orc.relres(op, b_p, b_T, host(p1), host(T1))) <= 2e-11


@pytest.mark.parametrize("prec", [0, 1])
def test_coarse_restriction_3d_matches_reference(prec):
    """3-D coarse levels of at least 2^20 cells restrict their residual with
    the plane-marching kernel: equal to the gather kernel (PT_OPT_FUSED off)
    bit for bit, on a level of ragged 64-column tiles (160 x 96 x 96), and
    the V-cycle and solve with it too."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = W.bubble_problem("b3r", 3, (320, 192, 192), [(0.45, 0.5, 0.55)], [0.2], W.P0,
                            10 * W.P0, div_amp=1e-6, div_seed=13)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, b_p, b_T, _ = D.setup(prob, prec, stream=stream)
        assert h.level_dims(1)[0] == (160, 96, 96)
        N1 = 160 * 96 * 96
        rng = np.random.default_rng(17)
        f_p, f_T = dev(rng.uniform(-1, 1, N1)), dev(rng.uniform(-1, 1, N1))
        u_p, u_T = dev(rng.uniform(-1e-9, 1e-9, N1)), dev(rng.uniform(-1e-3, 1e-3, N1))
        out = {}
        for fused in (1, 0):
            h.set_option(ptmg.PT_OPT_FUSED, fused)
            fc = h.restrict_residual(1, f_p, f_T, u_p, u_T)
            p, T = torch.empty_like(b_p), torch.empty_like(b_T)
            info = h.solve(b_p, b_T, p, T, rtol=1e-11)
            torch.cuda.synchronize()
            out[fused] = (fc[0].clone(), fc[1].clone(), p, T, info["cycles"], info["hist"])
    assert out[1][4] == out[0][4] and out[1][5] == out[0][5]
    for a, b in zip(out[1][:4], out[0][:4]):
        assert torch.equal(a, b), (a - b).abs().max().item()


@pytest.mark.parametrize("big", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
def test_coarse_single_sweep_3d_matches_reference(big, prec):
    """3-D coarse levels with one sweep on the way down only (or up only,
    PT_OPT_COARSE_SWEEPS 16 and 1) under an over-relaxed V(5,3) on the
    finest level: the fused kernels (plane-marching sweeps with stored
    faces on levels of 2^20+ cells when big) give the separate kernels'
    solution, cycles and history bit for bit, and the solve meets the
    tolerance against the oracle."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    if big:
        prob = W.bubble_problem("b3s", 3, (320, 192, 192), [(0.45, 0.5, 0.55)], [0.2], W.P0,
                                10 * W.P0, div_amp=1e-6, div_seed=14)
    else:
        prob = step_problems()["bubble3d_40x24x56"]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, gb_p, gb_T, _ = D.setup(prob, prec, stream=stream)
        h.set_option(ptmg.PT_OPT_OMEGA, 1100)
        for cs in (16, 1):
            h.set_option(ptmg.PT_OPT_COARSE_SWEEPS, cs)
            out = {}
            for fused in (1, 0):
                h.set_option(ptmg.PT_OPT_FUSED, fused)
                p, T = torch.empty_like(gb_p), torch.empty_like(gb_T)
                info = h.solve(gb_p, gb_T, p, T, rtol=1e-11, nu1=5, nu2=3, max_cycles=30)
                torch.cuda.synchronize()
                out[fused] = (p, T, info)
            (p1, T1, i1), (p0, T0, i0) = out[1], out[0]
            assert i1["status"] == i0["status"] == 0, (cs, i1["status"], i0["status"])
            assert i1["cycles"] == i0["cycles"] and i1["hist"] == i0["hist"], cs
            assert torch.equal(p1, p0) and torch.equal(T1, T0), cs
            if not big:
                op = orc.assemble(prob)
                b_p, b_T = orc.rhs(op, prob)
                assert max(orc.relres(op, b_p, b_T, host(p1), host(T1))) <= 2e-11


@pytest.mark.parametrize("nu", [(1, 1), (2, 1), (1, 2), (2, 2), (3, 2), (0, 2)])
@pytest.mark.parametrize("prec", [0, 1])
def test_coarse_half_cycles_match_reference(nu, prec):
    """2-D coarse levels run each visit of a V-cycle as one kernel (sweeps +
    residual + restriction down, prolongation + sweeps up, nu in {1, 2});
    V-cycles and solves equal the separate-kernel reference bit for bit, on
    coarse levels of several ragged tiles down to an odd coarsest grid."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = W.bubble_problem("b5", 2, (384, 320), [(0.4, 0.45)], [0.2], W.P0, 10 * W.P0,
                            div_amp=1e-6, div_seed=11)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, b_p, b_T, _ = D.setup(prob, prec, stream=stream)
        # the coarse levels take the pair under test, whatever the default
        h.set_option(ptmg.PT_OPT_COARSE_SWEEPS, 0)
        rng = np.random.default_rng(5)
        f_p, f_T = dev(rng.uniform(-1, 1, h.N)), dev(rng.uniform(-1, 1, h.N))
        out = {}
        for fused in (1, 0):
            h.set_option(ptmg.PT_OPT_FUSED, fused)
            e = h.vcycle(f_p, f_T, nu[0], nu[1])
            p, T = torch.empty_like(b_p), torch.empty_like(b_T)
            info = h.solve(b_p, b_T, p, T, rtol=1e-11, nu1=nu[0], nu2=nu[1])
            torch.cuda.synchronize()
            out[fused] = (e[0].clone(), e[1].clone(), p.clone(), T.clone(), info["cycles"])
    assert out[1][4] == out[0][4]
    for a, b in zip(out[1][:4], out[0][:4]):
        assert torch.equal(a, b), (a - b).abs().max().item()


@pytest.mark.parametrize("name", ["bubble2d_200x136", "explicit_64", "bubble3d_40x24x56"])
def test_speculation_changes_no_result(name):
    """Outer iterations enqueued ahead of the host's convergence test give
    the step-by-step loop's bits, cycles and history (zero guess, warm
    start, and a tolerance met at cycle 0)."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = step_problems()[name]
    h, b_p, b_T, _ = D.setup(prob, 1)
    out = {}
    for spec in (0, 1):
        h.set_option(ptmg.PT_OPT_SPECULATE, spec)
        assert h.get_option(ptmg.PT_OPT_SPECULATE) == spec
        p, T = torch.empty_like(b_p), torch.empty_like(b_T)
        i1 = h.solve(b_p, b_T, p, T, rtol=1e-11)
        u1 = h.last_cell_updates()
        # warm start from a rougher solution
        p2, T2 = torch.empty_like(b_p), torch.empty_like(b_T)
        h.solve(b_p, b_T, p2, T2, rtol=1e-4)
        i2 = h.solve(b_p, b_T, p2, T2, rtol=1e-11, zero_guess=False)
        # converged on arrival
        p3, T3 = p.clone(), T.clone()
        i3 = h.solve(b_p, b_T, p3, T3, rtol=1e-3, zero_guess=False)
        torch.cuda.synchronize()
        out[spec] = (p, T, i1, u1, p2, T2, i2, p3, T3, i3)
    a, b = out[0], out[1]
    for x, y in ((a[0], b[0]), (a[1], b[1]), (a[4], b[4]), (a[5], b[5]), (a[7], b[7]), (a[8], b[8])):
        assert torch.equal(x, y)
    for ia, ib in ((a[2], b[2]), (a[6], b[6]), (a[9], b[9])):
        assert ia["cycles"] == ib["cycles"] and ia["status"] == ib["status"] == 0
        assert ia["hist"] == ib["hist"]
    assert a[9]["cycles"] == 0 and torch.equal(b[7], b[0])
    assert a[3] == b[3]      # cell-updates count only the kept cycles


@pytest.mark.parametrize("prec", [0, 1])
def test_bicgstab_matches_oracle_and_helps_stiff(prec):
    """BiCGStab with the V-cycle as preconditioner: same answer as the oracle
    on a plain case and on stiff (diffusive-CFL) 2-D and 3-D cases, where it
    needs far fewer V-cycles than the defect-correction loop."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    cases = [
        step_problems()["bubble2d_200x136"],
        W.bubble_problem("st2", 2, (128, 128), [(0.5, 0.5)], [0.1], W.P0, W.P0,
                         div_amp=1e-6, div_seed=2, stiff=True),
        W.bubble_problem("st3", 3, (24, 24, 24), [(0.5, 0.5, 0.3)], [0.25], W.P0, 10 * W.P0,
                         div_amp=1e-6, div_seed=4, stiff=True),
    ]
    # with the diffusive time step the paper-form residual has a rounding
    # floor near 3e-11 in 3-D (large diffusion terms cancel), so the 3-D
    # case asks for 1e-10
    rtols = {"b2": 1e-11, "st2": 1e-11, "st3": 1e-10}
    for prob in cases:
        rtol = rtols[prob.name]
        op, b_p, b_T, p_ref, T_ref = orc.solve(prob, direct_max=40000)
        h, gb_p, gb_T, _ = D.setup(prob, prec)
        p, T = torch.empty_like(gb_p), torch.empty_like(gb_T)
        info = h.solve(gb_p, gb_T, p, T, rtol=rtol, max_cycles=80,
                       method=ptmg.PT_SOLVE_BICGSTAB)
        assert info["status"] == 0, (prob.name, info["status"])
        assert rel_err(host(p), p_ref) <= 1e-8 and rel_err(host(T), T_ref) <= 1e-8, prob.name
        rel = orc.relres(op, b_p, b_T, host(p), host(T))
        assert rel.max() <= 2 * rtol, (prob.name, rel)
        if prob.name != "b2":
            p2, T2 = torch.empty_like(gb_p), torch.empty_like(gb_T)
            dc = h.solve(gb_p, gb_T, p2, T2, rtol=rtol, max_cycles=200, raise_on_noconv=False)
            assert info["cycles"] < dc["cycles"], (prob.name, info["cycles"], dc["cycles"])
    # bitwise repeatable; the defect loop's option checks still apply
    h, gb_p, gb_T, _ = D.setup(cases[1], prec)
    outs = []
    for _ in range(2):
        p, T = torch.empty_like(gb_p), torch.empty_like(gb_T)
        h.solve(gb_p, gb_T, p, T, rtol=1e-11, max_cycles=80, method=ptmg.PT_SOLVE_BICGSTAB)
        torch.cuda.synchronize()
        outs.append((p, T))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    with pytest.raises(ptmg.PtMgError):
        h.solve(gb_p, gb_T, p, T, method=7)


@pytest.mark.parametrize("kind", ["phases", "state"])
@pytest.mark.parametrize("prec", [0, 1])
def test_step_equals_update_rhs_solve(kind, prec):
    """pt_mg_step (update + paper right-hand side + solve with one wait)
    gives the right-hand side, solution, cycle count and history of the
    three separate calls, bit for bit; an invalid field through the step
    is the update's error and leaves the handle not ready until a valid
    step."""
    import dataclasses
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    if kind == "phases":
        first = step_problems()["bubble2d_200x136"]
        second = W.bubble_problem("b2b", 2, (200, 136), [(0.55, 0.4)], [0.15], W.P0, 5 * W.P0,
                                  div_amp=1e-6, div_seed=8)
    else:
        first = W.state_problem("st1", 2, (200, 136), [(0.45, 0.5)], [0.2], seed=41)
        second = W.state_problem("st2", 2, (200, 136), [(0.5, 0.45)], [0.25], seed=42)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, _, _, _ = D.setup(first, prec, stream=stream)
        s2, t2 = D.to_device(second)
        div = t2.get("div")
        if div is None and "Us0" in t2:
            div = h.divergence(D.face_inputs(second, t2))
        # separate calls
        h.update(s2)
        b_p, b_T = h.paper_rhs(t2.get("p_adv"), t2.get("T_adv"), div)
        p1, T1 = torch.empty_like(b_p), torch.empty_like(b_T)
        i1 = h.solve(b_p, b_T, p1, T1, rtol=1e-12)
        # one call (the handle starts from the first problem again)
        s1, t1 = D.to_device(first)
        h.update(s1)
        c_p, c_T = torch.empty_like(b_p), torch.empty_like(b_T)
        p2, T2 = torch.empty_like(b_p), torch.empty_like(b_T)
        i2 = h.step(s2, div, c_p, c_T, p2, T2, rtol=1e-12)
        torch.cuda.synchronize()
        assert i1["cycles"] == i2["cycles"] and i1["hist"] == i2["hist"]
        for a, b in ((b_p, c_p), (b_T, c_T), (p1, p2), (T1, T2)):
            assert torch.equal(a, b)
        # an invalid volume fraction: the update's error, then not ready
        bad = dataclasses.replace(second, C=np.where(second.C > 0.5, 1.5, second.C))
        sb, tb = D.to_device(bad) if kind == "phases" else (None, None)
        if kind == "phases":
            with pytest.raises(ptmg.PtMgError) as e:
                h.step(sb, div, c_p, c_T, p2, T2, rtol=1e-12)
            assert e.value.status == ptmg.PT_ERR_ARG
            with pytest.raises(ptmg.PtMgError) as e:
                h.solve(b_p, b_T, p2, T2)
            assert e.value.status == ptmg.PT_ERR_STATE
            i3 = h.step(s2, div, c_p, c_T, p2, T2, rtol=1e-12)
            torch.cuda.synchronize()
            assert i3["cycles"] == i1["cycles"] and torch.equal(p1, p2)
        ex = W.explicit_const(32, 32)
        se, _ = D.to_device(ex)
        with pytest.raises(ptmg.PtMgError) as e:
            h.step(se, None, c_p, c_T, p2, T2)
        assert e.value.status == ptmg.PT_ERR_STATE


@pytest.mark.parametrize("prec", [0, 1])
def test_tail_cap_changes_no_result(prec):
    """Capping the single-block tail moves its upper levels to the grid
    kernels: fewer tail levels, the same solution and V-cycle bit for bit."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    # levels of 122880, 30720, 7680, 1920, 480, 120 and 30 cells
    prob = W.bubble_problem("b6", 2, (384, 320), [(0.4, 0.45)], [0.2], W.P0, 10 * W.P0,
                            div_amp=1e-6, div_seed=12)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, b_p, b_T, _ = D.setup(prob, prec, stream=stream)
        rng = np.random.default_rng(12)
        f_p, f_T = dev(rng.uniform(-1, 1, h.N)), dev(rng.uniform(-1, 1, h.N))
        out, levels = {}, {}
        for cap in (0, 480, 120, 16):
            h.set_option(ptmg.PT_OPT_TAIL_CELLS, cap)
            assert h.get_option(ptmg.PT_OPT_TAIL_CELLS) == cap
            levels[cap] = h.get_option(ptmg.PT_OPT_TAIL)
            p, T = torch.empty_like(b_p), torch.empty_like(b_T)
            h.solve(b_p, b_T, p, T, rtol=1e-12)
            e = h.vcycle(f_p, f_T)
            torch.cuda.synchronize()
            out[cap] = (p.clone(), T.clone(), e[0].clone(), e[1].clone())
        with pytest.raises(ptmg.PtMgError):
            h.set_option(ptmg.PT_OPT_TAIL_CELLS, -1)
    assert levels[0] >= levels[480] == 3 and levels[120] == 2 and levels[16] == 0
    for cap in (480, 120, 16):
        for a, b in zip(out[0], out[cap]):
            assert torch.equal(a, b), (a - b).abs().max().item()


def test_coarse_sweeps_option():
    """PT_OPT_COARSE_SWEEPS: by default the solve's own counts on every
    level; other settings change the V-cycle but the solve still meets the
    tolerance against the oracle; invalid values are refused."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = step_problems()["bubble2d_200x136"]
    op, b_p, b_T, p_ref, T_ref = orc.solve(prob)
    h, gb_p, gb_T, _ = D.setup(prob, 0)
    assert h.get_option(ptmg.PT_OPT_COARSE_SWEEPS) == 0
    hists = {}
    for v in (0, 17, 33, 16 * 2 + 1):
        h.set_option(ptmg.PT_OPT_COARSE_SWEEPS, v)
        p, T = torch.empty_like(gb_p), torch.empty_like(gb_T)
        info = h.solve(gb_p, gb_T, p, T, rtol=1e-12)
        assert info["status"] == 0
        assert max(orc.relres(op, b_p, b_T, host(p), host(T))) <= 2e-12
        hists[v] = info["hist"]
    assert hists[17] != hists[0]
    for bad in (-1, 9 * 16, 9, 256):
        with pytest.raises(ptmg.PtMgError):
            h.set_option(ptmg.PT_OPT_COARSE_SWEEPS, bad)


@pytest.mark.parametrize("prec", [0, 1])
def test_w_levels_match_oracle_and_help_stiff(prec):
    """PT_OPT_W_LEVELS: two coarse corrections per visit on the levels above
    the tail.  On stiff (diffusive-CFL) 2-D and 3-D steps the solve gives
    the oracle's answer in fewer cycles than the V-cycle; the fused and the
    separate kernels, and graph replay and direct launches, give the same
    bits; negative values are refused."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    # (problem, rtol, largest tail level): the 3-D grid keeps its tail to
    # 3^3 cells so that two levels run as a W-cycle; with the diffusive
    # step the 3-D paper-form residual has a rounding floor near 3e-11
    cases = [
        (W.bubble_problem("w2", 2, (256, 256), [(0.5, 0.5)], [0.1], W.P0, W.P0,
                          div_amp=1e-6, div_seed=2, stiff=True), 1e-11, 0),
        (W.bubble_problem("w3", 3, (24, 24, 24), [(0.5, 0.5, 0.3)], [0.25], W.P0, 10 * W.P0,
                          div_amp=1e-6, div_seed=4, stiff=True), 1e-10, 27),
    ]
    for prob, rtol, tail_cells in cases:
        op, b_p, b_T, p_ref, T_ref = orc.solve(prob, direct_max=70000)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            h, gb_p, gb_T, _ = D.setup(prob, prec, stream=stream)
            h.set_option(ptmg.PT_OPT_TAIL_CELLS, tail_cells)
            assert h.get_option(ptmg.PT_OPT_W_LEVELS) == 0
            cyc = {}
            for w in (0, 8):
                h.set_option(ptmg.PT_OPT_W_LEVELS, w)
                p, T = torch.empty_like(gb_p), torch.empty_like(gb_T)
                info = h.solve(gb_p, gb_T, p, T, rtol=rtol, max_cycles=200)
                assert info["status"] == 0, (prob.name, w, info["status"])
                P, Tt = host(p), host(T)
                assert rel_err(P, p_ref) <= 1e-8 and rel_err(Tt, T_ref) <= 1e-8, (prob.name, w)
                assert orc.relres(op, b_p, b_T, P, Tt).max() <= 2 * rtol, (prob.name, w)
                cyc[w] = info["cycles"]
            assert cyc[8] < cyc[0], (prob.name, cyc)
            # the same W-cycle through the other paths
            ref = None
            for fused, graphs in ((1, 0), (0, 0), (1, 1)):
                h.set_option(ptmg.PT_OPT_FUSED, fused)
                h.set_option(ptmg.PT_OPT_GRAPHS, graphs)
                p, T = torch.empty_like(gb_p), torch.empty_like(gb_T)
                info = h.solve(gb_p, gb_T, p, T, rtol=rtol, max_cycles=200)
                torch.cuda.synchronize()
                out = (p.clone(), T.clone(), info["cycles"])
                if ref is None:
                    ref = out
                else:
                    assert out[2] == ref[2] and torch.equal(out[0], ref[0]) and \
                        torch.equal(out[1], ref[1]), (prob.name, fused, graphs)
            with pytest.raises(ptmg.PtMgError):
                h.set_option(ptmg.PT_OPT_W_LEVELS, -1)


@pytest.mark.parametrize("name", ["bubble2d_200x136", "bubble3d_40x24x56", "explicit_64",
                                  "twobubble2d_96x80"])
@pytest.mark.parametrize("prec", [0, 1])
def test_small_hierarchy_kernel_matches_reference(name, prec):
    """The small end of the hierarchy (levels of at most 1024 cells, the
    coarsest matrix and its inverse) built by one single-block kernel on
    the fused path equals the separate kernels (PT_OPT_FUSED off) bit for
    bit: every level's operator and a whole solve."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = step_problems()[name]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, b_p, b_T, t = D.setup(prob, prec, stream=stream)
        s2, t2 = D.to_device(prob)
        nl = h.num_levels()
        out = {}
        for fused in (1, 0):
            h.set_option(ptmg.PT_OPT_FUSED, fused)
            h.update(s2, keepalive=t2)      # the hierarchy rebuilt on this path
            ops = [tuple(x.clone() for x in h.get_operator(l)) for l in range(1, nl)]
            p, T = torch.empty_like(b_p), torch.empty_like(b_T)
            h.set_option(ptmg.PT_OPT_FUSED, 1)
            info = h.solve(b_p, b_T, p, T, rtol=1e-12)
            torch.cuda.synchronize()
            assert info["status"] == 0
            out[fused] = (ops, p.clone(), T.clone(), info["hist"])
    (o1, p1, T1, h1), (o0, p0, T0, h0) = out[1], out[0]
    for l, (a, b) in enumerate(zip(o1, o0), start=1):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), l
    assert torch.equal(p1, p0) and torch.equal(T1, T0) and h1 == h0


def test_vcycle_h_independent_on_constant_family():
    """The 2-D constant-coefficient case (alpha_p = 1, alpha_T = 0.1,
    B = [[1, 0.3], [0.2, 1]]/dt, seeded f) at N = 64 ... 1024: the V(2,2)
    cycle's contraction per cycle stays bounded and the cycles to 1e-10
    stay within two of each other as h halves four times (multigrid's
    h-independence; the paper prints no iteration counts, so the bound is
    this library's own record)."""
    import workloads.device as D
    rec = []
    for n in (64, 128, 256, 512, 1024):
        prob = W.explicit_const(n, n)
        h, b_p, b_T, _ = D.setup(prob, 0)
        p, T = torch.empty_like(b_p), torch.empty_like(b_T)
        info = h.solve(b_p, b_T, p, T, rtol=1e-10, max_cycles=40)
        assert info["status"] == 0, n
        hist = np.array(info["hist"]).max(axis=1)
        rates = hist[2:] / hist[1:-1]       # steady contraction after the first cycle
        rec.append((n, info["cycles"], float(rates.max()) if rates.size else 0.0))
        print(f"# constant family N={n}: cycles {info['cycles']}, "
              f"contraction {rec[-1][2]:.2e}", flush=True)
        h.destroy()
    cycles = [c for _, c, _ in rec]
    assert max(cycles) - min(cycles) <= 2, rec
    assert max(r for _, _, r in rec) <= 0.1, rec


def _blocking_and_async(h, b_p, b_T, rtol, max_cycles, zero_guess=True, p0=None, T0=None):
    """The blocking solve and the stream-ordered one on the same handle, from
    the same start; returns both (p, T, info)."""
    out = []
    for mode in ("block", "async"):
        p = torch.empty_like(b_p) if p0 is None else p0.clone()
        T = torch.empty_like(b_T) if T0 is None else T0.clone()
        if mode == "block":
            info = h.solve(b_p, b_T, p, T, rtol=rtol, max_cycles=max_cycles,
                           zero_guess=zero_guess, raise_on_noconv=False)
        else:
            pend = h.solve_async(b_p, b_T, p, T, rtol=rtol, max_cycles=max_cycles,
                                 zero_guess=zero_guess)
            torch.cuda.synchronize()
            info = pend.result()
        out.append((p, T, info))
    return out


@pytest.mark.parametrize("name", ["bubble2d_200x136", "bubble3d_40x24x56"])
def test_answer_residual_is_the_reported_one(name):
    """Mixed precision from a zero guess keeps the first iterate (the FP32
    correction itself) as FP32 pairs in its buffer's memory: whether a
    solve stops after one cycle (the pairs in the caller's own p array or
    in the handle's buffer, by the parity the last solve left) or two, the
    residual of the returned answer is the one the solve reported, bit for
    bit, blocking and stream-ordered."""
    import workloads.device as D
    prob = step_problems()[name]
    h, b_p, b_T, _ = D.setup(prob, 1)
    p, T = torch.empty_like(b_p), torch.empty_like(b_T)
    tight = h.solve(b_p, b_T, p, T, rtol=1e-12)
    assert tight["cycles"] >= 2
    loose = 2.0 * max(tight["hist"][1])   # met after the first cycle
    for rtol, cycles in ((loose, 1), (loose, 1), (1e-12, tight["cycles"]), (loose, 1)):
        for (pa, Ta, info) in _blocking_and_async(h, b_p, b_T, rtol, 20):
            torch.cuda.synchronize()
            assert info["status"] == 0 and info["cycles"] == cycles
            _, _, rel = h.residual(b_p, b_T, pa, Ta, want_fields=False)
            assert rel == tuple(info["relres"]), (rtol, rel, info["relres"])


@pytest.mark.parametrize("prec", [0, 1])
def test_async_solve_equals_blocking(prec):
    """The stream-ordered solve (opts.async): the stop test on the device,
    every later launch a no-op, the answer moved into (p, T) by the stream,
    the record written by a host function.  Same bits, cycles, history and
    status as the blocking solve: 2-D and 3-D, a warm start, the mean
    constraint, max_cycles reached, and three solves enqueued back to back
    before one synchronisation."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    for name in ("bubble2d_200x136", "bubble3d_40x24x56"):
        prob = step_problems()[name]
        h, b_p, b_T, _ = D.setup(prob, prec)
        (p1, T1, i1), (p2, T2, i2) = _blocking_and_async(h, b_p, b_T, 1e-11, 12)
        assert i1["status"] == 0 and i2["status"] == 0, (name, i1["status"], i2["status"])
        assert i2["cycles"] == i1["cycles"] and i2["hist"] == i1["hist"], name
        assert torch.equal(p1, p2) and torch.equal(T1, T2), name
        # warm start from a perturbed answer; and a cap below the cycles needed
        (p1, T1, i1), (p2, T2, i2) = _blocking_and_async(
            h, b_p, b_T, 1e-12, 12, zero_guess=False, p0=p1 * (1 + 1e-9), T0=T1)
        assert i2["cycles"] == i1["cycles"] and torch.equal(p1, p2) and torch.equal(T1, T2)
        (p1, T1, i1), (p2, T2, i2) = _blocking_and_async(h, b_p, b_T, 1e-14, 1)
        assert i1["status"] == ptmg.PT_ERR_NOCONV and i2["status"] == ptmg.PT_ERR_NOCONV
        assert i2["cycles"] == i1["cycles"] == 1 and i2["hist"] == i1["hist"]
        assert torch.equal(p1, p2) and torch.equal(T1, T2)
        # three right-hand sides enqueued back to back, one synchronisation
        rhs = [(b_p * s, b_T * s) for s in (1.0, 0.5, 2.0)]
        ref = []
        for bp, bT in rhs:
            p, T = torch.empty_like(b_p), torch.empty_like(b_T)
            ref.append((p, T, h.solve(bp, bT, p, T, rtol=1e-11, max_cycles=12)))
        outs, pends = [], []
        for bp, bT in rhs:
            p, T = torch.empty_like(b_p), torch.empty_like(b_T)
            pends.append(h.solve_async(bp, bT, p, T, rtol=1e-11, max_cycles=12))
            outs.append((p, T))
        torch.cuda.synchronize()
        for (p, T), pend, (pr, Tr, ir) in zip(outs, pends, ref):
            inf = pend.result()
            assert inf["cycles"] == ir["cycles"] and inf["hist"] == ir["hist"]
            assert torch.equal(p, pr) and torch.equal(T, Tr)
    # the mean constraint (pure Neumann Poisson): the final shift is stream-ordered too
    n = (80, 48)
    N = n[0] * n[1]
    rng = np.random.default_rng(1)
    prob = W.Problem(name="poisson", dim=2, n=(80, 48, 1), h=1.0 / 80, mode="explicit",
                     alpha_p=1.0, alpha_T=0.25, B_const=(0.0, 0.0, 0.0, 0.0),
                     f_p=rng.uniform(-1, 1, N), f_T=rng.uniform(-1, 1, N), mean_constraint=True)
    h, b_p, b_T, _ = D.setup(prob, prec)
    (p1, T1, i1), (p2, T2, i2) = _blocking_and_async(h, b_p, b_T, 1e-11, 60)
    assert i1["status"] == 0 and i2["status"] == 0
    assert torch.equal(p1, p2) and torch.equal(T1, T2)
    # refused where it does not apply
    p, T = torch.empty_like(b_p), torch.empty_like(b_T)
    for kw in ({"max_cycles": ptmg.PT_MAX_HIST}, ):
        with pytest.raises(ptmg.PtMgError):
            h.solve_async(b_p, b_T, p, T, **kw)
    opts = ptmg.pt_solve_opts(1e-9, 10, 2, 2, 1, ptmg.PT_SOLVE_BICGSTAB, 1)
    info = ptmg.pt_solve_info()
    rc = ptmg.lib().pt_mg_solve(h._h, ptmg._ptr(b_p), ptmg._ptr(b_T), ptmg._ptr(p),
                                ptmg._ptr(T), ctypes.byref(opts), ctypes.byref(info))
    assert rc == ptmg.PT_ERR_ARG
    opts.method = ptmg.PT_SOLVE_DEFECT
    rc = ptmg.lib().pt_mg_solve_noalloc(h._h, ptmg._ptr(b_p), ptmg._ptr(b_T), ptmg._ptr(p),
                                        ptmg._ptr(T), ctypes.byref(opts), ctypes.byref(info))
    assert rc == ptmg.PT_ERR_ARG


@pytest.mark.parametrize("name", ["bubble2d_200x136", "bubble3d_40x24x56", "explicit_64"])
@pytest.mark.parametrize("prec", [0, 1])
def test_over_relaxation_fused_equals_reference(name, prec):
    """PT_OPT_OMEGA (over-relaxed finest-level sweeps): the fused sweeps and
    transfers give the separate kernels' solution, cycles and residual
    history bit for bit (PT_OPT_FUSED off), at V(3,2) and V(4,4) and from a
    zero guess (whose first sweep reads no iterate); the solve meets the
    tolerance against the oracle's own right-hand side; omega = 1 is the
    plain update; values outside 1..1999 are refused."""
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    prob = step_problems()[name]
    op = orc.assemble(prob)
    b_p, b_T = orc.rhs(op, prob)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        h, gb_p, gb_T, _ = D.setup(prob, prec, stream=stream)
        assert h.get_option(ptmg.PT_OPT_OMEGA) == 1000
        plain = h.solve(gb_p, gb_T, torch.empty_like(gb_p), torch.empty_like(gb_T),
                        rtol=1e-11, max_cycles=60)
        h.set_option(ptmg.PT_OPT_OMEGA, 1000)
        again = h.solve(gb_p, gb_T, torch.empty_like(gb_p), torch.empty_like(gb_T),
                        rtol=1e-11, max_cycles=60)
        assert again["hist"] == plain["hist"]
        h.set_option(ptmg.PT_OPT_OMEGA, 1100)
        for nu in ((3, 2), (4, 4)):
            out = {}
            for fused in (1, 0):
                h.set_option(ptmg.PT_OPT_FUSED, fused)
                p, T = torch.empty_like(gb_p), torch.empty_like(gb_T)
                info = h.solve(gb_p, gb_T, p, T, rtol=1e-11, nu1=nu[0], nu2=nu[1],
                               max_cycles=60)
                torch.cuda.synchronize()
                out[fused] = (p.clone(), T.clone(), info)
            (p1, T1, i1), (p0, T0, i0) = out[1], out[0]
            assert i1["status"] == i0["status"] == 0, (nu, i1["status"], i0["status"])
            assert i1["cycles"] == i0["cycles"] and i1["hist"] == i0["hist"], nu
            assert torch.equal(p1, p0) and torch.equal(T1, T0), nu
            assert max(orc.relres(op, b_p, b_T, host(p1), host(T1))) <= 2e-11
            assert i1["hist"] != plain["hist"]
        for bad in (0, 2000, -5):
            with pytest.raises(ptmg.PtMgError):
                h.set_option(ptmg.PT_OPT_OMEGA, bad)
