"""pt_mg_solve_noalloc: the solve that allocates nothing (its BiCGStab work
vectors live in the library's static per-GPU scratch) against pt_mg_solve,
the entry point it varies.  Same kernels on the same inputs, so the bar is
bit-for-bit equality of the solution, the cycle count and the residual
history, on two calls in a row (the second on a smaller grid, so that the
scratch holds the first call's vectors), plus the oracle's residual of the
answer, the size limit, and no change of the device's free memory."""
import ctypes

import numpy as np
import pytest

import oracle as orc
import workloads as W
from gpu_util import host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _stiff(name, dim, n, centre, radius, seed):
    return W.bubble_problem(name, dim, n, [centre], [radius], W.P0, 10 * W.P0,
                            div_amp=1e-6, div_seed=seed, stiff=True)


def _pair(h, gb_p, gb_T, rtol, method, noalloc):
    from paper_2206_11294_amd import ptmg  # noqa: F401
    p, T = torch.full_like(gb_p, 7.0), torch.full_like(gb_T, -3.0)
    info = h.solve(gb_p, gb_T, p, T, rtol=rtol, max_cycles=120, method=method, noalloc=noalloc)
    torch.cuda.synchronize()
    return p, T, info


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_equals_solve_two_calls(prec):
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    big = _stiff("na_big", 2, (176, 144), (0.45, 0.5), 0.15, 11)
    small = _stiff("na_small", 3, (20, 16, 24), (0.5, 0.5, 0.4), 0.3, 12)
    for prob, rtol in ((big, 1e-11), (small, 1e-10)):   # the smaller grid second
        print(f"# noalloc prec={prec} {prob.name} {prob.n}", flush=True)
        h, gb_p, gb_T, _ = D.setup(prob, prec)
        for method in (ptmg.PT_SOLVE_BICGSTAB, ptmg.PT_SOLVE_DEFECT):
            p0, T0, i0 = _pair(h, gb_p, gb_T, rtol, method, noalloc=True)
            p1, T1, i1 = _pair(h, gb_p, gb_T, rtol, method, noalloc=False)
            assert i0["status"] == i1["status"] == 0, (prob.name, method)
            assert torch.equal(p0, p1) and torch.equal(T0, T1), (prob.name, method)
            assert i0["cycles"] == i1["cycles"] and i0["hist"] == i1["hist"]
            op = orc.assemble(prob)
            b_p, b_T = orc.rhs(op, prob)
            assert orc.relres(op, b_p, b_T, host(p0), host(T0)).max() <= 2 * rtol
        h.destroy()


def test_noalloc_size_limit_and_no_allocation():
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    assert ptmg.PT_SCRATCH_MAX_CELLS == 1 << 20
    # a grid 6 % larger than the scratch (17 * 2^6 columns, so that it
    # coarsens): rejected before any work
    over = _stiff("na_over", 2, (1088, 1024), (0.5, 0.5), 0.1, 13)
    h, gb_p, gb_T, _ = D.setup(over, 1)
    p, T = torch.full_like(gb_p, 5.0), torch.full_like(gb_T, 6.0)
    with pytest.raises(ptmg.PtMgError) as e:
        h.solve(gb_p, gb_T, p, T, method=ptmg.PT_SOLVE_BICGSTAB, noalloc=True)
    assert e.value.status == ptmg.PT_ERR_ARG and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((p == 5.0).all()) and bool((T == 6.0).all())
    h.destroy()
    # the largest grid that fits: the solve takes no device memory, while
    # pt_mg_solve's first BiCGStab call allocates 128 bytes per cell
    fit = _stiff("na_fit", 2, (1024, 1024), (0.5, 0.5), 0.1, 14)
    h, gb_p, gb_T, _ = D.setup(fit, 1)
    p, T = torch.empty_like(gb_p), torch.empty_like(gb_T)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    a = h.solve(gb_p, gb_T, p, T, rtol=1e-11, max_cycles=120, method=ptmg.PT_SOLVE_BICGSTAB,
                noalloc=True)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    pa, Ta = p.clone(), T.clone()
    b = h.solve(gb_p, gb_T, p, T, rtol=1e-11, max_cycles=120, method=ptmg.PT_SOLVE_BICGSTAB)
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    work = 128 * fit.ncells
    assert free0 - free1 < work // 4, (free0, free1)
    assert free1 - free2 >= work, (free1, free2)
    assert a["status"] == b["status"] == 0 and a["cycles"] == b["cycles"]
    assert torch.equal(pa, p) and torch.equal(Ta, T)
    h.destroy()
