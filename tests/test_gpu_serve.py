"""The continuous-batching serving engine (pt_serve.h): every result is the
same bits alone and in the mix, admission by footprint queues instead of
failing, a poisoned request fails with its own status while the others
complete, and served results match the oracle."""
import numpy as np
import pytest

import oracle as orc
import workloads as W
from gpu_util import host, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES2D = [96, 128, 160, 192]
SIZES3D = [32, 40, 48]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _requests(ids):
    return [W.serve_request(i, SIZES2D, SIZES3D) for i in ids]


def _alone(prob, rtol):
    import workloads.device as D
    h, b_p, b_T, _ = D.setup(prob, 1)
    p, T = torch.empty_like(b_p), torch.empty_like(b_T)
    info = h.solve(b_p, b_T, p, T, rtol=rtol)
    return p, T, info


def _submit_all(srv, probs, rtol, t0=None):
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    out = []
    for prob in probs:
        s, t = D.to_device(prob)
        p = torch.empty(prob.ncells, dtype=torch.float64, device="cuda")
        T = torch.empty_like(p)
        rid = srv.submit(s, ptmg.PT_PREC_MIXED, p, T, div=t.get("div"), rtol=rtol, keepalive=t)
        out.append((rid, p, T, prob))
    return out


def _largest():
    """Requests of the serving mix's largest sizes, 2048^2 and 192^3: the
    first ids of each dimension drawn with only those sizes allowed."""
    out = {}
    rid = 100
    while len(out) < 2:
        pr = W.serve_request(rid, [2048], [192])
        out.setdefault(pr.dim, pr)
        rid += 1
    return [out[2], out[3]]


def test_results_identical_alone_and_in_the_mix():
    """Twelve small requests and the mix's largest two (2048^2, 192^3)."""
    from paper_2206_11294_amd import serve
    probs = _requests(range(6)) + _largest() + _requests(range(6, 12))
    assert {p.dim for p in probs} == {2, 3}
    assert max(p.ncells for p in probs if p.dim == 2) == 2048 ** 2
    assert max(p.ncells for p in probs if p.dim == 3) == 192 ** 3
    alone = [_alone(p, 1e-10) for p in probs]
    srv = serve.Server(hbm_budget=8 << 30, max_active=6)
    reqs = _submit_all(srv, probs, 1e-10)
    srv.run_until_idle()
    torch.cuda.synchronize()
    overlapped = 0
    infos = [srv.request(r[0]) for r in reqs]
    for (rid, p, T, prob), info, (pa, Ta, ia) in zip(reqs, infos, alone):
        assert info["status"] == 0, info
        assert info["cycles"] == ia["cycles"]
        assert torch.equal(p, pa) and torch.equal(T, Ta), prob.name
    # requests were on the device together
    for a in infos:
        if any(b is not a and b["t_admit"] < a["t_done"] and a["t_admit"] < b["t_done"] for b in infos):
            overlapped += 1
    assert overlapped >= 2
    srv.destroy()


def test_admission_by_footprint_queues():
    """A budget that holds about two requests: all complete, never more
    bytes in use than the budget, and an oversize request fails alone."""
    from paper_2206_11294_amd import ptmg, serve
    import workloads.device as D
    probs = _requests(range(20, 30))
    sizes = []
    for pr in probs:
        s, _ = D.to_device(pr)
        sizes.append(ptmg.footprint_bytes(s, ptmg.PT_PREC_MIXED))
    budget = int(2.2 * max(sizes))
    srv = serve.Server(hbm_budget=budget, max_active=8)
    big = W.bubble_problem("big", 3, (128, 128, 128), [(0.5, 0.5, 0.5)], [0.2], W.P0, 10 * W.P0)
    reqs = _submit_all(srv, probs[:5] + [big] + probs[5:], 1e-9)
    peak = 0
    while True:
        n = srv.progress(serve.now() + 0.0005)
        st = srv.stats()
        peak = max(peak, st["bytes"])
        assert st["bytes"] <= budget
        if st["queued"] == 0 and st["active"] == 0:
            break
    for rid, p, T, prob in reqs:
        info = srv.request(rid)
        if prob.name == "big":
            assert info["status"] == ptmg.PT_ERR_OOM
        else:
            assert info["status"] == 0, (prob.name, info)
    assert peak > max(sizes)          # more than one request was admitted at once
    srv.destroy()


def test_poisoned_requests_fail_alone():
    from paper_2206_11294_amd import ptmg, serve
    import workloads.device as D
    good = _requests(range(40, 44))
    bad_C = W.serve_request(44, SIZES2D, SIZES3D)
    C = bad_C.C.copy()
    C.reshape(-1)[3] = -0.5
    bad_C = W.Problem(**{**bad_C.__dict__, "C": C})
    srv = serve.Server(hbm_budget=4 << 30, max_active=4)
    reqs = _submit_all(srv, [good[0], bad_C, good[1]], 1e-9)
    # a request that cannot converge in one cycle
    s, t = D.to_device(good[2])
    p = torch.empty(good[2].ncells, dtype=torch.float64, device="cuda")
    T = torch.empty_like(p)
    rid_nc = srv.submit(s, ptmg.PT_PREC_MIXED, p, T, rtol=1e-14, max_cycles=1, keepalive=t)
    # a request with a NaN in its velocity divergence
    s3, t3 = D.to_device(good[3])
    div = torch.zeros(good[3].ncells, dtype=torch.float64, device="cuda")
    div[17] = float("nan")
    p3 = torch.empty_like(div)
    T3 = torch.empty_like(div)
    rid_nan = srv.submit(s3, ptmg.PT_PREC_MIXED, p3, T3, div=div, keepalive=(t3, div))
    srv.run_until_idle()
    st = {rid: srv.request(rid)["status"] for rid, *_ in reqs}
    assert st[reqs[0][0]] == 0 and st[reqs[2][0]] == 0
    assert st[reqs[1][0]] == ptmg.PT_ERR_ARG
    assert srv.request(rid_nc)["status"] == ptmg.PT_ERR_NOCONV
    assert srv.request(rid_nan)["status"] == ptmg.PT_ERR_NOCONV
    assert srv.stats()["bytes"] == 0
    srv.destroy()


def test_served_results_match_oracle():
    from paper_2206_11294_amd import serve
    probs = [p for p in _requests(range(60, 70)) if p.ncells <= 40000][:3]
    assert probs
    srv = serve.Server(hbm_budget=2 << 30, max_active=3)
    reqs = _submit_all(srv, probs, 1e-12)
    srv.run_until_idle()
    for rid, p, T, prob in reqs:
        assert srv.request(rid)["status"] == 0
        op, b_p, b_T, p_ref, T_ref = orc.solve(prob, rtol=1e-14, direct_max=0)
        assert rel_err(host(p), p_ref) <= 1e-8 and rel_err(host(T), T_ref) <= 1e-8
    srv.destroy()


def test_rz_and_state_requests_in_the_mix():
    """Axisymmetric and state-mode requests ride the same engine: each
    result is the same bits as the request solved alone."""
    import dataclasses
    from paper_2206_11294_amd import serve
    rng = np.random.default_rng(3)
    probs = _requests(range(40, 44))
    rz = [dataclasses.replace(W.serve_request(i, SIZES2D, [32]), axisymmetric=True)
          for i in range(50, 60)]
    probs += [p for p in rz if p.dim == 2][:2]
    st = W.state_problem("srv_state", 2, (128, 96), [(0.5, 0.5)], [0.2], seed=44)
    st = dataclasses.replace(st, uf_star=None,
                             div_ustar=(1e-6 / st.dt) * rng.uniform(-1, 1, st.C.shape))
    probs.append(st)
    assert sum(p.axisymmetric for p in probs) == 2
    alone = [_alone(p, 1e-10) for p in probs]
    srv = serve.Server(hbm_budget=8 << 30, max_active=6)
    reqs = _submit_all(srv, probs, 1e-10)
    srv.run_until_idle()
    torch.cuda.synchronize()
    for (rid, p, T, prob), (pa, Ta, ia) in zip(reqs, alone):
        info = srv.request(rid)
        assert info["status"] == 0, (prob.name, info)
        assert info["cycles"] == ia["cycles"]
        assert torch.equal(p, pa) and torch.equal(T, Ta), prob.name
    srv.destroy()
