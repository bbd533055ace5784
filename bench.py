#!/usr/bin/env python3
"""Benchmark of the coupled pressure-temperature multigrid solve on one GPU.

One step = one pass of the whole hot path over one synthetic input:
re-assembly of the operator and hierarchy, the paper's right-hand side
and the solve to tolerance (one pt_mg_step call; pt_mg_update +
pt_mg_solve for the explicit case), with every input already resident in
device memory.  The
state-mode workloads (state2d_1024, state3d_256) cover the implicit part
of the time step from the advected conserved variables to the updated
ones: the provisional pressure and temperature (pt_state_eval, Eqs. 20
and 23) feed the state-mode assembly, div u* comes from the provisional
face velocities (pt_mg_divergence), and after the solve the velocity
correction and the phase energy update (pt_mg_downstream, Eqs. unp1,
37-39) consume it.

The default workload is the largest single-GPU one: the 512^3 collapse-
like field (a sphere of radius 0.25 with gas at 0.01 p0 in liquid at
100 p0), solved with the FP32 V-cycle under FP64 iterative refinement.
For the mixed-precision workloads the same steps are then timed with the
plain FP64 V-cycle at the same size and tolerance, and reported beside.

Prints one JSON line: cell-updates/s of the timed steps, the roofline of
the dominant kernel (HIP-event durations of its launches inside the timed
region, algorithmic bytes per launch), the FP64 comparison, and the CPU
leg: the FP64 oracle timed on the host on a bounded sample of the same
workload, and the oracle's own residual of the last GPU solution.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision fp64|mixed]
  python bench.py --copy-calib BYTES    # plain copy kernel (counter calibration)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak
# The roofline kernel: the finest-grid fused red-black sweep, the kernel
# that moves the most bytes per V-cycle.
ROOFLINE_KERNEL = "smooth_fine"

# name -> (constructor, default precision, rtol)
WORKLOADS = {
    "explicit_64": ("explicit_const", "fp64", 1e-10),
    "bubble2d_1024": ("bubble2d", "fp64", 1e-12),
    "wall3d_256": ("wall3d", "mixed", 1e-12),
    "collapse3d_512": ("collapse3d", "mixed", 1e-12),
    "state2d_1024": ("state2d", "fp64", 1e-12),
    "state3d_256": ("state3d", "mixed", 1e-12),
    "axi2d_1024": ("axi2d", "fp64", 1e-12),
}

# Smoothing per acoustic workload: (nu1, nu2) on the finest level and
# 16 nu1 + nu2 below it (PT_OPT_COARSE_SWEEPS), and the over-relaxation of
# the finest level's sweeps (PT_OPT_OMEGA, in thousandths), each the setting
# that reached the tolerance in the least time per step when measured.
# Over-relaxed by 1.1 (the 3-D state step: 1.15) the finest sweeps take
# the solves from three cycles to two.  In 3-D the coarse levels take one
# sweep on the way down only (16): the acoustic operator is strongly
# diagonal, so a second coarse sweep changes no residual and costs a
# sweep of the 1/8-size level 1; 2-D keeps one each way, which runs each
# coarse visit as one kernel.  Whether a solve takes one
# cycle more or less sits on a threshold of the contraction, so the best
# setting moves between workloads.  Diffusive (--stiff) steps use the
# library's default V(2,2) on every level and omega = 1: one coarse sweep
# each way costs them cycles.
SWEEPS = {
    "explicit_64": (3, 2, 34),
    "bubble2d_1024": (4, 3, 17),
    "wall3d_256": (4, 3, 16),
    "collapse3d_512": (5, 3, 16),
    "state2d_1024": (4, 3, 17),
    "state3d_256": (4, 4, 16),
    "axi2d_1024": (5, 3, 17),
}
OMEGA = {
    "bubble2d_1024": 1100,
    "wall3d_256": 1100,
    "collapse3d_512": 1100,
    "state2d_1024": 1100,
    "state3d_256": 1150,
    "axi2d_1024": 1100,
}


def make_problem(name, stiff=False):
    import workloads as W
    if stiff and name not in ("bubble2d_1024", "wall3d_256"):
        raise SystemExit("--stiff applies to bubble2d_1024 and wall3d_256")
    if name == "explicit_64":
        return W.explicit_const(64, 64)
    if name == "bubble2d_1024":
        return W.bubble2d(1024, stiff=stiff)
    if name == "wall3d_256":
        return W.wall3d(256, stiff=stiff)
    if name == "collapse3d_512":
        return W.collapse3d(512)
    if name == "state2d_1024":
        return W.state2d(1024)
    if name == "state3d_256":
        return W.state3d(256)
    if name == "axi2d_1024":
        return W.axi2d(1024)
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash():
    """Hash of the files that hold the kernels and their launch shapes."""
    h = hashlib.sha256()
    for f in ("ptmg_kernels.hip", "ptmg_internal.h"):
        with open(os.path.join(ROOT, "paper_2206_11294_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload, kernel_class, launches_per_step):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counter summaries, when they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash() or rec.get("kernel_class") != kernel_class:
        return None
    return rec.get("hbm_bytes_per_launch")


def upstream_line(prob, state_ms):
    """Achieved bandwidth of the provisional-state kernel (state mode):
    per cell it reads C, m1, m2, E and dim momentum components and writes
    p_adv, T_adv, all float64, once."""
    if not state_ms:
        return None
    nbytes = prob.ncells * 8.0 * (4 + prob.dim + 2)
    ms = sum(state_ms) / len(state_ms)
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"kernel": "pt_state_eval", "bound": "hbm", "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "avg_launch_us": round(ms * 1e3, 2), "alg_bytes_per_launch": nbytes,
            "launches": len(state_ms)}


def transfer_sweep_line(timed):
    """The finest-grid sweep that also restricts its residual (or adds the
    prolonged correction), timed apart from the plain sweeps: algorithmic
    bytes are the sweep's plus the coarse level's f written (u read)."""
    st = timed.get("smooth_fine_transfer")
    if not st or not st["launches"]:
        return None
    ms = st["ms"] / st["launches"]
    nbytes = st["bytes"] / st["launches"]
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"kernel": "smooth_fine_transfer", "bound": "hbm", "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "avg_launch_us": round(ms * 1e3, 2), "alg_bytes_per_launch": nbytes,
            "launches": st["launches"]}


def downstream_line(timed):
    """Achieved bandwidth of pt_mg_downstream from the library's HIP-event
    timing (algorithmic bytes: every array it reads or writes, once)."""
    st = timed.get("downstream")
    if not st or not st["launches"]:
        return None
    ms = st["ms"] / st["launches"]
    nbytes = st["bytes"] / st["launches"]
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"kernel": "pt_mg_downstream", "bound": "hbm", "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "avg_launch_us": round(ms * 1e3, 2), "alg_bytes_per_launch": nbytes,
            "launches": st["launches"]}


def oracle_updates(orc, prob, cycles):
    """Cell-updates of the oracle's solve: per V-cycle 4 sweeps and one
    residual on every non-coarsest level, plus the two finest-grid
    residuals of the outer loop; one final residual."""
    import numpy as np  # noqa: F401
    n = list(prob.n)
    sizes = [n[0] * n[1] * n[2]]
    for _ in range(orc.mg_levels(prob.dim, prob.n) - 1):
        n = [n[a] // 2 if a < prob.dim else 1 for a in range(3)]
        sizes.append(n[0] * n[1] * n[2])
    per_cycle = sum(5 * s for s in sizes[:-1]) + 2 * sizes[0]
    return cycles * per_cycle + sizes[0]


def cpu_model():
    """The host CPU's model name (Linux), or the platform's processor."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(prob, rtol, budget_s):
    """The oracle as it stands, on the host cores, on a bounded sample of
    the same workload: whole steps (assembly, right-hand side, multigrid
    solve to the same tolerance) repeated until the budget is used; when
    one V-cycle already takes a large share of the budget, a single step
    capped at one V-cycle.  The oracle's assembly and operator applications
    are OpenMP loops over the host threads; its lexicographic Gauss-Seidel
    sweeps, restrictions and prolongations run on one thread."""
    import oracle as orc
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def one_step(max_cycles):
        t = time.perf_counter()
        op = orc.assemble(prob)
        b_p, b_T = orc.rhs(op, prob)
        p, T, cyc, hist = orc.mg_solve(op, b_p, b_T, rtol=rtol, max_cycles=max_cycles,
                                       pin_mean=prob.mean_constraint)
        if prob.uf_star is not None:
            orc.downstream(op, prob.dt, p, T, prob.C, prob.uf_star, prob.E1, prob.E2,
                           prob.uc_star, prob.kappa, prob.sigma,
                           mu=(prob.liquid.mu, prob.gas.mu))
        done = max_cycles if cyc < 0 else cyc
        return time.perf_counter() - t, oracle_updates(orc, prob, done), done

    total, updates, cycles = one_step(1)
    reps, capped = 1, True
    if total * 4 < budget_s:
        capped = False
        total, updates, reps, cycles = 0.0, 0, 0, 0
        while total < budget_s:
            dt, up, done = one_step(50)
            total += dt
            updates += up
            cycles += done
            reps += 1
    sample = (f"{prob.name}: {reps} oracle step(s) of "
              + ("provisional state + div u* + " if prob.mode == "state" else "")
              + "assembly + paper RHS + FP64 V(2,2) "
              f"lexicographic multigrid"
              + (" + velocity correction and phase energies" if prob.uf_star is not None else "")
              + f" ({cycles} V-cycles in all"
              + (", capped at one V-cycle" if capped else f", rtol {rtol:g}")
              + f"), {total:.1f} s")
    return {"value": updates / total, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle", "sample": sample, "cpu_model": cpu_model(),
            "threads": {"assembly_and_residuals": threads, "vcycle_sweeps_and_transfers": 1}}


def _make_serve_request(rid):
    import workloads as W
    return W.serve_request(rid)


def serve_bench(args):
    """The serving mix: Poisson arrivals at `rate`/s of requests drawn
    from a pool of distinct seeded requests (2-D 128^2..2048^2 and 3-D
    64^3..192^3, 1-4 bubbles, mixed precision to 1e-9) whose inputs are
    resident on the device, through the continuous-batching engine.
    Reports solves/s and p50/p99 latency (arrival to result ready) over the
    arrivals after the warm-up: one JSON line for the open-loop run at
    --serve-rate, then (--serve-sweep) one per rate of a saturation sweep."""
    import multiprocessing as mp

    import numpy as np
    import torch

    import workloads as W
    import workloads.device as D
    from paper_2206_11294_amd import ptmg, serve

    pool_n = args.serve_pool
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        probs = pool.map(_make_serve_request, range(pool_n))
    print(f"# serving pool of {pool_n} requests generated", file=sys.stderr, flush=True)
    entries = []
    for pr in probs:
        s, t = D.to_device(pr)
        p = torch.empty(pr.ncells, dtype=torch.float64, device="cuda")
        entries.append({"prob": pr, "s": s, "t": t, "p": p, "T": torch.empty_like(p),
                        "busy": None})
    del probs
    torch.cuda.synchronize()
    rtol = args.rtol if args.rtol is not None else 1e-9

    def window(rate, seconds, warmup):
        srv = serve.Server(hbm_budget=int(args.serve_budget_gb * (1 << 30)),
                           max_active=args.serve_slots, use_graphs=False,
                           omega_milli=args.serve_omega, coarse_sweeps=args.serve_coarse)
        arrivals = W.poisson_arrivals(rate, seconds, seed=4)
        t0 = serve.now() + 0.05
        submitted = []   # (rid, arrival time, problem)
        busy = []        # entries whose outputs are in use
        nxt = 0
        for ta in arrivals:
            srv.progress(t0 + ta)
            still = []
            for e in busy:   # release entries whose request finished
                if srv.request(e["busy"])["status"] in (-2, -3):
                    still.append(e)
                else:
                    e["busy"] = None
            busy = still
            # the next free pool entry (outputs of an entry are in use while busy)
            for _ in range(pool_n):
                e = entries[nxt % pool_n]
                nxt += 1
                if e["busy"] is None:
                    break
            else:
                srv.progress(float("inf"))
                for b in busy:
                    b["busy"] = None
                busy = []
            rid = srv.submit(e["s"], ptmg.PT_PREC_MIXED, e["p"], e["T"], div=e["t"].get("div"),
                             rtol=rtol, nu1=args.serve_nu[0], nu2=args.serve_nu[1],
                             t_arrival=t0 + ta, keepalive=e["t"])
            e["busy"] = rid
            busy.append(e)
            submitted.append((rid, ta, e["prob"]))
        srv.run_until_idle()
        torch.cuda.synchronize()
        for e in busy:
            e["busy"] = None
        lat, done_t, cycles, cells, status = [], [], [], [], []
        for rid, ta, pr in submitted:
            info = srv.request(rid)
            status.append(info["status"])
            if ta < warmup:
                continue
            lat.append(info["t_done"] - info["t_arrival"])
            done_t.append(info["t_done"] - t0)
            cycles.append(info["cycles"])
            cells.append(pr.ncells)
        srv.destroy()
        lat = np.array(lat)
        span = max(done_t) - warmup
        return {
            "metric": "coupled p-T solves/s at p99 latency (serving mix)",
            "value": len(lat) / span,
            "unit": "solves/s",
            "n_gpus": 1,
            "steps": len(lat),
            "warmup": int(sum(1 for _, ta, _ in submitted if ta < warmup)),
            "ms_per_step": 1e3 * float(np.mean(lat)),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32+f64",
            "data": "synthetic",
            "config": {"workload": "serving_mix", "rate_per_s": rate,
                       "seconds": seconds, "warmup_s": warmup, "pool": pool_n,
                       "slots": args.serve_slots, "hbm_budget_gb": args.serve_budget_gb,
                       "sweeps": list(args.serve_nu), "omega_milli": args.serve_omega,
                       "coarse_sweeps": args.serve_coarse,
                       "rtol": rtol,
                       "sizes_2d": [W.SERVE_SIZES_2D[0], W.SERVE_SIZES_2D[-1]],
                       "sizes_3d": [W.SERVE_SIZES_3D[0], W.SERVE_SIZES_3D[-1]]},
            "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                           "p90": 1e3 * float(np.percentile(lat, 90)),
                           "p99": 1e3 * float(np.percentile(lat, 99)),
                           "max": 1e3 * float(lat.max())},
            "mean_cycles": float(np.mean(cycles)),
            "mean_cells": float(np.mean(cells)),
            "failed": int(sum(1 for s_ in status if s_ != 0)),
        }

    print(json.dumps(window(args.serve_rate, args.serve_seconds, args.serve_warmup)),
          flush=True)
    for rate in ([float(r) for r in args.serve_sweep.split(",")] if args.serve_sweep else []):
        print(json.dumps(window(rate, args.serve_sweep_seconds, 5.0)), flush=True)


def grid_study():
    """Cycles to relres 1e-12 against the grid size, per workload family:
    the 2-D bubble at N = 64..1024 (FP64), the 3-D near-wall bubble at
    N = 32..256 and the 3-D collapse at N = 64..512 (mixed precision),
    each with the library's default smoothing (V(2,2) on every level,
    omega = 1) and with the workload's bench smoothing.  One JSON line per
    (family, N, smoothing): cycles, the residual history and the solve
    time (zero guess, the paper right-hand side)."""
    import time as _t

    import torch

    import workloads as W
    import workloads.device as D
    from paper_2206_11294_amd import ptmg
    families = [("bubble2d", lambda n: W.bubble2d(n), ptmg.PT_PREC_FP64, (64, 128, 256, 512, 1024),
                 "bubble2d_1024"),
                ("wall3d", lambda n: W.wall3d(n), ptmg.PT_PREC_MIXED, (32, 64, 128, 256),
                 "wall3d_256"),
                ("collapse3d", lambda n: W.collapse3d(n), ptmg.PT_PREC_MIXED, (64, 128, 256, 512),
                 "collapse3d_512")]
    for fam, make, prec, sizes, wl in families:
        for n in sizes:
            prob = make(n)
            h, b_p, b_T, _ = D.setup(prob, prec)
            p, T = torch.empty_like(b_p), torch.empty_like(b_T)
            nu1, nu2, coarse = SWEEPS[wl]
            for label, (a, b, cs, om) in (("V(2,2)", (2, 2, 0, 1000)),
                                          ("bench", (nu1, nu2, coarse, OMEGA.get(wl, 1000)))):
                h.set_option(ptmg.PT_OPT_COARSE_SWEEPS, cs)
                h.set_option(ptmg.PT_OPT_OMEGA, om)
                info = None
                for rep in range(3):
                    torch.cuda.synchronize()
                    t0 = _t.perf_counter()
                    info = h.solve(b_p, b_T, p, T, rtol=1e-12, nu1=a, nu2=b, max_cycles=60,
                                   raise_on_noconv=False)
                    torch.cuda.synchronize()
                    ms = (_t.perf_counter() - t0) * 1e3
                hist = [max(x) for x in info["hist"]]
                rates = [hist[k] / hist[k - 1] for k in range(2, len(hist))]
                print(json.dumps({"family": fam, "n": n, "precision": "mixed" if prec else "fp64",
                                  "smoothing": label, "sweeps": [a, b], "coarse_sweeps": cs,
                                  "omega": om / 1000, "status": info["status"],
                                  "cycles": info["cycles"], "relres_hist": hist,
                                  "contraction_after_first": rates, "ms_per_solve": ms}),
                      flush=True)
            del h


def stream_probe():
    """Attainable HBM bandwidth: plain copies of 2 GiB timed with HIP
    events (the library's copy kernel and torch's copy_), and the library's
    copy kernel on sizes that fit the 256 MB Infinity Cache (median of 20
    back-to-back launches, each timed on its own)."""
    import torch
    from paper_2206_11294_amd import ptmg
    nbytes = 2 << 30
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    res = {}
    for name, fn in (("pt_copy_kernel", lambda: ptmg.copy_kernel(dst, src, nbytes)),
                     ("torch_copy", lambda: dst.copy_(src))):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        res[name] = {"GB_per_s": round(2 * nbytes / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 4)}
    sizes = []
    for mb in (32, 64, 128, 256, 512):
        nb = mb << 20
        for _ in range(5):
            ptmg.copy_kernel(dst, src, nb)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(21)]
        for i in range(20):
            ev[i].record()
            ptmg.copy_kernel(dst, src, nb)
        ev[20].record()
        torch.cuda.synchronize()
        med = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(20))[10]
        sizes.append({"MB_copied": mb, "median_us": round(med * 1e3, 2),
                      "GB_per_s": round(2 * nb / (med * 1e-3) / 1e9, 1)})
    print(json.dumps({"stream_probe_bytes_moved": 2 * nbytes, **res,
                      "pt_copy_kernel_by_size": sizes}), flush=True)


def copy_calibration(nbytes):
    import torch
    from paper_2206_11294_amd import ptmg
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        ptmg.copy_kernel(dst, src, nbytes)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="collapse3d_512", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None)
    ap.add_argument("--method", choices=["defect", "bicgstab"], default="defect",
                    help="outer iteration: the defect-correction loop of Sec. 3, or "
                         "BiCGStab with the V-cycle as preconditioner")
    ap.add_argument("--stiff", action="store_true",
                    help="diffusive-CFL time step (bubble workloads)")
    ap.add_argument("--rtol", type=float, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="mixed-precision workloads: skip the FP64 steps timed beside")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="in the CPU leg, skip the oracle's residual of the GPU solution")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="BYTES")
    ap.add_argument("--nu1", type=int, default=None,
                    help="pre-sweeps on the finest level (default: the workload's)")
    ap.add_argument("--nu2", type=int, default=None,
                    help="post-sweeps on the finest level (default: the workload's)")
    ap.add_argument("--coarse-sweeps", type=int, default=None,
                    help="16 nu1 + nu2 below the finest level (PT_OPT_COARSE_SWEEPS; "
                         "default: the workload's)")
    ap.add_argument("--omega", type=int, default=None,
                    help="1000 x the finest level's over-relaxation (PT_OPT_OMEGA; "
                         "default: the workload's)")
    ap.add_argument("--w-levels", type=int, default=None,
                    help="levels below the finest visited as a W-cycle (PT_OPT_W_LEVELS; "
                         "default: 2 for diffusive 3-D steps, else 0, the V-cycle)")
    ap.add_argument("--tail-cells", type=int, default=None,
                    help="largest level of the single-block tail (PT_OPT_TAIL_CELLS)")
    ap.add_argument("--timing-every", type=int, default=7,
                    help="time one finest-grid smoothing run in this many")
    ap.add_argument("--serve", action="store_true", help="the serving mix instead of a workload")
    ap.add_argument("--stream-probe", action="store_true", help="copy bandwidth, then exit")
    ap.add_argument("--grid-study", action="store_true",
                    help="cycles to tolerance against the grid size per workload family, then exit")
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-seconds", type=float, default=130.0,
                    help="open-loop run length, warm-up included")
    ap.add_argument("--serve-warmup", type=float, default=10.0)
    ap.add_argument("--serve-pool", type=int, default=256,
                    help="distinct seeded requests resident on the device")
    ap.add_argument("--serve-sweep", default="",
                    help="comma-separated arrival rates of a saturation sweep after the run")
    ap.add_argument("--serve-sweep-seconds", type=float, default=35.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    # the serving mix's smoothing, measured fastest: V(3,2) on the finest
    # level over-relaxed by 1.1, one sweep each way below (two cycles
    # instead of 2.5 on average; the engine keeps up to above 1200/s)
    ap.add_argument("--serve-omega", type=int, default=1100,
                    help="PT_OPT_OMEGA of every request (0: the library default)")
    ap.add_argument("--serve-coarse", type=int, default=17,
                    help="PT_OPT_COARSE_SWEEPS of every request (0: the library default)")
    ap.add_argument("--serve-nu", type=int, nargs=2, default=[3, 2],
                    help="finest-level pre- and post-sweeps of every request")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(one request or grid per GPU); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads.device as D
    from paper_2206_11294_amd import ptmg

    if args.stream_probe:
        stream_probe()
        return
    if args.grid_study:
        grid_study()
        return
    if args.copy_calib:
        copy_calibration(args.copy_calib)
    if args.serve:
        serve_bench(args)
        return

    name = args.workload
    _, prec_default, rtol_default = WORKLOADS[name]
    prec_name = args.precision or prec_default
    rtol = args.rtol if args.rtol is not None else rtol_default
    prec = ptmg.PT_PREC_MIXED if prec_name == "mixed" else ptmg.PT_PREC_FP64
    prob = make_problem(name, args.stiff)
    nu1, nu2, coarse = (2, 2, 0) if args.stiff else SWEEPS[name]
    # diffusive 3-D steps: over-relaxed by 1.2 with the W-cycle below, 15
    # instead of 17 cycles at 256^3; 2-D diffusive steps gain nothing from it
    omega = (1200 if prob.dim == 3 else 1000) if args.stiff else OMEGA.get(name, 1000)
    args.omega = omega if args.omega is None else args.omega
    args.nu1 = nu1 if args.nu1 is None else args.nu1
    args.nu2 = nu2 if args.nu2 is None else args.nu2
    args.coarse_sweeps = coarse if args.coarse_sweeps is None else args.coarse_sweeps
    if args.w_levels is None:
        # diffusive 3-D steps: two coarse corrections per visit on levels 1
        # and 2 (17 instead of 37 cycles at 256^3, 33 % less time); the
        # acoustic steps and 2-D keep the V-cycle (in 2-D the coarse levels
        # cost too much to visit twice)
        args.w_levels = 2 if (args.stiff and prob.dim == 3) else 0
    method = ptmg.PT_SOLVE_BICGSTAB if args.method == "bicgstab" else ptmg.PT_SOLVE_DEFECT
    print(f"# workload {name} grid {prob.n} precision {prec_name} rtol {rtol:g}",
          file=sys.stderr, flush=True)

    run = timed_steps(prob, prec, rtol, method, args)
    h, info, p, T = run["h"], run["info"], run["p"], run["T"]
    stats, timed = run["stats"], run["timed"]
    elapsed, updates, cycles = run["elapsed"], run["updates"], run["cycles"]

    dom = ROOFLINE_KERNEL
    st = timed[dom]
    avg_ms = st["ms"] / max(st["launches"], 1)
    bytes_per_launch = st["bytes"] / max(st["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = traffic_from_profile(name, dom, stats[dom]["launches"] / args.steps)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "avg_launch_us": round(avg_ms * 1e3, 2),
                "alg_bytes_per_launch": bytes_per_launch, "timed_launches": st["launches"],
                "timed_every": args.timing_every}

    out = {
        "metric": "coupled p-T cell-updates/s",
        "value": updates / elapsed,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec_name == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": name, "grid": list(prob.n[: prob.dim]), "precision": prec_name,
                   "geometry": "axisymmetric r-z" if prob.axisymmetric else "cartesian",
                   "rtol": rtol, "cycles_per_solve": float(np.mean(cycles)),
                   "step": ("pt_state_eval + " if prob.mode == "state" else "")
                   + ("pt_mg_divergence + " if run["faces"] else "")
                   + ("pt_mg_update + pt_mg_solve" if prob.mode == "explicit" else
                      "pt_mg_step (update + paper RHS + solve)")
                   + (" + pt_mg_downstream" if run["faces"] else ""),
                   "method": args.method, "time_step": "diffusive" if args.stiff else "acoustic",
                   "tail_levels": run["tail_levels"], "w_levels": args.w_levels,
                   "omega": args.omega / 1000.0,
                   "sweeps": {"finest": [args.nu1, args.nu2],
                              "coarse": (list(divmod(args.coarse_sweeps, 16))
                                         if args.coarse_sweeps else [args.nu1, args.nu2])},
                   "footprint_bytes": run["footprint"],
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "transfer_sweep": transfer_sweep_line(timed),
        "upstream": upstream_line(prob, run["state_ms"]),
        "downstream": downstream_line(timed),
        "launches_per_step": {k: v["launches"] / args.steps for k, v in stats.items()},
        "relres_last": list(info["relres"]),
        "relres_hist_last": [[float("%.3g" % x) for x in pair] for pair in info["hist"]],
    }
    P, TT = p.cpu().numpy(), T.cpu().numpy()
    h.destroy()
    del run, h, p, T
    torch.cuda.empty_cache()

    if prec == ptmg.PT_PREC_MIXED and not args.no_fp64_compare:
        # the same steps with the plain FP64 V-cycle, same size and tolerance
        print("# the same steps with the FP64 V-cycle", file=sys.stderr, flush=True)
        ref = timed_steps(prob, ptmg.PT_PREC_FP64, rtol, method, args, roofline_timing=False)
        fp64_ms = 1e3 * ref["elapsed"] / args.steps
        out["fp64_same_steps"] = {
            "precision": "fp64", "rtol": rtol, "ms_per_step": fp64_ms,
            "cycles_per_solve": float(np.mean(ref["cycles"])),
            "cell_updates_per_s": ref["updates"] / ref["elapsed"],
            "relres_last": list(ref["info"]["relres"]),
            "mixed_speedup": fp64_ms / out["ms_per_step"]}
        ref["h"].destroy()
        del ref
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        # the CPU leg: the oracle timed on the host cores, and (grids it
        # assembles in seconds) its own residual of the last GPU solution
        out["cpu_baseline"] = cpu_baseline(prob, rtol, args.cpu_seconds)
        if not args.no_oracle_check and prob.ncells <= 150_000_000:
            import oracle as orc
            op = orc.assemble(prob)
            bp, bT = orc.rhs(op, prob)   # the oracle's own right-hand side
            out["oracle_relres_of_gpu_solution"] = [float(x)
                                                    for x in orc.relres(op, bp, bT, P, TT)]
    print(json.dumps(out), flush=True)


def timed_steps(prob, prec, rtol, method, args, roofline_timing=True):
    """W untimed and K timed steps of the workload on a handle of the
    given precision; the handle is returned alive with the last solution."""
    import torch

    import workloads.device as D
    from paper_2206_11294_amd import ptmg

    stream = torch.cuda.Stream()   # the library's stream (default priority)
    with torch.cuda.stream(stream):
        s, tens = D.to_device(prob)
        h = ptmg.PtMg(s, prec, stream=stream)
        if args.tail_cells is not None:
            h.set_option(ptmg.PT_OPT_TAIL_CELLS, args.tail_cells)
        h.set_option(ptmg.PT_OPT_COARSE_SWEEPS, args.coarse_sweeps)
        h.set_option(ptmg.PT_OPT_W_LEVELS, args.w_levels)
        h.set_option(ptmg.PT_OPT_OMEGA, args.omega)
        p = torch.empty(prob.ncells, dtype=torch.float64, device="cuda")
        T = torch.empty_like(p)
        rhs_p, rhs_T = torch.empty_like(p), torch.empty_like(p)

        state = D.state_record(prob, tens) if prob.mode == "state" else None
        state_ev = []    # (start, end) event pairs around the state kernel
        faces = D.face_inputs(prob, tens) if prob.uf_star is not None else None
        if faces is not None:
            div = torch.empty_like(p)
            U = [torch.empty_like(f) for f in faces]
            us = [tens[f"us{a}"] for a in range(prob.dim)]
            u = [torch.empty_like(x) for x in us]
            E1, E2 = torch.empty_like(p), torch.empty_like(p)

        def step():
            if state is not None:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                ptmg.state_eval(state, stream)
                b.record(stream)
                state_ev.append((a, b))
            if prob.mode == "explicit":
                h.update(s)
                b_p, b_T = tens["f_p"], tens["f_T"]
                info = h.solve(b_p, b_T, p, T, rtol=rtol, max_cycles=120, nu1=args.nu1,
                               nu2=args.nu2, method=method)
            else:
                # update + paper right-hand side + solve in one call
                if faces is not None:
                    h.divergence(faces, out=div)
                info = h.step(s, div if faces is not None else tens.get("div"), rhs_p, rhs_T,
                              p, T, rtol=rtol, max_cycles=120, nu1=args.nu1, nu2=args.nu2,
                              method=method)
            if faces is not None:
                h.downstream(p, T, tens["C"], faces, U, us, u, tens["E1"], tens["E2"], E1, E2,
                             tens["kappa"], prob.sigma)
            return info

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        if roofline_timing:
            # HIP events only around the finest-grid smoother (the kernel
            # the roofline reports), and only around one smoothing run in
            # `timing_every`, so that the timed steps carry little overhead
            h.set_timing(True, classes=[ROOFLINE_KERNEL, "smooth_fine_transfer"]
                         + (["downstream"] if faces is not None else []))
            h.set_option(ptmg.PT_OPT_TIMING_EVERY, args.timing_every)
        h.reset_stats()
        updates = 0
        cycles = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            info = step()
            updates += h.last_cell_updates()
            cycles.append(info["cycles"])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        stats = h.kernel_stats()
        timed = h.timed_stats()
        h.set_timing(False)
        state_ms = [a.elapsed_time(b) for a, b in state_ev[args.warmup:]]
    return {"h": h, "info": info, "p": p, "T": T, "stats": stats, "timed": timed,
            "elapsed": elapsed, "updates": updates, "cycles": cycles, "state_ms": state_ms,
            "faces": faces is not None, "tail_levels": h.get_option(ptmg.PT_OPT_TAIL),
            "footprint": ptmg.footprint_bytes(s, prec)}


if __name__ == "__main__":
    main()
