"""ctypes binding of the serving engine (include/pt_serve.h).

Argument marshalling only: admission, scheduling and every solve step run
in libptmg.  Arrays are float64 device tensors that must stay alive until
their request has finished.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional

import torch

from . import ptmg

PT_SERVE_QUEUED, PT_SERVE_ACTIVE = -3, -2


class pt_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_active", ctypes.c_int),
                ("use_graphs", ctypes.c_int), ("omega_milli", ctypes.c_int),
                ("coarse_sweeps", ctypes.c_int)]


class pt_request_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cycles", ctypes.c_int),
                ("relres", ctypes.c_double * 2), ("t_arrival", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("bytes", ctypes.c_size_t)]


_declared = False


def _lib():
    global _declared
    L = ptmg.lib()
    if not _declared:
        c_int, c_void, c_double = ctypes.c_int, ctypes.c_void_p, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "pt_server_now": (c_double, []),
            "pt_server_create": (c_int, [P(pt_server_config), P(c_void)]),
            "pt_server_submit": (c_int, [c_void, P(ptmg.pt_problem), c_int, c_void, c_void, c_void,
                                         c_void, c_void, P(ptmg.pt_solve_opts), c_double,
                                         P(ctypes.c_longlong)]),
            "pt_server_progress": (c_int, [c_void, c_double, P(c_int)]),
            "pt_server_request": (c_int, [c_void, ctypes.c_longlong, P(pt_request_info)]),
            "pt_server_stats": (c_int, [c_void, P(c_int), P(c_int), P(ctypes.c_longlong),
                                        P(ctypes.c_size_t)]),
            "pt_server_destroy": (None, [c_void]),
            "pt_server_last_error": (ctypes.c_char_p, [c_void]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _declared = True
    return L


def exported_symbols():
    return ["pt_server_now", "pt_server_create", "pt_server_submit", "pt_server_progress",
            "pt_server_request", "pt_server_stats", "pt_server_destroy", "pt_server_last_error"]


def now() -> float:
    return float(_lib().pt_server_now())


class Server:
    def __init__(self, hbm_budget: int, max_active: int = 8, use_graphs: bool = False,
                 omega_milli: int = 0, coarse_sweeps: int = 0):
        self._s = ctypes.c_void_p()
        cfg = pt_server_config(int(hbm_budget), int(max_active), int(use_graphs),
                               int(omega_milli), int(coarse_sweeps))
        rc = _lib().pt_server_create(ctypes.byref(cfg), ctypes.byref(self._s))
        if rc:
            raise ptmg.PtMgError(rc, _lib().pt_server_last_error(None).decode())
        self._keep: Dict[int, tuple] = {}

    def _check(self, rc):
        if rc:
            raise ptmg.PtMgError(rc, _lib().pt_server_last_error(self._s).decode())

    def submit(self, prob: ptmg.pt_problem, precision: int, p: torch.Tensor, T: torch.Tensor,
               b_p: Optional[torch.Tensor] = None, b_T: Optional[torch.Tensor] = None,
               div: Optional[torch.Tensor] = None, rtol: float = 1e-9, max_cycles: int = 50,
               nu1: int = 2, nu2: int = 2, zero_guess: bool = True,
               t_arrival: Optional[float] = None, keepalive=None) -> int:
        opts = ptmg.pt_solve_opts(rtol, max_cycles, nu1, nu2, int(zero_guess))
        rid = ctypes.c_longlong()
        t = now() if t_arrival is None else float(t_arrival)
        self._check(_lib().pt_server_submit(self._s, ctypes.byref(prob), precision,
                                            ptmg._ptr(b_p), ptmg._ptr(b_T), ptmg._ptr(div),
                                            ptmg._ptr(p), ptmg._ptr(T), ctypes.byref(opts), t,
                                            ctypes.byref(rid)))
        self._keep[rid.value] = (prob, p, T, b_p, b_T, div, keepalive)
        return rid.value

    def progress(self, until: float) -> int:
        n = ctypes.c_int()
        self._check(_lib().pt_server_progress(self._s, float(until), ctypes.byref(n)))
        return n.value

    def run_until_idle(self) -> None:
        self.progress(float("inf"))

    def request(self, rid: int) -> Dict:
        inf = pt_request_info()
        self._check(_lib().pt_server_request(self._s, rid, ctypes.byref(inf)))
        if inf.status not in (PT_SERVE_QUEUED, PT_SERVE_ACTIVE):
            self._keep.pop(rid, None)
        return {"status": inf.status, "cycles": inf.cycles,
                "relres": (inf.relres[0], inf.relres[1]), "t_arrival": inf.t_arrival,
                "t_admit": inf.t_admit, "t_done": inf.t_done, "bytes": inf.bytes}

    def stats(self) -> Dict:
        q, a, f, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong(), ctypes.c_size_t()
        self._check(_lib().pt_server_stats(self._s, ctypes.byref(q), ctypes.byref(a),
                                           ctypes.byref(f), ctypes.byref(b)))
        return {"queued": q.value, "active": a.value, "finished": f.value, "bytes": b.value}

    def destroy(self):
        if self._s:
            _lib().pt_server_destroy(self._s)
            self._s = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
