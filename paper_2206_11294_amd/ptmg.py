"""ctypes binding of libptmg (the C ABI in include/pt_mg.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch provides device memory (float64 CUDA/HIP tensors) and streams.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptmg.so")

PT_OK, PT_ERR_ARG, PT_ERR_OOM, PT_ERR_SINGULAR, PT_ERR_NOCONV, PT_ERR_HIP, PT_ERR_STATE = range(7)
STATUS_NAMES = {0: "PT_OK", 1: "PT_ERR_ARG", 2: "PT_ERR_OOM", 3: "PT_ERR_SINGULAR",
                4: "PT_ERR_NOCONV", 5: "PT_ERR_HIP", 6: "PT_ERR_STATE"}
PT_COEF_EXPLICIT, PT_COEF_PHASES, PT_COEF_STATE = 0, 1, 2
PT_PREC_FP64, PT_PREC_MIXED = 0, 1
PT_MAX_HIST = 64
PT_OPT_GRAPHS, PT_OPT_TAIL, PT_OPT_FUSED, PT_OPT_TIMING_EVERY, PT_OPT_SPECULATE = 1, 2, 3, 4, 5
PT_OPT_TAIL_CELLS = 6
PT_OPT_COARSE_SWEEPS = 7
PT_OPT_W_LEVELS = 8
PT_OPT_OMEGA = 9
KERNEL_CLASSES = ["outer_residual", "smooth_fine", "smooth_coarse", "restrict", "prolong",
                  "coarse_solve", "other", "downstream", "smooth_fine_transfer"]


class PtMgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class pt_phase(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in
                ("rho", "k", "cp", "cv", "c", "gamma", "Gamma", "Pi", "b", "beta", "q", "mu")]


_Dp = ctypes.c_void_p


class pt_problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
        ("mode", ctypes.c_int),
        ("alpha_p", _Dp), ("alpha_T", _Dp),
        ("alpha_p_const", ctypes.c_double), ("alpha_T_const", ctypes.c_double),
        ("B", _Dp), ("B_const", ctypes.c_double * 4),
        ("C", _Dp), ("liquid", pt_phase), ("gas", pt_phase), ("dt", ctypes.c_double),
        ("p_adv", _Dp), ("T_adv", _Dp),
        ("p_adv_const", ctypes.c_double), ("T_adv_const", ctypes.c_double),
        ("mean_constraint", ctypes.c_int),
        ("m1", _Dp), ("m2", _Dp), ("axisymmetric", ctypes.c_int),
    ]


class pt_state(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_longlong),
        ("C", _Dp), ("m1", _Dp), ("m2", _Dp), ("E", _Dp), ("mom", _Dp * 3),
        ("liquid", pt_phase), ("gas", pt_phase),
        ("p_adv", _Dp), ("T_adv", _Dp),
    ]


class pt_downstream(ctypes.Structure):
    _fields_ = [
        ("p", _Dp), ("T", _Dp), ("C", _Dp), ("kappa", _Dp), ("sigma", ctypes.c_double),
        ("U_star", _Dp * 3), ("U", _Dp * 3), ("u_star", _Dp * 3), ("u", _Dp * 3),
        ("E1_adv", _Dp), ("E2_adv", _Dp), ("E1", _Dp), ("E2", _Dp),
    ]


class pt_solve_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_cycles", ctypes.c_int),
                ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("zero_guess", ctypes.c_int),
                ("method", ctypes.c_int), ("async_", ctypes.c_int)]   # C field `async`


PT_SOLVE_DEFECT, PT_SOLVE_BICGSTAB = 0, 1
PT_SCRATCH_MAX_CELLS = 1 << 20   # pt_mg_solve_noalloc: largest BiCGStab grid


class AsyncSolve:
    """A stream-ordered solve in flight: result() after a stream sync."""

    def __init__(self, info, owner):
        self._info = info
        self._owner = owner

    def result(self) -> Dict:
        info = self._info
        n = info.hist_len
        out = {"status": info.status, "cycles": info.cycles,
               "relres": (info.relres[0], info.relres[1]),
               "hist": [(info.relres_hist[2 * q], info.relres_hist[2 * q + 1]) for q in range(n)],
               "t_solve_s": info.t_solve_s}
        if self in self._owner._pending:
            self._owner._pending.remove(self)
        return out


class pt_solve_info(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("relres", ctypes.c_double * 2),
                ("relres_hist", ctypes.c_double * (2 * PT_MAX_HIST)),
                ("hist_len", ctypes.c_int), ("t_solve_s", ctypes.c_double),
                ("status", ctypes.c_int)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libptmg.so (built by paper_2206_11294_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libptmg.so is not built ({LIB_PATH}); "
                              "run `python -m paper_2206_11294_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        c_int, c_void, c_double = ctypes.c_int, ctypes.c_void_p, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "pt_mg_footprint_bytes": (ctypes.c_size_t, [P(pt_problem), c_int]),
            "pt_state_eval": (c_int, [P(pt_state), c_void]),
            "pt_mg_setup": (c_int, [P(pt_problem), c_int, c_void, P(c_void)]),
            "pt_mg_update": (c_int, [c_void, P(pt_problem)]),
            "pt_mg_paper_rhs": (c_int, [c_void] + [c_void] * 5),
            "pt_mg_divergence": (c_int, [c_void, P(c_void), c_void]),
            "pt_mg_step": (c_int, [c_void, P(pt_problem)] + [c_void] * 5 + [P(pt_solve_opts),
                                                                           P(pt_solve_info)]),
            "pt_mg_downstream": (c_int, [c_void, P(pt_downstream)]),
            "pt_mg_solve": (c_int, [c_void, c_void, c_void, c_void, c_void,
                                    P(pt_solve_opts), P(pt_solve_info)]),
            "pt_mg_solve_noalloc": (c_int, [c_void, c_void, c_void, c_void, c_void,
                                            P(pt_solve_opts), P(pt_solve_info)]),
            "pt_mg_residual": (c_int, [c_void] + [c_void] * 6 + [P(c_double)]),
            "pt_mg_destroy": (None, [c_void]),
            "pt_mg_last_error": (ctypes.c_char_p, [c_void]),
            "pt_mg_num_levels": (c_int, [c_void]),
            "pt_mg_level_dims": (c_int, [c_void, c_int, P(c_int), P(c_double)]),
            "pt_mg_get_operator": (c_int, [c_void, c_int, c_void, c_void]),
            "pt_mg_smooth": (c_int, [c_void, c_int, c_void, c_void, c_void, c_void, c_int]),
            "pt_mg_restrict_residual": (c_int, [c_void, c_int] + [c_void] * 6),
            "pt_mg_prolong_add": (c_int, [c_void, c_int] + [c_void] * 4),
            "pt_mg_coarse_solve": (c_int, [c_void] + [c_void] * 4),
            "pt_mg_vcycle": (c_int, [c_void] + [c_void] * 4 + [c_int, c_int]),
            "pt_mg_set_timing": (c_int, [c_void, c_int]),
            "pt_mg_kernel_stats": (c_int, [c_void, c_int, P(ctypes.c_long), P(c_double),
                                           P(c_double)]),
            "pt_mg_timed_stats": (c_int, [c_void, c_int, P(ctypes.c_long), P(c_double),
                                          P(c_double)]),
            "pt_mg_reset_stats": (c_int, [c_void]),
            "pt_mg_last_cell_updates": (ctypes.c_longlong, [c_void]),
            "pt_copy_kernel": (c_int, [c_void, c_void, ctypes.c_size_t, c_void]),
            "pt_mg_set_option": (c_int, [c_void, c_int, c_int]),
            "pt_mg_get_option": (c_int, [c_void, c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> Sequence[str]:
    """Names of the C-ABI functions the binding uses."""
    lib()
    return ["pt_state_eval", "pt_mg_footprint_bytes", "pt_mg_setup", "pt_mg_update", "pt_mg_paper_rhs",
            "pt_mg_divergence", "pt_mg_downstream", "pt_mg_step",
            "pt_mg_solve", "pt_mg_solve_noalloc", "pt_mg_residual", "pt_mg_destroy", "pt_mg_last_error",
            "pt_mg_num_levels", "pt_mg_level_dims", "pt_mg_get_operator", "pt_mg_smooth",
            "pt_mg_restrict_residual", "pt_mg_prolong_add", "pt_mg_coarse_solve",
            "pt_mg_vcycle", "pt_mg_set_timing", "pt_mg_kernel_stats", "pt_mg_timed_stats", "pt_mg_reset_stats",
            "pt_mg_last_cell_updates", "pt_copy_kernel", "pt_mg_set_option",
            "pt_mg_get_option"]


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("fields must be contiguous float64 device tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def phase_struct(rho, k, cp, cv, c, gamma, Gamma, Pi, b, beta=0.0, q=0.0, mu=0.0) -> pt_phase:
    return pt_phase(rho, k, cp, cv, c, gamma, Gamma, Pi, b, beta, q, mu)


def footprint_bytes(prob: pt_problem, precision: int) -> int:
    return int(lib().pt_mg_footprint_bytes(ctypes.byref(prob), precision))


def state_eval(st: pt_state, stream=None) -> None:
    """pt_state_eval: provisional (p, T) into st.p_adv, st.T_adv (device
    tensors the caller keeps alive), asynchronous on `stream`."""
    rc = lib().pt_state_eval(ctypes.byref(st), _stream_ptr(stream))
    if rc:
        raise PtMgError(rc, lib().pt_mg_last_error(None).decode())


def copy_kernel(dst: torch.Tensor, src: torch.Tensor, nbytes: int, stream=None) -> None:
    rc = lib().pt_copy_kernel(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                              nbytes, _stream_ptr(stream))
    if rc:
        raise PtMgError(rc, lib().pt_mg_last_error(None).decode())


class PtMg:
    """One handle: assembled operator + hierarchy on the device."""

    def __init__(self, prob: pt_problem, precision: int = PT_PREC_FP64, stream=None,
                 keepalive=None):
        self._h = ctypes.c_void_p()
        self._pending = []   # stream-ordered solves whose record the stream writes later
        self.precision = precision
        self.N = prob.n[0] * prob.n[1] * prob.n[2]
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream
        rc = lib().pt_mg_setup(ctypes.byref(prob), precision, _stream_ptr(stream),
                               ctypes.byref(self._h))
        if rc:
            raise PtMgError(rc, lib().pt_mg_last_error(None).decode())

    # -- plumbing ----------------------------------------------------------
    def _check(self, rc: int):
        if rc not in (PT_OK,):
            raise PtMgError(rc, lib().pt_mg_last_error(self._h).decode())

    def _empty(self, n: Optional[int] = None) -> torch.Tensor:
        return torch.empty(self.N if n is None else n, dtype=torch.float64, device=self.device)

    def destroy(self):
        if self._h:
            lib().pt_mg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    # -- the C ABI ----------------------------------------------------------
    def update(self, prob: pt_problem, keepalive=None):
        self._check(lib().pt_mg_update(self._h, ctypes.byref(prob)))

    def paper_rhs(self, p_adv=None, T_adv=None, div_ustar=None) -> Tuple[torch.Tensor, torch.Tensor]:
        b_p, b_T = self._empty(), self._empty()
        self._check(lib().pt_mg_paper_rhs(self._h, _ptr(p_adv), _ptr(T_adv), _ptr(div_ustar),
                                          _ptr(b_p), _ptr(b_T)))
        return b_p, b_T

    def step(self, prob: pt_problem, div_ustar, b_p, b_T, p, T, rtol=1e-9, max_cycles=50,
             nu1=2, nu2=2, zero_guess=True, raise_on_noconv=True,
             method=PT_SOLVE_DEFECT) -> Dict:
        """pt_mg_step: update + paper right-hand side (into b_p, b_T) + solve."""
        opts = pt_solve_opts(rtol, max_cycles, nu1, nu2, int(zero_guess), int(method))
        info = pt_solve_info()
        rc = lib().pt_mg_step(self._h, ctypes.byref(prob), _ptr(div_ustar), _ptr(b_p), _ptr(b_T),
                              _ptr(p), _ptr(T), ctypes.byref(opts), ctypes.byref(info))
        if rc and (rc != PT_ERR_NOCONV or raise_on_noconv):
            self._check(rc)
        n = info.hist_len
        return {"status": rc, "cycles": info.cycles, "relres": (info.relres[0], info.relres[1]),
                "hist": [(info.relres_hist[2 * q], info.relres_hist[2 * q + 1]) for q in range(n)],
                "t_solve_s": info.t_solve_s}

    def divergence(self, U: Sequence[torch.Tensor], out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """pt_mg_divergence: div of the face velocities U[a] (one tensor per axis)."""
        div = self._empty() if out is None else out
        ptrs = (ctypes.c_void_p * 3)(*[_ptr(u) for u in U], *([None] * (3 - len(U))))
        self._check(lib().pt_mg_divergence(self._h, ptrs, _ptr(div)))
        return div

    def downstream(self, p, T, C, U_star, U, u_star=None, u=None, E1_adv=None, E2_adv=None,
                   E1=None, E2=None, kappa=None, sigma: float = 0.0) -> None:
        """pt_mg_downstream: velocity correction and phase energies into the
        given output tensors (U, u, E1, E2)."""
        d = pt_downstream()
        d.p, d.T, d.C, d.kappa = _ptr(p), _ptr(T), _ptr(C), _ptr(kappa)
        d.sigma = sigma
        for a in range(len(U_star)):
            d.U_star[a] = _ptr(U_star[a])
            d.U[a] = _ptr(U[a])
            if u_star is not None:
                d.u_star[a] = _ptr(u_star[a])
                d.u[a] = _ptr(u[a])
        d.E1_adv, d.E2_adv, d.E1, d.E2 = _ptr(E1_adv), _ptr(E2_adv), _ptr(E1), _ptr(E2)
        self._check(lib().pt_mg_downstream(self._h, ctypes.byref(d)))

    def solve(self, b_p, b_T, p, T, rtol=1e-9, max_cycles=50, nu1=2, nu2=2,
              zero_guess=True, raise_on_noconv=True, method=PT_SOLVE_DEFECT,
              noalloc=False) -> Dict:
        """pt_mg_solve, or pt_mg_solve_noalloc with noalloc=True."""
        opts = pt_solve_opts(rtol, max_cycles, nu1, nu2, int(zero_guess), int(method))
        info = pt_solve_info()
        fn = lib().pt_mg_solve_noalloc if noalloc else lib().pt_mg_solve
        rc = fn(self._h, _ptr(b_p), _ptr(b_T), _ptr(p), _ptr(T),
                ctypes.byref(opts), ctypes.byref(info))
        if rc and (rc != PT_ERR_NOCONV or raise_on_noconv):
            self._check(rc)
        n = info.hist_len
        return {"status": rc, "cycles": info.cycles, "relres": (info.relres[0], info.relres[1]),
                "hist": [(info.relres_hist[2 * q], info.relres_hist[2 * q + 1]) for q in range(n)],
                "t_solve_s": info.t_solve_s}

    def solve_async(self, b_p, b_T, p, T, rtol=1e-9, max_cycles=12, nu1=2, nu2=2,
                    zero_guess=True) -> "AsyncSolve":
        """pt_mg_solve in the stream-ordered mode: returns at once; the
        result (p, T and the record) is valid after the stream is synchronised."""
        opts = pt_solve_opts(rtol, max_cycles, nu1, nu2, int(zero_guess), PT_SOLVE_DEFECT, 1)
        info = pt_solve_info()
        self._check(lib().pt_mg_solve(self._h, _ptr(b_p), _ptr(b_T), _ptr(p), _ptr(T),
                                      ctypes.byref(opts), ctypes.byref(info)))
        pend = AsyncSolve(info, self)
        self._pending.append(pend)   # the stream writes `info` later: keep it alive
        return pend

    def residual(self, b_p, b_T, p, T, want_fields=True):
        r_p = self._empty() if want_fields else None
        r_T = self._empty() if want_fields else None
        rel = (ctypes.c_double * 2)()
        self._check(lib().pt_mg_residual(self._h, _ptr(b_p), _ptr(b_T), _ptr(p), _ptr(T),
                                         _ptr(r_p), _ptr(r_T), rel))
        return r_p, r_T, (rel[0], rel[1])

    def last_error(self) -> str:
        return lib().pt_mg_last_error(self._h).decode()

    def num_levels(self) -> int:
        return int(lib().pt_mg_num_levels(self._h))

    def level_dims(self, level: int):
        n = (ctypes.c_int * 3)()
        hl = ctypes.c_double()
        self._check(lib().pt_mg_level_dims(self._h, level, n, ctypes.byref(hl)))
        return (n[0], n[1], n[2]), hl.value

    def _nl(self, level):
        n, _ = self.level_dims(level)
        return n[0] * n[1] * n[2]

    def get_operator(self, level: int):
        Nl = self._nl(level)
        faces, B = self._empty(6 * Nl), self._empty(4 * Nl)
        self._check(lib().pt_mg_get_operator(self._h, level, _ptr(faces), _ptr(B)))
        return faces.view(6, Nl), B.view(4, Nl)

    def smooth(self, level, f_p, f_T, u_p, u_T, sweeps=1):
        self._check(lib().pt_mg_smooth(self._h, level, _ptr(f_p), _ptr(f_T), _ptr(u_p),
                                       _ptr(u_T), sweeps))

    def restrict_residual(self, level, f_p, f_T, u_p, u_T):
        Nc = self._nl(level + 1)
        fc_p, fc_T = self._empty(Nc), self._empty(Nc)
        self._check(lib().pt_mg_restrict_residual(self._h, level, _ptr(f_p), _ptr(f_T),
                                                  _ptr(u_p), _ptr(u_T), _ptr(fc_p), _ptr(fc_T)))
        return fc_p, fc_T

    def prolong_add(self, level, ec_p, ec_T, u_p, u_T):
        self._check(lib().pt_mg_prolong_add(self._h, level, _ptr(ec_p), _ptr(ec_T), _ptr(u_p),
                                            _ptr(u_T)))

    def coarse_solve(self, f_p, f_T):
        Nc = self._nl(self.num_levels() - 1)
        u_p, u_T = self._empty(Nc), self._empty(Nc)
        self._check(lib().pt_mg_coarse_solve(self._h, _ptr(f_p), _ptr(f_T), _ptr(u_p), _ptr(u_T)))
        return u_p, u_T

    def vcycle(self, f_p, f_T, nu1=2, nu2=2):
        e_p, e_T = self._empty(), self._empty()
        self._check(lib().pt_mg_vcycle(self._h, _ptr(f_p), _ptr(f_T), _ptr(e_p), _ptr(e_T),
                                       nu1, nu2))
        return e_p, e_T

    def set_timing(self, on, classes=None):
        """on: bool; classes: names from KERNEL_CLASSES to time (default all)."""
        if not on:
            code = 0
        elif classes is None:
            code = 1
        else:
            mask = 0
            for c in classes:
                mask |= 1 << KERNEL_CLASSES.index(c)
            code = 1 + 2 * mask
        self._check(lib().pt_mg_set_timing(self._h, code))

    def kernel_stats(self) -> Dict[str, Dict[str, float]]:
        out = {}
        for c, name in enumerate(KERNEL_CLASSES):
            n = ctypes.c_long()
            ms = ctypes.c_double()
            by = ctypes.c_double()
            self._check(lib().pt_mg_kernel_stats(self._h, c, ctypes.byref(n), ctypes.byref(ms),
                                                 ctypes.byref(by)))
            out[name] = {"launches": n.value, "ms": ms.value, "bytes": by.value}
        return out

    def timed_stats(self) -> Dict[str, Dict[str, float]]:
        """Per class: launches inside timed runs, their ms and bytes."""
        out = {}
        for c, name in enumerate(KERNEL_CLASSES):
            n = ctypes.c_long()
            ms = ctypes.c_double()
            by = ctypes.c_double()
            self._check(lib().pt_mg_timed_stats(self._h, c, ctypes.byref(n), ctypes.byref(ms),
                                                ctypes.byref(by)))
            out[name] = {"launches": n.value, "ms": ms.value, "bytes": by.value}
        return out

    def reset_stats(self):
        self._check(lib().pt_mg_reset_stats(self._h))

    def set_option(self, option: int, value: int):
        self._check(lib().pt_mg_set_option(self._h, option, int(value)))

    def get_option(self, option: int) -> int:
        return int(lib().pt_mg_get_option(self._h, option))

    def last_cell_updates(self) -> int:
        return int(lib().pt_mg_last_cell_updates(self._h))
