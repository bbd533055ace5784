"""FP64 CPU oracle for the coupled pressure-temperature solve.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may use it; the product library never does.  It shares no code
with the HIP path; the only common module is the seeded input generator
(`workloads`), which holds no solver arithmetic.

Exact solutions come from a sparse direct solve of the canonical system
(`direct_solve`, small and medium grids) or from the oracle's own FP64
multigrid defect-correction loop (`mg_solve`, any grid), whose answer is
certified by its own residual.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import shutil
import subprocess
import tempfile
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ptorc.c")
_LIB = os.path.join(_HERE, "libptorc.so")
_lib = None


def _compile(out: str, plant: int = 0) -> None:
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                           "-ffp-contract=off", "-std=c99", f"-DORC_PLANT={int(plant)}",
                           "-o", out, _SRC, "-lm"])


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    stale = (not os.path.exists(_LIB)
             or os.path.getmtime(_LIB) < os.path.getmtime(_SRC))
    if force or stale:
        tmp = _LIB + ".tmp"
        _compile(tmp)
        os.replace(tmp, _LIB)
    return _LIB


@contextlib.contextmanager
def planted(k: int):
    """Mutation checks of the pin tests: inside the block every oracle
    call goes to a private build with planted mistake k (ORC_PLANT in
    ptorc.c); the correct library is restored on exit."""
    global _lib
    saved = _load()
    d = tempfile.mkdtemp(prefix="ptorc_plant")
    try:
        path = os.path.join(d, f"libptorc_plant{int(k)}.so")
        _compile(path, k)
        lib = ctypes.CDLL(path)
        _declare(lib)
        _lib = lib
        yield
    finally:
        _lib = saved
        shutil.rmtree(d, ignore_errors=True)


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


class _Phase(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in
                ("rho", "k", "cp", "cv", "c", "gamma", "Gamma", "Pi", "b", "beta", "q")]


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_L = ctypes.POINTER(ctypes.c_long)
_P = ctypes.POINTER(_Phase)
_PP = ctypes.POINTER(_D)


def _declare(lib):
    c_long, c_int, c_double = ctypes.c_long, ctypes.c_int, ctypes.c_double
    sig = {
        "orc_beta": (c_double, [_P, c_double, c_double]),
        "orc_phase_lambdas": (None, [_P, c_double, c_double, c_double, _D]),
        "orc_block_from_lambdas": (None, [_D, _D]),
        "orc_cell_lambdas": (None, [c_double, _P, _P, c_double, c_double, c_double, _D, _D]),
        "orc_assemble_phases": (c_long, [c_long, _D, _P, _P, c_double, _D, c_double,
                                         _D, c_double, _D, _D, _D, _D]),
        "orc_paper_rhs": (None, [c_long, _D, _D, c_double, _D, c_double, _D, c_double,
                                 _D, _D]),
        "orc_state": (None, [c_long, c_int, _D, _D, _D, _D, _D, _P, _P, _D, _D]),
        "orc_sound2": (c_double, [_P, c_double, c_double]),
        "orc_assemble_state": (c_long, [c_long, _D, _D, _D, _P, _P, c_double, _D, _D, _D,
                                        _D, _D, _D]),
        "orc_canonical_rhs": (None, [c_long, _D, _D, _D, _D, _D]),
        "orc_faces_from_cells": (None, [c_int, _I, _D, _D, _D]),
        "orc_apply": (None, [c_int, _I, c_double, _D, c_int, _D, _D, _D, _D, _D]),
        "orc_residual": (None, [c_int, _I, c_double, _D, c_int, _D, _D, _D, _D, _D, _D, _D]),
        "orc_paper_residual": (None, [c_int, _I, c_double, _D, c_int, _D, _D, _D, _D, _D,
                                      _D, _D]),
        "orc_lex_sweep": (None, [c_int, _I, c_double, _D, c_int, _D, _D, _D, _D, _D]),
        "orc_rb_sweep": (None, [c_int, _I, c_double, _D, c_int, _D, _D, _D, _D, _D]),
        "orc_coarse_operator": (None, [c_int, _I, _D, _D, _D, _D]),
        "orc_restrict": (None, [c_int, _I, _D, _D, _D, _D]),
        "orc_prolong_add": (None, [c_int, _I, _D, _D, _D, _D]),
        "orc_dense_matrix": (None, [c_int, _I, c_double, _D, c_int, _D, c_int, _D]),
        "orc_lu": (c_int, [c_long, _D, _L]),
        "orc_lu_solve": (None, [c_long, _D, _L, _D]),
        "orc_mg_solve": (c_int, [c_int, _I, c_double, _D, c_int, _D, _D, _D, _D, _D, _D, _D,
                                 _D,
                                 c_double, c_int, c_int, c_int, c_int, _D]),
        "orc_mg_levels": (c_int, [c_int, _I]),
        "orc_divergence": (None, [c_int, _I, c_double, c_int, _PP, _D]),
        "orc_project": (None, [c_int, _I, c_double, c_double, _D, _D, _PP, _PP, _PP, _PP]),
        "orc_phase_pressures": (None, [c_long, _D, _D, _D, c_double, _D, _D]),
        "orc_energy_update": (None, [c_int, _I, c_double, c_double, _D, c_int, _D, _D, _D, _D,
                                     _PP,
                                     _D, _D, _D, _D, _D]),
        "orc_viscous_work": (None, [c_int, _I, c_double, c_int, _D, c_double, c_double, _PP, _PP,
                                    _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args


def _d(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.cast(None, _D)
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _dp(arrays):
    """Array of three double pointers (NULL where an axis is absent)."""
    if arrays is None:
        return ctypes.cast(None, _PP)
    ptrs = [_d(a) if a is not None else ctypes.cast(None, _D) for a in arrays]
    ptrs += [ctypes.cast(None, _D)] * (3 - len(ptrs))
    return (_D * 3)(*ptrs)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(-1)


def _dims(n) -> ctypes.Array:
    return (ctypes.c_int * 3)(*[int(v) for v in n])


def phase(ph) -> _Phase:
    """ctypes phase record from a workloads.Phase (the viscosity enters
    through viscous_work, not the record)."""
    return _Phase(ph.rho, ph.k, ph.cp, ph.cv, ph.c, ph.gamma, ph.Gamma, ph.Pi, ph.b, ph.beta,
                  ph.q)


# ---------------------------------------------------------------------------
# operator
# ---------------------------------------------------------------------------
@dataclass
class Operator:
    """Assembled canonical operator on one grid (all arrays flat, FP64).

    F: faces [6, N] ((component, axis) major; lower face of each cell),
    B: block [4, N] in the order (pp, pT, Tp, TT),
    lam: paper coefficients [4, N] (l1, l2, l3, l4) in phases mode, else None;
    p_adv, T_adv: the provisional state the operator was assembled at, when
    the problem gives it through conserved variables (state mode);
    axi: 1 for the axisymmetric r-z metric (y the radius), else 0.
    """
    dim: int
    n: Tuple[int, int, int]
    h: float
    F: np.ndarray
    B: np.ndarray
    lam: Optional[np.ndarray] = None
    a_p: Optional[np.ndarray] = None
    a_T: Optional[np.ndarray] = None
    p_adv: Optional[np.ndarray] = None
    T_adv: Optional[np.ndarray] = None
    axi: int = 0

    @property
    def N(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


def beta(ph, p: float, T: float) -> float:
    """Eq. (10)."""
    return _load().orc_beta(ctypes.byref(phase(ph)), p, T)


def phase_lambdas(ph, p: float, T: float, dt: float) -> np.ndarray:
    """Eqs. (29)-(32) for one phase: (l1, l2, l3, l4)."""
    out = np.zeros(4)
    _load().orc_phase_lambdas(ctypes.byref(phase(ph)), p, T, dt, _d(out))
    return out


def block_from_lambdas(lam) -> np.ndarray:
    lam = _f64(lam)
    out = np.zeros(4)
    _load().orc_block_from_lambdas(_d(lam), _d(out))
    return out


def cell_lambdas(C: float, liquid, gas, p: float, T: float, dt: float):
    lam, B = np.zeros(4), np.zeros(4)
    _load().orc_cell_lambdas(C, ctypes.byref(phase(liquid)), ctypes.byref(phase(gas)),
                             p, T, dt, _d(lam), _d(B))
    return lam, B


def faces_from_cells(dim, n, a_p, a_T) -> np.ndarray:
    a_p, a_T = _f64(a_p), _f64(a_T)
    N = a_p.size
    F = np.zeros(6 * N)
    _load().orc_faces_from_cells(dim, _dims(n), _d(a_p), _d(a_T), _d(F))
    return F.reshape(6, N)


def state(prob) -> Tuple[np.ndarray, np.ndarray]:
    """Provisional (p, T) of a state-mode problem, Eqs. (20) and (23)."""
    N = prob.ncells
    p, T = np.zeros(N), np.zeros(N)
    mom = None if prob.mom is None else np.concatenate([_f64(m) for m in prob.mom])
    _load().orc_state(N, prob.dim, _d(_f64(prob.C)), _d(_f64(prob.m1)), _d(_f64(prob.m2)),
                      _d(_f64(prob.E)), _d(mom), ctypes.byref(phase(prob.liquid)),
                      ctypes.byref(phase(prob.gas)), _d(p), _d(T))
    return p, T


def sound2(ph, rho: float, p: float) -> float:
    """Eq. (11)."""
    return _load().orc_sound2(ctypes.byref(phase(ph)), rho, p)


def assemble(prob) -> Operator:
    """Assemble the canonical operator of a workloads.Problem."""
    lib = _load()
    N = prob.ncells
    if prob.mode == "state":
        p_adv, T_adv = (state(prob) if prob.p_adv is None
                        else (_f64(prob.p_adv).copy(), _f64(prob.T_adv).copy()))
        a_p, a_T = np.zeros(N), np.zeros(N)
        lam, B = np.zeros(4 * N), np.zeros(4 * N)
        bad = lib.orc_assemble_state(N, _d(_f64(prob.C)), _d(_f64(prob.m1)),
                                     _d(_f64(prob.m2)), ctypes.byref(phase(prob.liquid)),
                                     ctypes.byref(phase(prob.gas)), prob.dt, _d(p_adv),
                                     _d(T_adv), _d(a_p), _d(a_T), _d(lam), _d(B))
        if bad:
            raise ValueError(f"{bad} cells with a non-positive block")
        F = faces_from_cells(prob.dim, prob.n, a_p, a_T)
        return Operator(prob.dim, prob.n, prob.h, F, B.reshape(4, N), lam.reshape(4, N),
                        a_p, a_T, p_adv, T_adv, axi=_axi(prob))
    if prob.mode == "explicit":
        a_p = np.full(N, float(prob.alpha_p))
        a_T = np.full(N, float(prob.alpha_T))
        B = np.repeat(np.asarray(prob.B_const, dtype=np.float64)[:, None], N, axis=1)
        F = faces_from_cells(prob.dim, prob.n, a_p, a_T)
        return Operator(prob.dim, prob.n, prob.h, F, np.ascontiguousarray(B), None, a_p, a_T,
                        axi=_axi(prob))
    C = _f64(prob.C)
    a_p, a_T = np.zeros(N), np.zeros(N)
    lam, B = np.zeros(4 * N), np.zeros(4 * N)
    p_adv = None if prob.p_adv is None else _f64(prob.p_adv)
    T_adv = None if prob.T_adv is None else _f64(prob.T_adv)
    bad = lib.orc_assemble_phases(N, _d(C), ctypes.byref(phase(prob.liquid)),
                                  ctypes.byref(phase(prob.gas)), prob.dt,
                                  _d(p_adv), prob.p_adv_const, _d(T_adv),
                                  prob.T_adv_const, _d(a_p), _d(a_T), _d(lam), _d(B))
    if bad:
        raise ValueError(f"{bad} cells with a non-positive block")
    F = faces_from_cells(prob.dim, prob.n, a_p, a_T)
    return Operator(prob.dim, prob.n, prob.h, F, B.reshape(4, N), lam.reshape(4, N),
                    a_p, a_T, axi=_axi(prob))


def _axi(prob) -> int:
    """1 for an axisymmetric r-z problem (2-D only)."""
    axi = int(bool(getattr(prob, "axisymmetric", False)))
    if axi and prob.dim != 2:
        raise ValueError("the axisymmetric metric needs a 2-D grid")
    return axi


def paper_rhs(op: Operator, prob) -> Tuple[np.ndarray, np.ndarray]:
    """b = (lambda_p, lambda_T) of Eqs. (33)-(34)."""
    N = op.N
    b_p, b_T = np.zeros(N), np.zeros(N)
    lam = np.ascontiguousarray(op.lam).reshape(-1)
    p_adv = None if prob.p_adv is None else _f64(prob.p_adv)
    T_adv = None if prob.T_adv is None else _f64(prob.T_adv)
    if op.p_adv is not None:
        p_adv, T_adv = op.p_adv, op.T_adv
    div = None if prob.div_ustar is None else _f64(prob.div_ustar)
    if div is None and getattr(prob, "uf_star", None) is not None:
        div = divergence(prob.dim, prob.n, prob.h, prob.uf_star, op.axi)
    _load().orc_paper_rhs(N, _d(lam), _d(p_adv), prob.p_adv_const, _d(T_adv),
                          prob.T_adv_const, _d(div), prob.dt, _d(b_p), _d(b_T))
    return b_p, b_T


def rhs(op: Operator, prob) -> Tuple[np.ndarray, np.ndarray]:
    """The mode-native right-hand side: paper b in phases mode, f otherwise."""
    if op.lam is None:
        return _f64(prob.f_p).copy(), _f64(prob.f_T).copy()
    return paper_rhs(op, prob)


def canonical_rhs(op: Operator, b_p, b_T) -> Tuple[np.ndarray, np.ndarray]:
    if op.lam is None:
        return _f64(b_p).copy(), _f64(b_T).copy()
    N = op.N
    f_p, f_T = np.zeros(N), np.zeros(N)
    lam = np.ascontiguousarray(op.lam).reshape(-1)
    _load().orc_canonical_rhs(N, _d(lam), _d(_f64(b_p)), _d(_f64(b_T)), _d(f_p), _d(f_T))
    return f_p, f_T


def _fb(op: Operator):
    return (np.ascontiguousarray(op.F).reshape(-1), np.ascontiguousarray(op.B).reshape(-1))


def apply(op: Operator, p, T) -> Tuple[np.ndarray, np.ndarray]:
    F, B = _fb(op)
    Ap, AT = np.zeros(op.N), np.zeros(op.N)
    _load().orc_apply(op.dim, _dims(op.n), op.h, _d(F), op.axi, _d(B), _d(_f64(p)), _d(_f64(T)),
                      _d(Ap), _d(AT))
    return Ap, AT


def residual(op: Operator, f_p, f_T, p, T) -> Tuple[np.ndarray, np.ndarray]:
    F, B = _fb(op)
    rp, rT = np.zeros(op.N), np.zeros(op.N)
    _load().orc_residual(op.dim, _dims(op.n), op.h, _d(F), op.axi, _d(B), _d(_f64(f_p)),
                         _d(_f64(f_T)), _d(_f64(p)), _d(_f64(T)), _d(rp), _d(rT))
    return rp, rT


def paper_residual(op: Operator, b_p, b_T, p, T) -> Tuple[np.ndarray, np.ndarray]:
    """res = b - L(a) of Eqs. (27)-(28) (phases mode)."""
    F, _ = _fb(op)
    lam = np.ascontiguousarray(op.lam).reshape(-1)
    rp, rT = np.zeros(op.N), np.zeros(op.N)
    _load().orc_paper_residual(op.dim, _dims(op.n), op.h, _d(F), op.axi, _d(lam), _d(_f64(b_p)),
                               _d(_f64(b_T)), _d(_f64(p)), _d(_f64(T)), _d(rp), _d(rT))
    return rp, rT


def relres(op: Operator, b_p, b_T, p, T) -> np.ndarray:
    """Per-component ||res||_2 / ||b||_2 in the mode-native (paper) form."""
    if op.lam is None:
        rp, rT = residual(op, b_p, b_T, p, T)
    else:
        rp, rT = paper_residual(op, b_p, b_T, p, T)
    return np.array([np.linalg.norm(rp) / np.linalg.norm(b_p),
                     np.linalg.norm(rT) / np.linalg.norm(b_T)])


# ---------------------------------------------------------------------------
# multigrid steps (for step-by-step comparisons)
# ---------------------------------------------------------------------------
def sweep(op: Operator, f_p, f_T, p, T, order: str = "rb"):
    """One block Gauss-Seidel sweep in place ("rb" or "lex")."""
    F, B = _fb(op)
    fn = _load().orc_rb_sweep if order == "rb" else _load().orc_lex_sweep
    assert p.dtype == np.float64 and T.dtype == np.float64
    fn(op.dim, _dims(op.n), op.h, _d(F), op.axi, _d(B), _d(_f64(f_p)), _d(_f64(f_T)), _d(p),
       _d(T))


def coarse_dims(dim, n):
    return tuple(int(n[a]) // 2 if a < dim else 1 for a in range(3))


def coarse_operator(op: Operator) -> Operator:
    nc = coarse_dims(op.dim, op.n)
    Nc = nc[0] * nc[1] * nc[2]
    F, B = _fb(op)
    Fc, Bc = np.zeros(6 * Nc), np.zeros(4 * Nc)
    _load().orc_coarse_operator(op.dim, _dims(op.n), _d(F), _d(B), _d(Fc), _d(Bc))
    return Operator(op.dim, nc, 2 * op.h, Fc.reshape(6, Nc), Bc.reshape(4, Nc), axi=op.axi)


def restrict(dim, n, r_p, r_T):
    nc = coarse_dims(dim, n)
    Nc = nc[0] * nc[1] * nc[2]
    fp, fT = np.zeros(Nc), np.zeros(Nc)
    _load().orc_restrict(dim, _dims(n), _d(_f64(r_p)), _d(_f64(r_T)), _d(fp), _d(fT))
    return fp, fT


def prolong_add(dim, n, e_p, e_T, p, T):
    assert p.dtype == np.float64 and T.dtype == np.float64
    _load().orc_prolong_add(dim, _dims(n), _d(_f64(e_p)), _d(_f64(e_T)), _d(p), _d(T))


def dense_matrix(op: Operator, pin_mean: bool = False) -> np.ndarray:
    F, B = _fb(op)
    m = 2 * op.N
    M = np.zeros(m * m)
    _load().orc_dense_matrix(op.dim, _dims(op.n), op.h, _d(F), op.axi, _d(B), int(pin_mean),
                             _d(M))
    return M.reshape(m, m)


def lu_solve_dense(M: np.ndarray, x: np.ndarray) -> np.ndarray:
    """The oracle's own LU with partial pivoting."""
    m = M.shape[0]
    A = np.ascontiguousarray(M, dtype=np.float64).copy().reshape(-1)
    piv = np.zeros(m, dtype=np.int64)
    if _load().orc_lu(m, _d(A), piv.ctypes.data_as(_L)):
        raise np.linalg.LinAlgError("singular")
    y = _f64(x).copy()
    _load().orc_lu_solve(m, _d(A), piv.ctypes.data_as(_L), _d(y))
    return y


def mg_levels(dim, n) -> int:
    return _load().orc_mg_levels(dim, _dims(n))


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------
def mg_solve(op: Operator, b_p, b_T, p0=None, T0=None, rtol: float = 1e-13,
             max_cycles: int = 200, nu1: int = 2, nu2: int = 2,
             pin_mean: bool = False):
    """Defect-correction multigrid solve (Sec. 3) in FP64.

    (b_p, b_T) is the mode-native right-hand side (paper b in phases mode).
    Returns (p, T, cycles, history[cycles+1, 2]); cycles = -1 when the
    tolerance was not reached within max_cycles.
    """
    N = op.N
    b_p, b_T = _f64(b_p), _f64(b_T)
    f_p, f_T = canonical_rhs(op, b_p, b_T)
    p = np.zeros(N) if p0 is None else _f64(p0).copy()
    T = np.zeros(N) if T0 is None else _f64(T0).copy()
    hist = np.zeros(2 * (max_cycles + 2))
    F, B = _fb(op)
    lam = None if op.lam is None else np.ascontiguousarray(op.lam).reshape(-1)
    cyc = _load().orc_mg_solve(op.dim, _dims(op.n), op.h, _d(F), op.axi, _d(B), _d(lam),
                               _d(b_p), _d(b_T), _d(f_p), _d(f_T), _d(p), _d(T),
                               rtol, max_cycles, nu1, nu2, int(pin_mean), _d(hist))
    ncyc = max_cycles if cyc < 0 else cyc
    return p, T, cyc, hist[: 2 * (ncyc + 1)].reshape(-1, 2)


def sparse_matrix(op: Operator):
    """The canonical operator as a scipy CSR matrix, unknowns [p; T]."""
    import scipy.sparse as sp
    N = op.N
    nx, ny, nz = op.n
    idx = np.arange(N).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    inv_h2 = 1.0 / (op.h * op.h)
    for c in range(2):
        diag = np.zeros(N)
        for a in range(op.dim):
            Fa = op.F[c * 3 + a].reshape(nz, ny, nx)
            ax = 2 - a
            sl_hi = [slice(None)] * 3
            sl_lo = [slice(None)] * 3
            sl_hi[ax] = slice(1, None)
            sl_lo[ax] = slice(0, -1)
            w = (Fa[tuple(sl_hi)] * inv_h2).reshape(-1)
            i_hi = idx[tuple(sl_hi)].reshape(-1)
            i_lo = idx[tuple(sl_lo)].reshape(-1)
            w_hi, w_lo = w, w          # the face's weight in its upper / lower cell's row
            if op.axi and a == 1:
                jf = (i_hi // nx) % ny   # radius of the face, in units of h
                w_hi = w * jf / (jf + 0.5)
                w_lo = w * jf / (jf - 0.5)
            off = c * N
            rows += [i_hi + off, i_lo + off]
            cols += [i_lo + off, i_hi + off]
            vals += [-w_hi, -w_lo]
            np.add.at(diag, i_hi, w_hi)
            np.add.at(diag, i_lo, w_lo)
        rows.append(np.arange(N) + c * N)
        cols.append(np.arange(N) + c * N)
        vals.append(diag + op.B[0 if c == 0 else 3])
    rows += [np.arange(N), np.arange(N) + N]
    cols += [np.arange(N) + N, np.arange(N)]
    vals += [op.B[1].copy(), op.B[2].copy()]
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(2 * N, 2 * N))
    return A


def direct_solve(op: Operator, b_p, b_T) -> Tuple[np.ndarray, np.ndarray]:
    """Sparse direct solve of A u = f (mode-native right-hand side)."""
    import scipy.sparse.linalg as spla
    f_p, f_T = canonical_rhs(op, b_p, b_T)
    A = sparse_matrix(op).tocsc()
    x = spla.spsolve(A, np.concatenate([f_p, f_T]))
    return x[: op.N].copy(), x[op.N:].copy()


def solve(prob, rtol: float = 1e-13, max_cycles: int = 200, direct_max: int = 70000):
    """Reference solution of a workloads.Problem: sparse direct when the grid
    has at most `direct_max` cells, else the oracle multigrid to `rtol`.
    Returns (op, b_p, b_T, p, T)."""
    op = assemble(prob)
    b_p, b_T = rhs(op, prob)
    if op.N <= direct_max:
        p, T = direct_solve(op, b_p, b_T)
    else:
        p, T, cyc, _ = mg_solve(op, b_p, b_T, rtol=rtol, max_cycles=max_cycles,
                                pin_mean=prob.mean_constraint)
        if cyc < 0:
            raise RuntimeError("oracle multigrid did not converge")
    return op, b_p, b_T, p, T


# ---------------------------------------------------------------------------
# after the solve: velocity correction and phase energies (Sec. 3)
# ---------------------------------------------------------------------------
def face_shape(dim, n, a) -> Tuple[int, ...]:
    """Array shape (x last) of the faces across axis a: n_a + 1 along a."""
    m = [int(v) for v in n[:dim]]
    m[a] += 1
    return tuple(m[dim - 1 - b] for b in range(dim))


def divergence(dim, n, h, U, axi: int = 0) -> np.ndarray:
    """Discrete div of face velocities U[a] (the div u* of Eqs. 17, 34)."""
    Us = [_f64(u) for u in U]
    out = np.zeros(int(n[0]) * int(n[1]) * int(n[2]))
    _load().orc_divergence(dim, _dims(n), h, int(axi), _dp(Us), _d(out))
    return out


def project(op: Operator, dt: float, p, U_star, u_star=None):
    """Eq. (unp1): face velocities (and, with u_star, cell velocities) after
    the correction by the pressure gradient.  Returns (U, u or None)."""
    Us = [_f64(u) for u in U_star]
    U = [np.zeros_like(u) for u in Us]
    cs = None if u_star is None else [_f64(u) for u in u_star]
    c = None if cs is None else [np.zeros_like(u) for u in cs]
    F, _ = _fb(op)
    _load().orc_project(op.dim, _dims(op.n), op.h, dt, _d(F), _d(_f64(p)), _dp(Us), _dp(U),
                        _dp(cs), _dp(c))
    return U, c


def phase_pressures(p, C, kappa=None, sigma: float = 0.0):
    """Eqs. (37)-(38)."""
    p, C = _f64(p), _f64(C)
    p1, p2 = np.zeros_like(p), np.zeros_like(p)
    _load().orc_phase_pressures(p.size, _d(p), _d(C), _d(None if kappa is None else _f64(kappa)),
                                sigma, _d(p1), _d(p2))
    return p1, p2


def viscous_work(op: Operator, C, mu, U, u) -> np.ndarray:
    """One-fluid viscous work div(mu (grad u + grad u^T) . u) of Eq. (39)
    per cell, mu = (mu_1, mu_2), face velocities U and cell velocities u."""
    Us = [_f64(x) for x in U]
    us = [_f64(x) for x in u]
    W = np.zeros(op.N)
    _load().orc_viscous_work(op.dim, _dims(op.n), op.h, op.axi, _d(_f64(C)), float(mu[0]),
                             float(mu[1]), _dp(Us), _dp(us), _d(W))
    return W


def energy_update(op: Operator, dt: float, C, p1, p2, T, U, E1_adv, E2_adv, W=None):
    """Eq. (39) with the one-fluid viscous work W (None: inviscid).
    Returns (E1, E2)."""
    E1a, E2a = _f64(E1_adv), _f64(E2_adv)
    E1, E2 = np.zeros_like(E1a), np.zeros_like(E2a)
    F, _ = _fb(op)
    Us = [_f64(u) for u in U]
    _load().orc_energy_update(op.dim, _dims(op.n), op.h, dt, _d(F), op.axi, _d(_f64(C)), _d(_f64(p1)),
                              _d(_f64(p2)), _d(_f64(T)), _dp(Us), _d(E1a), _d(E2a),
                              _d(None if W is None else _f64(W)), _d(E1), _d(E2))
    return E1, E2


def downstream(op: Operator, dt: float, p, T, C, U_star, E1_adv, E2_adv, u_star=None,
               kappa=None, sigma: float = 0.0, mu=None):
    """The end of the step in the paper's order: velocity correction
    (Eq. unp1), phase pressures (Eqs. 37-38), phase energies (Eq. 39), the
    latter with the viscous work of the corrected velocities when
    mu = (mu_1, mu_2) is given (needs u_star).
    Returns dict(U, u, p1, p2, E1, E2, W)."""
    U, u = project(op, dt, p, U_star, u_star)
    p1, p2 = phase_pressures(p, C, kappa, sigma)
    W = None
    if mu is not None and (mu[0] > 0 or mu[1] > 0):
        if u is None:
            raise ValueError("the viscous work needs the cell velocities")
        W = viscous_work(op, C, mu, U, u)
    E1, E2 = energy_update(op, dt, C, p1, p2, T, U, E1_adv, E2_adv, W)
    return {"U": U, "u": u, "p1": p1, "p2": p2, "E1": E1, "E2": E2, "W": W}
