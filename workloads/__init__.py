"""Seeded synthetic inputs for the coupled pressure-temperature solve.

This module only builds *inputs*: grids, volume-fraction fields of bubbles,
the phase property records, the time step, the velocity-divergence forcing
and explicit-mode coefficients.  It contains none of the solver's arithmetic
(no coupling coefficients, no operator, no right-hand side of the coupled
system): both the HIP library and the CPU oracle derive those from what is
returned here.

Property values (SI units, a 1 mm unit domain so that a radius of 0.1 is the
paper's R0 = 100 um):
  * liquid: rho = 1000, k = 0.6, c_p = 4000, c = 1500,
    gamma = c_p/c_v of water from Table 1 (4285/3610), and the NASG
    parameters of Table 1 (Gamma = 1.19, Pi = 7028e5 Pa, b = 6.61e-4,
    c_v = 3610) so that the thermal dilation follows Eq. (10);
  * gas: rho = 1, k = 0.6/23, c_p = 1000, c = 340, gamma = 1.4, ideal gas
    (Gamma = gamma, Pi = b = 0), so Eq. (10) reduces to 1/T.
The ratios 1000:1 (density), 23:1 (conductivity), 4:1 (heat capacity) and
the sound speeds 1500/340 are the workload's; the ambient state is
T0 = 293.15 K, p0 = 101325 Pa (Sec. 5).  The time step is the acoustic
CFL of 1/2 on the liquid sound speed (Algorithm 1 and Sec. 4.2), or the
diffusive CFL of 1/2 on the gas thermal diffusivity (Sec. 4.1) for the stiff
variant.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

T0 = 293.15
P0 = 101325.0
L_UNIT = 1.0e-3           # physical length of the unit domain [m]


@dataclasses.dataclass(frozen=True)
class Phase:
    """Per-phase property record.  beta <= 0 means: derive it from Eq. (10)."""
    rho: float
    k: float
    cp: float
    cv: float
    c: float
    gamma: float
    Gamma: float
    Pi: float
    b: float
    beta: float = 0.0
    q: float = 0.0          # NASG energy offset of Eq. (9) (state mode)
    mu: float = 0.0         # dynamic viscosity (viscous work of Eq. 39)

    def as_tuple(self) -> Tuple[float, ...]:
        return (self.rho, self.k, self.cp, self.cv, self.c, self.gamma,
                self.Gamma, self.Pi, self.b, self.beta, self.q, self.mu)


LIQUID = Phase(rho=1000.0, k=0.6, cp=4000.0, cv=3610.0, c=1500.0,
               gamma=4285.0 / 3610.0, Gamma=1.19, Pi=7028e5, b=6.61e-4)
GAS = Phase(rho=1.0, k=0.6 / 23.0, cp=1000.0, cv=1000.0 / 1.4, c=340.0,
            gamma=1.4, Gamma=1.4, Pi=0.0, b=0.0)

# State mode (densities and sound speeds from the cell state): the full
# Table 1 record of water (c_p = 4285, q) and an ideal gas; rho and c of
# these records are nominal only.
LIQUID_NASG = Phase(rho=1055.9, k=0.6, cp=4285.0, cv=3610.0, c=1500.0,
                    gamma=4285.0 / 3610.0, Gamma=1.19, Pi=7028e5, b=6.61e-4,
                    q=-1177788.0)
GAS_IDEAL = Phase(rho=1.2, k=0.6 / 23.0, cp=1000.0, cv=1000.0 / 1.4, c=340.0,
                  gamma=1.4, Gamma=1.4, Pi=0.0, b=0.0)

# Dynamic viscosities [Pa s] of water and air near 293 K, for the viscous
# work of the phase energies (Eq. 39) in the state-mode workloads.
MU_WATER = 1.0e-3
MU_AIR = 1.8e-5

# Reference conserved state of the state-mode workloads: phase densities
# and specific internal energies near (1 atm, 293 K) for the two records
# above (the liquid and the gas at 1 and 10 atm).  They are input data;
# the provisional pressure and temperature are what Eqs. (20), (23) make
# of them.
REF_LIQUID = (1055.899893, 81526.1000)          # rho [kg/m^3], e [J/kg]
REF_GAS = {1: (1.20974757, 209392.8571), 10: (12.0974757, 209392.8571)}


@dataclasses.dataclass
class Problem:
    """One coupled solve's inputs, host-side (numpy, float64).

    Arrays are laid out with x fastest: shape (nz, ny, nx) in 3-D and
    (ny, nx) in 2-D, flattened in C order to cell i + nx*(j + ny*k).
    """
    name: str
    dim: int
    n: Tuple[int, int, int]
    h: float
    mode: str                      # "explicit", "phases" or "state"
    # explicit mode (canonical form):  -div(a grad u) + B u = f
    alpha_p: float = 0.0
    alpha_T: float = 0.0
    B_const: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)  # (pp, pT, Tp, TT)
    f_p: Optional[np.ndarray] = None
    f_T: Optional[np.ndarray] = None
    # phases mode (paper form, Eqs. 27-34)
    C: Optional[np.ndarray] = None
    liquid: Phase = LIQUID
    gas: Phase = GAS
    dt: float = 0.0
    p_adv: Optional[np.ndarray] = None     # None -> p_adv_const everywhere
    p_adv_const: float = P0
    T_adv: Optional[np.ndarray] = None     # None -> T_adv_const everywhere
    T_adv_const: float = T0
    div_ustar: Optional[np.ndarray] = None  # None -> zero
    rtol: float = 1e-9
    precision: str = "fp64"                 # "fp64" or "mixed"
    mean_constraint: bool = False
    # state mode: advected conserved variables (Sec. 3); p_adv, T_adv are
    # derived from them (Eqs. 20, 23)
    m1: Optional[np.ndarray] = None         # C rho_1
    m2: Optional[np.ndarray] = None         # (1 - C) rho_2
    E: Optional[np.ndarray] = None          # total energy per volume
    mom: Optional[List[np.ndarray]] = None  # averaged momentum, one array per axis
    # face velocities u* (Eq. provel): one array per axis, n_a + 1 faces
    # along a (walls included), x fastest; when given, div u* is computed
    # from them and div_ustar is None
    uf_star: Optional[List[np.ndarray]] = None
    uc_star: Optional[List[np.ndarray]] = None  # u* at cell centres, one array per axis
    E1: Optional[np.ndarray] = None         # C rho_1 e_T,1 after advection
    E2: Optional[np.ndarray] = None         # (1 - C) rho_2 e_T,2 after advection
    kappa: Optional[np.ndarray] = None      # interface curvature [1/m]
    sigma: float = 0.0                      # surface tension [N/m]
    # axisymmetric r-z grid (2-D): x is the axis direction, y the radius
    # from the axis on the lower y wall
    axisymmetric: bool = False

    @property
    def ncells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def shape(self) -> Tuple[int, ...]:
        if self.dim == 2:
            return (self.n[1], self.n[0])
        return (self.n[2], self.n[1], self.n[0])


def _cell_centres(n: Sequence[int], dim: int, h: float) -> List[np.ndarray]:
    """Cell-centre coordinates (i+1/2)h as broadcastable arrays, x last."""
    axes = []
    for a in range(dim):
        x = (np.arange(n[a], dtype=np.float64) + 0.5) * h
        shp = [1] * dim
        shp[dim - 1 - a] = n[a]
        axes.append(x.reshape(shp))
    return axes


def bubble_fraction(dim: int, n: Sequence[int], h: float,
                    centres: Sequence[Sequence[float]],
                    radii: Sequence[float]) -> np.ndarray:
    """Liquid volume fraction C of gas bubbles, smoothed over one cell.

    s = min_b(|x - c_b| - R_b) is the signed distance to the nearest bubble
    surface at the cell centre (positive in the liquid), and
    C = clamp(1/2 + s/h, 0, 1).  Centres and radii are in metres.
    """
    xs = _cell_centres(n, dim, h)
    s = None
    for c, r in zip(centres, radii):
        d2 = 0.0
        for a in range(dim):
            d2 = d2 + (xs[a] - c[a]) ** 2
        sb = np.sqrt(d2) - r
        s = sb if s is None else np.minimum(s, sb)
    C = np.clip(0.5 + s / h, 0.0, 1.0)
    return np.ascontiguousarray(np.broadcast_to(C, tuple(
        n[dim - 1 - a] for a in range(dim))), dtype=np.float64)


def face_velocities(dim: int, n: Sequence[int], seed: int, amp: float,
                    noise: float) -> List[np.ndarray]:
    """Seeded face velocities inside closed walls: for each axis a, a few
    smooth modes sin(pi k x_a) prod_b cos(pi m x_b) of amplitude `amp` on the
    face centres (zero on the walls normal to a) plus uniform noise in
    [-noise, noise] on the interior faces.  Array shapes are x last, with
    n_a + 1 faces along a."""
    nn = _grid(dim, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for a in range(dim):
        m = list(nn[:dim])
        m[a] += 1
        shape = tuple(m[dim - 1 - b] for b in range(dim))
        u = np.zeros(shape)
        for _ in range(3):
            term = np.full(shape, amp * rng.uniform(-1.0, 1.0))
            for b in range(dim):
                shp = [1] * dim
                shp[dim - 1 - b] = m[b]
                if b == a:
                    x = np.arange(m[b]) / nn[b]
                    term = term * np.sin(math.pi * int(rng.integers(1, 4)) * x).reshape(shp)
                else:
                    x = (np.arange(m[b]) + 0.5) / nn[b]
                    term = term * np.cos(math.pi * int(rng.integers(0, 4)) * x).reshape(shp)
            u += term
        if noise:
            u += noise * rng.uniform(-1.0, 1.0, size=shape)
        wall = [slice(None)] * dim
        wall[dim - 1 - a] = 0
        u[tuple(wall)] = 0.0
        wall[dim - 1 - a] = -1
        u[tuple(wall)] = 0.0
        out.append(np.ascontiguousarray(u))
    return out


def interface_curvature(dim: int, C: np.ndarray, radius: float) -> np.ndarray:
    """(dim - 1)/R in cells cut by the interface (0 < C < 1), else 0: the
    curvature of a sphere (circle) of radius R."""
    return np.where((C > 0.0) & (C < 1.0), (dim - 1) / radius, 0.0)


SIGMA_WATER = 0.072             # surface tension of water-air near 20 C [N/m]


def acoustic_dt(h: float, c_liquid: float = LIQUID.c, cfl: float = 0.5) -> float:
    return cfl * h / c_liquid


def diffusive_dt(h: float, gas: Phase = GAS, cfl: float = 0.5) -> float:
    kappa = gas.k / (gas.rho * gas.cp)
    return cfl * h * h / kappa


def _grid(dim: int, n: Sequence[int]) -> Tuple[int, int, int]:
    n = tuple(int(v) for v in n)
    if dim == 2:
        return (n[0], n[1], 1)
    return (n[0], n[1], n[2])


def explicit_const(nx: int = 64, ny: int = 64, seed: int = 0,
                   dt: float = 1e-3) -> Problem:
    """2-D constant-coefficient case: alpha_p = 1, alpha_T = 0.1,
    B = [[1, 0.3], [0.2, 1]]/dt, unit square, f ~ U[-1, 1] (p then T)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.uniform(-1.0, 1.0, size=(2, ny, nx))
    return Problem(name=f"explicit_const_{nx}x{ny}", dim=2, n=(nx, ny, 1),
                   h=1.0 / nx, mode="explicit", alpha_p=1.0, alpha_T=0.1,
                   B_const=(1.0 / dt, 0.3 / dt, 0.2 / dt, 1.0 / dt),
                   f_p=np.ascontiguousarray(f[0]), f_T=np.ascontiguousarray(f[1]),
                   rtol=1e-10)


def bubble_problem(name: str, dim: int, n: Sequence[int],
                   centres_unit: Sequence[Sequence[float]],
                   radii_unit: Sequence[float], p_liquid: float, p_gas: float,
                   div_amp: float = 0.0, div_seed: int = 0,
                   dt: Optional[float] = None, stiff: bool = False,
                   rtol: float = 1e-9, precision: str = "fp64") -> Problem:
    """Bubbles in liquid on a uniform grid whose x extent is the unit domain.

    p_adv = C p_liquid + (1-C) p_gas, T_adv = T0, and the velocity
    divergence is (div_amp/dt) * xi with xi ~ U[-1, 1] (seed div_seed).
    """
    nn = _grid(dim, n)
    h = L_UNIT / nn[0]
    centres = [[L_UNIT * v for v in c] for c in centres_unit]
    radii = [L_UNIT * r for r in radii_unit]
    C = bubble_fraction(dim, nn, h, centres, radii)
    if dt is None:
        dt = diffusive_dt(h) if stiff else acoustic_dt(h)
    if p_liquid == p_gas:
        p_adv = None
    else:
        p_adv = C * p_liquid + (1.0 - C) * p_gas
    div = None
    if div_amp != 0.0:
        rng = np.random.Generator(np.random.PCG64(div_seed))
        div = (div_amp / dt) * rng.uniform(-1.0, 1.0, size=C.shape)
    return Problem(name=name, dim=dim, n=nn, h=h, mode="phases", C=C, dt=dt,
                   p_adv=p_adv, p_adv_const=p_liquid, T_adv=None,
                   T_adv_const=T0, div_ustar=div, rtol=rtol,
                   precision=precision)


def bubble2d(n: int = 1024, stiff: bool = False) -> Problem:
    """2-D single bubble: radius 0.1 at the centre, p_l = p_g = p0, forcing
    by a seeded velocity divergence of amplitude 1e-6/dt (seed 2)."""
    return bubble_problem(f"bubble2d_{n}" + ("_stiff" if stiff else ""), 2,
                          (n, n), [(0.5, 0.5)], [0.1], P0, P0,
                          div_amp=1e-6, div_seed=2, stiff=stiff)


def wall3d(n: int = 256, precision: str = "mixed", stiff: bool = False) -> Problem:
    """3-D bubble near a no-flux wall at z = 0: radius 0.2 centred at
    (0.5, 0.5, 0.24) (stand-off 1.2R), gas at 10 p0 in liquid at p0."""
    return bubble_problem(f"wall3d_{n}" + ("_stiff" if stiff else ""), 3,
                          (n, n, n), [(0.5, 0.5, 0.24)], [0.2], P0, 10 * P0,
                          stiff=stiff, precision=precision)


def collapse3d(n: int = 512, precision: str = "mixed") -> Problem:
    """3-D collapse-like field: radius 0.25 centred, gas at 0.01 p0 in
    liquid at 100 p0."""
    return bubble_problem(f"collapse3d_{n}", 3, (n, n, n),
                          [(0.5, 0.5, 0.5)], [0.25], 100 * P0, 0.01 * P0,
                          precision=precision)


def axi2d(n: int = 1024) -> Problem:
    """Axisymmetric r-z bubble near a rigid wall: radius 0.1 on the axis at
    axial distance 0.2 from the wall z = 0 (stand-off 2), gas at p0/20 in
    liquid at p0, forcing by a seeded velocity divergence of amplitude
    1e-6/dt (seed 2); x is the axial and y the radial coordinate."""
    prob = bubble_problem(f"axi2d_{n}", 2, (n, n), [(0.2, 0.0)], [0.1], P0, P0 / 20,
                          div_amp=1e-6, div_seed=2)
    return dataclasses.replace(prob, axisymmetric=True)


def state_problem(name: str, dim: int, n: Sequence[int],
                  centres_unit: Sequence[Sequence[float]], radii_unit: Sequence[float],
                  gas_atm: int = 1, u_amp: float = 1.0, seed: int = 12,
                  div_amp: float = 1e-6, precision: str = "fp64",
                  rtol: float = 1e-9, viscous: bool = True) -> Problem:
    """Bubbles in liquid given by advected conserved variables (Sec. 3):
    C from the bubble geometry; phase masses m1 = C rho_l, m2 = (1-C) rho_g
    and total energy E = C rho_l e_l + (1-C) rho_g e_g + 1/2 rho |u|^2
    from the reference states REF_LIQUID, REF_GAS[gas_atm] with seeded
    smooth relative variations (rho_g 5 %, e_l 1e-4, e_g 1 %); a smooth
    velocity of amplitude u_amp [m/s] per axis (momentum = rho u, phase
    energies E_i = m_i (e_i + |u|^2/2)); the acoustic time step; provisional
    face velocities u* of the same amplitude inside closed walls with seeded
    noise of amplitude div_amp h/dt on the interior faces (so that div u* has
    a rough part of order div_amp/dt); u* at the cell centres = u; the
    curvature of the first bubble in the cut cells, water's surface
    tension; water's and air's viscosities (none if not viscous)."""
    nn = _grid(dim, n)
    h = L_UNIT / nn[0]
    centres = [[L_UNIT * v for v in c] for c in centres_unit]
    radii = [L_UNIT * r for r in radii_unit]
    C = bubble_fraction(dim, nn, h, centres, radii)

    def unit(s):
        f = smooth_field(dim, nn, seed + s)
        m = np.abs(f).max()
        return f / m if m > 0 else f

    rho_l, e_l0 = REF_LIQUID
    rho_g0, e_g0 = REF_GAS[gas_atm]
    rho_g = rho_g0 * (1.0 + 0.05 * unit(1))
    e_l = e_l0 * (1.0 + 1e-4 * unit(2))
    e_g = e_g0 * (1.0 + 0.01 * unit(3))
    m1 = C * rho_l
    m2 = (1.0 - C) * rho_g
    rho = m1 + m2
    us = [u_amp * unit(4 + a) for a in range(dim)]
    mom = [np.ascontiguousarray(rho * u) for u in us]
    k2 = 0.5 * sum(u * u for u in us)
    E1 = m1 * (e_l + k2)
    E2 = m2 * (e_g + k2)
    E = E1 + E2
    dt = acoustic_dt(h)
    uf = face_velocities(dim, nn, seed + 10, u_amp, div_amp * h / dt)
    liquid = dataclasses.replace(LIQUID_NASG, mu=MU_WATER if viscous else 0.0)
    gas = dataclasses.replace(GAS_IDEAL, mu=MU_AIR if viscous else 0.0)
    return Problem(name=name, dim=dim, n=nn, h=h, mode="state", C=C,
                   liquid=liquid, gas=gas, dt=dt, div_ustar=None,
                   rtol=rtol, precision=precision, m1=np.ascontiguousarray(m1),
                   m2=np.ascontiguousarray(m2), E=np.ascontiguousarray(E), mom=mom,
                   uf_star=uf, uc_star=[np.ascontiguousarray(u) for u in us],
                   E1=np.ascontiguousarray(E1), E2=np.ascontiguousarray(E2),
                   kappa=interface_curvature(dim, C, radii[0]), sigma=SIGMA_WATER)


def state2d(n: int = 1024) -> Problem:
    """The 2-D bubble (radius 0.1, centred) given by its conserved state,
    gas and liquid near 1 atm, velocity 1 m/s."""
    return state_problem(f"state2d_{n}", 2, (n, n), [(0.5, 0.5)], [0.1], gas_atm=1)


def state3d(n: int = 256, precision: str = "mixed") -> Problem:
    """The near-wall 3-D bubble (radius 0.2 at (0.5, 0.5, 0.24)) given by
    its conserved state, gas near 10 atm, velocity 1 m/s."""
    return state_problem(f"state3d_{n}", 3, (n, n, n), [(0.5, 0.5, 0.24)], [0.2],
                         gas_atm=10, precision=precision)


# ---------------------------------------------------------------- serving mix
SERVE_SIZES_2D = [m * 2 ** k for k in range(5, 10) for m in (4, 5, 6, 7)
                  if 128 <= m * 2 ** k <= 2048]
SERVE_SIZES_3D = [m * 2 ** k for k in range(3, 7) for m in (4, 5, 6, 7)
                  if 64 <= m * 2 ** k <= 192]
SERVE_SIZES_2D = sorted(set(SERVE_SIZES_2D))
SERVE_SIZES_3D = sorted(set(SERVE_SIZES_3D))


def serve_request(rid: int, sizes2d: Sequence[int] = SERVE_SIZES_2D,
                  sizes3d: Sequence[int] = SERVE_SIZES_3D) -> Problem:
    """Request `rid` of the serving mix (seed 4*10**6 + rid): 2-D or 3-D with
    probability 1/2, an edge length drawn uniformly from the size list,
    1-4 non-overlapping bubbles of radius U[0.05, 0.2] with centres
    U[R, 1-R]^d (rejected when closer than R_a + R_b + 2h), gas at 10 p0,
    mixed precision to 1e-9."""
    rng = np.random.Generator(np.random.PCG64(4_000_000 + rid))
    dim = 2 if rng.random() < 0.5 else 3
    sizes = sizes2d if dim == 2 else sizes3d
    N = int(sizes[int(rng.integers(0, len(sizes)))])
    nb = int(rng.integers(1, 5))
    h_unit = 1.0 / N
    centres: List[List[float]] = []
    radii: List[float] = []
    tries = 0
    while len(radii) < nb and tries < 1000:
        tries += 1
        r = float(rng.uniform(0.05, 0.2))
        c = [float(rng.uniform(r, 1.0 - r)) for _ in range(dim)]
        ok = all(math.dist(c, c2) >= r + r2 + 2 * h_unit
                 for c2, r2 in zip(centres, radii))
        if ok:
            centres.append(c)
            radii.append(r)
    return bubble_problem(f"serve_{rid}_{dim}d_{N}", dim, (N,) * dim,
                          centres, radii, P0, 10 * P0, precision="mixed")


def poisson_arrivals(rate: float, duration: float, seed: int = 4) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        out.append(t)
    return np.asarray(out)


def smooth_field(dim: int, n: Sequence[int], seed: int, modes: int = 3) -> np.ndarray:
    """A seeded smooth field: a sum of a few low cosine modes with random
    amplitudes, on the cell centres of a unit-spaced grid."""
    nn = _grid(dim, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(nn[dim - 1 - a] for a in range(dim))
    out = np.zeros(shape)
    for _ in range(modes):
        term = np.full(shape, rng.uniform(-1.0, 1.0))
        for a in range(dim):
            k = int(rng.integers(0, 4))
            x = (np.arange(nn[a]) + 0.5) / nn[a]
            shp = [1] * dim
            shp[dim - 1 - a] = nn[a]
            term = term * np.cos(math.pi * k * x).reshape(shp)
        out += term
    return out
