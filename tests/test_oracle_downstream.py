"""Pins of the oracle's end-of-step functions: the velocity correction
(Eq. unp1 on faces and cells), the phase pressures (Eqs. 37-38) and the
phase energies (Eq. 39).  Each pin is a fact of the mathematics or of the
paper: closed forms on polynomial fields, the Laplace jump and the mixture
identity of Eqs. 37-38, conservation of the total energy without surface
tension, and Eq. 17 + Eq. 28 tying the corrected divergence to the solve.
CPU only; nothing here uses the HIP library."""
import dataclasses

import numpy as np
import pytest

import oracle as orc
import workloads as W


def _op(dim, n, h, a_p, a_T):
    """Operator with the given cell coefficients (the block is not used by
    the end-of-step functions)."""
    N = int(np.prod(n))
    F = orc.faces_from_cells(dim, n, np.broadcast_to(a_p, (N,)), np.broadcast_to(a_T, (N,)))
    return orc.Operator(dim, tuple(n), h, F, np.zeros((4, N)))


def _coords(dim, n, h, a, faces_of=None):
    """x_a at cell centres, or at the faces across axis `faces_of` (x last)."""
    m = list(n[:dim])
    if faces_of is not None:
        m[faces_of] += 1
    shape = tuple(m[dim - 1 - b] for b in range(dim))
    off = 0.0 if faces_of == a else 0.5
    x = (np.arange(m[a]) + off) * h
    shp = [1] * dim
    shp[dim - 1 - a] = m[a]
    return np.broadcast_to(x.reshape(shp), shape).copy()


GRIDS = [(2, (9, 7, 1)), (3, (6, 5, 4))]


def _zero_faces(dim, n):
    return [np.zeros(orc.face_shape(dim, n, a)) for a in range(dim)]


@pytest.mark.parametrize("dim,n", GRIDS)
def test_divergence_closed_form(dim, n):
    """U_a = c_a x_a on every face: div = sum_a c_a exactly, in every cell."""
    h = 0.25
    c = [1.5, -0.75, 2.0][:dim]
    U = [c[a] * _coords(dim, n, h, a, faces_of=a) for a in range(dim)]
    d = orc.divergence(dim, n, h, U)
    assert np.allclose(d, sum(c), rtol=0, atol=1e-12)


@pytest.mark.parametrize("dim,n", GRIDS)
def test_projection_closed_form(dim, n):
    """Uniform 1/rho = alpha and p = b x_0^2: interior faces across x are
    corrected by -dt alpha 2 b x_f, wall faces and the other axes not at all;
    cell velocities by -dt alpha 2 b x_c (the mean of the two face values),
    except next to a wall, where one face value is zero."""
    h, dt, alpha, b = 0.5, 0.1, 2.0, 3.0
    op = _op(dim, n, h, alpha, 1.0)
    x = _coords(dim, n, h, 0)
    p = (b * x * x).reshape(-1)
    rng = np.random.default_rng(1)
    Us = [rng.uniform(-1, 1, orc.face_shape(dim, n, a)) for a in range(dim)]
    us = [rng.uniform(-1, 1, x.shape) for _ in range(dim)]
    U, u = orc.project(op, dt, p, Us, us)
    xf = _coords(dim, n, h, 0, faces_of=0)
    want = Us[0] - dt * alpha * 2 * b * xf
    want[..., 0] = Us[0][..., 0]
    want[..., -1] = Us[0][..., -1]
    assert np.allclose(U[0].reshape(want.shape), want, rtol=1e-13, atol=1e-12)
    for a in range(1, dim):
        assert np.array_equal(U[a].reshape(Us[a].shape), Us[a])
    g = alpha * 2 * b * xf                      # face values of (1/rho) dp/dx
    g[..., 0] = 0.0
    g[..., -1] = 0.0
    want_c = us[0] - dt * 0.5 * (g[..., :-1] + g[..., 1:])
    assert np.allclose(u[0].reshape(x.shape), want_c, rtol=1e-13, atol=1e-12)
    inner = want_c[..., 1:-1]
    assert np.allclose(inner, us[0][..., 1:-1] - dt * alpha * 2 * b * x[..., 1:-1], rtol=1e-13)
    for a in range(1, dim):
        assert np.array_equal(u[a].reshape(x.shape), us[a])


def test_phase_pressures_laplace_jump_and_mixture():
    """Eqs. 37-38: p1 - p2 = sigma kappa (the Laplace jump) and
    C p1 + (1 - C) p2 = p (the one-fluid pressure); pure cells keep p."""
    rng = np.random.default_rng(2)
    N = 200
    p = rng.uniform(1e4, 1e6, N)
    C = rng.uniform(0, 1, N)
    C[:10] = 0.0
    C[10:20] = 1.0
    kappa = rng.uniform(-5e3, 5e3, N)
    sigma = 0.072
    p1, p2 = orc.phase_pressures(p, C, kappa, sigma)
    assert np.allclose(p1 - p2, sigma * kappa, rtol=1e-9, atol=1e-9)
    assert np.allclose(C * p1 + (1 - C) * p2, p, rtol=1e-15, atol=0)
    assert np.array_equal(p2[:10], p[:10]) and np.array_equal(p1[10:20], p[10:20])
    q1, q2 = orc.phase_pressures(p, C, None, sigma)
    assert np.array_equal(q1, p) and np.array_equal(q2, p)


@pytest.mark.parametrize("dim,n", GRIDS)
def test_energy_pressure_work_closed_forms(dim, n):
    """Without heat flux (uniform T): uniform p = P and U_0 = c x_f give
    div(p u) = P c in every cell; p = s x_0 and U_0 = u0 on every face
    (walls included) give u0 s inside and u0 s / 2 in the wall cells (the
    wall face takes the cell's own pressure)."""
    h, dt = 0.5, 0.01
    N = int(np.prod(n))
    rng = np.random.default_rng(3)
    C = rng.uniform(0, 1, N)
    op = _op(dim, n, h, 1.0, 0.7)
    T = np.full(N, 300.0)
    zero = np.zeros(N)
    P, c = 2.0e5, 3.0
    U = _zero_faces(dim, n)
    U[0] = c * _coords(dim, n, h, 0, faces_of=0)
    p = np.full(N, P)
    E1, E2 = orc.energy_update(op, dt, C, p, p, T, U, zero, zero)
    assert np.allclose(E1, -dt * C * P * c, rtol=1e-12, atol=0)
    assert np.allclose(E2, -dt * (1 - C) * P * c, rtol=1e-12, atol=0)
    s, u0 = 40.0, -1.5
    x = _coords(dim, n, h, 0)
    p = (s * x).reshape(-1)
    U = _zero_faces(dim, n)
    U[0] = np.full(orc.face_shape(dim, n, 0), u0)
    E1, E2 = orc.energy_update(op, dt, C, p, p, T, U, zero, zero)
    div = np.full(x.shape, u0 * s)
    div[..., 0] = u0 * s / 2
    div[..., -1] = u0 * s / 2
    assert np.allclose(E1, -dt * C * div.reshape(-1), rtol=1e-12, atol=0)
    assert np.allclose(E2, -dt * (1 - C) * div.reshape(-1), rtol=1e-12, atol=0)


@pytest.mark.parametrize("dim,n", GRIDS)
def test_energy_heat_flux_closed_form(dim, n):
    """No flow, uniform k and T = a x_0^2: div(k grad T) = 2 a k in the
    interior; a wall cell has only its inner face's flux, no heat crosses
    the wall."""
    h, dt, k, a = 0.5, 0.01, 0.6, 7.0
    N = int(np.prod(n))
    C = np.random.default_rng(4).uniform(0, 1, N)
    op = _op(dim, n, h, 1.0, k)
    x = _coords(dim, n, h, 0)
    T = (a * x * x).reshape(-1)
    p = np.full(N, 1e5)
    zero = np.zeros(N)
    E1, E2 = orc.energy_update(op, dt, C, p, p, T, _zero_faces(dim, n), zero, zero)
    nx = n[0]
    lap = np.full(x.shape, 2 * a * k)
    # lower wall cell: flux k (T_1 - T_0)/h through its upper face only
    lap[..., 0] = k * a * ((1.5 * h) ** 2 - (0.5 * h) ** 2) / h / h
    xl, xm = (nx - 0.5) * h, (nx - 1.5) * h
    lap[..., -1] = -k * a * (xl ** 2 - xm ** 2) / h / h
    assert np.allclose(E1, dt * C * lap.reshape(-1), rtol=1e-12, atol=0)
    assert np.allclose(E2, dt * (1 - C) * lap.reshape(-1), rtol=1e-12, atol=0)


@pytest.mark.parametrize("dim,n", GRIDS)
def test_total_energy_conserved_without_surface_tension(dim, n):
    """Closed walls and sigma = 0: the phase updates sum to flux
    differences that cancel over the grid, so the total energy is
    conserved to rounding; with surface tension the phase pressures differ
    and it is not (the paper's conservation claim excludes that case)."""
    N = int(np.prod(n))
    rng = np.random.default_rng(5)
    h, dt = 1e-3, 1e-6
    op = _op(dim, n, h, rng.uniform(1e-3, 1.0, N), rng.uniform(0.02, 0.6, N))
    C = rng.uniform(0, 1, N)
    p = rng.uniform(1e5, 2e5, N)
    T = rng.uniform(290, 310, N)
    U = [rng.uniform(-1, 1, orc.face_shape(dim, n, a)) for a in range(dim)]
    for a in range(dim):
        sl = [slice(None)] * dim
        sl[dim - 1 - a] = 0
        U[a][tuple(sl)] = 0.0
        sl[dim - 1 - a] = -1
        U[a][tuple(sl)] = 0.0
    zero = np.zeros(N)
    p1, p2 = orc.phase_pressures(p, C)
    E1, E2 = orc.energy_update(op, dt, C, p1, p2, T, U, zero, zero)
    scale = np.abs(E1).sum() + np.abs(E2).sum()
    assert abs((E1 + E2).sum()) <= 1e-13 * scale
    p1, p2 = orc.phase_pressures(p, C, rng.uniform(1e3, 2e3, N), 50.0)
    E1, E2 = orc.energy_update(op, dt, C, p1, p2, T, U, zero, zero)
    assert abs((E1 + E2).sum()) > 1e-9 * scale


def test_pure_phase_cells_update_one_phase():
    """C = 1 everywhere: the gas energy is untouched (C_2 = 0), and the
    liquid energy takes the whole one-fluid update."""
    dim, n = 2, (8, 6, 1)
    N = 48
    rng = np.random.default_rng(6)
    op = _op(dim, n, 0.1, 1e-3, 0.6)
    C = np.ones(N)
    p, T = rng.uniform(1e5, 2e5, N), rng.uniform(290, 310, N)
    U = [rng.uniform(-1, 1, orc.face_shape(dim, n, a)) for a in range(dim)]
    E1a, E2a = rng.uniform(1e7, 2e7, N), rng.uniform(1e5, 2e5, N)
    E1, E2 = orc.energy_update(op, 1e-6, C, p, p, T, U, E1a, E2a)
    assert np.array_equal(E2, E2a)
    F1, _ = orc.energy_update(op, 1e-6, np.full(N, 0.5), p, p, T, U, E1a * 0, E2a * 0)
    assert np.allclose(E1 - E1a, 2 * F1, rtol=1e-12, atol=4 * np.spacing(E1a.max()))


@pytest.mark.parametrize("dim,n", [(2, (24, 20, 1)), (3, (8, 6, 10))])
def test_corrected_divergence_follows_eq17_and_the_solve(dim, n):
    """Eq. (17) with Eq. (28) at the solution: the divergence of the
    corrected face velocities equals dt [lambda_3 (p - p_adv) +
    lambda_4 div(k grad T)], i.e. the compressibility and thermal-dilation
    terms of Eq. (19).  A sign, a time-step factor or a face coefficient
    in the correction that differs from the solve's breaks it."""
    prob = W.state_problem("div", dim, n, [(0.5,) * dim], [0.3])
    op, b_p, b_T, p, T = orc.solve(prob)
    U, _ = orc.project(op, prob.dt, p, prob.uf_star)
    dU = orc.divergence(dim, prob.n, prob.h, U)
    l3, l4 = op.lam[2], op.lam[3]
    # div(k grad T): minus the T diffusion of the canonical operator
    op0 = dataclasses.replace(op, B=np.zeros_like(op.B))
    _, AT = orc.apply(op0, np.zeros(op.N), T)
    want = prob.dt * (l3 * (p - op.p_adv) + l4 * (-AT))
    dstar = orc.divergence(dim, prob.n, prob.h, prob.uf_star)
    scale = np.linalg.norm(dU) + np.linalg.norm(dstar)
    assert np.linalg.norm(dU - want) <= 1e-6 * scale
    assert np.linalg.norm(dU - dstar) > 1e-3 * scale     # the correction acts


# ----------------------------------------------- viscous work of Eq. (39)
# W = div(mu (grad u + grad u^T) . u) for the end-of-step velocity: closed
# forms on linear fields (interior cells, where the discrete fluxes of a
# linear field are exact), telescoping fluxes, second order on a smooth
# field with free-slip walls, and planted mistakes.
MU = (1.0e-3, 1.8e-5)          # water and air viscosities [Pa s]


def _vel_fields(dim, n, h, fn):
    """Cell velocities u_b = fn(b, x) and face velocities U_a = fn(a, x_face),
    except that wall faces carry zero normal velocity (closed walls)."""
    xc = [_coords(dim, n, h, a) for a in range(dim)]
    u = [fn(b, xc).reshape(-1) for b in range(dim)]
    U = []
    for a in range(dim):
        xf = [_coords(dim, n, h, b, faces_of=a) for b in range(dim)]
        Ua = fn(a, xf)
        sl = [slice(None)] * dim
        sl[dim - 1 - a] = 0
        Ua[tuple(sl)] = 0.0
        sl[dim - 1 - a] = -1
        Ua[tuple(sl)] = 0.0
        U.append(Ua.reshape(-1))
    return U, u


def _interior(dim, n, depth):
    """Mask of cells at least `depth` cells from every wall."""
    m = np.ones(tuple(n[dim - 1 - b] for b in range(dim)), bool)
    for a in range(dim):
        sl = [slice(None)] * dim
        ax = dim - 1 - a
        idx = np.arange(n[a])
        keep = (idx >= depth) & (idx < n[a] - depth)
        shp = [1] * dim
        shp[ax] = n[a]
        m &= keep.reshape(shp)
    return m.reshape(-1)


def _mix(C):
    return C * MU[0] + (1 - C) * MU[1]


@pytest.mark.parametrize("dim,n", [(2, (10, 9, 1)), (3, (7, 8, 6))])
@pytest.mark.parametrize("c", [1.0, 0.35])
def test_viscous_simple_shear(dim, n, c):
    """u = (gamma y, 0, 0): the stress is mu gamma on the shear faces and
    div(tau . u) = mu gamma^2 in every cell off the walls."""
    h, g = 0.2, 3.0
    op = _op(dim, n, h, 1.0, 1.0)
    C = np.full(op.N, c)
    U, u = _vel_fields(dim, n, h, lambda b, x: g * x[1] if b == 0 else 0.0 * x[0])
    Wv = orc.viscous_work(op, C, MU, U, u)
    inner = _interior(dim, n, 1)
    np.testing.assert_allclose(Wv[inner], _mix(c) * g * g, rtol=1e-12)


@pytest.mark.parametrize("dim,n", [(2, (10, 9, 1)), (3, (7, 8, 6))])
def test_viscous_planar_extension(dim, n):
    """u = eps (x, -y) in 2-D: tau = 2 mu eps diag(1, -1), div(tau . u) =
    4 mu eps^2; in 3-D u = eps (x, y, -2z): 12 mu eps^2, off the walls."""
    h, e = 0.2, 0.7
    op = _op(dim, n, h, 1.0, 1.0)
    C = np.full(op.N, 0.6)
    coef = (1.0, -1.0) if dim == 2 else (1.0, 1.0, -2.0)
    U, u = _vel_fields(dim, n, h, lambda b, x: e * coef[b] * x[b])
    Wv = orc.viscous_work(op, C, MU, U, u)
    inner = _interior(dim, n, 1)
    expect = (4.0 if dim == 2 else 12.0) * _mix(0.6) * e * e
    np.testing.assert_allclose(Wv[inner], expect, rtol=1e-12)


@pytest.mark.parametrize("dim,n", [(2, (10, 9, 1)), (3, (7, 8, 6))])
def test_viscous_rigid_translation_is_zero(dim, n):
    h = 0.2
    op = _op(dim, n, h, 1.0, 1.0)
    rng = np.random.default_rng(3)
    C = rng.uniform(0, 1, op.N)
    vel = [2.0, -1.5, 0.5][:dim]
    U, u = _vel_fields(dim, n, h, lambda b, x: vel[b] + 0.0 * x[0])
    assert np.abs(orc.viscous_work(op, C, MU, U, u)).max() == 0.0


@pytest.mark.parametrize("dim,n,axi", [(2, (10, 9, 1), 0), (3, (7, 8, 6), 0), (2, (10, 9, 1), 1)])
def test_viscous_fluxes_telescope(dim, n, axi):
    """Random velocities and fractions, closed walls: the face fluxes cancel
    in pairs, so the volume integral of the viscous work is zero (r-z: with
    the cell volumes proportional to the radius)."""
    h = 0.2
    op = _op(dim, n, h, 1.0, 1.0)
    op = orc.Operator(op.dim, op.n, op.h, op.F, op.B, axi=axi)
    rng = np.random.default_rng(4)
    C = rng.uniform(0, 1, op.N)
    U, u = _vel_fields(dim, n, h, lambda b, x: rng.standard_normal(x[0].shape))
    Wv = orc.viscous_work(op, C, MU, U, u)
    vol = np.ones(op.N)
    if axi:
        vol = np.repeat(np.arange(n[1]) + 0.5, n[0])
    scale = np.abs(Wv * vol).sum()
    assert scale > 0 and abs((Wv * vol).sum()) <= 1e-13 * scale


def _smooth_case(n, plant=None):
    """u = (a sin(pi x) cos(pi y), b cos(pi x) sin(pi y)) on the unit square
    (free slip on every wall), uniform mu: error of W against the analytic
    div(mu (grad u + grad u^T) . u) on the cells two or more from a wall."""
    a, b = 1.0, 0.4
    h = 1.0 / n
    op = _op(2, (n, n, 1), h, 1.0, 1.0)
    C = np.ones(op.N)
    pi = np.pi

    def f(comp, x):
        X, Y = x[0], x[1]
        if comp == 0:
            return a * np.sin(pi * X) * np.cos(pi * Y)
        return b * np.cos(pi * X) * np.sin(pi * Y)

    U, u = _vel_fields(2, (n, n, 1), h, f)
    Wv = orc.viscous_work(op, C, MU, U, u)
    X, Y = _coords(2, (n, n, 1), h, 0).reshape(-1), _coords(2, (n, n, 1), h, 1).reshape(-1)
    # analytic: tau_xx = 2 mu u_x, tau_yy = 2 mu v_y, tau_xy = mu (u_y + v_x);
    # W = d/dx(tau_xx u + tau_xy v) + d/dy(tau_xy u + tau_yy v)
    s, c = np.sin, np.cos
    u_ = a * s(pi * X) * c(pi * Y); v_ = b * c(pi * X) * s(pi * Y)
    ux = a * pi * c(pi * X) * c(pi * Y); uy = -a * pi * s(pi * X) * s(pi * Y)
    vx = -b * pi * s(pi * X) * s(pi * Y); vy = b * pi * c(pi * X) * c(pi * Y)
    uxx = -a * pi * pi * s(pi * X) * c(pi * Y); uyy = -a * pi * pi * s(pi * X) * c(pi * Y)
    uxy = -a * pi * pi * c(pi * X) * s(pi * Y)
    vxx = -b * pi * pi * c(pi * X) * s(pi * Y); vyy = -b * pi * pi * c(pi * X) * s(pi * Y)
    vxy = -b * pi * pi * s(pi * X) * c(pi * Y)
    mu = MU[0]
    txx, tyy, txy = 2 * mu * ux, 2 * mu * vy, mu * (uy + vx)
    dtxx_dx, dtyy_dy = 2 * mu * uxx, 2 * mu * vyy
    dtxy_dx, dtxy_dy = mu * (uxy + vxx), mu * (uyy + vxy)
    W_exact = (dtxx_dx * u_ + txx * ux + dtxy_dx * v_ + txy * vx
               + dtxy_dy * u_ + txy * uy + dtyy_dy * v_ + tyy * vy)
    inner = _interior(2, (n, n, 1), 2)
    return np.abs(Wv - W_exact)[inner].max() / np.abs(W_exact).max()


def test_viscous_second_order():
    errs = [_smooth_case(n) for n in (16, 32, 64)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, errs


def test_viscous_pins_reject_planted_mistakes():
    """grad u alone, or the stress without its tangential-gradient term,
    fail the closed forms or the convergence pin."""
    with orc.planted(4):       # mu grad u instead of mu (grad u + grad u^T)
        with pytest.raises(AssertionError):
            test_viscous_planar_extension(2, (10, 9, 1))
    with orc.planted(5):       # no tangential-gradient term in tau_ab
        assert _smooth_case(32) > 0.05
    assert _smooth_case(32) < 0.02
