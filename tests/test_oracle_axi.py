"""Pins of the oracle's axisymmetric (r-z) metric: y is the radius from the
axis on the lower y wall, x the axial coordinate.  Each pin is a fact of
the cylindrical finite-volume operator: exact values of the discrete
Laplacian on polynomials, conservation and symmetry under the volume
weights, second-order convergence to the analytic cylindrical Laplacian,
the divergence of a radially linear flow, and Eq. 17 with Eq. 28 at the
axisymmetric solution.  CPU only; nothing here uses the HIP library."""
import dataclasses

import numpy as np
import pytest

import oracle as orc
import workloads as W


def _op(n, h, a_p=1.0, a_T=1.0, B=(0.0, 0.0, 0.0, 0.0), axi=1):
    N = n[0] * n[1]
    F = orc.faces_from_cells(2, n, np.full(N, a_p), np.full(N, a_T))
    Bm = np.repeat(np.asarray(B, dtype=np.float64)[:, None], N, axis=1)
    return orc.Operator(2, n, h, F, np.ascontiguousarray(Bm), axi=axi)


def _rz(n, h):
    """Cell-centre (r, z) arrays of shape (ny, nx): r along y, z along x."""
    r = ((np.arange(n[1]) + 0.5) * h)[:, None] * np.ones((1, n[0]))
    z = np.ones((n[1], 1)) * ((np.arange(n[0]) + 0.5) * h)[None, :]
    return r, z


def test_radial_laplacian_of_r_squared_is_four():
    """The cylindrical Laplacian of r^2 is 4, and the finite-volume form
    with face areas r_f and volumes r_c reproduces it exactly in every row
    but the outer wall's (the axis row included); z^2 gives 2."""
    n, h = (6, 9, 1), 0.3
    op = _op(n, h, a_T=0.7)
    r, z = _rz(n, h)
    zero = np.zeros(op.N)
    _, AT = orc.apply(op, zero, (r * r).reshape(-1))       # -div(a grad u)
    AT = AT.reshape(n[1], n[0])
    np.testing.assert_allclose(AT[:-1], -4 * 0.7, rtol=1e-12)
    _, AT = orc.apply(op, zero, (z * z).reshape(-1))
    AT = AT.reshape(n[1], n[0])
    np.testing.assert_allclose(AT[:, 1:-1], -2 * 0.7, rtol=1e-12)


def test_volume_weighted_conservation_and_symmetry():
    """With the cell volumes r_c as weights, the diffusion sums to zero over
    the grid (fluxes cancel across faces, none cross the axis or the walls)
    and is symmetric: <v, V A u> = <u, V A v>."""
    n, h = (7, 8, 1), 0.2
    N = n[0] * n[1]
    rng = np.random.default_rng(1)
    F = orc.faces_from_cells(2, n, rng.uniform(0.5, 2, N), rng.uniform(0.1, 1, N))
    op = orc.Operator(2, n, h, F, np.zeros((4, N)), axi=1)
    V = np.repeat((np.arange(n[1]) + 0.5)[:, None], n[0], axis=1).reshape(-1)
    u, v = rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)
    Ap, AT = orc.apply(op, u, v)
    scale = np.abs(V * Ap).sum()
    assert abs((V * Ap).sum()) <= 1e-13 * scale and abs((V * AT).sum()) <= 1e-13 * scale
    Au, _ = orc.apply(op, u, np.zeros(N))
    Av, _ = orc.apply(op, v, np.zeros(N))
    assert abs(v @ (V * Au) - u @ (V * Av)) <= 1e-12 * abs(v @ (V * Au))
    # without the metric the same weights break symmetry
    op0 = dataclasses.replace(op, axi=0)
    Au0, _ = orc.apply(op0, u, np.zeros(N))
    Av0, _ = orc.apply(op0, v, np.zeros(N))
    assert abs(v @ (V * Au0) - u @ (V * Av0)) > 1e-6 * abs(v @ (V * Au0))


def test_second_order_against_the_cylindrical_laplacian():
    """u = cos(pi r/R) cos(pi z/L) satisfies the wall conditions; with
    -lap u + u = f from the analytic cylindrical Laplacian, the discrete
    solution's error falls by about 4 per halving of h."""
    errs = []
    for m in (16, 32, 64):
        n = (m, m, 1)
        L = R = 1.0
        h = L / m
        op = _op(n, h, B=(1.0, 0.0, 0.0, 1.0))
        r, z = _rz(n, h)
        k = np.pi
        u = np.cos(k * r / R) * np.cos(k * z / L)
        lap = (-(k / R) ** 2 * u - (k / R) * np.sin(k * r / R) * np.cos(k * z / L) / r
               - (k / L) ** 2 * u)
        f = (-lap + u).reshape(-1)
        p, T = orc.direct_solve(op, f, f)
        errs.append(np.abs(p - u.reshape(-1)).max())
        np.testing.assert_allclose(p, T, rtol=0, atol=1e-12)
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.5 < q < 4.5 for q in ratios), (errs, ratios)


def test_divergence_of_radially_linear_flow():
    """U_r = c r on the radial faces: (1/r) d(r c r)/dr = 2c in every cell,
    the axis row included (no flux through r = 0)."""
    n, h, c = (5, 7, 1), 0.25, 1.5
    Ux = np.zeros(orc.face_shape(2, n, 0))
    Uy = c * (np.arange(n[1] + 1) * h)[:, None] * np.ones((1, n[0]))
    d = orc.divergence(2, n, h, [Ux, Uy], axi=1)
    np.testing.assert_allclose(d, 2 * c, rtol=1e-13)
    d0 = orc.divergence(2, n, h, [Ux, Uy], axi=0)
    np.testing.assert_allclose(d0, c, rtol=1e-13)


def test_energy_update_in_rz():
    """Uniform p = P and U_r = c r: div(p u) = 2 P c; closed walls and
    sigma = 0: the volume-weighted total energy is conserved."""
    n, h, dt = (6, 8, 1), 0.2, 1e-3
    N = n[0] * n[1]
    rng = np.random.default_rng(2)
    C = rng.uniform(0, 1, N)
    op = _op(n, h)
    P, c = 1e5, 2.0
    Ux = np.zeros(orc.face_shape(2, n, 0))
    Uy = c * (np.arange(n[1] + 1) * h)[:, None] * np.ones((1, n[0]))
    z = np.zeros(N)
    p = np.full(N, P)
    E1, E2 = orc.energy_update(op, dt, C, p, p, np.full(N, 300.0), [Ux, Uy], z, z)
    np.testing.assert_allclose(E1, -dt * C * 2 * P * c, rtol=1e-12)
    np.testing.assert_allclose(E2, -dt * (1 - C) * 2 * P * c, rtol=1e-12)
    # random flow inside closed walls, equal phase pressures (no surface
    # tension), random T: the volume-weighted total is conserved
    U = [rng.uniform(-1, 1, orc.face_shape(2, n, a)) for a in range(2)]
    U[0][:, 0] = U[0][:, -1] = 0.0
    U[1][0, :] = U[1][-1, :] = 0.0
    op = _op(n, h, a_T=0.4)
    V = np.repeat((np.arange(n[1]) + 0.5)[:, None], n[0], axis=1).reshape(-1)
    p = rng.uniform(1e5, 2e5, N)
    E1, E2 = orc.energy_update(op, dt, C, p, p, rng.uniform(290, 310, N), U, z, z)
    tot = V * (E1 + E2)
    assert abs(tot.sum()) <= 1e-13 * np.abs(tot).sum()


def test_corrected_divergence_follows_eq17_in_rz():
    """Eq. (17) with Eq. (28) at the axisymmetric solution: div U^{n+1} =
    dt [lambda_3 (p - p_adv) + lambda_4 div(k grad T)], all with the r-z
    metric (a bubble on the axis near the wall z = 0)."""
    prob = W.bubble_problem("axi", 2, (40, 24), [(0.3, 0.0)], [0.25], W.P0, 3 * W.P0)
    uf = W.face_velocities(2, prob.n, 5, 1.0, 1e-3)
    prob = dataclasses.replace(prob, uf_star=uf, axisymmetric=True)
    op, b_p, b_T, p, T = orc.solve(prob)
    assert op.axi == 1
    U, _ = orc.project(op, prob.dt, p, uf)
    dU = orc.divergence(2, prob.n, prob.h, U, axi=1)
    op0 = dataclasses.replace(op, B=np.zeros_like(op.B))
    _, AT = orc.apply(op0, np.zeros(op.N), T)
    p_adv = prob.p_adv.reshape(-1)
    want = prob.dt * (op.lam[2] * (p - p_adv) + op.lam[3] * (-AT))
    dstar = orc.divergence(2, prob.n, prob.h, uf, axi=1)
    scale = np.linalg.norm(dU) + np.linalg.norm(dstar)
    assert np.linalg.norm(dU - want) <= 1e-6 * scale
    # the Cartesian divergence of the same velocities does not satisfy it
    d_cart = orc.divergence(2, prob.n, prob.h, U, axi=0)
    assert np.linalg.norm(d_cart - want) > 1e-3 * scale


def test_mg_matches_direct_in_rz():
    """The oracle multigrid (its coarse levels rediscretised with the same
    metric) converges to the sparse direct solution."""
    prob = W.bubble_problem("axi", 2, (64, 48), [(0.25, 0.0)], [0.2], W.P0, 10 * W.P0,
                            div_amp=1e-6, div_seed=4)
    prob = dataclasses.replace(prob, axisymmetric=True)
    op = orc.assemble(prob)
    b_p, b_T = orc.rhs(op, prob)
    p_d, T_d = orc.direct_solve(op, b_p, b_T)
    p_m, T_m, cyc, _ = orc.mg_solve(op, b_p, b_T, rtol=1e-13, max_cycles=80)
    assert cyc > 0
    assert np.abs(p_m - p_d).max() <= 1e-8 * np.abs(p_d - prob.p_adv.reshape(-1)).max()
    assert np.abs(T_m - T_d).max() <= 1e-8
    rel = orc.relres(op, b_p, b_T, p_d, T_d)
    assert max(rel) <= 1e-12
