"""Pins of the oracle's provisional-state functions (state mode): Eqs. (20)
and (23) invert the NASG equation of state, Eq. (11) is the isentropic
derivative of that EoS, and the state-mode block is built from them.  CPU
only; nothing here uses the HIP library."""
import numpy as np
import pytest

import oracle as orc
import workloads as W

import dataclasses

LIQ, GAS = W.LIQUID_NASG, W.GAS_IDEAL
# Table 1 rounds Gamma (4285 / 3610 = 1.187 against 1.19): with c_p - c_v =
# (Gamma - 1) c_v the denominator of Eq. (23) is the thermal coefficient of
# the EoS behind Eq. (10), and the round trip is exact
LIQ_C = dataclasses.replace(LIQ, cp=LIQ.Gamma * LIQ.cv)


def nasg_density(ph, p, T):
    """Density of the NASG phase at (p, T): the specific volume
    v = (Gamma - 1) c_v T / (p + Pi) + b of the EoS behind Eq. (10)."""
    return 1.0 / ((ph.Gamma - 1.0) * ph.cv * T / (p + ph.Pi) + ph.b)


def nasg_energy(ph, rho, p):
    """Specific internal energy from Eq. (9):
    rho e = (p + Gamma Pi)(1 - rho b)/(Gamma - 1) + rho q."""
    return ((p + ph.Gamma * ph.Pi) * (1.0 - rho * ph.b) / (ph.Gamma - 1.0) + rho * ph.q) / rho


def nasg_pressure(ph, rho, e):
    """Eq. (9) solved for p at given (rho, e)."""
    return (rho * (e - ph.q)) * (ph.Gamma - 1.0) / (1.0 - rho * ph.b) - ph.Gamma * ph.Pi


def _conserved(C, p, T, u, liq=LIQ):
    """Conserved variables of cells at phase equilibrium (p, T), velocity u."""
    r1 = nasg_density(liq, p, T)
    r2 = nasg_density(GAS, p, T)
    e1 = nasg_energy(liq, r1, p)
    e2 = nasg_energy(GAS, r2, p)
    m1, m2 = C * r1, (1.0 - C) * r2
    rho = m1 + m2
    u2 = sum(ui * ui for ui in u)
    E = m1 * e1 + m2 * e2 + 0.5 * rho * u2
    return m1, m2, E, [rho * ui for ui in u]


def _problem(C, m1, m2, E, mom, dim=2, liq=LIQ):
    n = C.size
    return W.Problem(name="pin", dim=dim, n=(n, 1, 1), h=1e-5, mode="state", C=C,
                     liquid=liq, gas=GAS, dt=1e-9, m1=m1, m2=m2, E=E, mom=mom)


def test_state_inverts_the_nasg_eos():
    """Eqs. (20), (23) return the (p, T) the conserved variables were built
    from, for pure and mixed cells at phase equilibrium, moving or not."""
    rng = np.random.default_rng(3)
    n = 400
    C = rng.uniform(0, 1, n)
    C[:40] = 0.0
    C[40:80] = 1.0
    p = W.P0 * 10 ** rng.uniform(-0.3, 1.7, n)
    T = rng.uniform(280.0, 420.0, n)
    u = [rng.uniform(-5, 5, n), rng.uniform(-5, 5, n)]
    m1, m2, E, mom = _conserved(C, p, T, u, LIQ_C)
    P, TT = orc.state(_problem(C, m1, m2, E, mom, liq=LIQ_C))
    # the liquid's energy scale is ~1e9 J/m^3 against p ~ 1e5: rounding of
    # the differences of Eq. (20) bounds the agreement
    scale = np.abs(E) + np.abs(C * LIQ.Gamma * LIQ.Pi / (LIQ.Gamma - 1.0))
    den = C * (1 - m1 / np.where(C > 0, C, 1) * LIQ.b) / (LIQ.Gamma - 1) + (1 - C) / (GAS.Gamma - 1)
    assert np.all(np.abs(P - p) <= 1e-14 * 64 * scale / den + 1e-12 * p)
    assert np.all(np.abs(TT - T) <= 1e-9 * T)


def test_temperature_as_printed_with_table1():
    """With Table 1 as printed, Eq. (23) divides by rho (c_p - c_v) while the
    EoS of Eq. (10) has (Gamma - 1) c_v: a pure liquid cell built at
    (p, T) returns T (Gamma - 1) c_v / (c_p - c_v) (1.6 % above), and the
    pressure exactly."""
    n = 12
    C = np.ones(n)
    p = W.P0 * np.linspace(0.5, 30, n)
    T = np.linspace(285, 360, n)
    m1, m2, E, mom = _conserved(C, p, T, [np.zeros(n), np.zeros(n)])
    P, TT = orc.state(_problem(C, m1, m2, E, mom))
    ratio = (LIQ.Gamma - 1.0) * LIQ.cv / (LIQ.cp - LIQ.cv)
    assert np.allclose(TT, T * ratio, rtol=1e-10)
    assert np.allclose(P, p, rtol=1e-8)


def test_ideal_gas_closed_form():
    """A pure ideal-gas cell: p = (gamma - 1)(E - 1/2 |mom|^2 / rho) and
    T = p / (rho (c_p - c_v))."""
    rng = np.random.default_rng(4)
    n = 50
    C = np.zeros(n)
    rho = rng.uniform(0.1, 30, n)
    e = rng.uniform(1e5, 5e5, n)
    u = rng.uniform(-20, 20, n)
    m1, m2 = np.zeros(n), rho
    mom = [rho * u]
    E = rho * e + 0.5 * rho * u * u
    P, TT = orc.state(_problem(C, m1, m2, E, mom, dim=1 + 1))
    # dim 2 with a zero second momentum component
    P2, TT2 = orc.state(_problem(C, m1, m2, E, mom + [np.zeros(n)]))
    p_ref = (GAS.gamma - 1.0) * (E - 0.5 * mom[0] ** 2 / rho)
    assert np.allclose(P2, p_ref, rtol=1e-13, atol=0)
    assert np.allclose(TT2, p_ref / (rho * (GAS.cp - GAS.cv)), rtol=1e-13, atol=0)


def test_state_is_galilean():
    """Moving a cell (momentum with its kinetic energy added to E) leaves
    the provisional state unchanged."""
    rng = np.random.default_rng(5)
    n = 100
    C = rng.uniform(0, 1, n)
    p = W.P0 * rng.uniform(0.5, 20, n)
    T = rng.uniform(290, 350, n)
    m1, m2, E0, _ = _conserved(C, p, T, [np.zeros(n), np.zeros(n)])
    rho = m1 + m2
    u = [rng.uniform(-3, 3, n), rng.uniform(-3, 3, n)]
    E1 = E0 + 0.5 * rho * (u[0] ** 2 + u[1] ** 2)
    P0, T0 = orc.state(_problem(C, m1, m2, E0, None))
    P1, T1 = orc.state(_problem(C, m1, m2, E1, [rho * u[0], rho * u[1]]))
    assert np.allclose(P1, P0, rtol=1e-9, atol=1e-3) and np.allclose(T1, T0, rtol=1e-11)


@pytest.mark.parametrize("ph", [LIQ, GAS], ids=["liquid", "gas"])
def test_sound_speed_is_isentropic_derivative(ph):
    """Eq. (11) equals dp/drho at constant entropy of the EoS of Eq. (9):
    c^2 = (dp/drho)_e + (p / rho^2) (dp/de)_rho, by central differences."""
    for p, T in ((W.P0, 293.15), (50 * W.P0, 350.0), (0.3 * W.P0, 300.0)):
        rho = nasg_density(ph, p, T)
        e = nasg_energy(ph, rho, p)
        dr, de = 1e-6 * rho, 1e-6 * abs(e - ph.q)
        dpdr = (nasg_pressure(ph, rho + dr, e) - nasg_pressure(ph, rho - dr, e)) / (2 * dr)
        dpde = (nasg_pressure(ph, rho, e + de) - nasg_pressure(ph, rho, e - de)) / (2 * de)
        c2 = dpdr + p / rho ** 2 * dpde
        assert orc.sound2(ph, rho, p) == pytest.approx(c2, rel=1e-6)


def test_state_mode_block_of_pure_cells():
    """Pure cells: B_pp = gamma / (rho c^2 dt^2) with c^2 the isentropic
    derivative, B_TT = rho c_p / dt with rho = m_i / C_i, a_p = 1 / rho."""
    rng = np.random.default_rng(6)
    n = 20
    C = np.array([1.0] * 10 + [0.0] * 10)
    p = W.P0 * rng.uniform(0.5, 20, n)
    T = rng.uniform(290, 350, n)
    m1, m2, E, mom = _conserved(C, p, T, [np.zeros(n), np.zeros(n)])
    prob = _problem(C, m1, m2, E, mom)
    op = orc.assemble(prob)
    dt = prob.dt
    for i in range(n):
        ph = LIQ if C[i] == 1 else GAS
        rho = m1[i] if C[i] == 1 else m2[i]
        e = nasg_energy(ph, rho, op.p_adv[i])
        dr, de = 1e-6 * rho, 1e-6 * abs(e - ph.q)
        c2 = ((nasg_pressure(ph, rho + dr, e) - nasg_pressure(ph, rho - dr, e)) / (2 * dr)
              + op.p_adv[i] / rho ** 2 * (nasg_pressure(ph, rho, e + de)
                                          - nasg_pressure(ph, rho, e - de)) / (2 * de))
        assert op.B[0, i] == pytest.approx(ph.gamma / (rho * c2 * dt * dt), rel=1e-6)
        assert op.B[3, i] == pytest.approx(rho * ph.cp / dt, rel=1e-14)
        assert op.a_p[i] == pytest.approx(1.0 / rho, rel=1e-15)


def test_state_mode_mixed_block_is_fraction_average():
    """A mixed cell's block is the fraction average of the pure-phase
    blocks built at the phase densities m_i / C_i (phases-mode functions
    with those densities and Eq. (11) sound speeds)."""
    rng = np.random.default_rng(7)
    n = 30
    C = rng.uniform(0.05, 0.95, n)
    p = W.P0 * rng.uniform(0.5, 20, n)
    T = rng.uniform(290, 350, n)
    m1, m2, E, mom = _conserved(C, p, T, [np.zeros(n), np.zeros(n)])
    prob = _problem(C, m1, m2, E, mom)
    op = orc.assemble(prob)
    import dataclasses
    for i in range(n):
        blocks = []
        for ph, m, c in ((LIQ, m1[i], C[i]), (GAS, m2[i], 1 - C[i])):
            rho = m / c
            php = dataclasses.replace(ph, rho=rho, c=float(np.sqrt(orc.sound2(ph, rho, op.p_adv[i]))))
            lam = orc.phase_lambdas(php, op.p_adv[i], op.T_adv[i], prob.dt)
            blocks.append(np.array([-lam[2] + lam[3] * lam[1], lam[3] * lam[0], -lam[1], -lam[0]]))
        ref = C[i] * blocks[0] + (1 - C[i]) * blocks[1]
        assert np.allclose(op.B[:, i], ref, rtol=1e-13, atol=0)


def test_state_problem_solve_matches_direct():
    prob = W.state_problem("s", 2, (48, 40), [(0.45, 0.5)], [0.2], gas_atm=10, seed=9)
    op, b_p, b_T, p_ref, T_ref = orc.solve(prob, rtol=1e-14)
    f_p, f_T = orc.canonical_rhs(op, b_p, b_T)
    p_mg, T_mg, cyc, _ = orc.mg_solve(op, b_p, b_T, rtol=1e-14)
    assert np.max(np.abs(p_mg - p_ref)) <= 1e-9 * np.max(np.abs(p_ref))
    assert np.max(np.abs(T_mg - T_ref)) <= 1e-12 * np.max(np.abs(T_ref))
    assert 0.8 * W.P0 < p_ref.mean() < 12 * W.P0 and 280 < T_ref.mean() < 320
