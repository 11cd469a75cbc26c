"""Pins of the oracle's field sum, local law, per-wire solve and heat step
against closed forms, invariants and limits that hold independently of the
oracle's code."""
import math

import numpy as np
import pytest

import coil_synth as cs
import oracle

MU0 = 4e-7 * math.pi


def _coil_workload(layers, turns, ne, **kw):
    coil_kw = {k: kw.pop(k) for k in list(kw) if k in ("r_inner", "wire_side", "ramp", "z_center")}
    return cs.Workload(name="t", coils=[cs.Coil(layers=layers, turns=turns, ne=ne, **coil_kw)],
                       steps=1, dt=kw.pop("dt", 1e-4), jc_disorder=("none", 0.0), **kw)


# ----------------------------------------------------------------- superposition
def test_discrete_solenoid_on_axis_equals_sum_of_ring_closed_forms():
    w = _coil_workload(3, 40, 1, r_inner=0.02, wire_side=1e-3)
    s = oracle.Sim(w)
    r, z = s.get(oracle.R), s.get(oracle.Z)
    I = cs.random_currents(s.N, seed=11)
    zq = np.array([-0.03, -0.005, 0.0, 0.0101, 0.05])
    br, bz = s.field_points(I, np.zeros_like(zq), zq)
    for k, zz in enumerate(zq):
        ref = np.sum(MU0 * I * r * r / (2 * (r * r + (zz - z) ** 2) ** 1.5))
        assert bz[k] == pytest.approx(ref, rel=1e-12)
        assert br[k] == 0.0


def test_long_solenoid_interior_field():
    # 1 layer x 2000 turns, pitch 1 mm, R = 20 mm: B at the centre on axis is
    # mu0 n I L / sqrt(L^2 + 4 R^2) (thin finite solenoid), -> mu0 n I as L -> inf
    layers, turns, pitch, Ir = 1, 2000, 1e-3, 3.0
    w = _coil_workload(layers, turns, 1, r_inner=0.02, wire_side=pitch)
    s = oracle.Sim(w)
    R = 0.02 + pitch / 2
    I = np.full(s.N, Ir)
    L = turns * pitch
    br, bz = s.field_points(I, np.array([0.0, 0.5 * R]), np.array([0.0, 0.0]))
    n = 1 / pitch
    finite = MU0 * n * Ir * L / math.sqrt(L * L + 4 * R * R)
    assert bz[0] == pytest.approx(finite, rel=1e-6)
    assert bz[0] == pytest.approx(MU0 * n * Ir, rel=5e-4)
    # off axis inside: uniform to O((R/L)^2)
    assert bz[1] == pytest.approx(MU0 * n * Ir, rel=5e-4)


def test_thick_winding_centre_field():
    # uniform J over a thick winding R1..R2, length L: on-axis centre field
    # mu0 J L/2 ln[(R2 + sqrt(R2^2 + L^2/4)) / (R1 + sqrt(R1^2 + L^2/4))]
    layers, turns, ne = 8, 16, 4
    w = _coil_workload(layers, turns, ne, r_inner=0.02, wire_side=1e-3)
    s = oracle.Sim(w)
    d = 1e-3 / ne
    J = 1e6
    I = np.full(s.N, J * d * d)
    R1, R2, L = 0.02, 0.02 + layers * 1e-3, turns * 1e-3
    ref = MU0 * J * L / 2 * math.log((R2 + math.sqrt(R2 ** 2 + L * L / 4)) /
                                     (R1 + math.sqrt(R1 ** 2 + L * L / 4)))
    _, bz = s.field_points(I, np.array([0.0]), np.array([0.0]))
    assert bz[0] == pytest.approx(ref, rel=2e-5)


def test_field_targets_match_points_and_exclude_self():
    w = _coil_workload(2, 3, 2)
    s = oracle.Sim(w)
    I = cs.random_currents(s.N, seed=3)
    tgt = np.arange(s.N)
    br, bz = s.field_targets(I, tgt)
    # the element's own ring is excluded: recompute with the own current zeroed
    r, z = s.get(oracle.R), s.get(oracle.Z)
    for e in [0, 5, s.N - 1]:
        I2 = I.copy()
        I2[e] = 0.0
        pbr, pbz = s.field_points(I2, r[e:e + 1], z[e:e + 1])
        assert br[e] == pytest.approx(pbr[0], rel=1e-13, abs=1e-20)
        assert bz[e] == pytest.approx(pbz[0], rel=1e-13, abs=1e-20)


# ----------------------------------------------------------------- local law
def test_local_law_derivative_and_critical_point():
    w = _coil_workload(2, 2, 4, Jc0=1e6, Tc=18.0, B0=1.0)
    inp = cs.generate(w.replace(seed=7, jc_disorder=("gauss", 0.01)))
    I0 = cs.random_currents(w.n_elem, seed=8, scale=0.05)
    base = oracle.Sim(w, inp)
    base.set(oracle.I, I0)
    base.step()
    Jc, E, Ep = base.get(oracle.JC), base.get(oracle.E), base.get(oracle.EP)
    d2 = (1e-3 / 4) ** 2
    # dE/dJ by central differences on one element's own current (its own B
    # excludes its own ring, so nothing else moves)
    for e in [0, 9, 31]:
        h = abs(I0[e]) * 1e-6
        vals = []
        for sgn in (+1, -1):
            sim = oracle.Sim(w, inp)
            I = I0.copy()
            I[e] += sgn * h
            sim.set(oracle.I, I)
            sim.step()
            vals.append(sim.get(oracle.E)[e])
        fd = (vals[0] - vals[1]) / (2 * h / d2)
        assert fd == pytest.approx(Ep[e], rel=1e-6)
    # at |J| = Jc exactly the power law gives E = Ec (any n)
    sim = oracle.Sim(w, inp)
    I = I0.copy()
    I[3] = -Jc[3] * d2
    sim.set(oracle.I, I)
    sim.step()
    assert sim.get(oracle.E)[3] == pytest.approx(-w.Ec, rel=1e-12)
    # Jc factors: T >= Tc with J != 0 is a non-finite condition
    sim = oracle.Sim(w, inp)
    sim.set(oracle.I, I0)
    sim.set(oracle.T, np.full(w.n_elem, 18.5))
    assert sim.step() == -4


def test_zero_current_gives_zero_field_and_E():
    w = cs.workload("c1")
    s = oracle.Sim(w, cs.generate(w))
    for f in (oracle.BR, oracle.BZ, oracle.E, oracle.EP):
        assert np.all(s.get(f) == 0.0)
    s.step()
    assert np.all(s.get(oracle.E) == 0.0)
    assert np.all(s.get(oracle.BZ) == 0.0)  # B^0 from I^0 = 0


# ----------------------------------------------------------------- per-wire solve
def test_wire_net_current_and_flux_identity():
    w = cs.workload("c1_active")
    s = oracle.Sim(w, cs.generate(w))
    s.run(180)  # past the onset of penetration
    I_prev = s.get(oracle.I)
    phi_prev = s.get(oracle.PHI)
    s.step()
    I = s.get(oracle.I)
    dI = s.get(oracle.DI)
    E, Ep = s.get(oracle.E), s.get(oracle.EP)
    U = s.get(oracle.UW)
    phi = s.get(oracle.PHI)
    r = s.get(oracle.R)
    d2 = (1e-3 / 4) ** 2
    dIt = w.coils[0].ramp * w.dt
    assert np.allclose(I - I_prev, dI, rtol=0, atol=1e-15 * np.abs(I).max())
    for wi in range(s.Nw):
        el = s.wire_elems(wi)
        assert dI[el].sum() == pytest.approx(dIt, rel=1e-12)
        # Faraday per ring with the linearised EMF: dPhi = -dt (2 pi r E_lin + U)
        elin = E[el] + Ep[el] * dI[el] / d2
        dphi = phi[el] - phi_prev[el]
        ref = -w.dt * (2 * math.pi * r[el] * elin + U[wi])
        assert np.allclose(dphi, ref, rtol=0, atol=1e-10 * np.abs(dphi).max())
    assert s.scalars()["max_x"] > 1.0


def test_perfect_screening_keeps_flux_differences():
    # Jc -> inf: E = 0, every ring of a wire sees the same dPhi = -dt U_w
    w = _coil_workload(2, 3, 3, Jc0=1e30, ramp=5.0)
    s = oracle.Sim(w)
    s.run(20)
    phi = s.get(oracle.PHI)
    for wi in range(s.Nw):
        el = s.wire_elems(wi)
        assert np.ptp(phi[el]) < 1e-12 * np.abs(phi[el]).max()
        assert abs(s.get(oracle.I)[el].sum() - 5.0 * 20 * 1e-4) < 1e-15


# ----------------------------------------------------------------- Bean
@pytest.mark.parametrize("n_exp,tol", [(30.0, 0.05), (100.0, 0.02)])
def test_bean_critical_state_magnetisation(n_exp, tol):
    """One wire at R ~ 1 m (planar limit) in a ramped axial field, zero
    transport current, Jc independent of B and T.  Bean's critical state:
    once fully penetrated, J = +-Jc split by the mid-plane of the wire
    parallel to the field, so the magnetisation per volume is Jc w / 4
    (opposing the field change), for a square bar of side w."""
    wside, ne, Jc = 1e-3, 16, 1e7
    Ec = 1e-4
    dBa = 4 * Ec / wside  # E ~ Ec at the edges
    w = cs.Workload(name="bean", coils=[cs.Coil(layers=1, turns=1, ne=ne, r_inner=1.0 - wside / 2,
                                                wire_side=wside, ramp=0.0)],
                    steps=1, dt=1e-4, Ec=Ec, n=n_exp, Jc0=Jc, Tc=1e30, B0=1e30,
                    dBa_dt=dBa, jc_disorder=("none", 0.0), eps_range=(0.0, 0.0))
    s = oracle.Sim(w)
    Bp = MU0 * Jc * wside / 2  # full-penetration field of the slab
    nsteps = int(3 * Bp / dBa / w.dt)
    s.run(nsteps)
    I, r = s.get(oracle.I), s.get(oracle.R)
    V = 2 * math.pi * 1.0 * wside * wside
    M = np.sum(math.pi * r * r * I) / V
    M_bean = -Jc * wside / 4
    assert abs(M / M_bean - 1) < tol
    assert abs(I.sum()) < 1e-12 * np.abs(I).sum()


# ----------------------------------------------------------------- heat
def _heat_workload(layers, turns, ne, dt, **kw):
    return _coil_workload(layers, turns, ne, dt=dt, ramp=0.0, cp_exp=0.0, h0=0.0,
                          C0=2e3, k0=0.5, T_bath=4.2, **kw)


def _gauss_error_1d(ne):
    w = _heat_workload(1, 64, ne, dt=1e-4)
    s = oracle.Sim(w)
    z = s.get(oracle.Z)
    A, sig0 = 0.5, 2e-3
    s.set(oracle.T, 4.2 + A * np.exp(-z * z / (2 * sig0 ** 2)))
    nsteps = 200
    s.run(nsteps)
    alpha = 0.5 / 2e3
    t = nsteps * w.dt
    sig2 = sig0 ** 2 + 2 * alpha * t
    ref = 4.2 + A * sig0 / math.sqrt(sig2) * np.exp(-z * z / (2 * sig2))
    return np.abs(s.get(oracle.T) - ref).max() / A


def test_heat_axisymmetric_z_gaussian_and_second_order():
    """A z-only Gaussian, uniform in r, with h = 0 and constant C is an exact
    solution of the axisymmetric heat equation (1-D diffusion along z);
    the finite-volume error must be small and fall as d^2."""
    e4 = _gauss_error_1d(4)
    e8 = _gauss_error_1d(8)
    assert e4 < 1e-3
    assert 3.0 < e4 / e8 < 5.0


def test_heat_planar_2d_gaussian():
    w = _heat_workload(48, 48, 2, dt=1e-4)
    s = oracle.Sim(w, planar=True)
    r, z = s.get(oracle.R), s.get(oracle.Z)
    r0 = 0.02 + 0.024
    A, sig0 = 0.3, 2e-3
    s.set(oracle.T, 4.2 + A * np.exp(-((r - r0) ** 2 + z * z) / (2 * sig0 ** 2)))
    nsteps = 100
    s.run(nsteps)
    sig2 = sig0 ** 2 + 2 * (0.5 / 2e3) * nsteps * w.dt
    ref = 4.2 + A * sig0 ** 2 / sig2 * np.exp(-((r - r0) ** 2 + z * z) / (2 * sig2))
    assert np.abs(s.get(oracle.T) - ref).max() / A < 2e-3


def test_heat_substep_rule():
    # diffusion number alpha dt / d^2 at T_bath with the 0.9 safety factor
    for name, expect in [("c1", 2), ("c2", 4)]:
        w = cs.workload(name)
        if name == "c2":
            w = w.replace(coils=[cs.Coil(layers=2, turns=2, ne=8)])  # same d, small grid
        s = oracle.Sim(w)
        assert s.n_sub == expect
    # C4's quotient is exactly 4.0 (d = 1/6 mm, dt = 1e-4)
    w = cs.workload("c4").replace(coils=[cs.Coil(layers=2, turns=2, ne=6)])
    assert oracle.Sim(w).n_sub == 4


# ----------------------------------------------------------------- energy
def test_energy_balance_active_run():
    """Enthalpy form: stored heat = integrated Joule heat - heat lost to the
    bath through the borders (interior fluxes cancel pairwise)."""
    w = cs.workload("c1_active")
    s = oracle.Sim(w, cs.generate(w))
    s.run(350)
    sc = s.scalars()
    assert sc["Q"] > 1e-4 and sc["T_peak"] > 4.25
    assert sc["stored"] == pytest.approx(sc["Q"] - sc["Q_out"], rel=1e-12)


def test_energy_balance_insulated_stored_equals_joule():
    w = cs.workload("c1_active").replace(h0=0.0)
    s = oracle.Sim(w, cs.generate(w))
    s.run(300)
    sc = s.scalars()
    assert sc["Q_out"] == 0.0
    assert sc["stored"] == pytest.approx(sc["Q"], rel=1e-12)
