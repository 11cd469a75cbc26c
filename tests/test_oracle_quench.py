"""Pins of the oracle's normal-state path and of its per-wire flux-jump and
quench diagnostics (paper, Methods, E-J paragraph: one law covering the flux
creep, flux flow and normal states; Results: the criteria |J/Jc| > 1 for the
nucleation of a flux jump in a wire and rho > 0.95 rho_n for its quench).

Reading: the power-law resistivity rho_pl = E/J = (Ec/Jc) (|J|/Jc)^(n-1) acts
in parallel with the normal-state resistivity rho_n,
rho = rho_pl rho_n / (rho_pl + rho_n); Jc <= 0 is the normal state."""
import math

import numpy as np
import pytest

import coil_synth as cs
import oracle


def _one_element(**kw):
    """One wire of one element (its own ring is excluded from its field, so
    B = B_a = 0), Jc independent of T and B (Tc, B0 -> infinity), no strain:
    Jc = Jc0 exactly."""
    d = 1e-3
    ramp = kw.pop("ramp", 0.0)
    I0 = kw.pop("I0", 0.0)
    base = dict(steps=1, dt=1e-5, Jc0=1e8, Tc=1e30, B0=1e30, n=30.0, Ec=1e-4,
                jc_disorder=("none", 0.0), eps_range=(0.0, 0.0))
    base.update(kw)
    return cs.Workload(name="one", coils=[cs.Coil(layers=1, turns=1, ne=1, r_inner=0.02, wire_side=d,
                                                   ramp=ramp, I0=I0)], **base)


def test_parallel_law_at_the_crossover():
    """Where the power-law resistivity equals rho_n the two paths carry equal
    shares: E = rho_n J / 2 and dE/dJ = rho_n (n + 1) / 4.  With
    rho_n = (Ec/Jc) 2^(n-1) that point is J = 2 Jc."""
    n, Ec, Jc = 30.0, 1e-4, 1e8
    rho_n = Ec / Jc * 2.0 ** (n - 1)
    w = _one_element(rho_n=rho_n)
    s = oracle.Sim(w)
    J = 2.0 * Jc
    s.set(oracle.I, np.array([J * 1e-6]))
    assert s.step() == 0
    assert s.get(oracle.JC)[0] == Jc
    assert s.get(oracle.E)[0] == pytest.approx(rho_n * J / 2, rel=1e-14)
    assert s.get(oracle.EP)[0] == pytest.approx(rho_n * (n + 1) / 4, rel=1e-13)


def test_normal_state_above_tc():
    """T > Tc gives Jc = 0: with rho_n the element is a normal metal, E = rho_n J
    and dE/dJ = rho_n, and the step succeeds; without rho_n the same state is
    the pure power law's non-finite condition."""
    w = _one_element(Tc=18.0, rho_n=3e-10)
    s = oracle.Sim(w)
    s.set(oracle.I, np.array([5.0]))
    s.set(oracle.T, np.array([20.0]))
    assert s.step() == 0
    assert s.get(oracle.JC)[0] == 0.0
    assert s.get(oracle.E)[0] == pytest.approx(3e-10 * 5.0e6, rel=1e-15)
    assert s.get(oracle.EP)[0] == 3e-10
    s2 = oracle.Sim(_one_element(Tc=18.0))
    s2.set(oracle.I, np.array([5.0]))
    s2.set(oracle.T, np.array([20.0]))
    assert s2.step() == -4


@pytest.mark.parametrize("x", [0.3, 1.0, 1.5, 2.0, 4.0])
def test_parallel_law_derivative(x):
    """dE/dJ against central differences of E(J) across the flux-creep,
    crossover and flux-flow ranges."""
    n, Ec, Jc = 30.0, 1e-4, 1e8
    rho_n = Ec / Jc * 2.0 ** (n - 1)

    def E_of(J):
        s = oracle.Sim(_one_element(rho_n=rho_n))
        s.set(oracle.I, np.array([J * 1e-6]))
        assert s.step() == 0
        return s.get(oracle.E)[0], s.get(oracle.EP)[0]

    J = x * Jc
    h = J * 1e-6
    Ep = E_of(J)[1]
    fd = (E_of(J + h)[0] - E_of(J - h)[0]) / (2 * h)
    assert fd == pytest.approx(Ep, rel=1e-7)
    # limits: far below the crossover the power law, far above rho_n
    E, _ = E_of(J)
    p = Ec / Jc * x ** (n - 1)
    assert E / J < min(p, rho_n) * (1 + 1e-15)
    assert E / J > min(p, rho_n) / 2 * (1 - 1e-15)


def test_onset_and_quench_steps_closed_form():
    """One element carries the transport current itself: I^k = I0 + ramp k dt =
    (k + 1/2) A with Ic = Jc d^2 = 100 A, so |J|/Jc = (k + 1/2)/100 first
    exceeds 1 at k = 100.  With rho_n = (Ec/Jc) 1.5^(n-1) / 19 the resistivity
    rho_n p/(p + rho_n) first exceeds 0.95 rho_n where p = 19 rho_n, i.e. where
    |J|/Jc > 1.5: at k = 150.  The recorded heat, temperature and power are the
    wire's values at those steps (before the step's own Joule heat)."""
    n, Ec, Jc = 30.0, 1e-4, 1e8
    rho_n = Ec / Jc * 1.5 ** (n - 1) / 19.0
    w = _one_element(rho_n=rho_n, ramp=1e5, I0=0.5, C0=2e7)
    s = oracle.Sim(w)
    assert s.get(oracle.I)[0] == 0.5
    assert s.run(100) == 0
    Qw100 = s.get(oracle.QW)[0]
    assert s.get(oracle.ONSET)[0] == -1.0
    assert s.step() == 0
    assert s.get(oracle.ONSET)[0] == 100.0 and s.get(oracle.Q_ONSET)[0] == Qw100
    assert s.run(49) == 0
    I150, T150, Qw150 = s.get(oracle.I)[0], s.get(oracle.T)[0], s.get(oracle.QW)[0]
    assert I150 == pytest.approx(150.5, rel=1e-14)
    assert s.get(oracle.QUENCH)[0] == -1.0
    assert s.step() == 0
    assert s.get(oracle.QUENCH)[0] == 150.0
    assert s.get(oracle.Q_QUENCH)[0] == Qw150 and s.get(oracle.T_QUENCH)[0] == T150
    E150 = s.get(oracle.E)[0]
    assert s.get(oracle.P_QUENCH)[0] == pytest.approx(E150 * I150 / 1e-6, rel=1e-14)
    assert E150 / (I150 / 1e-6) > 0.95 * rho_n
    assert s.get(oracle.ONSET)[0] == 100.0  # first crossing only


def _quench4():
    """Small quench case: 4 layers x 4 turns of 4x4 elements, driven like the
    paper's quench study (transport ramp plus a background field ramp, both
    1000x faster than 2 A/s and 0.015 T/s), Jc0 = 5e8, rho_n = 3e-10 Ohm m."""
    return cs.Workload(name="quench4", coils=[cs.Coil(layers=4, turns=4, ne=4, ramp=2000.0)], steps=2000,
                       dt=5e-5, Jc0=5e8, dBa_dt=15.0, rho_n=3e-10, jc_disorder=("lognormal", 0.02), seed=7)


def test_quench_runs_through_tc_with_energy_balance():
    """Past Tc the normal-state path carries the current: the run completes,
    every wire nucleates and then quenches, T exceeds Tc, and the stored heat
    still equals the Joule heat minus the heat lost through the borders."""
    w = _quench4()
    s = oracle.Sim(w, cs.generate(w))
    assert s.run(w.steps) == 0
    sc = s.scalars()
    on, qu = s.get(oracle.ONSET), s.get(oracle.QUENCH)
    assert np.all(on >= 0) and np.all(qu >= 0) and np.all(qu >= on)
    assert sc["T_peak"] > 12.0
    assert sc["stored"] == pytest.approx(sc["Q"] - sc["Q_out"], rel=1e-12)
    assert np.all(s.get(oracle.Q_QUENCH) >= s.get(oracle.Q_ONSET))


def test_tangent_with_normal_state_path():
    """Tangent-linear model through the parallel law (flux-flow range reached)
    against central differences."""
    w = cs.workload("c1_active").replace(rho_n=3e-12)
    inp = cs.generate(w)
    nsteps = 250
    rng = np.random.Generator(np.random.PCG64(5))
    dcw = rng.standard_normal(w.n_wire)
    dramp = np.array([30.0])
    obj, dobj = oracle.tangent(w, inp, dcw, dramp, nsteps)

    def run(sign, h):
        i2 = dict(inp)
        i2["c_wire"] = inp["c_wire"] + sign * h * dcw
        coils = [cs.Coil(**{**c.__dict__, "ramp": c.ramp + sign * h * dramp[0]}) for c in w.coils]
        s = oracle.Sim(w.replace(coils=coils), i2)
        assert s.run(nsteps) == 0
        sc = s.scalars()
        return np.array([sc["Q"], sc["T_peak"]]), s

    h = 1e-6
    (qp, _), (qm, s) = run(+1, h), run(-1, h)
    fd = (qp - qm) / (2 * h)
    # the parallel path is active: some element's E/J is within a factor 10 of rho_n
    E, I = s.get(oracle.E), s.get(oracle.I)
    rho = np.abs(E) / np.maximum(np.abs(I) / (1e-3 / 4) ** 2, 1e-30)
    assert rho.max() > 0.1 * 3e-12
    assert dobj[0] == pytest.approx(fd[0], rel=2e-6)
    assert dobj[1] == pytest.approx(fd[1], rel=2e-5)
