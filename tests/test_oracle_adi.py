"""Pins of the oracle's alternating-direction implicit heat step (paper,
Methods, heat paragraph: ADI on the composite cross-section with c, kappa
and h proportional to T^3): analytic diffusion solutions at time steps far
beyond the explicit limit, the Robin decay eigenvalue, the Kirchhoff-transform
solution of the T^3 laws, the insulation time constant between two wires, and
the exact energy balance."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import coil_synth as cs
import oracle


def _heat(layers, turns, ne, dt, **kw):
    base = dict(steps=1, dt=dt, cp_exp=0.0, h0=0.0, C0=2e3, k0=0.5, T_bath=4.2, jc_disorder=("none", 0.0),
                heat_solver="adi")
    base.update(kw)
    return cs.Workload(name="adi", coils=[cs.Coil(layers=layers, turns=turns, ne=ne, r_inner=0.02,
                                                   wire_side=1e-3, ramp=0.0)], **base)


def _gauss_z_error(ne, dt, nsteps, theta=False):
    """z-only Gaussian (uniform in r) in an insulated coil: an exact solution of
    the axisymmetric heat equation.  theta: C and k both proportional to T^3,
    for which the Kirchhoff variable theta = k0 T_ref/4 (T/T_ref)^4 obeys the
    linear heat equation with alpha = k0/C0."""
    kw = dict(cp_exp=3.0, k_exp=3.0) if theta else {}
    w = _heat(1, 64, ne, dt, **kw)
    s = oracle.Sim(w)
    z = s.get(oracle.Z)
    A, sig0, T0, k0, C0 = 0.5, 2e-3, 4.2, 0.5, 2e3
    alpha = k0 / C0
    if theta:
        th_b = k0 * T0 / 4
        th0 = th_b * (1 + A * np.exp(-z * z / (2 * sig0 ** 2)))
        s.set(oracle.T, T0 * (4 * th0 / (k0 * T0)) ** 0.25)
    else:
        s.set(oracle.T, T0 + A * np.exp(-z * z / (2 * sig0 ** 2)))
    assert s.run(nsteps) == 0
    t = nsteps * dt
    sig2 = sig0 ** 2 + 2 * alpha * t
    g = sig0 / math.sqrt(sig2) * np.exp(-z * z / (2 * sig2))
    if theta:
        ref = T0 * (4 * (k0 * T0 / 4) * (1 + A * g) / (k0 * T0)) ** 0.25
        return np.abs(s.get(oracle.T) - ref).max() / (ref.max() - T0)
    return np.abs(s.get(oracle.T) - (T0 + A * g)).max() / A


def test_adi_gaussian_large_steps_second_order():
    """Constant coefficients: at 25x the explicit stability limit the ADI step
    (Crank-Nicolson along z for this 1-D solution) stays accurate, and the
    error falls about 4x when d and dt both halve."""
    e1 = _gauss_z_error(4, 1e-3, 20)   # alpha dt / d^2 = 16 (explicit limit ~0.25 per direction)
    e2 = _gauss_z_error(8, 5e-4, 40)
    assert e1 < 3e-3
    assert 3.3 < e1 / e2 < 4.7


def test_adi_kirchhoff_T3_laws():
    """C and k proportional to T^3: the Kirchhoff variable diffuses linearly.
    The lagged (step-start) coefficients make the step first order in time for
    nonlinear laws: the error must still fall at least 2x per halving."""
    e1 = _gauss_z_error(4, 2e-4, 100, theta=True)
    e2 = _gauss_z_error(8, 1e-4, 200, theta=True)
    assert e1 < 2e-2
    assert e1 / e2 > 1.9


def _robin_lambda(h, k, L):
    return brentq(lambda x: x * math.tan(x * L / 2) - h / k, 1e-9, math.pi / L * (1 - 1e-12))


def _robin_adi_error(ne, dt):
    """Planar square with the Robin condition on all borders: the slowest mode
    of the ADI step decays per step by g = ((1 - tau mu)/(1 + tau mu))^2 (tau =
    dt/2, mu the mode's rate per direction); mu against the analytic
    alpha lambda^2, lambda tan(lambda L/2) = h/k."""
    L, k0, C0, h0 = 8e-3, 0.5, 2e3, 1000.0
    w = _heat(8, 8, ne, dt, h0=h0)
    s = oracle.Sim(w, planar=True)
    x = s.get(oracle.R) - (0.02 + L / 2)
    y = s.get(oracle.Z)
    lam = _robin_lambda(h0, k0, L)
    s.set(oracle.T, 4.2 + 0.1 * np.cos(lam * x) * np.cos(lam * y))
    assert s.run(10) == 0
    a1 = (s.get(oracle.T) - 4.2).sum()
    assert s.run(20) == 0
    a2 = (s.get(oracle.T) - 4.2).sum()
    g = (a2 / a1) ** (1.0 / 20)
    sg = math.sqrt(g)
    tau = dt / 2
    mu = (1 - sg) / (tau * (1 + sg))
    return mu / (k0 / C0 * lam * lam) - 1.0


def test_adi_robin_decay_rate():
    e2 = _robin_adi_error(2, 5e-4)
    e4 = _robin_adi_error(4, 5e-4)
    assert abs(e2) < 4e-3 and abs(e4) < 1e-3
    assert 3.7 < e2 / e4 < 4.3


def _insulation_decay_error(k0, nsteps=5):
    """Two wires side by side (planar), an insulation layer of resistance R per
    area between them, no bath, each wire starting isothermal: the difference
    of the wires' mean temperatures against the lumped two-node network with
    G = (interface length) / (R + 2 d/(2 k0)), stepped with the same implicit
    midpoint rule; the network is the limit of large k0."""
    ne, R, C0 = 4, 5e-4, 2e3
    w = cs.Workload(name="ins", coils=[cs.Coil(layers=1, turns=2, ne=ne, r_inner=0.02, wire_side=1e-3,
                                                ramp=0.0)],
                    steps=1, dt=1e-4, cp_exp=0.0, h0=0.0, C0=C0, k0=k0, T_bath=4.2, jc_disorder=("none", 0.0),
                    heat_solver="adi", ins_R0=R)
    s = oracle.Sim(w, planar=True)
    z = s.get(oracle.Z)
    s.set(oracle.T, np.where(z < 0, 5.0, 4.5))
    d = 1e-3 / ne
    rate = 2 * (1e-3 / (R + d / k0)) / (C0 * 1e-3 * 1e-3)
    assert s.run(nsteps) == 0
    T = s.get(oracle.T)
    d1 = T[z < 0].mean() - T[z > 0].mean()
    tau = w.dt / 2
    g = (1 - tau * rate) / (1 + tau * rate)
    return (d1 / 0.5) / g ** nsteps - 1.0


def test_adi_insulation_time_constant():
    e3 = _insulation_decay_error(1e3)
    e4 = _insulation_decay_error(1e4)
    assert abs(e4) < 2e-4
    assert 8.0 < e3 / e4 < 12.0  # the lumped limit is approached as 1/k0


def test_adi_energy_balance_with_T3_laws_and_source():
    """Joule heating of the active C1 run, C, k and h proportional to T^3, an
    insulation layer between wires and a composite conductivity map: the stored
    heat equals the Joule heat minus the border outflow to rounding."""
    w = cs.workload("c1_active").replace(heat_solver="adi", k_exp=3.0, h_exp=3.0, ins_R0=2e-4)
    s = oracle.Sim(w, cs.generate(w))
    km = np.where(np.arange(w.n_elem) % 3 == 0, 0.05, 1.0)
    s.set(oracle.KMULT, km)
    assert s.run(300) == 0
    sc = s.scalars()
    assert sc["T_peak"] > 4.25 and sc["n_sub"] == 1
    assert sc["stored"] == pytest.approx(sc["Q"] - sc["Q_out"], rel=1e-12)


def test_adi_stable_far_beyond_explicit_limit():
    """A bump with Robin borders and dt 400x the explicit limit: the
    volume-weighted norm of T - T_bath falls every step (unconditional
    stability).  The Peaceman-Rachford step is not monotone at such steps: the
    stiffest modes change sign from step to step, and T may dip below the bath
    for a few steps before they decay."""
    w = _heat(4, 8, 4, 2e-2, h0=500.0)
    s = oracle.Sim(w)
    r, z, V = s.get(oracle.R), s.get(oracle.Z), s.get(oracle.V)
    T0 = 4.2 + np.exp(-((r - 0.022) ** 2 + z ** 2) / (2 * 1e-3 ** 2))
    s.set(oracle.T, T0)
    prev = np.sqrt((V * (T0 - 4.2) ** 2).sum())
    for _ in range(40):
        assert s.step() == 0
        T = s.get(oracle.T)
        n = np.sqrt((V * (T - 4.2) ** 2).sum())
        assert n < prev
        prev = n
    assert np.abs(T - 4.2).max() < 1e-6
