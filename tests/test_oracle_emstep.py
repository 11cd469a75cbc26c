"""Pins of the oracle's variable-step integration of the wire currents
(option em_tol: substeps dt / 2^m within a step, step-doubling error control,
local extrapolation; paper, Methods, Numerical Algorithm, last sentence: a
Runge-Kutta method with a variable time step for the electromagnetic
equations, against the divergences of the stiff power law).  Pinned by the
closed-form decay of a screening current under the power law, the reduction
to the fixed step where the law is linear, the error falling with the
tolerance, and the constraints and energy balance of an active run."""
import ctypes as C
import math

import numpy as np
import pytest

import coil_synth as cs
import oracle

WSIDE, NE, JC, EC, NEXP, R0 = 1e-3, 2, 1e7, 1e-4, 30.0, 100.0
D = WSIDE / NE
IC = JC * D * D


def _decay_workload(dt, **kw):
    """One wire of 2 x 2 elements at R = 100 m (the planar limit), no drive,
    Jc independent of B and T."""
    return cs.Workload(name="decay", coils=[cs.Coil(layers=1, turns=1, ne=NE, r_inner=R0 - WSIDE / 2,
                                                     wire_side=WSIDE, ramp=0.0)],
                       steps=1, dt=dt, Ec=EC, n=NEXP, Jc0=JC, Tc=1e30, B0=1e30, dBa_dt=0.0,
                       jc_disorder=("none", 0.0), eps_range=(0.0, 0.0), **kw)


def _mode_eigenvalue(s, v):
    """Rayleigh quotient of the wire's inductance matrix for the pattern v,
    the matrix built from the pinned ring functions (Maxwell's mutual
    inductance, the square-section self inductance)."""
    lib = oracle.lib()
    r, z = s.get(oracle.R), s.get(oracle.Z)
    n = r.size
    M = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            M[i, j] = (lib.orc_self_L(C.c_double(r[i]), C.c_double(D)) if i == j else
                       lib.orc_ring_M(C.c_double(r[j]), C.c_double(z[j]), C.c_double(r[i]), C.c_double(z[i])))
    assert np.linalg.norm(M @ v - (v @ M @ v) / (v @ v) * v) < 1e-4 * np.linalg.norm(M @ v)
    return float(v @ M @ v / (v @ v))


def _decay_error(dt, tol, T=2e-3):
    """Screening current +-i split by the wire's mid-plane r = R (a mode of
    the wire's inductance matrix by symmetry), decaying under
    lam di/dt = -2 pi R Ec (i/Ic)^n:
        i(t) = (i0^(1-n) + (n-1) 2 pi R Ec t / (lam Ic^n))^(-1/(n-1)).
    Returns the relative error of the amplitude at T and the substeps taken."""
    w = _decay_workload(dt, em_tol=tol, em_max_level=16)
    s = oracle.Sim(w)
    r = s.get(oracle.R)
    v = np.where(r < R0, 1.0, -1.0)
    lam = _mode_eigenvalue(s, v)
    i0 = 1.5 * IC
    s.set(oracle.I, i0 * v)
    subs = 0.0
    for _ in range(int(round(T / dt))):
        assert s.step() == 0
        subs += s.get(oracle.EMSUB).sum()
    amp = float((s.get(oracle.I) * v).sum() / v.size)
    a = 2 * math.pi * R0 * EC / (lam * IC ** NEXP)
    exact = (i0 ** (1 - NEXP) + (NEXP - 1) * a * T) ** (-1 / (NEXP - 1))
    return abs(amp - exact) / exact, subs


def test_power_law_decay_closed_form():
    """The fixed step of 1e-4 s is 3 % off in this stiff decay; the variable
    step at the same dt follows the closed form to the tolerance, with more
    substeps the tighter it is."""
    e_fixed, n_fixed = _decay_error(1e-4, 0.0)
    e3, n3 = _decay_error(1e-4, 1e-3)
    e5, n5 = _decay_error(1e-4, 1e-5)
    assert e_fixed > 1e-2 and n_fixed == 20
    assert e3 < 5e-5
    assert e5 < 2e-6
    assert n5 > n3 >= 20


def test_tolerance_controls_the_error():
    e2, _ = _decay_error(1e-4, 1e-2)
    e4, _ = _decay_error(1e-4, 1e-4)
    e6, _ = _decay_error(1e-4, 1e-6)
    assert e2 > e4 > e6
    assert e2 / e6 > 10


def test_linear_regime_equals_fixed_step():
    """The literal C1 configuration is deeply sub-critical (E' dt far below
    the inductances): the step is linear in the currents, so the variable
    step takes one substep per wire and reproduces the fixed step."""
    w = cs.workload("c1")
    inp = cs.generate(w)
    a = oracle.Sim(w, inp)
    b = oracle.Sim(w.replace(em_tol=1e-6), inp)
    assert a.run(100) == 0 and b.run(100) == 0
    for f in (oracle.I, oracle.PHI, oracle.UW, oracle.T):
        ref = a.get(f)
        assert np.abs(b.get(f) - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.all(b.get(oracle.EMSUB) == 1.0)


def test_active_run_constraints_energy_and_convergence():
    """Active C1 with the variable step: every wire carries I_t at every
    checkpoint, the energy balance is exact, some wires take several
    substeps, and the state converges as the tolerance tightens (first
    against the fixed step, then between tolerances)."""
    w, inp = cs.workload("c1_active"), None
    inp = cs.generate(w)
    runs = {}
    for tol in (1e-3, 1e-5, 1e-7):
        s = oracle.Sim(w.replace(em_tol=tol), inp)
        most = 0.0
        for k in range(300):
            assert s.step() == 0
            most = max(most, s.get(oracle.EMSUB).max())
        I = s.get(oracle.I)
        for wi in range(s.Nw):
            el = s.wire_elems(wi)
            assert abs(I[el].sum() - w.coils[0].ramp * w.dt * 300) <= 1e-12 * np.abs(I).max() * len(el)
        sc = s.scalars()
        assert sc["stored"] == pytest.approx(sc["Q"] - sc["Q_out"], rel=1e-12)
        runs[tol] = (I, most)
    ref = runs[1e-7][0]
    e3 = np.abs(runs[1e-3][0] - ref).max() / np.abs(ref).max()
    e5 = np.abs(runs[1e-5][0] - ref).max() / np.abs(ref).max()
    assert e5 < e3
    assert runs[1e-7][1] > runs[1e-5][1] > 1.0


def test_rejected_combinations():
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    for bad in (w.replace(em_tol=-1.0), w.replace(em_tol=1e-4, coupling="full"),
                w.replace(em_tol=1e-4, subelements=2), w.replace(em_tol=1e-4, em_max_level=40)):
        with pytest.raises(Exception):
            oracle.Sim(bad, inp)
    with pytest.raises(Exception):
        oracle.tangent(w.replace(em_tol=1e-4), inp, dramp=np.ones(1), nsteps=5)


def test_converges_to_fine_fixed_steps_with_drives():
    """Four wires of 2 x 2 elements under a transport ramp and a background
    ramp, with Jc independent of B and T, so that each wire's currents obey an
    ODE that does not depend on how time is stepped: 100 variable steps of
    1e-4 s at a tight tolerance land on 6400 fixed steps of dt/64 (the
    currents, the flux, and the Joule heat Q = sum q V dt), much closer than
    100 fixed steps do."""
    def run(dt, nsteps, tol):
        w = cs.Workload(name="drive", coils=[cs.Coil(layers=2, turns=2, ne=2, r_inner=0.02, wire_side=1e-3,
                                                      ramp=2000.0)],
                        steps=1, dt=dt, Ec=EC, n=NEXP, Jc0=2e7, Tc=1e30, B0=1e30, dBa_dt=0.5,
                        jc_disorder=("none", 0.0), eps_range=(0.0, 0.0), em_tol=tol, em_max_level=12)
        s = oracle.Sim(w)
        assert s.run(nsteps) == 0
        assert s.scalars()["max_x"] > 1.0
        return s.get(oracle.I), s.get(oracle.PHI), s.scalars()["Q"]

    I_ref, P_ref, Q_ref = run(1e-4 / 64, 6400, 0.0)
    I_a, P_a, Q_a = run(1e-4, 100, 1e-7)
    I_f, P_f, Q_f = run(1e-4, 100, 0.0)

    def err(a, b):
        return np.abs(a - b).max() / np.abs(b).max()
    assert err(I_a, I_ref) < 2e-4 and err(P_a, P_ref) < 2e-4 and abs(Q_a / Q_ref - 1) < 2e-3
    assert err(I_f, I_ref) > 10 * err(I_a, I_ref)
    assert abs(Q_f / Q_ref - 1) > 5 * abs(Q_a / Q_ref - 1)
