"""Pins of the oracle's tangent-linear model: central finite differences of
the (pinned) forward oracle, and the closed form of the sub-critical regime."""
import numpy as np
import pytest

import coil_synth as cs
import oracle


def _run_obj(w, inp, nsteps):
    s = oracle.Sim(w, inp)
    assert s.run(nsteps) == 0
    sc = s.scalars()
    return np.array([sc["Q"], sc["T_peak"]]), s


def _fd(w, inp, dcw, dramp, nsteps, h):
    def perturbed(sign):
        i2 = dict(inp)
        i2["c_wire"] = inp["c_wire"] + sign * h * dcw
        coils = [cs.Coil(**{**c.__dict__, "ramp": c.ramp + sign * h * dramp[i]}) for i, c in enumerate(w.coils)]
        return _run_obj(w.replace(coils=coils), i2, nsteps)[0]
    return (perturbed(+1) - perturbed(-1)) / (2 * h)


def test_tangent_matches_central_differences_active():
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    nsteps = 250
    rng = np.random.Generator(np.random.PCG64(3))
    dcw = rng.standard_normal(w.n_wire)
    dramp = np.array([30.0])  # per coil
    obj, dobj = oracle.tangent(w, inp, dcw, dramp, nsteps)
    ref, s = _run_obj(w, inp, nsteps)
    assert np.allclose(obj, ref, rtol=0, atol=0)  # same primal
    assert s.scalars()["max_x"] > 1.0 and ref[1] > w.T_bath + 0.01
    fd = _fd(w, inp, dcw, dramp, nsteps, h=1e-6)
    assert dobj[0] == pytest.approx(fd[0], rel=2e-6)
    assert dobj[1] == pytest.approx(fd[1], rel=2e-5)


def test_tangent_ramp_only_and_zero_direction():
    w = cs.workload("c1_active").replace(coils=[cs.Coil(layers=2, turns=2, ne=4, ramp=1000.0)])
    inp = cs.generate(w)
    _, dobj0 = oracle.tangent(w, inp, np.zeros(w.n_wire), np.zeros(1), 120)
    assert dobj0 == (0.0, 0.0)
    _, dobj = oracle.tangent(w, inp, None, np.array([1.0]), 200)
    fd = _fd(w, inp, np.zeros(w.n_wire), np.array([1.0]), 200, h=1e-3)
    assert dobj[0] == pytest.approx(fd[0], rel=1e-6)


def test_subcritical_closed_form_dQ_dcw():
    """Deep in the sub-critical regime E does not feed back on the currents, so
    Q_w is proportional to c_w^(-n) and dQ/dc_w = -n Q_w / c_w."""
    w = cs.workload("c1")
    inp = cs.generate(w)
    nsteps = 60
    _, s = _run_obj(w, inp, nsteps)
    Qw = s.get(oracle.QW)
    for wire in (0, 7, 31):
        dcw = np.zeros(w.n_wire)
        dcw[wire] = 1.0
        _, dobj = oracle.tangent(w, inp, dcw, None, nsteps)
        assert dobj[0] == pytest.approx(-w.n * Qw[wire] / inp["c_wire"][wire], rel=1e-9)
