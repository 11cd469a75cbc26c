"""Pins of the oracle's fully coupled A-V solve (every element current of the
coil enters every ring's flux; paper, Methods, "Numerical Algorithm": the
field of each subelement is updated from the net currents of all subelements
until the iteration converges).  The fluxes are recomputed in the tests from
the currents with an independent quadrature of Neumann's integral, so the
checks do not reuse the oracle's inductance matrix."""
import math

import numpy as np
import pytest

import coil_synth as cs
import oracle

MU0 = 4e-7 * math.pi


def _neumann_M(a, za, r, zr, npts=1 << 15):
    phi = np.arange(npts) * (2 * math.pi / npts)
    c = np.cos(phi)
    rho = np.sqrt(a * a + r * r - 2 * a * r * c + (za - zr) ** 2)
    return MU0 * a * r / 2 * np.sum(c / rho) * (2 * math.pi / npts)


def _inductance(s):
    """Full inductance matrix from Neumann's integral off the diagonal and the
    (separately pinned) square-section self inductance on it."""
    r, z = s.get(oracle.R), s.get(oracle.Z)
    d = math.sqrt(s.get(oracle.V)[0] / (2 * math.pi * r[0]))
    M = np.empty((s.N, s.N))
    for i in range(s.N):
        for j in range(s.N):
            M[i, j] = oracle.self_L(r[i], d) if i == j else _neumann_M(r[j], z[j], r[i], z[i])
    return M


def _wires(s):
    wire = np.empty(s.N, dtype=int)
    for wi in range(s.Nw):
        wire[s.wire_elems(wi)] = wi
    return wire


def test_single_wire_full_equals_transport():
    """With one wire there is no other wire: both couplings solve the same
    system, bitwise."""
    w = cs.workload("c1_active").replace(coils=[cs.Coil(layers=1, turns=1, ne=4, ramp=1000.0)])
    inp = cs.generate(w)
    a, b = oracle.Sim(w, inp), oracle.Sim(w.replace(coupling="full"), inp)
    assert a.run(300) == 0 and b.run(300) == 0
    for f in (oracle.I, oracle.T, oracle.PHI, oracle.BZ):
        assert np.array_equal(a.get(f), b.get(f))


def test_perfect_screening_uniform_flux_per_wire():
    """Jc -> infinity (E = 0): every ring of a wire sees the same flux change
    -dt U_w, so the true flux sum_j M_ej I_j of all currents is the same on all
    rings of a wire, while each wire carries the transport current.  The
    transport-only coupling does not have this property (it ignores the
    screening currents of the other wires)."""
    w = cs.Workload(name="scr", coils=[cs.Coil(layers=2, turns=2, ne=2, ramp=5.0)], steps=1, dt=1e-4,
                    Jc0=1e30, jc_disorder=("none", 0.0), coupling="full")
    s = oracle.Sim(w)
    M = _inductance(s)
    wire = _wires(s)
    assert s.run(20) == 0
    I = s.get(oracle.I)
    phi = M @ I
    assert np.allclose(s.get(oracle.PHI), phi, rtol=0, atol=1e-12 * np.abs(phi).max())
    for wi in range(s.Nw):
        assert np.ptp(phi[wire == wi]) <= 1e-12 * np.abs(phi).max()
        assert I[wire == wi].sum() == pytest.approx(5.0 * 20 * 1e-4, rel=1e-12)
    t = oracle.Sim(w.replace(coupling="transport"))
    assert t.run(20) == 0
    phi_t = M @ t.get(oracle.I)
    assert max(np.ptp(phi_t[wire == wi]) for wi in range(s.Nw)) > 1e-3 * np.abs(phi_t).max()


def test_resistive_circuit_equation_per_ring():
    """In the active regime, over one step every ring obeys the linearised
    circuit equation with the true flux of all currents:
    M (I^{k+1} - I^k) = -dt (2 pi r E_lin + U_w), E_lin = E + E' dI/d^2, with
    the constant dB_a = 0."""
    w = cs.workload("c1_active").replace(coils=[cs.Coil(layers=2, turns=3, ne=2, ramp=1000.0)], Jc0=5e7,
                                         coupling="full")
    inp = cs.generate(w)
    s = oracle.Sim(w, inp)
    M = _inductance(s)
    wire = _wires(s)
    assert s.run(150) == 0
    I0 = s.get(oracle.I)
    assert s.step() == 0
    I1, E, Ep, U = s.get(oracle.I), s.get(oracle.E), s.get(oracle.EP), s.get(oracle.UW)
    r = s.get(oracle.R)
    d2 = (1e-3 / 2) ** 2
    assert s.scalars()["max_x"] > 1.0
    dI = I1 - I0
    lhs = M @ dI
    rhs = -w.dt * (2 * math.pi * r * (E + Ep * dI / d2) + U[wire])
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-10 * np.abs(lhs).max())
    for wi in range(s.Nw):
        assert dI[wire == wi].sum() == pytest.approx(w.coils[0].ramp * w.dt, rel=1e-12)
