"""Pins of three oracle parts that the field, A-V and heat pins above do not
reach: the Robin border conductance of the heat step, the transport-flux
pattern Psi_u of the per-wire drive, and the three factors of Jc(B, T, eps).
Each is checked against a value fixed outside the oracle's code: an analytic
eigenvalue, an independent quadrature of Neumann's double line integral, and
literal numbers of the benchmark's Jc formula."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import coil_synth as cs
import oracle

MU0 = 4e-7 * math.pi


# ----------------------------------------------------------------- Robin border
def _robin_lambda(h, k, L):
    """Smallest lambda of X'' = -lambda^2 X on [0, L], symmetric about L/2, with
    -k X' = h X at both walls (heat lost to the bath through a film
    coefficient h): lambda tan(lambda L / 2) = h / k."""
    return brentq(lambda x: x * math.tan(x * L / 2) - h / k, 1e-9, math.pi / L * (1 - 1e-12))


def _robin_decay_error(ne, h0):
    """Planar square of side L = 8 mm, Robin condition h0 on all four borders,
    constant C and k, no source.  The slowest mode decays at
    alpha (lambda_x^2 + lambda_y^2); the oracle's rate is read from the decay of
    the stored heat over 200 steps (per explicit substep: factor 1 - h_s mu)."""
    L, k0, C0 = 8e-3, 0.5, 2e3
    w = cs.Workload(name="robin", coils=[cs.Coil(layers=8, turns=8, ne=ne, r_inner=0.02, wire_side=1e-3,
                                                  ramp=0.0)],
                    steps=1, dt=1e-4, cp_exp=0.0, h0=h0, C0=C0, k0=k0, T_bath=4.2,
                    jc_disorder=("none", 0.0))
    s = oracle.Sim(w, planar=True)
    x = s.get(oracle.R) - (0.02 + L / 2)
    y = s.get(oracle.Z)
    lam = _robin_lambda(h0, k0, L)
    s.set(oracle.T, 4.2 + 0.1 * np.cos(lam * x) * np.cos(lam * y))
    s.run(100)
    a1 = (s.get(oracle.T) - 4.2).sum()
    nstep = 200
    s.run(nstep)
    a2 = (s.get(oracle.T) - 4.2).sum()
    hs = w.dt / s.n_sub
    mu = (1.0 - (a2 / a1) ** (1.0 / (nstep * s.n_sub))) / hs
    return mu / (k0 / C0 * 2 * lam * lam) - 1.0


@pytest.mark.parametrize("h0", [250.0, 1000.0])
def test_robin_border_decay_rate_second_order(h0):
    """The border face conductance area / (1/h + d/(2k)) (film in series with
    the half cell) makes the finite-volume decay rate converge to the analytic
    Robin eigenvalue at second order; a conductance without the half cell, or
    with the film alone, converges at first order only (paper, Methods, heat
    paragraph: Robin condition h (T - T0) on the four borders)."""
    e2 = _robin_decay_error(2, h0)
    e4 = _robin_decay_error(4, h0)
    assert abs(e2) < 4e-3 and abs(e4) < 1e-3
    assert 3.7 < e2 / e4 < 4.3


# ----------------------------------------------------------------- Psi_u
def _neumann_M(a, za, r, zr, npts=1 << 16):
    """Mutual inductance of two coaxial filament rings from Neumann's formula
    M = mu0/(4 pi) double-integral dl1.dl2 / |x1 - x2|, reduced to one angle:
    mu0 a r / 2 * int_0^{2 pi} cos(phi) / sqrt(a^2 + r^2 - 2 a r cos(phi) + dz^2),
    trapezoid rule (spectrally accurate for a smooth periodic integrand)."""
    phi = np.arange(npts) * (2 * math.pi / npts)
    c = np.cos(phi)
    rho = np.sqrt(a * a + r * r - 2 * a * r * c + (za - zr) ** 2)
    return MU0 * a * r / 2 * np.sum(c / rho) * (2 * math.pi / npts)


def test_transport_flux_pattern_against_neumann_quadrature():
    """Psi_u,e: flux through element ring e per ampere of transport current
    when every OTHER wire of the coil carries it, spread evenly over its n_e
    elements: sum over elements j with w(j) != w(e) of M(e, j) / n_e.  The
    element's own wire is excluded (its current response is the unknown of
    the wire's A-V solve).  Here 2 layers x 3 turns of 2x2 elements (n_e = 4,
    24 elements), M by an independent quadrature of Neumann's integral."""
    w = cs.Workload(name="psi", coils=[cs.Coil(layers=2, turns=3, ne=2, r_inner=0.02, wire_side=1e-3)],
                    steps=1, dt=1e-4, jc_disorder=("none", 0.0))
    s = oracle.Sim(w)
    r, z, psi = s.get(oracle.R), s.get(oracle.Z), s.get(oracle.PSI)
    wire = np.empty(s.N, dtype=int)
    for wi in range(s.Nw):
        wire[s.wire_elems(wi)] = wi
    # public order e = i_r n_z + i_z; the wire of (i_r, i_z) is (i_r // 2) * 3 + i_z // 2
    ir, iz = np.divmod(np.arange(s.N), 6)
    assert np.array_equal(wire, (ir // 2) * 3 + iz // 2)
    n_e = 4
    ref = np.zeros(s.N)
    for e in range(s.N):
        for j in range(s.N):
            if wire[j] != wire[e]:
                ref[e] += _neumann_M(r[j], z[j], r[e], z[e]) / n_e
    assert np.allclose(psi, ref, rtol=1e-11, atol=0)


# ----------------------------------------------------------------- Jc(B, T, eps)
def test_jc_factors_literal_numbers():
    """Benchmark configuration 1's law Jc = c_w Jc0 mu (1 - T/Tc) B0/(B0 + |B|)
    (1 - 900 |eps|^1.7) on a one-element coil, where B is the background field
    alone (an element's own ring is excluded).  Inputs chosen so that every
    factor is a round number: c_w = 0.8, mu = 1.3, T = 9 K with Tc = 18 K
    (factor 1/2), |B| = B_a = 3 T with B0 = 1 T (factor 1/4), and
    |eps| = (1/1800)^(1/1.7) (factor 1/2).  Expected Jc = 0.8 * 2e10 * 1.3 *
    1/2 * 1/4 * 1/2 = 1.3e9 A/m^2; with a square law in strain, or a field
    factor B0/(B0 + 2|B|), it would be 1.41e9 or 7.4e8."""
    dt = 1e-4
    eps = -(1.0 / 1800.0) ** (1.0 / 1.7)
    w = cs.Workload(name="jc", coils=[cs.Coil(layers=1, turns=1, ne=1, r_inner=0.02, wire_side=1e-3, ramp=0.0)],
                    steps=1, dt=dt, dBa_dt=3.0 / dt, Jc0=2e10, Tc=18.0, B0=1.0, eps_coef=900.0, eps_pow=1.7,
                    jc_disorder=("none", 0.0))
    inp = {"jc0_mult": np.array([1.3]), "strain": np.array([eps]), "c_wire": np.array([0.8])}
    s = oracle.Sim(w, inp)
    assert s.step() == 0  # B_a(t_0) = 0, no current anywhere
    s.set(oracle.T, np.array([9.0]))
    assert s.step() == 0  # now B_a(t_1) = 3 T and T^1 = 9 K
    assert abs(s.get(oracle.BZ)[0] - 3.0) < 1e-14 and s.get(oracle.BR)[0] == 0.0
    assert s.get(oracle.JC)[0] == pytest.approx(1.3e9, rel=1e-13)
    # step 0: B = 0 (factor 1) and T = 4.2 K (factor 1 - 4.2/18 = 23/30), so
    # Jc = 0.8 * 2e10 * 1.3 * 23/30 * 1/2 = 7.973333...e9
    s2 = oracle.Sim(w, inp)
    s2.step()
    assert s2.get(oracle.JC)[0] == pytest.approx(7.9733333333333333e9, rel=1e-14)
