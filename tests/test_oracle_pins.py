"""Pins of the CPU oracle against facts that do not come from the oracle itself:
library routines (scipy, mpmath), textbook closed forms, brute-force
quadrature, identities and limits.  Each test names what fixes the value."""
import math

import numpy as np
import pytest

import oracle

MU0 = 4e-7 * math.pi


# ----------------------------------------------------------------- elliptic
def test_carlson_against_mpmath():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    for x, y, z in [(1, 2, 0), (2, 3, 4), (0.5, 1e-3, 7.0), (0, 1e-8, 1), (0.2, 0.2, 0.2)]:
        ref_f = float(mp.elliprf(x, y, z))
        assert abs(oracle.carlson_rf(x, y, z) / ref_f - 1) < 4e-15
    for x, y, z in [(0, 2, 1), (2, 3, 4), (0, 1e-8, 1), (1e-3, 0.5, 3.0)]:
        ref_d = float(mp.elliprd(x, y, z))
        assert abs(oracle.carlson_rd(x, y, z) / ref_d - 1) < 4e-15


def test_KE_special_values():
    K, E = oracle.ellip(1.0)  # m = 0
    assert K == pytest.approx(math.pi / 2, rel=1e-15, abs=0)
    assert E == pytest.approx(math.pi / 2, rel=1e-15, abs=0)
    _, E1 = oracle.ellip(1e-30)  # m -> 1: E(1) = 1
    assert abs(E1 - 1.0) < 1e-12
    # m = 1/2: K(1/2) = Gamma(1/4)^2 / (4 sqrt(pi))
    Kh, _ = oracle.ellip(0.5)
    assert Kh == pytest.approx(math.gamma(0.25) ** 2 / (4 * math.sqrt(math.pi)), rel=2e-15)


def test_KE_against_scipy_and_mpmath():
    from scipy.special import ellipe, ellipkm1
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    for m1 in np.concatenate([np.logspace(-12, -1, 23), np.linspace(0.05, 1.0, 20)]):
        K, E = oracle.ellip(m1)
        assert abs(K / ellipkm1(m1) - 1) < 3e-15
        assert abs(E / ellipe(1.0 - m1) - 1) < 2e-14  # scipy takes m, rounded near 1
        m = 1 - mp.mpf(float(m1))
        assert abs(K / float(mp.ellipk(m)) - 1) < 3e-15
        # E = R_F - (m/3) R_D cancels as m -> 1: error grows like eps * K(m)
        assert abs(E / float(mp.ellipe(m)) - 1) < 3e-15 * max(1.0, K)


def test_legendre_relation():
    # E K' + E' K - K K' = pi/2 pins K and E jointly over the whole range
    for m1 in np.linspace(0.01, 0.99, 41):
        K, E = oracle.ellip(m1)
        Kp, Ep = oracle.ellip(1.0 - m1)
        assert E * Kp + Ep * K - K * Kp == pytest.approx(math.pi / 2, rel=1e-14)


def test_K_log_asymptote():
    for m1 in [1e-8, 1e-10, 1e-12]:
        K, _ = oracle.ellip(m1)
        # K = ln(4/sqrt(m1)) + O(m1 ln m1)
        assert abs(K - math.log(4 / math.sqrt(m1))) < 10 * m1 * abs(math.log(m1))


# ----------------------------------------------------------------- ring field
def _biot_savart(a, zs, r, z, I=1.0, n=4096):
    """Trapezoid rule in the loop angle (spectrally accurate for a smooth
    periodic integrand) of dB = mu0 I / 4pi dl x R / |R|^3."""
    phi = (np.arange(n) + 0.5) * (2 * np.pi / n)
    c, s = np.cos(phi), np.sin(phi)
    dz = z - zs
    R3 = (r * r + a * a - 2 * a * r * c + dz * dz) ** 1.5
    w = 2 * np.pi / n
    br = MU0 * I / (4 * np.pi) * np.sum(a * c * dz / R3) * w
    bz = MU0 * I / (4 * np.pi) * np.sum((a * a - a * r * c) / R3) * w
    return br, bz


def test_ring_on_axis_closed_form():
    for R in [0.02, 0.05]:
        for z in [0.0, 0.003, 0.05, 0.4]:
            br, bz = oracle.ring_B(R, 0.0, 0.0, z, 3.0)
            ref = MU0 * 3.0 * R * R / (2 * (R * R + z * z) ** 1.5)
            assert bz == pytest.approx(ref, rel=1e-14)
            assert br == 0.0


@pytest.mark.parametrize("r,z", [(0.01, 0.0), (0.03, 0.004), (0.021, 0.0003), (0.05, -0.02),
                                 (0.0205, 0.0), (0.1, 0.3)])
def test_ring_against_biot_savart(r, z):
    a, zs = 0.02, 0.0
    br, bz = oracle.ring_B(a, zs, r, z, 1.7)
    qbr, qbz = _biot_savart(a, zs, r, z, 1.7)
    scale = math.hypot(qbr, qbz)
    assert abs(br - qbr) < 1e-12 * scale
    assert abs(bz - qbz) < 1e-12 * scale


def test_ring_divergence_free_and_flux_consistent():
    a, zs, I = 0.025, 0.001, 2.0
    for r, z in [(0.03, 0.004), (0.022, -0.002), (0.04, 0.01)]:
        h = 1e-6
        br_p, _ = oracle.ring_B(a, zs, r + h, z, I)
        br_m, _ = oracle.ring_B(a, zs, r - h, z, I)
        _, bz_p = oracle.ring_B(a, zs, r, z + h, I)
        _, bz_m = oracle.ring_B(a, zs, r, z - h, I)
        br, bz = oracle.ring_B(a, zs, r, z, I)
        div = ((r + h) * br_p - (r - h) * br_m) / (2 * h * r) + (bz_p - bz_m) / (2 * h)
        rho = math.hypot(r - a, z - zs)  # distance to the filament sets the scale
        assert abs(div) < 1e-6 * math.hypot(br, bz) / rho
        # flux Psi = M I through the ring at (r, z): dPsi/dz = -2 pi r B_r,
        # dPsi/dr = 2 pi r B_z  (B = curl A, Psi = 2 pi r A_phi)
        dpsi_dz = I * (oracle.ring_M(a, zs, r, z + h) - oracle.ring_M(a, zs, r, z - h)) / (2 * h)
        dpsi_dr = I * (oracle.ring_M(a, zs, r + h, z) - oracle.ring_M(a, zs, r - h, z)) / (2 * h)
        assert dpsi_dz == pytest.approx(-2 * math.pi * r * br, rel=1e-7, abs=1e-18)
        assert dpsi_dr == pytest.approx(2 * math.pi * r * bz, rel=1e-7, abs=1e-18)


def test_ring_near_and_far_limits():
    a, I = 0.03, 1.0
    # close to the filament: straight-wire field mu0 I / (2 pi rho)
    rho = 1e-6
    br, bz = oracle.ring_B(a, 0.0, a + rho, 0.0, I)
    assert math.hypot(br, bz) == pytest.approx(MU0 * I / (2 * math.pi * rho), rel=1e-3)
    # far away in the equatorial plane: dipole field -mu0 m / (4 pi R^3), m = pi a^2 I
    Rf = 100 * a
    br, bz = oracle.ring_B(a, 0.0, Rf, 0.0, I)
    assert bz == pytest.approx(-MU0 * math.pi * a * a * I / (4 * math.pi * Rf ** 3), rel=1e-3)
    assert abs(br) < 1e-15 * abs(bz)


# ----------------------------------------------------------------- inductance
def _neumann(a, zs, r, z, n=4096):
    """Neumann's formula reduced to one angle: M = mu0 a r / 2 int cos(phi)/R dphi."""
    phi = (np.arange(n) + 0.5) * (2 * np.pi / n)
    dz = z - zs
    R = np.sqrt(a * a + r * r - 2 * a * r * np.cos(phi) + dz * dz)
    return MU0 * a * r / 2 * np.sum(np.cos(phi) / R) * (2 * np.pi / n)


@pytest.mark.parametrize("a,zs,r,z", [(0.02, 0.0, 0.03, 0.01), (0.02, 0.0, 0.021, 0.0005),
                                      (0.05, 0.01, 0.02, -0.03), (0.03, 0.0, 0.03, 0.002)])
def test_mutual_inductance_neumann_and_symmetry(a, zs, r, z):
    M = oracle.ring_M(a, zs, r, z)
    assert M == pytest.approx(_neumann(a, zs, r, z), rel=1e-12)
    assert M == pytest.approx(oracle.ring_M(r, z, a, zs), rel=1e-14)


def test_self_inductance_square_section_by_filament_average():
    """Self inductance of a square-section ring = average of the filament
    mutual inductance over pairs of points of the section (uniform current).
    Brute force on an n x n filament split; the diagonal's weight vanishes as
    n grows, so this pins the geometric-mean-distance constant."""
    r, d, n = 0.1, 1e-3, 24
    h = d / n
    off = (np.arange(n) + 0.5) * h - d / 2
    pts = [(r + a, b) for a in off for b in off]
    tot = 0.0
    for i, (ri, zi) in enumerate(pts):
        for j, (rj, zj) in enumerate(pts):
            tot += oracle.self_L(ri, h) if i == j else oracle.ring_M(rj, zj, ri, zi)
    L = tot / len(pts) ** 2
    assert L == pytest.approx(oracle.self_L(r, d), rel=2e-5)


def test_gmd_constant_of_square():
    """exp(<ln|p-q|>) over the unit square, by quadrature."""
    from scipy import integrate
    val, _ = integrate.dblquad(lambda v, u: (1 - u) * (1 - v) * 0.5 * np.log(u * u + v * v),
                               0, 1, 0, 1, epsabs=1e-13, epsrel=1e-13)
    g = math.exp(4 * val)
    r, d = 0.05, 1e-3
    assert oracle.self_L(r, d) == pytest.approx(MU0 * r * (math.log(8 * r / (g * d)) - 2), rel=1e-12)
