"""GPU parity of the ADI heat step (COIL_HEAT_ADI: Peaceman-Rachford with
parallel cyclic reduction along grid columns and rows) against the oracle's
ADI step (Thomas algorithm), with constant coefficients, with the T^3 laws,
an insulation layer between wires and a composite conductivity map, and at
time steps far beyond the explicit limit.  Tolerances 1e-10 (FP64) and 1e-5
(mixed field pass) on T (literal and rise-relative), I and B."""
import sys

import numpy as np
import pytest

import coil_synth as cs
import oracle

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}
EPS = 2.220446049250313e-16


def rise_floor(w, T_max, rise):
    """Rounding floor of T - T_bath relative to its rise: the line systems of
    the ADI step have condition number kappa = 1 + 4 alpha dt / d^2 (alpha the
    largest diffusivity), so the two solvers (cyclic reduction on the GPU,
    Thomas in the oracle) can differ by about kappa eps T; 8 times that,
    relative to the rise, bounds the comparison from below."""
    d = min(c.wire_side / c.ne for c in w.coils)
    alpha = w.k0 * (T_max / w.T_ref) ** w.k_exp / (w.C0 * (w.T_bath / w.T_ref) ** w.cp_exp)
    kappa = 1 + 4 * alpha * w.dt / d ** 2
    return 8 * kappa * EPS * T_max / rise


def _pk():
    import paper_2403_07666_amd as pk
    return pk


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def nerr(a, b):
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / s) if s > 0 else float(np.abs(a).max())


def _compare(w, inp, prec, nsteps, chunks=3, kmult=None):
    pk = _pk()
    g = pk.Coil(w, inp, precision=prec)
    o = oracle.Sim(w, {k: v for k, v in inp.items() if k != "k_mult"})
    if kmult is not None:
        o.set(oracle.KMULT, kmult)
    tol = TOL[prec]
    for k in range(chunks):
        g.run(nsteps // chunks)
        assert o.run(nsteps // chunks) == 0
        To, Tg = o.get(oracle.T), g.get(pk.F_T)
        rise = float((To - w.T_bath).max())
        et = nerr(Tg, To)
        er = float(np.abs(Tg - To).max() / rise) if rise > 0 else 0.0
        eb = max(nerr(g.get(pk.F_BR), o.get(oracle.BR)), nerr(g.get(pk.F_BZ), o.get(oracle.BZ)))
        ei = nerr(g.get(pk.F_I), o.get(oracle.I))
        sg, so = g.scalars(), o.scalars()
        eq = abs(sg["Q"] - so["Q"]) / so["Q"] if so["Q"] > 0 else 0.0
        floor = rise_floor(w, float(To.max()), rise) if rise > 0 else 0.0
        _say(f"  {w.name} {prec} chunk {k}: T {et:.2e} dT {er:.2e} (floor {floor:.1e}) B {eb:.2e} I {ei:.2e} "
             f"Q {eq:.2e} rise {rise:.3e}")
        assert max(et, eb, ei, eq) <= tol and er <= max(tol, floor)
    sg = g.scalars()
    assert sg["stored"] == pytest.approx(sg["Q"] - sg["Q_out"], rel=1e-9)
    assert sg["n_sub"] == 1
    return g, o


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adi_constant_coefficients_active(prec):
    w = cs.workload("c1_active").replace(name="c1_adi", heat_solver="adi")
    _compare(w, cs.generate(w), prec, 300)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adi_composite_T3_active(prec):
    """k and h proportional to T^3, an epoxy layer between wires (R = 2e-4
    m^2 K/W) and a composite map (conductivity multiplier 0.05 on a seeded
    third of the elements)."""
    w = cs.workload("c1_active").replace(name="c1_adi_composite", heat_solver="adi", k_exp=3.0, h_exp=3.0,
                                         ins_R0=2e-4)
    inp = cs.generate(w)
    rng = np.random.Generator(np.random.PCG64(17))
    km = np.where(rng.random(w.n_elem) < 1 / 3, 0.05, 1.0)
    inp["k_mult"] = km
    _compare(w, inp, prec, 300, kmult=km)


def test_adi_far_beyond_explicit_limit():
    """A heated spot relaxing with dt 400x the explicit limit: GPU against the
    oracle step by step (both take the same non-monotone but stable steps)."""
    pk = _pk()
    w = cs.Workload(name="adi_big", coils=[cs.Coil(layers=4, turns=8, ne=4, ramp=0.0)], steps=1, dt=2e-2,
                    cp_exp=0.0, h0=500.0, heat_solver="adi", jc_disorder=("none", 0.0))
    g = pk.Coil(w)
    o = oracle.Sim(w)
    r, z = o.get(oracle.R), o.get(oracle.Z)
    T0 = 4.2 + np.exp(-((r - 0.022) ** 2 + z ** 2) / (2 * 1e-3 ** 2))
    g.set_state(pk.F_T, T0)
    o.set(oracle.T, T0)
    for _ in range(10):
        g.run(1)
        assert o.step() == 0
        Tg, To = g.get(pk.F_T), o.get(oracle.T)
        rise = float(np.abs(To - 4.2).max())
        e = nerr(Tg - 4.2, To - 4.2)
        _say(f"  far step: T {nerr(Tg, To):.2e} T-T_bath {e:.2e} (floor {rise_floor(w, float(To.max()), rise):.1e})")
        assert nerr(Tg, To) <= 1e-10
        assert e <= max(1e-10, rise_floor(w, float(To.max()), rise))
