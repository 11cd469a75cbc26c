"""GPU parity of the subelement model (config subelements = s: per wire, the
field-driven current I_H with zero net current per subelement and the
transport current I_I, two constrained solves with the wire matrix in LDS)
against the oracle's subelement solve.  Tolerances 1e-10 (FP64) and 1e-5
(mixed field pass), normwise on B, I, I_H, Phi, U_w, T (literal and
rise-relative) and Q."""
import sys

import numpy as np
import pytest

import coil_synth as cs
import oracle

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}
EPS = 2.220446049250313e-16


def rise_floor(T_max, rise):
    """Rounding floor of T - T_bath relative to its rise: T itself carries a
    few ulps of rounding (8 eps T_max bounds it), which at a rise of a few
    microkelvin is above 1e-10 of the rise."""
    return 8 * EPS * T_max / rise


def _pk():
    import paper_2403_07666_amd as pk
    return pk


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def nerr(a, b):
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / s) if s > 0 else float(np.abs(a).max())


def _compare(w, prec, nsteps, chunks=3):
    pk = _pk()
    inp = cs.generate(w)
    _say(f"  case {w.name} s={w.subelements} {prec}")
    g = pk.Coil(w, inp, precision=prec)
    o = oracle.Sim(w, inp)
    tol = TOL[prec]
    for k in range(chunks):
        g.run(nsteps // chunks)
        assert o.run(nsteps // chunks) == 0
        To, Tg = o.get(oracle.T), g.get(pk.F_T)
        rise = float((To - w.T_bath).max())
        e = {
            "B": max(nerr(g.get(pk.F_BR), o.get(oracle.BR)), nerr(g.get(pk.F_BZ), o.get(oracle.BZ))),
            "I": nerr(g.get(pk.F_I), o.get(oracle.I)),
            "IH": nerr(g.get(pk.F_IH), o.get(oracle.IH)),
            "Phi": nerr(g.get(pk.F_PHI), o.get(oracle.PHI)),
            "U": nerr(g.get(pk.F_UW), o.get(oracle.UW)),
            "T": nerr(Tg, To),
            "dT": float(np.abs(Tg - To).max() / rise) if rise > 0 else 0.0,
        }
        sg, so = g.scalars(), o.scalars()
        e["Q"] = abs(sg["Q"] - so["Q"]) / so["Q"] if so["Q"] > 0 else 0.0
        floor = rise_floor(float(To.max()), rise) if rise > 0 else 0.0
        _say(f"  {w.name} s={w.subelements} {prec} chunk {k}: " + " ".join(f"{a} {v:.2e}" for a, v in e.items())
             + f" rise {rise:.3e} (dT floor {floor:.1e})")
        dT = e.pop("dT")
        assert max(e.values()) <= tol and dT <= max(tol, floor)
    return g, o


def _c1_sub(s):
    return cs.workload("c1_active").replace(name="c1_sub", subelements=s)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_subelements_c1_active_against_oracle(prec):
    g, o = _compare(_c1_sub(2), prec, 300)
    assert o.scalars()["max_x"] > 1.0
    assert np.abs(o.get(oracle.IH)).max() > 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_subelements_64_per_wire_field_and_transport(prec):
    """ne = 8 (64 elements per wire, every lane of the wavefront) with 4 x 4
    subelements, a background ramp and a transport ramp."""
    w = cs.workload("c1_active").replace(name="c_sub16", subelements=4, dBa_dt=0.5, Jc0=1e8,
                                         coils=[cs.Coil(layers=2, turns=3, ne=8, ramp=2000.0)])
    g, o = _compare(w, prec, 300)
    assert np.abs(o.get(oracle.IH)).max() > 0


def test_single_subelement_matches_wire_kernel():
    """s = 1 on the GPU against the GPU's own wire model (the two-solve
    kernel against the one-solve kernels)."""
    pk = _pk()
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    a = pk.Coil(w, inp)
    b = pk.Coil(w.replace(subelements=1), inp)
    a.run(300)
    b.run(300)
    for f in (pk.F_I, pk.F_T, pk.F_PHI, pk.F_UW, pk.F_BZ):
        assert nerr(b.get(f), a.get(f)) <= 1e-11
    assert a.scalars()["max_x"] > 1.0


def test_subelements_snapshot_graph_and_rejections():
    pk = _pk()
    w = _c1_sub(2)
    inp = cs.generate(w)
    a = pk.Coil(w, inp)
    a.run(100)
    snap = a.save()
    a.run(100)
    b = pk.Coil(w, inp)
    b.load(snap)
    b.graph(10)
    for _ in range(10):
        b.run(10)
        b.synchronize()
    for f in (pk.F_I, pk.F_IH, pk.F_T, pk.F_PHI, pk.F_UW):
        assert np.array_equal(a.get(f), b.get(f))
    with pytest.raises(pk.CoilError) as ei:
        a.adjoint(10)
    assert ei.value.code == -1
    c = pk.Coil(cs.workload("c1_active"), inp)
    with pytest.raises(pk.CoilError):
        c.get(pk.F_IH)
