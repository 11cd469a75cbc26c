"""GPU parity of the variable-step integration of the wire currents (config
em_tol: substeps dt / 2^m within a step, step-doubling error control, local
extrapolation; kernel k_wire_em) against the oracle's.  The substep counts
per wire must agree exactly (the same accept/reject decisions), and the
state within 1e-10 (FP64) and 1e-5 (mixed field pass) on B, I, Phi, U_w, T
(literal, and rise-relative above T's rounding floor) and Q."""
import sys

import numpy as np
import pytest

import coil_synth as cs
import oracle

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}
EPS = 2.220446049250313e-16


def _pk():
    import paper_2403_07666_amd as pk
    return pk


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def nerr(a, b):
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / s) if s > 0 else float(np.abs(a).max())


def _compare(w, prec, nsteps, chunk):
    pk = _pk()
    inp = cs.generate(w)
    _say(f"  case {w.name} em_tol={w.em_tol} {prec}")
    g = pk.Coil(w, inp, precision=prec)
    o = oracle.Sim(w, inp)
    tol = TOL[prec]
    most, total = 0.0, 0.0
    for k in range(nsteps):
        g.run(1)
        assert o.step() == 0
        so = o.get(oracle.EMSUB)
        assert np.array_equal(g.get(pk.F_EM_SUBSTEPS), so), f"substep counts differ at step {k}"
        most, total = max(most, so.max()), total + so.sum()
        if (k + 1) % chunk:
            continue
        To, Tg = o.get(oracle.T), g.get(pk.F_T)
        rise = float((To - w.T_bath).max())
        e = {
            "B": max(nerr(g.get(pk.F_BR), o.get(oracle.BR)), nerr(g.get(pk.F_BZ), o.get(oracle.BZ))),
            "I": nerr(g.get(pk.F_I), o.get(oracle.I)),
            "Phi": nerr(g.get(pk.F_PHI), o.get(oracle.PHI)),
            "U": nerr(g.get(pk.F_UW), o.get(oracle.UW)),
            "T": nerr(Tg, To),
        }
        sg, sc = g.scalars(), o.scalars()
        e["Q"] = abs(sg["Q"] - sc["Q"]) / sc["Q"] if sc["Q"] > 0 else 0.0
        dT = float(np.abs(Tg - To).max() / rise) if rise > 0 else 0.0
        floor = 8 * EPS * float(To.max()) / rise if rise > 0 else 0.0
        _say(f"  {w.name} {prec} step {k + 1}: " + " ".join(f"{a} {v:.2e}" for a, v in e.items())
             + f" dT {dT:.2e} (floor {floor:.1e}) substeps max {most:.0f} total {total:.0f}")
        assert max(e.values()) <= tol and dT <= max(tol, floor)
    return g, o, most


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_variable_step_c1_active_against_oracle(prec):
    w = cs.workload("c1_active").replace(name="c1_em", em_tol=1e-5)
    g, o, most = _compare(w, prec, 300, 100)
    assert most > 1.0  # some wires took several substeps
    assert o.scalars()["max_x"] > 1.0


def test_variable_step_64_per_wire_against_oracle():
    """ne = 8 (64 elements per wire: the whole wavefront) in the active regime
    under a transport ramp and a background ramp, at a tight tolerance."""
    w = cs.workload("c1_active").replace(name="c_em64", em_tol=1e-7, dBa_dt=0.5, Jc0=1e8,
                                         coils=[cs.Coil(layers=2, turns=3, ne=8, ramp=2000.0)])
    g, o, most = _compare(w, "fp64", 200, 50)
    assert most > 1.0


def test_variable_step_stiff_decay_against_oracle():
    """A 2 x 2-element wire at R = 100 m with a screening current of 1.5 Ic
    decaying under the n = 30 power law (the oracle's closed-form pin case):
    the GPU takes the oracle's substeps and lands on its currents."""
    pk = _pk()
    w = cs.Workload(name="decay", coils=[cs.Coil(layers=1, turns=1, ne=2, r_inner=100.0 - 5e-4, wire_side=1e-3,
                                                  ramp=0.0)],
                    steps=1, dt=1e-4, Ec=1e-4, n=30.0, Jc0=1e7, Tc=1e30, B0=1e30, dBa_dt=0.0,
                    jc_disorder=("none", 0.0), eps_range=(0.0, 0.0), em_tol=1e-5, em_max_level=16)
    g = pk.Coil(w)
    o = oracle.Sim(w)
    r = o.get(oracle.R)
    I0 = 1.5 * 1e7 * (5e-4) ** 2 * np.where(r < 100.0, 1.0, -1.0)
    g.set_state(pk.F_I, I0)
    o.set(oracle.I, I0)
    subs = 0.0
    for _ in range(20):
        g.run(1)
        assert o.step() == 0
        assert np.array_equal(g.get(pk.F_EM_SUBSTEPS), o.get(oracle.EMSUB))
        subs += o.get(oracle.EMSUB).sum()
    assert subs > 20
    assert nerr(g.get(pk.F_I), o.get(oracle.I)) <= 1e-10
    assert nerr(g.get(pk.F_PHI), o.get(oracle.PHI)) <= 1e-10


def test_variable_step_graph_replay_and_rejections():
    """A captured graph of variable steps replays the eager run bitwise (the
    substep loop runs inside the kernel, so the graph holds the same kernel
    nodes as a fixed step); the adjoint and the substep field without the
    option are refused."""
    pk = _pk()
    w = cs.workload("c1_active").replace(em_tol=1e-5)
    inp = cs.generate(w)
    a = pk.Coil(w, inp)
    b = pk.Coil(w, inp)
    a.run(300)
    b.graph(10)
    for _ in range(30):
        b.run(10)
        b.synchronize()
    for f in (pk.F_I, pk.F_T, pk.F_PHI, pk.F_UW, pk.F_EM_SUBSTEPS):
        assert np.array_equal(a.get(f), b.get(f))
    with pytest.raises(pk.CoilError) as ei:
        a.adjoint(5)
    assert ei.value.code == -1
    b = pk.Coil(cs.workload("c1_active"), inp)
    with pytest.raises(pk.CoilError):
        b.get(pk.F_EM_SUBSTEPS)
