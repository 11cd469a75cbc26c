"""GPU parity of the fully coupled A-V solve (COIL_COUPLE_FULL: the flux of
every element current of the coil in every ring's circuit equation, solved by
preconditioned conjugate gradients with an FP64 flux pass) against the
oracle's dense constrained solve.  Tolerances 1e-10 (FP64) and 1e-5 (mixed
field pass), normwise on B, I, Phi and T."""
import sys

import numpy as np
import pytest

import coil_synth as cs
import oracle

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}


def _pk():
    import paper_2403_07666_amd as pk
    return pk


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def nerr(a, b):
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / s) if s > 0 else float(np.abs(a).max())


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_coupled_c1_active_against_oracle(prec):
    pk = _pk()
    w = cs.workload("c1_active").replace(coupling="full")
    inp = cs.generate(w)
    g = pk.Coil(w, inp, precision=prec)
    o = oracle.Sim(w, inp)
    tol = TOL[prec]
    for k in range(3):
        g.run(100)
        assert o.run(100) == 0
        To, Tg = o.get(oracle.T), g.get(pk.F_T)
        rise = float((To - w.T_bath).max())
        eb = max(nerr(g.get(pk.F_BR), o.get(oracle.BR)), nerr(g.get(pk.F_BZ), o.get(oracle.BZ)))
        ei = nerr(g.get(pk.F_I), o.get(oracle.I))
        ephi = nerr(g.get(pk.F_PHI), o.get(oracle.PHI))
        eu = nerr(g.get(pk.F_UW), o.get(oracle.UW))
        et = nerr(Tg, To)
        er = float(np.abs(Tg - To).max() / rise) if rise > 0 else 0.0
        sg = g.scalars()
        _say(f"  {prec} step {100 * (k + 1)}: B {eb:.2e} I {ei:.2e} Phi {ephi:.2e} U {eu:.2e} T {et:.2e} "
             f"dT {er:.2e} cg {int(sg['cg_iters'])} it, residual {sg['cg_residual']:.1e}")
        assert max(eb, ei, ephi, eu, et, er) <= tol
    assert o.scalars()["max_x"] > 1.0
    # the coupling matters here: the transport-only drive gives other currents
    t = oracle.Sim(w.replace(coupling="transport"), inp)
    assert t.run(300) == 0
    assert nerr(t.get(oracle.I), o.get(oracle.I)) > 0.1


def test_coupled_single_wire_equals_transport():
    pk = _pk()
    w = cs.workload("c1_active").replace(coils=[cs.Coil(layers=1, turns=1, ne=8, ramp=1000.0)])
    inp = cs.generate(w)
    a = pk.Coil(w, inp)
    b = pk.Coil(w.replace(coupling="full"), inp)
    a.run(200)
    b.run(200)
    for f in (pk.F_I, pk.F_T, pk.F_PHI, pk.F_BZ):
        assert nerr(b.get(f), a.get(f)) <= 1e-12
    # the starting residual is rounding noise: at most one iteration to see that
    assert b.scalars()["cg_iters"] <= 1


def test_coupled_graph_replay_and_adjoint_rejected():
    pk = _pk()
    w = cs.workload("c1_active").replace(coupling="full", coils=[cs.Coil(layers=2, turns=4, ne=4, ramp=1000.0)])
    inp = cs.generate(w)
    a = pk.Coil(w, inp, cg_max_iter=60)
    b = pk.Coil(w, inp, cg_max_iter=60)
    a.run(60)
    b.graph(5)  # every step's 60 iterations captured; those after convergence return at once
    for _ in range(12):
        b.run(5)
        b.synchronize()
    for f in (pk.F_I, pk.F_T, pk.F_PHI, pk.F_UW):
        assert np.array_equal(a.get(f), b.get(f))
    with pytest.raises(pk.CoilError) as ei:
        a.adjoint(10)
    assert ei.value.code == -1
