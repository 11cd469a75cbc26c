"""Batched ensembles of uneven coils in one launch, tile-shape independence,
the autotuner and its cache, graph replay of an ensemble."""
import os
import sys

import numpy as np
import pytest

import coil_synth as cs
import oracle

pytestmark = pytest.mark.gpu


def _pk():
    import paper_2403_07666_amd as pk
    return pk


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def nerr(a, b):
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / s) if s > 0 else float(np.abs(a).max())


def _ensemble():
    coils = [cs.Coil(2, 3, 6, ramp=700.0), cs.Coil(3, 4, 6, ramp=1500.0, r_inner=0.025),
             cs.Coil(1, 5, 6, ramp=300.0, z_center=0.002)]
    return cs.Workload(name="ens3", coils=coils, steps=100, dt=1e-4, Jc0=5e8,
                       jc_disorder=("lognormal", 0.02), seed=4)


def test_ensemble_equals_individual_runs():
    pk = _pk()
    w = _ensemble()
    inp = cs.generate(w)
    g = pk.Coil(w, inp)
    g.run(100)
    off, woff = 0, 0
    for co in w.coils:
        wi = w.replace(coils=[co])
        sl = slice(off, off + co.n_elem)
        inp_i = {"jc0_mult": inp["jc0_mult"][sl], "strain": inp["strain"][sl],
                 "c_wire": inp["c_wire"][woff:woff + co.n_wire]}
        gi = pk.Coil(wi, inp_i)
        gi.run(100)
        for f in (pk.F_I, pk.F_T, pk.F_BZ, pk.F_BR):
            e = nerr(g.get(f)[sl], gi.get(f))
            assert e <= 1e-12, (f, e)
        off += co.n_elem
        woff += co.n_wire


def test_ensemble_matches_oracle_active():
    pk = _pk()
    w = _ensemble()
    inp = cs.generate(w)
    o = oracle.Sim(w, inp)
    assert o.run(100) == 0
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-5)):
        g = pk.Coil(w, inp, precision=prec)
        g.run(100)
        eb = max(nerr(g.get(pk.F_BR), o.get(oracle.BR)), nerr(g.get(pk.F_BZ), o.get(oracle.BZ)))
        ei = nerr(g.get(pk.F_I), o.get(oracle.I))
        To = o.get(oracle.T)
        Tg = g.get(pk.F_T)
        et = np.abs(Tg - To).max() / max(To.max() - w.T_bath, 1e-30)
        etl = nerr(Tg, To)
        _say(f"ensemble {prec}: B {eb:.2e} I {ei:.2e} dT {et:.2e} T {etl:.2e}")
        assert To.max() - w.T_bath > 1e-3
        assert eb <= tol and ei <= tol and et <= tol and etl <= tol


def test_tile_shapes_agree_and_autotune_cache(tmp_path):
    pk = _pk()
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    ref = None
    for tb, ch, grid in ((64, 1, 0), (128, 4, 0), (256, 16, 512), (64, 2, 64)):
        g = pk.Coil(w, inp, algo="direct")
        g.set_tiles(tb, ch, grid)
        g.run(60)
        cur = (g.get(pk.F_I), g.get(pk.F_BZ), g.get(pk.F_T))
        if ref is None:
            ref = cur
        else:
            for a, b in zip(cur, ref):
                assert nerr(a, b) <= 1e-12
    path = os.path.join(str(tmp_path), "tune.jsonl")
    g = pk.Coil(w, inp, algo="direct")
    g.run(3)
    chosen = g.autotune(reps=2, cache_path=path)
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and '"key": "gfx950/fp64/' in lines[0]
    assert chosen[0] in (1, 2)
    g2 = pk.Coil(w, inp, algo="direct")
    assert g2.autotune(reps=2, cache_path=path) == chosen
    assert len(open(path).read().splitlines()) == 1  # served from the cache
    g2.run(60)
    assert nerr(g2.get(pk.F_I), ref[0]) <= 1e-12


def test_graph_replay_of_ensemble_is_bitwise():
    pk = _pk()
    w = _ensemble()
    inp = cs.generate(w)
    a = pk.Coil(w, inp, precision="mixed")
    b = pk.Coil(w, inp, precision="mixed")
    b.set_tiles(128, 2, 256)
    a.set_tiles(128, 2, 256)
    b.graph(25)
    a.run(100)
    b.run(100)
    for f in (pk.F_I, pk.F_T, pk.F_BZ):
        assert np.array_equal(a.get(f), b.get(f))


def test_c4_ensemble_full_size():
    """The 16-coil ensemble (seeded sizes, ~4.6e5 elements): field pass on seeded
    currents against the oracle at sampled targets of every coil; a few steps in
    mixed precision against FP64; persistent grid."""
    pk = _pk()
    w = cs.workload("c4")
    inp = cs.generate(w)
    _say("c4", w.n_elem, [(c.layers, c.turns) for c in w.coils])
    o = oracle.Sim(w, field_only=True)
    I = cs.random_currents(w.n_elem, seed=44)
    tg = []
    off = 0
    for i, co in enumerate(w.coils):
        tg.extend((off + cs.sample_indices(co.n_elem, 8, seed=100 + i)).tolist())
        off += co.n_elem
    tg = np.array(tg)
    obr, obz = o.field_targets(I, tg)
    scale = max(np.abs(obr).max(), np.abs(obz).max())
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-5)):
        g = pk.Coil(w, inp, precision=prec, grid_limit=1024)
        g.set_state(pk.F_I, I)
        g.compute_field()
        e = max(np.abs(g.get(pk.F_BR)[tg] - obr).max(), np.abs(g.get(pk.F_BZ)[tg] - obz).max()) / scale
        _say(f"c4 field {prec}: {e:.2e}")
        assert e <= tol
        g.close()
    runs = {}
    for prec in ("fp64", "mixed"):
        g = pk.Coil(w, inp, precision=prec, grid_limit=1024)
        g.run(3)
        runs[prec] = (g.get(pk.F_BR), g.get(pk.F_BZ), g.get(pk.F_I))
        g.close()
    for a, b in zip(runs["mixed"], runs["fp64"]):
        assert nerr(a, b) <= 1e-5


def test_timing_modes():
    """Event timing: mode 1 times every phase, mode 2 only the field kernel;
    neither changes the results; other modes are rejected."""
    pk = _pk()
    w = _ensemble()
    inp = cs.generate(w)
    g = pk.Coil(w, inp, precision="mixed")
    g.run(5)
    ref = g.get(pk.F_I)
    g.reset()
    g.timing(1)
    g.run(3)
    t1 = g.timing_read()
    g.timing(2)
    g.run(2)
    t2 = g.timing_read()
    g.timing(0)
    assert np.array_equal(g.get(pk.F_I), ref)
    # the heat substeps of a step run in two tiled launches (one when there is one substep)
    heat_launches = 1 if g.n_sub <= 1 else max(2, -(-g.n_sub // 8))
    assert [t1[k]["launches"] for k in ("field", "wire", "heat", "reduce")] == [3, 3, 3 * heat_launches, 3]
    assert all(t1[k]["ms"] > 0 for k in t1)
    assert t2["field"]["launches"] == 2 and t2["field"]["ms"] > 0
    assert all(t2[k]["launches"] == 0 and t2[k]["ms"] == 0 for k in ("wire", "heat", "reduce"))
    with pytest.raises(pk.CoilError):
        g.timing(3)
    g.close()


def test_autotuned_translation_runs_as_work_queue(tmp_path):
    """A TRANSLATION choice of the autotuner runs the work-queue launch even
    when a DIRECT tile shape with a persistent grid was set before."""
    import json
    pk = _pk()
    w = _ensemble()
    inp = cs.generate(w)
    path = os.path.join(str(tmp_path), "tune.jsonl")
    g = pk.Coil(w, inp, precision="mixed")
    g.autotune(reps=1, cache_path=path)
    rec = json.loads(open(path).read().splitlines()[0])
    rec.update({"algo": 2, "p1": 8, "p2": 0, "p3": 0})
    with open(path, "w") as f:
        f.write(json.dumps(rec) + "\n")
    g.close()
    g = pk.Coil(w, inp, precision="mixed")
    g.set_tiles(64, 2, 7)
    st = g.field_stats()
    assert st["algo"] == "direct" and st["workgroups"] == 7
    assert g.autotune(reps=1, cache_path=path) == (2, 8, 0, 0)
    st = g.field_stats()
    assert st["algo"] == "translation" and st["workgroups"] > 7
    assert st["workgroups"] <= st["items"]
    g.close()
