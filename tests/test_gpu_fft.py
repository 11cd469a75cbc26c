"""GPU checks of the fast-convolution field pass (COIL_ALGO_FFT) beyond the
shared parity cases (the field, run, adjoint and full-size tests are
parametrised over it): the 16-coil ensemble at full size against the oracle
at sampled targets, graph replay, the coupled solve on top of it, the
autotuner's use of it, and switching away from it."""
import json
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


def test_fft_c4_ensemble_full_size():
    """16 coils of uneven size (every coil its own DFT length) against the
    oracle at sampled targets of every coil; mixed steps against FP64."""
    pk = _pk()
    w = cs.workload("c4")
    inp = cs.generate(w)
    _say("c4 fft", w.n_elem)
    o = oracle.Sim(w, field_only=True)
    I = cs.random_currents(w.n_elem, seed=44)
    tg, off = [], 0
    for i, co in enumerate(w.coils):
        tg.extend((off + cs.sample_indices(co.n_elem, 8, seed=100 + i)).tolist())
        off += co.n_elem
    tg = np.array(tg)
    obr, obz = o.field_targets(I, tg)
    scale = max(np.abs(obr).max(), np.abs(obz).max())
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-5)):
        g = pk.Coil(w, inp, precision=prec, algo="fft")
        assert g.field_stats()["algo"] == "fft"
        g.set_state(pk.F_I, I)
        g.compute_field()
        e = max(np.abs(g.get(pk.F_BR)[tg] - obr).max(), np.abs(g.get(pk.F_BZ)[tg] - obz).max()) / scale
        _say(f"  c4 fft field {prec}: {e:.2e}")
        assert e <= tol
        g.close()
    runs = {}
    for prec in ("fp64", "mixed"):
        g = pk.Coil(w, inp, precision=prec, algo="fft")
        g.run(3)
        runs[prec] = (g.get(pk.F_BR), g.get(pk.F_BZ), g.get(pk.F_I))
        g.close()
    for a, b in zip(runs["mixed"], runs["fp64"]):
        assert nerr(a, b) <= 1e-5


def test_fft_graph_replay_bitwise():
    pk = _pk()
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    a = pk.Coil(w, inp, precision="mixed", algo="fft")
    b = pk.Coil(w, inp, precision="mixed", algo="fft")
    a.run(200)
    b.graph(10)
    for _ in range(20):
        b.run(10)
        b.synchronize()
    for f in (pk.F_I, pk.F_BR, pk.F_BZ, pk.F_T, pk.F_PHI):
        assert np.array_equal(a.get(f), b.get(f))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fft_coupled_solve_against_oracle(prec):
    """The coupled A-V solve with the field and the flux passes of its
    conjugate-gradient iteration both by fast convolution (the mutual
    inductance's FP64 spectra) against the oracle."""
    pk = _pk()
    w = cs.workload("c1_active").replace(coupling="full")
    inp = cs.generate(w)
    g = pk.Coil(w, inp, precision=prec, algo="fft")
    o = oracle.Sim(w, inp)
    for k in range(2):
        g.run(100)
        assert o.run(100) == 0
        e = max(nerr(g.get(pk.F_BR), o.get(oracle.BR)), nerr(g.get(pk.F_BZ), o.get(oracle.BZ)),
                nerr(g.get(pk.F_I), o.get(oracle.I)), nerr(g.get(pk.F_PHI), o.get(oracle.PHI)),
                nerr(g.get(pk.F_T), o.get(oracle.T)))
        sg = g.scalars()
        _say(f"  coupled fft {prec} step {100 * (k + 1)}: {e:.2e}, cg {int(sg['cg_iters'])} it")
        assert e <= (1e-10 if prec == "fp64" else 1e-5)


def test_fft_coupled_graph_replay_bitwise():
    """Graph-captured coupled steps (every CG iteration enqueued, the passes
    after convergence return at once) replay the eager run bitwise."""
    pk = _pk()
    w = cs.workload("c1_active").replace(coupling="full", coils=[cs.Coil(layers=2, turns=4, ne=4, ramp=1000.0)])
    inp = cs.generate(w)
    a = pk.Coil(w, inp, precision="fp64", algo="fft", cg_max_iter=60)
    b = pk.Coil(w, inp, precision="fp64", algo="fft", cg_max_iter=60)
    a.run(60)
    b.graph(5)
    for _ in range(12):
        b.run(5)
        b.synchronize()
    for f in (pk.F_I, pk.F_BR, pk.F_BZ, pk.F_T, pk.F_PHI):
        assert np.array_equal(a.get(f), b.get(f))


def test_fft_autotune_and_switching(tmp_path):
    """The autotuner times the fast convolution when it was set up at init and
    its choice reproduces the field; a cached choice of it is refused by a
    handle without spectra; set_tiles switches to the direct pass."""
    pk = _pk()
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    I = cs.random_currents(w.n_elem, seed=5)
    ref = pk.Coil(w, inp, precision="fp64", algo="translation")
    ref.set_state(pk.F_I, I)
    ref.compute_field()
    g = pk.Coil(w, inp, precision="fp64", algo="fft")

    def check(algo):
        assert g.field_stats()["algo"] == algo
        g.set_state(pk.F_I, I)
        g.compute_field()
        for f in (pk.F_BR, pk.F_BZ):
            assert nerr(g.get(f), ref.get(f)) <= 1e-12

    check("fft")
    path = os.path.join(str(tmp_path), "tune.jsonl")
    ch = g.autotune(reps=1, cache_path=path)
    assert ch[0] in (1, 2, 3)
    check({1: "direct", 2: "translation", 3: "fft"}[ch[0]])
    g.set_tiles(64, 2, 0)
    check("direct")
    rec = json.loads(open(path).read().splitlines()[0])
    rec.update({"algo": 3, "p1": 0, "p2": 0, "p3": 0})
    with open(path, "w") as fh:
        fh.write(json.dumps(rec) + "\n")
    assert g.autotune(reps=1, cache_path=path) == (3, 0, 0, 0)
    check("fft")
    with pytest.raises(pk.CoilError):
        ref.autotune(reps=1, cache_path=path)


@pytest.mark.parametrize("algo", ["translation", "fft"])
def test_overlapped_run_equals_single_steps(algo):
    """Under the fast convolution coil_run puts the heat step and the
    reductions of each step on a second stream, overlapping the next field
    pass; coil_step does not (nor does any step under the translation pass).
    Both give the same state bitwise: on the active run (T and the per-wire
    sums move), with report points (joins inside the run), and as a graph
    capture of overlapped steps."""
    pk = _pk()
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    a = pk.Coil(w, inp, precision="mixed", algo=algo)
    for _ in range(150):
        a.step()
    b = pk.Coil(w, inp, precision="mixed", algo=algo)
    seen = []
    b.run(150, report_every=40, cb=lambda d: seen.append(float(d[1])))
    c = pk.Coil(w, inp, precision="mixed", algo=algo)
    c.graph(10)
    c.run(150)
    assert seen == [40.0, 80.0, 120.0, 150.0]
    fields = (pk.F_I, pk.F_BR, pk.F_BZ, pk.F_T, pk.F_PHI, pk.F_QW, pk.F_UW)
    for g in (b, c):
        for f in fields:
            assert np.array_equal(a.get(f), g.get(f))
        sa, sg = a.scalars(), g.scalars()
        for k in ("Q", "T_peak", "max_x", "step"):
            assert sa[k] == sg[k]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", [(5, 1, 1), (1, 256, 8), (3, 33, 3)])
def test_fft_extreme_lengths_against_oracle(prec, shape):
    """DFT lengths at both ends: one element per row (L = 2, odd row count),
    2048 elements per row (L = 4096, the largest: 64 KiB of FP64 DFT in LDS),
    and a row of 99 (L = 256, most of it zero padding)."""
    pk = _pk()
    layers, turns, ne = shape
    w = cs.Workload(name="fftlen", coils=[cs.Coil(layers=layers, turns=turns, ne=ne, ramp=1.0)], steps=1, dt=1e-4)
    g = pk.Coil(w, precision=prec, algo="fft")
    o = oracle.Sim(w, field_only=True)
    I = cs.random_currents(w.n_elem, seed=3 + sum(shape))
    tg = cs.sample_indices(w.n_elem, min(w.n_elem, 256), seed=4)
    tg = np.unique(np.concatenate([tg, [0, w.n_elem - 1]]))
    g.set_state(pk.F_I, I)
    g.compute_field()
    obr, obz = o.field_targets(I, tg)
    scale = max(np.abs(obr).max(), np.abs(obz).max())
    e = max(np.abs(g.get(pk.F_BR)[tg] - obr).max(), np.abs(g.get(pk.F_BZ)[tg] - obz).max()) / scale
    _say(f"  fft {shape} {prec}: {e:.2e}")
    assert e <= (1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("variant", ["subelements", "em", "adi", "rho_n"])
def test_fft_with_extended_models_against_oracle(variant):
    """The fast-convolution field under the other wire and heat kernels (the
    subelement solve, the variable step, the ADI heat step, the normal-state
    path): FP64 runs of the active C1 case against the oracle."""
    pk = _pk()
    w = cs.workload("c1_active")
    w = {"subelements": w.replace(subelements=2, dBa_dt=0.5), "em": w.replace(em_tol=1e-5),
         "adi": w.replace(heat_solver="adi"), "rho_n": w.replace(rho_n=3e-10)}[variant]
    inp = cs.generate(w)
    g = pk.Coil(w, inp, precision="fp64", algo="fft")
    o = oracle.Sim(w, inp)
    g.run(150)
    assert o.run(150) == 0
    e = max(nerr(g.get(pk.F_BR), o.get(oracle.BR)), nerr(g.get(pk.F_BZ), o.get(oracle.BZ)),
            nerr(g.get(pk.F_I), o.get(oracle.I)), nerr(g.get(pk.F_PHI), o.get(oracle.PHI)))
    To, Tg = o.get(oracle.T), g.get(pk.F_T)
    rise = float((To - w.T_bath).max())
    dT = float(np.abs(Tg - To).max() / rise) if rise > 0 else 0.0
    floor = 8 * 2.220446049250313e-16 * float(To.max()) / rise if rise > 0 else 0.0
    if variant == "adi":  # the line solves' condition number, as in the ADI parity tests
        d = w.coils[0].wire_side / w.coils[0].ne
        alpha = w.k0 * (float(To.max()) / w.T_ref) ** w.k_exp / (w.C0 * (w.T_bath / w.T_ref) ** w.cp_exp)
        floor *= 1.0 + 4.0 * alpha * w.dt / d ** 2
    _say(f"  fft {variant}: {e:.2e} dT {dT:.2e} (floor {floor:.1e})")
    assert e <= 1e-10 and dT <= max(1e-10, floor)
