"""GPU parity of the HIP path against the CPU oracle on the same seeded inputs,
through the C ABI.  Tolerances: 1e-10 (FP64 mode) and 1e-5 (mixed mode),
normwise relative (max |x - x_ref| / max |x_ref|) on B, I and T; T also
relative to its rise above the bath when it rises."""
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
    scale = np.abs(b).max()
    if scale == 0.0:
        return float(np.abs(a).max())
    return float(np.abs(a - b).max() / scale)


def _coil(layers, turns, ne, **kw):
    return cs.Workload(name="t", coils=[cs.Coil(layers=layers, turns=turns, ne=ne, ramp=kw.pop("ramp", 1.0))],
                       steps=1, dt=kw.pop("dt", 1e-4), **kw)


# the last two have more than 256 element rows (264, and 261 padded to 264):
# two row blocks of the fast convolution, in FP64 its unpacked spectra
SHAPES = [(1, 1, 1), (1, 1, 8), (2, 3, 3), (3, 5, 4), (4, 8, 4), (5, 7, 6), (3, 9, 8), (33, 2, 8), (87, 1, 3)]


ALGOS = ["direct", "translation", "fft"]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", SHAPES)
def test_field_pass_random_currents(prec, shape, algo):
    """Field pass alone on seeded random currents: every target."""
    pk = _pk()
    w = _coil(*shape)
    _say("field", prec, shape, algo)
    g = pk.Coil(w, precision=prec, algo=algo)
    o = oracle.Sim(w)
    I = cs.random_currents(w.n_elem, seed=100 + sum(shape))
    g.set_state(pk.F_I, I)
    g.compute_field()
    br, bz = g.get(pk.F_BR), g.get(pk.F_BZ)
    obr, obz = o.field_targets(I, np.arange(w.n_elem))
    if w.n_elem == 1:
        assert br[0] == 0.0 and bz[0] == 0.0
        return
    e = max(nerr(br, obr), nerr(bz, obz))
    _say("  err", e)
    assert e <= TOL[prec]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_field_pass_ensemble_of_coils(prec, algo):
    pk = _pk()
    w = cs.Workload(name="ens", coils=[cs.Coil(2, 3, 4, ramp=1.0), cs.Coil(3, 2, 6, r_inner=0.03, ramp=2.0),
                                        cs.Coil(1, 5, 8, z_center=0.01, ramp=0.5),
                                        cs.Coil(2, 70, 8, r_inner=0.021, ramp=0.7)],
                    steps=1, dt=1e-4)
    g = pk.Coil(w, precision=prec, algo=algo)
    o = oracle.Sim(w)
    I = cs.random_currents(w.n_elem, seed=7)
    g.set_state(pk.F_I, I)
    g.compute_field()
    obr, obz = o.field_targets(I, np.arange(w.n_elem))
    e = max(nerr(g.get(pk.F_BR), obr), nerr(g.get(pk.F_BZ), obz))
    _say("ensemble", prec, e)
    assert e <= TOL[prec]


def _ragged_ensemble():
    # turns-element counts 12, 12, 40 and 560: every width leaves a ragged
    # last segment, and 560 spans two source chunks of every width
    return cs.Workload(name="ens", coils=[cs.Coil(2, 3, 4, ramp=1.0), cs.Coil(3, 2, 6, r_inner=0.03, ramp=2.0),
                                          cs.Coil(1, 5, 8, z_center=0.01, ramp=0.5),
                                          cs.Coil(2, 70, 8, r_inner=0.021, ramp=0.7)],
                       steps=1, dt=1e-4)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_every_segment_width(prec):
    """Translation pass with every forced segment width W = 2..8 against the
    oracle at every target; the widths agree with each other to summation order."""
    pk = _pk()
    w = _ragged_ensemble()
    g = pk.Coil(w, precision=prec, algo="translation")
    o = oracle.Sim(w)
    I = cs.random_currents(w.n_elem, seed=17)
    obr, obz = o.field_targets(I, np.arange(w.n_elem))
    g.set_state(pk.F_I, I)
    with pytest.raises(pk.CoilError):
        g.set_widths(9)
    with pytest.raises(pk.CoilError):
        g.set_widths(1)
    ref = None
    for W in [0, 2, 3, 4, 5, 6, 7, 8]:
        g.set_widths(W)
        g.compute_field()
        br, bz = g.get(pk.F_BR), g.get(pk.F_BZ)
        e = max(nerr(br, obr), nerr(bz, obz))
        _say("width", prec, W, g.field_stats()["items"], e)
        assert e <= TOL[prec]
        if ref is None:
            ref = (br, bz)
        else:
            # FP64: the same sums in the same order; mixed: FP32 partial sums
            # over 4W sources, so the rounding depends on W (each width is
            # within ~1e-7 of the oracle)
            assert max(nerr(br, ref[0]), nerr(bz, ref[1])) <= (1e-13 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_c1_full_run(prec, algo):
    """C1 (4 layers x 8 turns x 4x4 elements), literal constants, 500 steps."""
    pk = _pk()
    w = cs.workload("c1")
    inp = cs.generate(w)
    _say("c1 run", prec, algo)
    g = pk.Coil(w, inp, precision=prec, algo=algo)
    o = oracle.Sim(w, inp)
    for k in range(5):
        g.run(100)
        assert o.run(100) == 0
        eb = max(nerr(g.get(pk.F_BR), o.get(oracle.BR)), nerr(g.get(pk.F_BZ), o.get(oracle.BZ)))
        ei = nerr(g.get(pk.F_I), o.get(oracle.I))
        et = nerr(g.get(pk.F_T), o.get(oracle.T))
        # per-wire values (written by one lane of each wire's wavefront): the
        # loop voltage, and in FP64 the Joule heat (its power law amplifies the
        # mixed field error 30-fold at these deeply sub-critical currents)
        eu = nerr(g.get(pk.F_UW), o.get(oracle.UW))
        eqw = nerr(g.get(pk.F_QW), o.get(oracle.QW))
        _say(f"  step {100 * (k + 1)}: B {eb:.2e} I {ei:.2e} T {et:.2e} U_w {eu:.2e} Q_w {eqw:.2e}")
        assert eb <= TOL[prec] and ei <= TOL[prec] and et <= TOL[prec] and eu <= TOL[prec]
        assert prec != "fp64" or eqw <= TOL[prec]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_c1_active_run_temperature_and_joule(prec, algo):
    """Active variant: flux penetrates, E ~ Ec, T rises; T parity relative to
    the rise above the bath, Q and per-wire Q_w, peak temperature."""
    pk = _pk()
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    g = pk.Coil(w, inp, precision=prec, algo=algo)
    o = oracle.Sim(w, inp)
    g.run(350)
    assert o.run(350) == 0
    To, Tg = o.get(oracle.T), g.get(pk.F_T)
    rise = (To - w.T_bath).max()
    assert rise > 0.05
    et = np.abs(Tg - To).max() / rise
    sg, so = g.scalars(), o.scalars()
    eq = abs(sg["Q"] - so["Q"]) / so["Q"]
    eqw = nerr(g.get(pk.F_QW), o.get(oracle.QW))
    eb = max(nerr(g.get(pk.F_BR), o.get(oracle.BR)), nerr(g.get(pk.F_BZ), o.get(oracle.BZ)))
    ei = nerr(g.get(pk.F_I), o.get(oracle.I))
    _say(f"active {prec}: dT {et:.2e} Q {eq:.2e} Qw {eqw:.2e} B {eb:.2e} I {ei:.2e}")
    etl = nerr(Tg, To)
    _say(f"  literal T {etl:.2e}")
    tol = TOL[prec]
    assert et <= tol and etl <= tol and eq <= tol and eqw <= tol
    assert eb <= tol and ei <= tol
    assert abs(sg["T_peak"] - so["T_peak"]) <= TOL[prec] * so["T_peak"]
    if prec == "fp64":
        assert sg["T_peak_elem"] == so["T_peak_elem"] and sg["T_peak_step"] == so["T_peak_step"]
    # energy balance on the GPU state
    assert sg["stored"] == pytest.approx(sg["Q"] - sg["Q_out"], rel=1e-9)


def test_nonfinite_is_reported():
    pk = _pk()
    w = _coil(2, 2, 4)
    g = pk.Coil(w)
    I = cs.random_currents(w.n_elem, seed=1, scale=1e-3)
    g.set_state(pk.F_I, I)
    g.set_state(pk.F_T, np.full(w.n_elem, 19.0))  # above Tc: Jc = 0 with J != 0
    with pytest.raises(pk.CoilError) as ei:
        g.run(1)
    assert ei.value.code == -4
    g.reset()
    g.run(3)  # recovers after reset


def test_graph_replay_matches_eager_bitwise():
    pk = _pk()
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    a = pk.Coil(w, inp)
    b = pk.Coil(w, inp)
    b.graph(10)
    a.run(200)
    b.run(200)
    for f in (pk.F_I, pk.F_T, pk.F_BZ, pk.F_PHI):
        assert np.array_equal(a.get(f), b.get(f))
    # replay again after eager work and a reset
    b.reset()
    b.run(200)
    assert np.array_equal(a.get(pk.F_T), b.get(pk.F_T))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_translation_persistent_grid_is_bitwise(prec):
    """The translation pass on a persistent grid (fewer workgroups than items,
    each striding over the item list) gives the one-item-per-workgroup result
    bit for bit: every item is computed the same way wherever it runs."""
    pk = _pk()
    w = _ragged_ensemble()
    I = cs.random_currents(w.n_elem, seed=5)
    out = []
    for grid in (0, 7, 256):
        g = pk.Coil(w, precision=prec, algo="translation", grid_limit=grid)
        g.set_state(pk.F_I, I)
        g.compute_field()
        out.append((g.get(pk.F_BR), g.get(pk.F_BZ)))
        _say("grid", prec, grid, g.field_stats()["items"])
        g.close()
    for br, bz in out[1:]:
        assert np.array_equal(br, out[0][0]) and np.array_equal(bz, out[0][1])


def test_field_at_probes_against_oracle():
    pk = _pk()
    w = cs.Workload(name="t", coils=[cs.Coil(4, 8, 4), cs.Coil(2, 3, 6, r_inner=0.05, z_center=0.02)],
                    steps=1, dt=1e-4)
    g = pk.Coil(w)
    o = oracle.Sim(w, field_only=True)
    I = cs.random_currents(w.n_elem, seed=61)
    g.set_state(pk.F_I, I)
    r = np.array([0.0, 0.0, 0.005, 0.019, 0.0215, 0.03, 0.06, 0.1])
    z = np.array([0.0, 0.03, -0.01, 0.0, 0.0011, 0.004, 0.02, -0.05])
    br, bz = g.field_at(r, z)
    obr, obz = o.field_points(I, r, z)
    scale = max(np.abs(obr).max(), np.abs(obz).max())
    assert np.abs(br - obr).max() <= 1e-12 * scale and np.abs(bz - obz).max() <= 1e-12 * scale
    assert br[0] == 0.0 and br[1] == 0.0
    with pytest.raises(pk.CoilError):
        g.field_at(np.array([-1.0]), np.array([0.0]))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_save_load_resume_is_bitwise(prec):
    pk = _pk()
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    g = pk.Coil(w, inp, precision=prec)
    g.run(150)
    snap = g.save()
    g.run(150)
    a = [g.get(f) for f in (pk.F_I, pk.F_T, pk.F_PHI, pk.F_QW, pk.F_BZ)]
    sa = g.scalars()
    h = pk.Coil(w, inp, precision=prec)  # a fresh handle of the same configuration
    h.load(snap)
    assert h.scalars()["step"] == 150
    h.run(150)
    b = [h.get(f) for f in (pk.F_I, pk.F_T, pk.F_PHI, pk.F_QW, pk.F_BZ)]
    sb = h.scalars()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    for k in ("Q", "T_peak", "T_peak_elem", "T_peak_step", "Q_out", "stored"):
        assert sa[k] == sb[k], k
    with pytest.raises(pk.CoilError):
        pk.Coil(cs.workload("c1"), cs.generate(cs.workload("c1"))).load(snap[:100])
