"""GPU adjoint: transposed field pass (dot-product test), gradients against the
oracle's tangent-linear model, checkpoint/field-history invariance, and
central finite differences at the 384,000-element size."""
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


@pytest.mark.parametrize("algo", ["direct", "translation", "fft"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
# (33, 2, 8) and (87, 1, 3): 264 and 261 element rows, more than one 256-row
# block of the fast convolution's bin products (two target blocks and two
# source parts; in FP64 the unpacked spectra)
@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 4), (3, 9, 8), (5, 7, 6), (2, 70, 8), (33, 2, 8), (87, 1, 3)])
def test_field_transpose_dot_product(prec, tol, shape, algo):
    pk = _pk()
    w = cs.Workload(name="t", coils=[cs.Coil(*shape)], steps=1, dt=1e-4)
    g = pk.Coil(w, precision=prec, algo=algo)
    x = cs.random_currents(w.n_elem, seed=21)
    yr = cs.random_currents(w.n_elem, seed=22)
    yz = cs.random_currents(w.n_elem, seed=23)
    g.set_state(pk.F_I, x)
    g.compute_field()
    lhs = np.dot(g.get(pk.F_BR), yr) + np.dot(g.get(pk.F_BZ), yz)
    gt = g.field_transpose(yr, yz)
    rhs = np.dot(x, gt)
    scale = np.abs(x).sum() * np.abs(gt).max() + 1e-300
    _say("dot", prec, shape, algo, lhs, rhs)
    assert abs(lhs - rhs) <= tol * scale
    # and against the oracle's field sum, column by column on a few sources
    o = oracle.Sim(w, field_only=True)
    for j in (0, w.n_elem // 2, w.n_elem - 1):
        ej = np.zeros(w.n_elem)
        ej[j] = 1.0
        br, bz = o.field_targets(ej, np.arange(w.n_elem))
        ref = np.dot(br, yr) + np.dot(bz, yz)
        ref_abs = np.abs(br * yr).sum() + np.abs(bz * yz).sum()
        assert abs(gt[j] - ref) <= 10 * tol * ref_abs


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_field_transpose_every_width(prec, tol):
    """Transposed translation pass with every forced segment width: dot-product
    identity with the forward pass of the same width."""
    pk = _pk()
    w = cs.Workload(name="t", coils=[cs.Coil(2, 70, 8), cs.Coil(3, 2, 6, r_inner=0.03)], steps=1, dt=1e-4)
    g = pk.Coil(w, precision=prec, algo="translation")
    x = cs.random_currents(w.n_elem, seed=31)
    yr = cs.random_currents(w.n_elem, seed=32)
    yz = cs.random_currents(w.n_elem, seed=33)
    for W in (2, 3, 4, 5, 6, 7, 8):
        g.set_widths(W)
        g.set_state(pk.F_I, x)
        g.compute_field()
        lhs = np.dot(g.get(pk.F_BR), yr) + np.dot(g.get(pk.F_BZ), yz)
        gt = g.field_transpose(yr, yz)
        rhs = np.dot(x, gt)
        scale = np.abs(x).sum() * np.abs(gt).max() + 1e-300
        _say("dot width", prec, W, lhs, rhs)
        assert abs(lhs - rhs) <= tol * scale


def _direction(w, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(w.n_wire), rng.standard_normal(len(w.coils)) * 10.0


@pytest.mark.parametrize("algo", ["direct", "translation", "fft"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_adjoint_matches_oracle_tangent(prec, tol, algo):
    pk = _pk()
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    nsteps = 300
    g = pk.Coil(w, inp, precision=prec, algo=algo)
    for seed in (1, 2):
        dcw, dramp = _direction(w, seed)
        obj_o, dobj = oracle.tangent(w, inp, dcw, dramp, nsteps)
        for wQ, wT, k in ((1.0, 0.0, 0), (0.0, 1.0, 1)):
            gcw, gr, obj = g.adjoint(nsteps, wQ=wQ, wT=wT, ckpt_every=50)
            dd = float(np.dot(gcw, dcw) + np.dot(gr, dramp))
            _say(f"{prec} seed {seed} obj {k}: adjoint {dd:.12e} tangent {dobj[k]:.12e} "
                 f"Q {obj[0]:.6e}/{obj_o[0]:.6e} Tpk {obj[1]:.6f}/{obj_o[1]:.6f}")
            assert abs(obj[0] - obj_o[0]) <= tol * abs(obj_o[0])
            assert abs(dd - dobj[k]) <= tol * abs(dobj[k])


def test_adjoint_checkpoint_and_history_invariance():
    pk = _pk()
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    g = pk.Coil(w, inp)
    a = g.adjoint(260, wQ=1.0, wT=0.5, ckpt_every=50, store_field=True)
    b = g.adjoint(260, wQ=1.0, wT=0.5, ckpt_every=37, store_field=False)
    c = g.adjoint(260, wQ=1.0, wT=0.5, ckpt_every=260, store_field=True)
    for x in (b, c):
        assert np.array_equal(a[0], x[0]) and np.array_equal(a[1], x[1]) and a[2] == x[2]
    # the handle is reset: a forward run reproduces the objectives
    Q, Tp = g.objectives(260)
    assert (Q, Tp) == a[2]


def test_autograd_function():
    import torch
    pk = _pk()
    from paper_2403_07666_amd.autograd import CoilObjective
    w = cs.workload("c1_active")
    inp = cs.generate(w)
    g = pk.Coil(w, inp)
    cw = torch.ones(w.n_wire, dtype=torch.float64, requires_grad=True)
    ramp = torch.tensor([w.coils[0].ramp], dtype=torch.float64, requires_grad=True)
    obj = CoilObjective.apply(cw, ramp, g, 200)
    (obj[0] + 2.0 * obj[1]).backward()
    gcw, gr, o2 = g.adjoint(200, wQ=1.0, wT=2.0)
    assert np.allclose(cw.grad.numpy(), gcw, rtol=0, atol=0)
    assert np.allclose(ramp.grad.numpy(), gr, rtol=0, atol=0)
    assert obj[0].item() == o2[0]


def test_adjoint_central_differences_384k():
    """C5 size (60 layers x 100 turns x 8x8 = 384,000 elements), mixed precision,
    short horizon: dQ/dc_w by central differences (h = 1e-4) on seeded wires."""
    pk = _pk()
    w = cs.workload("c5")
    inp = cs.generate(w)
    nsteps = 3
    g = pk.Coil(w, inp, precision="mixed")
    gcw, gr, obj = g.adjoint(nsteps, wQ=1.0, wT=0.0, ckpt_every=2)
    wires = cs.fd_wires(w.n_wire, 20, 55)[:4]
    h = 1e-4
    for wi in wires:
        vals = []
        for sgn in (+1, -1):
            cw = inp["c_wire"].copy()
            cw[wi] += sgn * h
            g.set_params(cw, None)
            vals.append(g.objectives(nsteps)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        _say(f"wire {wi}: adjoint {gcw[wi]:.10e} fd {fd:.10e}")
        assert gcw[wi] == pytest.approx(fd, rel=1e-5)
    g.set_params(inp["c_wire"], None)


@pytest.mark.timeout(900)
def test_c5_active_central_differences_all_seeded_wires():
    """The adjoint configuration at full size (60 layers x 100 turns x 8x8 =
    384,000 elements) in its driven variant, FP64, over a 100-step horizon:
    dQ/dc_w on all 20 seeded wires and dQ/d(ramp) against central differences
    with h = 1e-4, relative error <= 1e-5."""
    pk = _pk()
    w = cs.workload("c5_active")
    inp = cs.generate(w)
    nsteps = 100
    g = pk.Coil(w, inp, precision="fp64")
    gcw, gr, obj = g.adjoint(nsteps, wQ=1.0, wT=0.0, ckpt_every=50)
    _say(f"c5_active: Q {obj[0]:.6e}")
    assert obj[0] > 1e-3
    h = 1e-4
    worst = 0.0
    for wi in cs.fd_wires(w.n_wire, 20, 55):
        vals = []
        for sgn in (+1, -1):
            cw = inp["c_wire"].copy()
            cw[wi] += sgn * h
            g.set_params(cw, None)
            vals.append(g.objectives(nsteps)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        rel = abs(gcw[wi] - fd) / abs(fd)
        worst = max(worst, rel)
        _say(f"  wire {wi}: adjoint {gcw[wi]:.10e} fd {fd:.10e} rel {rel:.2e}")
        assert rel <= 1e-5
    g.set_params(inp["c_wire"], None)
    rv = []
    for sgn in (+1, -1):
        g.set_params(None, np.array([w.coils[0].ramp + sgn * h]))
        rv.append(g.objectives(nsteps)[0])
    fdr = (rv[0] - rv[1]) / (2 * h)
    _say(f"  ramp: adjoint {gr[0]:.10e} fd {fdr:.10e}; worst wire {worst:.2e}")
    assert abs(gr[0] - fdr) <= 1e-5 * abs(fdr)
