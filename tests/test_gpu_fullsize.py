"""Parity at the full benchmark sizes (131,072 and 384,000 elements), in the
launch configuration the benchmark times: the field pass on seeded currents
against the oracle at sampled targets, and properties of the first steps that
hold at any size."""
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
@pytest.mark.parametrize("name", ["c2", "c5"])
def test_field_pass_sampled_targets(name, algo):
    pk = _pk()
    w = cs.workload(name)
    I = cs.random_currents(w.n_elem, seed=31)
    tg = cs.sample_indices(w.n_elem, 192, seed=32)
    # include the coil's corners and a few neighbours of the first sample
    tg = np.unique(np.concatenate([tg, [0, w.n_elem - 1, w.coils[0].n_z - 1, tg[0] + 1]]))
    o = oracle.Sim(w, field_only=True)
    obr, obz = o.field_targets(I, tg)
    scale = max(np.abs(obr).max(), np.abs(obz).max())
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-5)):
        g = pk.Coil(w, precision=prec, algo=algo)
        g.set_state(pk.F_I, I)
        g.compute_field()
        e = max(np.abs(g.get(pk.F_BR)[tg] - obr).max(), np.abs(g.get(pk.F_BZ)[tg] - obz).max()) / scale
        _say(f"{name} {algo} field {prec}: {e:.2e}")
        assert e <= tol
        g.close()


def test_c2_first_steps_properties():
    """Literal C2 (deeply sub-critical): every wire carries exactly the ramped
    transport current; with E negligible the per-step increments repeat, so
    I^k = k I^1; the flux pattern is the same in both precisions."""
    pk = _pk()
    w = cs.workload("c2")
    inp = cs.generate(w)
    out = {}
    for prec in ("fp64", "mixed"):
        g = pk.Coil(w, inp, precision=prec)
        g.run(1)
        I1 = g.get(pk.F_I)
        g.run(3)
        I4 = g.get(pk.F_I)
        out[prec] = (I1, I4, g.get(pk.F_BR), g.get(pk.F_BZ), g.get(pk.F_T))
        sc = g.scalars()
        assert sc["max_x"] < 1e-3 and sc["status"] == 0
        g.close()
    I1, I4 = out["fp64"][0], out["fp64"][1]
    co = w.coils[0]
    # wire sums (public order: rows of n_z, wires are ne x ne blocks)
    grid = I4.reshape(co.n_r, co.n_z).reshape(co.layers, co.ne, co.turns, co.ne).sum(axis=(1, 3))
    assert np.allclose(grid, 4 * co.ramp * w.dt, rtol=1e-12, atol=0)
    assert np.abs(I4 - 4 * I1).max() <= 1e-12 * np.abs(I4).max()
    for a, b in zip(out["mixed"][2:4], out["fp64"][2:4]):
        assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max()
    assert np.array_equal(out["fp64"][4], np.full(w.n_elem, w.T_bath))
