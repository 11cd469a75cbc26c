"""Full-size multi-step parity: the first steps of the 131,072-element coil on
the GPU against the oracle's stored values at seeded sampled elements and
wires (tests/golden/c2_prefix.json, written by tests/golden/make_c2_prefix.py
from the oracle alone).  Covers the device transport-flux pattern, the field
pass, the wire solve and the heat step at the benchmark size."""
import json
import os

import numpy as np
import pytest

import coil_synth as cs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_prefix.json")


def _pk():
    import paper_2403_07666_amd as pk
    return pk


def _nerr(a, b):
    b = np.asarray(b)
    s = np.abs(b).max()
    return float(np.abs(np.asarray(a) - b).max() / s) if s > 0 else float(np.abs(a).max())


@pytest.mark.parametrize("algo", ["translation", "direct", "fft"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_c2_prefix_against_oracle(prec, tol, algo):
    with open(GOLDEN) as f:
        gold = json.load(f)
    pk = _pk()
    w = cs.workload(gold["workload"].split("_")[0])
    assert w.name == gold["workload"] and w.n_elem == gold["n_elem"]
    inp = cs.generate(w)
    el = np.array(gold["elements"])
    wi = np.array(gold["wires"])
    g = pk.Coil(w, inp, precision=prec, algo=algo)
    assert _nerr(g.get(pk.F_PSI)[el], gold["psi"]) <= 1e-10  # FP64 in both modes
    for rec in gold["steps"]:
        g.step()
        sc = g.scalars()
        assert sc["step"] == rec["step"]
        errs = {
            "I": _nerr(g.get(pk.F_I)[el], rec["I"]),
            "B": max(_nerr(g.get(pk.F_BR)[el], rec["Br"]), _nerr(g.get(pk.F_BZ)[el], rec["Bz"])),
            "T": _nerr(g.get(pk.F_T)[el], rec["T"]),
            "Phi": _nerr(g.get(pk.F_PHI)[el], rec["Phi"]),
            "U": _nerr(g.get(pk.F_UW)[wi], rec["Uw"]),
        }
        print(prec, algo, rec["step"], {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
        # the first field pass acts on I = 0: B is exactly 0 on both sides
        for k, v in errs.items():
            assert v <= tol, (k, v)
        assert sc["sumU"] == pytest.approx(rec["sumU"], rel=tol)
