"""Write tests/golden/c2_prefix.json: the oracle's first steps of the full
131,072-element coil (32 layers x 64 turns x 8x8 elements, seeded inputs), at
seeded sampled elements and wires.

Calls only oracle/ and coil_synth/.  Cost: the oracle's transport-flux pattern
and every field pass are O(N^2) plain-C evaluations (~1.7e10 each), about 7.5
minutes each on 8 cores (the stored 20 steps took about 2.5 hours).

    python tests/golden/make_c2_prefix.py [--steps 20] [--out PATH]

The file is rewritten after every step, so a long run leaves a usable prefix.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import coil_synth as cs  # noqa: E402
import oracle  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    path = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{args.workload}_prefix.json")
    w = cs.workload(args.workload)
    inp = cs.generate(w)
    t0 = time.time()
    s = oracle.Sim(w, inp)
    print(f"create (incl. transport-flux pattern) {time.time() - t0:.0f} s", flush=True)
    elems = cs.sample_indices(w.n_elem, 512, seed=77)
    wires = cs.sample_indices(w.n_wire, 16, seed=78)
    rec = {
        "workload": w.name, "n_elem": w.n_elem, "n_wire": w.n_wire, "oracle_threads": oracle.threads(),
        "elements": elems.tolist(), "wires": wires.tolist(),
        "psi": s.get(oracle.PSI)[elems].tolist(), "steps": [],
    }
    for k in range(args.steps):
        t0 = time.time()
        rc = s.step()
        assert rc == 0
        sc = s.scalars()
        rec["steps"].append({
            "step": k + 1,
            "I": s.get(oracle.I)[elems].tolist(),
            "Br": s.get(oracle.BR)[elems].tolist(),
            "Bz": s.get(oracle.BZ)[elems].tolist(),
            "T": s.get(oracle.T)[elems].tolist(),
            "Phi": s.get(oracle.PHI)[elems].tolist(),
            "Uw": s.get(oracle.UW)[wires].tolist(),
            "Q": sc["Q"], "sumU": sc["sumU"], "max_x": sc["max_x"],
        })
        with open(path + ".tmp", "w") as f:
            json.dump(rec, f)
        os.replace(path + ".tmp", path)
        print(f"step {k + 1} {time.time() - t0:.0f} s, wrote {path}", flush=True)


if __name__ == "__main__":
    main()
