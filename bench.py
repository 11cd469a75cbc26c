"""Benchmark of the coil quench hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2] [--precision mixed]

A step is one full coil_step (field pass, local law + per-wire A-V solve,
explicit heat substeps, reductions) of the 131,072-element coil
(32 layers x 64 turns x 8x8 elements, seeded synthetic inputs), in mixed
precision, with all inputs resident in HBM.  The timed region is K steps
bracketed by device synchronisation; per-kernel durations come from HIP
events the library records on its own stream inside that region.

Validity: before the timed run, the configuration's whole run is made in
mixed precision and in FP64 from the same initial state and the normwise
relative error of B and T (mixed against FP64) is reported every 100 steps;
the run is flagged invalid above 1e-5.  The same check covers the driven
variant, and 200 steps of the 384,000-element adjoint configuration (literal
and driven).

Other legs after the timed run: the 16-coil ensemble, the adjoint/forward
ratio at 384,000 elements, the 20 x 20-turn quench workload (onset and quench
maps, propagation speed), and the CPU oracle baseline.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense, per GPU)
PEAK_FP32_TFLOPS = 157.3      # vector FP32 (published MI355X figure)
PEAK_FP64_TFLOPS = 78.6       # vector FP64: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_HBM_GBS = 8000.0
# Algorithmic work of the field pass (an FMA counts 2, a hardware
# transcendental 1).  One Green's-function evaluation (FP32 formula):
# al2/be2/dz^2 5, rsqrt 1, m1 2, log2 1, K 18, E 18, f 3, al2 K 1, B_z bracket
# 4, B_r bracket 5 -> 58 flop, plus 3 for the coordinates -> 61.  Direct pass:
# one evaluation and 2 accumulation FMAs per pair -> 65 flop per pair.
# Translation pass: each distinct value evaluated once per tile (61 flop) and
# 2 FMAs per pair (4 flop): FP32 FMAs in mixed mode, FP64 FMAs in FP64 mode.
FLOP_PER_EVAL = 61
FLOP_PER_PAIR_ACC = 4

# HBM bytes per launch of the dominant kernel, from two rocprofv3 counter runs
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors a 256 MiB device copy
# reads on the same counters; profiles/ holds the runs).  A record
# holds only while what sets the kernel's traffic is unchanged: the kernel
# source and the host code that plans its work items (the marked region of
# coil_api.hip).
TRAFFIC_SOURCES = {"translation": ("coil_field_tz.hip", "coil_field_tz.h"), "direct": ("coil_kernels.hip",),
                   "fft": ("coil_field_fft.hip", "coil_field_fft.h")}
PLAN_BEGIN, PLAN_END = "// ---- field-pass work plans (begin)", "// ---- field-pass work plans (end)"
MEASURED_TRAFFIC = {
    # (algorithm, workload, precision): (sha1 of the sources, bytes per launch)
    ("translation", "c2_medium_131k", "mixed"): ("49bf2f94a8592ed1a99a38e435825fb9ba4b2d98", 108509798),
    ("fft", "c2_medium_131k", "mixed"): ("eddfdffd22824495e75224e49986c4cc1c6adf01", 275440230),
}


def _code_only(text: str) -> str:
    """The source without its // and /* */ comments and blank lines: what sets the kernel's code."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())


def _sources_sha(algo: str) -> str:
    import hashlib
    csrc = os.path.join(ROOT, "paper_2403_07666_amd", "csrc")
    h = hashlib.sha1()
    for name in TRAFFIC_SOURCES[algo]:
        with open(os.path.join(csrc, name)) as f:
            h.update(_code_only(f.read()).encode())
    with open(os.path.join(csrc, "coil_api.hip")) as f:
        api = f.read()
    h.update(_code_only(api[api.index(PLAN_BEGIN):api.index(PLAN_END)]).encode())
    return h.hexdigest()


def _traffic(workload: str, precision: str, algo: str):
    rec = MEASURED_TRAFFIC.get((algo, workload, precision))
    if rec is None:
        return None
    return rec[1] if _sources_sha(algo) == rec[0] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def nerr(a, b):
    import numpy as np
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / s) if s > 0 else float(np.abs(a).max())


def precision_check(pk, cs, name: str, every: int = 100, direct_steps: int = 100, steps: int = 0) -> dict:
    """Mixed against FP64 over the configuration's whole run: B (normwise, both
    components) and T (literal, and relative to the rise above the bath when
    there is one) compared every `every` steps, maxima reported.  The FP64
    reference is the translation evaluation; the first `direct_steps` are also
    compared with the per-pair direct FP64 evaluation, an independent sum."""
    import numpy as np
    w = cs.workload(name)
    inp = cs.generate(w)
    nsteps = steps if steps > 0 else w.steps
    gm = pk.Coil(w, inp, precision="mixed")
    gr = pk.Coil(w, inp, precision="fp64")
    eb = et = ei = ephi = eq = etp = 0.0
    erise = None
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        gm.run(k)
        gr.run(k)
        done += k
        Tr = gr.get(pk.F_T)
        Tm = gm.get(pk.F_T)
        eb = max(eb, nerr(gm.get(pk.F_BR), gr.get(pk.F_BR)), nerr(gm.get(pk.F_BZ), gr.get(pk.F_BZ)))
        et = max(et, nerr(Tm, Tr))
        ei = max(ei, nerr(gm.get(pk.F_I), gr.get(pk.F_I)))
        ephi = max(ephi, nerr(gm.get(pk.F_PHI), gr.get(pk.F_PHI)))
        sm, sr = gm.scalars(), gr.scalars()
        if sr["Q"] != 0.0:
            eq = max(eq, abs(sm["Q"] - sr["Q"]) / abs(sr["Q"]))
        etp = max(etp, abs(sm["T_peak"] - sr["T_peak"]) / sr["T_peak"])
        rise = float(Tr.max() - w.T_bath)
        if rise > 0.0:
            erise = max(erise or 0.0, float(np.abs(Tm - Tr).max() / rise))
    t_peak = gr.scalars()["T_peak"]
    gr.close()
    gm.reset()
    gd = pk.Coil(w, inp, precision="fp64", algo="direct")
    gm.run(direct_steps)
    gd.run(direct_steps)
    ed = max(nerr(gm.get(pk.F_BR), gd.get(pk.F_BR)), nerr(gm.get(pk.F_BZ), gd.get(pk.F_BZ)))
    etd = nerr(gm.get(pk.F_T), gd.get(pk.F_T))
    gd.close()
    gm.close()
    res = {"workload": w.name, "steps": nsteps, "every": every, "rel_err_B": eb, "rel_err_T": et,
           "rel_err_T_rise": erise, "T_peak_fp64": t_peak,
           "rel_err_other": {"I": ei, "Phi": ephi, "Q": eq, "T_peak": etp},
           "vs_direct_fp64": {"steps": direct_steps, "rel_err_B": ed, "rel_err_T": etd},
           "valid": bool(eb <= 1e-5 and et <= 1e-5 and ed <= 1e-5 and etd <= 1e-5
                         and (erise is None or erise <= 1e-5))}
    log(f"[bench] {w.name}: mixed vs FP64 over {nsteps} steps: B {eb:.2e} T {et:.2e} "
        f"(rise-relative {erise}); vs direct FP64 at step {direct_steps}: B {ed:.2e} T {etd:.2e}")
    return res


def quench_leg(pk, cs, torch, name: str = "quench20_active", max_steps: int = 6000, every: int = 250) -> dict:
    """The quench workload (20 x 20 turns, transport and background field
    ramps, normal-state path): run until every wire has quenched (rho > 0.95
    rho_n) or max_steps, then per-wire onset and quench steps, the quench
    propagation speed 1/|grad t_q| over the wire grid (central differences,
    pitch = wire side), and the Joule heat Q_q of each wire between its onset
    and its quench."""
    import numpy as np
    w = cs.workload(name)
    inp = cs.generate(w)
    g = pk.Coil(w, inp, precision="mixed")
    co = w.coils[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < max_steps:
        g.run(every)
        done += every
        if (g.get(pk.F_QUENCH) >= 0).all():
            break
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    on, qu = g.get(pk.F_ONSET), g.get(pk.F_QUENCH)
    Qq = g.get(pk.F_Q_QUENCH) - g.get(pk.F_Q_ONSET)
    sc = g.scalars()
    g.close()
    tq = qu.reshape(co.layers, co.turns) * w.dt
    speed = None
    if (qu >= 0).all():
        gr, gz = np.gradient(tq, co.wire_side)
        gn = np.hypot(gr, gz)
        v = 1.0 / gn[gn > 0]
        speed = {"median_m_per_s": float(np.median(v)), "p90_m_per_s": float(np.percentile(v, 90)),
                 "max_m_per_s": float(v.max())}
    out = {"workload": w.name, "n_elem": w.n_elem, "steps": done, "steps_per_s": done / el,
           "wires": int(w.n_wire), "onset": int((on >= 0).sum()), "quenched": int((qu >= 0).sum()),
           "first_onset_step": float(on[on >= 0].min()) if (on >= 0).any() else None,
           "first_quench_step": float(qu[qu >= 0].min()) if (qu >= 0).any() else None,
           "last_quench_step": float(qu.max()) if (qu >= 0).all() else None,
           "T_peak": sc["T_peak"], "Q": sc["Q"], "propagation": speed,
           "Qq_range_J": [float(Qq.min()), float(Qq.max())] if (qu >= 0).all() else None}
    log(f"[bench] {w.name}: {out['quenched']}/{w.n_wire} wires quenched after {done} steps "
        f"({out['steps_per_s']:.0f} steps/s), T_peak {sc['T_peak']:.2f} K, speed {speed}")
    return out


def adi_leg(pk, cs, torch, steps: int = 200) -> dict:
    """The composite thermal model on the medium coil's driven variant: ADI
    heat step (copper-sheath conductivity 100 W/(m K) with an Nb3Sn core map,
    k and h proportional to T^3, epoxy between wires).  Reports the step rate,
    the heat phase per step, the energy balance, and the substeps the explicit
    step would need at the same conductivity (its stability limit)."""
    w = cs.composite(cs.workload("c2_active"))
    inp = cs.generate(w)
    inp["k_mult"] = cs.composite_map(w)
    g = pk.Coil(w, inp, precision="mixed")
    g.run(5)
    g.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    g.timing(True)
    g.run(20)
    ph = g.timing_read()
    g.timing(False)
    sc = g.scalars()
    g.close()
    explicit = pk.query(w.replace(heat_solver="explicit", k_exp=0.0, h_exp=0.0, ins_R0=0.0)).heat_substeps
    out = {"workload": w.name, "n_elem": w.n_elem, "steps": steps, "steps_per_s": steps / el,
           "heat_ms_per_step": ph["heat"]["ms"] / 20, "heat_launches_per_step": ph["heat"]["launches"] / 20,
           "explicit_substeps_needed": int(explicit), "T_peak": sc["T_peak"],
           "energy_balance_rel": abs(sc["stored"] - (sc["Q"] - sc["Q_out"])) / max(abs(sc["Q"]), 1e-300)}
    log(f"[bench] {w.name}: {out['steps_per_s']:.0f} steps/s, ADI heat {out['heat_ms_per_step'] * 1e3:.1f} us/step "
        f"(explicit would need {explicit} substeps), energy balance {out['energy_balance_rel']:.1e}")
    return out


def subelement_leg(pk, cs, torch, steps: int = 200) -> dict:
    """The subelement model on the medium coil's driven variant (131,072
    elements, 8 x 8 per wire as 4 x 4 subelements of 2 x 2 elements, mixed
    field pass): step rate and wire phase per step against the wire model's."""
    w = cs.workload("c2_active").replace(subelements=4)
    inp = cs.generate(w)
    out = {"workload": w.name + "_sub4x4", "n_elem": w.n_elem, "subelements_per_wire": 16, "steps": steps}
    for key, wl in (("subelements", w), ("wire_model", w.replace(subelements=0))):
        g = pk.Coil(wl, inp, precision="mixed")
        g.run(5)
        g.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.run(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g.timing(True)
        g.run(20)
        ph = g.timing_read()
        g.timing(False)
        g.close()
        out[key] = {"steps_per_s": steps / el, "wire_ms_per_step": ph["wire"]["ms"] / 20}
    log(f"[bench] {out['workload']}: {out['subelements']['steps_per_s']:.0f} steps/s, wire phase "
        f"{out['subelements']['wire_ms_per_step'] * 1e3:.1f} us/step (wire model "
        f"{out['wire_model']['steps_per_s']:.0f} steps/s, {out['wire_model']['wire_ms_per_step'] * 1e3:.1f} us)")
    return out


def coupled_leg(pk, cs, torch, steps: int = 5) -> dict:
    """The fully coupled inter-wire induction on the medium coil (131,072
    elements, driven variant, mixed field pass): per-step wall time, CG
    iterations to a relative residual of 1e-10, and the time of the coupled
    solve (wire phase) against the field pass; with the translation-reuse
    passes (the default) and with the fast-convolution ones (field and flux)."""
    w = cs.workload("c2_active").replace(coupling="full")
    inp = cs.generate(w)
    out = {"workload": w.name + "_coupled", "n_elem": w.n_elem, "steps": steps}
    for algo in ("auto", "fft"):
        g = pk.Coil(w, inp, precision="mixed", cg_tol=1e-10, cg_max_iter=200, algo=algo)
        g.run(2)
        g.timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.run(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ph = g.timing_read()
        g.timing(False)
        sc = g.scalars()
        g.close()
        rec = {"ms_per_step": 1e3 * el / steps, "cg_iters_last_step": int(sc["cg_iters"]),
               "cg_residual_last_step": sc["cg_residual"],
               "phase_ms_per_step": {k: v["ms"] / steps for k, v in ph.items()}}
        # each CG iteration is one FP64 all-pairs flux pass plus per-wire solves
        # and two global reductions: its time against the mixed field pass's
        it = max(1, rec["cg_iters_last_step"])
        rec["ms_per_cg_iteration"] = rec["phase_ms_per_step"]["wire"] / it
        log(f"[bench] {out['workload']} ({algo}): {rec['ms_per_step']:.1f} ms/step, {rec['cg_iters_last_step']} CG "
            f"iterations ({rec['ms_per_cg_iteration']:.3f} ms each, field pass "
            f"{rec['phase_ms_per_step']['field']:.3f} ms)")
        if algo == "auto":
            out.update(rec)
        else:
            out["fft"] = rec
    return out


def fft_spectra_bytes(w, precision: str) -> int:
    """Bytes of the fast-convolution pass's spectra (streamed once per pass):
    per coil 2 (L/2 + 1) n_r n_r4 reals, L the power of two >= 2 n_z - 1 and
    n_r4 the rows rounded up to 4."""
    total = 0
    for c in w.coils:
        nr, nz = c.layers * c.ne, c.turns * c.ne
        L = 2
        while L < 2 * nz - 1:
            L *= 2
        total += 2 * (L // 2 + 1) * nr * ((nr + 3) // 4 * 4)
    return total * (4 if precision == "mixed" else 8)


def fft_leg(pk, cs, torch, steps: int = 1000) -> dict:
    """The fast-convolution field evaluation (COIL_ALGO_FFT) on the medium coil
    (131,072 elements), the 16-coil ensemble (617,472) and the adjoint coil
    (384,000): step rate and field pass against the translation-reuse pass,
    mixed against FP64 and FP64 against the FP64 translation pass on the
    driven variant, and the adjoint over forward ratio with it.  The field pass is HBM-bound on its spectra;
    the effective rate below counts only their bytes over the whole pass
    (three kernels), a lower bound of the bin-product kernel's."""
    out = {}
    for name, n in (("c2", steps), ("c4", max(1, steps // 2)), ("c5", max(1, steps // 4))):
        w = cs.workload(name)
        inp = cs.generate(w)
        rec = {"n_elem": w.n_elem, "steps": n}
        for algo in ("fft", "translation"):
            t0 = time.perf_counter()
            g = pk.Coil(w, inp, precision="mixed", algo=algo)
            torch.cuda.synchronize()
            init = time.perf_counter() - t0
            g.run(5)
            m = n if algo == "fft" else max(1, n // 10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.run(m)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            g.timing(True)
            g.run(20)
            ph = g.timing_read()
            g.timing(False)
            g.close()
            rec[algo] = {"steps_per_s": m / el, "init_s": init,
                         "phase_ms_per_step": {k: v["ms"] / 20 for k, v in ph.items()}}
        sb = fft_spectra_bytes(w, "mixed")
        fms = rec["fft"]["phase_ms_per_step"]["field"]
        rec["spectra_bytes"] = sb
        rec["field_pass_effective_GBps"] = sb / (fms * 1e-3) / 1e9
        rec["speedup_steps_per_s"] = rec["fft"]["steps_per_s"] / rec["translation"]["steps_per_s"]
        log(f"[bench] fft {name}: {rec['fft']['steps_per_s']:.0f} steps/s (translation "
            f"{rec['translation']['steps_per_s']:.0f}), field pass {fms * 1e3:.1f} us, spectra {sb / 1e6:.0f} MB "
            f"-> {rec['field_pass_effective_GBps']:.0f} GB/s over the pass")
        out[name] = rec
    # validity on the driven variant: mixed against FP64 (both FFT), FP64 FFT against FP64 translation
    w = cs.workload("c2_active")
    inp = cs.generate(w)
    res = {}
    for key, prec, algo in (("mixed_fft", "mixed", "fft"), ("fp64_fft", "fp64", "fft"),
                            ("fp64_translation", "fp64", "translation")):
        g = pk.Coil(w, inp, precision=prec, algo=algo)
        g.run(300)
        res[key] = [g.get(f) for f in (pk.F_BR, pk.F_BZ, pk.F_I, pk.F_T)]
        g.close()
    out["driven_300_steps"] = {
        "mixed_vs_fp64": {k: nerr(a, b) for k, a, b in zip(("Br", "Bz", "I", "T"), res["mixed_fft"], res["fp64_fft"])},
        "fp64_vs_fp64_translation": {k: nerr(a, b) for k, a, b in zip(("Br", "Bz", "I", "T"), res["fp64_fft"],
                                                                          res["fp64_translation"])}}
    log(f"[bench] fft driven c2, 300 steps: mixed vs FP64 {out['driven_300_steps']['mixed_vs_fp64']}, "
        f"FP64 vs translation {out['driven_300_steps']['fp64_vs_fp64_translation']}")
    _, adj = _adjoint_ratio(pk, cs, torch, "c5", 200, 50, algo="fft")
    out["adjoint_c5"] = adj
    return out


def cpu_baseline(w, budget_s: float = 12.0) -> dict:
    """The oracle's field sum (the O(N^2) part of a step) on a bounded sample
    of targets of the same coil, all N sources, on the host cores; scaled to
    steps/s of the full coil."""
    import coil_synth as cs
    import oracle
    o = oracle.Sim(w, field_only=True)
    I = cs.random_currents(w.n_elem, seed=5)
    n = 32
    while True:
        tg = cs.sample_indices(w.n_elem, n, seed=9)
        t0 = time.perf_counter()
        o.field_targets(I, tg)
        dt = time.perf_counter() - t0
        if dt * 4 > budget_s or n >= w.n_elem:
            break
        n = min(w.n_elem, int(n * max(2.0, min(8.0, budget_s / max(dt, 1e-3) / 2))))
    pairs = n * (w.n_elem - 1)
    pps = pairs / dt
    # and a whole run of the small configuration (500 steps at 512 elements)
    w1 = cs.workload("c1")
    o1 = oracle.Sim(w1, cs.generate(w1))
    t0 = time.perf_counter()
    o1.run(w1.steps)
    c1_s = time.perf_counter() - t0
    return {
        "value": pps / w.pairs_per_pass(),
        "unit": "steps/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": f"field sum at {n} seeded targets x {w.n_elem} sources "
                  f"({pairs:.3g} pair evaluations, {dt:.1f} s); scaled by pairs per step",
        "pairs_per_s": pps,
        "c1_full_run_s": c1_s,
        "c1_steps_per_s": w1.steps / c1_s,
    }


def batched_leg(pk, cs, torch, steps: int = 50, warmup: int = 3, graph: int = 10) -> dict:
    """The 16-coil ensemble (seeded uneven sizes) in one launch per kernel,
    mixed precision, autotuned field pass, time loop replayed as a HIP graph."""
    w = cs.workload("c4")
    inp = cs.generate(w)
    g = pk.Coil(w, inp, precision="mixed")
    g.run(2)
    t0 = time.perf_counter()
    chosen = g.autotune(reps=2)
    tune_s = time.perf_counter() - t0
    g.reset()
    g.run(warmup)
    g.graph(graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pairs = w.pairs_per_pass()
    g.close()
    out = {
        "workload": w.name, "n_coils": len(w.coils), "n_elem": w.n_elem,
        "coils": [f"{c.layers}x{c.turns}" for c in w.coils],
        "steps": steps, "steps_per_s": steps / dt, "ms_per_step": 1e3 * dt / steps,
        "ginteractions_per_s": pairs * steps / dt / 1e9, "pairs_per_step": pairs,
        "graph_steps": graph, "autotuned": list(chosen), "autotune_s": tune_s,
    }
    log(f"[bench] ensemble {w.n_elem} elements: {out['steps_per_s']:.1f} steps/s, autotuned {chosen}")
    return out


def _adjoint_ratio(pk, cs, torch, name: str, steps: int, ckpt: int, algo: str = "auto"):
    w = cs.workload(name)
    inp = cs.generate(w)
    g = pk.Coil(w, inp, precision="mixed", algo=algo)
    g.run(2)
    g.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run(steps)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    maxx = g.scalars()["max_x"]
    t0 = time.perf_counter()
    gcw, gr, obj = g.adjoint(steps, wQ=1.0, wT=1.0, ckpt_every=ckpt)
    torch.cuda.synchronize()
    adj = time.perf_counter() - t0
    g.close()
    log(f"[bench] adjoint/forward at {w.n_elem} elements ({name}, {algo}), {steps} steps: {adj:.2f} s / "
        f"{fwd:.2f} s = {adj / fwd:.2f} (max |J|/Jc {maxx:.2f})")
    return w, {"workload": w.name, "steps": steps, "forward_s": fwd, "adjoint_s": adj,
               "adjoint_over_forward": adj / fwd, "max_J_over_Jc_last_step": maxx, "objectives": list(obj)}


def adjoint_leg(pk, cs, torch, steps: int, ckpt: int = 50, active_steps: int = 1000) -> dict:
    """Wall time of coil_adjoint (its own forward with checkpoints, recompute,
    reverse sweep) over that of a plain forward run, 384,000 elements, mixed:
    on the literal configuration over `steps` steps, and on its driven variant
    over `active_steps` steps, long enough for flux to penetrate (every wire
    then takes the factorising solve, forward and backward)."""
    w, lit = _adjoint_ratio(pk, cs, torch, "c5", steps, ckpt)
    out = {"workload": w.name, "n_elem": w.n_elem, "steps": steps, "ckpt_every": ckpt,
           "forward_s": lit["forward_s"], "adjoint_s": lit["adjoint_s"],
           "adjoint_over_forward": lit["adjoint_over_forward"], "field_history_in_hbm": True,
           "objectives": lit["objectives"]}
    if active_steps > 0:
        try:
            _, act = _adjoint_ratio(pk, cs, torch, "c5_active", active_steps, ckpt)
        except pk.CoilError as ex:  # e.g. the pure power law past Tc
            act = {"workload": "c5_active", "steps": active_steps, "error": str(ex)}
            log(f"[bench] driven adjoint leg: {ex}")
        out["driven"] = act
    return out


def c5_full(pk, cs, torch, precision: str, fd_steps: int) -> dict:
    """Full-size adjoint configuration: 60 layers x 100 turns x 8x8 elements,
    2000 steps, checkpoints every 50; gradients of Q with respect to the 6000
    per-wire Jc multipliers and the ramp rate."""
    import numpy as np
    w = cs.workload("c5")
    inp = cs.generate(w)
    g = pk.Coil(w, inp, precision=precision)
    g.run(2)
    g.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run(w.steps)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    log(f"[c5] forward {w.steps} steps: {fwd:.1f} s")
    t0 = time.perf_counter()
    gcw, gr, obj = g.adjoint(w.steps, wQ=1.0, wT=1.0, ckpt_every=50)
    torch.cuda.synchronize()
    adj = time.perf_counter() - t0
    log(f"[c5] adjoint {w.steps} steps: {adj:.1f} s -> {adj / fwd:.2f}")
    out = {
        "metric": "adjoint/forward wall time, 384k elements, 2000 steps, checkpoints every 50",
        "value": adj / fwd, "unit": "ratio", "higher_is_better": False, "precision": precision,
        "forward_s": fwd, "adjoint_s": adj, "objectives": list(obj),
    }
    g.close()
    # central differences in FP64 on the seeded wires over a bounded horizon, on the
    # literal configuration (whose Joule heat is tiny and vanishes on quiet wires)
    # and on its driven variant
    out["fd"] = [_fd_check(pk, cs, name, fd_steps) for name in ("c5", "c5_active")]
    return out


def _fd_check(pk, cs, name: str, fd_steps: int) -> dict:
    import numpy as np
    w = cs.workload(name)
    inp = cs.generate(w)
    g = pk.Coil(w, inp, precision="fp64")
    wires = cs.fd_wires(w.n_wire, 20, 55)
    gq, gqr, obj = g.adjoint(fd_steps, wQ=1.0, wT=0.0, ckpt_every=50)
    h = 1e-4
    per_wire = []
    for wi in wires:
        vals = []
        for sgn in (+1, -1):
            cw = inp["c_wire"].copy()
            cw[wi] += sgn * h
            g.set_params(cw, None)
            vals.append(g.objectives(fd_steps)[0])
        per_wire.append((int(wi), float(gq[wi]), (vals[0] - vals[1]) / (2 * h)))
        log(f"[{name}] FD wire {wi}: adjoint {gq[wi]:.6e} fd {per_wire[-1][2]:.6e}")
    g.set_params(inp["c_wire"], None)
    rvals = []
    for sgn in (+1, -1):
        g.set_params(None, np.array([w.coils[0].ramp + sgn * h]))
        rvals.append(g.objectives(fd_steps)[0])
    g.close()
    fdr = (rvals[0] - rvals[1]) / (2 * h)
    # relative error where the difference quotient resolves the derivative: its
    # round-off is about eps |Q| / h, so a wire counts when |fd| exceeds that by
    # 1e3; the others (Joule heat too small to move Q by more than an ulp, or
    # not at all) are counted, with their largest adjoint value
    floor = 2.220446049250313e-16 * abs(float(obj[0])) / h
    live = [(a, f) for _, a, f in per_wire if abs(f) > 1e3 * floor]
    rel = [abs(a - f) / abs(f) for a, f in live]
    res = {"workload": name, "steps": fd_steps, "h": h, "Q": float(obj[0]),
           "wires": per_wire, "fd_roundoff": floor, "n_resolved": len(live),
           "n_below_roundoff": len(per_wire) - len(live),
           "max_abs_adjoint_unresolved": max([abs(a) for _, a, f in per_wire if abs(f) <= 1e3 * floor], default=0.0),
           "max_rel_err_dQ_dcw": max(rel) if rel else None,
           "dQ_dramp": [float(gqr[0]), fdr],
           "rel_err_dQ_dramp": abs(gqr[0] - fdr) / abs(fdr) if fdr != 0 else None}
    log(f"[{name}] FD over {fd_steps} steps (Q {obj[0]:.3e}): {len(live)} resolved wires, max rel err "
        f"dQ/dc_w {res['max_rel_err_dQ_dcw']}, dQ/dramp {res['rel_err_dQ_dramp']}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--no-check", action="store_true", help="skip the FP64 validity run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--graph", type=int, default=0, help="capture the step loop in HIP graphs of this many steps")
    ap.add_argument("--algo", default="auto", choices=["auto", "direct", "translation", "fft"],
                    help="field-pass evaluation (both compute the same all-pairs sum)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 16-coil ensemble leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward leg")
    ap.add_argument("--no-quench", action="store_true", help="skip the 20 x 20-turn quench leg")
    ap.add_argument("--no-adi", action="store_true", help="skip the composite (ADI heat step) leg")
    ap.add_argument("--no-coupled", action="store_true", help="skip the fully coupled induction leg")
    ap.add_argument("--no-subelements", action="store_true", help="skip the subelement-model leg")
    ap.add_argument("--no-fft", action="store_true", help="skip the fast-convolution field-pass leg")
    ap.add_argument("--adjoint-steps", type=int, default=200,
                    help="horizon of the adjoint/forward timing at 384,000 elements")
    ap.add_argument("--c5-full", action="store_true",
                    help="instead of the default legs: time forward vs adjoint on the full 384,000-element, "
                         "2000-step configuration (checkpoints every 50) and check dQ/dc_w against central "
                         "differences (h = 1e-4) on the 20 seeded wires over --fd-steps steps")
    ap.add_argument("--fd-steps", type=int, default=100)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="first run a plain device copy of this many MB three times (a known-size "
                         "reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no multi-GPU "
              "path (its sharding is a design note)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import coil_synth as cs
    import paper_2403_07666_amd as pk

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 x {args.copy_calibration} MB device copy")
        del src, dst

    if args.c5_full:
        print(json.dumps(c5_full(pk, cs, torch, args.precision, args.fd_steps)))
        return

    # validity legs first (they also bring the GPU to its sustained clock
    # before the timed region)
    check = check_active = check_c5 = check_c5_active = None
    if not args.no_check and args.precision == "mixed":
        check = precision_check(pk, cs, args.workload)
        if args.workload in ("c1", "c2", "c3", "c5"):
            # the driven variant until shortly before its hot spot passes Tc
            # (C2: Jc reaches 0 near step 900, which the power law reports)
            check_active = precision_check(pk, cs, args.workload + "_active",
                                           steps=600 if args.workload in ("c2", "c5") else 0)
        if args.workload == "c2":
            # the adjoint configuration's size: 200 steps, literal and driven
            check_c5 = precision_check(pk, cs, "c5", steps=200, direct_steps=10)
            check_c5_active = precision_check(pk, cs, "c5_active", steps=200, direct_steps=10)

    w = cs.workload(args.workload)
    inp = cs.generate(w)
    log(f"[bench] {w.name}: N={w.n_elem} wires={w.n_wire} precision={args.precision}")
    t0 = time.perf_counter()
    g = pk.Coil(w, inp, precision=args.precision, algo=args.algo)
    log(f"[bench] init {time.perf_counter() - t0:.2f} s, substeps {g.n_sub}, "
        f"work items {g.sizes.n_work_items}")
    field_stats = g.field_stats()
    g.run(args.warmup)
    if args.graph > 0:
        g.graph(args.graph)
    else:
        g.timing(2)  # events around the field kernel only
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = g.timing_read() if args.graph == 0 else None
    g.timing(False)
    phases = None
    if args.graph == 0:
        # per-phase breakdown from a separate, shorter run with events around every phase
        g.timing(True)
        nph = max(1, min(args.steps, 50))
        g.run(nph)
        tp = g.timing_read()
        g.timing(False)
        phases = {k: v["ms"] / nph for k, v in tp.items()}
    sps = args.steps / elapsed
    log(f"[bench] {args.steps} steps in {elapsed:.3f} s -> {sps:.2f} steps/s")

    pairs = w.pairs_per_pass()
    fs = field_stats
    roofline = None
    if tm is not None and tm["field"]["launches"] > 0 and fs["algo"] == "fft":
        # the fast convolution streams its spectra once per pass: HBM-bound;
        # the events bracket the whole pass (row DFTs and bin products)
        avg_ms = tm["field"]["ms"] / tm["field"]["launches"]
        sb = fft_spectra_bytes(w, args.precision)
        achieved = sb / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": "k_fft_rows_fwd + k_fft_bins + k_fft_rows_inv (fast-convolution "
                    "field pass; the bytes are k_fft_bins' spectra)", "achieved": achieved, "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                    "traffic": _traffic(w.name, args.precision, "fft"),
                    "traffic_unit": "bytes per k_fft_bins launch (HBM, rocprofv3 FETCH_SIZE/WRITE_SIZE)",
                    "avg_launch_ms": avg_ms,
                    "bytes_per_launch": sb, "phase_ms_per_step": phases}
    elif tm is not None and tm["field"]["launches"] > 0:
        avg_ms = tm["field"]["ms"] / tm["field"]["launches"]
        flop = FLOP_PER_EVAL * fs["kernel_evals"] + FLOP_PER_PAIR_ACC * fs["pairs"]
        achieved = flop / (avg_ms * 1e-3) / 1e12
        tz = fs["algo"] == "translation"
        # the pair arithmetic dominates: FP32 in mixed mode (both evaluations),
        # FP64 in FP64 mode
        peak = PEAK_FP32_TFLOPS if args.precision == "mixed" else PEAK_FP64_TFLOPS
        roofline = {
            "bound": "alu",
            "kernel": ((("k_field_tz32" if args.precision == "mixed" else "k_field_tz64")
                        + " (translation-reuse all-pairs field pass)") if tz
                       else "k_field (direct all-pairs field pass)"),
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "frac_fp64_peak": achieved / PEAK_FP64_TFLOPS,
            "traffic": _traffic(w.name, args.precision, fs["algo"]),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE/WRITE_SIZE)",
            "avg_launch_ms": avg_ms,
            "flop_per_launch": flop,
            "pairs_per_launch": fs["pairs"],
            "kernel_evals_per_launch": fs["kernel_evals"],
            "flop_per_eval": FLOP_PER_EVAL,
            "flop_per_pair": FLOP_PER_PAIR_ACC,
            "phase_ms_per_step": phases,
        }

    g.close()

    batched = None
    if not args.no_batched:
        batched = batched_leg(pk, cs, torch)
    adjoint = None
    if not args.no_adjoint and args.adjoint_steps > 0:
        adjoint = adjoint_leg(pk, cs, torch, args.adjoint_steps)
    quench = None
    if not args.no_quench:
        quench = quench_leg(pk, cs, torch)
    adi = None
    if not args.no_adi:
        adi = adi_leg(pk, cs, torch)
    coupled = None
    if not args.no_coupled:
        coupled = coupled_leg(pk, cs, torch)
    subel = None
    if not args.no_subelements:
        subel = subelement_leg(pk, cs, torch)
    fft = None
    if not args.no_fft:
        fft = fft_leg(pk, cs, torch)

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(w)
        log(f"[bench] oracle {cpu['pairs_per_s']:.3g} pairs/s on {cpu['cores']} threads")

    out = {
        "metric": "steps/s @131k elems mixed vs FP64 (rel err<=1e-5); Ginteractions/s; adjoint/fwd",
        "value": sps,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "n_elem": w.n_elem,
            "n_wire": w.n_wire,
            "coil": f"{w.coils[0].layers} layers x {w.coils[0].turns} turns x "
                    f"{w.coils[0].ne}x{w.coils[0].ne} elements" if len(w.coils) == 1 else len(w.coils),
            "precision": args.precision,
            "dt": w.dt,
            "heat_substeps": g.n_sub,
            "seed": w.seed,
            "graph_steps": args.graph,
            "field_algo": field_stats["algo"],
        },
        "ginteractions_per_s": pairs * sps / 1e9,
        "paper_context": "the paper reports no wall-clock or throughput figures; its C/CUDA code ran on "
                         "GeForce RTX 4090 and RTX 3090 cards (FP64 at 1/64 of FP32)",
        "mixed_vs_fp64": check,
        "mixed_vs_fp64_driven": check_active,
        "mixed_vs_fp64_c5": check_c5,
        "mixed_vs_fp64_c5_driven": check_c5_active,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched": batched,
        "adjoint": adjoint,
        "quench": quench,
        "composite_adi": adi,
        "coupled_induction": coupled,
        "subelements": subel,
        "fft_field_pass": fft,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
