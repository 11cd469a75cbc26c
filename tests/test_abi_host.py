"""Host-side checks of the HIP library: it loads, exports every symbol the
header declares, validates configurations, sizes workspaces, and its
elliptic approximations match library values (no GPU work)."""
import math
import os
import re

import numpy as np
import pytest

import coil_synth as cs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _pk():
    import paper_2403_07666_amd as pk
    return pk


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "coil.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(coil_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    pk = _pk()
    L = pk.lib()
    declared = _declared_symbols()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(pk.EXPORTS)


def test_query_sizes_and_substeps_match_workloads():
    import oracle
    pk = _pk()
    for name, N, Nw, nsub in [("c1", 512, 32, 2), ("c2", 131072, 2048, 4), ("c5", 384000, 6000, 4)]:
        w = cs.workload(name)
        s = pk.query(w)
        assert (s.n_elem, s.n_wire, s.heat_substeps) == (N, Nw, nsub)
        assert s.workspace_bytes > 8 * 20 * N
    # the library's substep rule agrees with the oracle's on ensembles too
    w = cs.workload("c4").replace(coils=[cs.Coil(2, 3, 6), cs.Coil(3, 2, 6, ramp=2.0)])
    assert pk.query(w).heat_substeps == oracle.Sim(w).n_sub == 4


def test_validation_errors():
    pk = _pk()
    w = cs.workload("c1")
    bad = [
        w.replace(dt=0.0),
        w.replace(Jc0=-1.0),
        w.replace(coils=[cs.Coil(layers=1, turns=1, ne=9)]),  # 81 elements per wire
        w.replace(coils=[cs.Coil(layers=0, turns=1, ne=2)]),
        w.replace(h0=-1.0),
        w.replace(n=0.5),
    ]
    for b in bad:
        with pytest.raises(pk.CoilError) as ei:
            pk.query(b)
        assert ei.value.code == -1
    with pytest.raises(pk.CoilError):
        pk.query(w, precision=7)
    with pytest.raises(pk.CoilError):
        pk.query(w, tile_targets=100)
    with pytest.raises(pk.CoilError):
        pk.query(w, tile_sources=100)
    # options of the extended model
    for kw, wb in [({}, w.replace(rho_n=-1.0)), ({"geometry": 5}, w), ({"coupling": 7}, w),
                   ({"heat_solver": 9}, w), ({"cg_max_iter": -1}, w), ({}, w.replace(k_exp=float("nan")))]:
        with pytest.raises(pk.CoilError) as ei:
            pk.query(wb, **kw)
        assert ei.value.code == -1
    pk.query(w.replace(rho_n=3e-10), geometry="planar")
    pk.query(w.replace(coils=[cs.Coil(**{**w.coils[0].__dict__, "I0": 2.0})]))
    # subelement model: ne (4 here) a multiple of s, s <= 4, transport-only coupling
    for wb in [w.replace(subelements=-1), w.replace(subelements=5), w.replace(subelements=3),
               w.replace(subelements=2, coupling="full")]:
        with pytest.raises(pk.CoilError) as ei:
            pk.query(wb)
        assert ei.value.code == -1
    assert pk.query(w.replace(subelements=2)).workspace_bytes > pk.query(w).workspace_bytes
    # variable step: em_tol >= 0, em_max_level <= 16, wire model with transport coupling
    for wb in [w.replace(em_tol=-1e-3), w.replace(em_tol=1e-4, em_max_level=17),
               w.replace(em_tol=1e-4, coupling="full"), w.replace(em_tol=1e-4, subelements=2)]:
        with pytest.raises(pk.CoilError) as ei:
            pk.query(wb)
        assert ei.value.code == -1
    pk.query(w.replace(em_tol=1e-4, em_max_level=16))


def test_library_elliptic_approximations():
    from scipy.special import ellipe, ellipkm1
    pk = _pk()
    for m1 in np.concatenate([np.logspace(-9, -1, 33), np.linspace(0.02, 1.0, 50)]):
        K, E = pk.host_ellip(m1, pk.FP64)
        assert abs(K / ellipkm1(m1) - 1) < 1e-15
        assert abs(E / ellipe(1 - m1) - 1) < 1e-15 * max(1.0, -math.log(m1))
        k32, e32 = pk.host_ellip(m1, pk.MIXED)
        assert abs(k32 / ellipkm1(m1) - 1) < 3e-7
        assert abs(e32 / ellipe(1 - m1) - 1) < 3e-7


def test_fft_algorithm_workspace():
    """COIL_ALGO_FFT keeps per coil and bin (L/2 + 1 bins, L the DFT length, a
    power of two >= 2 n_z - 1) the n_r x n_r matrices of the G_z and G_r
    spectra in the pass's precision -- in FP64, for a coil of at most 256 rows,
    only the packed upper triangle of the symmetric G_r spectrum (rows padded
    to a multiple of 4) -- plus small buffers; an unknown algorithm is refused."""
    pk = _pk()
    w = cs.workload("c1")  # 4 layers x 8 turns of 4 x 4: n_r = 16, n_z = 32, L = 64
    nr, bins = 16, 33
    q, r = nr // 4, nr % 4
    tri = 4 * (q + 1) * (2 * q + r)  # rows j = 0 .. 15 of 4 ceil((j + 1) / 4) reals
    assert tri == sum(4 * (-(-(j + 1) // 4)) for j in range(nr))
    for prec, rs in (("fp64", 8), ("mixed", 4)):
        extra = pk.query(w, precision=prec, algo="fft").workspace_bytes - pk.query(w, precision=prec).workspace_bytes
        spec = bins * (nr * nr + (tri if prec == "fp64" else nr * nr)) * rs
        assert spec <= extra <= spec + 65536
        # the coupled solve adds the FP64 spectra of the mutual-inductance kernel
        wf = w.replace(coupling="full")
        more = (pk.query(wf, precision=prec, algo="fft").workspace_bytes
                - pk.query(wf, precision=prec).workspace_bytes - extra)
        assert abs(more - bins * nr * nr * 8) <= 4096
    with pytest.raises(pk.CoilError) as ei:
        pk.query(w, algo=4)
    assert ei.value.code == -1
