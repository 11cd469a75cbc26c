"""Pins of the oracle's subelement model (paper, Results, numerical algorithm
paragraph and the paragraph before it: a wire's subelements are uncoupled
under an external field, each keeping zero net current, and coupled under
transport current; the element current is J_H + J_I, both from the
resistivity of the total J^k).  Pinned by Bean's critical state of the
subelements, the reduction to the wire model when nothing splits, the
constraint invariants, and the cases where one component must stay zero."""
import math

import numpy as np
import pytest

import coil_synth as cs
import oracle

MU0 = 4e-7 * math.pi


def _bean(s_sub, n_exp=100.0, ne=16):
    """One wire at R ~ 1 m (planar limit) in a ramped axial field, no
    transport current, Jc independent of B and T (as in the wire-level Bean
    test), with s_sub x s_sub subelements."""
    wside, Jc, Ec = 1e-3, 1e7, 1e-4
    dBa = 4 * Ec / wside
    w = cs.Workload(name="bean_sub", coils=[cs.Coil(layers=1, turns=1, ne=ne, r_inner=1.0 - wside / 2,
                                                    wire_side=wside, ramp=0.0)],
                    steps=1, dt=1e-4, Ec=Ec, n=n_exp, Jc0=Jc, Tc=1e30, B0=1e30, dBa_dt=dBa,
                    jc_disorder=("none", 0.0), eps_range=(0.0, 0.0), subelements=s_sub)
    s = oracle.Sim(w)
    Bp = MU0 * Jc * wside / 2
    s.run(int(3 * Bp / dBa / w.dt))
    return s, w, Jc, wside


def _sub_index(s, w, s_sub):
    """Elements of wire 0 and the subelement of each, from its position."""
    return s.wire_elems(0), _sub_index_wire(s, w, 0, s_sub)


@pytest.mark.parametrize("s_sub,tol", [(0, 0.02), (2, 0.03), (4, 0.05)])
def test_bean_magnetisation_of_uncoupled_subelements(s_sub, tol):
    """Fully penetrated, each subelement carries +-Jc split by its own
    mid-plane parallel to the field: the magnetisation per volume is
    Jc (w/s)/4, so it falls as 1/s with the subelement count per side
    (computed here from the ideal pattern on the grid, ring radii included)."""
    s, w, Jc, wside = _bean(s_sub)
    I, r = s.get(oracle.I), s.get(oracle.R)
    V = 2 * math.pi * 1.0 * wside * wside
    M = np.sum(math.pi * r * r * I) / V
    n = max(s_sub, 1)
    el, sub = _sub_index(s, w, n)
    d2 = (wside / w.coils[0].ne) ** 2
    rc = np.array([r[el][sub == k].mean() for k in range(n * n)])
    ideal = -Jc * d2 * np.sign(r[el] - rc[sub])
    M_ideal = np.sum(math.pi * r[el] ** 2 * ideal) / V
    assert M_ideal == pytest.approx(-Jc * wside / (4 * n), rel=2e-3)
    assert abs(M / M_ideal - 1) < tol
    # zero net current in every subelement, to rounding
    for k in range(n * n):
        assert abs(I[el][sub == k].sum()) < 1e-12 * np.abs(I).sum()
    assert np.array_equal(s.get(oracle.IH), I) or s_sub == 0


def test_one_element_subelements_carry_no_field_current():
    """Subelements of one element each: a zero-net-current element carries
    nothing, so a field ramp without transport leaves every current at zero
    (to the rounding of the constrained solve, against Jc d^2 of the Bean
    state) and produces no heat (against the one-subelement run)."""
    s, w, Jc, wside = _bean(16, ne=16)
    ref, _, _, _ = _bean(1, ne=16)
    assert np.abs(s.get(oracle.I)).max() < 1e-7 * Jc * (wside / 16) ** 2
    assert s.scalars()["Q"] < 1e-12 * ref.scalars()["Q"]


def _c1(**kw):
    w = cs.workload("c1_active").replace(**kw)
    return w, cs.generate(w)


def test_single_subelement_equals_wire_model():
    """s = 1: the two constrained solves share the wire matrix and their drives
    add up to the wire model's, so the total current is the wire model's
    (the active C1 run: transport ramp, inter-wire drive, flux jumps)."""
    w, inp = _c1()
    a = oracle.Sim(w, inp)
    b = oracle.Sim(w.replace(subelements=1), inp)
    for _ in range(3):
        assert a.run(100) == 0 and b.run(100) == 0
        for f in (oracle.I, oracle.PHI, oracle.T, oracle.BZ, oracle.UW):
            ref = a.get(f)
            assert np.abs(b.get(f) - ref).max() <= 1e-11 * np.abs(ref).max()
    assert a.scalars()["max_x"] > 1.0
    assert b.scalars()["Q"] == pytest.approx(a.scalars()["Q"], rel=1e-11)


def test_transport_only_keeps_field_component_zero():
    """One wire, transport ramp, no background ramp: nothing drives J_H (no
    other wire, no dB_a), so I_H stays zero and the subelement run equals the
    wire model whatever the subelement count."""
    c = cs.Coil(layers=1, turns=1, ne=8, ramp=2000.0)
    w, inp = _c1(coils=[c], dBa_dt=0.0)
    a = oracle.Sim(w, inp)
    b = oracle.Sim(w.replace(subelements=4), inp)
    assert a.run(300) == 0 and b.run(300) == 0
    assert np.abs(b.get(oracle.IH)).max() == 0.0
    I = a.get(oracle.I)
    assert np.abs(b.get(oracle.I) - I).max() <= 1e-12 * np.abs(I).max()
    assert np.abs(I).max() > 0


def test_field_only_single_subelement_is_all_field_current():
    """No transport current and s = 1: J_I is never driven, so I_H is the
    whole current (and equals the wire model's)."""
    w, inp = _c1(coils=[cs.Coil(layers=2, turns=3, ne=8, ramp=0.0)], dBa_dt=0.5)
    a = oracle.Sim(w, inp)
    b = oracle.Sim(w.replace(subelements=1), inp)
    assert a.run(200) == 0 and b.run(200) == 0
    I = b.get(oracle.I)
    assert np.abs(I).max() > 0
    assert np.abs(b.get(oracle.IH) - I).max() <= 1e-14 * np.abs(I).max()
    assert np.abs(a.get(oracle.I) - I).max() <= 1e-11 * np.abs(I).max()


def test_invariants_and_split_matter_on_active_run():
    """Active C1 with 2 x 2 subelements per wire: zero net I_H per subelement
    and the transport current per wire at every checkpoint, the energy
    balance exact, and a response different from the wire model's (the
    split changes the physics)."""
    w, inp = _c1(subelements=2)
    s = oracle.Sim(w, inp)
    a = oracle.Sim(w.replace(subelements=0), inp)
    for k in range(3):
        assert s.run(100) == 0 and a.run(100) == 0
        I, IH = s.get(oracle.I), s.get(oracle.IH)
        scale = np.abs(I).max()
        for wi in range(s.Nw):
            el = s.wire_elems(wi)
            c = w.coils[0]
            It = c.ramp * w.dt * 100 * (k + 1)
            assert abs(I[el].sum() - It) <= 1e-12 * scale * len(el)
            sub = _sub_index_wire(s, w, wi, 2)
            for q in range(4):
                assert abs(IH[el][sub == q].sum()) <= 1e-12 * scale * len(el)
    sc = s.scalars()
    assert sc["stored"] == pytest.approx(sc["Q"] - sc["Q_out"], rel=1e-12)
    assert np.abs(s.get(oracle.I) - a.get(oracle.I)).max() > 0.05 * np.abs(a.get(oracle.I)).max()


def _sub_index_wire(s, w, wi, s_sub):
    el = s.wire_elems(wi)
    r, z = s.get(oracle.R)[el], s.get(oracle.Z)[el]
    c = w.coils[0]
    d = c.wire_side / c.ne
    a = np.floor((r - (r.min() - d / 2)) / (c.wire_side / s_sub)).astype(int)
    b = np.floor((z - (z.min() - d / 2)) / (c.wire_side / s_sub)).astype(int)
    return a * s_sub + b


def test_rejects_inconsistent_options():
    """ne not divisible by the subelement count, or the subelement model
    together with the fully coupled induction: the oracle refuses."""
    w, inp = _c1(subelements=3)
    with pytest.raises(Exception):
        oracle.Sim(w, inp)
    w, inp = _c1(subelements=2, coupling="full")
    with pytest.raises(Exception):
        oracle.Sim(w, inp)
