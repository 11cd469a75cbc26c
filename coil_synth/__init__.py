"""Seeded synthetic workloads for the coil quench hot path.

This module only describes workloads (geometry, material constants, time
step, seeds) and draws the seeded random inputs (strain, Jc0 disorder, weak
spots, ensemble sizes).  It holds none of the method's arithmetic: no field,
no constitutive law, no heat step.  Both the HIP library's callers and the
CPU oracle take their inputs from here, so the two sides see the same data.

Element order of every per-element array returned here ("public order"):
coils are concatenated; inside a coil the (r, z) grid is row-major,
``e = i_r * n_z + i_z`` with ``n_r = layers * ne`` radial and
``n_z = turns * ne`` axial elements.  Wire order: ``w = layer * turns + turn``,
coils concatenated.

Workload shapes follow the paper's coil model (Methods, Numerical Algorithm:
square array of wires, axisymmetric cross-section; Results: 20x20 and 40x40
turn coils) at the sizes of the five benchmark configurations.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Coil",
    "Workload",
    "workload",
    "generate",
    "fd_wires",
    "WORKLOADS",
]


@dataclass
class Coil:
    """One solenoid: ``layers`` radial x ``turns`` axial square wires of side
    ``wire_side``, each split into ``ne`` x ``ne`` square current elements.
    The winding pack spans r in [r_inner, r_inner + layers*wire_side] and is
    centred on z = z_center.  Transport current I_t(t) = I0 + ramp * t."""

    layers: int
    turns: int
    ne: int
    r_inner: float = 0.02
    z_center: float = 0.0
    wire_side: float = 1.0e-3
    ramp: float = 1.0
    I0: float = 0.0

    @property
    def n_r(self) -> int:
        return self.layers * self.ne

    @property
    def n_z(self) -> int:
        return self.turns * self.ne

    @property
    def n_elem(self) -> int:
        return self.n_r * self.n_z

    @property
    def n_wire(self) -> int:
        return self.layers * self.turns


@dataclass
class Workload:
    """A complete synthetic run: coils, material law constants, time step,
    precision and the seeded disorder recipe."""

    name: str
    coils: List[Coil]
    steps: int
    dt: float
    precision: str = "fp64"  # "fp64" or "mixed"
    # E-J power law and Jc(B, T, eps)
    Ec: float = 1.0e-4
    n: float = 30.0
    Jc0: float = 2.0e10
    Tc: float = 18.0
    B0: float = 1.0
    eps_coef: float = 900.0
    eps_pow: float = 1.7
    # thermal: C = C0 (T/T_ref)^cp_exp, constant k and h, bath T_bath
    C0: float = 2.0e3
    T_ref: float = 4.2
    cp_exp: float = 3.0
    k0: float = 0.5
    h0: float = 500.0
    T_bath: float = 4.2
    dBa_dt: float = 0.0  # background axial field ramp, T/s
    rho_n: float = 0.0  # normal-state resistivity in parallel with the power law, Ohm m (0 = off)
    k_exp: float = 0.0  # k = k0 (T/T_ref)^k_exp
    h_exp: float = 0.0  # h = h0 (T/T_ref)^h_exp
    coupling: str = "transport"  # inter-wire induction: "transport" or "full"
    heat_solver: str = "explicit"  # "explicit" (sub-cycled) or "adi"
    ins_R0: float = 0.0  # ADI: insulation resistance between wires, m^2 K/W
    subelements: int = 0  # 0: the wire model; s >= 1: s x s subelements per wire (I = I_H + I_I)
    em_tol: float = 0.0  # > 0: variable-step EM integration within the step (relative tolerance)
    em_max_level: int = 0  # finest EM substep dt / 2^level (0 -> 10)
    heat_substeps: int = 0  # 0 = automatic (stability rule)
    # disorder recipe
    seed: int = 1
    jc_disorder: Tuple[str, float] = ("gauss", 0.01)
    weak_spots: int = 0
    weak_factor: float = 0.7
    eps_range: Tuple[float, float] = (-0.003, 0.0)
    draw_ensemble: Optional[dict] = None  # recipe of a seeded ensemble, see _c4

    @property
    def n_elem(self) -> int:
        return sum(c.n_elem for c in self.coils)

    @property
    def n_wire(self) -> int:
        return sum(c.n_wire for c in self.coils)

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    def pairs_per_pass(self) -> int:
        """Number of ordered (target, source) pairs one all-pairs field pass
        evaluates: sum over coils of N_c (N_c - 1) (coils do not interact)."""
        return sum(c.n_elem * (c.n_elem - 1) for c in self.coils)

    def describe(self) -> dict:
        return {
            "workload": self.name,
            "n_coils": len(self.coils),
            "n_elem": self.n_elem,
            "n_wire": self.n_wire,
            "coils": [f"{c.layers}x{c.turns}x{c.ne}^2" for c in self.coils]
            if len(self.coils) <= 16
            else len(self.coils),
            "dt": self.dt,
            "steps": self.steps,
            "precision": self.precision,
            "seed": self.seed,
        }


def _c1() -> Workload:
    return Workload(
        name="c1_small_fp64",
        coils=[Coil(layers=4, turns=8, ne=4, ramp=1.0)],
        steps=500,
        dt=1.0e-4,
        seed=1,
        jc_disorder=("gauss", 0.01),
    )


def _c2() -> Workload:
    return Workload(
        name="c2_medium_131k",
        coils=[Coil(layers=32, turns=64, ne=8, ramp=2.0)],
        steps=2000,
        dt=5.0e-5,
        seed=2,
        jc_disorder=("lognormal", 0.02),
        weak_spots=5,
        weak_factor=0.7,
    )


def _c3() -> Workload:
    return _c1().replace(name="c3_small_mixed", precision="mixed")


_C4_LAYERS = (8, 16, 24, 32)
_C4_TURNS = (16, 32, 48, 64)


def _c4() -> Workload:
    w = Workload(
        name="c4_ensemble16",
        coils=[],
        steps=1000,
        dt=1.0e-4,
        seed=4,
        jc_disorder=("lognormal", 0.02),
        precision="mixed",
        draw_ensemble={"n": 16, "layers": _C4_LAYERS, "turns": _C4_TURNS,
                       "ne": 6, "ramp": (0.5, 5.0)},
    )
    rng = np.random.Generator(np.random.PCG64(w.seed))
    w.coils = _draw_ensemble(rng, w.draw_ensemble)
    return w


def _c5() -> Workload:
    return Workload(
        name="c5_adjoint_384k",
        coils=[Coil(layers=60, turns=100, ne=8, ramp=1.0)],
        steps=2000,
        dt=5.0e-5,
        seed=5,
        jc_disorder=("lognormal", 0.02),
        precision="mixed",
    )


def _quench20() -> Workload:
    """The paper's quench study (Results, quenches propagation in a coil):
    20 x 20 turns under a 2 A/s transport ramp and a 0.015 T/s background
    ramp, here with 8x8 elements per wire and the normal-state resistivity
    of a copper-stabilised wire."""
    return Workload(
        name="quench20",
        coils=[Coil(layers=20, turns=20, ne=8, ramp=2.0)],
        steps=4000,
        dt=5.0e-5,
        seed=20,
        jc_disorder=("lognormal", 0.02),
        dBa_dt=0.015,
        rho_n=3.0e-10,
        precision="mixed",
    )


def _draw_ensemble(rng: np.random.Generator, rec: dict) -> List[Coil]:
    n = rec["n"]
    layers = rng.choice(np.array(rec["layers"]), n)
    turns = rng.choice(np.array(rec["turns"]), n)
    ramps = rng.uniform(rec["ramp"][0], rec["ramp"][1], n)
    return [Coil(layers=int(layers[i]), turns=int(turns[i]), ne=int(rec["ne"]),
                 ramp=float(ramps[i])) for i in range(n)]


# "Active" variants: same grids, disorder and time step, but a faster
# transport ramp and a smaller Jc0, so that flux penetrates within the run:
# max |J|/Jc crosses 1 after roughly a third of the steps, E reaches Ec, the
# Joule source is non-zero and T rises.  The literal workloads stay deeply
# sub-critical (|J|/Jc ~ 1e-5): there E ~ Ec (|J|/Jc)^30 is ~1e-150 V/m and T
# stays at the bath temperature to the last bit.
# name -> (ramp multiplier, Jc0 in A/m^2); the background field ramp is
# scaled like the transport ramp
ACTIVE = {
    "quench20": (1000.0, 5.0e8),
    "c1": (1000.0, 5.0e8),
    "c3": (1000.0, 5.0e8),
    "c2": (1000.0, 5.0e8),
    "c5": (1000.0, 5.0e8),
    "c4": (200.0, 5.0e8),
}


WORKLOADS = {
    "c1": _c1,
    "c2": _c2,
    "c3": _c3,
    "c4": _c4,
    "c5": _c5,
    "quench20": _quench20,
}


def workload(name: str) -> Workload:
    """Named workload.  ``c1``..``c5`` are the five benchmark configurations;
    ``<name>_active`` is the same shape in the active regime (see ACTIVE)."""
    if name.endswith("_active"):
        base = name[: -len("_active")]
        w = WORKLOADS[base]()
        mult, jc0 = ACTIVE[base]
        coils = [dataclasses.replace(c, ramp=c.ramp * mult) for c in w.coils]
        return w.replace(name=w.name + "_active", Jc0=jc0, coils=coils, dBa_dt=w.dBa_dt * mult)
    return WORKLOADS[name]()


def generate(w: Workload) -> dict:
    """Seeded per-element and per-wire inputs of a workload, public order.

    Draw order from ``numpy.random.Generator(PCG64(seed))``:
    ensemble sizes (if any) first, then the strain eps (N uniform in
    ``eps_range``), then N standard normals g for the Jc0 multiplier
    (``gauss``: mu = max(1 + s g, 0.01); ``lognormal``: mu = exp(s g)),
    then the weak-spot element indices (``choice(N, k, replace=False)``),
    whose multipliers are scaled by ``weak_factor``.

    Returns ``jc0_mult`` (N,), ``strain`` (N,), ``c_wire`` (N_w,), all float64.
    """
    rng = np.random.Generator(np.random.PCG64(w.seed))
    if w.draw_ensemble is not None:
        _draw_ensemble(rng, w.draw_ensemble)  # advance the stream identically
    N = w.n_elem
    eps = rng.uniform(w.eps_range[0], w.eps_range[1], N)
    g = rng.standard_normal(N)
    kind, s = w.jc_disorder
    if kind == "gauss":
        mu = np.maximum(1.0 + s * g, 0.01)
    elif kind == "lognormal":
        mu = np.exp(s * g)
    elif kind == "none":
        mu = np.ones(N)
    else:
        raise ValueError(f"unknown disorder kind {kind!r}")
    if w.weak_spots > 0:
        idx = rng.choice(N, w.weak_spots, replace=False)
        mu[idx] *= w.weak_factor
    return {
        "jc0_mult": np.ascontiguousarray(mu, dtype=np.float64),
        "strain": np.ascontiguousarray(eps, dtype=np.float64),
        "c_wire": np.ones(w.n_wire, dtype=np.float64),
    }


def composite_map(w: Workload, core_k: float = 0.02) -> np.ndarray:
    """Thermal conductivity multipliers of a composite cross-section, public
    order: inside each wire the (ne-2) x (ne-2) core of elements stands for
    the Nb3Sn filament bundle (multiplier ``core_k``), the outer ring of
    elements for the copper sheath (1).  The epoxy between wires is the
    insulation resistance ``ins_R0`` of the workload, not a map entry."""
    out = []
    for c in w.coils:
        ir, iz = np.divmod(np.arange(c.n_elem), c.n_z)
        a, b = ir % c.ne, iz % c.ne
        core = (a > 0) & (a < c.ne - 1) & (b > 0) & (b < c.ne - 1)
        out.append(np.where(core, core_k, 1.0))
    return np.ascontiguousarray(np.concatenate(out), dtype=np.float64)


def composite(w: Workload) -> Workload:
    """The composite thermal model of a workload: ADI heat step, a copper-sheath
    conductivity k0 = 100 W/(m K), k and h proportional to T^3, and 25 um of
    epoxy (about 0.05 W/(m K) at 4.2 K) between wires, R = 5e-4 m^2 K / W."""
    return w.replace(name=w.name + "_composite", heat_solver="adi", k0=100.0, k_exp=3.0, h_exp=3.0, ins_R0=5e-4)


def random_currents(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded element currents (A) for exercising the field sum on its own:
    standard normals times ``scale``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(scale * rng.standard_normal(n), dtype=np.float64)


def fd_wires(n_wire: int = 6000, k: int = 20, seed: int = 55) -> np.ndarray:
    """Seeded wire indices for the finite-difference gradient checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n_wire, k, replace=False))


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """Seeded sorted sample of k distinct indices in [0, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = min(k, n)
    return np.sort(rng.choice(n, k, replace=False))
