"""Plain FP64 CPU oracle of the coil quench hot path (ctypes harness).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_2403_07666_amd``) and never imports it.

The arithmetic lives in ``coil_oracle.c`` (plain C, FP64, compensated sums);
this module only marshals arguments.  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "coil_oracle.c")
_LIB = os.path.join(_HERE, "libcoil_oracle.so")
MAXC = 64

# field ids (coil_oracle.h)
I, J, BR, BZ, T, PHI, QW, UW, E, EP, U, Q, PSI, R, Z, V, JC, DI = range(18)
# per-wire flux-jump / quench diagnostics
ONSET, QUENCH, Q_ONSET, Q_QUENCH, T_QUENCH, P_QUENCH = range(18, 24)
KMULT = 24  # per-element conductivity multiplier of the ADI heat step
IH = 25  # field-driven component of the element current (subelement model)
EMSUB = 26  # per wire: EM substeps of the last step (variable-step integration)
PER_WIRE = (QW, UW, ONSET, QUENCH, Q_ONSET, Q_QUENCH, T_QUENCH, P_QUENCH, EMSUB)


def build(force: bool = True) -> str:
    """Compile the oracle shared library in-tree with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c99", "-D_DEFAULT_SOURCE", "-O2", "-fopenmp", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class Cfg(C.Structure):
    _fields_ = [
        ("n_coils", C.c_int),
        ("layers", C.c_int * MAXC), ("turns", C.c_int * MAXC), ("ne", C.c_int * MAXC),
        ("r_inner", C.c_double * MAXC), ("z_center", C.c_double * MAXC),
        ("wire_side", C.c_double * MAXC),
        ("ramp", C.c_double * MAXC), ("I0", C.c_double * MAXC),
        ("dBa_dt", C.c_double),
        ("Ec", C.c_double), ("n", C.c_double), ("Jc0", C.c_double), ("Tc", C.c_double),
        ("B0", C.c_double), ("eps_coef", C.c_double), ("eps_pow", C.c_double),
        ("C0", C.c_double), ("T_ref", C.c_double), ("cp_exp", C.c_double),
        ("k0", C.c_double), ("h0", C.c_double), ("T_bath", C.c_double),
        ("dt", C.c_double),
        ("n_sub", C.c_int), ("planar", C.c_int),
        ("rho_n", C.c_double),
        ("coupling", C.c_int),
        ("heat_solver", C.c_int),
        ("k_exp", C.c_double), ("h_exp", C.c_double), ("ins_R0", C.c_double),
        ("subelements", C.c_int),
        ("em_tol", C.c_double), ("em_max_level", C.c_int),
    ]


_lib = None
_dp = C.POINTER(C.c_double)
_lp = C.POINTER(C.c_long)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        L.orc_ellip.argtypes = [C.c_double, _dp, _dp]
        L.orc_carlson_rf.argtypes = [C.c_double] * 3
        L.orc_carlson_rf.restype = C.c_double
        L.orc_carlson_rd.argtypes = [C.c_double] * 3
        L.orc_carlson_rd.restype = C.c_double
        L.orc_ring_B.argtypes = [C.c_double] * 5 + [_dp, _dp]
        L.orc_ring_M.argtypes = [C.c_double] * 4
        L.orc_ring_M.restype = C.c_double
        L.orc_self_L.argtypes = [C.c_double] * 2
        L.orc_self_L.restype = C.c_double
        L.orc_threads.restype = C.c_int
        L.orc_create.argtypes = [C.POINTER(Cfg), _dp, _dp, _dp]
        L.orc_create.restype = C.c_void_p
        L.orc_create_ex.argtypes = [C.POINTER(Cfg), _dp, _dp, _dp, C.c_int]
        L.orc_create_ex.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_n_elem.argtypes = [C.c_void_p]
        L.orc_n_elem.restype = C.c_long
        L.orc_n_wire.argtypes = [C.c_void_p]
        L.orc_n_wire.restype = C.c_long
        L.orc_n_sub.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p]
        L.orc_run.argtypes = [C.c_void_p, C.c_long]
        L.orc_get.argtypes = [C.c_void_p, C.c_int, _dp, C.c_long]
        L.orc_set.argtypes = [C.c_void_p, C.c_int, _dp, C.c_long]
        L.orc_scalars.argtypes = [C.c_void_p, _dp, C.c_int]
        L.orc_field_targets.argtypes = [C.c_void_p, _dp, C.c_long, _lp, _dp, _dp]
        L.orc_field_points.argtypes = [C.c_void_p, _dp, C.c_long, _dp, _dp, _dp, _dp]
        L.orc_wire_elems.argtypes = [C.c_void_p, C.c_long, _lp]
        if hasattr(L, "orc_tangent"):
            L.orc_tangent.argtypes = [C.POINTER(Cfg), _dp, _dp, _dp, _dp, _dp, C.c_long,
                                      _dp, _dp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- pure functions
def ellip(m1: float):
    """(K(m), E(m)) with the complementary parameter m1 = 1 - m."""
    k, e = C.c_double(), C.c_double()
    lib().orc_ellip(float(m1), C.byref(k), C.byref(e))
    return k.value, e.value


def carlson_rf(x, y, z):
    return lib().orc_carlson_rf(float(x), float(y), float(z))


def carlson_rd(x, y, z):
    return lib().orc_carlson_rd(float(x), float(y), float(z))


def ring_B(a, zs, r, z, I=1.0):
    br, bz = C.c_double(), C.c_double()
    lib().orc_ring_B(float(a), float(zs), float(r), float(z), float(I), C.byref(br), C.byref(bz))
    return br.value, bz.value


def ring_M(a, zs, r, z):
    return lib().orc_ring_M(float(a), float(zs), float(r), float(z))


def self_L(r, d):
    return lib().orc_self_L(float(r), float(d))


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(lib().orc_threads())


# ---------------------------------------------------------------- simulation
def make_cfg(w, n_sub: int | None = None, planar: bool = False) -> Cfg:
    """Oracle configuration from a ``coil_synth.Workload``."""
    c = Cfg()
    if len(w.coils) > MAXC:
        raise ValueError("too many coils for the oracle")
    c.n_coils = len(w.coils)
    for i, co in enumerate(w.coils):
        c.layers[i], c.turns[i], c.ne[i] = co.layers, co.turns, co.ne
        c.r_inner[i], c.z_center[i], c.wire_side[i] = co.r_inner, co.z_center, co.wire_side
        c.ramp[i], c.I0[i] = co.ramp, co.I0
    for k in ("dBa_dt", "Ec", "n", "Jc0", "Tc", "B0", "eps_coef", "eps_pow", "C0", "T_ref",
              "cp_exp", "k0", "h0", "T_bath", "dt"):
        setattr(c, k, float(getattr(w, k)))
    c.n_sub = int(w.heat_substeps if n_sub is None else n_sub)
    c.planar = 1 if planar else 0
    c.rho_n = float(getattr(w, "rho_n", 0.0))
    c.coupling = {"transport": 0, "full": 1}[getattr(w, "coupling", "transport")]
    c.heat_solver = {"explicit": 0, "adi": 1}[getattr(w, "heat_solver", "explicit")]
    c.k_exp = float(getattr(w, "k_exp", 0.0))
    c.h_exp = float(getattr(w, "h_exp", 0.0))
    c.ins_R0 = float(getattr(w, "ins_R0", 0.0))
    c.subelements = int(getattr(w, "subelements", 0))
    c.em_tol = float(getattr(w, "em_tol", 0.0))
    c.em_max_level = int(getattr(w, "em_max_level", 0))
    return c


class Sim:
    """One oracle simulation (public element order)."""

    def __init__(self, w, inputs: dict | None = None, n_sub: int | None = None,
                 planar: bool = False, field_only: bool = False):
        self.w = w
        self.cfg = make_cfg(w, n_sub=n_sub, planar=planar)
        L = lib()
        if inputs is None:
            inputs = {}
        self._keep = [_f64(inputs[k]) if k in inputs else None
                      for k in ("jc0_mult", "strain", "c_wire")]
        ptrs = [(_p(a) if a is not None else None) for a in self._keep]
        self.h = L.orc_create_ex(C.byref(self.cfg), *ptrs, 1 if field_only else 0)
        if not self.h:
            raise ValueError("oracle rejected the configuration")
        self.N = L.orc_n_elem(self.h)
        self.Nw = L.orc_n_wire(self.h)
        self.n_sub = L.orc_n_sub(self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def step(self) -> int:
        return lib().orc_step(self.h)

    def run(self, n: int) -> int:
        return lib().orc_run(self.h, int(n))

    def get(self, field: int) -> np.ndarray:
        n = self.Nw if field in PER_WIRE else self.N
        out = np.empty(n, dtype=np.float64)
        rc = lib().orc_get(self.h, field, _p(out), n)
        if rc:
            raise ValueError(f"bad field {field}")
        return out

    def set(self, field: int, values) -> None:
        v = _f64(values)
        if lib().orc_set(self.h, field, _p(v), v.size):
            raise ValueError(f"cannot set field {field}")

    def scalars(self) -> dict:
        v = np.empty(12, dtype=np.float64)
        lib().orc_scalars(self.h, _p(v), 12)
        keys = ["t", "step", "Q", "T_peak", "sumU", "max_x", "Q_out", "stored", "I_t",
                "T_peak_elem", "T_peak_step", "n_sub"]
        return dict(zip(keys, v.tolist()))

    def field_targets(self, I, targets):
        I = _f64(I)
        t = np.ascontiguousarray(targets, dtype=np.int64)
        br = np.empty(t.size)
        bz = np.empty(t.size)
        lib().orc_field_targets(self.h, _p(I), t.size, t.ctypes.data_as(_lp), _p(br), _p(bz))
        return br, bz

    def field_points(self, I, r, z):
        I, r, z = _f64(I), _f64(r), _f64(z)
        br = np.empty(r.size)
        bz = np.empty(r.size)
        lib().orc_field_points(self.h, _p(I), r.size, _p(r), _p(z), _p(br), _p(bz))
        return br, bz

    def wire_elems(self, w: int) -> np.ndarray:
        out = np.empty(4096, dtype=np.int64)
        n = lib().orc_wire_elems(self.h, int(w), out.ctypes.data_as(_lp))
        return out[:n].copy()


def tangent(w, inputs: dict, dc_wire=None, dramp=None, nsteps: int | None = None):
    """Forward-mode directional derivatives of (Q, T_peak) after nsteps along
    (dc_wire, dramp).  Returns (obj, dobj) as two 2-tuples."""
    cfg = make_cfg(w)
    keep = [_f64(inputs[k]) if inputs.get(k) is not None else None
            for k in ("jc0_mult", "strain", "c_wire")]
    ptr = [(_p(a) if a is not None else None) for a in keep]
    dcw = _f64(dc_wire) if dc_wire is not None else None
    drp = _f64(dramp) if dramp is not None else None
    obj = np.zeros(2)
    dobj = np.zeros(2)
    rc = lib().orc_tangent(C.byref(cfg), *ptr, _p(dcw) if dcw is not None else None,
                           _p(drp) if drp is not None else None, int(nsteps or w.steps),
                           _p(obj), _p(dobj))
    if rc:
        raise RuntimeError(f"oracle tangent failed ({rc})")
    return tuple(obj), tuple(dobj)
