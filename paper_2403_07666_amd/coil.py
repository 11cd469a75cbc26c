"""Thin ctypes binding over libcoil.so (include/coil.h).

Argument marshalling only: every step of the time step runs in the HIP
kernels of the library.  PyTorch provides the device workspace and the stream.
The binding never falls back to a CPU path: without the built library, or
without a GPU, constructing a ``Coil`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Callable, Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcoil.so")

# enum coil_status / coil_precision / coil_field (include/coil.h)
OK, E_INVAL, E_NOMEM, E_HIP, E_NONFINITE, E_STATE = 0, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
ALGO_AUTO, ALGO_DIRECT, ALGO_TRANSLATION, ALGO_FFT = 0, 1, 2, 3
F_I, F_J, F_BR, F_BZ, F_T, F_PHI, F_QW, F_UW, F_E, F_EP, F_U, F_Q, F_PSI, F_R, F_Z, F_DI, F_JC = range(17)
F_ONSET, F_QUENCH, F_Q_ONSET, F_Q_QUENCH, F_T_QUENCH, F_P_QUENCH = range(17, 23)
F_IH = 23  # subelement model: field-driven component of the element current
F_EM_SUBSTEPS = 24  # variable step: substeps per wire in the last step
PER_WIRE = (F_QW, F_UW, F_ONSET, F_QUENCH, F_Q_ONSET, F_Q_QUENCH, F_T_QUENCH, F_P_QUENCH, F_EM_SUBSTEPS)
AXISYMMETRIC, PLANAR = 0, 1
COUPLE_TRANSPORT, COUPLE_FULL = 0, 1
HEAT_EXPLICIT, HEAT_ADI = 0, 1

_i32p = C.POINTER(C.c_int32)
_dp = C.POINTER(C.c_double)


class CoilError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"coil error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("n_coils", C.c_int32),
        ("layers", _i32p), ("turns", _i32p), ("ne", _i32p),
        ("r_inner", _dp), ("z_center", _dp), ("wire_side", _dp), ("ramp", _dp),
        ("dBa_dt", C.c_double),
        ("Ec", C.c_double), ("n", C.c_double), ("Jc0", C.c_double), ("Tc", C.c_double),
        ("B0", C.c_double), ("eps_coef", C.c_double), ("eps_pow", C.c_double),
        ("C0", C.c_double), ("T_ref", C.c_double), ("cp_exp", C.c_double), ("k0", C.c_double),
        ("h0", C.c_double), ("T_bath", C.c_double),
        ("dt", C.c_double),
        ("heat_substeps", C.c_int32), ("precision", C.c_int32),
        ("near_k", C.c_double),
        ("tile_targets", C.c_int32), ("tile_sources", C.c_int32), ("grid_limit", C.c_int32),
        ("algo", C.c_int32),
        ("I0", _dp), ("rho_n", C.c_double), ("k_exp", C.c_double), ("h_exp", C.c_double),
        ("ins_R0", C.c_double),
        ("geometry", C.c_int32), ("coupling", C.c_int32), ("heat_solver", C.c_int32),
        ("cg_max_iter", C.c_int32), ("cg_tol", C.c_double),
        ("subelements", C.c_int32),
        ("em_tol", C.c_double), ("em_max_level", C.c_int32),
    ]


class Inputs(C.Structure):
    _fields_ = [("jc0_mult", _dp), ("strain", _dp), ("c_wire", _dp), ("k_mult", _dp)]


class Sizes(C.Structure):
    _fields_ = [("workspace_bytes", C.c_size_t), ("n_elem", C.c_int64), ("n_wire", C.c_int64),
                ("heat_substeps", C.c_int32), ("n_work_items", C.c_int32)]


REPORT_FN = C.CFUNCTYPE(None, _dp, C.c_int32, C.c_void_p)

EXPORTS = [
    "coil_query", "coil_init", "coil_step", "coil_run", "coil_compute_field", "coil_get",
    "coil_set_state", "coil_scalars", "coil_reset", "coil_timing", "coil_timing_read",
    "coil_graph", "coil_destroy", "coil_last_error", "coil_host_ellip", "coil_set_params",
    "coil_adjoint_query", "coil_adjoint", "coil_field_transpose", "coil_set_tiles", "coil_autotune",
    "coil_field_stats", "coil_field_at", "coil_save", "coil_load", "coil_set_widths",
    "coil_field_at_noalloc",
]
FIELD_AT_SCRATCH_BYTES = 8 << 20  # COIL_FIELD_AT_SCRATCH_BYTES

_lib = None


def lib():
    """Load libcoil.so (built in-tree by build.py); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2403_07666_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.coil_query.argtypes = [C.POINTER(Config), C.POINTER(Sizes)]
        L.coil_init.argtypes = [C.POINTER(Config), C.POINTER(Inputs), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.coil_step.argtypes = [vp]
        L.coil_run.argtypes = [vp, C.c_int64, C.c_int64, REPORT_FN, vp]
        L.coil_compute_field.argtypes = [vp]
        L.coil_get.argtypes = [vp, C.c_int32, vp, C.c_int64, C.c_int32]
        L.coil_set_state.argtypes = [vp, C.c_int32, vp, C.c_int64, C.c_int32]
        L.coil_scalars.argtypes = [vp, _dp, C.c_int32]
        L.coil_reset.argtypes = [vp]
        L.coil_timing.argtypes = [vp, C.c_int32]
        L.coil_timing_read.argtypes = [vp, _dp, C.POINTER(C.c_int64), C.c_int32]
        L.coil_graph.argtypes = [vp, C.c_int64]
        L.coil_destroy.argtypes = [vp]
        L.coil_destroy.restype = None
        L.coil_last_error.restype = C.c_char_p
        L.coil_host_ellip.argtypes = [C.c_double, C.c_int32, _dp, _dp]
        L.coil_set_params.argtypes = [vp, _dp, _dp]
        L.coil_adjoint_query.argtypes = [vp, C.c_int64, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
        L.coil_adjoint.argtypes = [vp, C.c_int64, C.c_double, C.c_double, C.c_int32, C.c_int32, vp,
                                   C.c_size_t, _dp, _dp, _dp]
        L.coil_field_transpose.argtypes = [vp, vp, vp, vp, C.c_int32]
        L.coil_set_tiles.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
        L.coil_set_widths.argtypes = [vp, C.c_int32]
        L.coil_autotune.argtypes = [vp, C.c_int32, C.c_char_p, _i32p]
        L.coil_field_stats.argtypes = [vp, _dp, C.c_int32]
        L.coil_field_at.argtypes = [vp, C.c_int64, _dp, _dp, _dp, _dp]
        L.coil_field_at_noalloc.argtypes = [vp, C.c_int64, vp, vp, vp, vp]
        L.coil_save.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
        L.coil_load.argtypes = [vp, vp, C.c_size_t]
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != OK:
        raise CoilError(rc, lib().coil_last_error().decode())


def host_ellip(m1: float, precision: int = FP64):
    """The library's K(m), E(m) approximations evaluated on the host (m1 = 1 - m)."""
    k, e = C.c_double(), C.c_double()
    check(lib().coil_host_ellip(float(m1), int(precision), C.byref(k), C.byref(e)))
    return k.value, e.value


def _prec_id(p) -> int:
    if p in (FP64, "fp64", "f64"):
        return FP64
    if p in (MIXED, "mixed"):
        return MIXED
    if isinstance(p, int):
        return p  # validated by the library
    raise ValueError(f"unknown precision {p!r}")


class _CfgHolder:
    """Keeps the per-coil arrays of a Config alive."""

    def __init__(self, w, precision=None, tile_targets=0, tile_sources=0, grid_limit=0,
                 near_k=0.0, heat_substeps=None, algo=ALGO_AUTO, geometry=None, coupling=None,
                 heat_solver=None, cg_max_iter=0, cg_tol=0.0):
        co = w.coils
        self.arr = {
            "layers": np.array([c.layers for c in co], dtype=np.int32),
            "turns": np.array([c.turns for c in co], dtype=np.int32),
            "ne": np.array([c.ne for c in co], dtype=np.int32),
            "r_inner": np.array([c.r_inner for c in co], dtype=np.float64),
            "z_center": np.array([c.z_center for c in co], dtype=np.float64),
            "wire_side": np.array([c.wire_side for c in co], dtype=np.float64),
            "ramp": np.array([c.ramp for c in co], dtype=np.float64),
            "I0": np.array([c.I0 for c in co], dtype=np.float64),
        }
        cfg = Config()
        cfg.n_coils = len(co)
        for k in ("layers", "turns", "ne"):
            setattr(cfg, k, self.arr[k].ctypes.data_as(_i32p))
        for k in ("r_inner", "z_center", "wire_side", "ramp", "I0"):
            setattr(cfg, k, self.arr[k].ctypes.data_as(_dp))
        for k in ("dBa_dt", "Ec", "n", "Jc0", "Tc", "B0", "eps_coef", "eps_pow", "C0", "T_ref",
                  "cp_exp", "k0", "h0", "T_bath", "dt"):
            setattr(cfg, k, float(getattr(w, k)))
        cfg.heat_substeps = int(w.heat_substeps if heat_substeps is None else heat_substeps)
        cfg.precision = _prec_id(w.precision if precision is None else precision)
        cfg.near_k = float(near_k)
        cfg.tile_targets = int(tile_targets)
        cfg.tile_sources = int(tile_sources)
        cfg.grid_limit = int(grid_limit)
        cfg.algo = {"auto": ALGO_AUTO, "direct": ALGO_DIRECT, "translation": ALGO_TRANSLATION,
                    "fft": ALGO_FFT}.get(algo, algo)
        cfg.rho_n = float(getattr(w, "rho_n", 0.0))
        cfg.k_exp = float(getattr(w, "k_exp", 0.0))
        cfg.h_exp = float(getattr(w, "h_exp", 0.0))
        geo = getattr(w, "geometry", "axisymmetric") if geometry is None else geometry
        cfg.geometry = {"axisymmetric": AXISYMMETRIC, "planar": PLANAR}.get(geo, geo)
        cpl = getattr(w, "coupling", "transport") if coupling is None else coupling
        cfg.coupling = {"transport": COUPLE_TRANSPORT, "full": COUPLE_FULL}.get(cpl, cpl)
        hs = getattr(w, "heat_solver", "explicit") if heat_solver is None else heat_solver
        cfg.heat_solver = {"explicit": HEAT_EXPLICIT, "adi": HEAT_ADI}.get(hs, hs)
        cfg.cg_max_iter = int(cg_max_iter)
        cfg.cg_tol = float(cg_tol)
        cfg.ins_R0 = float(getattr(w, "ins_R0", 0.0))
        cfg.subelements = int(getattr(w, "subelements", 0))
        cfg.em_tol = float(getattr(w, "em_tol", 0.0))
        cfg.em_max_level = int(getattr(w, "em_max_level", 0))
        self.cfg = cfg


def query(w, **kw) -> Sizes:
    h = _CfgHolder(w, **kw)
    s = Sizes()
    check(lib().coil_query(C.byref(h.cfg), C.byref(s)))
    return s


class Coil:
    """One handle of the HIP library on a CUDA/HIP device, with a torch-owned
    workspace and a dedicated (default-priority) torch stream."""

    def __init__(self, w, inputs: Optional[dict] = None, device: str = "cuda:0", **kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the coil library needs a GPU; none is visible")
        L = lib()
        self.w = w
        self.device = torch.device(device)
        self._cfg = _CfgHolder(w, **kw)
        sizes = Sizes()
        check(L.coil_query(C.byref(self._cfg.cfg), C.byref(sizes)))
        self.sizes = sizes
        self.N = int(sizes.n_elem)
        self.Nw = int(sizes.n_wire)
        self.n_sub = int(sizes.heat_substeps)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(device=self.device)
            self.ws = torch.empty(int(sizes.workspace_bytes), dtype=torch.uint8, device=self.device)
            torch.cuda.synchronize(self.device)
        if self.ws.data_ptr() % 256 != 0:
            raise RuntimeError("workspace is not 256-byte aligned")
        inputs = inputs or {}
        self._in_arrays = {k: np.ascontiguousarray(inputs[k], dtype=np.float64)
                           for k in ("jc0_mult", "strain", "c_wire", "k_mult") if inputs.get(k) is not None}
        if "k_mult" in self._in_arrays and self._in_arrays["k_mult"].size != self.N:
            raise ValueError("k_mult has the wrong length")
        if "jc0_mult" in self._in_arrays and self._in_arrays["jc0_mult"].size != self.N:
            raise ValueError("jc0_mult has the wrong length")
        if "strain" in self._in_arrays and self._in_arrays["strain"].size != self.N:
            raise ValueError("strain has the wrong length")
        if "c_wire" in self._in_arrays and self._in_arrays["c_wire"].size != self.Nw:
            raise ValueError("c_wire has the wrong length")
        inp = Inputs()
        for k, a in self._in_arrays.items():
            setattr(inp, k, a.ctypes.data_as(_dp))
        h = C.c_void_p()
        check(L.coil_init(C.byref(self._cfg.cfg), C.byref(inp), C.c_void_p(self.ws.data_ptr()),
                          C.c_size_t(self.ws.numel()), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    # -------------------------------------------------------------- lifetime
    def close(self) -> None:
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().coil_destroy(h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- stepping
    def step(self) -> None:
        check(lib().coil_step(self.h))

    def run(self, nsteps: int, report_every: int = 0,
            cb: Optional[Callable[[np.ndarray], None]] = None) -> None:
        if cb is not None and report_every > 0:
            def _tramp(diag, nd, _user):
                cb(np.ctypeslib.as_array(diag, shape=(nd,)).copy())
            fn = REPORT_FN(_tramp)
        else:
            fn = REPORT_FN()
            report_every = 0
        check(lib().coil_run(self.h, int(nsteps), int(report_every), fn, None))

    def compute_field(self) -> None:
        check(lib().coil_compute_field(self.h))

    def reset(self) -> None:
        check(lib().coil_reset(self.h))

    def graph(self, steps: int) -> None:
        check(lib().coil_graph(self.h, int(steps)))

    def synchronize(self) -> None:
        self.stream.synchronize()

    # -------------------------------------------------------------- state
    def get(self, field: int) -> np.ndarray:
        n = self.Nw if field in PER_WIRE else self.N
        out = np.empty(n, dtype=np.float64)
        check(lib().coil_get(self.h, int(field), out.ctypes.data_as(C.c_void_p), n, 0))
        return out

    def get_device(self, field: int):
        import torch
        n = self.Nw if field in PER_WIRE else self.N
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        check(lib().coil_get(self.h, int(field), C.c_void_p(out.data_ptr()), n, 1))
        self.stream.synchronize()
        return out

    def set_state(self, field: int, values) -> None:
        v = np.ascontiguousarray(values, dtype=np.float64)
        check(lib().coil_set_state(self.h, int(field), v.ctypes.data_as(C.c_void_p), v.size, 0))

    def scalars(self) -> dict:
        v = np.empty(15, dtype=np.float64)
        check(lib().coil_scalars(self.h, v.ctypes.data_as(_dp), 15))
        keys = ["t", "step", "Q", "T_peak", "sumU", "max_x", "Q_out", "stored", "status",
                "T_peak_elem", "T_peak_step", "n_sub", "n_work_items", "cg_iters", "cg_residual"]
        return dict(zip(keys, v.tolist()))

    # -------------------------------------------------------------- timing
    def timing(self, enable) -> None:
        """True / 1: time every phase; 2: only the field kernel; False / 0: stop."""
        mode = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
        check(lib().coil_timing(self.h, mode))

    def timing_read(self) -> dict:
        ms = np.zeros(4, dtype=np.float64)
        n = np.zeros(4, dtype=np.int64)
        check(lib().coil_timing_read(self.h, ms.ctypes.data_as(_dp),
                                     n.ctypes.data_as(C.POINTER(C.c_int64)), 4))
        names = ["field", "wire", "heat", "reduce"]
        return {nm: {"ms": float(ms[i]), "launches": int(n[i])} for i, nm in enumerate(names)}

    # -------------------------------------------------------------- parameters and adjoint
    def set_params(self, c_wire=None, ramp=None) -> None:
        cw = np.ascontiguousarray(c_wire, dtype=np.float64) if c_wire is not None else None
        rp = np.ascontiguousarray(ramp, dtype=np.float64) if ramp is not None else None
        if cw is not None and cw.size != self.Nw:
            raise ValueError("c_wire has the wrong length")
        if rp is not None and rp.size != len(self.w.coils):
            raise ValueError("ramp needs one value per coil")
        check(lib().coil_set_params(self.h, cw.ctypes.data_as(_dp) if cw is not None else None,
                                    rp.ctypes.data_as(_dp) if rp is not None else None))

    def field_transpose(self, bbar_r, bbar_z) -> np.ndarray:
        br = np.ascontiguousarray(bbar_r, dtype=np.float64)
        bz = np.ascontiguousarray(bbar_z, dtype=np.float64)
        out = np.empty(self.N, dtype=np.float64)
        check(lib().coil_field_transpose(self.h, br.ctypes.data_as(C.c_void_p), bz.ctypes.data_as(C.c_void_p),
                                         out.ctypes.data_as(C.c_void_p), 0))
        return out

    def adjoint_bytes(self, nsteps: int, ckpt_every: int = 50, store_field: bool = True) -> int:
        b = C.c_size_t()
        check(lib().coil_adjoint_query(self.h, int(nsteps), int(ckpt_every), 1 if store_field else 0, C.byref(b)))
        return int(b.value)

    def adjoint(self, nsteps: int, wQ: float = 1.0, wT: float = 0.0, ckpt_every: int = 50,
                store_field: bool = True):
        """Gradients of wQ Q + wT T_peak after nsteps with respect to the per-wire
        Jc multipliers and the per-coil ramp rates.  Returns (g_c_wire, g_ramp,
        (Q, T_peak)); leaves the handle reset to t = 0."""
        import torch
        nb = self.adjoint_bytes(nsteps, ckpt_every, store_field)
        with torch.cuda.device(self.device):
            ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
            torch.cuda.synchronize(self.device)
        gcw = np.zeros(self.Nw)
        gr = np.zeros(len(self.w.coils))
        obj = np.zeros(2)
        check(lib().coil_adjoint(self.h, int(nsteps), float(wQ), float(wT), int(ckpt_every),
                                 1 if store_field else 0, C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()),
                                 gcw.ctypes.data_as(_dp), gr.ctypes.data_as(_dp), obj.ctypes.data_as(_dp)))
        del ws
        return gcw, gr, (float(obj[0]), float(obj[1]))

    def objectives(self, nsteps: int):
        """Reset, run nsteps and return (Q, T_peak)."""
        self.reset()
        self.run(nsteps)
        sc = self.scalars()
        return sc["Q"], sc["T_peak"]

    # -------------------------------------------------------------- tiling
    def set_tiles(self, tile_targets: int, chunks: int = 0, grid_limit: int = 0) -> None:
        check(lib().coil_set_tiles(self.h, int(tile_targets), int(chunks), int(grid_limit)))

    def set_widths(self, w: int) -> None:
        """Segment width of the translation pass: 0 = automatic, 2..8 = 64 w targets everywhere."""
        check(lib().coil_set_widths(self.h, int(w)))

    def autotune(self, reps: int = 3, cache_path: Optional[str] = None):
        """Time the field-pass candidates and keep the fastest; returns
        (algo, p1, p2, p3): (2, source-row groups, 0, 0) for the translation
        evaluation, (1, tile_targets, chunks, grid_limit) for the direct one or
        (3, 0, 0, 0) for the fast convolution (a candidate only if set up at init)."""
        ch = np.zeros(4, dtype=np.int32)
        path = cache_path.encode() if cache_path else None
        check(lib().coil_autotune(self.h, int(reps), path, ch.ctypes.data_as(_i32p)))
        return tuple(int(v) for v in ch)

    def field_stats(self) -> dict:
        """Work of one field pass: pairs, Green's-function evaluations, algorithm, items."""
        v = np.zeros(6)
        check(lib().coil_field_stats(self.h, v.ctypes.data_as(_dp), 6))
        return {"pairs": v[0], "kernel_evals": v[1], "algo": {2: "translation", 3: "fft"}.get(int(v[2]), "direct"),
                "items": int(v[3]), "tile_targets": int(v[4]), "workgroups": int(v[5])}

    # -------------------------------------------------------------- probes and snapshots
    def field_at(self, r, z):
        """B_r, B_z (T) at points (r, z) in metres from the current currents."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        br = np.empty(r.size)
        bz = np.empty(r.size)
        check(lib().coil_field_at(self.h, r.size, r.ctypes.data_as(_dp), z.ctypes.data_as(_dp),
                                  br.ctypes.data_as(_dp), bz.ctypes.data_as(_dp)))
        return br, bz

    def field_at_noalloc(self, r, z, Br, Bz) -> None:
        """coil_field_at_noalloc: r, z, Br, Bz are float64 device tensors of one
        length; asynchronous on the handle's stream (synchronize() to wait)."""
        n = int(r.numel())
        for t in (r, z, Br, Bz):
            if t.numel() != n or not t.is_cuda or t.dtype.itemsize != 8 or not t.is_contiguous():
                raise ValueError("r, z, Br, Bz must be contiguous float64 device tensors of one length")
        check(lib().coil_field_at_noalloc(self.h, n, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()),
                                          C.c_void_p(Br.data_ptr()), C.c_void_p(Bz.data_ptr())))

    def save(self) -> bytes:
        need = C.c_size_t()
        check(lib().coil_save(self.h, None, 0, C.byref(need)))
        buf = (C.c_char * need.value)()
        check(lib().coil_save(self.h, C.cast(buf, C.c_void_p), need.value, None))
        return bytes(buf)

    def load(self, snap: bytes) -> None:
        buf = (C.c_char * len(snap)).from_buffer_copy(snap)
        check(lib().coil_load(self.h, C.cast(buf, C.c_void_p), len(snap)))
