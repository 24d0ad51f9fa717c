"""ctypes binding of the C ABI in ``include/tdi.h`` (argument marshalling only).

The entry points keep the C names (``tdi_plan_create``, ``tdi_run``, ...); every
step of the response runs in the HIP kernels of ``libtdi.so``.  PyTorch is used
only for device memory and streams.  If the library is missing the import
fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdi.so")

TDI_OK, TDI_EINVAL, TDI_ERANGE, TDI_ENOMEM, TDI_EDEVICE, TDI_EUNSUPPORTED, TDI_ESTATE = 0, -1, -2, -3, -4, -5, -6
TDI_ORBIT_FROZEN, TDI_ORBIT_ANALYTIC1, TDI_ORBIT_TABLE = 0, 1, 2
TDI_MODE_FULL, TDI_MODE_LFA, TDI_MODE_HYBRID = 0, 1, 2
TDI_FP64, TDI_FP32_BULK = 0, 1
TDI_CHANNELS_XYZ, TDI_CHANNELS_AET = 0, 1

EXPORTED = ["tdi_check_config", "tdi_check_batch", "tdi_plan_create", "tdi_run", "tdi_run_noalloc",
            "tdi_run_links",
            "tdi_plan_sync",
            "tdi_plan_kernel_times", "tdi_plan_set_timing", "tdi_plan_describe", "tdi_plan_destroy",
            "tdi_status_str",
            "tdi_check_noise", "tdi_ip_plan_create", "tdi_ip_run", "tdi_ip_kernel_times",
            "tdi_ip_plan_destroy"]


class TdiError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {tdi_status_str(status)} ({status})")
        self.status = status


class tdi_orbit(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("L_m", C.c_double),
                ("R_m", C.c_double), ("omega", C.c_double), ("kappa0", C.c_double),
                ("lambda0", C.c_double), ("t_freeze", C.c_double),
                ("table", C.POINTER(C.c_double)), ("n_table", C.c_int64),
                ("table_t0", C.c_double), ("table_dt", C.c_double)]


class tdi_source(C.Structure):
    _fields_ = [("beta", C.c_double), ("lambda_", C.c_double), ("psi", C.c_double),
                ("t0", C.c_double), ("dt", C.c_double), ("t_hyb", C.c_double)]


class tdi_config(C.Structure):
    _fields_ = [("tdi_gen", C.c_int32), ("mode", C.c_int32), ("interp_taps", C.c_int32),
                ("stencil_order", C.c_int32), ("lfa_equal_arms", C.c_int32),
                ("precision", C.c_int32), ("hyb_T_samples", C.c_double),
                ("hyb_sigma_samples", C.c_double), ("autotune", C.c_int32),
                ("use_graph", C.c_int32), ("channels", C.c_int32), ("lfa_terms", C.c_int32),
                ("nested_delays", C.c_int32), ("fast_tile_chunks", C.c_int32),
                ("lfa_x20_from_x15", C.c_int32)]


class tdi_noise(C.Structure):
    _fields_ = [("tdi_gen", C.c_int32), ("galactic", C.c_int32), ("T_obs_years", C.c_double),
                ("L_m", C.c_double), ("f_min", C.c_double), ("f_max", C.c_double)]


_lib = None


def lib():
    """Load libtdi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2505_09600_amd/build_lib.py")
        # torch ships its own HIP runtime: load it first so that the library binds
        # to the same runtime as the tensors and streams it is given
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.tdi_check_config.argtypes = [C.POINTER(tdi_config), C.POINTER(tdi_orbit)]
        L.tdi_check_batch.argtypes = [C.POINTER(tdi_config), C.c_int64, C.POINTER(tdi_source),
                                      C.POINTER(C.c_int64)]
        L.tdi_plan_create.argtypes = [C.POINTER(P), C.POINTER(tdi_config), C.POINTER(tdi_orbit),
                                      C.c_int64, C.c_int64, P]
        L.tdi_run.argtypes = [P, C.c_int64, C.POINTER(tdi_source), C.POINTER(C.c_int64),
                              P, P, P, P, P]
        L.tdi_run_noalloc.argtypes = [C.POINTER(tdi_config), C.POINTER(tdi_orbit), C.c_int64,
                                      C.POINTER(tdi_source), C.POINTER(C.c_int64), P, P, P, P, P, P]
        L.tdi_run_links.argtypes = [P, C.c_int64, C.POINTER(tdi_source), C.POINTER(C.c_int64), P, P, P]
        L.tdi_plan_sync.argtypes = [P]
        L.tdi_plan_kernel_times.argtypes = [P, C.POINTER(C.c_float), C.c_int32, C.POINTER(C.c_int32)]
        L.tdi_plan_describe.argtypes = [P, C.c_char_p, C.c_int32]
        L.tdi_plan_set_timing.argtypes = [P, C.c_int32]
        L.tdi_plan_destroy.argtypes = [P]
        L.tdi_check_noise.argtypes = [C.POINTER(tdi_noise)]
        L.tdi_ip_plan_create.argtypes = [C.POINTER(P), C.POINTER(tdi_noise), C.c_int32, C.c_double,
                                         C.c_int64, C.c_int64, C.c_int64, P]
        L.tdi_ip_run.argtypes = [P, C.c_int64, C.POINTER(C.c_int64), C.POINTER(P), C.POINTER(P), P]
        L.tdi_ip_kernel_times.argtypes = [P, C.POINTER(C.c_float), C.c_int32, C.POINTER(C.c_int32)]
        L.tdi_ip_plan_destroy.argtypes = [P]
        L.tdi_status_str.argtypes = [C.c_int]
        L.tdi_status_str.restype = C.c_char_p
        for name in EXPORTED:
            if name != "tdi_status_str":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


# --- thin wrappers with the C names -----------------------------------------
def tdi_status_str(s: int) -> str:
    return lib().tdi_status_str(int(s)).decode()


def tdi_check_config(cfg: tdi_config, orb: tdi_orbit) -> int:
    return lib().tdi_check_config(C.byref(cfg), C.byref(orb))


def tdi_check_batch(cfg: tdi_config, n_sources: int, src, offsets) -> int:
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    return lib().tdi_check_batch(C.byref(cfg), int(n_sources), src,
                                 offs.ctypes.data_as(C.POINTER(C.c_int64)))


def tdi_plan_create(cfg: tdi_config, orb: tdi_orbit, max_sources: int, max_total: int, stream: int = 0):
    h = C.c_void_p()
    st = lib().tdi_plan_create(C.byref(h), C.byref(cfg), C.byref(orb), int(max_sources),
                               int(max_total), C.c_void_p(stream))
    return st, h


def tdi_run(plan, n_sources: int, src, offsets, hp_ptr: int, hc_ptr: int, x_ptr: int, y_ptr: int,
            z_ptr: int) -> int:
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    return lib().tdi_run(plan, int(n_sources), src, offs.ctypes.data_as(C.POINTER(C.c_int64)),
                         C.c_void_p(hp_ptr), C.c_void_p(hc_ptr), C.c_void_p(x_ptr),
                         C.c_void_p(y_ptr), C.c_void_p(z_ptr))


def tdi_run_noalloc(cfg: tdi_config, orb: tdi_orbit, n_sources: int, src, offsets, hp_ptr: int,
                    hc_ptr: int, x_ptr: int, y_ptr: int, z_ptr: int, stream: int = 0) -> int:
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    return lib().tdi_run_noalloc(C.byref(cfg), C.byref(orb), int(n_sources), src,
                                 offs.ctypes.data_as(C.POINTER(C.c_int64)), C.c_void_p(hp_ptr),
                                 C.c_void_p(hc_ptr), C.c_void_p(x_ptr), C.c_void_p(y_ptr),
                                 C.c_void_p(z_ptr), C.c_void_p(stream))


def tdi_run_links(plan, n_sources: int, src, offsets, hp_ptr: int, hc_ptr: int, y_ptr: int) -> int:
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    return lib().tdi_run_links(plan, int(n_sources), src, offs.ctypes.data_as(C.POINTER(C.c_int64)),
                               C.c_void_p(hp_ptr), C.c_void_p(hc_ptr), C.c_void_p(y_ptr))


def tdi_plan_sync(plan) -> int:
    return lib().tdi_plan_sync(plan)


def tdi_plan_kernel_times(plan, cap: int = 256):
    buf = (C.c_float * cap)()
    n = C.c_int32()
    st = lib().tdi_plan_kernel_times(plan, buf, cap, C.byref(n))
    return st, [buf[i] for i in range(n.value)]


def tdi_plan_set_timing(plan, on: int) -> int:
    return lib().tdi_plan_set_timing(plan, int(on))


def tdi_plan_describe(plan) -> dict:
    buf = C.create_string_buffer(512)
    lib().tdi_plan_describe(plan, buf, 512)
    return json.loads(buf.value.decode())


def tdi_plan_destroy(plan) -> int:
    return lib().tdi_plan_destroy(plan)


# --- conveniences -------------------------------------------------------------
def make_orbit(d: dict) -> tdi_orbit:
    o = tdi_orbit(int(d["kind"]), 0, float(d["L"]), float(d["R"]), float(d["omega"]),
                  float(d["kappa0"]), float(d["lambda0"]), float(d.get("t_freeze", 0.0)))
    if d.get("table") is not None:
        tab = np.ascontiguousarray(d["table"], dtype=np.float64).reshape(-1, 3, 3)
        o._table = tab                       # kept alive with the struct
        o.table = tab.ctypes.data_as(C.POINTER(C.c_double))
        o.n_table = tab.shape[0]
        o.table_t0 = float(d["table_t0"])
        o.table_dt = float(d["table_dt"])
    return o


def make_config(d: dict, autotune: int = 0, use_graph: int = 0) -> tdi_config:
    return tdi_config(int(d["tdi_gen"]), int(d["mode"]), int(d["taps"]), int(d["stencil_order"]),
                      int(d.get("equal_arms", 0)), int(d.get("precision", 0)),
                      float(d["T_samples"]), float(d["sigma_samples"]), int(autotune), int(use_graph),
                      int(d.get("channels", 0)), int(d.get("lfa_terms", 0)),
                      int(d.get("nested_delays", 0)), int(d.get("fast_tile_chunks", 0)),
                      int(d.get("x20_from_x15", 0)))


def make_sources(records) -> C.Array:
    """tdi_source array from records with fields beta, lam, psi, t0, dt, t_hyb."""
    n = len(records)
    arr = (tdi_source * max(1, n))()
    for i, r in enumerate(records):
        arr[i] = tdi_source(float(r["beta"]), float(r["lam"]), float(r["psi"]), float(r["t0"]),
                            float(r["dt"]), float(r["t_hyb"]))
    return arr


class Plan:
    """RAII wrapper of a tdi_plan bound to a torch device and stream."""

    def __init__(self, cfg: dict, orbit: dict, max_sources: int, max_total: int,
                 autotune: bool = False, use_graph: bool = False, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the TDI library needs a HIP device (no CPU fallback)")
        self.torch = torch
        self.cfg_d = dict(cfg)
        self.cfg = make_config(cfg, int(autotune), int(use_graph))
        self.orb = make_orbit(orbit)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        st, h = tdi_plan_create(self.cfg, self.orb, max_sources, max_total, self.stream.cuda_stream)
        if st != TDI_OK:
            raise TdiError(st, "tdi_plan_create")
        self.handle = h
        self.fp32 = int(cfg.get("precision", 0)) == TDI_FP32_BULK

    def out_dtype(self):
        return self.torch.float32 if self.fp32 else self.torch.float64

    def run(self, sources, offsets, hp, hc, X=None, Y=None, Z=None):
        """Enqueue one batch.  hp, hc: float64 CUDA tensors; returns (X, Y, Z)."""
        torch = self.torch
        n = int(offsets[-1])
        if hp.dtype != torch.float64 or hc.dtype != torch.float64 or not hp.is_cuda or not hc.is_cuda:
            raise TypeError("hp, hc must be float64 device tensors")
        if not (hp.is_contiguous() and hc.is_contiguous()) or hp.numel() < n or hc.numel() < n:
            raise ValueError("hp, hc must be contiguous with at least offsets[-1] samples")
        outs = []
        for o in (X, Y, Z):
            if o is None:
                o = torch.empty(max(n, 1), dtype=self.out_dtype(), device=hp.device)
            elif o.dtype != self.out_dtype() or not o.is_contiguous() or o.numel() < n:
                raise TypeError("output tensors must be contiguous with the plan's output dtype")
            outs.append(o)
        src = sources if isinstance(sources, C.Array) else make_sources(sources)
        st = tdi_run(self.handle, len(offsets) - 1, src, offsets, hp.data_ptr(), hc.data_ptr(),
                     outs[0].data_ptr(), outs[1].data_ptr(), outs[2].data_ptr())
        if st != TDI_OK:
            raise TdiError(st, "tdi_run")
        return outs[0][:n], outs[1][:n], outs[2][:n]

    def run_links(self, sources, offsets, hp, hc, y=None):
        """Enqueue the six link outputs of one batch; returns a (6, total) view
        (slots +1, +2, +3, -1, -2, -3)."""
        torch = self.torch
        n = int(offsets[-1])
        if hp.dtype != torch.float64 or hc.dtype != torch.float64 or not hp.is_cuda or not hc.is_cuda:
            raise TypeError("hp, hc must be float64 device tensors")
        if not (hp.is_contiguous() and hc.is_contiguous()) or hp.numel() < n or hc.numel() < n:
            raise ValueError("hp, hc must be contiguous with at least offsets[-1] samples")
        if y is None:
            y = torch.empty(max(6 * n, 1), dtype=self.out_dtype(), device=hp.device)
        elif y.dtype != self.out_dtype() or not y.is_contiguous() or y.numel() < 6 * n:
            raise TypeError("y must be contiguous with 6 * offsets[-1] elements of the plan's dtype")
        src = sources if isinstance(sources, C.Array) else make_sources(sources)
        st = tdi_run_links(self.handle, len(offsets) - 1, src, offsets, hp.data_ptr(), hc.data_ptr(),
                           y.data_ptr())
        if st != TDI_OK:
            raise TdiError(st, "tdi_run_links")
        return y[:6 * n].view(6, n)

    def sync(self) -> int:
        return tdi_plan_sync(self.handle)

    def kernel_times(self):
        st, v = tdi_plan_kernel_times(self.handle)
        if st != TDI_OK:
            raise TdiError(st, "tdi_plan_kernel_times")
        return v

    def set_timing(self, on: bool):
        st = tdi_plan_set_timing(self.handle, int(bool(on)))
        if st != TDI_OK:
            raise TdiError(st, "tdi_plan_set_timing")

    def describe(self) -> dict:
        return tdi_plan_describe(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            tdi_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def response(batch, cfg: dict, orbit: dict, device="cuda:0", autotune=False, use_graph=False,
             info: dict | None = None):
    """One-shot helper: host Batch -> (X, Y, Z) numpy arrays computed on the GPU.
    If info is a dict it receives the plan's launch description."""
    import torch
    hp = torch.as_tensor(np.asarray(batch.hp), dtype=torch.float64, device=device)
    hc = torch.as_tensor(np.asarray(batch.hc), dtype=torch.float64, device=device)
    with Plan(cfg, orbit, max(1, batch.n_sources), max(1, batch.total), autotune, use_graph) as p:
        X, Y, Z = p.run(batch.sources, batch.offsets, hp, hc)
        st = p.sync()
        if st != TDI_OK:
            raise TdiError(st, "tdi_plan_sync")
        if info is not None:
            info.update(p.describe())
        return np.stack([X.double().cpu().numpy(), Y.double().cpu().numpy(), Z.double().cpu().numpy()])


# --- noise-weighted inner product ------------------------------------------------
def make_noise(d: dict) -> tdi_noise:
    return tdi_noise(int(d["tdi_gen"]), int(d["galactic"]), float(d["T_obs_years"]), float(d["L_m"]),
                     float(d["f_min"]), float(d["f_max"]))


def tdi_check_noise(noise: tdi_noise) -> int:
    return lib().tdi_check_noise(C.byref(noise))


def tdi_ip_plan_create(noise: tdi_noise, precision: int, dt: float, max_sources: int, max_total: int,
                       max_source: int, stream: int = 0):
    h = C.c_void_p()
    st = lib().tdi_ip_plan_create(C.byref(h), C.byref(noise), int(precision), float(dt), int(max_sources),
                                  int(max_total), int(max_source), C.c_void_p(stream))
    return st, h


def tdi_ip_run(plan, n_sources: int, offsets, x_ptrs, y_ptrs, out_ptr: int) -> int:
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    xa = (C.c_void_p * 3)(*[C.c_void_p(int(v)) for v in x_ptrs])
    ya = (C.c_void_p * 3)(*[C.c_void_p(int(v)) for v in y_ptrs])
    return lib().tdi_ip_run(plan, int(n_sources), offs.ctypes.data_as(C.POINTER(C.c_int64)), xa, ya,
                            C.c_void_p(out_ptr))


def tdi_ip_kernel_times(plan, cap: int = 192):
    buf = (C.c_float * cap)()
    n = C.c_int32()
    st = lib().tdi_ip_kernel_times(plan, buf, cap, C.byref(n))
    return st, [buf[i] for i in range(n.value)]


def tdi_ip_plan_destroy(plan) -> int:
    return lib().tdi_ip_plan_destroy(plan)


class IpPlan:
    """RAII wrapper of a tdi_ip_plan bound to a torch device and stream."""

    def __init__(self, noise: dict, precision: int, dt: float, max_sources: int, max_total: int,
                 max_source: int, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the TDI library needs a HIP device (no CPU fallback)")
        self.torch = torch
        self.fp64 = int(precision) == TDI_FP64
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        st, h = tdi_ip_plan_create(make_noise(noise), precision, dt, max_sources, max_total, max_source,
                                   self.stream.cuda_stream)
        if st != TDI_OK:
            raise TdiError(st, "tdi_ip_plan_create")
        self.handle = h

    def run(self, offsets, x3, y3, out=None):
        """x3, y3: three device tensors each (A, E, T) of the plan's dtype.
        Returns a (n_sources, 3, 3) float64 device tensor of <x|x>, <x|y>, <y|y>."""
        torch = self.torch
        dt = torch.float64 if self.fp64 else torch.float32
        n_src = len(offsets) - 1
        total = int(offsets[-1])
        for t in list(x3) + list(y3):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() < total:
                raise TypeError("inputs must be contiguous device tensors of the plan's dtype")
        if out is None:
            out = torch.empty((max(n_src, 1), 3, 3), dtype=torch.float64, device=x3[0].device)
        st = tdi_ip_run(self.handle, n_src, offsets, [t.data_ptr() for t in x3],
                        [t.data_ptr() for t in y3], out.data_ptr())
        if st != TDI_OK:
            raise TdiError(st, "tdi_ip_run")
        return out[:n_src]

    def kernel_times(self):
        st, v = tdi_ip_kernel_times(self.handle)
        if st != TDI_OK:
            raise TdiError(st, "tdi_ip_kernel_times")
        return v

    def close(self):
        if getattr(self, "handle", None):
            tdi_ip_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def header_symbols(path: str | None = None):
    """Function names declared in include/tdi.h."""
    import re
    path = path or os.path.join(os.path.dirname(_HERE), "include", "tdi.h")
    txt = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:tdi_status|const char\*)\s+(tdi_\w+)\s*\(", txt, re.M)))
