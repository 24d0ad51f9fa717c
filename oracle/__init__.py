"""ctypes binding of the FP64 CPU oracle (``oracle/tdi_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle is the independent, slow FP64 statement
of the paper's response used to check the HIP library.  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg import this module; the
library under ``paper_2505_09600_amd`` never does.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tdi_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

FULL, LFA, HYBRID = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Orbit(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad_", C.c_int32), ("L", C.c_double),
                ("R", C.c_double), ("omega", C.c_double), ("kappa0", C.c_double),
                ("lambda0", C.c_double), ("t_freeze", C.c_double),
                ("table", C.POINTER(C.c_double)), ("n_table", C.c_int64),
                ("table_t0", C.c_double), ("table_dt", C.c_double)]


class Config(C.Structure):
    _fields_ = [("tdi_gen", C.c_int32), ("mode", C.c_int32), ("taps", C.c_int32),
                ("stencil_order", C.c_int32), ("equal_arms", C.c_int32),
                ("lfa_terms", C.c_int32), ("nested_delays", C.c_int32), ("x20_from_x15", C.c_int32),
                ("T_samples", C.c_double),
                ("sigma_samples", C.c_double)]


class Source(C.Structure):
    _fields_ = [("beta", C.c_double), ("lam", C.c_double), ("psi", C.c_double),
                ("t0", C.c_double), ("dt", C.c_double), ("t_hyb", C.c_double)]


class Geom(C.Structure):
    _fields_ = [("T", C.c_double * 6), ("n", (C.c_double * 3) * 6),
                ("xi_p", C.c_double * 6), ("xi_c", C.c_double * 6),
                ("kn", C.c_double * 6), ("ds", C.c_double * 6), ("dr", C.c_double * 6),
                ("mu", C.c_double * 3), ("R", (C.c_double * 3) * 3)]


_lib = None
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        L.orc_link_ends.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_triad.argtypes = [C.c_double, C.c_double, _D, _D, _D]
        L.orc_positions.argtypes = [C.POINTER(Orbit), C.c_double, _D]
        L.orc_light_time.argtypes = [C.POINTER(Orbit), C.c_int, C.c_double]
        L.orc_light_time.restype = C.c_double
        L.orc_geometry.argtypes = [C.POINTER(Orbit), C.c_double, C.c_double, C.c_double, C.POINTER(Geom)]
        L.orc_split.argtypes = [C.c_int64, C.c_double, C.c_double, _I64, _D]
        L.orc_lagrange.argtypes = [_D, C.c_int64, C.c_int64, C.c_double, C.c_int]
        L.orc_lagrange.restype = C.c_double
        L.orc_lagrange_weights.argtypes = [C.c_double, C.c_int, _D]
        L.orc_stencil.argtypes = [_D, C.c_int64, C.c_int, C.c_int, C.c_double, _D]
        L.orc_links.argtypes = [C.POINTER(Config), C.POINTER(Orbit), C.POINTER(Source),
                                C.c_int64, _D, _D, _D]
        L.orc_link_outputs.argtypes = [C.POINTER(Config), C.POINTER(Orbit), C.POINTER(Source),
                                       C.c_int64, _D, _D, _D]
        L.orc_tdi_combine.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_double, _D, _D, _D, _D, _D]
        L.orc_tdi_combine_nested.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_double,
                                             _D, _D, _D, _D, _D]
        L.orc_nested_term.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_response.argtypes = [C.POINTER(Config), C.POINTER(Orbit), C.POINTER(Source),
                                   C.c_int64, _D, _D, _D, _D, _D]
        L.orc_response_at.argtypes = [C.POINTER(Config), C.POINTER(Orbit), C.POINTER(Source),
                                      C.c_int64, _D, _D, C.c_int64, _I64, _D, _D, _D]
        L.orc_response_batch.argtypes = [C.POINTER(Config), C.POINTER(Orbit), C.c_int64,
                                         C.POINTER(Source), _I64, _D, _D, _D, _D, _D]
        L.orc_response_batch_at.argtypes = [C.POINTER(Config), C.POINTER(Orbit), C.c_int64,
                                            C.POINTER(Source), _I64, _D, _D, _I64, _I64, _D, _D, _D]
        L.orc_response_abs_at.argtypes = [C.POINTER(Config), C.POINTER(Orbit), C.POINTER(Source),
                                          C.c_int64, _D, _D, C.c_int64, _I64, _D, _D, _D]
        L.orc_full_terms_absmax.argtypes = [C.POINTER(Config), C.POINTER(Orbit), C.POINTER(Source),
                                            C.c_int64, _D, _D, _D]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def make_orbit(d: dict) -> Orbit:
    o = Orbit(int(d["kind"]), 0, d["L"], d["R"], d["omega"], d["kappa0"], d["lambda0"],
              d.get("t_freeze", 0.0))
    if d.get("table") is not None:
        tab = np.ascontiguousarray(d["table"], dtype=np.float64).reshape(-1, 3, 3)
        o._table = tab                       # kept alive with the struct
        o.table = tab.ctypes.data_as(C.POINTER(C.c_double))
        o.n_table = tab.shape[0]
        o.table_t0 = float(d["table_t0"])
        o.table_dt = float(d["table_dt"])
    return o


def make_config(d: dict) -> Config:
    return Config(int(d["tdi_gen"]), int(d["mode"]), int(d["taps"]), int(d["stencil_order"]),
                  int(d.get("equal_arms", 0)), int(d.get("lfa_terms", 0)),
                  int(d.get("nested_delays", 0)), int(d.get("x20_from_x15", 0)), float(d["T_samples"]),
                  float(d["sigma_samples"]))


def make_source(rec) -> Source:
    return Source(float(rec["beta"]), float(rec["lam"]), float(rec["psi"]), float(rec["t0"]),
                  float(rec["dt"]), float(rec["t_hyb"]))


def link_ends(l: int):
    s, r = C.c_int(), C.c_int()
    lib().orc_link_ends(l, C.byref(s), C.byref(r))
    return s.value, r.value


def triad(beta, lam):
    k, u, v = np.zeros(3), np.zeros(3), np.zeros(3)
    lib().orc_triad(beta, lam, _dp(k), _dp(u), _dp(v))
    return k, u, v


def positions(orbit: dict, t: float):
    R = np.zeros((3, 3))
    o = make_orbit(orbit)
    lib().orc_positions(C.byref(o), t, _dp(R))
    return R


def light_time(orbit: dict, l: int, t: float) -> float:
    o = make_orbit(orbit)
    return lib().orc_light_time(C.byref(o), l, t)


def geometry(orbit: dict, beta, lam, t):
    o, g = make_orbit(orbit), Geom()
    lib().orc_geometry(C.byref(o), beta, lam, t, C.byref(g))
    return dict(T=np.array(g.T[:]), n=np.array([g.n[a][:] for a in range(6)]),
                xi_p=np.array(g.xi_p[:]), xi_c=np.array(g.xi_c[:]), kn=np.array(g.kn[:]),
                ds=np.array(g.ds[:]), dr=np.array(g.dr[:]), mu=np.array(g.mu[:]),
                R=np.array([g.R[i][:] for i in range(3)]))


def split(k: int, d: float, dt: float):
    i0, x = C.c_int64(), C.c_double()
    lib().orc_split(k, d, dt, C.byref(i0), C.byref(x))
    return i0.value, x.value


def lagrange(s, i0: int, x: float, N: int) -> float:
    s = _f64(s)
    return lib().orc_lagrange(_dp(s), len(s), i0, x, N)


def lagrange_weights(x: float, N: int):
    w = np.zeros(N)
    lib().orc_lagrange_weights(x, N, _dp(w))
    return w


def stencil(h, m: int, p: int, dt: float):
    h = _f64(h)
    g = np.zeros_like(h)
    lib().orc_stencil(_dp(h), len(h), m, p, dt, _dp(g))
    return g


def links(cfg: dict, orbit: dict, rec, hp, hc):
    hp, hc = _f64(hp), _f64(hc)
    y = np.zeros((6, len(hp)))
    c, o, s = make_config(cfg), make_orbit(orbit), make_source(rec)
    lib().orc_links(C.byref(c), C.byref(o), C.byref(s), len(hp), _dp(hp), _dp(hc), _dp(y))
    return y


def link_outputs(cfg: dict, orbit: dict, rec, hp, hc):
    """The six single-link outputs (6, n) in cfg's mode (full, LFA or hybrid)."""
    hp, hc = _f64(hp), _f64(hc)
    y = np.zeros((6, len(hp)))
    c, o, s = make_config(cfg), make_orbit(orbit), make_source(rec)
    lib().orc_link_outputs(C.byref(c), C.byref(o), C.byref(s), len(hp), _dp(hp), _dp(hc), _dp(y))
    return y


def tdi_combine(gen: int, N: int, dt: float, y, T, nested: bool = False):
    y, T = _f64(y), _f64(T)
    n = y.shape[1]
    X, Y, Z = np.zeros(n), np.zeros(n), np.zeros(n)
    fn = lib().orc_tdi_combine_nested if nested else lib().orc_tdi_combine
    fn(gen, N, n, dt, _dp(y), _dp(T), _dp(X), _dp(Y), _dp(Z))
    return X, Y, Z


def nested_term(t: int):
    """(sign, link, delays in the order applied) of term t in time-nested form."""
    sign, link, nd = C.c_int(), C.c_int(), C.c_int()
    d = (C.c_int * 8)()
    lib().orc_nested_term(t, C.byref(sign), C.byref(link), C.byref(nd), d)
    return sign.value, link.value, tuple(d[:nd.value])


def response(cfg: dict, orbit: dict, rec, hp, hc):
    hp, hc = _f64(hp), _f64(hc)
    n = len(hp)
    X, Y, Z = np.zeros(n), np.zeros(n), np.zeros(n)
    c, o, s = make_config(cfg), make_orbit(orbit), make_source(rec)
    lib().orc_response(C.byref(c), C.byref(o), C.byref(s), n, _dp(hp), _dp(hc),
                       _dp(X), _dp(Y), _dp(Z))
    return np.stack([X, Y, Z])


def response_at(cfg: dict, orbit: dict, rec, hp, hc, ks):
    hp, hc = _f64(hp), _f64(hc)
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    X, Y, Z = np.zeros(len(ks)), np.zeros(len(ks)), np.zeros(len(ks))
    c, o, s = make_config(cfg), make_orbit(orbit), make_source(rec)
    lib().orc_response_at(C.byref(c), C.byref(o), C.byref(s), len(hp), _dp(hp), _dp(hc),
                          len(ks), ks.ctypes.data_as(_I64), _dp(X), _dp(Y), _dp(Z))
    return np.stack([X, Y, Z])


def response_abs_at(cfg: dict, orbit: dict, rec, hp, hc, ks):
    """Rounding-error scale A_c(k) at sample indices ks (3, len(ks))."""
    hp, hc = _f64(hp), _f64(hc)
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    X, Y, Z = np.zeros(len(ks)), np.zeros(len(ks)), np.zeros(len(ks))
    c, o, s = make_config(cfg), make_orbit(orbit), make_source(rec)
    lib().orc_response_abs_at(C.byref(c), C.byref(o), C.byref(s), len(hp), _dp(hp), _dp(hc),
                              len(ks), ks.ctypes.data_as(_I64), _dp(X), _dp(Y), _dp(Z))
    return np.stack([X, Y, Z])


def fp64_tolerance(cfg, orbit, rec, hp, hc, ks, ref_at_ks, k_ops: float = 64.0, floor: float = 1e-12):
    """Per-channel FP64 parity bar: max(floor, k_ops * 2^-53 * kappa_c) with
    kappa_c = max A_c / max |X_c| over the sampled indices (conditioning)."""
    A = response_abs_at(cfg, orbit, rec, hp, hc, ks)
    peak = np.max(np.abs(ref_at_ks), axis=1)
    kappa = np.where(peak > 0, np.max(A, axis=1) / np.where(peak > 0, peak, 1.0), 0.0)
    return np.maximum(floor, k_ops * 2.0 ** -53 * kappa), kappa


def response_batch(cfg: dict, orbit: dict, batch):
    """Whole-batch response (OpenMP across sources) for a workload.Batch."""
    hp, hc = _f64(batch.hp), _f64(batch.hc)
    n = len(hp)
    X, Y, Z = np.zeros(n), np.zeros(n), np.zeros(n)
    srcs = (Source * max(1, batch.n_sources))(*[make_source(r) for r in batch.sources])
    offs = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    c, o = make_config(cfg), make_orbit(orbit)
    lib().orc_response_batch(C.byref(c), C.byref(o), batch.n_sources, srcs,
                             offs.ctypes.data_as(_I64), _dp(hp), _dp(hc), _dp(X), _dp(Y), _dp(Z))
    return np.stack([X, Y, Z])


def response_batch_at(cfg: dict, orbit: dict, batch, ks_per_source):
    """Sampled outputs of a batch: ks_per_source[i] lists sample indices of source i.
    Returns (3, sum of lengths) in the concatenated order (OpenMP across sources)."""
    hp, hc = _f64(batch.hp), _f64(batch.hc)
    lens = [len(k) for k in ks_per_source]
    koffs = np.zeros(len(lens) + 1, dtype=np.int64)
    koffs[1:] = np.cumsum(lens)
    ks = np.ascontiguousarray(np.concatenate([np.asarray(k, dtype=np.int64) for k in ks_per_source])
                              if lens else np.zeros(0, dtype=np.int64))
    m = int(koffs[-1])
    X, Y, Z = np.zeros(m), np.zeros(m), np.zeros(m)
    srcs = (Source * max(1, batch.n_sources))(*[make_source(r) for r in batch.sources])
    offs = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    c, o = make_config(cfg), make_orbit(orbit)
    lib().orc_response_batch_at(C.byref(c), C.byref(o), batch.n_sources, srcs, offs.ctypes.data_as(_I64),
                                _dp(hp), _dp(hc), koffs.ctypes.data_as(_I64), ks.ctypes.data_as(_I64),
                                _dp(X), _dp(Y), _dp(Z))
    return np.stack([X, Y, Z])


def full_terms_absmax(cfg: dict, orbit: dict, rec, hp, hc):
    hp, hc = _f64(hp), _f64(hc)
    out = np.zeros(3)
    c, o, s = make_config(cfg), make_orbit(orbit), make_source(rec)
    lib().orc_full_terms_absmax(C.byref(c), C.byref(o), C.byref(s), len(hp), _dp(hp), _dp(hc), _dp(out))
    return out


def num_threads() -> int:
    return lib().orc_num_threads()


def peak_rel_err(test, ref):
    """Per-channel max |test - ref| / max |ref| (3-vector)."""
    test = np.asarray(test, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    out = []
    for c in range(3):
        peak = float(np.max(np.abs(ref[c]))) if ref[c].size else 0.0
        err = float(np.max(np.abs(test[c] - ref[c]))) if ref[c].size else 0.0
        out.append(err / peak if peak > 0 else (0.0 if err == 0 else math.inf))
    return np.array(out)
