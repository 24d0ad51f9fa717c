"""Host-side checks of the C ABI (no GPU needed): symbols, validation codes."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_2505_09600_amd import tdi as T
from paper_2505_09600_amd import workload as W


@pytest.fixture(scope="module")
def L():
    return T.lib()


def _cfg(**kw):
    d = W.default_config(tdi_gen=20, mode=2, taps=32, stencil_order=4, precision=1)
    d.update(kw)
    return T.make_config(d)


def _orb(**kw):
    d = W.default_orbit()
    d.update(kw)
    return T.make_orbit(d)


def test_library_exports_every_declared_symbol(L):
    declared = T.header_symbols()
    assert set(declared) == set(T.EXPORTED)
    for name in declared:
        assert hasattr(L, name), name


def test_header_documents_each_entry_point():
    import os
    import re
    txt = open(os.path.join(os.path.dirname(T.__file__), "..", "include", "tdi.h")).read()
    for name in T.header_symbols():
        m = re.search(r"(/\*(?:(?!\*/).)*\*/)\s*\n\s*(?:tdi_status|const char\*)\s+" + name + r"\s*\(",
                      txt, re.S)
        assert m, f"{name} has no comment right above its declaration"


def test_status_strings(L):
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert T.tdi_status_str(s) and T.tdi_status_str(s) != "unknown status"
    assert T.tdi_status_str(42) == "unknown status"


@pytest.mark.parametrize("field,value,code", [
    ("tdi_gen", 30, T.TDI_EUNSUPPORTED),
    ("mode", 3, T.TDI_EUNSUPPORTED),
    ("precision", 2, T.TDI_EUNSUPPORTED),
    ("interp_taps", 12, T.TDI_ERANGE),
    ("interp_taps", 64, T.TDI_ERANGE),
    ("stencil_order", 6, T.TDI_ERANGE),
    ("lfa_equal_arms", 2, T.TDI_ERANGE),
    ("hyb_T_samples", 0.0, T.TDI_ERANGE),
    ("hyb_sigma_samples", -1.0, T.TDI_ERANGE),
    ("hyb_sigma_samples", math.nan, T.TDI_ERANGE),
    ("autotune", 5, T.TDI_ERANGE),
    ("channels", 2, T.TDI_EUNSUPPORTED),
    ("lfa_terms", 3, T.TDI_ERANGE),
    ("lfa_terms", -1, T.TDI_ERANGE),
    ("nested_delays", 2, T.TDI_ERANGE),
    ("nested_delays", -1, T.TDI_ERANGE),
    ("fast_tile_chunks", 3, T.TDI_ERANGE),
    ("fast_tile_chunks", 8, T.TDI_ERANGE),
    ("fast_tile_chunks", -1, T.TDI_ERANGE),
    ("lfa_x20_from_x15", 2, T.TDI_ERANGE),
    ("lfa_x20_from_x15", -1, T.TDI_ERANGE),
])
def test_config_validation(L, field, value, code):
    c = _cfg()
    assert T.tdi_check_config(c, _orb()) == T.TDI_OK
    setattr(c, field, value)
    assert T.tdi_check_config(c, _orb()) == code


@pytest.mark.parametrize("field,value,code", [
    ("kind", 7, T.TDI_EUNSUPPORTED),
    ("reserved", 1, T.TDI_EINVAL),
    ("L_m", -1.0, T.TDI_ERANGE),
    ("R_m", 1.0e9, T.TDI_ERANGE),
    ("omega", math.inf, T.TDI_ERANGE),
    ("omega", 1.0, T.TDI_ERANGE),
    ("kappa0", math.nan, T.TDI_ERANGE),
])
def test_orbit_validation(L, field, value, code):
    o = _orb()
    setattr(o, field, value)
    assert T.tdi_check_config(_cfg(), o) == code


def test_null_arguments(L):
    assert L.tdi_check_config(None, None) == T.TDI_EINVAL
    assert L.tdi_check_batch(None, 0, None, None) == T.TDI_EINVAL
    assert L.tdi_run(None, 0, None, None, None, None, None, None, None) == T.TDI_ESTATE
    assert L.tdi_plan_sync(None) == T.TDI_ESTATE
    assert L.tdi_plan_destroy(None) == T.TDI_EINVAL
    n = C.c_int32()
    assert L.tdi_plan_kernel_times(None, None, 0, C.byref(n)) == T.TDI_EINVAL
    assert L.tdi_plan_set_timing(None, 1) == T.TDI_ESTATE


def _recs(n=3, **kw):
    out = []
    for i in range(n):
        r = dict(beta=0.3, lam=1.0 + i, psi=0.2, t0=0.0, dt=10.0, t_hyb=math.inf)
        r.update(kw)
        out.append(r)
    return out


@pytest.mark.parametrize("kw,code", [
    ({}, T.TDI_OK),
    (dict(dt=0.0), T.TDI_ERANGE),
    (dict(dt=-1.0), T.TDI_ERANGE),
    (dict(beta=2.0), T.TDI_ERANGE),
    (dict(lam=math.nan), T.TDI_ERANGE),
    (dict(t_hyb=math.nan), T.TDI_ERANGE),
    (dict(t_hyb=-math.inf), T.TDI_OK),
    (dict(t0=math.inf), T.TDI_ERANGE),
])
def test_batch_validation(L, kw, code):
    src = T.make_sources(_recs(**kw))
    assert T.tdi_check_batch(_cfg(), 3, src, [0, 10, 10, 25]) == code


def test_offsets_validation(L):
    src = T.make_sources(_recs())
    assert T.tdi_check_batch(_cfg(), 3, src, [1, 10, 20, 30]) == T.TDI_EINVAL
    assert T.tdi_check_batch(_cfg(), 3, src, [0, 10, 5, 30]) == T.TDI_EINVAL
    assert T.tdi_check_batch(_cfg(), -1, src, [0]) == T.TDI_EINVAL
    assert T.tdi_check_batch(_cfg(), 0, None, [0]) == T.TDI_OK
    assert T.tdi_check_batch(_cfg(), 3, src, [0, 0, 0, 0]) == T.TDI_OK


def test_plan_create_without_device_reports_edevice(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    st, h = T.tdi_plan_create(_cfg(), _orb(), 4, 1000)
    assert st == T.TDI_EDEVICE
    assert not h.value


def test_plan_refuses_bad_config_before_device(L):
    c = _cfg(tdi_gen=7)
    st, h = T.tdi_plan_create(c, _orb(), 4, 1000)
    assert st == T.TDI_EUNSUPPORTED


def test_python_plan_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    with pytest.raises(RuntimeError):
        T.Plan(W.default_config(), W.default_orbit(), 1, 10)


def _noise(**kw):
    d = dict(tdi_gen=20, galactic=1, T_obs_years=1.0, L_m=2.5e9, f_min=1e-4, f_max=0.029)
    d.update(kw)
    return T.make_noise(d)


@pytest.mark.parametrize("field,value,code", [
    ("tdi_gen", 10, T.TDI_EUNSUPPORTED),
    ("galactic", 2, T.TDI_ERANGE),
    ("T_obs_years", 0.0, T.TDI_ERANGE),
    ("L_m", math.nan, T.TDI_ERANGE),
    ("f_min", 0.0, T.TDI_ERANGE),
    ("f_max", 1e-5, T.TDI_ERANGE),
    ("f_max", 0.031, T.TDI_ERANGE),     # past the first zero of the TDI 2.0 PSD, c/(4L)
])
def test_noise_validation(L, field, value, code):
    n = _noise()
    assert T.tdi_check_noise(n) == T.TDI_OK
    setattr(n, field, value)
    assert T.tdi_check_noise(n) == code


def test_noise_band_limit_depends_on_generation(L):
    # TDI 1.5 PSDs vanish first at c/(2L) = 0.06 Hz
    assert T.tdi_check_noise(_noise(tdi_gen=15, f_max=0.05)) == T.TDI_OK
    assert T.tdi_check_noise(_noise(tdi_gen=20, f_max=0.05)) == T.TDI_ERANGE


def test_ip_entry_points_without_device(L):
    st, h = T.tdi_ip_plan_create(_noise(), T.TDI_FP32_BULK, 10.0, 4, 1000, 500)
    assert st == T.TDI_EDEVICE and not h.value
    # argument errors are reported before any device work
    assert T.tdi_ip_plan_create(_noise(f_min=-1.0), T.TDI_FP32_BULK, 10.0, 4, 1000, 500)[0] == T.TDI_ERANGE
    assert T.tdi_ip_plan_create(_noise(), 7, 10.0, 4, 1000, 500)[0] == T.TDI_EUNSUPPORTED
    assert T.tdi_ip_plan_create(_noise(), T.TDI_FP32_BULK, 0.0, 4, 1000, 500)[0] == T.TDI_ERANGE
    # longest supported source: 2^25 (FP32), 2^23 (FP64)
    assert T.tdi_ip_plan_create(_noise(), T.TDI_FP64, 10.0, 4, 1 << 24, (1 << 23) + 1)[0] == T.TDI_ERANGE
    assert T.tdi_ip_plan_create(_noise(), T.TDI_FP32_BULK, 10.0, 4, 1 << 26, (1 << 25) + 1)[0] == T.TDI_ERANGE
    assert T.tdi_ip_plan_create(_noise(), T.TDI_FP64, 10.0, 4, 1 << 24, 1 << 23)[0] == T.TDI_EDEVICE
    assert T.tdi_ip_plan_create(_noise(), T.TDI_FP32_BULK, 10.0, 4, 1 << 26, 1 << 25)[0] == T.TDI_EDEVICE
    assert T.tdi_ip_run(None, 1, np.array([0, 5]), [0, 0, 0], [0, 0, 0], 0) == T.TDI_EINVAL
    assert T.lib().tdi_ip_plan_destroy(None) == T.TDI_EINVAL
    assert T.lib().tdi_ip_kernel_times(None, None, 0, None) == T.TDI_EINVAL


def _table_orb(n=16, dt=3600.0, **kw):
    tab = W.keplerian_orbit_table(0.0, dt, n)
    d = W.table_orbit(tab, 0.0, dt)
    d.update(kw)
    return d


def test_table_orbit_validation(L):
    c = _cfg()
    assert T.tdi_check_config(c, T.make_orbit(_table_orb())) == T.TDI_OK
    assert T.tdi_check_config(c, T.make_orbit(_table_orb(n=7))) == T.TDI_ERANGE
    assert T.tdi_check_config(c, T.make_orbit(_table_orb(table_dt=0.0))) == T.TDI_ERANGE
    bad = _table_orb()
    bad["table"] = bad["table"].copy()
    bad["table"][3, 1, 2] = math.nan
    assert T.tdi_check_config(c, T.make_orbit(bad)) == T.TDI_ERANGE
    o = T.make_orbit(_table_orb())
    o.table = None
    assert T.tdi_check_config(c, o) == T.TDI_EINVAL


def test_noalloc_host_checks_before_device(L):
    """tdi_run_noalloc: every argument error and limit is reported before any
    device call (fake device addresses are never touched)."""
    src = T.make_sources(_recs(3))
    offs = [0, 100, 200, 300]
    fake = 1 << 20
    cfg, orb = _cfg(), _orb()
    run = T.tdi_run_noalloc
    assert L.tdi_run_noalloc(None, None, 0, None, None, None, None, None, None, None, None) == T.TDI_EINVAL
    assert run(_cfg(tdi_gen=7), orb, 3, src, offs, fake, fake, fake, fake, fake) == T.TDI_EUNSUPPORTED
    assert run(cfg, orb, 3, src, [0, 100, 50, 300], fake, fake, fake, fake, fake) == T.TDI_EINVAL
    assert run(cfg, orb, 3, src, offs, 0, fake, fake, fake, fake) == T.TDI_EINVAL
    assert run(cfg, orb, 3, src, offs, fake + 4, fake, fake, fake, fake) == T.TDI_EINVAL
    assert run(cfg, orb, 0, None, [0], 0, 0, 0, 0, 0) == T.TDI_OK
    # the static scratch holds at most 256 sources
    big = T.make_sources(_recs(257))
    assert run(cfg, orb, 257, big, np.arange(258) * 10, fake, fake, fake, fake, fake) == T.TDI_ESTATE
    # sampled orbits need a device table: not available without allocation
    tab = W.keplerian_orbit_table(0.0, 1.0e4, 64)
    torb = T.make_orbit(W.table_orbit(tab, 0.0, 1.0e4))
    assert run(cfg, torb, 3, src, offs, fake, fake, fake, fake, fake) == T.TDI_EUNSUPPORTED
    import torch
    if not torch.cuda.is_available():
        assert run(cfg, orb, 3, src, offs, fake, fake, fake, fake, fake) == T.TDI_EDEVICE


def test_x20_shortcut_validation(L):
    """The TDI 2.0-from-1.5 LFA exists for TDI 2.0 only, is not combined with the
    next LFA term, and is not offered without allocation."""
    c = _cfg(x20_from_x15=1)
    assert T.tdi_check_config(c, _orb()) == T.TDI_OK
    assert T.tdi_check_config(_cfg(x20_from_x15=1, tdi_gen=15), _orb()) == T.TDI_ERANGE
    assert T.tdi_check_config(_cfg(x20_from_x15=1, lfa_terms=2), _orb()) == T.TDI_EUNSUPPORTED
    src = T.make_sources(_recs(3))
    fake = 1 << 20
    assert T.tdi_run_noalloc(c, _orb(), 3, src, [0, 100, 200, 300], fake, fake, fake, fake,
                             fake) == T.TDI_EUNSUPPORTED
