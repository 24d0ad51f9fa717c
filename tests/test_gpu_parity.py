"""GPU parity: the HIP library through its C ABI against the FP64 oracle.

Error metric per channel: max_k |X_gpu - X_oracle| / max_k |X_oracle|, over
every output sample.  FP64 bar: 1e-12 per channel, or 64 2^-53 kappa_c where
that is higher (``_tol64``: kappa_c = max A_c / max |X_c| from the oracle's
absolute-value evaluation; every source here has kappa below 141, so the bar is
1e-12 unless stated).  FP32-bulk bar: 1e-5.
"""
import math

import numpy as np
import pytest

from paper_2505_09600_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2505_09600_amd import tdi as T
    T.lib()
    return T


def _run_gpu(T, batch, cfg, orb, **kw):
    return T.response(batch, cfg, orb, **kw)


def _run_orc(orc, batch, cfg, orb):
    return orc.response_batch(cfg, orb, batch)


def _err(orc, got, ref):
    return orc.peak_rel_err(got, ref)


def _report(name, err, tol):
    tol = np.broadcast_to(np.asarray(tol, dtype=np.float64), (3,))
    print(f"[parity] {name}: err X,Y,Z = {err[0]:.3e} {err[1]:.3e} {err[2]:.3e}  "
          f"tol {tol[0]:.1e} {tol[1]:.1e} {tol[2]:.1e}", flush=True)


def _tol64(orc, batch, cfg, orb, ref):
    """Per-channel FP64 bar of a one-source batch: max(1e-12, 64 2^-53 kappa_c)."""
    rec, hp, hc = batch.source(0)
    ks = np.arange(len(hp))
    tol, _ = orc.fp64_tolerance(dict(cfg, precision=0), orb, rec, hp, hc, ks, ref)
    return tol


def _small_analytic(n=20000, mc=4e5, seed=11, dt=10.0, t0=3.0e6, hybrid=True):
    rng = np.random.default_rng(seed)
    beta = math.asin(rng.uniform(-1, 1))
    lam, psi, iota = rng.uniform(0, 2 * math.pi), rng.uniform(0, math.pi), math.acos(rng.uniform(-1, 1))
    rec, hp, hc, meta = W.make_source(mc, iota, beta, lam, psi, n, dt, t0=t0, hybrid=hybrid)
    return W._assemble([(rec, hp, hc, meta)], np)


def test_c1_full_fp64_frozen_tdi15(tdi, orc):
    batch, cfg, orb = W.config_c1()
    got = _run_gpu(tdi, batch, cfg, orb)
    ref = _run_orc(orc, batch, cfg, orb)
    err = _err(orc, got, ref)
    _report("c1 full fp64 tdi1.5 N16", err, 1e-12)
    assert np.all(err <= 1e-12)


@pytest.mark.parametrize("gen", [15, 20])
def test_full_fp64_analytic_orbit(tdi, orc, gen):
    batch = _small_analytic(mc=2e5)
    orb = W.default_orbit()
    cfg = W.default_config(tdi_gen=gen, mode=0, taps=32)
    got = _run_gpu(tdi, batch, cfg, orb)
    ref = _run_orc(orc, batch, cfg, orb)
    err = _err(orc, got, ref)
    tol = _tol64(orc, batch, cfg, orb, ref)
    _report(f"full fp64 tdi{gen} N32 analytic", err, tol)
    assert np.all(err <= tol)


@pytest.mark.parametrize("gen,p,eq", [(15, 2, 0), (15, 4, 1), (20, 2, 1), (20, 4, 0)])
def test_lfa_fp64(tdi, orc, gen, p, eq):
    batch = _small_analytic(mc=2e5)
    orb = W.default_orbit()
    cfg = W.default_config(tdi_gen=gen, mode=1, taps=32, stencil_order=p, equal_arms=eq)
    got = _run_gpu(tdi, batch, cfg, orb)
    ref = _run_orc(orc, batch, cfg, orb)
    err = _err(orc, got, ref)
    tol = _tol64(orc, batch, cfg, orb, ref)
    _report(f"lfa fp64 tdi{gen} p{p} eq{eq}", err, tol)
    assert np.all(err <= tol)


@pytest.mark.parametrize("gen", [15, 20])
def test_hybrid_fp64_and_fp32(tdi, orc, gen):
    batch = _small_analytic(mc=1.5e5, n=30000)
    assert math.isfinite(batch.sources[0]["t_hyb"])
    orb = W.default_orbit()
    cfg = W.default_config(tdi_gen=gen, mode=2, taps=32, stencil_order=4)
    ref = _run_orc(orc, batch, cfg, orb)
    got = _run_gpu(tdi, batch, cfg, orb)
    err = _err(orc, got, ref)
    tol = _tol64(orc, batch, cfg, orb, ref)
    _report(f"hybrid fp64 tdi{gen}", err, tol)
    assert np.all(err <= tol)
    got32 = _run_gpu(tdi, batch, dict(cfg, precision=1), orb)
    err32 = _err(orc, got32, ref)
    _report(f"hybrid fp32 tdi{gen}", err32, 1e-5)
    assert np.all(err32 <= 1e-5)


@pytest.mark.parametrize("eq", [0, 1])
@pytest.mark.parametrize("dt,mc,n,fast", [(10.0, 3e5, 40000, 1), (5.0, 6e5, 30000, 1), (60.0, 1e6, 8000, 0)])
def test_lfa_fp32_kernels(tdi, orc, dt, mc, n, fast, eq):
    """FP32-bulk LFA: the Taylor-table kernel (steps up to 40 s) and the
    per-output kernel used above it, both against the FP64 oracle, with the
    unequal time-dependent delays and with equal constant arms (eq = 1), TDI
    1.5 and 2.0 at stencil orders 2 and 4."""
    batch = _small_analytic(mc=mc, n=n, dt=dt, hybrid=False)
    orb = W.default_orbit()
    for gen, p in ((20, 4), (15, 2), (20, 2), (15, 4)):
        cfg = W.default_config(tdi_gen=gen, mode=1, taps=32, stencil_order=p, precision=1, equal_arms=eq)
        info = {}
        got = tdi.response(batch, cfg, orb, info=info)
        assert info["lfa_fast"] == fast
        ref = _run_orc(orc, batch, dict(cfg, precision=0), orb)
        err = _err(orc, got, ref)
        _report(f"lfa fp32 dt{dt:g} tdi{gen} p{p} eq{eq} fast{fast}", err, 1e-5)
        assert np.all(err <= 1e-5)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_ragged_batch_fp32_and_fp64(tdi, orc, mode):
    """Empty, single-sample, shorter-than-taps and multi-tile sources in one batch."""
    rng = np.random.default_rng(3)
    lens = [0, 1, 7, 31, 257, 1000, 4099, 0, 2600]
    parts = []
    for i, n in enumerate(lens):
        mc = 10 ** rng.uniform(5, 5.4)
        beta = math.asin(rng.uniform(-1, 1))
        if n < 64:
            # near the ecliptic pole |k.R|/c is a few seconds, so a few-sample source
            # still sees its own strain (elsewhere the SSB delay of up to 500 s moves
            # every read outside the data and both sides are exactly zero)
            beta = math.copysign(math.pi / 2 - 0.02, beta)
        rec, hp, hc, meta = W.make_source(mc, 0.7, beta, rng.uniform(0, 6.28),
                                          rng.uniform(0, 3.14), max(n, 1), 10.0, t0=1e6 * i)
        if n and mode == 2:
            rec["t_hyb"] = rec["t0"] + 0.6 * n * 10.0
        parts.append((rec, hp[:n], hc[:n], meta))
    batch = W._assemble(parts, np)
    orb = W.default_orbit()
    cfg = W.default_config(tdi_gen=20, mode=mode, taps=16, stencil_order=4)
    ref = _run_orc(orc, batch, cfg, orb)
    for prec in (0, 1):
        got = _run_gpu(tdi, batch, dict(cfg, precision=prec), orb)
        for i in range(batch.n_sources):
            a, b = batch.offsets[i], batch.offsets[i + 1]
            if b == a:
                continue
            # (a one-sample LFA output is exactly zero: odd-order central stencils
            # skip the centre and the neighbours are zero-extended)
            assert b - a < 7 or np.abs(ref[:, a:b]).max() > 0, "parity case without signal"
            if prec == 0:
                rec, hp, hc = batch.source(i)
                tol, _ = orc.fp64_tolerance(cfg, orb, rec, hp, hc, np.arange(b - a), ref[:, a:b])
            else:
                tol = np.full(3, 1e-5)
            err = _err(orc, got[:, a:b], ref[:, a:b])
            _report(f"ragged mode{mode} prec{prec} src{i} n={b - a}", err, tol)
            assert np.all(err <= tol)


def test_zero_strain_gives_zero(tdi):
    batch = _small_analytic(n=3000)
    batch.hp[:] = 0.0
    batch.hc[:] = 0.0
    for mode in (0, 1, 2):
        cfg = W.default_config(tdi_gen=20, mode=mode, taps=32)
        got = _run_gpu(tdi, batch, cfg, W.default_orbit())
        assert np.all(got == 0.0)


def test_graph_and_persistent_match_plain_launch(tdi, orc):
    batch = _small_analytic(mc=1.5e5, n=30000)
    orb = W.default_orbit()
    cfg = W.default_config(tdi_gen=20, mode=2, taps=32, precision=0)
    a = _run_gpu(tdi, batch, cfg, orb)
    b = _run_gpu(tdi, batch, cfg, orb, autotune=True, use_graph=True)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("graph", [False, True])
def test_untimed_runs_match_timed_runs(tdi, orc, graph):
    """tdi_plan_set_timing(0): the runs record no kernel events and give the
    same outputs, bit for bit, as timed runs; timing can be turned back on."""
    import torch
    batch = _small_analytic(n=30011, seed=17)
    orb = W.default_orbit()
    cfg = W.default_config(tdi_gen=20, mode=2, taps=32, stencil_order=4, precision=1)
    dev = torch.device("cuda:0")
    hp = torch.as_tensor(batch.hp, device=dev)
    hc = torch.as_tensor(batch.hc, device=dev)
    outs = [torch.empty(batch.total, dtype=torch.float32, device=dev) for _ in range(6)]
    src = tdi.make_sources(batch.sources)
    with tdi.Plan(cfg, orb, 1, batch.total, autotune=True, use_graph=graph) as plan:
        plan.run(src, batch.offsets, hp, hc, *outs[:3])
        assert plan.sync() == tdi.TDI_OK
        assert len(plan.kernel_times()) == 3
        plan.set_timing(False)
        for _ in range(3):
            plan.run(src, batch.offsets, hp, hc, *outs[3:])
        assert plan.sync() == tdi.TDI_OK
        assert len(plan.kernel_times()) == 0
        plan.set_timing(True)
        plan.run(src, batch.offsets, hp, hc, *outs[3:])
        assert plan.sync() == tdi.TDI_OK
        assert len(plan.kernel_times()) == 3
        # one source: fewer full-region tiles than compute units, so 16-output tiles
        assert plan.describe()["tile_full"] == 16
    for a, b in zip(outs[:3], outs[3:]):
        assert torch.equal(a, b)
    ref = _run_orc(orc, batch, cfg, orb)
    got = np.stack([o.double().cpu().numpy() for o in outs[3:]])
    err = _err(orc, got, ref)
    _report(f"untimed graph={graph}", err, 1e-5)
    assert np.all(err <= 1e-5)
