"""GPU parity with a sampled orbit (TABLE kind): eccentric Keplerian orbits
whose arms flex, sampled hourly, read by both sides through the same table.
Bars as for the analytic orbit: FP64 1e-12 (or the conditioning floor),
FP32-bulk 1e-5, per channel relative to its peak."""
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


def _orbit():
    t_lo, step = -2 * 86400.0, 3600.0
    return W.table_orbit(W.keplerian_orbit_table(t_lo, step, 24 * 40), t_lo, step)


def _batch():
    rng = np.random.default_rng(41)
    parts = []
    for n, t0 in ((7, 0.0), (3000, 5.0e4), (40000, 1.0e5)):
        beta = math.asin(rng.uniform(-1, 1))
        lam, psi, iota = rng.uniform(0, 2 * math.pi), rng.uniform(0, math.pi), math.acos(rng.uniform(-1, 1))
        parts.append(W.make_source(2.0e5, iota, beta, lam, psi, n, 10.0, t0))
    return W._assemble(parts, np)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_table_orbit_response(tdi, orc, mode, prec):
    batch, orb = _batch(), _orbit()
    cfg = W.default_config(tdi_gen=20, mode=mode, taps=32, stencil_order=4, precision=prec)
    got = tdi.response(batch, cfg, orb)
    ref = orc.response_batch(cfg, orb, batch)
    worst = 0.0
    for s in range(batch.n_sources):
        a, b = int(batch.offsets[s]), int(batch.offsets[s + 1])
        rec, hp, hc = batch.source(s)
        err = orc.peak_rel_err(got[:, a:b], ref[:, a:b])
        if prec == 0:
            ks = np.arange(b - a)
            tol, _ = orc.fp64_tolerance(cfg, orb, rec, hp, hc, ks, ref[:, a:b])
        else:
            tol = 1e-5
        assert np.all(err <= tol), (s, err, tol)
        worst = max(worst, float(np.max(err)))
    print(f"[parity] table orbit mode{mode} prec{prec}: max err {worst:.3e}", flush=True)


def test_table_orbit_links(tdi, orc):
    import torch
    batch, orb = _batch(), _orbit()
    cfg = W.default_config(tdi_gen=20, mode=2, taps=32, stencil_order=4, precision=0)
    hp = torch.as_tensor(np.asarray(batch.hp), dtype=torch.float64, device="cuda:0")
    hc = torch.as_tensor(np.asarray(batch.hc), dtype=torch.float64, device="cuda:0")
    with tdi.Plan(cfg, orb, batch.n_sources, batch.total) as p:
        y = p.run_links(batch.sources, batch.offsets, hp, hc).cpu().numpy()
        assert p.sync() == tdi.TDI_OK
    for s in range(batch.n_sources):
        a, b = int(batch.offsets[s]), int(batch.offsets[s + 1])
        ref = orc.link_outputs(cfg, orb, *batch.source(s))
        for l in range(6):
            assert np.max(np.abs(y[l, a:b] - ref[l])) <= 1e-12 * np.max(np.abs(ref[l]))


def test_table_orbit_coverage_is_checked(tdi):
    import torch
    batch, orb = _batch(), _orbit()
    late = batch.sources.copy()
    late["t0"][2] = 39 * 86400.0            # runs past the end of the table
    cfg = W.default_config(tdi_gen=20, mode=0, taps=32, stencil_order=4, precision=0)
    hp = torch.as_tensor(np.asarray(batch.hp), dtype=torch.float64, device="cuda:0")
    hc = torch.as_tensor(np.asarray(batch.hc), dtype=torch.float64, device="cuda:0")
    with tdi.Plan(cfg, orb, batch.n_sources, batch.total) as p:
        with pytest.raises(tdi.TdiError) as e:
            p.run(late, batch.offsets, hp, hc)
        assert e.value.status == tdi.TDI_ERANGE
