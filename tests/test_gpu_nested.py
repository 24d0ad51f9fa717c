"""GPU parity of the time-nested stage-2 delays (tdi_config.nested_delays = 1)
against the oracle's nested form: the analytic orbit and flexing Keplerian
orbits read from a table, full and hybrid modes, TDI 1.5 and 2.0.  Bars:
FP64 1e-12 (or the conditioning floor) and FP32-bulk 1e-5, per channel
relative to its peak.  In FP64 the nested result must also stand apart from
the non-nested oracle by more than ten times the bar (on both orbits), so the
comparison tells the two forms apart."""
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


def _orbit(table):
    if not table:
        return W.default_orbit()
    t_lo, step = -2 * 86400.0, 3600.0
    return W.table_orbit(W.keplerian_orbit_table(t_lo, step, 24 * 40), t_lo, step)


def _batch():
    rng = np.random.default_rng(43)
    parts = []
    for n, t0 in ((9, 0.0), (3000, 5.0e4), (40000, 1.0e5)):
        beta = math.asin(rng.uniform(-1, 1))
        lam, psi, iota = rng.uniform(0, 2 * math.pi), rng.uniform(0, math.pi), math.acos(rng.uniform(-1, 1))
        parts.append(W.make_source(2.0e5, iota, beta, lam, psi, n, 10.0, t0))
    return W._assemble(parts, np)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("gen", [15, 20])
@pytest.mark.parametrize("table", [False, True])
def test_nested_response(tdi, orc, table, gen, mode, prec):
    batch, orb = _batch(), _orbit(table)
    cfg = W.default_config(tdi_gen=gen, mode=mode, taps=32, stencil_order=4, precision=prec,
                           nested_delays=1)
    got = tdi.response(batch, cfg, orb)
    ref = orc.response_batch(cfg, orb, batch)
    flat = orc.response_batch(dict(cfg, nested_delays=0), orb, batch) if prec == 0 else None
    worst, apart = 0.0, 0.0
    for s in range(batch.n_sources):
        a, b = int(batch.offsets[s]), int(batch.offsets[s + 1])
        rec, hp, hc = batch.source(s)
        err = orc.peak_rel_err(got[:, a:b], ref[:, a:b])
        if prec == 0:
            ks = np.arange(b - a)
            tol, _ = orc.fp64_tolerance(cfg, orb, rec, hp, hc, ks, ref[:, a:b])
            apart = max(apart, float(np.max(orc.peak_rel_err(got[:, a:b], flat[:, a:b]) / tol)))
        else:
            tol = 1e-5
        assert np.all(err <= tol), (s, err, tol)
        worst = max(worst, float(np.max(err)))
    print(f"[parity] nested table={table} gen{gen} mode{mode} prec{prec}: max err {worst:.3e}"
          + (f", non-nested oracle at {apart:.1f}x the bar" if prec == 0 else ""), flush=True)
    if prec == 0:
        assert apart > 10.0

