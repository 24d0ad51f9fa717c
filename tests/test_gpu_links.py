"""GPU parity of the single-link outputs (tdi_run_links through the C ABI)
against the FP64 oracle, per link: max |GPU - oracle| / max |oracle|.

Bars: 1e-12 (FP64) and 1e-5 (FP32-bulk).  The links of these sources are
conditioned far better than the TDI combinations (a single difference of H at
two times, and omega L/c >~ 0.05 where a link peaks), so the response's FP64
bar holds without a conditioning allowance.
"""
import math

import numpy as np
import pytest

from paper_2505_09600_amd import workload as W

pytestmark = pytest.mark.gpu
TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def tdi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2505_09600_amd import tdi as T
    T.lib()
    return T


def _gpu_links(T, batch, cfg, orb):
    import torch
    hp = torch.as_tensor(np.asarray(batch.hp), dtype=torch.float64, device="cuda:0")
    hc = torch.as_tensor(np.asarray(batch.hc), dtype=torch.float64, device="cuda:0")
    with T.Plan(cfg, orb, max(1, batch.n_sources), max(1, batch.total)) as p:
        y = p.run_links(batch.sources, batch.offsets, hp, hc)
        st = p.sync()
        assert st == T.TDI_OK, T.tdi_status_str(st)
        return y.double().cpu().numpy()


def _check(orc, name, batch, cfg, orb, got, tol):
    worst = 0.0
    for s in range(batch.n_sources):
        a, b = int(batch.offsets[s]), int(batch.offsets[s + 1])
        rec, hp, hc = batch.source(s)
        ref = orc.link_outputs(cfg, orb, rec, hp, hc)
        for l in range(6):
            peak = np.max(np.abs(ref[l])) if b > a else 0.0
            err = np.max(np.abs(got[l, a:b] - ref[l])) if b > a else 0.0
            rel = err / peak if peak > 0 else err
            worst = max(worst, rel)
            assert rel <= tol, (name, s, b - a, l, rel)
    print(f"[parity] {name}: max err over links {worst:.3e}  tol {tol:.0e}", flush=True)


def _ragged():
    rng = np.random.default_rng(31)
    parts = []
    for i, n in enumerate((1, 7, 300, 5000, 23000)):
        beta = 1.45 if i < 2 else math.asin(rng.uniform(-1, 1))
        lam, psi, iota = rng.uniform(0, 2 * math.pi), rng.uniform(0, math.pi), math.acos(rng.uniform(-1, 1))
        parts.append(W.make_source(2.0e5, iota, beta, lam, psi, n, 10.0, 0.0))
    return W._assemble(parts, np)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_links_ragged(tdi, orc, mode, prec):
    batch = _ragged()
    cfg = W.default_config(tdi_gen=20, mode=mode, taps=32, stencil_order=4, precision=prec)
    orb = W.default_orbit()
    got = _gpu_links(tdi, batch, cfg, orb)
    _check(orc, f"links ragged mode{mode} prec{prec}", batch, cfg, orb, got, TOL[prec])


@pytest.mark.parametrize("prec", [0, 1])
def test_links_lfa_variants(tdi, orc, prec):
    """Second-order stencil, equal arms, 16 taps, frozen constellation."""
    batch = _ragged()
    orb = W.default_orbit(W.ORBIT_FROZEN, t_freeze=1.0e6)
    cfg = W.default_config(tdi_gen=15, mode=1, taps=16, stencil_order=2, equal_arms=1, precision=prec)
    got = _gpu_links(tdi, batch, cfg, orb)
    _check(orc, f"links lfa p2 equal-arms N16 prec{prec}", batch, cfg, orb, got, TOL[prec])


@pytest.mark.parametrize("prec", [0, 1])
def test_links_hybrid_long_source(tdi, orc, prec):
    """One 1e6-sample hybrid source (3906 tiles) through its switch."""
    n = 1_000_000
    rec, hp, hc, _ = W.make_source(2.0e5, 0.7, 0.2, 4.0, 1.0, n, 10.0, 0.0)
    assert math.isfinite(rec["t_hyb"])
    batch = W._assemble([(rec, hp, hc, {})], np)
    cfg = W.default_config(tdi_gen=20, mode=2, taps=32, stencil_order=4, precision=prec)
    orb = W.default_orbit()
    got = _gpu_links(tdi, batch, cfg, orb)
    _check(orc, f"links hybrid n=1e6 prec{prec}", batch, cfg, orb, got, TOL[prec])


def test_links_between_graph_replays(tdi, orc):
    """A link-output run between two graph-replayed responses on one plan
    leaves the response unchanged (both runs share the parameter block)."""
    import torch
    batch = _ragged()
    cfg = W.default_config(tdi_gen=20, mode=2, taps=32, stencil_order=4, precision=1)
    orb = W.default_orbit()
    hp = torch.as_tensor(np.asarray(batch.hp), dtype=torch.float64, device="cuda:0")
    hc = torch.as_tensor(np.asarray(batch.hc), dtype=torch.float64, device="cuda:0")
    with tdi.Plan(cfg, orb, batch.n_sources, batch.total, autotune=False, use_graph=True) as p:
        first = [v.clone() for v in p.run(batch.sources, batch.offsets, hp, hc)]
        y = p.run_links(batch.sources, batch.offsets, hp, hc)
        second = p.run(batch.sources, batch.offsets, hp, hc)
        assert p.sync() == tdi.TDI_OK
        for a, b in zip(first, second):
            assert torch.equal(a, b)
        ref = orc.link_outputs(cfg, orb, *batch.source(4))
        a, b = int(batch.offsets[4]), int(batch.offsets[5])
        got = y[:, a:b].double().cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mode", [1, 2])
def test_links_next_term(tdi, orc, mode, prec):
    """The optional m = 1 term of the single-link LFA (lfa_terms = 2)."""
    batch = _ragged()
    cfg = W.default_config(tdi_gen=20, mode=mode, taps=32, stencil_order=4, precision=prec)
    cfg["lfa_terms"] = 2
    orb = W.default_orbit()
    got = _gpu_links(tdi, batch, cfg, orb)
    _check(orc, f"links lfa two terms mode{mode} prec{prec}", batch, cfg, orb, got, TOL[prec])
