"""Tile shapes of the FP32-bulk LFA path (tdi_config.fast_tile_chunks): tiles of
one, two and four chunks of 2304 outputs each meet the FP32 bar against the
FP64 oracle and agree with one another; the autotuner picks one of them.
Lengths straddle the chunk and tile boundaries."""
import math

import numpy as np
import pytest

from paper_2505_09600_amd import workload as W

pytestmark = pytest.mark.gpu
CHUNK = 2304


@pytest.fixture(scope="module")
def tdi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2505_09600_amd import tdi as T
    T.lib()
    return T


def _batch():
    rng = np.random.default_rng(23)
    lens = [1, 700, CHUNK, CHUNK + 1, 2 * CHUNK, 2 * CHUNK + 1, 4 * CHUNK, 4 * CHUNK + 1, 30000]
    parts = []
    for n in lens:
        beta = math.asin(rng.uniform(-1, 1))
        if n < 64:
            beta = math.copysign(math.pi / 2 - 0.02, beta)
        parts.append(W.make_source(10 ** rng.uniform(5, 5.4), 0.7, beta, rng.uniform(0, 6.28),
                                   rng.uniform(0, 3.14), n, 10.0, 0.0))
    # one longer source through its switch (hybrid) or its ringdown (LFA)
    parts.append(W.make_source(2.0e5, 0.5, 0.3, 2.0, 1.0, 100000, 10.0, 0.0))
    return W._assemble(parts, np)


@pytest.mark.parametrize("mode,gen,p", [(2, 20, 4), (1, 20, 4), (2, 15, 2)])
def test_tile_shapes_match_oracle_and_each_other(tdi, orc, mode, gen, p):
    batch, orb = _batch(), W.default_orbit()
    base = W.default_config(tdi_gen=gen, mode=mode, taps=32, stencil_order=p, precision=1)
    ref = orc.response_batch(dict(base, precision=0), orb, batch)
    outs = {}
    for ch in (1, 2, 4):
        info = {}
        got = tdi.response(batch, dict(base, fast_tile_chunks=ch), orb, info=info)
        assert info["lfa_fast"] == 1 and info["tile_lfa"] == ch * CHUNK, info
        worst = 0.0
        for s in range(batch.n_sources):
            a, b = int(batch.offsets[s]), int(batch.offsets[s + 1])
            err = orc.peak_rel_err(got[:, a:b], ref[:, a:b])
            assert np.all(err <= 1e-5), (ch, s, b - a, err)
            worst = max(worst, float(np.max(err)))
        outs[ch] = got
        print(f"[parity] tiles of {ch} chunks mode{mode} tdi{gen}: max err {worst:.3e}", flush=True)
    for ch in (1, 2):
        for s in range(batch.n_sources):
            a, b = int(batch.offsets[s]), int(batch.offsets[s + 1])
            peak = np.max(np.abs(ref[:, a:b]), axis=1)
            d = np.max(np.abs(outs[ch][:, a:b] - outs[4][:, a:b]), axis=1)
            assert np.all(d <= 2e-6 * np.where(peak > 0, peak, 1.0)), (ch, s, d / peak)


def test_autotuner_picks_a_tile_shape(tdi, orc):
    """A single long source: the autotuner times every tile shape with the
    persistent grids and keeps one; the graph-replayed result meets the bar."""
    rec, hp, hc, _ = W.make_source(2.0e5, 0.9, -0.4, 4.0, 0.3, 300000, 10.0, 0.0)
    batch, orb = W._assemble([(rec, hp, hc, {})], np), W.default_orbit()
    cfg = W.default_config(tdi_gen=20, mode=2, taps=32, stencil_order=4, precision=1)
    info = {}
    got = tdi.response(batch, cfg, orb, autotune=True, use_graph=True, info=info)
    assert info["tuned"] == 1 and info["tile_lfa"] in (CHUNK, 2 * CHUNK, 4 * CHUNK), info
    ks = np.unique(np.linspace(0, batch.total - 1, 4000).astype(np.int64))
    ref = orc.response_at(dict(cfg, precision=0), orb, rec, hp, hc, ks)
    err = orc.peak_rel_err(got[:, ks], ref)
    print(f"[parity] autotuned tile {info['tile_lfa']}: err {np.max(err):.3e}", flush=True)
    assert np.all(err <= 1e-5)
