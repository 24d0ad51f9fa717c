"""Autotune cache (TDI_AUTOTUNE_CACHE): the first autotuned plan appends its
decision as one JSON line, a second plan with the same key takes that launch
without timing and produces the same outputs, lines that do not parse are
skipped, and a different option (the tap count) misses and appends a line."""
import json
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


def _batch():
    rng = np.random.default_rng(31)
    parts = [W.make_source(10 ** rng.uniform(5, 5.4), 0.7, math.asin(rng.uniform(-1, 1)), rng.uniform(0, 6.28),
                           rng.uniform(0, 3.14), n, 10.0, 0.0) for n in (5000, 23000, 60000)]
    parts.append(W.make_source(2.0e5, 0.5, 0.3, 2.0, 1.0, 100000, 10.0, 0.0))   # through its switch
    return W._assemble(parts, np)


def test_autotune_cache_round_trip(tdi, tmp_path, monkeypatch):
    path = tmp_path / "tune.jsonl"
    path.write_text('not a record\n{"key": "x", "grid_lfa": 1}\n')
    monkeypatch.setenv("TDI_AUTOTUNE_CACHE", str(path))
    batch, orb = _batch(), W.default_orbit()
    cfg = W.default_config(tdi_gen=20, mode=2, taps=32, stencil_order=4, precision=1)

    first = {}
    y1 = tdi.response(batch, cfg, orb, autotune=True, use_graph=True, info=first)
    assert first["tuned"] == 1 and first["tune_cache"] == 0, first
    lines = path.read_text().splitlines()
    assert len(lines) == 3, lines
    rec = json.loads(lines[-1])
    assert rec["key"].startswith("gfx950"), rec
    assert (rec["grid_lfa"], rec["grid_full"]) == (first["grid_lfa"], first["grid_full"]), (rec, first)
    assert rec["chunks"] * 2304 == first["tile_lfa"] and rec["stream"] == 1 - first["graph"], (rec, first)

    second = {}
    y2 = tdi.response(batch, cfg, orb, autotune=True, use_graph=True, info=second)
    assert second["tuned"] == 1 and second["tune_cache"] == 1, second
    for k in ("tile_lfa", "grid_lfa", "grid_full", "graph"):
        assert second[k] == first[k], (k, first, second)
    assert np.array_equal(y1, y2)
    assert len(path.read_text().splitlines()) == 3

    other = {}
    tdi.response(batch, dict(cfg, taps=16), orb, autotune=True, use_graph=True, info=other)
    assert other["tune_cache"] == 0, other
    lines = path.read_text().splitlines()
    assert len(lines) == 4 and ",taps=16," in json.loads(lines[-1])["key"], lines[-1]
    print(f"[autotune cache] {rec['key']}: grid_lfa {rec['grid_lfa']} grid_full {rec['grid_full']} "
          f"chunks {rec['chunks']} stream {rec['stream']}", flush=True)
