"""The seeded input generators (no response arithmetic): shapes, seeds, switch times."""
import math

import numpy as np

from paper_2505_09600_amd import workload as W


def test_c1_shape_and_frequency_range():
    batch, cfg, orb = W.config_c1()
    assert batch.n_sources == 1 and batch.total == 2 ** 14
    assert orb["kind"] == W.ORBIT_FROZEN and cfg["tdi_gen"] == 15 and cfg["taps"] == 16
    rec = batch.sources[0]
    t = rec["t0"] + np.arange(batch.total) * rec["dt"]
    _, _, f = W.chirp_series(t, 3e5, math.pi / 3, batch.meta[0]["t_c"], with_cut=False)
    assert abs(f[0] - 8.06e-4) / 8.06e-4 < 0.01
    assert abs(f[-1] - 2.64e-3) / 2.64e-3 < 0.01
    assert np.abs(batch.hp).max() <= 1.0 + 1e-12


def test_seeded_reproducibility_and_subsets():
    a = W.config_c4(n_sources=16, n_lo=2 ** 10, n_hi=2 ** 12)[0]
    b = W.config_c4(n_sources=16, n_lo=2 ** 10, n_hi=2 ** 12)[0]
    assert np.array_equal(a.hp, b.hp) and np.array_equal(a.offsets, b.offsets)
    sub = W.config_c4(n_sources=16, n_lo=2 ** 10, n_hi=2 ** 12, only=[3, 7])[0]
    for j, i in enumerate([3, 7]):
        ra, hpa, _ = a.source(i)
        rs, hps, _ = sub.source(j)
        assert np.array_equal(hpa, hps) and ra == rs


def test_c4_length_distribution():
    mc, beta, lam, psi, iota, n, e0 = W.draw_sources(1004, 512, 2 ** 18, 2 ** 22)
    assert n.min() >= 2 ** 18 and n.max() <= 2 ** 22
    assert 1.2e6 < n.mean() < 1.65e6
    assert np.all(np.abs(beta) <= math.pi / 2) and np.all((mc >= 1e5) & (mc <= 1e7))


def test_switch_time_matches_frequency_threshold():
    rec, hp, hc, meta = W.make_source(1.2e5, 0.5, 0.1, 0.2, 0.3, 40000, 10.0)
    assert math.isfinite(rec["t_hyb"])
    t = np.arange(40000) * 10.0
    _, _, f = W.chirp_series(t, 1.2e5, 0.5, meta["t_c"])
    k = int(round(rec["t_hyb"] / 10.0))
    f_sw = 0.05 * W.C_LIGHT / W.ARM_L
    assert f[k] >= f_sw and (k == 0 or f[k - 1] < f_sw)
    heavy, _, _, _ = W.make_source(5e6, 0.5, 0.1, 0.2, 0.3, 40000, 10.0)
    assert heavy["t_hyb"] == math.inf


def test_ringdown_is_continuous():
    mc, dt = 2e5, 10.0
    rec, hp, hc, meta = W.make_source(mc, 0.0, 0.1, 0.2, 0.0, 30000, dt)
    assert np.all(np.isfinite(hp)) and np.all(np.isfinite(hc))
    jumps = np.abs(np.diff(hp))
    assert jumps.max() < 1.0


def test_eccentric_modulation_changes_waveform():
    a = W.make_source(3e5, 0.4, 0.1, 0.2, 0.3, 5000, 5.0, e0=0.0)[1]
    b = W.make_source(3e5, 0.4, 0.1, 0.2, 0.3, 5000, 5.0, e0=0.2)[1]
    assert np.abs(a - b).max() > 1e-3
