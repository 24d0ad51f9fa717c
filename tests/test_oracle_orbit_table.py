"""Pins of the sampled-orbit (TABLE) geometry in the oracle.

- a table sampled from the analytic orbit reproduces the analytic response
  (8-point interpolation in time is exact to rounding at hour spacing);
- the Keplerian stand-in for orbit files agrees with the rigid first-order
  orbit to first order in e (its positions differ at O(e^2 R)) and its arms
  flex: the light times differ between links and drift in time.
"""
import math

import numpy as np
import pytest

from paper_2505_09600_amd import workload as W

C_LIGHT = 299792458.0


def _analytic_table(orc, orb, t0, dt, n):
    return np.array([orc.positions(orb, t0 + j * dt) for j in range(n)])


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_table_of_the_analytic_orbit_reproduces_it(orc, mode):
    orb = W.default_orbit()
    n, dt = 4000, 10.0
    rec, hp, hc, _ = W.make_source(2.0e5, 0.9, 0.3, 2.2, 0.7, n, dt, 1.0e5)
    t_lo, step = 1.0e5 - 86400.0, 1800.0
    tab = _analytic_table(orc, orb, t_lo, step, 200)
    torb = W.table_orbit(tab, t_lo, step)
    cfg = W.default_config(tdi_gen=20, mode=mode, taps=32, stencil_order=4)
    ref = np.array(orc.response(cfg, orb, rec, hp, hc))
    got = np.array(orc.response(cfg, torb, rec, hp, hc))
    err = np.max(np.abs(got - ref), axis=1) / np.max(np.abs(ref), axis=1)
    assert np.all(err < 1e-11), err


def test_keplerian_table_agrees_to_first_order(orc):
    orb = W.default_orbit()
    e = W.ARM_L / (2.0 * math.sqrt(3.0) * W.AU)
    tab = W.keplerian_orbit_table(0.0, 86400.0, 366)
    d = max(np.max(np.abs(tab[j] - orc.positions(orb, j * 86400.0))) for j in range(0, 366, 5))
    assert 0.5 * e * e * W.AU < d < 5.0 * e * e * W.AU


def test_keplerian_arms_flex(orc):
    step = 3600.0
    tab = W.keplerian_orbit_table(-86400.0, step, 24 * 400)
    torb = W.table_orbit(tab, -86400.0, step)
    ts = np.linspace(0.0, 3.0e7, 13)
    T = np.array([[orc.light_time(torb, l, t) for l in (1, 2, 3, -1, -2, -3)] for t in ts])
    rel = T * C_LIGHT / W.ARM_L - 1.0
    assert 1e-4 < np.max(np.abs(rel)) < 1e-2          # the arms flex at O(e) of L
    assert np.max(np.ptp(rel, axis=0)) > 1e-4          # and breathe over the year
    assert np.max(np.abs(T[:, :3] - T[:, 3:])) > 1e-9  # L_l != L_-l
