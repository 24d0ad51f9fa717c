"""Pins of the oracle's A, E, T channels, noise PSDs and inner product.

Each check is fixed by the paper's statements or by mathematics, not by the
oracle's own formulas: an explicit DFT sum, Parseval's theorem, the closed form
for an on-bin sinusoid, the orthonormality of the A, E, T map, the vanishing T
of the equal-arm LFA, and the low-frequency power laws and TDI-generation ratio
the paper states for the PSDs.  The absolute PSD level has no printed value to
pin against (parity unpinned for it; only its structure is pinned).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import noise as NZ

L_ARM = 2.5e9


def _flat(f):
    return np.ones_like(np.asarray(f, dtype=np.float64))


def test_fourier_matches_explicit_dft():
    rng = np.random.default_rng(3)
    n, dt = 11, 7.5
    x = rng.standard_normal(n)
    N = NZ.fft_length(n)
    assert N == 16
    got = NZ.fourier(x, N, dt)
    for k in range(N):
        ref = sum(x[j] * complex(math.cos(-2 * math.pi * j * k / N), math.sin(-2 * math.pi * j * k / N))
                  for j in range(n)) * dt
        assert abs(got[k] - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("n,N", [(1, 2), (2, 2), (3, 4), (1024, 1024), (1025, 2048)])
def test_fft_length(n, N):
    assert NZ.fft_length(n) == N


def test_parseval_one_sided():
    # no DC and no Nyquist content: the one-sided sum carries all the power
    N, dt = 64, 3.0
    t = np.arange(N) * dt
    x = 0.7 * np.cos(2 * math.pi * 3 * t / (N * dt)) + 1.3 * np.sin(2 * math.pi * 17 * t / (N * dt) + 0.4)
    got = NZ.inner(x, x, dt, _flat, 0.0, 1.0)
    assert abs(got - 2.0 * dt * np.sum(x * x)) <= 1e-12 * got


def test_on_bin_sinusoid_closed_form():
    N, dt, k0, a = 4096, 5.0, 301, 2.5
    f0 = k0 / (N * dt)
    t = np.arange(N) * dt
    x = a * np.cos(2 * math.pi * f0 * t + 0.3)
    S = NZ.psd_ae(f0, L_ARM, 20)
    got = NZ.inner(x, x, dt, lambda f: NZ.psd_ae(f, L_ARM, 20), 1e-5, 0.1)
    assert abs(got - a * a * N * dt / S) <= 1e-10 * got
    # quadrature partner: orthogonal under the inner product
    y = a * np.sin(2 * math.pi * f0 * t + 0.3)
    assert abs(NZ.inner(x, y, dt, lambda f: NZ.psd_ae(f, L_ARM, 20), 1e-5, 0.1)) <= 1e-10 * got


def test_inner_product_bilinear_symmetric_and_band():
    rng = np.random.default_rng(5)
    n, dt = 3000, 10.0
    x, y, z = rng.standard_normal((3, n))
    psd = lambda f: NZ.psd_t(f, L_ARM, 15)  # noqa: E731
    ip = lambda a, b: NZ.inner(a, b, dt, psd, 1e-4, 0.03)  # noqa: E731
    assert abs(ip(x, y) - ip(y, x)) <= 1e-12 * abs(ip(x, x))
    assert abs(ip(2 * x + z, y) - (2 * ip(x, y) + ip(z, y))) <= 1e-10 * ip(x, x)
    assert ip(x, y) ** 2 <= ip(x, x) * ip(y, y)
    # an empty band gives zero
    assert NZ.inner(x, y, dt, psd, 0.2, 0.3) == 0.0


def test_aet_orthonormal():
    rng = np.random.default_rng(1)
    X, Y, Z = rng.standard_normal((3, 50))
    A, E, T = NZ.aet(X, Y, Z)
    assert np.allclose(A * A + E * E + T * T, X * X + Y * Y + Z * Z, rtol=1e-13)
    M = np.array([NZ.aet(*np.eye(3)[:, i]) for i in range(3)]).T
    assert np.allclose(M @ M.T, np.eye(3), atol=1e-15)


def test_t_vanishes_for_equal_arm_lfa():
    """Equal-arm LFA: every channel reads link l at the same retarded time with
    the same prefactor, so X + Y + Z cancels and T carries no signal."""
    import oracle as O
    from paper_2505_09600_amd import workload as W
    n, dt = 3000, 10.0
    rec, hp, hc, _ = W.make_source(3e6, 0.7, 0.4, 1.1, 0.3, n, dt, 0.0, hybrid=False)
    cfg = W.default_config(tdi_gen=20, mode=1, taps=16, stencil_order=4, equal_arms=1)
    orb = W.default_orbit(W.ORBIT_FROZEN)
    X, Y, Z = O.response(cfg, orb, rec, hp, hc)
    A, E, T = NZ.aet(X, Y, Z)
    assert np.max(np.abs(A)) > 0
    assert np.max(np.abs(T)) <= 1e-12 * max(np.max(np.abs(A)), np.max(np.abs(E)))


def test_psd_tdi_generation_ratio():
    f = np.logspace(-5, -1, 200)
    x = 2 * math.pi * f * L_ARM / NZ.C_LIGHT
    for gal in (False, True):
        r_ae = NZ.psd_ae(f, L_ARM, 20, gal) / NZ.psd_ae(f, L_ARM, 15, gal)
        r_t = NZ.psd_t(f, L_ARM, 20, gal) / NZ.psd_t(f, L_ARM, 15, gal)
        assert np.allclose(r_ae, 4 * np.sin(2 * x) ** 2, rtol=1e-12)
        assert np.allclose(r_t, 4 * np.sin(2 * x) ** 2, rtol=1e-12)


def _slope(fun, f, h=1e-3):
    return (math.log(fun(f * (1 + h))) - math.log(fun(f * (1 - h)))) / (math.log(1 + h) - math.log(1 - h))


def test_psd_low_frequency_power_laws():
    """Sec. II.C: without the foreground, S_AE ~ f^-2 (TDI 1.5) and ~ f^0
    (TDI 2.0) at low frequency; the two differ by f^2."""
    f = 1e-6
    s15 = _slope(lambda v: float(NZ.psd_ae(v, L_ARM, 15, False)), f)
    s20 = _slope(lambda v: float(NZ.psd_ae(v, L_ARM, 20, False)), f)
    assert abs(s15 + 2.0) < 1e-3
    assert abs(s20) < 1e-3


def test_galactic_foreground_shape():
    f1, fk = NZ.gal_knees(1.0)
    assert 1e-4 < fk < 1e-2 and 1e-4 < f1 < 1e-2
    # the foreground switches off well above the knee and adds power below it
    hi = 0.05
    assert NZ.s_gal(hi, L_ARM) < 1e-6 * NZ.psd_ae(hi, L_ARM, 15, False)
    lo = 1e-3
    assert NZ.psd_ae(lo, L_ARM, 15, True) > NZ.psd_ae(lo, L_ARM, 15, False)
    assert np.all(NZ.s_gal(np.logspace(-5, -1, 50), L_ARM) >= 0)


def test_log_likelihood_of_identical_signals_is_zero():
    rng = np.random.default_rng(9)
    d = rng.standard_normal((3, 2000))
    noise = dict(L_m=L_ARM, tdi_gen=20, galactic=1, T_obs_years=1.0, f_min=1e-4, f_max=0.04)
    ip = NZ.inner_products(d, d, 5.0, noise)
    assert abs(NZ.log_likelihood(ip)) <= 1e-12 * np.sum(ip[:, 0])
    # and equals -1/2 <d-h|d-h> summed over channels
    h = 0.9 * d + 0.1 * rng.standard_normal((3, 2000))
    ip = NZ.inner_products(d, h, 5.0, noise)
    direct = NZ.inner_products(d - h, d - h, 5.0, noise)[:, 0].sum()
    assert abs(NZ.log_likelihood(ip) + 0.5 * direct) <= 1e-9 * abs(direct)
