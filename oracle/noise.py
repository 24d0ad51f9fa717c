"""FP64 oracle of the likelihood steps that follow the response.

TEST INFRASTRUCTURE ONLY: the slow, plain statement of the A, E, T channels,
the analytic noise PSDs and the noise-weighted inner product, used to check
the HIP library.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg import this module; the library never does.

Each function states the passage it follows.  The Fourier transform is the
library FFT of NumPy (a plain DFT, checked against an explicit sum in the
tests); nothing else is taken from a library.

Readings where the paper is silent (stated once, here and in the design notes):
- the continuous transform of Eq. (defFT) is approximated by dt times the DFT
  of the series zero-extended to the next power of two, N = max(2, 2^ceil(log2 n));
  zero extension matches the response's own convention outside [0, n-1];
- the integral of Eq. (scalar_product) is the sum over the one-sided DFT bins
  0 < f_k < 1/(2 dt) with f_min <= f_k <= f_max, times df = 1/(N dt); the DC and
  Nyquist bins are left out;
- T_obs in Eq. (sgal)'s f1 and f_knee relations is in years.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299792458.0

# Sec. II.C (noise model): acceleration and optical-metrology amplitudes
SQRT_S_ACC = 2.4e-15          # m s^-2 Hz^-1/2
SQRT_S_OMS = 7.9e-12          # m Hz^-1/2
# Eq. (sgal) and the f1 / f_knee relations that follow it
GAL_A = 1.28265531e-44
GAL_ALPHA = 1.62966700
GAL_F2 = 4.81078093e-4        # Hz
GAL_A1, GAL_B1 = -0.223499956, -2.70408439
GAL_AK, GAL_BK = -0.360976122, -2.37822436


def aet(X, Y, Z):
    """A, E, T defined at the end of Sec. II.B: A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6, T = (X + Y + Z)/sqrt3."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    A = (Z - X) / math.sqrt(2.0)
    E = (X - 2.0 * Y + Z) / math.sqrt(6.0)
    T = (X + Y + Z) / math.sqrt(3.0)
    return A, E, T


def s_pm(f):
    """Proof-mass noise of Sec. II.C (fractional-frequency units)."""
    f = np.asarray(f, dtype=np.float64)
    return (SQRT_S_ACC ** 2) * (2.0 * math.pi * f * C_LIGHT) ** -2 \
        * (1.0 + (4.0e-4 / f) ** 2) * (1.0 + (f / 8.0e-3) ** 4)


def s_op(f):
    """Optical-path noise of Sec. II.C (fractional-frequency units)."""
    f = np.asarray(f, dtype=np.float64)
    return (SQRT_S_OMS ** 2) * (2.0 * math.pi * f / C_LIGHT) ** 2 * (1.0 + (2.0e-3 / f) ** 4)


def gal_knees(T_obs_years: float):
    """(f1, f_knee) of the galactic foreground for an observation time in years."""
    lt = math.log10(T_obs_years)
    return 10.0 ** (GAL_A1 * lt + GAL_B1), 10.0 ** (GAL_AK * lt + GAL_BK)


def s_gal(f, L_m: float, T_obs_years: float = 1.0):
    """Galactic foreground, Eq. (sgal), with x = 2 pi f L / c."""
    f = np.asarray(f, dtype=np.float64)
    f1, fk = gal_knees(T_obs_years)
    x = 2.0 * math.pi * f * L_m / C_LIGHT
    return 2.0 * x ** 2 * np.sin(x) ** 2 * GAL_A * f ** (-7.0 / 3.0) \
        * np.exp(-(f / f1) ** GAL_ALPHA) * (1.0 + np.tanh((fk - f) / GAL_F2))


def tdi_lambda(f, L_m: float, tdi_gen: int):
    """Lambda(f) of Eqs. (SnAE), (SnT): 4 sin^2(2x) for TDI 2.0, 1 for TDI 1.5."""
    f = np.asarray(f, dtype=np.float64)
    if tdi_gen == 15:
        return np.ones_like(f)
    x = 2.0 * math.pi * f * L_m / C_LIGHT
    return 4.0 * np.sin(2.0 * x) ** 2


def psd_ae(f, L_m: float, tdi_gen: int, galactic: bool = True, T_obs_years: float = 1.0):
    """Single-sided PSD of A and E, Eq. (SnAE)."""
    f = np.asarray(f, dtype=np.float64)
    x = 2.0 * math.pi * f * L_m / C_LIGHT
    lam = tdi_lambda(f, L_m, tdi_gen)
    inst = 8.0 * lam * np.sin(x) ** 2 * (
        2.0 * (3.0 + 2.0 * np.cos(x) + np.cos(2.0 * x)) * s_pm(f) + (2.0 + np.cos(x)) * s_op(f))
    if galactic:
        inst = inst + 1.5 * lam * s_gal(f, L_m, T_obs_years)
    return inst


def psd_t(f, L_m: float, tdi_gen: int, galactic: bool = True, T_obs_years: float = 1.0):
    """Single-sided PSD of T, Eq. (SnT)."""
    f = np.asarray(f, dtype=np.float64)
    x = 2.0 * math.pi * f * L_m / C_LIGHT
    lam = tdi_lambda(f, L_m, tdi_gen)
    inst = 16.0 * lam * np.sin(x) ** 2 * (
        (1.0 - np.cos(x)) * s_op(f) + 8.0 * np.sin(x / 2.0) ** 4 * s_pm(f))
    if galactic:
        inst = inst + lam * s_gal(f, L_m, T_obs_years)
    return inst


def fft_length(n: int) -> int:
    """Zero-extended transform length: the next power of two, at least 2."""
    N = 2
    while N < n:
        N *= 2
    return N


def band_bins(N: int, dt: float, f_min: float, f_max: float):
    """Indices k of the one-sided bins used by the inner product."""
    k = np.arange(1, N // 2, dtype=np.int64)
    f = k / (N * dt)
    return k[(f >= f_min) & (f <= f_max)]


def fourier(x, N: int, dt: float):
    """dt times the DFT of x zero-extended to N samples: the discrete form of
    Eq. (defFT), e^{-2 pi i f t} with t measured from the first sample."""
    z = np.zeros(N, dtype=np.float64)
    z[:len(x)] = x
    return dt * np.fft.fft(z)


def inner(x, y, dt: float, psd, f_min: float, f_max: float):
    """<x|y> of Eq. (scalar_product) for one channel; psd is a callable S_n(f)."""
    n = max(len(x), len(y))
    N = fft_length(n)
    k = band_bins(N, dt, f_min, f_max)
    if k.size == 0:
        return 0.0
    xt = fourier(x, N, dt)[k]
    yt = fourier(y, N, dt)[k]
    f = k / (N * dt)
    df = 1.0 / (N * dt)
    return float(4.0 * np.sum(np.real(np.conj(xt) * yt) / psd(f)) * df)


def channel_psds(noise: dict):
    """(S_A = S_E, S_T) callables for a noise description with keys
    tdi_gen, galactic, T_obs_years, L_m."""
    L, g, gal, T = noise["L_m"], noise["tdi_gen"], bool(noise["galactic"]), noise["T_obs_years"]
    return (lambda f: psd_ae(f, L, g, gal, T)), (lambda f: psd_t(f, L, g, gal, T))


def inner_products(x3, y3, dt: float, noise: dict):
    """Per channel (A, E, T): (<x|x>, <x|y>, <y|y>) as a (3, 3) array."""
    sae, st = channel_psds(noise)
    out = np.zeros((3, 3))
    for c in range(3):
        psd = sae if c < 2 else st
        a, b = np.asarray(x3[c], np.float64), np.asarray(y3[c], np.float64)
        out[c, 0] = inner(a, a, dt, psd, noise["f_min"], noise["f_max"])
        out[c, 1] = inner(a, b, dt, psd, noise["f_min"], noise["f_max"])
        out[c, 2] = inner(b, b, dt, psd, noise["f_min"], noise["f_max"])
    return out


def log_likelihood(ip):
    """ln L = -1/2 sum_c <d - h|d - h>, Eq. (derived_likelihood), from the
    per-channel products of inner_products(d, h)."""
    ip = np.asarray(ip)
    return -0.5 * float(np.sum(ip[..., 0] - 2.0 * ip[..., 1] + ip[..., 2]))
