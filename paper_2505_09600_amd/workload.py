"""Seeded synthetic inputs for the LISA response: sources, strain series, orbits.

This module only *generates inputs*. It holds none of the response arithmetic
(no projection, interpolation, TDI, stencil or stitch), so both the HIP path and
the CPU oracle may consume what it produces without sharing method code.

The paper's waveforms (IMRPhenomTHM/TEHM) and LDC orbit classes are not
available, so the strain is a Newtonian quadrupole chirp with the shapes and
sizes of the paper's workloads (1e5..1e7 samples at 5..10 s, masses 1e5..1e7
solar masses; Sec. IV, timing subsection):

* f(tau) = (1/pi) (5 / (256 tau))^(3/8) tM^(-5/8),  tau = t_c - t,
  Phi(tau) = -2 (tau / (5 tM))^(5/8),  A proportional to f^(2/3), max A = 1;
* h+ = A (1 + cos^2 iota)/2 cos Phi,  hx = A cos iota sin Phi;
* inspiral cut at the ISCO GW frequency of the equal-mass binary
  (M = 2^(6/5) Mc), followed by an exponentially damped ringdown at f_cut
  (tau_d = 2/(pi f_cut)), continuous in phase and amplitude;
* optional eccentric modulation e(f) = e0 (f/f0)^(-19/18):
  Phi -> Phi + 2 e sin(Phi/2), A -> A (1 + e cos(Phi/2)).

The hybrid switch time follows the reading "first sample whose instantaneous
GW frequency reaches f_GW L / c = 0.05" (+inf when never reached), and the
leading-PN switch-time and LFA-fraction helpers restate Eqs. (thyb) and
(hybrid_ratio) of the hybrid-response section.

Arrays are float64.  ``xp`` may be numpy (default) or torch (for building
large batches directly in device memory).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Physical constants used to *describe* the inputs (orbit spec, chirp time scale).
C_LIGHT = 299792458.0                    # m/s
GMSUN_OVER_C3 = 4.925490947e-6           # s (solar mass in seconds)
AU = 1.495978707e11                      # m
ARM_L = 2.5e9                            # m, LISA nominal arm length
OMEGA_YR = 2.0 * math.pi / (365.25 * 86400.0)   # rad/s, Julian year

# Orbit kinds (same integer codes as the C ABI).
ORBIT_FROZEN = 0
ORBIT_ANALYTIC1 = 1
ORBIT_TABLE = 2

# tdi_source record layout shared by the C ABI and the oracle (host memory).
SOURCE_DTYPE = np.dtype([("beta", "<f8"), ("lam", "<f8"), ("psi", "<f8"),
                         ("t0", "<f8"), ("dt", "<f8"), ("t_hyb", "<f8")])


def default_orbit(kind: int = ORBIT_ANALYTIC1, t_freeze: float = 0.0,
                  kappa0: float = 0.0, lambda0: float = 0.0) -> dict:
    """Orbit spec: rigid equilateral first-order analytic orbit at 1 AU."""
    return dict(kind=int(kind), L=ARM_L, R=AU, omega=OMEGA_YR,
                kappa0=float(kappa0), lambda0=float(lambda0), t_freeze=float(t_freeze))


def keplerian_orbit_table(t0: float, dt: float, n: int, L: float = ARM_L, R: float = AU,
                          omega: float = OMEGA_YR, kappa0: float = 0.0, lambda0: float = 0.0):
    """Positions (n, 3, 3) of three spacecraft on exact Keplerian ellipses,
    sampled at t0 + j dt: semi-major axis R, eccentricity e = L/(2 sqrt3 R),
    inclination sqrt3 e, ascending node at beta_i + pi/2 and perihelion
    argument -pi/2 (beta_i = 2 pi i/3 + lambda0), mean anomaly
    omega t + kappa0 - beta_i.  To first order in e these are the rigid
    analytic orbit; at second order the arms flex (a stand-in for sampled
    orbit files).  Kepler's equation is solved by Newton iteration."""
    e = L / (2.0 * math.sqrt(3.0) * R)
    inc = math.sqrt(3.0) * e
    t = t0 + np.arange(n, dtype=np.float64) * dt
    out = np.zeros((n, 3, 3))
    for i in range(3):
        beta = 2.0 * math.pi * i / 3.0 + lambda0
        node, argp = beta + 0.5 * math.pi, -0.5 * math.pi
        M = omega * t + kappa0 - beta
        E = M.copy()
        for _ in range(30):
            E = E - (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
        xp = R * (np.cos(E) - e)
        yp = R * math.sqrt(1.0 - e * e) * np.sin(E)
        # perifocal -> ecliptic: rotate by argp, tilt by inc about the node line, rotate by node
        ca, sa = math.cos(argp), math.sin(argp)
        x1, y1 = ca * xp - sa * yp, sa * xp + ca * yp
        ci, si = math.cos(inc), math.sin(inc)
        y2, z2 = ci * y1, si * y1
        cn, sn = math.cos(node), math.sin(node)
        out[:, i, 0] = cn * x1 - sn * y2
        out[:, i, 1] = sn * x1 + cn * y2
        out[:, i, 2] = z2
    return out


def table_orbit(table, t0: float, dt: float, L: float = ARM_L) -> dict:
    """Orbit spec of a sampled table (TABLE kind); L is the nominal arm."""
    return dict(kind=ORBIT_TABLE, L=L, R=AU, omega=0.0, kappa0=0.0, lambda0=0.0, t_freeze=0.0,
                table=np.ascontiguousarray(table, dtype=np.float64), table_t0=float(t0),
                table_dt=float(dt))


def default_config(tdi_gen=20, mode=0, taps=32, stencil_order=4, equal_arms=0,
                   precision=0, T_samples=800.0, sigma_samples=20.0, channels=0,
                   nested_delays=0) -> dict:
    """Response configuration (hybrid defaults T = 800 dt, sigma = T/40;
    channels 0 = X, Y, Z, 1 = A, E, T; nested_delays 1 = time-nested delays
    in the full response)."""
    return dict(tdi_gen=int(tdi_gen), mode=int(mode), taps=int(taps),
                stencil_order=int(stencil_order), equal_arms=int(equal_arms),
                precision=int(precision), T_samples=float(T_samples),
                sigma_samples=float(sigma_samples), channels=int(channels),
                nested_delays=int(nested_delays))


# ----------------------------------------------------------------------------
# chirp model
# ----------------------------------------------------------------------------
def chirp_scales(mc_msun: float):
    """(tM, f_cut, tau_cut, tau_d) of the synthetic chirp for chirp mass Mc."""
    tM = mc_msun * GMSUN_OVER_C3
    m_tot = 2.0 ** 1.2 * tM
    f_cut = 1.0 / (6.0 ** 1.5 * math.pi * m_tot)
    tau_cut = (5.0 / 256.0) * (math.pi * f_cut) ** (-8.0 / 3.0) * tM ** (-5.0 / 3.0)
    tau_d = 2.0 / (math.pi * f_cut)
    return tM, f_cut, tau_cut, tau_d


def n_tail_samples(mc_msun: float, dt: float) -> int:
    """Ringdown tail length: ceil(10 tau_d / dt) + 64 samples."""
    return int(math.ceil(10.0 * chirp_scales(mc_msun)[3] / dt)) + 64


def _xp_of(x):
    if isinstance(x, np.ndarray):
        return np
    import torch
    return torch


def chirp_series(t, mc_msun: float, iota: float, t_c: float, e0: float = 0.0,
                 with_cut: bool = True):
    """h+, hx and the instantaneous GW frequency at times ``t`` (array, s)."""
    xp = _xp_of(t)
    tM, f_cut, tau_cut, tau_d = chirp_scales(mc_msun)
    t_cut = t_c - tau_cut if with_cut else math.inf
    tau = t_c - t
    if with_cut:
        tau_i = xp.where(tau > tau_cut, tau, tau * 0 + tau_cut)
    else:
        tau_i = tau
    f_i = (1.0 / math.pi) * (5.0 / (256.0 * tau_i)) ** 0.375 * tM ** (-0.625)
    phi_i = -2.0 * (tau_i / (5.0 * tM)) ** 0.625
    if with_cut:
        phi_cut = -2.0 * (tau_cut / (5.0 * tM)) ** 0.625
        dtr = t - t_cut
        ring = dtr > 0
        zero = dtr * 0
        dtr = xp.where(ring, dtr, zero)
        phi = xp.where(ring, phi_cut + 2.0 * math.pi * f_cut * dtr, phi_i)
        f = xp.where(ring, zero + f_cut, f_i)
        amp = (f / f_cut) ** (2.0 / 3.0) * xp.exp(-dtr / tau_d)
    else:
        phi, f = phi_i, f_i
        amp = f ** (2.0 / 3.0)
    if e0 != 0.0:
        f0 = f[0]
        ecc = e0 * (f / f0) ** (-19.0 / 18.0)
        phi = phi + 2.0 * ecc * xp.sin(0.5 * phi)
        amp = amp * (1.0 + ecc * xp.cos(0.5 * phi))
    amp = amp / amp.max()
    ci = math.cos(iota)
    hp = amp * (0.5 * (1.0 + ci * ci)) * xp.cos(phi)
    hc = amp * ci * xp.sin(phi)
    return hp, hc, f


def switch_time(t0: float, dt: float, f, fL_over_c: float = 0.05,
                arm: float = ARM_L) -> float:
    """t_Hyb at the first sample with f_GW >= fL_over_c * c / L (+inf if none)."""
    f_sw = fL_over_c * C_LIGHT / arm
    xp = _xp_of(f)
    idx = xp.nonzero(f >= f_sw)
    idx = idx[0] if xp is np else idx[:, 0]
    if len(idx) == 0:
        return math.inf
    return t0 + float(idx[0]) * dt


def t_hyb_leading_pn(t_c: float, f_hyb: float, mc_msun: float) -> float:
    """Switch time at leading PN order, Eq. (thyb) of the hybrid section."""
    tM = mc_msun * GMSUN_OVER_C3
    return t_c - f_hyb ** (-8.0 / 3.0) * 5.0 / (8.0 * math.pi) ** (8.0 / 3.0) * tM ** (-5.0 / 3.0)


def lfa_fraction(f_hyb: float, f_min: float, f_max: float | None = None) -> float:
    """Fraction of the waveform handled by the LFA, Eq. (hybrid_ratio);
    f_max=None gives the simplified form Eq. (hybrid_ratio_simplified)."""
    if f_max is None:
        return 1.0 - (f_hyb / f_min) ** (-8.0 / 3.0)
    a, b, c = f_min ** (-8 / 3), f_hyb ** (-8 / 3), f_max ** (-8 / 3)
    return (a - b) / (a - c)


# ----------------------------------------------------------------------------
# batches
# ----------------------------------------------------------------------------
@dataclass
class Batch:
    """CSR batch of sources: source i owns samples offsets[i]:offsets[i+1]."""
    sources: np.ndarray                 # SOURCE_DTYPE records (host)
    offsets: np.ndarray                 # int64, n_sources + 1
    hp: object                          # float64 flat (numpy or torch)
    hc: object
    meta: list = field(default_factory=list)   # per-source dict (mc, iota, e0, ...)

    @property
    def n_sources(self) -> int:
        return len(self.sources)

    @property
    def total(self) -> int:
        return int(self.offsets[-1])

    def source(self, i):
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        return self.sources[i], self.hp[a:b], self.hc[a:b]

    def subset(self, idx):
        """New batch (numpy) with the sources listed in idx."""
        recs, hps, hcs, offs, meta = [], [], [], [0], []
        for i in idx:
            r, a, b = self.source(int(i))
            recs.append(r)
            hps.append(_to_np(a))
            hcs.append(_to_np(b))
            offs.append(offs[-1] + len(hps[-1]))
            meta.append(self.meta[int(i)] if self.meta else {})
        return Batch(np.array(recs, dtype=SOURCE_DTYPE), np.array(offs, dtype=np.int64),
                     np.concatenate(hps) if hps else np.zeros(0),
                     np.concatenate(hcs) if hcs else np.zeros(0), meta)


def _to_np(a):
    if isinstance(a, np.ndarray):
        return a
    return a.detach().cpu().numpy()


def make_source(mc, iota, beta, lam, psi, n, dt, t0=0.0, e0=0.0, t_c=None,
                hybrid=True, xp=np, device=None):
    """One source: (record, hp, hc, meta).

    Without ``t_c`` the inspiral ends ``n_tail`` samples before the end and a
    ringdown fills the tail; with ``t_c`` there is no cut (pre-merger chirp).
    """
    if t_c is None:
        tM, f_cut, tau_cut, tau_d = chirp_scales(mc)
        t_cut = t0 + (n - n_tail_samples(mc, dt)) * dt
        t_c = t_cut + tau_cut
        with_cut = True
    else:
        with_cut = False
    if xp is np:
        t = t0 + np.arange(n, dtype=np.float64) * dt
    else:
        t = t0 + xp.arange(n, dtype=xp.float64, device=device) * dt
    hp, hc, f = chirp_series(t, mc, iota, t_c, e0=e0, with_cut=with_cut)
    t_hyb = switch_time(t0, dt, f) if hybrid else math.inf
    rec = np.array([(beta, lam, psi, t0, dt, t_hyb)], dtype=SOURCE_DTYPE)[0]
    meta = dict(mc=mc, iota=iota, e0=e0, t_c=t_c, n=n)
    return rec, hp, hc, meta


def _assemble(parts, xp):
    recs = np.array([p[0] for p in parts], dtype=SOURCE_DTYPE)
    offs = np.zeros(len(parts) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(p[1]) for p in parts])
    cat = np.concatenate if xp is np else xp.cat
    hp = cat([p[1] for p in parts]) if parts else np.zeros(0)
    hc = cat([p[2] for p in parts]) if parts else np.zeros(0)
    return Batch(recs, offs, hp, hc, [p[3] for p in parts])


def _sky(rng, size):
    beta = np.arcsin(rng.uniform(-1.0, 1.0, size))
    lam = rng.uniform(0.0, 2.0 * math.pi, size)
    psi = rng.uniform(0.0, math.pi, size)
    return beta, lam, psi


def config_c1(seed: int = 1001, n: int = 2 ** 14):
    """Plain full response, FP64, frozen constellation, one pre-merger chirp."""
    rng = np.random.default_rng(seed)
    beta, lam, psi = _sky(rng, 1)
    dt, t0, mc, iota = 5.0, 0.0, 3.0e5, math.pi / 3
    t_c = t0 + (n - 1) * dt + 3600.0
    part = make_source(mc, iota, beta[0], lam[0], psi[0], n, dt, t0, t_c=t_c, hybrid=False)
    batch = _assemble([part], np)
    cfg = default_config(tdi_gen=15, mode=0, taps=16, precision=0)
    orb = default_orbit(ORBIT_FROZEN, t_freeze=0.0)
    return batch, cfg, orb


def draw_sources(seed: int, n_sources: int, n_lo: float, n_hi: float, ecc=False):
    """(mc, beta, lam, psi, iota, n, e0) arrays drawn in this fixed order."""
    rng = np.random.default_rng(seed)
    mc = 10.0 ** rng.uniform(5.0, 7.0, n_sources)
    beta, lam, psi = _sky(rng, n_sources)
    iota = np.arccos(rng.uniform(-1.0, 1.0, n_sources))
    if n_lo == n_hi:
        n = np.full(n_sources, int(n_lo), dtype=np.int64)
    else:
        n = np.rint(2.0 ** rng.uniform(math.log2(n_lo), math.log2(n_hi), n_sources)).astype(np.int64)
    e0 = rng.uniform(0.0, 0.3, n_sources) if ecc else np.zeros(n_sources)
    return mc, beta, lam, psi, iota, n, e0


def config_c2(seed: int = 1002, n: int = 3155760, mode=0, precision=0, tdi_gen=20,
              stencil_order=4, equal_arms=0):
    """One year at dt = 10 s, analytic orbit, N = 32, TDI 2.0 (c3 adds LFA/hybrid)."""
    mc, beta, lam, psi, iota, _, _ = draw_sources(seed, 1, n, n)
    part = make_source(mc[0], iota[0], beta[0], lam[0], psi[0], n, 10.0, 0.0)
    batch = _assemble([part], np)
    cfg = default_config(tdi_gen=tdi_gen, mode=mode, taps=32, precision=precision,
                         stencil_order=stencil_order, equal_arms=equal_arms)
    return batch, cfg, default_orbit(ORBIT_ANALYTIC1)


def config_batch(seed: int = 1004, n_sources: int = 512, n_lo: float = 2 ** 18,
                 n_hi: float = 2 ** 22, dt: float = 10.0, ecc: bool = False,
                 mode: int = 2, precision: int = 1, tdi_gen: int = 20,
                 stencil_order: int = 4, xp=np, device=None, only=None):
    """Batched hybrid workload (c4: 512 sources, lengths log-uniform 2^18..2^22,
    dt = 10 s; c5: 4096 x 3e6 at dt = 5 s with eccentric modulation).

    ``only`` restricts generation to a subset of source indices (the draws are
    still made for the whole batch so a subset matches the full batch)."""
    mc, beta, lam, psi, iota, n, e0 = draw_sources(seed, n_sources, n_lo, n_hi, ecc)
    idx = range(n_sources) if only is None else only
    parts = [make_source(mc[i], iota[i], beta[i], lam[i], psi[i], int(n[i]), dt, 0.0,
                         e0=e0[i], xp=xp, device=device) for i in idx]
    batch = _assemble(parts, xp)
    cfg = default_config(tdi_gen=tdi_gen, mode=mode, taps=32, precision=precision,
                         stencil_order=stencil_order)
    return batch, cfg, default_orbit(ORBIT_ANALYTIC1)


def config_c4(**kw):
    return config_batch(seed=kw.pop("seed", 1004), **kw)


def config_c5(n_sources: int = 4096, n: int = 3000000, **kw):
    return config_batch(seed=kw.pop("seed", 1005), n_sources=n_sources, n_lo=n, n_hi=n,
                        dt=5.0, ecc=True, **kw)


def single_source_batch(hp, hc, beta, lam, psi, t0=0.0, dt=10.0, t_hyb=math.inf):
    """Wrap explicit arrays (e.g. analytic test signals) as a one-source batch."""
    rec = np.array([(beta, lam, psi, t0, dt, t_hyb)], dtype=SOURCE_DTYPE)[0]
    return _assemble([(rec, np.asarray(hp, dtype=np.float64),
                       np.asarray(hc, dtype=np.float64), {})], np)
