"""GPU parity of the A, E, T output channels and of the noise-weighted inner
product (through the C ABI) against the FP64 oracle.

Inner-product metric per source and channel: max |GPU - oracle| over the three
products <x|x>, <x|y>, <y|y>, divided by sqrt(<x|x> <y|y>) (the Cauchy-Schwarz
scale of <x|y>).  Bars: 1e-12 (FP64 transforms) and 1e-5 (FP32 transforms:
log2(N) <= 24 radix-4/2 stages at 2^-24 each, ~1e-6 at worst, summed in FP64;
the same 1e-5 as the response's FP32 bar).  Inputs are the
oracle's own responses or the seeded generator's series; FP32 runs give both
sides the same float-rounded inputs.
"""
import math

import numpy as np
import pytest

from oracle import noise as NZ
from paper_2505_09600_amd import workload as W

pytestmark = pytest.mark.gpu

NOISE20 = dict(tdi_gen=20, galactic=1, T_obs_years=1.0, L_m=W.ARM_L, f_min=1e-4, f_max=0.029)
NOISE15 = dict(tdi_gen=15, galactic=0, T_obs_years=1.0, L_m=W.ARM_L, f_min=3e-5, f_max=0.05)
TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def tdi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2505_09600_amd import tdi as T
    T.lib()
    return T


def _dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0").contiguous()


def _ip_gpu(T, noise, prec, dt, offsets, x3, y3, plan=None):
    import torch
    dtype = torch.float64 if prec == 0 else torch.float32
    xs = [_dev(a, dtype) for a in x3]
    ys = [_dev(a, dtype) for a in y3]
    out = plan.run(offsets, xs, ys)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _ip_orc(noise, dt, offsets, x3, y3):
    ref = np.zeros((len(offsets) - 1, 3, 3))
    for s in range(len(offsets) - 1):
        a, b = int(offsets[s]), int(offsets[s + 1])
        ref[s] = NZ.inner_products([v[a:b] for v in x3], [v[a:b] for v in y3], dt, noise)
    return ref


def _check(name, got, ref, tol):
    worst = 0.0
    for s in range(ref.shape[0]):
        for c in range(3):
            scale = math.sqrt(max(ref[s, c, 0] * ref[s, c, 2], 0.0))
            if scale == 0.0:
                assert np.all(got[s, c] == 0.0), (name, s, c, got[s, c])
                continue
            err = float(np.max(np.abs(got[s, c] - ref[s, c]))) / scale
            worst = max(worst, err)
            assert err <= tol, (name, s, c, err, got[s, c], ref[s, c])
    print(f"[parity] {name}: max err {worst:.3e}  tol {tol:.0e}", flush=True)
    return worst


def _rounded(a, prec):
    return np.asarray(a, dtype=np.float32).astype(np.float64) if prec == 1 else np.asarray(a, np.float64)


@pytest.mark.parametrize("prec", [0, 1])
def test_aet_channels(tdi, orc, prec):
    """channels = AET writes the orthonormal map of X, Y, Z (same batch run both ways)."""
    rng = np.random.default_rng(21)
    parts = []
    for n in (3, 5000, 23000):
        beta = math.asin(rng.uniform(-1, 1))
        lam, psi, iota = rng.uniform(0, 2 * math.pi), rng.uniform(0, math.pi), math.acos(rng.uniform(-1, 1))
        parts.append(W.make_source(2.5e5, iota, beta, lam, psi, n, 10.0, 0.0))
    batch = W._assemble(parts, np)
    cfg = W.default_config(tdi_gen=20, mode=2, taps=32, stencil_order=4, precision=prec)
    orb = W.default_orbit()
    xyz = tdi.response(batch, cfg, orb)
    aet = tdi.response(batch, dict(cfg, channels=1), orb)
    # the store applies the map in the output precision
    ref_map = np.array(NZ.aet(*xyz))
    ulp = 2.0 ** -52 if prec == 0 else 2.0 ** -23
    peak = np.max(np.abs(xyz))
    assert np.max(np.abs(aet - ref_map)) <= 8 * ulp * peak
    # and against the oracle's X, Y, Z mapped to A, E, T, relative to the X, Y, Z peak
    ref = np.array(NZ.aet(*orc.response_batch(cfg, orb, batch)))
    err = np.max(np.abs(aet - ref), axis=1) / np.max(np.abs(orc.response_batch(cfg, orb, batch)))
    tol = 1e-12 if prec == 0 else 1e-5
    print(f"[parity] aet prec{prec}: err A,E,T = {err[0]:.3e} {err[1]:.3e} {err[2]:.3e}  tol {tol:.0e}", flush=True)
    assert np.all(err <= tol)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("noise", [NOISE20, NOISE15], ids=["tdi20", "tdi15"])
def test_inner_product_ragged(tdi, orc, prec, noise):
    """Lengths across the one-pass / two-pass boundary, empty and tiny series,
    two runs on one plan (the second smaller)."""
    dt = 10.0
    rng = np.random.default_rng(7 + prec)
    lengths = [0, 1, 2, 3, 100, 4096, 4097, 8192, 8193, 16384, 16385, 20000, 65536, 100003]
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    total = int(offsets[-1])
    # chirps from the generator (x) and a perturbed copy plus white noise (y)
    x3 = np.zeros((3, total))
    y3 = np.zeros((3, total))
    for s, n in enumerate(lengths):
        if n == 0:
            continue
        a, b = int(offsets[s]), int(offsets[s + 1])
        _, hp, hc, _ = W.make_source(10 ** rng.uniform(5, 6.5), 0.9, 0.1, 0.2, 0.3, n, dt, 0.0)
        x3[:, a:b] = [hp, hc, hp - 0.5 * hc]
        y3[:, a:b] = 0.97 * x3[:, a:b] + 0.05 * rng.standard_normal((3, n))
    x3, y3 = _rounded(x3, prec), _rounded(y3, prec)
    ref = _ip_orc(noise, dt, offsets, x3, y3)
    with tdi.IpPlan(noise, prec, dt, len(lengths), total, max(lengths)) as plan:
        got = _ip_gpu(tdi, noise, prec, dt, offsets, x3, y3, plan)
        _check(f"ip ragged prec{prec} tdi{noise['tdi_gen']}", got, ref, TOL[prec])
        # second run on the same plan with a smaller batch
        sub = np.array([0, 4097, 4097 + 300], dtype=np.int64)
        xs = x3[:, offsets[7]:offsets[7] + int(sub[-1])]
        ys = y3[:, offsets[7]:offsets[7] + int(sub[-1])]
        got2 = _ip_gpu(tdi, noise, prec, dt, sub, xs, ys, plan)
        _check(f"ip second run prec{prec}", got2, _ip_orc(noise, dt, sub, xs, ys), TOL[prec])
        t = plan.kernel_times()
        assert len(t) == 6 and all(v >= 0 for v in t)


@pytest.mark.parametrize("prec", [0, 1])
def test_inner_product_of_responses(tdi, orc, prec):
    """Likelihood of a hybrid template against full-response data: both are
    oracle responses (A, E, T) of a source; the template's psi differs."""
    n, dt = 60000, 10.0
    rec, hp, hc, _ = W.make_source(3.0e5, 0.6, 0.3, 2.0, 0.4, n, dt, 0.0)
    batch = W._assemble([(rec, hp, hc, {})], np)
    orb = W.default_orbit()
    full = orc.response_batch(W.default_config(tdi_gen=20, mode=0), orb, batch)
    rec2 = rec.copy()
    rec2["psi"] = rec["psi"] + 0.02
    batch2 = W._assemble([(rec2, hp, hc, {})], np)
    hyb = orc.response_batch(W.default_config(tdi_gen=20, mode=2), orb, batch2)
    d3 = _rounded(np.array(NZ.aet(*full)), prec)
    h3 = _rounded(np.array(NZ.aet(*hyb)), prec)
    offsets = np.array([0, n], dtype=np.int64)
    ref = _ip_orc(NOISE20, dt, offsets, d3, h3)
    with tdi.IpPlan(NOISE20, prec, dt, 1, n, n) as plan:
        got = _ip_gpu(tdi, NOISE20, prec, dt, offsets, d3, h3, plan)
    _check(f"ip responses prec{prec}", got, ref, TOL[prec])
    lnl_ref = NZ.log_likelihood(ref[0])
    lnl_got = NZ.log_likelihood(got[0])
    print(f"[parity] lnL prec{prec}: gpu {lnl_got:.6e} oracle {lnl_ref:.6e}", flush=True)
    assert abs(lnl_got - lnl_ref) <= TOL[prec] * 4 * np.sum(ref[0, :, 0])


@pytest.mark.parametrize("prec,n", [(1, 4194304), (1, 3000000), (0, 4194304)])
def test_inner_product_full_size(tdi, orc, prec, n):
    """Benchmark-size series (2^22 and the 3e6-sample sources): the longest
    two-pass split of each precision."""
    dt = 10.0 if n != 3000000 else 5.0
    noise = dict(NOISE20, f_max=0.029 if dt == 10.0 else 0.029)
    rng = np.random.default_rng(n)
    _, hp, hc, _ = W.make_source(1e6, 1.0, 0.1, 0.2, 0.3, n, dt, 0.0, e0=0.2)
    x3 = np.array([hp, hc, hp + hc])
    y3 = np.array([hc, hp, hp - hc]) + 1e-3 * rng.standard_normal((3, n))
    x3, y3 = _rounded(x3, prec), _rounded(y3, prec)
    offsets = np.array([0, n], dtype=np.int64)
    ref = _ip_orc(noise, dt, offsets, x3, y3)
    with tdi.IpPlan(noise, prec, dt, 1, n, n) as plan:
        got = _ip_gpu(tdi, noise, prec, dt, offsets, x3, y3, plan)
    _check(f"ip full size n={n} prec{prec}", got, ref, TOL[prec])
