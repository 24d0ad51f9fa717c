"""The allocation-free entry point tdi_run_noalloc against tdi_run.

Both run the same kernels on the same inputs: the FP32-bulk hybrid TDI 2.0
(fast LFA path with its per-tile records, plus the full part) and the FP64
hybrid TDI 1.5, each called twice in a row through the C ABI, the second time
with a smaller batch, so the static scratch array is reused with stale
contents from the first call.  Bars: 1e-5 of each channel's peak (FP32-bulk),
1e-12 (FP64); with the same tile shape both paths compute every output the
same way, so the differences are expected to be zero.
"""
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


def _batch(seed, n_sources, n_lo, n_hi, mc_switch):
    """n_sources chirps of seeded lengths; the first one light enough to reach
    the hybrid switch (it has a full-response region)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(n_sources):
        n = int(rng.integers(n_lo, n_hi))
        mc = mc_switch if i == 0 else 10 ** rng.uniform(5.6, 7.0)
        beta = math.asin(rng.uniform(-1, 1))
        lam, psi, iota = rng.uniform(0, 2 * math.pi), rng.uniform(0, math.pi), math.acos(rng.uniform(-1, 1))
        parts.append(W.make_source(mc, iota, beta, lam, psi, n, 10.0, t0=1.0e6 + 1.0e5 * i))
    b = W._assemble(parts, np)
    assert math.isfinite(b.sources[0]["t_hyb"])
    return b


def _peak_rel(got, ref):
    return np.array([np.max(np.abs(got[c] - ref[c])) / np.max(np.abs(ref[c])) for c in range(3)])


def _both(T, batch, cfg_d, orb_d):
    import torch
    dev = "cuda:0"
    hp = torch.as_tensor(batch.hp, dtype=torch.float64, device=dev)
    hc = torch.as_tensor(batch.hc, dtype=torch.float64, device=dev)
    ref = T.response(batch, cfg_d, orb_d, device=dev)
    cfg = T.make_config(cfg_d)
    orb = T.make_orbit(orb_d)
    src = T.make_sources(batch.sources)
    fp32 = int(cfg_d.get("precision", 0)) == T.TDI_FP32_BULK
    dt = torch.float32 if fp32 else torch.float64
    n = batch.total
    outs = [torch.full((n,), float("nan"), dtype=dt, device=dev) for _ in range(3)]
    stream = torch.cuda.current_stream().cuda_stream
    st = T.tdi_run_noalloc(cfg, orb, batch.n_sources, src, batch.offsets, hp.data_ptr(), hc.data_ptr(),
                           outs[0].data_ptr(), outs[1].data_ptr(), outs[2].data_ptr(), stream)
    assert st == T.TDI_OK, T.tdi_status_str(st)
    torch.cuda.synchronize()
    got = np.stack([o.double().cpu().numpy() for o in outs])
    return got, ref


@pytest.mark.parametrize("precision,gen,tol", [(1, 20, 1e-5), (0, 15, 1e-12)])
def test_noalloc_matches_run_twice(tdi, precision, gen, tol):
    cfg = W.default_config(tdi_gen=gen, mode=2, taps=32, stencil_order=4, precision=precision)
    cfg["fast_tile_chunks"] = 4
    orb = W.default_orbit()
    for call, (seed, ns, lo, hi) in enumerate([(71, 5, 60000, 140000), (72, 2, 20000, 40000)]):
        batch = _batch(seed, ns, lo, hi, 2.0e5)
        print(f"[noalloc] precision={precision} gen={gen} call {call}: {ns} sources, {batch.total} samples",
              flush=True)
        got, ref = _both(tdi, batch, cfg, orb)
        assert np.all(np.isfinite(got))
        err = _peak_rel(got, ref)
        print(f"[noalloc]   peak-rel diff vs tdi_run X,Y,Z = {err[0]:.3e} {err[1]:.3e} {err[2]:.3e} "
              f"(tol {tol:.0e})", flush=True)
        assert np.all(err <= tol)
