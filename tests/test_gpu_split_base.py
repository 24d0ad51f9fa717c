"""FP32-bulk LFA and hybrid when a link delay crosses an integer inside a wave.

The split puts each use's integer base at ceil(q) (offset in [0, 1)); the
fast LFA path shares one base per wave of 576 outputs, so when a delay drifts
across an integer some uses belong to the neighbouring base, whose node set is
shifted by one sample.  For data the taps resolve this makes no difference,
but right at a merger (a kink in the amplitude, broadband at the sample scale)
the two interpolants differ by up to 4e-4 of the channel peak.  These sources
put such a crossing on the merger: link 1's fractional delay there is 0.012
samples (700-sample source) and 0.988 samples (4608-sample source, the
neighbouring base below).  The fast path's second pass over such links (the
uses on the neighbouring base) must bring them to the FP32 bar, and in the hybrid the switch comes 31 samples before the merger,
so the LFA still carries weight 0.15 there.
"""
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


def _sources():
    parts = [W.make_source(219473.88047358935, 0.7, 0.31171458350568465, 1.2671729642857517,
                           0.6845785204492111, 700, 10.0, 0.0)]
    rng = np.random.default_rng(23)
    for _ in range(4 * 4):         # the draws of the four sources before it in the tile-shape batch
        rng.uniform()
    beta, mc, lam, psi = np.arcsin(rng.uniform(-1, 1)), 10 ** rng.uniform(5, 5.4), rng.uniform(0, 6.28), \
        rng.uniform(0, 3.14)
    parts.append(W.make_source(mc, 0.7, beta, lam, psi, 4608, 10.0, 0.0))
    return W._assemble(parts, np)


@pytest.mark.parametrize("taps", [8, 16, 32])
@pytest.mark.parametrize("mode", [1, 2])
def test_merger_on_an_integer_crossing(tdi, orc, mode, taps):
    batch, orb = _sources(), W.default_orbit()
    cfg = W.default_config(tdi_gen=20, mode=mode, taps=taps, stencil_order=4, precision=1)
    info = {}
    got = tdi.response(batch, cfg, orb, info=info)
    assert info["lfa_fast"] == 1
    ref = orc.response_batch(dict(cfg, precision=0), orb, batch)
    for s in range(batch.n_sources):
        a, b = int(batch.offsets[s]), int(batch.offsets[s + 1])
        err = orc.peak_rel_err(got[:, a:b], ref[:, a:b])
        print(f"[parity] integer crossing at the merger, mode{mode} {taps} taps n={b - a}: "
              f"err X,Y,Z = {err[0]:.3e} {err[1]:.3e} {err[2]:.3e}", flush=True)
        assert np.all(err <= 1e-5), (s, err)
