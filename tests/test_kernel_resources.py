"""Register budget of the HIP kernels (compile only, no GPU).

The kernels are tuned to an occupancy that their registers allow; a change
that pushes one over its budget does not fail any parity test, it only spills
to scratch memory and runs slower (a launch bound of four workgroups on the
FP64 LFA kernel once spilled 464 bytes per lane and cost it a factor 2.2).
This test compiles the device code for gfx950 with the compiler's
resource-usage remarks and checks, per kernel:
  - scratch (spill) bytes per lane stay small: at most 128, which holds a few
    loop-invariant values reloaded once per tile (the general FP32 LFA kernel
    with the next term keeps 96-112 bytes there, in per-tile code), while a
    spilled working set of an inner loop runs to hundreds of bytes;
  - the FP32 LFA kernel and its pre-pass keep three waves per SIMD (the
    pre-pass is latency-bound: at two it took 0.49 ms of a 780M-sample step
    instead of 0.36).
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2505_09600_amd import build_lib

HIPCC = build_lib.HIPCC
MAX_SCRATCH = 128           # bytes per lane


def _remarks(src):
    out = os.path.join("/tmp", "tdi_res_" + os.path.basename(src) + ".o")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", os.path.join(build_lib.ROOT, "include"),
           "-I", build_lib.CSRC, "--cuda-device-only", "-c", src, "-o", out,
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            kernels[name] = {}
            continue
        m = re.search(r"(ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]|VGPRs): (\d+)", line)
        if m and name is not None:
            kernels[name][m.group(1).split()[0]] = int(m.group(2))
    return kernels


@pytest.fixture(scope="module")
def usage():
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    res = {}
    for n in ("tdi_kernels.hip", "tdi_ip_kernels.hip"):
        res.update(_remarks(os.path.join(build_lib.CSRC, n)))
    return res


def test_every_kernel_reported(usage):
    names = " ".join(usage)
    for k in ("k_lfa_fast", "k_lfa_prep", "k_full", "k_links", "k_ip_pass1", "k_ip_pass2"):
        assert k in names, k


def test_scratch_per_lane_small(usage):
    heavy = {k: v["ScratchSize"] for k, v in usage.items() if v.get("ScratchSize", 0) > MAX_SCRATCH}
    assert not heavy, heavy


def test_fast_lfa_keeps_three_waves_per_simd(usage):
    fast = {k: v for k, v in usage.items() if "k_lfa_fast" in k}
    assert len(fast) == 4, sorted(fast)          # 4, 8, 16 and 32 taps
    for k, v in fast.items():
        assert v["Occupancy"] >= 3, (k, v)


def test_fast_lfa_prepass_keeps_three_waves_per_simd(usage):
    prep = {k: v for k, v in usage.items() if "k_lfa_prep" in k}
    assert len(prep) == 4, sorted(prep)
    for k, v in prep.items():
        assert v["Occupancy"] >= 3, (k, v)
