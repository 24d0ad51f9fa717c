#!/usr/bin/env python3
"""Benchmark: batched FP32-bulk hybrid TDI 2.0 X,Y,Z on one MI355X.

Workload: 512 sources, lengths log-uniform in 2^18..2^22 samples at dt = 10 s
(7.26e8 samples in total), seeded uniform sky, polarisation and inclination,
log-uniform chirp mass 1e5..1e7 Msun, synthetic Newtonian chirps with ringdown
(seed 1004); first-order analytic orbits; 32-tap Lagrange interpolation,
4th-order LFA stencils, hybrid switch where f_GW L / c reaches 0.05,
T = 800 dt, sigma = T / 40.  Inputs are generated in device memory before the
timed region.  One step = one tdi_run over the whole batch (graph replay of the
persistent LFA and full-response kernels), synchronised after each step;
ms_per_step is the median step and value = samples / median step.

The line also carries the FP64 full, LFA and hybrid responses of the same batch,
the roofline of the dominant kernel (algorithmic HBM bytes per launch over its
median event-timed duration, with the VALU issue rate from the committed
counter summary when it matches the kernel source) and the FP64 CPU oracle
timed per mode on one core and on all cores.

Prints one JSON line (see the keys below).  --gpus N > 1 is not supported:
the response has no multi-GPU path in this build (sources would be sharded
across GPUs without communication).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TDI2 XYZ samples/s (batched, FP32-bulk vs FP64) at ≤1e-5 peak-rel error"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3              # published, with packed FP32
FP32_NONPACKED_TFLOPS = 78.6          # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (packed FP32 is off)
FP64_PEAK_TFLOPS = 78.6
VALU_SIMDS = 256 * 4                  # a wave64 VALU instruction occupies one 16-lane SIMD for 4 cycles
CLOCK_HZ = 2.4e9
BYTES_PER_SAMPLE_FP32 = 16 + 12       # read h+, hx (FP64), write X, Y, Z (FP32)
BYTES_PER_SAMPLE_FP64 = 16 + 24
TAPS = 32


def lfa_flops_per_sample(taps: int) -> int:
    """Algorithmic FP32 work of the LFA per output sample: six retarded reads,
    each a two-component N-tap Lagrange interpolation counted as N weights
    (4N flops) plus two N-tap dot products (4N flops)."""
    return 6 * (4 * taps + 4 * taps)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("tdi_kernels.hip", "tdi_internal.h"):
        with open(os.path.join(ROOT, "paper_2505_09600_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters(kernel_hash: str):
    """HBM bytes and VALU instructions per launch of the dominant kernel, from the
    committed rocprofv3 PMC summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "k_lfa_c4_counters.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_hash") != kernel_hash:
        return None
    return d


def _oracle_run(oracle, cfg, orb, sub, m, rng):
    """One oracle evaluation of a contiguous block of m outputs (at a seeded
    random start) in each source of sub; returns (outputs, seconds)."""
    lens = [int(sub.offsets[i + 1] - sub.offsets[i]) for i in range(sub.n_sources)]
    ks = []
    for n in lens:
        mm = min(m, n)
        a = int(rng.integers(0, n - mm + 1))
        ks.append(np.arange(a, a + mm, dtype=np.int64))
    t = time.perf_counter()
    oracle.response_batch_at(cfg, orb, sub, ks)
    return int(sum(len(k) for k in ks)), time.perf_counter() - t


def _oracle_rate(oracle, cfg, orb, sub, target_s, reps, rng):
    """Median samples/s of `reps` oracle runs, each sized to about target_s."""
    m = 256
    while True:
        nout, el = _oracle_run(oracle, cfg, orb, sub, m, rng)
        full = all(m >= int(sub.offsets[i + 1] - sub.offsets[i]) for i in range(sub.n_sources))
        if el >= 0.5 * target_s or full:
            break
        m = int(m * min(16.0, max(1.5, target_s / max(el, 1e-3))))
    rates = [nout / el]
    for _ in range(reps - 1):
        nout, el = _oracle_run(oracle, cfg, orb, sub, m, rng)
        rates.append(nout / el)
    return float(np.median(rates)), m, nout


def cpu_baseline(host_sub, cfg, orb, budget_s: float, modes: dict):
    """The FP64 oracle, as it stands, on a bounded seeded sample of the batch:
    contiguous blocks of outputs at seeded random positions of seeded random
    sources, evaluated with the oracle's sampled-output entry point (OpenMP
    across sources; a single source runs on one thread).  Each mode is timed at
    one core (one source) and on all cores (every source of the sample), as the
    median of five runs; the headline entry is the hybrid TDI 2.0 on all cores."""
    import oracle
    oracle.build(force=False)
    threads = oracle.num_threads()
    rng = np.random.default_rng(11)
    one = host_sub.subset([0])
    per = budget_s / (2.0 * 5.0 * len(modes))
    table = {}
    for name, c in modes.items():
        r1, m1, _ = _oracle_rate(oracle, c, orb, one, per, 5, rng)
        ra, ma, na = _oracle_rate(oracle, c, orb, host_sub, per, 5, rng)
        table[name] = {"one_core": r1, "all_cores": ra, "block_one_core": m1, "block_all_cores": ma,
                       "outputs_all_cores": na}
        print(f"[bench] oracle {name}: {r1:.3g} samples/s on 1 core, {ra:.3g} on {threads}",
              file=sys.stderr, flush=True)
    h = table["hybrid tdi2.0"]
    return {"value": h["all_cores"], "unit": "samples/s", "cores": threads, "kind": "oracle",
            "value_1core": h["one_core"], "modes": table, "timing": "median of 5 runs per entry",
            "sample": f"contiguous blocks of {h['block_all_cores']} outputs at seeded random positions in "
                      f"each of {host_sub.n_sources} seeded random sources of the batch ({h['outputs_all_cores']} "
                      f"outputs per run; one core: a block of {h['block_one_core']} outputs of one source), "
                      f"FP64 oracle, sampled-output entry point, OpenMP across sources"}


def time_plan(tdi, torch, hp, hc, recs, offsets, cfg, orb, steps, warmup, autotune=True, untimed=False):
    """Time one configuration with the library's autotuned plan (graph replay
    allowed); per-kernel times come from the plan's event records.  untimed:
    ms_per_run is then taken from a second loop without the event records
    (tdi_plan_set_timing), whose device markers cost microseconds per run."""
    dev = hp.device
    total = int(offsets[-1])
    dt = torch.float32 if cfg["precision"] == 1 else torch.float64
    X = torch.empty(total, dtype=dt, device=dev)
    Y = torch.empty_like(X)
    Z = torch.empty_like(X)
    src = tdi.make_sources(recs)
    with tdi.Plan(cfg, orb, len(recs), total, autotune=autotune, use_graph=True) as plan:
        for _ in range(warmup):
            plan.run(src, offsets, hp, hc, X, Y, Z)
        if plan.sync() != tdi.TDI_OK:
            raise RuntimeError("window check failed")
        plan.kernel_times()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.run(src, offsets, hp, hc, X, Y, Z)
        t_sub = time.perf_counter() - t0
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kt = plan.kernel_times()
        if plan.sync() != tdi.TDI_OK:
            raise RuntimeError("window check failed")
        el_timed = el
        if untimed:
            # median of 5 loops: a run of ~0.1 ms is exposed to host hiccups
            plan.set_timing(False)
            reps = []
            for _ in range(5):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    plan.run(src, offsets, hp, hc, X, Y, Z)
                t_s = time.perf_counter() - t0
                torch.cuda.synchronize()
                reps.append((time.perf_counter() - t0, t_s))
            if plan.sync() != tdi.TDI_OK:
                raise RuntimeError("window check failed")
            el, t_sub = sorted(reps)[len(reps) // 2]
        launch = plan.describe()
    del X, Y, Z
    runs = len(kt) // 3
    mean = [float(np.mean(kt[j::3][:runs])) if runs else float("nan") for j in range(3)]
    # host_ms_per_run: the host's enqueue time per run (the runs are asynchronous;
    # when it approaches ms_per_run the host, not the device, sets the pace)
    return {"ms_per_run": 1e3 * el / steps, "ms_per_run_timed": 1e3 * el_timed / steps,
            "host_ms_per_run": 1e3 * t_sub / steps, "samples_per_s": total * steps / el,
            "prep_ms": mean[0], "lfa_ms": mean[1], "full_ms": mean[2], "launch": launch}


def secondary(args):
    """Single-source configurations (c1-c3) and the sampler-scale batch (c5, two
    device-resident waves of 2048 sources whose per-wave times are summed)."""
    import torch
    from paper_2505_09600_amd import tdi
    from paper_2505_09600_amd import workload as W
    tdi.lib()
    dev = torch.device("cuda:0")
    out = {"metric": METRIC, "unit": "samples/s", "n_gpus": 1, "data": "synthetic",
           "higher_is_better": True}
    if args.config in ("c1", "c2", "c3"):
        runs = {}
        if args.config == "c1":
            batch, cfg, orb = W.config_c1()
            cases = {"full fp64 tdi1.5 N16": cfg}
            wl = "one pre-merger chirp, 2^14 samples at dt=5 s, frozen constellation (seed 1001)"
        else:
            batch, cfg, orb = W.config_c2()
            if args.config == "c2":
                cases = {f"full {p} tdi2.0 N32": dict(cfg, mode=0, precision=i) for i, p in ((0, "fp64"), (1, "fp32"))}
                # the same with time-nested delays (light times at each retarded time)
                cases.update({f"full {p} tdi2.0 N32 nested": dict(cfg, mode=0, precision=i, nested_delays=1)
                              for i, p in ((0, "fp64"), (1, "fp32"))})
            else:
                cases = {}
                for gen in (15, 20):
                    for st in (2, 4):
                        for i, pr in ((0, "fp64"), (1, "fp32")):
                            cases[f"lfa p{st} {pr} tdi{gen}"] = dict(cfg, mode=1, tdi_gen=gen, stencil_order=st, precision=i)
            wl = "one year at dt=10 s, 3155760 samples, analytic orbit (seed 1002)"
        hp = torch.as_tensor(batch.hp, device=dev)
        hc = torch.as_tensor(batch.hc, device=dev)
        for name, c in cases.items():
            runs[name] = time_plan(tdi, torch, hp, hc, batch.sources, batch.offsets, c, orb, args.steps, args.warmup,
                                   untimed=True)
            print(f"[bench] {args.config} {name}: {runs[name]['ms_per_run']:.3f} ms/run", file=sys.stderr, flush=True)
        if args.config == "c3":
            # the c3 recipe with a chirp mass that reaches the switch (hybrid)
            n = 3155760
            mc, beta, lam, psi, iota, _, _ = W.draw_sources(1003, 1, n, n)
            part = W.make_source(2.0e5, iota[0], beta[0], lam[0], psi[0], n, 10.0, 0.0)
            hb = W._assemble([part], np)
            hhp = torch.as_tensor(hb.hp, device=dev)
            hhc = torch.as_tensor(hb.hc, device=dev)
            for gen in (15, 20):
                for i, pr in ((0, "fp64"), (1, "fp32")):
                    name = f"hybrid {pr} tdi{gen} (mc 2e5, seed 1003)"
                    c = dict(cfg, mode=2, tdi_gen=gen, stencil_order=4, precision=i)
                    runs[name] = time_plan(tdi, torch, hhp, hhc, hb.sources, hb.offsets, c, orb, args.steps,
                                           args.warmup, untimed=True)
                    print(f"[bench] c3 {name}: {runs[name]['ms_per_run']:.3f} ms/run", file=sys.stderr, flush=True)
        out.update({"config": {"workload": f"{args.config}: {wl}"}, "runs": runs,
                    "steps": args.steps, "warmup": args.warmup})
        print(json.dumps(out), flush=True)
        return
    # c5: 4096 sources x 3e6 samples at dt = 5 s (eccentric modulation) in two waves
    n = 3000000
    mc, beta, lam, psi, iota, ns, e0 = W.draw_sources(1005, 4096, n, n, ecc=True)
    orb = W.default_orbit()
    waves = []
    for w in range(2):
        idx = range(2048 * w, 2048 * (w + 1))
        total = 2048 * n
        hp = torch.empty(total, dtype=torch.float64, device=dev)
        hc = torch.empty_like(hp)
        recs = []
        t_gen = time.perf_counter()
        for j, i in enumerate(idx):
            rec, a, b, _ = W.make_source(mc[i], iota[i], beta[i], lam[i], psi[i], n, 5.0, 0.0,
                                         e0=e0[i], xp=torch, device=dev)
            hp[j * n:(j + 1) * n] = a
            hc[j * n:(j + 1) * n] = b
            recs.append(rec)
            if (j + 1) % 512 == 0:
                print(f"[bench] c5 wave {w}: {j + 1} sources generated", file=sys.stderr, flush=True)
        recs = np.array(recs, dtype=W.SOURCE_DTYPE)
        offsets = np.arange(2049, dtype=np.int64) * n
        torch.cuda.synchronize()
        print(f"[bench] c5 wave {w}: generated {total} samples in {time.perf_counter() - t_gen:.1f} s",
              file=sys.stderr, flush=True)
        cfg = W.default_config(tdi_gen=20, mode=2, taps=32, stencil_order=4, precision=1)
        r = time_plan(tdi, torch, hp, hc, recs, offsets, cfg, orb, args.steps, args.warmup)
        print(f"[bench] c5 wave {w} hybrid fp32: {r['ms_per_run']:.2f} ms/run", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        if not args.no_fp64_reference:
            # FP64 outputs for the whole wave would not fit beside the strain:
            # the plain FP64 full response is timed on the wave's first 1024 sources
            c64 = W.default_config(tdi_gen=20, mode=0, taps=32, stencil_order=4, precision=0)
            r["fp64_full"] = time_plan(tdi, torch, hp, hc, recs[:1024], offsets[:1025], c64, orb,
                                       1, 1, autotune=False)
            r["fp64_full"]["sources"] = 1024
            print(f"[bench] c5 wave {w} full fp64 (1024 sources): "
                  f"{r['fp64_full']['ms_per_run']:.1f} ms/run", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        waves.append(r)
        del hp, hc
        torch.cuda.empty_cache()
    ms = sum(r["ms_per_run"] for r in waves)
    value = 4096 * n / (ms * 1e-3)
    out.update({"value": value, "ms_per_step": ms, "steps": args.steps, "warmup": args.warmup,
                "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                "config": {"workload": "c5: 4096 sources x 3e6 samples at dt=5 s, eccentric modulation "
                                       "(seed 1005), hybrid TDI 2.0 FP32-bulk, two device-resident waves "
                                       "of 2048 sources, per-wave times summed",
                           "total_samples": 4096 * n},
                "waves": waves})
    if not args.no_fp64_reference:
        ms64 = sum(r["fp64_full"]["ms_per_run"] for r in waves)
        v64 = 2048 * n / (ms64 * 1e-3)
        out["fp64_full_reference"] = {"value": v64, "unit": "samples/s",
                                      "config": "plain full response, FP64, TDI 2.0, timed on "
                                                "1024 sources of each wave"}
        out["speedup_vs_fp64_full"] = value / v64
    print(json.dumps(out), flush=True)


def likelihood(args):
    """The likelihood's steps after the response on the 512-source batch: the
    FP32-bulk hybrid response written as A, E, T, then the noise-weighted inner
    products of data and template per source (TDI 2.0 PSDs with the galactic
    foreground, 1e-4..0.029 Hz).  The data are the responses of the same sources
    at a polarisation angle 0.01 rad away."""
    import torch
    from paper_2505_09600_amd import tdi
    from paper_2505_09600_amd import workload as W
    tdi.lib()
    dev = torch.device("cuda:0")
    batch, cfg, orb = W.config_c4(n_sources=args.n_sources, xp=torch, device=dev)
    total = batch.total
    hp, hc = batch.hp.contiguous(), batch.hc.contiguous()
    cfg32 = dict(cfg, precision=1, mode=2, tdi_gen=20, taps=TAPS, stencil_order=4, channels=1)
    src_h = tdi.make_sources(batch.sources)
    recs_d = batch.sources.copy()
    recs_d["psi"] = recs_d["psi"] + 0.01
    src_d = tdi.make_sources(recs_d)
    H = [torch.empty(total, dtype=torch.float32, device=dev) for _ in range(3)]
    D = [torch.empty(total, dtype=torch.float32, device=dev) for _ in range(3)]
    noise = dict(tdi_gen=20, galactic=1, T_obs_years=1.0, L_m=W.ARM_L, f_min=1e-4, f_max=0.029)
    n_max = int(np.max(np.diff(batch.offsets)))
    out = torch.empty((batch.n_sources, 3, 3), dtype=torch.float64, device=dev)
    with tdi.Plan(cfg32, orb, batch.n_sources, total, autotune=True, use_graph=True) as plan, \
            tdi.IpPlan(noise, tdi.TDI_FP32_BULK, 10.0, batch.n_sources, total, n_max) as ip:
        plan.run(src_d, batch.offsets, hp, hc, *D)
        for _ in range(args.warmup):
            plan.run(src_h, batch.offsets, hp, hc, *H)
            ip.run(batch.offsets, D, H, out)
        if plan.sync() != tdi.TDI_OK:
            raise RuntimeError("window check failed")
        plan.kernel_times()
        ip.kernel_times()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ip.run(batch.offsets, D, H, out)
        torch.cuda.synchronize()
        t_ip = (time.perf_counter() - t0) / args.steps
        kt_ip = ip.kernel_times()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.run(src_h, batch.offsets, hp, hc, *H)
            ip.run(batch.offsets, D, H, out)
        torch.cuda.synchronize()
        t_all = (time.perf_counter() - t0) / args.steps
        kt_resp = plan.kernel_times()
        ip.kernel_times()
        ipv = out.cpu().numpy()
    runs = len(kt_ip) // 3
    p1, p2, rd = (float(np.mean(kt_ip[j::3][:runs])) for j in range(3))
    runs_r = len(kt_resp) // 3
    r_fit, r_lfa, r_full = (float(np.mean(kt_resp[j::3][:runs_r])) for j in range(3))
    lnl = -0.5 * np.sum(ipv[:, :, 0] - 2.0 * ipv[:, :, 1] + ipv[:, :, 2], axis=1)
    ip_ms = p1 + p2 + rd
    gbs = 24.0 * total / (ip_ms * 1e-3) / 1e9
    res = {"metric": "likelihood steps after the response: samples/s (FP32)", "unit": "samples/s",
           "n_gpus": 1, "data": "synthetic", "higher_is_better": True, "steps": args.steps,
           "warmup": args.warmup,
           "config": {"workload": "512 sources of the batched hybrid benchmark (seed 1004), A, E, T "
                                  "written by the response, inner products against data at psi + 0.01",
                      "total_samples": total, "band_hz": [1e-4, 0.029], "tdi": "2.0", "galactic": True},
           "inner_product": {"value": total / t_ip, "ms_per_step": 1e3 * t_ip, "pass1_ms": p1,
                             "pass2_ms": p2, "reduce_ms": rd,
                             "hbm_algorithmic_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                             "bytes_per_sample_algorithmic": 24},
           "response_plus_inner_product": {"value": total / t_all, "ms_per_step": 1e3 * t_all,
                                           "response_kernels_ms": [r_fit, r_lfa, r_full]},
           "lnL_finite": bool(np.all(np.isfinite(lnl))), "lnL_first": [float(v) for v in lnl[:3]]}
    print(json.dumps(res), flush=True)


def link_outputs(args):
    """The six single-link outputs of the 512-source batch (FP32-bulk hybrid:
    the per-link LFA before the switch, the full links after it, blended per
    link), timed with HIP events on the plan's stream."""
    import torch
    from paper_2505_09600_amd import tdi
    from paper_2505_09600_amd import workload as W
    tdi.lib()
    dev = torch.device("cuda:0")
    batch, cfg, orb = W.config_c4(n_sources=args.n_sources, xp=torch, device=dev)
    total = batch.total
    hp, hc = batch.hp.contiguous(), batch.hc.contiguous()
    src = tdi.make_sources(batch.sources)
    res = {"metric": "single-link outputs: samples/s (six links per sample)", "unit": "samples/s",
           "n_gpus": 1, "data": "synthetic", "higher_is_better": True, "steps": args.steps,
           "warmup": args.warmup,
           "config": {"workload": "512 sources of the batched hybrid benchmark (seed 1004), six links "
                                  "per sample, 32 taps, 4th-order first-derivative stencil",
                      "total_samples": total}, "runs": {}}
    for name, prec, mode in (("hybrid fp32", 1, 2), ("lfa fp32", 1, 1), ("full fp32", 1, 0), ("full fp64", 0, 0)):
        c = dict(cfg, precision=prec, mode=mode, tdi_gen=20, taps=TAPS, stencil_order=4)
        y = torch.empty(6 * total, dtype=torch.float32 if prec else torch.float64, device=dev)
        steps = args.steps if prec else max(1, args.steps // 5)
        with tdi.Plan(c, orb, batch.n_sources, total) as plan:
            for _ in range(args.warmup):
                plan.run_links(src, batch.offsets, hp, hc, y)
            if plan.sync() != tdi.TDI_OK:
                raise RuntimeError("window check failed")
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                plan.run_links(src, batch.offsets, hp, hc, y)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            if plan.sync() != tdi.TDI_OK:
                raise RuntimeError("window check failed")
        bps = 16 + 6 * (4 if prec else 8)
        gbs = bps * total / (ms * 1e-3) / 1e9
        res["runs"][name] = {"ms_per_run": ms, "samples_per_s": total / (ms * 1e-3),
                             "hbm_algorithmic_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                             "bytes_per_sample_algorithmic": bps}
        print(f"[bench] links {name}: {ms:.2f} ms", file=sys.stderr, flush=True)
        del y
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-sources", type=int, default=512)
    ap.add_argument("--tile-chunks", type=int, default=0, choices=[0, 1, 2, 4],
                    help="LFA tile shape of the fast path (chunks of 2304 outputs); 0 = autotuned")
    ap.add_argument("--orbit", default="analytic", choices=["analytic", "table"],
                    help="c4: the first-order analytic orbit (default) or flexing Keplerian orbits "
                         "read from an hourly position table")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-reference", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the LFA variant timings")
    ap.add_argument("--cpu-budget", type=float, default=40.0,
                    help="about the total time of the timed oracle runs (s), over all modes")
    ap.add_argument("--steps-only", action="store_true", help="only the timed hybrid steps (profiling)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the steps, copy a float32 buffer of this size three times (a plain "
                         "copy kernel of known traffic for scaling PMC byte counters)")
    ap.add_argument("--config", default="c4", choices=["c1", "c2", "c3", "c4", "c5", "lnl", "links"],
                    help="c4 (default): the headline batched hybrid line; c1-c3: single-source "
                         "timings of every mode; c5: the 4096-source batch in two waves; lnl: the "
                         "inner products that follow the response on the c4 batch; links: the six "
                         "single-link outputs of the c4 batch")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: only --gpus 1 is supported; the response has no multi-GPU path "
              "(a batch would be sharded by source across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)
    if args.config == "lnl":
        likelihood(args)
        return
    if args.config == "links":
        link_outputs(args)
        return
    if args.config != "c4":
        secondary(args)
        return

    import torch
    from paper_2505_09600_amd import tdi
    from paper_2505_09600_amd import workload as W

    tdi.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    batch, cfg, orb = W.config_c4(n_sources=args.n_sources, xp=torch, device=dev)
    cfg = dict(cfg, fast_tile_chunks=args.tile_chunks)
    if args.orbit == "table":
        # eccentric Keplerian orbits sampled hourly, spanning the longest source
        span = float(np.max(np.diff(batch.offsets))) * 10.0
        t_lo, step = -2 * 86400.0, 3600.0
        orb = W.table_orbit(W.keplerian_orbit_table(t_lo, step, int((span + 4 * 86400.0) / step)), t_lo, step)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    total = batch.total
    print(f"[bench] workload: {batch.n_sources} sources, {total} samples, generated in {t_gen:.1f} s",
          file=sys.stderr, flush=True)
    hp, hc = batch.hp.contiguous(), batch.hc.contiguous()
    src = tdi.make_sources(batch.sources)
    n_full_region = sum(1 for r in batch.sources if math.isfinite(r["t_hyb"]))

    cfg32 = dict(cfg, precision=1, mode=2, tdi_gen=20, taps=TAPS, stencil_order=4)
    X = torch.empty(total, dtype=torch.float32, device=dev)
    Y = torch.empty_like(X)
    Z = torch.empty_like(X)
    plan = tdi.Plan(cfg32, orb, batch.n_sources, total, autotune=True, use_graph=True)
    print("[bench] warmup (first run autotunes)", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        plan.run(src, batch.offsets, hp, hc, X, Y, Z)
    st = plan.sync()
    if st != tdi.TDI_OK:
        raise RuntimeError(f"window check failed during warmup: {tdi.tdi_status_str(st)}")
    plan.kernel_times()                               # drop the warmup records
    # K timed steps; each step is synchronised so that its own wall time is known
    torch.cuda.synchronize()
    step_s = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        plan.run(src, batch.offsets, hp, hc, X, Y, Z)
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - a)
    t1 = time.perf_counter()
    ktimes = plan.kernel_times()
    st = plan.sync()
    if st != tdi.TDI_OK:
        raise RuntimeError(f"window check failed: {tdi.tdi_status_str(st)}")
    launch = plan.describe()
    finite = bool(torch.isfinite(X).all().item() and torch.isfinite(Y).all().item()
                  and torch.isfinite(Z).all().item())
    el = t1 - t0
    ms_step = 1e3 * float(np.median(step_s))
    value = total / (ms_step * 1e-3)
    runs = len(ktimes) // 3                           # (fit pre-pass, LFA kernel, full kernel) per run
    fit_ms, lfa_ms, full_ms = ((float(np.median(ktimes[j::3][:runs])) for j in range(3)) if runs
                               else (float("nan"),) * 3)
    if args.calib_copy_mib > 0:
        nel = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {nel * 4} bytes read and written per launch",
              file=sys.stderr, flush=True)
        del a, b
    if args.steps_only:
        print(json.dumps({"ms_per_step": ms_step, "kernel_ms": lfa_ms, "fit_kernel_ms": fit_ms,
                          "full_kernel_ms": full_ms, "samples": total, "launch": launch}), flush=True)
        return
    plan.close()

    print(f"[bench] hybrid FP32-bulk: {ms_step:.2f} ms/step (median; mean {1e3 * el / args.steps:.2f}), "
          f"fit pre-pass {fit_ms:.3f} ms, LFA kernel {lfa_ms:.3f} ms, full kernel {full_ms:.3f} ms, "
          f"launch {launch}", file=sys.stderr, flush=True)
    # FP64 on the same batch: the plain full response (the reference this path
    # must beat), and the FP64 LFA and hybrid of the same configuration
    fp64 = {}
    if not args.no_fp64_reference:
        X64 = torch.empty(total, dtype=torch.float64, device=dev)
        Y64 = torch.empty_like(X64)
        Z64 = torch.empty_like(X64)
        for name, mode in (("full", 0), ("lfa", 1), ("hybrid", 2)):
            c64 = dict(cfg, precision=0, mode=mode, tdi_gen=20, taps=TAPS, stencil_order=4)
            p64 = tdi.Plan(c64, orb, batch.n_sources, total, autotune=True, use_graph=True)
            p64.run(src, batch.offsets, hp, hc, X64, Y64, Z64)
            p64.sync()
            p64.kernel_times()
            reps = []
            for _ in range(3):
                torch.cuda.synchronize()
                r0 = time.perf_counter()
                p64.run(src, batch.offsets, hp, hc, X64, Y64, Z64)
                torch.cuda.synchronize()
                reps.append(time.perf_counter() - r0)
            if p64.sync() != tdi.TDI_OK:
                raise RuntimeError("window check failed (FP64)")
            p64.close()
            ms = 1e3 * float(np.median(reps))
            fp64[name] = {"value": total / (ms * 1e-3), "unit": "samples/s", "ms_per_step": ms,
                          "config": f"{name} response, FP64, TDI 2.0, same batch, median of 3"}
            print(f"[bench] FP64 {name}: {ms:.2f} ms/step", file=sys.stderr, flush=True)
        del X64, Y64, Z64
    ref = fp64.get("full")

    # LFA variants on the same batch and hybrid window: the next term of the
    # central expansion (lfa_terms = 2, general LFA kernel) and TDI 2.0 from the
    # TDI 1.5 LFA series (FP64 TDI 1.5 pass, then derivative and read)
    variants = {}
    if not args.no_variants:
        for vname, extra in (("lfa_next_term", {"lfa_terms": 2}), ("x20_from_x15", {"x20_from_x15": 1})):
            for prec in (1, 0):
                cv = dict(cfg32, precision=prec, **extra)
                dt_out = torch.float32 if prec else torch.float64
                Xv = torch.empty(total, dtype=dt_out, device=dev)
                Yv, Zv = torch.empty_like(Xv), torch.empty_like(Xv)
                pv = tdi.Plan(cv, orb, batch.n_sources, total, autotune=True, use_graph=True)
                pv.run(src, batch.offsets, hp, hc, Xv, Yv, Zv)
                pv.sync()
                pv.kernel_times()
                reps = []
                for _ in range(3):
                    torch.cuda.synchronize()
                    r0 = time.perf_counter()
                    pv.run(src, batch.offsets, hp, hc, Xv, Yv, Zv)
                    torch.cuda.synchronize()
                    reps.append(time.perf_counter() - r0)
                kv = pv.kernel_times()
                if pv.sync() != tdi.TDI_OK:
                    raise RuntimeError(f"window check failed ({vname})")
                pv.close()
                del Xv, Yv, Zv
                ms = 1e3 * float(np.median(reps))
                key = f"{vname}_{'fp32' if prec else 'fp64'}"
                variants[key] = {"value": total / (ms * 1e-3), "unit": "samples/s", "ms_per_step": ms,
                                 "kernel_ms": [round(float(np.median(kv[j::3])), 3) for j in range(3)],
                                 "config": f"hybrid TDI 2.0, {vname}, {'FP32-bulk' if prec else 'FP64'}, "
                                           "same batch, median of 3; kernel_ms = (pre-pass or TDI 1.5 "
                                           "pass, LFA kernel, full kernel)"}
                print(f"[bench] variant {key}: {ms:.2f} ms/step", file=sys.stderr, flush=True)

    # roofline of the dominant kernel: HBM (algorithmic 28 B per sample) is the
    # roof the path is measured against; the VALU issue rate says what binds it
    achieved_gbs = BYTES_PER_SAMPLE_FP32 * total / (lfa_ms * 1e-3) / 1e9 if lfa_ms > 0 else float("nan")
    khash = kernel_source_hash()
    ctr = load_counters(khash)
    kname = (("k_lfa_fast<32>" if launch.get("lfa_fast") else "k_lfa<32,float>") +
             ("" if launch.get("graph_kernel_events") else " (+ k_full: whole graph replay)"))
    valu = None
    if ctr:
        insts = float(ctr["valu_insts_per_launch"])
        valu = {"insts_per_launch": insts, "lane_slots_per_sample": insts * 64.0 / total,
                "issue_frac": insts * 4.0 / (VALU_SIMDS * CLOCK_HZ * lfa_ms * 1e-3),
                "source": "profiles/k_lfa_c4_counters.json (SQ_INSTS_VALU, same kernel source)"}
    flops = lfa_flops_per_sample(TAPS) * total
    alg_tflops = flops / (lfa_ms * 1e-3) / 1e12 if lfa_ms > 0 else float("nan")
    roof = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": (ctr["hbm_bytes_per_launch"] if ctr else None),
            "kernel": kname, "kernel_ms": lfa_ms, "fit_kernel_ms": fit_ms, "full_kernel_ms": full_ms,
            "bytes_per_sample": BYTES_PER_SAMPLE_FP32, "samples_per_launch": total,
            "valu": valu,
            "algorithmic_fp32": {"flops_per_sample": lfa_flops_per_sample(TAPS), "tflops": alg_tflops,
                                 "vs_nonpacked_peak": alg_tflops / FP32_NONPACKED_TFLOPS,
                                 "note": "per-sample count of six two-component 32-tap reads (4N + 4N flops each); "
                                         "the kernel executes fewer flops (one precombined series per "
                                         "link, shared table weights), so this ratio can exceed 1 and "
                                         "is not a hardware rate"},
            "kernel_hash": khash}

    cpu = None
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(7)
        order = rng.permutation(batch.n_sources)[:32]
        host_sub = W.config_c4(n_sources=args.n_sources, only=[int(i) for i in order])[0]
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        modes = {"full tdi1.5": dict(cfg32, precision=0, mode=0, tdi_gen=15),
                 "full tdi2.0": dict(cfg32, precision=0, mode=0, tdi_gen=20),
                 "lfa tdi2.0": dict(cfg32, precision=0, mode=1, tdi_gen=20),
                 "hybrid tdi2.0": dict(cfg32, precision=0, mode=2, tdi_gen=20)}
        cpu = cpu_baseline(host_sub, cfg32, orb, args.cpu_budget, modes)

    out = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "ms_per_step_mean": 1e3 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched hybrid TDI 2.0, 512 sources, lengths log-uniform 2^18..2^22 at "
                               "dt=10 s (seed 1004), FP32-bulk with FP64 delays and stencils"
                               + ("; Keplerian orbits from an hourly table" if args.orbit == "table" else ""),
                   "n_sources": batch.n_sources, "total_samples": total, "taps": TAPS,
                   "stencil_order": 4, "tdi": "2.0", "mode": "hybrid",
                   "sources_with_full_region": n_full_region, "launch": launch,
                   "outputs_finite": finite},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64_full_reference": ref,
        "fp64": fp64,
        "lfa_variants": variants,
        "speedup_vs_fp64_full": (value / ref["value"]) if ref else None,
        "speedup_vs_fp64_hybrid": (value / fp64["hybrid"]["value"]) if "hybrid" in fp64 else None,
    }
    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
