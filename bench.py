#!/usr/bin/env python3
"""Throughput of the batched matched-filter search on one MI355X.

One step is one pass of the whole search over one data chunk: segment
setup (PSD weighting and the FP64 running sum for sigma^2), the bank's
generator constants, and the search itself (on-chip chirp generation,
correlation, the inverse transform, |z|^2 peaks, threshold triggers per
window and their merge across templates).  Inputs are resident in HBM when
the timed region starts.  The default workload is the 2^20-sample (256 s at
4096 Hz), 1024-template FP32 search with five injections.

Prints one JSON line.  The dominant kernel's roofline figure uses its
algorithmic bytes per launch (the FP32 intermediate: 8 n bytes written by
pass 1 or read by pass 2, per template) over its average launch time,
measured with HIP events on the launch stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "templates/sec (N=2^20 SNR series) FP32 vs split-BF16 MFMA; % HBM roofline"
HBM_PEAK_GBS = 8000.0
# name -> (library precision code, dtype tag of the arithmetic)
PRECISIONS = {"fp32": (0, "f32"), "split-bf16": (1, "bf16x3"), "split-fp16": (2, "f16x3")}
# bytes of the intermediate per complex value (written by pass 1, read by
# pass 2): FP32 pairs, or FP16 pairs on the split-precision paths
Y_BYTES = {"fp32": 8, "split-bf16": 4, "split-fp16": 4}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fp32-2^20.json")
KERNEL_SOURCES = ["paper_1006_4644_amd/csrc/kernels.hip",
                  "paper_1006_4644_amd/csrc/fft_device.h",
                  "paper_1006_4644_amd/csrc/mfma_device.h"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the kernel sources' code: comments and whitespace runs are
    dropped first, so that an edit to a comment does not orphan the traffic
    figures measured on the same machine code."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    # default: 100 timed steps after 20 warm-ups (~0.4 s of timed work for
    # the 1024-template bank at 2^20; the first tens of milliseconds run
    # before the clocks settle), fewer for the workloads whose step is long
    p.add_argument("--steps", type=int, default=None)
    p.add_argument("--warmup", type=int, default=None)
    p.add_argument("--workload", default="fp32-2^20")
    p.add_argument("--batch", type=int, default=0, help="templates per batch (0: built-in)")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="time budget of the CPU oracle baseline")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-copy-probe", action="store_true")
    p.add_argument("--no-graph", action="store_true",
                   help="skip timing the headline search as graph replays")
    p.add_argument("--graph-replays", type=int, default=20)
    p.add_argument("--chunk", type=int, default=0,
                   help="also search the bank in resumable chunks of this many templates "
                        "(device merge across chunks) and compare with the single call")
    p.add_argument("--no-chisq", action="store_true",
                   help="skip timing the chi-squared veto at the per-template peaks")
    p.add_argument("--chisq-bands", type=int, default=16)
    p.add_argument("--no-td", action="store_true",
                   help="skip the paper's two-polarization time-domain template form")
    p.add_argument("--no-stream", action="store_true",
                   help="skip the continuous-stream leg (overlap-save segments from host samples)")
    p.add_argument("--stream-segments", type=int, default=16)
    p.add_argument("--no-bank", action="store_true",
                   help="skip the template-bank placement leg")
    p.add_argument("--precision", default="fp32", choices=sorted(PRECISIONS),
                   help="arithmetic of the headline run")
    p.add_argument("--no-split", action="store_true",
                   help="skip the comparison runs at the other precisions")
    p.add_argument("--tune-cache", default=os.environ.get("CI_TUNE_CACHE", ""),
                   help="JSON cache of autotuned launch configurations, keyed by device, "
                        "length and precision (default: $CI_TUNE_CACHE; empty: none)")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep the default launch configuration")
    p.add_argument("--tune", default="",
                   help="explicit launch configuration C,J,P2,BATCH[,STREAMS[,P2_WAVE]] "
                        "(skips the autotuner)")
    args = p.parse_args()
    # (steps, warmup) by workload: about a second of timed work or less
    long_steps = {"precision-2^20": (20, 5), "3g-2^21": (1, 1)}
    dsteps, dwarm = long_steps.get(args.workload, (100, 20))
    if args.steps is None:
        args.steps = dsteps
    if args.warmup is None:
        args.warmup = dwarm
    return args


def configure(ctx, ci, args, tune_calls):
    """Launch configuration per (length, precision): explicit, from the
    launch-configuration cache (--tune-cache, default $CI_TUNE_CACHE) when it
    holds this device's entry, autotuned (tune_calls: [(seg, params, n, thr,
    window, log2n)]; then written to the cache), or the default."""
    out = {}
    cached, key = set(), None
    if args.tune_cache and not args.tune and not args.no_autotune:
        key = ci.device_key(0)
        cached = set(ci.load_tune_cache(ctx, args.tune_cache, key))
        if cached:
            log(f"[bench] launch configurations from {args.tune_cache}: {sorted(cached)}")
    for prec_name, (prec, _) in PRECISIONS.items():
        if args.no_split and prec_name != args.precision:
            continue
        for seg, params, n, thr, window, l2 in tune_calls:
            if args.tune:
                v = [int(x) for x in args.tune.split(",")]
                ctx.set_tune(l2, prec, *v[:4], streams=v[4] if len(v) > 4 else 2,
                             p2_wave=v[5] if len(v) > 5 else 0)
                cfg = ctx.get_tune(l2, prec)
            elif args.no_autotune or (l2, prec) in cached:
                cfg = ctx.get_tune(l2, prec)
            else:
                cfg = ctx.autotune(seg, params, thr, window, n=n, precision=prec)
            out[f"{prec_name}/2^{l2}"] = {k: cfg[k] for k in
                                          ("tile_c", "tile_j", "p2_per_cu", "batch", "streams",
                                           "p2_wave", "tuned")}
            log(f"[bench] launch configuration {prec_name} 2^{l2}: {out[f'{prec_name}/2^{l2}']}")
    if key is not None:
        ci.save_tune_cache(ctx, args.tune_cache, key)
    return out


def inject_on_gpu(ctx, seg, xt, wl, injs):
    """Add the injections to the data spectrum, using the library's own
    materialised templates (unit amplitude, t_c = phi_c = 0), shifted to
    t_c = j0/fs and rotated by phi_c, scaled to the target optimal SNR."""
    import torch
    from paper_1006_4644_amd import ci
    if not injs:
        return xt
    ib = np.array([[i.m1, i.m2] for i in injs])
    p, ht = ctx.gen_templates(seg, ib, htilde=True)
    torch.cuda.synchronize()
    s2 = ci.params_to_numpy(p)["sigma2"]
    k = torch.arange(wl.n // 2 + 1, device=xt.device, dtype=torch.int64)
    acc = xt.to(torch.complex128)
    for i, inj in enumerate(injs):
        ph = 2 * math.pi * ((k * inj.j0) % wl.n).to(torch.float64) / wl.n - inj.phi
        rot = torch.polar(torch.ones_like(ph), -ph)
        acc = acc + ht[i].to(torch.complex128) * rot * (inj.snr / math.sqrt(s2[i]))
    return acc.to(torch.complex64).contiguous()


def copy_probe_gbs():
    """Achieved bandwidth of a plain 2 GiB device copy (read + write)."""
    import torch
    n = 1 << 28  # float64 elements = 2 GiB
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * (n * 8) / (ms / 1e3) / 1e9


def device_record(device=0):
    """The GPU the run used: name, architecture, compute units, memory, and
    (when rocm-smi answers within a few seconds) its clocks as read at the
    end of the run, after the timed work (idle levels, not the clocks of the
    timed steps)."""
    import subprocess
    import torch
    p = torch.cuda.get_device_properties(device)
    rec = {"name": p.name, "arch": getattr(p, "gcnArchName", ""),
           "compute_units": p.multi_processor_count,
           "memory_gib": round(p.total_memory / 2**30, 1)}
    # Under a profiler its preloaded library initialises the GPU in every
    # child process too, and rocm-smi's interpreter hop would then replace
    # such a process: no clock query there.
    if any(k.startswith("ROCPROF") for k in os.environ) or \
            "rocprof" in os.environ.get("LD_PRELOAD", ""):
        return rec
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True,
                           text=True, timeout=10)
        if r.returncode == 0:
            card = next(iter(json.loads(r.stdout).values()))
            rec["clocks_at_end"] = {k: v for k, v in card.items() if "clock" in k.lower()}
    except Exception:  # clocks are informational only
        pass
    return rec


def hbm_probes(ctx):
    """The device's streaming ceilings with the library's probe kernels
    (16-byte non-temporal accesses, 2 GiB per direction): write-only,
    read-only and copy (read plus written) in GB/s."""
    import torch
    nbytes = 1 << 31
    buf = torch.empty(2 * nbytes, dtype=torch.uint8, device="cuda")
    out = {}
    for kind, name in ((0, "write_gbs"), (1, "read_gbs"), (2, "copy_gbs")):
        out[name] = round(ctx.hbm_probe(kind, buf, nbytes, reps=10), 1)
    del buf
    torch.cuda.empty_cache()
    return out


def _oracle_templates(x, psd, wl, bank, idx, budget_s):
    """Run the FP64 oracle's full per-template search over bank[idx] until
    budget_s has elapsed; returns (templates done, seconds)."""
    from oracle import mf_oracle as O
    thr2 = wl.snr_threshold ** 2
    t0 = time.perf_counter()
    done = 0
    for i in idx:
        zs, s2 = O.snr_series(x, psd, wl.n, wl.fs, wl.f_low, *bank[i])
        r2 = zs.real ** 2 + zs.imag ** 2
        O.peak(r2)
        O.window_triggers(r2, wl.window, thr2)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    return done, time.perf_counter() - t0


def cpu_baseline(xt_host, psd, wl, bank, budget_s):
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    one thread."""
    rng = np.random.default_rng(2024)
    order = rng.permutation(len(bank))
    done, el = _oracle_templates(xt_host.astype(np.complex128), psd, wl, bank, order, budget_s)
    return {"value": done / el, "unit": "templates/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} seeded-random templates of the {wl.name} bank, "
                      f"full per-template search (series, peak, window triggers), "
                      f"FP64 numpy, one thread, {el:.1f} s"}


# All-core oracle baseline: worker processes forked before the GPU is
# touched, each holding the workload's inputs, each running the unchanged
# oracle on its own share of a seeded sample for the same wall-clock budget.
_W = {}


def _cpu_worker_init(wl_name):
    from paper_1006_4644_amd import synth
    wl = synth.WORKLOADS[wl_name]
    psd = synth.make_psd(wl.n, wl.fs)
    x = synth.make_noise(wl.n, wl.fs, wl.f_low, psd, wl.noise_seed).astype(np.complex128)
    bank = synth.draw_masses(wl.n_templates, wl.m_min, wl.m_max, wl.dist, wl.bank_seed)
    _W.update(wl=wl, psd=psd, x=x, bank=bank)


def _cpu_worker_run(args):
    idx, budget_s = args
    return _oracle_templates(_W["x"], _W["psd"], _W["wl"], _W["bank"], idx, budget_s)


def cpu_worker_count() -> int:
    """Host cores for the all-core leg: the process's CPU affinity, at most
    16 (one GPU's share of the host)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def start_cpu_pool(wl_name):
    import multiprocessing as mp
    k = cpu_worker_count()
    return mp.get_context("fork").Pool(k, initializer=_cpu_worker_init, initargs=(wl_name,)), k


def cpu_baseline_all(pool, k, wl, budget_s):
    """The oracle on k worker processes at once (noise-only spectrum of the
    workload: the oracle's cost does not depend on the data values)."""
    rng = np.random.default_rng(2025)
    order = rng.permutation(wl.n_templates)
    # each worker walks its share of the bank, cycling, until the budget ends
    shares = [(np.tile(order[i::k], 64), budget_s) for i in range(k)]
    res = pool.map(_cpu_worker_run, shares)
    done = sum(r[0] for r in res)
    # the workers run side by side: the aggregate rate is the sum of theirs
    rate = sum(r[0] / r[1] for r in res if r[1] > 0)
    el = max(r[1] for r in res)
    return {"value": rate, "unit": "templates/s", "cores": k,
            "sample": f"{done} seeded-random templates of the {wl.name} bank (noise-only "
                      f"spectrum), full per-template search, FP64 numpy, {k} processes "
                      f"of one thread side by side, {el:.1f} s each"}


def chunked_timing(ctx, ci, seg, bank, wl, prec, chunk, peaks, trig, count, cap):
    """The bank in chunks of `chunk` templates (generator constants, merged
    search and device merge per chunk, no checkpoint), timed once, and its
    results compared with the headline step's single call (the last step of
    the timed run left its outputs in peaks / trig / count)."""
    import torch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    p, m, k = ctx.search_bank_chunked(seg, bank, wl.snr_threshold, wl.window, chunk,
                                      precision=prec)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kk, kr = int(k.cpu()[0]), int(count.cpu()[0])
    same = kk == kr and torch.equal(p, peaks[:len(bank)]) and \
        torch.equal(m[:kk], trig[:min(kr, cap)])
    log(f"[bench] chunked ({chunk} templates per chunk): {ms:.1f} ms, same results: {same}")
    return {"chunk": chunk, "ms": round(ms, 2), "templates_per_s": round(len(bank) / (ms / 1e3), 1),
            "merged_windows": kk, "equal_to_single_call": bool(same)}


def graph_timing(ctx, seg, params, peaks, trig, count, cap, wl, prec, n_t, reps):
    """The headline search alone (segment and parameters resident) as one
    graph launch of the whole schedule, captured once and replayed: the
    median of `reps` individually timed replays after three warm-ups."""
    import torch
    job = [dict(seg=seg, params=params, n=n_t, cap=cap, peaks=peaks, trig=trig,
                count=count)]
    for _ in range(3):
        ctx.search_classes(job, wl.snr_threshold, wl.window, merge=True, precision=prec,
                           graph=True)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.search_classes(job, wl.snr_threshold, wl.window, merge=True, precision=prec,
                           graph=True)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    captures, launches = ctx.graph_stats()
    med = float(np.median(ms))
    log(f"[bench] graph replay: median {med:.3f} ms over {reps} replays "
        f"({captures} capture(s), {launches} launches)")
    return {"median_ms": round(med, 4), "min_ms": round(min(ms), 4),
            "max_ms": round(max(ms), 4), "replays": reps, "captures": captures,
            "templates_per_s": round(n_t / (med / 1e3), 1),
            "path_hbm_frac": round(2.0 * 8 * wl.n * n_t / (med / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
            if prec == 0 else None}


def chisq_timing(ctx, ci, seg, params, peaks, n_t, bands, reps=10):
    """Time the chi-squared veto at every template's peak (one entry per
    template) on torch's current stream, where the call is enqueued."""
    import torch
    out = torch.empty(n_t, dtype=torch.float64, device=peaks.device)
    for _ in range(2):
        ctx.chisq(seg, params, peaks, n_t, bands=bands, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.chisq(seg, params, peaks, n_t, bands=bands, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    P = ci.params_to_numpy(params)
    bins = int(np.sum(np.maximum(P["k_high"].astype(np.int64) - P["k_low"] + 1, 0)))
    c = out.cpu().numpy()
    fin = c[np.isfinite(c)]
    log(f"[bench] chi-squared veto: {n_t} peaks, {bands} bands, {ms:.3f} ms")
    return {"entries": n_t, "bands": bands, "ms_per_call": round(ms, 4),
            "entries_per_s": round(n_t / (ms / 1e3), 1),
            "bins_per_s": round(bins / (ms / 1e3), 1),
            "median_chi2_per_dof": round(float(np.median(fin)) / (2 * bands - 2), 3)
            if len(fin) else None}


def bank_timing(ctx, ci, lib, seg, xt, psd, psd_d, wl, cap, headline, probes=8):
    """A bank placed for the workload's mass range at 3 % mismatch (host),
    its merged search timed on the workload's data, and its coverage probed
    on the GPU: noise-free unit-SNR chirps of random masses in the range,
    whose largest peak over the bank is their best match."""
    import torch
    n, fs, fl = wl.n, wl.fs, wl.f_low
    t0 = time.perf_counter()
    bank = lib.make_bank_lattice(wl.m_min, wl.m_max, 0.97, psd, n, fs, fl)
    host_s = time.perf_counter() - t0
    ctx.segment_update(seg, xt, psd_d)
    params = ctx.gen_templates(seg, bank)
    peaks = torch.empty((len(bank), 4), dtype=torch.int64, device=xt.device)
    trig = torch.empty((cap, 4), dtype=torch.int64, device=xt.device)
    count = torch.zeros(1, dtype=torch.int64, device=xt.device)
    ctx.find_triggers(seg, params, wl.snr_threshold, wl.window, cap=cap, merge=True,
                      peaks=peaks, trig=trig, count=count)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.find_triggers(seg, params, wl.snr_threshold, wl.window, cap=cap, merge=True,
                      peaks=peaks, trig=trig, count=count)
    e1.record()
    torch.cuda.synchronize()
    search_ms = e0.elapsed_time(e1)
    rng = np.random.default_rng(wl.bank_seed + 5)
    best = []
    for _ in range(probes):
        lm = np.exp(rng.uniform(math.log(wl.m_min), math.log(wl.m_max), 2))
        m1, m2 = float(lm.max()), float(lm.min())
        p1, ht = ctx.gen_templates(seg, [[m1, m2]], htilde=True)
        torch.cuda.synchronize()
        s2 = float(ci.params_to_numpy(p1)["sigma2"][0])
        x = (ht[0] / math.sqrt(s2)).contiguous()
        ctx.segment_update(seg, x, psd_d)
        prm = ctx.gen_templates(seg, bank)
        ctx.find_triggers(seg, prm, 0.5, n, cap=16, peaks=peaks)
        torch.cuda.synchronize()
        best.append(math.sqrt(float(ci.triggers_to_numpy(peaks)["rho2"].max())))
    ctx.segment_update(seg, xt, psd_d)
    log(f"[bench] bank: {len(bank)} templates placed in {host_s:.2f} s, search "
        f"{search_ms:.1f} ms, best match over {probes} probes >= {min(best):.4f}")
    return {"templates": int(len(bank)), "min_match": 0.97, "place_s": round(host_s, 3),
            "mass_range": [wl.m_min, wl.m_max], "search_ms": round(search_ms, 3),
            "templates_per_s": round(len(bank) / (search_ms / 1e3), 1),
            "probe_best_match_min": round(min(best), 5),
            "probe_best_match_median": round(float(np.median(best)), 5), "probes": probes}


def stream_timing(args, ctx, ci, bank, wl, headline):
    """Continuous stream: float32 strain pushed from host memory in chunks
    of 2^18 samples, overlap-save segments of n with stride n/2, per
    segment the spectrum, the PSD estimate, the templates' sigma^2 and the
    merged search of the bank over the valid half.  Timed from the first
    push to the last segment's triggers on the host."""
    import torch
    from paper_1006_4644_amd import synth
    n, fs = wl.n, wl.fs
    warm, K = 2, max(2, args.stream_segments)
    total = n + (warm + K - 1) * n // 2
    # coloured Gaussian noise of the workload's PSD as a time series
    xt = synth.make_noise(total, fs, wl.f_low, synth.make_psd(total, fs), wl.noise_seed + 77)
    x = (np.fft.irfft(xt, total) * fs).astype(np.float32)
    first = n + (warm - 1) * n // 2
    chunk = 1 << 18
    res = {}
    for tag, prec in (("fp32", ci.FP32), ("split-bf16", ci.SPLIT_BF16)):
        st = ctx.stream(bank, n, fs, wl.f_low, wl.snr_threshold, wl.window, psd_half_width=16,
                        cap=1 << 12, precision=prec)
        st.push(x[:first])
        st.poll(wait=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a in range(first, total, chunk):
            st.push(x[a:a + chunk])
        trig, done, flags = st.poll(wait=True)
        dt = time.perf_counter() - t0
        st.close()
        segs = done - warm
        v = segs * len(bank) / dt
        log(f"[bench] stream ({tag}): {segs} segments in {dt * 1e3:.1f} ms, {v:.0f} templates/s")
        res[tag] = (segs, dt, v, trig, flags)
    segs, dt, v, trig, flags = res["fp32"]
    return {"segments": segs, "n": n, "stride": n // 2, "ms_per_segment": round(dt * 1e3 / segs, 3),
            "templates_per_s": round(v, 1), "vs_headline": round(v / headline, 3),
            "realtime_factor": round(segs * (n // 2) / fs / dt, 1),
            "merged_triggers": int(len(trig)), "overflow": int(flags & 1),
            "split_bf16_templates_per_s": round(res["split-bf16"][2], 1)}


def td_timing(args, ctx, ci, seg, xt, psd_d, bank, n_t, cap, peaks, trig, count, wl,
              headline):
    """The same step with the paper's own template form: time-domain
    two-polarization templates generated, transformed and normalised per
    batch, correlated, two real inverse transforms packed into one, merged
    search.  Bytes per template that the form moves through HBM: template
    transform 24n (u generated inside its first pass), sigma^2 8n, pass 1
    16n (both mirror bins) + 8n, pass 2 8n: 56n in all."""
    import torch
    tdp = ctx.td_params(seg, bank)

    def step():
        ctx.segment_update(seg, xt, psd_d)
        ctx.td_params(seg, bank, out=tdp)
        ctx.td_find_triggers(seg, tdp, wl.snr_threshold, wl.window, cap=cap, merge=True,
                             peaks=peaks, trig=trig, count=count)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    steps = max(2, args.steps // 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    v = n_t / (ms / 1e3)
    gbs = 56.0 * wl.n * n_t / (ms / 1e3) / 1e9
    log(f"[bench] two-polarization form: {ms:.3f} ms/step, {v:.0f} templates/s")
    return {"value": round(v, 1), "unit": "templates/s", "ms_per_step": round(ms, 4),
            "steps": steps, "vs_headline": round(v / headline, 3),
            "model_bytes_per_template": 56 * wl.n, "model_gbs": round(gbs, 1),
            "model_frac": round(gbs / HBM_PEAK_GBS, 4),
            "merged_windows": int(count.cpu()[0])}


def run_classes(args, lib, ctx, wl):
    """The uneven bank in length classes: one segment per class, the whole
    schedule in one multi-class search per step."""
    import torch
    from paper_1006_4644_amd import ci, synth
    bank = synth.draw_masses(wl.n_templates, wl.m_min, wl.m_max, wl.dist, wl.bank_seed)
    classes = synth.CLASS_LENGTHS
    cls = lib.length_classes(bank, wl.fs, wl.f_low, classes)
    dev = torch.device("cuda", 0)
    cap = 1 << 16
    inputs, jobs, tune_calls, sizes = [], [], [], {}
    for c, n in enumerate(classes):
        idx = np.nonzero(cls == c)[0]
        if len(idx) == 0:
            continue
        psd = synth.make_psd(n, wl.fs)
        x = synth.make_noise(n, wl.fs, wl.f_low, psd, synth.class_noise_seed(wl, c))
        psd_d = torch.from_numpy(psd).cuda()
        xt = torch.from_numpy(x.astype(np.complex64)).cuda()
        seg = ctx.segment(xt, psd_d, n, wl.fs, wl.f_low)
        params = torch.empty((len(idx), 96), dtype=torch.uint8, device=dev)
        ctx.gen_templates(seg, bank[idx], out=params)
        jobs.append(dict(seg=seg, params=params, n=len(idx), cap=cap,
                         peaks=torch.empty((len(idx), 4), dtype=torch.int64, device=dev),
                         trig=torch.empty((cap, 4), dtype=torch.int64, device=dev),
                         count=torch.zeros(1, dtype=torch.int64, device=dev)))
        inputs.append((seg, xt, psd_d, bank[idx], params))
        tune_calls.append((seg, params, min(len(idx), 2048), wl.snr_threshold, wl.window,
                           n.bit_length() - 1))
        sizes[f"2^{n.bit_length() - 1}"] = int(len(idx))
    log(f"[bench] workload {wl.name}: classes {sizes}")
    tune_cfg = configure(ctx, ci, args, tune_calls)
    alg_bytes = {tag: sum(2.0 * Y_BYTES[tag] * jb["seg"].n * jb["n"] for jb in jobs)
                 for tag in PRECISIONS}

    def step(prec):
        for seg, xt, psd_d, b, params in inputs:
            ctx.segment_update(seg, xt, psd_d)
            ctx.gen_templates(seg, b, out=params)
        ctx.search_classes(jobs, wl.snr_threshold, wl.window, merge=True, precision=prec)

    def timed(prec, tag):
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            step(prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        v = wl.n_templates / (ms / 1e3)
        gbs = alg_bytes[tag] / (ms / 1e3) / 1e9
        log(f"[bench] {tag}: {ms:.3f} ms/step, {v:.0f} templates/s, {gbs:.0f} GB/s")
        return ms, v, gbs

    prec_code, dtype = PRECISIONS[args.precision]
    ms, value, gbs = timed(prec_code, args.precision)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "templates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": wl.name, "classes": sizes, "fs": wl.fs, "f_low": wl.f_low,
                   "templates": wl.n_templates,
                   "masses": f"{wl.dist} [{wl.m_min}, {wl.m_max}]",
                   "snr_threshold": wl.snr_threshold, "window": wl.window, "merge": True,
                   "precision": args.precision},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole schedule (intermediate bytes: 2 x 8 n_c per "
                               "template at FP32, 2 x 4 n_c on the split paths)"},
        "launch_config": tune_cfg,
    }
    if not args.no_split:
        paths = {}
        for tag, (prec, _) in PRECISIONS.items():
            if tag == args.precision:
                continue
            ms2, v2, gbs2 = timed(prec, tag)
            paths[tag] = {"value": round(v2, 1), "ms_per_step": round(ms2, 4),
                          "speedup_vs_headline": round(v2 / value, 3),
                          "path_hbm_frac": round(gbs2 / HBM_PEAK_GBS, 4)}
        out["precision_paths"] = paths
    out["device"] = device_record(0)
    for seg, *_ in inputs:
        seg.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the search "
              "shards by template bank across GPUs; the benchmark measures one "
              "GPU's share.", file=sys.stderr)
        sys.exit(2)

    # the all-core CPU baseline's workers are forked before anything touches
    # the GPU
    pool, pool_k = None, 0
    if not args.no_cpu_baseline and args.workload != "batched-classes":
        pool, pool_k = start_cpu_pool(args.workload)

    import torch
    from paper_1006_4644_amd import ci, synth

    lib = ci.load()
    ctx = lib.context(0)
    if args.batch:
        ctx.set_batch(args.batch)
    wl = synth.WORKLOADS[args.workload]
    if wl.name == "batched-classes":
        return run_classes(args, lib, ctx, wl)
    bank = synth.draw_masses(wl.n_templates, wl.m_min, wl.m_max, wl.dist, wl.bank_seed)
    injs = synth.draw_injections(wl, bank)
    psd = synth.make_psd(wl.n, wl.fs)
    noise = synth.make_noise(wl.n, wl.fs, wl.f_low, psd, wl.noise_seed)
    psd_d = torch.from_numpy(psd).cuda()
    xt = torch.from_numpy(noise.astype(np.complex64)).cuda()
    seg = ctx.segment(xt, psd_d, wl.n, wl.fs, wl.f_low)
    xt = inject_on_gpu(ctx, seg, xt, wl, injs)
    ctx.segment_update(seg, xt, psd_d)
    n_t = len(bank)
    cap = 1 << 20
    device = torch.device("cuda", 0)
    params = torch.empty((n_t, 96), dtype=torch.uint8, device=device)
    peaks = torch.empty((n_t, 4), dtype=torch.int64, device=device)
    trig = torch.empty((cap, 4), dtype=torch.int64, device=device)
    count = torch.zeros(1, dtype=torch.int64, device=device)
    log(f"[bench] workload {wl.name}: n={wl.n}, {n_t} templates, {len(injs)} injections")
    ctx.gen_templates(seg, bank, out=params)
    n_tune = min(n_t, 2048)
    tune_cfg = configure(ctx, ci, args, [(seg, params, n_tune, wl.snr_threshold, wl.window,
                                          wl.n.bit_length() - 1)])

    def step(precision):
        ctx.segment_update(seg, xt, psd_d)
        ctx.gen_templates(seg, bank, out=params)
        ctx.find_triggers(seg, params, wl.snr_threshold, wl.window, cap=cap, merge=True,
                          peaks=peaks, trig=trig, count=count, precision=precision)

    def timed(precision, tag):
        for _ in range(args.warmup):
            step(precision)
        torch.cuda.synchronize()
        log(f"[bench] {tag}: warmup done ({args.warmup} steps)")
        ctx.set_timing(True)
        ctx.kernel_times()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            step(precision)
        e1.record()
        torch.cuda.synchronize()
        total_ms = e0.elapsed_time(e1)
        kt = ctx.kernel_times()
        ctx.set_timing(False)
        found = int(count.cpu()[0])
        pk = ci.triggers_to_numpy(peaks).copy()
        log(f"[bench] {tag}: {args.steps} steps, {total_ms / args.steps:.3f} ms/step, "
            f"{n_t * args.steps / (total_ms / 1e3):.0f} templates/s, {found} merged windows")
        return total_ms, kt, found, pk

    prec_code, dtype = PRECISIONS[args.precision]
    total_ms, kt, nwin_found, pk32 = timed(prec_code, args.precision)
    ms_step = total_ms / args.steps
    value = n_t * args.steps / (total_ms / 1e3)

    # roofline of the dominant kernel
    name = max(kt, key=lambda k: kt[k][2])
    launches, tmpls, kms = kt[name]
    per_launch_ms = kms / launches
    bytes_per_launch = Y_BYTES[args.precision] * wl.n * (tmpls / launches)
    achieved = bytes_per_launch / (per_launch_ms / 1e3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        tp = tr.get("paths", {}).get(args.precision, {})
        if tp.get("source_hash") == kernel_source_hash() and name in tp.get("kernels", {}):
            k = tp["kernels"][name]
            traffic = k["bytes_per_template"] * (tmpls / launches)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": name,
                "avg_launch_ms": round(per_launch_ms, 4),
                "templates_per_launch": tmpls / launches}
    path_gbs = 2.0 * Y_BYTES[args.precision] * wl.n * n_t / (ms_step / 1e3) / 1e9
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "templates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "fs": wl.fs, "f_low": wl.f_low,
                   "templates": n_t, "masses": f"{wl.dist} [{wl.m_min}, {wl.m_max}]",
                   "injections": len(injs), "snr_threshold": wl.snr_threshold,
                   "window": wl.window, "merge": True, "precision": args.precision},
        "roofline": roofline,
        "path_hbm": {"algorithmic_bytes_per_template": 2 * Y_BYTES[args.precision] * wl.n,
                     "achieved_gbs": round(path_gbs, 1),
                     "frac": round(path_gbs / HBM_PEAK_GBS, 4)},
        "kernels_ms_per_step": {k: round(v[2] / args.steps, 4) for k, v in kt.items()},
        "merged_windows": nwin_found,
        "launch_config": tune_cfg,
    }
    if args.chunk > 0:
        # before the other precisions overwrite the headline run's outputs
        out["chunked"] = chunked_timing(ctx, ci, seg, bank, wl, prec_code, args.chunk,
                                        peaks, trig, count, cap)
    if not args.no_split:
        # the other arithmetic paths on the same workload; accuracy against
        # the FP64 oracle is checked by the test-suite, here the peak SNR of
        # each injection's template is compared with the headline run's
        paths = {}
        for tag, (prec, _) in PRECISIONS.items():
            if tag == args.precision:
                continue
            tms, kts, found, pks = timed(prec, tag)
            v = n_t * args.steps / (tms / 1e3)
            dev = max(abs(math.sqrt(pks["rho2"][i.tmpl]) - math.sqrt(pk32["rho2"][i.tmpl]))
                      / math.sqrt(pk32["rho2"][i.tmpl]) for i in injs if i.tmpl >= 0) \
                if any(i.tmpl >= 0 for i in injs) else None
            # the path's dominant kernel against the HBM roofline, and the
            # matrix-core rate of its second pass (radix-16 DFT-matrix
            # stages: 12 R3 16x16x32 products of 16384 flops per column of
            # N1 = 256 R3 points, N2 columns per template)
            dn = max(kts, key=lambda k: kts[k][2])
            dl, dt, dk = kts[dn]
            d_ach = Y_BYTES[tag] * wl.n * (dt / dl) / (dk / dl / 1e3) / 1e9
            lg = int(round(math.log2(wl.n)))
            n1 = 1 << ((lg + 1) // 2)
            mx_flop = 12 * (n1 // 256) * 16384 * (wl.n // n1)
            pl, pt, pk_ms = kts["pass2"]
            mx_tf = mx_flop * (pt / pl) / (pk_ms / pl / 1e3) / 1e12
            paths[tag] = {"value": round(v, 1), "ms_per_step": round(tms / args.steps, 4),
                          "speedup_vs_headline": round(v / value, 3),
                          "roofline": {"bound": "hbm", "achieved": round(d_ach, 1),
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": round(d_ach / HBM_PEAK_GBS, 4), "kernel": dn,
                                       "avg_launch_ms": round(dk / dl, 4),
                                       "templates_per_launch": dt / dl},
                          "mfma_pass2": ({"achieved": round(mx_tf, 1), "peak": 2500.0,
                                          "unit": "TFLOP/s", "frac": round(mx_tf / 2500.0, 4),
                                          "flop_per_template": mx_flop}
                                         if tag != "fp32" else None),
                          "path_hbm_frac": round(2.0 * Y_BYTES[tag] * wl.n * n_t
                                                 / (tms / args.steps / 1e3) / 1e9
                                                 / HBM_PEAK_GBS, 4),
                          "kernels_ms_per_step": {k: round(x[2] / args.steps, 4)
                                                  for k, x in kts.items()},
                          "injection_peak_rho_rel_dev_vs_headline": dev,
                          "merged_windows": found}
        out["precision_paths"] = paths
    # the graph leg times the headline-sized bank (a replay of a large bank
    # would take seconds each)
    if not args.no_graph and n_t <= 4096:
        out["graph_replay"] = graph_timing(ctx, seg, params, peaks, trig, count, cap, wl,
                                           prec_code, n_t, args.graph_replays)
    if not args.no_chisq:
        out["chisq_veto"] = chisq_timing(ctx, ci, seg, params, peaks, n_t, args.chisq_bands)
    if not args.no_stream:
        out["stream"] = stream_timing(args, ctx, ci, bank, wl, value)
    if not args.no_bank:
        out["bank_placement"] = bank_timing(ctx, ci, lib, seg, xt, psd, psd_d, wl, cap, value)
    if not args.no_td:
        out["two_polarization"] = td_timing(args, ctx, ci, seg, xt, psd_d, bank, n_t, cap,
                                            peaks, trig, count, wl, value)
    if not args.no_copy_probe:
        out["copy_probe_gbs"] = round(copy_probe_gbs(), 1)
        out["hbm_probes"] = hbm_probes(ctx)
        log(f"[bench] streaming ceilings: {out['hbm_probes']}")
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        cb = cpu_baseline(xt.cpu().numpy(), psd, wl, bank, args.cpu_seconds)
        single = dict(cb)
        if pool is not None:
            allc = cpu_baseline_all(pool, pool_k, wl, args.cpu_seconds)
            pool.close()
            pool.join()
            # the reported baseline uses every core it was given; the
            # one-thread rate stays beside it
            cb = {"value": allc["value"], "unit": "templates/s", "cores": allc["cores"],
                  "kind": "oracle", "sample": allc["sample"],
                  "single_core": {"value": single["value"], "cores": 1,
                                  "sample": single["sample"]},
                  "all_core": allc, "host_cpus": os.cpu_count(),
                  "gpu_speedup_vs_all_core": round(value / allc["value"], 1),
                  "gpu_speedup_vs_single_core": round(value / single["value"], 1)}
        out["cpu_baseline"] = cb
    out["device"] = device_record(0)
    seg.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
