#!/usr/bin/env python3
"""Throughput of the whole per-block path on one MI355X.

Workload: FAST-shaped block, 19 beams x 4096 channels of uint8 total power,
49.152 us samples, 10 s of data (203,450 samples), 2048-sample sub-intervals
(99 full sub-intervals; the 698-sample tail is not a full cell), synthetic
(seeded, generated on the GPU, device-resident before timing). One step is
one pass of the whole path over the block, by default the single call

    rfi_process_block   (sums -> eigen -> clip, sub-interval groups pipelined)

or, with --path stages, the three calls

    rfi_ccm_accumulate -> rfi_eig_batched -> rfi_flag

Metric: beam-sample GB/s = nbeam * nchan * nsub * L bytes / step time.
The roofline object is for the dominant kernel, timed with HIP events around
its own launches in the three-call path (one launch per step over the whole
block). Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
FP32_VALU_PEAK = 78.6e12       # non-packed FP32 FMA: 256 CU x 64 lanes x 2 x 2.4 GHz


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(spec, nsub_sample: int, nchan_sample: int):
    """The FP64 oracle, as it stands, on a bounded sample: the first
    nchan_sample channels of the first nsub_sample sub-intervals (bytes
    regenerated on the CPU)."""
    from oracle import pipeline
    from paper_2512_16278_amd import synth
    L = spec.L
    t0 = time.perf_counter()
    x = synth.generate(spec, 0, nsub_sample * L, 0, nchan_sample)
    tgen = time.perf_counter() - t0
    log(f"cpu baseline: sample generated in {tgen:.1f} s; running the oracle")
    t0 = time.perf_counter()
    cr, res, _ = pipeline.block(x, L, nsub_sample)
    dt = time.perf_counter() - t0
    nbytes = x.size
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    return {
        "value": nbytes / dt / 1e9, "unit": "GB/s", "cores": int(cores), "kind": "oracle",
        "sample": f"channels 0..{nchan_sample - 1} x {nsub_sample} sub-int(s) of {L} samples x "
                  f"{spec.nbeam} beams ({nbytes / 1e6:.0f} MB, {nsub_sample * nchan_sample} cells); "
                  f"oracle {dt:.2f} s, input generation {tgen:.1f} s not timed",
        "seconds": dt,
    }


MIX_NBEAM = (7, 19, 36, 72)
MIX_NCHAN = (1024, 4096, 8192)
MIX_L = (512, 1024, 4096)


def precision_split(dev, spec, data, blk, nsub, ev_time):
    """Precision split on the FAST-shaped block: exact int32 sums by the int8
    MFMA engine vs the dot4 VALU engine (bit-exact, timed); FP32 Jacobi, FP32
    Householder + Sturm and FP64 Jacobi on the GPU (timed), each against the
    FP64 oracle on sampled cells (per-cell eigenvalue error, residual of the
    dominant pair), and statistic and mask differences from the FP64 Jacobi
    over every cell."""
    import torch
    from oracle import pipeline
    from paper_2512_16278_amd import rfi, synth
    nb, nc, L = spec.nbeam, spec.nchan, spec.L
    ncell = nsub * nc
    npair = nb * (nb + 1) // 2
    sums = {}
    times = {}
    for name, var in (("mfma", rfi.RFI_CCM_MFMA), ("valu", rfi.RFI_CCM_VALU)):
        sx = torch.empty((nb, ncell), dtype=torch.int32, device=dev)
        sxy = torch.empty((npair, ncell), dtype=torch.int32, device=dev)
        cnt = torch.empty(nsub, dtype=torch.int32, device=dev)
        times[f"ccm_{name}_ms"] = ev_time(lambda: rfi.rfi_ccm_accumulate(
            blk, 0, L, nsub, sx, sxy, cnt, variant=var))
        sums[name] = (sx, sxy, cnt)
    exact = bool(torch.equal(sums["mfma"][0], sums["valu"][0]) and
                 torch.equal(sums["mfma"][1], sums["valu"][1]))
    del sums["valu"]
    sx, sxy, cnt = sums["mfma"]
    # (name, precision, solver): the FP32 per-lane Jacobi, the FP32 per-lane
    # Householder + Sturm solver (the default below 21 beams), the FP64 Jacobi
    runs = (("fp32", 32, rfi.RFI_EIG_LANE), ("fp32_householder", 32, rfi.RFI_EIG_LANE_TRI),
            ("fp64", 64, rfi.RFI_EIG_WAVE))
    res = {}
    for name, prec, solver in runs:
        stat = torch.empty(ncell, dtype=torch.float64, device=dev)
        status = torch.empty(ncell, dtype=torch.uint8, device=dev)
        ev = torch.empty((nb, ncell), dtype=torch.float32, device=dev)
        v1 = torch.empty((nb, ncell), dtype=torch.float32, device=dev)
        mask = torch.empty(ncell, dtype=torch.uint8, device=dev)
        times[f"eig_{name}_ms"] = ev_time(lambda: rfi.rfi_eig_batched(
            nb, nsub, nc, sx, sxy, cnt, stat, status, eigvals=ev, v1=v1, precision=prec,
            solver=solver))
        times[f"eig_{name}_stat_only_ms"] = ev_time(lambda: rfi.rfi_eig_batched(
            nb, nsub, nc, sx, sxy, cnt, stat, status, precision=prec, solver=solver))
        rfi.rfi_eig_batched(nb, nsub, nc, sx, sxy, cnt, stat, status, eigvals=ev, v1=v1,
                            precision=prec, solver=solver)
        rfi.rfi_flag(nsub, nc, stat, status, mask)
        torch.cuda.synchronize()
        res[name] = dict(stat=stat.cpu().numpy().reshape(nsub, nc),
                         ev=ev.cpu().numpy().reshape(nb, nsub, nc),
                         v1=v1.cpu().numpy().reshape(nb, nsub, nc),
                         status=status.cpu().numpy(), mask=mask.cpu().numpy())
    mask_diff = int(np.count_nonzero(res["fp32"]["mask"] != res["fp64"]["mask"]))
    # sampled cells against the oracle
    k, c_hi = 0, 256
    x = synth.generate(spec, k * L, (k + 1) * L, 0, c_hi)
    cr = pipeline.cells(x, L, 1)
    w_ref = cr.w[0]                                  # [c, n], |lambda| descending
    r_ref = cr.r[0]                                  # [c, n, n]
    out = {"sums_bit_exact_mfma_vs_valu": exact, "mask_disagreements_fp32_vs_fp64": mask_diff,
           "cells": ncell, "sample": f"sub-interval {k}, channels 0..{c_hi - 1} ({c_hi} cells)"}
    for name, prec, solver in runs:
        ev = res[name]["ev"][:, k, :c_hi].T.astype(np.float64)       # [c, n]
        v = res[name]["v1"][:, k, :c_hi].T.astype(np.float64)
        lam1 = w_ref[:, :1]
        nrel = np.abs(ev - w_ref) / np.abs(lam1)
        erel = np.abs(ev - w_ref) / np.abs(w_ref)
        s_err = np.abs(res[name]["stat"][k, :c_hi] - cr.stat[0])
        resid = np.linalg.norm(np.einsum("cab,cb->ca", r_ref, v) - ev[:, :1] * v, axis=1)
        out[name] = {
            "eig_norm_rel_max": float(nrel.max()), "eig_elem_rel_max": float(erel.max()),
            "stat_abs_max": float(s_err.max()), "resid_max": float(resid.max()),
            "not_converged": int(np.count_nonzero(res[name]["status"] & rfi.RFI_CELL_NOT_CONVERGED)),
            # over every cell of the block, against the FP64 Jacobi
            "stat_vs_fp64_all_cells_max": float(np.abs(res[name]["stat"] - res["fp64"]["stat"]).max()),
            "mask_vs_fp64_all_cells": int(np.count_nonzero(res[name]["mask"] != res["fp64"]["mask"])),
        }
    out.update({k2: round(v2, 4) for k2, v2 in times.items()})
    return out


def batch_bench(dev, nblocks=24, seed=11):
    """Uneven blocks (beam counts 7/19/36/72, channels 1024/4096/8192, L
    512/1024/4096, 0.1-2 s each) through (a) one rfi_process_block per
    block on one stream, (b) one rfi_process_batch, (c) one replay of the
    batch's HIP graph. Same blocks, same outputs; throughput in beam-sample
    GB/s of the full sub-intervals."""
    import torch
    from paper_2512_16278_amd import rfi, synth
    rng = np.random.default_rng(seed)
    pools = {}
    for F in MIX_NCHAN:
        spec = synth.mixed_spec(seed + F, max(MIX_NBEAM), F, 512, 2.1)
        t = torch.empty((spec.nbeam, spec.nsamp, F), dtype=torch.uint8, device=dev)
        ds = rfi.DeviceSynth(spec, dev)
        for b in range(spec.nbeam):
            ds.fill(t[b], b)
        pools[F] = t
    items, blocks, nbytes = [], [], 0
    per_class = {}
    for _ in range(nblocks):
        nb, F, L = int(rng.choice(MIX_NBEAM)), int(rng.choice(MIX_NCHAN)), int(rng.choice(MIX_L))
        nsamp = int(rng.uniform(0.1, 2.0) / synth.TSAMP)
        nsub = nsamp // L
        if nsub == 0:
            continue
        start = int(rng.integers(0, pools[F].shape[1] - nsamp))
        pool = pools[F]
        blk = rfi.make_block([pool[b, start:start + nsamp] for b in range(nb)], F)
        n = nsub * F
        it = dict(blk=blk, L=L, nsub=nsub,
                  stat=torch.empty(n, dtype=torch.float64, device=dev),
                  status=torch.empty(n, dtype=torch.uint8, device=dev),
                  mask=torch.empty(n, dtype=torch.uint8, device=dev))
        items.append(it)
        nbytes += nb * F * nsub * L
        per_class[nb] = per_class.get(nb, 0) + nb * F * nsub * L
    stream = torch.cuda.current_stream()
    wss = []
    for it in items:
        p = rfi.process_params(it["L"], it["nsub"])
        nbm = it["blk"].nbeam
        wss.append((p, torch.empty(rfi.rfi_process_workspace_size(nbm, it["blk"].nchan, p),
                                   dtype=torch.uint8, device=dev)))

    def separate():
        for it, (p, ws) in zip(items, wss):
            rfi.rfi_process_block(it["blk"], p, it["stat"], it["status"], it["mask"], ws)

    bt = rfi.Batch(items)
    bws = torch.empty(bt.workspace_size(), dtype=torch.uint8, device=dev)
    g = bt.graph(bws)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    t_sep = timed(separate)
    t_bat = timed(lambda: bt.run(bws))
    t_gr = timed(lambda: g.launch())
    g.close()
    # autotuner: per shape class, on the block with the most cells of the class
    sample = {}
    for it in items:
        nb = it["blk"].nbeam
        c = (nb + 16) // 16
        if c not in sample or it["nsub"] * it["blk"].nchan > sample[c]["nsub"] * sample[c]["blk"].nchan:
            sample[c] = it
    st = rfi.Batch(list(sample.values()))
    sws = torch.empty(st.workspace_size(), dtype=torch.uint8, device=dev)
    t0 = time.perf_counter()
    table = st.tune(sws)
    tune_s = time.perf_counter() - t0
    del sws
    tb = rfi.Batch(items, tune=table)
    tws = bws if tb.workspace_size() <= bws.numel() else torch.empty(
        tb.workspace_size(), dtype=torch.uint8, device=dev)
    tg = tb.graph(tws)
    t_tg = timed(lambda: tg.launch())
    tg.close()
    out = {"blocks": len(items), "bytes_gb": round(nbytes / 1e9, 2),
           "bytes_by_nbeam_gb": {str(k): round(v / 1e9, 2) for k, v in sorted(per_class.items())},
           "separate_ms": round(t_sep, 3), "batch_ms": round(t_bat, 3), "graph_ms": round(t_gr, 3),
           "tuned_graph_ms": round(t_tg, 3),
           "separate_gbs": round(nbytes / t_sep / 1e6, 1), "graph_gbs": round(nbytes / t_gr / 1e6, 1),
           "tuned_graph_gbs": round(nbytes / t_tg / 1e6, 1), "tune_s": round(tune_s, 2),
           "tune_table": [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in e.items()}
                          for e in rfi.tune_table_dict(table)]}
    del pools
    torch.cuda.empty_cache()
    return out


def serve_bench(dev, rates, nblocks, nstreams=8, seed=7, slots=8, budget=64 << 30):
    """Serving loop: Poisson arrivals of uneven blocks from nstreams streams.

    Each stream has one shape class (nbeam, nchan, L) drawn from the uneven
    mix; its blocks last U(0.1, 2) s (49.152 us samples) and are windows into
    a device-resident pool of synthetic data (pre-generated on the GPU: host
    generation at TB/s is impossible). For every arrival rate the same trace
    runs through a session with `slots` execution slots (continuous batching)
    and through a one-slot session (one block at a time). Throughput counts
    every ingested beam-sample; latency is submit -> results ready.
    """
    import torch
    from paper_2512_16278_amd import rfi, synth
    rng = np.random.default_rng(seed)
    pool_s = 2.2
    pools = {}
    for F in MIX_NCHAN:
        spec = synth.mixed_spec(seed + F, max(MIX_NBEAM), F, 512, pool_s)
        t = torch.empty((spec.nbeam, spec.nsamp, F), dtype=torch.uint8, device=dev)
        ds = rfi.DeviceSynth(spec, dev)
        for b in range(spec.nbeam):
            ds.fill(t[b], b)
        pools[F] = t
    torch.cuda.synchronize()
    shapes = [(int(rng.choice(MIX_NBEAM)), int(rng.choice(MIX_NCHAN)), int(rng.choice(MIX_L)))
              for _ in range(nstreams)]
    log(f"serving: {nstreams} streams {shapes}; pools {sum(p.numel() for p in pools.values()) / 1e9:.1f} GB")

    def trace(rate):
        r = np.random.default_rng(seed + int(rate))
        t = np.cumsum(r.exponential(1.0 / rate, size=nblocks))
        out = []
        for ta in t:
            si = int(r.integers(nstreams))
            nb, F, L = shapes[si]
            nsamp = int(r.uniform(0.1, 2.0) / synth.TSAMP)
            start = int(r.integers(0, pools[F].shape[1] - nsamp))
            out.append((float(ta), si, start, nsamp))
        return out

    def run(tr, nslot):
        with rfi.Session(max_inflight=nslot, hbm_budget=budget) as S:
            sids = [S.open_stream(nb, F, L) for nb, F, L in shapes]
            blks = []
            for ta, si, start, nsamp in tr:
                nb, F, L = shapes[si]
                pool = pools[F]
                blks.append(rfi.make_block([pool[b, start:start + nsamp] for b in range(nb)], F))
            tickets = []
            t0 = time.perf_counter()
            for (ta, si, start, nsamp), blk in zip(tr, blks):
                while time.perf_counter() - t0 < ta:
                    pass
                tickets.append(S.submit(sids[si], blk))
            lat, byts, t_first, t_last = [], 0, None, 0.0
            for (ta, si, start, nsamp), tk in zip(tr, tickets):
                r = S.wait(tk)
                if r.status != rfi.RFI_OK:
                    raise RuntimeError(f"serving block failed ({r.status})")
                lat.append((r.t_done_us - r.t_submit_us) / 1e3)
                t_first = r.t_submit_us if t_first is None else min(t_first, r.t_submit_us)
                t_last = max(t_last, r.t_done_us)
                nb, F, L = shapes[si]
                byts += nb * F * nsamp
                S.release(tk)
        lat = np.array(lat)
        span = (t_last - t_first) / 1e6
        return {"gbs": round(byts / span / 1e9, 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3), "span_s": round(span, 3)}

    out = {"streams": [list(s) for s in shapes], "blocks_per_rate": nblocks, "slots": slots,
           "budget_gb": budget / 2**30, "rates": []}
    run(trace(rates[0])[:4], slots)                    # warm-up (code objects, pools)
    for rate in rates:
        tr = trace(rate)
        a = run(tr, slots)
        b = run(tr, 1)
        log(f"serving rate {rate}/s: batched {a}  one-at-a-time {b}")
        out["rates"].append({"rate_per_s": rate, "batched": a, "one_at_a_time": b})
    del pools
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", default="mfma", choices=["mfma", "valu"])
    ap.add_argument("--precision", type=int, default=32, choices=[32, 64])
    ap.add_argument("--cpu-sample-subints", type=int, default=1)
    ap.add_argument("--cpu-sample-chans", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seconds", type=float, default=10.0)
    ap.add_argument("--path", default="fused", choices=["fused", "stages"])
    ap.add_argument("--group", type=int, default=0, help="sub-intervals per pipeline group")
    ap.add_argument("--serve-rates", default="200,2000",
                    help="arrival rates (blocks/s) of the serving run; empty = skip it")
    ap.add_argument("--serve-blocks", type=int, default=40, help="blocks per serving rate")
    ap.add_argument("--no-precision-split", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch comparison")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving loop and print its JSON")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the uneven-batch comparison and print its JSON")
    ap.add_argument("--quick", action="store_true",
                    help="time the steps only (no latency, stage split or CPU baseline)")
    ap.add_argument("--profile-run", action="store_true",
                    help="for counter collection: one copy, one streaming read, one three-call "
                         "step and one whole-block step, then the JSON line of those")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (cells are "
              "independent; several GPUs would each take a channel range)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_16278_amd import rfi, synth

    dev = torch.device("cuda:0")
    if args.batch_only:
        print(json.dumps({"batch": batch_bench(dev)}), flush=True)
        return
    if args.serve_only:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        print(json.dumps({"serving": serve_bench(dev, rates, args.serve_blocks)}), flush=True)
        return
    spec = synth.fast_spec(seconds=args.seconds)
    nb, nc, ns, L = spec.nbeam, spec.nchan, spec.nsamp, spec.L
    nsub = ns // L
    ncell = nsub * nc
    npair = nb * (nb + 1) // 2
    stride = (nc + 15) // 16 * 16
    log(f"workload: {nb} beams x {nc} ch x {ns} samples, L={L}, {nsub} sub-ints, "
        f"{spec.nbytes() / 1e9:.2f} GB")
    data = torch.empty((nb, ns, stride), dtype=torch.uint8, device=dev)
    ds = rfi.DeviceSynth(spec, dev)
    for b in range(nb):
        ds.fill(data[b], b)
    torch.cuda.synchronize()
    log("input generated on the GPU")

    # untimed plain copy of a known 1 GiB: the reference point that scales the
    # HBM byte counters of a profiler run (FETCH_SIZE / WRITE_SIZE per byte)
    calib = data.view(-1)[: 1 << 30].clone()
    del calib
    torch.cuda.synchronize()

    # measured streaming-read peak: the whole input read once by a plain
    # 16-byte-load kernel (median of 5, HIP events on the launch stream)
    sink = torch.empty(rfi.stream_read_sink_words(), dtype=torch.int32, device=dev)
    rd = []
    for _ in range(1 if args.profile_run else 6):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        rfi.stream_read(data, sink)
        b.record()
        torch.cuda.synchronize()
        rd.append(a.elapsed_time(b))
    rd = rd[1:] if len(rd) > 1 else rd
    read_gbs = data.numel() / (float(np.median(rd)) / 1e3) / 1e9
    log(f"streaming read of {data.numel() / 1e9:.2f} GB: {read_gbs:.0f} GB/s")

    blk = rfi.make_block(data, nc)
    sx = torch.empty((nb, ncell), dtype=torch.int32, device=dev)
    sxy = torch.empty((npair, ncell), dtype=torch.int32, device=dev)
    cnt = torch.empty(nsub, dtype=torch.int32, device=dev)
    stat = torch.empty(ncell, dtype=torch.float64, device=dev)
    status = torch.empty(ncell, dtype=torch.uint8, device=dev)
    mask = torch.empty(ncell, dtype=torch.uint8, device=dev)
    fstats = torch.zeros(48, dtype=torch.uint8, device=dev)
    fws = torch.empty(rfi.rfi_flag_workspace_size(nsub, nc), dtype=torch.uint8, device=dev)
    variant = rfi.RFI_CCM_MFMA if args.variant == "mfma" else rfi.RFI_CCM_VALU
    stream = torch.cuda.current_stream()

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    pp = rfi.process_params(L, nsub, group=args.group, eig_precision=args.precision)
    pws = torch.empty(rfi.rfi_process_workspace_size(nb, nc, pp), dtype=torch.uint8, device=dev)

    def step_stages(timed=None):
        if timed is not None:
            ev[0].record(stream)
        rfi.rfi_ccm_accumulate(blk, 0, L, nsub, sx, sxy, cnt, variant=variant)
        if timed is not None:
            ev[1].record(stream)
        rfi.rfi_eig_batched(nb, nsub, nc, sx, sxy, cnt, stat, status, precision=args.precision)
        if timed is not None:
            ev[2].record(stream)
        rfi.rfi_flag(nsub, nc, stat, status, mask, out=fstats, workspace=fws)
        if timed is not None:
            ev[3].record(stream)
            torch.cuda.synchronize()
            timed.append([ev[i].elapsed_time(ev[i + 1]) for i in range(3)])

    def step_fused():
        rfi.rfi_process_block(blk, pp, stat, status, mask, pws, out=fstats)

    step = step_fused if args.path == "fused" else step_stages
    if args.profile_run:
        step_stages()
        step_fused()
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "stream_read_gbs": round(read_gbs, 1)}), flush=True)
        return
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")

    # whole-step timing: K steps back to back between two synchronisations
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(args.steps):
        step()
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    log(f"timed {args.steps} steps ({args.path}): {ms_step:.3f} ms/step")
    if args.quick:
        nbytes_q = nb * nc * nsub * L
        print(json.dumps({"quick": True, "ms_per_step": round(ms_step, 4),
                          "value": round(nbytes_q / (ms_step / 1e3) / 1e9, 2),
                          "stream_read_gbs": round(read_gbs, 1), "group": args.group,
                          "path": args.path}), flush=True)
        return

    # block latency: each step alone, from an event before it to one after it
    lat = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(max(10, min(args.steps, 30))):
        e0.record(stream)
        step()
        e1.record(stream)
        torch.cuda.synchronize()
        lat.append(e0.elapsed_time(e1))
    lat = np.array(lat)

    # per-kernel timing in the three-call path (events between the calls)
    stages = []
    for _ in range(max(3, min(args.steps, 10))):
        step_stages(stages)
    st = np.array(stages)
    ms_ccm, ms_eig, ms_flag = np.median(st, axis=0)
    log(f"stages (median ms): ccm {ms_ccm:.3f}  eig {ms_eig:.3f}  flag {ms_flag:.3f}")
    # the timed path's own outputs, for the summary
    step()
    torch.cuda.synchronize()

    nbytes_in = nb * nc * nsub * L
    value = nbytes_in / (ms_step / 1e3) / 1e9
    # dominant kernel and its roofline
    ccm_bytes = nbytes_in + 4 * (nb + npair) * ncell          # bytes in + sums out
    ccm_gbs = ccm_bytes / (ms_ccm / 1e3) / 1e9
    flags = rfi.flag_stats_from_bytes(fstats.cpu().numpy().tobytes())
    # HBM bytes of the sums kernel from the committed counter summary, while
    # the kernel's source is the one those counters were taken on
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "ccm_traffic_fast19x4096.json")
    if os.path.exists(tpath):
        from paper_2512_16278_amd import prof_summary
        rec = json.load(open(tpath))
        if rec.get("source_sha256") == prof_summary.source_hash() and rec.get("traffic_bytes"):
            traffic = int(rec["traffic_bytes"])
    if ms_ccm >= ms_eig:
        roof = {"kernel": "ccm_mfma_kernel (64-channel tile, one launch per block)"
                          if variant == rfi.RFI_CCM_MFMA else "ccm_valu_kernel",
                "bound": "hbm", "achieved": round(ccm_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ccm_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "ms": round(float(ms_ccm), 4)}
    else:
        # algorithmic FP32 flops of the Jacobi: per sweep n(n-1)/2 rotations of
        # 6(n-2) + 12 flops; 6 sweeps (the typical count on noise-dominated cells)
        flop = ncell * 6 * (nb * (nb - 1) / 2) * (6 * (nb - 2) + 12)
        ach = flop / (ms_eig / 1e3)
        roof = {"kernel": "eig_lane_jacobi", "bound": "alu", "achieved": round(ach / 1e12, 2),
                "peak": FP32_VALU_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": round(ach / FP32_VALU_PEAK, 4), "traffic": None,
                "ms": round(float(ms_eig), 4)}

    def ev_time(fn, reps=3):
        ts = []
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts[1:]))

    psplit = None
    if not args.no_precision_split:
        del sx, sxy
        torch.cuda.empty_cache()
        psplit = precision_split(dev, spec, data, blk, nsub, ev_time)
        log(f"precision split: {psplit}")

    serving = None
    batch = None
    if args.serve_rates or not args.no_batch:
        del data
        torch.cuda.empty_cache()
    if not args.no_batch:
        batch = batch_bench(dev)
        log(f"uneven batch: {batch}")
    if args.serve_rates:
        torch.cuda.empty_cache()
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        serving = serve_bench(dev, rates, args.serve_blocks)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(spec, args.cpu_sample_subints, args.cpu_sample_chans)
        log(f"cpu baseline: {cpu['value'] * 1e3:.2f} MB/s on {cpu['cores']} threads")

    out = {
        "metric": "beam-sample GB/s through CCM+eigen+flag at 1 GPU; p50/p99 block latency",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded FAST-shaped, generated on the GPU)",
        "config": {"workload": f"FAST-shaped block: {nb} beams x {nc} channels x {ns} samples "
                               f"(10 s at 49.152 us), L={L}, {nsub} sub-ints, "
                               f"{nbytes_in / 1e9:.2f} GB", "nbeam": nb, "nchan": nc,
                   "L": L, "nsub": nsub, "path": args.path, "ccm": args.variant,
                   "eigen": ("fp32 householder+sturm, fp64 refinement" if args.precision == 32
                             else "fp64 jacobi")},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4)},
        "stages_ms": {"path": "three calls", "ccm": round(float(ms_ccm), 4),
                      "eig": round(float(ms_eig), 4), "flag": round(float(ms_flag), 4)},
        "hbm_frac_whole_path": round(value / HBM_PEAK_GBS, 4),
        "stream_read_gbs": round(read_gbs, 1),
        "frac_of_measured_read": round(value / read_gbs, 4),
        "flagged_cells": int(flags["nflag"]), "clip_iterations": int(flags["iterations"]),
        "roofline": roof,
        "precision_split": psplit,
        "batch": batch,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
