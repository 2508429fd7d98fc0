#!/usr/bin/env python3
"""Throughput benchmark of the gfx950 polar SCL decoder.

Workload: the paper's headline code (Sec. IV, Table III): N = 2048,
|A| = 1723 (1691 data bits + CRC-32 0x04C11DB7), Bhattacharyya frozen set at
4.5 dB, fully adaptive SSCL with L = 1 -> 2 -> ... -> 32 on CRC failure,
R0/R1/REP8-/SPC4 pruning, 8-bit saturated LLRs (Q6.2), BPSK over AWGN at
Eb/N0 = 3.5, 4.0 and 4.5 dB, 10^6 frames per point.  One step decodes the
three batches (one launch each); inputs are generated on the device before
the timed region and stay resident in HBM.

Prints one JSON line: whole-job information throughput (Mb/s of decoded data
bits), the dominant kernel's achieved fraction of the VALU roofline, FER and
latency per point, and the CPU oracle timed on a bounded host-made sample.
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

WORKLOAD = dict(name="fa_sscl_n2048_k1723_crc32_lmax32_i8", N=2048, K=1723, crc_len=32,
                crc_poly=0x04C11DB7, design=4.5, L_max=32, frac=2)
# MI355X: 256 CUs x 64 vector lanes per clock x 2.4 GHz (no FMA, no packing)
VALU_PEAK_OPS = 256 * 64 * 2.4e9
PAPER_CONTEXT_MBPS = {3.5: 24.4, 4.0: 227.3, 4.5: 425.9}  # one i5-6600K core, 8-bit FA
# counter summaries (HBM bytes per launch) and the sources each kernel is built from
TRAFFIC_FILES = {"k_sc<int8>": "hbm_traffic_k_sc_fa2048_i8.md",
                 "k_decode_list<int8,1,4>": "hbm_traffic_list_a_fa2048_i8.md",
                 "k_decode_list<int8,4,32>": "hbm_traffic_list_b_fa2048_i8.md"}
KERNEL_SOURCES = {"k_sc<int8>": ["sc.hip", "device_common.h", "kernels.h", "polar_internal.h"],
                  "k_decode_list<int8,1,4>": ["decode.hip", "device_common.h", "kernels.h",
                                              "polar_internal.h"],
                  "k_decode_list<int8,4,32>": ["decode.hip", "device_common.h", "kernels.h",
                                               "polar_internal.h"]}


def wilson(k, n, z=1.96):
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


def stage_schedule(L_max):
    s, l = [], 1
    while l < L_max:
        s.append(l)
        l *= 2
    s.append(L_max)
    return s


def cpu_baseline(points, frames_per_point, threads):
    """The CPU oracle as it stands, on a host-made sample of the workload."""
    import oracle as O
    from paper_1710_08314_amd import synth

    W = WORKLOAD
    fz = O.construct(W["N"], W["K"], 0, W["crc_len"], W["design"])
    code = O.Code(W["N"], W["K"], fz, W["crc_len"], W["crc_poly"], quant=O.I8, algo=O.FA_SCL,
                  L_max=W["L_max"], rep_max=8, spc_max=4)
    bits_total, secs = 0, 0.0
    per = {}
    for i, eb in enumerate(points):
        data, noise = synth.frames(7000 + i, 0, frames_per_point, code.k_data, code.n_tx)
        x = np.zeros((frames_per_point, code.N), np.uint8)
        for f in range(frames_per_point):
            x[f] = O.encode(fz, O.attach_crc(data[f], code.crc_len, code.crc_poly))
        llr = O.make_llr(code, x, noise, synth.sigma_for(eb, code.k_data, code.n_tx), W["frac"])
        t0 = time.perf_counter()
        r = O.decode(code, llr, threads=threads)
        dt = time.perf_counter() - t0
        secs += dt
        bits_total += frames_per_point * code.k_data
        per[str(eb)] = round(frames_per_point * code.k_data / dt / 1e6, 3)
    return {"value": round(bits_total / secs / 1e6, 3), "unit": "Mb/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{frames_per_point} host-generated frames per Eb/N0 point "
                      f"({', '.join(str(p) for p in points)} dB) of the same workload, "
                      f"frame-parallel over {threads} threads; decode time only",
            "per_point_mbps": per}


def calib_copy(nbytes):
    """A plain elementwise kernel of known traffic: y = -x over int32, reading
    and writing `nbytes` each, run three times.  Its FETCH_SIZE / WRITE_SIZE
    readings scale the decoder kernel's counters to bytes."""
    import torch

    n = nbytes // 4
    x = torch.ones(n, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": n * 4, "dispatches": 3}))


def kernel_source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1710_08314_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when there is none or the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES.get(kernel, "-"))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_hash(KERNEL_SOURCES[kernel]):
        return None
    try:
        return int(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=1_000_000, help="frames per Eb/N0 point")
    ap.add_argument("--points", default="3.5,4.0,4.5")
    ap.add_argument("--schedule", type=int, default=0, help="0 automatic, 1 plain")
    ap.add_argument("--cpu-frames", type=int, default=3000, help="oracle sample per point")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--compare-plain", type=int, default=1,
                    help="also time the plain one-launch form once per point")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.calib_copy:
        calib_copy(args.calib_copy)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: the decoder shards frames across GPUs with no "
              "collective, so only --gpus 1 is measured", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1710_08314_amd import polar as P

    torch.cuda.set_device(0)
    W = WORKLOAD
    points = [float(p) for p in args.points.split(",")]
    F = args.frames
    plan = P.Plan(W["N"], W["K"], W["crc_len"], W["crc_poly"], design_ebn0_db=W["design"],
                  algo=P.FA_SCL, L_max=W["L_max"], quant=P.I8, rep_max=8, spc_max=4)
    kd = plan.info.k_data
    stream = torch.cuda.current_stream()

    # ---- inputs, generated on the device (not timed)
    batches = []
    for i, eb in enumerate(points):
        data = P.gen_data(plan, 2000 + i, 0, F)
        code = P.encode(plan, data)
        llr = P.channel(plan, code, eb, 3000 + i, 0, frac_bits=W["frac"])
        del code
        batches.append((eb, data, llr))
    torch.cuda.synchronize()

    def decode_all(record=None):
        outs = []
        for eb, data, llr in batches:
            if record is not None:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            info, status, _ = P.decode_batch(plan, llr, schedule=args.schedule, stream=stream)
            if record is not None:
                e1.record(stream)
                record.append((eb, e0, e1))
            outs.append((info, status))
        return outs

    for _ in range(args.warmup):
        decode_all()
    torch.cuda.synchronize()
    events = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        outs = decode_all(events)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # ---- per point: FER, list-size histogram, algorithmic work
    sched = stage_schedule(W["L_max"])
    cum, acc = {}, 0
    for l in sched:
        acc += plan.stage_work(l)
        cum[l] = acc
    per_point, work_per_launch = {}, {}
    for (eb, data, llr), (info, status) in zip(batches, outs):
        err = (info != data).any(dim=1)
        n_err = int(err.sum().item())
        lu = status[:, 1].to(torch.int64)
        hist = torch.bincount(lu, minlength=W["L_max"] + 1).cpu().numpy()
        work = sum(int(hist[l]) * cum[l] for l in sched)
        work_per_launch[eb] = work
        lo, hi = wilson(n_err, F)
        per_point[str(eb)] = {"fer": n_err / F, "fer_ci95": [lo, hi],
                              "crc_fail": int((status[:, 0] == 0).sum().item()),
                              "L_used_hist": {str(l): int(hist[l]) for l in sched if hist[l]},
                              "avg_stages": float(sum(hist[l] * (sched.index(l) + 1)
                                                      for l in sched) / F)}
    # the plain form (one generic launch per configuration), same inputs
    plain_ms = {}
    if args.schedule == 0 and args.compare_plain:
        for eb, data, llr in batches:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            P.decode_batch(plan, llr, schedule=1, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            plain_ms[eb] = e0.elapsed_time(e1)
    kms = {}
    for eb, e0, e1 in events:
        kms.setdefault(eb, []).append(e0.elapsed_time(e1))
    for eb in points:
        ms = float(np.mean(kms[eb]))
        per_point[str(eb)]["kernel_ms"] = round(ms, 3)
        per_point[str(eb)]["info_mbps"] = round(F * kd / (ms / 1e3) / 1e6, 1)
        per_point[str(eb)]["paper_1core_context_mbps"] = PAPER_CONTEXT_MBPS.get(eb)
        if eb in plain_ms:
            per_point[str(eb)]["plain_launch_ms"] = round(plain_ms[eb], 3)
            per_point[str(eb)]["plain_info_mbps"] = round(F * kd / (plain_ms[eb] / 1e3) / 1e6, 1)

    # ---- per-kernel durations (HIP events recorded by the library on the
    # launch stream around each tier) and each tier's algorithmic work
    tier_ms = {t: 0.0 for t in ("sc", "list_a", "list_b")}
    tier_work = {t: 0 for t in tier_ms}
    for (eb, data, llr), (info, status) in zip(batches, outs):
        P.decode_batch(plan, llr, schedule=args.schedule, stream=stream, tier_timing=True)
        torch.cuda.synchronize()
        ms = P.last_tier_ms()
        for t in tier_ms:
            tier_ms[t] += ms[t]
        hist = torch.bincount(status[:, 1].to(torch.int64), minlength=W["L_max"] + 1).cpu().numpy()
        per_point[str(eb)]["tier_ms"] = {t: round(ms[t], 3) for t in tier_ms}
        for l in sched:
            reached = int(sum(hist[x] for x in sched if x >= l))
            tier = "sc" if l == 1 else ("list_a" if l <= 4 else "list_b")
            tier_work[tier] += reached * plan.stage_work(l)

    # ---- latency: per-frame decode time from device realtime stamps
    khz = P.device_clock_khz()
    lat = {}
    for eb, data, llr in batches:
        times = torch.zeros((F, 2), dtype=torch.int64, device="cuda")
        P.decode_batch(plan, llr, schedule=args.schedule, stream=stream, times=times)
        torch.cuda.synchronize()
        t = times.cpu().numpy().astype(np.float64)
        svc = (t[:, 1] - t[:, 0]) / khz * 1e3  # us
        done = (t[:, 1] - t[:, 0].min()) / khz * 1e3
        lat[str(eb)] = {"decode_p50_us": round(float(np.percentile(svc, 50)), 2),
                        "decode_p99_us": round(float(np.percentile(svc, 99)), 2),
                        "decode_max_us": round(float(svc.max()), 2),
                        "batch_completion_p50_us": round(float(np.percentile(done, 50)), 1),
                        "batch_completion_p99_us": round(float(np.percentile(done, 99)), 1)}
        per_point[str(eb)]["latency"] = lat[str(eb)]

    total_bits = args.steps * len(points) * F * kd
    value = total_bits / elapsed / 1e6
    kernel_names = {"sc": "k_sc<int8>", "list_a": "k_decode_list<int8,1,4>",
                    "list_b": "k_decode_list<int8,4,32>"}
    tiers = {}
    for t in tier_ms:
        if tier_ms[t] > 0:
            ach = tier_work[t] / (tier_ms[t] / 1e3)
            tiers[t] = {"kernel": kernel_names[t], "launch_ms": round(tier_ms[t] / len(points), 3),
                        "work_per_launch_ops": int(tier_work[t] / len(points)),
                        "achieved": round(ach / 1e12, 5), "frac": round(ach / VALU_PEAK_OPS, 6)}
    dom = max(tiers, key=lambda t: tiers[t]["launch_ms"])
    roofline = {"bound": "alu", "achieved": tiers[dom]["achieved"],
                "peak": round(VALU_PEAK_OPS / 1e12, 2), "unit": "Tops/s",
                "frac": tiers[dom]["frac"], "traffic": measured_traffic(tiers[dom]["kernel"]),
                "kernel": tiers[dom]["kernel"],
                "work_per_launch_ops": tiers[dom]["work_per_launch_ops"],
                "launch_ms": tiers[dom]["launch_ms"], "tiers": tiers}

    out = {
        "metric": "info Mb/s per MI355X at matched FER + p50/p99 decode latency, batched vs plain",
        "value": round(value, 1), "unit": "Mb/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i8",
        "data": "synthetic",
        "config": {"workload": W["name"], "N": W["N"], "K": W["K"], "k_data": kd,
                   "crc": "0x04C11DB7", "algo": "FA-SSCL", "L_max": W["L_max"],
                   "ebn0_db": points, "frames_per_point": F,
                   "schedule": "plain" if args.schedule == 1 else "automatic",
                   "coded_mbps": round(value * W["N"] / kd, 1),
                   "plain_mbps": (round(len(points) * F * kd / (sum(plain_ms.values()) / 1e3) / 1e6, 1)
                                  if plain_ms else None),
                   "per_point": per_point},
        "roofline": roofline,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(points, args.cpu_frames,
                                           min(16, os.cpu_count() or 1))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
