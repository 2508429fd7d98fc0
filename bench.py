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
# MI355X: 256 CUs x 128 vector lanes per clock x 2.4 GHz, the lane rate of the published fp32
# vector peak (157.3 TFLOP/s counting an FMA as two), with no FMA credit
VALU_PEAK_OPS = 256 * 128 * 2.4e9
HBM_PEAK_BYTES = 8.0e12  # MI355X HBM3E
PAPER_CONTEXT_MBPS = {3.5: 24.4, 4.0: 227.3, 4.5: 425.9}  # one i5-6600K core, 8-bit FA
# counter summaries (HBM bytes per launch) and the sources each kernel is built from
LIST_KERNELS = ["k_rq<11,2>", "k_rq<11,4>", "k_rq<11,8>", "k_rq<11,16>", "k_listp<32>",
                "k_listp_lds<32>"]
TRAFFIC_FILES = {"k_rq<11,1>": "hbm_traffic_k_rq1_fa2048_i8.md",
                 "k_rq<11,2>": "hbm_traffic_k_rq2_fa2048_i8.md",
                 "k_rq<11,4>": "hbm_traffic_k_rq4_fa2048_i8.md",
                 "k_rq<11,8>": "hbm_traffic_k_rq8_fa2048_i8.md",
                 "k_rq<11,16>": "hbm_traffic_k_rq16_fa2048_i8.md",
                 "k_listp<32>": "hbm_traffic_k_listp32_fa2048_i8.md",
                 "k_listp_lds<32>": "hbm_traffic_k_listp32_lds_fa2048_i8.md"}
_RQ_SRC = ["rq.hip", "device_common.h", "kernels.h", "polar_internal.h"]
_LISTP_SRC = ["scx.hip", "device_common.h", "kernels.h", "polar_internal.h"]
KERNEL_SOURCES = {"k_rq<11,1>": _RQ_SRC, "k_rq<11,2>": _RQ_SRC, "k_rq<11,4>": _RQ_SRC,
                  "k_rq<11,8>": _RQ_SRC, "k_rq<11,16>": _RQ_SRC,
                  "k_listp<32>": _LISTP_SRC, "k_listp_lds<32>": _LISTP_SRC}
# issue counters of the same profiled run (VALU busy per kernel)
ISSUE_FILE = "counters_issue_lds_fa2048_i8.md"


def wilson(k, n, z=1.96):
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    # the interval's ends are exactly 0 and 1 when no frame (every frame) fails
    return (0.0 if k == 0 else max(0.0, c - h), 1.0 if k == n else min(1.0, c + h))


def stage_schedule(L_max):
    s, l = [], 1
    while l < L_max:
        s.append(l)
        l *= 2
    s.append(L_max)
    return s


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    """Cores this process may run on (its affinity mask)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(points, frames_per_point, threads, frames_1core):
    """The CPU oracle as it stands, on a host-made sample of the workload:
    frame-parallel over every host core, then on one core (a smaller
    sample).  Returns the record and the oracle's frame errors per point."""
    import oracle as O
    from paper_1710_08314_amd import synth

    W = WORKLOAD
    fz = O.construct(W["N"], W["K"], 0, W["crc_len"], W["design"])
    code = O.Code(W["N"], W["K"], fz, W["crc_len"], W["crc_poly"], quant=O.I8, algo=O.FA_SCL,
                  L_max=W["L_max"], rep_max=8, spc_max=4)
    bits_total, secs, bits_1, secs_1 = 0, 0.0, 0, 0.0
    per, errs = {}, {}
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
        errs[eb] = int((r.info != data).any(axis=1).sum())
        m = min(frames_1core, frames_per_point)
        t0 = time.perf_counter()
        O.decode(code, llr[:m], threads=1)
        secs_1 += time.perf_counter() - t0
        bits_1 += m * code.k_data
    rec = {"value": round(bits_total / secs / 1e6, 3), "unit": "Mb/s", "cores": threads,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{frames_per_point} host-generated frames per Eb/N0 point "
                     f"({', '.join(str(p) for p in points)} dB) of the same workload, "
                     f"frame-parallel over {threads} threads (every core the process may use); "
                     f"decode time only; the one-core rate on the first {frames_1core} frames "
                     f"of each point",
           "per_point_mbps": per, "one_core_mbps": round(bits_1 / secs_1 / 1e6, 3),
           "oracle_frame_errors": {str(k): v for k, v in errs.items()}}
    return rec, errs


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
    or None when there is none or the kernel's sources changed since.  A
    tier of several kernels ("a + b") sums theirs."""
    if " + " in kernel:
        parts = [measured_traffic(k) for k in kernel.split(" + ")]
        return None if any(p is None for p in parts) else sum(parts)
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


def measured_valu_busy(kernel):
    """VALU busy fraction of `kernel` (wave64 VALU instructions x 4 cycles
    over the SIMDs' cycles) from the committed issue-counter summary, or None
    when there is none or the kernel's traffic summary (taken in the same
    run) no longer matches its sources.  A tier of several kernels takes the
    time-weighted mean of theirs."""
    names = kernel.split(" + ")
    if any(measured_traffic(k) is None for k in names):
        return None
    path = os.path.join(ROOT, "profiles", ISSUE_FILE)
    if not os.path.exists(path):
        return None
    rows = {}
    with open(path) as fh:
        for line in fh:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 8 and cells[0].startswith("`"):
                try:
                    rows[cells[0].strip("`")] = (float(cells[6]), float(cells[7].rstrip("%")) / 100)
                except ValueError:
                    pass
    if any(k not in rows for k in names):
        return None
    ms = sum(rows[k][0] for k in names)
    return sum(rows[k][0] * rows[k][1] for k in names) / ms if ms > 0 else None


def tier_bound(hbm_frac, valu_busy, op_frac):
    """A kernel's bound from its own counters: "hbm" when its measured HBM
    rate is a larger fraction of the HBM peak than its VALU busy fraction
    (or, without issue counters, its algorithmic-op fraction of the issue
    peak), else "alu"."""
    issue = valu_busy if valu_busy is not None else op_frac
    return "hbm" if (hbm_frac or 0.0) > issue else "alu"


def bench_uneven(args):
    """The batched uneven launch: 2^20 frames, each with its own (N, rate, L,
    shortening) -- about 15,000 plans -- CRC-11, int16, decoded in one call by
    the autotuned class schedule, then by a HIP-graph replay of it, then by
    the plain one-launch form.  Inputs are generated on the device per plan
    (data, systematic encoding, BPSK/AWGN at one Eb/N0 ~ U[1, 4] dB per plan:
    the fixed-list decoders' work does not depend on the channel)."""
    import torch

    from paper_1710_08314_amd import polar as P
    from paper_1710_08314_amd import synth

    torch.cuda.set_device(0)
    n = args.frames if args.frames != 1_000_000 else 1 << 20
    specs, plan_of, _ = synth.uneven_batch(3000, n)
    c, poly = synth.C3_CRC
    t0 = time.perf_counter()
    plans = [P.Plan(N, K, c, poly, design_ebn0_db=synth.C3_DESIGN_DB, n_shorten=S, algo=P.CA_SCL,
                    L=L, quant=P.I16) for (N, K, L, S) in specs]
    t_plan = time.perf_counter() - t0
    counts = np.bincount(plan_of, minlength=len(plans))
    # plan-major LLR regions, each frame slot padded to 16 bytes
    strides = [((p.info.n_tx * 2 + 15) // 16) * 16 for p in plans]
    region = np.zeros(len(plans) + 1, dtype=np.int64)
    region[1:] = np.cumsum(counts * np.array(strides, dtype=np.int64))
    d_llr = torch.empty(int(region[-1]), dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(3001)
    ebn0 = rng.uniform(1.0, 4.0, size=len(plans))
    for i, p in enumerate(plans):
        if counts[i] == 0:
            continue
        data = P.gen_data(p, 3002, 0, int(counts[i]))
        code = P.encode(p, data)
        llr = P.channel(p, code, float(ebn0[i]), 3003 + i, 0)
        dst = d_llr[int(region[i]):int(region[i + 1])].view(int(counts[i]), strides[i])
        dst[:, :p.info.n_tx * 2].copy_(llr.view(torch.uint8).view(int(counts[i]), -1))
    # frame descriptors in draw order
    slot = np.zeros(n, dtype=np.int64)
    seen = np.zeros(len(plans), dtype=np.int64)
    order = np.argsort(plan_of, kind="stable")
    sorted_plans = plan_of[order]
    starts = np.searchsorted(sorted_plans, np.arange(len(plans)))
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n) - starts[sorted_plans]
    st_arr = np.array(strides, dtype=np.int64)
    slot = region[plan_of] + rank * st_arr[plan_of]
    iw = np.array([p.info.info_words for p in plans], dtype=np.int64)[plan_of]
    out_off = np.concatenate([[0], np.cumsum(iw)[:-1]])
    desc = np.zeros((n, 4), dtype=np.uint32)
    desc[:, 0] = slot & 0xFFFFFFFF
    desc[:, 1] = slot >> 32
    desc[:, 2] = out_off
    desc[:, 3] = plan_of
    d_fr = torch.from_numpy(desc.view(np.int32)).cuda()
    kd = np.array([p.info.k_data for p in plans], dtype=np.int64)
    info_bits = int((kd[plan_of]).sum())
    coded_bits = int(np.array([p.info.n_tx for p in plans])[plan_of].sum())
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0 - t_plan
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.mean(ms))

    # autotune once (untimed), then the timed steps
    t1 = time.perf_counter()
    P.decode_batch(plans, d_llr, frames=d_fr, autotune=True, stream=stream)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t1
    sched = P.schedule_describe(plans)
    for _ in range(args.warmup):
        P.decode_batch(plans, d_llr, frames=d_fr, stream=stream)
    torch.cuda.synchronize()
    tw = time.perf_counter()
    ms_batched = timed(lambda: P.decode_batch(plans, d_llr, frames=d_fr, stream=stream), args.steps)
    elapsed = time.perf_counter() - tw
    g = P.Graph(plans, d_llr, frames=d_fr)
    g.launch(stream)
    torch.cuda.synchronize()
    ms_graph = timed(lambda: g.launch(stream), args.steps)
    ms_plain = None
    if args.compare_plain:
        ms_plain = timed(lambda: P.decode_batch(plans, d_llr, frames=d_fr, schedule=1,
                                                stream=stream), 1)
    # batched latency from device stamps: completion - batch start, decode time
    times = torch.zeros((n, 2), dtype=torch.int64, device="cuda")
    P.decode_batch(plans, d_llr, frames=d_fr, times=times, stream=stream)
    torch.cuda.synchronize()
    khz = P.device_clock_khz()
    t = times.cpu().numpy().astype(np.float64)
    svc = (t[:, 1] - t[:, 0]) / khz * 1e3
    done = (t[:, 1] - t[:, 0].min()) / khz * 1e3
    Ls = np.array([s_[2] for s_ in specs])[plan_of]
    per_L = {str(l): {"frames": int((Ls == l).sum()),
                      "decode_p50_us": round(float(np.percentile(svc[Ls == l], 50)), 1),
                      "decode_p99_us": round(float(np.percentile(svc[Ls == l], 99)), 1)}
             for l in synth.C3_L}
    mbps = lambda ms: round(info_bits / (ms / 1e3) / 1e6, 1)
    out = {
        "metric": "info Mb/s per MI355X at matched FER + p50/p99 decode latency, batched vs plain",
        "value": round(info_bits * args.steps / elapsed / 1e6, 1), "unit": "Mb/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i16", "data": "synthetic",
        "config": {"workload": "uneven_batch_2p20_crc11_i16", "frames": n, "plans": len(plans),
                   "info_bits": info_bits, "coded_bits": coded_bits,
                   "schedule": sched, "autotune_s": round(t_tune, 2),
                   "plan_setup_s": round(t_plan, 2), "input_gen_s": round(t_gen, 2),
                   "batched_kernel_ms": round(ms_batched, 3), "batched_info_mbps": mbps(ms_batched),
                   "graph_replay_ms": round(ms_graph, 3), "graph_info_mbps": mbps(ms_graph),
                   "plain_ms": None if ms_plain is None else round(ms_plain, 3),
                   "plain_info_mbps": None if ms_plain is None else mbps(ms_plain),
                   "coded_mbps": round(coded_bits / (ms_batched / 1e3) / 1e6, 1),
                   "latency": {"batch_completion_p50_us": round(float(np.percentile(done, 50)), 1),
                               "batch_completion_p99_us": round(float(np.percentile(done, 99)), 1),
                               "decode_p50_us": round(float(np.percentile(svc, 50)), 1),
                               "decode_p99_us": round(float(np.percentile(svc, 99)), 1),
                               "per_list_size": per_L}},
    }
    return out


def bench_served(args):
    """Served decoding: requests of mixed sizes (N in {32 .. 1024} with
    P(N) ~ 1/N, K ~ U{12 .. N/2} incl. CRC-11, FA-SSCL L = 1 -> 8, Eb/N0 ~
    U[0, 3] dB), pre-staged in HBM, released at Poisson arrival times of 0.5
    to 8 M requests/s into the library's serving loop (continuous batching
    over 4 HIP streams, frame budget), for float32 and int8 LLRs.  Latency is
    host-observed completion minus scheduled arrival.  Beside it: the same
    requests as one batch (device stamps) and as the plain one-launch form."""
    import torch

    from paper_1710_08314_amd import polar as P
    from paper_1710_08314_amd import synth

    torch.cuda.set_device(0)
    n = args.frames if args.frames != 1_000_000 else 1_000_000
    c, poly = synth.C4_CRC
    stream = torch.cuda.current_stream()
    results = {}
    for quant in ("f32", "i8"):
        qv = P.QUANT_NAMES[quant]
        es = P.ELEM_BYTES[qv]
        specs, plan_of, ebn0, _ = synth.served_requests(4100, n, 1.0e6)
        plans = [P.Plan(N, K, c, poly, design_ebn0_db=synth.C4_DESIGN_DB, algo=P.FA_SCL,
                        L_max=synth.C4_L_MAX, quant=qv) for (N, K) in specs]
        # LLR pool: per plan, its requests sorted by Eb/N0 in 8 chunks, each
        # generated at the chunk's median Eb/N0 (within ~0.2 dB of every draw)
        strides = np.array([((p.info.n_tx * es + 15) // 16) * 16 for p in plans], dtype=np.int64)
        slot = np.zeros(n, dtype=np.int64)
        order = np.lexsort((ebn0, plan_of))
        pool = int(strides[plan_of].sum())
        d_llr = torch.empty(pool, dtype=torch.uint8, device="cuda")
        off = 0
        pos = 0
        counts = np.bincount(plan_of, minlength=len(plans))
        for i, p in enumerate(plans):
            reqs = order[pos:pos + counts[i]]
            pos += counts[i]
            for ch in np.array_split(reqs, min(8, len(reqs))) if len(reqs) else []:
                m = len(ch)
                slot[ch] = off + np.arange(m) * strides[i]
                data = P.gen_data(p, 4101, off, m)
                code = P.encode(p, data)
                llr = P.channel(p, code, float(np.median(ebn0[ch])), 4102, off)
                dst = d_llr[off:off + m * int(strides[i])].view(m, int(strides[i]))
                dst[:, :p.info.n_tx * es].copy_(llr.view(torch.uint8).view(m, -1))
                off += m * int(strides[i])
        iw = np.array([p.info.info_words for p in plans], dtype=np.int64)[plan_of]
        out_off = np.concatenate([[0], np.cumsum(iw)[:-1]])
        desc = np.zeros((n, 4), dtype=np.uint32)
        desc[:, 0] = slot & 0xFFFFFFFF
        desc[:, 1] = slot >> 32
        desc[:, 2] = out_off
        desc[:, 3] = plan_of
        d_fr = torch.from_numpy(desc.view(np.int32)).cuda()
        info_bits = int(np.array([p.info.k_data for p in plans], dtype=np.int64)[plan_of].sum())
        n_words = int(iw.sum())
        # one batch (not served), with device stamps, and the plain form
        times = torch.zeros((n, 2), dtype=torch.int64, device="cuda")
        P.decode_batch(plans, d_llr, frames=d_fr, stream=stream)  # warm-up, plan table
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b_info, b_st, _ = P.decode_batch(plans, d_llr, frames=d_fr, stream=stream, times=times)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_batch = e0.elapsed_time(e1)
        khz = P.device_clock_khz()
        t = times.cpu().numpy().astype(np.float64)
        done = (t[:, 1] - t[:, 0].min()) / khz * 1e3
        e0.record(stream)
        P.decode_batch(plans, d_llr, frames=d_fr, schedule=1, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_plain = e0.elapsed_time(e1)
        hist = np.bincount(b_st[:, 1].cpu().numpy(), minlength=9)
        per_rate = {}
        # admission by frames and by device bytes (each request charged its
        # plan's in-flight figure): half of what 65,536 of the largest take
        budget = 65536 * max(p.frame_bytes() for p in plans) // 2
        srv = P.Server(n_slots=4, max_batch=16384, max_inflight=65536, budget_bytes=budget)
        for k, rate in enumerate(synth.C4_RATES_MREQ):
            rng = np.random.default_rng(4200 + k)
            gaps = rng.exponential(1.0 / rate, size=n)  # us
            arrival = np.cumsum(gaps) - gaps[0]
            info = torch.zeros(max(n_words, 1), dtype=torch.int32, device="cuda")
            status = torch.zeros((n, 8), dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            done_us, stats = srv.replay(plans, d_fr, arrival, d_llr, info, status, plan_of=plan_of)
            torch.cuda.synchronize()
            same = bool(torch.equal(status, b_st) and torch.equal(info[:n_words], b_info[:n_words]))
            lat = done_us - arrival
            per_rate[str(rate)] = {
                "offered_mreq_s": rate, "served_mreq_s": round(n / stats["session_us"], 3),
                "info_mbps": round(info_bits / stats["session_us"], 1),
                "latency_p50_us": round(float(np.percentile(lat, 50)), 1),
                "latency_p99_us": round(float(np.percentile(lat, 99)), 1),
                "batches": stats["batches"], "mean_batch": round(stats["mean_batch"], 1),
                "peak_inflight": stats["peak_inflight"],
                "peak_inflight_bytes": stats["peak_inflight_bytes"], "budget_bytes": budget,
                "results_equal_batch": same}
            print(f"served {quant} {rate} Mreq/s: {per_rate[str(rate)]}", file=sys.stderr,
                  flush=True)
        srv.close()
        results[quant] = {
            "requests": n, "plans": len(plans), "info_bits": info_bits,
            "L_used_hist": {str(l): int(hist[l]) for l in (1, 2, 4, 8) if hist[l]},
            "batched": {"kernel_ms": round(ms_batch, 3),
                        "info_mbps": round(info_bits / (ms_batch / 1e3) / 1e6, 1),
                        "completion_p50_us": round(float(np.percentile(done, 50)), 1),
                        "completion_p99_us": round(float(np.percentile(done, 99)), 1)},
            "plain": {"kernel_ms": round(ms_plain, 3),
                      "info_mbps": round(info_bits / (ms_plain / 1e3) / 1e6, 1)},
            "served": per_rate}
        del plans
    best = max(results["i8"]["served"].values(), key=lambda v: v["info_mbps"])
    out = {
        "metric": "info Mb/s per MI355X at matched FER + p50/p99 decode latency, batched vs plain",
        "value": best["info_mbps"], "unit": "Mb/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8", "data": "synthetic",
        "config": {"workload": "served_fa_lmax8_crc11_n32_1024", "per_quant": results},
    }
    return out


def bench_pruning(args):
    """Tree pruning sweep (Sec. III-B2 / the node study of Sec. IV): the
    headline code and decoder with the dedicated nodes enabled one family at a
    time -- none, R0, +REP8-, +R1, +SPC4 (the default), then SPC of any size
    and REP of any size -- reporting node-program length, throughput and FER
    at 3.5 and 4.5 dB (10^6 frames each unless --frames is given)."""
    import torch

    from paper_1710_08314_amd import polar as P

    torch.cuda.set_device(0)
    W = WORKLOAD
    F = args.frames
    stream = torch.cuda.current_stream()
    R0, R1, REP, SPC = P.NODE_R0, P.NODE_R1, P.NODE_REP, P.NODE_SPC
    variants = [("none", 0, 8, 4), ("R0", R0, 8, 4), ("R0+REP8", R0 | REP, 8, 4),
                ("R0+REP8+R1", R0 | REP | R1, 8, 4), ("R0+REP8+R1+SPC4", R0 | REP | R1 | SPC, 8, 4),
                ("R0+REP8+R1+SPC(any)", R0 | REP | R1 | SPC, 8, 0),
                ("R0+REP(any)+R1+SPC4", R0 | REP | R1 | SPC, 0, 4)]
    # the channel is the same for every variant: generate with the default plan
    base = P.Plan(W["N"], W["K"], W["crc_len"], W["crc_poly"], design_ebn0_db=W["design"],
                  algo=P.FA_SCL, L_max=W["L_max"], quant=P.I8, rep_max=8, spc_max=4)
    kd = base.info.k_data
    points = {}
    for i, eb in enumerate((3.5, 4.5)):
        data = P.gen_data(base, 2000 + i, 0, F)
        llr = P.channel(base, P.encode(base, data), eb, 3000 + i, 0, frac_bits=W["frac"])
        points[eb] = (data, llr)
    torch.cuda.synchronize()
    rows = []
    for name, enable, rep_max, spc_max in variants:
        plan = P.Plan(W["N"], W["K"], W["crc_len"], W["crc_poly"], design_ebn0_db=W["design"],
                      algo=P.FA_SCL, L_max=W["L_max"], quant=P.I8, node_enable=enable,
                      rep_max=rep_max, spc_max=spc_max)
        row = {"nodes": name, "n_ops": plan.info.n_ops, "r0": plan.info.n_r0, "r1": plan.info.n_r1,
               "rep": plan.info.n_rep, "spc": plan.info.n_spc,
               "leaves": plan.info.n_leaf_frozen + plan.info.n_leaf_info}
        for eb, (data, llr) in points.items():
            P.decode_batch(plan, llr, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            info, status, _ = P.decode_batch(plan, llr, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            fer = float((info != data).any(dim=1).float().mean().item())
            row[str(eb)] = {"ms": round(ms, 3), "info_mbps": round(F * kd / (ms / 1e3) / 1e6, 1),
                            "fer": fer}
        rows.append(row)
        print(f"pruning {row}", file=sys.stderr, flush=True)
    out = {"metric": "info Mb/s per MI355X at matched FER + p50/p99 decode latency, batched vs plain",
           "value": rows[4]["3.5"]["info_mbps"], "unit": "Mb/s", "n_gpus": 1, "steps": 1,
           "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "i8", "data": "synthetic",
           "config": {"workload": "pruning_sweep_fa2048_k1723_i8", "frames_per_point": F,
                      "variants": rows}}
    return out


QUANT_SWEEP = {"N": 1024, "K": 512, "crc_len": 24, "crc_poly": 0x1864CFB, "design": 2.5, "L": 8,
               "points": [1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0]}


def quant_oracle_leg(quant, points, frames, threads):
    """The cpu_baseline leg of the quantisation sweep: the oracle as it
    stands on a host-made sample of each point (decode time only), giving its
    frame and bit error counts for the matched-FER check.  The sample is made
    and decoded in chunks, so a 10^6-frame sample never sits in memory whole."""
    import concurrent.futures as cf

    import oracle as O
    from paper_1710_08314_amd import synth

    Q = QUANT_SWEEP
    oq = {"f32": O.F32, "i16": O.I16, "i8": O.I8}[quant]
    frac = {"f32": 0, "i16": 3, "i8": 2}[quant]
    fz = O.construct(Q["N"], Q["K"], 0, Q["crc_len"], Q["design"])
    # the GPU plan's node options: REP nodes of at most 8 positions in int8, any size otherwise
    code = O.Code(Q["N"], Q["K"], fz, Q["crc_len"], Q["crc_poly"], quant=oq, algo=O.CA_SCL, L=Q["L"],
                  rep_max=8 if quant == "i8" else 0, spc_max=4)
    chunk, part = 1 << 16, 1 << 12
    out, secs, bits = {}, 0.0, 0
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for i, eb in enumerate(points):
            sigma = synth.sigma_for(eb, code.k_data, code.n_tx)
            fe = be = 0
            for f0 in range(0, frames, chunk):
                n = min(chunk, frames - f0)
                data = np.zeros((n, code.k_data), np.uint8)
                llr = np.zeros((n, code.n_tx), O.DTYPES[oq])

                def make(j, f0=f0, n=n, data=data, llr=llr):
                    lo, hi = j, min(n, j + part)
                    d, z = synth.frames(9000 + i, f0 + lo, hi - lo, code.k_data, code.n_tx)
                    data[lo:hi] = d
                    llr[lo:hi] = O.make_frames(code, d, z, sigma, frac)

                list(ex.map(make, range(0, n, part)))
                t0 = time.perf_counter()
                r = O.decode(code, llr, threads=threads)
                secs += time.perf_counter() - t0
                bits += n * code.k_data
                wrong = r.info != data
                fe += int(wrong.any(axis=1).sum())
                be += int(wrong.sum())
            out[eb] = (fe, be)
            print(f"oracle {quant} {eb} dB: {frames} frames, {fe} frame errors", file=sys.stderr,
                  flush=True)
    return out, bits / secs / 1e6


def bench_quant(args):
    """The quantisation sweep at scale (the fixed-point study of Sec. III-B3):
    the (1024, 488 + CRC-24) code, Bhattacharyya design at 2.5 dB, CA-SCL
    L = 8, float32 / saturated int16 / saturated int8 LLRs at Eb/N0 = 1.0 ...
    4.0 dB, `--quant-frames` frames per point (10^7 by default) generated on
    the device in chunks (data, systematic encoding, BPSK / AWGN, the plan's
    quantiser), decoded, and their frame and bit errors counted on the
    device.  Beside each point the oracle decodes a host-made sample
    (`--quant-oracle` frames) and the GPU's FER must lie in the oracle's 95%
    interval or the two intervals overlap."""
    import torch

    from paper_1710_08314_amd import polar as P

    torch.cuda.set_device(0)
    Q = QUANT_SWEEP
    F, C = args.quant_frames, 1 << 20
    stream = torch.cuda.current_stream()
    pop = torch.tensor([bin(i).count("1") for i in range(256)], dtype=torch.int64, device="cuda")
    rows, oracle_mbps = {}, {}
    types = [t for t in ("f32", "i16", "i8") if t in args.quant_types.split(",")]
    for quant, pq in ((t, {"f32": P.F32, "i16": P.I16, "i8": P.I8}[t]) for t in types):
        plan = P.Plan(Q["N"], Q["K"], Q["crc_len"], Q["crc_poly"], design_ebn0_db=Q["design"],
                      algo=P.CA_SCL, L=Q["L"], quant=pq, rep_max=8 if quant == "i8" else 0, spc_max=4)
        kd = plan.info.k_data
        pts = {}
        for i, eb in enumerate(Q["points"]):
            fe, be, ms = 0, 0, 0.0
            for f0 in range(0, F, C):
                n = min(C, F - f0)
                data = P.gen_data(plan, 5000 + i, f0, n)
                llr = P.channel(plan, P.encode(plan, data), eb, 6000 + i, f0)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                info, _, _ = P.decode_batch(plan, llr, stream=stream)
                e1.record(stream)
                x = torch.bitwise_xor(info, data)
                fe += int((x != 0).any(dim=1).sum().item())
                be += int(pop[x.contiguous().view(torch.uint8).long()].sum().item())
                ms += e0.elapsed_time(e1)
                del data, llr, info, x
            fer, ber = fe / F, be / (F * kd)
            pts[str(eb)] = {"frames": F, "frame_errors": fe, "bit_errors": be, "fer": fer, "ber": ber,
                            "fer_ci95": list(wilson(fe, F)), "decode_ms": round(ms, 1),
                            "info_mbps": round(F * kd / (ms / 1e3) / 1e6, 1),
                            "coded_mbps": round(F * Q["N"] / (ms / 1e3) / 1e6, 1)}
            print(f"quant {quant} {eb} dB: {pts[str(eb)]}", file=sys.stderr, flush=True)
        rec = {"points": pts}
        if not args.no_cpu and args.quant_oracle > 0:
            errs, mbps = quant_oracle_leg(quant, Q["points"], args.quant_oracle, host_cores())
            oracle_mbps[quant] = round(mbps, 3)
            for eb in Q["points"]:
                pp = pts[str(eb)]
                ofe, obe = errs[eb]
                lo, hi = wilson(ofe, args.quant_oracle)
                pp["oracle_frame_errors"], pp["oracle_bit_errors"] = ofe, obe
                pp["oracle_fer_ci95"] = [lo, hi]
                glo, ghi = pp["fer_ci95"]
                pp["fer_matched"] = bool(lo <= pp["fer"] <= hi or (glo <= hi and lo <= ghi))
        rows[quant] = rec
    tot_bits = sum(p["frames"] * (Q["K"] - Q["crc_len"]) for r in rows.values() for p in r["points"].values())
    tot_ms = sum(p["decode_ms"] for r in rows.values() for p in r["points"].values())
    cpu = None
    if oracle_mbps:
        cpu = {"value": round(sum(oracle_mbps.values()) / len(oracle_mbps), 3), "unit": "Mb/s",
               "cores": host_cores(), "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{args.quant_oracle} host-generated frames per Eb/N0 point and LLR type, "
                         f"frame-parallel over {host_cores()} threads; decode time only; the mean "
                         f"of the types' rates",
               "per_quant_mbps": oracle_mbps}
    return {"metric": "info Mb/s per MI355X at matched FER + p50/p99 decode latency, batched vs plain",
            "value": round(tot_bits / (tot_ms / 1e3) / 1e6, 1), "unit": "Mb/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": round(tot_ms, 1), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32/i16/i8", "data": "synthetic",
            "cpu_baseline": cpu,
            "config": {"workload": "quant_sweep_n1024_k512_crc24_ca_l8", "frames_per_point": F,
                       "ebn0_db": Q["points"], "quants": rows}}


def headline(args):
    """The headline workload: FA-SSCL on the (2048, 1723) code at three Eb/N0
    points; returns the JSON record (value, per-point figures, roofline)."""
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
    per_point = {}
    for (eb, data, llr), (info, status) in zip(batches, outs):
        err = (info != data).any(dim=1)
        n_err = int(err.sum().item())
        lu = status[:, 1].to(torch.int64)
        hist = torch.bincount(lu, minlength=W["L_max"] + 1).cpu().numpy()
        lo, hi = wilson(n_err, F)
        per_point[str(eb)] = {"fer": n_err / F, "fer_ci95": [lo, hi], "frame_errors": n_err,
                              "crc_fail": int((status[:, 0] == 0).sum().item()),
                              "L_used_hist": {str(l): int(hist[l]) for l in sched if hist[l]},
                              "avg_stages": float(sum(hist[l] * (sched.index(l) + 1)
                                                      for l in sched) / F)}
    khz = P.device_clock_khz()

    def latency(llr, schedule, pl=plan):
        times = torch.zeros((F, 2), dtype=torch.int64, device="cuda")
        P.decode_batch(pl, llr, schedule=schedule, stream=stream, times=times)
        torch.cuda.synchronize()
        t = times.cpu().numpy().astype(np.float64)
        svc = (t[:, 1] - t[:, 0]) / khz * 1e3  # us
        done = (t[:, 1] - t[:, 0].min()) / khz * 1e3
        return {"decode_p50_us": round(float(np.percentile(svc, 50)), 2),
                "decode_p99_us": round(float(np.percentile(svc, 99)), 2),
                "decode_mean_us": round(float(svc.mean()), 2),
                "decode_max_us": round(float(svc.max()), 2),
                "batch_completion_p50_us": round(float(np.percentile(done, 50)), 1),
                "batch_completion_p99_us": round(float(np.percentile(done, 99)), 1)}

    # the plain form (one generic launch per configuration), same inputs:
    # time and per-frame latency
    plain_ms = {}
    if args.schedule == 0 and args.compare_plain:
        for eb, data, llr in batches:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            P.decode_batch(plan, llr, schedule=1, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            plain_ms[eb] = e0.elapsed_time(e1)
            per_point[str(eb)]["plain_latency"] = latency(llr, 1)
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
    tier_bytes = {t: 0 for t in tier_ms}
    # algorithmic HBM bytes of a frame-stage: its LLRs in, its data bits and status out
    alg_bytes = W["N"] + 4 * ((kd + 31) // 32) + 8
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
            # every list stage of this workload runs in the library's second
            # list interval (the first stays empty)
            tier = "sc" if l == 1 else "list_b"
            tier_work[tier] += reached * plan.stage_work(l)
            tier_bytes[tier] += reached * alg_bytes

    # ---- latency of the automatic schedule: per-frame decode time from
    # device realtime stamps
    for eb, data, llr in batches:
        per_point[str(eb)]["latency"] = latency(llr, args.schedule)

    # ---- partially adaptive SSCL (stages 1, L_max) on the same inputs
    pa = {}
    if args.pa:
        pplan = P.Plan(W["N"], W["K"], W["crc_len"], W["crc_poly"], design_ebn0_db=W["design"],
                       algo=P.PA_SCL, L_max=W["L_max"], quant=P.I8, rep_max=8, spc_max=4)
        for eb, data, llr in batches:
            P.decode_batch(pplan, llr, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            info, status, _ = P.decode_batch(pplan, llr, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            n_err = int((info != data).any(dim=1).sum().item())
            lat = latency(llr, 0, pplan)
            pa[str(eb)] = {"kernel_ms": round(ms, 3), "info_mbps": round(F * kd / (ms / 1e3) / 1e6, 1),
                           "fer": n_err / F, "fer_ci95": list(wilson(n_err, F)),
                           "decode_mean_us": lat["decode_mean_us"],
                           "decode_max_us": lat["decode_max_us"],
                           "decode_p99_us": lat["decode_p99_us"],
                           "fa_info_mbps": per_point[str(eb)]["info_mbps"],
                           "fa_decode_mean_us": per_point[str(eb)]["latency"]["decode_mean_us"],
                           "fa_decode_max_us": per_point[str(eb)]["latency"]["decode_max_us"]}

    total_bits = args.steps * len(points) * F * kd
    value = total_bits / elapsed / 1e6
    kernel_names = {"sc": "k_rq<11,1>", "list_a": "k_decode_list<int8,1,4>",
                    "list_b": " + ".join(LIST_KERNELS)}
    tiers = {}
    for t in tier_ms:
        if tier_ms[t] > 0 and tier_work[t] > 0:
            ach = tier_work[t] / (tier_ms[t] / 1e3)
            tiers[t] = {"kernel": kernel_names[t], "launch_ms": round(tier_ms[t] / len(points), 3),
                        "work_per_launch_ops": int(tier_work[t] / len(points)),
                        "achieved": round(ach / 1e12, 5), "frac": round(ach / VALU_PEAK_OPS, 6)}
            # measured HBM bytes per launch (counter summary), against the 8 TB/s peak
            tiers[t]["alg_bytes_per_launch"] = int(tier_bytes[t] / len(points))
            tb = measured_traffic(kernel_names[t])
            if tb:
                rate = tb / (tier_ms[t] / len(points) / 1e3)
                tiers[t].update({"traffic": tb, "hbm_tbs": round(rate / 1e12, 3),
                                 "hbm_frac": round(rate / HBM_PEAK_BYTES, 4)})
            # the bound, from the kernels' own counters: memory when the measured
            # HBM rate is the larger fraction of its peak than VALU busy is of
            # the issue rate (the algorithmic-op fraction where no counters are)
            busy = measured_valu_busy(kernel_names[t])
            if busy is not None:
                tiers[t]["valu_busy"] = round(busy, 4)
            tiers[t]["bound"] = tier_bound(tiers[t].get("hbm_frac"), busy, tiers[t]["frac"])
    # the dominant kernel: the single kernel with the longest average launch
    # (the L = 1 stage; each list stage runs as a launch of its own, shorter
    # on average over the points)
    dom = "sc" if "sc" in tiers else max(tiers, key=lambda t: tiers[t]["launch_ms"])
    roofline = {"bound": tiers[dom]["bound"], "achieved": tiers[dom]["achieved"],
                "peak": round(VALU_PEAK_OPS / 1e12, 2), "unit": "Tops/s",
                "frac": tiers[dom]["frac"], "traffic": measured_traffic(tiers[dom]["kernel"]),
                "kernel": tiers[dom]["kernel"],
                "work_per_launch_ops": tiers[dom]["work_per_launch_ops"],
                "launch_ms": tiers[dom]["launch_ms"], "tiers": tiers}
    if roofline["bound"] == "hbm":
        # algorithmic bytes per launch over the launch time (the counters' bytes are `traffic`)
        ab = tiers[dom]["alg_bytes_per_launch"] / (tiers[dom]["launch_ms"] / 1e3)
        roofline.update({"achieved": round(ab / 1e9, 1), "peak": HBM_PEAK_BYTES / 1e9,
                         "unit": "GB/s", "frac": round(ab / HBM_PEAK_BYTES, 4)})

    return {
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
                   "per_point": per_point, "pa_sscl": pa or None},
        "roofline": roofline,
    }


def compact_uneven(r):
    c = r["config"]
    return {"workload": c["workload"], "frames": c["frames"], "plans": c["plans"], "dtype": r["dtype"],
            "batched_info_mbps": c["batched_info_mbps"], "batched_kernel_ms": c["batched_kernel_ms"],
            "graph_info_mbps": c["graph_info_mbps"], "plain_info_mbps": c["plain_info_mbps"],
            "coded_mbps": c["coded_mbps"], "schedule": c["schedule"].split(";")[0],
            "latency": {k: v for k, v in c["latency"].items() if k != "per_list_size"}}


def compact_served(r):
    out = {"workload": r["config"]["workload"]}
    for q, v in r["config"]["per_quant"].items():
        out[q] = {"requests": v["requests"], "plans": v["plans"],
                  "batched_info_mbps": v["batched"]["info_mbps"],
                  "plain_info_mbps": v["plain"]["info_mbps"],
                  "served": {rate: {k: x[k] for k in ("served_mreq_s", "info_mbps", "latency_p50_us",
                                                       "latency_p99_us", "results_equal_batch")}
                             for rate, x in v["served"].items()}}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=1_000_000, help="frames per Eb/N0 point")
    ap.add_argument("--points", default="3.5,4.0,4.5")
    ap.add_argument("--schedule", type=int, default=0, help="0 automatic, 1 plain")
    ap.add_argument("--cpu-frames", type=int, default=3000, help="oracle sample per point")
    ap.add_argument("--cpu-frames-1core", type=int, default=500,
                    help="oracle one-core sample per point")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--compare-plain", type=int, default=1,
                    help="also time the plain one-launch form once per point")
    ap.add_argument("--pa", type=int, default=1, help="also run PA-SSCL (stages 1, L_max)")
    ap.add_argument("--extras", type=int, default=1,
                    help="also run compact records of the uneven batch and of serving")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (HBM counter calibration)")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "uneven", "served", "pruning", "quant"],
                    help="uneven: the batched uneven launch (2^20 frames of mixed codes); "
                         "served: Poisson arrivals of mixed-size requests through the serving loop; "
                         "quant: the quantisation sweep at scale")
    ap.add_argument("--quant-frames", type=int, default=10_000_000,
                    help="quant workload: frames per Eb/N0 point and LLR type")
    ap.add_argument("--quant-oracle", type=int, default=1_000_000,
                    help="quant workload: oracle sample per point (0: none)")
    ap.add_argument("--quant-types", default="f32,i16,i8",
                    help="quant workload: LLR types to sweep (comma list of f32, i16, i8)")
    args = ap.parse_args()
    if args.calib_copy:
        calib_copy(args.calib_copy)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: the decoder shards frames across GPUs with no "
              "collective, so only --gpus 1 is measured", file=sys.stderr)
        sys.exit(2)
    if args.workload in ("uneven", "served", "pruning", "quant"):
        r = {"uneven": bench_uneven, "served": bench_served, "pruning": bench_pruning,
             "quant": bench_quant}[args.workload](args)
        print(json.dumps(r))
        return

    out = headline(args)
    if args.extras:
        sub = argparse.Namespace(**vars(args))
        sub.frames = 1_000_000  # each workload's own default size
        sub.steps, sub.warmup, sub.compare_plain = 3, 1, 1
        out["config"]["batched_uneven"] = compact_uneven(bench_uneven(sub))
        out["config"]["served"] = compact_served(bench_served(sub))
    if not args.no_cpu:
        points = out["config"]["ebn0_db"]
        rec, errs = cpu_baseline(points, args.cpu_frames, host_cores(), args.cpu_frames_1core)
        out["cpu_baseline"] = rec
        # matched FER: the GPU's FER lies in the oracle sample's 95% interval
        for eb in points:
            pp = out["config"]["per_point"][str(eb)]
            lo, hi = wilson(errs[eb], args.cpu_frames)
            pp["oracle_fer_ci95"] = [lo, hi]
            pp["fer_matched"] = bool(lo <= pp["fer"] <= hi)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
