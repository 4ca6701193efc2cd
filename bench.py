#!/usr/bin/env python3
"""Benchmark of the fused compressed gate-apply path on one MI355X.

Default workload "qaoa34": the largest configuration that one GPU holds, a
34-qubit QAOA circuit (H on every qubit, p = 4 layers of Rzz on a seeded
3-regular graph and Rx mixers; 374 gates) on complex128 amplitudes, 2^20-
amplitude blocks (chunks of 1024 amplitudes), error bound 1e-5 on every gate,
256 GiB uncompressed.  The circuit is one continuing run cut into
warmup + steps windows of consecutive gates; a step is one window.  Inputs
(gate list, compressed state) are in HBM before timing.  Gates whose jobs
lie inside single chunks run fused (one pass per run), chunk-pair gates on
up to three chunk-index qubits run as one pass over groups of eight chunks, a gate
that does not fit beside the live streams sweeps into the other arena, and
the windows are cut at the boundaries of those passes.  Other workloads:
grover24+qft24 (the 24-qubit pair), grid30, grover34.

Prints one JSON line:
  value      = amplitudes through the fused kernel (touched chunks) per second
               of the timed region, in GAmp/s;
  roofline   = the fused kernel's algorithmic bytes (compressed streams read +
               written + 24 table/undo bytes per chunk) over its event-timed
               duration, against 8 TB/s, with the counter-measured traffic and
               VALU-busy fraction when the profiles match the kernel source;
  cpu_baseline = the CPU oracle on chunks exported from the same state, one
               core and all host cores.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "fused compressed gate-apply GAmp/s + compression ratio at fidelity ≥0.99"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def grover_fidelity(st, n, w, iters):
    """|<ideal|sim>| with ideal = closed form; uses sum of amplitudes and the
    marked amplitude (no full readout)."""
    theta = math.asin(2.0 ** (-n / 2))
    sign = (-1) ** iters
    beta = sign * math.sin((2 * iters + 1) * theta)
    alpha = sign * math.cos((2 * iters + 1) * theta) / math.sqrt((1 << n) - 1)
    total, norm2 = st.moments()
    aw = st.read([w])[0]
    ov = alpha * (total - aw) + beta * aw
    return abs(ov), math.sqrt(norm2), abs(aw)


def qft_fidelity(st, n, x_in):
    import torch
    N = 1 << n
    psi = torch.empty(st.nchunks * st.C, dtype=torch.float64, device="cuda")
    st.decode_to(0, st.nchunks, psi)
    psi = torch.view_as_complex(psi.view(-1, 2))
    y = torch.arange(N, device="cuda", dtype=torch.int64)
    rev = torch.zeros_like(y)
    for b in range(n):
        rev |= ((y >> b) & 1) << (n - 1 - b)
    ph = (2 * math.pi / N) * ((x_in * rev) % N).to(torch.float64)
    ideal = torch.polar(torch.full_like(ph, 1.0 / math.sqrt(N)), ph)
    ov = torch.sum(torch.conj(ideal) * psi).item()
    nrm = torch.linalg.vector_norm(psi).item()
    return abs(ov), nrm


def _cpu_worker(job):
    """One worker of the CPU leg: gate jobs of the oracle over exported chunks
    until its share of the budget is spent; returns (amplitudes, seconds)."""
    from oracle import qcz_oracle as oq
    gates, chunks, cb, C, level, flags, budget = job
    amps, t_all, k = 0, 0.0, 0
    while t_all < budget:
        g, c0, b0, c1, b1 = chunks[k % len(chunks)]
        gate = gates[g:g + 1]
        t0 = time.perf_counter()
        if c1 is None:
            oq.gate_job(gate, cb, C, c0, b0, level, flags=flags)
            amps += C // 2
        else:
            oq.gate_job(gate, cb, C, c0, b0, level, c1, b1, level, flags=flags)
            amps += C
        t_all += time.perf_counter() - t0
        k += 1
    return amps, t_all


def cpu_baseline(st, gates, level, budget_s: float, entropy: bool = False, desc: str = ""):
    """The C oracle on a bounded sample of the same workload: chunks exported
    from the GPU state where the timed region ended (each gate's input chunks,
    as the blockwise loop reads them), pushed through the oracle's decode ->
    gate -> encode (Sec. 3.1/3.3) for the workload's own gates.  First single-
    threaded, then one process per host core; GAmp/s over the amplitudes of
    the re-encoded chunks."""
    import multiprocessing as mp
    from oracle import qcz_oracle as oq
    cb, C = st.cb, st.C
    flags = oq.ENC_ENTROPY if entropy else 0
    rng = np.random.default_rng(7)
    sample = []
    for gi in range(len(gates)):
        g = gates[gi:gi + 1]
        q = int(g["target"][0])
        kind = int(g["kind"][0])
        for c in rng.choice(st.nchunks, size=4, replace=False):
            c = int(c)
            if kind in (0, 3) and q >= cb:
                c0 = c & ~(1 << (q - cb))
                c1 = c0 | (1 << (q - cb))
                sample.append((gi, c0, st.export_chunk(c0), c1, st.export_chunk(c1)))
            else:
                sample.append((gi, c, st.export_chunk(c), None, None))
    half = budget_s / 2
    a1, t1 = _cpu_worker((gates, sample, cb, C, level, flags, half))
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    cores = min(cores, int(os.environ.get("QCZ_CPU_WORKERS", "16")))   # the host's CPU share for one GPU
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(gates, sample[i::cores] or sample, cb, C, level, flags, half)
                                     for i in range(cores)])
    wall = time.perf_counter() - t0
    amps = sum(a for a, _ in res)
    model = ""
    try:
        model = next(x.split(":", 1)[1].strip() for x in open("/proc/cpuinfo") if x.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": amps / wall / 1e9, "unit": "GAmp/s", "cores": cores, "kind": "oracle",
            "single_core": a1 / t1 / 1e9, "cpu_model": model, "nproc": os.cpu_count(),
            "sample": "%s: %d chunk jobs (input chunks of the workload's gates, exported from the GPU state at the "
                      "end of the timed region) through the C oracle's decode -> gate -> encode, %.1f s on one core "
                      "then %.1f s wall on %d processes" % (desc, len(sample), t1, wall, cores)}


LARGE = {
    # name: (qubits, block_log2, description)
    "grid30": (30, 20, "30-qubit 5x6-grid random circuit, depth 20, {sqrtX, sqrtY, T} + CZ patterns, bound 1e-4"),
    "grover34": (34, 20, "34-qubit Grover, 8 iterations, bound 1e-5 (256 GiB uncompressed)"),
    "qaoa34": (34, 20, "34-qubit QAOA, p=4 on a seeded 3-regular graph, bound 1e-5 on every gate (Eq. (11) "
                       "fidelity lower bound >= 0.99 over the 374 gates); with --selector also the learned "
                       "per-block levels (256 GiB uncompressed)"),
}


def large_config(args, torch, cc, qcz):
    """A large configuration as one continuing run: the circuit is cut into
    warmup + steps windows of consecutive gates; the warmup windows run first,
    the timed steps are the rest (inputs: the gate list and the compressed
    state, both in HBM before timing).  Fidelity after the timed region."""
    n, bl, desc = LARGE[args.workload]
    free, _total = torch.cuda.mem_get_info()
    budget = 0
    w = None
    if args.workload == "grid30":
        gates, level, mode, pool = cc.grid_rcs(5, 6, 20, 3), 2, qcz.MODE_FIXED, 40 << 30
    elif args.workload == "grover34":
        w = cc.grover_marked(n, 4)
        gates = cc.concat([cc.grover_prefix(n)] + [cc.grover_iteration(n, w)] * 8)
        level, mode, pool = 1, qcz.MODE_FIXED, min(250 << 30, free - (12 << 30))
    else:
        gates = cc.qaoa(n, 4, 3, 5)[0]
        level, mode = 1, qcz.MODE_FIXED
        pool = min(250 << 30, free - (12 << 30))
    if args.level >= 0:
        level = args.level
    if args.gates:
        gates = gates[:args.gates]
    flags = qcz.FLAG_TIMING | qcz.FLAG_RANGES | (0 if args.no_fuse else qcz.FLAG_FUSE) | \
        (qcz.FLAG_ENTROPY if args.entropy else 0) | (0 if args.no_groups else qcz.FLAG_GROUPS)
    passes = args.warmup + args.steps
    if args.no_fuse:
        win = -(-len(gates) // passes)
        windows = [gates[k:k + win] for k in range(0, len(gates), win)]
    else:
        cb = min(bl, 10)
        windows = pass_windows(gates, cb, passes, not args.no_groups and not args.entropy,
                               group_bits=3 if n - cb >= 3 else 2)
    win = max(len(w) for w in windows)
    st = qcz.State(n, bl, mode=mode, level=level, budget=budget, pool_bytes=pool, flags=flags, batch=128)
    trace = [st.footprint()["compressed_bytes"]]
    walls = []
    t_all = None
    for p, wg in enumerate(windows):
        if p == args.warmup:
            torch.cuda.synchronize()
            st.reset_stats()
            c0 = st.footprint()["compactions"]
            t_all = time.perf_counter()
        t0 = time.perf_counter()
        st.apply(wg)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        fp = st.footprint()
        trace.append(fp["compressed_bytes"])
        log("%s window %d/%d (%d gates): level %d, compressed %.2f GB, %.2f s" % (
            args.workload, p + 1, len(windows), len(wg), fp["level"], fp["compressed_bytes"] / 1e9, walls[-1]))
    wall = time.perf_counter() - t_all if t_all is not None else 0.0
    stats = st.stats()
    fp = st.footprint()
    timed_steps = len(windows) - args.warmup
    fid = {"fidelity_lower_bound": fp["fidelity_lower_bound"]}
    if args.workload == "grid30":
        # the uncompressed fp64 reference: the same circuit in lossless mode (every stored value is the exact
        # fp64 result of the gate arithmetic), compared through qcz_overlap (Eq. (9))
        log("lossless fp64 reference run")
        ex = qcz.State(n, bl, mode=qcz.MODE_LOSSLESS, pool_bytes=40 << 30, flags=qcz.FLAG_RANGES, batch=128)
        ex.apply(gates)
        ov = st.overlap(ex)
        n2 = st.moments()[1]
        fid.update({"fidelity_raw": abs(ov), "fidelity_norm": abs(ov) / math.sqrt(n2)})
        ex.close()
    elif args.workload == "grover34" and not args.gates:
        f_raw, nrm, aw = grover_fidelity(st, n, w, 8)
        fid.update({"fidelity_raw": f_raw, "fidelity_norm": f_raw / nrm, "marked_probability": aw ** 2})
    amps = stats["amps_touched"]
    kms = stats["gate_kernel_ms"]
    timed = stats["timed_launches"]
    from paper_1911_04034_amd import profile_summary as ps
    suffix = "_entropy" if args.entropy else ""
    kinds = {0: ("job_kernel", "job_kernel<16, 2, ARENA, ARENA, gate%s>: one gate per pass" % suffix.replace("_", ", ")),
             1: ("run_kernel", "job_kernel<16, 2, ARENA, ARENA, gate, run%s>: a fused run of single-chunk gates per pass"
                 % suffix.replace("_", ", ")),
             2: ("group_kernel", "group_kernel<16, NB>: a run of chunk-pair gates on up to three chunk-index qubits per pass")}
    per = []
    for i, (tag, name) in kinds.items():
        L, ms, B = stats["kind_launches"][i], stats["kind_kernel_ms"][i], stats["kind_bytes"][i]
        if L == 0 or ms <= 0:
            continue
        t_bytes, t_hash = ps.read_traffic(os.path.join(ROOT, "profiles", "traffic_%s_%s%s.txt" % (tag, args.workload,
                                                                                              suffix)))
        busy, b_hash = ps.read_valu_busy(os.path.join(ROOT, "profiles", "counters_%s_%s%s.txt" % (tag, args.workload,
                                                                                              suffix)))
        achieved = B / (ms * 1e-3) / 1e9
        per.append({"kernel": name, "launches": L, "kernel_ms": round(ms, 1), "share_of_kernel_time": round(ms / kms, 4),
                    "avg_launch_us": round(ms / L * 1e3, 3), "algorithmic_bytes_per_launch": round(B / L, 1),
                    "achieved": round(achieved, 3), "frac": round(achieved / HBM_PEAK_GBS, 6),
                    "traffic": round(t_bytes, 1) if t_bytes is not None and t_hash == ps.kernel_hash() else None,
                    "alu_frac": busy.get(args.workload + suffix) if busy and b_hash == ps.kernel_hash() else None})
    dom = max(per, key=lambda k: k["kernel_ms"]) if per else {"kernel": None, "achieved": 0.0, "frac": 0.0,
                                                                "traffic": None, "alu_frac": None,
                                                                "avg_launch_us": 0.0,
                                                                "algorithmic_bytes_per_launch": 0.0, "launches": 0}
    roofline = {"bound": "hbm", "achieved": dom["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom["frac"], "traffic": dom["traffic"], "alu_frac": dom["alu_frac"], "kernel": dom["kernel"],
                "avg_launch_us": dom["avg_launch_us"], "algorithmic_bytes_per_launch": dom["algorithmic_bytes_per_launch"],
                "launches": dom["launches"], "all_launches": timed, "range_launches": stats["range_launches"],
                "sweep_gates": stats["sweep_gates"], "kernels": per}
    codecs = None
    if not args.gates:
        codecs = codec_comparison(torch, qcz, st, max(1, level))
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline(st, windows[-1], level, args.cpu_seconds, args.entropy,
                           "%d-qubit %s state after gate %d, its last %d gates" % (n, args.workload, len(gates),
                                                                                  len(windows[-1])))
    line = {
        "metric": METRIC, "value": round(amps / wall / 1e9, 4) if wall > 0 else 0.0, "unit": "GAmp/s", "n_gpus": 1,
        "steps": timed_steps, "warmup": args.warmup,
        "ms_per_step": round(wall / max(1, timed_steps) * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "qubits": n, "block_amplitudes": 1 << bl,
                   "bound": [0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1][level], "gates": int(len(gates)),
                   "gates_per_step": win, "final_level": fp["level"], "pool_bytes": int(pool),
                   "entropy_stage": bool(args.entropy), "fused_runs": not args.no_fuse,
                   "chunk_group_runs": not (args.no_groups or args.no_fuse or args.entropy),
                   "parallelism": "single GPU"},
        "compression_ratio_min": round(fp["raw_bytes"] / (fp["max_compressed"] + fp["table_bytes"]), 3),
        "compression_ratio_final": round(fp["ratio"], 3),
        "peak_compressed_bytes": fp["max_compressed"],
        "fidelity": fid,
        "logical_gamp_s": round(sum(len(wg) for wg in windows[args.warmup:]) * (1 << n) / wall / 1e9, 3)
        if wall > 0 else None,
        "fused_kernel_gamp_s": round(amps / (kms * 1e-3) / 1e9, 3) if kms > 0 else None,
        "kernel_share_of_wall": round(kms * 1e-3 / wall, 4) if wall > 0 else None,
        "compactions": fp["compactions"] - c0 if t_all is not None else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "codec_comparison": codecs,
    }
    if args.workload == "qaoa34" and args.selector:
        line["selector"] = selector_run(args, torch, cc, qcz, n, bl, gates, pool, trace, st,
                                        [0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1][level])
    if args.workload == "qaoa34" and not args.gates and args.fidelity_qubits:
        st.close()   # (also after the selector run, which closed it: closing twice is harmless)
        torch.cuda.empty_cache()
        line["fidelity"]["same_generator"] = qaoa_fidelity(qcz, cc, args.fidelity_qubits, bl, level, flags)
    print(json.dumps(line), flush=True)


def pass_windows(gates, cb, nwin, groups, max_run=64, group_bits=3):
    """Cut the gate list into nwin consecutive windows at the boundaries of
    the passes the library forms with fused runs (gates whose jobs lie inside
    single chunks: one pass per run of up to 64; chunk-pair gates: one pass
    each, or per run on at most group_bits target qubits with chunk-group
    runs), so that no step splits a pass; windows hold near-equal numbers of
    passes."""
    U1, DIAG1, DIAG2, X, MCZ = 0, 1, 2, 3, 4
    lo = (1 << cb) - 1
    passes, cur, kind, bits = [], [], None, set()
    for i in range(len(gates)):
        g = gates[i]
        k, t, cm = int(g["kind"]), int(g["target"]), int(g["control_mask"])
        if k in (DIAG1, DIAG2, MCZ) or t < cb:
            c = "single"
        elif k == X and (cm & lo) == 0:
            c = "permute"
        else:
            c = "pair"
        joins = (c == kind and len(cur) < max_run and
                 (c == "single" or (c == "pair" and groups and len(bits | {t}) <= group_bits)))
        if not joins and cur:
            passes.append(cur)
            cur, bits = [], set()
        cur.append(i)
        kind = c
        if c == "pair":
            bits.add(t)
    if cur:
        passes.append(cur)
    nwin = max(1, min(nwin, len(passes)))
    out, start = [], 0
    for w in range(nwin):
        end = round((w + 1) * len(passes) / nwin)
        idx = [i for p in passes[start:end] for i in p]
        out.append(gates[idx[0]:idx[-1] + 1])
        start = end
    return out


def codec_comparison(torch, qcz, st, level, nchunks=65536):
    """The paper's comparison of its lossy solutions (Sec. 4.2) on the final
    state: a contiguous sample of chunks from the middle of the state, decoded
    once, then encoded at the run's bound with Solution C (the state's codec),
    Solution C with the entropy stage, Solution D (re/im separated, with and
    without the entropy stage) and Solution B (log-domain prediction, 16,384
    bins, Huffman).  Compression ratio = raw bytes / stream bytes (4-byte
    padded); rates in GB/s of raw input through the encoder and the decoder
    (device timing of one call each, after one warm call)."""
    n = min(nchunks, st.nchunks)
    first = (st.nchunks - n) // 2
    C = st.C
    raw = torch.empty(n * C, dtype=torch.float64, device="cuda")
    st.decode_to(first, n, raw)
    raw = raw.view(n, C)
    out = {"sample": "%d chunks of %d amplitudes from the middle of the final state, bound %g" % (
        n, C // 2, [0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1][level])}
    variants = {"C": 0, "C+entropy": qcz.CODEC_ENTROPY, "D": qcz.CODEC_RESHUFFLE,
                "D+entropy": qcz.CODEC_RESHUFFLE | qcz.CODEC_ENTROPY, "B": qcz.CODEC_PREDICT}
    for name, flags in variants.items():
        try:
            qcz.encode_chunks(raw, level, codec_flags=flags)
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record()
            slots, sizes = qcz.encode_chunks(raw, level, codec_flags=flags)
            t1.record()
            torch.cuda.synchronize()
            enc_ms = t0.elapsed_time(t1)
            qcz.decode_chunks(slots, sizes, C)
            t0.record()
            dec = qcz.decode_chunks(slots, sizes, C)
            t1.record()
            torch.cuda.synchronize()
            dec_ms = t0.elapsed_time(t1)
            stream = int(((sizes.to(torch.int64) + 3) // 4 * 4).sum().item())
            ok = bool((sizes > 0).all().item())
            err = torch.abs(dec - raw) <= [0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1][level] * torch.abs(raw)
            out[name] = {"compression_ratio": round(raw.numel() * 8 / stream, 3),
                         "encode_gbs": round(raw.numel() * 8 / (enc_ms * 1e-3) / 1e9, 1),
                         "decode_gbs": round(raw.numel() * 8 / (dec_ms * 1e-3) / 1e9, 1),
                         "bound_held": bool(err.all().item()) and ok}
            del slots, sizes, dec
        except Exception as e:   # (a codec that rejects the chunk size)
            out[name] = {"error": str(e)}
    del raw
    torch.cuda.empty_cache()
    log("codec comparison: %s" % json.dumps(out))
    return out


def qaoa_fidelity(qcz, cc, n, bl, level, flags):
    """End-to-end fidelity of the compressed run against uncompressed fp64 on
    the same QAOA generator at n qubits: the reference is the lossless run
    (every stored value the exact fp64 result of the gate arithmetic),
    compared through qcz_overlap (Eq. (9))."""
    gates = cc.qaoa(n, 4, 3, 5)[0]
    log("fidelity: %d-qubit QAOA, lossless reference and level %d" % (n, level))
    ex = qcz.State(n, bl, mode=qcz.MODE_LOSSLESS, pool_bytes=48 << 30, flags=qcz.FLAG_FUSE | qcz.FLAG_RANGES,
                   batch=128)
    ex.apply(gates)
    lo = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=level, pool_bytes=24 << 30,
                   flags=(flags & ~qcz.FLAG_TIMING) | qcz.FLAG_RANGES, batch=128)
    lo.apply(gates)
    ov = lo.overlap(ex)
    n2_lo, n2_ex = lo.moments()[1], ex.moments()[1]
    fp = lo.footprint()
    out = {"qubits": n, "gates": int(len(gates)), "fidelity_raw": abs(ov),
           "fidelity_norm": abs(ov) / math.sqrt(n2_lo * n2_ex), "fidelity_lower_bound": fp["fidelity_lower_bound"],
           "compression_ratio_final": round(fp["ratio"], 3),
           "compression_ratio_lossless": round(ex.footprint()["ratio"], 3)}
    ex.close()
    lo.close()
    return out


def selector_run(args, torch, cc, qcz, n, bl, gates, pool, trace, st, beta):
    """The learned per-block levels at the rule's per-step budget (the bound
    of the run's level), trained on the device from teacher traces of small
    circuits."""
    from paper_1911_04034_amd import selector as sel
    train = [(cc.biased_local(12, 6, 8, 1), 12, 6), (cc.biased_local(13, 7, 8, 2), 13, 7),
             (cc.biased_local(13, 6, 8, 3), 13, 6), (cc.grover(12, 12, 11)[0], 12, 6),
             (cc.random_circuit_small(12, 12, 13), 12, 6), (cc.qft(12, cc.qft_input(12, 14)), 12, 6),
             (cc.qaoa(12, 3, 3, 15)[0], 12, 6)]
    log("selector: teacher traces and training")
    X, y = sel.training_set(train, (1e-5, 1e-4, 1e-3), 16)
    params, losses = sel.train(X, y, steps=1500, lr=3e-3, seed=0)
    acc = sel.accuracy(params, X, y)
    st.close()
    torch.cuda.empty_cache()
    st2 = qcz.State(n, bl, mode=qcz.MODE_PERBLOCK, level=0, pool_bytes=pool, batch=128, flags=qcz.FLAG_RANGES)
    st2.set_selector(params, beta, 16)
    t0 = time.perf_counter()
    strace = []
    for k in range(0, len(gates), 16):
        st2.apply(gates[k:k + 16])
        f2 = st2.footprint()
        strace.append(f2["compressed_bytes"])
        log("qaoa34 selector: %d/%d gates, compressed %.2f GB" % (min(k + 16, len(gates)), len(gates),
                                                                  f2["compressed_bytes"] / 1e9))
    torch.cuda.synchronize()
    f2 = st2.footprint()
    return {"train_samples": int(X.shape[0]), "train_loss": [round(losses[0], 4), round(losses[-1], 4)],
            "train_accuracy": round(acc, 4), "wall_s": round(time.perf_counter() - t0, 2),
            "mean_compressed_bytes": float(np.mean(strace)), "peak_compressed_bytes": f2["max_compressed"],
            "fidelity_lower_bound": f2["fidelity_lower_bound"],
            "rule_mean_compressed_bytes": float(np.mean(trace)),
            "gain_mean_bytes": round(float(np.mean(trace)) / float(np.mean(strace)), 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="qaoa34",
                    choices=["grover24+qft24", "grover24", "qft24"] + sorted(LARGE))
    ap.add_argument("--grover-iters", type=int, default=32,
                    help="Grover iterations per step (0: spread the full 3216 over warmup+steps)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=24.0,
                    help="CPU leg: half on one core, half on all host cores")
    ap.add_argument("--gates", type=int, default=0, help="large configurations: only the first GATES gates "
                    "(profiling runs)")
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--chunk-waves", type=int, default=0, help="wavefronts per chunk in the fused kernel (2, 4, 8)")
    ap.add_argument("--no-timing", action="store_true", help="launch from graphs instead of timing each kernel")
    ap.add_argument("--selector", action="store_true", help="qaoa34: also run the learned per-block selector")
    ap.add_argument("--fuse", action="store_true",
                    help="grover24/qft24: fuse runs of gates whose jobs lie inside single chunks (a separate figure)")
    ap.add_argument("--level", type=int, default=-1,
                    help="large configurations: error-bound level (0 lossless, 1..5: 1e-5 .. 1e-1)")
    ap.add_argument("--fidelity-qubits", type=int, default=30,
                    help="qaoa34: also measure the fidelity against lossless fp64 on the same generator at this "
                         "many qubits (0: skip)")
    ap.add_argument("--no-groups", action="store_true",
                    help="large configurations: chunk-pair gates one pass each instead of chunk-group runs on two "
                         "chunk-index qubits (QCZ_FLAG_GROUPS)")
    ap.add_argument("--no-fuse", action="store_true",
                    help="large configurations: one pass per gate instead of fused runs (QCZ_FLAG_FUSE)")
    ap.add_argument("--entropy", action="store_true",
                    help="the entropy-coding stage (per-lane Huffman codes of the residuals, QCZ_FLAG_ENTROPY)")
    ap.add_argument("--cache", action="store_true",
                    help="grover24/qft24: run with the compressed block cache (a separate figure: each gate is "
                         "then a planning kernel plus two job launches, timed together)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the compressed gate-apply path here has no multi-GPU exchange; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1911_04034_amd import circuits as cc
    from paper_1911_04034_amd import qcz

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        nb = args.calibrate_copy << 20
        a = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": nb}), flush=True)
        return
    if args.workload in LARGE:
        large_config(args, torch, cc, qcz)
        return
    n, bl, level = 24, 16, 1
    do_grover = "grover" in args.workload
    do_qft = "qft" in args.workload
    total_iters = cc.grover_optimal_iterations(n)
    passes = args.warmup + args.steps
    g_iters = args.grover_iters or (-(-total_iters // passes))
    flags = qcz.FLAG_GRAPH if args.no_timing else qcz.FLAG_TIMING
    if args.cache:
        flags |= qcz.FLAG_CACHE
    if args.fuse:
        flags |= qcz.FLAG_FUSE
    if args.entropy:
        flags |= qcz.FLAG_ENTROPY
    stream = torch.cuda.Stream()

    # --- inputs resident in HBM before timing -------------------------------
    grover = qft_states = None
    w = cc.grover_marked(n, 2)
    it = cc.grover_iteration(n, w)
    if do_grover:
        grover = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=level, pool_bytes=8 << 30, flags=flags,
                           batch=len(it), grid=args.grid, stream=stream, chunk_waves=args.chunk_waves)
        grover.apply(cc.grover_prefix(n))
    x_in = cc.qft_input(n, 2)
    qft_gates = cc.qft(n, x_in)
    if do_qft:
        qft_states = [qcz.State(n, bl, mode=qcz.MODE_FIXED, level=level, pool_bytes=4 << 30, flags=flags,
                                batch=256, grid=args.grid, stream=stream, chunk_waves=args.chunk_waves)
                      for _ in range(passes)]
    log("inputs ready: grover=%s qft=%s passes=%d grover_iters/step=%d" % (do_grover, do_qft, passes, g_iters))

    iters_done = 0
    min_ratio = float("inf")

    def one_pass(p):
        nonlocal iters_done, min_ratio
        if do_qft:
            qft_states[p].apply(qft_gates)
        if do_grover:
            k = min(g_iters, total_iters - iters_done) if total_iters > iters_done else g_iters
            for _ in range(k):
                grover.apply(it)
            iters_done += k

    def all_states():
        return ([grover] if grover else []) + (qft_states or [])

    for p in range(args.warmup):
        one_pass(p)
        log("warmup pass %d done" % p)
    for s in all_states():
        s.reset_stats()
    torch.cuda.synchronize()
    stream.synchronize()
    t0 = time.perf_counter()
    for p in range(args.warmup, passes):
        one_pass(p)
        log("timed pass %d done" % (p - args.warmup))
    stream.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0

    # --- results ---------------------------------------------------------
    stats = [s.stats() for s in all_states()]
    amps = sum(x["amps_touched"] for x in stats)
    launches = sum(x["gate_launches"] for x in stats)
    gates_total = sum(x["gate_launches"] + x["permute_launches"] for x in stats)
    rd = sum(x["bytes_read"] for x in stats)
    wr = sum(x["bytes_written"] for x in stats)
    tb = sum(x["table_bytes"] for x in stats)
    timed = sum(x["timed_launches"] for x in stats)
    kms = sum(x["gate_kernel_ms"] for x in stats)
    value = amps / wall / 1e9
    stops = sum(x["stops"] for x in stats)
    compactions = sum(s.footprint()["compactions"] for s in all_states())

    out_extra = {}
    fids = []
    if grover:
        fp = grover.footprint()
        f_raw, nrm, aw = grover_fidelity(grover, n, w, iters_done)
        fids.append(f_raw / nrm if nrm > 0 else 0.0)
        min_ratio = min(min_ratio, fp["raw_bytes"] / (fp["max_compressed"] + fp["table_bytes"]))
        out_extra["grover24"] = {"iterations": iters_done, "marked_probability": aw ** 2, "fidelity_raw": f_raw,
                                 "fidelity_norm": f_raw / nrm, "fidelity_lower_bound": fp["fidelity_lower_bound"],
                                 "ratio_final": fp["ratio"],
                                 "ratio_min": fp["raw_bytes"] / (fp["max_compressed"] + fp["table_bytes"])}
    if qft_states:
        s = qft_states[-1]
        fp = s.footprint()
        f_raw, nrm = qft_fidelity(s, n, x_in)
        fids.append(f_raw / nrm)
        r_min = fp["raw_bytes"] / (fp["max_compressed"] + fp["table_bytes"])
        min_ratio = min(min_ratio, r_min)
        out_extra["qft24"] = {"gates": len(qft_gates), "fidelity_raw": f_raw, "fidelity_norm": f_raw / nrm,
                              "fidelity_lower_bound": fp["fidelity_lower_bound"], "ratio_final": fp["ratio"],
                              "ratio_min": r_min}

    roofline = None
    traffic = None
    valu_busy = None
    if args.workload == "grover24+qft24" and not args.cache and not args.fuse:
        from paper_1911_04034_amd import profile_summary as ps
        t_bytes, t_hash = ps.read_traffic(os.path.join(ROOT, "profiles", "traffic_fused_kernel_grover24_qft24.txt"))
        if t_bytes is not None and t_hash == ps.kernel_hash():
            traffic = round(t_bytes, 1)
        # what bounds the kernel: SQ counters of the same source (VALU issue per SIMD)
        busy, b_hash = ps.read_valu_busy(os.path.join(ROOT, "profiles", "counters_fused_kernel_qft24_grover24.txt"))
        if busy and b_hash == ps.kernel_hash():
            valu_busy = busy
    if timed > 0:
        avg_ms = kms / timed
        bytes_per_launch = (rd + wr + tb) / timed   # per timed kernel (a fused run is one kernel)
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
                    "kernel": ("block cache: plan + leader job launch + follower copy kernel + remaining followers, per gate"
                               if args.cache else "job_kernel<16, ARENA, ARENA, gate> (fused decode-gate-encode)"),
                    "avg_launch_us": round(avg_ms * 1e3, 3), "algorithmic_bytes_per_launch": round(bytes_per_launch, 1),
                    "launches": timed, "valu_busy_per_simd": valu_busy}

    # The default run also reports the same workload with gate-layer fusion
    # (same bytes and fidelities; a separate figure, the headline stays gate
    # by gate).  It runs in a child process after this one's states are freed;
    # profiling commands pass --no-cpu-baseline and skip it.
    fused = None
    if (not args.no_cpu_baseline and args.workload == "grover24+qft24" and not (args.fuse or args.cache)
            and not args.no_timing):
        grover = qft_states = None
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        log("fused-run figure: child process")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--fuse", "--no-cpu-baseline",
                            "--steps", str(args.steps), "--warmup", str(args.warmup)],
                           stdout=subprocess.PIPE, text=True, timeout=900)
        lines = [x for x in r.stdout.splitlines() if x.startswith("{")]
        if r.returncode == 0 and lines:
            f = json.loads(lines[-1])
            fused = {"value": f["value"], "unit": "GAmp/s", "ms_per_step": f["ms_per_step"],
                     "fused_kernel_gamp_s": f["fused_kernel_gamp_s"], "kernels": f["roofline"]["launches"],
                     "avg_kernel_us": f["roofline"]["avg_launch_us"], "fidelity_min": f["fidelity_min"],
                     "command": "bench.py --fuse --steps %d --warmup %d" % (args.steps, args.warmup)}
        else:
            log("fused-run figure failed (status %d)" % r.returncode)

    cpu = None
    if not args.no_cpu_baseline:
        # dense chunks: the QFT state at the end of the timed region, with the circuit's last 40 gates
        qs = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=level, pool_bytes=4 << 30,
                       flags=qcz.FLAG_ENTROPY if args.entropy else 0)
        qs.apply(qft_gates)
        cpu = cpu_baseline(qs, qft_gates[-40:], level, args.cpu_seconds, args.entropy,
                           "24-qubit QFT state (bound 1e-5) and the QFT's last 40 gates")
        qs.close()

    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "GAmp/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "qubits": n, "block_amplitudes": 1 << bl, "bound": 1e-5,
                   "grover_iterations_total": iters_done, "gates_per_step": gates_total / max(1, args.steps),
                   "parallelism": "single GPU"},
        "compression_ratio_min": round(min_ratio, 3),
        "fidelity_min": round(min(fids), 6) if fids else None,
        "logical_gamp_s": round(gates_total * (1 << n) / wall / 1e9, 3),
        "fused_kernel_gamp_s": round(amps / (kms * 1e-3) / 1e9, 3) if kms > 0 else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "device_stops": stops,
        "compactions": compactions,
        "workloads": out_extra,
    }
    if fused is not None:
        line["fused_runs"] = fused
    if args.fuse:
        line["config"]["fused_runs"] = True
        line["roofline"]["kernel"] = "job_kernel fused runs of in-chunk gates + per-gate fused kernels"
    if args.cache:
        ch = sum(x["cache_hits"] for x in stats)
        line["config"]["block_cache"] = True
        line["block_cache"] = {"gates": sum(x["cache_gates"] for x in stats), "chunks_copied": ch,
                               "chunks_reencoded": sum(x["chunks_reencoded"] for x in stats),
                               "on_at_end": [x["cache_on"] for x in stats]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
