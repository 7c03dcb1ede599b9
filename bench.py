#!/usr/bin/env python3
"""Decoded Mbit/s of syndrome BP on MET-LDPC codes on one MI355X.

Default workload (``--workload mix``): three MET codes with N = 10^6 -- rates
0.1, 0.05 and 0.02 -- with 64 frames each at SNR 0.157 / 0.0757 / 0.0296 and
iteration budgets 100 / 150 / 200 (per-frame early exit).  A step decodes all
three batches: flooding sum-product BP of the paper's Methods (Steps 2-5) with
every part of the hot path (input layout, check and variable updates, syndrome
tests, outputs) on the GPU.  ``value`` is the batched form (all jobs in one
persistent launch captured in a HIP graph); the plain form (one decode call
per job, run one after the other) is timed on the same inputs and reported
beside it, with each job's FER for both (they decode identically).

``--workload single`` times the plain decoder on one code (default rate 0.1,
N = 10^6, 64 frames, SNR 0.157, 100 iterations).

    python bench.py [--steps K] [--warmup W] [--workload mix|single] ...

Prints one JSON line.  Speed counts N decoded bits per frame, as the paper's
Table 1 does (speed = N / (iterations x per-codeword latency)).  Inputs are
resident in HBM before the timed region.

The roofline object reports the kernel that moves most of the bytes (the
persistent kernel for the mix, the largest check class for a single code):
algorithmic bytes per launch (unique bytes it must read or write, see
``class_bytes_per_frame`` / ``variable_bytes_per_frame``) over its average
duration, measured with HIP events bracketing each launch on its stream.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from met_inputs import BJ_SNR, ITER_BUDGET, PROFILES, WATERFALL_SNR, make_frames  # noqa: E402

METRIC = "decoded Mbit/s at N=1e6, R=0.1/0.05/0.02 (batched vs plain, equal FER); % HBM peak"
HBM_PEAK_GBS = 8000.0
CODE_SEED = {"r0.1": 101, "r0.05": 102, "r0.02": 103}
FRAME_SEED = 5000
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
MIX = ("r0.1", "r0.05", "r0.02")
KERNEL_SOURCES = ("met_gpu.h", "met_decode.hip", "met_batched.hip", "met_code.cpp")  # kernels and the layout they read


def class_bytes_per_frame(cls: dict, W: int, first: bool = False, test: bool = True, cb: int = 4) -> float:
    """Unique bytes one check-kernel launch over a class of checks moves per
    frame and iteration (n checks of nm message and nl leaf edges each):

    read  c2v (4 B per message edge; not on iteration 1), the posteriors P of
          the distinct message VNs the class reaches (4 B each, gathered), leaf
          phi(L) (4 B per leaf edge), the syndrome (1 bit per check), previous
          leaf decisions (1 bit per leaf edge, early-exit test only) and the
          edge -> VN index (4 B per message edge, shared by the W frames);
    write c2v (4 B per message edge) and leaf decisions (1 bit per leaf edge).
    """
    n, nm, nl = cls["n_checks"], cls["n_msg"], cls["n_leaf"]
    # (cb: bytes of a stored message: 4, or 2 / 1 with half / 8-bit storage)
    b = (0 if first else cb * nm * n) + cb * nm * n + 4 * cls["n_msg_vn_touched"] + 4 * nl * n
    b += n / 8 + nl * n / 8 + 4 * nm * n / W
    if test:
        b += nl * n / 8
    return b


def check_bytes_per_frame(classes: list, W: int, first: bool = False, test: bool = True) -> float:
    """Sum over the check classes (all check kernels of one iteration)."""
    return sum(class_bytes_per_frame(c, W, first, test) for c in classes if c["n_msg"] >= 0)


def variable_bytes_per_frame(st: dict, W: int, cb: int = 4) -> float:
    """read c2v (gathered, 4 B per message edge) and L (4 B per message VN),
    the VN -> edge lists (shared by W frames); write P (4 B per message VN)."""
    e12, n2 = st["n_msg_edges"], st["n_msg_vn"]
    return cb * e12 + 8 * n2 + (4 * e12 + 4 * n2) / W


def materialised_bytes_per_frame(code) -> float:
    """The 16-byte-per-edge model of flooding BP with both message arrays
    stored (each type-1/2 message written once and read once per phase):
    16 E12 + 4 E3 + 4 N2 + E12 / 8 + (M + N2 + M2) / 8 + 8 E12 / 64 bytes per
    frame and iteration (M2: checks with a degree-1 neighbour)."""
    st = code.info()
    e12, e3, n2, m = st["n_msg_edges"], st["n_leaf_edges"], st["n_msg_vn"], st["M"]
    m2 = sum(c["n_checks"] for c in code.classes() if c["n_leaf"] > 0)
    return 16 * e12 + 4 * e3 + 4 * n2 + e12 / 8 + (m + n2 + m2) / 8 + 8 * e12 / 64


def wilson(k: int, n: int, z: float = 1.96):
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


# ----------------------------------------------------------------------------
# CPU baseline: the FP64 oracle as it stands, one frame per host core.

_CPU = {}


def _cpu_worker(task):
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import bp
    from oracle import code as oc

    prof, f = task
    code = _CPU["codes"][prof]
    bits, llr = make_frames(code.n, 1, BJ_SNR[prof] if _CPU["snr"] is None else _CPU["snr"], FRAME_SEED,
                            first_frame=f)
    syn = oc.syndrome(code, bits)
    t0 = time.perf_counter()
    bp.decode(code, llr, syn, _CPU["iters"], early_exit=False)
    return prof, time.perf_counter() - t0


def cpu_baseline(jobs, n: int, snr, sample_iters: int, max_workers: int) -> dict:
    """jobs: [(profile, frames, budget)].  Each host core decodes one frame of
    one job's code for sample_iters iterations (fixed mode); per-iteration times
    are extrapolated to the whole workload (every frame its full budget, as at
    these SNRs) spread over the cores."""
    import multiprocessing as mp

    from oracle import code as oc

    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(cores, max_workers))
    _CPU["codes"] = {p: oc.build(PROFILES[p], n, CODE_SEED[p]) for p, _, _ in jobs}
    _CPU["snr"] = snr
    _CPU["iters"] = sample_iters
    tasks = [(jobs[k % len(jobs)][0], k) for k in range(workers)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        durs = pool.map(_cpu_worker, tasks)
    wall = time.perf_counter() - t0
    per_iter = {}
    for prof, d in durs:
        per_iter.setdefault(prof, []).append(d / sample_iters)
    cpu_seconds = sum(b * budget * max(per_iter[p]) for p, b, budget in jobs)
    bits = sum(b for _, b, _ in jobs) * n
    mbit = bits / (cpu_seconds / workers) / 1e6
    return {
        "value": round(mbit, 4),
        "unit": "Mbit/s",
        "cores": workers,
        "kind": "oracle",
        "extrapolated": True,  # from the timed sample below to the whole workload, not a timed full decode
        "sample": "%d frames (one per core: %s), %d iterations each in fixed mode; the slowest frame's time per "
        "iteration of each code, times frames x budget of the workload, spread over %d cores (wall %.1f s)"
        % (workers, ", ".join("%d of %s" % (sum(1 for t in tasks if t[0] == p), p) for p, _, _ in jobs),
           sample_iters, workers, wall),
    }


# ----------------------------------------------------------------------------


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1711_01783_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload_key: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when it is missing or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(kernel + " | " + workload_key)
    if not e or e.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def active_frames(iters, conv, max_iter: int, early: bool):
    """Frames taking part in check update l and in variable update l, l = 1..max_iter:
    a frame that converged at iteration r runs check updates 1..r+1 (update r+1
    carries its test) and variable updates 1..r."""
    import numpy as np

    if not early:
        full = np.full(max_iter, len(iters))
        return full, full
    last_c = np.where(conv == 1, np.minimum(iters + 1, max_iter), max_iter)
    last_v = np.where(conv == 1, iters, max_iter)
    ls = np.arange(1, max_iter + 1)
    return (last_c[None, :] >= ls[:, None]).sum(1), (last_v[None, :] >= ls[:, None]).sum(1)


def job_bytes(code, iters, conv, max_iter: int, early: bool, W: int = 64, cb: int = 4):
    """Algorithmic bytes of one decode of a job: (check updates by class name,
    variable updates)."""
    classes = [c for c in code.classes() if c["n_msg"] >= 0]
    st = code.info()
    fc, fv = active_frames(iters, conv, max_iter, early)
    per_class = {}
    for c in classes:
        name = "k_check<%d,%d>" % (c["n_msg"], c["n_leaf"])
        b = 0.0
        for l in range(1, max_iter + 1):
            b += fc[l - 1] * class_bytes_per_frame(c, W, first=(l == 1), test=(early and l >= 2), cb=cb)
        per_class[name] = per_class.get(name, 0.0) + b
    var = float(fv.sum()) * variable_bytes_per_frame(st, W, cb)
    return per_class, var


def roofline(kernel: str, bytes_total: float, launches: int, total_ms: float, traffic) -> dict:
    avg_ms = total_ms / max(1, launches)
    per_launch = bytes_total / max(1, launches)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return {
        "kernel": kernel,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "algorithmic_bytes_per_launch": round(per_launch),
        "avg_launch_us": round(avg_ms * 1e3, 2),
    }


def timed(fn, steps: int, warmup: int):
    """Runs fn warmup times, then `steps` times between two events with the
    decoder's per-launch timing on; returns (elapsed ms, kernel times, last out)."""
    import torch

    import paper_1711_01783_amd as met

    out = None
    for _ in range(warmup):
        out = fn()
    torch.cuda.synchronize()
    met.timing_enable(True)
    met.timing_collect()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        out = fn()
    stop.record()
    torch.cuda.synchronize()
    ktimes = met.timing_collect()
    met.timing_enable(False)
    return start.elapsed_time(stop), ktimes, out


def timed_plain(fn, steps: int) -> float:
    import torch

    fn()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop)


def fer_summary(out, bits):
    import numpy as np

    dec = out.bits.cpu().numpy()
    conv = out.converged.cpu().numpy()
    iters = out.iterations.cpu().numpy()
    err = np.any(dec != bits, axis=1)
    k, b = int(err.sum()), len(err)
    lo, hi = wilson(k, b)
    return {"fer": round(k / b, 4), "fer_ci95": [round(lo, 4), round(hi, 4)], "converged": int(conv.sum()),
            "undetected_errors": int((err & (conv == 1)).sum()), "mean_iterations": round(float(iters.mean()), 2)}


def job_snr(args, prof: str) -> float:
    """The SNR of a job: --snr if given, else the waterfall point (--waterfall)
    or the workload's operating point."""
    if args.snr is not None:
        return args.snr
    return WATERFALL_SNR[prof] if args.waterfall else BJ_SNR[prof]


def copy_bandwidth() -> float:
    """Measured device-to-device copy rate in GB/s (bytes read + written)."""
    import torch

    n = 1 << 28  # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    ms = timed_plain(lambda: b.copy_(a), 5)
    del a, b
    return 2 * 4 * n * 5 / (ms * 1e-3) / 1e9


def end_to_end(jobs, dec, steps: int) -> dict:
    """One batched step with the inputs in pinned host memory: host-to-device
    copies of LLRs and syndromes, the decode, device-to-host copies of bits,
    iteration counts and flags (the paper's timing includes its copies)."""
    import torch

    h_in = [(j.llr.cpu().pin_memory(), j.syn.cpu().pin_memory()) for j in jobs]
    h_out = [(torch.empty(tuple(j.llr.shape), dtype=torch.uint8).pin_memory(),
              torch.empty(int(j.llr.shape[0]), dtype=torch.int32).pin_memory(),
              torch.empty(int(j.llr.shape[0]), dtype=torch.uint8).pin_memory()) for j in jobs]

    def step():
        for j, (hl, hs) in zip(jobs, h_in):
            j.llr.copy_(hl, non_blocking=True)
            j.syn.copy_(hs, non_blocking=True)
        outs = dec(jobs)
        for o, (hb, hi, hc) in zip(outs, h_out):
            hb.copy_(o.bits, non_blocking=True)
            hi.copy_(o.iterations, non_blocking=True)
            hc.copy_(o.converged, non_blocking=True)

    ms = timed_plain(step, steps) / steps
    bits = sum(int(j.llr.shape[0]) * int(j.llr.shape[1]) for j in jobs)
    moved = sum(hl.numel() * 4 + hs.numel() + hb.numel() + 5 * hi.numel()
                for (hl, hs), (hb, hi, _) in zip(h_in, h_out))
    return {"ms_per_step": round(ms, 3), "value": round(bits / (ms * 1e-3) / 1e6, 3),
            "host_device_bytes_per_step": moved}


def run_mix(args, cpu) -> dict:
    import numpy as np
    import torch

    import paper_1711_01783_amd as met

    dev = torch.device("cuda:0")
    n, B = args.n, args.frames
    jobs, truth = [], []
    for prof in MIX:
        code = met.Code.build(PROFILES[prof], n, CODE_SEED[prof])
        snr = job_snr(args, prof)
        bits, llr = make_frames(n, B, snr, FRAME_SEED)
        syn = met.syndrome(code, torch.from_numpy(bits).to(dev))
        budget = args.max_iter if args.max_iter is not None else ITER_BUDGET[prof]
        jobs.append(met.Job(code, torch.from_numpy(llr).to(dev), syn, budget, args.fixed_iters))
        truth.append(bits)
    wss = [torch.empty(met.workspace_bytes(j.code, B, j.fixed_iters) + 256, dtype=torch.uint8, device=dev)
           for j in jobs]
    torch.cuda.synchronize()
    early = not args.fixed_iters

    def plain():
        return [met.decode(j.code, j.llr, j.syn, j.max_iter, fixed_iters=j.fixed_iters, workspace=w,
                           check_steps_per_wave=args.check_steps, variable_chunk=args.vn_chunk)
                for j, w in zip(jobs, wss)]

    if args.plain_only:  # profiling runs of the plain form's launches alone
        for _ in range(args.warmup + args.steps):
            plain()
        torch.cuda.synchronize()
        return {"plain_only": True, "steps": args.steps, "warmup": args.warmup}

    # plain form: per-launch timing (for its roofline) adds two events to each of
    # its ~2000 launches per step, so its throughput is taken from a pass without
    if args.batched_only:  # profiling runs: the plain form's kernels would mix with the batched form's
        p_ms_ev, p_kt, p_out, p_ms = float("nan"), {}, None, float("nan")
    else:
        p_ms_ev, p_kt, p_out = timed(plain, args.steps, args.warmup)
        p_ms = timed_plain(plain, args.steps)
    del wss
    dec = met.BatchedDecoder(check_steps_per_wave=args.check_steps, blocks_per_cu=args.blocks_per_cu,
                             phase_launches=args.schedule in ("phase", "kinds", "jobs", "serial"),
                             stagger=not args.no_stagger,
                             streams=args.schedule if args.schedule in ("kinds", "jobs", "serial") else "one")
    shape = None
    if args.schedule == "auto" and not args.no_autotune and not args.check_steps and not args.blocks_per_cu:
        shape = dec.autotune(jobs)  # outside the timed region
    b_ms, b_kt, b_out = timed(lambda: dec(jobs), args.steps, args.warmup)
    expired = dec.barrier_expired()
    # per-launch timing runs the launch sequence outside a graph; the same steps
    # replayed from the captured graph, without events:
    g_ms = timed_plain(lambda: dec(jobs), args.steps)
    expired = expired or dec.barrier_expired()
    same = None if p_out is None else all(
        np.array_equal(a.bits.cpu().numpy(), b.bits.cpu().numpy())
        and np.array_equal(a.iterations.cpu().numpy(), b.iterations.cpu().numpy())
        and np.array_equal(a.converged.cpu().numpy(), b.converged.cpu().numpy())
        for a, b in zip(p_out, b_out))
    e2e = end_to_end(jobs, dec, min(args.steps, 3))
    copy_gbps = copy_bandwidth()

    total_bits = B * n * len(jobs) * args.steps
    # value: the graph replay without per-launch events (with one launch per
    # phase the events would bracket each of ~400 launches)
    b_val = total_bits / (g_ms * 1e-3) / 1e6
    p_val = total_bits / (p_ms * 1e-3) / 1e6
    sched = (shape or {}).get("schedule", "phase launches" if dec.tuning.batch_flags & 4 else "persistent")
    bk = "k_phase" if sched == "phase launches" else "k_persistent"
    wl = "batched mix: rates 0.1/0.05/0.02 N=%d B=%d each, budgets %s, %s" % (
        n, B, "/".join(str(j.max_iter) for j in jobs), "fixed" if args.fixed_iters else "early-exit")

    # algorithmic bytes of one step, per kernel, from each job's outcome
    check_bytes, var_bytes = {}, 0.0
    per_job = []
    for prof, j, o, bits in zip(MIX, jobs, b_out, truth):
        cls, var = job_bytes(j.code, o.iterations.cpu().numpy(), o.converged.cpu().numpy(), j.max_iter, early)
        for k, v in cls.items():
            check_bytes[k] = check_bytes.get(k, 0.0) + v
        var_bytes += var
        d = {"profile": prof, "snr": float(job_snr(args, prof)), "max_iter": j.max_iter}
        d.update(fer_summary(o, bits))
        d["plain_fer"] = None if p_out is None else fer_summary(p_out[len(per_job)], bits)["fer"]
        per_job.append(d)
    step_bytes = sum(check_bytes.values()) + var_bytes
    # the phase launches are timed per kind of tile (k_phase:...); the dominant
    # one is the (3,1) / (2,1) check launch, priced with those classes' bytes,
    # unless mixed launches (staggered phases on one stream) also hold such
    # tiles: then all phase launches are pooled with the whole step's bytes
    narrow = "k_phase:checks(3,1)(2,1)"
    roof_kt, roof_steps, roof_sched = b_kt, args.steps, None
    if dec.tuning.batch_flags & (8 | 16) and narrow in b_kt:
        # launches on parallel streams overlap, so their per-launch durations
        # do not price one launch: the dominant kernel is timed in a pass of
        # the same shape with the jobs' chains in turn on one stream
        rdec = met.BatchedDecoder()
        rdec.tuning = type(dec.tuning).from_buffer_copy(dec.tuning)
        rdec.tuning.batch_flags = (rdec.tuning.batch_flags & ~(8 | 16 | 32)) | 32
        rdec.workspace, rdec._ws_ptr = dec.workspace, dec._ws_ptr
        roof_steps = min(args.steps, 3)
        _ms, roof_kt, _o = timed(lambda: rdec(jobs), roof_steps, 1)
        roof_sched = "jobs in turn on one stream (same shape as the timed schedule, whose launches overlap)"
        del rdec
    if bk == "k_phase" and narrow in roof_kt and "k_phase:mixed" not in roof_kt:
        bk = narrow
        kl, kms = roof_kt[narrow]
        roof_bytes = check_bytes.get("k_check<3,1>", 0.0) + check_bytes.get("k_check<2,1>", 0.0)
        pooled = False
    else:
        kl = sum(v[0] for k, v in b_kt.items() if k.split(":")[0] == bk)
        kms = sum(v[1] for k, v in b_kt.items() if k.split(":")[0] == bk)
        roof_bytes = step_bytes
        pooled = True
    roof = roofline(bk, roof_bytes * (args.steps if pooled else roof_steps), kl, kms, measured_traffic(bk, wl))
    if roof_sched and not pooled:
        roof["timed_schedule"] = roof_sched
    # the whole step's algorithmic bytes over the graph replay's step time:
    # the rate of the schedule as a whole (with launches on parallel streams
    # the per-launch durations above overlap)
    roof["step_achieved"] = round(step_bytes / (g_ms / args.steps * 1e-3) / 1e9, 1)
    roof["step_frac"] = round(roof["step_achieved"] / HBM_PEAK_GBS, 4)
    # the same launches priced by the 16-byte-per-edge model (both message
    # arrays stored), for comparison; `frac` above uses the posterior form the
    # kernels implement (c2v stored, v2c re-formed from the posteriors)
    mat = sum(materialised_bytes_per_frame(j.code) * float(o.iterations.cpu().numpy().astype(np.float64).sum())
              for j, o in zip(jobs, b_out))
    roof["model"] = ("posterior form: c2v read and written per message edge, posteriors gathered once per "
                     "distinct row, leaf inputs, syndrome and decision bits (class_bytes_per_frame, "
                     "variable_bytes_per_frame)")
    if pooled:  # launches that carry the whole step: per launch
        mat_launch = mat * args.steps / max(1, kl)
        roof["materialised_16B_model"] = {
            "bytes_per_launch": round(mat_launch),
            "frac": round(mat_launch / (kms * 1e-3 / max(1, kl)) / 1e9 / HBM_PEAK_GBS, 4) if kms > 0 else None}
    else:  # the model prices the whole iteration: against the step time
        roof["materialised_16B_model"] = {
            "bytes_per_step": round(mat),
            "step_frac": round(mat / (g_ms / args.steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    pl, pms = p_kt.get("k_check<3,1>", (0, 0.0))
    plain_roof = roofline("k_check<3,1>", check_bytes.get("k_check<3,1>", 0.0) * args.steps, pl, pms,
                          measured_traffic("k_check<3,1>", wl))
    return {
        "value": round(b_val, 3),
        "ms_per_step": round(g_ms / args.steps, 3),
        "config": {
            "workload": "batched launch (one HIP graph, %s) of three jobs: MET codes of rate 0.1, 0.05 and 0.02 "
            "at N=%d, %d frames each, SNR %s, max %s iterations, %s; value = batched form"
            % (sched, n, B, "/".join("%g" % d["snr"] for d in per_job), "/".join(str(j.max_iter) for j in jobs),
               "fixed iterations" if args.fixed_iters else "per-frame early exit"),
            "N": n, "frames_per_job": B, "profiles": list(MIX), "code_seeds": [CODE_SEED[p] for p in MIX],
            "frame_seed": FRAME_SEED, "mode": "batched", "schedule": sched,
            "stagger": not (dec.tuning.batch_flags & 1),
            "streams": ("kinds" if dec.tuning.batch_flags & 8 else "jobs" if dec.tuning.batch_flags & 16
                        else "serial" if dec.tuning.batch_flags & 32 else "one"),
            "interleave": int((shape or {}).get("interleave") or 64),
        },
        "roofline": roof,
        "plain": {"value": round(p_val, 3), "ms_per_step": round(p_ms / args.steps, 3),
                  "ms_per_step_with_launch_timing": round(p_ms_ev / args.steps, 3),
                  "roofline": plain_roof,
                  "kernels_us": {k: {"launches": v[0], "avg_us": round(1e3 * v[1] / max(1, v[0]), 2)}
                                 for k, v in p_kt.items()}},
        "batched_over_plain": round(b_val / p_val, 4),
        "end_to_end_with_host_copies": e2e,
        "measured_copy_GBps": round(copy_gbps, 1),
        "ms_per_step_with_launch_timing": round(b_ms / args.steps, 3),
        "frac_of_measured_copy": {bk: round(roof["achieved"] / copy_gbps, 4),
                                  "k_check<3,1>": round(plain_roof["achieved"] / copy_gbps, 4)},
        "graph_replay": {"value": round(total_bits / (g_ms * 1e-3) / 1e6, 3),
                         "ms_per_step": round(g_ms / args.steps, 3)},
        "identical_outputs": bool(same),
        "autotuned_shape": shape,
        "barrier_expired": bool(expired),
        "jobs": per_job,
        "bytes_per_step": {"check": check_bytes, "variable": var_bytes},
        "kernels_us": {k: {"launches": v[0], "avg_us": round(1e3 * v[1] / max(1, v[0]), 2)} for k, v in b_kt.items()},
    }


def run_single(args, cpu) -> dict:
    import numpy as np
    import torch

    import paper_1711_01783_amd as met

    prof = args.profile
    snr = job_snr(args, prof)
    max_iter = args.max_iter if args.max_iter is not None else ITER_BUDGET[prof]
    n, B = args.n, args.frames
    dev = torch.device("cuda:0")
    code = met.Code.build(PROFILES[prof], n, CODE_SEED[prof])
    bits, llr = make_frames(n, B, snr, FRAME_SEED)
    d_llr = torch.from_numpy(llr).to(dev)
    d_syn = met.syndrome(code, torch.from_numpy(bits).to(dev))
    half = args.c2v_fp16
    q8 = args.c2v_q8 or args.check_lut
    lut = args.check_lut
    ws = torch.empty(met.workspace_bytes(code, B, args.fixed_iters, c2v_fp16=half, c2v_q8=q8) + 256,
                     dtype=torch.uint8,
                     device=dev)
    torch.cuda.synchronize()

    def step():
        return met.decode(code, d_llr, d_syn, max_iter, fixed_iters=args.fixed_iters, workspace=ws,
                          check_steps_per_wave=args.check_steps, variable_chunk=args.vn_chunk, c2v_fp16=half,
                          c2v_q8=q8, check_lut=lut)

    ms_ev, kt, out = timed(step, args.steps, args.warmup)
    # throughput from a pass without the per-launch events (they cost the
    # launch-bound small cases much of their time)
    ms = timed_plain(step, args.steps)
    value = B * n * args.steps / (ms * 1e-3) / 1e6
    W = 1 if B <= 1 else 4 if B <= 4 else 16 if B <= 16 else 32 if B <= 32 else 64
    early = not args.fixed_iters
    cls, var = job_bytes(code, out.iterations.cpu().numpy(), out.converged.cpu().numpy(), max_iter, early, W,
                         cb=2 if half else 1 if q8 else 4)
    classes = [c for c in code.classes() if c["n_msg"] >= 0]
    dom = max(classes, key=lambda c: c["n_checks"] * (c["n_msg"] + c["n_leaf"]))
    kname = "k_check<%d,%d>" % (dom["n_msg"], dom["n_leaf"])
    wl = "%s N=%d B=%d snr=%g max_iter=%d %s" % (prof, n, B, snr, max_iter, "early-exit" if early else "fixed")
    kl, kms = kt.get(kname, (0, 0.0))
    rec = {
        "value": round(value, 3),
        "ms_per_step": round(ms / args.steps, 3),
        "ms_per_step_with_launch_timing": round(ms_ev / args.steps, 3),
        "config": {
            "workload": "plain BP (one decode call per batch), rate %s MET profile, N=%d, %d frames, SNR %g, "
            "max %d iterations, %s" % (PROFILES[prof].rate, n, B, snr, max_iter,
                                     "per-frame early exit" if early else "fixed iterations"),
            "profile": prof, "N": n, "frames": B, "snr": snr, "max_iter": max_iter, "mode": "plain",
            "interleave": W, "code_seed": CODE_SEED[prof], "frame_seed": FRAME_SEED,
        },
        "roofline": roofline(kname, cls[kname] * args.steps, kl, kms, measured_traffic(kname, wl)),
        "kernels_us": {k: {"launches": v[0], "avg_us": round(1e3 * v[1] / max(1, v[0]), 2)} for k, v in kt.items()},
    }
    rec.update(fer_summary(out, bits))
    # per iteration of the slowest frame (small cases are launch-bound: this,
    # not the roofline, is their figure)
    rec["us_per_iteration"] = round(1e3 * ms / args.steps / max(1, int(out.iterations.max().item())), 2)
    if half or q8:  # the batched form stores float messages only
        rec["config"]["c2v_storage"] = "fp16" if half else "8-bit log-magnitude codes"
        if lut:
            rec["config"]["check_update"] = "table-driven (phi and output codes read from tables on the 8-bit grid)"
        return rec
    # the same job through the batched persistent launch (one graph replay per
    # decode), on the same inputs; outputs must be identical
    del ws
    job = [met.Job(code, d_llr, d_syn, max_iter, args.fixed_iters)]
    dec = met.BatchedDecoder()
    shape = None if args.no_autotune else dec.autotune(job)  # outside the timed region
    bout = dec(job)[0]
    b_ms = timed_plain(lambda: dec(job), args.steps)
    torch.cuda.synchronize()
    rec["batched"] = {
        "value": round(B * n * args.steps / (b_ms * 1e-3) / 1e6, 3),
        "ms_per_step": round(b_ms / args.steps, 3),
        "us_per_iteration": round(1e3 * b_ms / args.steps / max(1, int(bout.iterations.max().item())), 2),
        "identical_outputs": bool(np.array_equal(bout.bits.cpu().numpy(), out.bits.cpu().numpy())
                                  and np.array_equal(bout.iterations.cpu().numpy(), out.iterations.cpu().numpy())),
        "wait_expired": bool(dec.barrier_expired()),
        "autotuned_shape": shape,
    }
    rec["batched_over_plain"] = round(rec["batched"]["value"] / rec["value"], 4)
    return rec


def run_deg1(args) -> dict:
    """Table 1 analog: the three codes at N = --n, --frames frames, their
    iteration budgets in fixed-iteration mode (the paper runs every codeword to
    its budget), decoded with degree-1 variable nodes kept out of the
    iterations (the default) and with them iterated (MET_NO_DEG1_SKIP)."""
    import numpy as np
    import torch

    import paper_1711_01783_amd as met

    n, B = args.n, args.frames
    dev = torch.device("cuda:0")
    per, tot_bits, tot_ms = {}, 0.0, {True: 0.0, False: 0.0}
    for prof in MIX:
        snr = args.snr if args.snr is not None else BJ_SNR[prof]
        L = args.max_iter if args.max_iter is not None else ITER_BUDGET[prof]
        code = met.Code.build(PROFILES[prof], n, CODE_SEED[prof])
        bits, llr = make_frames(n, B, snr, FRAME_SEED)
        d_llr = torch.from_numpy(llr).to(dev)
        d_syn = met.syndrome(code, torch.from_numpy(bits).to(dev))
        rec, outs = {}, {}
        for skip in (True, False):
            ws = torch.empty(met.workspace_bytes(code, B, True, False, skip) + 256, dtype=torch.uint8, device=dev)

            def step():
                return met.decode(code, d_llr, d_syn, L, fixed_iters=True, workspace=ws, deg1_skip=skip)

            outs[skip] = step()
            ms = timed_plain(step, args.steps) / args.steps
            tot_ms[skip] += ms
            rec["skip" if skip else "all_vns"] = {
                "ms_per_decode": round(ms, 3), "us_per_iteration": round(1e3 * ms / L, 1),
                "Mbit_s": round(B * n / (ms * 1e-3) / 1e6, 3)}
            del ws
        torch.cuda.synchronize()
        a, b = outs[True], outs[False]
        rec["speedup_from_skipping"] = round(rec["all_vns"]["ms_per_decode"] / rec["skip"]["ms_per_decode"], 4)
        rec["frames_with_equal_bits"] = int(np.all(a.bits.cpu().numpy() == b.bits.cpu().numpy(), axis=1).sum())
        rec["iterations"] = L
        per[prof] = rec
        tot_bits += B * n
    return {
        "metric": "decoded Mbit/s with degree-1 variable nodes skipped vs iterated (Table 1 analog)",
        "value": round(tot_bits / (tot_ms[True] * 1e-3) / 1e6, 3),
        "unit": "Mbit/s",
        "ms_per_step": round(tot_ms[True], 3),
        "all_vns_value": round(tot_bits / (tot_ms[False] * 1e-3) / 1e6, 3),
        "config": {"workload": "plain BP, rates 0.1/0.05/0.02 at N=%d, %d frames each, fixed budgets %s; "
                               "value = degree-1 nodes skipped (default), all_vns_value = iterated" % (
                                   n, B, "/".join(str(ITER_BUDGET[p]) for p in MIX)),
                   "N": n, "frames": B, "profiles": list(MIX)},
        "per_code": per,
        "paper_speedup_from_skipping": {"r0.1": round(30.39 / 27.54, 4), "r0.05": round(21.23 / 18.49, 4),
                                        "r0.02": round(16.41 / 14.00, 4)},
    }


def _wbp_setup(prof: str, n: int, B: int, snr: float, seed: int):
    import torch

    import paper_1711_01783_amd as met

    code = met.Code.build(PROFILES[prof], n, CODE_SEED[prof])
    bits, llr = make_frames(n, B, snr, seed)
    d_bits = torch.from_numpy(bits).to("cuda:0")
    syn = met.syndrome(code, d_bits)
    sgn = 1.0 - 2.0 * d_bits.float()
    return code, torch.from_numpy(llr).to("cuda:0"), syn, sgn


def wbp_rooflines(code, frames: int, ktimes: dict) -> dict:
    """Rooflines of the weighted check update and of the check adjoint from
    per-launch timings.  Algorithmic bytes per frame: the weighted check update
    moves what the plain one does (without the syndrome test) plus the leaf
    LLRs (4 B per leaf edge, for the weighted leaf decision); the adjoint of a
    class reads P and Pbar rows of the VNs it touches, c2v and Cbar and writes
    Cbar (4 B each per message edge) and reads the leaf inputs."""
    classes = [c for c in code.classes() if c["n_msg"] >= 0]
    fwd = sum(class_bytes_per_frame(c, 64, first=False, test=False) + 4 * c["n_leaf"] * c["n_checks"]
              for c in classes)
    adj = sum(12 * c["n_msg"] * c["n_checks"] + 4 * c["n_leaf"] * c["n_checks"] + 8 * c["n_msg_vn_touched"]
              for c in classes)
    out = {}
    lw, msw = ktimes.get("k_check_weighted", (0, 0.0))
    if lw:
        iters = lw / max(1, len(classes))
        out["k_check_weighted"] = roofline("k_check_weighted (all classes of one iteration)", fwd * frames * iters,
                                           int(iters), msw, None)
    la, msa = ktimes.get("k_check_adj", (0, 0.0))
    if la:
        out["k_check_adj"] = roofline("k_check_adj (all classes of one iteration)", adj * frames * la, la, msa, None)
    return out


def run_wbp_train(args) -> dict:
    """Weighted-BP training steps: forward (L unrolled iterations, states kept
    every k-th), BCE loss, hand-written adjoint, Adam update of the [T, L]
    scales.  Batches rotate over a few resident ones."""
    import torch

    from paper_1711_01783_amd import wbp

    prof, n, B = args.profile, args.n, args.frames
    L, k = args.iters, args.ckpt or 10  # the training configuration keeps every 10th state
    snr = args.snr if args.snr is not None else BJ_SNR[prof]
    batches = [_wbp_setup(prof, n, B, snr, FRAME_SEED + 1000 * r) for r in range(4)]
    code = batches[0][0]
    T = code.info()["n_edge_types"]
    w = torch.ones(T, L, device="cuda:0", requires_grad=True)
    opt = torch.optim.Adam([w], lr=args.lr)
    losses = []
    held = _wbp_setup(prof, n, B, snr, FRAME_SEED + 99991)  # not trained on

    def held_loss():
        with torch.no_grad():
            post, _, _, _ = wbp.forward(held[0], held[1], held[2], w.detach().contiguous(), k)
            return float(torch.nn.functional.softplus(-held[3] * post).mean())

    loss_before = held_loss()

    def step(r=[0]):
        _, llr, syn, sgn = batches[r[0] % len(batches)]
        r[0] += 1
        opt.zero_grad(set_to_none=True)
        post = wbp.weighted_bp(w, batches[0][0], llr, syn, k)
        loss = torch.nn.functional.softplus(-sgn * post).mean()
        loss.backward()
        opt.step()
        losses.append(loss.detach())
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ms = timed_plain(step, args.steps)
    _, ktimes, _ = timed(step, 1, 0)  # per-launch timing for the rooflines
    hist = [float(x) for x in losses]
    return {
        "metric": "weighted-BP training: decoded Mbit/s (forward + adjoint + update per step)",
        "value": round(B * n * args.steps / (ms * 1e-3) / 1e6, 3) if ms > 0 else None,
        "unit": "Mbit/s",
        "ms_per_step": round(ms / args.steps, 3),
        "config": {"workload": "weighted BP training, rate %s MET profile, N=%d, %d frames per step, %d unrolled "
                               "iterations, checkpoint every %d, SNR %g, Adam lr %g, scales initialised to 1"
                               % (PROFILES[prof].rate, n, B, L, k, snr, args.lr),
                   "profile": prof, "N": n, "frames": B, "iterations": L, "ckpt_every": k, "snr": snr},
        "roofline": wbp_rooflines(code, B, ktimes),
        "heldout_loss_before": round(loss_before, 6), "heldout_loss_after": round(held_loss(), 6),
        "train_loss_first_rotation": round(sum(hist[:4]) / 4, 6), "train_loss_last_rotation": round(sum(hist[-4:]) / 4, 6),
        "training_steps": len(hist),
        "workspace_bytes": wbp.workspace_bytes(code, B, L, k),
    }


def run_wbp_eval(args) -> dict:
    """Forward + adjoint at full size, a few training steps, then FER of the
    trained scales against plain BP (fixed iterations, same budget) on fresh
    frames."""
    import numpy as np
    import torch

    import paper_1711_01783_amd as met
    from paper_1711_01783_amd import wbp

    prof, n, B = args.profile, args.n, args.frames
    L = args.iters
    k = args.ckpt or wbp.default_checkpoint_interval(L)
    snr = args.snr if args.snr is not None else BJ_SNR[prof]
    code, llr, syn, sgn = _wbp_setup(prof, n, B, snr, FRAME_SEED)
    T = code.info()["n_edge_types"]
    w = torch.ones(T, L, device="cuda:0", requires_grad=True)
    opt = torch.optim.Adam([w], lr=args.lr)

    def step():
        opt.zero_grad(set_to_none=True)
        post = wbp.weighted_bp(w, code, llr, syn, k)
        loss = torch.nn.functional.softplus(-sgn * post).mean()
        loss.backward()
        opt.step()
        return loss

    for _ in range(args.warmup):
        step()
    ms = timed_plain(step, args.steps)
    _, ktimes, _ = timed(step, 1, 0)  # per-launch timing for the rooflines
    # FER on fresh frames: trained scales vs plain BP, same syndromes, L iterations
    wt = w.detach().contiguous()
    errs_w = errs_p = conv_w = conv_p = 0
    total = 0
    r = 0
    while total < args.eval_frames:
        b = min(B, args.eval_frames - total)
        bits, l2 = make_frames(n, b, snr, FRAME_SEED + 7777, first_frame=total)
        d_bits = torch.from_numpy(bits).to("cuda:0")
        s2 = met.syndrome(code, d_bits)
        d_llr = torch.from_numpy(l2).to("cuda:0")
        _, bw, cw, _ = wbp.forward(code, d_llr, s2, wt, k)
        po = met.decode(code, d_llr, s2, L, fixed_iters=True)
        errs_w += int((bw != d_bits).any(dim=1).sum())
        errs_p += int((po.bits != d_bits).any(dim=1).sum())
        conv_w += int(cw.sum())
        conv_p += int(po.converged.sum())
        total += b
        r += 1
    return {
        "metric": "weighted-BP forward + adjoint: decoded Mbit/s per training step",
        "value": round(B * n * args.steps / (ms * 1e-3) / 1e6, 3) if ms > 0 else None,
        "unit": "Mbit/s",
        "ms_per_step": round(ms / args.steps, 3),
        "config": {"workload": "weighted BP forward + adjoint + Adam update, rate %s MET profile, N=%d, %d frames, "
                               "%d unrolled iterations, checkpoint every %d, SNR %g; then FER of the trained scales vs "
                               "plain BP (%d fixed iterations) on %d fresh frames"
                               % (PROFILES[prof].rate, n, B, L, k, snr, L, total),
                   "profile": prof, "N": n, "frames": B, "iterations": L, "ckpt_every": k, "snr": snr},
        "workspace_bytes": wbp.workspace_bytes(code, B, L, k),
        "roofline": wbp_rooflines(code, B, ktimes),
        "eval_frames": total,
        "fer_weighted": round(errs_w / total, 4), "fer_weighted_ci95": [round(x, 4) for x in wilson(errs_w, total)],
        "fer_plain": round(errs_p / total, 4), "fer_plain_ci95": [round(x, 4) for x in wilson(errs_p, total)],
        "converged_weighted": conv_w, "converged_plain": conv_p,
        "training_steps": args.warmup + args.steps + 2,
    }


def run_mdr(args) -> dict:
    """Multidimensional-reconciliation front end: Bob's rotation coefficients
    (met_mdr_bob) and Alice's LLRs (met_mdr_alice) for `frames` frames of N
    Gaussian raw keys in blocks of d = 8.  Algorithmic bytes per element: Bob
    reads y (4 B) and a bit (1 B) and writes alpha (4 B) and |y| (4 / d B);
    Alice reads x and alpha (8 B) and |y| (4 / d B) and writes an LLR (4 B)."""
    import numpy as np
    import torch

    import paper_1711_01783_amd as met
    from met_inputs import gaussian_raw_keys

    n, B, d = args.n, args.frames, 8
    snr = args.snr if args.snr is not None else BJ_SNR["r0.1"]
    x, y, u = gaussian_raw_keys(n, B, snr, FRAME_SEED)
    dev = torch.device("cuda:0")
    dx, dy, du = (torch.from_numpy(a).to(dev) for a in (x, y, u))
    alpha = torch.empty_like(dy)
    ynorm = torch.empty((B, n // d), dtype=torch.float32, device=dev)
    llr = torch.empty_like(dx)
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)
    lib = met.lib

    def bob():
        met.api.check(lib.met_mdr_bob(dy.data_ptr(), du.data_ptr(), B, n, d, alpha.data_ptr(), ynorm.data_ptr(), sp))

    def alice():
        met.api.check(lib.met_mdr_alice(dx.data_ptr(), alpha.data_ptr(), ynorm.data_ptr(), 1.0, B, n, d,
                                        llr.data_ptr(), sp))

    for _ in range(args.warmup):
        bob()
        alice()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps + 1)]
    ev[0].record()
    for k in range(args.steps):
        bob()
        ev[2 * k + 1].record()
        alice()
        ev[2 * k + 2].record()
    torch.cuda.synchronize()
    t_bob = sum(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(args.steps)) / args.steps
    t_alice = sum(ev[2 * k + 1].elapsed_time(ev[2 * k + 2]) for k in range(args.steps)) / args.steps
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    elems = B * n
    b_bob, b_alice = elems * (9 + 4 / d), elems * (12 + 4 / d)
    # signs of Alice's LLRs against Bob's bits: the virtual channel's raw error rate
    ber = float(np.mean((llr.cpu().numpy() < 0) != (u == 1)))
    return {
        "metric": "reconciliation front end Mbit/s (raw keys to decoder LLRs)",
        "value": round(elems / (ms * 1e-3) / 1e6, 1),
        "unit": "Mbit/s",
        "ms_per_step": round(ms, 4),
        "config": {"workload": "multidimensional reconciliation, d=8, %d frames of N=%d Gaussian raw keys, SNR %g"
                   % (B, n, snr), "N": n, "frames": B, "d": d, "snr": snr, "frame_seed": FRAME_SEED},
        "roofline": roofline("k_mdr_alice", b_alice, 1, t_alice, None),
        "kernels": {"k_mdr_bob": roofline("k_mdr_bob", b_bob, 1, t_bob, None),
                    "k_mdr_alice": roofline("k_mdr_alice", b_alice, 1, t_alice, None)},
        "virtual_channel_raw_ber": round(ber, 4),
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mix", choices=("mix", "single", "wbp-train", "wbp-eval", "deg1", "mdr"))
    ap.add_argument("--iters", type=int, default=50, help="weighted BP: unrolled iterations")
    ap.add_argument("--ckpt", type=int, default=0,
                    help="weighted BP: checkpoint interval (0 = 10 for training, about sqrt(L) for evaluation)")
    ap.add_argument("--lr", type=float, default=0.01, help="weighted BP: Adam learning rate")
    ap.add_argument("--eval-frames", type=int, default=1000, help="wbp-eval: fresh frames for the FER comparison")
    ap.add_argument("--profile", default="r0.1", choices=sorted(PROFILES), help="code of --workload single")
    ap.add_argument("--n", type=int, default=10**6)
    ap.add_argument("--frames", type=int, default=64, help="frames (per job for the mix)")
    ap.add_argument("--snr", type=float, default=None, help="override every job's SNR")
    ap.add_argument("--max-iter", type=int, default=None, help="override every job's budget")
    ap.add_argument("--fixed-iters", action="store_true")
    ap.add_argument("--c2v-fp16", action="store_true",
                    help="single: check-to-variable messages stored in half precision (MET_C2V_FP16)")
    ap.add_argument("--c2v-q8", action="store_true",
                    help="single: check-to-variable messages stored in 8 bits (MET_C2V_Q8)")
    ap.add_argument("--check-lut", action="store_true",
                    help="single: 8-bit message storage with the table-driven check update (MET_CHECK_LUT)")
    ap.add_argument("--waterfall", action="store_true",
                    help="jobs at the waterfall SNRs of their rates (0.19 / 0.10 / 0.065) instead of the "
                         "workload's operating points")
    ap.add_argument("--check-steps", type=int, default=0, help="check steps per wave (0 = default)")
    ap.add_argument("--vn-chunk", type=int, default=0, help="variable-kernel gathers in flight (0 = default)")
    ap.add_argument("--blocks-per-cu", type=int, default=0, help="persistent blocks per CU (0 = default)")
    ap.add_argument("--no-autotune", action="store_true", help="mix: keep the default persistent launch shape")
    ap.add_argument("--schedule", default="auto", choices=("auto", "phase", "kinds", "jobs", "serial", "persistent"),
                    help="mix: batched schedule (auto = autotuned; phase = one launch per phase, kinds = the same "
                         "with the launches of a phase on parallel streams, jobs = each job's launches a chain on "
                         "parallel streams, serial = those chains one job after the other, persistent = one persistent launch; all "
                         "with the default shape)")
    ap.add_argument("--no-stagger", action="store_true", help="mix: all jobs start in the same phase")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="mix: time the batched form only (profiling runs, where the plain form's launches of the "
                         "same kernels would mix with it)")
    ap.add_argument("--plain-only", action="store_true",
                    help="mix: run the plain form only, warmup + steps decodes of the three jobs, and print no "
                         "metric line (profiling runs of the plain form's kernels)")
    ap.add_argument("--cpu-iters", type=int, default=50, help="iterations per frame in the CPU sample")
    ap.add_argument("--cpu-workers", type=int, default=16)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 1 GiB device copies (scale for rocprofv3 byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        return 2

    if args.copy_calibration:
        import torch

        n = 1 << 28  # 1 GiB of float32
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": 4 * n, "copies": 5}))
        return 0

    if args.workload == "deg1":
        rec = run_deg1(args)
        rec.update({"n_gpus": 1, "steps": args.steps, "warmup": 1, "higher_is_better": True, "scaling": "weak",
                    "vs_baseline": None, "dtype": "f32",
                    "data": "synthetic: seeded uniform bits, BPSK over AWGN, FP32 LLRs; seeded random MET codes"})
        print(json.dumps(rec), flush=True)
        return 0

    if args.workload == "mdr":
        rec = run_mdr(args)
        rec.update({"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
                    "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                    "data": "synthetic: seeded Gaussian raw keys (X ~ N(0, SNR), Y = X + N(0, 1)), uniform bits"})
        print(json.dumps(rec), flush=True)
        return 0

    if args.workload in ("wbp-train", "wbp-eval"):
        rec = run_wbp_train(args) if args.workload == "wbp-train" else run_wbp_eval(args)
        rec.update({"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
                    "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                    "data": "synthetic: seeded uniform bits, BPSK over AWGN, FP32 LLRs; seeded random MET code"})
        print(json.dumps(rec), flush=True)
        return 0

    if args.workload == "mix":
        cpu_jobs = [(p, args.frames, args.max_iter or ITER_BUDGET[p]) for p in MIX]
    else:
        cpu_jobs = [(args.profile, args.frames, args.max_iter or ITER_BUDGET[args.profile])]
    cpu = None
    if not args.no_cpu_baseline:
        # before any GPU initialisation: the oracle runs in forked host processes
        cpu = cpu_baseline(cpu_jobs, args.n, args.snr, min(args.cpu_iters, min(b for _, _, b in cpu_jobs)),
                           args.cpu_workers)

    body = run_mix(args, cpu) if args.workload == "mix" else run_single(args, cpu)
    if body.get("plain_only"):
        print(json.dumps(body), flush=True)
        return 0
    rec = {
        "metric": METRIC,
        "value": body.pop("value"),
        "unit": "Mbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": body.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded uniform bits, BPSK over AWGN, FP32 LLRs; seeded random MET codes",
        "config": body.pop("config"),
        "roofline": body.pop("roofline"),
        "cpu_baseline": cpu,
    }
    rec.update(body)
    rec["tuning"] = {"check_steps_per_wave": args.check_steps, "variable_chunk": args.vn_chunk,
                     "blocks_per_cu": args.blocks_per_cu}
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
