#!/usr/bin/env python3
"""Upper-hood throughput on one MI355X.

One step = one device-resident upper-hood computation of the whole workload
(every round of Wagener merges: tile kernel, then merge passes), inputs
already resident in HBM.  Default workload: one set of n = 2^27 points, x iid
on the 2^-27 grid (sorted, float32), y uniform -- the bandwidth-roofline
configuration.  Prints ONE JSON line on stdout (progress goes to stderr).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "input points/sec (upper hull, 1 GPU) + % HBM roofline; batched vs plain"
KERNEL_SOURCES = ["paper_1203_5004_amd/csrc/wagener_hull.hip",
                  "paper_1203_5004_amd/csrc/uh_device.hpp"]
HOST_MARKER = "// " + "=" * 70 + " host"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the device code (comments and whitespace removed; the host
    part of the library source after its host marker is left out), so that a
    counter summary stays attached to the kernels it was measured on."""
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as fh:
            src = fh.read().split(HOST_MARKER)[0]
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload: str, strip: int):
    """HBM bytes per tile-kernel launch from the committed rocprofv3 --pmc
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"tile_kernel_{workload.replace('^', 'p')}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_hash") != kernel_hash() or d.get("strip") != strip:
        return None
    return d.get("hbm_bytes_per_launch")


class HipEvents:
    """Raw hipEvent_t handles for the library's profiling hook."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float),
                                                 ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        e = ctypes.c_void_p()
        assert self.hip.hipEventCreate(ctypes.byref(e)) == 0
        return e.value

    def elapsed_ms(self, a, b) -> float:
        ms = ctypes.c_float()
        assert self.hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(a),
                                            ctypes.c_void_p(b)) == 0
        return ms.value

    def destroy(self, e):
        self.hip.hipEventDestroy(ctypes.c_void_p(e))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads() -> int:
    """Host threads the all-cores oracle uses: the CPUs this process may run on,
    at most 16 (the host share of one GPU)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(avail, 16))


def cpu_baseline(pts_np, off, budget_s: float, threads: int, lib, both: bool = False,
                 unsorted: bool = False):
    """The oracle over the whole workload, repeated until budget_s, on `threads`
    threads (1: the single chain; more: chunks cut at equal-x runs for one set,
    whole sets per thread for a batch).  With both, the upper and the lower hood
    of every set (outputs laid out as the library's two halves); with unsorted,
    a stable sort of every set by x in front (numpy, one thread) and the corners
    mapped back to input indices."""
    import numpy as np
    import oracle
    t_total, reps = 0.0, 0
    out = cnt = None
    N, S = len(pts_np), len(off) - 1

    def hoods(src, lower):
        if threads == 1:
            fn = oracle.lower_hull_batched if lower else oracle.upper_hull_batched
            return fn(src, off, lib=lib)
        if S == 1:
            rc, idx = oracle.hood_mt(src, threads, lower=lower, lib=lib)
            o = np.zeros(max(N, 1), np.int32)
            o[:len(idx)] = idx
            return o, np.array([rc if rc else len(idx)], np.int64)
        _, o, c = oracle.hood_batched_mt(src, off, threads, lower=lower, lib=lib)
        return o, c

    while reps < 1 or t_total < budget_s:
        t0 = time.perf_counter()
        src, perm = pts_np, None
        if unsorted:
            perm = np.concatenate([off[s] + oracle.sort_order(pts_np[off[s]:off[s + 1]])
                                   for s in range(S)] or [np.zeros(0, np.int64)])
            src = pts_np[perm]
        out, cnt = hoods(src, False)
        if both:
            lo, lcnt = hoods(src, True)
            out, cnt = np.concatenate([out[:N], lo[:N]]), np.concatenate([cnt, lcnt])
        if unsorted:  # sorted positions -> set-relative input indices
            H = 2 if both else 1
            for h in range(H):
                for s in range(S):
                    a = h * N + off[s]
                    c = int(cnt[h * S + s])
                    out[a:a + c] = perm[off[s] + out[a:a + c]] - off[s]
        t_total += time.perf_counter() - t0
        reps += 1
    return N * reps / t_total, reps, t_total, out, cnt


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="uniform_2^27")
    ap.add_argument("--strip", type=int, default=16)
    ap.add_argument("--fan-in", type=int, default=0,
                    help="merge fan-in of the plan (0: the library's default)")
    ap.add_argument("--graph", action="store_true", help="replay each step as a hipGraph")
    ap.add_argument("--force-fallback", action="store_true",
                    help="predicate ablation: every orientation test takes the exact FP64 path")
    ap.add_argument("--autotune", action="store_true",
                    help="choose strip and fan-in by the library's autotuner on this workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=16.0,
                    help="seconds of oracle timing, split between one thread and all")
    ap.add_argument("--compare-plain", action="store_true",
                    help="also time the plain per-set method (one plan per set, launched "
                         "set by set from the host) against the batched plan")
    ap.add_argument("--read-reference", action="store_true",
                    help="also time the library's plain streaming read of the same input: the "
                         "bandwidth a simple read reaches on this GPU")
    ap.add_argument("--both-hoods", action="store_true",
                    help="upper and lower hood of every set from the same read (the convex "
                         "hull's two halves)")
    ap.add_argument("--unsorted", action="store_true",
                    help="shuffle every set (seeded) and let the library sort it by x on the "
                         "device first")
    ap.add_argument("--no-elimination", action="store_true",
                    help="UH_FLAG_NO_ELIMINATION: every point goes through the serial strip "
                         "hoods and every round of Wagener merges (the method itself, no "
                         "filter in front)")
    ap.add_argument("--check-signs", action="store_true",
                    help="UH_FLAG_CHECK_SIGNS: every orientation test also in 128-bit integers "
                         "(soundness check; slow)")
    ap.add_argument("--flush", action="store_true",
                    help="cold caches: overwrite a 1 GiB buffer before every timed step (outside "
                         "the step's own events), so the input is read from HBM, not the 256 MB "
                         "last-level cache")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device-to-device copy first (scale reference for "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU only (asked for {args.gpus}); "
              "the path would shard by contiguous point ranges, one per GPU, their hoods "
              "gathered to one GPU and merged there", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1203_5004_amd as uh
    import synth

    if args.workload not in synth.WORKLOADS:
        sys.exit(f"unknown workload {args.workload}; choose from {list(synth.WORKLOADS)}")
    t0 = time.perf_counter()
    pts_np, off = synth.WORKLOADS[args.workload][0]()
    log(f"[bench] generated {args.workload}: {len(pts_np)} points, {len(off) - 1} sets "
        f"in {time.perf_counter() - t0:.1f}s")

    if args.unsorted:
        t0 = time.perf_counter()
        rng = np.random.default_rng(20350)
        for s in range(len(off) - 1):
            seg = pts_np[off[s]:off[s + 1]]
            seg[...] = seg[rng.permutation(len(seg))]
        log(f"[bench] shuffled every set in {time.perf_counter() - t0:.1f}s")

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("[bench] calibration copy: 2 x 1 GiB device-to-device")
    pts = torch.from_numpy(pts_np).to(dev)
    N, S = len(pts_np), len(off) - 1
    flags = (uh.UH_FLAG_GRAPH if args.graph else 0) | \
        (uh.UH_FLAG_FORCE_FALLBACK if args.force_fallback else 0) | \
        (uh.UH_FLAG_BOTH_HOODS if args.both_hoods else 0) | \
        (uh.UH_FLAG_UNSORTED if args.unsorted else 0) | \
        (uh.UH_FLAG_NO_ELIMINATION if args.no_elimination else 0) | \
        (uh.UH_FLAG_CHECK_SIGNS if args.check_signs else 0)
    H = 2 if args.both_hoods else 1  # hoods per set
    fan_in = args.fan_in
    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        cfg, tms = uh.upper_hull_autotune(pts, off, flags=flags & ~uh.UH_FLAG_GRAPH, reps=3)
        args.strip, fan_in = cfg["strip"], cfg["fan_in"]
        tuned = {"strip": args.strip, "fan_in": fan_in, "ms": round(tms, 4),
                 "seconds": round(time.perf_counter() - t0, 1)}
        log(f"[bench] autotune: strip {args.strip}, fan-in {fan_in} ({tms:.3f} ms)")
    plan = uh.upper_hull_plan_create(off, strip=args.strip, fan_in=fan_in, flags=flags)
    plan_cfg = plan.config
    out_idx = torch.empty(max(H * N, 1), dtype=torch.int32, device=dev)
    out_cnt = torch.empty(H * S, dtype=torch.int32, device=dev)
    stats = uh.new_stats(H * S, dev)

    ev = HipEvents()
    probes = []
    if not args.graph:
        probes = [(ev.create(), ev.create()) for _ in range(args.steps)]

    # correctness of what is about to be timed: counters + status
    plan.run(pts, out_idx, out_cnt, stats)
    torch.cuda.synchronize()
    cnt_np = out_cnt.cpu().numpy()
    if np.any(cnt_np < 0):
        sys.exit(f"bench: data error status {cnt_np.min()}")
    st = uh.decode_stats(stats.cpu().numpy())
    evals, fallbacks = int(st["orient_evals"].sum()), int(st["fallbacks"].sum())
    sign_errors = int(st["sign_errors"].sum()) if args.check_signs else None

    for _ in range(args.warmup):
        plan.run(pts, out_idx, out_cnt)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps, {plan.launches} launches per step)")

    # Two timed passes of K steps each.  The step time comes from the first,
    # with nothing but the library's own launches on the stream.  The tile
    # kernel's duration comes from the second, with a pair of events recorded
    # around the tile kernel of every step (the library's probe hook): an
    # event recorded between two kernels holds the next launch back by some
    # microseconds, so it stays out of the step time.
    scratch = torch.empty(1 << 28, dtype=torch.float32, device=dev) if args.flush else None

    def timed_pass(with_probes):
        marks = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(args.steps)]
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        if scratch is None:
            # one untimed step first: the host enqueues the timed steps while
            # it runs, so the window holds the K steps back to back and not
            # the host's latency to the first launch
            plan.run(pts, out_idx, out_cnt)
            start.record()
        for k in range(args.steps):
            if scratch is not None:
                # cold caches: the cache-clearing write between steps is outside the
                # step's own events
                scratch.fill_(float(k))
                marks[k][0].record()
            if with_probes:
                plan.set_probe(*probes[k])
            plan.run(pts, out_idx, out_cnt)
            if scratch is not None:
                marks[k][1].record()
        if scratch is None:
            end.record()
        torch.cuda.synchronize()
        if with_probes:
            plan.set_probe(None, None)
        if scratch is not None:
            return sum(a.elapsed_time(b) for a, b in marks)
        return start.elapsed_time(end)

    total_ms = timed_pass(False)
    ms_step = total_ms / args.steps
    value = N / (ms_step * 1e-3)
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step, {value:.4g} points/s")

    tile_ms = None
    if probes:
        timed_pass(True)
        tile_ms = sum(ev.elapsed_ms(a, b) for a, b in probes) / len(probes)
        for a, b in probes:
            ev.destroy(a)
            ev.destroy(b)
    del scratch

    plain = None
    if args.compare_plain:
        log(f"[bench] plain per-set method: {S} plans ...")
        pflags = flags & (uh.UH_FLAG_BOTH_HOODS | uh.UH_FLAG_UNSORTED)
        plans = [uh.upper_hull_plan_create([0, int(off[s + 1] - off[s])], strip=args.strip,
                                           flags=pflags) for s in range(S)]
        scratch_idx = torch.empty(max(H * int(np.max(np.diff(off))), 1), dtype=torch.int32,
                                  device=dev)
        scratch_cnt = torch.empty(H * S, dtype=torch.int32, device=dev)
        if H == 1:
            views = [(pts[off[s]:off[s + 1]], out_idx[off[s]:max(off[s + 1], off[s] + 1)],
                      out_cnt[s:s + 1]) for s in range(S)]
        else:  # both hoods of each set into scratch; the counts are compared below
            views = [(pts[off[s]:off[s + 1]], scratch_idx, scratch_cnt[H * s:H * s + H])
                     for s in range(S)]
        for s in range(S):  # warm-up
            plans[s].run(*views[s])
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 5))
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record()
        for _ in range(reps):
            for s in range(S):
                plans[s].run(*views[s])
        end.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        gpu_ms = start.elapsed_time(end) / reps
        if H == 1:
            plain_ok = bool(np.array_equal(out_cnt.cpu().numpy(), cnt_np))
        else:
            sc = scratch_cnt.cpu().numpy().reshape(S, 2)
            plain_ok = bool(np.array_equal(sc[:, 0], cnt_np[:S]) and
                            np.array_equal(sc[:, 1], cnt_np[S:]))
        for pl in plans:
            pl.close()
        plain = {"ms_per_step": round(gpu_ms, 3), "host_wall_ms_per_step": round(wall * 1e3, 3),
                 "points_per_s": round(N / (gpu_ms * 1e-3), 1),
                 "batched_speedup": round(gpu_ms / ms_step, 2), "same_counts": plain_ok}
        log(f"[bench] plain: {gpu_ms:.3f} ms/step -> batched is {gpu_ms / ms_step:.2f}x faster")

    read_ref = None
    if args.read_reference:
        rms = uh.upper_hull_read_reference(pts, reps=20)
        read_ref = {"what": "plain coalesced read of the same points (upper_hull_read_reference)",
                    "ms": round(rms, 4), "GB/s": round(8.0 * N / (rms * 1e-3) / 1e9, 1)}
        log(f"[bench] plain read of the input: {rms:.4f} ms = {read_ref['GB/s']} GB/s")

    h_total = int(cnt_np.sum())
    alg_tile = 8.0 * N  # every point read once (float2)
    roofline = None
    if tile_ms:
        achieved = alg_tile / (tile_ms * 1e-3) / 1e9
        traffic = None if (args.both_hoods or args.unsorted or args.no_elimination) else \
            load_traffic(args.workload, args.strip)
        roofline = {"bound": "hbm", "kernel": "tile_kernel", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "tile_kernel_ms": round(tile_ms, 4),
                    "plain_read": read_ref}
    path_gbs = (8.0 * N + 4.0 * h_total) / (ms_step * 1e-3) / 1e9

    cpu = None
    checked = None
    if not args.no_cpu_baseline:
        import oracle
        import tempfile
        lib = oracle.load_native(tempfile.mkdtemp(prefix="uh_oracle_"))
        threads = cpu_threads()
        what = (f"whole workload ({N} points, {S} sets"
                f"{', both hoods' if H == 2 else ''}"
                f"{', sorted by x first (numpy, one thread)' if args.unsorted else ''})")
        log(f"[bench] timing the CPU oracle (-O3 -march=native) on 1 and {threads} threads ...")
        rate1, reps1, secs1, ref_out, ref_cnt = cpu_baseline(
            pts_np, off, args.cpu_budget / 2, 1, lib, both=args.both_hoods,
            unsorted=args.unsorted)
        rate, reps, secs, mt_out, mt_cnt = cpu_baseline(
            pts_np, off, args.cpu_budget / 2, threads, lib, both=args.both_hoods,
            unsorted=args.unsorted)
        got = out_idx.cpu().numpy()
        voff = np.concatenate([off[:-1] + h * N for h in range(H)])  # start of every output set
        checked = bool(np.array_equal(cnt_np, ref_cnt.astype(np.int32)) and all(
            np.array_equal(got[a:a + c], ref_out[a:a + c]) for a, c in zip(voff, cnt_np)))
        mt_same = bool(np.array_equal(mt_cnt, ref_cnt) and all(
            np.array_equal(mt_out[a:a + c], ref_out[a:a + c]) for a, c in zip(voff, cnt_np)))
        cpu = {"value": round(rate, 1), "unit": "points/s", "cores": threads, "kind": "oracle",
               "sample": f"{what}: {reps} run(s) in {secs:.1f} s on {threads} threads; "
                         f"{reps1} run(s) in {secs1:.1f} s on one thread",
               "single_thread_value": round(rate1, 1), "threads_equal_single": mt_same,
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
               "build": "gcc -O3 -march=native"}
        log(f"[bench] oracle {rate1:.4g} points/s (1 thread), {rate:.4g} ({threads} threads); "
            f"GPU result equals oracle: {checked}")

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_points": N, "sets": S, "strip": args.strip,
                   "tile_points": 64 * args.strip, "launches_per_step": plan.launches,
                   "fan_in": plan_cfg["fan_in"], "autotuned": tuned,
                   "graph": bool(args.graph), "force_fallback": bool(args.force_fallback),
                   "cold_cache": bool(args.flush),
                   "hoods": "upper and lower" if H == 2 else "upper",
                   "input_order": "shuffled (sorted on the device)" if args.unsorted else "by x",
                   "corners": h_total,
                   "orient_evals_per_point": round(evals / max(N, 1), 3),
                   "fallback_rate": (fallbacks / evals) if evals else 0.0,
                   "elimination": not args.no_elimination,
                   "sign_errors": sign_errors,
                   "path_hbm_frac": round(path_gbs / HBM_PEAK_GBS, 4),
                   "matches_oracle": checked},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain_per_set": plain,
    }
    print(json.dumps(line), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
