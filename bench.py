#!/usr/bin/env python3
"""Benchmark: particle cell-crossings per second on one MI355X.

One step = one pass of the whole tracking path over one batch: restore the
released particle state (device-to-device copy), track every particle to its
stopping condition through the C ABI (pt_track: counter reset, ordering sort,
tracking kernel), and read the run summary (pt_results).  Grids and particles
are resident in HBM before the timed region starts.  The K timed steps are
enqueued back to back on one stream and their summaries read afterwards, so
the timed region holds the device work of K steps and no host wait between
them.

Default workload (C4, the batched form of the metric): 16 realisations of a
100x100x10 grid of 10x10x2 m cells, lognormal K with geometric mean 10 m/d,
sigma^2 drawn from U[0.5, 4], correlation length 5 cells, heads 10/0 m
west/east, porosity 0.3; 64 particle groups of log-uniform sizes in [1e3, 2e6]
(1.77e7 particles) released in the 10 western columns, group g on realisation
g mod 16; endpoint mode, FP64, packed cell records, one hipGraph launch over
every group, with the autotuned launch of this device and workload
(paper_2302_13590_amd/tuning.json: schedule, block size, processing order).

Also timed in the same run: the other FP64 kernel and the mixed-precision
kernel on C4 (with its path and travel-time accuracy against the FP64 run and
against the oracle); C2 (FP64, mixed, pathline mode), C3 (FP64, mixed), C5
(timeseries, FP64 and mixed with the snapshot position error), C6 (transient
flow) and C7 (quadtree).  The CPU oracle is timed on the host cores on a
sample of C4, and the FP64 run is compared bitwise with the oracle on that
sample.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W] [--workload W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

METRIC = "particle cell-crossings/s at 1 GPU (FP64 vs mixed/batched); % HBM roofline"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes: per crossing, the cell's six face flows + porosity (8 B each) + flags (4 B)
# in FP64, six FP32 velocities + porosity + flags in mixed; per particle, the state read
# (cell 4, xi/eta/zeta/t 32, status 4, ncross 4, hash 8 = 52 B), written back (52 B) and
# the final global position (24 B)
BYTES_PER_CROSSING = {"fp64": 60, "mixed": 32}
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2 (FMA) x 2.4 GHz
BYTES_PER_PARTICLE = 52 + 52 + 24


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def host_cpu_model():
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def workload(name):
    import workloads
    try:
        return workloads.workload(name)
    except KeyError:
        raise SystemExit("unknown workload " + name)


DESCR = {
    "C1": "C1: 40x40x1 homogeneous K=10 m/d, 1e3 particles, endpoint",
    "C2": "C2: 100x100x10 lognormal K (sigma^2=1, corr. 5 cells), 1e6 particles, endpoint",
    "C3": "C3: 200x200x20 lognormal K (sigma^2=4, corr. 8 cells), 2 wells + recharge, 1e7 particles",
    "C4": "C4: 16 realisations 100x100x10 (sigma^2 ~ U[0.5,4]), 64 groups, 1.77e7 particles, batched",
    "C5": "C5: 200x200x20 lognormal K (sigma^2=2), 1e6 particles, timeseries 100 snapshots [1e6,100,3]",
    "C6": "C6: C2's grid under transient flow (12 time steps, a well switching on and off), 1e6 particles "
          "released in 10 stages, weak sinks pass through",
    "C7": "C7: quadtree grid, 3-layer aquifer refined around two wells (16,455 cells from 256x256x3 fine), "
          "1e6 particles over the top layer",
}


class Case:
    """Device-resident inputs of one workload and the timed step."""

    def __init__(self, w):
        import torch
        from paper_2302_13590_amd import pt
        self.pt, self.torch, self.w = pt, torch, w
        self.grids = [pt.load_any_grid(g) for g in w.grids]
        self.pristine = pt.DeviceParticles.from_numpy(w.particles, "cuda")
        self.work = self.pristine.clone()
        n = self.pristine.n
        self.out_xyz = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        self.snap = None
        if w.snap_times is not None:
            self.snap = torch.empty((n, len(w.snap_times), 3), dtype=torch.float64, device="cuda")
        self.stream = torch.cuda.current_stream()

    def opts(self, precision, schedule_name, **kw):
        pt = self.pt
        o = dict(precision=pt.PT_MIXED if precision == "mixed" else pt.PT_FP64,
                 schedule=pt.PT_SCHED_STATIC if schedule_name == "static" else pt.PT_SCHED_PERSISTENT,
                 layout=pt.PT_LAYOUT_CELL, use_graph=1, out_xyz=self.out_xyz, t_max=self.w.t_max)
        if self.snap is not None:
            o.update(mode=pt.PT_TIMESERIES, snap_times=self.w.snap_times, snap_xyz=self.snap)
        if self.w.tstep_end is not None:
            o.update(tstep_end=self.w.tstep_end)
        o.update(stop_at_sink=self.w.stop_at_sink)
        o.update(kw)
        return pt.make_opts(**o)

    def step(self, o):
        pt = self.pt
        self.work.copy_(self.pristine)
        run = pt.pt_track(self.grids, self.work, o, stream=self.stream,
                          group_offsets=self.w.group_offsets, group_grid=self.w.group_grid)
        s = pt.pt_results(run)
        run.release()
        return s

    def enqueue(self, o):
        """Restore the state and enqueue one tracking call (no host wait)."""
        self.work.copy_(self.pristine)
        return self.pt.pt_track(self.grids, self.work, o, stream=self.stream,
                                group_offsets=self.w.group_offsets, group_grid=self.w.group_grid)

    def run_steps(self, o, steps):
        """`steps` steps enqueued back to back on the stream, then their summaries."""
        runs = [self.enqueue(o) for _ in range(steps)]
        summ = [self.pt.pt_results(r) for r in runs]
        for r in runs:
            r.release()
        return summ

    def time(self, o, steps, warmup):
        torch = self.torch
        if warmup > 0:
            for _ in range(warmup):
                self.step(o)
            self.run_steps(o, steps)       # every pooled run has built its graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        summ = self.run_steps(o, steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        cross = summ[0]["crossings"]
        assert all(s["crossings"] == cross for s in summ), "crossing count changed between steps"
        # the tracking kernel's own device time (events just around its launch), and that of the
        # whole pt_track sequence (counter reset, ordering sort, tracking kernel, careful pass)
        kms = float(np.mean([s["track_ms"] for s in summ]))
        cms = float(np.mean([s["kernel_ms"] for s in summ]))
        return dict(wall_s=wall, ms_per_step=1e3 * wall / steps, crossings_per_step=cross,
                    value=cross * steps / wall, kernel_ms=kms, call_ms=cms, summary=summ[0])

    def time_pathline(self, precision, schedule_name, steps, warmup, **kw):
        """One step = restore the state, the count pass (offsets), the record pass (one record
        per crossing).  The record arrays are allocated once, before timing, at the size the
        first count pass reports."""
        pt, torch = self.pt, self.torch
        n = self.pristine.n
        offs = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        oc = self.opts(precision, schedule_name, mode=pt.PT_PATHLINE, path_offsets=offs, path_count_only=1, **kw)
        self.work.copy_(self.pristine)
        m = self.step(oc)["path_records"]
        records = pt.path_record_buffer(m)
        orec = self.opts(precision, schedule_name, mode=pt.PT_PATHLINE, path_offsets=offs, path_count_only=0,
                         path_cap=m, path_records=records, **kw)

        def enqueue():
            self.work.copy_(self.pristine)
            a = pt.pt_track(self.grids, self.work, oc, stream=self.stream,
                            group_offsets=self.w.group_offsets, group_grid=self.w.group_grid)
            b = pt.pt_track(self.grids, self.work, orec, stream=self.stream,
                            group_offsets=self.w.group_offsets, group_grid=self.w.group_grid)
            return a, b

        def run_steps(k):
            runs = [enqueue() for _ in range(k)]
            out = []
            for a, b in runs:
                sa, sb = pt.pt_results(a), pt.pt_results(b)
                a.release()
                b.release()
                assert sa["path_records"] == m and sb["path_records"] == m and sb["path_dropped"] == 0
                out.append((sa, sb))
            return out

        if warmup > 0:
            run_steps(max(warmup, steps))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        summ = run_steps(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        cross = summ[0][1]["crossings"]
        return dict(value=cross * steps / wall, ms_per_step=1e3 * wall / steps, crossings_per_step=cross,
                    records_per_step=m, record_bytes=m * 40 + (n + 1) * 8,
                    count_ms=float(np.mean([a["kernel_ms"] for a, _ in summ])),
                    record_ms=float(np.mean([b["kernel_ms"] for _, b in summ])))

    def release(self):
        for g in self.grids:
            g.release()


KERNEL_SOURCES = ["paper_2302_13590_amd/csrc/pt_kernels.hip", "paper_2302_13590_amd/csrc/pt_crmath.h",
                  "paper_2302_13590_amd/csrc/pt_crtables.h", "paper_2302_13590_amd/csrc/pt_internal.h"]
ROOT = os.path.dirname(os.path.abspath(__file__))


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_value(kind, key, workload, precision, schedule):
    """A figure of a committed rocprofv3 summary (profiles/track_<precision>_<workload>_<schedule>_
    <kind>.txt), if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "track_%s_%s_%s_%s.txt" % (precision, workload, schedule, kind))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if vals.get("kernel_sources_sha256") != kernel_sources_sha():
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def profiled_traffic(workload, precision, schedule):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE, WRITE_SIZE)."""
    return profile_value("counters", "hbm_bytes_per_launch", workload, precision, schedule)


def kernel_name(precision, schedule, timeseries=False, batched=False):
    return "k_track_%s<%s, cell, %s%s>" % ("static" if schedule == "static" else "persistent",
                                           "FP64" if precision == "fp64" else "mixed",
                                           "timeseries" if timeseries else "endpoint",
                                           ", batched" if batched else "")


def roofline(res, n, precision, workload, schedule, timeseries=False, batched=False):
    bytes_launch = res["crossings_per_step"] * BYTES_PER_CROSSING[precision] + n * BYTES_PER_PARTICLE
    achieved = bytes_launch / (res["kernel_ms"] * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 5),
           "traffic": profiled_traffic(workload, precision, schedule),
           "bytes_per_launch": int(bytes_launch), "kernel_ms": round(res["kernel_ms"], 4),
           "call_ms": round(res["call_ms"], 4),
           "kernel": kernel_name(precision, schedule, timeseries, batched)}
    # the vector-ALU view of the same kernel, from the committed instruction counters: issued VALU
    # cycles over the available ones, and the FP64 arithmetic rate (add, multiply, transcendental:
    # one flop per lane slot, FMA two) against the FP64 vector peak
    busy = profile_value("valu", "valu_busy", workload, precision, schedule)
    if busy is not None:
        out["valu_busy"] = busy
        cnt = [profile_value("valu", "SQ_INSTS_VALU_%s" % k, workload, precision, schedule)
               for k in ("ADD_F64", "MUL_F64", "FMA_F64", "TRANS_F64")]
        cross = profile_value("valu", "crossings_per_launch", workload, precision, schedule)
        if None not in cnt and cross:
            per_cross = 64.0 * (cnt[0] + cnt[1] + 2.0 * cnt[2] + cnt[3]) / cross
            tflops = per_cross * res["crossings_per_step"] / (res["kernel_ms"] * 1e-3) / 1e12
            out["alu"] = {"fp64_flops_per_crossing": round(per_cross, 1), "achieved": round(tflops, 2),
                          "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": round(tflops / FP64_VECTOR_PEAK_TFLOPS, 4), "valu_busy": busy}
    return out


def tuned_params(workload, precision, mode):
    from paper_2302_13590_amd import autotune
    return autotune.lookup(autotune.key(autotune.device_name(), workload, precision, mode))


def oracle_sample_indices(n, m):
    """Every ceil(n/m)-th particle: a bounded sample that spans every group of a batched run."""
    stride = max(1, -(-n // m))
    return np.arange(0, n, stride)


def oracle_on_sample(w, idx, threads):
    """The oracle (plain FP64 CPU tracker) on the particles idx of workload w, per group for
    batched runs; returns (result, seconds)."""
    from oracle import oracle as O
    sub = w.particles.subset(idx)
    t0 = time.perf_counter()
    if w.group_offsets is None:
        r = O.track(w.grids[0], sub, t_max=w.t_max, snap_times=w.snap_times, threads=threads)
    else:
        offs = np.searchsorted(idx, w.group_offsets).astype(np.int64)
        r = O.track_groups(w.grids, sub, offs, w.group_grid, t_max=w.t_max, threads=threads)
    return r, time.perf_counter() - t0


def cpu_share():
    """Host threads this process may use: the affinity mask, capped by OMP_NUM_THREADS when set
    (the CPU share of one GPU on a shared host)."""
    cores = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    return (min(cores, int(env)) if env.isdigit() and int(env) > 0 else cores), cores


def fp64_parity(state, r, idx):
    """Bitwise comparison of the FP64 GPU final state with the oracle on the sample."""
    eq = np.ones(idx.size, dtype=bool)
    for k in ("cell", "status", "ncross", "path_hash", "xi", "eta", "zeta", "t"):
        a, b = state[k][idx], getattr(r, k)
        eq &= (a == b) | (np.isnan(a) & np.isnan(b)) if a.dtype.kind == "f" else (a == b)
    a, b = state["out_xyz"][idx], r.out_xyz
    eq &= ((a == b) | (np.isnan(a) & np.isnan(b))).all(axis=1)
    return {"particles": int(idx.size), "bitwise_equal": int(eq.sum()),
            "reference": "the FP64 oracle (plain CPU tracker) on the CPU-baseline sample"}


def oracle_full(wname, threads, chunk=100_000):
    """The CPU oracle over every particle of workload wname (crossings/s on `threads` threads), in
    chunks of `chunk` consecutive particles timed one after another, with a progress line per chunk.
    The full-workload counterpart of the benchmark's bounded cpu_baseline sample; one JSON line."""
    if wname not in ("C1", "C2", "C3", "C4", "C5"):
        print("--oracle-full times the structured steady workloads C1-C5", file=sys.stderr)
        return 2
    w = workload(wname)
    n = w.particles.n
    total_s, total_cross = 0.0, 0
    for lo in range(0, n, chunk):
        idx = np.arange(lo, min(n, lo + chunk))
        r, dt = oracle_on_sample(w, idx, threads)
        total_s += dt
        total_cross += int(r.ncross.astype(np.int64).sum())
        log("oracle %s: particles %d..%d, %.1f s so far, %.4g crossings/s" % (
            wname, lo, idx[-1], total_s, total_cross / total_s))
    print(json.dumps({"kind": "oracle", "workload": DESCR[wname], "threads": threads, "particles": n,
                      "crossings": total_cross, "seconds": round(total_s, 2),
                      "value": total_cross / total_s, "unit": "cell-crossings/s", "cpu_model": host_cpu_model(),
                      "host_cores_visible": len(os.sched_getaffinity(0))}), flush=True)
    return 0


# launch parameters of the scheduling study (the tuned C2/C3 shapes of each kernel)
STUDY_LAUNCH = {"static": dict(block=256), "persistent": dict(block=256, refill=1, chunk=32, steps_per_refill=2)}


def scheduling_study(sigma2s, nps, reps):
    """Static vs persistent kernel on the first test case's shape (Results "Thread scheduling",
    the paper's Fig. 5 and 6 on 1-8 CPU threads): kernel time of each schedule for every
    variance and particle count, and their ratio T_persistent / T_static (the analogue of the
    paper's T_dyn / T_sta).  One JSON line per configuration, then a markdown table."""
    import torch
    from workloads import configs as C
    rows = []
    for s2 in sigma2s:
        t0 = time.perf_counter()
        C.tc1_grid(s2)
        log("TC1 grid sigma^2=%g ready in %.1fs" % (s2, time.perf_counter() - t0))
        for n in nps:
            case = Case(C.tc1(n, s2))
            row = {"sigma2": s2, "particles": n}
            for sched in ("static", "persistent"):
                o = case.opts("fp64", sched, **STUDY_LAUNCH[sched])
                case.step(o)   # warm-up (graph build)
                summ = [case.step(o) for _ in range(reps)]
                ms = float(np.median([q["kernel_ms"] for q in summ]))
                row[sched + "_ms"] = round(ms, 4)
                row["crossings"] = summ[0]["crossings"]
            nc = case.work.ncross.to(torch.float64)
            row["crossings_per_particle_mean"] = round(float(nc.mean()), 1)
            row["crossings_per_particle_max"] = int(nc.max())
            row["ratio_persistent_static"] = round(row["persistent_ms"] / row["static_ms"], 4)
            row["crossings_per_s_best"] = row["crossings"] / (1e-3 * min(row["static_ms"], row["persistent_ms"]))
            case.release()
            rows.append(row)
            print(json.dumps(row), flush=True)
    print("\n| sigma^2 | N_p | crossings/particle (mean / max) | static ms | persistent ms | T_pers/T_stat | best crossings/s |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        print("| %g | %.0e | %.1f / %d | %.3f | %.3f | %.3f | %.3g |" % (
            r["sigma2"], r["particles"], r["crossings_per_particle_mean"], r["crossings_per_particle_max"],
            r["static_ms"], r["persistent_ms"], r["ratio_persistent_static"], r["crossings_per_s_best"]))
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C4", choices=sorted(DESCR))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--schedule", default="auto", choices=["auto", "persistent", "static"],
                    help="auto: the autotuned launch for this workload (tuning.json)")
    ap.add_argument("--only", action="store_true",
                    help="time only the primary variant (no other variants, no CPU baseline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-workloads", action="store_true",
                    help="time only the chosen workload's variants, not the other workloads")
    ap.add_argument("--cpu-sample", type=int, default=500_000,
                    help="particles of the oracle's all-threads sample (the one-thread leg takes a tenth)")
    ap.add_argument("--lib", default=None,
                    help="load this build of libpt.so instead of the in-tree one (e.g. a copy of the "
                         "sources built with python -m paper_2302_13590_amd.build --src DIR --out PATH)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one plain elementwise copy of this many bytes (HBM-counter calibration)")
    ap.add_argument("--study", choices=["scheduling"],
                    help="instead of the benchmark line: static vs persistent on the first test case's "
                         "shape over variances and particle counts")
    ap.add_argument("--oracle-full", action="store_true",
                    help="instead of the benchmark line: the CPU oracle alone over every particle of the "
                         "workload on --oracle-threads threads, in chunks of 1e5 particles (no GPU)")
    ap.add_argument("--oracle-threads", type=int, default=1)
    ap.add_argument("--study-sigma2", default="0.1,1,2.5,5")
    ap.add_argument("--study-np", default="1e3,1e4,1e5,1e6,1e7")
    args = ap.parse_args()

    if args.oracle_full:
        return oracle_full(args.workload, args.oracle_threads)
    if args.gpus != 1:
        print("bench.py measures one GPU: the tracker runs on a single MI355X (particles are independent, "
              "so the path would shard by particle with no exchange until a final reduction of the counters).",
              file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    from paper_2302_13590_amd import accuracy as ACC
    from paper_2302_13590_amd import pt
    if args.lib:
        pt.load_library(os.path.abspath(args.lib))
    else:
        pt.load_library()
    if args.study == "scheduling":
        return scheduling_study([float(v) for v in args.study_sigma2.split(",")],
                                [int(float(v)) for v in args.study_np.split(",")], max(1, args.steps // 3))

    if args.copy_bytes > 0:
        # a plain streaming kernel of known traffic: reads and writes copy_bytes each
        n = args.copy_bytes // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 0.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    def launch(precision, schedule, wname, wmode):
        """Launch parameters: the autotuned ones when they use this schedule, else defaults."""
        tuned = tuned_params(wname, precision, wmode) or {}
        sched_id = 1 if schedule == "static" else 2
        if schedule == "auto" and tuned:
            return tuned, ("static" if tuned.get("schedule") == 1 else "persistent")
        if schedule == "auto":
            return dict(schedule=2), "persistent"
        if tuned.get("schedule") == sched_id:
            return tuned, schedule
        return dict(schedule=sched_id), schedule

    def state_of(case):
        d = case.work.to_numpy()
        d["out_xyz"] = case.out_xyz.cpu().numpy()
        return d

    def bench_workload(wname, precision, schedule, extra_variants, acc_oracle=None):
        """Time one workload: the primary kernel, then the variants; returns (primary, variants,
        FP64 final state, inputs)."""
        t0 = time.perf_counter()
        w = workload(wname)
        n = w.particles.n
        mode = "timeseries" if w.snap_times is not None else "endpoint"
        batched = len(w.grids) > 1 and w.tstep_end is None
        log("%s ready in %.1fs: %d particles, %d grid(s)" % (wname, time.perf_counter() - t0, n, len(w.grids)))
        case = Case(w)
        params, sched = launch(precision, schedule, wname, mode)
        primary = case.time(case.opts(precision, sched, **params), args.steps, args.warmup)
        primary.update(params=params, schedule=sched, mode=mode, batched=batched, n=n, workload=wname)
        log("%s %s/%s %s: %.4g crossings/s, %.3f ms/step, kernel %.3f ms" % (
            wname, precision, sched, params, primary["value"], primary["ms_per_step"], primary["kernel_ms"]))
        ref_state = state_of(case) if precision == "fp64" else None
        ref_snap = case.snap.clone() if (case.snap is not None and precision == "fp64") else None
        variants = {}
        for prec, sc in extra_variants:
            p2, s2 = launch(prec, sc, wname, mode)
            if (prec, s2) == (precision, sched):
                continue
            r = case.time(case.opts(prec, s2, **p2), args.steps, args.warmup)
            tag = "%s_%s_%s" % (wname, prec, s2)
            v = dict(value=r["value"], ms_per_step=round(r["ms_per_step"], 4),
                     kernel_ms=round(r["kernel_ms"], 4), crossings_per_step=r["crossings_per_step"],
                     recheck_tracks=r["summary"]["recheck_tracks"],
                     launch=p2, roofline_frac=roofline(r, n, prec, wname, s2, mode == "timeseries", batched)["frac"])
            if prec == "mixed" and ref_state is not None:
                mix = state_of(case)
                acc = ACC.path_agreement(mix, ref_state, w.particles.t)
                acc["reference"] = "the FP64 run of every particle (bitwise identical to the FP64 oracle in the parity tests)"
                v["accuracy"] = acc
                if ref_snap is not None:
                    tr = ACC.trajectory_error(case.snap, ref_snap)
                    tr["reference"] = "the FP64 run's snapshots of every particle"
                    v["trajectory_error"] = tr
                if acc_oracle is not None:
                    idx, ro = acc_oracle(w)
                    sub = {k: mix[k][idx] for k in ("status", "t", "ncross", "path_hash")}
                    ao = ACC.path_agreement(sub, {k: getattr(ro, k) for k in sub}, w.particles.t[idx])
                    ao["reference"] = "the FP64 oracle on %d sampled particles" % idx.size
                    v["accuracy_vs_oracle"] = ao
                    if ro.snap_xyz is not None:
                        to = ACC.trajectory_error(case.snap[torch.from_numpy(idx).cuda()].cpu().numpy(), ro.snap_xyz)
                        to["reference"] = "the FP64 oracle's snapshots of %d sampled particles" % idx.size
                        v["trajectory_error_vs_oracle"] = to
                log("%s mixed accuracy: path agreement %.4f, travel time rel. err. p50 %.2e p99 %.2e" % (
                    wname, acc["path_agreement"], acc["travel_time_rel_err"]["p50"], acc["travel_time_rel_err"]["p99"]))
            variants[tag] = v
            log("variant %s: %.4g crossings/s, kernel %.3f ms" % (tag, r["value"], r["kernel_ms"]))
        if mode == "endpoint" and wname == "C2" and not args.only:
            r = case.time_pathline("fp64", sched, args.steps, args.warmup, **params)
            variants["C2_fp64_pathline"] = dict(
                value=r["value"], ms_per_step=round(r["ms_per_step"], 4), count_ms=round(r["count_ms"], 4),
                record_ms=round(r["record_ms"], 4), records_per_step=r["records_per_step"],
                record_bytes_per_step=r["record_bytes"],
                launch=params, note="count pass + record pass per step (one record of 40 B per crossing)")
            log("variant pathline: %.4g crossings/s, count %.3f ms + record %.3f ms" % (
                r["value"], r["count_ms"], r["record_ms"]))
        case.release()
        del case
        torch.cuda.empty_cache()
        return primary, variants, ref_state, w

    threads, host_cores = cpu_share()
    cpu = {}

    def oracle_for_accuracy(w):
        """The oracle's sample of the primary workload (shared by the CPU baseline, the FP64 parity
        count and the mixed run's accuracy), computed once."""
        if "sample" not in cpu:
            idx = oracle_sample_indices(w.particles.n, args.cpu_sample)
            log("timing the CPU oracle on %d threads, %d particles" % (threads, idx.size))
            r, dt = oracle_on_sample(w, idx, threads)
            cpu["sample"] = (idx, r, dt)
        idx, r, _ = cpu["sample"]
        return idx, r

    want_cpu = not args.only and not args.no_cpu_baseline
    extra = [] if args.only else [("fp64", "static"), ("fp64", "persistent"), ("mixed", "auto")]
    primary, variants, ref_state, w = bench_workload(args.workload, args.precision, args.schedule, extra,
                                                     oracle_for_accuracy if want_cpu else None)
    n = primary["n"]
    out = {
        "metric": METRIC,
        "value": primary["value"],
        "unit": "cell-crossings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(primary["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": DESCR[args.workload], "particles": n,
                   "crossings_per_step": primary["crossings_per_step"], "precision": args.precision,
                   "schedule": primary["schedule"], "layout": "cell", "launch": "hipGraph",
                   "params": primary["params"], "block": primary["summary"]["block"],
                   "grid": primary["summary"]["grid"]},
        "roofline": roofline(primary, n, args.precision, args.workload, primary["schedule"],
                             primary["mode"] == "timeseries", primary["batched"]),
        # FP64: particles handed to the careful pass (an evaluation within 2^-96 of a rounding
        # boundary) and evaluations left undecided, in the first timed step
        "rounding": {"recheck_tracks": primary["summary"]["recheck_tracks"],
                     "cr_ambiguous": primary["summary"]["cr_ambiguous"]},
    }
    if want_cpu:
        idx, r = oracle_for_accuracy(w)
        dt = cpu["sample"][2]
        value = float(r.ncross.astype(np.int64).sum()) / dt
        idx1 = oracle_sample_indices(w.particles.n, max(1, args.cpu_sample // 10))
        r1, dt1 = oracle_on_sample(w, idx1, 1)
        v1 = float(r1.ncross.astype(np.int64).sum()) / dt1
        out["cpu_baseline"] = {
            "value": value, "unit": "cell-crossings/s", "cores": threads, "kind": "oracle",
            "sample": "every %d-th particle of the workload (%d particles, %d crossings), OpenMP dynamic over "
                      "particles on %d threads, %.1f s; 1 thread on every %d-th particle (%d): %.4g crossings/s, "
                      "%.1f s" % (max(1, int(idx[1] - idx[0])) if idx.size > 1 else 1, idx.size,
                                  int(r.ncross.astype(np.int64).sum()), threads, dt,
                                  max(1, int(idx1[1] - idx1[0])) if idx1.size > 1 else 1, idx1.size, v1, dt1),
            "host_cores_visible": host_cores, "cpu_model": host_cpu_model(),
            "one_thread": {"value": v1, "particles": int(idx1.size), "seconds": round(dt1, 2)},
        }
        if ref_state is not None:
            out["fp64_parity"] = fp64_parity(ref_state, r, idx)
            log("FP64 parity on the oracle sample: %d of %d particles bitwise equal" % (
                out["fp64_parity"]["bitwise_equal"], out["fp64_parity"]["particles"]))
    def small_oracle_sample(wc):
        """A 20,000-particle oracle sample of a further workload (its mixed run's accuracy)."""
        idx = oracle_sample_indices(wc.particles.n, 20_000)
        return idx, oracle_on_sample(wc, idx, threads)[0]

    if not args.only and not args.no_extra_workloads and args.workload == "C4":
        for wname, prec_list in (("C2", [("mixed", "auto")]), ("C3", [("mixed", "auto")]),
                                 ("C5", [("mixed", "auto")]), ("C6", []), ("C7", [])):
            pr, vr, _, _ = bench_workload(wname, "fp64", "auto", prec_list,
                                          small_oracle_sample if (wname == "C5" and want_cpu) else None)
            variants["%s_fp64_%s" % (wname, pr["schedule"])] = dict(
                value=pr["value"], ms_per_step=round(pr["ms_per_step"], 4), kernel_ms=round(pr["kernel_ms"], 4),
                recheck_tracks=pr["summary"]["recheck_tracks"],
                crossings_per_step=pr["crossings_per_step"], launch=pr["params"],
                roofline_frac=roofline(pr, pr["n"], "fp64", wname, pr["schedule"], pr["mode"] == "timeseries",
                                       pr["batched"])["frac"], workload=DESCR[wname])
            variants.update(vr)
    if variants:
        out["variants"] = variants
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
