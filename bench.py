"""Benchmark of the Yee FDTD hot path on one MI355X.

Headline workload: the 512^3 dielectric-scatterer cavity (16-entry material
table, 200 seeded spheres, soft sources on Ex, Ey and Ez, 16 probes), FP32
storage, fused kernel with T steps per HBM pass (by default the fastest of
T = 3, 4, 5 on this grid, measured by fdtd_tune_time_block after the
warm-up; FP32 results do not depend on T).  A "step" is one leapfrog
time step of the whole grid (H and E half-steps with materials, PEC walls,
sources, probes); --steps K steps are timed with HIP events on the solver's
stream, after --warmup W untimed steps, --repeats R times, and the median is
reported.  Inputs are resident in HBM before timing.

Prints one JSON line: G cell-updates/s, the HBM roofline fraction of the
dominant kernel at B_alg = 49 B per cell-update (no temporal reuse counted),
the FP16/BF16-storage rates beside it -- on the headline grid and on the two
precision grids (512^3 and 1024x512x256), each with its relative L2 error
against the FP64 oracle after a stated number of steps from zero fields --
p50/p99 per-solve latency, the serving run, and the CPU oracle timed on the
host cores.
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "G Yee cell-updates/s and % HBM roofline (FP32 vs FP16 store); p50/p99 latency"
# Arrival rate of the serving run, frozen after one calibration on MI355X:
# 0.7 x the saturated mixed throughput (173.2 G cell-updates/s with all 256
# requests queued at once) / the mean work per request (9.81 G) = 12.4 req/s.
SERVING_RATE = 12.4


def kernel_source_hash() -> str:
    """Hash of the kernel sources with comments and blank space removed, so
    that only a change of code retires the stored traffic figures."""
    import re
    h = hashlib.sha256()
    for name in ("yee_fused.hpp", "yee_fused.hip", "yee_fused_cpml.hip", "yee_device.hpp", "yee_internal.hpp",
                 "yee_plain.hip"):
        with open(os.path.join(ROOT, "paper_1301_4539_amd", "csrc", name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, storage: str, T):
    """Physical HBM bytes per launch (FETCH_SIZE + WRITE_SIZE from rocprofv3,
    scaled by the copy-kernel calibration) from the committed summary, if it
    was taken on the current kernel source; else None.  T: steps per pass of
    the fused kernel, or "plain" (bytes per step of the two plain kernels)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        e = d[f"{workload}/{storage}/" + (T if isinstance(T, str) else f"T{T}")]
        if e.get("kernel_hash") != kernel_source_hash():
            return None
        return float(e["bytes_per_launch"])
    except (KeyError, ValueError, OSError):
        return None


def median_rate(solver, cells, n, reps, torch, stream):
    """Median G cell-updates/s over `reps` timed runs of n steps, and the
    per-run rates."""
    runs = [cells * n / time_steps(solver, n, torch, stream) / 1e9 for _ in range(max(1, reps))]
    return float(np.median(runs)), runs


def rel_l2_chunked(a, b):
    """||a-b||_2/||b||_2 over all six components, FP64 accumulation (b is the
    FP64 reference), one z-slab at a time to bound host memory."""
    num = den = 0.0
    for c in range(a.shape[0]):
        for k0 in range(0, a.shape[1], 64):
            x = a[c, k0:k0 + 64].astype(np.float64)
            y = b[c, k0:k0 + 64]
            num += float(np.sum((x - y) ** 2))
            den += float(np.sum(y * y))
    return float(np.sqrt(num / den)) if den > 0 else float("nan")


def time_steps(solver, n, torch, stream):
    solver.synchronize()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    solver.step(n)
    ev1.record(stream)
    torch.cuda.synchronize()
    solver.synchronize()
    return ev0.elapsed_time(ev1) / 1e3


def launches_for(steps_done, n, T, storage):
    """Fused launches of one fdtd_step(n) call from step `steps_done`: full
    blocks from the current step for FP32 storage, blocks ending at absolute
    multiples of T for 16-bit storage."""
    c, s = 0, steps_done
    while n > 0:
        ln = min(T if storage == "fp32" else T - s % T, n)
        s += ln
        n -= ln
        c += 1
    return c


def cpu_baseline(wl, budget_s=15.0):
    """The oracle (FP32 operation-order mode, as it stands) on the host cores,
    over a bounded number of steps of the same grid."""
    import numpy as np
    import oracle
    prob = oracle.Problem.from_workload(wl)
    f = oracle.zero_fields(wl.nx, wl.ny, wl.nz, np.float32)
    t0 = time.perf_counter()
    prob.run_f32(f, 0, 2)
    per = (time.perf_counter() - t0) / 2
    n = int(max(2, min(200, budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    prob.run_f32(f, 2, n)
    dt = time.perf_counter() - t0
    # the same oracle on one thread, over a few more steps
    nt = oracle.threads()
    oracle.set_threads(1)
    try:
        n1 = int(max(1, min(20, 4.0 / max(per * nt, 1e-6))))
        t0 = time.perf_counter()
        prob.run_f32(f, 2 + n, n1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(nt)
    host = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            host = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": wl.cells * n / dt / 1e9, "unit": "G cell-updates/s", "cores": nt,
            "kind": "oracle",
            "sample": f"{wl.nx}x{wl.ny}x{wl.nz} {wl.name}, steps 3-{2 + n} ({n} steps) of the FP32 "
                      f"operation-order oracle from zero fields, {nt} OpenMP threads",
            "one_thread": {"value": wl.cells * n1 / dt1 / 1e9, "steps": n1}, "host_cpu": host}


def serving_leg(rate, n, torch, solo_sample=32):
    """256 requests (dims U{48..320}, 5-60 spheres, 200-3000 steps, FP32 or
    FP16 storage, 8 probes) with Poisson arrivals at `rate`; returns the
    summary of the continuous-batching engine (pipelined ticks), the same
    requests all queued at once (the saturated aggregate rate), and the rate
    of a sample of them solved one at a time (fdtd_step alone, work-weighted)
    for comparison."""
    from paper_1301_4539_amd import fdtd, serve, workload as W
    reqs = W.serving_requests(n=n, rate=rate, seed=1004)
    t0 = time.perf_counter()
    wls = {r.rid: r.workload() for r in reqs}
    print(f"[bench] serving: {n} request payloads built in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    eng = serve.Engine(serve.GpuBackend(wls), budget_bytes=24 << 30, max_slots=64, chunk=48)
    rep = eng.run(reqs)
    out = rep.summary()
    out.update({"rate_req_per_s": rate, "budget_GiB": 24, "max_slots": 64, "chunk_steps": 48,
                "age_step_s": eng.age_step, "max_boost": eng.max_boost,
                "T_by_storage": {"fp32": serve.DEFAULT_T[0], "fp16": serve.DEFAULT_T[1]},
                "mean_work_G": float(np.mean([r.nx * r.ny * r.nz * r.n_steps for r in reqs]) / 1e9)})
    # saturated: every request queued at t = 0
    sat = [dataclasses.replace(r, arrival=0.0) for r in reqs]
    rep_s = serve.Engine(serve.GpuBackend(wls), budget_bytes=24 << 30, max_slots=64, chunk=48).run(sat)
    ss = rep_s.summary()
    # solo: a seeded sample of the requests, each alone on the GPU (fused
    # kernel at its storage's T, fdtd_step over all its steps)
    pick = np.random.default_rng(7).choice(n, size=min(solo_sample, n), replace=False)
    work = secs = 0.0
    for q in pick:
        r = reqs[int(q)]
        w = wls[r.rid]
        sx = fdtd.Solver.from_workload(w, kernel=fdtd.KERNEL_FUSED, time_block=serve.DEFAULT_T[w.storage])
        try:
            secs += time_steps(sx, w.n_steps, torch, torch.cuda.current_stream())
            work += w.cells * w.n_steps
        finally:
            sx.close()
    solo = work / secs / 1e9
    out["saturated"] = {"throughput_G_per_s": ss["throughput_G_per_s"], "makespan_s": ss["makespan_s"],
                        "busy_while_pending": ss["busy_while_pending"], "p50_s": ss["p50_s"], "p99_s": ss["p99_s"],
                        "solo_G_per_s": solo, "solo_sample": len(pick),
                        "ratio_vs_solo": ss["throughput_G_per_s"] / solo}
    return out


WORKLOADS = ("spheres512", "spheres256", "precision512", "precision1024", "cavity402", "sphere402",
             "graded256", "open256")


def make_workload(W, name, storage):
    return {"spheres256": W.spheres256, "spheres512": W.spheres512, "cavity402": W.cavity402,
            "sphere402": W.sphere402, "graded256": W.graded256, "open256": W.open256,
            "precision512": lambda: W.precision512(storage), "precision1024": lambda: W.precision1024(storage)}[name]()


class Fp64Reference:
    """FP64 oracle states of the precision grids after `steps` steps from zero
    fields, computed on the host cores in a background thread while the GPU
    legs run (the oracle's C loops release the interpreter lock)."""

    def __init__(self, W, names, steps):
        import threading
        import oracle
        self.steps = steps
        self.out, self.secs, self.err = {}, {}, None
        self.threads = max(1, oracle.threads() - 2)      # leave cores to the launching thread

        def work():
            try:
                oracle.set_threads(self.threads)         # this thread's own OpenMP setting
                for name in names:
                    wl = make_workload(W, name, W.FP16)
                    prob = oracle.Problem.from_workload(wl)
                    f = oracle.zero_fields(wl.nx, wl.ny, wl.nz)
                    t0 = time.perf_counter()
                    prob.run_f64(f, 0, steps)
                    self.secs[name] = time.perf_counter() - t0
                    self.out[name] = f
            except Exception as e:          # reported by get()
                self.err = e
        self._t = threading.Thread(target=work, daemon=True)
        self._t.start()

    def get(self, name):
        self._t.join()
        if self.err is not None:
            raise self.err
        return self.out[name]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--repeats", type=int, default=5, help="timed runs of --steps steps; the median is reported")
    ap.add_argument("--T", type=int, default=0,
                    help="steps per HBM pass of the fused kernel (1..6; 0 = the library's automatic choice)")
    ap.add_argument("--workload", default="spheres512", choices=WORKLOADS)
    ap.add_argument("--kernel", default="fused", choices=["fused", "plain"],
                    help="kernel family of the timed run")
    ap.add_argument("--tiling", type=int, default=0, help="fused-kernel tile variant (0 = auto, 1..3)")
    ap.add_argument("--zchunk", type=int, default=0, help="planes per z chunk (0 = automatic)")
    ap.add_argument("--tune-steps", type=int, default=60,
                    help="with --T 0 and FP32 storage: steps per candidate T of fdtd_tune_time_block (0 = no tuning)")
    ap.add_argument("--solves", type=int, default=5, help="full solves for the latency percentiles")
    ap.add_argument("--error-steps", type=int, default=250,
                    help="steps from zero fields after which the 16-bit forms are compared with the FP64 oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip every leg but the timed one")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16"],
                    help="storage of the timed run")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the 256-request serving workload (Poisson arrivals, mixed FP32/FP16)")
    ap.add_argument("--serving-rate", type=float, default=SERVING_RATE,
                    help="Poisson arrival rate (requests/s) of the serving run")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (reference for HBM counter scaling)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print("copy calibration: 5 x (1 GiB read + 1 GiB written)", flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported in this build "
              f"(multi-GPU decomposition is design-only).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1301_4539_amd import fdtd, roofline, serve, workload as W

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    storage = {"fp32": W.FP32, "fp16": W.FP16, "bf16": W.BF16}[args.storage]
    wl = make_workload(W, args.workload, storage)
    cells = wl.cells
    T = args.T
    reps = args.repeats
    plain = args.kernel == "plain"
    if wl.cpml and not plain and T > 3:
        T = 2          # CPML layers run fused blocks of at most 3 steps; 2 is the fastest

    s = fdtd.Solver.from_workload(wl, storage=storage, kernel=fdtd.KERNEL_PLAIN if plain else fdtd.KERNEL_FUSED,
                                  time_block=T)
    s.set_tiling(args.tiling, args.zchunk)
    T = s.time_block                     # the automatic choice, if --T 0
    print(f"[bench] workload {wl.name} {wl.nx}x{wl.ny}x{wl.nz}, {args.storage}, T={T}, warmup {args.warmup}, "
          f"{reps} x {args.steps} steps", file=sys.stderr, flush=True)
    # One-time library start-up outside the timed region, whatever --warmup
    # says: a small solver with the same kernel, storage and T loads the code
    # object once.
    wi = W.spheres(40, 40, 40, 2, 2 * T, seed=7, n_sources=1, n_probes=1, rmin=2, rmax=4, name="init", storage=storage)
    si = fdtd.Solver.from_workload(wi, storage=storage, kernel=fdtd.KERNEL_PLAIN if plain else fdtd.KERNEL_FUSED,
                                   time_block=T)
    si.set_tiling(args.tiling, 0)
    si.step(2 * T)
    si.close()
    # Every timed launch does its full work (the zero-tile skip off), so the
    # algorithmic bytes per launch hold for each of them; the skip's effect
    # is measured on its own in latency_ms.
    s.set_zero_skip(False)
    if args.warmup:
        s.step(args.warmup)
    tuning = None
    if (args.T == 0 and args.tune_steps > 0 and not plain and storage == W.FP32 and not wl.cpml
            and wl.spacing is None):
        T, tns = s.tune_time_block(args.tune_steps)
        tuning = {"call": "fdtd_tune_time_block", "steps_each": args.tune_steps, "chosen": T,
                  "ms_per_step": {f"T{k}": v / 1e6 for k, v in tns.items()}}
        print(f"[bench] tuned T: {T} ({', '.join(f'T={k} {v / 1e6:.4f} ms/step' for k, v in tns.items())})",
              file=sys.stderr, flush=True)
    start = s.steps_done()
    value, runs = median_rate(s, cells, args.steps, reps, torch, stream)
    t = cells * args.steps / value / 1e9                     # seconds of the median run
    # a plain "launch" is one step's H and E kernel pair; every timed run
    # starts at a multiple of --steps past the warm-up
    launches = args.steps if plain else launches_for(start, args.steps, T, args.storage)
    b_alg = roofline.algorithmic_bytes(4 if storage == W.FP32 else 2)
    achieved = b_alg * cells * args.steps / t / 1e9          # GB/s, algorithmic
    traffic = measured_traffic(wl.name, args.storage, "plain" if plain else T)
    print(f"[bench] {args.storage}: {value:.2f} G cell-updates/s (median of {reps}: "
          f"{', '.join(f'{r:.1f}' for r in runs)}), {t * 1e3 / launches:.3f} ms per launch",
          file=sys.stderr, flush=True)

    extras = {"runs_G": runs, "T_tuning": tuning}
    if not args.no_extras:
        # FP64 references of the precision grids, computed on the host while
        # the GPU legs below run
        prec_names = ("precision512", "precision1024")
        ref64 = Fp64Reference(W, prec_names, args.error_steps) if args.error_steps > 0 else None

        # FP64 diagnostics (energy, div E, div H, max |value|) of the final
        # state, outside the timed region: cost per call, and its share of a
        # run that asks for them every 250 steps
        s.synchronize()
        d_ms = []
        for _ in range(5):
            t0 = time.perf_counter()
            dg = s.diagnostics()
            d_ms.append((time.perf_counter() - t0) * 1e3)
        dm = float(np.median(d_ms))
        extras["diagnostics"] = {"ms_per_call": dm, "share_every_250_steps": dm / (dm + 250 * t * 1e3 / args.steps),
                                 "energy": dg["energy"], "div_e_max": dg["div_e_max"], "div_h_max": dg["div_h_max"]}
        s.close()

        # per-solve latency: full solves of the workload (a fresh solver each,
        # so its sources run from step 0), from zero fields resident in HBM
        def solve_ms(w, skip, st=storage, tb=T):
            sx = fdtd.Solver.from_workload(w, storage=st, kernel=fdtd.KERNEL_FUSED, time_block=tb)
            try:
                sx.set_zero_skip(skip)
                return time_steps(sx, w.n_steps, torch, stream) * 1e3
            finally:
                sx.close()
        lat = [solve_ms(wl, True) for _ in range(args.solves)]
        lat0 = [solve_ms(wl, False) for _ in range(max(1, args.solves // 2))]
        extras["latency_ms"] = {"solve": f"{wl.n_steps} steps of {wl.name} from zero fields",
                                "p50": float(np.percentile(lat, 50)),
                                "p99": float(np.percentile(lat, 99)), "n": len(lat),
                                "p50_without_zero_skip": float(np.percentile(lat0, 50))}

        def rate(w, st, tb):
            """Median G cell-updates/s of the fused kernel on workload w, storage
            st, time block tb, full launches as in the timed leg."""
            sx = fdtd.Solver.from_workload(w, storage=st, kernel=fdtd.KERNEL_FUSED, time_block=tb)
            try:
                sx.set_zero_skip(False)
                if args.warmup:
                    sx.step(args.warmup)
                return median_rate(sx, w.cells, args.steps, reps, torch, stream)[0]
            finally:
                sx.close()

        # 16-bit storage on the headline grid, each at its fastest T (FP32
        # storage at the timed leg's T, 16-bit storage at T=3), and at
        # matched T (4, and 1 where both forms are bandwidth-bound)
        t16 = serve.DEFAULT_T[W.FP16]
        v16 = rate(wl, W.FP16, t16)
        v16_4 = rate(wl, W.FP16, 4) if t16 != 4 else v16
        v32_4 = value if (T == 4 and storage == W.FP32) else rate(wl, W.FP32, 4)
        v32_1, v16_1 = rate(wl, W.FP32, 1), rate(wl, W.FP16, 1)
        vbf = rate(wl, W.BF16, serve.DEFAULT_T[W.BF16])
        extras["fp16_store"] = {"value": v16, "T": t16, "ratio_vs_fp32": v16 / value,
                                "target_ratio": 1.7,
                                "roofline_frac": roofline.algorithmic_bytes(2) * v16 / roofline.HBM_PEAK_GBPS,
                                "T_fp32": T,
                                "matched_T": {"T4": {"fp32": v32_4, "fp16": v16_4, "ratio": v16_4 / v32_4},
                                              "T1": {"fp32": v32_1, "fp16": v16_1, "ratio": v16_1 / v32_1}},
                                "traffic": measured_traffic(wl.name, "fp16", t16)}
        extras["bf16_store"] = {"value": vbf, "T": serve.DEFAULT_T[W.BF16], "ratio_vs_fp32": vbf / value}
        print(f"[bench] fp16 (T={t16}): {v16:.2f} G cell-updates/s, x{v16 / value:.2f}; matched T=4 "
              f"x{v16_4 / value:.2f}, T=1 x{v16_1 / v32_1:.2f}; bf16 {vbf:.2f}", file=sys.stderr, flush=True)

        # the precision grids: 512^3 and 1024x512x256 (200 spheres, three
        # sources), FP16 and BF16 storage at T=3: rate, roofline fraction at
        # 25 B per cell-update, and relative L2 against the FP64 oracle after
        # --error-steps steps from zero fields (FP32 storage beside them)
        prec = {}
        for name in prec_names:
            entry = {}
            for fname, st, tb in (("fp16", W.FP16, t16), ("bf16", W.BF16, serve.DEFAULT_T[W.BF16]),
                                  ("fp32", W.FP32, T)):
                w = make_workload(W, name, st)
                e = {"T": tb}
                if fname != "fp32":
                    v = rate(w, st, tb)
                    e.update({"value": v, "roofline_frac": roofline.algorithmic_bytes(2) * v / roofline.HBM_PEAK_GBPS})
                if ref64 is not None:
                    sx = fdtd.Solver.from_workload(w, storage=st, kernel=fdtd.KERNEL_FUSED, time_block=tb)
                    try:
                        sx.step(args.error_steps)
                        got = sx.read_fields()
                    finally:
                        sx.close()
                    e["rel_l2_vs_fp64"] = rel_l2_chunked(got, ref64.get(name))
                    del got
                entry[fname] = e
            entry.update({"grid": [w.nx, w.ny, w.nz], "error_after_steps": args.error_steps,
                          "error_from": "zero fields, three Gaussian-modulated soft sources",
                          "oracle_fp64_s": ref64.secs.get(name) if ref64 else None,
                          "oracle_threads": ref64.threads if ref64 else None})
            prec[name] = entry
            print(f"[bench] {name}: fp16 {entry['fp16']['value']:.1f} G/s rel-L2 "
                  f"{entry['fp16'].get('rel_l2_vs_fp64', float('nan')):.2e}, bf16 {entry['bf16']['value']:.1f} G/s "
                  f"rel-L2 {entry['bf16'].get('rel_l2_vs_fp64', float('nan')):.2e}, fp32 rel-L2 "
                  f"{entry['fp32'].get('rel_l2_vs_fp64', float('nan')):.2e}", file=sys.stderr, flush=True)
        if ref64 is not None:
            ref64.out.clear()
        extras["precision"] = prec

        # the energy traced inside the pass (FP64 sums in the Faraday half-step
        # of one level per recorded state): every 250 steps, and every 4 steps
        # (one level of every launch); the automatic T
        def traced_rate(every):
            sx = fdtd.Solver.from_workload(wl, storage=storage, kernel=fdtd.KERNEL_FUSED, time_block=0)
            try:
                sx.set_zero_skip(False)
                sx.set_energy_trace(every)
                tb = sx.time_block
                if args.warmup:
                    sx.step(args.warmup)
                return median_rate(sx, cells, args.steps, reps, torch, stream)[0], tb
            finally:
                sx.close()
        (ve250, te), (ve4, _) = traced_rate(250), traced_rate(4)
        vu = value if te == T else v32_4 if te == 4 else rate(wl, storage, te)   # untraced, same T
        extras["energy_trace"] = {"every_250": ve250, "every_4": ve4, "T": te, "untraced": vu,
                                  "cost_every_4": 1.0 - ve4 / vu}
        print(f"[bench] energy trace (T={te}): every 250 steps {ve250:.2f}, every 4 steps {ve4:.2f} "
              f"G cell-updates/s (untraced {vu:.2f})", file=sys.stderr, flush=True)

        # the 256^3 grid of 40 spheres and one source, FP32 T=4 and FP16 T=3
        w256 = W.spheres256()
        extras["spheres256"] = {"fp32": {"value": rate(w256, W.FP32, 4), "T": 4},
                                "fp16": {"value": rate(w256, W.FP16, t16), "T": t16}}
        # deeper step gathering on the headline grid: FP32 at T = 4 (the
        # automatic choice), 5 and 6 (past the register file), and 16-bit
        # storage at 5 and 6 (slower than 3, but re-encoded less often)
        extras["deep_blocks"] = {
            "fp32": {f"T{tb}": (value if (tb == T and storage == W.FP32) else
                                v32_4 if tb == 4 else rate(wl, W.FP32, tb)) for tb in (4, 5, 6)},
            "fp16": {f"T{tb}": rate(wl, W.FP16, tb) for tb in (5, 6)}}
        print(f"[bench] 256^3: {extras['spheres256']}; deep blocks: {extras['deep_blocks']}",
              file=sys.stderr, flush=True)
        # graded cell sizes (per-index coefficient arrays), FP32, automatic T and tile shape
        wg = W.graded256()

        def graded_rate(st):
            sg = fdtd.Solver.from_workload(wg, storage=st)
            try:
                sg.set_zero_skip(False)
                if args.warmup:
                    sg.step(args.warmup)
                return median_rate(sg, wg.cells, args.steps, reps, torch, stream)[0]
            finally:
                sg.close()
        vg, vg16 = graded_rate(W.FP32), graded_rate(W.FP16)
        extras["graded_spacing"] = {"workload": wg.name, "value": vg, "unit": "G cell-updates/s",
                                    "ratio_vs_spheres256": vg / extras["spheres256"]["fp32"]["value"], "T": 3,
                                    "traffic": measured_traffic(wg.name, "fp32", 3), "fp16": vg16}
        print(f"[bench] graded spacing ({wg.name}): {vg:.2f} G cell-updates/s, FP16 storage {vg16:.2f}",
              file=sys.stderr, flush=True)
        # open space: CPML layers on every face, the fused kernel at the
        # automatic T (2) and T = 1, 3, and the plain kernel family; the plain
        # kernels without layers on the same grid for reference
        def plain_rate(w):
            sp = fdtd.Solver.from_workload(w, kernel=fdtd.KERNEL_PLAIN)
            try:
                n = max(1, args.steps // 5)
                sp.step(10)
                return median_rate(sp, w.cells, n, reps, torch, stream)[0]
            finally:
                sp.close()

        def cpml_rate(w, tb):
            sp = fdtd.Solver.from_workload(w, kernel=fdtd.KERNEL_AUTO if tb == 0 else fdtd.KERNEL_FUSED,
                                           time_block=tb)
            try:
                sp.set_zero_skip(False)
                sp.step(12)
                return median_rate(sp, w.cells, args.steps, reps, torch, stream)[0]
            finally:
                sp.close()
        wo = W.open256()
        vo = cpml_rate(wo, 0)
        vo_t = {f"T{tb}": cpml_rate(wo, tb) for tb in (1, 3)}
        vo_plain = plain_rate(wo)
        vp = plain_rate(w256)
        extras["cpml"] = {"workload": "open256", "value": vo, "unit": "G cell-updates/s", "kernel": "fused", "T": 2,
                          "fused_other_T": vo_t, "plain": vo_plain, "plain_without_layers": vp,
                          "layer": W.CPML_LAYER,
                          "traffic_per_launch": measured_traffic("open256", "fp32", 2),
                          "traffic_per_step_plain": measured_traffic("open256", "fp32", "plain")}
        print(f"[bench] CPML (open256): fused T=2 {vo:.2f} G cell-updates/s, {vo_t}; plain kernels "
              f"{vo_plain:.2f}; plain without layers {vp:.2f}", file=sys.stderr, flush=True)
        # a full solve from host buffers: create (material upload), upload of a
        # host initial state, the solve, read-back of fields and probes
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sx = fdtd.Solver.from_workload(w256, kernel=fdtd.KERNEL_FUSED, time_block=4)
        sx.set_fields(np.zeros((6, w256.nz + 1, w256.ny + 1, w256.nx + 1), np.float32))
        sx.step(w256.n_steps)
        sx.read_fields()
        sx.read_probes(0, w256.n_steps)
        sx.close()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        extras["pcie_inclusive"] = {"value": w256.cells * w256.n_steps / dt / 1e9, "unit": "G cell-updates/s",
                                    "wall_ms": dt * 1e3,
                                    "what": f"spheres256: create + set_fields(host) + {w256.n_steps} steps + "
                                            f"read_fields + read_probes, FP32 T=4"}
        # the paper's case S: a 400-cell perfect-conductor sphere in 402^3, a
        # 1300-step solve from zero fields, with the conductor interior's
        # tiles skipped and without (rates count every cell, as the paper does)
        ws = W.sphere402()
        case_s = {"workload": ws.name, "steps": ws.n_steps}
        for key, st, tb, skip in (("fp32", W.FP32, 4, True), ("fp16", W.FP16, 3, True),
                                  ("fp32_no_skip", W.FP32, 4, False)):
            sx = fdtd.Solver.from_workload(ws, storage=st, kernel=fdtd.KERNEL_FUSED, time_block=tb)
            try:
                sx.set_zero_skip(skip)
                ms = time_steps(sx, ws.n_steps, torch, stream) * 1e3
                sx_stats = sx.tile_stats()
            finally:
                sx.close()
            run, full = sx_stats
            case_s[key] = {"ms": ms, "value": ws.cells * ws.n_steps / ms / 1e6, "T": tb,
                           "tiles_dispatched_share": run / full if full else None}
        extras["case_s"] = case_s
        print(f"[bench] case S: FP32 {case_s['fp32']['ms']:.1f} ms, FP16 {case_s['fp16']['ms']:.1f} ms, "
              f"FP32 without skipping {case_s['fp32_no_skip']['ms']:.1f} ms", file=sys.stderr, flush=True)
        # streaming-copy ceiling on this GPU (torch copy of 2 GiB)
        x = torch.empty(1 << 29, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        extras["copy_GBps"] = 2 * x.numel() * 4 * 10 / (e0.elapsed_time(e1) / 1e3) / 1e9
        del x, y
    else:
        s.close()

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "G cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f32 math, f16 storage", "bf16": "f32 math, bf16 storage"}[args.storage],
        "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "nz": wl.nz, "storage": args.storage,
                   "kernel": args.kernel, "T": None if plain else T, "materials": len(wl.eps_r),
                   "spheres": {"spheres256": 40, "spheres512": 200, "precision512": 200, "precision1024x512x256": 200,
                               "graded256": 40, "open256": 40}.get(wl.name, 0),
                   "sources": len(wl.sources), "probes": len(wl.probes), "zero_skip": False,
                   "repeats": reps, "statistic": "median", "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": roofline.HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / roofline.HBM_PEAK_GBPS,
                     "traffic": traffic,
                     "alg_bytes_per_launch": b_alg * cells * args.steps / launches,
                     "kernel": "h_plain+e_plain<fp32>" if plain else f"yee_fused<T={T},{args.storage}>",
                     "bytes_per_cell_update": b_alg,
                     "avg_launch_ms": t * 1e3 / launches, "launches": launches},
    }
    line.update(extras)
    if not args.no_serving and not args.no_extras:
        line["serving"] = serving_leg(args.serving_rate, args.serving_requests, torch)
        print(f"[bench] serving: {line['serving']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
