"""Reduced-storage error study on the oracle (CPU only).

Runs the oracle's FP64 mode and its reduced-storage emulation (binary16 or
bfloat16 storage, FP32 arithmetic, re-encoding every T steps) side by side
on a seeded dielectric-sphere cavity driven by the Gaussian-modulated soft
sources, and prints the relative L2 error over all six components every
`every` steps.  The GPU kernels are bit-exact with the emulation for the
same T, so these errors are the GPU's.

    python -m oracle.error_study --n 64 --steps 2000 --every 250
"""
import argparse
import json
import sys

import numpy as np

from . import Problem, zero_fields


def study(n=48, steps=2000, every=250, spheres=12, fmts=(1, 2), Ts=(1, 2, 4), seed=1003, sources=3,
          lossless=False):
    sys.path.insert(0, __file__.rsplit("/oracle/", 1)[0])
    from paper_1301_4539_amd import workload as W
    wl = W.spheres(n, n, n, spheres, steps, seed=seed, n_sources=sources, n_probes=0,
                   rmin=max(2, n // 16), rmax=max(3, n // 6), name=f"study{n}")
    if lossless:
        wl.sigma[:] = 0.0
    prob = Problem.from_workload(wl)
    f64 = zero_fields(n, n, n)
    ref = {}
    for s in range(0, steps, every):
        prob.run_f64(f64, s, every)
        ref[s + every] = f64.copy()
    out = {"grid": n, "steps": steps, "spheres": spheres, "lossless": lossless, "rel_l2": {}}
    for fmt in fmts:
        for T in Ts:
            f = zero_fields(n, n, n, np.float32)
            st = prob.quantize_upload(f, fmt)
            errs = []
            for s in range(0, steps, every):
                prob.run_q(f, s, every, fmt, T, st)
                errs.append(W.rel_l2(f, ref[s + every]))
            key = f"{'fp16' if fmt == 1 else 'bf16'}/T{T}"
            out["rel_l2"][key] = errs
            print(key, " ".join(f"{e:.2e}" for e in errs), "sat" if st["flag"][0] else "", flush=True)
    return out


def study_workload(name, steps=2000, every=250, fmts=(1, 2), T=4, log=print):
    """FP64 reference and the reduced-storage emulations of one named
    configuration, advanced side by side (no snapshots kept)."""
    sys.path.insert(0, __file__.rsplit("/oracle/", 1)[0])
    from paper_1301_4539_amd import workload as W
    wl = {"precision512": W.precision512, "precision1024": W.precision1024}[name](W.FP16, n_steps=steps)
    prob = Problem.from_workload(wl)
    f64 = zero_fields(wl.nx, wl.ny, wl.nz)
    runs = []
    for fmt in fmts:
        f = zero_fields(wl.nx, wl.ny, wl.nz, np.float32)
        runs.append((fmt, f, prob.quantize_upload(f, fmt)))
    out = {"workload": name, "grid": [wl.nx, wl.ny, wl.nz], "T": T, "steps": steps, "rel_l2": {}}
    for s in range(0, steps, every):
        prob.run_f64(f64, s, every)
        for fmt, f, st in runs:
            prob.run_q(f, s, every, fmt, T, st)
            key = f"{'fp16' if fmt == 1 else 'bf16'}/T{T}"
            out["rel_l2"].setdefault(key, []).append(W.rel_l2(f, f64))
        log(f"{name} step {s + every}: " + " ".join(f"{k} {v[-1]:.3e}" for k, v in out["rel_l2"].items()))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=48)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=250)
    ap.add_argument("--spheres", type=int, default=12)
    ap.add_argument("--T", default="1,2,4")
    ap.add_argument("--lossless", action="store_true")
    ap.add_argument("--json", default=None)
    ap.add_argument("--workload", default=None, choices=["precision512", "precision1024"])
    a = ap.parse_args()
    if a.workload:
        r = study_workload(a.workload, a.steps, a.every, T=int(a.T.split(",")[-1]),
                           log=lambda m: print(m, flush=True))
    else:
        r = study(a.n, a.steps, a.every, a.spheres, Ts=tuple(int(t) for t in a.T.split(",")),
                  lossless=a.lossless)
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(r, fh, indent=1)


if __name__ == "__main__":
    main()
