"""Per-field error of both GPU forms against the FP64 oracle on the 810,448-
particle column after 1, 100 and 1000 steps (not collected by pytest; run as
``python tests/error_table.py --out FILE``; needs a GPU).

The oracle runs first, in chunks so that it reports progress, and records its
dt schedule; each GPU form then replays that schedule, so dt noise is not
counted as error.  Particles are matched by id.  For every field: max-norm
error over max |ref| and RMS error over RMS ref.  A one-thread oracle timing
of the first step is taken in a child process before the GPU is touched.
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import subprocess
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

FIELDS = ("x", "v", "m", "rho", "p", "E")


def one_thread_rate():
    code = ("import time, sph_synth as S; from oracle import cpu; wl = S.c2_column(); "
            "st = cpu.State.from_workload(wl); t = time.perf_counter(); cpu.run(wl.params, wl.grid, st, 1); "
            "print(wl.n / (time.perf_counter() - t), cpu.num_threads())")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True,
                         timeout=600, check=True)
    rate, thr = out.stdout.split()
    return float(rate), int(thr)


def errors(got: dict, ref) -> dict:
    e = {}
    for f in FIELDS:
        a = np.asarray(got[f], dtype=np.float64)
        b = np.asarray(getattr(ref, f), dtype=np.float64)
        d = a - b
        e[f] = {"max_rel": float(np.abs(d).max() / np.abs(b).max()),
                "rms_rel": float(np.sqrt((d * d).mean() / (b * b).mean()))}
    return e


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--snap", default="1,100,1000")
    ap.add_argument("--chunk", type=int, default=20)
    args = ap.parse_args()
    snaps = [int(s) for s in args.snap.split(",")]

    import sph_synth as S
    from oracle import cpu

    rate1, thr1 = one_thread_rate()
    print(f"oracle one thread: {rate1:.3e} particle-updates/s ({thr1} thread)", flush=True)

    wl = S.c2_column()
    st = cpu.State.from_workload(wl)
    dts, refs = [], {}
    done, t_or = 0, 0.0
    for target in snaps:
        while done < target:
            k = min(args.chunk, target - done)
            t0 = time.perf_counter()
            d, _ = cpu.run(wl.params, wl.grid, st, k)
            t_or += time.perf_counter() - t0
            dts.append(d)
            done += k
            print(f"oracle step {done}/{snaps[-1]} ({t_or:.1f} s)", flush=True)
        refs[target] = st.by_id().copy()
    dts = np.concatenate(dts)

    import torch

    from paper_2310_03596_amd.sim import Sim

    # control: the FP64 form from positions moved by about one FP32 rounding of
    # a bucket offset (|delta| <= 5e-10 m), to separate the flow's own
    # sensitivity from the FP32 form's arithmetic
    wlp = copy.copy(wl)
    wlp.x = wl.x + np.random.default_rng(6).uniform(-5e-10, 5e-10, size=wl.x.shape)
    table = {}
    for name, prec, w in (("fp32_split", 1, wl), ("fp64", 0, wl), ("fp64_x_perturbed_5e-10", 0, wlp)):
        sim = Sim(w, prec)
        done = 0
        table[name] = {}
        for target in snaps:
            sim.run(target - done, dts=dts[done:target])
            done = target
            torch.cuda.synchronize()
            table[name][str(target)] = errors(sim.state_by_id(), refs[target])
            print(f"{name} step {target}: " + ", ".join(
                f"{f} {v['max_rel']:.2e}/{v['rms_rel']:.2e}" for f, v in table[name][str(target)].items()),
                flush=True)
        del sim
    res = {"workload": f"fluid column, {wl.n} particles", "steps": snaps,
           "oracle_threads": cpu.num_threads(), "oracle_particle_updates_per_s": wl.n * snaps[-1] / t_or,
           "oracle_one_thread_particle_updates_per_s": rate1, "dt_first": float(dts[0]),
           "dt_last": float(dts[-1]), "errors": table,
           "columns": "max_rel = max|gpu - oracle| / max|oracle|; rms_rel = rms(gpu - oracle) / rms(oracle)"}
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print("done", flush=True)


if __name__ == "__main__":
    main()
