#!/usr/bin/env python3
"""Throughput of the particle-decomposition SPH hot path on one MI355X.

Workload: 3D fluid column collapse, 810,448 particles (water lattice
74 x 74 x 148 at dx = 5.4e-3 m in a 1.6 x 0.4 x 0.8 m reflective box),
h = 1.3 dx, rho0 = 1000, c0 = 40, gravity -9.81 z, CFL 0.3, hydrostatic
start.  One step = bucket hash + radix sort + reorder + bucket table
(Section I), local FORCE pass (Section II step e) and the update (step g);
inputs are resident in HBM before the timed region.

Prints one JSON line: particle-updates/s of the FP32 split-precision form
(value) and of the plain FP64 form, the roofline of the dominant kernel
(the FORCE pass's pair kernel) from HIP events the library records around
its launches, and the FP64 CPU
oracle timed on a bounded sample together with the per-field error of both
GPU forms against it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-updates/s (FP32 vs FP64 form, stated error) + adjoint/forward ratio"
# Algorithmic flops of the fluid FORCE pass (FMA = 2; add, mul, div, sqrt = 1),
# the same in both forms: the work of the plain definition of the pass, not
# of the kernel's evaluation of it.  Per candidate source: the position
# difference and the squared distance of the neighbour test.  Per pair within
# 2h: the pair terms written plainly (r, q, F, n, g, the normal velocities,
# the means, the acoustic Riemann solution, v*, E*, the six terms) and the
# accumulation of the six rates.  tests/test_flop_count.py counts them by
# evaluating that plain form with an operation-counting number type and checks
# its values against the oracle's pair terms.
FLOPS_CAND_ITEMS = {"x_j - x_i": 3, "|d|^2": 5}
FLOPS_PAIR_ITEMS = {"r = sqrt(r2)": 1, "q and F(q)": 5, "n = d / r": 3, "g = F n": 3, "u_i, u_j": 10,
                    "means of rho, c, p": 6, "Z": 1, "u* - ubar": 3, "p*": 4, "v*": 12, "E*": 9,
                    "A = 2 w_i w_j": 2, "Phi": 2, "traction p* g": 3, "mdot": 1, "mvdot": 9, "mEdot": 8,
                    "wdot": 10, "accumulate 6 rates": 6}
FLOPS_CAND = {p: sum(FLOPS_CAND_ITEMS.values()) for p in (0, 1)}
FLOPS_PAIR = {p: sum(FLOPS_PAIR_ITEMS.values()) for p in (0, 1)}
PEAK_TFLOPS = {1: 157.3, 0: 78.6}      # MI355X vector FP32 (published) / FP64
EVENT_EVERY = 10


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed steps of the FP64 form (default: --steps)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--only", choices=["fp32", "fp64", "both"], default="both")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward ratio leg")
    ap.add_argument("--no-share", action="store_true", help="skip the 8M + 2M share pass-set leg")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint leg and print its fields (for profiling it)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (scale for HBM counters)")
    return ap.parse_args()


COUNTERS = os.path.join(ROOT, "profiles", "pair_force_column_counters.md")
PAIR_SOURCES = ("paper_2310_03596_amd/csrc/interact.hip", "paper_2310_03596_amd/csrc/pair.hpp",
                "paper_2310_03596_amd/csrc/common.hpp")


def pair_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in PAIR_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(prec: int):
    """HBM bytes per FORCE launch from the committed counter summary (FETCH_SIZE
    + WRITE_SIZE, each scaled by the same counter on a copy of known size), or
    None when the summary is missing or the kernel sources changed since."""
    try:
        with open(COUNTERS) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    kv = {}
    for ln in lines:
        if ln.startswith("    ") and ":" in ln:
            k, v = ln.strip().split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != pair_source_hash():
        return None
    v = kv.get("traffic_bytes_per_launch_" + ("fp32" if prec == 1 else "fp64"))
    return int(v) if v else None


def time_forms(wl, plan, warmup):
    """Time each (prec, steps) of `plan` in order on its own Sim of `wl`.
    Every Sim is built and warmed up (`warmup` untimed steps) before the
    first timed step, and the work counts are taken after the last, so the
    timed runs follow one another with no host work between them and the
    GPU stays at its sustained clocks (it drops them within milliseconds of
    going idle, and a short timed run would otherwise measure the ramp)."""
    import torch
    from paper_2310_03596_amd.sim import Sim

    sims = {prec: Sim(wl, prec) for prec, _ in plan}
    for prec, _ in plan:
        for _ in range(warmup):
            sims[prec].step()
    torch.cuda.synchronize()
    timed = {}
    for prec, steps in plan:
        sim = sims[prec]
        # HIP events bracket the pair kernel of the FORCE call (recorded by the
        # library around that launch alone: sph_set_pair_events) in every
        # EVENT_EVERY-th timed step (an event pair costs a few microseconds of
        # queue time, so timing every launch would slow the steps being timed)
        sampled = list(range(0, steps, EVENT_EVERY))
        evs = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in sampled}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            sim.step(force_events=evs.get(k))
        torch.cuda.synchronize()
        timed[prec] = (time.perf_counter() - t0, evs)
    out = {}
    for prec, steps in plan:
        sim = sims[prec]
        wall, evs = timed[prec]
        force_ms = sum(a.elapsed_time(b) for a, b in evs.values()) / max(len(evs), 1)
        cand, pairs = sim.count_pairs()
        flops = cand * FLOPS_CAND[prec] + pairs * FLOPS_PAIR[prec]
        out[prec] = {
            "value": wl.n * steps / wall,
            "ms_per_step": 1e3 * wall / steps,
            "force_ms": force_ms,
            "candidates": cand,
            "pairs": pairs,
            "flops_per_launch": flops,
            "force_tflops": flops / (force_ms * 1e-3) / 1e12,
            "pair_evals_per_s": pairs / (force_ms * 1e-3),
            "candidates_per_s": cand / (force_ms * 1e-3),
            "diag": sim.diagnostics().tolist(),
        }
    del sims
    torch.cuda.empty_cache()
    return out


def other_workloads_leg():
    """Step throughput of the 8,000-particle cube (10 steps, launched one by
    one and replayed from a captured graph), the
    3,987,920-particle elastic-plastic cylinder (two interaction loops per
    step: GRADIENT, stress stage, FORCE; 20 steps) and the 6,668,204-particle
    hypervelocity impact (same loops, Mie-Gruneisen EOS; 20 steps from the
    first contact) in both forms."""
    import torch

    import sph_synth as S
    from paper_2310_03596_amd.sim import Sim

    from paper_2310_03596_amd.graph import StepGraph

    out = {}
    for name, make, steps in (("cube_8000", S.c1_cube, 10), ("cylinder_3987920", S.c3_cylinder, 20),
                              ("hvi_6668204", S.c6_hvi, 20)):
        wl = make()
        out[name] = {}
        for prec, tag in ((1, "fp32_split"), (0, "fp64")):
            sim = Sim(wl, prec)
            for _ in range(2):
                sim.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                sim.step()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            out[name][tag] = {"steps": steps, "ms_per_step": 1e3 * wall / steps,
                              "particle_updates_per_s": wl.n * steps / wall}
            if name == "cube_8000":
                # the launch-bound cube again, its steps replayed from one captured graph
                g = StepGraph(sim, steps=steps)
                g.replay()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.replay()
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                out[name][tag]["graph_ms_per_step"] = 1e3 * wall / steps
                out[name][tag]["graph_particle_updates_per_s"] = wl.n * steps / wall
                del g
            del sim
        del wl
        torch.cuda.empty_cache()
    return out


def adjoint_leg(prec, reps=5):
    """Adjoint/forward time ratio on the 250,047-particle box: 50 fixed-dt
    steps with checkpoints every 10 (forward: the rollout from the initial
    state already on the device), then the reverse pass (recompute of every
    segment, with its bucket tables, + reverse kernels).  Best of `reps`.
    Also returns the gradient (dJ/dv0, dJ/dc0) of the last round."""
    import torch

    import sph_synth as S
    from paper_2310_03596_amd.adjoint import KineticEnergyRollout

    wl = S.c5_box()
    best = None
    grad = None
    for _ in range(reps + 1):      # the first round warms up
        ro = KineticEnergyRollout(wl, prec, wl.extra["steps"], wl.extra["ckpt"], wl.extra["dt"])
        ro.prepare(wl.v, wl.params["c0"])   # host-to-device upload of the initial state
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ro.run()
        t1 = time.perf_counter()
        grad = ro.backward(1.0)
        t2 = time.perf_counter()
        cur = (t1 - t0, t2 - t1)
        best = cur if best is None or sum(cur) < sum(best) else best
        del ro
    fwd, bwd = best
    return {"n_particles": wl.n, "steps": wl.extra["steps"], "checkpoint_every": wl.extra["ckpt"],
            "forward_s": fwd, "backward_s": bwd, "adjoint_over_forward": bwd / fwd,
            "form": "FP32 split" if prec == 1 else "FP64"}, grad


def adjoint_error(g32, g64):
    """FP32-split gradient against the FP64 one: max-norm and RMS of the
    difference over those of the FP64 gradient, and the relative c0 error."""
    import numpy as np
    (v32, c32), (v64, c64) = g32, g64
    return {"dJ_dv0_maxnorm_rel": float(np.abs(v32 - v64).max() / np.abs(v64).max()),
            "dJ_dv0_rms_rel": float(np.sqrt(np.mean((v32 - v64) ** 2) / np.mean(v64 ** 2))),
            "dJ_dc0_rel": float(abs(c32 - c64) / abs(c64))}


def share_leg(reps=5):
    """One GPU's share of a 16-GPU decomposition (8M local + 2M remote), FP32:
    hash/sort/tables of both arrays, communication hash + compaction, payload
    packing, local-local and local-remote FORCE passes, timed per pass set."""
    import torch

    import sph_synth as S
    from paper_2310_03596_amd.sim import SharePass

    out = {}
    for layout in ("slab", "mixed"):
        loc, rem = S.c4_share(layout)
        sp = SharePass(loc, rem, 1)
        sp.run()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        t_b = t_ll = t_lr = t_rs = 0.0
        t0 = time.perf_counter()
        for _ in range(reps):
            ev[0].record()
            sp.build()          # both arrays from the generator's order
            ev[1].record()
            sp.mark()
            sp.pack()
            ev[2].record()
            sp.interact_local()
            ev[3].record()
            sp.interact_remote()
            ev[4].record()
            torch.cuda.synchronize()
            t_b += ev[0].elapsed_time(ev[1])
            t_ll += ev[2].elapsed_time(ev[3])
            t_lr += ev[3].elapsed_time(ev[4])
        wall = (time.perf_counter() - t0) / reps
        nb = int(sp.nb.cpu()[0])
        # step a as at every step of a run: both arrays re-sorted from the
        # order the previous sort left them in
        for _ in range(reps):
            ev[0].record()
            sp.resort()
            ev[1].record()
            torch.cuda.synchronize()
            t_rs += ev[0].elapsed_time(ev[1])
        out[layout] = {"local": loc.n, "remote": rem.n, "boundary": nb, "pass_set_ms": 1e3 * wall,
                       "local_particle_updates_per_s": loc.n / wall, "local_local_ms": t_ll / reps,
                       "local_remote_ms": t_lr / reps, "build_ms_from_generator_order": t_b / reps,
                       "build_ms_resort": t_rs / reps}
        del sp
        torch.cuda.empty_cache()
    return out


def decomposition_leg(steps=200, period=20):
    """The column as two GPUs' shares on one device (FP32 split): steps a-g
    for both sets with a balancing round every `period` steps.  Exchange-set
    fraction (both sets' boundary particles over all particles) after each
    round, for a random and a slab (median x) initial split; time per step
    of both sets, balancing included."""
    import numpy as np
    import torch

    import sph_synth as S
    from paper_2310_03596_amd import SPH_FP32_SPLIT
    from paper_2310_03596_amd.decomp import TwoSets

    wl = S.c2_column()
    out = {"particles": wl.n, "steps": steps, "balance_every": period}
    splits = {"random": np.random.default_rng(93).random(wl.n) < 0.5,
              "slab": wl.x[:, 0] > np.median(wl.x[:, 0])}
    for name, owner in splits.items():
        ts = TwoSets(wl, owner, SPH_FP32_SPLIT, period=period)
        fr = []
        for k in range(steps):
            ts.step()
            if k == 0 or (k + 1) % period == 0:
                fr.append(round(ts.exchange_fraction(), 5))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ts.step()
        torch.cuda.synchronize()
        out[name] = {"exchange_fraction_first_step_then_every_round": fr,
                     "ms_per_step_both_sets": (time.perf_counter() - t0) * 1e3 / steps}
    return out


def balance_leg(reps=3, types=False):
    """One round of the swap heuristic (Section III.A) between an 8M and a 2M
    particle set (the mixed share and its partner), FP32 split: both centres,
    both balancing hashes, both selections, the swap.  Fresh sets each
    repetition (a round changes them); the first round is the warm-up.  With
    types: two particle types (a bead of type 1 in type 0), each balanced
    towards its biased centres (Section III.B)."""
    import numpy as np
    import torch

    import sph_synth as S
    from paper_2310_03596_amd.balance import BalancePair, BalanceTypesPair

    a, b = S.c4_share("mixed")
    if types:
        lo = np.asarray(a.grid["origin"], dtype=np.float64)
        hi = lo + np.asarray(a.grid["dims"]) * a.grid["cell"]
        c, r = lo + 0.7 * (hi - lo), 0.25 * float((hi - lo).min())
        ta, tb = S.particle_types(a.x, c, r), S.particle_types(b.x, c, r)
    times, ks = [], []
    for r in range(reps + 1):
        bp = BalanceTypesPair(a, b, ta, tb, 2, 1) if types else BalancePair(a, b, 1)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        bp.centroids()
        ev[1].record()
        bp.hashes()
        ev[2].record()
        bp.selections()
        ev[3].record()
        bp.swap()
        ev[4].record()
        torch.cuda.synchronize()
        if r > 0:
            times.append([ev[q].elapsed_time(ev[q + 1]) for q in range(4)])
            ks.append(bp.k[0].cpu().tolist() if types else int(bp.k.cpu()[0]))
        del bp
    t = [sum(x[q] for x in times) / len(times) for q in range(4)]
    tot = sum(t)
    out = {"particles": a.n + b.n, "k_swapped": ks[0], "round_ms": tot, "centroids_ms": t[0], "hashes_ms": t[1],
           "selections_ms": t[2], "swap_ms": t[3], "particles_per_s": (a.n + b.n) / (tot * 1e-3)}
    if types:
        out["types"] = 2
        out["particles_of_type_1"] = int(ta.sum() + tb.sum())
    return out


def cpu_leg(wl, budget_s):
    """FP64 oracle from the initial state for a bounded number of steps, then
    both GPU forms on the same dt schedule; per-field error by particle id."""
    import numpy as np
    import torch
    from oracle import cpu
    from paper_2310_03596_amd.sim import Sim

    st = cpu.State.from_workload(wl)
    t0 = time.perf_counter()
    dts1, _ = cpu.run(wl.params, wl.grid, st, 1)
    t1 = time.perf_counter() - t0
    more = max(0, min(149, int(budget_s / max(t1, 1e-3)) - 1))
    t0 = time.perf_counter()
    # continuing run: its first dt is the EOS-stage dt of the current state,
    # which equals the previous step's next dt, so the schedule is unbroken
    dts2, _ = cpu.run(wl.params, wl.grid, st, more) if more else (np.zeros(0), None)
    tm = time.perf_counter() - t0
    nsteps = 1 + more
    dts_all = np.concatenate([dts1, dts2])
    t_total = t1 + tm
    ref = st.by_id()
    # the same oracle on one host thread, a few steps from the initial state
    threads = cpu.num_threads()
    cpu.set_threads(1)
    s1 = cpu.State.from_workload(wl)
    n1 = max(1, min(3, int(budget_s / 3 / max(t1 * threads, 1e-3))))
    t0 = time.perf_counter()
    cpu.run(wl.params, wl.grid, s1, n1)
    t_one = time.perf_counter() - t0
    cpu.set_threads(threads)
    errs = {}
    for name, prec in (("fp32_split", 1), ("fp64", 0)):
        sim = Sim(wl, prec)
        sim.run(nsteps, dts=dts_all)
        torch.cuda.synchronize()
        g = sim.state_by_id()
        e = {}
        for f, gf in (("x", "x"), ("v", "v"), ("rho", "rho"), ("E", "E"), ("m", "m")):
            a = np.asarray(g[gf], dtype=np.float64)
            b = np.asarray(getattr(ref, f), dtype=np.float64)
            e[f] = float(np.abs(a - b).max() / np.abs(b).max())
        B = wl.params["rho0"] * wl.params["c0"] ** 2
        e["p_over_rho0c0^2"] = float(np.abs(g["p"] - ref.p).max() / B)
        errs[name] = e
    return {
        "value": wl.n * nsteps / t_total,
        "unit": "particle-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {nsteps} steps of the same 810448-particle column from its initial state "
                  f"(FP64 C oracle, OpenMP over targets), {t_total:.1f} s",
        "steps": nsteps,
        "value_1_thread": wl.n * n1 / t_one,
        "sample_1_thread": f"first {n1} steps on one host thread, {t_one:.1f} s",
    }, {"steps": nsteps, "max_abs_err_over_max_abs_ref": errs}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU exchange is not built in this path", file=sys.stderr)
        sys.exit(2)
    import torch

    import sph_synth as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.adjoint_only:
        a32, g32 = adjoint_leg(1)
        a64, g64 = adjoint_leg(0)
        print(json.dumps({"adjoint": {"fp32_split": a32, "fp64": a64,
                                      "fp32_gradient_error_vs_fp64": adjoint_error(g32, g64)}}), flush=True)
        return
    wl = S.c2_column()
    out = {}
    res = {}
    # The other GPU legs run first and the column's two forms last, back to
    # back (the plain FP64 form, then the FP32 form, the headline; see
    # time_forms).
    legs = {}
    if not args.no_share:
        legs["other_workloads"] = other_workloads_leg()
    if not args.no_adjoint:
        a32, g32 = adjoint_leg(1)
        a64, g64 = adjoint_leg(0)
        legs["adjoint"] = {"fp32_split": a32, "fp64": a64, "fp32_gradient_error_vs_fp64": adjoint_error(g32, g64)}
        legs["adjoint_forward_ratio"] = a32["adjoint_over_forward"]
    if not args.no_share:
        legs["share_pass"] = share_leg()
        legs["balance_round"] = balance_leg()
        legs["balance_types_round"] = balance_leg(types=True)
        legs["decomposition"] = decomposition_leg()
    plan = []
    if args.only in ("fp64", "both"):
        plan.append((0, args.fp64_steps or args.steps))
    if args.only in ("fp32", "both"):
        plan.append((1, args.steps))
    res = time_forms(wl, plan, args.warmup)
    main_prec = 1 if 1 in res else 0
    r = res[main_prec]
    out.update({
        "metric": METRIC,
        "value": r["value"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if main_prec == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": "fluid column collapse 3D: 74x74x148 water lattice, dx=5.4e-3 m, "
                               "box 1.6x0.4x0.8 m, h=1.3dx, rho0=1000, c0=40, g=-9.81 z, CFL 0.3",
                   "n_particles": wl.n, "grid": wl.grid["dims"],
                   "form": "FP32 split (bucket index + float offset, pair sums accumulated in FP64; x, E in FP64)"
                   if main_prec == 1 else "plain FP64"},
        "roofline": {"bound": "alu", "kernel": "FORCE pass pair kernel (k_pairs, staging excluded)",
                     "achieved": r["force_tflops"], "peak": PEAK_TFLOPS[main_prec], "unit": "TFLOP/s",
                     "frac": r["force_tflops"] / PEAK_TFLOPS[main_prec], "traffic": recorded_traffic(main_prec),
                     "avg_launch_ms": r["force_ms"], "flops_per_launch": r["flops_per_launch"],
                     "units_per_launch": {"candidates": r["candidates"], "pairs_within_2h": r["pairs"]}},
        "pair_evals_per_s": r["pair_evals_per_s"],
        "candidates_per_s": r["candidates_per_s"],
    })
    if 0 in res and 1 in res:
        out["fp64_form"] = {"value": res[0]["value"], "ms_per_step": res[0]["ms_per_step"],
                            "steps": args.fp64_steps or args.steps, "force_ms": res[0]["force_ms"],
                            "force_tflops": res[0]["force_tflops"],
                            "frac_of_fp64_peak": res[0]["force_tflops"] / PEAK_TFLOPS[0]}
        out["fp32_over_fp64"] = res[1]["value"] / res[0]["value"]
    out.update(legs)
    if args.calib_copy_mb > 0:
        nbytes = args.calib_copy_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = nbytes
    if not args.no_cpu:
        cb, err = cpu_leg(wl, args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["error_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
