"""Throughput of the driven-lid-cavity time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--exec stream|persistent|graph|resident] [--solver sor|multigrid]
                    [--warm-start L] [--no-cpu] [--no-extras | --extras KEY,...]

A step is one SSPRK(5,4) step of the whole hot path (five stages, each with
transport RHS + stage combination, compact-Poisson SOR solve to tolerance,
Thom walls).  The headline workload is the 1024 x 1024 cavity at Re = 1e4,
started from rest, FP64, Poisson tolerance 1e-10, solved by the paper's
relaxation (four-colour SOR), timed over 1000 steps (the workload's run
length) after 5 warm-up steps.  Inputs are resident in HBM when timing starts.
Extras (same JSON line): the same workload with the multigrid solver, in
persistent execution and with resident solves; the 1024 x 1024 Re = 3e4
cavity in FP64 and in mixed precision (the same 200 steps); the 4096 x 4096
Re = 3e4 noise-start cavity (FP64 SOR and mixed SOR for the same two steps
after one warm-up step, with the rooflines of both sweep kernels at that size,
and FP64 multigrid); the coupled mode; the six-cavity Reynolds sweep (256^2
... 1024^2) and sixteen 128^2 cavities batched in one persistent launch per
stage (hipGraph, tile shape from the autotuner) against a stream per cavity
and the same cavities run one by one.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mcell-steps/s at 1024² (FP64 vs mixed+refine), achieved HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
BYTES_PER_SWEEP_NODE = {0: 24.0, 1: 12.0}   # FP64 / FP32: psi in, rhs in, psi out
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sor_traffic.json")
EXEC = {"stream": 0, "persistent": 1, "graph": 2, "resident": 3}


def _kernel_source_hash() -> str:
    """Hash of the code a sweep launch runs: the kernel source up to the end
    of the sweep kernel's definition (everything it can refer to) and the
    host function that launches it, with comments, blank lines and trailing
    blanks left out, so that only a change to that code invalidates the
    recorded counters (the file has no string literal holding a comment
    marker)."""
    path = os.path.join(ROOT, "paper_0809_3098_amd", "csrc", "cavity_kernels.hip")
    with open(path, encoding="utf-8") as f:
        lines = f.read().splitlines()
    k = next(i for i, ln in enumerate(lines) if "void k_sor(" in ln)
    end_a = next(i for i in range(k, len(lines)) if lines[i] == "}")
    b = next(i for i, ln in enumerate(lines) if ln.startswith("hipError_t sor_launch(")) - 1
    end_b = next(i for i in range(b, len(lines)) if lines[i] == "}")
    text = "\n".join(lines[:end_a + 1] + lines[b:end_b + 1])
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    code = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
    return hashlib.sha256("\n".join(ln for ln in code if ln).encode()).hexdigest()[:16]


def _traffic(key: str):
    """L2-miss bytes per sweep launch from committed PMC counters, if the sweep
    kernel's code is still the one they were taken on."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_source_sha256_16") != _kernel_source_hash():
        return None
    return rec.get("l2miss_bytes_per_launch")


def _cpu_baseline(n, re, steps):
    from oracle.cavity_oracle import CavityOracle
    cores = os.cpu_count() or 1
    o = CavityOracle(n, re, workers=cores)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return {"value": round(n * n * steps / dt / 1e6, 4), "unit": "Mcell-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps} steps of the {n}x{n} Re={re:g} cavity from rest; exact DST "
                      f"Poisson per stage (scipy.fft workers={cores}), NumPy elementwise on 1 "
                      f"thread; {dt:.1f} s"}


def _timed_steps(torch, cav, steps, warmup):
    dev = torch.device("cuda:0")
    if warmup:
        cav.step(warmup, want_stats=False)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    stats = cav.step(steps, want_stats=True) if steps else None
    torch.cuda.synchronize(dev)
    return time.perf_counter() - t0, stats


def _sweep_roofline(torch, cav, stream, launches, arith, key):
    """Roofline of the sweep kernel, from its average launch duration
    event-timed on the stream it runs on.

    A launch of S sweeps must move psi in, F in and psi out once (24 B per
    interior node in FP64, 12 B in FP32): those bytes over the launch time,
    against the 8 TB/s HBM peak, are ``achieved`` and ``frac``.  ``effective``
    counts 24 (12) B per node for each of the S sweeps, the per-sweep figure
    of a stencil sweep that reads and writes every field once; it exceeds what
    a launch moves because the S sweeps run on chip.  ``traffic`` is the
    L2-miss bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by the same
    counters of a 1 GiB copy) from the committed counter record of this
    kernel source, else null; at 1024^2 these are mostly served by the
    Infinity Cache, at 4096^2 by HBM."""
    tun = cav.tuning(0)
    s = tun["sweeps_per_launch32"] if arith else tun["sweeps_per_launch"]
    n = cav.params[0].n
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    cav.relax(2 * s, arith=arith)  # warm the scratch buffers
    ev0.record(stream)
    done, _ = cav.relax(launches * s, arith=arith)
    ev1.record(stream)
    ev1.synchronize()
    per_launch_s = ev0.elapsed_time(ev1) / 1e3 / (done // s)
    moved = BYTES_PER_SWEEP_NODE[arith] * (n - 2) ** 2
    achieved = moved / per_launch_s / 1e9
    eff = moved * s / per_launch_s / 1e9
    if arith:
        kern = f"k_sor<float,{tun['tile_x32']},{tun['tile_y32']},{s},{tun['threads32']}>"
    else:
        kern = f"k_sor<double,{tun['tile_x']},{tun['tile_y']},{s},{tun['threads']}>"
    traffic = _traffic(key)
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "traffic_kind": "L2-miss bytes per launch (Infinity Cache and HBM), rocprofv3 "
                           "FETCH_SIZE + WRITE_SIZE scaled by a 1 GiB copy",
           "kernel": kern, "n": n, "sweeps_per_launch": s, "bytes_per_launch": moved,
           "avg_launch_us": round(per_launch_s * 1e6, 3),
           "effective": {"bytes_per_launch": moved * s, "gbs": round(eff, 1),
                         "frac": round(eff / HBM_PEAK_GBS, 4),
                         "per": f"{int(BYTES_PER_SWEEP_NODE[arith])} B per node for each of "
                                f"the {s} sweeps of a launch"}}
    if traffic:
        out["traffic_gbs"] = round(traffic / per_launch_s / 1e9, 1)
        out["traffic_frac"] = round(traffic / per_launch_s / 1e9 / HBM_PEAK_GBS, 4)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the headline workload's whole run (1000 steps from rest), after 5 warm-up steps
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cavity1024_re1e4_fp64")
    ap.add_argument("--exec", default="stream", choices=sorted(EXEC))
    ap.add_argument("--warm-start", type=int, default=0,
                    help="start of each stage's solve: 0 default, 1 the previous stage's "
                         "psi, 2..8 extrapolation through that many steps")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="override the workload's precision (the headline run only)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip mixed and batched lines")
    ap.add_argument("--extras", default="all",
                    help="comma-separated subset of the extra lines: multigrid, mixed_head, "
                         "persistent, "
                         "resident, re3e4, n4096, coupled, re_sweep6_fp64, re_sweep6_mixed, "
                         "re_scan16_small_fp64 (default all)")
    ap.add_argument("--poisson-tol", type=float, default=None,
                    help="Poisson tolerance of the headline run (default: the workload's)")
    ap.add_argument("--solver", default="sor", choices=["sor", "multigrid"],
                    help="Poisson solver of the headline workload")
    ap.add_argument("--set-tuning", default="", metavar="KEY=VALUE,...",
                    help="launch configuration of the headline cavity (cavity_set_tuning "
                         "fields, e.g. check_every=64,inner_sweeps=300)")
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--relax-launches", type=int, default=200)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a cold 1 GiB device copy (torch), the known-size kernel the "
                         "HBM counters of a profiling run are scaled by")
    ap.add_argument("--extra-steps", type=int, default=10)
    ap.add_argument("--compare-steps", type=int, default=200,
                    help="steps of the FP64 and mixed runs of the 1024^2 Re 3e4 workload "
                         "(after --warmup steps)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON-lines cache of the autotuner (default: none, tune every run)")
    ap.add_argument("--log-run", default=None, metavar="JSONL",
                    help="instead of the bench: run the 4096^2 Re 3e4 noise-start cavity "
                         "(mixed, multigrid) for --log-steps steps, one monitor line per step")
    ap.add_argument("--log-steps", type=int, default=2000)
    ap.add_argument("--grid-study", default=None, metavar="JSONL",
                    help="instead of the bench: run the coarse-grid cavities of the grid "
                         "dependence study towards a steady state, one line per chunk")
    ap.add_argument("--study-workload", default="grid_dependence",
                    help="workload of --grid-study: grid_dependence (220^2, 300^2), "
                         "grid_dependence_1024, steady_table_1024 (Sec. 4 production runs)")
    ap.add_argument("--study-members", default=None,
                    help="comma-separated indices of the workload's members to run")
    ap.add_argument("--checkpoint", default=None, metavar="DIR",
                    help="save each cavity's psi, omega and step count there at its end")
    ap.add_argument("--resume", default=None, metavar="DIR",
                    help="continue each cavity from its state saved there (if any)")
    ap.add_argument("--study-steps", type=int, default=200000)
    ap.add_argument("--study-chunk", type=int, default=1000)
    ap.add_argument("--study-seconds", type=float, default=240.0,
                    help="wall-clock limit per cavity of the grid study")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): every workload here is "
              f"measured on a single MI355X.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0809_3098_amd import inputs
    from paper_0809_3098_amd.cavity import (CAVITY_FP64, CAVITY_MIXED, CAVITY_SOLVER_MG,
                                            CAVITY_WARM_LEVELS_FP64, CAVITY_WARM_LEVELS_MIXED,
                                            Cavity, Params)
    from paper_0809_3098_amd.workloads import WORKLOADS

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    if args.log_run:
        wl = WORKLOADS["cavity4096_re3e4_mixed_noise"]
        w0 = inputs.noise_omega0(wl["n"], wl["noise_amplitude"], wl["noise_seed"])
        cav = Cavity(Params(n=wl["n"], re=wl["re"], poisson_tol=wl["tol"],
                            precision=CAVITY_MIXED), device="cuda:0", stream=stream,
                     omega0=[w0])
        cav.set_tuning(solver=CAVITY_SOLVER_MG)
        t0 = time.perf_counter()
        with open(args.log_run, "w") as f:
            for k in range(args.log_steps):
                st = cav.step(1)[0]
                rec = {key: st[key] for key in ("step", "t", "res_psi", "res_omega",
                                                "domega_inf_over_dt", "ke", "last_resid_inf",
                                                "sweeps_last_step", "floor_limited", "status")}
                rec["wall_s"] = round(time.perf_counter() - t0, 3)
                f.write(json.dumps(rec) + "\n")
                if (k + 1) % 100 == 0:
                    f.flush()
                    print(json.dumps(rec), flush=True)
        cav.close()
        return

    if args.grid_study:
        # one handle per cavity, so that a cavity whose run blows up (a possible
        # outcome on a coarse grid) ends only its own run
        from paper_0809_3098_amd.cavity import CAVITY_ENONFINITE, CavityError
        wl = WORKLOADS[args.study_workload]
        members = wl["members"]
        if args.study_members:
            members = [members[int(k)] for k in args.study_members.split(",")]
        with open(args.grid_study, "a" if args.resume else "w") as f:
            for r, m in members:
                tag = f"n{m}_re{int(r)}"
                resume = None
                if args.resume:
                    # a state saved by an earlier run of this cavity: psi and omega
                    # after `step` steps, adopted as they are (cavity_create resume=1)
                    path = os.path.join(args.resume, f"{tag}.npz")
                    if os.path.exists(path):
                        resume = np.load(path)
                base = int(resume["step"]) if resume is not None else 0
                cav = Cavity(Params(n=m, re=r, dt=wl["dt"], poisson_tol=wl["tol"],
                                    resume=1 if resume is not None else 0),
                             device="cuda:0", stream=stream,
                             omega0=[resume["omega"]] if resume is not None else None,
                             psi0=[resume["psi"]] if resume is not None else None)
                # the multigrid solver reaches the same discrete solution with far
                # fewer launches per stage than SOR
                cav.set_tuning(solver=CAVITY_SOLVER_MG)
                t0 = time.perf_counter()
                done, first, outcome = 0, -1, "max_steps"
                while base + done < args.study_steps:
                    chunk = min(args.study_chunk, args.study_steps - base - done)
                    try:
                        steady, stats = cav.run_steady(chunk, 100)
                    except CavityError as e:
                        if e.code != CAVITY_ENONFINITE:
                            raise
                        outcome = f"non-finite after step {base + done}"
                        break
                    st = stats[0]
                    done = st["step"]
                    rec = {"n": m, "re": r, "step": base + done,
                           "t": round((base + done) * wl["dt"], 6),
                           "wall_s": round(time.perf_counter() - t0, 2),
                           "res_psi": st["res_psi"], "res_omega": st["res_omega"],
                           "ke": st["ke"], "domega_inf_over_dt": st["domega_inf_over_dt"],
                           "sweeps_last_step": st["sweeps_last_step"],
                           "steady_step": steady[0] + base if steady[0] >= 0 else -1}
                    f.write(json.dumps(rec) + "\n")
                    f.flush()
                    print(json.dumps(rec), flush=True)
                    if steady[0] >= 0:
                        first, outcome = steady[0] + base, "steady"
                        break
                    if time.perf_counter() - t0 > args.study_seconds:
                        outcome = "time limit"
                        break
                if args.checkpoint:
                    os.makedirs(args.checkpoint, exist_ok=True)
                    psi, omega = cav.fields()[:2]
                    np.savez(os.path.join(args.checkpoint, f"{tag}.npz"), psi=psi, omega=omega,
                             step=base + done)
                summary = {"n": m, "re": r, "dt": wl["dt"], "solver": "multigrid",
                           "outcome": outcome, "steady_step": first,
                           "steps": base + done, "t": round((base + done) * wl["dt"], 6),
                           "resumed_from_step": base,
                           "wall_s": round(time.perf_counter() - t0, 2)}
                f.write(json.dumps({"summary": summary}) + "\n")
                print(json.dumps({"summary": summary}), flush=True)
                cav.close()
        return

    def single(name, steps, warmup, mode, solver=0, precision=None, tuning=None, tol=None,
               warm=None):
        wl = WORKLOADS[name]
        prec = CAVITY_MIXED if wl["precision"] == "mixed" else CAVITY_FP64
        if precision is not None:
            prec = precision
        omega0 = None
        if wl["init"] == "noise":
            omega0 = [inputs.noise_omega0(wl["n"], wl["noise_amplitude"], wl["noise_seed"])]
        cav = Cavity(Params(n=wl["n"], re=wl["re"], poisson_tol=tol or wl["tol"], precision=prec,
                            warm_start=args.warm_start if warm is None else warm),
                     device="cuda:0", stream=stream, omega0=omega0)
        if solver:
            cav.set_tuning(solver=solver)
        if tuning:
            cav.set_tuning(**tuning)
        cav.set_exec(EXEC[mode])
        el, stats = _timed_steps(torch, cav, steps, warmup)
        n = wl["n"]
        out = {"value": round(n * n * steps / el / 1e6, 4) if steps else 0.0,
               "ms_per_step": round(1e3 * el / max(steps, 1), 3),
               "sweeps_per_stage": stats[0]["sweeps_last_step"] / 5 if stats else None,
               "floor_limited_last_step": stats[0]["floor_limited"] if stats else None,
               "domega_inf_over_dt": stats[0]["domega_inf_over_dt"] if stats else None,
               "steps": steps, "exec": mode,
               "solver": "multigrid" if solver else "sor",
               "precision": "mixed" if prec == CAVITY_MIXED else "fp64"}
        return cav, prec, out

    # ---- headline: FP64 1024^2
    prec_override = None if args.precision is None else (
        CAVITY_MIXED if args.precision == "mixed" else CAVITY_FP64)
    head_tuning = {}
    for kv in filter(None, args.set_tuning.split(",")):
        key, val = kv.split("=")
        head_tuning[key] = float(val) if key == "sor_omega" else int(val)
    cav, prec, head = single(args.workload, args.steps, args.warmup, args.exec,
                             CAVITY_SOLVER_MG if args.solver == "multigrid" else 0,
                             precision=prec_override, tuning=head_tuning,
                             tol=args.poisson_tol)
    wl = WORKLOADS[args.workload]
    n = wl["n"]
    roofline = _sweep_roofline(torch, cav, stream, args.relax_launches, 0,
                               f"{args.workload}:fp64")
    if prec == CAVITY_MIXED:
        head["roofline_fp32_sweep"] = _sweep_roofline(torch, cav, stream, args.relax_launches, 1,
                                                      f"{args.workload}:fp32")
    cav.close()

    extras = {}
    chosen = set() if args.no_extras else (
        {"multigrid", "mixed_head", "persistent", "resident", "re3e4", "n4096", "coupled",
         "re_sweep6_fp64", "re_sweep6_mixed", "re_scan16_small_fp64"} if args.extras == "all"
        else set(args.extras.split(",")))
    if "multigrid" in chosen:
        # same workload, multigrid solver (same compact equation, same tolerance), each
        # solve started from the interpolant through 7 steps (its fastest start: 407
        # Mcell-steps/s against 341 with the SOR default of 6)
        cmg, _, mg = single(args.workload, args.steps, args.warmup, "stream", CAVITY_SOLVER_MG,
                            warm=7)
        mg["warm_start_levels"] = 7
        mg["vcycles_per_stage"] = mg["sweeps_per_stage"] / 4 if mg["sweeps_per_stage"] else None
        cmg.close()
        extras["multigrid_1024_re1e4_fp64"] = mg
    if "mixed_head" in chosen and prec != CAVITY_MIXED:
        # mixed + refinement on the headline workload itself, same steps and warm-up.  Its
        # solves stop at the first FP64 residual check (taken after a Gauss-Seidel pair)
        # below the tolerance; the FP64 solves read the residual right after over-relaxed
        # sweeps, which at 1024^2 stays above 1e-10 until it drops within one check
        # interval to 30-70 times below it (1.5e-12 at the stops after 100 steps, 3e-12
        # late in the run)
        cmh, _, mh = single(args.workload, args.steps, args.warmup, args.exec,
                            precision=CAVITY_MIXED)
        cmh.close()
        mh["speedup_vs_fp64_same_workload"] = round(mh["value"] / head["value"], 3)
        extras["mixed_1024_re1e4"] = mh
    if "persistent" in chosen:
        # the persistent-kernel and resident-solve executions of the headline workload
        cp, _, pers = single(args.workload, args.extra_steps, 1, "persistent")
        cp.close()
        extras["persistent_1024_re1e4_fp64"] = pers
    if "resident" in chosen:
        if args.exec != "resident":
            cr, _, res = single(args.workload, args.steps, args.warmup, "resident")
            cr.close()
            extras["resident_1024_re1e4_fp64"] = res
        if args.exec != "stream":
            cs_, _, strm = single(args.workload, args.steps, args.warmup, "stream")
            cs_.close()
            extras["stream_1024_re1e4_fp64"] = strm
    if "re3e4" in chosen:
        # FP64 and mixed + refinement on the same workload (1024^2, Re 3e4), with the
        # same steps and warm-up
        c64, _, r64 = single("cavity1024_re3e4_mixed", args.compare_steps, args.warmup,
                             args.exec, precision=CAVITY_FP64)
        c64.close()
        extras["sor_fp64_1024_re3e4"] = r64
        cavm, _, mixed = single("cavity1024_re3e4_mixed", args.compare_steps, args.warmup,
                                args.exec)
        mixed["roofline_fp32_sweep"] = _sweep_roofline(torch, cavm, stream, args.relax_launches,
                                                       1, "cavity1024_re3e4_mixed:fp32")
        mixed["speedup_vs_fp64_same_workload"] = round(mixed["value"] / r64["value"], 3)
        cavm.close()
        extras["mixed_1024_re3e4"] = mixed
    if "n4096" in chosen:
        # 4096^2, Re 3e4, noise start (the HBM-resident case): FP64 SOR and mixed SOR for
        # the same steps (two after one warm-up), the rooflines of both sweep kernels at
        # this size, and FP64 multigrid
        key4 = "cavity4096_re3e4_mixed_noise"
        c4, _, f4 = single(key4, 2, 1, "stream", precision=CAVITY_FP64)
        f4["roofline_fp64_sweep"] = _sweep_roofline(torch, c4, stream, 40, 0, f"{key4}:fp64")
        c4.close()
        extras["cavity4096_re3e4_noise_fp64_sor"] = f4
        c4, _, m4 = single(key4, 2, 1, "stream")
        m4["roofline_fp32_sweep"] = _sweep_roofline(torch, c4, stream, 40, 1, f"{key4}:fp32")
        m4["speedup_vs_fp64_same_workload"] = round(m4["value"] / f4["value"], 3)
        c4.close()
        extras["cavity4096_re3e4_noise_mixed_sor"] = m4
        # per-step cross-check of the 4096^2 sweep rooflines: the bytes every sweep
        # launch of a step must move, over the whole step's time (all kernels)
        for rec, key in ((f4, "roofline_fp64_sweep"), (m4, "roofline_fp32_sweep")):
            rl = rec[key]
            launches = 5 * rec["sweeps_per_stage"] / rl["sweeps_per_launch"]
            rl["per_step_gbs"] = round(launches * rl["bytes_per_launch"] /
                                       (rec["ms_per_step"] / 1e3) / 1e9, 1)
        c4, _, g4 = single(key4, args.extra_steps, 1, "stream", CAVITY_SOLVER_MG, CAVITY_FP64)
        c4.close()
        extras["cavity4096_re3e4_noise_fp64_multigrid"] = g4
    if "coupled" in chosen:
        # coupled mode: a fixed 20 sweeps per stage with beta = 0.8 (no stopping test)
        cc = Cavity(Params(n=n, re=wl["re"], fixed_sweeps=20, sor_omega=0.8), device="cuda:0",
                    stream=stream)
        el, st = _timed_steps(torch, cc, args.steps, args.warmup)
        cc.close()
        extras["coupled_1024_re1e4_fixed20_beta0.8"] = {
            "value": round(n * n * args.steps / el / 1e6, 4),
            "ms_per_step": round(1e3 * el / args.steps, 3),
            "sweeps_per_stage": st[0]["sweeps_last_step"] / 5, "steps": args.steps}
    # batched Reynolds sweeps vs one cavity at a time: six cavities 256^2..1024^2
    # (FP64 and mixed) and sixteen 128^2 cavities (FP64)
    for wname, label, prec_b in (("re_sweep6", "fp64", CAVITY_FP64),
                                 ("re_sweep6", "mixed", CAVITY_MIXED),
                                 ("re_scan16_small", "fp64", CAVITY_FP64)):
        if f"{wname}_{label}" not in chosen:
            continue
        b = WORKLOADS[wname]
        cells = sum(m * m for _, m in b["members"])
        cb = Cavity([Params(n=m, re=r, poisson_tol=b["tol"], precision=prec_b)
                     for r, m in b["members"]], device="cuda:0", stream=stream)
        default_exec = cb.exec_mode()
        cb.set_exec(EXEC["graph"])
        # the persistent kernel's tile shape chosen by the autotuner (timed rounds)
        tuned = cb.autotune(-1, args.tune_cache)
        el, _ = _timed_steps(torch, cb, args.extra_steps, 1)
        cb.close()
        # the same batch in stream execution: one stream per cavity
        cb = Cavity([Params(n=m, re=r, poisson_tol=b["tol"], precision=prec_b)
                     for r, m in b["members"]], device="cuda:0", stream=stream)
        cb.set_exec(EXEC["stream"])
        el_st, _ = _timed_steps(torch, cb, args.extra_steps, 1)
        cb.close()
        seq = 0.0
        for r, m in b["members"]:
            cs = Cavity(Params(n=m, re=r, poisson_tol=b["tol"], precision=prec_b),
                        device="cuda:0", stream=stream)
            e1, _ = _timed_steps(torch, cs, args.extra_steps, 1)
            seq += e1
            cs.close()
        extras[f"{wname}_{label}"] = {
            "cells": cells,
            "batched_graph_mcell_steps_s": round(cells * args.extra_steps / el / 1e6, 4),
            "batched_streams_mcell_steps_s": round(cells * args.extra_steps / el_st / 1e6, 4),
            "sequential_stream_mcell_steps_s": round(cells * args.extra_steps / seq / 1e6, 4),
            "speedup": round(seq / el, 3), "speedup_streams": round(seq / el_st, 3),
            "default_exec": {v: k for k, v in EXEC.items()}[default_exec],
            "graph_tuning": {k: tuned[k] for k in ("tile_x", "tile_y", "sweeps_per_launch",
                                                   "threads", "tile_x32", "tile_y32",
                                                   "sweeps_per_launch32", "threads32",
                                                   "check_every", "inner_sweeps")},
            "steps": args.extra_steps}

    cpu = None if args.no_cpu else _cpu_baseline(n, wl["re"], args.cpu_steps)
    line = {
        "metric": METRIC, "value": head["value"], "unit": "Mcell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == CAVITY_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "re": wl["re"], "poisson_tol": args.poisson_tol or wl["tol"],
                   "precision": head["precision"], "solver": head["solver"], "init": wl["init"],
                   "exec": head["exec"],
                   "sweeps_per_stage": head["sweeps_per_stage"],
                   "floor_limited_last_step": head["floor_limited_last_step"],
                   **({"tuning": head_tuning} if head_tuning else {}),
                   "warm_start_levels": args.warm_start or (
                       CAVITY_WARM_LEVELS_MIXED if prec == CAVITY_MIXED
                       else CAVITY_WARM_LEVELS_FP64)},
        "roofline": roofline,
        **({"roofline_fp32_sweep": head["roofline_fp32_sweep"]}
           if "roofline_fp32_sweep" in head else {}),
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)
    if args.copy_calibration:
        # 1 GiB source, then 1 GiB of other writes so that the source has left
        # the caches, then one copy: its counters should read 1 GiB each way
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        evict = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(2.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize(dev)
        dst.copy_(src)
        torch.cuda.synchronize(dev)
        del src, evict, dst


if __name__ == "__main__":
    main()
