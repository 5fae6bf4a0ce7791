#!/usr/bin/env python
"""Adjoint solves per second on one MI355X.

Workload: the 32x8x8-cell Neo-Hookean beam (12,288 tets, 2,673 vertices,
E = 1e6 Pa, nu = 0.45) lying on the ground and pushed sideways, at friction
coefficients 1.0 (stick), 0.1 (slip) and 0.4 (mixed), plain FP64.  One step
of this benchmark is one adjoint solve of one recorded scene-step: setup
(per-tet SVD Jacobians, assembly, contact blocks, capacitance), the Krylov
solve to a relative residual of 1e-8, and the gradient contractions.  The
steps cycle over the recorded converged states of the three runs.

Also reported: the roofline of the dominant kernel (algorithmic bytes per
launch / average launch time, from HIP events on the launch stream over the
timed region) and the oracle's rate on the host cores (a bounded sample).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import glob
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "adjoint solves/sec at rel. residual 1e-8, mixed vs plain FP64; matvec HBM GB/s"
HBM_PEAK_GBPS = 8000.0
MUS = (1.0, 0.1, 0.4)


def load_states():
    """Converged beam states (written by tests/golden/make_beam_states.py)."""
    states = []
    for mu in MUS:
        path = os.path.join(ROOT, "tests", "golden", f"beam_states_mu{mu}.npz")
        if not os.path.exists(path):
            continue
        d = np.load(path)
        for t in range(int(d["steps"])):
            states.append({k: d[f"{k}{t}"] for k in ("q", "qbar", "vbar", "vid", "collider", "frame", "d_n",
                                                     "d_f", "fric", "delta", "lam")} | {"mu": mu, "t": t})
    if not states:
        raise SystemExit("no beam states found under tests/golden (run make_beam_states.py)")
    return states


def algorithmic_bytes(kernel, info, nc, m, ncv):
    nv, nnzb, nnzS = info["n_verts"], info["nnz_blocks"], info["nnz_S"]
    n3 = 3 * nv
    if kernel in ("S", "ST"):
        return nnzS * (8 + 4) + (nv + 1) * 8 + 2 * n3 * 8
    if kernel == "bsr":
        return nnzb * (72 + 4) + (nv + 1) * 4 + 2 * n3 * 8
    if kernel == "capinv":
        return m * m * 8 + m * 8 + n3 * 8
    if kernel == "Z":
        return nv * ncv * 8 + 2 * n3 * 8 + m * 8
    if kernel == "tet":
        return info["n_tets"] * (16 + 96 + 24 + 96 + 720)
    raise ValueError(kernel)


def cpu_baseline(spec, states, sample):
    """The oracle (direct sparse LU + refinement) on `sample` scene-steps."""
    from threadpoolctl import threadpool_limits

    from oracle import adjoint as adj
    from oracle.contact import ContactSet
    from oracle.forward import StepRecord
    from oracle.rollout import scene_disc

    disc = scene_disc(spec)
    gq = spec.loss_dir
    gv = np.zeros_like(gq)
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        for st in states[:sample]:
            cs = ContactSet(st["vid"], st["collider"], st["frame"], st["d_n"], st["d_f"], st["fric"].astype(bool))
            rec = StepRecord(cs, st["delta"], st["lam"], st["mu"])
            adj.adjoint_step(disc, st["q"], rec, gq, gv, spec.eps, spec.E, spec.nu)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "adjoint solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample} beam scene-steps (setup + direct sparse LU solve with long-double "
                      f"refinement + gradient contractions), single thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--roofline-kernel", default="S", choices=["S", "ST", "bsr", "capinv", "Z", "tet"])
    ap.add_argument("--cpu-sample", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2603_16478_amd import native
    from synth import beam_scene

    dev = "cuda"
    spec = beam_scene(mu=0.4)
    states = load_states()
    max_c = max(int(s["vid"].shape[0]) for s in states)
    scene = native.Scene(spec.mesh.rest, spec.mesh.tets, spec.density, spec.h, spec.eps, spec.E, spec.nu,
                         spec.gravity, spec.planes, spec.contact_margin, max_c)
    info = scene.info()
    # device copies of every recorded state
    dstates = []
    for st in states:
        n = int(st["vid"].shape[0])
        t = {"vid": torch.tensor(st["vid"].astype(np.int32), device=dev),
             "fric": torch.tensor(st["fric"].astype(np.int32), device=dev),
             "frame": torch.tensor(st["frame"].reshape(n, 9), dtype=torch.float64, device=dev),
             "delta": torch.tensor(st["delta"], dtype=torch.float64, device=dev),
             "lam": torch.tensor(st["lam"], dtype=torch.float64, device=dev),
             "q": torch.tensor(st["q"], dtype=torch.float64, device=dev)}
        t["cs"] = native.make_contact_state(n, t["vid"], t["fric"], t["frame"], t["delta"], t["lam"], st["mu"])
        t["m"] = int(3 * st["fric"].sum() + (n - st["fric"].sum()))
        t["ncv"] = int(np.unique(st["vid"]).shape[0])
        dstates.append(t)
    gq = torch.tensor(spec.loss_dir, dtype=torch.float64, device=dev)
    gv = torch.zeros_like(gq)
    z = torch.zeros_like(gq)
    dqbar, dvbar, dfext = torch.empty_like(gq), torch.empty_like(gq), torch.empty_like(gq)
    grad3 = torch.zeros(3, dtype=torch.float64, device=dev)
    opts = native.solve_opts(rtol=args.rtol, maxit=5000, restart=64)

    tuning = native.get_tuning(scene)
    if not args.no_autotune:
        t0s = dstates[0]
        native.adjoint_setup(scene, t0s["cs"], t0s["q"], opts)
        tuning = native.autotune(scene, gq, gv, z, opts, reps=3)

    iters = []

    def one(i):
        t = dstates[i % len(dstates)]
        native.adjoint_setup(scene, t["cs"], t["q"], opts)
        info_s = native.adjoint_solve(scene, gq, gv, z, opts)
        native.vjp_params(scene, z, gv, dqbar, dvbar, dfext, grad3)
        iters.append(info_s.iters)

    for i in range(args.warmup):
        one(i)
    torch.cuda.synchronize()
    iters.clear()
    native.profile_begin(scene, args.roofline_kernel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one(args.warmup + i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, launches = native.profile_end(scene, )
    # matvec (block-sparse Acal^T product) rate over a short separate region
    native.profile_begin(scene, "bsr")
    for i in range(min(args.steps, 6)):
        one(i)
    torch.cuda.synchronize()
    bms, blaunch = native.profile_end(scene)

    # mixed precision (FP32-stored matrices inside GMRES, FP64 refinement) on the same steps
    opts_m = native.solve_opts(rtol=args.rtol, maxit=5000, restart=64, prec=native.ADJ_MIXED, max_refine=8)
    miters = []

    def one_mixed(i):
        t = dstates[i % len(dstates)]
        native.adjoint_setup(scene, t["cs"], t["q"], opts_m)
        info_m = native.adjoint_solve(scene, gq, gv, z, opts_m)
        native.vjp_params(scene, z, gv, dqbar, dvbar, dfext, grad3)
        miters.append((info_m.iters, info_m.refine_steps))

    for i in range(args.warmup):
        one_mixed(i)
    torch.cuda.synchronize()
    miters.clear()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_mixed(args.warmup + i)
    torch.cuda.synchronize()
    dt_m = time.perf_counter() - t0

    # batched: the three independent runs (mu 1.0 / 0.1 / 0.4) at the same
    # step solved as one batch (one launch per phase, one GMRES per scene)
    by_t = {}
    for k, st in enumerate(states):
        by_t.setdefault(st["t"], []).append(k)
    groups = [v for _, v in sorted(by_t.items()) if len(v) == len(MUS)]
    batched = None
    if groups:
        specs = [beam_scene(mu=mu) for mu in MUS]
        batch = native.Batch([(sp.mesh.rest, sp.mesh.tets, sp.E, sp.nu) for sp in specs], spec.density, spec.h,
                             spec.eps, spec.gravity, spec.planes, spec.contact_margin, [max_c] * len(MUS))
        bgq = torch.cat([gq] * len(MUS))
        bgv = torch.zeros_like(bgq)
        bz = torch.zeros_like(bgq)
        bq = [torch.cat([dstates[k]["q"] for k in g]) for g in groups]
        bd = [torch.empty_like(bgq) for _ in range(3)]
        bgrad = torch.zeros(3 * len(MUS), dtype=torch.float64, device=dev)

        def run_batched(prec, nsteps, warm):
            o = native.solve_opts(rtol=args.rtol, maxit=5000, restart=64, prec=prec, max_refine=8)
            its = []
            for i in range(warm + nsteps):
                if i == warm:
                    torch.cuda.synchronize()
                    its.clear()
                    t0b = time.perf_counter()
                g = groups[i % len(groups)]
                native.batch_setup(batch, [dstates[k]["cs"] for k in g], bq[i % len(groups)], o)
                infos = native.batch_solve(batch, bgq, bgv, bz, o)
                native.batch_vjp(batch, bz, bgv, bd[0], bd[1], bd[2], bgrad)
                its.append(np.mean([f.iters for f in infos]))
            torch.cuda.synchronize()
            dtb = time.perf_counter() - t0b
            return {"value": len(MUS) * nsteps / dtb, "unit": "adjoint solves/s", "n_scenes": len(MUS),
                    "ms_per_batch": 1e3 * dtb / nsteps, "krylov_iters_mean": float(np.mean(its))}

        nb_steps = max(4, args.steps // len(MUS))
        batched = {"fp64": run_batched(native.ADJ_FP64, nb_steps, 2),
                   "mixed": run_batched(native.ADJ_MIXED, nb_steps, 2)}
        batched["fp64"]["speedup_vs_single_fp64"] = batched["fp64"]["value"] / (args.steps / dt)
        batched["mixed"]["speedup_vs_single_fp64"] = batched["mixed"]["value"] / (args.steps / dt)
        batch.close()

    t_avg = dstates[0]
    nc0 = int(states[0]["vid"].shape[0])
    abytes = algorithmic_bytes(args.roofline_kernel, info, nc0, t_avg["m"], t_avg["ncv"])
    avg_ms = kms / max(launches, 1)
    achieved = abytes / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    mv_bytes = algorithmic_bytes("bsr", info, nc0, t_avg["m"], t_avg["ncv"])
    mv_ms = bms / max(blaunch, 1)
    out = {
        "metric": METRIC,
        "value": args.steps / dt,
        "unit": "adjoint solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "beam 32x8x8 cells (12,288 tets, 2,673 vertices), E=1e6 Pa, nu=0.45, on the "
                        "ground under a sideways push; mu 1.0 / 0.1 / 0.4, recorded steps 0-3 of each; "
                        "plain FP64, GMRES(64) + Woodbury to rel. residual 1e-8",
            "n_scene_steps": len(states),
            "contacts": nc0,
            "capacitance_rows": t_avg["m"],
            "krylov_iters_mean": float(np.mean(iters)) if iters else None,
            "precision": "fp64",
            "tuning": tuning,
        },
        "roofline": {
            "kernel": {"S": "sparse-inverse product S x", "ST": "sparse-inverse product S^T x",
                       "bsr": "block-sparse Acal^T x", "capinv": "capacitance-inverse product",
                       "Z": "Woodbury correction Z t", "tet": "per-tet SVD Jacobian blocks"}[args.roofline_kernel],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": None,
            "algorithmic_bytes_per_launch": abytes,
            "avg_launch_us": 1e3 * avg_ms,
            "launches_timed": launches,
        },
        "matvec": {"bytes_per_launch": mv_bytes, "avg_launch_us": 1e3 * mv_ms,
                   "GB/s": mv_bytes / (mv_ms * 1e-3) / 1e9 if blaunch else None},
        "mixed": {"value": args.steps / dt_m, "unit": "adjoint solves/s",
                  "ms_per_step": 1e3 * dt_m / args.steps,
                  "krylov_iters_mean": float(np.mean([a for a, _ in miters])),
                  "refine_steps_mean": float(np.mean([b for _, b in miters])),
                  "speedup_vs_fp64": (args.steps / dt_m) / (args.steps / dt)},
        "batched": batched,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, states, args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
