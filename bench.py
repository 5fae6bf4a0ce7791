#!/usr/bin/env python
"""Adjoint solves per second on one MI355X.

Workload: the 32x8x8-cell Neo-Hookean beam (12,288 tets, 2,673 vertices,
E = 1e6 Pa, nu = 0.45) lying on the ground and pushed sideways, three runs at
friction coefficients 1.0 (stick), 0.1 (slip) and 0.4 (mixed).  One adjoint
solve = setup (per-tet SVD Jacobians, assembly, contact blocks, capacitance
and its inverse), the Krylov solve to a relative residual of 1e-8 and the
gradient contractions, on a recorded converged scene-step.

`value` is the whole-job rate of the reverse pass over the recorded steps
(the time recursion: each step's right-hand side comes from the next step's
gradient contractions).  The three runs are independent, so each time step
solves the three runs' adjoints as one batch (one launch per phase over all
three scenes, one GMRES per scene), in plain FP64, and the setup of the next
step runs on a second stream while a step is solved; a bench step is one
time step of the pass (three solves).  Also reported: the pass in mixed
precision and without the pipelining, one batch per step with a fixed
right-hand side (FP64 and mixed; the roofline kernels are timed there),
each scene solved alone (FP64 and mixed), the comparison preconditioners
of the backward solve, the beam with its end face held by bilateral
bindings (single scene, FP64), the as-rigid-as-possible and co-rotational
local steps (single scene, FP64), the full-size slab (FP64 and mixed), the
batched workload's boxes over their full size range (FP64 and mixed), a large batch (the
twelve recorded scene-steps four times: 48 scenes per launch, FP64 and
mixed, with the sparse-inverse product's bandwidth), the rooflines of the
two largest kernels, the batched Gauss-Jordan step and the batched
sparse-inverse product, the larger by time per batch as `roofline`
(algorithmic bytes per launch / average launch time from HIP events on the
launch stream, and the HBM traffic of the counter runs when the kernel
source still matches them), and the oracle's rate on one host core (a
bounded sample).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
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
sys.path.insert(0, ROOT)

METRIC = "adjoint solves/sec at rel. residual 1e-8, mixed vs plain FP64; matvec HBM GB/s"
HBM_PEAK_GBPS = 8000.0
MUS = (1.0, 0.1, 0.4)
CSRC = os.path.join(ROOT, "paper_2603_16478_amd", "csrc")
# calibrated HBM traffic per launch from the committed counter runs, one file
# per kernel, each tagged with a hash of the source it was measured on
COUNTERS = {"s_product": os.path.join(ROOT, "profiles", "s_product_batched_beam_counters.json"),
            "gj_wide": os.path.join(ROOT, "profiles", "gj_wide_slab_counters.json"),
            "lu_tiles": os.path.join(ROOT, "profiles", "lu_tiles_rest_slab_counters.json"),
            "gj_step": os.path.join(ROOT, "profiles", "gj_step_batched_beam_counters.json"),
            "s_product_single": os.path.join(ROOT, "profiles", "s_product_slab_counters.json"),
            "tet": os.path.join(ROOT, "profiles", "tet_assembly_slab_counters.json")}


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


def load_onset_states():
    """The beam's converged oracle states around its slip onsets (written by
    tests/golden/make_beam_onset.py), in the order of the stored oracle
    solutions of tests/golden/beam_onset_z.npz."""
    oz = np.load(os.path.join(ROOT, "tests", "golden", "beam_onset_z.npz"))
    states = []
    for mu in (0.1, 0.4):
        d = np.load(os.path.join(ROOT, "tests", "golden", f"beam_onset_mu{mu}.npz"))
        for k in range(int(d["steps"])):
            t = int(d[f"t{k}"])
            idx = [i for i in range(oz["z"].shape[0]) if oz["mu"][i] == mu and int(oz["t"][i]) == t]
            if len(idx) != 1:
                raise SystemExit(f"no stored oracle solution for the beam at mu={mu}, step {t}")
            states.append({key: d[f"{key}{k}"] for key in ("q", "vid", "fric", "frame", "delta", "lam")} |
                          {"mu": mu, "t": t, "index": idx[0]})
    return states


def s_product_bytes(info):
    """Algorithmic bytes of one sparse-inverse product y = S x (3 right-hand
    sides): values and column indices of S, row pointers, x and y."""
    nv, nnzS = info["n_verts"], info["nnz_S"]
    return nnzS * (8 + 4) + (nv + 1) * 8 + 2 * 3 * nv * 8


def sweep_bytes(info):
    """Algorithmic bytes of one sweep with the Cholesky factor (3 right-hand
    sides): values and row indices of L, x and y."""
    return info["nnz_L"] * (8 + 4) + 2 * 3 * info["n_verts"] * 8


def bsr_bytes(info):
    nv, nnzb = info["n_verts"], info["nnz_blocks"]
    return nnzb * (72 + 4) + (nv + 1) * 4 + 2 * 3 * nv * 8


def gj_step_bytes(mps):
    """Algorithmic bytes of the batched Gauss-Jordan block steps of one
    capacitance inversion: every step reads and writes each scene's padded
    mp x mp FP64 matrix once (the 32-wide panels and pivot blocks are
    re-read from cache); scene s takes mp_s / 32 steps.  Returns (bytes,
    launches)."""
    return sum((mp // 32) * 2 * 8 * mp * mp for mp in mps), max(mps) // 32


def gj_step_flops(mps):
    """Useful FP64 flops of the same steps: the rank-32 update of every
    output entry, plus A_ik P for the panel rows."""
    return sum((mp // 32) * (2 * 32 * mp * mp + 2 * 32 * 32 * mp) for mp in mps)


def _function_text(src, name):
    m = re.search(r"(?:__global__|__device__)[^;{]*?\b" + name + r"\b.*?\n}\n", src, re.S)
    return m.group(0) if m else src


GJ_FUNCTIONS = ("readlane_d", "rcp_newton", "max_dpp", "gj_rows_step", "invert32_rows", "gj_tile", "gj_next_pivot",
                "kb_gj_step_mfma")
LU_MIN = 4608  # padded capacitance size from which the library factors by block LU (default tuning)
LUT_FUNCTIONS = ("lu_tile_rest", "k_lu_tiles_rest")
GJW_FUNCTIONS = ("readlane_d", "rcp_newton", "max_dpp", "gj_rows_step", "invert32_rows", "k_gjw_pivot", "k_gjw_panel",
                 "k_gjw_tiles")


def kernel_source_hash(kernel):
    """Hash of the source text the kernel's counters depend on."""
    if kernel == "s_product":
        text = (_function_text(open(os.path.join(CSRC, "kernels_batch.hip")).read(), "kb_spmv_tasks") +
                _function_text(open(os.path.join(CSRC, "device_common.h")).read(), "row_dot3"))
    elif kernel == "s_product_single":
        text = (_function_text(open(os.path.join(CSRC, "kernels_krylov.hip")).read(), "k_spmv_tasks") +
                _function_text(open(os.path.join(CSRC, "device_common.h")).read(), "row_dot3"))
    elif kernel == "lu_tiles":
        src = open(os.path.join(CSRC, "kernels_dense.hip")).read()
        text = "".join(_function_text(src, f) for f in LUT_FUNCTIONS)
    elif kernel == "gj_wide":
        src = open(os.path.join(CSRC, "kernels_dense.hip")).read()
        text = "".join(_function_text(src, f) for f in GJW_FUNCTIONS)
    elif kernel == "tet":
        src = open(os.path.join(CSRC, "kernels_elastic.hip")).read()
        text = (_function_text(src, "k_tet_blocks") + _function_text(src, "k_assemble") +
                open(os.path.join(CSRC, "nh_local.h")).read())
    else:
        src = open(os.path.join(CSRC, "kernels_dense.hip")).read()
        m = re.search(r"struct GjShared \{.*?\};", src, re.S)
        text = "".join(_function_text(src, f) for f in GJ_FUNCTIONS) + (m.group(0) if m else src)
    return hashlib.sha1(text.encode()).hexdigest()


def measured_traffic(kernel):
    """Calibrated HBM bytes per launch from the committed counter runs, or
    None when the kernel changed since they were taken."""
    path = COUNTERS[kernel]
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_sha1") != kernel_source_hash(kernel):
        return None
    return d["bytes_per_launch"]


def batch_mps(native, batch, n_scenes):
    """Padded capacitance size of each scene after the last batch setup."""
    import ctypes
    lib = native.load()
    out = []
    for s in range(n_scenes):
        size = ctypes.c_int64()
        lib.adj_batch_debug_export(batch.handle, 1, s, None, 0, ctypes.byref(size))
        out.append(int(round((size.value // 8) ** 0.5)))
    return out


def cpu_baseline(spec, states, sample):
    """The oracle (direct sparse LU + refinement) on `sample` scene-steps,
    cycling over the recorded ones."""
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
        for i in range(sample):
            st = states[i % len(states)]
            cs = ContactSet(st["vid"], st["collider"], st["frame"], st["d_n"], st["d_f"], st["fric"].astype(bool))
            rec = StepRecord(cs, st["delta"], st["lam"], st["mu"])
            adj.adjoint_step(disc, st["q"], rec, gq, gv, spec.eps, spec.E, spec.nu)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "adjoint solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample} beam scene-steps, cycling over the {len(states)} recorded ones (setup + direct "
                      f"sparse LU solve with long-double refinement + gradient contractions), single thread, "
                      f"{dt:.1f} s"}


def boxes_leg(n_boxes, nsolve):
    """The batched workload (boxes with log-uniform tet counts in [2k, 100k]):
    the first `n_boxes` of the seeded 256, each at its seeded deformed state
    with the ground contacts of tests/golden/batch_contacts.npz and seeded
    sticking contact values, solved as one batch (setup + solve + VJP), FP64
    and mixed, timed `nsolve` times after one untimed.  Returns a dict."""
    import torch

    from paper_2603_16478_amd import native
    from synth.configs import batched_scenes, contact_values, perturbed_state

    d = np.load(os.path.join(ROOT, "tests", "golden", "batch_contacts.npz"))
    specs = batched_scenes(256, seed=3, tmax=1e5)[:n_boxes]
    off = d["off"]
    dev = "cuda"
    keep, states, qs = [], [], []
    for k, spec in enumerate(specs):
        a, b = int(off[k]), int(off[k + 1])
        n = b - a
        delta, lam = contact_values(n, spec.mu, seed=200 + k)
        t = {"vid": torch.tensor(d["vid"][a:b] if n else np.zeros(1, np.int32), dtype=torch.int32, device=dev),
             "fric": torch.tensor(d["fric"][a:b].astype(np.int32) if n else np.zeros(1, np.int32), device=dev),
             "frame": torch.tensor(d["frame"][a:b] if n else np.zeros((1, 9)), dtype=torch.float64, device=dev),
             "delta": torch.tensor(delta if n else np.zeros((1, 3)), dtype=torch.float64, device=dev),
             "lam": torch.tensor(lam if n else np.zeros((1, 3)), dtype=torch.float64, device=dev)}
        keep.append(t)
        states.append(native.make_contact_state(n, t["vid"], t["fric"], t["frame"], t["delta"], t["lam"], spec.mu))
        qs.append(perturbed_state(spec, seed=100 + k))
    s0 = specs[0]
    t0 = time.perf_counter()
    batch = native.Batch([(sp.mesh.rest, sp.mesh.tets, sp.E, sp.nu) for sp in specs], s0.density, s0.h, s0.eps,
                         s0.gravity, s0.planes, s0.contact_margin,
                         [max(1, int(off[k + 1] - off[k])) for k in range(len(specs))])
    t_build = time.perf_counter() - t0
    info = batch.union_scene().info()
    print(f"{len(specs)} boxes: batch built in {t_build:.1f} s (nnz(S) {info['nnz_S']}, nnz(L) {info['nnz_L']})",
          file=sys.stderr, flush=True)
    rng = np.random.default_rng(300)
    q = torch.tensor(np.concatenate(qs), device=dev)
    gq = torch.tensor(rng.standard_normal(q.shape), device=dev)
    gv = torch.zeros_like(gq)
    z = torch.zeros_like(gq)
    dq, dv, df = torch.empty_like(gq), torch.empty_like(gq), torch.empty_like(gq)
    grad = torch.zeros(3 * len(specs), dtype=torch.float64, device=dev)
    legs = {}
    for name, prec in (("fp64", native.ADJ_FP64), ("mixed", native.ADJ_MIXED)):
        o = native.solve_opts(rtol=1e-8, maxit=3000, restart=64, prec=prec, max_refine=8)
        native.batch_setup(batch, states, q, o)  # warm-up (Delassus of this contact set)
        native.batch_solve(batch, gq, gv, z, o, raise_noconv=False)
        torch.cuda.synchronize()
        its = []
        t2 = time.perf_counter()
        for _ in range(nsolve):
            native.batch_setup(batch, states, q, o)
            infos = native.batch_solve(batch, gq, gv, z, o, raise_noconv=False)
            native.batch_vjp(batch, z, gv, dq, dv, df, grad)
            its.append(max(i.iters for i in infos))
            worst = max(i.relres for i in infos)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t2
        legs[name] = {"value": len(specs) * nsolve / dt, "unit": "adjoint solves/s",
                      "ms_per_batch": 1e3 * dt / nsolve, "krylov_iters_max_mean": float(np.mean(its)),
                      "max_relres": worst}
        print(f"{len(specs)} boxes {name}: {legs[name]['ms_per_batch']:.1f} ms per batch, "
              f"{legs[name]['value']:.1f} solves/s, max relres {worst:.1e}", file=sys.stderr, flush=True)
    legs["mixed"]["speedup_vs_fp64"] = legs["mixed"]["value"] / legs["fp64"]["value"]
    # launch shapes: graph replay of the Krylov chunks (captured once per
    # setup), then the batched autotuner's choice, FP64
    o = native.solve_opts(rtol=1e-8, maxit=3000, restart=64, prec=native.ADJ_FP64, max_refine=8)

    def timed_fp64():
        native.batch_setup(batch, states, q, o)
        native.batch_solve(batch, gq, gv, z, o, raise_noconv=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(nsolve):
            native.batch_setup(batch, states, q, o)
            native.batch_solve(batch, gq, gv, z, o, raise_noconv=False)
            native.batch_vjp(batch, z, gv, dq, dv, df, grad)
        torch.cuda.synchronize()
        return len(specs) * nsolve / (time.perf_counter() - t2)

    default = native.batch_get_tuning(batch)
    native.batch_set_tuning(batch, chunk=8, graph=0, a_inv=1)
    products_rate = timed_fp64()
    native.batch_set_tuning(batch, chunk=8, graph=0, a_inv=2)
    sweeps_rate = timed_fp64()
    native.batch_set_tuning(batch, chunk=8, graph=1)
    graph_rate = timed_fp64()
    native.batch_set_tuning(batch, chunk=8, graph=0)
    native.batch_setup(batch, states, q, o)
    best = native.batch_autotune(batch, gq, gv, z, o, reps=2)
    tuned_rate = timed_fp64()
    legs["launch_shapes"] = {"fp64_default": default | {"value": legs["fp64"]["value"],
                                                        "note": "a_inv 0: sweeps when S holds more than 32 M and "
                                                                "4 nnz(L) entries"},
                             "fp64_products": {"chunk": 8, "graph": 0, "a_inv": 1, "value": products_rate},
                             "fp64_sweeps": {"chunk": 8, "graph": 0, "a_inv": 2, "value": sweeps_rate},
                             "fp64_graph": {"chunk": 8, "graph": 1, "a_inv": 0, "value": graph_rate},
                             "fp64_autotuned": best | {"value": tuned_rate}, "unit": "adjoint solves/s"}
    print(f"{len(specs)} boxes fp64: S products {products_rate:.1f}, sweeps {sweeps_rate:.1f}, graph replay "
          f"{graph_rate:.1f} solves/s, autotuned {best} {tuned_rate:.1f}", file=sys.stderr, flush=True)
    batch.close()
    return {"workload": f"batched boxes: the first {len(specs)} of 256 seeded boxes (log-uniform 2k-100k tets), "
                        f"{sum(sp.n_tets for sp in specs)} tets, {sum(sp.n_verts for sp in specs)} vertices, "
                        f"{int(off[len(specs)])} ground contacts; seeded deformed states and sticking values; "
                        "GMRES(64) + Woodbury to 1e-8",
            "batch_build_s": t_build, "nnz_S": info["nnz_S"], "nnz_L": info["nnz_L"], "adjoint": legs}


def quadruped_leg(steps, checkpoint):
    """The actuated quadruped (30,720 tets, 6,649 vertices, feet on the
    ground, mu 0.8): `steps` GPU forward steps driven by 64 seeded sinusoidal
    active-stress parameters per step, then the gradient of the
    centre-of-mass x shift with respect to the steps x 64 parameters through
    the Actuation and Rollout autograd layers (checkpoints every
    `checkpoint` steps, segments recomputed).  Returns a dict."""
    import torch

    from paper_2603_16478_amd import native
    from paper_2603_16478_amd.rollout import Actuation, GpuSim, Rollout
    from synth.configs import actuation_groups, actuation_params, quadruped_scene

    spec = quadruped_scene()
    group, fibre = actuation_groups(spec.mesh)
    sim = GpuSim(spec, max_contacts=400)
    native.set_actuation(sim.scene, group, fibre, 64)
    dev = "cuda"
    q0 = torch.tensor(spec.q0, device=dev)
    v0 = torch.tensor(spec.v0, device=dev)
    # centre-of-mass weights: the lumped vertex masses (density x a quarter
    # of each incident tet's volume)
    x = spec.mesh.rest[spec.mesh.tets]
    vol = np.abs(np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2))) / 6.0
    m = np.zeros(spec.n_verts)
    np.add.at(m, spec.mesh.tets.reshape(-1), np.repeat(vol / 4.0, 4))
    w = np.zeros((spec.n_verts, 3))
    w[:, 0] = -m / m.sum()
    wt = torch.tensor(w, device=dev)
    a = torch.tensor(actuation_params(steps, amplitude=2e3), device=dev, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qT, _ = Rollout.apply(q0, v0, Actuation.apply(a, sim), sim.params(spec.mu), sim, checkpoint)
    L = torch.sum(wt * qT)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"quadruped: {steps} steps, forward {t1 - t0:.1f} s, backward {t2 - t1:.1f} s", file=sys.stderr, flush=True)
    return {"workload": f"actuated quadruped (30,720 tets, 6,649 vertices), {steps} steps at h = 1e-3, 64 seeded "
                        f"sinusoidal active-stress parameters per step, checkpoints every {checkpoint} steps",
            "forward_steps_per_s": steps / (t1 - t0), "backward_steps_per_s": steps / (t2 - t1),
            "com_x_shift_m": -float(L.detach()) - float(np.sum(-w[:, 0] * spec.q0[:, 0])),
            "grad_norm": float(a.grad.norm())}


def eps_sweep_one(two_eps2, side, seconds):
    """Down-slope displacement of one cube on the slope after `seconds` of
    simulated time with the GPU forward step (h = 0.01 s, warm-started
    multipliers); prints one JSON object."""
    import torch

    from paper_2603_16478_amd.rollout import GpuSim
    from synth import slope_scene

    spec = slope_scene(side, two_eps2, duration=seconds)
    sim = GpuSim(spec, max_contacts=64)
    q = torch.tensor(spec.q0, device="cuda")
    v = torch.tensor(spec.v0, device="cuda")
    f = torch.zeros_like(q)
    x0 = torch.tensor(spec.q0[:, 0], device="cuda")
    track = []
    t0 = time.perf_counter()
    for t in range(spec.steps):
        q, v, _ = sim.step(q, v, f, spec.mu)
        if (t + 1) % max(1, spec.steps // 20) == 0:
            track.append(float((q[:, 0] - x0).mean()))
            print(f"2eps^2 {two_eps2:g} {side}: t = {(t + 1) * spec.h:.1f} s, {track[-1]:.4e} m", file=sys.stderr,
                  flush=True)
    dt = time.perf_counter() - t0
    sim.scene.close()
    print(json.dumps({"mu": spec.mu, "displacement_m": float((q[:, 0] - x0).mean()), "trajectory_m": track,
                      "ms_per_step": 1e3 * dt / spec.steps}))


SLAB_FIXTURE = os.path.join(ROOT, "tests", "golden", "slab_step50.npz")
FP64_PEAK_TFLOPS = 78.6


def slab_inputs():
    """The slab workload's measured step: the contact set stored with the
    oracle's solution (tests/golden/slab_step50.npz, written by
    tests/golden/make_oracle_z.py), the seeded state, contact values and
    right-hand side of synth (the same inputs the oracle solved)."""
    from synth.configs import contact_values, slab_last_step, slab_scene
    spec = slab_scene()
    d = np.load(SLAB_FIXTURE)
    _, q, gq, gv = slab_last_step(spec)
    delta, lam = contact_values(int(d["vid"].shape[0]), spec.mu)
    return spec, d, q, gq, gv, delta, lam


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def slab_headline(args):
    """Headline: the slab workload (64x32x32 cells, 393,216 tets, 70,785
    vertices, pressed by the sphere) at its last step, 3,022 contacts and
    9,018 capacitance rows.  One adjoint solve = adjoint_setup + adjoint_solve
    + vjp_params.  Cold: the Delassus product is rebuilt every solve (a new
    contact vertex set); warm: it is reused (the same contact vertex set, as
    along consecutive steps).  FP64 and mixed, each against the oracle's z.
    The kernels are timed live (HIP events on the launch stream) per class;
    the class with the largest time per solve is `roofline`."""
    import torch

    from paper_2603_16478_amd import native

    spec, d, qn, gqn, gvn, delta, lam = slab_inputs()
    n = int(d["vid"].shape[0])
    nfric = int(d["fric"].sum())
    t0 = time.perf_counter()
    scene = native.Scene(spec.mesh.rest, spec.mesh.tets, spec.density, spec.h, spec.eps, spec.E, spec.nu,
                         spec.gravity, spec.planes, spec.contact_margin, n)
    t_build = time.perf_counter() - t0
    info = scene.info()
    print(f"slab scene built in {t_build:.1f} s (nnz(L) {info['nnz_L']}, nnz(S) {info['nnz_S']})", file=sys.stderr,
          flush=True)
    dev = "cuda"
    tens = {"vid": torch.tensor(d["vid"].astype(np.int32), device=dev),
            "fric": torch.tensor(d["fric"].astype(np.int32), device=dev),
            "frame": torch.tensor(d["frame"].reshape(n, 9), dtype=torch.float64, device=dev),
            "delta": torch.tensor(delta, dtype=torch.float64, device=dev),
            "lam": torch.tensor(lam, dtype=torch.float64, device=dev)}
    cs = native.make_contact_state(n, tens["vid"], tens["fric"], tens["frame"], tens["delta"], tens["lam"], spec.mu)
    q = torch.tensor(qn, device=dev)
    gq = torch.tensor(gqn, device=dev)
    gv = torch.tensor(gvn, device=dev)
    z = torch.zeros_like(gq)
    dq, dv, df = torch.empty_like(gq), torch.empty_like(gq), torch.empty_like(gq)
    grad3 = torch.zeros(3, dtype=torch.float64, device=dev)
    zref = d["z"]

    def opts(prec, reuse):
        return native.solve_opts(rtol=args.rtol, maxit=3000, restart=64, prec=prec, max_refine=8,
                                 reuse_delassus=reuse)

    def solve(o):
        native.adjoint_setup(scene, cs, q, o)
        inf = native.adjoint_solve(scene, gq, gv, z, o)
        native.vjp_params(scene, z, gv, dq, dv, df, grad3)
        return inf

    def timed(o, k):
        its, ref = [], []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(k):
            inf = solve(o)
            its.append(inf.iters)
            ref.append(inf.refine_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        return {"value": k / dt, "ms_per_solve": 1e3 * dt / k, "solves": k, "krylov_iters_mean": float(np.mean(its)),
                "refinements_mean": float(np.mean(ref))}

    legs = {}
    m_rows = None
    for name, prec in (("fp64", native.ADJ_FP64), ("mixed", native.ADJ_MIXED), ("mixed_pc", native.ADJ_MIXED_PC)):
        for _ in range(max(1, args.warmup)):
            inf = solve(opts(prec, 1))
        m_rows = inf.m_rows
        cold = timed(opts(prec, 0), max(2, args.steps // 5))
        warm = timed(opts(prec, 1), args.steps)
        torch.cuda.synchronize()
        legs[name] = {"warm": warm, "cold": cold, "z_rel_err_vs_oracle": _rel(z.cpu().numpy(), zref)}
        print(f"slab {name}: warm {warm['ms_per_solve']:.1f} ms ({warm['krylov_iters_mean']:.0f} its), cold "
              f"{cold['ms_per_solve']:.1f} ms, z err {legs[name]['z_rel_err_vs_oracle']:.1e}", file=sys.stderr,
              flush=True)
    # live per-class kernel times, FP64, warm (the Delassus product on cold solves)
    nprof = 2
    prof = {}
    mp = ((m_rows + 127) // 128) * 128
    lu = mp >= LU_MIN
    for cls in ("gj", "S", "ST", "correction", "capinv", "bsr", "tet", "assemble", "gs_pass1", "gs_pass2",
                "delassus") + (("lu_tiles",) if lu else ()):
        o = opts(native.ADJ_FP64, 0 if cls == "delassus" else 1)
        solve(o)
        torch.cuda.synchronize()
        native.profile_begin(scene, cls)
        for _ in range(nprof):
            solve(o)
        ms, nl = native.profile_end(scene)
        prof[cls] = {"ms_per_solve": ms / nprof, "regions": nl, "avg_us": 1e3 * ms / max(nl, 1)}
    scene.close()
    torch.cuda.synchronize()
    nv, nt, nnzb, ncv = info["n_verts"], info["n_tets"], info["nnz_blocks"], int(np.unique(d["vid"]).size)
    # capacitance factorisation: algorithmic work 2/3 m^3 (an LU of the m x m
    # capacitance), the unit of the whole-factorisation figure
    gj = prof["gj"]
    gj_alg = 2.0 / 3.0 * m_rows ** 3
    gj_ach = gj_alg / (gj["avg_us"] * 1e-6) / 1e12
    whole = {"algorithmic_flops": gj_alg, "ms": gj["avg_us"] / 1e3, "tflops": gj_ach,
             "frac": gj_ach / FP64_PEAK_TFLOPS, "ms_per_solve": gj["ms_per_solve"]}
    if lu:
        # the trailing updates but their first tile column (that column and
        # the next pivot inverse run beside them): 2 * 128 * r (r - 128)
        # flops on the r x r trailing matrix (r = mp - 128 (k + 1)), one
        # launch per step with r > 128
        tiles = [2.0 * 128 * r * (r - 128) for r in range(mp - 128, 128, -128)]
        lt = prof["lu_tiles"]
        lt_fl = float(np.mean(tiles))
        lt_ach = lt_fl / (lt["avg_us"] * 1e-6) / 1e12
        roof_gj = {"kernel": "trailing update of the block-LU capacitance factorisation (k_lu_tiles_rest: A_ij -= "
                             "L_iK A_Kj on the 128 x 128 tiles below the pivot block and right of the next panel, "
                             "rank 128 on FP64 matrix cores, two blocks per CU, the tile's old values read in batches "
                             "beside the products), one launch per 128-column step",
                   "bound": "mfma", "achieved": lt_ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": lt_ach / FP64_PEAK_TFLOPS, "traffic": measured_traffic("lu_tiles"),
                   "algorithmic_flops_per_launch": lt_fl, "avg_launch_us": lt["avg_us"],
                   "launches_timed": lt["regions"], "ms_per_solve": lt["ms_per_solve"],
                   "factorisation": whole | {"kernels": "k_gjw_pivot, then per step k_lu_colpanel, k_lu_tiles_next "
                                                        "(next panel column and pivot inverse) beside "
                                                        "k_lu_tiles_rest on a second stream, then k_lu_rowpanels, "
                                                        "k_lu_group_inv, k_lu_group_apply"}}
    else:
        roof_gj = {"kernel": "capacitance inverse (wide Gauss-Jordan: k_gjw_pivot + k_gjw_panel + k_gjw_tiles "
                             "per 128-column step), one region per adjoint setup",
                   "bound": "mfma", "achieved": gj_ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": gj_ach / FP64_PEAK_TFLOPS, "traffic": measured_traffic("gj_wide"),
                   "algorithmic_flops_per_launch": gj_alg, "executed_flops_per_launch": 2.0 * mp ** 3,
                   "avg_launch_us": gj["avg_us"], "launches_timed": gj["regions"], "ms_per_solve": gj["ms_per_solve"]}
    # A^{-1} in the preconditioner: level-scheduled sweeps with L where S is
    # large (the library's automatic choice), else the S products
    sweeps = info["nnz_S"] >= 32_000_000 and info["nnz_S"] >= 4 * info["nnz_L"]
    sb = sweep_bytes(info) if sweeps else s_product_bytes(info)
    sp_ms = prof["S"]["ms_per_solve"] + prof["ST"]["ms_per_solve"]
    sp_avg = 1e3 * sp_ms * nprof / max(prof["S"]["regions"] + prof["ST"]["regions"], 1)
    sp_ach = sb / (sp_avg * 1e-6) / 1e9
    roof_s = {"kernel": ("level-scheduled supernodal sweeps with the Cholesky factor (L^{-1} P x and its "
                         "transpose, k_spmv_tasks per level), one of each per preconditioner apply" if sweeps else
                         "sparse-inverse products S x and S^T x (k_spmv_tasks), one of each per preconditioner "
                         "apply"),
              "bound": "hbm", "achieved": sp_ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
              "frac": sp_ach / HBM_PEAK_GBPS,
              "traffic": None if sweeps else measured_traffic("s_product_single"),
              "algorithmic_bytes_per_launch": sb, "avg_launch_us": sp_avg,
              "launches_timed": prof["S"]["regions"] + prof["ST"]["regions"], "ms_per_solve": sp_ms}
    # capacitance solve per apply: the factors (or the inverse) read once
    cs_b = mp * mp * 8 + (mp * 128 * 8 if lu else 0)
    ci = prof["capinv"]
    ci_ach = cs_b / (ci["avg_us"] * 1e-6) / 1e9
    roof_c = {"kernel": ("block-LU substitutions (k_wb_hq, then the pipelined forward and backward passes "
                          "k_lu_fwd_pipe, k_lu_bwd_pipe)"
                         if lu else
                         "capacitance-inverse product (k_wb_gather)") + ", one per preconditioner apply",
              "bound": "hbm", "achieved": ci_ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": ci_ach / HBM_PEAK_GBPS,
              "traffic": None, "algorithmic_bytes_per_launch": cs_b, "avg_launch_us": ci["avg_us"],
              "launches_timed": ci["regions"], "ms_per_solve": ci["ms_per_solve"]}
    ranked = sorted((roof_gj, roof_s, roof_c), key=lambda r: -r["ms_per_solve"])
    roofline, roofline_other = ranked[0], ranked[1:]
    # the product kernel also reads the basis vectors V_0..V_j for the first
    # Gram-Schmidt dots ((J + 1) / 2 on average over a cycle of J iterations)
    # and writes the flexible basis copy of its input
    its_f = legs["fp64"]["warm"]["krylov_iters_mean"]
    mvb = bsr_bytes(info) + ((its_f + 1) / 2 + 1) * 3 * info["n_verts"] * 8
    mv = prof["bsr"]
    tet_bytes = nt * (16 + 14 * 8) + nnzb * 9 * 8
    tet_us = prof["tet"]["avg_us"] + prof["assemble"]["avg_us"]
    dl = prof["delassus"]
    syrk_flops = float(nv) * ncv * ncv  # dense-equivalent Y^T Y (n_v x n_cv), symmetric half
    warm_f = legs["fp64"]["warm"]
    # value: the faster of the two mixed-precision modes (both are reported)
    best_mixed = max(("mixed", "mixed_pc"), key=lambda k: legs[k]["warm"]["value"])
    warm_m = legs[best_mixed]["warm"]
    return {
        "metric": METRIC,
        "value": warm_m["value"],
        "unit": "adjoint solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": warm_m["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed f32/f64",
        "data": "synthetic",
        "config": {
            "workload": "slab 64x32x32 cells (393,216 tets, 70,785 vertices), E=5e5 Pa, nu=0.45, mu=0.5, pressed "
                        "into the ground by a kinematic sphere of radius 0.192 m; its last step (top face on the "
                        "sphere at 0.093 m indentation): 3,022 contacts (2,145 ground, 877 sphere), 9,018 "
                        "capacitance rows; one step = one adjoint solve (setup + solve + VJP) to rel. residual "
                        "1e-8, GMRES(64) + Woodbury, Delassus product reused (warm); value = mixed precision",
            "n_contacts": n, "frictional": nfric, "m_rows": m_rows, "contact_vertices": ncv,
            "nnz_L": info["nnz_L"], "nnz_S": info["nnz_S"], "scene_build_s": t_build,
        },
        "fp64": warm_f | {"z_rel_err_vs_oracle": legs["fp64"]["z_rel_err_vs_oracle"], "cold": legs["fp64"]["cold"]},
        "mixed": legs["mixed"]["warm"] | {
            "mode": "ADJ_MIXED: FP64 refinement residual around inner GMRES with FP32 block values and FP32 "
                    "sweeps (FP64 Woodbury factors)",
            "z_rel_err_vs_oracle": legs["mixed"]["z_rel_err_vs_oracle"], "cold": legs["mixed"]["cold"],
            "speedup_vs_fp64": legs["mixed"]["warm"]["value"] / warm_f["value"]},
        "mixed_pc": legs["mixed_pc"]["warm"] | {
            "mode": "ADJ_MIXED_PC: one FP64 flexible GMRES (FP64 product, Gram-Schmidt and residual) whose "
                    "preconditioner runs the sweeps in FP32",
            "z_rel_err_vs_oracle": legs["mixed_pc"]["z_rel_err_vs_oracle"], "cold": legs["mixed_pc"]["cold"],
            "speedup_vs_fp64": legs["mixed_pc"]["warm"]["value"] / warm_f["value"]},
        "value_mode": best_mixed,
        "roofline": roofline,
        "roofline_other": roofline_other,
        "matvec": {"kernel": "Acal^T product fused with the first Gram-Schmidt dots (k_bsr_dots)",
                   "bytes_per_launch": mvb, "bytes_note": "blocks, indices, x, w, the flexible-basis copy of x "
                                                         "and the mean (J + 1) / 2 basis vectors read for the dots",
                   "avg_launch_us": mv["avg_us"],
                   "GB/s": mvb / (mv["avg_us"] * 1e-6) / 1e9 if mv["regions"] else None,
                   "frac": mvb / (mv["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBPS if mv["regions"] else None},
        "svd_jacobian": {"kernel": "per-tet SVD / Neo-Hookean projection Jacobian blocks (k_tet_blocks) + gather "
                                   "assembly (k_assemble)",
                         "algorithmic_bytes": tet_bytes, "us": tet_us,
                         "GB/s": tet_bytes / (tet_us * 1e-6) / 1e9,
                         "frac": tet_bytes / (tet_us * 1e-6) / 1e9 / HBM_PEAK_GBPS,
                         "traffic": measured_traffic("tet"),
                         "note": "algorithmic bytes: the per-tet inputs and the assembled blocks; traffic (counters, "
                                 "profiles/tet_assembly_slab_counters.json) adds the 90-double element blocks written "
                                 "by k_tet_blocks and gathered back by k_assemble"},
        # Y is sparse and the product skips its empty 64-row panels, so the
        # dense-equivalent rate below is not a matrix-core utilisation
        "delassus_syrk": {"kernel": "Y = S E, D = Y^T Y on FP64 matrix cores (k_y_panels + k_syrk_mfma, empty "
                                    "panels of Y skipped), cold solves only",
                          "dense_equivalent_flops": syrk_flops, "ms": dl["avg_us"] / 1e3,
                          "dense_equivalent_tflops": syrk_flops / (dl["avg_us"] * 1e-6) / 1e12
                          if dl["regions"] else None},
        "kernel_ms_per_solve": {k: v["ms_per_solve"] for k, v in prof.items()},
    }


def _oracle_box(k):
    """One oracle adjoint solve of box k of the batched workload (for the
    all-core baseline; runs in a worker process)."""
    from threadpoolctl import threadpool_limits
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from make_oracle_z import boxes_cases

    from oracle import adjoint as adj
    from oracle.rollout import scene_disc
    spec, q, rec, gq, gv = boxes_cases(k + 1)[k]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        adj.adjoint_step(scene_disc(spec), q, rec, gq, gv, spec.eps, spec.E, spec.nu)
        return time.perf_counter() - t0


def slab_cpu_baseline(args):
    """The oracle on the GPU host: one adjoint step of the slab workload at
    1/8 of its cells (32x16x16, the same recipe; SuperLU on the full slab
    takes tens of minutes) on one core, and the batched workload's first
    boxes over all cores (one box per worker process)."""
    from threadpoolctl import threadpool_limits

    from oracle import adjoint as adj
    from oracle.rollout import scene_disc
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from make_oracle_z import slab_case
    from synth.configs import slab_scene

    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    nproc = len(os.sched_getaffinity(0))
    spec, _, q, rec, gq, gv = slab_case(slab_scene(nx=32, ny=16, nz=16))
    disc = scene_disc(spec)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        adj.adjoint_step(disc, q, rec, gq, gv, spec.eps, spec.E, spec.nu)
        dt = time.perf_counter() - t0
    out = {"value": 1.0 / dt, "unit": "adjoint solves/s", "cores": 1, "kind": "oracle",
           "sample": f"one adjoint step (assembly, direct sparse LU with long-double refinement, contractions) of "
                     f"the slab workload at 32x16x16 cells ({spec.n_tets} tets, {rec.contacts.n} contacts), the "
                     f"same recipe at 1/8 of the cells, single thread, {dt:.1f} s",
           "host_cpus": nproc, "cpu_model": model}
    if args.cpu_boxes > 0:
        import multiprocessing as mp
        workers = max(1, min(16, nproc, args.cpu_boxes))
        ctx = mp.get_context("spawn")
        t0 = time.perf_counter()
        with ctx.Pool(workers) as pool:
            times = pool.map(_oracle_box, range(args.cpu_boxes), chunksize=1)
        wall = time.perf_counter() - t0
        out["all_core"] = {"value": args.cpu_boxes / wall, "unit": "adjoint solves/s", "cores": workers,
                           "kind": "oracle",
                           "sample": f"the first {args.cpu_boxes} boxes of the batched workload (one scene-step "
                                     f"each, {workers} worker processes, one thread each), wall {wall:.1f} s, "
                                     f"sum of per-box times {sum(times):.1f} s"}
    return out


def eps_sweep(seconds):
    """The smoothing sweep: the sliding and the sticking cube (friction
    tan(10 deg) -/+ 4e-4) at each 2 eps^2, one child process per run, all
    sharing the GPU (each run is bound by the forward step's host round
    trips).  This process itself does not use the GPU.  Prints one JSON
    line."""
    import subprocess

    runs = [(e, side) for e in (1e-15, 1e-12, 1e-9, 1e-6) for side in ("slip", "stick")]
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--eps-sweep-one", f"{e:g}", side,
                               f"{seconds:g}"], stdout=subprocess.PIPE, text=True) for e, side in runs]
    rows = {}
    status = 0
    for (e, side), p in zip(runs, procs):
        out, _ = p.communicate()
        if p.returncode != 0:
            status = p.returncode
            continue
        rows.setdefault(f"{e:g}", {})[side] = json.loads(out.strip().splitlines()[-1])
    for row in rows.values():
        if "slip" in row and "stick" in row:
            row["slip_over_stick"] = row["slip"]["displacement_m"] / row["stick"]["displacement_m"]
    print(json.dumps({"study": "smoothing sweep on the slope cube (10 deg, 4x4x4 cells, E 1e7 Pa, h 0.01 s)",
                      "seconds": seconds, "analytic_slip_m": 0.5 * 9.81 * np.cos(np.deg2rad(10.0)) * 4e-4
                      * seconds ** 2, "by_two_eps2": rows}))
    if status:
        sys.exit(status)


def beam_legs(args):
    """The beam workload (three runs at mu 1.0 / 0.1 / 0.4, recorded converged
    steps): the pipelined reverse pass, batched and single-scene solves, the
    launch-shape autotuner, the backward-solver comparison, the material
    models and bindings, with their own roofline kernels and oracle baseline.
    Returns a dict."""
    import torch

    from paper_2603_16478_amd import native
    from synth import beam_scene

    dev = "cuda"
    spec = beam_scene(mu=0.4)
    states = load_states()
    max_c = max(int(s["vid"].shape[0]) for s in states)
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
        dstates.append(t)
    gq = torch.tensor(spec.loss_dir, dtype=torch.float64, device=dev)
    gv = torch.zeros_like(gq)

    # ---- batched: the three runs at the same time step as one batch ----
    by_t = {}
    for k, st in enumerate(states):
        by_t.setdefault(st["t"], []).append(k)
    groups = [v for _, v in sorted(by_t.items()) if len(v) == len(MUS)]
    if not groups:
        raise SystemExit("the beam fixtures of all three runs are needed")
    specs = [beam_scene(mu=mu) for mu in MUS]
    batch = native.Batch([(sp.mesh.rest, sp.mesh.tets, sp.E, sp.nu) for sp in specs], spec.density, spec.h,
                         spec.eps, spec.gravity, spec.planes, spec.contact_margin, [max_c] * len(MUS))
    uscene = batch.union_scene()
    uinfo = uscene.info()
    bgq = torch.cat([gq] * len(MUS))
    bgv = torch.zeros_like(bgq)
    bz = torch.zeros_like(bgq)
    bq = [torch.cat([dstates[k]["q"] for k in g]) for g in groups]
    bd = [torch.empty_like(bgq) for _ in range(3)]
    bgrad = torch.zeros(3 * len(MUS), dtype=torch.float64, device=dev)

    def run_batched(prec, nsteps, warm, profile=None):
        o = native.solve_opts(rtol=args.rtol, maxit=5000, restart=64, prec=prec, max_refine=8)
        its = []
        prof = None
        t0b = time.perf_counter()
        for i in range(warm + nsteps):
            if i == warm:
                torch.cuda.synchronize()
                its.clear()
                if profile:
                    native.profile_begin(uscene, profile)
                t0b = time.perf_counter()
            g = groups[i % len(groups)]
            native.batch_setup(batch, [dstates[k]["cs"] for k in g], bq[i % len(groups)], o)
            infos = native.batch_solve(batch, bgq, bgv, bz, o)
            native.batch_vjp(batch, bz, bgv, bd[0], bd[1], bd[2], bgrad)
            its.append(np.mean([f.iters for f in infos]))
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t0b
        if profile:
            prof = native.profile_end(uscene)
        return {"value": len(MUS) * nsteps / dtb, "unit": "adjoint solves/s", "n_scenes": len(MUS),
                "ms_per_batch": 1e3 * dtb / nsteps, "krylov_iters_mean": float(np.mean(its))}, prof

    bfp64, (kms, launches) = run_batched(native.ADJ_FP64, args.steps, args.warmup, profile="S")
    nprof = len(groups)  # one pass over the time steps per profiled kernel class
    _, (mv_ms, mv_launch) = run_batched(native.ADJ_FP64, nprof, 0, profile="bsr")
    _, (st_ms, st_launch) = run_batched(native.ADJ_FP64, nprof, 0, profile="ST")
    _, (gj_ms, gj_launch) = run_batched(native.ADJ_FP64, nprof, 0, profile="gj_step")
    gj_b = gj_f = 0
    for g in groups:  # the profiled pass ran the groups in this order
        native.batch_setup(batch, [dstates[k]["cs"] for k in g], bq[groups.index(g)],
                           native.solve_opts(rtol=args.rtol, maxit=5000, restart=64))
        mps = batch_mps(native, batch, len(MUS))
        gj_b += gj_step_bytes(mps)[0]
        gj_f += gj_step_flops(mps)
    torch.cuda.synchronize()
    bmixed, _ = run_batched(native.ADJ_MIXED, args.steps, args.warmup)

    # ---- the reverse pass over the recorded steps (the headline) ----
    # Sec. 5.1's recursion: from the last recorded step down to the first,
    # each step's right-hand side is the previous step's dL/dqbar, dL/dvbar.
    # A bench step is one time step of the pass (the three runs' adjoint
    # steps, three solves); K steps = K // T full passes plus one pass over
    # the last K % T steps.
    T = len(groups)
    rc = [[dstates[k]["cs"] for k in g] for g in groups]
    rb = [native.Batch([(sp.mesh.rest, sp.mesh.tets, sp.E, sp.nu) for sp in specs], spec.density, spec.h, spec.eps,
                       spec.gravity, spec.planes, spec.contact_margin, [max_c] * len(MUS)) for _ in range(2)]
    rdf = [torch.empty_like(bgq) for _ in range(T)]
    rgrad = torch.zeros(3 * len(MUS), dtype=torch.float64, device=dev)

    def reverse_pass(n, prec, pipelined):
        """One pass over the last n recorded steps; returns the iteration counts."""
        o = native.solve_opts(rtol=args.rtol, maxit=5000, restart=64, prec=prec, max_refine=8)
        gq_, gv_ = bgq.clone(), torch.zeros_like(bgq)
        sl = range(T - n, T)
        if pipelined:
            infos = native.batch_reverse(rb[0], rb[1], [rc[t] for t in sl], [bq[t] for t in sl], gq_, gv_,
                                         [rdf[t] for t in sl], rgrad, o)
            return [i.iters for st_ in infos for i in st_]
        its = []
        for t in reversed(sl):
            native.batch_setup(rb[0], rc[t], bq[t], o)
            z_ = torch.zeros_like(gq_)
            its += [i.iters for i in native.batch_solve(rb[0], gq_, gv_, z_, o)]
            dq_, dv_ = torch.empty_like(gq_), torch.empty_like(gq_)
            native.batch_vjp(rb[0], z_, gv_, dq_, dv_, rdf[t], rgrad)
            gq_, gv_ = dq_, dv_
        return its

    def run_reverse(prec, pipelined, nsteps, warm):
        def steps_of(k):
            return [T] * (k // T) + ([k % T] if k % T else [])
        for n in steps_of(warm):
            reverse_pass(n, prec, pipelined)
        torch.cuda.synchronize()
        its = []
        t0r = time.perf_counter()
        for n in steps_of(nsteps):
            its += reverse_pass(n, prec, pipelined)
        torch.cuda.synchronize()
        dtr = time.perf_counter() - t0r
        return {"value": len(MUS) * nsteps / dtr, "unit": "adjoint solves/s", "time_steps": nsteps,
                "ms_per_time_step": 1e3 * dtr / nsteps, "krylov_iters_mean": float(np.mean(its))}

    rev = run_reverse(native.ADJ_FP64, True, args.steps, args.warmup)
    rev_mixed = run_reverse(native.ADJ_MIXED, True, args.steps, args.warmup)
    rev_step = run_reverse(native.ADJ_FP64, False, args.steps, args.warmup)
    for b_ in rb:
        b_.close()
    batch.close()

    # ---- a large batch: every recorded scene-step, four times (48 scenes) ----
    big = None
    if args.big_batch > 0:
        reps = args.big_batch
        ks = list(range(len(states))) * reps
        bspecs = [beam_scene(mu=states[k]["mu"]) for k in ks]
        bb = native.Batch([(sp.mesh.rest, sp.mesh.tets, sp.E, sp.nu) for sp in bspecs], spec.density, spec.h,
                          spec.eps, spec.gravity, spec.planes, spec.contact_margin, [max_c] * len(ks))
        bu = bb.union_scene()
        binfo = bu.info()
        qq = torch.cat([dstates[k]["q"] for k in ks])
        gg = torch.cat([gq] * len(ks))
        vv = torch.zeros_like(gg)
        zz = torch.zeros_like(gg)
        oo = [torch.empty_like(gg) for _ in range(3)]
        gr = torch.zeros(3 * len(ks), dtype=torch.float64, device=dev)
        css = [dstates[k]["cs"] for k in ks]

        def run_big(prec, nsteps, warm, profile=None):
            o = native.solve_opts(rtol=args.rtol, maxit=5000, restart=64, prec=prec, max_refine=8)
            t0g = time.perf_counter()
            for i in range(warm + nsteps):
                if i == warm:
                    torch.cuda.synchronize()
                    if profile:
                        native.profile_begin(bu, profile)
                    t0g = time.perf_counter()
                native.batch_setup(bb, css, qq, o)
                native.batch_solve(bb, gg, vv, zz, o)
                native.batch_vjp(bb, zz, vv, oo[0], oo[1], oo[2], gr)
            torch.cuda.synchronize()
            dtg = time.perf_counter() - t0g
            prof = native.profile_end(bu) if profile else None
            return {"value": len(ks) * nsteps / dtg, "unit": "adjoint solves/s", "ms_per_batch": 1e3 * dtg / nsteps}, prof

        gf, (gms, gl) = run_big(native.ADJ_FP64, 3, 1, profile="S")
        gm, (gmms, gml) = run_big(native.ADJ_MIXED, 3, 1, profile="S")
        gbytes = s_product_bytes(binfo)
        gbytes32 = binfo["nnz_S"] * (4 + 4) + (binfo["n_verts"] + 1) * 8 + 2 * 3 * binfo["n_verts"] * 8
        big = {"n_scenes": len(ks), "n_verts": binfo["n_verts"], "n_tets": binfo["n_tets"],
               "fp64": gf | {"s_product_GB/s": gbytes / (gms / max(gl, 1) * 1e-3) / 1e9,
                             "s_product_frac": gbytes / (gms / max(gl, 1) * 1e-3) / 1e9 / HBM_PEAK_GBPS},
               "mixed": gm | {"s_product_GB/s": gbytes32 / (gmms / max(gml, 1) * 1e-3) / 1e9,
                              "s_product_frac": gbytes32 / (gmms / max(gml, 1) * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                              "speedup_vs_fp64": gm["value"] / gf["value"]}}
        bb.close()

    # ---- each scene alone (single-scene path) ----
    scene = native.Scene(spec.mesh.rest, spec.mesh.tets, spec.density, spec.h, spec.eps, spec.E, spec.nu,
                         spec.gravity, spec.planes, spec.contact_margin, max_c)
    z = torch.zeros_like(gq)
    dqbar, dvbar, dfext = torch.empty_like(gq), torch.empty_like(gq), torch.empty_like(gq)
    grad3 = torch.zeros(3, dtype=torch.float64, device=dev)
    opts = native.solve_opts(rtol=args.rtol, maxit=5000, restart=64)
    tuning = native.get_tuning(scene)
    if not args.no_autotune:
        native.adjoint_setup(scene, dstates[0]["cs"], dstates[0]["q"], opts)
        tuning = native.autotune(scene, gq, gv, z, opts, reps=3)

    def run_single(prec):
        o = native.solve_opts(rtol=args.rtol, maxit=5000, restart=64, prec=prec, max_refine=8)
        its = []
        t0s = time.perf_counter()
        for i in range(args.warmup + args.steps):
            if i == args.warmup:
                torch.cuda.synchronize()
                its.clear()
                t0s = time.perf_counter()
            t = dstates[i % len(dstates)]
            native.adjoint_setup(scene, t["cs"], t["q"], o)
            info_s = native.adjoint_solve(scene, gq, gv, z, o)
            native.vjp_params(scene, z, gv, dqbar, dvbar, dfext, grad3)
            its.append(info_s.iters)
        torch.cuda.synchronize()
        dts = time.perf_counter() - t0s
        return {"value": args.steps / dts, "unit": "adjoint solves/s", "ms_per_step": 1e3 * dts / args.steps,
                "krylov_iters_mean": float(np.mean(its))}

    single = run_single(native.ADJ_FP64)
    single_mixed = run_single(native.ADJ_MIXED)
    single_mixed_pc = run_single(native.ADJ_MIXED_PC)

    # ---- the slip onsets: the converged oracle states around the steps
    # where the beam starts to slide (mu 0.1, steps 20-25; mu 0.4, steps
    # 84-89), each solve checked against the oracle's stored z ----
    onset = load_onset_states()
    oz = np.load(os.path.join(ROOT, "tests", "golden", "beam_onset_z.npz"))
    for st in onset:
        n = int(st["vid"].shape[0])
        st["dev"] = {"vid": torch.tensor(st["vid"].astype(np.int32), device=dev),
                     "fric": torch.tensor(st["fric"].astype(np.int32), device=dev),
                     "frame": torch.tensor(st["frame"].reshape(n, 9), dtype=torch.float64, device=dev),
                     "delta": torch.tensor(st["delta"], dtype=torch.float64, device=dev),
                     "lam": torch.tensor(st["lam"], dtype=torch.float64, device=dev),
                     "q": torch.tensor(st["q"], dtype=torch.float64, device=dev)}
        t = st["dev"]
        t["cs"] = native.make_contact_state(n, t["vid"], t["fric"], t["frame"], t["delta"], t["lam"], st["mu"])

    def run_onset(prec):
        o = native.solve_opts(rtol=args.rtol, maxit=5000, restart=64, prec=prec, max_refine=8)
        its, errs = [], []
        for st in onset:  # untimed pass: the error of every solve against the oracle
            native.adjoint_setup(scene, st["dev"]["cs"], st["dev"]["q"], o)
            native.adjoint_solve(scene, gq, gv, z, o)
            torch.cuda.synchronize()
            errs.append(_rel(z.cpu().numpy(), oz["z"][st["index"]]))
        torch.cuda.synchronize()
        t0s = time.perf_counter()
        nrep = max(1, args.steps // len(onset))
        for _ in range(nrep):
            for st in onset:
                native.adjoint_setup(scene, st["dev"]["cs"], st["dev"]["q"], o)
                inf = native.adjoint_solve(scene, gq, gv, z, o)
                native.vjp_params(scene, z, gv, dqbar, dvbar, dfext, grad3)
                its.append(inf.iters)
        torch.cuda.synchronize()
        dts = time.perf_counter() - t0s
        nsolve = nrep * len(onset)
        return {"value": nsolve / dts, "unit": "adjoint solves/s", "ms_per_step": 1e3 * dts / nsolve,
                "krylov_iters_mean": float(np.mean(its)), "z_rel_err_vs_oracle_max": float(max(errs))}

    onset_fp64 = run_onset(native.ADJ_FP64)
    onset_mixed = run_onset(native.ADJ_MIXED)
    onset_mixed_pc = run_onset(native.ADJ_MIXED_PC)
    slip_onset = {"steps": [f"mu={st['mu']} t={st['t']}" for st in onset], "fp64": onset_fp64,
                  "mixed": onset_mixed | {"speedup_vs_fp64": onset_mixed["value"] / onset_fp64["value"]},
                  "mixed_pc": onset_mixed_pc | {"speedup_vs_fp64": onset_mixed_pc["value"] / onset_fp64["value"]},
                  "note": "single scene, the oracle's converged states around the slip onsets "
                          "(tests/golden/beam_onset_mu*.npz), g_q = r, g_v = 0; z error against the oracle's "
                          "stored solutions (tests/golden/beam_onset_z.npz)"}
    print(f"slip onset: FP64 {onset_fp64['value']:.0f} solves/s (z err {onset_fp64['z_rel_err_vs_oracle_max']:.1e}), "
          f"mixed {onset_mixed['value']:.0f} (z err {onset_mixed['z_rel_err_vs_oracle_max']:.1e}), mixed_pc "
          f"{onset_mixed_pc['value']:.0f} (z err {onset_mixed_pc['z_rel_err_vs_oracle_max']:.1e})",
          file=sys.stderr, flush=True)

    # ---- backward-solver comparison: the same solves with the comparison
    # preconditioners (sparse inverse S^T S alone, block Jacobi), 2000
    # iterations at most; the setup skips the Woodbury factors for them ----
    def run_precond(pc, nsteps, method=native.ADJ_AUTO):
        o = native.solve_opts(rtol=args.rtol, maxit=2000, restart=64, precond=pc, method=method)
        its, conv, worst = [], 0, 0.0
        for i in range(2):  # warm-up
            t = dstates[i % len(dstates)]
            native.adjoint_setup(scene, t["cs"], t["q"], o)
            native.adjoint_solve(scene, gq, gv, z, o, raise_noconv=False)
        torch.cuda.synchronize()
        t0p = time.perf_counter()
        for i in range(nsteps):
            t = dstates[i % len(dstates)]
            native.adjoint_setup(scene, t["cs"], t["q"], o)
            inf = native.adjoint_solve(scene, gq, gv, z, o, raise_noconv=False)
            native.vjp_params(scene, z, gv, dqbar, dvbar, dfext, grad3)
            its.append(inf.iters)
            conv += int(inf.relres <= args.rtol)
            worst = max(worst, inf.relres)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0p
        return {"value": nsteps / dtp, "unit": "adjoint solves/s", "krylov_iters_mean": float(np.mean(its)),
                "converged": f"{conv}/{nsteps}", "max_relres": worst}

    n_pc = min(args.steps, len(dstates))
    precond_cmp = {"woodbury": run_precond(native.PRECOND_WOODBURY, n_pc),
                   "sparse_inverse_only": run_precond(native.PRECOND_SPARSE_INVERSE, n_pc),
                   "block_jacobi": run_precond(native.PRECOND_JACOBI, n_pc),
                   "point_jacobi": run_precond(native.PRECOND_POINT_JACOBI, n_pc),
                   "semi_implicit": run_precond(native.PRECOND_SPARSE_INVERSE, n_pc, native.ADJ_SEMI_IMPLICIT)}

    # ---- bilateral bindings: the beam's x = 0 end face held by compliant
    # bindings to its rest positions (the binding term changes only the
    # diagonal of the prefactored matrix and of the assembled blocks, so the
    # recorded contact states serve as they are) ----
    rest = spec.mesh.rest
    bvid = np.flatnonzero(np.isclose(rest[:, 0], rest[:, 0].min())).astype(np.int32)
    bE = 1e-6
    bscene = native.Scene(rest, spec.mesh.tets, spec.density, spec.h, spec.eps, spec.E, spec.nu, spec.gravity,
                          spec.planes, spec.contact_margin, max_c, bindings=(bvid, bE))
    btarget = torch.tensor(rest[bvid], dtype=torch.float64, device=dev)
    bdt = torch.empty_like(btarget)
    bdE = torch.empty(bvid.size, dtype=torch.float64, device=dev)

    def run_bound(nsteps, warm):
        o = native.solve_opts(rtol=args.rtol, maxit=5000, restart=64)
        its = []
        t0b = time.perf_counter()
        for i in range(warm + nsteps):
            if i == warm:
                torch.cuda.synchronize()
                its.clear()
                t0b = time.perf_counter()
            t = dstates[i % len(dstates)]
            native.adjoint_setup(bscene, t["cs"], t["q"], o)
            inf = native.adjoint_solve(bscene, gq, gv, z, o)
            native.vjp_params(bscene, z, gv, dqbar, dvbar, dfext, grad3)
            native.binding_vjp(bscene, z, t["q"], btarget, bdt, bdE)
            its.append(inf.iters)
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t0b
        return {"value": nsteps / dtb, "unit": "adjoint solves/s", "ms_per_step": 1e3 * dtb / nsteps,
                "krylov_iters_mean": float(np.mean(its))}

    bound = run_bound(args.steps, args.warmup) | {
        "n_bindings": int(bvid.size), "binding_compliance": bE,
        "vs_unbound_single_scene_fp64": None}
    bound["vs_unbound_single_scene_fp64"] = bound["value"] / single["value"]
    bscene.close()

    # ---- material models of the local step: the same single-scene solves
    # with the as-rigid-as-possible and co-rotational projections ----
    def run_material(code, nsteps, warm):
        mscene = native.Scene(spec.mesh.rest, spec.mesh.tets, spec.density, spec.h, spec.eps, spec.E, spec.nu,
                              spec.gravity, spec.planes, spec.contact_margin, max_c, material=code)
        o = native.solve_opts(rtol=args.rtol, maxit=5000, restart=64)
        its = []
        t0m = time.perf_counter()
        for i in range(warm + nsteps):
            if i == warm:
                torch.cuda.synchronize()
                its.clear()
                t0m = time.perf_counter()
            t = dstates[i % len(dstates)]
            native.adjoint_setup(mscene, t["cs"], t["q"], o)
            inf = native.adjoint_solve(mscene, gq, gv, z, o)
            native.vjp_params(mscene, z, gv, dqbar, dvbar, dfext, grad3)
            its.append(inf.iters)
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t0m
        mscene.close()
        return {"value": nsteps / dtm, "unit": "adjoint solves/s", "krylov_iters_mean": float(np.mean(its))}

    materials = {"neo_hookean": {"value": single["value"], "unit": "adjoint solves/s",
                                 "krylov_iters_mean": single["krylov_iters_mean"]},
                 "arap": run_material(native.MAT_ARAP, args.steps, args.warmup),
                 "corotational": run_material(native.MAT_COROT, args.steps, args.warmup)}

    abytes = s_product_bytes(uinfo)
    avg_ms = kms / max(launches, 1)
    achieved = abytes / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    mv_bytes = bsr_bytes(uinfo)
    mv_avg = mv_ms / max(mv_launch, 1)
    roof_s = {
        "kernel": "sparse-inverse product S x (kb_spmv_tasks, batched, three beams)",
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBPS,
        "traffic": measured_traffic("s_product"),
        "algorithmic_bytes_per_launch": abytes,
        "avg_launch_us": 1e3 * avg_ms,
        "launches_timed": launches,
        "kernel_ms_per_batch_incl_transpose": (kms / max(args.steps, 1)) + st_ms / max(nprof, 1),
    }
    gj_avg = gj_ms / max(gj_launch, 1)
    gj_bpl = gj_b / max(gj_launch, 1)
    gj_ach = gj_bpl / (gj_avg * 1e-3) / 1e9 if gj_launch else 0.0
    roof_gj = {
        "kernel": "Gauss-Jordan block step of the capacitance inverse (kb_gj_step_mfma, batched, three beams)",
        "bound": "hbm",
        "achieved": gj_ach,
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": gj_ach / HBM_PEAK_GBPS,
        "traffic": measured_traffic("gj_step"),
        "algorithmic_bytes_per_launch": gj_bpl,
        "avg_launch_us": 1e3 * gj_avg,
        "launches_timed": gj_launch,
        "fp64_tflops": gj_f / max(gj_launch, 1) / (gj_avg * 1e-3) / 1e12 if gj_launch else 0.0,
        "kernel_ms_per_batch": gj_ms / max(nprof, 1),
    }
    # the dominant kernel is the one with the larger total time per batch
    if roof_gj["kernel_ms_per_batch"] >= roof_s["kernel_ms_per_batch_incl_transpose"]:
        roofline, roofline_other = roof_gj, roof_s
    else:
        roofline, roofline_other = roof_s, roof_gj
    out = {
        "metric": METRIC,
        "value": rev["value"],
        "unit": "adjoint solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rev["ms_per_time_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "beam 32x8x8 cells (12,288 tets, 2,673 vertices), E=1e6 Pa, nu=0.45, on the ground under "
                        "a sideways push; three runs at mu 1.0 / 0.1 / 0.4, recorded steps 0-3 of each; reverse "
                        "pass over the recorded steps (each step's right-hand side from the next step's gradient "
                        "contractions), the three runs batched per step, the next step's setup on a second stream "
                        "while a step is solved; plain FP64, GMRES(64) + Woodbury to rel. residual 1e-8; one "
                        "bench step = one time step of the pass = three adjoint solves (setup + solve + VJP)",
            "n_scene_steps": len(states),
            "scenes_per_batch": len(MUS),
            "time_steps_per_pass": T,
            "contacts_per_scene": int(states[0]["vid"].shape[0]),
            "krylov_iters_mean": rev["krylov_iters_mean"],
            "single_scene_tuning": tuning,
        },
        "roofline": roofline,
        "roofline_other": roofline_other,
        "matvec": {"kernel": "Acal^T product fused with the first Gram-Schmidt dots (batched)",
                   "bytes_per_launch": mv_bytes, "avg_launch_us": 1e3 * mv_avg,
                   "GB/s": mv_bytes / (mv_avg * 1e-3) / 1e9 if mv_launch else None},
        "reverse_pass": {"pipelined_fp64": rev, "pipelined_mixed": rev_mixed, "stepwise_fp64": rev_step,
                         "pipelining_speedup": rev["value"] / rev_step["value"],
                         "mixed_speedup": rev_mixed["value"] / rev["value"]},
        "batched_per_step": {"note": "one batch per recorded time step, the same right-hand side every step "
                                     "(the roofline kernels are timed here)",
                             "fp64": bfp64, "mixed": bmixed | {"speedup_vs_fp64": bmixed["value"] / bfp64["value"]}},
        "single_scene": {"fp64": single, "mixed": single_mixed,
                         "mixed_pc": single_mixed_pc | {"speedup_vs_fp64": single_mixed_pc["value"] / single["value"]},
                         "batched_speedup_fp64": bfp64["value"] / single["value"]},
        "slip_onset": slip_onset,
        "preconditioners": precond_cmp | {"note": "single scene, FP64, one solve per recorded scene-step, "
                                                  "GMRES(64) to 1e-8 or 2000 iterations; semi_implicit: the "
                                                  "fixed-point iteration x <- x + A^-1 (b - Acal^T x), stopped "
                                                  "when its residual exceeds 1e6 |b|"},
        "large_batch": big,
        "materials": materials | {"note": "single scene, FP64, GMRES(64) + Woodbury to 1e-8, the recorded beam "
                                          "states with the local step of each model (the states were converged "
                                          "with Neo-Hookean; the adjoint system is defined at any state)"},
        "bindings": bound | {"note": "single scene, FP64, the beam's 81 x = 0 face vertices bound to their rest "
                                     "positions (compliance 1e-6 m/N), GMRES(64) + Woodbury to 1e-8; setup + "
                                     "solve + VJP + binding VJP per recorded scene-step"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline_beam"] = cpu_baseline(spec, states, args.cpu_sample)
    scene.close()
    batch.close()
    torch.cuda.synchronize()
    for k in ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline", "data"):
        out.pop(k, None)
    return out




def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--cpu-sample", type=int, default=40,
                    help="scene-steps the oracle solves for the beam legs' baseline (cycling over the recorded ones)")
    ap.add_argument("--cpu-boxes", type=int, default=16,
                    help="boxes of the batched workload the oracle solves for the all-core baseline (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--eps-sweep", type=float, default=0.0, metavar="SECONDS",
                    help="instead of the benchmark: the smoothing sweep on the slope cube, SECONDS of simulated "
                         "time per run on the GPU forward step")
    ap.add_argument("--slab-only", action="store_true",
                    help="only the headline (the full-size slab), without the beam, boxes and oracle legs")
    ap.add_argument("--no-beam", action="store_true", help="skip the beam legs")
    ap.add_argument("--quadruped", type=int, default=0, metavar="STEPS",
                    help="instead of the benchmark: the actuated quadruped rollout and its actuation gradient")
    ap.add_argument("--boxes", type=int, default=256,
                    help="boxes of the batched-workload leg (first of the seeded 256, all of them by default; "
                         "0: skip)")
    ap.add_argument("--boxes-only", action="store_true",
                    help="instead of the benchmark: only the batched-workload leg, printed as one JSON line")
    ap.add_argument("--eps-sweep-one", nargs=3, metavar=("TWO_EPS2", "SIDE", "SECONDS"), help=argparse.SUPPRESS)
    ap.add_argument("--big-batch", type=int, default=4,
                    help="copies of the twelve recorded scene-steps in the large-batch leg (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.slab_only:
        print(json.dumps(slab_headline(args)))
        return
    if args.quadruped > 0:
        print(json.dumps(quadruped_leg(args.quadruped, max(1, args.quadruped // 4))))
        return
    if args.boxes_only:
        print(json.dumps(boxes_leg(args.boxes, max(1, args.steps // 10))))
        return
    if args.eps_sweep_one:
        eps_sweep_one(float(args.eps_sweep_one[0]), args.eps_sweep_one[1], float(args.eps_sweep_one[2]))
        return
    if args.eps_sweep > 0:
        eps_sweep(args.eps_sweep)
        return

    line = slab_headline(args)
    if not args.no_beam:
        line["beam"] = beam_legs(args)
    if args.boxes > 0:
        line["batched_boxes"] = boxes_leg(args.boxes, 2)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = slab_cpu_baseline(args)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
