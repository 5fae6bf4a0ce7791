"""Write the oracle's adjoint solutions for the full-size parity tests (calls
only oracle/ and synth/):

* slab_step50.npz: the slab (64x32x32 cells) at its last step, top face on
  the sphere (synth.slab_indented_state at the poses of steps 49 and 50), the
  contacts the oracle's detection finds for that step (ground and sphere),
  seeded sticking contact values, and z = Acal^{-T} b for the seeded right
  hand side b = r + g_v / h (direct sparse LU with long-double refinement).
* boxes16_z.npz: the same for the first 16 boxes of the batched workload at
  their seeded deformed states (one z per box, packed).
* beam_onset_z.npz: z for every converged beam step stored around the slip
  onsets (beam_onset_mu0.1.npz, beam_onset_mu0.4.npz, written by
  make_beam_onset.py), for the loss direction alone (g_q = r, g_v = 0).

    python tests/golden/make_oracle_z.py [slab] [boxes] [onset]
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint as adj  # noqa: E402
from oracle.contact import ContactSet, detect, predict  # noqa: E402
from oracle.forward import StepRecord  # noqa: E402
from oracle.rollout import scene_disc  # noqa: E402
from synth import beam_scene  # noqa: E402
from synth.configs import (batched_scenes, contact_values, perturbed_state, slab_last_step,  # noqa: E402
                           slab_scene)

HERE = os.path.dirname(os.path.abspath(__file__))


def slab_case(spec=None):
    """(spec, qbar, q, record, g_q, g_v) of the slab's measured step."""
    spec = spec or slab_scene()
    T = spec.steps
    qbar, q, gq, gv = slab_last_step(spec)
    qt = predict(qbar, np.zeros_like(qbar), np.broadcast_to(spec.gravity, qbar.shape), spec.h)
    cs = detect(qbar, qt, spec.planes, spec.sphere_array(T - 1), spec.sphere_array(T), spec.contact_margin)
    delta, lam = contact_values(cs.n, spec.mu)
    return spec, qbar, q, StepRecord(cs, delta, lam, spec.mu), gq, gv


def boxes_cases(n=16):
    out = []
    rng = np.random.default_rng(300)
    for k, spec in enumerate(batched_scenes(n, seed=3, tmax=1e5)):
        q = perturbed_state(spec, seed=100 + k)
        qt = predict(q, np.zeros_like(q), np.broadcast_to(spec.gravity, q.shape), spec.h)
        cs = detect(q, qt, spec.planes, np.zeros((0, 4)), np.zeros((0, 4)), spec.contact_margin)
        delta, lam = contact_values(cs.n, spec.mu, seed=200 + k)
        gq = rng.standard_normal(q.shape)
        gv = 1e-3 * rng.standard_normal(q.shape)
        out.append((spec, q, StepRecord(cs, delta, lam, spec.mu), gq, gv))
    return out


def _solve(spec, q, rec, gq, gv):
    disc = scene_disc(spec)
    sysm = adj.assemble(disc, q, rec, spec.eps)
    b = gq.reshape(-1) + gv.reshape(-1) / spec.h
    z = adj.solve_transposed(sysm.Acal, b)
    res = np.linalg.norm(sysm.Acal.T @ z - b) / np.linalg.norm(b)
    return z.reshape(-1, 3), res


def write_slab():
    t0 = time.time()
    spec, qbar, q, rec, gq, gv = slab_case()
    cs = rec.contacts
    print(f"slab: {cs.n} contacts ({int((cs.collider == 0).sum())} ground, {int((cs.collider == 1).sum())} "
          f"sphere), {int(cs.fric.sum())} frictional, {cs.n + 2 * int(cs.fric.sum())} rows", flush=True)
    z, res = _solve(spec, q, rec, gq, gv)
    print(f"slab: oracle residual {res:.2e}, {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "slab_step50.npz"), vid=cs.vid, collider=cs.collider, frame=cs.frame,
                        d_n=cs.d_n, d_f=cs.d_f, fric=cs.fric, z=z, residual=res)


def write_boxes():
    t0 = time.time()
    zs, res = [], []
    for spec, q, rec, gq, gv in boxes_cases():
        z, r = _solve(spec, q, rec, gq, gv)
        zs.append(z)
        res.append(r)
        print(f"{spec.name}: {spec.n_tets} tets, {rec.contacts.n} contacts, residual {r:.1e}, "
              f"{time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "boxes16_z.npz"), z=np.concatenate(zs),
                        voff=np.cumsum([0] + [z.shape[0] for z in zs]), residual=np.array(res))


def onset_cases():
    """(mu, t, q, record) of every stored slip-onset step, mu 0.1 then 0.4."""
    out = []
    for mu in (0.1, 0.4):
        d = np.load(os.path.join(HERE, f"beam_onset_mu{mu}.npz"))
        for k in range(int(d["steps"])):
            cs = ContactSet(d[f"vid{k}"], d[f"collider{k}"], d[f"frame{k}"], d[f"d_n{k}"], d[f"d_f{k}"],
                            d[f"fric{k}"].astype(bool))
            out.append((mu, int(d[f"t{k}"]), d[f"q{k}"], StepRecord(cs, d[f"delta{k}"], d[f"lam{k}"], mu)))
    return out


def write_onset():
    zs, mus, ts, res = [], [], [], []
    for mu, t, q, rec in onset_cases():
        spec = beam_scene(mu=mu)
        z, r = _solve(spec, q, rec, spec.loss_dir, np.zeros_like(q))
        zs.append(z)
        mus.append(mu)
        ts.append(t)
        res.append(r)
        print(f"beam mu={mu} step {t}: {rec.contacts.n} contacts, residual {r:.1e}", flush=True)
    np.savez_compressed(os.path.join(HERE, "beam_onset_z.npz"), z=np.stack(zs), mu=np.array(mus), t=np.array(ts),
                        residual=np.array(res))


if __name__ == "__main__":
    which = sys.argv[1:] or ["boxes", "slab", "onset"]
    if "onset" in which:
        write_onset()
    if "boxes" in which:
        write_boxes()
    if "slab" in which:
        write_slab()
