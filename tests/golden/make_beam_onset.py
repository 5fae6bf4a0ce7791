"""Write tests/golden/beam_onset_mu{mu}.npz: converged beam states from the
oracle's forward rollout (32x8x8 cells, pushed sideways on the ground, the
push ramping 0 -> 50 N over 100 steps) around the step where the beam
starts to slide, steps [T0, T1) of a rollout of T1 steps: about step 22 at
mu = 0.1 and about step 86 at mu = 0.4.  Each stored step has the same keys
as tests/golden/make_beam_states.py.  Calls only oracle/ and synth/.

    python tests/golden/make_beam_onset.py MU T0 T1
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.rollout import run_forward  # noqa: E402
from synth import beam_scene  # noqa: E402


def main(mu: float, t0: int, t1: int):
    spec = beam_scene(mu=mu)
    ro = run_forward(spec, steps=t1)
    out = {"mu": mu, "t0": t0, "steps": t1 - t0}
    for t in range(t0, t1):
        rec = ro.records[t]
        cs = rec.contacts
        k = t - t0
        out[f"t{k}"] = t
        out[f"q{k}"] = ro.qs[t + 1]
        out[f"qbar{k}"] = ro.qs[t]
        out[f"vbar{k}"] = ro.vs[t]
        out[f"vid{k}"] = cs.vid
        out[f"collider{k}"] = cs.collider
        out[f"frame{k}"] = cs.frame
        out[f"d_n{k}"] = cs.d_n
        out[f"d_f{k}"] = cs.d_f
        out[f"fric{k}"] = cs.fric
        out[f"delta{k}"] = rec.delta
        out[f"lam{k}"] = rec.lam
        out[f"resid{k}"] = rec.residual
    for t, rec in enumerate(ro.records):
        lam = rec.lam
        slip = int(np.sum(np.hypot(lam[:, 1], lam[:, 2]) > 0.99 * mu * lam[:, 0])) if rec.contacts.n else 0
        print(f"mu={mu} step {t}: contacts {rec.contacts.n} frictional {int(rec.contacts.fric.sum())} at the "
              f"friction bound {slip} newton {rec.newton_iters} residual {rec.residual:.2e}", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"beam_onset_mu{mu}.npz")
    np.savez_compressed(path, **out)
    print("wrote", path)


if __name__ == "__main__":
    main(float(sys.argv[1]), int(sys.argv[2]), int(sys.argv[3]))
