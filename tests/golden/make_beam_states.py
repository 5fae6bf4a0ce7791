"""Write tests/golden/beam_states_mu{mu}.npz: converged beam states from the
oracle (32x8x8 cells, pushed sideways on the ground) for the first steps of
each friction coefficient.  Calls only oracle/ and synth/.

    python tests/golden/make_beam_states.py MU STEPS
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.rollout import run_forward  # noqa: E402
from synth import beam_scene  # noqa: E402


def main(mu: float, steps: int):
    spec = beam_scene(mu=mu)
    ro = run_forward(spec, steps=steps)
    out = {"mu": mu, "steps": steps}
    for t, rec in enumerate(ro.records):
        cs = rec.contacts
        out[f"q{t}"] = ro.qs[t + 1]
        out[f"qbar{t}"] = ro.qs[t]
        out[f"vbar{t}"] = ro.vs[t]
        out[f"vid{t}"] = cs.vid
        out[f"collider{t}"] = cs.collider
        out[f"frame{t}"] = cs.frame
        out[f"d_n{t}"] = cs.d_n
        out[f"d_f{t}"] = cs.d_f
        out[f"fric{t}"] = cs.fric
        out[f"delta{t}"] = rec.delta
        out[f"lam{t}"] = rec.lam
        out[f"resid{t}"] = rec.residual
        print(f"mu={mu} step {t}: contacts {cs.n} frictional {int(cs.fric.sum())} "
              f"newton {rec.newton_iters} residual {rec.residual:.2e}", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"beam_states_mu{mu}.npz")
    np.savez_compressed(path, **out)
    print("wrote", path)


if __name__ == "__main__":
    main(float(sys.argv[1]), int(sys.argv[2]))
