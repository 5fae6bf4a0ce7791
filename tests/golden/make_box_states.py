"""Write tests/golden/boxes8_states.npz: one converged step of the oracle's
forward solver for each of the first eight boxes of the reduced batched
workload (synth.batched_scenes(8, seed=3, tmax=8000)), started from rest
positions with the seeded tangential velocities: the converged positions
and each step's contact record.  Calls only oracle/ and synth/.

    python tests/golden/make_box_states.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.forward import solve_step  # noqa: E402
from oracle.rollout import scene_disc  # noqa: E402
from synth.configs import batched_scenes  # noqa: E402


def main():
    arrays = {}
    for k, spec in enumerate(batched_scenes(8, seed=3, tmax=8000)):
        disc = scene_disc(spec)
        q, _, rec, _ = solve_step(disc, spec.q0, spec.v0, spec.force(0), spec.gravity, spec.mu, spec.eps,
                                  spec.planes, margin=spec.contact_margin)
        cs = rec.contacts
        print(f"{spec.name}: verts {spec.n_verts}, contacts {cs.n}, frictional {int(cs.fric.sum())}", flush=True)
        for key, val in (("q", q), ("vid", cs.vid), ("collider", cs.collider), ("frame", cs.frame), ("d_n", cs.d_n),
                         ("d_f", cs.d_f), ("fric", cs.fric), ("delta", rec.delta), ("lam", rec.lam)):
            arrays[f"{key}{k}"] = val
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "boxes8_states.npz")
    np.savez_compressed(path, **arrays)
    print("wrote", path)


if __name__ == "__main__":
    main()
