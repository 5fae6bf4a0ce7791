"""Write tests/golden/batch_contacts.npz: for each box of the seeded 256-box
batched workload, the ground contacts that the oracle's detection finds at
the seeded deformed state synth.perturbed_state(spec, seed=100 + k) for the
first step.  Calls only oracle/ and synth/.

    python tests/golden/make_batch_contacts.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.contact import detect, predict  # noqa: E402
from synth.configs import batched_scenes, perturbed_state  # noqa: E402


def main():
    specs = batched_scenes(256, seed=3, tmax=1e5)
    off, vid, fric, frame = [0], [], [], []
    for k, spec in enumerate(specs):
        q = perturbed_state(spec, seed=100 + k)
        qt = predict(q, np.zeros_like(q), np.broadcast_to(spec.gravity, q.shape), spec.h)
        cs = detect(q, qt, spec.planes, np.zeros((0, 4)), np.zeros((0, 4)), spec.contact_margin)
        vid.append(cs.vid)
        fric.append(cs.fric)
        frame.append(cs.frame.reshape(-1, 9))
        off.append(off[-1] + cs.n)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_contacts.npz")
    np.savez_compressed(path, off=np.array(off, np.int64), vid=np.concatenate(vid).astype(np.int32),
                        fric=np.concatenate(fric), frame=np.concatenate(frame))
    print(f"{len(specs)} boxes, {off[-1]} contacts; wrote {path}")


if __name__ == "__main__":
    main()
