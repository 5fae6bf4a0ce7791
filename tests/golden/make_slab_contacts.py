"""Write tests/golden/slab_contacts.npz: the contact candidates of the
full-size slab (64x32x32 cells, sphere indenter) at the seeded perturbed
state of synth.perturbed_state, found by the oracle's detection for the
first step (ground plane and the sphere moving from its pose at step 0 to
its pose at step 1).  Calls only oracle/ and synth/.

    python tests/golden/make_slab_contacts.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.contact import detect, predict  # noqa: E402
from synth.configs import perturbed_state, slab_scene  # noqa: E402


def main():
    spec = slab_scene()
    q = perturbed_state(spec)
    qt = predict(q, np.zeros_like(q), np.broadcast_to(spec.gravity, q.shape), spec.h)
    cs = detect(q, qt, spec.planes, spec.sphere_array(0), spec.sphere_array(1), spec.contact_margin)
    print(f"slab contacts {cs.n}: {int((cs.collider == 0).sum())} ground, {int((cs.collider == 1).sum())} sphere")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "slab_contacts.npz")
    np.savez_compressed(path, vid=cs.vid, collider=cs.collider, frame=cs.frame, d_n=cs.d_n, d_f=cs.d_f,
                        fric=cs.fric)
    print("wrote", path)


if __name__ == "__main__":
    main()
