"""Writes gripper_dense_contact.npz: the FP64 oracle's result for one substep
of the gripper in dense contact (250,000 elastic particles, 96^3 grid, both
jaws started 0.065 m inside the ellipsoid's tips: about 2e4 contacts), at the
benchmark tolerance eps_r = 1e-6. Calls only the oracle and the seeded input
generator; takes a few minutes of one CPU core.

Stored: for the particles within three cells (in x) of the jaws' inner faces
(the only ones whose stencil can reach a contact node), in their original
order, the velocity after the substep (float32); the impulse and torque on
each jaw; the oracle's statistics of the substep.

    python tests/golden/make_gripper_dense.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2503_05046_amd import inputs as I  # noqa: E402

OVERLAP = 0.065
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gripper_dense_contact.npz")


def scene():
    s = I.gripper(overlap=OVERLAP)
    s.N = 1
    s.max_iter = 200_000
    return s


def near_jaws(s):
    """Particles within three cells (in x) of a jaw's inner face."""
    dx = s.envs[0].dx
    return np.abs(s.x[0].astype(np.float64) - 0.5) > 0.25 - OVERLAP - 3.0 * dx


def main():
    s = scene()
    sel = np.nonzero(near_jaws(s))[0]
    ora = O.OracleSim(s)
    t0 = time.time()
    rc, imp, st = ora.host_step()
    dt = time.time() - t0
    st = st[0]
    print(f"rc {rc}, {st['n_contacts']} contacts, {st['n_contact_nodes']} contact nodes, "
          f"{st['iterations']} iterations, {dt:.1f} s", flush=True)
    assert rc == O.OK
    np.savez_compressed(OUT, v=ora.v[:, sel].astype(np.float32), impulse=imp,
                        n_selected=len(sel), n_contacts=st["n_contacts"],
                        n_contact_nodes=st["n_contact_nodes"], iterations=st["iterations"],
                        residual=st["residual"], threshold=st["threshold"], seconds=dt)


if __name__ == "__main__":
    main()
