"""The differentiable configuration's Jacobian at a reduced size against
central finite differences of the FP64 oracle (stored by
tests/golden/make_c5_jacobian.py): 20,000 particles of the elastic cube with
the box started 2 mm inside it, one host step of 10 substeps, d(mean x, y, z
after the host step) with respect to (initial velocity offset x, y, z; Young's
modulus; box velocity x, y, z), through the torch.autograd path (one reverse
pass per row). Each column within 1e-3 of its largest entry.

Run on an MI355X: python -m pytest tests -m gpu
"""
import os
import sys

import numpy as np
import pytest

from paper_2503_05046_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_jacobian_20k.npz")


def test_c5_jacobian_reduced_size():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_05046_amd import diff
    from paper_2503_05046_amd import mpm as M
    M.load()
    ref = np.load(GOLDEN)
    scene = I.differentiable(n_particles=int(ref["n_particles"]))
    r = scene.rigids[0]
    scene.rigids[0] = type(r)(**{**r.__dict__, "t": (r.t[0] + float(ref["overlap"]), r.t[1], r.t[2])})
    scene.eps_r = 1e-10
    scene.max_iter = 2_000_000
    assert scene.N == int(ref["substeps"])
    sim = M.Sim(scene, tape_substeps=scene.N)
    path = diff.RigidPath(scene)
    dev = sim.device
    x0, v0, F0, C0 = (torch.from_numpy(a).to(dev) for a in (scene.x, scene.v, scene.F, scene.C))
    u = torch.zeros(3, dtype=torch.float32, device=dev, requires_grad=True)
    E = torch.tensor([scene.envs[0].E], dtype=torch.float64, requires_grad=True)
    V = torch.tensor([list(q.V) for q in scene.rigids], dtype=torch.float64, requires_grad=True)
    x, v, F, C = diff.simulate(sim, path, 1, 1, x0, v0 + u[:, None], F0, C0, E, V)
    com = x.mean(dim=1)
    J = np.zeros((3, 7))
    for a in range(3):
        gu, gE, gV = torch.autograd.grad(com[a], (u, E, V), retain_graph=a < 2)
        J[a] = [*gu.cpu().numpy().astype(np.float64), float(gE[0]), *gV[0].numpy()]
    sim.close()
    Jf = ref["J"]
    print(f"GPU adjoint:\n{J}\noracle central differences:\n{Jf}", flush=True)
    sys.stdout.flush()
    for k in range(7):
        scale = np.abs(Jf[:, k]).max()
        assert scale > 0.0, k
        assert np.abs(J[:, k] - Jf[:, k]).max() <= 1e-3 * scale, (k, J[:, k], Jf[:, k])
