"""The torch.autograd path (checkpointed segments over the library's reverse
pass) against central finite differences of the FP64 oracle.

Two segments of one host step each (two substeps per host step) over a scene
in contact with a half-space and a rotating, moving box; the loss is
c . (mean particle position after both segments). Gradients: with respect to
a uniform offset of every particle's initial velocity, Young's modulus, and
the box's velocity and angular velocity (which also move and turn the box
between host steps, across the segment boundary).

Run on an MI355X: python -m pytest tests -m gpu
"""
import numpy as np
import pytest

from paper_2503_05046_amd import inputs as I

pytestmark = pytest.mark.gpu

C_LOSS = np.array([0.3, -0.5, 0.8])
SEGMENTS = 2


@pytest.fixture(scope="module")
def torch_mpm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_05046_amd import mpm as M
    M.load()
    return torch, M


def _scene():
    s = I.tiny_random(P=300, seed=13, n=16, material=I.FIXED_COROTATED, with_box=True)
    s.envs[0].eps_s = 1e-2
    s.N = 2
    s.eps_r = 1e-12
    s.max_iter = 400000
    return s


def _oracle_loss(oracle, scene, du=None, dE=0.0, dV=None, dW=None):
    s = scene.copy()
    s.envs[0].E += dE
    if dV is not None:
        r = s.rigids[1]
        s.rigids[1] = type(r)(**{**r.__dict__, "V": tuple(np.array(r.V) + dV)})
    if dW is not None:
        r = s.rigids[1]
        s.rigids[1] = type(r)(**{**r.__dict__, "w": tuple(np.array(r.w) + dW)})
    ora = oracle.OracleSim(s)
    if du is not None:
        ora.v += du[:, None]
    for _ in range(SEGMENTS):
        rc, _, _ = ora.host_step()
        assert rc == 0
    return float(C_LOSS @ ora.x.mean(axis=1))


def test_autograd_segments_match_finite_differences(torch_mpm, oracle):
    torch, M = torch_mpm
    from paper_2503_05046_amd import diff
    scene = _scene()
    gpu_scene = scene.copy()
    gpu_scene.eps_r = 1e-10
    sim = M.Sim(gpu_scene, tape_substeps=scene.N)
    path = diff.RigidPath(scene)
    dev = sim.device
    x0, v0, F0, C0 = (torch.from_numpy(a).to(dev) for a in (scene.x, scene.v, scene.F, scene.C))
    u = torch.zeros(3, dtype=torch.float32, device=dev, requires_grad=True)
    E = torch.tensor([scene.envs[0].E], dtype=torch.float64, requires_grad=True)
    V = torch.tensor([list(r.V) for r in scene.rigids], dtype=torch.float64, requires_grad=True)
    Wt = torch.tensor([list(r.w) for r in scene.rigids], dtype=torch.float64, requires_grad=True)
    x, v, F, C = diff.simulate(sim, path, SEGMENTS, 1, x0, v0 + u[:, None], F0, C0, E, V, Wt)
    loss = (torch.from_numpy(C_LOSS).to(dev, torch.float32) * x.mean(dim=1)).sum()
    loss.backward()
    sim.close()
    g_u = u.grad.cpu().numpy().astype(np.float64)
    g_E = float(E.grad[0])
    g_V = V.grad[1].numpy()
    g_W = Wt.grad[1].numpy()
    eps = 1e-6
    fd_u = np.array([(_oracle_loss(oracle, scene, du=eps * np.eye(3)[k]) -
                      _oracle_loss(oracle, scene, du=-eps * np.eye(3)[k])) / (2 * eps) for k in range(3)])
    eE = 1e-6 * scene.envs[0].E
    fd_E = (_oracle_loss(oracle, scene, dE=eE) - _oracle_loss(oracle, scene, dE=-eE)) / (2 * eE)
    fd_V = np.array([(_oracle_loss(oracle, scene, dV=eps * np.eye(3)[k]) -
                      _oracle_loss(oracle, scene, dV=-eps * np.eye(3)[k])) / (2 * eps) for k in range(3)])
    fd_W = np.array([(_oracle_loss(oracle, scene, dW=eps * np.eye(3)[k]) -
                      _oracle_loss(oracle, scene, dW=-eps * np.eye(3)[k])) / (2 * eps) for k in range(3)])
    print(f"du: gpu {g_u} fd {fd_u}\ndE: gpu {g_E:.6e} fd {fd_E:.6e}\ndV: gpu {g_V} fd {fd_V}\n"
          f"dW: gpu {g_W} fd {fd_W}", flush=True)
    assert np.abs(g_u - fd_u).max() <= 1e-3 * np.abs(fd_u).max()
    assert abs(g_E - fd_E) <= 1e-3 * abs(fd_E) + 1e-14
    assert np.abs(g_V - fd_V).max() <= 1e-3 * np.abs(fd_V).max()
    assert np.abs(g_W - fd_W).max() <= 1e-3 * np.abs(fd_W).max()
    assert np.all(V.grad[0].numpy() == 0.0)  # static half-space
    assert np.all(Wt.grad[0].numpy() == 0.0)
