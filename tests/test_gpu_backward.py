"""Reverse pass of the HIP library against central finite differences of the
FP64 oracle.

Three scenes: one without contact (P2G, the grid update, G2P with the
fixed-corotated stress and the host step's sort in reverse), one in contact
with a half-space and a rotating, moving box (adding the contact solve,
differentiated at its optimum, and contact registration), and sand without
contact (the Drucker-Prager return map of the trial strain in all three of
its branches, and the Hencky stress of the projected and of the gathered F). Loss functionals
L_a = <W_a, a_final> (a in x, v, F, C, random weights W_a) after two host steps
of two substeps; for every pair (loss a, input field b) the directional
derivative of L_a along a random direction in b from mpm_step_backward is
compared with (L_a(s0 + eps d) - L_a(s0 - eps d)) / (2 eps) from the oracle.
For (x, x) and (F, F) the identity part <W_a, d> is removed from both before
the comparison, so the dynamics dominate what is checked.

Run on an MI355X: python -m pytest tests -m gpu
"""
import sys

import numpy as np
import pytest

from paper_2503_05046_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = (("x", 3), ("v", 3), ("F", 9), ("C", 9))
HOST_STEPS = 2


@pytest.fixture(scope="module")
def mpm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_05046_amd import mpm as M
    M.load()
    return M


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _free_scene(seed):
    """Random elastic state (velocities, deformations, affine matrices), no
    rigid bodies, well inside a 16^3 grid."""
    s = I.tiny_random(P=300, seed=seed, n=16, material=I.FIXED_COROTATED, with_box=False)
    s.rigids = []
    s.N = 2
    s.h = 2e-4
    return s


def _oracle_final(oracle, scene, shift=None, eps=0.0, dE=0.0, dnu=0.0):
    s = scene.copy()
    s.envs[0].E += dE
    s.envs[0].nu += dnu
    ora = oracle.OracleSim(s)
    if shift is not None:
        b, d = shift
        getattr(ora, b)[...] += eps * d
    for _ in range(HOST_STEPS):
        rc, _, _ = ora.host_step()
        assert rc == 0
    return {a: getattr(ora, a).copy() for a, _ in FIELDS}


@pytest.fixture(scope="module")
def reverse(mpm):
    """GPU adjoints dL_a/d(state0) for each loss field a, and dL_a/dE."""
    import torch
    scene = _free_scene(41)
    rng = np.random.default_rng(7)
    W = {a: rng.normal(size=(n, scene.P)) for a, n in FIELDS}
    sim = mpm.Sim(scene, tape_substeps=scene.N * HOST_STEPS)
    sim.tape_reset(True)
    for _ in range(HOST_STEPS):
        status, _, st = sim.step()
        assert status == 0 and st["max_contacts"] == 0
    pid = sim.pid.cpu().numpy()
    out = {}
    for a, _ in FIELDS:
        g = {b: torch.zeros((n, scene.P), dtype=torch.float32, device=sim.device) for b, n in FIELDS}
        g[a].copy_(torch.from_numpy(W[a][:, pid].astype(np.float32)))
        env_grads, _ = sim.backward(g["x"], g["v"], g["F"], g["C"])
        out[a] = ({b: g[b].cpu().numpy().astype(np.float64) for b, _ in FIELDS}, env_grads[0])
    sim.close()
    return scene, W, out


@pytest.mark.parametrize("a", [f for f, _ in FIELDS])
@pytest.mark.parametrize("b", [f for f, _ in FIELDS])
def test_state_gradient_matches_finite_differences(oracle, reverse, a, b):
    scene, W, out = reverse
    grad = out[a][0][b]
    names = [f for f, _ in FIELDS]
    rng = np.random.default_rng(100 + 10 * names.index(a) + names.index(b))
    d = rng.normal(size=grad.shape)
    eps = 1e-6 * (scene.envs[0].dx if b == "x" else 1.0)
    lp = (W[a] * _oracle_final(oracle, scene, (b, d), eps)[a]).sum()
    lm = (W[a] * _oracle_final(oracle, scene, (b, d), -eps)[a]).sum()
    fd = (lp - lm) / (2 * eps)
    gpu = float((grad * d).sum())
    if a == b and a in ("x", "F"):
        ident = float((W[a] * d).sum())
        fd, gpu = fd - ident, gpu - ident
    _log(f"L_{a} along d{b}: gpu {gpu:.6e} fd {fd:.6e}")
    assert abs(gpu - fd) <= 1e-3 * abs(fd) + 1e-7 * np.sqrt((W[a] ** 2).sum() * (d ** 2).sum()), (gpu, fd)


@pytest.mark.parametrize("a", [f for f, _ in FIELDS])
def test_youngs_modulus_gradient(oracle, reverse, a):
    scene, W, out = reverse
    E = scene.envs[0].E
    eps = 1e-6 * E
    lp = (W[a] * _oracle_final(oracle, scene, dE=eps)[a]).sum()
    lm = (W[a] * _oracle_final(oracle, scene, dE=-eps)[a]).sum()
    fd = (lp - lm) / (2 * eps)
    gpu = out[a][1][0]
    _log(f"dL_{a}/dE: gpu {gpu:.6e} fd {fd:.6e}")
    assert abs(gpu - fd) <= 1e-3 * abs(fd) + 1e-12, (gpu, fd)


def _contact_scene():
    """Random elastic state over a half-space, under a rotating box moving at
    (0.1, -0.05, 0) m/s: 60-65 contacts per substep. Soft friction (eps_s =
    1e-2) and tight solves keep the finite differences clean."""
    s = I.tiny_random(P=300, seed=13, n=16, material=I.FIXED_COROTATED, with_box=True)
    s.envs[0].eps_s = 1e-2
    s.N = 2
    s.eps_r = 1e-12
    s.max_iter = 400000
    return s


def _oracle_final_rigid(oracle, scene, dV=None, dw=None, dth=None):
    """The box's velocity or angular velocity shifted, or its initial pose
    turned by the rotation vector dth about its centre."""
    s = scene.copy()
    r = s.rigids[1]
    kw = dict(r.__dict__)
    if dV is not None:
        kw["V"] = tuple(np.array(r.V) + dV)
    if dw is not None:
        kw["w"] = tuple(np.array(r.w) + dw)
    if dth is not None:
        kw["R"] = tuple((_rotation(dth) @ np.array(r.R).reshape(3, 3)).reshape(-1))
    s.rigids[1] = type(r)(**kw)
    return _oracle_final(oracle, s)


def _rotation(phi):
    t = float(np.linalg.norm(phi))
    if t == 0.0:
        return np.eye(3)
    k = np.asarray(phi, np.float64) / t
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + np.sin(t) * K + (1.0 - np.cos(t)) * (K @ K)


@pytest.fixture(scope="module")
def reverse_contact(mpm):
    import torch
    scene = _contact_scene()
    rng = np.random.default_rng(8)
    W = {a: rng.normal(size=(n, scene.P)) for a, n in FIELDS}
    gpu_scene = scene.copy()
    gpu_scene.eps_r = 1e-10
    sim = mpm.Sim(gpu_scene, tape_substeps=scene.N * HOST_STEPS)
    sim.tape_reset(True)
    for _ in range(HOST_STEPS):
        status, _, st = sim.step()
        assert status == 0 and st["max_contacts"] > 0
    pid = sim.pid.cpu().numpy()
    out = {}
    for a, _ in FIELDS:
        g = {b: torch.zeros((n, scene.P), dtype=torch.float32, device=sim.device) for b, n in FIELDS}
        g[a].copy_(torch.from_numpy(W[a][:, pid].astype(np.float32)))
        env_grads, rig = sim.backward(g["x"], g["v"], g["F"], g["C"])
        out[a] = ({b: g[b].cpu().numpy().astype(np.float64) for b, _ in FIELDS}, env_grads[0], rig)
    sim.close()
    return scene, W, out


@pytest.mark.parametrize("a", [f for f, _ in FIELDS])
@pytest.mark.parametrize("b", [f for f, _ in FIELDS])
def test_contact_state_gradient_matches_finite_differences(oracle, reverse_contact, a, b):
    scene, W, out = reverse_contact
    grad = out[a][0][b]
    names = [f for f, _ in FIELDS]
    rng = np.random.default_rng(200 + 10 * names.index(a) + names.index(b))
    d = rng.normal(size=grad.shape)
    eps = 1e-6 * (scene.envs[0].dx if b == "x" else 1.0)
    lp = (W[a] * _oracle_final(oracle, scene, (b, d), eps)[a]).sum()
    lm = (W[a] * _oracle_final(oracle, scene, (b, d), -eps)[a]).sum()
    fd = (lp - lm) / (2 * eps)
    gpu = float((grad * d).sum())
    if a == b and a in ("x", "F"):
        ident = float((W[a] * d).sum())
        fd, gpu = fd - ident, gpu - ident
    _log(f"contact: L_{a} along d{b}: gpu {gpu:.6e} fd {fd:.6e}")
    assert abs(gpu - fd) <= 1e-3 * abs(fd) + 1e-7 * np.sqrt((W[a] ** 2).sum() * (d ** 2).sum()), (gpu, fd)


@pytest.mark.parametrize("a", [f for f, _ in FIELDS])
def test_contact_youngs_modulus_gradient(oracle, reverse_contact, a):
    scene, W, out = reverse_contact
    E = scene.envs[0].E
    eps = 1e-6 * E
    lp = (W[a] * _oracle_final(oracle, scene, dE=eps)[a]).sum()
    lm = (W[a] * _oracle_final(oracle, scene, dE=-eps)[a]).sum()
    fd = (lp - lm) / (2 * eps)
    gpu = out[a][1][0]
    _log(f"contact: dL_{a}/dE: gpu {gpu:.6e} fd {fd:.6e}")
    assert abs(gpu - fd) <= 1e-3 * abs(fd) + 1e-12, (gpu, fd)


@pytest.mark.parametrize("a", [f for f, _ in FIELDS])
def test_box_velocity_gradient(oracle, reverse_contact, a):
    """d L / d V of the kinematic box, through the contact bias, the lagged
    normal impulse and the box's advance between host steps."""
    scene, W, out = reverse_contact
    gpu = out[a][2]["dV_kinematic"][1]
    fd = np.zeros(3)
    for k in range(3):
        dv = np.zeros(3)
        dv[k] = 1e-6
        lp = (W[a] * _oracle_final_rigid(oracle, scene, dV=dv)[a]).sum()
        lm = (W[a] * _oracle_final_rigid(oracle, scene, dV=-dv)[a]).sum()
        fd[k] = (lp - lm) / 2e-6
    _log(f"contact: dL_{a}/dV: gpu {gpu} fd {fd}")
    assert np.abs(gpu - fd).max() <= 1e-3 * np.abs(fd).max() + 1e-9, (gpu, fd)
    assert np.all(out[a][2]["dV"][0] == 0.0)  # the half-space is static


@pytest.mark.parametrize("a", [f for f, _ in FIELDS])
@pytest.mark.parametrize("kind", ["w", "R"])
def test_box_rotation_gradient(oracle, reverse_contact, a, kind):
    """d L / d w of the kinematic box (through its velocity field in both host
    steps and through its turn before the second), and d L / d th for a
    rotation th of its initial pose about its centre (the normals, frames and
    penetrations of its contacts turn with it)."""
    scene, W, out = reverse_contact
    gpu = out[a][2]["dw_kinematic" if kind == "w" else "dR"][1]
    fd = np.zeros(3)
    for k in range(3):
        d = np.zeros(3)
        d[k] = 1e-6
        arg = "dw" if kind == "w" else "dth"
        lp = (W[a] * _oracle_final_rigid(oracle, scene, **{arg: d})[a]).sum()
        lm = (W[a] * _oracle_final_rigid(oracle, scene, **{arg: -d})[a]).sum()
        fd[k] = (lp - lm) / 2e-6
    _log(f"contact: dL_{a}/d{kind}: gpu {gpu} fd {fd}")
    assert np.abs(gpu - fd).max() <= 1e-3 * np.abs(fd).max() + 1e-9, (gpu, fd)
    for key in ("dw", "dR", "dw_kinematic"):
        assert np.all(out[a][2][key][0] == 0.0)  # the half-space is static


def _sand_scene():
    """Random sand state (Drucker-Prager, friction angle 30 degrees), no rigid
    bodies: 100 particles with velocities N(0, 0.9) m/s and random
    deformations, so that particles sit at the cone's tip, on its surface and
    inside it (elastic) in every substep."""
    s = I.tiny_random(P=100, seed=45, n=16, material=I.DRUCKER_PRAGER, with_box=False)
    s.rigids = []
    s.N = 2
    s.h = 2e-4
    s.v *= np.float32(3.0)
    return s


def _branch_margins(oracle, scene):
    """Per substep, the smallest distance of a particle's trial Hencky strain
    from the return map's branch boundaries (tr eps = 0 and the cone
    |dev eps| + kappa tr eps = 0), on the oracle's trajectory, and the count of
    particles in each branch."""
    env = scene.envs[0]
    mu = env.E / (2 * (1 + env.nu))
    la = env.E * env.nu / ((1 + env.nu) * (1 - 2 * env.nu))
    sphi = np.sin(np.radians(env.friction_angle))
    kappa = (3 * la + 2 * mu) / (2 * mu) * np.sqrt(2.0 / 3.0) * 2 * sphi / (3 - sphi)
    ora = oracle.OracleSim(scene)
    out = []
    for _ in range(scene.N * HOST_STEPS):
        F0 = ora.F.T.reshape(-1, 3, 3).copy()
        rc, _, _ = ora.substep()
        assert rc == 0
        Ft = (np.eye(3) + scene.h * ora.C.T.reshape(-1, 3, 3)) @ F0
        e = np.log(np.linalg.svd(Ft, compute_uv=False))
        tr = e.sum(axis=1)
        dg = np.linalg.norm(e - tr[:, None] / 3, axis=1) + kappa * tr
        counts = (int((tr >= 0).sum()), int(((tr < 0) & (dg > 0)).sum()), int(((tr < 0) & (dg <= 0)).sum()))
        out.append((float(np.minimum(np.abs(tr), np.abs(dg)).min()), counts))
    return out


@pytest.fixture(scope="module")
def reverse_sand(mpm, oracle):
    import torch
    scene = _sand_scene()
    margins = _branch_margins(oracle, scene)
    _log(f"sand: per substep (smallest branch margin, (tip, cone, elastic)): {margins}")
    # float32 forward and the oracle's finite differences take the same branch
    # for every particle when no trial strain lies near a boundary
    assert min(m for m, _ in margins) > 1e-5, margins
    assert all(min(c) > 0 for _, c in margins), margins
    rng = np.random.default_rng(9)
    W = {a: rng.normal(size=(n, scene.P)) for a, n in FIELDS}
    sim = mpm.Sim(scene, tape_substeps=scene.N * HOST_STEPS)
    sim.tape_reset(True)
    for _ in range(HOST_STEPS):
        status, _, st = sim.step()
        assert status == 0 and st["max_contacts"] == 0
    pid = sim.pid.cpu().numpy()
    out = {}
    for a, _ in FIELDS:
        g = {b: torch.zeros((n, scene.P), dtype=torch.float32, device=sim.device) for b, n in FIELDS}
        g[a].copy_(torch.from_numpy(W[a][:, pid].astype(np.float32)))
        env_grads, _ = sim.backward(g["x"], g["v"], g["F"], g["C"])
        out[a] = ({b: g[b].cpu().numpy().astype(np.float64) for b, _ in FIELDS}, env_grads[0])
    sim.close()
    return scene, W, out


@pytest.mark.parametrize("a", [f for f, _ in FIELDS])
@pytest.mark.parametrize("b", [f for f, _ in FIELDS])
def test_sand_state_gradient_matches_finite_differences(oracle, reverse_sand, a, b):
    scene, W, out = reverse_sand
    grad = out[a][0][b]
    names = [f for f, _ in FIELDS]
    rng = np.random.default_rng(300 + 10 * names.index(a) + names.index(b))
    d = rng.normal(size=grad.shape)
    # small steps keep every perturbed trajectory on the same branches
    eps = 1e-7 * (scene.envs[0].dx if b == "x" else 1.0)
    lp = (W[a] * _oracle_final(oracle, scene, (b, d), eps)[a]).sum()
    lm = (W[a] * _oracle_final(oracle, scene, (b, d), -eps)[a]).sum()
    fd = (lp - lm) / (2 * eps)
    gpu = float((grad * d).sum())
    if a == b and a in ("x", "F"):
        ident = float((W[a] * d).sum())
        fd, gpu = fd - ident, gpu - ident
    _log(f"sand: L_{a} along d{b}: gpu {gpu:.6e} fd {fd:.6e}")
    assert abs(gpu - fd) <= 1e-3 * abs(fd) + 1e-7 * np.sqrt((W[a] ** 2).sum() * (d ** 2).sum()), (gpu, fd)


@pytest.mark.parametrize("a", [f for f, _ in FIELDS])
def test_sand_youngs_modulus_gradient(oracle, reverse_sand, a):
    scene, W, out = reverse_sand
    E = scene.envs[0].E
    eps = 1e-7 * E
    lp = (W[a] * _oracle_final(oracle, scene, dE=eps)[a]).sum()
    lm = (W[a] * _oracle_final(oracle, scene, dE=-eps)[a]).sum()
    fd = (lp - lm) / (2 * eps)
    gpu = out[a][1][0]
    _log(f"sand: dL_{a}/dE: gpu {gpu:.6e} fd {fd:.6e}")
    assert abs(gpu - fd) <= 1e-3 * abs(fd) + 1e-12, (gpu, fd)


@pytest.mark.parametrize("a", [f for f, _ in FIELDS])
def test_sand_poisson_ratio_gradient(oracle, reverse_sand, a):
    """nu moves the cone's slope (3 la + 2 mu) alpha / (2 mu), which E leaves
    unchanged: this checks the return map's dependence on the Lame
    parameters through the cone."""
    scene, W, out = reverse_sand
    eps = 1e-7
    lp = (W[a] * _oracle_final(oracle, scene, dnu=eps)[a]).sum()
    lm = (W[a] * _oracle_final(oracle, scene, dnu=-eps)[a]).sum()
    fd = (lp - lm) / (2 * eps)
    gpu = out[a][1][1]
    _log(f"sand: dL_{a}/dnu: gpu {gpu:.6e} fd {fd:.6e}")
    assert abs(gpu - fd) <= 1e-3 * abs(fd) + 1e-9, (gpu, fd)
