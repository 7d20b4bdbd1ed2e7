"""Differentiable host steps for PyTorch.

`segment(sim, path, n_steps, step0, x, v, F, C, E, V, W=None)` advances a simulation by
n_steps host steps as a `torch.autograd.Function`. The forward pass keeps only
its inputs (a checkpoint); the backward pass restores them, runs the segment
again while the library records its tape, and calls the library's reverse
pass (`mpm_step_backward`). Chaining segments of K host steps therefore holds
one segment's tape at a time: checkpointing every K * N substeps.

The state tensors are [3|9, P] in the caller's particle order (the library's
internal cell order is undone on the way out and in). `E` holds Young's
modulus per environment: it must equal the modulus the simulation was created
with (the library's material table is fixed at creation), and it receives
dL/dE. `V` holds the linear velocity of every rigid body ([n_rigid, 3]; rows
of static bodies are ignored) and receives dL/dV: kinematic bodies move with
V and turn with their angular velocity from their initial pose, so the
derivative includes the effect of V on the poses of later host steps. `W`,
if given, holds the angular velocities ([n_rigid, 3], replacing the scene's)
and receives dL/dW in the same way: through the velocity field V + W x (x - t)
and through the turn of later poses.
Every step of the computation runs in the HIP library.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs as I
from . import mpm as M


def _rotation(w, angle_scale: float) -> np.ndarray:
    """Rotation by the angle |w| * angle_scale about w (Rodrigues)."""
    w = np.asarray(w, np.float64)
    wn = float(np.linalg.norm(w))
    th = wn * angle_scale
    if th == 0.0:
        return np.eye(3)
    k = w / wn
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + math.sin(th) * K + (1.0 - math.cos(th)) * (K @ K)


class RigidPath:
    """Poses and twists of a scene's rigid bodies at every host step: static
    bodies stay at their pose; kinematic bodies translate by N h V and turn
    by N h w per host step, from their initial pose."""

    def __init__(self, scene):
        self.dT = scene.N * scene.h
        self.bodies = [(np.array(r.R, np.float64).reshape(3, 3), np.array(r.t, np.float64),
                        np.array(r.w, np.float64), r.motion) for r in scene.rigids]

    def states(self, step: int, V, W=None) -> list:
        out = []
        for i, (R0, t0, w, motion) in enumerate(self.bodies):
            s = M.RigidState()
            if motion == I.KINEMATIC:
                Vi = np.asarray(V[i], np.float64)
                if W is not None:
                    w = np.asarray(W[i], np.float64)
                R = _rotation(w, step * self.dT) @ R0
                t = t0 + step * self.dT * Vi
                s.V[:] = list(Vi)
                s.w[:] = list(w)
            else:
                R, t = R0, t0
            s.R[:] = list(R.reshape(-1))
            s.t[:] = list(t)
            out.append(s)
        return out


def _left_jacobian(phi) -> np.ndarray:
    """J(phi) = I + (1 - cos t)/t^2 [phi]x + (t - sin t)/t^3 [phi]x^2, t = |phi|:
    Rot(phi + d) = Rot(J(phi) d) Rot(phi) to first order in d."""
    phi = np.asarray(phi, np.float64)
    t2 = float(phi @ phi)
    t = math.sqrt(t2)
    a = 0.5 - t2 / 24.0 if t < 1e-4 else (1.0 - math.cos(t)) / t2
    b = 1.0 / 6.0 - t2 / 120.0 if t < 1e-4 else (t - math.sin(t)) / (t2 * t)
    P = np.array([[0.0, -phi[2], phi[1]], [phi[2], 0.0, -phi[0]], [-phi[1], phi[0], 0.0]])
    return np.eye(3) + a * P + b * (P @ P)


def _run(sim, path, n_steps, step0, x, v, F, C, V, W=None, record: bool = False) -> None:
    sim.load_state(x, v, F, C)
    sim.tape_reset(record)
    Vn = V.detach().cpu().numpy().astype(np.float64).reshape(-1, 3)
    Wn = None if W is None else W.detach().cpu().numpy().astype(np.float64).reshape(-1, 3)
    for j in range(n_steps):
        status, _, _ = sim.step(path.states(step0 + j, Vn, Wn))
        if status != M.MPM_OK:
            # a contact solve that stopped at its iteration cap: the implicit
            # differentiation of the recorded solve assumes its optimum
            raise M.MPMError(status, f"host step {step0 + j} of a differentiated segment"
                                     f"{' (recording)' if record else ''}")


def _make_function():
    import torch

    class Segment(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sim, path, n_steps, step0, x, v, F, C, E, V, W):
            created = np.array([e.E for e in sim.scene.envs])
            if not np.allclose(E.detach().cpu().numpy(), created, rtol=1e-12, atol=0.0):
                raise ValueError("E must equal the Young's moduli the simulation was created with")
            ctx.sim, ctx.path, ctx.n_steps, ctx.step0 = sim, path, n_steps, step0
            ctx.has_w = W is not None
            ctx.save_for_backward(x, v, F, C, E, V, W if W is not None else V)
            _run(sim, path, n_steps, step0, x, v, F, C, V, W=W, record=False)
            return sim.state_tensors()

        @staticmethod
        def backward(ctx, gx, gv, gF, gC):
            x, v, F, C, E, V, W = ctx.saved_tensors
            if not ctx.has_w:
                W = None
            sim = ctx.sim
            _run(sim, ctx.path, ctx.n_steps, ctx.step0, x, v, F, C, V, W=W, record=True)
            pid = sim.pid.long()
            g = []
            for gt, ref in ((gx, x), (gv, v), (gF, F), (gC, C)):
                if gt is None:
                    gt = torch.zeros_like(ref)
                g.append(gt.detach().to(device=sim.device, dtype=torch.float32)[:, pid].contiguous())
            env_grads, rig = sim.backward(*g)
            dE = torch.tensor([e[0] for e in env_grads], dtype=E.dtype, device=E.device)
            dV = rig["dV_kinematic"] + ctx.step0 * ctx.path.dT * rig["dt"]
            dV = torch.from_numpy(dV).to(dtype=V.dtype, device=V.device)
            dW = None
            if W is not None:
                # the segment's first pose is Rot(b w) R0, b = step0 N h; a
                # change dw turns it by b J(b w) dw, which reaches the loss
                # through the rotation adjoint dR of that pose
                b = ctx.step0 * ctx.path.dT
                Wn = W.detach().cpu().numpy().astype(np.float64).reshape(-1, 3)
                dWn = rig["dw_kinematic"].copy()
                for i in range(Wn.shape[0]):
                    dWn[i] += b * _left_jacobian(b * Wn[i]).T @ rig["dR"][i]
                dW = torch.from_numpy(dWn).to(dtype=W.dtype, device=W.device)
            out = [t.to(dtype=ref.dtype, device=ref.device) for t, ref in zip(g, (x, v, F, C))]
            return (None, None, None, None, *out, dE, dV, dW)

    return Segment


_SEGMENT = None


def segment(sim, path: RigidPath, n_steps: int, step0: int, x, v, F, C, E, V, W=None):
    """n_steps host steps from host step step0 (its rigid poses follow `path`);
    returns (x, v, F, C) after them. See the module docstring."""
    global _SEGMENT
    if _SEGMENT is None:
        _SEGMENT = _make_function()
    return _SEGMENT.apply(sim, path, n_steps, step0, x, v, F, C, E, V, W)


def simulate(sim, path: RigidPath, n_segments: int, seg_steps: int, x, v, F, C, E, V, W=None):
    """n_segments chained segments of seg_steps host steps each."""
    state = (x, v, F, C)
    for s in range(n_segments):
        state = segment(sim, path, seg_steps, s * seg_steps, *state, E, V, W)
    return state
