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

import numpy as np

from . import mpm as M


class RigidPath:
    """The initial pose and twist of a scene's rigid bodies. Host step j of a
    kinematic body's path is its initial state advanced by j host steps of the
    library's kinematic rule (mpm_set_rigid_state); static bodies stay put."""

    def __init__(self, scene):
        self.dT = scene.N * scene.h
        self.bodies = [(tuple(r.R), tuple(r.t), tuple(r.V), tuple(r.w), r.motion) for r in scene.rigids]

    def state(self, i: int, V=None, W=None):
        """Initial state of body i, with the linear (V) and angular (W)
        velocity replaced when given."""
        R, t, V0, w0, motion = self.bodies[i]
        s = M.RigidState()
        s.R[:] = list(R)
        s.t[:] = list(t)
        s.V[:] = list(V0 if V is None else (float(a) for a in V))
        s.w[:] = list(w0 if W is None else (float(a) for a in W))
        return s


def _run(sim, path, n_steps, step0, x, v, F, C, V, W=None, record: bool = False) -> None:
    sim.load_state(x, v, F, C)
    sim.tape_reset(record)
    Vn = V.detach().cpu().numpy().astype(np.float64).reshape(-1, 3)
    Wn = None if W is None else W.detach().cpu().numpy().astype(np.float64).reshape(-1, 3)
    for i in range(len(path.bodies)):
        # the body's initial state, advanced to host step step0 by the library
        sim.set_rigid_state(i, path.state(i, Vn[i], None if Wn is None else Wn[i]), step0)
    for j in range(n_steps):
        status, _, _ = sim.step()
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
            # the library's adjoints of the twist of each body's initial state
            # (the reference set in _run), through every host step up to the
            # segment's end
            env_grads, rig = sim.backward(*g)
            dE = torch.tensor([e[0] for e in env_grads], dtype=E.dtype, device=E.device)
            dV = torch.from_numpy(rig["dV_kinematic"]).to(dtype=V.dtype, device=V.device)
            dW = None
            if W is not None:
                dW = torch.from_numpy(rig["dw_kinematic"]).to(dtype=W.dtype, device=W.device)
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
