"""Dynamic rigid bodies (the rigid side of the split integrated on the host
from each host step's impulses) through the C ABI, against the FP64 oracle.

Random elastic particles around a falling, spinning dynamic box over a
half-space: after three host steps the particle fields match the oracle at
the parity bar, and the box's twist and pose match the oracle's integration
of the same impulses. The graph path and the reverse pass refuse dynamic
bodies.

Run on an MI355X: python -m pytest tests -m gpu
"""
import sys

import numpy as np
import pytest

from paper_2503_05046_amd import inputs as I
from tests.parity import field_errors

pytestmark = pytest.mark.gpu


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


def _scene():
    s = I.tiny_random(P=300, seed=17, n=16, with_box=True)
    box = s.rigids[1]
    s.rigids = [s.rigids[0],
                I.RigidSpec(env=0, shape=I.BOX, mu=0.4, motion=I.DYNAMIC, half=box.half, R=box.R,
                            t=box.t, V=(0.1, -0.05, 0.0), w=(0.0, 0.0, 0.5), mass=0.5,
                            inertia=(6.8e-4, 8.7e-4, 1.0e-3), force=(0.0, 0.0, 1.0), torque=(2e-4, 0.0, 0.0))]
    s.envs[0].eps_s = 1e-2
    s.N = 2
    s.eps_r = 1e-10
    s.max_iter = 400000
    return s


def test_dynamic_box_matches_oracle(mpm, oracle):
    s = _scene()
    sim = mpm.Sim(s)
    ora = oracle.OracleSim(s)
    for step in range(3):
        status, imp, st = sim.step()
        assert status == 0
        rc, impo, _ = ora.host_step()
        assert rc == 0
        r = sim.rigid_state(1)
        q = ora.rig[1]
        dV = np.abs(np.array(r.V) - np.array(q.V)).max()
        dw = np.abs(np.array(r.w) - np.array(q.w)).max()
        dt = np.abs(np.array(r.t) - np.array(q.t)).max()
        dR = np.abs(np.array(r.R) - np.array(q.R)).max()
        _log(f"host step {step}: contacts {max(st['contacts'])}, box |dV| {dV:.2e} (|V| "
             f"{np.abs(np.array(q.V)).max():.3e}), |dw| {dw:.2e} (|w| {np.abs(np.array(q.w)).max():.3e}), "
             f"|dt| {dt:.2e}, |dR| {dR:.2e}")
        assert max(st["contacts"]) > 0
        # the twists from impulses that agree to the solve's tolerance; the
        # poses move by the host step's length times the twists
        tol_V = 1e-4 * np.abs(np.array(q.V)).max() + 1e-7
        tol_w = 1e-4 * np.abs(np.array(q.w)).max() + 1e-6
        assert dV <= tol_V and dw <= tol_w
        dT = s.N * s.h
        assert dt <= (step + 1) * dT * tol_V + 1e-12 and dR <= (step + 1) * dT * tol_w + 1e-12
    out = sim.state()
    sim.close()
    err = field_errors(out, ora, s.envs[0].dx)
    _log(f"particles after 3 host steps: {err}")
    assert max(err.values()) < 1e-5, err


def test_dynamic_body_refusals(mpm):
    s = _scene()
    sim = mpm.Sim(s, tape_substeps=s.N)
    with pytest.raises(RuntimeError, match="dynamic|kinematic bodies only"):
        sim.step_graph(1)
    sim.tape_reset(True)
    sim.step()
    import torch
    g = [torch.zeros((n, s.P), dtype=torch.float32, device=sim.device) for n in (3, 3, 9, 9)]
    with pytest.raises(RuntimeError, match="static and kinematic"):
        sim.backward(*g)
    sim.close()
    bad = _scene()
    r = bad.rigids[1]
    bad.rigids[1] = type(r)(**{**r.__dict__, "mass": 0.0})
    with pytest.raises(RuntimeError, match="mass"):
        mpm.Sim(bad)
