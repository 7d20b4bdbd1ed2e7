"""The graph path (mpm_step_graph) against the eager path (mpm_step) and the
FP64 oracle, through the C ABI.

Every replay is checked: a handle advanced by graph replays, with eager host
steps and host synchronisations between the replays, is compared after each
replay with a handle advanced eagerly by the same number of host steps
(particle fields, summed impulses, the pose of a kinematic box that the graph
advances on the device); the state after the first replay (two host steps)
is also compared with the oracle, at the parity bar of the other tests (over
more substeps the float32 state drifts from the FP64 oracle beyond it, on the
eager path alike).

Run on an MI355X: python -m pytest tests -m gpu
"""
import sys

import numpy as np
import pytest

from paper_2503_05046_amd import inputs as I
from tests.parity import field_errors, impulse_error

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


class _State:
    """Field arrays in the attribute form field_errors takes for its reference."""

    def __init__(self, d):
        self.x, self.v, self.F, self.C = d["x"], d["v"], d["F"], d["C"]


def _kinematic_scene():
    """Random elastic state over a half-space under a rotating box moving at
    (0.1, -0.05, 0) m/s (kinematic): contact from the first substep."""
    s = I.tiny_random(P=300, seed=17, n=16, material=I.FIXED_COROTATED, with_box=True)
    s.envs[0].eps_s = 1e-2
    s.N = 2
    s.eps_r = 1e-10
    s.max_iter = 400000
    return s


def _batched_scene():
    s = I.batched(n_envs=3, seed=23, p_min=300, p_max=1200, n=24, N=2)
    for env in s.envs:
        s.x[2, env.p_begin:env.p_end] -= np.float32(1.5 * env.dx)
        env.eps_s = 1e-2
    s.eps_r = 1e-10
    s.max_iter = 200000
    return s


def _pose(sim, i):
    r = sim.rigid_state(i)
    return np.array(list(r.R) + list(r.t))


def _check_replays(mpm, oracle, scene, label):
    dx = scene.envs[0].dx
    m_tot = sum(e.m_p * (e.p_end - e.p_begin) for e in scene.envs)
    eager = mpm.Sim(scene)
    graph = mpm.Sim(scene)
    n_eager = 0
    first = None
    # graph(2); eager step on both; graph(2); graph(2)
    plan = [("graph", 2), ("eager", 1), ("graph", 2), ("graph", 2)]
    for r, (kind, n) in enumerate(plan):
        imp_e = np.zeros((len(scene.rigids), 6))
        for _ in range(n):
            status, imp, _ = eager.step()
            assert status == 0
            imp_e += imp
        n_eager += n
        if kind == "graph":
            status, imp_g, st = graph.step_graph(n)
        else:
            status, imp_g, st = graph.step()
        assert status == 0
        assert max(st["contacts"]) > 0
        err = field_errors(graph.state(), _State(eager.state()), dx)
        _log(f"{label}: after {kind} x{n} ({n_eager} host steps): {err}")
        assert max(err.values()) < 1e-5, (r, err)
        assert impulse_error(imp_g, imp_e, m_tot, scene.h) < 1e-4, r
        for i, rig in enumerate(scene.rigids):
            if rig.motion == I.KINEMATIC:
                assert np.abs(_pose(graph, i) - _pose(eager, i)).max() < 1e-12, (r, i)
        if first is None:
            first = (n_eager, graph.state())
    graph.close()
    eager.close()
    # the first replay against the oracle, run on each environment alone
    n_first, out = first
    for e, env in enumerate(scene.envs):
        ora = oracle.OracleSim(scene, env=e)
        for _ in range(n_first):
            rc, _, _ = ora.host_step()
            assert rc == 0
        sl = slice(env.p_begin, env.p_end)
        g = {k: out[k][:, sl] for k in ("x", "v", "F", "C")}
        err = field_errors(g, ora, env.dx)
        _log(f"{label}: environment {e} against the oracle after {n_first} host steps: {err}")
        assert max(err.values()) < 1e-5, (e, err)


def test_graph_replays_match_eager_kinematic_box(mpm, oracle):
    _check_replays(mpm, oracle, _kinematic_scene(), "kinematic box")


def test_graph_replays_match_eager_batched(mpm, oracle):
    _check_replays(mpm, oracle, _batched_scene(), "batched, 3 environments")


def test_graph_refusals(mpm):
    """The graph path refuses n_steps < 1 and a recording tape."""
    s = _kinematic_scene()
    sim = mpm.Sim(s, tape_substeps=s.N)
    with pytest.raises(RuntimeError, match="n_steps"):
        sim.step_graph(0)
    sim.tape_reset(True)
    with pytest.raises(RuntimeError, match="tape"):
        sim.step_graph(1)
    sim.close()
