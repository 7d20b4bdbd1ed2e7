"""The solver's block-group size (contact nodes per block) and its autotuner:
every candidate gives the oracle's result, and the tuner returns one of them.

Run on an MI355X: python -m pytest tests -m gpu
"""
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


def _scene():
    s = I.batched(n_envs=3, seed=41, p_min=400, p_max=1500, n=24, N=2)
    for env in s.envs:
        s.x[2, env.p_begin:env.p_end] -= np.float32(1.5 * env.dx)
        env.eps_s = 1e-2
    s.eps_r = 1e-10
    s.max_iter = 200000
    return s


@pytest.mark.parametrize("spb", [16, 64, 512])
def test_block_group_size_keeps_results(mpm, oracle, spb):
    s = _scene()
    sim = mpm.Sim(s, solver_slots_per_block=spb)
    status, _, st = sim.step()
    assert status == 0 and max(st["contacts"]) > 0
    out = sim.state()
    sim.close()
    for e, env in enumerate(s.envs):
        ora = oracle.OracleSim(s, env=e)
        rc, _, _ = ora.host_step()
        assert rc == 0
        sl = slice(env.p_begin, env.p_end)
        err = field_errors({k: out[k][:, sl] for k in ("x", "v", "F", "C")}, ora, env.dx)
        assert max(err.values()) < 1e-5, (spb, e, err)


def test_autotune_returns_a_candidate(mpm):
    from paper_2503_05046_amd import autotune
    best, timing = autotune.tune(_scene(), candidates=(32, 128), warmup_steps=0, trial_steps=1)
    assert best in (32, 128) and set(timing) == {32, 128}
    assert all(t > 0 for t in timing.values())


def test_negative_block_size_is_refused(mpm):
    with pytest.raises(mpm.MPMError) as ei:
        mpm.Sim(_scene(), solver_slots_per_block=-1)
    assert ei.value.status == mpm.MPM_EINVAL
