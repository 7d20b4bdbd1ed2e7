"""Edge cases of the HIP path through the C ABI: degenerate and ragged sizes
against the FP64 oracle, an empty environment in a batched handle, and the
status paths (contact capacity, a particle leaving the grid, a non-finite
state, the iteration cap).

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


def _gpu_vs_oracle(mpm, oracle, scene, host_steps=1):
    sim = mpm.Sim(scene)
    for _ in range(host_steps):
        status, _, _ = sim.step()
        assert status == 0
    out = sim.state()
    sim.close()
    errs = []
    for e, env in enumerate(scene.envs):
        if env.p_end == env.p_begin:
            continue
        ora = oracle.OracleSim(scene, env=e)
        for _ in range(host_steps):
            rc, _, _ = ora.host_step()
            assert rc == 0
        sl = slice(env.p_begin, env.p_end)
        g = {k: out[k][:, sl] for k in ("x", "v", "F", "C")}
        errs.append(field_errors(g, ora, env.dx))
    return errs


@pytest.mark.parametrize("P", [1, 2, 63, 64, 65, 257])
def test_ragged_particle_counts(mpm, oracle, P):
    """One particle, and counts around the wave and block sizes, with the
    half-space and the moving box (contact where particles start below the
    plane)."""
    s = I.tiny_random(P=P, seed=100 + P, n=16, with_box=True)
    s.eps_r = 1e-10
    s.max_iter = 400000
    err = _gpu_vs_oracle(mpm, oracle, s)[0]
    _log(f"P = {P}: {err}")
    assert max(err.values()) < 1e-5, err


def test_empty_environment_in_a_batch(mpm, oracle):
    """A batched handle whose middle environment holds no particles: the
    others match the oracle run on them alone."""
    s = I.batched(n_envs=3, seed=31, p_min=300, p_max=900, n=24, N=2)
    e0, e1, e2 = s.envs
    keep = np.r_[np.arange(e0.p_begin, e0.p_end), np.arange(e2.p_begin, e2.p_end)]
    for k in ("x", "v", "F", "C"):
        setattr(s, k, np.ascontiguousarray(getattr(s, k)[:, keep]))
    n0, n2 = e0.p_end - e0.p_begin, e2.p_end - e2.p_begin
    e1.p_begin = e1.p_end = n0
    e2.p_begin, e2.p_end = n0, n0 + n2
    for env in (e0, e2):
        s.x[2, env.p_begin:env.p_end] -= np.float32(1.5 * env.dx)
        env.eps_s = 1e-2
    s.eps_r = 1e-10
    s.max_iter = 200000
    errs = _gpu_vs_oracle(mpm, oracle, s)
    _log(f"empty middle environment: {errs}")
    assert len(errs) == 2 and all(max(e.values()) < 1e-5 for e in errs), errs


def test_contact_capacity_overflow_leaves_state(mpm):
    """Capacity for one contact, several in the first substep: MPM_ENOMEM,
    and the caller's state is untouched (the step stops before its first
    G2P)."""
    s = I.tiny_random(P=300, seed=5, n=16, with_box=True)
    sim = mpm.Sim(s, max_contacts=1)
    before = sim.state()
    with pytest.raises(mpm.MPMError) as ei:
        sim.step()
    assert ei.value.status == mpm.MPM_ENOMEM
    after = sim.state()
    for k in ("x", "v", "F", "C"):
        assert np.array_equal(before[k], after[k]), k
    sim.close()


def test_particle_leaving_the_grid(mpm):
    s = I.tiny_random(P=8, seed=6, n=16, with_box=False)
    dx = s.envs[0].dx
    s.x[0, 0] = np.float32(1.0 - 1.2 * dx)  # stencil reaches past the last node
    sim = mpm.Sim(s)
    with pytest.raises(mpm.MPMError) as ei:
        sim.step()
    assert ei.value.status == mpm.MPM_EDOMAIN
    sim.close()


def test_non_finite_state(mpm):
    s = I.tiny_random(P=8, seed=7, n=16, with_box=False)
    s.v[0, 3] = np.float32(np.nan)
    sim = mpm.Sim(s)
    with pytest.raises(mpm.MPMError) as ei:
        sim.step()
    assert ei.value.status == mpm.MPM_ENAN
    sim.close()


def test_iteration_cap_is_a_warning(mpm):
    """max_iter = 1 in contact: MPM_ENOCONV is returned (a warning), the state
    is advanced with the last iterate and stays finite."""
    s = I.tiny_random(P=300, seed=8, n=16, with_box=True)
    s.max_iter = 1
    sim = mpm.Sim(s)
    x0 = sim.state()["x"]
    status, imp, st = sim.step()
    assert status == mpm.MPM_ENOCONV
    assert max(st["contacts"]) > 0 and max(st["iterations"]) <= 1
    out = sim.state()
    assert all(np.isfinite(out[k]).all() for k in ("x", "v", "F", "C"))
    assert not np.array_equal(out["x"], x0)
    sim.close()
