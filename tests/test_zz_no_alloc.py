"""mpm_step_static (one host step on the library's static workspace, no
handle, nothing allocated) against mpm_step on a fresh handle, through the C
ABI: two calls in a row, the second on a smaller scene, each compared with its
own handle-based run (particle fields in the caller's order at the parity bar
of the other GPU tests, impulses and torques, contact counts); and the size
limit refused before any device work.

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
    def __init__(self, d):
        self.x, self.v, self.F, self.C = d["x"], d["v"], d["F"], d["C"]


def _cube():
    """The elastic cube resting its lowest layer just above a plane and moving
    at (0.5, 0, -1) m/s: 8,000 particles, 32^3 grid, contact in most substeps."""
    s = I.plain_cube(contact=True)
    s.eps_r = 1e-10
    s.max_iter = 400000
    return s


def _tiny():
    """64 particles with a box and a plane, 16^3 grid: a much smaller layout."""
    s = I.tiny_random(P=64, seed=29, n=16, material=I.DRUCKER_PRAGER, with_box=True)
    s.envs[0].eps_s = 1e-2
    s.eps_r = 1e-10
    s.max_iter = 400000
    return s


def _compare(mpm, scene, label):
    dx = scene.envs[0].dx
    m_tot = sum(e.m_p * (e.p_end - e.p_begin) for e in scene.envs)
    _log(f"{label}: {scene.P} particles, workspace "
         f"{mpm.mpm_workspace_size(mpm.make_desc(scene, mpm.env_descs(scene))) / 2**20:.1f} MiB")
    ref = mpm.Sim(scene)
    st_ref = ref.step()
    ref_state = ref.state()
    ref.close()
    stat = mpm.StaticStep(scene)
    st_sta = stat.step()
    sta_state = stat.state()
    assert st_ref[0] == 0 and st_sta[0] == 0, (st_ref[0], st_sta[0])
    assert st_sta[2]["contacts"] == st_ref[2]["contacts"], (st_sta[2]["contacts"], st_ref[2]["contacts"])
    assert max(st_ref[2]["contacts"]) > 0
    err = field_errors(sta_state, _State(ref_state), dx)
    ierr = impulse_error(st_sta[1], st_ref[1], m_tot, scene.h)
    _log(f"{label}: static vs handle: {err}, impulses {ierr:.2e}, "
         f"iterations {st_sta[2]['iterations']} vs {st_ref[2]['iterations']}")
    assert max(err.values()) < 1e-5, err
    assert ierr < 1e-5, ierr


def test_static_step_matches_handle_two_calls(mpm):
    _compare(mpm, _cube(), "first call, contact cube")
    _compare(mpm, _tiny(), "second call, smaller scene")


def test_static_step_batched(mpm):
    """Three environments in one static call (a batched handle's solver
    path), against a handle."""
    s = I.batched(n_envs=3, seed=21, p_min=300, p_max=1500, n=24, N=2)
    for e in (0, 2):
        env = s.envs[e]
        s.x[2, env.p_begin:env.p_end] -= np.float32(1.5 * env.dx)
    for env in s.envs:
        env.eps_s = 1e-2
    s.eps_r = 1e-10
    s.max_iter = 200000
    _compare(mpm, s, "batched call, three environments")


def test_static_step_refuses_oversized_scene(mpm):
    """A scene whose workspace exceeds the static array is refused with
    MPM_ENOMEM before any device work (the pointers are never read)."""
    import torch
    s = I.granular_pour(n_particles=200_000, seed=1)
    envs = mpm.env_descs(s)
    d = mpm.make_desc(s, envs)
    assert mpm.mpm_workspace_size(d) > 64 * 2**20
    buf = torch.zeros(16, device="cuda:0")
    d.x = d.v = d.F = d.C = buf.data_ptr()
    d.stream = torch.cuda.current_stream().cuda_stream
    rig = [mpm.rigid_desc(r) for r in s.rigids]
    status = mpm.load().mpm_step_static(
        d, (mpm.RigidDesc * len(rig))(*rig), (mpm.ct.c_int32 * len(rig))(*[r.env for r in s.rigids]),
        len(rig), None, None)
    assert status == mpm.MPM_ENOMEM, status
    assert "static array" in mpm.mpm_last_error()
