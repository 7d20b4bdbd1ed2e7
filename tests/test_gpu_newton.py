"""The exact-Newton study variant of the contact solve (MPM_SOLVER_NEWTON:
the full Hessian system solved by preconditioned conjugate gradients for the
search direction, Algorithm 1's objective, stopping test and exact line
search) against the FP64 oracle, which runs Algorithm 1: both reach the
unique optimum of the contact problem (Sec. IV-B), so at a tight tolerance
the particle state and the impulses agree at the bar of the Algorithm 1
parity tests. Also checked: the variant needs far fewer outer iterations than
Algorithm 1 on the same substep, and reports its conjugate-gradient count.

Run on an MI355X: python -m pytest tests -m gpu
"""
import math
import sys

import numpy as np
import pytest

from paper_2503_05046_amd import inputs as I
from tests.parity import field_errors, impulse_error, m_norm

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


def _contact_state(oracle, substeps):
    """The plain-cube contact variant advanced by the oracle into sustained
    contact, rounded to float32 for both sides."""
    s = I.plain_cube(contact=True)
    ora = oracle.OracleSim(s)
    ora.env.max_iter = 100000
    for _ in range(substeps):
        ora.substep()
    s.x, s.v, s.F, s.C = (a.astype(np.float32) for a in (ora.x, ora.v, ora.F, ora.C))
    return s


def _run(mpm, scene, **kw):
    sim = mpm.Sim(scene, **kw)
    status, imp, st = sim.step()
    out = sim.state()
    sim.close()
    assert status == mpm.MPM_OK, status
    return out, imp, st


@pytest.mark.parametrize("spb", [16, 128])
def test_newton_contact_substep_tight(mpm, oracle, spb):
    """One substep of the cube in sustained contact at eps_r = 1e-10, with
    groups of many and of few blocks."""
    s = _contact_state(oracle, 22)
    s.N = 1
    s.eps_r = 1e-10
    s.max_iter = 400000
    _log(f"Newton variant: cube contact substep at eps_r = 1e-10, {spb} contact nodes per block")
    g, ig, st = _run(mpm, s, solver=mpm.SOLVER_NEWTON, solver_slots_per_block=spb)
    ora = oracle.OracleSim(s)
    rc, io, so = ora.host_step()
    assert rc == 0
    assert st["contacts"][0] == so[0]["n_contacts"] > 50
    e = field_errors(g, ora, s.envs[0].dx)
    _log(f"  Newton {st['iterations'][0]} iterations, {st['inner_iterations']} CG iterations; "
         f"oracle {so[0]['iterations']} iterations; errors {e}")
    assert max(e.values()) < 1e-5, e
    assert impulse_error(ig, io, s.envs[0].m_p * s.P, s.h) < 1e-4
    assert st["inner_iterations"] > 0
    assert st["iterations"][0] < so[0]["iterations"]


def test_newton_metric_tolerance(mpm, oracle):
    """At the benchmark tolerance (eps_r = 1e-6): within the bound the stopping
    test guarantees, as for Algorithm 1."""
    s = _contact_state(oracle, 22)
    s.N = 1
    s.max_iter = 100000
    g, ig, st = _run(mpm, s, solver=mpm.SOLVER_NEWTON)
    ora = oracle.OracleSim(s)
    rc, io, so = ora.host_step()
    st_o = so[0]
    assert st["residual"][0] < st["threshold"][0]
    m_p = s.envs[0].m_p
    bound = st["threshold"][0] + st_o["threshold"] + 1e-6 * math.sqrt(m_p * s.P)
    dv = m_norm(g["v"] - ora.v, m_p)
    _log(f"Newton variant at eps_r = 1e-6: |dv|_M {dv:.3e} (bound {bound:.3e}), "
         f"{st['iterations'][0]} iterations, {st['inner_iterations']} CG iterations")
    assert dv <= bound
    e = field_errors(g, ora, s.envs[0].dx)
    assert e["x"] < 1e-5 and e["F"] < 1e-5, e


@pytest.mark.parametrize("material", [I.FIXED_COROTATED, I.DRUCKER_PRAGER])
def test_newton_random_state_moving_box(mpm, oracle, material):
    """Random elastic or sand state over a half-space under a rotating,
    moving box, two substeps, against the oracle."""
    s = I.tiny_random(P=400, seed=31, n=24, material=material, with_box=True)
    s.envs[0].eps_s = 1e-2
    s.eps_r = 1e-10
    s.max_iter = 400000
    g, ig, st = _run(mpm, s, solver=mpm.SOLVER_NEWTON)
    ora = oracle.OracleSim(s)
    rc, io, so = ora.host_step()
    assert rc == 0
    assert list(st["contacts"]) == [q["n_contacts"] for q in so]
    assert min(st["contacts"]) > 0
    e = field_errors(g, ora, s.envs[0].dx)
    _log(f"Newton variant, random state (material {material}): {e}, iterations {st['iterations']}")
    assert max(e.values()) < 1e-5, e
    assert impulse_error(ig, io, s.envs[0].m_p * s.P, s.h) < 1e-4


def test_newton_batched_environments(mpm, oracle):
    """Four environments in one handle (one without contact), each against the
    oracle run on it alone."""
    s = I.batched(n_envs=4, seed=21, p_min=300, p_max=1500, n=24, N=2)
    for e in (0, 1, 3):
        env = s.envs[e]
        s.x[2, env.p_begin:env.p_end] -= np.float32(1.5 * env.dx)
    for env in s.envs:
        env.eps_s = 1e-2
    s.eps_r = 1e-10
    s.max_iter = 200000
    out, imp, st = _run(mpm, s, solver=mpm.SOLVER_NEWTON)
    for e, env in enumerate(s.envs):
        ora = oracle.OracleSim(s, env=e)
        rc, impo, sto = ora.host_step()
        sl = slice(env.p_begin, env.p_end)
        g = {k: out[k][:, sl] for k in ("x", "v", "F", "C")}
        err = field_errors(g, ora, env.dx)
        assert max(err.values()) < 1e-5, (e, err)
        rid = [i for i, r in enumerate(s.rigids) if r.env == e]
        assert impulse_error(imp[rid], impo, env.m_p * (env.p_end - env.p_begin), s.h) < 1e-4, e
