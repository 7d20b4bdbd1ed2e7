"""HIP path vs the FP64 oracle, through the C ABI, on seeded scenes.

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


def _run_both(mpm, oracle, scene, host_steps=1, basis=0, **sim_kw):
    """Step the scene on the GPU and in the oracle; returns (gpu state, oracle
    sim, gpu impulses, oracle impulses, gpu stats, oracle stats)."""
    sim = mpm.Sim(scene, **sim_kw)
    ora = oracle.OracleSim(scene, basis=basis)
    imp_g = np.zeros((len(scene.rigids), 6))
    imp_o = np.zeros((len(scene.rigids), 6))
    sg, so = [], []
    for _ in range(host_steps):
        status, imp, st = sim.step()
        imp_g += imp
        sg.append(st)
        rc, impo, sto = ora.host_step()
        imp_o += impo
        so.append(sto)
    out = sim.state()
    sim.close()
    return out, ora, imp_g, imp_o, sg, so


def test_sort_is_bit_exact(mpm, oracle):
    s = I.granular_pour(n_particles=200_000, seed=11)
    s.N = 1
    keys = oracle.cell_keys_f32(s.x, s.envs[0].origin, 1.0 / s.envs[0].dx, s.envs[0].dims)
    ref = oracle.stable_order(keys)
    _log("sort: 200k particles")
    sim = mpm.Sim(s)
    sim.step()
    pid = sim.pid.cpu().numpy()
    sim.close()
    assert np.array_equal(pid, ref)


def test_free_fall_one_and_hundred_substeps(mpm, oracle):
    s = I.plain_cube(contact=False)
    _log("free fall: plain cube, 1 substep")
    s1 = s.copy()
    s1.N = 1
    g, o, ig, io, sg, so = _run_both(mpm, oracle, s1)
    e = field_errors(g, o, s.envs[0].dx)
    assert max(e.values()) < 1e-5, e
    _log("free fall: plain cube, 100 substeps")
    g, o, ig, io, sg, so = _run_both(mpm, oracle, s, host_steps=10)
    e = field_errors(g, o, s.envs[0].dx)
    assert max(e.values()) < 1e-3, e
    # and the closed form
    h, k = s.h, 100
    gz = -9.81
    assert np.abs(g["v"][2] - k * h * gz).max() < 1e-5
    assert all(st["max_contacts"] == 0 for st in sg)


@pytest.mark.parametrize("material", [I.FIXED_COROTATED, I.DRUCKER_PRAGER])
def test_one_substep_random_state(mpm, oracle, material):
    """Random velocities, deformations and affine matrices; contacts with a
    half-space and a rotated, moving box; solved tightly so the comparison is
    at float32 level."""
    s = I.tiny_random(P=3000, seed=13, material=material, n=32)
    s.envs[0].eps_s = 1e-2  # softer friction keeps the tight solve short; the machinery is the same
    s.N = 1
    s.eps_r = 1e-10
    s.max_iter = 200000
    _log(f"random state, material {material}")
    g, o, ig, io, sg, so = _run_both(mpm, oracle, s)
    assert sg[0]["contacts"][0] == so[0][0]["n_contacts"] > 0
    e = field_errors(g, o, s.envs[0].dx)
    assert max(e.values()) < 1e-5, (e, sg[0], so[0])
    m_tot = s.envs[0].m_p * s.P
    assert impulse_error(ig, io, m_tot, s.h) < 1e-4


@pytest.mark.parametrize("walks", ["1", "2"])
@pytest.mark.parametrize("material", [I.FIXED_COROTATED, I.DRUCKER_PRAGER])
def test_dense_tiles_free_motion(mpm, oracle, material, walks, monkeypatch):
    """About 40 particles per cell (long P2G walks; with two walks per
    component and cell, each takes every other particle and their sums are
    added before the flush): two free-motion substeps of a random state
    against the oracle."""
    monkeypatch.setenv("MPM_P2G_WALKS", walks)
    s = I.tiny_random(P=20000, seed=17, n=32, material=material, with_box=False)
    s.rigids = []
    s.N = 2
    _log(f"dense tiles, material {material}, {walks} P2G walks")
    g, o, ig, io, sg, so = _run_both(mpm, oracle, s)
    assert sg[0]["max_contacts"] == 0
    e = field_errors(g, o, s.envs[0].dx)
    assert max(e.values()) < 1e-5, e


def _contact_state(oracle, substeps):
    """C1 contact variant advanced by the oracle into sustained contact; the
    state is rounded to float32 and handed to both sides."""
    s = I.plain_cube(contact=True)
    ora = oracle.OracleSim(s)
    ora.env.max_iter = 100000
    for _ in range(substeps):
        ora.substep()
    s.x, s.v, s.F, s.C = (a.astype(np.float32) for a in (ora.x, ora.v, ora.F, ora.C))
    return s


def test_contact_substep_metric_tolerance(mpm, oracle):
    """At the benchmark tolerance (eps_r = 1e-6) the two solves agree within
    the bound the stopping test guarantees."""
    s = _contact_state(oracle, 22)
    s.N = 1
    s.max_iter = 100000
    _log("plain cube contact substep at eps_r = 1e-6")
    g, o, ig, io, sg, so = _run_both(mpm, oracle, s)
    st_g, st_o = sg[0], so[0][0]
    assert st_g["contacts"][0] == st_o["n_contacts"] > 50
    assert st_g["residual"][0] < st_g["threshold"][0]
    m_p = s.envs[0].m_p
    bound = st_g["threshold"][0] + st_o["threshold"] + 1e-6 * math.sqrt(m_p * s.P)
    assert m_norm(g["v"] - o.v, m_p) <= bound
    e = field_errors(g, o, s.envs[0].dx)
    assert e["x"] < 1e-5 and e["F"] < 1e-5, e


def test_contact_substep_general_node_pass(mpm, oracle, monkeypatch):
    """The solver's general node pass (chunks of contact nodes, entries read
    from memory each iteration), which blocks too large for the compact pass
    take: forced for every block, at a tight tolerance."""
    monkeypatch.setenv("MPM_SOLVER_COMPACT", "0")
    s = _contact_state(oracle, 22)
    s.N = 1
    s.eps_r = 1e-10
    s.max_iter = 400000
    _log("plain cube contact substep, general node pass, eps_r = 1e-10")
    g, o, ig, io, sg, so = _run_both(mpm, oracle, s)
    e = field_errors(g, o, s.envs[0].dx)
    assert max(e.values()) < 1e-5, (e, sg[0], so[0])
    m_tot = s.envs[0].m_p * s.P
    assert impulse_error(ig, io, m_tot, s.h) < 1e-4


@pytest.mark.parametrize("spb", [16, 128])
def test_contact_substep_two_barrier_form(mpm, oracle, monkeypatch, spb):
    """The solver's two-barrier form (a contact pass gathers u_c between two
    group barriers), which environments with more contacts than the
    one-barrier form holds take: forced for every environment, with small and
    default block groups, at a tight tolerance."""
    monkeypatch.setenv("MPM_SOLVER_SCATTER", "0")
    s = _contact_state(oracle, 22)
    s.N = 1
    s.eps_r = 1e-10
    s.max_iter = 400000
    _log(f"plain cube contact substep, two-barrier form, {spb} contact nodes per block, eps_r = 1e-10")
    g, o, ig, io, sg, so = _run_both(mpm, oracle, s, solver_slots_per_block=spb)
    e = field_errors(g, o, s.envs[0].dx)
    assert max(e.values()) < 1e-5, (e, sg[0], so[0])
    m_tot = s.envs[0].m_p * s.P
    assert impulse_error(ig, io, m_tot, s.h) < 1e-4


def test_contact_substep_tight(mpm, oracle):
    s = _contact_state(oracle, 22)
    s.N = 1
    s.eps_r = 1e-10
    s.max_iter = 400000
    _log("plain cube contact substep at eps_r = 1e-10")
    g, o, ig, io, sg, so = _run_both(mpm, oracle, s)
    e = field_errors(g, o, s.envs[0].dx)
    assert max(e.values()) < 1e-5, (e, sg[0], so[0])
    m_tot = s.envs[0].m_p * s.P
    assert impulse_error(ig, io, m_tot, s.h) < 1e-4


def _batched_contact_scene(n_envs, seed, penetrating):
    """Independent environments in one handle; the particle blocks of the
    environments in `penetrating` start 1.5 dx inside their boxes, the others
    just above them (no contact in the first substeps)."""
    s = I.batched(n_envs=n_envs, seed=seed, p_min=300, p_max=1500, n=24, N=2)
    for e in penetrating:
        env = s.envs[e]
        s.x[2, env.p_begin:env.p_end] -= np.float32(1.5 * env.dx)
    for env in s.envs:
        env.eps_s = 1e-2  # softer friction keeps the tight solves short
    s.eps_r = 1e-10
    s.max_iter = 200000
    return s


def _compare_envs(mpm, oracle, s):
    sim = mpm.Sim(s)
    status, imp, st = sim.step()
    out = sim.state()
    sim.close()
    contacts = np.zeros(s.N, np.int64)
    for e, env in enumerate(s.envs):
        _log(f"  env {e}: {env.p_end - env.p_begin} particles, oracle")
        ora = oracle.OracleSim(s, env=e)
        rc, impo, sto = ora.host_step()
        contacts += np.array([q["n_contacts"] for q in sto])
        sl = slice(env.p_begin, env.p_end)
        g = {k: out[k][:, sl] for k in ("x", "v", "F", "C")}
        err = field_errors(g, ora, env.dx)
        assert max(err.values()) < 1e-5, (e, err)
        rid = [i for i, r in enumerate(s.rigids) if r.env == e]
        m_tot = env.m_p * (env.p_end - env.p_begin)
        assert impulse_error(imp[rid], impo, m_tot, s.h) < 1e-4, e
    assert list(st["contacts"]) == list(contacts)
    return contacts


def _combine(scenes):
    """Single-environment scenes as the environments of one batched scene
    (same h and N)."""
    import dataclasses
    envs, rigids, base = [], [], 0
    for e, sc in enumerate(scenes):
        assert len(sc.envs) == 1 and sc.h == scenes[0].h and sc.N == scenes[0].N
        envs.append(dataclasses.replace(sc.envs[0], p_begin=base, p_end=base + sc.P))
        rigids += [dataclasses.replace(r, env=e) for r in sc.rigids]
        base += sc.P
    cat = [np.ascontiguousarray(np.concatenate([getattr(sc, k) for sc in scenes], axis=1))
           for k in ("x", "v", "F", "C")]
    return I.Scene("mixed", scenes[0].h, scenes[0].N, envs, rigids, *cat)


def test_batched_dense_and_small_environments(mpm, oracle):
    """A batched handle whose first environment is a slab pressed into a plane
    (2,304 contacts: its group evaluates the line search distributed) beside
    two small ones in contact: every environment matches the oracle run on it
    alone."""
    slab = I.slab_on_plane(48, 2, (0.0, 0.0, 0.0), 0.5, seed=57, n=48, penetration=2e-5)
    rng = np.random.default_rng(57)
    slab.v = rng.normal(0.0, 1e-3, slab.v.shape).astype(np.float32)
    small = _batched_contact_scene(4, 21, penetrating=(0, 1, 3))
    parts = [slab] + [I.single_env(small, e) for e in (0, 1)]
    for sc in parts:
        sc.N = 1
    s = _combine(parts)
    s.eps_r = 1e-10
    s.max_iter = 400000
    _log("batched: the dense slab and two small environments, 1 substep")
    contacts = _compare_envs(mpm, oracle, s)
    assert contacts[0] > 2304


def test_batched_envs_solve_independently(mpm, oracle):
    """Four environments of different size and material in one handle, one of
    them without contact: each matches the oracle run on it alone (its own
    stopping test and line search)."""
    s = _batched_contact_scene(4, 21, penetrating=(0, 1, 3))
    _log("batched: 4 environments, 2 substeps")
    contacts = _compare_envs(mpm, oracle, s)
    assert contacts.min() > 0


def test_batched_envs_sharing_blocks(mpm, oracle, monkeypatch):
    """More environments than solver blocks: blocks take environments in turn."""
    monkeypatch.setenv("MPM_SOLVER_MAX_BLOCKS", "2")
    s = _batched_contact_scene(5, 22, penetrating=(0, 2, 3, 4))
    _log("batched: 5 environments on 2 solver blocks, 2 substeps")
    contacts = _compare_envs(mpm, oracle, s)
    assert contacts.min() > 0


@pytest.mark.parametrize("policy", ["truncated", "none"])
def test_sort_policy_arms(mpm, oracle, monkeypatch, policy):
    """The arms of the sort ablation (keys cut to their top 10 bits, or no
    reordering, with the plain scatter and gather): a random state under a
    moving box (contact in both substeps) and the cube in free fall over 10
    substeps, against the oracle."""
    monkeypatch.setenv("MPM_SORT_POLICY", policy)
    s = I.tiny_random(P=600, seed=41, n=24, material=I.DRUCKER_PRAGER, with_box=True)
    s.envs[0].eps_s = 1e-2
    s.eps_r = 1e-10
    s.max_iter = 400000
    _log(f"sort policy {policy}: random state under a moving box")
    g, o, ig, io, sg, so = _run_both(mpm, oracle, s)
    assert min(sg[0]["contacts"]) > 0
    e = field_errors(g, o, s.envs[0].dx)
    assert max(e.values()) < 1e-5, e
    assert impulse_error(ig, io, s.envs[0].m_p * s.P, s.h) < 1e-4
    c = I.plain_cube(contact=False)
    _log(f"sort policy {policy}: free fall, 10 substeps")
    g, o, ig, io, sg, so = _run_both(mpm, oracle, c)
    e = field_errors(g, o, c.envs[0].dx)
    assert max(e.values()) < 1e-5, e
