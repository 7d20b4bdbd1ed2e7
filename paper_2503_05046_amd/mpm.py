"""Python binding of libmpm (the C ABI of include/mpm.h), argument marshalling only.

Every step of the substep runs in the HIP library; PyTorch only provides device
memory (the caller-owned particle arrays and the workspace) and the stream.
There is no CPU fallback: importing this module on a machine without the built
library raises, and creating a simulation without a GPU fails in HIP.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Sequence

import numpy as np

from . import inputs as _inputs  # noqa: F401  (scene types are the natural input)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmpm.so")

MPM_OK, MPM_ENOCONV, MPM_EDOMAIN, MPM_ENAN, MPM_EINVAL, MPM_ENOMEM, MPM_EDEVICE = range(7)
STATUS_NAMES = {0: "MPM_OK", 1: "MPM_ENOCONV", 2: "MPM_EDOMAIN", 3: "MPM_ENAN", 4: "MPM_EINVAL",
                5: "MPM_ENOMEM", 6: "MPM_EDEVICE"}
FLAG_NOCONV, FLAG_DOMAIN, FLAG_NAN, FLAG_CAPACITY = 1, 2, 4, 8
SOLVER_QN, SOLVER_NEWTON = 0, 1

EXPORTED = ("mpm_workspace_size", "mpm_create", "mpm_add_rigid_sdf", "mpm_step", "mpm_step_graph",
            "mpm_get_rigid_state", "mpm_set_rigid_state", "mpm_profile", "mpm_destroy", "mpm_tape_reset",
            "mpm_step_backward", "mpm_step_static", "mpm_last_error")
KERNEL_CLASSES = ("sort", "p2g", "grid", "register", "setup", "solve", "g2p")


class EnvDesc(ct.Structure):
    _fields_ = [("dims", ct.c_int32 * 3), ("dx", ct.c_float), ("origin", ct.c_float * 3),
                ("gravity", ct.c_float * 3), ("material", ct.c_int32), ("E", ct.c_float),
                ("nu", ct.c_float), ("m_p", ct.c_float), ("V0", ct.c_float),
                ("friction_angle", ct.c_float), ("k", ct.c_double), ("d", ct.c_double),
                ("eps_s", ct.c_double), ("p_begin", ct.c_int64), ("p_end", ct.c_int64)]


class Desc(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32), ("n_envs", ct.c_int32),
                ("envs", ct.POINTER(EnvDesc)), ("h", ct.c_double), ("N", ct.c_int32),
                ("eps_r", ct.c_double), ("eps_a", ct.c_double), ("max_iter", ct.c_int32),
                ("ls_max_steps", ct.c_int32), ("n_particles", ct.c_int64),
                ("x", ct.c_void_p), ("v", ct.c_void_p), ("F", ct.c_void_p), ("C", ct.c_void_p),
                ("pid", ct.c_void_p), ("max_contacts", ct.c_int64), ("workspace", ct.c_void_p),
                ("workspace_bytes", ct.c_size_t), ("stream", ct.c_void_p),
                ("tape_substeps", ct.c_int32), ("solver_slots_per_block", ct.c_int32),
                ("solver", ct.c_int32)]


class EnvGrad(ct.Structure):
    _fields_ = [("dE", ct.c_double), ("dnu", ct.c_double)]


class RigidGrad(ct.Structure):
    _fields_ = [("dV", ct.c_double * 3), ("dt", ct.c_double * 3), ("dV_kinematic", ct.c_double * 3),
                ("dw", ct.c_double * 3), ("dR", ct.c_double * 3), ("dw_kinematic", ct.c_double * 3)]


class RigidDesc(ct.Structure):
    _fields_ = [("shape", ct.c_int32), ("normal", ct.c_double * 3), ("offset", ct.c_double),
                ("half", ct.c_double * 3), ("mu", ct.c_double), ("motion", ct.c_int32),
                ("R", ct.c_double * 9), ("t", ct.c_double * 3), ("V", ct.c_double * 3),
                ("w", ct.c_double * 3), ("mass", ct.c_double), ("inertia", ct.c_double * 3),
                ("force", ct.c_double * 3), ("torque", ct.c_double * 3)]


class RigidState(ct.Structure):
    _fields_ = [("R", ct.c_double * 9), ("t", ct.c_double * 3), ("V", ct.c_double * 3),
                ("w", ct.c_double * 3)]


class RigidImpulse(ct.Structure):
    _fields_ = [("impulse", ct.c_double * 3), ("torque", ct.c_double * 3)]


class StepStats(ct.Structure):
    _fields_ = [("flags", ct.c_int32), ("max_iterations", ct.c_int32),
                ("total_iterations", ct.c_int64), ("max_contacts", ct.c_int32),
                ("iterations", ct.POINTER(ct.c_int32)), ("contacts", ct.POINTER(ct.c_int32)),
                ("contact_nodes", ct.POINTER(ct.c_int32)), ("residual", ct.POINTER(ct.c_double)),
                ("threshold", ct.POINTER(ct.c_double)), ("total_inner_iterations", ct.c_int64)]


class ProfileData(ct.Structure):
    _fields_ = [("ms", ct.c_double * 7), ("launches", ct.c_int64 * 7),
                ("solver_iterations", ct.c_int64), ("solver_ls_rounds", ct.c_int64),
                ("solver_contact_iters", ct.c_int64), ("solver_node_iters", ct.c_int64),
                ("solver_contact_rounds", ct.c_int64), ("solver_phase_us", ct.c_double * 8)]


_lib = None
_live = None  # handles not yet closed (weak references), closed at interpreter exit


def _close_live() -> None:
    """atexit: release every handle still open while the HIP runtime and
    torch are intact (not from finalizers during interpreter teardown)."""
    for sim in list(_live or ()):
        try:
            sim.close()
        except Exception:
            pass


def load():
    """Load libmpm.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run paper_2503_05046_amd.build.build()")
        L = ct.CDLL(LIB_PATH)
        L.mpm_workspace_size.argtypes = [ct.POINTER(Desc), ct.POINTER(ct.c_size_t)]
        L.mpm_create.argtypes = [ct.POINTER(Desc), ct.POINTER(ct.c_void_p)]
        L.mpm_add_rigid_sdf.argtypes = [ct.c_void_p, ct.c_int32, ct.POINTER(RigidDesc),
                                        ct.POINTER(ct.c_int32)]
        L.mpm_step.argtypes = [ct.c_void_p, ct.POINTER(RigidState), ct.POINTER(RigidImpulse),
                               ct.POINTER(StepStats)]
        L.mpm_step_graph.argtypes = [ct.c_void_p, ct.c_int32, ct.POINTER(RigidImpulse), ct.POINTER(StepStats)]
        L.mpm_get_rigid_state.argtypes = [ct.c_void_p, ct.c_int32, ct.POINTER(RigidState)]
        L.mpm_set_rigid_state.argtypes = [ct.c_void_p, ct.c_int32, ct.POINTER(RigidState), ct.c_int32]
        L.mpm_profile.argtypes = [ct.c_void_p, ct.c_int32, ct.POINTER(ProfileData)]
        L.mpm_tape_reset.argtypes = [ct.c_void_p, ct.c_int32]
        L.mpm_step_backward.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                        ct.POINTER(EnvGrad), ct.POINTER(RigidGrad)]
        L.mpm_step_static.argtypes = [ct.POINTER(Desc), ct.POINTER(RigidDesc), ct.POINTER(ct.c_int32), ct.c_int32,
                                      ct.POINTER(RigidImpulse), ct.POINTER(StepStats)]
        L.mpm_destroy.argtypes = [ct.c_void_p]
        L.mpm_destroy.restype = None
        L.mpm_last_error.restype = ct.c_char_p
        for f in ("mpm_workspace_size", "mpm_create", "mpm_add_rigid_sdf", "mpm_step",
                  "mpm_get_rigid_state", "mpm_set_rigid_state", "mpm_profile", "mpm_step_static"):
            getattr(L, f).restype = ct.c_int
        _lib = L
    return _lib


def mpm_last_error() -> str:
    return load().mpm_last_error().decode()


class MPMError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {mpm_last_error()}")


def _check(status: int, where: str, allow=(MPM_OK,)) -> int:
    if status not in allow:
        raise MPMError(status, where)
    return status


def env_descs(scene) -> ct.Array:
    arr = (EnvDesc * len(scene.envs))()
    for i, e in enumerate(scene.envs):
        a = arr[i]
        a.dims[:] = [int(d) for d in e.dims]
        a.dx = e.dx
        a.origin[:] = list(e.origin)
        a.gravity[:] = list(e.gravity)
        a.material = e.material
        a.E, a.nu = e.E, e.nu
        a.m_p, a.V0 = e.rho * e.V0, e.V0
        a.friction_angle = e.friction_angle
        a.k, a.d, a.eps_s = e.k, e.d, e.eps_s
        a.p_begin, a.p_end = e.p_begin, e.p_end
    return arr


def make_desc(scene, envs: ct.Array, max_contacts: int = 0, ls_max_steps: int = 0,
              tape_substeps: int = 0, solver_slots_per_block: int = 0, solver: int = SOLVER_QN) -> Desc:
    d = Desc()
    d.struct_size = ct.sizeof(Desc)
    d.n_envs = len(scene.envs)
    d.envs = ct.cast(envs, ct.POINTER(EnvDesc))
    d.h, d.N = scene.h, scene.N
    d.eps_r, d.eps_a = scene.eps_r, scene.eps_a
    d.max_iter = scene.max_iter
    d.ls_max_steps = ls_max_steps
    d.n_particles = scene.P
    d.max_contacts = max_contacts
    d.tape_substeps = tape_substeps
    d.solver_slots_per_block = solver_slots_per_block
    d.solver = solver
    return d


def mpm_workspace_size(desc: Desc) -> int:
    n = ct.c_size_t(0)
    _check(load().mpm_workspace_size(ct.byref(desc), ct.byref(n)), "mpm_workspace_size")
    return n.value


def mpm_create(desc: Desc) -> ct.c_void_p:
    h = ct.c_void_p(0)
    _check(load().mpm_create(ct.byref(desc), ct.byref(h)), "mpm_create")
    return h


def rigid_desc(r) -> RigidDesc:
    q = RigidDesc()
    q.shape = r.shape
    q.normal[:] = list(r.normal)
    q.offset = r.offset
    q.half[:] = list(r.half)
    q.mu = r.mu
    q.motion = r.motion
    q.R[:] = list(r.R)
    q.t[:] = list(r.t)
    q.V[:] = list(r.V)
    q.w[:] = list(r.w)
    q.mass = getattr(r, "mass", 0.0)
    q.inertia[:] = list(getattr(r, "inertia", (0.0, 0.0, 0.0)))
    q.force[:] = list(getattr(r, "force", (0.0, 0.0, 0.0)))
    q.torque[:] = list(getattr(r, "torque", (0.0, 0.0, 0.0)))
    return q


def mpm_add_rigid_sdf(h, env: int, r: RigidDesc) -> int:
    rid = ct.c_int32(-1)
    _check(load().mpm_add_rigid_sdf(h, env, ct.byref(r), ct.byref(rid)), "mpm_add_rigid_sdf")
    return rid.value


def _stats_buffers(N: int):
    its, ncs, nns = (ct.c_int32 * N)(), (ct.c_int32 * N)(), (ct.c_int32 * N)()
    res, thr = (ct.c_double * N)(), (ct.c_double * N)()
    st = StepStats()
    st.iterations, st.contacts, st.contact_nodes = its, ncs, nns
    st.residual, st.threshold = res, thr
    return st, (its, ncs, nns, res, thr)


def _stats_dict(st, bufs) -> dict:
    its, ncs, nns, res, thr = bufs
    return dict(flags=st.flags, max_iterations=st.max_iterations,
                total_iterations=st.total_iterations, max_contacts=st.max_contacts,
                iterations=list(its), contacts=list(ncs), contact_nodes=list(nns),
                residual=list(res), threshold=list(thr), inner_iterations=st.total_inner_iterations)


def mpm_step_graph(h, n_rigid: int, N: int, n_steps: int):
    """n_steps host steps as one graph replay (the library's own rigid state).
    Returns (status, impulses [n_rigid, 6] summed over the steps, stats of the
    last host step)."""
    imp = (RigidImpulse * max(1, n_rigid))()
    st, bufs = _stats_buffers(N)
    status = load().mpm_step_graph(h, int(n_steps), imp, ct.byref(st))
    _check(status, "mpm_step_graph", allow=(MPM_OK, MPM_ENOCONV))
    out = np.array([[*imp[i].impulse, *imp[i].torque] for i in range(n_rigid)]).reshape(n_rigid, 6)
    return status, out, _stats_dict(st, bufs)


def mpm_step(h, n_rigid: int, N: int, states: Optional[Sequence[RigidState]] = None):
    """One host step. Returns (status, impulses [n_rigid, 6], stats dict)."""
    imp = (RigidImpulse * max(1, n_rigid))()
    its = (ct.c_int32 * N)()
    ncs = (ct.c_int32 * N)()
    nns = (ct.c_int32 * N)()
    res = (ct.c_double * N)()
    thr = (ct.c_double * N)()
    st = StepStats()
    st.iterations, st.contacts, st.contact_nodes = its, ncs, nns
    st.residual, st.threshold = res, thr
    sin = None
    if states is not None:
        sin = (RigidState * max(1, n_rigid))(*states)
    status = load().mpm_step(h, sin, imp, ct.byref(st))
    _check(status, "mpm_step", allow=(MPM_OK, MPM_ENOCONV))
    out = np.array([[*imp[i].impulse, *imp[i].torque] for i in range(n_rigid)]).reshape(n_rigid, 6)
    stats = dict(flags=st.flags, max_iterations=st.max_iterations,
                 total_iterations=st.total_iterations, max_contacts=st.max_contacts,
                 iterations=list(its), contacts=list(ncs), contact_nodes=list(nns),
                 residual=list(res), threshold=list(thr), inner_iterations=st.total_inner_iterations)
    return status, out, stats


def mpm_step_static(desc: Desc, rigids: Sequence[RigidDesc], rigid_env: Sequence[int], N: int):
    """One host step without a handle, on the library's static workspace
    (desc.workspace NULL). Returns (status, impulses [n_rigid, 6], stats dict)."""
    n = len(rigids)
    rig = (RigidDesc * max(1, n))(*rigids)
    env = (ct.c_int32 * max(1, n))(*[int(e) for e in rigid_env])
    imp = (RigidImpulse * max(1, n))()
    st, bufs = _stats_buffers(N)
    status = load().mpm_step_static(ct.byref(desc), rig, env, n, imp, ct.byref(st))
    _check(status, "mpm_step_static", allow=(MPM_OK, MPM_ENOCONV))
    out = np.array([[*imp[i].impulse, *imp[i].torque] for i in range(n)]).reshape(n, 6)
    return status, out, _stats_dict(st, bufs)


def mpm_get_rigid_state(h, rid: int) -> RigidState:
    s = RigidState()
    _check(load().mpm_get_rigid_state(h, rid, ct.byref(s)), "mpm_get_rigid_state")
    return s


def mpm_set_rigid_state(h, rid: int, state: RigidState, host_steps: int = 0) -> None:
    _check(load().mpm_set_rigid_state(h, rid, ct.byref(state), int(host_steps)), "mpm_set_rigid_state")


def mpm_profile(h, enable: int) -> dict:
    """Kernel-class event timing off (0), on (1), or on with the solver's phase
    timers (2, which lengthen the solve); returns what was accumulated."""
    p = ProfileData()
    _check(load().mpm_profile(h, int(enable), ct.byref(p)), "mpm_profile")
    return dict(ms={k: p.ms[i] for i, k in enumerate(KERNEL_CLASSES)},
                launches={k: p.launches[i] for i, k in enumerate(KERNEL_CLASSES)},
                solver_iterations=p.solver_iterations, solver_ls_rounds=p.solver_ls_rounds,
                solver_contact_iters=p.solver_contact_iters,
                solver_node_iters=p.solver_node_iters,
                solver_contact_rounds=p.solver_contact_rounds,
                solver_phase_us=dict(zip(("node_gather", "node_solve", "barrier1", "contact", "barrier2", "ls_setup", "ls_evals", "update"),
                                         list(p.solver_phase_us))))


def mpm_tape_reset(h, record: bool = True) -> None:
    _check(load().mpm_tape_reset(h, 1 if record else 0), "mpm_tape_reset")


def mpm_step_backward(h, gx: int, gv: int, gF: int, gC: int, n_envs: int, n_rigid: int):
    """Device pointers of the four adjoint arrays (updated in place); returns
    ([(dL/dE, dL/dnu)] per environment, {"dV", "dt", "dV_kinematic", "dw", "dR",
    "dw_kinematic"} arrays of shape [n_rigid, 3])."""
    g = (EnvGrad * n_envs)()
    r = (RigidGrad * max(1, n_rigid))()
    _check(load().mpm_step_backward(h, gx, gv, gF, gC, g, r), "mpm_step_backward")
    rig = {k: np.array([list(getattr(q, k)) for q in r[:n_rigid]]).reshape(n_rigid, 3)
           for k in ("dV", "dt", "dV_kinematic", "dw", "dR", "dw_kinematic")}
    return [(e.dE, e.dnu) for e in g], rig


def mpm_destroy(h) -> None:
    if h:
        load().mpm_destroy(h)


class Sim:
    """A scene resident on one GPU: torch owns the particle arrays and the
    workspace, the library steps them in place."""

    def __init__(self, scene, device: str = "cuda:0", max_contacts: int = 0,
                 ls_max_steps: int = 0, track_ids: bool = True, tape_substeps: int = 0,
                 solver_slots_per_block: int = 0, solver: int = SOLVER_QN):
        import torch
        load()
        self.torch = torch
        self.scene = scene
        self.device = torch.device(device)
        self.N = scene.N
        self.P = scene.P
        dev = self.device
        self.x = torch.from_numpy(np.ascontiguousarray(scene.x, np.float32)).to(dev)
        self.v = torch.from_numpy(np.ascontiguousarray(scene.v, np.float32)).to(dev)
        self.F = torch.from_numpy(np.ascontiguousarray(scene.F, np.float32)).to(dev)
        self.C = torch.from_numpy(np.ascontiguousarray(scene.C, np.float32)).to(dev)
        self.pid = torch.arange(self.P, dtype=torch.int32, device=dev) if track_ids else None
        self._envs = env_descs(scene)
        self.desc = make_desc(scene, self._envs, max_contacts, ls_max_steps, tape_substeps,
                              solver_slots_per_block, solver)
        self.ws_bytes = mpm_workspace_size(self.desc)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        d = self.desc
        d.x, d.v, d.F, d.C = (t.data_ptr() for t in (self.x, self.v, self.F, self.C))
        d.pid = self.pid.data_ptr() if self.pid is not None else None
        d.workspace, d.workspace_bytes = aligned, self.ws_bytes
        self.stream = torch.cuda.current_stream(dev)
        d.stream = self.stream.cuda_stream
        self.handle = mpm_create(d)
        global _live
        if _live is None:
            import atexit
            import weakref
            _live = weakref.WeakSet()
            atexit.register(_close_live)
        _live.add(self)
        self.rigid_ids = [mpm_add_rigid_sdf(self.handle, r.env, rigid_desc(r)) for r in scene.rigids]

    @property
    def n_rigid(self) -> int:
        return len(self.rigid_ids)

    def step(self, states=None):
        return mpm_step(self.handle, self.n_rigid, self.N, states)

    def step_graph(self, n_steps: int):
        """n_steps host steps in one HIP graph replay (see mpm_step_graph)."""
        return mpm_step_graph(self.handle, self.n_rigid, self.N, n_steps)

    def state(self, original_order: bool = True) -> dict:
        """Particle state as float32 numpy arrays (in the caller's original
        particle order when ids are tracked)."""
        self.torch.cuda.synchronize(self.device)
        out = {k: getattr(self, k).cpu().numpy() for k in ("x", "v", "F", "C")}
        if original_order and self.pid is not None:
            pid = self.pid.cpu().numpy()
            inv = np.empty_like(pid)
            inv[pid] = np.arange(pid.shape[0], dtype=pid.dtype)
            out = {k: a[:, inv] for k, a in out.items()}
        return out

    def tape_reset(self, record: bool = True) -> None:
        mpm_tape_reset(self.handle, record)

    def load_state(self, x, v, F, C) -> None:
        """Replace the state by (x, v, F, C) (tensors [3|9, P], any float dtype)
        in the caller's particle order, and reset the particle ids."""
        with self.torch.no_grad():
            for dst, src in ((self.x, x), (self.v, v), (self.F, F), (self.C, C)):
                dst.copy_(src.detach().to(device=self.device, dtype=self.torch.float32))
            if self.pid is not None:
                self.pid.copy_(self.torch.arange(self.P, dtype=self.torch.int32, device=self.device))

    def state_tensors(self):
        """(x, v, F, C) as new float32 tensors on the device in the order of the
        last load_state (or creation)."""
        inv = self.torch.argsort(self.pid.long())
        return tuple(t[:, inv].clone() for t in (self.x, self.v, self.F, self.C))

    def backward(self, gx, gv, gF, gC) -> list:
        """Reverse pass over the recorded steps. gx, gv, gF, gC: contiguous
        float32 tensors on the device, [3|9, P], the adjoint of the current
        state in its current particle order; overwritten in place with the
        adjoint of the state at the tape start, in the order it had then.
        Returns ([(dL/dE, dL/dnu)] per environment, rigid adjoints)."""
        for t in (gx, gv, gF, gC):
            if t.device != self.device or t.dtype != self.torch.float32 or not t.is_contiguous():
                raise ValueError("adjoints must be contiguous float32 tensors on the simulation device")
        return mpm_step_backward(self.handle, gx.data_ptr(), gv.data_ptr(), gF.data_ptr(), gC.data_ptr(),
                                 len(self.scene.envs), self.n_rigid)

    def profile(self, enable: int) -> dict:
        return mpm_profile(self.handle, enable)

    def rigid_state(self, i: int) -> RigidState:
        return mpm_get_rigid_state(self.handle, self.rigid_ids[i])

    def set_rigid_state(self, i: int, state: RigidState, host_steps: int = 0) -> None:
        """Body i at `state` advanced by host_steps kinematic host steps (the
        library's rule); `state` becomes its reference for the reverse pass."""
        mpm_set_rigid_state(self.handle, self.rigid_ids[i], state, host_steps)

    def close(self) -> None:
        if getattr(self, "handle", None):
            self.torch.cuda.synchronize(self.device)
            mpm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        import sys
        if sys.is_finalizing():
            return  # the atexit hook has released it; no HIP calls during teardown
        try:
            self.close()
        except Exception:
            pass


class StaticStep:
    """A scene's particle arrays on one GPU, stepped by mpm_step_static (no
    handle, no workspace: the library's static array). Rigid bodies stay at the
    scene's poses."""

    def __init__(self, scene, device: str = "cuda:0", max_contacts: int = 0, solver_slots_per_block: int = 0):
        import torch
        load()
        self.torch = torch
        self.scene = scene
        self.device = torch.device(device)
        dev = self.device
        self.x = torch.from_numpy(np.ascontiguousarray(scene.x, np.float32)).to(dev)
        self.v = torch.from_numpy(np.ascontiguousarray(scene.v, np.float32)).to(dev)
        self.F = torch.from_numpy(np.ascontiguousarray(scene.F, np.float32)).to(dev)
        self.C = torch.from_numpy(np.ascontiguousarray(scene.C, np.float32)).to(dev)
        self.pid = torch.arange(scene.P, dtype=torch.int32, device=dev)
        self._envs = env_descs(scene)
        d = make_desc(scene, self._envs, max_contacts, 0, 0, solver_slots_per_block)
        d.x, d.v, d.F, d.C = (t.data_ptr() for t in (self.x, self.v, self.F, self.C))
        d.pid = self.pid.data_ptr()
        d.workspace, d.workspace_bytes = None, 0
        d.stream = torch.cuda.current_stream(dev).cuda_stream
        self.desc = d
        order = sorted(range(len(scene.rigids)), key=lambda i: scene.rigids[i].env)
        self.order = order
        self.rigids = [rigid_desc(scene.rigids[i]) for i in order]
        self.rigid_env = [scene.rigids[i].env for i in order]

    def step(self):
        """One host step; impulses in the scene's rigid order."""
        status, imp, st = mpm_step_static(self.desc, self.rigids, self.rigid_env, self.scene.N)
        out = np.zeros_like(imp)
        out[self.order] = imp
        return status, out, st

    def state(self) -> dict:
        self.torch.cuda.synchronize(self.device)
        out = {k: getattr(self, k).cpu().numpy() for k in ("x", "v", "F", "C")}
        pid = self.pid.cpu().numpy()
        inv = np.empty_like(pid)
        inv[pid] = np.arange(pid.shape[0], dtype=pid.dtype)
        return {k: a[:, inv] for k, a in out.items()}
