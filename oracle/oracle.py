"""ctypes front-end of the FP64 CPU oracle (``oracle_mpm.c``).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use this module. It never imports the GPU package; scenes are
read by attribute (any object with the fields of an input scene works).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle_mpm.c")
LIB = os.path.join(HERE, "liboracle_mpm.so")

OK, NOCONV, DOMAIN, NAN, EINVAL = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Env(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int), ("dx", ct.c_double),
                ("origin", ct.c_double * 3), ("gravity", ct.c_double * 3),
                ("material", ct.c_int), ("E", ct.c_double), ("nu", ct.c_double),
                ("m_p", ct.c_double), ("V0", ct.c_double), ("friction_angle", ct.c_double),
                ("k", ct.c_double), ("d", ct.c_double), ("eps_s", ct.c_double),
                ("h", ct.c_double), ("N", ct.c_int), ("eps_r", ct.c_double),
                ("eps_a", ct.c_double), ("max_iter", ct.c_int), ("ls_max_iter", ct.c_int),
                ("basis", ct.c_int), ("solve_all_nodes", ct.c_int)]


class Rigid(ct.Structure):
    _fields_ = [("shape", ct.c_int), ("normal", ct.c_double * 3), ("offset", ct.c_double),
                ("half", ct.c_double * 3), ("mu", ct.c_double), ("motion", ct.c_int),
                ("R", ct.c_double * 9), ("t", ct.c_double * 3), ("V", ct.c_double * 3),
                ("w", ct.c_double * 3), ("mass", ct.c_double), ("inertia", ct.c_double * 3),
                ("force", ct.c_double * 3), ("torque", ct.c_double * 3)]


class Stats(ct.Structure):
    _fields_ = [("n_contacts", ct.c_int), ("iterations", ct.c_int), ("ls_steps", ct.c_int),
                ("converged", ct.c_int), ("residual", ct.c_double), ("threshold", ct.c_double),
                ("p_norm", ct.c_double), ("j_norm", ct.c_double), ("n_active_nodes", ct.c_int),
                ("n_contact_nodes", ct.c_int)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_D = ct.POINTER(ct.c_double)
_I = ct.POINTER(ct.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ct.CDLL(LIB)
        L.oracle_substep.argtypes = [ct.POINTER(Env), ct.POINTER(Rigid), ct.c_int, ct.c_int,
                                     _D, _D, _D, _D, _D, ct.POINTER(Stats), _D]
        L.oracle_host_step.argtypes = [ct.POINTER(Env), ct.POINTER(Rigid), ct.c_int, ct.c_int,
                                       _D, _D, _D, _D, _D, ct.POINTER(Stats)]
        L.oracle_stencil.argtypes = [ct.POINTER(Env), _D, _I, _D, _D]
        L.oracle_cell_keys_f32.argtypes = [ct.c_int, ct.POINTER(ct.c_float),
                                           ct.POINTER(ct.c_float), ct.c_float, ct.c_int,
                                           ct.c_int, ct.c_int, ct.POINTER(ct.c_uint)]
        L.oracle_stable_order.argtypes = [ct.c_int, ct.POINTER(ct.c_uint), _I]
        L.oracle_svd3.argtypes = [_D, _D, _D, _D]
        L.oracle_kirchhoff.argtypes = [ct.POINTER(Env), _D, _D]
        L.oracle_dp_project.argtypes = [ct.POINTER(Env), _D]
        L.oracle_dp_project.restype = ct.c_int
        L.oracle_contact_model.argtypes = [_D] + [ct.c_double] * 7 + [_D, _D]
        L.oracle_contact_model.restype = ct.c_double
        L.oracle_normal_impulse.argtypes = [ct.c_double] * 5
        L.oracle_normal_impulse.restype = ct.c_double
        L.oracle_sdf.argtypes = [ct.POINTER(Rigid), _D, _D]
        L.oracle_sdf.restype = ct.c_double
        L.oracle_contact_frame.argtypes = [ct.c_int, _D, _D]
        L.oracle_qn_solve.argtypes = [ct.POINTER(Env), ct.c_int, _D, _D, ct.c_int, _I, _D, _D,
                                      _D, _D, _D, _D, _D, _D, ct.POINTER(Stats), _D]
        L.oracle_contact_problem.argtypes = [ct.POINTER(Env), ct.POINTER(Rigid), ct.c_int,
                                             ct.c_int, _D, _D, _D, _D, ct.c_int, ct.c_int, _I,
                                             _D, _D, _I, _D, _D, _D, _D, _D, _D]
        L.oracle_advance_pose.argtypes = [ct.POINTER(Rigid), ct.c_double]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_I)


def make_env(scene, e: int = 0, basis: int = 0) -> Env:
    s = scene.envs[e]
    env = Env()
    env.nx, env.ny, env.nz = (int(v) for v in s.dims)
    env.dx = s.dx
    env.origin[:] = list(s.origin)
    env.gravity[:] = list(s.gravity)
    env.material = s.material
    env.E, env.nu = s.E, s.nu
    env.m_p, env.V0 = s.rho * s.V0, s.V0
    env.friction_angle = s.friction_angle
    env.k, env.d, env.eps_s = s.k, s.d, s.eps_s
    env.h, env.N = scene.h, scene.N
    env.eps_r, env.eps_a = scene.eps_r, scene.eps_a
    env.max_iter, env.ls_max_iter = scene.max_iter, scene.ls_max_iter
    env.basis = basis
    return env


def make_rigids(scene, e: int = 0):
    rs = [r for r in scene.rigids if r.env == e]
    arr = (Rigid * max(1, len(rs)))()
    for i, r in enumerate(rs):
        a = arr[i]
        a.shape = r.shape
        a.normal[:] = list(r.normal)
        a.offset = r.offset
        a.half[:] = list(r.half)
        a.mu = r.mu
        a.motion = r.motion
        a.R[:] = list(r.R)
        a.t[:] = list(r.t)
        a.V[:] = list(r.V)
        a.w[:] = list(r.w)
        a.mass = getattr(r, "mass", 0.0)
        a.inertia[:] = list(getattr(r, "inertia", (0.0, 0.0, 0.0)))
        a.force[:] = list(getattr(r, "force", (0.0, 0.0, 0.0)))
        a.torque[:] = list(getattr(r, "torque", (0.0, 0.0, 0.0)))
    return arr, len(rs)


class OracleSim:
    """FP64 copy of one environment of a scene, stepped by the oracle."""

    def __init__(self, scene, env: int = 0, basis: int = 0):
        s = scene.envs[env]
        sl = slice(s.p_begin, s.p_end)
        self.env = make_env(scene, env, basis)
        self.rig, self.n_rigid = make_rigids(scene, env)
        self.x = np.ascontiguousarray(scene.x[:, sl], np.float64)
        self.v = np.ascontiguousarray(scene.v[:, sl], np.float64)
        self.F = np.ascontiguousarray(scene.F[:, sl], np.float64)
        self.C = np.ascontiguousarray(scene.C[:, sl], np.float64)
        self.P = self.x.shape[1]

    def substep(self, impulse: Optional[np.ndarray] = None, lp_hist: bool = False):
        st = Stats()
        imp = impulse if impulse is not None else np.zeros(6 * max(1, self.n_rigid))
        hist = np.full(self.env.max_iter + 1, np.nan) if lp_hist else None
        rc = lib().oracle_substep(ct.byref(self.env), self.rig, self.n_rigid, self.P,
                                  _dp(self.x), _dp(self.v), _dp(self.F), _dp(self.C), _dp(imp),
                                  ct.byref(st), _dp(hist) if hist is not None else None)
        return rc, st, hist

    def host_step(self):
        st = (Stats * self.env.N)()
        imp = np.zeros(6 * max(1, self.n_rigid))
        rc = lib().oracle_host_step(ct.byref(self.env), self.rig, self.n_rigid, self.P,
                                    _dp(self.x), _dp(self.v), _dp(self.F), _dp(self.C), _dp(imp),
                                    st)
        return rc, imp[: 6 * self.n_rigid].reshape(-1, 6), [s.as_dict() for s in st]

    def contact_problem(self, max_nodes: int = 20000, max_c: int = 4000) -> dict:
        n_out = ct.c_int(0)
        m = np.zeros(max_nodes)
        vs = np.zeros(3 * max_nodes)
        nodes = np.zeros(27 * max_c, np.int32)
        w = np.zeros(27 * max_c)
        Rc = np.zeros(9 * max_c)
        b = np.zeros(3 * max_c)
        phi0 = np.zeros(max_c)
        n0 = np.zeros(max_c)
        mu = np.zeros(max_c)
        nc = lib().oracle_contact_problem(ct.byref(self.env), self.rig, self.n_rigid, self.P,
                                          _dp(self.x), _dp(self.v), _dp(self.F), _dp(self.C),
                                          max_nodes, max_c, ct.byref(n_out), _dp(m), _dp(vs),
                                          _ip(nodes), _dp(w), _dp(Rc), _dp(b), _dp(phi0),
                                          _dp(n0), _dp(mu))
        if nc < 0:
            raise RuntimeError(f"oracle_contact_problem failed ({nc})")
        n = n_out.value
        return dict(m=m[:n].copy(), vstar=vs[: 3 * n].reshape(n, 3).copy(),
                    nodes=nodes[: 27 * nc].reshape(nc, 27).copy(),
                    w=w[: 27 * nc].reshape(nc, 27).copy(), Rc=Rc[: 9 * nc].reshape(nc, 3, 3).copy(),
                    b=b[: 3 * nc].reshape(nc, 3).copy(), phi0=phi0[:nc].copy(),
                    n0=n0[:nc].copy(), mu=mu[:nc].copy())


def qn_solve(env: Env, prob: dict, v0: Optional[np.ndarray] = None, lp_hist: bool = False):
    """Run Algorithm 1 on an explicit contact problem (see ``contact_problem``)."""
    n = prob["m"].shape[0]
    nc = prob["phi0"].shape[0]
    v = np.ascontiguousarray((prob["vstar"] if v0 is None else v0).reshape(-1), np.float64).copy()
    gam = np.zeros(3 * max(nc, 1))
    st = Stats()
    hist = np.full(env.max_iter + 1, np.nan) if lp_hist else None
    c = lambda a, t=np.float64: np.ascontiguousarray(a, t).reshape(-1)
    arrs = [c(prob["m"]), c(prob["vstar"]), c(prob["nodes"], np.int32), c(prob["w"]),
            c(prob["Rc"]), c(prob["b"]), c(prob["phi0"]), c(prob["n0"]), c(prob["mu"])]
    rc = lib().oracle_qn_solve(ct.byref(env), n, _dp(arrs[0]), _dp(arrs[1]), nc, _ip(arrs[2]),
                               _dp(arrs[3]), _dp(arrs[4]), _dp(arrs[5]), _dp(arrs[6]),
                               _dp(arrs[7]), _dp(arrs[8]), _dp(v), _dp(gam), ct.byref(st),
                               _dp(hist) if hist is not None else None)
    return rc, v.reshape(n, 3), gam[: 3 * nc].reshape(nc, 3), st, hist


# ---- thin wrappers of the pieces ---------------------------------------

def stencil(env: Env, xp):
    xp = np.ascontiguousarray(xp, np.float64)
    base = np.zeros(3, np.int32)
    w = np.zeros(27)
    dpos = np.zeros(81)
    lib().oracle_stencil(ct.byref(env), _dp(xp), _ip(base), _dp(w), _dp(dpos))
    return base, w, dpos.reshape(27, 3)


def cell_keys_f32(xs: np.ndarray, origin, inv_dx: float, dims) -> np.ndarray:
    xs = np.ascontiguousarray(xs, np.float32)
    P = xs.shape[1]
    keys = np.zeros(P, np.uint32)
    org = (ct.c_float * 3)(*[float(o) for o in origin])
    lib().oracle_cell_keys_f32(P, xs.ctypes.data_as(ct.POINTER(ct.c_float)), org,
                               ct.c_float(inv_dx), int(dims[0]), int(dims[1]), int(dims[2]),
                               keys.ctypes.data_as(ct.POINTER(ct.c_uint)))
    return keys


def stable_order(keys: np.ndarray) -> np.ndarray:
    keys = np.ascontiguousarray(keys, np.uint32)
    perm = np.zeros(keys.shape[0], np.int32)
    lib().oracle_stable_order(keys.shape[0], keys.ctypes.data_as(ct.POINTER(ct.c_uint)), _ip(perm))
    return perm


def svd3(F):
    F = np.ascontiguousarray(np.asarray(F, np.float64).reshape(9))
    U, S, V = np.zeros(9), np.zeros(3), np.zeros(9)
    lib().oracle_svd3(_dp(F), _dp(U), _dp(S), _dp(V))
    return U.reshape(3, 3), S, V.reshape(3, 3)


def kirchhoff(env: Env, F):
    F = np.ascontiguousarray(np.asarray(F, np.float64).reshape(9))
    tau = np.zeros(9)
    lib().oracle_kirchhoff(ct.byref(env), _dp(F), _dp(tau))
    return tau.reshape(3, 3)


def dp_project(env: Env, F):
    F = np.ascontiguousarray(np.asarray(F, np.float64).reshape(9)).copy()
    proj = lib().oracle_dp_project(ct.byref(env), _dp(F))
    return F.reshape(3, 3), bool(proj)


def contact_model(vc, phi0, n0, mu, k, d, eps_s, h):
    vc = np.ascontiguousarray(vc, np.float64)
    g = np.zeros(3)
    G = np.zeros(9)
    ell = lib().oracle_contact_model(_dp(vc), phi0, n0, mu, k, d, eps_s, h, _dp(g), _dp(G))
    return ell, g, G.reshape(3, 3)


def normal_impulse(vn, phi0, k, d, h):
    return lib().oracle_normal_impulse(vn, phi0, k, d, h)


def sdf(rigid: Rigid, x):
    x = np.ascontiguousarray(x, np.float64)
    n = np.zeros(3)
    s = lib().oracle_sdf(ct.byref(rigid), _dp(x), _dp(n))
    return s, n


def contact_frame(basis: int, n):
    n = np.ascontiguousarray(n, np.float64)
    R = np.zeros(9)
    lib().oracle_contact_frame(basis, _dp(n), _dp(R))
    return R.reshape(3, 3)


def advance_pose(rigid: Rigid, dt: float):
    lib().oracle_advance_pose(ct.byref(rigid), dt)
