"""Comparison rules between the GPU library and the FP64 oracle.

Per field, err = max |gpu - oracle| / S with S_x = dx, S_v = max(max|v_oracle|,
1e-3 m/s), S_F = 1, S_C = S_v / dx. Contact-affected velocities can only agree
to the solver tolerance: both solves stop when |grad~| < thr, and because the
Hessian dominates M the iterate is within thr of the unique optimum in the
M-norm; G2P is an average, so sum_p m_p |dv_p|^2 <= sum_i m_i |dv_i|^2 and the
particle-velocity difference is bounded by thr_gpu + thr_oracle in that norm.
"""
import numpy as np


def field_errors(gpu: dict, ora, dx: float) -> dict:
    sv = max(float(np.abs(ora.v).max()), 1e-3)
    return {
        "x": float(np.abs(gpu["x"] - ora.x).max() / dx),
        "v": float(np.abs(gpu["v"] - ora.v).max() / sv),
        "F": float(np.abs(gpu["F"] - ora.F).max()),
        "C": float(np.abs(gpu["C"] - ora.C).max() / (sv / dx)),
    }


def m_norm(dv: np.ndarray, m_p: float) -> float:
    return float(np.sqrt(m_p * np.sum(dv.astype(np.float64) ** 2)))


def impulse_error(imp_gpu: np.ndarray, imp_ora: np.ndarray, m_tot: float, h: float,
                  arm: float = 1.0) -> float:
    """Largest relative difference of the impulses (columns 0-2, scale
    max(|impulse|, m g h)) and of their moments about the body origins
    (columns 3-5, scale max(|torque|, m g h arm); arm: a length of the scene,
    1 m by default, the domain's size)."""
    s_lin = max(float(np.abs(imp_ora[:, :3]).max()), m_tot * 9.81 * h)
    s_ang = max(float(np.abs(imp_ora[:, 3:]).max()), m_tot * 9.81 * h * arm)
    e_lin = float(np.abs(imp_gpu[:, :3] - imp_ora[:, :3]).max()) / s_lin
    e_ang = float(np.abs(imp_gpu[:, 3:] - imp_ora[:, 3:]).max()) / s_ang
    return max(e_lin, e_ang)


def rms_errors(gpu: dict, ora, dx: float) -> dict:
    """Root mean square over particles of the per-field errors of field_errors
    (same scales)."""
    sv = max(float(np.abs(ora.v).max()), 1e-3)
    scale = {"x": dx, "v": sv, "F": 1.0, "C": sv / dx}
    return {k: float(np.sqrt(np.mean(np.sum((gpu[k] - getattr(ora, k)) ** 2, axis=0))) / scale[k])
            for k in ("x", "v", "F", "C")}
