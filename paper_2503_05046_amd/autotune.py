"""Autotuner for the contact solver's block groups.

The solver gives every environment a group of blocks sized from its contact
nodes: `solver_slots_per_block` contact nodes per block (mpm_desc). Fewer
nodes per block spread the node and contact passes over more blocks but make
the group barriers wider and, when environments compete for the co-resident
blocks, shrink other groups; the best value depends on the scene. `tune`
times short runs of the same scene for each candidate, every run starting
from the scene's initial state on a handle of its own, and returns the
fastest; pass it to `Sim(..., solver_slots_per_block=...)`.
"""
from __future__ import annotations

import time

from . import mpm as M

DEFAULT_CANDIDATES = (64, 96, 128, 160, 192, 256)


def tune(scene, candidates=DEFAULT_CANDIDATES, warmup_steps: int = 0, trial_steps: int = 2,
         device: str = "cuda:0", log=None) -> tuple:
    """Returns (best value, {value: seconds per host step}). Each candidate
    runs warmup_steps untimed host steps (to reach the contact regime of
    interest) and then trial_steps timed ones."""
    import torch
    timing = {}
    for spb in candidates:
        sim = M.Sim(scene, device=device, solver_slots_per_block=int(spb))
        for _ in range(warmup_steps):
            sim.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(trial_steps):
            sim.step()
        torch.cuda.synchronize()
        timing[int(spb)] = (time.perf_counter() - t0) / max(1, trial_steps)
        sim.close()
        if log:
            log(f"autotune: {spb} contact nodes per solver block: {1e3 * timing[int(spb)]:.1f} ms per host step")
    best = min(timing, key=timing.get)
    return best, timing
