#!/usr/bin/env python
"""Throughput of the coupled MPM-rigid host step on one MI355X.

Workload: granular pour, 1,000,000 Drucker-Prager sand particles on a 128^3
grid (dx = 1/128) falling onto four static rigid boxes (mu = 0.4), substep
h = 1e-4 s, N = 10 substeps per host step, contact residual eps_r = 1e-6,
eps_a = FP64 machine epsilon. One benchmark step is one host step: the
once-per-step cell sort plus ten full substeps (P2G, grid update, contact
registration, the contact-node table, Algorithm 1 to convergence, G2P with the
return map). Inputs are seeded and synthetic and resident in HBM before the
timed region starts.

Prints one JSON line with the metric (particle-substeps/s), a roofline entry
for the kernel that takes most of the time, per-kernel figures measured with
HIP events inside the timed region, and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes (minimal float32 structure-of-arrays traffic).
P2G_BYTES_PER_PARTICLE = 60        # reads x, v, Q
G2P_BYTES_PER_PARTICLE = 144       # reads x, F; writes x, v, F, Q
SORT_BYTES_PER_PARTICLE = 210      # keys + stable sort passes + gather, once per host step
SOLVE_BYTES_PER_CONTACT_ITER = 52  # per Algorithm 1 iteration
SOLVE_BYTES_PER_NODE_ITER = 88
SOLVE_BYTES_PER_CONTACT_ROUND = 40  # per line-search reduction round


# The solver's HBM traffic per launch, measured with rocprofv3 PMC counters
# (FETCH_SIZE, WRITE_SIZE) and a plain device copy of known size for scale, is
# recorded in this summary together with a hash of the solver's sources; it is
# reported only while the sources still match.
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_traffic_solve_granular_pour_1M.md")
SOLVER_SOURCES = ("contact.hip", "contact_model.h", "mpm_internal.h", "sort_util.h")


def solver_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in SOLVER_SOURCES:
        with open(os.path.join(ROOT, "paper_2503_05046_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """Bytes per solver launch from the PMC summary, or None when there is no
    summary or the solver's sources changed since it was taken."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    fields = {}
    with open(PMC_SUMMARY) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("solver sources sha256") != solver_source_hash():
        return None
    try:
        return float(fields["HBM bytes per solver launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(n_bytes: int) -> int:
    """One plain device-to-device copy of n_bytes (the scale for the PMC byte
    counters)."""
    import torch
    n = n_bytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "check": float(dst[-1].item())}), flush=True)
    return 0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(state: dict, scene, budget_s: float) -> dict:
    """The FP64 oracle, as it stands, on substeps of a column of the same state
    (particles with x, y in [0.36, 0.44], all heights, over one box): as many
    substeps of one host step as fit in about budget_s / 3 seconds (at least
    one)."""
    import numpy as np
    from oracle import oracle as O
    O.build(force=not os.path.exists(O.LIB))
    x = state["x"]
    sel = np.nonzero((x[0] > 0.36) & (x[0] < 0.44) & (x[1] > 0.36) & (x[1] < 0.44))[0]
    sub = scene.copy()
    sub.x, sub.v, sub.F, sub.C = (np.ascontiguousarray(state[k][:, sel]) for k in ("x", "v", "F", "C"))
    sub.envs[0].p_begin, sub.envs[0].p_end = 0, len(sel)
    ora = O.OracleSim(sub)
    n_sub, contacts, iters, rc = 0, [], [], 0
    t0 = time.perf_counter()
    while n_sub < scene.N and (n_sub == 0 or time.perf_counter() - t0 < budget_s / 3):
        rc, st, _ = ora.substep()
        n_sub += 1
        contacts.append(st.n_contacts)
        iters.append(st.iterations)
        if rc >= 2:  # an error (1 is the iteration-cap warning)
            break
    dt = time.perf_counter() - t0
    return {"value": len(sel) * n_sub / dt, "unit": "particle-substeps/s", "cores": 1, "kind": "oracle",
            "sample": (f"{n_sub} substeps of a {len(sel)}-particle column (x, y in [0.36, 0.44]) of the "
                       f"benchmark state after the timed steps: {max(contacts)} contacts at most, "
                       f"{sum(iters)} solver iterations in all, {dt:.1f} s single-threaded FP64"),
            "status": rc}


def run_batched(args) -> int:
    """The batched form: 64 independent environments (log-uniform 5k-100k
    particles, 64^3 grids, elastic or sand, 1-3 boxes each) in one handle,
    against looping single-environment handles over the same environments.
    Looping all 64 at the contact tolerance takes minutes per host step, so
    the loop is timed on every 8th environment and scaled by the environment
    count (the per-environment solve is latency-bound, not size-bound)."""
    import numpy as np
    import torch
    from paper_2503_05046_amd import inputs as I
    from paper_2503_05046_amd import mpm as M

    scene = I.batched()
    scene.max_iter = args.max_iter
    P, N, n_envs = scene.P, scene.N, len(scene.envs)
    warm = args.warmup if args.warmup_set else 9  # contact starts near the 8th host step
    log(f"batched: {n_envs} environments, P={P}, warmup {warm}, steps {args.steps}")
    spb, tuning = 0, None
    if args.autotune:
        from paper_2503_05046_amd import autotune
        spb, tuning = autotune.tune(scene, candidates=(64, 96, 128, 192, 256), warmup_steps=warm,
                                    trial_steps=2, log=log)
        log(f"autotune: {spb} contact nodes per solver block")
    sim = M.Sim(scene, solver_slots_per_block=spb)
    for i in range(warm):
        sim.step()
    sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for i in range(args.steps):
        _, _, st = sim.step()
        iters += st["iterations"]
        log(f"batched step {i}: contacts {st['contacts']}, longest solve {max(st['iterations'])} iterations")
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    prof = sim.profile(False)
    sim.close()
    # the same host steps as one HIP graph replay (mpm_step_graph), on a second
    # handle warmed up the same way; the recording is inside the timed region
    gsim = M.Sim(scene, solver_slots_per_block=spb)
    for i in range(warm):
        gsim.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, gst = gsim.step_graph(args.steps)
    torch.cuda.synchronize()
    t_g = time.perf_counter() - t0
    log(f"graph: {args.steps} host steps in one replay, {t_g:.2f} s, last step contacts {gst['contacts']}")
    gsim.close()
    sub = list(range(0, n_envs, 8))
    sims = [M.Sim(I.single_env(scene, e)) for e in sub]
    for s in sims:
        for i in range(warm):
            s.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        for s in sims:
            s.step()
        log(f"loop step {i} done")
    torch.cuda.synchronize()
    t_sub = time.perf_counter() - t0
    for s in sims:
        s.close()
    t_loop = t_sub * n_envs / len(sub)
    value_b = P * N * args.steps / t_b
    value_l = P * N * args.steps / t_loop
    out = {
        "metric": "particle-substeps/s (batched, 64 environments, contact residual 1e-6)",
        "value": value_b, "unit": "particle-substeps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": warm, "ms_per_step": 1e3 * t_b / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": (f"batched: {n_envs} independent environments, {P} particles "
                                f"(log-uniform 5k-100k each), 64^3 grids, elastic/sand, 1-3 boxes, "
                                f"h=1e-4 s, {N} substeps per host step, eps_r=1e-6"),
                   "particles": P, "environments": n_envs},
        "loop": {"value": value_l, "ms_per_step": 1e3 * t_loop / args.steps,
                 "timed_environments": sub,
                 "method": "single-environment handles stepped in turn; time of the timed "
                           "environments scaled by 64 / 8"},
        "batched_over_loop": value_b / value_l,
        "solver_slots_per_block": spb or 128,
        "autotune": ({"chosen": spb, "ms_per_step": {k: round(1e3 * t, 1) for k, t in tuning.items()}}
                     if tuning else None),
        "graph": {"value": P * N * args.steps / t_g, "ms_per_step": 1e3 * t_g / args.steps,
                  "method": f"the {args.steps} timed host steps ({N * args.steps} substeps) as one "
                            f"HIP graph (mpm_step_graph), recording included"},
        "solve_share": prof["ms"]["solve"] / max(1e-9, sum(prof["ms"].values())),
        "longest_solve_iterations_mean": float(np.mean(iters)),
    }
    print(json.dumps(out), flush=True)
    return 0


def run_differentiable(args) -> int:
    """The backward form: 200k-particle elastic cube pushed by a box (C5), 50
    substeps (5 host steps) with a checkpoint every host step; the loss is the
    x coordinate of the final centre of mass, differentiated with respect to a
    uniform offset of the initial velocity, Young's modulus and the box
    velocity. Reports the forward-plus-backward rate and its cost relative to
    the plain forward."""
    import numpy as np
    import torch
    from paper_2503_05046_amd import diff
    from paper_2503_05046_amd import inputs as I
    from paper_2503_05046_amd import mpm as M

    scene = I.differentiable()
    scene.max_iter = args.max_iter
    P, N, steps = scene.P, scene.N, 5
    log(f"differentiable: P={P}, {steps} host steps of {N} substeps, checkpoint every host step")
    sim = M.Sim(scene, tape_substeps=N)
    path = diff.RigidPath(scene)
    dev = sim.device
    x0, v0, F0, C0 = (torch.from_numpy(a).to(dev) for a in (scene.x, scene.v, scene.F, scene.C))
    V0 = torch.tensor([list(r.V) for r in scene.rigids], dtype=torch.float64)
    E0 = torch.tensor([scene.envs[0].E], dtype=torch.float64)
    # plain forward (no tape, no autograd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    diff._run(sim, path, steps, 0, x0, v0, F0, C0, V0, record=False)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    log(f"forward: {t_fwd:.2f} s")
    # forward + backward through the checkpointed segments
    u = torch.zeros(3, dtype=torch.float32, device=dev, requires_grad=True)
    E = E0.clone().requires_grad_(True)
    V = V0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, v, F, C = diff.simulate(sim, path, steps, 1, x0, v0 + u[:, None], F0, C0, E, V)
    loss = x[0].mean()
    loss.backward()
    torch.cuda.synchronize()
    t_fb = time.perf_counter() - t0
    log(f"forward + backward: {t_fb:.2f} s")
    sim.close()
    out = {
        "metric": "particle-substeps/s (forward + backward, contact residual 1e-6)",
        "value": P * N * steps / t_fb, "unit": "particle-substeps/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": 1e3 * t_fb, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": (f"differentiable: {P}-particle elastic cube, 96^3 grid, pushed by a box at "
                                f"0.5 m/s, {N * steps} substeps, checkpoint every {N} substeps, "
                                f"eps_r=1e-6; one step = the whole forward-plus-backward run"),
                   "particles": P, "substeps": N * steps},
        "forward_s": t_fwd, "forward_backward_s": t_fb, "fwd_bwd_over_fwd": t_fb / t_fwd,
        "gradient": {"d_com_x/d_v0": u.grad.cpu().tolist(), "d_com_x/d_E": float(E.grad[0]),
                     "d_com_x/d_V_box": V.grad[0].tolist()},
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=("granular_pour", "batched", "differentiable"),
                    default="granular_pour")
    ap.add_argument("--particles", type=int, default=1_000_000)
    ap.add_argument("--max-iter", type=int, default=200_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--autotune", action="store_true",
                    help="batched workload: pick the solver's contact nodes per block with the autotuner first")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one device copy of BYTES (scale for the PMC byte counters)")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        return copy_calibration(args.copy_calibration)
    args.warmup_set = args.warmup is not None
    if args.warmup is None:
        args.warmup = 5
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (a single scene "
              "would shard into slabs, one per GPU, and the "
              "environments of the batched form would be assigned to GPUs whole). Run with --gpus 1.",
              file=sys.stderr)
        return 2
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "differentiable":
        return run_differentiable(args)

    import numpy as np
    import torch
    from paper_2503_05046_amd import inputs as I
    from paper_2503_05046_amd import mpm as M

    scene = I.granular_pour(n_particles=args.particles)
    scene.max_iter = args.max_iter
    log(f"scene {scene.name}: P={scene.P}, grid {tuple(scene.envs[0].dims)}, N={scene.N}, "
        f"h={scene.h}, eps_r={scene.eps_r}")
    sim = M.Sim(scene, device="cuda:0")
    P, N = scene.P, scene.N

    def run(k_steps, tag):
        per = []
        for i in range(k_steps):
            t = time.perf_counter()
            status, imp, st = sim.step()
            per.append(st)
            log(f"{tag} step {i}: {1e3 * (time.perf_counter() - t):.1f} ms, contacts max "
                f"{st['max_contacts']}, iterations/substep {st['iterations']}, flags {st['flags']}")
        return per

    run(args.warmup, "warmup")
    sim.profile(True)  # reset and start event timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = run(args.steps, "timed")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile(0)
    elapsed = t1 - t0
    value = P * N * args.steps / elapsed
    # one more host step, untimed, with the solver's phase timers on (their
    # clock reads lengthen the solve, so they stay out of the timed steps)
    sim.profile(2)
    run(1, "phase-timer")
    phase_prof = sim.profile(0)

    # per-kernel figures from the live events
    ms, launches = prof["ms"], prof["launches"]
    total_ms = sum(ms.values())
    sub_launches = max(1, launches["p2g"])
    solve_bytes = (SOLVE_BYTES_PER_CONTACT_ITER * prof["solver_contact_iters"] +
                   SOLVE_BYTES_PER_NODE_ITER * prof["solver_node_iters"] +
                   SOLVE_BYTES_PER_CONTACT_ROUND * prof["solver_contact_rounds"])
    algo_bytes = {
        "p2g": P2G_BYTES_PER_PARTICLE * P * launches["p2g"],
        "g2p": G2P_BYTES_PER_PARTICLE * P * launches["g2p"],
        "sort": SORT_BYTES_PER_PARTICLE * P * launches["sort"],
        "solve": solve_bytes,
    }
    kernels = {}
    for k in M.KERNEL_CLASSES:
        if launches[k] == 0:
            continue
        e = {"ms_total": round(ms[k], 3), "launches": int(launches[k]),
             "us_per_launch": round(1e3 * ms[k] / launches[k], 2),
             "share": round(ms[k] / total_ms, 4) if total_ms > 0 else None}
        if k in algo_bytes and ms[k] > 0:
            gbs = algo_bytes[k] / (ms[k] * 1e-3) / 1e9
            e["algo_GBps"] = round(gbs, 1)
            e["frac_hbm_peak"] = round(gbs / HBM_PEAK_GBS, 4)
        kernels[k] = e
    dominant = max(kernels, key=lambda k: kernels[k]["ms_total"])
    dom = kernels[dominant]
    roofline = {"kernel": dominant, "bound": "hbm", "achieved": dom.get("algo_GBps"),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom.get("frac_hbm_peak"),
                "traffic": measured_traffic() if dominant == "solve" else None}
    iters = [i for st in stats for i in st["iterations"]]
    contacts = [c for st in stats for c in st["contacts"]]
    nodes = [c for st in stats for c in st["contact_nodes"]]
    noconv = sum(1 for st in stats if st["flags"] & M.FLAG_NOCONV)
    solver = {
        "iterations_per_substep_mean": round(float(np.mean(iters)), 1),
        "iterations_per_substep_max": int(max(iters)),
        "contacts_mean": round(float(np.mean(contacts)), 1), "contacts_max": int(max(contacts)),
        "contact_nodes_mean": round(float(np.mean(nodes)), 1),
        "us_per_iteration": (round(1e3 * ms["solve"] / prof["solver_iterations"], 2)
                             if prof["solver_iterations"] else None),
        "ls_rounds_per_iteration": (round(prof["solver_ls_rounds"] / prof["solver_iterations"], 2)
                                    if prof["solver_iterations"] else None),
        "phase_us_per_iteration": ({k: round(v / phase_prof["solver_iterations"], 2)
                                    for k, v in phase_prof["solver_phase_us"].items()}
                                   if phase_prof["solver_iterations"] else None),
        "phase_us_note": "one extra untimed host step with the phase timers on",
        "host_steps_not_converged": noconv,
        "residual_over_threshold_max": max(
            (r / t for st in stats for r, t in zip(st["residual"], st["threshold"]) if t > 0),
            default=None),
    }
    out = {
        "metric": "particle-substeps/s (plain substep at contact residual 1e-6)",
        "value": value, "unit": "particle-substeps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": (f"granular pour: {P} Drucker-Prager sand particles, 128^3 grid, "
                                f"4 static boxes, h=1e-4 s, {N} substeps per host step, "
                                f"eps_r=1e-6; one step = one host step"),
                   "particles": P, "substeps_per_step": N, "parallelism": "single GPU"},
        "roofline": roofline,
        "kernels": kernels,
        "solver": solver,
    }
    state = sim.state()
    sim.close()
    if not args.no_cpu_baseline:
        log("cpu baseline: FP64 oracle on a column sample")
        out["cpu_baseline"] = cpu_baseline(state, scene, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    rc = main()
    if rc:
        sys.exit(rc)
