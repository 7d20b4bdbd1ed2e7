#!/usr/bin/env python
"""Throughput of the coupled MPM-rigid substep on one MI355X.

One invocation measures the three forms of the metric (particle-substeps/s at
contact residual eps_r = 1e-6, eps_a = FP64 machine epsilon), each on its
configuration, all inputs seeded, synthetic and resident in HBM before the
timed regions start:

* plain (the line's `value`): the granular pour, 1,000,000 Drucker-Prager
  sand particles on a 128^3 grid falling at 1 m/s onto four static boxes,
  h = 1e-4 s, N = 10 substeps per host step, 200 substeps = 20 host steps.
  One step = one host step (the once-per-step cell sort and ten substeps of
  P2G, grid update, registration, contact-node table, Algorithm 1 to
  convergence, G2P with the return map). The timed window is the K host
  steps after W warmup host steps of that 20-host-step run; a window that
  reaches past host step 19 continues on a fresh copy of the initial state
  (so K = 20 times every host step of the run exactly once);
* batched: 64 independent environments (log-uniform 5k-100k particles, 64^3
  grids, elastic or sand, 1-3 boxes each), the configuration's 100 substeps
  (10 host steps) in one handle, as a HIP graph replay, and looping
  single-environment handles over all 64 environments;
* forward + backward: a 200k-particle elastic cube pushed by a box, 50
  substeps with a checkpoint every 10, the loss x of the final centre of
  mass differentiated with respect to the initial velocity, E and the box
  velocity; cost relative to the plain forward, and the 3 x 7 Jacobian.

Also: the gripper in dense contact (250k particles, about 2e4 contacts), P2G
and G2P at 4M particles (past the 256 MB last-level cache), per-kernel
figures from HIP events recorded on the library's stream inside the timed
region, a roofline entry for the kernel that takes most of the time, and the
FP64 CPU oracle timed beside the GPU on one substep of the granular pour in
contact.
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
RUN_HOST_STEPS = 20    # the granular pour's 200 substeps
BATCH_HOST_STEPS = 10  # the batched configuration's 100 substeps
DIFF_HOST_STEPS = 5    # the differentiable configuration's 50 substeps

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


# Bandwidth of a plain device-to-device copy measured on this GPU at start-up
# (read plus write bytes over event time, the best of several copies of 1
# GiB): the rate a streaming kernel can reach here, beside the vendor peak.
_COPY_PEAK_GBS = None


def stream_copy_peak(n_bytes: int = 1 << 30, reps: int = 10) -> float:
    import torch
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = 0.0
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = max(best, 2.0 * n_bytes / (a.elapsed_time(b) * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return best


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def kernel_table(prof: dict, P: int) -> dict:
    """Per kernel class: event time, launches, and for the streaming kernels
    and the solver their algorithmic bytes over the time as a fraction of HBM
    peak."""
    from paper_2503_05046_amd import mpm as M
    ms, launches = prof["ms"], prof["launches"]
    total_ms = sum(ms.values())
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
            if _COPY_PEAK_GBS:
                e["frac_copy_peak"] = round(gbs / _COPY_PEAK_GBS, 4)
        kernels[k] = e
    return kernels


def substep_hbm(kernels: dict, prof: dict, P: int) -> dict:
    """The whole substep: the algorithmic bytes of P2G, G2P, the sort and the
    solve (the grid sweep's are not counted) over the event time of every
    kernel class, as a fraction of HBM peak."""
    launches = prof["launches"]
    algo = (P2G_BYTES_PER_PARTICLE * P * launches["p2g"] + G2P_BYTES_PER_PARTICLE * P * launches["g2p"] +
            SORT_BYTES_PER_PARTICLE * P * launches["sort"] +
            SOLVE_BYTES_PER_CONTACT_ITER * prof["solver_contact_iters"] +
            SOLVE_BYTES_PER_NODE_ITER * prof["solver_node_iters"] +
            SOLVE_BYTES_PER_CONTACT_ROUND * prof["solver_contact_rounds"])
    ms = sum(e["ms_total"] for e in kernels.values())
    gbs = algo / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    out = {"algo_bytes": algo, "ms_total": round(ms, 3), "algo_GBps": round(gbs, 1),
           "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 5)}
    if _COPY_PEAK_GBS:
        out["frac_copy_peak"] = round(gbs / _COPY_PEAK_GBS, 5)
    return out


def add_profiles(a: dict, b: dict) -> dict:
    out = {}
    for k, v in a.items():
        if isinstance(v, dict):
            out[k] = {q: v[q] + b[k][q] for q in v}
        else:
            out[k] = v + b[k]
    return out


def solver_summary(stats: list, prof: dict, phase_prof: dict) -> dict:
    import numpy as np
    from paper_2503_05046_amd import mpm as M
    iters = [i for st in stats for i in st["iterations"] if i > 0]
    contacts = [c for st in stats for c in st["contacts"]]
    nodes = [c for st in stats for c in st["contact_nodes"]]
    return {
        "iterations_per_contact_substep_mean": round(float(np.mean(iters)), 1) if iters else 0,
        "iterations_per_substep_max": int(max(iters)) if iters else 0,
        "contacts_mean": round(float(np.mean(contacts)), 1), "contacts_max": int(max(contacts)),
        "contact_nodes_mean": round(float(np.mean(nodes)), 1),
        "us_per_iteration": (round(1e3 * prof["ms"]["solve"] / prof["solver_iterations"], 2)
                             if prof["solver_iterations"] else None),
        "ls_rounds_per_iteration": (round(prof["solver_ls_rounds"] / prof["solver_iterations"], 2)
                                    if prof["solver_iterations"] else None),
        "phase_us_per_iteration": ({k: round(v / phase_prof["solver_iterations"], 2)
                                    for k, v in phase_prof["solver_phase_us"].items()}
                                   if phase_prof and phase_prof["solver_iterations"] else None),
        "host_steps_not_converged": sum(1 for st in stats if st["flags"] & M.FLAG_NOCONV),
        "residual_over_threshold_max": max(
            (r / t for st in stats for r, t in zip(st["residual"], st["threshold"]) if t > 0), default=None),
    }


# ---------------------------------------------------------------------------
# plain form: the granular pour
# ---------------------------------------------------------------------------
def run_plain(args) -> dict:
    import torch
    from paper_2503_05046_amd import inputs as I
    from paper_2503_05046_amd import mpm as M

    scene = I.granular_pour(n_particles=args.particles)
    scene.max_iter = args.max_iter
    P, N = scene.P, scene.N
    W, K = args.warmup, args.steps
    n_runs = (W + K + RUN_HOST_STEPS - 1) // RUN_HOST_STEPS
    log(f"plain: granular pour P={P}, grid {tuple(scene.envs[0].dims)}, N={N}, h={scene.h}, "
        f"eps_r={scene.eps_r}; warmup {W}, timed {K} host steps over {n_runs} copies of the run")
    sims = [M.Sim(scene, device="cuda:0") for _ in range(n_runs)]  # each from the initial state
    torch.cuda.synchronize()

    step_ms = []

    def step_at(j, tag):
        sim = sims[j // RUN_HOST_STEPS]
        t = time.perf_counter()
        status, imp, st = sim.step()
        ms = 1e3 * (time.perf_counter() - t)
        if tag == "timed":
            step_ms.append(ms)
        log(f"{tag} host step {j % RUN_HOST_STEPS} of run {j // RUN_HOST_STEPS}: "
            f"{ms:.1f} ms, contacts max {st['max_contacts']}, "
            f"iterations/substep {st['iterations']}, flags {st['flags']}")
        return st

    for j in range(W):
        step_at(j, "warmup")
    for s in sims:
        s.profile(True)  # reset and start event timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step_at(j, "timed") for j in range(W, W + K)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = None
    for s in sims:
        p = s.profile(0)
        prof = p if prof is None else add_profiles(prof, p)
    # one more host step, untimed, with the solver's phase timers on (their
    # clock reads lengthen the solve); on the first copy, in contact
    sims[0].profile(2)
    sims[0].step()
    phase_prof = sims[0].profile(0)
    for s in sims:
        s.close()
    kernels = kernel_table(prof, P)
    whole = substep_hbm(kernels, prof, P)
    solver = solver_summary(stats, prof, phase_prof)
    dominant = max(kernels, key=lambda k: kernels[k]["ms_total"])
    dom = kernels[dominant]
    roofline = {"kernel": dominant,
                "bound": "latency" if dominant == "solve" else "hbm",
                "achieved": dom.get("algo_GBps"), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom.get("frac_hbm_peak"),
                "traffic": measured_traffic() if dominant == "solve" else None}
    if dominant == "solve":
        roofline["us_per_iteration"] = solver["us_per_iteration"]
        roofline["note"] = ("Algorithm 1 is a chain of dependent steps per iteration (group barrier, "
                            "memory round trips, block reductions): latency-bound; frac is its "
                            "algorithmic bytes per launch over HBM peak, us_per_iteration its cost")
    return {
        "value": P * N * K / elapsed, "elapsed_s": elapsed, "ms_per_step": 1e3 * elapsed / K,
        "window": (f"host steps {W % RUN_HOST_STEPS}.. of the {RUN_HOST_STEPS}-host-step "
                   f"({RUN_HOST_STEPS * N}-substep) run after {W} warmup host steps, {K} timed; "
                   f"past host step {RUN_HOST_STEPS - 1} the window continues on a fresh copy of "
                   f"the initial state"),
        "host_step_ms": [round(t, 1) for t in step_ms],
        "roofline": roofline, "kernels": kernels, "substep_hbm": whole, "solver": solver, "scene": scene,
    }


def run_streaming_4m(args) -> dict:
    """P2G and G2P at 4M particles (the granular pour at 4x the density on the
    same 128^3 grid, before contact): the state (384 MB) exceeds the 256 MB
    last-level cache, so the kernels stream from HBM."""
    import torch
    from paper_2503_05046_amd import inputs as I
    from paper_2503_05046_amd import mpm as M
    scene = I.granular_pour(n_particles=4_000_000)
    sim = M.Sim(scene, device="cuda:0")
    sim.step()  # warm
    sim.profile(True)
    torch.cuda.synchronize()
    sim.step()
    torch.cuda.synchronize()
    prof = sim.profile(0)
    sim.close()
    k = kernel_table(prof, scene.P)
    return {"particles": scene.P, "p2g": k.get("p2g"), "g2p": k.get("g2p"), "sort": k.get("sort"),
            "grid": k.get("grid")}


def run_gripper_dense(args) -> dict:
    """The gripper in dense contact: both jaws started 0.065 m inside the
    ellipsoid's tips (about 2e4 particles inside the jaws), one substep from
    that state (the host step of one substep). At the benchmark tolerance
    eps_r = 1e-6 Algorithm 1 converges on this first substep; on the following
    substeps of the violent expulsion the block-diagonal iteration needs more
    than 2e5 iterations, so the line is the converged first substep, with the
    tolerance sweep of the same substep beside it (iterations, time, and the
    velocity change against the eps_r = 1e-6 result in the mass norm)."""
    import numpy as np
    import torch
    from paper_2503_05046_amd import inputs as I
    from paper_2503_05046_amd import mpm as M
    base = I.gripper(overlap=0.065)
    base.N = 1
    out = {"config": "gripper: 250000 elastic particles, 96^3 grid, two jaws closing at 0.05 m/s started 0.065 m "
                     "inside the tips, mu=0.8, h=1e-4 s, one substep from that state",
           "sweep": []}
    ref_v = None
    for eps_r in (1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 5e-2, 1e-1):
        scene = base.copy()
        scene.eps_r = eps_r
        scene.max_iter = args.max_iter
        sim = M.Sim(scene, device="cuda:0")
        sim.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status, imp, st = sim.step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = sim.profile(0)
        v = sim.state()["v"].astype(np.float64)
        sim.close()
        if ref_v is None:
            ref_v = v
        m_p = scene.envs[0].m_p
        drift = float(np.sqrt(m_p * np.sum((v - ref_v) ** 2)))
        row = {"eps_r": eps_r, "status": status, "iterations": st["iterations"][0], "seconds": round(dt, 4),
               "us_per_iteration": (round(1e3 * prof["ms"]["solve"] / prof["solver_iterations"], 2)
                                    if prof["solver_iterations"] else None),
               "contacts": st["contacts"][0], "contact_nodes": st["contact_nodes"][0],
               "dv_mass_norm_vs_1e-6": drift}
        log(f"gripper dense, eps_r {eps_r:g}: {row}")
        out["sweep"].append(row)
        if eps_r == 1e-6:
            out.update({"value": scene.P / dt, "unit": "particle-substeps/s", "seconds": dt,
                        "contacts": st["contacts"][0], "contact_nodes": st["contact_nodes"][0],
                        "iterations": st["iterations"][0], "us_per_iteration": row["us_per_iteration"],
                        "status": status})
    return out


def run_solver_variants(args) -> dict:
    """Algorithm 1 (block-diagonal quasi-Newton) against the exact-Newton study
    variant (the full Hessian system by preconditioned conjugate gradients)
    on one substep of two dense-contact states at eps_r = 1e-6: the granular
    pour started with its bottom layer 0.7 mm inside the box tops at 1 m/s,
    and the gripper with both jaws 0.065 m inside the ellipsoid. Both solves
    stop at the same test; their results differ by less than the sum of their
    thresholds in the mass norm."""
    import numpy as np
    import torch
    from paper_2503_05046_amd import inputs as I
    from paper_2503_05046_amd import mpm as M
    scenes = {"granular_pour": I.granular_pour(n_particles=args.particles, sink=0.5 / 128 + 7e-4),
              "gripper": I.gripper(overlap=0.065)}
    out = {}
    for name, scene in scenes.items():
        scene.N = 1
        scene.max_iter = args.max_iter
        rows = {}
        vs = {}
        for label, solver in (("quasi_newton", M.SOLVER_QN), ("exact_newton", M.SOLVER_NEWTON)):
            sim = M.Sim(scene, device="cuda:0", solver=solver)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            status, imp, st = sim.step()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            vs[label] = sim.state()["v"].astype(np.float64)
            sim.close()
            rows[label] = {"status": status, "seconds": round(dt, 4), "iterations": st["iterations"][0],
                           "cg_iterations": st["inner_iterations"], "contacts": st["contacts"][0],
                           "contact_nodes": st["contact_nodes"][0], "threshold": st["threshold"][0],
                           "residual": st["residual"][0]}
            log(f"solver variants, {name}, {label}: {rows[label]}")
        m_p = scene.envs[0].m_p
        rows["dv_mass_norm"] = float(np.sqrt(m_p * np.sum((vs["quasi_newton"] - vs["exact_newton"]) ** 2)))
        rows["threshold_sum"] = rows["quasi_newton"]["threshold"] + rows["exact_newton"]["threshold"]
        rows["speedup_exact_over_qn"] = rows["quasi_newton"]["seconds"] / rows["exact_newton"]["seconds"]
        out[name] = rows
    return out


def run_sort_policies(args) -> dict:
    """The sort ablation of Sec. V-A on the granular pour before contact (host
    steps 1-2 of the run, 20 substeps): full keys once per host step with the
    LDS-tiled P2G and G2P (the library's default), full keys every substep
    (one substep per host step), the paper's truncated 10-bit keys once per
    host step, and no reordering; the last two with the plain scatter (27 x 4
    float atomics per particle into the grid) and gather. Per-launch times from
    the library's HIP events."""
    import torch
    from paper_2503_05046_amd import inputs as I
    from paper_2503_05046_amd import mpm as M
    arms = [("tiles, once per host step", None, 10), ("tiles, every substep", None, 1),
            ("truncated 10-bit keys, once per host step", "truncated", 10), ("no sort", "none", 10)]
    out = []
    for label, policy, N in arms:
        if policy is None:
            os.environ.pop("MPM_SORT_POLICY", None)
        else:
            os.environ["MPM_SORT_POLICY"] = policy
        scene = I.granular_pour(n_particles=args.particles)
        scene.h, scene.N = scene.h, N
        sim = M.Sim(scene, device="cuda:0")
        sim.step()  # warm (no contact yet)
        sim.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_host = 20 // N
        for _ in range(n_host):
            status, imp, st = sim.step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = sim.profile(0)
        sim.close()
        k = kernel_table(prof, scene.P)
        row = {"arm": label, "us_per_substep": round(1e6 * dt / 20, 1),
               "sort_us_per_substep": round(1e3 * prof["ms"]["sort"] / 20, 1),
               "p2g_us": k["p2g"]["us_per_launch"], "grid_us": k["grid"]["us_per_launch"],
               "g2p_us": k["g2p"]["us_per_launch"], "contacts_max": st["max_contacts"]}
        log(f"sort policy: {row}")
        out.append(row)
    os.environ.pop("MPM_SORT_POLICY", None)
    return {"config": f"granular pour, {args.particles} particles, 128^3 grid, 20 substeps before contact",
            "arms": out}


def cpu_baseline(args) -> dict:
    """The FP64 oracle, as it stands, single-threaded, and the GPU library on
    the same input: one substep of the granular pour (1M particles) started
    with its bottom layer 0.7 mm inside the box tops at 1 m/s (the
    benchmark's contact density)."""
    import torch
    from oracle import oracle as O
    from paper_2503_05046_amd import inputs as I
    from paper_2503_05046_amd import mpm as M
    O.build(force=not os.path.exists(O.LIB))
    scene = I.granular_pour(n_particles=args.particles, sink=0.5 / 128 + 7e-4)
    scene.N = 1
    scene.max_iter = args.max_iter
    sim = M.Sim(scene, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, _, st_g = sim.step()
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    sim.close()
    log(f"cpu baseline: GPU {t_gpu:.3f} s, {st_g['iterations'][0]} iterations; now the oracle")
    ora = O.OracleSim(scene)
    t0 = time.perf_counter()
    rc, _, st_o = ora.host_step()
    t_cpu = time.perf_counter() - t0
    st_o = st_o[0]
    return {"value": scene.P / t_cpu, "unit": "particle-substeps/s", "cores": 1, "kind": "oracle",
            "sample": (f"one substep of the {scene.P}-particle granular pour started 0.7 mm inside the box "
                       f"tops at 1 m/s: {st_o['n_contacts']} contacts, {st_o['n_contact_nodes']} contact "
                       f"nodes, {st_o['iterations']} Algorithm 1 iterations, {t_cpu:.1f} s single-threaded "
                       f"FP64"),
            "status": rc, "oracle_iterations": st_o["iterations"],
            "gpu_same_sample": {"value": scene.P / t_gpu, "seconds": t_gpu,
                                "iterations": st_g["iterations"][0], "contacts": st_g["contacts"][0]},
            "host": host_info()}


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------
def run_batched(args) -> dict:
    import numpy as np
    import torch
    from paper_2503_05046_amd import inputs as I
    from paper_2503_05046_amd import mpm as M

    scene = I.batched()
    scene.max_iter = args.max_iter
    P, N, n_envs = scene.P, scene.N, len(scene.envs)
    K = BATCH_HOST_STEPS
    log(f"batched: {n_envs} environments, P={P}, the {K} host steps of the run")
    spb, tuning = 0, None
    if args.autotune:
        from paper_2503_05046_amd import autotune
        spb, tuning = autotune.tune(scene, candidates=(64, 96, 128, 192, 256), warmup_steps=8,
                                    trial_steps=2, log=log)
        log(f"autotune: {spb} contact nodes per solver block")
    # warm the kernels at these sizes (a throwaway handle, one host step)
    w = M.Sim(scene, solver_slots_per_block=spb)
    w.step()
    w.close()
    sim = M.Sim(scene, solver_slots_per_block=spb)
    sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    longest = []
    for i in range(K):
        _, _, st = sim.step()
        longest += st["iterations"]
        log(f"batched host step {i}: contacts {st['contacts']}, longest solve {max(st['iterations'])} iterations")
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    prof = sim.profile(False)
    sim.close()
    # the same run as one HIP graph replay (recording included)
    gsim = M.Sim(scene, solver_slots_per_block=spb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gsim.step_graph(K)
    torch.cuda.synchronize()
    t_g = time.perf_counter() - t0
    gsim.close()
    log(f"graph: {K} host steps in one replay, {t_g:.2f} s")
    # looping single-environment handles over every environment
    sims = [M.Sim(I.single_env(scene, e)) for e in range(n_envs)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        for s in sims:
            s.step()
        log(f"loop host step {i} done ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    for s in sims:
        s.close()
    value_b = P * N * K / t_b
    value_l = P * N * K / t_loop
    return {
        "metric": "particle-substeps/s (batched, 64 environments, contact residual 1e-6)",
        "value": value_b, "unit": "particle-substeps/s", "ms_per_host_step": 1e3 * t_b / K,
        "config": (f"batched: {n_envs} independent environments, {P} particles (log-uniform 5k-100k each), "
                   f"64^3 grids, elastic/sand, 1-3 boxes, h=1e-4 s, {K * N} substeps ({K} host steps), "
                   f"eps_r=1e-6"),
        "loop": {"value": value_l, "ms_per_host_step": 1e3 * t_loop / K,
                 "method": f"all {n_envs} single-environment handles stepped in turn, every host step"},
        "batched_over_loop": value_b / value_l,
        "graph": {"value": P * N * K / t_g, "ms_per_host_step": 1e3 * t_g / K,
                  "method": f"the {K} host steps as one HIP graph (mpm_step_graph), recording included"},
        "solver_slots_per_block": spb or 128,
        "autotune": ({"chosen": spb, "ms_per_step": {k: round(1e3 * t, 1) for k, t in tuning.items()}}
                     if tuning else None),
        "solve_share": prof["ms"]["solve"] / max(1e-9, sum(prof["ms"].values())),
        "longest_solve_iterations_mean": float(np.mean(longest)),
    }


# ---------------------------------------------------------------------------
# forward + backward form
# ---------------------------------------------------------------------------
def run_fwd_bwd(args) -> dict:
    import torch
    from paper_2503_05046_amd import diff
    from paper_2503_05046_amd import inputs as I
    from paper_2503_05046_amd import mpm as M

    scene = I.differentiable()
    scene.max_iter = args.max_iter
    P, N, steps = scene.P, scene.N, DIFF_HOST_STEPS
    log(f"forward + backward: P={P}, {steps} host steps of {N} substeps, checkpoint every host step")
    sim = M.Sim(scene, tape_substeps=N)
    path = diff.RigidPath(scene)
    dev = sim.device
    x0, v0, F0, C0 = (torch.from_numpy(a).to(dev) for a in (scene.x, scene.v, scene.F, scene.C))
    V0 = torch.tensor([list(r.V) for r in scene.rigids], dtype=torch.float64)
    E0 = torch.tensor([scene.envs[0].E], dtype=torch.float64)
    # one untimed host step first (first launches at these sizes)
    diff._run(sim, path, 1, 0, x0, v0, F0, C0, V0, record=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    diff._run(sim, path, steps, 0, x0, v0, F0, C0, V0, record=False)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    log(f"forward: {t_fwd:.2f} s")
    u = torch.zeros(3, dtype=torch.float32, device=dev, requires_grad=True)
    E = E0.clone().requires_grad_(True)
    V = V0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, v, F, C = diff.simulate(sim, path, steps, 1, x0, v0 + u[:, None], F0, C0, E, V)
    com = x.mean(dim=1)
    com[0].backward(retain_graph=True)
    torch.cuda.synchronize()
    t_fb = time.perf_counter() - t0
    log(f"forward + backward (row x): {t_fb:.2f} s")
    rows = [[*u.grad.cpu().tolist(), float(E.grad[0]), *V.grad[0].tolist()]]
    t0 = time.perf_counter()
    for a in (1, 2):  # the Jacobian's other rows: one more reverse pass each
        gu, gE, gV = torch.autograd.grad(com[a], (u, E, V), retain_graph=a < 2)
        rows.append([*gu.cpu().tolist(), float(gE[0]), *gV[0].tolist()])
    torch.cuda.synchronize()
    t_rows = time.perf_counter() - t0
    sim.close()
    return {
        "metric": "particle-substeps/s (forward + backward, contact residual 1e-6)",
        "value": P * N * steps / t_fb, "unit": "particle-substeps/s", "seconds": t_fb,
        "config": (f"differentiable: {P}-particle elastic cube, 96^3 grid, pushed by a box at 0.5 m/s, "
                   f"{N * steps} substeps, checkpoint every {N} substeps, eps_r=1e-6; loss x of the final "
                   f"centre of mass"),
        "forward_s": t_fwd, "forward_backward_s": t_fb, "fwd_bwd_over_fwd": t_fb / t_fwd,
        "forward_note": "both timed after one untimed host step on the same handle",
        "jacobian": {"rows": "d(mean x, mean y, mean z of the final particles)",
                     "columns": "d(initial velocity offset x, y, z), dE, d(box velocity x, y, z)",
                     "values": rows, "extra_rows_s": t_rows},
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--forms", default="plain,batched,fwd_bwd,gripper,4m,variants,sort",
                    help="comma-separated subset of plain, batched, fwd_bwd, gripper, 4m, variants, sort")
    ap.add_argument("--particles", type=int, default=1_000_000)
    ap.add_argument("--max-iter", type=int, default=200_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="batched form: pick the solver's contact nodes per block with the autotuner first")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one device copy of BYTES (scale for the PMC byte counters)")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (a single scene "
              "would shard into slabs, one per GPU, and the "
              "environments of the batched form would be assigned to GPUs whole). Run with --gpus 1.",
              file=sys.stderr)
        return 2
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        return 2
    forms = set(f.strip() for f in args.forms.split(",") if f.strip())

    out = {"metric": "particle-substeps/s (plain substep at contact residual 1e-6)"}
    global _COPY_PEAK_GBS
    _COPY_PEAK_GBS = stream_copy_peak()
    log(f"device copy: {_COPY_PEAK_GBS:.0f} GB/s (read + write)")
    if "plain" in forms:
        r = run_plain(args)
        scene = r.pop("scene")
        out.update({
            "value": r["value"], "unit": "particle-substeps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": (f"granular pour: {scene.P} Drucker-Prager sand particles, 128^3 grid, "
                                    f"4 static boxes, h=1e-4 s, {scene.N} substeps per host step, "
                                    f"{RUN_HOST_STEPS * scene.N} substeps, eps_r=1e-6; one step = one "
                                    f"host step"),
                       "particles": scene.P, "substeps_per_step": scene.N, "parallelism": "single GPU",
                       "window": r["window"]},
            "roofline": r["roofline"], "kernels": r["kernels"], "substep_hbm": r["substep_hbm"],
            "solver": r["solver"],
            "host_step_ms": r["host_step_ms"],
        })
    extra = {}
    if "4m" in forms:
        extra["streaming_4M"] = run_streaming_4m(args)
    if "gripper" in forms:
        extra["gripper_dense"] = run_gripper_dense(args)
    if "batched" in forms:
        extra["batched"] = run_batched(args)
    if "fwd_bwd" in forms:
        extra["fwd_bwd"] = run_fwd_bwd(args)
    if "variants" in forms:
        extra["solver_variants"] = run_solver_variants(args)
    if "sort" in forms:
        extra["sort_policies"] = run_sort_policies(args)
    if extra:
        out["forms"] = extra
    out["stream_copy_GBps"] = round(_COPY_PEAK_GBS, 1)
    if "plain" in forms and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    rc = main()
    if rc:
        sys.exit(rc)
