#!/usr/bin/env python
"""RKC stages/s of the explicit EQS hot path on one MI355X.

Workload (default "c2"): the unit cube meshed with 128^3 sub-cubes split into
6 P1 tets each (2,146,689 nodes, 12,582,912 tets, 2,113,407 free DOF),
grounded at z = 0, driven by sin(2 pi 50 t) at z = 1, with seeded spherical
microvaristor inclusions (5 % of the volume, kappa = 1e-10 (1 + (|E|/0.5)^alpha),
alpha ~ U[8, 14], eps_r ~ U[8, 15]) in an eps_r = 4, kappa = 1e-12 host.
Each RKC(16) step runs 16 stages; a stage is one fused element pass
(K(x)x + Dirichlet RHS), one AMG-preconditioned CG solve of M to rel-res 1e-8
(FP64 CG, FP32 AMG hierarchy and V-cycle), and one RKC combination.

Prints ONE JSON line (rank 0). `value` = stages/s of the timed steps with all
inputs resident in HBM. Beside it: the plain FP64 path (FP64 hierarchy) over
the same steps, the roofline of the dominant kernel from per-launch HIP events
in an instrumented window that follows the timed steps, optionally
(--learned-steps) every start vector over a common window and (--c3-steps) the
64-instance batched workload, and the FP64 CPU oracle timed on one stage of the
same workload (cpu_baseline). --gpus N > 1 exits: the library runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

METRIC = "RKC stages/s at 2.1M DOF (rel-res 1e-8), HBM GB/s; mixed+learned vs FP64"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def element_bytes(info):
    # algorithmic bytes of one element pass: per tet its connectivity (4 x 4 B)
    # and material id (4 B); per node its coordinates (24 B), potential (8 B)
    # and result (8 B), each array touched once. The library's packed tet
    # records need 8 B instead of 20; re-reads of nodes shared between element
    # blocks and the block node lists are overhead, not counted.
    return info["n_tets"] * 20 + info["n_nodes"] * (24 + 8 + 8)


def spmv_bytes(info, nnz):
    # CG product q = M z + beta q, p = z + beta p on the free DOF: value (8 B)
    # and column id (4 B) per stored nonzero, slice offsets, z read, p and q
    # read and written. With 16-bit column offsets the kernel reads 10 B per
    # nonzero, not 12.
    n = info["n_free"]
    return 12 * nnz + 4 * (n // 64 + 1) + 8 * n + 32 * n


def copy_probe(mib=512, reps=20):
    """Bandwidth of a plain device-to-device copy (torch's copy kernel) of
    `mib` MiB: the measured streaming ceiling beside the nominal peak, and the
    reference launch that scales the HBM byte counters."""
    import torch

    src = torch.empty(mib << 17, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for r in range(reps + 2):
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        ev[1].synchronize()
        if r >= 2:
            times.append(ev[0].elapsed_time(ev[1]) * 1e-3)
    times.sort()
    nbytes = 2 * src.numel() * 8
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_per_launch": nbytes, "median_us": round(times[len(times) // 2] * 1e6, 2),
            "GB/s": round(nbytes / times[len(times) // 2] / 1e9, 1)}


def read_probe(mib=1024, reps=20):
    """Bandwidth of a read-only pass (torch's sum) over `mib` MiB: the streaming
    ceiling for kernels that mostly read, as the sparse products do."""
    import torch

    src = torch.empty(mib << 17, dtype=torch.float64, device="cuda:0").fill_(1.0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for r in range(reps + 2):
        ev[0].record()
        src.sum()
        ev[1].record()
        ev[1].synchronize()
        if r >= 2:
            times.append(ev[0].elapsed_time(ev[1]) * 1e-3)
    times.sort()
    nbytes = src.numel() * 8
    del src
    torch.cuda.empty_cache()
    return {"bytes_per_launch": nbytes, "median_us": round(times[len(times) // 2] * 1e6, 2),
            "GB/s": round(nbytes / times[len(times) // 2] / 1e9, 1)}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c2_hbm_traffic.txt")
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_1612_09447_amd", "csrc", f) for f in ("kernels.hip", "sell.h")]


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel_class):
    """HBM bytes per launch of a kernel class from the committed counter
    summary, or None when there is none or the kernel sources have changed
    since the counters were taken."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    sha, val = None, None
    for ln in lines:
        f = ln.split()
        if len(f) >= 2 and f[0] == "source_sha256":
            sha = f[1]
        if len(f) >= 3 and f[0] == "traffic" and f[1] == kernel_class:
            val = int(f[2])
    return val if sha == kernel_source_hash() else None


def mixed_learned_vs_fp64(plain, learned, full):
    """Stage rate of the mixed-precision form with the network start vector
    relative to the plain FP64 path. `value`: both run the same timed steps
    from t = 0 (whole-run rates). Beside it, the product of same-window ratios
    from the start-vector comparison: network vs plain start (both mixed
    precision) times mixed precision vs FP64 (plain start)."""
    if not plain or "fp32_form_speedup" not in plain:
        return None
    out = {"fp32_form_vs_fp64": plain["fp32_form_speedup"]}
    if full and "mlp" in full and plain.get("steps") == full["mlp"]["steps"]:
        out["value"] = round(full["mlp"]["stages_per_s"] / plain["stages_per_s"], 3)
        out["basis"] = f"whole runs of {plain['steps']} steps: FP32 form + network start vector vs plain FP64"
        if "error_vs_fp64" in full["mlp"]:
            out["error_vs_fp64"] = full["mlp"]["error_vs_fp64"]
    if learned and "mlp" in learned:
        net = learned["mlp"]["stages_per_s"] / learned["previous"]["stages_per_s"]
        out["window_product"] = round(net * plain["fp32_form_speedup"], 3)
        out["network_vs_plain_start_in_window"] = round(net, 3)
    return out if "value" in out or "window_product" in out else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


# kernel classes timed one launch at a time (each launch is one kernel)
SINGLE_KERNEL_CLASSES = ("element", "spmv_M", "presmooth0", "postsmooth0", "restrict0", "prolong0", "postsmooth1",
                         "cg_update", "rkc_combine")
# classes spanning several kernels (bracketed by events on the stream)
MULTI_KERNEL_CLASSES = ("vcycle", "vcoarse", "finalise")
ALL_CLASSES = SINGLE_KERNEL_CLASSES + MULTI_KERNEL_CLASSES
KERNEL_NAMES = {"element": "k_kx<true> (element pass)", "spmv_M": "k_pcg_spmv", "presmooth0": "k_presmooth_res (finest)",
                "postsmooth0": "k_postsmooth (finest)", "restrict0": "k_restrict (finest level, R0)",
                "prolong0": "k_prolong (finest level, P0)", "postsmooth1": "k_postsmooth (level 1)",
                "cg_update": "k_pcg_update",
                "rkc_combine": "k_rkc_first / k_rkc_combine"}


def class_bytes(info, s_stages):
    """Algorithmic bytes per launch of every single-kernel class: each array
    the kernel must touch, once, at its own width (4 B per index; hierarchy
    values 4 B in the FP32 form, 8 B in FP64; CG vectors 8 B)."""
    n = info["n_free"]
    w = 4 if info["precision"] == 1 else 8
    rows, nnz = info["level_rows"], info["level_nnz"]
    pn, rn = info["level_p_nnz"], info["level_r_nnz"]
    n0 = rows[0]
    out = {
        "element": element_bytes(info),
        "spmv_M": spmv_bytes(info, info["nnz_M"]),
        "cg_update": 48 * n,  # x, r read and written; p, q read
        # Y_j from Y_0, Y_{j-1}, Y_{j-2}, F_{j-1}, F_0 (the first stage: Y_0, F_0),
        # the next stage's element-pass output cleared (not after the last)
        "rkc_combine": (32 + 56 * (s_stages - 2) + 48) * n // s_stages,
        # x = w D^-1 r, res = r - A w D^-1 r: operator, r (FP64), dinv, x, res
        "presmooth0": (w + 4) * nnz[0] + 4 * (n0 // 64 + 1) + n0 * (8 + 3 * w),
        # z = x + w D^-1 (r - A x) with r.z and r.z_old: operator, x gathered,
        # dinv, r (FP64), z_old read, z written
        "postsmooth0": (w + 4) * nnz[0] + 4 * (n0 // 64 + 1) + n0 * (2 * w + 24),
    }
    if len(rows) > 1:
        n1 = rows[1]
        out["restrict0"] = (w + 4) * rn[0] + 4 * (n1 + 1) + w * n0 + w * n1  # R0, res read, b_1 written
        out["prolong0"] = (w + 4) * pn[0] + 4 * (n0 + 1) + w * n1 + 2 * w * n0  # P0, x_1 read, x_0 updated
    if len(rows) > 2:
        n1 = rows[1]
        # level 1: out = x + w D^-1 (b - A x): operator, x gathered, dinv, b, out (hierarchy precision)
        out["postsmooth1"] = (w + 4) * nnz[1] + 4 * (n1 // 64 + 1) + n1 * 4 * w
    return out


def timed_steps(ctx, x, n, steps, tau, s, rtol, label, hist=None, steplog=None, stage_iters=None):
    """Run `steps` RKC steps from step index n; returns (elapsed s, per-step
    mean CG iterations per stage, guesses used, guard fallbacks). With `hist`
    (a device tensor [steps, n_nodes]) every step-end state is copied into it
    on the same stream (a device copy of one vector per step, inside the timed
    loop); a `stage_iters` list receives every stage's CG iterations."""
    import torch

    torch.cuda.synchronize()
    t1 = time.perf_counter()
    iters, used, fallbacks = [], 0, 0
    for k in range(steps):
        if steplog is not None:
            st = steplog.step(ctx, n + k, (n + k) * tau, tau, s, x, rtol, maxit=500)
        else:
            st = ctx.rkc_step((n + k) * tau, tau, s, x, rtol=rtol, maxit=500)
        if hist is not None:
            hist[k].copy_(x)
        iters.append(st["total_iters"] / st["stages"])
        if stage_iters is not None:
            stage_iters.extend(st["stage_iters"])
        used += st["guess_used"]
        fallbacks += st["guess_fallbacks"]
        if (k + 1) % max(1, steps // 5) == 0:
            log(f"[bench] {label} step {k + 1}/{steps} mean CG it/stage {sum(iters) / len(iters):.2f}")
    torch.cuda.synchronize()
    return time.perf_counter() - t1, iters, used, fallbacks


def run_gpu(case, precision, steps, warmup, rtol, prof_steps=0, guess="previous", flexible=0, learned_steps=0,
            learned_warmup=20, mlp_batch=256, keep_states=False, mlp_warmup=64, graph_iters=1, steplog=None,
            mlp_seed=4):
    """Time `steps` RKC steps (uninstrumented), then `prof_steps` more with every
    kernel class timed by HIP events on the context's stream. With
    learned_steps > 0 the same context then switches to the Galerkin and the
    network start vectors and times that many steps of each (after
    learned_warmup untimed steps that fill the snapshot window and the replay
    buffer)."""
    import torch

    import eqsgen
    from paper_1612_09447_amd import Context

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    t0 = time.perf_counter()
    ctx = Context(0, stream)
    ctx.set_graph_iters(graph_iters)
    info = ctx.setup_case(case, precision=precision, flexible=flexible)
    # PyTorch owns the device memory: the context moves into a torch workspace
    # sized for its largest start-vector setting of this run
    if guess == "mlp" or learned_steps > 0:
        ctx.set_guess("mlp", init=eqsgen.mlp_init(mlp_seed), batch=mlp_batch, warmup=mlp_warmup)
    elif guess != "previous":
        ctx.set_guess(guess)
    ws = ctx.use_torch_workspace()
    if guess != "mlp":
        ctx.set_guess(guess)
    info = ctx.info()
    assert info["device_bytes"] == 0
    setup_s = time.perf_counter() - t0
    log(f"[bench] setup precision={precision} guess={guess}: {setup_s:.1f}s\n" + ctx.describe())
    x = torch.zeros(case.n_nodes, dtype=torch.float64, device=dev)
    tau, s = case.tau, case.s
    n = 0
    for _ in range(warmup):
        ctx.rkc_step(n * tau, tau, s, x, rtol=rtol, maxit=500)
        n += 1
    hist = torch.empty((steps, case.n_nodes), dtype=torch.float64, device=dev) if keep_states else None
    stage_its = []
    elapsed, iters, used, fallbacks = timed_steps(ctx, x, n, steps, tau, s, rtol, f"{precision}/{guess}", hist,
                                                  steplog, stage_its)
    n += steps
    x_timed = x.cpu().numpy()  # state after warmup + timed steps (compared across precisions)
    prof, prof_elapsed = {}, 0.0
    if prof_steps > 0:
        ctx.profile_enable(ALL_CLASSES)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(prof_steps):
            ctx.rkc_step(n * tau, tau, s, x, rtol=rtol, maxit=500)
            n += 1
        torch.cuda.synchronize()
        prof_elapsed = time.perf_counter() - t2
        prof = {c: ctx.profile_read(c) for c in ALL_CLASSES}
        ctx.profile_enable(())
    learned = {}
    if learned_steps > 0:
        # every start vector runs the same steps from the same state: warm-up
        # steps (filling the snapshot window and the replay buffer), then the
        # timed ones
        x0 = x.clone()
        for kind in ("previous", "zero", "galerkin", "mor", "mlp"):
            x.copy_(x0)
            if kind == "mlp":
                ctx.set_guess("mlp", init=eqsgen.mlp_init(mlp_seed), batch=mlp_batch, warmup=mlp_warmup)
            else:
                ctx.set_guess(kind)
            timed_steps(ctx, x, n, learned_warmup, tau, s, rtol, f"{kind} warm-up")
            el, it, u, fb = timed_steps(ctx, x, n + learned_warmup, learned_steps, tau, s, rtol, kind)
            learned[kind] = {"stages_per_s": round(learned_steps * s / el, 2),
                             "mean_cg_iters_per_stage": round(sum(it) / len(it), 2),
                             "guess_used": u, "guard_fallbacks": fb}
        learned["window"] = {"first_step": n + learned_warmup, "steps": learned_steps,
                             "warmup_steps": learned_warmup, "mlp_pairs_per_stage": mlp_batch}
        ctx.set_guess("previous")
    ctx.close()
    del ws
    return dict(elapsed=elapsed, stages=steps * s, iters=iters, stage_iters=stage_its, info=info, prof=prof,
                prof_elapsed=prof_elapsed,
                prof_stages=prof_steps * s, setup_s=setup_s, x=x_timed, used=used, fallbacks=fallbacks, learned=learned,
                hist=hist)


def stage_iter_stats(its):
    """Mean, median and extremes of the timed stages' CG iterations."""
    if not its:
        return None
    import numpy as np

    a = np.asarray(its)
    return {"mean": round(float(a.mean()), 2), "p50": float(np.median(a)), "min": int(a.min()), "max": int(a.max()),
            "stages": int(a.size)}


def state_errors(hist, ref, free):
    """Error of every step-end state against the FP64 path's state at the same
    step, over the free nodes: the trajectory norm max_n |x_n - x_n^ref| /
    max_n |x_n^ref|, and the largest per-step ratio |x_n - x_n^ref| / |x_n^ref|."""
    import torch

    d = torch.linalg.vector_norm((hist - ref)[:, free], dim=1)
    r = torch.linalg.vector_norm(ref[:, free], dim=1)
    return {"traj_rel_err": float(f"{float(d.max() / r.max()):.3e}"),
            "max_step_rel_err": float(f"{float((d / r.clamp_min(1e-300)).max()):.3e}"),
            "steps_compared": int(hist.shape[0])}


def run_adaptive(case, precision, t_end, tol):
    """Error-controlled RKC over [0, t_end] (local error `tol` relative to the
    drive amplitude and relative to the potential, as Sec. V runs it), on a
    torch workspace; the fixed-step workload needs t_end / tau steps of s
    stages for the same interval."""
    import torch

    from paper_1612_09447_amd import Context

    dev = torch.device("cuda:0")
    ctx = Context(0, torch.cuda.current_stream(dev))
    ctx.setup_case(case, precision=precision)
    ws = ctx.use_torch_workspace()
    x = torch.zeros(case.n_nodes, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, steps = ctx.rkc_adaptive(0.0, t_end, x, case.rtol, tol * float(max(case.amp)), tol, case.tau, s_max=256)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    ctx.close()
    del ws
    fixed_stages = round(t_end / case.tau) * case.s
    acc = [d for d in steps if d["accepted"]]
    log(f"[bench] adaptive: {st['accepted']} accepted, {st['rejected']} rejected, {st['stages']} solves in {el:.2f}s")
    return {"t_end_s": t_end, "local_error_tol": tol, "accepted_steps": st["accepted"], "rejected_steps": st["rejected"],
            "max_stages": st["max_s"], "solves": st["stages"], "cg_iters": st["cg_iters"],
            "mean_cg_iters_per_solve": round(st["cg_iters"] / max(1, st["stages"]), 2), "wall_s": round(el, 3),
            "solves_per_s": round(st["stages"] / el, 1),
            "step_sizes_s": {"min": min(d["tau"] for d in acc), "max": max(d["tau"] for d in acc)},
            "fixed_step_solves_same_interval": fixed_stages,
            "solve_ratio_fixed_over_adaptive": round(fixed_stages / max(1, st["stages"]), 2)}


def run_p2(n, steps, warmup, prof_steps=1):
    """The second-order workload: 10-node tets on the n^3 Kuhn mesh (n = 64:
    2.1M free DOF), the c2 inclusion layout, RKC(16), FP32 AMG under FP64 CG,
    rel-res 1e-8; stages/s and the element pass against its bytes."""
    import eqsgen
    from paper_1612_09447_amd import EQS_PREC_FP32

    case = eqsgen.case_p2(n)
    r = run_gpu(case, EQS_PREC_FP32, steps, warmup, case.rtol, prof_steps=prof_steps)
    info = r["info"]
    out = {"workload": f"second-order (10-node) tets on {n}^3 cubes: {case.n_tets} tets, {info['n_free']} free DOF, "
                       f"nnz(M) {info['nnz_M']}, RKC s={case.s}, CG rel-res {case.rtol:g}, FP32 AMG",
           "steps": steps, "stages_per_s": round(r["stages"] / r["elapsed"], 2),
           "mean_cg_iters_per_stage": round(sum(r["iters"]) / len(r["iters"]), 2), "amg_levels": info["level_rows"]}
    if r["prof"]:
        el = r["prof"]["element"]
        # per tet its ten node ids (40 B) and material (4 B); per node 24 B
        # coordinates, 8 B potential, 8 B result
        nbytes = info["n_tets"] * 44 + info["n_nodes"] * 40
        a = nbytes / (el["avg_ms"] * 1e-3) / 1e9
        out["element_pass"] = {"avg_launch_us": round(el["avg_ms"] * 1e3, 2), "bytes_per_launch": nbytes,
                               "achieved_GBs": round(a, 1), "frac": round(a / HBM_PEAK_GBS, 4)}
        sp = r["prof"]["spmv_M"]
        sbytes = spmv_bytes(info, info["nnz_M"])
        out["spmv_M"] = {"avg_launch_us": round(sp["avg_ms"] * 1e3, 2), "bytes_per_launch": sbytes,
                         "frac": round(sbytes / (sp["avg_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def run_batched(steps, warmup, graph_iters=(1, 64)):
    """The batched workload: 64 independent instances (n in {16..48}^3) packed
    into one context, RKC(8) steps of all of them together, timed once per
    launch granularity in `graph_iters` (CG iterations per captured graph: 1,
    and one that spans a whole stage solve), each from rest over the same
    steps."""
    import torch

    import eqsgen
    from paper_1612_09447_amd import EQS_PREC_FP32, Batch, Context

    t0 = time.perf_counter()
    cases = eqsgen.case_batch()
    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    inputs = []
    for c in cases:
        ctx = Context(0, stream)
        ctx.set_inputs(c)
        inputs.append(ctx)
    b = Batch(inputs, precision=EQS_PREC_FP32, stream=stream)
    for ctx in inputs:
        ctx.close()
    setup_s = time.perf_counter() - t0
    dof = sum((c.n + 1) ** 2 * (c.n - 1) for c in cases)
    log(f"[bench] batched: {len(cases)} instances, {dof} free DOF, {sum(c.n_tets for c in cases)} tets, "
        f"setup {setup_s:.1f}s")
    tau, s, rtol = cases[0].tau, cases[0].s, cases[0].rtol
    runs, finals = {}, {}
    for g in graph_iters:
        b.set_graph_iters(g)
        xs = [torch.zeros(c.n_nodes, dtype=torch.float64, device="cuda:0") for c in cases]
        if warmup:
            b.rkc_steps(warmup, 0.0, tau, s, xs, rtol)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = b.rkc_steps(steps, warmup * tau, tau, s, xs, rtol)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        stages = steps * s * len(cases)
        runs[g] = {"stages_per_s_aggregate": round(stages / el, 1), "dof_stages_per_s": round(dof * steps * s / el, 1),
                   "cg_iters_per_instance_stage": {"min": round(float(res["iters"].min()) / (steps * s), 2),
                                                   "max": round(float(res["iters"].max()) / (steps * s), 2)}}
        finals[g] = torch.cat(xs)
        log(f"[bench] batched, {g} CG iterations per graph: {runs[g]['stages_per_s_aggregate']} instance-stages/s")
    b.close()
    g0 = graph_iters[0]
    best = max(runs, key=lambda g: runs[g]["stages_per_s_aggregate"])
    out = {"instances": len(cases), "free_dof": dof, "steps": steps, "s": s, **runs[best],
           "graph_iters": best, "by_graph_iters": {str(g): r for g, r in runs.items()},
           "precision": "FP64 CG + K(x)x, FP32 AMG", "setup_s": round(setup_s, 1)}
    if len(runs) > 1:
        # the launch granularity changes no arithmetic: the final states agree up to the solve tolerance
        ref = finals[g0]
        out["max_rel_state_diff_across_graph_forms"] = float(f"{max(float(torch.linalg.vector_norm(v - ref) / torch.linalg.vector_norm(ref)) for v in finals.values()):.3e}")
    return out


def cpu_baseline(case, x_user, step):
    """The oracle, as it stands, on one stage of the workload (single thread):
    F(t_n, Y_n) at the state the GPU run reached after `step` steps."""
    from oracle.eqs import EqsOracle

    t0 = time.perf_counter()
    orc = EqsOracle(case, solve_rtol=case.rtol)
    log(f"[bench] oracle setup {time.perf_counter() - t0:.1f}s")
    t = step * case.tau
    t1 = time.perf_counter()
    orc.F(t, x_user[orc.free])  # one stage: K(x)x over all tets + one SGS-PCG solve of M
    dt = time.perf_counter() - t1
    log(f"[bench] oracle stage {dt:.1f}s ({orc.last_iters} SGS-PCG iterations)")
    return dict(value=1.0 / dt, unit="stages/s", cores=1, kind="oracle",
                sample=f"stage 0 of step {step} (t={t:g} s, from the state the GPU run reached there): one "
                       f"element pass over {case.n_tets} tets + one SGS-PCG solve of M to rel-res {case.rtol:g} "
                       f"from a zero start ({orc.last_iters} iterations), {dt:.1f} s on 1 of {os.cpu_count()} "
                       f"cores ({cpu_model()})")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed RKC steps (the workload's 200)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c0", "c1", "c2"])
    ap.add_argument("--config", default="",
                    help="workload configuration (a name under eqsgen/configs or a JSON path): its recipe, "
                         "settings and start vector replace --workload and --guess")
    ap.add_argument("--n", type=int, default=None, help="override the mesh resolution (testing)")
    ap.add_argument("--plain-steps", type=int, default=-1,
                    help="timed steps of the plain FP64 path over the same steps (-1: as --steps, 0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prof-steps", type=int, default=3, help="instrumented steps after the timed ones")
    ap.add_argument("--guess", default="previous", choices=["previous", "zero", "galerkin", "mor", "mlp"])
    ap.add_argument("--mlp-seed", type=int, default=4, help="seed of the start-vector network's initial weights")
    ap.add_argument("--graphs", type=int, default=1, help="replay CG iterations as a captured HIP graph")
    ap.add_argument("--flexible", type=int, default=0, help="CG beta: 0 default, 1 Polak-Ribiere, 2 Fletcher-Reeves")
    ap.add_argument("--graph-iters", type=int, default=1, help="CG iterations per captured graph launch")
    ap.add_argument("--metrics-jsonl", default="",
                    help="append one JSON line per timed step of the main run to this file")
    ap.add_argument("--c3-steps", type=int, default=5, help="also time the 64-instance batched workload (0: skip)")
    ap.add_argument("--c3-graph-iters", default="1,64",
                    help="CG iterations per graph launch for the batched workload, one timed run each (comma list)")
    ap.add_argument("--mlp-batch", type=int, default=256, help="network training pairs per stage (<= 256)")
    ap.add_argument("--mlp-warmup", type=int, default=64,
                    help="training pairs collected before the network's start vector is used")
    ap.add_argument("--p2-steps", type=int, default=5, help="also time the second-order workload (0: skip)")
    ap.add_argument("--p2-n", type=int, default=64, help="cubes per edge of the second-order workload")
    ap.add_argument("--adaptive-ms", type=float, default=20.0,
                    help="also run error-controlled RKC (local error 1e-2) over this many ms (0: skip)")
    ap.add_argument("--full-runs", default="mlp,galerkin",
                    help="start vectors timed over the whole run beside the plain one (comma list; empty: none)")
    ap.add_argument("--learned-steps", type=int, default=5,
                    help="also time this many steps with each start vector (zero, Galerkin, fixed POD, network; "
                         "0: skip)")
    args = ap.parse_args()

    os.environ["EQS_USE_GRAPHS"] = "1" if args.graphs else "0"
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1 "
                                   "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)

    import eqsgen

    t0 = time.perf_counter()
    if args.config:
        cfg = eqsgen.load_config(args.config)
        if cfg["recipe"] not in ("c0", "c1", "c2"):
            print(json.dumps({"error": f"--config {args.config}: the timed run takes a single-context recipe "
                                       "(c0, c1, c2); the batched and second-order workloads are legs of their own"}))
            sys.exit(2)
        case = eqsgen.cases_from_config(cfg, n=args.n)[0]
        args.workload, args.guess = cfg["name"], cfg["guess"]
        args.mlp_seed = cfg.get("mlp_init_seed", 4)
    else:
        case = eqsgen.make_case(args.workload, n=args.n)
    log(f"[bench] workload {args.workload}: n={case.n} nodes={case.n_nodes} tets={case.n_tets} "
        f"({time.perf_counter() - t0:.1f}s to generate)")
    prec = "fp32" if case.precision == "fp32" else "fp64"
    from paper_1612_09447_amd import EQS_PREC_FP32, EQS_PREC_FP64

    main_prec = EQS_PREC_FP32 if prec == "fp32" else EQS_PREC_FP64
    copy = copy_probe()
    rd = read_probe()
    log(f"[bench] copy probe: {copy}; read probe: {rd}")
    steplog = None
    if args.metrics_jsonl:
        from paper_1612_09447_amd.steplog import StepLog

        steplog = StepLog(args.metrics_jsonl, run=f"{args.workload} main", precision=prec, guess=args.guess)
    r = run_gpu(case, main_prec, args.steps, args.warmup, case.rtol, prof_steps=args.prof_steps, guess=args.guess,
                flexible=args.flexible, learned_steps=args.learned_steps, mlp_batch=args.mlp_batch,
                keep_states=True, mlp_warmup=args.mlp_warmup, graph_iters=args.graph_iters, steplog=steplog,
                mlp_seed=args.mlp_seed)
    if steplog is not None:
        steplog.close()
    stages_per_s = r["stages"] / r["elapsed"]
    info = r["info"]
    prof = r["prof"]

    # roofline of the dominant single kernel: the class with the largest summed
    # time in the instrumented window
    per_class_bytes = class_bytes(info, case.s)
    roofline, breakdown = None, None
    if prof:
        rooflines = {}
        for k, nbytes in per_class_bytes.items():
            if not prof[k]["launches"]:
                continue
            a = nbytes / (prof[k]["avg_ms"] * 1e-3) / 1e9
            rooflines[k] = {"kernel": KERNEL_NAMES[k], "achieved": round(a, 1), "frac": round(a / HBM_PEAK_GBS, 4),
                            "avg_launch_us": round(prof[k]["avg_ms"] * 1e3, 2), "bytes_per_launch": nbytes,
                            "launches": prof[k]["launches"], "total_ms": round(prof[k]["total_ms"], 3),
                            "traffic": measured_traffic(k)}
        dominant = max(rooflines, key=lambda k: prof[k]["total_ms"])
        d = rooflines[dominant]
        roofline = {"bound": "hbm", "kernel": d["kernel"], "class": dominant,
                    "achieved": d["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": d["frac"], "traffic": d["traffic"],
                    "frac_of_copy": round(d["achieved"] / copy["GB/s"], 4),
                    "frac_of_read": round(d["achieved"] / rd["GB/s"], 4),
                    "bytes_per_launch": d["bytes_per_launch"], "avg_launch_us": d["avg_launch_us"],
                    "timing": f"start/stop events of every launch (hipExtLaunchKernelGGL) on the context stream, "
                              f"{args.prof_steps} instrumented steps following the timed ones",
                    "per_kernel": rooflines}
        breakdown = {k: {"launches": v["launches"], "avg_us": round(v["avg_ms"] * 1e3, 2),
                         "share_of_instrumented": round(v["total_ms"] * 1e-3 / r["prof_elapsed"], 4)}
                     for k, v in prof.items()}

    import torch

    free = torch.ones(case.n_nodes, dtype=torch.bool, device="cuda:0")
    free[torch.as_tensor(case.dir_nodes, dtype=torch.int64, device="cuda:0")] = False
    plain = None
    plain_steps = args.steps if args.plain_steps < 0 else args.plain_steps
    ref_hist = None
    if plain_steps > 0 and main_prec != EQS_PREC_FP64:
        p = run_gpu(case, EQS_PREC_FP64, plain_steps, args.warmup, case.rtol, keep_states=plain_steps == args.steps,
                    graph_iters=args.graph_iters)
        plain = {"stages_per_s": round(p["stages"] / p["elapsed"], 2),
                 "mean_cg_iters_per_stage": round(sum(p["iters"]) / len(p["iters"]), 2),
                 "steps": plain_steps}
        if plain_steps == args.steps:
            ref_hist = p["hist"]
            plain["fp32_form_speedup"] = round(stages_per_s / plain["stages_per_s"], 3)
            plain["fp32_form_error_vs_fp64"] = state_errors(r["hist"], ref_hist, free)
    r["hist"] = None

    # whole runs with the estimator start vectors, same steps as the main run
    full = {}
    for kind in [k for k in args.full_runs.split(",") if k]:
        f = run_gpu(case, main_prec, args.steps, args.warmup, case.rtol, guess=kind, mlp_batch=args.mlp_batch,
                    keep_states=ref_hist is not None, mlp_warmup=args.mlp_warmup, graph_iters=args.graph_iters)
        full[kind] = {"stages_per_s": round(f["stages"] / f["elapsed"], 2),
                      "mean_cg_iters_per_stage": round(sum(f["iters"]) / len(f["iters"]), 2),
                      "steps": args.steps, "guess_used": f["used"], "guard_fallbacks": f["fallbacks"],
                      "vs_plain_start": round(f["stages"] / f["elapsed"] / stages_per_s, 3)}
        if ref_hist is not None:
            full[kind]["error_vs_fp64"] = state_errors(f["hist"], ref_hist, free)
        f["hist"] = None
    ref_hist = None
    torch.cuda.empty_cache()

    c3_g = tuple(int(g) for g in args.c3_graph_iters.split(",") if g)
    batched = run_batched(args.c3_steps, 1, c3_g) if args.c3_steps > 0 else None
    adaptive = run_adaptive(case, main_prec, args.adaptive_ms * 1e-3, 1e-2) if args.adaptive_ms > 0 else None
    p2 = run_p2(args.p2_n, args.p2_steps, 1) if args.p2_steps > 0 else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(case, r["x"], args.warmup + args.steps)
        cpu["value"] = round(cpu["value"], 6)

    out = {
        "metric": METRIC,
        "value": round(stages_per_s, 2),
        "unit": "stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["elapsed"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if main_prec == EQS_PREC_FP32 else "f64",  # FP64 CG and element pass, FP32 V-cycle
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: unit cube, {case.n}^3 sub-cubes x 6 P1 tets ({case.n_tets} tets, "
                        f"{info['n_free']} free DOF), seeded varistor inclusions, RKC s={case.s}, "
                        f"tau={case.tau:g}, CG rel-res {case.rtol:g}",
            "precision": "FP64 CG + K(x)x, FP32 AMG V-cycle" if main_prec == EQS_PREC_FP32 else "FP64",
            "start_vector": args.guess,
            "guess_used": r["used"],
            "guess_fallbacks": r["fallbacks"],
            "graphs": bool(args.graphs),
            "cg_iters_per_graph_launch": args.graph_iters,
            "mean_cg_iters_per_stage": round(sum(r["iters"]) / len(r["iters"]), 2),
            "cg_iters_per_stage": stage_iter_stats(r["stage_iters"]),
            "amg_levels": info["level_rows"],
            "device_memory": f"torch workspace of {info['workspace_bytes']} bytes (eqs_set_workspace); "
                             f"library-allocated: {info['device_bytes']}",
            "nnz_M": info["nnz_M"],
            "setup_s": round(r["setup_s"], 1),
        },
        "roofline": roofline,
        "kernel_breakdown": breakdown,
        "copy_probe": copy,
        "read_probe": rd,
        "fp64_plain": plain,
        "start_vectors": r["learned"] or None,
        "start_vector_runs": full or None,
        "mixed_learned_vs_fp64": mixed_learned_vs_fp64(plain, r["learned"], full),
        "batched": batched,
        "adaptive": adaptive,
        "second_order": p2,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
