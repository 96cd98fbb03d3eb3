#!/usr/bin/env python3
"""Benchmark: state solves/s to a relative residual of 1e-8 on one MI355X.

Workload (the 512 x 256 Q1 plane-stress cantilever, 263,682 DOFs): seeded
two-scale random-field densities with 40 bars, left edge clamped, unit
point load at the right-mid node, 16 x 8 subdomains of 32 x 32 elements
with overlap 2, the same densities at Emin = 1e-3, 1e-6 and 1e-9.

One step = for each of the three contrasts: SIMP moduli from the densities,
the whole preconditioner setup (local factors, heat eigenproblems with the
threshold, coarse basis and K_0^+), and one PCG solve to relres 1e-8
(true residual verified).  The FP32-local ("mixed") path is the headline
value; the FP64 path is timed the same way beside it.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CONTRASTS = (1e-3, 1e-6, 1e-9)
SAMPLE_ITERS = 40       # oracle PCG iterations timed by the CPU baseline
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="run the CPU oracle's PCG to convergence instead of "
                         "timing its first iterations")
    ap.add_argument("--quick", action="store_true",
                    help="one contrast, no FP64 leg (for profiler runs)")
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the 3D one-level solve line")
    ap.add_argument("--no-matvec-probe", action="store_true",
                    help="skip the HBM-sized stiffness-product probe")
    ap.add_argument("--workload", choices=("cantilever", "batch", "serving", "topopt"),
                    default="cantilever",
                    help="cantilever: the 512x256 benchmark (default line); "
                         "batch: 64 uneven cantilevers solved in lockstep; "
                         "serving: Poisson stream of state+adjoint requests; "
                         "topopt: design loop (solve, gradient, OC step)")
    ap.add_argument("--topopt-steps", type=int, default=12)
    ap.add_argument("--topopt-emin", type=float, default=1e-6)
    ap.add_argument("--reuse-age", type=int, default=1,
                    help="design steps a setup may be reused (topopt)")
    ap.add_argument("--serve-reuse-age", type=int, default=0,
                    help="requests a run's setup may be reused (serving)")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--serve-runs", type=int, default=32)
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-rate", type=float, default=200.0,
                    help="mean arrival rate (requests/s)")
    ap.add_argument("--kernel-probe", action="store_true",
                    help="only launch the profiled kernels: first-level "
                         "applies (Emin 1e-6, FP32 path), stiffness products "
                         "on the probe mesh and a plain 1 GiB device copy "
                         "(the byte-counter calibration); prints their sizes")
    return ap.parse_args()


# Stiffness-product probe: a mesh well beyond the 256 MB last-level cache,
# so the matvec streams from HBM.
PROBE_NEL = (8192, 4096)


def matvec_bytes(nel):
    """Algorithmic HBM bytes of one stiffness product y = K x (2D Q1): x
    read and y written (FP64, two DOFs a node), the element moduli read
    (FP64) and the clamped-DOF mask read (one byte a DOF)."""
    nn = (nel[0] + 1) * (nel[1] + 1)
    n = 2 * nn
    return 8 * 2 * n + 8 * nel[0] * nel[1] + n


def matvec_probe(torch, launches=20):
    """Average event-timed duration of the stiffness product on PROBE_NEL."""
    import numpy as np
    import inputs
    import paper_2006_13387_amd as msp
    desc = inputs.problem_desc(2, PROBE_NEL, sub_nel=32, overlap=2)
    fixed = inputs.clamp_face_mask(desc, axis=0, side=0)
    rng = np.random.default_rng(7)
    s = msp.Solver(desc, fixed)
    s.set_densities(torch.tensor(rng.random(PROBE_NEL[0] * PROBE_NEL[1]),
                                 device="cuda"))
    x = torch.randn(s.n, device="cuda", dtype=torch.float64)
    for _ in range(3):
        s.apply_K(x)
    s.kernel_timing(enable=2)              # bit 1: stiffness product
    for _ in range(launches):
        s.apply_K(x)
    c, t = s.kernel_timing(enable=0)["cg_matvec"]
    s.close()
    ms = t / max(c, 1)
    b = matvec_bytes(PROBE_NEL)
    gbs = b / (ms * 1e-3) / 1e9
    return {"mesh": f"{PROBE_NEL[0]}x{PROBE_NEL[1]} Q1 ({s.n} DOFs)",
            "bytes_per_launch": int(b), "avg_launch_ms": round(ms, 5),
            "achieved_GBs": round(gbs, 1),
            "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4), "launches": int(c),
            "copy_reference": copy_reference(torch, b)}


def copy_reference(torch, nbytes, launches=10):
    """A plain device copy moving the same number of bytes (half read, half
    written; torch's copy kernel), event-timed: the attainable HBM rate for
    a streaming kernel on this device, for comparison."""
    n = int(nbytes) // 16
    a = torch.ones(n, device="cuda", dtype=torch.float64)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(launches):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / launches
    gbs = 16 * n / (ms * 1e-3) / 1e9
    del a, b
    return {"bytes": 16 * n, "avg_ms": round(ms, 5), "achieved_GBs": round(gbs, 1),
            "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


PROBE3_NEL = (384, 192, 192)
FP64_PEAK_TFLOPS = 78.6


def matvec3d_probe(torch, launches=10):
    """Event-timed 3D (H8) stiffness product on PROBE3_NEL (43M DOFs), against
    the FP64 ALU roof (the dense element product, 2 * 24 * 24 flops per
    element) and the HBM roof (x read, y written, E, one clamp byte per
    node)."""
    import numpy as np
    import inputs
    import paper_2006_13387_amd as msp
    desc = inputs.problem_desc(3, PROBE3_NEL, sub_nel=6, overlap=1)
    fixed = inputs.clamp_face_mask(desc, axis=0, side=0)
    rng = np.random.default_rng(8)
    nel = int(np.prod(PROBE3_NEL))
    s = msp.Solver(desc, fixed)
    s.set_densities(torch.tensor(rng.random(nel), device="cuda"))
    x = torch.randn(s.n, device="cuda", dtype=torch.float64)
    for _ in range(2):
        s.apply_K(x)
    s.kernel_timing(enable=2)
    for _ in range(launches):
        s.apply_K(x)
    c, t = s.kernel_timing(enable=0)["cg_matvec"]
    s.close()
    ms = t / max(c, 1)
    nn = int(np.prod([v + 1 for v in PROBE3_NEL]))
    flops = 2 * 24 * 24 * nel
    b = 8 * 3 * nn * 2 + 8 * nel + nn
    return {"mesh": f"{PROBE3_NEL[0]}x{PROBE3_NEL[1]}x{PROBE3_NEL[2]} H8 ({3 * nn} DOFs)",
            "avg_launch_ms": round(ms, 5), "launches": int(c),
            "flops_per_launch": flops, "achieved_TFLOPs": round(flops / (ms * 1e-3) / 1e12, 2),
            "frac_fp64_peak": round(flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
            "bytes_per_launch": b, "achieved_GBs": round(b / (ms * 1e-3) / 1e9, 1),
            "frac_hbm_peak": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


COUNTERS = os.path.join(ROOT, "profiles", "level1_apply_hbm_counters.json")
LEVEL1_SOURCES = ("paper_2006_13387_amd/csrc/k_local.hip",
                  "paper_2006_13387_amd/csrc/dev.h",
                  "paper_2006_13387_amd/csrc/common.h")


def level1_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in LEVEL1_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def level1_traffic(launches_by_contrast):
    """HBM bytes per first-level launch from the committed FETCH_SIZE /
    WRITE_SIZE counters, weighted like the timed launches; None when the
    kernel's sources changed since the counters were taken."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("source_sha256") != level1_source_hash():
        return None
    per = c["traffic_bytes_per_launch"]
    tot = sum(n for n in launches_by_contrast.values())
    if tot == 0 or any(k not in per for k in launches_by_contrast):
        return None
    return sum(n * per[k] for k, n in launches_by_contrast.items()) / tot


def solve3d_workload(torch):
    """The 96 x 48 x 48 H8 cantilever solved with the two-level M_EH+Rot
    preconditioner (3D heat coarse space, three rotations per coarse node,
    kmax 16): a warm-up solve, then two timed solves on the FP32-local path
    and one on the FP64 path, each the full setup (first-level inverses,
    heat eigenproblems, coarse basis, K_0 and its generalised inverse) and
    the PCG to relres 1e-8; the first-level application and the coarse
    restriction with the slab solve of K_0 are event-timed."""
    import inputs
    import numpy as np
    import paper_2006_13387_amd as msp
    p = inputs.config(2)
    rho = torch.tensor(p.rho, device="cuda")
    f = torch.tensor(p.f, device="cuda")
    out = {}
    for prec, reps in ((1, 2), (0, 1)):
        s = msp.Solver(dict(p.desc, precision=prec), p.fixed)
        s.set_densities(rho)
        s.solve(f, rtol=1e-8, maxit=20)          # warm-up: buffers, kernels
        secs, infos = [], []
        for _ in range(reps):
            s.set_densities(rho)
            s.kernel_timing(enable=(1 | 16))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = s.solve(f, rtol=1e-8, maxit=5000)
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t0)
            infos.append(info)
            if info["relres_true"] > 1e-8:
                raise RuntimeError(f"3D solve missed relres 1e-8: {info}")
        kt = s.kernel_timing(enable=0)
        q = s.query()
        s.close()
        sec = float(np.mean(secs))
        info = infos[-1]
        rec = {"solves_per_s": round(1.0 / sec, 4), "seconds": round(sec, 4),
               "setup_ms": round(info["t_setup_ms"], 1),
               "solve_ms": round(info["t_solve_ms"], 1),
               "iterations": info["iters"], "n_coarse": info["n_coarse"],
               "coarse_rank": info["coarse_rank"], "relres_true": info["relres_true"],
               "cond_est": round(info["cond_est"], 2)}
        if prec == 1:
            c, t = kt["level1_apply"]
            l1_b = q["level1_record_bytes"] + q["local_vec_entries"] * 16
            l1_ms = t / max(c, 1)
            gbs = l1_b / (l1_ms * 1e-3) / 1e9
            cr, tr = kt["coarse_restrict"]
            rec["level1_roofline"] = {"kernel": "k3s_apply (FP32 plane factors) + k3_level1_sum",
                                      "bound": "hbm", "bytes_per_launch": int(l1_b),
                                      "avg_launch_ms": round(l1_ms, 5),
                                      "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                                      "launches": int(c)}
            # restriction + the slab solve with K_0's block LDL^T factors
            rec["coarse_apply"] = {"kernels": "k3c_restrict + k3c_slab_step (forward and "
                                              "backward over the slabs of coarse nodes)",
                                   "avg_launch_ms": round(tr / max(cr, 1), 5)}
            out["fp32_local"] = rec
        else:
            out["fp64"] = rec
    return {"workload": f"cantilever3d_96x48x48 H8 ({len(p.fixed)} DOFs), 1024 "
                        "subdomains S=6 overlap 1, M_EH+Rot (3D heat coarse space, kmax 16, "
                        "3 rotations per coarse node), Emin 1e-6",
            **out}


# Table 2 of the paper (contrast 1): iterations, condition and coarse
# dimension as printed there, beside each method's run here (the paper's
# Poisson ratio, forces and random draws are not known exactly)
TABLE2_PAPER = {
    "M_EE": (14, 4.6, 243), "M_EE twice": (15, 5.0, 486),
    "M_EH": (15, 5.2, 243), "M_EH+Rot": (14, 4.6, 243),
    "M_EH+Rot;Rand 10": (24, 13.8, 243), "M_EH+Rot;Rand 15": (25, 15.6, 243),
    "M_EE;Rand 10": (20, 9.4, 243), "M_EE;Rand 15": (20, 9.4, 243)}


def table2_workload(torch):
    """The methods of the paper's Table 2 on its 100 x 100 example at
    contrast 1 (FP64 path, PCG to 1e-6): per method the iterations, the
    condition estimate, N_c and the setup and solve times of a warm run."""
    import inputs
    import paper_2006_13387_amd as msp
    p = inputs.config_p()
    variants = {
        "M_EE": dict(coarse_kind=1), "M_EE twice": dict(coarse_kind=2),
        "M_EH": dict(rot_enrich=0), "M_EH+Rot": {},
        "M_EH+Rot;Rand 10": dict(eig_random=10, eig_seed=1),
        "M_EH+Rot;Rand 15": dict(eig_random=15, eig_seed=1),
        "M_EE;Rand 10": dict(coarse_kind=1, eig_random=10, eig_seed=1),
        "M_EE;Rand 15": dict(coarse_kind=1, eig_random=15, eig_seed=1)}
    rho = torch.tensor(p.rho, device="cuda")
    f = torch.tensor(p.f, device="cuda")
    out = {}
    for name, extra in variants.items():
        s = msp.Solver(dict(p.desc, **extra), p.fixed)
        s.set_densities(rho)
        s.solve(f, rtol=p.tol)                    # warm-up
        s.set_densities(rho)
        _, info = s.solve(f, rtol=p.tol)
        s.close()
        it, cond, nc = TABLE2_PAPER[name]
        out[name] = {"iterations": info["iters"], "cond_est": round(info["cond_est"], 2),
                     "n_coarse": info["n_coarse"], "setup_ms": round(info["t_setup_ms"], 2),
                     "solve_ms": round(info["t_solve_ms"], 2),
                     "paper": {"iterations": it, "condition": cond, "coarse_dim": nc}}
    return {"workload": "square2d_100x100, 10x10 coarse blocks, vertex neighbourhoods, "
                        "every edge clamped, contrast 1, PCG to 1e-6, FP64 path",
            "methods": out}


def level1_hbm_probe(torch, solvers, rounds=3):
    """First-level applications taken in turn over the batch's problems
    with at least 128 subdomains (whose applications fill the chip), so
    that the records of one application were evicted from the 256 MB
    last-level cache by the others' since it last ran: algorithmic bytes
    over HIP-event time, read from HBM."""
    big = [s for s in solvers if s.query()["n_subdomains"] >= 128]
    if not big:
        return None
    rs = [torch.randn(s.n, device="cuda", dtype=torch.float64) for s in big]
    for s, r in zip(big, rs):
        s.apply_level1(r)
        s.kernel_timing(enable=1)
    for _ in range(rounds):
        for s, r in zip(big, rs):
            s.apply_level1(r)
    torch.cuda.synchronize()
    tot_b = tot_ms = 0.0
    launches = 0
    for s in big:
        c, t = s.kernel_timing(enable=0)["level1_apply"]
        tot_b += c * level1_bytes(s.query())
        tot_ms += t
        launches += c
    gbs = tot_b / (tot_ms * 1e-3) / 1e9
    return {"problems": len(big), "launches": int(launches),
            "records_total_MB": round(sum(s.query()["level1_record_bytes"] for s in big) / 1e6, 1),
            "bytes_per_launch": int(tot_b / max(launches, 1)),
            "avg_launch_ms": round(tot_ms / max(launches, 1), 5),
            "achieved_GBs": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


def batch_workload(torch, args):
    """64 independent 2D cantilevers of uneven size (128x64 .. 768x384,
    config-1 style densities at Emin 1e-6, FP32 local solves): setups, then
    the PCG solves of all of them in lockstep (one launch per iteration
    kernel, graph-captured chunks), against the same solves one at a time."""
    import inputs
    import paper_2006_13387_amd as msp
    t0 = time.perf_counter()
    probs = inputs.batch_configs(count=args.batch_count)
    log(f"[batch] {len(probs)} problems generated in {time.perf_counter() - t0:.1f} s; "
        f"{sum(len(p.f) for p in probs)} DOFs")
    solvers = [msp.Solver(p.desc, p.fixed) for p in probs]
    fs = [torch.tensor(p.f, device="cuda") for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, p in zip(solvers, probs):
        s.set_densities(torch.tensor(p.rho, device="cuda"))
        s.setup()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    b = msp.Batch()
    b.solve(solvers, fs, use_graph=True)           # warm-up: autotuning, graph capture
    if not b.tuning()["tuned"]:
        b.solve(solvers, fs, use_graph=True)
    res = {}
    for name, graph in (("batched_graph", True), ("batched_eager", False)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        us, infos = b.solve(solvers, fs, use_graph=graph)
        torch.cuda.synchronize()
        res[name] = time.perf_counter() - t0
    # the fixed launch shape (16 iterations a chunk, items problem by problem)
    bf = msp.Batch()
    bf.set_autotune(False)
    bf.solve(solvers, fs, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bf.solve(solvers, fs, use_graph=True)
    torch.cuda.synchronize()
    res["batched_graph_untuned_shape"] = time.perf_counter() - t0
    bf.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [s.solve(f)[1] for s, f in zip(solvers, fs)]
    torch.cuda.synchronize()
    res["one_at_a_time"] = time.perf_counter() - t0
    n = len(probs)
    conv = sum(1 for i in infos if i["relres_true"] <= 1e-8)
    out = {
        "metric": "batched state solves/s to relres 1e-8 (solve only, setups before)",
        "value": round(n / res["batched_graph"], 3), "unit": "solves/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "f64 (FP32 local inverses)",
        "data": "synthetic",
        "config": {"workload": f"{n} 2D cantilevers, sizes 128x64..768x384 Q1, "
                               "Emin 1e-6, S=32 overlap 2, FP32 local",
                   "dofs_total": int(sum(len(p.f) for p in probs))},
        "seconds": {k: round(v, 4) for k, v in res.items()},
        "setup_seconds_one_at_a_time": round(t_setup, 4),
        "speedup_batched_over_one_at_a_time": round(res["one_at_a_time"] / res["batched_graph"], 3),
        "iterations_max": max(i["iters"] for i in infos),
        "iterations_mean": round(sum(i["iters"] for i in infos) / n, 1),
        "converged_to_1e-8": conv,
        "relres_true_max": max(i["relres_true"] for i in infos),
        "same_as_one_at_a_time": all(i["iters"] == j["iters"] for i, j in zip(infos, seq)),
        "batch_stats": b.stats(),
        "autotuner": b.tuning(),
        "level1_hbm": level1_hbm_probe(torch, solvers),
    }
    print(json.dumps(out), flush=True)


def serving_workload(torch, args):
    """Poisson stream of state + adjoint requests from concurrent runs, 2D
    (256x128 .. 1024x512 Q1) and, for a quarter of them, 3D (48x24x24 ..
    96x48x48 H8), Emin 1e-6 / 1e-9, FP32 local solves: each request
    perturbs its run's densities (setup rebuilt) and warm-starts from the
    run's previous solutions."""
    import numpy as np
    import inputs
    import paper_2006_13387_amd as msp
    rng = np.random.default_rng(4)
    sizes = ((256, 128), (512, 256), (768, 384), (1024, 512))
    sizes3 = ((48, 24, 24), (72, 36, 36), (96, 48, 48))
    runs = []
    t0 = time.perf_counter()
    for r in range(args.serve_runs):
        emin = (1e-6, 1e-9)[int(rng.integers(2))]
        if r % 4 == 3:
            nel = sizes3[int(rng.integers(len(sizes3)))]
            runs.append(inputs.scaled_cantilever_3d(nel, 4000 + r, Emin=emin, precision=1))
        else:
            nel = sizes[int(rng.integers(len(sizes)))]
            runs.append(inputs.scaled_cantilever_2d(nel, 4000 + r, Emin=emin, precision=1))
    log(f"[serve] {len(runs)} runs generated in {time.perf_counter() - t0:.1f} s")
    # requests: run r's t-th request perturbs its densities
    order = [int(rng.integers(len(runs))) for _ in range(args.serve_requests)]
    count = [0] * len(runs)
    rho_now = [p.rho.copy() for p in runs]
    reqs = []
    for r in order:
        t = count[r]
        count[r] += 1
        p = runs[r]
        rho_now[r] = inputs.perturb(rho_now[r], p.desc["nel"], inputs.perturb_seed(4000 + r, t))
        fa = inputs.output_dof_load(p.desc, rho_now[r], p.fixed, 5000 + 100 * r + t)
        reqs.append((r, torch.tensor(rho_now[r], device="cuda"),
                     torch.tensor(p.f, device="cuda"), torch.tensor(fa, device="cuda")))
    arrivals = np.cumsum(rng.exponential(1.0 / args.serve_rate, len(reqs)))
    sv = msp.Server(250 << 30, 16)
    if args.serve_reuse_age > 0:
        sv.set_reuse(args.serve_reuse_age, 0)
    rid = [sv.add_run(p.desc, p.fixed) for p in runs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt = 0
    tickets = []
    while True:
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arrivals[nxt] <= now:
            r, rho, fs, fa = reqs[nxt]
            tickets.append(sv.submit(rid[r], rho, fs, fa)[0])
            nxt += 1
        st = sv.stats()
        if nxt == len(reqs) and st["completed"] == len(reqs):
            break
        if st["active"] == 0 and st["queued"] == 0 and nxt < len(reqs):
            time.sleep(max(0.0, arrivals[nxt] - now))
            continue
        sv.step()
    wall = time.perf_counter() - t0
    st = sv.stats()
    infos = [sv.result(t) for t in tickets]
    conv = sum(1 for a, b, _ in infos if a["relres_true"] <= 1e-8 and b["relres_true"] <= 1e-8)
    out = {
        "metric": "served state+adjoint solves/s and p50/p99 request latency",
        "value": round(st["solves_per_s"], 3), "unit": "solves/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "f64 (FP32 local inverses)",
        "data": "synthetic",
        "config": {"workload": f"{len(runs)} runs ({sum(p.desc['dim'] == 3 for p in runs)} "
                               "of them 3D 48x24x24..96x48x48 H8, the rest 2D "
                               "256x128..1024x512 Q1; Emin 1e-6/1e-9), "
                               f"{len(reqs)} requests, Poisson {args.serve_rate:g}/s, "
                               "perturbed densities (amplitude 0.05), warm starts",
                   "max_active": 16, "hbm_budget_gib": 250},
        "latency_ms": {"p50": round(st["p50_ms"], 2), "p99": round(st["p99_ms"], 2)},
        "wall_seconds": round(wall, 3),
        "requests_converged_to_1e-8": conv,
        "chunks": int(st["chunks"]),
        "reuse_age": args.serve_reuse_age,
        "setups_built": int(st["setups_built"]),
        "setups_reused": int(st["setups_reused"]),
    }
    print(json.dumps(out), flush=True)


def topopt_workload(torch, args):
    """A minimal minimum-compliance design loop on the 512 x 256 cantilever
    (Section 1): per design step one state solve (warm start from the last
    step), the density gradient and an optimality-criteria update (volume
    fraction 0.4, move 0.2), all on the device.  Run twice: rebuilding the
    preconditioner at every step, and reusing a setup for up to
    --reuse-age steps while a reused solve stays within the iterations of
    the solve right after a rebuild plus the iterations one setup costs
    (Section 1's update strategy; past that limit the solve rebuilds and
    continues)."""
    import inputs
    import paper_2006_13387_amd as msp
    p = inputs.config(1, Emin=args.topopt_emin, precision=1)
    f = torch.tensor(p.f, device="cuda")
    rho0 = torch.tensor(p.rho, device="cuda")
    res = {}
    for label, age in (("rebuild_every_step", 0), ("lazy_reuse", args.reuse_age)):
        s = msp.Solver(p.desc, p.fixed)
        rho = rho0.clone()
        u = torch.zeros_like(f)
        # warm-up step (library and kernels loaded), not timed
        s.set_densities(rho)
        s.solve(f, rtol=1e-8)
        s.close()
        s = msp.Solver(p.desc, p.fixed)
        iters, comps, reused, lim = [], [], 0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(args.topopt_steps):
            s.set_densities(rho)
            u, info = s.solve(f, u=u, warm=t > 0, rtol=1e-8)
            if (age > 0 and not info["setup_reused"] and info["t_setup_ms"] > 0
                    and (lim == 0 or info["iters"] <= lim)):
                # a solve on its own fresh setup (not one stopped at the limit)
                per_it = info["t_solve_ms"] / max(info["iters"], 1)
                lim = info["iters"] + int(info["t_setup_ms"] / per_it) + 1
                s.set_reuse(age, lim)
            iters.append(info["iters"])
            comps.append(info["compliance"])
            reused += int(info["setup_reused"])
            dg = s.sensitivity(rho, u)
            rho, _ = s.oc_update(rho, dg, 0.4, 0.2)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.close()
        res[label] = {"seconds": round(wall, 4),
                      "design_steps_per_s": round(args.topopt_steps / wall, 3),
                      "setups_reused": reused,
                      "setups_built": args.topopt_steps - reused,
                      "iterations": iters,
                      "compliance_first_last": [round(comps[0], 6), round(comps[-1], 6)]}
        log(f"[topopt] {label}: {wall:.3f} s, reused {reused}")
    out = {
        "metric": "design steps/s (state solve to relres 1e-8 + gradient + OC update)",
        "value": res["lazy_reuse"]["design_steps_per_s"], "unit": "steps/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "f64 (FP32 local inverses)",
        "data": "synthetic",
        "config": {"workload": f"cantilever2d_512x256_q1, Emin {args.topopt_emin:g}, "
                               f"{args.topopt_steps} design steps from the random-field "
                               "design, volume fraction 0.4, move 0.2, no filter",
                   "reuse_age": args.reuse_age},
        "runs": res,
        "speedup_lazy_reuse": round(res["rebuild_every_step"]["seconds"] /
                                    res["lazy_reuse"]["seconds"], 3),
    }
    print(json.dumps(out), flush=True)


def kernel_probe(torch):
    """Launch only the kernels whose HBM counters are collected: 10
    first-level applications per contrast on the 512 x 256 cantilever, 13
    stiffness products on the 8192 x 4096 probe, 5 first-level
    applications on the 96 x 48 x 48 workload, 5 plain 1 GiB copies."""
    import inputs
    import paper_2006_13387_amd as msp
    l1 = {}
    for e in CONTRASTS:                     # 10 launches per contrast, in order
        p = inputs.config(1, Emin=e)
        s = msp.Solver(dict(p.desc, precision=1), p.fixed)
        s.set_densities(torch.tensor(p.rho, device="cuda"))
        s.setup()
        r = torch.randn(s.n, device="cuda", dtype=torch.float64)
        for _ in range(10):
            s.apply_level1(r)
        torch.cuda.synchronize()
        l1[f"{e:g}"] = int(level1_bytes(s.query()))
        s.close()
    mv = matvec_probe(torch, launches=10)
    # 3D first level on the 96 x 48 x 48 workload (FP32 plane factors):
    # 5 applications
    p3 = inputs.config(2)
    s3 = msp.Solver(dict(p3.desc, eig_kmax=0, rot_enrich=0), p3.fixed)
    s3.set_densities(torch.tensor(p3.rho, device="cuda"))
    s3.setup()
    r3 = torch.randn(s3.n, device="cuda", dtype=torch.float64)
    for _ in range(5):
        s3.apply_level1(r3)
    torch.cuda.synchronize()
    q3 = s3.query()
    l1_3d = int(q3["level1_record_bytes"] + q3["local_vec_entries"] * 16)
    s3.close()
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, device="cuda", dtype=torch.float64).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"level1_bytes_per_launch": l1,
                      "level1_3d_bytes_per_launch": l1_3d,
                      "matvec_bytes_per_launch": mv["bytes_per_launch"],
                      "copy_bytes_read": nbytes, "copy_bytes_written": nbytes}))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_solvers(probs, precision, **extra):
    import paper_2006_13387_amd as msp
    return [msp.Solver(dict(p.desc, precision=precision, **extra), p.fixed) for p in probs]


def run_steps(torch, solvers, rho, f, nsteps, lat, infos):
    for _ in range(nsteps):
        for s in solvers:
            t0 = time.perf_counter()
            s.set_densities(rho)
            _, info = s.solve(f, rtol=1e-8)     # builds the setup first
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
            infos.append(info)
            if info["relres_true"] > 1e-8:
                raise RuntimeError(f"solve missed relres 1e-8: {info}")
            if info["setup_reused"] or not info["t_setup_ms"] > 0:
                raise RuntimeError("a benchmark step must build its setup")


def timed(torch, solvers, rho, f, steps):
    lat, infos = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(torch, solvers, rho, f, steps, lat, infos)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, lat, infos


def solve_only(torch, solvers, rho, f, reps):
    """Solves/s with the preconditioner already built (setup excluded)."""
    for s in solvers:
        s.set_densities(rho)
        s.setup()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    for _ in range(reps):
        for s in solvers:
            s.solve(f, rtol=1e-8)
            n += 1
    torch.cuda.synchronize()
    return n / (time.perf_counter() - t0)


def level1_bytes(q):
    """Algorithmic HBM bytes of one first-level application (a forward and
    a backward pass of the twisted sweep): the factor records it streams
    (inverse Schur block and couplings of every node row, read once per
    pass, the middle row's once per chain and pass, each subdomain in its
    selected precision), the local right-hand sides gathered (FP64) and the
    local solutions written (FP64)."""
    return q["level1_record_bytes"] + q["local_vec_entries"] * (8 + 8)


def cpu_baseline(full=False):
    """Time the CPU oracle on the benchmark workload at Emin = 1e-6 and
    express it as solves/s (setup + PCG per solve).

    The oracle runs as it stands, through its own whole-solve call: sparse
    assembly, sparse LU of every local system, the heat eigenproblems of
    every coarse neighbourhood with the threshold, its own coarse space and
    K_0 pseudo-inverse, then its PCG.  Default (bounded sample): the whole
    setup, and the first SAMPLE_ITERS PCG iterations, whose average cost is
    multiplied by the oracle's own iteration count to 1e-8 on this input
    (stored by the oracle-only golden script).  full=True runs the PCG to
    convergence instead.
    """
    import platform

    import inputs
    import oracle

    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = 1
    p = inputs.config(1, Emin=1e-6)
    with open(os.path.join(ROOT, "tests", "golden", "cantilever512_emin.json")) as fh:
        ref = json.load(fh)["contrasts"]["1e-06"]
    it_ref = int(ref["pcg"]["iters"])
    maxit = 5000 if full else SAMPLE_ITERS
    t0 = time.perf_counter()
    _, info, _ = oracle.solve(p.desc, p.rho, p.fixed, p.f, tol=1e-8, maxit=maxit)
    wall = time.perf_counter() - t0
    if full:
        iters = info.iters
        sec = info.t_setup + info.t_solve
    else:
        iters = it_ref
        sec = info.t_setup + it_ref * info.t_solve / max(info.iters, 1)
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    sample = ("512x256 cantilever at Emin 1e-6, the oracle's whole solve: "
              f"setup {info.t_setup:.1f} s (its N_c {info.n_coarse}), ")
    if full:
        sample += f"PCG to 1e-8 in {info.iters} iterations {info.t_solve:.1f} s"
    else:
        sample += (f"{info.iters} PCG iterations timed ({info.t_solve:.1f} s) and "
                   f"scaled to its {it_ref} iterations to 1e-8")
    sample += f"; {wall:.1f} s of oracle work; host {cpu}, {len(os.sched_getaffinity(0))} cores"
    return {"value": 1.0 / sec, "unit": "solves/s", "cores": int(blas_threads),
            "kind": "oracle", "sample": sample, "sec_per_solve": sec,
            "iters": iters, "n_coarse": int(info.n_coarse)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this solver has no "
              "multi-GPU path (sharding is described in DESIGN.md); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import inputs
    import paper_2006_13387_amd as msp
    msp.load_library()
    if args.kernel_probe:
        kernel_probe(torch)
        return
    if args.workload == "batch":
        batch_workload(torch, args)
        return
    if args.workload == "serving":
        serving_workload(torch, args)
        return
    if args.workload == "topopt":
        topopt_workload(torch, args)
        return
    contrasts = CONTRASTS[1:2] if args.quick else CONTRASTS
    probs = [inputs.config(1, Emin=e) for e in contrasts]
    rho = torch.tensor(probs[0].rho, device="cuda")
    f = torch.tensor(probs[0].f, device="cuda")
    log(f"[bench] workload {probs[0].name} n={len(probs[0].f)} "
        f"contrasts={contrasts}")
    mixed = make_solvers(probs, 1)
    fp64 = [] if args.quick else make_solvers(probs, 0)
    for _ in range(args.warmup):
        run_steps(torch, mixed, rho, f, 1, [], [])
        if fp64:
            run_steps(torch, fp64, rho, f, 1, [], [])
    log("[bench] warmup done")
    # headline: mixed path, level-1 kernel timed with events in the region
    for s in mixed:
        s.kernel_timing(enable=1)          # bit 0: first-level apply
    t_mixed, lat_mixed, inf_mixed = timed(torch, mixed, rho, f, args.steps)
    l1 = [s.kernel_timing(enable=0)["level1_apply"] for s in mixed]
    log(f"[bench] mixed: {t_mixed:.3f} s for {args.steps} steps")
    res = {}
    if fp64:
        t_fp64, lat_fp64, inf_fp64 = timed(torch, fp64, rho, f, args.steps)
        log(f"[bench] fp64: {t_fp64:.3f} s")
    # per-kernel breakdown on one extra pass (not in the timed region)
    for s in mixed:
        s.kernel_timing(enable=True)
    run_steps(torch, mixed, rho, f, 1, [], [])
    kt = {}
    for s in mixed:
        for k, (c, t) in s.kernel_timing(enable=0).items():
            a, b = kt.get(k, (0, 0.0))
            kt[k] = (a + c, b + t)
    so_mixed = solve_only(torch, mixed, rho, f, 1)
    so_fp64 = solve_only(torch, fp64, rho, f, 1) if fp64 else None
    nsolves = args.steps * len(mixed)
    value = nsolves / t_mixed
    q = mixed[0].query()
    launches = sum(c for c, _ in l1)
    l1_ms = sum(t for _, t in l1) / max(launches, 1)
    # each contrast has its own FP32/FP64 selection: weight its bytes by
    # its launches
    l1_tot_bytes = sum(c * level1_bytes(s.query()) for (c, _), s in zip(l1, mixed))
    l1_bytes = l1_tot_bytes / max(launches, 1)
    traffic = level1_traffic({f"{e:g}": c for e, (c, _) in zip(contrasts, l1)})
    if traffic is not None:
        traffic = int(traffic)
    achieved = l1_bytes / (l1_ms * 1e-3) / 1e9
    lat_sorted = sorted(lat_mixed)
    pct = lambda a, x: a[min(len(a) - 1, int(round(x * (len(a) - 1))))]
    out = {
        "metric": "state solves/s to relres 1e-8 (setup + solve per solve; "
                  "FP32-local mixed path)",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_mixed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (FP32 local inverses)",
        "data": "synthetic",
        "config": {"workload": "cantilever2d_512x256_q1 (263682 DOFs), "
                               "16x8 subdomains S=32 overlap 2, M_EH+Rot, "
                               "tau=2, kmax=16, Emin " +
                               "/".join(f"{e:g}" for e in contrasts),
                   "solves_per_step": len(mixed),
                   "rtol": 1e-8},
        "latency_ms": {"p50": round(1e3 * pct(lat_sorted, 0.5), 3),
                       "p99": round(1e3 * pct(lat_sorted, 0.99), 3)},
        "iterations": {f"{e:g}": i["iters"] for e, i in zip(contrasts, inf_mixed)},
        "coarse_dim": {f"{e:g}": i["n_coarse"] for e, i in zip(contrasts, inf_mixed)},
        "setup_ms": {f"{e:g}": round(i["t_setup_ms"], 3) for e, i in zip(contrasts, inf_mixed)},
        "relres_true_max": max(i["relres_true"] for i in inf_mixed),
        "solve_only_solves_per_s": round(so_mixed, 3),
        "kernel_ms": {k: round(t / max(c, 1), 4) for k, (c, t) in kt.items()},
        "kernel_ms_per_step_total": {k: round(t, 3) for k, (c, t) in kt.items()},
        "roofline": {"kernel": "level1_apply: k_level1<false> + k_level1<true> "
                               "(mixed FP32/FP64 factor records)",
                     "bound": "hbm", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_launch": int(l1_bytes),
                     "avg_launch_ms": round(l1_ms, 5),
                     "launches_timed": int(launches)},
    }
    if fp64:
        v64 = nsolves / t_fp64
        out["fp64_path"] = {
            "value": round(v64, 4),
            "solve_only_solves_per_s": round(so_fp64, 3),
            "iterations": {f"{e:g}": i["iters"] for e, i in zip(contrasts, inf_fp64)},
            "latency_ms_p50": round(1e3 * statistics.median(lat_fp64), 3)}
        out["mixed_over_fp64"] = round(value / v64, 4)
        out["mixed_over_fp64_solve_only"] = round(so_mixed / so_fp64, 4)
    if not args.quick:
        # the randomized heat eigen setup (Section 3, M_EH+Rot;Rand) on the
        # same workload and path, timed the same way; kmax + 5 snapshots
        # (the paper's rank guidance for k wanted modes)
        nsnap = probs[0].desc["eig_kmax"] + 5
        rnd = make_solvers(probs, 1, eig_random=nsnap, eig_seed=1)
        run_steps(torch, rnd, rho, f, 1, [], [])
        t_rnd, lat_rnd, inf_rnd = timed(torch, rnd, rho, f, args.steps)
        out["randomized_setup"] = {
            "method": f"M_EH+Rot;Rand, {nsnap} snapshots (FP32-local path)",
            "value": round(nsolves / t_rnd, 4),
            "iterations": {f"{e:g}": i["iters"] for e, i in zip(contrasts, inf_rnd)},
            "coarse_dim": {f"{e:g}": i["n_coarse"] for e, i in zip(contrasts, inf_rnd)},
            "setup_ms": {f"{e:g}": round(i["t_setup_ms"], 3) for e, i in zip(contrasts, inf_rnd)},
            "latency_ms_p50": round(1e3 * statistics.median(lat_rnd), 3)}
        for s_ in rnd:
            s_.close()
    if not args.quick:
        log("[bench] the paper's Table 2 methods")
        out["paper_table2"] = table2_workload(torch)
    if not args.quick and not args.no_3d:
        log("[bench] 3D two-level solve")
        out["solve3d"] = solve3d_workload(torch)
    if not args.no_matvec_probe:
        log("[bench] matvec probe")
        out["matvec_probe"] = matvec_probe(torch)
        log("[bench] 3D matvec probe")
        out["matvec3d_probe"] = matvec3d_probe(torch)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle sample)")
        cb = cpu_baseline(full=args.cpu_full)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores",
                                                  "kind", "sample")}
        out["cpu_baseline"]["value"] = round(cb["value"], 6)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
