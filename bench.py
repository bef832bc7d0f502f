#!/usr/bin/env python3
"""Throughput of the k-point CCSD T2 residual on one MI355X.

Workload (default): seeded synthetic system on a 3x3x3 k mesh (N_k = 27), n_occ = 8,
n_vir = 16 spin orbitals per k, integrals generated on the device by the seeded recipe
(complex Gaussians x 0.05/N_k, antisymmetrized and Hermitized), diagonal Fock, DIIS(6).
A step is one iteration of the whole path: the residual (tau, F, W_mnij, T1-dressed
<ab||ef>, ring W, ring product, T2 assembly, particle-particle and hole-hole ladders,
T1 residual), its norm, the correlation energy, the update t <- t + R/D and DIIS.
Inputs are resident in HBM before the timed region starts.

Prints one JSON line: value = residual evaluations per second of the headline path,
with the roofline of the dominant grouped product (the one with the largest total time;
HIP events on the library's stream) and of the ladder product, and the FP64 CPU oracle
timed on a bounded sample on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "T2 residual evals/s + TFLOP/s at N_k=27 (split-BF16 vs FP64, |ΔE|≤1e-8)"
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}  # dense MFMA TFLOP/s, MI355X


# Sources whose text fixes a GEMM kernel's memory traffic: the kernel file and the
# headers that define its tile order and operand storage.
KERNEL_SOURCES = {
    "fp64": ["paper_1911_00242_amd/csrc/gemm_f64.hip", "paper_1911_00242_amd/csrc/common.h"],
    "mixed": ["paper_1911_00242_amd/csrc/gemm_mixed.hip", "paper_1911_00242_amd/csrc/common.h",
              "paper_1911_00242_amd/csrc/mixed.h"],
}
PRODUCT_KERNEL = {"pp_ladder": "particle-particle ladder grouped GEMM", "hh_ladder": "hole-hole ladder grouped GEMM",
                  "w_mnij": "W_mnij grouped GEMM", "w_mbej": "W_mbej grouped GEMM",
                  "ring": "ring product grouped GEMM"}


def source_hash(key):
    import hashlib

    h = hashlib.sha256()
    for src in KERNEL_SOURCES[key.rsplit("_", 1)[1]]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()[:16]


def measured_record(key):
    """The committed rocprofv3 counter record of a product kernel (HBM bytes per launch, MFMA
    busy fraction, clock), or None when the kernel sources changed since it was taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[key]
        return rec if source_hash(key) == rec["source_sha256_16"] else None
    except (OSError, KeyError, ValueError):
        return None


def measured_traffic(key):
    rec = measured_record(key)
    return rec["hbm_bytes_per_launch"] if rec else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both")
    ap.add_argument("--grid", default="3,3,3")
    ap.add_argument("--no", type=int, default=8)
    ap.add_argument("--nv", type=int, default=16)
    ap.add_argument("--seed", type=int, default=303)
    ap.add_argument("--diis", type=int, default=6)
    ap.add_argument("--grouping", choices=["standard", "rearranged"], default="standard",
                    help="hole-hole grouping of the FP64 path: Sec. 2 (standard) or Sec. 3.3.4 (rearranged)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", type=float, default=0.0,
                    help="mixed path: run the autotuner with this error budget before timing (0 = keep the "
                         "default forms) and report its choices")
    ap.add_argument("--overlap", type=int, default=1,
                    help="mixed path: side kernels on a second stream beside the grouped products (0 = one stream)")
    ap.add_argument("--converge", type=int, default=1, help="after timing, iterate to convergence and "
                    "compare the paths' energies and amplitudes (0 = skip)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--tol-mixed", type=float, default=1e-7,
                    help="the split-BF16 residual has a rounding floor near 1e-8..1e-7 at N_k=27")
    ap.add_argument("--max-iter", type=int, default=60)
    ap.add_argument("--batch-summary", type=int, default=1,
                    help="also run the 96-system batched form on the mixed path and report it under 'batch'")
    ap.add_argument("--largest", default="5,4,2",
                    help="with the default workload, also time the mixed path on this mesh (the largest that "
                         "fits one MI355X at n_occ=8, n_vir=16) and report it under 'largest_instance' (0 = skip)")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead of the N_k=27 workload: the batched form, this many independent seeded "
                         "systems (shapes drawn from seed 40000), converged on both paths")
    return ap.parse_args()


def run_path(ck, torch, prec, grid, no, nv, seed, diis, steps, warmup, converge, tol, max_iter, grouping=0,
             autotune=0.0, overlap=True):
    N = grid[0] * grid[1] * grid[2]
    desc = dict(grid=grid, no=no, nv=nv, precision=prec, diis_space=diis, synthetic=1, seed=seed,
                eri_scale=0.05 / N, grouping=grouping if prec == 0 else 0)
    print(f"[bench] {('fp64', 'mixed')[prec]}: binding workspace", file=sys.stderr, flush=True)
    ctx = ck.Context([desc], device="cuda:0")
    ctx.set_overlap(overlap)
    # the timed passes measure the products in their chosen forms: precision escalation (a
    # convergence aid that changes forms once the norm stalls, as it does when iterating past
    # the floor with tolerance 0) stays off until the convergence phase
    ctx.set_escalation(False)
    tuned = None
    if autotune and prec == 1:
        ctx.iterate(1, 0.0)  # operands of real amplitudes in the buffers
        forms, rep = ctx.autotune(autotune)
        tuned = {"budget": autotune, "forms": {name: (ck.FORMS[f] if f >= 0 else None)
                                                for name, f in zip(ck.STAGES[:5], forms)},
                 "measured": {name: {ck.FORMS[a]: {"ms": rep[p, a, 0], "error": rep[p, a, 1]} for a in range(4)}
                              for p, name in enumerate(ck.STAGES[:5]) if p != 1}}
        print(f"[bench] autotune budget {autotune}: {tuned['forms']}", file=sys.stderr, flush=True)
    gemm_flops, other_flops = ctx.flops(0)
    # executed shapes of the five grouped products (the mixed path runs the ladder family
    # on canonical antisymmetric pairs, a quarter of the algorithmic work)
    shapes = {name: ctx.product_shape(name) for name in ck.STAGES[:5]}
    for w in range(warmup):
        ctx.iterate(1, 0.0)
        print(f"[bench] warmup {w + 1}/{warmup} done", file=sys.stderr, flush=True)
    # timed region: each iteration replayed from the captured graph (stage timing off)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    energy = None
    for s in range(steps):
        ctx.iterate(1, 0.0)
        energy = ctx.energy(0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] {steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)
    # per-product launch times: HIP events on the library's stream around every product
    # launch over as many further iterations (enqueued directly: events are not captured)
    ctx.timing(True)
    for s in range(steps):
        ctx.iterate(1, 0.0)
    stages = {name: ctx.timing_get(name) for name in ck.STAGES}
    ctx.timing(False)
    print(f"[bench] {steps} timed-stage steps done", file=sys.stderr, flush=True)
    exec_flops = sum(8.0 * G * M * Nn * K for (G, M, Nn, K) in shapes.values())
    forms = {name: ctx.product_form(name) for name in PRODUCT_KERNEL if name != "hh_ladder"} if prec == 1 else {}
    out = dict(seconds=dt, tuned=tuned, forms=forms, gemm_flops=gemm_flops, exec_flops=exec_flops, shapes=shapes, other_flops=other_flops,
               stages=stages,
               energy=energy, workspace_bytes=ctx.nbytes, rnorm=ctx.residual_norm(0))
    if converge:
        done = warmup + 2 * steps  # warm-up, timed and stage-timing iterations
        ctx.set_escalation(True)
        rc, it, rn = ctx.iterate(max(0, max_iter - done), tol)
        out.update(conv_rc=rc, conv_iters=done + it, conv_rnorm=rn, conv_energy=ctx.energy(0),
                   t2=ctx.get_amplitudes(0)[1])
        print(f"[bench] converge: rc={rc} evaluations={done + it} |R|={rn:.3e} E={out['conv_energy']}",
              file=sys.stderr, flush=True)
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return out


def largest_instance(ck, torch, a):
    """The mixed path on the largest mesh one GPU holds at the workload's block shape: its
    step time (captured iterations, as for the main line) and its dominant product."""
    grid = tuple(int(x) for x in a.largest.split(","))
    N = grid[0] * grid[1] * grid[2]
    steps = 3
    r = run_path(ck, torch, 1, grid, a.no, a.nv, a.seed, a.diis, steps, 1, 0, a.tol_mixed, a.max_iter)
    ms = 1000.0 * r["seconds"] / steps
    dom = max((k for k in PRODUCT_KERNEL if r["stages"][k][1]), key=lambda k: r["stages"][k][0])
    tot, n = r["stages"][dom]
    G, M, Nn, K = r["shapes"][dom]
    achieved = 24.0 * G * M * Nn * K / (tot / n / 1000.0) / 1e12
    return {"grid": list(grid), "N_k": N, "n_occ": a.no, "n_vir": a.nv, "evals_per_s": 1000.0 / ms,
            "ms_per_step": ms, "steps": steps, "workspace_gb": r["workspace_bytes"] / 1e9,
            "tflops": r["exec_flops"] / (ms / 1000.0) / 1e12,
            "dominant_product": {"kernel": PRODUCT_KERNEL[dom], "avg_launch_ms": tot / n,
                                 "achieved_tflops": achieved, "frac_of_bf16_peak": achieved / PEAK["bf16"]},
            "stages_ms_per_step": {k: v[0] / steps for k, v in r["stages"].items()}}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(no, nv, N_target):
    """The FP64 oracle on a bounded sample (about 10-25 s of CPU work): residuals on a
    2x2x2 mesh with the same per-k block shapes, repeated until 10 s have passed (at most
    four), the time per residual scaled to the target mesh by the N_k^4 algorithmic flop
    ratio; and one residual on a 2x1x1 mesh with a single BLAS thread, scaled the same way."""
    import numpy as np

    import synth
    from oracle import ccsd_k as O

    grid = (2, 2, 2)
    f, eris = synth.system(303, grid, no, nv, scale=0.05 / 8)
    t1, t2 = synth.test_amplitudes(1, grid, no, nv, scale=0.01)
    kc = O.kconserv(grid)
    reps = 0
    t0 = time.perf_counter()
    while reps < 4 and (reps == 0 or time.perf_counter() - t0 < 10.0):
        O.residual(f, eris, t1, t2, kc)
        reps += 1
    dt = (time.perf_counter() - t0) / reps
    threads = 1
    single = None
    try:
        from threadpoolctl import threadpool_info, threadpool_limits

        threads = max([x.get("num_threads", 1) for x in threadpool_info()] + [1])
        g1 = (2, 1, 1)
        f1, e1 = synth.system(303, g1, no, nv, scale=0.05 / 2)
        a1, a2 = synth.test_amplitudes(1, g1, no, nv, scale=0.01)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            O.residual(f1, e1, a1, a2, O.kconserv(g1))
            d1 = time.perf_counter() - t0
        r1 = (N_target / 2.0) ** 4
        single = {"value": 1.0 / (d1 * r1), "unit": "evals/s", "threads": 1,
                  "sample": f"one oracle residual on a 2x1x1 mesh ({d1:.2f} s), scaled by {r1:.0f}"}
    except Exception:
        pass
    ratio = (N_target / 8.0) ** 4
    return {"value": 1.0 / (dt * ratio), "unit": "evals/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{reps} oracle residual(s) on a 2x2x2 mesh with n_occ={no}, n_vir={nv} per k "
                      f"({dt:.2f} s each), scaled by the N_k^4 flop ratio {ratio:.0f} to N_k={N_target}",
            "sample_seconds": dt * reps, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "cpu_model": _cpu_model(), "one_thread": single}


def _batch_shapes(a):
    import synth

    return synth.batch_shapes(40000, a.batch or 96)


def _batch_converge(a, shapes, prec, tol, timed_steps):
    """Converge a batch of independent systems on one path.  The systems go into as few
    contexts as fit the memory budget, one context iterating all of its systems together
    (side by side on its lanes, each iteration one captured graph).  Returns per-system
    energies, convergence flags and norms, the time of each of the first timed_steps batched
    iterations (every system active, after one warm-up iteration) and the time to converge."""
    import numpy as np
    import torch

    import paper_1911_00242_amd as ck

    def desc(d):
        return dict(grid=d["grid"], no=d["no"], nv=d["nv"], precision=prec, diis_space=a.diis, synthetic=1,
                    seed=d["seed"], eri_scale=0.05 / int(np.prod(d["grid"])))

    sizes = []
    for d in shapes:
        c = ck.ccsd_k_init([desc(d)])
        sizes.append(ck.ccsd_k_workspace_bytes(c) + (1 << 16))
        ck.ccsd_k_free(c)
    groups, cur, tot = [], [], 0
    for i, nb in enumerate(sizes):
        if cur and tot + nb > 230e9:
            groups.append(cur)
            cur, tot = [], 0
        cur.append(i)
        tot += nb
    groups += [cur] if cur else []
    energy, conv, rnorm, iter_ms, total = {}, {}, {}, [], 0.0
    for gi, grp in enumerate(groups):
        print(f"[bench] batch {('fp64', 'mixed')[prec]}: group {gi} ({len(grp)} systems)", file=sys.stderr,
              flush=True)
        if timed_steps:
            with ck.Context([desc(shapes[i]) for i in grp], device="cuda:0") as c:
                c.iterate(1, 0.0)
                ms = []
                for s in range(timed_steps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    c.iterate(1, 0.0)
                    torch.cuda.synchronize()
                    ms.append(1000.0 * (time.perf_counter() - t0))
                iter_ms.append(ms)
            torch.cuda.empty_cache()
        with ck.Context([desc(shapes[i]) for i in grp], device="cuda:0") as c:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.iterate(a.max_iter, tol)
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
            for k, i in enumerate(grp):
                energy[i] = c.energy(k)
                rnorm[i] = c.residual_norm(k)
                conv[i] = rnorm[i] < tol
        torch.cuda.empty_cache()
    # a batched iteration of the whole batch: the groups' iterations at the same index
    per_iter = [sum(g[s] for g in iter_ms) for s in range(timed_steps)] if timed_steps else []
    return energy, conv, rnorm, per_iter, total


def batch_summary(a):
    """The batched form on the mixed path (the default bench line's "batch" key): systems
    converged per second and the time per batched iteration."""
    import numpy as np

    shapes = _batch_shapes(a)
    e, c, n, it, t = _batch_converge(a, shapes, 1, a.tol_mixed, 5)
    n_conv = sum(1 for i in range(len(shapes)) if c[i])
    return {"systems": len(shapes), "converged_mixed": n_conv, "systems_converged_per_s": n_conv / t,
            "seconds_to_converge": t, "tol": a.tol_mixed,
            "iteration_ms": {"p50": float(np.percentile(it, 50)), "p99": float(np.percentile(it, 99)),
                             "samples": len(it)} if it else None,
            "workload": f"{len(shapes)} seeded systems, N_k from {{1,2,4,8}}, n_occ from {{4,6,8,12}}, "
                        f"n_vir from {{8,16,24,32}} (seed 40000), integrals x 0.05/N_k, DIIS({a.diis})"}


def run_batch(a):
    """The batched form: a.batch independent systems (N_k from {1, 2, 4, 8}, n_occ from
    {4, 6, 8, 12}, n_vir from {8, 16, 24, 32}, drawn with tag 3 from seed 40000; system s has
    seed 40000 + s and integrals scaled by 0.05 / N_k), iterated with DIIS to convergence.
    Timed on the mixed path: the time per batched iteration over the first a.steps
    iterations (every system active), and the whole run to convergence (systems converged
    per second); the FP64 path converges the same systems for the per-system energy
    reference, and the oracle the smallest few."""
    import numpy as np

    import synth
    from oracle import ccsd_k as O

    shapes = _batch_shapes(a)
    e_mx, c_mx, n_mx, it_mx, t_mx = _batch_converge(a, shapes, 1, a.tol_mixed, a.steps)
    e_64, c_64, _, _, t_64 = _batch_converge(a, shapes, 0, a.tol, 0)
    both = [i for i in range(len(shapes)) if c_mx[i] and c_64[i]]
    de = [abs(e_mx[i] - e_64[i]) for i in both]
    # the oracle on the smallest systems (pp-ladder work N^4 o^2 v^4)
    work = sorted(range(len(shapes)), key=lambda i: int(np.prod(shapes[i]["grid"])) ** 4 * shapes[i]["no"] ** 2
                  * shapes[i]["nv"] ** 4)
    oracle = []
    for i in [j for j in work if c_mx[j] and c_64[j]][:3]:
        d = shapes[i]
        N = int(np.prod(d["grid"]))
        print(f"[bench] batch: oracle on system {i} {d['grid']} o={d['no']} v={d['nv']}", file=sys.stderr,
              flush=True)
        f, eris = synth.system(d["seed"], d["grid"], d["no"], d["nv"], scale=0.05 / N)
        ref = O.solve(f, eris, d["grid"], max_iter=a.max_iter, tol=a.tol, diis_space=a.diis)
        oracle.append({"system": i, "grid": list(d["grid"]), "n_occ": d["no"], "n_vir": d["nv"],
                       "converged": bool(ref["converged"]), "abs_dE_fp64": abs(e_64[i] - ref["energy"]),
                       "abs_dE_mixed": abs(e_mx[i] - ref["energy"])})
    n_conv = sum(1 for i in range(len(shapes)) if c_mx[i])
    line = {
        "metric": "systems converged/s (batched form)", "value": n_conv / t_mx, "unit": "systems/s",
        "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "bf16x3/f32acc+f64",
        "config": {"workload": f"{len(shapes)} independent seeded k-point CCSD systems, N_k from {{1,2,4,8}}, "
                               f"n_occ from {{4,6,8,12}}, n_vir from {{8,16,24,32}}, DIIS({a.diis})",
                   "seed": 40000},
        "systems": len(shapes), "converged_mixed": n_conv, "converged_fp64": sum(c_64.values()),
        "seconds_to_converge": {"mixed": t_mx, "fp64": t_64},
        "iteration_ms": {"p50": float(np.percentile(it_mx, 50)), "p99": float(np.percentile(it_mx, 99)),
                         "samples": len(it_mx)} if it_mx else None,
        "mixed_vs_fp64_abs_dE": {"max": max(de) if de else None, "median": float(np.median(de)) if de else None,
                                 "systems": len(de)},
        "oracle_subset": oracle,
        "unconverged_mixed": [{"system": i, "grid": list(shapes[i]["grid"]), "n_occ": shapes[i]["no"],
                               "n_vir": shapes[i]["nv"], "rnorm": n_mx[i]} for i in range(len(shapes)) if not c_mx[i]],
    }
    print(json.dumps(line), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (its grouped "
              "products are independent per momentum group, which is how they would be dealt to GPUs)",
              file=sys.stderr)
        sys.exit(2)
    if a.batch:
        run_batch(a)
        return
    import torch

    import paper_1911_00242_amd as ck

    grid = tuple(int(x) for x in a.grid.split(","))
    N = grid[0] * grid[1] * grid[2]
    paths = {"fp64": [0], "mixed": [1], "both": [0, 1]}[a.precision]
    res = {}
    for p in paths:
        res[p] = run_path(ck, torch, p, grid, a.no, a.nv, a.seed, a.diis, a.steps, a.warmup, a.converge,
                          a.tol if p == 0 else a.tol_mixed, a.max_iter, 1 if a.grouping == "rearranged" else 0,
                          a.autotune, bool(a.overlap))
    head = 1 if 1 in res else 0
    r = res[head]
    ms = 1000.0 * r["seconds"] / a.steps
    value = 1000.0 / ms
    tflops = r["exec_flops"] / (ms / 1000.0) / 1e12
    path = "fp64" if head == 0 else "mixed"
    peak, dtype, per_cmac = ((PEAK["fp64"], "f64", 8.0) if head == 0 else
                             (PEAK["bf16"], "bf16x3/f32acc+f64", 24.0))

    def roofline(name):
        """The product's executed work per launch (per_cmac flops per complex multiply-add:
        8 for FP64, 24 = 3 bf16 products x 4 real products x 2 for split-BF16) over its
        average launch time from HIP events on the library's stream."""
        tot_ms, n = r["stages"][name]
        G, M, Nn, K = r["shapes"][name]
        if not n or not G:
            return None
        avg = tot_ms / n
        unit_flops, pk = per_cmac, peak
        form = r["forms"].get(name, 0)
        if head == 1 and form == 2:  # three-term split: six bf16 products per real product
            unit_flops = 48.0
        elif head == 1 and form == 3:  # FP32 MFMA: four real products per complex MAC
            unit_flops, pk = 8.0, PEAK["fp32"]
        achieved = unit_flops * G * M * Nn * K / (avg / 1000.0) / 1e12
        # counters were taken on the default form of the profiled workload only
        rec = (measured_record(f"{name}_{path}") if (grid, a.no, a.nv) == ((3, 3, 3), 8, 16) and form == 0
               else None)
        traffic = rec["hbm_bytes_per_launch"] if rec else None
        out = {"bound": "mfma", "achieved": achieved, "peak": pk, "unit": "TFLOP/s", "frac": achieved / pk,
               "traffic": traffic / 1e9 if traffic else None, "traffic_unit": "GB per launch",
               "kernel": PRODUCT_KERNEL[name] + (" (both ladders, packed pairs)" if head == 1 and name == "pp_ladder"
                                                  else ""),
               "avg_launch_ms": avg, "shape": {"groups": G, "M": M, "N": Nn, "K": K}}
        if rec and "mfma_busy" in rec:
            # from the committed counter run: SQ_VALU_MFMA_BUSY_CYCLES over the SIMD cycles of
            # the launch, and the clock (GRBM_GUI_ACTIVE per XCD over the launch time); the
            # peak at that clock scales the 2.4 GHz figure
            out["counters"] = {"mfma_busy": rec["mfma_busy"], "clock_ghz": rec["clock_ghz"],
                               "frac_at_clock": achieved / (pk * rec["clock_ghz"] / 2.4),
                               "source": rec["summary"]}
        return out

    products = [k for k in PRODUCT_KERNEL if r["stages"][k][1]]
    dominant = max(products, key=lambda k: r["stages"][k][0])
    line = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"k-point CCSD T2 residual iteration, {grid[0]}x{grid[1]}x{grid[2]} mesh "
                               f"(N_k={N}), n_occ={a.no}, n_vir={a.nv} spin orbitals per k, DIIS({a.diis})",
                   "grid": list(grid), "n_occ": a.no, "n_vir": a.nv, "seed": a.seed},
        "tflops": tflops,
        "tflops_algorithmic": r["gemm_flops"] / (ms / 1000.0) / 1e12,
        "roofline": roofline(dominant),
        "roofline_ladder": roofline("pp_ladder"),
        "stages_ms_per_step": {k: v[0] / a.steps for k, v in r["stages"].items()},
        "energy": [r["energy"].real, r["energy"].imag],
    }
    if r.get("tuned"):
        line["autotune"] = r["tuned"]
    if 0 in res and 1 in res:
        line["fp64_path"] = {"evals_per_s": a.steps / res[0]["seconds"],
                             "tflops": res[0]["exec_flops"] * a.steps / res[0]["seconds"] / 1e12}
        line["speedup_vs_fp64"] = res[0]["seconds"] / res[1]["seconds"]
    if a.converge:
        import numpy as np

        line["convergence"] = {("fp64", "mixed")[p]: {"status": v["conv_rc"], "evaluations": v["conv_iters"],
                                                        "rnorm": v["conv_rnorm"],
                                                        "energy": [v["conv_energy"].real, v["conv_energy"].imag]}
                               for p, v in res.items()}
        if 0 in res and 1 in res:
            line["mixed_vs_fp64"] = {"abs_dE": abs(res[1]["conv_energy"] - res[0]["conv_energy"]),
                                     "max_abs_dT2": float(np.abs(res[1]["t2"] - res[0]["t2"]).max()),
                                     "reference": "FP64 GPU path converged to ||R|| < tol"}
    if a.batch_summary and (grid, a.no, a.nv) == ((3, 3, 3), 8, 16):
        line["batch"] = batch_summary(a)
    if a.largest != "0" and (grid, a.no, a.nv) == ((3, 3, 3), 8, 16):
        line["largest_instance"] = largest_instance(ck, torch, a)
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(a.no, a.nv, N)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    # Systems iterated together run on eight streams of the library's beside the context's
    # stream; the HIP runtime opens four hardware queues per process unless told otherwise,
    # so streams share queues and their kernels wait behind each other.  Sixteen queues give
    # every stream its own (the 96-system batch measured 149 ms per iteration against 155 ms
    # with four or eight).  Set before the runtime starts: torch and the library are loaded
    # inside main.
    os.environ["GPU_MAX_HW_QUEUES"] = "16"
    main()
