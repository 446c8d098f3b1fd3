"""Benchmark: LML + adjoint gradient of the sparsity-discovering exact GP at
N = 1,000,000 points on one MI355X (FP64).

One step = one full evaluation through the C ABI (sdgp_lml_grad): point
ordering, bump precompute, tile pruning, count + fill assembly of the sparse
covariance, block CG on [y, z_1..z_32], SLQ log-det from the CG
coefficients, and the adjoint gradient over all 387 hyperparameters.  Inputs
(x, y) are resident in HBM before the timed region.

Prints one JSON line: the headline value (evaluations per second), plus the
assembly rate, the SpMV bandwidth, the roofline of the dominant kernel (the
CG SpMM) measured with HIP events on the library's stream, and the oracle's
rate on a bounded sample of the same workload (CPU).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LML+grad evals/s at N=1M (FP64); assembly nnz/s; SpMV GB/s vs HBM peak"
METRIC_5M = "LML+grad evals/s at N=5M, 4-D space-time (FP64); assembly nnz/s; SpMV GB/s vs HBM peak"
HBM_PEAK_GBPS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--probes", type=int, default=32)
    p.add_argument("--rtol", type=float, default=1e-10)
    p.add_argument("--precond", choices=["lowrank", "none"], default="lowrank",
                   help="CG preconditioner (low-rank bump part of the SUM kernel, or none)")
    p.add_argument("--operator", choices=["assembled", "factored"], default=None,
                   help="CG operator: the fully assembled sparse K, or K_core (sparse) + F F^T (default: "
                        "factored for single evaluations; populations take the assembled operator only)")
    p.add_argument("--graph", type=int, default=0,
                   help="replay the CG iterations from a HIP graph (1; the SpMM is then not timed per launch)")
    p.add_argument("--spmm-blocks", type=int, default=0,
                   help="grid size of the CG SpMM (multiple of 8; 0: library default)")
    p.add_argument("--update-blocks", type=int, default=0,
                   help="grid size of the CG update kernels (0: library default)")
    p.add_argument("--autotune", type=int, default=1, choices=[0, 1, 2],
                   help="CG launch-shape autotuner (1: library default; the first warm-up step tunes)")
    p.add_argument("--fw-mfma", type=int, default=-1, choices=[-1, 0, 1],
                   help="F w products of the CG updates on the matrix cores (-1: automatic)")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--spmv-reps", type=int, default=50)
    p.add_argument("--probe-rtol", type=float, default=0.0,
                   help="tolerance of the probe columns in the timed steps (0: the same as --rtol)")
    p.add_argument("--probe-report", type=float, default=1e-6,
                   help="after the timed steps, one evaluation with the probe columns to this tolerance, "
                        "reported beside the benchmark (0: skip)")
    p.add_argument("--workload", choices=["uniform3d_n1000000", "spacetime4d_n5000000"],
                   default="uniform3d_n1000000",
                   help="uniform3d_n1000000: 1M points in the unit cube (the headline); spacetime4d_n5000000: "
                        "5M space-time points in 4-D with 32x8 bumps")
    p.add_argument("--population", type=int, default=0, metavar="B",
                   help="instead of the N=1M line, time a population of B hyperparameter vectors on a shared "
                        "N=200,000 point set: one batched call against B sequential calls")
    p.add_argument("--pop-n", type=int, default=200_000)
    p.add_argument("--assembly-only", type=int, default=0, metavar="K",
                   help="instead of the LML line, time K full-K assemblies (sorted order, noise on the diagonal) "
                        "of the workload and print their rate (the assembly part of the metric)")
    p.add_argument("--copy-ref-mib", type=int, default=0,
                   help="before the benchmark, copy a buffer of this many MiB three times (a plain device copy "
                        "of known size, the reference that scales profiler byte counters)")
    return p.parse_args()


def spmm_traffic(operator):
    """HBM bytes per CG SpMM launch (GB) from the committed counter summary,
    or None when the CG source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "cg_kernels_uniform3d_n1000000.txt")
    src = os.path.join(ROOT, "paper_2205_09070_amd", "csrc", "cg.hip")
    try:
        lines = open(path).read().splitlines()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    want, tr = None, None
    for line in lines:
        p = line.split()
        if line.startswith("source_sha256 cg.hip"):
            want = p[2]
        if line.startswith("traffic_gb_per_launch k_cg_spmm %s " % operator):
            tr = {"GB_per_launch": float(p[3]), "fetch_GB": float(p[5]), "write_GB": float(p[7])}
    if want != digest:
        return None
    return tr


def cpu_baseline(w):
    """Measured rate of the dense FP64 oracle (Cholesky LML + analytic
    gradient) on a spatial window of the same point set (same density,
    kernel and hyperparameters).  The O(n^3) extrapolation to the full N is
    reported beside it, labelled as a model."""
    from oracle import gp
    d = w.x.shape[1]
    side = (2800.0 / w.x.shape[0]) ** (1.0 / d)   # about 15 s of oracle work on the host
    m = np.all(w.x < side, axis=1)
    xs, ys = w.x[m], w.y[m]
    ns = xs.shape[0]
    t0 = time.perf_counter()
    gp.lml_grad(w.desc, w.h, xs, ys)
    dt = time.perf_counter() - t0
    n = w.x.shape[0]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / dt, "unit": "evals/s of the %d-point sample" % ns, "cores": threads,
            "kind": "oracle",
            "sample": "dense FP64 oracle LML+gradient (Cholesky) on the %d points of the [0,%.3f)^%d window "
                      "of the same point set: %.2f s per evaluation, measured" % (ns, side, d, dt),
            "sample_points": ns, "sample_s": dt,
            "model_evals_per_s_at_N": (1.0 / dt) * (ns / n) ** 3,
            "model": "not measured: the sample rate scaled to N=%d by the dense oracle's O(n^3) cost" % n}


def population(args, sd, wl, torch):
    """Batched population evaluation (one sdgp_lml_grad_batched call, CG
    iterations replayed from a HIP graph) against one sdgp_lml_grad call per
    member, on the same device, inputs resident in HBM."""
    dev = torch.device("cuda", 0)
    B = args.population
    w, H = wl.population_3d(n=args.pop_n, members=B)
    x = torch.from_numpy(w.x).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    pc = sd.PRECOND_LOWRANK if args.precond == "lowrank" else sd.PRECOND_NONE
    if args.operator == "factored":
        print("bench.py: populations take the assembled operator only (the library rejects the factored "
              "operator for sdgp_lml_grad_batched)", file=sys.stderr)
        sys.exit(2)
    args.operator = "assembled"
    op = sd.OPERATOR_ASSEMBLED
    est = sd.estimator(probes=args.probes, seed=1, cg_rtol=args.rtol, cg_max_iter=20000, precond=pc,
                       operator_form=op)
    ctx = sd.Context(0)
    ctx.set_option("autotune", args.autotune)
    print("population: N=%d B=%d" % (w.x.shape[0], B), file=sys.stderr, flush=True)
    # warm-up: one member each way
    ctx.lml_grad(w.desc, x, y, H[0], est)
    ctx.set_option("graph", 1)
    ctx.lml_grad_batched(w.desc, x, y, H[:1], est)
    # a small population first: the launch-shape tuner of the population
    # class runs here, outside the timed call
    ctx.lml_grad_batched(w.desc, x, y, H[:4], est)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vb, gb, st, infos = ctx.lml_grad_batched(w.desc, x, y, H, est)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    shape_b = {k: ctx.get_option("last_" + k) for k in ("spmm_blocks", "update_blocks", "union_spmm", "fw_mfma",
                                                         "tuned")}
    print("batched: %.2f s, CG launch shape %s" % (tb, shape_b), file=sys.stderr, flush=True)
    ctx.set_option("graph", 0)
    vs = np.zeros(B)
    its = []
    t0 = time.perf_counter()
    for m in range(B):
        vs[m], _, info = ctx.lml_grad(w.desc, x, y, H[m], est)
        its.append(info.cg_iters)
        print("  member %d: nnz/row %.1f cg iters %d" % (m, info.nnz / w.x.shape[0], info.cg_iters),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    print("sequential: %.2f s" % ts, file=sys.stderr, flush=True)
    rel = float(np.max(np.abs(vb - vs) / np.abs(vs)))
    nnz = [int(i.nnz) for i in infos]
    out = {"metric": "population LML+grad evals/s (N=%d, B=%d, FP64)" % (w.x.shape[0], B),
           "value": B / tb, "unit": "evals/s", "n_gpus": 1, "higher_is_better": True,
           "batched_evals_per_s": B / tb, "sequential_evals_per_s": B / ts, "speedup": ts / tb,
           "batched_s": tb, "sequential_s": ts, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "population3d_n%d_b%d: shared uniform [0,1)^3 points, per-member core radius "
                                  "(0.75 rho^2)^(1/3) with rho ~ U(0.005, 0.02), 8x4 shared bumps with per-member "
                                  "heights ~ U(0, 1), SUM combine, %d probes, CG rtol %g, preconditioner %s, "
                                  "operator %s" % (w.x.shape[0], B, args.probes, args.rtol, args.precond,
                                                   args.operator)},
           "cg_launch_shape_batched": shape_b,
           "member_status": [int(v) for v in st], "cg_iters": its,
           "nnz_per_row": [v / w.x.shape[0] for v in nnz],
           "max_rel_diff_batched_vs_sequential": rel}
    print(json.dumps(out))


def assembly_only(args, sd, w, wdesc, x, torch):
    """K timed full-K assemblies (sdgp_kernel_assemble_sorted: order, bump
    values, pruning, count and fill) after one untimed one."""
    ctx = sd.Context(0)
    s = ctx.stream
    nnz = ctx.kernel_nnz(w.desc, x, w.h)
    ctx.kernel_assemble(w.desc, x, w.h, add_noise=True, sorted_order=True, nnz=nnz)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(args.assembly_only):
        ctx.kernel_assemble(w.desc, x, w.h, add_noise=True, sorted_order=True, nnz=nnz)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / args.assembly_only
    print(json.dumps({"metric": "assembly nnz/s (full K, FP64)", "value": nnz / (ms * 1e-3), "unit": "nnz/s",
                      "ms_per_assembly": ms, "nnz": int(nnz), "assemblies": args.assembly_only,
                      "config": {"workload": wdesc}}))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only; --gpus %d is not supported (a multi-GPU "
              "path would shard rows with halo exchanges of P and is not implemented)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2205_09070_amd as sd
    from paper_2205_09070_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    if args.population > 0:
        population(args, sd, wl, torch)
        return
    if args.operator is None:
        args.operator = "factored"
    dev = torch.device("cuda", 0)
    if args.workload == "spacetime4d_n5000000":
        w = wl.spacetime_4d()
        wdesc = ("spacetime4d_n5000000: 5,000,000 points, x1..x3 uniform in [0,1), x4 on 365 time steps, "
                 "Wendland C2 core (l=4, ~50 core neighbours/row) + 32x8 bump functions, SUM combine")
    else:
        w = wl.uniform3d_1m()
        wdesc = ("uniform3d_n1000000: 1,000,000 points uniform in [0,1)^3, Wendland C2 core "
                 "(~60 core neighbours/row) + 16x4 bump functions, SUM combine")
    n = w.x.shape[0]
    x = torch.from_numpy(w.x).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    if args.copy_ref_mib > 0:
        src = torch.ones(args.copy_ref_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.assembly_only > 0:
        assembly_only(args, sd, w, wdesc, x, torch)
        return
    pc = sd.PRECOND_LOWRANK if args.precond == "lowrank" else sd.PRECOND_NONE
    op = sd.OPERATOR_FACTORED if args.operator == "factored" else sd.OPERATOR_ASSEMBLED
    est = sd.estimator(probes=args.probes, seed=1, cg_rtol=args.rtol, cg_max_iter=20000, precond=pc,
                       operator_form=op, probe_rtol=args.probe_rtol)
    ctx = sd.Context(0, timing=True)
    ctx.set_option("graph", args.graph)
    ctx.set_option("fw_mfma", args.fw_mfma)
    ctx.set_option("update_blocks", args.update_blocks)
    ctx.set_option("spmm_blocks", args.spmm_blocks)
    ctx.set_option("autotune", args.autotune)
    print("bench: N=%d dim=%d n1=%d n2=%d probes=%d" % (n, w.desc.dim, w.desc.n1, w.desc.n2, args.probes),
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        val, g, info = ctx.lml_grad(w.desc, x, y, w.h, est)
        print("warmup %d: lml %.10g cg iters %d (%.1f ms)" % (i, val, info.cg_iters, sum(info.ms)),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        val, g, info = ctx.lml_grad(w.desc, x, y, w.h, est)
        infos.append(info.to_dict())
        print("step %d: lml %.10g cg iters %d" % (i, val, info.cg_iters), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    K = args.steps
    value = K / dt
    ms_step = 1000.0 * dt / K
    # the same evaluation through the torch.autograd.Function path (forward
    # + backward), timed beside the plain call
    from paper_2205_09070_amd import autograd as sd_ag
    h_t = torch.tensor(w.h, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    out_ag = sd_ag.lml(h_t, ctx, w.desc, x, y, est)
    out_ag.backward()
    torch.cuda.synchronize()
    autograd_s = time.perf_counter() - ta
    autograd_same = bool(float(out_ag.detach()) == val and np.array_equal(h_t.grad.numpy(), g))
    # the same evaluation with the probe columns to a looser tolerance (y
    # keeps --rtol and finishes alone once the probes have stopped): an
    # option beside the benchmark's setting, not part of the timed value
    probe_report = None
    if args.probe_report > 0.0:
        est_p = sd.estimator(probes=args.probes, seed=1, cg_rtol=args.rtol, cg_max_iter=20000, precond=pc,
                             operator_form=op, probe_rtol=args.probe_report)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        vp, gp, ip = ctx.lml_grad(w.desc, x, y, w.h, est_p)
        torch.cuda.synchronize()
        probe_report = {"probe_rtol": args.probe_report, "s": time.perf_counter() - tp,
                        "cg_iters": ip.cg_iters, "y_alone_iters": ctx.get_option("last_y_tail"),
                        "lml_rel_diff": abs(vp - val) / abs(val),
                        "grad_max_rel_diff": float(np.abs(gp - g).max() / np.abs(g).max()),
                        "logdet_stderr": ip.logdet_stderr,
                        "note": "one evaluation after the timed steps with the probe columns' CG tolerance at "
                                "probe_rtol and y's at cg_rtol; differences against the timed result"}
        print("probe_rtol %g: %.3f s, %d iterations (%d on y alone)" % (
            args.probe_report, probe_report["s"], ip.cg_iters, probe_report["y_alone_iters"]),
            file=sys.stderr, flush=True)
    # phases (mean over timed steps)
    ms = np.mean(np.array([d["ms"] for d in infos]), axis=0)
    nnz = infos[-1]["nnz"]
    cand = infos[-1]["candidates"]
    asm_ms = float(ms[0] + ms[1] + ms[2] + ms[3] + ms[4])
    R = 1 + args.probes
    spmm_launches = sum(d["spmm_launches"] for d in infos)
    spmm_ms = sum(d["spmm_ms"] for d in infos)
    spmm_avg_ms = spmm_ms / spmm_launches if spmm_launches else float("nan")
    # algorithmic bytes of one CG SpMM launch: CSR (8 B value + 4 B column per
    # entry, 8 B row pointer per row), P read once, Q written once
    spmm_bytes = 12.0 * nnz + 8.0 * (n + 1) + 2.0 * 8.0 * n * R
    spmm_gbps = spmm_bytes / (spmm_avg_ms * 1e-3) / 1e9
    # full sparse covariance (all bump terms) in the solver's order: its
    # assembly rate and a plain SpMV (R = 1) on it
    s = ctx.stream
    full_nnz = ctx.kernel_nnz(w.desc, x, w.h)
    ctx.kernel_assemble(w.desc, x, w.h, add_noise=True, sorted_order=True, nnz=full_nnz)
    ea0 = torch.cuda.Event(enable_timing=True)
    ea1 = torch.cuda.Event(enable_timing=True)
    ea0.record(s)
    rp, col, vv, perm = ctx.kernel_assemble(w.desc, x, w.h, add_noise=True, sorted_order=True, nnz=full_nnz)
    ea1.record(s)
    ea1.synchronize()
    full_asm_ms = ea0.elapsed_time(ea1)
    xv = torch.randn(n, dtype=torch.float64, device=dev)
    yv = torch.empty_like(xv)
    for _ in range(3):
        ctx.csr_spmm(rp, col, vv, xv, out=yv)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(args.spmv_reps):
        ctx.csr_spmm(rp, col, vv, xv, out=yv)
    e1.record(s)
    e1.synchronize()
    spmv_ms = e0.elapsed_time(e1) / args.spmv_reps
    spmv_nnz = col.numel()
    spmv_bytes = 12.0 * spmv_nnz + 8.0 * (n + 1) + 8.0 * n + 8.0 * n
    spmv_gbps = spmv_bytes / (spmv_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC if args.workload == "uniform3d_n1000000" else METRIC_5M,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wdesc + ", %d Rademacher probes, CG rtol %g%s, preconditioner %s, operator %s"
                               % (args.probes, args.rtol,
                                  (" (probes %g)" % args.probe_rtol) if args.probe_rtol > 0 else "",
                                  args.precond, args.operator),
                   "points": n, "dim": int(w.desc.dim), "n1": w.desc.n1, "n2": w.desc.n2, "n_hyper": int(len(w.h)),
                   "probes": args.probes, "cg_rtol": args.rtol, "precond": args.precond,
                   "operator": args.operator, "graph": bool(args.graph)},
        "nnz": int(nnz),
        "nnz_per_row": nnz / n,
        "candidates": int(cand),
        "cg_iters": infos[-1]["cg_iters"],
        "phase_ms": {"order": ms[0], "bump": ms[1], "prune": ms[2], "count": ms[3], "fill": ms[4],
                     "cg": ms[5], "slq": ms[6], "adjoint": ms[7]},
        "assembly_nnz_per_s": spmv_nnz / (full_asm_ms * 1e-3),
        "assembly": {"matrix": "full K + noise", "nnz": int(spmv_nnz), "ms": full_asm_ms,
                     "note": "one sdgp_kernel_assemble_sorted call: order + bump + prune + count + fill"},
        "solver_matrix_assembly_ms": asm_ms,
        "spmv": {"ms": spmv_ms, "GBps": spmv_gbps, "frac_hbm": spmv_gbps / HBM_PEAK_GBPS, "bytes": spmv_bytes,
                 "matrix": "full assembled K + noise (%d nnz)" % spmv_nnz},
        "roofline": {"kernel": ("k_cg_spmm_u (CG SpMM over 4-row union lists" if ctx.get_option("last_union_spmm")
                               else "k_cg_spmm (CG SpMM over CSR rows") +
                              ", %d right-hand sides; algorithmic bytes of the CSR form)" % R, "bound": "hbm",
                     "achieved": spmm_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": spmm_gbps / HBM_PEAK_GBPS,
                     "traffic": ((spmm_traffic(args.operator) or {}).get("GB_per_launch")
                                 if args.workload == "uniform3d_n1000000" else None),
                     "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1, copy-scaled)",
                     "avg_launch_ms": spmm_avg_ms, "launches": spmm_launches,
                     "algorithmic_bytes_per_launch": spmm_bytes},
        "lml": val,
        "autograd_path": {"s": autograd_s, "plain_s": dt / K, "bitwise_equal_to_plain": autograd_same,
                          "note": "one evaluation through torch.autograd.Function (forward + backward) after "
                                  "the timed steps"},
        "probe_tolerance": probe_report,
        "cg_launch_shape": {k: ctx.get_option("last_" + k) for k in
                            ("spmm_blocks", "update_blocks", "union_spmm", "fw_mfma", "tuned")},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
