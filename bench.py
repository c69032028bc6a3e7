"""Benchmark: time to 1e-2 relative trace error of deflated MGMLMC on the 1024^2
Wilson-Schwinger lattice, mixed precision + batched RHS against plain FP64 single-RHS,
plus the achieved HBM bandwidth of the stencil kernels.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload schwinger1024]

One step = one complete MGMLMC estimate to relative error eps = 1e-2 (all levels: noise,
deflation projections, multigrid-preconditioned solves, sample dots, accumulation and
allocation) with identical sample sets in both precisions.  The timed steps carry no
timing events, so the recorded HIP graphs of the FGMRES iterations are replayed; the
dominant kernel's launch times come from a second pass over the same steps with events
around that kernel only (one event pair around each run of its back-to-back launches, such
as the colour sweeps of a smoother: launch time = run time / launches in the run).  Setup (hierarchy, coarsest eigensolve, explicit coarsest
inverse) is timed separately, like the paper's "eig.+direct" column, and added in the
setup-plus-trace totals.  Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to 1e-2 rel. trace error, mixed+batched vs FP64 (s); stencil HBM GB/s"
HBM_PEAK_GBPS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
HBM_CLASSES = ("wilson", "coarse", "sap", "coarse_gs", "restrict", "prolong", "gs_dots", "gs_update",
               "coarse_direct16", "coarse_direct8", "combine")
STENCIL_CLASSES = ("wilson", "coarse", "sap", "coarse_gs", "restrict", "prolong")
# source file of each timed kernel class (a recorded HBM traffic figure is only valid for the
# source it was measured on)
CLASS_SOURCE = {"wilson": "stencil.hip", "coarse": "stencil.hip", "sap": "stencil.hip", "coarse_gs": "stencil.hip",
                "restrict": "stencil.hip", "prolong": "stencil.hip", "gs_dots": "gram.hip", "gs_update": "gram.hip",
                "coarse_direct16": "dense.hip", "coarse_direct8": "dense.hip", "combine": "solver.hip"}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def timers(ctx, classes):
    out = {}
    for c in classes:
        n, ms, b = ctx.timing_get(c)
        out[c] = {"launches": n, "ms": ms, "bytes": b}
    return out


def source_digest(cls: str) -> str:
    path = os.path.join(ROOT, "paper_2211_15383_amd", "csrc", CLASS_SOURCE[cls])
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def recorded_traffic(cls: str, algorithmic_per_launch: float):
    """HBM bytes per launch of a kernel class from a committed rocprofv3 --pmc summary
    (FETCH_SIZE + WRITE_SIZE scaled by a copy kernel of known size), if it was measured on
    the current source of that kernel and on the same launch mix (algorithmic bytes per
    launch within 0.5 %); else (None, None)."""
    want = source_digest(cls)
    pat = re.compile(r"^traffic: class=(\S+) source_sha256=(\S+) bytes_per_launch=(\S+) "
                     r"algorithmic_bytes_per_launch=(\S+)")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md"))):
        with open(path) as f:
            for line in f:
                m = pat.match(line.strip())
                if (m and m.group(1) == cls and m.group(2) == want
                        and abs(float(m.group(4)) - algorithmic_per_launch) <= 5e-3 * algorithmic_per_launch):
                    return float(m.group(3)), os.path.basename(path)
    return None, None


def copy_ceiling(torch, nbytes: int = 1 << 30, reps: int = 10) -> float:
    """GB/s of a plain elementwise kernel reading and writing nbytes each (x + 1)."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.add(src, 1.0, out=dst)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(src, 1.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def kernel_rates(torch, dm, ctx, H, nlev: int, b: int, reps: int = 10):
    """Each stencil-class kernel alone at the workload's real shapes (b RHS, complex FP32,
    rows at the solver's padded work stride), reps launches after one warm-up: algorithmic
    bytes per launch / mean event time."""
    out = {}
    ctx.timing_select(None)
    ctx.timing(True)
    dev = "cuda:0"
    for l in range(1, nlev):
        ld, ldc = H.work_stride(l), H.work_stride(l + 1)
        x = torch.randn(b, ld, dtype=torch.complex64, device=dev)
        y = torch.randn(b, ld, dtype=torch.complex64, device=dev)
        xc = torch.randn(b, ldc, dtype=torch.complex64, device=dev)
        yc = torch.empty_like(xc)
        cases = [("wilson" if l == 1 else "coarse", dm.OP_D, x, y, ld, ld, 0),
                 ("restrict", dm.OP_RESTRICT, x, yc, ld, ldc, 0),
                 ("prolong", dm.OP_PROLONG, xc, y, ldc, ld, 0),
                 ("sap" if l == 1 else "coarse_gs", dm.OP_SMOOTH, x, y, ld, ld, 1)]
        for cls, op, a, o, lda, ldo, arg in cases:
            H.apply(op, l, a, o, dm.MIXED, arg, ld_in=lda, ld_out=ldo)
            ctx.timing_reset()
            for _ in range(reps):
                H.apply(op, l, a, o, dm.MIXED, arg, ld_in=lda, ld_out=ldo)
            nl, ms, by = ctx.timing_get(cls)
            out[f"{cls}_level{l}"] = {"launches": nl, "avg_us": 1e3 * ms / max(1, nl),
                                      "bytes_per_launch": by / max(1, nl),
                                      "GBps": by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0}
        del x, y, xc, yc
    ctx.timing(False)
    torch.cuda.synchronize()
    return out


def matrix_core_rates(torch, dm, ctx, H, D, L: int, b: int, reps: int = 10):
    """The deflation products (C = W^H X, X - W C: complex-FP32 matrix cores) and the coarsest
    solve of the V-cycle (the explicit inverse applied in complex FP16 when enabled) alone at
    the coarsest level's shape with b RHS, reps launches after one warm-up."""
    out = {}
    n = H.n(L)
    x = torch.randn(b, n, dtype=torch.complex128, device="cuda:0")
    y = torch.empty_like(x)
    c = torch.empty(b, D.k, dtype=torch.complex128, device="cuda:0")
    x32 = x.to(torch.complex64)
    y32 = torch.empty_like(x32)
    H.set_deflation(D)
    ctx.timing_select(None)
    ctx.timing(True)
    for name, cls, op, a, o in (("defl_coeffs", "defl_gemm", dm.OP_DEFL_C, x, c),
                                ("defl_project", "defl_gemm", dm.OP_DEFL_P, x, y),
                                ("coarsest_solve", "coarse_direct16", dm.OP_VCYCLE, x32, y32)):
        H.apply(op, L, a, o, dm.MIXED)
        ctx.timing_reset()
        for _ in range(reps):
            H.apply(op, L, a, o, dm.MIXED)
        nl, ms, work = ctx.timing_get(cls)
        out[f"{name}_level{L}"] = {"class": cls, "launches": nl, "avg_us": 1e3 * ms / max(1, nl),
                                   "work_per_launch": work / max(1, nl)}
    ctx.timing(False)
    H.set_deflation(None)
    torch.cuda.synchronize()
    return out


def method_comparison(torch, dm, ctx, name: str, eps: float, kdiff: int, hutch_k=(), diff=True):
    """The variants of the paper's Table 1 on one synthetic workload (mixed precision,
    coarsest term always deflated): plain MGMLMC; level 2 skipped (eq. 12); and each of
    those with the first difference term exactly deflated by its kdiff largest singular
    triplets (Sec. 4.2); then plain Hutchinson at the fine level deflated by each k in
    hutch_k (eqs. 4-7).  Returns setup and estimate seconds per variant."""
    from paper_2211_15383_amd.inputs import WORKLOADS, load_m0

    W = WORKLOADS[name]
    L = W.nlevels
    H = dm.Hierarchy(ctx, W.theta(), load_m0(name), W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed)
    t0 = time.perf_counter()
    Dc = dm.Deflation(H, L, W.k_defl, eig_rtol=1e-9)
    t_coarse = time.perf_counter() - t0
    H.set_deflation(Dc)  # the difference-level eigensolves use the deflated coarsest solve
    coarsest = "deflated fixed-count GMRES"
    try:  # the measured configuration's coarsest solve, where the level allows it
        H.coarsest_direct(Dc, dm.DIRECT_FP16)
        coarsest = "explicit inverse applied in complex FP16"
    except dm.DmlmcError:
        pass
    out = {"workload": name, "eps": eps, "k_coarsest": W.k_defl, "k_difference": kdiff,
           "coarsest_eigensolve_s": t_coarse, "coarsest_solve": coarsest, "variants": {}}
    for skip in ((), (2,)):
        b = 3 if skip else 2
        for defl in ((False, True) if diff else (False,)):
            label = ("skip2" if skip else "all_levels") + ("+diff_defl" if defl else "")
            td = 0.0
            term = [None] * L
            if defl:
                t0 = time.perf_counter()
                dd = dm.Deflation(H, 1, kdiff, eig_rtol=1e-9, level_b=b, solve_rtol=1e-12, prec=dm.MIXED)
                td = time.perf_counter() - t0
                term[0] = dd
            dm.mlmc_trace(H, Dc, eps, W.noise_seed, [W.n0] * L, W.rhs_block, prec=dm.MIXED, rtol=W.rtol,
                          skip=skip, term_defl=term)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = dm.mlmc_trace(H, Dc, eps, W.noise_seed, [W.n0] * L, W.rhs_block, prec=dm.MIXED, rtol=W.rtol,
                              skip=skip, term_defl=term)
            torch.cuda.synchronize()
            te = time.perf_counter() - t0
            out["variants"][label] = {"trace_s": te, "difference_eigensolve_s": td, "trace": r.trace,
                                      "rel_err": r.rel_err, "N": r.N, "var": r.var}
            log(f"method {label}: {te:.3f} s (+{td:.2f} s eigensolve) trace {r.trace:.4f} rel_err "
                f"{r.rel_err:.2e} N {r.N}")
    # plain Hutchinson at the fine level with exact deflation (Table 1's comparison rows)
    for kf in hutch_k:
        log(f"method hutchinson_exact_k{kf}: fine-level eigensolve")
        t0 = time.perf_counter()
        Df = dm.Deflation(H, 1, kf, eig_rtol=1e-9)
        tf = time.perf_counter() - t0
        kw = dict(prec=dm.MIXED, rtol=W.rtol, max_samples=1 << 15, coarsest=Dc)
        dm.hutchinson_trace(H, Df, eps, W.noise_seed, W.n0, W.rhs_block, **kw)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = dm.hutchinson_trace(H, Df, eps, W.noise_seed, W.n0, W.rhs_block, **kw)
        torch.cuda.synchronize()
        te = time.perf_counter() - t0
        label = f"hutchinson_exact_k{kf}"
        out["variants"][label] = {"trace_s": te, "fine_eigensolve_s": tf, "trace": r.trace, "rel_err": r.rel_err,
                                  "N": r.N, "var": r.var, "tr_defl": r.tr_defl}
        log(f"method {label}: {te:.3f} s (+{tf:.2f} s eigensolve) trace {r.trace:.4f} rel_err {r.rel_err:.2e} "
            f"N {r.N}")
        Df.close()
    H.set_deflation(None)
    return out


def gpu_same_sample(torch, dm, ctx, name: str, nsamp: int):
    """The library on the CPU baseline's exact work: the same workload, hierarchy recipe,
    noise indices and sample counts (mixed precision, fixed counts); setup excluded."""
    from paper_2211_15383_amd.inputs import WORKLOADS, load_m0

    W = WORKLOADS[name]
    L = W.nlevels
    H = dm.Hierarchy(ctx, W.theta(), load_m0(name), W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed)
    D = dm.Deflation(H, L, W.k_defl, eig_rtol=1e-9)
    kw = dict(prec=dm.MIXED, rtol=W.rtol, fixed_counts=True)
    dm.mlmc_trace(H, D, 1e-2, W.noise_seed, [nsamp] * L, W.rhs_block, **kw)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dm.mlmc_trace(H, D, 1e-2, W.noise_seed, [nsamp] * L, W.rhs_block, **kw)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    D.close()
    H.close()
    return sec


def cpu_baseline(name: str, nsamp: int):
    """The CPU checker as it stands (direct sparse-LU solves), on the named workload's
    three-level hierarchy, drawing `nsamp` samples per level.  Setup is excluded."""
    import numpy as np

    from oracle import deflation as odfl, mlmc as omlmc, multigrid as omg
    from paper_2211_15383_amd.inputs import WORKLOADS, load_m0

    W = WORKLOADS[name]
    m0 = load_m0(name)
    lv = omg.build_hierarchy(W.theta(), m0, W.aggs, W.ntv, W.n_inv, W.mg_seed)
    d = odfl.deflate(lv[-1].D, lv[-1].gamma5, W.k_defl)
    solver = omlmc.DirectSolver(lv)
    for l in range(1, len(lv) + 1):  # factorisations are setup
        solver.solve(l, np.zeros(lv[l - 1].n))
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):  # one core: the figure reported as cores = 1
        t0 = time.perf_counter()
        for l in range(1, len(lv) + 1):
            omlmc.sample_values(lv, solver, d, W.noise_seed, l, range(nsamp))
        return time.perf_counter() - t0


def cpu_baseline_fullsize(name: str, N, rtol: float):
    """The CPU checker as it stands on the benchmark's own 1024^2 workload, timed on a
    bounded subset and scaled to one estimate with the sample counts N of the GPU run.

    The checker cannot rebuild the library's inverse-iteration hierarchy at this size, so
    it uses the same lattice, mass and aggregation with its Z4 start vectors as test
    vectors (its parity hierarchy).  Timed: one level-2 solve (FGMRES + V-cycle to rtol;
    a level-2 solve occurs in two terms of every sample of levels 1 and 2) and one LU
    solve each at levels 3 and 4 (after their factorisation).  Not timed: the hierarchy,
    every factorisation and V-cycle setup (setup, reported separately), and the level-1 LU
    solves, whose factorisation alone takes minutes; the result is therefore a lower
    bound of the checker's time per estimate."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import multigrid as omg, noise as onoise, solvers
    from paper_2211_15383_amd.inputs import WORKLOADS, load_m0

    W = WORKLOADS[name]
    t0 = time.perf_counter()
    dims = W.level_dims()
    tv = [omg.start_vectors(W.mg_seed, l + 1, n, dims[l][0] * dims[l][1] * dims[l][2]) for l, n in enumerate(W.ntv)]
    lv = omg.build_hierarchy(W.theta(), load_m0(name), W.aggs, W.ntv, 0, W.mg_seed, import_tv=tv)
    t_hier = time.perf_counter() - t0
    L = len(lv)
    hs = solvers.HybridSolver(lv, rtol=rtol)
    t0 = time.perf_counter()
    for l in range(2, L + 1):
        hs.prepare(l)
    t_prep = time.perf_counter() - t0
    per_solve = {}
    for l in range(2, L + 1):
        x = onoise.z2_noise(W.noise_seed, l, 0, lv[l - 1].n).astype(np.complex128)
        t0 = time.perf_counter()
        hs.solve(l, x)
        per_solve[l] = time.perf_counter() - t0
        log(f"cpu baseline 1024^2: one level-{l} solve {per_solve[l]:.2f} s")
    # sample l < L solves on levels l and l + 1; the coarsest sample on level L
    per_sample = {l: per_solve.get(l, 0.0) + (per_solve[l + 1] if l < L else 0.0) for l in range(1, L + 1)}
    est = sum(N[l - 1] * per_sample[l] for l in range(1, L + 1))
    threads = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    return {"value": est, "unit": "s", "cores": threads, "kind": "oracle",
            "sample": f"{name}: one level-2 FGMRES+V-cycle solve to {rtol:g} and one LU solve at levels 3 and 4, "
                      f"timed on the parity hierarchy (Z4 test vectors) and scaled to one estimate with "
                      f"N = {list(N)}; level-1 solves and all setup excluded (lower bound)",
            "per_solve_s": per_solve, "setup_s": {"hierarchy": t_hier, "factorisations_and_vcycle": t_prep},
            "cpu_model": _cpu_model()}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="schwinger1024")
    ap.add_argument("--direct", choices=("fp16", "fp32", "fp8", "off"), default="fp16",
                    help="coarsest solve inside the complex-FP32 V-cycles: explicit inverse applied in "
                         "FP16, FP32 or the 8-bit form, or the iterative deflated GMRES")
    ap.add_argument("--skip-fp64", action="store_true", help="skip the FP64 single-RHS baseline run")
    ap.add_argument("--skip-cpu", action="store_true", help="skip the CPU checker baselines")
    ap.add_argument("--skip-direct-off", action="store_true",
                    help="skip the estimate with the iterative coarsest solve (no explicit inverse)")
    ap.add_argument("--converge-eps", type=float, default=1e-4,
                    help="tolerance of the extra convergence run, where the stopping rule sets N (0: skip)")
    ap.add_argument("--cpu-workload", default="schwinger128")
    ap.add_argument("--cpu-samples", type=int, default=128, help="samples per level of the CPU baseline")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the built-in launch rule of every kernel (skip the launch-variant autotuner)")
    ap.add_argument("--tune-cache", default=None, metavar="FILE",
                    help="launch-variant choices: read from FILE if it holds them, else tuned and written there "
                         "(profiler runs of the same build then launch the same kernels)")
    ap.add_argument("--skip-kernel-rates", action="store_true",
                    help="skip the per-kernel runs at the real shapes after the timed steps")
    ap.add_argument("--kernels-only", action="store_true",
                    help="after the setup, only run each hot kernel alone at the workload's shapes (stencil, "
                         "transfers, smoothers on levels 1-2, deflation products, coarsest apply) and print "
                         "their timings: a short program for profiler counter runs")
    ap.add_argument("--methods", default=None, metavar="WORKLOAD",
                    help="also time plain / skipped-level / difference-deflated MGMLMC on WORKLOAD")
    ap.add_argument("--methods-eps", type=float, default=1e-3)
    ap.add_argument("--methods-k", type=int, default=8)
    ap.add_argument("--methods-no-diff", action="store_true",
                    help="leave out the variants with a deflated difference term in --methods")
    ap.add_argument("--methods-hutch-k", default="", help="comma-separated fine-level deflation sizes for the "
                    "deflated plain Hutchinson rows of --methods")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the estimator's samples would shard across GPUs with one "
              f"all-reduce of a few doubles per level, but only --gpus 1 is built and measured "
              f"(got --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2211_15383_amd import dmlmc
    from paper_2211_15383_amd.inputs import WORKLOADS, load_m0

    W = WORKLOADS[args.workload]
    m0 = load_m0(W.name)
    L = W.nlevels
    ctx = dmlmc.Context(0)
    log(f"workload {W.name}: {W.Lx}x{W.Lt}, levels {L}, m0 {m0:.6f}, k {W.k_defl}")
    t0 = time.perf_counter()
    H = dmlmc.Hierarchy(ctx, W.theta(), m0, W.aggs, W.ntv, n_inv=W.n_inv, seed=W.mg_seed)
    torch.cuda.synchronize()
    t_hier = time.perf_counter() - t0
    log(f"hierarchy built in {t_hier:.2f} s: levels {[H.level_info(l) for l in range(1, L + 1)]}")
    t0 = time.perf_counter()
    D = dmlmc.Deflation(H, L, W.k_defl, eig_rtol=1e-9)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    log(f"deflation k={W.k_defl} in {t_eig:.2f} s, tr_defl {D.tr_defl:.6f}, {D.info()}")
    t0 = time.perf_counter()
    direct_mode = {"fp16": dmlmc.DIRECT_FP16, "fp32": dmlmc.DIRECT_FP32, "fp8": dmlmc.DIRECT_FP8,
                   "off": dmlmc.DIRECT_OFF}[args.direct]
    if direct_mode != dmlmc.DIRECT_OFF:  # explicit coarsest inverse for the complex-FP32 coarsest solves
        H.coarsest_direct(D, direct_mode)
    torch.cuda.synchronize()
    t_inv = time.perf_counter() - t0
    log(f"coarsest inverse (n = {H.n(L)}, {args.direct}) in {t_inv:.2f} s")
    tuned = None
    t_tune = 0.0
    if not args.no_tune:
        t0 = time.perf_counter()
        picks = H.tune_kernels(W.rhs_block, reps=10, cache_path=args.tune_cache)
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t0
        tuned = {f"level{l}_{k}": {"value": v, "us": round(bu, 2), "rule_us": round(du, 2)}
                 for (l, k), (v, bu, du) in sorted(picks.items())}
        log(f"kernel variants tuned in {t_tune:.2f} s: "
            + ", ".join(f"L{l} {k}={v} ({du:.1f} -> {bu:.1f} us)" for (l, k), (v, bu, du) in sorted(picks.items())))

    if args.kernels_only:
        copy_gbps = copy_ceiling(torch)  # also the profiler's calibration: 1 GiB read + 1 GiB written
        kr = kernel_rates(torch, dmlmc, ctx, H, min(L, 3), W.rhs_block)
        kr.update(matrix_core_rates(torch, dmlmc, ctx, H, D, L, W.rhs_block))
        kr["copy_1GiB"] = {"GBps": copy_gbps, "avg_us": 2 * (1 << 30) / copy_gbps / 1e3}
        for k, v in kr.items():
            log(f"kernel {k}: {v['avg_us']:.1f} us")
        print(json.dumps({"workload": W.name, "kernels": kr}), flush=True)
        return

    n0 = [W.n0] * L

    def run(prec, block):
        return dmlmc.mlmc_trace(H, D, W.eps, W.noise_seed, n0, block, prec=prec, rtol=W.rtol)

    for i in range(args.warmup):
        r = run(dmlmc.MIXED, W.rhs_block)
        log(f"warmup {i}: trace {r.trace:.4f} rel_err {r.rel_err:.3e} N {r.N} in {r.seconds:.3f} s")

    # breakdown pass (untimed): events around every launch of every kernel class
    ctx.timing_select(None)
    ctx.timing(True)
    ctx.timing_reset()
    r = run(dmlmc.MIXED, W.rhs_block)
    tb = timers(ctx, HBM_CLASSES + ("gs_fused", "defl_gemm", "coarse_direct"))
    ctx.timing(False)
    log(f"breakdown pass: {r.seconds:.3f} s (all kernel classes bracketed by events)")
    dom = max(HBM_CLASSES, key=lambda c: tb[c]["ms"])

    # timed steps: no events, so every complex-FP32 FGMRES iteration after the first two of
    # each shape is replayed from its recorded HIP graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        r = run(dmlmc.MIXED, W.rhs_block)
        results.append(r)
        log(f"step {i}: trace {r.trace:.4f} rel_err {r.rel_err:.3e} N {r.N} iters {r.iters} "
            f"level s {[round(c, 3) for c in r.cost_s]}")
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.steps

    # roofline pass: the same steps again with events around the dominant class only (runs
    # with events launch directly instead of replaying graphs)
    ctx.timing_select([dom])
    ctx.timing(True)
    ctx.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        run(dmlmc.MIXED, W.rhs_block)
    torch.cuda.synchronize()
    t_events = (time.perf_counter() - t0) / args.steps
    tm = timers(ctx, (dom,))
    ctx.timing(False)
    ctx.timing_select(None)
    log(f"roofline pass: {t_events:.3f} s per estimate with events around {dom}")

    conv = None
    if args.converge_eps > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = dmlmc.mlmc_trace(H, D, args.converge_eps, W.noise_seed, n0, W.rhs_block, prec=dmlmc.MIXED,
                              rtol=W.rtol)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        conv = {"eps": args.converge_eps, "seconds": tc, "N": rc.N, "rel_err": rc.rel_err, "trace": rc.trace,
                "level_seconds": rc.cost_s}
        log(f"convergence run eps {args.converge_eps:g}: {tc:.3f} s, N {rc.N}, rel_err {rc.rel_err:.3e}")
    copy_gbps = copy_ceiling(torch)
    log(f"copy kernel ceiling {copy_gbps:.0f} GB/s")
    kr = {} if args.skip_kernel_rates else kernel_rates(torch, dmlmc, ctx, H, min(L, 3), W.rhs_block)
    for k, v in kr.items():
        log(f"kernel {k}: {v['avg_us']:.1f} us, {v['GBps']:.0f} GB/s")
    kr_bytes = sum(v["bytes_per_launch"] * v["launches"] for v in kr.values())
    kr_s = sum(v["avg_us"] * 1e-6 * v["launches"] for v in kr.values())
    stencil_real_gbps = kr_bytes / kr_s / 1e9 if kr_s > 0 else 0.0

    fp64 = None
    if not args.skip_fp64:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r64 = run(dmlmc.FP64, 1)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        log(f"fp64 single-RHS: trace {r64.trace:.4f} rel_err {r64.rel_err:.3e} N {r64.N} in {t64:.2f} s")
        rel = abs(r64.trace - results[-1].trace) / abs(r64.trace)
        fp64 = {"seconds": t64, "trace": r64.trace, "N": r64.N, "trace_rel_diff_vs_mixed": rel,
                "level_seconds": r64.cost_s}
        if conv is not None:
            # the FP64 single-RHS time of the convergence run's counts, from its per-sample
            # time per level in the run above (not measured)
            conv["fp64_single_rhs_s_extrapolated"] = sum(
                r64.cost_s[l] / r64.N[l] * conv["N"][l] for l in range(L))

    direct_off = None
    if direct_mode != dmlmc.DIRECT_OFF and not args.skip_direct_off:
        H.coarsest_direct(D, dmlmc.DIRECT_OFF)  # frees the inverse: done after every run that uses it
        run(dmlmc.MIXED, W.rhs_block)  # warm-up: records the graphs of this configuration
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps_off = max(1, min(args.steps, 3))
        for _ in range(steps_off):
            r_off = run(dmlmc.MIXED, W.rhs_block)
        torch.cuda.synchronize()
        t_off = (time.perf_counter() - t0) / steps_off
        gain = t_off - t_mixed
        direct_off = {"seconds": t_off, "coarsest_solve": "deflated fixed-count GMRES", "iters": r_off.iters,
                      "trace_rel_diff_vs_direct": abs(r_off.trace - results[-1].trace) / abs(r_off.trace),
                      "inverse_setup_s": t_inv, "saving_per_estimate_s": gain,
                      "break_even_estimates": (t_inv / gain) if gain > 0 else None}
        log(f"iterative coarsest solve: {t_off:.3f} s per estimate (iters {r_off.iters}); the explicit inverse "
            f"saves {gain:.3f} s per estimate against {t_inv:.2f} s of setup")

    # dominant HBM-bound kernel class, measured inside the timed region
    d = tm[dom]
    avg_ms = d["ms"] / max(1, d["launches"])
    avg_bytes = d["bytes"] / max(1, d["launches"])
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic, traffic_src = recorded_traffic(dom, avg_bytes)
    st_bytes = sum(tb[c]["bytes"] for c in STENCIL_CLASSES)
    st_ms = sum(tb[c]["ms"] for c in STENCIL_CLASSES)
    stencil_gbps = st_bytes / (st_ms * 1e-3) / 1e9 if st_ms > 0 else 0.0
    g = tb["defl_gemm"]
    gemm_tflops = g["bytes"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else 0.0
    cdm = tb["coarse_direct"]
    direct_tflops = cdm["bytes"] / (cdm["ms"] * 1e-3) / 1e12 if cdm["ms"] > 0 else None
    c16 = tb["coarse_direct16"]
    direct16_gbps = c16["bytes"] / (c16["ms"] * 1e-3) / 1e9 if c16["ms"] > 0 else None

    methods = None
    if args.methods:
        ctx.verbose(1)  # the eigensolves of large deflations print one line per iteration
        hk = tuple(int(v) for v in args.methods_hutch_k.split(",") if v.strip())
        methods = method_comparison(torch, dmlmc, ctx, args.methods, args.methods_eps, args.methods_k, hk,
                                    diff=not args.methods_no_diff)

    cpu = cpu128 = None
    if not args.skip_cpu:
        log(f"cpu baseline: checker on {W.name}, bounded subset")
        cpu = cpu_baseline_fullsize(W.name, results[-1].N, W.rtol)
        log(f"cpu baseline {W.name}: >= {cpu['value']:.1f} s per estimate (extrapolated)")
        nsamp = args.cpu_samples
        log(f"cpu baseline: checker on {args.cpu_workload}, {nsamp} samples per level")
        sec = cpu_baseline(args.cpu_workload, nsamp)
        gsec = gpu_same_sample(torch, dmlmc, ctx, args.cpu_workload, nsamp)
        cpu128 = {"value": sec, "unit": "s", "cores": 1, "kind": "oracle",
                  "sample": f"{args.cpu_workload} (128^2, 3 levels, k=32): {nsamp} samples per level with "
                            f"direct sparse-LU solves, setup excluded, measured in full",
                  "gpu_same_sample_s": gsec}
        log(f"cpu baseline {args.cpu_workload} {sec:.2f} s; the GPU on the same samples {gsec:.3f} s")

    coarsest = {"fp16": "explicit inverse applied in complex FP16 (FP32 accumulation)",
                "fp32": "explicit inverse applied in complex FP32",
                "fp8": "explicit inverse applied from an 8-bit (E4M3, row-scaled) copy (FP32 accumulation)",
                "off": "deflated fixed-count GMRES"}[args.direct]
    out = {
        "metric": METRIC,
        "value": t_mixed,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64 (complex-FP16 operands: coarse Gauss-Seidel blocks, coarsest inverse)",
        "data": "synthetic",
        "config": {"workload": f"{W.name}: {W.Lx}x{W.Lt} Wilson-Schwinger, 4 levels (4x4,4x4,2x2 aggregates, "
                               f"8 tv/chirality), k={W.k_defl} coarsest deflation, coarsest solve {coarsest}, "
                               f"eps={W.eps}, rtol={W.rtol}, "
                               f"{W.n0} initial samples/level, RHS block {W.rhs_block}",
                   "m0": m0, "setup_hierarchy_s": t_hier, "setup_eigensolve_s": t_eig,
                   "setup_coarsest_inverse_s": t_inv, "setup_kernel_tuning_s": t_tune, "kernel_variants": tuned,
                   "coarsest_solve": coarsest,
                   "precision": "complex FP32 V-cycles, operators and Krylov basis inside FP64 refinement "
                                "(FP64 Arnoldi, residuals and sample dots); the coarse Gauss-Seidel blocks and "
                                "the coarsest inverse are read as complex FP16 (FP32 accumulation)",
                   "graphs": "timed steps replay recorded HIP graphs (no events in them)"},
        "estimate_with_events_s": t_events,
        "fp64_single_rhs_s": fp64["seconds"] if fp64 else None,
        "speedup_vs_fp64": (fp64["seconds"] / t_mixed) if fp64 else None,
        "fp64_run": fp64,
        "setup_plus_trace_s": {
            "mixed": t_hier + t_eig + t_inv + t_tune + t_mixed,
            "fp64_single_rhs": (t_hier + t_eig + fp64["seconds"]) if fp64 else None,
            "mixed_only_setup": {"coarsest_inverse_s": t_inv, "kernel_tuning_s": t_tune},
            "shared_setup": {"hierarchy_s": t_hier, "eigensolve_s": t_eig},
            "speedup": ((t_hier + t_eig + fp64["seconds"]) / (t_hier + t_eig + t_inv + t_tune + t_mixed)) if fp64 else None,
        },
        "direct_off": direct_off,
        "convergence_run": conv,
        "trace": results[-1].trace,
        "rel_err": results[-1].rel_err,
        "N": results[-1].N,
        "stencil_hbm_GBps": stencil_real_gbps,
        "stencil_hbm_frac": stencil_real_gbps / HBM_PEAK_GBPS,
        "stencil_kernels": kr,
        "stencil_hbm_GBps_in_estimate": stencil_gbps,
        "kernel_classes": tb,
        "defl_gemm_TFLOPs": gemm_tflops,
        "coarse_direct_TFLOPs": direct_tflops,
        "coarse_direct_frac_fp32_mfma": direct_tflops / FP32_MFMA_PEAK_TFLOPS if direct_tflops else None,
        "coarse_direct16_GBps": direct16_gbps,
        "coarse_direct16_frac_hbm": direct16_gbps / HBM_PEAK_GBPS if direct16_gbps else None,
        "copy_kernel_GBps": copy_gbps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel_class": dom, "launches": d["launches"], "avg_launch_ms": avg_ms,
                     "algorithmic_bytes_per_launch": avg_bytes, "traffic_summary": traffic_src},
        "cpu_baseline": cpu,
        "cpu_baseline_128": cpu128,
    }
    if methods is not None:
        out["methods"] = methods
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
