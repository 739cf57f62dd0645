"""Benchmark: factor + solve throughput of the MI355X block-tridiagonal SPD solver.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

One step is one bds_factor (recursive factorisation, the paper's Alg. 4) plus
one bds_solve (recursive solve, Alg. 5-7) of all d right-hand sides, with the
inputs resident in device memory.  Workspaces are allocated once before the
timed region (the paper's "Init" phase, which it also leaves out of its
totals).  Prints one JSON line.

Workloads (seeded synthetic inputs, see paper_2509_03015_amd/inputs.py):
  fp64     plain FP64, N=16384, n=128, d=16, block diagonally dominant
           (A_ii = G G^T/n + 5I, A_{i+1,i} ~ N(0,1)/sqrt(n)); the default.
  f32-k1e4 FP32 factor + FP64 refinement, N=16384, n=256, d=1, Kalman-smoother
           Hessian at kappa ~ 1e4 (likewise f32-k1e2, f32-k1e6, f64-k1e4 ...).
  kalman-neuro  the paper's smoothing example, FP64: latent n=256, m=1024
           observations, N=100 steps, measurement right-hand side; the error
           field is the relative residual and vs_baseline compares with the
           paper's factor + solve time (13.3 + 8.6 ms on its GPU).

The "roofline" object is for the kernel with the largest share of the step,
timed live with HIP events through the library's bds_trace_* calls; its
algorithmic flops and bytes come from the per-kernel model below, enumerated
over the reduction levels.  "cpu_baseline" times the CPU oracle (single
thread, plain C) on a leading sub-chain of the same system and scales it to
the whole workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "factor+solve solves/s and TFLOP/s vs plain FP64 at rel. error ≤1e-10, 1 GPU"
# the paper's factor + solve time (ms) for its smoothing example (N=100, n=256, m=1024, FP64)
PAPER_NEURO_MS = 13.3 + 8.6

# MI355X published peaks.
PEAK = {"hbm": 8000.0,                                   # GB/s
        "mfma_f64": 78.6, "mfma_f32": 157.3, "mfma_bf16": 2500.0}  # TFLOP/s

WORKLOADS = {
    "fp64": dict(kind="dd", N=16384, n=128, d=16, prec="f64"),
    # mixed precision refines to an estimated relative error of 1e-11, a factor 10
    # inside the metric's 1e-10
    "f32-k1e2": dict(kind="kalman", N=16384, n=256, d=1, prec="f32", kappa=1e2, refine_tol=1e-11),
    "f32-k1e4": dict(kind="kalman", N=16384, n=256, d=1, prec="f32", kappa=1e4, refine_tol=1e-11),
    "f32-k1e6": dict(kind="kalman", N=16384, n=256, d=1, prec="f32", kappa=1e6, refine_tol=1e-11),
    "f64-k1e2": dict(kind="kalman", N=16384, n=256, d=1, prec="f64", kappa=1e2),
    "f64-k1e4": dict(kind="kalman", N=16384, n=256, d=1, prec="f64", kappa=1e4),
    "f64-k1e6": dict(kind="kalman", N=16384, n=256, d=1, prec="f64", kappa=1e6),
    "bf16-k1e2": dict(kind="kalman", N=16384, n=256, d=1, prec="bf16", kappa=1e2, refine_tol=1e-11),
    # the small case: N=64, n=16, d=1, plain FP64 (latency-bound)
    "tiny": dict(kind="dd", N=64, n=16, d=1, prec="f64"),
    # many uneven systems, one launch per kernel and level: K=512, N~U{32..2048},
    # n in {8,16,32,64}, d in {1,4}; one step factorises and solves all of them
    "batched": dict(kind="batched", K=512, prec="f64"),
    "batched-f32": dict(kind="batched", K=512, prec="f32", refine_tol=1e-11),
    # differentiation: factor + solve + adjoint (dA, dB of sum(W*X)), Kalman kappa~1e4
    "adjoint": dict(kind="kalman", N=4096, n=32, d=4, prec="f64", kappa=1e4, adjoint=True),
    # the paper's smoothing example: latent n=256, m=1024 observations, N=100 steps, measurement right-hand side
    "kalman-neuro": dict(kind="neuro", N=100, n=256, d=1, m=1024, prec="f64"),
}


def levels(N: int, nstar: int):
    """Block counts M of the reduction levels (odd positions eliminated) and the coarse size."""
    Ms = []
    M = N
    while M > nstar:
        Ms.append(M)
        M = (M + 1) // 2
    return Ms, M


def kernel_model(N: int, n: int, d: int, nstar: int, esize: int):
    """Algorithmic flops and HBM bytes per step of each kernel.

    Per interior block (E = M // 2 per level), with n x n blocks of esize bytes:
      fac_diag    potrf n^3/3 + triangular inverse n^3/3; reads the lower
                  triangle of A_ii, writes L^-1 (lower):        n^2 * esize
      fac_couple  two triangular x dense products, n^3 each; reads L^-1 (half)
                  and both coupling blocks, writes both solved couplings
      fac_schur   per separator: two symmetric rank-n updates (n^3 each, lower
                  half); reads A_jj (half) and two solved couplings, writes
                  the next level's diagonal block (half)
      fac_schur_off  per inner separator pair: one product 2 n^3; reads two
                  solved couplings, writes the next level's coupling block
      sol_fwd_int L^-1 B_i: n^2 d; reads L^-1 (half) and B_i, writes Y_i
      sol_fwd_sep two products 4 n^2 d; reads 2 couplings, 2 Y, B_j, writes B'_j
      sol_bwd     two products and L^-T: 5 n^2 d; reads 2 couplings, L^-1
                  (half), Y_i, two X, writes X_i and copies a separator
    """
    Ms, Mc = levels(N, nstar)
    nn = n * n
    f, b = {}, {}

    def add(k, fl, by):
        f[k] = f.get(k, 0.0) + fl
        b[k] = b.get(k, 0.0) + by

    v = 8 * n * d  # one FP64 right-hand-side block
    for M in Ms:
        E, Mn = M // 2, (M + 1) // 2
        Er = (M - 1) // 2          # interiors with a right coupling
        add("fac_diag", E * (2.0 / 3.0) * n ** 3, E * nn * esize)
        add("fac_couple", (E + Er) * float(n) ** 3, E * 0.5 * nn * esize + (E + Er) * 2 * nn * esize)
        # diagonal Schur blocks: two lower-half symmetric rank-n updates per separator
        # (one per neighbouring interior, E + Er in all); read A_jj (half) and the two
        # solved couplings, write S_jj (half)
        add("fac_schur", (E + Er) * float(n) ** 3,
            Mn * 0.5 * nn * 8 + (E + Er) * nn * esize + Mn * 0.5 * nn * esize)
        # off-diagonal Schur blocks: one product 2 n^3 per inner separator pair
        add("fac_schur_off", (Mn - 1) * 2.0 * n ** 3, (Mn - 1) * 3 * nn * esize)
        add("sol_fwd_int", E * float(nn) * d, E * (0.5 * nn * esize + 2 * v))
        add("sol_fwd_sep", (E + Er) * 2.0 * nn * d, (E + Er) * (nn * esize + v) + Mn * 2 * v)
        add("sol_bwd", E * float(nn) * d + (E + Er) * 2.0 * nn * d,
            E * (0.5 * nn * esize + 4 * v) + (E + Er) * (nn * esize + v))
    # coarse system, sequential block Cholesky in FP64
    add("coarse_factor", Mc * (7.0 / 3.0) * n ** 3, Mc * 3 * nn * 8)
    add("coarse_solve", Mc * 6.0 * nn * d, Mc * (2 * nn * 8 + 3 * v))
    # one refinement iteration (mixed precision): FP64 residual R = B - A X over all
    # block rows (three n x n by n x d products per row; A read once), and the
    # update X += C with its norms
    add("residual", N * 6.0 * nn * d, (2 * N - 1) * nn * 8 + 3 * N * v)
    add("axpy_norm", N * 4.0 * n * d, 3 * N * v)
    return f, b


# kernels with an algorithmic model (candidates for the roofline entry)
MODELLED_KERNELS = ("fac_diag", "fac_couple", "fac_schur", "fac_schur_off", "coarse_factor", "sol_fwd_int",
                "sol_fwd_sep", "sol_bwd", "coarse_solve", "residual", "axpy_norm")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2509_03015_amd", "csrc", "bds_kernels.hip")


def source_digest() -> str:
    h = hashlib.sha256()
    for name in ("bds_kernels.hip", "bds_device.hpp", "bds_gemm.hpp", "bds_chol.hpp"):
        with open(os.path.join(ROOT, "paper_2509_03015_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it matches the current source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_digest") != source_digest():
        return None
    return rec.get("bytes_per_launch")


def make_inputs(w: dict, seed: int = 0):
    from paper_2509_03015_amd import inputs
    if w["kind"] == "dd":
        return inputs.gen_dd(w["N"], w["n"], w["d"], seed=seed)
    if w["kind"] == "neuro":
        return inputs.gen_kalman_neuro(w["N"], w["n"], w["m"], seed=seed)[:4]
    rho = inputs.KALMAN_RHO[w["n"]][w["kappa"]]
    return inputs.gen_kalman(w["N"], w["n"], w["d"], rho, seed=seed)


def cpu_baseline(Ad, As, B, budget_s: float = 15.0, adjoint: bool = False):
    """Oracle factor + solve (+ adjoint) on the leading sub-chain of Ns blocks, scaled to the full N."""
    import oracle
    N = Ad.shape[0]
    Ns = min(N, 64)
    W = np.ones_like(B)
    while True:
        t0 = time.perf_counter()
        X = oracle.solve(Ad[:Ns], As[:Ns - 1], B[:Ns])
        if adjoint:
            oracle.backward(Ad[:Ns], As[:Ns - 1], X, W[:Ns])
        dt = time.perf_counter() - t0
        if Ns >= N or dt * 2 > budget_s / 2:
            break
        Ns = min(N, Ns * 2)
    full_s = dt / Ns * N
    what = "factor + solve + adjoint" if adjoint else "factor + solve"
    return {"value": 1.0 / full_s, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 block-Cholesky {what} of the leading {Ns} of {N} blocks "
                      f"({dt:.2f} s, one thread), scaled by {N / Ns:g} to the full chain"}


def cpu_baseline_batched(systems, budget_s: float = 15.0):
    """Oracle on the first systems of the batch (OpenMP over systems), scaled to the whole batch."""
    import oracle
    K = len(systems)
    work = [s[0].shape[0] * s[0].shape[1] ** 3 for s in systems]
    k = min(K, 8)
    while True:
        t0 = time.perf_counter()
        _, used = oracle.solve_batched([(s[0], s[1], s[3]) for s in systems[:k]])
        dt = time.perf_counter() - t0
        if k >= K or dt * 2 > budget_s / 2:
            break
        k = min(K, k * 2)
    scale = sum(work) / sum(work[:k])
    return {"value": K / (dt * scale), "unit": "solves/s", "cores": int(used), "kind": "oracle",
            "sample": f"FP64 block-Cholesky factor + solve of the first {k} of {K} systems ({dt:.2f} s, "
                      f"{used} threads over systems), scaled by the work ratio {scale:.2f} (sum of N n^3)"}


def merged_model(models, names):
    """Sum per-system kernel models; fold fac_schur_off into fac_schur where the trace has no
    separate off-diagonal Schur launch (per-wave kernels, batched form)."""
    f, b = {}, {}
    for mf, mb in models:
        for k in mf:
            key = "fac_schur" if (k == "fac_schur_off" and "fac_schur_off" not in names) else k
            f[key] = f.get(key, 0.0) + mf[k]
            b[key] = b.get(key, 0.0) + mb[k]
    return f, b


def timed_steps(torch, stream, step, steps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--nstar", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-trace", action="store_true", help="time without per-kernel events")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (library rule for nstar and tile shapes)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only run a device copy of this size (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path in this build "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_03015_amd import _binding as bb
    from paper_2509_03015_amd import inputs, solver

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    bb.load()

    if args.copy_gib > 0:
        nel = int(args.copy_gib * (1 << 30)) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nel * 8, "copy_bytes_written": nel * 8, "launches": 3}))
        return

    w = WORKLOADS[args.workload]
    kind = w["kind"]
    prec = w["prec"]
    tol = w.get("refine_tol", 0.0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    t_gen = time.perf_counter()
    nstar_eff = args.nstar if args.nstar > 0 else 1
    esize = 8 if prec == "f64" else 4  # factor storage: FP64, else FP32 (BF16 rounds MFMA operands only)

    if kind == "batched":
        systems = inputs.gen_batched(w["K"], seed=0)
        t_gen = time.perf_counter() - t_gen
        Ads = [to(s[0]) for s in systems]
        Ass = [to(s[1]) if s[0].shape[0] > 1 else None for s in systems]
        Bs = [to(s[3]) for s in systems]
        Xs = [torch.empty_like(B) for B in Bs]
        t_init = time.perf_counter()
        F = solver.factor_batched(Ads, Ass, prec=prec, nstar=args.nstar)
        F.solve(Bs, outs=Xs, refine_tol=tol)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t_init
        t_tune = time.perf_counter()
        tuning = None if args.no_tune else {str(k): v for k, v in F.tune(Bs, refine_tol=tol).items()}
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t_tune

        def step():
            F.refactor()
            F.solve(Bs, outs=Xs, refine_tol=tol, check=False)

        def result_error():
            errs = [float(np.linalg.norm(X.cpu().numpy() - s[2]) / np.linalg.norm(s[2])) for X, s in zip(Xs, systems)]
            return max(errs)

        def info_iters():
            return max(int(r["iters"]) for r in F.check("bench"))

        shapes = [(s[0].shape[0], s[0].shape[1], s[3].shape[2]) for s in systems]
        per_step = len(systems)
        config = {"workload": args.workload, "K": len(systems), "N": "U{32..2048}", "n": "{8,16,32,64}",
                  "d": "{1,4}", "prec": prec, "generator": "dd", "nstar": nstar_eff}
    else:
        N, n, d = w["N"], w["n"], w["d"]
        Ad, As, Xt, B = make_inputs(w)
        t_gen = time.perf_counter() - t_gen
        Ad_t, As_t, B_t = to(Ad), to(As), to(B)
        X_t = torch.empty_like(B_t)
        adjoint = w.get("adjoint", False)
        Wt = to(np.random.default_rng(11).standard_normal(B.shape)) if adjoint else None
        t_init = time.perf_counter()
        F = solver.factor(Ad_t, As_t, prec=prec, nstar=args.nstar)
        F.solve(B_t, out=X_t, refine_tol=tol)
        if adjoint:
            F.backward(X_t, Wt)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t_init
        t_tune = time.perf_counter()
        tuning = None if args.no_tune else F.tune(B_t, refine_tol=tol)
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t_tune
        nstar_eff = F.nstar if F.nstar > 0 else nstar_eff

        def step():
            F.refactor()
            F.solve(B_t, out=X_t, refine_tol=tol, check=False)
            if adjoint:
                F.backward(X_t, Wt, check=False)

        def result_error():
            X = X_t.cpu().numpy()
            if kind == "neuro":
                # measurement right-hand side, no manufactured solution: the residual
                # ||A X - B||_2 / ||B||_2, as the paper reports for this example
                return float(np.linalg.norm(inputs.block_matvec(Ad, As, X) - B) / np.linalg.norm(B))
            return float(np.linalg.norm(X - Xt) / np.linalg.norm(Xt))

        def info_iters():
            return max(int(F.check("bench").get("iters", 0)), 0)

        shapes = [(N, n, d)]
        per_step = 1
        config = {"workload": args.workload, "N": N, "n": n, "d": d, "prec": prec, "generator": kind,
                  **({"kappa": w["kappa"]} if "kappa" in w else {}), "nstar": nstar_eff,
                  **({"adjoint": True} if adjoint else {})}
    print(f"[bench] workload {args.workload} ({prec}): inputs {t_gen:.1f} s, init {t_init:.2f} s, "
          f"tune {t_tune:.2f} s -> {tuning}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    # timed region: the library's own launch path (graph replay where it applies)
    stream = torch.cuda.current_stream(dev)
    ms_step, wall = timed_steps(torch, stream, step, args.steps)
    iters = info_iters() if prec != "f64" else 0

    # per-kernel durations (HIP events around every launch, which also makes the
    # library launch kernel by kernel) over a second run of the same steps
    kern, dropped, ms_step_traced = {}, 0, None
    if not args.no_trace:
        bb.trace_enable(args.steps * 65536 if kind == "batched" else args.steps * 4096)
        ms_step_traced, _ = timed_steps(torch, stream, step, args.steps)
        kern, dropped = bb.trace_read()
        bb.trace_enable(0)
    err = result_error()

    flops, bytes_ = merged_model([kernel_model(N_, n_, d_, nstar_eff, esize) for N_, n_, d_ in shapes], set(kern))
    adj = config.get("adjoint", False)
    solves = 1 + iters + (1 if adj else 0)   # the adjoint solves once more with the factor
    tot_flops = sum(flops[k] for k in flops if k.startswith("fac") or k == "coarse_factor") + \
        solves * sum(flops[k] for k in flops if k.startswith("sol") or k == "coarse_solve") + \
        iters * (flops["residual"] + flops["axpy_norm"])

    roof = None
    kernels = {}
    if kern:
        for k, (cnt, ms) in kern.items():
            kernels[k] = {"launches_per_step": cnt / args.steps, "ms_per_step": ms / args.steps}
        timed = {k: v for k, v in kern.items() if k in MODELLED_KERNELS}
        dom = max(timed, key=lambda k: timed[k][1])
        cnt, ms = timed[dom]
        per_step_launches = cnt / args.steps
        avg_ms = ms / cnt
        if dom.startswith("sol") or dom == "coarse_solve":
            mult = solves          # the first solve, one per refinement iteration, the adjoint's
        elif dom in ("residual", "axpy_norm"):
            mult = iters
        else:
            mult = 1
        # the kernel's roofline: MFMA-bound when its arithmetic intensity (algorithmic
        # flops per algorithmic HBM byte) reaches the ridge point peak_flops / peak_bw
        fl = flops[dom] * mult / per_step_launches
        by = bytes_[dom] * mult / per_step_launches
        peak_f, peak_b = PEAK["mfma_" + prec], PEAK["hbm"]
        ridge = peak_f * 1e12 / (peak_b * 1e9)
        bound = "mfma" if by == 0 or fl / by >= ridge else "hbm"
        if bound == "mfma":
            alg, peak, unit = fl, peak_f, "TFLOP/s"
            achieved = alg / (avg_ms * 1e-3) / 1e12
        else:
            alg, peak, unit = by, peak_b, "GB/s"
            achieved = alg / (avg_ms * 1e-3) / 1e9
        roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                "traffic": measured_traffic(dom, args.workload), "kernel": dom,
                "avg_launch_ms": avg_ms, "launches_per_step": per_step_launches,
                "algorithmic_per_launch": alg, "flops_per_launch": fl, "bytes_per_launch": by,
                "arith_intensity": fl / by if by else None, "ridge": ridge,
                "tflops": fl / (avg_ms * 1e-3) / 1e12, "gbps": by / (avg_ms * 1e-3) / 1e9,
                "share_of_step": (ms / args.steps) / ms_step_traced}

    out = {
        "metric": METRIC,
        "value": per_step * 1000.0 / ms_step,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": (per_step * 1000.0 / ms_step) / (1000.0 / PAPER_NEURO_MS)
        if args.workload == "kalman-neuro" else None,
        "dtype": prec,
        "data": "synthetic",
        "config": config,
        "tflops": tot_flops / (ms_step * 1e-3) / 1e12,
        "relerr_vs_manufactured": None if kind == "neuro" else err,
        **({"residual_rel": err} if kind == "neuro" else {}),
        "refine_iters": iters,
        "wall_s_timed": wall,
        "init_s": t_init,
        "tune_s": t_tune,
        "tuning": tuning,
        "roofline": roof,
        "kernels": kernels,
        "ms_per_step_kernel_by_kernel": ms_step_traced,
        "trace_dropped": dropped,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        if kind == "batched":
            out["cpu_baseline"] = cpu_baseline_batched(systems)
        else:
            out["cpu_baseline"] = cpu_baseline(Ad, As, B, adjoint=adj)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
