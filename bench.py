#!/usr/bin/env python3
"""Benchmark of the structured-operator conic solver on one MI355X.

Default workload (`deconv_n1M_k1025`): a *step* is one complete solve of the
large nonnegative deconvolution (n = 2^20 signal, 1025-tap Gaussian kernel,
Section V-C, eq. 6) to the 1e-4 relative KKT tolerance: setup (embedding vector
by CG), then HSDE ADMM steps (CG on I + A^T A with the convolution and its
adjoint, SOC / nonnegative projections, residual checks) until res_pri,
res_dual and gap are <= 1e-4.  Problem data are resident in HBM before the
timed region; each step restarts the iterates on the device.

Other workloads (`--workload`): `deconv_n1000_k101` (FP64, 1e-6),
`lasso_5000x10000` (FP32 dense lasso), `lasso_batch64_2000x8000` (64 lasso
instances sharing A, BF16 MFMA GEMMs; a step solves all 64), and
`serve_deconv_2000req` (replay of the 2000-request Poisson trace through the
continuous-batching server; one step = the whole replay),
`regls_dense_6000x3000` / `regls_conv_3000_k1365` (Section V-A: regularized least
squares by matrix-free CG to the 1e-8 relative residual, FP64; one step = one
solve) and `lasso_conv_3000_k1365` (lasso with the convolution operator).

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-1e-4 KKT residual & CG matvecs/s; batched solves/s, p50/p99 latency"
PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published dense FP32 vector peak
PEAK_FP64_VECTOR_TFLOPS = 78.6    # MI355X published FP64 vector peak
PEAK_BF16_MFMA_TFLOPS = 2500.0    # MI355X dense BF16 matrix peak
PEAK_HBM_GBS = 8000.0             # MI355X HBM3E


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def golden(name):
    """Stored oracle result (tests/golden/reference_objectives.json, written by
    tests/golden/make_reference.py from the oracle only), or None."""
    try:
        return json.load(open(os.path.join(ROOT, "tests", "golden", "reference_objectives.json"))).get(name)
    except (OSError, ValueError):
        return None


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()]))
    except Exception:
        return os.cpu_count()


def timed_solves(s, steps, warmup, label):
    import torch
    for i in range(warmup):
        s.reset()
        info = s.solve()
        log(f"{label} warmup {i}: {info[0]['status_name']} iters={info[0]['iters']} "
            f"cg={info[0]['cg_iters']} t={info[0]['setup_s'] + info[0]['solve_s']:.3f}s")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        s.reset()
        infos.append(s.solve())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if hasattr(s, "rounds"):
        r0, r1 = s.rounds()
        log(f"{label} check intervals since creation: {r0} ({r1} run again with more CG launches)")
    for i, inf in enumerate(infos):
        log(f"{label} step {i}: {inf[0]['status_name']} iters={inf[0]['iters']} cg={inf[0]['cg_iters']} "
            f"res=({inf[0]['res_pri']:.2e},{inf[0]['res_dual']:.2e},{inf[0]['gap']:.2e})")
    return infos, elapsed


def base_record(args, value, unit, elapsed, dtype, config):
    return {
        "metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * elapsed / max(args.steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic", "config": config,
    }


# ---------------------------------------------------------------- deconvolution (single)
def run_deconv(args, cfg):
    import numpy as np
    import torch
    import workloads as w
    import paper_1609_03488_amd as P

    data = w.make_deconv(cfg)
    n, k = cfg["n"], cfg["k"]
    pr = P.deconv_problem(data["c"], data["b"])
    stream = torch.cuda.Stream()
    prec = P.FP64 if cfg["precision"] == "fp64" else P.FP32
    tuned = None
    st = P.Settings.make(precision=prec, eps=cfg["eps"], check_every=10, normalize=args.normalize)
    if args.max_iters:
        st.max_iters = args.max_iters
    s = P.Solver(pr.op, pr.l, pr.q, st, stream=stream)
    s.set_data(0, pr.b, pr.c)
    log(f"workspace {s.workspace_bytes / 2**20:.1f} MiB")
    engine = int(st.conv_mfma) if prec == P.FP32 else 0   # (the settings' default engine)
    if prec == P.FP32 and args.conv_engine is not None:
        engine = args.conv_engine
        s.close()
        st.conv_mfma = engine
        s = P.Solver(pr.op, pr.l, pr.q, st, stream=stream)
        s.set_data(0, pr.b, pr.c)
        log(f"convolution {ENGINE_NAMES[engine]} (fixed)")
    elif prec == P.FP32 and not args.no_autotune:
        tuned = s.autotune(reps=10)
        engine = tuned["conv_mfma"]
        log(f"autotune: convolution {ENGINE_NAMES[engine]}, vector tiles of {tuned['vec_tile']}")
    infos, elapsed = timed_solves(s, args.steps, args.warmup, cfg["name"])
    last = infos[-1][0]
    t_fwd = s.kernel_time(0, 20)
    t_adj = s.kernel_time(1, 20)
    flop_fwd, flop_adj = 2.0 * k * (n + k - 1), 2.0 * k * n
    achieved = (flop_fwd + flop_adj) / ((t_fwd + t_adj) * 1e-3) / 1e12
    log(f"conv A {t_fwd * 1e3:.1f} us, A^T {t_adj * 1e3:.1f} us, {achieved:.1f} TFLOP/s direct-sum rate")
    verify = None
    if not args.no_verify:
        import oracle
        x, y, sl = s.solution(0)
        prog = oracle.deconv_program(data["c"], data["b"])
        rp, rd, gap, _, _ = oracle.scs.residuals(prog, x, y, 1.0, sl)
        f = oracle.deconv_objective(data["c"], data["b"], x[:n])
        noise = float(np.linalg.norm(data["b"] - np.convolve(data["c"], data["x_true"])))
        verify = {"res_pri_fp64": rp, "res_dual_fp64": rd, "gap_fp64": gap, "objective": f,
                  "objective_upper_bound_noise_norm": noise}
        same = golden(cfg["name"] + "_scs")
        if same is not None and same["eps"] == cfg["eps"] and same["normalize"] == args.normalize:
            verify["oracle_objective_same_method_and_eps"] = same["objective"]
            verify["rel_obj_err_vs_oracle"] = abs(f - same["objective"]) / same["objective"]
            verify["oracle_admm_iters"] = same["iters"]
        exact = golden(cfg["name"])
        if exact is not None:
            verify["exact_objective"] = exact["objective"]
            verify["rel_obj_err_vs_exact"] = abs(f - exact["objective"]) / exact["objective"]
        log("verify", verify)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # bounded sample: the same family at n_s <= 2^14 (same kernel, density,
        # noise), factorisation + setup + a few iterations timed; banded
        # factorisation and solves cost O(n k^2) and O(n k), so the time is
        # scaled by n / n_s and to the GPU's iteration count
        n_s = min(n, args.cpu_sample_n)
        if n_s < n:
            ds = w.deconv_instance(n_s, k, cfg["sigma"], cfg["density"], cfg["noise_var"], cfg["seed"])
        else:
            ds = data
        prog = oracle.deconv_program(ds["c"], ds["b"])
        t0 = time.perf_counter()
        fac = oracle.prepare(prog, args.normalize)[0].factor()   # of the scaled operator
        t_factor = time.perf_counter() - t0
        if n_s == n:
            # small enough: the complete oracle solve to the same tolerance
            res = oracle.scs_solve(prog, eps=cfg["eps"], check_every=10, fac=fac, normalize=args.normalize)
            t_solve = t_factor + res.setup_s + res.solve_s
            cpu = {"value": 1.0 / t_solve, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
                   "sample": (f"one complete FP64 banded-Cholesky SCS oracle solve of the same problem "
                              f"to eps {cfg['eps']:g} (normalize {args.normalize}): factorisation "
                              f"{t_factor:.2f} s, {res.iters} ADMM iterations, status {res.status}, "
                              f"{t_solve:.2f} s")}
        else:
            res = oracle.scs_solve(prog, eps=cfg["eps"], max_iters=args.cpu_iters, check_every=10, fac=fac,
                                   normalize=args.normalize)
            t_iter = res.solve_s / max(res.iters, 1)
            scale = n / n_s
            t_solve = scale * (t_factor + res.setup_s + last["iters"] * t_iter)
            cpu = {"value": 1.0 / t_solve, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
                   "sample": (f"FP64 banded-Cholesky SCS oracle on the same family at n = {n_s} "
                              f"(k = {k}): factorisation {t_factor:.1f} s + embedding setup "
                              f"{res.setup_s:.2f} s + {res.iters} ADMM iterations ({t_iter:.3f} s each) "
                              f"timed; x{scale:g} for n = {n} and extrapolated to the GPU's "
                              f"{last['iters']} iterations -> {t_solve:.0f} s per solve")}
        log("cpu", cpu)
    out = base_record(args, args.steps / elapsed, "solves/s", elapsed,
                      "f32" if prec == P.FP32 else "f64",
                      {"workload": cfg["name"], "n": n, "kernel_taps": k, "sigma": cfg["sigma"],
                       "eps": cfg["eps"], "variables": n + 1, "constraints": 2 * n + k,
                       "normalize": args.normalize, "scalars": "f64"})
    out.update({
        "time_to_eps_s": elapsed / args.steps, "admm_iters": last["iters"], "cg_iters": last["cg_iters"],
        "cg_matvecs_per_s": sum(i[0]["cg_iters"] for i in infos) / elapsed,
        "status": last["status_name"], "max_iters_cap": args.max_iters, "autotune": tuned,
        "roofline": conv_roofline(engine, prec == P.FP32, n, k, t_fwd, t_adj),
        "conv_direct_sum_equivalent_tflops": achieved,
        "cpu_baseline": cpu, "verify": verify,
    })
    return out


ENGINE_NAMES = {0: "on the vector ALU", 1: "on the matrix cores", 2: "by FFT (overlap-save)"}


def conv_roofline(engine, fp32, n, k, t_fwd_ms, t_adj_ms):
    """Roofline record of the convolution launches A and A^T (n inputs, k taps).

    Direct engines (vector ALU, matrix cores) are priced by the direct sum's
    2 k n_out flop per launch against the FP32 peak (157.3 TFLOP/s; FP64:
    78.6).  The FFT engine computes the same products with O(log) flops per
    output, so its binding roof is memory: algorithmic bytes per launch = the
    block's input and output, 4 (n + n + k - 1) bytes, against 8 TB/s (the
    direct-sum-equivalent rate is reported outside the roofline record)."""
    flop = {"A": 2.0 * k * (n + k - 1), "AT": 2.0 * k * n}
    us = {"A": t_fwd_ms * 1e3, "AT": t_adj_ms * 1e3}
    direct = (flop["A"] + flop["AT"]) / ((t_fwd_ms + t_adj_ms) * 1e-3) / 1e12
    if engine == 2:
        nbytes = 4.0 * (n + n + k - 1)
        achieved = 2 * nbytes / ((t_fwd_ms + t_adj_ms) * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": measured_traffic("k_conv_fft"),
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": "k_conv_fft (FP32 FFT overlap-save convolution A and its adjoint A^T)",
                "bytes_per_launch": nbytes, "launch_us": us}
    peak = PEAK_FP32_VECTOR_TFLOPS if fp32 else PEAK_FP64_VECTOR_TFLOPS
    return {"bound": "mfma" if engine == 1 else "alu", "achieved": direct, "peak": peak, "unit": "TFLOP/s",
            "frac": direct / peak,
            "traffic": measured_traffic("k_conv_mfma") if engine == 1 else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": ("k_conv_mfma (FP32 matrix-core convolution" if engine == 1 else
                       "k_conv (direct convolution") + " A and its adjoint A^T)",
            "flop_per_launch": flop, "launch_us": us}


def measured_traffic(kernel: str):
    """HBM bytes per launch (mean over the directions) of `kernel` from the
    counter record under profiles/, or None when there is none or the kernel's
    sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        rec = json.load(open(path))[kernel]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        try:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        except OSError:
            return None
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    per = [1024.0 * (rec["fetch_kib"][d] * rec["fetch_scale"] + rec["write_kib"][d] * rec["write_scale"])
           for d in rec["fetch_kib"]]
    return sum(per) / len(per)


# ---------------------------------------------------------------- dense lasso (single)
def run_lasso(args, cfg):
    import numpy as np
    import torch
    import workloads as w
    import paper_1609_03488_amd as P

    data = w.make_lasso(cfg)
    m, n = cfg["m"], cfg["n"]
    pr = P.lasso_problem(data["A"], data["b"], data["lam"])
    stream = torch.cuda.Stream()
    # stop at stop_eps (residuals 1e-5 <= the workload's 1e-4), the setting at
    # which the objective lands within 1e-4 of the optimum
    stop_eps = cfg.get("stop_eps", cfg["eps"])
    st = P.Settings.make(precision=P.FP32, eps=stop_eps, check_every=10, normalize=args.normalize)
    if args.max_iters:
        st.max_iters = args.max_iters
    s = P.Solver(pr.op, pr.l, pr.q, st, stream=stream)
    s.set_data(0, pr.b, pr.c)
    tuned = None
    if not args.no_autotune:
        tuned = s.autotune(reps=5)
        log(f"autotune: vector tiles of {tuned['vec_tile']}")
    infos, elapsed = timed_solves(s, args.steps, args.warmup, cfg["name"])
    last = infos[-1][0]
    t_a, t_at = s.kernel_time(2, 20), s.kernel_time(3, 20)
    bytes_a = 4.0 * m * n
    achieved = 2 * bytes_a / ((t_a + t_at) * 1e-3) / 1e9
    log(f"gemv A {t_a * 1e3:.1f} us, A^T {t_at * 1e3:.1f} us, {achieved:.0f} GB/s")
    verify = None
    import oracle
    prog = oracle.lasso_program(data["A"], data["b"], data["lam"])
    if not args.no_verify:
        x, y, sl = s.solution(0)
        rp, rd, gap, _, _ = oracle.scs.residuals(prog, x, y, 1.0, sl)
        f = oracle.lasso_objective(data["A"], data["b"], data["lam"], x[:n])
        ref = golden(cfg["name"])
        verify = {"res_pri_fp64": rp, "res_dual_fp64": rd, "gap_fp64": gap, "objective": f,
                  "exact_objective": ref["objective"] if ref else None,
                  "rel_obj_err_vs_exact": abs(f - ref["objective"]) / abs(ref["objective"]) if ref else None}
        log("verify", verify)
    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        res = oracle.scs_solve(prog, eps=stop_eps, check_every=10, normalize=args.normalize)
        t = time.perf_counter() - t0
        cpu = {"value": 1.0 / t, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
               "sample": f"complete FP64 oracle solve (dense Cholesky of 3I+4A^T A, {res.iters} ADMM "
                         f"iterations, status {res.status}) in {t:.1f} s"}
        log("cpu", cpu)
    out = base_record(args, args.steps / elapsed, "solves/s", elapsed, "f32",
                      {"workload": cfg["name"], "m": m, "n": n, "eps": cfg["eps"], "stop_eps": stop_eps,
                       "variables": 2 * n + 1, "constraints": 2 * n + m + 2, "normalize": args.normalize, "scalars": "f64"})
    out.update({
        "time_to_eps_s": elapsed / args.steps, "admm_iters": last["iters"], "cg_iters": last["cg_iters"],
        "cg_matvecs_per_s": sum(i[0]["cg_iters"] for i in infos) / elapsed, "status": last["status_name"],
        "autotune": tuned,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": measured_traffic("k_gemv"),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "k_gemv<float> (A and A^T, FP32, 200 MB each; fits the 256 MB MALL)",
                     "bytes_per_launch": bytes_a, "launch_us": {"A": t_a * 1e3, "AT": t_at * 1e3}},
        "cpu_baseline": cpu, "verify": verify,
    })
    return out


# ---------------------------------------------------------------- regularized least squares (CG)
def run_regls(args, cfg):
    import numpy as np
    import torch
    import workloads as w
    import paper_1609_03488_amd as P

    d = w.make_regls(cfg)
    n = cfg["n"]
    stream = torch.cuda.Stream()
    prec = P.FP64 if cfg["precision"] == "fp64" else P.FP32
    if d["kind"] == "dense":
        rs = P.RegLS(d["lam"], A=d["A"], precision=prec, stream=stream)
    else:
        rs = P.RegLS(d["lam"], taps=d["c"], n=n, precision=prec, stream=stream)
    for i in range(args.warmup):
        x, it = rs.solve(d["b"], tol=cfg["tol"])
        log(f"{cfg['name']} warmup {i}: {it} CG iterations")
    torch.cuda.synchronize()
    its = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, it = rs.solve(d["b"], tol=cfg["tol"])
        its.append(it)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"{cfg['name']}: {its} CG iterations, {1e3 * elapsed / args.steps:.2f} ms per solve")
    m = rs.m
    if d["kind"] == "dense":
        t_a, t_at = rs.solver.kernel_time(2, 20), rs.solver.kernel_time(3, 20)
        bytes_a = 8.0 * m * n
        achieved = 2 * bytes_a / ((t_a + t_at) * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                "kernel": f"k_gemv<double> (A and A^T, FP64, {bytes_a / 1e6:.0f} MB each)",
                "bytes_per_launch": bytes_a, "launch_us": {"A": t_a * 1e3, "AT": t_at * 1e3}}
    else:
        k = cfg["k"]
        t_a, t_at = rs.solver.kernel_time(0, 20), rs.solver.kernel_time(1, 20)
        flop_a, flop_at = 2.0 * k * (n + k - 1), 2.0 * k * n
        achieved = (flop_a + flop_at) / ((t_a + t_at) * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_VECTOR_TFLOPS, "traffic": None,
                "kernel": "k_conv<double> (FP64 vector-ALU convolution A and A^T)",
                "flop_per_launch": {"A": flop_a, "AT": flop_at},
                "launch_us": {"A": t_a * 1e3, "AT": t_at * 1e3}}
    log(f"operator A {t_a * 1e3:.1f} us, A^T {t_at * 1e3:.1f} us, {roof['achieved']:.1f} {roof['unit']}")
    import oracle
    verify = None
    if not args.no_verify:
        rhs = oracle.regls_rhs(d)
        ref = oracle.regls_solution(d)
        verify = {"rel_residual_fp64": float(np.linalg.norm(oracle.regls_apply_normal(d, x) - rhs) / np.linalg.norm(rhs)),
                  "rel_err_vs_closed_form": float(np.linalg.norm(x - ref) / np.linalg.norm(ref)),
                  "objective": oracle.regls_objective(d, x)}
        log("verify", verify)
    cpu = None
    if not args.no_cpu_baseline:
        reps, t0 = 0, time.perf_counter()
        while True:
            oracle.regls_solution(d)
            reps += 1
            if time.perf_counter() - t0 > 5.0 or reps >= 50:
                break
        t = (time.perf_counter() - t0) / reps
        cpu = {"value": 1.0 / t, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
               "sample": (f"the oracle's closed form (FP64 {'dense' if d['kind'] == 'dense' else 'banded'} "
                          f"Cholesky of lam I + A^T A and its solve), {reps} repetitions, {t:.3f} s each")}
        log("cpu", cpu)
    cfgout = {"workload": cfg["name"], "n": n, "m": m, "lam": float(d["lam"]), "tol": cfg["tol"],
              "operator": d["kind"]}
    if d["kind"] == "conv":
        cfgout["kernel_taps"] = cfg["k"]
    out = base_record(args, args.steps / elapsed, "solves/s", elapsed,
                      "f64" if prec == P.FP64 else "f32", cfgout)
    out.update({"time_to_tol_s": elapsed / args.steps, "cg_iters": its[-1],
                "cg_matvecs_per_s": sum(its) / elapsed, "roofline": roof, "cpu_baseline": cpu,
                "verify": verify})
    rs.close()
    return out


# ---------------------------------------------------------------- lasso with a convolution operator
def run_lasso_conv(args, cfg):
    import numpy as np
    import torch
    import workloads as w
    import paper_1609_03488_amd as P

    d = w.make_conv_lasso(cfg)
    n, k = cfg["n"], cfg["k"]
    pr = P.conv_lasso_problem(d["c"], d["b"], d["lam"])
    stream = torch.cuda.Stream()
    st = P.Settings.make(precision=P.FP32, eps=cfg["eps"], check_every=10, normalize=args.normalize)
    if args.max_iters:
        st.max_iters = args.max_iters
    s = P.Solver(pr.op, pr.l, pr.q, st, stream=stream)
    s.set_data(0, pr.b, pr.c)
    engine = 1
    tuned = None
    if not args.no_autotune:
        tuned = s.autotune(reps=10)
        engine = tuned["conv_mfma"]
        log(f"autotune: convolution {ENGINE_NAMES[engine]}, vector tiles of {tuned['vec_tile']}")
    infos, elapsed = timed_solves(s, args.steps, args.warmup, cfg["name"])
    last = infos[-1][0]
    t_a, t_at = s.kernel_time(0, 20), s.kernel_time(1, 20)
    roof = conv_roofline(engine, True, n, k, t_a, t_at)
    log(f"conv A {t_a * 1e3:.1f} us, A^T {t_at * 1e3:.1f} us, {roof['achieved']:.1f} {roof['unit']}")
    import oracle
    prog = oracle.conv_lasso_program(d["c"], d["b"], d["lam"])
    verify = None
    if not args.no_verify:
        x, y, sl = s.solution(0)
        rp, rd, gap, _, _ = oracle.scs.residuals(prog, x, y, 1.0, sl)
        xs = x[:n]
        r = np.convolve(d["c"], xs) - d["b"]
        f = float(0.5 * (r @ r) + d["lam"] * np.sum(np.abs(xs)))
        verify = {"res_pri_fp64": rp, "res_dual_fp64": rd, "gap_fp64": gap, "objective": f}
        log("verify", verify)
    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        res = oracle.scs_solve(prog, eps=cfg["eps"], check_every=10, normalize=args.normalize)
        t = time.perf_counter() - t0
        cpu = {"value": 1.0 / t, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
               "sample": f"complete FP64 oracle solve (banded Cholesky of 3I+4C^T C, {res.iters} ADMM "
                         f"iterations, status {res.status}) in {t:.1f} s"}
        log("cpu", cpu)
    out = base_record(args, args.steps / elapsed, "solves/s", elapsed, "f32",
                      {"workload": cfg["name"], "n": n, "kernel_taps": k, "eps": cfg["eps"],
                       "variables": 2 * n + 1, "constraints": 2 * n + (n + k - 1) + 2,
                       "normalize": args.normalize, "scalars": "f64"})
    out.update({
        "time_to_eps_s": elapsed / args.steps, "admm_iters": last["iters"], "cg_iters": last["cg_iters"],
        "cg_matvecs_per_s": sum(i[0]["cg_iters"] for i in infos) / elapsed, "status": last["status_name"],
        "autotune": tuned, "roofline": roof,
        "cpu_baseline": cpu, "verify": verify,
    })
    return out


# ---------------------------------------------------------------- batched lasso (BF16 MFMA)
def run_lasso_batch(args, cfg):
    import numpy as np
    import torch
    import workloads as w
    import paper_1609_03488_amd as P

    data = w.make_lasso_batch(cfg)
    m, n, B = cfg["m"], cfg["n"], cfg["batch"]
    prs = [P.lasso_problem(data["A"], data["b"][i], data["lam"][i]) for i in range(B)]
    stream = torch.cuda.Stream()
    # stop at stop_eps (residuals 1e-5 <= the workload's 1e-4), the setting at
    # which every instance's objective lands within 1e-4 of its optimum
    stop_eps = cfg.get("stop_eps", cfg["eps"])
    st = P.Settings.make(precision=P.BF16, eps=stop_eps, check_every=10, normalize=args.normalize)
    s = P.Solver(prs[0].op, prs[0].l, prs[0].q, st, batch=B, stream=stream)
    for i, pr in enumerate(prs):
        s.set_data(i, pr.b, pr.c)
    tuned = None
    if not args.no_autotune:
        tuned = s.autotune(reps=10)
        log(f"autotune: batched GEMM aims at {tuned['gemm_target_wgs']} workgroups, "
            f"vector tiles of {tuned['vec_tile']}")
    infos, elapsed = timed_solves(s, args.steps, args.warmup, cfg["name"])
    # the applies timed while the GPU is still busy from the solves (after the
    # host-side checks below its clocks would have dropped)
    s.kernel_time(2, 2), s.kernel_time(3, 2)
    gem = s.kernel_time(2, 20), s.kernel_time(3, 20)
    last = infos[-1]
    solves = B * args.steps
    verify = None
    import oracle
    if not args.no_verify:
        # every instance: residuals recomputed in FP64 and the objective against
        # its stored optimum
        worst, worst_obj = 0.0, 0.0
        refs = golden(cfg["name"]) or {}
        statuses = [inf["status_name"] for inf in last]
        for i in range(B):
            prog = oracle.lasso_program(data["A"], data["b"][i], data["lam"][i])
            x, y, sl = s.solution(i)
            rp, rd, gap, _, _ = oracle.scs.residuals(prog, x, y, 1.0, sl)
            worst = max(worst, rp, rd, gap)
            if str(i) in refs:
                f = oracle.lasso_objective(data["A"], data["b"][i], data["lam"][i], x[:n])
                worst_obj = max(worst_obj, abs(f - refs[str(i)]["objective"]) / refs[str(i)]["objective"])
        verify = {"worst_kkt_fp64": worst, "instances_checked": B,
                  "worst_rel_obj_err_vs_exact": worst_obj if refs else None,
                  "instances_with_exact_reference": len(refs),
                  "statuses": sorted(set(statuses)),
                  "certified_by_operator": sorted({{0: "fp64", 1: "fp32", 2: "bf16"}[inf["cert_precision"]]
                                                   for inf in last})}
        log("verify", verify)
    # plain one-at-a-time FP32 solver on the same instances (sample)
    nplain = min(B, args.plain_sample)
    st32 = P.Settings.make(precision=P.FP32, eps=stop_eps, check_every=10, normalize=args.normalize)
    s1 = P.Solver(prs[0].op, prs[0].l, prs[0].q, st32, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nplain):
        s1.set_data(0, prs[i].b, prs[i].c)
        s1.solve()
    torch.cuda.synchronize()
    plain = nplain / (time.perf_counter() - t0)
    log(f"plain FP32 one-at-a-time: {plain:.2f} solves/s (includes each instance's b/c upload)")
    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        prog = oracle.lasso_program(data["A"], data["b"][0], data["lam"][0])
        fac = oracle.prepare(prog, args.normalize)[0].factor()   # the scaled operator is shared

        tf = time.perf_counter() - t0
        nsamp = min(B, args.cpu_solves)
        t1 = time.perf_counter()
        for i in range(nsamp):
            p_i = oracle.lasso_program(data["A"], data["b"][i], data["lam"][i])
            oracle.scs_solve(p_i, eps=stop_eps, check_every=10, fac=fac, normalize=args.normalize)
        ts = (time.perf_counter() - t1) / nsamp
        cpu = {"value": B / (tf + B * ts), "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
               "sample": f"one shared factorisation ({tf:.1f} s) + {nsamp} of {B} sequential FP64 oracle "
                         f"solves ({ts:.2f} s each), extrapolated to {B}"}
        log("cpu", cpu)
    out = base_record(args, solves / elapsed, "solves/s", elapsed, "bf16",
                      {"workload": cfg["name"], "m": m, "n": n, "batch": B, "eps": cfg["eps"],
                       "stop_eps": stop_eps, "normalize": args.normalize,
                       "products": "bf16 MFMA, fp32 accumulation; refinement phase bf16 hi/lo; "
                                   "final test (and iterations where it fails) on the fp32 operator",
                       "autotune": tuned,
                       "scalars": "f64"})
    out.update({
        "time_per_batch_s": elapsed / args.steps,
        "admm_iters_max": max(i["iters"] for i in last),
        "plain_fp32_one_at_a_time_solves_per_s": plain,
        "speedup_vs_plain": (solves / elapsed) / plain if plain > 0 else None,
        "dense_apply_us": {"A": gem[0] * 1e3, "AT": gem[1] * 1e3},
        # algorithmic bytes of one apply in the BF16 phase: the BF16 matrix W_hi
        # (2 m n bytes), read once; the launch time covers pack + GEMM + reduce
        "roofline": {"bound": "hbm", "achieved": (2 * (2 * m * n)) / ((gem[0] + gem[1]) * 1e-3) / 1e9,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": (2 * (2 * m * n)) / ((gem[0] + gem[1]) * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "traffic": measured_traffic("k_gemm_bf16"),
                     "traffic_unit": "HBM bytes per k_gemm_bf16 launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated)",
                     "kernel": "pack + k_gemm_bf16 + reduce (A and A^T as BF16 MFMA GEMMs over the batch)",
                     "bytes_per_launch": 2 * m * n,
                     # three BF16 product terms (the input carried to FP32 accuracy) per apply
                     "mfma_tflops": (2 * 3 * 2 * m * n * B) / ((gem[0] + gem[1]) * 1e-3) / 1e12},
        "cpu_baseline": cpu, "verify": verify,
    })
    return out


# ---------------------------------------------------------------- serving replay
def run_serve(args, cfg):
    import numpy as np
    import torch
    import workloads as w
    import paper_1609_03488_amd as P
    from paper_1609_03488_amd.serve import replay

    trace = w.serving_trace(cfg["count"], cfg["rate"], cfg["seed"])
    if args.serve_count:
        trace = trace[:args.serve_count]
    log(f"generating {len(trace)} requests")
    probs = {}
    for r in trace:
        d = w.serving_request_data(r, cfg["density"], cfg["noise_var"])
        probs[r.rid] = (d, P.deconv_problem(d["c"], d["b"]))
    # small requests run whole steps in one workgroup (fused path), larger ones
    # one launch per kernel; both kinds share every round
    st = P.Settings.make(precision=P.FP32, eps=cfg["eps"], check_every=10, normalize=args.normalize,
                         cg_max_iters=args.serve_cg, fused_max=args.serve_fused_max)
    stream = torch.cuda.Stream()
    res = replay(trace, lambda r: probs[r.rid][1], settings=st, workspace_bytes=args.serve_ws << 30,
                 steps_per_call=10, stream=stream, log=log, keep_x=not args.no_verify)
    log(f"served {res['completed']} in {res['wall_s']:.1f}s: {res['solves_per_s']:.1f} solves/s, "
        f"p50 {res['p50_s']:.2f}s p99 {res['p99_s']:.2f}s")
    verify = None
    ref = golden(cfg["name"] + "_sample")
    if not args.no_verify:
        import oracle
        # parity on the seeded 5 % subsample spread over the trace's size range:
        # each served objective against the oracle's run of the same method to
        # the same eps (stored), and the noise-norm bound on every request
        done = {c.rid: c for c in res["completions"]}
        worst, worst_noise, checked = 0.0, 0.0, 0
        if ref is not None and ref["eps"] == cfg["eps"] and ref["normalize"] == args.normalize:
            for rid, r in ref["requests"].items():
                c = done.get(int(rid))
                if c is None:
                    continue
                d = probs[c.rid][0]
                f = oracle.deconv_objective(d["c"], d["b"], c.x)
                worst = max(worst, abs(f - r["objective"]) / r["objective"])
                checked += 1
        for c in res["completions"]:
            d = probs[c.rid][0]
            f = oracle.deconv_objective(d["c"], d["b"], c.x)
            noise = float(np.linalg.norm(d["b"] - np.convolve(d["c"], d["x_true"])))
            worst_noise = max(worst_noise, f / noise)
        verify = {"oracle_parity_requests": checked,
                  "worst_rel_obj_err_vs_oracle": worst if checked else None,
                  "max_objective_over_noise_norm": worst_noise, "solved": res["solved"]}
        log("verify", verify)
    # plain one-at-a-time FIFO on a prefix of the trace
    nfifo = min(len(trace), args.plain_sample)
    fifo = replay(trace[:nfifo], lambda r: probs[r.rid][1], settings=st,
                  workspace_bytes=2 << 30, max_slots=1, steps_per_call=10, stream=stream)
    log(f"FIFO one-at-a-time on {nfifo}: {fifo['solves_per_s']:.2f} solves/s")
    cpu = None
    if not args.no_cpu_baseline and ref is not None:
        import oracle
        # bounded sample: every 10th request of the stored subsample (10 requests
        # spread over the size range); for each, the factorisation, the setup and
        # a few iterations are timed and extrapolated to the oracle's own
        # iteration count for that request (stored with its objective)
        rids = sorted(ref["requests"], key=lambda k: ref["requests"][k]["n"])[5::10]
        tot, timed = 0.0, 0.0
        for rid in rids:
            r = ref["requests"][rid]
            d = probs[int(rid)][0]
            prog = oracle.deconv_program(d["c"], d["b"])
            t0 = time.perf_counter()
            fac = oracle.prepare(prog, args.normalize)[0].factor()
            t_factor = time.perf_counter() - t0
            rs = oracle.scs_solve(prog, eps=cfg["eps"], max_iters=args.cpu_iters, check_every=10, fac=fac,
                                  normalize=args.normalize)
            timed += time.perf_counter() - t0
            tot += t_factor + rs.setup_s + r["iters"] * rs.solve_s / max(rs.iters, 1)
        cpu = {"value": len(rids) / tot, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
               "sample": (f"{len(rids)} requests of the seeded 5 % subsample (every 10th by size, n "
                          f"{min(ref['requests'][k]['n'] for k in rids)}..{max(ref['requests'][k]['n'] for k in rids)}): "
                          f"FP64 oracle factorisation + setup + {args.cpu_iters} ADMM iterations timed "
                          f"({timed:.1f} s in all) and extrapolated to each request's oracle iteration count "
                          f"-> {tot:.0f} s for the {len(rids)}")}
        log("cpu", cpu)
    out = base_record(args, res["solves_per_s"], "solves/s", res["wall_s"], "f32",
                      {"workload": cfg["name"], "requests": len(trace), "rate_per_s": cfg["rate"],
                       "eps": cfg["eps"], "normalize": args.normalize, "scalars": "f64"})
    out.update({
        "p50_latency_s": res["p50_s"], "p99_latency_s": res["p99_s"], "completed": res["completed"],
        "solved": res["solved"], "mean_admm_iters": res["mean_iters"],
        "plain_fifo_solves_per_s": fifo["solves_per_s"],
        "plain_fifo_sample": nfifo, "cpu_baseline": cpu, "verify": verify,
    })
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="deconv_n1M_k1025")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--cpu-solves", type=int, default=4)
    ap.add_argument("--cpu-sample-n", type=int, default=1 << 14,
                    help="signal length of the deconvolution sample the oracle is timed on")
    ap.add_argument("--plain-sample", type=int, default=8)
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--normalize", type=int, default=None, choices=(0, 1, 2),
                    help="data scaling level of the solver (and of the oracle baseline); default: "
                         "1 for convolutions (block balancing inflates their spectral norm and "
                         "the CG systems), 2 for the dense lasso blocks")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default kernel choices instead of timing the candidates")
    ap.add_argument("--conv-engine", type=int, default=None, choices=(0, 1, 2),
                    help="FP32 convolution engine without autotuning (0 vector ALU, 1 matrix "
                         "cores, 2 FFT); for profiling runs of one engine")
    ap.add_argument("--max-iters", type=int, default=None,
                    help="cap on ADMM iterations (profiling runs; the JSON then says so)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB copied by a plain device copy after the run (counter calibration)")
    ap.add_argument("--serve-count", type=int, default=None)
    ap.add_argument("--serve-ws", type=int, default=16, help="server workspace, GiB")
    ap.add_argument("--serve-cg", type=int, default=3, help="CG iterations per step, upper bound")
    ap.add_argument("--serve-fused-max", type=int, default=3072,
                    help="largest n + m served by the fused one-workgroup-per-request path "
                         "(larger requests take one launch per kernel; with 60-120 requests "
                         "in flight the shared launches spread them over more of the chip)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              "the solver has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as w
    torch.cuda.set_device(0)
    cfg = w.workload(args.workload)
    log("workload", cfg["name"])
    fam = cfg["family"]
    if args.normalize is None:
        args.normalize = cfg.get("normalize", 2 if fam in ("lasso", "lasso_batch") else 1)
    if fam == "deconv":
        out = run_deconv(args, cfg)
    elif fam == "lasso":
        out = run_lasso(args, cfg)
    elif fam == "lasso_batch":
        out = run_lasso_batch(args, cfg)
    elif fam == "serve":
        out = run_serve(args, cfg)
    elif fam == "regls":
        out = run_regls(args, cfg)
    elif fam == "lasso_conv":
        out = run_lasso_conv(args, cfg)
    else:
        raise SystemExit(f"unknown workload family {fam}")
    if args.copy_calibration:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters scale
        # the counters of the solver's kernels to bytes
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
