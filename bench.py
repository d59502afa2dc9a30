"""Benchmark: parareal solves/s on one MI355X.

Default line: a ragged batch of 256 independent solves (each its own seeded
high-contrast medium, coarse grid 8x8..32x32, CEM-GMsFEM spaces built on the
GPU, 16..128 intervals of 32 fine steps, random smooth source), all solved
together by grouped launches, mixed FP32-MFMA path against the plain FP64
path, both to the relative stopping tolerance 1e-7 * max_n |x_n^0|_M. A step
is one batch solve: every solve runs Algorithm 1 (fine sweep over all its
intervals, coarse sweep with correction, stopping test) until its own test
holds. Inputs (blocks, sources, x0) are resident on the GPU before timing
starts; the set-up pipeline and the handles' FP64 factorisations are timed
separately.

Other workloads (--workload): c1 (one 200x200 problem, with the
forward+adjoint leg), c4 (400x400, 32 samples, forward + adjoint), wr (the
paper's waveform-relaxation fine solver).

Prints one JSON line. The CPU-baseline leg times the FP64 oracle on the host
on a seeded sample of the same workload and also supplies the reference the
GPU results' relative L2 errors are measured against.
"""
import argparse
import json
import os
import sys
import time


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


WORKLOAD = ("200x200 Q1 fine grid, 20x20 coarse grid, lognormal kappa (sigma 1, corr 0.05) with "
            "1e6 channels and inclusions, CEM-GMsFEM d1=800 (V_H1) d2=1200 (V_H2), N=64 intervals "
            "x P=64 fine steps, f=sin(pi x)sin(pi y)e^-t, u0=0, 1 sample, rel tol 1e-7")
METRIC = "parareal solves/sec to 1e-6 rel L2: batched FP32-MFMA+refine vs plain FP64"
PEAK_FP32_MFMA = 157.3   # TFLOP/s, MI355X dense FP32 matrix
PEAK_FP64_MFMA = 78.6
PEAK_HBM_TBPS = 8.0      # MI355X HBM3E

# HBM bytes per launch of the fine residual product, from two rocprofv3 --pmc
# passes (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0: the factors a 256 MiB device
# copy reads for the same counters), keyed by workload and the kernel's tile
# configuration (state-tile rows, operator-tile rows, K depth, split-K).
# Reported only when the timed run used that kernel class and configuration.
# (the 200x200 single-problem product's counters predate the current product
# kernel, so its line reports no traffic)
MEASURED_TRAFFIC = {# the 256-solve batch: FETCH_SIZE x 2 + WRITE_SIZE x 1 of the grouped FP32
                    # product over one batch solve, divided by its 558 fine-step launches
                    ("c2", 256): (2.0 * 6432177144.2 + 1.0 * 433136376.4) * 1024 / 2 / 558}


def time_solves(pr, x0, tol, steps, warmup, torch):
    """Warm-up (includes the autotuner's first visit of each product shape),
    then the timed region: exactly `steps` solves between two device
    synchronisations. A second pass of `steps` solves records HIP events
    around every launch (on the handle's stream) for per-kernel durations;
    it is not part of the throughput figure."""
    for _ in range(warmup):
        pr.solve(x0, tol=tol, norm="rel")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        X, iters, hist, st = pr.solve(x0, tol=tol, norm="rel")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pr.profile(True)
    t1 = time.perf_counter()
    for _ in range(steps):
        pr.solve(x0, tol=tol, norm="rel")
    torch.cuda.synchronize()
    dt_prof = time.perf_counter() - t1
    prof = pr.profile_read()
    pr.profile(False)
    return dt, X, iters, hist, st, prof, dt_prof


ADJ_WORKLOAD = ("same medium and spaces as the forward workload; source sum_i theta_{i,n} 1_{K_i}(x) "
                "1_{(t_n,t_{n+1}]}(t) over the 400 coarse elements (theta 400 x 64), loss "
                "1/2 |x(T)-r(T)|_M^2 + 1/2 sum_m dt_fine |x_m-r_m|_M^2 against the trajectory r of "
                "(theta_ref ~ N(0,1), x0_ref = 0), evaluated at theta_ref + 0.1 N(0,1), x0 = 0.1 N(0,1)/sqrt(D); "
                "forward and transposed parareal to rel tol 1e-7")


def adjoint_leg(args, torch, pe, build_problem, precs):
    """Forward + adjoint workload: one step is a forward parareal solve of
    the tracking error y = x - r (source theta - theta_ref, start x0: the
    scheme is linear) and the transposed parareal with the terminal and
    fine-step tracking cotangents (fine levels recomputed inside the
    intervals), giving dL/dtheta and dL/dx0."""
    import numpy as np
    t0 = time.perf_counter()
    p = build_problem("c3", verbose=False)
    log(f"adjoint workload c3 built in {time.perf_counter() - t0:.1f}s")
    d1, d2, N, P = p["d1"], p["d2"], p["N"], p["P"]
    D = d1 + d2
    rng = np.random.default_rng(3)
    theta_ref = p["H"][0]
    theta = theta_ref + 0.1 * rng.standard_normal(theta_ref.shape)
    x0 = torch.tensor(0.1 * rng.standard_normal((1, D)) / np.sqrt(D), device="cuda")
    dH = torch.tensor((theta - theta_ref)[None], device="cuda")
    M = np.block([[p["M11"], p["M12"]], [p["M12"].T, p["M22"]]])
    Mt = torch.tensor(M, device="cuda")
    tol = 1e-7
    out = {}
    for prec in precs:
        pr = pe.problem_from(dict(p, H=dH.cpu().numpy()), prec)

        def step():
            Y, itf, _, _ = pr.solve(x0, tol=tol, norm="rel")
            Xbar = torch.zeros_like(Y)
            Xbar[:, -1] = Y[:, -1] @ Mt
            r = pr.adjoint(Xbar=Xbar, beta=1.0, Ybnd=Y, dH=dH, tol=tol)
            return itf, r

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(args.steps):
            itf, r = step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - ts
        pr.profile(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        prof = pr.profile_read()
        pr.profile(False)
        out[prec] = dict(seconds=dt, it_fwd=int(itf[0]), it_adj=int(r["iters"][0]), prof=prof,
                         grad=np.concatenate([r["x0bar"].cpu().numpy().ravel(), r["Hbar"].cpu().numpy().ravel()]),
                         tiles=pr.last_tiles("adj_step"))
        log(f"adjoint {prec}: {args.steps} forward+adjoint solves in {dt:.3f}s, iterations fwd {itf[0]} "
            f"adj {r['iters'][0]}; launch timing: " +
            ", ".join(f"{k} {v[0]:.2f}ms/{v[1]}" for k, v in prof.items() if v[1]))
        pr.close()
    mixed = out[precs[0]]
    ms, n = mixed["prof"]["adj_step"]
    flops = 4.0 * D * D * N
    avg = (ms / n) * 1e-3 if n else float("nan")
    res = {"workload": ADJ_WORKLOAD, "name": "c3", "metric": "forward+adjoint solves/s (gradient wrt theta, x0)",
           "value": round(args.steps / mixed["seconds"], 4), "unit": "solves/s",
           "ms_per_step": round(1e3 * mixed["seconds"] / args.steps, 4), "precision": precs[0],
           "iterations": {"forward": mixed["it_fwd"], "adjoint": mixed["it_adj"]},
           "roofline": dict(kernel="gemm_nt_kernel<%s,%d,%d,%d> fused adjoint step ([A; A+Mh] Z^T nu), split-K %d"
                            % (("float" if precs[0] == "mixed" else "double",) + tuple(mixed["tiles"])),
                            bound="mfma", achieved=round(flops / avg / 1e12, 3),
                            peak=PEAK_FP32_MFMA if precs[0] == "mixed" else PEAK_FP64_MFMA, unit="TFLOP/s",
                            frac=round(flops / avg / 1e12 / (PEAK_FP32_MFMA if precs[0] == "mixed"
                                                            else PEAK_FP64_MFMA), 5),
                            traffic=None, avg_launch_us=round(avg * 1e6, 3), launches=n,
                            flops_per_launch=flops)}
    if len(precs) > 1:
        f64 = out[precs[1]]
        res["fp64"] = {"value": round(args.steps / f64["seconds"], 4), "unit": "solves/s",
                       "iterations": {"forward": f64["it_fwd"], "adjoint": f64["it_adj"]}}
        res["speedup_mixed_vs_fp64"] = round(f64["seconds"] / mixed["seconds"], 4)
        res["grad_rel_diff_mixed_vs_fp64"] = float("%.3e" % (np.linalg.norm(mixed["grad"] - f64["grad"]) /
                                                            np.linalg.norm(f64["grad"])))
    return res


C2_WORKLOAD = ("ragged batch of 256 independent solves, each with its own seeded medium and spaces: n_c ~ U{8..32} "
               "coarse grid (fine n = 10 n_c), kappa = 1 + floor(n_c/4) horizontal and vertical one-cell channels "
               "of contrast 10^U(4,6), CEM-GMsFEM d1 = 2 n_c^2, d2 = 3 n_c^2 built on the GPU, N ~ U{16..128} "
               "intervals x P = 32 fine steps at half the stable coarse step, source = 8 Fourier modes "
               "sin(p pi x) sin(q pi y), (p,q) ~ U{1..4}^2, N(0,1) time-constant amplitudes, u0 = 0, "
               "rel tol 1e-7")


def oracle_threads():
    """BLAS threads for the oracle's host run. numpy and scipy each bring
    their own OpenBLAS with one thread per core, and the oracle alternates
    calls into both: two pools of busy-waiting threads on the same cores slow
    its small products by 10-30x, so each pool gets half the cores. Returns
    (threads per pool, libraries)."""
    n = max(1, (os.cpu_count() or 2) // 2)
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threadpool_limits(limits=n, user_api="blas")
        info = threadpool_info()
        return (max([i.get("num_threads", 1) for i in info] or [1]),
                ",".join(sorted({i.get("internal_api", "?") for i in info})))
    except Exception:
        return os.cpu_count(), "?"


def _threads():
    return oracle_threads()


def batch_main(args, torch, pe):
    """Ragged batch of 256 different problems: all solves advance together;
    each fine step is one grouped launch per product over every solve's
    interval columns. A step is one batch solve (every solve to its own
    stopping test). The headline leg is timed over exactly `steps` batch
    solves; the comparison legs over max(2, steps // 4)."""
    import numpy as np
    from problem.batch import gpu_problem, solve_spec
    n_solves = args.solves
    t0 = time.perf_counter()
    specs = [solve_spec(b) for b in range(n_solves)]
    t_spec = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    probs = []
    for s in specs:
        p = gpu_problem(s)
        # the blocks wait in host memory between the legs, so each leg's
        # handles have the device to themselves
        for k in ("M11", "M12", "M22", "A11", "A12", "A22", "G"):
            p[k] = p[k].cpu().numpy()
        probs.append(p)
        if len(probs) % 64 == 0:
            log(f"c2: {len(probs)} problems built on the GPU ({time.perf_counter() - t0:.1f}s)")
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    t_parts = {k: round(sum(p["seconds"][k] for p in probs), 2) for k in probs[0]["seconds"]}
    log(f"c2: set-up pipeline parts (s): {t_parts}")
    Ns = [p["N"] for p in probs]
    d1 = [p["d1"] for p in probs]
    d2 = [p["d2"] for p in probs]
    log(f"c2: {n_solves} solves, sum N = {sum(Ns)}, D {min(a + b for a, b in zip(d1, d2))}.."
        f"{max(a + b for a, b in zip(d1, d2))}; media and sources {t_spec:.1f}s, GPU set-up pipeline "
        f"(spaces, blocks, stable step) {t_build:.1f}s")
    tol = 1e-7
    keys = ("M11", "M12", "M22", "A11", "A12", "A22")
    # fused-step flops of one fine step of each solve (the launches only
    # cover the solves still iterating: a solve takes part in (P - 1) step
    # launches per fine sweep it runs; the first step has no deviation)
    f_step = [2.0 * (a * a + 4.0 * a * b + 2.0 * b * b) * n for a, b, n in zip(d1, d2, Ns)]
    P = probs[0]["P"]
    rng = np.random.default_rng(7)
    # the oracle's sample: seeded solves it finishes in seconds each
    # (24 solves with D <= 2000, N <= 128: about 10-20 s of the oracle on 16 cores)
    sample = [int(b) for b in rng.permutation(n_solves) if d1[b] + d2[b] <= 2000][:24]
    # the headline leg is the refined mixed path (FP32 MFMA products, FP64
    # residual and FP32 correction of every fine step's implicit solve in the
    # sweeps at the state's scale); the unrefined mixed path and the plain
    # FP64 path are timed beside it
    names = [s for s in args.legs.split(",") if s]
    if args.no_fp64:
        names = [s for s in names if s != "fp64"]
    if not names or any(s not in ("mixed_refine", "mixed", "fp64") for s in names):
        raise SystemExit(f"bench.py: --legs takes mixed_refine, mixed, fp64 (got {args.legs})")
    legs = [(names[0], args.steps, args.warmup)] + [(s, max(2, args.steps // 4), min(args.warmup, 2))
                                                    for s in names[1:]]
    res = {}
    for prec, steps, warmup in legs:
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        handles = []
        for p in probs:
            pr = pe.Problem({k: p[k] for k in keys}, p["dt"], p["dt_fine"], p["N"], precision=prec, stream=stream)
            pr.set_source(p["G"], p["H"], "interval")
            handles.append(pr)
        bt = pe.Batch(handles)
        torch.cuda.synchronize()
        setup = time.perf_counter() - ts
        x0s = [torch.zeros((1, h.D), dtype=torch.float64, device="cuda") for h in handles]
        for _ in range(warmup):
            bt.solve(x0s, tol=tol, norm="rel")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            Xs, its, st = bt.solve(x0s, tol=tol, norm="rel")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        bt.profile(True)
        bt.solve(x0s, tol=tol, norm="rel")
        prof = bt.profile_read()
        bt.profile(False)
        it = np.array([int(i[0]) for i in its])
        res[prec] = dict(seconds=dt, steps=steps, setup=setup, prof=prof, iters=it, status=st,
                         X={b: Xs[b][0].cpu().numpy() for b in sample})
        log(f"c2 {prec}: {steps} batch solves in {dt:.3f}s ({n_solves * steps / dt:.1f} solves/s), "
            f"handles {setup:.1f}s, iterations mean {it.mean():.2f} max {it.max()}; launch timing: " +
            ", ".join(f"{k} {v[0]:.2f}ms/{v[1]}" for k, v in prof.items() if v[1]))
        bt.close()
        for h in handles:
            h.close()
        del handles, bt, Xs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if args.calib_copy_mb:
        nc = args.calib_copy_mb * (1 << 20) // 4
        ca = torch.ones(nc, dtype=torch.float32, device="cuda")
        cb = torch.empty_like(ca)
        torch.cuda.synchronize()
        cb.copy_(ca)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mb} MiB read + {args.calib_copy_mb} MiB written")
        del ca, cb
    head_name = names[0]
    head = res[head_name]
    refined = head_name == "mixed_refine"
    ms, n = head["prof"]["fine_step"]
    avg = (ms / n) * 1e-3
    # algorithmic work of the profiled batch solve's fine-step launches:
    # solve b runs one fine sweep per iteration, (P - 1) launches each.
    # Bytes per launch and solve: the FP32 operator's nonzero blocks
    # 4 (d1^2 + 4 d1 d2 + 2 d2^2) read once, and per interval column the FP32
    # state read (2 Dp x 4), the FP64 input state and anchor term read
    # (2 x Dp x 8), the FP64 and FP32 new state written (2 Dp x 12), and in
    # the refined first sweep the implicit equation's operands (2 Dp x 8)
    flops_total = sum(f * (P - 1) * int(k) for f, k in zip(f_step, head["iters"]))
    flops_res = flops_total / n
    Dps = [(a + 7) // 8 * 8 + (c + 7) // 8 * 8 for a, c in zip(d1, d2)]
    op_bytes = [4.0 * (a * a + 4.0 * a * c + 2.0 * c * c) for a, c in zip(d1, d2)]
    bytes_total = sum((P - 1) * (int(k) * (ob + 48.0 * dp * nn) + (16.0 * dp * nn if refined else 0.0))
                      for ob, dp, nn, k in zip(op_bytes, Dps, Ns, head["iters"]))
    bytes_res = bytes_total / n
    log(f"c2 {head_name}: fine-step launches of one batch solve: {n}, algorithmic bytes {bytes_total:.6e}, "
        f"flops {flops_total:.6e}")
    out = {"metric": METRIC, "value": round(n_solves * args.steps / head["seconds"], 3), "unit": "solves/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * head["seconds"] / args.steps, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if head_name == "fp64" else "f32",
           "data": "synthetic",
           "config": {"workload": C2_WORKLOAD, "name": "c2", "solves": n_solves, "sum_N": sum(Ns), "P": P,
                      "D_range": [min(a + b for a, b in zip(d1, d2)), max(a + b for a, b in zip(d1, d2))],
                      "precision": {"mixed_refine": "FP32 MFMA fine-step and coarse-correction products in "
                                                    "mass-whitened coordinates on FP64 anchors, with the FP64 "
                                                    "residual and FP32 correction of each fine step's implicit "
                                                    "V_H1 solve in the first (state-scale) sweep; FP64 "
                                                    "factorisations, state, jump norms",
                                    "mixed": "FP32 MFMA fine-step and coarse-correction products in "
                                             "mass-whitened coordinates on FP64 anchors; FP64 factorisations, "
                                             "state, jump norms",
                                    "fp64": "every product in FP64"}[head_name],
                      "gpu_setup_pipeline_parts_s": t_parts,
                      "iterations_mean": round(float(head["iters"].mean()), 3),
                      "iterations_max": int(head["iters"].max()),
                      "gpu_setup_pipeline_s": round(t_build, 2), "handles_setup_s": round(head["setup"], 2)},
           # the fused fine-step product of a ragged batch: N_b / 2 flops per
           # byte of each solve's FP32 operator (N_b = 16..128 interval
           # columns), 33 flop/B averaged over a batch solve's launches, above
           # the FP32 ridge (157.3 / 8 = 19.7 flop/B): matrix-core bound
           "roofline": dict(kernel="gemm_grouped_kernel<float,64,64,32> fused fine-step products of all solves",
                            bound="mfma", achieved=round(flops_res / avg / 1e12, 3), peak=PEAK_FP32_MFMA,
                            unit="TFLOP/s", frac=round(flops_res / avg / 1e12 / PEAK_FP32_MFMA, 5),
                            traffic=(round(MEASURED_TRAFFIC[("c2", n_solves)])
                                     if ("c2", n_solves) in MEASURED_TRAFFIC else None),
                            traffic_ratio=(round(MEASURED_TRAFFIC[("c2", n_solves)] / bytes_res, 3)
                                           if ("c2", n_solves) in MEASURED_TRAFFIC else None),
                            avg_launch_us=round(avg * 1e6, 3), launches=n, flops_per_launch=round(flops_res),
                            bytes_per_launch=round(bytes_res),
                            hbm_achieved_GBps=round(bytes_res / avg / 1e9, 1),
                            hbm_frac=round(bytes_res / avg / 1e12 / PEAK_HBM_TBPS, 5),
                            work_note="algorithmic flops (2(d1^2 + 4 d1 d2 + 2 d2^2) per interval column) and bytes "
                                      "(FP32 operator blocks once, FP32 state read, FP64 state and anchor read, FP64 "
                                      "and FP32 state written, refinement operands) of the solves each launch "
                                      "covered, averaged over the launches of one profiled batch solve (launches "
                                      "late in the solve cover only the solves still iterating); traffic: HBM bytes "
                                      "per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE, calibrated by a device "
                                      "copy of known size")}
    ms_r, n_r = head["prof"]["refine"]
    out["roofline"]["refine_launches"] = n_r
    out["roofline"]["refine_ms_per_batch_solve"] = round(ms_r, 3)
    out["config"]["headline_path"] = head_name
    for leg in names[1:]:
        if leg not in res:
            continue
        r = res[leg]
        out[leg] = {"value": round(n_solves * r["steps"] / r["seconds"], 3), "unit": "solves/s",
                    "steps": r["steps"], "iterations_mean": round(float(r["iters"].mean()), 3),
                    "handles_setup_s": round(r["setup"], 2)}
        out[f"speedup_vs_{leg}"] = round((r["seconds"] / r["steps"]) / (head["seconds"] / args.steps), 4)
        out[f"iterations_equal_{leg}"] = bool(np.array_equal(head["iters"], r["iters"]))
    if not args.no_cpu_baseline:
        import oracle.scheme as S
        threads, blas = _threads()
        t2 = time.perf_counter()
        errs = {k: [] for k in res}
        k_or = []
        for b in sample:
            p = probs[b]
            pc = {k: p[k] for k in keys}
            pc.update(dt=p["dt"], dt_fine=p["dt_fine"], N=p["N"], P=P, G=p["G"], H=p["H"], time_mode=1)
            bl, src = S.Blocks.from_problem(pc), S.Source.from_problem(pc)
            r = S.parareal(bl, src, np.zeros(bl.D), tol, rel=True)
            k_or.append(int(r["K"]))
            for k in res:
                kk = min(int(res[k]["iters"][b]), int(r["K"]))
                errs[k].append(S.rel_l2_M(bl, res[k]["X"][b], r["X"][kk]))
        dt_cpu = time.perf_counter() - t2
        # the oracle's cost scales with the fine-sweep work iterations x N x D^2
        work = [int(head["iters"][b]) * Ns[b] * (d1[b] + d2[b]) ** 2 for b in range(n_solves)]
        scale = sum(work) / sum(work[b] for b in sample)
        out["cpu_baseline"] = {"value": round(n_solves / (dt_cpu * scale), 6), "unit": "solves/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"{len(sample)} seeded solves of the batch with D <= 2000 (b = {sample}), "
                                         f"FP64 NumPy/SciPy parareal ({blas}), {dt_cpu:.1f}s, scaled to the whole "
                                         f"batch by the fine-sweep work iterations x N x D^2 (x{scale:.1f})"}
        out["rel_l2_vs_oracle_sampled"] = {k: [float(f"{e:.3e}") for e in v] for k, v in errs.items()}
        out["iterations_sampled"] = {"oracle": k_or, **{k: [int(res[k]["iters"][b]) for b in sample] for k in res}}
    print(json.dumps(out), flush=True)


C4_WORKLOAD = ("400x400 Q1 fine grid, 40x40 coarse, kappa = 1 with 10 horizontal + 10 vertical channels of 1e6, "
               "CEM-GMsFEM d1 = 3200, d2 = 4800, N = 256 intervals x P = 128, 32 samples of 8 Fourier modes with "
               "N(0,1) per-interval amplitudes, u0 = 0; forward parareal and transposed parareal (loss "
               "1/2 |x_N|_M^2 + 1/2 sum_n dt |x_n|_M^2) per step, both to rel tol 1e-7")


def large_main(args, torch, pe):
    """Large batched forward + adjoint: B = 32 samples share one problem;
    every fine-step product covers 32 x 256 = 8192 interval columns."""
    import numpy as np
    from problem import build_problem
    t0 = time.perf_counter()
    p = build_problem("c4")
    d1, d2, N, P, B = p["d1"], p["d2"], p["N"], p["P"], p["H"].shape[0]
    D = d1 + d2
    log(f"c4 built in {time.perf_counter() - t0:.1f}s: d1={d1} d2={d2} N={N} P={P} B={B}")
    tol = 1e-7
    M = np.block([[p["M11"], p["M12"]], [p["M12"].T, p["M22"]]])
    Mt = torch.tensor(M, device="cuda")
    x0 = torch.zeros((B, D), dtype=torch.float64, device="cuda")
    res = {}
    for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
        ts = time.perf_counter()
        pr = pe.problem_from(p, prec)
        torch.cuda.synchronize()
        setup = time.perf_counter() - ts

        def step():
            X, itf, _, _ = pr.solve(x0, tol=tol, norm="rel")
            Xbar = p["dt"] * (X @ Mt)
            Xbar[:, 0] = 0.0
            Xbar[:, -1] += X[:, -1] @ Mt
            r = pr.adjoint(Xbar=Xbar, tol=tol)
            log(f"c4 {prec}: step done ({time.perf_counter() - ts:.1f}s since set-up began)")
            return itf, r

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            itf, r = step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        pr.profile(True)
        step()
        torch.cuda.synchronize()
        prof = pr.profile_read()
        pr.profile(False)
        res[prec] = dict(seconds=dt, setup=setup, prof=prof, it_f=int(itf.max()), it_a=int(r["iters"].max()),
                         tiles=pr.last_tiles("fine_step"), tiles_adj=pr.last_tiles("adj_step"),
                         grad=np.concatenate([r["x0bar"].cpu().numpy().ravel(), r["Hbar"].cpu().numpy().ravel()]))
        log(f"c4 {prec}: {args.steps} forward+adjoint steps in {dt:.2f}s, iterations fwd {itf.max()} adj "
            f"{r['iters'].max()}, set-up {setup:.1f}s; launch timing: " +
            ", ".join(f"{k} {v[0]:.1f}ms/{v[1]}" for k, v in prof.items() if v[1]))
        pr.close()
        torch.cuda.empty_cache()
    mixed = res["mixed"]
    rf = 2.0 * (d1 * d1 + 4.0 * d1 * d2 + 2.0 * d2 * d2) * N * B
    ms, n = mixed["prof"]["fine_step"]
    ams, an = mixed["prof"]["adj_step"]
    avg, aavg = ms / n * 1e-3, ams / an * 1e-3
    af = 4.0 * D * D * N * B
    out = {"metric": "forward+adjoint parareal solves/sec (batched samples)",
           "value": round(B * args.steps / mixed["seconds"], 4), "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * mixed["seconds"] / args.steps, 2),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": C4_WORKLOAD, "name": "c4", "d1": d1, "d2": d2, "N": N, "P": P, "samples": B,
                      "iterations": {"forward": mixed["it_f"], "adjoint": mixed["it_a"]},
                      "setup_s": round(mixed["setup"], 2)},
           "roofline": dict(kernel="gemm_nt_kernel<float,%d,%d,%d> fused fine-step product, split-K %d"
                            % tuple(mixed["tiles"]), bound="mfma", achieved=round(rf / avg / 1e12, 3),
                            peak=PEAK_FP32_MFMA, unit="TFLOP/s", frac=round(rf / avg / 1e12 / PEAK_FP32_MFMA, 5),
                            traffic=None, avg_launch_us=round(avg * 1e6, 2), launches=n, flops_per_launch=rf),
           "adjoint_roofline": dict(kernel="gemm_nt_kernel<float,%d,%d,%d> fused adjoint step, split-K %d"
                                    % tuple(mixed["tiles_adj"]), achieved=round(af / aavg / 1e12, 3),
                                    peak=PEAK_FP32_MFMA, frac=round(af / aavg / 1e12 / PEAK_FP32_MFMA, 5),
                                    avg_launch_us=round(aavg * 1e6, 2), launches=an, flops_per_launch=af)}
    if "fp64" in res:
        f64 = res["fp64"]
        out["fp64"] = {"value": round(B * args.steps / f64["seconds"], 4), "unit": "solves/s",
                       "iterations": {"forward": f64["it_f"], "adjoint": f64["it_a"]}}
        out["speedup_mixed_vs_fp64"] = round(f64["seconds"] / mixed["seconds"], 4)
        out["grad_rel_diff_mixed_vs_fp64"] = float("%.3e" % (np.linalg.norm(mixed["grad"] - f64["grad"]) /
                                                            np.linalg.norm(f64["grad"])))
    print(json.dumps(out), flush=True)


WR_WORKLOAD = ("fine propagator by waveform relaxation with the alpha-circulant diagonalisation in time "
               "(FP64), applied to the interval start states of the first parareal iterate of the 200x200 "
               "workload ({split}, d1={d1}, d2={d2}, N={N} intervals x P={P} fine steps, "
               "f=sin(pi x)sin(pi y)e^-t)")


def wr_main(args, torch, pe):
    """The paper's fine solver (waveform relaxation, alpha-circulant
    diagonalisation) on the 200x200 workload: a step is one WR fine sweep
    (K0 iterations on all N intervals); the exact fine sweep (pe_fine_propagate,
    FP64) is timed beside it, and the error after each iteration is recorded
    for several alpha."""
    import numpy as np
    import oracle.wr as WR
    import oracle.scheme as S
    from problem import build_problem
    p = build_problem(args.config)
    d1, d2, N, P = p["d1"], p["d2"], p["N"], p["P"]
    D = d1 + d2
    split = {"nlmc_fm": "NLMC fracture/matrix split", "nlmc": "NLMC split as printed"}.get(
        p["cfg"].get("split", "cem"), "CEM-GMsFEM split")
    pr = pe.problem_from(p, "fp64")
    x0 = torch.as_tensor(p["x0"], dtype=torch.float64, device="cuda")
    X0, _, _, _ = pr.solve(x0, tol=0.0, k_max=0)          # coarse sweep: x_n^0
    Xin = X0[:, :N].contiguous()
    exact = pr.fine(Xin)
    nrm = torch.linalg.norm(exact).item()
    alpha, K0 = args.wr_alpha, args.wr_iters
    curves = {}
    for a in sorted({0.1, 0.05, alpha, 0.005}, reverse=True):
        ts = time.perf_counter()
        pr.fine_wr(Xin, a, 0)
        torch.cuda.synchronize()
        errs = []
        for k in range(1, 13):
            errs.append(float("%.3e" % (torch.linalg.norm(pr.fine_wr(Xin, a, k) - exact).item() / nrm)))
        curves[str(a)] = errs
        log(f"wr alpha {a}: rel err after 1..12 iterations {errs} ({time.perf_counter() - ts:.1f}s incl. set-up)")
    for _ in range(args.warmup):
        pr.fine_wr(Xin, alpha, K0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Y = pr.fine_wr(Xin, alpha, K0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err = torch.linalg.norm(Y - exact).item() / nrm
    # the exact sequential fine sweep, same inputs
    for _ in range(2):
        pr.fine(Xin)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        pr.fine(Xin)
    torch.cuda.synchronize()
    dt_exact = time.perf_counter() - t1
    pr.profile(True)
    pr.fine_wr(Xin, alpha, K0)
    torch.cuda.synchronize()
    prof = pr.profile_read()
    pr.profile(False)
    log("wr launch timing: " + ", ".join(f"{k} {v[0]:.2f}ms/{v[1]}" for k, v in prof.items() if v[1]))
    NB = N
    flops = {"wr_rhs": 4.0 * P * NB * d1 * d2, "wr_solve": 8.0 * NB * d1 * d1 * (P // 2 + 1),
             "wr_wstep": 2.0 * NB * d2 * d2}
    names = {"wr_rhs": "gemm_nt_kernel<double> right-hand-side products of eqs. (4.8)/(4.9) over all fine levels",
             "wr_solve": "gemm_grouped_kernel<double,64,64,16> the P/2+1 complex-shifted solves (real 2d1 x 2d1 "
                         "forms), one grouped launch",
             "wr_wstep": "gemm_nt_kernel<double> sequential V_H2 step"}
    dom = max(flops, key=lambda k: prof[k][0])
    ms, n = prof[dom]
    avg = ms / n * 1e-3
    classes = {k: dict(ms_per_sweep=round(prof[k][0], 3), launches=prof[k][1],
                       tflops=round(flops[k] * prof[k][1] / (prof[k][0] * 1e-3) / 1e12, 3) if prof[k][1] else None)
               for k in flops}
    out = {"metric": "WR fine sweeps/s (all 64 intervals, K0 iterations)", "value": round(args.steps / dt, 4),
           "unit": "sweeps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * dt / args.steps, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": WR_WORKLOAD.format(split=split, d1=d1, d2=d2, N=N, P=P),
                      "name": "wr-" + args.config, "d1": d1, "d2": d2, "N": N, "P": P, "alpha": alpha,
                      "K0": K0, "rel_err_vs_exact_F": float("%.3e" % err)},
           "roofline": dict(kernel=names[dom], bound="mfma", achieved=round(flops[dom] / avg / 1e12, 3),
                            peak=PEAK_FP64_MFMA, unit="TFLOP/s",
                            frac=round(flops[dom] / avg / 1e12 / PEAK_FP64_MFMA, 5), traffic=None,
                            avg_launch_us=round(avg * 1e6, 2), launches=n, flops_per_launch=flops[dom]),
           "classes": classes,
           "exact_fine_sweep": {"sweeps_per_s": round(args.steps / dt_exact, 4),
                                "ms_per_sweep": round(1e3 * dt_exact / args.steps, 3)},
           "convergence": {"rel_err_after_iterations_1_to_12": curves}}
    if not args.no_cpu_baseline:
        bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
        cols = Xin[0].cpu().numpy().T
        ns, bs = list(range(N)), [0] * N
        WR.wr_fine_cols(bl, src, cols, ns, bs, alpha, 1)      # factorisations (cached)
        t2 = time.perf_counter()
        WR.wr_fine_cols(bl, src, cols, ns, bs, alpha, 1)
        t_it = time.perf_counter() - t2
        out["cpu_baseline"] = {"value": round(1.0 / (t_it * K0), 5), "unit": "sweeps/s",
                               "cores": os.cpu_count(), "kind": "oracle",
                               "sample": f"one WR iteration on all {N} intervals ({t_it:.1f}s, shifted "
                                         f"factorisations cached), scaled to K0 = {K0} iterations"}
    print(json.dumps(out), flush=True)
    pr.close()


def cpu_baseline(p, tol):
    """The FP64 oracle's plain parareal on the same workload, one solve."""
    import oracle.scheme as S
    threads, blas = oracle_threads()
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    t0 = time.perf_counter()
    r = S.parareal(bl, src, p["x0"][0], tol, rel=True)
    dt = time.perf_counter() - t0
    return dict(seconds=dt, K=r["K"], X=r["X"][r["K"]], bl=bl, threads=threads, blas=blas)


def setup_leg(args, torch, pe, p):
    """Set-up pipeline of the default workload: CEM-GMsFEM basis functions
    and Galerkin blocks on the GPU (pe_cem_spaces) from the host's local
    spectral data (gpu_s; compared with the CPU generator's blocks and
    source factor, largest relative Frobenius difference) and with the local
    spectral problems on the GPU too (gpu_with_spectral_s, pe_local_spectral),
    timed beside the CPU generator's basis construction and projection."""
    import numpy as np

    from problem.build import CONFIGS, make_medium, project_blocks
    from problem.cem import CoarseGrid, cem_basis, local_spectral, split_spaces
    from problem.fem import FineGrid

    cfg = dict(CONFIGS[args.config])
    kappa = make_medium(cfg)
    fine = FineGrid(kappa)
    cg = CoarseGrid(fine, cfg["n_c"])
    J = cfg["J1"] + cfg["J2"]
    t0 = time.perf_counter()
    _, _, spsi = local_spectral(cg, J)
    t_spec = time.perf_counter() - t0
    loads = fine.load_smooth(lambda x, y: np.sin(np.pi * x) * np.sin(np.pi * y))[None]
    run = lambda: pe.cem_spaces(kappa, spsi, cfg["n_c"], cfg["layers"], cfg["J1"], loads=loads)
    run()
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = run()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t_gpu = sorted(times)[1]
    # the whole pipeline on the GPU: local spectral problems included
    run_all = lambda: pe.cem_spaces(kappa, None, cfg["n_c"], cfg["layers"], cfg["J1"], loads=loads, J=J)
    run_all()
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_all()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t_all = sorted(times)[1]
    err = max(float(np.linalg.norm(out[k].cpu().numpy() - p[k]) / np.linalg.norm(p[k]))
              for k in ("M11", "M12", "M22", "A11", "A12", "A22", "G"))
    res = {"what": "CEM-GMsFEM basis functions (eq. (3.2), one banded Cholesky per oversampled patch) and "
                   "Galerkin blocks of eq. (3.8) with the source factor, 400 patches, D = 2000",
           "gpu_s": round(t_gpu, 4), "host_spectral_s": round(t_spec, 3),
           "gpu_with_spectral_s": round(t_all, 4),
           "rel_diff_vs_cpu_generator": float(f"{err:.3e}")}
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        phis = cem_basis(cg, J, cfg["layers"], spsi)
        P1, P2 = split_spaces(cg, phis, cfg["J1"], cfg["J2"])
        project_blocks(fine, P1, P2)
        res["cpu_generator_s"] = round(time.perf_counter() - t0, 3)
        res["speedup_vs_cpu_generator"] = round(res["cpu_generator_s"] / t_gpu, 1)
    log(f"set-up pipeline: {res}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c1")
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c4", "wr"],
                    help="c2: ragged batch of 256 different solves (default line); c1: one 200x200 problem; "
                         "c4: 400x400, 32 samples, forward + adjoint; wr: the waveform-relaxation "
                         "fine solver on the 200x200 problem")
    ap.add_argument("--solves", type=int, default=256, help="solves in the ragged batch (c2)")
    ap.add_argument("--legs", default="mixed_refine,mixed,fp64",
                    help="c2: paths to run, the first is the headline (mixed_refine, mixed, fp64)")
    ap.add_argument("--wr-alpha", type=float, default=0.02)
    ap.add_argument("--wr-iters", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward+adjoint workload")
    ap.add_argument("--no-setup", action="store_true", help="skip the set-up pipeline leg")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a kernel of known "
                         "HBM traffic, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (--gpus {args.gpus} requested); "
              "the library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2411_09244_amd as pe
    from problem import build_problem

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c2":
        return batch_main(args, torch, pe)
    if args.workload == "c4":
        return large_main(args, torch, pe)
    if args.workload == "wr":
        return wr_main(args, torch, pe)
    tol = 1e-7
    t0 = time.perf_counter()
    p = build_problem(args.config, verbose=False)
    log(f"workload {args.config}: d1={p['d1']} d2={p['d2']} N={p['N']} P={p['P']} dt={p['dt']:.3e} "
        f"built in {time.perf_counter() - t0:.1f}s")
    d1, d2, N, P = p["d1"], p["d2"], p["N"], p["P"]
    D = d1 + d2
    x0 = torch.as_tensor(p["x0"], dtype=torch.float64, device="cuda")

    res = {}
    for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        pr = pe.problem_from(p, prec)
        torch.cuda.synchronize()
        setup = time.perf_counter() - ts
        dt, X, iters, hist, st, prof, dt_prof = time_solves(pr, x0, tol, args.steps, args.warmup, torch)
        res[prec] = dict(seconds=dt, X=X[0].cpu().numpy(), iters=int(iters[0]), status=st,
                         setup=setup, prof=prof, seconds_profiled=dt_prof,
                         tiles=pr.last_tiles("fine_step"), tiles_sweep=pr.last_tiles("fine_sweep"))
        log(f"{prec}: {args.steps} solves in {dt:.3f}s ({1e3 * dt / args.steps:.2f} ms/solve), "
            f"iterations {iters[0]}, set-up {setup:.2f}s; event-timed pass {1e3 * dt_prof / args.steps:.2f} ms/solve")
        log(f"{prec} launch timing: " + ", ".join(f"{k} {v[0]:.2f}ms/{v[1]}" for k, v in prof.items()))
        pr.close()

    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mb} MiB read + {args.calib_copy_mb} MiB written")
        del a, b

    mixed = res["mixed"]
    ms_per_step = 1e3 * mixed["seconds"] / args.steps
    value = args.steps / mixed["seconds"]

    # roofline of the dominant kernel: the fused fine-step product
    # Z_h W_h dev (the scheme's residual products (i), (iii) and the solves
    # (ii), (iv) folded into one operator), algorithmic
    # 2*(d1^2 + 4 d1 d2 + 2 d2^2) flops per column (its nonzero blocks), N
    # columns per step. With per-step launches the product kernel is timed
    # alone and its split-K reduction kernel beside it; the persistent sweep
    # (one cooperative launch for the P steps of a sweep, reductions and grid
    # synchronisations included) is timed per sweep: (P - 1) steps of flops.
    step_flops = 2.0 * (d1 * d1 + 4.0 * d1 * d2 + 2.0 * d2 * d2) * N
    step_bytes = (d1 * d1 + 4.0 * d1 * d2 + 2.0 * d2 * d2) * 4 + N * 2 * (d1 + d2) * 4
    ms_red, n_red = mixed["prof"]["splitk_reduce"]
    avg_red = (ms_red / n_red) * 1e-3 if n_red else 0.0
    if mixed["prof"]["fine_sweep"][1]:
        ms_tot, n_launch = mixed["prof"]["fine_sweep"]
        cls, tiles = "fine_sweep", tuple(mixed["tiles_sweep"])
        flops_per_launch, bytes_per_launch = (P - 1) * step_flops, (P - 1) * step_bytes
        kname = ("fine_sweep_persistent_kernel<float,%d,%d,%d> persistent fine sweep (%d fused steps, "
                 "split-K %%d, in-kernel reductions)" % (tiles[:3] + (P,))) % tiles[3]
    else:
        ms_tot, n_launch = mixed["prof"]["fine_step"]
        cls, tiles = "fine_step", tuple(mixed["tiles"])
        flops_per_launch, bytes_per_launch = step_flops, step_bytes
        kname = "gemm_nt_kernel<float,%d,%d,%d> fused fine-step product (Z W dev), split-K %d" % tiles
    avg_s = (ms_tot / n_launch) * 1e-3 if n_launch else float("nan")
    achieved = flops_per_launch / avg_s / 1e12
    traffic = MEASURED_TRAFFIC.get((args.config, cls, tiles))
    roofline = dict(kernel=kname, bound="mfma", achieved=round(achieved, 3), peak=PEAK_FP32_MFMA, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP32_MFMA, 5),
                    traffic=None if traffic is None else round(traffic),
                    avg_launch_us=round(avg_s * 1e6, 3), launches=n_launch,
                    flops_per_launch=flops_per_launch,
                    traffic_unit="bytes per launch (HBM, FETCH_SIZE+WRITE_SIZE, calibrated)",
                    algorithmic_bytes=round(bytes_per_launch))
    if cls == "fine_step":
        roofline["splitk_reduce_avg_us"] = round(avg_red * 1e6, 3)
        roofline["achieved_with_reduce"] = round(flops_per_launch / (avg_s + avg_red) / 1e12, 3)
    if traffic is not None:
        # HBM side of the same kernel: measured bytes per launch over the
        # live average duration, against the 8 TB/s HBM3E peak
        roofline["hbm_achieved_TBps"] = round(traffic / avg_s / 1e12, 3)
        roofline["hbm_frac"] = round(traffic / avg_s / 1e12 / PEAK_HBM_TBPS, 5)

    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD if args.config == "c1" else
                   ("200x200 workload of the default line with the NLMC fracture/matrix split of Section 3.2 "
                    f"(d1={d1} fracture functions, d2={d2} matrix functions), N={N} x P={P}, "
                    f"dt={p['dt']:.3e}, rel tol 1e-7" if args.config == "c1n" else args.config),
                   "name": args.config, "d1": d1, "d2": d2, "N": N, "P": P,
                   "samples": 1, "precision": "FP32 MFMA fine-step products in mass-whitened "
                   "coordinates; FP64 anchors, state, coarse sweep, jump norms and factorisations",
                   "iterations": mixed["iters"], "setup_s": round(mixed["setup"], 3)},
        "roofline": roofline,
    }
    if "fp64" in res:
        f64 = res["fp64"]
        out["fp64"] = {"value": round(args.steps / f64["seconds"], 4), "unit": "solves/s",
                       "ms_per_step": round(1e3 * f64["seconds"] / args.steps, 4),
                       "iterations": f64["iters"], "setup_s": round(f64["setup"], 3)}
        out["speedup_mixed_vs_fp64"] = round(f64["seconds"] / mixed["seconds"], 4)
        ms64, n64 = f64["prof"][cls]
        if n64:
            a64 = flops_per_launch / ((ms64 / n64) * 1e-3) / 1e12
            out["fp64"]["roofline"] = dict(bound="mfma", achieved=round(a64, 3), peak=PEAK_FP64_MFMA,
                                           unit="TFLOP/s", frac=round(a64 / PEAK_FP64_MFMA, 5))
    # peaks measured on this part (matrix-core loops, device copy) beside the
    # datasheet values the roofline fractions use
    pk = pe.probe_peaks()
    out["measured_peaks"] = {k: round(v, 2) for k, v in pk.items()}
    roofline["frac_of_measured_peak"] = round(achieved / pk["fp32_mfma_tflops"], 5)
    if "hbm_achieved_TBps" in roofline:
        roofline["hbm_frac_of_measured_copy"] = round(roofline["hbm_achieved_TBps"] / pk["hbm_copy_tbps"], 5)
    log(f"measured peaks: {pk}")
    if not args.no_setup and args.config == "c1":
        out["setup"] = setup_leg(args, torch, pe, p)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(args, torch, pe, build_problem, ["mixed"] if args.no_fp64 else ["mixed", "fp64"])
    if not args.no_cpu_baseline:
        import oracle.scheme as S
        log("cpu baseline: FP64 oracle parareal on the host ...")
        cb = cpu_baseline(p, tol)
        log(f"cpu baseline: {cb['seconds']:.1f}s, K={cb['K']}, threads={cb['threads']} ({cb['blas']})")
        out["cpu_baseline"] = {"value": round(1.0 / cb["seconds"], 6), "unit": "solves/s",
                               "cores": cb["threads"], "kind": "oracle",
                               "sample": "one full solve of the same workload (FP64 NumPy/SciPy "
                                         f"parareal, {cb['K']} iterations, intervals as matrix "
                                         f"columns), {cb['seconds']:.1f}s"}
        errs = {k: S.rel_l2_M(cb["bl"], v["X"], cb["X"]) for k, v in res.items()}
        out["rel_l2_vs_oracle"] = {k: float(f"{v:.3e}") for k, v in errs.items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
