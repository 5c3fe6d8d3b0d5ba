#!/usr/bin/env python3
"""Benchmark of the CPD hot path on one MI355X.

Workload (the 200^3 configuration): dense 200 x 200 x 200 FP32 tensor, planted rank R = 20 with
factor columns of pairwise correlation 0.5 (N(0,1) base, Cholesky mixing), Gaussian noise at
40 dB SNR; full Tensor Fox pipeline on the GPU: MLSVD compression -> dGN with PCG on the core ->
uncompression, with the thesis's defaults (maxiter 200, tol 1e-6, random CG caps).

One "step" is one complete cpd_solve on the resident tensor.  `value` is the seconds per solve
(time to the solver's stopping rule; at 40 dB the core error floor is ~3e-4, so the 1e-6 error
test cannot fire and the improvement test ends the run; the 50^3 workload, whose noise is
1e-6, reports its time to rel. err 1e-6 in `time_to_1e-6_s_50cube`).

Extra fields: per-kernel times from HIP events recorded on the launch stream inside the timed
region, the roofline of the dominant kernel, MTTKRP and Gram TFLOP/s on the same tensor, and the
FP64 CPU oracle timed on a bounded sample of the workload.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "fp64_TFLOPs": 78.6, "fp32_TFLOPs": 157.3, "bf16_TFLOPs": 2500.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-solve", action="store_true", help="skip the kernel-level extras")
    ap.add_argument("--legs", default="50cube,kernels,batch,600cube,learned",
                    help="comma list of the extra legs to run after the timed solves")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 512 MiB three times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


# HBM bytes per launch of a kernel, measured with two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch) over `bench.py --only-solve` and scaled by the same counters' reading
# for a plain copy of known size (`bench.py --copy-calibration`).  A figure is reported only while
# the kernel's sources hash to the digest it was taken with.
TRAFFIC = {
    # dgn_kernel on the 200^3 R = 20 workload (20^3 core, 19 iterations): FETCH_SIZE 72.5 KiB x 2.0,
    # WRITE_SIZE 29.56 KiB x 1.0 (profiles/dgn_kernel_200cube_traffic.md)
    "dgn": {"bytes": 148480 + 30272, "sources": ['dgn.hip', 'dgn_state.h', 'mfma_f64.h', 'common.h'], "digest": 'ad823d5eb81f4c75'},
}


def source_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2110_05997_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_of(kernel):
    t = TRAFFIC.get(kernel)
    if t is None or source_digest(t["sources"]) != t["digest"]:
        return None
    return t["bytes"]


def copy_calibration():
    import torch
    n = 64 << 20                       # 64 Mi doubles = 512 MiB each way
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.neg(a, out=b)            # one elementwise kernel: reads 512 MiB, writes 512 MiB
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_kib_each_way": n * 8 / 1024, "launches": 3}), flush=True)


def dgn_flops(core, R, log):
    """Algorithmic FP64 flops of the dGN kernel: per iteration the fused residual + 3 MTTKRPs
    (4 passes of R~1 R~2 R~3 R FMAs), three R~ x R x R Grams, and per CG iteration (plus one for
    J^T J x) the structured product: 3 Q products + 3 V Pi + 3 W Y, each R~ R^2 FMAs."""
    d = sum(core)
    n3 = core[0] * core[1] * core[2]
    per_it = 2 * (4 * n3 * R + d * R * R)
    hv = 2 * 3 * d * R * R
    return sum(per_it + (e["cg_iters"] + 1) * hv for e in log)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(see DESIGN.md for how the work would shard)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    import numpy as np
    import torch

    import paper_2110_05997_amd as cp
    import synth

    dev = torch.device("cuda:0")
    R, maxiter = 20, 200
    T, _, _ = synth.config2()
    Td = torch.as_tensor(T).to(dev)
    U = synth.cg_uniforms(maxiter, 0)
    _, _, _, core = cp.compress(Td, R)
    W0 = [torch.as_tensor(w).to(dev) for w in synth.init_factors(core, R, 0)]
    W0f = cp.flat_w0(W0, Td.device)   # concatenated once, outside the timed steps
    p = cp.params(maxiter=maxiter, cg_uniforms=U)
    ws = torch.empty(cp.workspace_bytes(Td.shape, R, p), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        cp.solve(Td, R, p, W0=W0f, ws=ws)
    torch.cuda.synchronize()

    # timed steps: HIP events around the dominant kernel only (the roofline's live measurement), so
    # that event recording for the other kernels stays out of the measured step
    cp.profile_reset()
    cp.profile_enable(True, kernels=["dgn"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = cp.solve(Td, R, p, W0=W0f, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cp.profile_enable(False)
    prof_dgn = cp.profile_read()["dgn"]
    info = res["info"]
    ms_per_step = 1000.0 * (t1 - t0) / args.steps
    # per-kernel breakdown: the same steps again, untimed, with every kernel's events
    cp.profile_reset()
    cp.profile_enable(True)
    for _ in range(args.steps):
        cp.solve(Td, R, p, W0=W0f, ws=ws)
    torch.cuda.synchronize()
    cp.profile_enable(False)
    prof = cp.profile_read()
    prof["dgn"] = prof_dgn

    # dGN trajectory of the last solve (same inputs every step) for the flop count
    Us, _, S, _ = cp.compress(Td, R, p)
    st = cp.DgnState(S, R, p, W0=W0, t_norm2=float(info["t_norm"]) ** 2)
    iters, stop, log = st.run()
    torch.cuda.synchronize()

    N = 200 ** 3
    kernels = {}
    for name, (n, ms) in prof.items():
        if n:
            kernels[name] = {"launches_per_step": n / args.steps, "avg_ms": ms / n,
                             "ms_per_step": ms / args.steps}
    # algorithmic work per launch
    work = {
        "gram": ("mfma", N * (200 + 1), "fp64_TFLOPs"),             # upper-triangle SYRK flops per mode
        "dgn": ("alu", dgn_flops(core, R, log), "fp64_TFLOPs"),
        "project": ("hbm", N * 4, "hbm_GBs"),                       # reads the FP32 tensor once
        "residual": ("hbm", N * 4, "hbm_GBs"),
    }
    dominant = max((k for k in kernels if k in work), key=lambda k: kernels[k]["ms_per_step"])
    bound, units, peak_key = work[dominant]
    avg_s = kernels[dominant]["avg_ms"] / 1000.0
    if bound == "hbm":
        achieved, unit = units / avg_s / 1e9, "GB/s"
    else:
        achieved, unit = units / avg_s / 1e12, "TFLOP/s"
    peak = PEAK[peak_key]
    roofline = {"kernel": dominant, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": traffic_of(dominant),
                "algorithmic_per_launch": units}

    out = {
        "metric": "CPD time-to-rel-err 1e-6 (s), MTTKRP TFLOP/s; learned vs plain init, 1 GPU",
        "value": ms_per_step / 1000.0,
        "unit": "s per CPD solve",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (FP32 input promoted; FP64 MFMA Grams, FP64 dGN)",
        "data": "synthetic planted rank-20 tensor",
        "config": {"workload": "dense 200x200x200 FP32, planted R=20, column correlation 0.5, SNR 40 dB; "
                               "MLSVD compression + dGN/PCG + uncompression", "R": R, "maxiter": maxiter,
                   "tol": 1e-6, "parallelism": "single GPU"},
        "solve": {"iters": info["iters"], "stop": cp.STOP_NAMES[info["stop_reason"]],
                  "core_dims": list(info["core_dims"]), "rel_err_core": info["rel_err_core"],
                  "rel_err_full": info["rel_err_full"]},
        "kernels": kernels,
        "roofline": roofline,
    }

    legs = set() if args.only_solve else set(args.legs.split(","))
    if "50cube" in legs:
        # 50^3 workload: time to rel. err 1e-6 (the solve stops at the first iteration below 1e-6)
        T1, _, _ = synth.config1()
        T1d = torch.as_tensor(T1).to(dev)
        _, _, _, c1 = cp.compress(T1d, 5)
        p1 = cp.params(cg_uniforms=synth.cg_uniforms(200, 0))
        W01 = cp.flat_w0([torch.as_tensor(w).to(dev) for w in synth.init_factors(c1, 5, 0)], T1d.device)
        ws1 = torch.empty(cp.workspace_bytes(T1d.shape, 5, p1), dtype=torch.uint8, device=dev)
        for _ in range(2):
            cp.solve(T1d, 5, p1, W0=W01, ws=ws1)
        torch.cuda.synchronize()
        times = []
        for _ in range(10):
            a = time.perf_counter()
            r1 = cp.solve(T1d, 5, p1, W0=W01, ws=ws1)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - a)
        out["time_to_1e-6_s_50cube"] = statistics.median(times) if r1["info"]["tol_iter"] > 0 else None
        out["solve_50cube"] = {"iters": r1["info"]["iters"], "stop": cp.STOP_NAMES[r1["info"]["stop_reason"]],
                               "rel_err_core": r1["info"]["rel_err_core"]}

    if "kernels" in legs:
        # full-tensor MTTKRP and Gram throughput on the 200^3 tensor
        Wf = [torch.randn(200, R, dtype=torch.float64, device=dev) for _ in range(3)]
        for mode in range(3):   # untimed: first launches load the kernels
            cp.gram(Td, mode)
        torch.cuda.synchronize()
        cp.profile_reset()
        cp.profile_enable(True)
        for _ in range(3):
            for mode in range(3):
                cp.gram(Td, mode)
        torch.cuda.synchronize()
        cp.profile_enable(False)
        n_g, ms_g = cp.profile_read()["gram"]
        out["gram_tflops"] = N * 201 / (ms_g / n_g / 1000.0) / 1e12
        mt = mttkrp_rates(cp, torch, Td, Wf, R, [("fp32_in_f64_mfma", cp.CPD_F64), ("fp32_in_f32_mfma", cp.CPD_F32)])
        out["mttkrp_tflops"] = mt["fp32_in_f64_mfma"]["tflops"]
        out["mttkrp_200cube"] = mt

    if "batch" in legs:
        # batched solver: 512 small planted CPDs (modes U{10..64}, ranks U{2..12}, 50 dB), one graph
        Ts4, Rs4, W04 = synth.batch_members(512, seed=0)
        B = cp.Batch([torch.as_tensor(t).to(dev) for t in Ts4], Rs4, cp.params(cg_uniforms=synth.cg_uniforms(200, 0)),
                     W0=W04, graph=True)
        infos = B.run()
        btimes = []
        for _ in range(5):
            a = time.perf_counter()
            B.run(read_info=False)
            torch.cuda.synchronize()
            btimes.append(time.perf_counter() - a)
        v, vms = B.variant()
        bt = statistics.median(btimes)
        out["batch_512"] = {"cpds_per_s": 512 / bt, "ms_per_batch": 1000.0 * bt, "gram_variant": v,
                            "gram_variant_ms": vms,
                            "median_rel_err_full": float(np.median([i["rel_err_full"] for i in infos])),
                            "median_iters": float(np.median([i["iters"] for i in infos]))}
        B.close()
    if "600cube" in legs:
        out["c3_600cube"] = bench_600cube(cp, synth, torch, dev)
    if "learned" in legs:
        out["c5_learned_init"] = bench_learned(torch)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(T, R, core, U)
    print(json.dumps(out), flush=True)


def cpd_diff(a, b, torch):
    """||[[a]] - [[b]]|| / ||[[b]]|| for two normalised CPDs (W list, lam) from factor inner products."""
    def inner(x, y):
        G = (x["W"][0].T @ y["W"][0]) * (x["W"][1].T @ y["W"][1]) * (x["W"][2].T @ y["W"][2])
        return float(x["lam"] @ G @ y["lam"])
    aa, bb, ab = inner(a, a), inner(b, b), inner(a, b)
    return max(aa + bb - 2 * ab, 0.0) ** 0.5 / bb ** 0.5


def bench_600cube(cp, synth, torch, dev):
    """600^3, R = 50, N(0,1) factors, 60 dB: the precision variant (Grams from a BF16 copy on the
    BF16 matrix cores, FP32 accumulation; projection, FP64 dGN and final error from the FP32 tensor)
    next to the same path with FP64 Grams from the FP32 tensor. N(0,1) start with seed 1 (from
    seed 0 the dGN stops in a swamp near 0.2)."""
    T, _, _ = synth.config3()
    Td = torch.as_tensor(T).to(dev)
    del T
    Tlo = Td.to(torch.bfloat16).contiguous()
    p = cp.params(cg_uniforms=synth.cg_uniforms(200, 0), seed=1)
    ws = torch.empty(cp.workspace_bytes(Td.shape, 50, p), dtype=torch.uint8, device=dev)
    res = {}
    for name in ("bf16_grams", "fp64_grams"):
        times = []
        for _ in range(4):
            torch.cuda.synchronize()
            a = time.perf_counter()
            r = cp.solve_mixed(Tlo, Td, 50, p, ws=ws) if name == "bf16_grams" else cp.solve(Td, 50, p, ws=ws)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - a)
        res[name] = r
        res[name + "_s"] = statistics.median(times[1:])
    # full-tensor MTTKRP (2 R N flop per mode) and Gram (N (I+1) per mode) on the FP32 tensor and
    # its BF16 copy
    Wf = [torch.randn(600, 50, dtype=torch.float64, device=dev) for _ in range(3)]
    m32 = mttkrp_rates(cp, torch, Td, Wf, 50, [("fp32_in_f64_mfma", cp.CPD_F64), ("fp32_in_f32_mfma", cp.CPD_F32)])
    m16 = mttkrp_rates(cp, torch, Tlo, Wf, 50, [("bf16_in_f64_mfma", cp.CPD_F64), ("bf16_in_f32_mfma", cp.CPD_F32),
                                                ("bf16_in_bf16_mfma", cp.CPD_BF16)])
    rates = {"mttkrp_tflops_fp32": m32["fp32_in_f64_mfma"]["tflops"],
             "mttkrp_tflops_bf16": m16["bf16_in_f64_mfma"]["tflops"],
             "mttkrp": {**m32, **m16},
             "gram": {**gram_rates(cp, torch, Td, [("fp32_in_f64_mfma", cp.CPD_F64)]),
                      **gram_rates(cp, torch, Tlo, [("bf16_in_bf16_mfma", cp.CPD_BF16)])}}
    return {"workload": "dense 600^3 FP32 (+ BF16 copy), planted R=50, SNR 60 dB",
            **rates,
            "s_per_solve_bf16_grams": res["bf16_grams_s"], "s_per_solve_fp64_grams": res["fp64_grams_s"],
            "rel_err_full_bf16_grams": res["bf16_grams"]["info"]["rel_err_full"],
            "rel_err_full_fp64_grams": res["fp64_grams"]["info"]["rel_err_full"],
            "iters_bf16_grams": res["bf16_grams"]["info"]["iters"],
            "iters_fp64_grams": res["fp64_grams"]["info"]["iters"],
            "reconstruction_diff_bf16_vs_fp64": cpd_diff(res["bf16_grams"], res["fp64_grams"], torch)}


def gram_rates(cp, torch, X, variants, reps=2):
    """Per compute dtype: mode-l Gram time (HIP events around the partial and reduction kernels),
    TFLOP/s on N (I_l + 1) flop (the upper half of the SYRK), the fraction of that dtype's matrix
    peak, and the largest error against the FP64 Gram relative to its largest entry."""
    N = X.numel()
    peak = {cp.CPD_F64: 78.6, cp.CPD_BF16: 2500.0}
    ref = [cp.gram(X, mode) for mode in range(3)]
    res = {}
    for tag, cd in variants:
        outs = [cp.gram(X, mode, cd) for mode in range(3)]
        torch.cuda.synchronize()
        err = max(float((o - r).abs().max() / r.abs().max()) for o, r in zip(outs, ref))
        cp.profile_reset()
        cp.profile_enable(True)
        for _ in range(reps):
            for mode in range(3):
                cp.gram(X, mode, cd)
        torch.cuda.synchronize()
        cp.profile_enable(False)
        n_g, ms_g = cp.profile_read()["gram"]
        s = ms_g / n_g / 1000.0
        tf = N * (X.shape[0] + 1) / s / 1e12
        res[tag] = {"us": s * 1e6, "tflops": tf, "frac_mfma_peak": tf / peak[cd], "max_rel_err_vs_f64": err}
    return res


def mttkrp_rates(cp, torch, X, Wf, R, variants, reps=2):
    """Per compute dtype: TFLOP/s (2 R N flop per mode), tensor bytes streamed per second, the
    fraction of the matrix-core peak of that dtype and of HBM, and the largest error against the
    FP64-MFMA result relative to its largest entry (that path is the one checked against the oracle
    to 1e-12).  Times are HIP events around the whole call (factor rounding, main and reduce kernels),
    averaged over reps x 3 modes."""
    N = X.numel()
    ebytes = X.element_size()
    peak = {cp.CPD_F64: 78.6, cp.CPD_F32: 157.3, cp.CPD_BF16: 2500.0}
    ref = [cp.mttkrp(X, Wf, mode, compute_dtype=cp.CPD_F64) for mode in range(3)]
    res = {}
    for tag, cd in variants:
        outs = [cp.mttkrp(X, Wf, mode, compute_dtype=cd) for mode in range(3)]   # untimed first launches
        torch.cuda.synchronize()
        err = max(float((o - r).abs().max() / r.abs().max()) for o, r in zip(outs, ref))
        cp.profile_reset()
        cp.profile_enable(True)
        for _ in range(reps):
            for mode in range(3):
                cp.mttkrp(X, Wf, mode, compute_dtype=cd)
        torch.cuda.synchronize()
        cp.profile_enable(False)
        n_m, ms_m = cp.profile_read()["mttkrp"]
        s = ms_m / n_m / 1000.0
        tf = 2 * R * N / s / 1e12
        gbs = N * ebytes / s / 1e9
        res[tag] = {"us": s * 1e6, "tflops": tf, "frac_mfma_peak": tf / peak[cd], "tensor_GBps": gbs,
                    "frac_hbm": gbs / 8000.0, "max_rel_err_vs_f64": err}
    return res


def bench_learned(torch, n_train=8192, epochs=20, n_test=100):
    """Learned vs MLSVD-energy vs N(0,1) starting points on new planted 100^3 rank-8 tensors compressed
    to a 16^3 core: the network (4096 -> 1024 -> 1024 -> 384) is trained here on n_train solver-
    generated pairs (the full 100k-pair run is the module's own driver: python -m
    paper_2110_05997_amd.learned)."""
    from paper_2110_05997_amd import learned as lr
    t0 = time.perf_counter()
    X, T, kept = lr.make_dataset(n_train, seed=0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net, hist = lr.train(X, T, epochs=epochs, batch=256)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    summ = lr.summarize(lr.evaluate(net, n_test, seed=1))
    steps = epochs * (kept // 256)
    flops_per_step = 6 * 256 * sum(a * b for a, b in zip(net.sizes[:-1], net.sizes[1:]))
    return {"workload": "planted 100^3 rank 8 (noiseless) -> fixed 16^3 core; MLP 4096-1024-1024-384",
            "n_train_requested": n_train, "n_train_kept": kept, "data_s": t1 - t0, "train_s": t2 - t1,
            "train_tflops": steps * flops_per_step / (t2 - t1) / 1e12, "loss_first_last": [hist[0], hist[-1]],
            "n_test": n_test, "eval": summ}


def cpu_baseline(T, R, core, U):
    """FP64 oracle on the host: one full solve of the same 200^3 tensor (compression by SVD of the
    three unfoldings + dGN + uncompression), same initial point and CG caps; median of 3."""
    import numpy as np

    import synth
    from oracle import cpd as ocpd
    from oracle import dgn as odgn
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    W0 = synth.init_factors(core, R, 0)
    Th = np.asarray(T, dtype=np.float64)
    times = []
    for _ in range(3):
        a = time.perf_counter()
        ref = ocpd.solve(Th, R, odgn.Params(), W0=W0, cg_uniforms=U)
        times.append(time.perf_counter() - a)
    return {"value": statistics.median(times), "unit": "s per CPD solve", "cores": threads, "kind": "oracle",
            "sample": "3 full solves of the 200^3 workload (same inputs, init and CG caps), median",
            "iters": ref["iters"]}


if __name__ == "__main__":
    main()
