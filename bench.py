#!/usr/bin/env python3
"""Benchmark of the tile SPD inverse on one MI355X.

One step = one explicit inversion of the n = 8192 matrix A = Q diag(lambda) Q^T
(lambda log-spaced over [1, 1e4], Q from a seeded QR) through the whole hot
path: copy-in to tiles, the pipelined renamed three-step tile DAG on the
persistent device scheduler, copy-out.  Each timed step inverts its own
pre-made copy of A that is already resident in HBM.

Prints one JSON line (rank 0).  Besides the throughput it reports the
roofline of the dominant kernel (the scheduler kernel, which runs every tile
task: n^3 algorithmic flops per launch, timed with HIP events on its stream),
the oracle timed on the host cores on a bounded sample, the parity of one
result against the analytic inverse, and pipelined vs unpipelined throughput.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6       # MI355X dense FP64 matrix peak
# sources that determine the scheduler kernel and the plan it runs: committed
# traffic counters are used only while these are unchanged
KERNEL_SRCS = [os.path.join(ROOT, "paper_1002_4057_amd", "csrc", f) for f in
               ("device.hip", "device.hpp", "tile_tasks.hpp", "mfma_tile.hpp", "sched_loop.hpp",
                "plan.hpp", "plan.cpp", "api.cpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sched_kernel_n8192.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per scheduler launch from committed rocprofv3 counters, or
    None when they are missing or were taken on a different kernel source."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    if d.get("kernel_sha256_16") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(n_sample: int, kappa: float):
    import numpy as np
    import oracle
    from paper_1002_4057_amd import inputs
    import torch
    a = inputs.spectrum(n_sample, kappa, seed=0, device="cuda").cpu().numpy()
    torch.cuda.synchronize()
    oracle.build()
    t0 = time.perf_counter()
    oracle.spd_inverse_lower(np.asfortranarray(a))
    dt = time.perf_counter() - t0
    return {"value": round(n_sample ** 3 / dt / 1e9, 3), "unit": "Gflop/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one full three-stage oracle inversion at n={n_sample} "
                      f"(same construction, kappa={kappa:g}), {dt:.1f} s wall"}


def time_events(fn, reps, prep=None):
    """Average milliseconds of fn() over reps, HIP events on torch's current
    stream (the stream the library launches on); prep() runs untimed before
    each call."""
    import torch
    times = []
    for _ in range(reps):
        if prep is not None:
            prep()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return sum(times) / len(times)


def batched_row(reps: int):
    """Batched workload: 8192 matrices, n uniform on {16..512} (seed 0),
    A_i = B_i B_i^T / n_i + 0.1 I, one persistent launch per step."""
    import numpy as np
    import torch
    import paper_1002_4057_amd as spd
    from paper_1002_4057_amd import inputs
    dev = torch.device("cuda:0")
    orders = inputs.batch_orders(8192, 16, 512, seed=0)
    mats = inputs.batched_wishart(orders, seed=0, shift=0.1)
    offs = np.concatenate([[0], np.cumsum([n * n for n in orders])]).astype(np.int64)
    host = torch.empty(int(offs[-1]), dtype=torch.float64)
    for m, n, o in zip(mats, orders, offs[:-1]):
        host[int(o):int(o) + n * n] = m.t().reshape(-1)   # column-major
    src = host.to(dev)
    buf = src.clone()
    ptrs = torch.tensor([buf.data_ptr() + 8 * int(o) for o in offs[:-1]], dtype=torch.int64,
                        device=dev)
    n_dev = torch.tensor(orders, dtype=torch.int32, device=dev)
    info = torch.zeros(len(orders), dtype=torch.int32, device=dev)
    work = spd.batched_spd_inverse_(ptrs, orders, n_dev, n_dev, info=info)   # warm: plans
    torch.cuda.synchronize()
    if int(info.abs().sum()) != 0:
        raise RuntimeError("batched warm-up reported INFO != 0")
    ms = time_events(lambda: spd.batched_spd_inverse_(ptrs, orders, n_dev, n_dev, work=work,
                                                      info=info),
                     reps, prep=lambda: buf.copy_(src))
    flops = float(sum(float(n) ** 3 for n in orders))
    return {"workload": "8192 SPD matrices, n uniform on [16,512] (seed 0), A_i = B_i B_i^T/n_i "
                        "+ 0.1 I, FP64, one persistent launch",
            "ms": round(ms, 3), "matrices_per_s": round(len(orders) / (ms / 1e3), 1),
            "gflops": round(flops / (ms / 1e3) / 1e9, 1), "flops": flops,
            "frac_fp64_peak": round(flops / (ms / 1e3) / 1e12 / PEAK_FP64_TFLOPS, 4),
            "reps": reps}


def ablation_row(spd, bufs, work, n: int, reps: int):
    """The paper's plan variants on the same n (Section 3 and its Table 1):
    renamed against in place, UDU against UUU loop order, the TRTRI(j)
    placement of step 2, and one device task per task of the paper
    (chain = 1), each with the planner's critical path in tasks.  Same
    synthetic input as the headline line; each variant is warmed once."""
    import torch
    variants = [("renamed UDU (default)", {}), ("in place UDU", {"renamed": 0}),
                ("renamed UUU", {"loop_order": 1}), ("in place UUU", {"renamed": 0, "loop_order": 1}),
                ("renamed UDU, TRTRI(j) first", {"trtri_first": 1}),
                ("renamed UDU, one task per paper task", {"chain": 1})]
    out = {"workload": f"single SPD inverse, n={n}, FP64 (same input as the headline line)",
           "reps": reps, "variants": {}}
    flops = float(n) ** 3
    for label, opts in variants:
        try:
            b = bufs[0].t().clone()
            rep = spd.spd_inverse_(b, work=work, report=True, **opts)   # plan + warm
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            for k in range(reps):
                spd.spd_inverse_(bufs[k].t(), work=work, **opts)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - s0) / reps * 1e3
            out["variants"][label] = {"ms": round(ms, 3), "gflops": round(flops / ms / 1e6, 1),
                                      "critical_path_tasks": rep["critical_path"],
                                      "device_tasks": rep["tasks"]}
        except Exception as e:   # a variant that fails is reported, not fatal
            out["variants"][label] = {"error": str(e)}
    return out


def steps_row(spd, a_cm, work, n: int, reps: int):
    """The steps of Algorithm 1 on their own, on the headline input: the
    Cholesky factor (step 1, n^3/3 flops) and the inverse from that factor
    (steps 2 and 3 after the factor prologue, 2n^3/3 flops)."""
    b = a_cm.clone()
    spd.cholesky_(b.t(), work=work, report=True)            # plan + warm
    lsrc = b.clone()                                         # L in the lower triangle
    ms_chol = time_events(lambda: spd.cholesky_(b.t(), work=work), reps,
                          prep=lambda: b.copy_(a_cm))
    spd.inverse_from_factor_(b.t(), work=work, report=True)  # plan + warm (b holds L)
    ms_inv = time_events(lambda: spd.inverse_from_factor_(b.t(), work=work), reps,
                         prep=lambda: b.copy_(lsrc))
    # the solve A X = B (factor, then both substitutions) for 128 right-hand
    # sides, n^3/3 + 2 n^2 nrhs flops
    import torch
    nrhs = 128
    bsrc = torch.randn(nrhs, n, dtype=torch.float64, device=a_cm.device)  # column-major n x nrhs
    bb = bsrc.clone()
    spd.solve_(b.t(), bb.t(), report=True)                    # plan + warm
    swork = torch.empty(spd.solve_workspace_bytes(n, nrhs), dtype=torch.uint8,
                        device=a_cm.device)

    def prep_solve():
        b.copy_(a_cm)
        bb.copy_(bsrc)
    ms_solve = time_events(lambda: spd.solve_(b.t(), bb.t(), work=swork), reps, prep=prep_solve)
    out = {"workload": f"n={n}, FP64, same input as the headline line; solve with {nrhs} "
                       "right-hand sides", "reps": reps}
    for key, ms, fl in (("cholesky", ms_chol, n ** 3 / 3.0), ("inverse_from_factor", ms_inv,
                                                                2.0 * n ** 3 / 3.0),
                        ("solve", ms_solve, n ** 3 / 3.0 + 2.0 * n * n * nrhs)):
        out[key] = {"ms": round(ms, 3), "gflops": round(fl / ms / 1e6, 1),
                    "frac_fp64_peak": round(fl / ms / 1e9 / PEAK_FP64_TFLOPS, 4)}
    return out


def backward_row(reps: int):
    """Differentiation workload (a): grad_A = -X sym(G) X at n = 4096."""
    import torch
    import paper_1002_4057_amd as spd
    from paper_1002_4057_amd import inputs
    dev = torch.device("cuda:0")
    n = 4096
    a = inputs.wishart_shift(n, seed=0).to(dev)
    g = inputs.randn((n, n), seed=1).to(dev)
    x = spd.spd_inverse(a)
    out = torch.empty_like(x)
    work = torch.empty(spd.backward_workspace_bytes(n), dtype=torch.uint8, device=dev)
    spd.spd_inverse_backward(x, g, work=work, out=out)
    torch.cuda.synchronize()
    ms = time_events(lambda: spd.spd_inverse_backward(x, g, work=work, out=out), reps)
    flops = 3.0 * float(n) ** 3
    return {"workload": "backward of the inverse, n=4096, FP64 (3 n^3 flops)",
            "ms": round(ms, 3), "gflops": round(flops / (ms / 1e3) / 1e9, 1),
            "frac_fp64_peak": round(flops / (ms / 1e3) / 1e12 / PEAK_FP64_TFLOPS, 4),
            "reps": reps}


def mixed_row(reps: int, n: int = 16384, kappa: float = 1e2):
    """Precision workload: FP64 form vs mixed-refined form (FP32 tile DAG +
    binary64 Newton-Schulz) at n = 16384, kappa = 1e2, time to solution of
    each and ||I - A X||_F / ||A||_F of each result (measured untimed with a
    library GEMM)."""
    import torch
    import paper_1002_4057_amd as spd
    from paper_1002_4057_amd import inputs
    dev = torch.device("cuda:0")
    a, q, lam = inputs.spectrum(n, kappa, seed=0, device="cuda", return_factors=True)
    del q, lam
    a_cm = a.t().contiguous()
    need = max(spd.workspace_bytes(n), spd.workspace_bytes(n, mode="mixed_fp32"))
    work = torch.empty(need, dtype=torch.uint8, device=dev)
    buf = a_cm.clone()
    anorm = torch.linalg.norm(a).item()

    def resid():
        low = torch.tril(buf.t())
        x = low + torch.tril(low, -1).t()
        r = torch.eye(n, dtype=torch.float64, device=dev) - a @ x
        return (torch.linalg.norm(r) / anorm).item()

    out = {"workload": f"precision form, n={n}, A = Q diag(lambda) Q^T, lambda log-spaced over "
                       f"[1,{kappa:g}]; FP64 vs mixed (FP32 tiles + binary64 refinement, "
                       f"stop at ||I-AX||_F/||A||_F <= 1e-13)"}
    reports = {}
    for label, mode in (("fp64", "fp64"), ("mixed_fp32", "mixed_fp32")):
        buf.copy_(a_cm)
        reports[label] = spd.spd_inverse_(buf.t(), mode=mode, work=work, report=True)   # warm
        ms = time_events(lambda: spd.spd_inverse_(buf.t(), mode=mode, work=work, report=True),
                         reps, prep=lambda: buf.copy_(a_cm))
        out[label] = {"ms": round(ms, 2), "gflops": round(float(n) ** 3 / (ms / 1e3) / 1e9, 1),
                      "resid_fro_rel": resid()}
    rep = reports["mixed_fp32"]
    out["mixed_fp32"].update({"refine_iters": rep["refine_iters"], "fell_back": rep["fell_back"],
                              "resid0_fro_rel": rep["resid0_fro_rel"]})
    out["speedup_mixed_over_fp64"] = round(out["fp64"]["ms"] / out["mixed_fp32"]["ms"], 3)
    out["reps"] = reps
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--kappa", type=float, default=1e4)
    ap.add_argument("--cpu-n", type=int, default=8192, help="oracle sample order (0 = skip)")
    ap.add_argument("--no-unpipelined", action="store_true")
    ap.add_argument("--rows", default="batched,backward,mixed,ablation,steps",
                    help="extra measured rows: batched, backward, mixed, ablation, steps "
                         "(comma list, '' = none)")
    ap.add_argument("--input", choices=["spectrum", "wishart"], default="spectrum",
                    help="wishart (B B^T/n + I, no QR) is for profiler counter runs only")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, run a plain device copy of this many MiB (profiler scale)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    import paper_1002_4057_amd as spd
    from paper_1002_4057_amd import inputs, _lib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lib = _lib.load()
    n, K, W = args.n, args.steps, args.warmup
    log(f"[bench] building input n={n} kappa={args.kappa:g} ({args.input})")
    if args.input == "spectrum":
        a, q, lam = inputs.spectrum(n, args.kappa, seed=0, device="cuda", return_factors=True)
    else:
        b0 = inputs.randn((n, n), 0).to(dev)
        a = b0 @ b0.t() / n + torch.eye(n, dtype=torch.float64, device=dev)
        a = 0.5 * (a + a.t())
        del b0
        q = lam = None
    a_cm = a.t().contiguous()                       # column-major storage of A
    bufs = [a_cm.clone() for _ in range(K + W)]
    work = torch.empty(spd.workspace_bytes(n), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    log(f"[bench] warmup {W}")
    for k in range(W):
        spd.spd_inverse_(bufs[K + k].t(), work=work)
    torch.cuda.synchronize()
    # parity of one result (untimed) against the analytic inverse
    rel = None
    if q is not None:
        x = bufs[K].t()                               # lower triangle holds A^{-1}
        ref = inputs.analytic_inverse(q, lam)
        low = torch.tril(x)
        xs = low + torch.tril(low, -1).t()
        rel = (torch.linalg.norm(xs - ref) / torch.linalg.norm(ref)).item()
        del xs, low, ref

    log(f"[bench] timing {K} steps")
    lib.spdinv_kernel_timer(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        spd.spd_inverse_(bufs[k].t(), work=work)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches = ctypes.c_longlong()
    sched_ms = lib.spdinv_kernel_timer_read(ctypes.byref(launches))
    lib.spdinv_kernel_timer(0)
    elapsed = t1 - t0
    flops = float(n) ** 3
    value = K * flops / elapsed / 1e9
    sched_avg_s = sched_ms / 1e3 / max(1, launches.value)
    achieved = flops / sched_avg_s / 1e12

    pipe = None
    if not args.no_unpipelined:
        reps = max(2, min(K, 4))
        res = {}
        for label, piped in (("pipelined", 1), ("unpipelined", 0)):
            spd.spd_inverse_(bufs[0].t().clone(), work=work, pipelined=piped)   # plan + warm
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            for k in range(reps):
                spd.spd_inverse_(bufs[k].t(), work=work, pipelined=piped)
            torch.cuda.synchronize()
            res[label] = round(reps * flops / (time.perf_counter() - s0) / 1e9, 1)
        pipe = {"pipelined_gflops": res["pipelined"], "unpipelined_gflops": res["unpipelined"],
                "steps": reps}

    ablation = None
    if "ablation" in [r for r in args.rows.split(",") if r]:
        log("[bench] ablation row")
        ablation = ablation_row(spd, bufs, work, n, max(2, min(K, 3)))

    if args.calibrate_copy > 0:
        # plain copy of known size, for scaling profiler byte counters
        nel = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calibrate_copy} MiB done")
        del src, dst

    rows = {}
    wanted = [r for r in args.rows.split(",") if r]
    if "batched" in wanted:
        log("[bench] batched row")
        rows["batched"] = batched_row(max(2, min(K, 5)))
    if "backward" in wanted:
        log("[bench] backward row")
        rows["backward"] = backward_row(max(2, min(K, 5)))
    if "mixed" in wanted:
        log("[bench] mixed row")
        rows["mixed"] = mixed_row(max(2, min(K, 3)))
    if ablation is not None:
        rows["ablation"] = ablation
    if "steps" in wanted:
        log("[bench] steps row")
        rows["steps"] = steps_row(spd, a_cm, work, n, max(2, min(K, 5)))

    cpu = None
    if args.cpu_n > 0:
        log(f"[bench] oracle sample n={args.cpu_n}")
        cpu = cpu_baseline(args.cpu_n, args.kappa)

    line = {
        "metric": "SPD-inverse Gflop/s (n^3 flops), FP64 vs mixed-refined at equal ‖I-AX‖",
        "value": round(value, 1),
        "unit": "Gflop/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(elapsed / K * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"single SPD inverse, n={n}, FP64, A=Q diag(lambda) Q^T, "
                               f"lambda log-spaced over [1,{args.kappa:g}]",
                   "n": n, "nb": 128, "kappa": args.kappa,
                   "variant": "renamed, UDU, pipelined"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                     "traffic": traffic_per_launch(), "kernel": "sched_kernel",
                     "kernel_ms": round(sched_avg_s * 1e3, 3)},
        "cpu_baseline": cpu,
        "parity": ({"rel_fro_vs_analytic": rel, "bar": 1e-12 * args.kappa} if rel is not None
                   else None),
        "pipelining": pipe,
        "rows": rows,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
