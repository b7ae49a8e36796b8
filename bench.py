#!/usr/bin/env python3
"""Benchmark of the tile SPD inverse on one MI355X.

Headline: the precision workload's FP64 cell, n = 16384, A = Q diag(lambda)
Q^T with lambda log-spaced over [1, 1e2] (Q from a seeded QR).  One step =
one explicit inversion through the whole hot path: copy-in to tiles, the
pipelined renamed three-step tile DAG on the persistent device scheduler,
copy-out.  Each timed step inverts its own pre-made copy of A, resident in
HBM.  Beside it ("precision" row), the FP64 form against the mixed-refined
forms (FP32 and BF16 tile DAGs + binary64 Newton-Schulz) at each condition
number of the workload, with each result's ||I - A X||_F / ||A||_F and error
against the analytic inverse; the same at n = 32768 ("large" row).

Prints one JSON line.  Besides the throughput it reports the roofline of
the dominant kernel (the scheduler kernel, which runs every tile task: n^3
algorithmic flops per launch, timed with HIP events on its stream), the
oracle timed on the host cores on bounded samples (all cores and one
thread), the parity of one result against the analytic inverse, and the
other workloads as rows: n = 8192 pipelined vs unpipelined and the paper's
plan variants, the batched form, the backward, the steps on their own.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6       # MI355X dense FP64 matrix peak
PEAK_FP32_TFLOPS = 157.3      # MI355X dense FP32 matrix peak
# sources that determine the scheduler kernel and the plan it runs: committed
# traffic counters are used only while these are unchanged
KERNEL_SRCS = [os.path.join(ROOT, "paper_1002_4057_amd", "csrc", f) for f in
               ("device.hip", "device.hpp", "tile_tasks.hpp", "mfma_tile.hpp", "sched_loop.hpp",
                "plan.hpp", "plan.cpp", "api.cpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sched_kernel_n16384.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_per_launch(n: int):
    """HBM bytes per scheduler launch from committed rocprofv3 counters, or
    None when they are missing, for another order, or were taken on a
    different kernel source."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    if d.get("kernel_sha256_16") != kernel_hash() or d.get("n") != n:
        return None
    return d.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def cpu_baseline(n_all: int, n_one: int, kappa: float):
    """The oracle (plain unblocked loops, binary64) on bounded samples of the
    headline construction: one inversion at n_all on every host core, one at
    n_one on one thread (the results do not depend on the thread count)."""
    import numpy as np
    import oracle
    from paper_1002_4057_amd import inputs
    oracle.build()
    out = {}
    nt0 = oracle.num_threads()
    for label, n_s, threads in (("all", n_all, nt0), ("one", n_one, 1)):
        if n_s <= 0:
            continue
        a = np.asfortranarray(inputs.spectrum(n_s, kappa, seed=0).numpy())
        oracle.set_num_threads(threads)
        t0 = time.perf_counter()
        oracle.spd_inverse_lower(a)
        dt = time.perf_counter() - t0
        out[label] = {"value": round(n_s ** 3 / dt / 1e9, 3), "cores": oracle.num_threads(),
                      "n": n_s, "s": round(dt, 1)}
    oracle.set_num_threads(nt0)
    allc, one = out.get("all"), out.get("one")
    head = allc or one
    res = {"value": head["value"], "unit": "Gflop/s", "cores": head["cores"], "kind": "oracle",
           "sample": (f"one full three-stage oracle inversion at n={head['n']} of the headline "
                      f"construction (kappa={kappa:g}) on {head['cores']} threads, "
                      f"{head['s']} s wall"),
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    if one is not None and allc is not None:
        res["one_thread"] = {"value": one["value"], "unit": "Gflop/s", "cores": 1,
                             "sample": f"one inversion at n={one['n']}, {one['s']} s wall"}
    return res


def time_events(fn, reps, prep=None, agg="mean"):
    """Milliseconds of fn() over reps (mean or median), HIP events on torch's
    current stream (the stream the library launches on); prep() runs untimed
    before each call."""
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
    return statistics.median(times) if agg == "median" else sum(times) / len(times)


def sym_from_lower_cm(buf_cm):
    """Full symmetric matrix from a column-major buffer whose lower triangle
    holds the result (buf_cm is the row-major storage, i.e. the transpose)."""
    import torch
    low = torch.tril(buf_cm.t())
    return low + torch.tril(low, -1).t()


def resid_rel(a, x):
    import torch
    n = a.shape[0]
    r = torch.eye(n, dtype=torch.float64, device=a.device) - a @ x
    return (torch.linalg.norm(r) / torch.linalg.norm(a)).item()


def precision_cells(n, q, kappas, modes, reps, work=None):
    """FP64 against the mixed-refined forms at each kappa: time to solution
    (median of reps, after one warm call), ||I - A X||_F / ||A||_F of the
    result and its relative error against the analytic inverse (both
    untimed, with library GEMMs)."""
    import torch
    import paper_1002_4057_amd as spd
    from paper_1002_4057_amd import inputs
    dev = q.device
    if work is None:
        need = max(spd.workspace_bytes(n, mode=m.partition("+")[0]) for m in modes)
        work = torch.empty(need, dtype=torch.uint8, device=dev)
    cells = {}
    for kappa in kappas:
        a, lam = inputs.spectrum_from_q(q, kappa)
        a_cm = a.t().contiguous()
        buf = torch.empty_like(a_cm)
        row = {}
        for label in modes:
            # "mode+c64": every refinement correction in binary64
            mode, _, flag = label.partition("+")
            mopts = {"correction64": 1} if flag == "c64" else {}
            log(f"[bench] precision n={n} kappa={kappa:g} {label}")
            buf.copy_(a_cm)
            rep = spd.spd_inverse_(buf.t(), mode=mode, work=work, report=True, **mopts)   # warm
            x = sym_from_lower_cm(buf)
            ref = inputs.analytic_inverse(q, lam)
            err = (torch.linalg.norm(x - ref) / torch.linalg.norm(ref)).item()
            del ref
            res = resid_rel(a, x)
            del x
            ms = time_events(lambda: spd.spd_inverse_(buf.t(), mode=mode, work=work, **mopts),
                             reps, prep=lambda: buf.copy_(a_cm), agg="median")
            cell = {"ms": round(ms, 2), "gflops": round(float(n) ** 3 / (ms / 1e3) / 1e9, 1),
                    "resid_fro_rel": res, "err_vs_analytic": err}
            if mode != "fp64":
                cell.update({"refine_iters": rep["refine_iters"], "fell_back": rep["fell_back"],
                             "converged": rep["converged"], "predicted_stop": rep["predicted"],
                             "resid0_fro_rel": rep["resid0_fro_rel"],
                             "fp32_corrections": rep["low_corrections"]})
            row[label] = cell
        if "fp64" in row:
            for label in modes:
                if label != "fp64":
                    row[label]["speedup_over_fp64"] = round(row["fp64"]["ms"] / row[label]["ms"],
                                                            3)
        cells[f"{kappa:g}"] = row
        del a, a_cm, buf
        torch.cuda.empty_cache()
    return cells


def batched_row(reps: int, mode: str = "fp64", group: int = 0, tune: bool = True):
    """Batched workload: 8192 matrices, n uniform on {16..512} (seed 0),
    A_i = B_i B_i^T / n_i + 0.1 I, in FP64 or FP32: one DAG over the batch in
    one persistent launch per step, timed eagerly and as the replay of a
    captured HIP graph (the matrices are restored untimed between steps)."""
    import numpy as np
    import torch
    import paper_1002_4057_amd as spd
    from paper_1002_4057_amd import inputs
    dev = torch.device("cuda:0")
    dtype = torch.float64 if mode == "fp64" else torch.float32
    esize = 8 if mode == "fp64" else 4
    orders = inputs.batch_orders(8192, 16, 512, seed=0)
    mats = inputs.batched_wishart(orders, seed=0, shift=0.1)
    offs = np.concatenate([[0], np.cumsum([n * n for n in orders])]).astype(np.int64)
    host = torch.empty(int(offs[-1]), dtype=dtype)
    for m, n, o in zip(mats, orders, offs[:-1]):
        host[int(o):int(o) + n * n] = m.t().reshape(-1).to(dtype)   # column-major
    src = host.to(dev)
    buf = src.clone()
    ptrs = torch.tensor([buf.data_ptr() + esize * int(o) for o in offs[:-1]], dtype=torch.int64,
                        device=dev)
    n_dev = torch.tensor(orders, dtype=torch.int32, device=dev)
    info = torch.zeros(len(orders), dtype=torch.int32, device=dev)
    opts = {"batch_group": group} if group else {}
    tuned = None
    if tune and not group:
        tuned = spd.autotune_batched(orders, mode, reps=2)
    work = spd.batched_spd_inverse_(ptrs, orders, n_dev, n_dev, mode=mode, info=info,
                                    **opts)   # warm: task lists
    torch.cuda.synchronize()
    if int(info.abs().sum()) != 0:
        raise RuntimeError("batched warm-up reported INFO != 0")
    ms = time_events(lambda: spd.batched_spd_inverse_(ptrs, orders, n_dev, n_dev, mode=mode,
                                                      work=work, info=info, **opts),
                     reps, prep=lambda: buf.copy_(src))
    # the same call captured in a HIP graph, replayed
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            spd.batched_spd_inverse_(ptrs, orders, n_dev, n_dev, mode=mode, work=work, info=info,
                                     **opts)
    torch.cuda.current_stream().wait_stream(s)
    ms_graph = time_events(g.replay, reps, prep=lambda: buf.copy_(src))
    torch.cuda.synchronize()
    if int(info.abs().sum()) != 0:
        raise RuntimeError("batched graph replay reported INFO != 0")
    flops = float(sum(float(n) ** 3 for n in orders))
    peak = PEAK_FP64_TFLOPS if mode == "fp64" else PEAK_FP32_TFLOPS
    best = min(ms, ms_graph)
    sched = (tuned or {}).get("batch_group", group)
    how = {-1: "one workgroup per matrix", -2: "one list-scheduled DAG over the batch"}.get(
        sched, f"one DAG over the batch in groups of {sched}" if sched and sched > 0
        else "the library's schedule")
    out = {"workload": "8192 SPD matrices, n uniform on [16,512] (seed 0), A_i = B_i B_i^T/n_i "
                       f"+ 0.1 I, {mode.upper()}, one persistent launch ({how})",
           "ms": round(ms, 3), "ms_graph_replay": round(ms_graph, 3),
           "matrices_per_s": round(len(orders) / (best / 1e3), 1),
           "gflops": round(flops / (best / 1e3) / 1e9, 1), "flops": flops,
           f"frac_{mode}_peak": round(flops / (best / 1e3) / 1e12 / peak, 4),
           "workspace_gb": round(work.numel() / 1e9, 2), "reps": reps, "tuned": tuned}
    del work, buf, src
    torch.cuda.empty_cache()
    return out


def c1_row(spd, n: int, reps: int, ablation: bool):
    """n = 8192, kappa = 1e4 (A = Q diag(lambda) Q^T): pipelined against
    unpipelined steps (the paper's pipelining comparison), and the paper's
    plan variants (Section 3 and its Table 1): renamed against in place, UDU
    against UUU loop order, the TRTRI(j) placement of step 2, and one device
    task per task of the paper (chain = 1), each with the planner's critical
    path in tasks."""
    import torch
    from paper_1002_4057_amd import inputs
    dev = torch.device("cuda:0")
    a, q, lam = inputs.spectrum(n, 1e4, seed=0, device=dev, return_factors=True)
    a_cm = a.t().contiguous()
    buf = a_cm.clone()
    variants = [("renamed UDU (default)", {}), ("renamed UDU, barriers between steps",
                                                {"pipelined": 0})]
    if ablation:
        variants += [("in place UDU", {"renamed": 0}), ("renamed UUU", {"loop_order": 1}),
                     ("in place UUU", {"renamed": 0, "loop_order": 1}),
                     ("renamed UDU, TRTRI(j) first", {"trtri_first": 1}),
                     ("renamed UDU, one task per paper task", {"chain": 1})]
    if ablation:
        # memory-constrained partial renaming: a fraction of the 2T copy tiles
        t = -(-n // 128)
        T = t * (t + 1) // 2
        for frac in (0.25, 0.5):
            k = int(2 * T * frac)
            variants.append((f"renamed UDU, partial renaming {int(frac * 100)}% of the copies "
                             f"({k} tiles)", {"rename_tiles": k}))
        # tree reduction of the step-2 chains (associativity, Section 4)
        for levels in (1, 2):
            variants.append((f"renamed UDU, step-2 chains as a {1 << levels}-leaf tree",
                             {"tree_levels": levels}))
            variants.append((f"renamed UUU, step-2 chains as a {1 << levels}-leaf tree",
                             {"loop_order": 1, "tree_levels": levels}))
    work = torch.empty(max(spd.workspace_bytes(n, **o) for _, o in variants), dtype=torch.uint8,
                       device=dev)
    spd.spd_inverse_(buf.t(), work=work, report=True)
    ref = inputs.analytic_inverse(q, lam)
    err = (torch.linalg.norm(sym_from_lower_cm(buf) - ref) / torch.linalg.norm(ref)).item()
    del ref, q
    flops = float(n) ** 3
    out = {"workload": f"single SPD inverse, n={n}, FP64, A=Q diag(lambda) Q^T, lambda "
                       f"log-spaced over [1,1e4]", "reps": reps, "err_vs_analytic": err}
    out["variants"] = {}
    for label, opts in variants:
        log(f"[bench] n={n} variant: {label}")
        try:
            buf.copy_(a_cm)
            rep = spd.spd_inverse_(buf.t(), work=work, report=True, **opts)   # plan + warm
            ms = time_events(lambda: spd.spd_inverse_(buf.t(), work=work, **opts), reps,
                             prep=lambda: buf.copy_(a_cm))
            out["variants"][label] = {"ms": round(ms, 3), "gflops": round(flops / ms / 1e6, 1),
                                      "critical_path_tasks": rep["critical_path"],
                                      "device_tasks": rep["tasks"],
                                      "workspace_gb": round(spd.workspace_bytes(n, **opts) / 1e9,
                                                            3)}
        except Exception as e:   # a variant that fails is reported, not fatal
            out["variants"][label] = {"error": str(e)}
    v = out["variants"]
    if "gflops" in v.get("renamed UDU, barriers between steps", {}):
        out["pipelining_gain"] = round(v["renamed UDU (default)"]["gflops"] /
                                       v["renamed UDU, barriers between steps"]["gflops"], 3)
    return out, a_cm, work


def tree_row(spd, reps: int):
    """Small orders (4 to 16 tiles per side, where the dependency chains and
    not the products bound the time): UDU and UUU loop orders with the step-2
    chains summed sequentially (the paper's plan) or as a fixed tree
    (associativity, Section 4), each against the FP64 oracle's bar through
    the analytic inverse."""
    import torch
    from paper_1002_4057_amd import inputs
    dev = torch.device("cuda:0")
    out = {"workload": "single SPD inverse, FP64, A=Q diag(lambda) Q^T, lambda log-spaced over "
                       "[1,1e4]", "reps": reps, "orders": {}}
    for n in (512, 1024, 2048):
        a, q, lam = inputs.spectrum(n, 1e4, seed=1, device=dev, return_factors=True)
        ref = inputs.analytic_inverse(q, lam)
        a_cm = a.t().contiguous()
        buf = a_cm.clone()
        work = torch.empty(spd.workspace_bytes(n, tree_levels=2), dtype=torch.uint8, device=dev)
        row = {}
        for lo, name in ((0, "UDU"), (1, "UUU")):
            for levels in (0, 1, 2):
                opts = {"loop_order": lo, "tree_levels": levels}
                log(f"[bench] tree n={n} {name} levels={levels}")
                buf.copy_(a_cm)
                rep = spd.spd_inverse_(buf.t(), work=work, report=True, **opts)
                err = (torch.linalg.norm(sym_from_lower_cm(buf) - ref) /
                       torch.linalg.norm(ref)).item()
                us = 1e3 * time_events(lambda: spd.spd_inverse_(buf.t(), work=work, **opts), reps,
                                       prep=lambda: buf.copy_(a_cm), agg="median")
                row[f"{name} tree_levels={levels}"] = {
                    "us": round(us, 1), "critical_path_tasks": rep["critical_path"],
                    "device_tasks": rep["tasks"], "err_vs_analytic": err}
        out["orders"][str(n)] = row
    return out


def steps_row(spd, a_cm, work, n: int, reps: int):
    """The steps of Algorithm 1 on their own, on the n = 8192 input: the
    Cholesky factor (step 1, n^3/3 flops), the inverse from that factor
    (steps 2 and 3 after the factor prologue, 2n^3/3 flops) and the solve
    with 128 right-hand sides."""
    b = a_cm.clone()
    spd.cholesky_(b.t(), work=work, report=True)            # plan + warm
    lsrc = b.clone()                                         # L in the lower triangle
    ms_chol = time_events(lambda: spd.cholesky_(b.t(), work=work), reps,
                          prep=lambda: b.copy_(a_cm))
    spd.inverse_from_factor_(b.t(), work=work, report=True)  # plan + warm (b holds L)
    ms_inv = time_events(lambda: spd.inverse_from_factor_(b.t(), work=work), reps,
                         prep=lambda: b.copy_(lsrc))
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
    out = {"workload": f"n={n}, FP64, the n={n} input; solve with {nrhs} right-hand sides",
           "reps": reps}
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
    row = {"workload": "backward of the inverse, n=4096, FP64 (3 n^3 flops)",
           "ms": round(ms, 3), "gflops": round(flops / (ms / 1e3) / 1e9, 1),
           "frac_fp64_peak": round(flops / (ms / 1e3) / 1e12 / PEAK_FP64_TFLOPS, 4),
           "reps": reps}
    del x, g, out, work
    # workload (b): 256 matrices of n = 256, forward and backward each one
    # batched launch
    nb, batch = 256, 256
    a = torch.stack([inputs.wishart_shift(nb, seed=k) for k in range(batch)]).to(dev)
    xs = spd.batched_spd_inverse(list(a))
    gs = [inputs.randn((nb, nb), seed=10000 + k).to(dev) for k in range(batch)]
    outs = [torch.empty((nb, nb), dtype=torch.float64, device=dev) for _ in xs]
    bwork = torch.empty(spd.batched_backward_workspace_bytes([nb] * batch), dtype=torch.uint8,
                        device=dev)
    xs = [v.contiguous() for v in xs]
    ptr = lambda ts: torch.tensor([v.data_ptr() for v in ts], dtype=torch.int64, device=dev)  # noqa
    px, pg, po = ptr(xs), ptr(gs), ptr(outs)
    nd = torch.full((batch,), nb, dtype=torch.int32, device=dev)
    orders = [nb] * batch
    spd.batched_spd_inverse_backward_(orders, nd, px, nd, pg, nd, po, nd, bwork)
    torch.cuda.synchronize()
    msb = time_events(lambda: spd.batched_spd_inverse_backward_(orders, nd, px, nd, pg, nd, po, nd,
                                                                bwork), reps)
    fb = 3.0 * float(nb) ** 3 * batch
    row["batched"] = {"workload": "backward of 256 inverses of n=256, FP64, one batched launch "
                                  "(3 n^3 flops each)",
                      "ms": round(msb, 3), "gflops": round(fb / (msb / 1e3) / 1e9, 1),
                      "frac_fp64_peak": round(fb / (msb / 1e3) / 1e12 / PEAK_FP64_TFLOPS, 4)}
    return row


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--kappa", type=float, default=1e2)
    ap.add_argument("--cpu-n", type=int, default=8192,
                    help="oracle sample order on every host core (0 = skip)")
    ap.add_argument("--cpu-n1", type=int, default=3072,
                    help="oracle sample order on one thread (0 = skip)")
    ap.add_argument("--rows", default="precision,large,c1,ablation,tree,batched,backward,steps",
                    help="extra measured rows (comma list, '' = none): precision (FP64 vs "
                         "mixed at the headline order), large (n = --large-n), c1 (n = 8192 "
                         "pipelined vs unpipelined), ablation (plan variants at n = 8192), "
                         "tree (step-2 tree reduction at small orders), batched, backward, steps")
    ap.add_argument("--kappas", default="1e2,1e6,1e10", help="precision row condition numbers")
    ap.add_argument("--modes", default="fp64,mixed_fp32,mixed_fp32+c64,mixed_bf16",
                    help="precision row modes (+c64: every refinement correction in binary64)")
    ap.add_argument("--large-n", type=int, default=32768)
    ap.add_argument("--large-kappas", default="1e2")
    ap.add_argument("--large-modes", default="fp64,mixed_fp32,mixed_bf16")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (built-in schedule choices)")
    ap.add_argument("--batch-group", type=int, default=0,
                    help="batched rows: matrices per dispatch group (0 = library choice)")
    ap.add_argument("--tuning-save", default="", metavar="FILE",
                    help="save the autotuner's table to FILE")
    ap.add_argument("--tuning-load", default="", metavar="FILE",
                    help="load a saved tuning table instead of running the autotuner")
    ap.add_argument("--input", choices=["spectrum", "wishart"], default="spectrum",
                    help="wishart (B B^T/n + I, no QR) is for profiler counter runs only")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, run a plain device copy of this many MiB (profiler scale)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the library inverts "
                                   "on one device); run it with --gpus 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    import paper_1002_4057_amd as spd
    from paper_1002_4057_amd import inputs, _lib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lib = _lib.load()
    n, K, W = args.n, args.steps, args.warmup
    wanted = [r for r in args.rows.split(",") if r]
    log(f"[bench] building input n={n} kappa={args.kappa:g} ({args.input})")
    if args.input == "spectrum":
        q = inputs.orthogonal(n, 0, device=dev)
        a, lam = inputs.spectrum_from_q(q, args.kappa)
    else:
        b0 = inputs.randn((n, n), 0).to(dev)
        a = b0 @ b0.t() / n + torch.eye(n, dtype=torch.float64, device=dev)
        a = 0.5 * (a + a.t())
        del b0
        q = lam = None
    tuned = None
    if args.tuning_load:
        # a table saved by an earlier run (the profiler runs use it, so that
        # their kernel statistics hold only the timed schedule's launches)
        spd.tuning_load(args.tuning_load)
        tuned = {"loaded_from": os.path.basename(args.tuning_load)}
    elif not args.no_tune:
        log(f"[bench] autotuning the schedule at n={n}")
        t0 = time.perf_counter()
        tuned = spd.autotune(n, reps=2)
        tuned["tuning_s"] = round(time.perf_counter() - t0, 1)
        if args.tuning_save:
            spd.tuning_save(args.tuning_save)
    a_cm = a.t().contiguous()                       # column-major storage of A
    bufs = [a_cm.clone() for _ in range(K + W)]
    work = torch.empty(spd.workspace_bytes(n), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    log(f"[bench] warmup {W}")
    rep = spd.spd_inverse_(bufs[K].t(), work=work, report=True) if W else None
    for k in range(1, W):
        spd.spd_inverse_(bufs[K + k].t(), work=work)
    torch.cuda.synchronize()
    # parity of one result (untimed) against the analytic inverse, and its residual
    parity = None
    if q is not None and W:
        x = sym_from_lower_cm(bufs[K])
        ref = inputs.analytic_inverse(q, lam)
        parity = {"rel_fro_vs_analytic": (torch.linalg.norm(x - ref) /
                                          torch.linalg.norm(ref)).item(),
                  "bar": 1e-12 * args.kappa, "resid_fro_rel": resid_rel(a, x)}
        del x, ref

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
    del bufs
    torch.cuda.empty_cache()

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
    kappas = [float(k) for k in args.kappas.split(",") if k]
    modes = [m for m in args.modes.split(",") if m]
    if "precision" in wanted and q is not None:
        del a, a_cm
        rows["precision"] = {
            "workload": f"precision form, n={n}, A = Q diag(lambda) Q^T, lambda log-spaced over "
                        "[1,kappa]; FP64 against mixed (FP32 or BF16 tile DAG, "
                        "Newton-Schulz refinement with binary64 residuals and FP32-MFMA "
                        "corrections but the last, or (+c64) every correction in binary64; "
                        "stop at ||I-AX||_F/||A||_F <= 1e-13); median of 3 after one warm call",
            "cells": precision_cells(n, q, kappas, modes, 3, work=None)}
    del q, work
    torch.cuda.empty_cache()
    if "large" in wanted and args.large_n > 0:
        nl = args.large_n
        log(f"[bench] large row n={nl}: building input")
        ql = inputs.orthogonal(nl, 0, device=dev)
        lk = [float(k) for k in args.large_kappas.split(",") if k]
        rows["large"] = {
            "workload": f"precision form at n={nl}, same construction; median of 2 after one "
                        "warm call",
            "cells": precision_cells(nl, ql, lk, [m for m in args.large_modes.split(",") if m],
                                     2)}
        del ql
        torch.cuda.empty_cache()
    if "c1" in wanted or "ablation" in wanted or "steps" in wanted:
        c1, a8_cm, work8 = c1_row(spd, 8192, max(2, min(K, 4)), "ablation" in wanted)
        rows["c1"] = c1
        if "steps" in wanted:
            log("[bench] steps row")
            rows["steps"] = steps_row(spd, a8_cm, work8, 8192, max(2, min(K, 5)))
        del a8_cm, work8
        torch.cuda.empty_cache()
    if "tree" in wanted:
        log("[bench] tree row")
        rows["tree"] = tree_row(spd, max(5, min(K, 20)))
    if "batched" in wanted:
        log("[bench] batched row (FP64)")
        rows["batched"] = batched_row(max(2, min(K, 5)), "fp64", args.batch_group,
                                      not args.no_tune)
        log("[bench] batched row (FP32)")
        rows["batched_fp32"] = batched_row(max(2, min(K, 5)), "fp32", args.batch_group,
                                           not args.no_tune)
    if "backward" in wanted:
        log("[bench] backward row")
        rows["backward"] = backward_row(max(2, min(K, 5)))

    cpu = None
    if args.cpu_n > 0 or args.cpu_n1 > 0:
        log(f"[bench] oracle samples n={args.cpu_n} (all cores), n={args.cpu_n1} (one thread)")
        cpu = cpu_baseline(args.cpu_n, args.cpu_n1, args.kappa)

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
        "config": {"workload": f"precision workload, FP64 cell: single SPD inverse, n={n}, "
                               f"A=Q diag(lambda) Q^T, lambda log-spaced over "
                               f"[1,{args.kappa:g}]",
                   "n": n, "nb": rep["nb"] if rep else None, "kappa": args.kappa,
                   "variant": "renamed, UDU, pipelined",
                   "workers": rep["workers"] if rep else None, "tuned": tuned},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                     "traffic": traffic_per_launch(n), "kernel": "sched_kernel",
                     "kernel_ms": round(sched_avg_s * 1e3, 3), "launches": launches.value},
        "cpu_baseline": cpu,
        "parity": parity,
        "rows": rows,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
