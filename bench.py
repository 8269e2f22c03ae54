"""Benchmark: PLS + RREF of a dense random 65536 x 65536 GF(2) matrix on one MI355X.

One step = gf2_pls (recursive PLS, MMPF base case, Schur products on fp4 MFMA)
followed by gf2_rref on a fresh copy of the input already resident in HBM
(every step has its own pristine copy, staged before the timed region).

Prints ONE JSON line.  value = GF(2) operations per second, with the
operation count 2*W, W = m n r - (m + n) r^2 / 2 + r^3 / 3 the classical
multiply-add count of a rank-r PLS (2 n^3 / 3 for a full-rank square matrix).
roofline: the dominant kernel (the MFMA Schur product): its algorithmic
operations 2*M*N*K per launch over its mean launch time, timed with HIP events
on the launch stream during the timed steps, against the dense matrix-core peak
of the operand type the schedule uses (fp4 by default, int8 on request).
int8_product: the same workload and schedule with the int8 matrix-core product
instead of fp4 (step time, GF(2) ops/s, and its product roofline against the
int8 dense peak); skipped with --no-int8 or an explicit --sched.
cpu_baseline: the CPU oracle (Gaussian PLS, Appendix A) timed on a smaller
matrix of the same kind on this host.
batched: the batched workload (4096 matrices, m and n log-uniform in
[64, 2048], density in {0.5, 0.1, 0.01}, planted rank in [min/2, min],
seed 7) decomposed by one persistent launch captured in a HIP graph, with
the fixed default schedule and with the learned cost model's per-matrix
schedules; matrices per second from HIP events around each graph replay
(inputs restored from a pristine copy between replays, outside the timing).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X dense matrix-core peaks (TOP/s) of the product's operand types
MFMA_PEAK_TOPS = {1: ("i8", 5000.0), 2: ("fp4", 10100.0)}

# HBM traffic of the product kernel per launch (bytes), from two rocprofv3 PMC
# passes over one step (FETCH_SIZE, then WRITE_SIZE), each scaled by what the
# counter reads for a 1 GiB plain copy in the same run (x2 and x1).  Valid only
# for the kernel source and operand type it was taken with (SHA-256 prefix,
# schur code); otherwise null.
PMC_TRAFFIC = {"source": "paper_1006_1744_amd/csrc/k_mfma.hip", "sha256_16": "6540eb0fa1bb053d",
               "schur": 2, "bytes_per_launch": 72191526,
               "profile": "profiles/gemm_mfma_traffic_65536.md"}


def pmc_traffic(schur: int):
    import hashlib
    if schur != PMC_TRAFFIC["schur"]:
        return None
    path = os.path.join(ROOT, PMC_TRAFFIC["source"])
    with open(path, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != PMC_TRAFFIC["sha256_16"]:
            return None
    return PMC_TRAFFIC["bytes_per_launch"]


def classical_ops(m: int, n: int, r: int) -> float:
    w = m * n * r - (m + n) * r * r / 2.0 + r ** 3 / 3.0
    return 2.0 * w


def cpu_baseline(n: int, seed: int) -> dict:
    import oracle
    import synth
    A = synth.random_half(n, n, seed)
    t0 = time.perf_counter()
    r, P, Q, Ap = oracle.pls(A, n, n)
    dt = time.perf_counter() - t0
    return {"value": classical_ops(n, n, r) / dt, "unit": "GF(2) ops/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"Gaussian PLS (C, OpenMP) of one {n}x{n} Bernoulli(1/2) matrix, seed {seed}: "
                      f"{dt:.2f} s, rank {r}"}


def batched_leg(g, torch, reps: int) -> dict:
    import synth
    from paper_1006_1744_amd import costmodel as cmod
    items = synth.batch_shapes(4096, 7)
    host = [synth.batch_matrix(it) for it in items]
    sizes = [a.size for a in host]
    flat = torch.empty(sum(sizes), dtype=torch.int64, device="cuda")
    mats, off = [], 0
    for a in host:
        v = flat[off:off + a.size].view(a.shape)
        v.copy_(g.to_device(a))
        mats.append(v)
        off += a.size
    pristine = flat.clone()
    b = g.Batch(mats, [(it.m, it.n) for it in items])
    cm = cmod.CostModel.load()
    learned = cm.predict(cmod.mix_features(items))
    out = {"workload": "4096 matrices, m,n log-uniform [64,2048], p in {0.5,0.1,0.01}, "
                       "planted rank in [min/2,min], seed 7",
           "graph": True}
    for name, per in (("default", None), ("learned", learned)):
        b.per_item = per
        flat.copy_(pristine)
        b.run()
        torch.cuda.synchronize()
        flat.copy_(pristine)
        stream = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=stream):
            b.run()
        ts = []
        for _ in range(reps):
            flat.copy_(pristine)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            graph.replay()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = sorted(ts)[len(ts) // 2]
        out[f"{name}_ms"] = round(ms, 3)
        out[f"{name}_matrices_per_s"] = round(4096 / ms * 1e3, 1)
        del graph
    b.per_item = None
    out["matrices_per_s"] = out["learned_matrices_per_s"]
    out["unit"] = "matrices/s"
    out["schedule"] = "learned per matrix (cost model), default for comparison"
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-n", type=int, default=57344)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-rref", action="store_true")
    ap.add_argument("--sched", type=str, default="")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-int8", action="store_true",
                    help="skip the second leg that times the same workload with the int8 product")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, one plain device copy of this many MiB (a known-size "
                         "dispatch that calibrates hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        return 2

    import torch

    import paper_1006_1744_amd as g
    import synth

    torch.cuda.set_device(0)
    n = m = args.n
    s = None
    if args.sched:
        k, t, c, sc = (int(x) for x in args.sched.split(","))
        s = g.Sched(k, t, c, sc)
    A = synth.random_half(m, n, args.seed)
    host = g.to_device(A, "cpu")
    del A
    ws = g.workspace(max(g.pls_workspace_bytes(m, n, s), g.rref_workspace_bytes(m, n)))
    P = torch.empty(m, dtype=torch.int32, device="cuda")
    Q = torch.empty(n, dtype=torch.int32, device="cuda")
    rank = torch.empty(1, dtype=torch.int32, device="cuda")
    R = torch.empty_like(host, device="cuda")

    def timed_leg(sch, steps, warmup):
        """warmup + steps PLS (+ RREF) steps under schedule sch, each on its own
        pristine device copy staged before the timed region; returns the step
        time (ms), the rank, the product-launch profile and the launch log."""
        nsteps = steps + warmup
        copies = [host.to("cuda") for _ in range(nsteps)]

        def step(i):
            g.pls(copies[i], m, n, sch, ws=ws, P=P, Q=Q, rank=rank)
            if not args.no_rref:
                g.rref(copies[i], m, n, Q, rank, R=R, ws=ws, s=sch)

        for i in range(warmup):
            step(i)
        torch.cuda.synchronize()
        g.prof_enable()
        g.prof_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(warmup, nsteps):
            step(i)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        launches = g.prof_launches()
        prof = g.prof_read()
        g.prof_disable()
        del copies
        torch.cuda.empty_cache()
        return (t1 - t0) * 1e3 / steps, int(rank.item()), prof, launches

    def product_roofline(sch, prof, launches, steps, ms):
        achieved = prof["ops"] / (prof["ms"] * 1e-3) / 1e12 if prof["ms"] > 0 else 0.0
        schur = (sch if sch is not None else g.default_sched()).schur
        if schur not in MFMA_PEAK_TOPS:
            sys.exit("bench.py: the roofline is defined for the MFMA Schur products (schur 1 or 2)")
        op_type, peak = MFMA_PEAK_TOPS[schur]
        alg_bytes = sum((M * K + N * K + 2 * M * N) / 8 for _, M, N, K in launches)
        return op_type, {
            "bound": "mfma",
            "kernel": f"gemm_dma_kernel<4> + gemm_dma_kernel<2> ({op_type} MFMA Schur product, "
                      "256x256 and 128x128 tiles)",
            "achieved": round(achieved, 1), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": pmc_traffic(schur),
            "alg_bytes_per_launch": round(alg_bytes / max(len(launches), 1)),
            "launches_per_step": prof["launches"] // max(steps, 1),
            "mean_launch_us": round(prof["ms"] * 1e3 / max(prof["launches"], 1), 2),
            "kernel_share_of_step": round(prof["ms"] / steps / ms, 3)}

    ms, r, prof, launches = timed_leg(s, args.steps, args.warmup)
    ops = classical_ops(m, n, r)
    value = ops / (ms * 1e-3)
    op_type, roofline = product_roofline(s, prof, launches, args.steps, ms)
    out = {"metric": "PLS+RREF of a dense random 65536x65536 GF(2) matrix (GF(2) ops/s)",
           "value": value, "unit": "GF(2) ops/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": f"u64/{op_type}",
           "data": "synthetic",
           "config": {"workload": f"PLS + RREF, {m}x{n} iid Bernoulli(1/2), seed {args.seed}",
                      "m": m, "n": n, "rank": r,
                      "schedule": str(s) if s is not None else str(g.default_sched())},
           "roofline": roofline}
    if not args.no_int8 and not args.sched:
        # the same workload with the int8 matrix-core product, against the int8 peak
        s0 = g.default_sched()
        s8 = g.Sched(s0.k, s0.tables, s0.cutoff, g.SCHUR_MFMA)
        ms8, r8, prof8, launches8 = timed_leg(s8, args.steps, args.warmup)
        _, roof8 = product_roofline(s8, prof8, launches8, args.steps, ms8)
        out["int8_product"] = {"schedule": str(s8), "ms_per_step": round(ms8, 3),
                               "value": classical_ops(m, n, r8) / (ms8 * 1e-3), "unit": "GF(2) ops/s",
                               "roofline": roof8}
    if not args.no_batch:
        out["batched"] = batched_leg(g, torch, max(3, args.steps))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.seed)
    if args.calib_copy_mib > 0:
        x = torch.ones(args.calib_copy_mib << 17, dtype=torch.int64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = x.numel() * 8
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
