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
(inputs restored from a pristine copy between replays, outside the timing);
also its aggregate GF(2) ops/s (sum of 2 W over the matrices / time) and HBM
GB/s (every matrix read and written once / time).
configs: one entry per further configuration and route, each timed as the
median of 3 runs after one warm-up, every run on a pristine device copy
(restored outside the timed region), wall clock with the device synchronised
around the call:
  wide_32768x131072  PLS and RREF of 32768 x 131072 Bernoulli(1/2) (seed 3),
                     each with its product roofline;
  sparse_65536       PLS + RREF of 65536^2 Bernoulli(0.01) (seed 2);
  xor_product_65536  PLS + RREF of the headline input with the XOR-popcount
                     product, its roofline against the vector-ALU peak;
  mmpf_vs_recursive_32768  PLS of 32768^2 Bernoulli(1/2) by MMPF alone and by
                     the recursion (plus the RREF);
  strips_4096        PLS + RREF of 4096^2 Bernoulli(1/2) by MMPF alone: time
                     per step and per 64-column strip;
  m4ri_4096          RREF of 4096^2 at p = 1/2 and 0.01 by M4RI, by the M+P
                     hybrid (0.15) and by PLS then RREF;
  solve_65536        64 right-hand sides solved from the headline input's PLS,
                     and a null-space basis of 16384 x 32768;
  practice_shapes    the four Table 2 shapes and densities (iid stand-ins):
                     RREF by PLS then RREF, M4RI, M+P 0.15 and M+P 0.20.
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

# Vector-ALU peak of the XOR-popcount product: 256 CUs x 64 lanes x 2.4 GHz
# = 39.3e12 32-bit lane operations/s; one v_bitop3_b32 (acc ^= a & b) covers 32
# bit products, i.e. 64 GF(2) operations (an AND and an XOR each).
VALU_LANE_OPS = 256 * 64 * 2.4e9
XOR_PEAK_TOPS = VALU_LANE_OPS * 64 / 1e12

# The paper's Table 2 (RREF of its practice matrices, 2.33 GHz Xeon E5345),
# seconds, as context for the stand-ins of the same shapes.
TABLE2_E5345_S = {"table2_row1": {"M4RI": 1.94, "PLS": 2.09, "M+P 0.15": 2.33, "M+P 0.20": 2.24},
                  "table2_row2": {"M4RI": 11.46, "PLS": 13.34, "M+P 0.15": 12.60, "M+P 0.20": 13.00},
                  "table2_row3": {"M4RI": 49.19, "PLS": 68.85, "M+P 0.15": 66.66, "M+P 0.20": 54.42},
                  "table2_row4": {"M4RI": 12.25, "PLS": 9.22, "M+P 0.15": 9.22, "M+P 0.20": 10.22}}

# HBM traffic of the product kernel per launch (bytes), from two rocprofv3 PMC
# passes over one step (FETCH_SIZE, then WRITE_SIZE), each scaled by what the
# counter reads for a 1 GiB plain copy in the same run (x2 and x1).  Valid only
# for the kernel source and operand type it was taken with (SHA-256 prefix,
# schur code); otherwise null.
PMC_TRAFFIC = {"source": "paper_1006_1744_amd/csrc/k_mfma.hip", "sha256_16": "3062ec207f4955fd",
               "schur": 2, "bytes_per_launch": 77258952,
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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_single_thread(n: int, seed: int) -> dict:
    """The oracle on one thread (a child process with OMP_NUM_THREADS=1)."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r); import oracle, synth; "
            "A = synth.random_half(%d, %d, %d); t = time.perf_counter(); "
            "r = oracle.pls(A, %d, %d)[0]; print(time.perf_counter() - t, r, oracle.threads())"
            % (ROOT, n, n, seed, n, n))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600, check=True)
    dt, r, th = res.stdout.split()[-3:]
    dt, r = float(dt), int(r)
    return {"value": classical_ops(n, n, r) / dt, "unit": "GF(2) ops/s", "cores": int(th),
            "sample": f"Gaussian PLS of one {n}x{n} Bernoulli(1/2) matrix, seed {seed}: "
                      f"{dt:.3f} s, rank {r}"}


def cpu_baseline(n: int, seed: int) -> dict:
    import oracle
    import synth
    A = synth.random_half(n, n, seed)
    t0 = time.perf_counter()
    r, P, Q, Ap = oracle.pls(A, n, n)
    dt = time.perf_counter() - t0
    del A, Ap
    return {"value": classical_ops(n, n, r) / dt, "unit": "GF(2) ops/s", "cores": oracle.threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"Gaussian PLS (C, OpenMP) of one {n}x{n} Bernoulli(1/2) matrix, seed {seed}: "
                      f"{dt:.2f} s, rank {r}",
            "single_thread_4096": cpu_single_thread(4096, seed)}


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
    learned = cm.predict_dev(cmod.batch_features(b))
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
    best_ms = min(out["default_ms"], out["learned_ms"])
    ops = sum(classical_ops(it.m, it.n, it.r) for it in items)
    moved = sum(2 * 8 * a.size for a in host)
    out["gf2_ops_per_s"] = ops / (best_ms * 1e-3)
    out["hbm_gb_per_s"] = round(moved / (best_ms * 1e-3) / 1e9, 1)
    out["hbm_frac"] = round(moved / (best_ms * 1e-3) / 8.0e12, 4)
    out["alg_bytes"] = moved
    out["matrices_per_s"] = out["learned_matrices_per_s"]
    out["unit"] = "matrices/s"
    out["schedule"] = "learned per matrix (cost model), default for comparison"
    return out


# ------------------------------------------------------------ further configs
def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def _timed(torch, prepare, body, reps=3, warmup=1):
    """Median wall time (ms) of body() over reps runs after warmup runs, each
    after prepare() (untimed), the device synchronised around the body."""
    ts = []
    for i in range(warmup + reps):
        prepare()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = body()
        torch.cuda.synchronize()
        if i >= warmup:
            ts.append((time.perf_counter() - t0) * 1e3)
    return _median(ts), out


def _product_roofline(g, schur, prof, launches):
    """The Schur products' rate over their HIP-event time against the peak of the
    unit they run on (matrix cores for fp4 / int8, vector ALUs for XOR)."""
    if prof["ms"] <= 0 or not launches:
        return None
    achieved = prof["ops"] / (prof["ms"] * 1e-3) / 1e12
    if schur in MFMA_PEAK_TOPS:
        op_type, peak = MFMA_PEAK_TOPS[schur]
        bound, kernel = "mfma", f"gemm_dma_kernel ({op_type} MFMA)"
    else:
        op_type, peak, bound, kernel = "u32", XOR_PEAK_TOPS, "alu", "gemm_xor_kernel (v_bitop3)"
    alg_bytes = sum((M * K + N * K + 2 * M * N) / 8 for _, M, N, K in launches)
    return {"bound": bound, "kernel": kernel, "achieved": round(achieved, 1),
            "peak": round(peak, 1), "unit": "TOP/s", "frac": round(achieved / peak, 4),
            "alg_bytes_per_launch": round(alg_bytes / len(launches)),
            "launches": prof["launches"], "mean_launch_us": round(prof["ms"] * 1e3 / prof["launches"], 2)}


def _pls_rref_leg(g, torch, A, m, n, s, label, profile=True):
    """PLS and RREF of A (separate event timings inside one run), median of 3."""
    src = g.to_device(A)
    work = torch.empty_like(src)
    R = torch.empty_like(src)
    ws = g.workspace(max(g.pls_workspace_bytes(m, n, s), g.rref_workspace_bytes(m, n)))
    P = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    Q = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    rank = torch.empty(1, dtype=torch.int32, device="cuda")
    split = []

    def body():
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        g.pls(work, m, n, s, ws=ws, P=P, Q=Q, rank=rank)
        e1.record()
        g.rref(work, m, n, Q, rank, R=R, ws=ws, s=s)
        e2.record()
        split.append((e0, e1, e2))

    def prepare():
        work.copy_(src)

    prepare()
    body()
    torch.cuda.synchronize()
    split.clear()
    if profile:
        g.prof_enable()
        g.prof_read()
    ms, _ = _timed(torch, prepare, body, reps=3, warmup=0)
    launches = g.prof_launches() if profile else []
    prof = g.prof_read() if profile else None
    if profile:
        g.prof_disable()
    pls_ms = _median([a.elapsed_time(b) for a, b, _ in split])
    rref_ms = _median([b.elapsed_time(c) for _, b, c in split])
    r = int(rank.item())
    sched = s if s is not None else g.default_sched()
    out = {"workload": label, "m": m, "n": n, "rank": r, "schedule": str(sched),
           "ms_per_step": round(ms, 3), "pls_ms": round(pls_ms, 3), "rref_ms": round(rref_ms, 3),
           "pls_gf2_ops_per_s": classical_ops(m, n, r) / (pls_ms * 1e-3),
           "rref_gf2_ops": 2.0 * r * r * (n - r) / 2.0}
    if profile:
        reps = 3
        out["product_roofline"] = _product_roofline(g, sched.schur, prof, launches)
        if out["product_roofline"]:
            out["product_roofline"]["launches"] //= reps
    del src, work, R, ws
    torch.cuda.empty_cache()
    return out


def _rref_routes_leg(g, torch, A, m, n, routes):
    """Time each RREF route (PLS+RREF, M4RI, M+P thresholds) on its own copy."""
    src = g.to_device(A)
    work = torch.empty_like(src)
    R = torch.empty_like(src)
    Q = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    P = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    rank = torch.empty(1, dtype=torch.int32, device="cuda")
    ws_pls = g.workspace(max(g.pls_workspace_bytes(m, n), g.rref_workspace_bytes(m, n)))
    ws_m4 = g.workspace(int(g.get_lib().gf2_m4ri_workspace_bytes(m, n)))
    ws_mp = g.workspace(int(g.get_lib().gf2_rref_mp_workspace_bytes(m, n, None)))
    out = {}

    def prepare():
        work.copy_(src)

    for route in routes:
        if route == "PLS":
            def body():
                g.pls(work, m, n, ws=ws_pls, P=P, Q=Q, rank=rank)
                g.rref(work, m, n, Q, rank, R=R, ws=ws_pls)
        elif route == "M4RI":
            def body():
                g.m4ri(work, m, n, Q=Q, rank=rank, ws=ws_m4)
        else:
            th = float(route.split()[1])

            def body(th=th):
                return g.rref_mp(work, m, n, th, Q=Q, rank=rank, ws=ws_mp)[2]
        ms, res = _timed(torch, prepare, body)
        out[route] = {"ms": round(ms, 3)}
        if route.startswith("M+P"):
            out[route]["switch_strip"] = res
    out["rank"] = int(rank.item())
    del src, work, R, ws_pls, ws_m4, ws_mp
    torch.cuda.empty_cache()
    return out


def configs_leg(g, torch, which) -> dict:
    import synth
    out = {}
    if "wide" in which:
        m, n = 32768, 131072
        A = synth.random_half(m, n, 3)
        out["wide_32768x131072"] = _pls_rref_leg(
            g, torch, A, m, n, None, "PLS + RREF, 32768x131072 iid Bernoulli(1/2), seed 3")
        del A
    if "sparse" in which:
        m = n = 65536
        A = synth.random_bernoulli(m, n, 0.01, 2)
        out["sparse_65536"] = _pls_rref_leg(
            g, torch, A, m, n, None, "PLS + RREF, 65536x65536 iid Bernoulli(0.01), seed 2")
        del A
    if "xor" in which:
        m = n = 65536
        A = synth.random_half(m, n, 1)
        s0 = g.default_sched()
        leg = _pls_rref_leg(g, torch, A, m, n, g.Sched(s0.k, s0.tables, s0.cutoff, g.SCHUR_XOR),
                            "PLS + RREF, 65536x65536 iid Bernoulli(1/2), seed 1, XOR-popcount "
                            "Schur product")
        leg["valu_peak_derivation"] = ("256 CUs x 64 lanes x 2.4 GHz = 39.3e12 32-bit ops/s; "
                                       "one v_bitop3_b32 = 32 bit products = 64 GF(2) ops")
        out["xor_product_65536"] = leg
        del A
    if "c2" in which:
        m = n = 32768
        A = synth.random_half(m, n, 1)
        rec = _pls_rref_leg(g, torch, A, m, n, None,
                            "32768x32768 iid Bernoulli(1/2), seed 1, recursive PLS + RREF",
                            profile=False)
        s0 = g.default_sched()
        mm = _pls_rref_leg(g, torch, A, m, n, g.Sched(s0.k, s0.tables, 1 << 20, s0.schur),
                           "32768x32768 iid Bernoulli(1/2), seed 1, MMPF only + RREF",
                           profile=False)
        out["mmpf_vs_recursive_32768"] = {"recursive": rec, "mmpf": mm}
        del A
    if "c1" in which:
        m = n = 4096
        A = synth.random_half(m, n, 1)
        s0 = g.default_sched()
        mm = _pls_rref_leg(g, torch, A, m, n, g.Sched(s0.k, s0.tables, 4096, s0.schur),
                           "4096x4096 iid Bernoulli(1/2), seed 1, MMPF only + RREF", profile=False)
        mm["us_per_strip"] = round(mm["pls_ms"] * 1e3 / (n // 64), 2)
        rec = _pls_rref_leg(g, torch, A, m, n, None,
                            "4096x4096 iid Bernoulli(1/2), seed 1, recursive PLS + RREF",
                            profile=False)
        out["strips_4096"] = {"mmpf": mm, "recursive": rec}
    if "m4ri" in which:
        leg = {}
        for label, A in (("p=0.5", synth.random_half(4096, 4096, 1)),
                         ("p=0.01", synth.random_bernoulli(4096, 4096, 0.01, 16))):
            leg[label] = _rref_routes_leg(g, torch, A, 4096, 4096, ("PLS", "M4RI", "M+P 0.15"))
        leg["workload"] = "RREF of 4096x4096 iid Bernoulli(p): PLS then RREF, M4RI, M+P 0.15"
        out["m4ri_4096"] = leg
    if "solve" in which:
        out["solve_65536"] = solve_leg(g, torch)
    if "practice" in which:
        leg = {"workload": "iid Bernoulli stand-ins with the shapes and densities of Table 2; "
                           "RREF by each route; paper_e5345_s = the paper's Table 2 seconds "
                           "(2.33 GHz Xeon E5345) for its own matrices, context only"}
        for sh in synth.PRACTICE_SHAPES:
            A = synth.practice_matrix(sh)
            res = _rref_routes_leg(g, torch, A, sh.m, sh.n, ("PLS", "M4RI", "M+P 0.15", "M+P 0.20"))
            res.update({"m": sh.m, "n": sh.n, "p": sh.p, "paper_e5345_s": TABLE2_E5345_S[sh.name]})
            leg[sh.name] = res
            del A
        out["practice_shapes"] = leg
    return out


def solve_leg(g, torch) -> dict:
    import numpy as np

    import synth
    m = n = 65536
    A = synth.random_half(m, n, 1)
    dA = g.to_device(A)
    del A
    P, Q, rank = g.pls(dA, m, n)
    rng = np.random.default_rng(5)
    B = g.to_device(rng.integers(0, np.iinfo(np.uint64).max, size=(m, 1), dtype=np.uint64,
                                 endpoint=True))
    X = torch.empty((n, 1), dtype=torch.int64, device="cuda")
    bad = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = g.workspace(int(g.get_lib().gf2_solve_workspace_bytes(m, n, 64)))
    ms, _ = _timed(torch, lambda: None,
                   lambda: g.solve(dA, m, n, P, Q, rank, B, 64, X=X, bad=bad, ws=ws))
    out = {"workload": "A X = B, 65536x65536 iid Bernoulli(1/2) (seed 1) from its PLS, "
                       "64 right-hand sides", "solve_ms": round(ms, 3)}
    del dA, B, X, ws
    torch.cuda.empty_cache()
    km, kn = 16384, 32768
    Ak = synth.random_half(km, kn, 6)
    dK = g.to_device(Ak)
    Pk, Qk, rk = g.pls(dK, km, kn)
    K = torch.empty((kn, kn // 64), dtype=torch.int64, device="cuda")
    wsk = g.workspace(int(g.get_lib().gf2_kernel_basis_workspace_bytes(km, kn)))
    ms, _ = _timed(torch, lambda: None, lambda: g.kernel_basis(dK, km, kn, Qk, rk, K=K, ws=wsk))
    out["kernel_basis"] = {"workload": "null-space basis of 16384x32768 iid Bernoulli(1/2) (seed 6) "
                                       "from its PLS", "ms": round(ms, 3),
                           "nullity": kn - int(rk.item())}
    del dK, K, wsk
    torch.cuda.empty_cache()
    return out


ALL_CONFIG_LEGS = ("wide", "sparse", "xor", "c2", "c1", "m4ri", "solve", "practice")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-n", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-rref", action="store_true")
    ap.add_argument("--sched", type=str, default="")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-int8", action="store_true",
                    help="skip the second leg that times the same workload with the int8 product")
    ap.add_argument("--configs", type=str, default=",".join(ALL_CONFIG_LEGS),
                    help="comma list of further configurations to time (empty: none): "
                         + ",".join(ALL_CONFIG_LEGS))
    ap.add_argument("--no-main", action="store_true",
                    help="skip the headline 65536^2 leg (for profiling single configurations)")
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

    out = {"metric": "PLS+RREF of a dense random 65536x65536 GF(2) matrix (GF(2) ops/s)",
           "value": None, "unit": "GF(2) ops/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": f"PLS + RREF, {m}x{n} iid Bernoulli(1/2), seed {args.seed}",
                      "m": m, "n": n,
                      "schedule": str(s) if s is not None else str(g.default_sched())}}
    if not args.no_main:
        ms, r, prof, launches = timed_leg(s, args.steps, args.warmup)
        ops = classical_ops(m, n, r)
        op_type, roofline = product_roofline(s, prof, launches, args.steps, ms)
        out.update({"value": ops / (ms * 1e-3), "ms_per_step": round(ms, 3),
                    "dtype": f"u64/{op_type}", "roofline": roofline})
        out["config"]["rank"] = r
    if not args.no_main and not args.no_int8 and not args.sched:
        # the same workload with the int8 matrix-core product, against the int8 peak
        s0 = g.default_sched()
        s8 = g.Sched(s0.k, s0.tables, s0.cutoff, g.SCHUR_MFMA)
        ms8, r8, prof8, launches8 = timed_leg(s8, args.steps, args.warmup)
        _, roof8 = product_roofline(s8, prof8, launches8, args.steps, ms8)
        out["int8_product"] = {"schedule": str(s8), "ms_per_step": round(ms8, 3),
                               "value": classical_ops(m, n, r8) / (ms8 * 1e-3), "unit": "GF(2) ops/s",
                               "roofline": roof8}
    del host, R, ws
    torch.cuda.empty_cache()
    if not args.no_batch:
        out["batched"] = batched_leg(g, torch, max(3, args.steps))
    legs = [x for x in args.configs.split(",") if x]
    unknown = [x for x in legs if x not in ALL_CONFIG_LEGS]
    if unknown:
        print(f"bench.py: unknown configuration legs {unknown}", file=sys.stderr)
        return 2
    if legs:
        out["configs"] = configs_leg(g, torch, legs)
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
