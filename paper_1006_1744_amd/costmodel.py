"""Schedule choice learned from the method's own timings: the autotuner's
timings and the cost models trained on them.

The decomposition's result never depends on the schedule, only its time does.
Two models, both fp32 networks 4 -> 64 -> 64 -> S trained and evaluated by the
library's own kernels, map a matrix's features to predicted log times of S
candidate schedules; the argmin is the schedule, the fixed default stays the
fallback, and exhaustive timings judge the regret.
* batched: the candidates of the batched call (strip width k x tables per pass,
  S = 20), timed on a batch of identical copies of one synthetic matrix.
* single: one matrix through gf2_pls, candidates k in {6, 8} x tables in {4, 8}
  x cutoff in {256, ..., 4096} x Schur product in {XOR, int8, fp4} (S = 60),
  shapes up to 65536 a side; training shapes are timed on a random subset of
  the candidates (masked partial labels), held-out shapes on all of them.
Features come from the matrices on the device (gf2_features: log2 m, log2 n,
the density of a row sample, and a rank estimate that is min(m, n) unless the
caller has a better one), never from the generator's parameters.

Run as a module to collect timings, train, evaluate and save a model:
    python -m paper_1006_1744_amd.costmodel batched-retrain
    python -m paper_1006_1744_amd.costmodel single-collect --part train --train 4000 --budget-s 500
    python -m paper_1006_1744_amd.costmodel single-collect --part test --test 1000 --budget-s 600
    python -m paper_1006_1744_amd.costmodel single-train --data-dir DIR --steps 6000
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import Batch, Sched, autotune, autotune_batched, costmodel_predict, features as dev_features, \
    items_of, mlp_adam, mlp_forward, mlp_grad, mlp_init, mlp_param_count, sched_candidates, \
    set_learned, to_device

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "data", "costmodel_batched.npz")
DATA_PATH = os.path.join(HERE, "data", "batched_timings.npz")
SINGLE_MODEL_PATH = os.path.join(HERE, "data", "costmodel_single.npz")
SINGLE_DATA_PATH = os.path.join(HERE, "data", "single_timings.npz")

# The single-matrix candidates (k, tables, cutoff, schur): a subset of the
# autotuner's space that spans all four of its dimensions.
SINGLE_TABLE = [(k, t, c, sc) for k in (6, 8) for t in (4, 8)
                for c in (256, 512, 1024, 2048, 4096) for sc in (0, 1, 2)]
SINGLE_DEFAULT = SINGLE_TABLE.index((8, 8, 2048, 2))
SINGLE_LOG2_RANGE = (6.0, 16.0)
SINGLE_LOG2_MN_MAX = 31.0   # training shapes hold at most 2^31 entries (sample_single_shapes)


def features(m, n, density, r_est) -> np.ndarray:
    """Raw features (log2 m, log2 n, density, r_est / min(m, n)), float32 rows."""
    m = np.asarray(m, np.float64)
    n = np.asarray(n, np.float64)
    r = np.asarray(r_est, np.float64)
    return np.stack([np.log2(m), np.log2(n), np.asarray(density, np.float64),
                     r / np.minimum(m, n)], axis=-1).astype(np.float32)


def candidates() -> list:
    return sched_candidates(64, 64, batched=True)


def sample_shapes(count: int, seed: int, lo: int = 64, hi: int = 2048):
    """Training / test shapes: the batched workload's distribution (m, n
    log-uniform, p in {0.5, 0.1, 0.01}, planted rank in [min/2, min]) for half,
    full-rank iid Bernoulli(p in {0.5, 0.01}) for the other half."""
    import synth
    out = []
    for t in range(count):
        u = [synth.splitmix(seed, 5 * t + q) for q in range(5)]
        f = [(x >> 11) * (1.0 / (1 << 53)) for x in u]
        m = int(round(math.exp(math.log(lo) + f[0] * (math.log(hi) - math.log(lo)))))
        n = int(round(math.exp(math.log(lo) + f[1] * (math.log(hi) - math.log(lo)))))
        mn = min(m, n)
        if u[2] & 1:
            p = (0.5, 0.1, 0.01)[u[3] % 3]
            r = (mn + 1) // 2 + int(u[4] % (mn - (mn + 1) // 2 + 1))
            out.append(dict(m=m, n=n, p=p, r=r, planted=True, seed=(seed * 7919 + t) & (2**63 - 1)))
        else:
            p = (0.5, 0.01)[u[3] % 2]
            out.append(dict(m=m, n=n, p=p, r=mn, planted=False,
                            seed=(seed * 7919 + t) & (2**63 - 1)))
    return out


def shape_matrix(sh):
    import synth
    if sh["planted"]:
        return synth.planted(sh["m"], sh["n"], sh["r"], sh["seed"], p=sh["p"], unit=True)
    return synth.random_bernoulli(sh["m"], sh["n"], sh["p"], sh["seed"])


def time_shape(sh, copies: int, cands, reps: int = 2) -> np.ndarray:
    """Fastest batched time (ms) of each candidate on `copies` copies of one
    matrix of the shape."""
    from . import to_device
    A = to_device(shape_matrix(sh))
    m, n = sh["m"], sh["n"]
    big = A.unsqueeze(0).repeat(copies, 1, 1).contiguous()
    work = torch.empty_like(big)
    trial_b = Batch([big[j] for j in range(copies)], [(m, n)] * copies)
    work_b = Batch([work[j] for j in range(copies)], [(m, n)] * copies)
    _, ms = autotune_batched(trial_b, work_b, cands, reps=reps)
    return np.array(ms, np.float64)


def collect(shapes, copies: int, cands, log=print) -> np.ndarray:
    T = np.zeros((len(shapes), len(cands)))
    t0 = time.time()
    for i, sh in enumerate(shapes):
        T[i] = time_shape(sh, copies, cands)
        if (i + 1) % 50 == 0:
            log(f"timed {i + 1}/{len(shapes)} shapes ({time.time() - t0:.1f} s)")
    return T


class CostModel:
    """The network's parameters and Adam state on the device, plus the table
    of schedules its outputs stand for."""

    def __init__(self, table, seed: int = 1, device="cuda"):
        self.table = [Sched(*s.astuple()) if isinstance(s, Sched) else Sched(*s) for s in table]
        self.S = len(self.table)
        P = mlp_param_count(self.S)
        self.params = torch.empty(P, dtype=torch.float32, device=device)
        mlp_init(self.params, self.S, seed)
        self.m1 = torch.zeros(P, dtype=torch.float32, device=device)
        self.m2 = torch.zeros(P, dtype=torch.float32, device=device)
        self.step = 0
        self.table_dev = torch.tensor([s.astuple() for s in self.table], dtype=torch.int32,
                                      device=device)

    def fit(self, feats, log_t, mask, steps=3000, lr=3e-3, log=None):
        dev = self.params.device
        F = torch.from_numpy(np.ascontiguousarray(feats, np.float32)).to(dev)
        Tt = torch.from_numpy(np.ascontiguousarray(log_t, np.float32)).to(dev)
        M = torch.from_numpy(np.ascontiguousarray(mask, np.float32)).to(dev)
        ic = 1.0 / max(1.0, float(np.sum(mask)))
        grad = None
        hist = []
        for it in range(steps):
            grad = mlp_grad(self.params, self.S, F, Tt, M, ic, out=grad)
            self.step += 1
            mlp_adam(self.params, self.S, grad, self.m1, self.m2, lr, self.step)
            if it % 500 == 0 or it == steps - 1:
                loss = float(grad[-1].item())
                hist.append((it, loss))
                if log:
                    log(f"step {it}: loss {loss:.5f}")
        return hist

    def predict_log_times(self, feats) -> np.ndarray:
        F = torch.from_numpy(np.ascontiguousarray(feats, np.float32)).to(self.params.device)
        return mlp_forward(self.params, self.S, F).cpu().numpy()

    def predict_dev(self, feats_dev: torch.Tensor) -> torch.Tensor:
        """As predict, for features already on the device."""
        return costmodel_predict(self.params, self.S, feats_dev.contiguous(), self.table_dev)

    def install(self, log2_lo=SINGLE_LOG2_RANGE[0], log2_hi=SINGLE_LOG2_RANGE[1],
                log2_mn_hi=SINGLE_LOG2_MN_MAX):
        """Make this model the choice of gf2_pls calls without a schedule, for the
        shapes it was trained on (the default elsewhere)."""
        set_learned(self.params, self.S, self.table_dev, log2_lo, log2_hi, log2_mn_hi)

    def predict(self, feats) -> torch.Tensor:
        """Per problem, the (k, tables, cutoff, schur) row of the predicted fastest
        schedule, as an int32 (N, 4) device tensor."""
        F = torch.from_numpy(np.ascontiguousarray(feats, np.float32)).to(self.params.device)
        return costmodel_predict(self.params, self.S, F, self.table_dev)

    def save(self, path=MODEL_PATH):
        os.makedirs(os.path.dirname(path), exist_ok=True)
        np.savez(path, params=self.params.cpu().numpy(),
                 table=np.array([s.astuple() for s in self.table], np.int32))

    @classmethod
    def load(cls, path=MODEL_PATH, device="cuda"):
        z = np.load(path, allow_pickle=False)
        cm = cls([tuple(int(v) for v in row) for row in z["table"]], device=device)
        cm.params.copy_(torch.from_numpy(z["params"]).to(device))
        return cm


def batch_features(b: Batch) -> torch.Tensor:
    """Features of a batch's matrices, measured on the device (gf2_features; the
    rank estimate is min(m, n): the batch carries no better one)."""
    return dev_features(b.items, b.count)


def matrix_features(mats, shapes) -> np.ndarray:
    """Device-measured features of a list of device matrices (host float32 rows)."""
    out = []
    for i in range(0, len(mats), 1024):
        out.append(dev_features(items_of(mats[i:i + 1024], shapes[i:i + 1024]),
                                len(mats[i:i + 1024])).cpu().numpy())
    return np.concatenate(out, axis=0) if out else np.zeros((0, 4), np.float32)


def time_batch(b: Batch, pristine, dev_mats, s=None, reps: int = 3) -> float:
    """Fastest of `reps` event-timed runs of the batch (inputs restored first)."""
    best = None
    for _ in range(reps):
        for t, p0 in zip(dev_mats, pristine):
            t.copy_(p0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.run(s)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def evaluate_mix(cm: "CostModel", count: int = 4096, seed: int = 7, reps: int = 3) -> dict:
    """Matrices/s on the batched workload with the default schedule, the best
    single schedule for the whole mix (autotuned on the mix itself) and the
    learned per-matrix schedules."""
    import synth
    from . import default_sched, to_device
    items = synth.batch_shapes(count, seed)
    mats = [to_device(synth.batch_matrix(it)) for it in items]
    pristine = [t.clone() for t in mats]
    shapes = [(it.m, it.n) for it in items]
    b = Batch(mats, shapes)
    work = [torch.empty_like(t) for t in mats]
    wb = Batch(work, shapes)
    tb = Batch(pristine, shapes)
    best_uniform, _ = autotune_batched(tb, wb, candidates(), reps=2)
    t_def = time_batch(b, pristine, mats, default_sched(), reps)
    t_uni = time_batch(b, pristine, mats, best_uniform, reps)
    b.per_item = cm.predict_dev(batch_features(b))
    t_learn = time_batch(b, pristine, mats, None, reps)
    b.per_item = None
    return {"count": count, "default_ms": t_def, "uniform_best_ms": t_uni,
            "uniform_best": list(best_uniform.astuple()), "learned_ms": t_learn,
            "default_matrices_per_s": count / t_def * 1e3,
            "uniform_best_matrices_per_s": count / t_uni * 1e3,
            "learned_matrices_per_s": count / t_learn * 1e3}


def regret(T: np.ndarray, choice: np.ndarray) -> float:
    """Geometric mean over problems of T[choice] / min T."""
    best = T.min(axis=1)
    got = T[np.arange(len(T)), choice]
    return float(np.exp(np.mean(np.log(got / best))))


# ------------------------------------------------------------ batched retrain
def batched_retrain(steps: int = 6000, out_dir: str = os.path.dirname(MODEL_PATH),
                    log=print) -> dict:
    """Retrain the batched model on the stored timings with features measured on
    the device from the same shapes' matrices; evaluate and save."""
    z = np.load(DATA_PATH, allow_pickle=False)
    table = [tuple(int(v) for v in row) for row in z["table"]]
    n_tr, n_te = z["times_train"].shape[0], z["times_test"].shape[0]
    feats = []
    for shapes in (sample_shapes(n_tr, 1000), sample_shapes(n_te, 2000)):
        mats = [to_device(shape_matrix(sh)) for sh in shapes]
        feats.append(matrix_features(mats, [(sh["m"], sh["n"]) for sh in shapes]))
        del mats
    ftr, fte = feats
    Ttr, Tte = z["times_train"], z["times_test"]
    cm = CostModel(table, seed=7)
    cm.fit(ftr, np.log(Ttr), np.ones_like(Ttr), steps=steps, log=log)
    os.makedirs(out_dir, exist_ok=True)
    cm.save(os.path.join(out_dir, os.path.basename(MODEL_PATH)))
    np.savez(os.path.join(out_dir, os.path.basename(DATA_PATH)), feats_train=ftr,
             times_train=Ttr, feats_test=fte, times_test=Tte, table=z["table"])
    pred = np.argmin(cm.predict_log_times(fte), axis=1)
    default = [i for i, sch in enumerate(table) if sch[:2] == (8, 8)][0]
    res = {"test_regret_learned": regret(Tte, pred),
           "test_regret_default": regret(Tte, np.full(len(Tte), default)),
           "train_regret_learned": regret(Ttr, np.argmin(cm.predict_log_times(ftr), axis=1))}
    log(json.dumps(res))
    res.update(evaluate_mix(cm))
    log(json.dumps(res))
    return res


# ------------------------------------------------------------ single matrix
def sample_single_shapes(count: int, seed: int, lo: int = 64, hi: int = 65536,
                         max_bits: int = 1 << 31):
    """Shapes of the single-matrix model: m, n log-uniform in [lo, hi] with at
    most max_bits entries (a matrix of 256 MiB; larger draws are redrawn), iid
    Bernoulli(p), p in {0.5, 0.01}, full rank expected."""
    import synth
    out = []
    t = 0
    while len(out) < count:
        u = [synth.splitmix(seed, 3 * t + q) for q in range(3)]
        t += 1
        f = [(x >> 11) * (1.0 / (1 << 53)) for x in u]
        m = int(round(math.exp(math.log(lo) + f[0] * (math.log(hi) - math.log(lo)))))
        n = int(round(math.exp(math.log(lo) + f[1] * (math.log(hi) - math.log(lo)))))
        if m * n > max_bits:
            continue
        out.append(dict(m=m, n=n, p=(0.5, 0.01)[u[2] % 2], seed=(seed * 7919 + t) & (2**63 - 1)))
    return out


def single_matrix(sh):
    import synth
    return synth.random_bernoulli(sh["m"], sh["n"], sh["p"], sh["seed"])


def collect_single(shapes, n_rand: int, reps: int, budget_s: float, seed: int, log=print):
    """Times (ms; NaN where not timed) of the SINGLE_TABLE candidates on each
    shape, with device-measured features.  n_rand < 0: every candidate;
    otherwise the default and n_rand others drawn at random.  Stops when the
    time budget is spent; returns (feats, times, shapes timed)."""
    rng = np.random.default_rng(seed)
    cands = [Sched(*c) for c in SINGLE_TABLE]
    F, T = [], []
    t0 = time.time()
    for i, sh in enumerate(shapes):
        if time.time() - t0 > budget_s:
            break
        m, n = sh["m"], sh["n"]
        A = to_device(single_matrix(sh))
        F.append(matrix_features([A], [(m, n)])[0])
        if n_rand < 0:
            idx = list(range(len(cands)))
        else:
            others = [j for j in range(len(cands)) if j != SINGLE_DEFAULT]
            idx = [SINGLE_DEFAULT] + list(rng.choice(others, size=n_rand, replace=False))
        row = np.full(len(cands), np.nan)
        _, ms = autotune(A, m, n, [cands[j] for j in idx], reps=reps)
        row[idx] = ms
        T.append(row)
        del A
        if (i + 1) % 25 == 0:
            log(f"timed {i + 1} shapes ({time.time() - t0:.0f} s)")
    return np.array(F, np.float32).reshape(-1, 4), np.array(T), len(T)


def single_regret(cm: "CostModel", feats, T) -> dict:
    pred = np.argmin(cm.predict_log_times(feats), axis=1)
    return {"regret_learned": regret(T, pred),
            "regret_default": regret(T, np.full(len(T), SINGLE_DEFAULT)),
            "shapes": int(len(T))}


def single_collect(part: str, count: int, n_rand: int, budget_s: float, out_dir: str,
                   log=print) -> str:
    """Time one part of the single-matrix data set ("train": masked labels,
    "test": every candidate) and save it as single_<part>.npz in out_dir."""
    seed = 3000 if part == "train" else 4000
    shapes = sample_single_shapes(count, seed)
    F, T, nt = collect_single(shapes, n_rand if part == "train" else -1, 1, budget_s,
                              5 if part == "train" else 6, log)
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, f"single_{part}.npz")
    np.savez(path, feats=F, times=T, table=np.array(SINGLE_TABLE, np.int32),
             shapes=np.array([[s["m"], s["n"], int(s["p"] == 0.5), s["seed"]]
                              for s in shapes[:nt]], np.int64))
    log(f"saved {nt} {part} shapes to {path}")
    return path


def single_train(data_dir: str, out_dir: str, steps: int, log=print) -> dict:
    """Train the single-matrix model on single_train.npz (masked), evaluate on
    single_test.npz (exhaustive), save the model and the merged timings."""
    tr = np.load(os.path.join(data_dir, "single_train.npz"), allow_pickle=False)
    te = np.load(os.path.join(data_dir, "single_test.npz"), allow_pickle=False)
    Ttr, ftr = tr["times"], tr["feats"]
    mask = np.isfinite(Ttr).astype(np.float32)
    target = np.where(mask > 0, np.log(np.where(mask > 0, Ttr, 1.0)), 0.0)
    cm = CostModel(SINGLE_TABLE, seed=11)
    cm.fit(ftr, target, mask, steps=steps, log=log)
    os.makedirs(out_dir, exist_ok=True)
    cm.save(os.path.join(out_dir, os.path.basename(SINGLE_MODEL_PATH)))
    np.savez(os.path.join(out_dir, os.path.basename(SINGLE_DATA_PATH)), feats_train=ftr,
             times_train=Ttr, shapes_train=tr["shapes"], feats_test=te["feats"],
             times_test=te["times"], shapes_test=te["shapes"], table=tr["table"])
    res = single_regret(cm, te["feats"], te["times"])
    res["train_shapes"] = int(len(Ttr))
    log(json.dumps(res))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["batched", "batched-retrain", "single-collect",
                                     "single-train"])
    ap.add_argument("--part", choices=["train", "test"], default="train")
    ap.add_argument("--data-dir", default="")
    ap.add_argument("--train", type=int, default=600)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--copies", type=int, default=0, help="copies per timed batch (0: fill the device)")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--n-rand", type=int, default=7,
                    help="single: candidates timed per training shape besides the default")
    ap.add_argument("--budget-s", type=float, default=900.0,
                    help="single: seconds of timing for training and held-out shapes together")
    ap.add_argument("--out-dir", default=os.path.dirname(MODEL_PATH))
    args = ap.parse_args()
    torch.cuda.init()
    log = lambda s: print(s, flush=True)  # noqa: E731
    if args.what == "batched-retrain":
        batched_retrain(args.steps, args.out_dir, log)
        return
    if args.what == "single-collect":
        count = args.train if args.part == "train" else args.test
        single_collect(args.part, count, args.n_rand, args.budget_s, args.out_dir, log)
        return
    if args.what == "single-train":
        single_train(args.data_dir or args.out_dir, args.out_dir, args.steps, log)
        return
    model_path = os.path.join(args.out_dir, os.path.basename(MODEL_PATH))
    data_path = os.path.join(args.out_dir, os.path.basename(DATA_PATH))
    props = torch.cuda.get_device_properties(0)
    copies = args.copies or 4 * props.multi_processor_count
    cands = candidates()
    train = sample_shapes(args.train, 1000)
    test = sample_shapes(args.test, 2000)
    log(f"timing {len(train)} + {len(test)} shapes x {len(cands)} schedules, {copies} copies")
    Ttr = collect(train, copies, cands, log=log)
    Tte = collect(test, copies, cands, log=log)
    feats = []
    for shapes in (train, test):
        mats = [to_device(shape_matrix(sh)) for sh in shapes]
        feats.append(matrix_features(mats, [(sh["m"], sh["n"]) for sh in shapes]))
    ftr, fte = feats
    os.makedirs(args.out_dir, exist_ok=True)
    np.savez(data_path, feats_train=ftr, times_train=Ttr, feats_test=fte, times_test=Tte,
             table=np.array([s.astuple() for s in cands], np.int32))
    cm = CostModel(cands, seed=7)
    cm.fit(ftr, np.log(Ttr), np.ones_like(Ttr), steps=args.steps, log=log)
    cm.save(model_path)
    pred = np.argmin(cm.predict_log_times(fte), axis=1)
    default = [i for i, s in enumerate(cands) if s.astuple()[:2] == (8, 8)][0]
    res = {"test_regret_learned": regret(Tte, pred),
           "test_regret_default": regret(Tte, np.full(len(Tte), default)),
           "train_regret_learned": regret(Ttr, np.argmin(cm.predict_log_times(ftr), axis=1))}
    log(json.dumps(res))
    log(json.dumps(evaluate_mix(cm)))


if __name__ == "__main__":
    main()
