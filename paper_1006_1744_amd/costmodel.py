"""Schedule choice for the batched decomposition: the autotuner's timings and
the learned cost model trained on them.

The decomposition's result never depends on the schedule (strip width k and
tables per pass for the batched path), only its time does.  Timings come from
the library's autotuner (gf2_autotune_batched): a batch of identical copies of
one synthetic matrix fills the device, every candidate schedule is run, and
the fastest time per candidate is kept.  The cost model (an fp32 network
4 -> 64 -> 64 -> S, trained and evaluated by the library's own kernels) maps a
matrix's features to predicted log times; its argmin is the schedule.  The
fixed default schedule stays the fallback, and the exhaustive timings are the
judge of the model's regret.

Run as a module to collect timings, train, evaluate and save the model:
    python -m paper_1006_1744_amd.costmodel --train 600 --test 200
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import Batch, Sched, autotune_batched, costmodel_predict, mlp_adam, mlp_forward, mlp_grad, \
    mlp_init, mlp_param_count, sched_candidates

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "data", "costmodel_batched.npz")
DATA_PATH = os.path.join(HERE, "data", "batched_timings.npz")


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


def mix_features(items) -> np.ndarray:
    """Features of the batched workload's items (density = the generator's p,
    rank estimate = the planted rank)."""
    return features([it.m for it in items], [it.n for it in items], [it.p for it in items],
                    [it.r for it in items])


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
    b.per_item = cm.predict(mix_features(items))
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=600)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--copies", type=int, default=0, help="copies per timed batch (0: fill the device)")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--out-dir", default=os.path.dirname(MODEL_PATH))
    args = ap.parse_args()
    model_path = os.path.join(args.out_dir, os.path.basename(MODEL_PATH))
    data_path = os.path.join(args.out_dir, os.path.basename(DATA_PATH))
    torch.cuda.init()
    from . import _ctx, ctx  # noqa: F401
    props = torch.cuda.get_device_properties(0)
    copies = args.copies or 4 * props.multi_processor_count
    cands = candidates()
    train = sample_shapes(args.train, 1000)
    test = sample_shapes(args.test, 2000)
    print(f"timing {len(train)} + {len(test)} shapes x {len(cands)} schedules, {copies} copies",
          flush=True)
    Ttr = collect(train, copies, cands, log=lambda s: print(s, flush=True))
    Tte = collect(test, copies, cands, log=lambda s: print(s, flush=True))
    ftr = features([s["m"] for s in train], [s["n"] for s in train], [s["p"] for s in train],
                   [s["r"] for s in train])
    fte = features([s["m"] for s in test], [s["n"] for s in test], [s["p"] for s in test],
                   [s["r"] for s in test])
    os.makedirs(args.out_dir, exist_ok=True)
    np.savez(data_path, feats_train=ftr, times_train=Ttr, feats_test=fte, times_test=Tte,
             table=np.array([s.astuple() for s in cands], np.int32))
    cm = CostModel(cands, seed=7)
    cm.fit(ftr, np.log(Ttr), np.ones_like(Ttr), steps=args.steps,
           log=lambda s: print(s, flush=True))
    cm.save(model_path)
    pred = np.argmin(cm.predict_log_times(fte), axis=1)
    default = [i for i, s in enumerate(cands) if s.astuple()[:2] == (8, 8)][0]
    res = {"test_regret_learned": regret(Tte, pred),
           "test_regret_default": regret(Tte, np.full(len(Tte), default)),
           "train_regret_learned": regret(Ttr, np.argmin(cm.predict_log_times(ftr), axis=1))}
    print(json.dumps(res), flush=True)
    print(json.dumps(evaluate_mix(cm)), flush=True)


if __name__ == "__main__":
    main()
