"""What the trained cost model gains over the method without it.

The committed model (trained on device timings by the library's own kernels)
is evaluated with the GPU forward kernel on the stored held-out timings
(regret against the exhaustive autotuner's best, and against the fixed
default), and on the 4096-matrix batched workload, where its per-matrix
schedules must beat the fixed default schedule."""
from __future__ import annotations

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1006_1744_amd as g  # noqa: E402
from paper_1006_1744_amd import costmodel as cmod  # noqa: E402


def test_trained_model_regret_on_held_out_shapes():
    z = np.load(cmod.DATA_PATH, allow_pickle=False)
    cm = cmod.CostModel.load()
    assert np.array_equal(np.array([s.astuple() for s in cm.table]), z["table"])
    T = z["times_test"]
    pred = np.argmin(cm.predict_log_times(z["feats_test"]), axis=1)
    default = [i for i, s in enumerate(cm.table) if s.astuple() == g.default_sched().astuple()[:2]
               + (s.cutoff, s.schur)][0]
    learned = cmod.regret(T, pred)
    fixed = cmod.regret(T, np.full(len(T), default))
    print(f"held-out regret: learned {learned:.4f}, default {fixed:.4f}", flush=True)
    assert learned <= 1.05
    assert learned < fixed


def test_learned_schedules_beat_default_on_batched_mix():
    cm = cmod.CostModel.load()
    res = cmod.evaluate_mix(cm, reps=3)
    print(res, flush=True)
    assert res["learned_ms"] < res["default_ms"]
