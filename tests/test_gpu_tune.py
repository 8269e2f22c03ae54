"""The autotuner on the GPU: it times every candidate, leaves the trial input
untouched, and whatever schedule it picks gives the oracle's bits."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1006_1744_amd as g  # noqa: E402


def test_autotune_single():
    m, n = 700, 900
    A = synth.random_half(m, n, 21)
    dA = g.to_device(A)
    cands = [g.Sched(8, 8, 128, g.SCHUR_MFMA), g.Sched(4, 1, 128, g.SCHUR_XOR),
             g.Sched(6, 2, 256, g.SCHUR_MFMA), g.Sched(8, 8, 4096, g.SCHUR_MFMA),
             g.Sched(5, 4, 512, g.SCHUR_XOR)]
    best, ms = g.autotune(dA, m, n, cands, reps=2)
    torch.cuda.synchronize()
    assert len(ms) == len(cands) and all(t > 0 for t in ms)
    assert best.astuple() == cands[int(np.argmin(ms))].astuple()
    assert np.array_equal(g.to_host(dA), A)            # the trial input is only read
    r, P, Q, Ap = oracle.pls(A, m, n)
    dB = g.to_device(A)
    gP, gQ, gr = g.pls(dB, m, n, best)
    torch.cuda.synchronize()
    assert int(gr.item()) == r and np.array_equal(g.to_host(dB), Ap)


def test_autotune_empty_candidate_list_gives_default():
    A = g.to_device(synth.random_half(64, 64, 2))
    best, ms = g.autotune(A, 64, 64, [], reps=1)
    assert best.astuple() == g.default_sched().astuple() and ms == []


def test_autotune_batched():
    m, n, copies = 300, 500, 40
    A = synth.planted(m, n, 200, 5, p=0.1)
    big = g.to_device(A).unsqueeze(0).repeat(copies, 1, 1).contiguous()
    work = torch.empty_like(big)
    trial = g.Batch([big[j] for j in range(copies)], [(m, n)] * copies)
    wb = g.Batch([work[j] for j in range(copies)], [(m, n)] * copies)
    cands = g.sched_candidates(m, n, batched=True)
    best, ms = g.autotune_batched(trial, wb, cands, reps=2)
    torch.cuda.synchronize()
    assert len(ms) == 20 and all(t > 0 for t in ms)
    assert best.astuple() == cands[int(np.argmin(ms))].astuple()
    r, P, Q, Ap = oracle.pls(A, m, n)
    assert np.array_equal(g.to_host(big[3]), A)
    assert np.array_equal(g.to_host(work[copies - 1]), Ap)
    assert np.all(wb.ranks.cpu().numpy() == r)
