"""GPU parity of the batched PLS (one persistent launch over many matrices)
against the CPU oracle, bit for bit per matrix: rank, P, Q and every word of
the in-place result, padding included."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU runs deselect the marker anyway
    pytest.skip("no GPU", allow_module_level=True)

import paper_1006_1744_amd as g  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_batch(mats_np, shapes):
    dev = [g.to_device(A) for A in mats_np]
    return g.Batch(dev, shapes), dev


def check_batch(b, dev, mats_np, shapes, label):
    ranks = b.ranks[:b.count].cpu().numpy()
    for j, (A, (m, n)) in enumerate(zip(mats_np, shapes)):
        r, P, Q, Ap = oracle.pls(A, m, n)
        gP, gQ = (x.cpu().numpy() for x in b.pq(j))
        assert ranks[j] == r, f"{label} item {j} ({m}x{n}): rank {ranks[j]} != {r}"
        assert np.array_equal(gQ, Q), f"{label} item {j} ({m}x{n}): Q differs"
        assert np.array_equal(gP, P), f"{label} item {j} ({m}x{n}): P differs"
        assert np.array_equal(g.to_host(dev[j]), Ap), f"{label} item {j} ({m}x{n}): A' differs"


def mixed_inputs(count, seed, hi=700):
    items = synth.batch_shapes(count, seed, lo=1, hi=hi)
    mats = [synth.batch_matrix(it) for it in items]
    shapes = [(it.m, it.n) for it in items]
    extra = [
        (synth.random_half(1, 1, 3), (1, 1)),
        (synth.random_half(1, 100, 4), (1, 100)),
        (synth.random_half(100, 1, 5), (100, 1)),
        (synth.random_half(64, 64, 6), (64, 64)),
        (synth.empty(300, 200), (300, 200)),
        (synth.random_bernoulli(700, 500, 0.002, 8), (700, 500)),
        (synth.random_half(130, 4096, 9), (130, 4096)),
        (synth.random_half(333, 250, 10, stride=6), (333, 250)),
        (synth.planted(512, 512, 100, 11, p=0.5), (512, 512)),
    ]
    for A, sh in extra:
        mats.append(A)
        shapes.append(sh)
    return mats, shapes


@pytest.mark.parametrize("sname,s", [("default", None), ("k4t8", g.Sched(4, 8, 512, 1)),
                                     ("k6t2", g.Sched(6, 2, 512, 0)), ("k8t1", g.Sched(8, 1, 512, 1))])
def test_batched_mixed(sname, s):
    mats, shapes = mixed_inputs(60, 3)
    say(f"[batch] mixed {len(mats)} items sched={sname}")
    b, dev = make_batch(mats, shapes)
    b.run(s)
    torch.cuda.synchronize()
    check_batch(b, dev, mats, shapes, sname)


def test_batched_per_item_scheds():
    mats, shapes = mixed_inputs(40, 5)
    say(f"[batch] per-item schedules, {len(mats)} items")
    b, dev = make_batch(mats, shapes)
    rng = np.random.default_rng(1)
    scheds = [(int(rng.integers(4, 9)), int(rng.choice([1, 2, 4, 8])), 512, 1) for _ in shapes]
    scheds[0] = (99, 3, 0, 0)   # out of range: falls back to the call's schedule
    b.set_scheds(scheds)
    b.run()
    torch.cuda.synchronize()
    check_batch(b, dev, mats, shapes, "per-item")


def test_batched_invalid_items_untouched():
    A = synth.random_half(100, 300, 1)
    B = synth.random_half(80, 90, 2)
    dA, dB = g.to_device(A), g.to_device(B)
    say("[batch] invalid descriptors")
    b = g.Batch([dA, dB], [(100, 300), (80, 90)])
    # item 0 claims more columns than its stride holds: rejected on the device
    bad = g.BatchItem(dA.data_ptr(), 100, 64 * dA.shape[1] + 1, dA.shape[1],
                      b.P.data_ptr(), b.Q.data_ptr())
    raw = torch.frombuffer(bytearray(bytes(bad)), dtype=torch.uint8).to(b.items.device)
    b.items[:raw.numel()].copy_(raw)
    b.run()
    torch.cuda.synchronize()
    ranks = b.ranks.cpu().numpy()
    assert ranks[0] == -1
    assert np.array_equal(g.to_host(dA), A)
    r, P, Q, Ap = oracle.pls(B, 80, 90)
    assert ranks[1] == r and np.array_equal(g.to_host(dB), Ap)


def test_batched_graph_replay():
    mats, shapes = mixed_inputs(50, 9)
    say(f"[batch] graph capture, {len(mats)} items")
    b, dev = make_batch(mats, shapes)
    pristine = [t.clone() for t in dev]
    s = g.Sched(5, 4, 512, 1)
    b.run(s)   # eager: reference result
    torch.cuda.synchronize()
    want = [t.clone() for t in dev]
    want_r = b.ranks.clone()
    want_p, want_q = b.P.clone(), b.Q.clone()
    for t, p in zip(dev, pristine):
        t.copy_(p)
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        b.run(s)
    for rep in range(3):
        for t, p in zip(dev, pristine):
            t.copy_(p)
        b.ranks.fill_(-7)
        b.P.fill_(-7)
        b.Q.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(b.ranks, want_r), f"replay {rep}: ranks"
        assert torch.equal(b.P, want_p) and torch.equal(b.Q, want_q), f"replay {rep}: P/Q"
        for j, (t, w) in enumerate(zip(dev, want)):
            assert torch.equal(t, w), f"replay {rep}: item {j}"
    check_batch(b, dev, mats, shapes, "graph")


def test_batched_full_workload():
    """The 4096-matrix workload (m, n log-uniform in [64, 2048], p in
    {0.5, 0.1, 0.01}, planted rank in [min/2, min], seed 7), every matrix
    compared with the oracle."""
    items = synth.batch_shapes(4096, 7)
    mats = [synth.batch_matrix(it) for it in items]
    shapes = [(it.m, it.n) for it in items]
    say("[batch] 4096 items, seed 7")
    b, dev = make_batch(mats, shapes)
    b.run()
    torch.cuda.synchronize()
    ranks = b.ranks.cpu().numpy()
    assert all(int(ranks[j]) == it.r for j, it in enumerate(items))
    check_batch(b, dev, mats, shapes, "full")
