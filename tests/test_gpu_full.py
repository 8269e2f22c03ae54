"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (one gf2_pls call with the default schedule, then gf2_rref), against the
CPU oracle run on the same input: rank, P, Q and every word of the in-place
result bit for bit.  The RREF is checked through properties that pin it at any
size (rows past the rank are zero, the pivot columns form the identity, and
S = U_Q R by Freivalds' test with 64 random vectors per identity, so a wrong R
passes with probability at most 2^-64), because forming it on the host by
Gauss-Jordan at these sizes would take minutes; element-wise RREF parity at
sizes that reach the same product tiles is in test_gpu_rref.py."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from rref_checks import check_rref_properties, s_rows

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1006_1744_amd as g  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_full(A, m, n, s=None, rref=True):
    dA = g.to_device(A)
    P, Q, rank = g.pls(dA, m, n, s)
    R = g.rref(dA, m, n, Q, rank, s=s) if rref else None
    torch.cuda.synchronize()
    return (int(rank.item()), P.cpu().numpy(), Q.cpu().numpy(), g.to_host(dA),
            g.to_host(R) if rref else None)


def compare(label, got, want):
    gr, gP, gQ, gAp = got[:4]
    r, P, Q, Ap = want
    assert gr == r, f"{label}: rank {gr} != {r}"
    assert np.array_equal(gQ, Q), f"{label}: Q differs"
    assert np.array_equal(gP, P), f"{label}: P differs"
    assert np.array_equal(gAp, Ap), f"{label}: A' differs"


def test_full_65536_dense_all_schur_variants():
    m = n = 65536
    A = synth.random_half(m, n, 1)
    say("[full] 65536^2 p=1/2 seed 1: GPU (fp4 MFMA Schur, default schedule)")
    got = run_full(A, m, n)
    say("[full] oracle")
    want = oracle.pls(A, m, n)
    compare("65536 fp4 MFMA", got, want)
    r = want[0]
    if r == n:   # full rank: the RREF is the identity
        I = np.zeros_like(got[4])
        idx = np.arange(n)
        I[idx, idx // 64] = np.left_shift(np.uint64(1), (idx % 64).astype(np.uint64))
        assert np.array_equal(got[4], I)
    else:
        check_rref_properties(got[4], s_rows(want[3], r, want[2], n), r, want[2], n)
    say("[full] GPU with the int8 MFMA Schur product")
    got_i = run_full(A, m, n, g.Sched(8, 8, 512, g.SCHUR_MFMA), rref=False)
    compare("65536 int8 MFMA", got_i, want)
    del got_i
    say("[full] GPU with the XOR-popcount Schur product")
    got_x = run_full(A, m, n, g.Sched(8, 8, 512, g.SCHUR_XOR), rref=False)
    compare("65536 XOR", got_x, want)


def test_full_65536_sparse_all_schur_variants():
    m = n = 65536
    A = synth.random_bernoulli(m, n, 0.01, 2)
    say("[full] 65536^2 p=0.01 seed 2")
    got = run_full(A, m, n)
    want = oracle.pls(A, m, n)
    compare("65536 sparse", got, want)
    r, P, Q, Ap = want
    check_rref_properties(got[4], s_rows(Ap, r, Q, n), r, Q, n)
    del got
    for name, v in (("int8 MFMA", g.SCHUR_MFMA), ("XOR", g.SCHUR_XOR)):
        say(f"[full] 65536^2 p=0.01 with the {name} Schur product")
        got_v = run_full(A, m, n, g.Sched(8, 8, 512, v), rref=False)
        compare(f"65536 sparse {name}", got_v, want)
        del got_v


def test_full_65536_dense_seed2():
    m = n = 65536
    A = synth.random_half(m, n, 2)
    say("[full] 65536^2 p=1/2 seed 2")
    got = run_full(A, m, n)
    compare("65536 seed 2", got, oracle.pls(A, m, n))


def test_full_32768_iid_mmpf_and_recursive():
    m = n = 32768
    A = synth.random_half(m, n, 1)
    say("[full] 32768^2 p=1/2 seed 1, recursive")
    want = oracle.pls(A, m, n)
    got = run_full(A, m, n)
    compare("32768 iid, recursive", got, want)
    r, P, Q, Ap = want
    if r < n:
        check_rref_properties(got[4], s_rows(Ap, r, Q, n), r, Q, n)
    del got
    say("[full] the same matrix by MMPF alone")
    got_m = run_full(A, m, n, g.Sched(8, 8, 1 << 20, g.SCHUR_FP4), rref=False)
    compare("32768 iid, MMPF", got_m, want)


def test_full_32768x131072_sparse():
    m, n = 32768, 131072
    A = synth.random_bernoulli(m, n, 0.01, 4)
    say("[full] 32768x131072 p=0.01 seed 4")
    got = run_full(A, m, n)
    want = oracle.pls(A, m, n)
    compare("32768x131072 sparse", got, want)
    r, P, Q, Ap = want
    check_rref_properties(got[4], s_rows(Ap, r, Q, n), r, Q, n)


def test_full_32768x131072_all_schur_variants():
    m, n = 32768, 131072
    A = synth.random_half(m, n, 3)
    say("[full] 32768x131072 p=1/2 seed 3")
    got = run_full(A, m, n)
    want = oracle.pls(A, m, n)
    compare("32768x131072", got, want)
    r, P, Q, Ap = want
    S = s_rows(Ap, r, Q, n)
    check_rref_properties(got[4], S, r, Q, n)
    del got
    for name, v in (("int8 MFMA", g.SCHUR_MFMA), ("XOR", g.SCHUR_XOR)):
        say(f"[full] 32768x131072 with the {name} Schur product (PLS and RREF)")
        got_v = run_full(A, m, n, g.Sched(8, 8, 512, v))
        compare(f"32768x131072 {name}", got_v, want)
        check_rref_properties(got_v[4], S, r, Q, n)
        del got_v


def test_full_32768_planted_rank_mmpf_and_recursive():
    m = n = 32768
    A = synth.planted(m, n, 24576, 4, p=0.5, unit=False)
    say("[full] 32768^2 planted rank 24576 (B C, Bernoulli(1/2) factors)")
    want = oracle.pls(A, m, n)
    assert want[0] == 24576
    got = run_full(A, m, n)
    compare("32768 planted, recursive", got, want)
    r, P, Q, Ap = want
    check_rref_properties(got[4], s_rows(Ap, r, Q, n), r, Q, n)
    say("[full] the same matrix by MMPF alone")
    got_m = run_full(A, m, n, g.Sched(8, 8, 1 << 20, g.SCHUR_MFMA), rref=False)
    compare("32768 planted, MMPF", got_m, want)
