"""The practice-shaped workload: iid Bernoulli stand-ins with the sizes and
densities of Table 2's four matrices (Section 7; the matrices themselves are not
available).  On each, the PLS is compared bit for bit with the oracle's Gaussian
PLS, and the reduced row echelon form reached by each of the paper's routes --
PLS then RREF, M4RI, and the M+P hybrid at the two thresholds of Table 2 (0.15
and 0.20) -- word for word with the oracle's Gauss-Jordan reduction."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU runs deselect the marker anyway
    pytest.skip("no GPU", allow_module_level=True)

import paper_1006_1744_amd as g  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("shape", synth.PRACTICE_SHAPES, ids=lambda s: s.name)
def test_practice_shape_all_routes(shape):
    m, n = shape.m, shape.n
    A = synth.practice_matrix(shape)
    say(f"[practice] {shape.name} {m}x{n} p={shape.p}: oracle PLS and Gauss-Jordan")
    r, P, Q, Ap = oracle.pls(A, m, n)
    rr, Rw, piv = oracle.rref(A, m, n)
    assert rr == r and np.array_equal(piv, Q[:r])

    def check_rref(label, got, gQ, grank):
        assert grank == r, f"{label}: rank {grank} != {r}"
        assert np.array_equal(gQ[:r], piv), f"{label}: pivot columns differ"
        assert np.array_equal(got, Rw), f"{label}: RREF differs"

    say(f"[practice] {shape.name}: PLS + RREF")
    dA = g.to_device(A)
    dP, dQ, drank = g.pls(dA, m, n)
    dR = g.rref(dA, m, n, dQ, drank)
    torch.cuda.synchronize()
    assert int(drank.item()) == r
    assert np.array_equal(dP.cpu().numpy(), P) and np.array_equal(dQ.cpu().numpy(), Q)
    assert np.array_equal(g.to_host(dA), Ap), "PLS differs"
    check_rref("PLS+RREF", g.to_host(dR), dQ.cpu().numpy(), r)
    del dR
    say(f"[practice] {shape.name}: M4RI")
    dA = g.to_device(A)
    mQ, mrank = g.m4ri(dA, m, n)
    torch.cuda.synchronize()
    check_rref("M4RI", g.to_host(dA), mQ.cpu().numpy(), int(mrank.item()))
    for th in (0.15, 0.20):
        dA = g.to_device(A)
        hQ, hrank, sw = g.rref_mp(dA, m, n, th)
        torch.cuda.synchronize()
        say(f"[practice] {shape.name}: M+P {th} switched at strip {sw}")
        check_rref(f"M+P {th}", g.to_host(dA), hQ.cpu().numpy(), int(hrank.item()))
