"""The full-size RREF checks (tests/rref_checks.py) accept the oracle's RREF and
reject every planted mistake: a flipped bit in a non-pivot column, in a pivot
column or past the rank, two rows exchanged, and the echelon rows S in place of
R."""
import numpy as np
import pytest

import oracle
import synth
from rref_checks import rref_violations, s_rows


@pytest.mark.parametrize("m,n,kind", [(40, 70, "half"), (90, 60, "planted"), (130, 200, "sparse"),
                                      (64, 64, "half"), (5, 3, "half")])
def test_rref_checks_accept_and_reject(m, n, kind):
    if kind == "half":
        A = synth.random_half(m, n, m + n)
    elif kind == "planted":
        A = synth.planted(m, n, 37, 3, p=0.5)
    else:
        A = synth.random_bernoulli(m, n, 0.05, 5)
    r, P, Q, Ap = oracle.pls(A, m, n)
    rr, R, piv = oracle.rref(A, m, n)
    assert rr == r and np.array_equal(piv, Q[:r])
    S = s_rows(Ap, r, Q, n)
    assert rref_violations(R, S, r, Q, n) == []
    Rb = oracle.unpack_bits(R, n)
    nonpiv = [j for j in range(n) if j not in set(Q[:r].tolist())]
    mutants = []
    if nonpiv and r:
        X = Rb.copy(); X[r // 2, nonpiv[len(nonpiv) // 2]] ^= 1; mutants.append(X)
    if r:
        X = Rb.copy(); X[0, Q[r - 1]] ^= 1; mutants.append(X)
    if r < m:
        X = Rb.copy(); X[m - 1, n - 1] ^= 1; mutants.append(X)
    if r >= 2:
        X = Rb.copy(); X[[0, 1]] = X[[1, 0]]; mutants.append(X)
    if r and not np.array_equal(oracle.unpack_bits(S, n), Rb[:r]):
        X = Rb.copy(); X[:r] = oracle.unpack_bits(S, n); mutants.append(X)
    assert mutants
    for X in mutants:
        assert rref_violations(oracle.pack_bits(X), S, r, Q, n) != []
