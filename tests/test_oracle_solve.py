"""Pins of the oracle's solving functions (A x = b and the null space from the
PLS) against what the mathematics fixes: brute force over every x on tiny
systems, the structure of the solution sets, and planted mistakes."""
import itertools

import numpy as np
import pytest

import oracle
import synth


def bits(A, n):
    return oracle.unpack_bits(A, n).astype(np.int64)


def all_x(n):
    return np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.int64)[:, ::-1]


@pytest.mark.parametrize("m,n", [(1, 1), (3, 5), (5, 3), (6, 6), (7, 9), (9, 7), (8, 8)])
@pytest.mark.parametrize("seed", range(3))
def test_solve_matches_brute_force(m, n, seed):
    rng = np.random.default_rng(1000 * m + 10 * n + seed)
    for planted_r in sorted({0, 1, min(m, n) // 2, min(m, n)}):
        A = synth.planted(m, n, planted_r, 17 + seed, p=0.5, unit=False) if planted_r else \
            oracle.pack_bits(np.zeros((m, n), np.uint8))
        Ab = bits(A, n)
        r, P, Q, Ap = oracle.pls(A, m, n)
        X = all_x(n)
        images = (X @ Ab.T) & 1                       # A x for every x, rows
        for trial in range(6):
            if trial % 2 == 0:                        # a consistent right-hand side
                b = images[rng.integers(0, len(X))].astype(np.uint8)
            else:
                b = rng.integers(0, 2, m).astype(np.uint8)
            x = oracle.solve_from_pls(b, m, n, r, P, Q, Ap)
            solvable = bool(np.any(np.all(images == b[None, :], axis=1)))
            assert (x is not None) == solvable
            if x is not None:
                assert np.array_equal((Ab @ x.astype(np.int64)) & 1, b)
                # non-pivot entries are zero
                piv = set(int(q) for q in Q[:r])
                assert all(x[j] == 0 for j in range(n) if j not in piv)


@pytest.mark.parametrize("m,n", [(4, 7), (7, 4), (6, 6), (9, 8)])
@pytest.mark.parametrize("seed", range(3))
def test_kernel_basis_matches_brute_force(m, n, seed):
    A = synth.random_bernoulli(m, n, 0.4, 50 + seed)
    Ab = bits(A, n)
    r, P, Q, Ap = oracle.pls(A, m, n)
    K = oracle.kernel_basis(m, n, r, Q, Ap)
    assert K.shape == (n - r, n)
    assert not np.any((Ab @ K.T.astype(np.int64)) & 1)
    # independent: the span has 2^(n-r) elements, equal to the brute-force kernel
    span = {tuple(((np.array(c, np.int64) @ K.astype(np.int64)) & 1).tolist())
            for c in itertools.product((0, 1), repeat=n - r)} if n - r else {tuple([0] * n)}
    X = all_x(n)
    kernel = {tuple(x.tolist()) for x in X if not np.any((Ab @ x) & 1)}
    assert span == kernel and len(kernel) == 2 ** (n - r)


def test_special_systems():
    m = n = 70
    I = oracle.pack_bits(np.eye(m, n, dtype=np.uint8))
    r, P, Q, Ap = oracle.pls(I, m, n)
    b = np.random.default_rng(1).integers(0, 2, m).astype(np.uint8)
    assert np.array_equal(oracle.solve_from_pls(b, m, n, r, P, Q, Ap), b)
    assert oracle.kernel_basis(m, n, r, Q, Ap).shape == (0, n)
    Z = oracle.pack_bits(np.zeros((m, n), np.uint8))
    r, P, Q, Ap = oracle.pls(Z, m, n)
    assert r == 0
    assert np.array_equal(oracle.solve_from_pls(np.zeros(m, np.uint8), m, n, r, P, Q, Ap),
                          np.zeros(n, np.uint8))
    assert oracle.solve_from_pls(np.eye(1, m, 5, dtype=np.uint8)[0], m, n, r, P, Q, Ap) is None
    assert np.array_equal(oracle.kernel_basis(m, n, r, Q, Ap), np.eye(n, dtype=np.uint8))


@pytest.mark.parametrize("m,n,rank", [(300, 400, 250), (400, 300, 300), (257, 257, 200)])
def test_solve_medium(m, n, rank):
    A = synth.planted(m, n, rank, 3, p=0.5, unit=True)
    Ab = bits(A, n)
    r, P, Q, Ap = oracle.pls(A, m, n)
    assert r == rank
    rng = np.random.default_rng(7)
    x0 = rng.integers(0, 2, n)
    b = ((Ab @ x0) & 1).astype(np.uint8)
    x = oracle.solve_from_pls(b, m, n, r, P, Q, Ap)
    assert x is not None and np.array_equal((Ab @ x.astype(np.int64)) & 1, b)
    K = oracle.kernel_basis(m, n, r, Q, Ap)
    assert K.shape == (n - r, n) and not np.any((Ab @ K.T.astype(np.int64)) & 1)
    # x0 - x lies in the span of K: appending it does not raise the rank
    KK = np.vstack([K, ((x0 - x.astype(np.int64)) & 1).astype(np.uint8)[None, :]])
    assert oracle.pls(oracle.pack_bits(KK), KK.shape[0], n)[0] == n - r


def test_planted_mistakes_are_caught(monkeypatch):
    """Each of three plausible mistakes in the solver (no forward substitution with
    L, no use of S's entries right of the pivots, no consistency rows) fails the
    brute-force check; the real solver passes it."""
    m, n = 7, 9
    # an instance where every mutation can matter: rows past the rank, a non-identity
    # triangle in L, and S coupling pivot columns (first such seed)
    for seed in range(200):
        A = synth.planted(m, n, 5, seed, p=0.5, unit=False)
        r, P, Q, Ap = oracle.pls(A, m, n)
        L, S = oracle.unpack_LS(Ap, m, n, r, Q)
        piv = [int(q) for q in Q[:r]]
        coupled = any(S[i, j] for i in range(r) for j in piv if j > piv[i])
        if r < m and np.any(np.tril(L[:r], -1)) and coupled:
            break
    else:
        pytest.fail("no suitable instance")
    Ab = bits(A, n)
    X = all_x(n)
    images = (X @ Ab.T) & 1
    rhs = [images[i].astype(np.uint8) for i in range(0, len(X), 7)] + \
          [np.array(v, np.uint8) for v in itertools.product((0, 1), repeat=m)]

    def fails():
        for b in rhs:
            x = oracle.solve_from_pls(b, m, n, r, P, Q, Ap)
            solvable = bool(np.any(np.all(images == b[None, :], axis=1)))
            if (x is not None) != solvable:
                return True
            if x is not None and not np.array_equal((Ab @ x.astype(np.int64)) & 1, b):
                return True
        return False

    assert not fails()
    real_unpack = oracle.unpack_LS

    def mutate(kind):
        def unpack(Ap_, m_, n_, r_, Q_):
            L, S = real_unpack(Ap_, m_, n_, r_, Q_)
            L, S = L.copy(), S.copy()
            if kind == "no_forward":
                L[:r_, :] = np.eye(r_, dtype=np.uint8)[:, :L.shape[1]]
            elif kind == "no_S_tail":
                for i in range(r_):
                    S[i, int(Q_[i]) + 1:] = 0
            elif kind == "no_consistency_rows":
                L[r_:, :] = 0
            return L, S
        return unpack

    for kind in ("no_forward", "no_S_tail", "no_consistency_rows"):
        monkeypatch.setattr(oracle, "unpack_LS", mutate(kind))
        assert fails(), kind
    monkeypatch.setattr(oracle, "unpack_LS", real_unpack)
    assert not fails()
