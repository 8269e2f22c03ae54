"""gf2_pls_noalloc (the entry point for callers that cannot allocate device
memory) against gf2_pls, through the C ABI: two calls in a row on one device, the
second on a smaller matrix (the shared scratch keeps the first call's contents),
each bit for bit equal to gf2_pls with a fresh workspace and to the oracle; and a
problem whose workspace exceeds the fixed scratch is refused with nothing
written."""
from __future__ import annotations

import ctypes
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


def run_both(A, m, n, s):
    dA1 = g.to_device(A)
    dA2 = g.to_device(A)
    P1, Q1, r1 = g.pls(dA1, m, n, s)
    P2, Q2, r2 = g.pls_noalloc(dA2, m, n, s)
    torch.cuda.synchronize()
    return ((int(r1.item()), P1.cpu().numpy(), Q1.cpu().numpy(), g.to_host(dA1)),
            (int(r2.item()), P2.cpu().numpy(), Q2.cpu().numpy(), g.to_host(dA2)))


@pytest.mark.parametrize("sched", [None, g.Sched(6, 4, 256, g.SCHUR_MFMA)])
def test_noalloc_matches_workspace_call_twice(sched):
    cases = [(3000, 2600, synth.random_half(3000, 2600, 71)),
             (900, 700, synth.planted(900, 700, 500, 72, p=0.5))]
    for m, n, A in cases:
        say(f"[noalloc] {m}x{n} sched={sched}")
        ref, got = run_both(A, m, n, sched)
        want = oracle.pls(A, m, n)
        for label, res in (("gf2_pls", ref), ("gf2_pls_noalloc", got)):
            assert res[0] == want[0], f"{label} rank"
            assert np.array_equal(res[1], want[1]), f"{label} P"
            assert np.array_equal(res[2], want[2]), f"{label} Q"
            assert np.array_equal(res[3], want[3]), f"{label} A'"


def test_noalloc_refuses_oversized_problem():
    lib = g.get_lib()
    limit = int(lib.gf2_pls_noalloc_max_bytes())
    m, n = 64, 65536 * 4   # the transposed Schur operands alone exceed the scratch
    assert g.pls_workspace_bytes(m, n) > limit
    A = torch.zeros((m, n // 64), dtype=torch.int64, device="cuda")
    A[0, 0] = 5
    P = torch.full((m,), -7, dtype=torch.int32, device="cuda")
    Q = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    rank = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    rc = lib.gf2_pls_noalloc(g.ctx(0), g.Mat(A.data_ptr(), m, n, A.shape[1]), P.data_ptr(),
                             Q.data_ptr(), rank.data_ptr(), None,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == -5   # GF2_E_UNSUPPORTED
    assert int(A[0, 0].item()) == 5 and int(A.abs().sum().item()) == 5
    assert int(rank.item()) == -7 and bool((P == -7).all()) and bool((Q == -7).all())
