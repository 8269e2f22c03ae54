"""Host-forced failures through the C-ABI on a real device context: each call
with a bad argument (workspace too small or missing, misaligned pointers, a
stride below ceil(n/64), null outputs, an invalid schedule, mismatched shapes)
returns its status code before anything is enqueued, and the matrix and the
output buffers keep their contents."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU runs deselect the marker anyway
    pytest.skip("no GPU", allow_module_level=True)

import paper_1006_1744_amd as g  # noqa: E402

E_ARG, E_ALIGN, E_WS, E_UNSUP = -1, -2, -3, -5


def sentinel(n, dtype=torch.int32):
    return torch.full((max(n, 1),), -7, dtype=dtype, device="cuda")


def test_pls_errors_leave_inputs_untouched():
    m, n = 300, 500
    A = synth.random_half(m, n, 5)
    dA = g.to_device(A)
    stride = dA.shape[1]
    L, c, st = g.get_lib(), g.ctx(), g._stream()
    need = g.pls_workspace_bytes(m, n)
    ws = g.workspace(need + 4096)
    P, Q, rank = sentinel(m), sentinel(n), sentinel(1)
    good = g.Mat(dA.data_ptr(), m, n, stride)

    def call(mat=good, wsp=ws.data_ptr(), wsb=need, p=P.data_ptr(), q=Q.data_ptr(),
             rk=rank.data_ptr(), s=None):
        return L.gf2_pls(c, mat, p, q, rk, s, wsp, wsb, st)

    assert call(wsb=need - 1) == E_WS
    assert call(wsp=None, wsb=0) == E_WS
    assert call(wsp=ws.data_ptr() + 8) == E_ALIGN
    assert call(mat=g.Mat(dA.data_ptr(), m, n, (n + 63) // 64 - 1)) == E_ALIGN
    assert call(mat=g.Mat(dA.data_ptr() + 4, m, n, stride)) == E_ALIGN
    assert call(mat=g.Mat(None, m, n, stride)) == E_ARG
    assert call(mat=g.Mat(dA.data_ptr(), -1, n, stride)) == E_UNSUP
    assert call(p=None) == E_ARG
    assert call(q=None) == E_ARG
    assert call(rk=None) == E_ARG
    assert call(s=ctypes.byref(g.Sched(3, 8, 512, g.SCHUR_FP4))) == E_ARG
    assert call(s=ctypes.byref(g.Sched(8, 8, 100, g.SCHUR_FP4))) == E_ARG
    assert L.gf2_pls(None, good, P.data_ptr(), Q.data_ptr(), rank.data_ptr(), None, ws.data_ptr(),
                     need, st) == E_ARG
    torch.cuda.synchronize()
    assert np.array_equal(g.to_host(dA), A)
    assert (P == -7).all() and (Q == -7).all() and (rank == -7).all()
    # the same buffers then work
    assert call() == 0
    torch.cuda.synchronize()
    assert int(rank.item()) == min(m, n)


def test_rref_errors_leave_inputs_untouched():
    m, n = 200, 330
    A = synth.random_half(m, n, 6)
    dA = g.to_device(A)
    P, Q, rank = g.pls(dA, m, n)
    torch.cuda.synchronize()
    Ap = g.to_host(dA)
    L, c, st = g.get_lib(), g.ctx(), g._stream()
    need = g.rref_workspace_bytes(m, n)
    ws = g.workspace(need + 4096)
    dR = torch.full_like(dA, -3)
    stride = dA.shape[1]
    good = g.Mat(dA.data_ptr(), m, n, stride)
    outm = g.Mat(dR.data_ptr(), m, n, stride)

    def call(a=good, r=outm, wsp=ws.data_ptr(), wsb=need, q=Q.data_ptr(), rk=rank.data_ptr(),
             s=None):
        return L.gf2_rref(c, a, q, rk, r, s, wsp, wsb, st)

    assert call(wsb=need - 1) == E_WS
    assert call(wsp=ws.data_ptr() + 16) == E_ALIGN
    assert call(r=good) == E_ARG                                   # R aliases A
    assert call(r=g.Mat(dR.data_ptr(), m - 1, n, stride)) == E_ARG  # shape mismatch
    assert call(r=g.Mat(dR.data_ptr(), m, n, (n + 63) // 64 - 1)) == E_ALIGN
    assert call(q=None) == E_ARG
    assert call(rk=None) == E_ARG
    assert call(s=ctypes.byref(g.Sched(8, 8, 512, 7))) == E_ARG
    torch.cuda.synchronize()
    assert np.array_equal(g.to_host(dA), Ap)
    assert (dR == -3).all()


def test_addmul_unpack_batched_errors():
    L, c, st = g.get_lib(), g.ctx(), g._stream()
    m, k, n = 100, 70, 130
    dA, dB = g.to_device(synth.random_half(m, k, 1)), g.to_device(synth.random_half(k, n, 2))
    C = synth.random_half(m, n, 3)
    dC = g.to_device(C)
    need = int(L.gf2_addmul_workspace_bytes(m, k, n))
    ws = g.workspace(need + 4096)
    MA, MB, MC = (g.Mat(dA.data_ptr(), m, k, dA.shape[1]), g.Mat(dB.data_ptr(), k, n, dB.shape[1]),
                  g.Mat(dC.data_ptr(), m, n, dC.shape[1]))
    assert L.gf2_addmul(c, MC, MA, MB, g.SCHUR_FP4, ws.data_ptr(), need - 1, st) == E_WS
    assert L.gf2_addmul(c, MC, MA, MB, 3, ws.data_ptr(), need, st) == E_ARG
    assert L.gf2_addmul(c, MC, MB, MA, g.SCHUR_FP4, ws.data_ptr(), need, st) == E_ARG
    # unpack: L_out / S_out of the wrong shape
    P, Q, rank = g.pls(g.to_device(synth.random_half(m, n, 4)), m, n)
    bad = g.Mat(dC.data_ptr(), m, n, dC.shape[1])
    assert L.gf2_pls_unpack(c, MC, Q.data_ptr(), rank.data_ptr(), bad, bad, st) == E_ARG
    # batched: workspace too small or misaligned
    mats = [g.to_device(synth.random_half(64, 64, 9))]
    b = g.Batch(mats, [(64, 64)])
    b.ranks.fill_(-7)
    nb = b.ws.numel()
    assert L.gf2_pls_batched(c, b.items.data_ptr(), 1, b.ranks.data_ptr(), None, None,
                             b.ws.data_ptr(), nb - 1, st) == E_WS
    assert L.gf2_pls_batched(c, b.items.data_ptr(), 1, b.ranks.data_ptr(), None, None,
                             b.ws.data_ptr() + 8, nb, st) == E_ALIGN
    assert L.gf2_pls_batched(c, b.items.data_ptr(), -1, b.ranks.data_ptr(), None, None,
                             b.ws.data_ptr(), nb, st) == E_ARG
    torch.cuda.synchronize()
    assert np.array_equal(g.to_host(dC), C)
    assert (b.ranks == -7).all()
