"""The C-ABI library loads and exports every function the public header declares;
host-side validation rejects bad arguments before any launch (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gf2pls.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gf2_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1006_1744_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    import paper_1006_1744_amd as g
    return g.get_lib()


def test_exports_everything_declared(lib):
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.gf2_status_str(code)


def test_sched_validation(lib):
    import paper_1006_1744_amd as g
    s = g.default_sched()
    assert lib.gf2_sched_valid(ctypes.byref(s)) == 1
    for schur in (g.SCHUR_XOR, g.SCHUR_MFMA, g.SCHUR_FP4):
        assert lib.gf2_sched_valid(ctypes.byref(g.Sched(8, 8, 512, schur))) == 1
    for bad in [g.Sched(3, 8, 512, 1), g.Sched(8, 3, 512, 1), g.Sched(8, 8, 100, 1),
                g.Sched(8, 8, 512, 3), g.Sched(8, 8, 512, -1), g.Sched(9, 8, 512, 0)]:
        assert lib.gf2_sched_valid(ctypes.byref(bad)) == 0
        assert lib.gf2_pls_workspace_bytes(100, 100, ctypes.byref(bad)) == 0


def test_workspace_sizes(lib):
    assert lib.gf2_pls_workspace_bytes(-1, 10, None) == 0
    assert lib.gf2_pls_workspace_bytes(4096, 4096, None) > 0
    a = lib.gf2_pls_workspace_bytes(65536, 65536, None)
    # the transposed product operands dominate: at most a quarter of the matrix for
    # a node's Schur operand and an eighth for the products inside triangular
    # solves, plus the base-block copy (at most 16 words per row) and small
    # per-panel state
    assert 0 < a <= 65536 * 65536 // 8 // 4 + 65536 * 65536 // 8 // 8 + 65536 * 16 * 8 + (1 << 20)
    assert lib.gf2_rref_workspace_bytes(100, 200) > 0
    assert lib.gf2_addmul_workspace_bytes(10, 10, 10) > 0


def test_null_context_rejected(lib):
    import paper_1006_1744_amd as g
    m = g.Mat(None, 10, 10, 1)
    assert lib.gf2_pls(None, m, None, None, None, None, None, 0, None) == -1
    assert lib.gf2_rref(None, m, None, None, m, None, None, 0, None) == -1
    assert lib.gf2_addmul(None, m, m, m, 0, None, 0, None) == -1


def test_sched_candidates_counts_and_validity():
    import paper_1006_1744_amd as g
    for m, n, batched, want in [(100, 100, False, 20), (300, 300, False, 80),
                                (5000, 5000, False, 300), (64, 4096, False, 260),
                                (64, 4097, False, 300), (3000, 3000, True, 20)]:
        c = g.sched_candidates(m, n, batched)
        assert len(c) == want
        assert len({x.astuple() for x in c}) == want
        assert all(g.get_lib().gf2_sched_valid(x) == 1 for x in c)
        if not batched:
            ncols = 64 * ((n + 63) // 64)
            # one MMPF-only entry per (k, tables) when some cutoff covers the width
            for k in range(4, 9):
                for t in (1, 2, 4, 8):
                    mm = [x for x in c if x.k == k and x.tables == t and x.cutoff >= ncols]
                    assert len(mm) == (1 if ncols <= 4096 else 0)


def test_mlp_param_counts():
    import paper_1006_1744_amd as g
    assert g.mlp_param_count(200) == 17480
    assert g.mlp_param_count(20) == 5780
    assert g.get_lib().gf2_mlp_param_count(0) < 0
    assert g.get_lib().gf2_mlp_param_count(257) < 0
