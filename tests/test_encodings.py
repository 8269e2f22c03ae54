"""Host-side checks of two encodings the GPU kernels rely on (pure Python models
of the arithmetic, no GPU):

* the matrix-core operand encodings of the Schur product: a lane's 32 K-bits
  become fp4 (e2m1) nibbles or int8 bytes whose products, summed over every
  (register, element), count exactly the K positions where both operands have a
  one, so the parity of the sum is the GF(2) dot product;
* the butterfly stage of the 64 x 64 bit transpose, in the form where each lane
  sends its value already shifted toward the partner and keeps its own half with
  one bit select: six stages give the transpose;
* the rows of a panel's L^-1 as the post pass forms them: the strictly lower
  part of L gathered into pivot order, then forward substitution by rows with
  only the low 32-bit halves changing before step 32.
"""
import random

import pytest

# e2m1 (OCP MX fp4): sign, 2 exponent bits (bias 1), 1 mantissa bit; exponent 0
# is subnormal (0.m * 2^0).
def e2m1(code: int) -> float:
    sign = -1.0 if code & 8 else 1.0
    e, mnt = (code >> 1) & 3, code & 1
    if e == 0:
        return sign * 0.5 * mnt
    return sign * (1.0 + 0.5 * mnt) * 2.0 ** (e - 1)


M32 = 0xFFFFFFFF


def fp4_a(w: int) -> list[int]:
    return [w & 0x11111111, w & 0x22222222, w & 0x44444444, (w >> 2) & 0x22222222]


def fp4_b(w: int) -> list[int]:
    return [(w << 2) & 0x44444444, w & 0x22222222, (w >> 2) & 0x11111111, (w >> 2) & 0x22222222]


def fp4_pair(lo: int, hi: int, side: str) -> list[list[int]]:
    """The kernel's form: the shifted copies of two consecutive K steps' words come
    from one 64-bit shift of (hi:lo) each way, then the same masks."""
    p = (hi << 32) | lo
    s2, l2 = p >> 2, (p << 2) & ((1 << 64) - 1)
    out = []
    for j, d in enumerate((lo, hi)):
        sj, lj = (s2 >> (32 * j)) & M32, (l2 >> (32 * j)) & M32
        if side == "a":
            out.append([d & 0x11111111, d & 0x22222222, d & 0x44444444, sj & 0x22222222])
        else:
            out.append([lj & 0x44444444, d & 0x22222222, sj & 0x11111111, sj & 0x22222222])
    return out


def i8_regs(w: int) -> list[int]:
    return [(w >> (4 * s + v)) & 0x01010101 for s in (0, 1) for v in range(4)]


def test_e2m1_table():
    # the codes the encoding uses, and the full non-negative range
    assert [e2m1(c) for c in range(8)] == [0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0]
    assert e2m1(0b1000) == 0.0 and e2m1(0b1010) == -1.0


@pytest.mark.parametrize("seed", range(4))
def test_fp4_operands_count_matching_bits(seed):
    rng = random.Random(seed)
    words = [0, 0xFFFFFFFF, 1, 1 << 31, 0x80000001] + [rng.getrandbits(32) for _ in range(300)]
    for wa in words:
        for wb in rng.sample(words, 20):
            ra, rb = fp4_a(wa), fp4_b(wb)
            total = 0.0
            for v in range(4):
                for n in range(8):
                    total += e2m1((ra[v] >> (4 * n)) & 15) * e2m1((rb[v] >> (4 * n)) & 15)
            assert total == bin(wa & wb).count("1")


def test_fp4_operands_map_each_bit_once():
    # bit k of w lands in exactly one (register, nibble) on each side, the same one
    for k in range(32):
        pa = [(v, n) for v, r in enumerate(fp4_a(1 << k)) for n in range(8) if (r >> (4 * n)) & 15]
        pb = [(v, n) for v, r in enumerate(fp4_b(1 << k)) for n in range(8) if (r >> (4 * n)) & 15]
        assert len(pa) == 1 and pa == pb
        v, n = pa[0]
        assert e2m1((fp4_a(1 << k)[v] >> (4 * n)) & 15) * e2m1((fp4_b(1 << k)[v] >> (4 * n)) & 15) == 1.0


@pytest.mark.parametrize("seed", range(2))
def test_fp4_pair_shifts_match_per_word(seed):
    # the bits a 64-bit shift carries across the two words land where the masks clear
    rng = random.Random(50 + seed)
    words = [0, M32, 1, 3, 1 << 30, 1 << 31, 0xC0000003] + [rng.getrandbits(32) for _ in range(200)]
    for lo in words:
        for hi in rng.sample(words, 20):
            assert fp4_pair(lo, hi, "a") == [fp4_a(lo), fp4_a(hi)]
            assert fp4_pair(lo, hi, "b") == [fp4_b(lo), fp4_b(hi)]


@pytest.mark.parametrize("seed", range(2))
def test_int8_operands_count_matching_bits(seed):
    rng = random.Random(100 + seed)
    for _ in range(500):
        wa, wb = rng.getrandbits(32), rng.getrandbits(32)
        ra, rb = i8_regs(wa), i8_regs(wb)
        total = sum(((ra[j] >> (8 * t)) & 255) * ((rb[j] >> (8 * t)) & 255)
                    for j in range(8) for t in range(4))
        assert total == bin(wa & wb).count("1")


M64 = (1 << 64) - 1
HI = [0xFFFFFFFF00000000, 0xFFFF0000FFFF0000, 0xFF00FF00FF00FF00,
      0xF0F0F0F0F0F0F0F0, 0xCCCCCCCCCCCCCCCC, 0xAAAAAAAAAAAAAAAA]


def transpose_stages(rows: list[int]) -> list[int]:
    v = list(rows)
    for k in range(6):
        s, mh = 32 >> k, HI[k]
        sent = [((x << s) & M64) if (lane & s) else (x >> s) for lane, x in enumerate(v)]
        q = [sent[lane ^ s] for lane in range(64)]
        keep = [mh if (lane & s) else (~mh & M64) for lane in range(64)]
        v = [(v[lane] & keep[lane]) | (q[lane] & ~keep[lane] & M64) for lane in range(64)]
    return v


@pytest.mark.parametrize("seed", range(3))
def test_transpose_stages(seed):
    rng = random.Random(seed)
    rows = [rng.getrandbits(64) for _ in range(64)]
    got = transpose_stages(rows)
    want = [sum(((rows[i] >> j) & 1) << i for i in range(64)) for j in range(64)]
    assert got == want
    assert transpose_stages(got) == rows


def linv_rows_model(u: list[int], q: list[int], ru: int) -> list[int]:
    """Lane t's result of the post pass's L^-1 routine: u[t] the pivot word of
    row t (0 past ru), q[t] its pivot column (t itself past ru)."""
    uq = [sum(((u[t] >> q[s]) & 1) << s for s in range(64)) for t in range(64)]
    low = [uq[t] & ((1 << t) - 1) if 0 < t < ru else 0 for t in range(64)]
    xlo = [(1 << t) if t < 32 else 0 for t in range(64)]
    xhi = [(1 << (t - 32)) if t >= 32 else 0 for t in range(64)]
    for s in range(63):
        f = [M32 if (low[t] >> s) & 1 else 0 for t in range(64)]   # bit s of the lower part
        rlo = xlo[s]                                                 # row s, final
        xlo = [xlo[t] ^ (rlo & f[t]) for t in range(64)]
        if s >= 32:
            rhi = xhi[s]
            xhi = [xhi[t] ^ (rhi & f[t]) for t in range(64)]
    return [(xhi[t] << 32) | xlo[t] for t in range(64)]


@pytest.mark.parametrize("seed", range(6))
def test_linv_rows_model_inverts_l(seed):
    rng = random.Random(200 + seed)
    ru = [1, 2, 31, 32, 33, 64][seed]
    # pivot columns: identity for even seeds, a scattered choice for odd ones
    cols = list(range(64))
    if seed % 2:
        rng.shuffle(cols)
    q = [cols[t] if t < ru else t for t in range(64)]
    u = [rng.getrandbits(64) if t < ru else 0 for t in range(64)]
    X = linv_rows_model(u, q, ru)
    # L[t][s] = bit q[s] of u[t] for s < t < ru, unit diagonal, identity past ru
    L = [sum((((u[t] >> q[s]) & 1) << s) for s in range(t)) | (1 << t) if t < ru else 1 << t
         for t in range(64)]
    for t in range(64):
        row = 0   # row t of L X over GF(2)
        for s in range(64):
            if (L[t] >> s) & 1:
                row ^= X[s]
        assert row == 1 << t
