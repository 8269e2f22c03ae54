"""The seeded generator: C and Python SplitMix64 agree, densities and shapes."""
import numpy as np

import synth


def test_splitmix_c_matches_python():
    lib = synth._load()
    for seed in (0, 1, 2, 12345, 2**63 + 5):
        for i in (0, 1, 2, 1000, 2**40):
            assert lib.synth_splitmix(seed, i) == synth.splitmix(seed, i)


def test_splitmix_published_first_outputs():
    # SplitMix64 with state 0: first outputs of the published generator
    assert synth.splitmix(0, 0) == 0xE220A8397B1DCDAF
    assert synth.splitmix(0, 1) == 0x6E789E6AA1B965F4


def test_half_words_and_padding():
    a = synth.random_half(5, 70, 3, stride=4)
    assert a.shape == (5, 4)
    assert int(a[2, 0]) == synth.splitmix(3, 2 * 2 + 0)
    assert not a[:, 2:].any()
    assert not (a[:, 1] >> np.uint64(6)).any()


def test_bernoulli_density():
    a = synth.random_bernoulli(200, 300, 0.1, 9)
    d = synth.density(a, 300)
    assert 0.09 < d < 0.11
    b = synth.random_bernoulli(200, 300, 0.1, 9)
    assert np.array_equal(a, b)


def test_batch_shapes():
    items = synth.batch_shapes(200, 7)
    assert all(64 <= it.m <= 2048 and 64 <= it.n <= 2048 for it in items)
    assert all((min(it.m, it.n) + 1) // 2 <= it.r <= min(it.m, it.n) for it in items)
    assert {it.p for it in items} == {0.5, 0.1, 0.01}
    assert synth.batch_shapes(5, 7)[3] == items[3]
