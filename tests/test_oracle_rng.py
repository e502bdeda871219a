"""Pins of the oracle's SplitMix64 probe generator (no GPU)."""
import numpy as np

from oracle import rng


def test_published_reference_outputs():
    """The reference implementation's first outputs (splitmix64.c with the
    state set to 0, and with 1234567, as printed with it and reproduced by
    other SplitMix64 ports): a wrong shift, multiplier or increment changes
    every one of them."""
    assert rng.splitmix64_stream(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                          0x06C45D188009454F]
    assert rng.splitmix64_stream(1234567, 3) == [6457827717110365317, 3203168211198807973,
                                                9817491932198370423]


def test_counter_form_equals_sequential_stepping():
    for seed in (0, 1, 2**63 + 5, 2**64 - 1):
        seq = rng.splitmix64_stream(seed, 500)
        closed = rng.splitmix64_at(seed, np.arange(1, 501))
        assert [int(v) for v in closed] == seq


def test_rademacher_layout_and_balance():
    n, nc, seed = 300, 7, 42
    Z = rng.rademacher(n, nc, seed)
    assert Z.shape == (n, nc) and set(np.unique(Z)) == {-1.0, 1.0}
    seq = rng.splitmix64_stream(seed, n * nc)
    want = np.array([-1.0 if v >> 63 else 1.0 for v in seq]).reshape(n, nc)
    assert np.array_equal(Z, want)   # row-major: element (i, c) is output i * nc + c + 1
    big = rng.rademacher(200_000, 5, 7)
    assert abs(big.mean()) < 4 / np.sqrt(big.size)   # fair signs within 4 sigma
    assert abs((big[:, 0] * big[:, 1]).mean()) < 4 / np.sqrt(big.shape[0])   # columns uncorrelated
