"""The host AVX2 lookup baseline agrees with the oracle on validity (CPU only)."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2010_03090_amd import baselines, synth

pytestmark = pytest.mark.skipif(not baselines.supported(), reason="no AVX2 on this host")


def test_agrees_with_oracle_short_strings():
    alpha = [0x00, 0x41, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF, 0xE0, 0xE1, 0xED,
             0xEE, 0xEF, 0xF0, 0xF1, 0xF4, 0xF5, 0xFF]
    for n in (0, 1, 2, 3):
        for t in itertools.product(alpha, repeat=n):
            b = np.array(t, np.uint8)
            assert baselines.is_valid(b) == oracle.is_valid(b), bytes(t).hex()


def test_agrees_with_oracle_around_block_edges():
    rng = np.random.default_rng(71)
    for variant in ("mixed", "emoji", "ascii", "cjk"):
        for n in (31, 32, 33, 63, 64, 65, 127, 128, 129, 1000, 4099):
            b = synth.text(n, variant, n)
            assert baselines.is_valid(b) and oracle.is_valid(b)
            for trial in range(12):
                c = b.copy()
                synth.inject(c, int(rng.integers(0, n)), int(rng.integers(0, 7)), trial)
                assert baselines.is_valid(c) == oracle.is_valid(c), (variant, n, trial)
    for n in range(0, 130):
        r = rng.integers(0, 256, n, dtype=np.uint8)
        assert baselines.is_valid(r) == oracle.is_valid(r)


def test_multithreaded_spans():
    b = synth.text(24 << 20, "mixed", 5)
    assert baselines.is_valid(b, nthreads=8)
    for pos in (1 << 20, (3 << 20) - 1, (3 << 20) - 2, 7 << 20, (24 << 20) - 2):
        c = b.copy()
        synth.inject(c, pos, "truncated_lead", pos)
        assert baselines.is_valid(c, nthreads=8) == oracle.is_valid(c) == False
