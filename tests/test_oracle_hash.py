"""The stimulus hash is the SplitMix64 output function; pinned to the
published SplitMix64 outputs for state 0 (tests/golden/splitmix64_seed0.txt)."""
from oracle import oracle as O
from tests.conftest import golden_lines

GAMMA = 0x9E3779B97F4A7C15


def test_splitmix64_published_outputs():
    want = [int(x, 16) for x in golden_lines("splitmix64_seed0.txt")]
    got = [O.hash64(k * GAMMA) for k in range(len(want))]
    assert got == want


def test_stimulus_is_nested_hash():
    # structure of the counter-based stimulus: the hash nested three times
    for seed in (0, 1, 0x5EED0000, 2**64 - 1):
        for p in (0, 3, 7):
            for t in (0, 1, 99999):
                assert O.stim(seed, p, t) == O.hash64(O.hash64(O.hash64(seed) ^ p) ^ t)


def test_stimulus_varies():
    vals = {O.stim(0x5EED0000, p, t) for p in range(8) for t in range(64)}
    assert len(vals) == 8 * 64
