"""The shared input generators: determinism and the published SplitMix64 values."""
import numpy as np

import synth


def test_splitmix64_reference_values():
    # SplitMix64 from seed 1234567: first outputs of Vigna's reference C code
    z = synth.splitmix64(1234567, 3)
    assert [int(v) for v in z] == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_streams_are_positional():
    a = synth.splitmix64(9, 100)
    b = synth.splitmix64(9, 50, start=50)
    assert np.array_equal(a[50:], b)


def test_subset_patterns():
    p = synth.random_subset_patterns(4, 5000, 32, 16)
    assert all(bin(int(v)).count("1") == 16 for v in p)
    bits = ((p[:, None] >> np.arange(32, dtype=np.uint64)) & np.uint64(1)).mean(axis=0)
    assert np.abs(bits - 0.5).max() < 0.05


def test_start_vector_unit():
    v = synth.start_vector(2, 1000)
    assert abs(np.dot(v, v) - 1) < 1e-14 and v.min() >= -1 and v.max() < 1
