import os

from oracle import rng

HERE = os.path.dirname(os.path.abspath(__file__))


def test_splitmix64_reference_vector():
    # published SplitMix64 conformance values for state 1234567
    vals = [int(l) for l in open(os.path.join(HERE, "golden", "splitmix64.txt")) if l.strip() and not l.startswith("#")]
    assert rng.splitmix64_sequence(1234567, 5) == vals


def test_draw_is_splitmix_stream():
    # draw(seed, stream, idx) is output idx+1 of SplitMix64 started at key(seed, stream)
    seed, stream = 99, rng.stream_code(2, 3, 4)
    key = rng.splitmix64_sequence(seed + rng.GAMMA * stream, 1)[0]
    seq = rng.splitmix64_sequence(key, 6)
    assert [rng.draw(seed, stream, j) for j in range(6)] == seq


def test_uniform_and_generator_ranges():
    for j in range(200):
        u = rng.uniform01(5, 77, j)
        assert 0.0 <= u < 1.0
    z = rng.lattice_generator(3, 11, 30, 101)
    assert all(1 <= v <= 100 for v in z)
    # streams are distinct
    assert rng.stream_code(1, 2, 3, 4) != rng.stream_code(1, 2, 4, 3)
