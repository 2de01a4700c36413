"""Counter-based random draws of the usFFT driver (oracle side).

Alg. 1 draws two kinds of random numbers: the tail components y'_j of the
sampling nodes (steps 1/2a and 2b) and, through Algorithm A, the generating
vectors z of the rank-1 lattices (App. A).  Both implementations draw them
from SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), written here from that published definition:

    state advances by GAMMA = 0x9E3779B97F4A7C15 (mod 2^64), output is
    mix64(state) with Stafford's "variant 13" finalizer.

Keying (a reading of this build; the paper leaves the generator open):
    key(seed, stream) = mix64(seed + GAMMA * (stream + 1))
    draw(seed, stream, idx) = mix64(key + GAMMA * (idx + 1))
    stream = kind << 56 | t << 40 | a << 16 | b

kinds: 1 = step-1 tail of stage (t, i=a), 2 = step-2 tail of stage (t, i=a),
       3 = step-2 lattice generator for J_t (attempt a, try b),
       4 = step-3 lattice generator (attempt a, try b).

Pinned by the SplitMix64 reference outputs for seed 1234567 in
tests/golden/splitmix64.txt.
"""

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15

KIND_TAIL1 = 1
KIND_TAIL2 = 2
KIND_LAT2 = 3
KIND_LAT3 = 4


def mix64(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_sequence(state: int, count: int):
    """The plain SplitMix64 stream: outputs 1..count from `state`."""
    out = []
    for _ in range(count):
        state = (state + GAMMA) & MASK64
        out.append(mix64(state))
    return out


def stream_code(kind: int, t: int, a: int, b: int = 0) -> int:
    return ((kind & 0xFF) << 56) | ((t & 0xFFFF) << 40) | ((a & 0xFFFFFF) << 16) | (b & 0xFFFF)


def draw(seed: int, stream: int, idx: int) -> int:
    key = mix64((seed + GAMMA * (stream + 1)) & MASK64)
    return mix64((key + GAMMA * (idx + 1)) & MASK64)


def uniform01(seed: int, stream: int, idx: int) -> float:
    """53-bit uniform double in [0, 1)."""
    return (draw(seed, stream, idx) >> 11) * (1.0 / 9007199254740992.0)


def lattice_generator(seed: int, stream: int, t: int, M: int):
    """z_j = 1 + draw mod (M-1), j < t: every component is a unit mod prime M."""
    return [1 + draw(seed, stream, j) % (M - 1) for j in range(t)]
