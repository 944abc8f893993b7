"""SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), evaluated in counter form with numpy uint64
arithmetic: output number i of a stream is mix64(state0 + (i + 1) * gamma).

Streams are separated by a 64-bit tag mixed into the starting state, so every
input family (bond constants, vacancies, axes, ...) draws its own numbers.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z):
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _start(seed, tag):
    s = np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    t = np.array([tag & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    with np.errstate(over="ignore"):
        return (_mix64(t + _GAMMA) ^ s)[0]


def splitmix64(seed, n, tag=0, offset=0):
    """n successive 64-bit outputs (uint64 array) of stream (seed, tag)."""
    i = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _start(seed, tag) + i * _GAMMA
    return _mix64(z)


def uniform01(seed, n, tag=0, offset=0):
    """Doubles in [0, 1) with 53 random bits."""
    z = splitmix64(seed, n, tag, offset)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal01(seed, n, tag=0):
    """Standard normal variates by the Box-Muller transform."""
    m = (n + 1) // 2
    u = uniform01(seed, 2 * m, tag)
    u1 = 1.0 - u[0::2]                      # (0, 1]
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])
    return z[:n]


def unit_vectors(seed, n, tag=0):
    """n points uniform on the unit sphere, shape (n, 3)."""
    u = uniform01(seed, 2 * n, tag)
    z = 2.0 * u[0::2] - 1.0
    phi = 2.0 * np.pi * u[1::2]
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    v = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    return v / np.linalg.norm(v, axis=1, keepdims=True)
