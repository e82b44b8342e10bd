"""Counter-based uniform random numbers, identical on the host and on the device.

Every random value used by a workload is a pure function of (seed, stream,
index), so any subset of a huge input can be regenerated on the host for the
oracle without materialising the rest, and the device generator in
``devgen.hip`` produces bit-identical values.

Definition (one 64-bit counter per value):

    x = seed * 0xD1B54A32D192ED03 + stream * 0x9E3779B97F4A7C15 + index   (mod 2^64)
    z = splitmix64_finalise(x + 0x9E3779B97F4A7C15)
    u = (z >> 11) * 2^-53                                               in [0, 1)
    U(lo, hi) = lo + (hi - lo) * u        (two separately rounded FP64 ops)

``splitmix64_finalise`` is the published SplitMix64 output function of Steele,
Lea and Flood (OOPSLA 2014): xor-shift 30, multiply, xor-shift 27, multiply,
xor-shift 31.  This module holds no tridiagonal-solver arithmetic.
"""
import numpy as np

_U64 = np.uint64
_SEED_MUL = _U64(0xD1B54A32D192ED03)
_GOLDEN = _U64(0x9E3779B97F4A7C15)
_M1 = _U64(0xBF58476D1CE4E5B9)
_M2 = _U64(0x94D049BB133111EB)
_TWO_M53 = float(2.0 ** -53)

# Stream ids: one per kind of random draw.
STREAM_A = 1
STREAM_B = 2
STREAM_C = 3
STREAM_D = 4
STREAM_X = 5
STREAM_NOISE = 6
STREAM_RAGGED_N = 7
STREAM_MARGIN = 8


def _finalise(z):
    z = (z ^ (z >> _U64(30))) * _M1
    z = (z ^ (z >> _U64(27))) * _M2
    return z ^ (z >> _U64(31))


def raw64(seed, stream, index):
    """64-bit hash of (seed, stream, index); index is an int or int ndarray."""
    idx = np.asarray(index, dtype=np.int64).astype(_U64)
    with np.errstate(over="ignore"):
        x = _U64(seed) * _SEED_MUL + _U64(stream) * _GOLDEN
        z = _finalise(idx + x + _GOLDEN)
    return z


def uniform01(seed, stream, index):
    """u in [0, 1) with 53 random bits."""
    z = raw64(seed, stream, index)
    return (z >> _U64(11)).astype(np.float64) * _TWO_M53


def uniform(seed, stream, index, lo, hi):
    """U(lo, hi) = lo + (hi - lo) * u, rounded exactly as the device does."""
    u = uniform01(seed, stream, index)
    span = np.float64(hi) - np.float64(lo)
    return np.float64(lo) + span * u
