"""Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and
Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3" (SC'11), written from
its published definition: ten rounds of two 32x32->64-bit multiplies with the
published multipliers, a Weyl-sequence key schedule with the published
increments, and the round permutation of the 4x32 variant.

Sample streams used by the renderers:
  key     = (seed & 0xffffffff, seed >> 32)
  counter = (pixel = y*W + x, sample, segment, camera or request id)
  words 0,1 drive the bounce direction sampled at the hit of that segment,
  word 2 drives Russian roulette after that reflection, word 3 is unused;
  camera jitter uses segment word 0xffffffff, words 0 and 1.
  A word w maps to u = (w >> 8) * 2^-24 in [0, 1 - 2^-24], exact in both
  float32 and float64.

Pinned by tests/test_oracle_philox.py against rocRAND's open-source
Philox4x32-10 (a library routine compiled from its header on the host).
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_LO = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, seed: int):
    """Return the four 32-bit output words (uint32 arrays, broadcast over the
    counter words) for counter (c0, c1, c2, c3) and 64-bit seed."""
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & _LO for c in (c0, c1, c2, c3))
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64((seed >> 32) & 0xFFFFFFFF)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _LO
            k1 = (k1 + _W1) & _LO
        p0 = _M0 * x0           # < 2^64: exact in uint64
        p1 = _M1 * x2
        x0, x1, x2, x3 = ((p1 >> _S32) ^ x1 ^ k0, p1 & _LO, (p0 >> _S32) ^ x3 ^ k1, p0 & _LO)
    return tuple(w.astype(np.uint32) for w in (x0, x1, x2, x3))


def to_unit(w):
    """u = (w >> 8) * 2^-24 as float64."""
    return (np.asarray(w, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * (2.0 ** -24)


def uniforms(pixel, sample, segment, stream_id, seed: int):
    """(u0, u1, u2, u3) float64 for the given counters."""
    return tuple(to_unit(w) for w in philox4x32_10(pixel, sample, segment, stream_id, seed))
