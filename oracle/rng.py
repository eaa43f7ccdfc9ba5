"""Counter-based random numbers and the logarithm used by the sampler.

The paper draws its index samples "without replacement" with probabilities
proportional to the measure of importance (Sec. 3.1, Algorithm 1, the sampling
step) but names no generator.  The reading used here is counter-based so that
any thread of the GPU and this oracle can draw the same number independently:

* Philox4x32-10 as defined by Salmon, Moraes, Dror, Shaw, "Parallel random
  numbers: as easy as 1, 2, 3", SC'11: 10 rounds of the 4x32 Philox S-box
  with multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key increments
  0x9E3779B9 / 0xBB67AE85; the key is bumped before every round but the first.
* A 64-bit word u = (out1 << 32) | out0 of one Philox block.
* uniform_open(u)  = (2*(u >> 12) + 1) * 2^-53, exactly, in (0, 1).
* uniform_closed0(u) = (u >> 11) * 2^-53, exactly, in [0, 1).
* ln(U) built only from IEEE-754 basic operations (no fused multiply-add):
  U = m * 2^e with m in [1, 2) by bit extraction; if m > sqrt(2) then m /= 2,
  e += 1; t = (m - 1)/(m + 1); p = Horner of sum_{n=0..11} t^(2n)/(2n+1) in
  t^2 with coefficients 1.0/(2n+1); ln m = (2t)*p; ln U = e*LN2 + ln m.

Every operation below is a single correctly rounded NumPy float64 operation,
so the result is fixed bit for bit by the definition.
"""

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)

# Stream tags (bits 24..31 of counter word 2); bits 20..23 carry the mode and
# bits 0..19 the repetition.
TAG_SAMPLE = 1
TAG_ALSINIT = 2
TAG_INIT = 3
TAG_GETRANK = 4


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 block function, vectorised over NumPy arrays.

    All arguments hold 32-bit values (any integer dtype, broadcastable).
    Returns the four 32-bit output words as uint64 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        # 32x32 -> 64-bit products are exact in uint64.
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def key_words(seed, tensor_id):
    """Philox key (k0, k1) for a 64-bit seed and a 32-bit tensor id."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, ((seed >> 32) ^ int(tensor_id)) & 0xFFFFFFFF


def make_tag(stream, mode, rep):
    return ((int(stream) & 0xFF) << 24) | ((int(mode) & 0xF) << 20) | (int(rep) & 0xFFFFF)


def bits64(seed, tensor_id, c0, c1, tag, t):
    """64-bit word (out1 << 32) | out0 for counter (c0, c1, tag, t)."""
    k0, k1 = key_words(seed, tensor_id)
    o0, o1, _, _ = philox4x32_10(c0, c1, tag, t, k0, k1)
    return (o1 << np.uint64(32)) | o0


def uniform_open(u):
    """(2*(u>>12)+1) * 2^-53: an exact double strictly inside (0, 1)."""
    m = (np.asarray(u, dtype=np.uint64) >> np.uint64(12)) * np.uint64(2) + np.uint64(1)
    return m.astype(np.float64) * (2.0 ** -53)


def uniform_closed0(u):
    """(u>>11) * 2^-53: an exact double in [0, 1)."""
    m = np.asarray(u, dtype=np.uint64) >> np.uint64(11)
    return m.astype(np.float64) * (2.0 ** -53)


SQRT2 = 1.4142135623730951          # nearest double to sqrt(2)
LN2 = 0.6931471805599453            # nearest double to ln(2)
_LN_COEF = [1.0 / (2 * n + 1) for n in range(12)]


def ln_basic(U):
    """Natural logarithm of positive normal doubles from basic operations.

    Follows the definition in the module docstring operation by operation.
    """
    U = np.asarray(U, dtype=np.float64)
    b = U.view(np.uint64)
    e = ((b >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) - 1023
    m = ((b & np.uint64(0x000FFFFFFFFFFFFF)) | np.uint64(1023 << 52)).view(np.float64)
    big = m > SQRT2
    m = np.where(big, m / 2.0, m)
    e = np.where(big, e + 1, e)
    t = (m - 1.0) / (m + 1.0)
    t2 = t * t
    p = np.full_like(t, _LN_COEF[11])
    for n in range(10, -1, -1):
        p = p * t2
        p = p + _LN_COEF[n]
    lnm = (2.0 * t) * p
    return e.astype(np.float64) * LN2 + lnm


def exp_variate(u):
    """Standard exponential variate E = -ln(U) with U = uniform_open(u)."""
    return -ln_basic(uniform_open(u))
