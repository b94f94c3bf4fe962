"""Philox-4xW counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).

Oracle code (test infrastructure only).

The generator maps a 4-word counter and a 2-word key to 4 words by R rounds
of the Philox S-box: two W x W -> 2W products of counter words 0 and 2 with
fixed multipliers; the high halves are XORed with the other two counter
words and the round key, and the four words are permuted.  The key is bumped
by two Weyl constants between rounds.  One generic implementation serves both
word widths so the 64-bit instance can be checked against NumPy's own
``numpy.random.Philox`` (4x64-10) and the 32-bit instance against the
published known-answer vectors.

Shading draws one Philox4x32-10 block per (pixel, sample): counter
(q, s, frame, 0) with q = j*W + i, key (seed mod 2^32, seed >> 32), and takes
u1 = (x0 >> 8) * 2^-24, u2 = (x1 >> 8) * 2^-24.  Both are multiples of 2^-24
in [0, 1), exactly representable in float32 and float64.
"""

import numpy as np

_PARAMS = {
    32: dict(m=(0xD2511F53, 0xCD9E8D57), w=(0x9E3779B9, 0xBB67AE85)),
    64: dict(m=(0xD2E7470EE14C6C93, 0xCA5A826395121157),
             w=(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)),
}


def _int_rows(x):
    """Rows of exact Python ints (never via a float array: 64-bit words)."""
    rows = x.tolist() if isinstance(x, np.ndarray) else list(x)
    if rows and not isinstance(rows[0], (list, tuple, np.ndarray)):
        rows = [rows]
    return [[int(v) for v in row] for row in rows]


def philox(counter, key, bits=32, rounds=10):
    """Philox-4x{bits}-{rounds} of counters ``[n][4]`` under keys ``[n][2]``.

    Exact integer arithmetic on Python ints (slow; for the known-answer and
    cross-library checks).  ``philox4x32`` below is the vectorised form used
    by the shading oracle.
    """
    p = _PARAMS[bits]
    mask = (1 << bits) - 1
    c = _int_rows(counter)
    k = _int_rows(key)
    if len(k) == 1 and len(c) > 1:
        k = k * len(c)
    out = []
    for ctr, kk in zip(c, k):
        x0, x1, x2, x3 = ctr
        k0, k1 = kk
        for r in range(rounds):
            if r > 0:
                k0 = (k0 + p["w"][0]) & mask
                k1 = (k1 + p["w"][1]) & mask
            p0 = x0 * p["m"][0]
            p1 = x2 * p["m"][1]
            hi0, lo0 = p0 >> bits, p0 & mask
            hi1, lo1 = p1 >> bits, p1 & mask
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        out.append([x0, x1, x2, x3])
    dtype = np.uint32 if bits == 32 else np.uint64
    return np.array(out, dtype=dtype)


def philox4x32(counter, key):
    """Vectorised Philox4x32-10: uint32 ``counter[n][4]``, ``key[n][2]`` or ``[2]``."""
    c = np.asarray(counter, np.uint64).reshape(-1, 4)
    k = np.broadcast_to(np.asarray(key, np.uint64).reshape(-1, 2), (c.shape[0], 2))
    mask = np.uint64(0xFFFFFFFF)
    m0, m1 = (np.uint64(v) for v in _PARAMS[32]["m"])
    w0, w1 = (np.uint64(v) for v in _PARAMS[32]["w"])
    x0, x1, x2, x3 = c[:, 0].copy(), c[:, 1].copy(), c[:, 2].copy(), c[:, 3].copy()
    k0, k1 = k[:, 0].copy(), k[:, 1].copy()
    s32 = np.uint64(32)
    for r in range(10):
        if r > 0:
            k0 = (k0 + w0) & mask
            k1 = (k1 + w1) & mask
        p0 = x0 * m0  # < 2^64: exact in uint64
        p1 = x2 * m1
        hi0, lo0 = p0 >> s32, p0 & mask
        hi1, lo1 = p1 >> s32, p1 & mask
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=1).astype(np.uint32)


def sample_uniforms(q, s, frame, seed):
    """(u1, u2) in [0,1) for pixel indices ``q`` and sample indices ``s``."""
    q = np.asarray(q, np.uint64)
    s = np.broadcast_to(np.asarray(s, np.uint64), q.shape)
    ctr = np.stack([q, s, np.full_like(q, frame), np.zeros_like(q)], axis=1)
    seed = int(seed)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], np.uint64)
    x = philox4x32(ctr, key).astype(np.uint64)
    scale = 2.0 ** -24
    return (x[:, 0] >> np.uint64(8)).astype(np.float64) * scale, \
        (x[:, 1] >> np.uint64(8)).astype(np.float64) * scale
