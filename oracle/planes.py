"""Reference for the plane-based tree hierarchy (TEST INFRASTRUCTURE).

Written from the paper's section on z-order trees:

* Eq. 2 -- ``msb(a, b)`` of two floats (sign / exponent / mantissa cases),
* Eq. 3-5 -- the dimension ``k`` of largest msb and the Morton level
  ``lvl(p, q) = (msb(p_k, q_k) + 1) * d - k``,
* Eq. 7 -- one level per gap between consecutive z-sorted points, with the
  -inf / +inf sentinel points at both ends,
* the node-size rule: the smallest node holding points g-1 and g reaches, on
  each side, up to the nearest gap with a strictly greater level, and its size
  is ``n = r_b - l_b``,
* tree planes: plane 0 keeps the gaps with ``n > N_max^(0)``; plane p keeps the
  plane p-1 splits with ``n > N_max^(p)`` and stores them as indices into the
  plane p-1 split array (Eq. 8 gives ``N_max^(p) = N_max^(0) * c**p``).

Plain Python loops; meant for small inputs and for the worked example of Fig. 3.
Also holds the integer Morton-key reading used by the GPU library (keys of
21 bits per dimension, dimension 0 most significant in each bit triple) so that
tests can recompute its gap levels and planes independently.
"""
from __future__ import annotations

import math

import numpy as np

EMAX_F32 = 128  # one larger than the largest float32 exponent (Eq. 2)


def _f32_parts(x: float):
    """(sign, exponent, 24-bit fixed-point mantissa) of a float32 value.

    Mantissa bit t stands for 2**(t - 23) times 2**exponent. Subnormals and
    zero use exponent -126 without the implicit bit; infinities take exponent
    128 (one above the largest finite exponent).
    """
    u = int(np.array([x], dtype=np.float32).view(np.uint32)[0])
    sign = u >> 31
    e_bits = (u >> 23) & 0xFF
    frac = u & 0x7FFFFF
    if e_bits == 0xFF:
        return sign, 128, 1 << 23
    if e_bits == 0:
        return sign, -126, frac
    return sign, e_bits - 127, (1 << 23) | frac


def msb(a: float, b: float) -> float:
    """Eq. 2: most significant differing bit of two float32 numbers.

    Equal values have no differing bit; they get -inf (lower than any level).
    """
    sa, ea, ma = _f32_parts(a)
    sb, eb, mb = _f32_parts(b)
    if sa != sb:
        if ma == 0 and mb == 0 and ea == eb:  # +0 and -0
            return -math.inf
        return EMAX_F32
    if ea != eb:
        return max(ea, eb)
    x = ma ^ mb
    if x == 0:
        return -math.inf
    return ea + (x.bit_length() - 1 - 23)


def lvl(p, q) -> float:
    """Eq. 3-5: Morton level of the smallest node holding points p and q."""
    d = len(p)
    ms = [msb(float(p[i]), float(q[i])) for i in range(d)]
    k = max(range(d), key=lambda i: (ms[i], -i))  # first occurrence of the max
    return (ms[k] + 1) * d - k


def gap_levels(sorted_points) -> list:
    """Eq. 7: levels of the N+1 gaps of z-sorted points, with -inf/+inf sentinels."""
    pts = [list(map(float, p)) for p in sorted_points]
    d = len(pts[0]) if pts else 1
    ext = [[-math.inf] * d] + pts + [[math.inf] * d]
    return [lvl(ext[g], ext[g + 1]) for g in range(len(pts) + 1)]


def node_sizes(levels) -> list:
    """Size of the smallest node spanning each gap (nearest strictly greater gap
    on each side). The two sentinel gaps get N."""
    N = len(levels) - 1
    n = [N] * (N + 1)
    for g in range(1, N):
        l = g - 1
        while l > 0 and not (levels[l] > levels[g]):
            l -= 1
        r = g + 1
        while r < N and not (levels[r] > levels[g]):
            r += 1
        n[g] = r - l
    return n


def planes(levels, nmax) -> list:
    """Split arrays of the tree planes for thresholds ``nmax[p]``.

    Plane 0 holds gap indices (point ranges [spl_i, spl_{i+1})); plane p > 0
    holds indices into the plane p-1 split array. The sentinel gaps are always
    kept, so every plane covers all points.
    """
    n = node_sizes(levels)
    N = len(levels) - 1
    out = []
    gaps = [g for g in range(N + 1) if g in (0, N) or n[g] > nmax[0]]
    out.append(gaps)
    for p in range(1, len(nmax)):
        prev = gaps
        keep = [j for j, g in enumerate(prev) if j in (0, len(prev) - 1) or n[g] > nmax[p]]
        out.append(keep)
        gaps = [prev[j] for j in keep]
    return out


# ---------------------------------------------------------------------------
# integer Morton keys (the GPU library's reading of the z-order)

KEY_BITS_PER_DIM = 21


def quantize(points: np.ndarray, bits: int = KEY_BITS_PER_DIM) -> np.ndarray:
    """Per-dimension integer cell coordinates, computed in float32.

    ``lo`` = per-dimension minimum, ``ext`` = largest per-dimension extent,
    ``inv = fl(2**bits / ext)`` (0 if ext is 0), and
    ``q = min(2**bits - 1, trunc(fl(fl(x - lo) * inv)))``. Every step is
    monotone in x, so the keys order points consistently with their
    coordinates.
    """
    p = np.asarray(points, dtype=np.float32)
    lo = p.min(axis=0)
    hi = p.max(axis=0)
    ext = np.float32((hi - lo).max())
    inv = np.float32(np.float32(2.0 ** bits) / ext) if ext > 0 else np.float32(0)
    if not np.isfinite(inv):
        inv = np.float32(0)
    t = (p - lo) * inv
    q = np.minimum(np.floor(t).astype(np.int64), 2 ** bits - 1)
    return q


def interleave(q: np.ndarray, bits: int = KEY_BITS_PER_DIM) -> np.ndarray:
    """Morton key: bit b of dimension i goes to key bit 3*b + (2 - i)."""
    q = np.asarray(q, dtype=np.uint64)
    key = np.zeros(q.shape[0], dtype=np.uint64)
    for b in range(bits):
        for i in range(3):
            bit = (q[:, i] >> np.uint64(b)) & np.uint64(1)
            key |= bit << np.uint64(3 * b + (2 - i))
    return key


def lvl_int(p, q) -> int:
    """Eq. 5 on non-negative integer coordinates (msb = highest differing bit)."""
    d = len(p)
    ms = [(int(p[i]) ^ int(q[i])).bit_length() - 1 for i in range(d)]
    k = max(range(d), key=lambda i: (ms[i], -i))
    if ms[k] < 0:
        return -1  # identical points
    return (ms[k] + 1) * d - k


SENTINEL_LEVEL = 255


def key_gap_levels(keys_sorted) -> np.ndarray:
    """Gap levels of sorted Morton keys, extended by the sorted position.

    Reading of the paper's Eq. 7 on integer keys: the level of the gap between
    sorted positions g-1 and g is the bit length of the XOR of their keys,
    offset by 32. Equal keys would give no level (the paper leaves msb of equal
    values undefined); this reading appends the 32-bit sorted position to each
    key, so equal keys get ``bitlen((g-1) XOR g)`` in [1, 32]. Both gap ends get
    the sentinel 255, above every real level.
    """
    k = [int(x) for x in keys_sorted]
    N = len(k)
    out = np.zeros(N + 1, dtype=np.int64)
    out[0] = out[N] = SENTINEL_LEVEL
    for g in range(1, N):
        x = k[g - 1] ^ k[g]
        out[g] = 32 + x.bit_length() if x else ((g - 1) ^ g).bit_length()
    return out
