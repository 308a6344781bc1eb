"""Seeded synthetic point sets for the kNN / friends-of-friends workloads.

This module holds input generation only: it contains none of the method's
arithmetic, and both the GPU library's tests and the CPU oracle's tests draw
their inputs from here.

The paper benchmarks on uniform random points in the unit cube (kNN comparison
and scaling sections) and on cosmological simulation snapshots (kNN across
domains, FoF performance section). The snapshots are not available, so a
clustered stand-in is used: Gaussian clumps (halo-like) on a uniform background
(field-like). The linking length follows the paper's Eq. 18,
``R_link = alpha * (V / N)**(1/3)`` with ``V = 1`` for the unit box.

All generation runs in float64 with numpy's ``default_rng`` and is cast to
float32 at the end; a coordinate that rounds up to 1.0f is replaced by 0.0f so
that every coordinate lies in [0, 1).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "uniform",
    "clustered",
    "clump_params",
    "clustered_device",
    "lattice",
    "linking_length",
    "batched_sets",
    "served_requests",
]


def _to_unit_f32(x: np.ndarray) -> np.ndarray:
    out = x.astype(np.float32)
    out[out >= np.float32(1.0)] = np.float32(0.0)
    return out


def uniform(n: int, seed: int) -> np.ndarray:
    """``n`` points uniform in [0,1)^3, float32, shape (n, 3), C-contiguous."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(_to_unit_f32(rng.random((n, 3))))


def _power_law_weights(rng: np.random.Generator, c: int, slope: float,
                       wmin: float, wmax: float) -> np.ndarray:
    """Inverse-CDF draws from pdf ~ w**slope (slope < -1) truncated to [wmin, wmax]."""
    a = slope + 1.0  # negative
    u = rng.random(c)
    lo, hi = wmin ** a, wmax ** a
    return (lo + u * (hi - lo)) ** (1.0 / a)


def _apportion(total: int, weights: np.ndarray) -> np.ndarray:
    """Largest-remainder split of ``total`` in proportion to ``weights``.

    Ties among equal remainders go to the lower clump id.
    """
    share = weights / weights.sum() * total
    base = np.floor(share).astype(np.int64)
    rest = total - int(base.sum())
    if rest > 0:
        rem = share - base
        order = np.lexsort((np.arange(len(weights)), -rem))
        base[order[:rest]] += 1
    return base


def clustered(n: int, clumps: int, seed: int, *, frac_clumped: float = 0.6,
              sigma_range=(0.002, 0.02), slope: float = -1.9,
              wmax: float = 1.0e4, return_info: bool = False):
    """Clumpy point set in [0,1)^3.

    ``round(frac_clumped * n)`` points sit in ``clumps`` isotropic Gaussian
    clumps (centres uniform, sigma log-uniform in ``sigma_range``, member counts
    proportional to power-law weights of the given slope truncated to
    [1, wmax]); the rest is a uniform background. Clump members wrap
    periodically into the unit cube. A final seeded shuffle makes the input
    order non-spatial.
    """
    rng = np.random.default_rng(seed)
    n_cl = int(round(frac_clumped * n)) if clumps > 0 else 0
    clumps = max(int(clumps), 1)
    centres = rng.random((clumps, 3))
    sig = np.exp(rng.uniform(math.log(sigma_range[0]), math.log(sigma_range[1]), clumps))
    w = _power_law_weights(rng, clumps, slope, 1.0, wmax)
    counts = _apportion(n_cl, w)
    owner = np.repeat(np.arange(clumps), counts)
    pts = np.empty((n, 3), dtype=np.float64)
    if n_cl:
        pts[:n_cl] = centres[owner] + sig[owner, None] * rng.standard_normal((n_cl, 3))
        np.mod(pts[:n_cl], 1.0, out=pts[:n_cl])
    pts[n_cl:] = rng.random((n - n_cl, 3))
    perm = rng.permutation(n)
    out = np.ascontiguousarray(_to_unit_f32(pts[perm]))
    if return_info:
        return out, {"max_clump": int(counts.max()) if n_cl else 0,
                     "n_clumped": n_cl, "clumps": clumps}
    return out


def lattice(m: int, spacing_log2: int = -4, offset=(0, 0, 0)) -> np.ndarray:
    """Cubic lattice of m^3 points with spacing 2**spacing_log2 (all exact in f32).

    Point index is ``(i * m + j) * m + l`` for lattice coordinates (i, j, l);
    coordinates are ``(i + offset[0]) * 2**spacing_log2`` and so on.
    """
    a = 2.0 ** spacing_log2
    g = np.arange(m, dtype=np.float64)
    i, j, l = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([(i.ravel() + offset[0]) * a, (j.ravel() + offset[1]) * a,
                    (l.ravel() + offset[2]) * a], axis=1)
    out = pts.astype(np.float32)
    assert np.all(out.astype(np.float64) == pts), "lattice not exact in float32"
    return np.ascontiguousarray(out)


def clump_params(n: int, clumps: int, seed: int, *, frac_clumped: float = 0.6,
                 sigma_range=(0.002, 0.02), slope: float = -1.9, wmax: float = 1.0e4):
    """The per-clump parameters of :func:`clustered` for one set: (number of
    clumped points, centres [C, 3], sigmas [C], member counts [C]), drawn with
    numpy exactly as :func:`clustered` draws them."""
    rng = np.random.default_rng(seed)
    n_cl = int(round(frac_clumped * n)) if clumps > 0 else 0
    clumps = max(int(clumps), 1)
    centres = rng.random((clumps, 3))
    sig = np.exp(rng.uniform(math.log(sigma_range[0]), math.log(sigma_range[1]), clumps))
    w = _power_law_weights(rng, clumps, slope, 1.0, wmax)
    return n_cl, centres, sig, _apportion(n_cl, w)


def clustered_device(n: int, seed: int, n_cl: int, centres, sig, counts, device="cuda"):
    """The recipe of :func:`clustered`, drawn on the GPU with torch on the
    current stream, for request streams too large to pre-generate.

    ``centres`` / ``sig`` / ``counts`` are device tensors of one set's clump
    parameters (:func:`clump_params`); the member offsets and the background
    are drawn with a torch generator seeded by ``seed``, and the input order
    is a random affine permutation i -> (a i + c) mod n (a coprime to n)
    instead of a full shuffle, so the values differ from :func:`clustered`
    for the same seed while the distribution is the same. Returns a float32
    (n, 3) tensor; no call waits for the device.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    pts = torch.empty((n, 3), dtype=torch.float64, device=device)
    if n_cl:
        owner = torch.repeat_interleave(torch.arange(centres.shape[0], device=device), counts,
                                        output_size=n_cl)
        off = torch.randn((n_cl, 3), generator=g, dtype=torch.float64, device=device)
        pts[:n_cl] = torch.remainder(centres[owner] + sig[owner, None] * off, 1.0)
    if n > n_cl:
        pts[n_cl:] = torch.rand((n - n_cl, 3), generator=g, dtype=torch.float64, device=device)
    rng = np.random.default_rng(int(seed) ^ 0x5EED)
    a = int(rng.integers(1, max(2, n)))
    while math.gcd(a, n) != 1:
        a += 1
    c = int(rng.integers(0, max(1, n)))
    perm = torch.remainder(torch.arange(n, device=device, dtype=torch.int64) * a + c, n)
    out = pts[perm].to(torch.float32)
    return torch.where(out >= 1.0, torch.zeros((), dtype=out.dtype, device=device), out)


def linking_length(n: int, alpha: float = 0.2, volume: float = 1.0) -> float:
    """Eq. 18 linking length, computed in float64 and rounded once to float32."""
    return float(np.float32(alpha * (volume / n) ** (1.0 / 3.0)))


def batched_sets(num_sets: int, seed: int, log2_min: float = 10.0,
                 log2_max: float = 18.0, clumps_per_2_24: int = 4096,
                 alpha: float = 0.2, size_only: bool = False):
    """Many independent clustered sets with log-uniform sizes.

    Returns (points concatenated [sum n, 3] f32, offsets [B+1] int64,
    b [B] float32 linking lengths). Set s uses seed ``(seed, s)``.
    """
    rng = np.random.default_rng(seed)
    sizes = np.floor(2.0 ** rng.uniform(log2_min, log2_max, num_sets)).astype(np.int64)
    offsets = np.zeros(num_sets + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    b = np.array([linking_length(int(s), alpha) for s in sizes], dtype=np.float32)
    if size_only:
        return None, offsets, b
    pts = np.empty((int(offsets[-1]), 3), dtype=np.float32)
    for s in range(num_sets):
        ns = int(sizes[s])
        c = max(1, int(round(clumps_per_2_24 * ns / 2.0 ** 24)))
        pts[offsets[s]:offsets[s + 1]] = clustered(ns, c, seed=[seed, s])
    return pts, offsets, b


def served_requests(count: int, seed: int, rate_hz: float = 2000.0,
                    log2_min: float = 12.0, log2_max: float = 22.0):
    """Open-loop request schedule: Poisson arrival times and request parameters.

    Each request is a dict with ``t`` (scheduled arrival, seconds), ``op``
    ("knn" or "fof"), ``k`` (for kNN), ``alpha`` (for FoF), ``n`` and
    ``seed`` (for its point set, drawn with :func:`clustered`).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, count)
    t = np.cumsum(gaps)
    reqs = []
    for r in range(count):
        n = int(np.floor(2.0 ** rng.uniform(log2_min, log2_max)))
        op = "knn" if rng.random() < 0.5 else "fof"
        k = int(rng.choice([8, 16, 32]))
        alpha = float(rng.choice([0.1, 0.2]))
        reqs.append({"t": float(t[r]), "op": op, "k": k, "alpha": alpha,
                     "n": n, "seed": 5_000_000 + r,
                     "clumps": max(1, int(round(4096 * n / 2.0 ** 24)))})
    return reqs
