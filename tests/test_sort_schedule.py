"""Host check of the compare-exchange schedule the long-list sorter uses.

The library sorts long interaction lists with a bitonic network split over
NW waves: for a step of pair distance j <= PW = M / 2 / NW, wave w handles
the pair indices [w PW, (w + 1) PW) and synchronizes with itself only. That
is correct only if those pairs touch no element outside [2 w PW, 2 (w + 1)
PW), and the whole schedule (the same index arithmetic as the kernel) must
sort. Both are checked here on the CPU for every size the sorter meets.
"""
import numpy as np
import pytest


def pair(i, j):
    a = ((i & ~(j - 1)) << 1) | (i & (j - 1))
    return a, a + j


def schedule(M):
    k = 2
    while k <= M:
        j = k >> 1
        while j > 0:
            yield k, j
            j >>= 1
        k <<= 1


@pytest.mark.parametrize("NW", [1, 4, 8])
@pytest.mark.parametrize("M", [16, 64, 512, 2048, 8192])
def test_wave_local_steps_stay_in_their_range(M, NW):
    if M < 2 * NW:
        pytest.skip("sorter pads to at least 2 NW keys")
    PW = (M >> 1) // NW
    i = np.arange(M >> 1)
    for k, j in schedule(M):
        if j > PW:
            continue
        a, b = pair(i, j)
        w = i // PW
        assert np.all(a >= 2 * w * PW) and np.all(b < 2 * (w + 1) * PW), (M, NW, k, j)


@pytest.mark.parametrize("M", [2, 16, 1024, 8192])
def test_schedule_sorts(M):
    rng = np.random.default_rng(M)
    for trial in range(3):
        s = rng.integers(0, 2 ** 63, size=M, dtype=np.uint64)
        if trial == 1:
            s[: M // 2] = s[0]  # many equal keys
        want = np.sort(s)
        i = np.arange(M >> 1)
        for k, j in schedule(M):
            a, b = pair(i, j)
            x, y = s[a].copy(), s[b].copy()
            up = (a & k) == 0
            swap = (x > y) == up
            s[a] = np.where(swap, y, x)
            s[b] = np.where(swap, x, y)
        assert np.array_equal(s, want)
