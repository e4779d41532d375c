"""Tile orders of the symmetric kernels (host models of their index arithmetic).

The contraction and the Cov refresh both walk the upper-triangle tile pairs (I <= J)
in bands of 8 tile-rows, column by column.  The contraction gives XCD w % 8 a
contiguous run of that order; the refresh gives XCD x the 8 tiles of column block
8a + x in every run of 64 workgroups.  This replays both mappings and checks that
they are bijections onto the pairs."""
import pytest


def band_order(w, T, ntiles, G=8):
    x, r = w % 8, w // 8
    base, rem = ntiles // 8, ntiles % 8
    t = x * base + min(x, rem) + r
    i0 = 0
    while True:
        h = min(T - i0, G)
        cnt = h * (h + 1) // 2 + h * (T - i0 - h)
        if t < cnt or i0 + h >= T:
            break
        t -= cnt
        i0 += G
    h = min(T - i0, G)
    tri = h * (h + 1) // 2
    if t < tri:
        jj = 0
        while t >= jj + 1:
            t -= jj + 1
            jj += 1
        return i0 + t, i0 + jj
    t -= tri
    return i0 + t % h, i0 + h + t // h


@pytest.mark.parametrize("T", [1, 2, 7, 8, 9, 15, 16, 17, 33, 79, 100, 257])
def test_band_order_is_a_bijection_onto_upper_pairs(T):
    n = T * (T + 1) // 2
    got = sorted(band_order(w, T, n) for w in range(n))
    assert got == sorted((i, j) for i in range(T) for j in range(i, T))


def test_band_order_runs_a_column_block_together():
    """Within a band, the G tiles of one column block are consecutive in the order."""
    T, n = 40, 40 * 41 // 2
    order = [None] * n
    for w in range(n):
        x, r = w % 8, w // 8
        base, rem = n // 8, n % 8
        order[x * base + min(x, rem) + r] = band_order(w, T, n)
    # past the band's triangle, positions come in runs of 8 with one J
    i0_band = [p for p in order if p[0] < 8]
    tail = [p for p in i0_band if p[1] >= 8]
    for k in range(0, len(tail), 8):
        assert len({p[1] for p in tail[k:k + 8]}) == 1


def refresh_order(w, T, ntiles):
    t = w
    if w < ntiles // 64 * 64:
        a, b, x = w >> 6, (w >> 3) & 7, w & 7
        t = 64 * a + 8 * x + b
    # the band walk of band_order without its XCD remap
    i0 = 0
    while True:
        h = min(T - i0, 8)
        cnt = h * (h + 1) // 2 + h * (T - i0 - h)
        if t < cnt or i0 + h >= T:
            break
        t -= cnt
        i0 += 8
    h = min(T - i0, 8)
    tri = h * (h + 1) // 2
    if t < tri:
        jj = 0
        while t >= jj + 1:
            t -= jj + 1
            jj += 1
        return i0 + t, i0 + jj
    t -= tri
    return i0 + t % h, i0 + h + t // h


@pytest.mark.parametrize("T", [1, 2, 7, 8, 9, 15, 16, 17, 33, 79, 100, 257, 1427])
def test_refresh_order_is_a_bijection_onto_upper_pairs(T):
    n = T * (T + 1) // 2
    got = sorted(refresh_order(w, T, n) for w in range(n))
    assert got == sorted((i, j) for i in range(T) for j in range(i, T))


def refresh_order_closed(w, T, ntiles):
    """The refresh's closed-form mapping (square roots instead of the band walk)."""
    import math
    t = w
    if w < ntiles // 64 * 64:
        a, b, x = w >> 6, (w >> 3) & 7, w & 7
        t = 64 * a + 8 * x + b
    G = 8
    nfull, c1 = T // G, G * (G + 1) // 2 + G * (T - G)

    def P(b):
        return b * c1 - G * G * b * (b - 1) // 2
    q = c1 + 0.5 * G * G
    disc = q * q - 2.0 * G * G * t
    b = int((q - math.sqrt(max(disc, 0.0))) / (G * G))
    b = max(0, min(nfull, b))
    while b > 0 and P(b) > t:
        b -= 1
    while b < nfull and P(b + 1) <= t:
        b += 1
    t -= P(b)
    i0 = b * G
    h = min(G, T - i0)
    tri = h * (h + 1) // 2
    if t < tri:
        jj = int((math.sqrt(8.0 * t + 1.0) - 1.0) * 0.5)
        while jj > 0 and jj * (jj + 1) // 2 > t:
            jj -= 1
        while (jj + 1) * (jj + 2) // 2 <= t:
            jj += 1
        return i0 + t - jj * (jj + 1) // 2, i0 + jj
    t -= tri
    return i0 + t % h, i0 + h + t // h


@pytest.mark.parametrize("T", [1, 2, 7, 8, 9, 15, 16, 17, 33, 64, 65, 79, 100, 257, 1427])
def test_refresh_closed_form_equals_band_walk(T):
    n = T * (T + 1) // 2
    step = max(1, n // 20000)
    for w in list(range(0, n, step)) + [n - 1]:
        assert refresh_order_closed(w, T, n) == refresh_order(w, T, n), (T, w)
