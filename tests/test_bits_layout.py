"""Write pattern of the contraction epilogue's candidate threshold words (host model).

The direct-to-LDS contraction kernels write the bitmap as 32-bit half-words from each
256 x 256 upper-triangle tile (8 waves of 64 x 128, 32 x 32 blocks): a block (bi, bj)
writes row row0 + l's half-word at its column block and, off the diagonal block, the
mirrored row col0 + l's half-word at its row block; diagonal tiles skip the blocks
below the diagonal.  This replays that index arithmetic (with the kernel's guards) on
the host and checks that every half-word of every row is written exactly once and
nothing outside the p x 2*ceil(p/64) half-word array is touched.

The split grid of the register-A kernel (each XCD's partial last round of tiles run as
two 256 x 128 halves, 8 waves of 64 x 64) is replayed the same way, together with its
workgroup -> (tile, half) mapping."""
import pytest


def _tile_in_order(t, T):
    """Tile t of the kernel's order: bands of 8 tile-rows, column by column."""
    G, i0 = 8, 0
    while True:
        h = min(G, T - i0)
        cnt = h * (h + 1) // 2 + h * (T - i0 - h)
        if t < cnt or i0 + h >= T:
            break
        t -= cnt
        i0 += G
    h = min(G, T - i0)
    tri = h * (h + 1) // 2
    if t < tri:
        jj = 0
        while t >= jj + 1:
            t -= jj + 1
            jj += 1
        return i0 + t, i0 + jj
    t -= tri
    return i0 + t % h, i0 + h + t // h


def _split_tiles(ntiles, per_xcd):
    """Tiles per XCD that the launcher splits (those of a partial last round that fill at
    most half of it)."""
    base, rem = divmod(ntiles, 8)
    if per_xcd < 2:
        return 0
    tail = (base + (1 if rem else 0)) % per_xcd
    if tail == 0 or 2 * tail > per_xcd:
        return 0
    return min(tail, base)


def _tile_of_split(w, ntiles, T, nsplit):
    x, r = w % 8, w // 8
    base, rem = divmod(ntiles, 8)
    start = x * base + min(x, rem)
    nfull = base + (1 if x < rem else 0) - nsplit
    if r < nfull:
        return _tile_in_order(start + r, T) + (-1,)
    q = r - nfull
    return _tile_in_order(start + nfull + q // 2, T) + (q & 1,)


def _regions(T, nsplit=None):
    """(I, J, [(bi, bj) blocks of every wave]) for each workgroup of the grid."""
    ntiles = T * (T + 1) // 2
    if nsplit is None:
        for I in range(T):
            for J in range(I, T):
                yield I, J, [(wm * 2 + i, wn * 4 + j) for wm in range(4) for wn in range(2)
                             for i in range(2) for j in range(4)]
        return
    for w in range(ntiles + 8 * nsplit):
        I, J, half = _tile_of_split(w, ntiles, T, nsplit)
        if half < 0:
            blocks = [(wm * 2 + i, wn * 4 + j) for wm in range(4) for wn in range(2)
                      for i in range(2) for j in range(4)]
        else:
            blocks = [(wm * 2 + i, (half * 128 + wn * 64) // 32 + j) for wm in range(4)
                      for wn in range(2) for i in range(2) for j in range(2)]
        yield I, J, blocks


def _writes(p, nsplit=None):
    BT, nwords = 256, (p + 63) // 64
    nh = 2 * nwords
    T = (p + BT - 1) // BT
    seen = {}
    for I, J, blocks in _regions(T, nsplit):
        rowI0, rowJ0 = I * BT, J * BT
        for bi, bj in blocks:
            diag = I == J
            if diag and bj < bi:
                continue
            dblk = diag and bi == bj
            row0, col0 = rowI0 + bi * 32, rowJ0 + bj * 32
            for l in range(32):
                targets = []
                if dblk:
                    if row0 + l < p:
                        targets.append((row0 + l, col0 >> 5))
                else:
                    if row0 + l < p and (col0 >> 5) < nh:
                        targets.append((row0 + l, col0 >> 5))
                    if col0 + l < p and (row0 >> 5) < nh:
                        targets.append((col0 + l, row0 >> 5))
                for t in targets:
                    seen[t] = seen.get(t, 0) + 1
    return seen, nh


@pytest.mark.parametrize("p", [1, 31, 64, 200, 256, 333, 511, 600, 700, 1025])
def test_every_half_word_written_once_in_bounds(p):
    seen, nh = _writes(p)
    assert all(0 <= r < p and 0 <= h < nh for (r, h) in seen)
    assert all(c == 1 for c in seen.values()), [k for k, c in seen.items() if c != 1][:5]
    assert len(seen) == p * nh


@pytest.mark.parametrize("p,per_xcd", [(1800, 32), (1025, 32), (4000, 4), (3000, 4), (5000, 2), (20000, 32)])
def test_split_grid_half_words_written_once(p, per_xcd):
    T = (p + 255) // 256
    nsplit = _split_tiles(T * (T + 1) // 2, per_xcd)
    assert nsplit > 0
    seen, nh = _writes(p, nsplit)
    assert all(0 <= r < p and 0 <= h < nh for (r, h) in seen)
    assert all(c == 1 for c in seen.values())
    assert len(seen) == p * nh


@pytest.mark.parametrize("T", list(range(1, 40)) + [79, 80, 157])
@pytest.mark.parametrize("per_xcd", [2, 3, 8, 32])
def test_split_grid_covers_every_tile_once(T, per_xcd):
    """Every tile of the upper triangle is one whole-tile workgroup or two half-tile
    workgroups (halves 0 and 1), every workgroup of the ntiles + 8 nsplit grid maps to a
    tile, and on each XCD the halves come after the whole tiles."""
    ntiles = T * (T + 1) // 2
    nsplit = _split_tiles(ntiles, per_xcd)
    assert 0 <= nsplit <= ntiles // 8
    got = {}
    last_full = {}
    first_half = {}
    for w in range(ntiles + 8 * nsplit):
        I, J, half = _tile_of_split(w, ntiles, T, nsplit)
        assert 0 <= I <= J < T
        got.setdefault((I, J), []).append(half)
        x, r = w % 8, w // 8
        if half < 0:
            last_full[x] = max(last_full.get(x, -1), r)
        else:
            first_half[x] = min(first_half.get(x, 1 << 30), r)
    assert len(got) == ntiles
    for halves in got.values():
        assert sorted(halves) in ([-1], [0, 1])
    for x in first_half:
        assert last_full.get(x, -1) < first_half[x]
    # the same order as the unsplit grid's mapping
    if nsplit:
        plain = [_tile_of_split(w, ntiles, T, 0)[:2] for w in range(ntiles)]
        assert sorted(plain) == sorted(got)


def test_split_counts_at_the_headline_shape():
    # p = 20,000: 79 tile rows, 3,160 tiles, 395 per XCD = 12 rounds of 32 and 11 more
    assert _split_tiles(79 * 80 // 2, 32) == 11
    # a full last round is left alone, and so is one more than half full
    assert _split_tiles(8 * 64, 32) == 0
    assert _split_tiles(8 * (64 + 17), 32) == 0
