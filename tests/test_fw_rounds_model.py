"""A CPU model of the blocked Floyd-Warshall rounds of csrc/fw.hip: the tile
sets of the interior launches (parts 0-3 of k_fw_inner over pivot blocks of
one, two or four tiles, the last blocks smaller), the diagonal-block closure
by rounds over half-size blocks, and the lookahead's split of a round (with
part 1 on the build stream, or on a stream of its own beside part 2).  The
model runs the rounds on small matrices (tiles of 4) and must give plain
Floyd-Warshall; the tile sets must be in bounds, disjoint where the lookahead
overlaps them, and cover each round's interior once.  This checks the host
and index logic of the rounds; the kernels themselves are checked against
the oracle on the GPU."""
import numpy as np
import pytest

INF = 2**31 - 1


def tri_index(b, m):
    # float32 estimate, then exact correction (as the kernel does)
    fm = np.float32(2.0 * m + 1.0)
    i = int((fm - np.sqrt(np.float32(fm * fm - np.float32(8.0) * np.float32(b)))) * np.float32(0.5))
    i = max(0, min(i, m - 1))
    while i > 0 and i * (2 * m - i + 1) // 2 > b:
        i -= 1
    while i + 1 < m and (i + 1) * (2 * m - i) // 2 <= b:
        i += 1
    return i, i + (b - i * (2 * m - i + 1) // 2)


def inner_tile(pt, part, b, c0, nt, nn):
    if part == 0:
        bi, bj = tri_index(b, nt - pt)
        return bi + (pt if bi >= c0 else 0), bj + (pt if bj >= c0 else 0)
    if part == 1:
        no = nt - pt - nn
        if b < nn * no:
            x = c0 + pt + b // no
            o = b % no
            y = o + (pt + nn if o >= c0 else 0)
            return min(x, y), max(x, y)
        bi, bj = tri_index(b - nn * no, nn)
        return c0 + pt + bi, c0 + pt + bj
    if part == 2:
        bi, bj = tri_index(b, nt - pt - nn)
        return bi + (pt + nn if bi >= c0 else 0), bj + (pt + nn if bj >= c0 else 0)
    m = nt - pt
    o = b % m
    return c0 + b // m, o + (pt if o >= c0 else 0)


def tri_count(m):
    return m * (m + 1) // 2 if m > 0 else 0


def count(nt, pt, part, nn):
    if part == 0:
        return tri_count(nt - pt)
    if part == 1:
        return nn * (nt - pt - nn) + tri_count(nn)
    if part == 2:
        return tri_count(nt - pt - nn)
    return pt * (nt - pt)


def blocks(nt, ptiles):
    out, c0 = [], 0
    while c0 < nt:
        pt = ptiles
        while pt > nt - c0:
            pt //= 2
        out.append((c0, pt))
        c0 += pt
    return out


def minplus(At, B):
    return np.min(At[:, :, None] + B[:, None, :], axis=0)


def floyd_warshall(M):
    M = M.copy()
    for k in range(M.shape[0]):
        M = np.minimum(M, M[:, k:k + 1] + M[k:k + 1, :])
    return M


def launch(A, nt, T, pt, c0, part, nn):
    """One k_fw_inner launch; its tiles read only values from before it."""
    tiles = [inner_tile(pt, part, b, c0, nt, nn) for b in range(count(nt, pt, part, nn))]
    for i, j in tiles:
        assert 0 <= i < nt and 0 <= j < nt and (part == 3 or i <= j)
    assert len(set(tiles)) == len(tiles)
    old = A.copy()
    rows = slice(c0 * T, (c0 + pt) * T)
    for i, j in tiles:
        c = np.minimum(old[i * T:(i + 1) * T, j * T:(j + 1) * T],
                       minplus(old[rows, i * T:(i + 1) * T], old[rows, j * T:(j + 1) * T]))
        A[i * T:(i + 1) * T, j * T:(j + 1) * T] = c
        A[j * T:(j + 1) * T, i * T:(i + 1) * T] = c.T
    return tiles


def close(A, c0, pt, T):
    s = slice(c0 * T, (c0 + pt) * T)
    if pt == 1:
        A[s, s] = floyd_warshall(A[s, s])
    else:
        sub = A[s, s].copy()
        rounds(sub, pt, T, pt // 2, False)
        A[s, s] = sub


def norm(i, j):
    return (i, j) if i <= j else (j, i)


def check_overlap(nt, cur, nxt, t1, t2):
    """Part 2 may run at the same time as part 1 and as the side stream's
    closure and panel of the next block (tiles as unordered pairs: every
    launch writes a tile and its transpose).  Part 2 must neither read what
    they write nor write what they read or write."""
    def reads(tiles):  # own tile and the current block's panel at its columns
        return {norm(i, j) for i, j in tiles} | {norm(a, x) for i, j in tiles for a in cur
                                                 for x in (i, j)}
    r1, w1 = reads(t1), {norm(i, j) for i, j in t1}
    r2, w2 = reads(t2), {norm(i, j) for i, j in t2}
    # side: the next block's diagonal closure, then its panel (a, j), a in it
    ws = {norm(a, b) for a in nxt for b in nxt} | {norm(a, j) for a in nxt for j in range(nt)}
    rs = set(ws)
    assert not (w2 & (r1 | w1 | rs | ws))
    assert not (r2 & (w1 | ws))


def rounds(A, nt, T, ptiles, lookahead):
    blk = blocks(nt, ptiles)
    for q, (c0, pt) in enumerate(blk):
        if not lookahead or q == 0:
            close(A, c0, pt, T)
            if nt > pt:
                launch(A, nt, T, pt, c0, 3, 0)
        if nt <= pt:
            continue
        if lookahead and q + 1 < len(blk):
            n0, npt = blk[q + 1]
            if lookahead == "p1":
                # part 1 on a stream of its own: part 2 may run before it and
                # before the side stream's work, which waits for part 1 only
                t2 = launch(A, nt, T, pt, c0, 2, npt)
                t1 = launch(A, nt, T, pt, c0, 1, npt)
                close(A, n0, npt, T)
                launch(A, nt, T, npt, n0, 3, 0)
            else:
                t1 = launch(A, nt, T, pt, c0, 1, npt)
                close(A, n0, npt, T)               # side stream, beside part 2
                launch(A, nt, T, npt, n0, 3, 0)
                t2 = launch(A, nt, T, pt, c0, 2, npt)
            nxt = set(range(n0, n0 + npt))
            assert all(i not in nxt and j not in nxt for i, j in t2)
            cur = set(range(c0, c0 + pt))
            check_overlap(nt, cur, nxt, t1, t2)
            assert set(t1) | set(t2) == {(i, j) for i in range(nt) for j in range(i, nt)
                                         if i not in cur and j not in cur}
            assert not set(t1) & set(t2)
        else:
            launch(A, nt, T, pt, c0, 0, 0)


@pytest.mark.parametrize("ptiles", [1, 2, 4])
@pytest.mark.parametrize("lookahead", [False, True, "p1"])
def test_rounds_equal_floyd_warshall(ptiles, lookahead):
    rng = np.random.default_rng(ptiles * 10 + {False: 0, True: 1, "p1": 2}[lookahead])
    T = 4
    for nt in range(1, 12):
        V = nt * T
        W = rng.integers(0, 50, (V, V)).astype(np.int64)
        W = np.where(rng.random((V, V)) < 0.3, W, INF)
        W = np.minimum(W, W.T)
        np.fill_diagonal(W, 0)
        A = W.copy()
        rounds(A, nt, T, ptiles, lookahead)
        assert np.array_equal(np.minimum(A, INF), np.minimum(floyd_warshall(W), INF)), nt


@pytest.mark.parametrize("nt", [3, 5, 217, 218, 219, 300])
def test_tile_sets_in_bounds_at_full_size(nt):
    # every launch's tiles are distinct and inside the matrix (no arithmetic)
    for ptiles in (1, 2, 4):
        blk = blocks(nt, ptiles)
        assert sum(pt for _, pt in blk) == nt
        for q, (c0, pt) in enumerate(blk):
            if nt <= pt or q not in (0, 1, len(blk) // 2, len(blk) - 2, len(blk) - 1):
                continue
            nn = blk[q + 1][1] if q + 1 < len(blk) else 0
            for part in [0, 3] + ([1, 2] if nn else []):
                seen = set()
                for b in range(count(nt, pt, part, nn)):
                    i, j = inner_tile(pt, part, b, c0, nt, nn)
                    assert 0 <= i < nt and 0 <= j < nt
                    seen.add((i, j))
                assert len(seen) == count(nt, pt, part, nn)
