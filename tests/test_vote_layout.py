"""The vote's paired LDS counters (two r cells per 32-bit word, the pair's
sum in the low 14 bits) are exact only while no cell pair of a theta row
collects 2^14 or more votes.  The kernel takes that layout for a slice only
when every row's table entries bound their pairs below that limit
(`vote_pair_bound` in the HIP sources).  These CPU checks confirm the bound
against brute force: with every pixel an edge (the worst case), the largest
count of two neighbouring r cells never exceeds it -- for random tables,
small-coefficient tables that must be refused, and the Q14 rotation table on
the largest frames the paired layout serves.  (Sec. 2.3 Eq. 3: the
accumulator must be the plain count.)"""
import numpy as np
import pytest

PAIR_MAX = 16383


def cdiv(a, b):
    return -(-a // b)


def pair_bound(W, H, C, S):
    """Restates vote_pair_bound: runs of columns per image row times the rows
    that can meet the strip, the smaller of the two orientations."""
    ac, as_ = abs(int(C)), abs(int(S))
    ym = min(H, cdiv(32768 + (W - 1) * ac, as_)) if as_ else H
    ym *= min(W, cdiv(32768, ac)) if ac else W
    xm = min(W, cdiv(32768 + (H - 1) * as_, ac)) if ac else W
    xm *= min(H, cdiv(32768, as_)) if as_ else H
    return min(ym, xm)


def worst_pair(W, H, C, S):
    """Largest number of pixels of a full W x H frame that fall in two
    neighbouring r cells of row (C, S), over both pairings of the cells."""
    y, x = np.mgrid[0:H, 0:W]
    v = x.astype(np.int64) * int(C) + y.astype(np.int64) * int(S) + 8192
    r = np.floor_divide(v, 16384).ravel()
    r -= r.min()
    cnt = np.bincount(r)
    c2 = np.concatenate([cnt, [0]])
    return int((c2[:-1] + c2[1:]).max())


def test_bound_holds_on_random_tables():
    rng = np.random.default_rng(7)
    for _ in range(400):
        W = int(rng.integers(1, 90))
        H = int(rng.integers(1, 90))
        scale = int(rng.choice([1, 4, 64, 1024, 16384, 32767]))
        C, S = (int(v) for v in rng.integers(-scale, scale + 1, 2))
        assert worst_pair(W, H, C, S) <= pair_bound(W, H, C, S), (W, H, C, S)


@pytest.mark.parametrize("q", [1, 6, 8])
def test_small_tables_are_refused_where_they_overflow(synth, q):
    """Q8, Q6 and C = S = 1 tables on a 640 x 480 frame: the rows whose
    pairs can overflow (all of them, for a full frame) are refused."""
    W, H = 640, 480
    n = 180
    if q == 1:
        C = np.ones(n, np.int64)
        S = np.ones(n, np.int64)
    else:
        a = np.arange(n) * np.pi / n
        C = np.round(np.cos(a) * 2 ** q).astype(np.int64)
        S = np.round(np.sin(a) * 2 ** q).astype(np.int64)
    over = 0
    for k in range(0, n, 7):
        w = worst_pair(W, H, C[k], S[k])
        assert w <= pair_bound(W, H, C[k], S[k])
        over += w > PAIR_MAX
    assert over > 0


@pytest.mark.parametrize("W,H", [(640, 480), (1920, 1080), (3840, 2160), (4094, 4094), (8000, 189)])
def test_rotation_table_pairs(synth, W, H):
    """Q14 table: the bound stays at most 3 max(W, H) and above the brute-force
    worst pair; where it admits the paired layout the pairs fit in 14 bits."""
    C, S = synth.trig_q14(360)
    big = W * H > 4_000_000
    rows = [0, 45, 89, 90, 91, 135, 180, 270, 315] if big \
        else range(0, 360, 9)
    for k in rows:
        b = pair_bound(W, H, C[k], S[k])
        w = worst_pair(W, H, C[k], S[k])
        assert w <= b <= 3 * max(W, H), (k, w, b)
        if b <= PAIR_MAX:
            assert w <= PAIR_MAX
