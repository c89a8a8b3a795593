"""Host-side checks of the site sets the fused-pair sweep (plan 300) gives its
workgroups, by brute force on small lattices.  The kernel is exact because
each set T is mapped onto itself by the shift x -> x - mu + nu (the update of
U_nu(x) reads the new U_mu only at x and x - mu + nu, Eq. (6)); these tests
restate the kernel's position -> site formulas and check that the sets
partition the sites of one parity, that each is closed under the shift, that
the kernel's shortcut for the position of x - mu + nu is right, and that the
trailing distance (`lag`) and the LDS ring/first-block lookups of the
block-by-block walk always find a first-pass result that is already there."""
import math

import pytest

SHAPES = [(4, 4, 4, 4), (2, 2, 2, 2), (8, 6, 10, 4), (2, 4, 2, 6), (12, 12, 12, 12), (6, 4, 10, 8),
          (8, 8, 6, 4), (4, 2, 6, 10), (32, 8, 6, 10)]
BLOCK = 256


def geometry(L):
    L0, L1, L2, L3 = L
    H0 = L0 // 2
    st = [1, H0, H0 * L1, H0 * L1 * L2]

    def half_of(x):
        return (x[0] >> 1) + x[1] * st[1] + x[2] * st[2] + x[3] * st[3]

    def site_of(h, p):
        r, hx = divmod(h, H0)
        r2, x1 = divmod(r, L1)
        x3, x2 = divmod(r2, L2)
        return [2 * hx + ((p + x1 + x2 + x3) & 1), x1, x2, x3]

    return H0, st, half_of, site_of


def pair_sets(L, which):
    """(n_t, n_wg, lag, orbit) as the launcher sets them (lag before the
    whole-set-in-LDS rule)."""
    L0, L1, L2, L3 = L
    H0 = L0 // 2
    if which == 0:
        return H0 * L1, L2 * L3, 2 * H0 - 1, 0
    gc = math.gcd(L2, L3)
    orbit = L2 // gc * L3
    return orbit * H0, gc * L1, H0, orbit


def position_site(L, which, j, pos, p):
    """The kernel's pair_site: half index and site of position pos of set j."""
    L0, L1, L2, L3 = L
    H0, st, half_of, site_of = geometry(L)
    if which == 0:
        h = j * H0 * L1 + pos
        return h, site_of(h, p)
    x1, o = divmod(j, math.gcd(L2, L3))
    t, h0 = divmod(pos, H0)
    x2 = (L2 - t % L2) % L2
    x3 = (o + t) % L3
    x = [2 * h0 + ((p + x1 + x2 + x3) & 1), x1, x2, x3]
    return h0 + x1 * st[1] + x2 * st[2] + x3 * st[3], x


def shifted_position(L, which, j, pos, h, x, orbit):
    """The kernel's pair_shift: position of x - mu + nu."""
    L0, L1, L2, L3 = L
    H0, st, _, _ = geometry(L)
    if which == 0:
        h1 = h - (L1 - 1) * st[1] if x[1] + 1 == L1 else h + st[1]   # + e_1
        h2 = h1 if x[0] & 1 else (h1 + H0 - 1 if x[0] == 0 else h1 - 1)  # - e_0
        return h2 - j * H0 * L1
    t = pos // H0
    return pos - t * H0 if t + 1 == orbit else pos + H0


@pytest.mark.parametrize("L", SHAPES)
@pytest.mark.parametrize("which", [0, 1])
def test_sets_partition_one_parity_and_are_shift_closed(L, which):
    mu, nu = (0, 1) if which == 0 else (2, 3)
    n_t, n_wg, lag, orbit = pair_sets(L, which)
    H0, st, half_of, site_of = geometry(L)
    half = L[0] * L[1] * L[2] * L[3] // 2
    for p in (0, 1):
        seen = set()
        for j in range(n_wg):
            pos_of = {}
            for pos in range(n_t):
                h, x = position_site(L, which, j, pos, p)
                assert sum(x) % 2 == p and half_of(x) == h and site_of(h, p) == x
                assert h not in seen
                seen.add(h)
                pos_of[h] = pos
            for h, pos in pos_of.items():
                x = site_of(h, p)
                y = list(x)
                y[mu] = (y[mu] - 1) % L[mu]
                y[nu] = (y[nu] + 1) % L[nu]
                assert half_of(y) in pos_of, "set not closed under x -> x - mu + nu"
                py = pos_of[half_of(y)]
                assert shifted_position(L, which, j, pos, h, x, orbit) == py
                # forward by at most lag, or wrapped into the first row of the set
                assert (pos <= py <= pos + lag) or py < H0
        assert len(seen) == half


@pytest.mark.parametrize("L", SHAPES + [(64, 64, 64, 64), (32, 32, 32, 32), (256, 4, 2, 2)])
@pytest.mark.parametrize("which", [0, 1])
def test_trailing_walk_finds_every_first_pass_result(L, which):
    """Block-by-block walk (sets of more than 3 * 256 sites): at step b the
    first pass has done blocks <= b, LDS holds blocks b - 1 and b in a ring and
    block 0 apart; the second pass's positions [256 b - lag, 256 (b + 1) - lag)
    must find pos and pos(x - mu + nu) there, and cover every position once."""
    n_t, _, lag, orbit = pair_sets(L, which)
    H0 = L[0] // 2
    if lag > BLOCK:
        pytest.skip("L0 > 256: the launcher rejects the plan")
    nblk = (n_t + BLOCK - 1) // BLOCK
    ring = [None, None]
    done, covered = set(), []
    for b in range(nblk + 1):
        if b < nblk:
            ring[b & 1] = b
            done.update(range(b * BLOCK, min(n_t, (b + 1) * BLOCK)))
        for lane in range(BLOCK):
            pos = b * BLOCK + lane - lag
            if not 0 <= pos < n_t:
                continue
            covered.append(pos)
            for x0par in (0, 1):
                if which == 0:
                    x1, h0 = divmod(pos, H0)
                    x0 = 2 * h0 + x0par
                    py = ((x1 + 1) % L[1]) * H0 + (((x0 - 1) % L[0]) >> 1)
                else:
                    t = pos // H0
                    py = pos - t * H0 if t + 1 == orbit else pos + H0
                for q in (pos, py):
                    assert q in done
                    blk = q // BLOCK
                    if blk == b or blk + 1 == b:
                        assert ring[blk & 1] == blk
                    else:
                        assert blk == 0
    assert sorted(covered) == list(range(n_t))
