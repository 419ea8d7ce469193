"""Pins for the oracle's descriptor (Eq. 2-3), mask (Eq. 5-7), cost (Eq. 4
and Eq. 8) and winner-take-all (Eq. 1).

Each pin checks the packed oracle against something other than itself:
bit-by-bit brute force with Python integers on tiny images, numpy's own
sort / percentile / unpackbits / argmin, invariants the definitions imply,
and exact recovery of a known constant disparity.
"""
import numpy as np
import pytest

from paper_1402_2020_amd import synth


def _clamp(x, lo, hi):
    return lo if x < lo else (hi if x > hi else x)


def _brute_bits(values, pattern, u, v, cmp):
    """Bits of one pixel as a Python int: bit i-1 = cmp(pair i)."""
    H, W = values.shape[:2]
    out = 0
    for i, (px, py, qx, qy) in enumerate(pattern.astype(int)):
        p = values[_clamp(v + py, 0, H - 1), _clamp(u + px, 0, W - 1)]
        q = values[_clamp(v + qy, 0, H - 1), _clamp(u + qx, 0, W - 1)]
        if cmp(p, q, i):
            out |= 1 << i
    return out


def _as_int(words):
    return sum(int(w) << (64 * j) for j, w in enumerate(words))


CASES = [(7, 5, 64, 3, 1.0), (12, 9, 128, 5, 1.5), (24, 16, 256, 7, 2.0), (17, 11, 192, 26, 4.0)]


@pytest.mark.parametrize("W,H,n,S,sigma", CASES)
def test_descriptor_brute_force(orc, W, H, n, S, sigma):
    img = synth.random_image(W * 1000 + n, W, H)
    pat = orc.make_pattern(S * 7 + n, n, S, sigma)
    desc = orc.describe(img, pat)
    I = orc.luma(img).astype(int)
    assert desc.shape == (H, W, n // 64)
    for v in range(H):
        for u in range(W):
            want = _brute_bits(I, pat, u, v, lambda p, q, i: p > q)
            assert _as_int(desc[v, u]) == want, (u, v)


def test_descriptor_monotone_invariance(orc):
    rng = np.random.Generator(np.random.PCG64(5))
    g = rng.integers(0, 128, (20, 30)).astype(np.uint8)
    f = np.sort(rng.choice(256, 128, replace=False)).astype(np.uint8)  # strictly increasing
    pat = orc.make_pattern(3, 256, 9, 2.0)
    a = orc.describe(synth.grey_image(g), pat)
    b = orc.describe(synth.grey_image(f[g]), pat)
    assert np.array_equal(a, b)
    # a decreasing map flips every bit whose two samples differ
    c = orc.describe(synth.grey_image((255 - g).astype(np.uint8)), pat)
    assert not np.array_equal(a, c)


def test_descriptor_flat_image_is_zero(orc):
    img = np.full((10, 13, 3), 77, np.uint8)
    pat = orc.make_pattern(4, 128, 7, 2.0)
    assert not orc.describe(img, pat).any()


def test_descriptor_horizontal_ramp(orc):
    # I(u, v) = 4u on a grey ramp: bit i is [clamp(u+px) > clamp(u+qx)]
    W, H = 40, 6
    g = np.tile((4 * np.arange(W)).astype(np.uint8), (H, 1))
    pat = orc.make_pattern(11, 64, 9, 2.5).astype(int)
    desc = orc.describe(synth.grey_image(g), pat)
    for u in (0, 3, 20, W - 1):
        want = sum(1 << i for i, (px, _, qx, _) in enumerate(pat)
                   if _clamp(u + px, 0, W - 1) > _clamp(u + qx, 0, W - 1))
        assert int(desc[2, u, 0]) == want


def _brute_weights(lab, pat, u, v):
    H, W = lab.shape[:2]
    lab = lab.astype(int)
    x = lab[v, u]
    w = []
    for px, py, qx, qy in pat.astype(int):
        p = lab[_clamp(v + py, 0, H - 1), _clamp(u + px, 0, W - 1)]
        q = lab[_clamp(v + qy, 0, H - 1), _clamp(u + qx, 0, W - 1)]
        w.append(max(int(np.abs(x - p).sum()), int(np.abs(x - q).sum())))
    return np.array(w)


@pytest.mark.parametrize("W,H,n,S,sigma", CASES)
def test_mask_brute_force(orc, W, H, n, S, sigma):
    img = synth.random_image(W * 77 + n, W, H)
    pat = orc.make_pattern(S * 13 + n, n, S, sigma)
    k = n // 4
    mask, T = orc.mask(img, pat)
    lab = orc.lab8(img)
    for v in range(H):
        for u in range(W):
            w = _brute_weights(lab, pat, u, v)
            assert np.array_equal(orc.weights(img, pat, u, v), w)
            t = int(np.sort(w)[k - 1])
            # the "quarter smallest value": numpy's linear 25th percentile
            # falls between the (k-1)th and kth order statistics; integer w
            # makes the mask identical for either
            pct = np.percentile(w, 25)
            assert T[v, u] == t
            assert np.array_equal(w <= t, w <= pct)
            m = _as_int(mask[v, u])
            assert m == sum(1 << i for i in range(n) if w[i] <= t)
            assert (w < t).sum() < k <= (w <= t).sum() == bin(m).count("1")


def test_mask_rank_extremes_and_flat(orc):
    img = synth.random_image(8, 16, 12)
    pat = orc.make_pattern(8, 128, 7, 2.0)
    m1, T1 = orc.mask(img, pat, k=1)
    mn, Tn = orc.mask(img, pat, k=128)
    w = orc.weights(img, pat, 5, 4)
    assert T1[4, 5] == w.min() and Tn[4, 5] == w.max()
    assert np.all(mn == np.uint64(0xFFFFFFFFFFFFFFFF))
    flat = np.full((9, 9, 3), 200, np.uint8)
    mf, Tf = orc.mask(flat, pat)
    assert not Tf.any() and np.all(mf == np.uint64(0xFFFFFFFFFFFFFFFF))


def test_cost_without_mask_is_hamming(orc):
    rng = np.random.Generator(np.random.PCG64(1))
    H, W, nw, dmax = 5, 19, 3, 7
    dl = rng.integers(0, 2**63, (H, W, nw), dtype=np.uint64) ^ rng.integers(0, 2, (H, W, nw), dtype=np.uint64) << np.uint64(63)
    dr = rng.integers(0, 2**63, (H, W, nw), dtype=np.uint64)
    cost = orc.cost_volume(dl, None, dr, dmax)
    for d in range(dmax):
        for u in range(W):
            if u - d < 0:
                assert np.all(cost[d, :, u] == orc.INVALID_COST)
                continue
            x = np.bitwise_xor(dl[:, u], dr[:, u - d])
            ham = np.unpackbits(x.view(np.uint8), axis=-1).sum(axis=-1)
            assert np.array_equal(cost[d, :, u], ham)


def test_cost_with_mask_brute_force(orc):
    rng = np.random.Generator(np.random.PCG64(2))
    H, W, nw, dmax = 4, 13, 2, 6
    r = lambda: rng.integers(0, 2**62, (H, W, nw), dtype=np.uint64) * np.uint64(3)
    dl, dr, m = r(), r(), r()
    cost = orc.cost_volume(dl, m, dr, dmax)
    for v in range(H):
        for u in range(W):
            for d in range(dmax):
                if u - d < 0:
                    assert cost[d, v, u] == 32767
                    continue
                want = ((_as_int(dl[v, u]) ^ _as_int(dr[v, u - d])) & _as_int(m[v, u])).bit_count()
                assert cost[d, v, u] == want
                assert 0 <= cost[d, v, u] <= _as_int(m[v, u]).bit_count()


def test_wta_is_first_argmin(orc):
    rng = np.random.Generator(np.random.PCG64(3))
    cost = rng.integers(0, 6, (9, 7, 11)).astype(np.int16)   # many ties
    assert np.array_equal(orc.wta(cost), np.argmin(cost, axis=0))


def test_flat_pair_gives_zero_disparity(orc):
    img = np.full((12, 20, 3), 90, np.uint8)
    pat = orc.make_pattern(6, 64, 5, 1.5)
    disp, cost = orc.match(img, img, pat, 8, want_cost=True)
    assert not disp.any()
    assert np.all(cost[:, :, 7:] == 0)


@pytest.mark.parametrize("d0,n,S", [(5, 256, 15), (11, 128, 9), (3, 64, 7)])
def test_constant_disparity_exact_recovery(orc, d0, n, S):
    # noise-free plane at disparity d0: away from the borders the true match
    # costs exactly 0, so WTA returns d0 unless an earlier d also costs 0
    # (then the lowest-d tie-break must return the first zero)
    sc = synth.constant_shift_pair(100 + d0, 64, 40, d0)
    pat = orc.make_pattern(d0, n, S, 4.0 * S / 26)
    r = S // 2
    dmax = d0 + 6
    disp, cost = orc.match(sc.left, sc.right, pat, dmax, want_cost=True)
    region = (slice(r, 40 - r), slice(d0 + r, 64 - r))
    assert np.all(cost[d0][region] == 0)
    c = cost[(slice(None),) + region]
    first_zero = np.argmax(c == 0, axis=0)
    assert np.array_equal(disp[region], first_zero)
    unique = (c[:d0] > 0).all(axis=0)
    assert np.all(disp[region][unique] == d0)
    assert unique.mean() > 0.9


def test_match_equals_composed_steps(orc):
    sc = synth.rect_scene(7, 48, 32, 12)
    pat = orc.make_pattern(9, 128, 9, 2.0)
    disp, cost = orc.match(sc.left, sc.right, pat, 12, want_cost=True)
    dl = orc.describe(sc.left, pat)
    dr = orc.describe(sc.right, pat)
    m, _ = orc.mask(sc.left, pat)
    vol = orc.cost_volume(dl, m, dr, 12)
    assert np.array_equal(cost, vol)
    assert np.array_equal(disp, orc.wta(vol))
    d0, c0 = orc.match(sc.left, sc.right, pat, 12, use_mask=False, want_cost=True)
    assert np.array_equal(c0, orc.cost_volume(dl, None, dr, 12))


def test_threads_do_not_change_results(orc):
    sc = synth.rect_scene(8, 64, 48, 16)
    pat = orc.make_pattern(10, 256, 15, 2.3)
    orc.set_threads(1)
    a = orc.match(sc.left, sc.right, pat, 16, want_cost=True)
    orc.set_threads(4)
    b = orc.match(sc.left, sc.right, pat, 16, want_cost=True)
    orc.set_threads(1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
