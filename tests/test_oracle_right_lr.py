"""Pins for the oracle's right-reference matching and left/right check (the
two depth maps and their consistency test that open the refinement step of
Section 3).

The right-reference matcher is written from its own definition (right view
as reference, partner (u + d, v) in the left view, the right view's mask);
it is pinned to the independently pinned left-reference matcher through the
mirror identity, to brute force on tiny images and to exact recovery of a
constant disparity.  The check is pinned to scene geometry: on layered
fronto-parallel scenes it must reject exactly the left pixels whose partner
shows another surface (the occlusion band left of a nearer surface, the
left border), which a wrong partner column such as u + d cannot reproduce.
"""
import numpy as np
import pytest

from paper_1402_2020_amd import synth


def _mirror(pattern):
    """Pattern of the horizontally mirrored image: x offsets change sign."""
    m = pattern.astype(np.int16).copy()
    m[:, 0] = -m[:, 0]
    m[:, 2] = -m[:, 2]
    return m.astype(np.int8)


def _flip(img):
    return np.ascontiguousarray(img[:, ::-1])


@pytest.mark.parametrize("W,H,n,S,dmax,use_mask", [(23, 9, 64, 5, 7, True), (40, 12, 256, 9, 12, True),
                                                   (31, 10, 128, 7, 31, False)])
def test_right_reference_is_the_mirrored_left_reference(orc, W, H, n, S, dmax, use_mask):
    # Right-reference matching of (L, R) with pattern P is left-reference
    # matching of (flip R, flip L) with the mirrored pattern, flipped back:
    # x_d = (u + d, v) becomes (u' - d, v) and border clamping mirrors too.
    L = synth.random_image(W * 7 + n, W, H)
    R = synth.random_image(W * 11 + n, W, H)
    pat = orc.make_pattern(n + S, n, S, S / 3.0)
    dr, cr = orc.match_right(L, R, pat, dmax, use_mask=use_mask, want_cost=True)
    dl, cl = orc.match(_flip(R), _flip(L), _mirror(pat), dmax, use_mask=use_mask, want_cost=True)
    assert np.array_equal(dr, dl[:, ::-1])
    assert np.array_equal(cr, cl[:, :, ::-1])


def test_right_reference_cost_brute_force(orc):
    W, H, n, S, dmax = 14, 6, 128, 5, 9
    L = synth.random_image(5, W, H)
    R = synth.random_image(6, W, H)
    pat = orc.make_pattern(77, n, S, 1.5)
    dL = orc.describe(L, pat)
    dR = orc.describe(R, pat)
    mR, _ = orc.mask(R, pat)
    disp, cost = orc.match_right(L, R, pat, dmax, want_cost=True)
    for v in range(H):
        for u in range(W):
            best = None
            for d in range(dmax):
                if u + d > W - 1:
                    want = 32767
                else:
                    x = 0
                    for j in range(n // 64):
                        x += bin((int(dR[v, u, j]) ^ int(dL[v, u + d, j])) & int(mR[v, u, j])).count("1")
                    want = x
                assert cost[d, v, u] == want, (u, v, d)
                if best is None or want < best[0]:
                    best = (want, d)
            assert disp[v, u] == best[1]


@pytest.mark.parametrize("d0,n,S", [(5, 256, 15), (3, 64, 7)])
def test_right_reference_constant_disparity(orc, d0, n, S):
    # right(u) = left(u + d0): right pixel u sees left pixel u + d0
    sc = synth.constant_shift_pair(90 + d0, 64, 24, d0)
    pat = orc.make_pattern(3, n, S, S / 3.0)
    disp, cost = orc.match_right(sc.left, sc.right, pat, d0 + 3, want_cost=True)
    r = S // 2
    inner = disp[r:24 - r, r:64 - 1 - d0 - r]
    assert np.all(cost[d0, r:24 - r, r:64 - 1 - d0 - r] == 0)
    assert np.mean(inner == d0) > 0.9


def test_lr_check_definition(orc):
    rng = np.random.default_rng(4)
    H, W = 7, 30
    dL = np.minimum(rng.integers(0, 6, (H, W)), np.arange(W)[None, :]).astype(np.int32)
    dR = rng.integers(0, 6, (H, W)).astype(np.int32)
    got = orc.lr_check(dL, dR, tol=1)
    for v in range(H):
        for u in range(W):
            d = dL[v, u]
            ok = u - d >= 0 and abs(d - dR[v, u - d]) <= 1
            assert got[v, u] == (d if ok else -1)
    assert np.array_equal(orc.lr_check(dL, dR, tol=100), dL)


def test_lr_check_of_consistent_maps(orc):
    # the two maps of a constant-disparity pair agree wherever both see the
    # textured overlap
    d0, n, S = 4, 256, 11
    sc = synth.constant_shift_pair(21, 48, 20, d0)
    pat = orc.make_pattern(9, n, S, S / 3.0)
    dl, _ = orc.match(sc.left, sc.right, pat, d0 + 3)
    dr, _ = orc.match_right(sc.left, sc.right, pat, d0 + 3)
    chk = orc.lr_check(dl, dr)
    r = S // 2
    inner = chk[r:20 - r, d0 + r:48 - r]
    assert np.mean(inner == d0) > 0.9
    assert np.all((chk == -1) | (chk == dl))


def _render_layers(W, H, layers):
    """Ground truth of a scene of fronto-parallel layers (x0, y0, w, h, d),
    given in left-view coordinates on a canvas wider than the image; a nearer
    layer (larger d) hides a farther one.  Returns the integer disparity maps
    of both views and the layer each pixel shows.  The right pixel ur shows
    the left position ur + d of a layer (Section 3: x_d = (u - d, v))."""
    dl = np.zeros((H, W), np.int32)
    dr = np.zeros((H, W), np.int32)
    sl = np.full((H, W), -1)
    sr = np.full((H, W), -1)
    for k, (x0, y0, w, h, d) in enumerate(layers):
        for v in range(max(0, y0), min(H, y0 + h)):
            for u in range(W):
                if x0 <= u < x0 + w and (sl[v, u] < 0 or d > dl[v, u]):
                    dl[v, u], sl[v, u] = d, k
                if x0 <= u + d < x0 + w and (sr[v, u] < 0 or d > dr[v, u]):
                    dr[v, u], sr[v, u] = d, k
    return dl, dr, sl, sr


def _occluded(dl, sl, sr):
    """Left pixels whose partner (u - d, v) lies outside the right view or
    shows another surface: what the left/right check must reject."""
    H, W = dl.shape
    occ = np.zeros((H, W), bool)
    for v in range(H):
        for u in range(W):
            ur = u - dl[v, u]
            occ[v, u] = ur < 0 or sr[v, ur] != sl[v, u]
    return occ


def test_lr_check_rejects_exactly_the_occlusion_band(orc):
    # A background at d = 3 and a full-height foreground strip at d = 9 over
    # left columns [30, 45): the background is hidden in the right view for
    # the 9 - 3 = 6 columns just left of the strip, [24, 30), and the left
    # border columns u < 3 have no partner.  Nothing else may be rejected.
    W, H = 64, 5
    dl, dr, sl, sr = _render_layers(W, H, [(0, 0, 200, H, 3), (30, 0, 15, H, 9)])
    want_invalid = np.zeros((H, W), bool)
    want_invalid[:, :3] = True
    want_invalid[:, 24:30] = True
    assert np.array_equal(_occluded(dl, sl, sr), want_invalid)   # the geometry itself
    for tol in (0, 1, 5):
        chk = orc.lr_check(dl, dr, tol=tol)
        assert np.array_equal(chk < 0, want_invalid), tol
        assert np.array_equal(chk[~want_invalid], dl[~want_invalid])


def test_lr_check_rejects_exactly_the_occluded_pixels_of_the_rectangle_scene(orc):
    # The layers of the 128x96 rectangle workload (distinct integer
    # disparities, at least 1 apart): with tol = 0 the check keeps a left
    # pixel exactly when its partner shows the same surface.
    sc = synth.rect_scene(14022020, 128, 96, 16)
    dl, dr, sl, sr = _render_layers(128, 96, sc.meta["layers"])
    assert np.array_equal(dl, sc.gt.astype(np.int32))
    occ = _occluded(dl, sl, sr)
    assert 0 < occ.sum() < occ.size // 4
    chk = orc.lr_check(dl, dr, tol=0)
    assert np.array_equal(chk < 0, occ)
    assert np.array_equal(chk[~occ], dl[~occ])
