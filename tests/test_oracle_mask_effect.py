"""What the mask is for (Section 3, Eq. 6-8, Fig. 1): near a depth
discontinuity a window straddles two surfaces, and plain BRIEF (Eq. 4) then
matches the colour step between them, so the nearer surface's disparity
spreads over the farther one (edge fattening).  The mask keeps only the
quarter of the pairs whose points resemble the centre pixel in Lab, which
mostly lie on the centre's own surface.

The pin is behavioural: on slanted-plane scenes whose surfaces have weak,
coarse texture and distinct colours (the situation the paper describes),
the oracle's masked matcher must make clearly fewer errors than plain BRIEF
within five pixels of a discontinuity.  A mask that selected the wrong pairs
(a flipped comparison against T, the weights of another pixel, T taken from
the wrong end of the order) loses that advantage.  Away from edges the mask
keeps only n/4 bits, so the whole-image rate is not pinned.
"""
import numpy as np
import pytest

from paper_1402_2020_amd import synth

N, S, DMAX = 512, 31, 40


def _bad_near_edges(orc, scene, pattern, use_mask):
    d = orc.match(scene.left, scene.right, pattern, DMAX, use_mask=use_mask)
    d = d[0] if isinstance(d, tuple) else d
    edge = synth.non_occluded(scene) & synth.near_discontinuity(scene)
    assert edge.sum() > 1000
    return float((np.abs(d - scene.gt) > 1.0)[edge].mean())


@pytest.mark.parametrize("seed", [14022041, 14022043])
def test_mask_halves_errors_near_discontinuities(orc, seed):
    pattern = orc.make_pattern(synth.PATTERN_SEED, N, S, 4.0 * S / 26)
    scene = synth.slanted_scene(seed, 240, 180, DMAX, n_regions=5, tinted=True,
                                tex_amp=12.0, tex_blur=2.0)
    bsm = _bad_near_edges(orc, scene, pattern, True)
    brief = _bad_near_edges(orc, scene, pattern, False)
    assert bsm < 0.7 * brief, (bsm, brief)


def test_mask_rank_n_is_plain_brief_near_edges(orc):
    """With k = n every pair passes (T is the largest weight), so the masked
    matcher is plain BRIEF exactly, edges included."""
    pattern = orc.make_pattern(synth.PATTERN_SEED, 128, 15, 4.0 * 15 / 26)
    scene = synth.slanted_scene(14022041, 96, 64, 24, n_regions=3, tinted=True,
                                tex_amp=12.0, tex_blur=2.0)
    a = orc.match(scene.left, scene.right, pattern, 24, k=128, use_mask=True)
    b = orc.match(scene.left, scene.right, pattern, 24, use_mask=False)
    a = a[0] if isinstance(a, tuple) else a
    b = b[0] if isinstance(b, tuple) else b
    np.testing.assert_array_equal(a, b)
