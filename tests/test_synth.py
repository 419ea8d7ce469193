"""CPU checks of the seeded input generators that the radiometric sweep
relies on: the radiometric change and the non-occlusion mask derived from
the generator's two ground-truth maps."""
import numpy as np

from paper_1402_2020_amd import synth


def test_radiometric_identity_saturation_and_offsets():
    img = synth.random_image(3, 40, 30)
    assert np.array_equal(synth.radiometric(img), img)
    doubled = synth.radiometric(img, gain=2.0).astype(int)
    assert np.all(doubled[img >= 128] == 255)
    assert np.all(np.abs(doubled[img < 127] - 2 * img[img < 127].astype(int)) <= 1)
    off = synth.radiometric(img, offset=(-300, 0, 300)).astype(int)
    assert np.all(off[..., 0] == 0) and np.all(off[..., 2] == 255)
    assert np.array_equal(off[..., 1], img[..., 1])


def test_non_occluded_mask_of_slanted_scene():
    sc = synth.slanted_scene(5, 160, 60, 24)
    m = synth.non_occluded(sc)
    assert m.shape == sc.gt.shape and 0.6 < m.mean() < 1.0
    # a left pixel whose partner falls left of the image is never visible
    u = np.arange(sc.gt.shape[1])[None, :]
    assert not np.any(m & (np.rint(u - sc.gt) < 0))
    # outputs of the generator are unchanged by the added ground truth
    again = synth.slanted_scene(5, 160, 60, 24)
    assert np.array_equal(again.left, sc.left) and np.array_equal(again.right, sc.right)
