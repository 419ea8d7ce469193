"""Pins for the oracle's voting refinement (Section 3, Eq. 9-10): closed
forms of W(x, d) for hand-built voter layouts, the colour term from grey
levels whose Lab8 values the colour pins fix, the tie-break, the window and
dmax limits, the fallback, and exact recovery of a constant disparity."""
import math

import numpy as np

from paper_1402_2020_amd import synth


def _grey(H, W, level=120):
    return np.full((H, W, 3), level, np.uint8)


def test_closed_form_votes_uniform_colour(orc):
    H, W = 9, 9
    img = _grey(H, W)
    chk = np.full((H, W), -1, np.int32)
    # around x = (4, 4): d = 3 at (3, 4) and (5, 4) (e = 1 each);
    # d = 5 at (4, 3) (e = 1) and (5, 5) (e = sqrt 2)
    chk[4, 3] = chk[4, 5] = 3
    chk[3, 4] = 5
    chk[5, 5] = 5
    fb = np.zeros((H, W), np.int32)
    out, votes = orc.vote_refine(img, chk, fb, dmax=8, radius=2, want_votes=True)
    w3 = 2 * math.exp(-1 / 16)
    w5 = math.exp(-1 / 16) + math.exp(-math.sqrt(2) / 16)
    assert math.isclose(votes[4, 4, 3], w3, rel_tol=1e-12)
    assert math.isclose(votes[4, 4, 5], w5, rel_tol=1e-12)
    assert out[4, 4] == 3
    # valid pixels keep their disparity
    assert out[4, 3] == 3 and out[3, 4] == 5


def test_colour_term_from_grey_levels(orc):
    H, W = 5, 5
    img = _grey(H, W, 100)
    img[2, 3] = 160                               # the d = 2 voter has another grey
    chk = np.full((H, W), -1, np.int32)
    chk[2, 1] = 1                                  # same colour, e = 1
    chk[2, 3] = 2                                  # colour distance c, e = 1
    fb = np.zeros((H, W), np.int32)
    lab = orc.lab8(img).astype(float)
    c = abs(lab[2, 3, 0] - lab[2, 2, 0])           # greys: a8 = b8 = 128
    assert lab[2, 3, 1] == lab[2, 2, 1] == 128 and lab[2, 3, 2] == lab[2, 2, 2] == 128
    out, votes = orc.vote_refine(img, chk, fb, dmax=4, radius=1, want_votes=True)
    assert math.isclose(votes[2, 2, 1], math.exp(-1 / 16), rel_tol=1e-12)
    assert math.isclose(votes[2, 2, 2], math.exp(-(c / 9 + 1 / 16)), rel_tol=1e-12)
    assert out[2, 2] == 1


def test_ties_window_dmax_and_fallback(orc):
    H, W = 7, 7
    img = _grey(H, W)
    chk = np.full((H, W), -1, np.int32)
    chk[3, 2] = 6          # tie: the same geometry for d = 6 and d = 4
    chk[3, 4] = 4
    chk[0, 0] = 1          # outside radius 1 of (3, 3)
    chk[2, 3] = 9          # d >= dmax: ignored
    fb = np.full((H, W), 7, np.int32)
    out, _ = orc.vote_refine(img, chk, fb, dmax=8, radius=1)
    assert out[3, 3] == 4                                     # lowest d among equal votes
    assert out[6, 6] == 7                                     # no voter in its window
    out2, _ = orc.vote_refine(img, chk, fb, dmax=8, radius=3)
    # radius 3 reaches (0, 0) from (3, 3): d = 1 gets a vote with e = sqrt 18,
    # too small to beat the neighbours at e = 1
    assert out2[3, 3] == 4 and out2[1, 1] == 1


def test_constant_disparity_is_restored(orc):
    rng = np.random.default_rng(2)
    sc = synth.constant_shift_pair(31, 40, 20, 6)
    chk = np.full((20, 40), 6, np.int32)
    holes = rng.random((20, 40)) < 0.15
    chk[holes] = -1
    out, _ = orc.vote_refine(sc.left, chk, np.zeros((20, 40), np.int32), dmax=8, radius=4)
    assert np.all(out == 6)
