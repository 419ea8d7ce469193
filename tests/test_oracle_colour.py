"""Pins for the oracle's colour steps: the intensity I(x) of Eq. 3 and the
CIELAB values used by the SAD of Eq. 5 (8-bit L8 = L*255/100, a8 = a+128,
b8 = b+128, sRGB with the D65 white).

The integer conversion is pinned to (a) exact special cases, (b) published
CIELAB values of sRGB colours, and (c) a double-precision CIE 1976 L*a*b*
computed in this test from a matrix derived independently from the sRGB
primaries' chromaticities, over all 2^24 colours.
"""
import os

import numpy as np
import pytest

from paper_1402_2020_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lab_reference_colours.txt")


@pytest.fixture(scope="module")
def all_colours():
    return synth.all_colours_image()


def test_luma_grey_identity(orc):
    img = synth.grey_image(np.arange(256, dtype=np.uint8).reshape(16, 16))
    assert np.array_equal(orc.luma(img), np.arange(256, dtype=np.uint8).reshape(16, 16))


def test_luma_close_to_bt601_all_colours(orc, all_colours):
    I = orc.luma(all_colours).astype(np.float64).ravel()
    rgb = all_colours.reshape(-1, 3).astype(np.float64)
    ref = 0.299 * rgb[:, 0] + 0.587 * rgb[:, 1] + 0.114 * rgb[:, 2]
    assert np.abs(I - ref).max() <= 1.0


def test_lab8_special_cases(orc):
    img = np.array([[[0, 0, 0], [255, 255, 255]]], np.uint8)
    lab = orc.lab8(img)
    assert lab[0, 0].tolist() == [0, 128, 128]
    assert lab[0, 1].tolist() == [255, 128, 128]
    greys = orc.lab8(synth.grey_image(np.arange(256, dtype=np.uint8).reshape(1, 256)))
    assert np.all(greys[..., 1] == 128) and np.all(greys[..., 2] == 128)
    # lightness is strictly increasing along the grey axis except where the
    # 8-bit quantisation of L collapses neighbours
    assert np.all(np.diff(greys[0, :, 0].astype(int)) >= 0)


def test_lab8_tables_shape(orc):
    lin, mq, f = orc.lab8_tables()
    assert lin[0] == 0 and lin[255] == 65535
    assert np.all(np.diff(lin.astype(int)) > 0)
    assert np.all(mq.sum(axis=1) == 16384)
    assert np.all(np.diff(f.astype(int)) >= 0) and f[65535] == 65535


def test_lab8_published_colours(orc):
    rows = [list(map(float, ln.split())) for ln in open(GOLDEN)
            if ln.strip() and not ln.startswith("#")]
    img = np.array([[r[:3] for r in rows]], np.uint8)
    lab = orc.lab8(img)[0].astype(float)
    ref = np.array([[r[3] * 2.55, r[4] + 128, r[5] + 128] for r in rows])
    assert np.abs(lab - ref).max() <= 1.0, (lab, ref)


def _textbook_lab8(rgb):
    """CIE 1976 L*a*b* in float64 with the sRGB->XYZ matrix derived from the
    primaries' chromaticities and the D65 white."""
    prim = [(0.64, 0.33), (0.30, 0.60), (0.15, 0.06)]
    wx, wy = 0.3127, 0.3290
    P = np.array([[x / y, 1.0, (1 - x - y) / y] for x, y in prim]).T
    white = np.array([wx / wy, 1.0, (1 - wx - wy) / wy])
    M = P * np.linalg.solve(P, white)
    u = rgb / 255.0
    lin = np.where(u <= 0.04045, u / 12.92, ((u + 0.055) / 1.055) ** 2.4)
    t = (lin @ M.T) / white
    e = 6.0 / 29.0
    f = np.where(t > e ** 3, np.cbrt(t), t / (3 * e * e) + 4.0 / 29.0)
    L = 116 * f[:, 1] - 16
    a = 500 * (f[:, 0] - f[:, 1])
    b = 200 * (f[:, 1] - f[:, 2])
    return np.stack([L * 2.55, a + 128, b + 128], axis=1)


@pytest.mark.slow
def test_lab8_close_to_textbook_all_colours(orc, all_colours):
    lab = orc.lab8(all_colours).reshape(-1, 3)
    rgb = all_colours.reshape(-1, 3)
    worst = 0.0
    for s in range(0, rgb.shape[0], 1 << 21):
        ref = np.clip(_textbook_lab8(rgb[s:s + (1 << 21)].astype(np.float64)), 0, 255)
        err = np.abs(lab[s:s + (1 << 21)].astype(np.float64) - ref)
        worst = max(worst, float(err.max()))
    # one 8-bit step of the real value: quantisation (0.5) plus the integer
    # tables and the chromaticity-derived matrix (< 0.5)
    assert worst < 1.0, worst
