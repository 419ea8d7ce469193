"""GPU parity of right-reference matching (bsm_match_right) and the
left/right consistency check (bsm_lr_check) with the CPU oracle, bit for
bit: the two depth maps and the valid/invalid classification that open the
refinement step of Section 3."""
import sys

import numpy as np
import pytest

from paper_1402_2020_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def bsm():
    from paper_1402_2020_amd import _bsm
    _bsm.load()
    return _bsm


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _ctx(bsm, orc, n, S, use_mask=True, seed=7):
    sigma = 4.0 * S / 26
    pat = orc.make_pattern(seed, n, S, sigma)
    return bsm.Context(n, S, sigma, pattern=pat, use_mask=use_mask), pat


CASES = [  # W, H, n, S, dmax, use_mask, volume
    (37, 23, 64, 7, 11, True, True),
    (128, 96, 256, 15, 16, True, True),
    (70, 41, 256, 26, 70, True, True),     # even window (the paper's S), dmax = W
    (53, 19, 192, 11, 20, True, True),     # n outside the fast cost kernels
    (99, 30, 1024, 31, 40, True, False),
    (64, 33, 512, 15, 25, False, True),    # Eq. 4, no mask
]


@pytest.mark.parametrize("W,H,n,S,dmax,use_mask,vol", CASES)
def test_match_right_equals_oracle(torch_cuda, bsm, orc, W, H, n, S, dmax, use_mask, vol):
    torch = torch_cuda
    _say(f"case: match_right W={W} H={H} n={n} S={S} dmax={dmax} mask={use_mask} vol={vol}")
    L = synth.random_image(W + 3 * n, W, H)
    R = synth.random_image(W + 5 * n, W, H)
    ctx, pat = _ctx(bsm, orc, n, S, use_mask)
    disp, cost = ctx.match_right(_dev(torch, L), _dev(torch, R), dmax, want_cost=vol)
    torch.cuda.synchronize()
    wd, wc = orc.match_right(L, R, pat, dmax, use_mask=use_mask, want_cost=vol)
    assert np.array_equal(disp.cpu().numpy(), wd)
    if vol:
        assert np.array_equal(cost.cpu().numpy(), wc)
    ctx.close()


def test_match_right_slanted_450x375_with_volume(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: match_right 450x375 slanted planes, n=1024, dmax=60, volume")
    sc = synth.config_scene(1)
    ctx, pat = _ctx(bsm, orc, 1024, 31, seed=synth.PATTERN_SEED)
    disp, cost = ctx.match_right(_dev(torch, sc.left), _dev(torch, sc.right), 60, want_cost=True)
    torch.cuda.synchronize()
    orc.set_threads(16)
    try:
        wd, wc = orc.match_right(sc.left, sc.right, pat, 60, want_cost=True)
    finally:
        orc.set_threads(1)
    assert np.array_equal(disp.cpu().numpy(), wd)
    assert np.array_equal(cost.cpu().numpy(), wc)
    ctx.close()


def test_lr_check_equals_oracle_on_matched_maps(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: lr_check on the two maps of the 128x96 rectangles scene")
    sc = synth.config_scene(0)
    ctx, pat = _ctx(bsm, orc, 256, 15, seed=synth.PATTERN_SEED)
    L, R = _dev(torch, sc.left), _dev(torch, sc.right)
    dl, _ = ctx.match(L, R, 16)
    dr, _ = ctx.match_right(L, R, 16)
    chk = ctx.lr_check(dl, dr, tol=1)
    torch.cuda.synchronize()
    want = orc.lr_check(dl.cpu().numpy(), dr.cpu().numpy(), tol=1)
    assert np.array_equal(chk.cpu().numpy(), want)
    # the oracle's own maps give the same classification
    odl, _ = orc.match(sc.left, sc.right, pat, 16)
    odr, _ = orc.match_right(sc.left, sc.right, pat, 16)
    assert np.array_equal(want, orc.lr_check(odl, odr, tol=1))
    valid = (want >= 0).mean()
    _say(f"valid fraction {valid:.3f}")
    assert 0.5 < valid < 1.0
    ctx.close()


@pytest.mark.parametrize("tol", [0, 1, 3])
def test_lr_check_random_maps_and_in_place(torch_cuda, bsm, orc, tol):
    torch = torch_cuda
    _say(f"case: lr_check random maps tol={tol}")
    rng = np.random.default_rng(tol)
    H, W = 17, 301
    dL = rng.integers(-1, 12, (H, W)).astype(np.int32)
    dR = rng.integers(-1, 12, (H, W)).astype(np.int32)
    ctx, _ = _ctx(bsm, orc, 64, 7)
    want = orc.lr_check(dL, dR, tol=tol)
    out = ctx.lr_check(_dev(torch, dL), _dev(torch, dR), tol=tol)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    dLd = _dev(torch, dL)
    ctx.lr_check(dLd, _dev(torch, dR), tol=tol, out=dLd)     # in place
    torch.cuda.synchronize()
    assert np.array_equal(dLd.cpu().numpy(), want)
    ctx.close()


def test_right_lr_validation(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: match_right / lr_check argument validation")
    ctx, _ = _ctx(bsm, orc, 64, 7)
    img = _dev(torch, np.zeros((10, 12, 3), np.uint8))
    with pytest.raises(bsm.BsmError) as e:
        ctx.match_right(img, img, 13)                          # dmax > W
    assert e.value.status == bsm.EINVAL
    d = torch.zeros((10, 12), dtype=torch.int32, device="cuda")
    with pytest.raises(bsm.BsmError) as e:
        ctx.lr_check(d, d, tol=1, out=d)                       # out aliases disp_right
    assert e.value.status == bsm.EINVAL
    with pytest.raises(bsm.BsmError) as e:
        ctx.lr_check(d, d.clone(), tol=-1)
    assert e.value.status == bsm.EINVAL
    ctx.close()
