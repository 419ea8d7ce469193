"""GPU parity of the voting refinement (bsm_vote_refine, Eq. 9-10) with the
CPU oracle.  The votes are real numbers summed in fp32 on the GPU and in
fp64 in the oracle, so the argmax is compared as follows: valid pixels and
pixels without voters must match exactly; a refined pixel must take the
oracle's disparity, or one whose oracle vote is within 1e-4 (relative) of
the oracle's largest vote (an fp32 sum of at most 127^2 terms in (0, 1]
carries a relative error far below that).  Votes are summed in a fixed
order, so repeated runs agree bit for bit."""
import sys

import numpy as np
import pytest

from paper_1402_2020_amd import synth

pytestmark = pytest.mark.gpu
REL_TOL = 1e-4


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


def _compare(got, want, votes, checked, fallback):
    valid = checked >= 0
    assert np.array_equal(got[valid], want[valid])
    inv = ~valid
    no_voter = inv & (votes.max(axis=2) == 0)
    assert np.array_equal(got[no_voter], fallback[no_voter])
    diff = np.argwhere(got != want)
    for v, u in diff:
        assert checked[v, u] < 0, (v, u)
        w = votes[v, u]
        assert got[v, u] >= 0 and w[got[v, u]] >= (1 - REL_TOL) * w[want[v, u]], (v, u)
    return len(diff), int(inv.sum())


@pytest.mark.parametrize("cfg,radius", [(0, 7), (1, 15)])
def test_vote_refine_after_lr_check(torch_cuda, bsm, orc, cfg, radius):
    torch = torch_cuda
    p = synth.CONFIG_PARAMS[cfg]
    _say(f"case: vote_refine on config scene {cfg}, radius {radius}")
    sc = synth.config_scene(cfg)
    pat = orc.make_pattern(synth.PATTERN_SEED, p["n"], p["S"], p["sigma"])
    ctx = bsm.Context(p["n"], p["S"], p["sigma"], pattern=pat)
    L, R = _dev(torch, sc.left), _dev(torch, sc.right)
    dl, _ = ctx.match(L, R, p["dmax"])
    dr, _ = ctx.match_right(L, R, p["dmax"])
    chk = ctx.lr_check(dl, dr, tol=1)
    ref = ctx.vote_refine(L, chk, dl, p["dmax"], radius=radius)
    torch.cuda.synchronize()
    chk_h, dl_h = chk.cpu().numpy(), dl.cpu().numpy()
    want, votes = orc.vote_refine(sc.left, chk_h, dl_h, p["dmax"], radius, want_votes=True)
    ties, invalid = _compare(ref.cpu().numpy(), want, votes, chk_h, dl_h)
    _say(f"invalid {invalid}, argmax near-ties resolved differently: {ties}")
    assert invalid > 0 and ties <= max(1, invalid // 100)
    ctx.close()


def test_vote_refine_random_maps(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: vote_refine random image and maps, 40% invalid")
    rng = np.random.default_rng(5)
    H, W, dmax = 29, 71, 9
    img = synth.random_image(17, W, H)
    chk = rng.integers(0, dmax + 2, (H, W)).astype(np.int32)   # some d >= dmax: not voters
    chk[rng.random((H, W)) < 0.4] = -1
    fb = rng.integers(0, dmax, (H, W)).astype(np.int32)
    ctx = bsm.Context(64, 7, 2.0, pattern=orc.make_pattern(1, 64, 7, 2.0))
    for radius in (0, 1, 3):
        got = ctx.vote_refine(_dev(torch, img), _dev(torch, chk), _dev(torch, fb), dmax,
                              radius=radius)
        torch.cuda.synchronize()
        want, votes = orc.vote_refine(img, chk, fb, dmax, radius, want_votes=True)
        _compare(got.cpu().numpy(), want, votes, chk, fb)
    ctx.close()


def test_vote_refine_validation(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: vote_refine argument validation")
    ctx = bsm.Context(64, 7, 2.0, pattern=orc.make_pattern(1, 64, 7, 2.0))
    img = _dev(torch, np.zeros((8, 9, 3), np.uint8))
    d = torch.zeros((8, 9), dtype=torch.int32, device="cuda")
    for kw in (dict(dmax=4097), dict(dmax=4, radius=64), dict(dmax=4, lambda_c=0.0)):
        with pytest.raises(bsm.BsmError) as e:
            ctx.vote_refine(img, d, d.clone(), **kw)
        assert e.value.status == bsm.EINVAL
    with pytest.raises(bsm.BsmError) as e:
        ctx.vote_refine(img, d, d.clone(), 4, out=d)        # out aliases checked
    assert e.value.status == bsm.EINVAL
    ctx.close()


def test_vote_refine_is_deterministic(torch_cuda, bsm, orc):
    # The votes are summed in a fixed order, so repeated runs on the same
    # input give bit-equal maps (floating-point atomics would not).
    torch = torch_cuda
    p = synth.CONFIG_PARAMS[1]
    _say("case: vote_refine determinism, config scene 1, radius 15, 4 runs")
    sc = synth.config_scene(1)
    pat = orc.make_pattern(synth.PATTERN_SEED, p["n"], p["S"], p["sigma"])
    ctx = bsm.Context(p["n"], p["S"], p["sigma"], pattern=pat)
    L, R = _dev(torch, sc.left), _dev(torch, sc.right)
    dl, _ = ctx.match(L, R, p["dmax"])
    dr, _ = ctx.match_right(L, R, p["dmax"])
    chk = ctx.lr_check(dl, dr, tol=1)
    first = ctx.vote_refine(L, chk, dl, p["dmax"], radius=15).cpu().numpy()
    for _ in range(3):
        again = ctx.vote_refine(L, chk, dl, p["dmax"], radius=15).cpu().numpy()
        assert np.array_equal(first, again)
    ctx.close()
