"""GPU parity: every output of the HIP path is compared with the CPU oracle,
element by element, on the same seeded inputs.  All outputs are integers, so
the bar is bit-exact (tolerance 0).

Calls go through the C ABI (ctypes binding); torch only provides device
memory and the stream.
"""
import os
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


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _ctx(bsm, orc, n, S, sigma=None, k=0, use_mask=True, seed=None):
    sigma = 4.0 * S / 26 if sigma is None else sigma
    pat = orc.make_pattern(seed if seed is not None else n * 1000 + S, n, S, sigma)
    return bsm.Context(n, S, sigma, pattern=pat, mask_rank=k, use_mask=use_mask), pat


# ---------------------------------------------------------------- colour --

def test_color_all_colours(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: colour pre-pass over all 2^24 colours")
    ctx, _ = _ctx(bsm, orc, 64, 3)
    img = synth.all_colours_image()
    packed = ctx.color(_dev(torch, img), want_lab=True).cpu().numpy().view(np.uint32)
    lab = orc.lab8(img)
    I = orc.luma(img)
    assert np.array_equal((packed >> 24).astype(np.uint8), I)
    assert np.array_equal((packed & 0xff).astype(np.uint8), lab[..., 0])
    assert np.array_equal(((packed >> 8) & 0xff).astype(np.uint8), lab[..., 1])
    assert np.array_equal(((packed >> 16) & 0xff).astype(np.uint8), lab[..., 2])
    luma_only = ctx.color(_dev(torch, img[:64]), want_lab=False).cpu().numpy().view(np.uint32)
    assert np.array_equal(luma_only, I[:64].astype(np.uint32) << 24)
    ctx.close()


# ------------------------------------------------------------ descriptor --

DESC_CASES = [
    # W, H, n, S, k
    (1, 1, 64, 3, 0),
    (37, 29, 64, 7, 0),
    (128, 96, 256, 15, 0),
    (200, 7, 192, 26, 0),
    (5, 300, 128, 31, 1),
    (70, 45, 1024, 31, 0),
    (66, 33, 512, 63, 200),
    (41, 23, 4096, 26, 0),
    (97, 35, 2048, 31, 2048),
]


@pytest.mark.parametrize("W,H,n,S,k", DESC_CASES)
def test_describe_parity(torch_cuda, bsm, orc, W, H, n, S, k):
    torch = torch_cuda
    _say(f"case: describe W={W} H={H} n={n} S={S} k={k}")
    ctx, pat = _ctx(bsm, orc, n, S, k=k)
    img = synth.slanted_scene(W * 31 + H, W, H, 4).left if W >= 8 and H >= 8 \
        else synth.random_image(W + H, W, H)
    img = np.ascontiguousarray(img[:H, :W])
    d_img = _dev(torch, img)
    desc, mask = ctx.describe(d_img, with_mask=True)
    desc2, nomask = ctx.describe(d_img, with_mask=False)
    torch.cuda.synchronize()
    assert nomask is None
    want_desc = orc.describe(img, pat)
    want_mask, _ = orc.mask(img, pat, k=k or n // 4)
    assert np.array_equal(_u64(desc), want_desc)
    assert np.array_equal(_u64(desc2), want_desc)
    assert np.array_equal(_u64(mask), want_mask)
    ctx.close()


@pytest.mark.parametrize("n", [64, 192, 512, 1536, 2048, 4096])
def test_describe_right_four_pixels_per_lane(torch_cuda, bsm, orc, n):
    # the other view's descriptor with four pixels per lane forced: the
    # byte-parallel register path (n a multiple of 512) and the staged path
    # (other n), on a width that leaves a ragged last tile (301 = 256 + 45)
    torch = torch_cuda
    _say(f"case: describe right view, four pixels per lane, n={n}")
    ctx, pat = _ctx(bsm, orc, n, 31)
    tune = ctx.tuning()
    tune["pair_right_px"] = 4
    ctx.set_tuning(tune)
    img = np.ascontiguousarray(synth.slanted_scene(1402 + n, 301, 19, 6).left)
    desc, _ = ctx.describe(_dev(torch, img), with_mask=False)
    torch.cuda.synchronize()
    assert np.array_equal(_u64(desc), orc.describe(img, pat))
    ctx.close()


def test_describe_flat_and_random(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: describe flat + uniform random")
    ctx, pat = _ctx(bsm, orc, 256, 15)
    flat = np.full((40, 50, 3), 130, np.uint8)
    desc, mask = ctx.describe(_dev(torch, flat), with_mask=True)
    assert not _u64(desc).any()
    assert np.all(_u64(mask) == np.uint64(0xFFFFFFFFFFFFFFFF))
    img = synth.random_image(3, 77, 51)
    desc, mask = ctx.describe(_dev(torch, img), with_mask=True)
    assert np.array_equal(_u64(desc), orc.describe(img, pat))
    assert np.array_equal(_u64(mask), orc.mask(img, pat)[0])
    ctx.close()


# ------------------------------------------------------------ cost + WTA --

COST_CASES = [
    # W, H, nw, dmax, mask, volume
    (7, 3, 1, 1, True, True),
    (7, 3, 1, 7, True, True),
    (130, 5, 4, 64, True, True),
    (131, 4, 4, 65, False, True),
    (300, 3, 16, 130, True, True),
    (257, 6, 16, 257, True, False),
    (450, 4, 16, 60, True, True),
    (129, 3, 2, 100, False, False),
    (260, 5, 8, 200, True, True),
    (96, 4, 3, 40, True, True),     # word-chunked kernel (nw not a power of two)
    (150, 3, 24, 70, False, True),  # word-chunked kernel
    (70, 2, 64, 33, True, True),    # word-chunked kernel, n = 4096
    (301, 3, 32, 300, True, True),  # several disparity chunks, ragged tile
    (1, 2, 5, 1, True, True),       # one pixel, partial word chunk
    (259, 2, 64, 97, False, False), # n = 4096, Eq. 4
    (200, 3, 9, 64, True, False),   # two full disparity chunks
]


@pytest.mark.parametrize("W,H,nw,dmax,use_mask,vol", COST_CASES)
def test_cost_wta_parity(torch_cuda, bsm, orc, W, H, nw, dmax, use_mask, vol):
    torch = torch_cuda
    _say(f"case: cost_wta W={W} H={H} nw={nw} dmax={dmax} mask={use_mask} vol={vol}")
    rng = np.random.Generator(np.random.PCG64(W * H + nw + dmax))
    # correlated descriptors so that minima are not all at d = 0
    # left(u) = right(u - s) ^ sparse noise, with s drawn in [0, dmax)
    base = rng.integers(0, 2**63, (H, W + dmax, nw), dtype=np.uint64)
    noise = rng.integers(0, 2**63, (H, W, nw), dtype=np.uint64) & \
        rng.integers(0, 2**63, (H, W, nw), dtype=np.uint64) & \
        rng.integers(0, 2**63, (H, W, nw), dtype=np.uint64)
    shift = int(rng.integers(0, dmax))
    dr = np.ascontiguousarray(base[:, dmax:dmax + W])
    dl = np.ascontiguousarray(base[:, dmax - shift:dmax - shift + W] ^ noise)
    m = rng.integers(0, 2**63, (H, W, nw), dtype=np.uint64) if use_mask else None
    ctx, _ = _ctx(bsm, orc, 64 * nw, 3)
    t = lambda a: None if a is None else _dev(torch, a.view(np.int64))
    disp, cost = ctx.cost_wta(t(dl), t(m), t(dr), dmax, want_cost=vol)
    torch.cuda.synchronize()
    want_cost = orc.cost_volume(dl, m, dr, dmax)
    want_disp = orc.wta(want_cost)
    assert np.array_equal(disp.cpu().numpy(), want_disp)
    if vol:
        assert np.array_equal(cost.cpu().numpy(), want_cost)
    ctx.close()


MFMA_CASES = [
    # W, H, nw, dmax, mask
    (1, 2, 1, 1, True),
    (31, 3, 2, 31, True),
    (33, 2, 4, 1, False),
    (97, 3, 8, 64, True),
    (130, 2, 16, 33, True),
    (300, 3, 16, 257, True),
    (257, 2, 16, 130, False),
    (64, 4, 16, 64, True),
    (450, 2, 16, 60, True),
    (259, 3, 16, 256, True),   # largest dmax with the volume on the matrix cores, odd W
    (77, 3, 4, 40, False),     # odd W, Eq. 4
    # tile pairs of the single-pair kernel: the block range without checks is
    # empty for the first pair and one or two blocks long for later ones
    (200, 2, 16, 96, True),
    (190, 3, 8, 129, False),
    # long descriptors: matrix cores in passes of 512 bits (no volume,
    # dmax <= 256), the word-chunked bitwise kernel otherwise
    (130, 3, 32, 64, True),    # n = 2048
    (97, 2, 48, 17, True),     # n = 3072, smallest dmax on the matrix cores
    (259, 3, 64, 256, True),   # n = 4096, nine right blocks, odd W
    (64, 2, 64, 33, False),    # n = 4096, Eq. 4
    (300, 2, 32, 257, True),   # n = 2048, dmax past the long kernel
]


@pytest.mark.parametrize("W,H,nw,dmax,use_mask", MFMA_CASES)
def test_cost_wta_matrix_core_and_bitwise(torch_cuda, bsm, orc, W, H, nw, dmax, use_mask):
    # the fused cost + WTA runs on the matrix cores by default (the cost as
    # an integer dot product; with a volume up to dmax 256); both kernels
    # must give the oracle's winners and volume
    torch = torch_cuda
    _say(f"case: cost_wta mfma and bitwise, with and without volume, W={W} H={H} nw={nw} dmax={dmax} "
         f"mask={use_mask}")
    rng = np.random.Generator(np.random.PCG64(7 * W + H + 13 * nw + dmax))
    base = rng.integers(0, 2**63, (H, W + dmax, nw), dtype=np.uint64)
    noise = rng.integers(0, 2**63, (H, W, nw), dtype=np.uint64) & \
        rng.integers(0, 2**63, (H, W, nw), dtype=np.uint64)
    shift = int(rng.integers(0, dmax))
    dr = np.ascontiguousarray(base[:, dmax:dmax + W])
    dl = np.ascontiguousarray(base[:, dmax - shift:dmax - shift + W] ^ noise)
    m = rng.integers(0, 2**63, (H, W, nw), dtype=np.uint64) if use_mask else None
    want_cost = orc.cost_volume(dl, m, dr, dmax)
    want = orc.wta(want_cost)
    ctx, _ = _ctx(bsm, orc, 64 * nw, 3)
    t = lambda a: None if a is None else _dev(torch, a.view(np.int64))
    for mfma in (1, 0):
        tune = ctx.tuning()
        tune["cost_mfma"] = mfma
        ctx.set_tuning(tune)
        disp, _ = ctx.cost_wta(t(dl), t(m), t(dr), dmax, want_cost=False)
        disp_v, cost = ctx.cost_wta(t(dl), t(m), t(dr), dmax, want_cost=True)
        torch.cuda.synchronize()
        assert np.array_equal(disp.cpu().numpy(), want), mfma
        assert np.array_equal(disp_v.cpu().numpy(), want), mfma
        assert np.array_equal(cost.cpu().numpy(), want_cost), mfma
    ctx.close()


def test_cost_wta_matrix_core_ties(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: matrix-core cost_wta, all-equal and all-different descriptors")
    ctx, _ = _ctx(bsm, orc, 1024, 3)
    z = torch.zeros((3, 100, 16), dtype=torch.int64, device="cuda")
    disp, _ = ctx.cost_wta(z, z, z, 70, want_cost=False)
    assert not disp.cpu().numpy().any()          # every cost 0: lowest d
    ones = torch.full((3, 100, 16), -1, dtype=torch.int64, device="cuda")
    disp, _ = ctx.cost_wta(ones, ones, z, 70, want_cost=False)
    assert not disp.cpu().numpy().any()          # every cost n: lowest d
    ctx.close()


def test_cost_ties_take_lowest_d(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: all-equal descriptors (every cost 0)")
    ctx, _ = _ctx(bsm, orc, 256, 3)
    z = torch.zeros((5, 140, 4), dtype=torch.int64, device="cuda")
    disp, cost = ctx.cost_wta(z, z, z, 90, want_cost=True)
    assert not disp.cpu().numpy().any()
    c = cost.cpu().numpy()
    for d in range(90):
        assert np.all(c[d, :, :d] == 32767) and np.all(c[d, :, d:] == 0)
    ctx.close()


# ------------------------------------------------------ whole pair paths --

def _match_case(torch, bsm, orc, scene, n, S, dmax, want_cost, threads=16):
    ctx, pat = _ctx(bsm, orc, n, S, seed=synth.PATTERN_SEED)
    L, R = _dev(torch, scene.left), _dev(torch, scene.right)
    disp, cost = ctx.match(L, R, dmax, want_cost=want_cost)
    disp2, _ = ctx.match(L, R, dmax, want_cost=False)
    torch.cuda.synchronize()
    orc.set_threads(threads)
    want_disp, want_cost_v = orc.match(scene.left, scene.right, pat, dmax, want_cost=want_cost)
    orc.set_threads(1)
    got = disp.cpu().numpy()
    assert np.array_equal(got, want_disp), np.argwhere(got != want_disp)[:5]
    assert np.array_equal(disp2.cpu().numpy(), got)   # deterministic, volume on/off agree
    if want_cost:
        assert np.array_equal(cost.cpu().numpy(), want_cost_v)
    ctx.close()


def test_match_rect_scene_128x96(torch_cuda, bsm, orc):
    _say("case: match 128x96 rectangles, n=256 S=15 dmax=16")
    p = synth.CONFIG_PARAMS[0]
    _match_case(torch_cuda, bsm, orc, synth.config_scene(0), p["n"], p["S"], p["dmax"], True)


def test_match_slanted_450x375_with_volume(torch_cuda, bsm, orc):
    _say("case: match 450x375 slanted planes, n=1024 S=31 dmax=60, volume")
    p = synth.CONFIG_PARAMS[1]
    _match_case(torch_cuda, bsm, orc, synth.config_scene(1), p["n"], p["S"], p["dmax"], True)


def test_match_slanted_1400x1100_radiometric(torch_cuda, bsm, orc):
    _say("case: match 1400x1100 slanted planes + radiometric change, n=1024 S=31 dmax=256")
    p = synth.CONFIG_PARAMS[2]
    _match_case(torch_cuda, bsm, orc, synth.config_scene(2), p["n"], p["S"], p["dmax"], False)


@pytest.mark.parametrize("n", [2048, 4096])
def test_match_long_descriptors(torch_cuda, bsm, orc, n):
    # the paper's n = 4096 (Section 4.1) and n = 2048: describe in chunks of
    # 16 pairs, cost on the matrix cores in passes of 512 bits
    _say(f"case: match 240x64 slanted planes, n={n} S=31 dmax=96")
    sc = synth.slanted_scene(14022033, 240, 64, 96)
    _match_case(torch_cuda, bsm, orc, sc, n, 31, 96, False)


def test_match_without_mask(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: match without mask (Eq. 4)")
    sc = synth.rect_scene(5, 100, 60, 16)
    ctx, pat = _ctx(bsm, orc, 256, 15, use_mask=False, seed=3)
    disp, cost = ctx.match(_dev(torch, sc.left), _dev(torch, sc.right), 16, want_cost=True)
    wd, wc = orc.match(sc.left, sc.right, pat, 16, use_mask=False, want_cost=True)
    assert np.array_equal(disp.cpu().numpy(), wd)
    assert np.array_equal(cost.cpu().numpy(), wc)
    ctx.close()


def test_match_constant_disparity_recovered(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: constant disparity 9 recovered exactly")
    sc = synth.constant_shift_pair(9, 96, 48, 9)
    ctx, pat = _ctx(bsm, orc, 256, 15, seed=1)
    disp, cost = ctx.match(_dev(torch, sc.left), _dev(torch, sc.right), 16, want_cost=True)
    c = cost.cpu().numpy()
    assert np.all(c[9, 7:41, 16:89] == 0)
    wd, _ = orc.match(sc.left, sc.right, pat, 16)
    assert np.array_equal(disp.cpu().numpy(), wd)
    ctx.close()


def test_match_batch_uneven(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: batch of uneven pairs")
    specs = synth.batch_specs(6)
    ctx, pat = _ctx(bsm, orc, 256, 15, seed=2)
    scenes = [synth.batch_scene(s, scale=0.12) for s in specs]
    items = [(_dev(torch, s.left), _dev(torch, s.right), s.dmax) for s in scenes]
    outs = ctx.match_batch(items, want_cost=True)
    torch.cuda.synchronize()
    for s, (disp, cost) in zip(scenes, outs):
        wd, wc = orc.match(s.left, s.right, pat, s.dmax, want_cost=True)
        assert np.array_equal(disp.cpu().numpy(), wd)
        assert np.array_equal(cost.cpu().numpy(), wc)
    ctx.close()


def test_device_calls_validate_arguments(torch_cuda, bsm, orc):
    torch = torch_cuda
    ctx, _ = _ctx(bsm, orc, 256, 15)
    img = torch.zeros((8, 8, 3), dtype=torch.uint8, device="cuda")
    d = torch.zeros((8, 8, 4), dtype=torch.int64, device="cuda")
    disp = torch.zeros((8, 8), dtype=torch.int32, device="cuda")
    lib = bsm.load()
    P = lambda t: None if t is None else t.data_ptr()
    assert lib.bsm_cost_wta(ctx.h, P(d), None, P(d), 8, 8, 9, P(disp), None, None) == bsm.EINVAL
    assert lib.bsm_cost_wta(ctx.h, P(d), None, P(d), 8, 8, 0, P(disp), None, None) == bsm.EINVAL
    assert lib.bsm_match(ctx.h, P(img), P(img), 8, 8, 23, 4, P(disp), None, None) == bsm.EINVAL
    assert lib.bsm_describe(ctx.h, P(img), 8, 8, 24, P(d) + 4, None, None) == bsm.EINVAL
    assert lib.bsm_match(ctx.h, P(img), P(img), 8, 8, 24, 4, P(disp), None, None) == bsm.OK
    torch.cuda.synchronize()
    ctx.close()


def test_match_alternating_streams(torch_cuda, bsm, orc):
    # the single-pair scratch moves between streams: each call must see its
    # own inputs and leave the previous call's results intact
    torch = torch_cuda
    _say("case: bsm_match alternating between two streams, pairs above 64 K pixels")
    p = synth.CONFIG_PARAMS[0]
    ctx, pat = _ctx(bsm, orc, p["n"], p["S"], seed=synth.PATTERN_SEED)
    scenes = [synth.slanted_scene(40 + i, 320, 210, 30) for i in range(3)]
    want = [orc.match(s.left, s.right, pat, 30)[0] for s in scenes]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for rep in range(2):
        for i, s in enumerate(scenes):
            st = streams[(i + rep) % 2]
            with torch.cuda.stream(st):
                L, R = _dev(torch, s.left), _dev(torch, s.right)
                d, _ = ctx.match(L, R, 30, stream=st)
                outs.append((i, d))
    torch.cuda.synchronize()
    for i, d in outs:
        assert np.array_equal(d.cpu().numpy(), want[i]), i
    ctx.close()
