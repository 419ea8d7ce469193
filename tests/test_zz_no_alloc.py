"""GPU checks of bsm_match_noalloc, the entry point that allocates nothing.

It runs bsm_match's kernels with the pair's scratch in the library's fixed
device array.  Its outputs must equal bsm_match's bit for bit (all outputs
are integers), on consecutive calls that reuse the array with a smaller
input second, across contexts that share the array, and on another
stream.  Calls go through the C ABI; torch only provides device memory and
streams.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_1402_2020_amd import synth

pytestmark = pytest.mark.gpu

MAX_BYTES = 64 << 20  # BSM_NOALLOC_MAX_BYTES


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


def _ctx(bsm, n, S):
    sigma = 4.0 * S / 26
    pat = bsm.bsm_make_pattern(synth.PATTERN_SEED, n, S, sigma)
    return bsm.Context(n, S, sigma, pattern=pat)


def _run(torch, bsm, ctx, entry, scene, want_cost, stream=None):
    """One call of `entry` (a C function of the library) on a scene; returns
    host copies of the disparity map and the volume."""
    dev = torch.device("cuda:0")
    H, W = scene.left.shape[:2]
    dmax = scene.dmax
    L = torch.from_numpy(np.ascontiguousarray(scene.left)).to(dev)
    R = torch.from_numpy(np.ascontiguousarray(scene.right)).to(dev)
    # outputs start as garbage, so a skipped write cannot pass by accident
    disp = torch.full((H, W), -7, dtype=torch.int32, device=dev)
    cost = torch.full((dmax, H, W), -7, dtype=torch.int16, device=dev) if want_cost else None
    s = stream if stream is not None else torch.cuda.current_stream()
    torch.cuda.synchronize()
    st = entry(ctx.h, C.c_void_p(L.data_ptr()), C.c_void_p(R.data_ptr()), W, H, 3 * W, dmax,
               C.c_void_p(disp.data_ptr()),
               C.c_void_p(cost.data_ptr()) if cost is not None else None,
               C.c_void_p(s.cuda_stream))
    assert st == bsm.OK, bsm.bsm_last_error()
    torch.cuda.synchronize()
    return disp.cpu().numpy(), (cost.cpu().numpy() if cost is not None else None)


def _same(a, b, what):
    da, ca = a
    db, cb = b
    bad = np.argwhere(da != db)
    assert bad.size == 0, f"{what}: disparity differs at {bad[:5].tolist()}"
    if ca is not None:
        bad = np.argwhere(ca != cb)
        assert bad.size == 0, f"{what}: volume differs at {bad[:5].tolist()}"


def test_noalloc_equals_match_on_two_calls_in_a_row(torch_cuda, bsm):
    lib = bsm.load()
    ctx = _ctx(bsm, 1024, 31)
    big = synth.config_scene(1)                 # 450 x 375, dmax 60
    small = synth.rect_scene(14022020, 128, 96, 16)
    for name, sc in (("450x375 dmax 60", big), ("128x96 dmax 16", small)):
        H, W = sc.left.shape[:2]
        assert ctx.footprint(W, H, sc.dmax) <= MAX_BYTES
        _say(f"noalloc vs match: {name}, n 1024, with volume")
        got = _run(torch_cuda, bsm, ctx, lib.bsm_match_noalloc, sc, True)
        want = _run(torch_cuda, bsm, ctx, lib.bsm_match, sc, True)
        _same(got, want, name)
    ctx.close()


def test_noalloc_contexts_share_the_array(torch_cuda, bsm):
    # two contexts (n 1024 and n 256, mask on) call in turn on one stream:
    # each call overwrites what it reads, so stale contents never leak
    lib = bsm.load()
    a = _ctx(bsm, 1024, 31)
    b = _ctx(bsm, 256, 15)
    sc_a = synth.slanted_scene(77, 300, 200, 48)
    sc_b = synth.rect_scene(14022020, 128, 96, 16)
    want_a = _run(torch_cuda, bsm, a, lib.bsm_match, sc_a, False)
    want_b = _run(torch_cuda, bsm, b, lib.bsm_match, sc_b, True)
    for rep in range(2):
        _say(f"shared array: round {rep}")
        _same(_run(torch_cuda, bsm, a, lib.bsm_match_noalloc, sc_a, False), want_a, "ctx n 1024")
        _same(_run(torch_cuda, bsm, b, lib.bsm_match_noalloc, sc_b, True), want_b, "ctx n 256")
    a.close()
    b.close()


def test_noalloc_on_another_stream(torch_cuda, bsm):
    lib = bsm.load()
    ctx = _ctx(bsm, 512, 21)
    sc = synth.slanted_scene(5, 256, 160, 40)
    want = _run(torch_cuda, bsm, ctx, lib.bsm_match, sc, True)
    side = torch_cuda.cuda.Stream()
    _say("noalloc on a second stream")
    got = _run(torch_cuda, bsm, ctx, lib.bsm_match_noalloc, sc, True, stream=side)
    _same(got, want, "side stream")
    ctx.close()


def test_noalloc_rejects_pairs_beyond_the_array(torch_cuda, bsm):
    lib = bsm.load()
    ctx = _ctx(bsm, 1024, 31)
    W, H, dmax = 1400, 1100, 256
    assert ctx.footprint(W, H, dmax) > MAX_BYTES
    dev = torch_cuda.device("cuda:0")
    img = torch_cuda.zeros((H, W, 3), dtype=torch_cuda.uint8, device=dev)
    disp = torch_cuda.full((H, W), -7, dtype=torch_cuda.int32, device=dev)
    torch_cuda.cuda.synchronize()
    st = lib.bsm_match_noalloc(ctx.h, img.data_ptr(), img.data_ptr(), W, H, 3 * W, dmax,
                               disp.data_ptr(), None, None)
    assert st == bsm.ETOOBIG
    assert "bsm_match_noalloc" in bsm.bsm_last_error()
    torch_cuda.cuda.synchronize()
    assert int((disp != -7).sum()) == 0      # nothing was enqueued
    # the context is still usable
    small = synth.rect_scene(14022020, 128, 96, 16)
    _same(_run(torch_cuda, bsm, ctx, lib.bsm_match_noalloc, small, False),
          _run(torch_cuda, bsm, ctx, lib.bsm_match, small, False), "after rejection")
    ctx.close()
