"""GPU tests of the batched path (bsm_match_batch), the launch tunings and
the autotuner.  Every result is compared bit for bit with the CPU oracle or
with the single-pair path (itself checked against the oracle)."""
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


def _scenes(count, scale, first=0):
    return [synth.batch_scene(s, scale=scale) for s in synth.batch_specs(first + count)[first:]]


def _check_batch_vs_oracle(torch, ctx, pat, orc, scenes, want_cost, use_mask=True):
    items = [(_dev(torch, s.left), _dev(torch, s.right), s.dmax) for s in scenes]
    outs = ctx.match_batch(items, want_cost=want_cost)
    torch.cuda.synchronize()
    orc.set_threads(8)
    try:
        for s, (disp, cost) in zip(scenes, outs):
            wd, wc = orc.match(s.left, s.right, pat, s.dmax, use_mask=use_mask,
                               want_cost=want_cost)
            assert np.array_equal(disp.cpu().numpy(), wd), (s.left.shape, s.dmax)
            if want_cost:
                assert np.array_equal(cost.cpu().numpy(), wc)
    finally:
        orc.set_threads(1)
    return outs


@pytest.mark.parametrize("n,S,scale,want_cost", [(256, 15, 0.15, True), (1024, 31, 0.12, False),
                                                 (64, 7, 0.1, True), (512, 31, 0.1, False)])
def test_batch_persistent_equals_oracle(torch_cuda, bsm, orc, n, S, scale, want_cost):
    _say(f"case: persistent batch n={n} S={S} scale={scale} volume={want_cost}")
    ctx, pat = _ctx(bsm, orc, n, S)
    _check_batch_vs_oracle(torch_cuda, ctx, pat, orc, _scenes(7, scale), want_cost)
    ctx.close()


@pytest.mark.parametrize("want_cost", [True, False])
def test_batch_without_mask(torch_cuda, bsm, orc, want_cost):
    _say(f"case: persistent batch, mask off (Eq. 4), volume={want_cost}")
    ctx, pat = _ctx(bsm, orc, 256, 15, use_mask=False)
    _check_batch_vs_oracle(torch_cuda, ctx, pat, orc, _scenes(5, 0.12), want_cost, use_mask=False)
    ctx.close()


@pytest.mark.parametrize("n,S,want_cost", [(256, 15, True), (1024, 31, False)])
def test_batch_degenerate_pairs(torch_cuda, bsm, orc, n, S, want_cost):
    # Pairs at the edges of the method in one persistent batch: a single
    # pixel, rows shorter than a tile, dmax = W, fewer rows than XCD queues
    # (empty cost queues), a ragged tall pair.
    torch = torch_cuda
    sizes = [(1, 1, 1), (3, 2, 3), (64, 1, 64), (33, 17, 33), (130, 5, 100), (7, 41, 2)]
    _say(f"case: persistent batch of degenerate pairs n={n} S={S} volume={want_cost}")
    ctx, pat = _ctx(bsm, orc, n, S)
    pairs = [(synth.random_image(500 + i, W, H), synth.random_image(600 + i, W, H), d)
             for i, (W, H, d) in enumerate(sizes)]
    items = [(_dev(torch, L), _dev(torch, R), d) for L, R, d in pairs]
    outs = ctx.match_batch(items, want_cost=want_cost)
    torch.cuda.synchronize()
    for (L, R, d), (disp, cost) in zip(pairs, outs):
        wd, wc = orc.match(L, R, pat, d, want_cost=want_cost)
        assert np.array_equal(disp.cpu().numpy(), wd), (L.shape, d)
        if want_cost:
            assert np.array_equal(cost.cpu().numpy(), wc), (L.shape, d)
    ctx.close()


def test_empty_batch(torch_cuda, bsm, orc):
    ctx, _ = _ctx(bsm, orc, 256, 15)
    assert ctx.match_batch([]) == []
    lib = bsm.load()
    assert lib.bsm_match_batch(ctx.h, None, 0, None) == bsm.OK
    assert lib.bsm_autotune(ctx.h, None, 0, 1, None, None, None) == bsm.EINVAL
    ctx.close()


def test_batch_sequential_fallback(torch_cuda, bsm, orc):
    _say("case: batch with n=192 (runs pair by pair)")
    ctx, pat = _ctx(bsm, orc, 192, 11)
    _check_batch_vs_oracle(torch_cuda, ctx, pat, orc, _scenes(3, 0.1), True)
    ctx.close()


def test_batch_graph_reused_across_shapes_and_replays(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: batch graph replays with different shapes and eager work between")
    ctx, pat = _ctx(bsm, orc, 256, 15)
    first = _scenes(5, 0.1)
    second = _scenes(7, 0.13, first=10)
    want = {}
    for s in first + second:
        want[id(s)] = orc.match(s.left, s.right, pat, s.dmax)[0]
    for rep in range(3):
        for group in (first, second):
            items = [(_dev(torch, s.left), _dev(torch, s.right), s.dmax) for s in group]
            outs = ctx.match_batch(items)
            # eager work of the program between replays
            junk = torch.randn(1000, device="cuda").sum()
            torch.cuda.synchronize()
            for s, (disp, _) in zip(group, outs):
                assert np.array_equal(disp.cpu().numpy(), want[id(s)]), rep
            del junk
    ctx.close()


def test_batch_graph_replays_as_the_pair_count_grows_and_shrinks(torch_cuda, bsm, orc):
    # The replayed graph must reach the queue counters and the work tables of
    # the current batch only: the tables are reallocated when a batch needs
    # more pairs than any before it, and their layout moves with the count.
    torch = torch_cuda
    _say("case: batch graph replays with 5, 9, 6, 12 pairs (and 2 pair by pair), tuning changed")
    ctx, pat = _ctx(bsm, orc, 256, 15)
    scenes = _scenes(12, 0.08, first=20)
    want = [orc.match(s.left, s.right, pat, s.dmax)[0] for s in scenes]
    tunings = [None, dict(desc_tile_w=32, cost_dchunk=32, blocks_per_cu=[0, 2, 0, 1]), None,
               dict(desc_tile_w=16, cost_dchunk=64, blocks_per_cu=[0, 0, 0, 0]), None]
    for count, tune in zip((5, 9, 6, 12, 2), tunings):
        if tune is not None:
            ctx.set_tuning(tune)
        group = list(range(count))
        items = [(_dev(torch, scenes[j].left), _dev(torch, scenes[j].right), scenes[j].dmax)
                 for j in group]
        outs = ctx.match_batch(items)
        torch.cuda.synchronize()
        for j, (disp, _) in zip(group, outs):
            assert np.array_equal(disp.cpu().numpy(), want[j]), (count, j)
    ctx.close()


def test_batches_queued_back_to_back(torch_cuda, bsm, orc):
    # Batches queued with no wait in between: each one rewrites the pinned
    # staging buffer and the device tables while the previous batch may
    # still run (the tables grow once, and one batch goes to another
    # stream, which makes the next one wait for it).
    torch = torch_cuda
    _say("case: five batches queued back to back, 5/6/5/9/5 pairs, one on a second stream")
    ctx, pat = _ctx(bsm, orc, 256, 15)
    groups = [_scenes(5, 0.1, first=30), _scenes(6, 0.12, first=35), _scenes(5, 0.08, first=41),
              _scenes(9, 0.1, first=46), _scenes(5, 0.1, first=55)]
    want = [[orc.match(s.left, s.right, pat, s.dmax)[0] for s in g] for g in groups]
    items = [[(_dev(torch, s.left), _dev(torch, s.right), s.dmax) for s in g] for g in groups]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    outs = []
    for k, group in enumerate(items):
        outs.append(ctx.match_batch(group, stream=side if k == 2 else None))
    torch.cuda.synchronize()
    for k, (group_out, group_want) in enumerate(zip(outs, want)):
        for j, ((disp, _), wd) in enumerate(zip(group_out, group_want)):
            assert np.array_equal(disp.cpu().numpy(), wd), (k, j)
    ctx.close()


def test_batch_equals_single_pair_path_full_size(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: batch of 6 full-size uneven pairs == single-pair path")
    ctx, pat = _ctx(bsm, orc, 1024, 31, seed=synth.PATTERN_SEED)
    scenes = _scenes(6, 1.0)
    items = [(_dev(torch, s.left), _dev(torch, s.right), s.dmax) for s in scenes]
    outs = ctx.match_batch(items)
    singles = [ctx.match(L, R, d)[0] for L, R, d in items]
    torch.cuda.synchronize()
    for (disp, _), single in zip(outs, singles):
        assert torch.equal(disp, single)
    # and one of them against the oracle (smallest, to bound CPU time)
    k = min(range(len(scenes)), key=lambda i: scenes[i].left.size * scenes[i].dmax)
    orc.set_threads(16)
    wd, _ = orc.match(scenes[k].left, scenes[k].right, pat, scenes[k].dmax)
    orc.set_threads(1)
    assert np.array_equal(outs[k][0].cpu().numpy(), wd)
    ctx.close()


TUNINGS = [dict(desc_tile_w=tw, cost_dchunk=dc, blocks_per_cu=[0, bm, 0, bc], cost_mfma=mf,
                batch_tile_h=8 if dc == 32 else 16)
           for tw in (16, 32) for dc in (32, 64) for bm, bc in ((0, 0), (2, 1)) for mf in (1, 0)
           if mf == 1 or (bm, bc) == (0, 0)]
_TUNING_SCENE = {}


def _tuning_scene(orc, pat):
    key = pat.tobytes()
    if key not in _TUNING_SCENE:
        sc = synth.slanted_scene(33, 300, 70, 130)
        _TUNING_SCENE[key] = sc, orc.match(sc.left, sc.right, pat, sc.dmax, want_cost=True)
    return _TUNING_SCENE[key]


@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: f"tw{t['desc_tile_w']}-th{t['batch_tile_h']}-"
                         f"dc{t['cost_dchunk']}-b{t['blocks_per_cu'][1]}{t['blocks_per_cu'][3]}-"
                         f"mfma{t['cost_mfma']}")
def test_tunings_do_not_change_results(torch_cuda, bsm, orc, tuning):
    # single pair with and without a volume, and a persistent five-pair
    # batch with and without volumes, under each launch choice
    torch = torch_cuda
    _say(f"case: tuning {tuning}")
    ctx, pat = _ctx(bsm, orc, 1024, 31, seed=11)
    sc, (wd, wc) = _tuning_scene(orc, pat)
    ctx.set_tuning(tuning)
    got = ctx.tuning()
    assert {k: got[k] for k in tuning} == tuning
    L, R = _dev(torch, sc.left), _dev(torch, sc.right)
    disp, cost = ctx.match(L, R, sc.dmax, want_cost=True)
    disp_nv, _ = ctx.match(L, R, sc.dmax, want_cost=False)
    outs = ctx.match_batch([(L, R, sc.dmax)] * 5, want_cost=False)
    outs_v = ctx.match_batch([(L, R, sc.dmax)] * 5, want_cost=True)
    torch.cuda.synchronize()
    assert np.array_equal(disp.cpu().numpy(), wd)
    assert np.array_equal(cost.cpu().numpy(), wc)
    assert np.array_equal(disp_nv.cpu().numpy(), wd)
    for o in outs:
        assert np.array_equal(o[0].cpu().numpy(), wd)
    for o in outs_v:
        assert np.array_equal(o[0].cpu().numpy(), wd)
        assert np.array_equal(o[1].cpu().numpy(), wc)
    ctx.close()


def test_set_tuning_validates(torch_cuda, bsm, orc):
    ctx, _ = _ctx(bsm, orc, 256, 15)
    for bad in (dict(desc_tile_w=8, cost_dchunk=64), dict(desc_tile_w=16, cost_dchunk=48),
                dict(desc_tile_w=16, cost_dchunk=64, blocks_per_cu=[0, 0, 0, 65]),
                dict(desc_tile_w=16, cost_dchunk=64, cost_mfma=2),
                dict(desc_tile_w=16, cost_dchunk=64, batch_tile_h=12),
                dict(desc_tile_w=16, cost_dchunk=64, pair_desc_th=6),
                dict(desc_tile_w=16, cost_dchunk=64, pair_right_px=2),
                dict(desc_tile_w=16, cost_dchunk=64, mfma_min_dmax=1),
                dict(desc_tile_w=16, cost_dchunk=64, mfma_min_dmax=258)):
        assert bsm.bsm_set_tuning(ctx.h, bsm.Tuning.from_dict(bad)) == bsm.EINVAL
    ctx.close()


def test_autotune_picks_a_candidate_and_keeps_results(torch_cuda, bsm, orc):
    torch = torch_cuda
    _say("case: autotune on a small uneven batch")
    ctx, pat = _ctx(bsm, orc, 256, 15)
    scenes = _scenes(5, 0.15)
    items = [(_dev(torch, s.left), _dev(torch, s.right), s.dmax) for s in scenes]
    best, ms = ctx.autotune(items, reps=2)
    assert best["desc_tile_w"] in (16, 32) and best["batch_tile_h"] in (8, 16)
    assert ms > 0
    assert ctx.tuning() == best
    _check_batch_vs_oracle(torch, ctx, pat, orc, scenes, False)
    ctx.close()


PAIR_TUNINGS = [dict(desc_tile_w=tw, cost_dchunk=64, pair_desc_th=th, pair_right_px=px,
                     mfma_min_dmax=md)
                for tw in (16, 32) for th in (4, 8) for px in (1, 4) for md in (2, 17, 257)
                if (tw, th, px) in ((16, 4, 1), (32, 8, 4)) or md == 17]


@pytest.mark.parametrize("tuning", PAIR_TUNINGS,
                         ids=lambda t: f"tw{t['desc_tile_w']}-th{t['pair_desc_th']}-"
                         f"px{t['pair_right_px']}-md{t['mfma_min_dmax']}")
def test_single_pair_tunings_do_not_change_results(torch_cuda, bsm, orc, tuning):
    # describe tile height, descriptor-only pixels per lane and the dmax
    # from which the matrix-core cost kernel runs (2: even dmax 5 on the
    # matrix cores; 257: the bitwise kernel everywhere), on a pair whose
    # width is not a multiple of any tile and on a short disparity range
    torch = torch_cuda
    _say(f"case: single-pair tuning {tuning}")
    ctx, pat = _ctx(bsm, orc, 1024, 31, seed=11)
    sc, (wd, wc) = _tuning_scene(orc, pat)
    ctx.set_tuning(tuning)
    L, R = _dev(torch, sc.left), _dev(torch, sc.right)
    disp, cost = ctx.match(L, R, sc.dmax, want_cost=True)
    disp_nv, _ = ctx.match(L, R, sc.dmax)
    small = synth.slanted_scene(34, 77, 23, 5)
    ws, wsc = orc.match(small.left, small.right, pat, 5, want_cost=True)
    ds, cs = ctx.match(_dev(torch, small.left), _dev(torch, small.right), 5, want_cost=True)
    torch.cuda.synchronize()
    assert np.array_equal(disp.cpu().numpy(), wd)
    assert np.array_equal(cost.cpu().numpy(), wc)
    assert np.array_equal(disp_nv.cpu().numpy(), wd)
    assert np.array_equal(ds.cpu().numpy(), ws)
    assert np.array_equal(cs.cpu().numpy(), wsc)
    ctx.close()


def test_batch_stage_times_keep_results(torch_cuda, bsm, orc):
    # the eagerly launched, event-timed batch writes what the graph writes
    torch = torch_cuda
    _say("case: bsm_batch_stage_times on 6 small uneven pairs")
    ctx, pat = _ctx(bsm, orc, 256, 15)
    scenes = _scenes(6, 0.2)
    items = [(_dev(torch, s.left), _dev(torch, s.right), s.dmax) for s in scenes]
    want = [d.clone() for d, _ in ctx.match_batch(items)]
    pairs, outs, keep = ctx._pairs(items, False)
    st, ms = bsm.bsm_batch_stage_times(ctx.h, pairs, None)
    assert st == bsm.OK, bsm.bsm_last_error()
    assert ms[0] > 0 and ms[1] > 0 and ms[2] > 0 and ms[3] >= 0
    torch.cuda.synchronize()
    for w, (d, _) in zip(want, outs):
        assert torch.equal(w, d)
    # four pairs take the per-pair path, which has no stages
    st, _ = bsm.bsm_batch_stage_times(ctx.h, pairs[:4], None)
    assert st == bsm.EINVAL
    del keep
    ctx.close()


def test_autotune_cache_miss_then_hit(torch_cuda, bsm, orc, tmp_path):
    import json
    torch = torch_cuda
    _say("case: bsm_autotune_cached, miss then hit, batch and single pair")
    ctx, pat = _ctx(bsm, orc, 256, 15)
    path = str(tmp_path / "tuning.json")
    scenes = _scenes(5, 0.15)
    items = [(_dev(torch, s.left), _dev(torch, s.right), s.dmax) for s in scenes]
    best, ms, hit = ctx.autotune_cached(items, path, reps=1)
    assert not hit and ms > 0
    one, ms1, hit1 = ctx.autotune_cached(items[:1], path, reps=1)
    assert not hit1 and one["pair_desc_th"] in (4, 8) and one["pair_right_px"] in (1, 4)
    data = json.load(open(path))
    assert len(data) == 2
    keys = sorted(data)
    assert any(" batch " in k for k in keys) and any(" pairs " in k for k in keys)
    ctx.set_tuning(dict(desc_tile_w=16, cost_dchunk=64))
    again, ms2, hit2 = ctx.autotune_cached(items, path, reps=1)
    assert hit2 and again == best and ms2 == pytest.approx(ms, rel=1e-6)
    assert ctx.tuning() == best
    _check_batch_vs_oracle(torch, ctx, pat, orc, scenes, False)
    ctx.close()
