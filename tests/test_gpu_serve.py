"""GPU tests of the serving path (bsm_serve_config / bsm_submit / bsm_poll /
bsm_drain): results of pairs served in a mix equal the CPU oracle and the
single-pair path, timestamps are ordered, and the admission limits (cap,
queue length) are enforced."""
import sys
import time

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


def _ctx(bsm, orc, n, S, seed=7):
    sigma = 4.0 * S / 26
    pat = orc.make_pattern(seed, n, S, sigma)
    return bsm.Context(n, S, sigma, pattern=pat), pat


def _scenes(count, scale, first=0):
    return [synth.batch_scene(s, scale=scale) for s in synth.batch_specs(first + count)[first:]]


def _wait(ctx, ticket, timeout=60.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        state, times, out = ctx.poll(ticket)
        if state != 0:
            return state, times, out
        time.sleep(0.0005)
    raise TimeoutError(f"ticket {ticket} still pending after {timeout} s")


def test_serve_mix_equals_oracle(torch_cuda, bsm, orc):
    _say("case: serving, 10 uneven pairs n=256 S=15, volume on every other pair")
    ctx, pat = _ctx(bsm, orc, 256, 15)
    scenes = _scenes(10, 0.15)
    tickets = [ctx.submit(s.left, s.right, s.dmax, want_cost=(i % 2 == 0))
               for i, s in enumerate(scenes)]
    ctx.drain()
    orc.set_threads(8)
    try:
        for i, (s, t) in enumerate(zip(scenes, tickets)):
            state, times, (disp, cost) = ctx.poll(t)
            assert state == 1
            assert times[0] <= times[1] <= times[2] <= times[3]
            wd, wc = orc.match(s.left, s.right, pat, s.dmax, want_cost=(i % 2 == 0))
            assert np.array_equal(disp, wd), (s.left.shape, s.dmax)
            if i % 2 == 0:
                assert np.array_equal(cost, wc)
    finally:
        orc.set_threads(1)
    ctx.close()


def test_serve_groups_of_growing_size_on_one_slot(torch_cuda, bsm, orc):
    # One pair first (each slot's first batch is small), then bursts that
    # form larger groups on the same slots, with the tuning changed between.
    _say("case: serving bursts of 1, 12, 5 pairs in groups of up to 8, tuning changed between")
    ctx, pat = _ctx(bsm, orc, 256, 15)
    # groups of five or more pairs run as persistent batches
    ctx.serve_config(8 << 30, 1024, 8)
    scenes = _scenes(12, 0.1, first=30)
    want = [orc.match(s.left, s.right, pat, s.dmax)[0] for s in scenes]
    for burst, tune in ((1, None), (12, dict(desc_tile_w=32, cost_dchunk=32,
                                             blocks_per_cu=[0, 2, 0, 1])), (5, None)):
        if tune is not None:
            ctx.set_tuning(tune)
        ts = [ctx.submit(scenes[j].left, scenes[j].right, scenes[j].dmax) for j in range(burst)]
        ctx.drain()
        for j, t in enumerate(ts):
            state, _, (disp, _) = ctx.poll(t)
            assert state == 1
            assert np.array_equal(disp, want[j]), (burst, j)
    st = ctx.serve_stats()
    _say(f"serve stats: {st}")
    assert st["completed"] == 18 and st["failed"] == 0
    # the burst of 12 arrived while earlier work ran: later pairs were
    # grouped, and groups ran on more than one slot at once
    assert st["max_group"] > 1 and st["max_slots_busy"] > 1
    ctx.close()


def test_serve_same_alone_and_in_the_mix(torch_cuda, bsm, orc):
    _say("case: serving n=1024 S=31, 6 pairs in a mix vs each alone vs bsm_match")
    torch = torch_cuda
    ctx, _ = _ctx(bsm, orc, 1024, 31)
    scenes = _scenes(6, 0.3, first=10)
    mixed = [ctx.submit(s.left, s.right, s.dmax) for s in scenes]
    ctx.drain()
    mixed = [ctx.poll(t)[2][0] for t in mixed]
    for s, got in zip(scenes, mixed):
        t = ctx.submit(s.left, s.right, s.dmax)
        state, _, (alone, _) = _wait(ctx, t)
        assert state == 1
        ref, _ = ctx.match(torch.from_numpy(s.left).cuda(), torch.from_numpy(s.right).cuda(),
                           s.dmax)
        torch.cuda.synchronize()
        assert np.array_equal(got, alone)
        assert np.array_equal(got, ref.cpu().numpy())
    ctx.close()


def test_serve_full_size_sample_equals_oracle(torch_cuda, bsm, orc):
    _say("case: serving full-size 1920x1080-class pair, sampled rows vs oracle")
    ctx, pat = _ctx(bsm, orc, 1024, 31)
    spec = max(synth.batch_specs(64), key=lambda s: s.W * s.H * s.dmax)
    s = synth.batch_scene(spec)
    state, _, (disp, _) = _wait(ctx, ctx.submit(s.left, s.right, s.dmax))
    assert state == 1
    # the oracle on a horizontal band: rows far enough from the band's edges
    # see the same neighbourhoods as in the full image
    r = 31 // 2
    v0, v1 = s.left.shape[0] // 2 - 8, s.left.shape[0] // 2 + 8
    band = slice(v0 - r, v1 + r)
    orc.set_threads(8)
    try:
        wd, _ = orc.match(np.ascontiguousarray(s.left[band]), np.ascontiguousarray(s.right[band]),
                          pat, s.dmax)
    finally:
        orc.set_threads(1)
    assert np.array_equal(disp[v0:v1], wd[r:r + (v1 - v0)])
    ctx.close()


def test_serve_too_big_and_queue_full(torch_cuda, bsm, orc):
    _say("case: serving admission limits (ETOOBIG, EAGAIN)")
    ctx, _ = _ctx(bsm, orc, 1024, 31)
    s = synth.batch_scene(synth.batch_specs(1)[0])
    ctx.serve_config(1 << 20, 64)
    with pytest.raises(bsm.BsmError) as e:
        ctx.submit(s.left, s.right, s.dmax)
    assert e.value.status == bsm.ETOOBIG
    # room for one pair at a time (a served pair holds a little more than the
    # scratch of bsm_match) and one waiting: fast submissions bounce
    ctx.serve_config(ctx.footprint(s.left.shape[1], s.left.shape[0], s.dmax) * 3 // 2, 1)
    tickets, bounced = [], 0
    for _ in range(12):
        try:
            tickets.append(ctx.submit(s.left, s.right, s.dmax))
        except bsm.BsmError as err:
            assert err.status == bsm.EAGAIN
            bounced += 1
    assert bounced > 0 and len(tickets) >= 1
    ctx.drain()
    outs = [ctx.poll(t) for t in tickets]
    assert all(o[0] == 1 for o in outs)
    for o in outs[1:]:
        assert np.array_equal(o[2][0], outs[0][2][0])
    with pytest.raises(bsm.BsmError) as e:
        ctx.poll(tickets[0])                   # reported once, then forgotten
    assert e.value.status == bsm.ENOTFOUND
    ctx.close()


def test_serve_invalid_arguments(torch_cuda, bsm, orc):
    _say("case: serving argument validation")
    ctx, _ = _ctx(bsm, orc, 256, 15)
    img = np.zeros((20, 30, 3), np.uint8)
    with pytest.raises(bsm.BsmError) as e:
        ctx.submit(img, img, 31)               # dmax > W
    assert e.value.status == bsm.EINVAL
    with pytest.raises(bsm.BsmError) as e:
        ctx.serve_config(0, 1)
    assert e.value.status == bsm.EINVAL
    with pytest.raises(bsm.BsmError) as e:
        ctx.serve_config(1 << 30, 1, -1)
    assert e.value.status == bsm.EINVAL
    with pytest.raises(bsm.BsmError) as e:
        ctx.poll(99)
    assert e.value.status == bsm.ENOTFOUND
    ctx.close()


def test_serve_concurrent_clients(torch_cuda, bsm, orc):
    # several host threads submit and poll at once (the serving calls lock
    # internally); every result equals the single-pair path's
    import threading
    torch = torch_cuda
    _say("case: serving, 3 client threads x 6 pairs, n=256 S=15")
    ctx, _ = _ctx(bsm, orc, 256, 15)
    scenes = _scenes(6, 0.12, first=40)
    want = []
    for s in scenes:
        d, _ = ctx.match(torch.from_numpy(s.left).cuda(), torch.from_numpy(s.right).cuda(), s.dmax)
        want.append(d.cpu().numpy())
    errors = []

    def client(c):
        try:
            for rep in range(2):
                ts = [(j, ctx.submit(s.left, s.right, s.dmax)) for j, s in enumerate(scenes)]
                for j, t in ts:
                    state, _, (disp, _) = _wait(ctx, t)
                    if state != 1 or not np.array_equal(disp, want[j]):
                        errors.append((c, rep, j, state))
        except Exception as e:  # reported below
            errors.append((c, repr(e)))

    threads = [threading.Thread(target=client, args=(c,)) for c in range(3)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors[:5]
    st = ctx.serve_stats()
    assert st["completed"] == 36 and st["failed"] == 0
    ctx.close()
