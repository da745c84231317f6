"""Batches of streams (include/tt_batch.h) on the GPU: every member of a batch
is computed exactly as when pushed alone (bitwise equal state), members of
different shapes form separate groups, a non-finite slice is rejected for its
own stream only, and batched results match the FP64 oracle."""

import numpy as np
import pytest

from oracle import ttals
from tests.gpu_util import say, to_device_slice, torch_cuda, rel
from ttgen import exact_tt_stream, config_c3

pytestmark = pytest.mark.gpu

M_TOL = 1e-5


def _members(shapes, T, seed0=100):
    out = []
    for q, (modes, ranks) in enumerate(shapes):
        st = exact_tt_stream(modes, ranks, ranks, T, seed0 + 2 * q, seed0 + 2 * q + 1, sigma=1e-2)
        init = st.init()
        out.append((st, init, list(st.frames(1, T))))
    return out


def _states_equal(a, b):
    ca, ga, ta = a.get_state()
    cb, gb, tb = b.get_state()
    return ta == tb and all(np.array_equal(x, y) for x, y in zip(ca, cb)) and np.array_equal(ga, gb)


def _run_alone_and_batched(torch, members, T):
    from paper_2606_31061_amd import TTBatch, TTStream
    alone = [TTStream(st.modes, st.ranks, init=init) for st, init, _ in members]
    batched = [TTStream(st.modes, st.ranks, init=init) for st, init, _ in members]
    batch = TTBatch(batched)
    dev = [[to_device_slice(torch, X) for X in xs] for _, _, xs in members]
    for t in range(T):
        for s, xs in zip(alone, dev):
            s.push(xs[t])
        batch.push([xs[t] for xs in dev])
    assert batch.synchronize() == [0] * len(members)
    for s in alone:
        s.synchronize()
    return alone, batched, batch


def test_same_shape_batch_is_bitwise_equal_to_solo_runs():
    torch = torch_cuda()
    T = 6
    members = _members([((24, 20, 3), (4, 4, 3))] * 5, T)
    say("batch: 5 streams of (24,20,3) r=(4,4,3)")
    alone, batched, batch = _run_alone_and_batched(torch, members, T)
    assert batch.info() == {"streams": 5, "groups": 1}
    for a, b in zip(alone, batched):
        assert _states_equal(a, b)
    # and the batched reconstructions follow the oracle
    for (st, init, xs), s in zip(members, batched):
        ref = ttals.run_stream(xs, init[0], init[1], keep_M=True)
        assert rel(s.reconstruct(), ref.infos[-1].M, np.linalg.norm(xs[-1])) <= M_TOL
    batch.close()


def test_mixed_shapes_form_groups_and_match_solo_runs():
    torch = torch_cuda()
    T = 5
    shapes = [((32, 32), (4, 4)), ((12, 10, 3), (4, 4, 3)), ((32, 32), (4, 4)),
              ((6, 5, 4, 3), (3, 4, 4, 2)), ((12, 10, 3), (4, 4, 3)), ((9,), (4,))]
    members = _members(shapes, T, seed0=300)
    say("batch: 6 streams in 4 shape groups")
    alone, batched, batch = _run_alone_and_batched(torch, members, T)
    assert batch.info() == {"streams": 6, "groups": 4}
    for a, b in zip(alone, batched):
        assert _states_equal(a, b)
    batch.close()


def test_full_size_order9_batch_matches_solo_runs():
    torch = torch_cuda()
    from paper_2606_31061_amd import TTBatch, TTStream
    st = config_c3(T=3)
    init = st.init()
    xs = [to_device_slice(torch, X) for X in st.frames(1, 3)]
    say("batch: 2 config-3 streams (order 9, 6.2M-element slices)")
    a = TTStream(st.modes, st.ranks, init=init)
    b1 = TTStream(st.modes, st.ranks, init=init)
    b2 = TTStream(st.modes, st.ranks, init=init)
    batch = TTBatch([b1, b2])
    for t in range(3):
        a.push(xs[t])
        batch.push([xs[t], xs[(t + 1) % 3]])
    assert batch.synchronize() == [0, 0]
    a.synchronize()
    assert _states_equal(a, b1)
    batch.close()


def test_nonfinite_slice_is_rejected_for_its_member_only():
    torch = torch_cuda()
    from paper_2606_31061_amd import TTBatch, TTStream
    T = 3
    members = _members([((24, 20, 3), (4, 4, 3))] * 3, T, seed0=500)
    say("batch: non-finite slice in member 1")
    streams = [TTStream(st.modes, st.ranks, init=init) for st, init, _ in members]
    solo = [TTStream(st.modes, st.ranks, init=init) for st, init, _ in members]
    batch = TTBatch(streams)
    dev = [[to_device_slice(torch, X) for X in xs] for _, _, xs in members]
    bad = dev[1][1].clone()
    bad[7] = float("nan")
    batch.push([d[0] for d in dev])
    batch.push([dev[0][1], bad, dev[2][1]])
    rej = batch.synchronize()
    assert rej == [0, 1, 0]
    for i, s in enumerate(solo):
        s.push(dev[i][0])
        if i != 1:
            s.push(dev[i][1])
        s.synchronize()
    for a, b in zip(solo, streams):
        assert _states_equal(a, b)
    assert [s.time() for s in streams] == [2, 1, 2]
    batch.close()


def _mixed_members(n, seed, T, max_elems=60000, noise_rel=None):
    """Streams of uneven order (3-5), mode sizes and ranks ({4,8,16,32},
    clamped to feasibility), low rank plus noise (sigma 1e-2, or noise_rel
    times the signal's RMS); every third member uses BF16 contractions."""
    from paper_2606_31061_amd.binding import tt_clamp_ranks
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < n:
        order = int(rng.integers(3, 6))
        hi = {3: 200, 4: 40, 5: 16}[order]
        modes = tuple(int(v) for v in rng.integers(4, hi + 1, order - 1))
        if int(np.prod(modes)) > max_elems:
            continue
        rank = int(rng.choice([4, 8, 16, 32]))
        ranks = tuple(int(v) for v in tt_clamp_ranks(modes, [rank] * len(modes)))
        q = len(out)
        st = exact_tt_stream(modes, ranks, ranks, T, seed + 10 * q, seed + 10 * q + 1, sigma=1e-2,
                             noise_rel=noise_rel)
        out.append((st, "bf16" if q % 3 == 2 else "f32"))
    return out


def test_heterogeneous_batch_is_bitwise_equal_to_solo_runs():
    torch = torch_cuda()
    from paper_2606_31061_amd import TTBatch, TTStream
    T = 3
    members = _mixed_members(10, 4100, T)
    say("heterogeneous batch of 10 streams, orders 3-5, f32 and bf16 contractions: "
        + "; ".join(f"{st.modes} r{st.ranks} {c}" for st, c in members))
    solo = [TTStream(st.modes, st.ranks, init=st.init(), compute=c) for st, c in members]
    batched = [TTStream(st.modes, st.ranks, init=st.init(), compute=c) for st, c in members]
    batch = TTBatch(batched)
    assert batch.info()["streams"] == 10
    dev = [[to_device_slice(torch, X.astype(np.float32)) for X in st.frames(1, T)] for st, _ in members]
    for t in range(T):
        for s, xs in zip(solo, dev):
            s.push(xs[t])
        batch.push([xs[t] for xs in dev])
    assert batch.synchronize() == [0] * 10
    for s in solo:
        s.synchronize()
    for a, b in zip(solo, batched):
        assert _states_equal(a, b)
    # the FP32 members follow the oracle
    for (st, c), s in zip(members, batched):
        if c != "f32":
            continue
        xs = [X.astype(np.float32).astype(np.float64) for X in st.frames(1, T)]
        init = st.init()
        ref = ttals.run_stream(xs, init[0], init[1], keep_M=True)
        assert rel(s.reconstruct(), ref.infos[-1].M, np.linalg.norm(xs[-1])) <= M_TOL
    batch.close()


def test_graph_replay_matches_eager_batch():
    """Pushes replayed from captured HIP graphs give bitwise the eager
    batch's states after every push, with eager work and synchronisation
    between the replays, across more pushes than there are descriptor slots
    and with a change of slice dtype (which recaptures)."""
    torch = torch_cuda()
    from paper_2606_31061_amd import TTBatch, TTStream
    T = 11
    members = _mixed_members(5, 5100, T)
    say("graph replay: 5 mixed streams, 11 pushes")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        eager = [TTStream(st.modes, st.ranks, init=st.init(), compute=c) for st, c in members]
        graphed = [TTStream(st.modes, st.ranks, init=st.init(), compute=c) for st, c in members]
        be = TTBatch(eager)
        bg = TTBatch(graphed, graph=True)
        dev = [[to_device_slice(torch, X.astype(np.float32)) for X in st.frames(1, T)] for st, _ in members]
        for t in range(T):
            xs = [d[t] if t != 7 else d[t].to(torch.float64) for d in dev]
            be.push(xs)
            bg.push(xs)
            assert be.synchronize() == [0] * 5 and bg.synchronize() == [0] * 5
            for a, b in zip(eager, graphed):
                assert _states_equal(a, b), t
            # eager work on the same stream between replays
            _ = (dev[0][t] * 2.0).sum().item()
        be.close()
        bg.close()


def test_wave_plan_streams_are_bitwise_equal_alone_and_batched():
    """TT_FLAG_WAVE_PLAN moves products of 2e5..4e5 multiply-adds from
    whole-GPU launches into the chain segments (config 3 has such a product,
    so the chain runs more operations); a stream with the flag gives the
    same bits alone and in a batch, and follows the oracle."""
    torch = torch_cuda()
    from paper_2606_31061_amd import TTBatch, TTStream
    st = config_c3(T=3)
    init = st.init()
    frames = list(st.frames(1, 3))
    xs = [to_device_slice(torch, X) for X in frames]
    say("batch: config-3 streams with the wave plan")
    counts = []
    for wave in (False, True):
        p = TTStream(st.modes, st.ranks, init=init, profile_ops=True, wave_plan=wave)
        p.push(xs[0])
        p.synchronize()
        counts.append(len(p.op_profile()))
        p.close()
    assert counts[1] > counts[0], counts
    a = TTStream(st.modes, st.ranks, init=init, wave_plan=True)
    b1 = TTStream(st.modes, st.ranks, init=init, wave_plan=True)
    b2 = TTStream(st.modes, st.ranks, init=init, wave_plan=True)
    batch = TTBatch([b1, b2])
    for t in range(3):
        a.push(xs[t])
        batch.push([xs[t], xs[(t + 1) % 3]])
    assert batch.synchronize() == [0, 0]
    a.synchronize()
    assert _states_equal(a, b1)
    ref = ttals.run_stream(frames, init[0], init[1], keep_M=True)
    assert rel(a.reconstruct(), ref.infos[-1].M, np.linalg.norm(frames[-1])) <= M_TOL
    batch.close()
    for s in (a, b1, b2):
        s.close()


def test_wave_plan_large_products_match_the_oracle():
    """A stream planned for batched waves whose right interface and tail
    contraction are 7,328 x 77 x 32 products (whole-GPU products with four
    outputs per thread) agrees with the oracle slice by slice, as the default
    plan does."""
    torch = torch_cuda()
    from paper_2606_31061_amd import TTStream
    modes, ranks = (40, 229, 77), (32, 32, 32)
    st = exact_tt_stream(modes, ranks, ranks, 6, 11, 12, sigma=1e-2)
    init = st.init()
    slices = list(st.frames(1, 6))
    ref = ttals.run_stream(slices, init[0], init[1], keep_M=True)
    for wave_plan in (False, True):
        say(f"large products: wave_plan={wave_plan}")
        s = TTStream(modes, ranks, init=init, split_point=1, wave_plan=wave_plan)
        worst = 0.0
        for X, info in zip(slices, ref.infos):
            s.push(to_device_slice(torch, X))
            worst = max(worst, rel(s.reconstruct(), info.M, np.linalg.norm(X)))
        s.close()
        assert worst <= M_TOL, (wave_plan, worst)
