"""The launch-shape tuner of the slice passes (TT_FLAG_AUTOTUNE): tuned
streams follow the FP64 oracle as untuned ones do, streams of one shape share
the tuned plan (bitwise equal alone and batched), and a tuned and an untuned
stream of one shape run different plans, so a batch keeps them apart."""

import numpy as np
import pytest

from oracle import ttals
from tests.gpu_util import rel, say, to_device_slice, torch_cuda
from ttgen import exact_tt_stream

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_tuned_stream_matches_oracle(compute):
    torch = torch_cuda()
    from paper_2606_31061_amd import TTStream
    st = exact_tt_stream((48, 40, 3), (8, 8, 3), (8, 8, 3), 8, 1201, 2201, sigma=1e-2)
    init = st.init()
    xs = list(st.frames(1, st.T))
    say(f"tuned stream (48,40,3) {compute}")
    s = TTStream(st.modes, st.ranks, init=init, compute=compute, autotune=True)
    res = ttals.run_stream(xs, init[0], init[1], keep_M=True)
    dt = torch.bfloat16 if compute == "bf16" else torch.float32
    for X, info in zip(xs, res.infos):
        s.push(to_device_slice(torch, X, dt))
        M = s.reconstruct()
        tol = 1e-5 if compute == "f32" else 2e-2
        assert rel(M, info.M, np.linalg.norm(X)) <= tol
    s.close()


def test_tuned_streams_batch_bitwise_and_groups():
    torch = torch_cuda()
    from paper_2606_31061_amd import TTBatch, TTStream
    T = 3
    sts = [exact_tt_stream((48, 40, 3), (8, 8, 3), (8, 8, 3), T, 1300 + q, 1400 + q, sigma=1e-2) for q in range(3)]
    say("tuned batch of 3 plus an untuned member")
    solo = [TTStream(st.modes, st.ranks, init=st.init(), autotune=True) for st in sts]
    members = [TTStream(st.modes, st.ranks, init=st.init(), autotune=True) for st in sts]
    untuned = TTStream(sts[0].modes, sts[0].ranks, init=sts[0].init())
    batch = TTBatch(members + [untuned])
    info = batch.info()
    assert info["streams"] == 4
    dev = [[to_device_slice(torch, X) for X in st.frames(1, T)] for st in sts]
    for t in range(T):
        for s, xs in zip(solo, dev):
            s.push(xs[t])
        batch.push([xs[t] for xs in dev] + [dev[0][t]])
    assert batch.synchronize() == [0, 0, 0, 0]
    for a, b in zip(solo, members):
        ca, ga, ta = a.get_state()
        cb, gb, tb = b.get_state()
        assert ta == tb == T
        assert all(np.array_equal(x, y) for x, y in zip(ca, cb)) and np.array_equal(ga, gb)
    # the untuned member still follows the tuned solo run to FP32 accuracy
    cu, gu, _ = untuned.get_state()
    c0, g0, _ = solo[0].get_state()
    M_u = ttals.reconstruct(cu, gu)
    M_0 = ttals.reconstruct(c0, g0)
    assert np.linalg.norm(M_u - M_0) <= 1e-5 * np.linalg.norm(M_0)
    batch.close()


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_pass_profile_times_the_passes(compute):
    """TT_FLAG_PROFILE_OPS: the slice passes' events give positive times, the
    contraction kernel alone no longer than its whole pass, and neither
    profiling nor the back-to-back pass timer changes the updates (bitwise
    equal to an unprofiled stream)."""
    torch = torch_cuda()
    from paper_2606_31061_amd import TTStream
    st = exact_tt_stream((48, 40, 3), (8, 8, 3), (8, 8, 3), 2, 1501, 1601, sigma=1e-2)
    dt = torch.bfloat16 if compute == "bf16" else torch.float32
    xs = [to_device_slice(torch, X, dt) for X in st.frames(1, 2)]
    say(f"pass profile {compute}")
    a = TTStream(st.modes, st.ranks, init=st.init(), compute=compute, profile_ops=True)
    b = TTStream(st.modes, st.ranks, init=st.init(), compute=compute)
    for x in xs:
        a.push(x)
        b.push(x)
        p = a.pass_profile()
        assert set(p) == {"pass1_kernel", "pass1", "pass2_kernel", "pass2"}
        assert 0.0 < p["pass1_kernel"] <= p["pass1"] and 0.0 < p["pass2_kernel"] <= p["pass2"]
    # timing the pass kernels back to back leaves the state and the next
    # update unchanged
    t = a.time_passes(xs, reps=3)
    assert set(t) == {"pass1_kernel", "pass1_reduce", "pass2_kernel", "pass2_reduce"}
    assert t["pass1_kernel"] > 0.0 and t["pass2_kernel"] > 0.0
    a.push(xs[1])
    b.push(xs[1])
    ca, ga, _ = a.get_state()
    cb, gb, _ = b.get_state()
    assert all(np.array_equal(x, y) for x, y in zip(ca, cb)) and np.array_equal(ga, gb)
    a.close()
    b.close()


def test_tuner_picks_the_split_point_per_shape():
    """With split_point = 0 the tuner picks k* among the modelled candidates;
    two streams of one shape get the same k* (cached pass times), and an
    explicit split point is kept."""
    torch_cuda()
    from paper_2606_31061_amd import TTStream
    st = exact_tt_stream((24, 20, 16, 3), (6, 8, 6, 3), (6, 8, 6, 3), 2, 1701, 1801, sigma=1e-2)
    say("tuned split point (24,20,16,3)")
    a = TTStream(st.modes, st.ranks, init=st.init(), autotune=True)
    b = TTStream(st.modes, st.ranks, init=st.init(), autotune=True)
    c = TTStream(st.modes, st.ranks, init=st.init(), autotune=True, split_point=1)
    ka, kb = a.info()["split_point"], b.info()["split_point"]
    assert ka == kb and 1 <= ka <= len(st.modes)
    assert c.info()["split_point"] == 1
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("compute", ["f32", "bf16"])
@pytest.mark.parametrize("autotune", [False, True])
def test_pass_kernel_names_follow_the_plan(compute, autotune):
    """The library names the contraction kernels its passes launch: FP32
    streams k_pass1 and k_pass2g (FP32 slices, 4 <= P <= 1280, r <= 32) or
    k_pass2; BF16 streams k_pass1b and, for pass 2, the
    LDS-staged k_pass2s by default where P % 8 == 0 and P <= 2304 (the tuner
    may pick either BF16 kernel)."""
    torch_cuda()
    from paper_2606_31061_amd import TTStream
    modes, ranks = (16, 18, 10), (4, 4, 4)
    say(f"pass kernel names {compute} autotune={autotune}")
    s = TTStream(modes, ranks, seed=3, compute=compute, autotune=autotune)
    k1, k2 = s.pass_kernels()
    sp = s.info()["split_point"]
    s.close()
    P = int(np.prod(modes[:sp]))
    if compute == "f32":
        # every rank here is 4: the grouped pass 2 applies where 4 <= P <= 1280
        assert (k1, k2) == ("k_pass1", "k_pass2g" if 4 <= P <= 1280 else "k_pass2")
    else:
        assert k1 == "k_pass1b"
        if autotune:
            assert k2 in ("k_pass2b", "k_pass2s")
            if P % 8 != 0:
                assert k2 == "k_pass2b"
        else:
            assert k2 == ("k_pass2s" if P % 8 == 0 and P <= 2304 else "k_pass2b")
