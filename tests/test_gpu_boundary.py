"""Boundary behaviour of the C ABI on the GPU: the allocator hook, allocation
failure, use after destroy, the temporal-core history against the oracle, and
the rules for streams registered with a server."""

import numpy as np
import pytest

from oracle import ttals
from tests.gpu_util import say, to_device_slice, torch_cuda
from ttgen import config_c1, exact_tt_stream

pytestmark = pytest.mark.gpu


class _TorchAllocator:
    """Device blocks from PyTorch's caching allocator, with a ledger."""

    def __init__(self, torch, fail_after=None):
        self.torch = torch
        self.live = {}
        self.calls = 0
        self.fail_after = fail_after

    def alloc(self, n):
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            return 0
        t = self.torch.empty(n, dtype=self.torch.uint8, device="cuda")
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def free(self, p):
        assert p in self.live, "free of a block the allocator did not hand out"
        del self.live[p]


def test_allocator_hook_serves_every_device_block():
    torch = torch_cuda()
    from paper_2606_31061_amd import TTStream, binding
    st = config_c1(T=12)
    init = st.init()
    xs = list(st.frames(1, st.T))
    say("allocator hook: c1 stream with a torch-backed allocator")
    ledger = _TorchAllocator(torch)
    al = binding.make_allocator(ledger.alloc, ledger.free)
    a = TTStream(st.modes, st.ranks, init=init, allocator=al)
    b = TTStream(st.modes, st.ranks, init=init)
    n_create = len(ledger.live)
    assert n_create > 0
    assert sum(t.numel() for t in ledger.live.values()) >= a.info()["device_bytes"] > 0
    for X in xs:
        a.push(X)                       # host slices: the staging block comes from the hook too
        b.push(X)
    Ma, Mb = a.reconstruct(), b.reconstruct()
    assert len(ledger.live) > n_create  # staging and reconstruction buffers
    ca, ga, _ = a.get_state()
    cb, gb, _ = b.get_state()
    assert all(np.array_equal(p, q) for p, q in zip(ca, cb)) and np.array_equal(ga, gb)
    assert np.array_equal(Ma, Mb)
    a.close()
    b.close()
    assert ledger.live == {}            # every block returned at destroy


def test_allocator_failure_is_oom_and_frees_what_was_taken():
    torch = torch_cuda()
    from paper_2606_31061_amd import TTStream, binding
    st = config_c1(T=2)
    say("allocator hook failing on its fourth call")
    ledger = _TorchAllocator(torch, fail_after=3)
    al = binding.make_allocator(ledger.alloc, ledger.free)
    with pytest.raises(binding.TTError) as e:
        TTStream(st.modes, st.ranks, init=st.init(), allocator=al)
    assert e.value.status == binding.TT_ERR_OOM
    assert ledger.calls == 4 and ledger.live == {}


def test_absurd_allocation_is_oom():
    torch_cuda()
    from paper_2606_31061_amd import TTStream, binding
    st = config_c1(T=2)
    say("history ring of 2^40 rows (32 TiB) must fail as OOM")
    with pytest.raises(binding.TTError) as e:
        TTStream(st.modes, st.ranks, init=st.init(), keep_history=True, history_capacity=1 << 40)
    assert e.value.status == binding.TT_ERR_OOM
    # the failed allocation leaves no error behind for the next launch to report
    s = TTStream(st.modes, st.ranks, init=st.init())
    s.push(next(st.frames(1, 1)))
    s.synchronize()
    s.close()


def test_use_after_destroy_is_invalid_arg():
    torch_cuda()
    from paper_2606_31061_amd import TTStream, binding
    st = config_c1(T=2)
    say("use after destroy")
    s = TTStream(st.modes, st.ranks, init=st.init())
    h = s._h
    s.close()
    lib = binding.load_library()
    assert lib.tt_stream_synchronize(h) == binding.TT_ERR_INVALID_ARG
    assert lib.tt_stream_push_slice(h, h, 1, 1) == binding.TT_ERR_INVALID_ARG
    assert lib.tt_stream_reconstruct(h, h, 0, 1) == binding.TT_ERR_INVALID_ARG
    assert lib.tt_stream_destroy(h) == binding.TT_ERR_INVALID_ARG


def test_history_rows_are_the_temporal_outputs_of_every_update():
    """Algorithm 1 outputs g_n[t] at every t.  On config 1's 200 slices the
    kept rows satisfy ||g_n[t]|| = ||M_t|| (the oracle's M_t) for every t and,
    as the oracle's g_n[t] (pin P8), each row is 1-sparse."""
    torch = torch_cuda()
    from paper_2606_31061_amd import TTStream
    st = config_c1()
    init = st.init()
    xs = list(st.frames(1, st.T))
    say("history ring: c1, 200 slices")
    ref = ttals.run_stream(xs, init[0], init[1], keep_M=True)
    s = TTStream(st.modes, st.ranks, init=init, keep_history=True, history_capacity=256)
    for X in xs:
        s.push(to_device_slice(torch, X))
    hist = s.history()
    assert hist.shape == (st.T, st.ranks[-1])
    for t, (row, info) in enumerate(zip(hist, ref.infos)):
        mn = np.linalg.norm(info.M)
        assert abs(np.linalg.norm(row) - mn) <= 1e-5 * info.Xnorm, t
        big = np.argmax(np.abs(row))
        rest = np.delete(row, big)
        assert np.max(np.abs(rest)) <= 1e-8 * mn, t
    # the oracle's final g agrees up to the sign of its one entry
    assert np.allclose(np.abs(hist[-1]), np.abs(ref.g), rtol=1e-5, atol=1e-8 * np.linalg.norm(ref.g))
    # a ring smaller than the stream keeps the latest rows
    s2 = TTStream(st.modes, st.ranks, init=init, keep_history=True, history_capacity=16)
    for X in xs[:40]:
        s2.push(to_device_slice(torch, X))
    h2 = s2.history()
    assert h2.shape == (16, st.ranks[-1])
    assert np.array_equal(h2, hist[24:40])
    # set_state restarts the history empty at the given t
    cores, g, _ = s2.get_state()
    s2.set_state(cores, g, 40)
    assert s2.history().shape[0] == 0
    s2.push(to_device_slice(torch, xs[40]))
    h3 = s2.history()
    assert h3.shape == (1, st.ranks[-1]) and np.array_equal(h3[0], hist[40])
    s.close()
    s2.close()


def test_server_registered_stream_rules():
    torch = torch_cuda()
    from paper_2606_31061_amd import TTBatch, TTServer, TTStream, binding
    sts = [exact_tt_stream((20, 18, 3), (6, 6, 3), (6, 6, 3), 4, 501 + q, 601 + q, sigma=1e-2) for q in range(3)]
    dev = [[to_device_slice(torch, X.astype(np.float32)) for X in st.frames(1, 4)] for st in sts]
    say("server: registered-stream rules")
    served = [TTStream(st.modes, st.ranks, init=st.init()) for st in sts]
    solo = [TTStream(st.modes, st.ranks, init=st.init()) for st in sts]
    sv = TTServer(max_wave=4, lanes=2)
    ids = [sv.add(s) for s in served]
    # direct pushes and batches of a registered stream are refused
    with pytest.raises(binding.TTError) as e:
        served[0].push(dev[0][0])
    assert e.value.status == binding.TT_ERR_STATE
    with pytest.raises(binding.TTError) as e:
        TTBatch([served[0]])
    assert e.value.status == binding.TT_ERR_STATE
    # state calls wait for the lanes: read right after poll() launched the wave
    for i in range(3):
        sv.submit(ids[i], dev[i][0], tag=i)
    sv.poll()
    for i in range(3):
        solo[i].push(dev[i][0])
        ca, ga, ta = served[i].get_state()
        cb, gb, tb = solo[i].get_state()
        assert ta == tb == 1 and np.array_equal(ga, gb) and all(np.array_equal(p, q) for p, q in zip(ca, cb))
    # destroying a registered stream drops its queued requests; its id is refused
    sv.submit(ids[1], dev[1][1], tag=10)
    sv.submit(ids[1], dev[1][2], tag=11)
    sv.submit(ids[2], dev[2][1], tag=12)
    served[1].close()
    with pytest.raises(binding.TTError) as e:
        sv.submit(ids[1], dev[1][3], tag=13)
    assert e.value.status == binding.TT_ERR_INVALID_ARG
    sv.drain()
    tags = sorted(r[0] for r in sv.take())
    assert 11 not in tags and 12 in tags
    # after the server is destroyed the streams are their own again
    sv.close()
    served[2].push(dev[2][2])
    solo[2].push(dev[2][1])
    solo[2].push(dev[2][2])
    assert np.array_equal(served[2].get_state()[1], solo[2].get_state()[1])
    for s in served[::2] + solo:
        s.close()


def test_wait_update_returns_the_committed_result():
    """tt_stream_wait_update: after it returns, the pushed update's result is
    committed (the next update's preparation may still run); the push to commit
    device time is reported and does not exceed push to all work."""
    torch = torch_cuda()
    from paper_2606_31061_amd import TTStream
    st = config_c1(T=6)
    init = st.init()
    xs = list(st.frames(1, st.T))
    say("wait_update on c1")
    ref = ttals.run_stream(xs, init[0], init[1], keep_M=True)
    s = TTStream(st.modes, st.ranks, init=init)
    s.wait_update()                     # nothing pushed yet: returns at once
    for X, info in zip(xs, ref.infos):
        s.push(to_device_slice(torch, X))
        s.wait_update()
        assert s.last_push_ms() > 0.0
        M = s.reconstruct()
        assert np.linalg.norm(M - info.M) <= 1e-5 * np.linalg.norm(X)
    assert s.time() == len(xs)
    s.close()
