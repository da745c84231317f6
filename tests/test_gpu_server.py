"""The serving loop (include/tt_server.h) on the GPU: requests from many
streams submitted as they arrive and run in continuous-batching waves on
several lanes give every stream bitwise the state of the same slices pushed
alone, in order; admission respects the per-stream order, the wave size and
the HBM budget; a non-finite slice is rejected for its own request only."""

import numpy as np
import pytest

from tests.gpu_util import say, to_device_slice, torch_cuda
from tests.test_gpu_batch import _mixed_members, _states_equal

pytestmark = pytest.mark.gpu


def _solo_runs(members, dev, order):
    from paper_2606_31061_amd import TTStream
    solo = [TTStream(st.modes, st.ranks, init=st.init(), compute=c) for st, c in members]
    for i, t in order:
        solo[i].push(dev[i][t])
    for s in solo:
        s.synchronize()
    return solo


@pytest.mark.parametrize("lanes,max_wave", [(1, 16), (3, 2)])
def test_server_matches_solo_runs(lanes, max_wave):
    torch = torch_cuda()
    from paper_2606_31061_amd import TTServer, TTStream
    T = 4
    members = _mixed_members(7, 6100 + lanes, T)
    say(f"server lanes={lanes} max_wave={max_wave}: 7 mixed streams x {T} slices")
    dev = [[to_device_slice(torch, X.astype(np.float32)) for X in st.frames(1, T)] for st, _ in members]
    rng = np.random.Generator(np.random.PCG64(lanes))
    # arrival order: interleaved, each stream's slices in order
    pending = {i: 0 for i in range(len(members))}
    order = []
    while any(pending[i] < T for i in pending):
        i = int(rng.choice([k for k in pending if pending[k] < T]))
        order.append((i, pending[i]))
        pending[i] += 1
    served = [TTStream(st.modes, st.ranks, init=st.init(), compute=c) for st, c in members]
    sv = TTServer(max_wave=max_wave, lanes=lanes,
                  hbm_budget=3 * max(st.n_elems for st, _ in members) * 4)
    ids = [sv.add(s) for s in served]
    for k, (i, t) in enumerate(order):
        sv.submit(ids[i], dev[i][t], tag=k)
        if k % 3 == 0:
            sv.poll()
    sv.drain()
    res = sv.take()
    assert sorted(r[0] for r in res) == list(range(len(order)))
    assert all(r[2] == 0 for r in res) and all(r[1] > 0 for r in res)
    # a stream's requests finish in submission order
    pos = {r[0]: j for j, r in enumerate(res)}
    for i in range(len(members)):
        mine = [k for k, (q, _) in enumerate(order) if q == i]
        assert [pos[k] for k in mine] == sorted(pos[k] for k in mine)
    st = sv.stats()
    assert st["retired"] == len(order) and st["queued"] == 0 and st["in_flight"] == 0
    assert st["peak_bytes"] <= 3 * max(s.n_elems for s, _ in members) * 4
    solo = _solo_runs(members, dev, order)
    for a, b in zip(solo, served):
        assert _states_equal(a, b)
    sv.close()


def test_server_rejects_nonfinite_request_only():
    torch = torch_cuda()
    from paper_2606_31061_amd import TTServer, TTStream
    T = 3
    members = _mixed_members(3, 7100, T)
    say("server non-finite request")
    dev = [[to_device_slice(torch, X.astype(np.float32)) for X in st.frames(1, T)] for st, _ in members]
    bad = dev[1][1].clone()
    bad[3] = float("inf")
    served = [TTStream(st.modes, st.ranks, init=st.init(), compute=c) for st, c in members]
    sv = TTServer(max_wave=8, lanes=2)
    ids = [sv.add(s) for s in served]
    tag = 0
    for t in range(T):
        for i in range(3):
            sv.submit(ids[i], bad if (i == 1 and t == 1) else dev[i][t], tag=100 * i + t)
            tag += 1
        sv.poll()
    sv.drain()
    res = {r[0]: r[2] for r in sv.take()}
    assert res == {100 * i + t: int(i == 1 and t == 1) for i in range(3) for t in range(T)}
    order = [(i, t) for t in range(T) for i in range(3) if not (i == 1 and t == 1)]
    solo = _solo_runs(members, dev, order)
    for a, b in zip(solo, served):
        assert _states_equal(a, b)
    assert [s.time() for s in served] == [3, 2, 3]
    sv.close()
