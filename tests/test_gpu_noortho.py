"""The "w/o Ortho" ablation (TT_FLAG_NO_ORTHO) on the GPU against its FP64
oracle (oracle/noortho.py), bitwise equality of batched and solo ablation
streams, and the ablation's reconstruction error over a longer stream next to
the proposed method's."""

import numpy as np
import pytest

from oracle import noortho, ttals
from tests.gpu_util import say, to_device_slice, torch_cuda
from ttgen import exact_tt_stream

pytestmark = pytest.mark.gpu

CASES = [((32, 32), (4, 4)), ((20, 18, 3), (6, 6, 3)), ((6, 5, 4, 3), (3, 4, 4, 2)), ((9,), (4,)),
         ((60, 80, 3), (8, 8, 3))]
# Distance allowed to the FP64 oracle, relative to ||X||.  The slice
# contractions run in FP32 against FP32 copies of the unnormalised right
# interface; the Gram solve amplifies their rounding by up to the condition
# number of B_k B_k^T (below about 1e3 on these short streams), so the FP32
# path's 1e-5 becomes 1e-4 here.
M_TOL_NOORTHO = 1e-4


@pytest.mark.parametrize("modes,ranks", CASES)
def test_noortho_stream_matches_oracle(modes, ranks):
    torch = torch_cuda()
    from paper_2606_31061_amd import TTStream
    st = exact_tt_stream(modes, ranks, ranks, 8, 71, 72, sigma=1e-2)
    init = st.init()
    xs = list(st.frames(1, st.T))
    say(f"no-ortho stream {modes} r{ranks}")
    ref = noortho.run_stream_noortho(xs, init[0], init[1], keep_M=True)
    s = TTStream(st.modes, st.ranks, init=init, no_ortho=True)
    worst = 0.0
    for X, info in zip(xs, ref.infos):
        s.push(to_device_slice(torch, X))
        M = s.reconstruct()
        worst = max(worst, float(np.linalg.norm(M - info.M) / np.linalg.norm(X)))
    print(f"[no-ortho parity] {modes} r{ranks}: max rel. distance {worst:.2e}")
    assert worst <= M_TOL_NOORTHO
    cores, g, t = s.get_state()
    assert t == len(xs)
    s.close()


def test_noortho_batch_bitwise_equal_to_solo():
    torch = torch_cuda()
    from paper_2606_31061_amd import TTBatch, TTStream
    sts = [exact_tt_stream((20, 18, 3), (6, 6, 3), (6, 6, 3), 3, 81 + q, 91 + q, sigma=1e-2) for q in range(2)]
    sts.append(exact_tt_stream((32, 32), (4, 4), (4, 4), 3, 99, 100, sigma=1e-2))
    say("no-ortho batch of 3")
    solo = [TTStream(st.modes, st.ranks, init=st.init(), no_ortho=True) for st in sts]
    mem = [TTStream(st.modes, st.ranks, init=st.init(), no_ortho=True) for st in sts]
    b = TTBatch(mem)
    dev = [[to_device_slice(torch, X) for X in st.frames(1, 3)] for st in sts]
    for t in range(3):
        for s, d in zip(solo, dev):
            s.push(d[t])
        b.push([d[t] for d in dev])
    assert b.synchronize() == [0, 0, 0]
    for x, y in zip(solo, mem):
        cx, gx, tx = x.get_state()
        cy, gy, ty = y.get_state()
        assert tx == ty == 3 and all(np.array_equal(p, q) for p, q in zip(cx, cy)) and np.array_equal(gx, gy)
    b.close()


def test_noortho_error_over_a_long_stream():
    """Both variants over 200 slices of a drifting stream, each against its
    own FP64 oracle on the same slices (the proposed method against
    oracle/ttals.py at the FP32-path tolerance, the ablation against
    oracle/noortho.py at M_TOL_NOORTHO), slice by slice; the RE curves of the
    four runs are printed side by side."""
    torch = torch_cuda()
    from paper_2606_31061_amd import TTStream
    st = exact_tt_stream((40, 36, 3), (8, 8, 3), (8, 8, 3), 200, 111, 112, sigma=1e-2, walk_step=0.2)
    init = st.init()
    xs = list(st.frames(1, st.T))
    say("no-ortho long stream (40,36,3) r(8,8,3), 200 slices: both oracles")
    ref_a = ttals.run_stream(xs, init[0], init[1], keep_M=True)
    ref_b = noortho.run_stream_noortho(xs, init[0], init[1], keep_M=True)
    say("no-ortho long stream: GPU runs")
    a = TTStream(st.modes, st.ranks, init=init)
    b = TTStream(st.modes, st.ranks, init=init, no_ortho=True)
    ea, eb, da, db = [], [], [], []
    for X, ia, ib in zip(xs, ref_a.infos, ref_b.infos):
        d = to_device_slice(torch, X)
        a.push(d)
        b.push(d)
        Ma, Mb = a.reconstruct(), b.reconstruct()
        xn = np.linalg.norm(X)
        ea.append(np.linalg.norm(X - Ma))
        eb.append(np.linalg.norm(X - Mb))
        da.append(np.linalg.norm(Ma - ia.M) / xn)
        db.append(np.linalg.norm(Mb - ib.M) / xn)
    ea, eb = np.array(ea), np.array(eb)
    xn = ref_a.Xnorm
    for t in (1, 5, 10, 50, 100, 200):
        print(f"[ablation] t={t:3d}: RE with ortho gpu {ea[t-1]/xn[t-1]:.5f} oracle {ref_a.E[t-1]/xn[t-1]:.5f}; "
              f"without gpu {eb[t-1]/xn[t-1]:.5f} oracle {ref_b.E[t-1]/xn[t-1]:.5f}")
    print(f"[ablation] stream RE: with ortho gpu {np.sqrt(np.sum(ea**2)/np.sum(xn**2)):.6f} oracle {ref_a.re:.6f}; "
          f"without gpu {np.sqrt(np.sum(eb**2)/np.sum(xn**2)):.6f} oracle {ref_b.re:.6f}; "
          f"max |dM|/|X| {max(da):.2e} / {max(db):.2e}")
    assert max(da) <= 1e-5, max(da)
    assert max(db) <= M_TOL_NOORTHO, max(db)
    re_a = np.sqrt(np.sum(ea ** 2) / np.sum(xn ** 2))
    assert abs(re_a - ref_a.re) <= 1e-5 * ref_a.re
    a.close()
    b.close()
