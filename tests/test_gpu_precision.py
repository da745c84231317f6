"""Precision of the two contraction variants per configuration (the precision
study of the BF16 variant): the stream's relative error RE = sqrt(sum_t
E_t^2 / sum_t ||X_t||^2) from the GPU path with FP32 and with BF16 slice
contractions, against the FP64 oracle on the same slices and initial cores.

Each case prints one line `[precision] config ... RE_oracle ... dRE_f32 ...
dRE_bf16 ...` (the deviation |RE_gpu - RE_oracle|) and asserts the bounds:
FP32 within 1e-5 of the oracle's error, relative (|RE_f32 - RE_oracle| <=
1e-5 RE_oracle: FP32 slices and interfaces, FP64 chain), BF16 within
RE_TOL_BF16 absolute (the slice and the interface rounded to BF16 at 2^-9
relative per entry)."""

import sys

import numpy as np
import pytest

from oracle import ttals
from tests.gpu_util import say, to_device_slice, torch_cuda
from ttgen import config_c1, config_c2, config_c3

pytestmark = pytest.mark.gpu

RE_TOL_F32 = 1e-5      # relative to the oracle's RE
RE_TOL_BF16 = 3e-3     # absolute

CASES = {
    # config: (spec factory, slices)
    "c1_order3_32x32_r4": (lambda: config_c1(T=200), 200),
    "c2_order4_240x320x3_r16": (lambda: config_c2(T=1000), 40),
    "c3_order9_1080x1920x3_r32": (lambda: config_c3(T=500), 20),
}


def _gpu_re(torch, spec, init, xs, compute):
    from paper_2606_31061_amd import TTStream
    s = TTStream(spec.modes, spec.ranks, init=init, compute=compute)
    dt = torch.bfloat16 if compute == "bf16" else torch.float32
    e2 = 0.0
    for X in xs:
        s.push(to_device_slice(torch, np.asarray(X, dtype=np.float32), dt))
        M = s.reconstruct()
        e2 += float(np.sum(np.square(np.asarray(X, dtype=np.float64) - M)))
    s.synchronize()
    s.close()
    return e2


@pytest.mark.parametrize("config", list(CASES))
def test_precision_per_config(config):
    torch = torch_cuda()
    make, T = CASES[config]
    spec = make()
    init = spec.init()
    xs = list(spec.frames(1, T))
    say(f"precision {config}: {T} slices, oracle then FP32 and BF16 contractions")
    res = ttals.run_stream(xs, init[0], init[1])
    xn2 = float(np.sum(np.square(res.Xnorm)))
    re_or = float(res.re)
    re_f32 = float(np.sqrt(_gpu_re(torch, spec, init, xs, "f32") / xn2))
    re_bf16 = float(np.sqrt(_gpu_re(torch, spec, init, xs, "bf16") / xn2))
    d32, d16 = abs(re_f32 - re_or), abs(re_bf16 - re_or)
    print(f"[precision] config {config} slices {T} RE_oracle {re_or:.6e} RE_f32 {re_f32:.6e} "
          f"dRE_f32 {d32:.2e} (rel {d32 / re_or:.2e}) RE_bf16 {re_bf16:.6e} dRE_bf16 {d16:.2e}", file=sys.stderr, flush=True)
    assert d32 <= RE_TOL_F32 * re_or, (config, re_f32, re_or, d32 / re_or)
    assert d16 <= RE_TOL_BF16, (config, re_bf16, re_or)
