"""Benchmark of the Online TT-ALS per-slice update on one MI355X.

One step = one update (Algorithm 1's loop body) of one stream with one new
slice, through the C ABI (tt_stream_push_slice).  Workload (default): the
high-order stream of 1080x1920x3 FP32 frames read as the order-9 slice
(8,9,15,8,16,15,3,1,1), 6,220,800 entries, TT-ranks (8,32,...,32).  The
frames are synthetic (low TT-rank plus noise) and resident in HBM before the
timed region; a pool of distinct frames larger than the 256 MB Infinity Cache
is cycled so each update reads its slice from HBM.

Prints one JSON line: slice updates/s (value), the roofline of the dominant
slice-streaming kernel, per-slice latency p50/p99, and the FP64 oracle timed
on the host cores on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name: str, pool=None):
    from ttgen import config_c2, config_c3
    if name == "c3":
        return config_c3(T=500), pool or 24
    if name == "c2":
        return config_c2(T=1000), pool or 64
    raise SystemExit(f"unknown workload {name}")


def pass_bytes(P, J, r, xbytes=4):
    """Algorithmic HBM bytes of one pass-1 and one pass-2 launch (slice of
    xbytes per element; FP32 interfaces; FP64 outputs)."""
    p1 = xbytes * P * J + 4 * r * J + 8 * P * r  # read X, read B_{k*}, write Z (FP64)
    p2 = xbytes * P * J + 4 * P * r + 8 * r * J  # read X, read A_{k*+1}, write Y (FP64)
    return p1, p2


def time_passes_in_update(stream, pool, steps):
    """Average device times (ms) of the two slice passes inside the update:
    HIP events recorded on the update's stream around each pass and after its
    contraction kernel (the stream was created with profile_ops)."""
    acc = {}
    for i in range(steps):
        stream.push(pool[i % len(pool)])
        for key, ms in stream.pass_profile().items():
            acc.setdefault(key, []).append(ms)
    return {key: float(np.mean(v)) for key, v in acc.items()}


# rocprofv3 HBM counters of the contraction kernels (FETCH_SIZE and WRITE_SIZE
# per dispatch, scaled by the same counters on a copy kernel of known size),
# stored with a hash of the kernel source they were taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "slice_pass_traffic.json")
KERNEL_SOURCES = {"f32": "paper_2606_31061_amd/csrc/pass_kernels.hip", "bf16": "paper_2606_31061_amd/csrc/pass_bf16.hip"}


def measured_traffic(workload, compute, kernel):
    """HBM bytes per launch of `kernel` from the stored counters, or None when
    there are none for this workload or the kernel source changed since."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        with open(os.path.join(ROOT, KERNEL_SOURCES[compute]), "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if rec.get("workload") != workload or rec.get("compute") != compute or not k or k.get("source_sha256") != digest:
        return None
    return float(k["fetch_bytes"] + k["write_bytes"])


def batched_section(torch, n_streams, rounds, warmup, compute, tune):
    """The batched workload: n_streams streams of order 3-5 with uneven mode
    sizes and ranks, advanced together (one TTBatch push = one update of
    every stream) with graph replay, against the same streams pushed one by
    one through the single-stream path."""
    from paper_2606_31061_amd import TTBatch, TTStream, binding
    from ttgen import config_c4_streams
    nfr = 3  # frames per stream: the round's frame set (317 MB) exceeds the 256 MB Infinity Cache
    specs = config_c4_streams(n_streams, 1004, T=nfr, clamp=binding.tt_clamp_ranks, max_elems=1 << 21)
    orders = sorted(len(sp.modes) + 1 for sp in specs)
    elems = [sp.n_elems for sp in specs]
    log(f"batched workload: {n_streams} streams, orders {orders[0]}-{orders[-1]}, slices {min(elems)}-{max(elems)} "
        f"elements ({sum(elems) / 1e6:.1f} M per round)")
    side = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(side):
        frames = [[torch.from_numpy(np.ascontiguousarray(X.reshape(-1, order="F"))).cuda() for X in sp.frames(1, nfr)]
                  for sp in specs]
        if compute == "bf16":
            frames = [[x.to(torch.bfloat16) for x in f] for f in frames]
        bytes_round = 0
        for sp in specs:
            members = TTStream(sp.modes, sp.ranks, init=sp.init(), compute=compute, autotune=tune)
            k = members.info()["split_point"]
            members.close()
            P, J, r = int(np.prod(sp.modes[:k])), int(np.prod(sp.modes[k:])), sp.ranks[k - 1]
            b1, b2 = pass_bytes(P, J, r, 2 if compute == "bf16" else 4)
            bytes_round += b1 + b2

        def run(batch_graph, solo):
            # batch members are planned for waves (TT_FLAG_WAVE_PLAN); the
            # one-after-another baseline keeps the plan that is fastest alone
            streams = [TTStream(sp.modes, sp.ranks, init=sp.init(), compute=compute, autotune=tune,
                                wave_plan=not solo) for sp in specs]
            b = None if solo else TTBatch(streams, graph=batch_graph)

            def one(i):
                if solo:
                    for st, f in zip(streams, frames):
                        st.push(f[i % nfr])
                else:
                    b.push([f[i % nfr] for f in frames])

            def sync():
                if solo:
                    for st in streams:
                        st.synchronize()
                else:
                    b.synchronize()
            for i in range(warmup):
                one(i)
            sync()
            side.synchronize()
            t0 = time.perf_counter()
            for i in range(rounds):
                one(i)
            sync()
            side.synchronize()
            el = time.perf_counter() - t0
            lat = []
            for i in range(max(rounds, 20)):
                ts = time.perf_counter()
                one(i)
                sync()
                lat.append((time.perf_counter() - ts) * 1e3)
            if b is not None:
                b.close()
            for st in streams:
                st.close()
            return n_streams * rounds / el, el * 1e3 / rounds, lat

        g_rate, g_ms, g_lat = run(True, False)
        log(f"batched (graph): {g_rate:.0f} updates/s, {g_ms:.3f} ms per round of {n_streams}")
        e_rate, e_ms, _ = run(False, False)
        log(f"batched (eager launches): {e_rate:.0f} updates/s")
        s_rate, s_ms, s_lat = run(False, True)
        log(f"single-stream path, streams one after another: {s_rate:.0f} updates/s")
    frame_bytes = sum(f[0].numel() * f[0].element_size() for f in frames) * nfr
    out = {
        "workload": f"c4_narrowed_{n_streams}_streams_order3-5_modes16-256_ranks4-32_slices_le_2M_entries",
        "narrowed": "shapes whose slice exceeds 2^21 entries are drawn again; the literal distribution (modes "
                    "uniform in [16, 256] at order 5) has slices of up to 4.3e9 entries (17 GB in FP32), which "
                    "64 resident streams cannot hold",
        "streams": n_streams,
        "plan": "members with TT_FLAG_WAVE_PLAN; the one-after-another baseline with the default plan",
        "frames_per_stream": nfr,
        "frame_set_bytes": frame_bytes,
        "rounds": rounds,
        "updates_per_s": g_rate,
        "ms_per_round": g_ms,
        "latency_ms_per_round": {"p50": float(np.percentile(g_lat, 50)), "p99": float(np.percentile(g_lat, 99))},
        "eager_updates_per_s": e_rate,
        "single_stream_updates_per_s": s_rate,
        "single_stream_latency_ms_per_round": {"p50": float(np.percentile(s_lat, 50)),
                                               "p99": float(np.percentile(s_lat, 99))},
        "speedup_vs_single_stream": g_rate / s_rate,
        "pass_bytes_per_round": bytes_round,
        "pass_hbm_gbs_aggregate": bytes_round / (g_ms * 1e-3) / 1e9,
    }
    return out


def serving_section(torch, spec, frames, n_streams, rate_hz, duration, compute, tune, max_wave, lanes,
                    budget_slices, single_seconds):
    """Serving: n_streams streams of the config-3 shape with Poisson arrivals at
    rate_hz each (seeded exponential gaps) for `duration` seconds, served with
    continuous batching (TTServer) under an HBM budget of budget_slices slices;
    then the first single_seconds of the same arrival trace through
    one-at-a-time single-stream serving.  Slices come from the resident frame
    pool `frames` (more bytes than the Infinity Cache holds)."""
    from paper_2606_31061_amd import TTServer, TTStream
    from ttgen import init_cores
    pool_n = len(frames)
    slice_bytes = frames[0].numel() * frames[0].element_size()
    rng = np.random.Generator(np.random.PCG64(1005))

    def trace(dur):
        arr = []
        for q in range(n_streams):
            t = rng.exponential(1.0 / rate_hz)
            while t < dur:
                arr.append((t, q))
                t += rng.exponential(1.0 / rate_hz)
        arr.sort()
        return arr

    def run(arrivals, mw, ln, budget):
        streams = [TTStream(spec.modes, spec.ranks, init=init_cores(spec.modes, spec.ranks, 5000 + q),
                            compute=compute, autotune=tune) for q in range(n_streams)]
        sv = TTServer(max_wave=mw, lanes=ln, hbm_budget=budget)
        ids = [sv.add(st) for st in streams]
        for q in range(n_streams):  # warm-up: one update per stream
            sv.submit(ids[q], frames[q % pool_n], tag=1 << 40)
        sv.drain()
        sv.take()
        w0 = sv.stats()["waves"]
        t0 = time.perf_counter()
        for k, (ta, q) in enumerate(arrivals):
            while time.perf_counter() - t0 < ta:
                sv.poll()
            sv.submit(ids[q], frames[k % pool_n], tag=k)
            sv.poll()
        sv.drain()
        el = time.perf_counter() - t0
        res = sv.take()
        st = sv.stats()
        sv.close()
        for x in streams:
            x.close()
        lat = np.array([r[1] for r in res]) * 1e3
        waves = st["waves"] - w0
        return {"requests": len(res), "elapsed_s": el, "updates_per_s": len(res) / el,
                "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                "waves": waves, "mean_wave": len(res) / max(waves, 1), "peak_admitted_bytes": st["peak_bytes"]}

    budget = budget_slices * slice_bytes
    arr = trace(duration)
    log(f"serving: {n_streams} streams x {rate_hz} Hz for {duration} s = {len(arr)} requests; "
        f"max_wave {max_wave}, lanes {lanes}, HBM budget {budget / 1e6:.0f} MB ({budget_slices} slices)")
    cont = run(arr, max_wave, lanes, budget)
    log(f"continuous batching: {cont['updates_per_s']:.0f} updates/s, p50 {cont['latency_ms']['p50']:.2f} ms "
        f"p99 {cont['latency_ms']['p99']:.2f} ms, mean wave {cont['mean_wave']:.1f}")
    short = [a for a in arr if a[0] < single_seconds]
    single = run(short, 1, 1, 0)
    log(f"single-stream serving ({len(short)} requests): {single['updates_per_s']:.0f} updates/s, "
        f"p50 {single['latency_ms']['p50']:.2f} ms p99 {single['latency_ms']['p99']:.2f} ms")
    return {"workload": f"c5_{n_streams}_streams_c3_shape_poisson_{rate_hz:g}hz", "compute": compute,
            "offered_updates_per_s": n_streams * rate_hz, "duration_s": duration,
            "frame_pool": pool_n, "frame_pool_bytes": pool_n * slice_bytes,
            "max_wave": max_wave, "lanes": lanes, "hbm_budget_bytes": budget,
            "continuous_batching": cont, "single_stream": single,
            "single_stream_trace_s": single_seconds}


def host_description():
    """nproc and the CPU model of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        nproc = os.cpu_count() or 1
    return {"nproc": nproc, "cpu_model": model}


def _oracle_rate(spec, seconds_budget, max_slices=50):
    from oracle import ttals
    cores, g = spec.init()
    n, t_used = 0, 0.0
    t = 1
    while t_used < seconds_budget and t <= max_slices:
        X = spec.frame(t)
        t0 = time.perf_counter()
        cores, g, _ = ttals.online_step(cores, g, X)
        t_used += time.perf_counter() - t0
        n += 1
        t += 1
    return n, t_used


def cpu_baseline(spec, seconds_budget: float):
    """The FP64 oracle as it stands, timed on the host on a bounded sample,
    twice: on every host core (the BLAS thread pool's default) and on one
    thread (the paper's single-thread setting, Section 5)."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    n, t_used = _oracle_rate(spec, seconds_budget / 2)
    out = {"value": n / t_used, "unit": "slice updates/s", "cores": int(threads), "kind": "oracle",
           "sample": f"first {n} slices of the same stream (literal FP64 Algorithm 1, NumPy), "
                     f"{t_used:.1f} s of CPU work on {threads} threads",
           "host": host_description()}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            n1, t1 = _oracle_rate(spec, seconds_budget / 2)
        out["single_thread"] = {"value": n1 / t1, "unit": "slice updates/s", "cores": 1,
                                "sample": f"first {n1} slices, {t1:.1f} s of CPU work"}
    return out


def write_traffic(fetch_db, write_db, workload, compute):
    """Writes TRAFFIC_FILE from two rocprofv3 --pmc databases of a bench run
    with --copy-calibration (one with FETCH_SIZE, one with WRITE_SIZE).  Each
    counter is scaled by bytes moved / counter value of the 256 MiB copy, and
    averaged over the last ten dispatches of each contraction kernel (those
    of the tuned plan, after the tuner's trial launches)."""
    import hashlib
    import re
    import sqlite3

    def read(db, counter):
        con = sqlite3.connect(db)
        rows = con.execute("select dispatch_id, kernel_name, value from counters_collection where counter_name = ? "
                           "order by dispatch_id", (counter,)).fetchall()
        con.close()
        return rows

    copy_bytes = 256 << 20
    out = {"workload": workload, "compute": compute, "kernels": {}}
    for counter, db, key in (("FETCH_SIZE", fetch_db, "fetch_bytes"), ("WRITE_SIZE", write_db, "write_bytes")):
        rows = read(db, counter)
        copies = [v for _, k, v in rows if "copyBuffer" in k and v * 1024 > copy_bytes / 4]
        if not copies:
            raise SystemExit(f"{db}: no copy calibration dispatch (run the bench with --copy-calibration)")
        scale = copy_bytes / (max(copies) * 1024.0)
        out[key.replace("_bytes", "_scale")] = scale
        with open(os.path.join(ROOT, KERNEL_SOURCES[compute]), "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
        passes = ([["k_pass1b"], ["k_pass2b", "k_pass2s"]] if compute == "bf16"
                  else [["k_pass1"], ["k_pass2g", "k_pass2"]])
        for kerns in passes:
            found = False
            for kern in kerns:
                vals = [v for _, k, v in rows if re.search(r"\b" + kern + r"[<(]", k)][-10:]
                if not vals:
                    continue
                found = True
                rec = out["kernels"].setdefault(kern, {"source_sha256": digest, "dispatches": len(vals)})
                rec[key] = float(np.mean(vals)) * 1024.0 * scale
            if not found:
                raise SystemExit(f"{db}: no {' or '.join(kerns)} dispatches")
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c3", choices=["c3", "c2"])
    ap.add_argument("--latency-steps", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=24.0,
                    help="CPU seconds of the oracle sample, split between the all-core and the one-thread run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--compute", default="f32", choices=["f32", "bf16"],
                    help="contraction precision of the headline; bf16 also stores the slices as BF16")
    ap.add_argument("--no-other-precision", action="store_true",
                    help="skip the single-stream measurement in the other contraction precision")
    ap.add_argument("--batch", type=int, default=64,
                    help="streams in the batched measurement (0: skip it)")
    ap.add_argument("--batch-rounds", type=int, default=20)
    ap.add_argument("--serve-streams", type=int, default=256,
                    help="streams in the serving measurement (0: skip it)")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-single-seconds", type=float, default=2.0,
                    help="seconds of the same trace replayed through one-at-a-time serving")
    ap.add_argument("--serve-rate", type=float, default=30.0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default pass launch shapes instead of tuning them for the workload")
    ap.add_argument("--pool", type=int, default=0,
                    help="distinct resident frames cycled (default: more than the Infinity Cache holds)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (the counter calibration kernel)")
    ap.add_argument("--profile-ops", action="store_true",
                    help="also print the per-operation times of the update's chain (stderr)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="host only: store the contraction kernels' HBM traffic from two rocprofv3 --pmc databases "
                         "(FETCH_SIZE, WRITE_SIZE) of a --copy-calibration run, then exit")
    args = ap.parse_args()
    if args.traffic_from:
        spec, _ = make_workload(args.workload, None)
        write_traffic(args.traffic_from[0], args.traffic_from[1], spec.name, args.compute)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: every stream's update runs on a single device and the library "
              "has no multi-GPU path; run with --gpus 1.", file=sys.stderr)
        raise SystemExit(2)

    import torch

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    spec, pool_n = make_workload(args.workload, args.pool or None)
    log(f"workload {spec.name}: modes {spec.modes} ranks {spec.ranks}; generating {pool_n} frames")
    pools = {"f32": []}
    for t in range(1, pool_n + 1):
        X = spec.frame(t)
        pools["f32"].append(torch.from_numpy(np.ascontiguousarray(X.reshape(-1, order="F"))).cuda())
    pools["bf16"] = [x.to(torch.bfloat16) for x in pools["f32"]]
    torch.cuda.synchronize()
    tune = not args.no_autotune
    other = "bf16" if args.compute == "f32" else "f32"

    main_res = single_stream_section(torch, spec, pools[args.compute], args.compute, tune, args)
    other_res = None
    if not args.no_other_precision:
        other_res = single_stream_section(torch, spec, pools[other], other, tune, args, quiet=True)

    if args.copy_calibration:
        # a plain copy of known size: rocprofv3's FETCH_SIZE / WRITE_SIZE of this
        # kernel calibrate the counters (bytes counted per byte moved)
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 bytes read, 268435456 bytes written")

    batched = None
    if args.batch > 0:
        batched = batched_section(torch, args.batch, args.batch_rounds, 3, args.compute, tune)

    serving = None
    if args.serve_streams > 0:
        serving = {}
        for c in (args.compute, other):
            serving[c] = serving_section(torch, spec, pools[c], args.serve_streams, args.serve_rate,
                                         args.serve_seconds, c, tune, max_wave=32, lanes=2, budget_slices=24,
                                         single_seconds=args.serve_single_seconds)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host (all cores, then one thread)")
        cpu = cpu_baseline(spec, args.cpu_seconds)

    k, P, J, r = main_res["split"]
    line = {
        "metric": "TT-ALS slice updates/s, HBM GB/s vs peak; p50/p99 per-slice latency",
        "value": main_res["value"],
        "unit": "slice updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.compute,
        "data": "synthetic",
        "config": {
            "workload": spec.name,
            "slice_modes": list(spec.modes),
            "tt_ranks": list(spec.ranks),
            "slice_elems": spec.n_elems,
            "split_point": k,
            "frame_pool": pool_n,
            "parallelism": "single stream, one GPU",
            "pass_plans": "tuned" if tune else "default",
        },
        "latency_ms": main_res["latency_ms"],
        "roofline": main_res["roofline"],
        "slice_kernels": main_res["slice_kernels"],
        "other_precision": other_res and {key: other_res[key] for key in
                                          ("compute", "value", "ms_per_step", "latency_ms", "roofline",
                                           "slice_kernels")},
        "batched": batched,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def single_stream_section(torch, spec, pool, compute, tune, args, quiet=False):
    """The headline measurement for one contraction precision: K timed
    updates of one stream over the resident frame pool, per-slice latency,
    and the slice-pass kernels (the roofline kernel, and the update-level
    fraction of the HBM roofline)."""
    from paper_2606_31061_amd import TTStream
    pool_n = len(pool)
    cores, g = spec.init()
    s = TTStream(spec.modes, spec.ranks, init=(cores, g), compute=compute, autotune=tune)
    info = s.info()
    k = info["split_point"]
    P = int(np.prod(spec.modes[:k]))
    J = int(np.prod(spec.modes[k:]))
    r = spec.ranks[k - 1]
    log(f"[{compute}] split point k*={k}: P={P} J={J} r={r}; device bytes {info['device_bytes']}")

    for i in range(args.warmup):
        s.push(pool[i % pool_n])
    s.synchronize()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        s.push(pool[(args.warmup + i) % pool_n])
    s.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[{compute}] timed {args.steps} steps in {elapsed:.4f} s: {args.steps / elapsed:.0f} updates/s")

    # per-slice latency, one slice at a time, each pushed once the handle is
    # idle (slices arriving with gaps): push to the committed result (the
    # update's output; the next update's preparation then runs on), and push
    # to all of the handle's work done
    lat, lat_all = [], []
    for i in range(args.latency_steps):
        s.synchronize()
        ts = time.perf_counter()
        s.push(pool[i % pool_n])
        s.wait_update()
        lat.append((time.perf_counter() - ts) * 1e3)
    dev_ms = s.last_push_ms()
    for i in range(args.latency_steps):
        ts = time.perf_counter()
        s.push(pool[i % pool_n])
        s.synchronize()
        lat_all.append((time.perf_counter() - ts) * 1e3)
    s.close()
    def pct(v, q):  # None when the latency runs were skipped (--latency-steps 0)
        return float(np.percentile(v, q)) if v else None

    if lat:
        log(f"[{compute}] latency push to commit p50 {pct(lat, 50):.3f} ms p99 {pct(lat, 99):.3f} ms; "
            f"push to all work done p50 {pct(lat_all, 50):.3f} ms")

    # the passes inside the update, and optionally the chain's operations
    sp = TTStream(spec.modes, spec.ranks, init=(cores, g), profile_ops=True, compute=compute, autotune=tune)
    kt = time_passes_in_update(sp, pool, args.kernel_reps)
    # the pass kernels alone, launched back to back over the resident frames
    # (HIP events around the whole run on the stream that launches them)
    kb = sp.time_passes(pool, reps=args.kernel_reps)
    knames = sp.pass_kernels()
    if args.profile_ops and not quiet:
        prof = sp.op_profile()
        tot = sum(p[2] for p in prof)
        log(f"chain operations of one update: {len(prof)} ops, {tot:.1f} us on the chain workgroup")
        for i, (kind, dims, us) in enumerate(prof):
            log(f"  op {i:3d} {kind:6s} m={dims[0]:6d} n={dims[1]:6d} k={dims[2]:6d} {us:9.2f} us")
    sp.close()
    b1, b2 = pass_bytes(P, J, r, 2 if compute == "bf16" else 4)
    gb = {key: (b1 if key.startswith("pass1") else b2) / (ms * 1e-3) / 1e9 for key, ms in kt.items()}
    log(f"[{compute}] in the update: pass1 {kt['pass1']*1e3:.1f} us (contraction kernel "
        f"{kt['pass1_kernel']*1e3:.1f} us), pass2 {kt['pass2']*1e3:.1f} us (contraction kernel "
        f"{kt['pass2_kernel']*1e3:.1f} us)")
    log(f"[{compute}] back to back: pass1 contraction {kb['pass1_kernel']:.2f} us + reduction "
        f"{kb['pass1_reduce']:.2f} us; pass2 contraction {kb['pass2_kernel']:.2f} us + reduction "
        f"{kb['pass2_reduce']:.2f} us")
    # the dominant kernel: the slower of the two contraction kernels
    dom = "pass1" if kb["pass1_kernel"] >= kb["pass2_kernel"] else "pass2"
    kname = knames[0] if dom == "pass1" else knames[1]
    dom_bytes = b1 if dom == "pass1" else b2
    achieved = dom_bytes / (kb[dom + "_kernel"] * 1e-6) / 1e9
    traffic = measured_traffic(spec.name, compute, kname)
    ms_step = elapsed * 1e3 / args.steps
    update_gbs = (b1 + b2) / (ms_step * 1e-3) / 1e9
    return {
        "compute": compute,
        "split": (k, P, J, r),
        "value": args.steps / elapsed,
        "ms_per_step": ms_step,
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99),
                       "device_last": dev_ms, "measured": "push to committed result, slices arriving with gaps",
                       "push_to_all_work_p50": pct(lat_all, 50),
                       "push_to_all_work_p99": pct(lat_all, 99)},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_source": (f"{os.path.relpath(TRAFFIC_FILE, ROOT)}: rocprofv3 FETCH_SIZE and WRITE_SIZE "
                                        f"of {kname} on the current kernel source, scaled by a 256 MiB copy")
                     if traffic is not None else None,
                     "bytes_per_launch": dom_bytes, "kernel_us": kb[dom + "_kernel"],
                     "update_bytes": b1 + b2, "update_gbs": update_gbs,
                     "update_frac": update_gbs / HBM_PEAK_GBS},
        "slice_kernels": {"pass1_bytes": b1, "pass2_bytes": b2,
                          "back_to_back_us": kb,
                          "back_to_back_gbs": {"pass1_kernel": b1 / (kb["pass1_kernel"] * 1e-6) / 1e9,
                                               "pass2_kernel": b2 / (kb["pass2_kernel"] * 1e-6) / 1e9},
                          "in_update_us": {key: ms * 1e3 for key, ms in kt.items()},
                          "in_update_gbs": gb},
    }


if __name__ == "__main__":
    main()
