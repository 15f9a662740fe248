#!/usr/bin/env python3
"""Throughput of the sparse, truncated state-vector hot path on one MI355X.

A step is one gate step of the whole hot path: group the state by the bits
outside the gate, apply the gate with the collision merge, rank, cut (p-mass
then top-k), renormalise and write the survivors. The default workload is the
48-qubit peaked circuit (16 + 16 layers of 24 Haar SU(4) on random qubit
pairs, eps = 0.01, complex64 amplitudes), cut to min(K = 2^24, L_0.99) after
every SU(4) step. Warm-up runs at least --warmup steps and then continues
until the state stops growing (2^24 terms on the default workload), so every
timed step processes the steady-state term count; the timed steps then
continue the same circuit.

metric: gate-term updates/s = (input terms of the timed steps) / time.
roofline: the kernel kind with the largest share of the step time, its
algorithmic bytes per launch over its average launch time (HIP events on the
library's stream), against 8 TB/s. traffic: the HBM bytes per launch that
rocprofv3's FETCH_SIZE and WRITE_SIZE counters recorded for that kernel
(copy-calibrated, read from the committed summary under profiles/) over the
same average launch time, in GB/s; null when the summary was taken on other
kernels than the ones built.
cpu_baseline: the C oracle on one gate step of the steady-state GPU state,
on all host cores (its OpenMP twin, bitwise the same result) and on one core
(the plain oracle), with the host CPU named.

--workload copy measures the streaming ceiling of this GPU: device-to-device
copies and an elementwise scale of 1 GiB, timed with HIP events.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per unit for each kernel kind (c64: 8-byte key + 8-byte
# amplitude per term; c128: 8 + 16). Units: input terms of the launch, plus
# output terms where a kernel writes them.
def kernel_bytes(kind: str, amp_bytes: int, n_in: float, n_out: float, n_side: float) -> float:
    term = 8 + amp_bytes
    if kind == "radix_pass":
        return 2 * term * n_in          # read and write every term once
    if kind == "radix_hist":
        return 8 * n_in                 # keys only
    if kind == "group_hist":
        # read every term once (partners are neighbours); keep the survivors
        # above the cut's window in the side slabs (about all of them)
        return term * n_in + term * n_out
    if kind == "group_extract":
        return term * n_in + 16 * n_side
    if kind == "group_emit":
        return 2 * term * n_out         # survivors copied out of the slabs
    if kind == "side_hist":
        return 8 * n_side
    if kind == "side_extract":
        return 16 * n_side
    if kind == "tile_kept":
        return 16 * n_side
    return 0.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300, help="timed gate steps")
    ap.add_argument("--warmup", type=int, default=30, help="untimed gate steps before timing")
    ap.add_argument("--profile-steps", type=int, default=60, help="gate steps timed per kernel")
    ap.add_argument("--precision", choices=["c64", "c128"], default=None,
                    help="amplitude precision of the 48q/24q workloads (default: the workload's, complex64)")
    ap.add_argument("--workload", default="48q", choices=["48q", "24q", "c4", "c5", "copy"],
                    help="48q: the 48-qubit circuit (default); 24q: a 24-qubit one; c4: 256 uneven circuits, "
                         "batched against the plain one-at-a-time loop; c5: Poisson arrivals served with "
                         "continuous batching against the plain loop; copy: the device's streaming ceiling")
    ap.add_argument("--max-warmup", type=int, default=200,
                    help="most warm-up steps spent waiting for the state to reach its steady size")
    ap.add_argument("--requests", type=int, default=1000, help="requests of the c5 workload")
    ap.add_argument("--spec-rate", type=float, default=200.0, help="c5: the specified arrival rate (req/s)")
    ap.add_argument("--load", type=float, default=0.7, help="c5 offered load, as a fraction of served capacity")
    ap.add_argument("--batch", type=int, default=256, help="circuits of the c4 workload")
    ap.add_argument("--fuse", type=int, default=0, metavar="M",
                    help="reorder and fuse the circuit into blocks of up to M qubits first (Sec. VI.A); 0 = off")
    ap.add_argument("--sort", default="8x16", choices=["8x16", "8x8", "11x16", "11x8"],
                    help="grouping-sort shape of the 48q/24q workloads: digit bits x keys per thread")
    ap.add_argument("--cpu-sample", type=int, default=1 << 24, help="terms in the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run one device-to-device copy of BYTES (the reference dispatch that scales the "
                         "FETCH_SIZE/WRITE_SIZE counters of a profiled run)")
    return ap.parse_args()


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the state by global "
              "key bits over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2607_07816_amd import circuits as C
    from paper_2607_07816_amd._lib import State

    if args.workload == "c4":
        return bench_batch(args)
    if args.workload == "c5":
        return bench_serve(args)
    if args.workload == "copy":
        return bench_copy(args)
    if args.workload == "48q":
        circuit, cfg = C.workload_48q()
        prec = cfg["precision"]
    else:
        circuit, cfg = C.workload_24q()
        prec = "c64"
    if args.precision:
        prec = args.precision
    K, p = cfg["K"], cfg["p"]
    if args.fuse:
        from paper_2607_07816_amd import compile as CC
        ng = len(circuit.gates)
        circuit = CC.compile_circuit(circuit, args.fuse)
        log(f"fused {ng} gates into {len(circuit.gates)} blocks of <= {args.fuse} qubits")
    amp_bytes = 8 if prec == "c64" else 16
    steps_avail = [i for i, t in enumerate(circuit.truncate_after) if t]
    need = max(args.warmup, args.max_warmup) + args.steps + args.profile_steps + 1
    if need > len(steps_avail):
        raise SystemExit(f"the circuit has {len(steps_avail)} truncated steps; asked for up to {need}")

    torch.cuda.init()
    dev = torch.cuda.current_device()
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_calibration} bytes done")
        del src, dst
    log(f"device {torch.cuda.get_device_name(dev)}; workload {circuit.name} n={circuit.n} K={K} p={p} {prec}")
    # 4-qubit blocks take the tiled passes when the state holds at most half
    # of the capacity
    st = State(circuit.n, K=K, p=p, precision=prec, capacity=2 * K if args.fuse >= 4 else K)
    if args.sort != "8x16":
        st.set_sort_shape(40, args.sort)
    gi = 0

    def run(nsteps):
        nonlocal gi
        done = 0
        while done < nsteps:
            qs, U = circuit.gates[gi]
            st.apply_gate(qs, U)
            if circuit.truncate_after[gi]:
                st.truncate()
                done += 1
            gi += 1

    # warm-up: at least --warmup steps, then on until the state stops
    # growing (it holds K terms, or the p-mass cut keeps it below K), so that
    # every timed step is a steady-state step
    t_w = time.perf_counter()
    run(args.warmup)
    warm = args.warmup
    full = min(K, 1 << circuit.n) if K else 1 << min(circuit.n, 62)
    n_now, flat = st.num_terms(), 0
    while n_now < full and flat < 5 and warm < args.max_warmup:
        run(1)
        warm += 1
        n_next = st.num_terms()
        flat = flat + 1 if n_next <= n_now else 0
        n_now = n_next
    torch.cuda.synchronize()
    log(f"warm-up {warm} steps (at least {args.warmup} asked) in {time.perf_counter() - t_w:.2f}s; "
        f"terms {n_now} of {full}")

    # timed region
    c0 = st.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c1 = st.counters()
    updates = c1["term_updates"] - c0["term_updates"]
    timed_steps = c1["gate_steps"] - c0["gate_steps"]
    timed_cand = c1["candidates"] - c0["candidates"]
    elapsed = t1 - t0
    value = updates / elapsed
    log(f"timed {timed_steps} steps: {elapsed:.3f}s, {updates} updates ({updates / max(timed_steps, 1):.0f} "
        f"per step), {value:.3e} updates/s")

    # per-kernel timing over further steps (HIP events on the library's stream)
    st.profile(True)
    st.kernel_times(reset=True)
    c2 = st.counters()
    run(args.profile_steps)
    kt = st.kernel_times()
    c3 = st.counters()
    st.profile(False)
    nsteps = c3["gate_steps"] - c2["gate_steps"]
    # per-launch units of the roofline: the profiled steps' own averages
    n_in = (c3["term_updates"] - c2["term_updates"]) / max(nsteps, 1)
    n_cand = (c3["candidates"] - c2["candidates"]) / max(nsteps, 1)
    n_out = min(n_in, K)
    n_side = n_cand / 8.0  # not measured per launch; only matters if side_hist dominates
    total_ms = sum(v[0] for v in kt.values())
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms, dom_n = kt[dom]
    avg_s = dom_ms / max(dom_n, 1) / 1e3
    per_launch = kernel_bytes(dom, amp_bytes, n_in, n_out, n_side)
    achieved = per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    step_bytes = sum(kernel_bytes(k, amp_bytes, n_in, n_out, n_side) * (v[1] / max(nsteps, 1))
                     for k, v in kt.items())
    log("kernel shares: " + ", ".join(f"{k} {v[0] / max(total_ms, 1e-9) * 100:.1f}% ({v[1]})"
                                      for k, v in sorted(kt.items(), key=lambda kv: -kv[1][0])))
    log(f"dominant {dom}: {avg_s * 1e6:.1f} us/launch, {per_launch / 1e6:.1f} MB/launch, {achieved:.0f} GB/s")

    # counter summaries exist for the headline configuration only (unfused
    # 48-qubit circuit, the precision in the file name)
    profile_tag = f"peaked48_K2e24_{prec}" if args.workload == "48q" and not args.fuse else None
    traffic_gbs = measured_traffic(dom, avg_s, profile_tag)

    key, prob = st.peak()
    log(f"state peak {key:#x} prob {prob:.4f} (hidden {circuit.hidden:#x})")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(st, circuit, gi, K, p, args.cpu_sample)
    st.close()

    line = {
        "metric": "gate-term updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / max(timed_steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {
            "workload": circuit.name + f"_K2^{K.bit_length() - 1}_p{p}_{prec}",
            "fused_max_m": args.fuse,
            "sort_shape": args.sort,
            "n_qubits": circuit.n,
            "K": K,
            "p": p,
            "warmup_steps_run": warm,
            "terms_per_step": updates / max(timed_steps, 1),
            "candidates_per_step": timed_cand / max(timed_steps, 1),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_gbs,
            "launch_terms": n_in,
            "launches_timed": dom_n,
            "step_algorithmic_GBps": step_bytes / (total_ms / max(nsteps, 1) / 1e3) / 1e9 if total_ms else None,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_batch(args):
    """Many uneven circuits: the plain loop (one circuit after another on one
    stream) against the batch runner in the configuration the autotuner picks
    on a sample of the same batch. Every circuit's result is checked to be
    identical between the two."""
    import torch

    from paper_2607_07816_amd import batch as B
    from paper_2607_07816_amd import circuits as C

    torch.cuda.init()
    t = time.perf_counter()
    ws = C.batch_workload(args.batch, 4)
    items = [(c, cfg["K"], cfg["p"]) for c, cfg in ws]
    log(f"{len(items)} circuits generated in {time.perf_counter() - t:.1f}s "
        f"({sum(len(c.gates) for c, _, _ in items)} gates)")
    packed = B.pack(items)
    # warm-up: code objects, allocator
    B.run_batch(items[:8], "c64", 4, 0)
    plain, t_plain = B.run_batch(items, "c64", 1, 0, packed=packed)
    upd = sum(r["term_updates"] for r in plain)
    log(f"plain loop: {t_plain:.2f}s, {upd} updates, {upd / t_plain:.3e} updates/s")
    t = time.perf_counter()
    choice, timings = B.autotune(items, "c64")
    t_tune = time.perf_counter() - t
    def tag(k):
        return f"s{k[0]}/g{k[1]}/sort{k[3]}@2^{k[2]}"

    log(f"autotune {t_tune:.1f}s: " + ", ".join(f"{tag(k)} {v:.2f}s" for k, v in sorted(timings.items())))
    sort = (choice[2], choice[3])
    res, t_batch = B.run_batch(items, "c64", choice[0], choice[1], packed=packed, sort=sort)
    same = all(all(a[f] == b[f] for f in ("peak_key", "peak_prob", "n_terms", "term_updates", "log10_cum_kept"))
               for a, b in zip(plain, res))
    # captured-step replay against eager launches, each at its best stream count
    eager = min((v for k, v in timings.items() if k[1] == 0), default=None)
    replay = min((v for k, v in timings.items() if k[1] > 0), default=None)
    log(f"batch {tag(choice)}: {t_batch:.2f}s, {upd / t_batch:.3e} updates/s, "
        f"{t_plain / t_batch:.2f}x the plain loop; results identical: {same}")
    if not same:
        raise SystemExit("batched results differ from the plain loop")
    line = {
        "metric": "gate-term updates/s",
        "value": upd / t_batch,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": sum(r["gate_steps"] for r in res),
        "warmup": 0,
        "ms_per_step": t_batch / max(sum(r["gate_steps"] for r in res), 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"batch{len(items)}_uneven_n16-40_K2^12-2^20_c64", "circuits": len(items),
                   "streams": choice[0], "graph_steps": choice[1],
                   "sort_small_log2": choice[2], "sort_shape": choice[3]},
        "plain_loop": {"value": upd / t_plain, "seconds": t_plain},
        "batch_seconds": t_batch,
        "speedup_vs_plain": t_plain / t_batch,
        "autotune": {"seconds": t_tune, "sample": "every 4th circuit",
                     "timings": {tag(k): v for k, v in sorted(timings.items())},
                     "sample_seconds_eager_best": eager, "sample_seconds_replay_best": replay},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def serve_run(items, arrivals, streams, active, turn, hbm, sample_every=0.5):
    """Submit items at the given arrival times (seconds from start) to a
    fresh server; returns (results in item order, makespan seconds, samples
    of the server's queue [(t, queued, active, done)] every sample_every s)."""
    import threading

    from paper_2607_07816_amd.serve import Server

    samples = []
    with Server("c64", streams, active, turn, hbm_bytes=hbm) as srv:
        tickets = [None] * len(items)
        stop = threading.Event()
        t0 = time.perf_counter()

        def submitter():
            for i, (c, K, p) in enumerate(items):
                d = arrivals[i] - (time.perf_counter() - t0)
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(c, K, p)

        def monitor():
            last = time.perf_counter()
            while not stop.wait(sample_every):
                st = srv.stats()
                now = time.perf_counter()
                samples.append((now - t0, st["queued"], st["active"], st["done"]))
                if now - last >= 15.0:  # a progress line now and then
                    log(f"  t={now - t0:.0f}s queued {st['queued']} active {st['active']} done {st['done']}")
                    last = now

        th = threading.Thread(target=submitter)
        th.start()
        mon = threading.Thread(target=monitor)
        mon.start()
        th.join()
        res = [srv.wait(t) for t in tickets]
        span = time.perf_counter() - t0
        stop.set()
        mon.join()
    return res, span, samples


def bench_serve(args):
    """Serving (continuous batching) of Poisson arrivals of uneven requests.

    1. The offered rate of the specification (--spec-rate, 200 req/s): all
       requests arrive at that rate; the server's queue is sampled while they
       arrive and drain, giving its served capacity (requests / makespan) and
       how fast the queue grows at that rate.
    2. A sustainable rate, --load (0.7) of that capacity: p50/p99 latency
       and throughput of the server.
    3. The plain loop (one stream, one request at a time, in arrival order)
       fed the same arrivals as 2.
    Every request's result must be identical in 2 and 3; its peak is also
    compared with the circuit's hidden bit string s."""
    import numpy as np
    import torch

    from paper_2607_07816_amd import circuits as C

    torch.cuda.init()
    t = time.perf_counter()
    ws = C.serving_workload(args.requests, 5)
    items = [(c, cfg["K"], cfg["p"]) for c, cfg in ws]
    hidden = [c.hidden for c, _ in ws]
    log(f"{len(items)} requests generated in {time.perf_counter() - t:.1f}s "
        f"({sum(len(c.gates) for c, _, _ in items)} gates)")
    free, total = torch.cuda.mem_get_info()
    # admission against the device's own memory: the server's budget is 90%
    # of what is free on it (the rest for the runtime and torch)
    hbm = int(free * 0.9)
    log(f"device memory: {total / 2**30:.1f} GiB, free {free / 2**30:.1f} GiB, server budget {hbm / 2**30:.1f} GiB")
    cfg = (16, 2, 8)
    serve_run(items[:4], [0.0] * 4, 4, 2, 8, 8 << 30)  # warm-up: code objects, allocator

    def summary(res, span, arrivals):
        lat = np.array([r["latency_seconds"] for r in res])
        return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean()), "makespan_s": span,
                "offered_rps": len(res) / max(arrivals[-1], 1e-9),
                "throughput_updates_per_s": sum(r["term_updates"] for r in res) / span,
                "throughput_requests_per_s": len(res) / span,
                "peak_is_hidden": sum(int(r["peak_key"] == h) for r, h in zip(res, hidden)) / len(res)}

    rng = np.random.default_rng(5)
    gaps = rng.exponential(1.0, size=len(items))  # unit-rate Poisson gaps, scaled per run
    # 1. the specification's rate
    arr_spec = np.cumsum(gaps / args.spec_rate).tolist()
    res0, span0, samp = serve_run(items, arr_spec, *cfg, hbm)
    cap_rps = len(items) / span0
    t_in = arr_spec[-1]
    during = [s_ for s_ in samp if s_[0] <= t_in] or samp[:1]
    q_end = (during[-1][1] + during[-1][2]) if during else 0
    spec = summary(res0, span0, arr_spec)
    spec.update({"served_capacity_rps": cap_rps, "arrival_window_s": t_in,
                 "backlog_at_last_arrival": int(q_end), "backlog_growth_rps": q_end / max(t_in, 1e-9),
                 "queue_samples": [[round(a, 2), int(b), int(c_), int(d)] for a, b, c_, d in samp[:: max(1, len(samp) // 60)]]})
    log(f"offered {spec['offered_rps']:.0f} req/s: served {cap_rps:.2f} req/s, backlog {q_end} after "
        f"{t_in:.1f}s of arrivals ({spec['backlog_growth_rps']:.0f} req/s growth), p50 {spec['p50_s']:.2f}s "
        f"p99 {spec['p99_s']:.2f}s")
    # 2. a sustainable rate
    lam = args.load * cap_rps
    arrivals = np.cumsum(gaps / lam).tolist()
    res_s, span_s, _ = serve_run(items, arrivals, *cfg, hbm)
    served = summary(res_s, span_s, arrivals)
    log(f"served at {lam:.2f} req/s: p50 {served['p50_s']:.3f}s p99 {served['p99_s']:.3f}s, "
        f"{served['throughput_updates_per_s']:.3e} updates/s, peak = s for {served['peak_is_hidden']:.1%}")
    # 3. the plain loop on the same arrivals
    res_p, span_p, _ = serve_run(items, arrivals, 1, 1, 1 << 30, hbm)
    plain = summary(res_p, span_p, arrivals)
    log(f"plain loop at {lam:.2f} req/s: p50 {plain['p50_s']:.3f}s p99 {plain['p99_s']:.3f}s, "
        f"{plain['throughput_updates_per_s']:.3e} updates/s")
    fields = ("peak_key", "peak_prob", "n_terms", "term_updates", "log10_cum_kept")
    same = all(all(a[f] == b[f] for f in fields) for a, b in zip(res_s, res_p))
    same0 = all(all(a[f] == b[f] for f in fields) for a, b in zip(res_s, res0))
    log(f"results identical served vs plain loop: {same}; vs the spec-rate run: {same0}")
    if not (same and same0):
        raise SystemExit("served results differ between runs")
    line = {
        "metric": "gate-term updates/s",
        "value": served["throughput_updates_per_s"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": sum(r["gate_steps"] for r in res_s),
        "warmup": 4,
        "ms_per_step": span_s / max(sum(r["gate_steps"] for r in res_s), 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"serve{len(items)}_poisson_n20-64_K2^14-2^22_topk-or-p0.99_c64",
                   "requests": len(items), "offered_rps": lam, "load_fraction": args.load,
                   "spec_rate_rps": args.spec_rate, "streams": cfg[0], "max_active": cfg[1],
                   "gates_per_turn": cfg[2], "hbm_budget_bytes": hbm, "device_bytes": total},
        "served": served,
        "plain_loop": plain,
        "spec_rate": spec,
        "speedup_vs_plain": served["throughput_updates_per_s"] / plain["throughput_updates_per_s"],
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def measured_traffic(kind: str, avg_s: float, tag):
    """HBM bytes per launch of `kind` from the committed counter summary of
    the configuration `tag`, over the live average launch time (GB/s); None
    if there is no summary for that kernel and configuration or the
    library's kernels changed since it was taken."""
    from paper_2607_07816_amd import profsum

    if tag is None:
        return None
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"{kind}_{tag}_hbm_traffic.txt")
    if not os.path.exists(path) or avg_s <= 0:
        return None
    rec = profsum.read_traffic(path)
    if rec.get("source_digest") != profsum.source_digest():
        log(f"{os.path.basename(path)} was taken on other kernels: traffic not reported")
        return None
    tb = float(rec["traffic_bytes_per_launch"])
    log(f"counter traffic of {kind}: {tb / 1e6:.1f} MB/launch")
    return tb / avg_s / 1e9


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(st, circuit, gi, K, p, sample_terms):
    """Time the C oracle on one gate step of (a sample of) the GPU's state:
    on all the host cores this process may use (the oracle's OpenMP twin)
    and on one core (the plain oracle); both must give the same terms."""
    import numpy as np

    from oracle import c_oracle

    keys, amps = st.read_terms()
    n = keys.shape[0]
    take = min(sample_terms, n)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(n, size=take, replace=False)) if take < n else np.arange(n)
    k, a = keys[idx], amps[idx]
    kk = max(1, int(K * take / max(n, 1)))
    # next truncated gate of the circuit
    while not circuit.truncate_after[gi]:
        gi += 1
    qs, U = circuit.gates[gi]
    c_oracle.build()
    threads = c_oracle.host_threads()
    t0 = time.perf_counter()
    km, am, _ = c_oracle.step(k, a, qs, U, kk, p, True, threads=threads)
    dt_all = time.perf_counter() - t0
    t0 = time.perf_counter()
    k1, a1, _ = c_oracle.step(k, a, qs, U, kk, p, True)
    dt_one = time.perf_counter() - t0
    km, am = c_oracle.sorted_terms(km, am)
    k1, a1 = c_oracle.sorted_terms(k1, a1)
    same = bool(np.array_equal(km, k1) and np.array_equal(am.view(np.uint64), a1.view(np.uint64)))
    model = host_cpu_model()
    log(f"cpu oracle on {take} terms, K={kk}: {dt_all:.2f}s on {threads} threads, {dt_one:.2f}s on one; "
        f"same terms: {same}; host {model}, os.cpu_count() = {os.cpu_count()}")
    if not same:
        raise SystemExit("the oracle's OpenMP twin differs from the plain oracle")
    what = (f"the whole steady state ({n} terms), K={kk}" if take == n else
            f"{take} of the {n} steady-state terms (random subset), K scaled to {kk}")
    return {
        "value": take / dt_all,
        "unit": "updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"one gate step (apply + truncate) of the C oracle, FP64, on {what}, p={p}",
        "one_core_value": take / dt_one,
        "cpu_model": model,
        "host_cpu_count": os.cpu_count(),
    }


def bench_copy(args):
    """The streaming ceiling of this GPU: a device-to-device copy and an
    elementwise scale of 1 GiB each way, HIP events around each repetition."""
    import torch

    torch.cuda.init()
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    res = {}
    for name, fn in (("copy", lambda: dst.copy_(src)), ("scale", lambda: torch.mul(src, 2.0, out=dst))):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(args.steps if args.steps < 300 else 20):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b) / 1e3)
        times.sort()
        med = times[len(times) // 2]
        res[name] = {"median_s": med, "GBps": 2 * nbytes / med / 1e9, "best_GBps": 2 * nbytes / times[0] / 1e9}
        log(f"{name}: 2 x {nbytes} bytes, median {med * 1e6:.1f} us, {2 * nbytes / med / 1e9:.0f} GB/s")
    line = {
        "metric": "device streaming bandwidth", "value": res["copy"]["GBps"], "unit": "GB/s", "n_gpus": 1,
        "steps": len(times), "warmup": 3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic", "config": {"workload": "copy_and_scale_1GiB"},
        "copy": res["copy"], "scale": res["scale"], "peak_GBps": HBM_PEAK_GBS,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
