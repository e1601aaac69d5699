#!/usr/bin/env python
"""Benchmark of the D3Q19 MRT-Smagorinsky LES hot path on one MI355X.

Prints ONE JSON line.  The headline workload is forced-HIT LES on a 100^3
periodic lattice in FP32 (Re = 2e4 at U0 = 0.043, C_s = 0.1 in
nu_t = (C_s Delta)^2 |S|, solenoidal forcing on |k| <= 2 with seeded phases,
1e-3 noise start) with its diagnostics every 500 lattice steps: the K_t / theta
statistics, the K_t map of the mid-z plane (copied to the host) and the energy
spectrum E(k), k <= N/2.  It streams A/B (two arrays): the 2 x 76 MB stay in the
last-level cache, where the step runs about 2 % faster than in place
(--streaming aa).  The 800^3 lines keep the in-place AA form, whose 39 GB
state is half of A/B's.

A bench "step" is one pass of the whole hot path over the workload: one
snapshot interval, i.e. 500 lattice time steps (one replay of a captured graph
of 500 fused stream-and-collide launches) followed by that interval's
diagnostics.  --steps K intervals are timed per repeat, --repeats R repeats
(default 5), each bracketed by a device synchronisation; ``value`` is the
median over the repeats of MLUPS (million lattice-cell updates per second, the
diagnostics included), with the state resident in HBM.  The default K = 40 is
the workload's 20 000 lattice steps.

Beside it the same line carries: the roofline of the step kernel (algorithmic
bytes 2 * 19 * 4 per cell update over its mean launch time, from HIP events
around the graph replays on the kernel's stream, next to the mean the committed
rocprofv3 trace records and a same-size device copy for the cache-resident
100^3 state), the 800^3 FP32 runs (AA, A/B, A/B with two steps per pass), the
800^3 FP16 / BF16 storage runs (and FP16 with two steps per pass) with their
K_t-statistics and spectral errors against the FP32 run, the batched-serving run
(p50/p99 completion latency and aggregate MLUPS), and the FP64 C oracle timed
on the host cores on a bounded sample.
"""
import argparse
import gc
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline, MRT-Smag 100^3/800^3; batched p50/p99 latency"
PEAK_HBM_GBS = 8000.0
BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_TABLE = "hbm_traffic_step_kernels_forced_hit_100_800.txt"
DURATION_TABLE = "durations_step_kernels_forced_hit_100_800.txt"


def _profile_row(table, workload_key, family):
    """The row of a committed per-lattice profile table for this lattice, if it was
    taken on the machine code of that kernel in the built library (else None)."""
    from paper_2512_23116_amd.rocprof_summary import kernel_code_sha
    path = os.path.join(ROOT, "profiles", table)
    if not os.path.exists(path):
        return None
    sha = kernel_code_sha(family)
    for line in open(path):
        parts = line.split()
        if len(parts) >= 5 and not line.startswith("#") and parts[0] == workload_key \
                and parts[1] == sha:
            return parts
    return None


def counter_traffic(workload_key, family="k_step"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the machine code of that kernel in the built library (else None)."""
    parts = _profile_row(TRAFFIC_TABLE, workload_key, family)
    return None if parts is None else float(parts[2]) + float(parts[3])


def profile_launch_us(workload_key, family="k_step"):
    """Mean duration of one step launch in the committed rocprofv3 kernel trace of
    this command, if it was taken on the machine code in the built library (else None)."""
    parts = _profile_row(DURATION_TABLE, workload_key, family)
    return None if parts is None else float(parts[2])


def device_copy_rate(nbytes, reps=200):
    """GB/s of a device-to-device copy of `nbytes` (read nbytes + write nbytes) on
    nonzero data, timed with HIP events over `reps` copies: the bandwidth a
    streaming kernel gets on a working set of that size (for 2 x 76 MB it stays
    in the 256 MB last-level cache)."""
    import torch
    n = nbytes // 4
    x = torch.rand(n, device="cuda") + 1.0
    y = torch.empty_like(x)
    for _ in range(20):
        y.copy_(x)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * n * 4 * reps / sec / 1e9


def cpu_model():
    """The host CPU's model name (lscpu), or None."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    for line in out.splitlines():
        if line.lower().startswith("model name"):
            return line.split(":", 1)[1].strip()
    return None


def run_workload(lbm, params, N, precision, streaming, intervals, warmup, repeats, interval):
    """The headline workload: `repeats` timed runs of `intervals` snapshot
    intervals each.  One interval = `interval` lattice steps (one graph replay)
    and then the K_t statistics, the K_t map of the mid-z plane and the spectrum
    E(k <= N/2) of the state reached, all collected before the repeat's clock
    stops.  The `warmup` intervals before the first repeat capture the graph and
    create the FFT plan and the analysis buffers."""
    import torch
    stream = torch.cuda.Stream()
    cfg = params.forced_hit(N)
    spg = interval if interval % 4 == 0 and interval <= 1024 else 64
    lat = lbm.Lattice((N, N, N), cfg["tau0"], cfg["C"], cfg["modes"], precision=precision,
                      streaming=streaming, smag_form=cfg["smag_form"], steps_per_graph=spg,
                      stream=stream)
    lat.init(lbm.LBM_INIT_NOISE, cfg["noise"], cfg["init_seed"])
    kmax, zmid = N // 2, N // 2

    # Each interval's snapshot (statistics, K_t map of the mid plane, spectrum) is
    # enqueued right after its steps and collected once the next interval's steps
    # are enqueued too (lbm_snapshot_begin / _end): the device never waits for the
    # host between intervals.
    for _ in range(warmup):
        lat.step(interval)
        lat.snapshot_begin(kmax, zmid)
        lat.snapshot_end()
    lat.sync()
    torch.cuda.synchronize()
    reps, last = [], None
    # The host runs one interval ahead of the device: a pause of the cyclic
    # garbage collector longer than an interval (a full pass over torch's objects
    # takes tens of ms) would leave the device idle.  It is run before each
    # repeat and kept off inside it, as timeit does.
    gc_was_enabled = gc.isenabled()
    for _ in range(repeats):
        events = []
        gc.collect()
        gc.disable()
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(intervals):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                lat.step(interval)
                e1.record(stream)
                events.append((e0, e1))
                if i > 0:
                    last = lat.snapshot_end()
                lat.snapshot_begin(kmax, zmid)
            last = lat.snapshot_end()
            lat.sync()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        finally:
            if gc_was_enabled:
                gc.enable()
        kern_s = sum(a.elapsed_time(b) for a, b in events) / 1e3
        cells = N ** 3 * intervals * interval
        reps.append(dict(wall_s=wall, mlups=cells / wall / 1e6,
                         ms_per_step=wall / intervals * 1e3,
                         avg_launch_us=kern_s / (intervals * interval) * 1e6))
    st, E, sl = last
    steps_done = lat.steps
    ceil = pattern_ceiling(lat, stream, 200)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    order = sorted(range(repeats), key=lambda i: reps[i]["mlups"])
    med = reps[order[repeats // 2]]
    bytes_per_launch = 2 * 19 * BYTES[precision] * N ** 3
    avg_us = statistics.median(r["avg_launch_us"] for r in reps)
    achieved = bytes_per_launch / (avg_us * 1e-6) / 1e9
    return dict(N=N, median=med, repeats=reps, avg_launch_us=avg_us, tau0=cfg["tau0"],
                spg=spg, steps_done=steps_done,
                roofline=dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s",
                              frac=achieved / PEAK_HBM_GBS, bytes_per_launch=bytes_per_launch),
                kt=dict(mean=st["kt_mean"], var=st["kt_var"], flat=st["kt_flat"],
                        theta_mean=st["theta_mean"], step=st["steps"]),
                kt_map_mean=float(sl.mean()), spectrum_last=[float(v) for v in E[:26]],
                pattern=ceil)


def launch_ms(stream, fn, n):
    """Mean ms per launch of `fn(n)` (n plain launches) from HIP events on `stream`."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn(n)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / n


def pattern_ceiling(lat, stream, n):
    """The step's data movement alone against the step: `n` plain launches of free
    streaming (lbm_stream_only: the same loads, stores, layout and block order, no
    arithmetic) and `n` plain step launches, ms per launch.  Changes the state (taken
    after the workload's last statistics)."""
    lat.stream_only(2)
    stream_ms = launch_ms(stream, lat.stream_only, n)
    lat.step(2)
    step_ms = launch_ms(stream, lat.step, n)
    return dict(stream_only_ms=round(stream_ms, 5), step_plain_ms=round(step_ms, 5),
                step_over_stream=round(step_ms / stream_ms, 4),
                note="plain launches, HIP events; stream_only = lbm_stream_only, the step's "
                     "loads and stores with no collision")


def run_lattice(lbm, params, N, precision, streaming, steps, warmup, diag_every, spg=64, tb=0,
                final_spectrum=0, ceiling=0):
    """Time `steps` steps; every `diag_every` steps take the K_t statistics: the
    diagnostics of the workload run inside the timed region.  With
    `final_spectrum` = K the spectrum E(0..K) of the last state is taken after the
    clock stops, and with `ceiling` = n the data-movement ceiling of the step's
    access pattern is measured after that (pattern_ceiling, n launches)."""
    import torch
    stream = torch.cuda.Stream()
    cfg = params.forced_hit(N)
    lat = lbm.Lattice((N, N, N), cfg["tau0"], cfg["C"], cfg["modes"], precision=precision,
                      streaming=streaming, smag_form=cfg["smag_form"], steps_per_graph=spg,
                      temporal_block=tb, stream=stream)
    lat.init(lbm.LBM_INIT_NOISE, cfg["noise"], cfg["init_seed"])
    stats = [lat.stats()] if warmup == 0 else []
    lat.step(warmup)
    lat.sync()
    events = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(diag_every, steps - done) if diag_every else steps
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.step(n)
        e1.record(stream)
        events.append((e0, e1))
        done += n
        if diag_every and done % diag_every == 0:
            stats.append(lat.stats())
    lat.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_s = sum(a.elapsed_time(b) for a, b in events) / 1e3
    final = lat.stats()
    spec_final = lat.spectrum(final_spectrum) if final_spectrum else None
    ceil = pattern_ceiling(lat, stream, ceiling) if ceiling and tb == 0 else None
    lat.close()
    del lat
    torch.cuda.empty_cache()
    ncell = N ** 3
    bytes_per_launch = 2 * 19 * BYTES[precision] * ncell
    avg = kern_s / steps
    achieved = bytes_per_launch / avg / 1e9
    return dict(N=N, steps=steps, wall_s=wall, mlups=ncell * steps / wall / 1e6,
                ms_per_step=wall / steps * 1e3, avg_launch_us=avg * 1e6,
                kernel_mlups=ncell / avg / 1e6,
                roofline=dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s",
                              frac=achieved / PEAK_HBM_GBS,
                              bytes_per_launch=bytes_per_launch),
                kt=dict(mean=final["kt_mean"], var=final["kt_var"], flat=final["kt_flat"],
                        theta_mean=final["theta_mean"], n_snapshots=len(stats)),
                kt_series=[dict(step=st["steps"], mean=st["kt_mean"], var=st["kt_var"],
                                flat=st["kt_flat"]) for st in stats],
                spectrum_final=spec_final, tau0=cfg["tau0"], pattern=ceil)


def cpu_baseline(N, target_s=12.0):
    from oracle import init_fields as I
    from oracle import ref_c
    from paper_2512_23116_amd import params
    cfg = params.forced_hit(N)
    lat = ref_c.Lattice((N, N, N), cfg["tau0"], cfg["C"], cfg["modes"],
                        smag_form=cfg["smag_form"])
    f = lat.init(I.KIND_NOISE, cfg["noise"], cfg["init_seed"])
    t = time.perf_counter()
    f = lat.step(f, 2)
    probe = time.perf_counter() - t
    n = max(2, min(200, int(target_s / max(probe / 2, 1e-6))))
    t = time.perf_counter()
    lat.step(f, n)
    dt = time.perf_counter() - t
    return dict(value=N ** 3 * n / dt / 1e6, unit="MLUPS", cores=ref_c.num_threads(),
                kind="oracle",
                sample=f"{N}^3 forced HIT, {n} steps of the plain C FP64 oracle (OpenMP)",
                cpu_model=cpu_model(), host_cpus=os.cpu_count())


def precision_errors(run, ref, N):
    """Errors of a reduced-precision run against the FP32 run of the same workload:
    relative error of the K_t mean / variance / flatness at every common snapshot
    after step 0 (max over snapshots and at the last one; at step 0 the K_t
    variance of the noise start is ~1e-21 and only measures the rounding of the
    initial state) and the spectral error
    max_{1<=k<=K} |E(k) / E_ref(k) - 1| of the last state for K = 8, 32, N/4."""
    ref_by_step = {s["step"]: s for s in ref["kt_series"]}
    worst = {"mean": 0.0, "var": 0.0, "flat": 0.0}
    last = {}
    for s in run["kt_series"]:
        r = ref_by_step.get(s["step"])
        if r is None or s["step"] == 0:
            continue
        for q in worst:
            e = abs(s[q] - r[q]) / abs(r[q])
            worst[q] = max(worst[q], e)
            last[q] = e
    spec = {}
    if run["spectrum_final"] is not None and ref["spectrum_final"] is not None:
        E, Er = run["spectrum_final"], ref["spectrum_final"]
        for K in (8, 32, N // 4):
            spec[f"k<={K}"] = max(abs(E[k] / Er[k] - 1.0) for k in range(1, K + 1))
    return dict(kt_rel_err_max=worst, kt_rel_err_last=last, spectrum_rel_err_last=spec)


def run_serving(n_req, steps, seed=2024):
    from paper_2512_23116_amd import serving
    # capacity: every request present at t = 0
    reqs = serving.make_requests(n_req, seed=seed, steps=steps)
    eng = serving.GpuEngine(max_slots=16, steps_per_graph=64)
    closed = serving.serve(reqs, eng, max_slots=16, hbm_budget=80e9)
    eng.close()
    mean_updates = sum(r.cells * r.steps for r in reqs) / len(reqs)
    rate = 0.8 * closed["busy_mlups"] * 1e6 / mean_updates
    log(f"serving closed batch: {closed['busy_mlups']:.0f} MLUPS busy, "
        f"{closed['aggregate_mlups']:.0f} aggregate, busy {closed['busy_frac']:.3f}, "
        f"{closed['wall_s']:.1f} s; Poisson rate {rate:.2f}/s")
    reqs = serving.make_requests(n_req, seed=seed, steps=steps, rate=rate)
    eng = serving.GpuEngine(max_slots=16, steps_per_graph=64)
    res = serving.serve(reqs, eng, max_slots=16, hbm_budget=80e9)
    eng.close()
    return dict(requests=n_req, steps_each=steps, arrival_rate_per_s=rate,
                offered_mlups=rate * mean_updates / 1e6,
                p50_s=res["p50_s"], p99_s=res["p99_s"],
                wait_p50_s=res["wait_p50_s"], wait_p99_s=res["wait_p99_s"],
                service_p50_s=res["service_p50_s"], service_p99_s=res["service_p99_s"],
                aggregate_mlups=res["aggregate_mlups"],
                busy_mlups=res["busy_mlups"], busy_frac=res["busy_frac"],
                busy_frac_when_work=res["busy_frac_when_work"], failed=res["failed"],
                capacity_mlups=closed["busy_mlups"],
                closed_batch={"wall_s": closed["wall_s"],
                              "aggregate_mlups": closed["aggregate_mlups"],
                              "busy_frac": closed["busy_frac"],
                              "busy_frac_when_work": closed["busy_frac_when_work"]},
                slots=16, hbm_budget_gb=80, group_mb=serving.GROUP_BYTES >> 20,
                note="busy = GPU time of the batched calls (HIP events); busy_frac_when_work "
                     "= busy / host time while a request was waiting, active or in flight")


def profile_run(lbm, params, args):
    """Known-size copy (the counter calibration), then a few plain step launches."""
    import torch
    n = 1 << 28                      # 2^28 floats = 1 GiB read + 1 GiB written per copy
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()
    log("profile: 3 copies of 1 GiB done")
    p = args.precision
    runs = [(args.N, p, args.streaming, 0, 8)]
    if not args.no_large:
        runs += [(args.large_N, p, "aa", 0, 4), (args.large_N, p, "ab", 0, 4),
                 (args.large_N, p, "ab", 2, 8)]
        if not args.no_precision:
            runs += [(args.large_N, "fp16", "aa", 0, 4), (args.large_N, "bf16", "aa", 0, 4),
                     (args.large_N, "fp16", "ab", 2, 8), (args.large_N, "bf16", "ab", 2, 8)]
    for N, prec, streaming, tb, steps in runs:
        # (AA and A/B one-step runs also time 4 launches of free streaming and 4 steps)
        run_lattice(lbm, params, N, prec, streaming, steps, 2, 0, spg=0, tb=tb,
                    ceiling=4 if tb == 0 and N == args.large_N else 0)
        log(f"profile: {N}^3 {prec} {streaming}{' two-step' if tb else ''}, "
            f"{steps} steps of plain launches done")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40,
                    help="timed bench steps per repeat; one bench step = one snapshot interval "
                         "(--diag-every lattice steps and their diagnostics)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed snapshot intervals")
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--N", type=int, default=100)
    ap.add_argument("--precision", default="fp32", choices=sorted(BYTES))
    ap.add_argument("--streaming", default="ab", choices=["aa", "ab"],
                    help="streaming of the headline lattice (A/B: two arrays; AA: in place)")
    ap.add_argument("--diag-every", type=int, default=500,
                    help="lattice steps per snapshot interval (one captured graph)")
    ap.add_argument("--steps-per-graph", type=int, default=500,
                    help="graph length of the 800^3 runs")
    ap.add_argument("--large-N", type=int, default=800)
    ap.add_argument("--large-steps", type=int, default=2000)
    ap.add_argument("--serving-requests", type=int, default=64)
    ap.add_argument("--serving-steps", type=int, default=5000)
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-large-ab", action="store_true",
                    help="skip the 800^3 A/B (two-array) measurement beside the AA one")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the 800^3 FP16 / BF16 storage runs compared with the FP32 one")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="short run for hardware counters: a 1 GiB copy of known size, then "
                         "plain (graph-free) step launches at N and large-N; no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the LES hot path here is single-device)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_23116_amd import lbm, params
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    lbm.lib()
    if args.profile:
        profile_run(lbm, params, args)
        return

    if args.steps < 1 or args.repeats < 1 or args.warmup < 0:
        print("--steps and --repeats must be >= 1, --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    log(f"main: {args.N}^3 {args.precision} {args.streaming}, {args.repeats} x {args.steps} "
        f"intervals of {args.diag_every} steps after {args.warmup} warm-up intervals")
    main_run = run_workload(lbm, params, args.N, args.precision, args.streaming, args.steps,
                            args.warmup, args.repeats, args.diag_every)
    med = main_run["median"]
    log(f"main: {med['mlups']:.0f} MLUPS (median of {args.repeats}; "
        f"{min(r['mlups'] for r in main_run['repeats']):.0f}-"
        f"{max(r['mlups'] for r in main_run['repeats']):.0f}), "
        f"{main_run['avg_launch_us']:.2f} us/launch, {main_run['roofline']['frac']:.3f} of HBM peak")
    key = f"{args.N}_{args.precision}_{args.streaming}"
    main_run["roofline"]["traffic"] = counter_traffic(key)
    # the state and the copy of the same bytes: cache-resident below 256 MB
    state_bytes = 19 * BYTES[args.precision] * args.N ** 3
    copy_gbs = device_copy_rate(state_bytes)
    log(f"main: device copy of {state_bytes / 1e6:.0f} MB at {copy_gbs:.0f} GB/s")

    large = None
    if not args.no_large:
        log(f"large: {args.large_N}^3 fp32 aa, {args.large_steps} steps")
        # no warm-up: K_t statistics from step 0 on (the module is loaded and the
        # clocks are up from the main run; graph capture costs ~1 ms of the timed span)
        large = run_lattice(lbm, params, args.large_N, "fp32", "aa", args.large_steps, 0,
                            args.diag_every, args.steps_per_graph,
                            final_spectrum=0 if args.no_precision else args.large_N // 4,
                            ceiling=10)
        large_copy_gbs = device_copy_rate(19 * 4 * args.large_N ** 3, reps=20)
        log(f"large: device copy of the state's bytes at {large_copy_gbs:.0f} GB/s; step "
            f"{large['pattern']['step_plain_ms']:.3f} ms vs free streaming "
            f"{large['pattern']['stream_only_ms']:.3f} ms per launch")
        large["roofline"]["traffic"] = counter_traffic(f"{args.large_N}_fp32_aa")
        log(f"large: {large['mlups']:.0f} MLUPS, {large['roofline']['frac']:.3f} of HBM peak")

    large_ab = large_tb2 = None
    if not args.no_large and not args.no_large_ab:
        log(f"large A/B: {args.large_N}^3 fp32 ab, {args.large_steps // 2} steps")
        large_ab = run_lattice(lbm, params, args.large_N, "fp32", "ab", args.large_steps // 2, 64,
                               args.diag_every, args.steps_per_graph, ceiling=10)
        log(f"large A/B: {large_ab['mlups']:.0f} MLUPS, {large_ab['roofline']['frac']:.3f} of HBM peak")
        log(f"large A/B two steps per pass: {args.large_N}^3 fp32, {args.large_steps} steps")
        large_tb2 = run_lattice(lbm, params, args.large_N, "fp32", "ab", args.large_steps, 64,
                                args.diag_every, args.steps_per_graph, tb=2)
        log(f"large A/B two steps per pass: {large_tb2['mlups']:.0f} MLUPS, "
            f"{large_tb2['roofline']['frac']:.3f} of the single-step HBM roofline")

    precision = {}
    if large and not args.no_precision:
        for prec in ("fp16", "bf16"):
            log(f"precision: {args.large_N}^3 {prec} aa, {args.large_steps} steps")
            pr = run_lattice(lbm, params, args.large_N, prec, "aa", args.large_steps, 0,
                             args.diag_every, args.steps_per_graph,
                             final_spectrum=args.large_N // 4, ceiling=10)
            rr = pr["roofline"]
            precision[prec] = {
                "workload": (f"forced HIT LES {args.large_N}^3, populations stored as {prec} "
                             "deviations with a per-run scale, FP32 collision, FP64 reductions, AA"),
                "mlups": round(pr["mlups"], 1), "steps": pr["steps"],
                "ms_per_step": round(pr["ms_per_step"], 4),
                "roofline": {"bound": "hbm", "achieved": round(rr["achieved"], 1),
                             "peak": rr["peak"], "unit": "GB/s", "frac": round(rr["frac"], 4),
                             "traffic": counter_traffic(f"{args.large_N}_{prec}_aa"),
                             "avg_launch_us": round(pr["avg_launch_us"], 2),
                             "profile_avg_launch_us":
                                 profile_launch_us(f"{args.large_N}_{prec}_aa"),
                             "pattern_ceiling": pr["pattern"]},
                "vs_fp32": precision_errors(pr, large, args.large_N)}
            log(f"precision: {prec} {pr['mlups']:.0f} MLUPS, {rr['frac']:.3f} of HBM peak, "
                f"K_t mean rel err {precision[prec]['vs_fp32']['kt_rel_err_max']['mean']:.2e}")
        # FP16 storage with two time steps per pass (A/B): the fastest form
        log(f"precision: {args.large_N}^3 fp16 A/B two steps per pass, {args.large_steps} steps")
        pr = run_lattice(lbm, params, args.large_N, "fp16", "ab", args.large_steps, 0,
                         args.diag_every, args.steps_per_graph, tb=2,
                         final_spectrum=args.large_N // 4)
        rr = pr["roofline"]
        pass_us = 2 * pr["avg_launch_us"]
        own = rr["bytes_per_launch"] / (pass_us * 1e-6) / 1e9
        precision["fp16_two_step"] = {
            "workload": (f"forced HIT LES {args.large_N}^3, fp16 deviations, A/B with two time "
                         "steps per pass (intermediate level in LDS)"),
            "mlups": round(pr["mlups"], 1), "steps": pr["steps"],
            "ms_per_step": round(pr["ms_per_step"], 4),
            "roofline": {"bound": "hbm", "achieved": round(own, 1), "peak": rr["peak"],
                         "unit": "GB/s", "frac": round(own / rr["peak"], 4),
                         "traffic": counter_traffic(f"{args.large_N}_fp16_ab_tb2", "k_step_tb2"),
                         "avg_launch_us": round(pass_us, 3),
                         "profile_avg_launch_us":
                             profile_launch_us(f"{args.large_N}_fp16_ab_tb2", "k_step_tb2")},
            "step_equivalent": {"achieved": round(rr["achieved"], 1), "frac": round(rr["frac"], 4)},
            "vs_fp32": precision_errors(pr, large, args.large_N)}
        log(f"precision: fp16 two steps per pass {pr['mlups']:.0f} MLUPS, "
            f"{rr['frac']:.3f} of the single-step HBM roofline")

    serving = None
    if not args.no_serving:
        log(f"serving: {args.serving_requests} requests x {args.serving_steps} steps")
        serving = run_serving(args.serving_requests, args.serving_steps)
        log(f"serving: p50 {serving['p50_s']:.2f} s, p99 {serving['p99_s']:.2f} s, "
            f"{serving['aggregate_mlups']:.0f} MLUPS aggregate of "
            f"{serving['offered_mlups']:.0f} offered, busy {serving['busy_frac']:.3f} "
            f"({serving['busy_frac_when_work']:.3f} while work was present)")

    cpu = None
    if not args.no_cpu:
        log("cpu baseline: C oracle on the host cores")
        cpu = cpu_baseline(args.N)
        log(f"cpu baseline: {cpu['value']:.2f} MLUPS on {cpu['cores']} threads")

    r = main_run["roofline"]
    mlups_all = [round(x["mlups"], 1) for x in main_run["repeats"]]
    out = {
        "metric": METRIC,
        "value": round(med["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(med["ms_per_step"], 4),
        "repeats": args.repeats,
        "value_repeats": mlups_all,
        "lattice_steps_per_step": args.diag_every,
        "ms_per_lattice_step": round(med["ms_per_step"] / args.diag_every, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64"}.get(args.precision, "f32"),
        "data": "synthetic",
        "config": {
            "workload": (f"forced HIT LES {args.N}^3 periodic, D3Q19 MRT-Smagorinsky C_s=0.1 "
                         f"(tau0={main_run['tau0']:.6f}, Re=2e4, U0=0.043), "
                         f"{args.precision} storage, "
                         f"{'A/B (two-array)' if args.streaming == 'ab' else 'AA (in-place)'} "
                         f"streaming, 16-mode |k|<=2 "
                         f"forcing, 1e-3 noise start; one step = {args.diag_every} lattice "
                         f"steps (one graph replay) + K_t/theta statistics + K_t map of the "
                         f"mid-z plane to host + energy spectrum E(k<={args.N // 2}) "
                         f"(lbm_snapshot_begin/_end: the next interval is enqueued before "
                         f"the host waits; every snapshot is collected inside the timed region); "
                         f"{args.steps} steps ({args.steps * args.diag_every} lattice steps, "
                         f"{args.steps} snapshots of each diagnostic) timed per repeat, "
                         f"median of {args.repeats} repeats after {args.warmup} warm-up steps"),
            "N": args.N, "precision": args.precision, "streaming": args.streaming,
            "steps_per_graph": main_run["spg"], "parallelism": "single GPU",
        },
        "roofline": {"bound": r["bound"], "achieved": round(r["achieved"], 1), "peak": r["peak"],
                     "unit": r["unit"], "frac": round(r["frac"], 4), "traffic": r["traffic"],
                     "kernel": f"k_step {args.precision} {args.streaming}",
                     "bytes_per_launch": r["bytes_per_launch"],
                     "avg_launch_us": round(main_run["avg_launch_us"], 3),
                     "avg_launch_source": "HIP events around the graph replays of the timed "
                                          "repeats (median), divided by the launches",
                     "profile_avg_launch_us": profile_launch_us(key),
                     "pattern_ceiling": main_run["pattern"],
                     "cache_resident": state_bytes < (256 << 20),
                     "device_copy_same_bytes": {
                         "GBs": round(copy_gbs, 1),
                         "frac": round(r["achieved"] / copy_gbs, 4),
                         "note": "torch device copy of the state's size on nonzero data, "
                                 "the streaming rate of this working set"}},
        "cpu_baseline": cpu,
        "kt": main_run["kt"],
        "diagnostics": {"every": args.diag_every,
                        "per_repeat": {"kt_stats": args.steps, "kt_maps": args.steps,
                                       "spectra": args.steps},
                        "lattice_steps_done": main_run["steps_done"],
                        "kt_map_mean_last": main_run["kt_map_mean"],
                        "spectrum_last_k0_25": main_run["spectrum_last"]},
    }
    if large:
        lr = large["roofline"]
        out["large"] = {"workload": f"forced HIT LES {args.large_N}^3 fp32 AA",
                        "mlups": round(large["mlups"], 1), "steps": large["steps"],
                        "ms_per_step": round(large["ms_per_step"], 4),
                        "roofline": {"bound": "hbm", "achieved": round(lr["achieved"], 1),
                                     "peak": lr["peak"], "unit": "GB/s",
                                     "frac": round(lr["frac"], 4), "traffic": lr["traffic"],
                                     "avg_launch_us": round(large["avg_launch_us"], 2),
                                     "profile_avg_launch_us":
                                         profile_launch_us(f"{args.large_N}_fp32_aa"),
                                     "pattern_ceiling": large["pattern"],
                                     "device_copy_same_bytes": {
                                         "GBs": round(large_copy_gbs, 1),
                                         "frac": round(lr["achieved"] / large_copy_gbs, 4)}},
                        "kt": large["kt"], "kt_series": large["kt_series"]}
    if large_ab:
        lr = large_ab["roofline"]
        out["large_ab"] = {"workload": f"forced HIT LES {args.large_N}^3 fp32 A/B (two arrays)",
                           "mlups": round(large_ab["mlups"], 1), "steps": large_ab["steps"],
                           "ms_per_step": round(large_ab["ms_per_step"], 4),
                           "roofline": {"bound": "hbm", "achieved": round(lr["achieved"], 1),
                                        "peak": lr["peak"], "unit": "GB/s",
                                        "frac": round(lr["frac"], 4),
                                        "traffic": counter_traffic(f"{args.large_N}_fp32_ab"),
                                        "avg_launch_us": round(large_ab["avg_launch_us"], 2),
                                        "profile_avg_launch_us":
                                            profile_launch_us(f"{args.large_N}_fp32_ab"),
                                        "pattern_ceiling": large_ab["pattern"]}}
    if large_tb2:
        lr = large_tb2["roofline"]
        # one launch = one pass = two time steps; its algorithmic bytes are one read
        # and one write of every population, the same as a single step's
        pass_us = 2 * large_tb2["avg_launch_us"]
        own = lr["bytes_per_launch"] / (pass_us * 1e-6) / 1e9
        out["large_tb2"] = {
            "workload": (f"forced HIT LES {args.large_N}^3 fp32 A/B, two time steps per pass "
                         "(intermediate level in LDS)"),
            "mlups": round(large_tb2["mlups"], 1), "steps": large_tb2["steps"],
            "ms_per_step": round(large_tb2["ms_per_step"], 4),
            "roofline": {"bound": "hbm", "achieved": round(own, 1), "peak": lr["peak"],
                         "unit": "GB/s", "frac": round(own / lr["peak"], 4),
                         "traffic": counter_traffic(f"{args.large_N}_fp32_ab_tb2", "k_step_tb2"),
                         "avg_launch_us": round(pass_us, 3),
                         "profile_avg_launch_us":
                             profile_launch_us(f"{args.large_N}_fp32_ab_tb2", "k_step_tb2")},
            "step_equivalent": {
                "achieved": round(lr["achieved"], 1), "frac": round(lr["frac"], 4),
                "note": "2*19*4 B per cell update / time: the bytes a one-step-per-pass "
                        "kernel must move for the same MLUPS"}}
    if precision:
        out["precision"] = precision
    if serving:
        out["serving"] = serving
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
