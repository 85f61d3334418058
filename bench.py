"""Benchmark of the Toeplitz-hash privacy-amplification hot path on one GPU.

Default workload (the value line): one privacy-amplification block at the
finite-size scale, n = 10^6 key bits, m = 250,000 output bits, i.i.d.
Bernoulli(0.5) key and seed bits (seeded, synthetic), plain path: each step
is one pa_toeplitz_hash call = seed and key column transforms, the fused
row pass (both row transforms, product, inverse), and the inverse column
pass with parity extraction.  Inputs are resident in HBM before timing.
The library's autotuner picks the four-step split per batch class before
the timed regions (--no-tune keeps the defaults).

Also reported on the same JSON line:
  * batched: 256 blocks of the same shape in one pa_toeplitz_hash_batched
    call (aggregate input Gb/s), each with its own seed;
  * batched_shared_seed: the same keys with one seed shared by all blocks
    (one Toeplitz matrix per distinct (n, m)), whose spectrum the library
    builds once per call;
  * batched_uneven: 256 blocks with n log-uniform in [2^18, 2^22] and
    m/n uniform in [0.05, 0.5], own seed each, one batched call (and the
    same call captured once as a graph and replayed: graph_Gbs);
  * large_block: one block of n = 12.8e6, m = 1.28e6 (plain path);
  * small_block: one block of n = 262,144, m = 65,536 (plain path);
  * modified_toeplitz: the S = (I, V) variant at the same shape, one block
    per call and 256 per batched call;
  * plan_path: the same block against a resident seed spectrum (key passes
    only), with the one-time spectrum build;
  * fft_pair: the FP64 complex-FFT form (two keys per transform) with its
    largest rounding error and its call-level HBM fraction;
  * serving: 10,000 requests (n log-uniform in [1e5, 1e7]) against 16
    resident seeds under an open-loop Poisson arrival process, p50/p99/max
    latency at offered loads 0.3/0.5/0.9 and the headline 0.7 of the
    measured saturated capacity (the headline as medians of three runs);
    every served result compared with the same request run alone;
  * roofline of the dominant kernel, from HIP events the library records
    with each launch on its own stream, over a repeat of the timed steps
    (algorithmic bytes and fp64 operations per launch / average duration);
  * parity: the timed outputs of the headline block, the small and the
    large block, every block of the 256-block batch, every 16th of the
    shared-seed batch and every 8th of the uneven batch, compared word for
    word with the CPU oracle;
  * cpu_baseline: the CPU oracle (packed AND + popcount parity) timed on
    this host's cores on full blocks of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-tune]
       [--batch B] [--serving COUNT] [--load RHO]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PA input Gb/s at n=10^6 plain vs batched; p50/p99 latency of serving loop"
HBM_PEAK_GBS = 8000.0                          # MI355X HBM3E, vendor figure
FP64_VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # CUs x SIMDs x lanes x clock: fp64 FMA/add issue rate
N_BITS, M_BITS = 1_000_000, 250_000


def progress(msg: str) -> None:
    print("bench: " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("pa_kernels.hip", "pa_internal.h"):
        with open(os.path.join(ROOT, "paper_1809_07592_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str = "plain", geometry=None):
    """Measured bytes per launch leaving the L2 (rocprofv3 FETCH_SIZE and
    WRITE_SIZE, calibrated by a copy) for one pass of a profiled workload
    ("plain", "batched" or "large"), if the counters were taken on the
    current kernel source and, when `geometry` ([log2 R, W, row_first,
    row_threads] in effect) is given, in that geometry (else None)."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    wd = d.get("workloads", {}).get(workload, {})
    if geometry is not None and wd.get("geometry") is not None and list(wd["geometry"]) != list(geometry):
        return None
    k = wd.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def geometry_in_effect(pa, L: int, batch_class: int) -> list:
    """[log2 R, W, row_first, row_threads] the library uses for L."""
    g = pa.tune_get_geometry(L, batch_class)
    return [g["log2_rows"], g["tile_width"], g["row_first"], g["row_threads"]]


def kernel_figures(prof: dict, workload: str, geometry=None) -> dict:
    """Per-pass figures from the library's profiler (HIP events recorded by
    each launch on its stream): average duration, algorithmic bytes and fp64
    operations per launch, and their fractions of the HBM and fp64 peaks;
    the measured traffic of the committed counter profile when it was taken
    on the same kernels in the same geometry."""
    out = {}
    for name, st in prof.items():
        avg_s = st["avg_ms"] * 1e-3
        b = st["alg_bytes"] / st["launches"]
        o = st["alg_ops"] / st["launches"]
        t = load_traffic(name, workload, geometry)
        out[name] = {"avg_us": st["avg_ms"] * 1e3, "launches": st["launches"], "alg_bytes_per_launch": b,
                     "alg_ops_per_launch": o, "hbm_GBs": b / avg_s / 1e9, "hbm_frac": b / avg_s / 1e9 / HBM_PEAK_GBS,
                     "fp64_Tops": o / avg_s / 1e12, "alu_frac": o / avg_s / 1e12 / FP64_VALU_PEAK_TOPS,
                     "traffic": t, "traffic_over_alg": None if t is None else t / b}
    return out


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    return e0.elapsed_time(e1) / steps, wall


def cpu_baseline(key, seed, n, m, run_s=4.0, runs=3):
    """The CPU oracle, built for this host's CPU (-march=native), timed on
    all cores of this process's affinity: `runs` runs of back-to-back full
    blocks of about run_s seconds each, the median run's rate reported; plus
    one block on one thread.  Returns (baseline dict, the oracle's output
    for the block)."""
    import oracle
    oracle.select_native()
    threads = len(os.sched_getaffinity(0))
    want = oracle.toeplitz_hash(key, n, seed, m, threads=threads)  # also warms the thread pool
    rates, samples = [], []
    for _ in range(runs):
        reps, t0 = 0, time.perf_counter()
        while True:
            oracle.toeplitz_hash(key, n, seed, m, threads=threads)
            reps += 1
            el = time.perf_counter() - t0
            if el >= run_s:
                break
        rates.append(n * reps / el / 1e9)
        samples.append("%d blocks in %.2f s" % (reps, el))
    t1 = time.perf_counter()
    oracle.toeplitz_hash(key, n, seed, m, threads=1)
    one = time.perf_counter() - t1
    rates_sorted = sorted(rates)
    return ({"value": rates_sorted[len(rates) // 2], "unit": "Gb/s", "cores": threads, "kind": "oracle",
             "sample": "median of %d runs of back-to-back full blocks of n=%d, m=%d (all %d outputs each): %s"
                       % (runs, n, m, m, "; ".join(samples)),
             "runs_Gbs": rates, "one_thread_Gbs": n / one / 1e9, "cpu_model": cpu_model(),
             "build": "gcc -O3 -march=native -fopenmp"}, want)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def batched_uneven_run(pa, wl, torch, np, count, stream, tune):
    """Uneven batch: `count` blocks with n log-uniform in [2^18, 2^22] and
    m/n uniform in [0.05, 0.5], each with its own key and seed, in one
    pa_toeplitz_hash_batched call (the library groups them by length).
    With tune, the library's autotuner first picks the batch-class geometry
    of every length on that length's own blocks (untimed); the batch is
    timed before and after."""
    shapes = wl.batched_shapes(count, 4)
    blocks = []
    for i, sh in enumerate(shapes):
        k_i, s_i = wl.key_and_seed(8, sh.n, sh.m, i)
        blocks.append((torch.from_numpy(k_i.view(np.int64)).cuda(), sh.n, torch.from_numpy(s_i.view(np.int64)).cuda(),
                       sh.m, torch.zeros(wl.words(sh.m), dtype=torch.int64, device="cuda")))

    def step():
        pa.toeplitz_hash_batched(blocks, stream=stream)

    bits = sum(sh.n for sh in shapes)
    lens = sorted({pa.transform_len(sh.n, sh.m) for sh in shapes})
    tuning = None
    if tune:
        untuned_ms, _ = time_steps(step, 5, 2, torch)
        per_len = {}
        for L in lens:
            c = sum(1 for sh in shapes if pa.transform_len(sh.n, sh.m) == L)
            r = pa.autotune(L, count=min(c, 16), reps=3, stream=stream)
            per_len[str(L)] = {"blocks": c, "log2_rows": r["log2_rows"], "tile_width": r["tile_width"],
                               "row_first": r["row_first"], "row_threads": r["row_threads"],
                               "best_us": r["best_us"], "default_us": r["default_us"]}
        tuning = {"untuned_ms_per_batch": untuned_ms, "untuned_Gbs": bits / (untuned_ms * 1e-3) / 1e9,
                  "lengths": per_len}
    # both launch forms, as direct calls and as captured graphs (the
    # library's default for both is the lanes form)
    forms = {}
    old = os.environ.get("PA_BATCH_FORM")
    try:
        for form in ("flat", "lanes"):
            os.environ["PA_BATCH_FORM"] = form
            fms, _ = time_steps(step, 5, 2, torch)
            pa.profile_collect()
            pa.profile_enable(True)
            step()
            torch.cuda.synchronize()
            launches = sum(st["launches"] for st in pa.profile_collect().values())
            pa.profile_enable(False)
            with pa.BatchGraph(blocks) as g:
                gms_f, _ = time_steps(lambda: g.launch(stream=stream), 5, 2, torch)
            forms[form] = {"Gbs": bits / (fms * 1e-3) / 1e9, "ms_per_batch": fms, "launches": launches,
                           "graph_Gbs": bits / (gms_f * 1e-3) / 1e9, "graph_ms_per_batch": gms_f}
    finally:
        if old is None:
            os.environ.pop("PA_BATCH_FORM", None)
        else:
            os.environ["PA_BATCH_FORM"] = old
    # every 8th block of the last timed run (a lanes-form graph replay,
    # with the tuned geometries), for the oracle comparison
    sample = []
    for i in range(0, count, 8):
        k_i, s_i = wl.key_and_seed(8, shapes[i].n, shapes[i].m, i)
        sample.append((k_i, s_i, shapes[i].n, shapes[i].m,
                       blocks[i][4].cpu().numpy().view(np.uint64)[: wl.words(shapes[i].m)].copy()))
    bms, gms = forms["lanes"]["ms_per_batch"], forms["lanes"]["graph_ms_per_batch"]
    return {"value": bits / (bms * 1e-3) / 1e9, "unit": "Gb/s", "blocks": count, "ms_per_batch": bms,
            "graph_Gbs": bits / (gms * 1e-3) / 1e9, "graph_ms_per_batch": gms, "forms": forms, "tuning": tuning,
            "sum_n": bits, "distinct_lengths": len(lens), "min_len": lens[0], "max_len": lens[-1],
            "shapes": "n = round(2^U(18,22)), m = max(1, round(n U(0.05, 0.5))), own seed per block"}, sample


def modified_run(pa, wl, torch, np, n, m, count, stream, steps):
    """Modified Toeplitz S = (I, V) at the headline shape: one block per call
    and `count` blocks per batched call (own key and n-1 description bits each)."""
    key = torch.from_numpy(wl.random_bits(n, wl.rng(6, wl.ROLE_KEY, 0)).view(np.int64)).cuda()
    v = torch.from_numpy(wl.random_bits(n - 1, wl.rng(6, wl.ROLE_SEED, 0)).view(np.int64)).cuda()
    out = torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")
    ms, _ = time_steps(lambda: pa.modified_toeplitz_hash(key, n, v, m, out, stream=stream), steps, 10, torch)
    blocks = []
    for i in range(count):
        k_i = torch.from_numpy(wl.random_bits(n, wl.rng(7, wl.ROLE_KEY, i)).view(np.int64)).cuda()
        v_i = torch.from_numpy(wl.random_bits(n - 1, wl.rng(7, wl.ROLE_SEED, i)).view(np.int64)).cuda()
        blocks.append((k_i, n, v_i, m, torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")))
    bms, _ = time_steps(lambda: pa.modified_toeplitz_hash_batched(blocks, stream=stream), 5, 2, torch)
    return {"plain_Gbs": n / (ms * 1e-3) / 1e9, "plain_ms_per_block": ms,
            "batched_Gbs": count * n / (bms * 1e-3) / 1e9, "batched_blocks": count, "batched_ms": bms,
            "transform_len": pa.transform_len(n - m, m),
            "definition": "y = x[0:m] ^ V x[m:n], V m x (n-m) Toeplitz of n-1 bits (Eq. 2-3)"}


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy GB/s (bytes read + written): the practical
    HBM ceiling beside the 8 TB/s vendor figure."""
    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    ms, _ = time_steps(lambda: b.copy_(a), reps, 2, torch)
    del a, b
    return {"GBs": 2 * nbytes / (ms * 1e-3) / 1e9, "bytes_copied": nbytes, "ms": ms}


def large_block_run(pa, wl, torch, np, stream, steps, tune):
    """One large block: n = 12.8e6 key bits, m = 1.28e6 outputs."""
    n, m = 12_800_000, 1_280_000
    if tune:
        pa.autotune(pa.transform_len(n, m), count=1, reps=5, stream=stream)
    k, s = wl.key_and_seed(3, n, m, 0)
    dk = torch.from_numpy(k.view(np.int64)).cuda()
    ds = torch.from_numpy(s.view(np.int64)).cuda()
    out = torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")
    step = lambda: pa.toeplitz_hash(dk, n, ds, m, out, stream=stream)
    ms, _ = time_steps(step, steps, 3, torch)
    pa.profile_collect()
    pa.profile_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    prof = pa.profile_collect()
    pa.profile_enable(False)
    L = pa.transform_len(n, m)
    g = pa.plan_info(L, *pa.tune_get(L, 0))
    res = {"value": n / (ms * 1e-3) / 1e9, "unit": "Gb/s", "ms_per_block": ms, "n": n, "m": m, "transform_len": L,
           "rows": g["rows"], "cols": g["cols"], "row_round_size": g["row_round_size"],
           "kernels": kernel_figures(prof, "large", geometry_in_effect(pa, L, 0))}
    return res, (k, s, n, m, out.cpu().numpy().view(np.uint64)[: wl.words(m)].copy())


def small_block_run(pa, wl, torch, np, stream, steps, tune):
    """One small block: n = 262,144 key bits, m = 65,536 outputs
    (several column tiles and row groups; every array fits in cache)."""
    n, m = 262_144, 65_536
    L = pa.transform_len(n, m)
    if tune:
        pa.autotune(L, count=1, reps=20, stream=stream)
    k, s = wl.key_and_seed(1, n, m, 0)
    dk = torch.from_numpy(k.view(np.int64)).cuda()
    ds = torch.from_numpy(s.view(np.int64)).cuda()
    out = torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")
    ms, _ = time_steps(lambda: pa.toeplitz_hash(dk, n, ds, m, out, stream=stream), steps, 10, torch)
    g = pa.plan_info(L, *pa.tune_get(L, 0))
    res = {"value": n / (ms * 1e-3) / 1e9, "unit": "Gb/s", "ms_per_block": ms, "n": n, "m": m, "transform_len": L,
           "rows": g["rows"], "cols": g["cols"]}
    return res, (k, s, n, m, out.cpu().numpy().view(np.uint64)[: wl.words(m)].copy())


def oracle_parity(cases):
    """Word-for-word comparison of timed GPU outputs with the CPU oracle:
    cases maps a name to a list of (key, seed, n, m, gpu_out) host arrays."""
    import numpy as np
    import oracle
    res = {}
    for name, items in cases.items():
        bad = 0
        for k, s, n, m, got in items:
            if not np.array_equal(got, oracle.toeplitz_hash(k, n, s, m)):
                bad += 1
        res[name] = {"blocks": len(items), "differing_blocks": bad, "equal": bad == 0}
    return res


def plan_run(pa, wl, torch, np, n, m, steps, stream):
    """Resident seed spectrum (pa_plan_*): one-time spectrum build, then
    per call only the key's passes (P1 on the key, P2 against the spectrum,
    P3)."""
    key, seed = wl.key_and_seed(2, n, m, 0)
    dk = torch.from_numpy(key.view(np.int64)).cuda()
    ds = torch.from_numpy(seed.view(np.int64)).cuda()
    out = torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = pa.Plan(ds, n + m - 1, stream=stream)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    ms, _ = time_steps(lambda: plan.hash(dk, n, m, out, stream=stream), steps, 10, torch)
    same = bool(torch.equal(out, pa.toeplitz_hash(dk, n, ds, m, stream=stream)))
    L = plan.transform_len
    plan.destroy()
    return {"Gbs": n / (ms * 1e-3) / 1e9, "ms_per_block": ms, "spectrum_build_ms": build_ms, "transform_len": L,
            "equals_plain": same,
            "definition": "key passes against a resident seed spectrum, n = 10^6, m = 250,000, one block per call"}


def fft_pair_run(pa, wl, torch, np, n, m, reps):
    """FP64 complex-FFT form: two keys sharing a seed per call (host waits
    for the rounding-error check each call)."""
    ka = torch.from_numpy(wl.random_bits(n, wl.rng(9, wl.ROLE_KEY, 0)).view(np.int64)).cuda()
    kb = torch.from_numpy(wl.random_bits(n, wl.rng(9, wl.ROLE_KEY, 1)).view(np.int64)).cuda()
    sd = torch.from_numpy(wl.random_bits(n + m - 1, wl.rng(9, wl.ROLE_SEED, 0)).view(np.int64)).cuda()
    oa = torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")
    ob = torch.zeros_like(oa)
    for _ in range(3):
        pa.toeplitz_hash_pair_fft(ka, kb, n, sd, m, oa, ob)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    worst, fallbacks = 0.0, 0
    for _ in range(reps):
        _, _, err, fb = pa.toeplitz_hash_pair_fft(ka, kb, n, sd, m, oa, ob)
        worst, fallbacks = max(worst, err), fallbacks + int(fb)
    el = (time.perf_counter() - t0) / reps
    L = pa.fft_pair_transform_len(n, m)
    # algorithmic HBM bytes of one call: complex doubles (16 B) written by
    # the column pass (seed and pair, 2L), read (2L) and written (L) by the
    # row pass, read (L) by the inverse column pass; plus the bit arrays, two
    # parity byte arrays and their packing
    alg = 16.0 * 6 * L + (2 * n + (n + m - 1)) / 8.0 + 2 * m * 2 + 2 * m / 8.0
    return {"Gbs": 2 * n / el / 1e9, "ms_per_pair": el * 1e3, "max_rounding_error": worst, "fallbacks": fallbacks,
            "transform_len": L, "alg_bytes_per_call": alg, "hbm_GBs_call": alg / el / 1e9,
            "hbm_frac_call": alg / el / 1e9 / HBM_PEAK_GBS,
            "definition": "two keys per complex FFT, wall time per call incl. the host-side error check; "
                          "hbm_* use that wall time"}


def serving_run(pa, wl, torch, np, count, load, budget_bytes=16 << 30, streams=4, max_inflight=512):
    """Open-loop Poisson serving run (see module docstring)."""
    n_seeds, seed_bits = 16, 1 << 24
    seeds = [torch.from_numpy(wl.random_bits(seed_bits, wl.rng(5, wl.ROLE_SEED, i)).view(np.int64)).cuda()
             for i in range(n_seeds)]
    pool = [torch.from_numpy(wl.random_bits(10_000_000, wl.rng(5, wl.ROLE_KEY, i)).view(np.int64)).cuda()
            for i in range(64)]
    reqs = wl.serving_requests(count, rate_per_s=1.0, n_seeds=n_seeds)  # unit rate: rescaled below
    offs, tot = [], 0
    for r in reqs:
        offs.append(tot)
        tot += wl.words(r.m)
    outs = torch.zeros(tot, dtype=torch.int64, device="cuda")
    # the server's streams are not ordered after torch's: the seeds, keys
    # and zeroed outputs must be complete before the server touches them
    torch.cuda.synchronize()

    def out_ptr(i):
        return outs.data_ptr() + 8 * offs[i]

    def run(srv, ids, arrivals):
        tickets, lag = [], []
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            if arrivals is not None:
                target = t0 + arrivals[i]
                while time.perf_counter() < target:
                    pass
                lag.append(max(0.0, time.perf_counter() - target) * 1e6)
            tickets.append(srv.submit(ids[r.seed_id], pool[i % len(pool)].data_ptr(), r.n, r.m, out_ptr(i)))
        srv.drain()
        el = time.perf_counter() - t0
        lat = [srv.latency_us(t) + (lag[i] if lag else 0.0) for i, t in enumerate(tickets)]
        return el, lat

    bits = sum(r.n for r in reqs)
    with pa.Server(budget_bytes, max_inflight=max_inflight, streams=streams) as srv:
        ids = [srv.register_seed(sd, seed_bits) for sd in seeds]
        run(srv, ids, None)                    # warm-up: builds the resident seed spectra
        run_sat_el, _ = run(srv, ids, None)    # saturated (all submitted at once): capacity
        cap_gbs = bits / run_sat_el / 1e9
        unit_arrivals = np.array([r.arrival_s for r in reqs])   # unit-rate Poisson times, rescaled per load
        # cold start: a fresh server at the headline load, every (seed,
        # length) spectrum built on first use while requests are served
        rate0 = load * cap_gbs * 1e9 / (bits / len(reqs))
        with pa.Server(budget_bytes, max_inflight=max_inflight, streams=streams) as cold_srv:
            cold_ids = [cold_srv.register_seed(sd, seed_bits) for sd in seeds]
            cel, clat = run(cold_srv, cold_ids, unit_arrivals / rate0)
            cst = cold_srv.stats()
        cla = np.array(clat) / 1e3
        cold = {"offered_load": load, "Gbs": bits / cel / 1e9, "p50_ms": float(np.percentile(cla, 50)),
                "p99_ms": float(np.percentile(cla, 99)), "max_ms": float(cla.max()),
                "spectra_built": cst["spectra_built"], "spectra_evicted": cst["spectra_evicted"]}
        progress("serving cold start at load %.1f: p50 %.3f ms p99 %.3f ms (%d spectra built on demand)"
                 % (load, cold["p50_ms"], cold["p99_ms"], cold["spectra_built"]))
        sweep = []
        for rho in [x for x in (0.3, 0.5, 0.9) if x != load] + [load]:   # headline load last
            rate = rho * cap_gbs * 1e9 / (bits / len(reqs))
            el, lat = run(srv, ids, unit_arrivals / rate)
            la = np.array(lat) / 1e3
            sweep.append({"offered_load": rho, "Gbs": bits / el / 1e9, "p50_ms": float(np.percentile(la, 50)),
                          "p99_ms": float(np.percentile(la, 99)), "max_ms": float(la.max())})
            progress("serving load %.1f: p50 %.3f ms p99 %.3f ms" % (rho, sweep[-1]["p50_ms"], sweep[-1]["p99_ms"]))
        # the headline load twice more: open-loop tails vary from run to run,
        # so the headline p50/p99 are the medians of three runs
        repeats = [sweep[-1]]
        for _ in range(2):
            el2, lat2 = run(srv, ids, unit_arrivals / rate)
            la2 = np.array(lat2) / 1e3
            repeats.append({"offered_load": load, "Gbs": bits / el2 / 1e9, "p50_ms": float(np.percentile(la2, 50)),
                            "p99_ms": float(np.percentile(la2, 99)), "max_ms": float(la2.max())})
        progress("serving load %.1f, three runs: p99 %s ms" % (load, " / ".join("%.3f" % r["p99_ms"] for r in repeats)))
        st = srv.stats()
    torch.cuda.synchronize()
    served = outs.cpu()
    mism = 0
    for i, r in enumerate(reqs):
        alone = pa.toeplitz_hash(pool[i % len(pool)], r.n, seeds[r.seed_id], r.m)
        if not torch.equal(alone.cpu()[: wl.words(r.m)], served[offs[i]: offs[i] + wl.words(r.m)]):
            mism += 1
    lat = np.array(lat) / 1e3
    med = lambda k: float(np.median([r[k] for r in repeats]))
    return {"requests": len(reqs), "offered_load": load, "arrival_rate_per_s": rate, "value": med("Gbs"),
            "unit": "Gb/s", "saturated_Gbs": cap_gbs, "p50_ms": med("p50_ms"), "p99_ms": med("p99_ms"),
            "max_ms": max(r["max_ms"] for r in repeats), "headline_runs": repeats,
            "headline": "medians of three runs at the offered load (max: the largest of the three)",
            "first_run_p50_ms": float(np.percentile(lat, 50)), "makespan_s": el,
            "budget_GiB": budget_bytes / 2**30, "streams": streams, "max_inflight": max_inflight,
            "peak_inflight": st["peak_inflight"], "batches": st["batches"],
            "peak_bytes_in_flight": st["peak_bytes_in_flight"], "mismatches_vs_alone": mism,
            "load_sweep": sweep, "cold_start": cold, "spectrum_bytes": st["spectrum_bytes"],
            "spectra_resident": st["spectra_resident"],
            "latency": "completion minus scheduled Poisson arrival (open loop)"}


def only_run(pa, wl, torch, np, args):
    """One workload, for profilers: the same inputs, autotuning and launch
    form as the full run, --steps timed steps after --warmup, then --steps
    more with the library's per-launch event timing (printed per pass)."""
    stream = torch.cuda.current_stream()
    if args.only in ("plain", "batched", "large"):
        n, m = (12_800_000, 1_280_000) if args.only == "large" else (N_BITS, M_BITS)
        count = args.batch if args.only == "batched" else 1
        L = pa.transform_len(n, m)
        if not args.no_tune:
            pa.autotune(L, count=count, reps=3 if count > 1 else 20, stream=stream)
        cfg = {"plain": 2, "batched": 4, "large": 3}[args.only]
        blocks = []
        for i in range(count):
            k, s_ = wl.key_and_seed(cfg, n, m, i)
            blocks.append((torch.from_numpy(k.view(np.int64)).cuda(), n, torch.from_numpy(s_.view(np.int64)).cuda(),
                           m, torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")))
        if count == 1:
            b = blocks[0]
            step = lambda: pa.toeplitz_hash(b[0], n, b[2], m, b[4], stream=stream)
        else:
            step = lambda: pa.toeplitz_hash_batched(blocks, stream=stream)
        geo = pa.tune_get_geometry(L, 0 if count == 1 else 1)
        bits = n * count
    else:
        shapes = wl.batched_shapes(args.batch, 4)
        blocks = []
        for i, sh in enumerate(shapes):
            k, s_ = wl.key_and_seed(8, sh.n, sh.m, i)
            blocks.append((torch.from_numpy(k.view(np.int64)).cuda(), sh.n, torch.from_numpy(s_.view(np.int64)).cuda(),
                           sh.m, torch.zeros(wl.words(sh.m), dtype=torch.int64, device="cuda")))
        step = lambda: pa.toeplitz_hash_batched(blocks, stream=stream)
        geo = {"lengths": len({pa.transform_len(sh.n, sh.m) for sh in shapes})}
        bits = sum(sh.n for sh in shapes)
    ms, _ = time_steps(step, args.steps, args.warmup, torch)
    # the same steps again with the library's per-launch events, so that a
    # profiler's kernel trace of this process can be set beside them
    pa.profile_collect()
    pa.profile_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = pa.profile_collect()
    pa.profile_enable(False)
    print(json.dumps({"only": args.only, "ms_per_step": ms, "Gbs": bits / (ms * 1e-3) / 1e9, "geometry": geo,
                      "steps": args.steps, "kernel_source_hash": kernel_source_hash(),
                      "event_avg_us": {k: v["avg_ms"] * 1e3 for k, v in prof.items()}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in default splits")
    ap.add_argument("--serving", type=int, default=10000, help="requests in the serving run (0: skip)")
    ap.add_argument("--load", type=float, default=0.7, help="offered load as a fraction of saturated capacity")
    ap.add_argument("--only", choices=["plain", "batched", "large", "uneven"],
                    help="run one workload for --steps steps (after the same untimed autotuning as the full "
                         "run) and print its time and geometry: for profiling runs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only (independent blocks shard by routing whole blocks to "
              "GPUs; no collective is involved); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1809_07592_amd as pa
    from paper_1809_07592_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.ones(2**28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 4, "copy_probe_bytes_written": b.numel() * 4}))
        return
    pa.lib()  # fails loudly if the HIP library is missing
    if args.only:
        only_run(pa, wl, torch, np, args)
        return
    n, m = N_BITS, M_BITS
    key, seed = wl.key_and_seed(2, n, m, 0)
    dk = torch.from_numpy(key.view(np.int64)).cuda()
    ds = torch.from_numpy(seed.view(np.int64)).cuda()
    out = torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        pa.toeplitz_hash(dk, n, ds, m, out, stream=stream)

    L = pa.transform_len(n, m)
    tuning = {"transform_len": L}
    if not args.no_tune:
        # the library's autotuner picks the (R, W) split per batch class; untimed
        tuning["plain"] = pa.autotune(L, count=1, reps=20, stream=stream)
        progress("autotune plain: log2_rows=%d tile_width=%d" % (tuning["plain"]["log2_rows"],
                                                                  tuning["plain"]["tile_width"]))
    tuning["plain_geometry"] = pa.plan_info(L, *pa.tune_get(L, 0))
    ms, wall = time_steps(step, args.steps, args.warmup, torch)
    value = n / (ms * 1e-3) / 1e9
    progress("plain path: %.3f ms/step, %.2f Gb/s" % (ms, value))

    # Per-kernel timing: the same steps again with the library's event
    # recording on (HIP events carried by each kernel launch on its stream,
    # hipExtLaunchKernel).  A separate pass, because recording events costs
    # the host about 10 us per launch, which would throttle the 40 us step.
    pa.profile_collect()
    pa.profile_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = pa.profile_collect()
    pa.profile_enable(False)
    kernels = kernel_figures(prof, "plain", geometry_in_effect(pa, L, 0))
    for name, st in prof.items():
        kernels[name]["share_of_step"] = st["total_ms"] / st["launches"] / ms
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"])
    kd = kernels[dom]
    bound = "alu" if kd["alu_frac"] >= kd["hbm_frac"] else "hbm"
    traffic = kd["traffic"]
    if bound == "alu":
        roofline = {"bound": "alu", "kernel": dom, "achieved": kd["fp64_Tops"], "peak": FP64_VALU_PEAK_TOPS,
                    "unit": "Tops/s (fp64 FMA/add)", "frac": kd["alu_frac"], "traffic": traffic}
    else:
        roofline = {"bound": "hbm", "kernel": dom, "achieved": kd["hbm_GBs"], "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": kd["hbm_frac"], "traffic": traffic}
    roofline_hbm = {"kernel": dom, "achieved": kd["hbm_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": kd["hbm_frac"]}

    # batched: args.batch blocks of the same shape in one submission
    batched = None
    batched_io = []
    shared, shared_io = None, []
    if args.batch > 0:
        blocks = []
        for i in range(args.batch):
            k_i, s_i = wl.key_and_seed(4, n, m, i)
            batched_io.append((k_i, s_i, n, m))
            blocks.append((torch.from_numpy(k_i.view(np.int64)).cuda(), n, torch.from_numpy(s_i.view(np.int64)).cuda(),
                           m, torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")))

        def bstep():
            pa.toeplitz_hash_batched(blocks, stream=stream)

        if not args.no_tune:
            tuning["batched"] = pa.autotune(L, count=args.batch, reps=3, stream=stream)
            progress("autotune batched: log2_rows=%d tile_width=%d" % (tuning["batched"]["log2_rows"],
                                                                        tuning["batched"]["tile_width"]))

        tuning["batched_geometry"] = pa.plan_info(L, *pa.tune_get(L, 1))
        bsteps = max(3, args.steps // 40)
        bms, _ = time_steps(bstep, bsteps, 2, torch)
        batched_io = [io + (b[4].cpu().numpy().view(np.uint64)[: wl.words(m)].copy(),)
                      for io, b in zip(batched_io, blocks)]
        with pa.BatchGraph(blocks) as bgraph:
            gms, _ = time_steps(lambda: bgraph.launch(stream=stream), bsteps, 2, torch)
        pa.profile_enable(True)
        bstep()
        torch.cuda.synchronize()
        bprof = pa.profile_collect()
        pa.profile_enable(False)
        bk = kernel_figures(bprof, "batched", geometry_in_effect(pa, L, 1))
        batched = {"value": args.batch * n / (bms * 1e-3) / 1e9, "unit": "Gb/s", "blocks": args.batch,
                   "ms_per_batch": bms, "kernels": bk,
                   "speedup_vs_plain": args.batch * n / (bms * 1e-3) / 1e9 / value,
                   "graph_Gbs": args.batch * n / (gms * 1e-3) / 1e9, "graph_ms_per_batch": gms}
        del blocks
        progress("batched: %.3f ms per %d blocks, %.2f Gb/s" % (bms, args.batch, batched["value"]))

        # the same blocks with one seed shared by all of them (one Toeplitz
        # matrix per distinct (n, m), the uneven configuration's rule): the
        # library builds the seed's spectrum once per call and runs every key
        # against it
        shared_seed = wl.random_bits(n + m - 1, wl.rng(4, wl.ROLE_SEED, 1 << 20))
        dss = torch.from_numpy(shared_seed.view(np.int64)).cuda()
        sblocks = [(torch.from_numpy(io[0].view(np.int64)).cuda(), n, dss, m,
                    torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")) for io in batched_io]

        def sstep():
            pa.toeplitz_hash_batched(sblocks, stream=stream)

        sms, _ = time_steps(sstep, bsteps, 2, torch)
        pa.profile_enable(True)
        sstep()
        torch.cuda.synchronize()
        sprof = pa.profile_collect()
        pa.profile_enable(False)
        shared_io = [(batched_io[i][0], shared_seed, n, m, sblocks[i][4].cpu().numpy().view(np.uint64)[: wl.words(m)].copy())
                     for i in range(0, args.batch, 16)]
        shared = {"value": args.batch * n / (sms * 1e-3) / 1e9, "unit": "Gb/s", "blocks": args.batch,
                  "ms_per_batch": sms, "speedup_vs_own_seeds": bms / sms,
                  "kernels": kernel_figures(sprof, "batched_shared_seed", geometry_in_effect(pa, L, 1))}
        del sblocks, dss
        progress("batched, one shared seed: %.3f ms per %d blocks, %.2f Gb/s" % (sms, args.batch, shared["value"]))

    uneven, uneven_io = (batched_uneven_run(pa, wl, torch, np, args.batch, stream, not args.no_tune)
                         if args.batch > 0 else (None, []))
    if uneven is not None:
        progress("batched uneven: %.3f ms per %d blocks, %.2f Gb/s" % (uneven["ms_per_batch"], args.batch,
                                                                       uneven["value"]))
    modified = modified_run(pa, wl, torch, np, n, m, args.batch, stream, args.steps) if args.batch > 0 else None
    if modified is not None:
        progress("modified Toeplitz: plain %.2f Gb/s, batched %.2f Gb/s" % (modified["plain_Gbs"],
                                                                          modified["batched_Gbs"]))
    planr = plan_run(pa, wl, torch, np, n, m, args.steps, stream)
    progress("plan path: %.2f Gb/s (spectrum built once in %.2f ms)" % (planr["Gbs"], planr["spectrum_build_ms"]))
    large, large_io = large_block_run(pa, wl, torch, np, stream, 20, not args.no_tune)
    progress("large block (n=12.8e6): %.2f Gb/s" % large["value"])
    small, small_io = small_block_run(pa, wl, torch, np, stream, args.steps, not args.no_tune)
    progress("small block (n=262144): %.2f Gb/s" % small["value"])
    fftp = fft_pair_run(pa, wl, torch, np, n, m, 50)
    progress("FFT pair: %.2f Gb/s, %.2f of HBM peak per call, max rounding error %.3g"
             % (fftp["Gbs"], fftp["hbm_frac_call"], fftp["max_rounding_error"]))
    serving = serving_run(pa, wl, torch, np, args.serving, args.load) if args.serving > 0 else None
    if serving is not None:
        progress("serving: done")
    copy = copy_bandwidth(torch)
    progress("device copy: %.0f GB/s" % copy["GBs"])
    alu = pa.alu_probe(stream)
    alu["fma_frac_of_peak"] = alu["fma_Tops"] / FP64_VALU_PEAK_TOPS
    progress("fp64 FMA: %.1f T/s, modular products: %.0f G/s" % (alu["fma_Tops"], alu["mulmod_Gops"]))
    # the fixed cost of each of the plain step's three launches (an empty
    # kernel of the same shape, back to back), and what one launch with
    # grid barriers or per-tile releases would cost instead
    pg = tuning["plain_geometry"]
    launch = {"colfwd_us": pa.launch_probe(2 * pg["col_tiles"], pg["col_threads"], stream=stream),
              "rowconv_us": pa.launch_probe(pg["rows"], pg["row_threads"], stream=stream),
              "colinv_us": pa.launch_probe(pg["col_tiles"], pg["col_threads"], stream=stream)}
    launch["step_floor_us"] = launch["colfwd_us"] + launch["rowconv_us"] + launch["colinv_us"]
    phase = pa.phase_probe(stream)
    progress("launch floor of the plain step: %.1f us; three phases %.1f us as launches, %.1f us with grid barriers"
             % (launch["step_floor_us"], phase["three_launches_us"], phase["cooperative_grid_sync_us"]))
    # the timed outputs against the CPU oracle, word for word
    plain_out = out.cpu().numpy().view(np.uint64)[: wl.words(m)].copy()
    cases = {"small_block_n262144": [small_io], "large_block_n12800000": [large_io]}
    if batched_io:
        cases["batched_256_n1e6"] = batched_io
    if shared_io:
        cases["batched_256_n1e6_shared_seed_every_16th_block"] = shared_io
    if uneven_io:
        cases["batched_uneven_every_8th_block"] = uneven_io
    parity = oracle_parity(cases)
    if args.no_cpu:
        import oracle
        want = oracle.toeplitz_hash(key, n, seed, m)
        cpu = None
    else:
        cpu, want = cpu_baseline(key, seed, n, m)
        progress("cpu baseline: %.4g %s" % (cpu["value"], cpu["unit"]))
    parity = dict({"headline_block_n1000000": {"blocks": 1, "differing_blocks": int(not np.array_equal(plain_out, want)),
                                              "equal": bool(np.array_equal(plain_out, want))}}, **parity)
    parity_ok = all(v["equal"] for v in parity.values())
    progress("parity against the oracle: %s" % ("all equal" if parity_ok else parity))
    line = {
        "metric": METRIC, "value": value, "unit": "Gb/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "single PA block, plain path: n=1000000 key bits, m=250000 output bits, "
                               "Bernoulli(0.5) key and seed bits, packed uint64", "n": n, "m": m,
                   "transform_len": pa.transform_len(n, m)},
        "wall_s_timed_region": wall,
        "parity": parity_ok, "parity_detail": parity,
        "roofline": roofline, "roofline_hbm": roofline_hbm, "kernels": kernels,
        "batched": batched, "batched_shared_seed": shared, "batched_uneven": uneven, "large_block": large, "small_block": small, "modified_toeplitz": modified,
        "plan_path": planr, "fft_pair": fftp,
        "serving": serving,
        "tuning": tuning, "copy_bandwidth": copy, "alu_probe": alu, "launch_probe": launch, "phase_probe": phase,
        "cpu_baseline": cpu,
        "context": {"paper_Mbps": 116, "paper_setting": "Virtex-6 FPGA at 200 MHz, modified Toeplitz, float FFT, "
                    "n = 2^20 (input rate; a different variant and hardware, so not a target)"},
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
