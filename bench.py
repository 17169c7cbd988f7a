"""Benchmark of the Falcon hot path on one MI355X.

One step = one pass of the whole path over the workload already resident in
HBM: compress (integer conversion, delta + zigzag, adaptive bit-plane
encoding sized in a first pass, a prefix sum of the chunk sizes, the chunks
written at their offsets in a second pass) followed by decompress (offsets,
bit-plane decoding, inverse transforms).  Workload: 268,435,456
float64 sensor-like values (2 GiB, 65,536-value segments at 1-6 decimal
places, 1% full-precision outliers, specials at 1e-5), seeded synthetic.

Prints one JSON line.  `value` is the round-trip throughput: original bytes
per step divided by the step time.  The timed steps are asynchronous calls
on one stream (falcon_compress, then falcon_decompress_n with the count and
dtype just compressed) with one wait at the end of the region; every
kernel's duration comes from the HIP events the library records for each
call, read afterwards (falcon_call_stage_ms).  Compress and decompress
throughputs (the paper's CT and DT, here device-resident) and the
compression ratio are reported beside it.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "compress/decompress GB/s + ratio; batched vs per-series launch; p99 latency"
WORKLOAD = ("sensor_f64: 268,435,456 float64 values (2 GiB) in 65,536-value segments, "
            "1-6 decimal places per segment, sinusoid + random walk, 1% full-precision "
            "outliers, NaN/+-Inf/-0.0/subnormal at 1e-5")


def kernel_source_digest():
    """Digest of the device code (every .hip source and the device headers)
    and of the build script that holds its compile flags."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_04140_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith(".hip") or name in ("codec_device.hpp", "codec_kernels.hpp"):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(ROOT, "paper_2511_04140_amd", "build.py"), "rb") as f:
        h.update(b"build.py\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, per_launch_algo_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_digest") != kernel_source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def _cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def _oracle_rate(x, threads, budget_s, step=1024 * 1025):
    """Compression then decompression of chunk-aligned slices of x's leading
    values through the oracle on `threads` threads (each slice a stream of
    its own; the oracle's C calls release the GIL), in rounds of `threads`
    slices until about budget_s seconds have passed.  Every round trip is
    checked.  Returns (values done, compress seconds, decompress seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle
    import numpy as np
    done = 0
    tc = td = 0.0
    t_start = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        while done < x.size and time.perf_counter() - t_start < budget_s:
            parts = [x[done + k * step: done + (k + 1) * step] for k in range(threads)]
            parts = [p for p in parts if p.size]
            t0 = time.perf_counter()
            ss = list(ex.map(oracle.compress, parts))
            t1 = time.perf_counter()
            ys = list(ex.map(oracle.decompress, ss))
            t2 = time.perf_counter()
            for p_, y in zip(parts, ys):
                assert np.array_equal(y.view(np.uint8), p_.view(np.uint8))
            tc += t1 - t0
            td += t2 - t1
            done += sum(p_.size for p_ in parts)
    return done, tc, td


def cpu_baseline(x, x32=None, budget_s=8.0):
    """The oracle as it stands on the host's cores (at most 16 threads, the
    host share of one GPU), on the leading values of the benchmark workload
    (a bounded sample, about budget_s seconds), compress + decompress; the
    same on one thread, and on the float32 workload when given."""
    model, nproc = _cpu_info()
    threads = max(1, min(16, nproc))
    done, tc, td = _oracle_rate(x, threads, budget_s)
    nbytes = done * x.itemsize
    out = {
        "value": round(nbytes / (tc + td) / 1e9, 6),
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {done:,} values ({nbytes / 2**20:.0f} MiB) of the workload in slices of "
                  f"1,048,576+ values, compress + decompress, {threads} threads",
        "compress_gbps": round(nbytes / tc / 1e9, 6),
        "decompress_gbps": round(nbytes / td / 1e9, 6),
        "cpu_model": model,
        "nproc": nproc,
    }
    d1, c1, e1 = _oracle_rate(x, 1, budget_s / 4)
    out["one_thread"] = {"values": d1, "gbps": round(d1 * x.itemsize / (c1 + e1) / 1e9, 6),
                         "compress_gbps": round(d1 * x.itemsize / c1 / 1e9, 6),
                         "decompress_gbps": round(d1 * x.itemsize / e1 / 1e9, 6)}
    if x32 is not None:
        d2, c2, e2 = _oracle_rate(x32, threads, budget_s / 2)
        out["float32"] = {"values": d2, "threads": threads, "gbps": round(d2 * 4 / (c2 + e2) / 1e9, 6),
                          "compress_gbps": round(d2 * 4 / c2 / 1e9, 6),
                          "decompress_gbps": round(d2 * 4 / e2 / 1e9, 6)}
    return out


def oracle_small_case(threads=None):
    """The 2^20-value walk (Gaussian steps from 100.0, two decimals) through
    the oracle: compression and decompression seconds on one thread, then on
    `threads` threads over chunk-aligned slices of the same values (each
    slice a stream of its own; the oracle's C calls release the GIL).  Every
    round trip is checked."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle
    import numpy as np
    from paper_2511_04140_amd import workloads as W
    x = W.walk_f64(1 << 20, seed=1)
    t0 = time.perf_counter()
    s = oracle.compress(x)
    t1 = time.perf_counter()
    y = oracle.decompress(s)
    t2 = time.perf_counter()
    assert np.array_equal(y.view(np.uint8), x.view(np.uint8))
    nt = threads or min(16, os.cpu_count() or 1)
    nc = (x.size + 1024) // 1025
    cuts = [min(x.size, 1025 * (nc * k // nt)) for k in range(nt + 1)]
    parts = [x[cuts[k]:cuts[k + 1]] for k in range(nt)]
    with ThreadPoolExecutor(nt) as ex:
        t3 = time.perf_counter()
        ss = list(ex.map(oracle.compress, parts))
        t4 = time.perf_counter()
        ys = list(ex.map(oracle.decompress, ss))
        t5 = time.perf_counter()
    assert all(np.array_equal(a.view(np.uint8), b.view(np.uint8)) for a, b in zip(parts, ys))
    return {"workload": "walk_f64: 1,048,576 float64 values (8 MiB), Gaussian walk from 100.0, 2 decimals",
            "ratio": round(len(s) / x.nbytes, 6),
            "one_thread": {"compress_s": round(t1 - t0, 4), "decompress_s": round(t2 - t1, 4)},
            "threads": nt,
            "all_threads": {"compress_s": round(t4 - t3, 4), "decompress_s": round(t5 - t4, 4)}}


def host_pipeline(codec, x, torch, reps=2):
    """Host -> host through the stream pipeline (Alg. 1): the default
    geometry (4 streams, 2048-chunk batches) from pinned and from pageable
    host buffers, and the paper's setting (16 streams, 4096 chunks) from
    pinned buffers; best of reps, GB/s of original bytes."""
    res = {}
    for label, ns, bc, pinned in (("pinned", 4, 2048, True), ("pageable", 4, 2048, False),
                                  ("pinned_16x4096", 16, 4096, True)):
        codec.set_pipeline(ns, bc)
        xh = torch.from_numpy(x)
        if pinned:
            xh = xh.pin_memory()
        sbuf = torch.empty(codec_bound(x), dtype=torch.uint8, pin_memory=pinned)
        ybuf = torch.empty(x.size, dtype=xh.dtype, pin_memory=pinned)
        tc = td = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            s = codec.compress_host(xh, out=sbuf)
            t1 = time.perf_counter()
            y = codec.decompress_host(s, out=ybuf)
            t2 = time.perf_counter()
            tc, td = min(tc, t1 - t0), min(td, t2 - t1)
        assert torch.equal(y.view(torch.uint8), xh.view(torch.uint8)), "host round trip failed"
        res[label] = {"n_streams": ns, "batch_chunks": bc,
                      "compress_gbps": round(x.nbytes / tc / 1e9, 3),
                      "decompress_gbps": round(x.nbytes / td / 1e9, 3)}
        del xh, sbuf, ybuf, s, y
    codec.set_pipeline()
    return res


def batched(codec, torch, reps=5):
    """10,000 series of uneven lengths and mixed dtypes (about 4 GB),
    device-resident: the one-series-per-launch path (falcon_compress_each /
    falcon_decompress_each: a C loop of asynchronous calls, one launch
    sequence per series, one wait at the end) against one tuned,
    graph-captured batch plan over all of them; both write to buffers of
    their own and must give identical bytes."""
    import numpy as np
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    dev = codec.device
    xs = W.batch_series()
    align = lambda v: (v + 255) // 256 * 256
    in_off, out_off, bounds = [], [], []
    ti = to = 0
    for x in xs:
        in_off.append(ti)
        ti += align(x.nbytes)
        b = C.compress_bound(x.size, torch.float64 if x.dtype == np.float64 else torch.float32)
        bounds.append(b)
        out_off.append(to)
        to += align(b)
    host = np.zeros(ti, np.uint8)
    for x, o in zip(xs, in_off):
        host[o:o + x.nbytes] = x.view(np.uint8)
    xin = torch.from_numpy(host).to(dev)
    del host
    tdt = lambda x: torch.float64 if x.dtype == np.float64 else torch.float32
    xv = [xin[o:o + x.nbytes].view(tdt(x)) for x, o in zip(xs, in_off)]
    outs = {k: torch.zeros(to, dtype=torch.uint8, device=dev) for k in ("loop", "plan")}
    ov = {k: [outs[k][o:o + b] for o, b in zip(out_off, bounds)] for k in outs}
    raw = sum(x.nbytes for x in xs)

    def wall(fn, r):
        best = float("inf")
        for _ in range(r):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    torch.cuda.synchronize()
    streams_loop = codec.compress_each(xv, outs=ov["loop"])
    t_loop = wall(lambda: codec.compress_each(xv, outs=ov["loop"]), 2)
    lens = [s_.numel() for s_ in streams_loop]
    plan = codec.plan_compress(xv, outs=ov["plan"], tune=True, graph=True)
    info = plan.info()
    plan.run(fetch=False)
    t_plan = wall(lambda: plan.run(fetch=False), reps)
    streams = plan.run()
    identical = [s_.numel() for s_ in streams] == lens and torch.equal(outs["loop"], outs["plan"])
    clen = sum(lens)
    # decompression of the same streams
    dv = {k: torch.zeros(ti, dtype=torch.uint8, device=dev) for k in ("loop", "plan")}
    dviews = {k: [dv[k][o:o + x.nbytes].view(tdt(x)) for x, o in zip(xs, in_off)] for k in dv}
    counts, dts = [x.size for x in xs], [tdt(x) for x in xs]
    codec.decompress_each(streams, counts, dts, outs=dviews["loop"])
    t_dloop = wall(lambda: codec.decompress_each(streams, counts, dts, outs=dviews["loop"]), 2)
    dplan = codec.plan_decompress(streams, counts, dts, outs=dviews["plan"], tune=True, graph=True)
    dinfo = dplan.info()
    dplan.run(fetch=False)
    t_dplan = wall(lambda: dplan.run(fetch=False), reps)
    identical = identical and torch.equal(dv["loop"], dv["plan"]) and torch.equal(dv["plan"], xin)
    sizes = sorted(x.size for x in xs)
    algo = raw + clen
    frac = lambda t: round(algo / t / 1e9 / HBM_PEAK_GBPS, 4)
    res = {
        "series": len(xs), "f64_series": int(sum(x.dtype == np.float64 for x in xs)),
        "values_min_median_max": [sizes[0], sizes[len(sizes) // 2], sizes[-1]],
        "bytes": raw, "stream_bytes": clen, "ratio": round(clen / raw, 6),
        "timing": "wall clock around each whole call, device synchronised before and after, best of runs; the "
                  "per-series path is falcon_compress_each / falcon_decompress_each (a C loop of asynchronous "
                  "calls, one wait), the batch path replays one tuned HIP graph",
        "compress": {"per_series_gbps": round(raw / t_loop / 1e9, 3),
                     "batched_gbps": round(raw / t_plan / 1e9, 3),
                     "speedup": round(t_loop / t_plan, 2),
                     "batched_hbm_frac": frac(t_plan), "per_series_hbm_frac": frac(t_loop),
                     "plan": {k: info[k] for k in ("split", "waves_per_group", "grid_percent", "candidates", "form")}},
        "decompress": {"per_series_gbps": round(raw / t_dloop / 1e9, 3),
                       "batched_gbps": round(raw / t_dplan / 1e9, 3),
                       "speedup": round(t_dloop / t_dplan, 2),
                       "batched_hbm_frac": frac(t_dplan), "per_series_hbm_frac": frac(t_dloop),
                       "plan": {k: dinfo[k] for k in ("split", "grid_percent", "candidates")}},
        "identical": bool(identical),
    }
    plan.close()
    dplan.close()
    return res


def serving(codec, torch, n_req=20000, rhos=(0.5, 0.8, 0.95), budget=64 << 30):
    """Poisson arrivals, 70% compress / 30% decompress, payloads 4 KB-64 MB
    log-uniform, float32/float64.  Two paths, each with the same HBM budget:
    the plain FIFO (one request per launch, one stream) and the served loop
    (continuous batching over 4 streams).  Each is first driven at
    saturation (every request submitted at once), then at offered loads of
    rho times its own saturation rate; both are also driven at two loads
    between the FIFO's saturation and the served loop's (geometrically
    spaced), where the FIFO is overloaded.  Latency = completion - submission
    of each request."""
    import numpy as np
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    dev = codec.device
    ps = W.serving_payloads()
    pd = [torch.from_numpy(p).to(dev) for p in ps]
    streams = [codec.compress(p).clone() for p in pd]
    rng = np.random.default_rng([6, 0])
    is_c = rng.random(n_req) < 0.7
    idx = rng.integers(0, len(ps), n_req)
    nbytes = np.array([p.nbytes for p in ps])
    total_bytes = int(nbytes[idx].sum())
    gaps = rng.exponential(1.0, n_req)  # unit-rate Poisson gaps, scaled per load

    def run(srv, lam):
        arrivals = None if lam is None else np.cumsum(gaps / lam)
        got = []
        t_start = time.perf_counter()
        for i in range(n_req):
            if arrivals is not None:
                t_next = t_start + arrivals[i]
                while time.perf_counter() < t_next:
                    for c in srv.poll(0):
                        srv.release(c)
                        got.append(c)
            k = int(idx[i])
            if is_c[i]:
                srv.submit_compress(pd[k], tag=i)
            else:
                srv.submit_decompress(streams[k], pd[k].numel(), pd[k].dtype, tag=i)
        t_sub = time.perf_counter() - t_start
        while len(got) < n_req:
            for c in srv.poll(20):
                srv.release(c)
                got.append(c)
        assert all(c["status"] == 0 for c in got)
        lat = np.array([c["complete_us"] - c["submit_us"] for c in got])
        span = (max(c["complete_us"] for c in got) - min(c["submit_us"] for c in got)) * 1e-6
        out = {"p50_us": round(float(np.percentile(lat, 50)), 1), "p99_us": round(float(np.percentile(lat, 99)), 1),
               "mean_us": round(float(lat.mean()), 1), "gbps": round(total_bytes / span / 1e9, 3),
               "req_per_s": round(n_req / span, 1)}
        if lam is not None:
            out["offered_req_per_s"] = round(lam, 1)
            out["submitted_req_per_s"] = round(n_req / t_sub, 1)
        return out

    res = {"requests": n_req, "payloads": len(ps), "mean_payload_mb": round(float(nbytes.mean()) / 1e6, 3),
           "hbm_budget_gib": budget >> 30, "fifo": {}, "served": {}}
    cfgs = {"fifo": dict(lanes=1, max_batch=1), "served": dict(lanes=4, max_batch=256)}
    sat = {}
    for k, cfg in cfgs.items():
        srv = C.Server(codec, hbm_budget=budget, **cfg)
        sat[k] = run(srv, None)
        res[k]["saturation"] = sat[k]
        for rho in rhos:
            res[k][f"rho_{rho}"] = run(srv, rho * sat[k]["req_per_s"])
        srv.close()
        torch.cuda.empty_cache()
    f_sat, s_sat = sat["fifo"]["req_per_s"], sat["served"]["req_per_s"]
    if s_sat > f_sat:
        res["between"] = {}
        for j in (1, 2):
            lam = f_sat * (s_sat / f_sat) ** (j / 3)
            row = {}
            for k, cfg in cfgs.items():
                srv = C.Server(codec, hbm_budget=budget, **cfg)
                row[k] = run(srv, lam)
                srv.close()
                torch.cuda.empty_cache()
            res["between"][f"{lam:.0f}_req_per_s"] = row
    return res


def float32_case(codec, torch, reps=10):
    """The 2 GiB float32 workload (2^29 values: low-precision sinusoid
    segments, then two interpolated 3-D fields at full precision):
    device-resident compression and decompression (median kernel time of
    reps calls) and host -> host through the pipeline, as for the float64
    workload."""
    from paper_2511_04140_amd import workloads as W
    x = W.mixed_f32(1 << 29, seed=3)
    xd = torch.from_numpy(x).cuda()
    ratio, c, d = _device_rates(codec, torch, xd, reps)
    del xd
    torch.cuda.empty_cache()
    algo = x.nbytes * (1 + ratio)  # values read + stream written (compression), the reverse for decompression
    ops = {op: {"achieved": round(algo / (x.nbytes / g), 2), "frac": round(algo / (x.nbytes / g) / HBM_PEAK_GBPS, 4)}
           for op, g in (("compress", c), ("decompress", d))}
    return {"workload": "mixed_f32: 536,870,912 float32 values (2 GiB)", "ratio": ratio,
            "compress_gbps": c, "decompress_gbps": d, "roofline_ops": ops,
            "host_pipeline": host_pipeline(codec, x, torch)}


def codec_bound(x):
    from paper_2511_04140_amd import codec as C
    import torch
    return C.compress_bound(x.size, torch.float64 if x.dtype.itemsize == 8 else torch.float32)


def ablation(codec, torch, x_c2, reps=5):
    """Sec. 5.4.2 (Fig. 12b): Falcon against Fal_Elf (Elf's trial-and-error
    decimal places), Fal_Sparse and Fal_Dense (one row scheme for every
    bit plane), device-resident, on the 1 Mi-value walk, the 2 GiB float64
    workload and the 2 GiB float32 workload.  Per variant: compressed /
    original bytes, and the median kernel time of compression (size pass,
    scan, write pass) and of decompression as GB/s of original bytes.  A
    Fal_Sparse stream whose chunks exceed the format's chunk bound is not
    decodable by the ordinary decoder (decompress_gbps null)."""
    import numpy as np
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    res = {}
    for label, make in (("walk_f64_2^20", lambda: W.walk_f64(1 << 20, seed=1)),
                        ("sensor_f64_2^28", lambda: x_c2),
                        ("mixed_f32_2^29", lambda: W.mixed_f32(1 << 29, seed=3))):
        x = make()
        xd = torch.from_numpy(x).cuda()
        yd = torch.empty_like(xd)
        code = 2 if x.dtype == np.float64 else 1
        row = {}
        for variant in ("falcon", "elf", "sparse", "dense"):
            sbuf = torch.empty(C.lib().falcon_compress_bound_variant(x.size, code, C.VARIANTS[variant]),
                               dtype=torch.uint8, device="cuda")
            kc, kd = [], []
            for _ in range(reps + 1):
                s = codec.compress_variant(xd, variant, out=sbuf)
                kc.append(codec.last_kernel_ms())
            dec = True
            for _ in range(reps + 1):
                try:
                    codec.decompress(s, out=yd)
                except C.FalconError:
                    dec = False
                    break
                kd.append(codec.last_kernel_ms())
            if dec:
                assert torch.equal(yd.view(torch.uint8), xd.view(torch.uint8)), (label, variant)
            row[variant] = {
                "ratio": round(s.numel() / x.nbytes, 6),
                "compress_gbps": round(x.nbytes / (float(np.median(kc[1:])) * 1e-3) / 1e9, 2),
                "decompress_gbps": round(x.nbytes / (float(np.median(kd[1:])) * 1e-3) / 1e9, 2) if dec else None,
            }
            del sbuf, s
        res[label] = row
        del xd, yd
        torch.cuda.empty_cache()
    return res


def full_range(codec, torch, wave_bytes=12 << 30, reps=3):
    """The 10,000-series batch with the full length range, log-uniform on
    [2^10, 2^24] values (about 109 GB, float64 and float32 mixed), streamed
    through the GPU in waves: the series are generated on the host a wave
    (at most wave_bytes of input) at a time, copied to the device, and each
    wave is compressed and decompressed by tuned, graph-captured batch plans
    (best of reps runs each).  Reports the device throughput over all waves
    and checks that every series round-trips."""
    import numpy as np
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    log = lambda m: print(f"[full-range] {m}", file=sys.stderr, flush=True)
    lens, is64, places = W.batch_layout(hi=1 << 24)
    nbytes = lens * np.where(is64, 8, 4)
    waves, cur, acc = [], [], 0
    for i in range(len(lens)):
        if cur and acc + nbytes[i] > wave_bytes:
            waves.append(cur)
            cur, acc = [], 0
        cur.append(i)
        acc += int(nbytes[i])
    waves.append(cur)
    tot = {"bytes": 0, "stream_bytes": 0, "compress_s": 0.0, "decompress_s": 0.0, "generate_s": 0.0, "h2d_s": 0.0}
    identical = True
    for k, wv in enumerate(waves):
        t0 = time.perf_counter()
        xs = W.batch_series(hi=1 << 24, select=wv)
        t1 = time.perf_counter()
        xd = [torch.from_numpy(x).cuda() for x in xs]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del xs
        tot["generate_s"] += t1 - t0
        tot["h2d_s"] += t2 - t1
        plan = codec.plan_compress(xd, tune=True, graph=True)
        plan.run(fetch=False)
        tc = []
        for _ in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            plan.run(fetch=False)
            torch.cuda.synchronize()
            tc.append(time.perf_counter() - a)
        streams = plan.run()
        counts = [x.numel() for x in xd]
        dts = [x.dtype for x in xd]
        dplan = codec.plan_decompress(streams, counts, dts, tune=True, graph=True)
        dplan.run(fetch=False)
        td = []
        for _ in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            dplan.run(fetch=False)
            torch.cuda.synchronize()
            td.append(time.perf_counter() - a)
        ys = dplan.run()
        ok = all(torch.equal(y.view(torch.uint8), x.view(torch.uint8)) for x, y in zip(xd, ys))
        identical = identical and ok
        wb = sum(x.numel() * x.element_size() for x in xd)
        tot["bytes"] += wb
        tot["stream_bytes"] += sum(s_.numel() for s_ in streams)
        tot["compress_s"] += min(tc)
        tot["decompress_s"] += min(td)
        log(f"wave {k + 1}/{len(waves)}: {len(wv)} series, {wb / 1e9:.2f} GB, compress {wb / min(tc) / 1e9:.0f} GB/s, "
            f"decompress {wb / min(td) / 1e9:.0f} GB/s, identical {ok}")
        dplan.close()
        plan.close()
        del xd, streams, ys, plan, dplan
        torch.cuda.empty_cache()
    return {"series": int(len(lens)), "waves": len(waves), "bytes": int(tot["bytes"]),
            "values_min_max": [int(lens.min()), int(lens.max())],
            "ratio": round(tot["stream_bytes"] / tot["bytes"], 6),
            "compress_gbps": round(tot["bytes"] / tot["compress_s"] / 1e9, 2),
            "decompress_gbps": round(tot["bytes"] / tot["decompress_s"] / 1e9, 2),
            "host_generate_s": round(tot["generate_s"], 1), "h2d_pageable_s": round(tot["h2d_s"], 1),
            "timing": "device-resident plan runs per wave (best of %d), summed over waves" % reps,
            "identical": identical}


def _device_rates(codec, torch, xd, reps=5):
    """Median kernel time of compression and of decompression over reps
    calls on a device-resident tensor; returns (ratio, compress GB/s,
    decompress GB/s) and checks the round trip."""
    import numpy as np
    from paper_2511_04140_amd import codec as C
    nbytes = xd.numel() * xd.element_size()
    sbuf = torch.empty(C.compress_bound(xd.numel(), xd.dtype), dtype=torch.uint8, device=xd.device)
    yd = torch.empty_like(xd)
    kc, kd = [], []
    for _ in range(reps + 1):
        s = codec.compress(xd, out=sbuf)
        kc.append(codec.last_kernel_ms())
        codec.decompress(s, out=yd)
        kd.append(codec.last_kernel_ms())
    assert torch.equal(yd.view(torch.uint8), xd.view(torch.uint8)), "round trip failed"
    tc, td = float(np.median(kc[1:])), float(np.median(kd[1:]))
    return (round(s.numel() / nbytes, 6), round(nbytes / (tc * 1e-3) / 1e9, 2),
            round(nbytes / (td * 1e-3) / 1e9, 2))


def studies(codec, torch):
    """Parameter studies of Sec. 5.3 on synthetic stand-ins:
    - beta: the sensor signal (no outliers or specials) rounded to 1..17
      significant digits, 2^26 values (512 MiB) each, device-resident
      (Fig. 10);
    - data size: prefixes of one 8 GiB sensor array from 100 MB to 8 GB,
      device-resident and host -> host through the pipeline from pinned
      buffers (Fig. 11);
    - batch size: the pipeline's batch from 0.5 to 8 x 1025 x 1024 values at
      4 and 16 streams on the 2 GiB prefix, pinned (the batch-size table)."""
    import numpy as np
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W
    log = lambda m: print(f"[studies] {m}", file=sys.stderr, flush=True)
    res = {"beta": {}, "data_size": {}, "batch": {}}
    for d in range(1, 18):
        xd = torch.from_numpy(W.significant_f64(1 << 26, 5, d)).cuda()
        r, c, dd = _device_rates(codec, torch, xd)
        res["beta"][d] = {"ratio": r, "compress_gbps": c, "decompress_gbps": dd}
        log(f"beta {d}: {res['beta'][d]}")
        del xd
    big = W.sensor_f64(1 << 30, seed=2)
    host = torch.from_numpy(big).pin_memory()
    del big
    sbuf = torch.empty(C.compress_bound(host.numel(), torch.float64), dtype=torch.uint8, pin_memory=True)
    ybuf = torch.empty(host.numel(), dtype=torch.float64, pin_memory=True)

    def host_rates(n, reps=3):
        tc = td = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            s = codec.compress_host(host[:n], out=sbuf)
            t1 = time.perf_counter()
            y = codec.decompress_host(s, out=ybuf[:n])
            t2 = time.perf_counter()
            tc, td = min(tc, t1 - t0), min(td, t2 - t1)
        assert torch.equal(y.view(torch.uint8), host[:n].view(torch.uint8)), "host round trip failed"
        return round(8 * n / tc / 1e9, 2), round(8 * n / td / 1e9, 2)

    codec.set_pipeline()
    for mb in (100, 250, 500, 1000, 2000, 4000, 8000):
        n = min(host.numel(), mb * 10 ** 6 // 8)
        xd = host[:n].cuda()
        r, c, dd = _device_rates(codec, torch, xd)
        del xd
        torch.cuda.empty_cache()
        hc, hd = host_rates(n)
        res["data_size"][f"{8 * n / 1e9:.2f} GB"] = {
            "ratio": r, "device_compress_gbps": c, "device_decompress_gbps": dd,
            "host_compress_gbps": hc, "host_decompress_gbps": hd}
        log(f"size {mb} MB: {res['data_size'][f'{8 * n / 1e9:.2f} GB']}")
    n2 = 1 << 28
    for ns in (4, 16):
        for bc in (512, 1024, 2048, 4096, 8192):
            codec.set_pipeline(ns, bc)
            hc, hd = host_rates(n2)
            res["batch"][f"{ns}x{bc}"] = {"n_streams": ns, "batch_values": bc * 1025,
                                          "host_compress_gbps": hc, "host_decompress_gbps": hd}
            log(f"batch {ns}x{bc}: {res['batch'][f'{ns}x{bc}']}")
    codec.set_pipeline()
    del host, sbuf, ybuf
    return res


def _kernel_short(name):
    """Short label of a kernel name as rocprofv3 prints it."""
    import re
    m = re.search(r"k_compress_pass<falcon_dev::TF(?:64|32), \d+, ([12]), 0,", name)
    if m:
        return "k_compress_pass<size>" if m.group(1) == "1" else "k_compress_pass<write>"
    for key, label in (("k_compress_queue<", "k_compress_queue"), ("k_compress_pass_mixed<", "k_compress_pass_mixed"),
                       ("k_decompress_mixed", "k_decompress_mixed"), ("k_decompress<", "k_decompress"),
                       ("k_scan_tiles", "k_scan_tiles"), ("k_scan_tile_sums", "k_scan_tile_sums"),
                       ("k_scan_apply", "k_scan_apply"), ("k_fill_u64", "k_fill_u64"),
                       ("k_batch_headers", "k_batch_headers"), ("k_gather_sizes", "k_gather_sizes")):
        if key in name:
            return label
    return name[:60]


def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def trace_summary(path, skip, last=0):
    """Per-kernel durations from a rocprofv3 --kernel-trace CSV, leaving out
    the first `skip` dispatches of every kernel (the warm-up steps), or
    keeping only the last `last` ones; prints a markdown table
    (microseconds)."""
    import numpy as np
    rows = _read_csv(path)
    by = {}
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Name")
        t = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0
        by.setdefault(name, []).append((int(r["Start_Timestamp"]), t))
    if last:
        print(f"Source: `{os.path.basename(path)}`; the last {last} dispatch(es) of each kernel.\n")
    else:
        print(f"Source: `{os.path.basename(path)}`; the first {skip} dispatch(es) of each kernel left out.\n")
    print("| kernel | full name (truncated) | dispatches | used | average us | median us | min us | max us |")
    print("|---|---|---|---|---|---|---|---|")
    out = {}
    for name, v in sorted(by.items(), key=lambda kv: -sum(t for _, t in kv[1])):
        v.sort()
        sel = v[-last:] if last else v[skip:]
        used = np.array([t for _, t in sel] or [t for _, t in v])
        out[_kernel_short(name)] = float(used.mean())
        print(f"| {_kernel_short(name)} | `{name[:70]}` | {len(v)} | {used.size} | {used.mean():.1f} | "
              f"{np.median(used):.1f} | {used.min():.1f} | {used.max():.1f} |")
    return out


def counter_summary(path, chunks):
    """Instruction and wait counters per chunk from a rocprofv3 --pmc CSV of
    SQ_INSTS_VALU, SQ_INSTS_SALU, SQ_INSTS_LDS, SQ_WAVE_CYCLES, SQ_WAIT_ANY
    and SQ_WAVES (one dispatch per kernel, `chunks` chunks); prints markdown.
    The VALU floor is the time the SIMDs need to issue those VALU
    instructions alone (4 cycles per wave64 instruction at 2.4 GHz on 1,024
    SIMDs)."""
    acc = {}
    for r in _read_csv(path):
        k = _kernel_short(r["Kernel_Name"])
        d = acc.setdefault((k, r.get("Dispatch_Id")), {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    print(f"Per chunk ({chunks:,} chunks per dispatch); wait = SQ_WAIT_ANY / SQ_WAVE_CYCLES.\n")
    print("| kernel | VALU | SALU | LDS | wait | VALU floor ms |")
    print("|---|---|---|---|---|---|")
    seen = set()
    for (k, _), d in acc.items():
        if k in seen or "SQ_INSTS_VALU" not in d or not k.startswith("k_"):
            continue
        seen.add(k)
        v, sa, lds = d["SQ_INSTS_VALU"] / chunks, d.get("SQ_INSTS_SALU", 0) / chunks, d.get("SQ_INSTS_LDS", 0) / chunks
        wait = d.get("SQ_WAIT_ANY", 0) / max(d.get("SQ_WAVE_CYCLES", 1), 1)
        floor_ms = d["SQ_INSTS_VALU"] * 4 / 1024 / 2.4e9 * 1e3
        print(f"| {k} | {v:.0f} | {sa:.0f} | {lds:.0f} | {wait:.0%} | {floor_ms:.3f} |")


def traffic_summary(fetch_csv, write_csv, bench_json):
    """HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch), scaled by what the same counters read for
    the plain device copy of the input that bench.py --copy-calibration runs
    (__amd_rocclr_copyBuffer: the input's bytes read and written), against
    the algorithmic bytes per launch that the benchmark line lists.  Prints
    markdown and the JSON record bench.py reads (profiles/hbm_traffic.json)."""
    import numpy as np
    with open(bench_json) as f:
        line = [ln for ln in f if ln.startswith("{")][-1]
    b = json.loads(line)
    nbytes = b["config"]["bytes"]

    def per_kernel(path, counter):
        acc = {}
        for r in _read_csv(path):
            if r.get("Counter_Name") != counter:
                continue
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return acc
    fk, wk = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    copy = [k for k in fk if "copyBuffer" in k]
    cf = max(fk[copy[0]]) if copy else None
    cw = max(wk[copy[0]]) if copy else None
    f_fac = nbytes / 1024 / cf if cf else 1.0
    w_fac = nbytes / 1024 / cw if cw else 1.0
    rec = {"kernel_digest": kernel_source_digest(), "workload": b["config"]["workload"],
           "calibration": {"fetch_factor": f_fac, "write_factor": w_fac, "copy_fetch_kib": cf, "copy_write_kib": cw},
           "kernels": {}}
    print(f"Calibration: the plain copy of {nbytes:,} bytes reads FETCH_SIZE = {cf:,.1f} KiB and WRITE_SIZE = "
          f"{cw:,.1f} KiB; scale factors {f_fac:.5f} and {w_fac:.5f}.\n")
    print("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (calibrated) | algorithmic bytes | ratio |")
    print("|---|---|---|---|---|---|")
    algo = b.get("kernel_algorithmic_bytes", {})
    for name in fk:
        short = _kernel_short(name)
        if short not in algo:
            continue
        fv, wv = float(np.median(fk[name])), float(np.median(wk.get(name, [0.0])))
        hbm = int(fv * 1024 * f_fac + wv * 1024 * w_fac)
        rec["kernels"][short] = {"fetch_kib": fv, "write_kib": wv, "hbm_bytes_per_launch": hbm,
                                 "algorithmic_bytes": algo[short]}
        print(f"| {short} | {fv:,.1f} | {wv:,.1f} | {hbm:,} | {algo[short]:,} | {hbm / algo[short]:.3f} |")
    print("\n```json\n" + json.dumps(rec, indent=1) + "\n```")
    return rec


def sweeps(codec, torch, x):
    """Host pipeline geometry (streams x batch) and compression schedulers x
    streams on the 2 GiB float64 workload from pinned buffers, and practical
    HBM ceilings from plain device operations on 2 GiB (a copy, a read-only
    reduction, a fill), each best of 5 with HIP events."""
    import numpy as np
    res = {"pipeline": {}, "schedulers": {}, "hbm_ceilings": {}}
    xh = torch.from_numpy(x).pin_memory()
    sbuf = torch.empty(codec_bound(x), dtype=torch.uint8, pin_memory=True)
    ybuf = torch.empty(x.size, dtype=torch.float64, pin_memory=True)

    def host_rates(reps=2):
        tc = td = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            s_ = codec.compress_host(xh, out=sbuf)
            t1 = time.perf_counter()
            codec.decompress_host(s_, out=ybuf)
            t2 = time.perf_counter()
            tc, td = min(tc, t1 - t0), min(td, t2 - t1)
        return round(x.nbytes / tc / 1e9, 2), round(x.nbytes / td / 1e9, 2)
    for ns in (1, 2, 4, 8, 16):
        for bc in (256, 1024, 2048, 4096):
            codec.set_pipeline(ns, bc)
            c, d = host_rates()
            res["pipeline"][f"{ns}x{bc}"] = {"compress_gbps": c, "decompress_gbps": d}
    codec.set_pipeline()
    for kind in ("event", "sync", "prealloc"):
        codec.set_scheduler(kind)
        for ns in (1, 2, 4, 8, 16, 32):
            codec.set_pipeline(ns, 2048)
            res["schedulers"][f"{kind}_{ns}"] = host_rates()[0]
    codec.set_scheduler("event")
    codec.set_pipeline()
    # ceilings: a pinned host -> device and device -> host copy, then device ops
    xd = torch.empty(x.size, dtype=torch.float64, device="cuda")
    yd = torch.empty_like(xd)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn, reps=5):
        best = float("inf")
        for _ in range(reps):
            ev[0].record()
            fn()
            ev[1].record()
            ev[1].synchronize()
            best = min(best, ev[0].elapsed_time(ev[1]))
        return best * 1e-3
    res["hbm_ceilings"]["h2d_pinned_gbps"] = round(x.nbytes / timed(lambda: xd.copy_(xh, non_blocking=True)) / 1e9, 2)
    res["hbm_ceilings"]["d2h_pinned_gbps"] = round(x.nbytes / timed(lambda: ybuf.copy_(xd, non_blocking=True)) / 1e9, 2)
    res["hbm_ceilings"]["copy_gbps (read+write)"] = round(2 * x.nbytes / timed(lambda: yd.copy_(xd)) / 1e9, 1)
    res["hbm_ceilings"]["read_gbps (sum)"] = round(x.nbytes / timed(lambda: xd.sum()) / 1e9, 1)
    res["hbm_ceilings"]["write_gbps (fill)"] = round(x.nbytes / timed(lambda: yd.fill_(1.0)) / 1e9, 1)
    del xh, sbuf, ybuf, xd, yd
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="values (default: the 2 GiB workload)")
    ap.add_argument("--workload", choices=("sensor_f64", "mixed_f32", "decimal_f64"), default="sensor_f64",
                    help="the workload of the timed steps (default: the 2 GiB float64 sensor series; "
                         "decimal_f64: the sensor signal at 6 significant digits, no outliers, 2 GiB)")
    ap.add_argument("--form", choices=("two_pass", "single_pass"), default="two_pass",
                    help="compression form of the timed steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-host", action="store_true", help="skip the host -> host pipeline measurement")
    ap.add_argument("--no-batched", action="store_true", help="skip the 10,000-series batched launch measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-ablation", action="store_true", help="skip the ablation-variant measurement")
    ap.add_argument("--no-float32", action="store_true", help="skip the 2 GiB float32 workload")
    ap.add_argument("--full-range", action="store_true",
                    help="also stream the full-length-range 10,000-series batch (about 109 GB) through the GPU")
    ap.add_argument("--studies", action="store_true",
                    help="also run the parameter studies (beta, data size, pipeline batch size)")
    ap.add_argument("--sweeps", action="store_true",
                    help="also sweep the host pipeline geometry and schedulers and measure HBM / PCIe ceilings")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run one plain device copy of the input "
                         "(its bytes read and written) as the reference for HBM byte counters")
    ap.add_argument("--only", choices=("batched", "serving"),
                    help="run only this section (no timed steps of the main workload); prints its JSON")
    ap.add_argument("--trace-summary", metavar="KERNEL_TRACE_CSV",
                    help="no GPU: summarise a rocprofv3 kernel trace (per-kernel durations) and exit")
    ap.add_argument("--skip", type=int, default=0, help="--trace-summary: dispatches per kernel to leave out")
    ap.add_argument("--last", type=int, default=0, help="--trace-summary: keep only the last dispatches per kernel")
    ap.add_argument("--counter-summary", nargs=2, metavar=("COUNTER_CSV", "CHUNKS"),
                    help="no GPU: instruction counters per chunk from a rocprofv3 SQ counter run, and exit")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON"),
                    help="no GPU: HBM bytes per launch from two rocprofv3 counter runs, and exit")
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(args.trace_summary, args.skip, args.last)
        return
    if args.counter_summary:
        counter_summary(args.counter_summary[0], int(args.counter_summary[1]))
        return
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this codec's multi-GPU "
              "sharding is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2511_04140_amd import codec as C
    from paper_2511_04140_amd import workloads as W

    if args.only:
        codec = C.Codec(0)
        res = batched(codec, torch) if args.only == "batched" else serving(codec, torch)
        codec.close()
        print(json.dumps({args.only: res}))
        return
    dev = torch.device("cuda", 0)
    f32 = args.workload == "mixed_f32"
    n = args.n or (1 << 29 if f32 else 1 << 28)
    if f32:
        x = W.mixed_f32(n, seed=3)
    elif args.workload == "decimal_f64":
        x = W.significant_f64(n, 5, 6)
    else:
        x = W.sensor_f64(n, seed=2)
    tdt = torch.float32 if f32 else torch.float64
    xd = torch.from_numpy(x).to(dev)
    nbytes = x.nbytes
    codec = C.Codec(0)
    # the timed steps run as a caller who keeps the data on the device would
    # run them: asynchronous calls, each decompression given the count and
    # dtype it was compressed with, one wait at the end of the region
    tcodec = C.Codec(0, blocking=False, form=args.form)
    cap = C.compress_bound(x.size, tdt)
    sbuf = torch.empty(cap, dtype=torch.uint8, device=dev)
    ybuf = torch.empty_like(xd)

    def step():
        holder = tcodec.compress_async(xd, sbuf)
        tcodec.decompress_n_async(sbuf, x.size, tdt, ybuf)
        return holder

    # warm-up (the first step also checks the round trip)
    for i in range(args.warmup):
        step()
        tcodec.sync()
        if i == 0:
            assert torch.equal(ybuf.view(torch.uint8), xd.view(torch.uint8)), "round trip failed"
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for _ in range(args.steps):
        holder = step()
    tcodec.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert torch.equal(ybuf.view(torch.uint8), xd.view(torch.uint8)), "round trip failed"
    s = sbuf[:holder.value]
    # stage times of the timed calls (HIP events the library recorded on the
    # launch stream), oldest first: compression, decompression, ... (the last
    # C.TIMED_CALLS calls of the region when it holds more)
    ncalls = min(2 * args.steps, C.TIMED_CALLS - C.TIMED_CALLS % 2)
    calls = [tcodec.call_stage_ms(b) for b in range(ncalls - 1, -1, -1)]
    sc, sd_ = calls[0::2], calls[1::2]
    kc, kd = [sum(v) for v in sc], [sum(v) for v in sd_]
    if args.copy_calibration:
        ybuf.copy_(xd)
        torch.cuda.synchronize()

    clen = s.numel()
    ratio = clen / nbytes
    step_s = (t1 - t0) / args.steps
    kc_ms, kd_ms = float(np.mean(kc)), float(np.mean(kd))
    nc = (x.size + 1024) // 1025
    # kernels of the path: their average durations over the timed steps (HIP
    # events on the launch stream) and the algorithmic bytes one launch moves
    if args.form == "two_pass":
        kernels = {
            "k_compress_pass<size>": (float(np.mean([v[0] for v in sc])), nbytes + 4 * nc),
            "k_scan (compress)": (float(np.mean([v[1] for v in sc])), 4 * nc + 8 * nc),
            "k_compress_pass<write>": (float(np.mean([v[2] for v in sc])), nbytes + clen - 4 * nc),
        }
    else:
        kernels = {"k_compress_queue": (float(np.mean([v[0] for v in sc])), nbytes + clen)}
    kernels.update({
        "k_scan (decompress)": (float(np.mean([v[1] for v in sd_])), 4 * nc + 8 * nc),
        "k_decompress": (float(np.mean([v[2] for v in sd_])), clen + nbytes),
    })
    dominant = max(kernels, key=lambda k: kernels[k][0])
    dom_ms, dom_bytes = kernels[dominant]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(dominant, dom_bytes) if args.workload == "sensor_f64" else None
    algo = nbytes + clen  # compression: values read, stream written; decompression the reverse

    # fraction of chunks in each case of Eq. 3 (header bytes alpha_max, beta_hat_max)
    sizes = s[32:32 + 4 * nc].view(torch.int32).to(torch.int64)
    offs = torch.cumsum(sizes, 0) - sizes
    a_bytes = s[32 + 4 * nc + offs]
    b_bytes = s[32 + 4 * nc + offs + 1]
    amax, bmax = (10, 6) if f32 else (22, 15)
    case1 = float(((a_bytes <= amax) & (b_bytes <= bmax)).float().mean().item())

    workload = {"sensor_f64": WORKLOAD,
                "mixed_f32": "mixed_f32: 536,870,912 float32 values (2 GiB): half sinusoid + N(0, 0.01^2) noise at "
                             "0-4 decimal places, half 512^3 interpolated fields at full precision",
                "decimal_f64": f"decimal_f64: {n:,} float64 values, the sensor signal rounded to 6 significant "
                               "digits (Case 1 chunks)"}[args.workload]
    out = {
        "metric": METRIC,
        "value": round(nbytes / step_s / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if f32 else "f64",
        "data": "synthetic",
        "config": {"workload": workload, "n": int(x.size), "bytes": int(nbytes),
                   "chunk": 1025, "resident": "HBM", "compression_form": args.form,
                   "calls": "asynchronous falcon_compress + falcon_decompress_n per step, one wait per timed region"},
        "compress_gbps": round(nbytes / (kc_ms * 1e-3) / 1e9, 3),
        "decompress_gbps": round(nbytes / (kd_ms * 1e-3) / 1e9, 3),
        "ratio": round(ratio, 6),
        "case1_chunk_fraction": round(case1, 6),
        "kernel_ms": {k: round(v[0], 4) for k, v in kernels.items()},
        "kernel_algorithmic_bytes": {k.split(" ")[0]: int(v[1]) for k, v in kernels.items() if "scan" not in k},
        "roofline": {
            "bound": "hbm",
            "kernel": dominant,
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "algorithmic_bytes": int(dom_bytes),
        },
        "roofline_ops": {
            "compress (all launches)": {
                "ms": round(kc_ms, 4), "achieved": round(algo / (kc_ms * 1e-3) / 1e9, 2),
                "frac": round(algo / (kc_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)},
            "decompress (scan + decoding kernel)": {
                "ms": round(kd_ms, 4), "achieved": round(algo / (kd_ms * 1e-3) / 1e9, 2),
                "frac": round(algo / (kd_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)},
        },
    }
    del sbuf, ybuf, s, xd
    if tcodec is not codec:
        tcodec.close()
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    log(f"device round trip: {out['value']} GB/s")
    if not args.no_host:
        out["host_pipeline"] = host_pipeline(codec, x, torch)
        log(f"host pipeline: {out['host_pipeline']}")
    if not args.no_float32 and not f32:
        out["float32"] = float32_case(codec, torch)
        log(f"float32: {out['float32']}")
    if not args.no_batched:
        out["batched"] = batched(codec, torch)
        torch.cuda.empty_cache()
        log(f"batched: {out['batched']}")
    if not args.no_serving:
        out["serving"] = serving(codec, torch)
        torch.cuda.empty_cache()
        log(f"serving: {out['serving']}")
    if not args.no_ablation and not f32:
        out["ablation"] = ablation(codec, torch, x)
        log(f"ablation: {out['ablation']}")
    if args.full_range:
        out["full_range"] = full_range(codec, torch)
    if args.studies:
        out["studies"] = studies(codec, torch)
        torch.cuda.empty_cache()
    if args.sweeps and not f32:
        out["sweeps"] = sweeps(codec, torch, x)
        log(f"sweeps: {out['sweeps']}")
    if not args.no_cpu_baseline:
        x32 = None if f32 else W.mixed_f32(1 << 24, seed=3, side=128)
        out["cpu_baseline"] = cpu_baseline(x, x32)
        if x32 is not None:
            out["cpu_baseline"]["float32"]["sample"] = ("mixed_f32 at 2^24 values (the same composition: half "
                                                       "low-precision sinusoid, half 128^3 fields)")
        out["cpu_baseline"]["small_case"] = oracle_small_case()
    codec.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
