"""Benchmark of the subset-DIC hot path on one MI355X.

A step correlates one 1024x1024 speckle pair from scratch with the images
already in device memory: reference gradients and per-POI records, the
brute-force ZNCC integer search and IC-GN refinement of all 36,864 POIs,
replayed as one HIP graph.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "POIs/s to IC-GN convergence (FP32 batched vs FP64 plain) at ≤1e-3 px"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2 (packed) x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP32_NONPACKED_PEAK_TFLOPS = 78.6
# dense bf16 matrix-core peak of the MI355X (no sparsity)
BF16_MFMA_PEAK_TFLOPS = 2500.0
MFMA_BLOCK = 32          # tuning search_block of the matrix-core search form
# sources whose hash keys each kernel's committed counter summary
KERNEL_SOURCES = {
    "search_mfma": ("k_search_mfma.hip", "search_common.h", "dic_device.h", "dic_internal.h"),
    "search_f32": ("k_search.hip", "search_common.h", "dic_device.h", "dic_internal.h"),
    "icgn_f32": ("k_icgn.hip", "refine_common.h", "dic_device.h", "dic_internal.h"),
    "nr_f32": ("k_nr.hip", "refine_common.h", "dic_device.h", "dic_internal.h"),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_affine_1024.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "sq_counters_affine_1024.json")
SIMDS = 256 * 4          # compute units x SIMDs
CLOCK_HZ = 2.4e9         # peak engine clock
# issue cycles of one wave64 instruction on a SIMD: vector ALU (16 lanes, 4
# passes) and v_mfma_f32_32x32x16_bf16 (8 passes of 4 cycles)
VALU_CYCLES, MFMA_CYCLES = 4, 32
CSRC = os.path.join(ROOT, "paper_1905_06228_amd", "csrc")


def kernel_source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        k = t["kernels"][kernel]
        srcs = KERNEL_SOURCES.get(kernel, tuple(k.get("sources", [])))
        if list(srcs) != list(k.get("sources", [])) or k.get("source_hash") != kernel_source_hash(srcs):
            return None
        return float(k["bytes_per_launch"])
    except (OSError, KeyError, ValueError, TypeError):
        return None


def measured_issue(kernel: str, kernel_ms: float):
    """Fractions of the kernel's time the SIMDs spend issuing its vector-ALU
    and matrix-core instructions: instruction counts per launch from the
    committed rocprofv3 SQ counter summary (if taken on the current source)
    times the issue cycles of one instruction, over SIMDs x clock x time."""
    try:
        with open(COUNTERS_FILE) as fh:
            t = json.load(fh)
        k = t["kernels"][kernel]
        srcs = KERNEL_SOURCES.get(kernel, tuple(k.get("sources", [])))
        if list(srcs) != list(k.get("sources", [])) or k.get("source_hash") != kernel_source_hash(srcs):
            return None
        cyc = SIMDS * CLOCK_HZ * kernel_ms * 1e-3
        return dict(valu_issue_frac=round(k["valu_insts_per_launch"] * VALU_CYCLES / cyc, 3),
                    mfma_issue_frac=round(k["mfma_insts_per_launch"] * MFMA_CYCLES / cyc, 3),
                    valu_insts_per_launch=k["valu_insts_per_launch"])
    except (OSError, KeyError, ValueError, TypeError):
        return None


def time_launches(torch, fn, reps: int) -> float:
    """Average ms of fn() over reps launches, HIP events on the current stream."""
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def host_cpu() -> dict:
    """The host's CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "usable_cores": usable, "os_cpu_count": os.cpu_count()}


def pool_size() -> int:
    """Oracle worker processes: the usable cores, at most 16 (one GPU's share
    of the host's cores)."""
    return max(1, min(16, host_cpu()["usable_cores"]))


_POOL_DATA = {}


def _pool_init(data):
    """Worker set-up: one BLAS thread per process; the images once per worker."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except ImportError:
        pass
    _POOL_DATA.update(data)


def _pool_correlate(args):
    from oracle import dic_oracle as O
    key, pois, M, S = args
    f, g = _POOL_DATA[key]
    return O.correlate(f, g, pois, M, S)


def _pool_batched(args):
    """One chunk of the batched workload's sample: renders pair k (the
    generator's NumPy recipe) and times the oracle on the POIs ``idx`` of its
    grid (rendering excluded)."""
    import dicgen
    from oracle import dic_oracle as O
    k, idx = args
    pr = dicgen.sinusoidal_batch(n_pairs=1, size=512, S=8, step=6, first=k)[0]
    t0 = time.perf_counter()
    O.correlate(pr.ref, pr.defm, pr.pois[idx], pr.M, pr.S)
    return time.perf_counter() - t0, len(idx), 2 * pr.M + 1


def _pool_znssd(args):
    from oracle import dic_oracle as O
    key, pois, M, P, up = args
    f, g = _POOL_DATA[key]
    return O.znssd_batch(f, g, pois, M, P, upstream=up)


def make_oracle_pool(procs: int, data: dict):
    """A spawn-started pool of oracle workers (made before any GPU call; the
    workers never touch the GPU)."""
    import multiprocessing as mp
    return mp.get_context("spawn").Pool(procs, initializer=_pool_init, initargs=(data,))


def cpu_baseline(pair, got, n_sample: int, seed: int = 11, pool=None, procs: int = 1,
                 extra=None):
    """The FP64 oracle, as it stands, on seeded samples of the benchmark's POIs:
    one process (one BLAS thread), and, with ``pool``, ``procs`` processes
    over chunks of a larger sample (the all-cores figure, reported as the
    value).  The single-process sample also checks the GPU result."""
    from oracle import dic_oracle as O

    idx = np.sort(np.random.default_rng(seed).choice(len(pair.pois), n_sample, replace=False))
    try:   # one thread: the figure is the oracle on one core
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(limits=1)
    except ImportError:
        limit = None
    t0 = time.perf_counter()
    ref = O.correlate(pair.ref, pair.defm, pair.pois[idx], pair.M, pair.S)
    dt = time.perf_counter() - t0
    if limit is not None:
        limit.restore_original_limits()
    ok = (ref["status"] == O.OK) & (got["status"][idx] == O.OK)
    duv = np.abs(got["p"][idx][ok][:, [0, 3]] - ref["p"][ok][:, [0, 3]])
    acc = dict(sample=int(n_sample),
               integer_exact=bool(np.array_equal(got["uv"][idx], ref["uv"])),
               status_equal=bool(np.array_equal(got["status"][idx], ref["status"])),
               max_err_px=float(duv.max(initial=0.0)),
               p99_err_px=float(np.percentile(duv.max(axis=1), 99)) if ok.any() else 0.0,
               mean_err_px=float(duv.mean()) if ok.any() else 0.0,
               max_dzncc=float(np.abs(got["zncc"][idx][ok] - ref["zncc"][ok]).max(initial=0.0)))
    cpu = host_cpu()
    single = dict(value=n_sample / dt, unit="POIs/s", cores=1, kind="oracle",
                  sample=f"{n_sample} seeded POIs of the 36,864-POI grid, FP64 NumPy oracle, "
                         f"one process, one BLAS thread, {dt:.1f} s",
                  seconds=dt)
    if pool is None:
        base = dict(single, cpu=cpu)
        return base, acc
    n_pool = min(len(pair.pois), 600 * procs)
    pidx = np.sort(np.random.default_rng(seed + 1).choice(len(pair.pois), n_pool, replace=False))
    chunks = [("pair", pair.pois[c], pair.M, pair.S) for c in np.array_split(pidx, 4 * procs)]
    t0 = time.perf_counter()
    pool.map(_pool_correlate, chunks)
    dtp = time.perf_counter() - t0
    base = dict(value=n_pool / dtp, unit="POIs/s", cores=procs, kind="oracle",
                sample=f"{n_pool} seeded POIs of the 36,864-POI grid, FP64 NumPy oracle, "
                       f"{procs} spawn-started processes (one BLAS thread each) over "
                       f"{len(chunks)} chunks, {dtp:.1f} s",
                seconds=dtp, cpu=cpu, single_process=single)
    if extra:
        base["other_workloads"] = extra(pool, procs)
    return base, acc


def oracle_other_workloads(pool, procs: int) -> dict:
    """The oracle on the whole rigid 256 x 256 pair (484 POIs, search and
    IC-GN) and on the whole differentiation workload (16,384 POIs, criterion
    and adjoint), over the pool."""
    import dicgen
    out = {}
    pr = dicgen.rigid_pair_256()
    chunks = [("rigid", q, pr.M, pr.S) for q in np.array_split(pr.pois, 4 * procs)]
    t0 = time.perf_counter()
    pool.map(_pool_correlate, chunks)
    dt = time.perf_counter() - t0
    out["rigid_256"] = dict(pois=len(pr.pois), seconds=round(dt, 2),
                            pois_per_s=round(len(pr.pois) / dt, 1), cores=procs)
    pr4 = dicgen.affine_pair_1024(size=1024, tag=4)
    pois = dicgen.gradient_grid_1024()
    N = len(pois)
    rng = np.random.default_rng(41)
    ctr = dicgen.true_displacement(pr4.field, pois.astype(np.float64))
    P = np.zeros((N, 6))
    P[:, 0], P[:, 3] = ctr[:, 0], ctr[:, 1]
    P[:, 1], P[:, 5] = 0.005, -0.0015
    P[:, [0, 3]] += rng.uniform(-0.3, 0.3, (N, 2))
    P[:, [1, 2, 4, 5]] += rng.uniform(-0.01, 0.01, (N, 4))
    up = rng.uniform(0.5, 2.0, N)
    parts = np.array_split(np.arange(N), 4 * procs)
    chunks = [("diff", pois[c], 12, P[c], up[c]) for c in parts]
    t0 = time.perf_counter()
    pool.map(_pool_znssd, chunks)
    dt = time.perf_counter() - t0
    out["differentiation"] = dict(pois=N, seconds=round(dt, 2), pois_per_s=round(N / dt, 1),
                                  cores=procs, what="criterion, dC/dp and dC/dG")
    out["batched"] = oracle_batched_sample(pool, procs)
    return out


def oracle_batched_sample(pool, procs: int, n_pairs: int = 8, per_pair: int = 128) -> dict:
    """The oracle on 8 seeded pairs of the batched workload (pairs 0..7, which
    hold all four subset sizes), 128 seeded POIs of each, search and IC-GN;
    the per-POI time of each subset size, weighted by the 64 pairs' POI
    counts and divided over the processes, extrapolates the whole workload."""
    import dicgen
    rng = np.random.default_rng(43)
    chunks = []
    for k in range(n_pairs):
        sub = dicgen.batch_pair_params(k)[2]
        n = len(dicgen.poi_grid(512, 512, sub // 2, 8, 6))
        idx = np.sort(rng.choice(n, per_pair, replace=False))
        chunks += [(k, c) for c in np.array_split(idx, 2)]
    t0 = time.perf_counter()
    res = pool.map(_pool_batched, chunks)
    wall = time.perf_counter() - t0
    per = {}
    for sec, n, sub in res:
        a = per.setdefault(sub, [0.0, 0])
        a[0] += sec
        a[1] += n
    t_poi = {sub: a[0] / a[1] for sub, a in per.items()}
    total_s, total_n = 0.0, 0
    for k in range(64):
        sub = dicgen.batch_pair_params(k)[2]
        n = len(dicgen.poi_grid(512, 512, sub // 2, 8, 6))
        total_n += n
        total_s += n * t_poi.get(sub, sum(t_poi.values()) / len(t_poi))
    est = total_s / procs
    return dict(sample=f"{n_pairs} seeded pairs (0..{n_pairs - 1}), {per_pair} seeded POIs each, "
                       f"search and IC-GN, {len(chunks)} chunks over {procs} processes "
                       f"({wall:.1f} s with each chunk's rendering)",
                pois=n_pairs * per_pair,
                seconds_per_poi_by_subset={str(k): round(v, 5) for k, v in sorted(t_poi.items())},
                extrapolated_pois=total_n, extrapolated_seconds=round(est, 1),
                pois_per_s=round(total_n / est, 1), cores=procs)


def sequence_bench(torch, dic, dicgen, dev, n_frames: int, reference: str = "first",
                   live_fps: float = 0.0, interp: str = "bicubic") -> dict:
    """Frames/s of the camera-scale sequence: frame k against frame 0
    (reference "first") or against frame k - 1 (reference "previous", the
    reference updated after every pair), seeded by the last OK result,
    4096 x 3000 frames of ~600k blobs under the
    heterogeneous strain field (noise 3), subset 29 x 29, step 7, search +-24
    around the seed.  Frames rendered on the device (same recipe as the NumPy
    generator); timed once with every frame resident in HBM and once from
    host memory through the driver's pinned double buffer.  ``interp``
    selects the refinement's interpolation (bicubic taps by default)."""
    H, W, M, S, step = 3000, 4096, 14, 24, 7
    t0 = time.perf_counter()
    frames = dicgen.sequence_frames_torch(n_frames, H, W, 600_000, noise=3.0, tag=5, pad=96.0,
                                          device=dev)
    torch.cuda.synchronize()
    render_s = time.perf_counter() - t0
    pois = dicgen.poi_grid(W, H, M, S, step)
    Q = torch.from_numpy(pois).to(dev)
    host = [f.cpu() for f in frames]
    flags = INTERP_FLAGS[interp](dic)
    dic.correlate_sequence(frames[:2], Q, M, S, reference=reference, flags=flags)   # load kernels
    torch.cuda.synchronize()

    def run(src):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = dic.correlate_sequence(src, Q, M, S, reference=reference, flags=flags)
        torch.cuda.synchronize()
        return res, time.perf_counter() - t

    res, t_dev = run(frames)
    _, t_host = run(host)
    last = res[-1]
    st = last["status"].cpu().numpy()
    ok = st == 0
    if reference == "first":
        truth = dicgen.true_displacement(dicgen.heterogeneous_strain(n_frames - 1),
                                         pois[ok].astype(np.float64))
    else:
        truth = dicgen.true_increment(dicgen.heterogeneous_strain(n_frames - 2),
                                      dicgen.heterogeneous_strain(n_frames - 1), pois[ok])
    p = last["p"].cpu().numpy()[ok]
    err = np.abs(p[:, [0, 3]] - truth)
    iters = [float(r["iters"].float()[r["status"] == 0].mean()) for r in res]
    return {"metric": "frames/s, camera-scale sequence", "value": round((n_frames - 1) / t_dev, 2),
            "unit": "frames/s", "frames_per_s_with_h2d": round((n_frames - 1) / t_host, 2),
            "ms_per_frame": round(t_dev * 1e3 / (n_frames - 1), 3),
            "ms_per_frame_with_h2d": round(t_host * 1e3 / (n_frames - 1), 3),
            "frames": n_frames, "pois_per_frame": int(len(pois)),
            "reference": reference, "last_frame_status_histogram": dic.status_histogram(st),
            "config": {"workload": "sequence_4096x3000: frames 1..K against "
                                   + ("frame 0" if reference == "first" else "frame k-1")
                                   + ", ~600k blobs, "
                                   "u = 0.002 k x (1 + 0.5 sin(2 pi y / 1500)), v = -0.0006 k y, "
                                   "noise sigma 3, subset 29x29, step 7, search +-24 around "
                                   "the seed", "form": "FP32 batched", "interp": interp},
            "render_s": round(render_s, 1),
            "mean_iterations_per_frame": [round(v, 3) for v in iters],
            "last_frame": {"ok_fraction": float(ok.mean()),
                           "mean_abs_err_vs_field_px": float(err.mean()),
                           "p99_abs_err_vs_field_px": float(np.percentile(err, 99))},
            "live": live_bench(torch, dic, dicgen, host, Q, pois, M, S, live_fps)
            if live_fps > 0 else None,
            "data": "synthetic"}


def batched_bench(torch, dic, dicgen, dev, reps: int) -> dict:
    """The batched workload: 64 independent 512 x 512 speckle pairs with
    sinusoidal fields, one subset size per pair from {15, 21, 31, 41}, step 6,
    search +-8, in one plan: every stage is one persistent launch over all
    pairs' POIs, the whole step replayed as a HIP graph.  POIs/s end to end,
    per-stage kernel times and the IC-GN roofline (the largest subsets, 41 x 41,
    run in the 28-slot refinement kernel)."""
    t0 = time.perf_counter()
    pairs = dicgen.sinusoidal_batch_torch(n_pairs=64, size=512, S=8, step=6, device=dev)
    torch.cuda.synchronize()
    render_s = time.perf_counter() - t0
    tens = [(p.ref, p.defm, torch.from_numpy(p.pois).to(dev), p.M, p.S) for p in pairs]
    specs, F, G, Q = dic.batch_layout(tens, dev)
    N = int(Q.shape[0])
    plan = dic.Plan(specs, dic.FP32_BATCHED, flags=dic.FLAG_USE_GRAPH)
    out = plan.new_outputs()
    ms = time_launches(torch, lambda: plan.correlate(F, G, Q, out=out), reps)
    st = dic.Plan(specs, dic.FP32_BATCHED, flags=dic.FLAG_CACHE_REF_PREP)
    st.tuning = plan.tuning
    so = st.new_outputs()
    t_prep = time_launches(torch, lambda: st.prepare_reference(F, Q), reps)
    t_box = time_launches(torch, lambda: st.prepare_deformed(G), reps)
    t_search = time_launches(torch, lambda: st.integer_search(
        F, G, Q, out=(so["uv"], so["zncc_int"], so["status_int"])), reps)
    t_icgn = time_launches(torch, lambda: st.icgn_refine(
        F, G, Q, so["uv"], so["status_int"],
        out=(so["p"], so["zncc"], so["iters"], so["status"])), reps)
    stat = out["status"].cpu().numpy()
    iters = out["iters"].cpu().numpy()[stat == 0]
    # algorithmic bytes and flops summed over the pairs' subset sizes
    icgn_bytes, flops, per_m = 0, 0.0, {}
    for p in pairs:
        n = (2 * p.M + 1) ** 2
        A = (2 * p.M + 4) ** 2
        icgn_bytes += (12 * n + 4 * A + 70) * len(p.pois)
        flops += 2.0 * (2 * p.S + 1) ** 2 * n * len(p.pois)
        per_m[2 * p.M + 1] = per_m.get(2 * p.M + 1, 0) + len(p.pois)
    gbs = icgn_bytes / (t_icgn * 1e-3) / 1e9
    tfl = flops / (t_search * 1e-3) / 1e12
    return {"pois": N, "pairs": len(pairs), "pois_per_subset": dict(sorted(per_m.items())),
            "ms_per_step": round(ms, 4), "pois_per_s": round(N / (ms * 1e-3), 1),
            "stages_ms": {"reference_prep": round(t_prep, 4),
                          "deformed_box_sums": round(t_box, 4),
                          "search": round(t_search, 4), "icgn": round(t_icgn, 4)},
            "icgn_pois_per_s": round(N / (t_icgn * 1e-3), 1),
            "mean_iterations": float(iters.mean()) if iters.size else 0.0,
            "ok_fraction": float((stat == 0).mean()),
            "status_histogram": dic.status_histogram(stat),
            "tuning": list(plan.tuning),
            "roofline_icgn": dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS,
                                  unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4), traffic=None,
                                  kernel="icgn_f32_kernel (28-, 16- and 8-slot instances)",
                                  kernel_ms=round(t_icgn, 4),
                                  algorithmic_bytes_per_launch=int(icgn_bytes)),
            "roofline_search": dict(bound="mfma", achieved=round(tfl, 2),
                                    peak=BF16_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                                    frac=round(tfl / BF16_MFMA_PEAK_TFLOPS, 4),
                                    kernel="search_mfma_kernel", kernel_ms=round(t_search, 4),
                                    algorithmic_flops_per_launch=flops),
            "render_s": round(render_s, 1),
            "config": {"workload": "batched: 64 independent 512x512 speckle pairs (8,000 blobs "
                                   "each), u = A sin(2 pi y / lam), v = A cos(2 pi x / lam), "
                                   "A ~ U(0.5, 2), lam ~ U(64, 256), subset per pair from "
                                   "{15, 21, 31, 41}, step 6, search +-8, one plan, HIP graph"}}


# algorithmic bytes of the ZNSSD adjoint per POI: the reference subset (4 n),
# the deformed patch read (4 A) and its gradient read and written (8 A), the
# warp, upstream scale, criterion and warp gradient (104 B) and the reference
# record's mean, norm and status (24 B)
def znssd_bytes_per_poi(M: int) -> int:
    n, A = (2 * M + 1) ** 2, (2 * M + 4) ** 2
    return 4 * n + 12 * A + 128


def adjoint_bench(torch, dic, dicgen, dev, reps: int) -> dict:
    """The differentiation workload: a 1024 x 1024 pair (the affine field with
    noise), 16,384 POIs on the 68 + 7k grid, subset 25 x 25, the warp off the
    optimum by a seeded offset; the forward criterion alone, and forward plus
    backward (dC/dp and dC/dG) in the float-atomic and the deterministic
    fixed-point modes."""
    pr = dicgen.affine_pair_1024(size=1024, tag=4)
    pois = dicgen.gradient_grid_1024()
    N, M = len(pois), 12
    rng = np.random.default_rng(41)
    ctr = dicgen.true_displacement(pr.field, pois.astype(np.float64))
    P = np.zeros((N, 6))
    P[:, 0], P[:, 3] = ctr[:, 0], ctr[:, 1]
    P[:, 1], P[:, 5] = 0.005, -0.0015            # the affine field's gradient terms
    P[:, [0, 3]] += rng.uniform(-0.3, 0.3, (N, 2))
    P[:, [1, 2, 4, 5]] += rng.uniform(-0.01, 0.01, (N, 4))
    up = rng.uniform(0.5, 2.0, N).astype(np.float32)
    F = torch.from_numpy(pr.ref).to(dev)
    G = torch.from_numpy(pr.defm).to(dev)
    Q = torch.from_numpy(pois).to(dev)
    Pd = torch.from_numpy(P).to(dev)
    U = torch.from_numpy(up).to(dev)
    c = torch.empty(N, dtype=torch.float32, device=dev)
    gp = torch.empty((N, 6), dtype=torch.float64, device=dev)
    gg = torch.zeros((1024, 1024), dtype=torch.float32, device=dev)
    res = {}
    B = znssd_bytes_per_poi(M) * N
    for mode, flags in (("atomic", 0), ("deterministic", dic.FLAG_DETERMINISTIC_BWD)):
        plan = dic.single_pair_plan(1024, 1024, M, 16, N, dic.FP32_BATCHED,
                                    flags=flags | dic.FLAG_CACHE_REF_PREP)
        plan.prepare_reference(F, Q)
        t_fwd = time_launches(torch, lambda: plan.znssd(F, G, Q, Pd, grad_c=U, c_out=c), reps)
        t_bwd = time_launches(torch, lambda: plan.znssd(F, G, Q, Pd, grad_c=U, c_out=c,
                                                        grad_p=gp, grad_def=gg), reps)
        gbs = B / (t_bwd * 1e-3) / 1e9
        res[mode] = {"forward_ms": round(t_fwd, 4), "forward_backward_ms": round(t_bwd, 4),
                     "pois_per_s": round(N / (t_bwd * 1e-3), 1),
                     "roofline": dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS,
                                      unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4),
                                      traffic=None, kernel="znssd_kernel",
                                      algorithmic_bytes_per_launch=int(B))}
    res["config"] = {"workload": "differentiation: 1024x1024 pair (16,000 blobs, u = 0.005x + "
                                 "1.3, v = -0.0015y - 0.6, noise sigma 2), 16,384 POIs at "
                                 "68 + 7k, subset 25x25, warp = the field's plus a seeded offset "
                                 "(u, v within 0.3 px, gradient terms within 0.01)"}
    return res


# plan flags of the refinement's interpolation options
INTERP_FLAGS = {
    "bicubic": lambda dic: 0,
    "bilinear": lambda dic: dic.FLAG_INTERP_BILINEAR,
    "bicubic_lut": lambda dic: dic.FLAG_BICUBIC_LUT,
    "bspline": lambda dic: dic.FLAG_INTERP_BSPLINE,
}


def live_bench(torch, dic, dicgen, host_frames, Q, pois, M, S, fps: float) -> dict:
    """The live policy: a camera thread offers the host frames at ``fps``;
    the correlator takes the newest frame, correlates it against the
    previously used one and waits for the result (as a display would); frames
    that arrive meanwhile are skipped.  Latency = frame offered -> its
    result on the host."""
    import threading
    H, W = host_frames[0].shape
    live = dic.LiveCorrelator(H, W, Q, M, S)
    offered = {}
    done = threading.Event()

    def camera():
        t0 = time.perf_counter()
        for k, f in enumerate(host_frames):
            wait = t0 + k / fps - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            offered[k] = time.perf_counter()
            live.put(f)
        done.set()

    cam = threading.Thread(target=camera)
    lat, used, results = [], [], []
    t_start = time.perf_counter()
    cam.start()
    while True:
        finished = done.is_set()
        ref_before = live.ref_seq
        o = live.step()
        if o is None:
            if live.ref_seq != ref_before:          # the first frame became the reference
                used.append(live.ref_seq)
                continue
            if finished:                            # nothing new and nothing more to come
                break
            time.sleep(0.0005)
            continue
        st = o["status"].cpu()                      # the display waits for the result
        lat.append(time.perf_counter() - offered[o["frame"]])
        used.append(o["frame"])
        results.append((o["reference"], o["frame"], o["p"].cpu().numpy(), st.numpy()))
    cam.join()
    elapsed = time.perf_counter() - t_start
    a, b, p, st = results[-1]
    ok = st == 0
    truth = dicgen.true_increment(None if a == 0 else dicgen.heterogeneous_strain(a),
                                  dicgen.heterogeneous_strain(b), pois[ok])
    err = np.abs(p[ok][:, [0, 3]] - truth)
    return {"camera_fps": fps, "frames_offered": len(host_frames),
            "pairs_correlated": len(results), "frames_skipped": live.mailbox.skipped,
            "processed_pairs_per_s": round(len(results) / elapsed, 2),
            "latency_ms_mean": round(1e3 * float(np.mean(lat)), 2),
            "latency_ms_max": round(1e3 * float(np.max(lat)), 2),
            "frames_used": used,
            "last_pair": {"reference": int(a), "frame": int(b), "ok_fraction": float(ok.mean()),
                          "mean_abs_err_vs_field_px": float(err.mean())}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pool", type=int, default=1,
                    help="1: also time the oracle over a pool of worker processes (all "
                         "usable cores, at most 16); 0: one process only")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--minimal", action="store_true",
                    help="time only the FP32 step and its stages (profiler runs)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the batched and differentiation workloads")
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--tuning", type=str, default=None,
                    help="search_block,search_occupancy,icgn_waves,icgn_slack (skips autotuning)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--reference", choices=("first", "previous"), default="first",
                    help="sequence benchmark: frame k against frame 0 or against frame k-1")
    ap.add_argument("--live-fps", type=float, default=0.0,
                    help="sequence benchmark: also run the live policy with a camera "
                         "offering the frames at this rate")
    ap.add_argument("--interp", choices=tuple(INTERP_FLAGS), default="bicubic",
                    help="sequence benchmark: the refinement's interpolation")
    ap.add_argument("--sequence-frames", type=int, default=0,
                    help="instead of the pair benchmark, time the camera-scale frame sequence "
                         "(4096x3000 frames, 239,932 POIs each) over this many frames")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: the hot path is a "
                          "single-device build; --gpus must be 1"}))
        return 2

    pool, procs, pair = None, 1, None
    if args.sequence_frames <= 0:
        import dicgen
        pair = dicgen.affine_pair_1024()
        if not args.no_cpu_baseline and args.cpu_pool and not args.minimal:
            # the oracle's worker pool starts before anything touches the GPU
            procs = pool_size()
            data = {"pair": (pair.ref, pair.defm)}
            if not args.no_configs:
                pr1 = dicgen.rigid_pair_256()
                pr4 = dicgen.affine_pair_1024(size=1024, tag=4)
                data.update(rigid=(pr1.ref, pr1.defm), diff=(pr4.ref, pr4.defm))
            pool = make_oracle_pool(procs, data)

    import torch

    import dicgen
    import paper_1905_06228_amd as dic

    dev = torch.device("cuda", 0)
    if args.sequence_frames > 0:
        print(json.dumps(sequence_bench(torch, dic, dicgen, dev, args.sequence_frames,
                                        args.reference, args.live_fps, args.interp)))
        return 0
    N = len(pair.pois)
    F = torch.from_numpy(pair.ref).to(dev)
    G = torch.from_numpy(pair.defm).to(dev)
    Q = torch.from_numpy(pair.pois).to(dev)
    H, W = pair.ref.shape

    # --- FP32 batched form, whole step as a graph ------------------------------
    plan = dic.single_pair_plan(W, H, pair.M, pair.S, N, dic.FP32_BATCHED,
                                flags=dic.FLAG_USE_GRAPH)
    if args.tuning:
        plan.tuning = tuple(int(v) for v in args.tuning.split(","))
    elif not args.no_autotune:
        plan.autotune(F, G, Q)
    out = plan.new_outputs()
    for _ in range(args.warmup):
        plan.correlate(F, G, Q, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.correlate(F, G, Q, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    got = {k: v.cpu().numpy() for k, v in out.items()}

    # --- per-stage kernel times (HIP events on the launch stream) --------------
    st = dic.single_pair_plan(W, H, pair.M, pair.S, N, dic.FP32_BATCHED,
                              flags=dic.FLAG_CACHE_REF_PREP)
    st.tuning = plan.tuning
    so = st.new_outputs()
    reps = max(5, args.steps // 2)
    t_prep = time_launches(torch, lambda: st.prepare_reference(F, Q), reps)
    t_box = time_launches(torch, lambda: st.prepare_deformed(G), reps)
    t_search = time_launches(torch, lambda: st.integer_search(
        F, G, Q, out=(so["uv"], so["zncc_int"], so["status_int"])), reps)
    t_icgn = time_launches(torch, lambda: st.icgn_refine(
        F, G, Q, so["uv"], so["status_int"],
        out=(so["p"], so["zncc"], so["iters"], so["status"])), reps)
    iters = got["iters"][got["status"] == 0]
    if args.minimal:
        # the FP32 step and its stages only (for profiler runs)
        print(json.dumps({"metric": METRIC, "value": round(N / (ms * 1e-3), 1), "unit": "POIs/s",
                          "ms_per_step": round(ms, 4), "minimal": True,
                          "stages_ms": {"reference_prep": round(t_prep, 4),
                                        "deformed_box_sums": round(t_box, 4),
                                        "search": round(t_search, 4), "icgn": round(t_icgn, 4)},
                          "tuning": list(plan.tuning)}), flush=True)
        return 0
    # Newton-Raphson refinement of the same search result (Sec. 2.2's other
    # sub-pixel method), both precisions
    nro = (so["p"].clone(), so["zncc"].clone(), so["iters"].clone(), so["status"].clone())
    t_nr = time_launches(torch, lambda: st.nr_refine(F, G, Q, so["uv"], so["status_int"], out=nro),
                         reps)
    nr_p, nr_it, nr_st = nro[0].cpu().numpy(), nro[2].cpu().numpy(), nro[3].cpu().numpy()
    # bilinear interpolation (Eq. 5) in both refinements of the same search
    # result, and the accuracy of each interpolant against the true field
    bp = dic.single_pair_plan(W, H, pair.M, pair.S, N, dic.FP32_BATCHED,
                              flags=dic.FLAG_CACHE_REF_PREP | dic.FLAG_INTERP_BILINEAR)
    bp.tuning = plan.tuning
    bil = {}
    truth = dicgen.true_displacement(pair.field, pair.pois.astype(np.float64))
    ref_err = {"icgn": (so["p"], so["status"]), "nr": (nro[0], nro[3])}
    for name, fn in (("icgn", bp.icgn_refine), ("nr", bp.nr_refine)):
        bo = tuple(torch.empty_like(x) for x in (so["p"], so["zncc"], so["iters"], so["status"]))
        t_b = time_launches(torch, lambda: fn(F, G, Q, so["uv"], so["status_int"], out=bo), reps)
        bpn, bit, bst = bo[0].cpu().numpy(), bo[2].cpu().numpy(), bo[3].cpu().numpy()
        cp, cst = ref_err[name][0].cpu().numpy(), ref_err[name][1].cpu().numpy()
        okb, okc = bst == 0, cst == 0
        eb = np.abs(bpn[okb][:, [0, 3]] - truth[okb])
        ec = np.abs(cp[okc][:, [0, 3]] - truth[okc])
        bil[name] = {"refine_ms": round(t_b, 4), "pois_per_s": round(N / (t_b * 1e-3), 1),
                     "bicubic_refine_ms": round(t_icgn if name == "icgn" else t_nr, 4),
                     "mean_iterations": float(bit[okb].mean()) if okb.any() else 0.0,
                     "ok_fraction": float(okb.mean()),
                     "mean_abs_error_px": float(eb.mean()) if okb.any() else None,
                     "bicubic_mean_abs_error_px": float(ec.mean()) if okc.any() else None,
                     "p99_abs_error_px": float(np.percentile(eb.max(axis=1), 99)) if okb.any() else None,
                     "bicubic_p99_abs_error_px": float(np.percentile(ec.max(axis=1), 99)) if okc.any() else None}
    # the bicubic coefficient table (look-up table of the interpolant): the
    # refinements with the plan's preparations cached, and uncached (the table
    # and the reference-side preparation rebuilt on every call)
    lut = {}
    for name, nrf in (("icgn", False), ("nr", True)):
        lo = tuple(torch.empty_like(x) for x in (so["p"], so["zncc"], so["iters"], so["status"]))
        t_l = {}
        for cached in (True, False):
            lp = dic.single_pair_plan(W, H, pair.M, pair.S, N, dic.FP32_BATCHED,
                                      flags=dic.FLAG_BICUBIC_LUT
                                      | (dic.FLAG_CACHE_REF_PREP if cached else 0))
            lp.tuning = plan.tuning
            fn = lp.nr_refine if nrf else lp.icgn_refine
            t_l[cached] = time_launches(
                torch, lambda: fn(F, G, Q, so["uv"], so["status_int"], out=lo), reps)
        lpn, lst = lo[0].cpu().numpy(), lo[3].cpu().numpy()
        cp, cst = ref_err[name][0].cpu().numpy(), ref_err[name][1].cpu().numpy()
        okl = (lst == 0) & (cst == 0)
        lut[name] = {"refine_ms": round(t_l[True], 4),
                     "refine_uncached_ms": round(t_l[False], 4),
                     "taps_refine_ms": round(t_icgn if name == "icgn" else t_nr, 4),
                     "max_vs_taps_px": float(np.abs(lpn[okl][:, [0, 3]] - cp[okl][:, [0, 3]]
                                                    ).max(initial=0)),
                     "status_equal_to_taps": float((lst == cst).mean())}
    # cubic B-spline interpolation (the spline option of Sec. 2.2): the
    # refinements with the plan's preparations cached and uncached (the
    # coefficient image and the reference-side preparation rebuilt every call),
    # and the accuracy against the true field beside bicubic's
    bsp = {}
    for name, nrf in (("icgn", False), ("nr", True)):
        bo = tuple(torch.empty_like(x) for x in (so["p"], so["zncc"], so["iters"], so["status"]))
        t_s = {}
        for cached in (True, False):
            sp = dic.single_pair_plan(W, H, pair.M, pair.S, N, dic.FP32_BATCHED,
                                      flags=dic.FLAG_INTERP_BSPLINE
                                      | (dic.FLAG_CACHE_REF_PREP if cached else 0))
            sp.tuning = plan.tuning
            fn = sp.nr_refine if nrf else sp.icgn_refine
            t_s[cached] = time_launches(
                torch, lambda: fn(F, G, Q, so["uv"], so["status_int"], out=bo), reps)
        spn, sit, sst = bo[0].cpu().numpy(), bo[2].cpu().numpy(), bo[3].cpu().numpy()
        cp, cst = ref_err[name][0].cpu().numpy(), ref_err[name][1].cpu().numpy()
        oks, okc = sst == 0, cst == 0
        es = np.abs(spn[oks][:, [0, 3]] - truth[oks])
        ec = np.abs(cp[okc][:, [0, 3]] - truth[okc])
        bsp[name] = {"refine_ms": round(t_s[True], 4),
                     "refine_uncached_ms": round(t_s[False], 4),
                     "bicubic_refine_ms": round(t_icgn if name == "icgn" else t_nr, 4),
                     "mean_iterations": float(sit[oks].mean()) if oks.any() else 0.0,
                     "ok_fraction": float(oks.mean()),
                     "mean_abs_error_px": float(es.mean()) if oks.any() else None,
                     "bicubic_mean_abs_error_px": float(ec.mean()) if okc.any() else None}
    # the whole pair (search and B-spline IC-GN) through one correlate call,
    # coefficients built beside the reference preparation
    cpb = dic.single_pair_plan(W, H, pair.M, pair.S, N, dic.FP32_BATCHED,
                               flags=dic.FLAG_INTERP_BSPLINE | dic.FLAG_USE_GRAPH)
    cpb.tuning = plan.tuning
    ob = cpb.new_outputs()
    bsp["correlate_ms"] = round(time_launches(torch, lambda: cpb.correlate(F, G, Q, out=ob),
                                              reps), 4)
    # particle swarm searches (Sec. 2.1, Eqs. 2-4) on the same pair, and the
    # modified swarm + Newton-Raphson pipeline (the paper's fastest combination)
    Rs = torch.from_numpy(dicgen.swarm_random(N, 7)).to(dev)
    swarm = {}
    uv_bfs, st_bfs = so["uv"].cpu().numpy(), so["status_int"].cpu().numpy()
    for name, mod in (("pso", False), ("modified_pso", True)):
        po = tuple(torch.empty_like(x) for x in (so["uv"], so["zncc_int"], so["status_int"],
                                                  so["iters"], so["iters"]))
        t_sw = time_launches(torch, lambda: st.pso_search(F, G, Q, Rs, modified=mod, out=po), reps)
        puv, pst, pgen, pev = (po[0].cpu().numpy(), po[2].cpu().numpy(), po[3].cpu().numpy(),
                               po[4].cpu().numpy())
        okp = (pst == 0) & (st_bfs == 0)
        swarm[name] = {"search_ms": round(t_sw, 4), "pois_per_s": round(N / (t_sw * 1e-3), 1),
                       "mean_evaluations": float(pev[pst == 0].mean()),
                       "mean_generations": float(pgen[pst == 0].mean()),
                       "integer_equal_to_brute_force": float(np.all(puv[okp] == uv_bfs[okp],
                                                                    axis=1).mean())}
        if mod:
            so2 = tuple(torch.empty_like(x) for x in (so["p"], so["zncc"], so["iters"], so["status"]))
            t_nr2 = time_launches(torch, lambda: st.nr_refine(F, G, Q, po[0], po[2], out=so2), reps)
            p2, s2 = so2[0].cpu().numpy(), so2[3].cpu().numpy()
            ok3 = (s2 == 0) & (nr_st == 0)
            swarm["modified_pso_then_nr"] = {
                "ms": round(t_sw + t_nr2, 4), "pois_per_s": round(N / ((t_sw + t_nr2) * 1e-3), 1),
                "final_within_1e-3px_of_brute_force_then_nr": float(
                    (np.abs(p2[ok3][:, [0, 3]] - nr_p[ok3][:, [0, 3]]).max(axis=1) <= 1e-3).mean())}

    # --- FP64 plain form ---------------------------------------------------------
    p64 = dic.single_pair_plan(W, H, pair.M, pair.S, N, dic.FP64_PLAIN)
    o64 = p64.new_outputs()
    p64.correlate(F, G, Q, out=o64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.fp64_steps):
        p64.correlate(F, G, Q, out=o64)
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) * 1e3 / args.fp64_steps
    g64 = {k: v.cpu().numpy() for k, v in o64.items()}
    t64_search = time_launches(torch, lambda: p64.integer_search(
        F, G, Q, out=(o64["uv"], o64["zncc_int"], o64["status_int"])), 1)
    t64_icgn = time_launches(torch, lambda: p64.icgn_refine(
        F, G, Q, o64["uv"], o64["status_int"],
        out=(o64["p"], o64["zncc"], o64["iters"], o64["status"])), 2)
    n64 = (o64["p"].clone(), o64["zncc"].clone(), o64["iters"].clone(), o64["status"].clone())
    t64_nr = time_launches(torch, lambda: p64.nr_refine(F, G, Q, o64["uv"], o64["status_int"],
                                                        out=n64), 2)
    nr64_p, nr64_st = n64[0].cpu().numpy(), n64[3].cpu().numpy()
    okn = (nr_st == 0) & (nr64_st == 0)
    nr_fp32_vs_fp64 = float(np.abs(nr_p[okn][:, [0, 3]] - nr64_p[okn][:, [0, 3]]).max(initial=0))
    ok2 = (got["status"] == 0) & (g64["status"] == 0)
    fp32_vs_fp64 = float(np.abs(got["p"][ok2][:, [0, 3]] - g64["p"][ok2][:, [0, 3]]).max(initial=0))

    # --- rooflines of the two large kernels; "roofline" is the longer one ------
    n = (2 * pair.M + 1) ** 2
    K = (2 * pair.S + 1) ** 2
    flops = 2.0 * K * n * N                      # one multiply-add per candidate and subset pixel
    achieved = flops / (t_search * 1e-3) / 1e12
    if plan.tuning[0] == MFMA_BLOCK:
        # bf16 Toeplitz products on the matrix cores; FP64 re-score decides
        kb = (2 * pair.M + 48) // 16
        tiles = 2 if 2 * pair.S + 1 == 33 else 1
        mfma_flops = (2 * pair.M + 1) * kb * tiles * (32 * 32 * 16 * 2) * N
        roof_search = dict(bound="mfma", achieved=round(achieved, 2), peak=BF16_MFMA_PEAK_TFLOPS,
                           unit="TFLOP/s", frac=round(achieved / BF16_MFMA_PEAK_TFLOPS, 4),
                           traffic=measured_traffic("search_mfma"),
                           kernel="search_mfma_kernel", kernel_ms=round(t_search, 4),
                           algorithmic_flops_per_launch=flops,
                           executed_mfma_flops_per_launch=mfma_flops,
                           executed_mfma_tflops=round(mfma_flops / (t_search * 1e-3) / 1e12, 1),
                           frac_of_fp32_vector_peak=round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                           issue=measured_issue("search_mfma", t_search))
    else:
        roof_search = dict(bound="alu", achieved=round(achieved, 2), peak=FP32_VECTOR_PEAK_TFLOPS,
                           unit="TFLOP/s", frac=round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                           traffic=measured_traffic("search_f32"), kernel="search_f32_kernel",
                           kernel_ms=round(t_search, 4), algorithmic_flops_per_launch=flops,
                           frac_of_nonpacked_fp32=round(achieved / FP32_NONPACKED_PEAK_TFLOPS, 4))
    A = (2 * pair.M + 4) ** 2
    icgn_bytes = (12 * n + 4 * A + 70) * N
    icgn_gbs = icgn_bytes / (t_icgn * 1e-3) / 1e9
    roof_icgn = dict(bound="hbm", achieved=round(icgn_gbs, 1), peak=HBM_PEAK_GBS,
                     unit="GB/s", frac=round(icgn_gbs / HBM_PEAK_GBS, 4),
                     traffic=measured_traffic("icgn_f32"), kernel="icgn_f32_kernel",
                     kernel_ms=round(t_icgn, 4), algorithmic_bytes_per_launch=icgn_bytes,
                     mean_iterations=float(iters.mean()) if iters.size else 0.0,
                     issue=measured_issue("icgn_f32", t_icgn))
    roofline = roof_search if t_search >= t_icgn else roof_icgn

    rec = {
        "metric": METRIC, "value": round(N / (ms * 1e-3), 1), "unit": "POIs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "affine_1024: one 1024x1024 float32 speckle pair (16,000 "
                               "Gaussian blobs), u = 0.005x + 1.3, v = -0.0015y - 0.6, noise "
                               "sigma 2, subset 31x31, step 5, search +-16, 36,864 POIs, "
                               "IC-GN stop |dp| < 1e-3 or 20 iterations",
                   "form": "FP32 batched: bf16 matrix-core search filter with FP64 re-score, "
                           "FP32 IC-GN with FP64 solve, HIP graph",
                   "tuning": list(plan.tuning)},
        "roofline": roofline,
        "rooflines": {"search": roof_search, "icgn": roof_icgn},
        "stages_ms": {"reference_prep": round(t_prep, 4), "deformed_box_sums": round(t_box, 4),
                      "search": round(t_search, 4), "icgn": round(t_icgn, 4)},
        "icgn_pois_per_s": round(N / (t_icgn * 1e-3), 1),
        "status_histogram": dic.status_histogram(got["status"]),
        "fp64_plain": {"pois_per_s": round(N / (ms64 * 1e-3), 1), "ms_per_step": round(ms64, 3),
                       "search_ms": round(t64_search, 3), "icgn_ms": round(t64_icgn, 3),
                       "icgn_pois_per_s": round(N / (t64_icgn * 1e-3), 1)},
        "fp32_over_fp64_plain": round(ms64 / ms, 2),
        "icgn_fp32_over_fp64_plain": round(t64_icgn / t_icgn, 2),
        "max_fp32_vs_fp64_plain_px": fp32_vs_fp64,
        "newton_raphson": {
            "refine_ms": round(t_nr, 4), "pois_per_s": round(N / (t_nr * 1e-3), 1),
            "fp64_plain_refine_ms": round(t64_nr, 3),
            "fp32_over_fp64_plain": round(t64_nr / t_nr, 2),
            "mean_iterations": float(nr_it[nr_st == 0].mean()) if (nr_st == 0).any() else 0.0,
            "ok_fraction": float((nr_st == 0).mean()),
            "max_fp32_vs_fp64_plain_px": nr_fp32_vs_fp64,
            "max_vs_icgn_px": float(np.abs(nr_p[okn & (got["status"] == 0)][:, [0, 3]]
                                           - got["p"][okn & (got["status"] == 0)][:, [0, 3]]
                                           ).max(initial=0)),
            "issue": measured_issue("nr_f32", t_nr),
        },
        "particle_swarm": swarm,
        "bilinear": bil,
        "bicubic_lut": lut,
        "bspline": bsp,
    }
    if not args.no_configs:
        rec["batched"] = batched_bench(torch, dic, dicgen, dev, reps)
        rec["differentiation"] = adjoint_bench(torch, dic, dicgen, dev, reps)
    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_probe_bytes_each_way"] = n * 4
    if not args.no_cpu_baseline:
        base, acc = cpu_baseline(pair, got, args.cpu_sample, pool=pool, procs=procs,
                                 extra=None if args.no_configs else oracle_other_workloads)
        if pool is not None:
            pool.close()
            pool.join()
        rec["cpu_baseline"] = base
        rec["accuracy_vs_oracle"] = acc
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
