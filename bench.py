#!/usr/bin/env python3
"""Benchmark: closest-hit BVH traversal with the alpha-mask intersector at 1080p.

Workload: 100k camera-facing alpha-masked billboards (200k triangles, 16 RGBA8
256x256 textures, ~40 % zero-alpha texels), 1920x1080 primary rays, alpha
threshold 0.5 (alpha byte >= 128).  One step = one rt_trace_closest launch
over all 2,073,600 rays (ray setup, traversal, triangle tests, alpha lookups,
hit output), inputs and BVH resident in device memory.

Prints ONE JSON line: Mrays/s, the roofline of the traversal kernel (HBM
bytes per launch measured by rocprofv3 over the launch time measured here,
against the 8 TB/s peak; the texture-addresser busy fraction, the roof the
counters show binding; and the bytes the method touches per ray, from exact
per-ray counts of a separate counting launch, as a request rate), and the CPU
oracle timed on this host's cores on the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --copy-calibration   # plain copy kernel for counter scaling
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
N_CUS, CLOCK_GHZ = 256, 2.4    # MI355X compute units and peak engine clock
# one texture addresser per CU, busy at most every cycle
PEAK_TA_GCYCLES = N_CUS * CLOCK_GHZ
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1912_12786_amd", "csrc", f)
                  for f in ("rt_traverse.hpp", "trace_kernels.hip", "rt_launch.hpp",
                            "rt_batch_layout.hpp")]
# the differentiable hit's other kernels (adjoint, refit), hashed apart so that
# the traversal's counter records stay keyed to the traversal sources alone
AUX_KERNEL_SOURCES = [os.path.join(ROOT, "paper_1912_12786_amd", "csrc", f)
                      for f in ("hit_backward.hip", "bvh_refit.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def emit(line: dict):
    """Prints one JSON result line, tagged with the kernel sources it ran."""
    line.setdefault("kernel_source_sha", kernel_source_sha())
    print(json.dumps(line), flush=True)


def kernel_source_sha(sources=None) -> str:
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def default_order(workload: str, kind: str, query: str) -> str:
    """The chunk order bench.py uses unless ``--order`` names one: longest
    path first for the alpha mask's closest, any and k-nearest hits and the
    accept-all closest hit on the billboards, where it was measured faster
    (also in a lane-per-ray shape without the queue, whose waves take their
    chunks in that order), ray-index order elsewhere, where it was measured
    slower."""
    if workload != "billboards":
        return "index"
    if kind == "alpha" and query in ("closest", "any", "multi"):
        return "longest-first"
    return "longest-first" if (kind, query) == ("default", "closest") else "index"


def default_build(workload: str, intersector, query: str):
    """(node layout, launch shape or None) bench.py uses unless --layout or
    --shape name them: 8-bit nodes for the spheres and the batch, where the
    node working set outgrows the caches, packed 48-byte nodes on the
    billboards, float32 nodes otherwise; the library's default shape except
    for the accept-all closest hit on the billboards, where the build
    autotuner chose a lane per ray without the queue (short, even rays lose
    more coherence to refills than the queue saves)."""
    kind = intersector or {"billboards": "alpha"}.get(workload)
    layout = ("q8" if workload in ("spheres", "batched") else
              "f32p" if workload == "billboards" and kind in ("alpha", "default") else "f32")
    shape = "64,8,64,0" if (workload, kind, query) == ("billboards", "default", "closest") else None
    return layout, shape


def find_counters(sha, workload, kind, query, layout, max_leaf, shape, ray_order,
                  schedule="index", order="index", waves=7):
    """The rocprofv3 counter record (``profiles/counters_*.json``) taken on
    exactly this kernel source and configuration, or None."""
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if not (name.startswith("counters_") and name.endswith(".json")):
            continue
        with open(os.path.join(PROFILES, name)) as f:
            rec = json.load(f)
        cfg = rec.get("config", {})
        if (rec.get("kernel_source_sha") == sha and cfg.get("workload") == workload
                and cfg.get("intersector") == kind and cfg.get("query") == query
                and cfg.get("layout") == layout and cfg.get("max_leaf") == max_leaf
                and cfg.get("launch_shape") == list(shape)
                and cfg.get("ray_order", "scanline") == ray_order
                and cfg.get("schedule", "index") == schedule
                and cfg.get("order", "index") == order
                and cfg.get("waves_per_simd") == waves):
            rec["file"] = os.path.join("profiles", name)
            return rec
    return None


def roofline(kernel_ms: float, alg_bytes: int, rec) -> dict:
    """The roofline object of the dominant kernel.

    ``achieved``/``frac``: HBM bytes per launch measured by rocprofv3
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's reading of the same
    counters; ``traffic``) over the mean launch time measured here, against
    the 8 TB/s HBM peak.  They are null when no counter record matches the
    current kernel source and configuration.  ``issue``: the texture
    addresser's busy fraction from the same record (every vector memory
    instruction passes through it), the roof the counters show binding.
    ``algorithmic_gbs``: the bytes the method touches per launch (per-ray
    counts x record sizes, cache hits included) over the same time; it is a
    request rate, not DRAM traffic, and may exceed the HBM peak."""
    sec = kernel_ms * 1e-3
    out = {"bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": None,
           "traffic": None}
    if rec is not None:
        if rec.get("traffic_bytes_per_launch") is not None:
            traffic = int(rec["traffic_bytes_per_launch"])
            gbs = traffic / sec / 1e9
            out.update(achieved=round(gbs, 1), frac=round(gbs / PEAK_HBM_GBS, 4), traffic=traffic)
        if rec.get("ta_busy_frac") is not None:
            ta = float(rec["ta_busy_frac"])
            out["limiter"] = rec.get("limiter", "vmem_issue")
            out["issue"] = {"bound": "vmem_issue", "unit": "G TA-cycles/s",
                            "achieved": round(ta * PEAK_TA_GCYCLES, 1), "peak": PEAK_TA_GCYCLES,
                            "frac": round(ta, 4),
                            "vmem_rd_wave_instr_per_launch": rec.get("vmem_rd_wave_instr"),
                            "valu_lane_utilisation": rec.get("valu_lane_utilisation")}
        out["counters_file"] = rec["file"]
    out["algorithmic_gbs"] = round(alg_bytes / sec / 1e9, 1)
    out["algorithmic_frac_of_hbm_peak"] = round(alg_bytes / sec / 1e9 / PEAK_HBM_GBS, 4)
    return out


def bytes_per_ray(counters: np.ndarray, kind: str, node_bytes: int = 64,
                  children: int = 2) -> np.ndarray:
    """Algorithmic bytes of one ray: its 32-byte ray record and 16-byte hit
    record, one node record (64 bytes, 32 in the compressed layout, 128 in the
    four-wide one) per inner node entered (box tests are the root's plus one
    per child of every inner node entered: two, or up to four in the wide
    layout, where bytes are counted per box test as a quarter record, exact
    for full nodes), one 48-byte triangle record per triangle test, and per
    alpha decision the 24 bytes of texture coordinates plus the 4-byte
    texel."""
    c = counters.astype(np.int64)
    b = (32 + 16 + node_bytes * (c[:, 0] - 1).clip(min=0) // children + 48 * c[:, 1])
    if kind == "alpha":
        b = b + 28 * c[:, 2]
    return b


def copy_calibration():
    import torch
    n = 1 << 28   # 1 GiB of float32
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    emit({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4,
                      "launches": 3})


COPY_BYTES = 1 << 30   # the calibration copy reads and writes 1 GiB


def _counter_rows(directory: str) -> list:
    """Every row of the rocprofv3 counter CSVs under ``directory``."""
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(directory, "**", "*counter_collection.csv"),
                                 recursive=True)):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    if not rows:
        raise SystemExit(f"no rocprofv3 counter CSV under {directory}")
    return rows


def _per_dispatch(rows, match, first_n=None) -> dict:
    """Mean value per dispatch of each counter over the dispatches of the
    kernels whose name ``match`` accepts (the first ``first_n`` of them, in
    dispatch order, when given), and the number of dispatches used."""
    by_dispatch = {}
    for r in rows:
        if not match(r["Kernel_Name"]):
            continue
        d = by_dispatch.setdefault(int(r["Dispatch_Id"]), {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    ids = sorted(by_dispatch)[:first_n] if first_n else sorted(by_dispatch)
    if not ids:
        raise SystemExit("no dispatch of the selected kernel in the counter CSV")
    names = set().union(*(by_dispatch[i] for i in ids))
    return {"n": len(ids), **{k: sum(by_dispatch[i].get(k, 0.0) for i in ids) / len(ids)
                              for k in names}}


def kernel_tail(shape, batched: bool, layout: str) -> str:
    """The end of the traversal kernel's demangled name for one launch shape,
    batched flag and node layout (its last template arguments)."""
    block, slots, chunk, queue = shape
    code = {"f32": 0, "q8": 1, "wide4": 2, "f32p": 3}[layout]
    return (f", {slots}, {block}, {chunk}, {'true' if queue else 'false'}, "
            f"{'true' if batched else 'false'}, {code}u>")


def ingest_counters(args, directory: str):
    """Writes ``profiles/counters_<config>.json`` from the rocprofv3 passes
    under ``directory``: ``issue/`` (texture-addresser and SQ counters) of
    ``bench.py --steps S --warmup W --no-cpu-baseline`` with this run's
    configuration flags, its stdout in ``issue.log`` (whose JSON line names
    the kernel sources measured) and, when present, ``fetch/`` (FETCH_SIZE) and
    ``write/`` (WRITE_SIZE) of the same command with ``copy_fetch/``,
    ``copy_write/`` of ``bench.py --copy-calibration``, which scale the two
    HBM counters.  Only the timed (non-counting) trace kernel of exactly this
    launch shape, batched flag and node layout is read; single-scene runs use
    their first W + S dispatches of it, the batched run every one (each
    traces the whole batch)."""
    from paper_1912_12786_amd import rtx
    batched = args.workload == "batched"
    kind = "default" if batched else (args.intersector or {
        "billboards": "alpha", "tiny": "default", "spheres": "procedural"}[args.workload])
    isect = {"alpha": "alpha_intersector", "default": "default_intersector",
             "procedural": "checker_intersector"}[kind]
    res = {"closest": "closest_result", "any": "any_result",
           "multi": f"multi_result<{args.k}>"}[args.query]
    shape = list(parse_shape(args.shape) or rtx.rt_launch_shapes()[0])
    tail = kernel_tail(shape, batched, args.layout)

    def trace_kernel(name):
        return ("trace_kernel<" in name and f"rtx::{isect}," in name and "counting" not in name
                and f"rtx::{res}" in name and tail in name)

    def copy_kernel(name):
        return "copy" in name.lower()

    def have(sub):
        return os.path.isdir(os.path.join(directory, sub))

    # the kernel sources the profiled runs were built from: the sha each run
    # printed in its JSON line (stdout of the profiled command, saved as
    # <pass>.log beside the pass's folder)
    shas = set()
    for sub in ("issue", "fetch", "write"):
        log_path = os.path.join(directory, sub + ".log")
        if not os.path.exists(log_path):
            continue
        with open(log_path, errors="replace") as f:
            for line in f:
                if line.startswith("{") and "kernel_source_sha" in line:
                    shas.add(json.loads(line)["kernel_source_sha"])
    if len(shas) != 1:
        raise SystemExit(f"expected one kernel_source_sha in the passes' logs, found {shas}")
    sha = shas.pop()

    n = None if batched else args.warmup + args.steps
    issue = _per_dispatch(_counter_rows(os.path.join(directory, "issue")), trace_kernel, n)
    grbm = issue["GRBM_GUI_ACTIVE"]          # summed over the 8 XCDs
    ta_busy = issue["TA_TA_BUSY_sum"] / N_CUS / (grbm / 8)
    lane_util = issue["SQ_THREAD_CYCLES_VALU"] / (64 * issue["SQ_ACTIVE_INST_VALU"])
    if batched:
        wl_name = "batched_64_scenes"
    else:
        wl_name = {"billboards": "billboards_200000_tris_1920x1080"}.get(args.workload)
        if wl_name is None:
            from paper_1912_12786_amd import workloads as W
            wl_name = {"tiny": W.tiny, "spheres": W.spheres}[args.workload]().name
    # tiles apply to scanline rays of an image (every single-scene workload is one)
    schedule = "index" if (batched or args.ray_order != "scanline") else args.schedule
    order = "index" if batched else (args.order or default_order(args.workload, kind, args.query))
    flags = (f"--workload {args.workload}" + ("" if batched else f" --intersector {kind} "
             f"--query {args.query} --ray-order {args.ray_order} --schedule {schedule} "
             f"--order {order}")
             + f" --layout {args.layout} --max-leaf {args.max_leaf}"
             + (f" --shape {args.shape}" if args.shape else "")
             + (f" --waves-per-simd {args.waves_per_simd}" if args.waves_per_simd else ""))
    waves = args.waves_per_simd or rtx.RT_DEFAULT_WAVES_PER_SIMD
    base = f"python3 bench.py {flags} --steps {args.steps} --warmup {args.warmup} --no-cpu-baseline"
    pmc = "rocprofv3 --pmc {} --output-format csv -d <out>/{} -o bench -- "
    rec = {
        "kernel_source_sha": sha,
        "config": {"workload": wl_name, "intersector": kind, "query": args.query,
                   "layout": args.layout, "max_leaf": args.max_leaf, "launch_shape": shape,
                   "ray_order": args.ray_order, "schedule": schedule, "order": order,
                   "waves_per_simd": waves},
        "kernel": f"trace_kernel<{isect}, {res}{tail}",
        "dispatches": {"issue": issue["n"]},
        "ta_busy_frac": round(ta_busy, 4),
        "limiter": "vmem_issue",
        "vmem_rd_wave_instr": int(round(issue["SQ_INSTS_VMEM_RD"])),
        "valu_wave_instr": int(round(issue["SQ_INSTS_VALU"])),
        "valu_lane_utilisation": round(lane_util, 4),
        "waves": int(round(issue["SQ_WAVES"])),
        "gpu_active_cycles_per_xcd": int(round(grbm / 8)),
        "commands": {"issue": pmc.format(" ".join(ISSUE_COUNTERS), "issue") + base},
    }
    if have("fetch") and have("write") and have("copy_fetch") and have("copy_write"):
        fetch = _per_dispatch(_counter_rows(os.path.join(directory, "fetch")), trace_kernel, n)
        write = _per_dispatch(_counter_rows(os.path.join(directory, "write")), trace_kernel, n)
        cf = _per_dispatch(_counter_rows(os.path.join(directory, "copy_fetch")), copy_kernel)
        cw = _per_dispatch(_counter_rows(os.path.join(directory, "copy_write")), copy_kernel)
        f_fac = COPY_BYTES / (cf["FETCH_SIZE"] * 1024)
        w_fac = COPY_BYTES / (cw["WRITE_SIZE"] * 1024)
        traffic = fetch["FETCH_SIZE"] * 1024 * f_fac + write["WRITE_SIZE"] * 1024 * w_fac
        rec["dispatches"].update(fetch=fetch["n"], write=write["n"])
        rec.update({
            "fetch_kib_per_dispatch": round(fetch["FETCH_SIZE"], 2),
            "write_kib_per_dispatch": round(write["WRITE_SIZE"], 2),
            "copy_calibration": {"bytes_copied": COPY_BYTES, "fetch_kib": round(cf["FETCH_SIZE"], 2),
                                 "write_kib": round(cw["WRITE_SIZE"], 2),
                                 "fetch_factor": round(f_fac, 5), "write_factor": round(w_fac, 5)},
            "traffic_bytes_per_launch": int(round(traffic)),
        })
        rec["commands"].update({
            "fetch": pmc.format("FETCH_SIZE", "fetch") + base,
            "write": pmc.format("WRITE_SIZE", "write") + base,
            "copy_fetch": pmc.format("FETCH_SIZE", "copy_fetch") + "python3 bench.py --copy-calibration",
            "copy_write": pmc.format("WRITE_SIZE", "copy_write") + "python3 bench.py --copy-calibration",
        })
    rec["commands"]["ingest"] = (f"python3 bench.py --ingest-counters <out> {flags} "
                                 f"--steps {args.steps} --warmup {args.warmup}")
    name = (f"counters_{args.workload}_{kind}_{args.query}_{args.layout}_leaf{args.max_leaf}_"
            f"{'x'.join(map(str, shape))}_{args.ray_order}_{schedule}_{order}_w{waves}.json")
    with open(os.path.join(PROFILES, name), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps({"written": os.path.join("profiles", name), **rec}))


# one pass of texture-addresser and SQ counters (within one pass's limits:
# 6 SQ, 1 TA, 1 GRBM)
ISSUE_COUNTERS = ("TA_TA_BUSY_sum", "GRBM_GUI_ACTIVE", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VALU",
                  "SQ_THREAD_CYCLES_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVES")


def _morton2(x: np.ndarray, y: np.ndarray, bits: int) -> np.ndarray:
    """Interleaves the low ``bits`` bits of x (even positions) and y (odd)."""
    k = np.zeros_like(x)
    for b in range(bits):
        k |= ((x >> b) & 1) << (2 * b) | ((y >> b) & 1) << (2 * b + 1)
    return k


def tile_order(wl, tile: int = 8, morton: bool = False) -> np.ndarray:
    """Permutation of a pinhole workload's primary rays (scanline order, the
    first width x height rays) into tile x tile pixel blocks (row-major inside
    a block, or Z-order with ``morton``); other rays keep their place."""
    w, h = int(wl.extra["width"]), int(wl.extra["height"])
    y, x = np.divmod(np.arange(w * h), w)
    inner = _morton2(x % tile, y % tile, int(tile).bit_length() - 1) if morton else (y % tile) * tile + x % tile
    key = ((y // tile) * ((w + tile - 1) // tile) + x // tile) * tile * tile + inner
    order = np.argsort(key, kind="stable")
    return np.concatenate([order, np.arange(w * h, wl.n_rays)])


def parse_shape(text):
    """--shape BLOCK,LDS_SLOTS,CHUNK,QUEUE -> tuple, or None for the default."""
    return tuple(int(x) for x in text.split(",")) if text else None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, kind, kind_kw, threads, budget_s=8.0, layout="f32", max_leaf=4):
    """The oracle as it stands, on this host's cores, on the same workload:
    oracle B (float32 BVH traversal of its own BVH, in the node layout the
    GPU run used) over every ray, repeated until about ``budget_s`` seconds
    have passed (median pass reported), the same on one thread over every
    16th ray, and oracle A (float64 brute force over every triangle) on a ray
    sample sized to about ``budget_s / 2`` seconds."""
    import oracle
    from paper_1912_12786_amd import workloads as W
    oracle.build(force=False)
    t0 = time.perf_counter()
    bvh = oracle.build_bvh(wl.vertices, max_leaf=max_leaf)
    if layout == "q8":
        bvh.qbox = oracle.quantize(bvh)["qbox"]
    if layout == "f32p":
        bvh.pbox = oracle.pack(bvh)["box"]
    t_build = time.perf_counter() - t0
    passes = []
    while not passes or (sum(passes) < budget_s and len(passes) < 50):
        t0 = time.perf_counter()
        oracle.traverse(wl.vertices, bvh, wl.rays, kind, count=False, threads=threads,
                        layout=layout, **kind_kw)
        passes.append(time.perf_counter() - t0)
    t_b = float(np.median(passes))
    sub = wl.rays[::16]
    t0 = time.perf_counter()
    oracle.traverse(wl.vertices, bvh, sub, kind, count=False, threads=1, layout=layout, **kind_kw)
    t_b1 = time.perf_counter() - t0
    # size the brute-force sample from a short probe
    probe = W.subsample_indices(wl.n_rays, None, None, seed=7, n_random=256)
    t0 = time.perf_counter()
    oracle.brute(wl.vertices, wl.rays, kind, ray_index=probe, threads=threads, **kind_kw)
    t_probe = time.perf_counter() - t0
    n_a = int(min(wl.n_rays, max(256, len(probe) * (budget_s / 2) / max(t_probe, 1e-3))))
    idx = W.subsample_indices(wl.n_rays, None, None, seed=8, n_random=n_a)
    t0 = time.perf_counter()
    oracle.brute(wl.vertices, wl.rays, kind, ray_index=idx, threads=threads, **kind_kw)
    t_a = time.perf_counter() - t0
    return {
        "value": round(wl.n_rays / t_b / 1e6, 3),
        "unit": "Mrays/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle B (float32 BVH traversal, {layout} nodes, leaves of <= {max_leaf}; "
                   f"its own BVH built in "
                   f"{t_build:.2f} s) over "
                   f"all {wl.n_rays} rays, {len(passes)} passes, median {t_b:.3f} s; oracle A "
                   f"(float64 brute force over all {wl.n_tris} triangles) on {len(idx)} sampled "
                   f"rays in {t_a:.2f} s"),
        "single_thread_mrays_s": round(sub.shape[0] / t_b1 / 1e6, 3),
        "bruteforce_mrays_s": round(len(idx) / t_a / 1e6, 6),
        "bruteforce_full_set_s": round(wl.n_rays * t_a / len(idx), 1),
        "cpu_model": cpu_model(),
    }


def timed(fn, steps, warmup, stream):
    """Mean wall time per call (ms) of fn over `steps` calls after `warmup`."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def bench_diff(args):
    """Differentiable hit: 512x512 rays, perturbed 50k-triangle geodesic sphere
    plus 5k alpha billboards; loss = sum w.(t, u, v).  Forward = one alpha
    closest-hit launch; forward+backward adds the zeroing of the vertex
    gradient and one rt_hit_backward launch; beside them the plain default
    intersector on the same scene and rays.  Without --shape the autotuner
    picks the launch shape of these 262 k rays (fewer than the resident
    lanes) first, untimed, on the alpha forward."""
    import torch
    from paper_1912_12786_amd import autotune, diff, rtx
    from paper_1912_12786_amd import workloads as W
    dev = torch.device("cuda:0")
    width = 512
    wl = W.diff_scene(width=width, height=width)
    tw = width if args.schedule == "tiles" else None  # 8x8 tiles of the square image
    scene = rtx.upload_scene(wl.triangles, wl.geom_ids, wl.texcoords, wl.textures, device=dev,
                             max_leaf=args.max_leaf)
    rays = torch.from_numpy(wl.rays).to(dev)
    n = wl.rays.shape[0]
    hits = torch.empty((n, 4), dtype=torch.float32, device=dev)
    V = torch.from_numpy(wl.vertices).to(dev)
    F = torch.from_numpy(wl.faces.astype(np.int32)).to(dev)
    w = torch.from_numpy(wl.weights).to(dev)
    gV = torch.zeros_like(V)
    gR = torch.empty_like(rays)
    ws = rtx.Workspace(dev)
    stream = torch.cuda.current_stream(dev)
    shape_ms = None
    if args.shape:
        shape = parse_shape(args.shape)
    else:
        shape, shape_ms = autotune.tune(
            "bench-diff-alpha",
            lambda sh: rtx.trace(scene, rays, "alpha", alpha_min=128, out=hits, workspace=ws,
                                 shape=sh, image_width=tw),
            cache_path=None, steps=10, warmup=2)
        log(f"autotuner: differentiable-hit launch shape {','.join(map(str, shape))}")

    def fwd():
        rtx.trace(scene, rays, "alpha", alpha_min=128, out=hits, workspace=ws, shape=shape,
                  image_width=tw)

    def fwd_bwd():
        fwd()
        gV.zero_()
        rtx.rt_hit_backward(rays.data_ptr(), hits.data_ptr(), w.data_ptr(), n, V.data_ptr(),
                            V.shape[0], F.data_ptr(), F.shape[0], gV.data_ptr(), gR.data_ptr(),
                            stream.cuda_stream)

    def plain():
        rtx.trace(scene, rays, "default", out=hits, workspace=ws, shape=shape, image_width=tw)

    # moving geometry: the same forward on a tree refitted on the device to
    # the vertices every step (rt_bvh_refit, then the 24-byte root box to the
    # host), against rebuilding the tree on the host (timed by wall clock)
    rs = rtx.RefitScene(wl.vertices, wl.faces, wl.geom_ids, wl.texcoords, wl.textures,
                        device=dev, max_leaf=args.max_leaf)

    def refit_only():
        rs.update(V)

    def refit_fwd():
        rs.update(V)
        rtx.trace(rs.scene, rays, "alpha", alpha_min=128, out=hits, workspace=ws, shape=shape,
                  image_width=tw)

    ms_f = timed(fwd, args.steps, args.warmup, stream)
    ms_fb = timed(fwd_bwd, args.steps, args.warmup, stream)
    ms_p = timed(plain, args.steps, args.warmup, stream)
    ms_r = timed(refit_only, args.steps, args.warmup, stream)
    ms_rf = timed(refit_fwd, args.steps, args.warmup, stream)
    rebuild = []
    for _ in range(3):
        t0 = time.perf_counter()
        rtx.upload_scene(wl.triangles, wl.geom_ids, wl.texcoords, wl.textures, device=dev,
                         max_leaf=args.max_leaf)
        torch.cuda.synchronize()
        rebuild.append((time.perf_counter() - t0) * 1e3)
    emit({
        "metric": "Mrays/s differentiable closest hit (alpha mask): forward, forward+backward, "
                  "plain default-intersector kernel on the same scene",
        "value": round(n / ms_fb / 1e3, 2), "unit": "Mrays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_tris": int(wl.faces.shape[0]), "max_leaf": args.max_leaf,
                   "n_vertices": int(wl.vertices.shape[0]), "n_rays": n,
                   "schedule": ("8x8 pixel tiles" if tw else "index order"),
                   "launch_shape": list(shape) if shape else None},
        "autotuned_shape_ms": shape_ms,
        "forward_mrays_s": round(n / ms_f / 1e3, 2),
        "forward_backward_mrays_s": round(n / ms_fb / 1e3, 2),
        "plain_default_mrays_s": round(n / ms_p / 1e3, 2),
        "refit_forward_mrays_s": round(n / ms_rf / 1e3, 2),
        "ms": {"forward": round(ms_f, 4), "forward_backward": round(ms_fb, 4),
               "plain_default": round(ms_p, 4), "device_refit": round(ms_r, 4),
               "device_refit_forward": round(ms_rf, 4),
               "host_rebuild_upload": round(float(np.median(rebuild)), 2)},
        "aux_kernel_source_sha": kernel_source_sha(AUX_KERNEL_SOURCES),
    })
    del diff


def bench_batched(args):
    """64 scenes of uneven size (5.1M triangles, 19.9M rays in total), default
    intersector, closest hit: one batched persistent launch (eager and replayed
    from a captured graph) against 64 separate per-scene launches (eager and
    graph-replayed).  The batched launch's shape is picked by the autotuner
    unless --shape names one."""
    import torch
    from paper_1912_12786_amd import autotune, rtx
    from paper_1912_12786_amd import workloads as W
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    scenes = W.batched()
    sc_list = [rtx.upload_scene(s["vertices"], device=dev, layout=args.layout,
                                max_leaf=args.max_leaf) for s in scenes]
    counts = [s["rays"].shape[0] for s in scenes]
    batch = rtx.Batch(sc_list, counts, "default", device=dev)
    rays = torch.from_numpy(np.concatenate([s["rays"] for s in scenes])).to(dev)
    torch.cuda.synchronize()
    log(f"batched workload: {len(scenes)} scenes, {sum(s['vertices'].shape[0] for s in scenes)} "
        f"tris, {rays.shape[0]} rays, prepared in {time.perf_counter() - t0:.1f} s")
    n = rays.shape[0]
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    ws = rtx.Workspace(dev)
    offs = batch.offsets
    views = [rays[offs[i]:offs[i + 1]] for i in range(len(scenes))]
    outs = [out[offs[i]:offs[i + 1]] for i in range(len(scenes))]
    stream = torch.cuda.current_stream(dev)

    best = None

    def batched(shape=None):
        batch.trace(rays, out=out, workspace=ws, shape=shape or best,
                    waves_per_simd=args.waves_per_simd)

    def separate():
        for sc, r, o in zip(sc_list, views, outs):
            if r.shape[0]:
                rtx.trace(sc, r, "default", out=o, workspace=ws)

    if args.shape:   # a given shape skips the autotuner
        best, tune_ms = parse_shape(args.shape), None
    else:
        best, tune_ms = autotune.tune("batched-64-scenes-default", batched, cache_path=None,
                                      steps=3, warmup=1)
    # grow the workspace to the largest need before any capture
    ws.get(max(rtx.rt_trace_batch_workspace_bytes(batch.info, rtx.shape_flag(best)),
               max(rtx.rt_trace_workspace_bytes(sc.view, c) for sc, c in zip(sc_list, counts))))

    def graph_of(fn):
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            fn()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        return g

    g_batched = graph_of(batched)
    g_separate = graph_of(separate)
    ms = {
        "batched_eager": timed(batched, args.steps, args.warmup, stream),
        "batched_graph": timed(g_batched.replay, args.steps, args.warmup, stream),
        "separate_eager": timed(separate, args.steps, args.warmup, stream),
        "separate_graph": timed(g_separate.replay, args.steps, args.warmup, stream),
    }
    emit({
        "metric": "Mrays/s closest hit over a batch of 64 scenes (default intersector): one "
                  "persistent launch vs 64 per-scene launches",
        "value": round(n / ms["batched_graph"] / 1e3, 2), "unit": "Mrays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched_{len(scenes)}_scenes", "n_scenes": len(scenes),
                   "node_layout": args.layout, "max_leaf": args.max_leaf,
                   "n_tris": int(sum(s["vertices"].shape[0] for s in scenes)), "n_rays": int(n),
                   "launch_shape": list(best),
                   "waves_per_simd": args.waves_per_simd or rtx.RT_DEFAULT_WAVES_PER_SIMD},
        "mrays_s": {k: round(n / v / 1e3, 2) for k, v in ms.items()},
        "ms": {k: round(v, 4) for k, v in ms.items()},
        "autotune_ms": tune_ms,
    })


def bench_dispatch(args):
    """Compile-time intersector vs the same decision dispatched at run time
    (an inlined switch, or an indirect call through a function table) on the
    billboard workload, for the default and the alpha-mask intersector."""
    import torch
    from paper_1912_12786_amd import rtx
    from paper_1912_12786_amd import workloads as W
    dev = torch.device("cuda:0")
    wl = W.billboards()
    scene = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures, device=dev)
    rays = torch.from_numpy(wl.rays).to(dev)
    n = wl.n_rays
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    ws = rtx.Workspace(dev)
    stream = torch.cuda.current_stream(dev)
    sc = scene.view
    res = {}
    for kind in ("default", "alpha"):
        params = rtx._params(scene, kind, 128, 8)
        for name, flags in (("compile_time", 0), ("runtime_switch", rtx.RT_FLAG_RUNTIME_SWITCH),
                            ("runtime_call", rtx.RT_FLAG_RUNTIME_CALL)):
            wptr, wb = ws.get(rtx.rt_trace_workspace_bytes(sc, n, flags))

            def fn():
                rtx.rt_trace_closest(sc, rays.data_ptr(), n, rtx.KINDS[kind], params, flags,
                                     out.data_ptr(), None, wptr, wb, stream.cuda_stream)
            ms = timed(fn, args.steps, args.warmup, stream)
            res[f"{kind}/{name}"] = {"ms": round(ms, 4), "mrays_s": round(n / ms / 1e3, 2)}
    emit({
        "metric": "Mrays/s closest hit, compile-time intersector vs run-time dispatch "
                  "(switch, indirect call) at 1080p billboards",
        "value": res["alpha/compile_time"]["mrays_s"], "unit": "Mrays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "dtype": "f32",
        "data": "synthetic", "config": {"workload": wl.name, "n_rays": n},
        "results": res})


def bench_instanced(args):
    """Object instancing: 2000 instances of three meshes at 1080p, closest hit
    (accept-all, or the alpha mask with per-mesh texture data), against the
    same scene flattened into one BVH of world-space triangles."""
    import torch
    from paper_1912_12786_amd import rtx
    from paper_1912_12786_amd import workloads as W
    dev = torch.device("cuda:0")
    kind = args.intersector or "default"
    wl = W.instanced(2000)
    akw = W.instanced_alpha(wl) if kind == "alpha" else {}
    isc = rtx.InstancedScene(wl["blas"], wl["inst_blas"], wl["inst_m"], wl["world_lo"],
                             wl["world_hi"], device=dev, max_leaf=args.max_leaf, **akw)
    wfo = wl["world_from_object"]
    flat = np.concatenate([np.einsum("ij,tkj->tki", wfo[q, :, :3],
                                     wl["blas"][b].astype(np.float64)) + wfo[q, :, 3]
                           for q, b in enumerate(wl["inst_blas"])]).astype(np.float32)
    if akw:
        fsc = rtx.upload_scene(flat, np.concatenate([akw["geom_ids"][b] for b in wl["inst_blas"]]),
                               np.concatenate([akw["texcoords"][b] for b in wl["inst_blas"]]),
                               akw["textures"], device=dev, max_leaf=args.max_leaf)
    else:
        fsc = rtx.upload_scene(flat, device=dev, max_leaf=args.max_leaf)
    rays = torch.from_numpy(wl["rays"]).to(dev)
    n = rays.shape[0]
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    ids = torch.empty((n,), dtype=torch.int32, device=dev)
    ws = rtx.Workspace(dev)
    stream = torch.cuda.current_stream(dev)
    # both launches take the image's rays in 8x8 tiles unless --schedule index
    tw = int(wl["width"]) if args.schedule == "tiles" else None
    ms_i = timed(lambda: isc.trace(rays, kind, out=out, inst_ids=ids, workspace=ws,
                                   image_width=tw), args.steps, args.warmup, stream)
    ms_f = timed(lambda: rtx.trace(fsc, rays, kind, out=out, workspace=ws, image_width=tw),
                 args.steps, args.warmup, stream)
    bytes_i = sum(int(b.tris.numel()) + (int(b.nodes.numel()) if b.nodes is not None else 0)
                  for b in isc.blas) + int(isc.tlas_tris.numel()) + int(isc.tlas_nodes.numel()) \
        + int(isc.table.numel())
    bytes_f = int(fsc.tris.numel()) + int(fsc.nodes.numel())
    if akw:  # texture coordinates (the shared textures are the same on both sides)
        bytes_i += sum(int(b.texcoords.numel()) * 4 for b in isc.blas)
        bytes_f += int(fsc.texcoords.numel()) * 4
    emit({
        "metric": f"Mrays/s closest hit ({kind}), instanced two-level BVH vs the flattened scene",
        "value": round(n / ms_i / 1e3, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["name"], "n_instances": 2000, "n_rays": n,
                   "max_leaf": args.max_leaf,
                   "world_tris": int(flat.shape[0]), "intersector": kind,
                   "schedule": ("8x8 pixel tiles" if tw else "index order")},
        "instanced_mrays_s": round(n / ms_i / 1e3, 2), "flattened_mrays_s": round(n / ms_f / 1e3, 2),
        "ms": {"instanced": round(ms_i, 4), "flattened": round(ms_f, 4)},
        "scene_bytes": {"instanced": bytes_i, "flattened": bytes_f}})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--ingest-counters", metavar="DIR", default=None,
                    help="write profiles/counters_<config>.json from rocprofv3 counter passes "
                         "under DIR (fetch/, write/, issue/, copy_fetch/, copy_write/) taken "
                         "with the same configuration flags; no GPU needed")
    ap.add_argument("--shape", default=None,
                    help="launch shape BLOCK,LDS_SLOTS,CHUNK,QUEUE (default: the library's default)")
    ap.add_argument("--intersector", default=None, choices=["alpha", "default", "procedural"],
                    help="default: alpha on billboards, accept-all on tiny, procedural checker "
                         "on spheres")
    ap.add_argument("--ray-order", default="scanline", choices=["scanline", "tiled", "morton"],
                    help="tiled: primary rays reordered into 8x8 pixel tiles before upload "
                         "(hits come back in that order); morton: the same tiles in Z-order")
    ap.add_argument("--max-leaf", type=int, default=None,
                    help="leaf size limit of the BVH build (1..7; the library's default is 4). "
                         "Default: 2 (measured fastest on the billboards, spheres, diff and "
                         "batched scenes), 4 for instanced (its bottom-level meshes; 2 is 1 %% "
                         "slower there). Not used by the dispatch ablation")
    ap.add_argument("--tune-build", action="store_true",
                    help="let the autotuner choose leaf size (2, 3, 4), node layout and launch "
                         "shape for the billboards/tiny/spheres workload (overrides --max-leaf, "
                         "--layout and --shape)")
    ap.add_argument("--layout", default=None, choices=["f32", "q8", "f32p", "wide4"],
                    help="inner-node layout: f32 = 64-B binary nodes with float32 boxes, q8 = "
                         "32-B binary nodes with 8-bit boxes (rt_bvh_compress), f32p = 48-B "
                         "binary nodes with float32 boxes carrying the child references "
                         "(rt_bvh_pack), wide4 = 128-B "
                         "four-wide nodes with float32 boxes (rt_bvh_widen). Default: q8 for the "
                         "spheres and batched workloads (measured faster: BVHs beyond the "
                         "caches), f32p for the alpha mask on the billboards (measured +1.6 %% "
                         "closest, +2.6 %% any hit), f32 otherwise")
    ap.add_argument("--schedule", default="tiles", choices=["tiles", "index"],
                    help="tiles: the image's rays are handed to lanes in 8x8 pixel tiles "
                         "(RT_FLAG_TILE_WIDTH; results and their order unchanged); index: in "
                         "ray-index order. Applies to the billboards, tiny, spheres and instanced "
                         "workloads (the spheres' primary rays)")
    ap.add_argument("--order", default=None, choices=["longest-first", "index"],
                    help="longest-first: chunks of rays handed out by decreasing stretch inside "
                         "the scene box (RT_FLAG_LONGEST_FIRST; results unchanged); default: "
                         "longest-first for the alpha-mask closest and any hit on the "
                         "billboards (measured +7.5 %% and +9 %%), index otherwise (measured "
                         "-0.5 to -3 %% with it: accept-all, the spheres' mixed primary and "
                         "bounce rays)")
    ap.add_argument("--waves-per-simd", type=int, default=None,
                    help="most resident waves per SIMD of a queue launch's persistent grid "
                         "(RT_FLAG_WAVES_PER_SIMD, 1..15; results unchanged); default: the "
                         "library's, 7")
    ap.add_argument("--query", default="closest", choices=["closest", "any", "multi"])
    ap.add_argument("--k", type=int, default=4, help="hits kept per ray by --query multi")
    ap.add_argument("--workload", default="billboards",
                    choices=["billboards", "tiny", "spheres", "diff", "batched", "dispatch",
                             "instanced"],
                    help="diff = differentiable hit on the perturbed icosphere (forward, "
                         "forward+backward, the plain kernel, and the forward on a tree "
                         "refitted on the device), reported on its own line")
    args = ap.parse_args()
    if args.max_leaf is None:
        args.max_leaf = 4 if args.workload == "instanced" else 2
    layout0, shape0 = default_build(args.workload, args.intersector, args.query)
    if args.layout is None:
        args.layout = layout0
    if args.shape is None and not args.tune_build:
        args.shape = shape0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the traversal shards by rays with no exchange "
              "step, so multi-GPU runs are not part of this benchmark", file=sys.stderr)
        sys.exit(2)

    if args.ingest_counters:
        ingest_counters(args, args.ingest_counters)
        return
    import torch
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "diff":
        bench_diff(args)
        return
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "dispatch":
        bench_dispatch(args)
        return
    if args.workload == "instanced":
        bench_instanced(args)
        return
    from paper_1912_12786_amd import rtx
    from paper_1912_12786_amd import workloads as W

    kind = args.intersector or {"billboards": "alpha", "tiny": "default",
                                "spheres": "procedural"}[args.workload]
    if kind == "alpha" and args.workload != "billboards":
        raise SystemExit("the alpha intersector needs the billboard workload's textures")
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    log(f"device {props.name} CUs={props.multi_processor_count} "
        f"gcn={getattr(props, 'gcnArchName', '?')}")
    t0 = time.perf_counter()
    wl = {"billboards": W.billboards, "tiny": W.tiny, "spheres": W.spheres}[args.workload]()
    if args.ray_order != "scanline":
        wl.rays = wl.rays[tile_order(wl, morton=args.ray_order == "morton")]
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    scene = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures, device=dev,
                             layout=args.layout, max_leaf=args.max_leaf)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    tuned = None
    if args.tune_build:
        from paper_1912_12786_amd import autotune
        del scene
        tw = int(wl.extra["width"]) if (args.schedule == "tiles" and args.ray_order == "scanline"
                                        and "width" in wl.extra) else None
        scene, tuned = autotune.tune_scene(
            f"bench-{wl.name}-{kind}-{args.query}", wl.vertices, torch.from_numpy(wl.rays).to(dev),
            kind, query=args.query, k=args.k, geom_ids=wl.geom_ids, texcoords=wl.texcoords,
            textures=wl.textures, cache_path=None, image_width=tw, device=dev)
        args.max_leaf, args.layout = tuned["max_leaf"], tuned["layout"]
        args.shape = ",".join(map(str, tuned["shape"]))
        args.order = "longest-first" if tuned["longest_first"] else "index"
        args.waves_per_simd = tuned["waves_per_simd"]
        log(f"autotuner: leaves <= {args.max_leaf}, {args.layout} nodes, shape {args.shape}, "
            f"{args.order} chunk order, {args.waves_per_simd} waves per SIMD")
        for name, tab in (("first pass, fastest 6", dict(sorted(tuned["ms"].items(),
                                                                 key=lambda kv: kv[1])[:6])),
                          ("finals", tuned["finals_ms"]), ("waves per SIMD", tuned["waves_ms"])):
            log(f"  {name}: " + ", ".join(f"{k} {v:.4f} ms" for k, v in tab.items()))
    log(f"workload {wl.name}: gen {t_gen:.2f} s, host BVH build + upload {t_build:.2f} s, "
        f"{scene.info.n_nodes} inner nodes, depth {scene.info.max_depth}")
    rays = torch.from_numpy(wl.rays).to(dev)
    query = args.query
    if query == "closest":
        hits = torch.empty((wl.n_rays, 4), dtype=torch.float32, device=dev)
    elif query == "any":
        hits = torch.empty((wl.n_rays,), dtype=torch.int32, device=dev)
    else:
        hits = torch.empty((wl.n_rays, args.k, 4), dtype=torch.float32, device=dev)
    ws = rtx.Workspace(dev)
    stream = torch.cuda.current_stream(dev)
    shape_ms = None
    # rays in scanline order over an image: lanes may take them in tiles
    width = int(wl.extra["width"]) if (args.schedule == "tiles" and args.ray_order == "scanline"
                                       and "width" in wl.extra) else None
    if query == "multi" and not args.shape:
        # the k-hit lists favour another launch shape than the closest hit
        # (lanes refilled from the queue lose more coherence over their longer
        # traversals), so the autotuner picks it here, untimed, on the same
        # schedule as the timed launches
        from paper_1912_12786_amd import autotune
        best, shape_ms = autotune.tune(
            f"bench-{wl.name}-{kind}-multi{args.k}",
            lambda sh: rtx.trace(scene, rays, kind, query="multi", k=args.k, alpha_min=128, out=hits,
                                 workspace=ws, shape=sh, image_width=width),
            cache_path=None, steps=10, warmup=2)
        args.shape = ",".join(map(str, best))
        log(f"autotuner: multi-hit launch shape {args.shape}")

    shape = parse_shape(args.shape)
    if args.order is None:
        args.order = default_order(args.workload, kind, query)
    lf = args.order == "longest-first"

    def time_launches(r, o, image_width=width):
        """(per-launch ms from HIP events on the launch stream, wall s) of
        args.steps launches over rays r into o, after args.warmup."""
        def step():
            rtx.trace(scene, r, kind, query=query, k=args.k, alpha_min=128, out=o, workspace=ws,
                      shape=shape, image_width=image_width, longest_first=lf,
                      waves_per_simd=args.waves_per_simd)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            starts[i].record(stream)
            step()
            ends[i].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return np.array([s.elapsed_time(e) for s, e in zip(starts, ends)]), wall

    # timed region: K launches on the current stream, HIP events around each
    per_launch_ms, wall = time_launches(rays, hits)
    ms_per_step = wall * 1e3 / args.steps
    mrays = wl.n_rays * args.steps / wall / 1e6
    split = None
    if args.workload == "spheres":  # primary and bounce rays on their own
        n_p = int(wl.extra["n_primary"])
        split = {}
        for name, sl in (("primary", slice(0, n_p)), ("bounce", slice(n_p, wl.n_rays))):
            ms, _ = time_launches(rays[sl], hits[sl], width if name == "primary" else None)
            split[name] = {"n_rays": sl.stop - sl.start, "kernel_ms_median": round(float(np.median(ms)), 4),
                           "mrays_s": round((sl.stop - sl.start) / float(np.median(ms)) / 1e3, 2)}

    # exact per-ray counts from a separate (untimed) counting launch
    _, cnt = rtx.trace(scene, rays, kind, query=query, k=args.k, alpha_min=128, count=True,
                       workspace=ws, shape=shape)
    torch.cuda.synchronize()
    counters = cnt.cpu().numpy().view(np.uint32)
    node_bytes = {"q8": 32, "f32p": 48, "wide4": 128}.get(args.layout, 64)
    alg_bytes = int(bytes_per_ray(counters, kind, node_bytes,
                                  4 if args.layout == "wide4" else 2).sum())
    # output records: 16-B hit (closest), 4-B occluder (any), k 16-B hits + 4-B count (multi)
    if query == "any":
        alg_bytes -= 12 * wl.n_rays
    elif query == "multi":
        alg_bytes += (16 * (args.k - 1) + 4) * wl.n_rays
    kernel_ms = float(per_launch_ms.mean())

    counters_rec = find_counters(kernel_source_sha(), wl.name, kind, query, args.layout,
                                 args.max_leaf, list(shape or rtx.rt_launch_shapes()[0]),
                                 args.ray_order, "tiles" if width else "index", args.order,
                                 args.waves_per_simd or rtx.RT_DEFAULT_WAVES_PER_SIMD)

    cpu = None
    if not args.no_cpu_baseline and query == "closest":
        threads = len(os.sched_getaffinity(0))
        kind_kw = dict(geom_ids=wl.geom_ids, texcoords=wl.texcoords, textures=wl.textures,
                       alpha_min=128) if kind == "alpha" else {}
        cpu = cpu_baseline(wl, kind, kind_kw, threads, layout=args.layout, max_leaf=args.max_leaf)

    mean_c = counters.mean(axis=0)
    result = {
        "metric": ("Mrays/s closest-hit w/ alpha-mask intersector at 1080p; HBM GB/s % of peak"
                   if args.workload == "billboards" and kind == "alpha" and query == "closest" else
                   f"Mrays/s {query} hit, {kind} intersector, {wl.name}; HBM GB/s % of peak"),
        "value": round(mrays, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": wl.name,
            "n_tris": wl.n_tris,
            "n_rays": wl.n_rays,
            "intersector": kind,
            "alpha_threshold": "0.5 (alpha byte >= 128)" if kind == "alpha" else None,
            "query": query if query != "multi" else f"multi (k={args.k})",
            "textures": "16 x 256x256 RGBA8" if wl.textures is not None else None,
            "ray_order": {"tiled": "8x8 tiles", "morton": "8x8 tiles, Z-order inside"}.get(
                args.ray_order, "scanline"),
            "schedule": ((f"lanes take the rays in 8x8 pixel tiles of the {width}-wide image"
                          if width else "lanes take the rays in index order")
                         + ("; chunks handed out longest path in the scene box first" if lf
                            else "")),
            "bvh": (f"binary SAH, leaves of <= {args.max_leaf} triangles, {scene.info.n_nodes} "
                    f"inner nodes, depth {scene.info.max_depth}"),
            "max_leaf": args.max_leaf,
            "node_layout": {"q8": "32-B nodes, 8-bit child boxes",
                            "f32p": "48-B nodes, float32 child boxes carrying the child "
                                    "references",
                            "wide4": "128-B four-wide nodes, float32 child boxes"}.get(
                                args.layout, "64-B nodes, float32 child boxes"),
            "launch_shape": ([int(x) for x in args.shape.split(",")] if args.shape
                             else list(rtx.rt_launch_shapes()[0])),
            "waves_per_simd": args.waves_per_simd or rtx.RT_DEFAULT_WAVES_PER_SIMD,
        },
        "roofline": roofline(kernel_ms, alg_bytes, counters_rec) | {
            "kernel": f"trace_kernel<{kind}_intersector, {query}>",
            "kernel_ms_mean": round(kernel_ms, 4),
            "kernel_ms_median": round(float(np.median(per_launch_ms)), 4),
            "kernel_ms_p10_p90": [round(float(np.percentile(per_launch_ms, 10)), 4),
                                  round(float(np.percentile(per_launch_ms, 90)), 4)],
            # launches that took over 1.5x the median (position in the timed
            # run, ms): HIP events bracket each launch, so a host-side delay
            # before the launch is enqueued shows here
            "slow_launches": [[int(i), round(float(per_launch_ms[i]), 3)] for i in
                              np.nonzero(per_launch_ms > 1.5 * np.median(per_launch_ms))[0]],
            "algorithmic_bytes_per_launch": alg_bytes,
            "bytes_per_ray_mean": round(alg_bytes / wl.n_rays, 1),
            "mean_counts_per_ray": {"box_tests": round(float(mean_c[0]), 2),
                                    "tri_tests": round(float(mean_c[1]), 2),
                                    "alpha_lookups": round(float(mean_c[2]), 2)},
        },
        "cpu_baseline": cpu,
    }
    if split:
        result["primary_bounce"] = split
    if tuned:
        result["autotuned_build"] = tuned
    if shape_ms:
        result["autotuned_shape_ms"] = shape_ms
    emit(result)


if __name__ == "__main__":
    main()
