"""Launch-shape autotuner.

Times every launch shape compiled into librtx (threads per block, LDS ring
slots, rays per chunk, persistent queue on/off) on a caller-supplied workload
and selects the fastest with rt_set_launch_shape.  Results do not depend on
the shape, only speed does.  Choices are cached per device and workload key
in a JSON file.
"""
from __future__ import annotations

import json
import os

from . import rtx

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rtx_autotune.json")


def _device_name(torch) -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}/{getattr(p, 'gcnArchName', '')}/{p.multi_processor_count}"


def time_shapes(run, steps: int = 10, warmup: int = 2, shapes=None) -> dict:
    """Mean milliseconds per call of ``run()`` for each launch shape that the
    traced scenes can use (compressed-node scenes run with the default shape
    only: the library refuses the others before launching anything)."""
    import torch
    shapes = shapes or rtx.rt_launch_shapes()
    saved = rtx.rt_launch_shapes()[0]
    times = {}
    stream = torch.cuda.current_stream()
    try:
        for sh in shapes:
            rtx.rt_set_launch_shape(*sh)
            try:
                run()
            except rtx.RtxError as e:
                if e.status != rtx.RT_ERR_UNSUPPORTED:
                    raise
                continue
            for _ in range(warmup):
                run()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(steps):
                run()
            b.record(stream)
            torch.cuda.synchronize()
            times[tuple(sh)] = a.elapsed_time(b) / steps
    finally:
        rtx.rt_set_launch_shape(*saved)
    return times


def tune(key: str, run, cache_path: str | None = DEFAULT_CACHE, steps: int = 10,
         warmup: int = 2, retune: bool = False):
    """Selects (and returns) the fastest shape for ``run`` under ``key``,
    reusing a cached choice for this device unless ``retune``."""
    import torch
    dev = _device_name(torch)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    entry = cache.get(dev, {}).get(key)
    valid = {tuple(s) for s in rtx.rt_launch_shapes()}
    if entry and not retune and tuple(entry["shape"]) in valid:
        best, times = tuple(entry["shape"]), entry.get("ms", {})
    else:
        t = time_shapes(run, steps, warmup)
        best = min(t, key=t.get)
        times = {",".join(map(str, k)): v for k, v in t.items()}
        if cache_path:
            cache.setdefault(dev, {})[key] = {"shape": list(best), "ms": times}
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(tmp, cache_path)
    rtx.rt_set_launch_shape(*best)
    return best, times
