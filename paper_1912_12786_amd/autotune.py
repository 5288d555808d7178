"""Autotuner for launch shapes and scene builds.

:func:`tune` times every launch shape compiled into librtx (threads per
block, LDS ring slots, rays per chunk, persistent queue on/off) on a
caller-supplied workload and returns the fastest; the caller passes it to its
trace calls (``shape=``), which select it per call.  Results do not depend on
the shape, only speed does.  :func:`tune_scene`
also chooses how a scene is built: the BVH leaf size limit and the node
layout (binary nodes with float32 or compressed 8-bit child boxes, binary
48-byte nodes with packed references, or four-wide nodes with float32 child
boxes), the chunk order, and the
persistent grid's waves per SIMD, which sets the rays each lane traces.  Those change the per-ray
box and triangle counts, and among hits of exactly equal t possibly which one
is reported, but not the closest or any-hit answer otherwise.  Choices are
cached per device and key in a JSON file.
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
    """Median milliseconds per call of ``run(shape)`` (HIP events around each
    call, so that one delayed launch does not decide) for each launch shape that
    the traced scenes can use (compressed-node scenes run with the default
    shape only, packed-node ones with it and its variant without the queue,
    four-wide ones with the default shape and its 16-slot variant: the library
    refuses the others before launching anything).
    ``run`` receives the shape tuple and passes it to its trace calls."""
    import torch
    shapes = shapes or rtx.rt_launch_shapes()
    times = {}
    stream = torch.cuda.current_stream()
    for sh in shapes:
        sh = tuple(sh)
        try:
            run(sh)
        except rtx.RtxError as e:
            if e.status != rtx.RT_ERR_UNSUPPORTED:
                raise
            continue
        for _ in range(warmup):
            run(sh)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for a, b in ev:
            a.record(stream)
            run(sh)
            b.record(stream)
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in ev)
        times[sh] = 0.5 * (ms[(steps - 1) // 2] + ms[steps // 2])
    return times


def _interleaved(cands, runner, shape_of, steps, warmup, rounds) -> dict:
    """Median over ``rounds`` of each candidate's median milliseconds per call,
    the candidates taken in turn within every round (``runner(c)`` is the
    ``run(shape)`` of candidate ``c``, ``shape_of(c)`` its launch shape)."""
    samples = {c: [] for c in cands}
    for _ in range(rounds):
        for c in cands:
            sh = tuple(shape_of(c))
            samples[c].append(time_shapes(runner(c), steps, warmup, shapes=[sh])[sh])
    out = {}
    for c, v in samples.items():
        v = sorted(v)
        out[c] = 0.5 * (v[(len(v) - 1) // 2] + v[len(v) // 2])
    return out


def tune(key: str, run, cache_path: str | None = DEFAULT_CACHE, steps: int = 10,
         warmup: int = 2, retune: bool = False):
    """Returns ``(shape, times)``: the fastest shape for ``run(shape)`` under
    ``key``, reusing a cached choice for this device unless ``retune``.
    Nothing global changes: the caller passes the shape to its trace calls."""
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
    return best, times


def _load_cache(cache_path):
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                return json.load(f)
        except (OSError, ValueError):
            return {}
    return {}


def _store(cache_path, cache):
    os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, cache_path)


def tune_scene(key: str, vertices, rays, intersector: str = "default", *, query: str = "closest",
               k: int = 1, geom_ids=None,
               texcoords=None, textures=None, alpha_min: int = 128, checker_n: int = 8,
               leaf_sizes=(2, 3, 4), layouts=("f32", "q8", "f32p", "wide4"),
               cache_path: str | None = DEFAULT_CACHE, longest_first=(False, True),
               image_width: int | None = None, waves=(4, 5, 6, 7, 8),
               steps: int = 5, warmup: int = 1, finals: int = 4, final_margin: float = 0.04,
               rounds: int = 3, retune: bool = False, device="cuda"):
    """Chooses the BVH leaf size, node layout, launch shape and chunk order
    (index or longest-path-first) that trace ``rays`` (device float32 [N, 8];
    ``query`` "closest", "any" or "multi" with ``k``; an image of
    ``image_width`` in scanline order when given)
    fastest through the scene, then, for a queue shape, the most resident
    waves per SIMD among ``waves`` for that choice.  The first pass times
    each candidate once, in a fixed order; the (at most ``finals``) fastest
    within ``final_margin`` of the best are then timed again in ``rounds``
    interleaved rounds, and so are the grid sizes, so that a drift of the
    clocks over the sweep does not decide between candidates a few percent
    apart: the median over the rounds decides.  Returns ``(scene, choice)``:
    the scene built that way and ``{"max_leaf", "layout", "shape",
    "longest_first", "waves_per_simd", "ms", "finals_ms", "waves_ms"}``
    (``waves_per_simd`` None for shapes without a queue; ``finals_ms`` empty
    when one candidate stood out); pass ``choice["shape"]``,
    ``choice["longest_first"]`` and ``choice["waves_per_simd"]`` to the trace
    calls.  A cached choice for this device and key is reused unless
    ``retune``."""
    import torch
    dev_name = _device_name(torch)
    cache = _load_cache(cache_path)
    valid = {tuple(s) for s in rtx.rt_launch_shapes()}
    entry = cache.get(dev_name, {}).get(key)
    kw = dict(alpha_min=alpha_min, checker_n=checker_n)

    def build(max_leaf, layout):
        return rtx.upload_scene(vertices, geom_ids, texcoords, textures, device=device,
                                layout=layout, max_leaf=max_leaf)

    if entry and not retune and tuple(entry["shape"]) in valid and "waves_per_simd" in entry:
        choice = entry
    else:
        ws = rtx.Workspace(device)
        # the output of the timed query: [N, 4] hits, [N] occluders (fit in
        # the same), or [N, k, 4] for the k nearest hits
        out = torch.empty((rays.shape[0], 4 * (max(1, k) if query == "multi" else 1)),
                          dtype=torch.float32, device=rays.device)
        timings = {}
        for max_leaf in leaf_sizes:
            for layout in layouts:
                scene = build(max_leaf, layout)
                for lf in longest_first:
                    t = time_shapes(lambda sh: rtx.trace(scene, rays, intersector, query=query,
                                                         k=k, out=out, workspace=ws, shape=sh,
                                                         image_width=image_width,
                                                         longest_first=lf, **kw), steps, warmup)
                    for shape, ms in t.items():
                        timings[(int(max_leaf), layout, shape, bool(lf))] = ms
                del scene
        ranked = sorted(timings, key=timings.get)
        finalists = [k for k in ranked[:max(1, finals)]
                     if timings[k] <= timings[ranked[0]] * (1.0 + final_margin)]
        finals_ms = {}
        if len(finalists) > 1 and rounds > 0:
            scenes = {k[:2]: None for k in finalists}
            for lk in scenes:
                scenes[lk] = build(*lk)
            finals_ms = _interleaved(
                finalists, lambda c: (lambda sh: rtx.trace(scenes[c[:2]], rays, intersector,
                                                            query=query, k=k, out=out,
                                                            workspace=ws, shape=sh,
                                                            image_width=image_width,
                                                            longest_first=c[3], **kw)),
                lambda c: c[2], steps, warmup, rounds)
            del scenes
            best = min(finals_ms, key=finals_ms.get)
        else:
            best = ranked[0]
        label = lambda k: f"{k[0]}/{k[1]}/{','.join(map(str, k[2]))}/{'lf' if k[3] else 'index'}"
        choice = {"max_leaf": best[0], "layout": best[1], "shape": list(best[2]),
                  "longest_first": best[3], "waves_per_simd": None,
                  "ms": {label(k): v for k, v in timings.items()},
                  "finals_ms": {label(k): v for k, v in finals_ms.items()}, "waves_ms": {}}
        if best[2][3] and waves:  # queue shape: size its persistent grid
            scene = build(best[0], best[1])
            wt = _interleaved(
                [int(w) for w in waves],
                lambda w: (lambda sh: rtx.trace(scene, rays, intersector, query=query, k=k,
                                                out=out, workspace=ws, shape=sh,
                                                image_width=image_width,
                                                longest_first=best[3], waves_per_simd=w, **kw)),
                lambda w: best[2], steps, warmup, max(1, rounds))
            del scene
            choice["waves_per_simd"] = min(wt, key=wt.get)
            choice["waves_ms"] = {str(w): v for w, v in wt.items()}
        if cache_path:
            cache.setdefault(dev_name, {})[key] = choice
            _store(cache_path, cache)
    return build(choice["max_leaf"], choice["layout"]), choice
