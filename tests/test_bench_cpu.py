"""Host logic of bench.py (no GPU): the one-GPU contract, the algorithmic
bytes model against hand counts, and the tiled ray order."""
import os
import subprocess
import sys

import numpy as np

import bench
from paper_1912_12786_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bytes_per_ray_hand_counts():
    # boxes, tris, candidates, accepted
    c = np.array([[1, 0, 0, 0],      # missed the root: ray + hit only
                  [7, 4, 1, 1],      # 3 inner nodes, 4 triangles, 1 alpha lookup
                  [73, 12, 2, 1]], np.uint32)
    alpha = bench.bytes_per_ray(c, "alpha")
    plain = bench.bytes_per_ray(c, "default")
    assert alpha.tolist() == [48, 48 + 3 * 64 + 4 * 48 + 28, 48 + 36 * 64 + 12 * 48 + 2 * 28]
    assert plain.tolist() == [48, 48 + 3 * 64 + 4 * 48, 48 + 36 * 64 + 12 * 48]


def test_tile_order_is_a_tiled_permutation():
    wl = W.tiny(24, 16)
    o = bench.tile_order(wl, tile=8)
    assert np.array_equal(np.sort(o), np.arange(wl.n_rays))
    # the first 64 entries are the top-left 8x8 pixel block, row by row
    first = o[:64]
    y, x = np.divmod(first, 24)
    assert y.max() < 8 and x.max() < 8
    assert np.array_equal(first[:8], np.arange(8))
    assert first[8] == 24


def test_bytes_per_ray_compressed_nodes():
    c = np.array([[7, 4, 1, 1]], np.uint32)
    assert bench.bytes_per_ray(c, "alpha", node_bytes=32).tolist() == [48 + 3 * 32 + 4 * 48 + 28]


def test_morton_tile_order():
    wl = W.tiny(24, 16)
    o = bench.tile_order(wl, tile=8, morton=True)
    assert np.array_equal(np.sort(o), np.arange(wl.n_rays))
    first = o[:64]
    y, x = np.divmod(first, 24)
    assert y.max() < 8 and x.max() < 8
    # Z-order: each aligned group of 4 is a 2x2 pixel quad, each group of 16 a 4x4 block
    assert (y[:4].tolist(), x[:4].tolist()) == ([0, 0, 1, 1], [0, 1, 0, 1])
    for g in range(0, 64, 16):
        assert y[g:g + 16].max() - y[g:g + 16].min() == 3 and x[g:g + 16].max() - x[g:g + 16].min() == 3
    assert (y[4], x[4]) == (0, 2)


def test_bytes_per_ray_wide_nodes():
    # root + one full wide node (4 box tests) + one wide node of 3 children:
    # 8 box tests after the root, 2 nodes, 256 B (counted per box test: 8 x 32)
    c = np.array([[9, 2, 1, 1]], np.uint32)
    assert bench.bytes_per_ray(c, "default", node_bytes=128, children=4).tolist() == \
        [48 + 8 * 32 + 2 * 48]


def test_default_builds_and_orders():
    """bench.py's per-workload defaults: the measured choices (packed nodes
    and longest-first order on the billboards for the alpha mask's queries
    and the accept-all closest hit, the latter without the queue; 8-bit
    nodes for the spheres and the batch)."""
    assert bench.default_build("billboards", None, "closest") == ("f32p", None)
    assert bench.default_build("billboards", "alpha", "any") == ("f32p", None)
    assert bench.default_build("billboards", "default", "closest") == ("f32p", "64,8,64,0")
    assert bench.default_build("billboards", "default", "any") == ("f32p", None)
    assert bench.default_build("spheres", None, "closest") == ("q8", None)
    assert bench.default_build("batched", None, "closest") == ("q8", None)
    assert bench.default_build("tiny", None, "closest") == ("f32", None)
    for q in ("closest", "any", "multi"):
        assert bench.default_order("billboards", "alpha", q) == "longest-first"
    assert bench.default_order("billboards", "default", "closest") == "longest-first"
    assert bench.default_order("billboards", "default", "any") == "index"
    assert bench.default_order("spheres", "procedural", "closest") == "index"
    assert bench.default_order("tiny", "default", "closest") == "index"
