"""Host-side checks of the Python binding that need no GPU: arguments that
would hand the GPU a host pointer are refused before anything is launched."""
import pytest


def test_hit_backward_refuses_host_tensors():
    import torch
    from paper_1912_12786_amd import diff
    rays = torch.zeros((4, 8))
    hits = torch.zeros((4, 4))
    g = torch.zeros((4, 3))
    V = torch.zeros((3, 3))
    F = torch.zeros((1, 3), dtype=torch.int32)
    with pytest.raises(ValueError, match="CUDA"):
        diff.hit_backward(rays, hits, g, V, F)
    with pytest.raises(ValueError, match="CUDA"):
        diff.DifferentiableHit.apply(rays, V, F, None, None, None)


def test_shape_flags():
    from paper_1912_12786_amd import rtx
    assert rtx.shape_flag(None) == 0
    assert rtx.RT_FLAG_SHAPE(3) == 3 << 8
    assert rtx.shape_flag(2) == rtx.RT_FLAG_SHAPE(2)
