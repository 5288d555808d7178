"""Host side of Python-defined intersectors (paper_1912_12786_amd.custom):
source generation and validation, and the parameter blocks of the libraries
__graft_entry__.build() compiled."""
import ctypes as C

import pytest

from paper_1912_12786_amd import custom
from tests.custom import python_defined as PD


def test_generate_source_validation():
    src = custom.generate_source("demo", [("n", "f32"), ("mask", "ptr:uint8_t")], "        return true;")
    assert "struct demo_intersector" in src and "const uint8_t * mask;" in src
    assert "demo_trace" in src and "demo_workspace_bytes" in src and "demo_last_error" in src
    with pytest.raises(ValueError):
        custom.generate_source("bad name", [], "return true;")
    with pytest.raises(ValueError):
        custom.generate_source("demo", [("x", "f64")], "return true;")
    with pytest.raises(ValueError):
        custom.generate_source("demo", [("x", "ptr:int; evil")], "return true;")
    with pytest.raises(ValueError):
        custom.generate_source("demo", [("1x", "u32")], "return true;")


@pytest.mark.parametrize("name", list(PD.SPECS))
def test_built_libraries_and_parameter_blocks(name):
    isect = PD.load(name)
    fields, _ = PD.SPECS[name]
    assert [f for f, _ in isect.params_type._fields_] == [f for f, _ in fields]
    if name == "user_alpha":
        # {const float2 *, const uint32_t *, uint32_t x 3}: 8-byte aligned, 32 bytes
        assert C.sizeof(isect.params_type) == 32
        p = isect.params(texcoords=0x1000, textures=0x2000, width=4, height=2, alpha_min=128)
        assert (p.texcoords, p.textures, p.width, p.height, p.alpha_min) == (0x1000, 0x2000, 4, 2, 128)
    with pytest.raises(ValueError, match="missing parameter"):
        isect.params()
