"""Intersectors that the test suite defines from Python (paper_1912_12786_amd.
custom): a checker and an alpha mask written as user code, which must match
the built-in ones bit for bit, and a wireframe mask none of the built-ins
offers.  __graft_entry__.build() compiles them into this folder."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))

SPECS = {
    "user_checker": (
        [("n", "f32")],
        """        const int a = int(floorf(p.n * c.u));
        const int b = int(floorf(p.n * c.v));
        return ((a + b) & 1) == 0;""",
    ),
    "user_alpha": (
        [("texcoords", "ptr:float2"), ("textures", "ptr:uint32_t"), ("width", "u32"),
         ("height", "u32"), ("alpha_min", "u32")],
        """        const float2 *tc = p.texcoords + 3 * size_t(c.prim_id);
        const float w0 = (1.0f - c.u) - c.v;
        const float s = fmaf(c.v, tc[2].x, fmaf(c.u, tc[1].x, w0 * tc[0].x));
        const float t = fmaf(c.v, tc[2].y, fmaf(c.u, tc[1].y, w0 * tc[0].y));
        const float xf = fminf(fmaxf(floorf(s * float(p.width)), 0.0f), float(p.width - 1));
        const float yf = fminf(fmaxf(floorf(t * float(p.height)), 0.0f), float(p.height - 1));
        const size_t i = (size_t(c.geom_id) * p.height + uint32_t(yf)) * p.width + uint32_t(xf);
        return (p.textures[i] >> 24) >= p.alpha_min;""",
    ),
    "wireframe": (
        [("width", "f32")],
        """        return fminf(fminf(c.u, c.v), (1.0f - c.u) - c.v) < p.width;""",
    ),
}


def lib_path(name: str) -> str:
    return os.path.join(HERE, f"lib{name}.so")


def build_all() -> None:
    from paper_1912_12786_amd import custom
    for name, (fields, accept) in SPECS.items():
        custom.build_intersector(name, fields, accept, HERE)


def load(name: str):
    from paper_1912_12786_amd import custom
    fields, _ = SPECS[name]
    return custom.CustomIntersector(lib_path(name), name, fields)
