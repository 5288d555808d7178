// Runs the library's host BVH builder, node compressor and node packer on seeded random
// scenes under AddressSanitizer / UndefinedBehaviorSanitizer (built and run by
// tests/test_sanitizers.py; exit status 0 iff every build succeeded and its
// basic invariants hold).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_1912_12786_amd/csrc/bvh_build.cpp"

static uint32_t lcg(uint32_t &s)
{
    s = s * 1664525u + 1013904223u;
    return s >> 8;
}

int main()
{
    uint32_t seed = 777;
    for (int scene = 0; scene < 8; ++scene) {
        const uint32_t n = scene == 0 ? 0 : 1 + lcg(seed) % 2000;
        const uint32_t max_leaf = 1 + uint32_t(scene) % 7;
        std::vector<float> v(9 * size_t(n));
        std::vector<uint32_t> geom(n);
        for (uint32_t k = 0; k < n; ++k) {
            const float c[3] = {float(lcg(seed) % 1000), float(lcg(seed) % 1000), float(lcg(seed) % 1000)};
            for (int j = 0; j < 9; ++j) v[9 * k + j] = c[j % 3] + float(lcg(seed) % 100) * 0.01f;
            if (k % 9 == 4)  // all centroids equal within a cluster: the median split
                for (int j = 0; j < 9; ++j) v[9 * k + j] = 5.0f;
            geom[k] = lcg(seed) % 16;
        }
        const uint32_t cap = rtx::max_inner_nodes(n, 1);
        std::vector<rtx::NodeRecord> nodes(cap ? cap : 1);
        std::vector<rtx::TriRecord> tris(n ? n : 1);
        rt_bvh_info info{};
        if (rtx::build_bvh(n ? v.data() : nullptr, geom.data(), n, max_leaf, nodes.data(), tris.data(),
                           &info) != RT_OK)
            return 1;
        if (info.n_nodes > cap || info.max_leaf != max_leaf) return 2;
        std::vector<uint32_t> seen(n, 0);
        for (uint32_t i = 0; i < n; ++i) {
            const uint32_t p = tris[i].u[3];
            if (p >= n || seen[p]++) return 3;  // every triangle exactly once
        }
        std::vector<rtx::NodeQ8Record> q(info.n_nodes ? info.n_nodes : 1);
        if (info.n_nodes && rtx::compress_nodes(nodes.data(), info.n_nodes, q.data()) != RT_OK) return 4;
        std::vector<rtx::NodePackedRecord> pk(info.n_nodes ? info.n_nodes : 1);
        if (info.n_nodes && rtx::pack_nodes(nodes.data(), info.n_nodes, pk.data()) != RT_OK) return 5;
        for (uint32_t i = 0; i < info.n_nodes; ++i)  // the references gather back
            for (int c = 0; c < 2; ++c) {
                const uint32_t *w = pk[i].u + 6 * c;
                const uint32_t ref = (w[0] & 0xFFu) | (w[1] & 0xFFu) << 8 | (w[2] & 0xFFu) << 16 |
                                     (w[3] & 0xFFu) << 24;
                if (ref != nodes[i].u[12 + c]) return 6;
            }
    }
    std::puts("builder ok");
    return 0;
}
