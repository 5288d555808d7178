/* Runs the oracle's builder, quantizer, packer and traversals on seeded random scenes
 * under AddressSanitizer / UndefinedBehaviorSanitizer (built and run by
 * tests/test_sanitizers.py; exit status 0 iff every call succeeded). */
#include "../../oracle/rt_oracle.c"

static uint32_t lcg(uint32_t *s)
{
    *s = *s * 1664525u + 1013904223u;
    return *s >> 8;
}

static float unit(uint32_t *s) { return (float)lcg(s) / 16777216.0f; }

int main(void)
{
    uint32_t seed = 12345;
    for (int scene = 0; scene < 6; ++scene) {
        const uint32_t n = 1 + lcg(&seed) % 300, m = 1 + lcg(&seed) % 200;
        float *v = malloc(sizeof(float) * 9 * n), *rays = malloc(sizeof(float) * 8 * m);
        uint32_t *geom = malloc(sizeof(uint32_t) * n);
        float *tc = malloc(sizeof(float) * 6 * n);
        uint32_t tex[2 * 4 * 4];
        for (uint32_t k = 0; k < 2 * 4 * 4; ++k) tex[k] = (lcg(&seed) & 0xFFu) << 24;
        for (uint32_t k = 0; k < n; ++k) {
            float c[3] = {unit(&seed), unit(&seed), unit(&seed)};
            for (int j = 0; j < 9; ++j) v[9 * k + j] = c[j % 3] + 0.2f * (unit(&seed) - 0.5f);
            if (k % 7 == 3) for (int j = 0; j < 3; ++j) v[9 * k + 6 + j] = v[9 * k + 3 + j];  /* zero area */
            geom[k] = lcg(&seed) % 2;
            for (int j = 0; j < 6; ++j) tc[6 * k + j] = unit(&seed);
        }
        for (uint32_t i = 0; i < m; ++i) {
            for (int j = 0; j < 3; ++j) rays[8 * i + j] = 2.0f * unit(&seed) - 0.5f;
            for (int j = 4; j < 7; ++j) rays[8 * i + j] = unit(&seed) - 0.5f;
            if (i % 5 == 0) rays[8 * i + 4] = 0.0f;
            rays[8 * i + 3] = 0.0f;
            rays[8 * i + 7] = INFINITY;
        }
        const uint32_t max_leaf = 1 + (uint32_t)scene;
        orc_node *nodes = malloc(sizeof(orc_node) * 2 * n);
        uint32_t *perm = malloc(sizeof(uint32_t) * n), nn = 0, depth = 0;
        if (orc_build_leaf(v, n, max_leaf, nodes, perm, &nn, &depth) != 0) return 1;
        uint32_t *frames = malloc(sizeof(uint32_t) * 3 * nn);
        uint8_t *q = malloc(12 * (size_t)nn);
        float *qbox = malloc(sizeof(float) * 12 * nn);
        if (orc_quantize(nodes, nn, frames, q, qbox) != 0) return 2;
        float *pbox = malloc(sizeof(float) * 12 * nn);
        uint32_t *prefs = malloc(sizeof(uint32_t) * 2 * nn);
        if (orc_pack(nodes, nn, pbox, prefs) != 0) return 6;
        orc_isect is;
        memset(&is, 0, sizeof is);
        is.texcoords = tc;
        is.textures = tex;
        is.n_tex = 2;
        is.width = 4;
        is.height = 4;
        is.alpha_min = 128;
        is.checker_n = 8;
        float *t = malloc(sizeof(float) * 3 * m), *u = malloc(sizeof(float) * 3 * m),
              *w = malloc(sizeof(float) * 3 * m);
        uint32_t *prim = malloc(sizeof(uint32_t) * 3 * m), *nh = malloc(sizeof(uint32_t) * m),
                 *cnt = malloc(sizeof(uint32_t) * 4 * m);
        for (int kind = ORC_DEFAULT; kind <= ORC_PROCEDURAL; ++kind)
            for (int layout = 0; layout < 3; ++layout) {
                const float *qb = layout == 2 ? pbox : (layout ? qbox : NULL);
                if (orc_traverse_layout(v, geom, n, nodes, perm, nn, qb, rays, m, kind, &is, 0, 0, t,
                                        prim, u, w, NULL, cnt, 2) != 0) return 3;
                if (orc_traverse_layout(v, geom, n, nodes, perm, nn, qb, rays, m, kind, &is, 1, 0, t,
                                        prim, u, w, NULL, cnt, 2) != 0) return 4;
                if (orc_traverse_layout(v, geom, n, nodes, perm, nn, qb, rays, m, kind, &is, 0, 3, t,
                                        prim, u, w, nh, cnt, 2) != 0) return 5;
            }
        free(v); free(rays); free(geom); free(tc); free(nodes); free(perm); free(frames); free(q);
        free(qbox); free(pbox); free(prefs); free(t); free(u); free(w); free(prim); free(nh); free(cnt);
    }
    puts("oracle ok");
    return 0;
}
