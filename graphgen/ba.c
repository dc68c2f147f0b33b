/* Preferential-attachment edge lists for many small graphs (input generation only).
 *
 * Graph g has ns[g] vertices and parameter k = ks[g]: it starts as a star from
 * vertex 0 to vertices 1..k; each later vertex t joins k distinct earlier vertices,
 * each drawn as an endpoint of a uniformly drawn existing edge (that is, with
 * probability proportional to degree), redrawing repeats up to a fixed number of
 * tries.  Random numbers: splitmix64 (Steele, Lea and Flood, 2014), one stream per
 * graph seeded from (seed, g).  Edges of graph g go to src/dst[eoff[g] .. eoff[g+1]),
 * where eoff is computed here from the actual counts; the caller sizes src/dst by
 * sum(ns[g] * ks[g]). */
#include <stdint.h>

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int ba_edges(int64_t G, const int64_t *ns, const int64_t *ks, uint64_t seed, int64_t *src, int64_t *dst,
             int64_t *eoff) {
    int64_t at = 0;
    for (int64_t g = 0; g < G; g++) {
        const int64_t n = ns[g], k = ks[g];
        eoff[g] = at;
        uint64_t st = seed ^ ((uint64_t)(g + 1) * 0xD1B54A32D192ED03ull);
        int64_t *s = src + at, *d = dst + at;
        int64_t ne = 0;
        if (n <= k) {  /* complete graph */
            for (int64_t a = 0; a < n; a++)
                for (int64_t b = a + 1; b < n; b++) { s[ne] = a; d[ne] = b; ne++; }
            at += ne;
            continue;
        }
        for (int64_t t = 1; t <= k; t++) { s[ne] = 0; d[ne] = t; ne++; }
        for (int64_t t = k + 1; t < n; t++) {
            int64_t chosen[16];
            int nc = 0;
            for (int tries = 0; nc < k && tries < 8 * k; tries++) {
                uint64_t r = splitmix64(&st) % (uint64_t)(2 * ne);
                int64_t e = (int64_t)(r >> 1);
                int64_t v = (r & 1) ? d[e] : s[e];
                int dup = 0;
                for (int i = 0; i < nc; i++) if (chosen[i] == v) { dup = 1; break; }
                if (!dup) chosen[nc++] = v;
            }
            for (int i = 0; i < nc; i++) { s[ne] = t; d[ne] = chosen[i]; ne++; }
        }
        at += ne;
    }
    eoff[G] = at;
    return 0;
}
