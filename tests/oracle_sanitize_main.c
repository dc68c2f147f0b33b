/* Driver for a sanitizer build of the CPU oracle (tests/test_oracle_sanitize.py):
 * every oref_* entry point on a few seeded random graphs, including empty rows and
 * an isolated vertex.  Exits non-zero when a call fails; AddressSanitizer and
 * UndefinedBehaviorSanitizer abort on any fault they see. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oref_enum_count(int32_t, const int64_t *, const int32_t *, int64_t *);
int oref_enum_induced(int32_t, const int64_t *, const int32_t *, int64_t *);
int oref_stage1(int32_t, const int64_t *, const int32_t *, int32_t *);
int oref_stage2(int32_t, const int64_t *, const int32_t *, int64_t *);
int oref_stage3(int32_t, const int64_t *, const int32_t *, const int32_t *, const int64_t *, int64_t *, int64_t *);
int oref_count(int32_t, const int64_t *, const int32_t *, int64_t *);
int oref_orbits_at(int32_t, const int64_t *, const int32_t *, int32_t, const int32_t *, int64_t *, int64_t *,
                   int32_t *);
int oref_stage23_at(int32_t, const int64_t *, const int32_t *, const int32_t *, int32_t, const int32_t *, int64_t *);
int oref_cycles4_total(int32_t, const int64_t *, const int32_t *, int64_t *);
int oref_k4_total(int32_t, const int64_t *, const int32_t *, int64_t *);
int oref_edge_k4(int32_t, const int64_t *, const int32_t *, int64_t, const int64_t *, int64_t *);
int oref_cycles4_at(int32_t, const int64_t *, const int32_t *, int32_t, const int32_t *, int64_t *);

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint64_t next(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
}

int main(void)
{
    for (int trial = 0; trial < 30; trial++) {
        int32_t n = 1 + (int32_t)(next() % 40);
        unsigned char *adj = calloc((size_t)n * n, 1);
        int p = (int)(next() % 100);
        for (int32_t a = 0; a < n; a++)
            for (int32_t b = a + 1; b < n; b++)
                if ((int)(next() % 100) < p && !(a == n - 1 || b == n - 1)) adj[a * n + b] = adj[b * n + a] = 1;
        int64_t *rp = malloc(sizeof(int64_t) * (n + 1));
        rp[0] = 0;
        for (int32_t a = 0; a < n; a++) {
            int64_t d = 0;
            for (int32_t b = 0; b < n; b++) d += adj[a * n + b];
            rp[a + 1] = rp[a] + d;
        }
        int64_t nnz = rp[n];
        int32_t *col = malloc(sizeof(int32_t) * (nnz ? nnz : 1));
        for (int32_t a = 0, k = 0; a < n; a++)
            for (int32_t b = 0; b < n; b++)
                if (adj[a * n + b]) col[k++] = b;
        int64_t *psi = malloc(sizeof(int64_t) * 15 * n), *psi2 = malloc(sizeof(int64_t) * 15 * n);
        int64_t *fv = malloc(sizeof(int64_t) * 9 * n), *k4 = malloc(sizeof(int64_t) * n);
        int64_t *ek = malloc(sizeof(int64_t) * (nnz ? nnz : 1)), *c4v = malloc(sizeof(int64_t) * n);
        int32_t *tri = malloc(sizeof(int32_t) * (nnz ? nnz : 1)), *scr = malloc(sizeof(int32_t) * (nnz ? nnz : 1));
        int32_t *xs = malloc(sizeof(int32_t) * n);
        for (int32_t x = 0; x < n; x++) xs[x] = x;
        int64_t c4 = 0, kk = 0, sl[2] = {0, nnz > 1 ? nnz - 1 : 0};
        int rc = 0;
        rc |= oref_enum_count(n, rp, col, psi);
        rc |= oref_enum_induced(n, rp, col, psi2);
        rc |= oref_stage1(n, rp, col, tri);
        rc |= oref_stage2(n, rp, col, k4);
        rc |= oref_stage3(n, rp, col, tri, k4, psi2, fv);
        rc |= oref_count(n, rp, col, psi);
        rc |= oref_orbits_at(n, rp, col, n, xs, psi2, fv, scr);
        rc |= oref_stage23_at(n, rp, col, tri, n, xs, psi2);
        rc |= oref_cycles4_total(n, rp, col, &c4);
        rc |= oref_k4_total(n, rp, col, &kk);
        rc |= oref_edge_k4(n, rp, col, 0, NULL, ek);
        if (nnz) rc |= oref_edge_k4(n, rp, col, 2, sl, ek);
        rc |= oref_cycles4_at(n, rp, col, n, xs, c4v);
        if (rc) {
            fprintf(stderr, "trial %d: an oracle call failed\n", trial);
            return 1;
        }
        free(adj); free(rp); free(col); free(psi); free(psi2); free(fv); free(k4); free(ek); free(c4v);
        free(tri); free(scr); free(xs);
    }
    printf("sanitized oracle: all calls clean\n");
    return 0;
}
