/*
 * Uniform random graph G(n, m) straight into symmetric sorted CSR: m vertex pairs
 * drawn uniformly (pair i from a counter-based splitmix64 stream, so the result does
 * not depend on the thread count), self-loops dropped, duplicates merged.  Input
 * generation only; it computes nothing of the counting method.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* uniform in [0, n) by the multiply-high method (bias below 2^-32 for n < 2^32) */
static inline int64_t below(uint64_t r, int64_t n) {
    return (int64_t)(((unsigned __int128)r * (uint64_t)n) >> 64);
}

static inline void pair_at(uint64_t seed, int64_t i, int64_t n, int64_t *u, int64_t *v) {
    uint64_t a = mix64(seed ^ mix64(2 * (uint64_t)i));
    uint64_t b = mix64(seed ^ mix64(2 * (uint64_t)i + 1));
    *u = below(a, n);
    *v = below(b, n);
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void sort_small(int32_t *a, int64_t len) {
    if (len > 32) {
        qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
        return;
    }
    for (int64_t i = 1; i < len; i++) {
        int32_t x = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > x) {
            a[j + 1] = a[j];
            j--;
        }
        a[j + 1] = x;
    }
}

/*
 * row_ptr: int64[n+1] (output); col: int32[2m] scratch and output (the first
 * row_ptr[n] entries hold the CSR).  Returns row_ptr[n], or -1 on bad arguments or
 * allocation failure.
 */
int64_t er_gnm_csr(int64_t n, int64_t m, uint64_t seed, int64_t *row_ptr, int32_t *col) {
    if (n <= 0 || m < 0 || n >= ((int64_t)1 << 31)) return -1;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *pos = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!cnt || !pos) {
        free(cnt);
        free(pos);
        return -1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; i++) {
        int64_t u, v;
        pair_at(seed, i, n, &u, &v);
        if (u == v) continue;
#pragma omp atomic
        cnt[u + 1]++;
#pragma omp atomic
        cnt[v + 1]++;
    }
    for (int64_t x = 0; x < n; x++) cnt[x + 1] += cnt[x];
    memcpy(pos, cnt, ((size_t)n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; i++) {
        int64_t u, v, pu, pv;
        pair_at(seed, i, n, &u, &v);
        if (u == v) continue;
#pragma omp atomic capture
        pu = pos[u]++;
#pragma omp atomic capture
        pv = pos[v]++;
        col[pu] = (int32_t)v;
        col[pv] = (int32_t)u;
    }
    /* sort and merge duplicates row by row; kept lengths into pos[x] */
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t x = 0; x < n; x++) {
        int32_t *r = col + cnt[x];
        int64_t len = cnt[x + 1] - cnt[x];
        sort_small(r, len);
        int64_t k = 0;
        for (int64_t j = 0; j < len; j++)
            if (k == 0 || r[j] != r[k - 1]) r[k++] = r[j];
        pos[x] = k;
    }
    /* compact rows in place, front to back (each row moves left or stays) */
    row_ptr[0] = 0;
    for (int64_t x = 0; x < n; x++) {
        int64_t dst = row_ptr[x];
        if (dst != cnt[x]) memmove(col + dst, col + cnt[x], (size_t)pos[x] * sizeof(int32_t));
        row_ptr[x + 1] = dst + pos[x];
    }
    free(cnt);
    free(pos);
    return row_ptr[n];
}
