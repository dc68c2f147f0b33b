/*
 * Test infrastructure: the CPU oracle for per-vertex non-induced orbit counts.
 *
 * Only the test suite, the smoke check and the bench's CPU-baseline leg may load
 * this file's library.  It is not part of the product path, includes no header
 * of the HIP library and shares no code with it.
 *
 * Two independent formulations live here:
 *
 *  1. oref_enum_*  -- the definition (Section 3, Definitions 3-5): every
 *     connected vertex set S, |S| = 2..4, is enumerated once (each set is grown
 *     from its smallest vertex through vertices larger than it), and every edge
 *     subset of E[S] that connects S is one non-induced occurrence, classified by
 *     (edge count, degree sequence) into the 15 orbits.  Exact and plain, usable on
 *     sparse graphs of a few thousand vertices and on small dense graphs.
 *
 *  2. oref_stage1/2/3, oref_count, oref_orbits_at -- the paper's three-stage
 *     method: Stage I per-edge triangle counts (Algorithm 1), Stage II the
 *     4-cliques through each vertex (what Algorithm 2 computes, counted here from
 *     the definition), Stage III f-variable probing over the four substructures of
 *     Table 1 followed by the non-induced equations of Section 5 and the Appendix.
 *
 *  3. oref_enum_induced -- the induced orbit counts (Definition 2), by the same
 *     enumeration as 1; oref_cycles4_total, oref_k4_total, oref_edge_k4 --
 *     whole-graph counts of 4-cycles and 4-cliques and the 4-cliques through each
 *     edge, exact checks on outputs too large for the per-vertex oracle.
 *
 * Readings taken where the text is silent, ambiguous or garbled (each one is
 * checked against formulation 1 and Python brute force by the tests):
 *   - Stage II: Algorithm 2 is not run as printed (its neigh buffer would have
 *     to be emptied for every (x, y) pair, with strict id tests, to find each
 *     4-clique once); its result, the 4-cliques through each vertex, is counted
 *     from the definition instead.
 *   - psi_1, psi_2, psi_3 are the non-induced 3-vertex counts found while probing:
 *     psi_1 sums d(y)-1 over neighbours y, psi_2 counts neighbour pairs, psi_3
 *     counts triangles at x.
 *   - Per occurrence terms of the f-variables (Table 1; the figure of the four
 *     substructures is missing):
 *       Triangle 1 (triangle {x,y,z} seen once, y > z):
 *           f12_14 += t(yz) - 1;  f10_13 += (d(y)-1-t(yz)) + (d(z)-1-t(yz))
 *       Triangle 2 (each triangle at x once):
 *           f13_14 += (t(xy)-1) + (t(xz)-1)
 *           f11_13 += (d(x)-1-t(xy)) + (d(x)-1-t(xz))
 *       Two-Star (unordered {y,z} in N(x), y and z not adjacent):
 *           f5_8 += (d(y)-1-t(xy)) + (d(z)-1-t(xz))
 *       Path (y in N(x), z in N(y), z != x, z not in N(x)):
 *           f6_9 += d(y)-2-t(xy)      (the triangles excluded are those on e_xy;
 *                                      reading them on e_yz breaks psi_6)
 *           f9_12 += t(yz);  f4_8 += d(z)-1-t(yz);  f8_12 += common[z]-1
 *     where common[z] = |N(x) and N(z)| for z outside N(x) and z != x, counted
 *     over every y (no ordering).
 *   - Every halving in the equations is exact: the numerator is checked to be
 *     even and the call fails with ORACLE_EODD otherwise.
 *
 * Numbers are int64 throughout.  Graphs are simple, symmetric CSR with each row
 * sorted ascending (row_ptr int64[n+1], col int32[row_ptr[n]]).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef int64_t i64;
typedef int32_t i32;

enum { ORACLE_OK = 0, ORACLE_EINVAL = -1, ORACLE_ENOMEM = -2, ORACLE_EODD = -3 };

/* f-variable order used by every function here (Table 1 order). */
enum { F12_14 = 0, F10_13, F13_14, F11_13, F5_8, F6_9, F9_12, F4_8, F8_12, NFV };

int oref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oref_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Slot of b in the sorted row of a, or -1. */
static i64 slot_of(const i64 *rp, const i32 *col, i32 a, i32 b)
{
    i64 lo = rp[a], hi = rp[a + 1];
    while (lo < hi) {
        i64 mid = lo + (hi - lo) / 2;
        if (col[mid] < b) lo = mid + 1; else hi = mid;
    }
    return (lo < rp[a + 1] && col[lo] == b) ? lo : -1;
}

static i64 deg_of(const i64 *rp, i32 v) { return rp[v + 1] - rp[v]; }

/* ------------------------------------------------------------------------- */
/* Formulation 1: the definition, by enumerating connected vertex sets.       */
/* ------------------------------------------------------------------------- */

/* Orbit of each vertex of a connected occurrence on k vertices with edge mask
 * over the pairs of S (pair p = (pi[p], pj[p])).  Returns 0 on success. */
static const int PI4[6] = {0, 0, 0, 1, 1, 2};
static const int PJ4[6] = {1, 2, 3, 2, 3, 3};

static int occurrence_orbits(int k, int npairs, const int *pi, const int *pj,
                             unsigned mask, int orb[4])
{
    int deg[4] = {0, 0, 0, 0};
    int ne = 0;
    for (int p = 0; p < npairs; p++)
        if (mask >> p & 1u) { deg[pi[p]]++; deg[pj[p]]++; ne++; }
    for (int v = 0; v < k; v++) if (deg[v] == 0) return -1;
    /* connectivity by repeated relaxation */
    int seen = 1, grew = 1;
    while (grew) {
        grew = 0;
        for (int p = 0; p < npairs; p++) {
            if (!(mask >> p & 1u)) continue;
            int a = pi[p], b = pj[p];
            if ((seen >> a & 1) != (seen >> b & 1)) { seen |= (1 << a) | (1 << b); grew = 1; }
        }
    }
    if (seen != (1 << k) - 1) return -1;
    if (k == 2) { orb[0] = orb[1] = 0; return 0; }
    if (k == 3) {
        for (int v = 0; v < 3; v++) orb[v] = (ne == 3) ? 3 : (deg[v] == 1 ? 1 : 2);
        return 0;
    }
    int maxd = 0;
    for (int v = 0; v < 4; v++) if (deg[v] > maxd) maxd = deg[v];
    for (int v = 0; v < 4; v++) {
        int d = deg[v];
        switch (ne) {
        case 3:
            if (maxd == 3) orb[v] = (d == 3) ? 7 : 6;          /* 3-star */
            else orb[v] = (d == 1) ? 4 : 5;                    /* 4-path */
            break;
        case 4:
            if (maxd == 2) orb[v] = 8;                         /* 4-cycle */
            else orb[v] = (d == 1) ? 9 : (d == 2 ? 10 : 11);   /* tailed triangle */
            break;
        case 5: orb[v] = (d == 2) ? 12 : 13; break;           /* diamond */
        case 6: orb[v] = 14; break;                            /* 4-clique */
        default: return -1;
        }
    }
    return 0;
}

/* Credits the occurrences on the connected vertex set S.  Non-induced (induced =
 * 0): every subset of the edges of G inside S that connects S.  Induced (induced =
 * 1): only the full edge set of G inside S, the subgraph G[S] (Definition 2). */
static void credit_set(const i64 *rp, const i32 *col, int k, const i32 *S, i64 *psi, int induced)
{
    static const int PI3[3] = {0, 0, 1}, PJ3[3] = {1, 2, 2};
    const int *pi = (k == 4) ? PI4 : PI3, *pj = (k == 4) ? PJ4 : PJ3;
    int npairs = k * (k - 1) / 2;
    unsigned present = 0;
    for (int p = 0; p < npairs; p++)
        if (slot_of(rp, col, S[pi[p]], S[pj[p]]) >= 0) present |= 1u << p;
    if (induced) {
        int orb[4];
        if (occurrence_orbits(k, npairs, pi, pj, present, orb) == 0)
            for (int v = 0; v < k; v++) {
#pragma omp atomic
                psi[(i64)S[v] * 15 + orb[v]] += 1;
            }
        return;
    }
    /* every subset of the present pairs */
    for (unsigned sub = present;; sub = (sub - 1) & present) {
        int orb[4];
        if (sub && occurrence_orbits(k, npairs, pi, pj, sub, orb) == 0)
            for (int v = 0; v < k; v++) {
#pragma omp atomic
                psi[(i64)S[v] * 15 + orb[v]] += 1;
            }
        if (sub == 0) break;
    }
}

/* Grow connected sets from their smallest vertex: every vertex added is larger
 * than S[0] and adjacent to the set; a set is reported once because extension
 * candidates are only neighbours of the newest vertex that are not adjacent to
 * any earlier member (the exclusive-neighbourhood rule), as in ESU. */
static int in_set(const i32 *S, int k, i32 v) { for (int i = 0; i < k; i++) if (S[i] == v) return 1; return 0; }

static int adjacent_to_set(const i64 *rp, const i32 *col, const i32 *S, int k, i32 v)
{
    for (int i = 0; i < k; i++) if (slot_of(rp, col, S[i], v) >= 0) return 1;
    return 0;
}

static void extend(const i64 *rp, const i32 *col, i32 *S, int k, i32 *ext, int next, i64 *psi,
                   i32 *buf, i64 bufcap, int induced)
{
    credit_set(rp, col, k, S, psi, induced);
    if (k == 4) return;
    /* ext[0..next) is the current extension set */
    for (int i = 0; i < next; i++) {
        i32 w = ext[i];
        /* new extension: remaining ext after w, plus exclusive neighbours of w */
        int nn = 0;
        i32 *ne = buf;
        for (int j = i + 1; j < next; j++) ne[nn++] = ext[j];
        for (i64 s = rp[w]; s < rp[w + 1]; s++) {
            i32 u = col[s];
            if (u <= S[0] || in_set(S, k, u) || u == w) continue;
            if (adjacent_to_set(rp, col, S, k, u)) continue;
            int dup = 0;
            for (int j = 0; j < nn; j++) if (ne[j] == u) { dup = 1; break; }
            if (!dup) {
                if (nn >= bufcap) return; /* cannot happen: cap sized by caller */
                ne[nn++] = u;
            }
        }
        S[k] = w;
        extend(rp, col, S, k + 1, ne, nn, psi, buf + nn, bufcap - nn, induced);
    }
}

/* Orbit counts by enumerating each connected vertex set once; psi int64[n*15]
 * (zeroed here); induced selects Definition 2 (G[S] only) over Definition 3. */
static int enum_orbits(i32 n, const i64 *rp, const i32 *col, i64 *psi, int induced)
{
    if (n < 0 || (n > 0 && (!rp || !col)) || !psi) return ORACLE_EINVAL;
    memset(psi, 0, sizeof(i64) * 15 * (size_t)n);
    i64 dmax = 0;
    for (i32 v = 0; v < n; v++) if (deg_of(rp, v) > dmax) dmax = deg_of(rp, v);
    i64 cap = 4 * (3 * dmax + 4);
    int err = 0;
#pragma omp parallel
    {
        i32 *buf = (i32 *)malloc(sizeof(i32) * (size_t)cap);
        if (!buf) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (i32 v = 0; v < n; v++) {
                i32 S[4];
                S[0] = v;
                int nn = 0;
                for (i64 s = rp[v]; s < rp[v + 1]; s++) if (col[s] > v) buf[nn++] = col[s];
                extend(rp, col, S, 1, buf, nn, psi, buf + nn, cap - nn, induced);
            }
            free(buf);
        }
    }
    return err ? ORACLE_ENOMEM : ORACLE_OK;
}

/* Non-induced orbit counts psi_k (Section 3, Definitions 3-5), int64[n*15]. */
int oref_enum_count(i32 n, const i64 *rp, const i32 *col, i64 *psi)
{
    return enum_orbits(n, rp, col, psi, 0);
}

/* Induced orbit counts psi'_k (Section 3, Definition 2: each connected vertex set S
 * contributes the one graphlet G[S]), int64[n*15], same orbit numbering. */
int oref_enum_induced(i32 n, const i64 *rp, const i32 *col, i64 *psi)
{
    return enum_orbits(n, rp, col, psi, 1);
}

/* ------------------------------------------------------------------------- */
/* Formulation 2: the paper's three stages.                                    */
/* ------------------------------------------------------------------------- */

/* Stage I (Algorithm 1): the i-th edge (x, y), x < y, taken in CSR order, gets
 * tri = |N(x) and N(y)| by a sorted merge.  The value is stored in both CSR slots
 * of the edge (tri int32[row_ptr[n]]) so later stages can read it from either end.
 * The loop runs over the edges themselves (in parallel chunks of slots), so a
 * vertex with a long row does not leave one thread all of its merges. */
int oref_stage1(i32 n, const i64 *rp, const i32 *col, i32 *tri)
{
    if (n < 0 || (n > 0 && (!rp || !col)) || (n > 0 && rp[n] > 0 && !tri)) return ORACLE_EINVAL;
    if (n == 0) return ORACLE_OK;
    const i64 nnz = rp[n];
    i32 *src = (i32 *)malloc(sizeof(i32) * (size_t)(nnz ? nnz : 1));
    if (!src) return ORACLE_ENOMEM;
#pragma omp parallel for schedule(dynamic, 256)
    for (i32 x = 0; x < n; x++)
        for (i64 s = rp[x]; s < rp[x + 1]; s++) src[s] = x;
#pragma omp parallel for schedule(dynamic, 64)
    for (i64 s = 0; s < nnz; s++) {
        i32 x = src[s], y = col[s];
        if (y < x) continue;
        i64 i = rp[x], j = rp[y];
        i32 c = 0;
        while (i < rp[x + 1] && j < rp[y + 1]) {
            if (col[i] < col[j]) i++;
            else if (col[i] > col[j]) j++;
            else { c++; i++; j++; }
        }
        tri[s] = c;
        tri[slot_of(rp, col, y, x)] = c;
    }
    free(src);
    return ORACLE_OK;
}

/* Stage II: K4[x] = the number of 4-cliques containing x (psi_14 of Section 5;
 * Algorithm 2 computes these counts).  A 4-clique through x is x together with a
 * triangle {a, b, c} of G inside N(x), so for every x the neighbours are marked
 * and each such triangle a < b < c is found once: from its edge (a, b), b > a, and
 * every c > b adjacent to a, to b and to x. */
int oref_stage2(i32 n, const i64 *rp, const i32 *col, i64 *K4)
{
    if (n < 0 || (n > 0 && (!rp || !col || !K4))) return ORACLE_EINVAL;
    if (n == 0) return ORACLE_OK;
    int err = 0;
#pragma omp parallel
    {
        unsigned char *inx = (unsigned char *)calloc((size_t)n, 1);
        unsigned char *ina = (unsigned char *)calloc((size_t)n, 1);
        if (!inx || !ina) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (i32 x = 0; x < n; x++) {
                i64 cliques = 0;
                for (i64 s = rp[x]; s < rp[x + 1]; s++) inx[col[s]] = 1;
                for (i64 s = rp[x]; s < rp[x + 1]; s++) {
                    i32 a = col[s];
                    for (i64 r = rp[a]; r < rp[a + 1]; r++) ina[col[r]] = 1;
                    for (i64 r = rp[a]; r < rp[a + 1]; r++) {
                        i32 b = col[r];
                        if (b <= a || !inx[b]) continue;
                        for (i64 q = rp[b]; q < rp[b + 1]; q++) {
                            i32 c = col[q];
                            if (c > b && inx[c] && ina[c]) cliques++;
                        }
                    }
                    for (i64 r = rp[a]; r < rp[a + 1]; r++) ina[col[r]] = 0;
                }
                for (i64 s = rp[x]; s < rp[x + 1]; s++) inx[col[s]] = 0;
                K4[x] = cliques;
            }
        }
        free(inx);
        free(ina);
    }
    return err ? ORACLE_ENOMEM : ORACLE_OK;
}

/* Per-thread scratch for Stage III. */
typedef struct {
    i32 *tx;        /* tx[z] = t(x, z) for z in N(x), -1 elsewhere */
    unsigned char *iny; /* neighbour marks of the current y (two-star test) */
    i64 *common;    /* common[z] for z outside N(x) */
    i32 *touched;   /* vertices with common[z] != 0 */
} scratch_t;

static int scratch_init(scratch_t *sc, i32 n, i64 dmax)
{
    sc->tx = (i32 *)malloc(sizeof(i32) * (size_t)(n ? n : 1));
    sc->iny = (unsigned char *)calloc((size_t)(n ? n : 1), 1);
    sc->common = (i64 *)calloc((size_t)(n ? n : 1), sizeof(i64));
    sc->touched = (i32 *)malloc(sizeof(i32) * (size_t)(n ? n : 1));
    (void)dmax;
    if (!sc->tx || !sc->iny || !sc->common || !sc->touched) return -1;
    for (i32 v = 0; v < n; v++) sc->tx[v] = -1;
    return 0;
}

static void scratch_free(scratch_t *sc)
{
    free(sc->tx); free(sc->iny); free(sc->common); free(sc->touched);
}

static i64 choose2(i64 a) { return a * (a - 1) / 2; }
static i64 choose3(i64 a) { return a * (a - 1) * (a - 2) / 6; }

/* Stage III for one vertex x: probe the four substructures (Table 1), then solve
 * the equations (Section 5, Appendix).  tri is indexed by CSR slot and must be
 * valid in row x and in every row y with y in N(x).  Writes psi[15] and f[9]. */
static int stage3_vertex(const i64 *rp, const i32 *col, const i32 *tri, i64 k4x,
                         i32 x, scratch_t *sc, i64 *psi, i64 *f)
{
    i64 dx = deg_of(rp, x);
    i64 fv[NFV];
    memset(fv, 0, sizeof fv);
    i64 psi1 = 0, pairs = 0, triangles = 0;

    for (i64 s = rp[x]; s < rp[x + 1]; s++) sc->tx[col[s]] = tri[s];

    /* 3-vertex counts and the two triangle substructures. */
    for (i64 s = rp[x]; s < rp[x + 1]; s++) {
        i32 y = col[s];
        i64 dy = deg_of(rp, y), txy = tri[s];
        psi1 += dy - 1;
        for (i64 r = rp[y]; r < rp[y + 1]; r++) {
            i32 z = col[r];
            if (z >= y || sc->tx[z] < 0) continue;   /* triangle {x,y,z}, y > z */
            i64 dz = deg_of(rp, z), tyz = tri[r], txz = sc->tx[z];
            triangles++;
            /* Triangle 1 */
            fv[F12_14] += tyz - 1;
            fv[F10_13] += (dy - 1 - tyz) + (dz - 1 - tyz);
            /* Triangle 2 */
            fv[F13_14] += (txy - 1) + (txz - 1);
            fv[F11_13] += (dx - 1 - txy) + (dx - 1 - txz);
        }
    }

    /* Two-Star: unordered pairs of neighbours of x. */
    for (i64 s = rp[x]; s < rp[x + 1]; s++) {
        i32 y = col[s];
        i64 dy = deg_of(rp, y), txy = tri[s];
        for (i64 r = rp[y]; r < rp[y + 1]; r++) sc->iny[col[r]] = 1;
        for (i64 q = s + 1; q < rp[x + 1]; q++) {
            i32 z = col[q];
            pairs++;
            if (sc->iny[z]) continue;
            i64 dz = deg_of(rp, z), txz = tri[q];
            fv[F5_8] += (dy - 1 - txy) + (dz - 1 - txz);
        }
        for (i64 r = rp[y]; r < rp[y + 1]; r++) sc->iny[col[r]] = 0;
    }

    /* Path x - y - z with z outside N(x): first fill common[], then the sums. */
    i64 ntouched = 0;
    for (i64 s = rp[x]; s < rp[x + 1]; s++) {
        i32 y = col[s];
        for (i64 r = rp[y]; r < rp[y + 1]; r++) {
            i32 z = col[r];
            if (z == x || sc->tx[z] >= 0) continue;
            if (sc->common[z]++ == 0) sc->touched[ntouched++] = z;
        }
    }
    for (i64 s = rp[x]; s < rp[x + 1]; s++) {
        i32 y = col[s];
        i64 dy = deg_of(rp, y), txy = tri[s];
        for (i64 r = rp[y]; r < rp[y + 1]; r++) {
            i32 z = col[r];
            if (z == x || sc->tx[z] >= 0) continue;
            i64 dz = deg_of(rp, z), tyz = tri[r];
            fv[F6_9] += dy - 2 - txy;
            fv[F9_12] += tyz;
            fv[F4_8] += dz - 1 - tyz;
            fv[F8_12] += sc->common[z] - 1;
        }
    }
    for (i64 i = 0; i < ntouched; i++) sc->common[sc->touched[i]] = 0;
    for (i64 s = rp[x]; s < rp[x + 1]; s++) sc->tx[col[s]] = -1;

    /* Equations (Section 5 and Appendix).  Halvings must be exact. */
    i64 h13 = fv[F13_14], h11 = fv[F11_13] + fv[F13_14], h9 = fv[F9_12];
    i64 h8 = fv[F13_14] + fv[F8_12], h6 = fv[F6_9] - fv[F13_14];
    if ((h13 | h11 | h9 | h8 | h6) & 1) return ORACLE_EODD;
    psi[0] = dx;
    psi[1] = psi1;
    psi[2] = pairs;
    psi[3] = triangles;
    psi[4] = 2 * fv[F12_14] + fv[F4_8] + fv[F10_13] + fv[F9_12];
    psi[5] = 2 * fv[F12_14] + fv[F5_8] + fv[F10_13] + fv[F11_13];
    psi[6] = h6 / 2 + fv[F10_13] + 2 * fv[F12_14];
    psi[7] = choose3(dx);
    psi[8] = h8 / 2;
    psi[9] = fv[F12_14] + h9 / 2;
    psi[10] = fv[F10_13] + 2 * fv[F12_14];
    psi[11] = h11 / 2;
    psi[12] = fv[F12_14];
    psi[13] = h13 / 2;
    psi[14] = k4x;
    (void)choose2;
    if (f) memcpy(f, fv, sizeof fv);
    return ORACLE_OK;
}

/* Stage III over all vertices.  psi int64[n*15]; fvars int64[n*9] or NULL. */
int oref_stage3(i32 n, const i64 *rp, const i32 *col, const i32 *tri, const i64 *K4,
                i64 *psi, i64 *fvars)
{
    if (n < 0 || (n > 0 && (!rp || !col || !K4 || !psi))) return ORACLE_EINVAL;
    if (n == 0) return ORACLE_OK;
    if (rp[n] > 0 && !tri) return ORACLE_EINVAL;
    int err = 0;
#pragma omp parallel
    {
        scratch_t sc;
        if (scratch_init(&sc, n, 0) != 0) {
#pragma omp atomic write
            err = ORACLE_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (i32 x = 0; x < n; x++) {
                int e = stage3_vertex(rp, col, tri, K4[x], x, &sc, psi + (i64)x * 15,
                                      fvars ? fvars + (i64)x * NFV : NULL);
                if (e) {
#pragma omp atomic write
                    err = e;
                }
            }
        }
        scratch_free(&sc);
    }
    return err;
}

/* The three stages in order (Algorithm 1). */
int oref_count(i32 n, const i64 *rp, const i32 *col, i64 *psi)
{
    if (n < 0 || (n > 0 && (!rp || !col || !psi))) return ORACLE_EINVAL;
    if (n == 0) return ORACLE_OK;
    i64 nnz = rp[n];
    i32 *tri = (i32 *)malloc(sizeof(i32) * (size_t)(nnz ? nnz : 1));
    i64 *K4 = (i64 *)malloc(sizeof(i64) * (size_t)n);
    if (!tri || !K4) { free(tri); free(K4); return ORACLE_ENOMEM; }
    int e = oref_stage1(n, rp, col, tri);
    if (!e) e = oref_stage2(n, rp, col, K4);
    if (!e) e = oref_stage3(n, rp, col, tri, K4, psi, NULL);
    free(tri);
    free(K4);
    return e;
}

/* Orbit counts of selected vertices only, for graphs too large for the full
 * oracle.  Stage I values are computed for the rows the probes read (row x and the
 * rows of its neighbours) by counting common neighbours with a mark array; psi_14
 * is the number of triangles inside N(x), i.e. the 4-cliques containing x (the
 * definition, since Algorithm 2 attributes globally).  xs int32[nq];
 * psi int64[nq*15]; fvars int64[nq*9] or NULL; tri_scratch int32[row_ptr[n]]
 * (caller-owned, contents overwritten). */
int oref_orbits_at(i32 n, const i64 *rp, const i32 *col, i32 nq, const i32 *xs,
                   i64 *psi, i64 *fvars, i32 *tri_scratch)
{
    if (n < 0 || nq < 0 || (nq > 0 && (!rp || !col || !xs || !psi || !tri_scratch)))
        return ORACLE_EINVAL;
    for (i32 q = 0; q < nq; q++) if (xs[q] < 0 || xs[q] >= n) return ORACLE_EINVAL;
    if (nq == 0) return ORACLE_OK;
    /* rows whose Stage I values are needed */
    unsigned char *need = (unsigned char *)calloc((size_t)n, 1);
    if (!need) return ORACLE_ENOMEM;
    for (i32 q = 0; q < nq; q++) {
        i32 x = xs[q];
        need[x] = 1;
        for (i64 s = rp[x]; s < rp[x + 1]; s++) need[col[s]] = 1;
    }
    i32 *rows = (i32 *)malloc(sizeof(i32) * (size_t)n);
    if (!rows) { free(need); return ORACLE_ENOMEM; }
    i64 nrows = 0;
    for (i32 v = 0; v < n; v++) if (need[v]) rows[nrows++] = v;
    int err = 0;
    /* t(y, z) = |N(y) and N(z)| (Algorithm 1), with N(y) marked: the members of N(z)
     * are tested against the marks, or, when N(z) is much longer than N(y), the
     * members of N(y) are searched in the sorted N(z) instead */
#pragma omp parallel
    {
        unsigned char *mark = (unsigned char *)calloc((size_t)n, 1);
        if (!mark) {
#pragma omp atomic write
            err = ORACLE_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (i64 i = 0; i < nrows; i++) {
                i32 y = rows[i];
                i64 dy = deg_of(rp, y);
                for (i64 r = rp[y]; r < rp[y + 1]; r++) mark[col[r]] = 1;
                for (i64 r = rp[y]; r < rp[y + 1]; r++) {
                    i32 z = col[r];
                    i32 c = 0;
                    if (deg_of(rp, z) <= 16 * dy) {
                        for (i64 u = rp[z]; u < rp[z + 1]; u++) c += mark[col[u]];
                    } else {
                        for (i64 u = rp[y]; u < rp[y + 1]; u++) c += slot_of(rp, col, z, col[u]) >= 0;
                    }
                    tri_scratch[r] = c;
                }
                for (i64 r = rp[y]; r < rp[y + 1]; r++) mark[col[r]] = 0;
            }
        }
        free(mark);
    }
    free(rows);
    free(need);
    if (err) return err;
#pragma omp parallel
    {
        scratch_t sc;
        if (scratch_init(&sc, n, 0) != 0) {
#pragma omp atomic write
            err = ORACLE_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (i32 q = 0; q < nq; q++) {
                i32 x = xs[q];
                /* 4-cliques containing x: triangles y < z < w inside N(x) */
                for (i64 s = rp[x]; s < rp[x + 1]; s++) sc.tx[col[s]] = 1;
                i64 k4 = 0;
                for (i64 s = rp[x]; s < rp[x + 1]; s++) {
                    i32 y = col[s];
                    for (i64 r = rp[y]; r < rp[y + 1]; r++) sc.iny[col[r]] = 1;
                    for (i64 r = rp[y]; r < rp[y + 1]; r++) {
                        i32 z = col[r];
                        if (z <= y || sc.tx[z] < 0) continue;
                        for (i64 u = rp[z]; u < rp[z + 1]; u++) {
                            i32 w = col[u];
                            if (w > z && sc.tx[w] >= 0 && sc.iny[w]) k4++;
                        }
                    }
                    for (i64 r = rp[y]; r < rp[y + 1]; r++) sc.iny[col[r]] = 0;
                }
                for (i64 s = rp[x]; s < rp[x + 1]; s++) sc.tx[col[s]] = -1;
                int e = stage3_vertex(rp, col, tri_scratch, k4, x, &sc, psi + (i64)q * 15,
                                      fvars ? fvars + (i64)q * NFV : NULL);
                if (e) {
#pragma omp atomic write
                    err = e;
                }
            }
        }
        scratch_free(&sc);
    }
    return err;
}

/* ------------------------------------------------------------------------- */
/* Whole-graph counts used as exact checks on large outputs: the number of     */
/* 4-cycles and of 4-cliques, and the 4-cliques through each edge.             */
/* ------------------------------------------------------------------------- */

/* The graph renumbered by a total order of the vertices, rows sorted: vertex
 * r is the r-th vertex in the order (degree, id) ascending.  Any total order
 * names every 4-cycle by its largest vertex and every 4-clique by its smallest;
 * ordering by degree only keeps the lists scanned below short. */
typedef struct {
    i64 *rp;   /* [n+1] */
    i32 *col;  /* [rp[n]] ranks, each row ascending */
} ranked_t;

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y);
}

static int cmp_i32(const void *a, const void *b)
{
    i32 x = *(const i32 *)a, y = *(const i32 *)b;
    return x < y ? -1 : (x > y);
}

static int ranked_build(i32 n, const i64 *rp, const i32 *col, ranked_t *R)
{
    R->rp = NULL;
    R->col = NULL;
    uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    i32 *rank = (i32 *)malloc(sizeof(i32) * (size_t)(n ? n : 1));
    R->rp = (i64 *)malloc(sizeof(i64) * (size_t)(n + 1));
    R->col = (i32 *)malloc(sizeof(i32) * (size_t)(rp[n] ? rp[n] : 1));
    if (!key || !rank || !R->rp || !R->col) {
        free(key); free(rank); free(R->rp); free(R->col);
        return ORACLE_ENOMEM;
    }
    for (i32 v = 0; v < n; v++) key[v] = ((uint64_t)deg_of(rp, v) << 32) | (uint32_t)v;
    qsort(key, (size_t)n, sizeof(uint64_t), cmp_u64);
    for (i32 r = 0; r < n; r++) rank[(i32)(key[r] & 0xffffffffu)] = r;
    R->rp[0] = 0;
    for (i32 r = 0; r < n; r++) R->rp[r + 1] = R->rp[r] + deg_of(rp, (i32)(key[r] & 0xffffffffu));
#pragma omp parallel for schedule(dynamic, 256)
    for (i32 r = 0; r < n; r++) {
        i32 v = (i32)(key[r] & 0xffffffffu);
        i64 o = R->rp[r];
        for (i64 s = rp[v]; s < rp[v + 1]; s++) R->col[o++] = rank[col[s]];
        qsort(R->col + R->rp[r], (size_t)(R->rp[r + 1] - R->rp[r]), sizeof(i32), cmp_i32);
    }
    free(key);
    free(rank);
    return ORACLE_OK;
}

static void ranked_free(ranked_t *R) { free(R->rp); free(R->col); }

/* Number of 4-cycles of G, each once.  A 4-cycle is named by its largest vertex
 * v and the vertex c opposite v; its other two vertices are common neighbours of
 * v and c below v.  So for a fixed v the cycles number sum over c < v of
 * C(k_c, 2), k_c = #{b < v : b adjacent to v and to c}. */
int oref_cycles4_total(i32 n, const i64 *rp, const i32 *col, i64 *out)
{
    if (n < 0 || (n > 0 && (!rp || !col)) || !out) return ORACLE_EINVAL;
    *out = 0;
    if (n == 0) return ORACLE_OK;
    ranked_t R;
    if (ranked_build(n, rp, col, &R)) return ORACLE_ENOMEM;
    int err = 0;
    i64 total = 0;
#pragma omp parallel reduction(+ : total)
    {
        i32 *k = (i32 *)calloc((size_t)n, sizeof(i32));
        i32 *touched = (i32 *)malloc(sizeof(i32) * (size_t)n);
        if (!k || !touched) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (i32 v = 0; v < n; v++) {
                i64 nt = 0;
                for (i64 s = R.rp[v]; s < R.rp[v + 1] && R.col[s] < v; s++) {
                    i32 b = R.col[s];
                    for (i64 q = R.rp[b]; q < R.rp[b + 1] && R.col[q] < v; q++) {
                        i32 c = R.col[q];
                        if (k[c]++ == 0) touched[nt++] = c;
                    }
                }
                for (i64 i = 0; i < nt; i++) {
                    i64 kc = k[touched[i]];
                    total += kc * (kc - 1) / 2;
                    k[touched[i]] = 0;
                }
            }
        }
        free(k);
        free(touched);
    }
    ranked_free(&R);
    if (err) return ORACLE_ENOMEM;
    *out = total;
    return ORACLE_OK;
}

/* Number of 4-cliques of G, each once.  A 4-clique is named by its smallest
 * vertex u; the other three are neighbours of u above it, pairwise adjacent: a
 * triangle of the graph H_u on the neighbours above u.  H_u is kept as bit rows
 * (row i: the neighbours above u adjacent to the i-th one and above it), and
 * every edge (i, p) of H_u closes as many triangles as rows i and p share bits. */
int oref_k4_total(i32 n, const i64 *rp, const i32 *col, i64 *out)
{
    if (n < 0 || (n > 0 && (!rp || !col)) || !out) return ORACLE_EINVAL;
    *out = 0;
    if (n == 0) return ORACLE_OK;
    ranked_t R;
    if (ranked_build(n, rp, col, &R)) return ORACLE_ENOMEM;
    int err = 0;
    i64 total = 0;
#pragma omp parallel reduction(+ : total)
    {
        i32 *pos = (i32 *)malloc(sizeof(i32) * (size_t)n);
        uint64_t *rows = NULL;
        i64 rows_cap = 0;
        if (!pos) {
#pragma omp atomic write
            err = 1;
        } else {
            for (i32 v = 0; v < n; v++) pos[v] = -1;
#pragma omp for schedule(dynamic, 16)
            for (i32 u = 0; u < n; u++) {
                i64 a = R.rp[u], e = R.rp[u + 1];
                while (a < e && R.col[a] < u) a++;        /* neighbours above u: R.col[a..e) */
                i64 du = e - a;
                if (du < 3) continue;
                i64 words = (du + 63) / 64;
                if (du * words > rows_cap) {
                    free(rows);
                    rows_cap = du * words;
                    rows = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)rows_cap);
                    if (!rows) {
                        rows_cap = 0;
#pragma omp atomic write
                        err = 1;
                        continue;
                    }
                }
                memset(rows, 0, sizeof(uint64_t) * (size_t)(du * words));
                for (i64 i = 0; i < du; i++) pos[R.col[a + i]] = (i32)i;
                for (i64 i = 0; i < du; i++) {
                    i32 v = R.col[a + i];
                    for (i64 q = R.rp[v + 1] - 1; q >= R.rp[v] && R.col[q] > v; q--) {
                        i32 p = pos[R.col[q]];
                        if (p >= 0) rows[i * words + p / 64] |= 1ull << (p % 64);
                    }
                }
                for (i64 i = 0; i < du; i++)
                    for (i64 w = 0; w < words; w++) {
                        uint64_t bits = rows[i * words + w];
                        while (bits) {
                            i64 p = w * 64 + __builtin_ctzll(bits);
                            bits &= bits - 1;
                            for (i64 x = 0; x < words; x++)
                                total += __builtin_popcountll(rows[i * words + x] & rows[p * words + x]);
                        }
                    }
                for (i64 i = 0; i < du; i++) pos[R.col[a + i]] = -1;
            }
        }
        free(pos);
        free(rows);
    }
    ranked_free(&R);
    if (err) return ORACLE_ENOMEM;
    *out = total;
    return ORACLE_OK;
}

/* 4-cliques through edges: for CSR slot s = (a, b), ek4 = the number of edges
 * {c, d} of G with c and d both common neighbours of a and b (each such edge makes
 * {a, b, c, d} a 4-clique, and every 4-clique through a and b arises once).  For
 * nq slots listed in slots (all rp[n] slots when slots is NULL); ek4 int64[nq]
 * (or int64[rp[n]]). */
int oref_edge_k4(i32 n, const i64 *rp, const i32 *col, i64 nq, const i64 *slots, i64 *ek4)
{
    if (n < 0 || (n > 0 && (!rp || !col)) || !ek4) return ORACLE_EINVAL;
    if (n == 0) return ORACLE_OK;
    const i64 nnz = rp[n];
    if (!slots) nq = nnz;
    for (i64 q = 0; slots && q < nq; q++) if (slots[q] < 0 || slots[q] >= nnz) return ORACLE_EINVAL;
    int err = 0;
#pragma omp parallel
    {
        unsigned char *inw = (unsigned char *)calloc((size_t)n, 1);
        i32 *w = (i32 *)malloc(sizeof(i32) * (size_t)n);
        if (!inw || !w) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (i64 q = 0; q < nq; q++) {
                i64 s = slots ? slots[q] : q;
                /* the row a that holds slot s */
                i64 lo = 0, hi = n;
                while (hi - lo > 1) {
                    i64 mid = (lo + hi) / 2;
                    if (rp[mid] <= s) lo = mid; else hi = mid;
                }
                i32 a = (i32)lo, b = col[s];
                /* W = N(a) and N(b) by a sorted merge */
                i64 nw = 0, i = rp[a], j = rp[b];
                while (i < rp[a + 1] && j < rp[b + 1]) {
                    if (col[i] < col[j]) i++;
                    else if (col[i] > col[j]) j++;
                    else { w[nw++] = col[i]; i++; j++; }
                }
                for (i64 k = 0; k < nw; k++) inw[w[k]] = 1;
                i64 ends = 0;   /* each edge inside W is seen from both ends */
                for (i64 k = 0; k < nw; k++)
                    for (i64 r = rp[w[k]]; r < rp[w[k] + 1]; r++) ends += inw[col[r]];
                for (i64 k = 0; k < nw; k++) inw[w[k]] = 0;
                ek4[q] = ends / 2;
            }
        }
        free(inw);
        free(w);
    }
    return err ? ORACLE_ENOMEM : ORACLE_OK;
}

/* Stages II and III for selected vertices, given the Stage I counts of the whole
 * graph (tri from oref_stage1): K4 of each x counted as in oref_stage2, then the
 * Stage III probe and equations of oref_stage3.  Used to time the three stages on
 * a vertex sample of a graph too large for a full run; psi int64[nq*15]. */
int oref_stage23_at(i32 n, const i64 *rp, const i32 *col, const i32 *tri, i32 nq, const i32 *xs,
                    i64 *psi)
{
    if (n < 0 || nq < 0 || (nq > 0 && (!rp || !col || !tri || !xs || !psi))) return ORACLE_EINVAL;
    for (i32 q = 0; q < nq; q++) if (xs[q] < 0 || xs[q] >= n) return ORACLE_EINVAL;
    if (nq == 0) return ORACLE_OK;
    int err = 0;
#pragma omp parallel
    {
        scratch_t sc;
        unsigned char *inx = (unsigned char *)calloc((size_t)n, 1);
        unsigned char *ina = (unsigned char *)calloc((size_t)n, 1);
        if (scratch_init(&sc, n, 0) != 0 || !inx || !ina) {
#pragma omp atomic write
            err = ORACLE_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (i32 q = 0; q < nq; q++) {
                i32 x = xs[q];
                i64 cliques = 0;
                for (i64 s = rp[x]; s < rp[x + 1]; s++) inx[col[s]] = 1;
                for (i64 s = rp[x]; s < rp[x + 1]; s++) {
                    i32 a = col[s];
                    for (i64 r = rp[a]; r < rp[a + 1]; r++) ina[col[r]] = 1;
                    for (i64 r = rp[a]; r < rp[a + 1]; r++) {
                        i32 b = col[r];
                        if (b <= a || !inx[b]) continue;
                        for (i64 u = rp[b]; u < rp[b + 1]; u++) {
                            i32 c = col[u];
                            if (c > b && inx[c] && ina[c]) cliques++;
                        }
                    }
                    for (i64 r = rp[a]; r < rp[a + 1]; r++) ina[col[r]] = 0;
                }
                for (i64 s = rp[x]; s < rp[x + 1]; s++) inx[col[s]] = 0;
                int e = stage3_vertex(rp, col, tri, cliques, x, &sc, psi + (i64)q * 15, NULL);
                if (e) {
#pragma omp atomic write
                    err = e;
                }
            }
        }
        scratch_free(&sc);
        free(inx);
        free(ina);
    }
    return err;
}

/* psi_8 of selected vertices from its definition: the 4-cycles through x are the
 * pairs of common neighbours of x and a vertex z != x opposite it, so psi_8(x) =
 * sum over z != x of C(|N(x) and N(z)|, 2), with the common neighbours counted
 * over every path x - y - z.  out int64[nq]. */
int oref_cycles4_at(i32 n, const i64 *rp, const i32 *col, i32 nq, const i32 *xs, i64 *out)
{
    if (n < 0 || nq < 0 || (nq > 0 && (!rp || !col || !xs || !out))) return ORACLE_EINVAL;
    for (i32 q = 0; q < nq; q++) if (xs[q] < 0 || xs[q] >= n) return ORACLE_EINVAL;
    int err = 0;
#pragma omp parallel
    {
        i64 *common = (i64 *)calloc((size_t)(n ? n : 1), sizeof(i64));
        i32 *touched = (i32 *)malloc(sizeof(i32) * (size_t)(n ? n : 1));
        if (!common || !touched) {
#pragma omp atomic write
            err = ORACLE_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (i32 q = 0; q < nq; q++) {
                i32 x = xs[q];
                i64 nt = 0, total = 0;
                for (i64 s = rp[x]; s < rp[x + 1]; s++) {
                    i32 y = col[s];
                    for (i64 r = rp[y]; r < rp[y + 1]; r++) {
                        i32 z = col[r];
                        if (z == x) continue;
                        if (common[z]++ == 0) touched[nt++] = z;
                    }
                }
                for (i64 i = 0; i < nt; i++) {
                    total += common[touched[i]] * (common[touched[i]] - 1) / 2;
                    common[touched[i]] = 0;
                }
                out[q] = total;
            }
        }
        free(common);
        free(touched);
    }
    return err;
}
