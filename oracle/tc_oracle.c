/*
 * CPU oracle for the degree-partitioned sampling triangle counter of
 * Kolountzakis, Miller, Peng and Tsourakakis, "Efficient Triangle Counting in
 * Large Graphs via Degree-based Vertex Partitioning" (arXiv:1011.0468).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded C that computes what
 * the device path computes, from the paper's definitions.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never does.  It shares no code with the device path.
 *
 * Readings where the paper leaves a choice open (each one also documented
 * with the design notes):
 *   - the edge coin is a counter-based hash (SplitMix64's output mixer) of the
 *     undirected pair and the seed; the paper leaves the random source open
 *     (section 3.1) and its own sampler draws geometric gaps (section 4.2.1);
 *   - the light/heavy split uses the sampled graph's m' and degrees, with the
 *     integer test b^2 deg^2 > a^2 m' for "heavy" (section 3.2 uses a = b = 1:
 *     light means deg <= m^(1/2));
 *   - the exact count charges each triangle to its lowest (degree, id) vertex;
 *     the all-heavy triangles form T_H and the rest T_L (section 3.2 gives the
 *     two vertex classes, not the rule that avoids double counting);
 *   - the random projection uses Rademacher signs instead of Gaussian entries
 *     (section 5.1), which keeps every quantity an exact integer.
 *
 * Parity pins: see the test suite.  Every function below is pinned by a test
 * that does not re-derive it from itself (closed forms, brute force, dense
 * linear algebra, published SplitMix64 output vectors, statistical laws).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Normalisation: the simple undirected graph of section 4.1 (duplicates and  */
/* self-loops removed), as sorted neighbour lists (section 4.2).              */
/* ------------------------------------------------------------------------- */

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/*
 * Build the symmetric sorted adjacency lists of E = {{u,v} : (u,v) or (v,u) in
 * the input, u != v}.  row_ptr has n+1 entries, col must hold 2*num_pairs.
 * Returns 0, or 1 if an id is outside [0,n), or 2 on allocation failure.
 */
int or_normalise(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst,
                 int64_t* row_ptr, int32_t* col, int64_t* m_out) {
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(num_pairs > 0 ? num_pairs : 1));
    if (!keys) return 2;
    int64_t k = 0;
    for (int64_t i = 0; i < num_pairs; ++i) {
        int64_t u = src[i], v = dst[i];
        if (u < 0 || u >= n || v < 0 || v >= n) { free(keys); return 1; }
        if (u == v) continue;
        uint64_t a = (uint64_t)(u < v ? u : v), b = (uint64_t)(u < v ? v : u);
        keys[k++] = (a << 32) | b;
    }
    qsort(keys, (size_t)k, sizeof(uint64_t), cmp_u64);
    int64_t m = 0;
    for (int64_t i = 0; i < k; ++i)
        if (i == 0 || keys[i] != keys[i - 1]) keys[m++] = keys[i];
    for (int64_t v = 0; v <= n; ++v) row_ptr[v] = 0;
    for (int64_t i = 0; i < m; ++i) {
        row_ptr[(keys[i] >> 32) + 1] += 1;
        row_ptr[(keys[i] & 0xffffffffu) + 1] += 1;
    }
    for (int64_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!fill) { free(keys); return 2; }
    for (int64_t v = 0; v < n; ++v) fill[v] = row_ptr[v];
    /* keys ascend by (a, b): row x first receives its smaller neighbours a < x
       in ascending order, then its larger neighbours b > x in ascending order */
    for (int64_t i = 0; i < m; ++i) {
        int64_t a = (int64_t)(keys[i] >> 32), b = (int64_t)(keys[i] & 0xffffffffu);
        col[fill[a]++] = (int32_t)b;
        col[fill[b]++] = (int32_t)a;
    }
    free(fill);
    free(keys);
    *m_out = m;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Edge sparsification (section 3.1): keep each edge independently with      */
/* probability p.  The coin is the SplitMix64 output mixer (Steele, Lea and   */
/* Flood, OOPSLA 2014) applied to the undirected pair and the seed.           */
/* ------------------------------------------------------------------------- */

uint64_t or_mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

/* keep threshold: floor(p * 2^53) */
uint64_t or_keep_threshold(double p) {
    return (uint64_t)(p * 9007199254740992.0);
}

/* 1 if the undirected edge {u,v} is kept under (seed, threshold) */
int or_keep(int32_t u, int32_t v, uint64_t seed, uint64_t threshold) {
    uint64_t s = or_mix64(seed ^ 0x54435F53414D504CULL);   /* "TC_SAMPL" */
    uint64_t lo = (uint64_t)(uint32_t)(u < v ? u : v);
    uint64_t hi = (uint64_t)(uint32_t)(u < v ? v : u);
    uint64_t h = or_mix64(or_mix64((lo << 32) | hi) ^ s);
    return (h >> 11) < threshold;
}

/*
 * Sampled graph G_p = (V, E_p) from a normalised graph: row_ptr_p (n+1) and
 * col_p (capacity row_ptr[n]).  Lists stay sorted.  Returns m' (edges kept).
 */
int64_t or_sample(int64_t n, const int64_t* row_ptr, const int32_t* col, double p, uint64_t seed,
                  int64_t* row_ptr_p, int32_t* col_p) {
    uint64_t thr = or_keep_threshold(p);
    int64_t pos = 0;
    for (int64_t u = 0; u < n; ++u) {
        row_ptr_p[u] = pos;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (or_keep((int32_t)u, col[e], seed, thr)) col_p[pos++] = col[e];
    }
    row_ptr_p[n] = pos;
    return pos / 2;
}

/* ------------------------------------------------------------------------- */
/* Triangle count: t = |{ {a,b,c} : ab, bc, ca in E }| (Table 1 notation).    */
/* ------------------------------------------------------------------------- */

/* rank order (deg, id), lexicographic */
static int rank_less(int64_t du, int64_t u, int64_t dv, int64_t v) {
    return du < dv || (du == dv && u < v);
}

/*
 * Count every triangle once, at its lowest (degree, id) vertex u: for each
 * oriented edge u -> v, count common out-neighbours by merging the two sorted
 * out-lists.  If per_vertex is not NULL it receives, for each u, the number of
 * triangles whose lowest-ranked vertex is u.
 */
int64_t or_count_triangles(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t* per_vertex) {
    int64_t m2 = row_ptr[n];
    int64_t* orp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t* ocol = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m2 / 2 + 1));
    if (!orp || !ocol) { free(orp); free(ocol); return -1; }
    int64_t pos = 0;
    for (int64_t u = 0; u < n; ++u) {
        orp[u] = pos;
        int64_t du = row_ptr[u + 1] - row_ptr[u];
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t v = col[e];
            int64_t dv = row_ptr[v + 1] - row_ptr[v];
            if (rank_less(du, u, dv, v)) ocol[pos++] = (int32_t)v;
        }
    }
    orp[n] = pos;
    int64_t total = 0;
    for (int64_t u = 0; u < n; ++u) {
        int64_t tu = 0;
        for (int64_t e = orp[u]; e < orp[u + 1]; ++e) {
            int64_t v = ocol[e];
            int64_t i = orp[u], iend = orp[u + 1], j = orp[v], jend = orp[v + 1];
            while (i < iend && j < jend) {
                if (ocol[i] < ocol[j]) ++i;
                else if (ocol[i] > ocol[j]) ++j;
                else { ++tu; ++i; ++j; }
            }
        }
        if (per_vertex) per_vertex[u] = tu;
        total += tu;
    }
    free(orp);
    free(ocol);
    return total;
}

/*
 * The same count by vertex id order: each triangle a < b < c is found from its
 * edge (a, b) by merging N(a) and N(b) restricted to ids above b.
 */
int64_t or_count_triangles_idorder(int64_t n, const int64_t* row_ptr, const int32_t* col) {
    int64_t total = 0;
    for (int64_t a = 0; a < n; ++a) {
        for (int64_t e = row_ptr[a]; e < row_ptr[a + 1]; ++e) {
            int64_t b = col[e];
            if (b <= a) continue;
            int64_t i = row_ptr[a], iend = row_ptr[a + 1], j = row_ptr[b], jend = row_ptr[b + 1];
            while (i < iend && j < jend) {
                if (col[i] < col[j]) ++i;
                else if (col[i] > col[j]) ++j;
                else { if (col[i] > b) ++total; ++i; ++j; }
            }
        }
    }
    return total;
}

/* Brute force over all vertex triples of a dense 0/1 adjacency (n x n, row-major). */
int64_t or_count_bruteforce(int64_t n, const uint8_t* adj) {
    int64_t t = 0;
    for (int64_t a = 0; a < n; ++a)
        for (int64_t b = a + 1; b < n; ++b) {
            if (!adj[a * n + b]) continue;
            for (int64_t c = b + 1; c < n; ++c)
                if (adj[a * n + c] && adj[b * n + c]) ++t;
        }
    return t;
}

/* ------------------------------------------------------------------------- */
/* Degree partition (section 3.2): heavy iff deg > c * m^(1/2), c = a/b, as   */
/* the integer test b^2 deg^2 > a^2 m.                                         */
/* ------------------------------------------------------------------------- */

int or_is_heavy(int64_t deg, int64_t m, int32_t a, int32_t b) {
    /* 128-bit products: exact for every int32 a, b and int64 deg, m < 2^62 */
    unsigned __int128 lhs = (unsigned __int128)(uint64_t)b * (uint64_t)b * (uint64_t)deg * (uint64_t)deg;
    unsigned __int128 rhs = (unsigned __int128)(uint64_t)a * (uint64_t)a * (uint64_t)m;
    return lhs > rhs;
}

/*
 * Exact count with the reported light/heavy split on a normalised graph:
 * out[0] = T, out[1] = T_L, out[2] = T_H (triangles with all three vertices
 * heavy), out[3] = number of heavy vertices, out[4] = m.
 * Returns 0 or 2 on allocation failure.
 */
int or_count_split(int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t a, int32_t b,
                   int64_t* out) {
    int64_t m = row_ptr[n] / 2;
    int64_t T = or_count_triangles(n, row_ptr, col, NULL);
    if (T < 0) return 2;
    /* induced subgraph on the heavy set, with the original ids kept */
    int64_t* hrp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t* hcol = (int32_t*)malloc(sizeof(int32_t) * (size_t)(row_ptr[n] + 1));
    if (!hrp || !hcol) { free(hrp); free(hcol); return 2; }
    int64_t pos = 0, h = 0;
    for (int64_t u = 0; u < n; ++u) {
        hrp[u] = pos;
        int heavy_u = or_is_heavy(row_ptr[u + 1] - row_ptr[u], m, a, b);
        h += heavy_u;
        if (!heavy_u) continue;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t v = col[e];
            if (or_is_heavy(row_ptr[v + 1] - row_ptr[v], m, a, b)) hcol[pos++] = (int32_t)v;
        }
    }
    hrp[n] = pos;
    int64_t TH = or_count_triangles(n, hrp, hcol, NULL);
    free(hrp);
    free(hcol);
    if (TH < 0) return 2;
    out[0] = T;
    out[1] = T - TH;
    out[2] = TH;
    out[3] = h;
    out[4] = m;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Rescaling (section 3.1): E[T_p] = p^3 t, so the estimate is T_p / p^3.     */
/* ------------------------------------------------------------------------- */

double or_estimate(int64_t T, double p) {
    volatile double p2 = p * p;          /* fixed order: (p*p)*p, no contraction */
    volatile double p3 = p2 * p;
    return (double)T / p3;
}

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/*
 * Median of means over S = num_seeds counts in G consecutive groups of S/G:
 * group sums are sorted; for odd G the middle sum, for even G the sum of the
 * two middle sums, is divided once by (number of sums taken) * (S/G) * p^3.
 */
double or_median_of_means(const int64_t* counts, int32_t num_seeds, int32_t num_groups, double p) {
    int32_t per = num_seeds / num_groups;
    int64_t* sums = (int64_t*)malloc(sizeof(int64_t) * (size_t)num_groups);
    for (int32_t g = 0; g < num_groups; ++g) {
        int64_t s = 0;
        for (int32_t i = 0; i < per; ++i) s += counts[g * per + i];
        sums[g] = s;
    }
    qsort(sums, (size_t)num_groups, sizeof(int64_t), cmp_i64);
    volatile double p2 = p * p;
    volatile double p3 = p2 * p;
    double r;
    if (num_groups % 2 == 0) {
        int64_t M = sums[num_groups / 2 - 1] + sums[num_groups / 2];
        volatile double den = 2.0 * (double)per;
        den = den * p3;
        r = (double)M / den;
    } else {
        volatile double den = (double)per;
        den = den * p3;
        r = (double)sums[(num_groups - 1) / 2] / den;
    }
    free(sums);
    return r;
}

/* ------------------------------------------------------------------------- */
/* Random projection (section 5.1): Y = sum_l r_l^T A^3 r_l.  With Rademacher */
/* vectors x_l, q_l = x_l^T A^3 x_l = (A x_l)^T A (A x_l) is an exact integer. */
/* ------------------------------------------------------------------------- */

/* sign of vector l at vertex i: +1 if the selected hash bit is 0, else -1 */
int or_rp_sign(uint64_t seed, int64_t l, int64_t i) {
    uint64_t r = or_mix64(seed ^ 0x52505F5452414345ULL);     /* "RP_TRACE" */
    uint64_t w = or_mix64(or_mix64(((uint64_t)(l >> 6) << 32) | (uint64_t)i) ^ r);
    return ((w >> (l & 63)) & 1ULL) ? -1 : 1;
}

/* q = x^T A^3 x for an explicit integer vector x (length n), with y = A x. */
int64_t or_quadform_a3(int64_t n, const int64_t* row_ptr, const int32_t* col, const int64_t* x) {
    int64_t* y = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t s = 0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) s += x[col[e]];
        y[i] = s;
    }
    int64_t q = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t z = 0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) z += y[col[e]];
        q += y[i] * z;
    }
    free(y);
    return q;
}

/*
 * q_l for l in [0,k), and the triangle estimate (sum_l q_l) / (6 k): the mean
 * of x^T A^3 x is tr(A^3), which is six times the triangle count.
 */
int or_rp_trace(int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t k, uint64_t seed,
                int64_t* q, double* tri_est) {
    int64_t* x = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!x) return 2;
    __int128 total = 0;
    for (int32_t l = 0; l < k; ++l) {
        for (int64_t i = 0; i < n; ++i) x[i] = or_rp_sign(seed, l, i);
        q[l] = or_quadform_a3(n, row_ptr, col, x);
        total += q[l];
    }
    free(x);
    *tri_est = (double)total / (6.0 * (double)k);
    return 0;
}

/* q_l for one vector index l (for checking sampled entries of a large run) */
int64_t or_rp_q(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t l, uint64_t seed) {
    int64_t* x = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) x[i] = or_rp_sign(seed, l, i);
    int64_t q = or_quadform_a3(n, row_ptr, col, x);
    free(x);
    return q;
}

/* ------------------------------------------------------------------------- */
/* Triple sampling (section 3.2, "Triple Sampling"; the Simple and Hybrid    */
/* columns of Table 2).                                                       */
/* ------------------------------------------------------------------------- */

/*
 * The candidate set U, in a fixed order: vertices u ascending; a vertex of
 * the wedge kind contributes its pairs of neighbour positions (a, b), a < b,
 * in colex order ((0,1), (0,2), (1,2), (0,3), ...), the triple
 * (N(u)[a], u, N(u)[b]); a vertex of the extension kind contributes, for each
 * neighbour position a (v = N(u)[a]) in order, each neighbour position j of v
 * (w = N(v)[j]), the triple (u, v, w).  Simple: every vertex is of the wedge
 * kind.  Hybrid: a vertex x is of the extension kind iff deg(x)^2 > m (the
 * degree split of section 3.2).  A wedge is closed iff its two ends are
 * adjacent; an extension (u, v, w) iff w != u and w is adjacent to u.  A
 * triangle appears once per wedge-kind vertex and twice per extension-kind
 * vertex, so a closed sample weighs 60 / (3 + its extension-kind vertices)
 * and the weights of one triangle's appearances sum to 60.
 */
static int ext_kind(int hybrid, int64_t deg, int64_t m) { return hybrid && deg * deg > m; }

static int adjacent(const int64_t* row_ptr, const int32_t* col, int32_t x, int32_t y) {
    int64_t lo = row_ptr[x], hi = row_ptr[x + 1];  /* sorted list of x: binary search for y */
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < y) lo = mid + 1;
        else hi = mid;
    }
    return lo < row_ptr[x + 1] && col[lo] == y;
}

/* number of triples of vertex u */
static int64_t triples_of(int hybrid, const int64_t* row_ptr, const int32_t* col, int64_t m, int64_t u) {
    const int64_t d = row_ptr[u + 1] - row_ptr[u];
    if (!ext_kind(hybrid, d, m)) return d * (d - 1) / 2;
    int64_t c = 0;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) c += row_ptr[col[e] + 1] - row_ptr[col[e]];
    return c;
}

/* |U|; prefix (n+1 entries, may be NULL) receives the start of each vertex's triples */
int64_t or_triples_size(int64_t n, const int64_t* row_ptr, const int32_t* col, int hybrid, int64_t* prefix) {
    const int64_t m = row_ptr[n] / 2;
    int64_t tot = 0;
    for (int64_t u = 0; u < n; ++u) {
        if (prefix) prefix[u] = tot;
        tot += triples_of(hybrid, row_ptr, col, m, u);
    }
    if (prefix) prefix[n] = tot;
    return tot;
}

/*
 * Triple r of U (0 <= r < |U|, prefix from or_triples_size): *x, *y, *z get
 * its vertices in the order of the definition above; returns its weight
 * (60 / (3 + extension-kind vertices)) if it is closed, else 0.
 */
int64_t or_triple_at(int64_t n, const int64_t* row_ptr, const int32_t* col, int hybrid, const int64_t* prefix,
                     int64_t r, int32_t* x, int32_t* y, int32_t* z) {
    const int64_t m = row_ptr[n] / 2;
    int64_t lo = 0, hi = n - 1;  /* the vertex u with prefix[u] <= r < prefix[u+1] */
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (prefix[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    const int64_t u = lo, k = r - prefix[u];
    const int64_t d = row_ptr[u + 1] - row_ptr[u];
    int closed;
    if (!ext_kind(hybrid, d, m)) {
        int64_t b = 1;  /* the largest b with b (b - 1) / 2 <= k */
        while ((b + 1) * b / 2 <= k) ++b;
        const int64_t a = k - b * (b - 1) / 2;
        *x = col[row_ptr[u] + a];
        *y = (int32_t)u;
        *z = col[row_ptr[u] + b];
        closed = adjacent(row_ptr, col, *x, *z);
    } else {
        int64_t e = row_ptr[u], acc = 0;  /* the neighbour position a holding k */
        while (acc + (row_ptr[col[e] + 1] - row_ptr[col[e]]) <= k) {
            acc += row_ptr[col[e] + 1] - row_ptr[col[e]];
            ++e;
        }
        const int32_t v = col[e];
        *x = (int32_t)u;
        *y = v;
        *z = col[row_ptr[v] + (k - acc)];
        closed = *z != (int32_t)u && adjacent(row_ptr, col, (int32_t)u, *z);
    }
    if (!closed) return 0;
    const int ne = ext_kind(hybrid, row_ptr[*x + 1] - row_ptr[*x], m) +
                   ext_kind(hybrid, row_ptr[*y + 1] - row_ptr[*y], m) +
                   ext_kind(hybrid, row_ptr[*z + 1] - row_ptr[*z], m);
    return 60 / (3 + ne);
}

/* index of sample i under seed: the high 64 bits of h * size, h a 64-bit hash of (seed, i) */
int64_t or_triple_index(uint64_t seed, int64_t i, int64_t size) {
    const uint64_t salt = or_mix64(seed ^ 0x54435F545249504CULL);  /* "TC_TRIPL" */
    const uint64_t h = or_mix64(or_mix64((uint64_t)i) ^ salt);
    return (int64_t)(((unsigned __int128)h * (uint64_t)size) >> 64);
}

/*
 * s samples of U with replacement: out[0] = |U|, out[1] = sum of the weights
 * of the closed samples, out[2] = closed samples.  Returns 0, or 2 on
 * allocation failure.  The estimate of t is |U| out[1] / (60 s).
 */
int or_triple_sample(int64_t n, const int64_t* row_ptr, const int32_t* col, int hybrid, int64_t s,
                     uint64_t seed, int64_t* out) {
    int64_t* prefix = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!prefix) return 2;
    const int64_t size = or_triples_size(n, row_ptr, col, hybrid, prefix);
    int64_t wsum = 0, closed = 0;
    for (int64_t i = 0; size > 0 && i < s; ++i) {
        int32_t x, y, z;
        const int64_t w = or_triple_at(n, row_ptr, col, hybrid, prefix, or_triple_index(seed, i, size), &x, &y, &z);
        wsum += w;
        closed += w > 0;
    }
    free(prefix);
    out[0] = size;
    out[1] = wsum;
    out[2] = closed;
    return 0;
}

/* |U| out[1] / (60 s), then rescaled by 1/p^3 as or_estimate does */
double or_triple_estimate(int64_t size, int64_t wsum, int64_t s, double p) {
    volatile double num = (double)size * (double)wsum;
    volatile double den = 60.0 * (double)s;
    volatile double t = num / den;
    volatile double p2 = p * p;
    volatile double p3 = p2 * p;
    return t / p3;
}

/* ------------------------------------------------------------------------- */
/* Semi-streaming variant (section 5.2): three passes over the edge stream,   */
/* the adjacency lists given in order.                                        */
/*                                                                            */
/* Pass 1: s1 = ceil(d m^(1/2) ln n) edges drawn uniformly with replacement   */
/* (the Lemma of section 5.2: every vertex of degree above m^(1/2) is then an */
/* endpoint of a drawn edge with probability at least 1 - n^(1-d)); their    */
/* endpoints are the heavy candidates C, and one more pass over the edges     */
/* (their degrees) keeps H = {x in C : deg(x)^2 > m}.                         */
/* Pass 2: the triples to check are U = L followed by X:                      */
/*   L: for every vertex u not in H (ascending), its wedges (N(u)[a], u,      */
/*      N(u)[b]), a < b positions in colex order; closed iff the ends are     */
/*      adjacent;                                                             */
/*   X: for every h in H (ascending) and every edge e = {v, w} (v < w, in     */
/*      (v, w) order), the pair (h; e); closed iff h is not in e and adjacent */
/*      to both ends.                                                         */
/* Every triangle has exactly three closed elements in U, one per vertex (a   */
/* wedge at a vertex outside H, a pair at a vertex of H), so with s draws     */
/* with replacement, t = |U| closed / (3 s) is unbiased.                      */
/* Pass 3: the closing edges the draws ask for are looked up in one pass over */
/* the edges; here the lookup is the definition itself (adjacency).          */
/*                                                                            */
/* Draw i of pass 1 is upper edge floor(h m / 2^64) (h = mix64(mix64(i) ^     */
/* mix64(seed ^ "TC_STRM1"))), draw j of pass 2 is element                    */
/* floor(h' |U| / 2^64) of U (h' = mix64(mix64(j) ^ mix64(seed ^             */
/* "TC_STRM2"))).                                                             */
/* ------------------------------------------------------------------------- */

static int64_t hi_mul(uint64_t h, uint64_t size) { return (int64_t)(((unsigned __int128)h * size) >> 64); }

int64_t or_stream_draws(int64_t n, int64_t m, double d) {
    if (n < 2 || m < 1) return 0;
    return (int64_t)ceil(d * sqrt((double)m) * log((double)n));
}

/* (u, v) of upper edge r (0 <= r < m): up[u] = number of neighbours of u
   above u, upre its exclusive prefix */
static void upper_edge(int64_t n, const int64_t* row_ptr, const int32_t* col, const int64_t* upre, int64_t r,
                       int32_t* u, int32_t* v) {
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (upre[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    const int64_t deg = row_ptr[lo + 1] - row_ptr[lo];
    const int64_t up = upre[lo + 1] - upre[lo];
    *u = (int32_t)lo;
    *v = col[row_ptr[lo] + (deg - up) + (r - upre[lo])];
}

/* closed elements among all of U for a given heavy set (flags[x] != 0):
   sums over every element, for the pins */
int64_t or_stream_closed_all(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint8_t* heavy) {
    int64_t closed = 0;
    for (int64_t u = 0; u < n; ++u) {
        if (heavy[u]) continue;
        for (int64_t a = row_ptr[u]; a < row_ptr[u + 1]; ++a)
            for (int64_t b = a + 1; b < row_ptr[u + 1]; ++b) closed += adjacent(row_ptr, col, col[a], col[b]);
    }
    for (int64_t h = 0; h < n; ++h) {
        if (!heavy[h]) continue;
        for (int64_t v = 0; v < n; ++v)
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                const int32_t w = col[e];
                if (w <= v || h == v || h == w) continue;
                closed += adjacent(row_ptr, col, (int32_t)h, (int32_t)v) && adjacent(row_ptr, col, (int32_t)h, w);
            }
    }
    return closed;
}

/*
 * The semi-streaming estimate with candidate multiplier d, s draws of pass 2
 * and the given seed.  out[0] = s1, out[1] = |C|, out[2] = |H|, out[3] = |L|,
 * out[4] = |U|, out[5] = edge queries of pass 3 (one per wedge, two per pair
 * whose vertex is not in its edge), out[6] = closed draws, out[7] = m.
 * heavy (n bytes, may be NULL) receives the flags of H.  Returns 0, or 2 on
 * allocation failure.
 */
int or_stream_estimate(int64_t n, const int64_t* row_ptr, const int32_t* col, double d, int64_t s, uint64_t seed,
                       int64_t* out, uint8_t* heavy) {
    const int64_t m = row_ptr[n] / 2;
    int64_t* upre = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t* lpre = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    uint8_t* cand = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t* hlist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!upre || !lpre || !cand || !hlist) {
        free(upre); free(lpre); free(cand); free(hlist);
        return 2;
    }
    upre[0] = 0;
    for (int64_t u = 0; u < n; ++u) {
        int64_t up = 0;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) up += col[e] > u;
        upre[u + 1] = upre[u] + up;
    }
    /* pass 1: candidates, then H */
    const int64_t s1 = or_stream_draws(n, m, d);
    const uint64_t salt1 = or_mix64(seed ^ 0x54435F5354524D31ULL); /* "TC_STRM1" */
    for (int64_t i = 0; i < s1; ++i) {
        int32_t u, v;
        upper_edge(n, row_ptr, col, upre, hi_mul(or_mix64(or_mix64((uint64_t)i) ^ salt1), (uint64_t)m), &u, &v);
        cand[u] = 1;
        cand[v] = 1;
    }
    int64_t nc = 0, nh = 0;
    for (int64_t x = 0; x < n; ++x) {
        nc += cand[x];
        const int64_t dx = row_ptr[x + 1] - row_ptr[x];
        const int hv = cand[x] && or_is_heavy(dx, m, 1, 1);
        if (heavy) heavy[x] = (uint8_t)hv;
        if (hv) hlist[nh++] = (int32_t)x;
        cand[x] = (uint8_t)hv; /* from here on: the flags of H */
    }
    /* pass 2: U = L (wedges at vertices outside H) followed by X = H x E */
    lpre[0] = 0;
    for (int64_t u = 0; u < n; ++u) {
        const int64_t du = row_ptr[u + 1] - row_ptr[u];
        lpre[u + 1] = lpre[u] + (cand[u] ? 0 : du * (du - 1) / 2);
    }
    const int64_t L = lpre[n], size = L + nh * m;
    const uint64_t salt2 = or_mix64(seed ^ 0x54435F5354524D32ULL); /* "TC_STRM2" */
    int64_t queries = 0, closed = 0;
    for (int64_t j = 0; size > 0 && j < s; ++j) {
        const int64_t r = hi_mul(or_mix64(or_mix64((uint64_t)j) ^ salt2), (uint64_t)size);
        if (r < L) {
            int64_t lo = 0, hi = n - 1; /* the vertex u with lpre[u] <= r < lpre[u+1] */
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo + 1) / 2;
                if (lpre[mid] <= r) lo = mid;
                else hi = mid - 1;
            }
            const int64_t k = r - lpre[lo];
            int64_t b = 1; /* the largest b with b (b - 1) / 2 <= k */
            while ((b + 1) * b / 2 <= k) ++b;
            const int64_t a = k - b * (b - 1) / 2;
            queries += 1;
            closed += adjacent(row_ptr, col, col[row_ptr[lo] + a], col[row_ptr[lo] + b]);
        } else {
            const int64_t q = r - L;
            const int32_t h = hlist[q / m];
            int32_t v, w;
            upper_edge(n, row_ptr, col, upre, q % m, &v, &w);
            if (h == v || h == w) continue;
            queries += 2;
            closed += adjacent(row_ptr, col, h, v) && adjacent(row_ptr, col, h, w);
        }
    }
    out[0] = s1;
    out[1] = nc;
    out[2] = nh;
    out[3] = L;
    out[4] = size;
    out[5] = queries;
    out[6] = closed;
    out[7] = m;
    free(upre); free(lpre); free(cand); free(hlist);
    return 0;
}

/* |U| closed / (3 s) */
double or_stream_value(int64_t size, int64_t closed, int64_t s) {
    volatile double num = (double)size * (double)closed;
    volatile double den = 3.0 * (double)s;
    return num / den;
}
