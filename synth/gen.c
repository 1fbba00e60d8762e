/*
 * Seeded synthetic graph generators (host C, single thread).
 *
 * This module produces raw edge lists only: (src, dst) int32 pairs that may
 * contain duplicates and self-loops.  It holds none of the triangle-counting
 * method's arithmetic; both the oracle and the device path consume its output.
 *
 * Random numbers come from PCG32 (M. E. O'Neill, "PCG: A Family of Simple Fast
 * Space-Efficient Statistically Good Algorithms for Random Number Generation",
 * 2014), written here from that published definition: an LCG over 64-bit state
 * with multiplier 6364136223846793005 and an XSH-RR output permutation.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

typedef struct { uint64_t state, inc; } pcg32;

static uint32_t pcg32_next(pcg32* g) {
    uint64_t old = g->state;
    g->state = old * 6364136223846793005ULL + g->inc;
    uint32_t xs = (uint32_t)(((old >> 18u) ^ old) >> 27u);
    uint32_t rot = (uint32_t)(old >> 59u);
    return (xs >> rot) | (xs << ((32u - rot) & 31u));
}

static void pcg32_seed(pcg32* g, uint64_t seed, uint64_t stream) {
    g->state = 0u;
    g->inc = (stream << 1u) | 1u;
    pcg32_next(g);
    g->state += seed;
    pcg32_next(g);
}

/* uniform double in [0,1) with 53 random bits */
static double pcg32_unit(pcg32* g) {
    uint64_t hi = pcg32_next(g) >> 5;   /* 27 bits */
    uint64_t lo = pcg32_next(g) >> 6;   /* 26 bits */
    return (double)((hi << 26) | lo) * (1.0 / 9007199254740992.0);
}

/* uniform integer in [0, bound) by Lemire's multiply-and-reject method */
static uint32_t pcg32_below(pcg32* g, uint32_t bound) {
    uint64_t m = (uint64_t)pcg32_next(g) * bound;
    uint32_t l = (uint32_t)m;
    if (l < bound) {
        uint32_t t = (uint32_t)(-bound) % bound;
        while (l < t) {
            m = (uint64_t)pcg32_next(g) * bound;
            l = (uint32_t)m;
        }
    }
    return (uint32_t)(m >> 32);
}

/* Fisher-Yates permutation of [0,n) */
static void random_permutation(int32_t* perm, int64_t n, pcg32* g) {
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)pcg32_below(g, (uint32_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each of num_edges pairs descends
 * `scale` levels of the adjacency matrix, choosing quadrant (0,0),(0,1),(1,0),(1,1)
 * with probabilities a, b, c, d=1-a-b-c.  Each level draws 16 random bits and
 * compares them with the cumulative thresholds rounded to 1/65536; no noise is
 * added.  If `permute`, a seeded random relabelling of the 2^scale vertices is
 * applied afterwards.
 */
int synth_rmat(int32_t scale, int64_t num_edges, double a, double b, double c,
               uint64_t seed, int32_t permute, int32_t* src, int32_t* dst) {
    if (scale < 1 || scale > 30 || num_edges < 0) return 1;
    uint32_t t0 = (uint32_t)lround(a * 65536.0);
    uint32_t t1 = (uint32_t)lround((a + b) * 65536.0);
    uint32_t t2 = (uint32_t)lround((a + b + c) * 65536.0);
    pcg32 g;
    pcg32_seed(&g, seed, 0x524d4154ULL);  /* stream "RMAT" */
    for (int64_t e = 0; e < num_edges; ++e) {
        uint32_t u = 0, v = 0, bits = 0;
        for (int32_t lvl = 0; lvl < scale; ++lvl) {
            if ((lvl & 1) == 0) bits = pcg32_next(&g);
            uint32_t r = (bits >> ((lvl & 1) * 16)) & 0xffffu;
            /* quadrant (0,0) if r < t0, (0,1) if r < t1, (1,0) if r < t2, else (1,1) */
            uint32_t ge0 = r >= t0, ge1 = r >= t1, ge2 = r >= t2;
            u = (u << 1) | ge1;
            v = (v << 1) | (ge0 ^ ge1 ^ ge2);
        }
        src[e] = (int32_t)u;
        dst[e] = (int32_t)v;
    }
    if (permute) {
        int64_t n = (int64_t)1 << scale;
        int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        if (!perm) return 2;
        pcg32 gp;
        pcg32_seed(&gp, seed, 0x5045524dULL);  /* stream "PERM" */
        random_permutation(perm, n, &gp);
        for (int64_t e = 0; e < num_edges; ++e) {
            src[e] = perm[src[e]];
            dst[e] = perm[dst[e]];
        }
        free(perm);
    }
    return 0;
}

/* Chung-Lu weights w_i = C * i^(-1/(beta-1)), i = 1..n, scaled so sum w = n * avg_deg. */
static void chung_lu_weights(int64_t n, double avg_deg, double beta, double* w, double* total) {
    double expo = -1.0 / (beta - 1.0);
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) { w[i] = pow((double)(i + 1), expo); s += w[i]; }
    double cst = (double)n * avg_deg / s;
    double t = 0.0;
    for (int64_t i = 0; i < n; ++i) { w[i] *= cst; t += w[i]; }
    *total = t;
}

/*
 * Chung-Lu (Chung & Lu 2002) with edge probability min(1, w_i w_j / S) for i < j.
 * mode 0: one independent coin per pair (O(n^2), for small n).
 * mode 1: the skipping method of Miller & Hagberg ("Efficient generation of
 *         networks with given expected degrees", WAW 2011), O(n + m) expected.
 * Output: up to max_edges pairs; *num_edges receives the count (returns 3 if
 * max_edges is too small).  If `permute`, vertex labels are randomly relabelled.
 */
int synth_chung_lu(int64_t n, double avg_deg, double beta, uint64_t seed, int32_t mode,
                   int32_t permute, int64_t max_edges, int32_t* src, int32_t* dst,
                   int64_t* num_edges) {
    if (n < 2 || beta <= 1.0 || avg_deg <= 0.0) return 1;
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    if (!w) return 2;
    double S;
    chung_lu_weights(n, avg_deg, beta, w, &S);
    pcg32 g;
    pcg32_seed(&g, seed, 0x43484c55ULL);  /* stream "CHLU" */
    int64_t cnt = 0;
    int rc = 0;
    if (mode == 0) {
        for (int64_t i = 0; i < n && !rc; ++i) {
            for (int64_t j = i + 1; j < n; ++j) {
                double pij = w[i] * w[j] / S;
                if (pij > 1.0) pij = 1.0;
                if (pcg32_unit(&g) < pij) {
                    if (cnt >= max_edges) { rc = 3; break; }
                    src[cnt] = (int32_t)i; dst[cnt] = (int32_t)j; ++cnt;
                }
            }
        }
    } else {
        for (int64_t u = 0; u < n - 1 && !rc; ++u) {
            int64_t v = u + 1;
            double p = w[u] * w[v] / S;
            if (p > 1.0) p = 1.0;
            while (v < n && p > 0.0) {
                if (p != 1.0) {
                    double r = pcg32_unit(&g);
                    if (r <= 0.0) r = 1e-300;
                    double skip = floor(log(r) / log1p(-p));
                    if (skip > (double)(n - v)) skip = (double)(n - v);
                    v += (int64_t)skip;
                }
                if (v < n) {
                    double q = w[u] * w[v] / S;
                    if (q > 1.0) q = 1.0;
                    if (pcg32_unit(&g) < q / p) {
                        if (cnt >= max_edges) { rc = 3; break; }
                        src[cnt] = (int32_t)u; dst[cnt] = (int32_t)v; ++cnt;
                    }
                    p = q;
                    v += 1;
                }
            }
        }
    }
    if (!rc && permute) {
        int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        if (!perm) { free(w); return 2; }
        pcg32 gp;
        pcg32_seed(&gp, seed, 0x5045524dULL);
        random_permutation(perm, n, &gp);
        for (int64_t e = 0; e < cnt; ++e) { src[e] = perm[src[e]]; dst[e] = perm[dst[e]]; }
        free(perm);
    }
    *num_edges = cnt;
    free(w);
    return rc;
}

/* Uniform random pairs over [0,n) (Erdos-Renyi style multigraph input, for tests). */
int synth_uniform_pairs(int64_t n, int64_t num_pairs, uint64_t seed, int32_t* src, int32_t* dst) {
    if (n < 1 || n > 0x7fffffffLL) return 1;
    pcg32 g;
    pcg32_seed(&g, seed, 0x554e4946ULL);  /* "UNIF" */
    for (int64_t e = 0; e < num_pairs; ++e) {
        src[e] = (int32_t)pcg32_below(&g, (uint32_t)n);
        dst[e] = (int32_t)pcg32_below(&g, (uint32_t)n);
    }
    return 0;
}

/* Poisson arrival times (exponential gaps with rate lam), and uniform integer draws, for request traces. */
int synth_poisson_arrivals(int64_t count, double lam, uint64_t seed, double* t_out) {
    if (lam <= 0.0) return 1;
    pcg32 g;
    pcg32_seed(&g, seed, 0x504f4953ULL);  /* "POIS" */
    double t = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        double u = pcg32_unit(&g);
        t += -log1p(-u) / lam;
        t_out[i] = t;
    }
    return 0;
}

int synth_uniform_ints(int64_t count, uint32_t bound, uint64_t seed, uint32_t stream, int32_t* out) {
    if (bound == 0) return 1;
    pcg32 g;
    pcg32_seed(&g, seed, stream);
    for (int64_t i = 0; i < count; ++i) out[i] = (int32_t)pcg32_below(&g, bound);
    return 0;
}
