/*
 * gen.c -- seeded synthetic tree generators.
 *
 * These produce the inputs that BOTH the CPU oracle and the GPU library are
 * run on.  They hold none of the dendrogram method's arithmetic: they only
 * draw tree shapes and edge weights.  The paper measures on real datasets
 * (Table 2) that are not available here; these shapes stand in for them and
 * span the same range of dendrogram skew.
 *
 * Random numbers: xoshiro256** (Blackman & Vigna, 2018) seeded through
 * splitmix64 (Steele, Lea & Flood, 2014), both public-domain published
 * generators, written here from their definitions.  Every generator takes a
 * 64-bit seed; the tree structure and the weights use two independent
 * streams so a shape can be re-weighted without changing it.
 *
 * Edge i of every generated tree is listed in generation order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct { uint64_t s[4]; } gen_rng;

static uint64_t gen_splitmix64(uint64_t* x)
{
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t gen_rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t gen_next(gen_rng* r)
{
    const uint64_t result = gen_rotl(r->s[1] * 5, 7) * 9;
    const uint64_t t = r->s[1] << 17;
    r->s[2] ^= r->s[0];
    r->s[3] ^= r->s[1];
    r->s[1] ^= r->s[2];
    r->s[0] ^= r->s[3];
    r->s[2] ^= t;
    r->s[3] = gen_rotl(r->s[3], 45);
    return result;
}

/* stream 0: tree structure; stream 1: weights; stream 2+: anything else. */
static void gen_seed(gen_rng* r, uint64_t seed, uint64_t stream)
{
    uint64_t x = seed ^ (stream * 0xD1B54A32D192ED03ull);
    for (int i = 0; i < 4; ++i) r->s[i] = gen_splitmix64(&x);
}

/* uniform double in [0, 1) with 53 random bits */
static double gen_u01(gen_rng* r) { return (double)(gen_next(r) >> 11) * 0x1.0p-53; }

/* uniform fp32 in [0, 1): the top 24 bits of a draw times 2^-24 (exact) */
static float gen_u01f(gen_rng* r) { return (float)((double)(gen_next(r) >> 40) * 0x1.0p-24); }

/* standard normal by Box-Muller in double, cosine branch only (2 draws) */
static double gen_normal(gen_rng* r)
{
    const double u1 = 1.0 - gen_u01(r);   /* (0, 1] */
    const double u2 = gen_u01(r);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

/* ---- weight laws ------------------------------------------------------ */

/* fp32 uniform [0,1) */
void gen_weights_uniform(int64_t m, uint64_t seed, float* w)
{
    gen_rng r; gen_seed(&r, seed, 1);
    for (int64_t i = 0; i < m; ++i) w[i] = gen_u01f(&r);
}

/* fp32(exp(N(mu, sigma))); then each edge independently, with probability
 * bridge_p, is multiplied by bridge_mul in fp32 (long inter-cluster bridges). */
void gen_weights_lognormal(int64_t m, uint64_t seed, double mu, double sigma,
                           double bridge_p, float bridge_mul, float* w)
{
    gen_rng r; gen_seed(&r, seed, 1);
    for (int64_t i = 0; i < m; ++i) w[i] = (float)exp(mu + sigma * gen_normal(&r));
    if (bridge_p > 0.0) {
        gen_rng b; gen_seed(&b, seed, 2);
        for (int64_t i = 0; i < m; ++i)
            if (gen_u01(&b) < bridge_p) w[i] = w[i] * bridge_mul;
    }
}

/* ---- shapes (u, v of n-1 edges) --------------------------------------- */

/* Random recursive tree: vertex i > 0 attaches to a uniform j < i.
 * Edge i-1 = (i, j). */
void gen_rrt(int64_t n, uint64_t seed, int32_t* u, int32_t* v)
{
    gen_rng r; gen_seed(&r, seed, 0);
    for (int64_t i = 1; i < n; ++i) {
        int64_t j = (int64_t)(gen_u01(&r) * (double)i);
        if (j >= i) j = i - 1;
        u[i - 1] = (int32_t)i;
        v[i - 1] = (int32_t)j;
    }
}

/* Preferential attachment: vertex i > 0 attaches to j < i with probability
 * proportional to deg(j) + 1.  The total weight over j < i is 3i - 2, so with
 * probability i / (3i - 2) pick a uniform vertex, otherwise a uniform entry of
 * the list of edge endpoints (each vertex appears deg(j) times there).
 * scratch must hold 2*(n-1) int32. Edge i-1 = (i, j). */
void gen_pref_attach(int64_t n, uint64_t seed, int32_t* u, int32_t* v, int32_t* scratch)
{
    gen_rng r; gen_seed(&r, seed, 0);
    int64_t ends = 0;
    for (int64_t i = 1; i < n; ++i) {
        const double coin = gen_u01(&r);
        const double pick = gen_u01(&r);
        int64_t j;
        if (coin * (double)(3 * i - 2) < (double)i) {
            j = (int64_t)(pick * (double)i);
            if (j >= i) j = i - 1;
        } else {
            int64_t k = (int64_t)(pick * (double)ends);
            if (k >= ends) k = ends - 1;
            j = scratch[k];
        }
        u[i - 1] = (int32_t)i;
        v[i - 1] = (int32_t)j;
        scratch[ends++] = (int32_t)i;
        scratch[ends++] = (int32_t)j;
    }
}

/* Caterpillar: a path (spine) of S vertices 0..S-1 and n-S leaves hung at
 * uniform spine positions.  Weights: spine edge k = (k, k+1) has
 * fp32(k/(S-1)) + fp32(U*noise); a leaf at spine position s has
 * fp32(s/(S-1)) + fp32(U*noise).  Spine edges are listed first. */
void gen_caterpillar(int64_t n, int64_t S, double noise, uint64_t seed,
                     int32_t* u, int32_t* v, float* w)
{
    gen_rng r; gen_seed(&r, seed, 0);
    gen_rng q; gen_seed(&q, seed, 1);
    if (S < 1) S = 1;
    if (S > n) S = n;
    const double den = S > 1 ? (double)(S - 1) : 1.0;
    int64_t e = 0;
    for (int64_t k = 0; k + 1 < S; ++k, ++e) {
        u[e] = (int32_t)k;
        v[e] = (int32_t)(k + 1);
        w[e] = (float)((double)k / den) + (float)(gen_u01(&q) * noise);
    }
    for (int64_t x = S; x < n; ++x, ++e) {
        int64_t s = (int64_t)(gen_u01(&r) * (double)S);
        if (s >= S) s = S - 1;
        u[e] = (int32_t)x;
        v[e] = (int32_t)s;
        w[e] = (float)((double)s / den) + (float)(gen_u01(&q) * noise);
    }
}

/* Path 0-1-2-...-(n-1); edge k = (k, k+1).  Weights are left to the caller. */
void gen_path(int64_t n, int32_t* u, int32_t* v)
{
    for (int64_t k = 0; k + 1 < n; ++k) { u[k] = (int32_t)k; v[k] = (int32_t)(k + 1); }
}

/* Star around vertex 0; edge i-1 = (i, 0). */
void gen_star(int64_t n, int32_t* u, int32_t* v)
{
    for (int64_t i = 1; i < n; ++i) { u[i - 1] = (int32_t)i; v[i - 1] = 0; }
}

/* Relabel vertices by a random permutation, shuffle the edge list and flip
 * each edge's orientation at random (Fisher-Yates).  Keeps the same tree. */
void gen_shuffle(int64_t n, uint64_t seed, int32_t* u, int32_t* v, float* w, int32_t* scratch)
{
    gen_rng r; gen_seed(&r, seed, 3);
    const int64_t m = n - 1;
    int32_t* perm = scratch; /* n entries */
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)(gen_u01(&r) * (double)(i + 1));
        if (j > i) j = i;
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    for (int64_t e = 0; e < m; ++e) { u[e] = perm[u[e]]; v[e] = perm[v[e]]; }
    for (int64_t e = m - 1; e > 0; --e) {
        int64_t j = (int64_t)(gen_u01(&r) * (double)(e + 1));
        if (j > e) j = e;
        int32_t tu = u[e]; u[e] = u[j]; u[j] = tu;
        int32_t tv = v[e]; v[e] = v[j]; v[j] = tv;
        float tw = w[e]; w[e] = w[j]; w[j] = tw;
    }
    for (int64_t e = 0; e < m; ++e) {
        if (gen_next(&r) >> 63) { int32_t t = u[e]; u[e] = v[e]; v[e] = t; }
    }
}

/* Raw draws for size distributions and arrival processes (Python side). */
void gen_uniform_f64(int64_t k, uint64_t seed, uint64_t stream, double* out)
{
    gen_rng r; gen_seed(&r, seed, stream);
    for (int64_t i = 0; i < k; ++i) out[i] = gen_u01(&r);
}

void gen_normal_f64(int64_t k, uint64_t seed, uint64_t stream, double* out)
{
    gen_rng r; gen_seed(&r, seed, stream);
    for (int64_t i = 0; i < k; ++i) out[i] = gen_normal(&r);
}

/* splitmix64 of (a, b): derives per-tree seeds in batched workloads. */
uint64_t gen_hash2(uint64_t a, uint64_t b)
{
    uint64_t x = a ^ gen_rotl(b, 32) ^ 0x632BE59BD9B4E019ull;
    gen_splitmix64(&x);
    return gen_splitmix64(&x);
}
