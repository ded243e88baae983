/*
 * Seeded synthetic preference profiles (ballots) for the Schulze method.
 *
 * This module only draws ballots.  It holds none of the method's arithmetic
 * (no pairwise counts, no widest paths): both the CPU oracle and the GPU
 * library receive the bytes it writes as plain input.
 *
 * Ballot format: n rows of L candidate ids, best first.  A row may end early;
 * the remaining entries are padding (0xFFFF for uint16 rows, -1 for int32
 * rows) and every candidate not listed is unranked, i.e. tied below all
 * ranked ones.  A preference profile of weak orders is exactly what the
 * paper's voting preliminaries take as input (Section 2.1).
 *
 * Randomness: every voter v of election e owns an independent stream of
 * SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) whose state starts at a hash of (seed, e, v).
 * Results therefore do not depend on the number of OpenMP threads.
 *
 * Models:
 *  - Mallows via the Repeated Insertion Model: item i (1-based, in reference
 *    order) is inserted at position j <= i with probability proportional to
 *    phi^(i-j).  The final permutation is recovered with a Fenwick tree: the
 *    item inserted last keeps its slot, and each earlier item takes the j-th
 *    free slot that later items left.
 *  - Plackett-Luce with Zipf weights: the candidate of popularity rank r
 *    (1-based) has weight r^-s; the top-k is drawn one place at a time with
 *    probability proportional to weight among the candidates not yet drawn
 *    (rejection of repeats from the full distribution, which is exact).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GEN_OK 0
#define GEN_EINVAL -1
#define GEN_ENOMEM -3

static inline uint64_t sm64_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Stream key for (seed, election, voter): three rounds of the SplitMix64
 * finaliser over the words, so neighbouring voters get unrelated streams. */
static inline uint64_t stream_key(uint64_t seed, uint64_t e, uint64_t v) {
    uint64_t s = seed ^ 0x5DEECE66Dull;
    uint64_t k = sm64_next(&s);
    s = k ^ (e * 0xD1B54A32D192ED03ull);
    k = sm64_next(&s);
    s = k ^ (v * 0x8CB92BA72F3D8DD7ull);
    return sm64_next(&s);
}

/* Uniform double in [0,1) with 53 random bits. */
static inline double u01(uint64_t *s) { return (double)(sm64_next(s) >> 11) * 0x1.0p-53; }

/* Uniform integer in [0, bound) by Lemire's multiply-shift with rejection. */
static inline uint64_t below(uint64_t *s, uint64_t bound) {
    for (;;) {
        uint64_t x = sm64_next(s);
        __uint128_t mm = (__uint128_t)x * bound;
        uint64_t lo = (uint64_t)mm;
        if (lo >= bound || lo >= (-bound) % bound) return (uint64_t)(mm >> 64);
    }
}

/* Seeded uniform permutation of 0..m-1 (Fisher-Yates). */
int gen_permutation(uint64_t seed, uint64_t stream, int32_t m, int32_t *perm) {
    if (m < 0 || (m > 0 && !perm)) return GEN_EINVAL;
    uint64_t s = stream_key(seed, 0xFFFFFFFFull, stream);
    for (int32_t i = 0; i < m; ++i) perm[i] = i;
    for (int32_t i = m - 1; i > 0; --i) {
        int32_t j = (int32_t)below(&s, (uint64_t)i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    return GEN_OK;
}

/* Draw k in {0..i-1} with P(k) proportional to phi^k (truncated geometric),
 * by inverting its distribution function.  tail = phi^i and log_phi =
 * log(phi) are passed in so that callers can compute them once. */
static inline int32_t trunc_geom_t(uint64_t *s, double phi, int32_t i, double tail, double log_phi) {
    double u = u01(s);
    if (phi >= 1.0) return (int32_t)(u * (double)i);
    if (phi <= 0.0) return 0;
    double k = floor(log1p(-u * (1.0 - tail)) / log_phi);
    if (k < 0) k = 0;
    if (k > (double)(i - 1)) k = (double)(i - 1);
    return (int32_t)k;
}

static inline int32_t trunc_geom(uint64_t *s, double phi, int32_t i) {
    if (phi >= 1.0 || phi <= 0.0) return trunc_geom_t(s, phi, i, 0.0, 0.0);
    return trunc_geom_t(s, phi, i, pow(phi, (double)i), log(phi));
}

static void store_id(void *out, int dtype32, int64_t idx, int32_t id) {
    if (dtype32) ((int32_t *)out)[idx] = id;
    else ((uint16_t *)out)[idx] = (uint16_t)id;
}

static void store_pad(void *out, int dtype32, int64_t idx) {
    if (dtype32) ((int32_t *)out)[idx] = -1;
    else ((uint16_t *)out)[idx] = 0xFFFF;
}

/* One Mallows ranking of m items around ref_order, written as ids best first.
 * scratch: m int32 (Fenwick tree) + m int32 (insertion offsets). */
static void mallows_one(uint64_t *s, int32_t m, double phi, const int32_t *ref_order, const double *tails,
                        double log_phi, int32_t *fen, int32_t *jpos, int32_t *out_ids) {
    /* insertion positions, 1-based: item i goes to slot j_i = i - k_i */
    for (int32_t i = 1; i <= m; ++i) jpos[i - 1] = i - trunc_geom_t(s, phi, i, tails[i - 1], log_phi);
    /* Fenwick tree over m free slots (all ones) */
    for (int32_t i = 1; i <= m; ++i) fen[i - 1] = 0;
    for (int32_t i = 1; i <= m; ++i) {
        fen[i - 1] += 1;
        int32_t p = i + (i & -i);
        if (p <= m) fen[p - 1] += fen[i - 1];
    }
    int32_t top = 1;
    while ((top << 1) <= m) top <<= 1;
    for (int32_t i = m; i >= 1; --i) {
        /* find the jpos[i-1]-th free slot */
        int32_t want = jpos[i - 1], pos = 0;
        for (int32_t step = top; step; step >>= 1) {
            int32_t nxt = pos + step;
            if (nxt <= m && fen[nxt - 1] < want) { pos = nxt; want -= fen[nxt - 1]; }
        }
        int32_t slot = pos + 1; /* 1-based */
        for (int32_t q = slot; q <= m; q += q & -q) fen[q - 1] -= 1;
        out_ids[slot - 1] = ref_order[i - 1];
    }
}

/*
 * Mallows profile.  Voter v (0 <= v < n) of election `election` gets a full
 * ranking; if (v % trunc_mod) < trunc_lt it is cut to its top trunc_k entries.
 * Output: n x L ids (L >= m for full rows; L >= trunc_k otherwise), padded.
 */
int gen_mallows(uint64_t seed, uint64_t election, int64_t n, int32_t m, double phi,
                const int32_t *ref_order, int32_t L, int32_t trunc_mod, int32_t trunc_lt,
                int32_t trunc_k, int dtype32, void *out) {
    if (n < 0 || m < 1 || L < 1 || !ref_order || !out) return GEN_EINVAL;
    if (!dtype32 && m > 65535) return GEN_EINVAL;
    int any_full = trunc_mod <= 0 || trunc_lt < trunc_mod;
    if (any_full && L < m) return GEN_EINVAL;
    if (trunc_mod > 0 && trunc_lt > 0 && (trunc_k < 0 || trunc_k > L)) return GEN_EINVAL;
    int err = GEN_OK;
    /* phi^i for i = 1..m and log(phi), shared by every voter */
    double *tails = (double *)malloc(sizeof(double) * (size_t)m);
    if (!tails) return GEN_ENOMEM;
    const double log_phi = (phi > 0.0 && phi < 1.0) ? log(phi) : 0.0;
    for (int32_t i = 1; i <= m; ++i) tails[i - 1] = (phi > 0.0 && phi < 1.0) ? pow(phi, (double)i) : 0.0;
#pragma omp parallel
    {
        int32_t *scr = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * 3);
        if (!scr) {
#pragma omp atomic write
            err = GEN_ENOMEM;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; ++v) {
            if (!scr) continue;
            uint64_t s = stream_key(seed, election, (uint64_t)v);
            mallows_one(&s, m, phi, ref_order, tails, log_phi, scr, scr + m, scr + 2 * (size_t)m);
            int32_t keep = m;
            if (trunc_mod > 0 && (v % trunc_mod) < trunc_lt) keep = trunc_k;
            int64_t base = v * (int64_t)L;
            for (int32_t t = 0; t < L; ++t) {
                if (t < keep) store_id(out, dtype32, base + t, scr[2 * (size_t)m + t]);
                else store_pad(out, dtype32, base + t);
            }
        }
        free(scr);
    }
    free(tails);
    return err;
}

/*
 * Plackett-Luce profile with Zipf(s) weights over popularity order pop_order
 * (pop_order[r] = candidate of popularity rank r+1).  Every voter ranks its
 * top k (k <= m) and leaves the rest unranked.  Output: n x L ids, L >= k.
 */
int gen_pl_zipf(uint64_t seed, uint64_t election, int64_t n, int32_t m, double s_exp,
                const int32_t *pop_order, int32_t k, int32_t L, int dtype32, void *out) {
    if (n < 0 || m < 1 || k < 0 || k > m || L < k || L < 1 || !pop_order || !out) return GEN_EINVAL;
    if (!dtype32 && m > 65535) return GEN_EINVAL;
    double *cum = (double *)malloc(sizeof(double) * (size_t)m);
    if (!cum) return GEN_ENOMEM;
    double acc = 0.0;
    for (int32_t r = 0; r < m; ++r) { acc += pow((double)(r + 1), -s_exp); cum[r] = acc; }
    const double total = acc;
#pragma omp parallel
    {
        int32_t chosen[4096];
        int32_t *pick = k <= 4096 ? chosen : (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
#pragma omp for schedule(dynamic, 256)
        for (int64_t v = 0; v < n; ++v) {
            uint64_t st = stream_key(seed, election, (uint64_t)v);
            int32_t got = 0;
            while (got < k) {
                double u = u01(&st) * total;
                /* first r with cum[r] > u */
                int32_t lo = 0, hi = m - 1;
                while (lo < hi) {
                    int32_t mid = lo + ((hi - lo) >> 1);
                    if (cum[mid] > u) hi = mid; else lo = mid + 1;
                }
                int dup = 0;
                for (int32_t t = 0; t < got; ++t) if (pick[t] == lo) { dup = 1; break; }
                if (!dup) pick[got++] = lo;
            }
            int64_t base = v * (int64_t)L;
            for (int32_t t = 0; t < L; ++t) {
                if (t < k) store_id(out, dtype32, base + t, pop_order[pick[t]]);
                else store_pad(out, dtype32, base + t);
            }
        }
        if (pick != chosen) free(pick);
    }
    free(cum);
    return GEN_OK;
}

/*
 * Top-k of a Mallows(phi) ranking around ref_order, by the inversion-vector
 * form of the model: the t-th ranked item is the (V_t)-th item (0-based) of
 * the reference order not yet chosen, with V_t independent and
 * P(V_t = v) proportional to phi^v for v in {0 .. m-t} (the same
 * distribution as the repeated insertion model, truncated after k places).
 * Output: n x L ids, L >= k, padded.
 */
int gen_mallows_topk(uint64_t seed, uint64_t election, int64_t n, int32_t m, double phi,
                     const int32_t *ref_order, int32_t k, int32_t L, int dtype32, void *out) {
    if (n < 0 || m < 1 || k < 0 || k > m || L < k || L < 1 || !ref_order || !out) return GEN_EINVAL;
    if (!dtype32 && m > 65535) return GEN_EINVAL;
#pragma omp parallel
    {
        int32_t taken[4096];
        int32_t *tk = k <= 4096 ? taken : (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
#pragma omp for schedule(dynamic, 256)
        for (int64_t v = 0; v < n; ++v) {
            uint64_t st = stream_key(seed, election, (uint64_t)v);
            int32_t nt = 0;  /* sorted reference positions already chosen */
            int64_t base = v * (int64_t)L;
            for (int32_t t = 0; t < k; ++t) {
                int32_t remaining = m - t;
                int32_t want = trunc_geom(&st, phi, remaining);  /* 0-based among remaining */
                /* the want-th unchosen reference position */
                int32_t pos = want, i = 0;
                while (i < nt && tk[i] <= pos) { ++pos; ++i; }
                /* insert pos into the sorted list */
                int32_t j = nt++;
                while (j > 0 && tk[j - 1] > pos) { tk[j] = tk[j - 1]; --j; }
                tk[j] = pos;
                store_id(out, dtype32, base + t, ref_order[pos]);
            }
            for (int32_t t = k; t < L; ++t) store_pad(out, dtype32, base + t);
        }
        if (tk != taken) free(tk);
    }
    return GEN_OK;
}

/* Uniform integers in [lo, hi] for per-election parameters (batch workloads). */
int gen_uniform_int(uint64_t seed, uint64_t stream, int64_t count, int64_t lo, int64_t hi, int64_t *out) {
    if (count < 0 || hi < lo || (count > 0 && !out)) return GEN_EINVAL;
    uint64_t s = stream_key(seed, 0xFFFFFFFEull, stream);
    for (int64_t i = 0; i < count; ++i) out[i] = lo + (int64_t)below(&s, (uint64_t)(hi - lo) + 1);
    return GEN_OK;
}

/* Uniform doubles in [lo, hi) for per-election parameters. */
int gen_uniform_real(uint64_t seed, uint64_t stream, int64_t count, double lo, double hi, double *out) {
    if (count < 0 || (count > 0 && !out)) return GEN_EINVAL;
    uint64_t s = stream_key(seed, 0xFFFFFFFDull, stream);
    for (int64_t i = 0; i < count; ++i) out[i] = lo + (hi - lo) * u01(&s);
    return GEN_OK;
}

/* Uniform integer ballots of a random length in [0, L] with random distinct ids:
 * an unstructured profile for edge-case tests (many ties, short lists). */
int gen_uniform_ballots(uint64_t seed, uint64_t election, int64_t n, int32_t m, int32_t L,
                        int32_t min_len, int dtype32, void *out) {
    if (n < 0 || m < 1 || L < 1 || L > m || min_len < 0 || min_len > L || !out) return GEN_EINVAL;
    if (!dtype32 && m > 65535) return GEN_EINVAL;
    int err = GEN_OK;
#pragma omp parallel
    {
        int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
        if (!perm) {
#pragma omp atomic write
            err = GEN_ENOMEM;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; ++v) {
            if (!perm) continue;
            uint64_t s = stream_key(seed, election, (uint64_t)v);
            int32_t len = min_len + (int32_t)below(&s, (uint64_t)(L - min_len) + 1);
            for (int32_t i = 0; i < m; ++i) perm[i] = i;
            for (int32_t i = 0; i < len; ++i) {
                int32_t j = i + (int32_t)below(&s, (uint64_t)(m - i));
                int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
            }
            int64_t base = v * (int64_t)L;
            for (int32_t t = 0; t < L; ++t) {
                if (t < len) store_id(out, dtype32, base + t, perm[t]);
                else store_pad(out, dtype32, base + t);
            }
        }
        free(perm);
    }
    return err;
}
