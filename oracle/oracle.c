/*
 * CPU oracle for the Schulze method's hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the GPU library.
 *
 * Every function here is the plain definition written out in 64-bit
 * integers, following the paper's voting preliminaries (Section 2.1):
 *
 *   oracle_pairwise   d[x][y] = total weight of voters with x strictly
 *                     preferred to y (weak orders; unranked candidates are
 *                     tied below all ranked ones).
 *   oracle_weights    edge weights of the weighted tournament graph: the
 *                     majority margin mu(x,y) = d[x][y] - d[y][x] where it is
 *                     positive (Section 2.1), or the winning-votes weight
 *                     d[x][y] where d[x][y] > d[y][x]; 0 means "no edge".
 *   oracle_closure    p(a,b) = width of a widest a->b path, width = smallest
 *                     edge weight on the path; computed by the classical
 *                     Floyd-Warshall recurrence over the (max,min) pair that
 *                     Section 5.2 names as the original sequential algorithm.
 *   oracle_rank       a beats b iff p(a,b) > p(b,a); winners are the
 *                     candidates nobody beats; ranking by (number of
 *                     candidates that beat x, id).
 *   oracle_widest_from / oracle_widest_to
 *                     single-source / single-target widest paths by the
 *                     textbook dense Dijkstra for bottleneck paths (the
 *                     path problems WP>= / WP> of the NL-membership proof,
 *                     Section 3).
 *
 * Candidate ids are 0..m-1.  Error codes: 0 ok, -1 bad argument, -3 out of
 * memory, -5 invalid ballot (id out of range or listed twice).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -3
#define ORC_EBALLOT -5

/* Read entry t of ballot row v; returns -1 for padding. */
static inline int64_t ballot_at(const void *ballots, int dtype32, int64_t L, int64_t v, int64_t t) {
    if (dtype32) {
        int32_t x = ((const int32_t *)ballots)[v * L + t];
        return x < 0 ? -1 : (int64_t)x;
    }
    uint16_t x = ((const uint16_t *)ballots)[v * L + t];
    return x == 0xFFFF ? -1 : (int64_t)x;
}

/*
 * Ranks of ballot v: rank[c] = place of c in the list (0 = best) for listed
 * candidates; every other entry of rank must hold m (unranked, tied below
 * all listed ones) on entry.  The listed part is the prefix before the first
 * padding entry.  Returns its length k, or -1 (with rank restored to all m)
 * if an id is out of range or repeated.
 */
static int64_t ballot_fill(const void *ballots, int dtype32, int64_t L, int64_t m, int64_t v,
                           int32_t *rank) {
    int64_t k = 0;
    for (int64_t t = 0; t < L; ++t) {
        int64_t c = ballot_at(ballots, dtype32, L, v, t);
        if (c < 0) break;
        if (c >= m || rank[c] != m) {
            for (int64_t u = 0; u < k; ++u) rank[ballot_at(ballots, dtype32, L, v, u)] = (int32_t)m;
            return -1;
        }
        rank[c] = (int32_t)t;
        ++k;
    }
    return k;
}

/* Undo ballot_fill for a ballot whose listed prefix has length k. */
static void ballot_clear(const void *ballots, int dtype32, int64_t L, int64_t m, int64_t v, int64_t k,
                         int32_t *rank) {
    for (int64_t t = 0; t < k; ++t) rank[ballot_at(ballots, dtype32, L, v, t)] = (int32_t)m;
}

/* o[y] += w for every y ranked strictly below a candidate of rank rc. */
__attribute__((target_clones("avx2", "default")))
static void add_row(int64_t *restrict o, const int32_t *restrict rank, int32_t rc, int64_t w, int64_t m) {
    for (int64_t y = 0; y < m; ++y) o[y] += rank[y] > rc ? w : 0;
}

/*
 * Pairwise counts for a list of output lines.  For line r with candidate
 * c = lines[r] (or c = r when lines == NULL):
 *   as_rows != 0:  out[r*m + y] = d[c][y]   (row c of d)
 *   as_rows == 0:  out[r*m + x] = d[x][c]   (column c of d)
 * d[x][y] adds the weight of every voter who lists x and lists y later or
 * not at all.  Threads take groups of LINE_GROUP output lines and walk over
 * all ballots for each group (a loop order only: every output entry is the
 * same sum over voters, and no two threads write the same line).
 */
#define LINE_GROUP 32
static int pairwise_lines(const void *ballots, int dtype32, int64_t n, int64_t L, int64_t m,
                          const uint32_t *weight, const int32_t *lines, int64_t nlines, int as_rows,
                          int64_t *out) {
    int err = ORC_OK;
    memset(out, 0, sizeof(int64_t) * (size_t)(nlines * m));
#pragma omp parallel
    {
        int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
        if (!rank) {
#pragma omp atomic write
            err = ORC_ENOMEM;
        } else {
            for (int64_t c = 0; c < m; ++c) rank[c] = (int32_t)m;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t g = 0; g < (nlines + LINE_GROUP - 1) / LINE_GROUP; ++g) {
            if (!rank) continue;
            const int64_t r0 = g * LINE_GROUP;
            const int64_t r1 = r0 + LINE_GROUP < nlines ? r0 + LINE_GROUP : nlines;
            for (int64_t v = 0; v < n; ++v) {
                const int64_t k = ballot_fill(ballots, dtype32, L, m, v, rank);
                if (k < 0) {
#pragma omp atomic write
                    err = ORC_EBALLOT;
                    break;
                }
                const int64_t w = weight ? (int64_t)weight[v] : 1;
                for (int64_t r = r0; r < r1; ++r) {
                    const int64_t c = lines ? lines[r] : r;
                    const int32_t rc = rank[c];
                    int64_t *o = out + r * m;
                    if (as_rows) {
                        /* an unlisted candidate is preferred to nobody */
                        if (rc < m) add_row(o, rank, rc, w, m);
                    } else {
                        /* x is preferred to c iff x is listed before place rc
                         * (rc = m: c unlisted, so every listed x is) */
                        const int64_t upto = rc < k ? rc : k;
                        for (int64_t t = 0; t < upto; ++t) o[ballot_at(ballots, dtype32, L, v, t)] += w;
                    }
                }
                ballot_clear(ballots, dtype32, L, m, v, k, rank);
            }
        }
        free(rank);
    }
    return err;
}

int oracle_pairwise(const void *ballots, int dtype32, int64_t n, int32_t L, int32_t m,
                    const uint32_t *weight, int64_t *d) {
    if (!ballots || !d || n < 0 || L < 1 || m < 1) return ORC_EINVAL;
    return pairwise_lines(ballots, dtype32, n, L, m, weight, NULL, m, 1, d);
}

/* Rows x = rows[r] of d: out[r*m + y] = d[x][y]. */
int oracle_pairwise_rows(const void *ballots, int dtype32, int64_t n, int32_t L, int32_t m,
                         const uint32_t *weight, const int32_t *rows, int64_t nrows, int64_t *out) {
    if (!ballots || !out || !rows || n < 0 || L < 1 || m < 1 || nrows < 0) return ORC_EINVAL;
    for (int64_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= m) return ORC_EINVAL;
    return pairwise_lines(ballots, dtype32, n, L, m, weight, rows, nrows, 1, out);
}

/* Columns y = cols[c] of d: out[c*m + x] = d[x][y]. */
int oracle_pairwise_cols(const void *ballots, int dtype32, int64_t n, int32_t L, int32_t m,
                         const uint32_t *weight, const int32_t *cols, int64_t ncols, int64_t *out) {
    if (!ballots || !out || !cols || n < 0 || L < 1 || m < 1 || ncols < 0) return ORC_EINVAL;
    for (int64_t c = 0; c < ncols; ++c)
        if (cols[c] < 0 || cols[c] >= m) return ORC_EINVAL;
    return pairwise_lines(ballots, dtype32, n, L, m, weight, cols, ncols, 0, out);
}

/* mode 0: winning votes, w = d[x][y] if d[x][y] > d[y][x] else 0.
 * mode 1: majority margin, w = d[x][y] - d[y][x] if positive else 0. */
int oracle_weights(const int64_t *d, int32_t m, int mode, int64_t *w) {
    if (!d || !w || m < 1 || (mode != 0 && mode != 1)) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < m; ++x)
        for (int64_t y = 0; y < m; ++y) {
            int64_t a = d[x * m + y], b = d[y * m + x];
            int64_t e = 0;
            if (x != y && a > b) e = mode == 0 ? a : a - b;
            w[x * m + y] = e;
        }
    return ORC_OK;
}

/*
 * Widest-path closure: p starts as w, then for every intermediate vertex k,
 * p[i][j] = max(p[i][j], min(p[i][k], p[k][j])).  Row k does not change in
 * round k (min(p[k][k], p[k][j]) <= p[k][j]), so rows i != k are updated in
 * parallel.  The diagonal is set to 0 at the end (a widest path from a
 * vertex to itself is not part of the method).
 */
__attribute__((target_clones("avx2", "default")))
static void relax_row(int64_t *restrict pi, const int64_t *restrict pk, int64_t pik, int64_t m) {
    for (int64_t j = 0; j < m; ++j) {
        int64_t via = pik < pk[j] ? pik : pk[j];
        pi[j] = via > pi[j] ? via : pi[j];
    }
}

int oracle_closure(const int64_t *w, int32_t m, int64_t *p) {
    if (!w || !p || m < 1) return ORC_EINVAL;
    const int64_t M = m;
    memcpy(p, w, sizeof(int64_t) * (size_t)(M * M));
    for (int64_t k = 0; k < M; ++k) {
        const int64_t *pk = p + k * M;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < M; ++i) {
            if (i == k) continue;
            relax_row(p + i * M, pk, p[i * M + k], M);
        }
    }
    for (int64_t i = 0; i < M; ++i) p[i * M + i] = 0;
    return ORC_OK;
}

/*
 * beaten_by[x] = number of y with p[y][x] > p[x][y] (y beats x);
 * is_winner[x] = (beaten_by[x] == 0); order = candidates sorted by
 * (beaten_by, id).  Returns the number of winners, or an error code < 0.
 */
int oracle_rank(const int64_t *p, int32_t m, int32_t *beaten_by, uint8_t *is_winner, int32_t *order) {
    if (!p || m < 1 || !beaten_by) return ORC_EINVAL;
    const int64_t M = m;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < M; ++x) {
        int32_t c = 0;
        for (int64_t y = 0; y < M; ++y)
            if (y != x && p[y * M + x] > p[x * M + y]) ++c;
        beaten_by[x] = c;
    }
    int32_t nw = 0;
    for (int64_t x = 0; x < M; ++x) {
        if (is_winner) is_winner[x] = beaten_by[x] == 0;
        nw += beaten_by[x] == 0;
    }
    if (order) {
        /* stable counting sort by beaten_by (values 0..m-1), ids ascending */
        int64_t *start = (int64_t *)calloc((size_t)M + 1, sizeof(int64_t));
        if (!start) return ORC_ENOMEM;
        for (int64_t x = 0; x < M; ++x) start[beaten_by[x] + 1]++;
        for (int64_t l = 0; l < M; ++l) start[l + 1] += start[l];
        for (int64_t x = 0; x < M; ++x) order[start[beaten_by[x]]++] = (int32_t)x;
        free(start);
    }
    return nw;
}

/*
 * Single-source widest paths from s by dense Dijkstra: out[v] = p(s, v) for
 * v != s, out[s] = 0.  Bottleneck values only grow along settled vertices,
 * so the vertex of largest tentative width is final when it is taken.
 */
static int widest_dijkstra(const int64_t *w, int64_t m, int64_t s, int transpose, int64_t *out) {
    int64_t *best = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    uint8_t *done = (uint8_t *)calloc((size_t)m, 1);
    if (!best || !done) { free(best); free(done); return ORC_ENOMEM; }
    for (int64_t v = 0; v < m; ++v) best[v] = 0;
    best[s] = INT64_MAX;
    for (int64_t it = 0; it < m; ++it) {
        int64_t u = -1;
        for (int64_t v = 0; v < m; ++v)
            if (!done[v] && (u < 0 || best[v] > best[u])) u = v;
        if (best[u] == 0) break; /* the rest is unreachable */
        done[u] = 1;
        for (int64_t v = 0; v < m; ++v) {
            if (done[v]) continue;
            int64_t e = transpose ? w[v * m + u] : w[u * m + v];
            int64_t cand = best[u] < e ? best[u] : e;
            if (cand > best[v]) best[v] = cand;
        }
    }
    for (int64_t v = 0; v < m; ++v) out[v] = v == s ? 0 : best[v];
    free(best);
    free(done);
    return ORC_OK;
}

/* out[v] = p(s, v) */
int oracle_widest_from(const int64_t *w, int32_t m, int32_t s, int64_t *out) {
    if (!w || !out || m < 1 || s < 0 || s >= m) return ORC_EINVAL;
    return widest_dijkstra(w, m, s, 0, out);
}

/* out[v] = p(v, t) */
int oracle_widest_to(const int64_t *w, int32_t m, int32_t t, int64_t *out) {
    if (!w || !out || m < 1 || t < 0 || t >= m) return ORC_EINVAL;
    return widest_dijkstra(w, m, t, 1, out);
}

/* Threads used by the parallel loops above (timing only: results do not depend on it);
 * returns the count in effect before the call. */
int oracle_set_threads(int threads) {
    const int before = omp_get_max_threads();
    if (threads > 0) omp_set_num_threads(threads);
    return before;
}
