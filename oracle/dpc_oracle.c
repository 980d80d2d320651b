/*
 * Plain CPU oracle for exact Density Peaks Clustering.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the HIP library.
 *
 * It is the paper's definitions written out with no index, no pruning and no
 * reordering:
 *   density          Section 3, Definition 1: rho_i counts every point j (i
 *                    itself included) with D(x_i, x_j) <= d_cut.
 *   dependent point  Section 3, Definitions 2 and 3: the nearest point of
 *                    strictly higher priority; the point of highest priority
 *                    has none and delta = infinity.
 *   labels           Section 3, Definitions 4 and 5 and the assignment rule
 *                    after them; Section 6.2, Algorithm 3 (single linkage on
 *                    the dependent forest).
 *
 * Readings where the paper is silent or ambiguous (each is listed in the
 * design notes):
 *   - Coordinates are int32; D^2 is computed exactly in 128-bit integers.
 *   - D <= d_cut is decided as D^2 <= T with T = floor(d_cut^2), and
 *     delta >= delta_min as delta^2 >= Td with Td = ceil(delta_min^2); both
 *     are exact for integer D^2.
 *   - Density ties are broken by index (Section 3, after Definition 2): the
 *     priority of point i is the pair (rho_i, -i), so the lower index ranks
 *     higher.  Distance ties are broken by point ID (Section 5, the write-min
 *     of Algorithm 2): the smaller index wins.
 *   - The point of highest priority gets dep = -1 and delta^2 = INT64_MAX.
 *   - Noise (rho < rho_min) gets label -1.  A non-noise point whose delta is
 *     below delta_min takes the label of its dependent point; a centre
 *     (delta >= delta_min) is labelled with its own index.
 *   - Indices are 0-based.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define OR_OK 0
#define OR_ERR_INVALID_ARG 1
#define OR_ERR_RANGE 2
#define OR_ERR_NOT_FOREST 3
#define OR_INF INT64_MAX

typedef __int128 i128;

static i128 sq_dist(const int32_t *P, int d, int64_t i, int64_t j)
{
    i128 s = 0;
    for (int k = 0; k < d; k++) {
        i128 t = (i128)P[i * d + k] - (i128)P[j * d + k];
        s += t * t;
    }
    return s;
}

/* Priority order of Definition 2 with the index tie-break: does j rank above i? */
static int ranks_above(const int32_t *rho, int64_t j, int64_t i)
{
    return rho[j] > rho[i] || (rho[j] == rho[i] && j < i);
}

/*
 * r^2 rounded down (round_up = 0) or up (round_up = 1) to an integer,
 * saturating at INT64_MAX.  r = m * 2^e exactly with a 53-bit integer m,
 * so r^2 = m^2 * 2^(2e) and the rounding is a shift of a 106-bit integer.
 */
int oracle_square_threshold(double r, int round_up, int64_t *out)
{
    if (out == NULL || isnan(r) || r < 0.0)
        return OR_ERR_INVALID_ARG;
    if (isinf(r)) {
        *out = OR_INF;
        return OR_OK;
    }
    if (r == 0.0) {
        *out = 0;
        return OR_OK;
    }
    int e;
    double f = frexp(r, &e);
    int64_t m = (int64_t)ldexp(f, 53);
    e -= 53;
    i128 m2 = (i128)m * (i128)m;
    i128 lim = (i128)OR_INF;
    int s = 2 * e;
    i128 v;
    if (s >= 0) {
        if (s > 63 || m2 > (lim >> s))
            v = lim;
        else
            v = m2 << s;
    } else {
        int sh = -s;
        if (sh >= 120) {
            v = (round_up && m2 > 0) ? 1 : 0;
        } else {
            v = m2 >> sh;
            if (round_up && (v << sh) != m2)
                v += 1;
        }
    }
    if (v > lim)
        v = lim;
    *out = (int64_t)v;
    return OR_OK;
}

/* Exact squared distances must fit in int64: the sum over axes of the squared
 * extent of the bounding box may not exceed INT64_MAX. */
int oracle_range_ok(const int32_t *P, int64_t n, int32_t d)
{
    if (n <= 0)
        return 1;
    i128 s = 0;
    for (int k = 0; k < d; k++) {
        int32_t lo = P[k], hi = P[k];
        for (int64_t i = 1; i < n; i++) {
            int32_t v = P[i * d + k];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        i128 w = (i128)hi - (i128)lo;
        s += w * w;
    }
    return s <= (i128)OR_INF;
}

/* Definition 1 for the queried points only: rho_q[t] for point q[t]. */
void oracle_density_at(const int32_t *P, int64_t n, int32_t d, int64_t T,
                       const int64_t *q, int64_t nq, int32_t *rho_q)
{
    for (int64_t t = 0; t < nq; t++) {
        int64_t i = q[t];
        int64_t c = 0;
        for (int64_t j = 0; j < n; j++)
            if (sq_dist(P, d, i, j) <= (i128)T)
                c++;
        rho_q[t] = (int32_t)c;
    }
}

/* Definition 1 for every point: each point is queried on its own, so every
 * pin of the whole-array density also pins the per-query form above. */
void oracle_density(const int32_t *P, int64_t n, int32_t d, int64_t T, int32_t *rho)
{
    for (int64_t i = 0; i < n; i++)
        oracle_density_at(P, n, d, T, &i, 1, &rho[i]);
}

/* Definitions 2 and 3 for the queried points: the lexicographic minimum of
 * (D^2, j) over every j ranking above q[t]; (-1, INT64_MAX) if there is none. */
void oracle_dependent_at(const int32_t *P, int64_t n, int32_t d, const int32_t *rho,
                         const int64_t *q, int64_t nq, int32_t *dep_q, int64_t *delta2_q)
{
    for (int64_t t = 0; t < nq; t++) {
        int64_t i = q[t];
        int64_t best = -1;
        i128 best_d = 0;
        for (int64_t j = 0; j < n; j++) {
            if (!ranks_above(rho, j, i))
                continue;
            i128 dd = sq_dist(P, d, i, j);
            if (best < 0 || dd < best_d || (dd == best_d && j < best)) {
                best = j;
                best_d = dd;
            }
        }
        dep_q[t] = (int32_t)best;
        delta2_q[t] = best < 0 ? OR_INF : (int64_t)best_d;
    }
}

/* Definitions 2 and 3 for every point.  With skip_noise set, points with
 * rho < rho_min are left at (-1, INT64_MAX), as Algorithm 1 skips them. */
void oracle_dependent(const int32_t *P, int64_t n, int32_t d, const int32_t *rho,
                      int32_t rho_min, int32_t skip_noise, int32_t *dep, int64_t *delta2)
{
    for (int64_t i = 0; i < n; i++) {
        if (skip_noise && rho[i] < rho_min) {
            dep[i] = -1;
            delta2[i] = OR_INF;
            continue;
        }
        oracle_dependent_at(P, n, d, rho, &i, 1, &dep[i], &delta2[i]);
    }
}

/*
 * Labels from Definitions 4 and 5: noise gets -1; a non-noise point follows
 * its dependent point while its delta^2 is below Td and takes the index of
 * the centre it reaches.  Every followed edge must lead to a point of strictly
 * higher priority (so the walk ends); otherwise the input is not a dependent
 * forest.  A label, once found, is reused by later walks that reach it.
 */
int oracle_cluster(int64_t n, const int32_t *rho, const int32_t *dep, const int64_t *delta2,
                   int32_t rho_min, int64_t Td, int32_t *label)
{
    const int32_t PENDING = -2;
    for (int64_t i = 0; i < n; i++)
        label[i] = rho[i] < rho_min ? -1 : PENDING;
    for (int64_t i = 0; i < n; i++) {
        if (label[i] != PENDING)
            continue;
        int64_t c = i;
        while (label[c] == PENDING && delta2[c] < Td) {
            int64_t p = dep[c];
            if (p < 0 || p >= n || !ranks_above(rho, p, c))
                return OR_ERR_NOT_FOREST;
            c = p;
        }
        int32_t root = label[c] == PENDING ? (int32_t)c : label[c];
        int64_t w = i;
        while (label[w] == PENDING) {
            label[w] = root;
            if (delta2[w] >= Td)
                break;
            w = dep[w];
        }
    }
    return OR_OK;
}

/* The whole method: thresholds, range check, density, dependents, labels. */
int oracle_run(const int32_t *P, int64_t n, int32_t d, double d_cut, int32_t rho_min,
               double delta_min, int32_t skip_noise, int32_t *rho, int32_t *dep,
               int64_t *delta2, int32_t *label)
{
    int64_t T, Td;
    if (n < 0 || d < 1 || d > 8 || rho_min < 0)
        return OR_ERR_INVALID_ARG;
    if (oracle_square_threshold(d_cut, 0, &T) != OR_OK)
        return OR_ERR_INVALID_ARG;
    if (isnan(delta_min))
        return OR_ERR_INVALID_ARG;
    if (delta_min <= 0.0)
        Td = 0;
    else if (oracle_square_threshold(delta_min, 1, &Td) != OR_OK)
        return OR_ERR_INVALID_ARG;
    if (n == 0)
        return OR_OK;
    if (!oracle_range_ok(P, n, d))
        return OR_ERR_RANGE;
    oracle_density(P, n, d, T, rho);
    oracle_dependent(P, n, d, rho, rho_min, skip_noise, dep, delta2);
    return oracle_cluster(n, rho, dep, delta2, rho_min, Td, label);
}
