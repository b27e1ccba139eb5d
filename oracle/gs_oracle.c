/*
 * GridShift FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * library path never calls it and shares no code with it.
 *
 * What it computes (GridShift, Kumar et al., arXiv 2206.02200):
 *   - Section 2.1 (i) and Algorithm 1 (initialisation): every point x_i is put
 *     in the grid cell with integer index floor(x_i / h), element-wise.  A cell
 *     holding at least one point is active; it keeps a point count C and a
 *     coordinate sum S (the running-mean centroid of Algorithm 1 times C).
 *   - Section 2.1 (ii), Eq. 1-2, in the parallel form of Eq. 6 (Section 2.2)
 *     and of the supplement's update of r_j: every active cell j moves to the
 *     count-weighted mean of the centroids of the active cells j+v,
 *     v in {-1,0,1}^d (itself included), all read from the same iteration.
 *     gso_fit_rule also offers the sequential form of Eq. 5 (Section 2.2):
 *     the cells are visited one after another and a visited cell's new
 *     centroid replaces its old one for the cells visited after it, in
 *     ascending key or colour by colour (gso_colour_order).
 *   - Section 2.1 (iii): the moved cell gets the key floor(p_j / h).
 *   - Section 2.1 (iv), Eq. 3-4: cells that land on one key merge; counts add,
 *     the centroid is the count-weighted mean, the point sets are united.
 *   - Section 2.1 (v) and Theorem 2: stop when no active cell has an active
 *     neighbour.  The iteration is also capped at max_iter rounds, and it stops
 *     early when one round leaves the state bitwise unchanged.
 *
 * Readings where the paper leaves floating point open (all FP64,
 * round-to-nearest-even, no fused multiply-add):
 *   - key of a value v: floor(fl(v / h)) (IEEE division, then floor);
 *   - point-to-cell sum: R over the members in ascending point index, where
 *     R(a_0..a_{L-1}) = a_0 if L = 1, else R(first P) + R(rest) with P the
 *     largest power of two below L;
 *   - 3^d neighbourhood sum: left fold over the active neighbours in
 *     ascending lexicographic key order (dimension 0 most significant);
 *     the weight sum is an exact integer;
 *   - merge sum: R over fl(C_j * p_j) for the merging cells in ascending old
 *     key order; the merged cell's key is the landing key, never recomputed
 *     from the merged mean;
 *   - cells and final clusters are numbered in ascending lexicographic key.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (x86-64 SSE2
 * doubles, so every operation is a single IEEE binary64 rounding).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    GSO_OK = 0,
    GSO_ERR_INVALID_ARG = 1,
    GSO_ERR_NONFINITE = 2,
    GSO_ERR_KEY_RANGE = 3,
    GSO_ERR_ALLOC = 4
};

enum { GSO_CONVERGED = 1u, GSO_STATIONARY = 2u, GSO_CAPPED = 4u };

/* ---------------------------------------------------------------------- */
/* Canonical pairwise sum R (the reading used for every multi-term sum).    */
/* ---------------------------------------------------------------------- */

double gso_pairwise_sum(const double* a, int64_t L)
{
    if (L <= 0)
        return -0.0; /* empty sum: the additive identity that keeps signed zeros */
    if (L == 1)
        return a[0];
    int64_t P = 1;
    while (P * 2 < L)
        P *= 2;
    return gso_pairwise_sum(a, P) + gso_pairwise_sum(a + P, L - P);
}

/* ---------------------------------------------------------------------- */
/* Lexicographic helpers on integer key vectors.                          */
/* ---------------------------------------------------------------------- */

static int cmp_keyvec(const int64_t* a, const int64_t* b, int d)
{
    for (int k = 0; k < d; k++) {
        if (a[k] < b[k])
            return -1;
        if (a[k] > b[k])
            return 1;
    }
    return 0;
}

/* qsort context, one per host thread: each call is single-threaded, and
 * independent calls may run on different threads at once. */
static _Thread_local const int64_t* g_sort_keys;
static _Thread_local int g_sort_d;

/* Order row indices by (key vector, index): a stable grouping by key. */
static int cmp_rows_by_key_then_index(const void* A, const void* B)
{
    int64_t i = *(const int64_t*)A, j = *(const int64_t*)B;
    int c = cmp_keyvec(g_sort_keys + i * g_sort_d, g_sort_keys + j * g_sort_d, g_sort_d);
    if (c)
        return c;
    return (i < j) ? -1 : (i > j);
}

/* Binary search of key vector q among m sorted, distinct key vectors. */
static int64_t find_cell(const int64_t* cell_key, int64_t m, int d, const int64_t* q)
{
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = cmp_keyvec(cell_key + mid * d, q, d);
        if (c == 0)
            return mid;
        if (c < 0)
            lo = mid + 1;
        else
            hi = mid;
    }
    return -1;
}

/* floor(fl(v / h)) as int64; fails if the result does not fit comfortably. */
static int key_of(double v, double h, int64_t* out)
{
    double q = floor(v / h);
    if (!(q > -4611686018427387904.0 && q < 4611686018427387904.0)) /* |q| < 2^62 */
        return GSO_ERR_KEY_RANGE;
    *out = (int64_t)q;
    return GSO_OK;
}

/* Enumerate v in {-1,0,1}^d in lexicographic order (dimension 0 most
 * significant): offset index r in [0, 3^d) has digit k equal to
 * (r / 3^(d-1-k)) % 3, minus one. */
static void offset_of(int64_t r, int d, int64_t* v)
{
    for (int k = d - 1; k >= 0; k--) {
        v[k] = (r % 3) - 1;
        r /= 3;
    }
}

/* ---------------------------------------------------------------------- */
/* Step 1: binning (Section 2.1 (i), Algorithm 1 initialisation).          */
/* ---------------------------------------------------------------------- */

/*
 * x [n][d] binary64.  Outputs with capacity n cells: keys [m][d], counts [m],
 * sums [m][d] (R over members in ascending point index), cell0 [n] (cell of
 * every point), *m_out.  Cells ascend in lexicographic key order.
 */
int gso_bin(const double* x, int64_t n, int32_t d, double h, int64_t* keys, int64_t* counts,
            double* sums, int64_t* cell0, int64_t* m_out)
{
    if (n < 0 || d < 1 || d > 16 || !(h > 0.0) || !isfinite(h))
        return GSO_ERR_INVALID_ARG;
    *m_out = 0;
    for (int64_t i = 0; i < n * d; i++)
        if (!isfinite(x[i]))
            return GSO_ERR_NONFINITE;
    if (n == 0)
        return GSO_OK;
    int rc = GSO_OK;
    int64_t* pkey = malloc(sizeof(int64_t) * n * d);
    int64_t* order = malloc(sizeof(int64_t) * n);
    double* tmp = malloc(sizeof(double) * n);
    if (!pkey || !order || !tmp) {
        rc = GSO_ERR_ALLOC;
        goto done;
    }
    for (int64_t i = 0; i < n; i++)
        for (int k = 0; k < d; k++)
            if ((rc = key_of(x[i * d + k], h, &pkey[i * d + k])) != GSO_OK)
                goto done;
    for (int64_t i = 0; i < n; i++)
        order[i] = i;
    g_sort_keys = pkey;
    g_sort_d = d;
    qsort(order, (size_t)n, sizeof(int64_t), cmp_rows_by_key_then_index);
    int64_t m = 0;
    for (int64_t a = 0; a < n;) {
        int64_t b = a + 1;
        while (b < n && cmp_keyvec(pkey + order[a] * d, pkey + order[b] * d, d) == 0)
            b++;
        memcpy(keys + m * d, pkey + order[a] * d, sizeof(int64_t) * d);
        counts[m] = b - a;
        for (int k = 0; k < d; k++) {
            for (int64_t r = a; r < b; r++)
                tmp[r - a] = x[order[r] * d + k];
            sums[m * d + k] = gso_pairwise_sum(tmp, b - a);
        }
        for (int64_t r = a; r < b; r++)
            cell0[order[r]] = m;
        m++;
        a = b;
    }
    *m_out = m;
done:
    free(pkey);
    free(order);
    free(tmp);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Step 2: stopping test (Section 2.1 (v), Theorem 2).                     */
/* ---------------------------------------------------------------------- */

/* 1 if some active cell has another active cell j+v, v != 0, else 0. */
int gso_has_neighbours(const int64_t* keys, int64_t m, int32_t d)
{
    int64_t n_off = 1, v[16], q[16];
    for (int k = 0; k < d; k++)
        n_off *= 3;
    for (int64_t j = 0; j < m; j++)
        for (int64_t r = 0; r < n_off; r++) {
            offset_of(r, d, v);
            int zero = 1;
            for (int k = 0; k < d; k++) {
                q[k] = keys[j * d + k] + v[k];
                zero &= (v[k] == 0);
            }
            if (!zero && find_cell(keys, m, d, q) >= 0)
                return 1;
        }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Step 3: shift (Eq. 1-2 in the parallel form of Eq. 6).                  */
/* ---------------------------------------------------------------------- */

/*
 * For every cell j: W_j = sum of C over the active cells j+v (v in
 * {-1,0,1}^d, self included), N_j = left fold of their sums S in ascending
 * key order, p_j = N_j / W_j.  Every read is of the given (round-t) table.
 * weights [m] receives W_j (may be NULL).
 */
void gso_shift(const int64_t* keys, const int64_t* counts, const double* sums, int64_t m, int32_t d,
               double* p, int64_t* weights)
{
    int64_t n_off = 1, v[16], q[16];
    for (int k = 0; k < d; k++)
        n_off *= 3;
    for (int64_t j = 0; j < m; j++) {
        int64_t W = 0;
        int first = 1;
        double* pj = p + j * d;
        for (int64_t r = 0; r < n_off; r++) {
            offset_of(r, d, v);
            for (int k = 0; k < d; k++)
                q[k] = keys[j * d + k] + v[k];
            int64_t nb = find_cell(keys, m, d, q);
            if (nb < 0)
                continue;
            W += counts[nb];
            for (int k = 0; k < d; k++)
                pj[k] = first ? sums[nb * d + k] : pj[k] + sums[nb * d + k];
            first = 0;
        }
        for (int k = 0; k < d; k++)
            pj[k] = pj[k] / (double)W;
        if (weights)
            weights[j] = W;
    }
}

/* ---------------------------------------------------------------------- */
/* Step 3, sequential form (Eq. 5, Section 2.2; Algorithm 1 writes S'(j)   */
/* in place while looping over the keys).                                  */
/* ---------------------------------------------------------------------- */

/*
 * The cells are visited one at a time, in the order order[0], order[1], ...
 * (a permutation of 0..m-1).  Visiting j computes W_j and the left fold N_j
 * in ascending neighbour key exactly as gso_shift does, except that a
 * neighbour k already visited in this sweep contributes C_k times its new
 * centroid, fl(C_k * p_k), in place of its sum S_k: the centroids are
 * updated in place and later cells read the updated value, while the
 * weights C stay those of the round's table.  p_j = N_j / W_j.
 * Returns GSO_ERR_ALLOC or GSO_OK.
 */
int gso_shift_seq(const int64_t* keys, const int64_t* counts, const double* sums, int64_t m, int32_t d,
                  const int64_t* order, double* p, int64_t* weights)
{
    int64_t n_off = 1, v[16], q[16];
    for (int k = 0; k < d; k++)
        n_off *= 3;
    double* cur = malloc(sizeof(double) * (m > 0 ? m : 1) * d); /* C_k * centroid_k */
    if (!cur)
        return GSO_ERR_ALLOC;
    memcpy(cur, sums, sizeof(double) * m * d);
    for (int64_t r0 = 0; r0 < m; r0++) {
        const int64_t j = order[r0];
        int64_t W = 0;
        int first = 1;
        double* pj = p + j * d;
        for (int64_t r = 0; r < n_off; r++) {
            offset_of(r, d, v);
            for (int k = 0; k < d; k++)
                q[k] = keys[j * d + k] + v[k];
            int64_t nb = find_cell(keys, m, d, q);
            if (nb < 0)
                continue;
            W += counts[nb];
            for (int k = 0; k < d; k++)
                pj[k] = first ? cur[nb * d + k] : pj[k] + cur[nb * d + k];
            first = 0;
        }
        for (int k = 0; k < d; k++) {
            pj[k] = pj[k] / (double)W;
            cur[j * d + k] = (double)counts[j] * pj[k];
        }
        if (weights)
            weights[j] = W;
    }
    free(cur);
    return GSO_OK;
}

/*
 * Colour of a cell: bit (d-1-k) is the parity of its integer coordinate k
 * (dimension 0 most significant).  Two distinct cells of one colour differ
 * by an even, hence non-zero by at least 2, amount in some coordinate, so
 * they are never neighbours: visiting the cells colour by colour, ascending
 * colour and ascending key within a colour, is a sequential sweep whose
 * cells of one colour could be visited in any order, or all at once.
 * order [m] receives that visiting order of the (key-sorted) cells.
 */
void gso_colour_order(const int64_t* keys, int64_t m, int32_t d, int64_t* order)
{
    int64_t r = 0;
    for (int64_t c = 0; c < ((int64_t)1 << d); c++)
        for (int64_t j = 0; j < m; j++) {
            int64_t cj = 0;
            for (int k = 0; k < d; k++)
                cj = (cj << 1) | (((keys[j * d + k] % 2) + 2) % 2);
            if (cj == c)
                order[r++] = j;
        }
}

/* ---------------------------------------------------------------------- */
/* Step 4: relocation and merge (Section 2.1 (iii)-(iv), Eq. 3-4).         */
/* ---------------------------------------------------------------------- */

/*
 * Cell j (count C_j, shifted position p_j) lands on key floor(fl(p_j / h)).
 * Cells sharing a landing key merge: C = sum C_j, S = R(fl(C_j * p_j)) over
 * the members in ascending j; the new key is the landing key.  Outputs with
 * capacity m: nkeys [nm][d], ncounts [nm], nsums [nm][d], g [m] (new index
 * of old cell j), *nm_out.  New cells ascend in key order.
 */
int gso_merge(const int64_t* counts, const double* p, int64_t m, int32_t d, double h, int64_t* nkeys,
              int64_t* ncounts, double* nsums, int64_t* g, int64_t* nm_out)
{
    *nm_out = 0;
    if (m == 0)
        return GSO_OK;
    int rc = GSO_OK;
    int64_t* kap = malloc(sizeof(int64_t) * m * d);
    int64_t* order = malloc(sizeof(int64_t) * m);
    double* tmp = malloc(sizeof(double) * m);
    if (!kap || !order || !tmp) {
        rc = GSO_ERR_ALLOC;
        goto done;
    }
    for (int64_t j = 0; j < m; j++)
        for (int k = 0; k < d; k++)
            if ((rc = key_of(p[j * d + k], h, &kap[j * d + k])) != GSO_OK)
                goto done;
    for (int64_t j = 0; j < m; j++)
        order[j] = j;
    g_sort_keys = kap;
    g_sort_d = d;
    qsort(order, (size_t)m, sizeof(int64_t), cmp_rows_by_key_then_index);
    int64_t nm = 0;
    for (int64_t a = 0; a < m;) {
        int64_t b = a + 1;
        while (b < m && cmp_keyvec(kap + order[a] * d, kap + order[b] * d, d) == 0)
            b++;
        memcpy(nkeys + nm * d, kap + order[a] * d, sizeof(int64_t) * d);
        int64_t C = 0;
        for (int64_t r = a; r < b; r++)
            C += counts[order[r]];
        ncounts[nm] = C;
        for (int k = 0; k < d; k++) {
            for (int64_t r = a; r < b; r++) {
                int64_t j = order[r];
                tmp[r - a] = (double)counts[j] * p[j * d + k];
            }
            nsums[nm * d + k] = gso_pairwise_sum(tmp, b - a);
        }
        for (int64_t r = a; r < b; r++)
            g[order[r]] = nm;
        nm++;
        a = b;
    }
    *nm_out = nm;
done:
    free(kap);
    free(order);
    free(tmp);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Trajectory tape (for the adjoint of the differentiable form).           */
/* ---------------------------------------------------------------------- */

/*
 * The discrete trajectory of one fit: the point -> initial cell map, the
 * initial sums, and for every round t the cell table it started from (keys,
 * counts), the integer weights W_j of its shift and its merge map g_t.  The
 * table of index T is the final one.  With all of it fixed, the map from the
 * coordinates to the modes is linear (Eq. 1-4 with constant keys, counts,
 * weights and groups).
 */
typedef struct gso_tape {
    int64_t n, m0;
    int32_t d, T;
    int64_t* cell0;  /* [n] */
    double* sums0;   /* [m0][d] */
    int64_t cap;     /* capacity of the per-round arrays, in cells */
    int32_t off_cap;
    int64_t* off;    /* [T+2]: round t's table is [off[t], off[t+1]) */
    int64_t* keys;   /* [.][d] */
    int64_t* counts;
    int64_t* W;
    int64_t* g;
} gso_tape;

static int tape_push_table(gso_tape* tp, int32_t t, const int64_t* key, const int64_t* cnt, int64_t m, int d)
{
    if (t + 2 > tp->off_cap) {
        int32_t nc = tp->off_cap ? 2 * tp->off_cap : 16;
        int64_t* o = realloc(tp->off, sizeof(int64_t) * nc);
        if (!o)
            return GSO_ERR_ALLOC;
        tp->off = o;
        tp->off_cap = nc;
    }
    const int64_t start = t == 0 ? 0 : tp->off[t];
    if (start + m > tp->cap) {
        int64_t nc = tp->cap ? 2 * tp->cap : 1024;
        while (nc < start + m)
            nc *= 2;
        int64_t* k2 = realloc(tp->keys, sizeof(int64_t) * nc * d);
        if (!k2)
            return GSO_ERR_ALLOC;
        tp->keys = k2;
        int64_t* c2 = realloc(tp->counts, sizeof(int64_t) * nc);
        if (!c2)
            return GSO_ERR_ALLOC;
        tp->counts = c2;
        int64_t* w2 = realloc(tp->W, sizeof(int64_t) * nc);
        if (!w2)
            return GSO_ERR_ALLOC;
        tp->W = w2;
        int64_t* g2 = realloc(tp->g, sizeof(int64_t) * nc);
        if (!g2)
            return GSO_ERR_ALLOC;
        tp->g = g2;
        tp->cap = nc;
    }
    tp->off[t] = start;
    tp->off[t + 1] = start + m;
    memcpy(tp->keys + start * d, key, sizeof(int64_t) * m * d);
    memcpy(tp->counts + start, cnt, sizeof(int64_t) * m);
    for (int64_t j = 0; j < m; j++) {
        tp->W[start + j] = 0;
        tp->g[start + j] = -1;
    }
    return GSO_OK;
}

void gso_tape_free(gso_tape* tp)
{
    if (!tp)
        return;
    free(tp->cell0);
    free(tp->sums0);
    free(tp->off);
    free(tp->keys);
    free(tp->counts);
    free(tp->W);
    free(tp->g);
    free(tp);
}

/* ---------------------------------------------------------------------- */
/* The whole fit.                                                         */
/* ---------------------------------------------------------------------- */

/* Update rules of a round's shift. */
enum { GSO_RULE_PARALLEL = 0, GSO_RULE_SEQ_KEY = 1, GSO_RULE_SEQ_COLOUR = 2 };

static int fit_impl(const double* x, int64_t n, int32_t d, double h, int32_t max_iter, int32_t rule,
                    int32_t* labels, double* modes, int64_t* counts, double* sums, int64_t* keys_out,
                    int64_t* m_hist, int64_t* K_out, int32_t* n_iter_out, uint32_t* flags_out, gso_tape* tp)
{
    if (n < 0 || d < 1 || d > 16 || max_iter < 0 || !(h > 0.0) || !isfinite(h))
        return GSO_ERR_INVALID_ARG;
    if (rule < GSO_RULE_PARALLEL || rule > GSO_RULE_SEQ_COLOUR || (tp && rule != GSO_RULE_PARALLEL))
        return GSO_ERR_INVALID_ARG;
    *K_out = 0;
    *n_iter_out = 0;
    *flags_out = 0;
    if (tp) {
        tp->n = n;
        tp->d = d;
        tp->T = 0;
    }
    if (n == 0) {
        *flags_out = GSO_CONVERGED;
        if (m_hist)
            m_hist[0] = 0;
        if (tp) {
            tp->m0 = 0;
            return tape_push_table(tp, 0, NULL, NULL, 0, d);
        }
        return GSO_OK;
    }
    int rc = GSO_OK;
    int64_t* cell0 = malloc(sizeof(int64_t) * n);
    int64_t* ckey = malloc(sizeof(int64_t) * n * d);
    int64_t* ccnt = malloc(sizeof(int64_t) * n);
    double* csum = malloc(sizeof(double) * n * d);
    int64_t *cur = NULL, *g = NULL, *nkey = NULL, *ncnt = NULL, *W = NULL, *order = NULL;
    double *p = NULL, *nsum = NULL;
    if (!cell0 || !ckey || !ccnt || !csum) {
        rc = GSO_ERR_ALLOC;
        goto done;
    }
    int64_t m = 0;
    if ((rc = gso_bin(x, n, d, h, ckey, ccnt, csum, cell0, &m)) != GSO_OK)
        goto done;
    const int64_t m0 = m;
    cur = malloc(sizeof(int64_t) * m0);
    g = malloc(sizeof(int64_t) * m0);
    nkey = malloc(sizeof(int64_t) * m0 * d);
    ncnt = malloc(sizeof(int64_t) * m0);
    W = malloc(sizeof(int64_t) * m0);
    p = malloc(sizeof(double) * m0 * d);
    nsum = malloc(sizeof(double) * m0 * d);
    order = malloc(sizeof(int64_t) * m0);
    if (!cur || !g || !nkey || !ncnt || !W || !p || !nsum || !order) {
        rc = GSO_ERR_ALLOC;
        goto done;
    }
    if (tp) {
        tp->m0 = m0;
        tp->cell0 = malloc(sizeof(int64_t) * n);
        tp->sums0 = malloc(sizeof(double) * m0 * d);
        if (!tp->cell0 || !tp->sums0) {
            rc = GSO_ERR_ALLOC;
            goto done;
        }
        memcpy(tp->cell0, cell0, sizeof(int64_t) * n);
        memcpy(tp->sums0, csum, sizeof(double) * m0 * d);
    }
    for (int64_t c = 0; c < m0; c++)
        cur[c] = c;

    uint32_t flags = 0;
    int32_t t = 0;
    for (;;) {
        if (m_hist)
            m_hist[t] = m;
        if (tp && (rc = tape_push_table(tp, t, ckey, ccnt, m, d)) != GSO_OK)
            goto done;
        if (!gso_has_neighbours(ckey, m, d)) {
            flags |= GSO_CONVERGED;
            break;
        }
        if (t == max_iter) {
            flags |= GSO_CAPPED;
            break;
        }
        if (rule == GSO_RULE_PARALLEL) {
            gso_shift(ckey, ccnt, csum, m, d, p, W);
        } else {
            if (rule == GSO_RULE_SEQ_KEY)
                for (int64_t c = 0; c < m; c++)
                    order[c] = c;
            else
                gso_colour_order(ckey, m, d, order);
            if ((rc = gso_shift_seq(ckey, ccnt, csum, m, d, order, p, W)) != GSO_OK)
                goto done;
        }
        int64_t nm = 0;
        if ((rc = gso_merge(ccnt, p, m, d, h, nkey, ncnt, nsum, g, &nm)) != GSO_OK)
            goto done;
        if (tp) {
            memcpy(tp->W + tp->off[t], W, sizeof(int64_t) * m);
            memcpy(tp->g + tp->off[t], g, sizeof(int64_t) * m);
        }
        int same = (nm == m);
        for (int64_t c = 0; same && c < m; c++) {
            same = (ccnt[c] == ncnt[c]) && cmp_keyvec(ckey + c * d, nkey + c * d, d) == 0;
            for (int k = 0; same && k < d; k++)
                same = memcmp(&csum[c * d + k], &nsum[c * d + k], sizeof(double)) == 0;
        }
        for (int64_t c = 0; c < m0; c++)
            cur[c] = g[cur[c]];
        memcpy(ckey, nkey, sizeof(int64_t) * nm * d);
        memcpy(ccnt, ncnt, sizeof(int64_t) * nm);
        memcpy(csum, nsum, sizeof(double) * nm * d);
        m = nm;
        t++;
        if (same) {
            flags |= GSO_STATIONARY;
            if (m_hist)
                m_hist[t] = m;
            if (tp && (rc = tape_push_table(tp, t, ckey, ccnt, m, d)) != GSO_OK)
                goto done;
            break;
        }
    }
    if (tp)
        tp->T = t;

    for (int64_t i = 0; i < n; i++)
        labels[i] = (int32_t)cur[cell0[i]];
    for (int64_t c = 0; c < m; c++) {
        counts[c] = ccnt[c];
        for (int k = 0; k < d; k++) {
            modes[c * d + k] = csum[c * d + k] / (double)ccnt[c];
            if (sums)
                sums[c * d + k] = csum[c * d + k];
            if (keys_out)
                keys_out[c * d + k] = ckey[c * d + k];
        }
    }
    *K_out = m;
    *n_iter_out = t;
    *flags_out = flags;
done:
    free(cell0);
    free(ckey);
    free(ccnt);
    free(csum);
    free(cur);
    free(g);
    free(nkey);
    free(ncnt);
    free(W);
    free(p);
    free(nsum);
    free(order);
    return rc;
}

/*
 * x        [n][d] row-major binary64 points (f32 data is widened exactly first)
 * h        cell side, finite and > 0
 * max_iter maximum number of shift+merge rounds (>= 0)
 * Outputs (caller-allocated, capacity n for the cluster arrays):
 *   labels [n]      cluster id of every point (ids ascend with final key)
 *   modes  [K][d]   fl(S_c / C_c)
 *   counts [K]      C_c
 *   sums   [K][d]   S_c (may be NULL)
 *   keys   [K][d]   final integer cell keys (may be NULL)
 *   m_hist [max_iter+1] active cells before each round and after the last
 *                   (may be NULL)
 *   K, n_iter (rounds executed), flags (GSO_CONVERGED / STATIONARY / CAPPED)
 * Loop: stop with CONVERGED when no cell has an active neighbour; else stop
 * with CAPPED when max_iter rounds have run; else shift and merge; stop with
 * STATIONARY when the round left keys, counts and sums bitwise unchanged.
 */
int gso_fit(const double* x, int64_t n, int32_t d, double h, int32_t max_iter,
            int32_t* labels, double* modes, int64_t* counts, double* sums, int64_t* keys_out,
            int64_t* m_hist, int64_t* K_out, int32_t* n_iter_out, uint32_t* flags_out)
{
    return fit_impl(x, n, d, h, max_iter, GSO_RULE_PARALLEL, labels, modes, counts, sums, keys_out, m_hist, K_out,
                    n_iter_out, flags_out, NULL);
}

/*
 * gso_fit with a choice of update rule for the shift of every round:
 *   0  parallel (Eq. 6): every cell reads the round's table (gso_shift);
 *   1  sequential (Eq. 5), the cells visited in ascending key;
 *   2  sequential (Eq. 5), the cells visited colour by colour
 *      (gso_colour_order), the sweep a device can run one colour at a time.
 * Relocation, merge (the merge values are fl(C_j * p_j) in every rule) and
 * the stopping tests are those of gso_fit.
 */
int gso_fit_rule(const double* x, int64_t n, int32_t d, double h, int32_t max_iter, int32_t rule,
                 int32_t* labels, double* modes, int64_t* counts, double* sums, int64_t* keys_out,
                 int64_t* m_hist, int64_t* K_out, int32_t* n_iter_out, uint32_t* flags_out)
{
    return fit_impl(x, n, d, h, max_iter, rule, labels, modes, counts, sums, keys_out, m_hist, K_out, n_iter_out,
                    flags_out, NULL);
}

/* The same fit, also recording the trajectory tape (*tape_out, freed with
 * gso_tape_free). */
int gso_fit_tape(const double* x, int64_t n, int32_t d, double h, int32_t max_iter,
                 int32_t* labels, double* modes, int64_t* counts, double* sums, int64_t* keys_out,
                 int64_t* m_hist, int64_t* K_out, int32_t* n_iter_out, uint32_t* flags_out, gso_tape** tape_out)
{
    gso_tape* tp = calloc(1, sizeof(gso_tape));
    *tape_out = NULL;
    if (!tp)
        return GSO_ERR_ALLOC;
    int rc = fit_impl(x, n, d, h, max_iter, GSO_RULE_PARALLEL, labels, modes, counts, sums, keys_out, m_hist, K_out,
                      n_iter_out, flags_out, tp);
    if (rc != GSO_OK) {
        gso_tape_free(tp);
        return rc;
    }
    *tape_out = tp;
    return GSO_OK;
}

/* Tape accessors: sizes, and copies of one round's table. */
void gso_tape_sizes(const gso_tape* tp, int64_t* n, int64_t* m0, int32_t* d, int32_t* T)
{
    *n = tp->n;
    *m0 = tp->m0;
    *d = tp->d;
    *T = tp->T;
}

int64_t gso_tape_round_cells(const gso_tape* tp, int32_t t) { return tp->off[t + 1] - tp->off[t]; }

void gso_tape_round(const gso_tape* tp, int32_t t, int64_t* keys, int64_t* counts, int64_t* W, int64_t* g)
{
    const int64_t a = tp->off[t], m = tp->off[t + 1] - tp->off[t];
    memcpy(keys, tp->keys + a * tp->d, sizeof(int64_t) * m * tp->d);
    memcpy(counts, tp->counts + a, sizeof(int64_t) * m);
    memcpy(W, tp->W + a, sizeof(int64_t) * m);
    memcpy(g, tp->g + a, sizeof(int64_t) * m);
}

void gso_tape_points(const gso_tape* tp, int64_t* cell0, double* sums0)
{
    memcpy(cell0, tp->cell0, sizeof(int64_t) * tp->n);
    memcpy(sums0, tp->sums0, sizeof(double) * tp->m0 * tp->d);
}

/* ---------------------------------------------------------------------- */
/* Adjoint along a fixed trajectory.                                       */
/* ---------------------------------------------------------------------- */

/*
 * With the tape fixed the modes are mu_c = S^T_c / C_c, S^{t+1}_G =
 * sum_{j in G} C_j p_j, p_j = N_j / W_j, N_j = sum_{k in N(j)} S^t_k and
 * S^0_c = sum_{i in c} x_i.  Reverse mode, in the same FP64 order for every
 * implementation:
 *   Sbar^T_c = mubar_c / C_c;
 *   q_j      = (C_j * Sbar^{t+1}_{g_t(j)}) / W_j;
 *   Sbar^t_k = left fold, over the active cells j+v of round t in ascending
 *              key (the neighbour relation is symmetric), of q_j;
 * and the gradient of point i is Sbar^0_{cell0(i)}.
 * mubar [K][d], sbar0 [m0][d].
 */
int gso_tape_adjoint(const gso_tape* tp, const double* mubar, double* sbar0)
{
    const int d = tp->d;
    const int32_t T = tp->T;
    const int64_t m0 = tp->m0;
    if (m0 == 0)
        return GSO_OK;
    double* sb = malloc(sizeof(double) * m0 * d);
    double* q = malloc(sizeof(double) * m0 * d);
    if (!sb || !q) {
        free(sb);
        free(q);
        return GSO_ERR_ALLOC;
    }
    {
        const int64_t a = tp->off[T], K = tp->off[T + 1] - tp->off[T];
        for (int64_t c = 0; c < K; c++)
            for (int k = 0; k < d; k++)
                sb[c * d + k] = mubar[c * d + k] / (double)tp->counts[a + c];
    }
    int64_t n_off = 1, v[16], qk[16];
    for (int k = 0; k < d; k++)
        n_off *= 3;
    for (int32_t t = T - 1; t >= 0; t--) {
        const int64_t a = tp->off[t], m = tp->off[t + 1] - tp->off[t];
        const int64_t* key = tp->keys + a * d;
        for (int64_t j = 0; j < m; j++)
            for (int k = 0; k < d; k++)
                q[j * d + k] = ((double)tp->counts[a + j] * sb[tp->g[a + j] * d + k]) / (double)tp->W[a + j];
        for (int64_t kc = 0; kc < m; kc++) {
            int first = 1;
            for (int64_t r = 0; r < n_off; r++) {
                offset_of(r, d, v);
                for (int k = 0; k < d; k++)
                    qk[k] = key[kc * d + k] + v[k];
                const int64_t j = find_cell(key, m, d, qk);
                if (j < 0)
                    continue;
                for (int k = 0; k < d; k++)
                    sb[kc * d + k] = first ? q[j * d + k] : sb[kc * d + k] + q[j * d + k];
                first = 0;
            }
        }
    }
    memcpy(sbar0, sb, sizeof(double) * m0 * d);
    free(sb);
    free(q);
    return GSO_OK;
}

/* Coordinate sums of every final cluster over its points, as R over the
 * cluster's initial cells in ascending cell order of their (initial) sums.
 * X [K][d]. */
int gso_tape_cluster_sums(const gso_tape* tp, double* X)
{
    const int d = tp->d;
    const int32_t T = tp->T;
    const int64_t m0 = tp->m0;
    const int64_t K = tp->off[T + 1] - tp->off[T];
    if (m0 == 0)
        return GSO_OK;
    int64_t* fin = malloc(sizeof(int64_t) * m0);
    double* tmp = malloc(sizeof(double) * m0);
    if (!fin || !tmp) {
        free(fin);
        free(tmp);
        return GSO_ERR_ALLOC;
    }
    for (int64_t c = 0; c < m0; c++) {
        int64_t cur = c;
        for (int32_t t = 0; t < T; t++)
            cur = tp->g[tp->off[t] + cur];
        fin[c] = cur;
    }
    for (int64_t c = 0; c < K; c++)
        for (int k = 0; k < d; k++) {
            int64_t L = 0;
            for (int64_t c0 = 0; c0 < m0; c0++)
                if (fin[c0] == c)
                    tmp[L++] = tp->sums0[c0 * d + k];
            X[c * d + k] = gso_pairwise_sum(tmp, L);
        }
    free(fin);
    free(tmp);
    return GSO_OK;
}

/* Point-to-mode loss L = R over points in ascending index of the left fold
 * over k of (x_ik - mu_{l(i),k})^2. */
double gso_point_mode_loss(const double* x, int64_t n, int32_t d, const int32_t* labels, const double* modes)
{
    if (n <= 0)
        return 0.0;
    double* tmp = malloc(sizeof(double) * n);
    if (!tmp)
        return NAN;
    for (int64_t i = 0; i < n; i++) {
        double acc = 0.0;
        for (int k = 0; k < d; k++) {
            const double e = x[i * d + k] - modes[(int64_t)labels[i] * d + k];
            acc = k == 0 ? e * e : acc + e * e;
        }
        tmp[i] = acc;
    }
    const double L = gso_pairwise_sum(tmp, n);
    free(tmp);
    return L;
}

/* ---------------------------------------------------------------------- */
/* binary128 replay of the loss along a fixed trajectory (for finite        */
/* differences).                                                          */
/* ---------------------------------------------------------------------- */

typedef __float128 q128;

static int replay_loss_q(const gso_tape* tp, const double* x, q128* out)
{
    const int d = tp->d;
    const int32_t T = tp->T;
    const int64_t n = tp->n, m0 = tp->m0;
    if (n == 0) {
        *out = 0;
        return GSO_OK;
    }
    q128* S = calloc((size_t)(m0 * d), sizeof(q128));
    q128* P = malloc(sizeof(q128) * m0 * d);
    q128* S2 = malloc(sizeof(q128) * m0 * d);
    int64_t* fin = malloc(sizeof(int64_t) * m0);
    if (!S || !P || !S2 || !fin) {
        free(S);
        free(P);
        free(S2);
        free(fin);
        return GSO_ERR_ALLOC;
    }
    for (int64_t i = 0; i < n; i++)
        for (int k = 0; k < d; k++)
            S[tp->cell0[i] * d + k] += (q128)x[i * d + k];
    int64_t n_off = 1, v[16], qk[16];
    for (int k = 0; k < d; k++)
        n_off *= 3;
    for (int32_t t = 0; t < T; t++) {
        const int64_t a = tp->off[t], m = tp->off[t + 1] - tp->off[t];
        const int64_t mn = tp->off[t + 2] - tp->off[t + 1];
        const int64_t* key = tp->keys + a * d;
        for (int64_t j = 0; j < m; j++) {
            for (int k = 0; k < d; k++)
                P[j * d + k] = 0;
            for (int64_t r = 0; r < n_off; r++) {
                offset_of(r, d, v);
                for (int k = 0; k < d; k++)
                    qk[k] = key[j * d + k] + v[k];
                const int64_t nb = find_cell(key, m, d, qk);
                if (nb >= 0)
                    for (int k = 0; k < d; k++)
                        P[j * d + k] += S[nb * d + k];
            }
            for (int k = 0; k < d; k++)
                P[j * d + k] /= (q128)tp->W[a + j];
        }
        for (int64_t c = 0; c < mn * d; c++)
            S2[c] = 0;
        for (int64_t j = 0; j < m; j++)
            for (int k = 0; k < d; k++)
                S2[tp->g[a + j] * d + k] += (q128)tp->counts[a + j] * P[j * d + k];
        memcpy(S, S2, sizeof(q128) * mn * d);
    }
    for (int64_t c = 0; c < m0; c++) {
        int64_t cur = c;
        for (int32_t t = 0; t < T; t++)
            cur = tp->g[tp->off[t] + cur];
        fin[c] = cur;
    }
    const int64_t af = tp->off[T];
    q128 L = 0;
    for (int64_t i = 0; i < n; i++) {
        const int64_t c = fin[tp->cell0[i]];
        const q128 C = (q128)tp->counts[af + c];
        for (int k = 0; k < d; k++) {
            const q128 e = (q128)x[i * d + k] - S[c * d + k] / C;
            L += e * e;
        }
    }
    *out = L;
    free(S);
    free(P);
    free(S2);
    free(fin);
    return GSO_OK;
}

/* Central difference of the replayed loss in coordinate (i, k):
 * (L(x with x_ik = fl(x_ik + eps)) - L(x with x_ik = fl(x_ik - eps))) / (step),
 * step being the exact difference of the two perturbed values; binary128
 * throughout.  The caller checks that both perturbed inputs follow the same
 * trajectory as x. */
int gso_tape_fd_q(const gso_tape* tp, const double* x, int64_t i, int32_t k, double eps, double* out)
{
    const int d = tp->d;
    const int64_t n = tp->n;
    double* xx = malloc(sizeof(double) * n * d);
    if (!xx)
        return GSO_ERR_ALLOC;
    memcpy(xx, x, sizeof(double) * n * d);
    const double xp = x[i * d + k] + eps, xm = x[i * d + k] - eps;
    q128 Lp = 0, Lm = 0;
    xx[i * d + k] = xp;
    int rc = replay_loss_q(tp, xx, &Lp);
    xx[i * d + k] = xm;
    if (rc == GSO_OK)
        rc = replay_loss_q(tp, xx, &Lm);
    free(xx);
    if (rc != GSO_OK)
        return rc;
    *out = (double)((Lp - Lm) / ((q128)xp - (q128)xm));
    return GSO_OK;
}

/* The replayed loss itself, as hi + lo. */
int gso_tape_replay_loss(const gso_tape* tp, const double* x, double* hi, double* lo)
{
    q128 L = 0;
    int rc = replay_loss_q(tp, x, &L);
    if (rc != GSO_OK)
        return rc;
    *hi = (double)L;
    *lo = (double)(L - (q128)*hi);
    return GSO_OK;
}
