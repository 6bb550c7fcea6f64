/*
 * oracle.c -- plain CPU oracle for the 2-domination number of cylinders
 * P_n x C_m computed with (min,+) matrix powers (Garzon, Martinez, Moreno,
 * Puertas, "HPC acceleration of large (min,+) matrix products to compute
 * domination-type parameters in graphs", arXiv 2409.17688).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * Notation: n = order of the path (the paper's m), m = order of the cycle (the
 * paper's n).  A word of length n over {0,1,2} is stored as its base-3 value
 * with the first letter p^1 as the most significant digit.
 *
 * Everything is computed the slow, obvious way, in 32/64-bit integers:
 *   - correct words: the forbidden patterns of Section 2.2, tested as strings;
 *   - arcs q -> p: the three labelling rules of Section 2.2, position by
 *     position; arc label = number of zeros of the successor p (Section 2.2);
 *   - (min,+) product: the semiring definition of Section 1,
 *     (A x B)_ij = min_k (a_ik + b_kj), with every sum >= INF taken as INF;
 *   - powers: Algorithm 2, A^k = A x A^(k-1);
 *   - gamma_2(P_n x C_m) = min_i (A^m)_ii (Theorem 2; Algorithm 5);
 *   - all-pairs shortest paths by Floyd-Warshall relaxation, for the same
 *     semiring applied to another workload;
 *   - recurrence search (Algorithm 3) and its minimal start (Algorithm 4),
 *     with "A^i - A^j is constant" read as A^i = b x A^j exactly (same INF
 *     pattern, every finite difference equal to one b);
 *   - the complementary construction: columns that are copies of the cycle,
 *     the rules of Section 2.2 read around the cycle, an open walk along the
 *     path with a start and an end vector, by (min,+) vector-matrix products
 *     (the small-cycle / any-path problem of Section 1, on Section 2.1).
 * The only liberty taken is skipping k when a_ik is INF, which cannot change
 * the result because every such sum is INF.  The row loop of the product is
 * split over OpenMP threads, as in the paper's multicore version (Section 3).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN 16

/* threads the row-parallel loops use */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* sets the number of threads for later calls (a timing knob; no result
 * depends on it) */
void oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0)
        omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* letters w[0..n-1] of a base-3 code, w[0] = p^1 (most significant) */
static void decode(uint32_t code, int n, int *w)
{
    for (int i = n - 1; i >= 0; --i) {
        w[i] = (int)(code % 3u);
        code /= 3u;
    }
}

/* Section 2.2: a correct word contains none of 020, 111, 211, 112, 212, does
 * not start with 11 or 12 and does not end with 11 or 21. */
int oracle_is_correct_word(int n, uint32_t code)
{
    int w[MAXN];
    char s[MAXN + 1];
    decode(code, n, w);
    for (int i = 0; i < n; ++i)
        s[i] = (char)('0' + w[i]);
    s[n] = '\0';
    static const char *inner[5] = {"020", "111", "211", "112", "212"};
    for (int t = 0; t < 5; ++t)
        if (strstr(s, inner[t]) != NULL)
            return 0;
    if (n >= 2) {
        if (strncmp(s, "11", 2) == 0 || strncmp(s, "12", 2) == 0)
            return 0;
        if (strcmp(s + n - 2, "11") == 0 || strcmp(s + n - 2, "21") == 0)
            return 0;
    }
    return 1;
}

/* Number of correct words of length n; when codes != NULL also writes their
 * base-3 codes in increasing order (the index order of the state matrix). */
int64_t oracle_words(int n, uint32_t *codes)
{
    if (n < 1 || n > MAXN)
        return -1;
    uint32_t total = 1;
    for (int i = 0; i < n; ++i)
        total *= 3u;
    int64_t cnt = 0;
    for (uint32_t x = 0; x < total; ++x) {
        if (oracle_is_correct_word(n, x)) {
            if (codes)
                codes[cnt] = x;
            ++cnt;
        }
    }
    return cnt;
}

int oracle_zeros(int n, uint32_t code)
{
    int w[MAXN], z = 0;
    decode(code, n, w);
    for (int i = 0; i < n; ++i)
        z += (w[i] == 0);
    return z;
}

/* Section 2.2, "p can follow q": for every position i
 *   q_i = 2            => p_i = 0
 *   p_i = 2            => exactly one of p_{i-1}, p_{i+1}, q_i is 0
 *   p_i = 1            => at least two of p_{i-1}, p_{i+1}, q_i are 0
 * where a neighbour outside the path (i = 1 or i = n) is simply absent. */
int oracle_follows(int n, uint32_t q_code, uint32_t p_code)
{
    int q[MAXN], p[MAXN];
    decode(q_code, n, q);
    decode(p_code, n, p);
    for (int i = 0; i < n; ++i) {
        if (q[i] == 2 && p[i] != 0)
            return 0;
        int zeros = (q[i] == 0);
        if (i > 0)
            zeros += (p[i - 1] == 0);
        if (i < n - 1)
            zeros += (p[i + 1] == 0);
        if (p[i] == 2 && zeros != 1)
            return 0;
        if (p[i] == 1 && zeros < 2)
            return 0;
    }
    return 1;
}

/* Algorithm 1: A[q][p] = zeros(p) if p can follow q, else INF.  Row-major
 * N x N int32 with leading dimension N.  Returns N, or -1 on bad n. */
int64_t oracle_state_matrix(int n, int32_t inf, int32_t *A)
{
    int64_t N = oracle_words(n, NULL);
    if (N < 0)
        return -1;
    uint32_t *w = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    oracle_words(n, w);
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j)
            A[i * N + j] = oracle_follows(n, w[i], w[j]) ? oracle_zeros(n, w[j]) : inf;
    free(w);
    return N;
}

/* Selected rows of Algorithm 1's matrix, for path orders whose whole matrix
 * is too large to hold (n = 11, 12): out[r][p] = zeros(p) if p can follow
 * word rows[r], else INF, by the same follows test as oracle_state_matrix.
 * rows[] index the correct words in increasing order; out is nrows x N
 * int32, leading dimension N.  Returns N, or -1 on bad n or a row index
 * outside 0..N-1 (nothing written then). */
int64_t oracle_state_rows(int n, int64_t nrows, const int64_t *rows, int32_t inf, int32_t *out)
{
    int64_t N = oracle_words(n, NULL);
    if (N < 0 || nrows < 0)
        return -1;
    for (int64_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= N)
            return -1;
    uint32_t *w = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    oracle_words(n, w);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r)
        for (int64_t j = 0; j < N; ++j)
            out[r * N + j] = oracle_follows(n, w[rows[r]], w[j]) ? oracle_zeros(n, w[j]) : inf;
    free(w);
    return N;
}

/* Section 1: C = A x B in the (min,+) semiring, saturating at INF.
 * C is M x N, A is M x K, B is K x N, all row-major int32 with the given
 * leading dimensions; inputs hold values in [0, INF].  C must not alias A or B. */
void oracle_minplus(int64_t M, int64_t N, int64_t K,
                    const int32_t *A, int64_t lda,
                    const int32_t *B, int64_t ldb,
                    int32_t *C, int64_t ldc, int32_t inf)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < M; ++i) {
        int32_t *c = C + i * ldc;
        for (int64_t j = 0; j < N; ++j)
            c[j] = inf;
        for (int64_t k = 0; k < K; ++k) {
            int32_t a = A[i * lda + k];
            if (a >= inf)
                continue; /* every a + b_kj >= INF: contributes INF */
            const int32_t *b = B + k * ldb;
            for (int64_t j = 0; j < N; ++j) {
                int32_t s = a + b[j];
                if (s > inf)
                    s = inf;
                if (s < c[j])
                    c[j] = s;
            }
        }
    }
}

/* min_i X_ii of an N x N matrix (Theorem 2 / Algorithm 5). */
int32_t oracle_trace_min(int64_t N, const int32_t *X, int64_t ldx, int32_t inf)
{
    int32_t best = inf;
    for (int64_t i = 0; i < N; ++i)
        if (X[i * ldx + i] < best)
            best = X[i * ldx + i];
    return best;
}

/* Algorithm 2 followed by Algorithm 5 on one chain:
 * gam[k-1] = min_i (A^k)_ii for k = 1..kmax, where A^1 = A and
 * A^k = A x A^(k-1).  Returns N, or -1 on bad arguments. */
int64_t oracle_gamma2_sweep(int n, int kmax, int32_t inf, int32_t *gam)
{
    int64_t N = oracle_words(n, NULL);
    if (N < 0 || kmax < 1)
        return -1;
    size_t bytes = (size_t)N * (size_t)N * sizeof(int32_t);
    int32_t *A = (int32_t *)malloc(bytes);
    int32_t *X = (int32_t *)malloc(bytes);
    int32_t *Y = (int32_t *)malloc(bytes);
    oracle_state_matrix(n, inf, A);
    memcpy(X, A, bytes);
    gam[0] = oracle_trace_min(N, X, N, inf);
    for (int k = 2; k <= kmax; ++k) {
        oracle_minplus(N, N, N, A, N, X, N, Y, N, inf);
        int32_t *t = X;
        X = Y;
        Y = t;
        gam[k - 1] = oracle_trace_min(N, X, N, inf);
    }
    free(A);
    free(X);
    free(Y);
    return N;
}

/* A^k by Algorithm 2, into out (N x N).  Returns N or -1. */
int64_t oracle_power(int n, int k, int32_t inf, int32_t *out)
{
    int64_t N = oracle_words(n, NULL);
    if (N < 0 || k < 1)
        return -1;
    size_t bytes = (size_t)N * (size_t)N * sizeof(int32_t);
    int32_t *A = (int32_t *)malloc(bytes);
    int32_t *T = (int32_t *)malloc(bytes);
    oracle_state_matrix(n, inf, A);
    memcpy(out, A, bytes);
    for (int i = 2; i <= k; ++i) {
        oracle_minplus(N, N, N, A, N, out, N, T, N, inf);
        memcpy(out, T, bytes);
    }
    free(A);
    free(T);
    return N;
}

/* X == b (x) Y exactly: same INF pattern and every finite entry of X equal to
 * the matching entry of Y plus one common b.  Writes b (0 when there is no
 * finite entry).  Returns 1 when it holds. */
static int constant_difference(int64_t cnt, const int32_t *X, const int32_t *Y,
                               int32_t inf, int64_t *b_out)
{
    int have = 0;
    int64_t b = 0;
    for (int64_t e = 0; e < cnt; ++e) {
        int xi = X[e] >= inf, yi = Y[e] >= inf;
        if (xi != yi)
            return 0;
        if (xi)
            continue;
        int64_t d = (int64_t)X[e] - (int64_t)Y[e];
        if (!have) {
            b = d;
            have = 1;
        } else if (d != b) {
            return 0;
        }
    }
    *b_out = b;
    return 1;
}

/* All-pairs shortest paths on the same semiring (Section 1), written as the
 * textbook Floyd-Warshall relaxation: D starts as W with a zero diagonal and,
 * for every intermediate vertex k in turn, D[i][j] = min(D[i][j],
 * D[i][k] + D[k][j]) with sums >= inf taken as inf.  Non-negative weights;
 * N x N row-major int32, leading dimension N. */
void oracle_apsp(int64_t N, const int32_t *W, int32_t inf, int32_t *D)
{
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j)
            D[i * N + j] = (i == j) ? 0 : (W[i * N + j] >= inf ? inf : W[i * N + j]);
    for (int64_t k = 0; k < N; ++k) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            const int64_t dik = D[i * N + k];
            if (dik >= inf)
                continue;
            for (int64_t j = 0; j < N; ++j) {
                int64_t t = dik + D[k * N + j];
                if (t > inf)
                    t = inf;
                if (t < D[i * N + j])
                    D[i * N + j] = (int32_t)t;
            }
        }
    }
}

/* The same test for callers: X and Y hold cnt entries each (row-major,
 * contiguous).  Returns 1 and writes *b_out when X = b (x) Y, else 0. */
int oracle_constant_difference(int64_t cnt, const int32_t *X, const int32_t *Y, int32_t inf,
                               int64_t *b_out)
{
    return constant_difference(cnt, X, Y, inf, b_out);
}

/* Algorithms 3 and 4 on the first K powers.
 * Algorithm 3: for i = K down to 1, for j = i-1 down to 1, the first pair with
 * A^i = b x A^j gives a = i - j, b, r0 = j.
 * Algorithm 4: starting at i = r0 + a and going down while i - a >= 1, m0 is
 * the last i - a for which A^i = b x A^(i-a) still holds.
 * out[0..3] = r0, a, b, m0.  Returns 1 when a recurrence was found, 0 when not,
 * -1 on bad arguments.  Memory: K dense N x N int32 powers. */
int oracle_recurrence(int n, int K, int32_t inf, int64_t *out)
{
    int64_t N = oracle_words(n, NULL);
    if (N < 0 || K < 2)
        return -1;
    int64_t cnt = N * N;
    size_t bytes = (size_t)cnt * sizeof(int32_t);
    int32_t **P = (int32_t **)calloc((size_t)K + 1, sizeof(int32_t *));
    P[1] = (int32_t *)malloc(bytes);
    oracle_state_matrix(n, inf, P[1]);
    for (int i = 2; i <= K; ++i) {
        P[i] = (int32_t *)malloc(bytes);
        oracle_minplus(N, N, N, P[1], N, P[i - 1], N, P[i], N, inf);
    }
    int found = 0;
    int64_t r0 = 0, a = 0, b = 0;
    for (int i = K; i >= 1 && !found; --i) {
        for (int j = i - 1; j >= 1; --j) {
            int64_t bb;
            if (constant_difference(cnt, P[i], P[j], inf, &bb)) {
                a = i - j;
                b = bb;
                r0 = j;
                found = 1;
                break;
            }
        }
    }
    int64_t m0 = -1;
    if (found) {
        for (int64_t i = r0 + a; i - a >= 1; --i) {
            int64_t bb;
            if (!constant_difference(cnt, P[i], P[i - a], inf, &bb) || bb != b)
                break;
            m0 = i - a;
        }
    }
    for (int i = 1; i <= K; ++i)
        free(P[i]);
    free(P);
    out[0] = r0;
    out[1] = a;
    out[2] = b;
    out[3] = m0;
    return found;
}

/* ------------------------------------------------------------------------
 * The complementary construction: columns that are copies of the cycle.
 *
 * Section 1 names the problem of a small cycle and any path, solved in the
 * companion work with (min,+) matrix-vector products; Section 2.1 gives the
 * general column digraph for any Cartesian product with a column structure.
 * Here a column is the cycle C_m (m >= 3) and the columns follow each other
 * along the path P_n, so a 2-dominating set is an open walk of n columns.
 * The letters and the three rules of Section 2.2 stay as they are, with the
 * neighbours of letter i inside the column taken modulo m (letters i - 1 and
 * i + 1 around the cycle).  The path has ends, so two boundary conditions
 * replace the closing arc of Theorem 2:
 *   - the first column has no column before it: its letters are labelled from
 *     their column alone (q_i counts as neither 0 nor 2);
 *   - the last column has no column after it, which is the only place a
 *     letter 2 could find its missing neighbour: it holds no 2.
 * gamma_2(P_n x C_m) is then the least label of such a walk: with s the start
 * vector (zeros(p) where p may open the walk, else INF) and e the end vector
 * (0 where p may close it, else INF), it is min_p (s x A^(n-1))_p + e_p.
 * ------------------------------------------------------------------------ */

/* Letters w[0..m-1] of a cyclic word are decoded as for the path words. */

/* A cyclic word is correct when no letter breaks a rule that its column
 * alone already decides, read around the cycle: no 2 with both column
 * neighbours 0 (the 020 window), no 1 with both column neighbours nonzero
 * (the 111, 211, 112, 212 windows).  There are no start or end windows. */
int oracle_is_correct_cyclic_word(int m, uint32_t code)
{
    int w[MAXN];
    if (m < 3 || m > MAXN)
        return 0;
    decode(code, m, w);
    for (int i = 0; i < m; ++i) {
        int left = w[(i + m - 1) % m], right = w[(i + 1) % m];
        if (w[i] == 2 && left == 0 && right == 0)
            return 0;
        if (w[i] == 1 && left != 0 && right != 0)
            return 0;
    }
    return 1;
}

/* Number of correct cyclic words of length m; with codes != NULL also their
 * base-3 codes in increasing order (the index order of the matrix below). */
int64_t oracle_cyclic_words(int m, uint32_t *codes)
{
    if (m < 3 || m > MAXN)
        return -1;
    uint32_t total = 1;
    for (int i = 0; i < m; ++i)
        total *= 3u;
    int64_t cnt = 0;
    for (uint32_t x = 0; x < total; ++x) {
        if (oracle_is_correct_cyclic_word(m, x)) {
            if (codes)
                codes[cnt] = x;
            ++cnt;
        }
    }
    return cnt;
}

/* "p can follow q" for cyclic columns: the rules of Section 2.2 with the
 * column neighbours of letter i taken modulo m.  q = NULL stands for the
 * missing column before the first one (no 0 and no 2 in it). */
static int cyclic_follows_letters(int m, const int *q, const int *p)
{
    for (int i = 0; i < m; ++i) {
        int qi = q ? q[i] : 1;
        if (qi == 2 && p[i] != 0)
            return 0;
        int zeros = (qi == 0) + (p[(i + m - 1) % m] == 0) + (p[(i + 1) % m] == 0);
        if (p[i] == 2 && zeros != 1)
            return 0;
        if (p[i] == 1 && zeros < 2)
            return 0;
    }
    return 1;
}

int oracle_cyclic_follows(int m, uint32_t q_code, uint32_t p_code)
{
    int q[MAXN], p[MAXN];
    if (m < 3 || m > MAXN)
        return 0;
    decode(q_code, m, q);
    decode(p_code, m, p);
    return cyclic_follows_letters(m, q, p);
}

/* The first column of the walk: p labelled from its own column only. */
int oracle_cyclic_can_start(int m, uint32_t p_code)
{
    int p[MAXN];
    if (m < 3 || m > MAXN)
        return 0;
    decode(p_code, m, p);
    return cyclic_follows_letters(m, NULL, p);
}

/* The last column of the walk: no letter 2. */
int oracle_cyclic_can_end(int m, uint32_t p_code)
{
    int p[MAXN];
    if (m < 3 || m > MAXN)
        return 0;
    decode(p_code, m, p);
    for (int i = 0; i < m; ++i)
        if (p[i] == 2)
            return 0;
    return 1;
}

/* The column digraph's matrix for cyclic columns (Algorithm 1 with the rules
 * above): A[q][p] = zeros(p) if p can follow q, else INF; N x N int32,
 * leading dimension N.  Returns N, or -1 on bad m. */
int64_t oracle_cyclic_state_matrix(int m, int32_t inf, int32_t *A)
{
    int64_t N = oracle_cyclic_words(m, NULL);
    if (N < 0)
        return -1;
    uint32_t *w = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    oracle_cyclic_words(m, w);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j)
            A[i * N + j] = oracle_cyclic_follows(m, w[i], w[j]) ? oracle_zeros(m, w[j]) : inf;
    free(w);
    return N;
}

/* The boundary vectors of the open walk: start[p] = zeros(p) if p may be the
 * first column, else INF; end[p] = 0 if p may be the last column, else INF.
 * Returns N, or -1 on bad m. */
int64_t oracle_cyclic_boundary(int m, int32_t inf, int32_t *start, int32_t *end)
{
    int64_t N = oracle_cyclic_words(m, NULL);
    if (N < 0)
        return -1;
    uint32_t *w = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    oracle_cyclic_words(m, w);
    for (int64_t j = 0; j < N; ++j) {
        start[j] = oracle_cyclic_can_start(m, w[j]) ? oracle_zeros(m, w[j]) : inf;
        end[j] = oracle_cyclic_can_end(m, w[j]) ? 0 : inf;
    }
    free(w);
    return N;
}

/* gamma_2(P_k x C_m) for k = 1..nmax by the vector chain x_1 = start,
 * x_(k+1) = x_k x A (a 1 x N by N x N product of Section 1), each answer
 * min_p x_k[p] + end[p] saturated at INF.  Returns N, or -1 on bad
 * arguments. */
int64_t oracle_path_gamma2_sweep(int m, int nmax, int32_t inf, int32_t *gam)
{
    int64_t N = oracle_cyclic_words(m, NULL);
    if (N < 0 || nmax < 1)
        return -1;
    int32_t *A = (int32_t *)malloc((size_t)N * (size_t)N * sizeof(int32_t));
    int32_t *x = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    int32_t *y = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    int32_t *e = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    oracle_cyclic_state_matrix(m, inf, A);
    oracle_cyclic_boundary(m, inf, x, e);
    for (int k = 1; k <= nmax; ++k) {
        if (k > 1) {
            oracle_minplus(1, N, N, x, N, A, N, y, N, inf);
            int32_t *t = x;
            x = y;
            y = t;
        }
        int32_t best = inf;
        for (int64_t j = 0; j < N; ++j) {
            int32_t s = x[j] + e[j];
            if (s > inf)
                s = inf;
            if (s < best)
                best = s;
        }
        gam[k - 1] = best;
    }
    free(A);
    free(x);
    free(y);
    free(e);
    return N;
}
