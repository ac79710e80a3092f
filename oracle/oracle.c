/*
 * oracle.c -- plain, slow CPU reference for multiple-double polynomial
 * evaluation and differentiation at truncated power series.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP path (no headers, helpers or tables): both follow the same written
 * specification of the multiple-double operations and of the operation
 * order, independently.
 *
 * What it computes (Verschelde, "Accelerated polynomial evaluation and
 * differentiation at power series in multiple double precision"):
 *   p = a_0 + sum_k a_k * z_{i_1} * ... * z_{i_{n_k}}        (Section 4, eq. (3))
 * and all partial derivatives dp/dz_i, where every product is the truncated
 * convolution of eq. (1) (Section 2), in m-fold double arithmetic.
 *
 * Coefficients and inputs are real m-doubles, or complex ones whose real and
 * imaginary parts are kept apart (Sections 2 and 5); see cmd_mul below.
 * Monomials may carry exponents: a_k prod z^e is the multilinear monomial with
 * the common factor a_k prod z^(e-1) from a table of powers (Section 3), and
 * each partial derivative is e times the multilinear one.
 *
 * Per monomial it runs the forward / backward / cross product recipe of
 * Section 3 (statement list and the n=5 example, eq. (2)), with the index
 * readings listed in the design notes: the forward chain multiplies by
 * z_{i_j}; the cross product c_j uses b_{n-2-j}.  Contributions are added
 * with the pairwise tree of Section 5 (adjacent pairs, odd element carried),
 * in the order fixed by the worked example (Section 4, the two addition steps
 * after eq. (5)).  Plain loops, no jobs, no layers.
 *
 * Multiple-double arithmetic (m limbs, limb 0 most significant) follows the
 * project's specification, built from published error-free transformations:
 *   two_sum  -- Knuth's branch-free TwoSum (6 flops, exact);
 *   two_prod -- p = RN(a*b), e = fma(a, b, -p) (exact);
 *   deposit  -- add a term into a per-level running sum S[lo], pushing each
 *               exact error one level down; the last level adds plainly;
 *   renorm   -- bottom-up TwoSum pass, then top-down TwoSum pass.
 * Compile with -ffp-contract=off and without fast-math: every + - * is one
 * IEEE binary64 round-to-nearest operation and fma() is the fused one.
 *
 * Parity pins: tests compare this file against exact rational arithmetic
 * (Python fractions), closed forms and integer-exact cases; see tests/.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXM 10
#define MAX_EXPONENT 64

/* ---------------------------------------------------------------- md ops -- */

static void two_sum(double a, double b, double *s, double *e)
{
    double ss = a + b;
    double bb = ss - a;
    double err = (a - (ss - bb)) + (b - bb);
    *s = ss;
    *e = err;
}

static void two_prod(double a, double b, double *p, double *e)
{
    double pp = a * b;
    *e = fma(a, b, -pp);
    *p = pp;
}

/* Add t into the level sums S[lo..m-1]: exact at levels lo..m-2, rounded at m-1. */
static void deposit(int m, double *S, int lo, double t)
{
    for (int j = lo; j < m - 1; ++j)
        two_sum(S[j], t, &S[j], &t);
    S[m - 1] = S[m - 1] + t;
}

/* Turn level sums S[0..m-1] into an m-limb expansion r (value preserved exactly). */
static void renorm(int m, const double *S, double *r)
{
    double u[MAXM];
    if (m == 1) {
        r[0] = S[0];
        return;
    }
    double s = S[m - 1];
    for (int j = m - 2; j >= 0; --j)
        two_sum(S[j], s, &s, &u[j + 1]);
    u[0] = s;
    r[0] = u[0];
    double e = u[1];
    for (int j = 1; j <= m - 2; ++j)
        two_sum(e, u[j + 1], &r[j], &e);
    r[m - 1] = e;
}

/* z = x + y in m-double arithmetic; z may alias x or y. */
static void md_add(int m, const double *x, const double *y, double *z)
{
    double S[MAXM];
    for (int k = 0; k < m; ++k)
        S[k] = x[k];
    for (int k = 0; k < m; ++k)
        deposit(m, S, k, y[k]);
    renorm(m, S, z);
}

/* z = x * y in m-double arithmetic (truncated product); z may alias x or y. */
static void md_mul(int m, const double *x, const double *y, double *z)
{
    double S[MAXM], E[MAXM], p, e;
    /* level k <= m-2 starts with the exact product x_0*y_k */
    for (int k = 0; k <= m - 2; ++k)
        two_prod(x[0], y[k], &S[k], &E[k]);
    /* last level: the products of level m-1, then those of level m */
    S[m - 1] = x[0] * y[m - 1];
    for (int i = 1; i <= m - 1; ++i)
        S[m - 1] = fma(x[i], y[m - 1 - i], S[m - 1]);
    for (int i = 1; i <= m - 1; ++i)
        S[m - 1] = fma(x[i], y[m - i], S[m - 1]);
    /* the low parts of x_0*y_k belong one level down */
    for (int k = 0; k <= m - 2; ++k)
        deposit(m, S, k + 1, E[k]);
    /* the remaining exact products x_i*y_{k-i}, i >= 1, of levels 1..m-2 */
    for (int k = 1; k <= m - 2; ++k) {
        for (int i = 1; i <= k; ++i) {
            two_prod(x[i], y[k - i], &p, &e);
            deposit(m, S, k, p);
            deposit(m, S, k + 1, e);
        }
    }
    renorm(m, S, z);
}

/* ------------------------------------------------- complex m-doubles -- */
/*
 * Complex coefficients (Section 2 and Section 5 keep real and imaginary parts
 * in separate arrays): a complex m-double is its real part, an m-double, then
 * its imaginary part, 2m doubles.  The product is the textbook
 *   (xr + xi i)(yr + yi i) = (xr yr - xi yi) + (xr yi + xi yr) i
 * with every product one md_mul; the real part is md_add(xr yr, -(xi yi)),
 * where the negation flips the sign of every limb (exact), and the imaginary
 * part is md_add(xr yi, xi yr).  The sum adds the two parts separately.
 * z may alias x or y.
 */
static void cmd_mul(int m, const double *x, const double *y, double *z)
{
    double rr[MAXM], ii[MAXM], ri[MAXM], ir[MAXM];
    md_mul(m, x, y, rr);
    md_mul(m, x + m, y + m, ii);
    md_mul(m, x, y + m, ri);
    md_mul(m, x + m, y, ir);
    for (int l = 0; l < m; ++l)
        ii[l] = -ii[l];
    md_add(m, rr, ii, z);
    md_add(m, ri, ir, z + m);
}

static void cmd_add(int m, const double *x, const double *y, double *z)
{
    md_add(m, x, y, z);
    md_add(m, x + m, y + m, z + m);
}

/* One coefficient operation of the series' number field: cx = 0 real, 1 complex. */
static void coef_mul(int m, int cx, const double *x, const double *y, double *z)
{
    if (cx)
        cmd_mul(m, x, y, z);
    else
        md_mul(m, x, y, z);
}

static void coef_add(int m, int cx, const double *x, const double *y, double *z)
{
    if (cx)
        cmd_add(m, x, y, z);
    else
        md_add(m, x, y, z);
}

/* x := e * x for a small positive integer e: one md_mul by the m-double
 * (e, 0, ..., 0); a complex x scales both parts. */
static void coef_scale(int m, int cx, double *x, int e)
{
    double E[MAXM] = {0};
    E[0] = (double)e;
    md_mul(m, x, E, x);
    if (cx)
        md_mul(m, x + m, E, x + m);
}

/* ------------------------------------------------------------ series ops -- */
/* A series is (d+1) coefficients of w doubles, w = m (real) or 2m (complex:
 * real limbs, then imaginary limbs): s[c*w + l]. */

/* z = x * y truncated at degree d (Section 2, eq. (1)): for each k,
 * z_k = x_0*y_k, then z_k += x_i*y_{k-i} for i = 1..k in increasing i.
 * z may alias x or y (the in-place update b := b * a of Section 3). */
static void conv(int m, int cx, int d, const double *x, const double *y, double *z, double *tmp)
{
    const size_t w = (size_t)m << cx;
    double p[2 * MAXM];
    for (int k = 0; k <= d; ++k) {
        double *acc = tmp + (size_t)k * w;
        coef_mul(m, cx, x, y + (size_t)k * w, acc);
        for (int i = 1; i <= k; ++i) {
            coef_mul(m, cx, x + (size_t)i * w, y + (size_t)(k - i) * w, p);
            coef_add(m, cx, acc, p, acc);
        }
    }
    memcpy(z, tmp, sizeof(double) * (size_t)(d + 1) * w);
}

/* upd := upd + inp, coefficientwise (Section 2, last paragraph; Section 5 addition job). */
static void series_add(int m, int cx, int d, double *upd, const double *inp)
{
    const size_t w = (size_t)m << cx;
    for (int k = 0; k <= d; ++k)
        coef_add(m, cx, upd + (size_t)k * w, inp + (size_t)k * w, upd + (size_t)k * w);
}

/* ---------------------------------------------------------- layout glue -- */

/* planar [w][count][d+1] -> series-major [count][(d+1)*w]; w = m, or 2m for
 * complex data, whose planes are the m real limbs, then the m imaginary ones */
static void from_planar(int m, int d, int count, const double *src, double *dst)
{
    for (int s = 0; s < count; ++s)
        for (int c = 0; c <= d; ++c)
            for (int l = 0; l < m; ++l)
                dst[((size_t)s * (d + 1) + c) * m + l] = src[((size_t)l * count + s) * (d + 1) + c];
}

static void to_planar(int m, int d, int count, int idx, const double *ser, double *dst)
{
    for (int c = 0; c <= d; ++c)
        for (int l = 0; l < m; ++l)
            dst[((size_t)l * count + idx) * (d + 1) + c] = ser[(size_t)c * m + l];
}

/* --------------------------------------------------------- monomial AD -- */

/*
 * Evaluate and differentiate one monomial a * z_{v[0]} * ... * z_{v[nk-1]}
 * (Section 3, with the readings noted above).  Writes the value series to
 * val and the partial derivative with respect to z_{v[j]} to der[j].
 * Z holds the n input series (series-major).  Work arrays: f, b, c of
 * nk series each, tmp one series.
 */
static void monomial(int m, int cx, int d, int nk, const int *v, const double *a, const double *Z,
                     double *val, double **der, double *f, double *b, double *c, double *tmp)
{
    const size_t S = (size_t)(d + 1) * ((size_t)m << cx);
#define ZS(idx) (Z + (size_t)(idx) * S)
#define F(j) (f + (size_t)((j) - 1) * S)  /* 1-based as in the paper */
#define B(j) (b + (size_t)((j) - 1) * S)
#define C(j) (c + (size_t)((j) - 1) * S)
#define I(j) (v[(j) - 1])                  /* i_j, 1-based position */
    const int n = nk;
    if (n == 1) {
        conv(m, cx, d, a, ZS(I(1)), F(1), tmp);
        memcpy(val, F(1), sizeof(double) * S);
        memcpy(der[0], a, sizeof(double) * S);
        return;
    }
    /* forward products: f_1 = a * z_{i_1}; f_j = f_{j-1} * z_{i_j} */
    conv(m, cx, d, a, ZS(I(1)), F(1), tmp);
    for (int j = 2; j <= n; ++j)
        conv(m, cx, d, F(j - 1), ZS(I(j)), F(j), tmp);
    if (n == 2) {
        /* b_1 = z_{i_2} * a (the n_k = 2 case of Section 5) */
        conv(m, cx, d, ZS(I(2)), a, B(1), tmp);
        memcpy(val, F(2), sizeof(double) * S);
        memcpy(der[0], B(1), sizeof(double) * S);
        memcpy(der[1], F(1), sizeof(double) * S);
        return;
    }
    /* backward products: b_1 = z_{i_n} * z_{i_{n-1}}; b_j = b_{j-1} * z_{i_{n-j}};
       then b_{n-2} := b_{n-2} * a */
    conv(m, cx, d, ZS(I(n)), ZS(I(n - 1)), B(1), tmp);
    for (int j = 2; j <= n - 2; ++j)
        conv(m, cx, d, B(j - 1), ZS(I(n - j)), B(j), tmp);
    conv(m, cx, d, B(n - 2), a, B(n - 2), tmp);
    /* cross products: c_j = f_j * b_{n-2-j} for j = 1..n-3; c_{n-2} = f_{n-2} * z_{i_n} */
    for (int j = 1; j <= n - 3; ++j)
        conv(m, cx, d, F(j), B(n - 2 - j), C(j), tmp);
    conv(m, cx, d, F(n - 2), ZS(I(n)), C(n - 2), tmp);
    /* value f_n; d/dz_{i_1} = b_{n-2}; d/dz_{i_{j+1}} = c_j; d/dz_{i_n} = f_{n-1} */
    memcpy(val, F(n), sizeof(double) * S);
    memcpy(der[0], B(n - 2), sizeof(double) * S);
    for (int j = 1; j <= n - 2; ++j)
        memcpy(der[j], C(j), sizeof(double) * S);
    memcpy(der[n - 1], F(n - 1), sizeof(double) * S);
#undef ZS
#undef F
#undef B
#undef C
#undef I
}

/*
 * Pairwise tree sum of a list of series (Section 5, addition jobs):
 * in each round, element 2p+1 := element 2p+1 + element 2p for every pair,
 * the survivors are the odd-positioned elements plus a carried last element
 * when the count is odd.  The result ends in the last element of the list.
 */
static void tree_sum(int m, int cx, int d, int len, double **items)
{
    int r = len;
    double **live = (double **)malloc(sizeof(double *) * (size_t)(len > 0 ? len : 1));
    for (int i = 0; i < len; ++i)
        live[i] = items[i];
    while (r > 1) {
        int w = 0;
        for (int p = 0; p < r / 2; ++p) {
            series_add(m, cx, d, live[2 * p + 1], live[2 * p]);
            live[w++] = live[2 * p + 1];
        }
        if (r % 2)
            live[w++] = live[r - 1];
        r = w;
    }
    free(live);
}

/* The schedule of tree_sum as pairs (input index, updated index) per round. */
int oracle_tree_schedule(int len, int *pairs, int *round_sizes, int max_rounds)
{
    int *live = (int *)malloc(sizeof(int) * (size_t)(len > 0 ? len : 1));
    int r = len, np = 0, nr = 0;
    for (int i = 0; i < len; ++i)
        live[i] = i;
    while (r > 1) {
        int w = 0;
        if (nr >= max_rounds) {
            free(live);
            return -1;
        }
        round_sizes[nr] = r / 2;
        for (int p = 0; p < r / 2; ++p) {
            pairs[2 * np] = live[2 * p];
            pairs[2 * np + 1] = live[2 * p + 1];
            ++np;
            live[w++] = live[2 * p + 1];
        }
        if (r % 2)
            live[w++] = live[r - 1];
        r = w;
        ++nr;
    }
    free(live);
    return nr;
}

/* ------------------------------------------------------------ the oracle -- */

static int check_support(int n, int N, const int *nvars, const int *vars)
{
    size_t pos = 0;
    if (n < 0 || N < 0)
        return -1;
    for (int k = 0; k < N; ++k) {
        if (nvars[k] < 1 || nvars[k] > n)
            return -1;
        for (int j = 0; j < nvars[k]; ++j) {
            int vj = vars[pos + j];
            if (vj < 0 || vj >= n)
                return -1;
            if (j > 0 && vj <= vars[pos + j - 1])
                return -1;
        }
        pos += nvars[k];
    }
    return 0;
}

/*
 * value [w][d+1], grad [w][n][d+1]; coeff [w][N+1][d+1] (a_0 first); z [w][n][d+1],
 * with w = m planes of real limbs, or (cx = 1) w = 2m planes: the m real limbs,
 * then the m imaginary limbs.  exps: NULL (every exponent one), or [sum n_k]
 * exponents 1..64 aligned with vars: monomial k is a_k prod_j z_{i_j}^{e_j}.
 * nthreads <= 0 leaves the OpenMP default.  Returns 0, or -1 on a bad support.
 */
int oracle_eval_and_diff_general(int m, int cx, int d, int n, int N, const int *nvars, const int *vars,
                                 const int *exps, const double *coeff, const double *z, double *value,
                                 double *grad, int nthreads)
{
    if (m < 1 || m > MAXM || cx < 0 || cx > 1 || d < 0 || check_support(n, N, nvars, vars))
        return -1;
    const int nl = m << cx; /* doubles per coefficient */
    const size_t S = (size_t)(d + 1) * nl;
    size_t total = 0;
    size_t *start = (size_t *)malloc(sizeof(size_t) * (size_t)(N + 1));
    for (int k = 0; k < N; ++k) {
        start[k] = total;
        total += (size_t)nvars[k];
    }
    start[N] = total;
    double *A = (double *)malloc(sizeof(double) * S * (size_t)(N + 1));
    double *Z = (double *)malloc(sizeof(double) * S * (size_t)(n > 0 ? n : 1));
    double *vals = (double *)malloc(sizeof(double) * S * (size_t)(N + 1));
    double *ders = (double *)malloc(sizeof(double) * S * (total > 0 ? total : 1));
    from_planar(nl, d, N + 1, coeff, A);
    from_planar(nl, d, n, z, Z);
    for (size_t q = 0; exps && q < total; ++q)
        if (exps[q] < 1 || exps[q] > MAX_EXPONENT) {
            free(start);
            free(A);
            free(Z);
            free(vals);
            free(ders);
            return -1;
        }
    /* Table of powers (Section 3, general exponents): P_i^1 = z_i and
     * P_i^p = P_i^{p-1} * z_i up to the largest e - 1 over the occurrences of
     * variable i; powoff[i] locates P_i^1, P_i^p follows at (p-1) series on. */
    int *maxp = (int *)calloc((size_t)(n > 0 ? n : 1), sizeof(int));
    size_t *powoff = (size_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(size_t));
    size_t npow = 0;
    for (size_t q = 0; q < total; ++q) {
        int e = exps ? exps[q] : 1;
        if (e - 1 > maxp[vars[q]])
            maxp[vars[q]] = e - 1;
    }
    for (int i = 0; i < n; ++i) {
        powoff[i] = npow;
        npow += (size_t)maxp[i];
    }
    double *Pt = (double *)malloc(sizeof(double) * S * (npow > 0 ? npow : 1));
    {
        double *tmp = (double *)malloc(sizeof(double) * S);
        for (int i = 0; i < n; ++i) {
            if (maxp[i] == 0)
                continue;
            double *P1 = Pt + powoff[i] * S;
            memcpy(P1, Z + (size_t)i * S, sizeof(double) * S);
            for (int p = 2; p <= maxp[i]; ++p)
                conv(m, cx, d, P1 + (size_t)(p - 2) * S, Z + (size_t)i * S, P1 + (size_t)(p - 1) * S, tmp);
        }
        free(tmp);
    }
    /* value list starts with a_0 */
    memcpy(vals, A, sizeof(double) * S);
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        int nmax = 1;
        for (int k = 0; k < N; ++k)
            if (nvars[k] > nmax)
                nmax = nvars[k];
        double *work = (double *)malloc(sizeof(double) * S * (size_t)(3 * nmax + 2));
        double **der = (double **)malloc(sizeof(double *) * (size_t)nmax);
        double *F = work + S * (size_t)(3 * nmax + 1);
#pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < N; ++k) {
            int nk = nvars[k];
            const int *v = vars + start[k];
            const int *e = exps ? exps + start[k] : NULL;
            /* common factor F = a_k * prod_j z_{i_j}^{e_j - 1}, in increasing j
               (a_k itself when every exponent is one) */
            memcpy(F, A + (size_t)(k + 1) * S, sizeof(double) * S);
            for (int j = 0; j < nk; ++j)
                if (e && e[j] >= 2)
                    conv(m, cx, d, F, Pt + (powoff[v[j]] + (size_t)(e[j] - 2)) * S, F, work + S * (size_t)(3 * nmax));
            for (int j = 0; j < nk; ++j)
                der[j] = ders + (start[k] + (size_t)j) * S;
            monomial(m, cx, d, nk, v, F, Z, vals + (size_t)(k + 1) * S, der,
                     work, work + S * (size_t)nmax, work + 2 * S * (size_t)nmax, work + 3 * S * (size_t)nmax);
            /* d/dz_{i_j} of a z^e factor: e_j times the multilinear derivative */
            for (int j = 0; j < nk; ++j)
                if (e && e[j] >= 2)
                    for (int c = 0; c <= d; ++c)
                        coef_scale(m, cx, der[j] + (size_t)c * nl, e[j]);
        }
        free(work);
        free(der);
    }
    /* value: tree over [a_0, f_{1,n_1}, ..., f_{N,n_N}] */
    {
        double **items = (double **)malloc(sizeof(double *) * (size_t)(N + 1));
        for (int k = 0; k <= N; ++k)
            items[k] = vals + (size_t)k * S;
        tree_sum(m, cx, d, N + 1, items);
        to_planar(nl, d, 1, 0, items[N], value);
        free(items);
    }
    /* gradient: list i holds the d/dz_i contributions in increasing monomial order */
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n; ++i) {
        int len = 0;
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < nvars[k]; ++j)
                if (vars[start[k] + j] == i)
                    ++len;
        if (len == 0) {
            for (int l = 0; l < nl; ++l)
                for (int c = 0; c <= d; ++c)
                    grad[((size_t)l * n + i) * (d + 1) + c] = 0.0;
            continue;
        }
        double **items = (double **)malloc(sizeof(double *) * (size_t)len);
        int w = 0;
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < nvars[k]; ++j)
                if (vars[start[k] + j] == i)
                    items[w++] = ders + (start[k] + (size_t)j) * S;
        tree_sum(m, cx, d, len, items);
        to_planar(nl, d, n, i, items[len - 1], grad);
        free(items);
    }
    free(start);
    free(A);
    free(Z);
    free(vals);
    free(ders);
    free(maxp);
    free(powoff);
    free(Pt);
    return 0;
}

/* The multilinear real case: value [m][d+1], grad [m][n][d+1]; coeff [m][N+1][d+1]; z [m][n][d+1]. */
int oracle_eval_and_diff(int m, int d, int n, int N, const int *nvars, const int *vars,
                         const double *coeff, const double *z, double *value, double *grad,
                         int nthreads)
{
    return oracle_eval_and_diff_general(m, 0, d, n, N, nvars, vars, NULL, coeff, z, value, grad, nthreads);
}

/* --------------------------------------------------------- the adjoint -- */
/*
 * Reverse pass for an upstream adjoint series ybar of the value series:
 * L = sum_t ybar_t p_t.  p is linear in every input series, p = z_i * g_i + (terms
 * free of z_i) with g_i = dp/dz_i, and p = a_k * M_k + (terms free of a_k) with
 * M_k = prod_{j in monomial k} z_j (eq. (3)); a coefficient s of z_i or a_k then
 * enters p_t through the coefficient t-s of g_i or M_k (eq. (1)), so
 *   zbar_i[s] = sum_{j=0..d-s} ybar[s+j] g_i[j],   abar_k[s] = sum_j ybar[s+j] M_k[j],
 *   abar_0 = ybar.
 * Each correlation coefficient s is md_mul(ybar_s, y_0), then
 * += md_mul(ybar_{s+j}, y_j) for j = 1..d-s, in increasing j.
 * M_k is built like the backward products before the multiplication by a_k:
 * n_k = 1: z_{i_1};  n_k = 2: z_{i_2} * z_{i_1};  n_k >= 3: b = z_{i_n} * z_{i_{n-1}},
 * b := b * z_{i_{n-j}} for j = 2..n-2, then M_k = b * z_{i_1}.
 */
static void corr(int m, int d, const double *x, const double *y, double *out)
{
    double p[MAXM];
    for (int s = 0; s <= d; ++s) {
        double *acc = out + (size_t)s * m;
        md_mul(m, x + (size_t)s * m, y, acc);
        for (int j = 1; j <= d - s; ++j) {
            md_mul(m, x + (size_t)(s + j) * m, y + (size_t)j * m, p);
            md_add(m, acc, p, acc);
        }
    }
}

static void monomial_product(int m, int d, int nk, const int *v, const double *Z, double *M, double *b,
                             double *tmp)
{
    const size_t S = (size_t)(d + 1) * m;
#define ZS(idx) (Z + (size_t)(idx) * S)
    if (nk == 1) {
        memcpy(M, ZS(v[0]), sizeof(double) * S);
        return;
    }
    if (nk == 2) {
        conv(m, 0, d, ZS(v[1]), ZS(v[0]), M, tmp);
        return;
    }
    conv(m, 0, d, ZS(v[nk - 1]), ZS(v[nk - 2]), b, tmp);
    for (int j = 2; j <= nk - 2; ++j)
        conv(m, 0, d, b, ZS(v[nk - 1 - j]), b, tmp);
    conv(m, 0, d, b, ZS(v[0]), M, tmp);
#undef ZS
}

/* coeff_bar [m][N+1][d+1], z_bar [m][n][d+1]; ybar [m][d+1]; grad as returned by
 * oracle_eval_and_diff for the same inputs. */
int oracle_eval_adjoint(int m, int d, int n, int N, const int *nvars, const int *vars, const double *z,
                        const double *grad, const double *ybar, double *coeff_bar, double *z_bar, int nthreads)
{
    if (m < 1 || m > MAXM || d < 0 || check_support(n, N, nvars, vars))
        return -1;
    const size_t S = (size_t)(d + 1) * m;
    size_t *start = (size_t *)malloc(sizeof(size_t) * (size_t)(N + 1));
    size_t tot = 0;
    for (int k = 0; k < N; ++k) {
        start[k] = tot;
        tot += (size_t)nvars[k];
    }
    double *Z = (double *)malloc(sizeof(double) * S * (size_t)(n > 0 ? n : 1));
    double *G = (double *)malloc(sizeof(double) * S * (size_t)(n > 0 ? n : 1));
    double *Y = (double *)malloc(sizeof(double) * S);
    from_planar(m, d, n, z, Z);
    from_planar(m, d, n, grad, G);
    from_planar(m, d, 1, ybar, Y);
    to_planar(m, d, N + 1, 0, Y, coeff_bar);
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        double *M = (double *)malloc(sizeof(double) * S * 4);
        double *b = M + S, *tmp = M + 2 * S, *out = M + 3 * S;
#pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < N; ++k) {
            monomial_product(m, d, nvars[k], vars + start[k], Z, M, b, tmp);
            corr(m, d, Y, M, out);
            to_planar(m, d, N + 1, k + 1, out, coeff_bar);
        }
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < n; ++i) {
            int present = 0;
            for (size_t q = 0; q < tot; ++q)
                if (vars[q] == i)
                    present = 1;
            if (!present) {
                for (int l = 0; l < m; ++l)
                    for (int c = 0; c <= d; ++c)
                        z_bar[((size_t)l * n + i) * (d + 1) + c] = 0.0;
                continue;
            }
            corr(m, d, Y, G + (size_t)i * S, out);
            to_planar(m, d, n, i, out, z_bar);
        }
        free(M);
    }
    free(start);
    free(Z);
    free(G);
    free(Y);
    return 0;
}

/* ---------------------------------------------- elementwise entry points -- */
/* x, y, z planar [w][count]; op 0 = add, 1 = mul (w = m); op 2 = complex add,
 * 3 = complex mul (w = 2m: real limbs, then imaginary limbs). */
int oracle_md_op(int op, int m, long count, const double *x, const double *y, double *z)
{
    if (m < 1 || m > MAXM || count < 0 || op < 0 || op > 3)
        return -1;
    const int cx = op >= 2, w = m << cx;
    for (long i = 0; i < count; ++i) {
        double a[2 * MAXM], b[2 * MAXM], r[2 * MAXM];
        for (int l = 0; l < w; ++l) {
            a[l] = x[(size_t)l * count + i];
            b[l] = y[(size_t)l * count + i];
        }
        if (op % 2 == 0)
            coef_add(m, cx, a, b, r);
        else
            coef_mul(m, cx, a, b, r);
        for (int l = 0; l < w; ++l)
            z[(size_t)l * count + i] = r[l];
    }
    return 0;
}

/* The two_sum / two_prod transforms themselves, planar [count]. */
int oracle_eft(int op, long count, const double *a, const double *b, double *hi, double *lo)
{
    for (long i = 0; i < count; ++i) {
        if (op == 0)
            two_sum(a[i], b[i], &hi[i], &lo[i]);
        else
            two_prod(a[i], b[i], &hi[i], &lo[i]);
    }
    return 0;
}

/*
 * Operation counts of md_add and md_mul for m limbs, obtained by walking the
 * same loops as above and counting instead of computing.
 * counts[0..3] = {add/sub, mul, fma, two_sum calls} for op (0 add, 1 mul).
 */
int oracle_op_counts(int op, int m, long *counts)
{
    long add = 0, mul = 0, fmas = 0, ts = 0;
    if (m < 1 || m > MAXM)
        return -1;
#define TS() (ts++, add += 6)
#define DEP(lo) do { for (int j_ = (lo); j_ < m - 1; ++j_) TS(); add += 1; } while (0)
    if (op == 0) {
        for (int k = 0; k < m; ++k)
            DEP(k);
    } else {
        for (int k = 0; k <= m - 2; ++k) { mul += 1; fmas += 1; }
        mul += 1;
        fmas += 2 * (m - 1);
        for (int k = 0; k <= m - 2; ++k)
            DEP(k + 1);
        for (int k = 1; k <= m - 2; ++k)
            for (int i = 1; i <= k; ++i) {
                mul += 1; fmas += 1;
                DEP(k);
                DEP(k + 1);
            }
    }
    if (m > 1) {
        for (int j = m - 2; j >= 0; --j) TS();
        for (int j = 1; j <= m - 2; ++j) TS();
    }
#undef TS
#undef DEP
    counts[0] = add;
    counts[1] = mul;
    counts[2] = fmas;
    counts[3] = ts;
    return 0;
}
