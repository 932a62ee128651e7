/* Body of the CPU oracle, instantiated once per floating-point type.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the solver library links this code.
 *
 * The includer defines
 *   REAL  - the arithmetic type (double or long double)
 *   SFX   - the symbol suffix (e.g. _f64, _ld)
 * Inputs and outputs are always double; REAL is only the working precision.
 *
 * Notation (paper, Sec. 2): X x_mu A is the mu-mode product, Y_(mu) = A X_(mu),
 * i.e. Y[.., i_mu, ..] = sum_j A[i_mu, j] X[.., j, ..].
 * Tensors are stored row-major: the last mode is the fastest.
 */
#define CAT_(a, b) a##b
#define CAT(a, b) CAT_(a, b)
#define FN(name) CAT(name, SFX)

/* Solve the s x s system M x = r in place by Gaussian elimination with
 * partial pivoting.  Returns 0 on success, ORC_SINGULAR on an exactly zero
 * pivot or a non-finite result. */
static int FN(small_gepp)(int s, REAL* M /* s*s row-major */, REAL* r) {
    for (int k = 0; k < s; ++k) {
        int piv = k;
        REAL best = M[k * s + k] < 0 ? -M[k * s + k] : M[k * s + k];
        for (int i = k + 1; i < s; ++i) {
            REAL v = M[i * s + k] < 0 ? -M[i * s + k] : M[i * s + k];
            if (v > best) { best = v; piv = i; }
        }
        if (best == 0) return ORC_SINGULAR;
        if (piv != k) {
            for (int j = 0; j < s; ++j) { REAL t = M[k * s + j]; M[k * s + j] = M[piv * s + j]; M[piv * s + j] = t; }
            REAL t = r[k]; r[k] = r[piv]; r[piv] = t;
        }
        for (int i = k + 1; i < s; ++i) {
            REAL f = M[i * s + k] / M[k * s + k];
            for (int j = k; j < s; ++j) M[i * s + j] -= f * M[k * s + j];
            r[i] -= f * r[k];
        }
    }
    for (int k = s - 1; k >= 0; --k) {
        REAL acc = r[k];
        for (int j = k + 1; j < s; ++j) acc -= M[k * s + j] * r[j];
        r[k] = acc / M[k * s + k];
        if (!isfinite((double)r[k])) return ORC_SINGULAR;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Laplace-like operator, eq. (1.4)/(2.2):  sum_mu X x_mu T_mu = B,
 * with every T_mu upper quasi-triangular (real Schur form, Sec. 2).
 *
 * The solution is unique when no sum of eigenvalues lambda_1+...+lambda_d
 * vanishes (Sec. 2).  The oracle computes it by plain block back-substitution
 * on the assembled operator without ever forming it:
 *   - each mode is partitioned into its 1x1 and 2x2 diagonal blocks;
 *   - a tuple p = (p_1..p_d) of such blocks couples only to tuples q >= p
 *     (componentwise), because every T_mu is block upper triangular;
 *   - tuples are visited so that every tuple q >= p is finished before p
 *     (hyperplanes sum(p) = const in decreasing order; tuples on one
 *     hyperplane never couple, so each hyperplane is a parallel loop);
 *   - for each element i of the tuple,
 *        r_i = B_i - sum_mu sum_{j beyond block p_mu} T_mu[i_mu, j] X[i with i_mu := j];
 *   - the <= 2^d unknowns of the tuple then solve
 *        (sum_mu I (x) .. (x) T_mu[p_mu, p_mu] (x) .. (x) I) x = r.
 * With trans != 0 the coefficients are T_mu^T (lower quasi-triangular) and
 * the tuples are visited in increasing order: this is the adjoint equation
 * sum_mu L x_mu T_mu^T = G.
 * ---------------------------------------------------------------------- */
int FN(oracle_lap_solve)(int d, const int64_t* n, const double* const* T,
                         const double* B, double* X, int trans) {
    int64_t stride[ORC_MAXD], N = 1;
    for (int mu = d - 1; mu >= 0; --mu) { stride[mu] = N; N *= n[mu]; }
    if (N == 0) return 0;
    /* Block partition per mode. */
    int64_t* bstart[ORC_MAXD];
    int64_t nb[ORC_MAXD];
    int rc = 0;
    for (int mu = 0; mu < d; ++mu) {
        bstart[mu] = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n[mu] + 1));
        if (orc_partition(n[mu], T[mu], bstart[mu], &nb[mu]) != 0) rc = ORC_INVALID;
    }
    if (rc) { for (int mu = 0; mu < d; ++mu) free(bstart[mu]); return rc; }

    REAL* Xw = (REAL*)malloc(sizeof(REAL) * (size_t)N);
    int64_t smax = 0;
    for (int mu = 0; mu < d; ++mu) smax += nb[mu] - 1;
    int64_t lead = 1; /* number of (p_0..p_{d-2}) combinations */
    for (int mu = 0; mu < d - 1; ++mu) lead *= nb[mu];
    int failed = 0;

    for (int64_t step = 0; step <= smax && !failed; ++step) {
        int64_t s = trans ? step : smax - step;
        #pragma omp parallel for schedule(dynamic, 64) reduction(|: failed)
        for (int64_t lin = 0; lin < lead; ++lin) {
            int64_t p[ORC_MAXD];
            int64_t rem = lin, acc = 0;
            for (int mu = d - 2; mu >= 0; --mu) { p[mu] = rem % nb[mu]; rem /= nb[mu]; acc += p[mu]; }
            int64_t last = s - acc;
            if (last < 0 || last >= nb[d - 1]) continue;
            p[d - 1] = last;
            /* Tuple geometry. */
            int64_t st[ORC_MAXD], sz[ORC_MAXD];
            int ne = 1;
            for (int mu = 0; mu < d; ++mu) {
                st[mu] = bstart[mu][p[mu]];
                sz[mu] = bstart[mu][p[mu] + 1] - st[mu];
                ne *= (int)sz[mu];
            }
            REAL r[ORC_MAXE], M[ORC_MAXE * ORC_MAXE];
            int64_t off[ORC_MAXE];
            for (int e = 0; e < ne; ++e) {
                /* local digits: mode 0 slowest */
                int64_t idx[ORC_MAXD];
                int rr = e;
                for (int mu = d - 1; mu >= 0; --mu) { idx[mu] = st[mu] + rr % sz[mu]; rr /= (int)sz[mu]; }
                int64_t o = 0;
                for (int mu = 0; mu < d; ++mu) o += idx[mu] * stride[mu];
                off[e] = o;
                REAL acc2 = (REAL)B[o];
                for (int mu = 0; mu < d; ++mu) {
                    const double* Tm = T[mu];
                    int64_t nm = n[mu], i = idx[mu];
                    if (!trans) {
                        for (int64_t j = st[mu] + sz[mu]; j < nm; ++j)
                            acc2 -= (REAL)Tm[i * nm + j] * Xw[o + (j - i) * stride[mu]];
                    } else {
                        for (int64_t j = 0; j < st[mu]; ++j)
                            acc2 -= (REAL)Tm[j * nm + i] * Xw[o + (j - i) * stride[mu]];
                    }
                }
                r[e] = acc2;
            }
            /* Diagonal coupling of the tuple's unknowns. */
            for (int e = 0; e < ne; ++e) {
                int64_t ie[ORC_MAXD];
                int re = e;
                for (int mu = d - 1; mu >= 0; --mu) { ie[mu] = re % sz[mu]; re /= (int)sz[mu]; }
                for (int f = 0; f < ne; ++f) {
                    int64_t jf[ORC_MAXD];
                    int rf = f;
                    for (int mu = d - 1; mu >= 0; --mu) { jf[mu] = rf % sz[mu]; rf /= (int)sz[mu]; }
                    REAL m = 0;
                    for (int mu = 0; mu < d; ++mu) {
                        int same = 1;
                        for (int nu = 0; nu < d; ++nu)
                            if (nu != mu && ie[nu] != jf[nu]) same = 0;
                        if (!same) continue;
                        int64_t a = st[mu] + ie[mu], b = st[mu] + jf[mu];
                        m += trans ? (REAL)T[mu][b * n[mu] + a] : (REAL)T[mu][a * n[mu] + b];
                    }
                    M[e * ne + f] = m;
                }
            }
            if (FN(small_gepp)(ne, M, r) != 0) { failed = 1; continue; }
            for (int e = 0; e < ne; ++e) Xw[off[e]] = r[e];
        }
    }
    if (!failed)
        for (int64_t t = 0; t < N; ++t) X[t] = (double)Xw[t];
    free(Xw);
    for (int mu = 0; mu < d; ++mu) free(bstart[mu]);
    return failed ? ORC_SINGULAR : 0;
}

/* Y = sum_mu X x_mu T_mu  (or with T_mu^T when trans != 0), eq. (2.2). */
void FN(oracle_lap_apply)(int d, const int64_t* n, const double* const* T,
                          const double* X, double* Y, int trans) {
    int64_t stride[ORC_MAXD], N = 1;
    for (int mu = d - 1; mu >= 0; --mu) { stride[mu] = N; N *= n[mu]; }
    #pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < N; ++o) {
        REAL acc = 0;
        for (int mu = 0; mu < d; ++mu) {
            int64_t i = (o / stride[mu]) % n[mu], nm = n[mu];
            int64_t base = o - i * stride[mu];
            for (int64_t j = 0; j < nm; ++j) {
                double t = trans ? T[mu][j * nm + i] : T[mu][i * nm + j];
                if (t != 0.0) acc += (REAL)t * (REAL)X[base + j * stride[mu]];
            }
        }
        Y[o] = (double)acc;
    }
}

/* Y = X x_mu M with M an (m x n_mu) row-major matrix; Y has n_mu replaced by m. */
void FN(oracle_mode_product)(int d, const int64_t* n, int mu, const double* M, int64_t m,
                             const double* X, double* Y) {
    int64_t outer = 1, inner = 1;
    for (int nu = 0; nu < mu; ++nu) outer *= n[nu];
    for (int nu = mu + 1; nu < d; ++nu) inner *= n[nu];
    int64_t nm = n[mu];
    /* Y[o, r, q] = sum_j M[r, j] X[o, j, q], the sum taken in increasing j.
     * The q range is cut into chunks of QC columns only so that the
     * X[o, :, chunk] panel a task reads stays in cache (and so that the
     * slowest mode, with outer = 1, still has parallel tasks); every output
     * is the same sum in the same order. */
    const int64_t QC = 64;
    const int64_t nq = (inner + QC - 1) / QC;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t task = 0; task < outer * nq; ++task) {
        const int64_t o = task / nq, q0 = (task % nq) * QC;
        const int64_t q1 = (q0 + QC < inner) ? q0 + QC : inner;
        for (int64_t r = 0; r < m; ++r)
            for (int64_t q = q0; q < q1; ++q) {
                REAL acc = 0;
                for (int64_t j = 0; j < nm; ++j)
                    acc += (REAL)M[r * nm + j] * (REAL)X[(o * nm + j) * inner + q];
                Y[(o * m + r) * inner + q] = (double)acc;
            }
    }
}

/* Pair operator (the two-matrices-per-mode family of the conclusions):
 *   Y = sum_mu X x_1 C_1 ... x_mu A_mu ... x_d C_d.
 * Element-wise: Y[i] = sum_j (sum_mu A_mu[i_mu,j_mu] prod_{nu!=mu} C_nu[i_nu,j_nu]) X[j].
 * Evaluated as d chains of plain mode products. */
void FN(oracle_pair_apply)(int d, const int64_t* n, const double* const* A,
                           const double* const* C, const double* X, double* Y) {
    int64_t N = 1;
    for (int mu = 0; mu < d; ++mu) N *= n[mu];
    double* t0 = (double*)malloc(sizeof(double) * (size_t)N);
    double* t1 = (double*)malloc(sizeof(double) * (size_t)N);
    for (int64_t o = 0; o < N; ++o) Y[o] = 0.0;
    for (int mu = 0; mu < d; ++mu) {
        memcpy(t0, X, sizeof(double) * (size_t)N);
        for (int nu = 0; nu < d; ++nu) {
            FN(oracle_mode_product)(d, n, nu, nu == mu ? A[nu] : C[nu], n[nu], t0, t1);
            double* sw = t0; t0 = t1; t1 = sw;
        }
        for (int64_t o = 0; o < N; ++o) Y[o] += t0[o];
    }
    free(t0); free(t1);
}

/* Pair-form solve by plain block back-substitution on the assembled operator
 * (definition of the unique solution).  A tuple p couples to every element j
 * with j_nu >= start(p_nu) in all modes, so the cost is O(N^2): small sizes
 * only. */
int FN(oracle_pair_solve_direct)(int d, const int64_t* n, const double* const* A,
                                 const double* const* C, const double* B, double* X) {
    int64_t stride[ORC_MAXD], N = 1;
    for (int mu = d - 1; mu >= 0; --mu) { stride[mu] = N; N *= n[mu]; }
    if (N == 0) return 0;
    int64_t* bstart[ORC_MAXD];
    int64_t nb[ORC_MAXD];
    int rc = 0;
    for (int mu = 0; mu < d; ++mu) {
        bstart[mu] = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n[mu] + 1));
        if (orc_partition(n[mu], A[mu], bstart[mu], &nb[mu]) != 0) rc = ORC_INVALID;
        for (int64_t r = 0; r < n[mu]; ++r)
            for (int64_t c = 0; c < r; ++c)
                if (C[mu][r * n[mu] + c] != 0.0) rc = ORC_INVALID;
    }
    if (rc) { for (int mu = 0; mu < d; ++mu) free(bstart[mu]); return rc; }
    REAL* Xw = (REAL*)calloc((size_t)N, sizeof(REAL));
    int64_t smax = 0;
    for (int mu = 0; mu < d; ++mu) smax += nb[mu] - 1;
    int64_t lead = 1;
    for (int mu = 0; mu < d - 1; ++mu) lead *= nb[mu];
    int failed = 0;
    for (int64_t s = smax; s >= 0 && !failed; --s) {
        #pragma omp parallel for schedule(dynamic, 1) reduction(|: failed)
        for (int64_t lin = 0; lin < lead; ++lin) {
            int64_t p[ORC_MAXD];
            int64_t rem = lin, acc = 0;
            for (int mu = d - 2; mu >= 0; --mu) { p[mu] = rem % nb[mu]; rem /= nb[mu]; acc += p[mu]; }
            int64_t last = s - acc;
            if (last < 0 || last >= nb[d - 1]) continue;
            p[d - 1] = last;
            int64_t st[ORC_MAXD], sz[ORC_MAXD];
            int ne = 1;
            int64_t region = 1;
            for (int mu = 0; mu < d; ++mu) {
                st[mu] = bstart[mu][p[mu]];
                sz[mu] = bstart[mu][p[mu] + 1] - st[mu];
                ne *= (int)sz[mu];
                region *= n[mu] - st[mu];
            }
            REAL r[ORC_MAXE], M[ORC_MAXE * ORC_MAXE];
            int64_t off[ORC_MAXE];
            for (int e = 0; e < ne; ++e) {
                int64_t idx[ORC_MAXD];
                int rr = e;
                for (int mu = d - 1; mu >= 0; --mu) { idx[mu] = st[mu] + rr % sz[mu]; rr /= (int)sz[mu]; }
                int64_t o = 0;
                for (int mu = 0; mu < d; ++mu) o += idx[mu] * stride[mu];
                off[e] = o;
                REAL acc2 = (REAL)B[o];
                /* every j with j_nu >= st_nu, outside the tuple */
                for (int64_t t = 0; t < region; ++t) {
                    int64_t jj[ORC_MAXD];
                    int64_t rt = t;
                    int inside = 1;
                    for (int mu = d - 1; mu >= 0; --mu) {
                        int64_t ext = n[mu] - st[mu];
                        jj[mu] = st[mu] + rt % ext; rt /= ext;
                        if (jj[mu] >= st[mu] + sz[mu]) inside = 0;
                    }
                    if (inside) continue;
                    REAL cpl = 0;
                    for (int mu = 0; mu < d; ++mu) {
                        REAL term = (REAL)A[mu][idx[mu] * n[mu] + jj[mu]];
                        for (int nu = 0; nu < d && term != 0; ++nu)
                            if (nu != mu) term *= (REAL)C[nu][idx[nu] * n[nu] + jj[nu]];
                        cpl += term;
                    }
                    if (cpl != 0) {
                        int64_t oj = 0;
                        for (int mu = 0; mu < d; ++mu) oj += jj[mu] * stride[mu];
                        acc2 -= cpl * Xw[oj];
                    }
                }
                r[e] = acc2;
            }
            for (int e = 0; e < ne; ++e) {
                int64_t ie[ORC_MAXD];
                int re = e;
                for (int mu = d - 1; mu >= 0; --mu) { ie[mu] = st[mu] + re % sz[mu]; re /= (int)sz[mu]; }
                for (int f = 0; f < ne; ++f) {
                    int64_t jf[ORC_MAXD];
                    int rf = f;
                    for (int mu = d - 1; mu >= 0; --mu) { jf[mu] = st[mu] + rf % sz[mu]; rf /= (int)sz[mu]; }
                    REAL m = 0;
                    for (int mu = 0; mu < d; ++mu) {
                        REAL term = (REAL)A[mu][ie[mu] * n[mu] + jf[mu]];
                        for (int nu = 0; nu < d && term != 0; ++nu)
                            if (nu != mu) term *= (REAL)C[nu][ie[nu] * n[nu] + jf[nu]];
                        m += term;
                    }
                    M[e * ne + f] = m;
                }
            }
            if (FN(small_gepp)(ne, M, r) != 0) { failed = 1; continue; }
            for (int e = 0; e < ne; ++e) Xw[off[e]] = r[e];
        }
    }
    if (!failed)
        for (int64_t t = 0; t < N; ++t) X[t] = (double)Xw[t];
    free(Xw);
    for (int mu = 0; mu < d; ++mu) free(bstart[mu]);
    return failed ? ORC_SINGULAR : 0;
}

/* Pair-form solve through the exact identity
 *   sum_mu X x_1 C_1 .. x_mu A_mu .. x_d C_d
 *     = (sum_mu X x_mu (C_mu^{-1} A_mu)) x_1 C_1 x_2 .. x_d C_d
 * (mode products in different modes commute; in one mode they compose).
 * Hence X solves the Laplace-like equation with coefficients C_mu^{-1} A_mu
 * (still upper quasi-triangular with the same bumps) and right-hand side
 * B x_1 C_1^{-1} .. x_d C_d^{-1}.  Every triangular solve with C_mu is plain
 * back-substitution.  Cost O(d n N + F_tri): usable at full sizes. */
int FN(oracle_pair_solve_reduced)(int d, const int64_t* n, const double* const* A,
                                  const double* const* C, const double* B, double* X) {
    int64_t N = 1;
    for (int mu = 0; mu < d; ++mu) N *= n[mu];
    double* At[ORC_MAXD];
    for (int mu = 0; mu < d; ++mu) {
        int64_t nm = n[mu];
        At[mu] = (double*)malloc(sizeof(double) * (size_t)(nm * nm));
        /* column by column: C y = A[:, c] */
        for (int64_t c = 0; c < nm; ++c)
            for (int64_t r = nm - 1; r >= 0; --r) {
                REAL acc = (REAL)A[mu][r * nm + c];
                for (int64_t k = r + 1; k < nm; ++k) acc -= (REAL)C[mu][r * nm + k] * (REAL)At[mu][k * nm + c];
                At[mu][r * nm + c] = (double)(acc / (REAL)C[mu][r * nm + r]);
            }
    }
    /* Right-hand side: fiber-wise back-substitution with each C_mu.  Kept in
     * REAL between modes. */
    REAL* W = (REAL*)malloc(sizeof(REAL) * (size_t)N);
    for (int64_t o = 0; o < N; ++o) W[o] = (REAL)B[o];
    for (int mu = 0; mu < d; ++mu) {
        int64_t outer = 1, inner = 1, nm = n[mu];
        for (int nu = 0; nu < mu; ++nu) outer *= n[nu];
        for (int nu = mu + 1; nu < d; ++nu) inner *= n[nu];
        #pragma omp parallel for schedule(static)
        for (int64_t oq = 0; oq < outer * inner; ++oq) {
            int64_t o = oq / inner, q = oq % inner;
            for (int64_t r = nm - 1; r >= 0; --r) {
                REAL acc = W[(o * nm + r) * inner + q];
                for (int64_t k = r + 1; k < nm; ++k)
                    acc -= (REAL)C[mu][r * nm + k] * W[(o * nm + k) * inner + q];
                W[(o * nm + r) * inner + q] = acc / (REAL)C[mu][r * nm + r];
            }
        }
    }
    double* Bt = (double*)malloc(sizeof(double) * (size_t)N);
    for (int64_t o = 0; o < N; ++o) Bt[o] = (double)W[o];
    free(W);
    int rc = FN(oracle_lap_solve)(d, n, (const double* const*)At, Bt, X, 0);
    free(Bt);
    for (int mu = 0; mu < d; ++mu) free(At[mu]);
    return rc;
}

/* ------------------------------------------------------------------------
 * Second operator class, eq. (1.5) / (3.1):
 *   X x_1 A_1 + X x_1 C x_2 A_2 x_3 ... x_d A_d = B,
 * matrix I (x) .. (x) I (x) A_1 + A_d (x) .. (x) A_2 (x) C (Sec. 3).
 * Modes here are 0-based: A[0] and C act on mode 0, A[1..d-1] on modes 1..
 * Element-wise:
 *   Y[i] = sum_j A_1[i_0, j_0] X[j_0, i_1..]
 *        + sum_j C[i_0, j_0] A_2[i_1, j_1] .. A_d[i_{d-1}, j_{d-1}] X[j].
 * Evaluated as plain mode products. */
void FN(oracle_gsylv_apply)(int d, const int64_t* n, const double* const* A, const double* C,
                            const double* X, double* Y) {
    int64_t N = 1;
    for (int mu = 0; mu < d; ++mu) N *= n[mu];
    double* t0 = (double*)malloc(sizeof(double) * (size_t)N);
    double* t1 = (double*)malloc(sizeof(double) * (size_t)N);
    FN(oracle_mode_product)(d, n, 0, A[0], n[0], X, Y);
    FN(oracle_mode_product)(d, n, 0, C, n[0], X, t0);
    for (int mu = 1; mu < d; ++mu) {
        FN(oracle_mode_product)(d, n, mu, A[mu], n[mu], t0, t1);
        double* sw = t0; t0 = t1; t1 = sw;
    }
    for (int64_t o = 0; o < N; ++o) Y[o] += t0[o];
    free(t0); free(t1);
}

/* Second-class solve by plain block back-substitution on the assembled
 * operator (definition of the unique solution, which exists iff the pencil
 * A_1 + lambda C is regular and none of its eigenvalues is an eigenvalue of
 * -A_d (x) .. (x) A_2, Sec. 3).  A_mu upper quasi-triangular, C upper
 * triangular.  The tuples are the products of the 1x1 / 2x2 diagonal blocks
 * of A_1 .. A_d; tuple p couples to the elements j with j_0 >= start(p_0)
 * and j_nu >= start(p_nu) for nu >= 1 (A_1 only along mode 0, the product
 * term over the whole orthant), so tuples are visited by decreasing
 * hyperplane and each element's right-hand side is
 *   r_i = B_i - sum over j outside the tuple of (operator entry)(i, j) X[j].
 * The tuple's unknowns solve the tuple block of the operator by Gaussian
 * elimination with partial pivoting.  Cost O(N^2): small sizes only. */
int FN(oracle_gsylv_solve_direct)(int d, const int64_t* n, const double* const* A, const double* C,
                                  const double* B, double* X) {
    int64_t stride[ORC_MAXD], N = 1;
    for (int mu = d - 1; mu >= 0; --mu) { stride[mu] = N; N *= n[mu]; }
    if (N == 0) return 0;
    int64_t* bstart[ORC_MAXD];
    int64_t nb[ORC_MAXD];
    int rc = 0;
    for (int mu = 0; mu < d; ++mu) {
        bstart[mu] = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n[mu] + 1));
        if (orc_partition(n[mu], A[mu], bstart[mu], &nb[mu]) != 0) rc = ORC_INVALID;
    }
    for (int64_t r = 0; r < n[0]; ++r)
        for (int64_t c = 0; c < r; ++c)
            if (C[r * n[0] + c] != 0.0) rc = ORC_INVALID;
    if (rc) { for (int mu = 0; mu < d; ++mu) free(bstart[mu]); return rc; }
    REAL* Xw = (REAL*)calloc((size_t)N, sizeof(REAL));
    int64_t smax = 0;
    for (int mu = 0; mu < d; ++mu) smax += nb[mu] - 1;
    int64_t lead = 1;
    for (int mu = 0; mu < d - 1; ++mu) lead *= nb[mu];
    int failed = 0;
    /* operator entry between elements i and j (given by coordinates) */
    #define GSYLV_ENTRY(ii, jj, out)                                              \
        do {                                                                     \
            int same = 1;                                                        \
            for (int nu = 1; nu < d; ++nu) if ((ii)[nu] != (jj)[nu]) same = 0;    \
            REAL v_ = same ? (REAL)A[0][(ii)[0] * n[0] + (jj)[0]] : 0;           \
            REAL pr_ = (REAL)C[(ii)[0] * n[0] + (jj)[0]];                        \
            for (int nu = 1; nu < d && pr_ != 0; ++nu)                           \
                pr_ *= (REAL)A[nu][(ii)[nu] * n[nu] + (jj)[nu]];                 \
            (out) = v_ + pr_;                                                    \
        } while (0)
    for (int64_t s = smax; s >= 0 && !failed; --s) {
        #pragma omp parallel for schedule(dynamic, 1) reduction(|: failed)
        for (int64_t lin = 0; lin < lead; ++lin) {
            int64_t p[ORC_MAXD];
            int64_t rem = lin, acc = 0;
            for (int mu = d - 2; mu >= 0; --mu) { p[mu] = rem % nb[mu]; rem /= nb[mu]; acc += p[mu]; }
            int64_t last = s - acc;
            if (last < 0 || last >= nb[d - 1]) continue;
            p[d - 1] = last;
            int64_t st[ORC_MAXD], sz[ORC_MAXD];
            int ne = 1;
            int64_t region = 1;
            for (int mu = 0; mu < d; ++mu) {
                st[mu] = bstart[mu][p[mu]];
                sz[mu] = bstart[mu][p[mu] + 1] - st[mu];
                ne *= (int)sz[mu];
                region *= n[mu] - st[mu];
            }
            REAL r[ORC_MAXE], M[ORC_MAXE * ORC_MAXE];
            int64_t off[ORC_MAXE];
            for (int e = 0; e < ne; ++e) {
                int64_t idx[ORC_MAXD];
                int rr = e;
                for (int mu = d - 1; mu >= 0; --mu) { idx[mu] = st[mu] + rr % sz[mu]; rr /= (int)sz[mu]; }
                int64_t o = 0;
                for (int mu = 0; mu < d; ++mu) o += idx[mu] * stride[mu];
                off[e] = o;
                REAL acc2 = (REAL)B[o];
                for (int64_t t = 0; t < region; ++t) {
                    int64_t jj[ORC_MAXD];
                    int64_t rt = t;
                    int inside = 1;
                    for (int mu = d - 1; mu >= 0; --mu) {
                        int64_t ext = n[mu] - st[mu];
                        jj[mu] = st[mu] + rt % ext; rt /= ext;
                        if (jj[mu] >= st[mu] + sz[mu]) inside = 0;
                    }
                    if (inside) continue;
                    REAL cpl;
                    GSYLV_ENTRY(idx, jj, cpl);
                    if (cpl != 0) {
                        int64_t oj = 0;
                        for (int mu = 0; mu < d; ++mu) oj += jj[mu] * stride[mu];
                        acc2 -= cpl * Xw[oj];
                    }
                }
                r[e] = acc2;
            }
            for (int e = 0; e < ne; ++e) {
                int64_t ie[ORC_MAXD];
                int re = e;
                for (int mu = d - 1; mu >= 0; --mu) { ie[mu] = st[mu] + re % sz[mu]; re /= (int)sz[mu]; }
                for (int f = 0; f < ne; ++f) {
                    int64_t jf[ORC_MAXD];
                    int rf = f;
                    for (int mu = d - 1; mu >= 0; --mu) { jf[mu] = st[mu] + rf % sz[mu]; rf /= (int)sz[mu]; }
                    REAL m;
                    GSYLV_ENTRY(ie, jf, m);
                    M[e * ne + f] = m;
                }
            }
            if (FN(small_gepp)(ne, M, r) != 0) { failed = 1; continue; }
            for (int e = 0; e < ne; ++e) Xw[off[e]] = r[e];
        }
    }
    #undef GSYLV_ENTRY
    if (!failed)
        for (int64_t t = 0; t < N; ++t) X[t] = (double)Xw[t];
    free(Xw);
    for (int mu = 0; mu < d; ++mu) free(bstart[mu]);
    return failed ? ORC_SINGULAR : 0;
}

/* Gradient of L = <G, X> with respect to T_mu when X solves the Laplace-like
 * equation: with Lam the adjoint solution (sum_nu Lam x_nu T_nu^T = G),
 *   dT_mu[a, b] = - sum over all i with i_mu = a of Lam[i] X[i with i_mu := b],
 * i.e. dT_mu = -Lam_(mu) X_(mu)^T.  mask != 0 zeroes entries outside the
 * quasi-triangular pattern (upper triangle + nonzero bump subdiagonals). */
void FN(oracle_grad_T)(int d, const int64_t* n, int mu, const double* Tmu,
                       const double* Lam, const double* X, double* dT, int mask) {
    int64_t outer = 1, inner = 1, nm = n[mu];
    for (int nu = 0; nu < mu; ++nu) outer *= n[nu];
    for (int nu = mu + 1; nu < d; ++nu) inner *= n[nu];
    #pragma omp parallel for schedule(static)
    for (int64_t ab = 0; ab < nm * nm; ++ab) {
        int64_t a = ab / nm, b = ab % nm;
        REAL acc = 0;
        for (int64_t o = 0; o < outer; ++o)
            for (int64_t q = 0; q < inner; ++q)
                acc += (REAL)Lam[(o * nm + a) * inner + q] * (REAL)X[(o * nm + b) * inner + q];
        double v = -(double)acc;
        if (mask) {
            int keep = (b >= a) || (b == a - 1 && Tmu[a * nm + b] != 0.0);
            if (!keep) v = 0.0;
        }
        dT[ab] = v;
    }
}

#undef FN
#undef CAT
#undef CAT_
