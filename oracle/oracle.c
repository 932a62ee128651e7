/* CPU oracle for Kronecker-structured tensor equations
 * (Chen & Kressner, "Recursive blocked algorithms for linear systems with
 * Kronecker product structure").
 *
 * TEST INFRASTRUCTURE ONLY: this library is loaded by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark, never by the
 * solver library.  It shares no code, header or table with the GPU path.
 *
 * Everything here is a plain definition written out in loops:
 *   - Laplace-like operator (eq. 1.4 / 2.2) and its solve by element-wise
 *     (1x1 / 2x2 block) back-substitution;
 *   - the adjoint (transposed) solve by forward substitution;
 *   - the pair operator  sum_mu X x_1 C_1 .. x_mu A_mu .. x_d C_d  and its
 *     solve, both directly and through the C^{-1} reduction;
 *   - the second operator class X x_1 A_1 + X x_1 C x_2 A_2 .. x_d A_d
 *     (eq. 1.5 / 3.1) and its direct solve;
 *   - mu-mode products (Sec. 2) and the coefficient gradient -Lam_(mu) X_(mu)^T;
 *   - the flop count of the method.
 * Instantiated in double (_f64) and x87 long double (_ld).
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXD 6
#define ORC_MAXE 64 /* 2^ORC_MAXD unknowns per tuple */
#define ORC_INVALID 1
#define ORC_SINGULAR 2

/* Partition 0..n-1 into the diagonal blocks of an upper quasi-triangular
 * matrix: a nonzero T[i+1][i] makes {i, i+1} a 2x2 block.  Returns
 * ORC_INVALID if T is not upper quasi-triangular (entry below the first
 * subdiagonal, or two adjacent nonzero subdiagonal entries). */
static int orc_partition(int64_t n, const double* T, int64_t* bstart, int64_t* nb) {
    for (int64_t r = 0; r < n; ++r)
        for (int64_t c = 0; c + 1 < r; ++c)
            if (T[r * n + c] != 0.0) return ORC_INVALID;
    int64_t k = 0, i = 0;
    while (i < n) {
        bstart[k++] = i;
        if (i + 1 < n && T[(i + 1) * n + i] != 0.0) {
            if (i + 2 < n && T[(i + 2) * n + i + 1] != 0.0) return ORC_INVALID;
            i += 2;
        } else {
            i += 1;
        }
    }
    bstart[k] = n;
    *nb = k;
    return 0;
}

#define REAL double
#define SFX _f64
#include "oracle_impl.h"
#undef REAL
#undef SFX

#define REAL long double
#define SFX _ld
#include "oracle_impl.h"
#undef REAL
#undef SFX

/* Flops of the method on upper quasi-triangular coefficients, one fused
 * multiply-add counted as two flops:
 *   F_tri = 2 * sum_mu (n_mu (n_mu - 1) / 2 + bumps_mu) * N / n_mu.
 * This is exactly the multiply-add count of element-wise back-substitution
 * (every strictly upper entry of T_mu, and every bump subdiagonal, meets every
 * fiber along mode mu once), and therefore of any recursive reordering of it
 * (Sec. 2.1). */
double oracle_flops_tri(int d, const int64_t* n, const double* const* T) {
    double N = 1.0;
    for (int mu = 0; mu < d; ++mu) N *= (double)n[mu];
    double f = 0.0;
    for (int mu = 0; mu < d; ++mu) {
        int64_t nm = n[mu], bumps = 0;
        for (int64_t i = 0; i + 1 < nm; ++i)
            if (T[mu][(i + 1) * nm + i] != 0.0) ++bumps;
        double off = (double)nm * (double)(nm - 1) / 2.0 + (double)bumps;
        if (nm > 0) f += 2.0 * off * N / (double)nm;
    }
    return f;
}

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }
#else
int oracle_num_threads(void) { return 1; }
void oracle_set_threads(int t) { (void)t; }
#endif
