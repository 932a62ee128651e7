// Host real Schur decomposition A = U T U^T, the reduction step of
// Algorithm 1 (Sec. 2): T upper quasi-triangular with 1x1 and 2x2 diagonal
// blocks, U orthogonal.  Method (Golub & Van Loan, Matrix Computations,
// Sec. 7.4-7.5): Householder reduction to upper Hessenberg form, then the
// Francis implicit double-shift QR iteration with deflation on the full
// matrix (so that T and U are both kept), and finally every 2x2 block
// standardised by a plane rotation: real eigenvalues -> split into two 1x1
// blocks; complex pair -> equal diagonal entries and off-diagonals of
// opposite sign.  Row-major n x n storage throughout.
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "tt_internal.h"

namespace tt {

namespace {

struct Mat {
    int n;
    std::vector<double> a;
    explicit Mat(int n_) : n(n_), a((size_t)n_ * n_, 0.0) {}
    double& operator()(int i, int j) { return a[(size_t)i * n + j]; }
    double operator()(int i, int j) const { return a[(size_t)i * n + j]; }
};

// Householder vector v (v[0] = 1) and beta with (I - beta v v^T) x = alpha e_1.
// Returns beta (0 when x is already a multiple of e_1).
double householder(const double* x, int m, double* v) {
    double sigma = 0.0;
    for (int i = 1; i < m; ++i) sigma += x[i] * x[i];
    v[0] = 1.0;
    for (int i = 1; i < m; ++i) v[i] = x[i];
    if (sigma == 0.0) return 0.0;
    const double mu = std::sqrt(x[0] * x[0] + sigma);
    // v0 = x0 - mu computed without cancellation
    const double v0 = (x[0] <= 0.0) ? x[0] - mu : -sigma / (x[0] + mu);
    const double beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
    for (int i = 1; i < m; ++i) v[i] = x[i] / v0;
    return beta;
}

// rows r0..r0+m-1 of H, columns c0..c1-1:  H <- (I - beta v v^T) H
void apply_left(Mat& H, int r0, int m, int c0, int c1, const double* v, double beta) {
    if (beta == 0.0) return;
    for (int j = c0; j < c1; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += v[i] * H(r0 + i, j);
        s *= beta;
        for (int i = 0; i < m; ++i) H(r0 + i, j) -= s * v[i];
    }
}

// columns c0..c0+m-1 of H, rows r0..r1-1:  H <- H (I - beta v v^T)
void apply_right(Mat& H, int c0, int m, int r0, int r1, const double* v, double beta) {
    if (beta == 0.0) return;
    for (int i = r0; i < r1; ++i) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += H(i, c0 + j) * v[j];
        s *= beta;
        for (int j = 0; j < m; ++j) H(i, c0 + j) -= s * v[j];
    }
}

// Plane rotation G = [[c, -s], [s, c]] on indices k, k+1 of an isolated
// diagonal block: T <- G^T T G, U <- U G (full rows and columns; the entries
// outside the quasi-triangular pattern that they touch are zero).
void rotate(Mat& T, Mat& U, int k, double c, double s) {
    const int n = T.n;
    for (int j = 0; j < n; ++j) {  // rows: G^T
        double x = T(k, j), y = T(k + 1, j);
        T(k, j) = c * x + s * y;
        T(k + 1, j) = -s * x + c * y;
    }
    for (int i = 0; i < n; ++i) {  // columns: G
        double x = T(i, k), y = T(i, k + 1);
        T(i, k) = c * x + s * y;
        T(i, k + 1) = -s * x + c * y;
        double ux = U(i, k), uy = U(i, k + 1);
        U(i, k) = c * ux + s * uy;
        U(i, k + 1) = -s * ux + c * uy;
    }
}

// Standardise the 2x2 diagonal block at rows/columns k, k+1.
void standardize_block(Mat& T, Mat& U, int k) {
    const double a = T(k, k), b = T(k, k + 1), c = T(k + 1, k), d = T(k + 1, k + 1);
    if (c == 0.0) return;
    const double p = 0.5 * (a - d);
    const double disc = p * p + b * c;
    if (disc >= 0.0) {
        // real eigenvalues: rotate an eigenvector onto e_1 -> upper triangular
        const double sq = std::sqrt(disc);
        const double lam = 0.5 * (a + d) + (p >= 0.0 ? sq : -sq);
        double v1 = b, v2 = lam - a;        // from row 1: (a - lam) v1 + b v2 = 0
        double w1 = lam - d, w2 = c;        // from row 2: c v1 + (d - lam) v2 = 0
        if (std::hypot(w1, w2) > std::hypot(v1, v2)) {
            v1 = w1;
            v2 = w2;
        }
        const double r = std::hypot(v1, v2);
        if (r == 0.0) return;
        rotate(T, U, k, v1 / r, v2 / r);
        T(k + 1, k) = 0.0;
    } else {
        // complex pair: equal diagonal entries,
        // (a - d) cos 2t + (b + c) sin 2t = 0
        const double th = 0.5 * std::atan2(-(a - d), b + c);
        rotate(T, U, k, std::cos(th), std::sin(th));
        const double m = 0.5 * (T(k, k) + T(k + 1, k + 1));
        T(k, k) = m;
        T(k + 1, k + 1) = m;
    }
}

int schur_one(int n, const double* A, double* Tout, double* Uout, std::string& err) {
    Mat H(n), U(n);
    std::memcpy(H.a.data(), A, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) U(i, i) = 1.0;
    for (double x : H.a)
        if (!std::isfinite(x)) {
            err = "coefficient matrix has a non-finite entry";
            return TT_EINVAL;
        }
    std::vector<double> x((size_t)n + 3), v((size_t)n + 3);
    // 1. Hessenberg reduction
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        for (int i = 0; i < m; ++i) x[i] = H(k + 1 + i, k);
        const double beta = householder(x.data(), m, v.data());
        apply_left(H, k + 1, m, k, n, v.data(), beta);
        apply_right(H, k + 1, m, 0, n, v.data(), beta);
        apply_right(U, k + 1, m, 0, n, v.data(), beta);
        for (int i = k + 2; i < n; ++i) H(i, k) = 0.0;
    }
    // 2. Francis double-shift QR with deflation
    const double eps = std::ldexp(1.0, -52);
    double anorm = 0.0;
    for (double x2 : H.a) anorm = std::fmax(anorm, std::fabs(x2));
    int p = n - 1, iter = 0, total = 0;
    while (p >= 1) {
        int l = p;
        while (l >= 1) {
            double s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
            if (s == 0.0) s = anorm;
            if (std::fabs(H(l, l - 1)) <= eps * s) {
                H(l, l - 1) = 0.0;
                break;
            }
            --l;
        }
        if (l == p) {  // 1x1 block converged
            --p;
            iter = 0;
            continue;
        }
        if (l == p - 1) {  // 2x2 block converged
            standardize_block(H, U, p - 1);
            p -= 2;
            iter = 0;
            continue;
        }
        if (++total > 40 * n) {
            err = "QR iteration did not converge";
            return TT_EINVAL;
        }
        ++iter;
        double s, t;
        if (iter % 11 == 10) {  // exceptional shift
            const double w = std::fabs(H(p, p - 1)) + std::fabs(H(p - 1, p - 2));
            const double z = H(p, p) + 0.75 * w;
            s = 2.0 * z;
            t = z * z;
        } else {
            s = H(p - 1, p - 1) + H(p, p);
            t = H(p - 1, p - 1) * H(p, p) - H(p - 1, p) * H(p, p - 1);
        }
        double xx = H(l, l) * H(l, l) + H(l, l + 1) * H(l + 1, l) - s * H(l, l) + t;
        double yy = H(l + 1, l) * (H(l, l) + H(l + 1, l + 1) - s);
        double zz = H(l + 1, l) * H(l + 2, l + 1);
        for (int k = l; k <= p - 2; ++k) {
            double xv[3] = {xx, yy, zz};
            double vv[3];
            const double beta = householder(xv, 3, vv);
            const int q = (k > l) ? k - 1 : l;
            apply_left(H, k, 3, q, n, vv, beta);
            const int r = (k + 4 < p + 1) ? k + 4 : p + 1;
            apply_right(H, k, 3, 0, r, vv, beta);
            apply_right(U, k, 3, 0, n, vv, beta);
            if (k > l) {
                H(k + 1, k - 1) = 0.0;
                H(k + 2, k - 1) = 0.0;
            }
            xx = H(k + 1, k);
            yy = H(k + 2, k);
            if (k < p - 2) zz = H(k + 3, k);
        }
        {
            double xv[2] = {xx, yy};
            double vv[2];
            const double beta = householder(xv, 2, vv);
            apply_left(H, p - 1, 2, p - 2, n, vv, beta);
            apply_right(H, p - 1, 2, 0, p + 1, vv, beta);
            apply_right(U, p - 1, 2, 0, n, vv, beta);
            H(p, p - 2) = 0.0;
        }
    }
    // 3. exact zeros below the quasi-triangular pattern
    for (int i = 0; i < n; ++i)
        for (int j = 0; j + 1 < i; ++j) H(i, j) = 0.0;
    for (int i = 1; i < n; ++i)
        if (H(i, i - 1) != 0.0 && i >= 2 && H(i - 1, i - 2) != 0.0) {
            err = "internal: consecutive nonzero subdiagonals after QR";
            return TT_EINVAL;
        }
    std::memcpy(Tout, H.a.data(), sizeof(double) * (size_t)n * n);
    std::memcpy(Uout, U.a.data(), sizeof(double) * (size_t)n * n);
    return TT_OK;
}

// ---------------------------------------------------------------------------
// Real generalized Schur (QZ) decomposition of a pencil (A, C), the host step
// of Algorithm 4 (Sec. 3): A = Q S Z^T, C = Q T Z^T with S upper
// quasi-triangular, T upper triangular, Q and Z orthogonal.  Method
// (Golub & Van Loan, Sec. 7.7; Moler & Stewart): QR of C, Givens reduction
// to Hessenberg-triangular form, the implicit double-shift QZ iteration with
// deflation on the full matrices, and every converged 2x2 block with real
// eigenvalues split into two 1x1 blocks.  C must be nonsingular (a tiny
// diagonal entry of T, i.e. an infinite eigenvalue, is reported).

// rows i1, i2 of M, columns c0..c1-1:  (x, y) <- (c x + s y, -s x + c y)
void rot_rows(Mat& M, int i1, int i2, double c, double s, int c0, int c1) {
    for (int j = c0; j < c1; ++j) {
        const double x = M(i1, j), y = M(i2, j);
        M(i1, j) = c * x + s * y;
        M(i2, j) = -s * x + c * y;
    }
}

// columns j1, j2 of M, rows r0..r1-1:  (x, y) <- (c x - s y, s x + c y)
void rot_cols(Mat& M, int j1, int j2, double c, double s, int r0, int r1) {
    for (int i = r0; i < r1; ++i) {
        const double x = M(i, j1), y = M(i, j2);
        M(i, j1) = c * x - s * y;
        M(i, j2) = s * x + c * y;
    }
}

// Right reflector (I - beta w w^T) of length m with x^T (I - beta w w^T) =
// alpha e_m^T (x = the m entries of a row): the left reflector of the
// reversed row, reversed.
double householder_last(const double* x, int m, double* w) {
    double xr[3], vr[3];
    for (int i = 0; i < m; ++i) xr[i] = x[m - 1 - i];
    const double beta = householder(xr, m, vr);
    for (int i = 0; i < m; ++i) w[i] = vr[m - 1 - i];
    return beta;
}

int qz_one(int n, const double* A, const double* C, double* Sout, double* Tout, double* Qout, double* Zout,
           std::string& err) {
    Mat H(n), R(n), Q(n), Z(n);
    std::memcpy(H.a.data(), A, sizeof(double) * (size_t)n * n);
    std::memcpy(R.a.data(), C, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) Q(i, i) = Z(i, i) = 1.0;
    for (size_t i = 0; i < H.a.size(); ++i)
        if (!std::isfinite(H.a[i]) || !std::isfinite(R.a[i])) {
            err = "coefficient matrix has a non-finite entry";
            return TT_EINVAL;
        }
    std::vector<double> x((size_t)n + 3), v((size_t)n + 3);
    // 1. C = Q_1 R
    for (int k = 0; k + 1 < n; ++k) {
        const int m = n - k;
        for (int i = 0; i < m; ++i) x[i] = R(k + i, k);
        const double beta = householder(x.data(), m, v.data());
        apply_left(R, k, m, k, n, v.data(), beta);
        apply_left(H, k, m, 0, n, v.data(), beta);
        apply_right(Q, k, m, 0, n, v.data(), beta);
        for (int i = k + 1; i < n; ++i) R(i, k) = 0.0;
    }
    // 2. Hessenberg-triangular form: zero H below the subdiagonal column by
    // column (left rotations), each fill-in of R removed by a right rotation
    for (int j = 0; j + 2 < n; ++j)
        for (int i = n - 1; i >= j + 2; --i) {
            double a = H(i - 1, j), b = H(i, j);
            if (b != 0.0) {
                const double r = std::hypot(a, b), c = a / r, s = b / r;
                rot_rows(H, i - 1, i, c, s, j, n);
                rot_rows(R, i - 1, i, c, s, i - 1, n);
                rot_cols(Q, i - 1, i, c, -s, 0, n);  // Q <- Q G^T
                H(i, j) = 0.0;
            }
            a = R(i, i - 1);
            b = R(i, i);
            if (a != 0.0) {
                const double r = std::hypot(a, b), c = b / r, s = a / r;
                rot_cols(R, i - 1, i, c, s, 0, i + 1);
                rot_cols(H, i - 1, i, c, s, 0, n);
                rot_cols(Z, i - 1, i, c, s, 0, n);
                R(i, i - 1) = 0.0;
            }
        }
    // 3. double-shift QZ with deflation
    const double eps = std::ldexp(1.0, -52);
    double anorm = 0.0, bnorm = 0.0;
    for (size_t i = 0; i < H.a.size(); ++i) {
        anorm = std::fmax(anorm, std::fabs(H.a[i]));
        bnorm = std::fmax(bnorm, std::fabs(R.a[i]));
    }
    if (bnorm == 0.0) {
        err = "C is zero";
        return TT_ESINGULAR;
    }
    auto singular = [&](int lo, int hi) {
        for (int k = lo; k <= hi; ++k)
            if (std::fabs(R(k, k)) <= eps * bnorm) return true;
        return false;
    };
    int p = n - 1, iter = 0, total = 0;
    while (p >= 1) {
        int l = p;
        while (l >= 1) {
            double s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
            if (s == 0.0) s = anorm;
            if (std::fabs(H(l, l - 1)) <= eps * s) {
                H(l, l - 1) = 0.0;
                break;
            }
            --l;
        }
        if (singular(l, p)) {
            err = "C is singular to working precision (infinite generalized eigenvalue)";
            return TT_ESINGULAR;
        }
        if (l == p) {  // 1x1 block converged
            --p;
            iter = 0;
            continue;
        }
        if (l == p - 1) {  // 2x2 block converged: split it when its eigenvalues are real
            const int k = p - 1;
            const double h00 = H(k, k), h01 = H(k, k + 1), h10 = H(k + 1, k), h11 = H(k + 1, k + 1);
            const double r00 = R(k, k), r01 = R(k, k + 1), r11 = R(k + 1, k + 1);
            // det(H2 - lam R2) = qa lam^2 + qb lam + qc
            const double qa = r00 * r11, qb = -(h00 * r11 + h11 * r00 - h10 * r01), qc = h00 * h11 - h01 * h10;
            const double disc = qb * qb - 4.0 * qa * qc;
            if (disc >= 0.0) {
                const double sq = std::sqrt(disc);
                const double q = -0.5 * (qb + (qb >= 0.0 ? sq : -sq));
                const double lam = (std::fabs(q) > 0.0 && std::fabs(qa) > 0.0) ? q / qa : qc / q;
                // right eigenvector z: (H2 - lam R2) z = 0 from the larger row
                const double m00 = h00 - lam * r00, m01 = h01 - lam * r01, m10 = h10, m11 = h11 - lam * r11;
                double z0 = m01, z1 = -m00;
                if (std::hypot(m10, m11) > std::hypot(m00, m01)) {
                    z0 = m11;
                    z1 = -m10;
                }
                const double zr = std::hypot(z0, z1);
                if (zr > 0.0) {
                    // columns (k, k+1) <- first column z / |z|
                    const double c = z0 / zr, s = z1 / zr;
                    rot_cols(H, k, k + 1, c, -s, 0, k + 2);
                    rot_cols(R, k, k + 1, c, -s, 0, k + 2);
                    rot_cols(Z, k, k + 1, c, -s, 0, n);
                    // rows (k, k+1): zero R(k+1, k) (H(k+1, k) follows)
                    const double a = R(k, k), b = R(k + 1, k);
                    const double r = std::hypot(a, b);
                    if (r > 0.0) {
                        const double cc = a / r, ss = b / r;
                        rot_rows(H, k, k + 1, cc, ss, k, n);
                        rot_rows(R, k, k + 1, cc, ss, k, n);
                        rot_cols(Q, k, k + 1, cc, -ss, 0, n);
                    }
                    H(k + 1, k) = 0.0;
                    R(k + 1, k) = 0.0;
                }
            }
            p -= 2;
            iter = 0;
            continue;
        }
        if (++total > 40 * n) {
            err = "QZ iteration did not converge";
            return TT_EINVAL;
        }
        ++iter;
        // shifts: eigenvalues of the trailing 2x2 block of M = H R^-1
        double s, t;
        {
            const double r00 = R(p - 2, p - 2), r01 = R(p - 2, p - 1), r02 = R(p - 2, p);
            const double r11 = R(p - 1, p - 1), r12 = R(p - 1, p), r22 = R(p, p);
            const double i11 = 1.0 / r11, i22 = 1.0 / r22;
            const double i01 = -r01 * i11 / r00, i12 = -r12 * i22 / r11;
            const double i02 = -(r01 * i12 + r02 * i22) / r00;
            const double ma = H(p - 1, p - 2) * i01 + H(p - 1, p - 1) * i11;
            const double mb = H(p - 1, p - 2) * i02 + H(p - 1, p - 1) * i12 + H(p - 1, p) * i22;
            const double mc = H(p, p - 1) * i11;
            const double md = H(p, p - 1) * i12 + H(p, p) * i22;
            if (iter % 11 == 10) {  // exceptional shift
                const double w = std::fabs(mc) + std::fabs(H(p - 1, p - 2) * i11);
                const double z = md + 0.75 * w;
                s = 2.0 * z;
                t = z * z;
            } else {
                s = ma + md;
                t = ma * md - mb * mc;
            }
        }
        // first column of (M - a1 I)(M - a2 I) at the window start
        double xx, yy, zz;
        {
            const double u0 = H(l, l) / R(l, l), u1 = H(l + 1, l) / R(l, l);
            const double w1 = u1 / R(l + 1, l + 1);
            const double w0 = (u0 - R(l, l + 1) * w1) / R(l, l);
            xx = H(l, l) * w0 + H(l, l + 1) * w1 - s * u0 + t;
            yy = H(l + 1, l) * w0 + H(l + 1, l + 1) * w1 - s * u1;
            zz = H(l + 2, l + 1) * w1;
        }
        for (int k = l; k <= p - 2; ++k) {
            double xv[3] = {xx, yy, zz}, vv[3];
            double beta = householder(xv, 3, vv);
            const int q = (k > l) ? k - 1 : l;
            apply_left(H, k, 3, q, n, vv, beta);
            apply_left(R, k, 3, k, n, vv, beta);
            apply_right(Q, k, 3, 0, n, vv, beta);
            if (k > l) {
                H(k + 1, k - 1) = 0.0;
                H(k + 2, k - 1) = 0.0;
            }
            const int rh = (k + 4 < p + 1) ? k + 4 : p + 1;  // rows of H touched by the bulge
            // restore R: zero R(k+2, k), R(k+2, k+1), then R(k+1, k)
            double rv[3] = {R(k + 2, k), R(k + 2, k + 1), R(k + 2, k + 2)}, w[3];
            beta = householder_last(rv, 3, w);
            apply_right(R, k, 3, 0, k + 3, w, beta);
            apply_right(H, k, 3, 0, rh, w, beta);
            apply_right(Z, k, 3, 0, n, w, beta);
            R(k + 2, k) = 0.0;
            R(k + 2, k + 1) = 0.0;
            double rv2[2] = {R(k + 1, k), R(k + 1, k + 1)}, w2[2];
            beta = householder_last(rv2, 2, w2);
            apply_right(R, k, 2, 0, k + 2, w2, beta);
            apply_right(H, k, 2, 0, rh, w2, beta);
            apply_right(Z, k, 2, 0, n, w2, beta);
            R(k + 1, k) = 0.0;
            xx = H(k + 1, k);
            yy = H(k + 2, k);
            if (k < p - 2) zz = H(k + 3, k);
        }
        {
            double xv[2] = {xx, yy}, vv[2];
            double beta = householder(xv, 2, vv);
            apply_left(H, p - 1, 2, p - 2, n, vv, beta);
            apply_left(R, p - 1, 2, p - 1, n, vv, beta);
            apply_right(Q, p - 1, 2, 0, n, vv, beta);
            H(p, p - 2) = 0.0;
            double rv2[2] = {R(p, p - 1), R(p, p)}, w2[2];
            beta = householder_last(rv2, 2, w2);
            apply_right(R, p - 1, 2, 0, p + 1, w2, beta);
            apply_right(H, p - 1, 2, 0, p + 1, w2, beta);
            apply_right(Z, p - 1, 2, 0, n, w2, beta);
            R(p, p - 1) = 0.0;
        }
    }
    // 4. exact zeros below the patterns
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j + 1 < i; ++j) H(i, j) = 0.0;
        for (int j = 0; j < i; ++j) R(i, j) = 0.0;
    }
    for (int i = 2; i < n; ++i)
        if (H(i, i - 1) != 0.0 && H(i - 1, i - 2) != 0.0) {
            err = "internal: consecutive nonzero subdiagonals after QZ";
            return TT_EINVAL;
        }
    if (singular(0, n - 1)) {
        err = "C is singular to working precision (infinite generalized eigenvalue)";
        return TT_ESINGULAR;
    }
    std::memcpy(Sout, H.a.data(), sizeof(double) * (size_t)n * n);
    std::memcpy(Tout, R.a.data(), sizeof(double) * (size_t)n * n);
    std::memcpy(Qout, Q.a.data(), sizeof(double) * (size_t)n * n);
    std::memcpy(Zout, Z.a.data(), sizeof(double) * (size_t)n * n);
    return TT_OK;
}

}  // namespace

int schur_real(int n, const double* A, double* T, double* U, std::string& err) {
    if (n <= 0) return TT_OK;
    return schur_one(n, A, T, U, err);
}

int qz_real(int n, const double* A, const double* C, double* S, double* T, double* Q, double* Z,
            std::string& err) {
    if (n <= 0) return TT_OK;
    return qz_one(n, A, C, S, T, Q, Z, err);
}

// Several independent decompositions (one per mode) on host threads.
int schur_real_many(int count, const int* n, const double* const* A, double* const* T, double* const* U,
                    std::string& err) {
    std::vector<int> rc((size_t)count, TT_OK);
    std::vector<std::string> msg((size_t)count);
    std::vector<std::thread> th;
    for (int i = 0; i < count; ++i)
        th.emplace_back([&, i] { rc[(size_t)i] = schur_real(n[i], A[i], T[i], U[i], msg[(size_t)i]); });
    for (auto& t : th) t.join();
    for (int i = 0; i < count; ++i)
        if (rc[(size_t)i]) {
            err = msg[(size_t)i];
            return rc[(size_t)i];
        }
    return TT_OK;
}

// Merged coefficient of two adjacent modes (Sec. 2.2, Algorithm 3's merge
// in the real quasi-triangular case).  With the outer (slower) mode a and the
// inner mode b, the two terms X x_a A_a + X x_b A_b act on the merged index
// m = i_a n_b + i_b as
//     A' = A_a (x) I_b + I_a (x) A_b,
// which is block upper triangular but not quasi-triangular where A_a has a
// 2x2 block (j, j+1): its (j+1, j) block is A_a[j+1][j] I.  A perfect shuffle
// of block rows and columns j, j+1 (order (j, 0), (j+1, 0), (j, 1), ...) makes
// the region block upper triangular with 2x2 diagonal blocks, 4x4 where A_b
// has a 2x2 block too (Sec. 2.2, the example after eq. (2.9)).  A 4x4 block
// is brought to real Schur form by the host QR iteration; a 2x2 block is
// already a valid diagonal block.  Result: A' = V Tm V^T with V = P Q
// orthogonal (permutation times block-diagonal orthogonal) and Tm upper
// quasi-triangular.  perm[r] = the merged index at position r of the
// shuffled order.  All matrices row-major, na*nb squared.
int merge_modes(int na, const double* Ta, int nb, const double* Tb, double* Tm, double* V, int* perm,
                std::string& err) {
    const int nm = na * nb;
    const size_t NN = (size_t)nm * (size_t)nm;
    std::vector<double> A(NN, 0.0);
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < nb; ++ib) {
            const int r = ia * nb + ib;
            for (int ja = 0; ja < na; ++ja) A[(size_t)r * nm + (size_t)(ja * nb + ib)] += Ta[ia * na + ja];
            for (int jb = 0; jb < nb; ++jb) A[(size_t)r * nm + (size_t)(ia * nb + jb)] += Tb[ib * nb + jb];
        }
    // perfect shuffle of the block pairs of A_a's 2x2 blocks
    std::vector<int> p;
    p.reserve((size_t)nm);
    for (int ja = 0; ja < na;) {
        const bool two = ja + 1 < na && Ta[(ja + 1) * na + ja] != 0.0;
        if (two) {
            for (int ib = 0; ib < nb; ++ib) {
                p.push_back(ja * nb + ib);
                p.push_back((ja + 1) * nb + ib);
            }
            ja += 2;
        } else {
            for (int ib = 0; ib < nb; ++ib) p.push_back(ja * nb + ib);
            ja += 1;
        }
    }
    std::vector<double> Ap(NN);
    for (int r = 0; r < nm; ++r)
        for (int c = 0; c < nm; ++c) Ap[(size_t)r * nm + c] = A[(size_t)p[r] * nm + p[c]];
    // diagonal blocks of the shuffled matrix and their orthogonal factors
    std::vector<double> Q(NN, 0.0);
    std::vector<int> bstart;
    for (int r = 0; r < nm;) {
        int sz = 1;
        const int ia = p[r] / nb, ib = p[r] % nb;
        const bool twoa = ia + 1 < na && Ta[(ia + 1) * na + ia] != 0.0 && p[r] == ia * nb + ib &&
                          r + 1 < nm && p[r + 1] == (ia + 1) * nb + ib;
        const bool twob = ib + 1 < nb && Tb[(ib + 1) * nb + ib] != 0.0;
        if (twoa) sz = twob ? 4 : 2;
        else sz = twob ? 2 : 1;
        bstart.push_back(r);
        if (sz == 4) {
            double B4[16], T4[16], U4[16];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) B4[i * 4 + j] = Ap[(size_t)(r + i) * nm + r + j];
            std::string e2;
            const int rc = schur_real(4, B4, T4, U4, e2);
            if (rc) {
                err = "merge: real Schur form of a 4x4 diagonal block failed: " + e2;
                return rc;
            }
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) Q[(size_t)(r + i) * nm + r + j] = U4[i * 4 + j];
        } else {
            for (int i = 0; i < sz; ++i) Q[(size_t)(r + i) * nm + r + i] = 1.0;
        }
        r += sz;
    }
    bstart.push_back(nm);
    // Tm = Q^T Ap Q blockwise (Q block diagonal); entries below the block
    // diagonal are zero, a 4x4 diagonal block takes its Schur form exactly
    std::fill(Tm, Tm + NN, 0.0);
    const int nblk = (int)bstart.size() - 1;
    for (int bi = 0; bi < nblk; ++bi) {
        const int r0 = bstart[(size_t)bi], r1 = bstart[(size_t)bi + 1];
        for (int bj = bi; bj < nblk; ++bj) {
            const int c0 = bstart[(size_t)bj], c1 = bstart[(size_t)bj + 1];
            for (int i = r0; i < r1; ++i)
                for (int j = c0; j < c1; ++j) {
                    double acc = 0.0;
                    for (int k = r0; k < r1; ++k)
                        for (int l = c0; l < c1; ++l)
                            acc += Q[(size_t)k * nm + i] * Ap[(size_t)k * nm + l] * Q[(size_t)l * nm + j];
                    Tm[(size_t)i * nm + j] = acc;
                }
        }
        if (r1 - r0 == 4) {
            double B4[16], T4[16], U4[16];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) B4[i * 4 + j] = Ap[(size_t)(r0 + i) * nm + r0 + j];
            std::string e2;
            (void)schur_real(4, B4, T4, U4, e2);
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) Tm[(size_t)(r0 + i) * nm + r0 + j] = T4[i * 4 + j];
        }
    }
    // V = P Q: row p[r] of V is row r of Q
    for (int r = 0; r < nm; ++r)
        for (int c = 0; c < nm; ++c) V[(size_t)p[r] * nm + c] = Q[(size_t)r * nm + c];
    for (int r = 0; r < nm; ++r) perm[r] = p[r];
    return TT_OK;
}

}  // namespace tt
