// Leaf solve of the recursive triangular solve (gfx950).
//
// At the leaves of Algorithm 2 (size <= n_min per mode) the paper solves the
// small Laplace-like system directly.  Here one workgroup (256 threads) owns
// one leaf block B and
//   1. loads the right-hand side X[B] - sum_{mu>=1} A_mu[B] (mode-0 updates
//      were subtracted from X in place, the others wait in accumulators) and
//      the diagonal blocks T_mu[B, B] into LDS;
//   2. subtracts the contribution of the next block along each mode,
//      T_mu[B, B+1] x_mu X[B+1] -- the update of the split between two
//      adjacent leaves, which the schedule leaves to the leaf itself;
//   3. partitions each mode of the block into the 1x1 / 2x2 diagonal blocks
//      of the quasi-triangular T_mu and solves block back-substitution over
//      the tuples of those blocks: tuples on one hyperplane of the tuple grid
//      are independent, so each hyperplane is one parallel step.  In a step
//      every unknown forms its right-hand side (one thread per unknown) and a
//      tuple with widths w_mu couples its ne = prod w_mu unknowns by
//      sum_mu I (x) T_mu[p_mu, p_mu] (x) I: ne = 1 is a division by the
//      eigenvalue sum, larger tuples are small dense solves in registers;
//   4. stores the solved block.
// The hyperplane order of the tuple grid depends only on the number of tuples
// per mode, so the planner precomputes one ordered list per grid shape.
#include "tt_internal.h"

namespace tt {

namespace {

// Gaussian elimination with partial pivoting on a small system held in
// registers (all indices static).  Returns false on a zero pivot or a
// non-finite result.
template <int NE>
__device__ inline bool gepp_small(double (&M)[NE][NE], double (&r)[NE]) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < NE; ++k) {
#pragma unroll
        for (int i = k + 1; i < NE; ++i) {
            if (fabs(M[i][k]) > fabs(M[k][k])) {
#pragma unroll
                for (int j = 0; j < NE; ++j) {
                    double t = M[k][j];
                    M[k][j] = M[i][j];
                    M[i][j] = t;
                }
                double t = r[k];
                r[k] = r[i];
                r[i] = t;
            }
        }
        const double piv = M[k][k];
        if (piv == 0.0) ok = false;
#pragma unroll
        for (int i = k + 1; i < NE; ++i) {
            const double f = M[i][k] / piv;
#pragma unroll
            for (int j = k; j < NE; ++j) M[i][j] -= f * M[k][j];
            r[i] -= f * r[k];
        }
    }
#pragma unroll
    for (int k = NE - 1; k >= 0; --k) {
        double acc = r[k];
#pragma unroll
        for (int j = k + 1; j < NE; ++j) acc -= M[k][j] * r[j];
        r[k] = acc / M[k][k];
        if (!isfinite(r[k])) ok = false;
    }
    return ok;
}

// Matrix of a tuple with K = log2(NE) modes of width 2.  Dm[j] is the 2x2
// diagonal block (row-major) of the j-th such mode in increasing mode order;
// the last of them owns bit 0 of the local unknown index.  c is the sum of the
// 1x1 diagonal entries of the other modes:  M = sum_j I (x) D_j (x) I + c I.
template <int NE>
__device__ inline void tuple_matrix(double (&M)[NE][NE], const double (&Dm)[4][4], double c) {
    constexpr int K = (NE == 2) ? 1 : (NE == 4) ? 2 : (NE == 8) ? 3 : 4;
#pragma unroll
    for (int q = 0; q < NE; ++q)
#pragma unroll
        for (int q2 = 0; q2 < NE; ++q2) {
            double m = (q == q2) ? c : 0.0;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int b = K - 1 - j;
                if (((q ^ q2) & ~(1 << b)) == 0) m += Dm[j][((q >> b) & 1) * 2 + ((q2 >> b) & 1)];
            }
            M[q][q2] = m;
        }
}

// 4 unknowns (2x2 blocks in two modes): with D_0 = [p q; r t] and
// K = D_1 + c I, the splitting below reduces to two 2x2 solves (Cramer).
__device__ inline bool tuple_solve4(const double (&Dm)[4][4], double c, double (&b)[4]) {
    const double p = Dm[0][0], q = Dm[0][1], r = Dm[0][2], t = Dm[0][3];
    const double k00 = Dm[1][0] + c, k01 = Dm[1][1], k10 = Dm[1][2], k11 = Dm[1][3] + c;
    // S = K + tI, Q = S (K + pI) - q r I, rhs = S b0 - q b1
    const double s00 = k00 + t, s11 = k11 + t;
    const double q00 = s00 * (k00 + p) + k01 * k10 - q * r, q01 = s00 * k01 + k01 * (k11 + p);
    const double q10 = k10 * (k00 + p) + s11 * k10, q11 = k10 * k01 + s11 * (k11 + p) - q * r;
    const double y0 = s00 * b[0] + k01 * b[1] - q * b[2], y1 = k10 * b[0] + s11 * b[1] - q * b[3];
    const double dq = q00 * q11 - q01 * q10;
    const double x0 = (q11 * y0 - q01 * y1) / dq, x1 = (q00 * y1 - q10 * y0) / dq;
    const double z0 = b[2] - r * x0, z1 = b[3] - r * x1;
    const double ds = s00 * s11 - k01 * k10;
    const double x2 = (s11 * z0 - k01 * z1) / ds, x3 = (s00 * z1 - k10 * z0) / ds;
    b[0] = x0;
    b[1] = x1;
    b[2] = x2;
    b[3] = x3;
    return dq != 0.0 && ds != 0.0 && isfinite(x0) && isfinite(x1) && isfinite(x2) && isfinite(x3);
}

// 8 unknowns: with D_0 = [p q; r t] and K the 4x4 matrix of the other two
// 2x2 modes (plus c I), the system splits into
//   (K + pI) x0 + q x1 = b0,   r x0 + (K + tI) x1 = b1,
// so with S = K + tI (the 4-unknown matrix with shift c + t):
//   [S^2 + (p - t) S - q r I] x0 = S b0 - q b1   (dense 4x4), and
//   S x1 = b1 - r x0                             (4-unknown tuple solve).
// S is rebuilt by the second solve, so the elimination holds only Q.
__device__ inline bool tuple_solve8(const double (&Dm)[4][4], double c, double (&b)[8]) {
    const double p = Dm[0][0], q = Dm[0][1], r = Dm[0][2], t = Dm[0][3];
    const double D2[4][4] = {{Dm[1][0], Dm[1][1], Dm[1][2], Dm[1][3]},
                             {Dm[2][0], Dm[2][1], Dm[2][2], Dm[2][3]},
                             {0, 0, 0, 0},
                             {0, 0, 0, 0}};
    double Q[4][4], rhs[4];
    {
        double S[4][4];
        tuple_matrix<4>(S, D2, c + t);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double acc = (p - t) * S[i][j] + ((i == j) ? -q * r : 0.0);
#pragma unroll
                for (int l = 0; l < 4; ++l) acc = fma(S[i][l], S[l][j], acc);
                Q[i][j] = acc;
            }
            double acc = -q * b[4 + i];
#pragma unroll
            for (int l = 0; l < 4; ++l) acc = fma(S[i][l], b[l], acc);
            rhs[i] = acc;
        }
    }
    bool ok = gepp_small<4>(Q, rhs);
    double r4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        b[i] = rhs[i];
        r4[i] = b[4 + i] - r * rhs[i];
    }
    ok = tuple_solve4(D2, c + t, r4) && ok;
#pragma unroll
    for (int i = 0; i < 4; ++i) b[4 + i] = r4[i];
    return ok;
}

// 16 unknowns (2x2 blocks in four modes) by the same splitting along the
// first block: K is the 8x8 matrix of the other three modes plus c I,
//   [K^2 + (p + t) K + (p t - q r) I] x0 = (K + tI) b0 - q b1   (dense 8x8),
//   (K + tI) x1 = b1 - r x0                                    (8 unknowns).
__device__ inline bool tuple_solve16(const double (&Dm)[4][4], double c, double (&b)[16]) {
    const double p = Dm[0][0], q = Dm[0][1], r = Dm[0][2], t = Dm[0][3];
    double D3[4][4] = {{Dm[1][0], Dm[1][1], Dm[1][2], Dm[1][3]},
                       {Dm[2][0], Dm[2][1], Dm[2][2], Dm[2][3]},
                       {Dm[3][0], Dm[3][1], Dm[3][2], Dm[3][3]},
                       {0, 0, 0, 0}};
    double Q[8][8], rhs[8];
    {
        double K[8][8];
        tuple_matrix<8>(K, D3, c);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                double acc = (p + t) * K[i][j] + (i == j ? p * t - q * r : 0.0);
#pragma unroll
                for (int l = 0; l < 8; ++l) acc = fma(K[i][l], K[l][j], acc);
                Q[i][j] = acc;
            }
            double acc = t * b[i] - q * b[8 + i];
#pragma unroll
            for (int l = 0; l < 8; ++l) acc = fma(K[i][l], b[l], acc);
            rhs[i] = acc;
        }
    }
    bool ok = gepp_small<8>(Q, rhs);
    double r8[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        b[i] = rhs[i];
        r8[i] = b[8 + i] - r * rhs[i];
    }
    ok = tuple_solve8(D3, c + t, r8) && ok;
#pragma unroll
    for (int i = 0; i < 8; ++i) b[8 + i] = r8[i];
    return ok;
}

// The same solve as a call: the 512-thread order-4 leaf has half the
// registers of the 256-thread one, and inlined, the sixteen-unknown solve
// would spill registers of the whole kernel.
__device__ __attribute__((noinline)) bool tuple_solve16_call(const double (&Dm)[4][4], double c, double (&b)[16]) {
    return tuple_solve16(Dm, c, b);
}

// Exact e / s for 0 <= e < 2^16 and s >= 1, from rs = 1.0f / s: the value
// (e + 0.5) / s < 2^16 / s lies at least 0.5 / s from an integer, while the
// float product is off by at most 2^-23 * 2^16 / s = 2^-7 / s.
__device__ inline int qdiv(int e, float rs) { return (int)(((float)e + 0.5f) * rs); }

constexpr int kLoadBatch = 8;

// sum_{j < len} L[to + j] L[xo + j xs] along one fibre (LDS offsets in
// doubles), four terms per step.  The T rows carry four zeros past their end
// and the X index is clamped to the fibre, so the last step needs no masking.
__device__ inline double lds_dot(const double* L, int to, int xo, int xs, int len) {
    double a0 = 0.0, a1 = 0.0;
    const int last = xo + (len - 1) * xs;
    for (int j = 0; j < len; j += 4) {
        const int x0 = xo + j * xs;
        a0 = fma(L[to + j], L[x0], a0);
        a1 = fma(L[to + j + 1], L[min(x0 + xs, last)], a1);
        a0 = fma(L[to + j + 2], L[min(x0 + 2 * xs, last)], a0);
        a1 = fma(L[to + j + 3], L[min(x0 + 3 * xs, last)], a1);
    }
    return a0 + a1;
}

// The same sum split over a pair of lanes: lane q of the pair takes the terms
// j = q, q + 2, ...; T past the row end is the first zero of its padding.
__device__ inline double lds_dot_pair(const double* L, int to, int xo, int xs, int len, int q) {
    double a0 = 0.0, a1 = 0.0;
    const int last = xo + (len - 1) * xs, tz = to + len;
    for (int j = q; j < len; j += 8) {
        const int x0 = xo + j * xs;
        a0 = fma(L[to + j], L[x0], a0);
        a1 = fma(L[min(to + j + 2, tz)], L[min(x0 + 2 * xs, last)], a1);
        a0 = fma(L[min(to + j + 4, tz)], L[min(x0 + 4 * xs, last)], a0);
        a1 = fma(L[min(to + j + 6, tz)], L[min(x0 + 6 * xs, last)], a1);
    }
    return a0 + a1;
}

// Small system of a tuple with 2x2 blocks in some modes (a: first rows,
// w: widths); the right-hand sides of its unknowns are already in Xs.
template <int D, bool CALL16 = false>
__device__ inline bool coupled_solve(double* Xs, double* const (&Ts)[D], const int (&tp)[D], const int (&ls)[D],
                                     const int (&a)[D], const int (&w)[D], int e0) {
    int ne = 1;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) ne *= w[mu];
    double cdiag = 0.0, Dm[4][4];
    int kb = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) Dm[j][v] = 0.0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const double* Tm = Ts[mu] + a[mu] * tp[mu] + a[mu];
        if (w[mu] == 2) {
            const double d0 = Tm[0], d1 = Tm[1], d2 = Tm[tp[mu]], d3 = Tm[tp[mu] + 1];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j == kb) {
                    Dm[j][0] = d0;
                    Dm[j][1] = d1;
                    Dm[j][2] = d2;
                    Dm[j][3] = d3;
                }
            ++kb;
        } else {
            cdiag += Tm[0];
        }
    }
    constexpr int NEMAX = 1 << D;
    int eq[NEMAX];
    double rb[NEMAX];
#pragma unroll
    for (int q = 0; q < NEMAX; ++q) {
        // unknown q: the last width-2 mode owns bit 0
        int e = e0, rq = q;
#pragma unroll
        for (int mu = D - 1; mu >= 0; --mu) {
            const int d = (w[mu] == 2) ? (rq & 1) : 0;
            if (w[mu] == 2) rq >>= 1;
            e += d * ls[mu];
        }
        eq[q] = e;
        rb[q] = (q < ne) ? Xs[e] : 0.0;
    }
    bool ok = true;
    if (ne == 2) {
        const double m00 = Dm[0][0] + cdiag, m01 = Dm[0][1], m10 = Dm[0][2], m11 = Dm[0][3] + cdiag;
        const double det = m00 * m11 - m01 * m10;
        const double x0 = (m11 * rb[0] - m01 * rb[1]) / det;
        const double x1 = (m00 * rb[1] - m10 * rb[0]) / det;
        if (det == 0.0 || !isfinite(x0) || !isfinite(x1)) ok = false;
        Xs[eq[0]] = x0;
        Xs[eq[1]] = x1;
    } else if (ne == 4) {
        double r4[4] = {rb[0], rb[1], rb[2], rb[3]};
        if (!tuple_solve4(Dm, cdiag, r4)) ok = false;
#pragma unroll
        for (int q = 0; q < 4; ++q) Xs[eq[q]] = r4[q];
    } else if (ne == 8) {
        double r8[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) r8[q] = rb[q];
        if (!tuple_solve8(Dm, cdiag, r8)) ok = false;
#pragma unroll
        for (int q = 0; q < 8; ++q) Xs[eq[q]] = r8[q];
    } else {
        if constexpr (D == 4) {  // 2x2 blocks in every mode
            double r16[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) r16[q] = rb[q];
            if (!(CALL16 ? tuple_solve16_call(Dm, cdiag, r16) : tuple_solve16(Dm, cdiag, r16))) ok = false;
#pragma unroll
            for (int q = 0; q < 16; ++q) Xs[eq[q]] = r16[q];
        }
    }
    return ok;
}

// Explicit inverse of the matrix of a tuple with two or four unknowns (2x2
// blocks in one or two modes) and the LDS offsets of its unknowns; the
// matrix depends on T only, so this runs before the unknowns' right-hand
// sides exist.  With the first 2x2 block D_0 = [p q; r t], K = D_1 + c I and
// Q = (K + tI)(K + pI) - q r I, the four-unknown matrix [K + pI, qI; rI, K + tI]
// has the inverse [Q^-1 (K + tI), -q Q^-1; -r Q^-1, (K + pI) Q^-1] (all blocks
// are polynomials in K, so they commute).
template <int D>
__device__ inline bool tuple_inverse(double* const (&Ts)[D], const int (&tp)[D], const int (&ls)[D],
                                     const int (&a)[D], const int (&w)[D], double (&Mi)[4][4], int (&eq)[4]) {
    double cdiag = 0.0, p = 0.0, q = 0.0, r = 0.0, t = 0.0, k00 = 0.0, k01 = 0.0, k10 = 0.0, k11 = 0.0;
    int ne = 1, e0 = 0, s0 = 0, s1 = 0;  // strides of the width-2 modes (bit 1, bit 0 of the unknown index)
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const double* Tm = Ts[mu] + a[mu] * tp[mu] + a[mu];
        e0 += a[mu] * ls[mu];
        if (w[mu] == 2) {
            const double d0 = Tm[0], d1 = Tm[1], d2 = Tm[tp[mu]], d3 = Tm[tp[mu] + 1];
            // the first width-2 mode lands in (p q r t), the second in K
            if (ne == 1) {
                p = d0, q = d1, r = d2, t = d3;
                s1 = ls[mu];
            } else {
                k00 = d0, k01 = d1, k10 = d2, k11 = d3;
                s0 = ls[mu];
            }
            ne *= 2;
        } else {
            cdiag += Tm[0];
        }
    }
    if (ne == 2) {
        const double m00 = p + cdiag, m11 = t + cdiag;
        const double rd = 1.0 / (m00 * m11 - q * r);
        Mi[0][0] = m11 * rd, Mi[0][1] = -q * rd;
        Mi[1][0] = -r * rd, Mi[1][1] = m00 * rd;
        eq[0] = e0, eq[1] = e0 + s1, eq[2] = e0, eq[3] = e0;
        return isfinite(rd);
    }
    k00 += cdiag, k11 += cdiag;
    // S = K + tI, P = K + pI, Q = S P - q r I
    const double s00 = k00 + t, s11 = k11 + t, p00 = k00 + p, p11 = k11 + p;
    const double q00 = s00 * p00 + k01 * k10 - q * r, q01 = s00 * k01 + k01 * p11;
    const double q10 = k10 * p00 + s11 * k10, q11 = k10 * k01 + s11 * p11 - q * r;
    const double rd = 1.0 / (q00 * q11 - q01 * q10);
    const double i00 = q11 * rd, i01 = -q01 * rd, i10 = -q10 * rd, i11 = q00 * rd;  // Q^-1
    Mi[0][0] = i00 * s00 + i01 * k10, Mi[0][1] = i00 * k01 + i01 * s11;
    Mi[1][0] = i10 * s00 + i11 * k10, Mi[1][1] = i10 * k01 + i11 * s11;
    Mi[0][2] = -q * i00, Mi[0][3] = -q * i01, Mi[1][2] = -q * i10, Mi[1][3] = -q * i11;
    Mi[2][0] = -r * i00, Mi[2][1] = -r * i01, Mi[3][0] = -r * i10, Mi[3][1] = -r * i11;
    Mi[2][2] = p00 * i00 + k01 * i10, Mi[2][3] = p00 * i01 + k01 * i11;
    Mi[3][2] = k10 * i00 + p11 * i10, Mi[3][3] = k10 * i01 + p11 * i11;
    // unknown index: bit 1 -> first width-2 mode, bit 0 -> second
    eq[0] = e0, eq[1] = e0 + s0, eq[2] = e0 + s1, eq[3] = e0 + s1 + s0;
    return isfinite(rd);
}

}  // namespace

// NT threads per leaf: 256 for blocks up to 16^3 (three such workgroups share
// a CU: ~50 KB of LDS each), 64 (one wave, no cross-wave barriers) for blocks
// up to 10^3, whose hyperplanes hold at most ~75 unknowns; 512 (two lanes per
// unknown) for launches with few leaves.  The order-3 kernel is held to
// three waves per SIMD worth of registers; the 256-thread order-4 kernel
// keeps its 16-unknown tuple solve in registers (one wave per SIMD), the
// 512-thread one (two waves per SIMD) calls it out of line.  OCC = 2: the
// 256-thread order-4 kernel at two waves per SIMD (the 16-unknown solve out
// of line, some registers spilled), for launches of more than two leaves
// per CU, where two leaves per CU outrun one faster leaf.
template <int D, int NT, int OCC = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(OCC ? OCC : (D == 4 ? 1 : 3)))) void leaf_kernel(const LeafDesc* __restrict__ leaves, int64_t first,
                                                      const ProbDesc* __restrict__ probs,
                                                      const LeafShape* __restrict__ shapes,
                                                      const uint16_t* __restrict__ ents,
                                                      const int32_t* __restrict__ hoffs, int* status,
                                                      LeafGeom geom) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    constexpr int LPE = (NT > kLeafNT) ? 2 : 1;  // lanes per unknown in the dot products
    const LeafDesc L = leaves[first + blockIdx.x];
    const ProbDesc& P = probs[L.prob];

    int r0[D], sz[D], ls[D], nx[D];
    int64_t gs[D];
    float rsz[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const int b = L.blk[mu];
        const auto* bst = to_global(P.bst[mu]);
        r0[mu] = bst[b];
        const int r1 = bst[b + 1];
        sz[mu] = r1 - r0[mu];
        nx[mu] = ((L.flags >> (4 + mu)) & 1) ? bst[b + 2] - r1 : 0;
        gs[mu] = P.stride[mu];
        rsz[mu] = 1.0f / (float)sz[mu];
    }
    ls[D - 1] = 1;
#pragma unroll
    for (int mu = D - 2; mu >= 0; --mu) ls[mu] = ls[mu + 1] * sz[mu + 1];
    const int cap = ls[0] * sz[0];

    // LDS: Xs | Ts (diagonal blocks, row pitch sz + 4, zero padded) | union
    // {adjacent T blocks (one part per mode); element records + coupled-tuple list} | per-mode
    // bit tables | offsets
    double* Xs = lds;
    double* Ts[D];
    int toff[D], tp[D];  // offsets of Ts[mu] from lds (doubles), row pitch
    {
        int o = geom.cap;
#pragma unroll
        for (int mu = 0; mu < D; ++mu) {
            Ts[mu] = lds + o;
            toff[mu] = o;
            tp[mu] = sz[mu] + 4;
            o += geom.bm[mu] * (geom.bm[mu] + 4);
        }
    }
    double* Ta = lds + geom.cap + geom.tsum;
    uint16_t* rec = (uint16_t*)Ta;                         // geom.cap element records
    uint16_t* clist = rec + geom.cap;                      // geom.maxcpl coupled tuples
    uint64_t* rbits = (uint64_t*)(Ta + geom.uwords);       // row -> 2 bits: gap - 1, width - 1
    uint32_t* tbits = (uint32_t*)(rbits + D);              // tuple -> 1 bit: width - 1
    int32_t* hof = (int32_t*)(tbits + D + (D & 1));        // tuple offsets per hyperplane
    int32_t* eoff = hof + geom.maxH + 1;                   // element offsets per hyperplane
    int32_t* coff = eoff + geom.maxH + 1;                  // coupled-tuple offsets per hyperplane
    int32_t* wsum = coff + geom.maxH + 1;                  // wave totals of the block scan
    const LeafShape sh = shapes[L.shape];
    for (int i = tid; i <= sh.H; i += NT) hof[i] = hoffs[sh.hoff + i];

    gdouble* __restrict__ X = to_global(P.X);
    int64_t gbase = 0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) gbase += (int64_t)r0[mu] * gs[mu];

    // local element index -> global offset (relative to gbase)
    auto goff = [&](int e) {
        int64_t g = 0;
#pragma unroll
        for (int mu = D - 1; mu >= 1; --mu) {
            const int q = qdiv(e, rsz[mu]);
            g += (int64_t)(e - q * sz[mu]) * gs[mu];
            e = q;
        }
        return g + (int64_t)e * gs[0];
    };

    // ---- 1. right-hand side and diagonal blocks: from X when mode-0 updates
    // have reached the block (they start from B), else from B itself
    const gdouble* __restrict__ rhs = (L.flags & 1) ? X : to_global(P.B);
    for (int base = 0; base < cap; base += NT * kLoadBatch) {
        double v[kLoadBatch];
        int64_t g[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int e = base + u * NT + tid;
            g[u] = (e < cap) ? gbase + goff(e) : -1;
            v[u] = (g[u] >= 0) ? rhs[g[u]] : 0.0;
        }
#pragma unroll
        for (int mu = 1; mu < D; ++mu) {
            if (!((L.flags >> mu) & 1)) continue;  // uniform
            const gdouble* __restrict__ A = to_global(P.A[mu]);
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u)
                if (g[u] >= 0) v[u] -= A[g[u]];
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int e = base + u * NT + tid;
            if (e < cap) Xs[e] = v[u];
        }
    }
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const gdouble* T = to_global(P.T[mu]);
        const int64_t n = P.n[mu];
        const float rtp = 1.0f / (float)tp[mu];
        for (int e = tid; e < sz[mu] * tp[mu]; e += NT) {
            const int i = qdiv(e, rtp), j = e - i * tp[mu];
            Ts[mu][e] = (j < sz[mu]) ? T[(int64_t)(r0[mu] + i) * n + r0[mu] + j] : 0.0;
        }
    }
    __syncthreads();

    // ---- 2. 1x1 / 2x2 diagonal blocks of every mode (thread mu scans its block)
    if (tid < D) {
        const int mu = tid;
        int m = sz[0], t0 = toff[0], pt = tp[0];
#pragma unroll
        for (int nu = 1; nu < D; ++nu)
            if (nu == mu) {
                m = sz[nu];
                t0 = toff[nu];
                pt = tp[nu];
            }
        int p = 0, i = 0;
        uint64_t rb = 0;
        uint32_t tb = 0;
        while (i < m) {
            const int w = (i + 1 < m && lds[t0 + (i + 1) * pt + i] != 0.0) ? 2 : 1;
            if (w == 2) {
                rb |= (uint64_t)3 << (2 * i) | (uint64_t)2 << (2 * i + 2);  // gap 2 / 1, width 2
                tb |= 1u << p;
            }
            i += w;
            ++p;
        }
        rbits[mu] = rb;
        tbits[mu] = tb;
    }

    // ---- 3. contributions of the next block along each mode,
    // T_mu[B, B+1] x_mu X[B+1]: T_mu[B, B+1] staged in LDS (mode mu's part
    // of the union region, odd row pitch), one thread per fibre along mu
    auto ta_of = [&](int mu) { return Ta + mu * geom.tamax; };
    // row pitch: 17 with zeros past nx (one unmasked chunk of sixteen
    // columns), else nx | 1
    auto ta_pitch = [&](int mu) { return nx[mu] <= 16 ? 17 : (nx[mu] | 1); };
    auto stage = [&](int mu) {
        const int nxm = nx[mu], tpn = ta_pitch(mu), r1 = r0[mu] + sz[mu];
        const int w = (nxm <= 16) ? 16 : nxm;
        const gdouble* T = to_global(P.T[mu]);
        const int64_t n = P.n[mu];
        double* ta = ta_of(mu);
        for (int e = tid; e < sz[mu] * w; e += NT) {
            const int i = e / w, j = e - (e / w) * w;
            ta[i * tpn + j] = (j < nxm) ? T[(int64_t)(r0[mu] + i) * n + r1 + j] : 0.0;
        }
    };
    auto fibre_origin = [&](int mu, int f, int& eb, int64_t& gb) {
        eb = 0;
        gb = gbase;
        int rem = f;
#pragma unroll
        for (int nu = D - 1; nu >= 0; --nu) {
            if (nu == mu) continue;
            const int q = qdiv(rem, rsz[nu]);
            const int c = rem - q * sz[nu];
            rem = q;
            eb += c * ls[nu];
            gb += (int64_t)c * gs[nu];
        }
    };
    // the fibre of the next block, sixteen rows at a time in registers
    // (clamped loads, zeroed past nx)
    auto load16 = [&](int mu, int64_t gb, int jc, double (&xn)[16]) {
        const int64_t nstep = (int64_t)sz[mu] * gs[mu];  // from row r0+i to row r1+i
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const bool v = jc + j < nx[mu];
            const double x = X[gb + nstep + (int64_t)(v ? jc + j : jc) * gs[mu]];
            xn[j] = v ? x : 0.0;
        }
    };
    // one row of T_mu[B, B+1] per output element; each lane starts its row
    // loop at its own row: the fibres of consecutive lanes lie a power of two
    // apart for some modes, and in step they would all update one LDS bank
    // (with the odd pitch the T reads of different rows fall in different
    // banks too)
    auto apply16 = [&](int mu, int eb, int jc, const double (&xn)[16]) {
        const int nxm = nx[mu], tpn = ta_pitch(mu), rot = tid % sz[mu];
        const double* ta = ta_of(mu);
        if (nxm <= 16) {  // uniform: zero padded, no masking
            for (int ii = 0; ii < sz[mu]; ++ii) {
                const int i = (ii + rot < sz[mu]) ? ii + rot : ii + rot - sz[mu];
                const double* ti = ta + i * tpn;
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int j = 0; j < 16; j += 2) {
                    a0 = fma(ti[j], xn[j], a0);
                    a1 = fma(ti[j + 1], xn[j + 1], a1);
                }
                Xs[eb + i * ls[mu]] -= a0 + a1;
            }
            return;
        }
        for (int ii = 0; ii < sz[mu]; ++ii) {
            const int i = (ii + rot < sz[mu]) ? ii + rot : ii + rot - sz[mu];
            const double* ti = ta + i * tpn + jc;
            double a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int j = 0; j < 16; j += 2) {
                const double t0 = (jc + j < nxm) ? ti[(jc + j < nxm) ? j : 0] : 0.0;
                const double t1 = (jc + j + 1 < nxm) ? ti[(jc + j + 1 < nxm) ? j + 1 : 0] : 0.0;
                a0 = fma(t0, xn[j], a0);
                a1 = fma(t1, xn[j + 1], a1);
            }
            Xs[eb + i * ls[mu]] -= a0 + a1;
        }
    };
    {
#pragma unroll
        for (int mu = 0; mu < D; ++mu) {
            if (nx[mu] == 0) continue;  // uniform over the workgroup
            stage(mu);
            const int F = cap / sz[mu];
            // at most one fibre per thread and one chunk: its loads are
            // issued before the barrier that publishes the T block
            const bool one = F <= NT && nx[mu] <= 16;  // uniform
            double xp[16];
            int ebp = 0;
            if (one && tid < F) {
                int64_t gb = 0;
                fibre_origin(mu, tid, ebp, gb);
                load16(mu, gb, 0, xp);
            }
            __syncthreads();
            if (one) {
                if (tid < F) apply16(mu, ebp, 0, xp);
            } else {
                for (int f = tid; f < F; f += NT) {
                    int eb = 0;
                    int64_t gb = 0;
                    fibre_origin(mu, f, eb, gb);
                    for (int jc = 0; jc < nx[mu]; jc += 16) {
                        double xn[16];
                        load16(mu, gb, jc, xn);
                        apply16(mu, eb, jc, xn);
                    }
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();  // tables of step 2 visible, Ta free
    uint64_t rowbits[D];
    uint32_t tupbits[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        rowbits[mu] = rbits[mu];
        tupbits[mu] = tbits[mu];
    }

    // ---- 4. element lists: the shape's tuples expanded to their unknowns,
    // hyperplane by hyperplane, and the coupled tuples (block-wide scan)
    constexpr int kBits = (D == 4) ? kTupBits4 : kTupBits3;
    constexpr int kCB = 16 / D;  // bits of a row index in an element record
    // tuple p of mode mu starts at row p + (number of 2x2 blocks before it)
    auto decode = [&](uint32_t en, int* a, int* w) {
        int ne = 1;
#pragma unroll
        for (int mu = 0; mu < D; ++mu) {
            const int p = (en >> (kBits * mu)) & ((1 << kBits) - 1);
            a[mu] = p + __popc(tupbits[mu] & ((1u << p) - 1u));
            w[mu] = 1 + ((tupbits[mu] >> p) & 1);
            ne *= w[mu];
        }
        return ne;
    };
    {
        const int per = (sh.count + NT - 1) / NT;
        const int t0 = min(sh.count, tid * per), t1 = min(sh.count, t0 + per);
        // entries four at a time, so that their global loads overlap
        auto load4 = [&](int tb, uint32_t (&e4)[4]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) e4[u] = ents[sh.ent + min(tb + u, t1 - 1)];
        };
        int cnt = 0;  // elements | coupled tuples << 16
        for (int tb = t0; tb < t1; tb += 4) {
            uint32_t e4[4];
            load4(tb, e4);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                int a[D], w[D];
                const int ne = decode(e4[u], a, w);
                if (tb + u < t1) cnt += ne + ((ne > 1) ? (1 << 16) : 0);
            }
        }
        // exclusive block scan: wave scan by shuffles, then wave totals
        const int lane = tid & 63, wv = tid >> 6;
        int inc = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(inc, d, 64);
            if (lane >= d) inc += v;
        }
        if (lane == 63) wsum[wv] = inc;
        __syncthreads();
        int before = 0;
        for (int k = 0; k < wv; ++k) before += wsum[k];
        int on = (before + inc - cnt) & 0xffff, oc = (before + inc - cnt) >> 16;
        int h = 0, hnext = 0;
        if (t0 < t1) {
            int lo = 0, hi = sh.H;  // hof[lo] <= t0 < hof[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (hof[mid] <= t0) lo = mid; else hi = mid;
            }
            h = lo;
            hnext = hof[h + 1];
            if (hof[h] == t0) {
                eoff[h] = on;
                coff[h] = oc;
            }
        }
        for (int tb = t0; tb < t1; tb += 4) {
            uint32_t e4[4];
            load4(tb, e4);
            for (int u = 0; u < 4 && tb + u < t1; ++u) {
                const int t = tb + u;
                if (t == hnext) {  // first tuple of the next hyperplane(s)
                    while (hof[h + 1] <= t) ++h;
                    hnext = hof[h + 1];
                    eoff[h] = on;
                    coff[h] = oc;
                }
                uint32_t e = e4[0];
#pragma unroll
                for (int k = 1; k < 4; ++k)
                    if (u == k) e = e4[k];
                int a[D], w[D];
                const int ne = decode(e, a, w);
                for (int q = 0; q < ne; ++q) {
                    // unknown q: the last width-2 mode owns bit 0
                    uint32_t r = 0;
                    int rq = q;
#pragma unroll
                    for (int mu = D - 1; mu >= 0; --mu) {
                        const int d = (w[mu] == 2) ? (rq & 1) : 0;
                        if (w[mu] == 2) rq >>= 1;
                        r |= (uint32_t)(a[mu] + d) << (kCB * mu);
                    }
                    rec[on++] = (uint16_t)r;
                }
                if (ne > 1) clist[oc++] = (uint16_t)e;
            }
        }
        if (tid == NT - 1) {
            eoff[sh.H] = on;
            coff[sh.H] = oc;
        }
    }
    __syncthreads();

    // ---- 5. block back-substitution, one tuple hyperplane per step.
    // Coupled tuples with up to four unknowns are taken by the highest
    // threads, which hold no unknowns of the step while its hyperplane has
    // fewer than NT - (coupled tuples) unknowns: they invert their small
    // matrix (T only) while the other threads form right-hand sides, and
    // apply the inverse after the barrier.  (A) every unknown forms its
    // right-hand side (unknowns of 1x1 tuples also divide by their
    // eigenvalue sum), (B)
    // coupled tuples solve their small systems.
    bool ok = true;
    for (int h = 0; h < sh.H; ++h) {
        const int ebeg = eoff[h], eend = eoff[h + 1];
        const int cbeg = coff[h], cend = coff[h + 1];
        const int kc = cbeg + (NT - 1 - tid);
        uint32_t cen = 0;
        // defined on every path, so nothing of a previous step stays live
        int pne = 0, peq[4] = {0, 0, 0, 0};
        double Mi[4][4] = {};
        if (kc < cend) {
            int a[D], w[D];
            cen = clist[kc];
            pne = decode(cen, a, w);
            if (pne <= 4 && !tuple_inverse<D>(Ts, tp, ls, a, w, Mi, peq)) ok = false;
        }
        // LPE lanes per unknown: both lanes of a pair take the same unknown,
        // so they stay converged for the exchange of their partial sums
        for (int i = ebeg + tid / LPE; i < eend; i += NT / LPE) {
            const uint32_t r = rec[i];
            int c[D], e = 0;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) {
                c[mu] = (r >> (kCB * mu)) & ((1 << kCB) - 1);
                e += c[mu] * ls[mu];
            }
            double cd = 0.0, acc = 0.0;
            bool single = true;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) {
                const int b2 = (int)(rowbits[mu] >> (2 * c[mu])) & 3;
                const int gap = 1 + (b2 & 1);
                single = single && !(b2 & 2);
                const int dg = toff[mu] + c[mu] * (tp[mu] + 1);
                cd += lds[dg];
                if constexpr (LPE == 1)
                    acc += lds_dot(lds, dg + gap, e + gap * ls[mu], ls[mu], sz[mu] - c[mu] - gap);
                else
                    acc += lds_dot_pair(lds, dg + gap, e + gap * ls[mu], ls[mu], sz[mu] - c[mu] - gap, tid & 1);
            }
            if constexpr (LPE == 2) acc += __shfl_xor(acc, 1);
            if (LPE == 1 || (tid & 1) == 0) {
                const double rhs = lds[e] - acc;
                if (single) {
                    const double x = rhs / cd;
                    if (cd == 0.0 || !isfinite(x)) ok = false;
                    lds[e] = x;
                } else {
                    lds[e] = rhs;
                }
            }
        }
        if (cend > cbeg) {  // uniform
            __syncthreads();
            if (pne == 2 || pne == 4) {
                double rb[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) rb[q] = Xs[peq[q]];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q >= pne) break;
                    double x = 0.0;
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        if (s < pne) x = fma(Mi[q][s], rb[s], x);
                    if (!isfinite(x)) ok = false;
                    Xs[peq[q]] = x;
                }
            }
            // this thread's larger tuple, then tuples beyond one per thread
            for (int m = 0;; ++m) {
                const int k = m ? cbeg + m * NT + tid : kc;
                if (k >= cend) break;
                if (m == 0 && pne <= 4) continue;
                int a[D], w[D];
                decode(clist[k], a, w);
                int e0 = 0;
#pragma unroll
                for (int mu = 0; mu < D; ++mu) e0 += a[mu] * ls[mu];
                if (!coupled_solve<D, (D == 4 && (NT > kLeafNT || OCC == 2))>(Xs, Ts, tp, ls, a, w, e0)) ok = false;
            }
        }
        __syncthreads();
    }
    if (!ok) atomicOr(status, 1);

    // ---- 6. store the solved block
    for (int base = 0; base < cap; base += NT * kLoadBatch) {
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int e = base + u * NT + tid;
            if (e < cap) X[gbase + goff(e)] = Xs[e];
        }
    }
}

LeafGeom leaf_geometry(int D, const int* bmax, int maxtup, int maxcpl, int maxH) {
    LeafGeom g{};
    g.maxtup = maxtup;
    g.maxcpl = maxcpl;
    g.maxH = maxH;
    g.cap = 1;
    for (int mu = 0; mu < kMaxD; ++mu) g.bm[mu] = (mu < D) ? bmax[mu] : 1;
    for (int mu = 0; mu < D; ++mu) {
        g.cap *= bmax[mu];
        g.tsum += bmax[mu] * (bmax[mu] + 4);
        // T_mu[B, B+1] at an odd pitch (17 for up to sixteen columns)
        g.tamax = std::max(g.tamax, bmax[mu] * std::max(17, bmax[mu] | 1));
    }
    // union of the adjacent block (doubles) and the element records plus the
    // coupled-tuple list (u16 each)
    g.uwords = std::max(D * g.tamax, ((g.cap + maxcpl) * 2 + 7) / 8);
    return g;
}

int leaf_lds_bytes(int D, const int* bmax, int maxtup, int maxcpl, int maxH) {
    const LeafGeom g = leaf_geometry(D, bmax, maxtup, maxcpl, maxH);
    return (g.cap + g.tsum + g.uwords + D) * (int)sizeof(double) + (D + 1) * (int)sizeof(uint32_t) +
           (3 * (maxH + 1) + kLeafNTWide / 64) * (int)sizeof(int32_t);
}

hipError_t launch_leaf(int D, const LeafDesc* leaves, int64_t first, int64_t count, const ProbDesc* probs,
                       const LeafShape* shapes, const uint16_t* ents, const int32_t* hoffs, int* status,
                       const int* bmax, int maxtup, int maxcpl, int maxH, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int lds = leaf_lds_bytes(D, bmax, maxtup, maxcpl, maxH);
    const LeafGeom geom = leaf_geometry(D, bmax, maxtup, maxcpl, maxH);
    const bool small = geom.cap <= 1000;
    // a launch with at most one leaf per CU gives each order-3 leaf 512
    // threads (two lanes per unknown): the CU would otherwise hold one
    // 256-thread leaf and idle; order 4 (whose 512-thread kernel spills
    // registers) takes it with at most one leaf per two CUs
    int cus = 0, dev = 0;  // CUs of the current device (queried per launch: a process may drive several GPUs)
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 0;
    const bool wide = !small && cus > 0 && count <= ((D == 4) ? cus / 2 : cus);
    const bool dense4 = D == 4 && !small && cus > 0 && count > 2 * (int64_t)cus;
    dim3 grid((unsigned)count), block(small ? 64 : (wide ? kLeafNTWide : kLeafNT));
    const void* fn = (D == 3) ? (small ? (const void*)leaf_kernel<3, 64>
                                       : (wide ? (const void*)leaf_kernel<3, kLeafNTWide>
                                               : (const void*)leaf_kernel<3, kLeafNT>))
                              : (small ? (const void*)leaf_kernel<4, 64>
                                       : (wide ? (const void*)leaf_kernel<4, kLeafNTWide>
                                               : (dense4 ? (const void*)leaf_kernel<4, kLeafNT, 2>
                                                         : (const void*)leaf_kernel<4, kLeafNT>)));
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    if (wide && D == 4)
        hipLaunchKernelGGL((leaf_kernel<4, kLeafNTWide>), grid, block, lds, st, leaves, first, probs, shapes, ents,
                           hoffs, status, geom);
    else if (wide)
        hipLaunchKernelGGL((leaf_kernel<3, kLeafNTWide>), grid, block, lds, st, leaves, first, probs, shapes, ents,
                           hoffs, status, geom);
    else if (D == 3 && small)
        hipLaunchKernelGGL((leaf_kernel<3, 64>), grid, block, lds, st, leaves, first, probs, shapes, ents, hoffs,
                           status, geom);
    else if (D == 3)
        hipLaunchKernelGGL((leaf_kernel<3, kLeafNT>), grid, block, lds, st, leaves, first, probs, shapes, ents, hoffs,
                           status, geom);
    else if (small)
        hipLaunchKernelGGL((leaf_kernel<4, 64>), grid, block, lds, st, leaves, first, probs, shapes, ents, hoffs,
                           status, geom);
    else if (dense4)
        hipLaunchKernelGGL((leaf_kernel<4, kLeafNT, 2>), grid, block, lds, st, leaves, first, probs, shapes, ents,
                           hoffs, status, geom);
    else
        hipLaunchKernelGGL((leaf_kernel<4, kLeafNT>), grid, block, lds, st, leaves, first, probs, shapes, ents,
                           hoffs, status, geom);
    return hipGetLastError();
}

}  // namespace tt
