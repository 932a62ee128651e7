// Leaf solve of the second operator class (Sec. 3, gfx950).
//
// After the exact reduction by C^{-1} (Sec. 3) the equation reads
//   X x_0 T_0 + X x_1 A_1 x_2 A_2 .. x_{D-1} A_{D-1} = B
// (internal modes 0..D-1; T_0 = C^{-1} A_1 of the paper and A_1 .. A_{D-1}
// its A_2 .. A_d, all upper quasi-triangular).  Element i depends on the
// elements that are larger in mode 0 alone (T_0) and on every element of the
// orthant j_nu >= i_nu, nu >= 1, at the same i_0 (the product term).  The
// block schedule is the Laplace-like one; what reaches a leaf block I from
// outside is
//   * mode 0: T_0[I_0, J_0] x_0 X[J_0, I'] (already in X, as for the
//     Laplace-like form, plus the adjacent block applied here);
//   * the product term over the orthant, which telescopes through the
//     partial products W_k (k = 1 .. D-2) and the accumulators V_nu of the
//     updates along mode nu (V_nu = sum over J_nu > I_nu of
//     A_nu[I_nu, J_nu] x_nu W_{nu-1}[.., J_nu, ..], W_0 = X):
//        W_k[I] = W_{k-1}[I] x_k A_k[I_k, I_k] + V_k[I],
//     so W_k[I] = Z_k + K_k with the in-block partial products
//        Z_k = X[I] x_1 A_1[I_1, I_1] .. x_k A_k[I_k, I_k]
//     and K_1 = V_1, K_k = K_{k-1} x_k A_k[I_k, I_k] + V_k.
// The same telescoping inside the block makes every unknown cost O(D n_min):
// when the unknowns of a tuple (1x1 / 2x2 diagonal blocks per mode) are
// solved, every element past the tuple in some mode is known, and with
//   S_0 = sum_{j_0 past the tuple} T_0[c_0, j_0] X[c | j_0],
//   S_k = sum_{j_k past the tuple} A_k[c_k, j_k] Z_{k-1}[c | j_k]  (Z_0 = X),
// the product term of unknown c is Z_{D-1}[c] = P x + q with P the tuple's
// Kronecker product of the diagonal blocks of A_1 .. A_{D-1} and q the same
// chain applied to the S_k: q_1 = S_1, q_k = A_k,tuple q_{k-1} + S_k.  The
// tuple system is (T_0,tuple (x) I + I (x) P) x = R - S_0 - q with
// R = B - K_{D-1} (minus the outside mode-0 terms); afterwards
// Z_k = A_k,tuple Z_{k-1} + S_k is stored for the unknowns of the tuple.
//
// One workgroup per leaf block (one wave for blocks of at most 1000
// unknowns, else 256 threads):
//   1. right-hand side and the chain K_1 .. K_{D-1} (with the adjacent
//      block along each mode, T_mu[I_mu, I_mu + 1] applied to the next
//      block's X or W_{mu-1}); W_k := K_k written for k = 1 .. D-2;
//   2. tuples hyperplane by hyperplane: 1x1 tuples one per thread in
//      registers; coupled tuples are queued; after a barrier their sums
//      past the tuple are formed one per thread, then each tuple of 2 or 4
//      unknowns is solved by one thread in registers, larger ones by sixteen
//      lanes together (Gaussian elimination with partial pivoting
//      throughout);
//   3. X stored, W_k += Z_k.
// LDS: X and Z_1 .. Z_{D-2} of the block (Z_1 holds the K chain in step 1),
// the diagonal blocks, and a union of the staged off-diagonal block with the
// sums past the coupled tuples.
#include "tt_internal.h"

#include <algorithm>
#include <vector>

namespace tt {

namespace {

constexpr int kL2NT = 256;   // threads per leaf block (one wave up to kL2Small unknowns)
constexpr int kL2Small = 1000;
constexpr int kFib = 24;     // longest fibre held in registers
static_assert(kFib >= kMaxLeaf, "fibre registers must hold a leaf block edge");

template <int D>
struct L2Tup {
    static constexpr int CH = 32;            // coupled tuples of <= 4 unknowns per round
    static constexpr int sbuf = CH * 4 * D;  // their sums past the tuple
};

// LDS carving (doubles) for the largest block of a launch.
struct L2Geom {
    int cap;     // prod bmax
    int bm;      // max bmax
    int tp;      // row pitch of the diagonal blocks (bm + 1)
    int top;     // row pitch of the staged off-diagonal block (odd)
    int oX, oZ, oTd, oU, oList, total;  // oZ: Z_1 (Z_2 after it for D = 4)
    int maxhyp;  // most tuples on one hyperplane of the largest grid
};

// most grid points with equal coordinate sum in a box of edges e[0..D-1]
int max_hyperplane(int D, const int* e) {
    std::vector<int64_t> cnt(1, 1);
    for (int mu = 0; mu < D; ++mu) {
        std::vector<int64_t> nxt(cnt.size() + (size_t)e[mu] - 1, 0);
        for (size_t s = 0; s < cnt.size(); ++s)
            for (int j = 0; j < e[mu]; ++j) nxt[s + (size_t)j] += cnt[s];
        cnt.swap(nxt);
    }
    return (int)*std::max_element(cnt.begin(), cnt.end());
}

L2Geom l2_geometry(int D, const int* bmax) {
    L2Geom g{};
    g.cap = 1;
    g.bm = 1;
    for (int mu = 0; mu < D; ++mu) {
        g.cap *= bmax[mu];
        g.bm = std::max(g.bm, bmax[mu]);
    }
    g.tp = g.bm + 1;
    g.top = g.bm | 1;
    g.oX = 0;
    g.oZ = g.cap;
    g.oTd = g.oZ + (D - 2) * g.cap;
    g.oU = g.oTd + D * g.bm * g.tp;
    const int pool = (D == 4) ? L2Tup<4>::sbuf : L2Tup<3>::sbuf;
    g.oList = g.oU + std::max(g.bm * g.top, pool);
    g.maxhyp = max_hyperplane(D, bmax);
    // coupled-tuple queue (u32) and three counters, in doubles
    g.total = g.oList + (g.maxhyp + 3 + 1) / 2;
    return g;
}

// Exact e / s for 0 <= e < 2^16 and s >= 1 from rs = 1.0f / s: the value
// (e + 0.5) / s lies at least 0.5 / s from an integer, while the float
// product is off by at most 2^-23 * 2^16 / s = 2^-7 / s.
__device__ inline int qdiv2(int e, float rs) { return (int)(((float)e + 0.5f) * rs); }

// Gaussian elimination with partial pivoting on a 4 x 4 system in registers
// (all indices static); false on a zero pivot or a non-finite result.
__device__ inline bool gepp4(double (&M)[4][4], double (&r)[4]) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int i = k + 1; i < 4; ++i) {
            const bool sw = fabs(M[i][k]) > fabs(M[k][k]);
#pragma unroll
            for (int j = k; j < 4; ++j) {
                const double t = M[k][j];
                M[k][j] = sw ? M[i][j] : t;
                M[i][j] = sw ? t : M[i][j];
            }
            const double t = r[k];
            r[k] = sw ? r[i] : t;
            r[i] = sw ? t : r[i];
        }
        if (M[k][k] == 0.0) ok = false;
        const double rp = 1.0 / M[k][k];
#pragma unroll
        for (int i = k + 1; i < 4; ++i) {
            const double f = M[i][k] * rp;
#pragma unroll
            for (int j = k + 1; j < 4; ++j) M[i][j] = fma(-f, M[k][j], M[i][j]);
            r[i] = fma(-f, r[k], r[i]);
        }
    }
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        double acc = r[k];
#pragma unroll
        for (int j = k + 1; j < 4; ++j) acc = fma(-M[k][j], r[j], acc);
        r[k] = acc / M[k][k];
        if (!isfinite(r[k])) ok = false;
    }
    return ok;
}

// sum_{j = j0}^{len - 1} row[j] src[(j - c) st]: src points at the element
// of row c, two partial sums
__device__ inline double ldot(const double* row, const double* src, int c, int j0, int len, int st) {
    double a0 = 0.0, a1 = 0.0;
    int j = j0;
    for (; j + 1 < len; j += 2) {
        a0 = fma(row[j], src[(j - c) * st], a0);
        a1 = fma(row[j + 1], src[(j + 1 - c) * st], a1);
    }
    if (j < len) a0 = fma(row[j], src[(j - c) * st], a0);
    return a0 + a1;
}

}  // namespace

template <int D, int NT>
__global__ __launch_bounds__(NT) void leaf2_kernel(const LeafDesc* __restrict__ leaves, int64_t first,
                                                      const ProbDesc* __restrict__ probs,
                                                      const LeafShape* __restrict__ shapes,
                                                      const uint16_t* __restrict__ ents,
                                                      const int32_t* __restrict__ hoffs, int* status, L2Geom g) {
    using Tup = L2Tup<D>;
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const LeafDesc L = leaves[first + blockIdx.x];
    const ProbDesc& P = probs[L.prob];
    double* Xs = lds + g.oX;
    double* Zs = lds + g.oZ;  // Z_1 (the K chain during set-up); Z_2 at Zs + cap
    double* Td = lds + g.oTd;
    double* U = lds + g.oU;   // staged off-diagonal block | coupled-tuple scratch
    uint32_t* qlist = (uint32_t*)(lds + g.oList);
    uint32_t* qcnt = qlist + g.maxhyp;  // three counters, hyperplane h uses h % 3
    const int tp = g.tp;

    int r0[D], sz[D], nx[D], ls[D];
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
    int64_t gbase = 0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) gbase += (int64_t)r0[mu] * gs[mu];
    // local element e -> global offset from gbase
    auto goff = [&](int e) {
        int64_t o = 0;
#pragma unroll
        for (int mu = D - 1; mu >= 1; --mu) {
            const int q = qdiv2(e, rsz[mu]);
            o += (int64_t)(e - q * sz[mu]) * gs[mu];
            e = q;
        }
        return o + (int64_t)e * gs[0];
    };
    // fibre f along mode mu -> local and global offsets of its first element
    auto fibre = [&](int mu, int f, int& eb, int64_t& gb) {
        eb = 0;
        gb = gbase;
#pragma unroll
        for (int nu = D - 1; nu >= 0; --nu) {
            if (nu == mu) continue;
            const int q = qdiv2(f, rsz[nu]);
            const int c = f - q * sz[nu];
            f = q;
            eb += c * ls[nu];
            gb += (int64_t)c * gs[nu];
        }
    };
    // dst += sgn * T_mu[I_mu, I_mu + 1] x_mu src[next block along mu] (src
    // global; the off-diagonal block is staged in U), one fibre per thread
    auto adjacent = [&](int mu, const gdouble* __restrict__ src, double* dst, double sgn) {
        const int nxm = nx[mu];
        const gdouble* T = to_global(P.T[mu]);
        const int64_t n = P.n[mu];
        for (int e = tid; e < sz[mu] * nxm; e += NT) {
            const int i = e / nxm, j = e - (e / nxm) * nxm;
            U[i * g.top + j] = T[(int64_t)(r0[mu] + i) * n + r0[mu] + sz[mu] + j];
        }
        __syncthreads();
        const int F = cap / sz[mu];
        const int64_t nstep = (int64_t)sz[mu] * gs[mu];
        for (int f = tid; f < F; f += NT) {
            int eb;
            int64_t gb;
            fibre(mu, f, eb, gb);
            for (int jc = 0; jc < nxm; jc += 16) {
                double xn[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const bool v = jc + j < nxm;
                    const double x = src[gb + nstep + (int64_t)(v ? jc + j : jc) * gs[mu]];
                    xn[j] = v ? x : 0.0;
                }
                for (int i = 0; i < sz[mu]; ++i) {
                    const double* ti = U + i * g.top + jc;
                    double a = 0.0;
#pragma unroll
                    for (int j = 0; j < 16; ++j)
                        if (jc + j < nxm) a = fma(ti[j], xn[j], a);
                    dst[eb + i * ls[mu]] += sgn * a;
                }
            }
        }
        __syncthreads();
    };
    // buf = buf x_mu T_mu[I_mu, I_mu] in place, one fibre per thread
    auto diag_product = [&](int mu, double* buf) {
        const int F = cap / sz[mu];
        const double* Tm = Td + mu * g.bm * tp;
        for (int f = tid; f < F; f += NT) {
            int eb;
            int64_t gb;
            fibre(mu, f, eb, gb);
            double v[kFib];
#pragma unroll
            for (int j = 0; j < kFib; ++j) v[j] = (j < sz[mu]) ? buf[eb + j * ls[mu]] : 0.0;
            for (int i = 0; i < sz[mu]; ++i) {
                double a = 0.0;
#pragma unroll
                for (int j = 0; j < kFib; ++j)
                    if (j < sz[mu]) a = fma(Tm[i * tp + j], v[j], a);
                buf[eb + i * ls[mu]] = a;
            }
        }
        __syncthreads();
    };

    // ---- 1. right-hand side, diagonal blocks, V_1
    gdouble* __restrict__ X = to_global(P.X);
    {
        const gdouble* __restrict__ rhs = (L.flags & 1) ? X : to_global(P.B);
        const gdouble* __restrict__ V1 = to_global(P.A[1]);
        const bool hv = (L.flags >> 1) & 1;
        for (int e = tid; e < cap; e += NT) {
            const int64_t o = gbase + goff(e);
            Xs[e] = rhs[o];
            Zs[e] = hv ? V1[o] : 0.0;
        }
    }
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const gdouble* T = to_global(P.T[mu]);
        const int64_t n = P.n[mu];
        for (int e = tid; e < sz[mu] * sz[mu]; e += NT) {
            const int i = e / sz[mu], j = e - (e / sz[mu]) * sz[mu];
            Td[mu * g.bm * tp + i * tp + j] = T[(int64_t)(r0[mu] + i) * n + r0[mu] + j];
        }
    }
    if (tid < 3) qcnt[tid] = 0;
    __syncthreads();

    // ---- adjacent blocks of modes 0 and 1: R -= T_0[I_0, I_0+1] x_0 X[next],
    // K_1 += A_1[I_1, I_1+1] x_1 X[next]
    if (nx[0]) adjacent(0, X, Xs, -1.0);  // uniform
    if (nx[1]) adjacent(1, X, Zs, 1.0);

    // ---- K chain: W_{k-1} := K_{k-1}, K_k = K_{k-1} x_k A_k[I_k, I_k] + V_k
    // + A_k[I_k, I_k+1] x_k W_{k-1}[next];  R -= K_{D-1}
#pragma unroll
    for (int k = 2; k < D; ++k) {
        gdouble* __restrict__ Wk = to_global(P.W[k - 1]);
        for (int e = tid; e < cap; e += NT) Wk[gbase + goff(e)] = Zs[e];
        __syncthreads();
        diag_product(k, Zs);
        if ((L.flags >> k) & 1) {
            const gdouble* __restrict__ Vk = to_global(P.A[k]);
            for (int e = tid; e < cap; e += NT) Zs[e] += Vk[gbase + goff(e)];
            __syncthreads();
        }
        if (nx[k]) adjacent(k, to_global(P.W[k - 1]), Zs, 1.0);
    }
    for (int e = tid; e < cap; e += NT) Xs[e] -= Zs[e];

    // ---- tuple structure per mode: bit p of tb[mu] set if tuple p is a 2x2 block
    uint32_t tb[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const double* Tm = Td + mu * g.bm * tp;
        uint32_t b = 0;
        int p = 0, i = 0;
        while (i < sz[mu]) {
            const bool two = i + 1 < sz[mu] && Tm[(i + 1) * tp + i] != 0.0;
            if (two) b |= 1u << p;
            i += two ? 2 : 1;
            ++p;
        }
        tb[mu] = b;
    }
    __syncthreads();  // R complete; Z_1 free

    // ---- 2. tuples hyperplane by hyperplane
    constexpr int kBits = (D == 4) ? kTupBits4 : kTupBits3;
    const LeafShape sh = shapes[L.shape];
    bool ok = true;
    auto decode = [&](uint32_t en, int (&a)[D], int (&w)[D]) {
        int ne = 1;
#pragma unroll
        for (int mu = 0; mu < D; ++mu) {
            const int p = (en >> (kBits * mu)) & ((1 << kBits) - 1);
            a[mu] = p + __popc(tb[mu] & ((1u << p) - 1u));
            w[mu] = 1 + ((tb[mu] >> p) & 1);
            ne *= w[mu];
        }
        return ne;
    };
    auto tdiag = [&](int mu, int i, int j) { return Td[mu * g.bm * tp + i * tp + j]; };
    // sum past the tuple (rows from..sz-1) of row c of mode mu's diagonal
    // block against X (mu = 0, 1) or Z_{mu-1}, at element e
    auto past = [&](int mu, int c, int from, int e) {
        const double* row = Td + mu * g.bm * tp + c * tp;
        const double* src = (mu <= 1) ? Xs : Zs + (mu - 2) * cap;
        return ldot(row, src + e, c, from, sz[mu], ls[mu]);
    };

    // coupled tuple of 8 or 16 unknowns, sixteen lanes together (lane u of
    // the group owns unknown u and row u of the tuple's system; rows past ne
    // are identity rows): sums past the tuple per lane, the q chain through
    // lane shuffles, Gaussian elimination with partial pivoting across the
    // lanes (pivot search by a butterfly, row exchange and the pivot row by
    // shuffles), back-substitution, then X and the Z chain
    auto coupled16 = [&](const int (&a)[D], const int (&w)[D], int ne, int u) {
        int bit[D];
        {
            int b = 0;
#pragma unroll
            for (int mu = D - 1; mu >= 0; --mu) {
                bit[mu] = (w[mu] == 2) ? b : -1;
                if (w[mu] == 2) ++b;
            }
        }
        auto coord = [&](int v, int mu) { return a[mu] + ((bit[mu] >= 0) ? ((v >> bit[mu]) & 1) : 0); };
        const bool act = u < ne;
        int cu[D], e = 0;
#pragma unroll
        for (int mu = 0; mu < D; ++mu) {
            cu[mu] = coord(u, mu);
            e += cu[mu] * ls[mu];
        }
        double S[D];
#pragma unroll
        for (int mu = 0; mu < D; ++mu) S[mu] = act ? past(mu, cu[mu], a[mu] + w[mu], e) : 0.0;
        double r = act ? Xs[e] - S[0] : 0.0;
        // partner of u along mode k (itself for a 1x1 mode)
        auto partner = [&](int k) { return (bit[k] >= 0) ? (u ^ (1 << bit[k])) : u; };
        // one step of the chain: A_k,tuple applied to v (held one per lane) plus add
        auto chain = [&](int k, double v, double add) {
            const int pu = partner(k);
            const double vp = __shfl(v, pu, 16);
            double s = fma(tdiag(k, cu[k], cu[k]), v, add);
            if (bit[k] >= 0) s = fma(tdiag(k, cu[k], coord(pu, k)), vp, s);
            return act ? s : 0.0;
        };
        double q = S[1];
#pragma unroll
        for (int k = 2; k < D; ++k) q = chain(k, q, S[k]);
        r -= q;
        // row u of M = T_0,tuple (x) I + I (x) (A_1 (x) .. (x) A_{D-1})_tuple
        double Mr[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            double m = (u == v) ? 1.0 : 0.0;
            if (act && v < ne) {
                bool rest = true;
#pragma unroll
                for (int k = 1; k < D; ++k) rest = rest && cu[k] == coord(v, k);
                m = rest ? tdiag(0, cu[0], coord(v, 0)) : 0.0;
                if (cu[0] == coord(v, 0)) {
                    double pr = 1.0;
#pragma unroll
                    for (int k = 1; k < D; ++k) pr *= tdiag(k, cu[k], coord(v, k));
                    m += pr;
                }
            }
            Mr[v] = m;
        }
        bool good = true;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            // pivot: the largest |M[i][k]| over rows i >= k (ties: lower row)
            double key = (u >= k) ? fabs(Mr[k]) : -1.0;
            int idx = u;
#pragma unroll
            for (int m = 8; m >= 1; m >>= 1) {
                const double ok2 = __shfl_xor(key, m, 16);
                const int oi = __shfl_xor(idx, m, 16);
                if (ok2 > key || (ok2 == key && oi < idx)) {
                    key = ok2;
                    idx = oi;
                }
            }
            if (!(key > 0.0)) good = false;
            const int pv = idx;
            // exchange rows k and pv
            const int src = (u == k) ? pv : ((u == pv) ? k : u);
#pragma unroll
            for (int j = k; j < 16; ++j) Mr[j] = __shfl(Mr[j], src, 16);
            r = __shfl(r, src, 16);
            // eliminate below the pivot with row k
            const double pk = __shfl(Mr[k], k, 16), rk = __shfl(r, k, 16);
            const double f = (u > k) ? Mr[k] / pk : 0.0;
#pragma unroll
            for (int j = k + 1; j < 16; ++j) Mr[j] = fma(-f, __shfl(Mr[j], k, 16), Mr[j]);
            r = fma(-f, rk, r);
        }
        // back-substitution: x_k from lane k, broadcast to the group
        double x = 0.0, xs[16];
#pragma unroll
        for (int k = 15; k >= 0; --k) {
            double acc = r;
#pragma unroll
            for (int j = k + 1; j < 16; ++j) acc = fma(-Mr[j], xs[j], acc);
            const double xk = acc / Mr[k];
            xs[k] = __shfl(xk, k, 16);
            if (u == k) x = xk;
        }
        if (act && !isfinite(x)) good = false;
        if (act) Xs[e] = x;
        double z = x;
#pragma unroll
        for (int k = 1; k <= D - 2; ++k) {
            z = chain(k, z, S[k]);
            if (act) Zs[(k - 1) * cap + e] = z;
        }
        return good;
    };

    // coupled tuple of 2 or 4 unknowns in registers; Sk[u * D + mu] holds
    // the sum past the tuple of unknown u along mode mu
    double* Sb = U;
    auto coupled_reg = [&](const int (&a)[D], const int (&w)[D], int ne, const double* Sk) {
        // bit of each width-2 mode in the local unknown index (the last such
        // mode owns bit 0): at most two such modes here
        int bit[D];
        {
            int b = 0;
#pragma unroll
            for (int mu = D - 1; mu >= 0; --mu) {
                bit[mu] = (w[mu] == 2) ? b : -1;
                if (w[mu] == 2) ++b;
            }
        }
        int cu[4][D], e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            e[u] = 0;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) {
                cu[u][mu] = a[mu] + ((bit[mu] >= 0) ? ((u >> bit[mu]) & 1) : 0);
                e[u] += cu[u][mu] * ls[mu];
            }
        }
        double r[4], q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            r[u] = (u < ne) ? Xs[e[u]] - Sk[u * D] : 0.0;
            q[u] = (u < ne) ? Sk[u * D + 1] : 0.0;
        }
        // partner of u along mode k: u ^ 1 or u ^ 2 (static indices)
        auto step = [&](int k, const double (&src)[4], double (&dst)[4]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double v1 = src[u ^ 1], v2 = src[u ^ 2];
                double s = fma(tdiag(k, cu[u][k], cu[u][k]), src[u], (u < ne) ? Sk[u * D + k] : 0.0);
                if (bit[k] >= 0) {
                    const int pu = (bit[k] == 0) ? (u ^ 1) : (u ^ 2);
                    s = fma(tdiag(k, cu[u][k], cu[pu & 3][k]), (bit[k] == 0) ? v1 : v2, s);
                }
                dst[u] = (u < ne) ? s : 0.0;
            }
        };
#pragma unroll
        for (int k = 2; k < D; ++k) {
            double q2[4];
            step(k, q, q2);
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = q2[u];
        }
        double M[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            r[u] -= q[u];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                bool rest = true;
#pragma unroll
                for (int k = 1; k < D; ++k) rest = rest && cu[u][k] == cu[v][k];
                double m = rest ? tdiag(0, cu[u][0], cu[v][0]) : 0.0;
                if (cu[u][0] == cu[v][0]) {
                    double pr = 1.0;
#pragma unroll
                    for (int k = 1; k < D; ++k) pr *= tdiag(k, cu[u][k], cu[v][k]);
                    m += pr;
                }
                M[u][v] = (u < ne && v < ne) ? m : ((u == v) ? 1.0 : 0.0);
            }
        }
        const bool good = gepp4(M, r);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (u < ne) Xs[e[u]] = r[u];
        double prev[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) prev[u] = r[u];
#pragma unroll
        for (int k = 1; k <= D - 2; ++k) {
            double cur[4];
            step(k, prev, cur);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u < ne) Zs[(k - 1) * cap + e[u]] = cur[u];
                prev[u] = cur[u];
            }
        }
        return good;
    };

    for (int h = 0; h < sh.H; ++h) {
        const int tb0 = hoffs[sh.hoff + h], tb1 = hoffs[sh.hoff + h + 1];
        uint32_t* cnt = qcnt + h % 3;
        // the counter of hyperplane h + 1 was last read in step h - 2
        if (tid == 0) qcnt[(h + 1) % 3] = 0;
        for (int t = tb0 + tid; t < tb1; t += NT) {
            const uint32_t en = ents[sh.ent + t];
            int a[D], w[D];
            if (decode(en, a, w) > 1) {
                qlist[atomicAdd(cnt, 1u)] = en;
                continue;
            }
            int e = 0;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) e += a[mu] * ls[mu];
            const double s0 = past(0, a[0], a[0] + 1, e);
            double S[D];
#pragma unroll
            for (int k = 1; k < D; ++k) S[k] = past(k, a[k], a[k] + 1, e);
            double dk[D];
#pragma unroll
            for (int mu = 0; mu < D; ++mu) dk[mu] = tdiag(mu, a[mu], a[mu]);
            double p = dk[1], q = S[1];
#pragma unroll
            for (int k = 2; k < D; ++k) {
                p *= dk[k];
                q = fma(q, dk[k], S[k]);
            }
            const double den = dk[0] + p;
            const double x = (Xs[e] - s0 - q) / den;
            if (den == 0.0 || !isfinite(x)) ok = false;
            Xs[e] = x;
            double z = x;
#pragma unroll
            for (int k = 1; k <= D - 2; ++k) {
                z = fma(dk[k], z, S[k]);
                Zs[(k - 1) * cap + e] = z;
            }
        }
        __syncthreads();
        const int nc = (int)*cnt;  // uniform
        if (nc > 0) {
            // tuples of 2 or 4 unknowns, CH at a time: (1) every sum past a
            // tuple (unknown u, mode mu) by its own thread, (2) one thread
            // per tuple forms and solves its system in registers
            for (int c0 = 0; c0 < nc; c0 += Tup::CH) {
                const int ch = min(Tup::CH, nc - c0);
                for (int i = tid; i < ch * 4 * D; i += NT) {
                    const int k = i / (4 * D), u = (i / D) & 3, mu = i - (i / D) * D;
                    int a[D], w[D];
                    const int ne = decode(qlist[c0 + k], a, w);
                    if (ne > 4 || u >= ne) continue;
                    int e = 0, cm = 0, b = 0;
#pragma unroll
                    for (int nu = D - 1; nu >= 0; --nu) {
                        int c = a[nu];
                        if (w[nu] == 2) c += (u >> b++) & 1;
                        e += c * ls[nu];
                        if (nu == mu) cm = c;
                    }
                    Sb[i] = past(mu, cm, a[mu] + w[mu], e);
                }
                __syncthreads();
                for (int k = tid; k < ch; k += NT) {
                    int a[D], w[D];
                    const int ne = decode(qlist[c0 + k], a, w);
                    if (ne <= 4 && !coupled_reg(a, w, ne, Sb + k * 4 * D)) ok = false;
                }
                __syncthreads();
            }
            // tuples of 8 or 16 unknowns (2x2 blocks in three or more modes):
            // sixteen lanes per tuple, the groups of the workgroup in turn
            {
                constexpr int G = NT / 16;
                const int grp = tid / 16, u = tid % 16;
                int j = 0;
                for (int k = 0; k < nc; ++k) {
                    int a[D], w[D];
                    const int ne = decode(qlist[k], a, w);
                    if (ne <= 4) continue;
                    if (j++ % G == grp && !coupled16(a, w, ne, u)) ok = false;  // uniform in the group
                }
            }
            __syncthreads();
        }
    }
    if (!ok) atomicOr(status, 1);

    // ---- 3. store X; W_k += Z_k (W_k holds K_k, written above by this thread)
    for (int e = tid; e < cap; e += NT) {
        const int64_t o = gbase + goff(e);
        X[o] = Xs[e];
#pragma unroll
        for (int k = 1; k <= D - 2; ++k) {
            gdouble* Wk = to_global(P.W[k]);
            Wk[o] += Zs[(k - 1) * cap + e];
        }
    }
}

int leaf2_lds_bytes(int D, const int* bmax) { return (int)(l2_geometry(D, bmax).total * sizeof(double)); }

hipError_t launch_leaf2(int D, const LeafDesc* leaves, int64_t first, int64_t count, const ProbDesc* probs,
                        const LeafShape* shapes, const uint16_t* ents, const int32_t* hoffs, int* status,
                        const int* bmax, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const L2Geom g = l2_geometry(D, bmax);
    const int lds = (int)(g.total * sizeof(double));
    const bool small = g.cap <= kL2Small;
    const void* fn = (D == 3) ? (small ? (const void*)leaf2_kernel<3, 64> : (const void*)leaf2_kernel<3, kL2NT>)
                              : (small ? (const void*)leaf2_kernel<4, 64> : (const void*)leaf2_kernel<4, kL2NT>);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)count), block(small ? 64 : kL2NT);
    if (D == 3 && small)
        hipLaunchKernelGGL((leaf2_kernel<3, 64>), grid, block, lds, st, leaves, first, probs, shapes, ents, hoffs,
                           status, g);
    else if (D == 3)
        hipLaunchKernelGGL((leaf2_kernel<3, kL2NT>), grid, block, lds, st, leaves, first, probs, shapes, ents, hoffs,
                           status, g);
    else if (small)
        hipLaunchKernelGGL((leaf2_kernel<4, 64>), grid, block, lds, st, leaves, first, probs, shapes, ents, hoffs,
                           status, g);
    else
        hipLaunchKernelGGL((leaf2_kernel<4, kL2NT>), grid, block, lds, st, leaves, first, probs, shapes, ents, hoffs,
                           status, g);
    return hipGetLastError();
}

}  // namespace tt
