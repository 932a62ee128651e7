// Leaf solve of the second operator class (Sec. 3, gfx950).
//
// After the exact reduction by C^{-1} (Sec. 3 below) the equation reads
//   X x_0 T_0 + X x_1 A_1 x_2 A_2 .. x_{D-1} A_{D-1} = B
// (internal modes 0..D-1; T_0 = C^{-1} A_1 of the paper and A_1 .. A_{D-1}
// its A_2 .. A_d, all upper quasi-triangular).  Element i depends on the
// elements that are larger in mode 0 alone (T_0) and on every element of the
// orthant j_nu >= i_nu, nu >= 1, at the same i_0 (the product term).  The
// block schedule is the Laplace-like one; what reaches a leaf block I from
// outside is
//   * mode 0: T_0[I_0, J_0] x_0 X[J_0, I']            (already in X, as for
//     the Laplace-like form, plus the adjacent block applied here);
//   * the product term over the orthant, which telescopes through the
//     partial products W_k (k = 1 .. D-2) and the accumulators V_nu of the
//     updates along mode nu (V_nu = sum over J_nu > I_nu of
//     A_nu[I_nu, J_nu] x_nu W_{nu-1}[.., J_nu, ..], W_0 = X):
//        W_k[I] = W_{k-1}[I] x_k A_k[I_k, I_k] + V_k[I],
//     so the product term of I is W_{D-1}[I] = P(X[I]) + K with
//        P(X[I]) = X[I] x_1 A_1[I_1,I_1] .. x_{D-1} A_{D-1}[I_{D-1},I_{D-1}],
//        K = (..(V_1 x_2 A_2[I_2,I_2] + V_2) x_3 .. ) + V_{D-1}.
// The leaf (one 64-lane wave per block) subtracts K, solves the block's own
// equation X x_0 T_0[I_0,I_0] + P(X) = R by block back-substitution over the
// tuples of the diagonal blocks' 1x1 / 2x2 blocks (one lane per tuple of a
// hyperplane; coupled tuples by Gaussian elimination with partial pivoting
// in LDS), and writes X and W_1 .. W_{D-2}.
#include "tt_internal.h"

namespace tt {

namespace {

constexpr int kL2NT = 64;        // one wave per leaf block
constexpr int kL2Slot = 72;      // LDS doubles of a lane's elimination scratch (8 unknowns)
constexpr int kL2Big = 272;      // the same for a 16-unknown tuple (order 4), lane 0 only

// LDS carving (doubles) for the largest block of a launch.
struct L2Geom {
    int cap;          // prod bmax
    int bm;           // max bmax
    int oX, oV, oK, oN, oTd, oTo, oSc, oBig, total;
};

__host__ __device__ inline L2Geom l2_geometry(int D, const int* bmax) {
    L2Geom g{};
    g.cap = 1;
    g.bm = 1;
    for (int mu = 0; mu < D; ++mu) {
        g.cap *= bmax[mu];
        g.bm = bmax[mu] > g.bm ? bmax[mu] : g.bm;
    }
    g.oX = 0;
    g.oV = g.oX + g.cap;                  // V_1 .. V_{D-1}
    g.oK = g.oV + (D - 1) * g.cap;        // scratch tensor (K, partial products)
    g.oN = g.oK + g.cap;                  // adjacent block of a source tensor
    g.oTd = g.oN + g.cap;                 // diagonal blocks T_mu[I_mu, I_mu]
    g.oTo = g.oTd + D * g.bm * g.bm;      // one off-diagonal block T_mu[I_mu, I_mu + 1]
    g.oSc = g.oTo + g.bm * g.bm;          // per-lane elimination scratch
    g.oBig = g.oSc + kL2NT * kL2Slot;
    g.total = g.oBig + (D == 4 ? kL2Big : 0);
    return g;
}

// dst (+)= src x_nu M over a block with extents ext (row-major, last mode
// fastest): dst[.., r, ..] (+)= sum_{j < cols} M[r * ldm + j] src[.., j, ..],
// where src has extent `cols` in mode nu and dst extent `rows`.  All lanes.
template <int D>
__device__ inline void lds_modeprod(double* dst, const double* src, const double* M, int ldm, int nu,
                                    const int (&ext)[4], int rows, int cols, bool acc, int tid) {
    int inner = 1, outer = 1;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        if (mu > nu) inner *= ext[mu];
        if (mu < nu) outer *= ext[mu];
    }
    const int total = outer * rows * inner;
    for (int e = tid; e < total; e += kL2NT) {
        const int q = e % inner, r = (e / inner) % rows, o = e / (inner * rows);
        double s = 0.0;
        for (int j = 0; j < cols; ++j) s = fma(M[r * ldm + j], src[(o * cols + j) * inner + q], s);
        const int di = (o * rows + r) * inner + q;
        dst[di] = acc ? dst[di] + s : s;
    }
}

// Gaussian elimination with partial pivoting on an s x s system held in LDS
// (row-major M, right-hand side r); false on a zero pivot or a non-finite
// result.
__device__ inline bool lds_gepp(int s, double* M, double* r) {
    bool ok = true;
    for (int k = 0; k < s; ++k) {
        int piv = k;
        double best = fabs(M[k * s + k]);
        for (int i = k + 1; i < s; ++i)
            if (fabs(M[i * s + k]) > best) {
                best = fabs(M[i * s + k]);
                piv = i;
            }
        if (best == 0.0) ok = false;
        if (piv != k) {
            for (int j = 0; j < s; ++j) {
                const double t = M[k * s + j];
                M[k * s + j] = M[piv * s + j];
                M[piv * s + j] = t;
            }
            const double t = r[k];
            r[k] = r[piv];
            r[piv] = t;
        }
        const double rp = 1.0 / M[k * s + k];
        for (int i = k + 1; i < s; ++i) {
            const double f = M[i * s + k] * rp;
            for (int j = k + 1; j < s; ++j) M[i * s + j] = fma(-f, M[k * s + j], M[i * s + j]);
            r[i] = fma(-f, r[k], r[i]);
        }
    }
    for (int k = s - 1; k >= 0; --k) {
        double acc = r[k];
        for (int j = k + 1; j < s; ++j) acc = fma(-M[k * s + j], r[j], acc);
        r[k] = acc / M[k * s + k];
        if (!isfinite(r[k])) ok = false;
    }
    return ok;
}

}  // namespace

template <int D>
__global__ __launch_bounds__(kL2NT) void leaf2_kernel(const LeafDesc* __restrict__ leaves, int64_t first,
                                                      const ProbDesc* __restrict__ probs,
                                                      const LeafShape* __restrict__ shapes,
                                                      const uint16_t* __restrict__ ents,
                                                      const int32_t* __restrict__ hoffs, int* status, L2Geom g) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const LeafDesc L = leaves[first + blockIdx.x];
    const ProbDesc& P = probs[L.prob];
    double* Xs = lds + g.oX;
    double* Ks = lds + g.oK;
    double* Nb = lds + g.oN;
    double* To = lds + g.oTo;
    const int bm = g.bm;

    int r0[4] = {0, 0, 0, 0}, sz[4] = {1, 1, 1, 1}, nx[4] = {0, 0, 0, 0};
    int64_t gs[4] = {0, 0, 0, 0};
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const int b = L.blk[mu];
        const auto* bst = to_global(P.bst[mu]);
        r0[mu] = bst[b];
        const int r1 = bst[b + 1];
        sz[mu] = r1 - r0[mu];
        nx[mu] = ((L.flags >> (4 + mu)) & 1) ? bst[b + 2] - r1 : 0;
        gs[mu] = P.stride[mu];
    }
    int cap = 1;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) cap *= sz[mu];
    int64_t gbase = 0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) gbase += (int64_t)r0[mu] * gs[mu];
    // local element e (row-major over sz) -> global offset from gbase
    auto goff = [&](int e, const int (&ext)[4]) {
        int64_t o = 0;
#pragma unroll
        for (int mu = D - 1; mu >= 0; --mu) {
            o += (int64_t)(e % ext[mu]) * gs[mu];
            e /= ext[mu];
        }
        return o;
    };

    // ---- right-hand side, accumulators, diagonal blocks
    gdouble* __restrict__ X = to_global(P.X);
    const gdouble* __restrict__ rhs = (L.flags & 1) ? X : to_global(P.B);
    for (int e = tid; e < cap; e += kL2NT) {
        const int64_t o = gbase + goff(e, sz);
        Xs[e] = rhs[o];
#pragma unroll
        for (int nu = 1; nu < D; ++nu)
            lds[g.oV + (nu - 1) * g.cap + e] = ((L.flags >> nu) & 1) ? to_global(P.A[nu])[o] : 0.0;
    }
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const gdouble* T = to_global(P.T[mu]);
        const int64_t n = P.n[mu];
        for (int e = tid; e < sz[mu] * sz[mu]; e += kL2NT) {
            const int i = e / sz[mu], j = e % sz[mu];
            lds[g.oTd + mu * bm * bm + i * bm + j] = T[(int64_t)(r0[mu] + i) * n + r0[mu] + j];
        }
    }
    __syncthreads();

    // ---- the adjacent block along each mode: mode 0 subtracts
    // T_0[I_0, I_0+1] x_0 X[next]; mode nu >= 1 adds A_nu[I_nu, I_nu+1] x_nu
    // S_nu[next] to V_nu (S_1 = X, S_nu = W_{nu-1})
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const int nxm = nx[mu];
        if (nxm == 0) continue;  // uniform
        const gdouble* T = to_global(P.T[mu]);
        const int64_t n = P.n[mu];
        const gdouble* S = to_global(P.S[mu]);
        int ext[4] = {sz[0], sz[1], sz[2], sz[3]};
        ext[mu] = nxm;
        int ncap = 1;
#pragma unroll
        for (int nu = 0; nu < D; ++nu) ncap *= ext[nu];
        const int64_t nbase = gbase + (int64_t)sz[mu] * gs[mu];
        for (int e = tid; e < ncap; e += kL2NT) Nb[e] = S[nbase + goff(e, ext)];
        for (int e = tid; e < sz[mu] * nxm; e += kL2NT) {
            const int i = e / nxm, j = e % nxm;
            To[i * bm + j] = T[(int64_t)(r0[mu] + i) * n + r0[mu] + sz[mu] + j];
        }
        __syncthreads();
        if (mu == 0) {
            // Ks = T_0[I_0, I_0+1] x_0 X[next], then Xs -= Ks
            lds_modeprod<D>(Ks, Nb, To, bm, 0, ext, sz[0], nxm, false, tid);
            __syncthreads();
            for (int e = tid; e < cap; e += kL2NT) Xs[e] -= Ks[e];
        } else {
            lds_modeprod<D>(lds + g.oV + (mu - 1) * g.cap, Nb, To, bm, mu, ext, sz[mu], nxm, true, tid);
        }
        __syncthreads();
    }

    // ---- K = (..(V_1 x_2 A_2 + V_2) x_3 A_3 ..) + V_{D-1}, R = Xs - K
    {
        // Ks <- V_1, then Ks <- Ks x_nu A_nu + V_nu (through Nb)
        for (int e = tid; e < cap; e += kL2NT) Ks[e] = lds[g.oV + e];
        __syncthreads();
#pragma unroll
        for (int nu = 2; nu < D; ++nu) {
            lds_modeprod<D>(Nb, Ks, lds + g.oTd + nu * bm * bm, bm, nu, sz, sz[nu], sz[nu], false, tid);
            __syncthreads();
            for (int e = tid; e < cap; e += kL2NT) Ks[e] = Nb[e] + lds[g.oV + (nu - 1) * g.cap + e];
            __syncthreads();
        }
        for (int e = tid; e < cap; e += kL2NT) Xs[e] -= Ks[e];
    }

    // ---- tuple structure per mode: bit p of tb[mu] set if tuple p is a 2x2 block
    uint32_t tb[4] = {0, 0, 0, 0};
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const double* Td = lds + g.oTd + mu * bm * bm;
        int p = 0, i = 0;
        while (i < sz[mu]) {
            const bool two = i + 1 < sz[mu] && Td[(i + 1) * bm + i] != 0.0;
            if (two) tb[mu] |= 1u << p;
            i += two ? 2 : 1;
            ++p;
        }
    }
    int ls[4];
    ls[D - 1] = 1;
#pragma unroll
    for (int mu = D - 2; mu >= 0; --mu) ls[mu] = ls[mu + 1] * sz[mu + 1];
    __syncthreads();

    // ---- block back-substitution, one tuple hyperplane per step (one lane
    // per tuple; tuples of 16 unknowns by lane 0 after the others)
    constexpr int kBits = (D == 4) ? kTupBits4 : kTupBits3;
    const LeafShape sh = shapes[L.shape];
    const double* Td0 = lds + g.oTd;
    bool ok = true;
    // right-hand side of element (c) of a tuple starting at a with widths w,
    // and the tuple's system; sc: M (ne x ne) then r (ne)
    auto tuple_solve = [&](const int (&a)[4], const int (&w)[4], double* sc) {
        int ne = 1;
#pragma unroll
        for (int mu = 0; mu < D; ++mu) ne *= w[mu];
        double* M = sc;
        double* r = sc + ne * ne;
        for (int e = 0; e < ne; ++e) {
            int c[4] = {0, 0, 0, 0}, rem = e;
#pragma unroll
            for (int mu = D - 1; mu >= 0; --mu) {
                c[mu] = a[mu] + rem % w[mu];
                rem /= w[mu];
            }
            int le = 0;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) le += c[mu] * ls[mu];
            double acc = Xs[le];
            // mode 0: rows past the tuple's mode-0 rows
            for (int j = a[0] + w[0]; j < sz[0]; ++j) acc -= Td0[c[0] * bm + j] * Xs[le + (j - c[0]) * ls[0]];
            // product term over the orthant j' >= a' (modes >= 1) outside the
            // tuple's rows, at the same i_0
            int ext[4] = {1, 1, 1, 1}, span = 1;
#pragma unroll
            for (int mu = 1; mu < D; ++mu) {
                ext[mu] = sz[mu] - a[mu];
                span *= ext[mu];
            }
            for (int t = 0; t < span; ++t) {
                int j[4] = {0, 0, 0, 0}, rt = t;
                bool inside = true;
#pragma unroll
                for (int mu = D - 1; mu >= 1; --mu) {
                    j[mu] = a[mu] + rt % ext[mu];
                    rt /= ext[mu];
                    if (j[mu] >= a[mu] + w[mu]) inside = false;
                }
                if (inside) continue;
                double pr = 1.0;
                int lj = c[0] * ls[0];
#pragma unroll
                for (int mu = 1; mu < D; ++mu) {
                    pr *= lds[g.oTd + mu * bm * bm + c[mu] * bm + j[mu]];
                    lj += j[mu] * ls[mu];
                }
                acc -= pr * Xs[lj];
            }
            r[e] = acc;
            // row e of the tuple's system
            for (int f = 0; f < ne; ++f) {
                int cf[4] = {0, 0, 0, 0}, rf = f;
#pragma unroll
                for (int mu = D - 1; mu >= 0; --mu) {
                    cf[mu] = a[mu] + rf % w[mu];
                    rf /= w[mu];
                }
                bool same = true;
#pragma unroll
                for (int mu = 1; mu < D; ++mu) same = same && (c[mu] == cf[mu]);
                double m = same ? Td0[c[0] * bm + cf[0]] : 0.0;
                double pr = (c[0] == cf[0]) ? 1.0 : 0.0;
#pragma unroll
                for (int mu = 1; mu < D; ++mu) pr *= lds[g.oTd + mu * bm * bm + c[mu] * bm + cf[mu]];
                M[e * ne + f] = m + pr;
            }
        }
        const bool good = lds_gepp(ne, M, r);
        for (int e = 0; e < ne; ++e) {
            int rem = e, le = 0;
#pragma unroll
            for (int mu = D - 1; mu >= 0; --mu) {
                le += (a[mu] + rem % w[mu]) * ls[mu];
                rem /= w[mu];
            }
            Xs[le] = r[e];
        }
        return good;
    };
    auto decode = [&](uint32_t en, int (&a)[4], int (&w)[4]) {
        int ne = 1;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            a[mu] = 0;
            w[mu] = 1;
        }
#pragma unroll
        for (int mu = 0; mu < D; ++mu) {
            const int p = (en >> (kBits * mu)) & ((1 << kBits) - 1);
            a[mu] = p + __popc(tb[mu] & ((1u << p) - 1u));
            w[mu] = 1 + ((tb[mu] >> p) & 1);
            ne *= w[mu];
        }
        return ne;
    };
    double* slot = lds + g.oSc + tid * kL2Slot;
    for (int h = 0; h < sh.H; ++h) {
        const int tb0 = hoffs[sh.hoff + h], tb1 = hoffs[sh.hoff + h + 1];
        for (int t = tb0 + tid; t < tb1; t += kL2NT) {
            int a[4], w[4];
            const int ne = decode(ents[sh.ent + t], a, w);
            if (ne <= 8 && !tuple_solve(a, w, slot)) ok = false;
        }
        if constexpr (D == 4) {
            __syncthreads();
            if (tid == 0)
                for (int t = tb0; t < tb1; ++t) {
                    int a[4], w[4];
                    if (decode(ents[sh.ent + t], a, w) == 16 && !tuple_solve(a, w, lds + g.oBig)) ok = false;
                }
        }
        __syncthreads();
    }
    if (!ok) atomicOr(status, 1);

    // ---- partial products W_k = W_{k-1} x_k A_k[I_k, I_k] + V_k (W_0 = X),
    // k = 1 .. D-2, for the updates along modes k+1
    if constexpr (D >= 3) {
        const double* src = Xs;
#pragma unroll
        for (int k = 1; k <= D - 2; ++k) {
            double* dst = (k % 2 == 1) ? Ks : Nb;
            lds_modeprod<D>(dst, src, lds + g.oTd + k * bm * bm, bm, k, sz, sz[k], sz[k], false, tid);
            __syncthreads();
            gdouble* Wg = to_global(P.W[k]);
            for (int e = tid; e < cap; e += kL2NT) {
                const double v = dst[e] + lds[g.oV + (k - 1) * g.cap + e];
                dst[e] = v;
                Wg[gbase + goff(e, sz)] = v;
            }
            __syncthreads();
            src = dst;
        }
    }

    // ---- store the solved block
    for (int e = tid; e < cap; e += kL2NT) X[gbase + goff(e, sz)] = Xs[e];
}

int leaf2_lds_bytes(int D, const int* bmax) {
    return (int)(l2_geometry(D, bmax).total * sizeof(double));
}

hipError_t launch_leaf2(int D, const LeafDesc* leaves, int64_t first, int64_t count, const ProbDesc* probs,
                        const LeafShape* shapes, const uint16_t* ents, const int32_t* hoffs, int* status,
                        const int* bmax, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const L2Geom g = l2_geometry(D, bmax);
    const int lds = (int)(g.total * sizeof(double));
    const void* fn = (D == 3) ? (const void*)leaf2_kernel<3> : (const void*)leaf2_kernel<4>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    if (D == 3)
        hipLaunchKernelGGL(leaf2_kernel<3>, dim3((unsigned)count), dim3(kL2NT), lds, st, leaves, first, probs, shapes,
                           ents, hoffs, status, g);
    else
        hipLaunchKernelGGL(leaf2_kernel<4>, dim3((unsigned)count), dim3(kL2NT), lds, st, leaves, first, probs, shapes,
                           ents, hoffs, status, g);
    return hipGetLastError();
}

}  // namespace tt
