// gfx950 kernels of the triangular Kronecker solve.
//
//   leaf_kernel   - solves one leaf block of the recursion (the "solve full
//                   system" base case of Algorithm 2, Sec. 2.1) in LDS by
//                   block back-substitution over its 1x1 / 2x2 diagonal
//                   blocks, hyperplane by hyperplane.
//   upd_kernel    - the right-hand-side update of Algorithm 2,
//                   B_1 <- B_1 - X_2 x_mu A_mu(1:k, k+1:n_mu), for one pencil,
//                   on FP64 MFMA (v_mfma_f64_16x16x4f64).
#include "tt_internal.h"

namespace tt {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Small dense solve (Gaussian elimination with partial pivoting), all indices
// static so that the system stays in registers.  Returns false on a zero
// pivot or a non-finite result.
// ---------------------------------------------------------------------------
template <int NE>
__device__ inline bool gepp_small(double (&M)[NE][NE], double (&r)[NE], int ne) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        if (k < ne) {
#pragma unroll
            for (int i = k + 1; i < NE; ++i) {
                if (i < ne && fabs(M[i][k]) > fabs(M[k][k])) {
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
            double piv = M[k][k];
            if (piv == 0.0) ok = false;
#pragma unroll
            for (int i = k + 1; i < NE; ++i) {
                if (i < ne) {
                    double f = M[i][k] / piv;
#pragma unroll
                    for (int j = 0; j < NE; ++j)
                        if (j >= k) M[i][j] -= f * M[k][j];
                    r[i] -= f * r[k];
                }
            }
        }
    }
#pragma unroll
    for (int k = NE - 1; k >= 0; --k) {
        if (k < ne) {
            double acc = r[k];
#pragma unroll
            for (int j = 0; j < NE; ++j)
                if (j > k && j < ne) acc -= M[k][j] * r[j];
            r[k] = acc / M[k][k];
            if (!isfinite(r[k])) ok = false;
        }
    }
    return ok;
}

// ---------------------------------------------------------------------------
// Leaf kernel.  One workgroup per leaf block.  LDS holds the block of X (the
// updated right-hand side on entry), the D diagonal blocks of T, and the
// partition of each mode of the block into 1x1 / 2x2 diagonal blocks.
// A tuple p of such diagonal blocks depends only on tuples q >= p; tuples on
// one hyperplane sum(p) = s are independent, so each hyperplane is one
// parallel step.  A tuple with w_mu in {1,2} per mode has ne = prod w_mu
// unknowns coupled by  sum_mu I (x) T_mu[p_mu, p_mu] (x) I:
//   ne = 1     -> one division by the eigenvalue sum (the common case),
//   ne = 2, 4  -> Gaussian elimination with partial pivoting in registers,
//   ne >= 8    -> (bumps in >= 3 modes at once, rare) queued and solved by a
//                 few threads with the system staged in LDS.
// ---------------------------------------------------------------------------
// Element index of local unknown q of a tuple.
template <int D>
__device__ inline int tuple_elem(const int* ls, const int* a, const int* w, int q) {
    int e = 0;
#pragma unroll
    for (int mu = D - 1; mu >= 0; --mu) {
        e += (a[mu] + q % w[mu]) * ls[mu];
        q /= w[mu];
    }
    return e;
}

// Coupling coefficient between local unknowns q and q2 of a tuple.
template <int D>
__device__ inline double tuple_coupling(double* const* Ts, const int* sz, const int* a, const int* w, int q,
                                        int q2) {
    int dq[D], dq2[D];
    int rq = q, rq2 = q2;
#pragma unroll
    for (int mu = D - 1; mu >= 0; --mu) {
        dq[mu] = rq % w[mu];
        rq /= w[mu];
        dq2[mu] = rq2 % w[mu];
        rq2 /= w[mu];
    }
    double m = 0.0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        bool same = true;
#pragma unroll
        for (int nu = 0; nu < D; ++nu)
            if (nu != mu && dq[nu] != dq2[nu]) same = false;
        if (same) m += Ts[mu][(a[mu] + dq[mu]) * sz[mu] + a[mu] + dq2[mu]];
    }
    return m;
}

constexpr int kAdjMax = 32;  // largest leaf block edge (checked by the planner)
constexpr int kBatch = 8;    // global loads a thread keeps in flight

// ---------------------------------------------------------------------------
// Small systems of one tuple.  A tuple of diagonal blocks with widths
// w_mu in {1, 2} couples its ne = prod w_mu unknowns by
//   M = sum_mu I (x) T_mu[p_mu, p_mu] (x) I.
// With k modes of width 2 (taken in increasing mode order, the last one
// owning bit 0 of the local index q) and c the sum of the 1x1 diagonal
// entries of the other modes, M = sum_j (I (x) D_j (x) I) + c I where D_j is
// the j-th 2x2 block.
// ---------------------------------------------------------------------------
template <int NE>
__device__ inline void tuple_matrix(double (&M)[NE][NE], const double (&Dm)[4][4], double c) {
    constexpr int K = (NE == 2) ? 1 : (NE == 4) ? 2 : 3;
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

// 8 unknowns (2x2 blocks in three modes): eliminate along the first block.
// With K the 4x4 operator of the other two modes and D_0 = [p q; r t]:
//   (K + pI) x0 + q x1 = b0,   r x0 + (K + tI) x1 = b1
//   =>  [(K + tI)(K + pI) - q r I] x0 = (K + tI) b0 - q b1,
//       (K + tI) x1 = b1 - r x0.
__device__ inline bool tuple_solve8(const double (&Dm)[4][4], double c, double (&b)[8]) {
    double Km[4][4];
    double D2[4][4] = {{Dm[1][0], Dm[1][1], Dm[1][2], Dm[1][3]}, {Dm[2][0], Dm[2][1], Dm[2][2], Dm[2][3]},
                       {0, 0, 0, 0}, {0, 0, 0, 0}};
    tuple_matrix<4>(Km, D2, c);
    const double p = Dm[0][0], q = Dm[0][1], r = Dm[0][2], t = Dm[0][3];
    double S[4][4], Q[4][4], rhs[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) S[i][j] = Km[i][j] + (i == j ? t : 0.0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double acc = (i == j) ? -q * r : 0.0;
#pragma unroll
            for (int l = 0; l < 4; ++l) acc += S[i][l] * (Km[l][j] + (l == j ? p : 0.0));
            Q[i][j] = acc;
        }
        double acc = -q * b[4 + i];
#pragma unroll
        for (int l = 0; l < 4; ++l) acc += S[i][l] * b[l];
        rhs[i] = acc;
    }
    bool ok = gepp_small<4>(Q, rhs, 4);
    double rhs1[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        b[i] = rhs[i];
        rhs1[i] = b[4 + i] - r * rhs[i];
    }
    ok = gepp_small<4>(S, rhs1, 4) && ok;
#pragma unroll
    for (int i = 0; i < 4; ++i) b[4 + i] = rhs1[i];
    return ok;
}

// Packed element record of the per-hyperplane lists: local coordinates
// (5 bits per mode for D = 3, 4 bits for D = 4), bit 24+mu set when the
// coordinate is the first row of a 2x2 block of mode mu, bit 31 set when the
// element's tuple is 1x...x1.
template <int D>
struct ElemRec {
    static constexpr int kBits = (D == 3) ? 5 : 4;
    __device__ static inline uint32_t make(const int* c, int first_mask, bool single) {
        uint32_t v = 0;
#pragma unroll
        for (int mu = 0; mu < D; ++mu) v |= (uint32_t)c[mu] << (kBits * mu);
        return v | ((uint32_t)first_mask << 24) | (single ? 0x80000000u : 0u);
    }
    __device__ static inline void coords(uint32_t v, int* c) {
#pragma unroll
        for (int mu = 0; mu < D; ++mu) c[mu] = (v >> (kBits * mu)) & ((1 << kBits) - 1);
    }
};

// ---------------------------------------------------------------------------
// Leaf kernel.  One workgroup per leaf block B.  On entry X[B] holds the
// right-hand side minus the updates of mode 0; the updates of the other
// modes wait in their accumulators.  The kernel
//   1. loads X[B] - sum_mu A_mu[B] and the diagonal blocks T_mu[B, B] to LDS;
//   2. subtracts the contribution of the next block along each mode
//      (T_mu[B, B+1] x_mu X[B+1]: the split between two adjacent leaves);
//   3. runs block back-substitution over the 1x1 / 2x2 diagonal blocks
//      ("tuples") of the leaf, hyperplane by hyperplane: a tuple depends only
//      on tuples that are larger in one index, so the tuples of one
//      hyperplane are independent.  Per hyperplane, phase A gives every
//      (element, mode) pair to its own thread, which sums T_mu[i, j] X[.., j, ..]
//      over the rows j past the element's diagonal block; phase B completes
//      each 1x1x1 tuple with one division by its eigenvalue sum and solves
//      each larger tuple's small system;
//   4. stores X[B].
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(kLeafThreads) void leaf_kernel(
    const LeafDesc* __restrict__ leaves, int64_t first, const ProbDesc* __restrict__ probs,
    int* __restrict__ status, int bm0, int bm1, int bm2, int bm3) {
    extern __shared__ double smem[];
    constexpr int NEMAX = 1 << D;
    constexpr int kSlots = (D == 4) ? 2 : 0;  // threads that solve tuples with ne = 16
    const int tid = threadIdx.x;
    const LeafDesc L = leaves[first + blockIdx.x];
    const ProbDesc& P = probs[L.prob];
    const int bm[4] = {bm0, bm1, bm2, bm3};

    int st[D], sz[D], ls[D], sa[D];
    int64_t gs[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const int32_t* b = P.bst[mu];
        st[mu] = b[L.blk[mu]];
        sz[mu] = b[L.blk[mu] + 1] - st[mu];
        sa[mu] = (L.flags & (1 << (4 + mu))) ? b[L.blk[mu] + 2] - b[L.blk[mu] + 1] : 0;
        gs[mu] = P.stride[mu];
    }
    ls[D - 1] = 1;
#pragma unroll
    for (int mu = D - 2; mu >= 0; --mu) ls[mu] = ls[mu + 1] * sz[mu + 1];
    const int ne_all = ls[0] * sz[0];
    int64_t gbase = 0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) gbase += (int64_t)st[mu] * gs[mu];

    // ---- LDS carve-up (see leaf_lds_bytes)
    int cap = 1, psum = 0, emax = 2;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        cap *= bm[mu];
        psum += bm[mu];
    }
#pragma unroll
    for (int mu = 0; mu < D - 1; ++mu) emax *= bm[mu];
    if (emax > cap) emax = cap;
    double* Xs = smem;
    double* cursor = Xs + cap;
    double* Ts[D];
    double* Ta[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        Ts[mu] = cursor;
        cursor += bm[mu] * bm[mu];
    }
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        Ta[mu] = cursor;
        cursor += bm[mu] * bm[mu];
    }
    double* Pp = cursor;  // D * emax partial sums of one hyperplane
    cursor += D * emax;
    double* scratch = cursor;  // kSlots x (NEMAX*NEMAX + NEMAX), order 4 only
    cursor += kSlots * (NEMAX * NEMAX + NEMAX);
    uint32_t* elist = reinterpret_cast<uint32_t*>(cursor);  // cap
    uint16_t* tlist = reinterpret_cast<uint16_t*>(elist + cap);  // cap: slot | (log2 ne << 11)
    int* icur = reinterpret_cast<int*>(tlist + cap + (cap & 1));
    int* tstart[D];
    int* tidx[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        tstart[mu] = icur;
        icur += bm[mu] + 1;
        tidx[mu] = icur;
        icur += bm[mu];
    }
    int* ntup = icur;
    icur += D;
    const int nplanes_max = psum + 1;
    int* ecnt = icur;  // per hyperplane: count, then fill cursor
    icur += nplanes_max;
    int* eoff = icur;
    icur += nplanes_max + 1;
    int* tcnt = icur;
    icur += nplanes_max;
    int* toff = icur;
    icur += nplanes_max + 1;

    double* __restrict__ Xg = P.X;
    const double* Ag[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) Ag[mu] = (mu >= 1 && (L.flags & (1 << mu))) ? P.A[mu] : nullptr;

    // ---- 1. right-hand side X[B] - sum_mu A_mu[B], kBatch loads in flight
    auto goff = [&](int e) {
        int64_t off = gbase;
        int rem = e;
#pragma unroll
        for (int mu = D - 1; mu >= 1; --mu) {
            const int l = rem % sz[mu];
            rem /= sz[mu];
            off += (int64_t)l * gs[mu];
        }
        return off + (int64_t)rem * gs[0];
    };
    for (int base = 0; base < ne_all; base += kLeafThreads * kBatch) {
        double v[kBatch];
        int64_t offs[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = base + u * kLeafThreads + tid;
            offs[u] = (e < ne_all) ? goff(e) : gbase;
            v[u] = (e < ne_all) ? Xg[offs[u]] : 0.0;
        }
#pragma unroll
        for (int mu = 1; mu < D; ++mu)
            if (Ag[mu]) {
#pragma unroll
                for (int u = 0; u < kBatch; ++u)
                    if (base + u * kLeafThreads + tid < ne_all) v[u] -= Ag[mu][offs[u]];
            }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = base + u * kLeafThreads + tid;
            if (e < ne_all) Xs[e] = v[u];
        }
    }
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const double* Tg = P.T[mu];
        const int64_t nm = P.n[mu];
        const int nd = sz[mu] * sz[mu], na = sz[mu] * sa[mu];
        for (int base = 0; base < nd + na; base += kLeafThreads * 2) {
            double v[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = base + u * kLeafThreads + tid;
                double x = 0.0;
                if (e < nd) {
                    x = Tg[(int64_t)(st[mu] + e / sz[mu]) * nm + st[mu] + e % sz[mu]];
                } else if (e < nd + na) {
                    const int f = e - nd;
                    x = Tg[(int64_t)(st[mu] + f / sa[mu]) * nm + st[mu] + sz[mu] + f % sa[mu]];
                }
                v[u] = x;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = base + u * kLeafThreads + tid;
                if (e < nd)
                    Ts[mu][e] = v[u];
                else if (e < nd + na)
                    Ta[mu][e - nd] = v[u];
            }
        }
    }
    for (int i = tid; i < nplanes_max; i += kLeafThreads) {
        ecnt[i] = 0;
        tcnt[i] = 0;
    }
    __syncthreads();

    // ---- 2. contributions of the next block along each mode: one thread per
    // fiber along mu; the fiber of the next block sits in registers and meets
    // every row of T_mu[B, B+1].
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        if (sa[mu] == 0) continue;
        const int ncol = ne_all / sz[mu];
        const int64_t smu = gs[mu];
        for (int col = tid; col < ncol; col += kLeafThreads) {
            int64_t gb = gbase + (int64_t)sz[mu] * smu;
            int lb = 0, rem = col;
#pragma unroll
            for (int nu = D - 1; nu >= 0; --nu) {
                if (nu == mu) continue;
                const int l = rem % sz[nu];
                rem /= sz[nu];
                lb += l * ls[nu];
                gb += (int64_t)l * gs[nu];
            }
            double xa[kAdjMax];
#pragma unroll
            for (int j = 0; j < kAdjMax; ++j) xa[j] = (j < sa[mu]) ? Xg[gb + j * smu] : 0.0;
            for (int l = 0; l < sz[mu]; ++l) {
                const double* Tr = Ta[mu] + l * sa[mu];
                double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
                for (int j = 0; j < kAdjMax; j += 2) {
                    if (j < sa[mu]) acc0 = fma(Tr[j], xa[j], acc0);
                    if (j + 1 < sa[mu]) acc1 = fma(Tr[j + 1], xa[j + 1], acc1);
                }
                Xs[lb + l * ls[mu]] -= acc0 + acc1;
            }
        }
        __syncthreads();
    }

    // ---- tuple partition of each mode: tstart (first row of each diagonal
    // block), tidx (block index of each row)
    if (tid < D) {
        const int mu = tid;
        int k = 0, i = 0;
        const int s = sz[mu];
        const double* Tm = Ts[mu];
        while (i < s) {
            tstart[mu][k] = i;
            const int w = (i + 1 < s && Tm[(i + 1) * s + i] != 0.0) ? 2 : 1;
            for (int q = 0; q < w; ++q) tidx[mu][i + q] = k;
            ++k;
            i += w;
        }
        tstart[mu][k] = s;
        ntup[mu] = k;
    }
    __syncthreads();
    int nt[D];
    int smax = 0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        nt[mu] = ntup[mu];
        smax += nt[mu] - 1;
    }
    int lead = 1;  // tuples of the leading D-1 modes: one thread each
#pragma unroll
    for (int mu = 0; mu < D - 1; ++mu) lead *= nt[mu];

    // ---- per-hyperplane lists.  Every tuple reserves ne consecutive slots of
    // its hyperplane's element list; tuples with ne > 1 are also listed with
    // their base slot.
    for (int pass = 0; pass < 2; ++pass) {
        for (int lin = tid; lin < lead; lin += kLeafThreads) {
            int p[D];
            int rem = lin, plane0 = 0;
#pragma unroll
            for (int mu = D - 2; mu >= 0; --mu) {
                p[mu] = rem % nt[mu];
                rem /= nt[mu];
                plane0 += p[mu];
            }
            int a[D], w[D], nel = 1;
#pragma unroll
            for (int mu = 0; mu < D - 1; ++mu) {
                a[mu] = tstart[mu][p[mu]];
                w[mu] = tstart[mu][p[mu] + 1] - a[mu];
                nel *= w[mu];
            }
            for (int pl = 0; pl < nt[D - 1]; ++pl) {
                a[D - 1] = tstart[D - 1][pl];
                w[D - 1] = tstart[D - 1][pl + 1] - a[D - 1];
                const int ne = nel * w[D - 1];
                const int plane = plane0 + pl;
                if (pass == 0) {
                    atomicAdd(&ecnt[plane], ne);
                    if (ne > 1) atomicAdd(&tcnt[plane], 1);
                } else {
                    const int base = atomicAdd(&ecnt[plane], ne);
                    int fm = 0;
#pragma unroll
                    for (int mu = 0; mu < D; ++mu)
                        if (w[mu] == 2) fm |= 1 << mu;
                    for (int q = 0; q < ne; ++q) {
                        int c[D], rq = q;
#pragma unroll
                        for (int mu = D - 1; mu >= 0; --mu) {
                            const int d = (w[mu] == 2) ? (rq & 1) : 0;
                            if (w[mu] == 2) rq >>= 1;
                            c[mu] = a[mu] + d;
                        }
                        int first_mask = 0;
#pragma unroll
                        for (int mu = 0; mu < D; ++mu)
                            if ((fm >> mu) & 1 && c[mu] == a[mu]) first_mask |= 1 << mu;
                        elist[base + q] = ElemRec<D>::make(c, first_mask, ne == 1);
                    }
                    // slot relative to the start of the hyperplane's list
                    if (ne > 1)
                        tlist[atomicAdd(&tcnt[plane], 1)] =
                            (uint16_t)((base - eoff[plane]) | ((31 - __builtin_clz((unsigned)ne)) << 11));
                }
            }
        }
        __syncthreads();
        if (pass == 0 && tid == 0) {
            int ea = 0, ta = 0;
            for (int i = 0; i <= smax; ++i) {
                eoff[i] = ea;
                ea += ecnt[i];
                ecnt[i] = eoff[i];
                toff[i] = ta;
                ta += tcnt[i];
                tcnt[i] = toff[i];
            }
            eoff[smax + 1] = ea;
            toff[smax + 1] = ta;
        }
        __syncthreads();
    }

    // ---- 3. hyperplanes
    bool ok = true;
    for (int s = smax; s >= 0; --s) {
        const int e0 = eoff[s], nel = eoff[s + 1] - e0;
        // phase A: partial sums per (element, mode)
        for (int it = tid; it < D * nel; it += kLeafThreads) {
            const int j = it / D, mu = it - j * D;
            const uint32_t rec = elist[e0 + j];
            int c[D];
            ElemRec<D>::coords(rec, c);
            int e = 0;
#pragma unroll
            for (int nu = 0; nu < D; ++nu) e += c[nu] * ls[nu];
            const int i = c[mu];
            const int js = i + 1 + ((rec >> (24 + mu)) & 1);
            const int len = sz[mu] - js;
            const double* Tr = Ts[mu] + i * sz[mu] + js;
            const double* Xp = Xs + e + (js - i) * ls[mu];
            const int step = ls[mu];
            double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
            int k = 0;
            for (; k + 3 < len; k += 4) {
                acc0 = fma(Tr[k], Xp[k * step], acc0);
                acc1 = fma(Tr[k + 1], Xp[(k + 1) * step], acc1);
                acc2 = fma(Tr[k + 2], Xp[(k + 2) * step], acc2);
                acc3 = fma(Tr[k + 3], Xp[(k + 3) * step], acc3);
            }
            for (; k < len; ++k) acc0 = fma(Tr[k], Xp[k * step], acc0);
            Pp[it] = (acc0 + acc1) + (acc2 + acc3);
        }
        __syncthreads();
        // phase B: 1x1x1 tuples (one thread per element, from the bottom) and
        // larger tuples (one thread per tuple, from the top)
        for (int j = tid; j < nel; j += kLeafThreads) {
            const uint32_t rec = elist[e0 + j];
            if (!(rec >> 31)) continue;
            int c[D];
            ElemRec<D>::coords(rec, c);
            int e = 0;
            double dg = 0.0, r = 0.0;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) {
                e += c[mu] * ls[mu];
                dg += Ts[mu][c[mu] * sz[mu] + c[mu]];
                r += Pp[D * j + mu];
            }
            const double x = (Xs[e] - r) / dg;
            if (dg == 0.0 || !isfinite(x)) ok = false;
            Xs[e] = x;
        }
        const int t0 = toff[s], ntu = toff[s + 1] - t0;
        for (int ti = kLeafThreads - 1 - tid; ti < ntu; ti += kLeafThreads) {
            const uint32_t tr = tlist[t0 + ti];
            const int base = tr & 0x7ff, ne = 1 << (tr >> 11);
            const uint32_t rec0 = elist[e0 + base];
            int a[D], w[D];
            ElemRec<D>::coords(rec0, a);  // first element = lowest coordinates
            int eb = 0, kb = 0;
            double cdiag = 0.0;
            double Dm[4][4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) Dm[j][v] = 0.0;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) {
                w[mu] = ((rec0 >> (24 + mu)) & 1) ? 2 : 1;
                eb += a[mu] * ls[mu];
                const double* Tm = Ts[mu] + a[mu] * sz[mu] + a[mu];
                if (w[mu] == 2) {
                    const double d0 = Tm[0], d1 = Tm[1], d2 = Tm[sz[mu]], d3 = Tm[sz[mu] + 1];
                    // compact the 2x2 blocks in mode order (static indices only)
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
            // right-hand sides in local order (last mode fastest = bit 0)
            double rb[8];
            int eidx[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                eidx[q] = eb;
                rb[q] = 0.0;
                if (q < ne) {
                    int rq = q, e = eb;
#pragma unroll
                    for (int mu = D - 1; mu >= 0; --mu)
                        if (w[mu] == 2) {
                            e += (rq & 1) * ls[mu];
                            rq >>= 1;
                        }
                    eidx[q] = e;
                    double r = Xs[e];
#pragma unroll
                    for (int mu = 0; mu < D; ++mu) r -= Pp[D * (base + q) + mu];
                    rb[q] = r;
                }
            }
            bool tok = true;
            if (ne == 2) {
                double M[2][2], r2[2] = {rb[0], rb[1]};
                tuple_matrix<2>(M, Dm, cdiag);
                tok = gepp_small<2>(M, r2, 2);
                rb[0] = r2[0];
                rb[1] = r2[1];
            } else if (ne == 4) {
                double M[4][4], r4[4] = {rb[0], rb[1], rb[2], rb[3]};
                tuple_matrix<4>(M, Dm, cdiag);
                tok = gepp_small<4>(M, r4, 4);
#pragma unroll
                for (int q = 0; q < 4; ++q) rb[q] = r4[q];
            } else if (ne == 8) {
                tok = tuple_solve8(Dm, cdiag, rb);
            } else {
                tok = false;  // ne = 16 is handled below
            }
            if (ne <= 8) {
                if (!tok) ok = false;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (q < ne) Xs[eidx[q]] = rb[q];
            }
        }
        if (D == 4) {
            // ne = 16 (2x2 blocks in all four modes): staged in LDS
            if (tid < kSlots) {
                double* Ms = scratch + tid * (NEMAX * NEMAX + NEMAX);
                double* rs = Ms + NEMAX * NEMAX;
                for (int ti = tid; ti < ntu; ti += kSlots) {
                    const uint32_t tr = tlist[t0 + ti];
                    const int base = tr & 0x7ff, ne = 1 << (tr >> 11);
                    if (ne != 16) continue;
                    const uint32_t rec0 = elist[e0 + base];
                    int a[D], w[D];
                    ElemRec<D>::coords(rec0, a);
#pragma unroll
                    for (int mu = 0; mu < D; ++mu) w[mu] = 2;
                    for (int q = 0; q < ne; ++q) {
                        double r = Xs[tuple_elem<D>(ls, a, w, q)];
                        for (int mu = 0; mu < D; ++mu) r -= Pp[D * (base + q) + mu];
                        rs[q] = r;
                        for (int q2 = 0; q2 < ne; ++q2) Ms[q * ne + q2] = tuple_coupling<D>(Ts, sz, a, w, q, q2);
                    }
                    for (int k = 0; k < ne; ++k) {
                        int piv = k;
                        for (int i2 = k + 1; i2 < ne; ++i2)
                            if (fabs(Ms[i2 * ne + k]) > fabs(Ms[piv * ne + k])) piv = i2;
                        if (piv != k) {
                            for (int j = 0; j < ne; ++j) {
                                double t = Ms[k * ne + j];
                                Ms[k * ne + j] = Ms[piv * ne + j];
                                Ms[piv * ne + j] = t;
                            }
                            double t = rs[k];
                            rs[k] = rs[piv];
                            rs[piv] = t;
                        }
                        const double pv = Ms[k * ne + k];
                        if (pv == 0.0) ok = false;
                        for (int i2 = k + 1; i2 < ne; ++i2) {
                            const double f = Ms[i2 * ne + k] / pv;
                            for (int j = k; j < ne; ++j) Ms[i2 * ne + j] -= f * Ms[k * ne + j];
                            rs[i2] -= f * rs[k];
                        }
                    }
                    for (int k = ne - 1; k >= 0; --k) {
                        double acc = rs[k];
                        for (int j = k + 1; j < ne; ++j) acc -= Ms[k * ne + j] * rs[j];
                        rs[k] = acc / Ms[k * ne + k];
                        if (!isfinite(rs[k])) ok = false;
                    }
                    for (int q = 0; q < ne; ++q) Xs[tuple_elem<D>(ls, a, w, q)] = rs[q];
                }
            }
        }
        __syncthreads();
    }
    if (!ok) atomicOr(status, 1);

    // ---- 4. store the solved block
    for (int base = 0; base < ne_all; base += kLeafThreads * kBatch) {
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = base + u * kLeafThreads + tid;
            if (e < ne_all) Xg[goff(e)] = Xs[e];
        }
    }
}

int leaf_lds_bytes(int D, const int* bmax) {
    int cap = 1, tsum = 0, isum = 0, psum = 0, emax = 2;
    for (int mu = 0; mu < D; ++mu) {
        cap *= bmax[mu];
        tsum += 2 * bmax[mu] * bmax[mu];
        isum += 2 * bmax[mu] + 1;
        psum += bmax[mu];
    }
    for (int mu = 0; mu < D - 1; ++mu) emax *= bmax[mu];
    if (emax > cap) emax = cap;
    const int nemax = 1 << D;
    const int slots = (D == 4) ? 2 : 0;
    const int dbl = cap + tsum + D * emax + slots * (nemax * nemax + nemax);
    const int ints = isum + D + 4 * (psum + 1) + 2;
    return dbl * (int)sizeof(double) + cap * (int)sizeof(uint32_t) + (cap + (cap & 1)) * (int)sizeof(uint16_t) +
           ints * (int)sizeof(int);
}

// ---------------------------------------------------------------------------
// Update kernel: one workgroup per 64x64 output tile of one pencil update of
// the recursion (Algorithm 2's B_1 <- B_1 - X_2 x_mu A_mu(1:k, k+1:n_mu)):
//   C[r, c] (+)= sum_k A[r, k] * Bx[k, c]
// with A = T_mu[r0 + r, k0 + k], Bx[k, c] = X[col_off(c) + (k0 + k) s_mu],
// and C[r, c] the target element at col_off(c) + (r0 + r) s_mu: X itself for
// mode 0 (subtract), the accumulator of mode mu otherwise (add, or store for
// the first contribution).  The 64x64 tile is four 32x32 wave tiles of 2x2
// MFMA 16x16x4 FP64 blocks; K advances in chunks of 16 staged through LDS.
// For the fastest mode (s_mu = 1) the roles are transposed so that the
// contiguous index runs along the MFMA columns.
//
// v_mfma_f64_16x16x4f64 lane layout (gfx950): A[i][k] from lane 16k + i,
// B[k][j] from lane 16k + j, D[i][j] in lane 16 (i % 4) + j, element i / 4.
// ---------------------------------------------------------------------------
constexpr int kKC = 16;      // K chunk
constexpr int kLdsRow = 80;  // 64 + 16 doubles: rows k and k+1 use disjoint bank halves

__device__ inline int64_t pencil_col_offset(const UpdDesc& t, int c) {
    int64_t off = t.xbase;
    int rem = c;
    off += (int64_t)(rem % t.ext[2]) * t.ostr[2];
    rem /= t.ext[2];
    off += (int64_t)(rem % t.ext[1]) * t.ostr[1];
    rem /= t.ext[1];
    off += (int64_t)rem * t.ostr[0];
    return off;
}

__device__ inline void mfma_chunk(const double* As, const double* Bs, int wr, int wc, int li, int lk,
                                  dbl4 (&acc)[2][2]) {
#pragma unroll
    for (int kk = 0; kk < kKC; kk += 4) {
        const double* Ak = As + (kk + lk) * kLdsRow;
        const double* Bk = Bs + (kk + lk) * kLdsRow;
        double a0 = Ak[wr + li], a1 = Ak[wr + 16 + li];
        double b0 = Bk[wc + li], b1 = Bk[wc + 16 + li];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
}

__global__ __launch_bounds__(kUpdThreads) void upd_kernel(const UpdDesc* __restrict__ tasks,
                                                          const WorkItem* __restrict__ items,
                                                          int64_t first,
                                                          const ProbDesc* __restrict__ probs, int D) {
    __shared__ double As[kKC * kLdsRow];
    __shared__ double Bs[kKC * kLdsRow];
    __shared__ int64_t colOff[kTile];
    const int tid = threadIdx.x;
    const WorkItem wi = items[first + blockIdx.x];
    const UpdDesc t = tasks[wi.task];
    const ProbDesc& P = probs[t.prob];
    const int mode = t.mode;
    const double* __restrict__ X = P.X;
    double* __restrict__ C = (mode == 0) ? P.X : P.A[mode];
    const double* __restrict__ T = P.T[mode];
    const int64_t nmu = P.n[mode];
    const int64_t smu = P.stride[mode];
    const bool right = (mode == D - 1);
    const bool store = (t.flags & 1) != 0;
    const double sgn = (mode == 0) ? -1.0 : 1.0;
    const int col0 = (right ? wi.ta : wi.tb) * kTile;  // pencil columns
    const int row0 = (right ? wi.tb : wi.ta) * kTile;  // target rows in mode mu

    if (tid < kTile) {
        int c = col0 + tid;
        colOff[tid] = (c < t.P) ? pencil_col_offset(t, c) : 0;
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    dbl4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int nchunk = (t.K + kKC - 1) / kKC;

    if (!right) {
        // MFMA rows = target rows r, MFMA columns = pencil columns c.
        // loaders: A: (row = tid/4, k = 4*(tid%4)..+3); B: (k = tid/16, c = 4*(tid%16)..+3)
        const int la_r = tid >> 2, la_k = (tid & 3) * 4;
        const int lb_k = tid >> 4, lb_c = (tid & 15) * 4;
        double ra[4], rb[4];
        int64_t boff[4];
        bool bval[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            boff[i] = colOff[lb_c + i];
            bval[i] = (col0 + lb_c + i) < t.P;
        }
        const bool aval_r = (row0 + la_r) < t.M;
        const double* Arow = T + (int64_t)(t.r0 + row0 + la_r) * nmu + t.k0;
        auto gload = [&](int kc) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int k = kc + la_k + i;
                ra[i] = (aval_r && k < t.K) ? Arow[k] : 0.0;
            }
            int kb = kc + lb_k;
            bool kvalid = kb < t.K;
            int64_t roff = (int64_t)(t.k0 + kb) * smu;
#pragma unroll
            for (int i = 0; i < 4; ++i) rb[i] = (kvalid && bval[i]) ? X[boff[i] + roff] : 0.0;
        };
        gload(0);
        for (int ch = 0; ch < nchunk; ++ch) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 4; ++i) As[(la_k + i) * kLdsRow + la_r] = ra[i];
#pragma unroll
            for (int i = 0; i < 4; ++i) Bs[lb_k * kLdsRow + lb_c + i] = rb[i];
            __syncthreads();
            if (ch + 1 < nchunk) gload((ch + 1) * kKC);
            mfma_chunk(As, Bs, wr, wc, li, lk, acc);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = wc + 16 * j + li;
            if (col0 + c >= t.P) continue;
            const int64_t coff = colOff[c];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = wr + 16 * i + 4 * v + lk;
                    if (row0 + r < t.M) {
                        double* p = C + coff + (int64_t)(t.r0 + row0 + r) * smu;
                        const double val = sgn * acc[i][j][v];
                        *p = store ? val : *p + val;
                    }
                }
        }
    } else {
        // MFMA rows = pencil columns c, MFMA columns = target rows r.
        const int lr = tid >> 2, lk4 = (tid & 3) * 4;
        const bool cval = (col0 + lr) < t.P;
        const bool rval = (row0 + lr) < t.M;
        const double* Xrow = X + colOff[lr] + t.k0;
        const double* Trow = T + (int64_t)(t.r0 + row0 + lr) * nmu + t.k0;
        double ra[4], rb[4];
        auto gload = [&](int kc) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int k = kc + lk4 + i;
                ra[i] = (cval && k < t.K) ? Xrow[k] : 0.0;
                rb[i] = (rval && k < t.K) ? Trow[k] : 0.0;
            }
        };
        gload(0);
        for (int ch = 0; ch < nchunk; ++ch) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                As[(lk4 + i) * kLdsRow + lr] = ra[i];
                Bs[(lk4 + i) * kLdsRow + lr] = rb[i];
            }
            __syncthreads();
            if (ch + 1 < nchunk) gload((ch + 1) * kKC);
            mfma_chunk(As, Bs, wr, wc, li, lk, acc);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = wr + 16 * i + 4 * v + lk;
                if (col0 + c >= t.P) continue;
                const int64_t coff = colOff[c];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int r = wc + 16 * j + li;
                    if (row0 + r < t.M) {
                        double* p = C + coff + t.r0 + row0 + r;
                        const double val = sgn * acc[i][j][v];
                        *p = store ? val : *p + val;
                    }
                }
            }
    }
}

__global__ void zero_int_kernel(int* p, int count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

__global__ void copy_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_leaf(int D, const LeafDesc* leaves, int64_t first, int64_t count,
                       const ProbDesc* probs, int* status, const int* bmax, int lds_bytes,
                       hipStream_t st) {
    if (count <= 0) return hipSuccess;
    dim3 grid((unsigned)count), block(kLeafThreads);
    if (lds_bytes > 64 * 1024) {
        hipError_t e = (D == 3) ? hipFuncSetAttribute((const void*)leaf_kernel<3>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes)
                                : hipFuncSetAttribute((const void*)leaf_kernel<4>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
    }
    if (D == 3) {
        hipLaunchKernelGGL(leaf_kernel<3>, grid, block, lds_bytes, st, leaves, first, probs, status,
                           bmax[0], bmax[1], bmax[2], 1);
    } else {
        hipLaunchKernelGGL(leaf_kernel<4>, grid, block, lds_bytes, st, leaves, first, probs, status,
                           bmax[0], bmax[1], bmax[2], bmax[3]);
    }
    return hipGetLastError();
}

hipError_t launch_update(int D, const UpdDesc* tasks, const WorkItem* items, int64_t first,
                         int64_t count, const ProbDesc* probs, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(upd_kernel, dim3((unsigned)count), dim3(kUpdThreads), 0, st, tasks, items, first, probs, D);
    return hipGetLastError();
}

hipError_t launch_zero_int(int* p, int count, hipStream_t st) {
    hipLaunchKernelGGL(zero_int_kernel, dim3((count + 255) / 256), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

}  // namespace tt
