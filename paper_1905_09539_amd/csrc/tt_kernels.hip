// gfx950 kernels of the triangular Kronecker solve.
//
//   leaf_kernel   - solves one leaf block of the recursion (the "solve full
//                   system" base case of Algorithm 2, Sec. 2.1) in LDS by
//                   block back-substitution over its 1x1 / 2x2 diagonal
//                   blocks, hyperplane by hyperplane.
//   upd_kernel    - the right-hand-side update of Algorithm 2,
//                   B_1 <- B_1 - X_2 x_mu A_mu(1:k, k+1:n_mu), for one pencil,
//                   on FP64 MFMA (v_mfma_f64_16x16x4f64).
#include <algorithm>

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

// Packed element record of the per-hyperplane lists:
//   bits 0-15  local coordinates (5 bits per mode for D = 3, 4 for D = 4)
//   bits 16-19 index q of the element inside its tuple (last mode = bit 0)
//   bits 20-22 log2 of the tuple's number of unknowns ne
//   bits 24-27 bit mu set when the coordinate is the first row of a 2x2 block
template <int D>
struct ElemRec {
    static constexpr int kBits = (D == 3) ? 5 : 4;
    __device__ static inline uint32_t make(const int* c, int q, int lne, int first_mask) {
        uint32_t v = 0;
#pragma unroll
        for (int mu = 0; mu < D; ++mu) v |= (uint32_t)c[mu] << (kBits * mu);
        return v | ((uint32_t)q << 16) | ((uint32_t)lne << 20) | ((uint32_t)first_mask << 24);
    }
    __device__ static inline void coords(uint32_t v, int* c) {
#pragma unroll
        for (int mu = 0; mu < D; ++mu) c[mu] = (v >> (kBits * mu)) & ((1 << kBits) - 1);
    }
    __device__ static inline int q(uint32_t v) { return (v >> 16) & 15; }
    __device__ static inline int lne(uint32_t v) { return (v >> 20) & 7; }
    __device__ static inline int fmask(uint32_t v) { return (v >> 24) & 15; }
};

// 2x2 blocks (mode order) and diagonal sum of the 1x1 modes of the tuple whose
// first element has local coordinates a and first-row mask fm.
template <int D>
__device__ inline void tuple_blocks(double* const* Ts, const int* sz, const int* a, int fm, double (&Dm)[4][4],
                                    double& cdiag) {
    int kb = 0;
    cdiag = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) Dm[j][v] = 0.0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const double* Tm = Ts[mu] + a[mu] * sz[mu] + a[mu];
        if ((fm >> mu) & 1) {
            const double d0 = Tm[0], d1 = Tm[1], d2 = Tm[sz[mu]], d3 = Tm[sz[mu] + 1];
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
}

// Slot classes of a hyperplane's element list, in layout order: tuples with
// 16, 8, 4, 2 unknowns, then 1x..x1 tuples.  Each class region starts at a
// multiple of its tuple size, so no tuple straddles a 64-lane wavefront.
__device__ inline int ne_class(int lne) { return 4 - lne; }  // lne 4 -> 0, ..., 0 -> 4

constexpr int kPoolWant = 4096;  // doubles of precomputed tuple inverses per leaf

// ---------------------------------------------------------------------------
// Leaf kernel.  One workgroup per leaf block B.  On entry X[B] holds the
// right-hand side minus the updates of mode 0; the updates of the other
// modes wait in their accumulators.  The kernel
//   1. loads X[B] - sum_mu A_mu[B] and the diagonal blocks T_mu[B, B] to LDS;
//   2. subtracts the contribution of the next block along each mode
//      (T_mu[B, B+1] x_mu X[B+1]: the split between two adjacent leaves);
//   3. partitions each mode into its 1x1 / 2x2 diagonal blocks, lists the
//      elements of every tuple hyperplane (tuples of 16, 8, 4, 2 unknowns
//      first, each aligned to its size), and inverts the small systems
//      M_p = sum_mu I (x) T_mu[p_mu, p_mu] (x) I of the tuples with 4 or 8
//      unknowns, one column per thread;
//   4. runs block back-substitution hyperplane by hyperplane: a tuple depends
//      only on tuples that are larger in one index, so the tuples of one
//      hyperplane are independent.  Phase A gives every (element, mode) its
//      own thread for the sum of T_mu[i, j] X[.., j, ..] over the rows j past
//      the element's diagonal block; phase B gives every element its own
//      thread, which forms the right-hand sides of its tuple and writes its
//      unknown: a division by the eigenvalue sum (1 unknown), Cramer's rule
//      (2 unknowns), a row of the precomputed inverse (4 or 8), or Gaussian
//      elimination with partial pivoting (16, or when the inverse pool is
//      full).  A tuple's threads share one wavefront, so they all read the
//      right-hand sides before any of them writes;
//   5. stores X[B].
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(kLeafThreads) void leaf_kernel(
    const LeafDesc* __restrict__ leaves, int64_t first, const ProbDesc* __restrict__ probs,
    int* __restrict__ status, int bm0, int bm1, int bm2, int bm3, int kPoolMax) {
    extern __shared__ double smem[];
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

    // ---- LDS carve-up (sizes must match leaf_lds_bytes)
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
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        Ts[mu] = cursor;
        cursor += bm[mu] * bm[mu];
    }
    // the blocks next to the diagonal are only needed before the partial
    // sums exist, so the two share storage
    double* Pp = cursor;  // D * emax partial sums of one hyperplane
    double* Ta[D];
    {
        double* c2 = cursor;
#pragma unroll
        for (int mu = 0; mu < D; ++mu) {
            Ta[mu] = c2;
            c2 += bm[mu] * bm[mu];
        }
    }
    int tsum = 0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) tsum += bm[mu] * bm[mu];
    cursor += max(D * emax, tsum);
    double* pool = cursor;  // precomputed inverses of tuples with 4 or 8 unknowns
    cursor += kPoolMax;
    uint32_t* elist = reinterpret_cast<uint32_t*>(cursor);  // cap element records
    uint16_t* pslot = reinterpret_cast<uint16_t*>(elist + cap);  // cap: pool offset at a tuple's first slot
    int* icur = reinterpret_cast<int*>(pslot + cap + (cap & 1));
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
    int* ccnt = icur;  // per hyperplane and class: tuple count, then fill cursor
    icur += 5 * nplanes_max;
    int* cbase = icur;  // per hyperplane and class: first slot of the class region
    icur += 5 * nplanes_max;
    int* eoff = icur;  // per hyperplane: first slot; eoff[smax+1] = total
    icur += nplanes_max + 1;
    int* poolcnt = icur;
    icur += 1;

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
    for (int i = tid; i < 5 * nplanes_max; i += kLeafThreads) ccnt[i] = 0;
    if (tid == 0) *poolcnt = 0;
    __syncthreads();

    // ---- 2. contributions of the next block along each mode on FP64 MFMA:
    // for every fiber f along mu (the other modes' coordinates),
    //   Xs[f, l] -= sum_j T_mu[B_l, (B+1)_j] X[B+1][f, j],
    // i.e. C (sz x F) -= A (sz x sa) * Bx (sa x F): one 16-row tile per 16
    // rows of the leaf, 16 fibers per MFMA column tile, K in steps of 4.
    {
        const int lane = tid & 63, wave = tid >> 6;
        const int li = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int mu = 0; mu < D; ++mu) {
            if (sa[mu] == 0) continue;
            const int nf = ne_all / sz[mu];
            const int ntc = (nf + 15) >> 4, ntr = (sz[mu] + 15) >> 4, nks = (sa[mu] + 3) >> 2;
            const int64_t smu = gs[mu];
            for (int tile = wave; tile < ntc * ntr; tile += kLeafThreads / 64) {
                const int tc = tile % ntc, tr = tile / ntc;
                // this lane's fiber (MFMA column) and its offsets
                const int f = tc * 16 + li;
                int lb = 0;
                int64_t gb = gbase + (int64_t)sz[mu] * smu;
                {
                    int rem = (f < nf) ? f : 0;
#pragma unroll
                    for (int nu = D - 1; nu >= 0; --nu) {
                        if (nu == mu) continue;
                        const int l = rem % sz[nu];
                        rem /= sz[nu];
                        lb += l * ls[nu];
                        gb += (int64_t)l * gs[nu];
                    }
                }
                const int arow = tr * 16 + li;
                dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
                for (int ks = 0; ks < nks; ++ks) {
                    const int kk = ks * 4 + lk;
                    const double av = (arow < sz[mu] && kk < sa[mu]) ? Ta[mu][arow * sa[mu] + kk] : 0.0;
                    const double bv = (f < nf && kk < sa[mu]) ? Xg[gb + kk * smu] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
                if (f < nf) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = tr * 16 + 4 * v + lk;
                        if (row < sz[mu]) Xs[lb + row * ls[mu]] -= acc[v];
                    }
                }
            }
            __syncthreads();
        }
    }

    // ---- 3a. tuple partition of each mode
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
    int lead = 1;
#pragma unroll
    for (int mu = 0; mu < D - 1; ++mu) lead *= nt[mu];

    // ---- 3b. per-hyperplane element lists, ordered by tuple class
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
            int a[D], w[D], lne0 = 0;
#pragma unroll
            for (int mu = 0; mu < D - 1; ++mu) {
                a[mu] = tstart[mu][p[mu]];
                w[mu] = tstart[mu][p[mu] + 1] - a[mu];
                lne0 += w[mu] - 1;
            }
            for (int pl = 0; pl < nt[D - 1]; ++pl) {
                a[D - 1] = tstart[D - 1][pl];
                w[D - 1] = tstart[D - 1][pl + 1] - a[D - 1];
                const int lne = lne0 + w[D - 1] - 1, ne = 1 << lne;
                const int plane = plane0 + pl;
                const int cls = ne_class(lne);
                if (pass == 0) {
                    atomicAdd(&ccnt[plane * 5 + cls], 1);
                } else {
                    const int base = cbase[plane * 5 + cls] + atomicAdd(&ccnt[plane * 5 + cls], 1) * ne;
                    int fm = 0;
#pragma unroll
                    for (int mu = 0; mu < D; ++mu)
                        if (w[mu] == 2) fm |= 1 << mu;
                    for (int q = 0; q < ne; ++q) {
                        int c[D], rq = q;
#pragma unroll
                        for (int mu = D - 1; mu >= 0; --mu) {
                            const int dd = (w[mu] == 2) ? (rq & 1) : 0;
                            if (w[mu] == 2) rq >>= 1;
                            c[mu] = a[mu] + dd;
                        }
                        int first_mask = 0;
#pragma unroll
                        for (int mu = 0; mu < D; ++mu)
                            if (((fm >> mu) & 1) && c[mu] == a[mu]) first_mask |= 1 << mu;
                        elist[base + q] = ElemRec<D>::make(c, q, lne, first_mask);
                    }
                    if (ne == 4 || ne == 8) {
                        const int po = atomicAdd(poolcnt, ne * ne);
                        pslot[base] = (po + ne * ne <= kPoolMax) ? (uint16_t)po : (uint16_t)0xffff;
                    }
                }
            }
        }
        __syncthreads();
        if (pass == 0 && tid < 64) {
            // slot offsets: one lane per hyperplane chunk of 64 (wave scan)
            int carry = 0;
            for (int c0 = 0; c0 <= smax; c0 += 64) {
                const int pl = c0 + tid;
                int tot = 0;
                if (pl <= smax) {
                    int off = 0;
#pragma unroll
                    for (int cls = 0; cls < 5; ++cls) {
                        const int ne = 1 << (4 - cls);
                        cbase[pl * 5 + cls] = off;  // relative for now
                        off += ccnt[pl * 5 + cls] * ne;
                    }
                    tot = off;
                }
                int incl = tot;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int y = __shfl_up(incl, d, 64);
                    if (tid >= d) incl += y;
                }
                if (pl <= smax) {
                    const int start = carry + incl - tot;
                    eoff[pl] = start;
#pragma unroll
                    for (int cls = 0; cls < 5; ++cls) {
                        cbase[pl * 5 + cls] += start;
                        ccnt[pl * 5 + cls] = 0;
                    }
                }
                carry += __shfl(incl, 63, 64);
            }
            if (tid == 0) eoff[smax + 1] = carry;
        }
        __syncthreads();
    }

    // ---- 3c. inverses of the tuple systems with 4 or 8 unknowns: one thread
    // per (tuple, column); column q solves M x = e_q in registers
    const int total = eoff[smax + 1];
    for (int sl = tid; sl < total; sl += kLeafThreads) {
        const uint32_t rec = elist[sl];
        const int lne = ElemRec<D>::lne(rec);
        if (lne != 2 && lne != 3) continue;
        const int q = ElemRec<D>::q(rec), ne = 1 << lne;
        const int b0 = sl - q;
        const int po = pslot[b0];
        if (po == 0xffff) continue;
        const uint32_t rec0 = elist[b0];
        int a[D];
        ElemRec<D>::coords(rec0, a);
        double Dm[4][4], cdiag;
        tuple_blocks<D>(Ts, sz, a, ElemRec<D>::fmask(rec0), Dm, cdiag);
        bool tok;
        if (ne == 4) {
            double M[4][4], r4[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) r4[i] = (i == q) ? 1.0 : 0.0;
            tuple_matrix<4>(M, Dm, cdiag);
            tok = gepp_small<4>(M, r4, 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) pool[po + i * 4 + q] = r4[i];
        } else {
            double r8[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) r8[i] = (i == q) ? 1.0 : 0.0;
            tok = tuple_solve8(Dm, cdiag, r8);
#pragma unroll
            for (int i = 0; i < 8; ++i) pool[po + i * 8 + q] = r8[i];
        }
        if (!tok) atomicOr(status, 1);
    }
    __syncthreads();

    // ---- 4. hyperplanes
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
            const int js = i + 1 + ((ElemRec<D>::fmask(rec) >> mu) & 1);
            const int len = sz[mu] - js;
            double acc0 = 0.0, acc1 = 0.0;
            if (len > 0) {
                const double* Tr = Ts[mu] + i * sz[mu] + js;
                const double* Xp = Xs + e + (js - i) * ls[mu];
                const int step = ls[mu];
                for (int k0 = 0; k0 < len; k0 += 16) {
                    double tv[16], xv[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int k = min(k0 + u, len - 1);
                        tv[u] = Tr[k];
                        xv[u] = Xp[k * step];
                    }
#pragma unroll
                    for (int u = 0; u < 16; u += 2) {
                        if (k0 + u < len) acc0 = fma(tv[u], xv[u], acc0);
                        if (k0 + u + 1 < len) acc1 = fma(tv[u + 1], xv[u + 1], acc1);
                    }
                }
            }
            Pp[it] = acc0 + acc1;
        }
        __syncthreads();
        // phase B: one thread per element of the hyperplane
        for (int j = tid; j < nel; j += kLeafThreads) {
            const uint32_t rec = elist[e0 + j];
            const int lne = ElemRec<D>::lne(rec), q = ElemRec<D>::q(rec);
            int c[D];
            ElemRec<D>::coords(rec, c);
            int e = 0;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) e += c[mu] * ls[mu];
            double x;
            if (lne == 0) {
                double dg = 0.0, r = Xs[e];
#pragma unroll
                for (int mu = 0; mu < D; ++mu) {
                    dg += Ts[mu][c[mu] * sz[mu] + c[mu]];
                    r -= Pp[D * j + mu];
                }
                x = r / dg;
                if (dg == 0.0 || !isfinite(x)) ok = false;
            } else {
                const int ne = 1 << lne, b0 = j - q;
                const uint32_t rec0 = elist[e0 + b0];
                int a[D];
                ElemRec<D>::coords(rec0, a);
                const int fm = ElemRec<D>::fmask(rec0);
                // right-hand sides of the whole tuple (last bumped mode = bit 0)
                constexpr int NEM = 1 << D;
                double rb[NEM];
#pragma unroll
                for (int qq = 0; qq < NEM; ++qq) {
                    rb[qq] = 0.0;
                    if (qq < ne) {
                        int rq = qq, eq = 0;
#pragma unroll
                        for (int mu = D - 1; mu >= 0; --mu) {
                            int dd = 0;
                            if ((fm >> mu) & 1) {
                                dd = rq & 1;
                                rq >>= 1;
                            }
                            eq += (a[mu] + dd) * ls[mu];
                        }
                        double r = Xs[eq];
#pragma unroll
                        for (int mu = 0; mu < D; ++mu) r -= Pp[D * (b0 + qq) + mu];
                        rb[qq] = r;
                    }
                }
                const int po = (ne == 4 || ne == 8) ? (int)pslot[e0 + b0] : 0xffff;
                if (ne == 2) {
                    double Dm[4][4], cdiag;
                    tuple_blocks<D>(Ts, sz, a, fm, Dm, cdiag);
                    const double m00 = Dm[0][0] + cdiag, m01 = Dm[0][1], m10 = Dm[0][2], m11 = Dm[0][3] + cdiag;
                    const double det = m00 * m11 - m01 * m10;
                    x = (q == 0) ? (m11 * rb[0] - m01 * rb[1]) / det : (m00 * rb[1] - m10 * rb[0]) / det;
                    if (det == 0.0 || !isfinite(x)) ok = false;
                } else if (po != 0xffff) {
                    const double* Mi = pool + po + q * ne;
                    double acc = 0.0;
#pragma unroll
                    for (int qq = 0; qq < 8; ++qq)
                        if (qq < ne) acc = fma(Mi[qq], rb[qq], acc);
                    x = acc;
                    if (!isfinite(x)) ok = false;
                } else if (ne <= 8) {
                    // inverse pool full: eliminate in registers
                    double Dm[4][4], cdiag;
                    tuple_blocks<D>(Ts, sz, a, fm, Dm, cdiag);
                    if (ne == 4) {
                        double M[4][4], r4[4] = {rb[0], rb[1], rb[2], rb[3]};
                        tuple_matrix<4>(M, Dm, cdiag);
                        if (!gepp_small<4>(M, r4, 4)) ok = false;
                        x = r4[0];
#pragma unroll
                        for (int qq = 1; qq < 4; ++qq)
                            if (qq == q) x = r4[qq];
                    } else {
                        double r8[8];
#pragma unroll
                        for (int qq = 0; qq < 8; ++qq) r8[qq] = rb[qq];
                        if (!tuple_solve8(Dm, cdiag, r8)) ok = false;
                        x = r8[0];
#pragma unroll
                        for (int qq = 1; qq < 8; ++qq)
                            if (qq == q) x = r8[qq];
                    }
                } else {
                    x = 0.0;
                    if constexpr (D == 4) {
                        // 16 unknowns (2x2 blocks in every mode; rare)
                        double M[16][16];
                        int w[D];
#pragma unroll
                        for (int mu = 0; mu < D; ++mu) w[mu] = 2;
#pragma unroll
                        for (int q1 = 0; q1 < 16; ++q1)
#pragma unroll
                            for (int q2 = 0; q2 < 16; ++q2) M[q1][q2] = tuple_coupling<D>(Ts, sz, a, w, q1, q2);
                        if (!gepp_small<16>(M, rb, 16)) ok = false;
                        x = rb[0];
#pragma unroll
                        for (int qq = 1; qq < 16; ++qq)
                            if (qq == q) x = rb[qq];
                    }
                }
            }
            // every thread of this wavefront has read its right-hand sides
            // (program order within a wavefront) before any writes below
            Xs[e] = x;
        }
        __syncthreads();
    }
    if (!ok) atomicOr(status, 1);

    // ---- 5. store the solved block
    for (int base = 0; base < ne_all; base += kLeafThreads * kBatch) {
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = base + u * kLeafThreads + tid;
            if (e < ne_all) Xg[goff(e)] = Xs[e];
        }
    }
}

// LDS bytes of the leaf kernel without the inverse pool; the pool gets what
// is left of the 160 KB (up to kPoolWant doubles).
static int leaf_lds_base_bytes(int D, const int* bmax) {
    int cap = 1, tsum = 0, isum = 0, psum = 0, emax = 2;
    for (int mu = 0; mu < D; ++mu) {
        cap *= bmax[mu];
        tsum += bmax[mu] * bmax[mu];
        isum += 2 * bmax[mu] + 1;
        psum += bmax[mu];
    }
    for (int mu = 0; mu < D - 1; ++mu) emax *= bmax[mu];
    if (emax > cap) emax = cap;
    const int dbl = cap + tsum + std::max(D * emax, tsum);
    const int ints = isum + D + 11 * (psum + 1) + 2;
    return dbl * (int)sizeof(double) + cap * (int)sizeof(uint32_t) + (cap + (cap & 1)) * (int)sizeof(uint16_t) +
           ints * (int)sizeof(int);
}

int leaf_pool_doubles(int D, const int* bmax) {
    const int room = (160 * 1024 - leaf_lds_base_bytes(D, bmax)) / (int)sizeof(double);
    return std::max(0, std::min(kPoolWant, room));
}

int leaf_lds_bytes(int D, const int* bmax) {
    return leaf_lds_base_bytes(D, bmax) + leaf_pool_doubles(D, bmax) * (int)sizeof(double);
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

// LP = false: FP64 MFMA.  LP = true: operands rounded to FP32 and
// v_mfma_f32_16x16x4f32 with FP32 accumulation (the low-precision updates of
// mixed-precision refinement); its result element v of lane 16 g + j is
// D[4 g + v][j] instead of the FP64 instruction's D[4 v + g][j].
template <bool LP>
struct MfmaAcc {
    typedef double type __attribute__((ext_vector_type(4)));
};
template <>
struct MfmaAcc<true> {
    typedef float type __attribute__((ext_vector_type(4)));
};

template <bool LP>
__device__ inline int mfma_row(int v, int g) {
    return LP ? 4 * g + v : 4 * v + g;
}

template <bool LP>
__device__ inline void mfma_chunk(const double* As, const double* Bs, int wr, int wc, int li, int lk,
                                  typename MfmaAcc<LP>::type (&acc)[2][2]) {
#pragma unroll
    for (int kk = 0; kk < kKC; kk += 4) {
        const double* Ak = As + (kk + lk) * kLdsRow;
        const double* Bk = Bs + (kk + lk) * kLdsRow;
        double a0 = Ak[wr + li], a1 = Ak[wr + 16 + li];
        double b0 = Bk[wc + li], b1 = Bk[wc + 16 + li];
        if constexpr (LP) {
            const float fa0 = (float)a0, fa1 = (float)a1, fb0 = (float)b0, fb1 = (float)b1;
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa0, fb0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa0, fb1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa1, fb0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa1, fb1, acc[1][1], 0, 0, 0);
        } else {
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
}

template <bool LP>
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
    typename MfmaAcc<LP>::type acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = typename MfmaAcc<LP>::type{0, 0, 0, 0};
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
            mfma_chunk<LP>(As, Bs, wr, wc, li, lk, acc);
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
                    const int r = wr + 16 * i + mfma_row<LP>(v, lk);
                    if (row0 + r < t.M) {
                        double* p = C + coff + (int64_t)(t.r0 + row0 + r) * smu;
                        const double val = sgn * (double)acc[i][j][v];
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
            mfma_chunk<LP>(As, Bs, wr, wc, li, lk, acc);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = wr + 16 * i + mfma_row<LP>(v, lk);
                if (col0 + c >= t.P) continue;
                const int64_t coff = colOff[c];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int r = wc + 16 * j + li;
                    if (row0 + r < t.M) {
                        double* p = C + coff + t.r0 + row0 + r;
                        const double val = sgn * (double)acc[i][j][v];
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
                           bmax[0], bmax[1], bmax[2], 1, leaf_pool_doubles(3, bmax));
    } else {
        hipLaunchKernelGGL(leaf_kernel<4>, grid, block, lds_bytes, st, leaves, first, probs, status,
                           bmax[0], bmax[1], bmax[2], bmax[3], leaf_pool_doubles(4, bmax));
    }
    return hipGetLastError();
}

hipError_t launch_update(int D, const UpdDesc* tasks, const WorkItem* items, int64_t first,
                         int64_t count, const ProbDesc* probs, int lp, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (lp)
        hipLaunchKernelGGL(upd_kernel<true>, dim3((unsigned)count), dim3(kUpdThreads), 0, st, tasks, items, first,
                           probs, D);
    else
        hipLaunchKernelGGL(upd_kernel<false>, dim3((unsigned)count), dim3(kUpdThreads), 0, st, tasks, items, first,
                           probs, D);
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
