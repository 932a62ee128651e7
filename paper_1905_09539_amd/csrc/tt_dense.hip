// Dense tensor kernels around the triangular solve (gfx950, FP64 MFMA):
//   modeprod_kernel - Y = alpha (X x_mu M) + beta Z, the mode-mu product of
//                     Sec. 2 used by the Schur transforms of Algorithm 1
//                     (B x_mu U_mu^T before the solve, X x_mu U_mu after),
//                     by the C_mu^{-1} reduction of the pair form and by the
//                     FP64 residual of iterative refinement (modes of at
//                     most 16 rows: modeprod_small_kernel, one thread per
//                     fibre; large FP64 products: modeprod128_kernel);
//   gram_batched_kernel - split-K partial sums of P_(mu) Q_(mu)^T for a table
//                     of (problem, mode) jobs: the coefficient gradients
//                     -Lam_(mu) X_(mu)^T of the adjoint;
//   gram_reduce_batched_kernel, axpy, norms and precision conversions.
//
// A tensor of shape (n_1..n_d) in C order is viewed, for mode mu, as
// [L][n_mu][R] with L = prod_{nu<mu} n_nu and R = prod_{nu>mu} n_nu.
#include <algorithm>
#include "tt_bf16.h"
#include "tt_internal.h"

namespace tt {

namespace {

constexpr int kDT = 64;      // output tile edge
constexpr int kDKC = 16;     // K chunk staged through LDS
constexpr int kDRow = 80;    // LDS row pitch (doubles)
constexpr int kDThreads = 256;
static_assert(kDT == kGramTile && kDKC == kGramKC, "Gram job planning assumes the kernel's tile and K chunk");

// 2x2 blocks of 16x16x4 MFMA per wave over one K chunk.  LP = 0:
// v_mfma_f64_16x16x4f64; LP = 1: operands rounded to FP32 and
// v_mfma_f32_16x16x4f32 with FP32 accumulation; LP = 2: operands split into
// three BF16 terms and six-term products on v_mfma_f32_16x16x16_bf16 (one
// 16x16x16 step per chunk, tt_bf16.h).  Lane layout: A[i][k] from lane
// 16k + i, B[k][j] from lane 16k + j (16x16x16: lane 16 (k / 4) + i holds
// k % 4 of four); result element v of lane 16 g + j is D[4 v + g][j] (FP64)
// or D[4 g + v][j] (FP32 accumulation).
template <int LP>
struct MAcc {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct MAcc<0> {
    typedef double type __attribute__((ext_vector_type(4)));
};

template <int LP>
__device__ inline int mrow(int v, int g) {
    return LP ? 4 * g + v : 4 * v + g;
}

template <int LP>
__device__ inline void mfma_chunk16(const double* As, const double* Bs, int wr, int wc, int li, int lk,
                                    typename MAcc<LP>::type (&acc)[2][2]) {
    if constexpr (LP == 2) {
        const double* A0 = As + 4 * lk * kDRow;
        const double* B0 = Bs + 4 * lk * kDRow;
        Split4 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int r = wr + 16 * i + li, c = wc + 16 * i + li;
            a[i] = split4(A0[r], A0[kDRow + r], A0[2 * kDRow + r], A0[3 * kDRow + r]);
            b[i] = split4(B0[c], B0[kDRow + c], B0[2 * kDRow + c], B0[3 * kDRow + c]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16x6(a[i], b[j], acc[i][j]);
    } else {
#pragma unroll
        for (int kk = 0; kk < kDKC; kk += 4) {
            const double* Ak = As + (kk + lk) * kDRow;
            const double* Bk = Bs + (kk + lk) * kDRow;
            double a0 = Ak[wr + li], a1 = Ak[wr + 16 + li];
            double b0 = Bk[wc + li], b1 = Bk[wc + 16 + li];
            if constexpr (LP == 1) {
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
}

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2).
// Renumber so that every XCD works on a contiguous range of logical tiles:
// tiles that share an operand then share an L2.
__device__ inline int64_t xcd_tile(int64_t b, int64_t nblocks) {
    if (nblocks % 8 != 0) return b;
    return (b % 8) * (nblocks / 8) + b / 8;
}

}  // namespace

// ---------------------------------------------------------------------------
// Mode product.  Y[l, i, r] = alpha * sum_j M[i, j] X[l, j, r] + beta * Z[l, i, r]
// with M row-major nout x nin (ld = nin).  Z may equal Y (read before write);
// Y must not overlap X.  upper: M is upper triangular (square), so a tile
// of output rows i >= i0 starts its K loop at the chunk holding j = i0 (the
// skipped chunks hold only zeros of M; the sums are unchanged).
//   R > 1 : MFMA rows = i (M rows), columns = c = l R + r (X columns).
//   R == 1: MFMA rows = l (X rows, contiguous along j), columns = i.
// Grid: row tiles x column tiles, flattened, renumbered per XCD.
// ---------------------------------------------------------------------------
template <int LP>
__global__ __launch_bounds__(kDThreads) void modeprod_kernel(const double* __restrict__ X, double* Y,
                                                             const double* Z,
                                                             const double* __restrict__ M, int64_t L,
                                                             int nin, int nout, int64_t R, double alpha,
                                                             double beta, int upper) {
    __shared__ double As[kDKC * kDRow];
    __shared__ double Bs[kDKC * kDRow];
    __shared__ int64_t colOff[kDT];
    const int tid = threadIdx.x;
    const bool colpath = R > 1;
    const int64_t rows = colpath ? nout : L;
    const int64_t cols = colpath ? L * R : nout;
    const int64_t nrt = (rows + kDT - 1) / kDT;
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t row0 = (t % nrt) * kDT;
    const int64_t col0 = (t / nrt) * kDT;
    const int K = nin;

    const int lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    typename MAcc<LP>::type acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = typename MAcc<LP>::type{0, 0, 0, 0};
    const int nchunk = (K + kDKC - 1) / kDKC;
    // first K chunk: output rows of M start at row0 (R > 1) or col0 (R == 1)
    const int ch0 = upper ? (int)min<int64_t>((colpath ? row0 : col0) / kDKC, nchunk) : 0;

    if (colpath) {
        if (tid < kDT) {
            int64_t c = col0 + tid;
            int64_t l = c / R, r = c - (c / R) * R;
            colOff[tid] = (c < cols) ? l * (int64_t)nin * R + r : 0;
        }
        __syncthreads();
        const int la_r = tid >> 2, la_k = (tid & 3) * 4;
        const int lb_k = tid >> 4, lb_c = (tid & 15) * 4;
        double ra[4], rb[4];
        int64_t boff[4];
        bool bval[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            boff[i] = colOff[lb_c + i];
            bval[i] = (col0 + lb_c + i) < cols;
        }
        const bool aval = (row0 + la_r) < rows;
        const double* Arow = M + (row0 + la_r) * (int64_t)nin;
        auto gload = [&](int kc) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int k = kc + la_k + i;
                ra[i] = (aval && k < K) ? Arow[k] : 0.0;
            }
            int kb = kc + lb_k;
            bool kv = kb < K;
            int64_t roff = (int64_t)kb * R;
#pragma unroll
            for (int i = 0; i < 4; ++i) rb[i] = (kv && bval[i]) ? X[boff[i] + roff] : 0.0;
        };
        gload(ch0 * kDKC);
        for (int ch = ch0; ch < nchunk; ++ch) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 4; ++i) As[(la_k + i) * kDRow + la_r] = ra[i];
#pragma unroll
            for (int i = 0; i < 4; ++i) Bs[lb_k * kDRow + lb_c + i] = rb[i];
            __syncthreads();
            if (ch + 1 < nchunk) gload((ch + 1) * kDKC);
            mfma_chunk16<LP>(As, Bs, wr, wc, li, lk, acc);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = wc + 16 * j + li;
            if (col0 + c >= cols) continue;
            const int64_t c64 = col0 + c;
            const int64_t l = c64 / R, r = c64 - l * R;
            const int64_t obase = l * (int64_t)nout * R + r;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = row0 + wr + 16 * i + mrow<LP>(v, lk);
                    if (row < rows) {
                        const int64_t o = obase + row * R;
                        double val = alpha * (double)acc[i][j][v];
                        if (beta != 0.0) val += beta * Z[o];
                        Y[o] = val;
                    }
                }
        }
    } else {
        // rows l (X[l][0..nin)), columns i (M[i][0..nin)), both contiguous in k
        const int lr = tid >> 2, lk4 = (tid & 3) * 4;
        const bool xv = (row0 + lr) < rows;
        const bool mv = (col0 + lr) < cols;
        const double* Xrow = X + (row0 + lr) * (int64_t)nin;
        const double* Mrow = M + (col0 + lr) * (int64_t)nin;
        double ra[4], rb[4];
        auto gload = [&](int kc) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int k = kc + lk4 + i;
                ra[i] = (xv && k < K) ? Xrow[k] : 0.0;
                rb[i] = (mv && k < K) ? Mrow[k] : 0.0;
            }
        };
        gload(ch0 * kDKC);
        for (int ch = ch0; ch < nchunk; ++ch) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                As[(lk4 + i) * kDRow + lr] = ra[i];
                Bs[(lk4 + i) * kDRow + lr] = rb[i];
            }
            __syncthreads();
            if (ch + 1 < nchunk) gload((ch + 1) * kDKC);
            mfma_chunk16<LP>(As, Bs, wr, wc, li, lk, acc);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t l = row0 + wr + 16 * i + mrow<LP>(v, lk);
                if (l >= rows) continue;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int64_t col = col0 + wc + 16 * j + li;
                    if (col < cols) {
                        const int64_t o = l * nout + col;
                        double val = alpha * (double)acc[i][j][v];
                        if (beta != 0.0) val += beta * Z[o];
                        Y[o] = val;
                    }
                }
            }
    }
}

// ---------------------------------------------------------------------------
// Split-K Gram product of two tensors of the same shape [L][n][R]:
//   W[s][a][b] = sum_{k in chunk s} P[a, k] Q[b, k],  k = l R + r,
// P[a, k] = P[l n R + a R + r].  One workgroup per (a tile, b tile, chunk);
// the batched kernel maps its workgroups to jobs through their wg_first.
// ---------------------------------------------------------------------------
__device__ inline void gram_block(const gdouble* __restrict__ P, const gdouble* __restrict__ Q,
                                  gdouble* __restrict__ W, int n, int64_t L, int64_t R, int64_t kchunk, int a0,
                                  int b0, int s) {
    __shared__ double As[kDKC * kDRow];
    __shared__ double Bs[kDKC * kDRow];
    __shared__ int64_t kOff[kDKC];
    const int tid = threadIdx.x;
    const int64_t K = L * R;
    const int64_t kbeg = (int64_t)s * kchunk;
    const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
    const int64_t nR = (int64_t)n * R;

    const int lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    MAcc<false>::type acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = MAcc<false>::type{0.0, 0.0, 0.0, 0.0};

    if (R > 1) {
        // thread: row a = tid / 4 (of both tiles), 4 consecutive k
        const int ar = tid >> 2, ak = (tid & 3) * 4;
        const bool pa = (a0 + ar) < n, qb = (b0 + ar) < n;
        const gdouble* Pr = P + (int64_t)(a0 + ar) * R;
        const gdouble* Qr = Q + (int64_t)(b0 + ar) * R;
        double ra[4], rb[4];
        for (int64_t kc = kbeg; kc < kend; kc += kDKC) {
            __syncthreads();
            if (tid < kDKC) {
                int64_t k = kc + tid;
                int64_t l = k / R;
                kOff[tid] = (k < kend) ? l * nR + (k - l * R) : -1;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t o = kOff[ak + i];
                ra[i] = (pa && o >= 0) ? Pr[o] : 0.0;
                rb[i] = (qb && o >= 0) ? Qr[o] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                As[(ak + i) * kDRow + ar] = ra[i];
                Bs[(ak + i) * kDRow + ar] = rb[i];
            }
            __syncthreads();
            mfma_chunk16<false>(As, Bs, wr, wc, li, lk, acc);
        }
    } else {
        // R == 1: P[l][a], contiguous along a; thread: k = tid / 16, 4 consecutive a
        const int kk = tid >> 4, ac = (tid & 15) * 4;
        double ra[4], rb[4];
        for (int64_t kc = kbeg; kc < kend; kc += kDKC) {
            const int64_t k = kc + kk;
            const bool kv = k < kend;
            const gdouble* Pr = P + k * n;
            const gdouble* Qr = Q + k * n;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ra[i] = (kv && a0 + ac + i < n) ? Pr[a0 + ac + i] : 0.0;
                rb[i] = (kv && b0 + ac + i < n) ? Qr[b0 + ac + i] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                As[kk * kDRow + ac + i] = ra[i];
                Bs[kk * kDRow + ac + i] = rb[i];
            }
            __syncthreads();
            mfma_chunk16<false>(As, Bs, wr, wc, li, lk, acc);
        }
    }
    gdouble* Ws = W + (int64_t)s * n * n;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int a = a0 + wr + 16 * i + mrow<false>(v, lk);
            if (a >= n) continue;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int b = b0 + wc + 16 * j + li;
                if (b < n) Ws[(int64_t)a * n + b] = acc[i][j][v];
            }
        }
}

// the last job whose range starts at or before idx (ranges ascending)
template <bool EL>
__device__ inline int gram_job_of(const GramJob* __restrict__ jobs, int njobs, int64_t idx) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((EL ? jobs[mid].el_first : jobs[mid].wg_first) <= idx)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kDThreads) void gram_batched_kernel(const GramJob* __restrict__ jobs, int njobs) {
    const GramJob& J = jobs[gram_job_of<false>(jobs, njobs, blockIdx.x)];
    const int64_t b = (int64_t)blockIdx.x - J.wg_first;
    const int nt = (J.n + kDT - 1) / kDT;
    const int tile = (int)(b % (nt * nt)), s = (int)(b / (nt * nt));
    gram_block(to_global(J.P), to_global(J.Q), to_global(J.W), J.n, J.L, J.R, J.kchunk, (tile % nt) * kDT, (tile / nt) * kDT, s);
}

__global__ void gram_reduce_batched_kernel(const GramJob* __restrict__ jobs, int njobs, int64_t elems,
                                           double scale) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < elems;
         g += (int64_t)gridDim.x * blockDim.x) {
        const GramJob& J = jobs[gram_job_of<true>(jobs, njobs, g)];
        const int64_t e = g - J.el_first, nn = (int64_t)J.n * J.n;
        const int a = (int)(e / J.n), b = (int)(e - (e / J.n) * J.n);
        const bool keep = J.dense || a <= b || (a == b + 1 && to_global(J.T)[e] != 0.0);
        const gdouble* W = to_global(J.W);
        double acc = 0.0;
        if (keep)
            for (int s = 0; s < J.nsplit; ++s) acc += W[(int64_t)s * nn + e];
        to_global(J.out)[e] = keep ? scale * acc : 0.0;
    }
}

__global__ void axpy_kernel(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

// Per-block partial sums of squares of x and of y (deterministic order).
__global__ void sumsq2_kernel(const double* __restrict__ x, const double* __restrict__ y, int64_t n,
                              double* __restrict__ part) {
    __shared__ double sx[256], sy[256];
    double ax = 0.0, ay = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double a = x[i], b = y ? y[i] : 0.0;
        ax += a * a;
        ay += b * b;
    }
    sx[threadIdx.x] = ax;
    sy[threadIdx.x] = ay;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sx[threadIdx.x] += sx[threadIdx.x + w];
            sy[threadIdx.x] += sy[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sx[0];
        part[2 * blockIdx.x + 1] = sy[0];
    }
}

__global__ void f64_to_f32_kernel(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}

__global__ void f32_to_f64_kernel(const float* __restrict__ x, double* __restrict__ y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}

// ---------------------------------------------------------------------------
// The same mode product on 128x128 tiles (FP64): four waves of 64x64, each
// 4x4 MFMA 16x16x4 blocks, so every K chunk staged through LDS feeds four
// times the MFMA work of the 64x64 tile for the same two barriers, and each
// operand element read from memory serves twice as many products.  Used for
// large products (the dense transforms and the refinement residuals).
// ---------------------------------------------------------------------------
constexpr int kBT = 128;    // tile edge
constexpr int kBRow = 144;  // LDS row pitch (doubles): the two K rows a half-wave reads fall in disjoint bank halves

__global__ __launch_bounds__(kDThreads) __attribute__((amdgpu_waves_per_eu(2))) void modeprod128_kernel(const double* __restrict__ X, double* Y,
                                                                const double* Z, const double* __restrict__ M,
                                                                int64_t L, int nin, int nout, int64_t R,
                                                                double alpha, double beta, int upper) {
    __shared__ double As[kDKC * kBRow];
    __shared__ double Bs[kDKC * kBRow];
    __shared__ int64_t colOff[kBT];
    const int tid = threadIdx.x;
    const bool colpath = R > 1;
    const int64_t rows = colpath ? nout : L;
    const int64_t cols = colpath ? L * R : nout;
    const int64_t nrt = (rows + kBT - 1) / kBT;
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t row0 = (t % nrt) * kBT;
    const int64_t col0 = (t / nrt) * kBT;
    const int K = nin;
    const int nchunk = (K + kDKC - 1) / kDKC;
    const int ch0 = upper ? (int)min<int64_t>((colpath ? row0 : col0) / kDKC, nchunk) : 0;

    const int lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const int li = lane & 15, lk = lane >> 4;
    MAcc<0>::type acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = MAcc<0>::type{0.0, 0.0, 0.0, 0.0};

    // loaders: A rows (contiguous along K) as 128 rows x 16: row tid / 2,
    // eight consecutive K from (tid % 2) * 8; B as 16 x 128 (colpath: one
    // column per lane, K rows 8 * (tid / 128) ..; rowpath: like A)
    const int ar = tid >> 1, ak = (tid & 1) * 8;
    const int bc = tid & 127, bk = (tid >> 7) * 8;
    double ra[8], rb[8];
    const bool aval = colpath ? (row0 + ar) < rows : (row0 + ar) < rows;
    const double* Arow = colpath ? M + (row0 + ar) * (int64_t)nin : X + (row0 + ar) * (int64_t)nin;
    const bool bval = colpath ? (col0 + bc) < cols : (col0 + ar) < cols;
    const double* Brow = colpath ? nullptr : M + (col0 + ar) * (int64_t)nin;
    if (colpath && tid < kBT) {
        const int64_t c = col0 + tid;
        const int64_t l = c / R, r = c - (c / R) * R;
        colOff[tid] = (c < cols) ? l * (int64_t)nin * R + r : 0;
    }
    __syncthreads();
    const int64_t boff = colpath ? colOff[bc] : 0;
    auto gload = [&](int kc) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = kc + ak + i;
            ra[i] = (aval && k < K) ? Arow[k] : 0.0;
        }
        if (colpath) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = kc + bk + i;
                rb[i] = (bval && k < K) ? X[boff + (int64_t)k * R] : 0.0;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = kc + ak + i;
                rb[i] = (bval && k < K) ? Brow[k] : 0.0;
            }
        }
    };
    gload(ch0 * kDKC);
    for (int ch = ch0; ch < nchunk; ++ch) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 8; ++i) As[(ak + i) * kBRow + ar] = ra[i];
        if (colpath) {
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[(bk + i) * kBRow + bc] = rb[i];
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[(ak + i) * kBRow + ar] = rb[i];
        }
        __syncthreads();
        if (ch + 1 < nchunk) gload((ch + 1) * kDKC);
#pragma unroll
        for (int kk = 0; kk < kDKC; kk += 4) {
            const double* Ak = As + (kk + lk) * kBRow + wr + li;
            const double* Bk = Bs + (kk + lk) * kBRow + wc + li;
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = Ak[16 * i];
                b[i] = Bk[16 * i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    // D[i][j] of a block: element v of lane 16 g + j holds row 4 v + g
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t col = col0 + wc + 16 * j + li;
        if (col >= cols) continue;
        int64_t obase = 0, rstride = 1;
        if (colpath) {
            const int64_t l = col / R, r = col - l * R;
            obase = l * (int64_t)nout * R + r;
            rstride = R;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = row0 + wr + 16 * i + 4 * v + lk;
                if (row >= rows) continue;
                const int64_t o = colpath ? obase + row * rstride : row * nout + col;
                double val = alpha * acc[i][j][v];
                if (beta != 0.0) val += beta * Z[o];
                Y[o] = val;
            }
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static unsigned elem_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    return (unsigned)b;
}

// Mode product of a small mode (nin, nout <= 16), FP64: one thread per fibre
// (l, r) keeps its nin inputs in registers and forms its nout outputs from M
// in LDS.  An 8-row mode would fill an eighth of a 64-row MFMA tile; here
// the pass is bound by HBM (each element read and written once), and
// consecutive threads take consecutive r, so every load and store of a
// wave is contiguous when R > 1 (R = 1: staged through LDS).  256 threads.
constexpr int kSmallMode = 16;
__global__ __launch_bounds__(256) void modeprod_small_kernel(const double* __restrict__ X, double* Y,
                                                             const double* Z, const double* __restrict__ M,
                                                             int64_t L, int nin, int nout, int64_t R,
                                                             double alpha, double beta) {
    __shared__ double Ms[kSmallMode * kSmallMode];
    for (int e = threadIdx.x; e < nout * nin; e += blockDim.x) Ms[e] = M[e];
    __syncthreads();
    if (R == 1) {  // uniform
        // the last mode: fibres are contiguous runs of nin (nout) values, so
        // 256 fibres go through LDS and the global loads and stores of a
        // wave stay contiguous
        __shared__ double buf[256 * kSmallMode];
        const int tid = threadIdx.x;
        for (int64_t f0 = (int64_t)blockIdx.x * 256; f0 < L; f0 += (int64_t)gridDim.x * 256) {
            const int nfb = (int)min((int64_t)256, L - f0);
            const double* xb = X + f0 * nin;
            for (int e = tid; e < nfb * nin; e += 256) buf[e] = xb[e];
            __syncthreads();
            double xv[kSmallMode];
#pragma unroll
            for (int k = 0; k < kSmallMode; ++k) xv[k] = (k < nin && tid < nfb) ? buf[tid * nin + min(k, nin - 1)] : 0.0;
            __syncthreads();
            if (tid < nfb)
                for (int i = 0; i < nout; ++i) {
                    double acc = 0.0;
#pragma unroll
                    for (int k = 0; k < kSmallMode; ++k)
                        if (k < nin) acc = fma(Ms[i * nin + k], xv[k], acc);
                    buf[tid * nout + i] = alpha * acc;
                }
            __syncthreads();
            const int64_t yb = f0 * nout;
            for (int e = tid; e < nfb * nout; e += 256) {
                double val = buf[e];
                if (beta != 0.0) val += beta * Z[yb + e];
                Y[yb + e] = val;
            }
            __syncthreads();
        }
        return;
    }
    const int64_t nf = L * R;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = f / R, r = f - l * R;
        const double* x = X + l * nin * R + r;
        double xv[kSmallMode];
#pragma unroll
        for (int k = 0; k < kSmallMode; ++k) xv[k] = (k < nin) ? x[(int64_t)min(k, nin - 1) * R] : 0.0;
        const int64_t ob = l * nout * R + r;
        for (int i = 0; i < nout; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < kSmallMode; ++k)
                if (k < nin) acc = fma(Ms[i * nin + k], xv[k], acc);
            double val = alpha * acc;
            if (beta != 0.0) val += beta * Z[ob + i * R];
            Y[ob + i * R] = val;
        }
    }
}

hipError_t launch_modeprod(const double* X, double* Y, const double* Z, const double* M, int64_t L, int nin,
                           int nout, int64_t R, double alpha, double beta, int lp, hipStream_t st, bool upper) {
    if (L <= 0 || R <= 0 || nout <= 0) return hipSuccess;
    if (lp == 0 && nin <= kSmallMode && nout <= kSmallMode) {
        const int64_t blocks = std::min<int64_t>((L * R + 255) / 256, 8192);
        hipLaunchKernelGGL(modeprod_small_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, Y, Z, M, L, nin,
                           nout, R, alpha, beta);
        return hipGetLastError();
    }
    const int64_t rows = (R > 1) ? nout : L;
    const int64_t cols = (R > 1) ? L * R : nout;
    const int64_t tiles = ((rows + kDT - 1) / kDT) * ((cols + kDT - 1) / kDT);
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    const int64_t tiles128 = ((rows + kBT - 1) / kBT) * ((cols + kBT - 1) / kBT);
    if (lp == 0 && rows >= kBT && cols >= kBT && tiles128 >= 1024) {
        hipLaunchKernelGGL(modeprod128_kernel, dim3((unsigned)tiles128), dim3(kDThreads), 0, st, X, Y, Z, M, L, nin,
                           nout, R, alpha, beta, upper && nin == nout ? 1 : 0);
        return hipGetLastError();
    }
    if (lp == 2)
        hipLaunchKernelGGL(modeprod_kernel<2>, dim3((unsigned)tiles), dim3(kDThreads), 0, st, X, Y, Z, M, L, nin,
                           nout, R, alpha, beta, upper && nin == nout ? 1 : 0);
    else if (lp == 1)
        hipLaunchKernelGGL(modeprod_kernel<1>, dim3((unsigned)tiles), dim3(kDThreads), 0, st, X, Y, Z, M, L, nin,
                           nout, R, alpha, beta, upper && nin == nout ? 1 : 0);
    else
        hipLaunchKernelGGL(modeprod_kernel<0>, dim3((unsigned)tiles), dim3(kDThreads), 0, st, X, Y, Z, M, L, nin,
                           nout, R, alpha, beta, upper && nin == nout ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_gram_batched(const GramJob* jobs, int njobs, int64_t wgs, int64_t elems, double scale,
                               hipStream_t st) {
    if (njobs <= 0 || wgs <= 0) return hipSuccess;
    hipLaunchKernelGGL(gram_batched_kernel, dim3((unsigned)wgs), dim3(kDThreads), 0, st, jobs, njobs);
    hipLaunchKernelGGL(gram_reduce_batched_kernel, dim3(elem_grid(elems)), dim3(256), 0, st, jobs, njobs, elems,
                       scale);
    return hipGetLastError();
}

hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(axpy_kernel, dim3(elem_grid(n)), dim3(256), 0, st, y, x, a, n);
    return hipGetLastError();
}

int sumsq_blocks() { return 512; }

hipError_t launch_sumsq2(const double* x, const double* y, int64_t n, double* part, hipStream_t st) {
    hipLaunchKernelGGL(sumsq2_kernel, dim3(sumsq_blocks()), dim3(256), 0, st, x, y, n, part);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double* x, float* y, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(f64_to_f32_kernel, dim3(elem_grid(n)), dim3(256), 0, st, x, y, n);
    return hipGetLastError();
}

hipError_t launch_f32_to_f64(const float* x, double* y, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(f32_to_f64_kernel, dim3(elem_grid(n)), dim3(256), 0, st, x, y, n);
    return hipGetLastError();
}

}  // namespace tt
