// gfx950 kernels of the triangular Kronecker solve (the leaf solve is in
// tt_leaf.hip).
//
//   upd_kernel    - the right-hand-side update of Algorithm 2,
//                   B_1 <- B_1 - X_2 x_mu A_mu(1:k, k+1:n_mu), for one pencil,
//                   on FP64 MFMA (v_mfma_f64_16x16x4f64).
#include <algorithm>

#include "tt_bf16.h"
#include "tt_internal.h"

namespace tt {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Update kernel: one workgroup per output tile of one pencil update of the
// recursion (Algorithm 2's B_1 <- B_1 - X_2 x_mu A_mu(1:k, k+1:n_mu)):
//   C[r, c] (+)= sum_k A[r, k] * Bx[k, c]
// with A = T_mu[r0 + r, k0 + k], Bx[k, c] = X[col_off(c) + (k0 + k) s_mu],
// and C[r, c] the target element at col_off(c) + (r0 + r) s_mu: X itself for
// mode 0 (subtract), the accumulator of mode mu otherwise (add, or store for
// the first contribution).  A 64x64 tile is four 32x32 wave tiles of 2x2
// MFMA 16x16x4 FP64 blocks (tasks with more than 64 target rows: 128 x 64
// tiles, two such blocks per wave; 17 to 32 target rows: 32 x 128 tiles; at
// most 16 target rows: 16 x 256 tiles);
// K advances in chunks of 16 staged through LDS.
// For the fastest mode (s_mu = 1) the roles are transposed so that the
// contiguous index runs along the MFMA columns.
//
// v_mfma_f64_16x16x4f64 lane layout (gfx950): A[i][k] from lane 16k + i,
// B[k][j] from lane 16k + j, D[i][j] in lane 16 (i % 4) + j, element i / 4.
// ---------------------------------------------------------------------------
constexpr int kKC = 16;      // K chunk
constexpr int kLdsRow = 80;  // 64 + 16 doubles: rows k and k+1 use disjoint bank halves
constexpr int kWideTDoubles = kKC * 17;                 // wide tile: 16 x 17 T block
constexpr int kWideDoubles = kWideTDoubles + kKC * (4 * 64 + 16);  // plus 16 x 272 pencil block
constexpr int kUpdSmemDoubles = (kWideDoubles > 2 * kKC * kLdsRow) ? kWideDoubles : 2 * kKC * kLdsRow;

// Operand loads of the update kernel are never skipped: a lane whose element
// lies outside the tile reads this zero instead.  A masked load (select after
// a load) is turned back into a branch around the load by the compiler, with
// a wait for the load inside the branch; a load from a selected address stays
// unconditional, so the loads of the next chunks remain in flight.
__device__ double kZeroOperand[2];

__device__ inline const gdouble* pick(bool valid, const gdouble* p) {
    return valid ? p : (const gdouble*)to_global(&kZeroOperand[0]);
}

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

// LP = 0: FP64 MFMA.  LP = 1: operands rounded to FP32 and
// v_mfma_f32_16x16x4f32 with FP32 accumulation; LP = 2: operands split into
// three BF16 terms, six-term products on v_mfma_f32_16x16x16_bf16 with FP32
// accumulation (tt_bf16.h).  LP 1 and 2 are the low-precision updates of
// mixed-precision refinement; their result element v of lane 16 g + j is
// D[4 g + v][j] instead of the FP64 instruction's D[4 v + g][j].
template <int LP>
struct MfmaAcc {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct MfmaAcc<0> {
    typedef double type __attribute__((ext_vector_type(4)));
};

template <int LP>
__device__ inline int mfma_row(int v, int g) {
    return LP ? 4 * g + v : 4 * v + g;
}

// One K chunk of a 64x64 tile: each wave's 32x32 block as 2x2 MFMA 16x16x4
// blocks, operands from LDS.  An operand is staged either as [k][row] with
// pitch KP (kLdsRow for 64-wide blocks) or (ARK / BRK) as [row][k] with
// pitch kRkRow (odd, so the sixteen rows a lane group reads fall in
// distinct banks).
constexpr int kRkRow = kKC + 1;
template <int LP, bool ARK, bool BRK, int KP = kLdsRow>
__device__ inline void mfma_chunk_l(const double* As, const double* Bs, int wr, int wc, int li, int lk,
                                    typename MfmaAcc<LP>::type (&acc)[2][2]) {
    if constexpr (LP == 2) {
        // one 16x16x16 step: this lane's K values are 4 lk .. 4 lk + 3
        auto A = [&](int r, int k) { return ARK ? As[r * kRkRow + k] : As[k * KP + r]; };
        auto B = [&](int c, int k) { return BRK ? Bs[c * kRkRow + k] : Bs[k * KP + c]; };
        const int k0 = 4 * lk;
        Split4 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int r = wr + 16 * i + li, c = wc + 16 * i + li;
            a[i] = split4(A(r, k0), A(r, k0 + 1), A(r, k0 + 2), A(r, k0 + 3));
            b[i] = split4(B(c, k0), B(c, k0 + 1), B(c, k0 + 2), B(c, k0 + 3));
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16x6(a[i], b[j], acc[i][j]);
    } else {
#pragma unroll
    for (int kk = 0; kk < kKC; kk += 4) {
        const int k = kk + lk;
        const double a0 = ARK ? As[(wr + li) * kRkRow + k] : As[k * KP + wr + li];
        const double a1 = ARK ? As[(wr + 16 + li) * kRkRow + k] : As[k * KP + wr + 16 + li];
        const double b0 = BRK ? Bs[(wc + li) * kRkRow + k] : Bs[k * KP + wc + li];
        const double b1 = BRK ? Bs[(wc + 16 + li) * kRkRow + k] : Bs[k * KP + wc + 16 + li];
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

// K loop over nchunk chunks with two register sets of operands in flight:
// chunk c is computed while chunks c+1 and c+2 load.  load(set, k) fills a
// set from K offset k, stage(set) moves it to LDS, compute() consumes LDS.
// The steady state has no conditional load, so the wait before each stage
// leaves the other set's loads outstanding; the last one to three chunks
// are peeled.
template <class Load, class Stage, class Compute>
__device__ inline void k_pipeline(int nchunk, Load&& load, Stage&& stage, Compute&& compute) {
    load(0, 0);
    load(1, min(1, nchunk - 1) * kKC);  // a repeated chunk 0 when nchunk == 1
    int ch = 0;
    for (; ch + 3 < nchunk; ch += 2) {
        stage(0);
        load(0, (ch + 2) * kKC);
        compute();
        stage(1);
        load(1, (ch + 3) * kKC);
        compute();
    }
    stage(0);
    if (ch + 2 < nchunk) load(0, (ch + 2) * kKC);
    compute();
    if (ch + 1 < nchunk) {
        stage(1);
        compute();
    }
    if (ch + 2 < nchunk) {
        stage(0);
        compute();
    }
}

// The same K loop with one chunk in flight (set 0 only), for tiles whose
// accumulators leave no registers for a second set.
template <class Load, class Stage, class Compute>
__device__ inline void k_single(int nchunk, Load&& load, Stage&& stage, Compute&& compute) {
    load(0, 0);
    for (int ch = 0; ch < nchunk; ++ch) {
        stage(0);
        if (ch + 1 < nchunk) load(0, (ch + 1) * kKC);
        compute();
    }
}

// Wide tile for updates with at most 16 target rows (the 64x64 tile would
// leave 3/4 of its MFMA rows idle): 16 target rows x 256 pencil columns, each
// wave a 16 x 64 strip of four 16x16 MFMA blocks.  Left path: MFMA rows are
// the target rows; right path (fastest mode): MFMA rows are pencil columns.
// Pencils of at most 128 (64) columns share a tile: tasks wi.task ..
// wi.task + wi.tb, which differ only in their pencil, each own a slot of 128
// (64) columns.  colOff holds -1 for a column outside every pencil.
template <int LP>
__device__ inline void upd_wide(const UpdDesc* __restrict__ tasks, const UpdDesc& t, const WorkItem& wi,
                                const gdouble* __restrict__ X, gdouble* __restrict__ C,
                                const gdouble* __restrict__ T, int64_t nmu, int64_t smu, bool right, bool store,
                                const gdouble* B0, double sgn, double* As, double* Bs, int64_t* colOff) {
    constexpr int kW = 4 * kTile;   // 256 pencil columns
    constexpr int kWRow = kW + 16;  // LDS row pitch of the 256-wide operand
    constexpr int kTRow = 17;       // LDS pitch of the 16x16 T block (odd: conflict-free staging)
    const int tid = threadIdx.x;
    const int col0 = wi.ta * kW;
    const int g = upd_wide_slots(t.P);  // uniform
    if (g == 1) {
        colOff[tid] = (col0 + tid < t.P) ? pencil_col_offset(t, col0 + tid) : -1;
    } else {
        // column tid: slot tid >> sh, column tid & (2^sh - 1) of that slot's pencil
        const int sh = (g == 4) ? 6 : 7;
        const int slot = tid >> sh, c = tid & ((1 << sh) - 1);
        const UpdDesc& ts = tasks[wi.task + min(slot, (int)wi.tb)];  // a task of the tile in any case
        colOff[tid] = (slot <= wi.tb && c < t.P) ? pencil_col_offset(ts, c) : -1;
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    typename MfmaAcc<LP>::type acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = typename MfmaAcc<LP>::type{0, 0, 0, 0};
    const int nchunk = (t.K + kKC - 1) / kKC;
    // loaders: one value of the 16x16 T block and one pencil column (16
    // values along K) per thread
    const int tr = tid >> 4, tk = tid & 15;
    const bool tval = tr < t.M;
    const gdouble* Trow = T + (int64_t)(t.r0 + tr) * nmu + t.k0;
    const int64_t coff = colOff[tid];
    const bool cval = coff >= 0;
    // right path (fastest mode): the K run of a column is contiguous, so
    // eight lanes share one column (two doubles each, one 128-byte line per
    // eight lanes) and the block is staged as [c][k] with an odd pitch;
    // thread tid takes columns j * 32 + tid / 8, K pair tid % 8
    constexpr int kCRow = kKC + 1;
    const int rk = 2 * (tid & 7);
    double ra, rb[kKC];  // one chunk in flight
    auto gload = [&](double& ra, double (&rb)[kKC], int kc) {
        ra = *pick(tval && kc + tk < t.K, Trow + kc + tk);
        if (!right) {
#pragma unroll
            for (int k = 0; k < kKC; ++k)
                rb[k] = *pick(cval && kc + k < t.K, X + coff + (int64_t)(t.k0 + kc + k) * smu);
        } else {
#pragma unroll
            for (int j = 0; j < kKC / 2; ++j) {
                const int c = j * 32 + (tid >> 3);
                const bool cv = colOff[c] >= 0;
                const gdouble* xr = X + colOff[c] + t.k0 + kc + rk;
                rb[2 * j] = *pick(cv && kc + rk < t.K, xr);
                rb[2 * j + 1] = *pick(cv && kc + rk + 1 < t.K, xr + 1);
            }
        }
    };
    auto stage = [&](double ra, const double (&rb)[kKC]) {
        __syncthreads();
        As[tk * kTRow + tr] = ra;  // T block as [k][r]
        if (!right) {
#pragma unroll
            for (int k = 0; k < kKC; ++k) Bs[k * kWRow + tid] = rb[k];  // pencil data as [k][c]
        } else {
#pragma unroll
            for (int j = 0; j < kKC / 2; ++j) {  // pencil data as [c][k]
                double* d = Bs + (j * 32 + (tid >> 3)) * kCRow + rk;
                d[0] = rb[2 * j];
                d[1] = rb[2 * j + 1];
            }
        }
        __syncthreads();
    };
    auto compute = [&]() {
        if constexpr (LP == 2) {
            // one 16x16x16 step per block: K values 4 lk .. 4 lk + 3 of this lane
            const int k0 = 4 * lk;
            const Split4 ts = split4(As[k0 * kTRow + li], As[(k0 + 1) * kTRow + li], As[(k0 + 2) * kTRow + li],
                                     As[(k0 + 3) * kTRow + li]);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = wave * 64 + b * 16 + li;
                auto xv = [&](int k) { return right ? Bs[c * kCRow + k] : Bs[k * kWRow + c]; };
                const Split4 xs = split4(xv(k0), xv(k0 + 1), xv(k0 + 2), xv(k0 + 3));
                acc[b] = right ? mfma_bf16x6(xs, ts, acc[b]) : mfma_bf16x6(ts, xs, acc[b]);
            }
        } else {
#pragma unroll
        for (int kk = 0; kk < kKC; kk += 4) {
            const double tv = As[(kk + lk) * kTRow + li];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = wave * 64 + b * 16 + li;
                const double xv = right ? Bs[c * kCRow + kk + lk] : Bs[(kk + lk) * kWRow + c];
                if constexpr (LP == 1) {
                    const float ft = (float)tv, fx = (float)xv;
                    acc[b] = right ? __builtin_amdgcn_mfma_f32_16x16x4f32(fx, ft, acc[b], 0, 0, 0)
                                   : __builtin_amdgcn_mfma_f32_16x16x4f32(ft, fx, acc[b], 0, 0, 0);
                } else {
                    acc[b] = right ? __builtin_amdgcn_mfma_f64_16x16x4f64(xv, tv, acc[b], 0, 0, 0)
                                   : __builtin_amdgcn_mfma_f64_16x16x4f64(tv, xv, acc[b], 0, 0, 0);
                }
            }
        }
        }
    };
    gload(ra, rb, 0);
    for (int ch = 0; ch < nchunk; ++ch) {
        stage(ra, rb);
        if (ch + 1 < nchunk) gload(ra, rb, (ch + 1) * kKC);
        compute();
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            // left: D[r][c] with r = mfma row, c = lane column; right: D[c][r]
            const int i = mfma_row<LP>(v, lk);
            const int c = wave * 64 + b * 16 + (right ? i : li);
            const int r = right ? li : i;
            if (colOff[c] < 0 || r >= t.M) continue;
            const int64_t o = colOff[c] + (int64_t)(t.r0 + r) * smu;
            const double val = sgn * (double)acc[b][v];
            C[o] = store ? (B0 ? B0[o] + val : val) : C[o] + val;
        }
}

// The 64-column tile path: TR = 1 gives 64x64 output tiles, TR = 2 tiles of
// 128 target rows x 64 pencil columns (tasks with more than 64 target rows:
// each source chunk staged in LDS then feeds twice the MFMA work, and a task
// re-reads its source panel half as often).  Four waves; each wave owns
// 32 TR x 32 of the tile as TR stacked 32x32 blocks of 2x2 MFMA 16x16 tiles
// (left path: stacked along the target rows, the MFMA rows; right path:
// along the target rows, the MFMA columns).
template <int LP, int TR>
__device__ inline void upd_tile(const UpdDesc& t, const WorkItem& wi, const gdouble* __restrict__ X,
                                gdouble* __restrict__ C, const gdouble* __restrict__ T, int64_t nmu, int64_t smu,
                                bool right, bool store, const gdouble* B0, double sgn, double* smem,
                                int64_t* colOff) {
    constexpr int kRows = kTile * TR;  // target rows of the tile
    // LDS: the [row][k] blocks (pitch kRkRow) of up to kRows rows and the
    // 16 x 80 [k][c] pencil block
    constexpr int kBOff = (kRows * kRkRow > kKC * kLdsRow) ? kRows * kRkRow : kKC * kLdsRow;
    static_assert(kBOff + kRows * kRkRow <= kUpdSmemDoubles && kBOff + kKC * kLdsRow <= kUpdSmemDoubles,
                  "update tile exceeds its LDS buffer");
    double* As = smem;
    double* Bs = smem + kBOff;
    const int tid = threadIdx.x;
    const int col0 = (right ? wi.ta : wi.tb) * kTile;  // pencil columns
    const int row0 = (right ? wi.tb : wi.ta) * kRows;  // target rows in mode mu

    if (tid < kTile) {
        int c = col0 + tid;
        colOff[tid] = (c < t.P) ? pencil_col_offset(t, c) : 0;
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    typename MfmaAcc<LP>::type acc[TR][2][2];
#pragma unroll
    for (int h = 0; h < TR; ++h)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[h][i][j] = typename MfmaAcc<LP>::type{0, 0, 0, 0};
    const int nchunk = (t.K + kKC - 1) / kKC;
    // two chunks in flight for 64-row tiles, one for 128-row tiles (their
    // accumulators take twice the registers)
    auto k_loop = [](int nch, auto&& load, auto&& stage, auto&& compute) {
        if constexpr (TR == 1)
            k_pipeline(nch, load, stage, compute);
        else
            k_single(nch, load, stage, compute);
    };

    if (!right) {
        // MFMA rows = target rows r, MFMA columns = pencil columns c; wave
        // rows wr .. wr + 32 TR, columns wc .. wc + 32.
        // loaders: A (T rows, contiguous along K): rows tid/8 + 32 j, K pair
        // tid%8, staged as [r][k]; B (pencil data): column tid%64 (one column
        // per lane: consecutive lanes read consecutive memory within a
        // pencil row), K rows 4*(tid/64)..+3
        const int wr = (wave >> 1) * 32 * TR, wc = (wave & 1) * 32;
        const int la_r = tid >> 3, la_k = 2 * (tid & 7);
        const int lb_c = tid & 63, lb_k = (tid >> 6) * 4;
        double ra0[4 * TR], rb0[4], ra1[4 * TR], rb1[4];  // two chunks in flight
        const bool bval = (col0 + lb_c) < t.P;
        const gdouble* Bcol = X + colOff[lb_c] + (int64_t)(t.k0 + lb_k) * smu;
        bool aval[2 * TR];
        const gdouble* Arow[2 * TR];
#pragma unroll
        for (int j = 0; j < 2 * TR; ++j) {
            aval[j] = (row0 + la_r + 32 * j) < t.M;
            Arow[j] = T + (int64_t)(t.r0 + row0 + la_r + 32 * j) * nmu + t.k0 + la_k;
        }
        auto gload = [&](double (&ra)[4 * TR], double (&rb)[4], int kc) {
#pragma unroll
            for (int j = 0; j < 2 * TR; ++j)
#pragma unroll
                for (int e = 0; e < 2; ++e) ra[2 * j + e] = *pick(aval[j] && kc + la_k + e < t.K, Arow[j] + kc + e);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                rb[i] = *pick(bval && kc + lb_k + i < t.K, Bcol + (int64_t)(kc + i) * smu);
        };
        auto stage = [&](const double (&ra)[4 * TR], const double (&rb)[4]) {
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 2 * TR; ++j)
#pragma unroll
                for (int e = 0; e < 2; ++e) As[(la_r + 32 * j) * kRkRow + la_k + e] = ra[2 * j + e];
#pragma unroll
            for (int i = 0; i < 4; ++i) Bs[(lb_k + i) * kLdsRow + lb_c] = rb[i];
            __syncthreads();
        };
        k_loop(
            nchunk, [&](int set, int kc) { set ? gload(ra1, rb1, kc) : gload(ra0, rb0, kc); },
            [&](int set) { set ? stage(ra1, rb1) : stage(ra0, rb0); },
            [&]() {
#pragma unroll
                for (int h = 0; h < TR; ++h) mfma_chunk_l<LP, true, false>(As, Bs, wr + 32 * h, wc, li, lk, acc[h]);
            });
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = wc + 16 * j + li;
            if (col0 + c >= t.P) continue;
            const int64_t coff = colOff[c];
#pragma unroll
            for (int h = 0; h < TR; ++h)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = wr + 32 * h + 16 * i + mfma_row<LP>(v, lk);
                        if (row0 + r < t.M) {
                            const int64_t o = coff + (int64_t)(t.r0 + row0 + r) * smu;
                            const double val = sgn * (double)acc[h][i][j][v];
                            C[o] = store ? (B0 ? B0[o] + val : val) : C[o] + val;
                        }
                    }
        }
    } else {
        // MFMA rows = pencil columns c, MFMA columns = target rows r; wave
        // columns wr .. wr + 32, target rows wc .. wc + 32 TR.  Both operands
        // are contiguous along K: eight lanes share a row of either block
        // (one 128-byte line per eight lanes) and the blocks are staged as
        // [row][k] with an odd pitch.  Thread tid takes rows tid / 8 + 32 j,
        // K pair tid % 8.
        const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32 * TR;
        const int lr = tid >> 3, rk = 2 * (tid & 7);
        const gdouble* Xr[2];
        const gdouble* Tr[2 * TR];
        bool cval[2], rval[2 * TR];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int q = lr + 32 * j;
            cval[j] = (col0 + q) < t.P;
            Xr[j] = X + colOff[q] + t.k0 + rk;
        }
#pragma unroll
        for (int j = 0; j < 2 * TR; ++j) {
            const int q = lr + 32 * j;
            rval[j] = (row0 + q) < t.M;
            Tr[j] = T + (int64_t)(t.r0 + row0 + q) * nmu + t.k0 + rk;
        }
        double ra0[4], rb0[4 * TR], ra1[4], rb1[4 * TR];  // two chunks in flight
        auto gload = [&](double (&ra)[4], double (&rb)[4 * TR], int kc) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const bool kv = kc + rk + e < t.K;
#pragma unroll
                for (int j = 0; j < 2; ++j) ra[2 * j + e] = *pick(cval[j] && kv, Xr[j] + kc + e);
#pragma unroll
                for (int j = 0; j < 2 * TR; ++j) rb[2 * j + e] = *pick(rval[j] && kv, Tr[j] + kc + e);
            }
        };
        auto stage = [&](const double (&ra)[4], const double (&rb)[4 * TR]) {
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 2; ++e) {
#pragma unroll
                for (int j = 0; j < 2; ++j) As[(lr + 32 * j) * kRkRow + rk + e] = ra[2 * j + e];
#pragma unroll
                for (int j = 0; j < 2 * TR; ++j) Bs[(lr + 32 * j) * kRkRow + rk + e] = rb[2 * j + e];
            }
            __syncthreads();
        };
        k_loop(
            nchunk, [&](int set, int kc) { set ? gload(ra1, rb1, kc) : gload(ra0, rb0, kc); },
            [&](int set) { set ? stage(ra1, rb1) : stage(ra0, rb0); },
            [&]() {
#pragma unroll
                for (int h = 0; h < TR; ++h) mfma_chunk_l<LP, true, true>(As, Bs, wr, wc + 32 * h, li, lk, acc[h]);
            });
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = wr + 16 * i + mfma_row<LP>(v, lk);
                if (col0 + c >= t.P) continue;
                const int64_t coff = colOff[c];
#pragma unroll
                for (int h = 0; h < TR; ++h)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int r = wc + 32 * h + 16 * j + li;
                        if (row0 + r < t.M) {
                            const int64_t o = coff + t.r0 + row0 + r;
                            const double val = sgn * (double)acc[h][i][j][v];
                            C[o] = store ? (B0 ? B0[o] + val : val) : C[o] + val;
                        }
                    }
            }
    }
}

// Flat tile for updates with 17 to 32 target rows (a 64-row tile would leave
// half or more of its MFMA rows idle): 32 target rows x 128 pencil columns,
// each wave a 32x32 block of 2x2 MFMA 16x16 blocks side by side along the
// pencil columns.  Left path: MFMA rows are the target rows, the pencil
// block is staged [k][c] at pitch kFlatRow; right path (fastest mode): MFMA
// rows are pencil columns, both blocks [row][k] at pitch kRkRow.
constexpr int kFlatCols = 2 * kTile;
constexpr int kFlatRow = kFlatCols + 16;  // rows k and k+1 in disjoint bank halves
template <int LP>
__device__ inline void upd_flat(const UpdDesc& t, const WorkItem& wi, const gdouble* __restrict__ X,
                                gdouble* __restrict__ C, const gdouble* __restrict__ T, int64_t nmu, int64_t smu,
                                bool right, bool store, const gdouble* B0, double sgn, double* smem,
                                int64_t* colOff) {
    // LDS: left  As = T block [r][k] (32 x kRkRow), Bs = pencil block [k][c] (16 x kFlatRow);
    //      right As = pencil block [c][k] (128 x kRkRow), Bs = T block [r][k] (32 x kRkRow)
    constexpr int kBOff = kFlatCols * kRkRow;  // 2176 doubles: the larger first block
    static_assert(kBOff + kKC * kFlatRow <= kUpdSmemDoubles && kBOff + 32 * kRkRow <= kUpdSmemDoubles,
                  "flat tile exceeds its LDS buffer");
    double* As = smem;
    double* Bs = smem + kBOff;
    const int tid = threadIdx.x;
    const int col0 = wi.ta * kFlatCols;  // pencil columns (the only tile index: at most 32 target rows)

    if (tid < kFlatCols) {
        const int c = col0 + tid;
        colOff[tid] = (c < t.P) ? pencil_col_offset(t, c) : 0;
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    typename MfmaAcc<LP>::type acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = typename MfmaAcc<LP>::type{0, 0, 0, 0};
    const int nchunk = (t.K + kKC - 1) / kKC;

    if (!right) {
        // loaders: T row tid / 8, K pair tid % 8; pencil column tid % 128,
        // K rows 8 (tid / 128) .. + 7
        const int la_r = tid >> 3, la_k = 2 * (tid & 7);
        const int lb_c = tid & (kFlatCols - 1), lb_k = (tid >> 7) * 8;
        const bool aval = la_r < t.M;
        const gdouble* Arow = T + (int64_t)(t.r0 + la_r) * nmu + t.k0 + la_k;
        const bool bval = (col0 + lb_c) < t.P;
        const gdouble* Bcol = X + colOff[lb_c] + (int64_t)(t.k0 + lb_k) * smu;
        double ra0[2], rb0[8], ra1[2], rb1[8];  // two chunks in flight
        auto gload = [&](double (&ra)[2], double (&rb)[8], int kc) {
#pragma unroll
            for (int e = 0; e < 2; ++e) ra[e] = *pick(aval && kc + la_k + e < t.K, Arow + kc + e);
#pragma unroll
            for (int i = 0; i < 8; ++i) rb[i] = *pick(bval && kc + lb_k + i < t.K, Bcol + (int64_t)(kc + i) * smu);
        };
        auto stage = [&](const double (&ra)[2], const double (&rb)[8]) {
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 2; ++e) As[la_r * kRkRow + la_k + e] = ra[e];
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[(lb_k + i) * kFlatRow + lb_c] = rb[i];
            __syncthreads();
        };
        const int wc = wave * 32;
        k_pipeline(
            nchunk, [&](int set, int kc) { set ? gload(ra1, rb1, kc) : gload(ra0, rb0, kc); },
            [&](int set) { set ? stage(ra1, rb1) : stage(ra0, rb0); },
            [&]() { mfma_chunk_l<LP, true, false, kFlatRow>(As, Bs, 0, wc, li, lk, acc); });
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = wc + 16 * j + li;
            if (col0 + c >= t.P) continue;
            const int64_t coff = colOff[c];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * i + mfma_row<LP>(v, lk);
                    if (r < t.M) {
                        const int64_t o = coff + (int64_t)(t.r0 + r) * smu;
                        const double val = sgn * (double)acc[i][j][v];
                        C[o] = store ? (B0 ? B0[o] + val : val) : C[o] + val;
                    }
                }
        }
    } else {
        // loaders: rows tid / 8 + 32 j of the pencil block (j < 4) and row
        // tid / 8 of the T block, K pair tid % 8 (eight lanes per row)
        const int lr = tid >> 3, rk = 2 * (tid & 7);
        const gdouble* Xr[4];
        bool cval[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = lr + 32 * j;
            cval[j] = (col0 + q) < t.P;
            Xr[j] = X + colOff[q] + t.k0 + rk;
        }
        const bool rval = lr < t.M;
        const gdouble* Tr = T + (int64_t)(t.r0 + lr) * nmu + t.k0 + rk;
        double ra0[8], rb0[2], ra1[8], rb1[2];  // two chunks in flight
        auto gload = [&](double (&ra)[8], double (&rb)[2], int kc) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const bool kv = kc + rk + e < t.K;
#pragma unroll
                for (int j = 0; j < 4; ++j) ra[2 * j + e] = *pick(cval[j] && kv, Xr[j] + kc + e);
                rb[e] = *pick(rval && kv, Tr + kc + e);
            }
        };
        auto stage = [&](const double (&ra)[8], const double (&rb)[2]) {
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 2; ++e) {
#pragma unroll
                for (int j = 0; j < 4; ++j) As[(lr + 32 * j) * kRkRow + rk + e] = ra[2 * j + e];
                Bs[lr * kRkRow + rk + e] = rb[e];
            }
            __syncthreads();
        };
        const int wr = wave * 32;
        k_pipeline(
            nchunk, [&](int set, int kc) { set ? gload(ra1, rb1, kc) : gload(ra0, rb0, kc); },
            [&](int set) { set ? stage(ra1, rb1) : stage(ra0, rb0); },
            [&]() { mfma_chunk_l<LP, true, true>(As, Bs, wr, 0, li, lk, acc); });
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = wr + 16 * i + mfma_row<LP>(v, lk);
                if (col0 + c >= t.P) continue;
                const int64_t coff = colOff[c];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int r = 16 * j + li;
                    if (r < t.M) {
                        const int64_t o = coff + t.r0 + r;
                        const double val = sgn * (double)acc[i][j][v];
                        C[o] = store ? (B0 ? B0[o] + val : val) : C[o] + val;
                    }
                }
            }
    }
}

template <int LP>
__global__ __launch_bounds__(kUpdThreads) __attribute__((amdgpu_waves_per_eu(3))) void upd_kernel(const UpdDesc* __restrict__ tasks,
                                                          const WorkItem* __restrict__ items,
                                                          int64_t first,
                                                          const ProbDesc* __restrict__ probs, int D) {
    // one LDS buffer, carved per path: 64-column tiles a 64 TR x 17 T block
    // ([r][k]) and a 16 x 80 pencil block ([k][c]; fastest mode: a 64 x 17
    // [c][k] block); wide tiles a 16 x 17 T block and a 16 x 272 pencil
    // block (fastest mode: 256 x 17)
    __shared__ double smem[kUpdSmemDoubles];
    __shared__ int64_t colOff[4 * kTile];
    const WorkItem wi = items[first + blockIdx.x];
    if (wi.task < 0) return;  // padding of the per-XCD tile layout (uniform)
    const UpdDesc t = tasks[wi.task];
    const ProbDesc& P = probs[t.prob];
    const int mode = t.mode;
    // source of the products: X, or a partial product of the second class
    const gdouble* __restrict__ X = to_global(P.S[mode]);
    gdouble* __restrict__ C = to_global((mode == 0) ? P.X : P.A[mode]);
    const gdouble* __restrict__ T = to_global(P.T[mode]);
    const int64_t nmu = P.n[mode];
    const int64_t smu = P.stride[mode];
    const bool right = (mode == D - 1);
    const bool store = (t.flags & 1) != 0;
    const double sgn = (mode == 0) ? -1.0 : 1.0;
    // the first mode-0 update of a block starts from the right-hand side B
    const gdouble* B0 = (mode == 0 && store) ? to_global(P.B) : nullptr;
    if (t.M <= 16) {  // uniform over the workgroup
        upd_wide<LP>(tasks, t, wi, X, C, T, nmu, smu, right, store, B0, sgn, smem, smem + kWideTDoubles, colOff);
        return;
    }
    // uniform; the planner sizes the task's tiles by the same rule
    if (t.M > kTile)
        upd_tile<LP, 2>(t, wi, X, C, T, nmu, smu, right, store, B0, sgn, smem, colOff);
    else if (t.M > 32)
        upd_tile<LP, 1>(t, wi, X, C, T, nmu, smu, right, store, B0, sgn, smem, colOff);
    else
        upd_flat<LP>(t, wi, X, C, T, nmu, smu, right, store, B0, sgn, smem, colOff);
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
hipError_t launch_update(int D, const UpdDesc* tasks, const WorkItem* items, int64_t first,
                         int64_t count, const ProbDesc* probs, int lp, int leaf_lds, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    // Unused LDS padding that holds the update to two workgroups per CU while
    // a leaf workgroup (leaf_lds bytes) still fits beside them: with its
    // registers alone three would fit, and leaves running concurrently would
    // find no room on the CU.
    size_t pad = 0;
    if (leaf_lds > 0) {
        int dev = 0, cu_lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cu_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess) {
            constexpr int gran = 512;  // LDS allocation unit
            constexpr int stat = (int)sizeof(double) * (kUpdSmemDoubles + 4 * kTile);  // the kernel's own
            const int leaf = (leaf_lds + gran - 1) / gran * gran;
            const int u = (cu_lds / 3 / gran + 1) * gran;  // the least of which three do not fit
            if (2 * u + leaf <= cu_lds && u > stat && u <= 64 * 1024) pad = (size_t)(u - stat);
        }
    }
    if (lp == 2)
        hipLaunchKernelGGL(upd_kernel<2>, dim3((unsigned)count), dim3(kUpdThreads), pad, st, tasks, items, first,
                           probs, D);
    else if (lp == 1)
        hipLaunchKernelGGL(upd_kernel<1>, dim3((unsigned)count), dim3(kUpdThreads), pad, st, tasks, items, first,
                           probs, D);
    else
        hipLaunchKernelGGL(upd_kernel<0>, dim3((unsigned)count), dim3(kUpdThreads), pad, st, tasks, items, first,
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
