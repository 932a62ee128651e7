// Internal declarations shared by the host planner/API (tt_api.cpp) and the
// gfx950 kernels (tt_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tt.h"

namespace tt {

constexpr int kMaxD = 4;          // internal order (d < 3 is promoted to 3)
constexpr int kLeafNT = 256;      // threads of the workgroup owning one leaf block
constexpr int kLeafNTWide = 512;  // the same for launches with at most one leaf per CU (order 4: per two CUs)
constexpr int kMaxLeaf = 24;      // largest leaf block edge
constexpr int kUpdThreads = 256;  // one workgroup per 64x64 update tile
constexpr int kTile = 64;

// Global-memory views of the pointers the kernels read from device tables.
// A pointer loaded from memory is generic to the compiler, which then emits
// flat loads and stores; a flat access counts against the LDS counter as
// well, so every wait for an LDS result would also wait for all memory loads
// in flight (no prefetch survives an LDS read).
typedef __attribute__((address_space(1))) double gdouble;
template <typename T>
__device__ inline __attribute__((address_space(1))) T* to_global(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Per-problem description as the kernels see it (device table).
struct ProbDesc {
    double* X;                   // solution; mode-0 updates accumulate into it
    const double* B;             // right-hand side (may equal X): read by the
                                 // first mode-0 update of a block, or by its
                                 // leaf when the block has none
    double* A[kMaxD];            // per-mode update accumulators (modes >= 1;
                                 // mode 0 updates go straight into X)
    const double* T[kMaxD];      // coefficients (device, row-major n x n)
    const int32_t* bst[kMaxD];   // block starts per mode (device), m+1 entries
    int64_t n[kMaxD];
    int64_t stride[kMaxD];
    // Second operator class (Sec. 3, after the exact C^{-1} reduction):
    //   X x_0 T_0 + X x_1 A_1 x_2 A_2 .. x_{D-1} A_{D-1} = B.
    // Mode-mu updates read S[mu]: X for mode 0 and 1, the partial products
    // W[mu-1] for mu >= 2, where W[k] (k = 1 .. D-2), written by each leaf,
    // holds sum over j_1 >= i_1 .. j_k >= i_k of A_1[i_1, j_1] .. A_k[i_k, j_k]
    // X[i_0, j_1 .. j_k, i_{k+1} ..] (block-wise: the leaf's diagonal blocks
    // applied to its solution plus the accumulator of that mode).  The
    // Laplace-like form reads X in every mode.
    const double* S[kMaxD];
    double* W[kMaxD];
    int32_t cls;                 // 0: Laplace-like, 1: second class
    int32_t pad_;
};

// One leaf block: problem index and block coordinates.
struct LeafDesc {
    int32_t prob;
    int16_t blk[kMaxD];
    int32_t flags;               // bit 0: the block's right-hand side is in X
                                 // (it received mode-0 updates), else in B;
                                 // bit mu >= 1: subtract accumulator A[mu];
                                 // bit 4+mu: the next block along mu exists
                                 // (its contribution is applied in the leaf)
    int32_t shape;               // index of the tuple-grid shape (LeafShape)
};

// Hyperplane-ordered tuple list of one tuple-grid shape (m_0, ..., m_{D-1}
// diagonal blocks per mode): entries ents[ent + hoffs[hoff + h] ...
// ent + hoffs[hoff + h + 1]) are the tuples of hyperplane h, coordinates
// packed in kTupBits(D) bits per mode.
struct LeafShape {
    int32_t ent, hoff, H, count;
};
constexpr int kTupBits3 = 5;     // D = 3: tuple coordinates < 32
constexpr int kTupBits4 = 4;     // D = 4: tuple coordinates < 16

// LDS geometry of the leaf kernel for the largest block of a launch.
struct LeafGeom {
    int cap;                     // prod bmax
    int tsum;                    // sum bmax^2
    int tamax;                   // doubles of one staged T_mu[B, B+1] (odd pitch)
    int maxtup;                  // largest tuple grid (entries)
    int maxcpl;                  // most coupled tuples (a 2x2 block in some mode) of a leaf
    int maxH;                    // most hyperplanes
    int uwords;                  // doubles of the union region
    int bm[kMaxD];
};

// One right-looking update of the dyadic recursion along mode mu:
//   X[.., r0:r0+M, ..] -= T_mu[r0:r0+M, k0:k0+K] x_mu X[.., k0:k0+K, ..]
// restricted to one pencil: the product of the blocks of the other modes.
// ext/ostr list the other modes in increasing mode order (last = fastest).
struct UpdDesc {
    int64_t xbase;               // offset of the pencil origin (mode-mu index 0)
    int32_t prob;
    int32_t r0, M, k0, K;
    int32_t P;                   // number of pencil columns = prod(ext)
    int32_t ext[3];
    int16_t mode;                // mode mu of the update
    int16_t flags;               // bit 0: first contribution to these targets
                                 // (store instead of accumulate; mode 0 adds
                                 // the right-hand side B to what it stores)
    int64_t ostr[3];             // strides of the other modes
};

// One output tile of an update task.
struct WorkItem {
    int32_t task;
    int16_t ta, tb;              // tile indices (meaning depends on the kernel);
                                 // 16 x 256 tiles: tb + 1 consecutive tasks share the tile
};

// Pencils per 16 x 256 tile: tasks with at most 16 target rows whose
// pencils have at most 64 (128) columns share a tile four (two) at a time
// when they agree in everything but the pencil (mode, rows, sources,
// columns, first-contribution flag); each owns a slot of 64 (128) columns.
__host__ __device__ inline int upd_wide_slots(int P) { return P <= 64 ? 4 : (P <= 128 ? 2 : 1); }

// Output tiles of an update task: na x nb, item (ta, tb) with ta < na and
// tb < nb.  At most 16 target rows: 16 x 256 tiles (ta: 256 pencil columns;
// nb = 1, the item's tb counts the other tasks sharing the tile); 17 to 32:
// 32 x 128 tiles (ta: 128 pencil columns, nb = 1); more than 64: 128
// target rows x 64 pencil columns; else 64 x 64.  For
// modes below D - 1, ta counts target rows and tb pencil columns; for the
// fastest mode (right: MFMA rows are pencil columns) the reverse.
inline void upd_tile_grid(const UpdDesc& t, bool right, int& na, int& nb) {
    if (t.M <= 16) {
        na = (t.P + 4 * kTile - 1) / (4 * kTile);
        nb = 1;
        return;
    }
    if (t.M <= 32) {  // 32 target rows x 128 pencil columns: ta counts the columns
        na = (t.P + 2 * kTile - 1) / (2 * kTile);
        nb = 1;
        return;
    }
    const int th = (t.M > kTile) ? 2 * kTile : kTile;  // target rows per tile
    const int nr = (t.M + th - 1) / th, nc = (t.P + kTile - 1) / kTile;
    na = right ? nc : nr;
    nb = right ? nr : nc;
}

// One wave of the schedule: the leaf blocks of hyperplane k and the update
// tiles that became ready after hyperplane k-1.  The two run concurrently
// (on two streams): the updates write only blocks of hyperplanes >= k+1.
struct Wave {
    int64_t leaf_first = 0, leaf_count = 0;
    int64_t item_first = 0, item_count = 0;
    double leaf_flops = 0, leaf_bytes = 0;
    double upd_flops = 0, upd_bytes = 0;
};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct HostProblem {
    int d_user = 0;              // order given by the caller
    int D = 3;                   // internal order
    int64_t n[kMaxD] = {1, 1, 1, 1};
    int64_t stride[kMaxD] = {0, 0, 0, 0};
    std::vector<double> T[kMaxD];          // host copies (row-major)
    std::vector<int32_t> bst[kMaxD];       // block starts
    int m[kMaxD] = {1, 1, 1, 1};
    int64_t N = 0;
};

struct PlanStats {
    double flops = 0;            // method flops (FMA = 2)
    double flops_leaf = 0;
    double flops_update = 0;
    int64_t waves = 0;
    int64_t leaves = 0;
    int64_t tasks = 0;
    int64_t items = 0;
    int64_t launches = 0;
    int bmax[kMaxD] = {0, 0, 0, 0};
};

// Host-side schedule (built without touching the GPU).
struct Schedule {
    int D = 3;
    int cls = 0;                 // 0: Laplace-like, 1: second class (Sec. 3)
    std::vector<HostProblem> probs;
    std::vector<LeafDesc> leaves;
    std::vector<UpdDesc> tasks;
    std::vector<WorkItem> items;
    std::vector<Wave> waves;
    PlanStats stats;
    int bmax[kMaxD] = {1, 1, 1, 1};
    std::vector<LeafShape> shapes;
    std::vector<uint16_t> ents;
    std::vector<int32_t> hoffs;
    int maxtup = 1, maxcpl = 1, maxH = 1;
};

// Planner entry: problems must have D, n, stride, T filled.  Returns a
// status and a message.
int build_schedule(Schedule& s, int nmin, std::string& err);
int leaf_lds_bytes(int D, const int* bmax, int maxtup, int maxcpl, int maxH);
int partition_mode(int64_t n, const double* T, int b, std::vector<int32_t>& bst, std::string& err);

// Kernel launchers (tt_kernels.hip).
hipError_t launch_leaf(int D, const LeafDesc* leaves, int64_t first, int64_t count, const ProbDesc* probs,
                       const LeafShape* shapes, const uint16_t* ents, const int32_t* hoffs, int* status,
                       const int* bmax, int maxtup, int maxcpl, int maxH, hipStream_t st);
// Leaves of the second operator class (tt_leaf2.hip): one wave per block of
// at most 1000 unknowns, else 256 threads.
hipError_t launch_leaf2(int D, const LeafDesc* leaves, int64_t first, int64_t count, const ProbDesc* probs,
                        const LeafShape* shapes, const uint16_t* ents, const int32_t* hoffs, int* status,
                        const int* bmax, hipStream_t st);
int leaf2_lds_bytes(int D, const int* bmax);
// leaf_lds: LDS bytes of a leaf workgroup that should fit on a CU beside two
// update workgroups (0: no limit on update workgroups per CU)
hipError_t launch_update(int D, const UpdDesc* tasks, const WorkItem* items, int64_t first,
                         int64_t count, const ProbDesc* probs, int lp, int leaf_lds, hipStream_t st);
hipError_t launch_zero_int(int* p, int count, hipStream_t st);
hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t st);

// Dense kernels (tt_dense.hip).  Tensor viewed as [L][n_mu][R] for mode mu.
// Y = alpha (X x_mu M) + beta Z with M row-major nout x nin; Z may be Y.
// upper: M is upper triangular (square), its zero K chunks are skipped
hipError_t launch_modeprod(const double* X, double* Y, const double* Z, const double* M, int64_t L, int nin,
                           int nout, int64_t R, double alpha, double beta, int lp, hipStream_t st,
                           bool upper = false);
// Several Gram products in two launches (one split-K Gram pass over all jobs,
// one reduce pass): job j owns workgroups [wg_first, wg_first + nt^2 nsplit)
// and output elements [el_first, el_first + n^2).
constexpr int kGramTile = 64;  // output tile edge of the Gram kernels
constexpr int kGramKC = 16;    // their K chunk
struct GramJob {
    const double* P;
    const double* Q;
    double* W;
    const double* T;
    double* out;
    int64_t L, R, kchunk, wg_first, el_first;
    int n, nsplit, dense, pad;
};
hipError_t launch_gram_batched(const GramJob* jobs, int njobs, int64_t wgs, int64_t elems, double scale,
                               hipStream_t st);
hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t st);
int sumsq_blocks();
hipError_t launch_sumsq2(const double* x, const double* y, int64_t n, double* part, hipStream_t st);
hipError_t launch_f64_to_f32(const double* x, float* y, int64_t n, hipStream_t st);
hipError_t launch_f32_to_f64(const float* x, double* y, int64_t n, hipStream_t st);

// Host real Schur decomposition A = U T U^T (tt_schur.cpp), row-major.
int qz_real(int n, const double* A, const double* C, double* S, double* T, double* Q, double* Z,
            std::string& err);
int schur_real(int n, const double* A, double* T, double* U, std::string& err);
int merge_modes(int na, const double* Ta, int nb, const double* Tb, double* Tm, double* V, int* perm,
                std::string& err);
int schur_real_many(int count, const int* n, const double* const* A, double* const* T, double* const* U,
                    std::string& err);

}  // namespace tt
