// C ABI of the solver (declared in include/tt.h): argument validation, plan
// construction (host) and the ordered launch sequence on one HIP stream.
#include <algorithm>
#include <chrono>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "tt_internal.h"

namespace tt {

static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define TT_HIP_CHECK(expr)                                                                 \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(TT_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

struct PtrPack {
    double* p[64];
    const double* b[64];
};

__global__ void set_x_ptrs_kernel(ProbDesc* probs, PtrPack pack, int first, int count) {
    int i = threadIdx.x;
    if (i < count) {
        ProbDesc& P = probs[first + i];
        P.X = pack.p[i];
        P.B = pack.b[i];
        // update sources: X, or the second class's partial products
        for (int mu = 0; mu < kMaxD; ++mu) P.S[mu] = (P.cls == 1 && mu >= 2) ? P.W[mu - 1] : pack.p[i];
    }
}

// In-place reversal of the element order of a tensor (all modes reversed).
__global__ void reverse_inplace_kernel(double* x, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n / 2; i += stride) {
        double a = x[i], b = x[n - 1 - i];
        x[i] = b;
        x[n - 1 - i] = a;
    }
}
__global__ void reverse_copy_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[n - 1 - i];
}

static unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned)b;
}

}  // namespace tt

using namespace tt;

enum PlanKind { KIND_TRI = 0, KIND_PAIR = 1, KIND_GENERAL = 2 };

struct tt_plan_s {
    Schedule sched;
    int trans = 0;
    int count = 0;
    int kind = KIND_TRI;
    std::vector<int> d_user;
    // device
    ProbDesc* d_probs = nullptr;
    LeafDesc* d_leaves = nullptr;
    LeafShape* d_shapes = nullptr;
    uint16_t* d_ents = nullptr;
    int32_t* d_hoffs = nullptr;
    UpdDesc* d_tasks = nullptr;
    WorkItem* d_items = nullptr;
    int* d_status = nullptr;
    std::vector<void*> owned;  // device buffers allocated by the library
    // caller-provided device workspace (tt_opts::workspace): every device
    // buffer is carved from it instead of allocated; uploads are then ordered
    // on up_stream (the stream of the options)
    char* ws_base = nullptr;
    size_t ws_cap = 0, ws_used = 0;
    hipStream_t up_stream = nullptr;
    // all launches on the caller's stream (no side stream, no events)
    bool serial_only = false;
    std::vector<char> image;     // host images of uploaded tables
    std::vector<ProbDesc> pdesc;
    hipStream_t side = nullptr;  // stream of the update launches
    std::vector<hipEvent_t> evL, evU;
    hipEvent_t ev_start = nullptr;
    hipStream_t last_stream = nullptr;
    double build_seconds = 0;
    double schur_seconds = 0;
    int device = 0;
    // pipelines (pair form, dense coefficients): mode products applied to B
    // before the triangular solve (pre) and to its result after (post), one
    // row-major n_mu x n_mu device matrix per user mode; W: one tensor of
    // workspace
    std::vector<double*> pre, post;
    std::vector<const double*> upper;  // uploaded matrices that are upper triangular
    double* W = nullptr;
    double pipe_flops = 0;
    // coefficient gradients (allocated on first use): split-K Gram workspace,
    // the job table (pinned host staging + device copy) and an event marking
    // the end of its last upload
    double* gW = nullptr;
    size_t gW_size = 0;
    std::vector<GramJob> gJobsHost;
    GramJob* gJobsDev = nullptr;
    int gJobsCap = 0;
    hipEvent_t gJobsEv = nullptr;
    // mixed precision with FP64 refinement (dense coefficients)
    int prec = TT_FP64;
    double tol = 1e-13;
    int max_iter = 10;
    std::vector<double*> Adev;   // dense A_mu (device) for the FP64 residual
    double* R = nullptr;         // residual / correction tensor
    double* part = nullptr;      // norm partial sums (device)
    std::vector<double> part_host;  // host copy
    double last_info[2] = {0, 0};
    // the solve recorded as a HIP graph (tt_plan_solve_graph) and the
    // (B, X, stream) it was recorded for
    hipGraphExec_t gexec = nullptr;
    const double* gB = nullptr;
    double* gX = nullptr;
    hipStream_t gst = nullptr;
    hipEvent_t gdone = nullptr;  // recorded after every graph launch (the caller's
                                 // stream may be gone when the plan is destroyed)

    ~tt_plan_s() {
        if (gdone) {
            (void)hipEventSynchronize(gdone);
            (void)hipEventDestroy(gdone);
        }
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (side) (void)hipStreamSynchronize(side);
        for (hipEvent_t e : evL) (void)hipEventDestroy(e);
        for (hipEvent_t e : evU) (void)hipEventDestroy(e);
        if (ev_start) (void)hipEventDestroy(ev_start);
        if (side) (void)hipStreamDestroy(side);
        if (gJobsEv) (void)hipEventSynchronize(gJobsEv);
        // uploads into a caller workspace are asynchronous on up_stream and
        // read host vectors of this plan
        if (ws_base) (void)hipStreamSynchronize(up_stream);
        for (void* p : owned) (void)hipFree(p);
        if (gJobsEv) (void)hipEventDestroy(gJobsEv);
    }
};

namespace {

// Validate the shape arguments of one problem and fill the host description
// (without coefficients).  Orders below 3 are promoted to 3 by leading modes of
// size 1 whose coefficient is the 1x1 zero matrix (X x_mu 0 = 0 leaves the
// operator unchanged).
int describe_problem(int d, const int64_t* n, int D, HostProblem& hp) {
    if (d < 1 || d > 4) return fail(TT_EINVAL, "order d must be 1..4");
    if (!n) return fail(TT_EINVAL, "n is NULL");
    for (int mu = 0; mu < d; ++mu)
        if (n[mu] < 0 || n[mu] > (int64_t)1 << 30) return fail(TT_EINVAL, "mode size out of range");
    hp.d_user = d;
    hp.D = D;
    const int lead = D - d;
    for (int mu = 0; mu < D; ++mu) hp.n[mu] = (mu < lead) ? 1 : n[mu - lead];
    int64_t s = 1;
    for (int mu = D - 1; mu >= 0; --mu) {
        hp.stride[mu] = s;
        s *= hp.n[mu];
    }
    hp.N = s;
    return TT_OK;
}

// Place the user's coefficients (host, row-major, one vector per user mode)
// into the internal problem.  trans != 0: the adjoint sum L x_mu T^T = G is
// an upper quasi-triangular system in reversed index order with
// T'[i][j] = T[n-1-j][n-1-i].
void set_host_coefficients(HostProblem& hp, const std::vector<std::vector<double>>& Tu, int trans) {
    const int lead = hp.D - hp.d_user;
    for (int mu = 0; mu < hp.D; ++mu) {
        const int64_t nm = hp.n[mu];
        hp.T[mu].assign((size_t)(nm * nm), 0.0);
        if (mu < lead || nm == 0) continue;
        const std::vector<double>& src = Tu[(size_t)(mu - lead)];
        if (!trans) {
            hp.T[mu] = src;
        } else {
            for (int64_t i = 0; i < nm; ++i)
                for (int64_t j = 0; j < nm; ++j) hp.T[mu][i * nm + j] = src[(nm - 1 - j) * nm + (nm - 1 - i)];
        }
    }
}

// Copy d device matrices (n[mu] x n[mu]) to host vectors.
int fetch_matrices(int d, const int64_t* n, const double* const* M, std::vector<std::vector<double>>& out) {
    out.assign((size_t)d, {});
    for (int mu = 0; mu < d; ++mu) {
        const int64_t nm = n[mu];
        out[(size_t)mu].assign((size_t)(nm * nm), 0.0);
        if (nm == 0) continue;
        if (!M[mu]) return fail(TT_EINVAL, "coefficient pointer is NULL");
        TT_HIP_CHECK(hipMemcpy(out[(size_t)mu].data(), M[mu], sizeof(double) * (size_t)(nm * nm),
                               hipMemcpyDeviceToHost));
    }
    return TT_OK;
}

int fetch_coefficients(const double* const* T, int trans, HostProblem& hp) {
    std::vector<std::vector<double>> Tu;
    int rc = fetch_matrices(hp.d_user, hp.n + (hp.D - hp.d_user), T, Tu);
    if (rc) return rc;
    set_host_coefficients(hp, Tu, trans);
    return TT_OK;
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device buffer of a plan: carved from the caller's workspace when the plan
// has one (256-byte aligned, TT_ENOMEM with the needed size when it runs
// out), else allocated and owned by the plan.
int dev_alloc(tt_plan_s* P, size_t bytes, void** out, const char* what) {
    *out = nullptr;
    bytes = align256(std::max<size_t>(bytes, 1));
    if (P->ws_base) {
        if (P->ws_used + bytes > P->ws_cap)
            return fail(TT_ENOMEM, std::string("workspace too small for ") + what + ": needs at least " +
                                       std::to_string(P->ws_used + bytes) + " bytes, has " +
                                       std::to_string(P->ws_cap));
        *out = P->ws_base + P->ws_used;
        P->ws_used += bytes;
        return TT_OK;
    }
    if (hipMalloc(out, bytes) != hipSuccess) {
        *out = nullptr;
        return fail(TT_ENOMEM, std::string("hipMalloc failed (") + what + ")");
    }
    P->owned.push_back(*out);
    return TT_OK;
}

// Host -> device copy of plan data: ordered on the options' stream when the
// memory is the caller's workspace (earlier work there may still use it),
// else synchronous.
int to_device(tt_plan_s* P, void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return TT_OK;
    if (P->ws_base) {
        TT_HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, P->up_stream));
    } else {
        TT_HIP_CHECK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    }
    return TT_OK;
}

template <typename V>
int upload(tt_plan_s* P, const std::vector<V>& v, V** dst) {
    *dst = nullptr;
    if (v.empty()) return TT_OK;
    int rc = dev_alloc(P, sizeof(V) * v.size(), (void**)dst, "plan tables");
    if (rc) return rc;
    return to_device(P, *dst, v.data(), sizeof(V) * v.size());
}

int upload_matrix(tt_plan_s* P, const std::vector<double>& m, double** out) {
    int rc = dev_alloc(P, sizeof(double) * m.size(), (void**)out, "coefficient matrix");
    if (rc) return rc;
    // an upper triangular matrix (C^{-1} of the pair forms) lets the mode
    // product skip its zero K chunks
    const int64_t n = (int64_t)std::llround(std::sqrt((double)m.size()));
    bool up = n * n == (int64_t)m.size();
    for (int64_t i = 1; up && i < n; ++i)
        for (int64_t j = 0; j < i; ++j)
            if (m[(size_t)(i * n + j)] != 0.0) {
                up = false;
                break;
            }
    if (up) P->upper.push_back(*out);
    return to_device(P, *out, m.data(), sizeof(double) * m.size());
}

bool is_upper(const tt_plan_s* P, const double* M) {
    return std::find(P->upper.begin(), P->upper.end(), M) != P->upper.end();
}

// flops of one pass of mode products (one FMA = 2 flops): 2 n N per dense
// matrix, (n + 1) N per upper triangular one (n (n + 1) / 2 FMAs per fibre)
double chain_flops(const tt_plan_s* P, const std::vector<double*>& mats) {
    const HostProblem& hp = P->sched.probs[0];
    const int lead = hp.D - hp.d_user;
    double f = 0;
    for (size_t mu = 0; mu < mats.size() && (int)mu < hp.d_user; ++mu) {
        if (!mats[mu]) continue;
        const double n = (double)hp.n[lead + (int)mu];
        f += (is_upper(P, mats[mu]) ? n + 1.0 : 2.0 * n) * (double)hp.N;
    }
    return f;
}

int alloc_tensor(tt_plan_s* P, int64_t N, double** out) {
    return dev_alloc(P, sizeof(double) * (size_t)std::max<int64_t>(1, N), (void**)out, "workspace tensor");
}

// Set while solve_tri_tensor_noalloc builds its plan: the plan then runs
// every launch on the caller's stream (no side stream and no events).
thread_local bool t_serial_plan = false;

// Take the options' workspace (if any) for the plan's device buffers.
void adopt_workspace(tt_plan_s* P, const tt_opts* opts) {
    P->serial_only = t_serial_plan;
    if (!opts || !opts->workspace) return;
    P->ws_base = (char*)opts->workspace;
    P->ws_cap = opts->workspace_bytes;
    P->ws_used = 0;
    // keep the carved buffers 256-byte aligned whatever the base
    const size_t mis = (size_t)((uintptr_t)P->ws_base & 255);
    if (mis) {
        const size_t skip = 256 - mis;
        P->ws_base += skip;
        P->ws_cap = P->ws_cap > skip ? P->ws_cap - skip : 0;
    }
    P->up_stream = (hipStream_t)opts->stream;
}

// Device bytes finish_plan takes for a built schedule (tables, coefficient
// copies, block starts, accumulators, status word), as dev_alloc rounds them.
size_t plan_table_bytes(const Schedule& s) {
    auto al = align256;
    size_t cbytes = 0, abytes = 0;
    for (const HostProblem& hp : s.probs)
        for (int mu = 0; mu < s.D; ++mu) {
            cbytes += al(sizeof(double) * std::max<size_t>(1, hp.T[mu].size()));
            cbytes += al(sizeof(int32_t) * hp.bst[mu].size());
            if (mu >= 1 && hp.N > 0) abytes += al(sizeof(double) * (size_t)hp.N);
        }
    auto tb = [&](size_t n, size_t sz) { return n ? al(n * sz) : 0; };
    return al(std::max<size_t>(cbytes, 1)) + (abytes ? al(abytes) : 0) + tb(s.probs.size(), sizeof(ProbDesc)) +
           tb(s.leaves.size(), sizeof(LeafDesc)) + tb(s.shapes.size(), sizeof(LeafShape)) +
           tb(s.ents.size(), sizeof(uint16_t)) + tb(s.hoffs.size(), sizeof(int32_t)) +
           tb(s.tasks.size(), sizeof(UpdDesc)) + tb(s.items.size(), sizeof(WorkItem)) + al(sizeof(int) * 4);
}

int finish_plan(tt_plan_s* P, int nmin) {
    std::string err;
    int rc = build_schedule(P->sched, nmin, err);
    if (rc) return fail(rc, err);
    Schedule& s = P->sched;
    // One device buffer for every problem's coefficients and block starts
    // (filled by one copy from a packed host image) and one for the update
    // accumulators: a batched plan makes two allocations instead of several
    // per problem and mode.
    auto al = align256;
    size_t cbytes = 0, abytes = 0;
    for (const HostProblem& hp : s.probs)
        for (int mu = 0; mu < s.D; ++mu) {
            cbytes += al(sizeof(double) * std::max<size_t>(1, hp.T[mu].size()));
            cbytes += al(sizeof(int32_t) * hp.bst[mu].size());
            // accumulator of the updates of mode mu (mode 0 updates X itself)
            if (mu >= 1 && hp.N > 0) abytes += al(sizeof(double) * (size_t)hp.N);
        }
    char* dc = nullptr;
    char* da = nullptr;
    if ((rc = dev_alloc(P, cbytes, (void**)&dc, "coefficients"))) return rc;
    if (abytes > 0 && (rc = dev_alloc(P, abytes, (void**)&da, "update accumulators"))) return rc;
    // second class: the partial products W_1 .. W_{D-2} written by the leaves
    std::vector<std::vector<double*>> wt(s.probs.size());
    if (s.cls == 1)
        for (size_t i = 0; i < s.probs.size(); ++i)
            for (int k = 1; k <= s.D - 2; ++k) {
                double* w = nullptr;
                if ((rc = alloc_tensor(P, s.probs[i].N, &w))) return rc;
                wt[i].push_back(w);
            }
    std::vector<char> image(cbytes, 0);
    std::vector<ProbDesc> pd(s.probs.size());
    size_t co = 0, ao = 0;
    for (size_t i = 0; i < s.probs.size(); ++i) {
        HostProblem& hp = s.probs[i];
        ProbDesc& d = pd[i];
        std::memset(&d, 0, sizeof(d));
        for (int mu = 0; mu < kMaxD; ++mu) {
            d.n[mu] = (mu < s.D) ? hp.n[mu] : 1;
            d.stride[mu] = (mu < s.D) ? hp.stride[mu] : 0;
        }
        d.cls = s.cls;
        for (size_t k = 0; k < wt[i].size(); ++k) d.W[k + 1] = wt[i][k];
        for (int mu = 0; mu < s.D; ++mu) {
            if (!hp.T[mu].empty()) std::memcpy(image.data() + co, hp.T[mu].data(), sizeof(double) * hp.T[mu].size());
            d.T[mu] = (double*)(dc + co);
            co += al(sizeof(double) * std::max<size_t>(1, hp.T[mu].size()));
            std::memcpy(image.data() + co, hp.bst[mu].data(), sizeof(int32_t) * hp.bst[mu].size());
            d.bst[mu] = (int32_t*)(dc + co);
            co += al(sizeof(int32_t) * hp.bst[mu].size());
            if (mu >= 1 && hp.N > 0) {
                d.A[mu] = (double*)(da + ao);
                ao += al(sizeof(double) * (size_t)hp.N);
            }
        }
    }
    P->image = std::move(image);  // kept until the plan is destroyed (asynchronous upload)
    if ((rc = to_device(P, dc, P->image.data(), cbytes))) return rc;
    P->pdesc = std::move(pd);
    if ((rc = upload(P, P->pdesc, &P->d_probs))) return rc;
    if ((rc = upload(P, s.leaves, &P->d_leaves))) return rc;
    if ((rc = upload(P, s.shapes, &P->d_shapes))) return rc;
    if ((rc = upload(P, s.ents, &P->d_ents))) return rc;
    if ((rc = upload(P, s.hoffs, &P->d_hoffs))) return rc;
    if ((rc = upload(P, s.tasks, &P->d_tasks))) return rc;
    if ((rc = upload(P, s.items, &P->d_items))) return rc;
    // status word: cleared by every solve before its first launch
    if ((rc = dev_alloc(P, sizeof(int) * 4, (void**)&P->d_status, "status word"))) return rc;
    TT_HIP_CHECK(launch_zero_int(P->d_status, 4, P->up_stream));
    if (P->serial_only) return TT_OK;
    TT_HIP_CHECK(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking));
    P->evL.resize(s.waves.size());
    P->evU.resize(s.waves.size());
    for (auto& e : P->evL) TT_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& e : P->evU) TT_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    TT_HIP_CHECK(hipEventCreateWithFlags(&P->ev_start, hipEventDisableTiming));
    return TT_OK;
}

// Solution and right-hand-side pointers of the problems (B = NULL: the
// right-hand side is already in X).
int set_pointers(tt_plan_s* P, double* const* X, int count, hipStream_t st, const double* const* B = nullptr) {
    for (int first = 0; first < count; first += 64) {
        PtrPack pack;
        int c = std::min(64, count - first);
        for (int i = 0; i < c; ++i) {
            pack.p[i] = X[first + i];
            pack.b[i] = B ? B[first + i] : X[first + i];
        }
        hipLaunchKernelGGL(set_x_ptrs_kernel, dim3(1), dim3(64), 0, st, P->d_probs, pack, first, c);
        TT_HIP_CHECK(hipGetLastError());
    }
    return TT_OK;
}

// The launch sequence of one solve (X already holds the right-hand side).
// Wave k: the leaf blocks of hyperplane k on the caller's stream, and on the
// plan's side stream the updates that became ready after hyperplane k-1.
// Leaves of wave k wait for the updates of wave k-1; updates of wave k wait
// for the leaves of wave k-1.  So the updates of wave k run concurrently with
// the leaves of wave k (they write only hyperplanes >= k+1).
// With prof != NULL, timing events bracket every launch (profiling only).
struct ProfEvents {
    std::vector<hipEvent_t> lb, la, ub, ua;
    bool serial = false;  // every launch on the caller's stream
};

// The leaf launch of a schedule's operator class.
hipError_t launch_leaf_any(const Schedule& s, const LeafDesc* leaves, int64_t first, int64_t count,
                           const ProbDesc* probs, const LeafShape* shapes, const uint16_t* ents, const int32_t* hoffs,
                           int* status, const int* bmax, int maxtup, int maxcpl, int maxH, hipStream_t st) {
    if (s.cls == 1) return launch_leaf2(s.D, leaves, first, count, probs, shapes, ents, hoffs, status, bmax, st);
    return launch_leaf(s.D, leaves, first, count, probs, shapes, ents, hoffs, status, bmax, maxtup, maxcpl, maxH, st);
}

int run_schedule(tt_plan_s* P, hipStream_t st, ProfEvents* prof = nullptr, int lp = 0) {
    Schedule& s = P->sched;
    if (P->serial_only) {
        // one stream: wave k's leaves, then the updates ready after them
        const int leaf_lds = leaf_lds_bytes(s.D, s.bmax, s.maxtup, s.maxcpl, s.maxH);
        for (const Wave& wv : s.waves) {
            TT_HIP_CHECK(launch_leaf_any(s, P->d_leaves, wv.leaf_first, wv.leaf_count, P->d_probs, P->d_shapes,
                                     P->d_ents, P->d_hoffs, P->d_status, s.bmax, s.maxtup, s.maxcpl, s.maxH,
                                     st));
            TT_HIP_CHECK(launch_update(s.D, P->d_tasks, P->d_items, wv.item_first, wv.item_count, P->d_probs, lp,
                                       leaf_lds, st));
        }
        P->last_stream = st;
        return TT_OK;
    }
    TT_HIP_CHECK(hipEventRecord(P->ev_start, st));
    TT_HIP_CHECK(hipStreamWaitEvent(P->side, P->ev_start, 0));
    const size_t W = s.waves.size();
    const int leaf_lds = leaf_lds_bytes(s.D, s.bmax, s.maxtup, s.maxcpl, s.maxH);
    for (size_t k = 0; k < W; ++k) {
        const Wave& wv = s.waves[k];
        if (k >= 1) TT_HIP_CHECK(hipStreamWaitEvent(st, P->evU[k - 1], 0));
        if (prof) TT_HIP_CHECK(hipEventRecord(prof->lb[k], st));
        TT_HIP_CHECK(launch_leaf_any(s, P->d_leaves, wv.leaf_first, wv.leaf_count, P->d_probs, P->d_shapes,
                                 P->d_ents, P->d_hoffs, P->d_status, s.bmax, s.maxtup, s.maxcpl, s.maxH, st));
        if (prof) TT_HIP_CHECK(hipEventRecord(prof->la[k], st));
        TT_HIP_CHECK(hipEventRecord(P->evL[k], st));
        // a serial profiling pass runs each kernel alone (updates on the
        // caller's stream)
        const bool serial = prof && prof->serial;
        hipStream_t us = serial ? st : P->side;
        if (k >= 1 && !serial) TT_HIP_CHECK(hipStreamWaitEvent(P->side, P->evL[k - 1], 0));
        if (prof) TT_HIP_CHECK(hipEventRecord(prof->ub[k], us));
        TT_HIP_CHECK(launch_update(s.D, P->d_tasks, P->d_items, wv.item_first, wv.item_count, P->d_probs, lp,
                                   leaf_lds, us));
        if (prof) TT_HIP_CHECK(hipEventRecord(prof->ua[k], us));
        TT_HIP_CHECK(hipEventRecord(P->evU[k], us));
    }
    if (W > 0) TT_HIP_CHECK(hipStreamWaitEvent(st, P->evU[W - 1], 0));
    P->last_stream = st;
    return TT_OK;
}

int prepare_inputs(tt_plan_s* P, const double* const* B, double* const* X, hipStream_t st) {
    for (int i = 0; i < P->count; ++i) {
        const HostProblem& hp = P->sched.probs[(size_t)i];
        if (hp.N == 0) continue;
        if (!B[i] || !X[i]) return fail(TT_EINVAL, "tensor pointer is NULL");
        if (!P->trans) {
            // no copy: the first mode-0 update of a block, or its leaf, reads B
        } else {
            if (B[i] != X[i]) {
                hipLaunchKernelGGL(reverse_copy_kernel, dim3(grid_for(hp.N)), dim3(256), 0, st, B[i], X[i], hp.N);
            } else {
                hipLaunchKernelGGL(reverse_inplace_kernel, dim3(grid_for(hp.N)), dim3(256), 0, st, X[i], hp.N);
            }
            TT_HIP_CHECK(hipGetLastError());
        }
    }
    return set_pointers(P, X, P->count, st, P->trans ? nullptr : B);
}

int finish_outputs(tt_plan_s* P, double* const* X, hipStream_t st) {
    if (!P->trans) return TT_OK;
    for (int i = 0; i < P->count; ++i) {
        const HostProblem& hp = P->sched.probs[(size_t)i];
        if (hp.N == 0) continue;
        hipLaunchKernelGGL(reverse_inplace_kernel, dim3(grid_for(hp.N)), dim3(256), 0, st, X[i], hp.N);
        TT_HIP_CHECK(hipGetLastError());
    }
    return TT_OK;
}

int internal_order(const int* d, int count) {
    int D = 3;
    for (int i = 0; i < count; ++i)
        if (d[i] == 4) D = 4;
    return D;
}

// Mode-mu view [L][n_mu][R] of the (single) problem's user tensor.
void mode_view(const HostProblem& hp, int mu, int64_t& L, int64_t& nm, int64_t& R) {
    const int lead = hp.D - hp.d_user;
    L = 1;
    R = 1;
    for (int nu = 0; nu < hp.d_user; ++nu) {
        if (nu < mu) L *= hp.n[lead + nu];
        if (nu > mu) R *= hp.n[lead + nu];
    }
    nm = hp.n[lead + mu];
}

// Apply one mode product per user mode, in mode order, starting from src and
// ending in fin; intermediate results alternate between fin and other.  If the
// first target would be src itself, src is first copied to the free buffer.
int apply_chain(tt_plan_s* P, const double* src, double* fin, double* other, const std::vector<double*>& mats,
                int lp, hipStream_t st) {
    const HostProblem& hp = P->sched.probs[0];
    // the modes that carry a matrix (a NULL entry leaves its mode unchanged)
    std::vector<int> modes;
    for (size_t i = 0; i < mats.size(); ++i)
        if (mats[i]) modes.push_back((int)i);
    const int m = (int)modes.size();
    if (m == 0) {
        if (src != fin) TT_HIP_CHECK(launch_copy(src, fin, hp.N, st));
        return TT_OK;
    }
    const double* cur = src;
    double* t0 = ((m - 1) % 2 == 0) ? fin : other;
    if (t0 == cur) {
        double* o = (cur == fin) ? other : fin;
        TT_HIP_CHECK(launch_copy(cur, o, hp.N, st));
        cur = o;
    }
    for (int i = 0; i < m; ++i) {
        double* tgt = ((m - 1 - i) % 2 == 0) ? fin : other;
        int64_t L, nm, R;
        mode_view(hp, modes[(size_t)i], L, nm, R);
        const double* M = mats[(size_t)modes[(size_t)i]];
        TT_HIP_CHECK(launch_modeprod(cur, tgt, nullptr, M, L, (int)nm, (int)nm, R, 1.0, 0.0, lp, st, is_upper(P, M)));
        cur = tgt;
    }
    return TT_OK;
}

// One pass of the plan's method for a single problem: B -> X.
//   TRI:     copy, triangular solve (adjoint plans reverse the order);
//   PAIR:    X = B x_mu C_mu^{-1} (all modes), triangular solve in X;
//   GENERAL: B~ = B x_mu U_mu^T, triangular solve, X = X~ x_mu U_mu.
// lp = 1 runs the recursion updates and the transforms in FP32 MFMA, lp = 2
// in three-term BF16 MFMA with FP32 accumulation; the leaves stay FP64.
int run_pipeline(tt_plan_s* P, const double* B, double* X, int lp, hipStream_t st) {
    if (P->kind == KIND_TRI) {
        int rc = prepare_inputs(P, &B, &X, st);
        if (!rc) rc = run_schedule(P, st, nullptr, lp);
        if (!rc) rc = finish_outputs(P, &X, st);
        return rc;
    }
    const HostProblem& hp = P->sched.probs[0];
    if (hp.N == 0) return TT_OK;
    if (!B || !X) return fail(TT_EINVAL, "tensor pointer is NULL");
    double* S = X;
    int rc;
    if (P->kind == KIND_PAIR) {
        rc = apply_chain(P, B, X, P->W, P->pre, lp, st);
    } else {
        S = (hp.d_user % 2 == 0) ? X : P->W;
        rc = apply_chain(P, B, S, (S == X) ? P->W : X, P->pre, lp, st);
    }
    if (rc) return rc;
    if ((rc = set_pointers(P, &S, 1, st))) return rc;
    if ((rc = run_schedule(P, st, nullptr, lp))) return rc;
    if (P->kind == KIND_GENERAL) rc = apply_chain(P, S, X, P->W, P->post, lp, st);
    return rc;
}

// Mixed precision with FP64 iterative refinement:
//   X_0 = solve_lp(B);  repeat  R = B - sum_mu X x_mu A_mu  (FP64),
//   D = solve_lp(R),  X += D  until ||D||_F / ||X||_F <= tol or max_iter.
// The iteration contracts linearly: D_{k+1} ~ rho D_k with rho estimated as
// ratio_k / ratio_{k-1}, and D_{k+1} is about the error left in X after the
// k-th correction.  So from the second correction on it also stops when
// rho < 1/2 and rho * ratio_k <= tol (that next correction would be below
// tol), which saves the last low-precision solve and FP64 residual.
int run_refined(tt_plan_s* P, const double* B, double* X, hipStream_t st) {
    const HostProblem& hp = P->sched.probs[0];
    P->last_info[0] = 0;
    P->last_info[1] = 0;
    if (hp.N == 0) return TT_OK;
    if (B == X) return fail(TT_EINVAL, "mixed precision needs X distinct from B (B enters every residual)");
    const int lp = (P->prec == TT_MP_BF16) ? 2 : 1;
    int rc = run_pipeline(P, B, X, lp, st);
    if (rc) return rc;
    const int nb = sumsq_blocks();
    double prev = 0.0;
    for (int it = 1; it <= P->max_iter; ++it) {
        TT_HIP_CHECK(launch_copy(B, P->R, hp.N, st));
        for (int mu = 0; mu < hp.d_user; ++mu) {
            int64_t L, nm, Rr;
            mode_view(hp, mu, L, nm, Rr);
            TT_HIP_CHECK(launch_modeprod(X, P->R, P->R, P->Adev[(size_t)mu], L, (int)nm, (int)nm, Rr, -1.0, 1.0, 0,
                                         st));
        }
        if ((rc = run_pipeline(P, P->R, P->R, lp, st))) return rc;
        TT_HIP_CHECK(launch_axpy(X, P->R, 1.0, hp.N, st));
        TT_HIP_CHECK(launch_sumsq2(P->R, X, hp.N, P->part, st));
        TT_HIP_CHECK(hipMemcpyAsync(P->part_host.data(), P->part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, st));
        TT_HIP_CHECK(hipStreamSynchronize(st));
        double dd = 0, xx = 0;
        for (int b = 0; b < nb; ++b) {
            dd += P->part_host[2 * b];
            xx += P->part_host[2 * b + 1];
        }
        const double ratio = (xx > 0) ? std::sqrt(dd / xx) : 0.0;
        P->last_info[0] = it;
        P->last_info[1] = ratio;
        if (!std::isfinite(ratio)) return fail(TT_ESINGULAR, "refinement produced a non-finite correction");
        if (ratio <= P->tol) return TT_OK;
        if (it >= 2 && prev > 0.0) {
            const double rho = ratio / prev;
            if (rho < 0.5 && rho * ratio <= P->tol) return TT_OK;
        }
        prev = ratio;
    }
    return fail(TT_ENOTCONV, "mixed-precision refinement did not reach the tolerance");
}

int setup_refinement(tt_plan_s* P, const std::vector<std::vector<double>>& A, const tt_opts* opts) {
    P->prec = opts ? opts->prec : TT_FP64;
    if (P->prec == TT_FP64) return TT_OK;
    if (P->prec != TT_MP_FP32 && P->prec != TT_MP_BF16) return fail(TT_EINVAL, "unknown precision");
    if (P->count != 1 || P->trans) return fail(TT_EINVAL, "mixed precision needs a single, non-adjoint problem");
    P->tol = opts->tol > 0 ? opts->tol : 1e-13;
    P->max_iter = opts->max_iter > 0 ? opts->max_iter : 10;
    const HostProblem& hp = P->sched.probs[0];
    P->Adev.assign(A.size(), nullptr);
    int rc;
    for (size_t mu = 0; mu < A.size(); ++mu)
        if ((rc = upload_matrix(P, A[mu], &P->Adev[mu]))) return rc;
    if ((rc = alloc_tensor(P, hp.N, &P->R))) return rc;
    if ((rc = dev_alloc(P, sizeof(double) * 2 * sumsq_blocks(), (void**)&P->part, "norm partial sums"))) return rc;
    P->part_host.assign((size_t)2 * sumsq_blocks(), 0.0);
    return TT_OK;
}

// Top level of one (possibly refined) solve of a single-problem plan.
int solve_single(tt_plan_s* P, const double* B, double* X, hipStream_t st) {
    TT_HIP_CHECK(launch_zero_int(P->d_status, 4, st));
    P->last_stream = st;
    if (P->prec != TT_FP64) return run_refined(P, B, X, st);
    return run_pipeline(P, B, X, 0, st);
}

// Plan of a single problem from host coefficients (row-major, one vector per
// user mode), without the device work of finish_plan.
int plan_begin(tt_plan_s* P, int d, const int64_t* n, const std::vector<std::vector<double>>& Tu, int trans) {
    P->trans = trans;
    P->count = 1;
    P->sched.D = (d == 4) ? 4 : 3;
    P->sched.probs.resize(1);
    int rc = describe_problem(d, n, P->sched.D, P->sched.probs[0]);
    if (rc) return rc;
    set_host_coefficients(P->sched.probs[0], Tu, trans);
    P->d_user.push_back(d);
    (void)hipGetDevice(&P->device);
    return TT_OK;
}

// Single-problem plan of a triangular equation (Laplace-like, cls 0, or the
// second class, cls 1) with host coefficients T (n[mu] x n[mu]) and
// optional mode products applied to B before the solve (pre[mu]) and to its
// result after it (post[mu]); empty matrices skip a mode, an empty post
// vector skips the post-transforms.
int pipeline_plan(tt_plan_s* P, int d, const int64_t* n, const std::vector<std::vector<double>>& T,
                  const std::vector<std::vector<double>>& pre, const std::vector<std::vector<double>>& post, int cls,
                  const tt_opts* opts) {
    int rc;
    if ((rc = plan_begin(P, d, n, T, 0))) return rc;
    P->sched.cls = cls;
    P->kind = post.empty() ? KIND_PAIR : KIND_GENERAL;
    if ((rc = finish_plan(P, opts ? opts->nmin : 0))) return rc;
    const HostProblem& hp = P->sched.probs[0];
    P->pre.assign((size_t)d, nullptr);
    for (int mu = 0; mu < d; ++mu)
        if (!pre[(size_t)mu].empty() && (rc = upload_matrix(P, pre[(size_t)mu], &P->pre[(size_t)mu]))) return rc;
    if (!post.empty()) {
        P->post.assign((size_t)d, nullptr);
        for (int mu = 0; mu < d; ++mu)
            if (!post[(size_t)mu].empty() && (rc = upload_matrix(P, post[(size_t)mu], &P->post[(size_t)mu])))
                return rc;
    }
    if ((rc = alloc_tensor(P, hp.N, &P->W))) return rc;
    P->pipe_flops = P->sched.stats.flops + chain_flops(P, P->pre) + chain_flops(P, P->post);
    return TT_OK;
}

// row-major Kronecker product of two square matrices (empty = identity of
// size q / p)
std::vector<double> kron_sq(const std::vector<double>& A, int64_t p, const std::vector<double>& B, int64_t q) {
    const int64_t m = p * q;
    std::vector<double> K((size_t)(m * m), 0.0);
    for (int64_t i = 0; i < p; ++i)
        for (int64_t j = 0; j < p; ++j) {
            const double a = A.empty() ? (i == j ? 1.0 : 0.0) : A[(size_t)(i * p + j)];
            if (a == 0.0) continue;
            for (int64_t k = 0; k < q; ++k)
                for (int64_t l = 0; l < q; ++l) {
                    const double b = B.empty() ? (k == l ? 1.0 : 0.0) : B[(size_t)(k * q + l)];
                    K[(size_t)((i * q + k) * m + j * q + l)] = a * b;
                }
        }
    return K;
}

std::vector<double> matmul_sq(const std::vector<double>& A, const std::vector<double>& B, int64_t m) {
    std::vector<double> C((size_t)(m * m), 0.0);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = 0; k < m; ++k) {
            const double a = A[(size_t)(i * m + k)];
            if (a == 0.0) continue;
            for (int64_t j = 0; j < m; ++j) C[(size_t)(i * m + j)] += a * B[(size_t)(k * m + j)];
        }
    return C;
}

// Order 5 (Sec. 2.4, Algorithm 3): the adjacent modes (a, a+1) with the
// smallest n_a n_{a+1} are merged into one mode whose coefficient is
// Tm = V^T (T_a (x) I + I (x) T_{a+1}) V (merge_modes: perfect shuffle and
// real Schur forms of its 4x4 diagonal blocks); the merged mode's pre- and
// post-transforms become V^T (pre_a (x) pre_{a+1}) and
// (post_a (x) post_{a+1}) V.  T and pre (5 entries, empty = none) and post
// (5 entries, or no entries for none) are replaced by their 4-mode versions
// (post always has 4, the merged mode's V at least), n4 receives the merged
// shape.
int merge_order5(const int64_t* n, std::vector<std::vector<double>>& T, std::vector<std::vector<double>>& pre,
                 std::vector<std::vector<double>>& post, int64_t* n4) {
    int a = 0;
    for (int k = 1; k < 4; ++k)
        if (n[k] * n[k + 1] < n[a] * n[a + 1]) a = k;
    const int64_t na = n[a], nb = n[a + 1], nm = na * nb;
    if (nm > 2048) return fail(TT_EINVAL, "order 5: the two merged modes exceed 2048 rows together");
    std::vector<double> Tm((size_t)(nm * nm)), V((size_t)(nm * nm));
    std::vector<int> perm((size_t)nm);
    std::string err;
    if (nm > 0) {
        int rc = merge_modes((int)na, T[(size_t)a].data(), (int)nb, T[(size_t)a + 1].data(), Tm.data(), V.data(),
                             perm.data(), err);
        if (rc) return fail(rc, err);
    }
    std::vector<double> Vt((size_t)(nm * nm));
    for (int64_t i = 0; i < nm; ++i)
        for (int64_t j = 0; j < nm; ++j) Vt[(size_t)(i * nm + j)] = V[(size_t)(j * nm + i)];
    std::vector<double> pm = (pre[(size_t)a].empty() && pre[(size_t)a + 1].empty())
                                 ? Vt
                                 : matmul_sq(Vt, kron_sq(pre[(size_t)a], na, pre[(size_t)a + 1], nb), nm);
    const bool hp = !post.empty() && !(post[(size_t)a].empty() && post[(size_t)a + 1].empty());
    std::vector<double> qm = hp ? matmul_sq(kron_sq(post[(size_t)a], na, post[(size_t)a + 1], nb), V, nm) : V;
    // the merged mode always has a post-transform (V)
    std::vector<std::vector<double>> T4, pre4, post4;
    for (int k = 0; k < 5; ++k) {
        if (k == a + 1) continue;
        const bool m = (k == a);
        T4.push_back(m ? Tm : T[(size_t)k]);
        pre4.push_back(m ? pm : pre[(size_t)k]);
        post4.push_back(m ? qm : (post.empty() ? std::vector<double>() : post[(size_t)k]));
        n4[(int)T4.size() - 1] = m ? nm : n[k];
    }
    T.swap(T4);
    pre.swap(pre4);
    post.swap(post4);
    return TT_OK;
}

}  // namespace

// Upper bound of the device bytes of one single-problem plan and call (see
// tt_workspace_bytes).  Every term mirrors an allocation of this file with
// the counts the planner can produce for ANY 2x2-block pattern:
//   blocks per mode  m <= ceil(n / b) + 1 (near-equal split, one extra block
//                    when a moved boundary leaves a block over b rows; the
//                    full-block split is taken only when it has no more);
//   leaf edge        <= b + 1 (a near-equal block of ceil(n/m) <= b rows
//                       grows by one when its first boundary moves down
//                       past a 2x2 block; a move up is taken only when the
//                       block stays within b; full blocks have <= b rows);
//   tasks            <= 2 D leaves (types (1) and (2) per block and mode);
//   update tiles     <= tiles of the tasks' (M, P) + 8 padding items a wave,
//                       where per pencil and mode the targets of one tree
//                       level cover at most n rows, for both task types;
//   tuple shapes     distinct tuple counts per mode <= min(m, leaf edge).
// Tables, coefficient copies, block starts, accumulators and status word of
// a plan with leaf edge b (see plan_bound_bytes).
static double plan_tables_bound(int D, const int64_t* nn, int b, double N) {
    auto al = align256;
    size_t coef = 0;
    double L = 1, S = 1, ents = 1, W = 1, lev_rows = 0;
    int64_t m[kMaxD], bm[kMaxD];
    for (int mu = 0; mu < D; ++mu) {
        const int64_t nm = nn[mu];
        m[mu] = (nm == 0) ? 0 : std::min<int64_t>(nm, (nm + b - 1) / b + 1);
        bm[mu] = std::max<int64_t>(1, std::min<int64_t>(nm, b + 1));
        coef += al(sizeof(double) * (size_t)std::max<int64_t>(1, nm * nm)) + al(sizeof(int32_t) * (size_t)(m[mu] + 1));
        L *= (double)m[mu];
        W += (double)std::max<int64_t>(0, m[mu] - 1);
        const int64_t distinct = std::min<int64_t>(m[mu], bm[mu]);
        S *= (double)std::max<int64_t>(1, distinct);
        double tsum = 0;  // sum of the largest `distinct` tuple counts <= bm
        for (int64_t k = 0; k < distinct; ++k) tsum += (double)(bm[mu] - k);
        ents *= std::max(1.0, tsum);
    }
    double Pmax = 1;
    for (int mu = 0; mu < D - 1; ++mu) Pmax *= (double)bm[mu];
    const double tasks = 2.0 * D * L;
    for (int mu = 0; mu < D; ++mu) {
        const double levels = std::log2(std::max<double>(2.0, (double)m[mu])) + 2.0;
        lev_rows += 2.0 * levels * (double)nn[mu] * L / std::max<double>(1.0, (double)m[mu]) / kTile;
    }
    const double items = std::ceil(Pmax / kTile) * (lev_rows + tasks) + 8.0 * W;
    double Hmax = 1;
    for (int mu = 0; mu < D; ++mu) Hmax += (double)bm[mu];
    double bytes = (double)coef + al(sizeof(ProbDesc)) + L * sizeof(LeafDesc) + S * sizeof(LeafShape) +
                   ents * sizeof(uint16_t) + S * (Hmax + 1) * sizeof(int32_t) + tasks * sizeof(UpdDesc) +
                   items * sizeof(WorkItem) + 9 * 256.0;  // alignment of the tables, status word
    bytes += (double)(D - 1) * (double)al((size_t)(8.0 * N));  // update accumulators
    return bytes;
}

size_t plan_bound_bytes(int d, const int64_t* n, int prec) {
    if (d < 1 || d > 4 || !n) return 0;
    const int D = (d == 4) ? 4 : 3;
    int64_t nn[kMaxD] = {1, 1, 1, 1};
    for (int mu = 0; mu < d; ++mu) {
        if (n[mu] < 0) return 0;
        nn[D - d + mu] = n[mu];
    }
    auto al = align256;
    double N = 1;
    size_t mats = 0;
    for (int mu = 0; mu < D; ++mu) {
        N *= (double)nn[mu];
        mats += al(sizeof(double) * (size_t)std::max<int64_t>(1, nn[mu] * nn[mu]));
    }
    if (N == 0) return 4096;
    // Laplace-like, pair, dense and adjoint calls: default leaf edge 16 / 8,
    // plus the largest of their extras: dense pipeline (pre, post, one
    // tensor) with refinement (dense A, residual tensor, norm partial sums),
    // the pair form (pre, one tensor), the adjoint's gradient workspace
    const double tensor = (double)al((size_t)(8.0 * N));
    double general = 2.0 * (double)mats + tensor;
    if (prec != TT_FP64) general += (double)mats + tensor + al(sizeof(double) * 2 * (size_t)sumsq_blocks());
    const double pair = (double)mats + tensor;
    double gtiles = 0;
    for (int mu = 0; mu < D; ++mu) gtiles += std::pow(std::ceil((double)nn[mu] / kGramTile), 2.0);
    const double want = std::max(1.0, std::floor(4096.0 / std::max(1.0, gtiles)));
    double grads = al(sizeof(GramJob) * (size_t)D);
    for (int mu = 0; mu < D; ++mu) {
        if (nn[mu] == 0) continue;
        const double K = N / (double)nn[mu];
        const double ns = std::min(want, std::max(1.0, std::floor(K / 512.0)));
        grads += ns * (double)nn[mu] * (double)nn[mu] * 8.0;
    }
    grads = (double)al((size_t)grads);
    const double lap = plan_tables_bound(D, nn, (D >= 4) ? 8 : 16, N) + std::max(std::max(general, pair), grads);
    // second class: leaf edge 8 / 5, partial products W_1 .. W_{D-2}, pre
    // and post matrices and one pipeline tensor
    const double cls2 = plan_tables_bound(D, nn, (D >= 4) ? 5 : 8, N) + (double)(D - 2) * tensor + 2.0 * (double)mats +
                        tensor;
    return (size_t)std::ceil(std::max(lap, cls2)) + 4096;
}

// Scratch of the allocation-free solve (solve_tri_tensor_noalloc): the
// plan's tables, the update accumulators and the status word.  Each GPU
// holds its own copy from module load until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(void** out) {
    int dev = 0;
    TT_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TT_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        TT_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(TT_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TT_OK;
}

extern "C" {

size_t tt_workspace_bytes(int d, const int64_t* n, int prec) { return plan_bound_bytes(d, n, prec); }

int solve_tri_tensor_noalloc(int d, const int64_t* n, const double* const* T, const double* const* C,
                             const double* B, double* X, tt_opts* opts) {
    tt_opts o;
    tt_opts_default(&o);
    if (opts) o = *opts;
    if (o.prec != TT_FP64) return fail(TT_EINVAL, "the allocation-free solve is FP64 only");
    void* ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    o.workspace = ws;
    o.workspace_bytes = kNoAllocScratchBytes;
    tt_plan p = nullptr;
    t_serial_plan = true;
    rc = tt_plan_create(&p, d, n, T, C, 0, &o);
    t_serial_plan = false;
    if (rc == TT_ENOMEM)
        return fail(TT_EINVAL, std::string("problem too large for the allocation-free solve (64 MiB of scratch): ") +
                                   tt_last_error());
    if (rc) return rc;
    std::unique_ptr<tt_plan_s> guard(p);
    rc = tt_plan_solve(p, B, X, o.stream);
    if (opts) {
        opts->info[0] = opts->info[1] = 0;
        opts->info[2] = p->build_seconds;
    }
    if (rc) return rc;
    return tt_plan_status(p);
}

int tt_opts_default(tt_opts* o) {
    if (!o) return fail(TT_EINVAL, "opts is NULL");
    std::memset(o, 0, sizeof(*o));
    o->nmin = 0;
    o->prec = TT_FP64;
    o->tol = 1e-13;
    o->max_iter = 10;
    o->stream = nullptr;
    return TT_OK;
}

const char* tt_status_str(int s) {
    switch (s) {
        case TT_OK: return "TT_OK";
        case TT_EINVAL: return "TT_EINVAL";
        case TT_ESINGULAR: return "TT_ESINGULAR";
        case TT_ENOMEM: return "TT_ENOMEM";
        case TT_EHIP: return "TT_EHIP";
        case TT_ENOTCONV: return "TT_ENOTCONV";
        default: return "TT_UNKNOWN";
    }
}

const char* tt_last_error(void) { return g_last_error.c_str(); }

int tt_plan_create_batched(tt_plan* out, int count, const int* d, const int64_t* const* n,
                           const double* const* const* T, int trans, const tt_opts* opts) {
    if (!out) return fail(TT_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !d || !n || !T) return fail(TT_EINVAL, "bad batch arguments");
    if (opts && opts->prec != TT_FP64)
        return fail(TT_EINVAL, "batched plans are FP64 only (mixed precision: tt_plan_create, tt_plan_create_general)");
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<tt_plan_s> P(new tt_plan_s());
    adopt_workspace(P.get(), opts);
    P->trans = trans ? 1 : 0;
    P->count = count;
    const int D = internal_order(d, count);
    P->sched.D = D;
    P->sched.probs.resize((size_t)count);
    for (int i = 0; i < count; ++i) {
        if (d[i] == 4 && D != 4) return fail(TT_EINVAL, "internal");
        if (D == 4 && d[i] != 4) return fail(TT_EINVAL, "a batch mixes order 4 with lower orders");
        int rc = describe_problem(d[i], n[i], D, P->sched.probs[(size_t)i]);
        if (rc) return rc;
        if (!T[i]) return fail(TT_EINVAL, "coefficient array is NULL");
        rc = fetch_coefficients(T[i], P->trans, P->sched.probs[(size_t)i]);
        if (rc) return rc;
        P->d_user.push_back(d[i]);
    }
    (void)hipGetDevice(&P->device);
    int rc = finish_plan(P.get(), opts ? opts->nmin : 0);
    if (rc) return rc;
    P->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = P.release();
    return TT_OK;
}

// Pair form: sum_mu X x_1 C_1 .. x_mu A_mu .. x_d C_d = B.  Since
// X x_mu A_mu = (X x_mu C_mu^{-1} A_mu) x_mu C_mu and mode products in
// different modes commute, the operator equals the Laplace-like operator of
// T'_mu = C_mu^{-1} A_mu followed by x_1 C_1 ... x_d C_d.  So
// X = L(T')^{-1} (B x_1 C_1^{-1} ... x_d C_d^{-1}).  T'_mu keeps the
// quasi-triangular pattern of A_mu exactly (row i of C^{-1} starts at column i).
static int pair_reduce(int d, const int64_t* n, std::vector<std::vector<double>>& A,
                       const std::vector<std::vector<double>>& C, std::vector<std::vector<double>>& Cinv) {
    Cinv.assign((size_t)d, {});
    for (int mu = 0; mu < d; ++mu) {
        const int64_t m = n[mu];
        const std::vector<double>& c = C[(size_t)mu];
        for (int64_t i = 0; i < m; ++i) {
            if (c[(size_t)(i * m + i)] == 0.0 || !std::isfinite(c[(size_t)(i * m + i)]))
                return fail(TT_EINVAL, "C has a zero or non-finite diagonal entry");
            for (int64_t j = 0; j < i; ++j)
                if (c[(size_t)(i * m + j)] != 0.0) return fail(TT_EINVAL, "C is not upper triangular");
        }
        // C^{-1} column by column (back-substitution)
        std::vector<double> ci((size_t)(m * m), 0.0);
        for (int64_t j = 0; j < m; ++j) {
            for (int64_t i = j; i >= 0; --i) {
                double acc = (i == j) ? 1.0 : 0.0;
                for (int64_t k = i + 1; k <= j; ++k) acc -= c[(size_t)(i * m + k)] * ci[(size_t)(k * m + j)];
                ci[(size_t)(i * m + j)] = acc / c[(size_t)(i * m + i)];
            }
        }
        // T' = C^{-1} A (rows of C^{-1} start at the diagonal)
        std::vector<double> t((size_t)(m * m), 0.0);
        const std::vector<double>& a = A[(size_t)mu];
        for (int64_t i = 0; i < m; ++i)
            for (int64_t k = i; k < m; ++k) {
                const double f = ci[(size_t)(i * m + k)];
                if (f == 0.0) continue;
                const int64_t j0 = (k >= 1) ? k - 1 : 0;
                for (int64_t j = j0; j < m; ++j) t[(size_t)(i * m + j)] += f * a[(size_t)(k * m + j)];
            }
        A[(size_t)mu] = std::move(t);
        Cinv[(size_t)mu] = std::move(ci);
    }
    return TT_OK;
}


// Order 5 with device coefficients: Laplace-like (C NULL) or pair form (C:
// exact C^{-1} reduction per mode), then the merge of two modes
// (merge_order5) and a 4-mode plan with the merged mode's transforms.
static int plan_order5(tt_plan_s* P, const int64_t* n, const double* const* T, const double* const* C,
                       const tt_opts* opts) {
    for (int mu = 0; mu < 5; ++mu)
        if (n[mu] < 0 || n[mu] > (int64_t)1 << 30) return fail(TT_EINVAL, "mode size out of range");
    if (opts && opts->prec != TT_FP64) return fail(TT_EINVAL, "order 5 is FP64 only");
    std::vector<std::vector<double>> A, Cm, Cinv, pre(5), post;
    int rc;
    if ((rc = fetch_matrices(5, n, T, A))) return rc;
    for (int mu = 0; mu < 5; ++mu) {
        std::vector<int32_t> bst;
        std::string err;
        if (partition_mode(n[mu], A[(size_t)mu].data(), 2, bst, err)) return fail(TT_EINVAL, err);
    }
    if (C) {
        if ((rc = fetch_matrices(5, n, C, Cm))) return rc;
        if ((rc = pair_reduce(5, n, A, Cm, Cinv))) return rc;
        pre = Cinv;
    }
    int64_t n4[4];
    if ((rc = merge_order5(n, A, pre, post, n4))) return rc;
    return pipeline_plan(P, 4, n4, A, pre, post, 0, opts);
}

int tt_plan_create(tt_plan* out, int d, const int64_t* n, const double* const* T,
                   const double* const* C, int trans, const tt_opts* opts) {
    if (d == 5) {
        if (!out) return fail(TT_EINVAL, "out is NULL");
        *out = nullptr;
        if (!T || !n) return fail(TT_EINVAL, "NULL argument");
        if (trans) return fail(TT_EINVAL, "adjoint plans support orders 1 to 4");
        auto t0 = std::chrono::steady_clock::now();
        std::unique_ptr<tt_plan_s> P(new tt_plan_s());
        adopt_workspace(P.get(), opts);
        int rc = plan_order5(P.get(), n, T, C, opts);
        if (rc) return rc;
        P->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = P.release();
        return TT_OK;
    }
    if (!C) {
        if (!out) return fail(TT_EINVAL, "out is NULL");
        *out = nullptr;
        if (!T) return fail(TT_EINVAL, "coefficient array is NULL");
        tt_plan p = nullptr;
        tt_opts o64;
        tt_opts_default(&o64);
        if (opts) o64 = *opts;
        o64.prec = TT_FP64;
        int rc = tt_plan_create_batched(&p, 1, &d, &n, &T, trans, &o64);
        if (rc) return rc;
        std::unique_ptr<tt_plan_s> P(p);
        if (opts && opts->prec != TT_FP64) {
            std::vector<std::vector<double>> Tu;
            if ((rc = fetch_matrices(d, n, T, Tu))) return rc;
            if ((rc = setup_refinement(P.get(), Tu, opts))) return rc;
        }
        *out = P.release();
        return TT_OK;
    }
    if (!out) return fail(TT_EINVAL, "out is NULL");
    *out = nullptr;
    if (trans) return fail(TT_EINVAL, "adjoint plans of the pair form are not supported");
    if (!T) return fail(TT_EINVAL, "coefficient array is NULL");
    if (opts && opts->prec != TT_FP64) return fail(TT_EINVAL, "mixed precision is not supported for the pair form");
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<tt_plan_s> P(new tt_plan_s());
    adopt_workspace(P.get(), opts);
    HostProblem probe;
    int rc = describe_problem(d, n, (d == 4) ? 4 : 3, probe);
    if (rc) return rc;
    std::vector<std::vector<double>> A, Cm, Cinv;
    if ((rc = fetch_matrices(d, n, T, A))) return rc;
    if ((rc = fetch_matrices(d, n, C, Cm))) return rc;
    if ((rc = pair_reduce(d, n, A, Cm, Cinv))) return rc;
    if ((rc = plan_begin(P.get(), d, n, A, 0))) return rc;
    P->kind = KIND_PAIR;
    if ((rc = finish_plan(P.get(), opts ? opts->nmin : 0))) return rc;
    const HostProblem& hp = P->sched.probs[0];
    P->pre.assign((size_t)d, nullptr);
    for (int mu = 0; mu < d; ++mu)
        if ((rc = upload_matrix(P.get(), Cinv[(size_t)mu], &P->pre[(size_t)mu]))) return rc;
    if ((rc = alloc_tensor(P.get(), hp.N, &P->W))) return rc;
    P->pipe_flops = P->sched.stats.flops + chain_flops(P.get(), P->pre);
    P->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = P.release();
    return TT_OK;
}

int tt_plan_create_general(tt_plan* out, int d, const int64_t* n, const double* const* A_host,
                           const tt_opts* opts) {
    if (!out) return fail(TT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!A_host) return fail(TT_EINVAL, "coefficient array is NULL");
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<tt_plan_s> P(new tt_plan_s());
    adopt_workspace(P.get(), opts);
    if (d == 5) {
        // host Schur of every mode, then the merge of two modes (order 5)
        if (!n) return fail(TT_EINVAL, "n is NULL");
        if (opts && opts->prec != TT_FP64) return fail(TT_EINVAL, "order 5 is FP64 only");
        std::vector<std::vector<double>> T(5), U(5), pre(5), post(5);
        std::vector<int> ni(5);
        std::vector<const double*> ap(5);
        std::vector<double*> tp(5), up(5);
        for (int mu = 0; mu < 5; ++mu) {
            if (n[mu] < 0 || n[mu] > 16384) return fail(TT_EINVAL, "mode size out of range");
            if (!A_host[mu] && n[mu] > 0) return fail(TT_EINVAL, "coefficient pointer is NULL");
            T[(size_t)mu].assign((size_t)(n[mu] * n[mu]), 0.0);
            U[(size_t)mu].assign((size_t)(n[mu] * n[mu]), 0.0);
            ni[(size_t)mu] = (int)n[mu];
            ap[(size_t)mu] = A_host[mu];
            tp[(size_t)mu] = T[(size_t)mu].data();
            up[(size_t)mu] = U[(size_t)mu].data();
        }
        std::string err;
        int rc = schur_real_many(5, ni.data(), ap.data(), tp.data(), up.data(), err);
        if (rc) return fail(rc, err);
        P->schur_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int mu = 0; mu < 5; ++mu) {
            const int64_t m = n[mu];
            pre[(size_t)mu].assign((size_t)(m * m), 0.0);
            for (int64_t i = 0; i < m; ++i)
                for (int64_t j = 0; j < m; ++j)
                    pre[(size_t)mu][(size_t)(i * m + j)] = U[(size_t)mu][(size_t)(j * m + i)];
            post[(size_t)mu] = U[(size_t)mu];
        }
        int64_t n4[4];
        if ((rc = merge_order5(n, T, pre, post, n4))) return rc;
        if ((rc = pipeline_plan(P.get(), 4, n4, T, pre, post, 0, opts))) return rc;
        P->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = P.release();
        return TT_OK;
    }
    HostProblem probe;
    int rc = describe_problem(d, n, (d == 4) ? 4 : 3, probe);
    if (rc) return rc;
    std::vector<std::vector<double>> A((size_t)d), T((size_t)d), U((size_t)d), Ut((size_t)d);
    std::vector<int> ni((size_t)d);
    std::vector<const double*> ap((size_t)d);
    std::vector<double*> tp((size_t)d), up((size_t)d);
    for (int mu = 0; mu < d; ++mu) {
        if (n[mu] > 16384) return fail(TT_EINVAL, "mode size too large for the host Schur decomposition");
        if (!A_host[mu] && n[mu] > 0) return fail(TT_EINVAL, "coefficient pointer is NULL");
        const size_t nn = (size_t)(n[mu] * n[mu]);
        A[(size_t)mu].assign(A_host[mu], A_host[mu] + nn);
        T[(size_t)mu].assign(nn, 0.0);
        U[(size_t)mu].assign(nn, 0.0);
        ni[(size_t)mu] = (int)n[mu];
        ap[(size_t)mu] = A[(size_t)mu].data();
        tp[(size_t)mu] = T[(size_t)mu].data();
        up[(size_t)mu] = U[(size_t)mu].data();
    }
    std::string err;
    if ((rc = schur_real_many(d, ni.data(), ap.data(), tp.data(), up.data(), err))) return fail(rc, err);
    P->schur_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int mu = 0; mu < d; ++mu) {
        const int64_t m = n[mu];
        Ut[(size_t)mu].assign((size_t)(m * m), 0.0);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < m; ++j) Ut[(size_t)mu][(size_t)(i * m + j)] = U[(size_t)mu][(size_t)(j * m + i)];
    }
    if ((rc = plan_begin(P.get(), d, n, T, 0))) return rc;
    P->kind = KIND_GENERAL;
    if ((rc = finish_plan(P.get(), opts ? opts->nmin : 0))) return rc;
    const HostProblem& hp = P->sched.probs[0];
    P->pre.assign((size_t)d, nullptr);
    P->post.assign((size_t)d, nullptr);
    for (int mu = 0; mu < d; ++mu) {
        if ((rc = upload_matrix(P.get(), Ut[(size_t)mu], &P->pre[(size_t)mu]))) return rc;
        if ((rc = upload_matrix(P.get(), U[(size_t)mu], &P->post[(size_t)mu]))) return rc;
    }
    if ((rc = alloc_tensor(P.get(), hp.N, &P->W))) return rc;
    if ((rc = setup_refinement(P.get(), A, opts))) return rc;
    P->pipe_flops = P->sched.stats.flops + chain_flops(P.get(), P->pre) + chain_flops(P.get(), P->post);
    P->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = P.release();
    return TT_OK;
}

// Dense pairs (A_mu, C_mu): per mode the QZ decomposition A = Q S Z^T,
// C = Q T Z^T turns the equation into the triangular pair (S_mu, T_mu) for
// X~ = X x_mu Z_mu^T (all modes) with right-hand side B x_mu Q_mu^T, and the
// pair reduction of the triangular pair form into the Laplace-like equation
// with T_mu^{-1} S_mu and right-hand side B x_mu (T_mu^{-1} Q_mu^T).  So the
// GPU runs the dense pipeline with pre-transforms T_mu^{-1} Q_mu^T and
// post-transforms Z_mu.
int tt_plan_create_general_pair(tt_plan* out, int d, const int64_t* n, const double* const* A_host,
                                const double* const* C_host, const tt_opts* opts) {
    if (!out) return fail(TT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!A_host || !C_host) return fail(TT_EINVAL, "coefficient array is NULL");
    if (opts && opts->prec != TT_FP64) return fail(TT_EINVAL, "mixed precision is not supported for the pair form");
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<tt_plan_s> P(new tt_plan_s());
    adopt_workspace(P.get(), opts);
    HostProblem probe;
    int rc = describe_problem(d, n, (d == 4) ? 4 : 3, probe);
    if (rc) return rc;
    std::vector<std::vector<double>> S((size_t)d), T((size_t)d), Q((size_t)d), Z((size_t)d), Tinv;
    for (int mu = 0; mu < d; ++mu) {
        if (n[mu] > 16384) return fail(TT_EINVAL, "mode size too large for the host QZ decomposition");
        if ((!A_host[mu] || !C_host[mu]) && n[mu] > 0) return fail(TT_EINVAL, "coefficient pointer is NULL");
        const size_t nn = (size_t)(n[mu] * n[mu]);
        for (auto* v : {&S, &T, &Q, &Z}) (*v)[(size_t)mu].assign(nn, 0.0);
    }
    {
        std::vector<int> rcs((size_t)d, TT_OK);
        std::vector<std::string> msg((size_t)d);
        std::vector<std::thread> th;
        for (int mu = 0; mu < d; ++mu)
            th.emplace_back([&, mu] {
                rcs[(size_t)mu] = qz_real((int)n[mu], A_host[mu], C_host[mu], S[(size_t)mu].data(),
                                          T[(size_t)mu].data(), Q[(size_t)mu].data(), Z[(size_t)mu].data(),
                                          msg[(size_t)mu]);
            });
        for (auto& t : th) t.join();
        for (int mu = 0; mu < d; ++mu)
            if (rcs[(size_t)mu]) return fail(rcs[(size_t)mu], "mode " + std::to_string(mu) + ": " + msg[(size_t)mu]);
    }
    P->schur_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if ((rc = pair_reduce(d, n, S, T, Tinv))) return rc;  // S <- T^{-1} S
    std::vector<std::vector<double>> pre((size_t)d);
    for (int mu = 0; mu < d; ++mu) {  // pre = T^{-1} Q^T (T^{-1} upper triangular)
        const int64_t m = n[mu];
        const std::vector<double>& ti = Tinv[(size_t)mu];
        const std::vector<double>& q = Q[(size_t)mu];
        std::vector<double>& pm = pre[(size_t)mu];
        pm.assign((size_t)(m * m), 0.0);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t k = i; k < m; ++k) {
                const double f = ti[(size_t)(i * m + k)];
                if (f == 0.0) continue;
                for (int64_t j = 0; j < m; ++j) pm[(size_t)(i * m + j)] += f * q[(size_t)(j * m + k)];
            }
    }
    if ((rc = plan_begin(P.get(), d, n, S, 0))) return rc;
    P->kind = KIND_GENERAL;
    if ((rc = finish_plan(P.get(), opts ? opts->nmin : 0))) return rc;
    const HostProblem& hp = P->sched.probs[0];
    P->pre.assign((size_t)d, nullptr);
    P->post.assign((size_t)d, nullptr);
    for (int mu = 0; mu < d; ++mu) {
        if ((rc = upload_matrix(P.get(), pre[(size_t)mu], &P->pre[(size_t)mu]))) return rc;
        if ((rc = upload_matrix(P.get(), Z[(size_t)mu], &P->post[(size_t)mu]))) return rc;
    }
    if ((rc = alloc_tensor(P.get(), hp.N, &P->W))) return rc;
    P->pipe_flops = P->sched.stats.flops + chain_flops(P.get(), P->pre) + chain_flops(P.get(), P->post);
    P->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = P.release();
    return TT_OK;
}

// Second operator class (Sec. 3, eq. (3.1)) with triangular coefficients,
// after the exact reduction by C^{-1} along mode 1 (C upper triangular, so
// C^{-1} A_1 keeps the quasi-triangular pattern of A_1, and mode products in
// different modes commute):
//   X x_1 (C^{-1} A_1) + X x_2 A_2 .. x_d A_d = B x_1 C^{-1}.
// Orders 1 and 2 are Laplace-like after the reduction (d = 1: the empty
// product is the identity, (C^{-1} A_1 + I) x = C^{-1} b; d = 2: a
// Sylvester equation); orders 3 and 4 use the second-class leaves.
// A[mu], pre[mu]: host row-major; pre: mode products applied to B first
// (empty vectors skip a mode); post likewise after the solve.
static int gsylv_plan(tt_plan_s* P, int d, const int64_t* n, std::vector<std::vector<double>> T,
                      const std::vector<std::vector<double>>& pre, const std::vector<std::vector<double>>& post,
                      const tt_opts* opts) {
    if (d == 1) {
        const int64_t m = n[0];
        for (int64_t i = 0; i < m; ++i) T[0][(size_t)(i * m + i)] += 1.0;
    }
    return pipeline_plan(P, d, n, T, pre, post, (d >= 3) ? 1 : 0, opts);
}

int tt_plan_create_gsylv(tt_plan* out, int d, const int64_t* n, const double* const* A, const double* C,
                         const tt_opts* opts) {
    if (!out) return fail(TT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!A || !C) return fail(TT_EINVAL, "coefficient array is NULL");
    if (opts && opts->prec != TT_FP64) return fail(TT_EINVAL, "the second operator class is FP64 only");
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<tt_plan_s> P(new tt_plan_s());
    adopt_workspace(P.get(), opts);
    HostProblem probe;
    int rc = describe_problem(d, n, (d == 4) ? 4 : 3, probe);
    if (rc) return rc;
    std::vector<std::vector<double>> T, Cm, Cinv;
    if ((rc = fetch_matrices(d, n, A, T))) return rc;
    const double* Cp[1] = {C};
    if ((rc = fetch_matrices(1, n, Cp, Cm))) return rc;
    std::vector<std::vector<double>> T0(1, T[0]);
    if ((rc = pair_reduce(1, n, T0, Cm, Cinv))) return rc;  // T0 <- C^{-1} A_1
    T[0] = T0[0];
    std::vector<std::vector<double>> pre((size_t)d);
    pre[0] = Cinv[0];
    if ((rc = gsylv_plan(P.get(), d, n, T, pre, {}, opts))) return rc;
    P->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = P.release();
    return TT_OK;
}

// Algorithm 4: real generalized Schur decomposition A_1 = Q S Z^T,
// C = Q T Z^T (host QZ) and real Schur decompositions A_mu = U_mu Tq_mu
// U_mu^T (mu >= 2, host); then B~ = B x_1 (T^{-1} Q^T) x_mu U_mu^T, the
// triangular second-class solve with T^{-1} S and Tq_mu, and
// X = X~ x_1 Z x_mu U_mu.
int tt_plan_create_gsylv_general(tt_plan* out, int d, const int64_t* n, const double* const* A_host,
                                 const double* C_host, const tt_opts* opts) {
    if (!out) return fail(TT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!A_host || !C_host) return fail(TT_EINVAL, "coefficient array is NULL");
    if (opts && opts->prec != TT_FP64) return fail(TT_EINVAL, "the second operator class is FP64 only");
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<tt_plan_s> P(new tt_plan_s());
    adopt_workspace(P.get(), opts);
    HostProblem probe;
    int rc = describe_problem(d, n, (d == 4) ? 4 : 3, probe);
    if (rc) return rc;
    for (int mu = 0; mu < d; ++mu) {
        if (n[mu] > 16384) return fail(TT_EINVAL, "mode size too large for the host Schur decomposition");
        if (!A_host[mu] && n[mu] > 0) return fail(TT_EINVAL, "coefficient pointer is NULL");
    }
    const int64_t n0 = n[0];
    const size_t nn0 = (size_t)(n0 * n0);
    std::vector<std::vector<double>> T((size_t)d), pre((size_t)d), post((size_t)d);
    std::vector<double> S(nn0), Tc(nn0), Q(nn0), Z(nn0);
    std::vector<std::vector<double>> U((size_t)d);
    std::vector<int> rcs((size_t)d, TT_OK);
    std::vector<std::string> msg((size_t)d);
    {
        std::vector<std::thread> th;
        th.emplace_back([&] {
            rcs[0] = qz_real((int)n0, A_host[0], C_host, S.data(), Tc.data(), Q.data(), Z.data(), msg[0]);
        });
        for (int mu = 1; mu < d; ++mu)
            th.emplace_back([&, mu] {
                const size_t nn = (size_t)(n[mu] * n[mu]);
                T[(size_t)mu].assign(nn, 0.0);
                U[(size_t)mu].assign(nn, 0.0);
                rcs[(size_t)mu] = schur_real((int)n[mu], A_host[mu], T[(size_t)mu].data(), U[(size_t)mu].data(),
                                             msg[(size_t)mu]);
            });
        for (auto& t : th) t.join();
        for (int mu = 0; mu < d; ++mu)
            if (rcs[(size_t)mu]) return fail(rcs[(size_t)mu], "mode " + std::to_string(mu) + ": " + msg[(size_t)mu]);
    }
    P->schur_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::vector<std::vector<double>> S1(1, S), T1(1, Tc), Tinv;
    if ((rc = pair_reduce(1, n, S1, T1, Tinv))) return rc;  // S <- T^{-1} S
    T[0] = S1[0];
    // pre: mode 1 T^{-1} Q^T, modes mu >= 2 U_mu^T; post: Z, U_mu
    pre[0].assign(nn0, 0.0);
    for (int64_t i = 0; i < n0; ++i)
        for (int64_t k = i; k < n0; ++k) {
            const double f = Tinv[0][(size_t)(i * n0 + k)];
            if (f == 0.0) continue;
            for (int64_t j = 0; j < n0; ++j) pre[0][(size_t)(i * n0 + j)] += f * Q[(size_t)(j * n0 + k)];
        }
    post[0] = Z;
    for (int mu = 1; mu < d; ++mu) {
        const int64_t m = n[mu];
        pre[(size_t)mu].assign((size_t)(m * m), 0.0);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < m; ++j) pre[(size_t)mu][(size_t)(i * m + j)] = U[(size_t)mu][(size_t)(j * m + i)];
        post[(size_t)mu] = U[(size_t)mu];
    }
    if ((rc = gsylv_plan(P.get(), d, n, T, pre, post, opts))) return rc;
    P->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = P.release();
    return TT_OK;
}

int solve_gsylv_tensor(int d, const int64_t* n, const double* const* A, const double* C, const double* B,
                       double* X, tt_opts* opts) {
    tt_plan p = nullptr;
    int rc = tt_plan_create_gsylv(&p, d, n, A, C, opts);
    if (rc) return rc;
    std::unique_ptr<tt_plan_s> guard(p);
    rc = tt_plan_solve(p, B, X, opts ? (hipStream_t)opts->stream : nullptr);
    if (rc) return rc;
    return tt_plan_status(p);
}

int solve_gsylv_general_tensor(int d, const int64_t* n, const double* const* A_host, const double* C_host,
                               const double* B, double* X, tt_opts* opts) {
    tt_plan p = nullptr;
    int rc = tt_plan_create_gsylv_general(&p, d, n, A_host, C_host, opts);
    if (rc) return rc;
    std::unique_ptr<tt_plan_s> guard(p);
    rc = tt_plan_solve(p, B, X, opts ? (hipStream_t)opts->stream : nullptr);
    if (opts) opts->info[2] = p->build_seconds;
    if (rc) return rc;
    return tt_plan_status(p);
}

int tt_plan_solve_batched(tt_plan plan, const double* const* B, double* const* X, void* stream) {
    if (!plan || !B || !X) return fail(TT_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    if (plan->count == 1) return solve_single(plan, B[0], X[0], st);
    TT_HIP_CHECK(launch_zero_int(plan->d_status, 4, st));
    plan->last_stream = st;
    int rc = prepare_inputs(plan, B, X, st);
    if (rc) return rc;
    rc = run_schedule(plan, st);
    if (rc) return rc;
    return finish_outputs(plan, X, st);
}

int tt_plan_solve(tt_plan plan, const double* B, double* X, void* stream) {
    if (!plan) return fail(TT_EINVAL, "plan is NULL");
    if (plan->count != 1) return fail(TT_EINVAL, "batched plan: use tt_plan_solve_batched");
    return solve_single(plan, B, X, (hipStream_t)stream);
}

int tt_copy_device(const double* src, double* dst, int64_t n, void* stream) {
    if (n < 0 || (n > 0 && (!src || !dst))) return fail(TT_EINVAL, "bad copy arguments");
    TT_HIP_CHECK(launch_copy(src, dst, n, (hipStream_t)stream));
    return TT_OK;
}

int tt_plan_solve_graph(tt_plan plan, const double* B, double* X, void* stream) {
    if (!plan) return fail(TT_EINVAL, "plan is NULL");
    if (plan->count != 1 || plan->prec != TT_FP64)
        return fail(TT_EINVAL, "graph solve needs a single-problem FP64 plan");
    hipStream_t st = (hipStream_t)stream;
    if (!st) return fail(TT_EINVAL, "graph solve needs a created stream (the default stream cannot be captured)");
    if (!(plan->gexec && plan->gB == B && plan->gX == X && plan->gst == st)) {
        if (plan->gexec) {
            TT_HIP_CHECK(hipEventSynchronize(plan->gdone));  // its last launch has finished
            (void)hipGraphExecDestroy(plan->gexec);
            plan->gexec = nullptr;
        }
        if (!plan->gdone) TT_HIP_CHECK(hipEventCreateWithFlags(&plan->gdone, hipEventDisableTiming));
        // the launch sequence of one solve (status reset, input copy, every
        // wave's leaf and update launches, the side stream forked and joined
        // by events): kernels and event edges only
        hipGraph_t g = nullptr;
        TT_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const int rc = solve_single(plan, B, X, st);
        const hipError_t ce = hipStreamEndCapture(st, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        TT_HIP_CHECK(ce);
        const hipError_t ie = hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) plan->gexec = nullptr;
        TT_HIP_CHECK(ie);
        plan->gB = B;
        plan->gX = X;
        plan->gst = st;
    }
    plan->last_stream = st;
    TT_HIP_CHECK(hipGraphLaunch(plan->gexec, st));
    TT_HIP_CHECK(hipEventRecord(plan->gdone, st));
    return TT_OK;
}

int tt_plan_info(tt_plan plan, double* out) {
    if (!plan || !out) return fail(TT_EINVAL, "NULL argument");
    out[0] = plan->last_info[0];
    out[1] = plan->last_info[1];
    out[2] = plan->build_seconds;
    out[3] = plan->schur_seconds;
    return TT_OK;
}

// One profiled solve; fills the per-class totals of tt_plan_profile into out
// (when not NULL) and, per wave, six numbers into waves (when not NULL):
// leaf launch start and end, update launch start and end (milliseconds from
// the first leaf launch; -1 for an empty launch), leaf blocks and update tiles.
static int profile_run(tt_plan plan, const double* B, double* X, void* stream, int serial, double* out,
                       double* waves, int64_t cap) {
    if (!plan) return fail(TT_EINVAL, "NULL argument");
    if (plan->count != 1 || plan->kind != KIND_TRI || plan->prec != TT_FP64)
        return fail(TT_EINVAL, "profile needs a single-problem FP64 triangular plan");
    hipStream_t st = (hipStream_t)stream;
    TT_HIP_CHECK(launch_zero_int(plan->d_status, 4, st));
    plan->last_stream = st;
    const size_t W = plan->sched.waves.size();
    ProfEvents pe;
    pe.serial = serial != 0;
    for (auto* v : {&pe.lb, &pe.la, &pe.ub, &pe.ua}) {
        v->resize(W);
        for (auto& e : *v) TT_HIP_CHECK(hipEventCreate(&e));
    }
    int rc = prepare_inputs(plan, &B, &X, st);
    if (!rc) rc = run_schedule(plan, st, &pe);
    if (!rc) rc = finish_outputs(plan, &X, st);
    if (!rc) {
        TT_HIP_CHECK(hipStreamSynchronize(st));
        for (int k = 0; k < 12; ++k) out[k] = 0;
        for (size_t k = 0; k < W; ++k) {
            const Wave& wv = plan->sched.waves[k];
            float ms = 0;
            if (wv.leaf_count > 0) {
                TT_HIP_CHECK(hipEventElapsedTime(&ms, pe.lb[k], pe.la[k]));
                out[0] += ms;
                out[1] += wv.leaf_flops;
                out[2] += wv.leaf_bytes;
                out[3] += 1;
            }
            if (wv.item_count > 0) {
                TT_HIP_CHECK(hipEventElapsedTime(&ms, pe.ub[k], pe.ua[k]));
                out[4] += ms;
                out[5] += wv.upd_flops;
                out[6] += wv.upd_bytes;
                out[7] += 1;
            }
        }
        if (W > 0) {
            float ms = 0;
            TT_HIP_CHECK(hipEventElapsedTime(&ms, pe.lb[0], pe.ua[W - 1]));
            out[8] = ms;  // first leaf start to last update end
        }
        if (waves) {
            for (size_t k = 0; k < W && (int64_t)k < cap; ++k) {
                const Wave& wv = plan->sched.waves[k];
                double* o = waves + 6 * k;
                float a = 0, b = 0;
                o[0] = o[1] = o[2] = o[3] = -1.0;
                if (wv.leaf_count > 0) {
                    TT_HIP_CHECK(hipEventElapsedTime(&a, pe.lb[0], pe.lb[k]));
                    TT_HIP_CHECK(hipEventElapsedTime(&b, pe.lb[0], pe.la[k]));
                    o[0] = a, o[1] = b;
                }
                if (wv.item_count > 0) {
                    TT_HIP_CHECK(hipEventElapsedTime(&a, pe.lb[0], pe.ub[k]));
                    TT_HIP_CHECK(hipEventElapsedTime(&b, pe.lb[0], pe.ua[k]));
                    o[2] = a, o[3] = b;
                }
                o[4] = (double)wv.leaf_count;
                o[5] = (double)wv.item_count;
            }
        }
    }
    for (auto* v : {&pe.lb, &pe.la, &pe.ub, &pe.ua})
        for (auto& e : *v) (void)hipEventDestroy(e);
    return rc;
}

int tt_plan_profile(tt_plan plan, const double* B, double* X, void* stream, int serial, double* out) {
    if (!out) return fail(TT_EINVAL, "NULL argument");
    return profile_run(plan, B, X, stream, serial, out, nullptr, 0);
}

int tt_plan_profile_waves(tt_plan plan, const double* B, double* X, void* stream, int serial, double* waves,
                          int64_t cap) {
    if (!waves || cap < 0) return fail(TT_EINVAL, "NULL argument or negative capacity");
    double tot[12];
    return profile_run(plan, B, X, stream, serial, tot, waves, cap);
}

int tt_plan_status(tt_plan plan) {
    if (!plan) return fail(TT_EINVAL, "plan is NULL");
    TT_HIP_CHECK(hipStreamSynchronize(plan->last_stream));
    int h = 0;
    TT_HIP_CHECK(hipMemcpy(&h, plan->d_status, sizeof(int), hipMemcpyDeviceToHost));
    if (h) return fail(TT_ESINGULAR, "zero pivot or non-finite value in a leaf solve (an eigenvalue sum vanished?)");
    return TT_OK;
}

double tt_plan_flops(tt_plan plan) {
    if (!plan) return 0.0;
    return plan->kind == KIND_TRI ? plan->sched.stats.flops : plan->pipe_flops;
}

int tt_plan_destroy(tt_plan plan) {
    delete plan;
    return TT_OK;
}

static void report(tt_plan_s* P, tt_opts* opts) {
    if (!opts) return;
    opts->info[0] = P->last_info[0];
    opts->info[1] = P->last_info[1];
    opts->info[2] = P->build_seconds;
}

int solve_tri_tensor(int d, const int64_t* n, const double* const* T, const double* const* C,
                     const double* B, double* X, tt_opts* opts) {
    tt_plan p = nullptr;
    int rc = tt_plan_create(&p, d, n, T, C, 0, opts);
    if (rc) return rc;
    std::unique_ptr<tt_plan_s> guard(p);
    hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
    rc = tt_plan_solve(p, B, X, st);
    report(p, opts);
    if (rc) return rc;
    return tt_plan_status(p);
}

int solve_tri_tensor_batched(int count, const int* d, const int64_t* const* n,
                             const double* const* const* T, const double* const* B,
                             double* const* X, tt_opts* opts) {
    tt_plan p = nullptr;
    int rc = tt_plan_create_batched(&p, count, d, n, T, 0, opts);
    if (rc) return rc;
    std::unique_ptr<tt_plan_s> guard(p);
    hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
    rc = tt_plan_solve_batched(p, B, X, st);
    if (rc) return rc;
    return tt_plan_status(p);
}

int solve_general_tensor(int d, const int64_t* n, const double* const* A_host, const double* B,
                         double* X, tt_opts* opts) {
    tt_plan p = nullptr;
    int rc = tt_plan_create_general(&p, d, n, A_host, opts);
    if (rc) return rc;
    std::unique_ptr<tt_plan_s> guard(p);
    hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
    rc = tt_plan_solve(p, B, X, st);
    report(p, opts);
    if (rc) return rc;
    return tt_plan_status(p);
}

// Coefficient gradients of one problem: dT[mu] = -Lam_(mu) X_(mu)^T, masked
// to the pattern of T[mu] unless dense.  W: split-K workspace.
// dT[i][mu] = -Lam_i (mu) X_i (mu)^T (masked unless dense) for every problem i
// with dT[i] != NULL, as two batched launches over all (problem, mode) pairs.
static int grads_batched(tt_plan_s* P, const double* const* const* T, const double* const* X,
                         const double* const* Lam, double* const* const* dT, int dense_grad, hipStream_t st) {
    std::vector<GramJob> jobs;
    int64_t tiles = 0;
    for (int i = 0; i < P->count; ++i) {
        if (!dT[i]) continue;
        const HostProblem& hp = P->sched.probs[(size_t)i];
        if (hp.N == 0) continue;
        if (!T[i] || !X[i] || !Lam[i]) return fail(TT_EINVAL, "tensor or coefficient pointer is NULL");
        const int lead = hp.D - hp.d_user;
        for (int mu = 0; mu < hp.d_user; ++mu) {
            const int n = (int)hp.n[lead + mu];
            if (!dT[i][mu] || n == 0) continue;
            if (!T[i][mu]) return fail(TT_EINVAL, "coefficient pointer is NULL");
            GramJob J{};
            J.P = Lam[i];
            J.Q = X[i];
            J.T = T[i][mu];
            J.out = dT[i][mu];
            J.n = n;
            J.dense = dense_grad;
            J.L = 1;
            J.R = 1;
            for (int nu = 0; nu < hp.d_user; ++nu) {
                if (nu < mu) J.L *= hp.n[lead + nu];
                if (nu > mu) J.R *= hp.n[lead + nu];
            }
            const int nt = (n + kGramTile - 1) / kGramTile;
            tiles += (int64_t)nt * nt;
            jobs.push_back(J);
        }
    }
    if (jobs.empty()) return TT_OK;
    // split K so that the whole batch has ~4096 workgroups, at least 512
    // terms per split
    const int64_t want = std::max<int64_t>(1, 4096 / std::max<int64_t>(tiles, 1));
    int64_t wg = 0, el = 0;
    size_t ws = 0;
    std::vector<size_t> woff;
    for (GramJob& J : jobs) {
        const int64_t K = J.L * J.R;
        int64_t ns = std::min<int64_t>(want, std::max<int64_t>(1, K / 512));
        int64_t kc = (K + ns - 1) / ns;
        kc = (kc + kGramKC - 1) / kGramKC * kGramKC;
        ns = (K + kc - 1) / kc;
        J.nsplit = (int)ns;
        J.kchunk = kc;
        J.wg_first = wg;
        J.el_first = el;
        woff.push_back(ws);
        const int nt = (J.n + kGramTile - 1) / kGramTile;
        wg += (int64_t)nt * nt * ns;
        el += (int64_t)J.n * J.n;
        ws += (size_t)ns * (size_t)J.n * (size_t)J.n;
    }
    if (ws > P->gW_size) {
        // grown only when a call needs more: the old buffer stays with the
        // plan (work already enqueued may still read it), so no
        // synchronisation is needed here
        int rc2 = dev_alloc(P, sizeof(double) * ws, (void**)&P->gW, "gradient split-K workspace");
        if (rc2) return rc2;
        P->gW_size = ws;
    }
    for (size_t j = 0; j < jobs.size(); ++j) jobs[j].W = P->gW + woff[j];
    const int nj = (int)jobs.size();
    if (!P->gJobsEv) TT_HIP_CHECK(hipEventCreateWithFlags(&P->gJobsEv, hipEventDisableTiming));
    TT_HIP_CHECK(hipEventSynchronize(P->gJobsEv));  // the previous upload has read the staging buffer
    if (nj > P->gJobsCap) {
        int rc2 = dev_alloc(P, sizeof(GramJob) * nj, (void**)&P->gJobsDev, "gradient job table");
        if (rc2) return rc2;
        P->gJobsCap = nj;
    }
    P->gJobsHost = jobs;
    TT_HIP_CHECK(hipMemcpyAsync(P->gJobsDev, P->gJobsHost.data(), sizeof(GramJob) * nj, hipMemcpyHostToDevice, st));
    TT_HIP_CHECK(hipEventRecord(P->gJobsEv, st));
    TT_HIP_CHECK(launch_gram_batched(P->gJobsDev, nj, wg, el, -1.0, st));
    return TT_OK;
}

int tt_plan_coefficient_grads(tt_plan plan, const double* const* const* T, const double* const* X,
                              const double* const* Lam, double* const* const* dT, int dense_grad, void* stream) {
    if (!plan || !T || !X || !Lam || !dT) return fail(TT_EINVAL, "NULL argument");
    if (plan->kind != KIND_TRI) return fail(TT_EINVAL, "coefficient gradients need a triangular plan");
    hipStream_t st = (hipStream_t)stream;
    plan->last_stream = st;
    return grads_batched(plan, T, X, Lam, dT, dense_grad, st);
}

int solve_backward_batched(int count, const int* d, const int64_t* const* n,
                           const double* const* const* T, const double* const* X,
                           const double* const* G, double* const* dB, double* const* const* dT,
                           int dense_grad, tt_opts* opts) {
    if (count < 1 || !d || !n || !T || !G || !dB) return fail(TT_EINVAL, "NULL argument");
    if (dT && !X) return fail(TT_EINVAL, "X is needed for the coefficient gradients");
    tt_plan p = nullptr;
    int rc = tt_plan_create_batched(&p, count, d, n, T, 1, opts);
    if (rc) return rc;
    std::unique_ptr<tt_plan_s> guard(p);
    hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
    // Lam: sum_mu Lam x_mu T_mu^T = G, into dB
    if ((rc = tt_plan_solve_batched(p, G, dB, st))) return rc;
    if (dT) {
        if (!X) return fail(TT_EINVAL, "X is needed for the coefficient gradients");
        if ((rc = grads_batched(p, T, X, (const double* const*)dB, dT, dense_grad, st))) return rc;
    }
    return tt_plan_status(p);
}

int solve_backward(int d, const int64_t* n, const double* const* T, const double* X,
                   const double* G, double* dB, double* const* dT, int dense_grad, tt_opts* opts) {
    const double* const* Tb[1] = {T};
    const double* Xb[1] = {X};
    const double* Gb[1] = {G};
    double* dBb[1] = {dB};
    double* const* dTb[1] = {dT};
    return solve_backward_batched(1, &d, &n, Tb, Xb, Gb, dBb, dT ? dTb : nullptr, dense_grad, opts);
}

// Host-only real Schur decomposition (the host step of solve_general_tensor).
int tt_schur_host(int n, const double* A, double* T, double* U) {
    if (n < 0 || (n > 0 && (!A || !T || !U))) return fail(TT_EINVAL, "bad arguments");
    std::string err;
    int rc = schur_real(n, A, T, U, err);
    if (rc) return fail(rc, err);
    return TT_OK;
}

int tt_merge_modes_host(int na, const double* Ta, int nb, const double* Tb, double* Tm, double* V, int* perm) {
    if (na < 0 || nb < 0 || (int64_t)na * nb > 4096) return fail(TT_EINVAL, "bad sizes");
    if (na * nb > 0 && (!Ta || !Tb || !Tm || !V || !perm)) return fail(TT_EINVAL, "NULL argument");
    for (int k = 0; k < 2; ++k) {
        std::vector<int32_t> bst;
        std::string err;
        if (partition_mode(k ? nb : na, k ? Tb : Ta, 2, bst, err)) return fail(TT_EINVAL, err);
    }
    std::string err;
    int rc = merge_modes(na, Ta, nb, Tb, Tm, V, perm, err);
    if (rc) return fail(rc, err);
    return TT_OK;
}

int tt_qz_host(int n, const double* A, const double* C, double* S, double* T, double* Q, double* Z) {
    if (n < 0 || (n > 0 && (!A || !C || !S || !T || !Q || !Z))) return fail(TT_EINVAL, "bad arguments");
    std::string err;
    int rc = qz_real(n, A, C, S, T, Q, Z, err);
    if (rc) return fail(rc, err);
    return TT_OK;
}

// Host-only schedule query (no GPU calls): builds the plan of a problem with
// HOST coefficients and reports its statistics.  out[0..12] = flops,
// flops_leaf, flops_update, waves, leaves, tasks, work items, launches,
// bmax[0..3], dependency check (0 = the schedule respects every dependency).
int tt_schedule_info(int d, const int64_t* n, const double* const* T_host, int nmin, double* out) {
    return tt_schedule_info_class(d, n, T_host, nmin, 0, out);
}

int tt_schedule_info_class(int d, const int64_t* n, const double* const* T_host, int nmin, int cls, double* out) {
    if (!out || !T_host) return fail(TT_EINVAL, "NULL argument");
    if (cls != 0 && cls != 1) return fail(TT_EINVAL, "cls must be 0 (Laplace-like) or 1 (second class)");
    Schedule s;
    s.D = (d == 4) ? 4 : 3;
    s.cls = cls;
    s.probs.resize(1);
    int rc = describe_problem(d, n, s.D, s.probs[0]);
    if (rc) return rc;
    HostProblem& hp = s.probs[0];
    const int lead = s.D - d;
    for (int mu = 0; mu < s.D; ++mu) {
        int64_t nm = hp.n[mu];
        hp.T[mu].assign((size_t)(nm * nm), 0.0);
        if (mu >= lead && nm > 0) {
            if (!T_host[mu - lead]) return fail(TT_EINVAL, "coefficient is NULL");
            std::memcpy(hp.T[mu].data(), T_host[mu - lead], sizeof(double) * (size_t)(nm * nm));
        }
    }
    std::string err;
    rc = build_schedule(s, nmin, err);
    if (rc) return fail(rc, err);
    const PlanStats& st = s.stats;
    out[0] = st.flops;
    out[1] = st.flops_leaf;
    out[2] = st.flops_update;
    out[3] = (double)st.waves;
    out[4] = (double)st.leaves;
    out[5] = (double)st.tasks;
    out[6] = (double)st.items;
    out[7] = (double)st.launches;  // two per wave (leaf + update)
    for (int mu = 0; mu < 4; ++mu) out[8 + mu] = st.bmax[mu];
    out[13] = (double)plan_table_bytes(s);
    // Dependency check: replay the waves.  In wave k the updates (ready
    // after wave k-1) run concurrently with the leaves of wave k, so an update
    // must read only blocks solved before wave k and write only blocks of
    // waves > k; a leaf needs every block after it along each mode solved and
    // every contribution except the adjacent block's delivered.
    const int D = s.D;
    int64_t total = 1;
    for (int mu = 0; mu < D; ++mu) total *= hp.m[mu];
    std::vector<int> solved((size_t)total, 0);
    // per (block, mode): delivered source blocks, their index sum and
    // square sum (a source delivered twice and another never is caught)
    std::vector<int> pending((size_t)total * D, 0);
    std::vector<int64_t> psum((size_t)total * D, 0), psq((size_t)total * D, 0);
    auto lin = [&](const int* I) {
        int64_t l = 0;
        for (int mu = 0; mu < D; ++mu) l = l * hp.m[mu] + I[mu];
        return l;
    };
    auto wave_of = [&](const int* I) {
        int64_t w = 0;
        for (int mu = 0; mu < D; ++mu) w += hp.m[mu] - 1 - I[mu];
        return w;
    };
    auto find_blk = [&](int nu, int64_t idx) {
        int b = 0;
        while (b <= hp.m[nu] && hp.bst[nu][b] != idx) ++b;
        return b;
    };
    int bad = 0;
    std::vector<uint8_t> task_seen(s.tasks.size(), 0);
    for (size_t k = 0; k < s.waves.size(); ++k) {
        const Wave& wv = s.waves[k];
        std::vector<int32_t> seen_tasks;  // tasks of this wave already replayed (tiles interleave)
        struct Delivery {
            int64_t at;
            int slo, shi;
        };
        std::vector<Delivery> deliveries;
        for (int64_t q = 0; q < wv.item_count && !bad; ++q) {
            const WorkItem& w = s.items[(size_t)(wv.item_first + q)];
            if (w.task < 0) continue;  // padding
            if ((size_t)w.task >= s.tasks.size()) { bad = 1; break; }
            // a 16 x 256 tile serves tasks w.task .. w.task + w.tb, which
            // must differ in their pencil only
            const UpdDesc& t0 = s.tasks[(size_t)w.task];
            const int npk = (t0.M <= 16) ? w.tb + 1 : 1;
            if (npk < 1 || npk > upd_wide_slots(t0.P) || (size_t)w.task + npk > s.tasks.size()) { bad = 1; break; }
            for (int j = 1; j < npk; ++j) {
                const UpdDesc& tj = s.tasks[(size_t)(w.task + j)];
                if (tj.prob != t0.prob || tj.mode != t0.mode || tj.r0 != t0.r0 || tj.M != t0.M || tj.k0 != t0.k0 ||
                    tj.K != t0.K || tj.P != t0.P || (tj.flags & 1) != (t0.flags & 1))
                    bad = 1;
            }
            for (int j = 0; j < npk && !bad; ++j) {
                const int32_t ti = w.task + j;
                if (task_seen[(size_t)ti]) continue;
                task_seen[(size_t)ti] = 1;
                seen_tasks.push_back(ti);
                const UpdDesc& t = s.tasks[(size_t)ti];
                const int mu = t.mode;
                int I[kMaxD];
                int64_t rem = t.xbase;
                for (int nu = 0; nu < D; ++nu) {
                    if (nu == mu) { I[nu] = 0; continue; }
                    int64_t idx = rem / hp.stride[nu];
                    rem -= idx * hp.stride[nu];
                    I[nu] = find_blk(nu, idx);
                    if (I[nu] >= hp.m[nu]) bad = 1;
                }
                if (bad) break;
                const int lo = find_blk(mu, t.r0), hi_t = find_blk(mu, t.r0 + t.M);
                const int slo = find_blk(mu, t.k0), shi = find_blk(mu, t.k0 + t.K);
                if (hi_t > hp.m[mu] || shi > hp.m[mu] || hi_t > slo) { bad = 1; break; }
                for (int b = slo; b < shi; ++b) {
                    I[mu] = b;
                    if (!solved[(size_t)lin(I)]) bad = 1;
                }
                for (int b = lo; b < hi_t; ++b) {
                    I[mu] = b;
                    if (solved[(size_t)lin(I)] || wave_of(I) <= (int64_t)k) bad = 1;
                    deliveries.push_back({lin(I) * D + mu, slo, shi});
                }
            }
        }
        for (int32_t t : seen_tasks) task_seen[(size_t)t] = 0;
        if (bad) break;
        for (int64_t q = 0; q < wv.leaf_count; ++q) {
            const LeafDesc& lf = s.leaves[(size_t)(wv.leaf_first + q)];
            int I[kMaxD];
            for (int mu = 0; mu < D; ++mu) I[mu] = lf.blk[mu];
            if (wave_of(I) != (int64_t)k) bad = 1;
            for (int mu = 0; mu < D; ++mu) {
                int J[kMaxD];
                std::memcpy(J, I, sizeof(J));
                for (int c = I[mu] + 1; c < hp.m[mu]; ++c) {
                    J[mu] = c;
                    if (!solved[(size_t)lin(J)]) bad = 1;
                }
                const int adj = (I[mu] + 1 < hp.m[mu]) ? 1 : 0;
                if (((lf.flags >> (4 + mu)) & 1) != adj) bad = 1;
                const size_t at = (size_t)lin(I) * D + mu;
                if (pending[at] + adj != hp.m[mu] - 1 - I[mu]) bad = 1;
                int64_t es = 0, eq = 0;  // sources I+2 .. m-1
                for (int64_t b = I[mu] + 2; b < hp.m[mu]; ++b) {
                    es += b;
                    eq += b * b;
                }
                if (psum[at] != es || psq[at] != eq) bad = 1;
                // bit 0: right-hand side in X (mode-0 updates arrived); bits mu >= 1: accumulators
                if (((lf.flags >> mu) & 1) != (pending[(size_t)lin(I) * D + mu] > 0 ? 1 : 0)) bad = 1;
            }
        }
        for (int64_t q = 0; q < wv.leaf_count; ++q) {
            const LeafDesc& lf = s.leaves[(size_t)(wv.leaf_first + q)];
            int I[kMaxD];
            for (int mu = 0; mu < D; ++mu) I[mu] = lf.blk[mu];
            solved[(size_t)lin(I)] = 1;
        }
        // the updates of this wave complete before the next wave
        for (const Delivery& dv : deliveries) {
            pending[(size_t)dv.at] += dv.shi - dv.slo;
            for (int64_t b = dv.slo; b < dv.shi; ++b) {
                psum[(size_t)dv.at] += b;
                psq[(size_t)dv.at] += b * b;
            }
        }
    }
    for (int64_t k = 0; k < total; ++k)
        if (!solved[(size_t)k]) bad = 1;
    // every task's output tiles appear exactly once (the items of a wave are
    // interleaved over the XCDs and padded with task -1)
    {
        std::vector<std::vector<uint8_t>> hit(s.tasks.size());
        std::vector<int> tiles_b(s.tasks.size(), 1);
        for (size_t ti = 0; ti < s.tasks.size(); ++ti) {
            const UpdDesc& t = s.tasks[ti];
            const bool right = (t.mode == D - 1);
            int na = 1, nb = 1;
            upd_tile_grid(t, right, na, nb);
            hit[ti].assign((size_t)na * nb, 0);
            tiles_b[ti] = nb;
        }
        for (const WorkItem& w : s.items) {
            if (w.task < 0) continue;
            if ((size_t)w.task >= s.tasks.size()) { bad = 1; break; }
            const bool wide = s.tasks[(size_t)w.task].M <= 16;
            const int npk = wide ? w.tb + 1 : 1, tb = wide ? 0 : w.tb;
            if (npk < 1 || (size_t)w.task + npk > s.tasks.size()) { bad = 1; break; }
            for (int j = 0; j < npk; ++j) {
                auto& h = hit[(size_t)(w.task + j)];
                const int nb = tiles_b[(size_t)(w.task + j)];
                const size_t at = (size_t)w.ta * nb + tb;
                if (w.ta < 0 || tb < 0 || tb >= nb || at >= h.size() || h[at]) { bad = 1; break; }
                h[at] = 1;
            }
            if (bad) break;
        }
        for (const auto& h : hit)
            for (uint8_t v : h)
                if (!v) bad = 1;
    }
    out[12] = bad;
    return TT_OK;
}

}  // extern "C"
