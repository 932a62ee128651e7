// C ABI of the solver (declared in include/tt.h): argument validation, plan
// construction (host) and the ordered launch sequence on one HIP stream.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
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
};

__global__ void set_x_ptrs_kernel(ProbDesc* probs, PtrPack pack, int first, int count) {
    int i = threadIdx.x;
    if (i < count) probs[first + i].X = pack.p[i];
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

struct tt_plan_s {
    Schedule sched;
    int trans = 0;
    int count = 0;
    std::vector<int> d_user;
    // device
    ProbDesc* d_probs = nullptr;
    LeafDesc* d_leaves = nullptr;
    UpdDesc* d_tasks = nullptr;
    WorkItem* d_items = nullptr;
    int* d_status = nullptr;
    std::vector<void*> owned;  // T copies, block-start arrays, accumulators
    hipStream_t side = nullptr;  // stream of the update launches
    std::vector<hipEvent_t> evL, evU;
    hipEvent_t ev_start = nullptr;
    hipStream_t last_stream = nullptr;
    double build_seconds = 0;
    int device = 0;

    ~tt_plan_s() {
        if (side) (void)hipStreamSynchronize(side);
        for (hipEvent_t e : evL) (void)hipEventDestroy(e);
        for (hipEvent_t e : evU) (void)hipEventDestroy(e);
        if (ev_start) (void)hipEventDestroy(ev_start);
        if (side) (void)hipStreamDestroy(side);
        for (void* p : owned) (void)hipFree(p);
        if (d_probs) (void)hipFree(d_probs);
        if (d_leaves) (void)hipFree(d_leaves);
        if (d_tasks) (void)hipFree(d_tasks);
        if (d_items) (void)hipFree(d_items);
        if (d_status) (void)hipFree(d_status);
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

int fetch_coefficients(const double* const* T, int trans, HostProblem& hp) {
    const int lead = hp.D - hp.d_user;
    for (int mu = 0; mu < hp.D; ++mu) {
        const int64_t nm = hp.n[mu];
        hp.T[mu].assign((size_t)(nm * nm), 0.0);
        if (mu < lead) continue;
        const double* src = T[mu - lead];
        if (!src && nm > 0) return fail(TT_EINVAL, "coefficient pointer is NULL");
        if (nm == 0) continue;
        std::vector<double> tmp((size_t)(nm * nm));
        TT_HIP_CHECK(hipMemcpy(tmp.data(), src, sizeof(double) * (size_t)(nm * nm), hipMemcpyDeviceToHost));
        if (!trans) {
            hp.T[mu] = std::move(tmp);
        } else {
            // adjoint: sum L x_mu T^T = G becomes an upper quasi-triangular
            // system in reversed index order with T'[i][j] = T[n-1-j][n-1-i]
            for (int64_t i = 0; i < nm; ++i)
                for (int64_t j = 0; j < nm; ++j) hp.T[mu][i * nm + j] = tmp[(nm - 1 - j) * nm + (nm - 1 - i)];
        }
    }
    return TT_OK;
}

template <typename V>
int upload(const std::vector<V>& v, V** dst) {
    *dst = nullptr;
    if (v.empty()) return TT_OK;
    if (hipMalloc((void**)dst, sizeof(V) * v.size()) != hipSuccess) return fail(TT_ENOMEM, "hipMalloc failed");
    TT_HIP_CHECK(hipMemcpy(*dst, v.data(), sizeof(V) * v.size(), hipMemcpyHostToDevice));
    return TT_OK;
}

int finish_plan(tt_plan_s* P, int nmin) {
    std::string err;
    int rc = build_schedule(P->sched, nmin, err);
    if (rc) return fail(rc, err);
    Schedule& s = P->sched;
    std::vector<ProbDesc> pd(s.probs.size());
    for (size_t i = 0; i < s.probs.size(); ++i) {
        HostProblem& hp = s.probs[i];
        ProbDesc& d = pd[i];
        std::memset(&d, 0, sizeof(d));
        for (int mu = 0; mu < kMaxD; ++mu) {
            d.n[mu] = (mu < s.D) ? hp.n[mu] : 1;
            d.stride[mu] = (mu < s.D) ? hp.stride[mu] : 0;
        }
        for (int mu = 0; mu < s.D; ++mu) {
            double* t = nullptr;
            int32_t* b = nullptr;
            size_t tb = sizeof(double) * std::max<size_t>(1, hp.T[mu].size());
            if (hipMalloc((void**)&t, tb) != hipSuccess) return fail(TT_ENOMEM, "hipMalloc failed");
            P->owned.push_back(t);
            if (!hp.T[mu].empty())
                TT_HIP_CHECK(hipMemcpy(t, hp.T[mu].data(), sizeof(double) * hp.T[mu].size(), hipMemcpyHostToDevice));
            if (hipMalloc((void**)&b, sizeof(int32_t) * hp.bst[mu].size()) != hipSuccess)
                return fail(TT_ENOMEM, "hipMalloc failed");
            P->owned.push_back(b);
            TT_HIP_CHECK(hipMemcpy(b, hp.bst[mu].data(), sizeof(int32_t) * hp.bst[mu].size(), hipMemcpyHostToDevice));
            d.T[mu] = t;
            d.bst[mu] = b;
            // accumulator of the updates of mode mu (mode 0 updates X itself)
            if (mu >= 1 && hp.N > 0) {
                double* acc = nullptr;
                if (hipMalloc((void**)&acc, sizeof(double) * (size_t)hp.N) != hipSuccess)
                    return fail(TT_ENOMEM, "hipMalloc failed (update accumulators)");
                P->owned.push_back(acc);
                d.A[mu] = acc;
            }
        }
    }
    if ((rc = upload(pd, &P->d_probs))) return rc;
    if ((rc = upload(s.leaves, &P->d_leaves))) return rc;
    if ((rc = upload(s.tasks, &P->d_tasks))) return rc;
    if ((rc = upload(s.items, &P->d_items))) return rc;
    if (hipMalloc((void**)&P->d_status, sizeof(int) * 4) != hipSuccess) return fail(TT_ENOMEM, "hipMalloc failed");
    TT_HIP_CHECK(hipMemset(P->d_status, 0, sizeof(int) * 4));
    TT_HIP_CHECK(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking));
    P->evL.resize(s.waves.size());
    P->evU.resize(s.waves.size());
    for (auto& e : P->evL) TT_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& e : P->evU) TT_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    TT_HIP_CHECK(hipEventCreateWithFlags(&P->ev_start, hipEventDisableTiming));
    return TT_OK;
}

int set_pointers(tt_plan_s* P, double* const* X, int count, hipStream_t st) {
    for (int first = 0; first < count; first += 64) {
        PtrPack pack;
        int c = std::min(64, count - first);
        for (int i = 0; i < c; ++i) pack.p[i] = X[first + i];
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
};

int run_schedule(tt_plan_s* P, hipStream_t st, ProfEvents* prof = nullptr) {
    Schedule& s = P->sched;
    TT_HIP_CHECK(launch_zero_int(P->d_status, 4, st));
    TT_HIP_CHECK(hipEventRecord(P->ev_start, st));
    TT_HIP_CHECK(hipStreamWaitEvent(P->side, P->ev_start, 0));
    const size_t W = s.waves.size();
    for (size_t k = 0; k < W; ++k) {
        const Wave& wv = s.waves[k];
        if (k >= 1) TT_HIP_CHECK(hipStreamWaitEvent(st, P->evU[k - 1], 0));
        if (prof) TT_HIP_CHECK(hipEventRecord(prof->lb[k], st));
        TT_HIP_CHECK(launch_leaf(s.D, P->d_leaves, wv.leaf_first, wv.leaf_count, P->d_probs, P->d_status,
                                 s.bmax, s.leaf_lds_bytes, st));
        if (prof) TT_HIP_CHECK(hipEventRecord(prof->la[k], st));
        TT_HIP_CHECK(hipEventRecord(P->evL[k], st));
        if (k >= 1) TT_HIP_CHECK(hipStreamWaitEvent(P->side, P->evL[k - 1], 0));
        if (prof) TT_HIP_CHECK(hipEventRecord(prof->ub[k], P->side));
        TT_HIP_CHECK(launch_update(s.D, P->d_tasks, P->d_items, wv.item_first, wv.item_count, P->d_probs,
                                   P->side));
        if (prof) TT_HIP_CHECK(hipEventRecord(prof->ua[k], P->side));
        TT_HIP_CHECK(hipEventRecord(P->evU[k], P->side));
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
            if (B[i] != X[i]) TT_HIP_CHECK(launch_copy(B[i], X[i], hp.N, st));
        } else {
            if (B[i] != X[i]) {
                hipLaunchKernelGGL(reverse_copy_kernel, dim3(grid_for(hp.N)), dim3(256), 0, st, B[i], X[i], hp.N);
            } else {
                hipLaunchKernelGGL(reverse_inplace_kernel, dim3(grid_for(hp.N)), dim3(256), 0, st, X[i], hp.N);
            }
            TT_HIP_CHECK(hipGetLastError());
        }
    }
    return set_pointers(P, X, P->count, st);
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

}  // namespace

extern "C" {

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
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<tt_plan_s> P(new tt_plan_s());
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

int tt_plan_create(tt_plan* out, int d, const int64_t* n, const double* const* T,
                   const double* const* C, int trans, const tt_opts* opts) {
    if (C) return fail(TT_EINVAL, "pair form (C != NULL) is not supported by plans");
    return tt_plan_create_batched(out, 1, &d, &n, &T, trans, opts);
}

int tt_plan_solve_batched(tt_plan plan, const double* const* B, double* const* X, void* stream) {
    if (!plan || !B || !X) return fail(TT_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    int rc = prepare_inputs(plan, B, X, st);
    if (rc) return rc;
    rc = run_schedule(plan, st);
    if (rc) return rc;
    return finish_outputs(plan, X, st);
}

int tt_plan_solve(tt_plan plan, const double* B, double* X, void* stream) {
    if (!plan) return fail(TT_EINVAL, "plan is NULL");
    if (plan->count != 1) return fail(TT_EINVAL, "batched plan: use tt_plan_solve_batched");
    return tt_plan_solve_batched(plan, &B, &X, stream);
}

int tt_plan_profile(tt_plan plan, const double* B, double* X, void* stream, double* out) {
    if (!plan || !out) return fail(TT_EINVAL, "NULL argument");
    if (plan->count != 1) return fail(TT_EINVAL, "profile needs a single-problem plan");
    hipStream_t st = (hipStream_t)stream;
    const size_t W = plan->sched.waves.size();
    ProfEvents pe;
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
            TT_HIP_CHECK(hipEventElapsedTime(&ms, pe.lb[0], pe.la[W - 1]));
            out[8] = ms;  // first leaf start to last leaf end
        }
    }
    for (auto* v : {&pe.lb, &pe.la, &pe.ub, &pe.ua})
        for (auto& e : *v) (void)hipEventDestroy(e);
    return rc;
}

int tt_plan_status(tt_plan plan) {
    if (!plan) return fail(TT_EINVAL, "plan is NULL");
    TT_HIP_CHECK(hipStreamSynchronize(plan->last_stream));
    int h = 0;
    TT_HIP_CHECK(hipMemcpy(&h, plan->d_status, sizeof(int), hipMemcpyDeviceToHost));
    if (h) return fail(TT_ESINGULAR, "zero pivot or non-finite value in a leaf solve (an eigenvalue sum vanished?)");
    return TT_OK;
}

double tt_plan_flops(tt_plan plan) { return plan ? plan->sched.stats.flops : 0.0; }

int tt_plan_destroy(tt_plan plan) {
    delete plan;
    return TT_OK;
}

int solve_tri_tensor(int d, const int64_t* n, const double* const* T, const double* const* C,
                     const double* B, double* X, tt_opts* opts) {
    if (C) return fail(TT_EINVAL, "pair form is not available in this build");
    tt_plan p = nullptr;
    int rc = tt_plan_create(&p, d, n, T, nullptr, 0, opts);
    if (rc) return rc;
    std::unique_ptr<tt_plan_s> guard(p);
    hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
    if (opts) opts->info[2] = p->build_seconds;
    rc = tt_plan_solve(p, B, X, st);
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
    (void)d; (void)n; (void)A_host; (void)B; (void)X; (void)opts;
    return fail(TT_EINVAL, "solve_general_tensor is not available in this build");
}

int solve_backward(int d, const int64_t* n, const double* const* T, const double* X,
                   const double* G, double* dB, double* const* dT, int dense_grad, tt_opts* opts) {
    (void)d; (void)n; (void)T; (void)X; (void)G; (void)dB; (void)dT; (void)dense_grad; (void)opts;
    return fail(TT_EINVAL, "solve_backward is not available in this build");
}

int solve_backward_batched(int count, const int* d, const int64_t* const* n,
                           const double* const* const* T, const double* const* X,
                           const double* const* G, double* const* dB, double* const* const* dT,
                           int dense_grad, tt_opts* opts) {
    (void)count; (void)d; (void)n; (void)T; (void)X; (void)G; (void)dB; (void)dT; (void)dense_grad;
    (void)opts;
    return fail(TT_EINVAL, "solve_backward_batched is not available in this build");
}

// Host-only schedule query (no GPU calls): builds the plan of a problem with
// HOST coefficients and reports its statistics.  out[0..12] = flops,
// flops_leaf, flops_update, waves, leaves, tasks, work items, launches,
// bmax[0..3], dependency check (0 = the schedule respects every dependency).
int tt_schedule_info(int d, const int64_t* n, const double* const* T_host, int nmin, double* out) {
    if (!out || !T_host) return fail(TT_EINVAL, "NULL argument");
    Schedule s;
    s.D = (d == 4) ? 4 : 3;
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
    // Dependency check: replay the waves.  In wave k the updates (ready
    // after wave k-1) run concurrently with the leaves of wave k, so an update
    // must read only blocks solved before wave k and write only blocks of
    // waves > k; a leaf needs every block after it along each mode solved and
    // every contribution except the adjacent block's delivered.
    const int D = s.D;
    int64_t total = 1;
    for (int mu = 0; mu < D; ++mu) total *= hp.m[mu];
    std::vector<int> solved((size_t)total, 0);
    std::vector<int> pending((size_t)total * D, 0);
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
    for (size_t k = 0; k < s.waves.size(); ++k) {
        const Wave& wv = s.waves[k];
        int64_t last_task = -1;
        std::vector<std::pair<int64_t, int>> deliveries;
        for (int64_t q = 0; q < wv.item_count; ++q) {
            const WorkItem& w = s.items[(size_t)(wv.item_first + q)];
            if (w.task == last_task) continue;
            last_task = w.task;
            const UpdDesc& t = s.tasks[(size_t)w.task];
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
                deliveries.push_back({lin(I) * D + mu, shi - slo});
            }
        }
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
                if (pending[(size_t)lin(I) * D + mu] + adj != hp.m[mu] - 1 - I[mu]) bad = 1;
                if (mu >= 1 && (((lf.flags >> mu) & 1) != (pending[(size_t)lin(I) * D + mu] > 0 ? 1 : 0))) bad = 1;
            }
        }
        for (int64_t q = 0; q < wv.leaf_count; ++q) {
            const LeafDesc& lf = s.leaves[(size_t)(wv.leaf_first + q)];
            int I[kMaxD];
            for (int mu = 0; mu < D; ++mu) I[mu] = lf.blk[mu];
            solved[(size_t)lin(I)] = 1;
        }
        // the updates of this wave complete before the next wave
        for (auto& dv : deliveries) pending[(size_t)dv.first] += dv.second;
    }
    for (int64_t k = 0; k < total; ++k)
        if (!solved[(size_t)k]) bad = 1;
    out[12] = bad;
    return TT_OK;
}

}  // extern "C"
