// Host planner: leaf-block partition, hyperplane waves and the dyadic update
// schedule of the recursive triangular solve.
//
// Algorithm 2 of the paper splits the largest mode at k ~ n_mu/2 (moving k by
// one when A_mu(k+1,k) != 0, Sec. 2.1), solves the upper half, updates the
// lower half with X_2 x_mu A_mu(1:k, k+1:n_mu), and recurses down to blocks of
// size n_min.  Unrolled, every coefficient entry T_mu[i, j] (j past i's
// diagonal block) is applied exactly once, either inside a leaf (i and j in
// the same leaf block) or by the update of the unique split that separates
// their blocks.  Along each mode those splits form a binary tree over the
// leaf-block indices: the split with midpoint c (c = 1, 2, 3, ...) separates
// R0 = [c - s, c) from R1 = [c, c + s) where s is the lowest set bit of c.
//
// Any order that solves a block after everything it depends on gives the same
// X (the solution is unique).  The GPU schedule therefore runs the leaves as
// hyperplane wavefronts over the block grid (block I depends only on blocks
// that are larger in one index and equal in the others, all on earlier
// hyperplanes) and applies each split's update per pencil -- the line of
// blocks along mode mu through I -- as soon as the block at its midpoint c
// is solved.  At that moment all of R1 is solved and no block of R0 is, so
// the update is exactly the one of Algorithm 2, restricted to one pencil.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>

#include "tt_internal.h"

namespace tt {

int partition_mode(int64_t n, const double* T, int b, std::vector<int32_t>& bst, std::string& err) {
    bst.clear();
    if (n <= 0) {
        bst.push_back(0);
        return TT_OK;
    }
    // structure: zero below the first subdiagonal, no two consecutive bumps
    for (int64_t r = 2; r < n; ++r)
        for (int64_t c = 0; c + 1 < r; ++c)
            if (T[r * n + c] != 0.0) {
                err = "coefficient is not upper quasi-triangular: nonzero entry below the subdiagonal at (" +
                      std::to_string(r) + "," + std::to_string(c) + ")";
                return TT_EINVAL;
            }
    for (int64_t i = 1; i + 1 < n; ++i)
        if (T[i * n + i - 1] != 0.0 && T[(i + 1) * n + i] != 0.0) {
            err = "coefficient is not upper quasi-triangular: consecutive nonzero subdiagonal entries at row " +
                  std::to_string(i);
            return TT_EINVAL;
        }
    // m = ceil(n / b) blocks of near-equal size (at most b rows), each ideal
    // boundary moved by one row when it would cut a 2x2 block (to the next
    // row as Algorithm 2 does if that keeps the block within b rows, else to
    // the previous one).  Algorithm 2 moves k to k + 1 instead;
    // any split with A(k+1, k) = 0 is valid (Sec. 2.1).
    auto cuts_bump = [&](int64_t k) { return k > 0 && k < n && T[k * n + k - 1] != 0.0; };
    auto split = [&](int64_t m) {
        bst.clear();
        bst.push_back(0);
        int big = 0;
        for (int64_t k = 1; k < m; ++k) {
            int64_t q = (k * n + m / 2) / m;
            if (cuts_bump(q)) q = (q + 1 - bst.back() <= b && q + 1 < n) ? q + 1 : q - 1;
            if (q <= bst.back()) continue;
            big = std::max(big, (int)(q - bst.back()));
            bst.push_back((int32_t)q);
        }
        big = std::max(big, (int)(n - bst.back()));
        bst.push_back((int32_t)n);
        return big;
    };
    // one more block when a moved boundary leaves a block over b rows
    const int64_t m = (n + b - 1) / b;
    if (split(m) > b && m + 1 <= n) split(m + 1);
    // Full blocks: b rows each (b - 1 where the boundary would cut a 2x2
    // block), the remainder in a last, thinner block.  Taken when it needs no
    // more blocks than the near-equal split: the update tiles of full blocks
    // are full (a pencil of two b = 16 blocks is exactly 256 columns, K and M
    // are multiples of 16), while near-equal blocks of 15 or 16 rows leave
    // most tiles ragged.  A thin last block also folds into the split tree
    // when the count is 2^L + 1.
    if (b >= 2) {
        std::vector<int32_t> full{0};
        while (full.back() < n) {
            int64_t q = (int64_t)full.back() + b;
            if (q >= n) q = n;
            else if (cuts_bump(q)) q -= 1;  // no two consecutive bumps: q - 1 is free
            full.push_back((int32_t)q);
        }
        if (full.size() <= bst.size()) bst.swap(full);
    }
    for (size_t i = 0; i + 1 < bst.size(); ++i)
        if (bst[i + 1] - bst[i] > kMaxLeaf) {
            err = "leaf block larger than " + std::to_string(kMaxLeaf) + " rows; use a smaller nmin";
            return TT_EINVAL;
        }
    return TT_OK;
}

static inline int lowbit(int c) { return c & (-c); }

// Number of 1x1 / 2x2 diagonal blocks of T (n x n, row-major) in rows
// [r0, r1), and how many of them are 1x1.
static int tuple_count(const std::vector<double>& T, int64_t n, int64_t r0, int64_t r1, int* ones) {
    int m = 0, o = 0;
    for (int64_t i = r0; i < r1; ++m) {
        const bool two = i + 1 < r1 && T[(size_t)((i + 1) * n + i)] != 0.0;
        o += two ? 0 : 1;
        i += two ? 2 : 1;
    }
    *ones = o;
    return m;
}

// Index of the tuple-grid shape (m_0, ..., m_{D-1}), creating its
// hyperplane-ordered tuple list on first use.  Tuple p depends on the tuples
// that are larger in one coordinate and equal in the others, so hyperplane
// h = sum_mu (m_mu - 1 - p_mu) only depends on hyperplanes < h.
static int32_t shape_index(Schedule& s, std::map<std::array<int, kMaxD>, int32_t>& known,
                           const std::array<int, kMaxD>& m) {
    auto it = known.find(m);
    if (it != known.end()) return it->second;
    const int D = s.D;
    int H = 1, total = 1;
    for (int mu = 0; mu < D; ++mu) {
        H += m[mu] - 1;
        total *= m[mu];
    }
    const int bits = (D == 4) ? kTupBits4 : kTupBits3;
    std::vector<std::vector<uint16_t>> byh((size_t)H);
    for (int lin = 0; lin < total; ++lin) {
        int rem = lin, h = 0;
        uint32_t ent = 0;
        for (int mu = D - 1; mu >= 0; --mu) {
            const int p = rem % m[mu];
            rem /= m[mu];
            h += m[mu] - 1 - p;
            ent |= (uint32_t)p << (bits * mu);
        }
        byh[(size_t)h].push_back((uint16_t)ent);
    }
    LeafShape sh{};
    sh.ent = (int32_t)s.ents.size();
    sh.hoff = (int32_t)s.hoffs.size();
    sh.H = H;
    sh.count = total;
    int off = 0;
    for (int h = 0; h < H; ++h) {
        s.hoffs.push_back(off);
        for (uint16_t e : byh[(size_t)h]) s.ents.push_back(e);
        off += (int)byh[(size_t)h].size();
    }
    s.hoffs.push_back(off);
    s.maxtup = std::max(s.maxtup, total);
    s.maxH = std::max(s.maxH, H);
    const int32_t idx = (int32_t)s.shapes.size();
    s.shapes.push_back(sh);
    known[m] = idx;
    return idx;
}

int build_schedule(Schedule& s, int nmin, std::string& err) {
    const int D = s.D;
    // default leaf edge: 16 (order 3) / 8 (order 4); the second class's
    // leaves (one wave per block of at most 1000 unknowns, D - 1 block
    // tensors in LDS) take 8 / 5
    if (nmin <= 0) nmin = (s.cls == 1) ? ((D >= 4) ? 5 : 8) : ((D >= 4) ? 8 : 16);
    if (nmin < 2) nmin = 2;
    if (nmin > 20) {
        err = "nmin must be at most 20";
        return TT_EINVAL;
    }
    for (int mu = 0; mu < kMaxD; ++mu) s.bmax[mu] = 1;
    s.shapes.clear();
    s.ents.clear();
    s.hoffs.clear();
    s.maxtup = 1;
    s.maxcpl = 1;
    s.maxH = 1;
    std::map<std::array<int, kMaxD>, int32_t> known_shapes;
    s.leaves.clear();
    s.tasks.clear();
    s.items.clear();
    s.waves.clear();
    s.stats = PlanStats();

    int64_t W = 0;
    for (auto& p : s.probs) {
        int64_t N = 1;
        for (int mu = 0; mu < D; ++mu) N *= p.n[mu];
        p.N = N;
        for (int mu = 0; mu < D; ++mu) {
            int rc = partition_mode(p.n[mu], p.T[mu].data(), nmin, p.bst[mu], err);
            if (rc) return rc;
            p.m[mu] = (int)p.bst[mu].size() - 1;
            if (p.m[mu] > 32767) {
                err = "too many leaf blocks along one mode";
                return TT_EINVAL;
            }
            for (int b = 0; b < p.m[mu]; ++b)
                s.bmax[mu] = std::max<int>(s.bmax[mu], p.bst[mu][b + 1] - p.bst[mu][b]);
        }
        if (N == 0) continue;
        int64_t w = 1;
        for (int mu = 0; mu < D; ++mu) w += p.m[mu] - 1;
        W = std::max(W, w);
    }

    // bucket the leaf blocks of every problem by wave
    std::vector<std::vector<LeafDesc>> waves((size_t)W);
    for (size_t pi = 0; pi < s.probs.size(); ++pi) {
        const HostProblem& p = s.probs[pi];
        if (p.N == 0) continue;
        int64_t total = 1;
        for (int mu = 0; mu < D; ++mu) total *= p.m[mu];
        for (int64_t lin = 0; lin < total; ++lin) {
            LeafDesc L{};
            L.prob = (int32_t)pi;
            int64_t rem = lin, w = 0;
            for (int mu = D - 1; mu >= 0; --mu) {
                L.blk[mu] = (int16_t)(rem % p.m[mu]);
                rem /= p.m[mu];
                w += p.m[mu] - 1 - L.blk[mu];
            }
            for (int mu = D; mu < kMaxD; ++mu) L.blk[mu] = 0;
            waves[(size_t)w].push_back(L);
        }
    }

    // Per (problem, mode, block): whether a tree update has already been
    // scheduled for it (the first one stores, later ones accumulate).
    std::vector<std::vector<uint8_t>> received(s.probs.size());
    for (size_t pi = 0; pi < s.probs.size(); ++pi) {
        int64_t total = 1;
        for (int mu = 0; mu < D; ++mu) total *= s.probs[pi].m[mu];
        received[pi].assign((size_t)(total * D), 0);
    }
    auto block_lin = [&](const HostProblem& p, const int* I) {
        int64_t l = 0;
        for (int mu = 0; mu < D; ++mu) l = l * p.m[mu] + I[mu];
        return l;
    };

    // Tasks triggered after each wave, executed together with the next one.
    std::vector<std::vector<int32_t>> triggered((size_t)W + 1);
    double fl_leaf = 0, fl_upd = 0;
    auto add_task = [&](const HostProblem& p, int pi, const int* I, int mu, int lo, int hi_t, int src_lo,
                        int src_hi, int64_t trigger_wave) {
        // targets: blocks [lo, hi_t) along mu; sources: blocks [src_lo, src_hi)
        if (lo >= hi_t || src_lo >= src_hi) return;
        UpdDesc t{};
        t.prob = pi;
        t.mode = (int16_t)mu;
        t.r0 = p.bst[mu][lo];
        t.M = p.bst[mu][hi_t] - t.r0;
        t.k0 = p.bst[mu][src_lo];
        t.K = p.bst[mu][src_hi] - t.k0;
        int64_t xb = 0;
        int q = 0;
        int ext[3] = {1, 1, 1};
        int64_t ostr[3] = {0, 0, 0};
        for (int nu = 0; nu < D; ++nu) {
            if (nu == mu) continue;
            int64_t st = p.bst[nu][I[nu]];
            xb += st * p.stride[nu];
            ext[q] = p.bst[nu][I[nu] + 1] - (int32_t)st;
            ostr[q] = p.stride[nu];
            ++q;
        }
        if (q == 2) {  // slot 2 is the fastest of the other modes
            ext[2] = ext[1];
            ostr[2] = ostr[1];
            ext[1] = ext[0];
            ostr[1] = ostr[0];
            ext[0] = 1;
            ostr[0] = 0;
        }
        t.xbase = xb;
        for (int i = 0; i < 3; ++i) {
            t.ext[i] = ext[i];
            t.ostr[i] = ostr[i];
        }
        t.P = ext[0] * ext[1] * ext[2];
        if (t.M <= 0 || t.K <= 0 || t.P <= 0) return;
        // store or accumulate: uniform over the targets of one task
        int nrec = 0;
        int J[kMaxD];
        for (int nu = 0; nu < D; ++nu) J[nu] = I[nu];
        for (int b = lo; b < hi_t; ++b) {
            J[mu] = b;
            uint8_t& r = received[(size_t)pi][(size_t)(block_lin(p, J) * D + mu)];
            nrec += r;
            r = 1;
        }
        if (nrec == 0) t.flags |= 1;  // first contribution (mode 0: from B into X)
        if (nrec != 0 && nrec != hi_t - lo) t.flags |= 2;  // inconsistent (checked below)
        triggered[(size_t)trigger_wave].push_back((int32_t)s.tasks.size());
        s.tasks.push_back(t);
    };

    // Leaves per wave and the tree updates they trigger.  Along each mode the
    // split with midpoint c and half-width s = lowbit(c) >= 2 sends R1 =
    // [c, c+s) to R0 = [c-s, c); the pair (c-1, c) of adjacent blocks is left
    // to the leaf of block c-1, which reads block c itself.  The rest is
    //   (1) targets [c-s, c-1) from sources [c, c+s), ready once c is solved;
    //   (2) target  c-1        from sources [c+1, c+s), ready once c+1 is.
    // Both have at least one hyperplane of slack before their targets run.
    // With m = 2^L + 1 blocks (a partition pushed one block past a power of
    // two by the 2x2 blocks) the splits run over 2^L blocks whose last one is
    // the pair {m-2, m-1}: every update whose sources end at block m-2 also
    // takes block m-1, block m-3 receives block m-1 in a task of its own, and
    // the lone split at c = m-1 (a rank-|block| update of every other block,
    // a whole pass over the tensor) disappears.
    for (int64_t w = 0; w < W; ++w) {
        for (const LeafDesc& L0 : waves[(size_t)w]) {
            const HostProblem& p = s.probs[(size_t)L0.prob];
            int I[kMaxD];
            for (int mu = 0; mu < D; ++mu) I[mu] = L0.blk[mu];
            for (int mu = 0; mu < D; ++mu) {
                const int m = p.m[mu];
                const bool fold = m >= 5 && ((m - 1) & (m - 2)) == 0;
                const int mt = fold ? m - 1 : m;  // blocks of the split tree
                const int c = I[mu];
                auto src_end = [&](int e) { return (fold && e >= mt) ? m : std::min(e, m); };
                if (fold && c == m - 1) {  // block m-3 from block m-1
                    add_task(p, L0.prob, I, mu, m - 3, m - 2, m - 1, m, w);
                    continue;
                }
                // type (1): this block is the midpoint c
                if (c >= 1) {
                    const int sb = lowbit(c);
                    if (sb >= 2) add_task(p, L0.prob, I, mu, c - sb, c - 1, c, src_end(c + sb), w);
                }
                // type (2): this block is c + 1 for the midpoint c = I - 1
                const int c2 = c - 1;
                if (c2 >= 1) {
                    const int sb = lowbit(c2);
                    if (sb >= 2) add_task(p, L0.prob, I, mu, c2 - 1, c2, c2 + 1, src_end(c2 + sb), w);
                }
            }
        }
    }
    for (const UpdDesc& t : s.tasks)
        if (t.flags & 2) {
            err = "internal: mixed first/accumulated targets in one update";
            return TT_EINVAL;
        }

    // Per (problem, mode, block): tuples, 1x1 tuples and 2x2 blocks.
    struct BlockInfo {
        int tuples, ones, bumps;
    };
    std::vector<std::vector<std::vector<BlockInfo>>> binfo(s.probs.size());
    for (size_t pi = 0; pi < s.probs.size(); ++pi) {
        const HostProblem& p = s.probs[pi];
        binfo[pi].resize((size_t)D);
        for (int mu = 0; mu < D; ++mu)
            for (int b = 0; b < p.m[mu]; ++b) {
                const int64_t r0 = p.bst[mu][b], r1 = p.bst[mu][b + 1], nm = p.n[mu];
                BlockInfo bi{};
                bi.tuples = tuple_count(p.T[mu], nm, r0, r1, &bi.ones);
                for (int64_t i = r0; i + 1 < r1; ++i)
                    if (p.T[mu][(size_t)((i + 1) * nm + i)] != 0.0) ++bi.bumps;
                binfo[pi][(size_t)mu].push_back(bi);
            }
    }

    // Leaf flags: accumulator reads and the adjacent block.
    std::vector<int32_t> order;
    std::vector<std::vector<WorkItem>> xq(8);  // per-XCD tile queues of one wave
    struct Unit {                              // tasks sharing the tiles of one item group
        int32_t task[4];
        int n;
    };
    std::vector<Unit> units;
    std::map<std::array<int64_t, 8>, size_t> open_units;
    std::vector<UpdDesc> ntasks;               // tasks in item order
    ntasks.reserve(s.tasks.size());
    for (int64_t w = 0; w < W; ++w) {
        Wave wv;
        wv.leaf_first = (int64_t)s.leaves.size();
        for (LeafDesc L : waves[(size_t)w]) {
            const HostProblem& p = s.probs[(size_t)L.prob];
            int I[kMaxD];
            for (int mu = 0; mu < D; ++mu) I[mu] = L.blk[mu];
            L.flags = 0;
            std::array<int, kMaxD> tm = {1, 1, 1, 1};
            int all = 1, single = 1;
            for (int mu = 0; mu < D; ++mu) {
                // bit 0: the right-hand side is in X (mode-0 updates); bits
                // mu >= 1: accumulators to subtract
                if (received[(size_t)L.prob][(size_t)(block_lin(p, I) * D + mu)]) L.flags |= 1 << mu;
                if (I[mu] + 1 < p.m[mu]) L.flags |= 1 << (4 + mu);
                const BlockInfo& bi = binfo[(size_t)L.prob][(size_t)mu][(size_t)I[mu]];
                tm[mu] = bi.tuples;
                all *= bi.tuples;
                single *= bi.ones;
            }
            s.maxcpl = std::max(s.maxcpl, all - single);
            L.shape = shape_index(s, known_shapes, tm);
            s.leaves.push_back(L);
            // algorithmic work: in-block back-substitution + the adjacent blocks
            int64_t sz[kMaxD], ne = 1;
            for (int mu = 0; mu < D; ++mu) {
                sz[mu] = p.bst[mu][I[mu] + 1] - p.bst[mu][I[mu]];
                ne *= sz[mu];
            }
            double lf = 0, lb = 16.0 * (double)ne;
            for (int mu = 0; mu < D; ++mu) {
                const int64_t bumps = binfo[(size_t)L.prob][(size_t)mu][(size_t)I[mu]].bumps;
                double off = (double)sz[mu] * (double)(sz[mu] - 1) / 2.0 + (double)bumps;
                lf += 2.0 * off * (double)(ne / sz[mu]);
                lb += 8.0 * (double)(sz[mu] * sz[mu]);
                if (mu >= 1 && (L.flags & (1 << mu))) lb += 8.0 * (double)ne;  // accumulator read
                if (L.flags & (1 << (4 + mu))) {
                    int64_t sa = p.bst[mu][I[mu] + 2] - p.bst[mu][I[mu] + 1];
                    lf += 2.0 * (double)sz[mu] * (double)sa * (double)(ne / sz[mu]);
                    lb += 8.0 * (double)(ne / sz[mu]) * (double)sa + 8.0 * (double)(sz[mu] * sa);
                }
            }
            wv.leaf_flops += lf;
            wv.leaf_bytes += lb;
            fl_leaf += lf;
        }
        wv.leaf_count = (int64_t)s.leaves.size() - wv.leaf_first;
        // update tiles triggered by the previous wave
        wv.item_first = (int64_t)s.items.size();
        if (w >= 1) {
            // longest tiles first (the work of a tile grows with K and its
            // height), so that
            // the launch does not end on a few long tiles; tiles of one task
            // stay adjacent
            order = triggered[(size_t)(w - 1)];
            auto tile_work = [&](int32_t k) {  // K x (target rows of a tile / 64)
                const UpdDesc& t = s.tasks[(size_t)k];
                return (int64_t)t.K * ((t.M > kTile) ? 2 : 1);
            };
            std::stable_sort(order.begin(), order.end(),
                             [&](int32_t a, int32_t b) { return tile_work(a) > tile_work(b); });
            // Workgroups go to the XCDs round-robin (workgroup i to XCD i % 8):
            // the tiles of one task that read the same source panel (same
            // pencil columns) are dealt to one XCD, so the panel is fetched
            // into one L2 instead of several.  Groups fill the least loaded
            // XCD queue in order; the queues are interleaved, and the ragged
            // tail is padded with empty items (task -1).
            // units: one task, or (second class) up to upd_wide_slots(P)
            // tasks with at most 16 target rows that differ only in their
            // pencil and share one 16 x 256 tile (filled in order of first
            // appearance).  The Laplace-like schedules gain nothing from the
            // shared tiles (their small pencils are the few through a thin
            // block) and were measured slower with them at order 5.
            units.clear();
            open_units.clear();
            for (int32_t tid : order) {
                const UpdDesc& t = s.tasks[(size_t)tid];
                const int g = (t.M <= 16 && s.cls == 1) ? upd_wide_slots(t.P) : 1;
                if (g == 1) {
                    units.push_back(Unit{{tid, 0, 0, 0}, 1});
                    continue;
                }
                const std::array<int64_t, 8> key = {t.prob, t.mode, t.r0, t.M, t.k0, t.K, t.P, t.flags & 1};
                auto it = open_units.find(key);
                if (it == open_units.end()) {
                    open_units[key] = units.size();
                    units.push_back(Unit{{tid, 0, 0, 0}, 1});
                } else {
                    Unit& un = units[it->second];
                    un.task[un.n++] = tid;
                    if (un.n == g) open_units.erase(it);
                }
            }
            for (auto& q : xq) q.clear();
            for (const auto& u : units) {
                // the unit's tasks take consecutive indices of the final task list
                const int32_t nt = (int32_t)ntasks.size();
                for (int j = 0; j < u.n; ++j) {
                    const UpdDesc& t = s.tasks[(size_t)u.task[j]];
                    ntasks.push_back(t);
                    const double f = 2.0 * (double)t.M * (double)t.K * (double)t.P;
                    wv.upd_flops += f;
                    fl_upd += f;
                    wv.upd_bytes += 8.0 * (((t.flags & 1) && t.mode != 0 ? 1.0 : 2.0) * (double)t.M * t.P +
                                           (double)t.K * t.P + (double)t.M * t.K);
                }
                const UpdDesc& t = s.tasks[(size_t)u.task[0]];
                const bool right = (t.mode == D - 1);
                int na = 1, nb = 1;
                upd_tile_grid(t, right, na, nb);
                // a group: the tiles sharing pencil columns (b for the left
                // path, a for the right path; every wide tile alone)
                const int ng = (t.M <= 16) ? na : (right ? na : nb);
                const int gs = (t.M <= 16) ? 1 : (right ? nb : na);
                for (int g = 0; g < ng; ++g) {
                    size_t x = 0;
                    for (size_t y = 1; y < xq.size(); ++y)
                        if (xq[y].size() < xq[x].size()) x = y;
                    for (int e = 0; e < gs; ++e) {
                        int a = 0, b = 0;
                        if (t.M <= 16) {
                            a = g;
                            b = u.n - 1;  // tasks sharing the tile
                        } else if (right) {
                            a = g;
                            b = e;
                        } else {
                            a = e;
                            b = g;
                        }
                        xq[x].push_back(WorkItem{nt, (int16_t)a, (int16_t)b});
                    }
                }
            }
            size_t rounds = 0;
            for (const auto& q : xq) rounds = std::max(rounds, q.size());
            for (size_t r = 0; r < rounds; ++r)
                for (const auto& q : xq) s.items.push_back(r < q.size() ? q[r] : WorkItem{-1, 0, 0});
        }
        wv.item_count = (int64_t)s.items.size() - wv.item_first;
        s.waves.push_back(wv);
    }
    if (!triggered[(size_t)(W > 0 ? W - 1 : 0)].empty()) {
        err = "internal: updates triggered by the last wave";
        return TT_EINVAL;
    }
    if (ntasks.size() != s.tasks.size()) {
        err = "internal: update tasks lost in the tile layout";
        return TT_EINVAL;
    }
    s.tasks.swap(ntasks);

    for (int mu = 0; mu < D; ++mu)
        if (s.bmax[mu] > ((D == 4) ? (1 << kTupBits4) : kMaxLeaf)) {
            err = "leaf block too large (at most " + std::to_string(D == 4 ? (1 << kTupBits4) : kMaxLeaf) +
                  " rows per mode); lower nmin";
            return TT_EINVAL;
        }
    const int lds_need = (s.cls == 1) ? leaf2_lds_bytes(D, s.bmax) : leaf_lds_bytes(D, s.bmax, s.maxtup, s.maxcpl, s.maxH);
    if (lds_need > 160 * 1024) {
        err = "leaf block does not fit in LDS; lower nmin";
        return TT_EINVAL;
    }
    s.stats.flops_leaf = fl_leaf;
    s.stats.flops_update = fl_upd;
    s.stats.flops = fl_leaf + fl_upd;
    s.stats.waves = W;
    s.stats.leaves = (int64_t)s.leaves.size();
    s.stats.tasks = (int64_t)s.tasks.size();
    s.stats.items = (int64_t)s.items.size();
    s.stats.launches = 2 * (int64_t)s.waves.size();
    for (int mu = 0; mu < kMaxD; ++mu) s.stats.bmax[mu] = s.bmax[mu];
    return TT_OK;
}

}  // namespace tt
