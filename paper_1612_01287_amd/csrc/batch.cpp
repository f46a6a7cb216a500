// Batches: many Sod or Bjorken instances of uneven size advanced by one launch
// per RK stage (Sod) or one launch per call (Bjorken).
//
// Work items of a Sod batch are (instance, tile) pairs.  Workgroups are dealt
// to the eight XCDs round-robin, so the item list is laid out as eight
// interleaved per-XCD queues: tiles of one instance stay in contiguous runs
// on one XCD (their shared halo cells meet in one L2), the queues carry equal
// estimated cost, and each queue runs its costliest items first.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>
#include <functional>
#include <vector>

#include "imex.h"
#include "rsl_impl.h"

struct rsl_batch {
    int n = 0, kind = 0, dtype = 0;
    std::vector<const rsl_quad*> quads;
    std::vector<rsl_problem> probs;
    std::vector<double> dt, t;
    std::vector<size_t> f_off, w_off;
    size_t f_bytes = 0, w_bytes = 0;
    std::vector<rsl::InstDesc> host_desc;   // offsets, not pointers
    void* dmem = nullptr;                   // descriptors + items
    rsl::BatchLaunch launch{};
    size_t bj_lds = 0;
    int device = -1;
    // concurrency across velocity classes: helper streams joined by events
    bool streams_ready = false;
    hipStream_t aux[rsl::kClasses] = {};
    hipEvent_t ev_fork = nullptr, ev_join[rsl::kClasses] = {};
    // captured graph of nsteps steps
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    void* g_f = nullptr;
    void* g_w = nullptr;
    int g_steps = -1;
    hipStream_t g_stream = nullptr;
    // Bjorken: groups of up to 16 instances sharing one velocity set (matrix-core path)
    double* states = nullptr;     // Sod: device [n][4] initial states (n_L, T_L, n_R, T_R)
    int* groups = nullptr;        // device [ngroups][16]
    int ngroups = 0;
    size_t mfma_lds = 0;
    bool use_mfma = false;
    int bj_path = -1;             // -1 automatic, 0 per-instance kernel, 1 matrix cores
    int ql_first[5] = {}, ql_count[5] = {};   // groups of each Q_L (1..4)
    std::vector<int> group_sizes;             // live instances per group, launch order
    bool merged = false;                      // Sod: every instance in one class (launch.all)
    // implicit-explicit steps: instances created with RSL_FLAG_IMEX (CFL bound
    // only) make the batch refuse the explicit steps; item lists built at the
    // first rsl_batch_step_imex
    bool imex = false;
    void* imex_mem = nullptr;
    rsl::ImexItems imex_items{};
};

namespace rsl {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Estimated cost of one tile of instance i in units of one cell-velocity update;
// the per-cell work (Landau frame, equilibrium coefficients) is ~25 updates.
double tile_cost(const rsl_quad* q) { return (double)kLanes * (q->V + 25.0); }

std::vector<int2> schedule(const rsl_batch* b, int cls, int tc) {
    const int X = 8;
    std::vector<int> order;
    for (int i = 0; i < b->n; ++i)
        if (cls < 0 || stage_class_of(b->quads[i]->V) == cls) order.push_back(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return b->quads[a]->V > b->quads[c]->V; });
    std::vector<std::vector<std::pair<double, int2>>> q(X);
    std::vector<double> load(X, 0.0);
    for (int i : order) {
        const int nt = (b->probs[i].nz + tc - 1) / tc;
        const double c = tile_cost(b->quads[i]) * tc / kTileCells;
        const int run = std::max(1, (nt + X - 1) / X);
        for (int t0 = 0; t0 < nt; t0 += run) {
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            for (int t = t0; t < std::min(nt, t0 + run); ++t) {
                q[x].push_back({c, make_int2(i, t)});
                load[x] += c;
            }
        }
    }
    size_t per = 0;
    for (auto& v : q) {
        std::stable_sort(v.begin(), v.end(), [](const auto& a, const auto& c) { return a.first > c.first; });
        per = std::max(per, v.size());
    }
    std::vector<int2> items(per * X, make_int2(-1, -1));
    for (size_t s = 0; s < per; ++s)
        for (int x = 0; x < X; ++x)
            if (s < q[x].size()) items[s * X + x] = q[x][s].second;
    return items;
}

}  // namespace

// Cost of one matrix-core Bjorken group on one CU, per RK stage, in units of
// one v_mfma_f64_16x16x4f64 (64 cycles), fitted to measured stage times at
// Q_xi = 40, 100, 200 with 1 and 3 column tiles: a part independent of the
// column tiles (moments, closure, barriers) that grows with Q_xi, and per
// column tile the k-steps of the busiest SIMD (waves w and w + 4 share a
// SIMD; wave w owns row blocks w and w + 8) plus the vector epilogue.
double bj_group_cost(int Q, int tiles) {
    const int RT = (Q + 15) / 16, KT = 4 * RT;
    int rb = 0;
    for (int simd = 0; simd < 4; ++simd) {
        int c = 0;
        for (int w = simd; w < 8; w += 4)
            for (int u = 0; u < 2; ++u) c += w + 8 * u < RT;
        rb = std::max(rb, c);
    }
    const double q = std::max(Q - 40, 0);
    return 84.0 + 1.22 * q + tiles * ((double)rb * KT + 31.0 + 0.2 * q);
}

// Longest-first list schedule of group costs on ncu CUs (one workgroup per
// CU, dispatched in list order as CUs free up): its makespan.
double bj_makespan(std::vector<double> cost, int ncu) {
    std::sort(cost.begin(), cost.end(), std::greater<double>());
    std::priority_queue<double, std::vector<double>, std::greater<double>> cu;
    for (int k = 0; k < ncu; ++k) cu.push(0.0);
    double span = 0.0;
    for (double c : cost) {
        const double t = cu.top() + c;
        cu.pop();
        cu.push(t);
        span = std::max(span, t);
    }
    return span;
}

// Bjorken groups: instances sharing one rsl_quad, up to 16 per group, live
// instances first (the kernel skips column tiles past the last live one);
// groups of one Q_L are contiguous (one launch each), costliest first.  One
// workgroup per group and per CU: when a few velocity sets are much larger
// than the rest, their full groups would be the critical path of the launch,
// so the instances of a set whose full group costs more than a cap are spread
// over groups of fewer column tiles.  The cap (a multiple of the average load
// per CU with full groups) is the one whose list schedule ends first.
std::vector<int> bj_groups(const rsl_batch* b, int ncu) {
    std::vector<int> order(b->n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        const rsl_quad *qa = b->quads[a], *qc = b->quads[c];
        if (qa->QL != qc->QL) return qa->QL < qc->QL;
        return qa->Q != qc->Q ? qa->Q > qc->Q : qa < qc;
    });
    std::vector<std::pair<size_t, size_t>> sets;   // runs of one rsl_quad in `order`
    for (size_t s = 0; s < order.size();) {
        size_t e = s;
        while (e < order.size() && b->quads[order[e]] == b->quads[order[s]]) ++e;
        sets.push_back({s, e});
        s = e;
    }
    auto tiles_of = [](int n, int QL) { return (n * QL + 15) / 16; };
    double total = 0.0;
    for (auto& st : sets) {
        const rsl_quad* q = b->quads[order[st.first]];
        for (size_t m = st.second - st.first; m > 0; m -= std::min<size_t>(m, 16))
            total += bj_group_cost(q->Q, tiles_of((int)std::min<size_t>(m, 16), q->QL));
    }
    ncu = std::max(ncu, 1);
    struct G { int QL; double cost; size_t first; int n; };
    auto make_plan = [&](double cap) {
        std::vector<G> groups;
        for (auto& st : sets) {
            const rsl_quad* q = b->quads[order[st.first]];
            const int m = (int)(st.second - st.first);
            int per = std::min(16, 16 / q->QL);          // one column tile
            for (int t = 2; t <= q->QL; ++t)
                if (bj_group_cost(q->Q, t) <= cap) per = std::min(16, 16 * t / q->QL);
            const int ng = (m + per - 1) / per;
            for (int g = 0, s = 0; g < ng; ++g) {
                const int n = m / ng + (g < m % ng);     // sizes as even as possible
                groups.push_back({q->QL, bj_group_cost(q->Q, tiles_of(n, q->QL)), st.first + s, n});
                s += n;
            }
        }
        return groups;
    };
    auto span_of = [&](const std::vector<G>& groups) {
        double span = 0.0;
        for (int ql = 1; ql <= 4; ++ql) {      // one launch per Q_L, one after the other
            std::vector<double> c;
            for (const G& g : groups)
                if (g.QL == ql) c.push_back(g.cost);
            if (!c.empty()) span += bj_makespan(c, ncu);
        }
        return span;
    };
    std::vector<G> best;
    double best_span = 0.0;
    for (double mult : {1e30, 2.0, 1.6, 1.3, 1.15, 1.0}) {
        std::vector<G> plan = make_plan(mult * total / ncu);
        const double span = span_of(plan);
        if (best.empty() || span < best_span * (1.0 - 1e-9)) {
            best = std::move(plan);
            best_span = span;
        }
    }
    std::stable_sort(best.begin(), best.end(), [](const G& x, const G& y) {
        return x.QL != y.QL ? x.QL < y.QL : x.cost > y.cost;
    });
    std::vector<int> g;
    for (const G& gr : best) {
        for (int k = 0; k < 16; ++k) g.push_back(k < gr.n ? order[gr.first + k] : -1);
    }
    return g;
}

// Tile widths of the stage kernel variants: index 0 -> 63 cells, 1 -> 31 cells;
// index 2 -> the 64-cell tiles of the per-cell kernel.
constexpr int kTileWidths[3] = {kTileCells, 31, kCellTile};

int tw_index(int var) { return stage_variant_tile_cells(var) == kTileWidths[0] ? 0 : 1; }

void use_variant(StageClass& cl, int var) {
    cl.var = var;
    const int t = tw_index(var);
    cl.items = cl.items_tw[t];
    cl.nitems = cl.nitems_tw[t];
}

int batch_upload(rsl_batch* b) {
    std::vector<std::vector<int2>> items(3 * (kClasses + 1));
    size_t total = 0;
    std::vector<int> groups;
    if (b->kind == RSL_BJORKEN) {
        b->use_mfma = true;
        for (int i = 0; i < b->n; ++i)
            if (!bj_mfma_fits(b->quads[i]->Q, b->quads[i]->QL)) b->use_mfma = false;
        if (b->use_mfma) {
            int ncu = 0;
            if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) ncu = 0;
            groups = bj_groups(b, ncu > 0 ? ncu : 256);
            b->ngroups = (int)groups.size() / 16;
            for (int g = 0; g < b->ngroups; ++g) {
                int n = 0;
                while (n < 16 && groups[16 * g + n] >= 0) ++n;
                b->group_sizes.push_back(n);
            }
            for (int g = 0; g < b->ngroups; ++g) {
                const int ql = b->quads[groups[16 * g]]->QL;
                if (b->ql_count[ql] == 0) b->ql_first[ql] = g;
                ++b->ql_count[ql];
            }
            for (int i = 0; i < b->n; ++i)
                b->mfma_lds = std::max(b->mfma_lds, bj_mfma_lds_bytes(b->quads[i]->Q, b->quads[i]->QL));
            total += align_up(sizeof(int) * groups.size(), 256);
        }
    }
    if (b->kind == RSL_SOD)
        for (int c = 0; c <= kClasses; ++c)          // c = kClasses: every instance
            for (int t = 0; t < 3; ++t) {
                items[3 * c + t] = schedule(b, c < kClasses ? c : -1, kTileWidths[t]);
                total += align_up(sizeof(int2) * items[3 * c + t].size(), 256);
            }
    std::vector<double> states;
    if (b->kind == RSL_SOD) {
        for (int i = 0; i < b->n; ++i) {
            const rsl_problem& p = b->probs[i];
            states.insert(states.end(), {p.n_L, p.T_L, p.n_R, p.T_R});
        }
        total += align_up(sizeof(double) * states.size(), 256);
    }
    const size_t dbytes = align_up(sizeof(InstDesc) * b->n, 256);
    int rc = hip_check(hipMalloc(&b->dmem, dbytes + std::max<size_t>(total, 256)), "hipMalloc(batch)");
    if (rc) return rc;
    rc = hip_check(hipMemcpy(b->dmem, b->host_desc.data(), sizeof(InstDesc) * b->n, hipMemcpyHostToDevice),
                   "hipMemcpy(batch descriptors)");
    size_t off = dbytes;
    for (int c = 0; c <= kClasses && rc == RSL_OK; ++c) {
        StageClass& cl = c < kClasses ? b->launch.cl[c] : b->launch.all;
        cl.descs = (const InstDesc*)b->dmem;
        cl.maxV = 0;
        for (int i = 0; i < b->n; ++i)
            if (b->kind == RSL_SOD && (c == kClasses || stage_class_of(b->quads[i]->V) == c))
                cl.maxV = std::max(cl.maxV, b->quads[i]->V);
        for (int t = 0; t < 3 && rc == RSL_OK; ++t) {
            const std::vector<int2>& it = items[3 * c + t];
            cl.items_tw[t] = (const int2*)((char*)b->dmem + off);
            cl.nitems_tw[t] = (int)it.size();
            if (!it.empty())
                rc = hip_check(hipMemcpy((char*)b->dmem + off, it.data(), sizeof(int2) * it.size(),
                                         hipMemcpyHostToDevice), "hipMemcpy(batch items)");
            off += align_up(sizeof(int2) * it.size(), 256);
        }
        use_variant(cl, stage_default_variant(c < kClasses ? c : kClasses - 1));
    }
    if (rc == RSL_OK && !groups.empty()) {
        b->groups = (int*)((char*)b->dmem + off);
        rc = hip_check(hipMemcpy(b->groups, groups.data(), sizeof(int) * groups.size(), hipMemcpyHostToDevice),
                       "hipMemcpy(batch groups)");
        off += align_up(sizeof(int) * groups.size(), 256);
    }
    if (rc == RSL_OK && !states.empty()) {
        b->states = (double*)((char*)b->dmem + off);
        rc = hip_check(hipMemcpy(b->states, states.data(), sizeof(double) * states.size(), hipMemcpyHostToDevice),
                       "hipMemcpy(batch states)");
    }
    return rc;
}

int batch_streams(rsl_batch* b) {
    if (b->streams_ready) return RSL_OK;
    int rc = hip_check(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming), "hipEventCreate");
    for (int c = 0; c < kClasses && rc == RSL_OK; ++c) {
        rc = hip_check(hipStreamCreateWithFlags(&b->aux[c], hipStreamNonBlocking), "hipStreamCreate");
        if (rc == RSL_OK) rc = hip_check(hipEventCreateWithFlags(&b->ev_join[c], hipEventDisableTiming), "hipEventCreate");
    }
    b->streams_ready = rc == RSL_OK;
    return rc;
}

// One RK stage of every Sod instance: the velocity classes run as concurrent
// launches (forked from and joined back into the caller's stream), or the
// whole batch as one class.
int batch_stage_all(rsl_batch* b, int stage, char* f, char* w, hipStream_t s, int seq) {
    int rc = RSL_OK;
    auto run = [&](const StageClass& cl, hipStream_t st) {
        return launch_sod_class_stage(cl, b->dtype, stage, f, w, st, seq);
    };
    if (b->merged) return run(b->launch.all, s);
    int used[kClasses], nu = 0;
    for (int c = 0; c < kClasses; ++c)
        if (b->launch.cl[c].nitems) used[nu++] = c;
    if (nu <= 1) return nu ? run(b->launch.cl[used[0]], s) : RSL_OK;
    rc = batch_streams(b);
    if (rc) return rc;
    if ((rc = hip_check(hipEventRecord(b->ev_fork, s), "hipEventRecord"))) return rc;
    for (int k = 1; k < nu && rc == RSL_OK; ++k)
        rc = hip_check(hipStreamWaitEvent(b->aux[k], b->ev_fork, 0), "hipStreamWaitEvent");
    for (int k = 0; k < nu && rc == RSL_OK; ++k) rc = run(b->launch.cl[used[k]], k ? b->aux[k] : s);
    for (int k = 1; k < nu && rc == RSL_OK; ++k) {
        rc = hip_check(hipEventRecord(b->ev_join[k], b->aux[k]), "hipEventRecord");
        if (rc == RSL_OK) rc = hip_check(hipStreamWaitEvent(s, b->ev_join[k], 0), "hipStreamWaitEvent");
    }
    return rc;
}

// nsteps RK3 steps of every Sod instance.  Velocity classes hold disjoint
// instances, so each class runs all its stages on a stream of its own (forked
// from and joined back into the caller's stream once per call): no
// cross-stream wait between stages, and one class's per-cell kernel overlaps
// another class's stream kernel.
int batch_sod_steps(rsl_batch* b, char* f, char* w, int nsteps, hipStream_t s) {
    if (b->merged) {
        int rc = RSL_OK;
        for (int it = 0; it < nsteps && rc == RSL_OK; ++it)
            for (int st = 1; st <= 3 && rc == RSL_OK; ++st)
                rc = launch_sod_class_stage(b->launch.all, b->dtype, st, f, w, s, 3 * it + st - 1);
        return rc;
    }
    int used[kClasses], nu = 0;
    for (int c = 0; c < kClasses; ++c)
        if (b->launch.cl[c].nitems) used[nu++] = c;
    int rc = RSL_OK;
    if (nu > 1) {
        if ((rc = batch_streams(b))) return rc;
        if ((rc = hip_check(hipEventRecord(b->ev_fork, s), "hipEventRecord"))) return rc;
        for (int k = 1; k < nu && rc == RSL_OK; ++k)
            rc = hip_check(hipStreamWaitEvent(b->aux[k], b->ev_fork, 0), "hipStreamWaitEvent");
    }
    for (int k = 0; k < nu && rc == RSL_OK; ++k)
        for (int it = 0; it < nsteps && rc == RSL_OK; ++it)
            for (int st = 1; st <= 3 && rc == RSL_OK; ++st)
                rc = launch_sod_class_stage(b->launch.cl[used[k]], b->dtype, st, f, w, k ? b->aux[k] : s,
                                            3 * it + st - 1);
    if (nu > 1)
        for (int k = 1; k < nu && rc == RSL_OK; ++k) {
            rc = hip_check(hipEventRecord(b->ev_join[k], b->aux[k]), "hipEventRecord");
            if (rc == RSL_OK) rc = hip_check(hipStreamWaitEvent(s, b->ev_join[k], 0), "hipStreamWaitEvent");
        }
    return rc;
}

int batch_steps(rsl_batch* b, char* f, char* w, int nsteps, hipStream_t s) {
    int rc = RSL_OK;
    if (b->kind == RSL_SOD) {
        if (nsteps > 0) rc = batch_sod_steps(b, f, w, nsteps, s);
    } else if (nsteps > 0) {
        const bool mfma = b->use_mfma && b->bj_path != 0;
        if (mfma) {
            for (int ql = 1; ql <= 4 && rc == RSL_OK; ++ql) {
                if (b->ql_count[ql] == 0) continue;
                rc = launch_bj_mfma((const InstDesc*)b->dmem, b->groups + 16 * b->ql_first[ql], b->ql_count[ql], ql,
                                    b->mfma_lds, b->dtype, f, w, nsteps, s);
            }
        } else {
            rc = launch_bj_batch_steps((const InstDesc*)b->dmem, b->n, b->bj_lds, b->dtype, f, w, 0.0, 0.0, nsteps, s);
        }
    }
    return rc;
}

void batch_drop_graph(rsl_batch* b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->g_steps = -1;
}

}  // namespace rsl

using namespace rsl;

namespace {

const char* const kImexOnly =
    "the batch holds instances created with RSL_FLAG_IMEX (CFL bound only): step it with rsl_batch_step_imex";

// Item lists of the implicit-explicit steps, uploaded once.
int imex_items(rsl_batch* b) {
    if (b->imex_mem) return RSL_OK;
    std::vector<std::vector<int2>> cls(kImexClasses);
    std::vector<int2> x;
    for (int i = 0; i < b->n; ++i) {
        const int Q = b->quads[i]->Q, nz = b->probs[i].nz;
        const int c = imex_class(Q), per = imex_cells_per_item(Q);
        for (int s0 = 0; s0 < nz; s0 += per) cls[c].push_back(make_int2(i, s0));
        for (int s0 = 0; s0 < nz; s0 += imex_cells_per_explicit_item()) x.push_back(make_int2(i, s0));
    }
    size_t total = align_up(sizeof(int2) * x.size(), 256);
    for (const auto& v : cls) total += align_up(sizeof(int2) * v.size(), 256);
    void* mem = nullptr;
    if (hipMalloc(&mem, total) != hipSuccess) return set_error(RSL_EINVAL, "hipMalloc(imex items) failed");
    std::vector<char> host(total, 0);
    size_t off = 0;
    ImexItems it{};
    for (int c = 0; c < kImexClasses; ++c) {
        std::memcpy(host.data() + off, cls[c].data(), sizeof(int2) * cls[c].size());
        it.items[c] = (const int2*)((char*)mem + off);
        it.n[c] = (int)cls[c].size();
        off += align_up(sizeof(int2) * cls[c].size(), 256);
    }
    std::memcpy(host.data() + off, x.data(), sizeof(int2) * x.size());
    it.x = (const int2*)((char*)mem + off);
    it.nx = (int)x.size();
    const int rc = hip_check(hipMemcpy(mem, host.data(), total, hipMemcpyHostToDevice), "hipMemcpy(imex items)");
    if (rc) {
        (void)hipFree(mem);
        return rc;
    }
    b->imex_mem = mem;
    b->imex_items = it;
    return RSL_OK;
}

}  // namespace

extern "C" {

int rsl_batch_create(const rsl_quad* const* quads, const rsl_problem* problems, const double* dt, int n,
                     rsl_batch** out) {
    if (!out) return set_error(RSL_EINVAL, "null output pointer");
    *out = nullptr;
    if (n <= 0 || !quads || !problems || !dt) return set_error(RSL_EINVAL, "empty batch or null arrays");
    rsl_batch* b = new rsl_batch();
    b->n = n;
    b->kind = problems[0].problem;
    b->dtype = problems[0].dtype;
    int rc = RSL_OK;
    size_t f_total = 0, w_total = 0;
    for (int i = 0; i < n && rc == RSL_OK; ++i) {
        const rsl_quad* q = quads[i];
        const rsl_problem& p = problems[i];
        if (!q || !q->on_device) rc = set_error(RSL_EINVAL, "batch instance without a device rsl_quad");
        else if (p.problem != b->kind || p.dtype != b->dtype)
            rc = set_error(RSL_EINVAL, "a batch holds one problem kind and one dtype");
        else {
            size_t fb = 0, wb = 0;
            rc = rsl_sizes(q, &p, &fb, &wb);
            const bool imex = p.problem == RSL_SOD && (p.flags & RSL_FLAG_IMEX);
            b->imex = b->imex || imex;
            if (rc == RSL_OK && (rc = imex ? check_cfl(q, &p, dt[i]) : check_stability(q, &p, dt[i])))
                set_error(rc, "batch instance " + std::to_string(i) + ": " + rsl_last_error());
            if (rc == RSL_OK) {
                b->quads.push_back(q);
                b->probs.push_back(p);
                b->dt.push_back(dt[i]);
                b->t.push_back(p.problem == RSL_SOD ? 0.0 : 1.0);
                b->f_off.push_back(f_total);
                b->w_off.push_back(w_total);
                f_total += align_up(fb, 256);
                w_total += align_up(wb, 256);
            }
        }
    }
    if (rc == RSL_OK) {
        (void)hipGetDevice(&b->device);
        b->f_bytes = f_total;
        b->w_bytes = w_total;
        for (int i = 0; i < n; ++i) {
            InstDesc d = make_desc(b->quads[i], &b->probs[i], (void*)b->f_off[i], (void*)b->w_off[i], b->dt[i]);
            b->host_desc.push_back(d);
            if (b->kind == RSL_BJORKEN) b->bj_lds = std::max(b->bj_lds, bj_lds_bytes(b->quads[i]->V));
        }
        rc = batch_upload(b);
    }
    if (rc != RSL_OK) {
        if (b->dmem) (void)hipFree(b->dmem);
        delete b;
        return rc;
    }
    *out = b;
    return RSL_OK;
}

void rsl_batch_free(rsl_batch* b) {
    if (!b) return;
    batch_drop_graph(b);
    if (b->streams_ready) {
        (void)hipEventDestroy(b->ev_fork);
        for (int c = 0; c < kClasses; ++c) {
            (void)hipStreamDestroy(b->aux[c]);
            (void)hipEventDestroy(b->ev_join[c]);
        }
    }
    if (b->dmem) (void)hipFree(b->dmem);
    if (b->imex_mem) (void)hipFree(b->imex_mem);
    delete b;
}

int rsl_batch_sizes(const rsl_batch* b, size_t* f_bytes, size_t* work_bytes) {
    if (!b) return set_error(RSL_EINVAL, "null rsl_batch");
    if (f_bytes) *f_bytes = b->f_bytes;
    if (work_bytes) *work_bytes = b->w_bytes;
    return RSL_OK;
}

int rsl_batch_offset(const rsl_batch* b, int i, size_t* f_offset) {
    if (!b || i < 0 || i >= b->n || !f_offset) return set_error(RSL_EINVAL, "bad batch index");
    *f_offset = b->f_off[i];
    return RSL_OK;
}

int rsl_batch_time(const rsl_batch* b, int i, double* t) {
    if (!b || i < 0 || i >= b->n || !t) return set_error(RSL_EINVAL, "bad batch index");
    *t = b->t[i];
    return RSL_OK;
}

int rsl_batch_init(rsl_batch* b, void* f_dev, void* work_dev, void* hip_stream) {
    if (!b || !f_dev || !work_dev) return set_error(RSL_EINVAL, "null argument");
    if (b->kind == RSL_SOD) {
        // every instance in two launches: boundary states (and cleared status
        // words), then the initial populations over the 64-cell tiles
        const StageClass& all = b->launch.all;
        const int rc = launch_sod_batch_init(all.descs, b->states, b->n, all.items_tw[2], all.nitems_tw[2], b->dtype,
                                             (char*)f_dev, (char*)work_dev, (hipStream_t)hip_stream);
        if (rc) return rc;
        for (int i = 0; i < b->n; ++i) b->t[i] = 0.0;
        return RSL_OK;
    }
    for (int i = 0; i < b->n; ++i) {
        int rc = rsl_init(b->quads[i], &b->probs[i], (char*)f_dev + b->f_off[i], (char*)work_dev + b->w_off[i],
                          hip_stream);
        if (rc) return rc;
        b->t[i] = b->kind == RSL_SOD ? 0.0 : 1.0;
    }
    return RSL_OK;
}

int rsl_batch_stage(rsl_batch* b, void* f_dev, void* work_dev, int stage, void* hip_stream) {
    if (!b || !f_dev || !work_dev) return set_error(RSL_EINVAL, "null argument");
    if (b->kind != RSL_SOD) return set_error(RSL_EINVAL, "single stages exist for Sod batches only");
    if (stage < 1 || stage > 3) return set_error(RSL_EINVAL, "stage must be 1, 2 or 3");
    if (b->imex) return set_error(RSL_EUNSTABLE, kImexOnly);
    return batch_stage_all(b, stage, (char*)f_dev, (char*)work_dev, (hipStream_t)hip_stream, 0);
}

int rsl_batch_step(rsl_batch* b, void* f_dev, void* work_dev, int nsteps, void* hip_stream) {
    if (!b || !f_dev || !work_dev) return set_error(RSL_EINVAL, "null argument");
    if (nsteps < 0) return set_error(RSL_EINVAL, "nsteps < 0");
    if (b->imex) return set_error(RSL_EUNSTABLE, kImexOnly);
    const int rc = batch_steps(b, (char*)f_dev, (char*)work_dev, nsteps, (hipStream_t)hip_stream);
    if (rc == RSL_OK)
        for (int i = 0; i < b->n; ++i) b->t[i] += nsteps * b->dt[i];
    return rc;
}

int rsl_batch_graph_step(rsl_batch* b, void* f_dev, void* work_dev, int nsteps, void* hip_stream) {
    if (!b || !f_dev || !work_dev) return set_error(RSL_EINVAL, "null argument");
    if (nsteps <= 0) return set_error(RSL_EINVAL, "nsteps must be > 0");
    if (b->imex) return set_error(RSL_EUNSTABLE, kImexOnly);
    hipStream_t s = (hipStream_t)hip_stream;
    if (!s) return set_error(RSL_EINVAL, "graph replay needs an explicit (non-default) stream");
    int rc = RSL_OK;
    if (!b->gexec || b->g_f != f_dev || b->g_w != work_dev || b->g_steps != nsteps || b->g_stream != s) {
        batch_drop_graph(b);
        if (b->kind == RSL_SOD && (rc = batch_streams(b))) return rc;
        if ((rc = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture")))
            return rc;
        rc = batch_steps(b, (char*)f_dev, (char*)work_dev, nsteps, s);
        hipGraph_t g = nullptr;
        const int rc2 = hip_check(hipStreamEndCapture(s, &g), "hipStreamEndCapture");
        if (rc == RSL_OK) rc = rc2;
        if (rc != RSL_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        b->graph = g;
        if ((rc = hip_check(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0), "hipGraphInstantiate"))) {
            batch_drop_graph(b);
            return rc;
        }
        b->g_f = f_dev;
        b->g_w = work_dev;
        b->g_steps = nsteps;
        b->g_stream = s;
    }
    if ((rc = hip_check(hipGraphLaunch(b->gexec, s), "hipGraphLaunch"))) return rc;
    for (int i = 0; i < b->n; ++i) b->t[i] += nsteps * b->dt[i];
    return RSL_OK;
}

int rsl_batch_moments(rsl_batch* b, const void* f_dev, void* work_dev, double* out_dev, int fields,
                      void* hip_stream) {
    if (!b || !f_dev || !work_dev || !out_dev) return set_error(RSL_EINVAL, "null argument");
    size_t row = 0;
    for (int i = 0; i < b->n; ++i) {
        int rc = rsl_moments(b->quads[i], &b->probs[i], (const char*)f_dev + b->f_off[i],
                             (char*)work_dev + b->w_off[i], out_dev + row * fields, fields, hip_stream);
        if (rc) return rc;
        row += b->probs[i].problem == RSL_SOD ? b->probs[i].nz : 1;
    }
    return RSL_OK;
}

int rsl_batch_set_path(rsl_batch* b, int path) {
    if (!b || path < -1 || path > 1) return set_error(RSL_EINVAL, "bad batch path");
    if (path == 1 && !b->use_mfma) return set_error(RSL_EUNSUPPORTED, "matrix-core path not available for this batch");
    b->bj_path = path;
    batch_drop_graph(b);
    return RSL_OK;
}

int rsl_batch_groups(const rsl_batch* b, int* ngroups, int* sizes, int cap) {
    if (!b || !ngroups || cap < 0) return set_error(RSL_EINVAL, "bad batch group query");
    *ngroups = b->use_mfma ? b->ngroups : 0;
    if (sizes)
        for (int g = 0; g < std::min(*ngroups, cap); ++g) sizes[g] = b->group_sizes[g];
    return RSL_OK;
}

int rsl_stage_variant(int var, int* waves, int* vel_per_slot, int* lanes_per_vel, int* max_v, int* cell_waves,
                      int* form) {
    int W, NV, TW, WC, fm;
    if (!stage_variant_shape(var, &W, &NV, &TW, &fm, &WC))
        return set_error(RSL_EINVAL, "unknown stage kernel variant");
    if (form) *form = fm;
    if (waves) *waves = W;
    if (vel_per_slot) *vel_per_slot = NV;
    if (lanes_per_vel) *lanes_per_vel = TW;
    if (max_v) *max_v = stage_variant_capacity(var);
    if (cell_waves) *cell_waves = WC;
    return RSL_OK;
}

int rsl_batch_variant(const rsl_batch* b, int cls, int* var, int* max_v) {
    if (!b || cls < 0 || cls > kClasses) return set_error(RSL_EINVAL, "bad batch class");
    const StageClass& cl = cls < kClasses ? b->launch.cl[cls] : b->launch.all;
    if (var) *var = cl.nitems && (cls < kClasses || b->merged) ? cl.var : -1;
    if (max_v) *max_v = cl.maxV;
    return RSL_OK;
}

int rsl_batch_set_variant(rsl_batch* b, int cls, int var) {
    if (!b || cls < 0 || cls > kClasses) return set_error(RSL_EINVAL, "bad batch class");
    if (b->kind != RSL_SOD) return set_error(RSL_EINVAL, "kernel variants exist for Sod batches only");
    if (cls == kClasses && var < 0) {
        b->merged = false;
        batch_drop_graph(b);
        return RSL_OK;
    }
    StageClass& cl = cls < kClasses ? b->launch.cl[cls] : b->launch.all;
    if (var < 0) var = stage_default_variant(cls);
    const int cap = stage_variant_capacity(var);
    if (cap == 0) return set_error(RSL_EINVAL, "unknown stage kernel variant");
    if (cap < cl.maxV) return set_error(RSL_EINVAL, "variant holds fewer velocities than the class needs");
    use_variant(cl, var);
    if (cls == kClasses) b->merged = true;
    batch_drop_graph(b);
    return RSL_OK;
}

int rsl_batch_autotune(rsl_batch* b, void* f_dev, void* work_dev, int reps, void* hip_stream, int* chosen) {
    if (!b || !f_dev || !work_dev) return set_error(RSL_EINVAL, "null argument");
    if (b->kind != RSL_SOD) return set_error(RSL_EINVAL, "kernel variants exist for Sod batches only");
    if (reps <= 0) return set_error(RSL_EINVAL, "reps must be > 0");
    if (b->imex) return set_error(RSL_EUNSTABLE, kImexOnly);
    hipStream_t s = (hipStream_t)hip_stream;
    char* f = (char*)f_dev;
    char* w = (char*)work_dev;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = hip_check(hipEventCreate(&e0), "hipEventCreate");
    if (rc == RSL_OK) rc = hip_check(hipEventCreate(&e1), "hipEventCreate");
    for (int c = 0; c < kClasses && rc == RSL_OK; ++c) {
        StageClass& cl = b->launch.cl[c];
        if (chosen) chosen[c] = -1;
        if (!cl.nitems) continue;
        // stage 1 once, so that stage 2 (which reads f and f^(1) and writes
        // only f^(2) and the status word) can be repeated on valid data
        use_variant(cl, stage_default_variant(c));
        rc = launch_sod_class_stage(cl, b->dtype, 1, f, w, s, 0);
        int best = cl.var;
        float best_ms = 1e30f;
        for (int v = 0; rc == RSL_OK && stage_variant_capacity(v) > 0; ++v) {
            if (stage_variant_capacity(v) < cl.maxV) continue;
            use_variant(cl, v);
            // (the loop form's stage 2 reads the coefficients a previous stage
            // left; their values do not change the work, so the timing holds)
            rc = launch_sod_class_stage(cl, b->dtype, 2, f, w, s, 1);
            if (rc == RSL_OK) rc = hip_check(hipEventRecord(e0, s), "hipEventRecord");
            for (int r = 0; r < reps && rc == RSL_OK; ++r)
                rc = launch_sod_class_stage(cl, b->dtype, 2, f, w, s, 1);
            if (rc == RSL_OK) rc = hip_check(hipEventRecord(e1, s), "hipEventRecord");
            if (rc == RSL_OK) rc = hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.0f;
            if (rc == RSL_OK) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            if (rc == RSL_OK && ms < best_ms) {
                best_ms = ms;
                best = v;
            }
        }
        use_variant(cl, best);
        if (chosen) chosen[c] = best;
    }
    // then the whole batch: the classes on their streams against every
    // instance in one class, per variant that takes the largest V, timed on
    // 2 reps whole steps replayed from a captured graph (as graph_step runs
    // them), best of two
    void* fsave = nullptr;
    auto time_all = [&](float* ms) {
        *ms = 1e30f;
        int r2 = RSL_OK;
        hipGraphExec_t ge = nullptr;
        // every candidate from the same state (the cost of a step depends on it)
        auto restore = [&]() {
            return hip_check(hipMemcpyAsync(f, fsave, b->f_bytes, hipMemcpyDeviceToDevice, s), "restore f");
        };
        if (s) {
            if (b->launch.all.nitems && (r2 = batch_streams(b))) return r2;
            r2 = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            if (r2 == RSL_OK) {
                const int r3 = batch_sod_steps(b, f, w, 2 * reps, s);
                hipGraph_t g = nullptr;
                const int r4 = hip_check(hipStreamEndCapture(s, &g), "hipStreamEndCapture");
                r2 = r3 != RSL_OK ? r3 : r4;
                if (r2 == RSL_OK) r2 = hip_check(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0), "hipGraphInstantiate");
                if (g) (void)hipGraphDestroy(g);
            }
        }
        auto run = [&]() {
            return ge ? hip_check(hipGraphLaunch(ge, s), "hipGraphLaunch") : batch_sod_steps(b, f, w, 2 * reps, s);
        };
        if (r2 == RSL_OK) r2 = restore();
        if (r2 == RSL_OK) r2 = run();
        for (int trial = 0; trial < 2 && r2 == RSL_OK; ++trial) {
            float t = 0.0f;
            r2 = restore();
            if (r2 == RSL_OK) r2 = hip_check(hipEventRecord(e0, s), "hipEventRecord");
            if (r2 == RSL_OK) r2 = run();
            if (r2 == RSL_OK) r2 = hip_check(hipEventRecord(e1, s), "hipEventRecord");
            if (r2 == RSL_OK) r2 = hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
            if (r2 == RSL_OK) r2 = hip_check(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
            if (r2 == RSL_OK) *ms = std::min(*ms, t);
        }
        if (ge) (void)hipGraphExecDestroy(ge);
        return r2;
    };
    // (whole steps on the real data: f is saved first and restored after)
    const bool whole = rc == RSL_OK && b->launch.all.nitems;
    if (whole) {
        rc = hip_check(hipMalloc(&fsave, b->f_bytes), "hipMalloc(autotune copy of f)");
        if (rc == RSL_OK) rc = hip_check(hipMemcpyAsync(fsave, f, b->f_bytes, hipMemcpyDeviceToDevice, s), "copy f");
    }
    if (whole && rc == RSL_OK) {
        b->merged = false;
        float best_ms = 1e30f;
        rc = time_all(&best_ms);
        int best = -1;
        for (int v = 0; rc == RSL_OK && stage_variant_capacity(v) > 0; ++v) {
            if (stage_variant_capacity(v) < b->launch.all.maxV) continue;
            use_variant(b->launch.all, v);
            b->merged = true;
            float ms = 0.0f;
            rc = time_all(&ms);
            if (rc == RSL_OK && ms < best_ms) {
                best_ms = ms;
                best = v;
            }
        }
        b->merged = best >= 0;
        if (best >= 0) use_variant(b->launch.all, best);
    }
    if (fsave) {
        const int rc2 = hip_check(hipMemcpyAsync(f, fsave, b->f_bytes, hipMemcpyDeviceToDevice, s), "restore f");
        const int rc3 = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        (void)hipFree(fsave);
        if (rc == RSL_OK) rc = rc2 != RSL_OK ? rc2 : rc3;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    batch_drop_graph(b);
    return rc;
}

int rsl_batch_status(rsl_batch* b, void* work_dev, void* hip_stream, int* first_bad) {
    if (!b || !work_dev) return set_error(RSL_EINVAL, "null argument");
    if (first_bad) *first_bad = -1;
    for (int i = 0; i < b->n; ++i) {
        int rc = rsl_status(b->quads[i], &b->probs[i], (char*)work_dev + b->w_off[i], hip_stream);
        if (rc) {
            if (first_bad) *first_bad = i;
            return rc;
        }
    }
    return RSL_OK;
}

int rsl_batch_instance_status(rsl_batch* b, void* work_dev, void* hip_stream, int* status) {
    if (!b || !work_dev || !status) return set_error(RSL_EINVAL, "null argument");
    for (int i = 0; i < b->n; ++i) {
        const int rc = rsl_status(b->quads[i], &b->probs[i], (char*)work_dev + b->w_off[i], hip_stream);
        if (rc != RSL_OK && rc != RSL_ENONFINITE) return rc;
        status[i] = rc;
    }
    return RSL_OK;
}

}  // extern "C"

int rsl_batch_step_imex(rsl_batch* b, void* f_dev, void* work_dev, int nsteps, void* hip_stream) {
    if (!b || !f_dev || !work_dev) return set_error(RSL_EINVAL, "null argument");
    if (b->kind != RSL_SOD) return set_error(RSL_EUNSUPPORTED, "IMEX steps are built for Sod batches");
    if (nsteps < 0) return set_error(RSL_EINVAL, "nsteps < 0");
    int rc;
    for (int i = 0; i < b->n; ++i)
        if ((rc = check_cfl(b->quads[i], &b->probs[i], b->dt[i])))
            return set_error(rc, "batch instance " + std::to_string(i) + ": " + rsl_last_error());
    if (nsteps == 0) return RSL_OK;
    if ((rc = imex_items(b))) return rc;
    rc = launch_imex_batch_steps(b->launch.all.descs, b->imex_items, b->dtype, (char*)f_dev, (char*)work_dev, nsteps,
                                 (hipStream_t)hip_stream);
    if (rc) return rc;
    for (int i = 0; i < b->n; ++i) b->t[i] += nsteps * b->dt[i];
    return RSL_OK;
}
