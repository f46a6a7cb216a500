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
#include <vector>

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
    int stash_limit = -1;                   // -1: chosen by the library
};

namespace rsl {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Estimated cost of one tile of instance i in units of one cell-velocity update;
// the per-cell work (Landau frame, equilibrium coefficients) is ~25 updates.
double tile_cost(const rsl_quad* q) { return (double)kLanes * (q->V + 25.0); }

std::vector<int2> schedule(const rsl_batch* b) {
    const int X = 8;
    std::vector<int> order(b->n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return b->quads[a]->V > b->quads[c]->V; });
    std::vector<std::vector<std::pair<double, int2>>> q(X);
    std::vector<double> load(X, 0.0);
    for (int i : order) {
        const int nt = (b->probs[i].nz + kTileCells - 1) / kTileCells;
        const double c = tile_cost(b->quads[i]);
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

int batch_upload(rsl_batch* b) {
    std::vector<int2> items;
    if (b->kind == RSL_SOD) {
        items = schedule(b);
        const size_t es = b->dtype == RSL_F64 ? 8 : 4;
        // LDS windows: by default every instance whose window fits in 64 KiB
        // (two workgroups per CU) uses one, unless all fit in the per-WG limit.
        size_t maxw = 0, limit = b->stash_limit >= 0 ? (size_t)b->stash_limit : 0;
        for (int i = 0; i < b->n; ++i) maxw = std::max(maxw, (size_t)b->quads[i]->V * kWin * es);
        if (b->stash_limit < 0) {
            const size_t cap = sod_max_lds() - sod_red_bytes();
            limit = maxw <= cap ? maxw : 64 * 1024 - sod_red_bytes();
        }
        size_t used = 0;
        for (int i = 0; i < b->n; ++i) {
            const size_t w = (size_t)b->quads[i]->V * kWin * es;
            if (w <= limit) used = std::max(used, w);
        }
        b->launch.stash_limit = (int)limit;
        b->launch.lds_bytes = sod_red_bytes() + used;
    }
    const size_t dbytes = align_up(sizeof(InstDesc) * b->n, 256);
    const size_t ibytes = sizeof(int2) * items.size();
    int rc = hip_check(hipMalloc(&b->dmem, dbytes + std::max<size_t>(ibytes, 256)), "hipMalloc(batch)");
    if (rc) return rc;
    rc = hip_check(hipMemcpy(b->dmem, b->host_desc.data(), sizeof(InstDesc) * b->n, hipMemcpyHostToDevice),
                   "hipMemcpy(batch descriptors)");
    if (rc) return rc;
    if (ibytes)
        rc = hip_check(hipMemcpy((char*)b->dmem + dbytes, items.data(), ibytes, hipMemcpyHostToDevice),
                       "hipMemcpy(batch items)");
    b->launch.descs = (const InstDesc*)b->dmem;
    b->launch.items = (const int2*)((char*)b->dmem + dbytes);
    b->launch.nitems = (int)items.size();
    return rc;
}

}  // namespace rsl

using namespace rsl;

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
            if (rc == RSL_OK && !(dt[i] > 0.0 && std::isfinite(dt[i]))) rc = set_error(RSL_EINVAL, "dt must be > 0");
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
    if (b->dmem) (void)hipFree(b->dmem);
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
    return launch_sod_batch_stage(b->launch, b->dtype, stage, (char*)f_dev, (char*)work_dev, (hipStream_t)hip_stream);
}

int rsl_batch_step(rsl_batch* b, void* f_dev, void* work_dev, int nsteps, void* hip_stream) {
    if (!b || !f_dev || !work_dev) return set_error(RSL_EINVAL, "null argument");
    if (nsteps < 0) return set_error(RSL_EINVAL, "nsteps < 0");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = RSL_OK;
    if (b->kind == RSL_SOD) {
        for (int it = 0; it < nsteps && rc == RSL_OK; ++it)
            for (int st = 1; st <= 3 && rc == RSL_OK; ++st)
                rc = launch_sod_batch_stage(b->launch, b->dtype, st, (char*)f_dev, (char*)work_dev, s);
    } else if (nsteps > 0) {
        rc = launch_bj_batch_steps(b->launch.descs, b->n, b->bj_lds, b->dtype, (char*)f_dev, (char*)work_dev, 0.0,
                                   0.0, nsteps, s);
    }
    if (rc == RSL_OK)
        for (int i = 0; i < b->n; ++i) b->t[i] += nsteps * b->dt[i];
    return rc;
}

int rsl_batch_moments(rsl_batch* b, const void* f_dev, void* work_dev, double* out_dev, void* hip_stream) {
    if (!b || !f_dev || !work_dev || !out_dev) return set_error(RSL_EINVAL, "null argument");
    size_t row = 0;
    for (int i = 0; i < b->n; ++i) {
        int rc = rsl_moments(b->quads[i], &b->probs[i], (const char*)f_dev + b->f_off[i],
                             (char*)work_dev + b->w_off[i], out_dev + row * RSL_NMOM, hip_stream);
        if (rc) return rc;
        row += b->probs[i].problem == RSL_SOD ? b->probs[i].nz : 1;
    }
    return RSL_OK;
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

}  // extern "C"
