// Batched and served forms of the CDUGKS library (see include/cdugks.h), and
// the launch-shape autotuner.
//
// Batched: all problems of a batch advance together.  Per step there is one
// persistent launch per class (storage precision, whether the problems have
// Dirichlet sides, the reconstruction option, and whether they have an
// external acceleration) for the face sums and for the update,
// and one launch each for the per-face and per-cell closures over all
// problems.  Step sequences are captured as HIP graphs of chunk_steps steps.
// Every kernel computes each (problem, tile, velocity slice) item exactly as
// the single-problem path does, so a problem's result does not depend on the
// batch it runs in.
//
// Served: a host thread admits queued requests while slots and the device
// memory budget allow, runs the active set as a batch in chunks, and retires
// requests at chunk boundaries when their step count is reached.
#include "cdugks.h"
#include "cdugks_host.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using namespace cdg;

namespace {

struct StorageClass {
    int storage = 0;
    bool dirichlet = false;  // members have Dirichlet sides (face-sum variant)
    bool single_slope = false;  // members use the single-slope reconstruction
    bool accel = false;  // members have an external acceleration (kernel variants)
    int maxd = 1;
    WorkItem* items_fs = nullptr;  // device
    int n_fs = 0, grid_fs = 0;
    WorkItem* items_up = nullptr;  // device
    int n_up = 0, grid_up = 0;
    int* queue = nullptr;  // device work counters: [0] face sums, [1] update
};

int device_cus() {
    static int cus = -1;
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    if (cus < 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        else
            cus = 256;
        (void)hipGetLastError();
    }
    return cus;
}

// ---------------------------------------------------------------------------
// autotuner table: class key -> update slices and persistent grid factor
// ---------------------------------------------------------------------------
struct TuneEntry {
    int upd_slices = 0;   // 0 = the occupancy rule
    int grid_factor = 1;  // persistent grid = factor x resident slots
    int face_tile = -1;   // face-sum tile shape of single-problem launches (-1: the default)
};

std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;

std::string class_key(const Resolved& r) {
    long long nb = 1;
    while (nb < r.N) nb <<= 1;  // cell-count bucket: next power of two
    char buf[128];
    snprintf(buf, sizeof buf, "d%d_s%d_r%d_a%d_v%lld_n%lld", r.D, r.storage, r.recon, r.has_accel ? 1 : 0, r.V, nb);
    return buf;
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("CDUGKS_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    // one entry per line: "key upd_slices grid_factor [face_tile]"
    char line[256];
    while (fgets(line, sizeof line, f)) {
        char key[128];
        int us = 0, gf = 1, ft = -1;
        const int got = sscanf(line, "%127s %d %d %d", key, &us, &gf, &ft);
        if (got >= 3) g_tune[key] = TuneEntry{us, gf, got == 4 ? ft : -1};
    }
    fclose(f);
}

void tune_save_locked() {
    const char* path = getenv("CDUGKS_TUNE_CACHE");
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    for (auto& kv : g_tune)
        fprintf(f, "%s %d %d %d\n", kv.first.c_str(), kv.second.upd_slices, kv.second.grid_factor,
                kv.second.face_tile);
    fclose(f);
    rename(tmp.c_str(), path);
}

TuneEntry tune_lookup(const Resolved& r) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(class_key(r));
    return it == g_tune.end() ? TuneEntry{} : it->second;
}

}  // namespace

// ---------------------------------------------------------------------------
// batch object
// ---------------------------------------------------------------------------
struct cdugks_batch {
    std::vector<cdugks_ctx*> ctxs;
    hipStream_t stream = nullptr;
    int chunk = 2;
    int phase = 0;  // 0: every context at the parity it had when batched
    char* dev = nullptr;
    Problem* d_probs[2] = {nullptr, nullptr};
    long long* d_face_off = nullptr;
    long long* d_cell_off = nullptr;
    long long face_total = 0, cell_total = 0;
    std::vector<StorageClass> classes;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    std::vector<hipStream_t> others;  // streams of members other than the batch stream
    hipEvent_t ev = nullptr;
};

namespace {

hipError_t enqueue_batch_step(cdugks_batch* b, int phase) {
    hipError_t e;
    const int np = (int)b->ctxs.size();
    const Problem* probs = b->d_probs[phase];
    for (auto& c : b->classes)
        if ((e = launch_face_sums_batched(probs, c.items_fs, c.n_fs, c.grid_fs, c.maxd, c.storage, c.dirichlet,
                                          c.single_slope, c.accel, c.queue, c.queue + 1, b->stream)) != hipSuccess)
            return e;
    if ((e = launch_face_close_batched(probs, b->d_face_off, np, b->face_total, b->stream)) != hipSuccess) return e;
    if ((e = launch_cell_close_batched(probs, b->d_cell_off, np, b->cell_total, b->stream)) != hipSuccess) return e;
    for (auto& c : b->classes)
        if ((e = launch_update_batched(probs, c.items_up, c.n_up, c.grid_up, c.maxd, c.storage, c.accel,
                                       c.queue + 1, c.queue, b->stream)) != hipSuccess)
            return e;
    return hipSuccess;
}

hipError_t capture_batch(cdugks_batch* b, int phase, hipGraphExec_t* exec) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int s = 0; s < b->chunk && le == hipSuccess; ++s) le = enqueue_batch_step(b, (phase + s) & 1);
    e = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

void batch_free(cdugks_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (int k = 0; k < 2; ++k)
        if (b->graph[k]) (void)hipGraphExecDestroy(b->graph[k]);
    if (b->dev) (void)hipFree(b->dev);
    if (b->ev) (void)hipEventDestroy(b->ev);
    for (auto* c : b->ctxs) c->in_batch = false;
    delete b;
}

// Tiles along axis d of a problem in the batched tile shape.
int batched_tiles(const Resolved& r, int d) {
    const TileExt t = tile_shape(r.D, batched_face_tile(r.D, r.storage));
    const int te[3] = {t.x, t.y, t.z};
    return (r.ne[d] + te[d] - 1) / te[d];
}

// Velocity slices of a problem's update items in a batch: the autotuner's
// split for the problem's class when it has one (its trials time this very
// path), else at least BATCH_UPD_VELOCITIES velocities per item (all of them
// for smaller velocity sets), never more slices than the problem's own plan.
constexpr int BATCH_UPD_VELOCITIES = 256;
int batch_update_slices(const Resolved& r) {
    if (const int tu = tune_lookup(r).upd_slices; tu > 0) return (int)std::min<long long>(tu, r.V);
    const long long s = std::max(1LL, r.V / BATCH_UPD_VELOCITIES);
    return (int)std::min<long long>(s, std::max(1, r.nslices_upd));
}

// Build device tables for a set of contexts.
int batch_build(cdugks_ctx* const* ctxs, int count, int chunk_steps, cdugks_batch** out) {
    if (!out) return fail(CDUGKS_ERR_INVALID, "null output pointer");
    *out = nullptr;
    if (!ctxs || count <= 0) return fail(CDUGKS_ERR_INVALID, "empty batch");
    hipStream_t stream = ctxs[0]->stream;
    for (int j = 0; j < count; ++j) {
        if (!ctxs[j]) return fail(CDUGKS_ERR_INVALID, "null context in batch");
        if (ctxs[j]->in_batch) return fail(CDUGKS_ERR_BUSY, "context already belongs to a batch");
        if (ctxs[j]->sticky) return fail(ctxs[j]->sticky, "context is in an error state");
        for (int k = 0; k < j; ++k)
            if (ctxs[k] == ctxs[j]) return fail(CDUGKS_ERR_INVALID, "context listed twice");
    }
    cdugks_batch* b = new (std::nothrow) cdugks_batch();
    if (!b) return fail(CDUGKS_ERR_NOMEM, "host allocation failed");
    b->ctxs.assign(ctxs, ctxs + count);
    b->stream = stream;
    for (int j = 0; j < count; ++j)
        if (ctxs[j]->stream != stream &&
            std::find(b->others.begin(), b->others.end(), ctxs[j]->stream) == b->others.end())
            b->others.push_back(ctxs[j]->stream);
    if (!b->others.empty() && hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return fail(CDUGKS_ERR_DEVICE, "event create");
    }
    b->chunk = std::max(2, chunk_steps + (chunk_steps & 1));  // even: parity returns

    // host tables
    std::vector<Problem> probs[2];
    std::vector<long long> face_off(count), cell_off(count);
    long long ft = 0, ct = 0;
    for (int j = 0; j < count; ++j) {
        cdugks_ctx* c = ctxs[j];
        for (int p = 0; p < 2; ++p) {
            Problem P = c->P;
            set_pingpong(P, c->r, c->base, c->cur ^ p);
            // batched launches run the batched tile shape of the problem's
            // dimension and storage form (the same result as any other shape)
            P.tile = batched_face_tile(c->r.D, c->r.storage);
            for (int d = 0; d < 3; ++d) P.tiles1[d] = batched_tiles(c->r, d);
            probs[p].push_back(P);
        }
        face_off[j] = ft;
        cell_off[j] = ct;
        // each problem's closure threads start on a workgroup boundary
        ft += (c->r.NE * c->r.D + WG - 1) / WG * WG;
        ct += (c->r.N + WG - 1) / WG * WG;
    }
    b->face_total = ft;
    b->cell_total = ct;
    // work lists per class, sorted by estimated cost (largest first):
    // 3 storage forms x (with, without Dirichlet sides) x 2 reconstructions x
    // (with, without an external acceleration)
    constexpr int NCLASS = 24;
    std::vector<std::vector<WorkItem>> fs(NCLASS), up(NCLASS);
    std::vector<std::vector<double>> cfs(NCLASS), cup(NCLASS);
    int maxd[NCLASS] = {};
    auto class_of = [](const Resolved& r) {
        return ((2 * r.storage + (r.any_dirichlet ? 1 : 0)) * 2 + r.recon) * 2 + (r.has_accel ? 1 : 0);
    };
    for (int j = 0; j < count; ++j) {
        const Resolved& r = ctxs[j]->r;
        const int s = class_of(r);
        maxd[s] = std::max(maxd[s], r.D);
        const int nt = batched_tiles(r, 0) * batched_tiles(r, 1) * batched_tiles(r, 2);
        const double vpt = (double)r.V / r.nslices;
        for (int sl = 0; sl < r.nslices; ++sl)
            for (int t = 0; t < nt; ++t) {
                fs[s].push_back(WorkItem{j, t, sl, 0});
                cfs[s].push_back(vpt * r.D * (r.D + 1));
            }
        // Update items take the batch's own velocity split: the update forms
        // no sums, so its split never changes a result, and the batch has
        // work enough to fill the device without the many short slices a
        // small problem uses alone, each of which loads the cell's and its
        // faces' coefficient sets again.
        const int nb = (int)((r.N + WG - 1) / WG);
        const int us = batch_update_slices(r);
        const double vpu = (double)r.V / us;
        for (int sl = 0; sl < us; ++sl)
            for (int t = 0; t < nb; ++t) {
                up[s].push_back(WorkItem{j, t, sl, us});
                cup[s].push_back(vpu * r.D);
            }
    }
    auto sort_by_cost = [](std::vector<WorkItem>& it, const std::vector<double>& cost) {
        std::vector<size_t> idx(it.size());
        for (size_t k = 0; k < idx.size(); ++k) idx[k] = k;
        std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t c) { return cost[a] > cost[c]; });
        std::vector<WorkItem> o(it.size());
        for (size_t k = 0; k < idx.size(); ++k) o[k] = it[idx[k]];
        it.swap(o);
    };
    size_t bytes = 0;
    auto reserve = [&](size_t n) {
        size_t o = bytes;
        bytes += (n + 255) & ~size_t(255);
        return o;
    };
    size_t o_p0 = reserve(sizeof(Problem) * count), o_p1 = reserve(sizeof(Problem) * count);
    size_t o_fo = reserve(sizeof(long long) * count), o_co = reserve(sizeof(long long) * count);
    size_t o_fs[NCLASS], o_up[NCLASS], o_q[NCLASS];
    for (int s = 0; s < NCLASS; ++s) {
        sort_by_cost(fs[s], cfs[s]);
        sort_by_cost(up[s], cup[s]);
        o_fs[s] = reserve(sizeof(WorkItem) * std::max<size_t>(1, fs[s].size()));
        o_up[s] = reserve(sizeof(WorkItem) * std::max<size_t>(1, up[s].size()));
        o_q[s] = reserve(2 * sizeof(int));  // zero in the uploaded image
    }
    hipError_t e = hipMalloc(&b->dev, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return fail(CDUGKS_ERR_NOMEM, "batch tables (%zu bytes)", bytes);
    }
    std::vector<char> host(bytes, 0);
    std::memcpy(host.data() + o_p0, probs[0].data(), sizeof(Problem) * count);
    std::memcpy(host.data() + o_p1, probs[1].data(), sizeof(Problem) * count);
    std::memcpy(host.data() + o_fo, face_off.data(), sizeof(long long) * count);
    std::memcpy(host.data() + o_co, cell_off.data(), sizeof(long long) * count);
    for (int s = 0; s < NCLASS; ++s) {
        if (!fs[s].empty()) std::memcpy(host.data() + o_fs[s], fs[s].data(), sizeof(WorkItem) * fs[s].size());
        if (!up[s].empty()) std::memcpy(host.data() + o_up[s], up[s].data(), sizeof(WorkItem) * up[s].size());
    }
    if ((e = hipMemcpyAsync(b->dev, host.data(), bytes, hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "batch table upload");
    }
    b->d_probs[0] = (Problem*)(b->dev + o_p0);
    b->d_probs[1] = (Problem*)(b->dev + o_p1);
    b->d_face_off = (long long*)(b->dev + o_fo);
    b->d_cell_off = (long long*)(b->dev + o_co);
    const int cus = device_cus();
    for (int s = 0; s < NCLASS; ++s) {
        if (fs[s].empty()) continue;
        StorageClass sc;
        sc.storage = s / 8;
        sc.dirichlet = (s / 4) % 2 == 1;
        sc.single_slope = (s / 2) % 2 == 1;
        sc.accel = s % 2 == 1;
        sc.maxd = maxd[s];
        // persistent grids: resident slots (times the tuned factor of the
        // largest class member), never more than the work items
        int gf = 1;
        for (int j = 0; j < count; ++j)
            if (class_of(ctxs[j]->r) == s) gf = std::max(gf, tune_lookup(ctxs[j]->r).grid_factor);
        int bfs = std::max(1, batched_blocks_per_cu(sc.maxd, sc.storage, sc.accel, false));
        int bup = std::max(1, batched_blocks_per_cu(sc.maxd, sc.storage, sc.accel, true));
        sc.items_fs = (WorkItem*)(b->dev + o_fs[s]);
        sc.n_fs = (int)fs[s].size();
        sc.grid_fs = (int)std::min<long long>(sc.n_fs, (long long)cus * bfs * gf);
        sc.queue = (int*)(b->dev + o_q[s]);
        sc.items_up = (WorkItem*)(b->dev + o_up[s]);
        sc.n_up = (int)up[s].size();
        sc.grid_up = (int)std::min<long long>(sc.n_up, (long long)cus * bup * gf);
        b->classes.push_back(sc);
    }
    for (auto* c : b->ctxs) c->in_batch = true;
    *out = b;
    return CDUGKS_OK;
}

int batch_advance(cdugks_batch* b, int64_t nsteps) {
    if (!b) return fail(CDUGKS_ERR_INVALID, "null batch");
    if (nsteps < 0) return fail(CDUGKS_ERR_INVALID, "negative step count");
    for (auto* c : b->ctxs)
        if (c->sticky) return fail(c->sticky, "a batched context is in an error state");
    hipError_t e;
    // members living on other streams: their earlier work comes first
    for (hipStream_t o : b->others)
        if ((e = hipEventRecord(b->ev, o)) != hipSuccess || (e = hipStreamWaitEvent(b->stream, b->ev, 0)) != hipSuccess)
            return hip_fail(e, "stream join");
    int64_t left = nsteps;
    while (left >= b->chunk) {
        hipGraphExec_t& g = b->graph[b->phase];
        if (!g && (e = capture_batch(b, b->phase, &g)) != hipSuccess) return hip_fail(e, "batch graph capture");
        if ((e = hipGraphLaunch(g, b->stream)) != hipSuccess) return hip_fail(e, "batch graph launch");
        left -= b->chunk;  // chunk is even: phase unchanged
    }
    for (; left > 0; --left) {
        if ((e = enqueue_batch_step(b, b->phase)) != hipSuccess) return hip_fail(e, "batch step");
        b->phase ^= 1;
    }
    for (auto* c : b->ctxs) {
        c->steps += nsteps;
        if (nsteps & 1) c->cur ^= 1;
    }
    // and later work on those streams waits for the batch
    if (!b->others.empty()) {
        if ((e = hipEventRecord(b->ev, b->stream)) != hipSuccess) return hip_fail(e, "stream join");
        for (hipStream_t o : b->others)
            if ((e = hipStreamWaitEvent(o, b->ev, 0)) != hipSuccess) return hip_fail(e, "stream join");
    }
    return CDUGKS_OK;
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ---------------------------------------------------------------------------
// served form
// ---------------------------------------------------------------------------
namespace {

struct Request {
    uint64_t ticket = 0;
    cdugks_space sp{};
    cdugks_velocity ve{};
    cdugks_params pa{};
    std::vector<double> rho, u, T;
    int64_t nsteps = 0;
    size_t bytes = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = CDUGKS_PENDING;  // read and written under the server lock
    int final_status = CDUGKS_OK;
    std::string error;
    cdugks_ctx* ctx = nullptr;
    int64_t remaining = 0;
    long long N = 0;
    int D = 1;
};

}  // namespace

struct cdugks_server {
    size_t budget = 0;
    int max_active = 1;
    int chunk = 100;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;  // the creating thread's device; the worker thread runs on it
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request*> queue;
    std::vector<Request*> active;
    std::map<uint64_t, Request*> live;  // every submitted, not yet collected request
    uint64_t next_ticket = 1;
    size_t used = 0;
    bool stop = false;
    std::thread worker;
};

namespace {

void server_loop(cdugks_server* s) {
    // a new thread starts on device 0; a failure here surfaces as the
    // requests' init errors
    (void)hipSetDevice(s->device);
    cdugks_batch* batch = nullptr;
    bool dirty = true;
    for (;;) {
        std::vector<Request*> admit;
        {
            std::unique_lock<std::mutex> lock(s->mu);
            s->cv.wait(lock, [&] { return s->stop || !s->queue.empty() || !s->active.empty(); });
            if (s->stop && s->queue.empty() && s->active.empty()) break;
            // admission at a chunk boundary: first come, first served, while
            // slots and the memory budget allow
            while (!s->queue.empty() && (int)(s->active.size() + admit.size()) < s->max_active &&
                   s->used + s->queue.front()->bytes <= s->budget) {
                Request* r = s->queue.front();
                s->queue.pop_front();
                s->used += r->bytes;
                admit.push_back(r);
            }
        }
        for (Request* r : admit) {
            r->t_admit = now_s();
            int rc = cdugks_init(&r->sp, &r->ve, &r->pa, r->rho.data(), r->u.data(), r->T.data(), s->stream,
                                 nullptr, 0, &r->ctx);
            std::lock_guard<std::mutex> lock(s->mu);
            if (rc) {
                r->status = rc;
                r->error = cdugks_last_error();
                r->t_done = now_s();
                s->used -= r->bytes;
                s->cv.notify_all();
                continue;
            }
            r->remaining = r->nsteps;
            s->active.push_back(r);
            dirty = true;
        }
        std::vector<Request*> act;
        {
            std::lock_guard<std::mutex> lock(s->mu);
            act = s->active;
        }
        if (act.empty()) continue;
        if (dirty) {
            if (batch) batch_free(batch);
            batch = nullptr;
            std::vector<cdugks_ctx*> cs;
            for (Request* r : act) cs.push_back(r->ctx);
            int rc = batch_build(cs.data(), (int)cs.size(), s->chunk, &batch);
            if (rc) {
                std::string msg = cdugks_last_error();
                std::lock_guard<std::mutex> lock(s->mu);
                for (Request* r : act) {
                    r->status = rc;
                    r->error = msg;
                    r->t_done = now_s();
                    cdugks_destroy(r->ctx);
                    r->ctx = nullptr;
                    s->used -= r->bytes;
                }
                s->active.clear();
                s->cv.notify_all();
                continue;
            }
            dirty = false;
        }
        // one chunk, cut short so that requests end exactly at their count
        int64_t steps = s->chunk;
        for (Request* r : act) steps = std::min(steps, r->remaining);
        int rc = steps > 0 ? batch_advance(batch, steps) : CDUGKS_OK;
        if (rc == CDUGKS_OK) (void)hipStreamSynchronize(s->stream);
        std::vector<Request*> done;
        for (Request* r : act) {
            r->remaining -= steps;
            int st = rc;
            if (st == CDUGKS_OK) st = cdugks_sync(r->ctx);  // per-request error flag
            if (st != CDUGKS_OK || r->remaining <= 0) {
                r->final_status = st;
                if (st != CDUGKS_OK) r->error = cdugks_last_error();
                done.push_back(r);
            }
        }
        if (!done.empty()) {
            batch_free(batch);  // releases in_batch on every context
            batch = nullptr;
            dirty = true;
            for (Request* r : done) {
                if (r->final_status == CDUGKS_OK) {
                    r->rho.assign(r->N, 0.0);
                    r->u.assign((size_t)r->D * r->N, 0.0);
                    r->T.assign(r->N, 0.0);
                    int mr = cdugks_moments(r->ctx, r->rho.data(), r->u.data(), r->T.data(), 0);
                    if (mr) {
                        r->final_status = mr;
                        r->error = cdugks_last_error();
                    }
                } else {
                    r->rho.clear();
                    r->u.clear();
                    r->T.clear();
                }
                cdugks_destroy(r->ctx);
                r->ctx = nullptr;
                r->t_done = now_s();
            }
            std::lock_guard<std::mutex> lock(s->mu);
            for (Request* r : done) {
                s->active.erase(std::find(s->active.begin(), s->active.end(), r));
                s->used -= r->bytes;
                r->status = r->final_status;  // published under the lock
            }
            s->cv.notify_all();
        }
    }
    if (batch) batch_free(batch);
}

}  // namespace

extern "C" {

int cdugks_batch_create(cdugks_ctx* const* ctxs, int count, int chunk_steps, cdugks_batch** out) {
    return batch_build(ctxs, count, chunk_steps, out);
}

int cdugks_batch_step(cdugks_batch* batch, int64_t nsteps) { return batch_advance(batch, nsteps); }

void cdugks_batch_destroy(cdugks_batch* batch) { batch_free(batch); }

int cdugks_server_create(size_t hbm_budget, int max_active, int chunk_steps, void* hip_stream,
                         cdugks_server** out) {
    if (!out) return fail(CDUGKS_ERR_INVALID, "null output pointer");
    *out = nullptr;
    if (hbm_budget == 0 || max_active <= 0 || chunk_steps <= 0)
        return fail(CDUGKS_ERR_INVALID, "budget, slots and chunk must be positive");
    cdugks_server* s = new (std::nothrow) cdugks_server();
    if (!s) return fail(CDUGKS_ERR_NOMEM, "host allocation failed");
    s->budget = hbm_budget;
    s->max_active = max_active;
    // even, like a batch's graph chunk: a full chunk then replays the
    // captured graph instead of launching its steps one by one
    s->chunk = chunk_steps + (chunk_steps & 1);
    hipError_t de = hipGetDevice(&s->device);
    if (de != hipSuccess) {
        delete s;
        return hip_fail(de, "get device");
    }
    s->stream = (hipStream_t)hip_stream;
    if (!s->stream) {
        hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete s;
            return hip_fail(e, "stream create");
        }
        s->own_stream = true;
    }
    try {
        s->worker = std::thread(server_loop, s);
    } catch (...) {
        if (s->own_stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return fail(CDUGKS_ERR_UNKNOWN, "could not start the server thread");
    }
    *out = s;
    return CDUGKS_OK;
}

int cdugks_submit(cdugks_server* s, const cdugks_space* space, const cdugks_velocity* vel,
                  const cdugks_params* params, const double* rho, const double* u, const double* T,
                  int64_t nsteps, uint64_t* ticket) {
    if (!s || !ticket || !rho || !u || !T) return fail(CDUGKS_ERR_INVALID, "null argument");
    if (nsteps < 0) return fail(CDUGKS_ERR_INVALID, "negative step count");
    Resolved r;
    int rc = resolve(space, vel, params, rho, &r);
    if (rc) return rc;
    if (r.bytes > s->budget)
        return fail(CDUGKS_ERR_TOO_LARGE, "request needs %zu bytes, budget is %zu", r.bytes, s->budget);
    for (long long c = 0; c < r.N; ++c)
        if (!(rho[c] > 0.0) || !(T[c] > 0.0) || !std::isfinite(rho[c]) || !std::isfinite(T[c]))
            return fail(CDUGKS_ERR_INVALID, "non-physical initial moments at cell %lld", c);
    Request* q = new (std::nothrow) Request();
    if (!q) return fail(CDUGKS_ERR_NOMEM, "host allocation failed");
    q->sp = *space;
    q->ve = *vel;
    q->pa = *params;
    q->rho.assign(rho, rho + r.N);
    q->u.assign(u, u + (size_t)r.D * r.N);
    q->T.assign(T, T + r.N);
    q->nsteps = nsteps;
    q->bytes = r.bytes;
    q->N = r.N;
    q->D = r.D;
    q->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lock(s->mu);
        if (s->stop) {
            delete q;
            return fail(CDUGKS_ERR_INVALID, "server is shutting down");
        }
        q->ticket = s->next_ticket++;
        s->queue.push_back(q);
        s->live[q->ticket] = q;
    }
    s->cv.notify_all();
    *ticket = q->ticket;
    return CDUGKS_OK;
}

int cdugks_poll(cdugks_server* s, uint64_t ticket, double* rho, double* u, double* T, double* t_queue_s,
                double* t_service_s) {
    if (!s) return fail(CDUGKS_ERR_INVALID, "null server");
    Request* r = nullptr;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        auto it = s->live.find(ticket);
        if (it == s->live.end())
            return fail(CDUGKS_ERR_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
        if (it->second->status == CDUGKS_PENDING) return CDUGKS_PENDING;
        r = it->second;
        s->live.erase(it);
    }
    int status = r->status;
    if (t_queue_s) *t_queue_s = r->t_admit - r->t_submit;
    if (t_service_s) *t_service_s = r->t_done - r->t_admit;
    if (status == CDUGKS_OK) {
        if (rho) std::memcpy(rho, r->rho.data(), sizeof(double) * r->N);
        if (u) std::memcpy(u, r->u.data(), sizeof(double) * r->D * r->N);
        if (T) std::memcpy(T, r->T.data(), sizeof(double) * r->N);
    } else {
        fail(status, "request failed: %s", r->error.c_str());
    }
    delete r;
    return status;
}

void cdugks_server_destroy(cdugks_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->live) delete kv.second;  // queued, failed or uncollected
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

int cdugks_autotune(cdugks_ctx* c, int steps_per_trial) {
    if (!c || steps_per_trial <= 0) return fail(CDUGKS_ERR_INVALID, "bad argument");
    if (c->in_batch) return fail(CDUGKS_ERR_BUSY, "context belongs to a batch");
    if (c->sticky) return fail(c->sticky, "context is in an error state");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(CDUGKS_ERR_DEVICE, "event create");
    // face-sum tile shapes usable for this problem: each times steps_per_trial
    // face-sum launches on the current state (rerunning the first phase of a
    // step changes nothing the next step reads before rewriting it)
    int best_tile = 0;
    {
        double best_ft = 1e300;
        for (int t = 0; t < tile_shape_count(c->r.D); ++t) {
            if (!face_tile_usable(c->r, t)) continue;
            Resolved rt = c->r;
            set_face_tile(rt, t);
            Problem P = c->P;
            set_pingpong(P, c->r, c->base, c->cur);
            P.tile = t;
            for (int d = 0; d < 3; ++d) P.tiles1[d] = rt.tiles1[d];
            float ms = 0.f;
            hipError_t he = launch_face_sums(P, c->stream);  // warm-up
            if (he == hipSuccess) he = hipEventRecord(e0, c->stream);
            for (int k = 0; k < steps_per_trial && he == hipSuccess; ++k) he = launch_face_sums(P, c->stream);
            if (he == hipSuccess) he = hipEventRecord(e1, c->stream);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return hip_fail(he, "face-sum tile trial");
            }
            if (ms < best_ft) {
                best_ft = ms;
                best_tile = t;
            }
        }
    }
    // candidates: update slices (occupancy rule x {1/2, 1, 2, 4}) and the
    // persistent grid factor {1, 2}; every candidate gives the same result
    const int base = c->r.nslices_upd;
    int cand_slices[4] = {std::max(1, base / 2), base, base * 2, base * 4};
    int best_s = base, best_g = 1;
    double best_t = 1e300;
    const Resolved saved = c->r;
    int rc = CDUGKS_OK;
    for (int gf = 1; gf <= 2 && rc == CDUGKS_OK; ++gf) {
        for (int k = 0; k < 4 && rc == CDUGKS_OK; ++k) {
            int sl = (int)std::min<long long>(cand_slices[k], saved.V);
            c->r.nslices_upd = sl;
            c->P.nslices_upd = sl;
            {
                std::lock_guard<std::mutex> lock(g_tune_mu);
                tune_load_locked();
                g_tune[class_key(c->r)] = TuneEntry{sl, gf, best_tile};
            }
            cdugks_batch* b = nullptr;
            cdugks_ctx* one[1] = {c};
            rc = batch_build(one, 1, steps_per_trial, &b);
            if (rc) break;
            rc = batch_advance(b, 2);  // warm-up
            float ms = 0.f;
            if (rc == CDUGKS_OK && hipEventRecord(e0, b->stream) == hipSuccess) {
                rc = batch_advance(b, steps_per_trial);
                if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                    rc = fail(CDUGKS_ERR_DEVICE, "timing");
            }
            batch_free(b);
            if (rc == CDUGKS_OK && ms < best_t) {
                best_t = ms;
                best_s = sl;
                best_g = gf;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the context takes the winners; its captured step graphs hold the old
    // launch shapes and are captured again at the next step
    c->r.nslices_upd = best_s;
    c->P.nslices_upd = best_s;
    set_face_tile(c->r, best_tile);
    c->P.tile = c->r.tile;
    for (int d = 0; d < 3; ++d) c->P.tiles1[d] = c->r.tiles1[d];
    for (int k = 0; k < 2; ++k)
        if (c->graph[k]) {
            (void)hipGraphExecDestroy(c->graph[k]);
            c->graph[k] = nullptr;
        }
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[class_key(c->r)] = TuneEntry{best_s, best_g, best_tile};
        tune_save_locked();
    }
    if (rc) return rc;
    return cdugks_sync(c);
}

}  // extern "C"

namespace cdg {
// Used by resolve(): the tuned update slices and face-sum tile shape of a
// problem class, if any.
int tuned_update_slices(const Resolved& r) { return tune_lookup(r).upd_slices; }
int tuned_face_tile(const Resolved& r) { return tune_lookup(r).face_tile; }
}  // namespace cdg
