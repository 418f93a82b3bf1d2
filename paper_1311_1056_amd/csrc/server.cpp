// server.cpp -- continuous batching of independent CL runs (cl_server_* in
// clgc.h).
//
// Arena layout (caller-owned device memory, the HBM budget):
//   [ per precision group: BatchHdr | RunArgs[kMaxRuns] | GatherRec[kMaxRuns] ]
//   [ run heap: one cl_lattice region per admitted run (first-fit allocator) ]
// A batch step launches each kernel kind once per precision group over the
// concatenated logical blocks of the group's runs (the two groups as parallel
// branches of the captured graph).  The launches use a fixed
// persistent grid and read the run table from device memory, so the captured
// step graph stays valid while runs come and go; it is keyed only by the
// launch sequence (largest cooling count, theta / D_2 present, groups present).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "../../include/clgc.h"
#include "engine.hpp"
#include "host.hpp"

using namespace clgc;

namespace {

constexpr int kPersistentGrid = 2048;  // physical blocks per batched launch

struct Run {
    uint64_t id = 0;
    cl_run_desc desc{};
    size_t off = 0, bytes = 0;
    cl_lattice* lat = nullptr;
    int steps_done = 0;
    double t_submit = 0, t_admit = 0, t_finish = 0;
    std::vector<float> step_ms;
    int status = CL_OK;
    cl_obs obs{};
    int64_t V = 0;
};

// final links of the finished runs submitted with keep_links, until taken
struct Kept {
    int64_t V = 0;
    std::vector<double> links;
};

}  // namespace

struct cl_server {
    char* arena = nullptr;
    size_t arena_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    // the second precision group's branch of a captured step, and the events
    // that fork it from and join it to the first
    hipStream_t cap_stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    Heap heap;
    size_t heap_base = 0;
    std::chrono::steady_clock::time_point t0;
    uint64_t next_id = 1;
    std::deque<std::unique_ptr<Run>> pending;
    std::vector<std::unique_ptr<Run>> active;
    std::deque<std::unique_ptr<Run>> done;
    // device tables and their pinned host images, one set per precision
    BatchHdr* d_hdr[2] = {nullptr, nullptr};
    RunArgs* d_runs[2] = {nullptr, nullptr};
    GatherRec* d_gather[2] = {nullptr, nullptr};
    BatchHdr* h_hdr[2] = {nullptr, nullptr};
    RunArgs* h_runs[2] = {nullptr, nullptr};
    GatherRec* h_gather[2] = {nullptr, nullptr};
    std::vector<Run*> group[2];
    bool dirty = true;
    // captured batch step
    hipGraphExec_t graph = nullptr;
    int graph_key[8] = {0};
    // statistics
    int64_t batch_steps = 0, link_updates = 0;
    double busy_s = 0;
    std::vector<float> all_step_ms;
    std::vector<float> waits;
    std::map<uint64_t, Kept> kept;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

size_t tables_bytes()
{
    return 2 * (align256(sizeof(BatchHdr)) + align256(sizeof(RunArgs) * kMaxRuns) +
                align256(sizeof(GatherRec) * kMaxRuns));
}

cl_status validate_run(const cl_run_desc* r)
{
    if (!r) return fail(CL_EINVAL, "run desc is NULL");
    cl_status st = check_desc(&r->lattice);
    if (st) return st;
    if (r->n_steps < 1) return fail(CL_EINVAL, "n_steps must be >= 1");
    if (!(r->step.eps0 > 0) || !std::isfinite(r->step.eps0)) return fail(CL_EINVAL, "eps0 must be > 0");
    if (r->cool.n_steps < 0 || r->cool.n_steps > kMaxCoolHist)
        return fail(CL_EINVAL, "cooling steps must be in 0..%d", kMaxCoolHist);
    if (r->cool.mode < 0 || r->cool.mode > 2) return fail(CL_EINVAL, "unknown cooling mode");
    if (!(r->cool.eps_c >= 0) || !std::isfinite(r->cool.alpha)) return fail(CL_EINVAL, "bad cooling parameters");
    return CL_OK;
}

// the run's descriptor with this run's step and cooling parameters
RunArgs run_args(const Run& r)
{
    RunArgs a = r.lat->args;
    a.eps0 = r.desc.step.eps0;
    a.adaptive = r.desc.step.adaptive != 0;
    a.drift_bound = r.desc.step.drift_bound;
    a.eps_c = r.desc.cool.eps_c;
    a.alpha = r.desc.cool.alpha;
    a.mode = r.desc.cool.mode;
    a.n_cool = r.desc.cool.n_steps;
    return a;
}

cl_status admit(cl_server* s)
{
    while (!s->pending.empty()) {
        Run& r = *s->pending.front();
        size_t off = 0;
        // FIFO: the head waits for a batch slot and memory to free up
        if (!admit_head(s->heap, r.bytes, (int)s->group[r.desc.lattice.precision].size(), kMaxRuns, &off)) break;
        r.off = off;
        cl_status st = cl_lattice_create(&r.desc.lattice, s->arena + s->heap_base + off, r.bytes, s->stream, &r.lat);
        if (st == CL_OK) st = cl_lattice_init(r.lat, 1, r.desc.sigma_x, r.desc.sigma_y);
        if (st != CL_OK) {
            s->heap.release(off, r.bytes);
            return st;
        }
        r.t_admit = s->now();
        s->group[r.desc.lattice.precision].push_back(&r);
        s->active.push_back(std::move(s->pending.front()));
        s->pending.pop_front();
        s->dirty = true;
    }
    return CL_OK;
}

cl_status upload_tables(cl_server* s)
{
    for (int g = 0; g < 2; ++g) {
        BatchHdr& h = *s->h_hdr[g];
        std::memset(&h, 0, sizeof h);
        h.nrun = (int)s->group[g].size();
        for (int k = 0; k < NKIND; ++k) h.begin[k][0] = 0;
        for (int i = 0; i < h.nrun; ++i) {
            const RunArgs a = run_args(*s->group[g][i]);
            s->h_runs[g][i] = a;
            for (int k = 0; k < NKIND; ++k) h.begin[k][i + 1] = h.begin[k][i] + a.nblk[k];
        }
        for (int k = 0; k < NKIND; ++k) h.total[k] = h.begin[k][h.nrun];
        HIP_TRY(hipMemcpyAsync(s->d_hdr[g], s->h_hdr[g], sizeof(BatchHdr), hipMemcpyHostToDevice, s->stream));
        if (h.nrun)
            HIP_TRY(hipMemcpyAsync(s->d_runs[g], s->h_runs[g], sizeof(RunArgs) * h.nrun, hipMemcpyHostToDevice,
                                   s->stream));
    }
    s->dirty = false;
    return CL_OK;
}

Launch group_launch(cl_server* s, int g, hipStream_t st)
{
    Launch L;
    L.hdr = s->d_hdr[g];
    L.runs = s->d_runs[g];
    for (int k = 0; k < NKIND; ++k) L.blocks[k] = kPersistentGrid;
    L.nrun = kMaxRuns;
    L.stream = st;
    return L;
}

// one batched step of one precision group: the sequence a single lattice
// runs, with each launch covering every run of the group
cl_status enqueue_group_step(cl_server* s, int g, int max_nc, bool any_theta, bool any_grad, hipStream_t st)
{
    const Launch L = group_launch(s, g, st);
    if (any_theta) HIP_TRY(launch_clover(L, g, 1));
    HIP_TRY(launch_drift(L, g, any_theta));
    HIP_TRY(launch_update(L, g));
    HIP_TRY(launch_finalize(L, FIN_UPDATE, 0));
    for (int i = 0; i < max_nc; ++i) {
        if (any_grad) {
            HIP_TRY(launch_gradnorm(L, g, i));
        }
        HIP_TRY(launch_cool(L, g, 0, i));
        HIP_TRY(launch_cool(L, g, 1, i));
    }
    if (max_nc > 0) HIP_TRY(launch_finalize(L, FIN_COOL, -1));  // each run's last cooling step
    HIP_TRY(launch_gather(L, s->d_gather[g]));
    return CL_OK;
}

cl_status ensure_graph(cl_server* s)
{
    int key[8] = {0};
    for (int g = 0; g < 2; ++g) {
        int mx = 0, th = 0, gr = 0;
        for (Run* r : s->group[g]) {
            mx = std::max(mx, r->desc.cool.n_steps);
            th |= r->lat->has_theta ? 1 : 0;
            gr |= r->desc.cool.mode == CL_ALPHA_GRAD ? 1 : 0;
        }
        key[4 * g + 0] = s->group[g].empty() ? 0 : 1;
        key[4 * g + 1] = mx;
        key[4 * g + 2] = th;
        key[4 * g + 3] = gr;
    }
    if (s->graph && std::memcmp(key, s->graph_key, sizeof key) == 0) return CL_OK;
    if (s->graph) {
        HIP_TRY(hipGraphExecDestroy(s->graph));
        s->graph = nullptr;
    }
    hipGraph_t gph = nullptr;
    cl_status st = CL_OK;
    hipError_t e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        // With both precision groups present their steps are independent (their
        // runs, tables and gather records are disjoint): the FP64 group on the
        // capture stream, the mixed group on a second stream forked from it and
        // joined back, so the graph holds two parallel branches whose kernels
        // can share the GPU.
        const bool both = key[0] && key[4];
        hipStream_t st1 = both ? s->cap_stream2 : s->cap_stream;
        if (both) {
            e = hipEventRecord(s->ev_fork, s->cap_stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(s->cap_stream2, s->ev_fork, 0);
        }
        for (int g = 0; g < 2 && st == CL_OK && e == hipSuccess; ++g)
            if (key[4 * g]) st = enqueue_group_step(s, g, key[4 * g + 1], key[4 * g + 2] != 0, key[4 * g + 3] != 0,
                                                     g == 0 ? s->cap_stream : st1);
        if (both && st == CL_OK && e == hipSuccess) {
            e = hipEventRecord(s->ev_join, s->cap_stream2);
            if (e == hipSuccess) e = hipStreamWaitEvent(s->cap_stream, s->ev_join, 0);
        }
        const hipError_t e2 = hipStreamEndCapture(s->cap_stream, &gph);
        if (e == hipSuccess) e = e2;
    }
    if (st != CL_OK) {
        if (gph) (void)hipGraphDestroy(gph);
        return st;
    }
    if (e != hipSuccess) return fail(CL_EHIP, "capture of a batched step: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gph);
    if (e != hipSuccess) return fail(CL_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    s->graph = ex;
    std::memcpy(s->graph_key, key, sizeof key);
    return CL_OK;
}

cl_status retire(cl_server* s, size_t idx, int status)
{
    Run& r = *s->active[idx];
    r.status = status;
    cl_status st = cl_measure(r.lat, &r.obs);
    if (st != CL_OK && st != CL_ENONFINITE) return st;
    if (r.desc.keep_links) {
        Kept k;
        k.V = r.V;
        k.links.resize((size_t)r.V * 72);
        if ((st = cl_lattice_get_links(r.lat, k.links.data(), k.links.size())) != CL_OK) return st;
        s->kept[r.id] = std::move(k);
    }
    if ((st = cl_lattice_destroy(r.lat)) != CL_OK) return st;
    r.lat = nullptr;
    s->heap.release(r.off, r.bytes);
    r.t_finish = s->now();
    s->waits.push_back((float)(r.t_admit - r.t_submit));
    auto& grp = s->group[r.desc.lattice.precision];
    grp.erase(std::find(grp.begin(), grp.end(), &r));
    s->done.push_back(std::move(s->active[idx]));
    s->active.erase(s->active.begin() + idx);
    s->dirty = true;
    return CL_OK;
}

}  // namespace

extern "C" {

cl_status cl_server_create(void* arena, size_t arena_bytes, void* hip_stream, cl_server** out)
{
    if (!arena || !out) return fail(CL_EINVAL, "arena and out must not be NULL");
    if ((uintptr_t)arena & 255) return fail(CL_EINVAL, "arena must be 256-byte aligned");
    if (arena_bytes <= tables_bytes()) return fail(CL_ENOMEM, "arena smaller than the server tables");
    auto s = std::make_unique<cl_server>();
    s->arena = (char*)arena;
    s->arena_bytes = arena_bytes;
    s->stream = (hipStream_t)hip_stream;
    s->t0 = std::chrono::steady_clock::now();
    size_t off = 0;
    for (int g = 0; g < 2; ++g) {
        s->d_hdr[g] = (BatchHdr*)(s->arena + off);
        off += align256(sizeof(BatchHdr));
        s->d_runs[g] = (RunArgs*)(s->arena + off);
        off += align256(sizeof(RunArgs) * kMaxRuns);
        s->d_gather[g] = (GatherRec*)(s->arena + off);
        off += align256(sizeof(GatherRec) * kMaxRuns);
        HIP_TRY(hipHostMalloc((void**)&s->h_hdr[g], sizeof(BatchHdr), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&s->h_runs[g], sizeof(RunArgs) * kMaxRuns, hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&s->h_gather[g], sizeof(GatherRec) * kMaxRuns, hipHostMallocDefault));
    }
    s->heap_base = off;
    s->heap.reset(arena_bytes - off);
    HIP_TRY(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&s->cap_stream2, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
    *out = s.release();
    return CL_OK;
}

cl_status cl_server_submit(cl_server* s, const cl_run_desc* run, uint64_t* run_id)
{
    if (!s) return fail(CL_EINVAL, "server is NULL");
    cl_status st = validate_run(run);
    if (st) return st;
    auto r = std::make_unique<Run>();
    r->desc = *run;
    r->bytes = layout_of(run->lattice).total;
    if (align256(r->bytes) > s->heap.size())
        return fail(CL_EBUDGET, "run needs %zu bytes, the arena has %zu", r->bytes, s->heap.size());
    r->id = s->next_id++;
    r->t_submit = s->now();
    r->V = (int64_t)run->lattice.dims[0] * run->lattice.dims[1] * run->lattice.dims[2] * run->lattice.dims[3];
    if (run_id) *run_id = r->id;
    s->pending.push_back(std::move(r));
    return CL_OK;
}

cl_status cl_server_steps(cl_server* s, int max_steps, int* n_active, int* n_pending)
{
    if (!s) return fail(CL_EINVAL, "server is NULL");
    if (max_steps < 1) return fail(CL_EINVAL, "max_steps = %d, must be >= 1", max_steps);
    const double t_begin = s->now();
    cl_status st = admit(s);
    if (st) return st;
    if (!s->active.empty()) {
        if (s->dirty && (st = upload_tables(s)) != CL_OK) return st;
        if ((st = ensure_graph(s)) != CL_OK) return st;
        // as many batch steps as the call allows without taking any run past
        // its last step; one synchronisation for all of them
        int n = max_steps;
        for (const auto& r : s->active) n = std::min(n, r->desc.n_steps - r->steps_done);
        n = std::max(n, 1);
        for (int k = 0; k < n; ++k) HIP_TRY(hipGraphLaunch(s->graph, s->stream));
        for (int g = 0; g < 2; ++g)
            if (!s->group[g].empty())
                HIP_TRY(hipMemcpyAsync(s->h_gather[g], s->d_gather[g], sizeof(GatherRec) * s->group[g].size(),
                                       hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        const double ms_all = 1e3 * (s->now() - t_begin);
        const float ms = (float)(ms_all / n);  // per batch step
        s->busy_s += ms_all * 1e-3;
        s->batch_steps += n;
        // per-run bookkeeping; collect retirements first (retire edits the groups)
        std::vector<std::pair<Run*, int>> finished;
        for (int g = 0; g < 2; ++g)
            for (size_t i = 0; i < s->group[g].size(); ++i) {
                Run* r = s->group[g][i];
                const GatherRec& gr = s->h_gather[g][i];
                // the run's own step counter: a run stops advancing when its
                // status leaves ST_OK (the kernels then leave its links as
                // they are), so it counts the steps actually taken
                const int adv = (int)(gr.step - r->steps_done);
                for (int k = 0; k < adv; ++k) {
                    r->step_ms.push_back(ms);
                    s->all_step_ms.push_back(ms);
                }
                r->steps_done += adv;
                s->link_updates += 4 * r->V * adv;
                if (gr.status != ST_OK) finished.push_back({r, CL_ENONFINITE});
                else if (r->steps_done >= r->desc.n_steps) finished.push_back({r, CL_OK});
            }
        for (auto& f : finished) {
            size_t idx = 0;
            while (s->active[idx].get() != f.first) ++idx;
            if ((st = retire(s, idx, f.second)) != CL_OK) return st;
        }
    }
    if (n_active) *n_active = (int)s->active.size();
    if (n_pending) *n_pending = (int)s->pending.size();
    return CL_OK;
}

cl_status cl_server_step(cl_server* s, int* n_active, int* n_pending)
{
    return cl_server_steps(s, 1, n_active, n_pending);
}

cl_status cl_server_poll(cl_server* s, cl_run_result* out, int cap, int* n_done)
{
    if (!s || !n_done || (cap > 0 && !out)) return fail(CL_EINVAL, "NULL argument");
    int n = 0;
    while (n < cap && !s->done.empty()) {
        const Run& r = *s->done.front();
        cl_run_result& o = out[n++];
        std::memset(&o, 0, sizeof o);
        o.run_id = r.id;
        o.tag = r.desc.tag;
        o.status = r.status;
        o.steps_done = r.steps_done;
        o.obs = r.obs;
        o.t_submit = r.t_submit;
        o.t_admit = r.t_admit;
        o.t_finish = r.t_finish;
        o.step_ms_p50 = percentile(r.step_ms, 0.5);
        o.step_ms_p99 = percentile(r.step_ms, 0.99);
        o.link_updates = 4 * r.V * r.steps_done;
        s->done.pop_front();
    }
    *n_done = n;
    return CL_OK;
}

cl_status cl_server_stats_get(cl_server* s, cl_server_stats* o)
{
    if (!s || !o) return fail(CL_EINVAL, "NULL argument");
    std::memset(o, 0, sizeof *o);
    o->pending = (int)s->pending.size();
    o->active = (int)s->active.size();
    o->finished = (int)s->waits.size();
    o->bytes_in_use = s->heap.used();
    o->bytes_budget = s->heap.size();
    o->batch_steps = s->batch_steps;
    o->link_updates = s->link_updates;
    o->busy_s = s->busy_s;
    o->step_ms_p50 = percentile(s->all_step_ms, 0.5);
    o->step_ms_p99 = percentile(s->all_step_ms, 0.99);
    o->wait_s_p50 = percentile(s->waits, 0.5);
    o->wait_s_p99 = percentile(s->waits, 0.99);
    return CL_OK;
}

cl_status cl_server_take_links(cl_server* s, uint64_t run_id, double* host, size_t n_doubles)
{
    if (!s || !host) return fail(CL_EINVAL, "NULL argument");
    auto it = s->kept.find(run_id);
    if (it == s->kept.end())
        return fail(CL_EINVAL, "run %llu has no kept links (not finished, not kept, or already taken)",
                    (unsigned long long)run_id);
    if (n_doubles != it->second.links.size())
        return fail(CL_EINVAL, "expected %zu doubles, got %zu", it->second.links.size(), n_doubles);
    std::memcpy(host, it->second.links.data(), n_doubles * sizeof(double));
    s->kept.erase(it);
    return CL_OK;
}

cl_status cl_server_destroy(cl_server* s)
{
    if (!s) return fail(CL_EINVAL, "server is NULL");
    hipError_t e = hipStreamSynchronize(s->stream);
    for (auto& r : s->active)
        if (r->lat) (void)cl_lattice_destroy(r->lat);
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    if (s->cap_stream2) (void)hipStreamDestroy(s->cap_stream2);
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    for (int g = 0; g < 2; ++g) {
        if (s->h_hdr[g]) (void)hipHostFree(s->h_hdr[g]);
        if (s->h_runs[g]) (void)hipHostFree(s->h_runs[g]);
        if (s->h_gather[g]) (void)hipHostFree(s->h_gather[g]);
    }
    delete s;
    if (e != hipSuccess) return fail(CL_EHIP, "cl_server_destroy: %s", hipGetErrorString(e));
    return CL_OK;
}

}  // extern "C"
