// Independent magnetospheres stepped together, and the sort-interval
// autotuner.  Both are built on the single-context entry points.
//
// Batch: every system is an ordinary context (a "view") whose kernels run on
// one of a few library-owned streams.  Systems are assigned to the streams by
// longest-processing-time-first bin packing on an estimated cost (particle
// slots plus grid nodes), so small grids, whose kernels cannot fill the chip
// alone, run concurrently with others.  A batch step forks from the caller's
// stream with an event, issues one step of every system per time step
// (systems interleaved across the streams), and joins back with one event per
// stream, so the caller's stream sees the whole batch step as one ordered
// operation.
//
// Autotune: the sort costs a pass over all particle state, while sorted
// particles make the push's gather and deposit local; the best interval
// depends on the workload, as do the push's chunk (particles per thread) and
// the field step's slab height.  The tuner checkpoints the context to host
// memory, times whole sort cycles of each candidate from that same state
// (after one untimed cycle, whose first sort is a full one), one parameter
// after the other, restores the checkpoint and keeps the
// fastest values.  None of them changes the arithmetic, so the choice
// changes results by the order of floating-point atomic additions in the
// deposit and nothing else.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "ffpic_internal.h"

// one batch sort cycle as a graph, with the host state of every system it
// starts from and leaves; a grouped graph also owns the job tables its
// launches read
struct BatchGraph {
    int steps = 0;
    int mode = 1;
    int gppt = 0;                     // grouped push chunk it was captured with
    std::vector<ffpic::CycleState> pre, post;
    hipGraphExec_t exec = nullptr;
    void *tables = nullptr;
};

struct ffpic_batch {
    hipStream_t caller = nullptr;
    std::vector<ffpic_ctx *> ctx;
    std::vector<hipStream_t> streams;
    std::vector<int> lane;            // stream of each system
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;     // one per stream
    // graph-captured batch cycles: captured from origin, which forks to the
    // lane streams and joins them back (mode 1), or grouped launches of all
    // systems on origin (mode 2, where every system allows it); mode 0: no
    // graphs
    int graph_mode = 2;
    int grouped_ppt = 0;              // grouped pushes: particles per thread, 0 = each system's
    int *gctr = nullptr;              // work counters of the grouped launches
    int push_slots[12] = {}, field_slots[8] = {}, psi_slots = 0;
    int64_t grouped_launches = 0;
    double mode_ms[3] = {0, 0, 0};    // batch-step time of each graph mode at the last tuning
    hipStream_t origin = nullptr;
    hipEvent_t gfork = nullptr, gjoin = nullptr;
    std::vector<BatchGraph> graphs;
    int64_t graph_builds = 0, graph_launches = 0;
    std::string last_error;
};

namespace {

constexpr int kMaxStreams = 4;        // hardware queues a process gets by default

struct BFail {
    int code;
    std::string msg;
};

#define BCHK(x)                                                                           \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) throw BFail{FFPIC_EHIP, std::string(#x ": ") + hipGetErrorString(e_)}; \
    } while (0)

template <class F>
int bguard(ffpic_batch *b, F &&f) {
    try {
        f();
        return FFPIC_OK;
    } catch (const BFail &e) {
        if (b) b->last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        if (b) b->last_error = "host allocation failed";
        return FFPIC_ENOMEM;
    } catch (const std::exception &e) {
        if (b) b->last_error = e.what();
        return FFPIC_EHIP;
    }
}

double cost_of(const ffpic_desc &d) {
    double parts = 0;
    for (int s = 0; s < d.nspec && s < FFPIC_MAX_SPECIES; s++) parts += (double)d.capacity[s];
    // one node of the field step costs about as much as four particle pushes
    return parts + 4.0 * (double)(d.nr + 1) * (double)(d.nth + 1);
}

void destroy_batch_graphs(ffpic_batch *b) {
    if (!b->graphs.empty() && b->origin) (void)hipStreamSynchronize(b->origin);
    for (auto &g : b->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.tables) (void)hipFree(g.tables);
    }
    b->graphs.clear();
}

void release(ffpic_batch *b) {
    destroy_batch_graphs(b);
    if (b->origin) (void)hipStreamDestroy(b->origin);
    if (b->gfork) (void)hipEventDestroy(b->gfork);
    if (b->gjoin) (void)hipEventDestroy(b->gjoin);
    b->origin = nullptr;
    b->gfork = b->gjoin = nullptr;
    if (b->gctr) (void)hipFree(b->gctr);
    b->gctr = nullptr;
    for (size_t k = 0; k < b->ctx.size(); k++) {
        if (!b->ctx[k]) continue;
        b->ctx[k]->batch_owned = false;
        ffpic_destroy(b->ctx[k]);
    }
    b->ctx.clear();
    for (auto s : b->streams) (void)hipStreamDestroy(s);
    b->streams.clear();
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (auto e : b->join) (void)hipEventDestroy(e);
    b->join.clear();
}

// A batch cycle (the least common multiple of the systems' sort intervals,
// up to 64 steps) can be a graph when every system's next cycle can (see
// graphable_cycle) and every system stands at the start of one of its own
// cycles.
int batch_cycle(const ffpic_batch *b) {
    if (b->graph_mode == 0) return 0;
    int64_t k = 1;
    for (ffpic_ctx *c : b->ctx) {
        const int si = c->d.sort_interval;
        if (si < 1 || c->step % si != 0 || !ffpic::graphable_cycle(c)) return 0;
        k = k / std::gcd<int64_t>(k, si) * si;
        if (k > 64) return 0;
    }
    return (int)k;
}

bool same_states(const std::vector<ffpic::CycleState> &a, const std::vector<ffpic::CycleState> &b) {
    if (a.size() != b.size()) return false;
    for (size_t k = 0; k < a.size(); k++)
        if (std::memcmp(&a[k], &b[k], sizeof(ffpic::CycleState)) != 0) return false;
    return true;
}

void launch_batch_graph(ffpic_batch *b, hipGraphExec_t exec) {
    BCHK(hipEventRecord(b->gfork, b->caller));
    BCHK(hipStreamWaitEvent(b->origin, b->gfork, 0));
    BCHK(hipGraphLaunch(exec, b->origin));
    BCHK(hipEventRecord(b->gjoin, b->origin));
    BCHK(hipStreamWaitEvent(b->caller, b->gjoin, 0));
    b->graph_launches++;
}

// Grouped cycles: every system FP32-mixed, with no plasma sources (their
// kernels are per system and read per-step arguments).
bool grouped_possible(const ffpic_batch *b) {
    for (const ffpic_ctx *c : b->ctx) {
        if (c->fp64 || c->d.nspec < 1) return false;
        if (c->d.inject_kappa > 0.0 || c->d.gj_extract > 0.0 || c->d.gamma_th > 0.0) return false;
    }
    return true;
}

bool grouped_ok(const ffpic_batch *b) { return b->graph_mode == 2 && grouped_possible(b); }

// Host copies of the job tables of a grouped cycle, laid out as they go to
// device memory (each array at a 256-byte boundary), and the device
// addresses the captured launches read them from.
struct Tables {
    std::vector<char> host;
    char *dev = nullptr;
    size_t cap = 0;
    size_t put(const void *p, size_t n) {
        const size_t off = (host.size() + 255) & ~(size_t)255;
        if (off + n > cap) throw BFail{FFPIC_EHIP, "grouped job tables exceed their bound"};
        host.resize(off + n);
        std::memcpy(host.data() + off, p, n);
        return off;
    }
};

// one launch's jobs: their bytes back to back and the first item of each
struct Group {
    std::vector<char> jobs;
    std::vector<int> starts{0};
    int njobs() const { return (int)starts.size() - 1; }
    int items() const { return starts.back(); }
    // the table pair in device memory
    std::pair<const void *, const int *> place(Tables &T) const {
        const size_t oj = T.put(jobs.data(), jobs.size());
        const size_t os = T.put(starts.data(), starts.size() * sizeof(int));
        return {T.dev + oj, (const int *)(T.dev + os)};
    }
};

size_t table_bound(const ffpic_batch *b, int steps) {
    size_t n = b->ctx.size(), sp = 0;
    for (const ffpic_ctx *c : b->ctx) sp += (size_t)c->d.nspec;
    // per step: two tables (jobs, first items) for each of the flux, mask,
    // up to 12 push and up to 8 field launches, each array starting at a
    // 256-byte boundary
    const size_t pad = 256;
    const size_t psi = n * ffpic::psi_job_bytes() + (n + 1) * 4 + 2 * pad;
    const size_t mask = n * ffpic::mask_job_bytes() + (n + 1) * 4 + 2 * pad;
    const size_t push = sp * ffpic::push_job_bytes() + (sp + 12) * 4 + 24 * pad;
    const size_t field = n * ffpic::field_job_bytes() + (n + 8) * 4 + 16 * pad;
    return (size_t)steps * (psi + mask + push + field) + pad;
}

void grouped_setup(ffpic_batch *b) {
    if (b->gctr) return;
    BCHK(hipMalloc((void **)&b->gctr, 2 * sizeof(int)));
    BCHK(hipMemset(b->gctr, 0, 2 * sizeof(int)));
    BCHK(hipDeviceSynchronize());
    for (int k = 0; k < 12; k++) b->push_slots[k] = ffpic::push_group_slots(k);
    for (int k = 0; k < 8; k++) b->field_slots[k] = ffpic::field_group_slots(k);
    b->psi_slots = ffpic::psi_group_slots();
}

// One batch step as grouped launches on stream st (being captured): the
// flux functions and masks of all systems, then each system's sort if it
// sorts this step (its own launches, on its own stream's branch, forked from
// st and joined back), then the pushes of all systems grouped by kernel
// instance, then their field steps likewise.  The host bookkeeping of every
// system follows what ffpic_step does for that step.
void grouped_step(ffpic_batch *b, hipStream_t st, Tables &T) {
    int *ctr = b->gctr;
    const std::vector<ffpic_ctx *> &sys = b->ctx;
    const int n = (int)sys.size();
    std::vector<char> tmp(std::max({ffpic::psi_job_bytes(), ffpic::mask_job_bytes(),
                                    ffpic::push_job_bytes(), ffpic::field_job_bytes()}));
    Group psi, mask;
    for (ffpic_ctx *c : sys) {
        int m = ffpic::psi_job32(c, tmp.data());
        psi.jobs.insert(psi.jobs.end(), tmp.begin(), tmp.begin() + ffpic::psi_job_bytes());
        psi.starts.push_back(psi.items() + m);
        m = ffpic::mask_job32(c, tmp.data());
        mask.jobs.insert(mask.jobs.end(), tmp.begin(), tmp.begin() + ffpic::mask_job_bytes());
        mask.starts.push_back(mask.items() + m);
    }
    {
        auto t = psi.place(T);
        ffpic::psi_group_launch(st, t.first, t.second, n, std::min(psi.items(), b->psi_slots),
                                ctr);
        t = mask.place(T);
        ffpic::mask_group_launch(st, t.first, t.second, n, std::min(mask.items(), 4096));
    }
    // each sorting system's own launches on its own stream's branch, so
    // that the sorts of different systems may overlap
    bool sorts = false;
    for (ffpic_ctx *c : sys) sorts = sorts || ffpic::step_sorts(c);
    if (sorts) {
        BCHK(hipEventRecord(b->fork, st));
        for (auto l : b->streams) BCHK(hipStreamWaitEvent(l, b->fork, 0));
        for (ffpic_ctx *c : sys) {
            if (!ffpic::step_sorts(c)) continue;
            // the push of this step places the sorted order
            for (int s = 0; s < c->d.nspec; s++) ffpic::sort_species(c, s, true);
        }
        for (size_t l = 0; l < b->streams.size(); l++) {
            BCHK(hipEventRecord(b->join[l], b->streams[l]));
            BCHK(hipStreamWaitEvent(st, b->join[l], 0));
        }
    }
    Group push[12];
    for (ffpic_ctx *c : sys) {
        for (int s = 0; s < c->d.nspec; s++) {
            if (c->sp[s].nub == 0) continue;
            Group &g = push[ffpic::push_group_key(c, s, b->grouped_ppt)];
            const int m = ffpic::push_job(c, s, tmp.data(), b->grouped_ppt);
            g.jobs.insert(g.jobs.end(), tmp.begin(), tmp.begin() + ffpic::push_job_bytes());
            g.starts.push_back(g.items() + m);
        }
    }
    for (int k = 0; k < 12; k++) {
        if (push[k].njobs() == 0 || push[k].items() == 0) continue;
        auto t = push[k].place(T);
        ffpic::push_group_launch(st, k, t.first, t.second, push[k].njobs(),
                                 std::min(push[k].items(), b->push_slots[k]), ctr);
    }
    Group field[8];
    for (ffpic_ctx *c : sys) {
        int key = 0;
        const int m = ffpic::field_job(c, tmp.data(), &key);
        Group &g = field[key];
        g.jobs.insert(g.jobs.end(), tmp.begin(), tmp.begin() + ffpic::field_job_bytes());
        g.starts.push_back(g.items() + m);
    }
    for (int k = 0; k < 8; k++) {
        if (field[k].njobs() == 0) continue;
        auto t = field[k].place(T);
        ffpic::field_group_launch(st, k, t.first, t.second, field[k].njobs(),
                                  std::min(field[k].items(), b->field_slots[k]), ctr);
    }
    for (ffpic_ctx *c : sys) c->step++;
}

// k steps of every system as one graph: the systems' launches go to their
// lane streams, each forked from the capture stream and joined back into
// it, so the graph keeps the systems independent of each other; or, where
// every system allows it, grouped launches of all systems on the capture
// stream
void run_batch_cycle(ffpic_batch *b, int k) {
    std::vector<ffpic::CycleState> pre;
    pre.reserve(b->ctx.size());
    for (ffpic_ctx *c : b->ctx) pre.push_back(ffpic::get_cycle_state(c));
    for (auto &g : b->graphs) {
        const bool gr = grouped_ok(b);
        if (g.steps == k && same_states(g.pre, pre) && g.mode == (gr ? 2 : 1) &&
            (!gr || g.gppt == b->grouped_ppt)) {
            launch_batch_graph(b, g.exec);
            if (g.mode == 2) b->grouped_launches++;
            for (size_t q = 0; q < b->ctx.size(); q++) {
                ffpic::put_cycle_state(b->ctx[q], g.post[q]);
                b->ctx[q]->step += k;
            }
            return;
        }
    }
    if (!b->origin) {
        BCHK(hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking));
        BCHK(hipEventCreateWithFlags(&b->gfork, hipEventDisableTiming));
        BCHK(hipEventCreateWithFlags(&b->gjoin, hipEventDisableTiming));
    }
    std::vector<int64_t> step0;
    std::vector<hipStream_t> own;
    for (ffpic_ctx *c : b->ctx) {
        step0.push_back(c->step);
        own.push_back(c->stream);
    }
    const bool grouped = grouped_ok(b);
    Tables T;
    auto restore = [&] {
        for (size_t q = 0; q < b->ctx.size(); q++) {
            ffpic::put_cycle_state(b->ctx[q], pre[q]);
            b->ctx[q]->step = step0[q];
            b->ctx[q]->stream = own[q];
        }
        if (T.dev) (void)hipFree(T.dev);
    };
    if (grouped) {
        grouped_setup(b);
        T.cap = table_bound(b, k);
        BCHK(hipMalloc((void **)&T.dev, T.cap));
        T.host.reserve(T.cap);
    }
    hipGraph_t graph = nullptr;
    BCHK(hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal));
    try {
        if (grouped) {
            for (int i = 0; i < k; i++) grouped_step(b, b->origin, T);
        } else {
            BCHK(hipEventRecord(b->fork, b->origin));
            for (auto s : b->streams) BCHK(hipStreamWaitEvent(s, b->fork, 0));
            for (int i = 0; i < k; i++)
                for (ffpic_ctx *c : b->ctx) ffpic::steps_one_by_one(c, 1);
            for (size_t s = 0; s < b->streams.size(); s++) {
                BCHK(hipEventRecord(b->join[s], b->streams[s]));
                BCHK(hipStreamWaitEvent(b->origin, b->join[s], 0));
            }
        }
    } catch (...) {
        (void)hipStreamEndCapture(b->origin, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        restore();
        throw;
    }
    BCHK(hipStreamEndCapture(b->origin, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        restore();
        throw BFail{FFPIC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
    }
    if (grouped) {
        // the tables the captured launches read, in place before the first
        // replay
        const hipError_t ec = hipMemcpy(T.dev, T.host.data(), T.host.size(), hipMemcpyHostToDevice);
        if (ec != hipSuccess) {
            (void)hipGraphExecDestroy(exec);
            restore();
            throw BFail{FFPIC_EHIP, std::string("job tables: ") + hipGetErrorString(ec)};
        }
    }
    if (b->graphs.size() >= 4) destroy_batch_graphs(b);
    BatchGraph g;
    g.steps = k;
    g.mode = grouped ? 2 : 1;
    g.gppt = b->grouped_ppt;
    g.pre = pre;
    for (ffpic_ctx *c : b->ctx) g.post.push_back(ffpic::get_cycle_state(c));
    g.exec = exec;
    g.tables = T.dev;
    b->graphs.push_back(std::move(g));
    b->graph_builds++;
    launch_batch_graph(b, exec);
    if (grouped) b->grouped_launches++;
}

std::string cache_key(const ffpic_ctx *c) {
    std::ostringstream o;
    o << c->nr << ' ' << c->nth << ' ' << c->d.precision << ' ' << c->d.nspec;
    return o.str();
}

int64_t total_slots(ffpic_ctx *c) {
    int64_t n = 0;
    for (int s = 0; s < c->d.nspec; s++) {
        int64_t k = 0;
        if (ffpic_num_particles(c, s, &k) == FFPIC_OK) n += k;
    }
    return n;
}

// ms per step of `steps` steps from the current state, timed with events on
// the context's stream
double time_steps(ffpic_ctx *c, int steps) {
    hipEvent_t e0, e1;
    BCHK(hipEventCreate(&e0));
    BCHK(hipEventCreate(&e1));
    BCHK(hipEventRecord(e0, c->stream));
    int rc = ffpic_step(c, steps);
    BCHK(hipEventRecord(e1, c->stream));
    BCHK(hipEventSynchronize(e1));
    float ms = 0;
    BCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != FFPIC_OK) throw BFail{rc, std::string("step failed: ") + ffpic_last_error(c)};
    return ms / steps;
}

// the three tuned settings of a context
struct Setting {
    int interval, rows, ppt;
};

Setting setting_of(const ffpic_ctx *c) { return {c->d.sort_interval, c->fused_rows, c->push_ppt}; }

void apply(ffpic_ctx *c, const Setting &v) {
    c->d.sort_interval = v.interval;
    c->fused_rows = v.rows;
    c->push_ppt = v.ppt;
}

void tune_one(ffpic_ctx *c, double budget_ms, ffpic_tuning *out) {
    auto t0 = std::chrono::steady_clock::now();
    auto elapsed_ms = [&] {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    int rc = ffpic_sync(c);
    if (rc != FFPIC_OK) throw BFail{rc, std::string("context in error: ") + ffpic_last_error(c)};
    size_t len = 0;
    rc = ffpic_save(c, nullptr, &len);
    if (rc != FFPIC_OK) throw BFail{rc, ffpic_last_error(c)};
    std::vector<char> ckpt(len);
    rc = ffpic_save(c, ckpt.data(), &len);
    if (rc != FFPIC_OK) throw BFail{rc, ffpic_last_error(c)};
    const Setting keep = setting_of(c);
    const int timing = c->timing;
    c->timing = 0;
    ffpic_tuning t{};
    Setting best = keep;
    // one parameter after the other, the first candidate of each always
    // timed; every candidate times whole sort cycles from the checkpoint
    struct Param {
        int kind;
        std::vector<int> values;
    };
    std::vector<Param> params = {{FFPIC_TUNE_SORT_INTERVAL, {8, 4, 16, 2, 32, 1}},
                                 {FFPIC_TUNE_FIELD_ROWS, {0, 32, 64, 128, 16}}};
    if (!c->fp64) params.push_back({FFPIC_TUNE_PUSH_PPT, {16, 8, 32}});
    try {
        double last_ms = 0;
        for (const Param &pm : params) {
            double best_ms = 0;
            bool first = true;
            for (int v : pm.values) {
                if (t.ncand >= FFPIC_TUNE_MAX) break;
                Setting cand = best;
                if (pm.kind == FFPIC_TUNE_SORT_INTERVAL) cand.interval = v;
                if (pm.kind == FFPIC_TUNE_FIELD_ROWS) cand.rows = v;
                if (pm.kind == FFPIC_TUNE_PUSH_PPT) cand.ppt = v;
                // whole cycles, at least 8 steps
                const int steps = cand.interval * std::max(1, (8 + cand.interval - 1) / cand.interval);
                if (!first && elapsed_ms() + last_ms * (steps + cand.interval) * 1.5 > budget_ms)
                    continue;
                rc = ffpic_restore(c, ckpt.data(), len);
                if (rc != FFPIC_OK) throw BFail{rc, ffpic_last_error(c)};
                apply(c, cand);
                // A restored context sorts in full at its first sort; one
                // untimed cycle first, so that the timed cycles sort
                // incrementally as in a run
                c->step = 0;
                rc = ffpic_step(c, cand.interval);
                if (rc == FFPIC_OK) rc = ffpic_sync(c);
                if (rc != FFPIC_OK) throw BFail{rc, std::string("step failed: ") + ffpic_last_error(c)};
                const double ms = time_steps(c, steps);
                t.cand_kind[t.ncand] = pm.kind;
                t.cand[t.ncand] = v;
                t.ms_per_step[t.ncand] = ms;
                t.ncand++;
                last_ms = ms;
                if (first || ms < best_ms) {
                    best_ms = ms;
                    best = cand;
                }
                first = false;
            }
        }
    } catch (...) {
        (void)ffpic_restore(c, ckpt.data(), len);
        apply(c, keep);
        c->timing = timing;
        throw;
    }
    rc = ffpic_restore(c, ckpt.data(), len);
    c->timing = timing;
    if (rc != FFPIC_OK) {
        apply(c, keep);
        throw BFail{rc, ffpic_last_error(c)};
    }
    apply(c, best);
    t.sort_interval = best.interval;
    t.field_rows = best.rows;
    t.push_ppt = c->fp64 ? 0 : best.ppt;
    t.total_ms = elapsed_ms();
    if (out) *out = t;
    if (const char *path = std::getenv("FFPIC_TUNING_CACHE")) {
        if (*path) {
            std::ofstream f(path, std::ios::app);
            if (f)
                f << cache_key(c) << ' ' << total_slots(c) << ' ' << best.interval << ' '
                  << best.rows << ' ' << best.ppt << '\n';
        }
    }
}

// ms per batch step of whole batch cycles in graph mode `mode` (grouped
// pushes with `gppt` particles per thread), from the state every system
// was checkpointed in: the steps to a common cycle start and three cycles
// (a restored system's first sort is a full one, launched step by step;
// then the graphs of both buffer parities are captured), then one timed
// cycle
double time_batch_mode(ffpic_batch *b, int mode, int gppt,
                       const std::vector<std::vector<char>> &ckpt, int cycle) {
    for (size_t q = 0; q < b->ctx.size(); q++) {
        const int rc = ffpic_restore(b->ctx[q], ckpt[q].data(), ckpt[q].size());
        if (rc != FFPIC_OK) throw BFail{rc, ffpic_last_error(b->ctx[q])};
    }
    if (mode != b->graph_mode || gppt != b->grouped_ppt) destroy_batch_graphs(b);
    b->graph_mode = mode;
    b->grouped_ppt = gppt;
    int64_t lead = 0;   // steps to the next common cycle start
    for (ffpic_ctx *c : b->ctx) lead = std::max<int64_t>(lead, (cycle - c->step % cycle) % cycle);
    int rc = ffpic_batch_step(b, (int32_t)(lead + 3 * cycle));
    if (rc == FFPIC_OK) rc = ffpic_batch_sync(b);
    if (rc != FFPIC_OK) throw BFail{rc, b->last_error};
    hipEvent_t e0, e1;
    BCHK(hipEventCreate(&e0));
    BCHK(hipEventCreate(&e1));
    BCHK(hipEventRecord(e0, b->caller));
    rc = ffpic_batch_step(b, cycle);
    BCHK(hipEventRecord(e1, b->caller));
    BCHK(hipEventSynchronize(e1));
    float ms = 0;
    BCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != FFPIC_OK) throw BFail{rc, b->last_error};
    return ms / cycle;
}

// After each system's settings are tuned: for a batch that can run as
// grouped launches, time whole batch cycles with per-system graphs, with
// grouped launches using each system's push chunk, and with grouped
// launches using 16 particles per thread for every system (the per-system
// chunk is chosen for one system filling the GPU alone; grouped, all
// systems fill it together), from the same checkpoint of every system;
// restore the checkpoint and keep the fastest.  Which one wins depends on
// the batch: per-system graphs let one system's push overlap another's
// field step; grouped launches need far fewer launches per step.
void tune_batch_mode(ffpic_batch *b) {
    b->mode_ms[0] = b->mode_ms[1] = b->mode_ms[2] = 0;
    if (b->graph_mode == 0 || !grouped_possible(b)) return;
    int64_t cycle = 1;
    for (ffpic_ctx *c : b->ctx) {
        // graph capture possible once the system has sorted (a restored
        // system sorts in full first)
        const int si = c->d.sort_interval;
        if (si < 1 || !c->use_graph || c->timing || c->d.rr_ramp_n > 0) return;
        cycle = cycle / std::gcd<int64_t>(cycle, si) * si;
        if (cycle > 64) return;
    }
    const int keep = b->graph_mode, keep_ppt = b->grouped_ppt;
    std::vector<std::vector<char>> ckpt(b->ctx.size());
    for (size_t q = 0; q < b->ctx.size(); q++) {
        size_t len = 0;
        int rc = ffpic_save(b->ctx[q], nullptr, &len);
        if (rc == FFPIC_OK) {
            ckpt[q].resize(len);
            rc = ffpic_save(b->ctx[q], ckpt[q].data(), &len);
        }
        if (rc != FFPIC_OK) throw BFail{rc, ffpic_last_error(b->ctx[q])};
    }
    // (mode, grouped chunk); each timed twice, alternating, the faster of
    // its two timings kept: a single cycle's time varies by a few per cent
    const int cand[3][2] = {{1, 0}, {2, 0}, {2, 16}};
    double ms[3] = {0, 0, 0};
    int best = 0;
    try {
        for (int rep = 0; rep < 2; rep++)
            for (int k = 0; k < 3; k++) {
                const double t = time_batch_mode(b, cand[k][0], cand[k][1], ckpt, (int)cycle);
                ms[k] = rep == 0 ? t : std::min(ms[k], t);
            }
        for (int k = 1; k < 3; k++)
            if (ms[k] < ms[best]) best = k;
    } catch (...) {
        for (size_t q = 0; q < b->ctx.size(); q++)
            (void)ffpic_restore(b->ctx[q], ckpt[q].data(), ckpt[q].size());
        destroy_batch_graphs(b);
        b->graph_mode = keep;
        b->grouped_ppt = keep_ppt;
        throw;
    }
    for (size_t q = 0; q < b->ctx.size(); q++) {
        const int rc = ffpic_restore(b->ctx[q], ckpt[q].data(), ckpt[q].size());
        if (rc != FFPIC_OK) throw BFail{rc, ffpic_last_error(b->ctx[q])};
    }
    destroy_batch_graphs(b);
    b->mode_ms[1] = ms[0];
    b->mode_ms[2] = std::min(ms[1], ms[2]);
    b->graph_mode = cand[best][0];
    b->grouped_ppt = best == 0 ? keep_ppt : cand[best][1];
}

}  // namespace

namespace ffpic {

// settings for a descriptor that asks for the tuned ones (sort interval 0):
// the last cache entry with the same grid, precision and species count,
// else interval 8, automatic slab rows and 16 particles per thread
void tuned_settings(const ffpic_desc *d, int *interval, int *rows, int *ppt) {
    *interval = 8;
    *rows = 0;
    *ppt = 16;
    const char *path = std::getenv("FFPIC_TUNING_CACHE");
    if (!path || !*path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        long nr, nth, prec, nspec, nslots, si, rw = 0, pp = 16;
        if (!(in >> nr >> nth >> prec >> nspec >> nslots >> si)) continue;
        if (!(in >> rw >> pp)) { rw = 0; pp = 16; }
        if (nr == d->nr && nth == d->nth && prec == d->precision && nspec == d->nspec && si >= 1 &&
            si <= 1024 && rw >= 0 && rw <= 4096 && (pp == 8 || pp == 16 || pp == 32)) {
            *interval = (int)si;
            *rows = (int)rw;
            *ppt = (int)pp;
        }
    }
}

}  // namespace ffpic

extern "C" {

int ffpic_batch_create(int n, const ffpic_desc *d, void *stream, ffpic_batch **out) {
    if (!out) return FFPIC_EINVAL;
    *out = nullptr;
    if (n < 1 || !d) return FFPIC_EINVAL;
    ffpic_batch *b = new (std::nothrow) ffpic_batch();
    if (!b) return FFPIC_ENOMEM;
    int rc = bguard(b, [&] {
        b->caller = (hipStream_t)stream;
        int ns = std::min(n, kMaxStreams);
        for (int s = 0; s < ns; s++) {
            hipStream_t h;
            BCHK(hipStreamCreateWithFlags(&h, hipStreamNonBlocking));
            b->streams.push_back(h);
            hipEvent_t e;
            BCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            b->join.push_back(e);
        }
        BCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        // longest processing time first onto the least loaded stream
        std::vector<int> order(n);
        for (int k = 0; k < n; k++) order[k] = k;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return cost_of(d[x]) > cost_of(d[y]); });
        std::vector<double> load(ns, 0.0);
        b->lane.assign(n, 0);
        for (int k : order) {
            int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            b->lane[k] = s;
            load[s] += cost_of(d[k]);
        }
        b->ctx.assign(n, nullptr);
        for (int k = 0; k < n; k++) {
            ffpic_ctx *c = nullptr;
            int r = ffpic_create(&d[k], b->streams[b->lane[k]], &c);
            if (r != FFPIC_OK)
                throw BFail{r, "system " + std::to_string(k) + ": descriptor rejected or allocation failed"};
            c->batch_owned = true;
            b->ctx[k] = c;
        }
    });
    if (rc != FFPIC_OK) {
        release(b);
        delete b;
        return rc;
    }
    *out = b;
    return FFPIC_OK;
}

int ffpic_batch_view(ffpic_batch *b, int k, ffpic_ctx **view) {
    if (!b || !view) return FFPIC_EINVAL;
    if (k < 0 || k >= (int)b->ctx.size()) {
        b->last_error = "system index out of range";
        return FFPIC_EINVAL;
    }
    *view = b->ctx[k];
    return FFPIC_OK;
}

int ffpic_batch_size(const ffpic_batch *b) { return b ? (int)b->ctx.size() : 0; }

int ffpic_batch_step(ffpic_batch *b, int32_t nsteps) {
    return bguard(b, [&] {
        if (!b) throw BFail{FFPIC_EINVAL, "batch is NULL"};
        if (nsteps < 0) throw BFail{FFPIC_EINVAL, "negative step count"};
        if (nsteps == 0) return;
        BCHK(hipEventRecord(b->fork, b->caller));
        for (auto s : b->streams) BCHK(hipStreamWaitEvent(s, b->fork, 0));
        int failed = FFPIC_OK;
        std::string why;
        for (int k = 0; k < nsteps && failed == FFPIC_OK;) {
            // whole batch cycles as graphs
            const int kc = batch_cycle(b);
            if (kc > 0 && nsteps - k >= kc) {
                // the graph runs from the capture stream, ordered after the
                // lane streams' earlier work by the caller's stream: join
                // the lanes into the caller first
                for (size_t s = 0; s < b->streams.size(); s++) {
                    BCHK(hipEventRecord(b->join[s], b->streams[s]));
                    BCHK(hipStreamWaitEvent(b->caller, b->join[s], 0));
                }
                try {
                    run_batch_cycle(b, kc);
                } catch (const BFail &e) {
                    failed = e.code;
                    why = e.msg;
                    break;
                } catch (const std::exception &e) {
                    failed = FFPIC_EHIP;
                    why = e.what();
                    break;
                }
                // and the lanes' later work after the graph
                BCHK(hipEventRecord(b->fork, b->caller));
                for (auto s : b->streams) BCHK(hipStreamWaitEvent(s, b->fork, 0));
                k += kc;
                continue;
            }
            for (size_t q = 0; q < b->ctx.size(); q++) {
                int r = ffpic_step(b->ctx[q], 1);
                if (r != FFPIC_OK) {
                    failed = r;
                    why = "system " + std::to_string(q) + ": " + ffpic_last_error(b->ctx[q]);
                    break;
                }
            }
            k++;
        }
        // join even after a failure, so the caller's stream stays ordered
        for (size_t s = 0; s < b->streams.size(); s++) {
            BCHK(hipEventRecord(b->join[s], b->streams[s]));
            BCHK(hipStreamWaitEvent(b->caller, b->join[s], 0));
        }
        if (failed != FFPIC_OK) throw BFail{failed, why};
    });
}

int ffpic_batch_sync(ffpic_batch *b) {
    return bguard(b, [&] {
        if (!b) throw BFail{FFPIC_EINVAL, "batch is NULL"};
        for (size_t q = 0; q < b->ctx.size(); q++) {
            int r = ffpic_sync(b->ctx[q]);
            if (r != FFPIC_OK)
                throw BFail{r, "system " + std::to_string(q) + ": " + ffpic_last_error(b->ctx[q])};
        }
    });
}

int ffpic_batch_set_graph(ffpic_batch *b, int mode) {
    return bguard(b, [&] {
        if (!b) throw BFail{FFPIC_EINVAL, "batch is NULL"};
        if (mode < 0 || mode > 2) throw BFail{FFPIC_EINVAL, "graph mode must be 0, 1 or 2"};
        if (mode != b->graph_mode) destroy_batch_graphs(b);
        b->graph_mode = mode;
    });
}

int ffpic_batch_graph_stats(ffpic_batch *b, int64_t *builds, int64_t *launches) {
    if (!b) return FFPIC_EINVAL;
    if (builds) *builds = b->graph_builds;
    if (launches) *launches = b->graph_launches;
    return FFPIC_OK;
}

int ffpic_batch_set_grouped_chunk(ffpic_batch *b, int32_t ppt) {
    return bguard(b, [&] {
        if (!b) throw BFail{FFPIC_EINVAL, "batch is NULL"};
        if (ppt != 0 && ppt != 8 && ppt != 16 && ppt != 32)
            throw BFail{FFPIC_EINVAL, "grouped push chunk must be 0, 8, 16 or 32"};
        if (ppt != b->grouped_ppt) destroy_batch_graphs(b);
        b->grouped_ppt = ppt;
    });
}

int ffpic_batch_get_graph(const ffpic_batch *b, int32_t *mode, int32_t *grouped_ppt,
                          double ms_per_step[3]) {
    if (!b || !mode) return FFPIC_EINVAL;
    *mode = b->graph_mode;
    if (grouped_ppt) *grouped_ppt = b->grouped_ppt;
    if (ms_per_step)
        for (int k = 0; k < 3; k++) ms_per_step[k] = b->mode_ms[k];
    return FFPIC_OK;
}

int ffpic_batch_grouped_launches(const ffpic_batch *b, int64_t *launches) {
    if (!b || !launches) return FFPIC_EINVAL;
    *launches = b->grouped_launches;
    return FFPIC_OK;
}

const char *ffpic_batch_last_error(const ffpic_batch *b) {
    return b ? b->last_error.c_str() : "no batch";
}

int ffpic_batch_destroy(ffpic_batch *b) {
    if (!b) return FFPIC_EINVAL;
    for (auto s : b->streams) (void)hipStreamSynchronize(s);
    release(b);
    delete b;
    return FFPIC_OK;
}

int ffpic_autotune(ffpic_ctx *ctx, double budget_ms, ffpic_tuning *out) {
    if (!ctx) return FFPIC_EINVAL;
    if (!(budget_ms > 0)) {
        ctx->last_error = "budget must be positive";
        return FFPIC_EINVAL;
    }
    try {
        tune_one(ctx, budget_ms, out);
        return FFPIC_OK;
    } catch (const BFail &e) {
        ctx->last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        ctx->last_error = "host allocation failed";
        return FFPIC_ENOMEM;
    } catch (const std::exception &e) {
        ctx->last_error = e.what();
        return FFPIC_EHIP;
    }
}

int ffpic_batch_autotune(ffpic_batch *b, double budget_ms, ffpic_tuning *out) {
    return bguard(b, [&] {
        if (!b) throw BFail{FFPIC_EINVAL, "batch is NULL"};
        if (!(budget_ms > 0)) throw BFail{FFPIC_EINVAL, "budget must be positive"};
        double each = budget_ms / (double)b->ctx.size();
        for (size_t q = 0; q < b->ctx.size(); q++) {
            int r = ffpic_autotune(b->ctx[q], each, out ? out + q : nullptr);
            if (r != FFPIC_OK)
                throw BFail{r, "system " + std::to_string(q) + ": " + ffpic_last_error(b->ctx[q])};
        }
        tune_batch_mode(b);
    });
}

}  // extern "C"
