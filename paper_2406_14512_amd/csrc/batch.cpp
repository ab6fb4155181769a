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
// memory, times whole sort cycles of each candidate from that same state,
// one parameter after the other, restores the checkpoint and keeps the
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
// starts from and leaves
struct BatchGraph {
    int steps = 0;
    std::vector<ffpic::CycleState> pre, post;
    hipGraphExec_t exec = nullptr;
};

struct ffpic_batch {
    hipStream_t caller = nullptr;
    std::vector<ffpic_ctx *> ctx;
    std::vector<hipStream_t> streams;
    std::vector<int> lane;            // stream of each system
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;     // one per stream
    // graph-captured batch cycles: captured from origin, which forks to the
    // lane streams and joins them back
    bool use_graph = true;
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
    for (auto &g : b->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
}

void release(ffpic_batch *b) {
    destroy_batch_graphs(b);
    if (b->origin) (void)hipStreamDestroy(b->origin);
    if (b->gfork) (void)hipEventDestroy(b->gfork);
    if (b->gjoin) (void)hipEventDestroy(b->gjoin);
    b->origin = nullptr;
    b->gfork = b->gjoin = nullptr;
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
    if (!b->use_graph) return 0;
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

// k steps of every system as one graph: the systems' launches go to their
// lane streams, each forked from the capture stream and joined back into
// it, so the graph keeps the systems independent of each other
void run_batch_cycle(ffpic_batch *b, int k) {
    std::vector<ffpic::CycleState> pre;
    pre.reserve(b->ctx.size());
    for (ffpic_ctx *c : b->ctx) pre.push_back(ffpic::get_cycle_state(c));
    for (auto &g : b->graphs) {
        if (g.steps == k && same_states(g.pre, pre)) {
            launch_batch_graph(b, g.exec);
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
    for (ffpic_ctx *c : b->ctx) step0.push_back(c->step);
    auto restore = [&] {
        for (size_t q = 0; q < b->ctx.size(); q++) {
            ffpic::put_cycle_state(b->ctx[q], pre[q]);
            b->ctx[q]->step = step0[q];
        }
    };
    hipGraph_t graph = nullptr;
    BCHK(hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal));
    try {
        BCHK(hipEventRecord(b->fork, b->origin));
        for (auto s : b->streams) BCHK(hipStreamWaitEvent(s, b->fork, 0));
        for (int i = 0; i < k; i++)
            for (ffpic_ctx *c : b->ctx) ffpic::steps_one_by_one(c, 1);
        for (size_t s = 0; s < b->streams.size(); s++) {
            BCHK(hipEventRecord(b->join[s], b->streams[s]));
            BCHK(hipStreamWaitEvent(b->origin, b->join[s], 0));
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
    if (b->graphs.size() >= 4) destroy_batch_graphs(b);
    BatchGraph g;
    g.steps = k;
    g.pre = pre;
    for (ffpic_ctx *c : b->ctx) g.post.push_back(ffpic::get_cycle_state(c));
    g.exec = exec;
    b->graphs.push_back(std::move(g));
    b->graph_builds++;
    launch_batch_graph(b, exec);
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
                if (!first && elapsed_ms() + last_ms * steps * 1.5 > budget_ms) continue;
                rc = ffpic_restore(c, ckpt.data(), len);
                if (rc != FFPIC_OK) throw BFail{rc, ffpic_last_error(c)};
                apply(c, cand);
                c->step = 0;              // the first timed step sorts
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

int ffpic_batch_set_graph(ffpic_batch *b, int on) {
    return bguard(b, [&] {
        if (!b) throw BFail{FFPIC_EINVAL, "batch is NULL"};
        b->use_graph = on != 0;
        if (!b->use_graph) destroy_batch_graphs(b);
    });
}

int ffpic_batch_graph_stats(ffpic_batch *b, int64_t *builds, int64_t *launches) {
    if (!b) return FFPIC_EINVAL;
    if (builds) *builds = b->graph_builds;
    if (launches) *launches = b->graph_launches;
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
    });
}

}  // extern "C"
