// Batching, serving and the contact-angle query of the C ABI (include/semlbm.h).
//
// A batch groups its bound members by (dimension, N, kernel path); every kernel of the time
// step runs once per group and covers all of the group's members (block tables map each block to a
// member and to a block of that member).  The server keeps a queue of requests, admits
// them while slots and arena bytes are free, advances all active solves as one batch in
// rounds of check_every steps, and retires each solve when its kinetic energy has dropped
// below the threshold (Sec. 3: KE_max is the paper's equilibrium measure) or its step
// budget is spent.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_set>
#include <vector>

#include "../../include/semlbm.h"
#include "ctx.hpp"

using namespace slbm;

static_assert(kStaticScratchBytes == SLBM_STATIC_SCRATCH_BYTES, "static scratch size of the header");

// ------------------------------------------------------------------------------------------
// batch
// ------------------------------------------------------------------------------------------
struct slbm_batch {
    void *stream = nullptr;
    std::vector<slbm_ctx *> members;
    bool dirty = true;
    // One launch shape of a group's kernels: elements per block of the element kernels and
    // the order of the block tables.  Every shape gives the same bits (each element's and
    // node's arithmetic does not depend on which block runs it), so the tuner may switch
    // shapes between any two steps.
    struct Shape {
        int epb = 1;       // elements per block (1, or as many as fit in 256 threads)
        bool xcd = true;   // XCD-aware block order (contiguous ranges per die), else plain order
        LaunchPlan ep{}, np{}, sp{};  // element, every node, nodes past the interior range
        double us = 0.0;   // measured device time of one step of the group (0: not measured)
    };
    struct Group {
        int d = 0, N = 0;
        bool fused = true;     // kernel path of every member
        std::vector<int> idx;  // member indices
        int64_t elements = 0;
        std::vector<Shape> shapes;
        int pick = 0;          // index into shapes
        bool measured = false; // pick chosen by timing (here or earlier, from the tuning cache)
        LaunchPlan ep{}, np{}, sp{}; // shapes[pick]
        SolveDesc *desc = nullptr;  // device
        double *diag_out = nullptr; // device [2 * members]
    };
    std::vector<Group> groups;
    bool tables_ok = false;  // dmem holds the current groups' launch tables
    void *dmem = nullptr;
    size_t dcap = 0;
    slbm_status status = SLBM_OK;
    // graphs of 1 and 10 batched steps for the current membership (captured lazily)
    void *graph[2] = {nullptr, nullptr};
    bool use_graph = true;
    // autotuner: timed shapes per (d, N, path, size class of the group), kept across
    // membership changes
    bool autotune = true;
    static constexpr int kTuneReps = 3;  // timed steps per shape (after one warm-up step)
    struct Tuned { int pick; std::vector<double> us; };
    std::map<std::vector<int64_t>, Tuned> cache;

    static std::vector<int64_t> key_of(const Group &g) {
        int64_t cls = 0;  // size class: floor(log2(elements))
        while ((int64_t)2 << cls <= g.elements) ++cls;
        return {g.d, g.N, g.fused ? 1 : 0, cls};
    }

    void drop_graphs() {
        destroy_graph(graph[0]);
        destroy_graph(graph[1]);
        graph[0] = graph[1] = nullptr;
    }

    int enqueue_group(const Group &g, const LaunchPlan &ep, const LaunchPlan &sp, int64_t n,
                      void *on = nullptr) const {
        return enqueue_steps(g.d, g.N, ep, sp, n, on ? on : stream, g.fused);
    }

    // Concurrent groups: the groups share no data, so each group's chain of steps runs on a
    // stream of its own, forked from and joined back into the batch's stream by events (in a
    // captured graph these are parallel branches).  Small groups then overlap their launch
    // and latency floors, and large ones each other's tails.
    bool concurrent = true;
    std::vector<void *> side;     // hipStream_t per group (default priority)
    std::vector<void *> join_ev;  // hipEvent_t per group
    void *fork_ev = nullptr;      // hipEvent_t

    int ensure_side() {
        if (!fork_ev && hipEventCreateWithFlags((hipEvent_t *)&fork_ev, hipEventDisableTiming) != hipSuccess)
            return (int)hipErrorOutOfMemory;
        while (side.size() < groups.size()) {
            hipStream_t s = nullptr;
            hipEvent_t e = nullptr;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return (int)hipErrorOutOfMemory;
            side.push_back(s);
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return (int)hipErrorOutOfMemory;
            join_ev.push_back(e);
        }
        return 0;
    }

    int enqueue(int64_t n) {
        if (!concurrent || groups.size() < 2) {
            for (int64_t s = 0; s < n; ++s)
                for (auto &g : groups) {
                    const int e = enqueue_group(g, g.ep, g.sp, 1);
                    if (e) return e;
                }
            return 0;
        }
        int e = ensure_side();
        hipStream_t st = (hipStream_t)stream;
        if (!e) e = (int)hipEventRecord((hipEvent_t)fork_ev, st);
        for (size_t gi = 0; gi < groups.size() && !e; ++gi) {
            hipStream_t ss = (hipStream_t)side[gi];
            e = (int)hipStreamWaitEvent(ss, (hipEvent_t)fork_ev, 0);
            if (!e) e = enqueue_group(groups[gi], groups[gi].ep, groups[gi].sp, n, ss);
            if (!e) e = (int)hipEventRecord((hipEvent_t)join_ev[gi], ss);
            if (!e) e = (int)hipStreamWaitEvent(st, (hipEvent_t)join_ev[gi], 0);
        }
        return e;
    }

    int run(int64_t n) {
        if (n <= 0) return 0;
        if (use_graph && stream != nullptr) {
            // each graph is captured when a call first needs it (n % 10 single steps, n / 10
            // runs of ten)
            const int sizes[2] = {1, 10};
            const bool need[2] = {n % 10 != 0, n >= 10};
            for (int k = 0; k < 2 && use_graph; ++k)
                if (need[k] && !graph[k]) {
                    struct A { slbm_batch *b; int steps; } a{this, sizes[k]};
                    auto fn = [](void *, void *p) -> int {
                        A *x = (A *)p;
                        return x->b->enqueue(x->steps);
                    };
                    if (capture_graph(stream, &graph[k], fn, &a)) {
                        (void)hipGetLastError();
                        use_graph = false;
                        drop_graphs();
                    }
                }
            if (use_graph) {
                int e = 0;
                int64_t left = n;
                while (left >= 10 && !e) { e = launch_graph(graph[1], stream); left -= 10; }
                while (left > 0 && !e) { e = launch_graph(graph[0], stream); left -= 1; }
                return e;
            }
        }
        return enqueue(n);
    }

    // Steps the tuner spends on a group: one warm-up and kTuneReps timed steps per shape.
    static int64_t tune_steps(const Group &g) { return (int64_t)g.shapes.size() * (1 + kTuneReps); }

    // Time every shape of group g on its members' own time steps (each step a replay of a
    // one-step graph of the group, or plain launches where the stream cannot be captured)
    // and pick the fastest.  The group advances tune_steps(g) steps; waits for the device.
    int tune(Group &g) {
        hipStream_t st = (hipStream_t)stream;
        hipEvent_t ev[kTuneReps + 1] = {};
        int e = 0;
        for (int r = 0; r <= kTuneReps && !e; ++r) e = (int)hipEventCreate(&ev[r]);
        for (size_t k = 0; k < g.shapes.size() && !e; ++k) {
            struct A { const slbm_batch *b; const Group *g; const Shape *s; } a{this, &g, &g.shapes[k]};
            auto fn = [](void *, void *p) -> int {
                const A *x = (const A *)p;
                return x->b->enqueue_group(*x->g, x->s->ep, x->s->sp, 1);
            };
            void *gr = nullptr;
            if (use_graph && stream != nullptr && capture_graph(stream, &gr, fn, &a)) {
                (void)hipGetLastError();
                gr = nullptr;
            }
            auto once = [&]() { return gr ? launch_graph(gr, stream) : fn(nullptr, &a); };
            e = once();
            for (int r = 0; r <= kTuneReps && !e; ++r) {
                e = (int)hipEventRecord(ev[r], st);
                if (!e && r < kTuneReps) e = once();
            }
            if (!e) e = (int)hipEventSynchronize(ev[kTuneReps]);
            float best = -1.0f;
            for (int r = 0; r < kTuneReps && !e; ++r) {
                float ms = 0.0f;
                e = (int)hipEventElapsedTime(&ms, ev[r], ev[r + 1]);
                if (!e && (best < 0.0f || ms < best)) best = ms;
            }
            destroy_graph(gr);
            g.shapes[k].us = 1e3 * (double)best;
        }
        for (auto &x : ev)
            if (x) (void)hipEventDestroy(x);
        if (e) return e;
        int pick = 0;
        for (size_t k = 1; k < g.shapes.size(); ++k)
            if (g.shapes[k].us < g.shapes[pick].us) pick = (int)k;
        select(g, pick, true);
        Tuned t{pick, {}};
        for (auto &s : g.shapes) t.us.push_back(s.us);
        cache[key_of(g)] = t;
        return 0;
    }

    void select(Group &g, int k, bool measured) {
        if (g.pick != k) ++layout_gen;
        g.pick = k;
        g.measured = measured;
        g.ep = g.shapes[k].ep;
        g.np = g.shapes[k].np;
        g.sp = g.shapes[k].sp;
    }

    // Tune the groups that have more than one shape and no timing yet, when this call's
    // n steps cover the tuner's steps; every group then catches up to the same step count
    // with plain launches.  Returns the steps every member has advanced (or -1).
    int64_t tune_pending(int64_t n) {
        std::vector<int64_t> used(groups.size(), 0);
        int64_t mx = 0;
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            Group &g = groups[gi];
            if (g.measured || g.shapes.size() < 2 || tune_steps(g) > n) continue;
            if (tune(g)) return -1;
            used[gi] = tune_steps(g);
            mx = std::max(mx, used[gi]);
        }
        if (mx == 0) return 0;
        drop_graphs();  // captured with the previous shapes
        for (size_t gi = 0; gi < groups.size(); ++gi)
            if (used[gi] < mx && enqueue_group(groups[gi], groups[gi].ep, groups[gi].sp, mx - used[gi]))
                return -1;
        return mx;
    }

    ~slbm_batch() {
        drop_graphs();
        if (dmem || !side.empty()) (void)hipStreamSynchronize((hipStream_t)stream);
        for (void *x : side) (void)hipStreamDestroy((hipStream_t)x);
        for (void *x : join_ev) (void)hipEventDestroy((hipEvent_t)x);
        if (fork_ev) (void)hipEventDestroy((hipEvent_t)fork_ev);
        if (dmem) (void)hipFree(dmem);
    }

    // element blocks of member c under a block shape
    static int eblocks(const slbm_ctx *c, int epb) { return (int)((c->E + epb - 1) / epb); }

    // block table [2][len] (member, block within member) over n logical blocks in XCD-aware
    // order (hardware block b runs logical block xcd_logical(b, n), so each die works on a
    // contiguous range; padded with -1) or in plain order
    static int table_len(int n, bool xcd) { return xcd ? xcd_grid(n) : n; }
    static void fill_table(int *h, int n, bool xcd, const std::vector<int> &s, const std::vector<int> &l) {
        const int len = table_len(n, xcd);
        for (int b = 0; b < len; ++b) {
            const int j = xcd ? xcd_logical(b, n) : b;
            h[b] = j < n ? s[j] : 0;
            h[len + b] = j < n ? l[j] : -1;
        }
    }

    // Host side of a membership change: groups by (d, N, path), stale-partial bookkeeping,
    // candidate launch shapes and each group's pick (the tuned one for its key, else the
    // fixed rule).  Launch tables are laid out afterwards (make_tables, or the static path).
    slbm_status regroup() {
        drop_graphs();
        groups.clear();
        tables_ok = false;
        ++layout_gen;
        // groups by (d, N, path): members start from the path they step alone with; a
        // fused group whose members together exceed unfused_above(dim) local nodes then
        // steps with the unfused kernels, as a single mesh of that size would
        for (int i = 0; i < (int)members.size(); ++i) {
            slbm_ctx *c = members[i];
            Group *g = nullptr;
            for (auto &x : groups)
                if (x.d == c->dq && x.N == c->N && x.fused == c->fused) g = &x;
            if (!g) {
                groups.emplace_back();
                g = &groups.back();
                g->d = c->dq;
                g->N = c->N;
                g->fused = c->fused;
            }
            g->idx.push_back(i);
            g->elements += c->E;
        }
        for (auto &g : groups) {
            if (!g.fused) continue;
            int64_t nl = 0;
            for (int i : g.idx) nl += members[i]->Nl;
            if (nl > unfused_above(members[g.idx[0]]->dim)) g.fused = false;
        }
        // the unfused kernels leave Laplacian partials of the last stage's input behind: a
        // fused-path member of an unfused group needs them recomputed before it steps fused
        // again (here, or at slbm_step once it leaves the batch); members of fused groups
        // that were stepped unfused get them now, ahead of any step on the batch stream
        for (auto &g : groups)
            for (int i : g.idx) {
                slbm_ctx *c = members[i];
                if (!g.fused && c->fused) c->rl_stale = true;
                if (g.fused && c->refresh_lap() != 0) return SLBM_EDEVICE;
            }
        // candidate shapes per group: one element per block and (where more than one
        // element fits) wide blocks, each in XCD-aware and plain block order
        for (auto &g : groups) {
            const int w = epb_wide(g.d, g.N);
            for (int epb : {1, w}) {
                if (epb == w && w == 1 && !g.shapes.empty()) break;
                for (bool xcd : {true, false}) {
                    Shape s;
                    s.epb = epb;
                    s.xcd = xcd;
                    g.shapes.push_back(s);
                }
            }
        }
        for (auto &g : groups) {
            auto it = cache.find(key_of(g));
            if (it != cache.end() && it->second.us.size() == g.shapes.size()) {
                for (size_t k = 0; k < g.shapes.size(); ++k) g.shapes[k].us = it->second.us[k];
                g.pick = it->second.pick;
                g.measured = true;
            } else {
                const int w = epb_wide(g.d, g.N);
                int nbw = 0;
                for (int i : g.idx) nbw += eblocks(members[i], w);
                const int want = nbw >= 256 ? w : 1;
                g.pick = 0;
                for (size_t k = 0; k < g.shapes.size(); ++k)
                    if (g.shapes[k].epb == want && g.shapes[k].xcd) { g.pick = (int)k; break; }
                g.measured = false;
            }
        }
        dirty = false;
        return SLBM_OK;
    }

    // the groups' launch tables for every candidate shape in library-allocated device memory
    slbm_status rebuild() {
        if (dirty)
            if (slbm_status s = regroup()) return s;
        if (tables_ok) return SLBM_OK;
        // one device block: per group [descs][e tables per shape][n tables per order][diag out]
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        auto counts = [&](const Group &g, int epb, int *ne, int *nn, int *ns) {
            *ne = *nn = *ns = 0;
            for (int i : g.idx) {
                *ne += eblocks(members[i], epb);
                *nn += members[i]->n_nblocks;
                *ns += members[i]->n_sblocks;
            }
        };
        size_t total = 0;
        std::vector<size_t> goff;
        for (auto &g : groups) {
            goff.push_back(total);
            total += al(sizeof(SolveDesc) * g.idx.size()) + al(sizeof(double) * 2 * g.idx.size());
            int ne = 0, nn = 0, ns = 0;
            for (auto &s : g.shapes) {
                counts(g, s.epb, &ne, &nn, &ns);
                total += al(sizeof(int) * 2 * table_len(ne, s.xcd)) + al(sizeof(int) * 2 * table_len(nn, s.xcd)) +
                         al(sizeof(int) * 2 * table_len(ns, s.xcd));
            }
        }
        hipStream_t st = (hipStream_t)stream;
        if (total > dcap) {
            if (dmem) {
                (void)hipStreamSynchronize(st);
                (void)hipFree(dmem);
                dmem = nullptr;
            }
            size_t cap = std::max(total, (size_t)1 << 16);
            if (hipMalloc(&dmem, cap) != hipSuccess) {
                dcap = 0;
                return SLBM_ENOMEM;
            }
            dcap = cap;
        }
        std::vector<char> host(total, 0);
        char *base = (char *)dmem;
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            Group &g = groups[gi];
            size_t o = goff[gi];
            g.desc = reinterpret_cast<SolveDesc *>(base + o);
            SolveDesc *dh = reinterpret_cast<SolveDesc *>(host.data() + o);
            o += al(sizeof(SolveDesc) * g.idx.size());
            g.diag_out = reinterpret_cast<double *>(base + o);
            o += al(sizeof(double) * 2 * g.idx.size());
            for (int k = 0; k < (int)g.idx.size(); ++k) dh[k] = members[g.idx[k]]->desc;
            for (auto &s : g.shapes) {
                std::vector<int> le_s, le_l, ln_s, ln_l, ls_s, ls_l;  // logical order
                for (int k = 0; k < (int)g.idx.size(); ++k) {
                    slbm_ctx *c = members[g.idx[k]];
                    for (int b = 0; b < eblocks(c, s.epb); ++b) { le_s.push_back(k); le_l.push_back(b); }
                    for (int b = 0; b < c->n_nblocks; ++b) { ln_s.push_back(k); ln_l.push_back(b); }
                    for (int b = 0; b < c->n_sblocks; ++b) { ls_s.push_back(k); ls_l.push_back(b); }
                }
                const int ne = (int)le_s.size(), nn = (int)ln_s.size(), ns = (int)ls_s.size();
                const int te = table_len(ne, s.xcd), tn = table_len(nn, s.xcd), ts = table_len(ns, s.xcd);
                fill_table(reinterpret_cast<int *>(host.data() + o), ne, s.xcd, le_s, le_l);
                int *et = reinterpret_cast<int *>(base + o);
                o += al(sizeof(int) * 2 * te);
                fill_table(reinterpret_cast<int *>(host.data() + o), nn, s.xcd, ln_s, ln_l);
                int *nt = reinterpret_cast<int *>(base + o);
                o += al(sizeof(int) * 2 * tn);
                fill_table(reinterpret_cast<int *>(host.data() + o), ns, s.xcd, ls_s, ls_l);
                int *st_ = reinterpret_cast<int *>(base + o);
                o += al(sizeof(int) * 2 * ts);
                s.ep = LaunchPlan{g.desc, et, et + te, te, 0, s.epb, te};
                s.np = LaunchPlan{g.desc, nt, nt + tn, tn, 0, 0, tn};
                s.sp = LaunchPlan{g.desc, st_, st_ + ts, ts, 0, 0, ts};
            }
            select(g, g.pick, g.measured);
        }
        if (total) {
            if (hipMemcpyAsync(dmem, host.data(), total, hipMemcpyHostToDevice, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return SLBM_EDEVICE;
        }
        tables_ok = true;
        return SLBM_OK;
    }

    // Allocation-free stepping.  The tables of each group's chosen shape are laid out in the
    // per-device static array (no device allocation) and uploaded when the array does not
    // already hold this batch's current layout; the groups then step one after another on
    // the batch's stream with plain launches (no graphs, no tuning, no extra streams).
    slbm_status step_static(int64_t n) {
        if (dirty)
            if (slbm_status s = regroup()) return s;
        void *base_v = nullptr;
        if (static_scratch(&base_v)) return SLBM_EDEVICE;
        char *base = (char *)base_v;
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        size_t total = 0;
        std::vector<size_t> goff;
        std::vector<int> ne(groups.size()), nn(groups.size());
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const Group &g = groups[gi];
            const Shape &sh = g.shapes[g.pick];
            ne[gi] = nn[gi] = 0;
            for (int i : g.idx) {
                ne[gi] += eblocks(members[i], sh.epb);
                nn[gi] += members[i]->n_sblocks;
            }
            goff.push_back(total);
            total += al(sizeof(SolveDesc) * g.idx.size()) + al(sizeof(int) * 2 * table_len(ne[gi], sh.xcd)) +
                     al(sizeof(int) * 2 * table_len(nn[gi], sh.xcd));
        }
        if (total > kStaticScratchBytes) {
            status = SLBM_ENOMEM;
            return SLBM_ENOMEM;  // the launch tables exceed the static array
        }
        std::vector<LaunchPlan> sep(groups.size()), snp(groups.size());
        std::vector<char> img(total, 0);
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const Group &g = groups[gi];
            const Shape &sh = g.shapes[g.pick];
            size_t o = goff[gi];
            SolveDesc *dd = reinterpret_cast<SolveDesc *>(base + o);
            SolveDesc *dh = reinterpret_cast<SolveDesc *>(img.data() + o);
            for (int k = 0; k < (int)g.idx.size(); ++k) dh[k] = members[g.idx[k]]->desc;
            o += al(sizeof(SolveDesc) * g.idx.size());
            std::vector<int> le_s, le_l, ln_s, ln_l;
            for (int k = 0; k < (int)g.idx.size(); ++k) {
                slbm_ctx *c = members[g.idx[k]];
                for (int b = 0; b < eblocks(c, sh.epb); ++b) { le_s.push_back(k); le_l.push_back(b); }
                for (int b = 0; b < c->n_sblocks; ++b) { ln_s.push_back(k); ln_l.push_back(b); }
            }
            const int te = table_len(ne[gi], sh.xcd), tn = table_len(nn[gi], sh.xcd);
            fill_table(reinterpret_cast<int *>(img.data() + o), ne[gi], sh.xcd, le_s, le_l);
            int *et = reinterpret_cast<int *>(base + o);
            o += al(sizeof(int) * 2 * te);
            fill_table(reinterpret_cast<int *>(img.data() + o), nn[gi], sh.xcd, ln_s, ln_l);
            int *nt = reinterpret_cast<int *>(base + o);
            sep[gi] = LaunchPlan{dd, et, et + te, te, 0, sh.epb, te};
            snp[gi] = LaunchPlan{dd, nt, nt + tn, tn, 0, 0, tn};
        }
        hipStream_t st = (hipStream_t)stream;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return SLBM_EDEVICE;
        if (!static_holds(dev, id, layout_gen)) {
            // launches queued earlier on this stream may still read the array's previous
            // tables; the upload waits for them and completes before the steps are queued
            if (hipStreamSynchronize(st) != hipSuccess ||
                hipMemcpyAsync(base, img.data(), total, hipMemcpyHostToDevice, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return SLBM_EDEVICE;
            static_claim(dev, id, layout_gen);
        }
        for (size_t gi = 0; gi < groups.size(); ++gi)
            if (enqueue_group(groups[gi], sep[gi], snp[gi], n)) return SLBM_EDEVICE;
        return SLBM_OK;
    }

    // which batch layout each device's static array holds (batch id, layout generation)
    static std::mutex &static_mu() { static std::mutex m; return m; }
    static std::map<int, std::pair<uint64_t, uint64_t>> &static_owner() {
        static std::map<int, std::pair<uint64_t, uint64_t>> m;
        return m;
    }
    static bool static_holds(int dev, uint64_t bid, uint64_t gen) {
        std::lock_guard<std::mutex> lk(static_mu());
        auto it = static_owner().find(dev);
        return it != static_owner().end() && it->second == std::make_pair(bid, gen);
    }
    static void static_claim(int dev, uint64_t bid, uint64_t gen) {
        std::lock_guard<std::mutex> lk(static_mu());
        static_owner()[dev] = {bid, gen};
    }
    static uint64_t next_id() {
        static std::mutex m;
        static uint64_t k = 0;
        std::lock_guard<std::mutex> lk(m);
        return ++k;
    }
    const uint64_t id = next_id();   // distinguishes batches (addresses may be reused)
    uint64_t layout_gen = 0;         // bumped at every regroup and shape change
};

extern "C" slbm_status slbm_batch_create(void *hip_stream, slbm_batch **out) {
    return slbm_guard([&]() -> slbm_status {
        if (!out) return SLBM_EINVAL;
        *out = new (std::nothrow) slbm_batch();
        if (!*out) return SLBM_ENOMEM;
        (*out)->stream = hip_stream;
        const char *ng = std::getenv("SLBM_NO_GRAPH");
        (*out)->use_graph = !(ng && ng[0] == '1');
        const char *sg = std::getenv("SLBM_SERIAL_GROUPS");
        (*out)->concurrent = !(sg && sg[0] == '1');
        const char *at = std::getenv("SLBM_AUTOTUNE");
        (*out)->autotune = !(at && at[0] == '0');
        return SLBM_OK;
    });
}

extern "C" slbm_status slbm_batch_add(slbm_batch *b, slbm_ctx *c) {
    return slbm_guard([&]() -> slbm_status {
        if (!b || !c) return SLBM_EINVAL;
        if (!c->bound || !c->has_state) return SLBM_ESTATE;
        if (c->stream != b->stream) return SLBM_EINVAL;
        if (std::find(b->members.begin(), b->members.end(), c) != b->members.end()) return SLBM_EINVAL;
        b->members.push_back(c);
        b->dirty = true;
        return SLBM_OK;
    });
}

extern "C" slbm_status slbm_batch_remove(slbm_batch *b, slbm_ctx *c) {
    return slbm_guard([&]() -> slbm_status {
        if (!b || !c) return SLBM_EINVAL;
        auto it = std::find(b->members.begin(), b->members.end(), c);
        if (it == b->members.end()) return SLBM_EINVAL;
        b->members.erase(it);
        b->dirty = true;
        return SLBM_OK;
    });
}

extern "C" int slbm_batch_size(const slbm_batch *b) { return b ? (int)b->members.size() : 0; }

extern "C" slbm_status slbm_batch_set_autotune(slbm_batch *b, int on) {
    return slbm_guard([&]() -> slbm_status {
        if (!b || (on != 0 && on != 1)) return SLBM_EINVAL;
        b->autotune = on == 1;
        return SLBM_OK;
    });
}

extern "C" slbm_status slbm_batch_shapes(slbm_batch *b, slbm_batch_shape *out, int max, int *count) {
    return slbm_guard([&]() -> slbm_status {
        if (!b || !count || max < 0 || (max > 0 && !out)) return SLBM_EINVAL;
        if (!b->members.empty())
            if (slbm_status s = b->rebuild()) return s;
        const int ng = b->members.empty() ? 0 : (int)b->groups.size();
        *count = ng;
        for (int gi = 0; gi < std::min(ng, max); ++gi) {
            const auto &g = b->groups[gi];
            slbm_batch_shape &r = out[gi];
            r = slbm_batch_shape{};
            r.dim = g.d == 2 ? 2 : 3;
            r.lattice = g.d == 2 ? 9 : (g.d == 3 ? 19 : 13);
            r.order = g.N;
            r.fused = g.fused ? 1 : 0;
            r.members = (int)g.idx.size();
            r.elements = g.elements;
            r.n_shapes = std::min((int)g.shapes.size(), SLBM_MAX_SHAPES);
            for (int k = 0; k < r.n_shapes; ++k) {
                r.epb[k] = g.shapes[k].epb;
                r.xcd[k] = g.shapes[k].xcd ? 1 : 0;
                r.us_per_step[k] = g.shapes[k].us;
            }
            r.chosen = g.pick;
            r.measured = g.measured ? 1 : 0;
        }
        return SLBM_OK;
    });
}

extern "C" slbm_status slbm_batch_step(slbm_batch *b, int64_t n) {
    return slbm_guard([&]() -> slbm_status {
        if (!b || n < 0) return SLBM_EINVAL;
        if (b->members.empty() || n == 0) return SLBM_OK;
        if (slbm_status s = b->rebuild()) return s;
        int64_t done = 0;
        if (b->autotune && (done = b->tune_pending(n)) < 0) return SLBM_EDEVICE;
        if (b->run(n - done)) return SLBM_EDEVICE;
        for (slbm_ctx *c : b->members) c->step += n;
        // every unfused step leaves the Laplacian partials of its last stage's input behind,
        // also after a state upload cleared the flag since the rebuild
        for (auto &g : b->groups)
            if (!g.fused)
                for (int i : g.idx)
                    if (b->members[i]->fused) b->members[i]->rl_stale = true;
        return SLBM_OK;
    });
}

extern "C" slbm_status slbm_batch_step_static(slbm_batch *b, int64_t n) {
    return slbm_guard([&]() -> slbm_status {
        if (!b || n < 0) return SLBM_EINVAL;
        if (b->members.empty() || n == 0) return SLBM_OK;
        if (slbm_status s = b->step_static(n)) return s;
        for (slbm_ctx *c : b->members) c->step += n;
        for (auto &g : b->groups)
            if (!g.fused)
                for (int i : g.idx)
                    if (b->members[i]->fused) b->members[i]->rl_stale = true;
        return SLBM_OK;
    });
}

extern "C" slbm_status slbm_batch_kinetic_energy(slbm_batch *b, double *ke, double *mass) {
    return slbm_guard([&]() -> slbm_status {
        if (!b) return SLBM_EINVAL;
        if (b->members.empty()) return SLBM_OK;
        if (slbm_status s = b->rebuild()) return s;
        hipStream_t st = (hipStream_t)b->stream;
        std::vector<std::vector<double>> outs(b->groups.size());
        for (size_t gi = 0; gi < b->groups.size(); ++gi) {
            auto &g = b->groups[gi];
            int e = launch_diag(g.d, g.N, g.np, b->stream);
            if (e == 0) e = launch_diag_final(g.desc, (int)g.idx.size(), b->stream, g.diag_out);
            if (e) return SLBM_EDEVICE;
            outs[gi].resize(2 * g.idx.size());
            if (hipMemcpyAsync(outs[gi].data(), g.diag_out, 2 * sizeof(double) * g.idx.size(),
                               hipMemcpyDeviceToHost, st) != hipSuccess)
                return SLBM_EDEVICE;
        }
        if (hipStreamSynchronize(st) != hipSuccess) return SLBM_EDEVICE;
        for (size_t gi = 0; gi < b->groups.size(); ++gi)
            for (size_t k = 0; k < b->groups[gi].idx.size(); ++k) {
                const int m = b->groups[gi].idx[k];
                if (ke) ke[m] = outs[gi][2 * k];
                if (mass) mass[m] = outs[gi][2 * k + 1];
            }
        return SLBM_OK;
    });
}

extern "C" void slbm_batch_destroy(slbm_batch *b) { delete b; }

// ------------------------------------------------------------------------------------------
// contact angle (host): mid-density crossings, Kasa circle/sphere fit, wall intersection
// ------------------------------------------------------------------------------------------
namespace {

// solve the small dense system A x = r (n <= 4) by Gaussian elimination with pivoting
bool solve_small(int n, double A[4][4], double *r, double *x) {
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[i][k]) > std::fabs(A[piv][k])) piv = i;
        if (A[piv][k] == 0.0) return false;
        if (piv != k) {
            for (int j = 0; j < n; ++j) std::swap(A[k][j], A[piv][j]);
            std::swap(r[k], r[piv]);
        }
        for (int i = k + 1; i < n; ++i) {
            const double m = A[i][k] / A[k][k];
            for (int j = k; j < n; ++j) A[i][j] -= m * A[k][j];
            r[i] -= m * r[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = r[k];
        for (int j = k + 1; j < n; ++j) s -= A[k][j] * x[j];
        x[k] = s / A[k][k];
    }
    return true;
}

}  // namespace

extern "C" slbm_status slbm_contact_angle(slbm_ctx *c, const slbm_wall_geom *w, double *theta_deg) {
    return slbm_guard([&]() -> slbm_status {
        if (!c || !w || !theta_deg) return SLBM_EINVAL;
        if (slbm_status s = c->require_bound(true)) return s;
        const int dim = c->dim, Np = c->Np, nloc = c->nloc;
        std::vector<double> rho(c->Ng);
        int e = (int)hipMemcpyAsync(rho.data(), c->desc.rho, sizeof(double) * c->Ng, hipMemcpyDeviceToHost,
                                    (hipStream_t)c->stream);
        if (e == 0) e = (int)hipStreamSynchronize((hipStream_t)c->stream);
        if (e) return c->hip_check(e, "contact_angle");
        const double level = 0.5 * (c->prm.rho_l + c->prm.rho_v);
        const double excl = 2.0 * c->prm.delta;
        std::unordered_set<uint64_t> seen;
        std::vector<double> pts;
        for (int64_t el = 0; el < c->E; ++el)
            for (int a = 0; a < dim; ++a) {
                const int s = c->stride(a);
                for (int n = 0; n < nloc; ++n) {
                    if (c->along(n, a) == Np - 1) continue;
                    const int64_t l1 = el * nloc + n, l2 = l1 + s;
                    const uint32_t g1 = (uint32_t)c->lgid[l1], g2 = (uint32_t)c->lgid[l2];
                    const uint64_t key = ((uint64_t)std::min(g1, g2) << 32) | std::max(g1, g2);
                    const double r1 = rho[g1] - level, r2 = rho[g2] - level;
                    if ((r1 == 0.0 && r2 == 0.0) || r1 * r2 > 0.0) continue;
                    if (!seen.insert(key).second) continue;
                    const double t = r1 / (r1 - r2);
                    double p[3] = {0, 0, 0};
                    for (int k = 0; k < dim; ++k) {
                        const double x1 = c->xyz[l1 * dim + k], x2 = c->xyz[l2 * dim + k];
                        p[k] = x1 + t * (x2 - x1);
                    }
                    double dist;
                    if (w->kind == 0) {
                        double dd = 0.0;
                        for (int k = 0; k < dim; ++k) dd += (p[k] - w->point[k]) * w->normal[k];
                        dist = std::fabs(dd);
                    } else {
                        double r2s = 0.0;
                        for (int k = 0; k < dim; ++k) r2s += (p[k] - w->point[k]) * (p[k] - w->point[k]);
                        dist = std::sqrt(r2s) - w->radius;
                    }
                    if (dist < excl) continue;
                    for (int k = 0; k < dim; ++k) pts.push_back(p[k]);
                }
            }
        const int64_t np = (int64_t)pts.size() / dim;
        if (np < dim + 2) return c->fail(SLBM_EINVAL, "contact angle: too few interface points (%lld)", (long long)np);
        // Kasa fit about the centroid: |y|^2 + b.y + k = 0 with y = p - m
        double m[3] = {0, 0, 0};
        for (int64_t i = 0; i < np; ++i)
            for (int k = 0; k < dim; ++k) m[k] += pts[i * dim + k];
        for (int k = 0; k < dim; ++k) m[k] /= (double)np;
        const int nu = dim + 1;
        double A[4][4] = {}, rhs[4] = {}, x[4] = {};
        for (int64_t i = 0; i < np; ++i) {
            double row[4], y2 = 0.0;
            for (int k = 0; k < dim; ++k) {
                row[k] = pts[i * dim + k] - m[k];
                y2 += row[k] * row[k];
            }
            row[dim] = 1.0;
            for (int r = 0; r < nu; ++r) {
                for (int q = 0; q < nu; ++q) A[r][q] += row[r] * row[q];
                rhs[r] -= row[r] * y2;
            }
        }
        if (!solve_small(nu, A, rhs, x)) return c->fail(SLBM_EINVAL, "contact angle: singular fit");
        double cen[3] = {0, 0, 0}, c2 = 0.0;
        for (int k = 0; k < dim; ++k) {
            cen[k] = -0.5 * x[k];
            c2 += cen[k] * cen[k];
            cen[k] += m[k];
        }
        const double R = std::sqrt(c2 - x[dim]);
        double cth;
        if (w->kind == 0) {
            double dd = 0.0;
            for (int k = 0; k < dim; ++k) dd += (cen[k] - w->point[k]) * w->normal[k];
            cth = dd / R;
        } else {
            double d2 = 0.0;
            for (int k = 0; k < dim; ++k) d2 += (cen[k] - w->point[k]) * (cen[k] - w->point[k]);
            const double Rw = w->radius;
            cth = (Rw * Rw + R * R - d2) / (2.0 * R * Rw);
        }
        cth = std::max(-1.0, std::min(1.0, cth));
        *theta_deg = std::acos(cth) * 180.0 / M_PI;
        return SLBM_OK;
    });
}

// ------------------------------------------------------------------------------------------
// server
// ------------------------------------------------------------------------------------------
namespace {
struct Request {
    uint64_t id = 0;
    slbm_status prep_status = SLBM_OK;
    slbm_request r{};
    std::vector<double> xyz, wcos, wub;
    std::vector<int32_t> gid, wface;
    slbm_result res{};
    slbm_ctx *ctx = nullptr;
    size_t off = 0, bytes = 0;
    int64_t steps = 0;
    slbm_status job_status = SLBM_OK;  // result of the last worker job run for it
};

// first-fit allocator over the arena (offsets 256-byte aligned)
struct Arena {
    std::map<size_t, size_t> free_;  // offset -> size
    void init(size_t bytes) { free_.clear(); if (bytes) free_[0] = bytes; }
    bool alloc(size_t n, size_t &off) {
        n = (n + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n) {
        n = (n + 255) & ~(size_t)255;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};
}  // namespace

struct slbm_server {
    slbm_server_cfg cfg{};
    std::chrono::steady_clock::time_point t0;
    std::map<uint64_t, Request *> all;
    std::vector<Request *> active;
    uint64_t next_id = 1;
    Arena arena;
    slbm_batch *batch = nullptr;
    // host-side preparation (context creation and mesh processing) runs on worker threads
    // while the device advances the active solves
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> to_prepare;          // submitted, not yet prepared
    std::map<uint64_t, Request *> prepared;    // ready for admission, by id
    int preparing = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
    static constexpr std::chrono::milliseconds kColdStartWait{50};
    // jobs the tick hands to the workers and waits for, ahead of any preparation: binding
    // the requests it has just admitted (workspace uploads and initial state, each worker on
    // a stream of its own) and the contact angles of the solves it retires.  A round then
    // pays for the slowest of these rather than for their sum.
    enum JobKind { kBind, kAngle };
    std::deque<std::pair<JobKind, Request *>> jobs;
    int jobs_left = 0;
    int device = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void worker() {
        (void)hipSetDevice(device);
        hipStream_t ws = nullptr;
        if (hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess) ws = nullptr;
        void *own = ws ? (void *)ws : cfg.hip_stream;
        for (;;) {
            Request *r = nullptr;
            bool job = false;
            JobKind kind = kBind;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stopping || !jobs.empty() || !to_prepare.empty(); });
                if (!jobs.empty()) {
                    job = true;
                    kind = jobs.front().first;
                    r = jobs.front().second;
                    jobs.pop_front();
                } else if (!to_prepare.empty()) {
                    r = to_prepare.front();
                    to_prepare.pop_front();
                    ++preparing;
                } else {
                    break;  // stopping
                }
            }
            if (job) {
                run_job(kind, r, own);
                {
                    std::lock_guard<std::mutex> lk(mu);
                    --jobs_left;
                }
                cv.notify_all();
                continue;
            }
            slbm_ctx *c = nullptr;
            slbm_params p = r->r.params;
            slbm_status st = slbm_create(&p, &c);
            if (st == SLBM_OK)
                st = slbm_set_mesh(c, r->r.E, r->xyz.data(), r->gid.data(), r->r.n_global,
                                   r->r.n_wall_faces, r->wface.empty() ? nullptr : r->wface.data(),
                                   r->wcos.empty() ? nullptr : r->wcos.data(),
                                   r->wub.empty() ? nullptr : r->wub.data());
            if (st != SLBM_OK && c) {
                slbm_destroy(c);
                c = nullptr;
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                r->ctx = c;
                r->prep_status = st;
                prepared[r->id] = r;
                --preparing;
            }
            cv.notify_all();
        }
        if (ws) (void)hipStreamDestroy(ws);
    }

    void run_job(JobKind kind, Request *r, void *own) {
        if (kind == kBind) {
            slbm_status st = slbm_bind(r->ctx, (char *)cfg.arena + r->off, r->bytes, own);
            if (st == SLBM_OK) st = slbm_init_tanh(r->ctx, r->r.x0, r->r.R, r->r.noise_amp, r->r.params.seed);
            // the uploads have completed (bind and init synchronise their stream): from here
            // on the solve is stepped and queried on the server's stream
            if (st == SLBM_OK) r->ctx->stream = cfg.hip_stream;
            r->job_status = st;
        } else {
            // a retired solve is no longer stepped: read its density on this worker's stream
            // (the server's stream, which produced it, is idle)
            r->ctx->stream = own;
            double th = NAN;
            r->job_status = slbm_contact_angle(r->ctx, &r->r.wall, &th);
            r->res.theta_deg = r->job_status == SLBM_OK ? th : NAN;
            if (r->r.state_out) {
                int64_t st = 0;
                const slbm_status s2 = slbm_get_state(r->ctx, r->r.state_out, &st);
                if (r->job_status == SLBM_OK) r->job_status = s2;
            }
        }
    }

    // hand one job per request to the workers and wait until all have finished
    void run_jobs(JobKind kind, const std::vector<Request *> &rs) {
        if (rs.empty()) return;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (Request *r : rs) jobs.emplace_back(kind, r);
            jobs_left += (int)rs.size();
        }
        cv.notify_all();
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return jobs_left == 0; });
    }

    ~slbm_server() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stopping = true;
        }
        cv.notify_all();
        for (auto &t : workers) t.join();
        for (auto &kv : all)
            if (kv.second->ctx) slbm_destroy(kv.second->ctx);
        for (auto &kv : all) delete kv.second;
        slbm_batch_destroy(batch);
    }

    void finish(Request *r, slbm_status st) {
        r->res.status = st;
        r->res.steps = r->steps;
        r->res.t_done = now();
        if (r->ctx) {
            slbm_destroy(r->ctx);
            r->ctx = nullptr;
        }
        if (r->bytes) {
            arena.release(r->off, r->bytes);
            r->bytes = 0;
        }
        r->xyz.clear(); r->xyz.shrink_to_fit();
        r->gid.clear(); r->gid.shrink_to_fit();
    }

    // admission of a prepared request: reserve its arena bytes (it is then bound by a
    // worker), or finish it with its error.  Returns 0 if it must wait for arena bytes,
    // 1 if it was finished, 2 if it was reserved.  `reserved` counts the requests reserved
    // in this round and not yet active.
    int admit(Request *r, size_t reserved) {
        if (r->prep_status != SLBM_OK || !r->ctx) { finish(r, r->prep_status ? r->prep_status : SLBM_EINVAL); return 1; }
        const size_t need = slbm_workspace_bytes(r->ctx);
        size_t off = 0;
        if (need > cfg.arena_bytes) { finish(r, SLBM_ENOMEM); return 1; }
        if (!arena.alloc(need, off)) {
            // with no active or reserved solve the arena is entirely free: this request can
            // never fit
            if (active.empty() && reserved == 0) { finish(r, SLBM_ENOMEM); return 1; }
            return 0;
        }
        r->off = off;
        r->bytes = need;
        return 2;
    }

    int pending() {
        std::lock_guard<std::mutex> lk(mu);
        return (int)(active.size() + to_prepare.size() + prepared.size()) + preparing;
    }
};

extern "C" slbm_status slbm_server_create(const slbm_server_cfg *cfg, slbm_server **out) {
    return slbm_guard([&]() -> slbm_status {
        if (!cfg || !out || !cfg->arena || cfg->max_slots <= 0 || cfg->check_every <= 0) return SLBM_EINVAL;
        slbm_server *s = new (std::nothrow) slbm_server();
        if (!s) return SLBM_ENOMEM;
        s->cfg = *cfg;
        s->t0 = std::chrono::steady_clock::now();
        s->arena.init(cfg->arena_bytes);
        if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
        if (slbm_batch_create(cfg->hip_stream, &s->batch) != SLBM_OK) { delete s; return SLBM_ENOMEM; }
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const unsigned nw = std::min(8u, std::max(1u, hw / 2));
        try {
            for (unsigned k = 0; k < nw; ++k) s->workers.emplace_back([s] { s->worker(); });
        } catch (...) {
            // fewer workers than asked for: fine while at least one runs
        }
        if (s->workers.empty()) {
            delete s;
            return SLBM_ENOMEM;
        }
        *out = s;
        return SLBM_OK;
    });
}

extern "C" slbm_status slbm_server_submit(slbm_server *s, const slbm_request *r, uint64_t *id) {
    return slbm_guard([&]() -> slbm_status {
        if (!s || !r || !r->xyz || !r->gid || r->E <= 0) return SLBM_EINVAL;
        const int dim = r->params.lattice == 19 ? 3 : 2;
        const int64_t nloc = nloc_of(dim, r->params.N);
        Request *q = new (std::nothrow) Request();
        if (!q) return SLBM_ENOMEM;
        q->id = s->next_id++;
        q->r = *r;
        q->xyz.assign(r->xyz, r->xyz + r->E * nloc * dim);
        q->gid.assign(r->gid, r->gid + r->E * nloc);
        if (r->n_wall_faces > 0) {
            q->wface.assign(r->wall_face, r->wall_face + 2 * r->n_wall_faces);
            q->wcos.assign(r->wall_cos, r->wall_cos + r->n_wall_faces);
            if (r->wall_ub) q->wub.assign(r->wall_ub, r->wall_ub + dim * r->n_wall_faces);
        }
        q->r.xyz = nullptr;
        q->r.gid = nullptr;
        q->r.wall_face = nullptr;
        q->r.wall_cos = nullptr;
        q->r.wall_ub = nullptr;
        q->res.status = 1;
        q->res.t_arrive = s->now();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->all[q->id] = q;
            s->to_prepare.push_back(q);
        }
        s->cv.notify_one();
        if (id) *id = q->id;
        return SLBM_OK;
    });
}

extern "C" slbm_status slbm_server_tick(slbm_server *s, int *pending) {
    return slbm_guard([&]() -> slbm_status {
        if (!s) return SLBM_EINVAL;
        // cold start (no active solve, the device idle): let the preparations already submitted
        // finish (at most kColdStartWait) so that they start together rather than one round
        // apart, which would leave their last round with only the late ones on the device
        if (s->active.empty()) {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait_for(lk, slbm_server::kColdStartWait,
                           [&] { return s->stopping || (s->preparing == 0 && s->to_prepare.empty()); });
        }
        // admission: prepared requests in submission order while slots and arena bytes allow;
        // the workers bind the admitted ones together, then they join the batch
        std::vector<Request *> admitted;
        for (;;) {
            if ((int)(s->active.size() + admitted.size()) >= s->cfg.max_slots) break;
            Request *r = nullptr;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (s->prepared.empty()) break;
                r = s->prepared.begin()->second;
            }
            const int a = s->admit(r, admitted.size());
            if (a == 0) break;
            if (a == 2) admitted.push_back(r);
            std::lock_guard<std::mutex> lk(s->mu);
            s->prepared.erase(r->id);
        }
        s->run_jobs(slbm_server::kBind, admitted);
        for (Request *r : admitted) {
            slbm_status st = r->job_status;
            if (st == SLBM_OK) st = slbm_batch_add(s->batch, r->ctx);
            if (st != SLBM_OK) { s->finish(r, st); continue; }
            r->res.t_admit = s->now();
            s->active.push_back(r);
        }
        if (!s->active.empty()) {
            // the device advances every active solve while the workers prepare new requests
            if (slbm_status st = slbm_batch_step(s->batch, s->cfg.check_every)) return st;
            std::vector<double> ke(s->active.size()), mass(s->active.size());
            if (slbm_status st = slbm_batch_kinetic_energy(s->batch, ke.data(), mass.data())) return st;
            std::vector<Request *> keep, retired;
            for (size_t i = 0; i < s->active.size(); ++i) {
                Request *r = s->active[i];
                r->steps += s->cfg.check_every;
                r->res.ke_max = ke[i];
                const double lim = r->r.params.ke_limit > 0.0 ? r->r.params.ke_limit : 1.0;
                const bool bad = !(ke[i] <= lim);
                const bool done = ke[i] < s->cfg.ke_stop || r->steps >= s->cfg.max_steps;
                if (bad || done) {
                    slbm_batch_remove(s->batch, r->ctx);
                    if (bad) s->finish(r, SLBM_EDIVERGED);
                    else retired.push_back(r);
                } else {
                    keep.push_back(r);
                }
            }
            s->active.swap(keep);
            // contact angles of the retired solves, on the workers (the device is idle: the
            // kinetic-energy readout above synchronised the server's stream)
            s->run_jobs(slbm_server::kAngle, retired);
            for (Request *r : retired) s->finish(r, SLBM_OK);
        } else {
            // nothing to run: wait for a worker to finish a preparation
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->prepared.empty() && (s->preparing > 0 || !s->to_prepare.empty()))
                s->cv.wait_for(lk, std::chrono::milliseconds(5));
        }
        if (pending) *pending = s->pending();
        return SLBM_OK;
    });
}

extern "C" slbm_status slbm_server_poll(slbm_server *s, uint64_t id, slbm_result *out) {
    return slbm_guard([&]() -> slbm_status {
        if (!s || !out) return SLBM_EINVAL;
        auto it = s->all.find(id);
        if (it == s->all.end()) return SLBM_EINVAL;
        *out = it->second->res;
        return SLBM_OK;
    });
}

extern "C" slbm_status slbm_server_drain(slbm_server *s) {
    return slbm_guard([&]() -> slbm_status {
        if (!s) return SLBM_EINVAL;
        int pending = 1;
        while (pending > 0)
            if (slbm_status st = slbm_server_tick(s, &pending)) return st;
        return SLBM_OK;
    });
}

extern "C" double slbm_server_clock(const slbm_server *s) { return s ? s->now() : 0.0; }

extern "C" void slbm_server_destroy(slbm_server *s) { delete s; }
