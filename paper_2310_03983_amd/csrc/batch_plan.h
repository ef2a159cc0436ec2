// Host-side plan of the dependency-driven batched schedule (no HIP types,
// so host tests can build plans and check them).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <queue>
#include <utility>
#include <vector>

namespace apsp {

// Task kinds of the schedule: the first pivot closure of a graph; the fused
// next pivot (round r's update of tile (r+1, r+1), then its closure); a row
// or column panel tile of round r; a remainder tile of round r.
enum BatchTaskKind : int32_t { kTaskClose = 0, kTaskFused = 1, kTaskRow = 2, kTaskCol = 3, kTaskRem = 4 };

// One task (48 bytes): tile coordinates in tiles of the graph's round width.
struct BatchTask {
    int32_t kind;           // BatchTaskKind
    int32_t graph;
    int32_t round;          // FW round whose pivot band the task uses
    int32_t a, b;           // panel tile a; remainder tile (a, b); fused pivot (a, a)
    int32_t wait0, need0;   // wait until counters[wait0] >= need0 (wait0 < 0: none)
    int32_t wait1, need1;
    int32_t signal;         // counter incremented when done (< 0: none)
    int32_t width;          // the graph's round width (64 or 128)
    int32_t sub;            // products: -1 the whole tile, else 64 x 64 sub-tile (si | sj << 8)
};

// Round width of a graph of n vertices under a per-class plan: classes are
// bounded by class_max[0] < class_max[1] < ...; a graph takes the width of
// the first class with n <= class_max[c], the last class otherwise.
inline int class_width(int n, int nclass, const int32_t* class_max, const int32_t* class_width)
{
    for (int c = 0; c < nclass; ++c)
        if (n <= class_max[c]) return class_width[c];
    return class_width[nclass - 1];
}

// Dependency-driven plan: the tasks of every graph's Floyd-Warshall rounds
// (graph g's rounds widths[g] wide), in level order (level 0: every graph's
// first pivot closure; level 2r+1: round r's panel tiles; level 2r+2: the
// next pivot and round r's remainder tiles), graphs as listed in `order`
// within a level.  Every dependency points to an earlier level, so the list
// is a topological order.
//
// With subs[g] = 0 a product task covers a whole tile and the next pivot is
// one fused task (round r's update of tile (r+1, r+1), then its closure).
// With subs[g] = 64 every product is cut into 64 x 64 sub-tiles, one task
// each, and the next pivot is its update sub-tiles followed by a closure
// task, so each step on a graph's chain of dependent steps runs on up to four
// workgroups.  The panel sub-tiles of one tile read rows (or columns) that
// the others rewrite; since the pivot block is closed, any mix of old and
// new values gives the same result for int32 (values only decrease and
// X* (min,+) X* = X*), and fp32 stays within rounding.
//
// Counters per graph with nb >= 2 rounds: piv[r] (pivot r closed), pan[r]
// (panel tasks of round r done), rem[r] (remainder tasks of round r done),
// upd[r] (update tasks of pivot r done, sub-tiled graphs).
inline void build_queue_plan(const int32_t* widths, const int32_t* subs, int32_t count, const int32_t* h_sizes,
                             const std::vector<int32_t>& order, std::vector<BatchTask>& tasks, int32_t& ncounters)
{
    // counters only for the graphs listed in `order` (a subset of the batch
    // when the tasks are split into several queues)
    std::vector<int32_t> base(count, -1), nbs(count, 0);
    int32_t nc = 0, max_nb = 0;
    for (int32_t g : order) {
        nbs[g] = (h_sizes[g] + widths[g] - 1) / widths[g];
        max_nb = std::max(max_nb, nbs[g]);
        if (nbs[g] >= 2) {
            base[g] = nc;
            nc += 4 * nbs[g];
        }
    }
    auto piv = [&](int32_t g, int r) { return base[g] + r; };
    auto pan = [&](int32_t g, int r) { return base[g] + nbs[g] + r; };
    auto rem = [&](int32_t g, int r) { return base[g] + 2 * nbs[g] + r; };
    auto upd = [&](int32_t g, int r) { return base[g] + 3 * nbs[g] + r; };
    // extent of tile t of graph g, and its number of sub-tiles per side
    auto ext = [&](int32_t g, int t) { return std::min(widths[g], h_sizes[g] - t * widths[g]); };
    auto nsub = [&](int32_t g, int e) { return subs[g] > 0 ? (e + subs[g] - 1) / subs[g] : 1; };
    auto task = [&](int kind, int32_t g, int r, int a, int b, int sub, int w0, int n0, int w1, int n1, int sig) {
        BatchTask t{};
        t.kind = kind;
        t.graph = g;
        t.round = r;
        t.a = a;
        t.b = b;
        t.wait0 = w0;
        t.need0 = n0;
        t.wait1 = w1;
        t.need1 = n1;
        t.signal = sig;
        t.width = widths[g];
        t.sub = sub;
        tasks.push_back(t);
    };
    // every (sub-)tile task of tile (i, j): calls emit(sub code)
    auto tiles_of = [&](int32_t g, int i, int j, auto&& emit) {
        if (subs[g] <= 0) {
            emit(-1);
            return;
        }
        const int mi = nsub(g, ext(g, i)), mj = nsub(g, ext(g, j));
        for (int si = 0; si < mi; ++si)
            for (int sj = 0; sj < mj; ++sj) emit(si | (sj << 8));
    };
    auto count_tiles = [&](int32_t g, int i, int j) { return nsub(g, ext(g, i)) * nsub(g, ext(g, j)); };
    // tasks of round r's panels / remainder (excluding the next pivot tile)
    auto npan = [&](int32_t g, int r) {
        int c = 0;
        for (int t = 0; t < nbs[g]; ++t)
            if (t != r) c += count_tiles(g, r, t) + count_tiles(g, t, r);
        return c;
    };
    auto nrem = [&](int32_t g, int r) {
        int c = 0;
        const int nb = nbs[g];
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j)
                if (i != r && j != r && !(r + 1 < nb && i == r + 1 && j == r + 1)) c += count_tiles(g, i, j);
        return c;
    };
    tasks.clear();
    const int32_t listed = (int32_t)order.size();
    for (int32_t q = 0; q < listed; ++q) {   // level 0
        const int32_t g = order[q];
        if (h_sizes[g] > 1) task(kTaskClose, g, 0, 0, 0, -1, -1, 0, -1, 0, nbs[g] >= 2 ? piv(g, 0) : -1);
    }
    for (int r = 0; r < max_nb; ++r) {
        for (int32_t q = 0; q < listed; ++q) {   // level 2r+1: pivot r closed (sub-tiled), panels of round r
            const int32_t g = order[q];
            const int nb = nbs[g];
            if (nb < 2 || r >= nb) continue;
            if (r > 0 && subs[g] > 0)
                task(kTaskClose, g, r, r, r, -1, upd(g, r), count_tiles(g, r, r), -1, 0, piv(g, r));
            // round r-1's remainder skipped tile (r, r), which the next-pivot tasks did
            const int nprev = r > 0 ? nrem(g, r - 1) : 0;
            for (int t = 0; t < nb; ++t) {
                if (t == r) continue;
                tiles_of(g, r, t, [&](int sc) {
                    task(kTaskRow, g, r, t, 0, sc, piv(g, r), 1, nprev > 0 ? rem(g, r - 1) : -1, nprev, pan(g, r));
                });
                tiles_of(g, t, r, [&](int sc) {
                    task(kTaskCol, g, r, t, 0, sc, piv(g, r), 1, nprev > 0 ? rem(g, r - 1) : -1, nprev, pan(g, r));
                });
            }
        }
        for (int32_t q = 0; q < listed; ++q) {   // level 2r+2: next pivot and remainder of round r
            const int32_t g = order[q];
            const int nb = nbs[g];
            if (nb < 2 || r >= nb) continue;
            const int np = npan(g, r);
            const bool next = r + 1 < nb;
            if (next) {
                if (subs[g] > 0)
                    tiles_of(g, r + 1, r + 1, [&](int sc) {
                        task(kTaskRem, g, r, r + 1, r + 1, sc, pan(g, r), np, -1, 0, upd(g, r + 1));
                    });
                else
                    task(kTaskFused, g, r, r + 1, r + 1, -1, pan(g, r), np, -1, 0, piv(g, r + 1));
            }
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < nb; ++j) {
                    if (i == r || j == r || (next && i == r + 1 && j == r + 1)) continue;
                    tiles_of(g, i, j, [&](int sc) {
                        task(kTaskRem, g, r, i, j, sc, pan(g, r), np, -1, 0, rem(g, r));
                    });
                }
        }
    }
    ncounters = nc;
}

// Estimated duration of a task in microseconds (a coarse model of the
// kernel's tiles: closures grow with the block's area and depth, products
// with their terms).  Only the ratios matter: they rank tasks for ordering.
struct TaskCost {
    double close_us = 6.0, close_scale_us = 38.0;   // closure of a w-block: close_us + close_scale_us (w/128)^2
    double tile_us = 4.0, tile_scale_us = 26.0;      // product of M x N x K: tile_us + tile_scale_us MNK/128^3
};

inline double task_us(const BatchTask& t, const int32_t* h_sizes, const TaskCost& c)
{
    const int n = h_sizes[t.graph], B = t.width;
    auto width = [&](int tile) { return std::min(B, n - tile * B); };
    const double bk = width(t.round);
    auto close = [&](double w) { return c.close_us + c.close_scale_us * (w / 128.0) * (w / 128.0); };
    auto prod = [&](double m, double nn, double k) {
        return c.tile_us + c.tile_scale_us * (m * nn * k) / (128.0 * 128.0 * 128.0);
    };
    // extent of a (sub-)tile side of length e: sub-tile index s of 64
    auto part = [&](double e, int s) { return t.sub < 0 ? e : std::min(64.0, e - 64.0 * s); };
    const int si = t.sub < 0 ? 0 : (t.sub & 0xff), sj = t.sub < 0 ? 0 : (t.sub >> 8);
    switch (t.kind) {
    case kTaskClose: return close(width(t.a));
    case kTaskFused: return prod(width(t.a), width(t.a), bk) + close(width(t.a));
    case kTaskRow: return prod(part(bk, si), part(width(t.a), sj), bk);
    case kTaskCol: return prod(part(width(t.a), si), part(bk, sj), bk);
    default: return prod(part(width(t.a), si), part(width(t.b), sj), bk);
    }
}

// Reorders a topologically ordered task list by list scheduling on
// `workers` concurrent workgroups: a simulation starts, whenever a worker is
// free, the ready task (every counter it waits for at its target) with the
// longest estimated path to the end of its graph, and the tickets follow the
// simulated start order.  A task starts only after the tasks it waits for
// finished, so the new order is topological too (the queue still drains).
inline void order_queue_plan(std::vector<BatchTask>& tasks, int32_t ncounters, int workers, const int32_t* h_sizes,
                             const TaskCost& cost)
{
    const int T = (int)tasks.size();
    if (T < 2 || workers < 1) return;
    std::vector<double> dur(T), rank(T, 0.0);
    for (int i = 0; i < T; ++i) dur[i] = task_us(tasks[i], h_sizes, cost);
    // successors: the tasks waiting on the counter a task signals
    std::vector<std::vector<int>> waiting(ncounters);
    for (int i = 0; i < T; ++i) {
        if (tasks[i].wait0 >= 0) waiting[tasks[i].wait0].push_back(i);
        if (tasks[i].wait1 >= 0) waiting[tasks[i].wait1].push_back(i);
    }
    // longest path to the end, in reverse topological (= current) order
    for (int i = T - 1; i >= 0; --i) {
        double best = 0.0;
        if (tasks[i].signal >= 0)
            for (int j : waiting[tasks[i].signal]) best = std::max(best, rank[j]);
        rank[i] = dur[i] + best;
    }
    std::vector<int32_t> cnt(ncounters, 0);
    auto ready = [&](int i) {
        const BatchTask& t = tasks[i];
        return (t.wait0 < 0 || cnt[t.wait0] >= t.need0) && (t.wait1 < 0 || cnt[t.wait1] >= t.need1);
    };
    std::priority_queue<std::pair<double, int>> rq;   // (rank, -index): highest rank, then earliest index
    for (int i = 0; i < T; ++i)
        if (ready(i)) rq.push({rank[i], -i});
    std::vector<char> queued(T, 0);
    for (int i = 0; i < T; ++i) queued[i] = ready(i);
    using Ev = std::pair<double, int>;      // (finish time, task)
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> running;
    std::vector<int> order;
    order.reserve(T);
    double now = 0.0;
    int free = workers;
    while ((int)order.size() < T) {
        while (free > 0 && !rq.empty()) {
            const int i = -rq.top().second;
            rq.pop();
            order.push_back(i);
            running.push({now + dur[i], i});
            --free;
        }
        if (running.empty()) break;   // cannot happen for a topological list
        const Ev e = running.top();
        running.pop();
        now = e.first;
        ++free;
        const int s = tasks[e.second].signal;
        if (s >= 0) {
            ++cnt[s];
            for (int j : waiting[s])
                if (!queued[j] && ready(j)) {
                    queued[j] = 1;
                    rq.push({rank[j], -j});
                }
        }
    }
    if ((int)order.size() != T) return;   // keep the level order
    std::vector<BatchTask> out(T);
    for (int q = 0; q < T; ++q) out[q] = tasks[order[q]];
    tasks.swap(out);
}

// XCD-local queues: every graph's tasks go to one of `nxcd` queues (one per
// XCD, so a graph's tiles are written and read through one L2), graphs
// assigned largest estimated work first to the least loaded queue; each
// queue is built in level order and list-scheduled on `workers_per_xcd`
// workgroups.  tasks receives the queues back to back, qoff[x] .. qoff[x+1]
// the tickets of queue x.  Counters are laid out per queue, each queue's
// block starting on a multiple of `counter_align` counters (graphs of
// different queues never share a cache line of counters).
inline void build_xcd_queues(const int32_t* widths, const int32_t* subs, int32_t count, const int32_t* h_sizes,
                             const std::vector<int32_t>& order, int nxcd, int workers_per_xcd, int counter_align,
                             const TaskCost& cost, std::vector<BatchTask>& tasks, std::vector<int32_t>& qoff,
                             int32_t& ncounters)
{
    nxcd = std::max(nxcd, 1);
    // estimated work of each graph: the sum of its tasks' durations
    std::vector<std::vector<int32_t>> members(nxcd);
    std::vector<double> load(nxcd, 0.0);
    for (int32_t q = 0; q < count; ++q) {   // order: largest first
        const int32_t g = order[q];
        std::vector<BatchTask> one;
        int32_t nc1 = 0;
        const std::vector<int32_t> solo{g};
        build_queue_plan(widths, subs, count, h_sizes, solo, one, nc1);
        double w = 0.0;
        for (const BatchTask& t : one) w += task_us(t, h_sizes, cost);
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += w;
        members[x].push_back(g);
    }
    tasks.clear();
    qoff.assign(nxcd + 1, 0);
    ncounters = 0;
    for (int x = 0; x < nxcd; ++x) {
        std::vector<BatchTask> part;
        int32_t nc = 0;
        build_queue_plan(widths, subs, count, h_sizes, members[x], part, nc);
        order_queue_plan(part, nc, workers_per_xcd, h_sizes, cost);
        for (BatchTask& t : part) {
            if (t.wait0 >= 0) t.wait0 += ncounters;
            if (t.wait1 >= 0) t.wait1 += ncounters;
            if (t.signal >= 0) t.signal += ncounters;
        }
        ncounters += (nc + counter_align - 1) / counter_align * counter_align;
        tasks.insert(tasks.end(), part.begin(), part.end());
        qoff[x + 1] = (int32_t)tasks.size();
    }
}

}  // namespace apsp
