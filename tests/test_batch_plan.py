"""The dependency-driven batched schedule's task list, checked on the host
(no GPU).  A small C++ driver builds the plan with the library's own
planner (csrc/batch_plan.h) and prints it; the test then checks that

* it is a topological order: every counter a task waits for reaches its
  target through tasks with smaller tickets (so the queue always drains),
  and no target exceeds the number of tasks that signal that counter;
* it is race-free: under random interleavings of tasks whose waits are
  met, a task never starts before every earlier task it conflicts with (one
  of the two writes a tile the other reads or writes) has finished, so
  every such run is equivalent to running the tasks one by one in ticket
  order;
* it computes APSP: executing the tasks in such interleavings (closures by
  the oracle's triple loop on the block, products by the oracle's min-plus
  product, Sec. 2 Eq. 1 and Sec. 3 Eq. 2) yields the oracle's Floyd-Warshall
  result for every graph.
"""
import os
import subprocess
import textwrap

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_03983_amd", "csrc")
INF = 1 << 30

DRIVER = textwrap.dedent(r"""
    #include <cstdio>
    #include <cstdlib>
    #include <numeric>
    #include "batch_plan.h"
    int main(int argc, char** argv) {
        const int B = std::atoi(argv[1]);         // round width of graphs with n > split
        const int split = std::atoi(argv[2]);     // graphs with n <= split use width 2 B
        const int workers = std::atoi(argv[3]);   // 0: level order as built
        const int nxcd = std::atoi(argv[4]);      // > 0: one queue per XCD (workers per XCD)
        const int sub = std::atoi(argv[5]);       // sub-tile size of the products of graphs with n > split (0: none)
        std::vector<int32_t> n;
        for (int i = 6; i < argc; ++i) n.push_back(std::atoi(argv[i]));
        std::vector<int32_t> widths, subs;
        for (int32_t x : n) {
            widths.push_back(x > split ? B : 2 * B);
            subs.push_back(x > split ? sub : 0);
        }
        std::vector<int32_t> order(n.size());
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return n[a] > n[b]; });
        std::vector<apsp::BatchTask> t;
        int32_t nc = 0;
        std::vector<int32_t> qoff{0};
        if (nxcd > 0) {
            apsp::build_xcd_queues(widths.data(), subs.data(), (int32_t)n.size(), n.data(), order, nxcd,
                                   std::max(workers, 1), 64,
                                   apsp::TaskCost{}, t, qoff, nc);
        } else {
            apsp::build_queue_plan(widths.data(), subs.data(), (int32_t)n.size(), n.data(), order, t, nc);
            if (workers > 0) apsp::order_queue_plan(t, nc, workers, n.data(), apsp::TaskCost{});
            qoff.push_back((int32_t)t.size());
        }
        std::printf("%d %zu\n", nc, t.size());
        for (int32_t v : qoff) std::printf("%d ", v);
        std::printf("\n");
        for (const auto& x : t)
            std::printf("%d %d %d %d %d %d %d %d %d %d %d %d\n", x.kind, x.graph, x.round, x.a, x.b, x.wait0, x.need0,
                        x.wait1, x.need1, x.signal, x.width, x.sub);
        return 0;
    }
""")

CLOSE, FUSED, ROW, COL, REM = range(5)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("plan")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = str(d / "driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", exe], check=True)
    return exe


def plan(driver, B, sizes, workers=0, split=-1, nxcd=0, queues=False, sub=0):
    """Tasks of a batch: graphs with n > split use round width B (products in
    sub x sub sub-tiles when sub > 0), the others 2 B; nxcd > 0 splits them
    into that many queues (returned with queues)."""
    out = subprocess.run([driver, str(B), str(split), str(workers), str(nxcd), str(sub), *map(str, sizes)],
                         check=True, capture_output=True, text=True).stdout
    lines = out.strip().splitlines()
    nc, nt = map(int, lines[0].split())
    qoff = list(map(int, lines[1].split()))
    tasks = [tuple(map(int, l.split())) for l in lines[2:]]
    assert len(tasks) == nt and qoff[-1] == nt
    return (nc, tasks, qoff) if queues else (nc, tasks)


def tiles(task, B, n):
    """(reads, writes) of a task as sets of (graph, row block, column block)
    of its graph, in blocks of min(round width, 64), so whole tiles and
    64 x 64 sub-tiles compare."""
    kind, g, r, a, b = task[:5]
    W, sub = task[10], task[11]
    n = SIZES_OF[g]

    U = min(W, 64)   # block unit: whole tiles and 64 x 64 sub-tiles both align to it

    def blocks(i, j, part=None, rows=None, cols=None):
        """U-blocks of tile (i, j) (restricted to the 64-row / 64-column
        sub-range `rows` / `cols` of the tile)."""
        r0, r1 = i * W, min(n, (i + 1) * W)
        c0, c1 = j * W, min(n, (j + 1) * W)
        if rows is not None:
            r0, r1 = r0 + 64 * rows, min(r1, r0 + 64 * (rows + 1))
        if cols is not None:
            c0, c1 = c0 + 64 * cols, min(c1, c0 + 64 * (cols + 1))
        return {(g, x, y) for x in range(r0 // U, (r1 + U - 1) // U) for y in range(c0 // U, (c1 + U - 1) // U)}

    si, sj = (None, None) if sub < 0 else (sub & 0xff, sub >> 8)
    if kind == CLOSE:
        return blocks(a, a), blocks(a, a)
    if kind == FUSED:
        return blocks(a, r) | blocks(r, a) | blocks(a, a), blocks(a, a)
    if kind == ROW:   # rows si of X*, columns sj of the panel tile (every row), writes (si, sj)
        return blocks(r, r, rows=si) | blocks(r, a, cols=sj), blocks(r, a, rows=si, cols=sj)
    if kind == COL:
        return blocks(a, r, rows=si) | blocks(r, r, cols=sj), blocks(a, r, rows=si, cols=sj)
    return blocks(a, r, rows=si) | blocks(r, b, cols=sj) | blocks(a, b, rows=si, cols=sj), \
        blocks(a, b, rows=si, cols=sj)


SIZES_OF = {}


def benign(t1, t2):
    """Sub-tiles of one in-place panel tile read what the others rewrite: the
    pivot block is closed, so any mix of old and new values gives the same
    result (checked by the results of the random interleavings)."""
    return t1[0] in (ROW, COL) and t1[:5] == t2[:5] and t1[11] >= 0


def check_topological(nc, tasks):
    signalers = [[] for _ in range(nc)]
    for q, t in enumerate(tasks):
        if t[9] >= 0:
            signalers[t[9]].append(q)
    for q, t in enumerate(tasks):
        for w, need in ((t[5], t[6]), (t[7], t[8])):
            if w < 0:
                continue
            assert need <= len(signalers[w]), f"task {q} waits for {need} of {len(signalers[w])}"
            assert sum(1 for s in signalers[w] if s < q) >= need, f"task {q} waits on later tickets"


def run(oracle, nc, tasks, mats, B, seed, slots=12):
    """Executes the tasks in a random interleaving allowed by the counters;
    a task reads its inputs when it starts and writes when it finishes."""
    rng = np.random.default_rng(seed)
    D = [m.copy() for m in mats]
    SIZES_OF.clear()
    SIZES_OF.update({g: m.shape[0] for g, m in enumerate(mats)})
    cnt = [0] * nc
    nxt, running, done = 0, [], 0
    finished = set()

    width = {}
    for t in tasks:
        width[t[1]] = t[10]

    def blk(g, i, j):
        n = D[g].shape[0]
        W = width[g]
        return slice(i * W, min(n, (i + 1) * W)), slice(j * W, min(n, (j + 1) * W))

    def ready(t):
        return all(w < 0 or cnt[w] >= need for w, need in ((t[5], t[6]), (t[7], t[8])))

    def sub_of(t):
        return (None, None) if t[11] < 0 else (t[11] & 0xff, t[11] >> 8)

    def part(sl, k):
        """Rows (or columns) k*64 .. of a tile slice (all of them when k is None)."""
        if k is None:
            return sl
        return slice(sl.start + 64 * k, min(sl.stop, sl.start + 64 * (k + 1)))

    def compute(t):
        kind, g, r, a, b = t[:5]
        M = D[g]
        si, sj = sub_of(t)
        if kind == CLOSE:
            rs = blk(g, a, a)
            return {(g, a, a, None, None): oracle.fw_i32(M[rs])}
        if kind == FUSED:
            X = oracle.minplus_i32(M[blk(g, a, r)], M[blk(g, r, a)], M[blk(g, a, a)])
            return {(g, a, a, None, None): oracle.fw_i32(X)}
        if kind == ROW:
            (pr, pc), (tr, tc) = blk(g, r, r), blk(g, r, a)
            X = M[part(pr, si), pc]
            Rt = M[tr, part(tc, sj)]
            Cc = M[part(tr, si), part(tc, sj)]
            return {(g, r, a, si, sj): oracle.minplus_i32(X, Rt, Cc)}
        if kind == COL:
            (tr, tc), (pr, pc) = blk(g, a, r), blk(g, r, r)
            Ct = M[part(tr, si), tc]
            X = M[pr, part(pc, sj)]
            Cc = M[part(tr, si), part(tc, sj)]
            return {(g, a, r, si, sj): oracle.minplus_i32(Ct, X, Cc)}
        (ar, ac), (br, bc), (cr, cc) = blk(g, a, r), blk(g, r, b), blk(g, a, b)
        return {(g, a, b, si, sj): oracle.minplus_i32(M[part(ar, si), ac], M[br, part(bc, sj)],
                                                      M[part(cr, si), part(cc, sj)])}

    while done < len(tasks):
        # tickets are taken in order; a task starts once its waits are met
        can_take = nxt < len(tasks) and len(running) < slots
        if can_take and (not running or rng.random() < 0.6):
            running.append([nxt, None])
            nxt += 1
            continue
        # advance a running task -- usually the latest ticket, so later tasks
        # race ahead of earlier ones -- by starting it (if ready) or finishing it
        k = len(running) - 1 if rng.random() < 0.7 else int(rng.integers(len(running)))
        q, res = running[k]
        t = tasks[q]
        if res is None:
            if not ready(t):
                if all(r_[1] is None and not ready(tasks[r_[0]]) for r_ in running) and nxt >= len(tasks):
                    raise AssertionError("no running task can make progress")
                continue
            reads, writes = tiles(t, B, None)
            # every earlier task that touches what this one reads or writes
            # (a write on either side) has finished: the run is equivalent to
            # executing the tasks one by one in ticket order
            for p_ in range(q):
                if p_ in finished or benign(t, tasks[p_]):
                    continue
                r2, w2 = tiles(tasks[p_], B, None)
                assert not (w2 & (reads | writes)) and not (writes & r2), \
                    f"task {q} starts before task {p_}, which it conflicts with, has finished"
            running[k][1] = compute(t)
        else:
            for (g, i, j, si, sj), val in res.items():
                rs, cs = blk(g, i, j)
                D[g][part(rs, si), part(cs, sj)] = val
            if t[9] >= 0:
                cnt[t[9]] += 1
            finished.add(q)
            running.pop(k)
            done += 1
    return D


def rand_graph(rng, n, p):
    W = np.where(rng.random((n, n)) < p, rng.integers(1, 100, (n, n)), INF).astype(np.int32)
    np.fill_diagonal(W, 0)
    return W


@pytest.mark.parametrize("B,sizes", [
    (4, [1, 2, 3, 4, 5, 8, 9, 12, 13, 17, 0, 6]),
    (4, [16, 15, 3, 11, 7, 1, 14, 10]),
    (8, [33, 8, 17, 24, 25, 40, 1, 9]),
    (128, [129, 300, 40, 512, 256, 385, 1, 0, 128]),
])
@pytest.mark.parametrize("workers", [0, 3, 512])
@pytest.mark.parametrize("split", [-1, 9])
@pytest.mark.parametrize("sub", [0, 64])
def test_queue_plan(oracle, driver, B, sizes, workers, split, sub):
    """Level order as built (workers = 0) and the list-scheduled order the
    library uses (on 3 and on 512 simulated workgroups); one round width for
    every graph, or width 2 B for graphs with n <= split; whole-tile products
    or 64 x 64 sub-tile tasks (128-wide rounds only)."""
    if sub and B != 128:
        pytest.skip("sub-tiles are cut from 128-wide tiles")
    nc, tasks = plan(driver, B, sizes, workers, split, sub=sub)
    if workers:
        assert sorted(tasks) == sorted(plan(driver, B, sizes, 0, split, sub=sub)[1])   # the same tasks, reordered
    check_topological(nc, tasks)
    rng = np.random.default_rng(sum(sizes) + B)
    mats = [rand_graph(rng, n, min(0.5, 3.0 / max(n, 1))) for n in sizes]
    refs = [oracle.fw_i32(W) for W in mats]
    for seed in range(3 if B == 128 else 8):
        out = run(oracle, nc, tasks, mats, B, seed)
        for n, got, ref in zip(sizes, out, refs):
            np.testing.assert_array_equal(got, ref, err_msg=f"n={n} seed={seed}")


def test_queue_plan_counts(driver):
    # the 128-wide plan of graphs with 1..4 rounds: 1, 7, 25 and 61 tasks
    for n, want in ((100, 1), (200, 7), (300, 25), (500, 61)):
        _, tasks = plan(driver, 128, [n])
        assert len(tasks) == want, (n, len(tasks))
        assert all(t[10] == 128 for t in tasks)
    _, tasks = plan(driver, 64, [500, 100], split=128)   # 500 in 64-wide rounds (8), 100 in one 128 block
    assert sum(1 for t in tasks if t[1] == 0) == 1 + 8 * (8 * 8 - 1) and all(t[10] == 64 for t in tasks if t[1] == 0)


@pytest.mark.parametrize("nxcd", [1, 3, 8])
def test_xcd_queues(oracle, driver, nxcd):
    """One queue per XCD: every graph's tasks in one queue, each queue
    topological on its own (a task waits only for counters its own queue
    signals, through smaller tickets), counter blocks of different queues
    disjoint and 64-aligned; queues run interleaved in any way give the
    oracle's distances."""
    sizes = [129, 300, 40, 512, 256, 385, 1, 0, 128, 77, 200, 260]
    nc, tasks, qoff = plan(driver, 128, sizes, workers=4, nxcd=nxcd, queues=True)
    assert sorted(t[:5] + t[10:] for t in tasks) == sorted(t[:5] + t[10:] for t in plan(driver, 128, sizes)[1])
    owner = {}
    for x in range(nxcd):
        part = tasks[qoff[x]:qoff[x + 1]]
        graphs = {t[1] for t in part}
        for g in graphs:
            assert owner.setdefault(g, x) == x, f"graph {g} in two queues"
        cnts = {c for t in part for c in (t[5], t[7], t[9]) if c >= 0}
        for c in cnts:
            assert owner.setdefault(("c", c // 64), x) == x, f"counter block {c // 64} shared by queues"
        check_topological(nc, part)
    # every queue's tickets in order; queues interleaved at random
    rng = np.random.default_rng(nxcd)
    mats = [rand_graph(rng, n, min(0.5, 3.0 / max(n, 1))) for n in sizes]
    refs = [oracle.fw_i32(W) for W in mats]
    merged = []
    pos = [qoff[x] for x in range(nxcd)]
    while any(pos[x] < qoff[x + 1] for x in range(nxcd)):
        x = int(rng.choice([x for x in range(nxcd) if pos[x] < qoff[x + 1]]))
        merged.append(tasks[pos[x]])
        pos[x] += 1
    out = run(oracle, nc, merged, mats, 128, 1)
    for n, got, ref in zip(sizes, out, refs):
        np.testing.assert_array_equal(got, ref, err_msg=f"n={n}")
