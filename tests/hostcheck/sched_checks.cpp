// sched_checks.cpp -- the run server's admission policy and first-fit
// allocator (sched.hpp, the code the server runs) on a fake clock, built with
// g++ alone.  Prints one line per check; exit status 0 iff all pass.
//
//   heap      random alloc / release sequences against a brute-force model
//             of the arena in 256-byte units: the same offsets (lowest
//             fitting range), used bytes, and one free range once all is
//             released
//   serving   Poisson arrivals of runs of the served mix's sizes into an
//             arena smaller than the mix; every tick admits from the head of
//             the queue, advances each active run one step and retires the
//             finished ones: the arena never holds more than its size, live
//             ranges never overlap, runs are admitted in arrival order, a run
//             that arrives to an idle server with room waits no tick, every
//             run finishes, and the arena ends whole
//   quantile  percentile on known samples
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <random>
#include <vector>

#include "sched.hpp"

using namespace clgc;

static int g_fail = 0;

static void report(bool ok, const char* what)
{
    std::printf("%s %s\n", ok ? "ok" : "FAIL", what);
    if (!ok) ++g_fail;
}

// brute force: a map of 256-byte units, first fit by linear scan
struct Model {
    std::vector<char> used;
    explicit Model(size_t units) : used(units, 0) {}
    bool alloc(size_t n, size_t* off)
    {
        const size_t u = align256(n) / 256;
        for (size_t s = 0; s + u <= used.size(); ++s) {
            size_t k = 0;
            while (k < u && !used[s + k]) ++k;
            if (k == u) {
                for (size_t j = 0; j < u; ++j) used[s + j] = 1;
                *off = s * 256;
                return true;
            }
            s += k;  // skip past the used unit that stopped the run
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        for (size_t j = 0; j < align256(n) / 256; ++j) used[off / 256 + j] = 0;
    }
};

static void check_heap()
{
    std::mt19937_64 rng(11);
    bool ok = true;
    for (int trial = 0; trial < 50 && ok; ++trial) {
        const size_t units = 64 + rng() % 4000;
        Heap h;
        h.reset(units * 256);
        Model m(units);
        std::vector<std::pair<size_t, size_t>> live;
        for (int op = 0; op < 2000 && ok; ++op) {
            if (live.empty() || rng() % 3) {
                const size_t n = 1 + rng() % (units * 256 / 8);
                size_t a = 0, b = 0;
                const bool fa = h.alloc(n, &a), fb = m.alloc(n, &b);
                ok = fa == fb && (!fa || a == b);
                if (fa) live.push_back({a, n});
            } else {
                const size_t i = rng() % live.size();
                h.release(live[i].first, live[i].second);
                m.release(live[i].first, live[i].second);
                live.erase(live.begin() + (long)i);
            }
            size_t used = 0;
            for (auto& l : live) used += align256(l.second);
            ok = ok && h.used() == used;
        }
        for (auto& l : live) h.release(l.first, l.second);
        ok = ok && h.used() == 0 && h.free_ranges() == 1;
    }
    report(ok, "heap: first fit equals the brute-force model, frees coalesce");
}

struct FakeRun {
    int id;
    size_t bytes;
    int group, steps, done = 0;
    long t_submit = 0, t_admit = -1, t_finish = -1;
    size_t off = 0;
};

static void check_serving(double rate, size_t budget, int n_runs, unsigned seed, bool overload, const char* what)
{
    // footprints of the served shapes (links, drift, clover and scratch of
    // 6^4, 8^4, 12^4, 16^4, 8^3x16, 24^3x8 in FP64; mixed about half)
    const size_t sizes[] = {2613248, 8257536, 41801728, 132122624, 16515072, 222937088};
    std::mt19937_64 rng(seed);
    std::exponential_distribution<double> gap(rate);
    std::vector<FakeRun> runs(n_runs);
    double t = 0;
    for (int i = 0; i < n_runs; ++i) {
        t += gap(rng);
        runs[i].id = i;
        runs[i].group = (int)(rng() % 2);
        runs[i].bytes = sizes[rng() % 6] / (runs[i].group ? 2 : 1);
        runs[i].steps = 50 + (int)(rng() % 451);
        runs[i].t_submit = (long)std::ceil(t);
    }
    Heap heap;
    heap.reset(budget);
    std::deque<FakeRun*> pending;
    std::vector<FakeRun*> active;
    std::vector<int> admitted;
    int next = 0, finished = 0, groups[2] = {0, 0};
    size_t max_pending = 0;
    bool ok = true;
    for (long now = 0; finished < n_runs && now < 10000000; ++now) {
        while (next < n_runs && runs[next].t_submit <= now) pending.push_back(&runs[next++]);
        while (!pending.empty()) {  // the server's admission loop
            FakeRun* r = pending.front();
            size_t off = 0;
            if (!admit_head(heap, r->bytes, groups[r->group], 256, &off)) break;
            r->off = off;
            r->t_admit = now;
            groups[r->group]++;
            active.push_back(r);
            admitted.push_back(r->id);
            pending.pop_front();
        }
        max_pending = std::max(max_pending, pending.size());
        // invariants of the arena
        size_t used = 0;
        for (FakeRun* r : active) {
            used += align256(r->bytes);
            ok = ok && r->off + align256(r->bytes) <= budget;
            for (FakeRun* q : active)
                if (q != r) ok = ok && (q->off + align256(q->bytes) <= r->off || r->off + align256(r->bytes) <= q->off);
        }
        ok = ok && used == heap.used() && used <= budget;
        // one batch step: every active run advances; finished runs retire
        for (size_t i = 0; i < active.size();) {
            FakeRun* r = active[i];
            if (++r->done >= r->steps) {
                r->t_finish = now;
                heap.release(r->off, r->bytes);
                groups[r->group]--;
                active.erase(active.begin() + (long)i);
                ++finished;
            } else {
                ++i;
            }
        }
    }
    ok = ok && finished == n_runs && heap.used() == 0 && heap.free_ranges() == 1;
    for (int i = 0; i < (int)admitted.size(); ++i) ok = ok && admitted[i] == i;  // arrival order
    // a run arriving when nothing waits and the arena has room is admitted at once
    int immediate = 0;
    for (auto& r : runs) immediate += r.t_admit == r.t_submit;
    ok = ok && immediate > 0;
    // over capacity the queue must build (admission is what holds runs back)
    ok = ok && (overload ? max_pending >= 20 : true);
    std::vector<float> waits;
    for (auto& r : runs) waits.push_back((float)(r.t_admit - r.t_submit));
    char line[200];
    std::snprintf(line, sizeof line, "%s (%d runs, wait p50 %.0f p99 %.0f ticks, queue up to %zu)", what, n_runs,
                  percentile(waits, 0.5), percentile(waits, 0.99), max_pending);
    report(ok, line);
}

static void check_quantiles()
{
    const std::vector<float> v = {5, 1, 4, 2, 3};
    bool ok = percentile(v, 0.5) == 3.0 && percentile(v, 0.0) == 1.0 && percentile(v, 1.0) == 5.0;
    ok = ok && std::fabs(percentile(v, 0.99) - 4.96) < 1e-6 && percentile({}, 0.5) == 0.0;
    report(ok, "percentiles interpolate between order statistics");
}

int main()
{
    check_heap();
    check_serving(1.0 / 400.0, size_t(2) << 30, 256, 5, false, "serving below capacity: FIFO, arena invariants");
    check_serving(1.0 / 4.0, size_t(1) << 30, 256, 6, true, "serving over capacity: queue builds, FIFO, arena invariants");
    check_quantiles();
    std::printf("%s: %d failed\n", g_fail ? "FAIL" : "PASS", g_fail);
    return g_fail ? 1 : 0;
}
