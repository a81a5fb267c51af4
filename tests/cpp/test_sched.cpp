// Host unit test of the serving scheduler (admission by footprint, continuous
// batching of row chunks).  Built with g++ by tests/test_sched_cpu.py.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "../../paper_2105_08722_amd/csrc/sched.h"

using namespace encore;

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);          \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static SchedJob mk(int64_t id, size_t fp, uint64_t cls, int64_t rows, int64_t split)
{
    SchedJob j;
    j.id = id; j.footprint = fp; j.cls = cls; j.nrows = rows; j.split_rows = split;
    return j;
}

static void test_admission_fifo()
{
    Scheduler s(100, 8);
    SchedJob a = mk(1, 60, 0, 10, 4), b = mk(2, 50, 0, 10, 4), c = mk(3, 30, 0, 10, 4), d = mk(4, 120, 0, 10, 4);
    CHECK(s.submit(&a));
    CHECK(s.submit(&b));
    CHECK(s.submit(&c));
    CHECK(!s.submit(&d));              // larger than the whole budget
    auto adm = s.admit();
    CHECK(adm.size() == 1 && adm[0] == &a);   // b does not fit; c waits behind b
    CHECK(s.used() == 60);
    CHECK(s.admit().empty());
    s.ready(&a);
    s.finish(&a, true);
    CHECK(s.used() == 0 && a.state == SchedJob::DONE);
    adm = s.admit();
    CHECK(adm.size() == 2 && adm[0] == &b && adm[1] == &c);
    CHECK(s.used() == 80 && s.peak() == 80);
}

static void test_max_active()
{
    Scheduler s(1000, 2);
    SchedJob j[4] = {mk(1, 1, 0, 5, 1), mk(2, 1, 0, 5, 1), mk(3, 1, 0, 5, 1), mk(4, 1, 0, 5, 1)};
    for (auto& x : j) CHECK(s.submit(&x));
    CHECK(s.admit().size() == 2);
    CHECK(s.queued() == 2);
}

static void test_pick_classes_and_splits()
{
    Scheduler s(1000, 8);
    SchedJob a = mk(1, 1, 7, 100, 16), b = mk(2, 1, 9, 50, 8), c = mk(3, 1, 7, 30, 4);
    for (SchedJob* x : {&a, &b, &c}) CHECK(s.submit(x));
    for (SchedJob* x : s.admit()) s.ready(x);
    // slice of 40 rows: oldest job a (class 7), then c of the same class; b waits
    auto p = s.pick(40);
    CHECK(p.size() == 2);
    CHECK(p[0].job == &a && p[0].r0 == 0 && p[0].r1 == 32);   // whole splits of 16
    CHECK(p[1].job == &c && p[1].r0 == 0 && p[1].r1 == 8);    // 8 rows left, splits of 4
    // next pick while those run: only b is idle
    auto q = s.pick(40);
    CHECK(q.size() == 1 && q[0].job == &b && q[0].r0 == 0 && q[0].r1 == 40);
    CHECK(s.pick(40).empty());
    CHECK(s.slice_done(p).empty());
    auto r = s.pick(1000);
    CHECK(r.size() == 2 && r[0].job == &a && r[0].r0 == 32 && r[0].r1 == 100 && r[1].job == &c &&
          r[1].r0 == 8 && r[1].r1 == 30);
    auto done = s.slice_done(r);
    CHECK(done.size() == 2);
    // a split longer than the slice still progresses as the first chunk
    Scheduler t(1000, 8);
    SchedJob big = mk(1, 1, 0, 100, 64);
    CHECK(t.submit(&big));
    for (SchedJob* x : t.admit()) t.ready(x);
    auto u = t.pick(10);
    CHECK(u.size() == 1 && u[0].r0 == 0 && u[0].r1 == 64);
}

// Random arrivals, lanes and completions: every job's rows are covered once, in
// order, in whole splits, never two chunks of one job at once, and the budget holds.
static void test_random_simulation()
{
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 200; ++trial) {
        const size_t budget = 200 + rng() % 800;
        Scheduler s(budget, 1 + (int)(rng() % 6));
        const int njobs = 1 + (int)(rng() % 40);
        std::vector<SchedJob> jobs(njobs);
        std::vector<int64_t> covered(njobs, 0);
        for (int i = 0; i < njobs; ++i)
            jobs[i] = mk(i, 1 + rng() % budget, rng() % 3, 1 + (int64_t)(rng() % 500), 1 + (int64_t)(rng() % 64));
        int submitted = 0, finished = 0;
        const int nlanes = 1 + (int)(rng() % 3);
        std::vector<std::vector<SchedChunk>> lane(nlanes);
        std::map<const SchedJob*, int> inflight;
        int guard = 0;
        while (finished < njobs && ++guard < 100000) {
            if (submitted < njobs && rng() % 3 == 0) {
                CHECK(s.submit(&jobs[submitted]));
                ++submitted;
            }
            for (SchedJob* x : s.admit()) s.ready(x);
            CHECK(s.used() <= budget);
            const int l = (int)(rng() % nlanes);
            if (lane[l].empty()) {
                const int64_t slice = 1 + (int64_t)(rng() % 300);
                lane[l] = s.pick(slice);
                int64_t rows = 0;
                uint64_t cls = lane[l].empty() ? 0 : lane[l][0].job->cls;
                for (const SchedChunk& c : lane[l]) {
                    const int i = (int)c.job->id;
                    CHECK(c.job->cls == cls);
                    CHECK(c.r0 == covered[i]);                      // in order, no gap, no overlap
                    CHECK(c.r0 % c.job->split_rows == 0);            // whole splits
                    CHECK(c.r1 > c.r0 && c.r1 <= c.job->nrows);
                    CHECK(inflight[c.job]++ == 0);                   // one chunk per job in flight
                    covered[i] = c.r1;
                    rows += c.r1 - c.r0;
                }
                if (lane[l].size() > 1) CHECK(rows <= slice);
            } else {
                for (const SchedChunk& c : lane[l]) inflight[c.job]--;
                for (SchedJob* x : s.slice_done(lane[l])) {
                    s.finish(x, true);
                    ++finished;
                }
                lane[l].clear();
            }
        }
        CHECK(finished == njobs);
        for (int i = 0; i < njobs; ++i) CHECK(covered[i] == jobs[i].nrows);
        CHECK(s.used() == 0 && s.active() == 0 && s.queued() == 0);
    }
}

int main()
{
    test_admission_fifo();
    test_max_active();
    test_pick_classes_and_splits();
    test_random_simulation();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("sched: all passed\n");
    return 0;
}
