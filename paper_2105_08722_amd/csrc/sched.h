// Scheduling policy of the serving loop: admission by device-memory footprint
// and iteration-level (continuous) batching of primary-row chunks.  Pure C++,
// no HIP: the server drives it under its lock, and a host unit test drives it
// with fake jobs.
//
// Policy
//  * Admission: jobs wait in arrival order; the head is admitted while its
//    footprint fits in what the budget leaves and fewer than max_active jobs are
//    admitted.  A job whose footprint alone exceeds the budget is refused at
//    submit.  (Strict arrival order: a large job at the head is never starved by
//    smaller ones behind it.)
//  * Batching: an iteration ("slice") takes the oldest admitted job that is not
//    running and still has rows, then adds, oldest first, every other idle job
//    of the same class (same kernels and tables) until slice_rows rows.  A job
//    contributes whole coupling splits (rows r0..r1 with r0 a multiple of its
//    split length), and is never in two slices at once, so its rows are reduced
//    in order and its result does not depend on the mix.
//  * Jobs arriving while slices run are admitted at the next iteration.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

namespace encore {

struct SchedJob {
    int64_t id = 0;
    size_t footprint = 0;    // device bytes held from admission to completion
    uint64_t cls = 0;        // jobs of one class can share a slice
    int64_t nrows = 0;       // primaries
    int64_t split_rows = 1;  // coupling split length (> 0)
    // state
    enum State { QUEUED, ADMITTED, READY, DONE, FAILED } state = QUEUED;
    int64_t next_row = 0;    // rows [0, next_row) done or in flight
    bool busy = false;       // in a running slice (or being set up)
    uint64_t order = 0;      // arrival order
    void* user = nullptr;    // the caller's job record
};

struct SchedChunk {
    SchedJob* job;
    int64_t r0, r1;
};

class Scheduler {
public:
    Scheduler(size_t budget, int max_active) : budget_(budget), max_active_(max_active) {}

    size_t budget() const { return budget_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t queued() const { return queue_.size(); }
    size_t active() const { return active_.size(); }

    // false: the job can never fit (footprint > budget)
    bool submit(SchedJob* j)
    {
        if (j->footprint > budget_) return false;
        j->state = SchedJob::QUEUED;
        j->order = next_order_++;
        queue_.push_back(j);
        return true;
    }

    // Admits from the head of the queue; returns the newly admitted jobs
    // (state ADMITTED, busy: the caller sets them up and calls ready()).
    std::vector<SchedJob*> admit()
    {
        std::vector<SchedJob*> out;
        while (!queue_.empty() && (int)active_.size() < max_active_ &&
               used_ + queue_.front()->footprint <= budget_) {
            SchedJob* j = queue_.front();
            queue_.pop_front();
            used_ += j->footprint;
            peak_ = std::max(peak_, used_);
            j->state = SchedJob::ADMITTED;
            j->busy = true;
            active_.push_back(j);
            out.push_back(j);
        }
        return out;
    }

    // set-up of an admitted job finished
    void ready(SchedJob* j)
    {
        j->state = SchedJob::READY;
        j->busy = false;
    }

    // Next slice: chunks of idle READY jobs of one class (see the policy above).
    // Empty when no job has rows to run.
    std::vector<SchedChunk> pick(int64_t slice_rows, size_t max_chunks = 4096)
    {
        std::vector<SchedChunk> out;
        SchedJob* first = nullptr;
        for (SchedJob* j : active_)
            if (runnable(j) && (!first || j->order < first->order)) first = j;
        if (!first) return out;
        std::vector<SchedJob*> same;
        for (SchedJob* j : active_)
            if (runnable(j) && j->cls == first->cls) same.push_back(j);
        std::sort(same.begin(), same.end(), [](const SchedJob* a, const SchedJob* b) { return a->order < b->order; });
        int64_t rows = 0;
        for (SchedJob* j : same) {
            if (rows >= slice_rows || out.size() >= max_chunks) break;
            int64_t take = j->nrows - j->next_row;
            if (take > slice_rows - rows) {
                take = (slice_rows - rows) / j->split_rows * j->split_rows;
                // the first chunk of a slice always makes progress
                if (take == 0 && out.empty()) take = std::min(j->split_rows, j->nrows - j->next_row);
            }
            if (take <= 0) continue;
            out.push_back(SchedChunk{j, j->next_row, j->next_row + take});
            j->next_row += take;
            j->busy = true;
            rows += take;
        }
        return out;
    }

    // A slice finished; returns the jobs whose every row is now done (they stay
    // busy until finish()).
    std::vector<SchedJob*> slice_done(const std::vector<SchedChunk>& chunks)
    {
        std::vector<SchedJob*> complete;
        for (const SchedChunk& c : chunks) {
            if (c.job->next_row >= c.job->nrows) complete.push_back(c.job);
            else c.job->busy = false;
        }
        return complete;
    }

    // Job done (or failed): releases its footprint.
    void finish(SchedJob* j, bool ok)
    {
        auto it = std::find(active_.begin(), active_.end(), j);
        if (it != active_.end()) {
            active_.erase(it);
            used_ -= j->footprint;
        } else {
            auto q = std::find(queue_.begin(), queue_.end(), j);
            if (q != queue_.end()) queue_.erase(q);
        }
        j->busy = false;
        j->state = ok ? SchedJob::DONE : SchedJob::FAILED;
    }

private:
    static bool runnable(const SchedJob* j)
    {
        return j->state == SchedJob::READY && !j->busy && j->next_row < j->nrows;
    }

    size_t budget_;
    int max_active_;
    size_t used_ = 0, peak_ = 0;
    uint64_t next_order_ = 0;
    std::deque<SchedJob*> queue_;
    std::vector<SchedJob*> active_;
};

}  // namespace encore
