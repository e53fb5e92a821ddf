// serve_core.hpp - host side of the transcoding server: request admission, the
// device memory pool, batch formation and latency statistics. No HIP here: the
// device work sits behind the Executor interface, so the same scheduler runs
// with the HIP executor (hiputf.hip) or with a fake one on a virtual clock.
//
// Continuous batching. Requests queue in arrival order. Whenever an executor
// slot (one in-flight batch: a stream and its staging memory) is free, the
// scheduler takes requests from the head of the queue, as many as fit the
// batch limits, the in-flight request limit and the largest free range of the
// device pool, and launches them as one batch. Batches already on the device
// keep running meanwhile, so requests that arrive while others are being
// processed join the next batch instead of waiting for a queue to drain.
// Admission is strictly first come, first served: a request at the head that
// does not fit yet waits for memory to be freed and no later request passes
// it, so none starves.
//
// A batch occupies one contiguous pool range laid out as
//   [documents table | inputs | outputs | results]
// (each request's input and output 16-byte aligned), the same layout as its
// pinned staging buffer, so one host-to-device copy carries the table and the
// inputs and one device-to-host copy brings back outputs and results.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <deque>
#include <vector>

#include "hiputf.h"

namespace hu {
namespace serve {

constexpr uint64_t kAlign = 16;
constexpr uint64_t kRegionAlign = 256;

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

inline bool op_valid(uint32_t op) { return op <= HU_OP_CONVERT_UTF16LE_TO_UTF8; }
inline uint64_t in_unit(uint32_t op) { return op >= HU_OP_VALIDATE_UTF16LE ? 2 : 1; }
inline bool op_converts(uint32_t op)
{
    return op == HU_OP_CONVERT_UTF8_TO_UTF16LE || op == HU_OP_CONVERT_UTF16LE_TO_UTF8;
}
inline uint64_t out_unit(uint32_t op) { return op == HU_OP_CONVERT_UTF8_TO_UTF16LE ? 2 : 1; }

// Largest output of a request in code units: one UTF-16 word per UTF-8 byte;
// three UTF-8 bytes per UTF-16 word.
inline uint64_t worst_out_units(uint32_t op, uint64_t n_units)
{
    if (op == HU_OP_CONVERT_UTF8_TO_UTF16LE)
        return n_units;
    if (op == HU_OP_CONVERT_UTF16LE_TO_UTF8)
        return 3 * n_units;
    return 0;
}

struct Request {
    // from the caller
    uint64_t tag = 0;
    uint32_t op = 0;
    const void *src = nullptr;
    uint64_t n_units = 0;
    void *dst = nullptr;          // may be null: the output is not copied out
    uint64_t dst_cap = 0;         // output capacity in code units
    int64_t t_arrive = 0;         // ns
    void *user = nullptr;         // owner's bookkeeping, untouched here
    // set by the scheduler
    uint64_t in_bytes = 0;        // input bytes
    uint64_t dev_cap = 0;         // output capacity given to the device, in code units
    uint64_t in_off = 0;          // offsets inside the batch region
    uint64_t out_off = 0;
    hu_result result{};
    bool rejected = false;        // could never run; completed without device work
    int64_t t_done = 0;

    uint64_t out_bytes() const { return dev_cap * out_unit(op); }
};

// Region layout of a batch: documents table, inputs, outputs, results.
struct Layout {
    uint64_t in_begin = 0, out_begin = 0, results_off = 0, bytes = 0;
};

inline uint64_t docs_bytes(uint64_t n) { return align_up(n * sizeof(hu_doc), kRegionAlign); }

// Region bytes for n requests with the given input and output byte sums
// (each already rounded to kAlign).
inline uint64_t region_bytes(uint64_t n, uint64_t in_sum, uint64_t out_sum)
{
    return align_up(docs_bytes(n) + in_sum + out_sum + n * sizeof(hu_result), kRegionAlign);
}

struct Batch {
    int slot = -1;
    std::vector<Request *> reqs;
    Layout lay;
    uint64_t pool_off = 0;
    int64_t t_launch = 0;
    int64_t device_ns = 0;        // filled by the executor on completion, when it measures it
};

// Assigns every request its offsets and returns the layout.
inline Layout lay_out(Batch &b)
{
    Layout l;
    l.in_begin = docs_bytes(b.reqs.size());
    uint64_t p = l.in_begin;
    for (Request *r : b.reqs) {
        r->in_off = p;
        p += align_up(r->in_bytes, kAlign);
    }
    l.out_begin = p;
    for (Request *r : b.reqs) {
        r->out_off = p;
        p += align_up(r->out_bytes(), kAlign);
    }
    l.results_off = p;
    p += b.reqs.size() * sizeof(hu_result);
    l.bytes = align_up(p, kRegionAlign);
    return l;
}

// Device memory pool as a ring of batch ranges. Ranges are taken at the head
// and given back in any order; the tail advances over given-back ranges.
class RingPool {
public:
    explicit RingPool(uint64_t cap) : cap_(cap) {}

    uint64_t capacity() const { return cap_; }
    uint64_t used() const { return used_; }

    // Largest range reserve() can hand out now.
    uint64_t largest_free() const
    {
        if (live_.empty())
            return cap_;
        const uint64_t front = live_.front().off, end = live_.back().off + live_.back().bytes;
        if (live_.back().off >= front)        // not wrapped: space after the head and before the tail
            return std::max(cap_ - end, front);
        return front - end;
    }

    bool reserve(uint64_t bytes, uint64_t *off)
    {
        if (bytes == 0 || bytes > cap_)
            return false;
        uint64_t at;
        if (live_.empty()) {
            at = 0;
        } else {
            const uint64_t front = live_.front().off, end = live_.back().off + live_.back().bytes;
            if (live_.back().off >= front) {
                if (cap_ - end >= bytes)
                    at = end;
                else if (front >= bytes)
                    at = 0;
                else
                    return false;
            } else {
                if (front - end >= bytes)
                    at = end;
                else
                    return false;
            }
        }
        live_.push_back({at, bytes, false});
        used_ += bytes;
        *off = at;
        return true;
    }

    void release(uint64_t off)
    {
        for (Range &r : live_) {
            if (r.off == off && !r.freed) {
                r.freed = true;
                used_ -= r.bytes;
                break;
            }
        }
        while (!live_.empty() && live_.front().freed)
            live_.pop_front();
    }

private:
    struct Range {
        uint64_t off, bytes;
        bool freed;
    };
    uint64_t cap_;
    uint64_t used_ = 0;
    std::deque<Range> live_;
};

// Device side of a batch. All calls come from the scheduler's thread.
class Executor {
public:
    virtual ~Executor() = default;
    virtual int slots() const = 0;                 // batches in flight at most
    virtual uint64_t slot_bytes() const = 0;       // largest batch region
    virtual uint32_t slot_requests() const = 0;    // most requests per batch
    // Starts the batch in slot b.slot at pool offset b.pool_off. Returns 0, or
    // an HU_ERR_* code (the batch then completes at once with that error).
    virtual int launch(Batch &b) = 0;
    virtual bool done(const Batch &b) = 0;
    // Fills every request's result (and copies its output out).
    virtual void collect(Batch &b) = 0;
};

struct Config {
    uint64_t pool_bytes = 8ull << 30;
    uint32_t max_in_flight = 65536;     // requests admitted and not yet completed
    uint32_t max_batch_requests = 4096;
    uint64_t max_batch_bytes = 0;       // 0: the executor's slot size
};

// Nearest-rank percentile of a sample (p in (0, 100]); 0 for an empty one.
inline int64_t percentile(std::vector<int64_t> v, double p)
{
    if (v.empty())
        return 0;
    std::sort(v.begin(), v.end());
    double rank = p / 100.0 * (double)v.size();
    uint64_t k = (uint64_t)rank;
    if ((double)k < rank)
        ++k;
    if (k == 0)
        k = 1;
    if (k > v.size())
        k = v.size();
    return v[k - 1];
}

class Scheduler {
public:
    Scheduler(const Config &cfg, Executor *ex)
        : cfg_(cfg), ex_(ex), pool_(cfg.pool_bytes), free_slots_()
    {
        for (int s = ex_->slots() - 1; s >= 0; --s)
            free_slots_.push_back(s);
        batch_cap_ = cfg_.max_batch_bytes ? std::min(cfg_.max_batch_bytes, ex_->slot_bytes()) : ex_->slot_bytes();
        req_cap_ = std::min<uint64_t>(cfg_.max_batch_requests, ex_->slot_requests());
    }

    // Takes a request in arrival order. One that can never run (unknown op,
    // larger than a batch or the pool) completes at the next step with
    // HU_ERR_INVALID_ARGUMENT without affecting any other.
    void enqueue(Request *r)
    {
        r->in_bytes = r->n_units * (op_valid(r->op) ? in_unit(r->op) : 1);
        r->dev_cap = op_converts(r->op) ? std::min(r->dst_cap, worst_out_units(r->op, r->n_units)) : 0;
        const uint64_t alone = region_bytes(1, align_up(r->in_bytes, kAlign), align_up(r->out_bytes(), kAlign));
        if (!op_valid(r->op) || r->n_units > (1ull << 38) || alone > batch_cap_ || alone > pool_.capacity() ||
            (r->n_units && r->src == nullptr)) {
            r->result.error = HU_ERR_INVALID_ARGUMENT;
            r->result.reserved = 0;
            r->result.count = 0;
            r->rejected = true;
            rejected_.push_back(r);
            return;
        }
        queue_.push_back(r);
    }

    // One scheduling round at time `now`: finished batches hand back their
    // requests (appended to `done`) and memory, then new batches start while
    // slots, memory and queued requests allow. Returns batches launched.
    int step(int64_t now, std::vector<Request *> &done)
    {
        for (Request *r : rejected_) {
            r->t_done = now;
            done.push_back(r);
        }
        rejected_.clear();
        for (auto it = running_.begin(); it != running_.end();) {
            Batch &b = *it;
            if (b.slot >= 0 && !ex_->done(b)) {
                ++it;
                continue;
            }
            if (b.slot >= 0)
                ex_->collect(b);
            finish(b, now, done);
            it = running_.erase(it);
        }
        int launched = 0;
        while (!free_slots_.empty() && !queue_.empty()) {
            Batch b;
            uint64_t in_sum = 0, out_sum = 0, n = 0;
            const uint64_t room = std::min(batch_cap_, pool_.largest_free());
            for (Request *r : queue_) {
                if (n >= req_cap_ || in_flight_ + n >= cfg_.max_in_flight)
                    break;
                const uint64_t i2 = in_sum + align_up(r->in_bytes, kAlign);
                const uint64_t o2 = out_sum + align_up(r->out_bytes(), kAlign);
                if (region_bytes(n + 1, i2, o2) > room)
                    break;
                in_sum = i2;
                out_sum = o2;
                ++n;
            }
            if (n == 0)
                break;                       // the head waits for memory or slots
            b.reqs.assign(queue_.begin(), queue_.begin() + (long)n);
            b.lay = lay_out(b);
            if (!pool_.reserve(b.lay.bytes, &b.pool_off))
                break;                       // not expected: the batch was sized to the largest free range
            queue_.erase(queue_.begin(), queue_.begin() + (long)n);
            b.slot = free_slots_.back();
            free_slots_.pop_back();
            b.t_launch = now;
            in_flight_ += n;
            ++batches_;
            batch_requests_ += n;
            const int rc = ex_->launch(b);
            if (rc != HU_OK) {
                for (Request *r : b.reqs) {
                    r->result.error = rc;
                    r->result.reserved = 0;
                    r->result.count = 0;
                }
                free_slots_.push_back(b.slot);
                b.slot = -1;                 // completes at the next step
            }
            running_.push_back(std::move(b));
            ++launched;
        }
        return launched;
    }

    bool idle() const { return queue_.empty() && running_.empty() && rejected_.empty(); }
    size_t queued() const { return queue_.size(); }
    size_t running_batches() const { return running_.size(); }
    uint64_t in_flight() const { return in_flight_; }
    uint64_t pool_used() const { return pool_.used(); }
    uint64_t batches() const { return batches_; }
    uint64_t batch_requests() const { return batch_requests_; }
    int64_t device_ns() const { return device_ns_; }

private:
    void finish(Batch &b, int64_t now, std::vector<Request *> &done)
    {
        for (Request *r : b.reqs) {
            r->t_done = now;
            done.push_back(r);
        }
        in_flight_ -= b.reqs.size();
        device_ns_ += b.device_ns;
        pool_.release(b.pool_off);
        if (b.slot >= 0)
            free_slots_.push_back(b.slot);
    }

    Config cfg_;
    Executor *ex_;
    RingPool pool_;
    std::vector<int> free_slots_;
    std::deque<Request *> queue_;
    std::vector<Request *> rejected_;
    std::deque<Batch> running_;
    uint64_t batch_cap_ = 0, req_cap_ = 0;
    uint64_t in_flight_ = 0, batches_ = 0, batch_requests_ = 0;
    int64_t device_ns_ = 0;
};

}  // namespace serve
}  // namespace hu
