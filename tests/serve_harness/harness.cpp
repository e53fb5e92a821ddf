// Test harness for the server's host logic (serve_core.hpp): the scheduler
// with a fake executor on a virtual clock, and the ring pool, behind a small
// C interface for ctypes. No GPU: a batch "runs" for a fixed virtual time and
// reports count = n_units for every request.
#include <cstdint>
#include <cstring>
#include <vector>

#include "serve_core.hpp"

using namespace hu::serve;

namespace {

class FakeExecutor final : public Executor {
public:
    FakeExecutor(int slots, uint64_t slot_bytes, uint32_t slot_requests, int64_t latency, int64_t ps_per_byte)
        : slots_(slots), slot_bytes_(slot_bytes), slot_requests_(slot_requests), latency_(latency),
          ps_per_byte_(ps_per_byte), busy_(slots, false)
    {
    }
    int slots() const override { return slots_; }
    uint64_t slot_bytes() const override { return slot_bytes_; }
    uint32_t slot_requests() const override { return slot_requests_; }

    int launch(Batch &b) override
    {
        if (busy_[b.slot])
            return -1000;                       // the scheduler handed out a busy slot
        if (fail_next_) {
            fail_next_ = false;
            return HU_ERR_DEVICE;
        }
        busy_[b.slot] = true;
        uint64_t bytes = 0;
        for (Request *r : b.reqs)
            bytes += r->in_bytes;
        finish_at_.resize(slots_);
        finish_at_[b.slot] = now + latency_ + (int64_t)(bytes * ps_per_byte_ / 1000);
        last_.clear();
        for (Request *r : b.reqs)
            last_.push_back(r->tag);
        if (b.lay.bytes > slot_bytes_)
            return -1001;                       // the scheduler exceeded the slot size
        return HU_OK;
    }
    bool done(const Batch &b) override { return now >= finish_at_[b.slot]; }
    void collect(Batch &b) override
    {
        busy_[b.slot] = false;
        for (Request *r : b.reqs) {
            r->result.error = HU_OK;
            r->result.reserved = 0;
            r->result.count = r->n_units;
        }
    }

    int64_t now = 0;
    bool fail_next_ = false;
    std::vector<uint64_t> last_;

private:
    int slots_;
    uint64_t slot_bytes_;
    uint32_t slot_requests_;
    int64_t latency_, ps_per_byte_;
    std::vector<bool> busy_;
    std::vector<int64_t> finish_at_;
};

struct Harness {
    FakeExecutor ex;
    Scheduler sched;
    std::vector<Request *> done;
    Harness(const Config &c, int slots, uint64_t slot_bytes, uint32_t slot_requests, int64_t latency, int64_t ps)
        : ex(slots, slot_bytes, slot_requests, latency, ps), sched(c, &ex)
    {
    }
};

}  // namespace

extern "C" {

void *h_create(uint64_t pool, uint64_t slot_bytes, uint32_t slot_requests, int slots, uint32_t max_batch,
               uint32_t max_in_flight, int64_t latency_ns, int64_t ps_per_byte)
{
    Config c;
    c.pool_bytes = pool;
    c.max_batch_requests = max_batch;
    c.max_in_flight = max_in_flight;
    return new Harness(c, slots, slot_bytes, slot_requests, latency_ns, ps_per_byte);
}

void h_destroy(void *h) { delete static_cast<Harness *>(h); }

void h_submit(void *hp, uint64_t tag, uint32_t op, uint64_t n_units, uint64_t dst_cap, int64_t t_arrive, int has_src)
{
    static const char dummy[1] = {0};
    Request *r = new Request();
    r->tag = tag;
    r->op = op;
    r->n_units = n_units;
    r->src = has_src ? dummy : nullptr;
    r->dst_cap = dst_cap;
    r->t_arrive = t_arrive;
    static_cast<Harness *>(hp)->sched.enqueue(r);
}

void h_fail_next_launch(void *hp) { static_cast<Harness *>(hp)->ex.fail_next_ = true; }

// One step at `now`; completions (tag, error, count, latency) go to the
// arrays (at most max_out; the rest stay for the next call). Returns the
// number of batches launched.
int h_step(void *hp, int64_t now, uint64_t *tags, int32_t *errs, uint64_t *counts, int64_t *lat, uint32_t max_out,
           uint32_t *n_out)
{
    Harness *h = static_cast<Harness *>(hp);
    h->ex.now = now;
    const int launched = h->sched.step(now, h->done);
    uint32_t k = 0;
    while (k < max_out && !h->done.empty()) {
        Request *r = h->done.front();
        h->done.erase(h->done.begin());
        tags[k] = r->tag;
        errs[k] = r->result.error;
        counts[k] = r->result.count;
        lat[k] = r->t_done - r->t_arrive;
        ++k;
        delete r;
    }
    *n_out = k;
    return launched;
}

uint64_t h_pool_used(void *hp) { return static_cast<Harness *>(hp)->sched.pool_used(); }
uint64_t h_in_flight(void *hp) { return static_cast<Harness *>(hp)->sched.in_flight(); }
uint64_t h_queued(void *hp) { return static_cast<Harness *>(hp)->sched.queued(); }
uint64_t h_running(void *hp) { return static_cast<Harness *>(hp)->sched.running_batches(); }
uint64_t h_batches(void *hp) { return static_cast<Harness *>(hp)->sched.batches(); }
int h_idle(void *hp) { return static_cast<Harness *>(hp)->sched.idle() ? 1 : 0; }

uint32_t h_last_batch(void *hp, uint64_t *tags, uint32_t max)
{
    const std::vector<uint64_t> &v = static_cast<Harness *>(hp)->ex.last_;
    uint32_t k = 0;
    for (; k < max && k < v.size(); ++k)
        tags[k] = v[k];
    return (uint32_t)v.size();
}

int64_t h_percentile(const int64_t *v, uint64_t n, double p) { return percentile(std::vector<int64_t>(v, v + n), p); }

uint64_t h_region_bytes(uint64_t n, uint64_t in_sum, uint64_t out_sum) { return region_bytes(n, in_sum, out_sum); }

void *rp_create(uint64_t cap) { return new RingPool(cap); }
void rp_destroy(void *p) { delete static_cast<RingPool *>(p); }
int rp_reserve(void *p, uint64_t bytes, uint64_t *off) { return static_cast<RingPool *>(p)->reserve(bytes, off) ? 1 : 0; }
void rp_release(void *p, uint64_t off) { static_cast<RingPool *>(p)->release(off); }
uint64_t rp_largest(void *p) { return static_cast<RingPool *>(p)->largest_free(); }
uint64_t rp_used(void *p) { return static_cast<RingPool *>(p)->used(); }

}  // extern "C"
