// serve.hip - the transcoding server behind hu_server_* (hiputf.h): a
// scheduler thread running serve::Scheduler (serve_core.hpp) with a HIP
// executor. Host code only; the device work is hu_batch_run (or, on the plain
// comparison path, the single-buffer async calls).
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "hiputf.h"
#include "serve_core.hpp"

namespace hu {
namespace serve {
namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// One batch slot: a stream, its events, pinned staging laid out like the
// batch's pool region, and the batch (or single-call) workspace.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t k0 = nullptr, k1 = nullptr, done = nullptr;
    uint8_t *staging = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
};

class HipExecutor final : public Executor {
public:
    HipExecutor(uint8_t *pool, int n_slots, uint64_t slot_bytes, uint32_t slot_requests, bool plain,
                hu_tuning tuning)
        : pool_(pool), slots_(n_slots), slot_bytes_(slot_bytes), slot_requests_(slot_requests), plain_(plain),
          tuning_(tuning)
    {
    }

    ~HipExecutor() override { release(); }

    int init()
    {
        size_t ws_bytes;
        if (plain_) {
            ws_bytes = 0;
            for (int op = HU_OP_VALIDATE_UTF8; op <= HU_OP_CONVERT_UTF16LE_TO_UTF8; ++op) {
                const size_t units = op >= HU_OP_VALIDATE_UTF16LE ? slot_bytes_ / 2 : slot_bytes_;
                const size_t b = hu_workspace_bytes(op, units);
                ws_bytes = b > ws_bytes ? b : ws_bytes;
            }
        } else {
            ws_bytes = hu_batch_workspace_bytes(slot_requests_, slot_bytes_);
        }
        for (Slot &s : slots_) {
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreate(&s.k0) != hipSuccess || hipEventCreate(&s.k1) != hipSuccess ||
                hipEventCreate(&s.done) != hipSuccess)
                return HU_ERR_DEVICE;
            if (hipHostMalloc((void **)&s.staging, slot_bytes_, hipHostMallocDefault) != hipSuccess) {
                s.staging = nullptr;
                return HU_ERR_DEVICE;
            }
            // Write every page once now: the process's first write to a page
            // of the staging buffer takes a fault, and a batch reaching into
            // fresh pages would add those faults to its requests' latency.
            std::memset(s.staging, 0, slot_bytes_);
            if (hipMalloc(&s.ws, ws_bytes) != hipSuccess) {
                s.ws = nullptr;
                return HU_ERR_DEVICE;
            }
            s.ws_bytes = ws_bytes;
            if (hu_workspace_init(s.ws, ws_bytes, s.stream) != HU_OK || hipStreamSynchronize(s.stream) != hipSuccess)
                return HU_ERR_DEVICE;
        }
        return warm_up();
    }

    // Runs two batches of empty documents (one document; more than one
    // planning block of documents) so that every kernel of the batch path has
    // been launched once before the first request arrives.
    int warm_up()
    {
        if (plain_)
            return HU_OK;
        Slot &s = slots_[0];
        const uint32_t sizes[2] = {1u, slot_requests_ < 2048u ? slot_requests_ : 2048u};
        for (uint32_t n : sizes) {
            const size_t res_off = (n * sizeof(hu_doc) + 255) & ~(size_t)255;
            if (res_off + n * sizeof(hu_result) > slot_bytes_)
                continue;
            std::memset(s.staging, 0, n * sizeof(hu_doc));   // empty documents, op 0 (validate UTF-8)
            if (hipMemcpyAsync(pool_, s.staging, n * sizeof(hu_doc), hipMemcpyHostToDevice, s.stream) != hipSuccess)
                return HU_ERR_DEVICE;
            const int rc = hu_batch_run(reinterpret_cast<const hu_doc *>(pool_), n, 0, pool_, pool_,
                                        reinterpret_cast<hu_result *>(pool_ + res_off), &tuning_, s.ws, s.ws_bytes,
                                        s.stream);
            if (rc != HU_OK)
                return rc;
            if (hipStreamSynchronize(s.stream) != hipSuccess)
                return HU_ERR_DEVICE;
        }
        return HU_OK;
    }

    int slots() const override { return (int)slots_.size(); }
    uint64_t slot_bytes() const override { return slot_bytes_; }
    uint32_t slot_requests() const override { return plain_ ? 1u : slot_requests_; }

    int launch(Batch &b) override
    {
        Slot &s = slots_[b.slot];
        uint8_t *h = s.staging;
        uint8_t *d = pool_ + b.pool_off;
        const size_t n = b.reqs.size();
        hu_doc *docs = reinterpret_cast<hu_doc *>(h);
        for (size_t i = 0; i < n; ++i) {
            const Request *r = b.reqs[i];
            docs[i].src_off = r->in_off;
            docs[i].n_units = r->n_units;
            docs[i].dst_off = r->out_off;
            docs[i].dst_cap = r->dev_cap;
            docs[i].op = r->op;
            docs[i].reserved = 0;
            if (r->in_bytes)
                std::memcpy(h + r->in_off, r->src, r->in_bytes);
        }
        if (hipMemcpyAsync(d, h, b.lay.out_begin, hipMemcpyHostToDevice, s.stream) != hipSuccess ||
            hipEventRecord(s.k0, s.stream) != hipSuccess)
            return HU_ERR_DEVICE;
        hu_result *d_results = reinterpret_cast<hu_result *>(d + b.lay.results_off);
        int rc = HU_OK;
        if (plain_) {
            for (size_t i = 0; i < n && rc == HU_OK; ++i)
                rc = single(b.reqs[i], d, d_results + i, s);
        } else {
            rc = hu_batch_run(reinterpret_cast<const hu_doc *>(d), (uint32_t)n, b.lay.out_begin - b.lay.in_begin, d,
                              d, d_results, &tuning_, s.ws, s.ws_bytes, s.stream);
        }
        if (rc != HU_OK)
            return rc;
        if (hipEventRecord(s.k1, s.stream) != hipSuccess ||
            hipMemcpyAsync(h + b.lay.out_begin, d + b.lay.out_begin, b.lay.bytes - b.lay.out_begin,
                           hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
            hipEventRecord(s.done, s.stream) != hipSuccess)
            return HU_ERR_DEVICE;
        return HU_OK;
    }

    bool done(const Batch &b) override { return hipEventQuery(slots_[b.slot].done) != hipErrorNotReady; }

    void collect(Batch &b) override
    {
        Slot &s = slots_[b.slot];
        const bool ok = hipEventSynchronize(s.done) == hipSuccess;
        float ms = 0.f;
        if (ok && hipEventElapsedTime(&ms, s.k0, s.k1) == hipSuccess)
            b.device_ns = (int64_t)(ms * 1e6);
        const hu_result *res = reinterpret_cast<const hu_result *>(s.staging + b.lay.results_off);
        for (size_t i = 0; i < b.reqs.size(); ++i) {
            Request *r = b.reqs[i];
            if (!ok) {
                r->result.error = HU_ERR_DEVICE;
                r->result.reserved = 0;
                r->result.count = 0;
                continue;
            }
            r->result = res[i];
            if (r->dst && op_converts(r->op) && r->result.error == HU_OK && r->result.count <= r->dev_cap)
                std::memcpy(r->dst, s.staging + r->out_off, r->result.count * out_unit(r->op));
        }
    }

    void release()
    {
        for (Slot &s : slots_) {
            if (s.stream)
                (void)hipStreamSynchronize(s.stream);
            if (s.ws)
                (void)hipFree(s.ws);
            if (s.staging)
                (void)hipHostFree(s.staging);
            if (s.k0)
                (void)hipEventDestroy(s.k0);
            if (s.k1)
                (void)hipEventDestroy(s.k1);
            if (s.done)
                (void)hipEventDestroy(s.done);
            if (s.stream)
                (void)hipStreamDestroy(s.stream);
            s = Slot();
        }
    }

private:
    // One request through its single-buffer async call.
    static int single(const Request *r, uint8_t *d, hu_result *res, Slot &s)
    {
        const void *src = d + r->in_off;
        void *dst = d + r->out_off;
        switch (r->op) {
        case HU_OP_VALIDATE_UTF8:
            return validate_utf8_async((const uint8_t *)src, r->n_units, res, s.ws, s.ws_bytes, s.stream);
        case HU_OP_UTF16_LENGTH_FROM_UTF8:
            return utf16_length_from_utf8_async((const uint8_t *)src, r->n_units, res, s.ws, s.ws_bytes, s.stream);
        case HU_OP_CONVERT_UTF8_TO_UTF16LE:
            return convert_utf8_to_utf16le_async((const uint8_t *)src, r->n_units, (uint16_t *)dst, r->dev_cap, res,
                                                 s.ws, s.ws_bytes, s.stream);
        case HU_OP_VALIDATE_UTF16LE:
            return validate_utf16le_async((const uint16_t *)src, r->n_units, res, s.ws, s.ws_bytes, s.stream);
        case HU_OP_UTF8_LENGTH_FROM_UTF16LE:
            return utf8_length_from_utf16le_async((const uint16_t *)src, r->n_units, res, s.ws, s.ws_bytes,
                                                  s.stream);
        default:
            return convert_utf16le_to_utf8_async((const uint16_t *)src, r->n_units, (uint8_t *)dst, r->dev_cap, res,
                                                 s.ws, s.ws_bytes, s.stream);
        }
    }

    uint8_t *pool_;
    std::vector<Slot> slots_;
    uint64_t slot_bytes_;
    uint32_t slot_requests_;
    bool plain_;
    hu_tuning tuning_;
};

// Completion target of a replayed request.
struct ReplaySink {
    hu_completion *out;
    std::atomic<uint64_t> *remaining;
};

class Server {
public:
    int create(const hu_server_config &c)
    {
        if (hipGetDevice(&device_) != hipSuccess)
            return HU_ERR_DEVICE;
        Config cfg;
        cfg.pool_bytes = c.pool_bytes ? c.pool_bytes : (8ull << 30);
        const uint64_t batch_bytes = c.batch_bytes ? c.batch_bytes : (256ull << 20);
        cfg.max_batch_requests = c.batch_requests ? c.batch_requests : 4096u;
        cfg.max_in_flight = c.max_in_flight ? c.max_in_flight : 65536u;
        const int n_slots = c.plain ? 1 : (c.slots ? (int)c.slots : 3);
        if (n_slots > 64 || batch_bytes > cfg.pool_bytes || batch_bytes < 4096)
            return HU_ERR_INVALID_ARGUMENT;
        if (hipMalloc((void **)&pool_, cfg.pool_bytes) != hipSuccess) {
            pool_ = nullptr;
            return HU_ERR_DEVICE;
        }
        // Touch the whole pool once before any request is timed (first use of
        // fresh device memory is slower); the slots' non-blocking streams do
        // not wait for the null stream, hence the synchronisation.
        if (hipMemsetAsync(pool_, 0, cfg.pool_bytes, nullptr) != hipSuccess ||
            hipStreamSynchronize(nullptr) != hipSuccess)
            return HU_ERR_DEVICE;
        exec_ = new (std::nothrow) HipExecutor(pool_, n_slots, batch_bytes, cfg.max_batch_requests, c.plain != 0,
                                               c.tuning);
        if (exec_ == nullptr)
            return HU_ERR_DEVICE;
        const int rc = exec_->init();
        if (rc != HU_OK)
            return rc;
        sched_ = new (std::nothrow) Scheduler(cfg, exec_);
        if (sched_ == nullptr)
            return HU_ERR_DEVICE;
        thread_ = std::thread([this] { loop(); });
        return HU_OK;
    }

    ~Server()
    {
        if (thread_.joinable()) {
            {
                std::lock_guard<std::mutex> lk(in_mu_);
                stop_ = true;
            }
            in_cv_.notify_all();
            thread_.join();
        }
        delete sched_;
        delete exec_;
        if (pool_)
            (void)hipFree(pool_);
        for (Request *r : incoming_)
            delete r;
    }

    int submit(const hu_request *req, int64_t t_arrive, void *sink)
    {
        Request *r = new (std::nothrow) Request();
        if (r == nullptr)
            return HU_ERR_DEVICE;
        r->tag = req->tag;
        r->op = req->op;
        r->src = req->src;
        r->n_units = req->n_units;
        r->dst = req->dst;
        r->dst_cap = req->dst_cap;
        r->t_arrive = t_arrive;
        r->user = sink;
        {
            std::lock_guard<std::mutex> lk(in_mu_);
            incoming_.push_back(r);
            ++submitted_;
        }
        in_cv_.notify_one();
        return HU_OK;
    }

    int poll(hu_completion *out, uint32_t max, uint32_t *n_out, int64_t timeout_ns)
    {
        std::unique_lock<std::mutex> lk(out_mu_);
        if (completions_.empty() && timeout_ns > 0)
            out_cv_.wait_for(lk, std::chrono::nanoseconds(timeout_ns), [this] { return !completions_.empty(); });
        uint32_t k = 0;
        while (k < max && !completions_.empty()) {
            out[k++] = completions_.front();
            completions_.pop_front();
        }
        *n_out = k;
        return HU_OK;
    }

    int replay(const hu_request *reqs, const int64_t *arrival, uint64_t n, hu_completion *out)
    {
        std::atomic<uint64_t> remaining(n);
        std::vector<ReplaySink> sinks(n);
        for (uint64_t i = 0; i < n; ++i)
            sinks[i] = ReplaySink{&out[i], &remaining};
        const int64_t t0 = now_ns();
        uint64_t i = 0;
        while (i < n) {
            const int64_t now = now_ns();
            const int64_t due = t0 + arrival[i];
            if (now < due) {
                if (due - now > 200000)
                    std::this_thread::sleep_for(std::chrono::nanoseconds(due - now - 100000));
                continue;
            }
            // every request already due goes in under one lock
            std::vector<Request *> batch;
            while (i < n && t0 + arrival[i] <= now) {
                Request *r = new (std::nothrow) Request();
                if (r == nullptr)
                    return HU_ERR_DEVICE;
                r->tag = reqs[i].tag;
                r->op = reqs[i].op;
                r->src = reqs[i].src;
                r->n_units = reqs[i].n_units;
                r->dst = reqs[i].dst;
                r->dst_cap = reqs[i].dst_cap;
                r->t_arrive = t0 + arrival[i];
                r->user = &sinks[i];
                batch.push_back(r);
                ++i;
            }
            {
                std::lock_guard<std::mutex> lk(in_mu_);
                incoming_.insert(incoming_.end(), batch.begin(), batch.end());
                submitted_ += batch.size();
            }
            in_cv_.notify_one();
        }
        std::unique_lock<std::mutex> lk(out_mu_);
        out_cv_.wait(lk, [&] { return remaining.load() == 0; });
        return HU_OK;
    }

    void stats(hu_server_stats *o)
    {
        std::lock_guard<std::mutex> lk(out_mu_);
        std::memset(o, 0, sizeof *o);
        {
            std::lock_guard<std::mutex> lk2(in_mu_);
            o->submitted = submitted_;
        }
        o->completed = completed_;
        o->rejected = rejected_;
        o->batches = batches_;
        o->input_bytes = in_bytes_;
        o->output_bytes = out_bytes_;
        o->p50_ns = percentile(latencies_, 50.0);
        o->p99_ns = percentile(latencies_, 99.0);
        o->max_ns = latencies_.empty() ? 0 : *std::max_element(latencies_.begin(), latencies_.end());
        o->device_ns = device_ns_;
        o->mean_batch = batches_ ? (double)batch_requests_ / (double)batches_ : 0.0;
    }

    void reset_stats()
    {
        std::lock_guard<std::mutex> lk(out_mu_);
        {
            std::lock_guard<std::mutex> lk2(in_mu_);
            submitted_ = 0;
        }
        completed_ = rejected_ = in_bytes_ = out_bytes_ = 0;
        latencies_.clear();
        stats_base_batches_ = sched_batches_;
        stats_base_requests_ = sched_requests_;
        stats_base_device_ = sched_device_;
        batches_ = batch_requests_ = 0;
        device_ns_ = 0;
    }

private:
    void loop()
    {
        (void)hipSetDevice(device_);
        std::vector<Request *> arrivals, done;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(in_mu_);
                if (incoming_.empty() && sched_->idle() && !stop_)
                    in_cv_.wait_for(lk, std::chrono::milliseconds(2));
                arrivals.swap(incoming_);
                if (stop_ && arrivals.empty() && sched_->idle())
                    break;
            }
            for (Request *r : arrivals)
                sched_->enqueue(r);
            arrivals.clear();
            const int launched = sched_->step(now_ns(), done);
            if (!done.empty())
                complete(done);
            if (launched == 0 && done.empty() && sched_->running_batches() > 0)
                std::this_thread::yield();
        }
    }

    void complete(std::vector<Request *> &done)
    {
        {
            std::lock_guard<std::mutex> lk(out_mu_);
            sched_batches_ = sched_->batches();
            sched_requests_ = sched_->batch_requests();
            sched_device_ = sched_->device_ns();
            batches_ = sched_batches_ - stats_base_batches_;
            batch_requests_ = sched_requests_ - stats_base_requests_;
            device_ns_ = sched_device_ - stats_base_device_;
            for (Request *r : done) {
                hu_completion c;
                c.tag = r->tag;
                c.result = r->result;
                c.latency_ns = r->t_done - r->t_arrive;
                ++completed_;
                if (r->rejected)
                    ++rejected_;
                if (r->result.error == HU_OK) {
                    in_bytes_ += r->in_bytes;
                    if (op_converts(r->op))
                        out_bytes_ += r->result.count * out_unit(r->op);
                }
                latencies_.push_back(c.latency_ns);
                if (r->user) {
                    ReplaySink *s = static_cast<ReplaySink *>(r->user);
                    *s->out = c;
                    s->remaining->fetch_sub(1);
                } else {
                    completions_.push_back(c);
                }
                delete r;
            }
        }
        out_cv_.notify_all();
        done.clear();
    }

    int device_ = 0;
    uint8_t *pool_ = nullptr;
    HipExecutor *exec_ = nullptr;
    Scheduler *sched_ = nullptr;
    std::thread thread_;

    std::mutex in_mu_;
    std::condition_variable in_cv_;
    std::vector<Request *> incoming_;
    bool stop_ = false;
    uint64_t submitted_ = 0;

    std::mutex out_mu_;
    std::condition_variable out_cv_;
    std::deque<hu_completion> completions_;
    std::vector<int64_t> latencies_;
    uint64_t completed_ = 0, rejected_ = 0, in_bytes_ = 0, out_bytes_ = 0;
    uint64_t batches_ = 0, batch_requests_ = 0;
    int64_t device_ns_ = 0;
    uint64_t sched_batches_ = 0, sched_requests_ = 0, stats_base_batches_ = 0, stats_base_requests_ = 0;
    int64_t sched_device_ = 0, stats_base_device_ = 0;
};

}  // namespace
}  // namespace serve
}  // namespace hu

extern "C" {

int hu_server_create(const hu_server_config *cfg, void **server)
{
    if (server == nullptr)
        return HU_ERR_INVALID_ARGUMENT;
    *server = nullptr;
    hu_server_config c;
    std::memset(&c, 0, sizeof c);
    if (cfg)
        c = *cfg;
    auto *s = new (std::nothrow) hu::serve::Server();
    if (s == nullptr)
        return HU_ERR_DEVICE;
    const int rc = s->create(c);
    if (rc != HU_OK) {
        delete s;
        return rc;
    }
    *server = s;
    return HU_OK;
}

int hu_server_submit(void *server, const hu_request *req)
{
    if (server == nullptr || req == nullptr)
        return HU_ERR_INVALID_ARGUMENT;
    return static_cast<hu::serve::Server *>(server)->submit(req, hu::serve::now_ns(), nullptr);
}

int hu_server_poll(void *server, hu_completion *out, uint32_t max, uint32_t *n_out, int64_t timeout_ns)
{
    if (server == nullptr || n_out == nullptr || (out == nullptr && max > 0))
        return HU_ERR_INVALID_ARGUMENT;
    return static_cast<hu::serve::Server *>(server)->poll(out, max, n_out, timeout_ns);
}

int hu_server_replay(void *server, const hu_request *reqs, const int64_t *arrival_ns, uint64_t n,
                     hu_completion *out)
{
    if (server == nullptr || (n > 0 && (reqs == nullptr || arrival_ns == nullptr || out == nullptr)))
        return HU_ERR_INVALID_ARGUMENT;
    for (uint64_t i = 1; i < n; ++i)
        if (arrival_ns[i] < arrival_ns[i - 1])
            return HU_ERR_INVALID_ARGUMENT;
    return static_cast<hu::serve::Server *>(server)->replay(reqs, arrival_ns, n, out);
}

int hu_server_stats_get(void *server, hu_server_stats *out)
{
    if (server == nullptr || out == nullptr)
        return HU_ERR_INVALID_ARGUMENT;
    static_cast<hu::serve::Server *>(server)->stats(out);
    return HU_OK;
}

int hu_server_stats_reset(void *server)
{
    if (server == nullptr)
        return HU_ERR_INVALID_ARGUMENT;
    static_cast<hu::serve::Server *>(server)->reset_stats();
    return HU_OK;
}

void hu_server_destroy(void *server)
{
    delete static_cast<hu::serve::Server *>(server);
}

}  // extern "C"
