// Continuous-batching request scheduler of the serving loop (host C++ only,
// no HIP): requests queue up, each execution slot (one device stream) pulls
// the next batch as soon as it is free, so batches form while earlier ones
// still run, and a batch is admitted only while the memory of the batches in
// flight fits the cap. The device work is behind the Executor interface, so
// the scheduler is tested on the CPU with a fake executor.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace mrc_serve {

constexpr int kOk = 0, kInval = -1, kNoMem = -2, kBusy = -5, kState = -6;
constexpr int kQuery = 0, kInsert = 1;

struct Request {
    uint64_t ticket = 0;
    int kind = kQuery;
    std::vector<int32_t> tokens;
    double t_submit = 0;
};

struct Hit {
    int64_t id;
    float s;
};

struct Result {
    int status = kOk;
    int kind = kQuery;
    int64_t id = -1;     // insert: assigned database id
    int n_hits = 0;      // query: rows >= tau
    std::vector<Hit> top;
    double t_submit = 0, t_start = 0, t_done = 0;
};

struct Batch {
    int kind = kQuery;
    std::vector<Request> reqs;
    int64_t tokens = 0;
    size_t bytes = 0;     // admitted memory estimate
};

class Executor {
   public:
    virtual ~Executor() = default;
    virtual int slots() const = 0;
    // Memory the batch needs on the device while it runs.
    virtual size_t batch_bytes(int kind, int64_t n_docs, int64_t n_tokens) const = 0;
    // Run a batch on slot `slot`; fill one result per request (status per
    // result). Return value kOk, or an error that fails the whole batch.
    virtual int run(int slot, Batch& b, std::vector<Result>& out) = 0;
};

struct Options {
    int max_batch = 256;
    int64_t max_batch_tokens = 1 << 22;
    int max_queue = 100000;
    size_t mem_cap = (size_t)1 << 34;
    int max_wait_us = 200;       // a partial batch may wait this long for more arrivals
};

struct Stats {
    uint64_t submitted = 0, rejected = 0, completed = 0, failed = 0, batches = 0;
    size_t peak_in_flight_bytes = 0;
    int peak_concurrent_batches = 0;
};

class Scheduler {
   public:
    Scheduler(Executor* ex, const Options& o);
    ~Scheduler();
    int submit(const int32_t* tokens, int64_t len, int kind, uint64_t* ticket);
    // n documents at once (document i is tokens[offsets[i], offsets[i + 1])),
    // queued in order under one lock while the queue has room: *accepted of
    // them go in, with tickets[0, *accepted). kOk when all did, kBusy when the
    // queue filled first.
    int submit_many(const int64_t* offsets, const int32_t* tokens, int64_t n, int kind, uint64_t* tickets,
                    int64_t* accepted);
    // kOk with the result (removed from the table), kBusy while pending,
    // kInval for an unknown ticket. wait_ms > 0 blocks up to that long.
    int poll(uint64_t ticket, Result* out, int wait_ms);
    void stop();  // drain the queue, join the slots
    Stats stats();
    double now_ms() const;

   private:
    void slot_loop(int slot);
    bool form_batch(std::unique_lock<std::mutex>& lk, Batch* b);

    Executor* ex_;
    Options opt_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<Request> queue_;
    std::unordered_map<uint64_t, Result> done_;
    std::unordered_map<uint64_t, bool> pending_;
    uint64_t next_ticket_ = 1;
    size_t in_flight_bytes_ = 0;
    int running_ = 0;
    bool stopping_ = false;
    Stats st_;
    std::vector<std::thread> threads_;
    std::chrono::steady_clock::time_point t0_;
};

}  // namespace mrc_serve
