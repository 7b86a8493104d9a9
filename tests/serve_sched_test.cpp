// CPU test of the continuous-batching scheduler with a fake executor.
// Prints "OK <name>" per check; exits non-zero on the first failure.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>

#include "../paper_1810_03099_amd/csrc/serve_core.h"

using namespace mrc_serve;

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::fprintf(stderr, "FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                             \
        }                                                             \
    } while (0)

struct Fake : Executor {
    int n_slots;
    int sleep_us;
    size_t per_token;
    std::atomic<int> running{0}, peak{0}, batches{0};
    std::atomic<int> fail_next{0};
    std::atomic<long> max_batch_seen{0};
    std::atomic<uint64_t> last_first_ticket{0};
    std::atomic<bool> order_ok{true};
    Fake(int s, int us, size_t pt) : n_slots(s), sleep_us(us), per_token(pt) {}
    int slots() const override { return n_slots; }
    size_t batch_bytes(int, int64_t n, int64_t t) const override { return (size_t)t * per_token + (size_t)n; }
    int run(int, Batch& b, std::vector<Result>& out) override {
        int r = ++running;
        int p = peak.load();
        while (r > p && !peak.compare_exchange_weak(p, r)) {}
        ++batches;
        long mb = max_batch_seen.load();
        while ((long)b.reqs.size() > mb && !max_batch_seen.compare_exchange_weak(mb, (long)b.reqs.size())) {}
        for (size_t i = 1; i < b.reqs.size(); ++i)
            if (b.reqs[i].ticket <= b.reqs[i - 1].ticket) order_ok = false;
        std::this_thread::sleep_for(std::chrono::microseconds(sleep_us));
        int rc = kOk;
        if (fail_next.exchange(0)) rc = -4;
        for (size_t i = 0; i < b.reqs.size(); ++i) {
            out[i].status = kOk;
            out[i].n_hits = (int)b.reqs[i].tokens.size();   // echo: lets the test match results to requests
            out[i].id = (int64_t)b.reqs[i].ticket;
        }
        --running;
        return rc;
    }
};

static void test_basic_and_fifo() {
    Fake ex(2, 2000, 1);
    Options o;
    o.max_batch = 8;
    o.max_wait_us = 500;
    Scheduler s(&ex, o);
    std::vector<uint64_t> t;
    std::vector<int32_t> tok(100, 1);
    for (int i = 0; i < 200; ++i) {
        uint64_t k = 0;
        CHECK(s.submit(tok.data(), i % 50, i % 7 == 0 ? kInsert : kQuery, &k) == kOk);
        t.push_back(k);
    }
    for (int i = 0; i < 200; ++i) {
        Result r;
        CHECK(s.poll(t[i], &r, 5000) == kOk);
        CHECK(r.status == kOk && r.n_hits == i % 50 && r.id == (int64_t)t[i]);
        CHECK(r.kind == (i % 7 == 0 ? kInsert : kQuery));
        CHECK(r.t_done >= r.t_start && r.t_start >= r.t_submit);
    }
    Result r;
    CHECK(s.poll(t[0], &r, 0) == kInval);          // each result is handed out once
    CHECK(ex.max_batch_seen.load() <= 8 && ex.order_ok.load());
    CHECK(ex.peak.load() == 2);                    // both slots ran batches at the same time
    std::printf("OK basic_fifo_batches batches=%d\n", ex.batches.load());
}

static void test_mixed_kinds_batch_together() {
    // one slot kept busy by a first request while 64 alternating inserts and
    // queries queue up: they must leave in two batches of 32 (one per kind),
    // each in arrival order, not in 64 batches of one
    Fake ex(1, 20000, 1);
    Options o;
    o.max_batch = 64;
    o.max_wait_us = 0;
    Scheduler s(&ex, o);
    std::vector<int32_t> tok(10, 1);
    uint64_t first;
    CHECK(s.submit(tok.data(), 5, kQuery, &first) == kOk);
    std::this_thread::sleep_for(std::chrono::milliseconds(5));   // the slot picks it up
    std::vector<uint64_t> t;
    for (int i = 0; i < 64; ++i) {
        uint64_t k;
        CHECK(s.submit(tok.data(), 1 + i % 9, i % 2 ? kQuery : kInsert, &k) == kOk);
        t.push_back(k);
    }
    for (int i = 0; i < 64; ++i) {
        Result r;
        CHECK(s.poll(t[i], &r, 10000) == kOk && r.status == kOk);
        CHECK(r.kind == (i % 2 ? kQuery : kInsert) && r.n_hits == 1 + i % 9);
    }
    Result r;
    CHECK(s.poll(first, &r, 10000) == kOk);
    CHECK(ex.order_ok.load() && ex.max_batch_seen.load() == 32 && ex.batches.load() == 3);
    std::printf("OK mixed_kinds batches=%d\n", ex.batches.load());
}

static void test_submit_many() {
    // CSR submission: tickets in order, one result per document; a full queue
    // takes a prefix; bad offsets queue nothing
    Fake ex(1, 3000, 1);
    Options o;
    o.max_batch = 16;
    o.max_queue = 40;
    o.max_wait_us = 0;
    Scheduler s(&ex, o);
    std::vector<int64_t> off(1, 0);
    std::vector<int32_t> tok;
    for (int d = 0; d < 64; ++d) {
        for (int j = 0; j < d % 11; ++j) tok.push_back(d);
        off.push_back((int64_t)tok.size());
    }
    std::vector<uint64_t> t(64);
    int64_t acc = -1;
    CHECK(s.submit_many(off.data(), tok.data(), 30, kQuery, t.data(), &acc) == kOk && acc == 30);
    for (int d = 1; d < 30; ++d) CHECK(t[d] == t[d - 1] + 1);
    for (int d = 0; d < 30; ++d) {
        Result r;
        CHECK(s.poll(t[d], &r, 10000) == kOk && r.status == kOk && r.n_hits == d % 11);
    }
    // one slot busy with a long first request, then 64 documents into a queue of 40
    uint64_t first;
    int32_t one = 1;
    CHECK(s.submit(&one, 1, kQuery, &first) == kOk);
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
    CHECK(s.submit_many(off.data(), tok.data(), 64, kInsert, t.data(), &acc) == kBusy);
    CHECK(acc >= 39 && acc < 64);
    for (int64_t d = 0; d < acc; ++d) {
        Result r;
        CHECK(s.poll(t[d], &r, 10000) == kOk && r.status == kOk && r.kind == kInsert && r.n_hits == d % 11);
    }
    Result r;
    CHECK(s.poll(first, &r, 10000) == kOk);
    std::vector<int64_t> bad = {0, 3, 2, 5};
    CHECK(s.submit_many(bad.data(), tok.data(), 3, kQuery, t.data(), &acc) == kInval && acc == 0);
    CHECK(s.submit_many(off.data(), tok.data(), 2, 9, t.data(), &acc) == kInval && acc == 0);
    CHECK(s.submit_many(off.data(), tok.data(), 0, kQuery, t.data(), &acc) == kOk && acc == 0);
    std::printf("OK submit_many accepted_of_64=%ld\n", (long)acc);
}

static void test_memory_admission() {
    // every token costs 1000 bytes; cap 150000: at most ~150 tokens in flight
    Fake ex(4, 3000, 1000);
    Options o;
    o.max_batch = 64;
    o.mem_cap = 150000;
    o.max_wait_us = 0;
    Scheduler s(&ex, o);
    std::vector<int32_t> tok(100, 3);
    std::vector<uint64_t> t;
    for (int i = 0; i < 40; ++i) {
        uint64_t k;
        CHECK(s.submit(tok.data(), 60, kQuery, &k) == kOk);
        t.push_back(k);
    }
    uint64_t big;
    std::vector<int32_t> huge(200, 1);
    CHECK(s.submit(huge.data(), 200, kQuery, &big) == kOk);   // 200 tokens alone exceed the cap
    for (auto k : t) {
        Result r;
        CHECK(s.poll(k, &r, 10000) == kOk && r.status == kOk);
    }
    Result r;
    CHECK(s.poll(big, &r, 10000) == kOk && r.status == kNoMem);
    Stats st = s.stats();
    CHECK(st.peak_in_flight_bytes <= 150000);
    CHECK(st.failed == 1 && st.completed == 40);
    std::printf("OK memory_admission peak_bytes=%zu concurrent=%d\n", st.peak_in_flight_bytes, st.peak_concurrent_batches);
}

static void test_queue_full_and_failures() {
    Fake ex(1, 20000, 1);
    Options o;
    o.max_batch = 1;
    o.max_queue = 5;
    o.max_wait_us = 0;
    Scheduler s(&ex, o);
    int32_t tok[4] = {1, 2, 3, 4};
    std::vector<uint64_t> ok;
    int busy = 0;
    for (int i = 0; i < 30; ++i) {
        uint64_t k;
        int rc = s.submit(tok, 4, kQuery, &k);
        if (rc == kOk) ok.push_back(k);
        else if (rc == kBusy) ++busy;
        else CHECK(false);
    }
    CHECK(busy > 0);
    for (auto k : ok) {
        Result r;
        CHECK(s.poll(k, &r, 20000) == kOk && r.status == kOk);
    }
    ex.fail_next = 1;
    uint64_t a, b;
    CHECK(s.submit(tok, 4, kQuery, &a) == kOk);
    Result ra;
    CHECK(s.poll(a, &ra, 20000) == kOk && ra.status == -4);       // executor error fails that batch
    CHECK(s.submit(tok, 4, kQuery, &b) == kOk);
    Result rb;
    CHECK(s.poll(b, &rb, 20000) == kOk && rb.status == kOk);      // and later batches still run
    CHECK(s.submit(nullptr, 3, kQuery, &a) == kInval);
    CHECK(s.submit(tok, 4, 7, &a) == kInval);
    std::printf("OK queue_full_and_failures busy=%d\n", busy);
}

static void test_concurrent_submitters_and_stop() {
    Fake ex(3, 300, 1);
    Options o;
    o.max_batch = 16;
    o.max_wait_us = 100;
    Scheduler s(&ex, o);
    std::atomic<int> got{0};
    std::vector<std::thread> th;
    for (int w = 0; w < 6; ++w)
        th.emplace_back([&, w] {
            int32_t tok[8] = {0, 1, 2, 3, 4, 5, 6, 7};
            for (int i = 0; i < 300; ++i) {
                uint64_t k;
                if (s.submit(tok, (w + i) % 8, kQuery, &k) != kOk) continue;
                Result r;
                if (s.poll(k, &r, 20000) == kOk && r.status == kOk && r.n_hits == (w + i) % 8) ++got;
            }
        });
    for (auto& t : th) t.join();
    CHECK(got.load() == 1800);
    // stop drains what is queued
    int32_t tok[2] = {1, 1};
    std::vector<uint64_t> ks(50);
    for (auto& k : ks) CHECK(s.submit(tok, 2, kQuery, &k) == kOk);
    s.stop();
    for (auto k : ks) {
        Result r;
        CHECK(s.poll(k, &r, 0) == kOk && r.status == kOk);
    }
    uint64_t k;
    CHECK(s.submit(tok, 2, kQuery, &k) == kState);
    std::printf("OK concurrent_submitters_and_stop\n");
}

int main() {
    test_basic_and_fifo();
    test_mixed_kinds_batch_together();
    test_submit_many();
    test_memory_admission();
    test_queue_full_and_failures();
    test_concurrent_submitters_and_stop();
    std::printf("ALL OK\n");
    return 0;
}
