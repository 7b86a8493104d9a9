// Continuous-batching scheduler (see serve_core.h).
#include "serve_core.h"

#include <algorithm>
#include <chrono>

namespace mrc_serve {

Scheduler::Scheduler(Executor* ex, const Options& o) : ex_(ex), opt_(o), t0_(std::chrono::steady_clock::now()) {
    if (opt_.max_batch < 1) opt_.max_batch = 1;
    if (opt_.max_batch_tokens < 1) opt_.max_batch_tokens = 1;
    for (int s = 0; s < ex_->slots(); ++s) threads_.emplace_back(&Scheduler::slot_loop, this, s);
}

Scheduler::~Scheduler() { stop(); }

double Scheduler::now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_).count();
}

int Scheduler::submit(const int32_t* tokens, int64_t len, int kind, uint64_t* ticket) {
    if (len < 0 || (len > 0 && !tokens) || (kind != kQuery && kind != kInsert) || !ticket) return kInval;
    Request r;
    r.kind = kind;
    r.tokens.assign(tokens, tokens + len);
    std::lock_guard<std::mutex> g(mu_);
    if (stopping_) return kState;
    if ((int)queue_.size() >= opt_.max_queue) {
        ++st_.rejected;
        return kBusy;
    }
    r.ticket = next_ticket_++;
    r.t_submit = now_ms();
    *ticket = r.ticket;
    pending_[r.ticket] = true;
    queue_.push_back(std::move(r));
    ++st_.submitted;
    cv_work_.notify_one();
    return kOk;
}

int Scheduler::submit_many(const int64_t* offsets, const int32_t* tokens, int64_t n, int kind, uint64_t* tickets,
                           int64_t* accepted) {
    if (!accepted) return kInval;
    *accepted = 0;
    if (n < 0 || (n > 0 && (!offsets || !tickets)) || (kind != kQuery && kind != kInsert)) return kInval;
    for (int64_t i = 0; i < n; ++i)
        if (offsets[i + 1] < offsets[i] || (offsets[i + 1] > offsets[i] && !tokens)) return kInval;
    std::vector<Request> rs((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        rs[i].kind = kind;
        rs[i].tokens.assign(tokens + offsets[i], tokens + offsets[i + 1]);
    }
    std::lock_guard<std::mutex> g(mu_);
    if (stopping_) return kState;
    int64_t i = 0;
    for (; i < n && (int)queue_.size() < opt_.max_queue; ++i) {
        Request& r = rs[i];
        r.ticket = next_ticket_++;
        r.t_submit = now_ms();
        tickets[i] = r.ticket;
        pending_[r.ticket] = true;
        queue_.push_back(std::move(r));
        ++st_.submitted;
    }
    *accepted = i;
    st_.rejected += (uint64_t)(n - i);
    if (i) cv_work_.notify_all();
    return i == n ? kOk : kBusy;
}

int Scheduler::poll(uint64_t ticket, Result* out, int wait_ms) {
    std::unique_lock<std::mutex> lk(mu_);
    auto deadline = std::chrono::steady_clock::now() + std::chrono::milliseconds(std::max(0, wait_ms));
    while (true) {
        auto it = done_.find(ticket);
        if (it != done_.end()) {
            if (out) *out = std::move(it->second);
            done_.erase(it);
            return kOk;
        }
        if (!pending_.count(ticket)) return kInval;
        if (wait_ms <= 0 || cv_done_.wait_until(lk, deadline) == std::cv_status::timeout) {
            if (done_.count(ticket)) continue;
            return kBusy;
        }
    }
}

// Take requests of the head's kind, in arrival order (requests of the other
// kind are passed over, and stay at the front for the next batch), while the
// batch stays within max_batch, max_batch_tokens and the memory cap. The
// oldest request always goes in the next batch, so neither kind starves; a
// query sees the rows committed before its batch starts. Called with mu_ held.
bool Scheduler::form_batch(std::unique_lock<std::mutex>& lk, Batch* b) {
    (void)lk;
    b->reqs.clear();
    b->tokens = 0;
    b->bytes = 0;
    if (queue_.empty()) return false;
    b->kind = queue_.front().kind;
    int64_t n = 0, toks = 0;
    size_t bytes = 0;
    std::vector<size_t> take;
    for (size_t i = 0; i < queue_.size() && n < opt_.max_batch; ++i) {
        const Request& r = queue_[i];
        if (r.kind != b->kind) continue;
        const int64_t t2 = toks + (int64_t)r.tokens.size();
        if (n > 0 && t2 > opt_.max_batch_tokens) break;
        const size_t by = ex_->batch_bytes(b->kind, n + 1, t2);
        if (in_flight_bytes_ + by > opt_.mem_cap) break;
        take.push_back(i);
        ++n;
        toks = t2;
        bytes = by;
    }
    if (n == 0) return false;
    // only the prefix up to the last request taken changes: the skipped
    // requests of other kinds in it go back to the front in their order
    const size_t end = take.back() + 1;
    std::vector<Request> skipped;
    skipped.reserve(end - take.size());
    size_t t = 0;
    for (size_t i = 0; i < end; ++i) {
        if (t < take.size() && take[t] == i) {
            b->reqs.push_back(std::move(queue_[i]));
            ++t;
        } else {
            skipped.push_back(std::move(queue_[i]));
        }
    }
    queue_.erase(queue_.begin(), queue_.begin() + (std::ptrdiff_t)end);
    for (size_t i = skipped.size(); i-- > 0;) queue_.push_front(std::move(skipped[i]));
    b->tokens = toks;
    b->bytes = bytes;
    return true;
}

void Scheduler::slot_loop(int slot) {
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
        cv_work_.wait(lk, [&] { return stopping_ || !queue_.empty(); });
        if (queue_.empty()) {
            if (stopping_) return;
            continue;
        }
        // a partial batch waits briefly for more arrivals (bounded)
        if ((int)queue_.size() < opt_.max_batch && opt_.max_wait_us > 0 && !stopping_) {
            cv_work_.wait_for(lk, std::chrono::microseconds(opt_.max_wait_us),
                              [&] { return stopping_ || (int)queue_.size() >= opt_.max_batch; });
            if (queue_.empty()) continue;
        }
        Batch b;
        if (!form_batch(lk, &b)) {
            // the head does not fit next to the batches in flight
            if (running_ == 0) {
                // nothing will free memory: the head request alone exceeds the cap
                Request r = std::move(queue_.front());
                queue_.pop_front();
                Result res;
                res.status = kNoMem;
                res.kind = r.kind;
                res.t_submit = r.t_submit;
                res.t_start = res.t_done = now_ms();
                pending_.erase(r.ticket);
                done_[r.ticket] = std::move(res);
                ++st_.failed;
                cv_done_.notify_all();
                continue;
            }
            cv_work_.wait(lk);  // woken when a batch completes
            continue;
        }
        in_flight_bytes_ += b.bytes;
        ++running_;
        ++st_.batches;
        st_.peak_in_flight_bytes = std::max(st_.peak_in_flight_bytes, in_flight_bytes_);
        st_.peak_concurrent_batches = std::max(st_.peak_concurrent_batches, running_);
        const double t_start = now_ms();
        lk.unlock();
        std::vector<Result> out(b.reqs.size());
        int rc = ex_->run(slot, b, out);
        const double t_done = now_ms();
        lk.lock();
        for (size_t i = 0; i < b.reqs.size(); ++i) {
            Result& r = out[i];
            if (rc != kOk) r.status = rc;
            r.kind = b.kind;
            r.t_submit = b.reqs[i].t_submit;
            r.t_start = t_start;
            r.t_done = t_done;
            if (r.status == kOk) ++st_.completed;
            else ++st_.failed;
            pending_.erase(b.reqs[i].ticket);
            done_[b.reqs[i].ticket] = std::move(r);
        }
        in_flight_bytes_ -= b.bytes;
        --running_;
        cv_done_.notify_all();
        cv_work_.notify_all();
    }
}

void Scheduler::stop() {
    {
        std::lock_guard<std::mutex> g(mu_);
        if (stopping_ && threads_.empty()) return;
        stopping_ = true;
    }
    cv_work_.notify_all();
    for (auto& t : threads_)
        if (t.joinable()) t.join();
    threads_.clear();
}

Stats Scheduler::stats() {
    std::lock_guard<std::mutex> g(mu_);
    return st_;
}

}  // namespace mrc_serve
