// Request queue of the serving loop (pss_server_*): tickets, first-come-
// first-served admission into batches by memory budget, completion,
// cancellation and latency / throughput accounting.  It holds no device code
// and calls no HIP function, so the same logic runs under a fake executor in
// host-only tests (built with the address, undefined-behaviour and thread
// sanitizers); pss_server.hip supplies the workers that run each batch on the
// GPU.
#pragma once

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <functional>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/pss.h"

namespace pss {

class RequestQueue {
 public:
  // Bytes one batch of m requests of these types, n keys in total and a
  // longest request of max_len keys, needs in a worker's share; false when
  // no such batch can be planned.
  using BatchBytes =
      std::function<bool(pss_key_t, pss_val_t, uint64_t n, uint32_t m, uint64_t max_len,
                         size_t *bytes)>;

  static constexpr uint32_t kMaxBatchRequests = 8192;
  // latencies of the most recent kLatencySamples completed requests (a ring)
  static constexpr size_t kLatencySamples = size_t(1) << 22;

  RequestQueue(size_t share, BatchBytes batch_bytes)
      : share_(share), batch_bytes_(std::move(batch_bytes)) {}

  size_t share() const { return share_; }

  // Admit a request (arguments already checked by the caller).  A request
  // whose batch of one would not fit a share is refused with PSS_ERR_BUDGET.
  pss_status submit(const pss_request &r, uint64_t now_ns, uint64_t *ticket, std::string *err) {
    *ticket = 0;
    if (r.n > 0) {
      size_t bytes = 0;
      const bool ok = batch_bytes_(r.key, r.val, r.n, 1, r.n, &bytes);
      if (!ok || bytes > share_) {
        std::lock_guard<std::mutex> lk(mu_);
        ++rejected_;
        char m[200];
        snprintf(m, sizeof m, "request of %llu keys needs %zu bytes, above the %zu bytes per stream",
                 (unsigned long long)r.n, bytes, share_);
        *err = m;
        return PSS_ERR_BUDGET;
      }
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stop_) {
        *err = "server is shutting down";
        return PSS_ERR_INVALID;
      }
      const uint64_t tk = next_ticket_++;
      Req q;
      q.r = r;
      q.arrival = r.arrival_ns ? r.arrival_ns : now_ns;
      ++submitted_;
      if (r.n == 0) {
        q.state = kDone;
        ++completed_;
        record_latency((float)((double)(now_ns > q.arrival ? now_ns - q.arrival : 0) * 1e-6));
      } else {
        queue_.push_back(tk);
      }
      reqs_.emplace(tk, q);
      *ticket = tk;
    }
    if (r.n) cv_work_.notify_one();
    else cv_done_.notify_all();
    return PSS_OK;
  }

  // Worker side: wait for queued work, then take in arrival order every
  // queued request of the head's types that still fits one share.  Returns
  // false once the queue is stopped.  The batch's bytes count as in use
  // until finish_batch.
  bool next_batch(std::vector<uint64_t> *tickets, std::vector<pss_request> *reqs, size_t *bytes) {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_work_.wait(lk, [&] { return stop_ || !queue_.empty(); });
      if (stop_) return false;
      form_batch(tickets, bytes);
      if (tickets->empty()) continue;
      reqs->clear();
      for (uint64_t tk : *tickets) reqs->push_back(reqs_[tk].r);
      in_use_ += *bytes;
      if (!queue_.empty()) cv_work_.notify_one();
      return true;
    }
  }

  // Worker side: the batch finished with status st at time now_ns.
  void finish_batch(const std::vector<uint64_t> &tickets, pss_status st, uint64_t now_ns,
                    size_t bytes) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      uint64_t keys = 0;
      for (uint64_t tk : tickets) {
        Req &q = reqs_[tk];
        q.state = kDone;
        q.result = st;
        if (st == PSS_OK) {
          ++completed_;
          keys_completed_ += q.r.n;
          keys += q.r.n;
          record_latency((float)((double)(now_ns - q.arrival) * 1e-6));
          if (first_arrival_ == 0 || q.arrival < first_arrival_) first_arrival_ = q.arrival;
        } else {
          ++failed_;
        }
      }
      ++batches_;
      batch_requests_ += tickets.size();
      batch_keys_ += keys;
      last_done_ = std::max(last_done_, now_ns);
      in_use_ -= bytes;
    }
    cv_done_.notify_all();
  }

  pss_status poll(uint64_t ticket, int *done, pss_status *result, std::string *err) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) {
      *err = "unknown ticket";
      return PSS_ERR_INVALID;
    }
    *done = it->second.state == kDone;
    if (*done) {
      if (result) *result = it->second.result;
      reqs_.erase(it);
    }
    return PSS_OK;
  }

  pss_status wait(uint64_t ticket, pss_status *result, std::string *err) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) {
      *err = "unknown ticket";
      return PSS_ERR_INVALID;
    }
    cv_done_.wait(lk, [&] {
      it = reqs_.find(ticket);
      return it == reqs_.end() || it->second.state == kDone;
    });
    if (it == reqs_.end()) {
      *err = "ticket collected by another call";
      return PSS_ERR_INVALID;
    }
    if (result) *result = it->second.result;
    reqs_.erase(it);
    return PSS_OK;
  }

  pss_status cancel(uint64_t ticket, std::string *err) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = reqs_.find(ticket);
      if (it == reqs_.end()) {
        *err = "unknown ticket";
        return PSS_ERR_INVALID;
      }
      if (it->second.state != kQueued) {
        *err = "request already launched or finished";
        return PSS_ERR_BUSY;
      }
      it->second.state = kDone;  // form_batch drops it from the queue
      it->second.result = PSS_ERR_CANCELLED;
      ++cancelled_;
    }
    cv_done_.notify_all();
    return PSS_OK;
  }

  void stats(pss_stats *out) {
    std::vector<float> lat;
    pss_stats s{};
    {
      std::lock_guard<std::mutex> lk(mu_);
      s.submitted = submitted_;
      s.completed = completed_;
      s.rejected = rejected_;
      s.cancelled = cancelled_;
      s.failed = failed_;
      s.batches = batches_;
      s.keys_completed = keys_completed_;
      if (last_done_ > first_arrival_ && first_arrival_)
        s.keys_per_s = (double)keys_completed_ / ((double)(last_done_ - first_arrival_) * 1e-9);
      if (batches_) {
        s.mean_batch_requests = (double)batch_requests_ / (double)batches_;
        s.mean_batch_keys = (double)batch_keys_ / (double)batches_;
      }
      s.budget_in_use = in_use_;
      uint64_t queued = 0;
      for (uint64_t tk : queue_) {
        auto it = reqs_.find(tk);
        if (it != reqs_.end() && it->second.state == kQueued) ++queued;
      }
      s.queued = queued;
      lat = latency_ms_;
    }
    if (!lat.empty()) {
      // nearest-rank percentiles
      auto pct = [&](double p) {
        size_t k = (size_t)std::ceil(p * (double)lat.size());
        k = std::min(std::max<size_t>(k, 1), lat.size()) - 1;
        std::nth_element(lat.begin(), lat.begin() + k, lat.end());
        return (double)lat[k];
      };
      double sum = 0, mx = 0;
      for (float v : lat) {
        sum += v;
        mx = std::max(mx, (double)v);
      }
      s.latency_mean_ms = sum / (double)lat.size();
      s.latency_max_ms = mx;
      s.latency_p50_ms = pct(0.50);
      s.latency_p99_ms = pct(0.99);
    }
    *out = s;
  }

  void reset_stats() {
    std::lock_guard<std::mutex> lk(mu_);
    submitted_ = completed_ = rejected_ = cancelled_ = failed_ = 0;
    batches_ = batch_requests_ = batch_keys_ = keys_completed_ = 0;
    first_arrival_ = last_done_ = 0;
    latency_ms_.clear();
    latency_next_ = 0;
  }

  // Cancel every queued request and wake every waiter; next_batch returns
  // false from then on.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      for (uint64_t tk : queue_) {
        auto it = reqs_.find(tk);
        if (it != reqs_.end() && it->second.state == kQueued) {
          it->second.state = kDone;
          it->second.result = PSS_ERR_CANCELLED;
        }
      }
      queue_.clear();
    }
    cv_work_.notify_all();
    cv_done_.notify_all();
  }

 private:
  enum ReqState { kQueued = 0, kLaunched = 1, kDone = 2 };
  struct Req {
    pss_request r{};
    uint64_t arrival = 0;
    int state = kQueued;
    pss_status result = PSS_OK;
  };

  void record_latency(float ms) {
    if (latency_ms_.size() < kLatencySamples) {
      latency_ms_.push_back(ms);
    } else {
      latency_ms_[latency_next_] = ms;
      latency_next_ = (latency_next_ + 1) % kLatencySamples;
    }
  }

  // Called with the lock held.
  void form_batch(std::vector<uint64_t> *batch, size_t *bytes) {
    batch->clear();
    *bytes = 0;
    std::deque<uint64_t> keep;
    bool have_type = false, closed = false;
    pss_key_t key = PSS_U32;
    pss_val_t val = PSS_VAL_NONE;
    uint64_t total = 0, max_len = 0;
    while (!queue_.empty()) {
      const uint64_t tk = queue_.front();
      queue_.pop_front();
      auto it = reqs_.find(tk);
      if (it == reqs_.end() || it->second.state != kQueued) continue;  // cancelled
      Req &q = it->second;
      if (!have_type) {
        key = q.r.key;
        val = q.r.val;
        have_type = true;
      }
      bool take = false;
      if (!closed && q.r.key == key && q.r.val == val && batch->size() < kMaxBatchRequests) {
        const uint64_t ml = std::max(max_len, q.r.n);
        size_t b = 0;
        if (batch_bytes_(key, val, total + q.r.n, (uint32_t)batch->size() + 1, ml, &b) &&
            b <= share_) {
          take = true;
          total += q.r.n;
          max_len = ml;
          *bytes = b;
        } else {
          closed = true;  // keep first-come-first-served order within the type
        }
      }
      if (take) {
        q.state = kLaunched;
        batch->push_back(tk);
      } else {
        keep.push_back(tk);
      }
    }
    queue_.swap(keep);
  }

  const size_t share_;
  const BatchBytes batch_bytes_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<uint64_t> queue_;  // tickets in arrival order (cancelled ones are skipped)
  std::unordered_map<uint64_t, Req> reqs_;
  uint64_t next_ticket_ = 1;
  bool stop_ = false;
  uint64_t submitted_ = 0, completed_ = 0, rejected_ = 0, cancelled_ = 0, failed_ = 0;
  uint64_t batches_ = 0, batch_requests_ = 0, batch_keys_ = 0, keys_completed_ = 0;
  uint64_t first_arrival_ = 0, last_done_ = 0;
  uint64_t in_use_ = 0;
  std::vector<float> latency_ms_;
  size_t latency_next_ = 0;
};

}  // namespace pss
