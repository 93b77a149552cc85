// Host-only test of the serving loop's request queue (pss_queue.hpp) under a
// fake executor: worker threads take batches from the queue exactly as the
// GPU workers do, and "run" each batch by sorting its requests with the CPU
// oracle (host arrays), sleeping in proportion to the batch's keys.  Built
// with the address + undefined-behaviour sanitizers and, separately, with
// the thread sanitizer.  Checks:
//   - admission: a request whose batch of one exceeds a worker's share is
//     refused (PSS_ERR_BUDGET); no batch ever exceeds a share;
//   - continuous batching: requests submitted while the workers are busy
//     join later batches (more than one request per batch on average);
//   - every completed request equals the plain definition of its result
//     (keys ascending, ties in input order), alone and in the mix;
//   - a batch failed on purpose fails exactly its own requests; the others
//     finish bit-exact, and the budget in use returns to 0;
//   - cancellation of queued requests, and shutdown with requests queued.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../oracle/pses_oracle.h"
#include "../../paper_2305_05245_amd/csrc/pss_queue.hpp"

static int failures = 0;
#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Bytes a batch occupies in a share: about what the GPU workers plan for
// (staging + output + workspace per key, tables per request).
bool fake_batch_bytes(pss_key_t key, pss_val_t val, uint64_t n, uint32_t m, uint64_t,
                      size_t *bytes) {
  const size_t kb = (key == PSS_U32 || key == PSS_I32 || key == PSS_F32) ? 4 : 8;
  *bytes = (size_t)n * (3 * kb + (val == PSS_VAL_U32 ? 12 : 0)) + (size_t)m * 48 + 4096;
  return true;
}

struct HostReq {
  std::vector<int64_t> keys, out;
  std::vector<uint32_t> vals, vout;
  uint64_t ticket = 0;
  pss_status result = PSS_OK;
};

// The plain definition: keys ascending, equal keys in input order (the
// payload is the input index).
void reference(const HostReq &r, std::vector<int64_t> *k, std::vector<uint32_t> *v) {
  std::vector<std::pair<int64_t, uint32_t>> p(r.keys.size());
  for (size_t i = 0; i < p.size(); ++i) p[i] = {r.keys[i], r.vals[i]};
  std::stable_sort(p.begin(), p.end(),
                   [](const auto &a, const auto &b) { return a.first < b.first; });
  k->resize(p.size());
  v->resize(p.size());
  for (size_t i = 0; i < p.size(); ++i) {
    (*k)[i] = p[i].first;
    (*v)[i] = p[i].second;
  }
}

struct Executor {
  pss::RequestQueue *q;
  std::atomic<int> batch_seq{0};
  int fail_batch = -1;  // index of the batch to fail on purpose
  std::atomic<uint64_t> max_bytes{0};
  std::atomic<int> over_share{0};
  std::vector<std::thread> th;

  void run() {
    std::vector<uint64_t> tickets;
    std::vector<pss_request> rs;
    size_t bytes = 0;
    while (q->next_batch(&tickets, &rs, &bytes)) {
      const int id = batch_seq.fetch_add(1);
      if (bytes > q->share()) over_share.fetch_add(1);
      uint64_t keys = 0;
      pss_status st = PSS_OK;
      if (id == fail_batch) {
        st = PSS_ERR_HIP;  // as a failed launch would report
      } else {
        for (const pss_request &r : rs) {
          keys += r.n;
          const int rc = oracle_pses(3, r.n, r.keys_in, r.vals_in, 4, 4, r.keys_out, r.vals_out,
                                     nullptr, nullptr, nullptr, nullptr, nullptr, 0);
          if (rc != ORACLE_OK) st = PSS_ERR_HIP;
        }
      }
      std::this_thread::sleep_for(std::chrono::microseconds(200 + keys / 64));
      q->finish_batch(tickets, st, now_ns(), bytes);
    }
  }
  void start(int workers) {
    for (int i = 0; i < workers; ++i) th.emplace_back([this] { run(); });
  }
  void join() {
    for (auto &t : th) t.join();
  }
};

pss_request make_request(HostReq &h) {
  pss_request r{};
  r.key = PSS_I64;
  r.val = PSS_VAL_U32;
  r.keys_in = h.keys.data();
  r.keys_out = h.out.data();
  r.vals_in = h.vals.data();
  r.vals_out = h.vout.data();
  r.n = h.keys.size();
  r.arrival_ns = 0;
  return r;
}

}  // namespace

int main() {
  std::mt19937_64 rng(14);
  const size_t share = 24 * 20000 + 4096 * 4;  // about 20000 keys per batch
  pss::RequestQueue q(share, fake_batch_bytes);
  Executor ex;
  ex.q = &q;
  ex.fail_batch = 3;
  ex.start(3);

  // requests: log-uniform sizes 2^4..2^13, half uniform keys, half {0,1,2}
  const int n_req = 600;
  std::vector<HostReq> reqs(n_req);
  std::uniform_real_distribution<double> U(4.0, 13.0);
  for (int i = 0; i < n_req; ++i) {
    const size_t n = (size_t)std::llround(std::pow(2.0, U(rng)));
    HostReq &h = reqs[i];
    h.keys.resize(n);
    h.vals.resize(n);
    for (size_t j = 0; j < n; ++j) {
      h.keys[j] = (i % 2) ? (int64_t)rng() : (int64_t)(rng() % 3);
      h.vals[j] = (uint32_t)j;
    }
    h.out.assign(n, 0);
    h.vout.assign(n, 0);
  }

  // admission: a batch of one larger than a share is refused
  {
    HostReq big;
    big.keys.assign(40000, 1);
    big.vals.assign(40000, 0);
    big.out.assign(40000, 0);
    big.vout.assign(40000, 0);
    pss_request r = make_request(big);
    uint64_t t = 1;
    std::string err;
    CHECK(q.submit(r, now_ns(), &t, &err) == PSS_ERR_BUDGET);
    CHECK(t == 0 && !err.empty());
  }

  // bursts of arrivals: each burst lands while the workers are busy
  std::vector<uint64_t> cancelled;
  for (int i = 0; i < n_req; ++i) {
    pss_request r = make_request(reqs[i]);
    std::string err;
    CHECK(q.submit(r, now_ns(), &reqs[i].ticket, &err) == PSS_OK);
    if (i % 97 == 50) {  // cancel one that is probably still queued
      if (q.cancel(reqs[i].ticket, &err) == PSS_OK) cancelled.push_back(reqs[i].ticket);
    }
    if (i % 40 == 39) std::this_thread::sleep_for(std::chrono::milliseconds(2));
  }
  int ok = 0, failed = 0, was_cancelled = 0;
  for (int i = 0; i < n_req; ++i) {
    std::string err;
    pss_status st = PSS_OK;
    CHECK(q.wait(reqs[i].ticket, &st, &err) == PSS_OK);
    reqs[i].result = st;
    if (st == PSS_OK) {
      ++ok;
      std::vector<int64_t> k;
      std::vector<uint32_t> v;
      reference(reqs[i], &k, &v);
      CHECK(k == reqs[i].out);
      CHECK(v == reqs[i].vout);
    } else if (st == PSS_ERR_CANCELLED) {
      ++was_cancelled;
      CHECK(std::find(cancelled.begin(), cancelled.end(), reqs[i].ticket) != cancelled.end());
    } else {
      CHECK(st == PSS_ERR_HIP);
      ++failed;
    }
    // a collected ticket is forgotten
    int done = 0;
    CHECK(q.poll(reqs[i].ticket, &done, nullptr, &err) == PSS_ERR_INVALID);
  }
  pss_stats s{};
  q.stats(&s);
  CHECK(failed > 0);  // the batch failed on purpose held at least one request
  CHECK((int)s.failed == failed);
  CHECK((int)s.completed == ok);
  CHECK((int)s.cancelled == was_cancelled);
  CHECK(s.submitted == (uint64_t)n_req);
  CHECK(s.rejected == 1);
  CHECK(s.budget_in_use == 0);
  CHECK(s.queued == 0);
  CHECK(s.mean_batch_requests > 1.0);
  CHECK(ex.over_share.load() == 0);
  CHECK(s.latency_p50_ms <= s.latency_p99_ms && s.latency_p99_ms <= s.latency_max_ms);
  CHECK(s.keys_per_s > 0);

  // the same requests alone (a fresh queue, one request per batch) give the
  // same outputs as in the mix
  {
    pss::RequestQueue q1(share, fake_batch_bytes);
    Executor ex1;
    ex1.q = &q1;
    ex1.start(1);
    for (int i = 0; i < n_req; i += 7) {
      if (reqs[i].result != PSS_OK) continue;
      HostReq alone = reqs[i];
      std::fill(alone.out.begin(), alone.out.end(), 0);
      std::fill(alone.vout.begin(), alone.vout.end(), 0);
      pss_request r = make_request(alone);
      uint64_t t = 0;
      std::string err;
      pss_status st = PSS_OK;
      CHECK(q1.submit(r, now_ns(), &t, &err) == PSS_OK);
      CHECK(q1.wait(t, &st, &err) == PSS_OK && st == PSS_OK);
      CHECK(alone.out == reqs[i].out && alone.vout == reqs[i].vout);
    }
    q1.stop();
    ex1.join();
  }

  // shutdown with requests queued: they complete as cancelled
  {
    pss::RequestQueue q2(share, fake_batch_bytes);  // no workers: nothing runs
    std::vector<uint64_t> t(5);
    for (int i = 0; i < 5; ++i) {
      pss_request r = make_request(reqs[i]);
      std::string err;
      CHECK(q2.submit(r, now_ns(), &t[i], &err) == PSS_OK);
    }
    q2.stop();
    for (int i = 0; i < 5; ++i) {
      std::string err;
      pss_status st = PSS_OK;
      CHECK(q2.wait(t[i], &st, &err) == PSS_OK && st == PSS_ERR_CANCELLED);
    }
    pss_request r = make_request(reqs[0]);
    uint64_t t2 = 0;
    std::string err;
    CHECK(q2.submit(r, now_ns(), &t2, &err) == PSS_ERR_INVALID);
  }

  q.stop();
  ex.join();
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("serving queue checks passed: %d ok, %d failed on purpose, %d cancelled, "
              "%.2f requests per batch\n",
              ok, failed, was_cancelled, s.mean_batch_requests);
  return 0;
}
