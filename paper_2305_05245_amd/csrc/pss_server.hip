// Serving loop of libpss (pss_server_*): a first-come-first-served queue of
// independent sort requests, continuous batching into per-stream workers, and
// latency / throughput accounting.  Every batch is one segmented sort (one
// segment per request) between a gather kernel, which packs the requests'
// inputs into the worker's batch buffer, and a scatter kernel, which copies
// the sorted segments back to each request's outputs.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pss.h"
#include "pss_internal.hpp"

namespace {

constexpr uint32_t kCopyThreads = 256;
constexpr uint32_t kCopyItems = 16;
constexpr uint64_t kCopyChunk = (uint64_t)kCopyThreads * kCopyItems;  // elements per workgroup
constexpr uint32_t kMaxBatchRequests = 8192;
constexpr uint32_t kMaxWorkers = 16;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

// Per-batch tables, uploaded once per batch.  Pointers travel as uint64.
struct CopyTables {
  const uint64_t *seg_off;    // m + 1: request i occupies [seg_off[i], seg_off[i+1]) of the batch
  const uint64_t *chunk_off;  // m + 1: prefix sums of ceil(n_i / kCopyChunk)
  const uint64_t *kptr;       // m: request key arrays (inputs for gather, outputs for scatter)
  const uint64_t *vptr;       // m: request value arrays (unused for keys-only batches)
  uint32_t m;
};

// One workgroup copies one chunk of up to kCopyChunk elements of one request,
// between the request's own array and its place in the batch buffer.
template <typename T, bool KV, bool GATHER>
__global__ __launch_bounds__(kCopyThreads) void batch_copy_kernel(CopyTables t, T *batch_keys,
                                                                  uint32_t *batch_vals) {
  const uint64_t c = blockIdx.x;
  uint32_t lo = 0, hi = t.m;  // largest s with chunk_off[s] <= c (the grid is chunk_off[m])
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (t.chunk_off[mid] <= c) lo = mid; else hi = mid;
  }
  const uint32_t s = lo;
  const uint64_t first = (c - t.chunk_off[s]) * kCopyChunk;
  const uint64_t n_s = t.seg_off[s + 1] - t.seg_off[s];
  const uint64_t len = n_s - first < kCopyChunk ? n_s - first : kCopyChunk;
  const uint64_t base = t.seg_off[s] + first;
  T *req_k = reinterpret_cast<T *>(t.kptr[s]) + first;
  T *bat_k = batch_keys + base;
  uint32_t *req_v = KV ? reinterpret_cast<uint32_t *>(t.vptr[s]) + first : nullptr;
  uint32_t *bat_v = KV ? batch_vals + base : nullptr;
  // every load of the chunk first (all in flight together), then the stores
  T tk[kCopyItems];
  uint32_t tv[KV ? kCopyItems : 1];
#pragma unroll
  for (uint32_t u = 0; u < kCopyItems; ++u) {
    const uint64_t i = (uint64_t)u * kCopyThreads + threadIdx.x;
    if (i < len) {
      tk[u] = GATHER ? req_k[i] : bat_k[i];
      if constexpr (KV) tv[u] = GATHER ? req_v[i] : bat_v[i];
    }
  }
#pragma unroll
  for (uint32_t u = 0; u < kCopyItems; ++u) {
    const uint64_t i = (uint64_t)u * kCopyThreads + threadIdx.x;
    if (i < len) {
      (GATHER ? bat_k : req_k)[i] = tk[u];
      if constexpr (KV) (GATHER ? bat_v : req_v)[i] = tv[u];
    }
  }
}

template <typename T, bool KV>
hipError_t launch_copy(bool gather, const CopyTables &t, uint64_t chunks, void *bk, uint32_t *bv,
                       hipStream_t s) {
  if (chunks == 0) return hipSuccess;
  if (gather)
    hipLaunchKernelGGL((batch_copy_kernel<T, KV, true>), dim3((uint32_t)chunks), dim3(kCopyThreads),
                       0, s, t, (T *)bk, bv);
  else
    hipLaunchKernelGGL((batch_copy_kernel<T, KV, false>), dim3((uint32_t)chunks), dim3(kCopyThreads),
                       0, s, t, (T *)bk, bv);
  return hipGetLastError();
}

hipError_t launch_batch_copy(bool gather, int kbytes, bool kv, const CopyTables &t, uint64_t chunks,
                             void *bk, uint32_t *bv, hipStream_t s) {
  if (kbytes == 8)
    return kv ? launch_copy<uint64_t, true>(gather, t, chunks, bk, bv, s)
              : launch_copy<uint64_t, false>(gather, t, chunks, bk, bv, s);
  return kv ? launch_copy<uint32_t, true>(gather, t, chunks, bk, bv, s)
            : launch_copy<uint32_t, false>(gather, t, chunks, bk, bv, s);
}

enum ReqState { kQueued = 0, kLaunched = 1, kDone = 2 };

struct Req {
  pss_request r;
  uint64_t arrival = 0;
  int state = kQueued;
  pss_status result = PSS_OK;
};

// Device layout of one batch inside a worker's share of the budget.
struct BatchLayout {
  size_t stage_k = 0, stage_v = 0, out_k = 0, out_v = 0, tables = 0, ws = 0, ws_bytes = 0, total = 0;
};

pss_status batch_layout(pss_key_t key, pss_val_t val, uint64_t n, uint32_t m, uint64_t max_len,
                        const pss_tuning &tu, BatchLayout *L) {
  const size_t kb = (size_t)pss::key_bytes((int)key);
  const bool kv = val == PSS_VAL_U32;
  pss_tuning t = tu;
  t.max_seg_len = std::max<uint64_t>(max_len, 1);
  size_t ws = 0;
  const pss_status st = pss_segmented_workspace_bytes(nullptr, key, val, n, m, &t, &ws);
  if (st != PSS_OK) return st;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  L->tables = take(((size_t)2 * (m + 1) + (size_t)4 * m) * 8);
  L->stage_k = take(n * kb);
  L->stage_v = kv ? take(n * 4) : 0;
  L->out_k = take(n * kb);
  L->out_v = kv ? take(n * 4) : 0;
  L->ws = take(ws);
  L->ws_bytes = ws;
  L->total = off;
  return PSS_OK;
}

struct Worker {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  pss_ctx *ctx = nullptr;
  char *slab = nullptr;
  uint64_t *host_tables = nullptr;  // pinned, sized for kMaxBatchRequests
  std::thread th;
};

}  // namespace

struct pss_server {
  int device = 0;
  size_t budget = 0, share = 0;
  pss_tuning tuning{2048, 4096, 0};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;  // tickets in arrival order (cancelled ones are skipped)
  std::unordered_map<uint64_t, Req> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<std::unique_ptr<Worker>> workers;
  // counters
  uint64_t submitted = 0, completed = 0, rejected = 0, cancelled = 0, failed = 0;
  uint64_t batches = 0, batch_requests = 0, batch_keys = 0, keys_completed = 0;
  uint64_t first_arrival = 0, last_done = 0;
  // latencies of the most recent kLatencySamples completed requests (a ring)
  static constexpr size_t kLatencySamples = size_t(1) << 22;
  std::vector<float> latency_ms;
  size_t latency_next = 0;
  void record_latency(float ms) {
    if (latency_ms.size() < kLatencySamples) {
      latency_ms.push_back(ms);
    } else {
      latency_ms[latency_next] = ms;
      latency_next = (latency_next + 1) % kLatencySamples;
    }
  }
};

namespace {

pss_status server_fail(pss_status s, const std::string &msg) {
  pss::set_thread_error(msg.c_str());
  return s;
}

// Take, in arrival order, the queued requests of the head's types that fit
// one worker's share.  Called with the lock held.
void form_batch(pss_server *sv, std::vector<uint64_t> &batch) {
  batch.clear();
  std::deque<uint64_t> keep;
  bool have_type = false, closed = false;
  pss_key_t key = PSS_U32;
  pss_val_t val = PSS_VAL_NONE;
  uint64_t total = 0, max_len = 0;
  while (!sv->queue.empty()) {
    const uint64_t tk = sv->queue.front();
    sv->queue.pop_front();
    auto it = sv->reqs.find(tk);
    if (it == sv->reqs.end() || it->second.state != kQueued) continue;  // cancelled
    Req &q = it->second;
    if (!have_type) {
      key = q.r.key;
      val = q.r.val;
      have_type = true;
    }
    bool take = false;
    if (!closed && q.r.key == key && q.r.val == val && batch.size() < kMaxBatchRequests) {
      BatchLayout L;
      const uint64_t ml = std::max(max_len, q.r.n);
      if (batch_layout(key, val, total + q.r.n, (uint32_t)batch.size() + 1, ml, sv->tuning, &L) ==
              PSS_OK &&
          L.total <= sv->share) {
        take = true;
        total += q.r.n;
        max_len = ml;
      } else {
        closed = true;  // keep first-come-first-served order within the type
      }
    }
    if (take) {
      q.state = kLaunched;
      batch.push_back(tk);
    } else {
      keep.push_back(tk);
    }
  }
  sv->queue.swap(keep);
}

// Sort one batch on the worker's stream and wait for it.
pss_status run_batch(pss_server *sv, Worker *w, const std::vector<pss_request> &rs) {
  const uint32_t m = (uint32_t)rs.size();
  const pss_key_t key = rs[0].key;
  const pss_val_t val = rs[0].val;
  const bool kv = val == PSS_VAL_U32;
  const int kb = pss::key_bytes((int)key);
  uint64_t n = 0, max_len = 0, chunks = 0;
  uint64_t *h = w->host_tables;
  uint64_t *h_seg = h, *h_chunk = h + (m + 1), *h_kin = h + 2 * (m + 1), *h_vin = h_kin + m;
  uint64_t *h_kout = h_vin + m, *h_vout = h_kout + m;
  h_seg[0] = 0;
  h_chunk[0] = 0;
  for (uint32_t i = 0; i < m; ++i) {
    n += rs[i].n;
    max_len = std::max(max_len, rs[i].n);
    chunks += (rs[i].n + kCopyChunk - 1) / kCopyChunk;
    h_seg[i + 1] = n;
    h_chunk[i + 1] = chunks;
    h_kin[i] = (uint64_t)(uintptr_t)rs[i].keys_in;
    h_vin[i] = (uint64_t)(uintptr_t)rs[i].vals_in;
    h_kout[i] = (uint64_t)(uintptr_t)rs[i].keys_out;
    h_vout[i] = (uint64_t)(uintptr_t)rs[i].vals_out;
  }
  BatchLayout L;
  pss_status st = batch_layout(key, val, n, m, max_len, sv->tuning, &L);
  if (st != PSS_OK) return st;
  if (L.total > sv->share) return server_fail(PSS_ERR_BUDGET, "batch exceeds the worker's share");
  char *base = w->slab;
  uint64_t *d = (uint64_t *)(base + L.tables);
  hipError_t e;
  hipStream_t s = w->stream;
  const size_t tbytes = ((size_t)2 * (m + 1) + (size_t)4 * m) * 8;
  if ((e = hipMemcpyAsync(d, h, tbytes, hipMemcpyHostToDevice, s)) != hipSuccess)
    return server_fail(PSS_ERR_HIP, std::string("batch tables: ") + hipGetErrorString(e));
  CopyTables in{d, d + (m + 1), d + 2 * (m + 1), d + 2 * (m + 1) + m, m};
  CopyTables out{d, d + (m + 1), d + 2 * (m + 1) + 2 * m, d + 2 * (m + 1) + 3 * m, m};
  void *stage_k = base + L.stage_k, *out_k = base + L.out_k;
  uint32_t *stage_v = kv ? (uint32_t *)(base + L.stage_v) : nullptr;
  uint32_t *out_v = kv ? (uint32_t *)(base + L.out_v) : nullptr;
  if ((e = launch_batch_copy(true, kb, kv, in, chunks, stage_k, stage_v, s)) != hipSuccess)
    return server_fail(PSS_ERR_HIP, std::string("gather launch: ") + hipGetErrorString(e));
  pss_tuning tu = sv->tuning;
  tu.max_seg_len = std::max<uint64_t>(max_len, 1);
  st = pss_segmented_sort(w->ctx, key, val, stage_k, out_k, stage_v, out_v, n, d, m, &tu,
                          base + L.ws, L.ws_bytes, s);
  if (st != PSS_OK) return server_fail(st, pss_last_error(w->ctx));
  if ((e = launch_batch_copy(false, kb, kv, out, chunks, out_k, out_v, s)) != hipSuccess)
    return server_fail(PSS_ERR_HIP, std::string("scatter launch: ") + hipGetErrorString(e));
  if ((e = hipEventRecord(w->done, s)) != hipSuccess ||
      (e = hipEventSynchronize(w->done)) != hipSuccess)
    return server_fail(PSS_ERR_HIP, std::string("batch completion: ") + hipGetErrorString(e));
  return PSS_OK;
}

void worker_loop(pss_server *sv, Worker *w) {
  hipSetDevice(sv->device);
  std::vector<uint64_t> batch;
  std::vector<pss_request> rs;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
      if (sv->stop) return;
      form_batch(sv, batch);
      if (batch.empty()) continue;
      rs.clear();
      for (uint64_t tk : batch) rs.push_back(sv->reqs[tk].r);
      if (!sv->queue.empty()) sv->cv_work.notify_one();
    }
    const pss_status st = run_batch(sv, w, rs);
    const uint64_t t = now_ns();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      uint64_t keys = 0;
      for (uint64_t tk : batch) {
        Req &q = sv->reqs[tk];
        q.state = kDone;
        q.result = st;
        if (st == PSS_OK) {
          ++sv->completed;
          sv->keys_completed += q.r.n;
          keys += q.r.n;
          sv->record_latency((float)((double)(t - q.arrival) * 1e-6));
          if (sv->first_arrival == 0 || q.arrival < sv->first_arrival) sv->first_arrival = q.arrival;
        } else {
          ++sv->failed;
        }
      }
      ++sv->batches;
      sv->batch_requests += batch.size();
      sv->batch_keys += keys;
      sv->last_done = std::max(sv->last_done, t);
    }
    sv->cv_done.notify_all();
  }
}

void destroy_workers(pss_server *sv) {
  for (auto &w : sv->workers) {
    if (w->th.joinable()) w->th.join();
    if (w->done) hipEventDestroy(w->done);
    if (w->stream) hipStreamDestroy(w->stream);
    if (w->slab) hipFree(w->slab);
    if (w->host_tables) hipHostFree(w->host_tables);
    if (w->ctx) pss_destroy(w->ctx);
  }
  sv->workers.clear();
}

}  // namespace

extern "C" {

pss_status pss_server_create(pss_ctx *ctx, size_t hbm_budget_bytes, uint32_t max_streams,
                             const pss_tuning *tuning, pss_server **out) {
  if (!ctx || !out) return server_fail(PSS_ERR_INVALID, "null context or output pointer");
  *out = nullptr;
  if (max_streams == 0 || max_streams > kMaxWorkers)
    return server_fail(PSS_ERR_INVALID, "max_streams must be 1..16");
  if (tuning && (tuning->small_max_2k > 2048 || tuning->small_max_4k > 4096 ||
                 tuning->small_max_2k > tuning->small_max_4k))
    return server_fail(PSS_ERR_INVALID, "tuning: need small_max_2k <= small_max_4k, <= 2048, <= 4096");
  const size_t share = hbm_budget_bytes / max_streams / kAlign * kAlign;
  if (share < ((size_t)1 << 20))
    return server_fail(PSS_ERR_BUDGET, "budget below 1 MiB per stream");
  std::unique_ptr<pss_server> sv(new pss_server());
  sv->device = pss::ctx_device(ctx);
  sv->budget = hbm_budget_bytes;
  sv->share = share;
  if (tuning) sv->tuning = *tuning;
  sv->tuning.max_seg_len = 0;
  for (uint32_t i = 0; i < max_streams; ++i) {
    std::unique_ptr<Worker> w(new Worker());
    hipError_t e;
    pss_status st = pss_create(sv->device, &w->ctx);
    if (st != PSS_OK) {
      sv->workers.push_back(std::move(w));
      destroy_workers(sv.get());
      return st;
    }
    if ((e = hipSetDevice(sv->device)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&w->done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipMalloc((void **)&w->slab, share)) != hipSuccess ||
        (e = hipHostMalloc((void **)&w->host_tables,
                           ((size_t)2 * (kMaxBatchRequests + 1) + (size_t)4 * kMaxBatchRequests) * 8,
                           hipHostMallocDefault)) != hipSuccess) {
      sv->workers.push_back(std::move(w));
      destroy_workers(sv.get());
      return server_fail(e == hipErrorOutOfMemory ? PSS_ERR_BUDGET : PSS_ERR_HIP,
                         std::string("server resources: ") + hipGetErrorString(e));
    }
    sv->workers.push_back(std::move(w));
  }
  for (auto &w : sv->workers) w->th = std::thread(worker_loop, sv.get(), w.get());
  *out = sv.release();
  return PSS_OK;
}

pss_status pss_submit(pss_server *sv, const pss_request *req, uint64_t *ticket) {
  if (!sv || !req || !ticket) return server_fail(PSS_ERR_INVALID, "null argument");
  *ticket = 0;
  const pss_request &r = *req;
  if ((int)r.key < 0 || (int)r.key > 5) return server_fail(PSS_ERR_INVALID, "unknown key type");
  if (r.val != PSS_VAL_NONE && r.val != PSS_VAL_U32)
    return server_fail(PSS_ERR_INVALID, "unknown value type");
  if (r.n > PSS_MAX_KEYS) return server_fail(PSS_ERR_UNSUPPORTED, "n >= 2^31 is not supported");
  const size_t kb = (size_t)pss::key_bytes((int)r.key);
  if (r.n > 0) {
    if (!r.keys_in || !r.keys_out) return server_fail(PSS_ERR_INVALID, "null key pointer");
    const uintptr_t a = (uintptr_t)r.keys_in, b = (uintptr_t)r.keys_out;
    if ((a | b) % kb) return server_fail(PSS_ERR_INVALID, "key arrays not naturally aligned");
    if (a < b + r.n * kb && b < a + r.n * kb)
      return server_fail(PSS_ERR_INVALID, "keys_in and keys_out overlap");
    if (r.val == PSS_VAL_U32) {
      if (!r.vals_in || !r.vals_out) return server_fail(PSS_ERR_INVALID, "null value pointer");
      const uintptr_t c = (uintptr_t)r.vals_in, d = (uintptr_t)r.vals_out;
      if ((c | d) % 4) return server_fail(PSS_ERR_INVALID, "value arrays not aligned");
      if (c < d + r.n * 4 && d < c + r.n * 4)
        return server_fail(PSS_ERR_INVALID, "vals_in and vals_out overlap");
    }
    BatchLayout L;
    const pss_status st = batch_layout(r.key, r.val, r.n, 1, r.n, sv->tuning, &L);
    if (st != PSS_OK || L.total > sv->share) {
      std::lock_guard<std::mutex> lk(sv->mu);
      ++sv->rejected;
      char m[200];
      snprintf(m, sizeof m, "request of %llu keys needs %zu bytes, above the %zu bytes per stream",
               (unsigned long long)r.n, L.total, sv->share);
      return server_fail(st != PSS_OK ? st : PSS_ERR_BUDGET, m);
    }
  }
  const uint64_t t = now_ns();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return server_fail(PSS_ERR_INVALID, "server is shutting down");
    const uint64_t tk = sv->next_ticket++;
    Req q;
    q.r = r;
    q.arrival = r.arrival_ns ? r.arrival_ns : t;
    ++sv->submitted;
    if (r.n == 0) {
      q.state = kDone;
      ++sv->completed;
      sv->record_latency((float)((double)(t > q.arrival ? t - q.arrival : 0) * 1e-6));
    } else {
      sv->queue.push_back(tk);
    }
    sv->reqs.emplace(tk, q);
    *ticket = tk;
  }
  if (r.n) sv->cv_work.notify_one();
  else sv->cv_done.notify_all();
  return PSS_OK;
}

pss_status pss_poll(pss_server *sv, uint64_t ticket, int *done, pss_status *result) {
  if (!sv || !done) return server_fail(PSS_ERR_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return server_fail(PSS_ERR_INVALID, "unknown ticket");
  *done = it->second.state == kDone;
  if (*done) {
    if (result) *result = it->second.result;
    sv->reqs.erase(it);
  }
  return PSS_OK;
}

pss_status pss_wait(pss_server *sv, uint64_t ticket, pss_status *result) {
  if (!sv) return server_fail(PSS_ERR_INVALID, "null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return server_fail(PSS_ERR_INVALID, "unknown ticket");
  sv->cv_done.wait(lk, [&] {
    it = sv->reqs.find(ticket);
    return it == sv->reqs.end() || it->second.state == kDone;
  });
  if (it == sv->reqs.end()) return server_fail(PSS_ERR_INVALID, "ticket collected by another call");
  if (result) *result = it->second.result;
  sv->reqs.erase(it);
  return PSS_OK;
}

pss_status pss_cancel(pss_server *sv, uint64_t ticket) {
  if (!sv) return server_fail(PSS_ERR_INVALID, "null server");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return server_fail(PSS_ERR_INVALID, "unknown ticket");
    if (it->second.state != kQueued)
      return server_fail(PSS_ERR_BUSY, "request already launched or finished");
    it->second.state = kDone;  // form_batch drops it from the queue
    it->second.result = PSS_ERR_CANCELLED;
    ++sv->cancelled;
  }
  sv->cv_done.notify_all();
  return PSS_OK;
}

pss_status pss_server_stats(pss_server *sv, pss_stats *out) {
  if (!sv || !out) return server_fail(PSS_ERR_INVALID, "null argument");
  std::vector<float> lat;
  pss_stats s{};
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    s.submitted = sv->submitted;
    s.completed = sv->completed;
    s.rejected = sv->rejected;
    s.cancelled = sv->cancelled;
    s.failed = sv->failed;
    s.batches = sv->batches;
    s.keys_completed = sv->keys_completed;
    if (sv->last_done > sv->first_arrival && sv->first_arrival)
      s.keys_per_s = (double)sv->keys_completed / ((double)(sv->last_done - sv->first_arrival) * 1e-9);
    if (sv->batches) {
      s.mean_batch_requests = (double)sv->batch_requests / (double)sv->batches;
      s.mean_batch_keys = (double)sv->batch_keys / (double)sv->batches;
    }
    lat = sv->latency_ms;
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
  return PSS_OK;
}

pss_status pss_server_reset_stats(pss_server *sv) {
  if (!sv) return server_fail(PSS_ERR_INVALID, "null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->submitted = sv->completed = sv->rejected = sv->cancelled = sv->failed = 0;
  sv->batches = sv->batch_requests = sv->batch_keys = sv->keys_completed = 0;
  sv->first_arrival = sv->last_done = 0;
  sv->latency_ms.clear();
  sv->latency_next = 0;
  return PSS_OK;
}

void pss_server_destroy(pss_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    for (uint64_t tk : sv->queue) {
      auto it = sv->reqs.find(tk);
      if (it != sv->reqs.end() && it->second.state == kQueued) {
        it->second.state = kDone;
        it->second.result = PSS_ERR_CANCELLED;
      }
    }
    sv->queue.clear();
  }
  sv->cv_work.notify_all();
  sv->cv_done.notify_all();
  destroy_workers(sv);
  delete sv;
}

}  // extern "C"
