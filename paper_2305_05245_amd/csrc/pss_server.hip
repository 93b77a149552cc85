// Serving loop of libpss (pss_server_*): a first-come-first-served queue of
// independent sort requests (pss_queue.hpp: admission, batching, accounting),
// continuous batching into per-stream workers.  Every batch is one segmented
// sort (one segment per request) between a gather kernel, which packs the
// requests' inputs into the worker's batch buffer, and a scatter kernel, which
// copies the sorted segments back to each request's outputs.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <cstdio>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pss.h"
#include "pss_internal.hpp"
#include "pss_queue.hpp"

namespace {

constexpr uint32_t kCopyThreads = 256;
constexpr uint32_t kCopyItems = 16;
constexpr uint64_t kCopyChunk = (uint64_t)kCopyThreads * kCopyItems;  // elements per workgroup
constexpr uint32_t kMaxBatchRequests = pss::RequestQueue::kMaxBatchRequests;
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
  uint32_t *host_error = nullptr;   // pinned: the device error word after a batch
  std::thread th;
};

}  // namespace

struct pss_server {
  int device = 0;
  size_t budget = 0, share = 0;
  pss_tuning tuning{2048, 4096, 0, 0, 0};
  std::unique_ptr<pss::RequestQueue> queue;
  std::vector<std::unique_ptr<Worker>> workers;
};

namespace {

pss_status server_fail(pss_status s, const std::string &msg) {
  pss::set_thread_error(msg.c_str());
  return s;
}

// Sort one batch on the worker's stream and wait for it.  Every exit waits
// for whatever the batch queued, so its requests' buffers, the worker's slab
// and its pinned tables are idle once the batch is reported done.
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
  hipStream_t s = w->stream;
  // after something was queued: wait for it, then report the failure
  auto abort_batch = [&](pss_status code, const std::string &msg) {
    (void)hipStreamSynchronize(s);
    return server_fail(code, msg);
  };
  const size_t tbytes = ((size_t)2 * (m + 1) + (size_t)4 * m) * 8;
  hipError_t e = pss::inject_fault(pss::kInjectLaunch)
                     ? hipErrorLaunchFailure
                     : hipMemcpyAsync(d, h, tbytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess)
    return abort_batch(PSS_ERR_HIP, std::string("batch tables: ") + hipGetErrorString(e));
  CopyTables in{d, d + (m + 1), d + 2 * (m + 1), d + 2 * (m + 1) + m, m};
  CopyTables out{d, d + (m + 1), d + 2 * (m + 1) + 2 * m, d + 2 * (m + 1) + 3 * m, m};
  void *stage_k = base + L.stage_k, *out_k = base + L.out_k;
  uint32_t *stage_v = kv ? (uint32_t *)(base + L.stage_v) : nullptr;
  uint32_t *out_v = kv ? (uint32_t *)(base + L.out_v) : nullptr;
  e = pss::inject_fault(pss::kInjectLaunch)
          ? hipErrorLaunchFailure
          : launch_batch_copy(true, kb, kv, in, chunks, stage_k, stage_v, s);
  if (e != hipSuccess)
    return abort_batch(PSS_ERR_HIP, std::string("gather launch: ") + hipGetErrorString(e));
  pss_tuning tu = sv->tuning;
  tu.max_seg_len = std::max<uint64_t>(max_len, 1);
  st = pss_segmented_sort(w->ctx, key, val, stage_k, out_k, stage_v, out_v, n, d, m, &tu,
                          base + L.ws, L.ws_bytes, s);
  if (st != PSS_OK) return abort_batch(st, pss_last_error(w->ctx));
  e = pss::inject_fault(pss::kInjectLaunch)
          ? hipErrorLaunchFailure
          : launch_batch_copy(false, kb, kv, out, chunks, out_k, out_v, s);
  if (e != hipSuccess)
    return abort_batch(PSS_ERR_HIP, std::string("scatter launch: ") + hipGetErrorString(e));
  // the device error word once the batch's kernels are done
  if ((e = pss::read_device_error_async(w->host_error, s)) != hipSuccess)
    return abort_batch(PSS_ERR_HIP, std::string("error word copy: ") + hipGetErrorString(e));
  if ((e = hipEventRecord(w->done, s)) != hipSuccess ||
      (e = hipEventSynchronize(w->done)) != hipSuccess)
    return abort_batch(PSS_ERR_HIP, std::string("batch completion: ") + hipGetErrorString(e));
  if (*w->host_error != 0) {
    char msg[120];
    snprintf(msg, sizeof msg, "device error word 0x%x after the batch (see pss_device_check)",
             *w->host_error);
    return server_fail(PSS_ERR_HIP, msg);
  }
  return PSS_OK;
}

void worker_loop(pss_server *sv, Worker *w) {
  (void)hipSetDevice(sv->device);
  std::vector<uint64_t> batch;
  std::vector<pss_request> rs;
  size_t bytes = 0;
  while (sv->queue->next_batch(&batch, &rs, &bytes)) {
    const pss_status st = run_batch(sv, w, rs);
    sv->queue->finish_batch(batch, st, now_ns(), bytes);
  }
}

void destroy_workers(pss_server *sv) {
  for (auto &w : sv->workers) {
    if (w->th.joinable()) w->th.join();
    if (w->done) (void)hipEventDestroy(w->done);
    if (w->stream) (void)hipStreamDestroy(w->stream);
    if (w->slab) (void)hipFree(w->slab);
    if (w->host_tables) (void)hipHostFree(w->host_tables);
    if (w->host_error) (void)hipHostFree(w->host_error);
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
  if (tuning && tuning->fan_log2 != 0 && tuning->fan_log2 != 5 && tuning->fan_log2 != 6)
    return server_fail(PSS_ERR_INVALID, "tuning: fan_log2 must be 0, 5 or 6");
  const size_t share = hbm_budget_bytes / max_streams / kAlign * kAlign;
  if (share < ((size_t)1 << 20))
    return server_fail(PSS_ERR_BUDGET, "budget below 1 MiB per stream");
  std::unique_ptr<pss_server> sv(new pss_server());
  sv->device = pss::ctx_device(ctx);
  sv->budget = hbm_budget_bytes;
  sv->share = share;
  if (tuning) sv->tuning = *tuning;
  sv->tuning.max_seg_len = 0;
  const pss_tuning tu = sv->tuning;
  sv->queue.reset(new pss::RequestQueue(
      share, [tu](pss_key_t key, pss_val_t val, uint64_t n, uint32_t m, uint64_t max_len,
                  size_t *bytes) {
        BatchLayout L;
        if (batch_layout(key, val, n, m, max_len, tu, &L) != PSS_OK) return false;
        *bytes = L.total;
        return true;
      }));
  for (uint32_t i = 0; i < max_streams; ++i) {
    std::unique_ptr<Worker> w(new Worker());
    hipError_t e;
    pss_status st = pss_create(sv->device, &w->ctx);
    if (st != PSS_OK) {
      sv->workers.push_back(std::move(w));
      destroy_workers(sv.get());
      return st;
    }
    const size_t tables = ((size_t)2 * (kMaxBatchRequests + 1) + (size_t)4 * kMaxBatchRequests) * 8;
    // allocations, with the fault injection of pss_debug_inject (an armed
    // allocation fails as out of memory)
    auto injected = [] { return pss::inject_fault(pss::kInjectAlloc); };
    if ((e = hipSetDevice(sv->device)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&w->done, hipEventDisableTiming)) != hipSuccess ||
        (e = injected() ? hipErrorOutOfMemory : hipMalloc((void **)&w->slab, share)) !=
            hipSuccess ||
        (e = injected() ? hipErrorOutOfMemory
                        : hipHostMalloc((void **)&w->host_tables, tables, hipHostMallocDefault)) !=
            hipSuccess ||
        (e = injected() ? hipErrorOutOfMemory
                        : hipHostMalloc((void **)&w->host_error, sizeof(uint32_t),
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
  if (!pss::valid_enum(r.key, 5)) return server_fail(PSS_ERR_INVALID, "unknown key type");
  if (!pss::valid_enum(r.val, 1)) return server_fail(PSS_ERR_INVALID, "unknown value type");
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
  }
  std::string err;
  const pss_status st = sv->queue->submit(r, now_ns(), ticket, &err);
  return st == PSS_OK ? st : server_fail(st, err);
}

pss_status pss_poll(pss_server *sv, uint64_t ticket, int *done, pss_status *result) {
  if (!sv || !done) return server_fail(PSS_ERR_INVALID, "null argument");
  std::string err;
  const pss_status st = sv->queue->poll(ticket, done, result, &err);
  return st == PSS_OK ? st : server_fail(st, err);
}

pss_status pss_wait(pss_server *sv, uint64_t ticket, pss_status *result) {
  if (!sv) return server_fail(PSS_ERR_INVALID, "null server");
  std::string err;
  const pss_status st = sv->queue->wait(ticket, result, &err);
  return st == PSS_OK ? st : server_fail(st, err);
}

pss_status pss_cancel(pss_server *sv, uint64_t ticket) {
  if (!sv) return server_fail(PSS_ERR_INVALID, "null server");
  std::string err;
  const pss_status st = sv->queue->cancel(ticket, &err);
  return st == PSS_OK ? st : server_fail(st, err);
}

pss_status pss_server_stats(pss_server *sv, pss_stats *out) {
  if (!sv || !out) return server_fail(PSS_ERR_INVALID, "null argument");
  sv->queue->stats(out);
  return PSS_OK;
}

pss_status pss_server_reset_stats(pss_server *sv) {
  if (!sv) return server_fail(PSS_ERR_INVALID, "null server");
  sv->queue->reset_stats();
  return PSS_OK;
}

void pss_server_destroy(pss_server *sv) {
  if (!sv) return;
  sv->queue->stop();
  destroy_workers(sv);
  delete sv;
}

}  // extern "C"
