// Serving loop: requests of different sizes and key types arrive over time;
// the server keeps their buffers on the device inside an arena the size of
// its HBM budget, admits a batch only when its buffers fit, groups pending
// requests of one key class into a batch (continuous batching: a batch is
// formed whenever a stream slot is free, from whatever is pending), sorts
// each batch with the enqueue-only segmented sort on the slot's stream (a
// batch of one request straight from the caller's buffers), so the host
// thread never waits on the device, and reports per-request completion
// with event-timed latency.  Several slots
// keep batches overlapping on the device.  The caller drives progress from
// one host thread (submit / poll / release).
#include <chrono>
#include <cstring>
#include <new>
#include <vector>

#include "host_internal.hpp"
#include "server.hpp"
#include "server_core.hpp"

using namespace ahs;

namespace {

int key_bytes(int dtype) { return (dtype == AHS_U32 || dtype == AHS_F32 || dtype == AHS_I32) ? 4 : 8; }
uint64_t a256(uint64_t x) { return (x + 255) / 256 * 256; }

struct BatchMem {
  uint64_t kin, kout, vin, vout, offs, chosen, status, desc, ws, total;
  size_t ws_bytes;
};

BatchMem batch_mem(uint64_t n, uint32_t nseg, int dtype, int pay) {
  BatchMem m;
  const uint64_t kb = (uint64_t)key_bytes(dtype);
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o += a256(bytes ? bytes : 1);
    return at;
  };
  m.kin = take(kb * n);
  m.kout = take(kb * n);
  m.vin = pay ? take(4 * n) : 0;
  m.vout = pay ? take(4 * n) : 0;
  m.offs = take(8 * ((uint64_t)nseg + 1));
  m.chosen = take(nseg);
  m.status = take(4);
  m.desc = take(sizeof(CopyDesc) * 2 * (uint64_t)nseg);
  m.ws_bytes = ahs_segmented_workspace_bytes(n, nseg, (ahs_dtype)dtype, pay);
  m.ws = take(m.ws_bytes);
  m.total = o;
  return m;
}

struct Batch {
  BatchPlan plan;
  BatchMem mem;
  uint64_t arena_off = 0;
  int slot = -1;
  hipEvent_t done = nullptr;
  uint32_t unreleased = 0;
};

struct Slot {
  hipStream_t s = nullptr;
  int64_t batch = -1;
  char* pinned = nullptr;  // offsets | descriptors | chosen | status
};

double host_ms(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct ahs_server {
  ahs_server_config cfg;
  ahs_context* ctx = nullptr;
  char* base = nullptr;  // arena of cfg.hbm_budget_bytes
  Arena arena;
  ServerCore core;
  std::vector<Slot> slots;
  std::unordered_map<int64_t, Batch> batches;
  int64_t next_batch = 0;
  std::vector<uint64_t> done_ids;  // finished, not yet returned by poll
  std::vector<hipEvent_t> events;  // pool for input-ready events
  std::chrono::steady_clock::time_point t0_host;
  hipEvent_t t0_ev = nullptr;
  uint64_t batches_run = 0, requests_batched = 0, peak_used = 0;
  size_t pinned_bytes = 0;

  hipEvent_t take_event() {
    if (!events.empty()) {
      hipEvent_t e = events.back();
      events.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    return e;
  }
};

namespace {

ahs_status launch_batch(ahs_server* S, int si, const BatchPlan& plan, uint64_t arena_off, const BatchMem& m) {
  ahs_context* ctx = S->ctx;
  Slot& sl = S->slots[si];
  const int64_t bid = S->next_batch++;
  Batch& B = S->batches[bid];
  B.plan = plan;
  B.mem = m;
  B.arena_off = arena_off;
  B.slot = si;
  B.unreleased = (uint32_t)plan.ids.size();
  S->core.start(plan, bid);
  char* b = S->base + arena_off;
  const uint32_t nseg = (uint32_t)plan.ids.size();
  const uint64_t kb = (uint64_t)key_bytes(plan.dtype);
  char* h_chosen = sl.pinned + S->pinned_bytes - a256(S->cfg.max_batch_requests) - 256;
  char* h_status = sl.pinned + S->pinned_bytes - 256;
  // host staging: offsets and copy descriptors
  uint64_t* h_offs = reinterpret_cast<uint64_t*>(sl.pinned);
  CopyDesc* h_desc = reinterpret_cast<CopyDesc*>(sl.pinned + a256(8 * ((uint64_t)S->cfg.max_batch_requests + 1)));
  uint32_t ndesc = 0;
  uint64_t max_bytes = 0;
  h_offs[0] = 0;
  // a batch of one request is sorted straight from the caller's buffers;
  // several are gathered into the batch's contiguous block first
  const void* kin = b + m.kin;
  const uint32_t* vin = plan.pay ? reinterpret_cast<const uint32_t*>(b + m.vin) : nullptr;
  if (nseg == 1) {
    const Request& r = S->core.reqs.at(plan.ids[0]);
    kin = r.kin;
    vin = plan.pay ? r.vin : nullptr;
  }
  for (uint32_t i = 0; i < nseg; ++i) {
    Request& r = S->core.reqs.at(plan.ids[i]);
    h_offs[i + 1] = h_offs[i] + r.n;
    if (r.ready) {
      if (ctx->check(hipStreamWaitEvent(sl.s, (hipEvent_t)r.ready, 0), "wait input") != AHS_OK) return AHS_E_DEVICE;
    }
    if (r.n && nseg > 1) {
      h_desc[ndesc++] = CopyDesc{r.kin, b + m.kin + kb * r.offset, kb * r.n};
      if (plan.pay) h_desc[ndesc++] = CopyDesc{r.vin, b + m.vin + 4 * r.offset, 4 * r.n};
      max_bytes = std::max<uint64_t>(max_bytes, kb * r.n);
    }
  }
  if (ctx->check(hipMemcpyAsync(b + m.offs, h_offs, 8 * ((size_t)nseg + 1), hipMemcpyHostToDevice, sl.s), "copy") !=
      AHS_OK)
    return AHS_E_DEVICE;
  if (ndesc) {
    if (ctx->check(hipMemcpyAsync(b + m.desc, h_desc, sizeof(CopyDesc) * ndesc, hipMemcpyHostToDevice, sl.s),
                   "copy") != AHS_OK)
      return AHS_E_DEVICE;
    if (ctx->check(launch_gather_copy(reinterpret_cast<const CopyDesc*>(b + m.desc), ndesc, max_bytes, sl.s),
                   "gather") != AHS_OK)
      return AHS_E_DEVICE;
  }
  ahs_status st = ahs_sort_segmented_async(
      ctx, kin, b + m.kout, vin,
      plan.pay ? reinterpret_cast<uint32_t*>(b + m.vout) : nullptr, reinterpret_cast<uint64_t*>(b + m.offs), nseg,
      plan.keys, plan.max_n, (ahs_dtype)plan.dtype, AHS_AUTO, &S->cfg.cfg, b + m.ws, m.ws_bytes, sl.s,
      reinterpret_cast<uint8_t*>(b + m.chosen), nullptr, reinterpret_cast<uint32_t*>(b + m.status));
  if (st != AHS_OK) return st;
  if (ctx->check(hipMemcpyAsync(h_chosen, b + m.chosen, nseg, hipMemcpyDeviceToHost, sl.s), "copy") != AHS_OK ||
      ctx->check(hipMemcpyAsync(h_status, b + m.status, 4, hipMemcpyDeviceToHost, sl.s), "copy") != AHS_OK)
    return AHS_E_DEVICE;
  if (!B.done && ctx->check(hipEventCreate(&B.done), "event") != AHS_OK) return AHS_E_DEVICE;
  if (ctx->check(hipEventRecord(B.done, sl.s), "record") != AHS_OK) return AHS_E_DEVICE;
  sl.batch = bid;
  S->batches_run += 1;
  S->requests_batched += nseg;
  S->peak_used = std::max(S->peak_used, S->arena.used());
  return AHS_OK;
}

// Retires finished batches and launches new ones into free slots.
ahs_status progress(ahs_server* S) {
  for (size_t si = 0; si < S->slots.size(); ++si) {
    Slot& sl = S->slots[si];
    if (sl.batch < 0) continue;
    Batch& B = S->batches.at(sl.batch);
    const hipError_t q = hipEventQuery(B.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return S->ctx->check(q, "batch completion");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, S->t0_ev, B.done);
    const double done_ms = (double)ms;
    const char* h_chosen = sl.pinned + S->pinned_bytes - a256(S->cfg.max_batch_requests) - 256;
    uint32_t dev_status = 0;
    memcpy(&dev_status, sl.pinned + S->pinned_bytes - 256, 4);
    for (size_t i = 0; i < B.plan.ids.size(); ++i) {
      const uint64_t id = B.plan.ids[i];
      Request& r = S->core.reqs.at(id);
      if (r.ready) {
        S->events.push_back((hipEvent_t)r.ready);
        r.ready = nullptr;
      }
      S->core.complete(id, dev_status ? (int)AHS_E_DEVICE : (int)AHS_OK, (uint8_t)h_chosen[i], done_ms);
      S->done_ids.push_back(id);
    }
    sl.batch = -1;
  }
  for (size_t si = 0; si < S->slots.size(); ++si) {
    if (S->slots[si].batch >= 0) continue;
    if (S->core.pending.empty()) break;
    const BatchPlan plan = S->core.plan_next();
    const BatchMem m = batch_mem(plan.keys, (uint32_t)plan.ids.size(), plan.dtype, plan.pay);
    if (m.total > S->arena.capacity() || (plan.ids.size() > 1 && S->arena.largest_free() < m.total)) {
      // the plan does not fit: take the oldest request alone, or fail it
      // when it cannot fit even in an empty arena
      const uint64_t id = plan.ids[0];
      Request& r = S->core.reqs.at(id);
      BatchPlan one;
      one.ids.push_back(id);
      one.keys = r.n;
      one.max_n = r.n;
      one.dtype = r.dtype;
      one.pay = r.pay;
      const BatchMem m1 = batch_mem(one.keys, 1, one.dtype, one.pay);
      if (m1.total > S->arena.capacity()) {
        if (r.ready) {
          S->events.push_back((hipEvent_t)r.ready);
          r.ready = nullptr;
        }
        S->core.fail_pending_head((int)AHS_E_OOM, host_ms(S->t0_host));
        S->done_ids.push_back(id);
        --si;  // the slot is still free: try the next request
        continue;
      }
      const uint64_t off1 = S->arena.alloc(m1.total);
      if (off1 == UINT64_MAX) break;  // admission: wait until a batch is released
      AHS_TRY(launch_batch(S, (int)si, one, off1, m1));
      continue;
    }
    const uint64_t off = S->arena.alloc(m.total);
    if (off == UINT64_MAX) break;  // admission: wait until a batch is released
    AHS_TRY(launch_batch(S, (int)si, plan, off, m));
  }
  return AHS_OK;
}

}  // namespace

extern "C" void ahs_server_config_init(ahs_server_config* c) {
  if (!c) return;
  memset(c, 0, sizeof *c);
  c->hbm_budget_bytes = 48000000000ull;
  c->max_batch_keys = 1ull << 26;
  c->max_batch_requests = 1024;
  c->slots = 4;
  ahs_config_init(&c->cfg, AHS_PRESET_GPU);
}

extern "C" ahs_status ahs_server_create(int device, const ahs_server_config* cfg, ahs_server** out) {
  if (!out) return AHS_E_INVALID_ARG;
  *out = nullptr;
  ahs_server_config c;
  if (cfg) c = *cfg; else ahs_server_config_init(&c);
  if (c.slots < 1 || c.slots > 16 || c.max_batch_requests < 1 || c.max_batch_requests > 65535 ||
      c.hbm_budget_bytes < (1u << 20) || c.cfg.use_model || c.cfg.k_count == 0)
    return AHS_E_INVALID_ARG;
  ahs_server* S = new (std::nothrow) ahs_server();
  if (!S) return AHS_E_OOM;
  S->cfg = c;
  ahs_status st = ahs_context_create(device, &S->ctx);
  if (st != AHS_OK) {
    delete S;
    return st;
  }
  auto fail = [&](ahs_status e) {
    ahs_server_destroy(S);
    return e;
  };
  if (hipMalloc(reinterpret_cast<void**>(&S->base), c.hbm_budget_bytes) != hipSuccess) {
    S->base = nullptr;
    return fail(AHS_E_OOM);
  }
  S->arena.reset(c.hbm_budget_bytes);
  S->core.lim.max_batch_keys = c.max_batch_keys ? c.max_batch_keys : (1ull << 26);
  S->core.lim.max_batch_requests = c.max_batch_requests;
  S->pinned_bytes = a256(8 * ((uint64_t)c.max_batch_requests + 1)) +
                    a256(sizeof(CopyDesc) * 2 * (uint64_t)c.max_batch_requests) + a256(c.max_batch_requests) + 256;
  S->slots.resize(c.slots);
  for (auto& sl : S->slots) {
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess) return fail(AHS_E_DEVICE);
    if (hipHostMalloc(reinterpret_cast<void**>(&sl.pinned), S->pinned_bytes, hipHostMallocDefault) != hipSuccess) {
      sl.pinned = nullptr;
      return fail(AHS_E_OOM);
    }
  }
  // the two clock origins are taken together: the GPU's (an event that has
  // completed) and the host's right after it
  if (hipEventCreate(&S->t0_ev) != hipSuccess) return fail(AHS_E_DEVICE);
  if (hipEventRecord(S->t0_ev, S->slots[0].s) != hipSuccess || hipEventSynchronize(S->t0_ev) != hipSuccess)
    return fail(AHS_E_DEVICE);
  S->t0_host = std::chrono::steady_clock::now();
  if (c.autotune) {
    for (int dt = 0; dt < NUM_KEY_KINDS; ++dt)
      for (int pay = 0; pay < 2; ++pay) {
        st = ahs_segmented_autotune(S->ctx, (ahs_dtype)dt, pay, S->slots[0].s, nullptr, nullptr);
        if (st != AHS_OK) return fail(st);
      }
  }
  *out = S;
  return AHS_OK;
}

extern "C" double ahs_server_now_ms(ahs_server* S) { return S ? host_ms(S->t0_host) : 0.0; }

extern "C" ahs_status ahs_server_submit(ahs_server* S, ahs_dtype dtype, uint64_t n, const void* d_keys,
                                        const uint32_t* d_vals, void* src_stream, double arrival_ms,
                                        uint64_t* out_id) {
  if (!S || !out_id) return AHS_E_INVALID_ARG;
  if ((int)dtype < 0 || (int)dtype > (int)AHS_I64) return S->ctx->fail(AHS_E_INVALID_ARG, "bad dtype");
  if (n >= (1ull << 32)) return S->ctx->fail(AHS_E_UNSUPPORTED, "requests hold fewer than 2^32 keys");
  if (n && !d_keys) return S->ctx->fail(AHS_E_INVALID_ARG, "null key pointer");
  if ((reinterpret_cast<uintptr_t>(d_keys) | reinterpret_cast<uintptr_t>(d_vals)) & 3u)
    return S->ctx->fail(AHS_E_INVALID_ARG, "buffers must be 4-byte aligned");
  const double now = host_ms(S->t0_host);
  const uint64_t id = S->core.add((int)dtype, d_vals ? 1 : 0, n, arrival_ms < 0 ? now : arrival_ms);
  Request& r = S->core.reqs.at(id);
  r.kin = d_keys;
  r.vin = d_vals;
  if (n) {
    hipEvent_t e = S->take_event();
    if (!e || S->ctx->check(hipEventRecord(e, (hipStream_t)src_stream), "record input") != AHS_OK)
      return AHS_E_DEVICE;
    r.ready = e;
  }
  *out_id = id;
  return S->cfg.lazy_dispatch ? AHS_OK : progress(S);
}

extern "C" ahs_status ahs_server_poll(ahs_server* S, ahs_server_result* out, uint32_t max, uint32_t* count,
                                      double wait_ms) {
  if (!S || !count || (max && !out)) return AHS_E_INVALID_ARG;
  *count = 0;
  const double until = host_ms(S->t0_host) + (wait_ms > 0 ? wait_ms : 0.0);
  for (;;) {
    AHS_TRY(progress(S));
    if (!S->done_ids.empty() || wait_ms <= 0 || host_ms(S->t0_host) >= until) break;
    bool busy = !S->core.pending.empty();
    for (auto& sl : S->slots) busy = busy || sl.batch >= 0;
    if (!busy) break;
  }
  uint32_t k = 0;
  while (k < max && k < S->done_ids.size()) {
    const Request& r = S->core.reqs.at(S->done_ids[k]);
    ahs_server_result& o = out[k];
    memset(&o, 0, sizeof o);
    o.id = r.id;
    o.status = r.status;
    o.chosen = r.chosen;
    o.n = r.n;
    o.dtype = (ahs_dtype)r.dtype;
    o.arrival_ms = r.arrival_ms;
    o.done_ms = r.done_ms;
    if (r.status == AHS_OK && r.batch >= 0) {
      const Batch& B = S->batches.at(r.batch);
      char* b = S->base + B.arena_off;
      o.d_keys_out = b + B.mem.kout + (uint64_t)key_bytes(r.dtype) * r.offset;
      o.d_vals_out = r.pay ? reinterpret_cast<const uint32_t*>(b + B.mem.vout + 4 * r.offset) : nullptr;
    }
    ++k;
  }
  S->done_ids.erase(S->done_ids.begin(), S->done_ids.begin() + k);
  *count = k;
  return AHS_OK;
}

extern "C" ahs_status ahs_server_release(ahs_server* S, uint64_t id) {
  if (!S) return AHS_E_INVALID_ARG;
  auto it = S->core.reqs.find(id);
  if (it == S->core.reqs.end()) return S->ctx->fail(AHS_E_INVALID_ARG, "unknown request %llu", (unsigned long long)id);
  Request& r = it->second;
  if (r.state == ReqState::PENDING || r.state == ReqState::RUNNING)
    return S->ctx->fail(AHS_E_INVALID_ARG, "request %llu has not completed", (unsigned long long)id);
  const int64_t b = r.batch;
  S->core.reqs.erase(it);
  if (b >= 0) {
    Batch& B = S->batches.at(b);
    if (--B.unreleased == 0) {
      S->arena.release(B.arena_off);
      if (B.done) (void)hipEventDestroy(B.done);
      S->batches.erase(b);
    }
  }
  return progress(S);
}

extern "C" ahs_status ahs_server_stats(ahs_server* S, ahs_server_statistics* out) {
  if (!S || !out) return AHS_E_INVALID_ARG;
  memset(out, 0, sizeof *out);
  const ServerCore& c = S->core;
  out->submitted = c.submitted();
  out->completed = c.completed();
  out->failed = c.failed();
  out->pending = c.pending.size();
  for (auto& sl : S->slots) out->running_batches += sl.batch >= 0 ? 1 : 0;
  out->batches = S->batches_run;
  out->mean_batch_requests = S->batches_run ? (double)S->requests_batched / (double)S->batches_run : 0.0;
  out->keys_completed = c.keys_done();
  out->p50_ms = c.percentile(50.0);
  out->p99_ms = c.percentile(99.0);
  out->max_ms = c.max_latency();
  out->mean_ms = c.mean_latency();
  out->first_arrival_ms = c.first_arrival();
  out->last_done_ms = c.last_done();
  const double span = out->last_done_ms - out->first_arrival_ms;
  out->gkeys_per_s = span > 0 ? (double)out->keys_completed / (span * 1e-3) / 1e9 : 0.0;
  out->arena_used_bytes = S->arena.used();
  out->arena_peak_bytes = S->peak_used;
  return AHS_OK;
}

extern "C" void ahs_server_destroy(ahs_server* S) {
  if (!S) return;
  for (auto& sl : S->slots) {
    if (sl.s) {
      (void)hipStreamSynchronize(sl.s);
      (void)hipStreamDestroy(sl.s);
    }
    if (sl.pinned) (void)hipHostFree(sl.pinned);
  }
  for (auto& kv : S->batches)
    if (kv.second.done) (void)hipEventDestroy(kv.second.done);
  for (auto& kv : S->core.reqs)
    if (kv.second.ready) (void)hipEventDestroy((hipEvent_t)kv.second.ready);
  for (auto e : S->events) (void)hipEventDestroy(e);
  if (S->t0_ev) (void)hipEventDestroy(S->t0_ev);
  if (S->base) (void)hipFree(S->base);
  if (S->ctx) ahs_context_destroy(S->ctx);
  delete S;
}
