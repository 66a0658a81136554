// C entry points over the serving loop's scheduling core (a header-only,
// device-free class) so that its policy can be tested on a host alone.
#include <cstdint>

#include "server_core.hpp"

using ahs::Arena;
using ahs::BatchPlan;
using ahs::ServerCore;

extern "C" {

void* arena_new(uint64_t cap) { return new Arena(cap); }
void arena_delete(void* a) { delete static_cast<Arena*>(a); }
uint64_t arena_alloc(void* a, uint64_t bytes) { return static_cast<Arena*>(a)->alloc(bytes); }
int arena_release(void* a, uint64_t off) { return static_cast<Arena*>(a)->release(off) ? 1 : 0; }
uint64_t arena_used(void* a) { return static_cast<Arena*>(a)->used(); }
uint64_t arena_largest(void* a) { return static_cast<Arena*>(a)->largest_free(); }
uint64_t arena_ranges(void* a) { return static_cast<Arena*>(a)->free_ranges(); }

void* core_new(uint64_t max_keys, uint32_t max_reqs) {
  ServerCore* c = new ServerCore();
  c->lim.max_batch_keys = max_keys;
  c->lim.max_batch_requests = max_reqs;
  return c;
}
void core_delete(void* c) { delete static_cast<ServerCore*>(c); }
uint64_t core_add(void* c, int dtype, int pay, uint64_t n, double arrival) {
  return static_cast<ServerCore*>(c)->add(dtype, pay, n, arrival);
}
// Plans the next batch, writes its ids; start != 0 also starts it as batch b.
uint32_t core_plan(void* c, uint64_t* ids, uint32_t max, uint64_t* keys, int start, int64_t b) {
  ServerCore* s = static_cast<ServerCore*>(c);
  const BatchPlan p = s->plan_next();
  uint32_t k = 0;
  for (; k < p.ids.size() && k < max; ++k) ids[k] = p.ids[k];
  *keys = p.keys;
  if (start) s->start(p, b);
  return (uint32_t)p.ids.size();
}
uint64_t core_offset(void* c, uint64_t id) { return static_cast<ServerCore*>(c)->reqs.at(id).offset; }
uint32_t core_pending(void* c, uint64_t* ids, uint32_t max) {
  ServerCore* s = static_cast<ServerCore*>(c);
  uint32_t k = 0;
  for (uint64_t id : s->pending) {
    if (k < max) ids[k] = id;
    ++k;
  }
  return k;
}
void core_complete(void* c, uint64_t id, int status, double done_ms) {
  static_cast<ServerCore*>(c)->complete(id, status, 0, done_ms);
}
double core_percentile(void* c, double q) { return static_cast<ServerCore*>(c)->percentile(q); }
uint64_t core_completed(void* c) { return static_cast<ServerCore*>(c)->completed(); }
uint64_t core_failed(void* c) { return static_cast<ServerCore*>(c)->failed(); }
uint64_t core_keys_done(void* c) { return static_cast<ServerCore*>(c)->keys_done(); }
}
