// Scheduling core of the serving loop, free of any device call so that it
// can be exercised on a host alone: a first-fit arena over the HBM budget,
// the pending queue in arrival order, batch formation (continuous batching:
// whenever a slot is free, the oldest pending request's key class is batched
// with the later pending requests of the same class, up to the batch
// limits), per-request bookkeeping and latency statistics.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

namespace ahs {

// First-fit allocator over [0, capacity) with coalescing of free ranges.
class Arena {
 public:
  explicit Arena(uint64_t capacity = 0) { reset(capacity); }
  void reset(uint64_t capacity) {
    cap_ = capacity;
    used_ = 0;
    free_.clear();
    if (capacity) free_[0] = capacity;
  }
  // Offset of a block of `bytes` (a multiple of `align`), or UINT64_MAX.
  uint64_t alloc(uint64_t bytes, uint64_t align = 256) {
    bytes = (bytes + align - 1) / align * align;
    if (bytes == 0) bytes = align;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      const uint64_t off = it->first, sz = it->second;
      const uint64_t start = (off + align - 1) / align * align;
      if (start + bytes > off + sz) continue;
      free_.erase(it);
      if (start > off) free_[off] = start - off;
      if (start + bytes < off + sz) free_[start + bytes] = off + sz - (start + bytes);
      used_ += bytes;
      sizes_[start] = bytes;
      return start;
    }
    return UINT64_MAX;
  }
  bool release(uint64_t off) {
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return false;
    uint64_t start = off, size = s->second;
    sizes_.erase(s);
    used_ -= size;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + size) {
      size += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        size += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = size;
    return true;
  }
  uint64_t used() const { return used_; }
  uint64_t capacity() const { return cap_; }
  size_t free_ranges() const { return free_.size(); }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (auto& f : free_) m = std::max(m, f.second);
    return m;
  }

 private:
  uint64_t cap_ = 0, used_ = 0;
  std::map<uint64_t, uint64_t> free_;   // offset -> size
  std::map<uint64_t, uint64_t> sizes_;  // allocated offset -> size
};

enum class ReqState : int { PENDING = 0, RUNNING = 1, DONE = 2, FAILED = 3 };

struct Request {
  uint64_t id = 0;
  int dtype = 0;
  int pay = 0;
  uint64_t n = 0;
  double arrival_ms = 0.0;
  double done_ms = 0.0;
  ReqState state = ReqState::PENDING;
  int64_t batch = -1;    // batch holding the request's buffers
  uint64_t offset = 0;   // key offset inside the batch
  int status = 0;        // ahs_status of the request
  uint8_t chosen = 0;
  const void* kin = nullptr;     // caller's input (device)
  const uint32_t* vin = nullptr;
  void* ready = nullptr;         // event the input waits on (device layer)
};

struct BatchPlan {
  std::vector<uint64_t> ids;  // in arrival order
  uint64_t keys = 0, max_n = 0;
  int dtype = 0, pay = 0;
};

struct ServerLimits {
  uint64_t max_batch_keys = 1ull << 26;
  uint32_t max_batch_requests = 1024;
};

class ServerCore {
 public:
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> pending;
  ServerLimits lim;

  uint64_t add(int dtype, int pay, uint64_t n, double arrival_ms) {
    Request r;
    r.id = next_id_++;
    r.dtype = dtype;
    r.pay = pay;
    r.n = n;
    r.arrival_ms = arrival_ms;
    reqs[r.id] = r;
    pending.push_back(r.id);
    ++submitted_;
    return r.id;
  }

  // The next batch: the oldest pending request and the later pending
  // requests of its class while both limits hold (the first request is
  // always taken, whatever its size).
  BatchPlan plan_next() const {
    BatchPlan p;
    if (pending.empty()) return p;
    const Request& h = reqs.at(pending.front());
    p.dtype = h.dtype;
    p.pay = h.pay;
    for (uint64_t id : pending) {
      const Request& r = reqs.at(id);
      if (r.dtype != h.dtype || r.pay != h.pay) continue;
      if (!p.ids.empty() &&
          (p.ids.size() >= lim.max_batch_requests || p.keys + r.n > lim.max_batch_keys))
        break;
      p.ids.push_back(id);
      p.keys += r.n;
      p.max_n = std::max(p.max_n, r.n);
    }
    return p;
  }

  // Marks the plan's requests as running in batch `b` at consecutive key
  // offsets and removes them from the pending queue.
  void start(const BatchPlan& p, int64_t b) {
    uint64_t off = 0;
    for (uint64_t id : p.ids) {
      Request& r = reqs.at(id);
      r.state = ReqState::RUNNING;
      r.batch = b;
      r.offset = off;
      off += r.n;
    }
    std::deque<uint64_t> rest;
    size_t k = 0;
    for (uint64_t id : pending) {
      if (k < p.ids.size() && id == p.ids[k]) {
        ++k;
        continue;
      }
      rest.push_back(id);
    }
    pending.swap(rest);
  }

  void fail_pending_head(int status, double now_ms) {
    const uint64_t id = pending.front();
    pending.pop_front();
    Request& r = reqs.at(id);
    r.state = ReqState::FAILED;
    r.status = status;
    r.done_ms = now_ms;
    ++failed_;
  }

  void complete(uint64_t id, int status, uint8_t chosen, double done_ms) {
    Request& r = reqs.at(id);
    r.status = status;
    r.chosen = chosen;
    r.done_ms = done_ms;
    if (status == 0) {
      r.state = ReqState::DONE;
      lat_.push_back(done_ms - r.arrival_ms);
      keys_done_ += r.n;
      first_arrival_ = std::min(first_arrival_, r.arrival_ms);
      last_done_ = std::max(last_done_, done_ms);
    } else {
      r.state = ReqState::FAILED;
      ++failed_;
    }
  }

  // Nearest-rank percentile of the completed requests' latencies.
  double percentile(double q) const {
    if (lat_.empty()) return 0.0;
    std::vector<double> v(lat_);
    std::sort(v.begin(), v.end());
    size_t rank = (size_t)(q / 100.0 * (double)v.size() + 0.999999999);
    if (rank < 1) rank = 1;
    if (rank > v.size()) rank = v.size();
    return v[rank - 1];
  }
  double mean_latency() const {
    if (lat_.empty()) return 0.0;
    double s = 0.0;
    for (double x : lat_) s += x;
    return s / (double)lat_.size();
  }
  double max_latency() const { return lat_.empty() ? 0.0 : *std::max_element(lat_.begin(), lat_.end()); }
  uint64_t completed() const { return lat_.size(); }
  uint64_t failed() const { return failed_; }
  uint64_t submitted() const { return submitted_; }
  uint64_t keys_done() const { return keys_done_; }
  double first_arrival() const { return lat_.empty() ? 0.0 : first_arrival_; }
  double last_done() const { return lat_.empty() ? 0.0 : last_done_; }

 private:
  uint64_t next_id_ = 1, submitted_ = 0, failed_ = 0, keys_done_ = 0;
  std::vector<double> lat_;
  double first_arrival_ = 1e300, last_done_ = -1e300;
};

}  // namespace ahs
