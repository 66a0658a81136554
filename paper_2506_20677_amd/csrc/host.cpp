// Host side of the C ABI (include/ahs.h): argument checks, workspace
// layout, the decision engine and the launch sequence of every strategy.
#include "ahs.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "host_internal.hpp"
#include "static_scratch.hpp"
#include "kernels.hpp"

using namespace ahs;

static_assert(sizeof(ahs_feature_vector) == sizeof(DevFeatures), "feature vector layout");

// ------------------------------------------------------------------ context
ahs_context::~ahs_context() {
  for (auto& r : pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : event_pool) (void)hipEventDestroy(e);
  if (pinned) (void)hipHostFree(pinned);
}

ahs_status ahs_context::fail(ahs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error = buf;
  return s;
}

ahs_status ahs_context::check(hipError_t e, const char* what) {
  if (e == hipSuccess) return AHS_OK;
  return fail(AHS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

hipEvent_t ahs_context::take_event() {
  if (!event_pool.empty()) {
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void ahs_context::prof_begin(const char* name, hipStream_t s, double bytes) {
  if (!profiling || capturing) return;
  Rec r;
  r.name = name;
  r.bytes = bytes;
  r.a = take_event();
  r.b = take_event();
  (void)hipEventRecord(r.a, s);
  pending.push_back(r);
}

void ahs_context::prof_end(hipStream_t s) {
  if (!profiling || capturing || pending.empty()) return;
  (void)hipEventRecord(pending.back().b, s);
}

void ahs_context::prof_set_last_bytes(const char* name, double bytes) {
  for (auto it = pending.rbegin(); it != pending.rend(); ++it) {
    if (it->name == name) {
      it->bytes = bytes;
      return;
    }
  }
}

void ahs_context::prof_collect() {
  for (auto& r : pending) {
    (void)hipEventSynchronize(r.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    auto& t = totals[r.name];
    t.launches += 1;
    t.ms += ms;
    t.bytes += r.bytes;
    event_pool.push_back(r.a);
    event_pool.push_back(r.b);
  }
  pending.clear();
}

extern "C" ahs_status ahs_context_create(int device, ahs_context** out) {
  if (!out) return AHS_E_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return AHS_E_DEVICE;
  ahs_context* c = new (std::nothrow) ahs_context();
  if (!c) return AHS_E_OOM;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return AHS_E_DEVICE;
  }
  c->cu_count = (uint32_t)prop.multiProcessorCount;
  c->device_name = prop.gcnArchName;
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(device);
  if (hipHostMalloc(&c->pinned, ahs_context::PINNED_BYTES, hipHostMallocDefault) != hipSuccess) {
    hipSetDevice(prev);
    delete c;
    return AHS_E_OOM;
  }
  // the fixed scratch of ahs_sort_static on this device (its address is
  // per device; looked up here, with the device current, once per device)
  if (ahs::static_scratch_address(device, &c->static_scratch) != hipSuccess) {
    hipSetDevice(prev);
    delete c;
    return AHS_E_DEVICE;
  }
  hipSetDevice(prev);
  *out = c;
  return AHS_OK;
}

extern "C" void ahs_context_destroy(ahs_context* ctx) { delete ctx; }

extern "C" ahs_status ahs_context_set_model(ahs_context* ctx, const ahs_model* model) {
  if (!ctx) return AHS_E_INVALID_ARG;
  ctx->model = model;
  return AHS_OK;
}

extern "C" uint32_t ahs_device_cu_count(const ahs_context* ctx) { return ctx ? ctx->cu_count : 0u; }

extern "C" const char* ahs_last_error(const ahs_context* ctx) {
  return ctx ? ctx->last_error.c_str() : "no context";
}

extern "C" const char* ahs_status_str(ahs_status s) {
  switch (s) {
    case AHS_OK: return "ok";
    case AHS_E_INVALID_ARG: return "invalid argument";
    case AHS_E_UNSUPPORTED: return "unsupported";
    case AHS_E_NAN: return "NaN key";
    case AHS_E_WORKSPACE: return "workspace too small";
    case AHS_E_OOM: return "out of host memory";
    case AHS_E_DEVICE: return "device error";
    case AHS_E_NO_MODEL: return "no model attached";
    case AHS_E_PARSE: return "model file malformed";
  }
  return "unknown status";
}

// ------------------------------------------------------------------ profiling
extern "C" ahs_status ahs_profile_enable(ahs_context* ctx, int on) {
  if (!ctx) return AHS_E_INVALID_ARG;
  ctx->prof_collect();
  ctx->profiling = on != 0;
  return AHS_OK;
}

extern "C" ahs_status ahs_profile_reset(ahs_context* ctx) {
  if (!ctx) return AHS_E_INVALID_ARG;
  ctx->prof_collect();
  ctx->totals.clear();
  return AHS_OK;
}

extern "C" ahs_status ahs_profile_query(ahs_context* ctx, const char* kernel, uint64_t* launches, double* total_ms,
                                        double* algo_bytes) {
  if (!ctx || !kernel) return AHS_E_INVALID_ARG;
  ctx->prof_collect();
  auto it = ctx->totals.find(kernel);
  const bool none = it == ctx->totals.end();
  if (launches) *launches = none ? 0 : it->second.launches;
  if (total_ms) *total_ms = none ? 0.0 : it->second.ms;
  if (algo_bytes) *algo_bytes = none ? 0.0 : it->second.bytes;
  return AHS_OK;
}

extern "C" size_t ahs_profile_dump(ahs_context* ctx, char* buf, size_t len) {
  if (!ctx) return 0;
  ctx->prof_collect();
  std::string s;
  char line[256];
  for (auto& kv : ctx->totals) {
    snprintf(line, sizeof line, "%s %llu %.6f %.0f\n", kv.first.c_str(), (unsigned long long)kv.second.launches,
             kv.second.ms, kv.second.bytes);
    s += line;
  }
  if (buf && len) {
    size_t m = std::min(len - 1, s.size());
    memcpy(buf, s.data(), m);
    buf[m] = 0;
  }
  return s.size() + 1;
}

// ------------------------------------------------------------------ config / select
extern "C" ahs_status ahs_config_init(ahs_config* cfg, int preset) {
  if (!cfg) return AHS_E_INVALID_ARG;
  cfg->n_small = 20;
  cfg->use_model = 0;
  cfg->k_count = 4096;
  cfg->k_radix = 1000000;
  cfg->h_ratio = 0.7;
  cfg->ml_min_n = 1000;
  cfg->k_count_cap = 65536;
  switch (preset) {
    case AHS_PRESET_GPU: return AHS_OK;
    case AHS_PRESET_PAPER_TEXT: cfg->k_count = 1000; return AHS_OK;
    case AHS_PRESET_PAPER_TABLE2: cfg->k_count = 1024; return AHS_OK;
    case AHS_PRESET_MI355X_CALIBRATED:  // Sec. III-C, eq. (1) on this GPU's timings
      cfg->n_small = 48;
      cfg->k_count = 5000;
      return AHS_OK;
  }
  return AHS_E_INVALID_ARG;
}

// The FSM of Sec. III-A in the paper's order; then the predictor of Sec.
// III-H for n >= ml_min_n, whose counting verdict is only honoured below the
// counting cap.
extern "C" ahs_status ahs_select(const ahs_feature_vector* f, const ahs_config* cfg, const ahs_model* model,
                                 ahs_strategy* out) {
  if (!f || !cfg || !out || cfg->k_count == 0) return AHS_E_INVALID_ARG;
  if (f->n <= cfg->n_small) {
    *out = AHS_INSERTION;
    return AHS_OK;
  }
  ahs_strategy s;
  if (f->span <= cfg->k_count - 1) {
    s = AHS_COUNTING;
  } else if (f->span >= cfg->k_radix && f->entropy_bits < cfg->h_ratio * std::log2((double)f->nbins)) {
    s = AHS_RADIX;
  } else {
    s = AHS_QUICK;
  }
  if (cfg->use_model && f->n >= cfg->ml_min_n) {
    if (!model) return AHS_E_NO_MODEL;
    ahs_strategy m;
    ahs_status st = ahs_model_predict(model, f, &m);
    if (st != AHS_OK) return st;
    if (!(m == AHS_COUNTING && f->span >= cfg->k_count_cap)) s = m;
  }
  *out = s;
  return AHS_OK;
}
