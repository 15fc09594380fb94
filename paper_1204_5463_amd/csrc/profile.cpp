// Per-kernel-class timing with HIP events (see dw_profile_* in dwsap.h).
#include <hip/hip_runtime.h>

#include "dw_internal.hpp"

namespace dw {

static thread_local Profiler* t_prof = nullptr;
static thread_local ProfTagV t_tag;

Profiler* prof_current() { return t_prof; }

ProfTag::ProfTag(int kind, unsigned long long mask) : prev(t_tag) {
  t_tag.kind = kind;
  t_tag.mask = mask;
}
ProfTag::~ProfTag() { t_tag = prev; }

ProfScope::ProfScope(dw_ctx ctx) : prev(t_prof) { t_prof = (ctx && ctx->prof.on) ? &ctx->prof : nullptr; }
ProfScope::~ProfScope() {
  prof_flush();
  t_prof = prev;
}

static hipEvent_t get_event(Profiler* p) {
  hipEvent_t e = nullptr;
  if (!p->pool.empty()) {
    e = p->pool.back();
    p->pool.pop_back();
    return e;
  }
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

KTimer::KTimer(int kclass, hipStream_t stream) : s(stream), kc(kclass) {
  Profiler* pr = t_prof;
  if (!pr) return;
  std::lock_guard<std::mutex> lk(pr->mu);
  a = get_event(pr);
  if (a && hipEventRecord(a, s) == hipSuccess) p = pr;
}

void KTimer::done(double bytes, double flops) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(p->mu);
  hipEvent_t b = get_event(p);
  if (!b || hipEventRecord(b, s) != hipSuccess) {
    p->pool.push_back(a);
    if (b) p->pool.push_back(b);
    return;
  }
  p->pending.push_back(Profiler::Rec{kc, a, b, bytes, flops, t_tag});
  p = nullptr;
}

void prof_flush(Profiler* p) {
  if (!p) p = t_prof;
  if (!p) return;
  std::lock_guard<std::mutex> lk(p->mu);
  std::vector<Profiler::Rec> keep;
  for (auto& r : p->pending) {
    if (hipEventQuery(r.b) != hipSuccess) {
      keep.push_back(r);
      continue;
    }
    if (r.tag.kind != kTagNone) {
      p->held.push_back(r);
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      dw_kernel_stats& k = p->acc[r.kc];
      k.launches += 1;
      k.ms += ms;
      k.bytes += r.bytes;
      k.flops += r.flops;
    }
    p->pool.push_back(r.a);
    p->pool.push_back(r.b);
  }
  p->pending.swap(keep);
}

}  // namespace dw

using namespace dw;

extern "C" {

dw_status dw_profile_enable(dw_ctx ctx, int32_t on) {
  clear_error();
  if (!ctx) {
    set_error("dw_profile_enable: null context");
    return DW_EINVAL;
  }
  std::lock_guard<std::mutex> lk(ctx->prof.mu);
  ctx->prof.on = on != 0;
  return DW_OK;
}

dw_status dw_profile_get(dw_ctx ctx, int32_t kclass, dw_kernel_stats* out) {
  clear_error();
  if (!ctx || !out || kclass < 0 || kclass >= DW_K_COUNT) {
    set_error("dw_profile_get: invalid argument");
    return DW_EINVAL;
  }
  prof_flush(&ctx->prof);
  std::lock_guard<std::mutex> lk(ctx->prof.mu);
  *out = ctx->prof.acc[kclass];
  return DW_OK;
}

dw_status dw_profile_reset(dw_ctx ctx) {
  clear_error();
  if (!ctx) {
    set_error("dw_profile_reset: null context");
    return DW_EINVAL;
  }
  std::lock_guard<std::mutex> lk(ctx->prof.mu);
  for (auto& k : ctx->prof.acc) k = dw_kernel_stats{};
  return DW_OK;
}

}  // extern "C"
