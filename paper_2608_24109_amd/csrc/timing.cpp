// Per-kernel timing hooks: when enabled, every kernel launch of the library is bracketed by two
// HIP events recorded on the stream it is launched on; exm_timing_collect waits for them and
// accumulates the elapsed time per kernel name. Off by default (no events are created).
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "exm_internal.h"

namespace exm {
namespace {

struct Pending {
  const char* name;
  hipEvent_t a, b;
};
struct Total {
  std::string name;
  double ms = 0.0;
  int64_t launches = 0;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::vector<Total> g_totals;

void drop_pending_locked() {
  for (const Pending& p : g_pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending.clear();
}

}  // namespace

KernelTimer::KernelTimer(const char* name, hipStream_t s) : name_(name), s_(s) {
  if (!g_on.load(std::memory_order_relaxed)) return;
  if (hipEventCreate(&a_) != hipSuccess) {
    a_ = nullptr;
    (void)hipGetLastError();
    return;
  }
  if (hipEventRecord(a_, s_) != hipSuccess) {
    (void)hipEventDestroy(a_);
    a_ = nullptr;
    (void)hipGetLastError();
  }
}

KernelTimer::~KernelTimer() {
  if (!a_) return;
  hipEvent_t b = nullptr;
  if (hipEventCreate(&b) != hipSuccess || hipEventRecord(b, s_) != hipSuccess) {
    if (b) (void)hipEventDestroy(b);
    (void)hipEventDestroy(a_);
    (void)hipGetLastError();
    return;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_pending.push_back(Pending{name_, a_, b});
}

}  // namespace exm

using namespace exm;

extern "C" {

exm_status exm_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  drop_pending_locked();
  g_totals.clear();
  g_on.store(on != 0);
  return EXM_OK;
}

exm_status exm_timing_collect(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  exm_status st = EXM_OK;
  for (const Pending& p : g_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) {
      (void)hipGetLastError();
      st = fail(EXM_E_HIP, std::string("exm_timing_collect: event of ") + p.name + " failed");
      continue;
    }
    Total* t = nullptr;
    for (Total& x : g_totals)
      if (x.name == p.name) t = &x;
    if (!t) {
      g_totals.push_back(Total{p.name, 0.0, 0});
      t = &g_totals.back();
    }
    t->ms += ms;
    t->launches += 1;
  }
  drop_pending_locked();
  return st;
}

int32_t exm_timing_count(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (int32_t)g_totals.size();
}

const char* exm_timing_name(int32_t i) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (i >= 0 && i < (int32_t)g_totals.size()) ? g_totals[i].name.c_str() : nullptr;
}

double exm_timing_total_ms(int32_t i) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (i >= 0 && i < (int32_t)g_totals.size()) ? g_totals[i].ms : 0.0;
}

int64_t exm_timing_launches(int32_t i) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (i >= 0 && i < (int32_t)g_totals.size()) ? g_totals[i].launches : 0;
}

}  // extern "C"
