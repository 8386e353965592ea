// Optional HIP-event timing of kernel launches (gw_profile_*).
#include <mutex>
#include <string>
#include <vector>

#include "gw_internal.hpp"

namespace gw {
namespace {

struct Rec {
  std::string name;
  hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

ProfScope::ProfScope(hipStream_t s, const char* name) : s_(s), name_(name) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  a_ = get_event();
  b_ = get_event();
  if (a_ && b_ && hipEventRecord(a_, s_) == hipSuccess) active_ = true;
}

ProfScope::~ProfScope() {
  if (!active_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (hipEventRecord(b_, s_) == hipSuccess) g_recs.push_back(Rec{name_, a_, b_});
}

}  // namespace gw

using namespace gw;

extern "C" {

int gw_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return GW_OK;
}

int gw_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (Rec& r : g_recs) {
    hipEventSynchronize(r.b);
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return GW_OK;
}

int gw_profile_query(const char* name, int* launches, double* total_ms) {
  if (!name || !launches || !total_ms) return fail(GW_ERR_INVALID_ARG, "gw_profile_query: null argument");
  std::lock_guard<std::mutex> lk(g_mu);
  int n = 0;
  double tot = 0.0;
  for (Rec& r : g_recs) {
    if (r.name != name) continue;
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    ++n;
    tot += ms;
  }
  *launches = n;
  *total_ms = tot;
  return GW_OK;
}

}  // extern "C"
