// Event-pair kernel timing (off unless enabled through the C ABI).
#include <mutex>
#include <vector>

#include "fcgno.h"
#include "prof.h"

namespace fcgno {

namespace {
struct Pending { int k; hipEvent_t a, b; };
std::mutex g_mu;
unsigned g_mask = 0u;
std::vector<hipEvent_t> g_pool;
std::vector<Pending> g_pending;
hipEvent_t g_open[PK_COUNT];
long long g_count[PK_COUNT];
double g_ms[PK_COUNT];

hipEvent_t take_event() {
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

bool prof_on() { return g_mask != 0u; }
bool prof_on(int k) { return (g_mask >> k) & 1u; }

void prof_begin(int k, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t e = take_event();
  if (e && hipEventRecord(e, s) == hipSuccess) g_open[k] = e;
  else g_open[k] = nullptr;
}

void prof_end(int k, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_open[k]) return;
  hipEvent_t e = take_event();
  if (e && hipEventRecord(e, s) == hipSuccess) g_pending.push_back({k, g_open[k], e});
  g_open[k] = nullptr;
}

bool prof_kernel_events(int k, hipEvent_t* a, hipEvent_t* b) {
  if (!prof_on(k)) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  *a = take_event();
  *b = take_event();
  if (*a && *b) return true;
  if (*a) g_pool.push_back(*a);
  if (*b) g_pool.push_back(*b);
  return false;
}

void prof_kernel_done(int k, hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_pending.push_back({k, a, b});
}

void prof_collect() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_count[p.k] += 1;
      g_ms[p.k] += ms;
    }
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
}

}  // namespace fcgno

using namespace fcgno;

extern "C" void fcgno_profile_enable(int32_t mask) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_mask = (unsigned)mask & ((1u << PK_COUNT) - 1u);
}

extern "C" void fcgno_profile_reset(void) {
  prof_collect();
  std::lock_guard<std::mutex> lk(g_mu);
  for (int k = 0; k < PK_COUNT; ++k) { g_count[k] = 0; g_ms[k] = 0.0; }
}

extern "C" fcgno_status fcgno_profile_read(int32_t kernel, int64_t* launches, double* total_ms) {
  if (kernel < 0 || kernel >= PK_COUNT || !launches || !total_ms) return FCGNO_E_INVALID;
  prof_collect();
  std::lock_guard<std::mutex> lk(g_mu);
  *launches = g_count[kernel];
  *total_ms = g_ms[kernel];
  return FCGNO_OK;
}
