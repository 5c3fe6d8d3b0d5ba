// HIP-event timing of the path's main kernels (cpd_profile_* in cpd.h).
#include "common.h"

#include <vector>

namespace cpd {
namespace {

struct Pending {
  int which;
  hipEvent_t start, stop;
  bool closed;
};

bool g_on = false;
std::vector<Pending> g_pending;
int64_t g_launches[CPD_PK_COUNT];
double g_ms[CPD_PK_COUNT];

}  // namespace

void prof_begin(int which, hipStream_t s) {
  if (!g_on) return;
  Pending p{which, nullptr, nullptr, false};
  if (hipEventCreate(&p.start) != hipSuccess) return;
  if (hipEventCreate(&p.stop) != hipSuccess) { (void)hipEventDestroy(p.start); return; }
  (void)hipEventRecord(p.start, s);
  g_pending.push_back(p);
}

void prof_end(int which, hipStream_t s) {
  if (!g_on) return;
  for (auto it = g_pending.rbegin(); it != g_pending.rend(); ++it) {
    if (it->which == which && !it->closed) {
      (void)hipEventRecord(it->stop, s);
      it->closed = true;
      return;
    }
  }
}

}  // namespace cpd

using namespace cpd;

extern "C" {

void cpd_profile_enable(int32_t on) { g_on = (on != 0); }

void cpd_profile_reset(void) {
  for (auto& p : g_pending) {
    if (p.closed) (void)hipEventSynchronize(p.stop);
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  g_pending.clear();
  for (int i = 0; i < CPD_PK_COUNT; ++i) { g_launches[i] = 0; g_ms[i] = 0.0; }
}

cpd_status cpd_profile_read(cpd_kernel_time* out) {
  std::vector<Pending> keep;
  for (auto& p : g_pending) {
    if (!p.closed) { keep.push_back(p); continue; }
    CPD_HIP_CHECK(hipEventSynchronize(p.stop));
    float ms = 0.f;
    CPD_HIP_CHECK(hipEventElapsedTime(&ms, p.start, p.stop));
    g_ms[p.which] += ms;
    g_launches[p.which] += 1;
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  g_pending.swap(keep);
  if (out)
    for (int i = 0; i < CPD_PK_COUNT; ++i) { out[i].launches = g_launches[i]; out[i].total_ms = g_ms[i]; }
  return CPD_OK;
}

}  // extern "C"
