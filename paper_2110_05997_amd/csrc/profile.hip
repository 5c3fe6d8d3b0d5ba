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
uint32_t g_mask = ~0u;                 // kernels timed while enabled (bit k: cpd_profile_kernel k)
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;        // events of finished measurements, reused

bool take_event(hipEvent_t* e) {
  if (!g_pool.empty()) { *e = g_pool.back(); g_pool.pop_back(); return true; }
  return hipEventCreate(e) == hipSuccess;
}
int64_t g_launches[CPD_PK_COUNT];
double g_ms[CPD_PK_COUNT];

}  // namespace

// One workgroup of `blockDim.x` threads chaining `reps` block sums (one barrier and one LDS round
// trip each, alternating two slot arrays as the dGN kernel does): the floor under every reduction
// of the one-workgroup dGN.
__global__ __launch_bounds__(1024) void block_sum_probe_kernel(int reps, long long* __restrict__ ticks,
                                                               double* __restrict__ sink) {
  __shared__ double slots[2][16];
  double v = (double)threadIdx.x;
  __syncthreads();
  const long long t0 = wall_clock64();
  for (int i = 0; i < reps; ++i) v = block_sum(v * 1e-3, slots[i & 1]);
  __syncthreads();
  const long long t1 = wall_clock64();
  if (threadIdx.x == 0) {
    ticks[0] = t1 - t0;
    sink[0] = v;
  }
}

double wall_ns_per_tick() {
  static thread_local int dev_cached = -1;
  static thread_local double f = 10.0;   // 100 MHz, replaced by the device's reported rate
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return f;
  if (dev != dev_cached) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      f = 1e6 / (double)khz;
    dev_cached = dev;
  }
  return f;
}

void prof_begin(int which, hipStream_t s) {
  if (!g_on || !((g_mask >> which) & 1u)) return;
  Pending p{which, nullptr, nullptr, false};
  if (!take_event(&p.start)) return;
  if (!take_event(&p.stop)) { g_pool.push_back(p.start); return; }
  (void)hipEventRecord(p.start, s);
  g_pending.push_back(p);
}

void prof_end(int which, hipStream_t s) {
  if (!g_on || !((g_mask >> which) & 1u)) return;
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

cpd_status cpd_profile_block_sum_ns(int32_t nthreads, int32_t reps, void* ws, size_t ws_bytes, double* ns_out,
                                    void* stream) {
  CPD_REQUIRE(ws && ws_bytes >= 16 && ns_out && reps >= 1 && nthreads >= 64 && nthreads <= 1024 &&
                  nthreads % 64 == 0,
              "cpd_profile_block_sum_ns: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  long long* ticks = (long long*)ws;
  double* sink = (double*)((char*)ws + 8);
  hipLaunchKernelGGL(block_sum_probe_kernel, dim3(1), dim3(nthreads), 0, s, reps, ticks, sink);
  CPD_LAUNCH_CHECK();
  long long h = 0;
  CPD_HIP_CHECK(hipMemcpyAsync(&h, ticks, sizeof(h), hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  *ns_out = (double)h * wall_ns_per_tick() / (double)reps;
  return CPD_OK;
}

void cpd_profile_select(uint32_t mask) { g_mask = mask; }

void cpd_profile_reset(void) {
  for (auto& p : g_pending) {
    if (p.closed) (void)hipEventSynchronize(p.stop);
    g_pool.push_back(p.start);
    g_pool.push_back(p.stop);
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
    g_pool.push_back(p.start);
    g_pool.push_back(p.stop);
  }
  g_pending.swap(keep);
  if (out)
    for (int i = 0; i < CPD_PK_COUNT; ++i) { out[i].launches = g_launches[i]; out[i].total_ms = g_ms[i]; }
  return CPD_OK;
}

}  // extern "C"
