// Host helpers shared by the single-mixture and batched C ABI layers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/msd.h"
#include "msd_launch.h"

namespace msd {
namespace host {

int fail(int status, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int validate(const msd_problem* p);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int lattice_d(int lat) {
  return (lat == MSD_D1Q3 || lat == MSD_D1Q2) ? 1 : ((lat == MSD_D2Q5 || lat == MSD_D2Q4 || lat == MSD_D2Q9) ? 2 : 3);
}
// q = 2d + 1 with a rest direction, 2d without; 9 and 15 with diagonals
inline int lattice_q(int lat) {
  return lat == MSD_D2Q9 ? 9 : (lat == MSD_D3Q15 ? 15 : 2 * lattice_d(lat) + (lat <= MSD_D3Q7 ? 1 : 0));
}

constexpr int kDiagBlocksMax = 1024;

// Workspace layout of one mixture (byte offsets from the workspace base).
struct Layout {
  int64_t nodes = 0, plane = 0;
  size_t consts_off = 0, partials_off = 0, diag_out_off = 0, ref_off = 0, half_off[2] = {0, 0};
  size_t half_bytes = 0, total = 0;
  int diag_blocks = 0;
};

Layout layout_for(const msd_problem* p);
void fill_kernel_problem(const msd_problem* problem, int64_t plane, Problem* out);
hipError_t dispatch(Op op, const LaunchArgs& a);
void default_launch(const msd_problem* p, msd_launch* l);

// --- tuning ------------------------------------------------------------------
// 64-bit FNV-1a hash (keys of the tuning cache).
inline uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* b = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}
// GPU architecture name of the current device ("gfx950"), "unknown" on error.
std::string device_arch();
// Tuning cache: a text file of lines "<key> <v1> ... <vk> <ms per step>".
// lookup returns true and fills vals/ms when the key is present with k values.
bool cache_lookup(const char* path, const std::string& key, int k, int64_t* vals, double* ms);
void cache_store(const char* path, const std::string& key, int k, const int64_t* vals, double ms);

// Times candidates 0..n-1: apply(i) selects one (nonzero status: skipped, time
// -1), then one warm-up step, `steps` steps between two events on `stream`, and
// restore() puts state and time back.  Stops once budget_ms of timed GPU work
// is spent (<= 0: no limit; untried candidates get -1).  One trial of a few
// milliseconds can be off by several per cent, so the `refine` fastest
// candidates are then timed twice more and keep their best time.  Returns the
// index of the fastest candidate in *best (-1 if none ran) or a status.
template <class Apply, class Step, class Restore>
int time_candidates(hipStream_t stream, int n, int steps, double budget_ms, Apply apply, Step step, Restore restore,
                    double* ms, int* best, int refine = 4) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(e, "tuning events");
  *best = -1;
  double spent = 0.0;
  int st = MSD_OK;
  // one timed trial of candidate i: its ms per step, or -1 if it does not apply
  auto trial = [&](int i, double* out) -> int {
    *out = -1.0;
    if (apply(i) != MSD_OK) return MSD_OK;
    int s = step(1);
    if (s != MSD_OK) return s;
    hipError_t he = hipEventRecord(e0, stream);
    if (he != hipSuccess) return hip_fail(he, "tuning event");
    s = step(steps);
    if (s != MSD_OK) return s;
    he = hipEventRecord(e1, stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float t = 0.0f;
    if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
    if (he != hipSuccess) return hip_fail(he, "tuning timing");
    spent += t;
    *out = (double)t / steps;
    return restore();
  };
  for (int i = 0; i < n; ++i) ms[i] = -1.0;
  for (int i = 0; i < n && st == MSD_OK; ++i) {
    if (budget_ms > 0 && spent >= budget_ms) break;
    st = trial(i, &ms[i]);
  }
  std::vector<int> top;
  for (int i = 0; i < n; ++i)
    if (ms[i] >= 0) top.push_back(i);
  std::sort(top.begin(), top.end(), [&](int a, int b) { return ms[a] < ms[b]; });
  if ((int)top.size() > refine) top.resize((size_t)std::max(refine, 0));
  for (int again = 0; again < 2 && st == MSD_OK && top.size() > 1; ++again)
    for (int i : top) {
      if (st != MSD_OK || (budget_ms > 0 && spent >= 2 * budget_ms)) break;
      double t = -1.0;
      st = trial(i, &t);
      if (t >= 0 && t < ms[i]) ms[i] = t;
    }
  for (int i = 0; i < n; ++i)
    if (ms[i] >= 0 && (*best < 0 || ms[i] < ms[*best])) *best = i;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

}  // namespace host
}  // namespace msd

// Host handle of one mixture (msd_create); the batch layer also builds
// temporary handles over parts of a batch workspace (msd_batch_step_separate).
struct msd_sim {
  msd_problem prob;          // pointers inside are not kept
  msd::Problem kp;           // kernel copy of the problem
  msd::host::Layout L;
  int m = 0, q = 0, d = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int cur = 0;               // which half holds the state
  int64_t t = 0;
  bool initialised = false;
  msd_launch launch{};
  // resident workgroups of the blocked kernels by steps per pass (0: not queried)
  mutable int resident_fwd[msd::kMaxStepsPerPass + 1] = {};
  mutable int resident_adj[msd::kMaxStepsPerPass + 1] = {};
  mutable int n_cu = 0;
  mutable int lds_per_cu = -1;   // LDS bytes per CU of the device (0: unknown)
  msd_health health{1e-2, 1e-4};  // limits of the divergence checks in msd_diagnostics
  double rho1 = 0.0, rho2 = 0.0;  // largest relaxation radii found by msd_create
};
