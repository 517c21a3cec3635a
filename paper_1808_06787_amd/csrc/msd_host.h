// Host helpers shared by the single-mixture and batched C ABI layers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/msd.h"
#include "msd_launch.h"

namespace msd {
namespace host {

int fail(int status, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int validate(const msd_problem* p);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int lattice_q(int lat) { return lat == MSD_D1Q3 ? 3 : (lat == MSD_D2Q5 ? 5 : 7); }
inline int lattice_d(int lat) { return lat == MSD_D1Q3 ? 1 : (lat == MSD_D2Q5 ? 2 : 3); }

constexpr int kDiagBlocksMax = 1024;

// Workspace layout of one mixture (byte offsets from the workspace base).
struct Layout {
  int64_t nodes = 0, plane = 0;
  size_t consts_off = 0, partials_off = 0, diag_out_off = 0, half_off[2] = {0, 0};
  size_t half_bytes = 0, total = 0;
  int diag_blocks = 0;
};

Layout layout_for(const msd_problem* p);
void fill_kernel_problem(const msd_problem* problem, int64_t plane, Problem* out);
hipError_t dispatch(Op op, const LaunchArgs& a);
void default_launch(const msd_problem* p, msd_launch* l);

}  // namespace host
}  // namespace msd
