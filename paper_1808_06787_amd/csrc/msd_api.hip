// C ABI of the solver (include/msd.h): validation, workspace layout, time
// stepping and read-out.  Host code here only checks arguments, lays out the
// caller's workspace and launches kernels; all arithmetic of the method runs
// on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cstddef>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/msd.h"
#include "msd_host.h"
#include "msd_launch.h"

namespace msd {
namespace host {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(MSD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

bool cache_lookup(const char* path, const std::string& key, int k, int64_t* vals, double* ms) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    char* save = nullptr;
    const char* tok = strtok_r(line, " \t\n", &save);
    if (!tok || key != tok) continue;
    int64_t v[16];
    int got = 0;
    while (got <= k && (tok = strtok_r(nullptr, " \t\n", &save))) {
      if (got < k) v[got] = std::strtoll(tok, nullptr, 10);
      else *ms = std::strtod(tok, nullptr);
      ++got;
    }
    if (got == k + 1) {   // the last matching line wins
      for (int i = 0; i < k; ++i) vals[i] = v[i];
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, int k, const int64_t* vals, double ms) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s", key.c_str());
  for (int i = 0; i < k; ++i) std::fprintf(f, " %lld", (long long)vals[i]);
  std::fprintf(f, " %.6f\n", ms);
  std::fclose(f);
}

int validate(const msd_problem* p) {
  if (!p) return fail(MSD_EINVAL, "problem is NULL");
  if (p->abi != MSD_ABI_VERSION) return fail(MSD_EABI, "problem.abi = %d, library ABI = %d", p->abi, MSD_ABI_VERSION);
  if (p->lattice < MSD_D1Q3 || p->lattice > MSD_D3Q15)
    return fail(MSD_EINVAL, "unknown lattice %d", p->lattice);
  if (p->n_species < 2 || p->n_species > MSD_MAX_SPECIES)
    return fail(MSD_EINVAL, "n_species = %d outside [2, %d]", p->n_species, MSD_MAX_SPECIES);
  if (p->precision != MSD_F32 && p->precision != MSD_F64) return fail(MSD_EINVAL, "unknown precision %d", p->precision);
  const int d = lattice_d(p->lattice);
  const int64_t ext[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a) {
    if (ext[a] < 1) return fail(MSD_EINVAL, "extent %d is %lld", a, (long long)ext[a]);
    if (a >= d && ext[a] != 1) return fail(MSD_EINVAL, "extent %d must be 1 on a %dD lattice", a, d);
    if (ext[a] > (int64_t)1 << 30) return fail(MSD_EINVAL, "extent %d too large", a);
  }
  if (p->nx * p->ny * p->nz >= ((int64_t)1 << 31)) return fail(MSD_EINVAL, "more than 2^31 - 1 nodes");
  if (p->dilute != 0 && p->dilute != 1) return fail(MSD_EINVAL, "dilute = %d must be 0 or 1", p->dilute);
  if (p->plane_pad < 0 || p->plane_pad % 64 || p->plane_pad > (1 << 24))
    return fail(MSD_EINVAL, "plane_pad = %d must be a multiple of 64 in [0, 2^24]", p->plane_pad);
  if (!p->D) return fail(MSD_EINVAL, "D is NULL");
  const int N = p->n_species;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      if (i == j) continue;
      const double v = p->D[i * N + j];
      if (!(v > 0.0) || !std::isfinite(v)) return fail(MSD_EDIFF, "D[%d][%d] = %g is not positive", i, j, v);
      if (v != p->D[j * N + i]) return fail(MSD_EDIFF, "D is not symmetric at (%d, %d)", i, j);
    }
  if (!(p->c_t > 0.0) || !std::isfinite(p->c_t)) return fail(MSD_EINVAL, "c_t = %g must be positive", p->c_t);
  if (p->relax != MSD_RELAX_PAPER && p->relax != MSD_RELAX_SRT && p->relax != MSD_RELAX_TRT)
    return fail(MSD_ERELAX, "unknown relax %d", p->relax);
  if (p->relax == MSD_RELAX_TRT && !(p->trt_magic > 0.0 && std::isfinite(p->trt_magic)))
    return fail(MSD_ERELAX, "trt_magic = %g must be positive", p->trt_magic);
  bool need_wall = false;
  for (int a = 0; a < 3; ++a) {
    const int lo = p->bc[2 * a], hi = p->bc[2 * a + 1];
    for (int s = 0; s < 2; ++s) {
      const int b = p->bc[2 * a + s];
      if (b != MSD_BC_PERIODIC && b != MSD_BC_ZERO_FLUX && b != MSD_BC_DIRICHLET)
        return fail(MSD_EINVAL, "unknown face condition %d", b);
      if (a >= d && b != MSD_BC_PERIODIC) return fail(MSD_EINVAL, "faces of unused axis %d must be periodic", a);
      if (b == MSD_BC_DIRICHLET) need_wall = true;
    }
    if ((lo == MSD_BC_PERIODIC) != (hi == MSD_BC_PERIODIC))
      return fail(MSD_EINVAL, "periodic faces on axis %d must come in pairs", a);
  }
  auto on_simplex = [N](const double* x) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) {
      if (!std::isfinite(x[i])) return false;
      s += x[i];
    }
    return std::fabs(s - 1.0) <= 1e-9;
  };
  if (need_wall) {
    if (!p->xi_wall) return fail(MSD_EINVAL, "Dirichlet faces need xi_wall");
    for (int f = 0; f < 6; ++f)
      if (p->bc[f] == MSD_BC_DIRICHLET && !on_simplex(p->xi_wall + f * N))
        return fail(MSD_ECOMP, "wall composition of face %d does not sum to 1", f);
  }
  if (p->linearized) {
    if (!p->xi_ref) return fail(MSD_EINVAL, "linearized needs xi_ref");
    if (!on_simplex(p->xi_ref)) return fail(MSD_ECOMP, "xi_ref does not sum to 1");
  }
  return MSD_OK;
}

void fill_kernel_problem(const msd_problem* problem, int64_t plane, Problem* out) {
  Problem& kp = *out;
  std::memset(&kp, 0, sizeof(kp));
  kp.nx = (int32_t)problem->nx;
  kp.ny = (int32_t)problem->ny;
  kp.nz = (int32_t)problem->nz;
  kp.relax = problem->relax;
  kp.magic = problem->relax == MSD_RELAX_TRT ? problem->trt_magic : 3.0 / 16.0;
  kp.linearized = problem->linearized ? 1 : 0;
  kp.dilute = problem->dilute ? 1 : 0;
  for (int f = 0; f < 6; ++f) kp.bc[f] = problem->bc[f];
  kp.plane = plane;
  kp.c_t = problem->c_t;
  const int N = problem->n_species;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) kp.D[i][j] = (i == j) ? 1.0 : problem->D[i * N + j];
  for (int f = 0; f < 6; ++f)
    for (int i = 0; i < N; ++i)
      kp.wall[f][i] = (problem->bc[f] == MSD_BC_DIRICHLET) ? problem->xi_wall[f * N + i] : 0.0;
  if (problem->linearized)
    for (int i = 0; i < N; ++i) kp.xi_ref[i] = problem->xi_ref[i];
}

hipError_t dispatch(Op op, const LaunchArgs& a) {
  switch (a.lattice) {
    case MSD_D1Q3: return msd::dispatch<1>(op, a);
    case MSD_D2Q5: return msd::dispatch<2>(op, a);
    case MSD_D3Q7: return msd::dispatch<3>(op, a);
    case MSD_D1Q2: return msd::dispatch<4>(op, a);
    case MSD_D2Q4: return msd::dispatch<5>(op, a);
    case MSD_D3Q6: return msd::dispatch<6>(op, a);
    case MSD_D2Q9: return msd::dispatch<7>(op, a);
    case MSD_D3Q15: return msd::dispatch<8>(op, a);
    default: return hipErrorInvalidValue;
  }
}

Layout layout_for(const msd_problem* p) {
  Layout L;
  const int m = p->n_species - 1, q = lattice_q(p->lattice), s = p->precision;
  L.nodes = p->nx * p->ny * p->nz;
  // Planes hold the node count rounded up to 64 values (so that every plane
  // starts 256-byte aligned) plus an optional caller-chosen pad.
  L.plane = (L.nodes + 63) / 64 * 64 + p->plane_pad;
  L.diag_blocks = (int)std::min<int64_t>(kDiagBlocksMax, (L.nodes + 255) / 256);
  size_t off = 0;
  L.consts_off = off;
  off = align_up(off + msd::kConstsBytes, 256);
  L.partials_off = off;
  off = align_up(off + sizeof(double) * (size_t)L.diag_blocks * (3 * p->n_species + 1), 256);
  L.diag_out_off = off;
  // diagnostics use 3N + 1 values, the adjoint's dL/dD N * N
  off = align_up(off + sizeof(double) * (MSD_MAX_SPECIES * MSD_MAX_SPECIES + 3 * MSD_MAX_SPECIES + 1), 256);
  // diagnostics of the initial field (its species totals are the reference of the drift check)
  L.ref_off = off;
  off = align_up(off + sizeof(double) * (3 * MSD_MAX_SPECIES + 1), 256);
  L.half_bytes = align_up((size_t)m * q * (size_t)L.plane * s, 256);
  L.half_off[0] = off;
  off += L.half_bytes;
  L.half_off[1] = off;
  off += L.half_bytes;
  L.total = off;
  return L;
}

// Defaults from measurements on MI355X (4096^2 D2Q5 and 512^3 D3Q7, FP32): the
// one-node-per-thread kernel with 256-thread row tiles runs at the speed of a
// plain copy of the same planes; vector widths 2/4, streaming hints and plane
// padding do not improve on it.  Remapping tiles onto XCDs helps in 3D (+1.5 %)
// and costs 3 % in 2D.  In 2D the temporally blocked sweep with six steps per
// pass is 3.6x faster than one step per pass (4096^2 ternary FP32: 68.7 vs
// 245 us per step; four steps per pass 84.8 us, five 74.4 us); the species
// count and precision may lower the steps per pass.
void default_launch(const msd_problem* p, msd_launch* l) {
  std::memset(l, 0, sizeof(*l));
  l->block_x = (int)std::min<int64_t>(256, (p->nx + 63) / 64 * 64);
  l->block_y = std::max(1, (int)std::min<int64_t>(256 / l->block_x, p->ny));
  l->xcd_remap = lattice_d(p->lattice) == 3 ? 1 : 0;
  l->lds_resident = 1;
  l->nontemporal = 0;
  l->vec = 0;
  l->temporal = (p->lattice == MSD_D2Q5 || p->lattice == MSD_D2Q4)
                    ? msd::kMaxStepsPerPass
                    : ((p->lattice == MSD_D3Q7 || p->lattice == MSD_D3Q6) ? msd::k3dStepsPerPass : 0);
  l->seg_rows = 0;
  l->tile_x = 0;
  l->tile_y = 0;
}

}  // namespace host
}  // namespace msd

using namespace msd::host;


static_assert(sizeof(msd_problem) == 120 && offsetof(msd_problem, c_t) == 64 && offsetof(msd_problem, bc) == 80 &&
                  offsetof(msd_problem, dilute) == 108 && offsetof(msd_problem, trt_magic) == 112,
              "msd_problem layout (ABI version 3 and later)");
static_assert(sizeof(msd_launch) == 40 && offsetof(msd_launch, tile_x) == 32, "msd_launch layout (ABI version 4)");

namespace {

msd::LaunchArgs base_args(const msd_sim* s) {
  msd::LaunchArgs a;
  a.p = s->kp;
  a.lattice = s->prob.lattice;
  a.m = s->m;
  a.prec = s->prob.precision;
  a.stream = s->stream;
  a.consts = s->ws + s->L.consts_off;
  a.n_species = s->prob.n_species;
  a.block_x = s->launch.block_x;
  a.block_y = s->launch.block_y;
  a.xcd_remap = s->launch.xcd_remap;
  a.nontemporal = s->launch.nontemporal;
  a.vec = s->launch.vec;
  if (s->lds_per_cu < 0) {
    int dev = 0, v = 0;
    s->lds_per_cu = (hipGetDevice(&dev) == hipSuccess &&
                     hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess)
                        ? v
                        : 0;
  }
  // the forward blocked sweep runs fastest with at most two workgroups per CU
  // (measured on 2048^2 to 16384^2 lattices): each reserves over a third of the LDS
  a.blocked_lds_floor = s->lds_per_cu > 0 ? s->lds_per_cu / 3 + 1 : 0;
  return a;
}

// Plan of the blocked sweep (or of the blocked adjoint) for this handle: steps
// per pass (the largest count up to the requested one whose on-chip window
// fits; 0: one step per pass) and rows per workgroup segment.  Automatic
// segments (seg_rows = 0) are sized from the number of workgroups the device
// holds at once (see below; measured on 1024^2 to 16384^2 lattices with 3 to 5
// species), at least 8 rows; if 8-row segments leave fewer than 512
// workgroups, one step per pass is faster (small domains: measured on 512^2 to
// 4096^2 ternary FP32 lattices).  32-bit in-plane offsets need plane bytes < 4 GiB.
struct BlockedPlan {
  int tb = 0;
  int seg = 0;
  int cols = msd::kBlockedCols;   // tile width of full passes (remainders use kBlockedCols)
};

BlockedPlan blocked_plan(const msd_sim* s, bool adjoint = false) {
  BlockedPlan pl;
  // the forward sweep on D2Q5 and D2Q4, the blocked adjoint pass on D2Q5 with B of Eq. (2-10)
  const bool d2q5 = s->prob.lattice == MSD_D2Q5;
  if (!d2q5 && !(s->prob.lattice == MSD_D2Q4 && !adjoint)) return pl;
  if (adjoint && s->prob.dilute) return pl;
  if ((uint64_t)s->kp.plane * (uint64_t)s->prob.precision >= (1ull << 32)) return pl;
  const bool xy_walls = s->prob.bc[0] != MSD_BC_PERIODIC || s->prob.bc[2] != MSD_BC_PERIODIC;
  int tb = 0;
  for (int t = s->launch.temporal; t >= 2; --t)
    if (adjoint ? msd::adjoint_blocked_cols(s->m, t, s->prob.precision) > 0
                : msd::blocked_cols(s->m, t, s->prob.precision) > 0 &&
                      (!xy_walls || msd::blocked_walls_ok(s->m, t, s->prob.precision))) {
      tb = t;
      break;
    }
  if (tb == 0) return pl;
  // wide domains: the 512-column tile where one exists, at its own steps per
  // pass if that is fewer (m = 3: five steps on 512 columns beat six on 256)
  if (d2q5 && !adjoint && !s->prob.dilute && (!xy_walls || msd::blocked_wide_walls_ok(s->m)) &&
      s->prob.nx >= msd::kWideMinNx)
    for (int t = tb; t >= 2; --t)
      if (msd::blocked_wide_ok(s->m, t, s->prob.precision)) {
        tb = t;
        pl.cols = msd::kBlockedColsWide;
        break;
      }
  const int64_t W = pl.cols - 2 * tb;
  const int64_t tiles_x = (s->prob.nx + W - 1) / W;
  auto groups = [&](int64_t seg) { return tiles_x * ((s->prob.ny + seg - 1) / seg); };
  int seg = s->launch.seg_rows;
  if (seg <= 0) {
    if (groups(8) < 512) return pl;
    int& cached = (adjoint ? s->resident_adj : s->resident_fwd)[tb];
    if (cached == 0) {
      msd::LaunchArgs a = base_args(s);
      a.tb = tb;
      a.cols = pl.cols;
      a.adjoint = adjoint ? 1 : 0;
      int res[2] = {0, 0};
      a.out_int = res;
      if (dispatch(msd::Op::BlockedResident, a) != hipSuccess || res[0] <= 0 || res[1] <= 0) {
        res[0] = 1024;
        res[1] = 256;
      }
      cached = res[0];
      s->n_cu = res[1];
    }
    if (adjoint) {
      // about 1.35 rounds of the resident workgroups; where that would take
      // segments below 8 rows (small domains), about two workgroups per CU
      // instead (1024^2 ternary FP32: 10-row segments 42.5 ms per 2000 adjoint
      // steps, 8 rows 44.5 ms, 12 rows 47.7 ms, 16 rows 57.3 ms)
      const int64_t target = (int64_t)cached * 27 / 20;
      int64_t rows = (tiles_x * s->prob.ny + target - 1) / target;
      if (rows < 8) {
        const int64_t two_per_cu = 2 * std::max(s->n_cu, 1);
        rows = (tiles_x * s->prob.ny + two_per_cu - 1) / two_per_cu;
      }
      seg = (int)std::max<int64_t>(8, std::min<int64_t>(rows, s->prob.ny));
    } else {
      // Forward sweep: about k * 2 workgroups per CU in all (at most what the
      // device holds at once for k = 1), with the segments as tall as that
      // allows; k doubles while segments stay at least 128 rows tall.  Two
      // waves per SIMD nearly saturate the VALU here, so tall segments (few
      // halo rows) win over occupancy on small lattices, and more workgroups
      // balance better on large ones.
      const int64_t half = std::max(1, std::min(cached, 2 * std::max(s->n_cu, 1)));
      const int64_t ny = s->prob.ny;
      auto seg_for = [&](int64_t k) {
        const int64_t per_tile = std::max<int64_t>(1, k * half / tiles_x);
        return (ny + per_tile - 1) / per_tile;
      };
      int64_t rows = seg_for(1);
      for (int64_t k = 2; k <= 64; k *= 2) {
        const int64_t r = seg_for(k);
        if (r < 128) break;
        rows = r;
      }
      seg = (int)std::max<int64_t>(8, std::min<int64_t>(rows, ny));
    }
  }
  pl.tb = tb;
  pl.seg = seg;
  return pl;
}

// Plan of the temporally blocked 3D sweep (D3Q7, D3Q6): output tile and
// z-planes per workgroup, or tb = 0 for one step per pass.  Automatic segments
// (seg_rows = 0) give about sixteen workgroups per CU in all (one workgroup of
// up to 1024 threads fits a CU at a time), at least 8 planes each (512^3
// quaternary FP32, 64 x 9 tiles, ms per step: 8 planes 3.59, 16 3.34, 32 3.21,
// 48 3.27, 64 3.21, 103 3.26); if 8-plane segments leave fewer than 512
// workgroups the domain is too small to fill the device and one step per pass
// is used.
struct Blocked3dPlan {
  int tb = 0;
  int tx = 0, ty = 0, zseg = 0;
};

Blocked3dPlan blocked3d_plan(const msd_sim* s) {
  Blocked3dPlan pl;
  if (!msd::blocked3d_ok(s->prob.lattice, s->m, s->prob.precision) || s->prob.dilute) return pl;
  if (s->launch.temporal < 2) return pl;
  if ((uint64_t)s->kp.plane * (uint64_t)s->prob.precision >= (1ull << 32)) return pl;
  const int maxt = msd::blocked3d_max_threads(s->m);
  const int tx = s->launch.tile_x > 0 ? s->launch.tile_x : (int)std::min<int64_t>(msd::k3dTileX, s->prob.nx);
  const int ty = s->launch.tile_y > 0 ? s->launch.tile_y : (int)std::min<int64_t>(maxt / (tx + 2) - 2, s->prob.ny);
  if (tx < 1 || ty < 1 || (tx + 2) * (ty + 2) > maxt) return pl;
  const int64_t tiles = ((s->prob.nx + tx - 1) / tx) * ((s->prob.ny + ty - 1) / ty);
  int zseg = s->launch.seg_rows;
  if (zseg <= 0) {
    const int64_t nz = s->prob.nz;
    if (tiles * ((nz + 7) / 8) < 512) return pl;
    int cus = s->n_cu;
    if (cus <= 0) {
      int dev = 0, v = 0;
      cus = (hipGetDevice(&dev) == hipSuccess &&
             hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
                ? v
                : 256;
      s->n_cu = cus;
    }
    const int64_t target = 16 * (int64_t)cus;
    const int64_t segs = std::max<int64_t>(1, (target + tiles - 1) / tiles);
    zseg = (int)std::max<int64_t>(8, (nz + segs - 1) / segs);
  }
  pl.tb = msd::k3dStepsPerPass;
  pl.tx = tx;
  pl.ty = ty;
  pl.zseg = zseg;
  return pl;
}

// ---------------------------------------------------------------------------
// Relaxation radii on the host (msd_relaxation_radius, msd_create).
// ---------------------------------------------------------------------------
double lattice_cs2(int lat) {
  switch (lat) {
    case MSD_D3Q7: return 0.25;
    case MSD_D1Q2: return 1.0;
    case MSD_D2Q4: return 0.5;
    default: return 1.0 / 3.0;   // D1Q3, D2Q5, D3Q6, D2Q9, D3Q15
  }
}

constexpr int kMaxM = MSD_MAX_SPECIES - 1;

// Spectral radius of the m x m matrix A by Gelfand's formula: A^(2^s) by
// repeated squaring, renormalised by its largest entry each time, the log
// scale accumulated; log rho = lim log ||A^k|| / k.
double spectral_radius(const double (&A)[kMaxM][kMaxM], int m) {
  double P[kMaxM][kMaxM], Q[kMaxM][kMaxM];
  double big = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) big = std::max(big, std::fabs(A[i][j]));
  if (big == 0.0) return 0.0;
  double logs = std::log(big);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) P[i][j] = A[i][j] / big;
  double k = 1.0;
  for (int it = 0; it < 48; ++it) {
    double mx = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        double acc = 0.0;
        for (int l = 0; l < m; ++l) acc += P[i][l] * P[l][j];
        Q[i][j] = acc;
        mx = std::max(mx, std::fabs(acc));
      }
    if (mx == 0.0) return 0.0;   // nilpotent
    logs = 2.0 * logs + std::log(mx);
    k *= 2.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) P[i][j] = Q[i][j] / mx;
  }
  return std::exp(logs / k);
}

// Radii of I - Lambda_1 and I - Lambda_2 at composition xi (N values; the
// first N - 1 are used, xi_N = 1 - their sum), for a validated problem.
void relax_radius(const msd_problem* p, const double* xi, double* rho1, double* rho2) {
  const int N = p->n_species, m = N - 1;
  double xb[MSD_MAX_SPECIES];
  double xn = 1.0;
  for (int i = 0; i < m; ++i) {
    xb[i] = p->linearized && p->xi_ref ? p->xi_ref[i] : xi[i];
    xn -= xb[i];
  }
  auto R = [&](int i, int j) { return 1.0 / p->D[i * N + j]; };
  const double h = 0.5 * lattice_cs2(p->lattice);
  // A = I + (a/2) B with B of Eq. (2-10) (or the diagonal dilute-species B)
  double A[kMaxM][2 * kMaxM] = {};
  for (int i = 0; i < m; ++i) {
    double bii;
    if (p->dilute) {
      bii = xn * R(i, m);
      for (int k = 0; k < m; ++k)
        if (k != i) bii += xb[k] * R(i, k);
    } else {
      bii = R(i, m);
      for (int k = 0; k < m; ++k) {
        if (k == i) continue;
        const double S = R(i, k) - R(i, m);
        bii += xb[k] * S;
        A[i][k] = -h * xb[i] * S;
      }
    }
    A[i][i] = 1.0 + h * bii;
    A[i][m + i] = 1.0;
  }
  // K = A^-1 by Gauss-Jordan elimination with partial pivoting
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    if (piv != c)
      for (int j = 0; j < 2 * m; ++j) std::swap(A[c][j], A[piv][j]);
    const double inv = 1.0 / A[c][c];
    for (int j = 0; j < 2 * m; ++j) A[c][j] *= inv;
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      const double f = A[r][c];
      for (int j = 0; j < 2 * m; ++j) A[r][j] -= f * A[c][j];
    }
  }
  // I - Lambda_1 = 2K - I; Lambda_2 replaces the diagonal by the product rule
  // (1/l1 - 1/2)(1/l2 - 1/2) = magic (Eq. (3-16) is magic = 3/16) unless SRT
  double M1[kMaxM][kMaxM], M2[kMaxM][kMaxM];
  const double magic = p->relax == MSD_RELAX_TRT ? p->trt_magic : 3.0 / 16.0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const double l1 = (i == j ? 2.0 : 0.0) - 2.0 * A[i][m + j];
      M1[i][j] = (i == j ? 1.0 : 0.0) - l1;
      double l2 = l1;
      if (i == j && p->relax != MSD_RELAX_SRT) {
        const double g1 = 1.0 - 4.0 * magic;
        l2 = 2.0 * (2.0 - l1) / (2.0 - g1 * l1);
      }
      M2[i][j] = (i == j ? 1.0 : 0.0) - l2;
    }
  *rho1 = spectral_radius(M1, m);
  *rho2 = spectral_radius(M2, m);
}

bool use_lds(const msd_sim* s) {
  if (!s->launch.lds_resident) return false;
  const int64_t cap = msd::lds_resident_max_nodes(s->m, s->q, s->prob.precision);
  return s->L.nodes <= cap && s->L.nodes <= 4096;
}

}  // namespace

extern "C" {

int msd_abi_version(void) { return MSD_ABI_VERSION; }

const char* msd_last_error(void) { return g_last_error.c_str(); }

const char* msd_strerror(int status) {
  switch (status) {
    case MSD_OK: return "ok";
    case MSD_EINVAL: return "invalid argument";
    case MSD_EDIFF: return "invalid diffusivity matrix";
    case MSD_ECOMP: return "composition off the simplex";
    case MSD_ERELAX: return "invalid relaxation rule";
    case MSD_EHIP: return "HIP runtime error";
    case MSD_EDIVERGED: return "non-finite mole fractions";
    case MSD_ENOMEM: return "workspace too small";
    case MSD_EABI: return "ABI version mismatch";
    case MSD_ESTATE: return "call not valid in this state";
    default: return "unknown status";
  }
}

size_t msd_workspace_bytes(const msd_problem* problem, int32_t* status) {
  const int st = validate(problem);
  if (status) *status = st;
  if (st != MSD_OK) return 0;
  return layout_for(problem).total;
}

int msd_create(const msd_problem* problem, void* d_ws, size_t ws_bytes, void* stream, msd_sim** out) {
  if (!out) return fail(MSD_EINVAL, "out is NULL");
  *out = nullptr;
  const int st = validate(problem);
  if (st != MSD_OK) return st;
  const Layout L = layout_for(problem);
  if (!d_ws) return fail(MSD_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(MSD_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(MSD_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  msd_sim* s = new (std::nothrow) msd_sim();
  if (!s) return fail(MSD_EINVAL, "host allocation failed");
  s->prob = *problem;
  s->prob.D = nullptr;
  s->prob.xi_wall = nullptr;
  s->prob.xi_ref = nullptr;
  s->L = L;
  s->m = problem->n_species - 1;
  s->q = lattice_q(problem->lattice);
  s->d = lattice_d(problem->lattice);
  s->ws = static_cast<char*>(d_ws);
  s->stream = static_cast<hipStream_t>(stream);
  fill_kernel_problem(problem, L.plane, &s->kp);
  default_launch(problem, &s->launch);
  // relaxation radii at the pure species, the equimolar mixture, the Dirichlet
  // face compositions and the linearisation composition
  {
    const int N = problem->n_species;
    double xi[MSD_MAX_SPECIES];
    auto check = [&]() {
      double r1 = 0.0, r2 = 0.0;
      relax_radius(problem, xi, &r1, &r2);
      s->rho1 = std::max(s->rho1, r1);
      s->rho2 = std::max(s->rho2, r2);
    };
    for (int v = 0; v < N; ++v) {
      for (int i = 0; i < N; ++i) xi[i] = i == v ? 1.0 : 0.0;
      check();
    }
    for (int i = 0; i < N; ++i) xi[i] = 1.0 / N;
    check();
    if (problem->xi_wall)
      for (int f = 0; f < 6; ++f)
        if (problem->bc[f] == MSD_BC_DIRICHLET) {
          for (int i = 0; i < N; ++i) xi[i] = problem->xi_wall[f * N + i];
          check();
        }
    if (problem->linearized && problem->xi_ref) {
      for (int i = 0; i < N; ++i) xi[i] = problem->xi_ref[i];
      check();
    }
  }
  *out = s;
  return MSD_OK;
}

int msd_set_stream(msd_sim* s, void* stream) {
  if (!s) return fail(MSD_EINVAL, "sim is NULL");
  s->stream = static_cast<hipStream_t>(stream);
  return MSD_OK;
}

int msd_set_launch(msd_sim* s, const msd_launch* l) {
  if (!s || !l) return fail(MSD_EINVAL, "NULL argument");
  msd_launch v = *l;
  if (v.block_x == 0 && v.block_y == 0) {
    msd_launch d;
    default_launch(&s->prob, &d);
    v.block_x = d.block_x;
    v.block_y = d.block_y;
  }
  if (v.nontemporal < 0 || v.nontemporal > 7) return fail(MSD_EINVAL, "nontemporal mask %d", v.nontemporal);
  if (v.temporal < 0 || v.temporal > msd::kMaxStepsPerPass)
    return fail(MSD_EINVAL, "temporal = %d must be 0..%d", v.temporal, msd::kMaxStepsPerPass);
  if (v.seg_rows < 0 || v.seg_rows > (1 << 20)) return fail(MSD_EINVAL, "seg_rows = %d", v.seg_rows);
  if (v.tile_x < 0 || v.tile_y < 0 || (v.tile_x > 0) != (v.tile_y > 0) ||
      (v.tile_x > 0 && (v.tile_x + 2) * (v.tile_y + 2) > 1024))
    return fail(MSD_EINVAL, "tile %d x %d: both 0, or both positive with (tile_x + 2) * (tile_y + 2) <= 1024",
                v.tile_x, v.tile_y);
  if (v.vec != 0 && v.vec != 1 && v.vec != 2 && v.vec != 4)
    return fail(MSD_EINVAL, "vec = %d must be 0, 1, 2 or 4", v.vec);
  if (v.block_x < 64 || v.block_x % 64 || v.block_y < 1 || v.block_x * v.block_y > 256)
    return fail(MSD_EINVAL, "block %d x %d: block_x must be a positive multiple of 64, product <= 256", v.block_x,
                v.block_y);
  s->launch = v;
  return MSD_OK;
}

int msd_get_launch(const msd_sim* s, msd_launch* l) {
  if (!s || !l) return fail(MSD_EINVAL, "NULL argument");
  *l = s->launch;
  return MSD_OK;
}

int msd_steps_per_pass(const msd_sim* s) {
  if (!s) return fail(MSD_EINVAL, "NULL argument");
  const int tb = std::max(blocked_plan(s).tb, blocked3d_plan(s).tb);
  return tb >= 2 ? tb : 1;
}

int msd_init(msd_sim* s, const void* d_xi0, int32_t xi0_precision) {
  if (!s || !d_xi0) return fail(MSD_EINVAL, "NULL argument");
  if (xi0_precision != MSD_F32 && xi0_precision != MSD_F64) return fail(MSD_EINVAL, "xi0_precision %d", xi0_precision);
  msd::LaunchArgs a = base_args(s);
  a.consts_out = s->ws + s->L.consts_off;
  hipError_t e = dispatch(msd::Op::Constants, a);
  if (e != hipSuccess) return hip_fail(e, "constants kernel");
  a.xi0 = d_xi0;
  a.in_prec = xi0_precision;
  s->cur = 0;
  a.dst = s->ws + s->L.half_off[0];
  e = dispatch(msd::Op::Init, a);
  if (e != hipSuccess) return hip_fail(e, "init kernel");
  // totals of the initial field: the reference of the drift check in msd_diagnostics
  a.src = s->ws + s->L.half_off[0];
  a.pull = 0;
  a.partials = reinterpret_cast<double*>(s->ws + s->L.partials_off);
  a.diag_out = reinterpret_cast<double*>(s->ws + s->L.ref_off);
  a.diag_blocks = s->L.diag_blocks;
  e = dispatch(msd::Op::DiagPartial, a);
  if (e != hipSuccess) return hip_fail(e, "diagnostics kernel");
  e = dispatch(msd::Op::DiagFinal, a);
  if (e != hipSuccess) return hip_fail(e, "diagnostics reduction kernel");
  s->t = 0;
  s->initialised = true;
  return MSD_OK;
}

int msd_step(msd_sim* s, int64_t nsteps) {
  if (!s) return fail(MSD_EINVAL, "sim is NULL");
  if (!s->initialised) return fail(MSD_ESTATE, "msd_step before msd_init");
  if (nsteps < 0) return fail(MSD_EINVAL, "nsteps < 0");
  if (nsteps == 0) return MSD_OK;
  msd::LaunchArgs a = base_args(s);
  if (use_lds(s)) {
    a.src = s->ws + s->L.half_off[s->cur];
    a.dst = s->ws + s->L.half_off[1 - s->cur];
    a.pull = s->t > 0 ? 1 : 0;
    a.nsteps = nsteps;
    const hipError_t e = dispatch(msd::Op::StepLds, a);
    if (e != hipSuccess) return hip_fail(e, "LDS-resident step kernel");
    s->cur = 1 - s->cur;
    s->t += nsteps;
    return MSD_OK;
  }
  const BlockedPlan plan = blocked_plan(s);
  const Blocked3dPlan plan3 = blocked3d_plan(s);
  const int tb = std::max(plan.tb, plan3.tb);
  int64_t n = 0;
  // Blocked runs: the first step after msd_init reads pre-collision values and
  // runs alone; the rest runs in ceil(rest / tb) passes of near-equal length
  // (lengths floor and ceil of rest / passes, the longer ones first), so a run
  // whose length is not a multiple of tb has no short remainder pass.
  const int64_t first = (tb >= 2 && s->t == 0) ? 1 : 0;
  const int64_t rest = nsteps - std::min<int64_t>(first, nsteps);
  const int64_t passes = tb >= 2 ? (rest + tb - 1) / tb : 0;
  const int64_t base = passes > 0 ? rest / passes : 0, longer = passes > 0 ? rest % passes : 0;
  int64_t pass_index = 0;
  while (n < nsteps) {
    a.src = s->ws + s->L.half_off[s->cur];
    a.dst = s->ws + s->L.half_off[1 - s->cur];
    a.pull = s->t > 0 ? 1 : 0;
    int64_t done = 1;
    hipError_t e;
    const int pass = (tb >= 2 && n >= first) ? (int)(base + (pass_index < longer ? 1 : 0)) : 1;
    if (pass >= 2 && plan3.tb >= 2) {
      a.tb = pass;
      a.tile_x = plan3.tx;
      a.tile_y = plan3.ty;
      a.seg_rows = plan3.zseg;
      e = dispatch(msd::Op::StepBlocked3d, a);
      done = pass;
    } else if (pass >= 2) {
      // the full-length passes take the plan's tile width, shorter ones kBlockedCols
      a.tb = pass;
      a.cols = pass == tb ? plan.cols : 0;
      a.seg_rows = plan.seg;
      e = dispatch(msd::Op::StepBlocked, a);
      done = pass;
    } else {
      e = dispatch(msd::Op::Step, a);
    }
    if (e != hipSuccess) return hip_fail(e, "step kernel");
    if (tb >= 2 && n >= first) ++pass_index;
    s->cur = 1 - s->cur;
    s->t += done;
    n += done;
  }
  return MSD_OK;
}

int64_t msd_time(const msd_sim* s) { return s ? s->t : -1; }

int msd_read_moments(msd_sim* s, int32_t out_precision, void* d_xi, void* d_J, void* d_grad) {
  if (!s || !d_xi) return fail(MSD_EINVAL, "NULL argument");
  if (!s->initialised) return fail(MSD_ESTATE, "read before msd_init");
  if (out_precision != MSD_F32 && out_precision != MSD_F64) return fail(MSD_EINVAL, "out_precision %d", out_precision);
  msd::LaunchArgs a = base_args(s);
  a.src = s->ws + s->L.half_off[s->cur];
  a.pull = s->t > 0 ? 1 : 0;
  a.out_prec = out_precision;
  a.out_xi = d_xi;
  a.out_J = d_J;
  a.out_grad = d_grad;
  const hipError_t e = dispatch(msd::Op::Read, a);
  if (e != hipSuccess) return hip_fail(e, "read kernel");
  return MSD_OK;
}

int msd_diagnostics(msd_sim* s, double* h_mass, double* h_min, double* h_max, int64_t* h_nonfinite) {
  if (!s) return fail(MSD_EINVAL, "sim is NULL");
  if (!s->initialised) return fail(MSD_ESTATE, "diagnostics before msd_init");
  msd::LaunchArgs a = base_args(s);
  a.src = s->ws + s->L.half_off[s->cur];
  a.pull = s->t > 0 ? 1 : 0;
  a.partials = reinterpret_cast<double*>(s->ws + s->L.partials_off);
  a.diag_out = reinterpret_cast<double*>(s->ws + s->L.diag_out_off);
  a.diag_blocks = s->L.diag_blocks;
  hipError_t e = dispatch(msd::Op::DiagPartial, a);
  if (e != hipSuccess) return hip_fail(e, "diagnostics kernel");
  e = dispatch(msd::Op::DiagFinal, a);
  if (e != hipSuccess) return hip_fail(e, "diagnostics reduction kernel");
  const int N = s->prob.n_species;
  double host[3 * MSD_MAX_SPECIES + 1], ref[MSD_MAX_SPECIES];
  e = hipMemcpyAsync(host, a.diag_out, sizeof(double) * (3 * N + 1), hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics copy");
  e = hipMemcpyAsync(ref, s->ws + s->L.ref_off, sizeof(double) * N, hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics copy");
  e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics synchronise");
  for (int i = 0; i < N; ++i) {
    if (h_mass) h_mass[i] = host[i];
    if (h_min) h_min[i] = host[N + i];
    if (h_max) h_max[i] = host[2 * N + i];
  }
  const int64_t bad = (int64_t)host[3 * N];
  if (h_nonfinite) *h_nonfinite = bad;
  if (bad) return fail(MSD_EDIVERGED, "%lld non-finite mole fractions", (long long)bad);
  const msd_health& hl = s->health;
  for (int i = 0; i < N; ++i)
    if (hl.neg_tol >= 0.0 && host[N + i] < -hl.neg_tol)
      return fail(MSD_EDIVERGED, "mole fraction of species %d down to %g (below -%g)", i + 1, host[N + i],
                  hl.neg_tol);
  bool dirichlet = false;
  for (int f = 0; f < 6; ++f) dirichlet = dirichlet || s->prob.bc[f] == MSD_BC_DIRICHLET;
  if (!dirichlet && hl.mass_rtol >= 0.0)
    for (int i = 0; i < N; ++i)
      if (std::fabs(host[i] - ref[i]) > hl.mass_rtol * (double)s->L.nodes)
        return fail(MSD_EDIVERGED, "total of species %d drifted from %.17g to %.17g (more than %g per node)", i + 1,
                    ref[i], host[i], hl.mass_rtol);
  return MSD_OK;
}

int msd_set_health(msd_sim* s, const msd_health* h) {
  if (!s || !h) return fail(MSD_EINVAL, "NULL argument");
  if (std::isnan(h->neg_tol) || std::isnan(h->mass_rtol)) return fail(MSD_EINVAL, "NaN limit");
  s->health = *h;
  return MSD_OK;
}

int msd_get_health(const msd_sim* s, msd_health* h) {
  if (!s || !h) return fail(MSD_EINVAL, "NULL argument");
  *h = s->health;
  return MSD_OK;
}

int msd_relaxation_radius(const msd_problem* problem, const double* h_xi, int32_t count, double* h_rho) {
  const int st = validate(problem);
  if (st != MSD_OK) return st;
  if (count < 0 || (count > 0 && (!h_xi || !h_rho))) return fail(MSD_EINVAL, "count = %d or NULL arrays", count);
  const int N = problem->n_species;
  for (int32_t c = 0; c < count; ++c) relax_radius(problem, h_xi + (size_t)c * N, &h_rho[2 * c], &h_rho[2 * c + 1]);
  return MSD_OK;
}

int msd_stability(const msd_sim* s, double* h_rho1, double* h_rho2) {
  if (!s) return fail(MSD_EINVAL, "sim is NULL");
  if (h_rho1) *h_rho1 = s->rho1;
  if (h_rho2) *h_rho2 = s->rho2;
  return MSD_OK;
}

size_t msd_state_bytes(const msd_sim* s) {
  if (!s) return 0;
  return (size_t)s->m * s->q * (size_t)s->L.plane * s->prob.precision;
}

int msd_save(const msd_sim* s, void* d_dst, int64_t* h_step) {
  if (!s || !d_dst) return fail(MSD_EINVAL, "NULL argument");
  if (!s->initialised) return fail(MSD_ESTATE, "save before msd_init");
  const hipError_t e = hipMemcpyAsync(d_dst, s->ws + s->L.half_off[s->cur], msd_state_bytes(s),
                                      hipMemcpyDeviceToDevice, s->stream);
  if (e != hipSuccess) return hip_fail(e, "save copy");
  if (h_step) *h_step = s->t;
  return MSD_OK;
}

int msd_restore(msd_sim* s, const void* d_src, int64_t step) {
  if (!s || !d_src) return fail(MSD_EINVAL, "NULL argument");
  if (step < 0) return fail(MSD_EINVAL, "step < 0");
  if (!s->initialised) {
    // constants are produced by msd_init; a restore needs them as well
    return fail(MSD_ESTATE, "restore before msd_init");
  }
  const hipError_t e = hipMemcpyAsync(s->ws + s->L.half_off[s->cur], d_src, msd_state_bytes(s),
                                      hipMemcpyDeviceToDevice, s->stream);
  if (e != hipSuccess) return hip_fail(e, "restore copy");
  s->t = step;
  return MSD_OK;
}

int msd_record(msd_sim* s, int64_t nsteps, void* d_stack) {
  if (!s || !d_stack) return fail(MSD_EINVAL, "NULL argument");
  if (!s->initialised) return fail(MSD_ESTATE, "msd_record before msd_init");
  if (nsteps < 0) return fail(MSD_EINVAL, "nsteps < 0");
  if (nsteps == 0) return MSD_OK;
  const size_t sb = msd_state_bytes(s);
  char* stack = static_cast<char*>(d_stack);
  msd::LaunchArgs a = base_args(s);
  const BlockedPlan plan = blocked_plan(s);
  int64_t n = 0;
  while (n < nsteps) {
    a.src = n == 0 ? (const void*)(s->ws + s->L.half_off[s->cur]) : (const void*)(stack + (size_t)(n - 1) * sb);
    a.dst = stack + (size_t)n * sb;
    a.pull = (s->t + n) > 0 ? 1 : 0;
    int64_t done = 1;
    hipError_t e;
    const int pass = (int)std::min<int64_t>(plan.tb, nsteps - n);
    if (plan.tb >= 2 && s->t + n > 0 && pass >= 2) {
      // one pass writes the states after each of its steps into consecutive slots
      a.tb = pass;
      a.cols = pass == plan.tb ? plan.cols : 0;
      a.seg_rows = plan.seg;
      a.rec_stride = (int64_t)(sb / (size_t)s->prob.precision);
      e = dispatch(msd::Op::StepBlocked, a);
      a.rec_stride = 0;
      done = pass;
    } else {
      e = dispatch(msd::Op::Step, a);
    }
    if (e != hipSuccess) return hip_fail(e, "step kernel");
    n += done;
  }
  const hipError_t e = hipMemcpyAsync(s->ws + s->L.half_off[s->cur], stack + (size_t)(nsteps - 1) * sb, sb,
                                      hipMemcpyDeviceToDevice, s->stream);
  if (e != hipSuccess) return hip_fail(e, "record copy");
  s->t += nsteps;
  return MSD_OK;
}

// Workgroup slots of the dL/dR accumulator: enough for the one-step adjoint
// tiling and for the blocked adjoint's (tile, segment) workgroups.
static int64_t adjoint_slots(const msd_sim* s) {
  const int64_t bx = (int64_t)s->launch.block_x * msd::kAdjointNodesPerThread, by = s->launch.block_y;
  int64_t slots = (s->prob.nx + bx - 1) / bx * ((s->prob.ny + by - 1) / by) * s->prob.nz;
  const BlockedPlan plan = blocked_plan(s, true);
  if (plan.tb >= 2) {
    const int64_t W = msd::kBlockedCols - 2 * plan.tb;
    slots = std::max<int64_t>(slots, (s->prob.nx + W - 1) / W * ((s->prob.ny + plan.seg - 1) / plan.seg));
  }
  return slots;
}

size_t msd_adjoint_accum_bytes(const msd_sim* s) {
  if (!s) return 0;
  return sizeof(double) * (size_t)adjoint_slots(s) * s->m * (s->m + 1);
}

int msd_adjoint_begin(msd_sim* s, void* d_accum) {
  if (!s || !d_accum) return fail(MSD_EINVAL, "NULL argument");
  msd::LaunchArgs a = base_args(s);
  a.partials = static_cast<double*>(d_accum);
  a.fill_count = (int64_t)(msd_adjoint_accum_bytes(s) / sizeof(double));
  const hipError_t e = dispatch(msd::Op::FillZero, a);
  if (e != hipSuccess) return hip_fail(e, "fill kernel");
  return MSD_OK;
}

int msd_adjoint_seed(msd_sim* s, const double* d_dL_dxi, void* d_adj_out) {
  if (!s || !d_dL_dxi || !d_adj_out) return fail(MSD_EINVAL, "NULL argument");
  if (!s->initialised) return fail(MSD_ESTATE, "adjoint before msd_init");
  msd::LaunchArgs a = base_args(s);
  a.xi0 = d_dL_dxi;
  a.dst = d_adj_out;
  a.pull = s->t > 0 ? 1 : 0;
  const hipError_t e = dispatch(msd::Op::AdjointSeed, a);
  if (e != hipSuccess) return hip_fail(e, "adjoint seed kernel");
  return MSD_OK;
}

int msd_adjoint_step(msd_sim* s, int64_t t, const void* d_state_prev, const void* d_adj_in, void* d_adj_out,
                     void* d_accum) {
  if (!s || !d_state_prev || !d_adj_in || !d_adj_out || !d_accum) return fail(MSD_EINVAL, "NULL argument");
  if (!s->initialised) return fail(MSD_ESTATE, "adjoint before msd_init");
  if (t < 1) return fail(MSD_EINVAL, "adjoint step t = %lld < 1", (long long)t);
  if (d_adj_in == d_adj_out) return fail(MSD_EINVAL, "adjoint input and output must differ");
  msd::LaunchArgs a = base_args(s);
  a.src = d_state_prev;
  a.adj_in = d_adj_in;
  a.dst = d_adj_out;
  a.pull = t >= 2 ? 1 : 0;   // s_{t-1} holds pre-collision values only for t = 1
  a.partials = static_cast<double*>(d_accum);
  const hipError_t e = dispatch(msd::Op::AdjointStep, a);
  if (e != hipSuccess) return hip_fail(e, "adjoint step kernel");
  return MSD_OK;
}

int msd_adjoint_steps(msd_sim* s, int64_t t_hi, int64_t t_lo, const void* d_state_lo, const void* d_stack,
                      void* d_adj_a, void* d_adj_b, void* d_accum, int32_t* h_result_in_b) {
  if (!s || !d_state_lo || !d_adj_a || !d_adj_b || !d_accum || !h_result_in_b)
    return fail(MSD_EINVAL, "NULL argument");
  if (t_lo < 0 || t_hi < t_lo) return fail(MSD_EINVAL, "steps (%lld, %lld]", (long long)t_lo, (long long)t_hi);
  if (t_hi - t_lo > 1 && !d_stack) return fail(MSD_EINVAL, "stack is NULL");
  if (!s->initialised) return fail(MSD_ESTATE, "adjoint before msd_init");
  if (d_adj_a == d_adj_b) return fail(MSD_EINVAL, "the two adjoint buffers must differ");
  const size_t sb = msd_state_bytes(s);
  void* a = d_adj_a;
  void* b = d_adj_b;
  int in_b = 0;
  // s_j for t_lo <= j < t_hi: the segment's first state, else its stack slot
  auto state = [&](int64_t j) {
    return j == t_lo ? d_state_lo : (const void*)(static_cast<const char*>(d_stack) + (size_t)(j - t_lo - 1) * sb);
  };
  const BlockedPlan plan = blocked_plan(s, true);
  int64_t t = t_hi;
  while (t > t_lo) {
    int64_t done = 1;
    if (plan.tb >= 2 && t - plan.tb >= std::max<int64_t>(t_lo, 1)) {
      // adjoint steps t .. t - tb + 1 in one pass; every level pulls its state
      msd::LaunchArgs la = base_args(s);
      for (int l = 1; l <= plan.tb; ++l) la.states[l - 1] = state(t - l);
      la.adj_in = a;
      la.dst = b;
      la.tb = plan.tb;
      la.seg_rows = plan.seg;
      la.partials = static_cast<double*>(d_accum);
      const hipError_t e = dispatch(msd::Op::AdjointBlocked, la);
      if (e != hipSuccess) return hip_fail(e, "blocked adjoint kernel");
      done = plan.tb;
    } else {
      const int st = msd_adjoint_step(s, t, state(t - 1), a, b, d_accum);
      if (st != MSD_OK) return st;
    }
    void* tmp = a;
    a = b;
    b = tmp;
    in_b ^= 1;
    t -= done;
  }
  *h_result_in_b = in_b;
  return MSD_OK;
}

int msd_adjoint_finish(msd_sim* s, const void* d_adj0, const void* d_accum, double* d_dL_dxi0, double* h_dL_dD) {
  if (!s || !d_adj0 || !d_accum) return fail(MSD_EINVAL, "NULL argument");
  msd::LaunchArgs a = base_args(s);
  a.adj_in = d_adj0;
  hipError_t e;
  if (d_dL_dxi0) {
    a.out_xi = d_dL_dxi0;
    e = dispatch(msd::Op::AdjointXi0, a);
    if (e != hipSuccess) return hip_fail(e, "adjoint initial-field kernel");
  }
  if (h_dL_dD) {
    a.partials = static_cast<double*>(const_cast<void*>(d_accum));
    a.accum_slots = adjoint_slots(s);
    a.diag_out = reinterpret_cast<double*>(s->ws + s->L.diag_out_off);
    e = dispatch(msd::Op::AdjointDD, a);
    if (e != hipSuccess) return hip_fail(e, "adjoint diffusivity kernel");
    const int N = s->prob.n_species;
    double host[MSD_MAX_SPECIES * MSD_MAX_SPECIES];
    e = hipMemcpyAsync(host, a.diag_out, sizeof(double) * N * N, hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint copy");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint synchronise");
    for (int i = 0; i < N * N; ++i) h_dL_dD[i] = host[i];
  } else {
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint synchronise");
  }
  return MSD_OK;
}

// Scratch of msd_adjoint: the dL/dR accumulator, two adjoint buffers and a
// recomputation stack of every - 1 states, each 256-byte aligned.
struct AdjointScratch {
  size_t acc = 0, a0 = 0, a1 = 0, stack = 0, total = 0;
};

static AdjointScratch adjoint_scratch(const msd_sim* s, int64_t every) {
  AdjointScratch L;
  const size_t sb = align_up(msd_state_bytes(s), 256);
  L.acc = 0;
  L.a0 = align_up(msd_adjoint_accum_bytes(s), 256);
  L.a1 = L.a0 + sb;
  L.stack = L.a1 + sb;
  L.total = L.stack + (size_t)std::max<int64_t>(every - 1, 1) * msd_state_bytes(s);
  return L;
}

size_t msd_adjoint_scratch_bytes(const msd_sim* s, int64_t every) {
  if (!s || every < 1) return 0;
  return adjoint_scratch(s, every).total;
}

int msd_forward_checkpointed(msd_sim* s, int64_t nsteps, int64_t every, void* d_ckpts) {
  if (!s) return fail(MSD_EINVAL, "sim is NULL");
  if (nsteps < 0 || every < 1) return fail(MSD_EINVAL, "nsteps = %lld, every = %lld", (long long)nsteps,
                                           (long long)every);
  if (nsteps > 0 && !d_ckpts) return fail(MSD_EINVAL, "checkpoint buffer is NULL");
  if (!s->initialised || s->t != 0) return fail(MSD_ESTATE, "checkpointed runs start right after msd_init");
  const size_t sb = msd_state_bytes(s);
  char* ck = static_cast<char*>(d_ckpts);
  for (int64_t j = 0; s->t < nsteps; ++j) {
    int st = msd_save(s, ck + (size_t)j * sb, nullptr);
    if (st != MSD_OK) return st;
    st = msd_step(s, std::min(every, nsteps - s->t));
    if (st != MSD_OK) return st;
  }
  return MSD_OK;
}

int msd_adjoint(msd_sim* s, int64_t nsteps, int64_t every, const void* d_ckpts, const double* d_dL_dxi,
                double* d_dL_dxi0, double* h_dL_dD, void* d_scratch, size_t scratch_bytes) {
  if (!s || !d_dL_dxi || !d_scratch) return fail(MSD_EINVAL, "NULL argument");
  if (nsteps < 0 || every < 1) return fail(MSD_EINVAL, "nsteps = %lld, every = %lld", (long long)nsteps,
                                           (long long)every);
  if (nsteps > 0 && !d_ckpts) return fail(MSD_EINVAL, "checkpoint buffer is NULL");
  if (!s->initialised || s->t != nsteps)
    return fail(MSD_ESTATE, "the handle is at time %lld, not at the end (%lld) of the checkpointed run",
                (long long)s->t, (long long)nsteps);
  if (reinterpret_cast<uintptr_t>(d_scratch) % 256) return fail(MSD_EINVAL, "scratch must be 256-byte aligned");
  const AdjointScratch L = adjoint_scratch(s, every);
  if (scratch_bytes < L.total) return fail(MSD_ENOMEM, "scratch of %zu bytes, %zu needed", scratch_bytes, L.total);
  char* w = static_cast<char*>(d_scratch);
  void* acc = w + L.acc;
  void* a = w + L.a0;
  void* b = w + L.a1;
  void* stack = w + L.stack;
  const size_t sb = msd_state_bytes(s);
  const char* ck = static_cast<const char*>(d_ckpts);
  int st = msd_adjoint_begin(s, acc);
  if (st != MSD_OK) return st;
  st = msd_adjoint_seed(s, d_dL_dxi, a);
  if (st != MSD_OK) return st;
  const int64_t segs = (nsteps + every - 1) / every;
  for (int64_t j = segs - 1; j >= 0; --j) {
    const int64_t t0 = j * every, t1 = std::min(t0 + every, nsteps);
    const void* c0 = ck + (size_t)j * sb;
    if (t1 - t0 > 1) {
      st = msd_restore(s, c0, t0);
      if (st != MSD_OK) return st;
      st = msd_record(s, t1 - t0 - 1, stack);
      if (st != MSD_OK) return st;
    }
    int32_t in_b = 0;
    st = msd_adjoint_steps(s, t1, t0, c0, stack, a, b, acc, &in_b);
    if (st != MSD_OK) return st;
    if (in_b) std::swap(a, b);
  }
  return msd_adjoint_finish(s, a, acc, d_dL_dxi0, h_dL_dD);
}

}  // extern "C"

// Scratch of msd_adjoint_noalloc: a device array in this file's code object
// (each GPU the library runs on holds its own copy until the process ends).
// In host code its name stands for a host-side symbol, not a device address:
// the device address comes from hipGetSymbolAddress, once per device, and only
// that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[MSD_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
int static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(MSD_EINVAL, "device %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MSD_OK;
}

}  // namespace

extern "C" {

int msd_adjoint_noalloc(msd_sim* s, int64_t nsteps, int64_t every, const void* d_ckpts, const double* d_dL_dxi,
                        double* d_dL_dxi0, double* h_dL_dD) {
  if (!s || !d_dL_dxi) return fail(MSD_EINVAL, "NULL argument");
  if (every < 1) return fail(MSD_EINVAL, "every = %lld", (long long)every);
  const size_t need = adjoint_scratch(s, every).total;
  if (need > MSD_STATIC_SCRATCH_BYTES)
    return fail(MSD_ENOMEM, "adjoint scratch of %zu bytes exceeds the static array of %zu bytes (msd_adjoint takes "
                "caller scratch of any size)", need, (size_t)MSD_STATIC_SCRATCH_BYTES);
  void* p = nullptr;
  const int st = static_scratch(&p);
  if (st != MSD_OK) return st;
  return msd_adjoint(s, nsteps, every, d_ckpts, d_dL_dxi, d_dL_dxi0, h_dL_dD, p, MSD_STATIC_SCRATCH_BYTES);
}

int msd_tune(msd_sim* s, const msd_launch* candidates, int32_t count, int32_t steps, double budget_ms,
             const char* cache_path, int32_t flags, void* d_scratch, size_t scratch_bytes, msd_launch* h_best,
             double* h_ms_per_step, double* h_trial_ms) {
  if (!s) return fail(MSD_EINVAL, "sim is NULL");
  if (steps < 1) return fail(MSD_EINVAL, "steps = %d", steps);
  if (count < 0 || (count > 0 && !candidates)) return fail(MSD_EINVAL, "count = %d", count);
  if (!s->initialised) return fail(MSD_ESTATE, "tuning before msd_init");
  // key: architecture, lattice, precision, species, extents, faces
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s|sim|%d|%d|N%d|%lldx%lldx%lld|%d%d%d%d%d%d", device_arch().c_str(),
                s->prob.lattice, s->prob.precision, s->prob.n_species, (long long)s->prob.nx, (long long)s->prob.ny,
                (long long)s->prob.nz, s->prob.bc[0], s->prob.bc[1], s->prob.bc[2], s->prob.bc[3], s->prob.bc[4],
                s->prob.bc[5]);
  const std::string key = buf;
  constexpr int K = 10;
  auto pack = [](const msd_launch& l, int64_t* v) {
    v[0] = l.block_x; v[1] = l.block_y; v[2] = l.xcd_remap; v[3] = l.lds_resident;
    v[4] = l.nontemporal; v[5] = l.vec; v[6] = l.temporal; v[7] = l.seg_rows;
    v[8] = l.tile_x; v[9] = l.tile_y;
  };
  auto unpack = [](const int64_t* v) {
    msd_launch l;
    l.block_x = (int32_t)v[0]; l.block_y = (int32_t)v[1]; l.xcd_remap = (int32_t)v[2]; l.lds_resident = (int32_t)v[3];
    l.nontemporal = (int32_t)v[4]; l.vec = (int32_t)v[5]; l.temporal = (int32_t)v[6]; l.seg_rows = (int32_t)v[7];
    l.tile_x = (int32_t)v[8]; l.tile_y = (int32_t)v[9];
    return l;
  };
  int64_t cached[K];
  double cms = 0.0;
  if (!(flags & MSD_TUNE_IGNORE_CACHE) && cache_lookup(cache_path, key, K, cached, &cms)) {
    const msd_launch l = unpack(cached);
    const int st = msd_set_launch(s, &l);
    if (st == MSD_OK) {
      if (h_best) *h_best = l;
      if (h_ms_per_step) *h_ms_per_step = cms;
      return MSD_OK;
    }
  }
  std::vector<msd_launch> cand;
  if (count > 0) {
    cand.assign(candidates, candidates + count);
  } else {
    const int blocks[5][2] = {{256, 1}, {128, 2}, {64, 4}, {128, 1}, {64, 1}};
    msd_launch base = s->launch;
    for (auto& b : blocks)
      for (int vec : {0, 1, 4})
        for (int xcd : {0, 1})
          for (int nt : {0, 7}) {
            if (vec > 0 && lattice_q(s->prob.lattice) > 2 * lattice_d(s->prob.lattice) + 1) continue;  // no vector kernel
            msd_launch l = base;
            l.block_x = b[0]; l.block_y = b[1]; l.vec = vec; l.xcd_remap = xcd; l.nontemporal = nt; l.temporal = 0;
            cand.push_back(l);
          }
    if (s->prob.lattice == MSD_D2Q5 || s->prob.lattice == MSD_D2Q4)
      for (int tb : {2, 3, 4, 5, 6})
        for (int seg : {0, 16, 32, 48})
          for (int nt : {0, 1}) {
            msd_launch l = base;
            l.temporal = tb; l.seg_rows = seg; l.nontemporal = nt; l.vec = 0;
            cand.push_back(l);
          }
    if (msd::blocked3d_ok(s->prob.lattice, s->m, s->prob.precision) && !s->prob.dilute) {
      const int tiles[5][2] = {{0, 0}, {62, 14}, {30, 30}, {64, 6}, {126, 6}};
      for (auto& t : tiles)
        for (int zseg : {0, 16, 32, 64})
          for (int xcd : {0, 1}) {
            msd_launch l = base;
            l.temporal = msd::k3dStepsPerPass; l.tile_x = t[0]; l.tile_y = t[1]; l.seg_rows = zseg;
            l.xcd_remap = xcd; l.vec = 0;
            cand.push_back(l);
          }
    }
  }
  const size_t sb = msd_state_bytes(s);
  if (!d_scratch || scratch_bytes < sb) return fail(MSD_ENOMEM, "scratch of %zu bytes, %zu needed", scratch_bytes, sb);
  const msd_launch keep = s->launch;
  int64_t t0 = 0;
  int st = msd_save(s, d_scratch, &t0);
  if (st != MSD_OK) return st;
  std::vector<double> ms(cand.size(), -1.0);
  int best = -1;
  st = time_candidates(
      s->stream, (int)cand.size(), steps, budget_ms, [&](int i) { return msd_set_launch(s, &cand[i]); },
      [&](int n) { return msd_step(s, n); }, [&]() { return msd_restore(s, d_scratch, t0); }, ms.data(), &best);
  if (h_trial_ms)
    for (size_t i = 0; i < cand.size(); ++i) h_trial_ms[i] = ms[i];
  if (st != MSD_OK) {
    msd_set_launch(s, &keep);
    return st;
  }
  if (best < 0) {
    msd_set_launch(s, &keep);
    return fail(MSD_EINVAL, "no candidate launch could run");
  }
  st = msd_set_launch(s, &cand[best]);
  if (st != MSD_OK) return st;
  int64_t v[K];
  pack(s->launch, v);
  cache_store(cache_path, key, K, v, ms[best]);
  if (h_best) *h_best = s->launch;
  if (h_ms_per_step) *h_ms_per_step = ms[best];
  return MSD_OK;
}

int msd_destroy(msd_sim* s) {
  delete s;
  return MSD_OK;
}

}  // extern "C"
