// Host-side launch interface between the C ABI layer and the per-lattice
// kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "msd_device.h"

namespace msd {

enum class Op {
  Constants, Init, Step, StepLds, Read, DiagPartial, DiagFinal, BatchStep,
  AdjointSeed, AdjointStep, AdjointXi0, AdjointDD, FillZero, StepBlocked, BatchStepBlocked,
  AdjointBlocked, BlockedResident, StepBlocked3d
};

// Constants block written once per problem by the setup kernel and read by
// every sweep kernel through uniform (scalar-cache) loads: R = 1/D (m rows of
// N entries), Dirichlet face values and the linearisation composition, in the
// sweep's precision.
template <typename T>
struct Consts {
  T R[kMaxSpecies][kMaxSpecies];
  T wall[6][kMaxSpecies];
  T xref[kMaxSpecies];
  // collision coefficients (CollideCoef): A = I + (a/2) B as an affine map of
  // the composition, and the relaxation-rule factors
  T a0[kMaxSpecies];
  T ds[kMaxSpecies];
  T da[kMaxSpecies][kMaxSpecies];
  T ea[kMaxSpecies][kMaxSpecies];
  T ga[kMaxSpecies][kMaxSpecies];
  T rule[7];
};
constexpr size_t kConstsBytes = 4096;   // >= sizeof(Consts<double>) = 2712
static_assert(sizeof(Consts<double>) <= kConstsBytes, "constants block too small");

// One mixture of a batch, as the batched sweep sees it (device array, read
// through uniform loads).  Offsets are bytes into the batch workspace.
struct BatchInst {
  Problem p;
  int32_t m;
  int32_t reserved;
  uint64_t half_off[2];
  uint64_t consts_off;
};

// One workgroup of a batched launch: which mixture, which tile of it.
struct BatchTile {
  uint32_t inst;
  uint32_t tile;
};

struct LaunchArgs {
  Problem p;
  int lattice = 0, m = 0, prec = 4;
  hipStream_t stream = nullptr;
  // sweep
  const void* src = nullptr;
  void* dst = nullptr;
  const void* consts = nullptr;
  void* consts_out = nullptr;
  int pull = 1;
  int block_x = 256, block_y = 1;
  int xcd_remap = 1;
  int nontemporal = 0;
  int vec = 1;               // nodes per thread of the vectorised sweep (0: general kernel)
  int tb = 0;                // steps per pass of the temporally blocked sweep
  int seg_rows = 32;         // rows per workgroup segment of the blocked sweep
  int walls = 0;             // blocked batch launch: some mixture has a non-periodic face
  int cols = 0;              // blocked sweep of one mixture: tile width (0: kBlockedCols)
  int dilute = 0;            // batch launches: the range holds dilute-species mixtures
  int64_t rec_stride = 0;    // blocked sweep: elements between recorded states (0: no recording)
  const void* states[4] = {nullptr, nullptr, nullptr, nullptr};   // blocked adjoint: s_{t-1}, ..., s_{t-TB}
  int64_t accum_slots = 0;   // adjoint: workgroup slots of the dL/dR accumulator
  int blocked_lds_floor = 0; // blocked sweep: LDS bytes each workgroup reserves at least (caps residency)
  int adjoint = 0;           // BlockedResident: query the adjoint kernel
  int* out_int = nullptr;    // BlockedResident: [0] workgroups resident at once, [1] CUs
  int64_t nsteps = 1;        // StepLds: steps done inside one launch
  int tile_x = 0, tile_y = 0; // StepBlocked3d: output tile per workgroup (seg_rows: z-planes per workgroup)
  // init
  const void* xi0 = nullptr;
  int in_prec = 8;
  // read-out
  void* out_xi = nullptr;
  void* out_J = nullptr;
  void* out_grad = nullptr;
  int out_prec = 8;
  // diagnostics
  double* partials = nullptr;
  double* diag_out = nullptr;
  int diag_blocks = 0;
  int n_species = 0;
  // batched sweep
  const BatchInst* insts = nullptr;
  const BatchTile* tiles = nullptr;
  uint32_t tile_begin = 0, ntiles = 0;
  char* ws = nullptr;
  int cur = 0;
  // adjoint
  const void* adj_in = nullptr;
  int64_t fill_count = 0;
};

// Temporally blocked D2Q5 sweep (k_step_blocked): workgroup width in columns
// for m evolved species, tb steps per pass and value size `bytes`, or 0 when
// the kernel would not fit.  The sweep runs two waves per SIMD (two
// workgroups per CU), so each lane may hold up to 256 VGPRs: the per-thread
// register window (7m values per time level plus the input rows) and the
// collision's temporaries.  The largest tb that stays within that was read off
// the compiled kernels (single and batched alike): FP32 with x and y periodic
// m <= 3: 6, m = 4: 5 (236 VGPRs on D2Q5); with an x or y wall the face code
// costs registers: m <= 2: 6, m = 3: 5, m = 4: 3 (the walled instantiations
// would spill one step further); FP64 m = 1: 6, m = 2: 3, m >= 3: none.  The
// LDS exchange of the x-directions takes (tb - 1) levels * 2 rows * 2
// directions * m * cols values (<= 64 KiB here).
constexpr int kBlockedCols = 256;
constexpr int kMaxStepsPerPass = 6;
constexpr int blocked_max_tb(int m, int bytes) {
  return bytes == 4 ? (m <= 3 ? 6 : m == 4 ? 5 : 0) : (m == 1 ? 6 : m == 2 ? 3 : 0);
}
// The limit of the walled instantiations.
constexpr int blocked_max_tb_walls(int m, int bytes) {
  return bytes == 4 ? (m <= 2 ? 6 : m == 3 ? 5 : m == 4 ? 3 : 0) : blocked_max_tb(m, bytes);
}
constexpr bool blocked_walls_ok(int m, int tb, int bytes) { return tb <= blocked_max_tb_walls(m, bytes); }
constexpr int blocked_cols(int m, int tb, int bytes) {
  return (tb >= 2 && tb <= kMaxStepsPerPass && tb <= blocked_max_tb(m, bytes) &&
          (tb - 1) * 2 * 2 * m * kBlockedCols * bytes <= 64 * 1024)
             ? kBlockedCols
             : 0;
}

// Wide tiles for wide domains: 512 columns halve the share of the 2 tb halo
// columns per tile.  Measured in FP32: ternary (tb = 6) 8192^2 8 % faster,
// quaternary (tb = 5, periodic in x and y) 8192^2 and 12288^2 10-12 % faster,
// 4096^2 unchanged, 2048^2 and the batch slower; so the host plan takes them
// from kWideMinNx columns on.  LDS exchange per workgroup 80 KiB (m = 2) and
// 96 KiB (m = 3); one workgroup per CU, two waves per SIMD as with 256
// columns.  The quaternary walled instantiation would spill registers, so
// quaternary problems with x or y walls keep 256 columns.
constexpr int kBlockedColsWide = 512;
constexpr int kWideMinNx = 6144;
constexpr bool blocked_wide_ok(int m, int tb, int bytes) {
  return bytes == 4 && ((m <= 2 && tb == 6) || (m == 3 && tb == 5));
}
constexpr bool blocked_wide_walls_ok(int m) { return m <= 2; }

// Temporally blocked adjoint sweep (k_adjoint_blocked): workgroup width for m
// evolved species, tb adjoint steps per pass and value size, or 0 when its
// register window (7m values per level) next to the pulled state, the incoming
// adjoint and the transposed collision (3 x 5m values) would exceed 80 VGPRs.
constexpr int adjoint_blocked_cols(int m, int tb, int bytes) {
  return (tb >= 2 && tb <= 4 && (7 * m * tb + 15 * m) * bytes / 4 <= 80 &&
          tb * 2 * 2 * m * kBlockedCols * bytes <= 64 * 1024)
             ? kBlockedCols
             : 0;
}

// Temporally blocked 3D sweep (k_step_blocked3d, D3Q7 and D3Q6): two steps
// per pass, FP32, up to three evolved species, the full collision.  One
// workgroup fills a CU; its thread count bounds the registers of each lane:
// 1024 threads (128 VGPRs) for m <= 2, 768 (170 VGPRs) for m = 3, whose window
// (prefetched source plane, two collisions, the z ring) does not fit 128
// without spilling (read off the compiled kernels); larger m or FP64 would
// spill at any size.  Default output tile 64 columns by as many rows as the
// thread bound allows (64 x 13 and 64 x 9); LDS: two planes of the four
// in-plane populations of m species per thread.
constexpr int k3dStepsPerPass = 2;
constexpr int k3dTileX = 64;
constexpr bool blocked3d_ok(int lattice, int m, int bytes) {
  return (lattice == 3 || lattice == 6) && bytes == 4 && m >= 1 && m <= 3;
}
constexpr int blocked3d_max_threads(int m) { return m <= 2 ? 1024 : 768; }

// Nodes per thread of the adjoint sweep (see k_adjoint_step).
constexpr int kAdjointNodesPerThread = 4;

// Largest domain (nodes) the single-workgroup LDS-resident sweep accepts for a
// given m, q and value size: two copies of m*q values per node in <= 64 KiB.
inline int64_t lds_resident_max_nodes(int m, int q, int bytes) {
  return (64 * 1024) / (2 * (int64_t)m * q * bytes);
}

template <int LAT>
hipError_t dispatch(Op op, const LaunchArgs& a);

extern template hipError_t dispatch<1>(Op, const LaunchArgs&);
extern template hipError_t dispatch<2>(Op, const LaunchArgs&);
extern template hipError_t dispatch<3>(Op, const LaunchArgs&);
extern template hipError_t dispatch<4>(Op, const LaunchArgs&);
extern template hipError_t dispatch<5>(Op, const LaunchArgs&);
extern template hipError_t dispatch<6>(Op, const LaunchArgs&);

}  // namespace msd
