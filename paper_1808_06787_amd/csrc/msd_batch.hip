// C ABI of batches of independent mixtures (include/msd.h, "Batches").
// Host code validates, lays out the caller's workspace, builds the mixture and
// tile tables and launches kernels; the arithmetic runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/msd.h"
#include "msd_host.h"
#include "msd_launch.h"

using namespace msd::host;

namespace {

struct Member {
  msd_problem prob;          // host pointers cleared
  msd::Problem kp;
  int m = 0;
  int64_t nodes = 0, plane = 0;
  size_t consts_off = 0, half_off[2] = {0, 0}, state_bytes = 0;
  int diag_blocks = 0;
  bool initialised = false;
  int cur = 0;               // which half holds the state
  msd_launch single;         // launch of the single-mixture sweep (reference schedule)
};

// Mixtures launched together.  Blocked ranges (tb >= 2, one species count)
// also have a table of blocked tiles; the one-step tiles serve their first step
// and remainders.  Every mixture of a range has the same `cur`.
struct Range {
  int mmax = 0;
  uint32_t begin = 0, count = 0;
  int tb = 0, seg = 0, walls = 0;
  int dilute = 0;            // all members use the dilute-species collision
  uint32_t bbegin = 0, bcount = 0;
  std::vector<int> members;
};

struct BatchLayout {
  size_t desc_off = 0, tiles_off = 0, partials_off = 0, diag_out_off = 0, total = 0;
  int64_t max_tiles = 0;
  std::vector<size_t> consts_off, half_off0, half_off1, state_bytes;
  std::vector<int64_t> plane;
};

int validate_batch(const msd_problem* probs, int32_t count) {
  if (!probs) return fail(MSD_EINVAL, "problems is NULL");
  if (count < 1) return fail(MSD_EINVAL, "count = %d", count);
  for (int32_t b = 0; b < count; ++b) {
    const int st = validate(&probs[b]);
    if (st != MSD_OK) return st;
    if (probs[b].lattice != probs[0].lattice || probs[b].precision != probs[0].precision)
      return fail(MSD_EINVAL, "mixture %d: all mixtures of a batch share lattice and precision", b);
  }
  return MSD_OK;
}

BatchLayout batch_layout(const msd_problem* probs, int32_t count) {
  BatchLayout L;
  const int q = lattice_q(probs[0].lattice), s = probs[0].precision;
  size_t off = 0;
  L.desc_off = off;
  off = align_up(off + sizeof(msd::BatchInst) * (size_t)count, 256);
  // one-step tiles of 64 x 1 nodes at most, plus at most as many blocked tiles
  for (int32_t b = 0; b < count; ++b)
    L.max_tiles += 2 * ((probs[b].nx + 63) / 64 * probs[b].ny * probs[b].nz);
  L.tiles_off = off;
  off = align_up(off + sizeof(msd::BatchTile) * (size_t)L.max_tiles, 256);
  L.partials_off = off;
  off = align_up(off + sizeof(double) * kDiagBlocksMax * (3 * MSD_MAX_SPECIES + 1), 256);
  L.diag_out_off = off;
  off = align_up(off + sizeof(double) * (3 * MSD_MAX_SPECIES + 1), 256);
  for (int32_t b = 0; b < count; ++b) {
    const int64_t nodes = probs[b].nx * probs[b].ny * probs[b].nz;
    const int64_t plane = (nodes + 63) / 64 * 64 + probs[b].plane_pad;
    const size_t half = align_up((size_t)(probs[b].n_species - 1) * q * (size_t)plane * s, 256);
    L.plane.push_back(plane);
    L.consts_off.push_back(off);
    off = align_up(off + msd::kConstsBytes, 256);
    L.half_off0.push_back(off);
    off += half;
    L.half_off1.push_back(off);
    off += half;
    L.state_bytes.push_back((size_t)(probs[b].n_species - 1) * q * (size_t)plane * s);
  }
  L.total = off;
  return L;
}

}  // namespace

struct msd_batch {
  int count = 0, lattice = 0, prec = 4, q = 0, d = 0;
  std::vector<Member> mem;
  BatchLayout L;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  std::vector<msd::BatchInst> h_desc;
  std::vector<msd::BatchTile> h_tiles;
  std::vector<Range> ranges;
  msd_schedule sched{};
  int64_t t = 0;
  int lds_per_cu = -1;   // LDS bytes per CU of the device (0: unknown)
  // HIP graph of one span of full passes (see msd_batch_step), captured on a
  // stream of its own; valid for the current schedule and the buffer halves
  // the ranges were on at capture (graph_cur)
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t capture_stream = nullptr;
  int64_t graph_span = 0;
  std::vector<int> graph_cur;
  bool graph_failed = false;
};

namespace {

msd::LaunchArgs member_args(const msd_batch* b, int idx) {
  const Member& M = b->mem[idx];
  msd::LaunchArgs a;
  a.p = M.kp;
  a.lattice = b->lattice;
  a.m = M.m;
  a.prec = b->prec;
  a.stream = b->stream;
  a.consts = b->ws + M.consts_off;
  a.n_species = M.m + 1;
  a.block_x = M.single.block_x;
  a.block_y = M.single.block_y;
  a.xcd_remap = M.single.xcd_remap;
  a.nontemporal = M.single.nontemporal;
  a.vec = M.single.vec;
  return a;
}

// Steps per pass for a class of `m` evolved species under schedule `sc`: the
// largest count up to sc.temporal whose on-chip window fits (the walled window
// if any member has an x or y wall: the class then launches the walled
// instantiation), 0 for one step.
int class_steps_per_pass(const msd_batch* b, const std::vector<int>& g, int m) {
  if (b->lattice != MSD_D2Q5 || b->sched.temporal < 2) return 0;
  bool walls = false;
  for (int i : g) {
    if ((uint64_t)b->mem[i].plane * (uint64_t)b->prec >= (1ull << 32)) return 0;
    const msd_problem& p = b->mem[i].prob;
    if (p.bc[0] != MSD_BC_PERIODIC || p.bc[2] != MSD_BC_PERIODIC) walls = true;
  }
  for (int t = b->sched.temporal; t >= 2; --t)
    if (msd::blocked_cols(m, t, b->prec) > 0 && (!walls || msd::blocked_walls_ok(m, t, b->prec))) return t;
  return 0;
}

void push_tiles(std::vector<msd::BatchTile>& out, const std::vector<int>& g, const std::vector<uint32_t>& nt,
                int order) {
  uint32_t most = 0;
  for (uint32_t n : nt) most = std::max(most, n);
  if (order == MSD_ORDER_INTERLEAVED) {
    for (uint32_t k = 0; k < most; ++k)
      for (size_t j = 0; j < g.size(); ++j)
        if (k < nt[j]) out.push_back({(uint32_t)g[j], k});
  } else {
    for (size_t j = 0; j < g.size(); ++j)
      for (uint32_t k = 0; k < nt[j]; ++k) out.push_back({(uint32_t)g[j], k});
  }
}

void drop_graph(msd_batch* b) {
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  b->graph_exec = nullptr;
  b->graph_span = 0;
  b->graph_cur.clear();
}

int build_tiles(msd_batch* b) {
  drop_graph(b);
  const msd_schedule& sc = b->sched;
  // launches over several mixtures need them on the same buffer half
  for (Member& M : b->mem) {
    if (M.cur == 0) continue;
    const hipError_t e = hipMemcpyAsync(b->ws + M.half_off[0], b->ws + M.half_off[1], M.state_bytes,
                                        hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch state move");
    M.cur = 0;
  }
  std::vector<int> idx(b->count);
  for (int i = 0; i < b->count; ++i) idx[i] = i;
  // Mixtures with the full and with the dilute-species collision run in
  // separate launches (different kernel instantiations).
  std::vector<std::vector<int>> groups;
  std::vector<int> group_dilute;
  const bool by_class = sc.mode == MSD_BATCH_PER_CLASS || (b->lattice == MSD_D2Q5 && sc.temporal >= 2);
  for (int dil = 0; dil <= 1; ++dil) {
    if (by_class) {
      for (int m = 1; m < MSD_MAX_SPECIES; ++m) {
        std::vector<int> g;
        for (int i : idx)
          if (b->mem[i].m == m && (b->mem[i].prob.dilute != 0) == (dil != 0)) g.push_back(i);
        if (!g.empty()) {
          groups.push_back(g);
          group_dilute.push_back(dil);
        }
      }
    } else {
      std::vector<int> g;
      for (int i : idx)
        if ((b->mem[i].prob.dilute != 0) == (dil != 0)) g.push_back(i);
      if (!g.empty()) {
        groups.push_back(g);
        group_dilute.push_back(dil);
      }
    }
  }
  b->h_tiles.clear();
  b->ranges.clear();
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const std::vector<int>& g = groups[gi];
    Range r;
    r.members = g;
    r.dilute = group_dilute[gi];
    r.begin = (uint32_t)b->h_tiles.size();
    std::vector<uint32_t> nt(g.size());
    for (size_t j = 0; j < g.size(); ++j) {
      const msd_problem& p = b->mem[g[j]].prob;
      const uint32_t tx = (uint32_t)((p.nx + sc.block_x - 1) / sc.block_x);
      const uint32_t ty = (uint32_t)((p.ny + sc.block_y - 1) / sc.block_y);
      nt[j] = tx * ty * (uint32_t)p.nz;
      r.mmax = std::max(r.mmax, b->mem[g[j]].m);
    }
    push_tiles(b->h_tiles, g, nt, sc.order);
    r.count = (uint32_t)b->h_tiles.size() - r.begin;
    if (by_class) r.tb = class_steps_per_pass(b, g, r.mmax);
    if (r.tb >= 2) {
      r.seg = sc.seg_rows > 0 ? sc.seg_rows : 16;
      const int64_t W = msd::kBlockedCols - 2 * r.tb;
      r.bbegin = (uint32_t)b->h_tiles.size();
      for (size_t j = 0; j < g.size(); ++j) {
        const msd_problem& p = b->mem[g[j]].prob;
        nt[j] = (uint32_t)(((p.nx + W - 1) / W) * ((p.ny + r.seg - 1) / r.seg));
        if (p.bc[0] != MSD_BC_PERIODIC || p.bc[2] != MSD_BC_PERIODIC) r.walls = 1;
      }
      push_tiles(b->h_tiles, g, nt, sc.order);
      r.bcount = (uint32_t)b->h_tiles.size() - r.bbegin;
    }
    b->ranges.push_back(r);
  }
  if ((int64_t)b->h_tiles.size() > b->L.max_tiles) return fail(MSD_EINVAL, "tile table overflow");
  // the host copy must stay untouched until the upload has been consumed
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "batch tile table synchronise");
  e = hipMemcpyAsync(b->ws + b->L.tiles_off, b->h_tiles.data(), sizeof(msd::BatchTile) * b->h_tiles.size(),
                     hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return hip_fail(e, "batch tile table upload");
  e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "batch tile table synchronise");
  return MSD_OK;
}

int check_index(const msd_batch* b, int32_t index) {
  if (!b) return fail(MSD_EINVAL, "batch is NULL");
  if (index < 0 || index >= b->count) return fail(MSD_EINVAL, "index %d outside [0, %d)", index, b->count);
  return MSD_OK;
}

}  // namespace

extern "C" {

size_t msd_batch_workspace_bytes(const msd_problem* problems, int32_t count, int32_t* status) {
  const int st = validate_batch(problems, count);
  if (status) *status = st;
  if (st != MSD_OK) return 0;
  return batch_layout(problems, count).total;
}

int msd_batch_create(const msd_problem* problems, int32_t count, void* d_ws, size_t ws_bytes, void* stream,
                     msd_batch** out) {
  if (!out) return fail(MSD_EINVAL, "out is NULL");
  *out = nullptr;
  const int st = validate_batch(problems, count);
  if (st != MSD_OK) return st;
  if (!d_ws) return fail(MSD_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(MSD_EINVAL, "workspace must be 256-byte aligned");
  const BatchLayout L = batch_layout(problems, count);
  if (ws_bytes < L.total) return fail(MSD_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  msd_batch* b = new (std::nothrow) msd_batch();
  if (!b) return fail(MSD_EINVAL, "host allocation failed");
  b->count = count;
  b->lattice = problems[0].lattice;
  b->prec = problems[0].precision;
  b->q = lattice_q(b->lattice);
  b->d = lattice_d(b->lattice);
  b->L = L;
  b->ws = static_cast<char*>(d_ws);
  b->stream = static_cast<hipStream_t>(stream);
  b->mem.resize(count);
  b->h_desc.resize(count);
  for (int32_t i = 0; i < count; ++i) {
    Member& M = b->mem[i];
    M.prob = problems[i];
    M.prob.D = nullptr;
    M.prob.xi_wall = nullptr;
    M.prob.xi_ref = nullptr;
    M.m = problems[i].n_species - 1;
    M.nodes = problems[i].nx * problems[i].ny * problems[i].nz;
    M.plane = L.plane[i];
    M.consts_off = L.consts_off[i];
    M.half_off[0] = L.half_off0[i];
    M.half_off[1] = L.half_off1[i];
    M.state_bytes = L.state_bytes[i];
    M.diag_blocks = (int)std::min<int64_t>(kDiagBlocksMax, (M.nodes + 255) / 256);
    fill_kernel_problem(&problems[i], M.plane, &M.kp);
    default_launch(&problems[i], &M.single);
    M.single.lds_resident = 0;
    msd::BatchInst& D = b->h_desc[i];
    std::memset(&D, 0, sizeof(D));
    D.p = M.kp;
    D.m = M.m;
    D.half_off[0] = M.half_off[0];
    D.half_off[1] = M.half_off[1];
    D.consts_off = M.consts_off;
  }
  hipError_t e = hipMemcpyAsync(b->ws + L.desc_off, b->h_desc.data(), sizeof(msd::BatchInst) * count,
                                hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "batch table upload");
  }
  b->sched.block_x = 64;
  b->sched.block_y = 4;
  b->sched.mode = MSD_BATCH_FUSED;
  b->sched.order = MSD_ORDER_INSTANCE;
  b->sched.xcd_remap = 0;
  b->sched.nontemporal = 0;
  b->sched.temporal = b->lattice == MSD_D2Q5 ? msd::kMaxStepsPerPass : 0;
  b->sched.seg_rows = 0;
  b->sched.graph = 1;
  const int s2 = build_tiles(b);
  if (s2 != MSD_OK) {
    delete b;
    return s2;
  }
  *out = b;
  return MSD_OK;
}

int msd_batch_set_schedule(msd_batch* b, const msd_schedule* sc) {
  if (!b || !sc) return fail(MSD_EINVAL, "NULL argument");
  if (sc->block_x < 64 || sc->block_x % 64 || sc->block_y < 1 || sc->block_x * sc->block_y > 256)
    return fail(MSD_EINVAL, "block %d x %d", sc->block_x, sc->block_y);
  if (sc->mode != MSD_BATCH_FUSED && sc->mode != MSD_BATCH_PER_CLASS) return fail(MSD_EINVAL, "mode %d", sc->mode);
  if (sc->order != MSD_ORDER_INSTANCE && sc->order != MSD_ORDER_INTERLEAVED)
    return fail(MSD_EINVAL, "order %d", sc->order);
  if (sc->nontemporal < 0 || sc->nontemporal > 7) return fail(MSD_EINVAL, "nontemporal %d", sc->nontemporal);
  if (sc->temporal < 0 || sc->temporal > msd::kMaxStepsPerPass)
    return fail(MSD_EINVAL, "temporal = %d must be 0..%d", sc->temporal, msd::kMaxStepsPerPass);
  if (sc->seg_rows < 0 || sc->seg_rows > (1 << 20)) return fail(MSD_EINVAL, "seg_rows = %d", sc->seg_rows);
  if (sc->graph != 0 && sc->graph != 1) return fail(MSD_EINVAL, "graph = %d must be 0 or 1", sc->graph);
  b->sched = *sc;
  return build_tiles(b);
}

int msd_batch_get_schedule(const msd_batch* b, msd_schedule* sc) {
  if (!b || !sc) return fail(MSD_EINVAL, "NULL argument");
  *sc = b->sched;
  return MSD_OK;
}

int64_t msd_batch_tiles(const msd_batch* b) { return b ? (int64_t)b->h_tiles.size() : -1; }

int64_t msd_batch_time(const msd_batch* b) { return b ? b->t : -1; }

int msd_batch_init(msd_batch* b, int32_t index, const void* d_xi0, int32_t xi0_precision) {
  const int st = check_index(b, index);
  if (st != MSD_OK) return st;
  if (!d_xi0) return fail(MSD_EINVAL, "xi0 is NULL");
  if (xi0_precision != MSD_F32 && xi0_precision != MSD_F64) return fail(MSD_EINVAL, "xi0_precision %d", xi0_precision);
  if (b->t != 0) return fail(MSD_ESTATE, "batch mixtures are initialised at time 0 only");
  b->mem[index].cur = 0;
  msd::LaunchArgs a = member_args(b, index);
  a.consts_out = b->ws + b->mem[index].consts_off;
  hipError_t e = dispatch(msd::Op::Constants, a);
  if (e != hipSuccess) return hip_fail(e, "constants kernel");
  a.xi0 = d_xi0;
  a.in_prec = xi0_precision;
  a.dst = b->ws + b->mem[index].half_off[0];
  e = dispatch(msd::Op::Init, a);
  if (e != hipSuccess) return hip_fail(e, "init kernel");
  b->mem[index].initialised = true;
  return MSD_OK;
}

static int all_initialised(const msd_batch* b) {
  for (int i = 0; i < b->count; ++i)
    if (!b->mem[i].initialised) return fail(MSD_ESTATE, "mixture %d not initialised", i);
  return MSD_OK;
}

}  // extern "C"

namespace {

// Launches of nsteps steps of every range on b->stream; advances the ranges'
// buffer halves and the batch time.
int step_direct(msd_batch* b, int64_t nsteps) {
  msd::LaunchArgs a;
  a.lattice = b->lattice;
  a.prec = b->prec;
  a.stream = b->stream;
  a.insts = reinterpret_cast<const msd::BatchInst*>(b->ws + b->L.desc_off);
  a.tiles = reinterpret_cast<const msd::BatchTile*>(b->ws + b->L.tiles_off);
  a.ws = b->ws;
  a.block_x = b->sched.block_x;
  a.block_y = b->sched.block_y;
  a.xcd_remap = b->sched.xcd_remap;
  a.nontemporal = b->sched.nontemporal;
  if (b->lds_per_cu < 0) {
    int dev = 0, v = 0;
    b->lds_per_cu = (hipGetDevice(&dev) == hipSuccess &&
                     hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess)
                        ? v
                        : 0;
  }
  // at most two workgroups of the blocked sweep per CU, as for one mixture
  a.blocked_lds_floor = b->lds_per_cu > 0 ? b->lds_per_cu / 3 + 1 : 0;
  // each range runs its own sequence of launches (the mixtures are independent)
  for (const Range& r : b->ranges) {
    int cur = b->mem[r.members[0]].cur;
    a.m = r.mmax;
    a.dilute = r.dilute;
    int64_t n = 0;
    while (n < nsteps) {
      const int64_t t = b->t + n;
      a.cur = cur;
      int64_t done = 1;
      hipError_t e;
      const int64_t rest = nsteps - n;
      if (r.tb >= 2 && t > 0 && rest >= 2) {
        // full passes of tb steps, then one shorter pass for a remainder of at
        // least two steps (so that a call runs the same passes whether or not
        // its whole spans come from a graph).  A shorter pass reuses the tile
        // table of tb-step passes: its tiles are at least as wide, so the table
        // covers the mixture, and entries past its last segment store nothing.
        const int len = (int)std::min<int64_t>(r.tb, rest);
        a.tb = len;
        a.seg_rows = r.seg;
        a.walls = r.walls;
        a.tile_begin = r.bbegin;
        a.ntiles = r.bcount;
        e = dispatch(msd::Op::BatchStepBlocked, a);
        done = len;
      } else {
        a.pull = t > 0 ? 1 : 0;
        a.tile_begin = r.begin;
        a.ntiles = r.count;
        e = dispatch(msd::Op::BatchStep, a);
      }
      if (e != hipSuccess) return hip_fail(e, "batched step kernel");
      cur = 1 - cur;
      n += done;
    }
    for (int i : r.members) b->mem[i].cur = cur;
  }
  b->t += nsteps;
  return MSD_OK;
}

int64_t gcd64(int64_t x, int64_t y) { return y == 0 ? x : gcd64(y, x % y); }

// Steps of one graph span: twice the least common multiple of the ranges'
// steps per pass, so that every range runs whole passes and an even number of
// them (and ends on the buffer half it started from).
int64_t graph_span(const msd_batch* b) {
  int64_t l = 1;
  for (const Range& r : b->ranges) {
    const int64_t tb = r.tb >= 2 ? r.tb : 1;
    l = l / gcd64(l, tb) * tb;
  }
  return 2 * l;
}

std::vector<int> range_halves(const msd_batch* b) {
  std::vector<int> c;
  for (const Range& r : b->ranges) c.push_back(b->mem[r.members[0]].cur);
  return c;
}

// Capture one span of launches (nothing runs) and instantiate it.
int capture_graph(msd_batch* b, int64_t span) {
  drop_graph(b);
  hipError_t e = hipSuccess;
  if (!b->capture_stream) {
    e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      b->capture_stream = nullptr;
      return hip_fail(e, "batch capture stream");
    }
  }
  const std::vector<int> halves = range_halves(b);
  const int64_t t0 = b->t;
  hipStream_t keep = b->stream;
  e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "batch graph capture");
  b->stream = b->capture_stream;
  const int st = step_direct(b, span);
  b->stream = keep;
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
  // the capture recorded launches only: put time and halves back
  b->t = t0;
  for (size_t k = 0; k < b->ranges.size(); ++k)
    for (int i : b->ranges[k].members) b->mem[i].cur = halves[k];
  if (st != MSD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e2 != hipSuccess) return hip_fail(e2, "batch graph capture");
  e = hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->graph_exec = nullptr;
    return hip_fail(e, "batch graph instantiate");
  }
  b->graph_span = span;
  b->graph_cur = halves;
  return MSD_OK;
}

}  // namespace

extern "C" {

int msd_batch_step(msd_batch* b, int64_t nsteps) {
  if (!b) return fail(MSD_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(MSD_EINVAL, "nsteps < 0");
  int st = all_initialised(b);
  if (st != MSD_OK) return st;
  int64_t n = 0;
  if (b->sched.graph && !b->graph_failed && nsteps > 0) {
    // the step from time 0 reads pre-collision values: always direct
    if (b->t == 0) {
      st = step_direct(b, 1);
      if (st != MSD_OK) return st;
      n = 1;
    }
    const int64_t span = graph_span(b);
    const int64_t reps = (nsteps - n) / span;
    if (reps >= 1) {
      if (!b->graph_exec || b->graph_span != span || b->graph_cur != range_halves(b)) {
        st = capture_graph(b, span);
        if (st != MSD_OK) {
          // no graph on this device or stream setup: launch directly from now on
          b->graph_failed = true;
          drop_graph(b);
        }
      }
      if (b->graph_exec) {
        for (int64_t r = 0; r < reps; ++r) {
          const hipError_t e = hipGraphLaunch(b->graph_exec, b->stream);
          if (e != hipSuccess) return hip_fail(e, "batch graph launch");
        }
        b->t += reps * span;
        n += reps * span;
      }
    }
  }
  return step_direct(b, nsteps - n);
}

int msd_batch_step_separate(msd_batch* b, int64_t nsteps) {
  if (!b) return fail(MSD_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(MSD_EINVAL, "nsteps < 0");
  const int st0 = all_initialised(b);
  if (st0 != MSD_OK) return st0;
  for (int i = 0; i < b->count; ++i) {
    Member& M = b->mem[i];
    // a single-mixture handle over this mixture's part of the batch workspace,
    // with the default launch of a new handle
    msd_sim s;
    s.prob = M.prob;
    s.kp = M.kp;
    s.L.nodes = M.nodes;
    s.L.plane = M.plane;
    s.L.consts_off = M.consts_off;
    s.L.half_off[0] = M.half_off[0];
    s.L.half_off[1] = M.half_off[1];
    s.L.half_bytes = M.state_bytes;
    s.m = M.m;
    s.q = b->q;
    s.d = b->d;
    s.ws = b->ws;
    s.stream = b->stream;
    s.cur = M.cur;
    s.t = b->t;
    s.initialised = true;
    default_launch(&M.prob, &s.launch);
    const int st = msd_step(&s, nsteps);
    if (st != MSD_OK) return st;
    M.cur = s.cur;
  }
  b->t += nsteps;
  return MSD_OK;
}

int msd_batch_step_each(msd_batch* b, int64_t nsteps) {
  if (!b) return fail(MSD_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(MSD_EINVAL, "nsteps < 0");
  const int st = all_initialised(b);
  if (st != MSD_OK) return st;
  for (int64_t n = 0; n < nsteps; ++n) {
    for (int i = 0; i < b->count; ++i) {
      Member& M = b->mem[i];
      msd::LaunchArgs a = member_args(b, i);
      a.src = b->ws + M.half_off[M.cur];
      a.dst = b->ws + M.half_off[1 - M.cur];
      a.pull = b->t > 0 ? 1 : 0;
      const hipError_t e = dispatch(msd::Op::Step, a);
      if (e != hipSuccess) return hip_fail(e, "step kernel");
      M.cur = 1 - M.cur;
    }
    b->t += 1;
  }
  return MSD_OK;
}

int msd_batch_read_moments(msd_batch* b, int32_t index, int32_t out_precision, void* d_xi, void* d_J, void* d_grad) {
  const int st = check_index(b, index);
  if (st != MSD_OK) return st;
  if (!d_xi) return fail(MSD_EINVAL, "xi is NULL");
  if (!b->mem[index].initialised) return fail(MSD_ESTATE, "mixture %d not initialised", index);
  if (out_precision != MSD_F32 && out_precision != MSD_F64) return fail(MSD_EINVAL, "out_precision %d", out_precision);
  msd::LaunchArgs a = member_args(b, index);
  a.src = b->ws + b->mem[index].half_off[b->mem[index].cur];
  a.pull = b->t > 0 ? 1 : 0;
  a.out_prec = out_precision;
  a.out_xi = d_xi;
  a.out_J = d_J;
  a.out_grad = d_grad;
  const hipError_t e = dispatch(msd::Op::Read, a);
  if (e != hipSuccess) return hip_fail(e, "read kernel");
  return MSD_OK;
}

int msd_batch_diagnostics(msd_batch* b, int32_t index, double* h_mass, double* h_min, double* h_max,
                          int64_t* h_nonfinite) {
  const int st = check_index(b, index);
  if (st != MSD_OK) return st;
  if (!b->mem[index].initialised) return fail(MSD_ESTATE, "mixture %d not initialised", index);
  msd::LaunchArgs a = member_args(b, index);
  a.src = b->ws + b->mem[index].half_off[b->mem[index].cur];
  a.pull = b->t > 0 ? 1 : 0;
  a.partials = reinterpret_cast<double*>(b->ws + b->L.partials_off);
  a.diag_out = reinterpret_cast<double*>(b->ws + b->L.diag_out_off);
  a.diag_blocks = b->mem[index].diag_blocks;
  hipError_t e = dispatch(msd::Op::DiagPartial, a);
  if (e != hipSuccess) return hip_fail(e, "diagnostics kernel");
  e = dispatch(msd::Op::DiagFinal, a);
  if (e != hipSuccess) return hip_fail(e, "diagnostics reduction kernel");
  const int N = b->mem[index].m + 1;
  double host[3 * MSD_MAX_SPECIES + 1];
  e = hipMemcpyAsync(host, a.diag_out, sizeof(double) * (3 * N + 1), hipMemcpyDeviceToHost, b->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics copy");
  e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics synchronise");
  for (int i = 0; i < N; ++i) {
    if (h_mass) h_mass[i] = host[i];
    if (h_min) h_min[i] = host[N + i];
    if (h_max) h_max[i] = host[2 * N + i];
  }
  const int64_t bad = (int64_t)host[3 * N];
  if (h_nonfinite) *h_nonfinite = bad;
  if (bad) return fail(MSD_EDIVERGED, "%lld non-finite mole fractions", (long long)bad);
  return MSD_OK;
}

size_t msd_batch_state_bytes(const msd_batch* b) {
  if (!b) return 0;
  size_t s = 0;
  for (const Member& M : b->mem) s += M.state_bytes;
  return s;
}

int msd_batch_save(const msd_batch* b, void* d_dst, int64_t* h_step) {
  if (!b || !d_dst) return fail(MSD_EINVAL, "NULL argument");
  char* dst = static_cast<char*>(d_dst);
  for (const Member& M : b->mem) {
    const hipError_t e =
        hipMemcpyAsync(dst, b->ws + M.half_off[M.cur], M.state_bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch save copy");
    dst += M.state_bytes;
  }
  if (h_step) *h_step = b->t;
  return MSD_OK;
}

int msd_batch_restore(msd_batch* b, const void* d_src, int64_t step) {
  if (!b || !d_src) return fail(MSD_EINVAL, "NULL argument");
  if (step < 0) return fail(MSD_EINVAL, "step < 0");
  const int st = all_initialised(b);
  if (st != MSD_OK) return st;
  const char* src = static_cast<const char*>(d_src);
  for (const Member& M : b->mem) {
    const hipError_t e =
        hipMemcpyAsync(b->ws + M.half_off[M.cur], src, M.state_bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch restore copy");
    src += M.state_bytes;
  }
  b->t = step;
  return MSD_OK;
}

int msd_batch_tune(msd_batch* b, const msd_schedule* candidates, int32_t count, int32_t steps, double budget_ms,
                   const char* cache_path, int32_t flags, void* d_scratch, size_t scratch_bytes, msd_schedule* h_best,
                   double* h_ms_per_step, double* h_trial_ms) {
  if (!b) return fail(MSD_EINVAL, "batch is NULL");
  if (steps < 1) return fail(MSD_EINVAL, "steps = %d", steps);
  if (count < 0 || (count > 0 && !candidates)) return fail(MSD_EINVAL, "count = %d", count);
  int st = all_initialised(b);
  if (st != MSD_OK) return st;
  // key: architecture, lattice, precision, mixture count and a hash of the
  // sorted (N, extents, faces) of the mixtures
  std::vector<std::array<int64_t, 10>> sig;
  for (const Member& M : b->mem)
    sig.push_back({M.m + 1, M.prob.nx, M.prob.ny, M.prob.nz, M.prob.bc[0], M.prob.bc[1], M.prob.bc[2], M.prob.bc[3],
                   M.prob.bc[4], M.prob.bc[5]});
  std::sort(sig.begin(), sig.end());
  const uint64_t h = fnv1a(sig.data(), sig.size() * sizeof(sig[0]));
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s|batch|%d|%d|%d|%016llx", device_arch().c_str(), b->lattice, b->prec, b->count,
                (unsigned long long)h);
  const std::string key = buf;
  constexpr int K = 9;
  auto pack = [](const msd_schedule& c, int64_t* v) {
    v[0] = c.block_x; v[1] = c.block_y; v[2] = c.mode; v[3] = c.order;
    v[4] = c.xcd_remap; v[5] = c.nontemporal; v[6] = c.temporal; v[7] = c.seg_rows; v[8] = c.graph;
  };
  auto unpack = [](const int64_t* v) {
    msd_schedule c;
    c.block_x = (int32_t)v[0]; c.block_y = (int32_t)v[1]; c.mode = (int32_t)v[2]; c.order = (int32_t)v[3];
    c.xcd_remap = (int32_t)v[4]; c.nontemporal = (int32_t)v[5]; c.temporal = (int32_t)v[6]; c.seg_rows = (int32_t)v[7];
    c.graph = (int32_t)v[8];
    return c;
  };
  int64_t cached[K];
  double cms = 0.0;
  if (!(flags & MSD_TUNE_IGNORE_CACHE) && cache_lookup(cache_path, key, K, cached, &cms)) {
    const msd_schedule c = unpack(cached);
    if (msd_batch_set_schedule(b, &c) == MSD_OK) {
      if (h_best) *h_best = c;
      if (h_ms_per_step) *h_ms_per_step = cms;
      return MSD_OK;
    }
  }
  std::vector<msd_schedule> cand;
  if (count > 0) {
    cand.assign(candidates, candidates + count);
  } else {
    const int blocks[5][2] = {{64, 4}, {128, 2}, {256, 1}, {64, 2}, {64, 1}};
    for (auto& bl : blocks)
      for (int mode : {MSD_BATCH_FUSED, MSD_BATCH_PER_CLASS})
        for (int order : {MSD_ORDER_INSTANCE, MSD_ORDER_INTERLEAVED})
          for (int xcd : {0, 1}) {
            msd_schedule c{};
            c.block_x = bl[0]; c.block_y = bl[1]; c.mode = mode; c.order = order; c.xcd_remap = xcd;
            c.graph = b->sched.graph;
            cand.push_back(c);
          }
    if (b->lattice == MSD_D2Q5)
      for (int tb : {2, 3, 4, 5, 6})
        for (int seg : {8, 12, 16, 24, 32, 48, 64, 128})
          for (int order : {MSD_ORDER_INSTANCE, MSD_ORDER_INTERLEAVED}) {
            msd_schedule c{};
            c.block_x = 64; c.block_y = 4; c.mode = MSD_BATCH_PER_CLASS; c.order = order;
            c.temporal = tb; c.seg_rows = seg; c.graph = b->sched.graph;
            cand.push_back(c);
          }
  }
  const size_t sb = msd_batch_state_bytes(b);
  if (!d_scratch || scratch_bytes < sb) return fail(MSD_ENOMEM, "scratch of %zu bytes, %zu needed", scratch_bytes, sb);
  const msd_schedule keep = b->sched;
  int64_t t0 = 0;
  st = msd_batch_save(b, d_scratch, &t0);
  if (st != MSD_OK) return st;
  std::vector<double> ms(cand.size(), -1.0);
  int best = -1;
  st = time_candidates(
      b->stream, (int)cand.size(), steps, budget_ms, [&](int i) { return msd_batch_set_schedule(b, &cand[i]); },
      [&](int n) { return msd_batch_step(b, n); }, [&]() { return msd_batch_restore(b, d_scratch, t0); }, ms.data(),
      &best);
  if (h_trial_ms)
    for (size_t i = 0; i < cand.size(); ++i) h_trial_ms[i] = ms[i];
  if (st != MSD_OK || best < 0) {
    msd_batch_set_schedule(b, &keep);
    return st != MSD_OK ? st : fail(MSD_EINVAL, "no candidate schedule could run");
  }
  st = msd_batch_set_schedule(b, &cand[best]);
  if (st != MSD_OK) return st;
  int64_t v[K];
  pack(b->sched, v);
  cache_store(cache_path, key, K, v, ms[best]);
  if (h_best) *h_best = b->sched;
  if (h_ms_per_step) *h_ms_per_step = ms[best];
  return MSD_OK;
}

int msd_batch_destroy(msd_batch* b) {
  if (b) {
    (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  }
  delete b;
  return MSD_OK;
}

}  // extern "C"
