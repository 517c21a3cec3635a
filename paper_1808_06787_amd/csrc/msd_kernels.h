// Kernels of the sweep, templated on lattice, number of evolved species and
// precision, plus the per-lattice dispatch.  Included by one translation unit
// per lattice.
//
// Storage: every distribution buffer holds m*q planes of `plane` values
// (plane >= nodes, padded), plane (i, k) at offset (i*q + k)*plane.  A buffer
// holds post-collision values f^+(x, t-1) at the node that produced them
// (pull layout); only right after msd_init does it hold the pre-collision
// f(x, 0), which the first sweep reads without propagation (pull = 0).
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>

#include "msd_launch.h"

namespace msd {

// ---------------------------------------------------------------------------
// Tiling: a 1D grid of tiles of block_x * block_y nodes in one z-plane.  With
// XCD remapping, the hardware's round-robin of workgroups over the 8 XCDs is
// undone so that each XCD walks a contiguous range of tiles (neighbouring
// rows, whose lines the +-y pulls re-read, then sit in the same L2).
// ---------------------------------------------------------------------------
struct Tiling {
  uint32_t tiles_x, tiles_y, tiles;
  uint32_t remap;
};

__device__ __forceinline__ uint32_t logical_tile(const Tiling& t) {
  const uint32_t L = blockIdx.x;
  if (!t.remap) return L;
  const uint32_t q = t.tiles >> 3, r = t.tiles & 7u, x = L & 7u;
  return x * q + (x < r ? x : r) + (L >> 3);
}

template <typename T>
__device__ __forceinline__ void store_value(T* p, T v, int nontemporal) {
  if (nontemporal)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

template <int M, typename T>
struct NodeConsts {
  T R[M][M + 1];
  T wall[6][M];
  T xref[M];
  CollideCoef<M, T> cc;
};

template <int M, typename T>
__device__ __forceinline__ void load_consts(const Consts<T>* __restrict__ c, NodeConsts<M, T>& nc) {
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j <= M; ++j) nc.R[i][j] = c->R[i][j];
#pragma unroll
  for (int f = 0; f < 6; ++f)
#pragma unroll
    for (int i = 0; i < M; ++i) nc.wall[f][i] = c->wall[f][i];
#pragma unroll
  for (int i = 0; i < M; ++i) nc.xref[i] = c->xref[i];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    nc.cc.a0[i] = c->a0[i];
    nc.cc.ds[i] = c->ds[i];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      if (k == i) continue;
      nc.cc.da[i][k] = c->da[i][k];
      nc.cc.ea[i][k] = c->ea[i][k];
      nc.cc.ga[i][k] = c->ga[i][k];
    }
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) nc.cc.rule[j] = c->rule[j];
}

// ---------------------------------------------------------------------------
// Setup: reciprocal diffusivities, face data and the collision coefficients in
// the sweep's precision (computed in FP64, rounded once).  With h = cs2/2
// (a = cs2 dt, dt = 1) and S_ik = R_ik - R_iN, Eq. (2-10) gives
//   A_ii = 1 + h (R_iN + sum_{k != i} xb_k S_ik),  A_ik = -h xb_i S_ik.
// ---------------------------------------------------------------------------
template <int LAT, int M, typename T>
__global__ void k_constants(Problem p, int n_species, Consts<T>* out) {
  const int t = threadIdx.x;
  if (t < kMaxSpecies * kMaxSpecies) {
    const int i = t / kMaxSpecies, j = t % kMaxSpecies;
    out->R[i][j] = (i != j && i < n_species && j < n_species) ? T(1.0 / p.D[i][j]) : T(0);
    double da = 0.0, ea = 0.0, ga = 0.0;
    if (i < M && j < M && i != j) {
      const double h = 0.5 * Lattice<LAT>::cs2;
      const double S = 1.0 / p.D[i][j] - 1.0 / p.D[i][M];
      if (p.linearized) {
        ga = p.dilute ? 0.0 : -h * p.xi_ref[i] * S;
      } else {
        da = h * S;
        ea = p.dilute ? 0.0 : -h * S;
      }
    }
    out->da[i][j] = T(da);
    out->ea[i][j] = T(ea);
    out->ga[i][j] = T(ga);
  }
  if (t < 6 * kMaxSpecies) out->wall[t / kMaxSpecies][t % kMaxSpecies] = T(p.wall[t / kMaxSpecies][t % kMaxSpecies]);
  if (t < kMaxSpecies) {
    out->xref[t] = T(p.xi_ref[t]);
    double a0 = 1.0, ds = 0.0;
    if (t < M) {
      const double h = 0.5 * Lattice<LAT>::cs2;
      const double rN = 1.0 / p.D[t][M];
      double d = rN;
      if (p.linearized) {
        for (int k = 0; k < M; ++k)
          if (k != t) d += p.xi_ref[k] * (1.0 / p.D[t][k] - rN);
        if (p.dilute) d -= p.xi_ref[t] * rN;   // xi_N R_iN carries -xi_i R_iN
      } else if (p.dilute) {
        ds = -h * rN;
      }
      a0 = 1.0 + h * d;
    }
    out->a0[t] = T(a0);
    out->ds[t] = T(ds);
  }
  if (t == 0) {
    // Eq. (3-16) is the product rule with 3/16; SRT has no even correction
    const bool srt = p.relax == 1;
    const double sg = srt ? 0.0 : 1.0;
    const double magic = p.relax == 2 ? p.magic : 3.0 / 16.0;
    out->rule[0] = T(sg);
    out->rule[1] = T(0.5 * sg);
    out->rule[2] = T(-sg);
    out->rule[3] = T(1.0 - 0.5 * sg);
    out->rule[4] = T(sg - 2.0);
    out->rule[5] = T(srt ? 0.0 : 1.0 - 4.0 * magic);
    out->rule[6] = T(srt ? 1.0 : 8.0 * magic);
  }
}

// ---------------------------------------------------------------------------
// Initialisation f_k^i(x, 0) = w_k xi_i(x, 0) (Sec. 4, Eq. (3-3)).
// ---------------------------------------------------------------------------
template <int LAT, int M, typename T, typename TI>
__global__ __launch_bounds__(256) void k_init(Problem p, const TI* __restrict__ xi0, T* __restrict__ dst) {
  using L = Lattice<LAT>;
  const int64_t nodes = (int64_t)p.nx * p.ny * p.nz;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nodes) return;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const T xi = T(xi0[(int64_t)i * nodes + idx]);
#pragma unroll
    for (int k = 0; k < L::Q; ++k) dst[(int64_t)(i * L::Q + k) * p.plane + idx] = T(L::w(k)) * xi;
  }
}

__device__ __forceinline__ bool tile_node(const Problem& p, const Tiling& tl, NodePos& n) {
  const uint32_t tile = logical_tile(tl);
  const uint32_t tx = tile % tl.tiles_x;
  const uint32_t rest = tile / tl.tiles_x;
  const uint32_t ty = rest % tl.tiles_y;
  const uint32_t tz = rest / tl.tiles_y;
  n.c[0] = (int32_t)(tx * blockDim.x + threadIdx.x);
  n.c[1] = (int32_t)(ty * blockDim.y + threadIdx.y);
  n.c[2] = (int32_t)tz;
  if (n.c[0] >= p.nx || n.c[1] >= p.ny) return false;
  n.idx = n.c[0] + (int64_t)p.nx * (n.c[1] + (int64_t)p.ny * n.c[2]);
  return true;
}

// ---------------------------------------------------------------------------
// One fused time step: pull-propagate (with face rules), collide, store.
// ---------------------------------------------------------------------------
// DIL: the dilute-species collision (a separate instantiation, chosen at launch).
template <int LAT, int M, typename T, bool DIL = false>
__global__ __launch_bounds__(256) void k_step(Problem p, const T* __restrict__ src, T* __restrict__ dst,
                                               const Consts<T>* __restrict__ cst, int pull, Tiling tl,
                                               int nontemporal) {
  constexpr int Q = Lattice<LAT>::Q;
  NodePos n;
  if (!tile_node(p, tl, n)) return;
  NodeConsts<M, T> nc;
  load_consts<M, T>(cst, nc);
  T f[M][Q];
  gather_node<LAT, M, T>(p, src, n, pull != 0, f, nc.wall, nontemporal);
  collide_node<LAT, M, T, DIL>(f, nc.cc);
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int k = 0; k < Q; ++k)
      store_value(dst + (int64_t)(i * Q + k) * p.plane + n.idx, f[i][k], nontemporal & NT_STORE);
}

// ---------------------------------------------------------------------------
// Vectorised sweep: each thread owns V consecutive x-nodes of one row and moves
// them with aligned V-wide loads and stores; plane offsets are 32-bit so that
// every access is (uniform plane base) + (per-lane offset).  The +-x neighbours
// of a thread's segment come from the adjacent lanes by a shuffle; only the
// first / last lane of a wave, and the lanes at a row end, load them.
// Requires block_x % 64 == 0 (a wave is one row segment), nx % V == 0 and
// plane * sizeof(T) < 2^32.
// ---------------------------------------------------------------------------
template <typename T, int V>
struct VecOf {
  typedef T type __attribute__((ext_vector_type(V)));
};

template <typename T, int V>
__device__ __forceinline__ typename VecOf<T, V>::type vload(const T* base, uint32_t idx, bool nt) {
  const auto* p = reinterpret_cast<const typename VecOf<T, V>::type*>(reinterpret_cast<const char*>(base) +
                                                                      idx * (uint32_t)sizeof(T));
  return nt ? __builtin_nontemporal_load(p) : *p;
}

template <typename T>
__device__ __forceinline__ T sload(const T* base, uint32_t idx, bool nt) {
  const T* p = reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(T));
  return nt ? __builtin_nontemporal_load(p) : *p;
}

template <typename T, int V>
__device__ __forceinline__ void vstore(T* base, uint32_t idx, typename VecOf<T, V>::type v, int nontemporal) {
  auto* p = reinterpret_cast<typename VecOf<T, V>::type*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(T));
  if (nontemporal)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

template <int LAT, int M, typename T, int V>
__global__ __launch_bounds__(256) void k_step_vec(Problem p, const T* __restrict__ src, T* __restrict__ dst,
                                                  const Consts<T>* __restrict__ cst, int pull, Tiling tl,
                                                  int nontemporal) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q;
  using VT = typename VecOf<T, V>::type;
  const uint32_t tile = logical_tile(tl);
  const uint32_t tx = tile % tl.tiles_x;
  const uint32_t rest = tile / tl.tiles_x;
  const uint32_t ty = rest % tl.tiles_y;
  const uint32_t tz = rest / tl.tiles_y;
  const int32_t x0 = (int32_t)((tx * blockDim.x + threadIdx.x) * V);
  const int32_t y = (int32_t)(ty * blockDim.y + threadIdx.y);
  const int32_t z = (int32_t)tz;
  if (x0 >= p.nx || y >= p.ny) return;
  const uint32_t nx = (uint32_t)p.nx;
  const uint32_t idx0 = (uint32_t)x0 + nx * ((uint32_t)y + (uint32_t)p.ny * (uint32_t)z);
  const int lane = (int)(threadIdx.x & 63u);
  NodeConsts<M, T> nc;
  load_consts<M, T>(cst, nc);
  const bool nt_al = (nontemporal & NT_LOAD_ALIGNED) != 0;
  const bool nt_sh = (nontemporal & NT_LOAD_SHIFTED) != 0;

  T f[V][M][Q];
  if (!pull) {
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const VT v = vload<T, V>(src + (size_t)(i * Q + k) * p.plane, idx0, nt_al);
#pragma unroll
        for (int j = 0; j < V; ++j) f[j][i][k] = v[j];
      }
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int a = L::axis(k);
      const int s = L::sgn(k);
      const int kb = L::opp(k);
      const int face = 2 * (a < 0 ? 0 : a) + (s > 0 ? 0 : 1);
      if (a < 0) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
          const VT v = vload<T, V>(src + (size_t)(i * Q + k) * p.plane, idx0, nt_al);
#pragma unroll
          for (int j = 0; j < V; ++j) f[j][i][k] = v[j];
        }
      } else if (a > 0) {
        // y or z: the whole segment pulls from one neighbouring row (wave-uniform)
        const uint32_t ext = (uint32_t)(a == 1 ? p.ny : p.nz);
        const uint32_t st = a == 1 ? nx : nx * (uint32_t)p.ny;
        const uint32_t coord = (uint32_t)(a == 1 ? y : z);
        const bool edge = (s > 0) ? (coord == 0) : (coord == ext - 1);
        const int kind = edge ? p.bc[face] : BC_PERIODIC;
        if (kind == BC_PERIODIC) {
          const uint32_t off = edge ? (s > 0 ? idx0 + (ext - 1) * st : idx0 - (ext - 1) * st)
                                    : (s > 0 ? idx0 - st : idx0 + st);
#pragma unroll
          for (int i = 0; i < M; ++i) {
            const VT v = vload<T, V>(src + (size_t)(i * Q + k) * p.plane, off, nt_al);
#pragma unroll
            for (int j = 0; j < V; ++j) f[j][i][k] = v[j];
          }
        } else {
#pragma unroll
          for (int i = 0; i < M; ++i) {
            const VT v = vload<T, V>(src + (size_t)(i * Q + kb) * p.plane, idx0, nt_al);
            const T wb = T(2.0 * L::w(kb)) * nc.wall[face][i];
#pragma unroll
            for (int j = 0; j < V; ++j) f[j][i][k] = (kind == BC_ZERO_FLUX) ? v[j] : wb - v[j];
          }
        }
      } else {
        // x: own aligned vector, one value from the neighbouring lane
#pragma unroll
        for (int i = 0; i < M; ++i) {
          const T* pk = src + (size_t)(i * Q + k) * p.plane;
          const VT v = vload<T, V>(pk, idx0, nt_sh);
          if (s > 0) {
            const T from_lane = __shfl_up(v[V - 1], 1, 64);
            T left;
            if (x0 == 0) {
              const int kind = p.bc[0];
              if (kind == BC_PERIODIC) {
                left = sload(pk, idx0 + nx - 1, nt_sh);
              } else {
                const T back = sload(src + (size_t)(i * Q + kb) * p.plane, idx0, nt_sh);
                left = (kind == BC_ZERO_FLUX) ? back : T(2.0 * L::w(kb)) * nc.wall[0][i] - back;
              }
            } else if (lane == 0) {
              left = sload(pk, idx0 - 1, nt_sh);
            } else {
              left = from_lane;
            }
            f[0][i][k] = left;
#pragma unroll
            for (int j = 1; j < V; ++j) f[j][i][k] = v[j - 1];
          } else {
            const T from_lane = __shfl_down(v[0], 1, 64);
            T right;
            if ((uint32_t)x0 + V == nx) {
              const int kind = p.bc[1];
              if (kind == BC_PERIODIC) {
                right = sload(pk, idx0 + V - nx, nt_sh);
              } else {
                const T back = sload(src + (size_t)(i * Q + kb) * p.plane, idx0 + V - 1, nt_sh);
                right = (kind == BC_ZERO_FLUX) ? back : T(2.0 * L::w(kb)) * nc.wall[1][i] - back;
              }
            } else if (lane == 63) {
              right = sload(pk, idx0 + V, nt_sh);
            } else {
              right = from_lane;
            }
#pragma unroll
            for (int j = 0; j + 1 < V; ++j) f[j][i][k] = v[j + 1];
            f[V - 1][i][k] = right;
          }
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < V; ++j) collide_node<LAT, M, T>(f[j], nc.cc);
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      VT o;
#pragma unroll
      for (int j = 0; j < V; ++j) o[j] = f[j][i][k];
      vstore<T, V>(dst + (size_t)(i * Q + k) * p.plane, idx0, o, nontemporal & NT_STORE);
    }
}

// Global-memory access from a uniform base and a 32-bit per-lane byte offset.
// scalar_base hides the base behind an empty asm with an SGPR operand, so the
// compiler keeps it in scalar registers and emits the base + 32-bit-offset
// form instead of re-associating it into 64-bit per-lane address arithmetic.
using gbyte = __attribute__((address_space(1))) char;
__device__ __forceinline__ uint64_t scalar_base(const void* p) {
  uint64_t a = reinterpret_cast<uint64_t>(p);
  asm volatile("" : "+s"(a));
  return a;
}
// A uniform 64-bit value the compiler must re-read where it is used (so that
// products with it are not hoisted and kept live across a loop).
__device__ __forceinline__ uint64_t opaque_u64(uint64_t v) {
  asm volatile("" : "+s"(v));
  return v;
}
template <typename T>
__device__ __forceinline__ T gload(uint64_t base, uint32_t off, bool nt) {
  const auto* q = reinterpret_cast<const __attribute__((address_space(1))) T*>(
      reinterpret_cast<const gbyte*>(base) + off);
  return nt ? __builtin_nontemporal_load(q) : *q;
}
template <typename T>
__device__ __forceinline__ void gstore(uint64_t base, uint32_t off, T v, int nt) {
  auto* q = reinterpret_cast<__attribute__((address_space(1))) T*>(reinterpret_cast<gbyte*>(base) + off);
  if (nt)
    __builtin_nontemporal_store(v, q);
  else
    *q = v;
}

// Range-checked store: a raw buffer over [base, base + bytes) drops a store
// whose offset is outside it (an offset of 0xFFFFFFFF writes nothing).
template <typename T>
__device__ __forceinline__ void bstore(uint64_t base, uint32_t bytes, uint32_t off, T v) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, (int)off, 0, 0);
  } else {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, (int)off, 0, 0);
  }
}

// ---------------------------------------------------------------------------
// Temporally blocked sweep on the axial 2D lattices (D2Q5; D2Q4, which has no
// rest direction, the same way without it): TB time steps per pass over HBM.
//
// Workgroup (tile, segment) owns output columns [x0, x0 + W), W = C - 2 TB, and
// output rows [y0, y1).  Thread c holds column x = x0 - TB + c (a halo of TB
// columns each side; wrapped for periodic x) at every time level.  The
// workgroup marches over the input rows y0 - TB .. y1 - 1 + TB (wrapped for
// periodic y); in iteration j the input row r_in = y0 - TB + j arrives and
// level l produces row r_in - l from rows r - 1, r, r + 1 of level l - 1 (one
// pull-propagation + collision); level TB writes the output row.
//
// Pull propagation takes the y-directions from the same column, so each level
// keeps them in registers: a ring of three rows (rest, +y, -y), the row a
// level produced in iteration j in slot j mod 3.  Only the two x-directions
// cross columns: level 0 (the input) loads its neighbours' values from memory,
// and levels 1 .. TB-1 pass theirs through LDS, two rows per level in slots
// chosen by iteration parity, so one barrier per iteration orders every LDS
// write after the reads of the previous occupant of its slot.  The march is
// unrolled six times (the period of both), which turns every ring slot, LDS
// slot and prefetch buffer into a compile-time choice: no register moves to
// shift windows, no per-row address arithmetic.
//
// The first 2 TB iterations (the prologue, fully unrolled) fill the levels:
// level l has its first row in iteration 2 l, and the output level none.  In
// the main part every level has a row in every iteration; the output level
// stores through range-checked buffer stores (lanes outside the output are
// masked by offset, not by a branch), so every iteration issues the same
// stores and the wait for the next input row does not also wait for them.
// Level l is valid on columns [l, C - l); invalid columns compute values that
// no valid node reads.  Rows beyond a y wall are skipped, and nodes beyond a
// wall are never read: the face rule at a boundary node reads the node
// itself.  Offsets within a plane are 32-bit (the host checks plane bytes <
// 4 GiB).  WALLS = false is the instantiation for a fully periodic domain: no
// face code.
// ---------------------------------------------------------------------------
template <int J>
using Iter = std::integral_constant<int, J>;
// f(Iter<0>{}), f(Iter<1>{}), ... in order
template <typename F, int... Js>
__device__ __forceinline__ void for_each_iter(F&& f, std::integer_sequence<int, Js...>) {
  (f(Iter<Js>{}), ...);
}

template <int M, typename T, int TB, int C, bool WALLS, bool DIL = false, int LAT = 2>
__device__ __forceinline__ void blocked_tile(const Problem& p, const T* __restrict__ src, T* __restrict__ dst,
                                             const Consts<T>* __restrict__ cst, int seg_rows, uint32_t tx,
                                             uint32_t seg, int nontemporal, int64_t rec_stride = 0) {
  using L = Lattice<LAT>;
  static_assert(LAT == 2 || LAT == 5, "the axial 2D lattices D2Q5 and D2Q4");
  constexpr int Q = L::Q, P = M * Q, W = C - 2 * TB;
  // D2Q5 order: 0 rest, 1 +x, 2 +y, 3 -x, 4 -y; D2Q4 (no rest): 0 +x, 1 +y, 2 -x, 3 -y.
  constexpr bool REST = LAT == 2;
  constexpr int KXP = REST ? 1 : 0, KYP = KXP + 1, KXM = KXP + 2, KYM = KXP + 3;
  static_assert(L::axis(KXP) == 0 && L::sgn(KXP) > 0 && L::axis(KXM) == 0 && L::sgn(KXM) < 0, "x directions");
  static_assert(L::axis(KYP) == 1 && L::sgn(KYP) > 0 && L::axis(KYM) == 1 && L::sgn(KYM) < 0, "y directions");
  // x-direction populations of the two most recent rows of levels 1 .. TB-1:
  // [level - 1][slot][+x/-x][species][column].  Level 0 (the input rows)
  // takes its x-neighbours straight from memory instead.
  __shared__ T xs[TB - 1][2][2][M][C];

  const int c = (int)threadIdx.x;
  const int cm = c > 0 ? c - 1 : 0, cp = c < C - 1 ? c + 1 : C - 1;
  const int nx = p.nx, ny = p.ny;
  const int x0 = (int)tx * W;
  const int y0 = (int)seg * seg_rows;
  const int y1 = min(y0 + seg_rows, ny);
  const int x = x0 - TB + c;
  // WALLS = false is only launched on a fully periodic domain
  const bool px = !WALLS || p.bc[0] == BC_PERIODIC, py = !WALLS || p.bc[2] == BC_PERIODIC;
  const bool x_in = x >= 0 && x < nx;
  const bool col_ok = x_in || px;
  const uint32_t xl = (uint32_t)(x_in ? x : (((x % nx) + nx) % nx));
  // neighbour columns (wrapped; at a wall the face rule replaces what they give)
  const uint32_t xlm = xl > 0 ? xl - 1 : (uint32_t)nx - 1, xlp = xl + 1 < (uint32_t)nx ? xl + 1 : 0;
  // a tile that reaches an x wall (uniform): only there do x-pulls need the face rule
  const bool tile_xwall = !px && (x0 - TB <= 0 || x0 - TB + C - 1 >= nx - 1);
  const bool wall_xlo = !px && x == 0, wall_xhi = !px && x == nx - 1;
  const bool out_col = c >= TB && c < C - TB && x_in;
  NodeConsts<M, T> nc;
  load_consts<M, T>(cst, nc);
  const bool nt_ld = (nontemporal & NT_LOAD_ALIGNED) != 0;
  const int nt_st = nontemporal & NT_STORE;

  // ring[level][slot][rest/+y/-y][species] (levels 0 .. TB-1)
  T ring[TB][3][3][M];
  // level 0, by iteration parity: the left neighbour's +x and the right
  // neighbour's -x (what level 1 pulls), and the node's own +x/-x (what the
  // face rule at an x wall reads)
  T nb[2][2][M], own[2][2][M];
  // prefetched input rows, by iteration parity
  T ld[2][P], ldn[2][2][M];
#pragma unroll
  for (int l = 0; l < TB; ++l)
#pragma unroll
    for (int sl = 0; sl < 3; ++sl)
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < M; ++i) ring[l][sl][j][i] = T(0);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int i = 0; i < M; ++i) nb[b][d][i] = own[b][d][i] = ldn[b][d][i] = T(0);

  // Planes are walked from an opaque scalar base (scalar_base) in steps of the
  // plane stride: every access is that scalar base plus the lane's 32-bit
  // offset, and no per-plane base is hoisted out of the row loop (which would
  // hold one SGPR pair per plane and level for the whole kernel).
  const uint64_t pstride = (uint64_t)p.plane * sizeof(T);
  const uint32_t plane_bytes = (uint32_t)pstride;   // < 4 GiB (checked by the host)

  auto load_row = [&](int r, T (&row_v)[P], T (&nb_v)[2][M]) __attribute__((always_inline)) {
    const bool r_in = r >= 0 && r < ny;
    const int rl = r_in ? r : (((r % ny) + ny) % ny);
    // the scalar base is taken outside the (lane-divergent with walls) branch
    uint64_t b = scalar_base(src);
    if (col_ok && (r_in || py)) {
      const uint32_t row = (uint32_t)rl * (uint32_t)nx;
      const uint32_t off = (row + xl) * (uint32_t)sizeof(T);
      const uint32_t offm = (row + xlm) * (uint32_t)sizeof(T), offp = (row + xlp) * (uint32_t)sizeof(T);
#pragma unroll
      for (int pl = 0; pl < P; ++pl, b += pstride) {
        row_v[pl] = gload<T>(b, off, nt_ld);
        // the left neighbour's +x and the right neighbour's -x of the same plane
        if (pl % Q == KXP) nb_v[0][pl / Q] = gload<T>(b, offm, nt_ld);
        if (pl % Q == KXM) nb_v[1][pl / Q] = gload<T>(b, offp, nt_ld);
      }
    } else {
#pragma unroll
      for (int pl = 0; pl < P; ++pl) row_v[pl] = T(0);
#pragma unroll
      for (int i = 0; i < M; ++i) nb_v[0][i] = nb_v[1][i] = T(0);
    }
  };
  // Dirichlet face: 2 w xi_wall minus the node's own opposite population; zero flux: that population.
  auto face = [&](int fk, int kb, int i, T back) {
    return (p.bc[fk] == BC_ZERO_FLUX) ? back : T(2.0 * L::w(kb)) * nc.wall[fk][i] - back;
  };

  const int r_last = y1 - 1 + TB;
  // Iteration j of the march (jc: j itself in the prologue, j mod 6 in the
  // main part, which starts at j = 2 TB).
  auto iteration = [&](int r_in, auto jc, auto main_c) __attribute__((always_inline)) {
    constexpr int JJ = decltype(jc)::value;
    constexpr bool MAIN = decltype(main_c)::value;
    constexpr int J = JJ % 6;
    constexpr int B = J & 1;   // this row's prefetch buffer and level-0 parity slot
    __syncthreads();
#pragma unroll
    for (int i = 0; i < M; ++i) {
      if constexpr (REST) ring[0][J % 3][0][i] = ld[B][i * Q];
      ring[0][J % 3][1][i] = ld[B][i * Q + KYP];
      ring[0][J % 3][2][i] = ld[B][i * Q + KYM];
      own[B][0][i] = ld[B][i * Q + KXP];
      own[B][1][i] = ld[B][i * Q + KXM];
#pragma unroll
      for (int d = 0; d < 2; ++d) nb[B][d][i] = ldn[B][d][i];
    }
    // the next input row (past the last one it is a harmless in-bounds or zero load)
    load_row(r_in + 1, ld[B ^ 1], ldn[B ^ 1]);
#pragma unroll
    for (int lvl = 1; lvl <= TB; ++lvl) {
      // level lvl - 1 produced rows r - 1, r, r + 1 in iterations j - 2, j - 1, j
      if (!MAIN && (lvl == TB || JJ < 2 * lvl)) continue;   // no row yet (compile time)
      const int r = r_in - lvl;
      const int lp = lvl - 1;
      const int sm = (J + 4) % 3, s0 = (J + 2) % 3, sp = J % 3;
      const int sx = (J - lvl) & 1;   // LDS slot of row r at level lp (and of this level's row)
      if (lvl < TB && !py && (r < 0 || r >= ny)) continue;   // beyond a y wall
      T f[M][Q];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        if constexpr (REST) f[i][0] = ring[lp][s0][0][i];
        f[i][KXP] = lp == 0 ? nb[B ^ 1][0][i] : xs[lp > 0 ? lp - 1 : 0][sx][0][i][cm];
        f[i][KXM] = lp == 0 ? nb[B ^ 1][1][i] : xs[lp > 0 ? lp - 1 : 0][sx][1][i][cp];
        f[i][KYP] = ring[lp][sm][1][i];
        f[i][KYM] = ring[lp][sp][2][i];
      }
      if constexpr (WALLS) {
        if (tile_xwall) {
#pragma unroll
          for (int i = 0; i < M; ++i) {
            const T own_xm = lp == 0 ? own[B ^ 1][1][i] : xs[lp > 0 ? lp - 1 : 0][sx][1][i][c];
            const T own_xp = lp == 0 ? own[B ^ 1][0][i] : xs[lp > 0 ? lp - 1 : 0][sx][0][i][c];
            if (wall_xlo) f[i][KXP] = face(0, KXM, i, own_xm);
            if (wall_xhi) f[i][KXM] = face(1, KXP, i, own_xp);
          }
        }
        if (!py && r == 0) {
#pragma unroll
          for (int i = 0; i < M; ++i) f[i][KYP] = face(2, KYM, i, ring[lp][s0][2][i]);
        }
        if (!py && r == ny - 1) {
#pragma unroll
          for (int i = 0; i < M; ++i) f[i][KYM] = face(3, KYP, i, ring[lp][s0][1][i]);
        }
      }
      collide_node<LAT, M, T, DIL>(f, nc.cc);
      if (lvl < TB) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
          xs[lvl < TB ? lvl - 1 : 0][sx][0][i][c] = f[i][KXP];
          xs[lvl < TB ? lvl - 1 : 0][sx][1][i][c] = f[i][KXM];
          if constexpr (REST) ring[lvl < TB ? lvl : 0][sp][0][i] = f[i][0];
          ring[lvl < TB ? lvl : 0][sp][1][i] = f[i][KYP];
          ring[lvl < TB ? lvl : 0][sp][2][i] = f[i][KYM];
        }
      }
      // The output level (main part only) stores the pass's output; recording
      // (rec_stride > 0, uniform) also stores every intermediate level, level
      // l at dst + (l - 1) rec_stride.
      if (lvl == TB) {
        const uint32_t off = out_col ? ((uint32_t)r * (uint32_t)nx + (uint32_t)x) * (uint32_t)sizeof(T) : 0xFFFFFFFFu;
        uint64_t b = scalar_base(dst);
        if (rec_stride > 0) b += (uint64_t)(TB - 1) * (uint64_t)rec_stride * sizeof(T);
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
          for (int k = 0; k < Q; ++k, b += pstride) bstore<T>(b, plane_bytes, off, f[i][k]);
      } else if (rec_stride > 0 && out_col && r >= y0 && r < y1) {
        const uint32_t off = ((uint32_t)r * (uint32_t)nx + (uint32_t)x) * (uint32_t)sizeof(T);
        uint64_t b = scalar_base(dst) + (uint64_t)(lvl - 1) * (uint64_t)rec_stride * sizeof(T);
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
          for (int k = 0; k < Q; ++k, b += pstride) gstore<T>(b, off, f[i][k], nt_st);
      }
    }
  };
  // The tile needs its output columns and TB halo columns on either side.  In the
  // last tile of a row (nx not a multiple of W) whole waves can lie beyond them:
  // such a wave (uniform flag) only takes part in the march's barriers, one per
  // row.  What the live lanes then read of its LDS columns reaches halo lanes
  // only, as at the tile's right edge.
  const bool live = __builtin_amdgcn_readfirstlane((c & ~63) < min(W, nx - x0) + 2 * TB ? 1 : 0) != 0;
  if (!live) {
    for (int j = 0; j < max(y1 - y0, 0) + 2 * TB; ++j) __syncthreads();
    return;
  }
  load_row(y0 - TB, ld[0], ldn[0]);
  for_each_iter([&](auto jc) __attribute__((always_inline)) {
    iteration(y0 - TB + decltype(jc)::value, jc, std::false_type{});
  }, std::make_integer_sequence<int, 2 * TB>{});
  constexpr int P0 = (2 * TB) % 6;
  for (int r0 = y0 + TB;; r0 += 6) {
    if (r0 > r_last) break;
    iteration(r0, Iter<(P0 + 0) % 6>{}, std::true_type{});
    if (r0 + 1 > r_last) break;
    iteration(r0 + 1, Iter<(P0 + 1) % 6>{}, std::true_type{});
    if (r0 + 2 > r_last) break;
    iteration(r0 + 2, Iter<(P0 + 2) % 6>{}, std::true_type{});
    if (r0 + 3 > r_last) break;
    iteration(r0 + 3, Iter<(P0 + 3) % 6>{}, std::true_type{});
    if (r0 + 4 > r_last) break;
    iteration(r0 + 4, Iter<(P0 + 4) % 6>{}, std::true_type{});
    if (r0 + 5 > r_last) break;
    iteration(r0 + 5, Iter<(P0 + 5) % 6>{}, std::true_type{});
  }
}

template <int M, typename T, int TB, int C, bool WALLS, int LAT = 2>
__global__ __launch_bounds__(C) void k_step_blocked(Problem p, const T* __restrict__ src, T* __restrict__ dst,
                                                    const Consts<T>* __restrict__ cst, int seg_rows,
                                                    uint32_t tiles_x, int nontemporal, int64_t rec_stride) {
  blocked_tile<M, T, TB, C, WALLS, false, LAT>(p, src, dst, cst, seg_rows, blockIdx.x % tiles_x,
                                               blockIdx.x / tiles_x, nontemporal, rec_stride);
}

// The same sweep with the dilute-species collision (diagonal A).  Its register
// needs differ from the full model's, so it asks the compiler for the two
// waves per SIMD the host plan assumes.
template <int M, typename T, int TB, int C, bool WALLS, int LAT = 2>
__global__ __launch_bounds__(C, 2) void k_step_blocked_dilute(Problem p, const T* __restrict__ src,
                                                              T* __restrict__ dst, const Consts<T>* __restrict__ cst,
                                                              int seg_rows, uint32_t tiles_x, int nontemporal,
                                                              int64_t rec_stride) {
  blocked_tile<M, T, TB, C, WALLS, true, LAT>(p, src, dst, cst, seg_rows, blockIdx.x % tiles_x,
                                              blockIdx.x / tiles_x, nontemporal, rec_stride);
}

// The blocked sweep over the mixtures of one batch class (equal m): workgroup
// g takes tile table entry tile_begin + g, i.e. (mixture, column tile + segment
// * column tiles of that mixture); cur selects each mixture's source buffer.
// rec_stride is 0 in every launch (a batch records nothing); it is taken at run
// time, as in the single-mixture sweep, because with a compile-time 0 the
// compiler schedules the march differently and holds more registers (quinary,
// three steps: 256 VGPRs instead of 186; four steps would not fit two waves
// per SIMD).
template <int M, typename T, int TB, int C, bool WALLS, bool DIL>
__device__ __forceinline__ void batch_blocked_body(const BatchInst* __restrict__ insts,
                                                   const BatchTile* __restrict__ tiles, uint32_t tile_begin,
                                                   char* __restrict__ ws, int cur, int seg_rows, int nontemporal,
                                                   int64_t rec_stride) {
  constexpr int W = C - 2 * TB;
  // The table entries are uniform but read by vector loads: move the fields the
  // tile uses to scalar registers (the tile addresses planes from scalar bases).
  auto u32 = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
  auto u64 = [&](uint64_t v) { return ((uint64_t)u32((uint32_t)(v >> 32)) << 32) | u32((uint32_t)v); };
  const BatchTile btv = tiles[tile_begin + blockIdx.x];
  const BatchTile bt{u32(btv.inst), u32(btv.tile)};
  const BatchInst* I = insts + bt.inst;
  Problem p;
  p.nx = (int32_t)u32((uint32_t)I->p.nx);
  p.ny = (int32_t)u32((uint32_t)I->p.ny);
  p.nz = 1;
  p.relax = (int32_t)u32((uint32_t)I->p.relax);
  p.linearized = (int32_t)u32((uint32_t)I->p.linearized);
#pragma unroll
  for (int f = 0; f < 6; ++f) p.bc[f] = (int32_t)u32((uint32_t)I->p.bc[f]);
  p.plane = (int64_t)u64((uint64_t)I->p.plane);
  const uint32_t tiles_x = (uint32_t)((p.nx + W - 1) / W);
  const T* src = reinterpret_cast<const T*>(ws + u64(I->half_off[cur]));
  T* dst = reinterpret_cast<T*>(ws + u64(I->half_off[1 - cur]));
  const Consts<T>* cst = reinterpret_cast<const Consts<T>*>(ws + u64(I->consts_off));
  blocked_tile<M, T, TB, C, WALLS, DIL>(p, src, dst, cst, seg_rows, bt.tile % tiles_x, bt.tile / tiles_x,
                                        nontemporal, rec_stride);
}

template <int M, typename T, int TB, int C, bool WALLS>
__global__ __launch_bounds__(C) void k_batch_step_blocked(const BatchInst* __restrict__ insts,
                                                          const BatchTile* __restrict__ tiles, uint32_t tile_begin,
                                                          char* __restrict__ ws, int cur, int seg_rows,
                                                          int nontemporal, int64_t rec_stride) {
  batch_blocked_body<M, T, TB, C, WALLS, false>(insts, tiles, tile_begin, ws, cur, seg_rows, nontemporal,
                                                rec_stride);
}

// A class of dilute-species mixtures (diagonal A); two waves per SIMD as for
// k_step_blocked_dilute.
template <int M, typename T, int TB, int C, bool WALLS>
__global__ __launch_bounds__(C, 2) void k_batch_step_blocked_dilute(const BatchInst* __restrict__ insts,
                                                                    const BatchTile* __restrict__ tiles,
                                                                    uint32_t tile_begin, char* __restrict__ ws, int cur,
                                                                    int seg_rows, int nontemporal,
                                                                    int64_t rec_stride) {
  batch_blocked_body<M, T, TB, C, WALLS, true>(insts, tiles, tile_begin, ws, cur, seg_rows, nontemporal,
                                               rec_stride);
}

// ---------------------------------------------------------------------------
// Small domains: one workgroup keeps both ping-pong copies in LDS and runs all
// requested steps in one launch (launch latency would otherwise dominate).
// ---------------------------------------------------------------------------
template <int LAT, int M, typename T>
__global__ __launch_bounds__(256) void k_step_lds(Problem p, const T* __restrict__ src, T* __restrict__ dst,
                                                   const Consts<T>* __restrict__ cst, int first_pull,
                                                   int64_t nsteps) {
  constexpr int Q = Lattice<LAT>::Q;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t nodes = (int64_t)p.nx * p.ny * p.nz;
  T* A = reinterpret_cast<T*>(smem_raw);
  T* B = A + (int64_t)M * Q * nodes;
  NodeConsts<M, T> nc;
  load_consts<M, T>(cst, nc);
  for (int64_t e = threadIdx.x; e < (int64_t)M * Q * nodes; e += blockDim.x) {
    const int64_t pl = e / nodes, j = e % nodes;
    A[e] = src[pl * p.plane + j];
  }
  __syncthreads();
  Problem lp = p;
  lp.plane = nodes;
  for (int64_t s = 0; s < nsteps; ++s) {
    const bool pull = (s > 0) || (first_pull != 0);
    for (int64_t j = threadIdx.x; j < nodes; j += blockDim.x) {
      NodePos n;
      n.idx = j;
      n.c[0] = (int32_t)(j % p.nx);
      const int64_t r = j / p.nx;
      n.c[1] = (int32_t)(r % p.ny);
      n.c[2] = (int32_t)(r / p.ny);
      T f[M][Q];
      gather_node<LAT, M, T>(lp, (const T*)A, n, pull, f, nc.wall);
      if (p.dilute)
        collide_node<LAT, M, T, true>(f, nc.cc);
      else
        collide_node<LAT, M, T>(f, nc.cc);
#pragma unroll
      for (int i = 0; i < M; ++i)
#pragma unroll
        for (int k = 0; k < Q; ++k) B[(int64_t)(i * Q + k) * nodes + j] = f[i][k];
    }
    __syncthreads();
    T* t = A;
    A = B;
    B = t;
  }
  for (int64_t e = threadIdx.x; e < (int64_t)M * Q * nodes; e += blockDim.x) {
    const int64_t pl = e / nodes, j = e % nodes;
    dst[pl * p.plane + j] = A[e];
  }
}

// ---------------------------------------------------------------------------
// Observables at the current time (Eqs. (3-15), (2-3b), (3-27), (2-12)):
// xi (N planes), J = c_t K m1 and grad xi = -(2/a)(I - K) m1 (m*d planes each).
// ---------------------------------------------------------------------------
template <int LAT, int M, typename T, typename TO>
__global__ __launch_bounds__(256) void k_read(Problem p, const T* __restrict__ src,
                                               const Consts<T>* __restrict__ cst, int pull, Tiling tl,
                                               TO* __restrict__ oxi, TO* __restrict__ oJ, TO* __restrict__ og) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q, DD = L::D;
  NodePos n;
  if (!tile_node(p, tl, n)) return;
  const int64_t nodes = (int64_t)p.nx * p.ny * p.nz;
  NodeConsts<M, T> nc;
  load_consts<M, T>(cst, nc);
  T f[M][Q];
  gather_node<LAT, M, T>(p, src, n, pull != 0, f, nc.wall);
  T xi[M], m1[M][DD];
  T tot = T(0);
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T s = f[i][0];
#pragma unroll
    for (int k = 1; k < Q; ++k) s += f[i][k];
    xi[i] = s;
    tot += s;
#pragma unroll
    for (int d = 0; d < DD; ++d) m1[i][d] = T(0);
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
      for (int d = 0; d < DD; ++d) {
        if (L::c(k, d) > 0) m1[i][d] += f[i][k];
        if (L::c(k, d) < 0) m1[i][d] -= f[i][k];
      }
  }
#pragma unroll
  for (int i = 0; i < M; ++i) oxi[(int64_t)i * nodes + n.idx] = TO(xi[i]);
  oxi[(int64_t)M * nodes + n.idx] = TO(T(1) - tot);
  if (!oJ && !og) return;
  T xb[M];
#pragma unroll
  for (int i = 0; i < M; ++i) xb[i] = p.linearized ? nc.xref[i] : xi[i];
  T K[M][M];
  if (p.dilute)
    ms_inverse_dilute<M, T>(xb, nc.R, T(0.5 * L::cs2), K);
  else
    ms_inverse<M, T>(xb, nc.R, T(0.5 * L::cs2), K);
#pragma unroll
  for (int i = 0; i < M; ++i) {
#pragma unroll
    for (int d = 0; d < DD; ++d) {
      T km = T(0);
#pragma unroll
      for (int j = 0; j < M; ++j) km += K[i][j] * m1[j][d];
      const int64_t o = (int64_t)(i * DD + d) * nodes + n.idx;
      if (oJ) oJ[o] = TO(T(p.c_t) * km);
      if (og) og[o] = TO(-(T(2) / T(L::cs2)) * (m1[i][d] - km));
    }
  }
}

// ---------------------------------------------------------------------------
// Diagnostics: per-workgroup partial sums (FP64), minima, maxima and non-finite
// counts over all N species, then a single-workgroup pass in fixed order.
// Partial layout per workgroup: [N sums][N minima][N maxima][1 count].
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

constexpr int kDiagThreads = 256;

template <int LAT, int M, typename T>
__global__ __launch_bounds__(kDiagThreads) void k_diag_partial(Problem p, const T* __restrict__ src,
                                                              const Consts<T>* __restrict__ cst, int pull,
                                                              double* __restrict__ partials) {
  constexpr int Q = Lattice<LAT>::Q, N = M + 1, W = 3 * N + 1;
  const int64_t nodes = (int64_t)p.nx * p.ny * p.nz;
  NodeConsts<M, T> nc;
  load_consts<M, T>(cst, nc);
  double sum[N], mn[N], mx[N], bad = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    sum[i] = 0.0;
    mn[i] = __builtin_huge_val();
    mx[i] = -__builtin_huge_val();
  }
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nodes; j += (int64_t)gridDim.x * blockDim.x) {
    NodePos n;
    n.idx = j;
    n.c[0] = (int32_t)(j % p.nx);
    const int64_t r = j / p.nx;
    n.c[1] = (int32_t)(r % p.ny);
    n.c[2] = (int32_t)(r / p.ny);
    T f[M][Q];
    gather_node<LAT, M, T>(p, src, n, pull != 0, f, nc.wall);
    double tot = 0.0;
#pragma unroll
    for (int i = 0; i <= M; ++i) {
      double x;
      if (i < M) {
        T s = f[i][0];
#pragma unroll
        for (int k = 1; k < Q; ++k) s += f[i][k];
        x = (double)s;
        tot += x;
      } else {
        x = 1.0 - tot;
      }
      if (__builtin_isfinite(x)) {
        sum[i] += x;
        mn[i] = fmin(mn[i], x);
        mx[i] = fmax(mx[i], x);
      } else {
        bad += 1.0;
      }
    }
  }
  __shared__ double red[kDiagThreads / 64][3 * kMaxSpecies + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double a = wave_sum(sum[i]), b = wave_min(mn[i]), c = wave_max(mx[i]);
    if (lane == 0) {
      red[wv][i] = a;
      red[wv][N + i] = b;
      red[wv][2 * N + i] = c;
    }
  }
  const double bb = wave_sum(bad);
  if (lane == 0) red[wv][3 * N] = bb;
  __syncthreads();
  if (threadIdx.x < W) {
    const int e = threadIdx.x;
    double v = red[0][e];
    for (int w = 1; w < kDiagThreads / 64; ++w) {
      const double u = red[w][e];
      if (e < N || e == 3 * N)
        v += u;
      else if (e < 2 * N)
        v = fmin(v, u);
      else
        v = fmax(v, u);
    }
    partials[(int64_t)blockIdx.x * W + e] = v;
  }
}

// Templated on the lattice only so that each per-lattice unit owns its copy.
// One workgroup of kDiagThreads threads: thread t combines the partials of
// workgroups t, t + kDiagThreads, ... in that order, then a halving tree in
// LDS combines the threads; the order is fixed, so the result is
// deterministic.
template <int LAT>
__global__ __launch_bounds__(kDiagThreads) void k_diag_final(const double* __restrict__ partials, int blocks, int N,
                                                            double* __restrict__ out) {
  __shared__ double red[kDiagThreads];
  const int W = 3 * N + 1;
  const int t = (int)threadIdx.x;
  for (int e = 0; e < W; ++e) {
    const int kind = (e < N || e == 3 * N) ? 0 : (e < 2 * N ? 1 : 2);   // sum, min, max
    double v = kind == 0 ? 0.0 : (kind == 1 ? __builtin_huge_val() : -__builtin_huge_val());
    for (int b = t; b < blocks; b += kDiagThreads) {
      const double u = partials[(int64_t)b * W + e];
      v = kind == 0 ? v + u : (kind == 1 ? fmin(v, u) : fmax(v, u));
    }
    red[t] = v;
    __syncthreads();
    for (int h = kDiagThreads / 2; h > 0; h >>= 1) {
      if (t < h) {
        const double u = red[t + h];
        red[t] = kind == 0 ? red[t] + u : (kind == 1 ? fmin(red[t], u) : fmax(red[t], u));
      }
      __syncthreads();
    }
    if (t == 0) out[e] = red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Batched sweep: one launch advances every tile of every mixture of a batch by
// one step.  Workgroup b reads its (mixture, tile) from the tile table and
// runs the same per-node body as k_step with that mixture's problem, buffers
// and constants; the number of evolved species (uniform per workgroup) selects
// the template instance, up to MMAX.
// ---------------------------------------------------------------------------
template <int LAT, int M, typename T, bool DIL>
__device__ __forceinline__ void batch_tile_body(const Problem& p, const T* __restrict__ src, T* __restrict__ dst,
                                                const Consts<T>* __restrict__ cst, uint32_t tile, int pull,
                                                int nontemporal) {
  constexpr int Q = Lattice<LAT>::Q;
  const uint32_t tiles_x = ((uint32_t)p.nx + blockDim.x - 1) / blockDim.x;
  const uint32_t tiles_y = ((uint32_t)p.ny + blockDim.y - 1) / blockDim.y;
  const uint32_t tx = tile % tiles_x;
  const uint32_t rest = tile / tiles_x;
  const uint32_t ty = rest % tiles_y;
  const uint32_t tz = rest / tiles_y;
  NodePos n;
  n.c[0] = (int32_t)(tx * blockDim.x + threadIdx.x);
  n.c[1] = (int32_t)(ty * blockDim.y + threadIdx.y);
  n.c[2] = (int32_t)tz;
  if (n.c[0] >= p.nx || n.c[1] >= p.ny) return;
  n.idx = n.c[0] + (int64_t)p.nx * (n.c[1] + (int64_t)p.ny * n.c[2]);
  NodeConsts<M, T> nc;
  load_consts<M, T>(cst, nc);
  T f[M][Q];
  gather_node<LAT, M, T>(p, src, n, pull != 0, f, nc.wall, nontemporal);
  collide_node<LAT, M, T, DIL>(f, nc.cc);
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int k = 0; k < Q; ++k)
      store_value(dst + (int64_t)(i * Q + k) * p.plane + n.idx, f[i][k], nontemporal & NT_STORE);
}

// DIL: a range of dilute-species mixtures (a separate instantiation).
template <int LAT, int MMAX, typename T, bool DIL = false>
__global__ __launch_bounds__(256) void k_batch_step(const BatchInst* __restrict__ insts,
                                                    const BatchTile* __restrict__ tiles, uint32_t tile_begin,
                                                    uint32_t ntiles, char* __restrict__ ws, int cur, int pull,
                                                    int remap, int nontemporal) {
  Tiling tl;
  tl.tiles = ntiles;
  tl.remap = (uint32_t)remap;
  const uint32_t L = logical_tile(tl);
  const BatchTile bt = tiles[tile_begin + L];
  const BatchInst* I = insts + bt.inst;
  const int m = I->m;
  const T* src = reinterpret_cast<const T*>(ws + I->half_off[cur]);
  T* dst = reinterpret_cast<T*>(ws + I->half_off[1 - cur]);
  const Consts<T>* cst = reinterpret_cast<const Consts<T>*>(ws + I->consts_off);
  const Problem& p = I->p;
#define MSD_BATCH_CASE(MM)                                                              \
  case MM:                                                                              \
    if constexpr (MM <= MMAX) batch_tile_body<LAT, MM, T, DIL>(p, src, dst, cst, bt.tile, pull, nontemporal); \
    break;
  switch (m) {
    MSD_BATCH_CASE(1)
    MSD_BATCH_CASE(2)
    MSD_BATCH_CASE(3)
    MSD_BATCH_CASE(4)
    MSD_BATCH_CASE(5)
    MSD_BATCH_CASE(6)
    MSD_BATCH_CASE(7)
    default:
      break;
  }
#undef MSD_BATCH_CASE
}

// ---------------------------------------------------------------------------
// Adjoint sweep.  Adjoint buffers hold dL/df^t, the derivative with respect to
// the pre-collision distributions at time t, at their own node.  Forward step
// t is g^t = C(f^{t-1}) and f^t = P(g^t) (P the propagation, f^{t-1} = P(s_{t-1})
// for t >= 2 and f^0 = s_0).  Its adjoint reads dL/df^t through the transposed
// propagation (dL/dg^t = P^T dL/df^t), recomputes f^{t-1} from s_{t-1}, applies
// the transposed collision Jacobian and stores dL/df^{t-1} at the node; dL/dR
// is accumulated per tile in FP64.
// ---------------------------------------------------------------------------
template <int LAT, int M, typename T>
__global__ __launch_bounds__(256) void k_adjoint_seed(Problem p, const double* __restrict__ G, T* __restrict__ adj,
                                                      int pull, Tiling tl) {
  constexpr int Q = Lattice<LAT>::Q;
  NodePos n;
  if (!tile_node(p, tl, n)) return;
  const int64_t nodes = (int64_t)p.nx * p.ny * p.nz;
  // xi_i = sum_k f_ik (i < N) and xi_N = 1 - sum: dL/df_ik = G_i - G_N for every k
  const double gN = G[(int64_t)M * nodes + n.idx];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const T v = T(G[(int64_t)i * nodes + n.idx] - gN);
#pragma unroll
    for (int k = 0; k < Q; ++k) adj[(int64_t)(i * Q + k) * p.plane + n.idx] = v;
  }
}

// The adjoint sweep gives each thread kAdjointNodesPerThread nodes (from
// consecutive block_x-wide strips along x), so that one workgroup reduction of
// dL/dR covers 4 * 256 nodes.
// DIL: the dilute-species collision (a separate instantiation, chosen at launch).
template <int LAT, int M, typename T, bool A32, bool DIL = false>
__global__ __launch_bounds__(256) void k_adjoint_step(Problem p, const T* __restrict__ state_prev,
                                                      const T* __restrict__ adj_in, T* __restrict__ adj_out,
                                                      const Consts<T>* __restrict__ cst, int pull, Tiling tl,
                                                      double* __restrict__ racc) {
  constexpr int Q = Lattice<LAT>::Q, E = M * (M + 1), NPT = kAdjointNodesPerThread;
  const uint32_t tile = logical_tile(tl);
  const uint32_t tx = tile % tl.tiles_x;
  const uint32_t rest = tile / tl.tiles_x;
  const uint32_t ty = rest % tl.tiles_y;
  const uint32_t tz = rest / tl.tiles_y;
  // this thread's dL/dR over its nodes in the sweep's precision, reduced in FP64 below
  T Rbar[M][M + 1];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j <= M; ++j) Rbar[i][j] = T(0);
  NodeConsts<M, T> nc;
  load_consts<M, T>(cst, nc);
  const Planes<T, A32> S{state_prev, p.plane}, A{adj_in, p.plane};
  NodePos n;
  n.c[1] = (int32_t)(ty * blockDim.y + threadIdx.y);
  n.c[2] = (int32_t)tz;
  for (int j = 0; j < NPT; ++j) {
    n.c[0] = (int32_t)((tx * NPT + j) * blockDim.x + threadIdx.x);
    if (n.c[0] >= p.nx || n.c[1] >= p.ny) continue;
    n.idx = n.c[0] + (int64_t)p.nx * (n.c[1] + (int64_t)p.ny * n.c[2]);
    T f[M][Q], u[M][Q], fb[M][Q];
    if (pull) {
#pragma unroll
      for (int k = 0; k < Q; ++k) pull_dir<LAT, M, T, A32>(p, S, n, k, f, nc.wall, false);
    } else {
#pragma unroll
      for (int i = 0; i < M; ++i)
#pragma unroll
        for (int k = 0; k < Q; ++k) f[i][k] = S(i * Q + k, n.idx);
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) pull_dir<LAT, M, T, A32>(p, A, n, k, u, nc.wall, true);
    collide_node_adjoint<LAT, M, T, DIL>(f, u, nc.R, nc.xref, p.linearized != 0, nc.cc, fb, Rbar);
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        T* plane_out = adj_out + (int64_t)(i * Q + k) * p.plane;
        if constexpr (A32)
          *reinterpret_cast<T*>(reinterpret_cast<char*>(plane_out) + (uint32_t)n.idx * (uint32_t)sizeof(T)) = fb[i][k];
        else
          plane_out[n.idx] = fb[i][k];
      }
  }
  // workgroup sum of dL/dR, added to this tile's accumulator slot
  __shared__ double red[4][E];
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j <= M; ++j) {
      const double s = wave_sum((double)Rbar[i][j]);
      if (lane == 0) red[wv][i * (M + 1) + j] = s;
    }
  __syncthreads();
  const int waves = (int)((blockDim.x * blockDim.y + 63) / 64);
  if (tid < E) {
    double s = red[0][tid];
    for (int w = 1; w < waves; ++w) s += red[w][tid];
    racc[(int64_t)tile * E + tid] += s;
  }
}

// ---------------------------------------------------------------------------
// Temporally blocked adjoint sweep (D2Q5): TB adjoint steps per pass, for the
// forward steps t, t-1, ..., t-TB+1.  Level 0 holds a_t (read once); level l
// produces a_{t-l} from level l-1 through the transposed propagation and from
// the state s_{t-l}, pulled straight from memory.  The transposed pull takes
// the y-directions from the same column (u_+y(r) = a_+y(r+1), u_-y(r) =
// a_-y(r-1)), so each level keeps a register window as the forward blocked
// sweep does, with the x-directions exchanged through LDS.  dL/dR is summed
// only over the nodes a workgroup owns (its output rows and columns at every
// level), so overlapping halos are not counted twice; the per-workgroup FP64
// sum goes to accumulator slot blockIdx.x.
// ---------------------------------------------------------------------------
template <typename T>
struct AdjStates {
  const T* s[4];   // s[l - 1] = s_{t-l}
};

template <int M, typename T, int TB, int C, bool WALLS>
__global__ __launch_bounds__(C) void k_adjoint_blocked(Problem p, AdjStates<T> S, const T* __restrict__ adj_in,
                                                       T* __restrict__ adj_out, const Consts<T>* __restrict__ cst,
                                                       int seg_rows, uint32_t tiles_x, double* __restrict__ racc) {
  using L = Lattice<2>;
  constexpr int Q = L::Q, P = M * Q, W = C - 2 * TB, E = M * (M + 1);
  static_assert(L::axis(1) == 0 && L::sgn(1) > 0 && L::axis(3) == 0 && L::sgn(3) < 0, "x directions");
  static_assert(L::axis(2) == 1 && L::sgn(2) > 0 && L::axis(4) == 1 && L::sgn(4) < 0, "y directions");
  constexpr int KXP = 1, KYP = 2, KXM = 3, KYM = 4;
  __shared__ T xs[TB][2][2][M][C];
  __shared__ double red[C / 64][E];

  const int c = (int)threadIdx.x;
  const int cm = c > 0 ? c - 1 : 0, cp = c < C - 1 ? c + 1 : C - 1;
  const int nx = p.nx, ny = p.ny;
  const uint32_t tx = blockIdx.x % tiles_x;
  const uint32_t seg = blockIdx.x / tiles_x;
  const int x0 = (int)tx * W;
  const int y0 = (int)seg * seg_rows;
  const int y1 = min(y0 + seg_rows, ny);
  const int x = x0 - TB + c;
  // WALLS = false is only launched on a fully periodic domain
  const bool px = !WALLS || p.bc[0] == BC_PERIODIC, py = !WALLS || p.bc[2] == BC_PERIODIC;
  const bool x_in = x >= 0 && x < nx;
  const bool col_ok = x_in || px;
  const bool col_own = c >= TB && c < C - TB && x_in;
  const int xl = x_in ? x : (((x % nx) + nx) % nx);
  // neighbour columns of the pull from a state (wrapped; at a wall the face rule applies instead)
  const int xlm = xl > 0 ? xl - 1 : nx - 1, xlp = xl < nx - 1 ? xl + 1 : 0;
  const bool tile_xwall = !px && (x0 - TB <= 0 || x0 - TB + C - 1 >= nx - 1);
  const bool wall_xlo = !px && x == 0, wall_xhi = !px && x == nx - 1;
  NodeConsts<M, T> nc;
  load_consts<M, T>(cst, nc);
  const bool lin = p.linearized != 0;
  // this thread's dL/dR over a pass (at most TB (seg_rows + 2 TB) nodes) in the
  // sweep's precision, reduced in FP64 below
  T Rbar[M][M + 1];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j <= M; ++j) Rbar[i][j] = T(0);

  // Per level (0 .. TB-1): -y of row r-1; rest/+y/-y of rows r (cur) and r+1 (nxt).
  T yprev[TB][M], cur[TB][3][M], nxt[TB][3][M];
#pragma unroll
  for (int l = 0; l < TB; ++l)
#pragma unroll
    for (int i = 0; i < M; ++i) {
      yprev[l][i] = T(0);
#pragma unroll
      for (int j = 0; j < 3; ++j) cur[l][j][i] = nxt[l][j][i] = T(0);
    }
  // value of plane pl at (row, col): an opaque scalar plane start plus a 32-bit lane offset
  const uint64_t pstride = (uint64_t)p.plane * sizeof(T);
  auto at = [&](const T* base, int pl, int row, int col) {
    const uint32_t off = ((uint32_t)row * (uint32_t)nx + (uint32_t)col) * (uint32_t)sizeof(T);
    return gload<T>(scalar_base(base) + (uint64_t)pl * opaque_u64(pstride), off, false);
  };
  T ld_row[P];
  auto load_row = [&](int r) {
    const bool r_in = r >= 0 && r < ny;
    const int rl = r_in ? r : (((r % ny) + ny) % ny);
    // planes walked from one scalar base in steps of the plane stride
    uint64_t b = scalar_base(adj_in);
    if (col_ok && (r_in || py)) {
      const uint32_t off = ((uint32_t)rl * (uint32_t)nx + (uint32_t)xl) * (uint32_t)sizeof(T);
#pragma unroll
      for (int pl = 0; pl < P; ++pl, b += pstride) ld_row[pl] = gload<T>(b, off, false);
    } else {
#pragma unroll
      for (int pl = 0; pl < P; ++pl) ld_row[pl] = T(0);
    }
  };
  auto advance = [&](int l) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
      yprev[l][i] = cur[l][2][i];
#pragma unroll
      for (int j = 0; j < 3; ++j) cur[l][j][i] = nxt[l][j][i];
    }
  };
  auto enter = [&](int l, int r, const T (&g)[M][Q]) {
    const int s = r & 1;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      xs[l][s][0][i][c] = g[i][KXP];
      xs[l][s][1][i][c] = g[i][KXM];
      nxt[l][0][i] = g[i][0];
      nxt[l][1][i] = g[i][KYP];
      nxt[l][2][i] = g[i][KYM];
    }
  };
  // transposed face rule: the adjoint of a zero-flux face passes the value on, of a Dirichlet face negates it
  auto tface = [&](int fk, T v) { return (p.bc[fk] == BC_ZERO_FLUX) ? v : -v; };
  auto face = [&](int fk, int kb, int i, T back) {
    return (p.bc[fk] == BC_ZERO_FLUX) ? back : T(2.0 * L::w(kb)) * nc.wall[fk][i] - back;
  };

  const int r_last = y1 - 1 + TB;
  // waves wholly beyond the tile's output and halo columns (the last tile of a
  // row) take part in the barriers only and add nothing to dL/dR, as in the
  // forward row march
  const bool live = __builtin_amdgcn_readfirstlane((c & ~63) < min(W, nx - x0) + 2 * TB ? 1 : 0) != 0;
  int r_in = y0 - TB;
  if (!live) {
    for (; r_in <= r_last; ++r_in) __syncthreads();
  } else {
    load_row(r_in);
    for (; r_in <= r_last; ++r_in) {
      __syncthreads();
      {
        T g[M][Q];
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
          for (int k = 0; k < Q; ++k) g[i][k] = ld_row[i * Q + k];
        advance(0);
        enter(0, r_in, g);
      }
      if (r_in < r_last) load_row(r_in + 1);
#pragma unroll
      for (int lvl = 1; lvl <= TB; ++lvl) {
        const int r = r_in - lvl;
        const int lp = lvl - 1;
        const int s = r & 1;
        const bool row_ok = r >= y0 - TB + lvl && r <= r_last - lvl && (py || (r >= 0 && r < ny));
        if (lvl < TB) advance(lvl);
        if (!row_ok) continue;
        // u = dL/dg at this node: the transposed pull of a_{t-l+1}
        T u[M][Q];
#pragma unroll
        for (int i = 0; i < M; ++i) {
          u[i][0] = cur[lp][0][i];
          u[i][KXP] = xs[lp][s][0][i][cp];
          u[i][KXM] = xs[lp][s][1][i][cm];
          u[i][KYP] = nxt[lp][1][i];
          u[i][KYM] = yprev[lp][i];
        }
        // f = f^{t-l} at this node: the pull of s_{t-l}, planes walked from one scalar base
        const int rl = (r >= 0 && r < ny) ? r : (((r % ny) + ny) % ny);
        const int rlm = rl > 0 ? rl - 1 : ny - 1, rlp = rl < ny - 1 ? rl + 1 : 0;
        const T* st = S.s[lp];
        T f[M][Q];
        if (col_ok) {
          const uint32_t row = (uint32_t)rl * (uint32_t)nx, sz = (uint32_t)sizeof(T);
          uint32_t off[Q];
          off[0] = (row + (uint32_t)xl) * sz;
          off[KXP] = (row + (uint32_t)xlm) * sz;
          off[KXM] = (row + (uint32_t)xlp) * sz;
          off[KYP] = ((uint32_t)rlm * (uint32_t)nx + (uint32_t)xl) * sz;
          off[KYM] = ((uint32_t)rlp * (uint32_t)nx + (uint32_t)xl) * sz;
          uint64_t b = scalar_base(st);
#pragma unroll
          for (int i = 0; i < M; ++i)
#pragma unroll
            for (int k = 0; k < Q; ++k, b += pstride) f[i][k] = gload<T>(b, off[k], false);
        } else {
#pragma unroll
          for (int i = 0; i < M; ++i)
#pragma unroll
            for (int k = 0; k < Q; ++k) f[i][k] = T(0);
        }
        if constexpr (WALLS) {
          if (tile_xwall) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
              if (wall_xlo) {
                f[i][KXP] = face(0, KXM, i, at(st, i * Q + KXM, rl, xl));
                u[i][KXM] = tface(0, xs[lp][s][0][i][c]);
              }
              if (wall_xhi) {
                f[i][KXM] = face(1, KXP, i, at(st, i * Q + KXP, rl, xl));
                u[i][KXP] = tface(1, xs[lp][s][1][i][c]);
              }
            }
          }
          if (!py && r == 0) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
              f[i][KYP] = face(2, KYM, i, at(st, i * Q + KYM, rl, xl));
              u[i][KYM] = tface(2, cur[lp][1][i]);
            }
          }
          if (!py && r == ny - 1) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
              f[i][KYM] = face(3, KYP, i, at(st, i * Q + KYP, rl, xl));
              u[i][KYP] = tface(3, cur[lp][2][i]);
            }
          }
        }
        T g[M][Q];
        if (r >= y0 && r < y1) {
          collide_node_adjoint<2, M, T>(f, u, nc.R, nc.xref, lin, nc.cc, g, Rbar);
        } else {
          T Rhalo[M][M + 1] = {};
          collide_node_adjoint<2, M, T>(f, u, nc.R, nc.xref, lin, nc.cc, g, Rhalo);
        }
        if (lvl < TB) {
          enter(lvl, r, g);
        } else if (col_own && r >= y0 && r < y1) {
          const uint32_t off = ((uint32_t)r * (uint32_t)nx + (uint32_t)x) * (uint32_t)sizeof(T);
          uint64_t b = scalar_base(adj_out);
#pragma unroll
          for (int i = 0; i < M; ++i)
#pragma unroll
            for (int k = 0; k < Q; ++k, b += pstride) gstore<T>(b, off, g[i][k], 0);
        }
      }
    }
  }
  // workgroup sum of dL/dR over the owned columns, added to this workgroup's slot
  const int lane = c & 63, wv = c >> 6;
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j <= M; ++j) {
      const double v = wave_sum(col_own ? (double)Rbar[i][j] : 0.0);
      if (lane == 0) red[wv][i * (M + 1) + j] = v;
    }
  __syncthreads();
  if (c < E) {
    double v = red[0][c];
#pragma unroll
    for (int w = 1; w < C / 64; ++w) v += red[w][c];
    racc[(int64_t)blockIdx.x * E + c] += v;
  }
}

template <int LAT, int M, typename T>
__global__ __launch_bounds__(256) void k_adjoint_xi0(Problem p, const T* __restrict__ adj0, double* __restrict__ out,
                                                     Tiling tl) {
  using L = Lattice<LAT>;
  NodePos n;
  if (!tile_node(p, tl, n)) return;
  const int64_t nodes = (int64_t)p.nx * p.ny * p.nz;
  // f^0_ik = w_k xi0_i (Sec. 4 initialisation)
#pragma unroll
  for (int i = 0; i < M; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) s += L::w(k) * (double)adj0[(int64_t)(i * L::Q + k) * p.plane + n.idx];
    out[(int64_t)i * nodes + n.idx] = s;
  }
}

// dL/dD for the symmetric pair (i, j): -(Rbar_ij + Rbar_ji) / D_ij^2, where
// Rbar_ji exists only when both species are evolved.  One workgroup, fixed
// summation order over tiles.
template <int LAT, int M>
__global__ void k_adjoint_dD(Problem p, const double* __restrict__ racc, uint32_t tiles, double* __restrict__ out) {
  constexpr int E = M * (M + 1), N = M + 1;
  __shared__ double tot[E];
  const int e = threadIdx.x;
  if (e < E) {
    double s = 0.0;
    for (uint32_t t = 0; t < tiles; ++t) s += racc[(int64_t)t * E + e];
    tot[e] = s;
  }
  __syncthreads();
  if (e < N * N) {
    const int i = e / N, j = e % N;
    double g = 0.0;
    if (i != j) {
      if (i < M) g += tot[i * (M + 1) + j];
      if (j < M) g += tot[j * (M + 1) + i];
      g = -g / (p.D[i][j] * p.D[i][j]);
    }
    out[e] = g;
  }
}

template <int LAT>
__global__ void k_fill_zero(double* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

}  // namespace msd

#include "msd_blocked3d.h"

namespace msd {

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------
inline Tiling make_tiling(const LaunchArgs& a, int V = 1) {
  Tiling t;
  const int64_t span = (int64_t)a.block_x * V;
  t.tiles_x = (uint32_t)((a.p.nx + span - 1) / span);
  t.tiles_y = (uint32_t)((a.p.ny + a.block_y - 1) / a.block_y);
  t.tiles = t.tiles_x * t.tiles_y * (uint32_t)a.p.nz;
  t.remap = a.xcd_remap ? 1u : 0u;
  return t;
}

template <int M, typename T, int TB>
hipError_t launch_adjoint_blocked_tb(const LaunchArgs& a) {
  constexpr int C = adjoint_blocked_cols(M, TB, (int)sizeof(T));
  if constexpr (C == 0) {
    return hipErrorInvalidValue;
  } else {
    constexpr int W = C - 2 * TB;
    const uint32_t tiles_x = (uint32_t)((a.p.nx + W - 1) / W);
    const uint32_t segs = (uint32_t)((a.p.ny + a.seg_rows - 1) / a.seg_rows);
    const bool walls = a.p.bc[0] != BC_PERIODIC || a.p.bc[2] != BC_PERIODIC;
    AdjStates<T> S;
    for (int l = 0; l < 4; ++l) S.s[l] = static_cast<const T*>(a.states[l]);
    const T* ain = static_cast<const T*>(a.adj_in);
    T* aout = static_cast<T*>(a.dst);
    const Consts<T>* cst = static_cast<const Consts<T>*>(a.consts);
    if (walls)
      hipLaunchKernelGGL((k_adjoint_blocked<M, T, TB, C, true>), dim3(tiles_x * segs), dim3(C), 0, a.stream, a.p, S,
                         ain, aout, cst, a.seg_rows, tiles_x, a.partials);
    else
      hipLaunchKernelGGL((k_adjoint_blocked<M, T, TB, C, false>), dim3(tiles_x * segs), dim3(C), 0, a.stream, a.p,
                         S, ain, aout, cst, a.seg_rows, tiles_x, a.partials);
    return hipSuccess;
  }
}

// Dynamic LDS the forward blocked sweep adds to its own so that each
// workgroup holds at least a.blocked_lds_floor bytes: the host sets the floor
// to keep at most two workgroups on a CU, where the sweep runs fastest.
template <int M, typename T, int TB, int C>
constexpr int blocked_lds_bytes() {
  return (TB - 1) * 2 * 2 * M * C * (int)sizeof(T);
}
template <int M, typename T, int TB, int C>
size_t blocked_lds_pad(const LaunchArgs& a) {
  constexpr int own = blocked_lds_bytes<M, T, TB, C>();
  return a.blocked_lds_floor > own ? (size_t)(a.blocked_lds_floor - own) : 0;
}

// Workgroups of a blocked kernel (sweep or adjoint) that the whole device holds
// at once: resident workgroups per CU (registers and LDS, with the sweep's
// reservation) times the CU count; out[1] is the CU count.
template <int M, typename T, int TB, int LAT = 2>
hipError_t blocked_resident(const LaunchArgs& a, int* out) {
  out[0] = out[1] = 0;
  constexpr int C = blocked_cols(M, TB, (int)sizeof(T)), CA = adjoint_blocked_cols(M, TB, (int)sizeof(T));
  const bool walls = a.p.bc[0] != BC_PERIODIC || a.p.bc[2] != BC_PERIODIC;
  int per_cu = 0;
  hipError_t e = hipSuccess;
  // D2Q4 has the forward sweep in 256-column tiles only (no wide tiles, no blocked adjoint)
  if (LAT != 2 && (a.adjoint || a.cols == kBlockedColsWide)) return hipErrorInvalidValue;
  if (a.adjoint) {
    if constexpr (CA > 0) {
      e = walls ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adjoint_blocked<M, T, TB, CA, true>, CA, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adjoint_blocked<M, T, TB, CA, false>, CA, 0);
    }
  } else if (a.cols == kBlockedColsWide) {
    if constexpr (blocked_wide_ok(M, TB, (int)sizeof(T))) {
      constexpr int CW = kBlockedColsWide;
      const size_t pad = blocked_lds_pad<M, T, TB, CW>(a);
      if (walls) {
        if constexpr (blocked_wide_walls_ok(M))
          e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_blocked<M, T, TB, CW, true>, CW, pad);
        else
          return hipErrorInvalidValue;
      } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_blocked<M, T, TB, CW, false>, CW, pad);
      }
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    if constexpr (C > 0) {
      const size_t pad = blocked_lds_pad<M, T, TB, C>(a);
      if (walls) {
        if constexpr (blocked_walls_ok(M, TB, (int)sizeof(T)))
          e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_blocked<M, T, TB, C, true, LAT>, C, pad);
        else
          return hipErrorInvalidValue;
      } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_blocked<M, T, TB, C, false, LAT>, C, pad);
      }
    }
  }
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  out[0] = per_cu * cus;
  out[1] = cus;
  return hipSuccess;
}

template <int M, typename T>
hipError_t launch_adjoint_blocked(const LaunchArgs& a) {
  if (a.tb == 2) return launch_adjoint_blocked_tb<M, T, 2>(a);
  if (a.tb == 3) return launch_adjoint_blocked_tb<M, T, 3>(a);
  if (a.tb == 4) return launch_adjoint_blocked_tb<M, T, 4>(a);
  return hipErrorInvalidValue;
}

// The wide (512-column) tile for the full model, where the host plan chose it.
template <int M, typename T, int TB>
hipError_t launch_blocked_wide(const LaunchArgs& a) {
  if constexpr (!blocked_wide_ok(M, TB, (int)sizeof(T))) {
    return hipErrorInvalidValue;
  } else {
    constexpr int C = kBlockedColsWide, W = C - 2 * TB;
    if (a.p.dilute) return hipErrorInvalidValue;
    const uint32_t tiles_x = (uint32_t)((a.p.nx + W - 1) / W);
    const uint32_t segs = (uint32_t)((a.p.ny + a.seg_rows - 1) / a.seg_rows);
    const bool walls = a.p.bc[0] != BC_PERIODIC || a.p.bc[2] != BC_PERIODIC;
    const T* src = static_cast<const T*>(a.src);
    T* dst = static_cast<T*>(a.dst);
    const Consts<T>* cst = static_cast<const Consts<T>*>(a.consts);
    const size_t pad = blocked_lds_pad<M, T, TB, C>(a);
    if (walls) {
      if constexpr (blocked_wide_walls_ok(M))
        hipLaunchKernelGGL((k_step_blocked<M, T, TB, C, true>), dim3(tiles_x * segs), dim3(C), pad, a.stream, a.p,
                           src, dst, cst, a.seg_rows, tiles_x, a.nontemporal, a.rec_stride);
      else
        return hipErrorInvalidValue;
    } else {
      hipLaunchKernelGGL((k_step_blocked<M, T, TB, C, false>), dim3(tiles_x * segs), dim3(C), pad, a.stream, a.p,
                         src, dst, cst, a.seg_rows, tiles_x, a.nontemporal, a.rec_stride);
    }
    return hipSuccess;
  }
}

template <int M, typename T, int TB, int LAT = 2>
hipError_t launch_blocked_tb(const LaunchArgs& a) {
  constexpr int C = blocked_cols(M, TB, (int)sizeof(T));
  if (a.cols == kBlockedColsWide) {
    if constexpr (LAT == 2)
      return launch_blocked_wide<M, T, TB>(a);
    else
      return hipErrorInvalidValue;
  }
  if constexpr (C == 0) {
    return hipErrorInvalidValue;
  } else {
    constexpr int W = C - 2 * TB;
    const uint32_t tiles_x = (uint32_t)((a.p.nx + W - 1) / W);
    const uint32_t segs = (uint32_t)((a.p.ny + a.seg_rows - 1) / a.seg_rows);
    const bool walls = a.p.bc[0] != BC_PERIODIC || a.p.bc[2] != BC_PERIODIC;
    const T* src = static_cast<const T*>(a.src);
    T* dst = static_cast<T*>(a.dst);
    const Consts<T>* cst = static_cast<const Consts<T>*>(a.consts);
    const size_t pad = blocked_lds_pad<M, T, TB, C>(a);
    const dim3 grid(tiles_x * segs);
    if (walls) {
      // walled instantiations only up to their own (smaller) window
      if constexpr (!blocked_walls_ok(M, TB, (int)sizeof(T))) {
        return hipErrorInvalidValue;
      } else if (a.p.dilute) {
        hipLaunchKernelGGL((k_step_blocked_dilute<M, T, TB, C, true, LAT>), grid, dim3(C), pad, a.stream, a.p, src,
                           dst, cst, a.seg_rows, tiles_x, a.nontemporal, a.rec_stride);
      } else {
        hipLaunchKernelGGL((k_step_blocked<M, T, TB, C, true, LAT>), grid, dim3(C), pad, a.stream, a.p, src, dst, cst,
                           a.seg_rows, tiles_x, a.nontemporal, a.rec_stride);
      }
    } else if (a.p.dilute) {
      hipLaunchKernelGGL((k_step_blocked_dilute<M, T, TB, C, false, LAT>), grid, dim3(C), pad, a.stream, a.p, src,
                         dst, cst, a.seg_rows, tiles_x, a.nontemporal, a.rec_stride);
    } else {
      hipLaunchKernelGGL((k_step_blocked<M, T, TB, C, false, LAT>), grid, dim3(C), pad, a.stream, a.p, src, dst,
                         cst, a.seg_rows, tiles_x, a.nontemporal, a.rec_stride);
    }
    return hipSuccess;
  }
}

template <int M, typename T, int TB>
hipError_t launch_batch_blocked_tb(const LaunchArgs& a) {
  constexpr int C = blocked_cols(M, TB, (int)sizeof(T));
  if constexpr (C == 0) {
    return hipErrorInvalidValue;
  } else {
    if (a.ntiles == 0) return hipSuccess;
    const size_t pad = blocked_lds_pad<M, T, TB, C>(a);
    const dim3 grid(a.ntiles);
    const int64_t no_record = 0;
    if (a.walls) {
      // walled instantiations only up to their own (smaller) window
      if constexpr (!blocked_walls_ok(M, TB, (int)sizeof(T))) {
        return hipErrorInvalidValue;
      } else if (a.dilute) {
        hipLaunchKernelGGL((k_batch_step_blocked_dilute<M, T, TB, C, true>), grid, dim3(C), pad, a.stream, a.insts,
                           a.tiles, a.tile_begin, a.ws, a.cur, a.seg_rows, a.nontemporal, no_record);
      } else {
        hipLaunchKernelGGL((k_batch_step_blocked<M, T, TB, C, true>), grid, dim3(C), pad, a.stream, a.insts, a.tiles,
                           a.tile_begin, a.ws, a.cur, a.seg_rows, a.nontemporal, no_record);
      }
    } else if (a.dilute) {
      hipLaunchKernelGGL((k_batch_step_blocked_dilute<M, T, TB, C, false>), grid, dim3(C), pad, a.stream, a.insts,
                         a.tiles, a.tile_begin, a.ws, a.cur, a.seg_rows, a.nontemporal, no_record);
    } else {
      hipLaunchKernelGGL((k_batch_step_blocked<M, T, TB, C, false>), grid, dim3(C), pad, a.stream, a.insts, a.tiles,
                         a.tile_begin, a.ws, a.cur, a.seg_rows, a.nontemporal, no_record);
    }
    return hipSuccess;
  }
}

template <int M, typename T>
hipError_t launch_batch_blocked(const LaunchArgs& a) {
  if (a.tb == 2) return launch_batch_blocked_tb<M, T, 2>(a);
  if (a.tb == 3) return launch_batch_blocked_tb<M, T, 3>(a);
  if (a.tb == 4) return launch_batch_blocked_tb<M, T, 4>(a);
  if (a.tb == 5) return launch_batch_blocked_tb<M, T, 5>(a);
  if (a.tb == 6) return launch_batch_blocked_tb<M, T, 6>(a);
  return hipErrorInvalidValue;
}

template <int M, typename T, int LAT = 2>
hipError_t launch_blocked(const LaunchArgs& a) {
  if (a.tb == 2) return launch_blocked_tb<M, T, 2, LAT>(a);
  if (a.tb == 3) return launch_blocked_tb<M, T, 3, LAT>(a);
  if (a.tb == 4) return launch_blocked_tb<M, T, 4, LAT>(a);
  if (a.tb == 5) return launch_blocked_tb<M, T, 5, LAT>(a);
  if (a.tb == 6) return launch_blocked_tb<M, T, 6, LAT>(a);
  return hipErrorInvalidValue;
}

// Width of the vectorised sweep for this launch: the requested vec (1, 2, 4)
// when the extents and offsets allow it, else 0 (the general 64-bit kernel).
template <typename T>
int vec_width(const LaunchArgs& a) {
  if (a.vec <= 0 || a.block_x % 64) return 0;
  if ((uint64_t)a.p.plane * sizeof(T) >= (1ull << 32)) return 0;
  for (int v = a.vec; v >= 1; v >>= 1)
    if (a.p.nx % v == 0) return v;
  return 0;
}

template <int LAT, int M, typename T>
hipError_t run(Op op, const LaunchArgs& a) {
  const Consts<T>* cst = static_cast<const Consts<T>*>(a.consts);
  const int64_t nodes = (int64_t)a.p.nx * a.p.ny * a.p.nz;
  switch (op) {
    case Op::Constants:
      hipLaunchKernelGGL((k_constants<LAT, M, T>), dim3(1), dim3(64), 0, a.stream, a.p, a.n_species,
                         static_cast<Consts<T>*>(a.consts_out));
      break;
    case Op::Init: {
      const dim3 grid((unsigned)((nodes + 255) / 256));
      if (a.in_prec == 8)
        hipLaunchKernelGGL((k_init<LAT, M, T, double>), grid, dim3(256), 0, a.stream, a.p,
                           static_cast<const double*>(a.xi0), static_cast<T*>(a.dst));
      else
        hipLaunchKernelGGL((k_init<LAT, M, T, float>), grid, dim3(256), 0, a.stream, a.p,
                           static_cast<const float*>(a.xi0), static_cast<T*>(a.dst));
      break;
    }
    case Op::Step: {
      // the vectorised kernel shares x-neighbours between lanes: axis-aligned lattices only
      // (and the full Maxwell-Stefan collision only)
      const int V = (Lattice<LAT>::diag || a.p.dilute) ? 0 : vec_width<T>(a);
      const Tiling tl = make_tiling(a, V > 0 ? V : 1);
      const dim3 grid(tl.tiles), block(a.block_x, a.block_y);
      const T* src = static_cast<const T*>(a.src);
      T* dst = static_cast<T*>(a.dst);
      bool done = false;
      if constexpr (!Lattice<LAT>::diag) {
        done = true;
        if (V == 4)
          hipLaunchKernelGGL((k_step_vec<LAT, M, T, 4>), grid, block, 0, a.stream, a.p, src, dst, cst, a.pull, tl,
                             a.nontemporal);
        else if (V == 2)
          hipLaunchKernelGGL((k_step_vec<LAT, M, T, 2>), grid, block, 0, a.stream, a.p, src, dst, cst, a.pull, tl,
                             a.nontemporal);
        else if (V == 1)
          hipLaunchKernelGGL((k_step_vec<LAT, M, T, 1>), grid, block, 0, a.stream, a.p, src, dst, cst, a.pull, tl,
                             a.nontemporal);
        else
          done = false;
      }
      if (!done && a.p.dilute)
        hipLaunchKernelGGL((k_step<LAT, M, T, true>), grid, block, 0, a.stream, a.p, src, dst, cst, a.pull, tl,
                           a.nontemporal);
      else if (!done)
        hipLaunchKernelGGL((k_step<LAT, M, T>), grid, block, 0, a.stream, a.p, src, dst, cst, a.pull, tl,
                           a.nontemporal);
      break;
    }
    case Op::StepLds: {
      const int threads = (int)(nodes < 256 ? ((nodes + 63) / 64) * 64 : 256);
      const size_t shmem = 2 * sizeof(T) * (size_t)M * Lattice<LAT>::Q * (size_t)nodes;
      hipLaunchKernelGGL((k_step_lds<LAT, M, T>), dim3(1), dim3(threads), shmem, a.stream, a.p,
                         static_cast<const T*>(a.src), static_cast<T*>(a.dst), cst, a.pull, a.nsteps);
      break;
    }
    case Op::Read: {
      const Tiling tl = make_tiling(a);
      if (a.out_prec == 8)
        hipLaunchKernelGGL((k_read<LAT, M, T, double>), dim3(tl.tiles), dim3(a.block_x, a.block_y), 0, a.stream,
                           a.p, static_cast<const T*>(a.src), cst, a.pull, tl, static_cast<double*>(a.out_xi),
                           static_cast<double*>(a.out_J), static_cast<double*>(a.out_grad));
      else
        hipLaunchKernelGGL((k_read<LAT, M, T, float>), dim3(tl.tiles), dim3(a.block_x, a.block_y), 0, a.stream,
                           a.p, static_cast<const T*>(a.src), cst, a.pull, tl, static_cast<float*>(a.out_xi),
                           static_cast<float*>(a.out_J), static_cast<float*>(a.out_grad));
      break;
    }
    case Op::DiagPartial:
      hipLaunchKernelGGL((k_diag_partial<LAT, M, T>), dim3(a.diag_blocks), dim3(kDiagThreads), 0, a.stream, a.p,
                         static_cast<const T*>(a.src), cst, a.pull, a.partials);
      break;
    case Op::DiagFinal:
      hipLaunchKernelGGL(k_diag_final<LAT>, dim3(1), dim3(kDiagThreads), 0, a.stream, a.partials, a.diag_blocks,
                         M + 1, a.diag_out);
      break;
    case Op::AdjointSeed: {
      const Tiling tl = make_tiling(a);
      hipLaunchKernelGGL((k_adjoint_seed<LAT, M, T>), dim3(tl.tiles), dim3(a.block_x, a.block_y), 0, a.stream, a.p,
                         static_cast<const double*>(a.xi0), static_cast<T*>(a.dst), a.pull, tl);
      break;
    }
    case Op::AdjointStep: {
      const Tiling tl = make_tiling(a, kAdjointNodesPerThread);
      const bool a32 = (uint64_t)a.p.plane * sizeof(T) < (1ull << 32);
      const dim3 grid(tl.tiles), block(a.block_x, a.block_y);
      const T* sp = static_cast<const T*>(a.src);
      const T* ain = static_cast<const T*>(a.adj_in);
      T* aout = static_cast<T*>(a.dst);
      if (a.p.dilute) {
        if (a32)
          hipLaunchKernelGGL((k_adjoint_step<LAT, M, T, true, true>), grid, block, 0, a.stream, a.p, sp, ain, aout,
                             cst, a.pull, tl, a.partials);
        else
          hipLaunchKernelGGL((k_adjoint_step<LAT, M, T, false, true>), grid, block, 0, a.stream, a.p, sp, ain, aout,
                             cst, a.pull, tl, a.partials);
      } else {
        if (a32)
          hipLaunchKernelGGL((k_adjoint_step<LAT, M, T, true>), grid, block, 0, a.stream, a.p, sp, ain, aout, cst,
                             a.pull, tl, a.partials);
        else
          hipLaunchKernelGGL((k_adjoint_step<LAT, M, T, false>), grid, block, 0, a.stream, a.p, sp, ain, aout, cst,
                             a.pull, tl, a.partials);
      }
      break;
    }
    case Op::AdjointXi0: {
      const Tiling tl = make_tiling(a);
      hipLaunchKernelGGL((k_adjoint_xi0<LAT, M, T>), dim3(tl.tiles), dim3(a.block_x, a.block_y), 0, a.stream, a.p,
                         static_cast<const T*>(a.adj_in), static_cast<double*>(a.out_xi), tl);
      break;
    }
    case Op::AdjointDD: {
      const Tiling tl = make_tiling(a, kAdjointNodesPerThread);
      const uint32_t slots = a.accum_slots > 0 ? (uint32_t)a.accum_slots : tl.tiles;
      hipLaunchKernelGGL((k_adjoint_dD<LAT, M>), dim3(1), dim3(64), 0, a.stream, a.p, a.partials, slots,
                         a.diag_out);
      break;
    }
    case Op::FillZero:
      hipLaunchKernelGGL(k_fill_zero<LAT>, dim3(256), dim3(256), 0, a.stream, a.partials, a.fill_count);
      break;
    case Op::StepBlocked:
      if constexpr (LAT == 2 || LAT == 5) {
        const hipError_t e = launch_blocked<M, T, LAT>(a);
        if (e != hipSuccess) return e;
      } else {
        return hipErrorInvalidValue;
      }
      break;
    case Op::BlockedResident:
      if constexpr (LAT == 2 || LAT == 5) {
        hipError_t e = hipErrorInvalidValue;
        if (a.tb == 2) e = blocked_resident<M, T, 2, LAT>(a, a.out_int);
        if (a.tb == 3) e = blocked_resident<M, T, 3, LAT>(a, a.out_int);
        if (a.tb == 4) e = blocked_resident<M, T, 4, LAT>(a, a.out_int);
        if (a.tb == 5) e = blocked_resident<M, T, 5, LAT>(a, a.out_int);
        if (a.tb == 6) e = blocked_resident<M, T, 6, LAT>(a, a.out_int);
        return e;
      } else {
        return hipErrorInvalidValue;
      }
    case Op::StepBlocked3d:
      if constexpr ((LAT == 3 || LAT == 6) && M <= 3 && sizeof(T) == 4) {
        const hipError_t e = launch_blocked3d<LAT, M, T>(a);
        if (e != hipSuccess) return e;
      } else {
        return hipErrorInvalidValue;
      }
      break;
    case Op::AdjointBlocked:
      if constexpr (LAT == 2) {
        const hipError_t e = launch_adjoint_blocked<M, T>(a);
        if (e != hipSuccess) return e;
      } else {
        return hipErrorInvalidValue;
      }
      break;
    case Op::BatchStepBlocked:
      if constexpr (LAT == 2) {
        const hipError_t e = launch_batch_blocked<M, T>(a);
        if (e != hipSuccess) return e;
      } else {
        return hipErrorInvalidValue;
      }
      break;
    case Op::BatchStep:
      // here M is the largest number of evolved species in the launch
      if (a.ntiles == 0) break;
      if (a.dilute)
        hipLaunchKernelGGL((k_batch_step<LAT, M, T, true>), dim3(a.ntiles), dim3(a.block_x, a.block_y), 0, a.stream,
                           a.insts, a.tiles, a.tile_begin, a.ntiles, a.ws, a.cur, a.pull, a.xcd_remap,
                           a.nontemporal);
      else
        hipLaunchKernelGGL((k_batch_step<LAT, M, T>), dim3(a.ntiles), dim3(a.block_x, a.block_y), 0, a.stream,
                           a.insts, a.tiles, a.tile_begin, a.ntiles, a.ws, a.cur, a.pull, a.xcd_remap,
                           a.nontemporal);
      break;
  }
  return hipGetLastError();
}

template <int LAT, int M>
hipError_t run_prec(Op op, const LaunchArgs& a) {
  return a.prec == 8 ? run<LAT, M, double>(op, a) : run<LAT, M, float>(op, a);
}

template <int LAT>
hipError_t dispatch(Op op, const LaunchArgs& a) {
  switch (a.m) {
    case 1: return run_prec<LAT, 1>(op, a);
    case 2: return run_prec<LAT, 2>(op, a);
    case 3: return run_prec<LAT, 3>(op, a);
    case 4: return run_prec<LAT, 4>(op, a);
    case 5: return run_prec<LAT, 5>(op, a);
    case 6: return run_prec<LAT, 6>(op, a);
    case 7: return run_prec<LAT, 7>(op, a);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace msd
