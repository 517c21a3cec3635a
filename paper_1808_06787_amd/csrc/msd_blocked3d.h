// Temporally blocked 3D sweep: two time steps per pass over HBM on the axial
// 3D lattices (D3Q7, D3Q6).  Included by msd_kernels.h.
//
// A workgroup owns an output tile of TX x TY nodes in x and y and a segment of
// z-planes [z0, z1).  Its threads form an (TX + 2) x (TY + 2) block: thread
// (cx, cy) holds the column x = x0 - 1 + cx, y = y0 - 1 + cy (wrapped across
// periodic faces) and marches up the planes.  In iteration j the first level
// (time t + 1) computes plane p = z0 - 1 + j straight from the source buffer
// (pull propagation with the face rules of Sec. 4, collision), for the whole
// block, i.e. the tile and a ring of one node; the second level (time t + 2)
// then computes plane p - 1 of the tile from first-level values kept on chip:
//   * the in-plane directions (+-x, +-y) of plane p - 1 from the neighbouring
//     threads, through LDS (two planes in slots chosen by iteration parity);
//   * the rest population and the z-directions from the thread's own column,
//     in registers: the +z population of plane p - 2, the rest population of
//     plane p - 1 and the -z population of plane p (two-slot ring by parity).
// The second level stores the pass's output; the first level's values never
// leave the chip.  One barrier per iteration (at its top) orders every LDS
// write after the reads of the previous occupant of its slot.  The source
// values of plane p + 1 are loaded while the second level of plane p - 1 is
// computed (prefetch by one plane).
//
// Faces: a pull whose source lies beyond a wall takes the node's own opposite
// population (zero flux: as is; Dirichlet: 2 w xi_wall minus it).  First-level
// nodes beyond a wall are not computed (nobody reads them: the face rule at a
// boundary node reads the node itself); periodic faces wrap.  Offsets within a
// plane are 32-bit (the host checks plane bytes < 4 GiB).
#pragma once

namespace msd {

// Axial 3D lattices: direction k moves along axis(k) by sgn(k); the in-plane
// directions get LDS slots 0..3 (+x, -x, +y, -y).
template <int LAT>
__host__ __device__ constexpr int inplane_slot(int k) {
  using L = Lattice<LAT>;
  return L::axis(k) == 0 ? (L::sgn(k) > 0 ? 0 : 1) : (L::axis(k) == 1 ? (L::sgn(k) > 0 ? 2 : 3) : -1);
}

template <int LAT, int M, typename T, bool WALLS>
__global__ __launch_bounds__(blocked3d_max_threads(M)) void k_step_blocked3d(
    Problem p, const T* __restrict__ src, T* __restrict__ dst, const Consts<T>* __restrict__ cst, int TX, int TY,
    uint32_t tiles_x, uint32_t tiles_y, int zseg, int remap) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q;
  static_assert(L::D == 3 && !L::diag, "axial 3D lattices only");
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);

  // Block position (cx, cy) of this thread: the first TX * TY threads hold the
  // tile's own columns row by row, the others the ring around it (bottom and
  // top rows, then the left and right columns), so that the second level (tile
  // columns only) leaves whole waves idle instead of masking lanes.  LDS is
  // indexed by block position, n = cy * EX + cx.
  const int EX = TX + 2, EY = TY + 2;
  const int E1 = EX * EY;
  const int t = (int)threadIdx.x;
  const int inner = TX * TY;
  int cx, cy;
  if (t < inner) {
    cx = 1 + t % TX;
    cy = 1 + t / TX;
  } else {
    const int h = t - inner;
    if (h < EX) {
      cx = h;
      cy = 0;
    } else if (h < 2 * EX) {
      cx = h - EX;
      cy = EY - 1;
    } else if (h < 2 * EX + TY) {
      cx = 0;
      cy = 1 + (h - 2 * EX);
    } else {
      cx = EX - 1;
      cy = 1 + (h - 2 * EX - TY);
    }
  }
  const int n = cy * EX + cx;

  // Tile from the workgroup index; with remap each XCD (workgroups dealt round
  // robin over 8) walks a contiguous range of tiles, x fastest.
  uint32_t tile = blockIdx.x;
  if (remap) {
    const uint32_t ng = gridDim.x, q8 = ng >> 3, r8 = ng & 7u, xcd = tile & 7u;
    tile = xcd * q8 + (xcd < r8 ? xcd : r8) + (tile >> 3);
  }
  const uint32_t bx = tile % tiles_x;
  const uint32_t rest_t = tile / tiles_x;
  const uint32_t by = rest_t % tiles_y;
  const uint32_t bz = rest_t / tiles_y;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int x0 = (int)bx * TX, y0 = (int)by * TY;
  const int z0 = (int)bz * zseg, z1 = min(z0 + zseg, nz);

  const bool px = !WALLS || p.bc[0] == BC_PERIODIC, py = !WALLS || p.bc[2] == BC_PERIODIC;
  const bool pz = !WALLS || p.bc[4] == BC_PERIODIC;
  const int gx = x0 - 1 + cx, gy = y0 - 1 + cy;
  const bool x_in = gx >= 0 && gx < nx, y_in = gy >= 0 && gy < ny;
  const bool col_ok = (x_in || px) && (y_in || py);
  const int xl = x_in ? gx : ((gx % nx) + nx) % nx;
  const int yl = y_in ? gy : ((gy % ny) + ny) % ny;
  const bool inner_t = t < inner;
  const bool out_col = inner_t && x_in && y_in;
  const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
  const uint32_t col = (uint32_t)xl + (uint32_t)nx * (uint32_t)yl;
  // a block whose columns include a node next to an x or y wall (uniform): only
  // there can an in-plane pull need the face rule
  const bool tile_wall = WALLS && ((!px && (x0 - 1 <= 0 || x0 + TX >= nx - 1)) ||
                                   (!py && (y0 - 1 <= 0 || y0 + TY >= ny - 1)));

  // Collision coefficients in registers; the Dirichlet face values are read
  // from the constants block where a face rule needs them (rarely), which keeps
  // registers free for the march.
  CollideCoef<M, T> cc;
  {
    NodeConsts<M, T> nc;
    load_consts<M, T>(cst, nc);
    cc = nc.cc;
  }
  auto wall_at = [&](int face, int i) -> T { return cst->wall[face][i]; };

  // In-plane sources of this column (fixed for the whole march): the source
  // column of each in-plane direction (wrapped across periodic faces), and
  // whether it lies beyond a wall (then the face rule applies).
  int32_t src_col[4];
  bool wall_dir[4];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const int a = L::axis(k), s = L::sgn(k), d = inplane_slot<LAT>(k);
    if (d < 0) continue;
    const int c = a == 0 ? xl : yl, ext = a == 0 ? nx : ny;
    const int face = 2 * a + (s > 0 ? 0 : 1);
    const bool edge = s > 0 ? (c == 0) : (c == ext - 1);
    const bool wall = WALLS && edge && p.bc[face] != BC_PERIODIC;
    const int cs = edge ? (s > 0 ? ext - 1 : 0) : c - s;
    src_col[d] = a == 0 ? cs + nx * yl : xl + nx * cs;
    wall_dir[d] = wall;
  }

  const uint64_t pstride = (uint64_t)p.plane * sizeof(T);
  // First-level loads of plane pl (wrapped); beyond a z wall nothing is loaded.
  // Planes are walked from an opaque scalar base in steps of the plane stride
  // (species-major, direction-minor), each access that base plus the lane's
  // 32-bit offset.  Where a pull may hit a wall (a wall block, or a plane next
  // to a z wall) the plane of the node's own opposite population is chosen per
  // lane instead.
  auto load_plane = [&](int pl, T (&ld)[M][Q]) __attribute__((always_inline)) {
    const bool p_in = pl >= 0 && pl < nz;
    if (!col_ok || !(p_in || pz)) return;
    const int zl = p_in ? pl : ((pl % nz) + nz) % nz;
    const uint32_t own = (uint32_t)zl * nxy + col;
    const bool z_edge = WALLS && !pz && (zl == 0 || zl == nz - 1);
    uint32_t off[Q];
    bool flip[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int a = L::axis(k), s = L::sgn(k), d = inplane_slot<LAT>(k);
      off[k] = own;
      flip[k] = false;
      if (a == 2) {
        const bool edge = s > 0 ? (zl == 0) : (zl == nz - 1);
        const int face = 4 + (s > 0 ? 0 : 1);
        flip[k] = WALLS && edge && p.bc[face] != BC_PERIODIC;
        const int zs = edge ? (s > 0 ? nz - 1 : 0) : zl - s;
        off[k] = flip[k] ? own : (uint32_t)zs * nxy + col;
      } else if (d >= 0) {
        flip[k] = wall_dir[d];
        off[k] = flip[k] ? own : (uint32_t)zl * nxy + (uint32_t)src_col[d];
      }
    }
    uint64_t b = scalar_base(src);
    if (!(tile_wall || z_edge)) {
#pragma unroll
      for (int i = 0; i < M; ++i)
#pragma unroll
        for (int k = 0; k < Q; ++k, b += pstride) ld[i][k] = gload<T>(b, off[k] * (uint32_t)sizeof(T), false);
    } else {
#pragma unroll
      for (int i = 0; i < M; ++i)
#pragma unroll
        for (int k = 0; k < Q; ++k, b += pstride) {
          const int kb = L::opp(k);
          const uint64_t bb = b + (uint64_t)((int64_t)(kb - k) * (int64_t)pstride);
          ld[i][k] = gload<T>(flip[k] ? bb : b, off[k] * (uint32_t)sizeof(T), false);
        }
    }
  };
  // Dirichlet faces: the pulled own opposite population v becomes 2 w xi_wall - v
  auto dirichlet_fix = [&](int pl, T (&f)[M][Q]) __attribute__((always_inline)) {
    if constexpr (WALLS) {
      const int zl = (pl >= 0 && pl < nz) ? pl : ((pl % nz) + nz) % nz;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const int a = L::axis(k), s = L::sgn(k), d = inplane_slot<LAT>(k), kb = L::opp(k);
        if (a < 0) continue;
        const int face = 2 * a + (s > 0 ? 0 : 1);
        bool fix;
        if (a == 2)
          fix = (s > 0 ? (zl == 0) : (zl == nz - 1)) && p.bc[face] == BC_DIRICHLET;
        else
          fix = wall_dir[d] && p.bc[face] == BC_DIRICHLET;
        if (fix) {
#pragma unroll
          for (int i = 0; i < M; ++i) f[i][k] = T(2.0 * L::w(kb)) * wall_at(face, i) - f[i][k];
        }
      }
    }
  };

  // ring[slot][i]: first-level rest, +z and -z populations of the plane a
  // first-level iteration of that parity produced
  constexpr int KZP = 5 - (LAT == 6 ? 1 : 0), KZM = 6 - (LAT == 6 ? 1 : 0);
  static_assert(L::axis(KZP) == 2 && L::sgn(KZP) > 0 && L::axis(KZM) == 2 && L::sgn(KZM) < 0, "z directions");
  constexpr bool REST = L::opp(0) == 0 && L::axis(0) < 0;
  T rs[2][M], zp[2][M], zm[2][M];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int i = 0; i < M; ++i) rs[b][i] = zp[b][i] = zm[b][i] = T(0);
  T ld[M][Q];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int k = 0; k < Q; ++k) ld[i][k] = T(0);

  const int nj = (z1 - z0) + 2;
  auto lds_at = [&](int slot, int d, int i, int th) -> T& { return lds[((slot * 4 + d) * M + i) * E1 + th]; };

  auto iteration = [&](int j, auto parity) __attribute__((always_inline)) {
    constexpr int B = decltype(parity)::value;   // j & 1
    const int pl = z0 - 1 + j;                   // first-level plane
    __syncthreads();
    T f1[M][Q];
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int k = 0; k < Q; ++k) f1[i][k] = ld[i][k];
    const bool pl_ok = col_ok && ((pl >= 0 && pl < nz) || pz);
    if (pl_ok) {
      dirichlet_fix(pl, f1);
      collide_node<LAT, M, T>(f1, cc);
    }
    // the next plane's source values travel while this iteration computes
    if (j + 1 < nj) load_plane(pl + 1, ld);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int d = inplane_slot<LAT>(k);
      if (d < 0) continue;
#pragma unroll
      for (int i = 0; i < M; ++i) lds_at(B, d, i, n) = f1[i][k];
    }
    if (j >= 2 && inner_t) {
      // second level: plane qz = pl - 1 of the tile (inner threads, whose
      // neighbours are all in the block)
      const int qz = pl - 1;
      T f2[M][Q];
      const int tm_x = n - 1, tp_x = n + 1, tm_y = n - EX, tp_y = n + EX;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const int a = L::axis(k), s = L::sgn(k), d = inplane_slot<LAT>(k);
        if (a < 0) {
#pragma unroll
          for (int i = 0; i < M; ++i) f2[i][k] = rs[B ^ 1][i];
        } else if (a == 2) {
          // +z pulls plane qz - 1 (two iterations back), -z pulls plane qz + 1 (this one)
#pragma unroll
          for (int i = 0; i < M; ++i) f2[i][k] = s > 0 ? zp[B][i] : f1[i][k];
          if constexpr (WALLS) {
            const int face = 4 + (s > 0 ? 0 : 1);
            const bool edge = s > 0 ? (qz == 0) : (qz == nz - 1);
            if (edge && p.bc[face] != BC_PERIODIC) {
              const int kb = L::opp(k);
#pragma unroll
              for (int i = 0; i < M; ++i) {
                const T own = s > 0 ? zm[B ^ 1][i] : zp[B ^ 1][i];   // plane qz's own opposite population
                f2[i][k] = p.bc[face] == BC_ZERO_FLUX ? own : T(2.0 * L::w(kb)) * wall_at(face, i) - own;
              }
            }
          }
        } else {
          const int th = a == 0 ? (s > 0 ? tm_x : tp_x) : (s > 0 ? tm_y : tp_y);
#pragma unroll
          for (int i = 0; i < M; ++i) f2[i][k] = lds_at(B ^ 1, d, i, th);
          if constexpr (WALLS) {
            if (wall_dir[d]) {
              const int face = 2 * a + (s > 0 ? 0 : 1);
              const int kb = L::opp(k), db = inplane_slot<LAT>(kb);
#pragma unroll
              for (int i = 0; i < M; ++i) {
                const T own = lds_at(B ^ 1, db, i, n);
                f2[i][k] = p.bc[face] == BC_ZERO_FLUX ? own : T(2.0 * L::w(kb)) * wall_at(face, i) - own;
              }
            }
          }
        }
      }
      collide_node<LAT, M, T>(f2, cc);
      if (out_col) {
        const uint32_t off = ((uint32_t)qz * nxy + col) * (uint32_t)sizeof(T);
        uint64_t b = scalar_base(dst);
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
          for (int k = 0; k < Q; ++k, b += pstride) gstore<T>(b, off, f2[i][k], 0);
      }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
      if constexpr (REST) rs[B][i] = f1[i][0];
      zp[B][i] = f1[i][KZP];
      zm[B][i] = f1[i][KZM];
    }
  };

  load_plane(z0 - 1, ld);
  for (int j = 0; j < nj; j += 2) {
    iteration(j, std::integral_constant<int, 0>{});
    if (j + 1 < nj) iteration(j + 1, std::integral_constant<int, 1>{});
  }
}

// LDS bytes of one workgroup: two plane slots of four in-plane populations of m
// species per thread.
inline size_t blocked3d_lds_bytes(int m, int bytes, int tx, int ty) {
  return (size_t)2 * 4 * m * (size_t)(tx + 2) * (ty + 2) * bytes;
}

template <int LAT, int M, typename T>
hipError_t launch_blocked3d(const LaunchArgs& a) {
  if constexpr (Lattice<LAT>::D != 3 || Lattice<LAT>::diag) {
    return hipErrorInvalidValue;
  } else {
    const int tx = a.tile_x, ty = a.tile_y, zseg = a.seg_rows;
    if (tx < 1 || ty < 1 || zseg < 1 || (tx + 2) * (ty + 2) > blocked3d_max_threads(M)) return hipErrorInvalidValue;
    if (a.p.dilute) return hipErrorInvalidValue;
    const uint32_t tiles_x = (uint32_t)((a.p.nx + tx - 1) / tx), tiles_y = (uint32_t)((a.p.ny + ty - 1) / ty);
    const uint32_t segs = (uint32_t)((a.p.nz + zseg - 1) / zseg);
    const bool walls = a.p.bc[0] != BC_PERIODIC || a.p.bc[2] != BC_PERIODIC || a.p.bc[4] != BC_PERIODIC;
    const size_t shmem = blocked3d_lds_bytes(M, (int)sizeof(T), tx, ty);
    const dim3 grid(tiles_x * tiles_y * segs), block((tx + 2) * (ty + 2));
    const T* src = static_cast<const T*>(a.src);
    T* dst = static_cast<T*>(a.dst);
    const Consts<T>* cst = static_cast<const Consts<T>*>(a.consts);
    if (walls) {
      if (shmem > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step_blocked3d<LAT, M, T, true>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
      }
      hipLaunchKernelGGL((k_step_blocked3d<LAT, M, T, true>), grid, block, shmem, a.stream, a.p, src, dst, cst, tx, ty,
                         tiles_x, tiles_y, zseg, a.xcd_remap);
    } else {
      if (shmem > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step_blocked3d<LAT, M, T, false>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
      }
      hipLaunchKernelGGL((k_step_blocked3d<LAT, M, T, false>), grid, block, shmem, a.stream, a.p, src, dst, cst, tx,
                         ty, tiles_x, tiles_y, zseg, a.xcd_remap);
    }
    return hipSuccess;
  }
}

}  // namespace msd
