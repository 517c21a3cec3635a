// Device building blocks of the Maxwell-Stefan MRT lattice Boltzmann sweep.
//
// Per node the sweep needs, for the m = N-1 evolved species:
//   xi_i = sum_k f_k^i                                     (Eq. (3-15))
//   B(xi)                                                  (Eq. (2-10))
//   K = (I + (a/2) B)^-1,  a = cs2 dt                      (see below)
//   Lambda_1 = 2 (I - K)                                   (Eq. (3-26) with D~ = B^-1)
//   Lambda_2 = Lambda_1 with the diagonal of Eq. (3-16)
//   relaxation of Eq. (3-13a) and the back-transform.
//
// Two algebraic rewrites make this cheap and exact up to rounding:
// (1) Eq. (3-26) gives Lambda_1 = (D~/a + I/2)^-1 = a (I + (a/2) B)^-1 B
//     = 2 (I - K): one small inverse per node instead of two.
// (2) On D1Q3, D2Q5 and D3Q7 every moment row is either odd or even under
//     k -> opposite(k), first-order rows are exactly the odd ones, and the
//     conserved row has m - m^eq = 0.  The moment-space relaxation
//     M^-1 Lambda M (f - f^eq) therefore equals
//         Lambda_1 odd(f - f^eq) + Lambda_2 even(f - f^eq)
//     with odd/even the antisymmetric/symmetric parts over opposite pairs,
//     whatever moment matrix is used.  With Lambda_2 = Lambda_1 + diag(delta):
//         f^+_k = f_k - Lambda_1 (f_k - w_k xi) - delta * even_k.
// The flux follows the same way: with grad xi = -(1/a) Lambda_1 m1
// (Eq. (3-27)) and J = -c_t D~ grad xi (Eq. (2-12)), J = c_t K m1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msd {

constexpr int kMaxSpecies = 8;
constexpr int BC_PERIODIC = 0, BC_ZERO_FLUX = 1, BC_DIRICHLET = 2;

// ---------------------------------------------------------------------------
// Lattices (Sec. 3.1).  c(k, a) is component a of direction k.  On the
// lattices without diagonal directions (diag = false) direction k moves along
// axis(k) by sgn(k) (axis -1 for rest), which the row-marching kernels use.
// ---------------------------------------------------------------------------
template <int LAT> struct Lattice;

#define MSD_AXIAL_COMPONENTS                                                                   \
  static constexpr bool diag = false;                                                           \
  __host__ __device__ static constexpr int c(int k, int a) { return axis(k) == a ? sgn(k) : 0; }

// Eq. (3-5): c = (0, 1, -1), w = (2/3, 1/6, 1/6).
template <> struct Lattice<1> {
  static constexpr int D = 1, Q = 3;
  __host__ __device__ static constexpr int axis(int k) { return k == 0 ? -1 : 0; }
  __host__ __device__ static constexpr int sgn(int k) { return k == 0 ? 0 : (k == 1 ? 1 : -1); }
  __host__ __device__ static constexpr int opp(int k) { return k == 0 ? 0 : 3 - k; }
  __host__ __device__ static constexpr double w(int k) { return k == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
  static constexpr double cs2 = 1.0 / 3.0;
  MSD_AXIAL_COMPONENTS
};

// Eq. (3-7): directions (0,0), (1,0), (0,1), (-1,0), (0,-1); w = (1/3, 1/6 x4).
template <> struct Lattice<2> {
  static constexpr int D = 2, Q = 5;
  __host__ __device__ static constexpr int axis(int k) { return k == 0 ? -1 : ((k - 1) & 1); }
  __host__ __device__ static constexpr int sgn(int k) { return k == 0 ? 0 : (k <= 2 ? 1 : -1); }
  __host__ __device__ static constexpr int opp(int k) { return k == 0 ? 0 : (k <= 2 ? k + 2 : k - 2); }
  __host__ __device__ static constexpr double w(int k) { return k == 0 ? 1.0 / 3.0 : 1.0 / 6.0; }
  static constexpr double cs2 = 1.0 / 3.0;
  MSD_AXIAL_COMPONENTS
};

// Eq. (3-10): directions 0, +x, -x, +y, -y, +z, -z; w = (1/4, 1/8 x6).
// Its second moment is sum_k w_k c_kx^2 = 1/4, which replaces the D2Q5 factor
// c^2/3 of Eqs. (3-22), (3-26) and (3-27).
template <> struct Lattice<3> {
  static constexpr int D = 3, Q = 7;
  __host__ __device__ static constexpr int axis(int k) { return k == 0 ? -1 : (k - 1) / 2; }
  __host__ __device__ static constexpr int sgn(int k) { return k == 0 ? 0 : ((k & 1) ? 1 : -1); }
  __host__ __device__ static constexpr int opp(int k) { return k == 0 ? 0 : ((k & 1) ? k + 1 : k - 1); }
  __host__ __device__ static constexpr double w(int k) { return k == 0 ? 0.25 : 0.125; }
  static constexpr double cs2 = 0.25;
  MSD_AXIAL_COMPONENTS
};

// Lattices without a rest direction (q = 2d, equal weights 1/(2d)); their
// second moments sum_k w_k c_kx^2 are 1 (D1Q2), 1/2 (D2Q4) and 1/3 (D3Q6).
// Lattice ids 4, 5, 6 follow the ABI's enum.
// Eq. (3-4): c = (1, -1), w = 1/2.
template <> struct Lattice<4> {
  static constexpr int D = 1, Q = 2;
  __host__ __device__ static constexpr int axis(int) { return 0; }
  __host__ __device__ static constexpr int sgn(int k) { return k == 0 ? 1 : -1; }
  __host__ __device__ static constexpr int opp(int k) { return 1 - k; }
  __host__ __device__ static constexpr double w(int) { return 0.5; }
  static constexpr double cs2 = 1.0;
  MSD_AXIAL_COMPONENTS
};

// Eq. (3-6): directions (1,0), (0,1), (-1,0), (0,-1); w = 1/4.
template <> struct Lattice<5> {
  static constexpr int D = 2, Q = 4;
  __host__ __device__ static constexpr int axis(int k) { return k & 1; }
  __host__ __device__ static constexpr int sgn(int k) { return k < 2 ? 1 : -1; }
  __host__ __device__ static constexpr int opp(int k) { return (k + 2) & 3; }
  __host__ __device__ static constexpr double w(int) { return 0.25; }
  static constexpr double cs2 = 0.5;
  MSD_AXIAL_COMPONENTS
};

// Eq. (3-9): directions +x, -x, +y, -y, +z, -z; w = 1/6.
template <> struct Lattice<6> {
  static constexpr int D = 3, Q = 6;
  __host__ __device__ static constexpr int axis(int k) { return k >> 1; }
  __host__ __device__ static constexpr int sgn(int k) { return (k & 1) ? -1 : 1; }
  __host__ __device__ static constexpr int opp(int k) { return k ^ 1; }
  __host__ __device__ static constexpr double w(int) { return 1.0 / 6.0; }
  static constexpr double cs2 = 1.0 / 3.0;
  MSD_AXIAL_COMPONENTS
};

#undef MSD_AXIAL_COMPONENTS

// Component of a diagonal direction from a bit mask: bit k set -> +1, else -1.
__host__ __device__ constexpr int sign_bit(unsigned mask, int k) { return ((mask >> k) & 1u) ? 1 : -1; }

// Eq. (3-8): directions (0,0), (1,0), (0,1), (-1,0), (0,-1), (1,1), (-1,1),
// (-1,-1), (1,-1); w = (4/9, 1/9 x4, 1/36 x4); second moment 1/3.
template <> struct Lattice<7> {
  static constexpr int D = 2, Q = 9;
  static constexpr bool diag = true;
  __host__ __device__ static constexpr int c(int k, int a) {
    return (k == 0 || a > 1) ? 0
                             : (k <= 4 ? (((k - 1) & 1) == a ? (k <= 2 ? 1 : -1) : 0)
                                       : sign_bit(a == 0 ? 0x120u : 0x060u, k));   // +x: 5, 8; +y: 5, 6
  }
  __host__ __device__ static constexpr int opp(int k) {
    return k == 0 ? 0 : (k <= 4 ? (k <= 2 ? k + 2 : k - 2) : ((k - 3) & 3) + 5);
  }
  __host__ __device__ static constexpr double w(int k) {
    return k == 0 ? 4.0 / 9.0 : (k <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  static constexpr double cs2 = 1.0 / 3.0;
};

// Eq. (3-11): directions 0, +x, -x, +y, -y, +z, -z, then (1,1,1), (1,-1,-1),
// (1,-1,1), (1,1,-1), (-1,1,1), (-1,-1,-1), (-1,-1,1), (-1,1,-1);
// w = (2/9, 1/9 x6, 1/72 x8); second moment 1/3.
template <> struct Lattice<8> {
  static constexpr int D = 3, Q = 15;
  static constexpr bool diag = true;
  __host__ __device__ static constexpr int c(int k, int a) {
    return k == 0 ? 0
                  : (k <= 6 ? ((k - 1) / 2 == a ? ((k & 1) ? 1 : -1) : 0)
                            : sign_bit(a == 0 ? 0x0780u : (a == 1 ? 0x4C80u : 0x2A80u), k));
  }
  __host__ __device__ static constexpr int opp(int k) {
    return k == 0 ? 0
                  : (k <= 6 ? ((k & 1) ? k + 1 : k - 1)
                            : ((k == 7 || k == 8 || k == 11 || k == 12) ? 19 - k : 23 - k));
  }
  __host__ __device__ static constexpr double w(int k) {
    return k == 0 ? 2.0 / 9.0 : (k <= 6 ? 1.0 / 9.0 : 1.0 / 72.0);
  }
  static constexpr double cs2 = 1.0 / 3.0;
};

// Compile-time checks of every table: opposite directions are negatives with
// equal weights, the weights sum to 1, first moments vanish, the second moment
// is isotropic with value cs2 and the mixed second moments vanish.
template <int LAT>
constexpr bool lattice_consistent() {
  using L = Lattice<LAT>;
  double ws = 0.0;
  for (int k = 0; k < L::Q; ++k) {
    ws += L::w(k);
    if (L::opp(L::opp(k)) != k || L::w(L::opp(k)) != L::w(k)) return false;
    for (int a = 0; a < 3; ++a)
      if (L::c(L::opp(k), a) != -L::c(k, a) || (a >= L::D && L::c(k, a) != 0)) return false;
  }
  if ((ws - 1.0) * (ws - 1.0) > 1e-28) return false;
  for (int a = 0; a < L::D; ++a)
    for (int b = 0; b < L::D; ++b) {
      double m1 = 0.0, m2 = 0.0;
      for (int k = 0; k < L::Q; ++k) {
        m1 += L::w(k) * L::c(k, a);
        m2 += L::w(k) * L::c(k, a) * L::c(k, b);
      }
      const double want = a == b ? L::cs2 : 0.0;
      if (m1 * m1 > 1e-28 || (m2 - want) * (m2 - want) > 1e-28) return false;
    }
  return true;
}
static_assert(lattice_consistent<1>() && lattice_consistent<2>() && lattice_consistent<3>() &&
                  lattice_consistent<4>() && lattice_consistent<5>() && lattice_consistent<6>() &&
                  lattice_consistent<7>() && lattice_consistent<8>(),
              "lattice tables");

// ---------------------------------------------------------------------------
// Kernel parameters (passed by value in the kernel argument segment).
// Host arrays of the problem are copied in verbatim; every derived quantity
// (1/D_ij, relaxation matrices, ...) is computed on the device.
// ---------------------------------------------------------------------------
struct Problem {
  int32_t nx, ny, nz;
  int32_t relax;          // 0 paper rule (Eq. (3-16)), 1 SRT, 2 TRT
  int32_t linearized;     // 1: B at xi_ref
  int32_t dilute;         // 1: B of the dilute-species approximation (diagonal)
  int32_t bc[6];          // x_lo, x_hi, y_lo, y_hi, z_lo, z_hi
  int64_t plane;          // elements between consecutive planes of a buffer
  double c_t;
  double D[kMaxSpecies][kMaxSpecies];
  double wall[6][kMaxSpecies];
  double xi_ref[kMaxSpecies];
  double magic;           // TRT: (1/lambda_1 - 1/2)(1/lambda_2 - 1/2) per species
};

// 1/x.  FP32: the hardware reciprocal, within 1 ulp of the quotient (an IEEE
// FP32 division costs about ten instructions); FP64: the IEEE quotient.
template <typename T>
__device__ __forceinline__ T recip(T x) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_amdgcn_rcpf(x);
  } else {
    return T(1) / x;
  }
}

// ---------------------------------------------------------------------------
// Small dense inverse of A = I + (a/2) B, times `scale`.  The eigenvalues of B are real and
// positive for compositions on the simplex, so A is never singular; its
// off-diagonal entries can exceed the diagonal, hence the pivoting for m >= 5
// (closed forms by cofactors for m <= 4).
// ---------------------------------------------------------------------------
template <int M, typename T>
__device__ __forceinline__ void invert_small(T (&A)[M][M], T (&K)[M][M], T scale = T(1)) {
  if constexpr (M == 1) {
    K[0][0] = scale * recip(A[0][0]);
  } else if constexpr (M == 2) {
    const T inv = scale * recip(A[0][0] * A[1][1] - A[0][1] * A[1][0]);
    K[0][0] = A[1][1] * inv;
    K[0][1] = -A[0][1] * inv;
    K[1][0] = -A[1][0] * inv;
    K[1][1] = A[0][0] * inv;
  } else if constexpr (M == 3) {
    const T c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    const T c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    const T c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    const T inv = scale * recip(A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02);
    K[0][0] = c00 * inv;
    K[1][0] = c01 * inv;
    K[2][0] = c02 * inv;
    K[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * inv;
    K[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * inv;
    K[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * inv;
    K[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * inv;
    K[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * inv;
    K[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * inv;
  } else if constexpr (M == 4) {
    // Cofactors from the 2 x 2 minors of rows 0-1 (s) and rows 2-3 (c): the
    // Laplace expansion by complementary minors gives det = sum +-s c, and
    // each adjugate entry is three products of an entry with a minor.
    const T(&a)[4][4] = A;
    const T s0 = a[0][0] * a[1][1] - a[1][0] * a[0][1], s1 = a[0][0] * a[1][2] - a[1][0] * a[0][2];
    const T s2 = a[0][0] * a[1][3] - a[1][0] * a[0][3], s3 = a[0][1] * a[1][2] - a[1][1] * a[0][2];
    const T s4 = a[0][1] * a[1][3] - a[1][1] * a[0][3], s5 = a[0][2] * a[1][3] - a[1][2] * a[0][3];
    const T c5 = a[2][2] * a[3][3] - a[3][2] * a[2][3], c4 = a[2][1] * a[3][3] - a[3][1] * a[2][3];
    const T c3 = a[2][1] * a[3][2] - a[3][1] * a[2][2], c2 = a[2][0] * a[3][3] - a[3][0] * a[2][3];
    const T c1 = a[2][0] * a[3][2] - a[3][0] * a[2][2], c0 = a[2][0] * a[3][1] - a[3][0] * a[2][1];
    const T inv = scale * recip(s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0);
    K[0][0] = (a[1][1] * c5 - a[1][2] * c4 + a[1][3] * c3) * inv;
    K[0][1] = (a[0][2] * c4 - a[0][1] * c5 - a[0][3] * c3) * inv;
    K[0][2] = (a[3][1] * s5 - a[3][2] * s4 + a[3][3] * s3) * inv;
    K[0][3] = (a[2][2] * s4 - a[2][1] * s5 - a[2][3] * s3) * inv;
    K[1][0] = (a[1][2] * c2 - a[1][0] * c5 - a[1][3] * c1) * inv;
    K[1][1] = (a[0][0] * c5 - a[0][2] * c2 + a[0][3] * c1) * inv;
    K[1][2] = (a[3][2] * s2 - a[3][0] * s5 - a[3][3] * s1) * inv;
    K[1][3] = (a[2][0] * s5 - a[2][2] * s2 + a[2][3] * s1) * inv;
    K[2][0] = (a[1][0] * c4 - a[1][1] * c2 + a[1][3] * c0) * inv;
    K[2][1] = (a[0][1] * c2 - a[0][0] * c4 - a[0][3] * c0) * inv;
    K[2][2] = (a[3][0] * s4 - a[3][1] * s2 + a[3][3] * s0) * inv;
    K[2][3] = (a[2][1] * s2 - a[2][0] * s4 - a[2][3] * s0) * inv;
    K[3][0] = (a[1][1] * c1 - a[1][0] * c3 - a[1][2] * c0) * inv;
    K[3][1] = (a[0][0] * c3 - a[0][1] * c1 + a[0][2] * c0) * inv;
    K[3][2] = (a[3][1] * s1 - a[3][0] * s3 - a[3][2] * s0) * inv;
    K[3][3] = (a[2][0] * s3 - a[2][1] * s1 + a[2][2] * s0) * inv;
  } else {
    // Gauss-Jordan on [A | I] with partial pivoting; row swaps are done with
    // selects so that every index stays compile-time (registers only).
    T W[M][2 * M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
#pragma unroll
      for (int j = 0; j < M; ++j) {
        W[i][j] = A[i][j];
        W[i][M + j] = (i == j) ? scale : T(0);
      }
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
#pragma unroll
      for (int r = c + 1; r < M; ++r) {
        const bool sw = fabs(W[r][c]) > fabs(W[c][c]);
#pragma unroll
        for (int j = 0; j < 2 * M; ++j) {
          const T a = W[c][j], b = W[r][j];
          W[c][j] = sw ? b : a;
          W[r][j] = sw ? a : b;
        }
      }
      const T inv = recip(W[c][c]);
#pragma unroll
      for (int j = 0; j < 2 * M; ++j) W[c][j] *= inv;
#pragma unroll
      for (int r = 0; r < M; ++r) {
        if (r == c) continue;
        const T fac = W[r][c];
#pragma unroll
        for (int j = 0; j < 2 * M; ++j) W[r][j] -= fac * W[c][j];
      }
    }
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int j = 0; j < M; ++j) K[i][j] = W[i][M + j];
  }
}

// K = (I + (a/2) B(xb))^-1 with B of Eq. (2-10) at composition xb (m values;
// the eliminated species is 1 - sum).  With xi_N = 1 - sum_{k<N} xi_k,
//   B_ii = R_iN + sum_{k != i, k < N} xi_k (R_ik - R_iN),  B_ij = -xi_i (R_ij - R_iN)
// where R = 1/D (sigma_ij of Eq. (2-6)).
template <int M, typename T>
__device__ __forceinline__ void ms_inverse(const T (&xb)[M], const T (&R)[M][M + 1], T half_a,
                                           T (&K)[M][M]) {
  T A[M][M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T diag = R[i][M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      if (k == i) continue;
      const T s = R[i][k] - R[i][M];
      diag += xb[k] * s;
      A[i][k] = -half_a * xb[i] * s;
    }
    A[i][i] = T(1) + half_a * diag;
  }
  invert_small<M, T>(A, K);
}

// K = A^-1 of the dilute-species approximation: diagonal, A_ii = 1 + (a/2)
// (sum_{k != i, k < N} xb_k R_ik + xb_N R_iN) with xb_N = 1 - sum_k xb_k.
template <int M, typename T>
__device__ __forceinline__ void ms_inverse_dilute(const T (&xb)[M], const T (&R)[M][M + 1], T half_a,
                                                  T (&K)[M][M]) {
  T xN = T(1);
#pragma unroll
  for (int k = 0; k < M; ++k) xN -= xb[k];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T b = xN * R[i][M];
#pragma unroll
    for (int k = 0; k < M; ++k)
      if (k != i) b += xb[k] * R[i][k];
#pragma unroll
    for (int j = 0; j < M; ++j) K[i][j] = T(0);
    K[i][i] = T(1) / (T(1) + half_a * b);
  }
}

// Fused multiply-add in the sweep's precision.
__device__ __forceinline__ float mad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double mad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Per-problem collision coefficients (uniform values, computed once by the
// setup kernel).  A = I + (a/2) B(xb) of Eq. (2-10) is affine in the
// composition:
//   A_ii = a0_i + sum_{k != i} xi_k da_ik,   A_ik = xi_i ea_ik + ga_ik   (k != i)
// with da_ik = (a/2)(R_ik - R_iN) = -ea_ik, ga_ik = 0, a0_i = 1 + (a/2) R_iN;
// the linearised mode freezes A at xi_ref (da = ea = 0, a0 and ga hold
// A(xi_ref)).  The dilute-species approximation (Eqs. (2-16), (2-17)) makes A
// diagonal, A_ii = 1 + (a/2) sum_{k != i, k <= N} xi_k R_ik; with xi_N
// eliminated that is a0_i + sum_{k != i} xi_k da_ik + xi_i ds_i, ds_i =
// -(a/2) R_iN (collide_node with DIL = true).  rule[] switches the relaxation rule without a branch: with
// sigma = 1 for Eq. (3-16) and TRT and 0 for SRT, and the TRT parameter
// magic (3/16 for Eq. (3-16)), it holds (sigma, sigma/2, -sigma, 1 - sigma/2,
// sigma - 2, 1 - 4 magic, 8 magic) (SRT: 0 and 1 for the last two; see
// collide_node).
template <int M, typename T>
struct CollideCoef {
  T a0[M];
  T ds[M];          // dilute mode only: coefficient of xi_i in A_ii
  T da[M][M];
  T ea[M][M];
  T ga[M][M];
  T rule[7];
};

// Collision of one node in place: f[i][k] <- f^+ (Eq. (3-13a) + back-transform).
//
// With K2 = 2 A^-1, Lambda_1 = 2 (I - K) = 2I - K2.  The even parameter of
// species i from the product rule (1/lambda_1 - 1/2)(1/lambda_2 - 1/2) = magic
// (Eq. (3-16) is magic = 3/16, where lambda_2 = 8 (2 - lambda_1)/(8 - lambda_1)),
// in terms of kd = K2_ii (lambda_1 = 2 - kd):
//   lambda_2 / 2 = kd / (8 magic + (1 - 4 magic) kd),
// so hd = (lambda_2 - lambda_1)/2 = kd / (8 magic + (1 - 4 magic) kd) + kd/2 - 1
// (for 3/16: 4 kd/(6 + kd) + kd/2 - 1).  The denominator stays positive for
// kd in (0, 2) and any magic > 0.
// The relaxation f^+_k = f_k - G neq_k - hd * neq_kbar with G = Lambda_1 +
// diag(hd) (the pair form of Lambda_1 odd + Lambda_2 even) runs as a chain of
// FMAs with nG = -G:  nG_ij = K2_ij (i != j), nG_ii = kd - 2 - hd.
// Direction 0 takes what the others leave of xi: sum_k f^+_k = xi exactly in
// real arithmetic (sum_k neq_k = 0 because sum_k w_k = 1), so the species
// totals change only by unbiased rounding, never by the rounded weights.
//
// DIL = true is the dilute-species approximation: A is diagonal, so K2 = 2 A^-1
// needs one reciprocal per species and the relaxation couples no species.
template <int LAT, int M, typename T, bool DIL = false>
__device__ __forceinline__ void collide_node(T (&f)[M][Lattice<LAT>::Q], const CollideCoef<M, T>& cc) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q;
  T xi[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T s = f[i][0];
#pragma unroll
    for (int k = 1; k < Q; ++k) s += f[i][k];
    xi[i] = s;
  }
  T nG[M][M], nhd[M];
  if constexpr (DIL) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
      T d = mad(xi[i], cc.ds[i], cc.a0[i]);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        if (k == i) continue;
        d = mad(xi[k], cc.da[i][k], d);
        nG[i][k] = T(0);
      }
      nG[i][i] = T(2) * recip(d);
    }
  } else {
    T A[M][M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      T d = cc.a0[i];
#pragma unroll
      for (int k = 0; k < M; ++k) {
        if (k == i) continue;
        d = mad(xi[k], cc.da[i][k], d);
        A[i][k] = mad(xi[i], cc.ea[i][k], cc.ga[i][k]);
      }
      A[i][i] = d;
    }
    invert_small<M, T>(A, nG, T(2));
  }
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const T kd = nG[i][i];
    const T r = recip(mad(kd, cc.rule[5], cc.rule[6]));
    const T t = kd * cc.rule[0];
    const T hd = mad(t, r, mad(kd, cc.rule[1], cc.rule[2]));
    nG[i][i] = mad(-t, r, mad(kd, cc.rule[3], cc.rule[4]));
    nhd[i] = -hd;
  }

  T neq[M][Q];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int k = 0; k < Q; ++k)
      if (k > 0 || L::opp(k) != 0) neq[i][k] = mad(T(-L::w(k)), xi[i], f[i][k]);
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T rest = xi[i];
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      T acc = f[i][k];
#pragma unroll
      for (int j = 0; j < M; ++j)
        if (!DIL || j == i) acc = mad(nG[i][j], neq[j][k], acc);
      acc = mad(nhd[i], neq[i][L::opp(k)], acc);
      f[i][k] = acc;
      rest -= acc;
    }
    f[i][0] = rest;
  }
}

// ---------------------------------------------------------------------------
// Node addressing and pull propagation with the face rules of Sec. 4.
// ---------------------------------------------------------------------------
struct NodePos {
  int32_t c[3];     // coordinates
  int64_t idx;      // linear index (x fastest)
};

template <int LAT>
__device__ __forceinline__ int64_t axis_stride(const Problem& p, int a) {
  return a == 0 ? int64_t(1) : (a == 1 ? int64_t(p.nx) : int64_t(p.nx) * p.ny);
}

__device__ __forceinline__ int32_t extent(const Problem& p, int a) {
  return a == 0 ? p.nx : (a == 1 ? p.ny : p.nz);
}

// Load with an optional non-temporal (streaming) hint.
template <typename T>
__device__ __forceinline__ T ld(const T* p, bool nt) {
  return nt ? __builtin_nontemporal_load(p) : *p;
}

// Bits of the non-temporal mask of a sweep launch.
constexpr int NT_STORE = 1, NT_LOAD_ALIGNED = 2, NT_LOAD_SHIFTED = 4;

// Where direction k of node n reads from on a lattice with diagonal
// directions: the node x - s c_k (s = 1 for propagation, -1 for its transpose),
// wrapped across periodic faces; its linear index goes to `off`.  Returns -1
// for that case, else the wall face (2 axis + side) that decides because
// x - s c_k lies beyond it: among the wall faces crossed, the one of the
// lowest axis (a direction leaving through an edge or corner of the box
// crosses two or three faces).  `kind` receives that face's boundary kind.
// Face numbers are compile-time constants inside the unrolled loop; callers
// select per-face values with wall_value so that no array is indexed at run
// time (which would move the constants to scratch memory).
template <int LAT>
__device__ __forceinline__ int diag_source(const Problem& p, const NodePos& n, int k, int s, int64_t& off,
                                           int& kind) {
  using L = Lattice<LAT>;
  int face = -1;
  kind = BC_PERIODIC;
  off = n.idx;
#pragma unroll
  for (int a = L::D - 1; a >= 0; --a) {
    const int c = s * L::c(k, a);
    if (c == 0) continue;
    const int32_t ext = extent(p, a);
    const int64_t st = axis_stride<LAT>(p, a);
    const bool edge = (c > 0) ? (n.c[a] == 0) : (n.c[a] == ext - 1);
    const int fa = 2 * a + (c > 0 ? 0 : 1);
    if (edge && p.bc[fa] != BC_PERIODIC) {   // lower axes come later and win
      face = fa;
      kind = p.bc[fa];
    }
    off += edge ? (int64_t)c * (ext - 1) * st : -(int64_t)c * st;
  }
  return face;
}

// wall[face][i] for a face number known only at run time, by a chain of
// selects between registers.  The empty asm statements pin each candidate in a
// register; without them the compiler turns the chain back into one indexed
// load, which puts the whole constant block in scratch memory.
template <int LAT, int M, typename T>
__device__ __forceinline__ T wall_value(const T (&wall)[6][M], int face, int i) {
  T v = wall[0][i];
  asm volatile("" : "+v"(v));
#pragma unroll
  for (int f = 1; f < 2 * Lattice<LAT>::D; ++f) {
    T c = wall[f][i];
    asm volatile("" : "+v"(c));
    v = (face == f) ? c : v;
  }
  return v;
}

// f_k^i(x, t) for all i of one direction k: the post-collision value of the
// source node x - c_k, or at a wall face
//   zero flux:  f_kbar^+(x)            (half-way bounce-back)
//   Dirichlet: -f_kbar^+(x) + 2 w_kbar xi_b   (half-way anti-bounce-back)
// `src` is the post-collision buffer; plane(i, k) is at src + (i*Q + k)*plane.
template <int LAT, int M, typename T>
__device__ __forceinline__ void pull_direction(const Problem& p, const T* src, const NodePos& n, int k,
                                               T (&out)[M][Lattice<LAT>::Q], const T (&wall)[6][M], int nt) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q;
  const bool nt_al = (nt & NT_LOAD_ALIGNED) != 0;
  if constexpr (L::diag) {
    int64_t off;
    int kind;
    const int face = diag_source<LAT>(p, n, k, 1, off, kind);
    if (face < 0) {
#pragma unroll
      for (int i = 0; i < M; ++i) out[i][k] = ld(src + (int64_t)(i * Q + k) * p.plane + off, nt_al);
    } else {
      const int kb = L::opp(k);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const T back = ld(src + (int64_t)(i * Q + kb) * p.plane + n.idx, nt_al);
        out[i][k] = (kind == BC_ZERO_FLUX) ? back
                                           : (T(2.0 * L::w(kb)) * wall_value<LAT, M, T>(wall, face, i) - back);
      }
    }
  } else {
    const int a = L::axis(k);
    if (a < 0) {
#pragma unroll
      for (int i = 0; i < M; ++i) out[i][k] = ld(src + (int64_t)(i * Q + k) * p.plane + n.idx, nt_al);
      return;
    }
    const bool nt_sh = (a == 0) ? (nt & NT_LOAD_SHIFTED) != 0 : nt_al;
    const int s = L::sgn(k);
    const int32_t ext = extent(p, a);
    const int64_t st = axis_stride<LAT>(p, a);
    const bool edge = (s > 0) ? (n.c[a] == 0) : (n.c[a] == ext - 1);
    const int face = 2 * a + (s > 0 ? 0 : 1);
    const int kind = edge ? p.bc[face] : BC_PERIODIC;
    if (kind == BC_PERIODIC) {
      const int64_t off = edge ? n.idx + (int64_t)s * (ext - 1) * st : n.idx - (int64_t)s * st;
#pragma unroll
      for (int i = 0; i < M; ++i) out[i][k] = ld(src + (int64_t)(i * Q + k) * p.plane + off, nt_sh);
    } else {
      const int kb = L::opp(k);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const T back = ld(src + (int64_t)(i * Q + kb) * p.plane + n.idx, nt_al);
        out[i][k] = (kind == BC_ZERO_FLUX) ? back : (T(2.0 * L::w(kb)) * wall[face][i] - back);
      }
    }
  }
}

template <int LAT, int M, typename T>
__device__ __forceinline__ void gather_node(const Problem& p, const T* src, const NodePos& n, bool pull,
                                            T (&f)[M][Lattice<LAT>::Q], const T (&wall)[6][M], int nt = 0) {
  constexpr int Q = Lattice<LAT>::Q;
  if (!pull) {
    const bool nt_al = (nt & NT_LOAD_ALIGNED) != 0;
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int k = 0; k < Q; ++k) f[i][k] = ld(src + (int64_t)(i * Q + k) * p.plane + n.idx, nt_al);
    return;
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) pull_direction<LAT, M, T>(p, src, n, k, f, wall, nt);
}

// ---------------------------------------------------------------------------
// Adjoint building blocks.
// ---------------------------------------------------------------------------

// Transpose of the propagation, read as a gather.  The forward pull delivers
// g_k(y) to exactly one pre-collision value: f_k(y + c_k) inside the domain
// (wrapping at periodic faces), or, where y + c_k lies beyond a wall face,
// f_kbar(y) by bounce-back (+1) or anti-bounce-back (-1).  So, with fbar the
// adjoint of the pre-collision values, gbar_k(y) = fbar_k(y + c_k) or
// +-fbar_kbar(y) at such a face.
template <int LAT, int M, typename T>
__device__ __forceinline__ void pull_direction_transposed(const Problem& p, const T* src, const NodePos& n, int k,
                                                          T (&out)[M][Lattice<LAT>::Q]) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q;
  if constexpr (L::diag) {
    int64_t off;
    int kind;
    const int face = diag_source<LAT>(p, n, k, -1, off, kind);
    if (face < 0) {
#pragma unroll
      for (int i = 0; i < M; ++i) out[i][k] = src[(int64_t)(i * Q + k) * p.plane + off];
    } else {
      const int kb = L::opp(k);
      const bool zf = kind == BC_ZERO_FLUX;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const T v = src[(int64_t)(i * Q + kb) * p.plane + n.idx];
        out[i][k] = zf ? v : -v;
      }
    }
  } else {
    const int a = L::axis(k);
    if (a < 0) {
#pragma unroll
      for (int i = 0; i < M; ++i) out[i][k] = src[(int64_t)(i * Q + k) * p.plane + n.idx];
      return;
    }
    const int s = L::sgn(k);
    const int32_t ext = extent(p, a);
    const int64_t st = axis_stride<LAT>(p, a);
    // the face that direction k leaves the domain through
    const bool edge = (s > 0) ? (n.c[a] == ext - 1) : (n.c[a] == 0);
    const int face = 2 * a + (s > 0 ? 1 : 0);
    const int kind = edge ? p.bc[face] : BC_PERIODIC;
    if (kind == BC_PERIODIC) {
      const int64_t off = edge ? n.idx - (int64_t)s * (ext - 1) * st : n.idx + (int64_t)s * st;
#pragma unroll
      for (int i = 0; i < M; ++i) out[i][k] = src[(int64_t)(i * Q + k) * p.plane + off];
    } else {
      const int kb = L::opp(k);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const T v = src[(int64_t)(i * Q + kb) * p.plane + n.idx];
        out[i][k] = (kind == BC_ZERO_FLUX) ? v : -v;
      }
    }
  }
}

// Plane accessor: plane pl of a buffer at base + pl * plane.  With A32 the
// per-lane part of the address is a 32-bit byte offset from the (uniform)
// plane start, which needs plane * sizeof(T) < 2^32.
template <typename T, bool A32>
struct Planes {
  const T* base;
  int64_t plane;
  __device__ __forceinline__ T operator()(int pl, int64_t idx) const {
    if constexpr (A32) {
      const char* b = reinterpret_cast<const char*>(base + (int64_t)pl * plane);
      return *reinterpret_cast<const T*>(b + (uint32_t)idx * (uint32_t)sizeof(T));
    } else {
      return base[(int64_t)pl * plane + idx];
    }
  }
};

// pull_direction / pull_direction_transposed over a plane accessor.
template <int LAT, int M, typename T, bool A32>
__device__ __forceinline__ void pull_dir(const Problem& p, const Planes<T, A32>& src, const NodePos& n, int k,
                                         T (&out)[M][Lattice<LAT>::Q], const T (&wall)[6][M], bool transposed) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q;
  if constexpr (L::diag) {
    int64_t off;
    int kind;
    const int face = diag_source<LAT>(p, n, k, transposed ? -1 : 1, off, kind);
    const int kb = L::opp(k);
    if (face < 0) {
#pragma unroll
      for (int i = 0; i < M; ++i) out[i][k] = src(i * Q + k, off);
    } else if (!transposed) {
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const T back = src(i * Q + kb, n.idx);
        out[i][k] = (kind == BC_ZERO_FLUX) ? back
                                           : (T(2.0 * L::w(kb)) * wall_value<LAT, M, T>(wall, face, i) - back);
      }
    } else {
      const bool zf = kind == BC_ZERO_FLUX;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const T v = src(i * Q + kb, n.idx);
        out[i][k] = zf ? v : -v;
      }
    }
  } else {
    const int a = L::axis(k);
    if (a < 0) {
#pragma unroll
      for (int i = 0; i < M; ++i) out[i][k] = src(i * Q + k, n.idx);
      return;
    }
    const int s = transposed ? -L::sgn(k) : L::sgn(k);   // read from x - s c
    const int32_t ext = extent(p, a);
    const int64_t st = axis_stride<LAT>(p, a);
    const bool edge = (s > 0) ? (n.c[a] == 0) : (n.c[a] == ext - 1);
    const int face = 2 * a + (s > 0 ? 0 : 1);
    const int kind = edge ? p.bc[face] : BC_PERIODIC;
    const int kb = L::opp(k);
    if (kind == BC_PERIODIC) {
      const int64_t off = edge ? n.idx + (int64_t)s * (ext - 1) * st : n.idx - (int64_t)s * st;
#pragma unroll
      for (int i = 0; i < M; ++i) out[i][k] = src(i * Q + k, off);
    } else if (!transposed) {
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const T back = src(i * Q + kb, n.idx);
        out[i][k] = (kind == BC_ZERO_FLUX) ? back : (T(2.0 * L::w(kb)) * wall[face][i] - back);
      }
    } else {
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const T v = src(i * Q + kb, n.idx);
        out[i][k] = (kind == BC_ZERO_FLUX) ? v : -v;
      }
    }
  }
}

// Reverse-mode derivative of collide_node.  Given the pre-collision f of one
// node and u = dL/df^+, returns fbar = dL/df and adds dL/dR (R = 1/D, entry
// [i][j] for i < m, j <= m) into Rbar.  The forward quantities are recomputed
// exactly as collide_node computes them:
//   g = f - Lambda_1 neq - diag(delta) even,  Lambda_1 = 2 (I - K),
//   K = (I + h B)^-1,  delta_i = sigma (phi(Lambda_1_ii) - Lambda_1_ii),
//   phi(l) = 2 (2 - l) / (2 - g1 l)  (the product rule; g1 = 1 - 4 magic, g0 = 8 magic,
//   so phi'(l) = -2 g0 / (2 - g1 l)^2; for magic = 3/16 phi(l) = 8 (l - 2)/(l - 8)),
// with sigma, g1, g0 = rule[0], rule[5], rule[6] of the collision coefficients.
// DIL = true differentiates the dilute-species collision (diagonal B).  The
// dL/dR terms of the node are added into Rbar in its own type RT (the callers
// keep a per-thread sum in the sweep's precision and reduce it in FP64).
template <int LAT, int M, typename T, bool DIL = false, typename RT>
__device__ __forceinline__ void collide_node_adjoint(const T (&f)[M][Lattice<LAT>::Q], const T (&u)[M][Lattice<LAT>::Q],
                                                     const T (&R)[M][M + 1], const T (&xref)[M], bool linearized,
                                                     const CollideCoef<M, T>& cc, T (&fbar)[M][Lattice<LAT>::Q],
                                                     RT (&Rbar)[M][M + 1]) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q;
  const T h = T(0.5 * L::cs2);
  T xi[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T s = f[i][0];
#pragma unroll
    for (int k = 1; k < Q; ++k) s += f[i][k];
    xi[i] = s;
  }
  T xb[M];
#pragma unroll
  for (int i = 0; i < M; ++i) xb[i] = linearized ? xref[i] : xi[i];
  T K[M][M];
  if constexpr (DIL)
    ms_inverse_dilute<M, T>(xb, R, h, K);
  else
    ms_inverse<M, T>(xb, R, h, K);
  T L1[M][M], delta[M], dphi[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
#pragma unroll
    for (int j = 0; j < M; ++j) L1[i][j] = (i == j ? T(2) : T(0)) - T(2) * K[i][j];
    const T l = L1[i][i];
    const T rd = recip(T(2) - cc.rule[5] * l);
    delta[i] = cc.rule[0] * (T(2) * (T(2) - l) * rd - l);
    dphi[i] = cc.rule[0] * (T(-2) * cc.rule[6] * rd * rd - T(1));   // d delta / d lambda
  }
  T neq[M][Q];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T s = T(0);
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      neq[i][k] = f[i][k] - T(L::w(k)) * xi[i];
      s += neq[i][k];
    }
    neq[i][0] = -s;
  }

  // g_ik = f_ik - sum_j L1_ij neq_jk - delta_i ev_ik, with the even part
  // ev_ik = (neq_ik + neq_ikbar)/2 equal on the two directions of a pair
  // (k != kbar) and ev_ik = neq_ik on a direction that is its own opposite:
  // the pair terms of dL/ddelta and of dL/dneq are taken once per pair.
  T nbar[M][Q], L1bar[M][M], dbar[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T d = T(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int kb = L::opp(k);
      if (k == kb)
        d -= u[i][k] * neq[i][k];
      else if (k < kb)
        d -= (u[i][k] + u[i][kb]) * (T(0.5) * (neq[i][k] + neq[i][kb]));
    }
    dbar[i] = d;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < Q; ++k) acc -= u[i][k] * neq[j][k];
      L1bar[i][j] = acc;
    }
  }
#pragma unroll
  for (int j = 0; j < M; ++j)
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      T acc = T(0);
#pragma unroll
      for (int i = 0; i < M; ++i) acc -= L1[i][j] * u[i][k];
      nbar[j][k] = acc;
    }
  // even part: dL/dev_ik = -delta_i u_ik, spread back over the pair
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int kb = L::opp(k);
      if (k == kb) {
        nbar[i][k] -= delta[i] * u[i][k];
      } else if (k < kb) {
        const T e = T(-0.5) * delta[i] * (u[i][k] + u[i][kb]);
        nbar[i][k] += e;
        nbar[i][kb] += e;
      }
    }
#pragma unroll
  for (int i = 0; i < M; ++i) L1bar[i][i] += dbar[i] * dphi[i];

  // neq_ik = f_ik - w_k xi_i
  T xibar[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T s = T(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      fbar[i][k] = u[i][k] + nbar[i][k];
      s -= T(L::w(k)) * nbar[i][k];
    }
    xibar[i] = s;
  }

  // Lambda_1 = 2 (I - K):  Kbar = -2 L1bar;  K = A^-1: Abar = -K^T Kbar K^T;  A = I + h B: Bbar = h Abar
  T Kbar[M][M], tmp[M][M], Bbar[M][M];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) Kbar[i][j] = T(-2) * L1bar[i][j];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < M; ++l) acc += Kbar[i][l] * K[j][l];   // (Kbar K^T)_ij
      tmp[i][j] = acc;
    }
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < M; ++l) acc += K[l][i] * tmp[l][j];    // (K^T tmp)_ij
      Bbar[i][j] = -h * acc;
    }

  if constexpr (DIL) {
    // B_ij = 0 (i != j), B_ii = sum_{k != i, k < N} xb_k R_ik + xb_N R_iN with
    // xb_N = 1 - sum_k xb_k: dB_ii/dxb_k = S_ik (k != i), dB_ii/dxb_i = -R_iN,
    // dB_ii/dR_ik = xb_k, dB_ii/dR_iN = xb_N
    T xN = T(1);
#pragma unroll
    for (int k = 0; k < M; ++k) xN -= xb[k];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const T bb = Bbar[i][i];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        if (j == i) continue;
        if (!linearized) xibar[j] += bb * (R[i][j] - R[i][M]);
        Rbar[i][j] += RT(bb * xb[j]);
      }
      if (!linearized) xibar[i] -= bb * R[i][M];
      Rbar[i][M] += RT(bb * xN);
    }
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int k = 0; k < Q; ++k) fbar[i][k] += xibar[i];
    return;
  }
  // B_ij = -xb_i S_ij (i != j), B_ii = R_iN + sum_{k != i} xb_k S_ik,  S_ik = R_ik - R_iN:
  //   dL/dR_ij = Bbar_ii xb_j - Bbar_ij xb_i = c_ij (j != i),  dL/dR_iN = Bbar_ii - sum_{j != i} c_ij
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T rN = Bbar[i][i];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      if (j == i) continue;
      const T S = R[i][j] - R[i][M];
      if (!linearized) {
        xibar[i] -= Bbar[i][j] * S;            // off-diagonal B_ij
        xibar[j] += Bbar[i][i] * S;            // diagonal B_ii depends on xb_j through S_ij
      }
      const T c = Bbar[i][i] * xb[j] - Bbar[i][j] * xb[i];
      Rbar[i][j] += RT(c);
      rN -= c;
    }
    Rbar[i][M] += RT(rN);
  }
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int k = 0; k < Q; ++k) fbar[i][k] += xibar[i];
}

}  // namespace msd
