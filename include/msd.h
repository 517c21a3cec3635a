/*
 * msd.h - C ABI of the MI355X lattice Boltzmann solver for Maxwell-Stefan
 * diffusion in N-component mixtures.
 *
 * Method: Chai, Guo, Wang & Shi, "Maxwell-Stefan theory based lattice
 * Boltzmann model for diffusion in multicomponent mixtures".  Every quantity
 * crossing this boundary is in lattice units (dx = dt = 1; physical D_ij map
 * to D_ij dt / dx^2, Sec. 3.1 after Eq. (3-11)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Species 1..N of the paper are 0..N-1 here.  Species N-1 (the paper's n)
 *   is the eliminated one (Sec. 2, Eq. (2-8a)); only m = N-1 species carry
 *   distributions (Sec. 3.1, Eq. (3-2)).
 * - Node fields ("planes") are dense arrays of nx*ny*nz values with x fastest,
 *   then y, then z.  A multi-plane buffer holds its planes back to back.
 * - Pointers named d_* are device pointers (HIP device memory on the GPU the
 *   handle was created on); h_* are host pointers.  The library never
 *   allocates device memory: all device storage is a caller-owned workspace.
 * - Work is enqueued on the HIP stream given at creation (a hipStream_t passed
 *   as void*; NULL is the default stream) and is asynchronous unless the
 *   entry point says it synchronises.
 * - Every int-returning call returns MSD_OK (0) or a negative status; a
 *   thread-local description of the last failure is in msd_last_error().
 * - A handle must not be used from two host threads at once.
 */
#ifndef MSD_H
#define MSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define MSD_API __attribute__((visibility("default")))
#else
#define MSD_API
#endif

#define MSD_ABI_VERSION 4
#define MSD_MAX_SPECIES 8

/* Lattices: velocity sets and weights of Sec. 3.1, Eqs. (3-5), (3-7), (3-10),
 * the lattices without a rest direction, Eqs. (3-4), (3-6), (3-9), and the
 * lattices with diagonal directions, Eqs. (3-8) (D2Q9) and (3-11) (D3Q15).  On
 * the last two the odd moments relax with lambda_1 and the even ones with
 * lambda_2; a diagonal direction that leaves the box through an edge or corner
 * takes the rule of the wall face of the lowest axis it crosses (x, then y,
 * then z; periodic faces only wrap). */
enum msd_lattice {
  MSD_D1Q3 = 1, MSD_D2Q5 = 2, MSD_D3Q7 = 3, MSD_D1Q2 = 4, MSD_D2Q4 = 5, MSD_D3Q6 = 6, MSD_D2Q9 = 7, MSD_D3Q15 = 8
};

/* Storage and arithmetic precision of the sweep (bytes per value). */
enum msd_precision { MSD_F32 = 4, MSD_F64 = 8 };

/* Second-order relaxation: MSD_RELAX_PAPER is Eq. (3-16) (lambda_2^ii =
 * 8(lambda_1^ii - 2)/(lambda_1^ii - 8), off-diagonal lambda_2^ij = lambda_1^ij);
 * MSD_RELAX_SRT sets every relaxation parameter to lambda_1 (the single-
 * relaxation-time special case named after Eq. (3-14)); MSD_RELAX_TRT is the
 * two-relaxation-time case named there (odd moments with lambda_1, even ones
 * with lambda_2), lambda_2^ii fixed by (1/lambda_1^ii - 1/2)(1/lambda_2^ii - 1/2)
 * = msd_problem.trt_magic and off-diagonals as in Eq. (3-16), which is the
 * trt_magic = 3/16 case. */
enum msd_relax { MSD_RELAX_PAPER = 0, MSD_RELAX_SRT = 1, MSD_RELAX_TRT = 2 };

/* Face conditions, Sec. 4: half-way bounce-back gives zero flux, half-way
 * anti-bounce-back holds a Dirichlet mole fraction.  Periodic faces come in
 * pairs. */
enum msd_bc { MSD_BC_PERIODIC = 0, MSD_BC_ZERO_FLUX = 1, MSD_BC_DIRICHLET = 2 };

enum msd_status {
  MSD_OK = 0,
  MSD_EINVAL = -1,      /* bad lattice, extents, species count, faces or pointer */
  MSD_EDIFF = -2,       /* D not symmetric or an off-diagonal D_ij <= 0 (Sec. 2, after Eq. (2-7)) */
  MSD_ECOMP = -3,       /* a composition (wall or reference) off the simplex */
  MSD_ERELAX = -4,      /* unknown relaxation rule, or a TRT parameter that is not > 0 */
  MSD_EHIP = -5,        /* a HIP runtime call failed; msd_last_error() has its text */
  MSD_EDIVERGED = -6,   /* diagnostics found non-finite mole fractions */
  MSD_ENOMEM = -7,      /* workspace smaller than msd_workspace_bytes() */
  MSD_EABI = -8,        /* problem.abi != MSD_ABI_VERSION */
  MSD_ESTATE = -9       /* call not valid in the handle's current state */
};

/* The problem as the paper states it: lattice, N, the Maxwell-Stefan
 * diffusivities D_ij, relaxation rule, faces and (optionally) the
 * linearised-theory reference composition.  All host arrays are read during
 * msd_create / msd_workspace_bytes only and stay owned by the caller. */
typedef struct msd_problem {
  int32_t abi;              /* MSD_ABI_VERSION */
  int32_t lattice;          /* enum msd_lattice */
  int32_t n_species;        /* N, 2 .. MSD_MAX_SPECIES */
  int32_t precision;        /* enum msd_precision */
  int64_t nx, ny, nz;       /* extents; unused dimensions must be 1; nx*ny*nz < 2^31 */
  const double* D;          /* N*N row-major, symmetric, D_ij > 0 for i != j; diagonal ignored */
  const double* xi_wall;    /* 6*N row-major face values [x_lo, x_hi, y_lo, y_hi, z_lo, z_hi][N],
                               read for Dirichlet faces only; may be NULL if none */
  const double* xi_ref;     /* N values; used when linearized != 0 */
  double c_t;               /* total molar concentration in J = -c_t D~ grad xi (Eq. (2-12)); > 0 */
  int32_t relax;            /* enum msd_relax */
  int32_t linearized;       /* 0: B(xi) at the local composition (Eq. (2-10));
                               1: B frozen at xi_ref (linearised theory, constant D~) */
  int32_t bc[6];            /* enum msd_bc for faces x_lo, x_hi, y_lo, y_hi, z_lo, z_hi */
  int32_t plane_pad;        /* extra values between consecutive distribution planes: a multiple
                               of 64, >= 0 (0 = planes of the node count rounded up to 64) */
  int32_t dilute;           /* 0: B of Eq. (2-10); 1: the dilute-species approximation of Remark III,
                               Eqs. (2-16), (2-17), for every evolved species: B diagonal with
                               B_ii = sum_{k != i} xi_k / D_ik (each species follows Fick's law with
                               its own composition-dependent D_eff).  With linearized = 1 the
                               diagonal is frozen at xi_ref.  Runs in the single-step and the
                               temporally blocked sweeps, in batches (dilute mixtures in
                               launches of their own) and in the adjoint (single adjoint
                               steps) */
  double trt_magic;         /* MSD_RELAX_TRT only: the product parameter, finite and > 0 */
} msd_problem;

typedef struct msd_sim msd_sim;
typedef struct msd_batch msd_batch;

/* ---------------------------------------------------------------------------
 * Single mixture
 * ------------------------------------------------------------------------- */

/* Bytes of device workspace msd_create needs for this problem (two ping-pong
 * distribution buffers of m*q planes each, padded, plus reduction scratch).
 * Returns 0 and sets *status (if non-NULL) on an invalid problem. */
MSD_API size_t msd_workspace_bytes(const msd_problem* problem, int32_t* status);

/* Validate the problem, lay out the workspace d_ws (>= msd_workspace_bytes,
 * 256-byte aligned, caller-owned, must outlive the handle) and return a host
 * handle in *out.  No kernel is launched.  Errors: EABI, EINVAL, EDIFF, ECOMP,
 * ERELAX, ENOMEM. */
MSD_API int msd_create(const msd_problem* problem, void* d_ws, size_t ws_bytes, void* stream, msd_sim** out);

/* Replace the stream used by later calls. */
MSD_API int msd_set_stream(msd_sim* sim, void* stream);

/* Initialise f_k^i(x, 0) = w_k xi_i(x, 0) (Sec. 4, initialisation; Eq. (3-3)) and
 * reset the time to 0.  d_xi0 holds N (or at least N-1) planes in precision
 * xi0_precision (MSD_F32 or MSD_F64); planes beyond N-1 are not read, since
 * xi of the eliminated species follows from Eq. (2-3b). */
MSD_API int msd_init(msd_sim* sim, const void* d_xi0, int32_t xi0_precision);

/* Advance nsteps >= 0 time steps of Eq. (3-13): at every node, collision in
 * moment space with the Maxwell-Stefan relaxation matrices (Eqs. (2-10),
 * (2-11), (3-26), (3-16)) fused with propagation and the face rules of Sec. 4.
 * Asynchronous. */
MSD_API int msd_step(msd_sim* sim, int64_t nsteps);

/* Number of steps taken since msd_init (or the value given to msd_restore). */
MSD_API int64_t msd_time(const msd_sim* sim);

/* Write the observables of the pre-collision state at the current time:
 *   d_xi   : N planes, xi_i = sum_k f_k^i (Eq. (3-15)) and xi_N = 1 - sum (Eq. (2-3b));
 *   d_J    : m*d planes [species][component x,y,z], J = -c_t D~ grad xi (Eq. (2-12)),
 *            or NULL;
 *   d_grad : m*d planes, grad xi from the non-equilibrium first moments
 *            (Eq. (3-27), with the lattice's sound speed squared), or NULL.
 * out_precision (MSD_F32 / MSD_F64) is the element type of all outputs. */
MSD_API int msd_read_moments(msd_sim* sim, int32_t out_precision, void* d_xi, void* d_J, void* d_grad);

/* Conservation diagnostics of the current state, computed on the device with
 * a deterministic two-pass reduction in FP64 and copied to the host (this
 * call synchronises the stream): per-species totals sum_x xi_i (constant for
 * periodic and zero-flux faces, Eq. (2-1)), per-species minimum and maximum
 * (arrays of N; may be NULL) and the number of non-finite mole fractions.
 * Returns MSD_EDIVERGED (outputs filled, msd_last_error names the check) when
 *   - any mole fraction is not finite;
 *   - a mole fraction is below -neg_tol (msd_health; mole fractions of a
 *     converging run stay in [0, 1] up to rounding);
 *   - a species total differs from its value at msd_init by more than
 *     mass_rtol times the node count (checked only when no face is Dirichlet:
 *     periodic and zero-flux faces conserve every total, Eq. (2-1)).  msd_init
 *     records the totals of the initial field; msd_restore keeps them. */
MSD_API int msd_diagnostics(msd_sim* sim, double* h_mass, double* h_min, double* h_max, int64_t* h_nonfinite);

/* Limits of the divergence checks in msd_diagnostics; a negative value turns a
 * check off.  Defaults: neg_tol = 1e-2, mass_rtol = 1e-4. */
typedef struct msd_health {
  double neg_tol;
  double mass_rtol;
} msd_health;
MSD_API int msd_set_health(msd_sim* sim, const msd_health* health);
MSD_API int msd_get_health(const msd_sim* sim, msd_health* health);

/* Linear stability of the relaxation (host computation, no device work).  At
 * each of `count` compositions (N mole fractions each, xi_N taken as 1 - the sum
 * of the first N - 1 as in the sweep; with problem->linearized the composition
 * is ignored and B is taken at xi_ref) this forms B (Eq. (2-10), or the
 * dilute-species B of Remark III), Lambda_1 = 2 (I - (I + (a/2) B)^-1) (Eq. (3-26)
 * with D~ = B^-1) and Lambda_2 (Eq. (3-16), TRT or SRT as the problem says), and
 * returns the spectral radii of I - Lambda_1 and I - Lambda_2 in h_rho[2 c] and
 * h_rho[2 c + 1]: the factors by which one collision scales the odd and the even
 * non-equilibrium moments.  Both below 1 is needed for the relaxation to damp
 * them (eig Lambda in (0, 2) for real eigenvalues); Eq. (3-16) can exceed that
 * at extreme compositions.  Radii come from Gelfand's formula (norms of
 * repeated squares), accurate to far below 1e-6.  Errors: MSD_EINVAL and the
 * problem validation codes. */
MSD_API int msd_relaxation_radius(const msd_problem* problem, const double* h_xi, int32_t count, double* h_rho);

/* The largest radii msd_create found over the compositions it checks: the N
 * pure species, the equimolar mixture, the Dirichlet face compositions and
 * xi_ref (linearised theory).  A value >= 1 warns that the relaxation does not
 * damp every mode there (the handle is still created). */
MSD_API int msd_stability(const msd_sim* sim, double* h_rho1, double* h_rho2);

/* Checkpoint / restart: the state is the m*q planes of distributions of the
 * current buffer; msd_state_bytes is its size.  msd_save copies it (device to
 * device, asynchronous) into d_dst and returns the time in *h_step;
 * msd_restore copies it back and sets the time. */
MSD_API size_t msd_state_bytes(const msd_sim* sim);
MSD_API int msd_save(const msd_sim* sim, void* d_dst, int64_t* h_step);
MSD_API int msd_restore(msd_sim* sim, const void* d_src, int64_t step);

/* Free the host handle (the workspace stays the caller's). */
MSD_API int msd_destroy(msd_sim* sim);

/* ---------------------------------------------------------------------------
 * Reverse mode (adjoint) of the sweep
 *
 * For a scalar loss L of the mole fractions at time T, these calls give
 * dL/dxi(0) (the evolved species' initial fields) and dL/dD_ij.  The forward
 * step t reads the buffer state s_{t-1} (the state after step t-1; s_0 is the
 * initial f(0)) and writes s_t; the pre-collision distributions at time t are
 * f^t = P(s_t) (P the propagation with the face rules of Sec. 4; f^0 = s_0).
 * Adjoint buffers hold a_t = dL/df^t at each node, in the layout and precision
 * of a state (msd_state_bytes).  The adjoint of step t maps a_t to a_{t-1}: it
 * reads a_t through the transposed propagation, recomputes f^{t-1} from
 * s_{t-1}, and applies the transposed collision Jacobian (through B of
 * Eq. (2-10), the local solve, Eq. (3-26) and Eq. (3-16)).  A driver
 * checkpoints states during the forward run (msd_save), recomputes segments
 * with msd_record and walks the adjoint steps backwards.
 * ------------------------------------------------------------------------- */

/* Advance nsteps from the current state and also store the state after each
 * step in consecutive slots of msd_state_bytes bytes at d_stack (slot s holds
 * the state after step time+s+1). */
MSD_API int msd_record(msd_sim* sim, int64_t nsteps, void* d_stack);

/* Bytes of the FP64 accumulator of dL/dD (one slot per workgroup of the
 * current launch configuration, which must stay unchanged through one adjoint
 * pass), and its reset (a fill kernel). */
MSD_API size_t msd_adjoint_accum_bytes(const msd_sim* sim);
MSD_API int msd_adjoint_begin(msd_sim* sim, void* d_accum);

/* a_T from dL/dxi at the current time T: d_dL_dxi holds N FP64 planes (the
 * derivative with respect to every species' mole fraction, the last one
 * included; xi_i = sum_k f_k^i (Eq. (3-15)), xi_N = 1 - sum of the others,
 * Eq. (2-3b)). */
MSD_API int msd_adjoint_seed(msd_sim* sim, const double* d_dL_dxi, void* d_adj_out);

/* One adjoint step for forward step t >= 1: d_state_prev is s_{t-1}, d_adj_in
 * is a_t, d_adj_out receives a_{t-1} (must not alias d_adj_in); dL/dD terms are
 * added into d_accum. */
MSD_API int msd_adjoint_step(msd_sim* sim, int64_t t, const void* d_state_prev, const void* d_adj_in,
                             void* d_adj_out, void* d_accum);

/* The adjoint steps t = t_hi, t_hi - 1, ..., t_lo + 1 of one recomputed
 * segment in one call: the state read by step t is d_state_lo (s_{t_lo}) for
 * t = t_lo + 1 and slot t - t_lo - 2 of d_stack (as written by msd_record from
 * time t_lo) otherwise.  a_{t_hi} is read from d_adj_a; the two adjoint buffers
 * alternate and *h_result_in_b reports where a_{t_lo} ends (0: d_adj_a,
 * 1: d_adj_b). */
MSD_API int msd_adjoint_steps(msd_sim* sim, int64_t t_hi, int64_t t_lo, const void* d_state_lo, const void* d_stack,
                              void* d_adj_a, void* d_adj_b, void* d_accum, int32_t* h_result_in_b);

/* From a_0 and the accumulator: dL/dxi(0) (N-1 FP64 planes, or NULL) and the
 * N x N matrix dL/dD (host, row-major, or NULL; entry (i, j) = (j, i) is the
 * derivative with respect to the symmetric pair D_ij = D_ji, diagonal 0).
 * Synchronises the stream. */
MSD_API int msd_adjoint_finish(msd_sim* sim, const void* d_adj0, const void* d_accum, double* d_dL_dxi0,
                               double* h_dL_dD);

/* One-call reverse mode.  msd_forward_checkpointed advances a handle that
 * msd_init has just initialised (time 0) by nsteps, storing the state at the
 * start of every segment of `every` steps: ceil(nsteps / every) states of
 * msd_state_bytes bytes, segment j's at d_ckpts + j * msd_state_bytes (device
 * memory, caller-owned).  msd_adjoint then takes dL/dxi at time nsteps (N FP64
 * planes, the handle must still be at that time) and returns dL/dxi(0) (N-1
 * FP64 device planes, or NULL) and dL/dD (host N x N, or NULL) as
 * msd_adjoint_finish does, recomputing each segment once (msd_record) and
 * running its adjoint steps backwards (msd_adjoint_steps).  d_scratch
 * (caller-owned, 256-byte aligned, at least msd_adjoint_scratch_bytes for the
 * same `every` and launch configuration) holds the accumulator, two adjoint
 * buffers and the recomputation stack.  The handle's state is left at an
 * intermediate time.  Errors: MSD_EINVAL (NULL, nsteps < 0, every < 1),
 * MSD_ESTATE (not at time 0 / not at time nsteps), MSD_ENOMEM (scratch too
 * small); msd_adjoint_scratch_bytes returns 0 for invalid arguments. */
MSD_API size_t msd_adjoint_scratch_bytes(const msd_sim* sim, int64_t every);
MSD_API int msd_forward_checkpointed(msd_sim* sim, int64_t nsteps, int64_t every, void* d_ckpts);
MSD_API int msd_adjoint(msd_sim* sim, int64_t nsteps, int64_t every, const void* d_ckpts, const double* d_dL_dxi,
                        double* d_dL_dxi0, double* h_dL_dD, void* d_scratch, size_t scratch_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid hipMalloc):
 * msd_adjoint with its scratch (accumulator, adjoint buffers, recomputation
 * stack) in a device array that the library's code object holds, one per GPU
 * the library runs on, MSD_STATIC_SCRATCH_BYTES in size and kept until the
 * process ends.  Arguments and results as msd_adjoint; the caller still passes
 * the checkpoints, dL/dxi and the outputs.  Nothing is allocated: no hipMalloc,
 * hipFree or allocating library routine.  The array's address on the current
 * device is looked up once per device (the handle's device must be current).
 * MSD_ENOMEM when msd_adjoint_scratch_bytes for this handle and `every` exceeds
 * MSD_STATIC_SCRATCH_BYTES (nothing is launched then).  Every call on one GPU
 * shares that GPU's array and leaves its contents behind (the accumulator is
 * cleared by a kernel at the start of each call): calls that overlap on one
 * GPU, from two threads or on two streams, race and give wrong results. */
#define MSD_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
MSD_API int msd_adjoint_noalloc(msd_sim* sim, int64_t nsteps, int64_t every, const void* d_ckpts,
                                const double* d_dL_dxi, double* d_dL_dxi0, double* h_dL_dD);

/* ---------------------------------------------------------------------------
 * Launch tuning of the single-mixture sweep
 * ------------------------------------------------------------------------- */

/* block_x * block_y threads per workgroup (block_x a multiple of 64, product
 * <= 256; 0 = library default); xcd_remap = 1 maps consecutive tiles to one
 * of the eight XCDs so that neighbouring rows share an L2; lds_resident = 1
 * allows the single-workgroup kernel that keeps a small domain in LDS for all
 * steps of one msd_step call (used only when the domain fits). */
typedef struct msd_launch {
  int32_t block_x;
  int32_t block_y;
  int32_t xcd_remap;
  int32_t lds_resident;
  int32_t nontemporal;      /* bit mask of streaming (non-temporal) hints: 1 stores, 2 loads of
                               unshifted and y/z-shifted planes, 4 loads of x-shifted planes */
  int32_t vec;              /* nodes per thread of the vectorised sweep: 1, 2 or 4 (aligned
                               vector accesses; used when nx % vec == 0, else the largest
                               power of two dividing nx); 0 (default) selects the general
                               one-node-per-thread kernel */
  int32_t temporal;         /* at most this many steps per pass over HBM; 0 or 1: one step
                               per pass.  D2Q5 and D2Q4: 2 .. 6 (temporally blocked sweep:
                               each workgroup marches along y with the intermediate time
                               levels of a few rows on chip; the blocked adjoint pass is
                               D2Q5-only).  The library takes the largest count up
                               to this one whose on-chip window fits the species count and
                               precision (FP32 with x and y periodic: m <= 3 up to 6, m = 4
                               up to 5; FP32 with an x or y wall: m <= 2 up to 6, m = 3 up to
                               5, m = 4 up to 3; FP64: m = 1 up to 6, m = 2 up to 3; else one
                               step per pass).
                               D2Q5 FP32 problems with nx >= 6144 use 512-column tiles for
                               full passes (m <= 2 at six steps; m = 3 at five steps when x
                               and y are periodic), all other passes 256-column tiles.
                               D3Q7 and D3Q6: 2 (two steps per pass: each workgroup marches
                               along z over an x-y tile and a ring of one node, the first
                               step's values kept on chip), for FP32 with m <= 3 and the full
                               Maxwell-Stefan collision; any value >= 2 means 2 there.
                               Default 6 for D2Q5 and D2Q4, 2 for D3Q7 and D3Q6, 0 otherwise; values
                               outside 0 .. 6 are MSD_EINVAL */
  int32_t seg_rows;         /* D2Q5 blocked sweep: rows per workgroup; 0 (default):
                               automatic.  Forward: about k * 2 workgroups per CU in all,
                               with k doubling (up to 64) while segments stay at least 128
                               rows tall; the adjoint's blocked passes: about 1.35 times the
                               workgroups the device runs at once.  Segments are at least 8
                               rows, and one step per pass is used when 8-row segments give
                               fewer than 512 workgroups (small domains run faster
                               unblocked).  3D blocked sweep: z-planes per workgroup; 0:
                               automatic (at least 8 planes, about sixteen workgroups per CU
                               in all); one step per pass when 8-plane segments give fewer than
                               512 workgroups.  Negative or above 2^20 is MSD_EINVAL */
  int32_t tile_x;           /* 3D blocked sweep: output tile of tile_x * tile_y nodes per
                               workgroup, which runs (tile_x + 2) * (tile_y + 2) threads: at
                               most 1024 (768 for three evolved species; a larger tile runs
                               one step per pass); 0 (default): automatic (64 x 13, 64 x 9
                               for three evolved species, or the domain's extent where
                               smaller).  Both 0, or both positive with at most 1024
                               threads, else MSD_EINVAL */
  int32_t tile_y;
} msd_launch;

MSD_API int msd_set_launch(msd_sim* sim, const msd_launch* launch);
MSD_API int msd_get_launch(const msd_sim* sim, msd_launch* launch);

/* Tuning by measurement.  Each candidate launch is applied, run for one
 * warm-up step and `steps` timed steps (HIP events on the handle's stream) from
 * the current state, which is saved to d_scratch (caller-owned device memory of
 * at least msd_state_bytes) and restored with the time after every trial, so
 * tuning leaves the simulation unchanged.  candidates: `count` launches, or
 * count = 0 for the library's list (tile shapes, vector widths, XCD remapping,
 * streaming hints, and for D2Q5 steps per pass and segment heights).
 * budget_ms > 0 stops once that much timed GPU work is spent.  The four
 * fastest candidates are then timed twice more (up to twice the budget) and
 * keep their best time, since one trial of a few milliseconds can be off by
 * several per cent.  The fastest launch is applied and returned in *h_best
 * with its milliseconds per step; h_trial_ms (NULL, or one entry per
 * candidate) receives every candidate's best time (-1 if not run).  cache_path (NULL: none) is a text file of lines "<key>
 * <8 launch fields> <ms>" keyed by GPU architecture, lattice, precision,
 * species count, extents and faces: a hit is applied without timing (unless
 * flags has MSD_TUNE_IGNORE_CACHE) and a new result is appended.  Errors:
 * MSD_EINVAL, MSD_ESTATE (not initialised), MSD_ENOMEM (scratch too small). */
enum { MSD_TUNE_IGNORE_CACHE = 1 };
MSD_API int msd_tune(msd_sim* sim, const msd_launch* candidates, int32_t count, int32_t steps, double budget_ms,
                     const char* cache_path, int32_t flags, void* d_scratch, size_t scratch_bytes,
                     msd_launch* h_best, double* h_ms_per_step, double* h_trial_ms);

/* Time steps the sweep advances per pass over HBM (one kernel launch) under the
 * current launch configuration: the temporally blocked count (2..6) or 1.  The
 * step from time 0 (from the state msd_init writes) runs alone; msd_step splits
 * the rest of a call into passes of at most this many steps whose lengths differ
 * by at most one (longer passes first).  Negative status (MSD_EINVAL) for a NULL
 * handle. */
MSD_API int msd_steps_per_pass(const msd_sim* sim);

/* ---------------------------------------------------------------------------
 * Batches of independent mixtures
 *
 * A batch holds `count` mixtures on one lattice and in one precision; their
 * number of species, extents, diffusivities, faces and relaxation rules may
 * all differ.  One msd_batch_step launch advances every node of every mixture
 * by one time step of Eq. (3-13) (each mixture exactly as msd_step would); the
 * tile schedule decides how workgroups map onto mixtures.  All mixtures share
 * one clock: they are initialised at time 0 and step together.
 * ------------------------------------------------------------------------- */

enum msd_batch_mode {
  MSD_BATCH_FUSED = 0,      /* one launch per step over all tiles of all mixtures */
  MSD_BATCH_PER_CLASS = 1   /* one launch per step and per distinct N */
};
enum msd_tile_order {
  MSD_ORDER_INSTANCE = 0,   /* the tiles of a mixture are consecutive workgroups */
  MSD_ORDER_INTERLEAVED = 1 /* workgroups cycle over mixtures */
};

typedef struct msd_schedule {
  int32_t block_x;          /* tile width in nodes (multiple of 64), block_x*block_y <= 256 */
  int32_t block_y;
  int32_t mode;             /* enum msd_batch_mode */
  int32_t order;            /* enum msd_tile_order */
  int32_t xcd_remap;        /* 1: consecutive tiles of a launch on one XCD */
  int32_t nontemporal;      /* streaming-hint mask, as in msd_launch */
  int32_t temporal;         /* D2Q5: at most this many steps (2..6) per pass over HBM with the
                               temporally blocked sweep, as in msd_launch (each class of equal
                               N takes the largest count its on-chip window allows, the
                               walled limits if any member has an x or y wall; classes
                               then launch separately whatever `mode` says, and block_x,
                               block_y, order apply to their single steps); 0 or 1: one step
                               per launch.  Default 6 for D2Q5, 0 otherwise */
  int32_t seg_rows;         /* rows per workgroup of the blocked sweep (0: 16) */
  int32_t graph;            /* 1 (default): msd_batch_step captures the launches of a span of
                               full passes (twice the least common multiple of the classes'
                               steps per pass, so every class ends on the buffer half it
                               started from) into a HIP graph once per schedule and replays
                               it for as many whole spans as a call holds (at t > 0); the
                               rest of the call, and calls shorter than a span, launch
                               directly.  0: always launch directly */
} msd_schedule;

/* Workspace bytes for a batch (every mixture's buffers and constants plus the
 * mixture table and the largest tile table any schedule needs).  Returns 0 and
 * sets *status on invalid input (each problem is validated as in
 * msd_workspace_bytes; all must share lattice and precision; count >= 1). */
MSD_API size_t msd_batch_workspace_bytes(const msd_problem* problems, int32_t count, int32_t* status);

/* Create a batch over the caller's workspace (>= msd_batch_workspace_bytes,
 * 256-byte aligned).  Uploads the mixture and tile tables (asynchronously, on
 * the stream).  The default schedule is 64 x 4 tiles, fused, instance order. */
MSD_API int msd_batch_create(const msd_problem* problems, int32_t count, void* d_ws, size_t ws_bytes, void* stream,
                             msd_batch** out);

/* Initialise mixture `index` from N planes of its mole fractions (as msd_init).
 * Valid only while the batch time is 0. */
MSD_API int msd_batch_init(msd_batch* batch, int32_t index, const void* d_xi0, int32_t xi0_precision);

/* Advance every mixture by nsteps with the batch schedule (requires every
 * mixture initialised).  With blocked passes each class runs full passes of its
 * steps per pass, then one shorter pass for a remainder of two or more steps (a
 * single step for a remainder of one), the same passes whether or not whole
 * spans are replayed from the graph.  Asynchronous. */
MSD_API int msd_batch_step(msd_batch* batch, int64_t nsteps);

/* Reference schedules, mixture after mixture on the batch's stream:
 * msd_batch_step_each runs one launch of the single-step sweep per mixture per
 * step; msd_batch_step_separate advances each mixture exactly as its own
 * msd_sim handle with the default launch would (msd_step's plan: the
 * LDS-resident kernel for tiny domains, temporally blocked passes where the
 * plan takes them, else single steps), i.e. what `count` separate handles
 * do. */
MSD_API int msd_batch_step_each(msd_batch* batch, int64_t nsteps);
MSD_API int msd_batch_step_separate(msd_batch* batch, int64_t nsteps);

MSD_API int64_t msd_batch_time(const msd_batch* batch);

/* Observables of mixture `index` at the current time, as msd_read_moments. */
MSD_API int msd_batch_read_moments(msd_batch* batch, int32_t index, int32_t out_precision, void* d_xi, void* d_J,
                                   void* d_grad);

/* Diagnostics of mixture `index`, as msd_diagnostics (synchronises). */
MSD_API int msd_batch_diagnostics(msd_batch* batch, int32_t index, double* h_mass, double* h_min, double* h_max,
                                  int64_t* h_nonfinite);

/* Schedule (re)selection; rebuilds and uploads the tile table. */
MSD_API int msd_batch_set_schedule(msd_batch* batch, const msd_schedule* schedule);
MSD_API int msd_batch_get_schedule(const msd_batch* batch, msd_schedule* schedule);

/* Whole-batch checkpoint: the current distributions of every mixture, packed
 * back to back (msd_batch_state_bytes in total); restore sets the batch time. */
MSD_API size_t msd_batch_state_bytes(const msd_batch* batch);
MSD_API int msd_batch_save(const msd_batch* batch, void* d_dst, int64_t* h_step);
MSD_API int msd_batch_restore(msd_batch* batch, const void* d_src, int64_t step);

/* Tuning of the tile schedule by measurement, as msd_tune does for one mixture:
 * candidates are schedules (count = 0: the library's list of tile shapes,
 * fused or per-class launches, tile orders, XCD remapping, and for D2Q5 steps
 * per pass and segment heights), d_scratch holds msd_batch_state_bytes, and
 * the cache key hashes every mixture's species count, extents and faces. */
MSD_API int msd_batch_tune(msd_batch* batch, const msd_schedule* candidates, int32_t count, int32_t steps,
                           double budget_ms, const char* cache_path, int32_t flags, void* d_scratch,
                           size_t scratch_bytes, msd_schedule* h_best, double* h_ms_per_step, double* h_trial_ms);

/* Number of workgroups of one msd_batch_step launch under the current schedule
 * (all classes together). */
MSD_API int64_t msd_batch_tiles(const msd_batch* batch);

MSD_API int msd_batch_destroy(msd_batch* batch);

/* ---------------------------------------------------------------------------
 * Errors and version
 * ------------------------------------------------------------------------- */

MSD_API const char* msd_strerror(int status);
MSD_API const char* msd_last_error(void);
MSD_API int msd_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MSD_H */
