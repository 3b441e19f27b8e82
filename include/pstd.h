/*
 * pstd.h - C ABI of libpstd: the time-step hot path of the sine/cosine-basis PSTD method
 * (Wise, Jaros, Cox & Treeby, "Pseudospectral time-domain (PSTD) methods for the wave equation:
 * realising boundary conditions with discrete sine and cosine transforms", arXiv:2005.00322)
 * on AMD Instinct MI355X (gfx950).
 *
 * The library solves the linear acoustic system of Eq. (wave_eq),
 *     du/dt = -(1/rho0) dp/dx,   dp/dt = -rho0 c0^2 du/dx,
 * in a rectangular box whose faces are each sound-hard (Neumann) or sound-soft (Dirichlet), with the
 * staggered DTT-based scheme of Eq. (dtt_pstd_solution) (1D) and its 2D/3D form (§4.3): per axis a
 * forward discrete sine/cosine transform, a multiply by +-k with the sine<->cosine type switch of
 * Table transform_choices, the inverse transform onto the staggered grid, then the leapfrog update.
 *
 * Grid layout (all arrays row-major, the LAST axis contiguous):
 *   - an axis with n pressure nodes has walls on nodes 0 and n-1 (spacing dx, length L = (n-1) dx);
 *   - p has shape n[0] x ... x n[ndim-1]; p must be 0 on Dirichlet wall nodes (pstd_state_init
 *     zeroes them and the step keeps them 0);
 *   - u[a] (velocity along axis a) has the shape of p with n[a] replaced by n[a]-1 and sits at the
 *     staggered points (j + 1/2) dx of axis a.
 * A step advances (p^n, u^{n-1/2}) to (p^{n+1}, u^{n+1/2}).
 *
 * Conventions: every call returns a pstd_status (0 = success); nothing throws across the ABI.
 * Device pointers are plain HIP device addresses; the caller owns every buffer it passes in and the
 * library never frees caller memory.  A plan owns its operator tables and work buffers and runs all
 * its kernels on the HIP stream given at creation (0 = the null stream); calls return once the work
 * is enqueued.  A plan is used from one host thread at a time.  pstd_last_error() returns a
 * thread-local message for the last failing call.
 */
#ifndef PSTD_H
#define PSTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PSTD_OK = 0,
  PSTD_E_INVALID_ARG = -1,  /* null pointer, bad enum, n < 3, non-positive dx/dt/c0/rho0 ...      */
  PSTD_E_UNSTABLE = -2,     /* c0 dt / dx above 2 / (dx max|k|) (the 2/pi limit of §4.2 in 1D)    */
  PSTD_E_UNSUPPORTED = -3,  /* size or mode the library does not handle                            */
  PSTD_E_HIP = -4,          /* a HIP runtime call failed (message in pstd_last_error)              */
  PSTD_E_OOM = -5,          /* device allocation failed                                            */
  PSTD_E_NONFINITE = -6     /* the state holds NaN or Inf (pstd_check_finite)                      */
} pstd_status;

/* Boundary condition of one face (§1: Neumann = sound-hard, Dirichlet = sound-soft). */
/* Boundary of one face.  PERIODIC (both faces of an axis, the Fourier basis of Eq. (fourier_pstd_solution),
 * §2): the axis is one period of n nodes and its particle velocity has n staggered points instead of
 * n - 1; such axes run on the dense contraction path or, in 2D FP32 plans, the fused path (not the FFT,
 * 1D or batched paths). */
/* NEUMANN_HALF / DIRICHLET_HALF (right faces only): the wall lies half a step beyond the last node, at
 * (n - 1/2) dx, on the last of n staggered points (groups III/IV of Table DTT_wavenumber_groups: DTT types
 * V-VIII, implied period 2n - 1).  Such axes run on the dense contraction path or the fused 2D path. */
typedef enum {
  PSTD_NEUMANN = 0, PSTD_DIRICHLET = 1, PSTD_PERIODIC = 2, PSTD_NEUMANN_HALF = 3, PSTD_DIRICHLET_HALF = 4
} pstd_bc;

/* Arithmetic of the transform contractions.  FP64: state and operators in double.  FP32: state and
 * operators in float, FP32 accumulation.  SPLIT_BF16: float state; each contraction is
 * A_hi X_hi + A_hi X_lo + A_lo X_hi with bfloat16 hi/lo parts and FP32 accumulation (2D and 3D grids; a
 * 1D plan, a single line with no matrix-matrix product, computes as FP32). */
typedef enum { PSTD_FP64 = 0, PSTD_FP32 = 1, PSTD_SPLIT_BF16 = 2 } pstd_precision;

typedef struct {
  int32_t ndim;   /* 1, 2 or 3 */
  int64_t n[3];   /* pressure nodes per axis, both wall nodes included, n >= 3 */
} pstd_grid;

/* Caller-owned device state.  p and u[0..ndim-1] are double (PSTD_FP64) or float (otherwise). */
typedef struct {
  void* p;
  void* u[3];
  int64_t step;   /* time-step counter, advanced by pstd_step */
} pstd_state;

typedef struct pstd_plan_s* pstd_plan;

/* Create a plan: homogeneous medium, rho0 = 1000 kg/m^3, FP32, null stream.
 * bc_per_face = {x-, x+, y-, y+, z-, z+} (entries beyond 2*ndim are ignored).
 * Builds, in FP64 on the host, the per-axis operators of Table transform_choices: the velocity
 * operator G_a = T2^{-1} diag(a1) T1 ((n-1) x n) and the pressure operator D_a = T1^{-1} diag(a2) T2
 * (n x (n-1)), with the DC/Nyquist entries dropped or zero-padded as in the appendix tables
 * "Differentiation with staggered grids", folds -dt/rho0 and -dt rho0 c0^2 into them, rounds them to
 * the plan's precision and copies them to the device.  Axes that start on the FFT path (see pstd_path)
 * get FFT tables instead (twiddles and the spectral multipliers, also formed in FP64).  Sizes: n <= 4097
 * per axis on the dense path; up to 8193 (FP32 state) or 4097 (FP64) where 2(n-1) = 16 x 2^a 3^b 5^c; a
 * periodic axis of a float state up to 8192 points where n is a power of two (the FFT path).
 * Returns PSTD_E_UNSTABLE if the time step is above the
 * stability limit, PSTD_E_UNSUPPORTED for sizes outside these limits. */
int pstd_plan_create(const pstd_grid* grid, double dx, double dt, double c0,
                     const int32_t bc_per_face[6], pstd_plan* out);

/* As pstd_plan_create with density, precision, an optional sound-speed map and a stream.
 * c0_map_dev: nullable device array of float c0(x) on the p nodes (same shape as p); when given, the
 * pressure step uses c0(x)^2 pointwise (an extension beyond the paper's homogeneous medium) and c0 is
 * only used for the stability check (pass the map's maximum).  The map must outlive the plan.
 * hip_stream: a hipStream_t or NULL. */
int pstd_plan_create_ex(const pstd_grid* grid, double dx, double dt, double c0,
                        const int32_t bc_per_face[6], double rho0, int32_t precision,
                        const float* c0_map_dev, void* hip_stream, pstd_plan* out);

/* Prepare a caller-filled state: zero p on Dirichlet wall nodes, then set u[a]^{-1/2}.
 * u_mode 0: u^{-1/2} = +(dt / (2 rho0)) G_a p^0, i.e. particle velocity zero at t = 0 on the
 *           staggered time grid (the reading of "set to zero, accounting for the staggered grid",
 *           §4.2);  u_mode 1: u^{-1/2} = 0;  u_mode 2: keep the caller's u.
 * Sets state->step = 0. */
int pstd_state_init(pstd_plan plan, pstd_state* state, int32_t u_mode);

/* Advance the state by n_steps >= 0 steps of Eq. (dtt_pstd_solution) (§4.3 for 2D/3D): every u_a from
 * p^n first, then p^{n+1} from all u_a^{n+1/2}.  Asynchronous on the plan's stream.  The steps replay
 * captured HIP graphs (whole chunks of 50 steps, then one graph of the remaining steps; 1D plans of at most
 * 1365 nodes with walls on nodes run one kernel instead); a graph is captured on first use for the
 * state's buffers and kept by the plan (one full-chunk graph and one of the last other length). */
int pstd_step(pstd_plan plan, pstd_state* state, int64_t n_steps);

/* Capture, without running anything, the graphs a later pstd_step(plan, state, n_steps) replays, so that
 * the capture cost stays out of a timed or latency-critical call.  Synchronous on the host; enqueues no
 * work.  Same arguments and errors as pstd_step. */
int pstd_step_prepare(pstd_plan plan, const pstd_state* state, int64_t n_steps);

/* Execution path of pstd_step.
 *   PER_AXIS: one dense contraction kernel per axis and half step (axes up to 4097 nodes).
 *   FUSED:    2D FP32 grids of at most 512 x 512 nodes, walls or periodic axes: two kernels per step
 *             (every velocity tile, then every pressure tile with both axes' terms).
 *   FFT:      every axis whose extended period 2(n-1) is 16 x 2^a 3^b 5^c (up to 16384 for a float state,
 *             8192 for FP64) applies its operators as LDS-resident FFTs of the field's symmetric
 *             extension (§3.2: each DTT is a DFT of an evenly or oddly extended sequence), one kernel per
 *             axis and half step, and so does a periodic axis of a float state whose n is a power of two
 *             from 256 to 8192 (the DFT of the line itself, Eq. (fourier_pstd_solution)); other axes stay
 *             dense.
 *   AUTO:     FUSED where it applies; otherwise FFT on axes above 512 nodes (1D plans: above 1365) and
 *             dense contractions elsewhere.
 *   FFT_GENERIC: FFT, with every axis on the mixed-radix kernel.  Under the other paths an FP32 axis
 *             whose 2(n-1) is a power of two from 256 to 8192 runs a kernel specialised to that length
 *             (radix-16 passes, twiddles and spectral multipliers from tables formed in FP64).
 *   STORED:   PER_AXIS, with every split-bf16 contraction reading its operator's entries from memory.
 *             Under the other paths a SPLIT_BF16 contraction whose operator has between 193 and 384
 *             rows and at most 512 columns forms its operator slices on the chip from the operator's
 *             Toeplitz and Hankel parts (pstd_axis_operator_structure), which reads two vectors
 *             instead of the matrix.
 * All compute the same step and replay captured HIP graphs; the choice changes speed and rounding only. */
typedef enum {
  PSTD_PATH_AUTO = 0, PSTD_PATH_PER_AXIS = 1, PSTD_PATH_FUSED = 2, PSTD_PATH_FFT = 3, PSTD_PATH_STORED = 4,
  PSTD_PATH_FFT_GENERIC = 5
} pstd_path;

/* Select the execution path of later pstd_step calls (builds dense operators on first use when an axis
 * moves off the FFT path).  PSTD_E_UNSUPPORTED if the plan cannot use it. */
int pstd_plan_set_path(pstd_plan plan, int32_t path);

/* One term of the step on its own: which = 0 applies the velocity update of axis `axis`,
 * u_a += -(dt/rho0) G_a p (Eq. (dtt_pstd_solution_a) along that axis); which = 1 applies that axis's share
 * of the pressure update, p += -(dt rho0 c0^2) D_a u_a (one summand of Eq. (dtt_pstd_solution_b) in the
 * form of §4.3).  A full step is every which = 0 term followed by every which = 1 term.  axis = -1
 * applies the whole phase (every axis) the way pstd_step does it: one kernel on the FUSED path; one for
 * the velocity terms of all axes when every axis runs on the FFT path with one power-of-two transform
 * length (float state); one per axis otherwise.  Asynchronous on the plan's stream; state->step is not
 * changed. */
int pstd_apply_axis(pstd_plan plan, pstd_state* state, int32_t axis, int32_t which);

/* p_out = (1+R)/2 * p_neumann + (1-R)/2 * p_dirichlet, elementwise over count floats.
 * The single-reflection form of §5's weighted sum of Neumann and Dirichlet fields for one real
 * reflection coefficient R on every face (exact until doubly reflected arrivals).  p_out may alias
 * either input.  Asynchronous on hip_stream (NULL = null stream). */
int pstd_combine_R(const float* p_dirichlet, const float* p_neumann, double R,
                   float* p_out, int64_t count, void* hip_stream);

/* p_out = sum_i w[i] * fields[i], elementwise over count floats (the general weighted sum of §5;
 * weights from w = M^T r / 4 per axis).  fields: host array of nfields device pointers.  p_out may
 * alias fields[0].  Asynchronous on hip_stream. */
int pstd_combine_fields(const float* const* fields, const double* w, int32_t nfields,
                        float* p_out, int64_t count, void* hip_stream);

/* Host only (no GPU needed): the basic fields and weights of §5 for an arbitrary real reflection
 * coefficient on every face.  R: 2 ndim coefficients, (left, right) per axis (1 reflects like a rigid
 * wall, -1 like a pressure-release wall, 0 absorbs; any finite value is accepted).  The solution for
 * these faces is sum_f w_out[f] p_f over the 4^ndim solutions p_f of the same problem with the basic
 * walls of field f: per axis the walls (N,N), (N,D), (D,N), (D,D) take the weights (1/4) M^T r with
 * r = (R_L, 1, R_R, R_L R_R) and §5's image matrix M, and a field's weight is the product over its axes
 * (separable image sources).  Field f = sum_a c_a 4^(ndim-1-a) with c_a the index of axis a's wall pair
 * in that order.  bc_out: 4^ndim x 2 ndim pstd_bc values (field f, axis a, left then right) in the
 * layout of pstd_plan_create's bc_per_face; w_out: 4^ndim weights.  Exact while no wave has been
 * reflected twice by the same pair of walls (until t = 2 L / c0 on the shortest axis; 3 L / c0 where
 * both walls absorb).  Returns PSTD_E_INVALID_ARG for ndim outside 1..3, a null pointer or a
 * non-finite coefficient. */
int pstd_face_weights(int32_t ndim, const double* R, int32_t* bc_out, double* w_out);

/* Check that p and every u_a are finite.  Synchronises the plan's stream.  Returns PSTD_OK or
 * PSTD_E_NONFINITE. */
int pstd_check_finite(pstd_plan plan, const pstd_state* state);

/* Copy the plan's device operators back to the host as double (for inspection and tests).
 * which: 0 = velocity operator G_a ((n_a-1) x n_a), 1 = pressure operator D_a (n_a x (n_a-1)), both
 * with the time-step constants folded in and rounded to the plan's precision (SPLIT_BF16 returns
 * hi + lo).  out must hold the matrix row-major.  Synchronous. */
int pstd_plan_get_operator(pstd_plan plan, int32_t axis, int32_t which, double* out);

/* Host only (no GPU needed): the unscaled FP64 operator of one axis, exactly as the plan builder forms
 * it before folding the time-step constants in.  n nodes, boundary pair (bc_left, bc_right), spacing dx.
 * which 0: velocity operator T2^{-1} diag(a1) T1, (n-1) x n row-major (derivative of p on the
 * staggered points); which 1: pressure operator T1^{-1} diag(a2) T2, n x (n-1) row-major.  A periodic
 * pair (both PSTD_PERIODIC) gives the n x n operators of Eq. (fourier_pstd_solution), a half-step right
 * wall the n x n operators of its DTT types V-VIII.  out must hold the matrix.  Synchronous. */
int pstd_axis_operator(int64_t n, int32_t bc_left, int32_t bc_right, double dx, int32_t which, double* out);

/* Toeplitz-plus-Hankel form of the same operator (host only, no GPU needed).  Each operator is a forward
 * trig transform, a diagonal and an inverse one (§3.2, Eq. (dtt_pstd_solution_a)/(dtt_pstd_solution_b));
 * products of the two transforms' cosines and sines are trig functions of the difference and of the sum
 * of the output and input indices, so with R x C the operator's shape
 *     A[r][c] = wr[r] * wc[c] * (f[r - c + C - 1] + g[r + c]),
 * where f and g hold R + C - 1 values each (caller-owned) and the weights are one except
 * w[0] = wr[0], w[1] = wr[R-1], w[2] = wc[0], w[3] = wc[C-1] (a wall node counted once in the
 * symmetric extension, or held at zero).  f and g are determined up to one constant per parity of
 * r + c, chosen to minimise the sum of their squares.  *resid (nullable) receives the largest entry
 * error relative to max|A|.  PSTD_E_UNSUPPORTED if the operator has no such form (then only
 * *resid is written), PSTD_E_INVALID_ARG as pstd_axis_operator.  (Tolerance 1e-9, far below FP32
 * rounding; a boundary line below 1e-12 max|A| counts as zero.)  The split-bf16 contractions use the form
 * to build their operator slices on the chip (see pstd_plan_set_path). */
int pstd_axis_operator_structure(int64_t n, int32_t bc_left, int32_t bc_right, double dx, int32_t which,
                                 double* f, double* g, double* w, double* resid);

/* Collocated differentiation (§3.3) and half-step interpolation (§3.4) of a wall-bounded axis: which
 *   2 = PSTD_OP_GRAD_NODES   d/dx on the n nodes (n x n): forward T1, times a1 k, inverse of the
 *                            symmetry opposite to p's (the DC / Nyquist entries dropped or zero-filled);
 *   3 = PSTD_OP_GRAD_STAG    d/dx on the n - 1 staggered points ((n-1) x (n-1)), from T2 and a2 k;
 *   4 = PSTD_OP_NODES_TO_STAG a field of p's symmetry resampled half a step onto the staggered points
 *                            ((n-1) x n), forward T1 and the half-sample inverse of the same parity;
 *   5 = PSTD_OP_STAG_TO_NODES a field of u's symmetry (a particle velocity) resampled onto the nodes
 *                            (n x (n-1)), forward T2 and the whole-sample inverse of the same parity.
 * pstd_axis_operator with these values returns the FP64 matrix (derivatives include 1/dx); a periodic
 * pair gives PSTD_E_UNSUPPORTED.  Columns / rows of nodes outside a sequence's sample (a Dirichlet node
 * of p, a Neumann node of the derivative of p) are zero. */
enum { PSTD_OP_GRAD_NODES = 2, PSTD_OP_GRAD_STAG = 3, PSTD_OP_NODES_TO_STAG = 4, PSTD_OP_STAG_TO_NODES = 5 };

/* Apply one of the operators above along `axis` of a device field: out = A in, on the plan's stream
 * with the dense contraction kernels in the plan's precision (double for FP64, float otherwise; the
 * SPLIT_BF16 plan uses the split products).  in and out are row-major, contiguous, distinct, with the
 * plan's extents on every other axis and the operator's column / row count on `axis` (for example
 * PSTD_OP_STAG_TO_NODES along axis a maps u[a] onto the p grid).  The operator is built in FP64 and kept
 * by the plan on first use (synchronous then); later calls are asynchronous.  Errors: PSTD_E_INVALID_ARG
 * for null pointers, in == out, a bad axis or which; PSTD_E_UNSUPPORTED for a periodic axis or one above
 * 4097 nodes. */
int pstd_apply_axis_operator(pstd_plan plan, int32_t axis, int32_t which, const void* in, void* out);

/* Number of elements of p / of u[axis] for this plan. */
int64_t pstd_plan_numel(pstd_plan plan, int32_t field /* -1 = p, 0..2 = u[axis] */);

int pstd_plan_destroy(pstd_plan plan);

/* ---- Batched 2D solves: many independent boxes stepped by one persistent launch ----------------------
 * A batch holds `count` independent 2D FP32 solves of possibly different sizes, boundary faces,
 * spacings, time steps and sound speeds (density rho0 shared), all on the batch's stream.  Each solve is
 * the 2D scheme of §4.3; the paired Neumann/Dirichlet solves of one physical instance are two entries
 * combined afterwards with pstd_batch_combine_R.  Operators are built in FP64 once per distinct
 * (n, boundary pair) and shared.  pstd_batch_step runs all requested steps of all solves in one
 * persistent kernel launch of at most as many blocks as the GPU holds: per step a velocity phase over
 * every solve's velocity tiles, a grid-wide barrier, a pressure phase over every pressure tile, a second
 * barrier. */
typedef struct pstd_batch_s* pstd_batch;

/* n: count x 2 (nx, ny) nodes per solve, each >= 3 and <= 512; bc: count x 4 faces {x-, x+, y-, y+};
 * dx, dt, c0: count values each.  Returns PSTD_E_UNSTABLE if any solve is above its stability limit. */
int pstd_batch_create(int32_t count, const int64_t* n, const int32_t* bc, const double* dx, const double* dt,
                      const double* c0, double rho0, void* hip_stream, pstd_batch* out);

/* Heterogeneous media (an extension beyond the paper's homogeneous box): c0_maps holds count device
 * pointers, each null or an nx x ny float map of c0(x) for that solve; the pressure updates of those
 * solves then use c0(x)^2 pointwise (density stays rho0).  The stability check of pstd_batch_create
 * used the c0 passed there, so pass each map's maximum as c0.  The maps are squared into buffers the
 * batch owns; the caller's maps may be freed after the call's work completes.  Asynchronous. */
int pstd_batch_set_c0_maps(pstd_batch batch, const float* const* c0_maps);

/* Prepare caller-filled states (count of them, FP32 p and u[0], u[1]) as pstd_state_init does. */
int pstd_batch_state_init(pstd_batch batch, pstd_state* states, int32_t u_mode);

/* Advance every solve by n_steps: per 1024 steps one persistent launch (with the kernel that zeroes its
 * tile tickets and barrier counters) replayed from a captured HIP graph.  Asynchronous. */
int pstd_batch_step(pstd_batch batch, pstd_state* states, int64_t n_steps);

/* out[i] = (1+R[i])/2 p_neumann + (1-R[i])/2 p_dirichlet for npairs pairs; pairs = npairs x 2 solve
 * indices (dirichlet, neumann) of equally sized solves; out[i] holds nx*ny floats (may alias either p). */
int pstd_batch_combine_R(pstd_batch batch, const pstd_state* states, const int32_t* pairs, const double* R,
                         float* const* out, int32_t npairs);

/* Launch configuration of pstd_batch_step: resident block count (0 = the occupancy maximum), tile
 * order within a phase (0 = longest contraction first, 1 = solve by solve) and output tile edge (32:
 * 32 x 32 tiles on FP32 MFMA 16x16x4; 64: 64 x 64 tiles on FP32 MFMA 32x32x2; 16: when every solve has
 * one shape of at most 512 x 512 nodes, no persistent launch but two fused phase launches per step over
 * all solves, each block one 16 x 16 tile of one solve, replayed from captured graphs; blocks and order
 * are then unused).  Returns PSTD_E_UNSUPPORTED for tile 16 on other batches. */
int pstd_batch_set_config(pstd_batch batch, int32_t blocks, int32_t order, int32_t tile);

/* Autotuner: time every candidate configuration (tile edge x block count x order, and tile 16 where it
 * applies) for trial_steps steps on scratch state buffers (the caller's states are not touched), keep
 * the fastest and, if cache_path is not NULL, store it in a small JSON file keyed by a signature of the
 * batch; a later call with a matching file skips the timing.  config_out (nullable, 4 ints): blocks, order, tile, 1 if taken from the cache.
 * Synchronous. */
int pstd_batch_autotune(pstd_batch batch, int32_t trial_steps, const char* cache_path, int32_t* config_out);

/* Wait for the batch's stream and report whether every grid barrier of the launches since the last
 * call completed: PSTD_E_HIP if one gave up waiting (its blocks were not all resident, e.g. because other
 * work held the GPU), in which case the states are not valid. */
int pstd_batch_synchronize(pstd_batch batch);

int pstd_batch_destroy(pstd_batch batch);

/* ---- DCT-basis neural-operator surrogate -------------------------------------------------------------
 * Not a method of the paper: a learned map from (p0, c0 map) on an H x W grid to the pressure after a
 * fixed number of PSTD steps, trained on fields the solver produces; the solver remains its fallback and
 * the reference for its error.  Network (all parameters FP32, contractions on bf16 matrix cores with FP32
 * accumulation):
 *   features f = [p0, (c0 - 1500)/100, x, y] with x = i/(H-1), y = j/(W-1)
 *   lift     v = P f + pb                                   P: C x 4
 *   layer l  v = GELU(W_l v + b_l + IDCT(R_l . DCT(v)))      W_l: C x C; R_l: (Mm/2) x (Mm/2) x C x C
 *   project  q = GELU(Q1 v + q1b),  out = Q2 q + q2b         Q1: Hp x C; Q2: Hp
 * DCT: orthonormal DCT-II along both axes keeping the Mm lowest modes; IDCT: its transpose; R_l mixes
 * channels per mode, one matrix per 2 x 2 block of modes.  GELU is x Phi(x) with the normal CDF; the
 * kernels evaluate Phi in the forward pass with Hastings' rational approximation of erfc (Abramowitz &
 * Stegun 7.1.26, absolute error <= 1.5e-7) and use the exact erf in the backward pass.  The flat
 * parameter vector is P, pb, then per layer (R_l, W_l, b_l), then Q1, q1b, Q2, q2b, each row-major.
 * Loss: batch mean of |out - target|^2 / |target|^2. */
typedef struct {
  int32_t H, W;        /* grid */
  int32_t channels;    /* C, 1 .. 32 */
  int32_t modes;       /* Mm, even, <= H, <= W and <= 256 */
  int32_t layers;      /* 1 .. 16 */
  int32_t hidden;      /* Hp, 1 .. 256 */
  int32_t max_batch;   /* buffers are sized for this batch */
  int32_t split;       /* 1: each product as hi*hi + hi*lo + lo*hi bf16 parts (near FP32), 0: one bf16 product */
} pstd_nop_config;

typedef struct pstd_nop_s* pstd_nop;

/* Create a surrogate with zero parameters on hip_stream (NULL = null stream).  Allocates every buffer
 * for cfg->max_batch (about (7 + 3 layers) x batch x C x H x W floats plus 4 x batch x Hp x H x W). */
int pstd_nop_create(const pstd_nop_config* cfg, void* hip_stream, pstd_nop* out);
/* Length of the flat parameter vector (-1 for a null handle). */
int64_t pstd_nop_param_count(pstd_nop nop);
/* Copy host FP32 parameters in (and reset the Adam moments and step count) / out.  n must equal the
 * parameter count.  Synchronous. */
int pstd_nop_set_params(pstd_nop nop, const float* host, int64_t n);
int pstd_nop_get_params(pstd_nop nop, float* host, int64_t n);
/* Copy the gradient of the last pstd_nop_backward to the host.  Synchronous. */
int pstd_nop_get_grads(pstd_nop nop, float* host, int64_t n);
/* out[b] = network(p0[b], c0[b]) for b < batch (device arrays of batch x H x W floats, row-major) and keep
 * the activations for a following pstd_nop_backward.  Asynchronous on the surrogate's stream. */
int pstd_nop_forward(pstd_nop nop, const float* p0, const float* c0, float* out, int32_t batch);
/* The same map for inference: stores no activations (a following pstd_nop_backward is refused). */
int pstd_nop_infer(pstd_nop nop, const float* p0, const float* c0, float* out, int32_t batch);
/* Gradient of the loss of the last forward against target (device, batch x H x W) into the surrogate's
 * gradient buffer; *loss (nullable) receives the loss (synchronises when given). */
int pstd_nop_backward(pstd_nop nop, const float* target, double* loss);
/* One Adam step (Kingma & Ba, with bias correction) on the parameters with the current gradient. */
int pstd_nop_adam_step(pstd_nop nop, double lr, double beta1, double beta2, double eps);
/* err[b] = |pred[b] - target[b]| / |target[b]| for b < batch (device fields, host err).  Synchronous. */
int pstd_nop_relative_errors(pstd_nop nop, const float* pred, const float* target, int32_t batch, double* err);
/* Input statistics for the surrogate's gate, per sample b < batch (device p0, c0; host stats, batch x 4):
 * min c0, max c0, max |p0| and the share of sum p0^2 on nodes within `margin` of a wall.  A caller
 * compares them with the training distribution and sends samples outside it (or every sample, when the
 * surrogate's validated error exceeds the tolerance) to the PSTD solver instead.  Synchronous. */
int pstd_nop_input_stats(pstd_nop nop, const float* p0, const float* c0, int32_t batch, int32_t margin, double* stats);
int pstd_nop_destroy(pstd_nop nop);
/* The surrogate's gate: when it may answer instead of the solver.  validated_error is its relative L2
 * error against the solver on held-out pairs (a high quantile); a request whose tolerance is below it
 * always goes to the solver.  The other fields bound the training distribution: the sound-speed range,
 * the largest |p0| and the largest share of sum p0^2 within wall_margin nodes of a wall. */
typedef struct {
  double validated_error;
  double c0_lo, c0_hi;
  double p_max;
  int32_t wall_margin;
  double wall_share_max;
} pstd_nop_gate;

/* The PSTD problem the surrogate stands for, which the fallback solves: spacing, time step, density,
 * faces {x-, x+, y-, y+} (Neumann or Dirichlet) and the number of steps (the network predicts the pressure
 * after that many steps from rest, u^{-1/2} as pstd_state_init's u_mode 0). */
typedef struct {
  double dx, dt, rho0;
  int32_t bc[4];
  int64_t steps;
} pstd_nop_problem;

/* Answer batch requests (device p0, c0 maps, out: batch x H x W floats each; any batch size): the
 * input statistics of pstd_nop_input_stats decide per sample whether it lies inside the gate's
 * training distribution; samples inside it are answered by the network when gate->validated_error <=
 * tol, every other sample by the FP32 batched solver of pstd_batch_* (its c0 map squared pointwise, its
 * stability limit from the map's maximum), whose pressure is stepped in place in out.  fallback (host,
 * batch entries, nullable) receives 1 for solver answers; n_fallback (nullable) their count.
 * Synchronous; allocates the fallback solves' velocity buffers for the duration of the call.
 * Not a method of the paper: the solver remains the surrogate's fallback and the reference for its error. */
int pstd_nop_predict(pstd_nop nop, const pstd_nop_gate* gate, const pstd_nop_problem* problem, const float* p0,
                     const float* c0, float* out, int32_t batch, double tol, int32_t* fallback, int32_t* n_fallback);


/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): err[b] = |pred[b] - target[b]|_2 / |target[b]|_2 (0 where the
 * target is zero) for b < batch, the measure of pstd_nop_relative_errors without a surrogate handle.
 * pred, target: device arrays of batch x count floats; err: device array of batch doubles (caller-owned).
 * Sums in FP64.  Enqueues two kernels on hip_stream (NULL = null stream) and nothing else: no allocation,
 * copy or synchronisation.  The per-block partial sums live in a 1 MiB array that the library keeps on
 * each GPU it runs on until the process ends; every call on a GPU shares it, so calls that overlap on one
 * GPU (several streams or host threads) race.  PSTD_E_INVALID_ARG for null pointers or batch, count < 1;
 * PSTD_E_UNSUPPORTED for batch above 65536. */
int pstd_relative_errors_static(const float* pred, const float* target, int32_t batch, int64_t count, double* err,
                                void* hip_stream);

const char* pstd_status_string(int status);
const char* pstd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PSTD_H */
