/*
 * kfvm.h - C-ABI of the MI355X (gfx950) KFVM-WENO right-hand-side library.
 *
 * The library evaluates the semi-discrete right-hand side of the compressible
 * Euler equations (paper section 1, eq. model and eq. euler, ideal-gas law with
 * ratio of specific heats gamma) on a uniform Cartesian grid with the
 * kernel-based finite volume WENO-AO scheme of May & Lee (arXiv 2401.16543),
 * and advances it with the three-stage SSP Runge-Kutta method of Shu & Osher.
 *
 * Boundaries are periodic unless kfvm_set_boundary says otherwise (outflow,
 * reflecting, inflow).
 *
 * The right-hand side follows the paper's section 5.3: per cell the linearised
 * primitive variables W = Phi U with Phi from the cell's own average (section
 * 3.4.2, eq. consToLPMat), point values and derivatives from precomputed kernel
 * reconstruction vectors (section 2.1, eq. reconVec; section 3.3), smoothness
 * indicators (eq. smoothIndic), WENO-JS form nonlinear weights with eps = 1e-40
 * (eq. nlinWts), the WENO-AO blend (eq. wenoAOrec), u = Phi^-1 w (eq.
 * recVarToCons), the positivity limiter of section 4, an HLLC or HLL Riemann
 * solver with Batten wavespeeds at every face Gauss point (section 6), and the
 * Gauss-Legendre face integral of the fluxes.
 *
 * Conventions
 *  - Every entry point returns int: KFVM_OK (0) or a negative error code; no
 *    C++ exception crosses the ABI.  kfvm_last_error() gives a message.
 *  - State arrays are device pointers to float64 in struct-of-arrays layout
 *    U[v][z][y][x] (x fastest), v over (rho, rho u, rho v[, rho w], E): 4
 *    variables in 2D, 5 in 3D.  They are owned by the caller.
 *  - Work is queued on the context's HIP stream (kfvm_set_stream; default the
 *    null stream) and is asynchronous unless stated otherwise.
 *  - A context owns its weight tables and workspace, allocated in kfvm_init
 *    and freed in kfvm_destroy; the per-path face buffers (float64 for the
 *    FP64 path, float32 for the split path) are allocated on the path's first
 *    use (out of memory then: KFVM_ERR_HIP).  Contexts are independent; one
 *    context must not be used from two threads at once.
 */
#ifndef KFVM_H
#define KFVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    KFVM_OK = 0,
    KFVM_ERR_ARG = -1,          /* bad dimension, order, size, pointer or mode */
    KFVM_ERR_HIP = -2,          /* HIP runtime error; message in kfvm_last_error */
    KFVM_ERR_NONPHYSICAL = -3,  /* a cell average with rho <= 0, p <= 0 or a non-finite value */
    KFVM_ERR_STATE = -4         /* context not initialised, or a required setting missing */
};

enum { KFVM_FP64 = 0, KFVM_SPLIT_F16 = 1, KFVM_SPLIT_BF16 = 2 };   /* kfvm_set_precision */
enum { KFVM_HLLC = 0, KFVM_HLL = 1 };                              /* kfvm_set_riemann */
enum { KFVM_CFL_SUM = 0, KFVM_CFL_MAX_AXIS = 1 };                  /* kfvm_set_cfl_form */
enum { KFVM_IND_NONE = 0, KFVM_IND_KXRCF = 1 };                    /* kfvm_set_indicator */
enum { KFVM_BC_PERIODIC = 0, KFVM_BC_OUTFLOW = 1, KFVM_BC_REFLECTING = 2, KFVM_BC_INFLOW = 3 }; /* kfvm_set_boundary */

typedef struct kfvm_ctx kfvm_ctx;

/* Periodic box of n[a] cells of width dx[a] per axis a (n[2], dx[2] ignored in 2D).
 * Every n[a] must be at least 2R + 2. */
typedef struct {
    int dim;
    int n[3];
    double dx[3];
} kfvm_mesh;

/* Reconstruction vectors (section 2.1, eq. recVec1; section 3.3; section 5.1),
 * in unit-cell coordinates.  Layout, which must match the library's own stencil
 * definition exactly (it is validated):
 *  - offsets[n0][dim]: S0 = {|i|^2 <= R^2} in lexicographic order of (x, y[, z]),
 *    x slowest (section 3.1);
 *  - stencil q = 0 is S0, q = 1 the ball of radius R-1, q >= 2 the biased cones
 *    along +x, -x, +y, -y[, +z, -z]; members[stencil_ptr[q] .. stencil_ptr[q+1])
 *    are indices into S0 in increasing order;
 *  - tables: for each stencil in turn a row-major [n_pts + n_der][N_q] block:
 *    n_pts face-point rows, s = (2 a + side) R^(dim-1) + g (normal axis a, side 0
 *    the lower face, g the Gauss index over the transverse axes, first slowest),
 *    then n_der rows for the derivatives 0 < |alpha| <= R ordered by degree, then
 *    lexicographically descending;
 *  - gamma_lin[n_stencils]: linear weights (section 3.2).
 * The library copies what it needs; the caller keeps ownership. */
typedef struct {
    int dim, R;
    int n0;
    const int *offsets;
    int n_stencils;
    const int *stencil_ptr;
    const int *members;
    int n_pts, n_der;
    const double *tables;
    const double *gamma_lin;
} kfvm_weights;

/* Host-side statistics, filled by kfvm_stats (synchronising), of the last
 * reconstruction (the last kfvm_rhs, the last stage of kfvm_step, or the last
 * kfvm_face_states). */
typedef struct {
    long long limiter_cells;     /* cells whose Riemann states the limiter scaled (a factor below one) */
    long long weno_cell_vars;    /* (cell, variable) pairs reconstructed with WENO-AO (all of them unless a
                                    gate, the indicator or kfvm_set_flags chose) */
    long long cell_vars;         /* all (cell, variable) pairs */
    int error;                   /* sticky device error code (0 or KFVM_ERR_NONPHYSICAL) */
    double min_rho, min_p;       /* least density and pressure over the admissible cells of the state passed
                                    to the last kfvm_cfl_dt (NaN before the first call) */
} kfvm_stats_t;

/* Create a context for `mesh`.  order 5 selects R = 2, order 7 selects R = 3
 * (the full stencil reproduces polynomials of degree 2R-1, section 3.1).
 * gamma > 1 is the ratio of specific heats.  weights == NULL builds the tables
 * in binary128 arithmetic (kfvm_weights_build); otherwise they are validated
 * and copied.  Allocates the device workspace and uploads the tables on the
 * current HIP device.  Defaults: FP64, HLLC, limiter on with kappa = 0.5. */
int kfvm_init(kfvm_ctx **ctx, const kfvm_mesh *mesh, int order, double gamma, const kfvm_weights *weights);

/* kfvm_init with tables built at kernel length scale ell_hat = l / Delta (in
 * cells) instead of 5, the paper's fixed choice (section 5.1; l is the
 * hyperparameter of the squared-exponential kernel of section 2.1).  The
 * polynomial part keeps the design order at any l; the 3D R = 3 weights grow
 * with l (largest face-point weight ~2 at 5, ~35 at 20, ~1600 at 100), which
 * amplifies rounding.  ell_hat outside (0, 100] (or NaN) returns KFVM_ERR_ARG
 * before any device call; otherwise as kfvm_init with weights == NULL. */
int kfvm_init_length_scale(kfvm_ctx **ctx, const kfvm_mesh *mesh, int order, double gamma, double ell_hat);

/* dUdt = L(U): the right-hand side on the whole grid.  U and dUdt are distinct
 * device buffers of nvar * ncells float64 (aliasing is rejected). */
int kfvm_rhs(kfvm_ctx *ctx, const double *U, double *dUdt);

/* One SSP-RK3 step of size dt on U, in place:
 *   U1 = U + dt L(U),  U2 = 3/4 U + 1/4 (U1 + dt L(U1)),  U <- 1/3 U + 2/3 (U2 + dt L(U2)).
 * If any stage meets a non-physical state (a cell average or reconstructed
 * state with rho <= 0, p <= 0 or a non-finite value, or a non-finite flux), U is
 * left unmodified and KFVM_ERR_NONPHYSICAL is reported by kfvm_status /
 * kfvm_stats (or returned, see kfvm_set_checking).  The decision is taken on
 * the device, in stream order: the call does not synchronise for it. */
int kfvm_step(kfvm_ctx *ctx, double *U, double dt);

/* One step of SSP(4,3,2) (section 6): the four-stage third-order SSP Runge-Kutta
 * method of Kraaijevanger, with h = dt / 2,
 *   U1 = U + h L(U),  U2 = U1 + h L(U1),  U3 = 2/3 U + 1/3 (U2 + h L(U2)),
 *   U_out = U3 + h L(U3),
 * and the embedded three-stage second-order SSP method, which shares the first
 * stages: Uhat = 1/3 U + 2/3 (U2 + h L(U2)) = 2 U3 - U.  *err_host (host memory)
 * receives the root mean square over every (variable, cell) of
 * (U_out - Uhat) / (atol + rtol max(|U|, |U_out|)), for error-based step-size
 * control by the caller (accept when it is at most one).  U is not modified;
 * U and U_out are distinct device buffers of nvar * ncells float64.
 * Synchronising; returns KFVM_ERR_NONPHYSICAL if a stage met a non-physical
 * state.  atol, rtol >= 0 with atol + rtol > 0. */
int kfvm_step_ssp432(kfvm_ctx *ctx, const double *U, double *U_out, double dt, double atol, double rtol,
                     double *err_host);

/* dt = cfl / max_cells sum_a (|u_a| + c_s) / dx_a.  Synchronising; the result is
 * written to host memory. */
int kfvm_cfl_dt(kfvm_ctx *ctx, const double *U, double cfl, double *dt_host);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): kfvm_cfl_dt with its result
 * left in device memory and no allocation of any kind in the call.
 * out_dev: caller-owned device buffer of 3 float64 on the context's device;
 * out_dev[0] = cfl / max_c sum_d (|u_d| + c_s) / Delta_d (or the largest-axis
 * form, kfvm_set_cfl_form), out_dev[1] and out_dev[2] the least density and
 * pressure over the admissible cells: the values kfvm_cfl_dt computes, by the
 * same kernels.  U: device, nvar * ncells float64.  Enqueued on the context's
 * stream; nothing is copied to the host and the call does not synchronise
 * (kfvm_stats' min_rho / min_p are not updated).  A non-admissible cell raises
 * the sticky KFVM_ERR_NONPHYSICAL word (kfvm_status), as kfvm_cfl_dt does.
 * Scratch: the reduction's 1024 per-block partials (3 float64 each) sit in a
 * library-wide device array of 24 KiB, one per GPU, held until the process
 * ends; any grid size fits, since the reduction strides over the grid.  Every
 * call on one GPU shares that array: calls that overlap on one GPU (other
 * streams, other threads) race.  Errors: KFVM_ERR_STATE (null context),
 * KFVM_ERR_ARG (null pointer, cfl <= 0), KFVM_ERR_HIP (launch). */
int kfvm_cfl_dt_noalloc(kfvm_ctx *ctx, const double *U, double cfl, double *out_dev);

/* Queue subsequent work on this HIP stream (hipStream_t passed as void*). */
int kfvm_set_stream(kfvm_ctx *ctx, void *hip_stream);

/* Arithmetic of the weight-apply and smoothness-indicator contractions:
 * KFVM_FP64 (default), or split hi/lo half-precision operands on the matrix
 * cores with float32 accumulation (KFVM_SPLIT_F16, KFVM_SPLIT_BF16); the
 * nonlinear-weight normalisation, the limiter, the Riemann fluxes and the
 * Runge-Kutta update stay in float64 (the split modes take the Riemann
 * solver's wave-speed estimates S_L, S_R in float32: the fluxes move by their
 * rounding times the jump between the two states).  The split modes need fewer
 * than 2^27 (about 1.3e8, a 512^3 grid) cells (KFVM_ERR_ARG otherwise). */
int kfvm_set_precision(kfvm_ctx *ctx, int mode);

/* Boundary conditions of one axis (section 5.3: ghost cells filled by them,
 * step 1; Riemann states outside the domain from the inner ones, step 4).
 * lower, upper: KFVM_BC_PERIODIC on both sides (the default), or per side
 *  - KFVM_BC_OUTFLOW: ghost cells copy the nearest interior cell (zero-order
 *    extrapolation); the outer Riemann state is the inner one;
 *  - KFVM_BC_REFLECTING: ghost cells are the mirror images with the normal
 *    momentum negated; so is the outer Riemann state;
 *  - KFVM_BC_INFLOW: ghost cells and outer Riemann states take the given state,
 *    lower_state / upper_state: host pointers to nvar conserved values (ignored
 *    for other kinds; the library copies them).
 * At a corner ghost cell the first inflow axis in x, y, z order gives the state,
 * otherwise every axis clamps or mirrors its index; the normal momentum of every
 * reflecting axis is then negated.  The KXRCF jump at a boundary face is taken
 * against the outer state; the learned gate sees the ghost-filled averages.
 * Every precision mode supports them.  Errors: KFVM_ERR_ARG (axis, kind,
 * periodic on one side only, missing inflow state), KFVM_ERR_NONPHYSICAL (an
 * inflow state with rho <= 0 or p <= 0).
 * The first non-periodic axis allocates dim * nvar * (largest boundary plane)
 * float64 of boundary-face fluxes. */
int kfvm_set_boundary(kfvm_ctx *ctx, int axis, int lower, int upper, const double *lower_state,
                      const double *upper_state);

/* Positivity limiter of section 4: enabled != 0 turns it on; the bounds are
 * the 3^d neighbourhood's extrema widened by the factor (1 +- kappa (1 - eta)),
 * 0 <= kappa < 1, with the flattener eta = 0 unless kfvm_set_flattener turns
 * it on. */
int kfvm_set_limiter(kfvm_ctx *ctx, int enabled, double kappa);

/* The limiter's flattener eta (section 4: rho_max (1 + kappa - kappa eta),
 * rho_min and p_min (1 - kappa + kappa eta), eta tending to one where the flow
 * compresses).  The paper takes eta's rule from a cited reference; this library
 * reads it as a ramp in the undivided velocity divergence
 * d = sum_a (v_a(c + e_a) - v_a(c - e_a)) / 2 (neighbours through the ghost
 * fill) against the least sound speed c_min of the cell's 3^d block:
 * eta = min(1, max(0, -d / (k1 c_min) - 1)).  k1 > 0 turns it on with that
 * onset; k1 = 0 (the default) gives eta = 0.  Every precision mode supports it.
 * Errors: KFVM_ERR_ARG (k1 negative or not finite). */
int kfvm_set_flattener(kfvm_ctx *ctx, double k1);

/* The formula of kfvm_cfl_dt (section 6 caps steps by a CFL number without
 * stating one): KFVM_CFL_SUM (default) takes dt = cfl / max over cells of
 * sum_a (|u_a| + c) / dx_a, KFVM_CFL_MAX_AXIS the largest single term instead
 * (steps up to dim times longer).  Errors: KFVM_ERR_ARG (unknown form). */
int kfvm_set_cfl_form(kfvm_ctx *ctx, int form);

/* KFVM_HLLC (default) or KFVM_HLL (section 6). */
int kfvm_set_riemann(kfvm_ctx *ctx, int solver);

/* checking != 0: kfvm_rhs and kfvm_step synchronise the stream and return
 * KFVM_ERR_NONPHYSICAL if the device raised it (the flag is then cleared). */
int kfvm_set_checking(kfvm_ctx *ctx, int checking);

/* Synchronise; return and clear the sticky device error code. */
int kfvm_status(kfvm_ctx *ctx);

/* Synchronise and fill *out. */
int kfvm_stats(kfvm_ctx *ctx, kfvm_stats_t *out);

/* Test hook: the limited Riemann states of the last kfvm_rhs input, converted to
 * conserved variables, as states[cell][s][v] (device buffer of ncells * n_pts *
 * nvar float64).  Recomputes them from U. */
int kfvm_face_states(kfvm_ctx *ctx, const double *U, double *states);

/* Build the reconstruction tables of (dim, R) with kernel length scale ell_hat
 * (in cells; the paper uses 5) into tables[capacity], layout as in kfvm_weights.
 * Returns the number of float64 written, or a negative code. Host only. */
int kfvm_weights_build(int dim, int R, double ell_hat, double *tables, int capacity);

/* Number of float64 in the tables of (dim, R), or a negative code. */
int kfvm_weights_size(int dim, int R);

/* Per-(variable, cell) reconstruction choice, a caller-owned device array
 * flags[nvar][ncells] of bytes: nonzero = WENO-AO (section 3.2), 0 = the linear
 * full-stencil value (what a troubled-cell gate decides; section 3.5 describes
 * the paper's own indicator).  NULL (the default) = WENO-AO everywhere.  The
 * array must stay valid while work that reads it is queued.  A non-NULL array
 * turns the gate and the indicator off. */
int kfvm_set_flags(kfvm_ctx *ctx, const uint8_t *flags);

/* ---- KXRCF troubled-cell indicator (section 3.5, eq. kxrcf) ----------------
 * The two-pass Riemann-state procedure of section 5.3.  First pass: unlimited
 * states from the full stencil S0 (its face-point rows applied to the conserved
 * averages) at the Gauss points of every face, from both sides.  A cell takes
 * the linear S0 value for all its variables when
 *     max_s |q+_s - q-_s| / <Q>  <  Delta^m,
 * s over the Gauss points of its 2 dim faces, q = p / rho^gamma of the state
 * from the cell (-) and from the neighbour across the face (+), <Q> the same of
 * the cell's average, Delta the cell width (the largest dx); otherwise WENO-AO
 * for all its variables.  A cell whose average or any of those point states has
 * rho <= 0 or p <= 0 is flagged.  The first pass runs in float64 in either
 * precision mode. */

/* kind = KFVM_IND_KXRCF: every subsequent kfvm_rhs, kfvm_step stage and
 * kfvm_face_states runs the indicator on its input and reconstructs with its
 * decisions; m > 0 is the power of Delta (the paper uses 3/2).  Turns the gate
 * and kfvm_set_flags off.  KFVM_IND_NONE (the default) turns it off.  Allocates
 * dim * ncells float64 of jumps and nvar * ncells bytes of flags on first use. */
int kfvm_set_indicator(kfvm_ctx *ctx, int kind, double m);

/* Run the indicator once on U with power m: jumps[dim][ncells] float64 (optional
 * device buffer) receives, per axis a, the largest |q+ - q-| over the Gauss points
 * of each cell's upper face along a (infinity where a state is not admissible);
 * flags[nvar][ncells] bytes (optional device buffer) the decisions, 1 = WENO-AO.
 * With NULL outputs the context's own buffers receive them (kfvm_get_flags
 * reads the flags).  Asynchronous. */
int kfvm_kxrcf(kfvm_ctx *ctx, const double *U, double m, double *jumps, uint8_t *flags);

/* ---- learned troubled-cell gate -------------------------------------------
 * A small network decides per (variable, cell) whether the WENO-AO machinery
 * (substencils, smoothness indicators, nonlinear weights; section 3.2-3.3) is
 * needed or the linear full-stencil value suffices, in place of the paper's
 * KXRCF indicator (section 3.5).  Network: n_in -> 32 -> 32 -> 1 logit, GELU
 * (tanh form) after both hidden layers; n_in = 25 in 2D (the 5 x 5 window of the
 * variable around the cell, offsets lexicographic with x slowest) and 33 in 3D
 * (the radius-2 sphere S0 in its stencil order).  Inputs: increments W_h - W_c
 * of the linearised primitive variable divided by 2^ex, where max|W_h - W_c| lies
 * in [2^(ex-1), 2^ex).  Parameters: one float32 vector W1[32][n_in], b1[32],
 * W2[32][32], b2[32], w3[32], b3.  Inference runs the hidden layers on BF16
 * matrix cores with float32 accumulation (inputs, W1, W2 and the first hidden
 * activations rounded to BF16); training keeps float32 masters. */

/* Sizes of the gate network for dim (host only). */
int kfvm_mlp_sizes(int dim, int *n_in, int *n_params);

/* Enable the gate in the split-precision path: params is a device float32
 * vector (copied), a (variable, cell) takes WENO-AO when its logit exceeds
 * threshold and its largest S0 increment exceeds 2^-40 of the variable's scale
 * (density, sound speed or pressure of the cell; below that every stencil holds
 * W_c to rounding and WENO-AO equals the linear value).  params == NULL
 * disables it.  Clears kfvm_set_flags. */
int kfvm_set_gate(kfvm_ctx *ctx, const float *params, float threshold);

/* Copy the decisions of the last gated or indicator-driven reconstruction (or
 * of the last kfvm_kxrcf without a flags buffer), flags[nvar][ncells] bytes
 * (1 = WENO-AO), to a device buffer (asynchronous). */
int kfvm_get_flags(kfvm_ctx *ctx, uint8_t *flags);

/* Training samples from state U: x[nvar][ncells][n_in] float32 gate inputs and
 * ratio[nvar][ncells] float32 = omega_0 / gamma_0 of the FP64 WENO-AO
 * reconstruction (eq. nlinWts; 1 where the variable is linear).  Device buffers;
 * x may be NULL (the labels alone, e.g. to measure the gate's misclassification). */
int kfvm_gate_samples(kfvm_ctx *ctx, const double *U, float *x, float *ratio);

/* One training step on a batch of B samples x[B][n_in], labels y[B] in {0, 1}
 * (device buffers): mean loss pos_weight y softplus(-z) + (1 - y) softplus(z) of
 * the logit z, its gradient (straight through the BF16 roundings), reduced in
 * a fixed order, and, if lr > 0, one Adam step (beta 0.9, 0.999, eps 1e-8, bias
 * corrected at step t >= 1) on params with moments adam_m, adam_v.  loss (one
 * float), grad (n_params) and logits (B) are optional outputs; y may be NULL
 * when lr == 0. */
int kfvm_mlp_train_step(kfvm_ctx *ctx, const float *x, const float *y, int B, float *params, float *adam_m,
                        float *adam_v, int t, float lr, float pos_weight, float *loss, float *grad, float *logits);

/* on != 0: bracket every subsequent kernel launch with HIP events on the
 * context's stream (adds a few microseconds per launch). */
int kfvm_set_timing(kfvm_ctx *ctx, int on);

/* Synchronise; write the summed device time in milliseconds and the launch
 * count of each kernel class since the last call (index 0: reconstruction,
 * 1: face flux, 2: flux difference and stage update, 3: the KXRCF indicator's
 * first pass and flags) into ms[n], launches[n] (n >= 4), and forget the
 * recorded events. */
int kfvm_kernel_times(kfvm_ctx *ctx, double *ms, long long *launches, int n);

/* Message of the last error on this context (never NULL). */
const char *kfvm_last_error(const kfvm_ctx *ctx);

/* Free the context and its device memory (after synchronising its stream). */
void kfvm_destroy(kfvm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* KFVM_H */
