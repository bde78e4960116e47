// Internal interface between the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kfvm {

// Boundary conditions per axis and side (section 5.3, steps 1 and 4).
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECTING = 2, BC_INFLOW = 3 };

struct Geom {
    int n[3];          // cells per axis (n[2] = 1 in 2D)
    long ncell;
    double dx[3];
    double gamma;
    int periodic;               // every axis periodic: ghost cells are a plain index wrap
    int cfl_max_axis;           // CFL step: 0 the sum over axes of (|u_a| + c) / dx_a, 1 its largest term
    int bc[3][2];               // BC_* per axis and side (lower, upper)
    double bc_state[3][2][5];   // conserved inflow state per axis and side
};

struct Limiter {
    int on;
    double kappa;
    double flat_k1;     // > 0: the flattener eta narrows the kappa widening (flattener_eta); 0: eta = 0
};

// Device buffers owned by a context.
struct Work {
    double *face;      // [n_pts][nvar][ncell] Riemann states in reconstruction variables
    double *theta;     // [2][ncell] density and pressure scaling of the limiter
    double *fbar;      // [dim][nvar][ncell] Gauss-integrated flux through each cell's lower faces
    double *stage[2];  // [nvar][ncell] Runge-Kutta stage states
    double *cfl_part;  // per-block maxima of the CFL reduction
    int *err;          // device error code the kernels raise (sticky word, or a step's own word)
    const int *guard;  // optional: the update writes nothing while *guard != 0 (a step's last stage)
    unsigned long long *counts;  // [2] scratch of kfvm_stats: limiter cells, WENO (cell, var) pairs
    const uint8_t *flags_in;   // optional [nvar][ncell] gate decisions (1 = WENO)
    float *inc32;      // blended increments w_s - W_c (split-precision path), inc_index layout
    double *fbar_top;  // [dim][nvar][plane] fluxes through the upper boundary faces of non-periodic axes
    long plane;        // largest boundary plane (cells), the stride of fbar_top
};

// Layout of the split path's float32 face-point increments: points in groups of
// four, each cell's group one 16-byte vector,
// [point / 8][nvar][(point / 4) % 2][ncell][point % 4].  A half-wave holds a
// cell's four consecutive points tau .. tau + 3 (tau a multiple of 4) and
// writes them with one vector store; the other half-wave's group, tau + 4 when
// bit 2 of tau is clear, lies 4 ncell floats away.  inc_index gives the offset
// of (point, variable) for cell 0; cell c adds 4 c.  inc_points: the allocated
// point count (n_pts rounded up to whole groups of eight).
__host__ __device__ constexpr long inc_index(int tau, int v, int nvar, long ncell)
{
    return ((long)((tau >> 3) * nvar + v) * 2 + ((tau >> 2) & 1)) * ncell * 4 + (tau & 3);
}
__host__ __device__ constexpr int inc_points(int npts) { return (npts + 7) / 8 * 8; }

// index of a cell in the boundary plane of axis a: its other two coordinates, the lower axis fastest
__host__ __device__ inline long plane_index(int a, int cx, int cy, int cz, const int *n)
{
    return a == 0 ? cy + (long)n[1] * cz : (a == 1 ? cx + (long)n[0] * cz : cx + (long)n[0] * cy);
}

// Matrix-core operands of the split-precision path, in the per-lane layout of
// v_mfma_f32_32x32x16: [tile][k-step][hi, lo][lane] slots of 8 16-bit values.
struct MixTables {
    const uint4 *full;   // every stencil, rows interleaved as target * 8 + stencil
    const uint4 *lin;    // S0 face-point rows only
    int sw;              // weights are scaled by 2^sw
};

struct Tables {
    const double *w;      // packed reconstruction tables (device)
    const double *wch;    // the same in chunk layout (ChunkLayout<3, 3, 8>), 3D R = 3 only
};

constexpr int FP64_CHUNK = 8;    // members per chunk of the chunked FP64 reconstruction

// Optional per-kernel timing: when `on`, every launch is bracketed by HIP events
// on the launch stream; the host sums the elapsed times later.
enum { KT_RECON = 0, KT_FLUX = 1, KT_UPDATE = 2, KT_INDICATOR = 3, KT_COUNT = 4 };
struct Timing {
    int on;
    void (*record)(void *self, int kind, hipStream_t s, int begin);
    void *self;
};

// Launchers, one per (dim, R); all asynchronous on `s`.
// stage: 0 -> out = L(Uin); 1, 2, 3 -> the SSP-RK3 stage combinations with U0
// (1 is also Uin + dt L(Uin) of SSP(4,3)); 4 -> 2/3 U0 + 1/3 (Uin + dt L(Uin)).
hipError_t launch_rhs_fp64(int dim, int R, const Geom &g, const Tables &t, const Work &w, const Limiter &lim,
                           int riemann, const double *U0, const double *Uin, double *out, int stage, double dt,
                           hipStream_t s, const Timing &tm);
hipError_t launch_update(int dim, const Geom &g, const Work &w, const double *U0, const double *Uin, double *out,
                         int stage, double dt, hipStream_t s);
// *word = 0, and (merge) *sticky = *word where it is set: one thread each, so a
// caller's stream order keeps them and no memset node enters a captured graph
hipError_t launch_err_reset(int *word, hipStream_t s);
hipError_t launch_err_merge(int *sticky, const int *word, hipStream_t s);
// Learned troubled-cell gate fused into the split-precision reconstruction
// (w == nullptr: no gate).  w: BF16 operand slots of W1 and W2 (8 values per lane
// and slot, see rhs_mixed.hip); vec: b1[32], b2[32], w3[32], b3.
struct GateArgs {
    const uint4 *w;
    const float *vec;
    float thr;
    uint8_t *flags_out;   // [nvar][ncell] decisions of the last evaluation (1 = WENO-AO)
    uint8_t *raw;         // [ncell] network decisions, bit v per variable (3D order 7: before dilation)
};

bool mixed_supported(int dim, int R);
int gate_operand_slots(int dim);
int gate_slot_input(int dim, int k);   // network input fed by W1 operand column k, or -1
int gate_w1_exp(int dim);              // power of two folded into the W1 operand
int mixed_operand_slots(int dim, int R, int which);   // which: 0 full, 1 lin; 16-byte slots
hipError_t launch_rhs_mixed(int dim, int R, bool bf16, const Geom &g, const MixTables &t, const Work &w,
                            const Limiter &lim, int riemann, const double *U0, const double *Uin, double *out,
                            int stage, double dt, double *states, hipStream_t s, const Timing &tm,
                            const GateArgs &ga);
hipError_t launch_face_states(int dim, int R, const Geom &g, const Tables &t, const Work &w, const Limiter &lim,
                              const double *U, double *states, hipStream_t s);
hipError_t launch_cfl(int dim, const Geom &g, const Work &w, const double *U, double cfl, double *dt_dev,
                      hipStream_t s);
// The same reduction with its per-block partials in the library's static
// device array (rhs_fp64.hip): cfl_scratch_address gives that array's address
// on the current device (looked up once per device), which launch_cfl_scratch
// takes as scratch_dev.  No allocation.
constexpr int CFL_PARTS = 1024;                    // per-block partials of the CFL reduction
constexpr int CFL_SCRATCH_DOUBLES = 3 * CFL_PARTS;
constexpr int MAX_DEVICES = 64;
hipError_t cfl_scratch_address(double **ptr);
hipError_t launch_cfl_scratch(int dim, const Geom &g, double *scratch_dev, int *err, const double *U, double cfl,
                              double *out_dev, hipStream_t s);
// SSP(4,3,2): *out = root mean square over M values of (Up - (2 U3 - U)) /
// (atol + rtol max(|U|, |Up|)); part: at least 1024 doubles of scratch.
hipError_t launch_ssp_error(const double *U, const double *U3, const double *Up, long M, double atol, double rtol,
                            double *part, double *out, hipStream_t s);
// counts[0] += cells with a limiter factor below one (theta[2][ncell]);
// counts[1] += nonzero bytes of flags[nvar][ncell] (skipped when flags is null)
hipError_t launch_count_stats(const double *theta, const uint8_t *flags, long ncell, int nvar,
                              unsigned long long *counts, hipStream_t s);

// KXRCF indicator (kxrcf.hip): jumps J[dim][ncell] of the upper faces, then
// (flags != nullptr) flags[nvar][ncell] = 1 where eq. kxrcf fails for threshold thr.
// kw: the S0 face-point rows laid out [axis][side][member][Gauss point], side 0
// the upper face of the cell, side 1 the lower face of its upper neighbour.
// Non-periodic grids: the jumps at boundary faces come from the outer states the
// boundary conditions give (upper faces into J, lower faces into Jlo[dim][plane],
// plane stride `plane`); w0: the FP64 tables (stencil 0 leads).
int kxrcf_table_size(int dim, int R);
hipError_t launch_kxrcf(int dim, int R, const Geom &g, const double *kw, const double *w0, const double *U, double *J,
                        double *Jlo, long plane, uint8_t *flags, double thr, hipStream_t s);

// gate network: training and sample export (mlp.hip)
int mlp_n_in(int dim);
int mlp_n_params(int dim);
size_t mlp_workspace_floats(int dim, int B);
hipError_t launch_gate_inputs(int dim, const Geom &g, const double *U, float *x, hipStream_t s);
hipError_t launch_mlp_train(int dim, const float *x, const float *y, int B, float *prm, float *m, float *v, int t,
                            float lr, float pos_weight, float *loss, float *grad, float *logits, float *ws,
                            hipStream_t s);
hipError_t launch_recon_ratio(int dim, int R, const Geom &g, const Tables &t, const Work &w, const Limiter &lim,
                              const double *U, float *ratio, hipStream_t s);

}  // namespace kfvm
