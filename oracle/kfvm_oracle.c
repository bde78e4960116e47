/*
 * Oracle: KFVM-WENO right-hand side, positivity limiter, Riemann solvers and
 * SSP-RK3 step for the compressible Euler equations on a uniform
 * Cartesian grid (periodic, or with outflow, reflecting and inflow
 * boundaries), in plain binary64 C.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link or call this
 * library; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code with the GPU library.
 *
 * It follows the paper's order of operations (section 5.3 "Time advancement"):
 * for every cell
 *   1. ghost cells: index wrap on periodic axes, the boundary conditions on the
 *      others (neighbor_state);
 *   2. Riemann states: the transformation matrix Phi of the linearised
 *      primitive variables from the cell's own average (section 3.4.2,
 *      eq. consToLPMat), W_h = Phi U_h over S0 (eq. consToRecVar), per
 *      component and per (sub)stencil the point values r.g and derivative
 *      values (eq. reconVec), the smoothness indicators (eq. smoothIndic, with no
 *      extra grid factor), the WENO-JS form weights (eq. nlinWts, eps = 1e-40),
 *      the WENO-AO blend (eq. wenoAOrec), then u_s = Phi^-1 w_s
 *      (eq. recVarToCons, eq. lpToConsMat);
 *   3. the positivity limiter of section 4 (density scaling eq. ppThetaRho and
 *      eq. ppCorrectDens, pressure scaling by bisection eq. thetapRoot, eq. thetaP
 *      and eq. ppCorrectPres), with kappa a parameter and the flattener eta
 *      either 0 or the compression ramp of flattener() below;
 *   4. Riemann states outside the domain from the inner ones at boundary
 *      faces (ghost_face_states);
 *   5. an approximate Riemann solver at every face Gauss point: HLLC (Toro,
 *      "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 10) or HLL
 *      (Harten, Lax and van Leer 1983), with the wavespeed estimates of Batten et
 *      al. (1997) from Roe averages (section 6);
 *   6. Gauss-Legendre face integral of the fluxes and the flux difference.
 * With the KXRCF indicator on (section 3.5 "Local smoothness indicators" and
 * the two-pass procedure of section 5.3), step 2 first forms unlimited states
 * from S0 on every cell and flags the cells whose relative entropy jump across
 * a face reaches Delta^m (eq. kxrcf); only flagged cells take WENO-AO.
 * The time step is the three-stage SSP Runge-Kutta method of Shu and Osher
 * (1988).  Its stages are written out literally.
 *
 * Data layout: U[v][z][y][x] with x fastest (struct of arrays); 2D grids have
 * nz = 1 and 4 variables (rho, rho u, rho v, E), 3D grids 5 (rho, rho u, rho v,
 * rho w, E).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXD 3
#define MAXV 5
#define MAXST 8

enum { OK = 0, ERR_ARG = -1, ERR_NONPHYSICAL = -3 };

typedef struct {
    int dim, R, nvar;
    int n[3];              /* cells per axis; n[2] = 1 in 2D */
    double dx[3];          /* grid spacing per axis */
    double gamma;          /* ratio of specific heats */
    int n0;                /* |S0| */
    const int *s0;         /* [n0][dim] unit-cell offsets of S0 */
    int nst;               /* number of (sub)stencils: 2 + 2 dim */
    const int *mem_ptr;    /* [nst + 1] start of each member list in mem */
    const int *mem;        /* member indices into S0 */
    const int *w_ptr;      /* [nst] start of each stencil's table in w */
    const double *w;       /* row-major tables [n_pts + n_der][N_q] */
    const double *lin_w;   /* [nst] linear weights gamma_q */
    int n_pts, n_der;      /* face points per cell, derivative rows */
    const double *gl_w;    /* [R] Gauss-Legendre weights on [-1/2, 1/2], summing to 1 */
    double eps;            /* epsilon of the nonlinear weights */
    int limiter;           /* 0: off, 1: on */
    double kappa;          /* bound widening of the limiter */
    int riemann;           /* 0: HLLC, 1: HLL */
    int weno;              /* 1: WENO-AO; 0: linear S0 reconstruction only */
    const uint8_t *flags;  /* optional [nvar][cells]: 1 = WENO, 0 = linear (gate replay) */
    double kxrcf_m;        /* > 0: the KXRCF indicator with threshold Delta^m picks the WENO cells */
    int bc[3][2];          /* boundary condition per axis and side (lower, upper): BC_* below */
    double bc_state[3][2][MAXV];   /* conserved inflow state per axis and side */
    double flat_k1;        /* > 0: the flattener eta of the limiter bounds (flattener()); 0: eta = 0 */
    int cfl_max_axis;      /* CFL step: 0 the sum over axes of (|u_a| + c) / dx_a, 1 its largest term */
} oracle_ctx;

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECTING = 2, BC_INFLOW = 3 };

/* ---------------------------------------------------------------- grid --- */
static long ncells(const oracle_ctx *c) { return (long)c->n[0] * c->n[1] * c->n[2]; }

static long wrap_index(const oracle_ctx *c, long cell, const int *off)
{
    long i = cell % c->n[0], j = (cell / c->n[0]) % c->n[1], k = cell / ((long)c->n[0] * c->n[1]);
    long o[3] = {0, 0, 0};
    for (int a = 0; a < c->dim; ++a) o[a] = off[a];
    i = ((i + o[0]) % c->n[0] + c->n[0]) % c->n[0];
    j = ((j + o[1]) % c->n[1] + c->n[1]) % c->n[1];
    k = ((k + o[2]) % c->n[2] + c->n[2]) % c->n[2];
    return i + c->n[0] * (j + c->n[1] * k);
}

static void load_cell(const oracle_ctx *c, const double *U, long cell, double *u)
{
    long N = ncells(c);
    for (int v = 0; v < c->nvar; ++v) u[v] = U[v * N + cell];
}

/* ------------------------------------------------- boundary conditions --- */
/* The average of the cell at offset off from `cell`, through the boundary
 * conditions (the ghost fill of section 5.3, step 1).  Along a periodic axis the
 * index wraps.  Past a non-periodic boundary the ghost cell is the nearest
 * interior cell (outflow: zero-order extrapolation), the mirror-image cell
 * (reflecting) or the given state (inflow).  When several axes leave the grid
 * (a corner ghost), the first inflow axis in x, y, z order gives the state,
 * otherwise every axis clamps or mirrors its index; the normal momentum of
 * every reflecting axis is then negated. */
static void neighbor_state(const oracle_ctx *c, const double *U, long cell, const int *off, double *u)
{
    long idx[3] = {cell % c->n[0], (cell / c->n[0]) % c->n[1], cell / ((long)c->n[0] * c->n[1])};
    int flip[3] = {0, 0, 0}, fixed = -1;
    for (int a = 0; a < c->dim; ++a) {
        long g = idx[a] + off[a], n = c->n[a];
        if (g >= 0 && g < n) {
            idx[a] = g;
            continue;
        }
        int side = g < 0 ? 0 : 1, kind = c->bc[a][side];
        if (kind == BC_PERIODIC) {
            idx[a] = ((g % n) + n) % n;
        } else if (kind == BC_OUTFLOW) {
            idx[a] = side ? n - 1 : 0;
        } else if (kind == BC_REFLECTING) {
            idx[a] = side ? 2 * n - 1 - g : -1 - g;
            flip[a] = 1;
        } else {
            if (fixed < 0) fixed = 2 * a + side;
            idx[a] = side ? n - 1 : 0;
        }
    }
    if (fixed >= 0)
        for (int v = 0; v < c->nvar; ++v) u[v] = c->bc_state[fixed / 2][fixed % 2][v];
    else
        load_cell(c, U, idx[0] + c->n[0] * (idx[1] + (long)c->n[1] * idx[2]), u);
    for (int a = 0; a < c->dim; ++a)
        if (flip[a]) u[1 + a] = -u[1 + a];
}

/* Does the face of `cell` on this side of axis a lie on a non-periodic boundary? */
static int on_boundary(const oracle_ctx *c, long cell, int a, int side)
{
    if (c->bc[a][side] == BC_PERIODIC) return 0;
    long i = a == 0 ? cell % c->n[0] : (a == 1 ? (cell / c->n[0]) % c->n[1] : cell / ((long)c->n[0] * c->n[1]));
    return side ? i == c->n[a] - 1 : i == 0;
}

/* Riemann states outside the domain (section 5.3, step 4): at the Gauss points of
 * the boundary face on this side of axis a, the outer state from the inner one
 * (outflow: the same; reflecting: normal momentum negated; inflow: the given
 * state), written where face_flux reads the outer cell's states: the upper face
 * rows of a ghost below (side 0), the lower face rows of a ghost above (side 1). */
static void ghost_face_states(const oracle_ctx *c, int a, int side, const double *own, double *ghost)
{
    int nv = c->nvar, ng = c->n_pts / (2 * c->dim);
    for (int g = 0; g < ng; ++g) {
        const double *in = own + ((2 * a + side) * ng + g) * nv;
        double *out = ghost + ((2 * a + 1 - side) * ng + g) * nv;
        int kind = c->bc[a][side];
        for (int v = 0; v < nv; ++v) out[v] = kind == BC_INFLOW ? c->bc_state[a][side][v] : in[v];
        if (kind == BC_REFLECTING) out[1 + a] = -out[1 + a];
    }
}

/* ----------------------------------------------------------------- EOS --- */
/* p = (gamma - 1) (E - rho |u|^2 / 2) (section 1, eq. euler) */
static double pressure(const oracle_ctx *c, const double *u)
{
    double ke = 0.0;
    for (int a = 0; a < c->dim; ++a) ke += u[1 + a] * u[1 + a];
    ke = 0.5 * ke / u[0];
    return (c->gamma - 1.0) * (u[c->dim + 1] - ke);
}

static int admissible(const oracle_ctx *c, const double *u)
{
    for (int v = 0; v < c->nvar; ++v)
        if (!isfinite(u[v])) return 0;
    return u[0] > 0.0 && pressure(c, u) > 0.0;
}

/* ----------------------------------------------------------- flattener --- */
/* The flattener eta of the limiter bounds (section 4).  The paper takes kappa
 * and eta from a rule it cites but does not state; this is a reading: eta
 * rises from 0 to 1 with the compression of the flow at the cell, measured by
 * the undivided velocity divergence
 *     d = sum_a (v_a(c + e_a) - v_a(c - e_a)) / 2
 * (neighbours through the ghost fill) against the least sound speed c_min of
 * the 3^d block:
 *     eta = min(1, max(0, -d / (k1 c_min) - 1)),
 * so eta = 0 wherever d >= -k1 c_min (expansion, uniform or mildly compressed
 * flow: the bounds keep their kappa widening) and eta = 1 wherever
 * d <= -2 k1 c_min (strong compression: the bounds are the neighbourhood's own
 * extrema).  k1 = flat_k1; without it eta = 0.  Every state of the block must be
 * admissible (the caller has checked). */
static double flattener(const oracle_ctx *c, const double *U, long cell)
{
    if (!(c->flat_k1 > 0.0)) return 0.0;
    double d = 0.0;
    for (int a = 0; a < c->dim; ++a) {
        int op[3] = {0, 0, 0}, om[3] = {0, 0, 0};
        op[a] = 1;
        om[a] = -1;
        double up[MAXV], um[MAXV];
        neighbor_state(c, U, cell, op, up);
        neighbor_state(c, U, cell, om, um);
        d += 0.5 * (up[1 + a] / up[0] - um[1 + a] / um[0]);
    }
    double cmin = INFINITY;
    int lo[3] = {-1, -1, -1}, hi[3] = {1, 1, 1};
    if (c->dim < 3) lo[2] = hi[2] = 0;
    for (int dz = lo[2]; dz <= hi[2]; ++dz)
        for (int dy = lo[1]; dy <= hi[1]; ++dy)
            for (int dx = lo[0]; dx <= hi[0]; ++dx) {
                int off[3] = {dx, dy, dz};
                double un[MAXV];
                neighbor_state(c, U, cell, off, un);
                double cs = sqrt(c->gamma * pressure(c, un) / un[0]);
                if (cs < cmin) cmin = cs;
            }
    double eta = -d / (c->flat_k1 * cmin) - 1.0;
    return eta < 0.0 ? 0.0 : (eta > 1.0 ? 1.0 : eta);
}

/* ----------------------------------------- linearised primitive variables --- */
/* Phi = dV/dU at the reference state (eq. consToLPMat); in 2D the u_3 row and
 * column are dropped.  Dense nvar x nvar matrices, row-major. */
static void phi_matrices(const oracle_ctx *c, const double *ref, double *Phi, double *Phi_inv)
{
    int d = c->dim, nv = c->nvar, e = d + 1;
    double g = c->gamma, rho = ref[0], u[MAXD], uu = 0.0;
    for (int a = 0; a < d; ++a) { u[a] = ref[1 + a] / rho; uu += u[a] * u[a]; }
    memset(Phi, 0, sizeof(double) * nv * nv);
    memset(Phi_inv, 0, sizeof(double) * nv * nv);
    Phi[0 * nv + 0] = 1.0;
    for (int a = 0; a < d; ++a) {
        Phi[(1 + a) * nv + 0] = -u[a] / rho;
        Phi[(1 + a) * nv + 1 + a] = 1.0 / rho;
        Phi[e * nv + 1 + a] = (1.0 - g) * u[a];
    }
    Phi[e * nv + 0] = (g - 1.0) * uu / 2.0;
    Phi[e * nv + e] = g - 1.0;
    /* Phi^-1 = dU/dV (eq. primMat).  The energy row holds dE/du_i = rho u_i:
     * the matrix printed as eq. lpToConsMat shows u_i there, which is not the
     * inverse of eq. consToLPMat; the definition as the exact inverse wins. */
    Phi_inv[0 * nv + 0] = 1.0;
    for (int a = 0; a < d; ++a) {
        Phi_inv[(1 + a) * nv + 0] = u[a];
        Phi_inv[(1 + a) * nv + 1 + a] = rho;
        Phi_inv[e * nv + 1 + a] = rho * u[a];
    }
    Phi_inv[e * nv + 0] = uu / 2.0;
    Phi_inv[e * nv + e] = 1.0 / (g - 1.0);
}

static void matvec(int nv, const double *A, const double *x, double *y)
{
    for (int i = 0; i < nv; ++i) {
        double s = 0.0;
        for (int j = 0; j < nv; ++j) s += A[i * nv + j] * x[j];
        y[i] = s;
    }
}

/* --------------------------------------------- Riemann states of one cell --- */
/* states: [n_pts][nvar].  Returns OK or ERR_NONPHYSICAL. */
static int cell_states_ex(const oracle_ctx *c, const double *U, long cell, double *states, float *ratio,
                          double *betas);

static int cell_states(const oracle_ctx *c, const double *U, long cell, double *states)
{
    return cell_states_ex(c, U, cell, states, NULL, NULL);
}

/* ratio (optional): omega_0 / gamma_0 per variable, 1 where the variable is linear;
 * betas (optional): the smoothness indicator of every stencil, betas[k * nst + q] */
static int cell_states_ex(const oracle_ctx *c, const double *U, long cell, double *states, float *ratio,
                          double *betas)
{
    int nv = c->nvar, n0 = c->n0, np = c->n_pts, nd = c->n_der;
    long N = ncells(c);
    double ref[MAXV], Phi[MAXV * MAXV], Phi_inv[MAXV * MAXV];
    load_cell(c, U, cell, ref);
    if (!admissible(c, ref)) return ERR_NONPHYSICAL;
    phi_matrices(c, ref, Phi, Phi_inv);

    /* W_h = Phi U_h over S0 (eq. consToRecVar) */
    double *W = (double *)malloc(sizeof(double) * n0 * nv);
    for (int h = 0; h < n0; ++h) {
        double uh[MAXV];
        neighbor_state(c, U, cell, c->s0 + h * c->dim, uh);
        matvec(nv, Phi, uh, W + h * nv);
    }

    double *wpt = (double *)malloc(sizeof(double) * np * nv);   /* w_s in W variables */
    double *vals = (double *)malloc(sizeof(double) * MAXST * np);
    for (int k = 0; k < nv; ++k) {
        double beta[MAXST], om[MAXST];
        for (int q = 0; q < c->nst; ++q) {
            int Nq = c->mem_ptr[q + 1] - c->mem_ptr[q];
            const int *mem = c->mem + c->mem_ptr[q];
            const double *tab = c->w + c->w_ptr[q];
            /* point values: one dot product per target (eq. reconVec) */
            for (int s = 0; s < np; ++s) {
                double acc = 0.0;
                for (int j = 0; j < Nq; ++j) acc += tab[s * Nq + j] * W[mem[j] * nv + k];
                vals[q * np + s] = acc;
            }
            /* smoothness indicator: sum of squared derivative values (eq. smoothIndic) */
            double b = 0.0;
            for (int a = 0; a < nd; ++a) {
                double acc = 0.0;
                for (int j = 0; j < Nq; ++j) acc += tab[(np + a) * Nq + j] * W[mem[j] * nv + k];
                b += acc * acc;
            }
            beta[q] = b;
            if (betas) betas[k * c->nst + q] = b;
        }
        int use_weno = c->weno;
        if (c->flags) use_weno = c->flags[(long)k * N + cell] != 0;
        if (!use_weno) {
            for (int s = 0; s < np; ++s) wpt[s * nv + k] = vals[0 * np + s];
            if (ratio) ratio[k] = 1.0f;
            continue;
        }
        /* nonlinear weights (eq. nlinWts) */
        double sum = 0.0;
        for (int q = 0; q < c->nst; ++q) {
            om[q] = c->lin_w[q] / (beta[q] * beta[q] + c->eps);
            sum += om[q];
        }
        for (int q = 0; q < c->nst; ++q) om[q] /= sum;
        if (ratio) ratio[k] = (float)(om[0] / c->lin_w[0]);
        /* WENO-AO blend (eq. wenoAOrec) */
        for (int s = 0; s < np; ++s) {
            double f = om[0] / c->lin_w[0] * vals[0 * np + s];
            for (int q = 1; q < c->nst; ++q)
                f += (om[q] - om[0] * c->lin_w[q] / c->lin_w[0]) * vals[q * np + s];
            wpt[s * nv + k] = f;
        }
    }
    /* back to conserved variables (eq. recVarToCons) */
    for (int s = 0; s < np; ++s) matvec(nv, Phi_inv, wpt + s * nv, states + s * nv);
    free(W);
    free(wpt);
    free(vals);

    if (!c->limiter) return OK;

    /* ------------------------------------ positivity limiter (section 4) --- */
    double rmax = -INFINITY, rmin = INFINITY, pmin = INFINITY;
    int lo[3] = {-1, -1, -1}, hi[3] = {1, 1, 1};
    if (c->dim < 3) lo[2] = hi[2] = 0;
    for (int dz = lo[2]; dz <= hi[2]; ++dz)
        for (int dy = lo[1]; dy <= hi[1]; ++dy)
            for (int dx = lo[0]; dx <= hi[0]; ++dx) {
                int off[3] = {dx, dy, dz};
                double un[MAXV];
                neighbor_state(c, U, cell, off, un);
                if (!admissible(c, un)) return ERR_NONPHYSICAL;
                double pn = pressure(c, un);
                if (un[0] > rmax) rmax = un[0];
                if (un[0] < rmin) rmin = un[0];
                if (pn < pmin) pmin = pn;
            }
    /* bounds widened by kappa (1 - eta): rho_max (1 + kappa - kappa eta),
     * rho_min (1 - kappa + kappa eta), p_min (1 - kappa + kappa eta) */
    double eta = flattener(c, U, cell);
    double f = c->kappa * (1.0 - eta);
    rmax *= 1.0 + f;
    rmin *= 1.0 - f;
    pmin *= 1.0 - f;

    /* density scaling (eq. ppThetaRho): only the violated side of each bound */
    double th = 1.0;
    for (int s = 0; s < np; ++s) {
        double rs = states[s * nv + 0];
        if (rs < rmin) {
            double t = (ref[0] - rmin) / (ref[0] - rs);
            if (t < th) th = t;
        } else if (rs > rmax) {
            double t = (rmax - ref[0]) / (rs - ref[0]);
            if (t < th) th = t;
        }
    }
    if (th < 1.0)
        for (int s = 0; s < np; ++s)
            for (int v = 0; v < nv; ++v)
                states[s * nv + v] = ref[v] + th * (states[s * nv + v] - ref[v]);   /* eq. ppCorrectDens */

    /* pressure scaling (eq. thetapRoot, eq. thetaP) by 60 bisection steps */
    double thp = 1.0;
    for (int s = 0; s < np; ++s) {
        if (pressure(c, states + s * nv) >= pmin) continue;
        double a = 0.0, b = 1.0;
        for (int it = 0; it < 60; ++it) {
            double m = 0.5 * (a + b), um[MAXV];
            for (int v = 0; v < nv; ++v) um[v] = ref[v] + m * (states[s * nv + v] - ref[v]);
            if (pressure(c, um) >= pmin) a = m; else b = m;
        }
        if (a < thp) thp = a;
    }
    if (thp < 1.0)
        for (int s = 0; s < np; ++s)
            for (int v = 0; v < nv; ++v)
                states[s * nv + v] = ref[v] + thp * (states[s * nv + v] - ref[v]);  /* eq. ppCorrectPres */
    return OK;
}

/* ----------------------------------------------------- Riemann solvers --- */
static void phys_flux(const oracle_ctx *c, const double *u, int a, double p, double *F)
{
    int d = c->dim, e = d + 1;
    double un = u[1 + a] / u[0];
    F[0] = u[1 + a];
    for (int b = 0; b < d; ++b) F[1 + b] = u[1 + b] * un + (b == a ? p : 0.0);
    F[e] = un * (u[e] + p);
}

/* Numerical flux across a face with normal axis a; uL on the lower side. */
static void riemann(const oracle_ctx *c, const double *uL, const double *uR, int a, double *F)
{
    int d = c->dim, nv = c->nvar, e = d + 1;
    double g = c->gamma;
    double pL = pressure(c, uL), pR = pressure(c, uR);
    double rL = uL[0], rR = uR[0];
    double vL[MAXD], vR[MAXD], qL = 0.0, qR = 0.0;
    for (int b = 0; b < d; ++b) {
        vL[b] = uL[1 + b] / rL; vR[b] = uR[1 + b] / rR;
        qL += vL[b] * vL[b]; qR += vR[b] * vR[b];
    }
    double cL = sqrt(g * pL / rL), cR = sqrt(g * pR / rR);
    double HL = (uL[e] + pL) / rL, HR = (uR[e] + pR) / rR;
    /* Roe averages for the Batten et al. wavespeeds */
    double sL = sqrt(rL), sR = sqrt(rR), vt[MAXD], qt = 0.0;
    for (int b = 0; b < d; ++b) { vt[b] = (sL * vL[b] + sR * vR[b]) / (sL + sR); qt += vt[b] * vt[b]; }
    double Ht = (sL * HL + sR * HR) / (sL + sR);
    double ct = sqrt((g - 1.0) * (Ht - 0.5 * qt));
    double SL = fmin(vL[a] - cL, vt[a] - ct);
    double SR = fmax(vR[a] + cR, vt[a] + ct);
    double FL[MAXV], FR[MAXV];
    phys_flux(c, uL, a, pL, FL);
    phys_flux(c, uR, a, pR, FR);

    if (c->riemann == 1) {   /* HLL */
        if (SL >= 0.0) { memcpy(F, FL, sizeof(double) * nv); return; }
        if (SR <= 0.0) { memcpy(F, FR, sizeof(double) * nv); return; }
        for (int v = 0; v < nv; ++v)
            F[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (uR[v] - uL[v])) / (SR - SL);
        return;
    }
    /* HLLC */
    if (SL >= 0.0) { memcpy(F, FL, sizeof(double) * nv); return; }
    if (SR <= 0.0) { memcpy(F, FR, sizeof(double) * nv); return; }
    double Ss = (pR - pL + rL * vL[a] * (SL - vL[a]) - rR * vR[a] * (SR - vR[a]))
              / (rL * (SL - vL[a]) - rR * (SR - vR[a]));
    const double *uK = Ss >= 0.0 ? uL : uR;
    const double *FK = Ss >= 0.0 ? FL : FR;
    double SK = Ss >= 0.0 ? SL : SR, rK = Ss >= 0.0 ? rL : rR, pK = Ss >= 0.0 ? pL : pR;
    const double *vK = Ss >= 0.0 ? vL : vR;
    double fac = rK * (SK - vK[a]) / (SK - Ss), us[MAXV];
    us[0] = fac;
    for (int b = 0; b < d; ++b) us[1 + b] = fac * (b == a ? Ss : vK[b]);
    us[e] = fac * (uK[e] / rK + (Ss - vK[a]) * (Ss + pK / (rK * (SK - vK[a]))));
    for (int v = 0; v < nv; ++v) F[v] = FK[v] + SK * (us[v] - uK[v]);
}

/* Gauss-Legendre tensor weight of transverse index g on a face with normal a */
static double face_weight(const oracle_ctx *c, int g)
{
    double w = 1.0;
    for (int t = 0; t < c->dim - 1; ++t) {
        w *= c->gl_w[g % c->R];
        g /= c->R;
    }
    return w;
}

/* Face-averaged flux through the upper face (normal a) of `cell`, from the
 * Riemann states of the cell (upper side) and its upper neighbour (lower side). */
static void face_flux(const oracle_ctx *c, const double *st_lo, const double *st_hi, int a, double *Fbar)
{
    int nv = c->nvar, ng = c->n_pts / (2 * c->dim);
    for (int v = 0; v < nv; ++v) Fbar[v] = 0.0;
    for (int g = 0; g < ng; ++g) {
        const double *uL = st_lo + ((2 * a + 1) * ng + g) * nv;   /* upper face of the lower cell */
        const double *uR = st_hi + ((2 * a + 0) * ng + g) * nv;   /* lower face of the upper cell */
        double F[MAXV];
        riemann(c, uL, uR, a, F);
        double w = face_weight(c, g);
        for (int v = 0; v < nv; ++v) Fbar[v] += w * F[v];
    }
}

/* ------------------------------- KXRCF troubled-cell indicator (3.5) --- */
/* Unlimited Riemann states of one cell, the first pass of section 5.3: the S0
 * point rows of the table applied to the conserved averages.  (Reconstructing
 * W = Phi U and mapping back with Phi^-1 gives the same values: the linear
 * reconstruction commutes with the constant matrix Phi.)  states: [n_pts][nvar]. */
static void unlimited_states(const oracle_ctx *c, const double *U, long cell, double *states)
{
    int nv = c->nvar, np = c->n_pts, N0 = c->mem_ptr[1] - c->mem_ptr[0];
    const int *mem = c->mem + c->mem_ptr[0];
    const double *tab = c->w + c->w_ptr[0];
    for (int i = 0; i < np * nv; ++i) states[i] = 0.0;
    for (int j = 0; j < N0; ++j) {
        double u[MAXV];
        neighbor_state(c, U, cell, c->s0 + mem[j] * c->dim, u);
        for (int s = 0; s < np; ++s)
            for (int v = 0; v < nv; ++v) states[s * nv + v] += tab[s * N0 + j] * u[v];
    }
}

/* The indicator variable, the entropy q = p / rho^gamma; 0 when u is not admissible. */
static int entropy(const oracle_ctx *c, const double *u, double *q)
{
    if (!admissible(c, u)) return 0;
    *q = pressure(c, u) / pow(u[0], c->gamma);
    return 1;
}

/* Largest |q+ - q-| over the Gauss points of the face with normal a between a
 * lower cell (states st_lo, its upper face) and its upper neighbour (st_hi, its
 * lower face); INFINITY when a state is not admissible. */
static double face_jump(const oracle_ctx *c, const double *st_lo, const double *st_hi, int a)
{
    int nv = c->nvar, ng = c->n_pts / (2 * c->dim);
    double J = 0.0;
    for (int g = 0; g < ng; ++g) {
        double qm, qp;
        if (!entropy(c, st_lo + ((2 * a + 1) * ng + g) * nv, &qm) ||
            !entropy(c, st_hi + ((2 * a + 0) * ng + g) * nv, &qp))
            return INFINITY;
        double j = fabs(qp - qm);
        if (j > J) J = j;
    }
    return J;
}

/* Left side of eq. kxrcf for one cell: the largest jump over the Gauss points of
 * all its faces divided by <Q> = p / rho^gamma of its average (INFINITY when a
 * state involved is not admissible).  jumps (optional): [2 dim] per-face maxima,
 * the lower face of axis a at 2a, the upper one at 2a + 1. */
static double kxrcf_measure(const oracle_ctx *c, const double *U, long cell, double *jumps)
{
    int nv = c->nvar, np = c->n_pts;
    double *own = (double *)malloc(sizeof(double) * np * nv * 2), *nb = own + np * nv;
    double u[MAXV], Q = 0.0, J = 0.0;
    load_cell(c, U, cell, u);
    int okQ = entropy(c, u, &Q);
    unlimited_states(c, U, cell, own);
    for (int a = 0; a < c->dim; ++a)
        for (int side = 0; side < 2; ++side) {
            int off[3] = {0, 0, 0};
            off[a] = side ? 1 : -1;
            if (on_boundary(c, cell, a, side))
                ghost_face_states(c, a, side, own, nb);
            else
                unlimited_states(c, U, wrap_index(c, cell, off), nb);
            double j = side ? face_jump(c, own, nb, a) : face_jump(c, nb, own, a);
            if (jumps) jumps[2 * a + side] = j;
            if (!(j <= J)) J = j;
        }
    free(own);
    return okQ ? J / Q : INFINITY;
}

/* Delta^m with Delta the cell width (the largest spacing when they differ) */
static double kxrcf_threshold(const oracle_ctx *c, double m)
{
    double delta = c->dx[0];
    for (int a = 1; a < c->dim; ++a)
        if (c->dx[a] > delta) delta = c->dx[a];
    return pow(delta, m);
}

/* The cell needs WENO unless eq. kxrcf holds (measure < Delta^m) */
static uint8_t kxrcf_flag(double measure, double thr) { return !(measure < thr); }

/* KXRCF decisions on the whole grid: flags[nvar][cells] (every variable of a
 * flagged cell takes WENO-AO); measure (optional) [cells]; jumps (optional)
 * [cells][2 dim]. */
int oracle_kxrcf(const oracle_ctx *c, const double *U, double m, uint8_t *flags, double *measure, double *jumps)
{
    long N = ncells(c);
    double thr = kxrcf_threshold(c, m);
#pragma omp parallel for schedule(dynamic, 64)
    for (long cell = 0; cell < N; ++cell) {
        double r = kxrcf_measure(c, U, cell, jumps ? jumps + cell * 2 * c->dim : NULL);
        if (measure) measure[cell] = r;
        uint8_t f = kxrcf_flag(r, thr);
        for (int v = 0; v < c->nvar; ++v) flags[v * N + cell] = f;
    }
    return OK;
}

/* KXRCF measure (left side of eq. kxrcf) at a list of cells only, for spot
 * checks on grids too large for the whole-grid routine.  measure: [count]. */
int oracle_kxrcf_cells(const oracle_ctx *c, const double *U, long count, const long *cells, double *measure)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < count; ++i) measure[i] = kxrcf_measure(c, U, cells[i], NULL);
    return OK;
}

/* The flattener eta of every cell (0 where the limiter's neighbourhood holds a
 * state that is not admissible).  eta: [cells]. */
int oracle_flattener(const oracle_ctx *c, const double *U, double *eta)
{
    long N = ncells(c);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long cell = 0; cell < N; ++cell) {
        int ok = 1;
        int lo[3] = {-1, -1, -1}, hi[3] = {1, 1, 1};
        if (c->dim < 3) lo[2] = hi[2] = 0;
        for (int dz = lo[2]; dz <= hi[2]; ++dz)
            for (int dy = lo[1]; dy <= hi[1]; ++dy)
                for (int dx = lo[0]; dx <= hi[0]; ++dx) {
                    int off[3] = {dx, dy, dz};
                    double un[MAXV];
                    neighbor_state(c, U, cell, off, un);
                    ok = ok && admissible(c, un);
                }
        eta[cell] = ok ? flattener(c, U, cell) : 0.0;
        bad |= !ok;
    }
    return bad ? ERR_NONPHYSICAL : OK;
}

/* ----------------------------------------------------------- exported --- */
/* All Riemann states: states[cell][n_pts][nvar]. */
int oracle_states(const oracle_ctx *c, const double *U, double *states)
{
    long N = ncells(c);
    int err = OK;
    /* two-pass procedure (section 5.3): the indicator's flags select WENO-AO */
    oracle_ctx cc = *c;
    uint8_t *fl = NULL;
    if (c->kxrcf_m > 0.0) {
        fl = (uint8_t *)malloc((size_t)N * c->nvar);
        if (!fl) return ERR_ARG;
        oracle_kxrcf(c, U, c->kxrcf_m, fl, NULL, NULL);
        cc.flags = fl;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (long cell = 0; cell < N; ++cell) {
        int e = cell_states(&cc, U, cell, states + cell * c->n_pts * c->nvar);
        if (e != OK) {
#pragma omp atomic write
            err = e;
        }
    }
    free(fl);
    return err;
}

/* dU/dt on the whole grid (section 5.3, steps 1-6). */
int oracle_rhs(const oracle_ctx *c, const double *U, double *dUdt)
{
    long N = ncells(c);
    int nv = c->nvar, np = c->n_pts;
    double *st = (double *)malloc(sizeof(double) * N * np * nv);
    if (!st) return ERR_ARG;
    int err = oracle_states(c, U, st);
    if (err != OK) { free(st); return err; }
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < N; ++cell) {
        double acc[MAXV] = {0};
        double *gh = (double *)malloc(sizeof(double) * np * nv);
        const double *own = st + cell * np * nv;
        for (int a = 0; a < c->dim; ++a) {
            int up[3] = {0, 0, 0}, dn[3] = {0, 0, 0};
            up[a] = 1; dn[a] = -1;
            double Fp[MAXV], Fm[MAXV];
            if (on_boundary(c, cell, a, 1)) {
                ghost_face_states(c, a, 1, own, gh);
                face_flux(c, own, gh, a, Fp);
            } else {
                face_flux(c, own, st + wrap_index(c, cell, up) * np * nv, a, Fp);
            }
            if (on_boundary(c, cell, a, 0)) {
                ghost_face_states(c, a, 0, own, gh);
                face_flux(c, gh, own, a, Fm);
            } else {
                face_flux(c, st + wrap_index(c, cell, dn) * np * nv, own, a, Fm);
            }
            for (int v = 0; v < nv; ++v) acc[v] -= (Fp[v] - Fm[v]) / c->dx[a];
        }
        for (int v = 0; v < nv; ++v) dUdt[v * N + cell] = acc[v];
        free(gh);
    }
    free(st);
    return OK;
}

/* dU/dt at a list of cells only, for spot checks on grids too large for the
 * whole-grid routine.  out: [count][nvar]. */
int oracle_rhs_cells(const oracle_ctx *c, const double *U, long count, const long *cells, double *out)
{
    int nv = c->nvar, np = c->n_pts, err = OK;
    long N = ncells(c);
    /* with the indicator on, the flags of every cell whose states enter (each
     * sampled cell and its face neighbours) */
    oracle_ctx cc = *c;
    uint8_t *fl = NULL;
    if (c->kxrcf_m > 0.0) {
        fl = (uint8_t *)calloc((size_t)N * nv, 1);
        if (!fl) return ERR_ARG;
        double thr = kxrcf_threshold(c, c->kxrcf_m);
        long nneed = count * (2 * c->dim + 1);
        long *target = (long *)malloc(sizeof(long) * nneed);
        uint8_t *f = (uint8_t *)malloc(nneed);
#pragma omp parallel for schedule(dynamic, 1)
        for (long k = 0; k < nneed; ++k) {
            long cell = cells[k / (2 * c->dim + 1)];
            int r = (int)(k % (2 * c->dim + 1)), off[3] = {0, 0, 0};
            if (r > 0) off[(r - 1) / 2] = (r - 1) % 2 ? 1 : -1;
            /* a neighbour past a non-periodic boundary is no cell: the sampled one stands in */
            target[k] = r > 0 && on_boundary(c, cell, (r - 1) / 2, (r - 1) % 2) ? cell : wrap_index(c, cell, off);
            f[k] = kxrcf_flag(kxrcf_measure(c, U, target[k], NULL), thr);
        }
        for (long k = 0; k < nneed; ++k)
            for (int v = 0; v < nv; ++v) fl[v * N + target[k]] = f[k];
        free(target);
        free(f);
        cc.flags = fl;
    }
    c = &cc;
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < count; ++i) {
        long cell = cells[i];
        double *st = (double *)malloc(sizeof(double) * np * nv * 3);
        double acc[MAXV] = {0};
        int e = cell_states(c, U, cell, st);
        for (int a = 0; a < c->dim && e == OK; ++a) {
            int up[3] = {0, 0, 0}, dn[3] = {0, 0, 0};
            up[a] = 1; dn[a] = -1;
            if (on_boundary(c, cell, a, 1))
                ghost_face_states(c, a, 1, st, st + np * nv);
            else
                e = cell_states(c, U, wrap_index(c, cell, up), st + np * nv);
            if (e == OK && on_boundary(c, cell, a, 0))
                ghost_face_states(c, a, 0, st, st + 2 * np * nv);
            else if (e == OK)
                e = cell_states(c, U, wrap_index(c, cell, dn), st + 2 * np * nv);
            if (e != OK) break;
            double Fp[MAXV], Fm[MAXV];
            face_flux(c, st, st + np * nv, a, Fp);
            face_flux(c, st + 2 * np * nv, st, a, Fm);
            for (int v = 0; v < nv; ++v) acc[v] -= (Fp[v] - Fm[v]) / c->dx[a];
        }
        if (e != OK) {
#pragma omp atomic write
            err = e;
        }
        for (int v = 0; v < nv; ++v) out[i * nv + v] = acc[v];
        free(st);
    }
    free(fl);
    return err;
}

/* One SSP-RK3 step (Shu-Osher form), U updated in place. */
int oracle_step(const oracle_ctx *c, double *U, double dt)
{
    long M = ncells(c) * c->nvar;
    double *L = (double *)malloc(sizeof(double) * M);
    double *U1 = (double *)malloc(sizeof(double) * M);
    double *U2 = (double *)malloc(sizeof(double) * M);
    int err = oracle_rhs(c, U, L);
    if (err == OK) {
        for (long i = 0; i < M; ++i) U1[i] = U[i] + dt * L[i];
        err = oracle_rhs(c, U1, L);
    }
    if (err == OK) {
        for (long i = 0; i < M; ++i) U2[i] = 0.75 * U[i] + 0.25 * (U1[i] + dt * L[i]);
        err = oracle_rhs(c, U2, L);
    }
    if (err == OK)
        for (long i = 0; i < M; ++i) U[i] = U[i] / 3.0 + 2.0 / 3.0 * (U2[i] + dt * L[i]);
    free(L);
    free(U1);
    free(U2);
    return err;
}

/* One step of SSP(4,3,2): the four-stage third-order strong-stability-preserving
 * Runge-Kutta method of Kraaijevanger with the embedded three-stage second-order
 * SSP method (section 6).  In Shu-Osher form with h = dt / 2:
 *   U1 = U + h L(U),  U2 = U1 + h L(U1),  U3 = 2/3 U + 1/3 (U2 + h L(U2)),
 *   U+ = U3 + h L(U3).
 * The embedded method shares the first three stages: Uhat = 1/3 U + 2/3 (U2 +
 * h L(U2)) = 2 U3 - U.  err_norm is the root mean square over every (variable,
 * cell) of (U+ - Uhat) / (atol + rtol max(|U|, |U+|)).  U is kept; U_out
 * receives U+. */
int oracle_step_ssp432(const oracle_ctx *c, const double *U, double dt, double atol, double rtol, double *U_out,
                       double *err_norm)
{
    long M = ncells(c) * c->nvar;
    double h = 0.5 * dt;
    double *L = (double *)malloc(sizeof(double) * M);
    double *U1 = (double *)malloc(sizeof(double) * M);
    double *U2 = (double *)malloc(sizeof(double) * M);
    double *U3 = (double *)malloc(sizeof(double) * M);
    int err = oracle_rhs(c, U, L);
    if (err == OK) {
        for (long i = 0; i < M; ++i) U1[i] = U[i] + h * L[i];
        err = oracle_rhs(c, U1, L);
    }
    if (err == OK) {
        for (long i = 0; i < M; ++i) U2[i] = U1[i] + h * L[i];
        err = oracle_rhs(c, U2, L);
    }
    if (err == OK) {
        for (long i = 0; i < M; ++i) U3[i] = 2.0 / 3.0 * U[i] + 1.0 / 3.0 * (U2[i] + h * L[i]);
        err = oracle_rhs(c, U3, L);
    }
    if (err == OK) {
        double acc = 0.0;
        for (long i = 0; i < M; ++i) {
            U_out[i] = U3[i] + h * L[i];
            double uhat = 2.0 * U3[i] - U[i];
            double sc = atol + rtol * fmax(fabs(U[i]), fabs(U_out[i]));
            double e = (U_out[i] - uhat) / sc;
            acc += e * e;
        }
        *err_norm = sqrt(acc / (double)M);
    }
    free(L);
    free(U1);
    free(U2);
    free(U3);
    return err;
}

/* dt = cfl / max_cell sum_a (|u_a| + c_s) / dx_a */
int oracle_cfl_dt(const oracle_ctx *c, const double *U, double cfl, double *dt)
{
    long N = ncells(c);
    double m = 0.0;
    int err = OK;
    for (long cell = 0; cell < N; ++cell) {
        double u[MAXV];
        load_cell(c, U, cell, u);
        if (!admissible(c, u)) { err = ERR_NONPHYSICAL; continue; }
        double cs = sqrt(c->gamma * pressure(c, u) / u[0]), s = 0.0;
        for (int a = 0; a < c->dim; ++a) {
            double r = (fabs(u[1 + a] / u[0]) + cs) / c->dx[a];
            if (c->cfl_max_axis) s = r > s ? r : s;
            else s += r;
        }
        if (s > m) m = s;
    }
    *dt = cfl / m;
    return err;
}

/* Riemann solver on single state pairs, for unit tests: uL, uR, F are [count][nvar]. */
void oracle_riemann(const oracle_ctx *c, long count, const double *uL, const double *uR, int axis, double *F)
{
    for (long i = 0; i < count; ++i)
        riemann(c, uL + i * c->nvar, uR + i * c->nvar, axis, F + i * c->nvar);
}

/* omega_0 / gamma_0 of every (variable, cell): out[nvar][cells] (the gate's label source). */
int oracle_omega_ratio(const oracle_ctx *c, const double *U, float *out)
{
    long N = ncells(c);
    int nv = c->nvar, err = OK;
#pragma omp parallel for schedule(dynamic, 64)
    for (long cell = 0; cell < N; ++cell) {
        double *st = (double *)malloc(sizeof(double) * c->n_pts * nv);
        float r[MAXV];
        int e = cell_states_ex(c, U, cell, st, r, NULL);
        if (e != OK) {
#pragma omp atomic write
            err = e;
        }
        for (int k = 0; k < nv; ++k) out[k * N + cell] = r[k];
        free(st);
    }
    return err;
}

/* Smoothness indicators beta[k][q] (eq. smoothIndic) of one cell, for unit tests. */
int oracle_smoothness(const oracle_ctx *c, const double *U, long cell, double *beta)
{
    double *st = (double *)malloc(sizeof(double) * c->n_pts * c->nvar);
    int e = cell_states_ex(c, U, cell, st, NULL, beta);
    free(st);
    return e;
}

/* Phi and Phi^-1 at a reference state, for unit tests. */
void oracle_phi(const oracle_ctx *c, const double *ref, double *Phi, double *Phi_inv)
{
    phi_matrices(c, ref, Phi, Phi_inv);
}
