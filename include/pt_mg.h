/*
 * pt_mg.h -- C ABI of libptmg, a multigrid solver for the implicit, two-way
 * coupled pressure-temperature system of an all-Mach VoF time step
 * (Saade, Lohse & Fuster, "A multigrid solver for the coupled
 * pressure-temperature equations in an all-Mach solver with VoF").
 *
 * The problem (Sec. 3, Eqs. 27-34).  On a uniform 2-D or 3-D grid of
 * cubic cells of size h, each cell carries the pressure p and temperature T
 * at the end of the step.  In the paper's form
 *     div(k grad T) + l1 T + l2 p                   = lT      (Eq. 27)
 *     div(grad p / rho) + l3 p + l4 div(k grad T)   = lp      (Eq. 28)
 * with l1 = -rho c_p/dt, l2 = beta T_adv/dt,
 * l3 = -(gamma/(rho c^2) - beta^2 T_adv/(rho c_p))/dt^2 (Eqs. 29-31),
 * l4 = beta/(rho c_p dt) (Eq. 32 read as the form that makes Eq. 28 equal
 * to Eq. 19 divided by dt), lT = l1 T_adv + l2 p_adv and
 * lp = l3 p_adv + div(u*)/dt (Eqs. 33-34).  The library solves the
 * equivalent canonical form, obtained by the exact row operations
 * T-row := -(Eq. 27), p-row := -(Eq. 28 - l4 * Eq. 27):
 *     -div(a_p grad p) + Bpp p + BpT T = f_p        a_p = 1/rho
 *     -div(a_T grad T) + BTp p + BTT T = f_T        a_T = k
 * with Bpp = -l3 + l4 l2, BpT = l4 l1, BTp = -l2, BTT = -l1,
 * f_T = -lT, f_p = -lp + l4 lT.
 *
 * Discretisation: cell-centred finite volumes, zero flux through every
 * boundary face, face coefficient = harmonic mean of the two cell values
 * (a face is closed when both are zero).  Mixed cells use the averaging
 * rule of Sec. 3 with the liquid (reference-phase) volume fraction C:
 * rho and k are averaged, and so is each phase's canonical block; the
 * cell's l1..l4 are the ones that reproduce the averaged block.
 *
 * Solve (Sec. 3, defect correction): repeat { residual in FP64; stop when
 * max over components of ||res||_2/||b||_2 <= rtol (paper row form);
 * one multigrid V-cycle on the correction; add it }.  The V-cycle runs in
 * FP64 (PT_PREC_FP64) or FP32 (PT_PREC_MIXED: FP32 smoother, restriction
 * and prolongation under FP64 iterative refinement; the coarsest grid is
 * always solved in FP64).
 *
 * Conventions for every function below.
 *  - Field pointers are HIP device pointers to contiguous float64 arrays of
 *    the grid's N = n[0]*n[1]*n[2] cells, cell (i,j,k) at i + n[0]*(j +
 *    n[1]*k) (x fastest).  p and T are separate arrays.
 *  - Work is ordered on the stream given to pt_mg_setup (NULL = the null
 *    stream).  Calls return when their results are in the caller's arrays
 *    unless stated otherwise.
 *  - The caller owns every array it passes; the library never keeps a
 *    caller pointer past the call.  The handle owns its device memory
 *    until pt_mg_destroy.
 *  - Functions return a pt_status; nothing is thrown across the ABI.  After
 *    an error the handle stays valid; pt_mg_last_error gives a message.
 *  - A handle must not be used by two host threads at once.
 */
#ifndef PT_MG_H
#define PT_MG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pt_mg_s *pt_mg_t;

typedef enum {
    PT_OK = 0,
    PT_ERR_ARG = 1,       /* invalid argument (dims, h, dt, C outside [0,1], non-finite input, ...) */
    PT_ERR_OOM = 2,       /* device allocation failed */
    PT_ERR_SINGULAR = 3,  /* a cell block has det <= 0 or a non-positive diagonal */
    PT_ERR_NOCONV = 4,    /* max_cycles reached, or a residual norm was not finite */
    PT_ERR_HIP = 5,       /* HIP runtime error */
    PT_ERR_STATE = 6      /* call not valid for this handle (wrong mode, level, ...) */
} pt_status;

typedef enum { PT_COEF_EXPLICIT = 0, PT_COEF_PHASES = 1, PT_COEF_STATE = 2 } pt_coef_mode;
typedef enum { PT_PREC_FP64 = 0, PT_PREC_MIXED = 1 } pt_precision;

/* Per-phase properties (SI).  beta <= 0: thermal dilation from Eq. (10),
 * beta = (Gamma-1) c_v / ((Gamma-1) c_v T + b (p + Pi)), evaluated at the
 * cell's (p_adv, T_adv); an ideal gas has Gamma = gamma, Pi = b = 0, which
 * gives 1/T.  gamma = c_p/c_v and the sound speed c enter l3 (Eq. 31).
 * q is the energy offset of the NASG EoS (Eq. 9), used by pt_state_eval.
 * mu is the dynamic viscosity (Pa s) of the viscous work in the phase
 * energies of Eq. (39) (pt_mg_downstream); 0 for an inviscid phase.
 * In PT_COEF_STATE mode rho and c are not used: each cell's phase density
 * comes from its conserved variables and the sound speed from Eq. (11). */
typedef struct {
    double rho, k, cp, cv, c, gamma, Gamma, Pi, b, beta, q, mu;
} pt_phase;

/* Problem description.  Unused fields are ignored; arrays are device
 * pointers and are read during pt_mg_setup / pt_mg_update only. */
typedef struct {
    int dim;                 /* 2 or 3 */
    int n[3];                /* cells per axis (>= 2 on active axes); n[2] = 1 in 2-D */
    double h;                /* cell size, > 0 */
    int mode;                /* pt_coef_mode */
    /* PT_COEF_EXPLICIT: canonical form given directly. */
    const double *alpha_p;   /* cell a_p [N] or NULL -> alpha_p_const */
    const double *alpha_T;   /* cell a_T [N] or NULL -> alpha_T_const */
    double alpha_p_const, alpha_T_const;
    const double *B;         /* [4][N] component-major (pp, pT, Tp, TT) or NULL -> B_const */
    double B_const[4];
    /* PT_COEF_PHASES: paper form (Eqs. 27-34). */
    const double *C;         /* liquid volume fraction [N], in [0, 1] */
    pt_phase liquid, gas;    /* phase 1 = liquid (reference phase), phase 2 = gas */
    double dt;               /* time step, > 0 */
    const double *p_adv;     /* provisional pressure [N] or NULL -> p_adv_const */
    const double *T_adv;     /* provisional temperature [N] or NULL -> T_adv_const */
    double p_adv_const, T_adv_const;
    /* Pure-Neumann Poisson limit only (every B entry zero): fix the free
     * constant of each component by a zero mean (the right-hand side is
     * projected to zero mean).  PT_ERR_ARG if set while B is not zero. */
    int mean_constraint;
    /* PT_COEF_STATE: the paper form with the cell state of Sec. 3.  Uses C,
     * liquid, gas, dt as PT_COEF_PHASES, the arrays p_adv and T_adv (both
     * required, e.g. from pt_state_eval), and the phase masses per volume
     * m1 = C rho_1, m2 = (1 - C) rho_2 [N]: each phase present in a cell
     * (fraction > 0, mass > 0) has density m_i / C_i, the sound speed of
     * Eq. (11) at that density and p_adv, and beta of Eq. (10); its block
     * is weighted by its fraction as in PT_COEF_PHASES, a_p = 1/(m1 + m2),
     * a_T = C k_1 + (1 - C) k_2. */
    const double *m1, *m2;
    /* 1: axisymmetric r-z grid (2-D only, else PT_ERR_ARG), the geometry of
     * the paper's bubble computations (Sec. 4): x is the axial and y the
     * radial coordinate, the axis is the lower y boundary, and cell row j
     * lies between the radii j h and (j + 1) h.  Every equation is per unit
     * volume with the cylindrical divergence: a radial face between rows
     * j - 1 and j counts, in the row-i equation, its coefficient times
     * r_face / r_i (areas proportional to the radius, volumes to the
     * centre radius), so no flux crosses the axis; axial faces are
     * unchanged.  The same metric applies in pt_mg_divergence and
     * pt_mg_downstream.  0: Cartesian. */
    int axisymmetric;
} pt_problem;

typedef struct {
    double rtol;             /* stop when max_c ||res_c||/||b_c|| <= rtol (paper row form) */
    int max_cycles;          /* V-cycles at most (<= PT_MAX_HIST - 1 recorded) */
    int nu1, nu2;            /* pre/post red-black smoothing sweeps (0..8) */
    int zero_guess;          /* 1: start from zero, ignoring the contents of p, T */
    /* PT_SOLVE_DEFECT (0): the defect-correction loop of Sec. 3 (residual,
     * test, V-cycle on the correction, update).  PT_SOLVE_BICGSTAB (1):
     * BiCGStab on the canonical system with the V-cycle as right
     * preconditioner, for time steps far above the acoustic one where the
     * plain loop contracts slowly; same stop test (paper row form, true
     * FP64 residual every iteration), max_cycles counts V-cycles (two per
     * iteration).  BiCGStab is synchronous (pt_mg_solve only), does not take
     * the mean constraint, and its first use on a handle allocates 8 FP64
     * work vectors of 2N doubles, kept until pt_mg_destroy. */
    int method;
    /* 1: stream-ordered (pt_mg_solve, defect-correction loop only).  The
     * call enqueues every outer iteration up to max_cycles (<= PT_MAX_HIST
     * - 1) on the handle's stream and returns PT_OK at once; nothing waits
     * on the host.  After each residual a one-thread kernel takes the stop
     * test of Sec. 3 on the device, and once it is met every later launch
     * of the solve returns at entry.  p, T and *info are valid once the
     * stream has passed the solve (a stream or device synchronisation):
     * the stream writes *info through a host function, so `info` must stay
     * valid until then; info->status carries the outcome (PT_OK or
     * PT_ERR_NOCONV).  Results are those of the blocking solve, bit for
     * bit.  Costs: the launches after the stop still run as no-ops (a few
     * microseconds each), so max_cycles should not be far above the cycles
     * needed; the first use allocates a small pinned record (kept until
     * pt_mg_destroy), so pt_mg_solve_noalloc refuses it; pt_mg_step and
     * BiCGStab refuse it too; pt_mg_last_cell_updates reads 0 after it. */
    int async;
} pt_solve_opts;

#define PT_SOLVE_DEFECT 0
#define PT_SOLVE_BICGSTAB 1

#define PT_MAX_HIST 64

typedef struct {
    int cycles;                        /* V-cycles performed */
    double relres[2];                  /* final (p, T) relative residual, paper row form */
    double relres_hist[2 * PT_MAX_HIST]; /* (p, T) after 0, 1, ... cycles */
    int hist_len;                      /* number of recorded pairs */
    double t_solve_s;                  /* wall time of the call */
    int status;                        /* same as the return value */
} pt_solve_info;

/* Advected conserved variables of one grid (Sec. 3), for pt_state_eval.
 * Device float64 arrays [n]. */
typedef struct {
    int dim;                 /* 2 or 3: momentum components read */
    long long n;             /* cells, >= 1 */
    const double *C;         /* liquid volume fraction C_1 */
    const double *m1, *m2;   /* phase masses per volume C_1 rho_1, C_2 rho_2 */
    const double *E;         /* total energy per volume of the cell (both phases) */
    const double *mom[3];    /* averaged momentum per axis, or all NULL (at rest) */
    pt_phase liquid, gas;    /* NASG records (Gamma, Pi, b, q, cp, cv); ideal gas:
                              * Gamma = gamma, Pi = b = q = 0 */
    double *p_adv, *T_adv;   /* outputs */
} pt_state;

/* Provisional pressure and temperature from the advected conserved
 * variables through the EoS (Sec. 3): Eq. (20),
 *   p = (E - 1/2 rho |u|^2 - bar(Gamma Pi (1 - rho b)/(Gamma - 1) + rho q))
 *       / bar((1 - rho b)/(Gamma - 1)),
 * with rho = m1 + m2, u = mom / rho, and Eq. (23),
 *   T = (bar(1 - rho b) p + bar(Pi (1 - rho b))) / bar(rho (c_p - c_v)),
 * where bar(phi) = C_1 phi(rho_1) + C_2 phi(rho_2), rho_i = m_i / C_i (the
 * bars are formed as sums of C_i- and m_i-weighted terms, so a phase
 * absent from a cell adds nothing and nothing is divided by C_i).
 * Asynchronous on hip_stream (hipStream_t or NULL); no host
 * synchronisation and no allocation.  Cells are not validated here
 * (pt_mg_setup / pt_mg_update reject non-physical states).  PT_ERR_ARG
 * for a NULL field, dim or n out of range, or Gamma <= 1. */
int pt_state_eval(const pt_state *s, void *hip_stream);

/* Device bytes that pt_mg_setup will allocate for this problem and
 * precision (the handle's hierarchy, coarse inverse and work buffers).
 * 0 if the problem is invalid.  For admission control. */
size_t pt_mg_footprint_bytes(const pt_problem *prob, int precision);

/* Assemble the operator (Sec. 3: averaging rule; Eqs. 27-32 via the
 * canonical form above) and build the multigrid hierarchy for the given
 * V-cycle precision (pt_precision): coarse coefficients, and the inverse
 * of the coarsest-grid matrix in FP64.  hip_stream is a hipStream_t or
 * NULL.  On success *out owns all device memory; on failure *out = NULL.
 * Errors: PT_ERR_ARG, PT_ERR_OOM, PT_ERR_SINGULAR, PT_ERR_HIP. */
int pt_mg_setup(const pt_problem *prob, int precision, void *hip_stream, pt_mg_t *out);

/* Re-assemble with new coefficient fields (same dim, n, mode) into the
 * existing handle, without allocating (one call per time step).  Errors as
 * pt_mg_setup; on error the handle must be updated again before a solve. */
int pt_mg_update(pt_mg_t h, const pt_problem *prob);

/* Right-hand side of the paper form, Eqs. (33)-(34):
 * b_T = l1 T_adv + l2 p_adv, b_p = l3 p_adv + div_ustar / dt, with the
 * cell coefficients of the handle (PT_COEF_PHASES or PT_COEF_STATE, else
 * PT_ERR_STATE).  p_adv / T_adv NULL -> the constants given at setup;
 * div_ustar NULL -> zero.  Outputs b_p, b_T [N]. */
int pt_mg_paper_rhs(pt_mg_t h, const double *p_adv, const double *T_adv,
                    const double *div_ustar, double *b_p, double *b_T);

/* Solve L(a) = b (Sec. 3, defect correction).  b is mode-native: the
 * paper's (lp, lT) in PT_COEF_PHASES, the canonical (f_p, f_T) in
 * PT_COEF_EXPLICIT.  p, T [N] are the initial guess on entry (unless
 * opts->zero_guess) and the solution on return.  opts NULL -> rtol 1e-9,
 * 50 cycles, V(2,2), zero guess.  info may be NULL.  Returns PT_OK, or
 * PT_ERR_NOCONV with the last iterate in p, T and info filled. */
int pt_mg_solve(pt_mg_t h, const double *b_p, const double *b_T, double *p, double *T,
                const pt_solve_opts *opts, pt_solve_info *info);

/* For callers that cannot allocate device memory: code that runs between
 * HIP graph captures, serving loops and harnesses that forbid hipMalloc.
 * pt_mg_solve with the same arguments, results, errors and info, except
 * that no call allocates device or host memory: with opts->method =
 * PT_SOLVE_BICGSTAB the eight FP64 work vectors (128 bytes per cell, which
 * pt_mg_solve allocates on its first BiCGStab call on a handle) live in the
 * library's static device scratch of PT_SCRATCH_BYTES (128 MiB, held on
 * each GPU the library runs on until the process ends), so grids of at
 * most PT_SCRATCH_MAX_CELLS = 2^20 cells; a larger grid fails with
 * PT_ERR_ARG before anything is enqueued.  The defect method needs no work
 * memory beyond the handle's and runs exactly as pt_mg_solve.  The scratch
 * is shared by every call on one GPU and keeps the last call's contents
 * (the vectors that must start at zero are cleared by each call): calls
 * that overlap on one GPU (from two host threads, or on two handles whose
 * streams run concurrently) race.  Timing (pt_mg_set_timing) creates its
 * HIP events on first use; leave it off where nothing may be created. */
#define PT_SCRATCH_MAX_CELLS (1ll << 20)
#define PT_SCRATCH_BYTES (16ll * 8 * PT_SCRATCH_MAX_CELLS)
int pt_mg_solve_noalloc(pt_mg_t h, const double *b_p, const double *b_T, double *p, double *T,
                        const pt_solve_opts *opts, pt_solve_info *info);

/* One implicit step in one call: pt_mg_update(prob), the paper right-hand
 * side of Eqs. (33)-(34) from prob->p_adv, prob->T_adv and div_ustar into
 * b_p, b_T (as pt_mg_paper_rhs), and pt_mg_solve(b, p, T, opts, info), the
 * work of Algorithm 1's implicit p-T solve.  Everything is enqueued on the
 * handle's stream with the host waiting only where the solve reads its
 * norms; the assembly checks of pt_mg_update are read with the first
 * norms.  Results, outputs and errors are those of the three calls in
 * sequence (an assembly error leaves the handle not ready and b, p, T
 * unspecified).  PT_COEF_PHASES or PT_COEF_STATE only (PT_ERR_STATE
 * otherwise); b_p, b_T, p, T [N] are caller-owned device arrays. */
int pt_mg_step(pt_mg_t h, const pt_problem *prob, const double *div_ustar, double *b_p,
               double *b_T, double *p, double *T, const pt_solve_opts *opts,
               pt_solve_info *info);

/* Residual in FP64, mode-native form: res = b - L(a) of Eqs. (27)-(28)
 * (PT_COEF_PHASES) or f - A u (PT_COEF_EXPLICIT).  p, T [N] are the
 * iterate, or both NULL for a zero iterate (res = b, the first residual
 * of a solve from a zero guess; the same values and norms as with zero
 * arrays).  r_p, r_T [N] may be NULL.  relres (may be NULL) receives
 * ||res_c||_2 / ||b_c||_2 for c = p, T, reduced in a fixed order (bitwise
 * reproducible). */
int pt_mg_residual(pt_mg_t h, const double *b_p, const double *b_T, const double *p,
                   const double *T, double *r_p, double *r_T, double relres[2]);

/* ---------------------------------------------------------------------
 * The end of the step, after the solve (Sec. 3).
 *
 * Face velocities: U[a] (a < dim) holds the velocity component normal to
 * the faces across axis a: n[a] + 1 faces along a (both walls included)
 * and n[b] along every other axis b.  The face at (i,j,k) is the lower
 * face of cell (i,j,k); its index is i + m0*(j + m1*k) with
 * m_b = n[b] + (b == a).  Device float64 arrays, caller-owned.
 * --------------------------------------------------------------------- */

/* Divergence of face velocities per cell, the sum over axes of
 * (U_a on the upper face - U_a on the lower face) / h: the div u* that
 * Eq. (17) and lambda_p of Eq. (34) use (pass it to pt_mg_paper_rhs).
 * U[0 .. dim-1] as above (U[dim..2] ignored), div [N] output.  Any mode.
 * PT_ERR_ARG for a NULL array. */
int pt_mg_divergence(pt_mg_t h, const double *const U[3], double *div);

/* Fields of pt_mg_downstream.  Cell arrays [N]; U arrays as above. */
typedef struct {
    const double *p, *T;         /* the solution of pt_mg_solve */
    const double *C;             /* liquid volume fraction C_1 (the assembly's) */
    const double *kappa;         /* interface curvature, or NULL: no surface tension */
    double sigma;                /* surface tension coefficient */
    const double *U_star[3];     /* provisional face velocities u* (Eq. provel) */
    double *U[3];                /* out: face velocities at the end of the step;
                                  * must not overlap U_star */
    const double *u_star[3];     /* provisional cell velocities, or all NULL */
    double *u[3];                /* out: cell velocities (may be u_star), or all NULL */
    const double *E1_adv, *E2_adv; /* phase total energies per volume after
                                  * advection, C_i rho_i e_T,i; both NULL: no
                                  * energy update */
    double *E1, *E2;             /* out (may be E1_adv, E2_adv) */
} pt_downstream;

/* The step's end in one pass over the grid: the velocity correction of
 * Eq. (unp1) and the phase energies of Eq. (39) with the phase pressures
 * of Eqs. (37)-(38).
 *  - Faces: U = U* - dt a_f (p_R - p_L)/h on interior faces, a_f the p
 *    face coefficient of the assembly (harmonic mean of 1/rho), so that
 *    div U is the one of Eq. (17) the solve used; wall faces keep U*.
 *  - Cells: u = u* - dt g, g along each axis the mean of a_f (p_R - p_L)/h
 *    on the cell's two faces across that axis (0 on a wall face).
 *  - p_1 = p + (1 - C) sigma kappa, p_2 = p - C sigma kappa.
 *  - E_i = E_i^adv + dt C_i [ -div(p_i U) + W + div(k grad T) ], C_1 = C,
 *    C_2 = 1 - C; the pressure-work flux on a face is the mean of the two
 *    cells' p_i times U (on a wall face the cell's own p_i); the heat flux
 *    is k_f (T_R - T_L)/h with the T face coefficient of the assembly, zero
 *    through the walls.
 *  - W = div(mu (grad u + grad u^T) . u), the viscous work of Eq. (39) for
 *    the corrected velocities, when a phase has mu > 0 (needs u_star and u):
 *    the flux through the face between cells L and R across axis a is
 *    sum_b tau_ab u_b with u_a the face velocity U and u_b (b != a) the mean
 *    of the two cells' u_b; tau_aa = 2 mu_f (u_a,R - u_a,L)/h and tau_ab =
 *    mu_f ((u_b,R - u_b,L)/h + the mean over L, R of the centred difference
 *    of u_a along b, mirrored at a wall); mu_f the mean of the two cells'
 *    C mu_1 + (1 - C) mu_2; no flux through the walls.  It runs as a
 *    second pass over the grid.
 * dt, h, 1/rho, k and the viscosities are those of the last pt_mg_setup /
 * pt_mg_update (PT_COEF_PHASES or PT_COEF_STATE; PT_ERR_STATE otherwise).
 * Returns when the outputs are written.  PT_ERR_ARG for a NULL p, T, C,
 * U_star[a] or U[a] (a < dim), U[a] == U_star[a], only one of u_star / u
 * given for an axis, exactly one of E1_adv, E2_adv, E1, E2 missing, or a
 * viscous phase without cell velocities. */
int pt_mg_downstream(pt_mg_t h, const pt_downstream *d);

void pt_mg_destroy(pt_mg_t h);

/* Last error message of the handle, or of the calling thread when h is
 * NULL (errors of pt_mg_setup).  Never NULL. */
const char *pt_mg_last_error(pt_mg_t h);

/* ---------------------------------------------------------------------
 * Multigrid steps on one level, for step-by-step comparison and
 * measurement.  The paper cites its multigrid without details (Sec. 3);
 * the steps are this library's: red-black 2x2-block Gauss-Seidel,
 * residual with averaging restriction to the 2^dim children's parent,
 * cell-centred linear prolongation, coarse coefficients by averaging the
 * fine faces that make up a coarse face and the 2^dim children's blocks,
 * and an exact FP64 solve on the coarsest grid.  All arrays are FP64
 * device arrays of the level's cell count, canonical form; they are
 * converted to and from the handle's V-cycle precision.
 * --------------------------------------------------------------------- */

/* Number of levels (finest = 0) and the grid of one level. */
int pt_mg_num_levels(pt_mg_t h);
int pt_mg_level_dims(pt_mg_t h, int level, int n[3], double *hl);

/* The level's operator as the V-cycle uses it: faces [6][N_l] with
 * index (component*3 + axis)*N_l + cell = coefficient of the face between
 * the cell and its lower neighbour along the axis (0 on the boundary;
 * axis 2 unused in 2-D), and the block [4][N_l] (pp, pT, Tp, TT). */
int pt_mg_get_operator(pt_mg_t h, int level, double *faces, double *B);

/* `sweeps` red-black sweeps in place on (u_p, u_T): cells with i+j+k even
 * first, then odd, each solving its 2x2 block with the latest neighbours. */
int pt_mg_smooth(pt_mg_t h, int level, const double *f_p, const double *f_T,
                 double *u_p, double *u_T, int sweeps);

/* Coarse right-hand side fc = mean over the 2^dim children of f - A u on
 * `level`; fc has the cell count of level+1. */
int pt_mg_restrict_residual(pt_mg_t h, int level, const double *f_p, const double *f_T,
                            const double *u_p, const double *u_T, double *fc_p,
                            double *fc_T);

/* u += P e on `level` from e on level+1 (linear interpolation: along each
 * axis 3/4 of the parent and 1/4 of the parent's neighbour on the fine
 * cell's side, the parent itself at a boundary). */
int pt_mg_prolong_add(pt_mg_t h, int level, const double *ec_p, const double *ec_T,
                      double *u_p, double *u_T);

/* Exact FP64 solve on the coarsest level: u = A^-1 f. */
int pt_mg_coarse_solve(pt_mg_t h, const double *f_p, const double *f_T, double *u_p,
                       double *u_T);

/* One V(nu1, nu2) cycle on level 0 for A e = f from a zero guess. */
int pt_mg_vcycle(pt_mg_t h, const double *f_p, const double *f_T, double *e_p,
                 double *e_T, int nu1, int nu2);

/* ---------------------------------------------------------------------
 * Measurement.
 * --------------------------------------------------------------------- */

/* Kernel classes timed with HIP events when timing is on. */
typedef enum {
    PT_K_OUTER_RESIDUAL = 0,  /* FP64 residual (+ update) + norm partial sums, finest grid */
    PT_K_SMOOTH_FINE = 1,     /* red-black smoother, finest grid (one launch = one sweep) */
    PT_K_SMOOTH_COARSE = 2,   /* smoother, coarser grids */
    PT_K_RESTRICT = 3,        /* residual + restriction, all levels */
    PT_K_PROLONG = 4,         /* prolongation + correction, all levels */
    PT_K_COARSE_SOLVE = 5,    /* coarsest-grid solve */
    PT_K_OTHER = 6,           /* norm reduction, conversions, copies */
    PT_K_DOWNSTREAM = 7,      /* pt_mg_downstream (velocity correction + phase energies) */
    PT_K_SMOOTH_FINE_T = 8,   /* finest-grid sweep with a transfer inside: the restriction
                                 of its residual, or the prolonged correction added */
    PT_K_COUNT = 9
} pt_kernel_class;

/* HIP-event timing (off by default): on = 0 off, 1 every kernel class,
 * otherwise 1 + 2 * (bit mask of pt_kernel_class values) times only those
 * classes.  A run of back-to-back launches of one class (the nu sweeps of
 * one smoothing step on one level, or a single launch) is bracketed by one
 * event pair on the handle's stream; option PT_OPT_TIMING_EVERY = n times
 * only every n-th run of each class (the events themselves cost a few
 * microseconds of stream time). */
int pt_mg_set_timing(pt_mg_t h, int on);

/* All launches of one class since the last reset and their algorithmic
 * bytes (the model of each kernel: every array it must read or write
 * once, halos excluded), plus the summed milliseconds of its timed runs. */
int pt_mg_kernel_stats(pt_mg_t h, int kernel_class, long *launches, double *ms,
                       double *bytes);
/* The timed runs of one class alone: their launches, summed milliseconds
 * and algorithmic bytes (bytes / ms is the class's achieved bandwidth).
 * Call after the stream has been synchronised; pairs still in flight are
 * counted once they complete. */
int pt_mg_timed_stats(pt_mg_t h, int kernel_class, long *launches, double *ms, double *bytes);
int pt_mg_reset_stats(pt_mg_t h);

/* Cell-updates performed by the last pt_mg_solve: smoother cell updates
 * on every level plus residual evaluations (the finest-grid FP64 one and
 * the one inside each restriction). */
long long pt_mg_last_cell_updates(pt_mg_t h);

/* Execution options of a handle (results are the same either way):
 *  PT_OPT_GRAPHS: replay the coarse-level part of each V-cycle from a HIP
 *    graph captured on first use, and the hierarchy build after each
 *    assembly from another (needs a non-null stream); default 0: direct
 *    launches measured 2-5 % faster per 2-D step and no slower in 3-D.
 *  PT_OPT_TAIL: run the coarsest levels that fit in one block's LDS as a
 *    single-block kernel; default 1.  pt_mg_get_option returns, for
 *    PT_OPT_TAIL, the number of levels the tail covers (0 if none).
 *  PT_OPT_FUSED: each red-black sweep as one fused pass over memory, the
 *    finest level's transfers inside its sweeps, and (from the next
 *    pt_mg_update) the levels of at most 1024 cells and the coarsest
 *    inverse built by one single-block kernel; 0: two colour passes and
 *    separate kernels (the reference path, equal bit for bit); default 1.
 *  PT_OPT_TIMING_EVERY: with timing on, time one run in every n of each
 *    class (n >= 1, default 1; PT_ERR_ARG otherwise).
 *  PT_OPT_SPECULATE: enqueue the next outer iteration (V-cycle, FP64
 *    update, residual and norms) before the host has read the current
 *    norms, whenever the contraction seen so far predicts that the
 *    current iterate misses the tolerance by a factor of 3 or more (and,
 *    from a zero guess, the first cycle at once; the contraction of that
 *    first cycle is taken no smaller than the last one of the handle's
 *    previous solve).  The solution, cycles
 *    and history are those of the step-by-step loop; a wrong guess costs
 *    one V-cycle of device time.  Default 1.
 *  PT_OPT_TAIL_CELLS: the largest level (in cells) the single-block tail
 *    may hold; 0 (default): as many coarse levels as fit its LDS.  The
 *    levels above it run as grid kernels with the same arithmetic.
 *  PT_OPT_COARSE_SWEEPS: 16 nu1 + nu2, the pre- and post-sweeps on the
 *    levels below the finest (each 0..8, not both 0); 0: the solve's own
 *    nu1, nu2 on every level (the default).  Steps whose coarse
 *    levels are dominated by the acoustic block term converge as fast with
 *    17 (one sweep each way) for less time; diffusion-dominated steps need
 *    the full counts there.  Unlike the options
 *    above this changes the V-cycle, and so the iterates and cycle
 *    counts; the converged solution is the one the tolerance admits
 *    either way.
 *  PT_OPT_W_LEVELS: w >= 0; each visit of levels 1 .. w (those above the
 *    single-block tail) corrects twice on its coarse level (a second pass
 *    of sweeps, residual, coarse cycle, prolongation and sweeps from the
 *    iterate the first left), a W-cycle there; the finest level and the
 *    tail stay V.  0 (default): the V-cycle.  On time steps far above the
 *    acoustic one (diffusion-dominated, with the 1000:1 density jump)
 *    the V-cycle's coarse levels lose accuracy level by level and the
 *    cycle contracts ever more slowly as the grid grows; the W-cycle's
 *    contraction stays near the two-grid one, for more coarse-level work
 *    per cycle.  Like PT_OPT_COARSE_SWEEPS this changes the iterates and
 *    cycle counts, not the converged solution.
 *  PT_OPT_OMEGA: 1000 omega, 1..1999; the finest level's red-black block
 *    Gauss-Seidel updates become u + omega (u_GS - u) (over-relaxation;
 *    coarser levels keep omega = 1).  1000 (default): the plain update.
 *    With 1100 the 512^3 collapse step of the mixed-precision solve
 *    reaches 1e-12 in two cycles of V(4,4) instead of three of V(4,3).
 *    Changes the iterates and cycle counts, not the converged solution. */
typedef enum {
    PT_OPT_GRAPHS = 1,
    PT_OPT_TAIL = 2,
    PT_OPT_FUSED = 3,
    PT_OPT_TIMING_EVERY = 4,
    PT_OPT_SPECULATE = 5,
    PT_OPT_TAIL_CELLS = 6,
    PT_OPT_COARSE_SWEEPS = 7,
    PT_OPT_W_LEVELS = 8,
    PT_OPT_OMEGA = 9
} pt_option;
int pt_mg_set_option(pt_mg_t h, int option, int value);
int pt_mg_get_option(pt_mg_t h, int option);

/* A plain device copy of `bytes` bytes on the stream (hipStream_t or
 * NULL), for calibrating bandwidth counters.  Asynchronous. */
int pt_copy_kernel(void *dst, const void *src, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PT_MG_H */
