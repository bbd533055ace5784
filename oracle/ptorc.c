/*
 * ptorc.c -- FP64 CPU oracle for the coupled pressure-temperature solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes (Saade, Lohse & Fuster, "A multigrid solver for the
 * coupled pressure-temperature equations in an all-Mach solver with VoF"):
 *
 *   paper form (Eqs. 27-28), a = [T p], per unit volume:
 *     div(k grad T) + l1 T + l2 p            = lT
 *     div(grad p / rho) + l3 p + l4 div(k grad T) = lp
 *   with l1..l4, lT, lp of Eqs. 29-34 (l4 read as beta/(rho c_p dt), the
 *   form that makes Eq. 28 equal to Eq. 19 divided by dt).
 *
 *   canonical form, obtained by the exact row operations
 *     T-row := -(paper T-row),  p-row := -(paper p-row - l4 * paper T-row):
 *     -div(a_p grad p) + Bpp p + BpT T = f_p,   a_p = 1/rho
 *     -div(a_T grad T) + BTp p + BTT T = f_T,   a_T = k
 *     Bpp = -l3 + l4 l2, BpT = l4 l1, BTp = -l2, BTT = -l1,
 *     f_T = -lT, f_p = -lp + l4 lT.
 *
 * Geometry: Cartesian 2-D / 3-D, or axisymmetric r-z (2-D, y the radius
 * from the axis on the lower y wall; every diffusion term and divergence
 * then carries the face-area / cell-volume metric of axi_face).
 *
 * Discretisation: cell-centred finite volumes on a uniform grid of spacing h
 * (second order, as the paper states in Sec. 4.1), homogeneous Neumann
 * (zero flux) on every boundary face, face coefficient = harmonic mean of
 * the two cell values.  Mixed cells (Sec. 3, averaging rule): the per-phase
 * canonical blocks are averaged with the liquid volume fraction C, and so
 * are rho and k.  Cell index = i + nx*(j + ny*k).
 *
 * Solver: the defect-correction loop of Sec. 3 (residual, stop test,
 * approximate solve of the correction, update) around a plain FP64 V(2,2)
 * multigrid cycle (lexicographic 2x2-block Gauss-Seidel, averaging
 * restriction, linear prolongation, face-averaged coarse coefficients,
 * dense LU with partial pivoting on the coarsest grid).  The paper only
 * cites its multigrid; these choices change the speed, not the converged
 * result.  The step functions (red-black sweep, restriction, prolongation,
 * coarse operator) are exported for step-by-step comparisons.
 *
 * Also here: the provisional state from the advected conserved variables
 * (Eqs. 20, 23) and the end of the step that consumes the solution: the
 * velocity correction (Eq. unp1) on faces and at cell centres, the phase
 * pressures (Eqs. 37-38) and the phase total energies (Eq. 39).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Planted mistakes, for the mutation checks of the pin tests only: the
 * tests compile a private copy of this file with ORC_PLANT = k and check
 * that the pins reject it.  Every other build uses 0 (no mistake).
 *   1: face coefficient = arithmetic instead of harmonic mean
 *   2: cell a_p = C/rho_l + (1-C)/rho_g instead of 1/(C rho_l + (1-C) rho_g)
 *   3: cell a_T = 1/(C/k_l + (1-C)/k_g) instead of C k_l + (1-C) k_g
 *   4: viscous stress mu grad u instead of mu (grad u + grad u^T)
 *   5: viscous stress without the tangential-gradient term (g_ba) */
#ifndef ORC_PLANT
#define ORC_PLANT 0
#endif

typedef struct {
    double rho, k, cp, cv, c, gamma, Gamma, Pi, b, beta, q;
} orc_phase;

/* ------------------------------------------------------------------ */
/* thermodynamics                                                      */
/* ------------------------------------------------------------------ */

/* Thermal dilation, Eq. (10) (NASG); with Pi = b = 0 it is 1/T. */
double orc_beta(const orc_phase *ph, double p, double T)
{
    if (ph->beta > 0.0) return ph->beta;
    double gcv = (ph->Gamma - 1.0) * ph->cv;
    return gcv / (gcv * T + ph->b * (p + ph->Pi));
}

/* Per-phase coefficients, Eqs. (29)-(32): lam = {l1, l2, l3, l4}. */
void orc_phase_lambdas(const orc_phase *ph, double p, double T, double dt,
                       double lam[4])
{
    double beta = orc_beta(ph, p, T);
    double rcp = ph->rho * ph->cp;
    lam[0] = -rcp / dt;
    lam[1] = beta * T / dt;
    lam[2] = -(ph->gamma / (ph->rho * ph->c * ph->c) - beta * beta * T / rcp) / (dt * dt);
    lam[3] = beta / (rcp * dt);
}

/* Canonical 2x2 block from paper coefficients; order (pp, pT, Tp, TT). */
void orc_block_from_lambdas(const double lam[4], double B[4])
{
    B[0] = -lam[2] + lam[3] * lam[1];
    B[1] = lam[3] * lam[0];
    B[2] = -lam[1];
    B[3] = -lam[0];
}

/* Cell coefficients of a (possibly mixed) cell: per-phase blocks averaged
 * with C; the cell's paper coefficients are the ones that reproduce that
 * averaged block (l1, l2 averaged; l4 = BpT / l1; l3 = -Bpp + l4 l2). */
void orc_cell_lambdas(double C, const orc_phase *liq, const orc_phase *gas,
                      double p, double T, double dt, double lam[4], double B[4])
{
    double l_liq[4], l_gas[4], B_liq[4], B_gas[4];
    orc_phase_lambdas(liq, p, T, dt, l_liq);
    orc_phase_lambdas(gas, p, T, dt, l_gas);
    orc_block_from_lambdas(l_liq, B_liq);
    orc_block_from_lambdas(l_gas, B_gas);
    for (int q = 0; q < 4; q++) B[q] = C * B_liq[q] + (1.0 - C) * B_gas[q];
    lam[0] = -B[3];
    lam[1] = -B[2];
    lam[3] = B[1] / lam[0];
    lam[2] = -B[0] + lam[3] * lam[1];
}

/* Assembly of a whole grid (phases mode).  Outputs cell a_p = 1/rho_bar,
 * a_T = k_bar, the cell paper coefficients lam[4n] (component-major) and
 * the canonical block B[4n] (component-major).  p_adv / T_adv may be NULL
 * (then the constants are used).  Returns the number of cells whose block
 * has a non-positive determinant or diagonal. */
long orc_assemble_phases(long n, const double *C, const orc_phase *liq,
                         const orc_phase *gas, double dt,
                         const double *p_adv, double p_const,
                         const double *T_adv, double T_const,
                         double *a_p, double *a_T, double *lam, double *B)
{
    long bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(static)
    for (long i = 0; i < n; i++) {
        double c = C[i];
        double p = p_adv ? p_adv[i] : p_const;
        double T = T_adv ? T_adv[i] : T_const;
        double l[4], b[4];
        orc_cell_lambdas(c, liq, gas, p, T, dt, l, b);
#if ORC_PLANT == 2
        a_p[i] = c / liq->rho + (1.0 - c) / gas->rho;
#else
        a_p[i] = 1.0 / (c * liq->rho + (1.0 - c) * gas->rho);
#endif
#if ORC_PLANT == 3
        a_T[i] = 1.0 / (c / liq->k + (1.0 - c) / gas->k);
#else
        a_T[i] = c * liq->k + (1.0 - c) * gas->k;
#endif
        for (int q = 0; q < 4; q++) {
            lam[q * n + i] = l[q];
            B[q * n + i] = b[q];
        }
        if (!(b[0] > 0.0 && b[3] > 0.0 && b[0] * b[3] - b[1] * b[2] > 0.0)) bad++;
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* provisional state from the advected conserved variables            */
/* ------------------------------------------------------------------ */

/* Provisional pressure, Eq. (20), and temperature, Eq. (23), of n cells
 * from the advected conserved variables of Sec. 3: C (liquid volume
 * fraction), m1 = C rho_1 and m2 = (1 - C) rho_2 (phase masses per
 * volume), E (the cell's total energy per volume, both phases) and the
 * averaged momentum mom[dim * n] (component-major; NULL: at rest).  The
 * bar average of a phase quantity phi(rho_i) is C phi(rho_1) +
 * (1 - C) phi(rho_2) with rho_i = m_i / C_i (a phase absent from the cell
 * adds nothing); the kinetic energy is 1/2 rho_bar |u_bar|^2 with
 * rho_bar = m1 + m2 and u_bar = mom / rho_bar. */
void orc_state(long n, int dim, const double *C, const double *m1, const double *m2,
               const double *E, const double *mom, const orc_phase *liq,
               const orc_phase *gas, double *p, double *T)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) {
        const double frac[2] = {C[i], 1.0 - C[i]};
        const double mass[2] = {m1[i], m2[i]};
        const orc_phase *ph[2] = {liq, gas};
        double e_static = 0.0, inv_gm1 = 0.0;          /* the two bars of Eq. (20) */
        double vol = 0.0, vol_pi = 0.0, heat = 0.0;    /* the three bars of Eq. (23) */
        for (int q = 0; q < 2; q++) {
            if (frac[q] <= 0.0) continue;
            const double rho = mass[q] / frac[q];
            const double G = ph[q]->Gamma, Pi = ph[q]->Pi, b = ph[q]->b;
            const double free_vol = 1.0 - rho * b;
            e_static += frac[q] * (G * Pi / (G - 1.0) * free_vol + rho * ph[q]->q);
            inv_gm1 += frac[q] * (free_vol / (G - 1.0));
            vol += frac[q] * free_vol;
            vol_pi += frac[q] * (Pi * free_vol);
            heat += frac[q] * (rho * (ph[q]->cp - ph[q]->cv));
        }
        const double rho_bar = m1[i] + m2[i];
        double u2 = 0.0;
        if (mom)
            for (int a = 0; a < dim; a++) {
                const double u = mom[(long)a * n + i] / rho_bar;
                u2 += u * u;
            }
        const double pc = (E[i] - 0.5 * rho_bar * u2 - e_static) / inv_gm1;
        p[i] = pc;
        T[i] = (vol * pc + vol_pi) / heat;
    }
}

/* Sound speed squared of a phase, Eq. (11). */
double orc_sound2(const orc_phase *ph, double rho, double p)
{
    return ph->Gamma * (p + ph->Pi) / (rho * (1.0 - rho * ph->b));
}

/* Assembly from the cell state (state mode): in each cell every phase
 * present has the density rho_i = m_i / C_i, the sound speed of Eq. (11)
 * at (rho_i, p_adv), the thermal dilation of Eq. (10) at (p_adv, T_adv)
 * and the gamma of its record; its coefficients (Eqs. 29-32) and canonical
 * block follow as in the phases mode; the blocks and k are averaged with
 * the phase fractions, and a_p = 1 / (m1 + m2).  Outputs as
 * orc_assemble_phases; returns the number of non-positive blocks. */
long orc_assemble_state(long n, const double *C, const double *m1, const double *m2,
                        const orc_phase *liq, const orc_phase *gas, double dt,
                        const double *p_adv, const double *T_adv, double *a_p, double *a_T,
                        double *lam, double *B)
{
    long bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(static)
    for (long i = 0; i < n; i++) {
        const double frac[2] = {C[i], 1.0 - C[i]};
        const double mass[2] = {m1[i], m2[i]};
        const orc_phase *src[2] = {liq, gas};
        const double p = p_adv[i], T = T_adv[i];
        double b[4] = {0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < 2; q++) {
            if (frac[q] <= 0.0) continue;
            orc_phase ph = *src[q];
            ph.rho = mass[q] / frac[q];
            ph.c = sqrt(orc_sound2(&ph, ph.rho, p));
            double l[4], bq[4];
            orc_phase_lambdas(&ph, p, T, dt, l);
            orc_block_from_lambdas(l, bq);
            for (int k = 0; k < 4; k++) b[k] += frac[q] * bq[k];
        }
        a_p[i] = 1.0 / (m1[i] + m2[i]);
        a_T[i] = C[i] * liq->k + (1.0 - C[i]) * gas->k;
        double l[4];
        l[0] = -b[3];
        l[1] = -b[2];
        l[3] = b[1] / l[0];
        l[2] = -b[0] + l[3] * l[1];
        for (int q = 0; q < 4; q++) {
            lam[q * n + i] = l[q];
            B[q * n + i] = b[q];
        }
        if (!(b[0] > 0.0 && b[3] > 0.0 && b[0] * b[3] - b[1] * b[2] > 0.0)) bad++;
    }
    return bad;
}

/* Paper right-hand side, Eqs. (33)-(34): bT = l1 T_adv + l2 p_adv,
 * bp = l3 p_adv + div(u*)/dt.  div may be NULL (zero). */
void orc_paper_rhs(long n, const double *lam, const double *p_adv, double p_const,
                   const double *T_adv, double T_const, const double *div,
                   double dt, double *b_p, double *b_T)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) {
        double p = p_adv ? p_adv[i] : p_const;
        double T = T_adv ? T_adv[i] : T_const;
        double d = div ? div[i] : 0.0;
        b_T[i] = lam[0 * n + i] * T + lam[1 * n + i] * p;
        b_p[i] = lam[2 * n + i] * p + d / dt;
    }
}

/* Canonical right-hand side from the paper one (same row operations). */
void orc_canonical_rhs(long n, const double *lam, const double *b_p,
                       const double *b_T, double *f_p, double *f_T)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) {
        f_T[i] = -b_T[i];
        f_p[i] = -b_p[i] + lam[3 * n + i] * b_T[i];
    }
}

/* ------------------------------------------------------------------ */
/* grids, faces and the operator                                       */
/* ------------------------------------------------------------------ */

/* Face arrays: F[(c*3 + a)*n + cell] is the coefficient on the face between
 * `cell` and its lower neighbour along axis a (0 on the lower boundary),
 * c = 0 for p, 1 for T.  Axes a >= dim are unused and zero. */

static long idx3(const int *n, long i, long j, long k)
{
    return i + (long)n[0] * (j + (long)n[1] * k);
}

/* Level-0 faces: harmonic mean of the two cell values (0 when both are 0). */
void orc_faces_from_cells(int dim, const int *n, const double *a_p,
                          const double *a_T, double *F)
{
    long N = (long)n[0] * n[1] * n[2];
    memset(F, 0, sizeof(double) * 6 * N);
    const double *cell[2] = {a_p, a_T};
    for (int c = 0; c < 2; c++)
        for (int a = 0; a < dim; a++) {
            double *Fa = F + (long)(c * 3 + a) * N;
#pragma omp parallel for schedule(static)
            for (long k = 0; k < n[2]; k++)
                for (long j = 0; j < n[1]; j++)
                    for (long i = 0; i < n[0]; i++) {
                        long ii[3] = {i, j, k};
                        if (ii[a] == 0) continue;
                        ii[a] -= 1;
                        long me = idx3(n, i, j, k);
                        long lo = idx3(n, ii[0], ii[1], ii[2]);
                        double L = cell[c][lo], R = cell[c][me];
                        /* a zero coefficient on either side closes the face */
#if ORC_PLANT == 1
                        Fa[me] = 0.5 * (L + R);
#else
                        Fa[me] = (L + R > 0.0) ? 2.0 * L * R / (L + R) : 0.0;
#endif
                    }
        }
}

/* Axisymmetric (r-z) metric: y is the radius, measured from the axis on
 * the lower y wall.  In units of the grid spacing the lower face of row j
 * is at r = j and the cell centre at r = j + 1/2.  A finite volume's
 * radial faces have areas proportional to their radius and its axial faces
 * and volume to the centre radius, so per unit volume a radial face counts
 * r_face / r_centre and an axial face 1 (the cylindrical divergence
 * (1/r) d/dr (r a du/dr) + d/dz (a du/dz)). */
static double axi_face(long j_face, long j_cell)
{
    return (double)j_face / ((double)j_cell + 0.5);
}

/* Diffusion part of the canonical operator at one cell, component c:
 * sum over faces of m_f a_f (u_i - u_nbr) / h^2 (zero flux through the
 * boundary), m_f = 1, or the r-z metric of axi_face on radial faces when
 * axi.  Also returns the sum of the face weights. */
static double diffusion_at(int dim, const int *n, double h, const double *F, int axi,
                           int c, const double *u, long i, long j, long k,
                           double *diag)
{
    long N = (long)n[0] * n[1] * n[2];
    long me = idx3(n, i, j, k);
    long ii[3] = {i, j, k};
    double acc = 0.0, dsum = 0.0;
    double inv_h2 = 1.0 / (h * h);
    for (int a = 0; a < dim; a++) {
        const double *Fa = F + (long)(c * 3 + a) * N;
        if (ii[a] > 0) {
            long t[3] = {i, j, k};
            t[a] -= 1;
            long lo = idx3(n, t[0], t[1], t[2]);
            double w = Fa[me] * inv_h2;
            if (axi && a == 1) w *= axi_face(j, j);
            acc += w * (u[me] - u[lo]);
            dsum += w;
        }
        if (ii[a] < n[a] - 1) {
            long t[3] = {i, j, k};
            t[a] += 1;
            long hi = idx3(n, t[0], t[1], t[2]);
            double w = Fa[hi] * inv_h2;
            if (axi && a == 1) w *= axi_face(j + 1, j);
            acc += w * (u[me] - u[hi]);
            dsum += w;
        }
    }
    if (diag) *diag = dsum;
    return acc;
}

/* A u in canonical form.  B is component-major [4n]. */
void orc_apply(int dim, const int *n, double h, const double *F, int axi, const double *B,
               const double *p, const double *T, double *Ap, double *AT)
{
    long N = (long)n[0] * n[1] * n[2];
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n[2]; k++)
        for (long j = 0; j < n[1]; j++)
            for (long i = 0; i < n[0]; i++) {
                long me = idx3(n, i, j, k);
                double dp = diffusion_at(dim, n, h, F, axi, 0, p, i, j, k, NULL);
                double dT = diffusion_at(dim, n, h, F, axi, 1, T, i, j, k, NULL);
                Ap[me] = dp + B[0 * N + me] * p[me] + B[1 * N + me] * T[me];
                AT[me] = dT + B[2 * N + me] * p[me] + B[3 * N + me] * T[me];
            }
}

/* r = f - A u (canonical form). */
void orc_residual(int dim, const int *n, double h, const double *F, int axi, const double *B,
                  const double *f_p, const double *f_T, const double *p,
                  const double *T, double *r_p, double *r_T)
{
    long N = (long)n[0] * n[1] * n[2];
    orc_apply(dim, n, h, F, axi, B, p, T, r_p, r_T);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; i++) {
        r_p[i] = f_p[i] - r_p[i];
        r_T[i] = f_T[i] - r_T[i];
    }
}

/* Residual of the paper form directly from Eqs. (27)-(28):
 * res_T = bT - (div(k grad T) + l1 T + l2 p),
 * res_p = bp - (div(grad p/rho) + l3 p + l4 div(k grad T)).
 * Here div(a grad u) at a cell = -(diffusion_at). */
void orc_paper_residual(int dim, const int *n, double h, const double *F, int axi,
                        const double *lam, const double *b_p, const double *b_T,
                        const double *p, const double *T, double *res_p,
                        double *res_T)
{
    long N = (long)n[0] * n[1] * n[2];
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n[2]; k++)
        for (long j = 0; j < n[1]; j++)
            for (long i = 0; i < n[0]; i++) {
                long me = idx3(n, i, j, k);
                double divp = -diffusion_at(dim, n, h, F, axi, 0, p, i, j, k, NULL);
                double divT = -diffusion_at(dim, n, h, F, axi, 1, T, i, j, k, NULL);
                double l1 = lam[me], l2 = lam[N + me], l3 = lam[2 * N + me],
                       l4 = lam[3 * N + me];
                res_T[me] = b_T[me] - (divT + l1 * T[me] + l2 * p[me]);
                res_p[me] = b_p[me] - (divp + l3 * p[me] + l4 * divT);
            }
}

static double dot(long N, const double *x, const double *y)
{
    double s = 0.0;
    for (long i = 0; i < N; i++) s += x[i] * y[i];
    return s;
}

/* ------------------------------------------------------------------ */
/* multigrid steps                                                     */
/* ------------------------------------------------------------------ */

/* Solve the 2x2 block equations of one cell with its neighbours fixed. */
static void block_update(int dim, const int *n, double h, const double *F, int axi,
                         const double *B, const double *f_p, const double *f_T,
                         double *p, double *T, long i, long j, long k)
{
    long N = (long)n[0] * n[1] * n[2];
    long me = idx3(n, i, j, k);
    double sp, sT;
    /* diffusion_at(u) = S u_me - sum w u_nbr, so the neighbour sum is
     * S u_me - diffusion_at(u). */
    double dp = diffusion_at(dim, n, h, F, axi, 0, p, i, j, k, &sp);
    double dT = diffusion_at(dim, n, h, F, axi, 1, T, i, j, k, &sT);
    double gp = f_p[me] + (sp * p[me] - dp);
    double gT = f_T[me] + (sT * T[me] - dT);
    double a = B[0 * N + me] + sp, b = B[1 * N + me];
    double c = B[2 * N + me], d = B[3 * N + me] + sT;
    double det = a * d - b * c;
    p[me] = (d * gp - b * gT) / det;
    T[me] = (a * gT - c * gp) / det;
}

/* One lexicographic block Gauss-Seidel sweep (x fastest). */
void orc_lex_sweep(int dim, const int *n, double h, const double *F, int axi, const double *B,
                   const double *f_p, const double *f_T, double *p, double *T)
{
    for (long k = 0; k < n[2]; k++)
        for (long j = 0; j < n[1]; j++)
            for (long i = 0; i < n[0]; i++)
                block_update(dim, n, h, F, axi, B, f_p, f_T, p, T, i, j, k);
}

/* One red-black block Gauss-Seidel sweep: cells with (i+j+k) even first,
 * then the odd ones, each using the latest neighbour values. */
void orc_rb_sweep(int dim, const int *n, double h, const double *F, int axi, const double *B,
                  const double *f_p, const double *f_T, double *p, double *T)
{
    for (int colour = 0; colour < 2; colour++)
        for (long k = 0; k < n[2]; k++)
            for (long j = 0; j < n[1]; j++)
                for (long i = 0; i < n[0]; i++)
                    if (((i + j + k) & 1) == colour)
                        block_update(dim, n, h, F, axi, B, f_p, f_T, p, T, i, j, k);
}

/* Coarse grid of n: every axis < dim halved. */
static void coarse_dims(int dim, const int *n, int *nc)
{
    for (int a = 0; a < 3; a++) nc[a] = (a < dim) ? n[a] / 2 : 1;
}

/* Coarse operator: coarse face coefficient = mean of the 2^(dim-1) fine
 * faces that make it up; coarse block = mean of the 2^dim children. */
void orc_coarse_operator(int dim, const int *n, const double *F, const double *B,
                         double *Fc, double *Bc)
{
    int nc[3];
    coarse_dims(dim, n, nc);
    long N = (long)n[0] * n[1] * n[2];
    long Nc = (long)nc[0] * nc[1] * nc[2];
    int nchild = 1 << dim;
    memset(Fc, 0, sizeof(double) * 6 * Nc);
    for (long K = 0; K < nc[2]; K++)
        for (long J = 0; J < nc[1]; J++)
            for (long I = 0; I < nc[0]; I++) {
                long C = idx3(nc, I, J, K);
                long base[3] = {2 * I, dim > 1 ? 2 * J : J, dim > 2 ? 2 * K : K};
                for (int q = 0; q < 4; q++) {
                    double s = 0.0;
                    for (int m = 0; m < nchild; m++) {
                        long ch[3] = {base[0] + (m & 1), base[1] + ((m >> 1) & 1),
                                      base[2] + ((m >> 2) & 1)};
                        s += B[q * N + idx3(n, ch[0], ch[1], ch[2])];
                    }
                    Bc[q * Nc + C] = s / nchild;
                }
                long Cc[3] = {I, J, K};
                for (int c = 0; c < 2; c++)
                    for (int a = 0; a < dim; a++) {
                        if (Cc[a] == 0) continue;   /* boundary face */
                        double s = 0.0;
                        int cnt = 0;
                        for (int m = 0; m < nchild; m++) {
                            long ch[3] = {base[0] + (m & 1), base[1] + ((m >> 1) & 1),
                                          base[2] + ((m >> 2) & 1)};
                            if (ch[a] != base[a]) continue;  /* lower-face children */
                            s += F[(long)(c * 3 + a) * N + idx3(n, ch[0], ch[1], ch[2])];
                            cnt++;
                        }
                        Fc[(long)(c * 3 + a) * Nc + C] = s / cnt;
                    }
            }
}

/* Coarse right-hand side: mean of the 2^dim children of the fine residual. */
void orc_restrict(int dim, const int *n, const double *r_p, const double *r_T,
                  double *fc_p, double *fc_T)
{
    int nc[3];
    coarse_dims(dim, n, nc);
    int nchild = 1 << dim;
    for (long K = 0; K < nc[2]; K++)
        for (long J = 0; J < nc[1]; J++)
            for (long I = 0; I < nc[0]; I++) {
                long base[3] = {2 * I, dim > 1 ? 2 * J : J, dim > 2 ? 2 * K : K};
                double sp = 0.0, sT = 0.0;
                for (int m = 0; m < nchild; m++) {
                    long f = idx3(n, base[0] + (m & 1), base[1] + ((m >> 1) & 1),
                                  base[2] + ((m >> 2) & 1));
                    sp += r_p[f];
                    sT += r_T[f];
                }
                long C = idx3(nc, I, J, K);
                fc_p[C] = sp / nchild;
                fc_T[C] = sT / nchild;
            }
}

/* u += P e: cell-centred linear interpolation.  Along each axis a fine cell
 * lies a quarter coarse cell from its parent's centre: weight 3/4 on the
 * parent, 1/4 on the parent's neighbour on the fine cell's side (the parent
 * itself at a boundary, i.e. zero normal gradient). */
void orc_prolong_add(int dim, const int *n, const double *e_p, const double *e_T,
                     double *p, double *T)
{
    int nc[3];
    coarse_dims(dim, n, nc);
    for (long k = 0; k < n[2]; k++)
        for (long j = 0; j < n[1]; j++)
            for (long i = 0; i < n[0]; i++) {
                long fi[3] = {i, j, k};
                long par[3], nb[3];
                for (int a = 0; a < 3; a++) {
                    if (a >= dim) { par[a] = nb[a] = fi[a]; continue; }
                    par[a] = fi[a] / 2;
                    long s = (fi[a] % 2 == 0) ? -1 : 1;
                    nb[a] = par[a] + s;
                    if (nb[a] < 0 || nb[a] >= nc[a]) nb[a] = par[a];
                }
                double vp = 0.0, vT = 0.0;
                for (int m = 0; m < (1 << dim); m++) {
                    double w = 1.0;
                    long c[3] = {par[0], par[1], par[2]};
                    for (int a = 0; a < dim; a++) {
                        if ((m >> a) & 1) { c[a] = nb[a]; w *= 0.25; }
                        else w *= 0.75;
                    }
                    long C = idx3(nc, c[0], c[1], c[2]);
                    vp += w * e_p[C];
                    vT += w * e_T[C];
                }
                long me = idx3(n, i, j, k);
                p[me] += vp;
                T[me] += vT;
            }
}

/* ------------------------------------------------------------------ */
/* dense coarsest solve                                                */
/* ------------------------------------------------------------------ */

/* Dense matrix of the canonical operator, unknown ordering
 * [p_0 .. p_{N-1}, T_0 .. T_{N-1}].  M is (2N)x(2N), row-major.  With
 * `pin_mean`, the all-ones block (scaled by the mean diagonal) is added to
 * each component's diagonal block, which fixes the constant mode of a pure
 * Neumann Poisson problem to zero mean for a zero-mean right-hand side. */
void orc_dense_matrix(int dim, const int *n, double h, const double *F, int axi,
                      const double *B, int pin_mean, double *M)
{
    long N = (long)n[0] * n[1] * n[2];
    long M2 = 2 * N;
    memset(M, 0, sizeof(double) * M2 * M2);
    double *e = calloc(N, sizeof(double));
    double *z = calloc(N, sizeof(double));
    double *Ap = malloc(sizeof(double) * N), *AT = malloc(sizeof(double) * N);
    for (long col = 0; col < M2; col++) {
        memset(e, 0, sizeof(double) * N);
        e[col % N] = 1.0;
        if (col < N) orc_apply(dim, n, h, F, axi, B, e, z, Ap, AT);
        else orc_apply(dim, n, h, F, axi, B, z, e, Ap, AT);
        for (long r = 0; r < N; r++) {
            M[r * M2 + col] = Ap[r];
            M[(N + r) * M2 + col] = AT[r];
        }
    }
    if (pin_mean) {
        for (int c = 0; c < 2; c++) {
            double dsum = 0.0;
            for (long r = 0; r < N; r++) dsum += M[(c * N + r) * M2 + c * N + r];
            double s = dsum / ((double)N * N);
            for (long r = 0; r < N; r++)
                for (long q = 0; q < N; q++) M[(c * N + r) * M2 + c * N + q] += s;
        }
    }
    free(e); free(z); free(Ap); free(AT);
}

/* LU with partial pivoting, in place; returns 0 on success. */
int orc_lu(long m, double *A, long *piv)
{
    for (long k = 0; k < m; k++) {
        long pr = k;
        double best = fabs(A[k * m + k]);
        for (long r = k + 1; r < m; r++)
            if (fabs(A[r * m + k]) > best) { best = fabs(A[r * m + k]); pr = r; }
        piv[k] = pr;
        if (best == 0.0) return 1;
        if (pr != k)
            for (long q = 0; q < m; q++) {
                double t = A[k * m + q]; A[k * m + q] = A[pr * m + q]; A[pr * m + q] = t;
            }
        for (long r = k + 1; r < m; r++) {
            double l = A[r * m + k] / A[k * m + k];
            A[r * m + k] = l;
            for (long q = k + 1; q < m; q++) A[r * m + q] -= l * A[k * m + q];
        }
    }
    return 0;
}

void orc_lu_solve(long m, const double *LU, const long *piv, double *x)
{
    for (long k = 0; k < m; k++) {
        long pr = piv[k];
        if (pr != k) { double t = x[k]; x[k] = x[pr]; x[pr] = t; }
    }
    for (long r = 0; r < m; r++)
        for (long q = 0; q < r; q++) x[r] -= LU[r * m + q] * x[q];
    for (long r = m - 1; r >= 0; r--) {
        for (long q = r + 1; q < m; q++) x[r] -= LU[r * m + q] * x[q];
        x[r] /= LU[r * m + r];
    }
}

/* ------------------------------------------------------------------ */
/* the multigrid solver                                                */
/* ------------------------------------------------------------------ */

#define ORC_MAX_LEVELS 24

typedef struct {
    int n[3];
    long N;
    double h;
    double *F, *B;            /* faces [6N], block [4N] */
    double *f_p, *f_T, *u_p, *u_T, *r_p, *r_T;
} orc_level;

typedef struct {
    int dim, nlev, pin_mean, axi;
    orc_level L[ORC_MAX_LEVELS];
    double *LU;
    long *piv;
    long m;
} orc_mg;

static void level_alloc(orc_level *lv, const int *n, double h)
{
    for (int a = 0; a < 3; a++) lv->n[a] = n[a];
    lv->N = (long)n[0] * n[1] * n[2];
    lv->h = h;
    lv->F = calloc(6 * lv->N, sizeof(double));
    lv->B = calloc(4 * lv->N, sizeof(double));
    lv->f_p = calloc(lv->N, sizeof(double)); lv->f_T = calloc(lv->N, sizeof(double));
    lv->u_p = calloc(lv->N, sizeof(double)); lv->u_T = calloc(lv->N, sizeof(double));
    lv->r_p = calloc(lv->N, sizeof(double)); lv->r_T = calloc(lv->N, sizeof(double));
}

static void level_free(orc_level *lv)
{
    free(lv->F); free(lv->B); free(lv->f_p); free(lv->f_T);
    free(lv->u_p); free(lv->u_T); free(lv->r_p); free(lv->r_T);
}

/* Coarsen while every active axis is even and at least 4 long, and the
 * grid has more than 8 cells. */
static int can_coarsen(int dim, const int *n)
{
    long N = (long)n[0] * n[1] * n[2];
    if (N <= 8) return 0;
    for (int a = 0; a < dim; a++)
        if (n[a] % 2 != 0 || n[a] < 4) return 0;
    return 1;
}

static void mg_build(orc_mg *mg, int dim, const int *n, double h, const double *F0, int axi,
                     const double *B0, int pin_mean)
{
    memset(mg, 0, sizeof(*mg));
    mg->dim = dim;
    mg->axi = axi;
    mg->pin_mean = pin_mean;
    level_alloc(&mg->L[0], n, h);
    memcpy(mg->L[0].F, F0, sizeof(double) * 6 * mg->L[0].N);
    memcpy(mg->L[0].B, B0, sizeof(double) * 4 * mg->L[0].N);
    int l = 0;
    while (l + 1 < ORC_MAX_LEVELS && can_coarsen(dim, mg->L[l].n)) {
        int nc[3];
        coarse_dims(dim, mg->L[l].n, nc);
        level_alloc(&mg->L[l + 1], nc, 2.0 * mg->L[l].h);
        orc_coarse_operator(dim, mg->L[l].n, mg->L[l].F, mg->L[l].B,
                            mg->L[l + 1].F, mg->L[l + 1].B);
        l++;
    }
    mg->nlev = l + 1;
    orc_level *c = &mg->L[l];
    mg->m = 2 * c->N;
    mg->LU = malloc(sizeof(double) * mg->m * mg->m);
    mg->piv = malloc(sizeof(long) * mg->m);
    orc_dense_matrix(dim, c->n, c->h, c->F, axi, c->B, pin_mean, mg->LU);
    orc_lu(mg->m, mg->LU, mg->piv);
}

static void mg_free(orc_mg *mg)
{
    for (int l = 0; l < mg->nlev; l++) level_free(&mg->L[l]);
    free(mg->LU); free(mg->piv);
}

/* V(nu1, nu2) cycle on level l for A e = f (e starts at zero). */
static void vcycle(orc_mg *mg, int l, int nu1, int nu2)
{
    orc_level *lv = &mg->L[l];
    int dim = mg->dim;
    memset(lv->u_p, 0, sizeof(double) * lv->N);
    memset(lv->u_T, 0, sizeof(double) * lv->N);
    if (l == mg->nlev - 1) {
        double *x = malloc(sizeof(double) * mg->m);
        memcpy(x, lv->f_p, sizeof(double) * lv->N);
        memcpy(x + lv->N, lv->f_T, sizeof(double) * lv->N);
        if (mg->pin_mean) {
            double mp = 0, mT = 0;
            for (long i = 0; i < lv->N; i++) { mp += x[i]; mT += x[lv->N + i]; }
            mp /= lv->N; mT /= lv->N;
            for (long i = 0; i < lv->N; i++) { x[i] -= mp; x[lv->N + i] -= mT; }
        }
        orc_lu_solve(mg->m, mg->LU, mg->piv, x);
        memcpy(lv->u_p, x, sizeof(double) * lv->N);
        memcpy(lv->u_T, x + lv->N, sizeof(double) * lv->N);
        free(x);
        return;
    }
    for (int s = 0; s < nu1; s++)
        orc_lex_sweep(dim, lv->n, lv->h, lv->F, mg->axi, lv->B, lv->f_p, lv->f_T, lv->u_p,
                      lv->u_T);
    orc_residual(dim, lv->n, lv->h, lv->F, mg->axi, lv->B, lv->f_p, lv->f_T, lv->u_p, lv->u_T,
                 lv->r_p, lv->r_T);
    orc_level *cv = &mg->L[l + 1];
    orc_restrict(dim, lv->n, lv->r_p, lv->r_T, cv->f_p, cv->f_T);
    vcycle(mg, l + 1, nu1, nu2);
    orc_prolong_add(dim, lv->n, cv->u_p, cv->u_T, lv->u_p, lv->u_T);
    for (int s = 0; s < nu2; s++)
        orc_lex_sweep(dim, lv->n, lv->h, lv->F, mg->axi, lv->B, lv->f_p, lv->f_T, lv->u_p,
                      lv->u_T);
}

/*
 * Defect-correction solve (Sec. 3): starting from the guess in (p, T),
 * repeat { residual; stop when small; one V-cycle on the correction; add }.
 *
 * Inputs are the level-0 faces F [6N], block B [4N] and canonical RHS.
 * When lam != NULL (phases mode) the stop test uses the paper-form
 * residual of Eqs. (27)-(28) against the paper right-hand side (b_p, b_T);
 * otherwise the canonical residual against (f_p, f_T).  The test is
 * max over components of ||res_c||_2 / ||b_c||_2 <= rtol.
 * hist (may be NULL) receives 2 numbers per residual evaluation.
 * Returns the number of V-cycles performed, or -1 if max_cycles was hit.
 */
int orc_mg_solve(int dim, const int *n, double h, const double *F, int axi, const double *B,
                 const double *lam, const double *b_p, const double *b_T,
                 const double *f_p, const double *f_T, double *p, double *T,
                 double rtol, int max_cycles, int nu1, int nu2, int pin_mean,
                 double *hist)
{
    orc_mg mg;
    mg_build(&mg, dim, n, h, F, axi, B, pin_mean);
    orc_level *l0 = &mg.L[0];
    long N = l0->N;
    memcpy(l0->f_p, f_p, sizeof(double) * N);
    memcpy(l0->f_T, f_T, sizeof(double) * N);
    const double *np_ = lam ? b_p : f_p, *nT_ = lam ? b_T : f_T;
    double bn[2] = {sqrt(dot(N, np_, np_)), sqrt(dot(N, nT_, nT_))};
    double *rp = malloc(sizeof(double) * N), *rT = malloc(sizeof(double) * N);
    double *rfp = malloc(sizeof(double) * N), *rfT = malloc(sizeof(double) * N);
    int cycles = 0, done = 0;
    for (;;) {
        if (lam) orc_paper_residual(dim, n, h, F, axi, lam, b_p, b_T, p, T, rp, rT);
        else orc_residual(dim, n, h, F, axi, B, f_p, f_T, p, T, rp, rT);
        double rel[2];
        rel[0] = bn[0] > 0 ? sqrt(dot(N, rp, rp)) / bn[0] : sqrt(dot(N, rp, rp));
        rel[1] = bn[1] > 0 ? sqrt(dot(N, rT, rT)) / bn[1] : sqrt(dot(N, rT, rT));
        if (hist) { hist[2 * cycles] = rel[0]; hist[2 * cycles + 1] = rel[1]; }
        if (rel[0] <= rtol && rel[1] <= rtol) { done = 1; break; }
        if (cycles >= max_cycles) break;
        /* correction equation in canonical form */
        orc_residual(dim, n, h, l0->F, axi, l0->B, f_p, f_T, p, T, rfp, rfT);
        memcpy(l0->f_p, rfp, sizeof(double) * N);
        memcpy(l0->f_T, rfT, sizeof(double) * N);
        vcycle(&mg, 0, nu1, nu2);
        for (long i = 0; i < N; i++) { p[i] += l0->u_p[i]; T[i] += l0->u_T[i]; }
        if (pin_mean) {
            double mp = 0, mT = 0;
            for (long i = 0; i < N; i++) { mp += p[i]; mT += T[i]; }
            mp /= N; mT /= N;
            for (long i = 0; i < N; i++) { p[i] -= mp; T[i] -= mT; }
        }
        cycles++;
    }
    free(rp); free(rT); free(rfp); free(rfT);
    mg_free(&mg);
    return done ? cycles : -1;
}

/* Number of multigrid levels the oracle builds for a grid. */
int orc_mg_levels(int dim, const int *n)
{
    int m[3] = {n[0], n[1], n[2]}, l = 1;
    while (can_coarsen(dim, m)) { int c[3]; coarse_dims(dim, m, c); memcpy(m, c, sizeof m); l++; }
    return l;
}

/* ------------------------------------------------------------------ */
/* after the solve: velocity correction and phase energies (Sec. 3)    */
/* ------------------------------------------------------------------ */

/* Face velocities: U[a] holds the velocity component normal to the faces
 * across axis a.  There are n_a + 1 faces along a (both walls included)
 * and n_b along every other axis b; face (i,j,k) is the lower face of cell
 * (i,j,k).  Index i + m0*(j + m1*k) with m_b = n_b + (b == a). */
static long fidx(const int *n, int a, long i, long j, long k)
{
    long m0 = n[0] + (a == 0), m1 = n[1] + (a == 1);
    return i + m0 * (j + m1 * k);
}

/* Discrete divergence of face velocities: the sum over axes of
 * (m_hi U on the upper face - m_lo U on the lower face) / h, m = 1 or the
 * r-z metric of axi_face on radial faces.  This is the div u* of Eq. (17)
 * and of lambda_p in Eq. (34). */
void orc_divergence(int dim, const int *n, double h, int axi, const double *const *U,
                    double *div)
{
    for (long k = 0; k < n[2]; k++)
        for (long j = 0; j < n[1]; j++)
            for (long i = 0; i < n[0]; i++) {
                double s = 0.0;
                for (int a = 0; a < dim; a++) {
                    long up[3] = {i, j, k};
                    up[a] += 1;
                    double m_lo = 1.0, m_hi = 1.0;
                    if (axi && a == 1) { m_lo = axi_face(j, j); m_hi = axi_face(j + 1, j); }
                    s += (m_hi * U[a][fidx(n, a, up[0], up[1], up[2])]
                          - m_lo * U[a][fidx(n, a, i, j, k)]) / h;
                }
                div[idx3(n, i, j, k)] = s;
            }
}

/* (1/rho) dp/dn on face (i,j,k) across axis a: the p face coefficient of
 * the solve (the face mean of 1/rho, F[a]) times the pressure difference
 * between the upper and the lower cell over h.  Zero on the two walls,
 * where the solve has no flux either. */
static double face_accel(const int *n, int a, double h, const double *F, const double *p,
                         long i, long j, long k)
{
    long ii[3] = {i, j, k};
    if (ii[a] == 0 || ii[a] == n[a]) return 0.0;
    long N = (long)n[0] * n[1] * n[2];
    long R = idx3(n, i, j, k);
    ii[a] -= 1;
    long L = idx3(n, ii[0], ii[1], ii[2]);
    return F[(long)a * N + R] * (p[R] - p[L]) / h;
}

/* Velocity correction, Eq. (unp1): u^{n+1} = u* - dt (1/rho) grad p^{n+1}.
 * On faces, with the face coefficient of the solve, so that the divergence
 * of the corrected face velocities is the one of Eq. (17) that the solve
 * used.  At cell centres (us, u not NULL), (1/rho) grad p along each axis is
 * the mean of its values on the cell's two faces across that axis. */
void orc_project(int dim, const int *n, double h, double dt, const double *F,
                 const double *p, const double *const *Us, double *const *U,
                 const double *const *us, double *const *u)
{
    for (int a = 0; a < dim; a++) {
        long m[3] = {n[0], n[1], n[2]};
        m[a] += 1;
        for (long k = 0; k < m[2]; k++)
            for (long j = 0; j < m[1]; j++)
                for (long i = 0; i < m[0]; i++) {
                    long f = fidx(n, a, i, j, k);
                    U[a][f] = Us[a][f] - dt * face_accel(n, a, h, F, p, i, j, k);
                }
    }
    if (!us || !u) return;
    for (long k = 0; k < n[2]; k++)
        for (long j = 0; j < n[1]; j++)
            for (long i = 0; i < n[0]; i++) {
                long c = idx3(n, i, j, k);
                for (int a = 0; a < dim; a++) {
                    long up[3] = {i, j, k};
                    up[a] += 1;
                    double g_lo = face_accel(n, a, h, F, p, i, j, k);
                    double g_hi = face_accel(n, a, h, F, p, up[0], up[1], up[2]);
                    u[a][c] = us[a][c] - dt * 0.5 * (g_lo + g_hi);
                }
            }
}

/* Phase pressures from the one-fluid pressure, Eqs. (37)-(38):
 * p1 = p + (1 - C) sigma kappa, p2 = p - C sigma kappa (kappa NULL: none). */
void orc_phase_pressures(long N, const double *p, const double *C, const double *kappa,
                         double sigma, double *p1, double *p2)
{
    for (long c = 0; c < N; c++) {
        double sk = kappa ? sigma * kappa[c] : 0.0;
        p1[c] = p[c] + (1.0 - C[c]) * sk;
        p2[c] = p[c] - C[c] * sk;
    }
}

/* Phase total energies at the end of the step, Eq. (39) without the viscous
 * work (inviscid): for phase i, with C_1 = C and C_2 = 1 - C,
 *   (C_i rho_i e_T,i)^{n+1} = (C_i rho_i e_T,i)^(adv)
 *                             + dt C_i [ -div(p_i u) + div(k grad T) ],
 * the heat flux -q_i = k grad T^{n+1} being the one of the T equation (face
 * coefficient F[3 + a], zero through the walls).  The pressure-work flux on
 * a face is the mean of the two cells' p_i times the face velocity; on a
 * wall face the cell's own p_i (zero normal gradient, as in the solve).
 * With axi, the flux differences carry the r-z metric of the divergence. */
/* Viscous work of Eq. (39), one-fluid, per unit volume:
 *     W = div( mu (grad u + grad u^T) . u )
 * for the end-of-step velocity u^{n+1}, written as the sum over the faces
 * of a cell of the normal flux (tau . u)_a on the faces across axis a.  On
 * the face between the cells L and R across axis a:
 *   - velocity: the normal component is the face velocity U_a, every
 *     other component the mean of the two cells' velocities;
 *   - stress (Stokes' hypothesis, no bulk viscosity):
 *       tau_aa = 2 mu_f (u_a(R) - u_a(L)) / h,
 *       tau_ab = mu_f [ (u_b(R) - u_b(L)) / h + (g_ba(L) + g_ba(R)) / 2 ],  b != a,
 *     g_ba(c) the centred difference of u_a along b at cell c, with the
 *     value mirrored across a wall (zero gradient);
 *   - mu_f: the mean of the two cells' mu_bar = C mu_1 + (1 - C) mu_2.
 * No flux crosses a wall (no penetration, free slip).  r-z: radial faces
 * carry the metric of axi_face, as the other fluxes.  u[b] are the cell
 * velocities per axis, U[a] the face velocities. */
static double cell_vel(const int *n, const double *const *u, int b, long i, long j, long k)
{
    return u[b][idx3(n, i, j, k)];
}

/* centred difference of u_a along b at cell (i,j,k), mirrored at walls */
static double grad_c(const int *n, double h, const double *const *u, int a, int b,
                     long i, long j, long k)
{
    long lo[3] = {i, j, k}, hi[3] = {i, j, k};
    if (lo[b] > 0) lo[b] -= 1;
    if (hi[b] < n[b] - 1) hi[b] += 1;
    return (cell_vel(n, u, a, hi[0], hi[1], hi[2]) - cell_vel(n, u, a, lo[0], lo[1], lo[2]))
           / (2.0 * h);
}

/* normal viscous work flux (tau . u)_a on the interior face between L = me - e_a and R = me */
static double visc_flux(int dim, const int *n, double h, const double *C, double mu1,
                        double mu2, const double *const *U, const double *const *u, int a,
                        long i, long j, long k)
{
    long L[3] = {i, j, k};
    L[a] -= 1;
    long cL = idx3(n, L[0], L[1], L[2]), cR = idx3(n, i, j, k);
    double muL = C[cL] * mu1 + (1.0 - C[cL]) * mu2;
    double muR = C[cR] * mu1 + (1.0 - C[cR]) * mu2;
    double mu_f = 0.5 * (muL + muR);
    double flux = 0.0;
    for (int b = 0; b < dim; b++) {
        double ub_f, tau;
        double duR = cell_vel(n, u, b, i, j, k), duL = cell_vel(n, u, b, L[0], L[1], L[2]);
        if (b == a) {
            ub_f = U[a][fidx(n, a, i, j, k)];
#if ORC_PLANT == 4
            tau = mu_f * (duR - duL) / h;
#else
            tau = 2.0 * mu_f * (duR - duL) / h;
#endif
        } else {
            ub_f = 0.5 * (duL + duR);
            double gL = grad_c(n, h, u, a, b, L[0], L[1], L[2]);
            double gR = grad_c(n, h, u, a, b, i, j, k);
#if ORC_PLANT == 4 || ORC_PLANT == 5
            (void)gL;
            (void)gR;
            tau = mu_f * (duR - duL) / h;
#else
            tau = mu_f * ((duR - duL) / h + 0.5 * (gL + gR));
#endif
        }
        flux += tau * ub_f;
    }
    return flux;
}

void orc_viscous_work(int dim, const int *n, double h, int axi, const double *C, double mu1,
                      double mu2, const double *const *U, const double *const *u, double *W)
{
    for (long k = 0; k < n[2]; k++)
        for (long j = 0; j < n[1]; j++)
            for (long i = 0; i < n[0]; i++) {
                long c = idx3(n, i, j, k);
                double w = 0.0;
                for (int a = 0; a < dim; a++) {
                    long ii[3] = {i, j, k};
                    double f_lo = 0.0, f_hi = 0.0;
                    if (ii[a] > 0) f_lo = visc_flux(dim, n, h, C, mu1, mu2, U, u, a, i, j, k);
                    if (ii[a] < n[a] - 1) {
                        long t[3] = {i, j, k};
                        t[a] += 1;
                        f_hi = visc_flux(dim, n, h, C, mu1, mu2, U, u, a, t[0], t[1], t[2]);
                    }
                    double m_lo = 1.0, m_hi = 1.0;
                    if (axi && a == 1) { m_lo = axi_face(j, j); m_hi = axi_face(j + 1, j); }
                    w += (m_hi * f_hi - m_lo * f_lo) / h;
                }
                W[c] = w;
            }
}

/* Phase energies of Eq. (39): pressure work, viscous work W (one-fluid,
 * from orc_viscous_work, or NULL: inviscid) and heat flux, each phase
 * taking its volume fraction of the one-fluid terms. */
void orc_energy_update(int dim, const int *n, double h, double dt, const double *F, int axi,
                       const double *C, const double *p1, const double *p2, const double *T,
                       const double *const *U, const double *E1a, const double *E2a,
                       const double *Wv, double *E1, double *E2)
{
    long N = (long)n[0] * n[1] * n[2];
    for (long k = 0; k < n[2]; k++)
        for (long j = 0; j < n[1]; j++)
            for (long i = 0; i < n[0]; i++) {
                long c = idx3(n, i, j, k);
                double w1 = 0.0, w2 = 0.0, q = 0.0;   /* div(p1 u), div(p2 u), div(k grad T) */
                for (int a = 0; a < dim; a++) {
                    long ii[3] = {i, j, k};
                    /* lower face */
                    double u_lo = U[a][fidx(n, a, i, j, k)];
                    double P1lo = p1[c], P2lo = p2[c], q_lo = 0.0;
                    if (ii[a] > 0) {
                        long t[3] = {i, j, k};
                        t[a] -= 1;
                        long L = idx3(n, t[0], t[1], t[2]);
                        P1lo = 0.5 * (p1[L] + p1[c]);
                        P2lo = 0.5 * (p2[L] + p2[c]);
                        q_lo = F[(long)(3 + a) * N + c] * (T[c] - T[L]) / h;
                    }
                    /* upper face */
                    long t[3] = {i, j, k};
                    t[a] += 1;
                    double u_hi = U[a][fidx(n, a, t[0], t[1], t[2])];
                    double P1hi = p1[c], P2hi = p2[c], q_hi = 0.0;
                    if (ii[a] < n[a] - 1) {
                        long R = idx3(n, t[0], t[1], t[2]);
                        P1hi = 0.5 * (p1[c] + p1[R]);
                        P2hi = 0.5 * (p2[c] + p2[R]);
                        q_hi = F[(long)(3 + a) * N + R] * (T[R] - T[c]) / h;
                    }
                    double m_lo = 1.0, m_hi = 1.0;
                    if (axi && a == 1) { m_lo = axi_face(j, j); m_hi = axi_face(j + 1, j); }
                    w1 += (m_hi * P1hi * u_hi - m_lo * P1lo * u_lo) / h;
                    w2 += (m_hi * P2hi * u_hi - m_lo * P2lo * u_lo) / h;
                    q += (m_hi * q_hi - m_lo * q_lo) / h;
                }
                double wv = Wv ? Wv[c] : 0.0;
                E1[c] = E1a[c] + dt * C[c] * (-w1 + wv + q);
                E2[c] = E2a[c] + dt * (1.0 - C[c]) * (-w2 + wv + q);
            }
}
