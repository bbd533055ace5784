// Internal declarations shared by the kernels and the host driver of libptmg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "pt_mg.h"

namespace ptmg {

// Vector types of one precision: a (p, T) pair and a 2x2 block.
template <typename R> struct VT;
template <> struct VT<float> { using v2 = float2; using v4 = float4; };
template <> struct VT<double> { using v2 = double2; using v4 = double4; };

// Constants of the finest-grid operator of phases mode.  Per phase i
// (0 liquid, 1 gas) the canonical block of Eqs. 29-32 is
//   [[K1, -beta/dt^2], [-beta T/dt, K2]],  K1 = gamma/(rho c^2 dt^2),
//   K2 = rho c_p/dt,
// (Bpp = -l3 + l4 l2 and BpT = l4 l1 with l4 = beta/(rho c_p dt): the
// beta^2 terms of l3 and l4 l2 cancel), with beta fixed or from Eq. (10)
// at (p, T); the cell block is the C-average of the two,
//   [[C K1_1 + (1-C) K1_2, -bb/dt^2], [-bb T/dt, C K2_1 + (1-C) K2_2]],
// bb = C beta_1 + (1-C) beta_2, so a cell's block is kept as the pair
// (C, bb) and T (compact block), and the cell coefficients are
// a_p = 1/(C rho_1 + (1-C) rho_2), a_T = C k_1 + (1-C) k_2.
template <typename R> struct CBK {
    R K1[2], K2[2];
    R idt, idt2;            // 1/dt, 1/dt^2
};
struct OpK {
    double rho[2], k[2];
    double beta[2];              // > 0: fixed; 0: Eq. (10)
    double gcv[2], b[2], Pi[2];  // Eq. (10): beta = gcv / (gcv T + b (p + Pi))
    CBK<double> blk;
};

// One grid level as the kernels see it.  Level 0 has cell coefficients
// (faces are their harmonic means) and its block stored, or in phases mode
// the compact block (cb, T0 and the constants k); coarser levels store
// face coefficients (lower face of each cell, 0 on the boundary).
// Coefficients are unscaled; kernels multiply by inv_h2.
template <typename R> struct Lvl {
    int nx, ny, nz;
    long long N;
    double inv_h2;
    const typename VT<R>::v2 *ac;              // cell (a_p, a_T), level 0 stored only
    const typename VT<R>::v2 *fx, *fy, *fz;    // faces, coarse levels only
    const typename VT<R>::v4 *B;               // block (pp, pT, Tp, TT), unless cb
    typename VT<R>::v2 *u;                     // unknowns (p, T)
    typename VT<R>::v2 *f;                     // right-hand side (p, T)
    // axisymmetric r-z grids, level 0 only (null otherwise): per row j,
    // (j/(j+1/2), (j+1)/(j+1/2), j+1/2, j), the radial face metric of the
    // lower and upper face per unit volume, the cell radius and the lower
    // face radius in units of h
    const typename VT<R>::v4 *axm;
    // level 0, compact block (cb non-null): (C, bb) per cell, T at
    // T0[g & tmask] (tmask 0: one T for every cell), and the constants
    const typename VT<R>::v2 *cb;
    const R *T0;
    long long tmask;
    CBK<R> k;
    // non-null: the launch does nothing once *gate != 0 (the stream-ordered
    // solve has decided to stop)
    const int *gate;
    R omega;
};

// Outer FP64 residual arguments (finest grid).
template <typename RV> struct OuterArgs {
    int nx, ny, nz;
    long long N;
    double inv_h2;
    const double4 *axm;            // r-z metric per row (2-D) or null
    int phases;                    // 1: paper form (b = (lp, lT)), 0: canonical
    const double2 *ac;             // FP64 cell coefficients (unread with the compact block)
    const double4 *B;              // FP64 block, or
    const double2 *cb;             // the compact block (non-null) as in Lvl
    const double *T0;
    long long tmask;
    CBK<double> k;
    double rho[2], kc[2];          // compact block: a_p = 1/(C rho_1 + (1-C) rho_2),
                                   // a_T = C k_1 + (1-C) k_2 formed from C
    const double *b_p, *b_T;       // mode-native right-hand side (null: zero)
    const double *bshift;          // [2] sums of b (mean constraint) or null
    double bshift_scale;           // b -= bshift_scale * bshift (1/N: the mean)
    const double *src_p, *src_T;   // current iterate (null: zero)
    double *dst_p, *dst_T;         // updated iterate (update = 1)
    // the iterate as (p, T) pairs in the V-cycle's precision where that
    // holds it exactly (the first from a zero guess is the correction
    // itself): read instead of src_p, src_T; written instead of dst_p, dst_T
    const typename VT<RV>::v2 *src32;
    typename VT<RV>::v2 *dst32;
    const typename VT<RV>::v2 *du; // correction of the last V-cycle (update = 1)
    typename VT<RV>::v2 *r;        // canonical residual out (V-cycle RHS) or null
    double *res_p, *res_T;         // mode-native residual out or null
    double *r64_p, *r64_T;         // canonical residual out in FP64 or null
    double *partials;              // [4 * gridDim.x]: sum res_p^2, res_T^2, b_p^2, b_T^2
    int update;
    const int *gate;               // as in Lvl
};

// Stream-ordered solve: what the stop test writes after each residual
// (pinned host memory), and the device words the launches read: gate[0]
// != 0 once the solve has stopped, gate[1] the final outer iteration k.
struct AsyncInfo {
    int status;           // PT_OK, PT_ERR_NOCONV, or -1 while running
    int cycles;
    int hist_len;
    int nonfinite;
    double relres[2];
    double hist[2 * PT_MAX_HIST];
};

struct AsmArgs {
    long long N;
    int mode;
    // explicit
    const double *alpha_p, *alpha_T;
    double alpha_p_const, alpha_T_const;
    const double *B;
    double B_const[4];
    // phases
    const double *C;
    pt_phase liq, gas;
    double dt;
    const double *p_adv, *T_adv;
    double p_adv_const, T_adv_const;
    // state
    const double *m1, *m2;
    // outputs: the cell coefficients and the stored block (B64 null: the
    // block is kept compact) ...
    double2 *ac64;
    double4 *B64;
    float2 *ac32;   // may be null
    float4 *B32;    // may be null
    // ... or, phases mode in mixed precision, the compact block with its T
    // (T_cells 0: the one T in element 0); k64: the phases' constants
    double2 *cb64;  // null: not compact
    double *T64;
    float2 *cb32;
    float *T32;
    int T_cells;
    OpK k64;
    // phases and state mode: the paper right-hand side (Eqs. 33-34) formed
    // with the block, into b_p, b_T (null: not formed); div null: zero
    const double *div;
    double *b_p, *b_T;
    int *flags;     // [0] argument errors, [1] singular blocks, [2] nonzero B
};

enum { FLAG_ARG = 0, FLAG_SINGULAR = 1, FLAG_BNONZERO = 2, FLAG_PIVOT = 3, NFLAGS = 4 };

constexpr int kBlock = 256;
constexpr int kMaxLevels = 24;
constexpr int kMaxTail = 8;

// Arguments of the single-block tail cycle: global views of its levels and
// the LDS byte offsets of each level's u, f, fx, fy, fz, B.
// The small end of the hierarchy build (launch_hier_small): coarsen
// g[0] -> ... -> g[nl-1], then the dense matrix of g[nl-1] (pin: mean
// constraint) into M0 and its Gauss-Jordan inverse (m x m) into Ainv.
template <typename R> struct HierSmallArgs {
    int nl, pin, m;
    Lvl<R> g[kMaxTail];
    double *M0, *Ainv;
    int *flags;
};
// false (nothing launched) when m exceeds the LDS inverse or nl is not 2..kMaxTail
template <typename R>
bool launch_hier_small(int dim, const HierSmallArgs<R> &a, hipStream_t s);

template <typename R> struct TailArgs {
    int nl, m, nu1, nu2;
    Lvl<R> g[kMaxTail];
    int off[kMaxTail][6];
    const double *Ainv;
    int ainv_off;   // LDS offset of a copy of Ainv, or -1 (read from global memory)
};

// Provisional state (Eqs. 20, 23) of n cells.
void launch_state(const pt_state &st, hipStream_t s);

// Krylov vector kernels (FP64 pairs of arrays p, T of N cells).
// out = a x + b y (+ c z when z_p is not null); out may alias x, y or z.
void launch_lin3(long long N, double *out_p, double *out_T, double a, const double *x_p,
                 const double *x_T, double b, const double *y_p, const double *y_T, double c,
                 const double *z_p, const double *z_T, hipStream_t s);
// Two dot products d0 = <x, y>, d1 = <z, w> over both components, as
// fixed-order partial sums [4 per block] (d0, d1, 0, 0) for launch_reduce4;
// z_p null: d1 = 0.  Returns the block count.
int launch_dot2(long long N, const double *x_p, const double *x_T, const double *y_p,
                const double *y_T, const double *z_p, const double *z_T, const double *w_p,
                const double *w_T, double *partials, hipStream_t s);

// End-of-step pass on the finest grid: face and cell velocity correction
// and phase energies (pt_mg_downstream).  Face arrays per axis as in
// pt_mg.h; the 3-D-only members are null in 2-D.
struct DownArgs {
    int nx, ny, nz;
    double inv_h, dt, sigma;
    const double2 *ac;                 // FP64 cell (1/rho, k)
    const double *p, *T, *C, *kappa;   // kappa null: no surface tension
    const double *Ux, *Uy, *Uz;        // provisional face velocities
    double *Vx, *Vy, *Vz;              // corrected face velocities
    const double *ux, *uy, *uz;        // provisional cell velocities (null: none)
    double *vx, *vy, *vz;
    const double *E1a, *E2a;           // null: no energy update
    double *E1, *E2;
    const double4 *axm;                // r-z metric per row (2-D) or null
};
void launch_downstream(int dim, const DownArgs &a, hipStream_t s);
// Viscous work of Eq. (39) added to the phase energies E1, E2 in place,
// from the end-of-step face velocities U and cell velocities u (every axis
// < dim non-null).
struct ViscArgs {
    int nx, ny, nz;
    double inv_h, dt, mu1, mu2;
    const double *C;
    const double *Ux, *Uy, *Uz;        // face velocities
    const double *ux, *uy, *uz;        // cell velocities
    const double4 *axm;                // r-z metric per row (2-D) or null
    double *E1, *E2;
};
void launch_viscous(int dim, const ViscArgs &a, hipStream_t s);
// div = sum over axes of (U upper face - U lower face) * inv_h.
void launch_divergence(int dim, int nx, int ny, int nz, double inv_h, const double *Ux,
                       const double *Uy, const double *Uz, const double4 *axm, double *div,
                       hipStream_t s);
// Fill the r-z metric table of ny rows in FP64 and, if m32 is not null, FP32.
void launch_axi_metric(int ny, double4 *m64, float4 *m32, hipStream_t s);

// ---- launch wrappers (implemented in ptmg_kernels.hip) --------------------
void launch_assemble(const AsmArgs &a, hipStream_t s);
void launch_fill_ac64(long long N, const double2 *cb, const double rho[2], const double kc[2],
                      double2 *ac, hipStream_t s);
// Eqs. (33)-(34) with the finest FP64 operator L (stored or derived).
void launch_paper_rhs(const Lvl<double> &L, const double *p_adv, double p_const,
                      const double *T_adv, double T_const, const double *div, double dt,
                      double *b_p, double *b_T, hipStream_t s);

template <typename RV>
int launch_outer_zm(int dim, const OuterArgs<RV> &a, hipStream_t s);   // returns #blocks
// the stop test of outer iteration k on the norms of its residual
void launch_async_decide(const double *norms, int k, double rtol, int max_cycles, int *gate,
                         AsyncInfo *info, hipStream_t s);
// the answer u_k into (p, T): from (xp, xT) when k + parity is odd, zero
// when k = 0 from a zero guess, from the FP32 pairs k1 when k = 1 and k1
// is given, else already there
void launch_async_final(const int *gate, int parity, int zero_guess, const double *xp,
                        const double *xT, const float2 *k1, double *p, double *T, long long N,
                        hipStream_t s);
// FP32 (p, T) pairs into FP64 p, T (k1 may alias p)
void launch_pairs_to_fp64(const float2 *k1, double *p, double *T, long long N, hipStream_t s);
void launch_gate_reset(int *gate, AsyncInfo *info, hipStream_t s);
int outer_zm_blocks(int dim, int nx, int ny, int nz);
int reduce_scratch(int nblocks);   // extra partial slots launch_reduce4 needs
void launch_reduce4(const double *partials, int nblocks, double *out4, hipStream_t s,
                    const int *gate = nullptr);
void launch_sum2(long long N, const double *x, const double *y, double *partials, int nblocks,
                 double *out2, hipStream_t s);   // out2 = (sum x, sum y), fixed order
int sum2_blocks(long long N);
void launch_shift2(long long N, double *x, double *y, const double *mean2, double scale,
                   hipStream_t s);  // x -= scale*sum2[0], y -= scale*sum2[1]

template <typename R>
void launch_rb_pass(int dim, int level0, const Lvl<R> &L, int color, int zero_guess,
                    hipStream_t s);
// 2-D finest level: one sweep, optionally with the prolonged correction
// added on load (pro) or the restricted residual written to C.f (res).
template <typename R>
void launch_tile2x(const Lvl<R> &L, const Lvl<R> &C, typename VT<R>::v2 *uo, int zero_guess,
                   int pro, int res, hipStream_t s);
// 2-D coarse level, nu in {1, 2}: down = nu sweeps from zero + restricted
// residual into C.f; up = prolongation from C.u + nu sweeps into uo.
template <typename R>
void launch_half2(bool up, int nu, const Lvl<R> &L, const Lvl<R> &C, typename VT<R>::v2 *uo,
                  hipStream_t s);
template <typename R>
void launch_rb_fused(int dim, const Lvl<R> &L, typename VT<R>::v2 *uo, int zero_guess, int faces,
                     hipStream_t s);
// 3-D finest level, FP32: one sweep with the residual restricted into C.f
// (the last pre-smoothing sweep); a no-op for FP64 (LDS-bound).
template <typename R>
void launch_rb_fused3r(const Lvl<R> &L, const Lvl<R> &C, typename VT<R>::v2 *uo, int zero_guess,
                       hipStream_t s);
template <typename R>
void launch_restrict(int dim, int level0, const Lvl<R> &F, const Lvl<R> &C, hipStream_t s);
template <typename R>
void launch_restrict_zm(int dim, const Lvl<R> &F, const Lvl<R> &C, hipStream_t s,
                        bool faces = false);  // finest grid, or (faces) a 3-D coarse level
template <typename R> size_t tail_level_lds(int dim, long long N);
template <typename R>
bool launch_tail(int dim, const TailArgs<R> &a, size_t lds_bytes, hipStream_t s);
template <typename R> void tail_set_lds_limit(int dim, size_t bytes);
template <typename R>
void launch_prolong(int dim, const Lvl<R> &F, const Lvl<R> &C, hipStream_t s);
// zm: a 3-D finest level coarsens with the plane-marching kernel (bitwise
// the gather kernel's result)
template <typename RIN, typename ROUT>
void launch_coarsen(int dim, int level0, const Lvl<RIN> &F, typename VT<ROUT>::v2 *fx,
                    typename VT<ROUT>::v2 *fy, typename VT<ROUT>::v2 *fz,
                    typename VT<ROUT>::v4 *B, hipStream_t s, bool zm = false);
template <typename R>
void launch_coarse_dense(int dim, int level0, const Lvl<R> &L, int pin_mean, double *M,
                         hipStream_t s);
void launch_gj_step(const double *A, double *Bm, int m, int k, int *flags, hipStream_t s);
bool launch_gj_lds(const double *A, double *Ainv, int m, int *flags, hipStream_t s);  // m <= 128
template <typename R>
void launch_coarse_apply(const double *Ainv, int m, const R *f, R *u, hipStream_t s,
                         const int *gate = nullptr);
template <typename R>
void launch_export_op(int dim, int level0, const Lvl<R> &L, double *faces, double *B,
                      hipStream_t s);
template <typename R>
void launch_pack(long long N, const double *p, const double *T, typename VT<R>::v2 *out,
                 hipStream_t s);
template <typename R>
void launch_unpack(long long N, const typename VT<R>::v2 *in, double *p, double *T,
                   hipStream_t s);
template <typename RIN, typename ROUT>
void launch_convert(long long n, const RIN *in, ROUT *out, hipStream_t s);
void launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
void launch_zero(void *p, size_t bytes, hipStream_t s, const int *gate = nullptr);
void launch_zero2(void *p, void *q, size_t bytes, hipStream_t s);   // both arrays
void launch_flags_out(const int *src, int *dst, int n, hipStream_t s);   // n <= 64

// ---- handle internals used by the serving engine (ptmg_host.hip) ---------
constexpr int PT_RUNNING = -1;
int handle_create(const pt_problem *prob, int precision, hipStream_t stream, char *dev_mem,
                  size_t bytes, void *pinned, pt_mg_t *out, std::string *err);
hipEvent_t handle_event(pt_mg_t h);
int handle_setup_check(pt_mg_t h);
size_t handle_plan_bytes(const pt_problem *prob, int precision);
int solve_begin(pt_mg_t h, const double *b_p, const double *b_T, double *p, double *T,
                const pt_solve_opts *opts);
int solve_advance(pt_mg_t h, pt_solve_info *info);
int handle_paper_rhs_async(pt_mg_t h, const double *p_adv, const double *T_adv,
                           const double *div_ustar, double *b_p, double *b_T);
const char *handle_error(pt_mg_t h);

}  // namespace ptmg
