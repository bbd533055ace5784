// HIP kernels of libptmg (gfx950, wave64).
//
// Grid conventions: cell (i, j, k) at i + nx*(j + ny*k); 2-D grids have
// nz = 1.  Unknowns and right-hand sides of the V-cycle are interleaved
// (p, T) pairs; the caller's FP64 fields are separate p and T arrays.
//
// The operator is the canonical form of the paper's coupled system
// (Eqs. 27-28 after the row operations T-row := -Eq. 27,
// p-row := -(Eq. 28 - l4 Eq. 27)):
//   (A u)_c = sum_faces w_c (u_c,cell - u_c,nbr) + (B u)_c,   w = a_face / h^2,
// with zero flux through boundary faces.
#include <algorithm>
#include <cstdlib>

#include <mutex>

#include "ptmg_internal.h"

namespace ptmg {

// ---------------------------------------------------------------- helpers
// Quotient of the V-cycle arithmetic (smoothers, transfers, coarse
// operators): the V-cycle approximates the correction and the FP64 outer
// residual decides the answer, so its quotients need not be correctly
// rounded.  FP32: the hardware reciprocal (1 ulp) times the numerator.
// FP64: the hardware reciprocal seed refined by two Newton steps
// (x <- x + x (1 - b x); the relative error squares at each step), times
// the numerator: half the instructions of a rounded division, which bounds
// the FP64 sweeps.  The outer residual and the end-of-step pass divide
// exactly (harm_exact).
template <typename R> __device__ __forceinline__ R quot(R a, R b);
template <> __device__ __forceinline__ float quot<float>(float a, float b)
{
    return a * __builtin_amdgcn_rcpf(b);
}
template <> __device__ __forceinline__ double quot<double>(double a, double b)
{
    double x = __builtin_amdgcn_rcp(b);
    double e = __builtin_fma(-b, x, 1.0);
    x = __builtin_fma(x, e, x);
    e = __builtin_fma(-b, x, 1.0);
    x = __builtin_fma(x, e, x);
    return a * x;
}

// Fused multiply-add written out, where two kernels must round alike
// whatever the compiler contracts elsewhere.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Over-relaxation of a block Gauss-Seidel update: old + omega (new - old);
// omega = 1 leaves the plain update (coarse levels always, the finest
// level unless PT_OPT_OMEGA says otherwise).
// The update enters as a value the compiler cannot see into (an empty
// asm statement holds it in a register), so that no kernel contracts the
// difference with the product that formed the update and every kernel
// rounds alike.
template <typename T> __device__ __forceinline__ T opaque(T v)
{
    asm volatile("" : "+v"(v));
    return v;
}
template <typename R, typename V2>
__device__ __forceinline__ V2 relax(R omega, V2 o, V2 old)
{
    if (omega != R(1)) {
        o.x = fmadd(omega, opaque(o.x) - old.x, old.x);
        o.y = fmadd(omega, opaque(o.y) - old.y, old.y);
    }
    return o;
}

// The harmonic mean 2ab/(a+b) of two non-negative coefficients, zero when
// both are zero: the sum is taken no smaller than the least normal number,
// so a zero pair gives 0 * (finite reciprocal) = 0 without a select, and
// every normal sum gives the plain quotient.
template <typename R>
__device__ __forceinline__ R harm(R a, R b)
{
    constexpr R tiny = sizeof(R) == 4 ? R(1.17549435e-38f) : R(2.2250738585072014e-308);
    const R s = fmax(a + b, tiny);
    return quot(R(2) * a * b, s);
}

template <typename V2>
__device__ __forceinline__ V2 harm2(V2 a, V2 b)
{
    V2 o;
    o.x = harm(a.x, b.x);
    o.y = harm(a.y, b.y);
    return o;
}

// The harmonic mean with a correctly rounded division (FP64 operator of
// record: outer residual, end of the step).
__device__ __forceinline__ double harm_exact(double a, double b)
{
    const double s = a + b;
    return s > 0.0 ? 2.0 * a * b / s : 0.0;
}
// A launch of a stream-ordered solve does nothing once the solve has
// stopped (the flag is written by an earlier launch on the same stream).
__device__ __forceinline__ bool gated(const int *gate) { return gate && *gate != 0; }

__device__ __forceinline__ double2 harm2_exact(double2 a, double2 b)
{
    return make_double2(harm_exact(a.x, b.x), harm_exact(a.y, b.y));
}

// ------------------------------------------------ finest-grid operator
// Phases mode (the assembly, FP64): cell coefficients a_p = 1/(C rho_1 +
// (1-C) rho_2), a_T = C k_1 + (1-C) k_2, thermal dilations of Eq. (10) at
// (p, T) (or fixed), and their C-average bb.  Divisions are correctly
// rounded; every multiply-add is written out (fmadd) or kept as a
// separate product, so that each kernel computes the same bits.
__device__ __forceinline__ double2 phases_ac(const double (&rho)[2], const double (&kc)[2],
                                             double C)
{
    const double g = 1.0 - C;
    return make_double2(1.0 / fmadd(C, rho[0], g * rho[1]), fmadd(C, kc[0], g * kc[1]));
}
__device__ __forceinline__ double phases_beta(const OpK &k, int q, double p, double T)
{
    if (k.beta[q] > 0.0) return k.beta[q];
    return k.gcv[q] / fmadd(k.gcv[q], T, k.b[q] * (p + k.Pi[q]));
}

// The block of a cell from its compact form (C, bb) and T.
template <typename R>
__device__ __forceinline__ typename VT<R>::v4 compact_B(const CBK<R> &k, R C, R bb, R T)
{
    const R g = R(1) - C;
    typename VT<R>::v4 B;
    B.x = fmadd(C, k.K1[0], g * k.K1[1]);
    B.y = -bb * k.idt2;
    B.z = -(bb * T) * k.idt;
    B.w = fmadd(C, k.K2[0], g * k.K2[1]);
    return B;
}

// The finest level's block at cell g, stored or compact (coarse levels:
// the stored block).
template <typename R>
__device__ __forceinline__ typename VT<R>::v4 cell_B(const Lvl<R> &L, long long g)
{
    if (!L.cb) return L.B[g];
    const typename VT<R>::v2 c = L.cb[g];
    return compact_B(L.k, c.x, c.y, L.T0[g & L.tmask]);
}
template <typename R>
__device__ __forceinline__ typename VT<R>::v2 cell_ac(const Lvl<R> &L, long long g)
{
    return L.ac[g];
}

// Two-stage access for the kernels that load planes ahead of their use:
// the raw load (the stored block, or the compact block with T) and the
// arithmetic that finishes it where it is used, so that the loads stay in
// flight meanwhile.
template <typename R>
__device__ __forceinline__ typename VT<R>::v4 cell_B_raw(const Lvl<R> &L, long long g)
{
    if (!L.cb) return L.B[g];
    const typename VT<R>::v2 c = L.cb[g];
    typename VT<R>::v4 r;
    r.x = c.x;
    r.y = c.y;
    r.z = L.T0[g & L.tmask];
    r.w = R(0);
    return r;
}
template <typename R>
__device__ __forceinline__ typename VT<R>::v4 cell_B_fin(const Lvl<R> &L, typename VT<R>::v4 r)
{
    if (!L.cb) return r;
    return compact_B(L.k, r.x, r.y, r.z);
}

// The smoothers' and the V-cycle's restriction's access: the block is
// compact only on the finest level of an FP32 V-cycle, so an FP64 V-cycle's
// kernels read the stored block and carry no compact path.
template <typename R>
__device__ __forceinline__ typename VT<R>::v4 sweep_B(const Lvl<R> &L, long long g)
{
    if constexpr (sizeof(R) == 8) return L.B[g];
    else return cell_B(L, g);
}
template <typename R>
__device__ __forceinline__ typename VT<R>::v4 sweep_B_raw(const Lvl<R> &L, long long g)
{
    if constexpr (sizeof(R) == 8) return L.B[g];
    else return cell_B_raw(L, g);
}
template <typename R>
__device__ __forceinline__ typename VT<R>::v4 sweep_B_fin(const Lvl<R> &L, typename VT<R>::v4 r)
{
    if constexpr (sizeof(R) == 8) return r;
    else return cell_B_fin(L, r);
}

// The same for the FP64 outer residual (OuterArgs).
template <typename A> __device__ __forceinline__ double4 op_B64_raw(const A &a, long long g)
{
    if (!a.cb) return a.B[g];
    const double2 c = a.cb[g];
    return make_double4(c.x, c.y, a.T0[g & a.tmask], 0.0);
}
template <typename A> __device__ __forceinline__ double4 op_B64_fin(const A &a, double4 r)
{
    if (!a.cb) return r;
    return compact_B(a.k, r.x, r.y, r.z);
}

// Block-to-work mapping that is XCD-aware: the hardware deals
// consecutive block ids to the 8 XCDs in turn, so XCD x runs blocks
// b = x, x + 8, ...; block b takes logical index (blocks of XCDs before x)
// + b / 8, which gives each XCD (and its L2) a contiguous run of work
// whose halos overlap.  With q = nb / 8 and r = nb % 8, XCD x has
// q + (x < r) blocks, so the map is a bijection of [0, nb).
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int x = b & 7, q = nb >> 3, r = nb & 7;
    return x * q + min(x, r) + (b >> 3);
}

__device__ __forceinline__ void decode(long long t, int nx, int ny, int &i, int &j, int &k)
{
    i = (int)(t % nx);
    long long r = t / nx;
    j = (int)(r % ny);
    k = (int)(r / ny);
}

// Face coefficient (unscaled) between cell `me` and neighbour `q` along
// `axis`; `upper` when q is the upper neighbour.
template <typename R, bool CF>
__device__ __forceinline__ typename VT<R>::v2 face_coef(const Lvl<R> &L,
                                                        typename VT<R>::v2 am, long long me,
                                                        long long q, int axis, bool upper)
{
    if (CF) return harm2(am, cell_ac(L, q));
    const typename VT<R>::v2 *F = axis == 0 ? L.fx : (axis == 1 ? L.fy : L.fz);
    return upper ? F[q] : F[me];
}

// Radial face coefficient per unit volume on an r-z grid: the face's
// harmonic coefficient times r_face / r_cell (the row's metric m).  Every
// level-0 kernel applies it the same way (before the 1/h^2 scaling), so
// that the fused and the reference paths agree bit for bit.
template <typename V2, typename V4>
__device__ __forceinline__ void axi_face(V2 &w, const V4 &m, bool upper)
{
    const auto f = upper ? m.y : m.x;
    w.x *= f;
    w.y *= f;
}

// Sums over the faces of cell (i,j,k): S = sum w, nb = sum w u_nbr (when
// USE_U), per component.  Face order: x-, x+, y-, y+, z-, z+.
template <typename R, int DIM, bool CF, bool USE_U>
__device__ __forceinline__ void gather(const Lvl<R> &L, int i, int j, int k, long long me,
                                       R &nbp, R &nbT, R &Sp, R &ST)
{
    using V2 = typename VT<R>::v2;
    const R ih2 = (R)L.inv_h2;
    nbp = nbT = Sp = ST = R(0);
    V2 am;
    if (CF) am = cell_ac(L, me);
    const long long sx = 1, sy = L.nx, sz = (long long)L.nx * L.ny;
    auto acc = [&](long long q, int axis, bool upper) {
        V2 w = face_coef<R, CF>(L, am, me, q, axis, upper);
        if (CF && axis == 1 && L.axm) axi_face(w, L.axm[j], upper);
        R wp = w.x * ih2, wT = w.y * ih2;
        Sp += wp;
        ST += wT;
        if (USE_U) {
            V2 uq = L.u[q];
            nbp += wp * uq.x;
            nbT += wT * uq.y;
        }
    };
    if (i > 0) acc(me - sx, 0, false);
    if (i < L.nx - 1) acc(me + sx, 0, true);
    if (j > 0) acc(me - sy, 1, false);
    if (j < L.ny - 1) acc(me + sy, 1, true);
    if (DIM == 3) {
        if (k > 0) acc(me - sz, 2, false);
        if (k < L.nz - 1) acc(me + sz, 2, true);
    }
}

__device__ __forceinline__ void block_reduce_store(double *v, int width, double *out)
{
    for (int q = 0; q < width; q++)
        for (int off = 32; off >= 1; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    __shared__ double sm[4][kBlock / 64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int q = 0; q < width; q++) sm[q][w] = v[q];
    __syncthreads();
    if (threadIdx.x < (unsigned)width) {
        double s = 0.0;
        for (int i = 0; i < kBlock / 64; i++) s += sm[threadIdx.x][i];
        out[threadIdx.x] = s;
    }
}

static inline unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------- assembly
// Per cell, the canonical block and the cell coefficients.  Phases mode:
// per phase Eqs. 29-32 with l4 = beta/(rho c_p dt), which give
// Bpp = -l3 + l4 l2 = gamma/(rho c^2 dt^2), BpT = l4 l1 = -beta/dt^2,
// BTp = -l2 = -beta T/dt, BTT = -l1 = rho c_p/dt, averaged with the liquid
// fraction C (the averaging rule of Sec. 3) and kept compact.  State mode:
// each phase's block weighted by its fraction from its own density;
// explicit mode: the given coefficients.
// The paper right-hand side of one cell (Eqs. 33-34) from its block (the
// lambdas as the block holds them: l1 = -B_TT, l2 = -B_Tp, l4 = B_pT / l1,
// l3 = -B_pp + l4 l2), its provisional p, T and div u*.  Every product and
// sum is written out, so the assembly (which forms it with the block) and
// k_paper_rhs round it the same way.
__device__ __forceinline__ void paper_rhs_cell(double4 B, double p, double T, double d, double dt,
                                               double &bp, double &bT)
{
    const double l1 = -B.w, l2 = -B.z, l4 = B.y / l1, l3 = fmadd(l4, l2, -B.x);
    bT = fmadd(l1, T, opaque(l2 * p));
    bp = fmadd(l3, p, d / dt);
}

__global__ __launch_bounds__(kBlock) void k_assemble(AsmArgs a)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= a.N) return;
    double2 ac;
    double4 B;
    double rp = 0.0, rT = 0.0;   // p, T of the paper right-hand side
    bool argbad = false;
    if (a.mode == PT_COEF_STATE) {
        // each phase's block weighted by its fraction, written with the
        // phase mass m_i = C_i rho_i so that nothing is divided by C_i:
        // C_i Bpp = gamma (C_i - m_i b) / (Gamma (p + Pi) dt^2)  (Eq. 11 in
        // gamma / (rho c^2)), C_i BpT = -C_i beta / dt^2, C_i BTp =
        // -C_i beta T / dt, C_i BTT = m_i c_p / dt (Eqs. 29-32)
        const double c = a.C[t], p = a.p_adv[t], T = a.T_adv[t];
        rp = p;
        rT = T;
        const double frac[2] = {c, 1.0 - c}, mass[2] = {a.m1[t], a.m2[t]};
        const pt_phase *ph[2] = {&a.liq, &a.gas};
        argbad = !(c >= 0.0 && c <= 1.0) || !isfinite(p) || !(T > 0.0) || !isfinite(T);
        B.x = B.y = B.z = B.w = 0.0;
        const double idt = 1.0 / a.dt;
        for (int q = 0; q < 2; q++) {
            const pt_phase &f = *ph[q];
            if (!(mass[q] >= 0.0)) argbad = true;
            if (frac[q] <= 0.0) continue;
            if (!(mass[q] > 0.0) || !(p + f.Pi > 0.0) || !(frac[q] - mass[q] * f.b > 0.0))
                argbad = true;
            double beta = f.beta;
            if (!(beta > 0.0)) {
                const double gcv = (f.Gamma - 1.0) * f.cv;
                beta = gcv / (gcv * T + f.b * (p + f.Pi));
            }
            B.x += f.gamma * (frac[q] - mass[q] * f.b) / (f.Gamma * (p + f.Pi)) * idt * idt;
            B.y += -frac[q] * beta * idt * idt;
            B.z += -frac[q] * beta * T * idt;
            B.w += mass[q] * f.cp * idt;
        }
        ac.x = 1.0 / (mass[0] + mass[1]);
        ac.y = c * a.liq.k + (1.0 - c) * a.gas.k;
    } else if (a.mode == PT_COEF_PHASES) {
        // cell coefficients, and the block kept compact: (C, bb) with
        // bb = C beta_1 + (1 - C) beta_2, and T where it varies per cell
        double c = a.C[t];
        double p = a.p_adv ? a.p_adv[t] : a.p_adv_const;
        double T = a.T_adv ? a.T_adv[t] : a.T_adv_const;
        rp = p;
        rT = T;
        argbad = !(c >= 0.0 && c <= 1.0) || !isfinite(p) || !(T > 0.0) || !isfinite(T);
        const double bb = fmadd(c, phases_beta(a.k64, 0, p, T), (1.0 - c) * phases_beta(a.k64, 1, p, T));
        B = compact_B(a.k64.blk, c, bb, T);
        ac = phases_ac(a.k64.rho, a.k64.k, c);
        if (a.cb64) {
            const bool wT = a.T_cells || t == 0;
            a.cb64[t] = make_double2(c, bb);
            a.cb32[t] = make_float2((float)c, (float)bb);
            if (wT) {
                a.T64[t] = T;
                a.T32[t] = (float)T;
            }
        }
    } else {
        ac.x = a.alpha_p ? a.alpha_p[t] : a.alpha_p_const;
        ac.y = a.alpha_T ? a.alpha_T[t] : a.alpha_T_const;
        if (a.B) {
            B.x = a.B[t];
            B.y = a.B[a.N + t];
            B.z = a.B[2 * a.N + t];
            B.w = a.B[3 * a.N + t];
        } else {
            B.x = a.B_const[0];
            B.y = a.B_const[1];
            B.z = a.B_const[2];
            B.w = a.B_const[3];
        }
        if (B.x != 0.0 || B.y != 0.0 || B.z != 0.0 || B.w != 0.0) atomicOr(&a.flags[FLAG_BNONZERO], 1);
    }
    argbad = argbad || !(ac.x >= 0.0) || !(ac.y >= 0.0) || !isfinite(ac.x) || !isfinite(ac.y) ||
             !isfinite(B.x) || !isfinite(B.y) || !isfinite(B.z) || !isfinite(B.w);
    bool sing = !(B.x > 0.0 && B.w > 0.0 && B.x * B.w - B.y * B.z > 0.0);
    if (argbad) atomicOr(&a.flags[FLAG_ARG], 1);
    if (sing) atomicOr(&a.flags[FLAG_SINGULAR], 1);
    if (a.b_p) paper_rhs_cell(B, rp, rT, a.div ? a.div[t] : 0.0, a.dt, a.b_p[t], a.b_T[t]);
    if (a.ac64) a.ac64[t] = ac;
    if (a.B64) a.B64[t] = B;
    if (a.ac32) a.ac32[t] = make_float2((float)ac.x, (float)ac.y);
    if (a.B32) a.B32[t] = make_float4((float)B.x, (float)B.y, (float)B.z, (float)B.w);
}

void launch_assemble(const AsmArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_assemble, dim3(nblk(a.N)), dim3(kBlock), 0, s, a);
}

// Phases mode: the FP64 cell coefficients from the compact block's C, as
// the assembly forms them.
struct AcK {
    double rho[2], kc[2];
};
__global__ __launch_bounds__(kBlock) void k_fill_ac64(long long N, const double2 *cb, AcK k,
                                                      double2 *ac)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= N) return;
    ac[t] = phases_ac(k.rho, k.kc, cb[t].x);
}

void launch_fill_ac64(long long N, const double2 *cb, const double rho[2], const double kc[2],
                      double2 *ac, hipStream_t s)
{
    AcK k;
    for (int q = 0; q < 2; q++) {
        k.rho[q] = rho[q];
        k.kc[q] = kc[q];
    }
    hipLaunchKernelGGL(k_fill_ac64, dim3(nblk(N)), dim3(kBlock), 0, s, N, cb, k, ac);
}

// Provisional state (Eqs. 20, 23) from the advected conserved variables;
// the phase averages are sums of fraction- and mass-weighted terms.
__global__ __launch_bounds__(kBlock) void k_state(pt_state st)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= st.n) return;
    const double c = st.C[t];
    const double frac[2] = {c, 1.0 - c}, mass[2] = {st.m1[t], st.m2[t]};
    const pt_phase *ph[2] = {&st.liquid, &st.gas};
    double e_static = 0.0, inv_gm1 = 0.0, vol = 0.0, vol_pi = 0.0, heat = 0.0;
    for (int q = 0; q < 2; q++) {
        const pt_phase &f = *ph[q];
        const double free_vol = frac[q] - mass[q] * f.b;   // C_i (1 - rho_i b)
        const double gpi = f.Gamma * f.Pi / (f.Gamma - 1.0);
        e_static += gpi * free_vol + mass[q] * f.q;
        inv_gm1 += free_vol / (f.Gamma - 1.0);
        vol += free_vol;
        vol_pi += f.Pi * free_vol;
        heat += mass[q] * (f.cp - f.cv);
    }
    const double rho = mass[0] + mass[1];
    double m2 = 0.0;
    for (int d = 0; d < st.dim; d++) {
        if (!st.mom[d]) continue;
        const double m = st.mom[d][t];
        m2 += m * m;
    }
    const double p = (st.E[t] - 0.5 * m2 / rho - e_static) / inv_gm1;
    st.p_adv[t] = p;
    st.T_adv[t] = (vol * p + vol_pi) / heat;
}

void launch_state(const pt_state &st, hipStream_t s)
{
    hipLaunchKernelGGL(k_state, dim3(nblk(st.n)), dim3(kBlock), 0, s, st);
}

// ---------------------------------------------- Krylov vector kernels
__global__ __launch_bounds__(kBlock) void k_lin3(long long N, double *op, double *oT, double a,
                                                 const double *xp, const double *xT, double b,
                                                 const double *yp, const double *yT, double c,
                                                 const double *zp, const double *zT)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= N) return;
    double vp = a * xp[t] + b * yp[t];
    double vT = a * xT[t] + b * yT[t];
    if (zp) {
        vp += c * zp[t];
        vT += c * zT[t];
    }
    op[t] = vp;
    oT[t] = vT;
}

void launch_lin3(long long N, double *out_p, double *out_T, double a, const double *x_p,
                 const double *x_T, double b, const double *y_p, const double *y_T, double c,
                 const double *z_p, const double *z_T, hipStream_t s)
{
    hipLaunchKernelGGL(k_lin3, dim3(nblk(N)), dim3(kBlock), 0, s, N, out_p, out_T, a, x_p, x_T,
                       b, y_p, y_T, c, z_p, z_T);
}

// Grid-strided over a fixed block count, so the partial sums (and the
// fixed-order reduction after them) do not depend on timing.
__global__ __launch_bounds__(kBlock) void k_dot2(long long N, const double *xp, const double *xT,
                                                 const double *yp, const double *yT,
                                                 const double *zp, const double *zT,
                                                 const double *wp, const double *wT,
                                                 double *partials)
{
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < N; t += stride) {
        v[0] += xp[t] * yp[t] + xT[t] * yT[t];
        if (zp) v[1] += zp[t] * wp[t] + zT[t] * wT[t];
    }
    block_reduce_store(v, 4, partials + 4ll * blockIdx.x);
}

int launch_dot2(long long N, const double *x_p, const double *x_T, const double *y_p,
                const double *y_T, const double *z_p, const double *z_T, const double *w_p,
                const double *w_T, double *partials, hipStream_t s)
{
    const int nb = sum2_blocks(N);
    hipLaunchKernelGGL(k_dot2, dim3(nb), dim3(kBlock), 0, s, N, x_p, x_T, y_p, y_T, z_p, z_T,
                       w_p, w_T, partials);
    return nb;
}

// Paper right-hand side (Eqs. 33-34) from the cell block:
// l1 = -BTT, l2 = -BTp, l4 = BpT / l1, l3 = -Bpp + l4 l2.
__global__ __launch_bounds__(kBlock) void k_paper_rhs(Lvl<double> L, const double *p_adv,
                                                      double p_const, const double *T_adv,
                                                      double T_const, const double *div, double dt,
                                                      double *b_p, double *b_T)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= L.N) return;
    const double p = p_adv ? p_adv[t] : p_const;
    const double T = T_adv ? T_adv[t] : T_const;
    paper_rhs_cell(cell_B(L, t), p, T, div ? div[t] : 0.0, dt, b_p[t], b_T[t]);
}

void launch_paper_rhs(const Lvl<double> &L, const double *p_adv, double p_const,
                      const double *T_adv, double T_const, const double *div, double dt,
                      double *b_p, double *b_T, hipStream_t s)
{
    hipLaunchKernelGGL(k_paper_rhs, dim3(nblk(L.N)), dim3(kBlock), 0, s, L, p_adv, p_const,
                       T_adv, T_const, div, dt, b_p, b_T);
}



// Fixed-order reduction of per-block partial sums (`width` per block).
__global__ __launch_bounds__(kBlock) void k_reduce(const double *partials, int nblocks, int width,
                                                   double *out, const int *gate)
{
    if (gated(gate)) return;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        for (int q = 0; q < width; q++) v[q] += partials[(long long)b * width + q];
    block_reduce_store(v, width, out);
}

// First stage of a two-stage fixed-order reduction: block b sums the
// partials [b*kChunk, (b+1)*kChunk) (width doubles each).
constexpr int kChunk = 1024;
__global__ __launch_bounds__(kBlock) void k_reduce_stage(const double *partials, int nblocks,
                                                         int width, double *out, const int *gate)
{
    if (gated(gate)) return;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int b0 = blockIdx.x * kChunk;
    const int b1 = min(b0 + kChunk, nblocks);
    for (int b = b0 + threadIdx.x; b < b1; b += kBlock)
        for (int q = 0; q < width; q++) v[q] += partials[(long long)b * width + q];
    block_reduce_store(v, width, out + (long long)blockIdx.x * width);
}

int reduce_scratch(int nblocks) { return nblocks > kChunk ? (nblocks + kChunk - 1) / kChunk : 0; }

// partials[0 .. 4*nblocks) -> out4; uses partials[4*nblocks ..
// 4*(nblocks + reduce_scratch(nblocks))) as scratch.
void launch_reduce4(const double *partials, int nblocks, double *out4, hipStream_t s,
                    const int *gate)
{
    const int g2 = reduce_scratch(nblocks);
    if (g2 == 0) {
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, partials, nblocks, 4, out4, gate);
        return;
    }
    double *mid = const_cast<double *>(partials) + 4ll * nblocks;
    hipLaunchKernelGGL(k_reduce_stage, dim3(g2), dim3(kBlock), 0, s, partials, nblocks, 4, mid,
                       gate);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, mid, g2, 4, out4, gate);
}

// Grid-strided over at most kSumBlocks blocks (used once per solve).
constexpr int kSumBlocks = 1024;
__global__ __launch_bounds__(kBlock) void k_sum2(long long N, const double *x, const double *y,
                                                 double *partials)
{
    double v[2] = {0.0, 0.0};
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < N; t += stride) {
        v[0] += x[t];
        v[1] += y[t];
    }
    block_reduce_store(v, 2, partials + 2ll * blockIdx.x);
}

int sum2_blocks(long long N) { return (int)std::min<long long>(nblk(N), kSumBlocks); }

void launch_sum2(long long N, const double *x, const double *y, double *partials, int nblocks,
                 double *out2, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum2, dim3(sum2_blocks(N)), dim3(kBlock), 0, s, N, x, y, partials);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, partials, nblocks, 2, out2,
                       (const int *)nullptr);
}

__global__ __launch_bounds__(kBlock) void k_shift2(long long N, double *x, double *y,
                                                   const double *sum2, double scale)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= N) return;
    x[t] -= scale * sum2[0];
    y[t] -= scale * sum2[1];
}

void launch_shift2(long long N, double *x, double *y, const double *sum2, double scale,
                   hipStream_t s)
{
    hipLaunchKernelGGL(k_shift2, dim3(nblk(N)), dim3(kBlock), 0, s, N, x, y, sum2, scale);
}

// ------------------------------------------------------------ smoother
// One colour of a red-black 2x2-block Gauss-Seidel sweep: each cell of
// colour (i+j+k) mod 2 == color solves
//   (B + diag(S_p, S_T)) u = f + sum_faces w u_nbr
// by Cramer's rule.  zero_guess: the neighbours are taken as zero (first
// red pass from a zero initial guess; the stale values are never read).
// The block Gauss-Seidel update of one cell (shared by the grid kernels
// and the single-block tail cycle, whose arrays live in LDS).
template <typename R, int DIM, bool CF, bool USE_U>
__device__ __forceinline__ void rb_cell(const Lvl<R> &L, int i, int j, int k, long long me,
                                        bool old_zero = false)
{
    using V2 = typename VT<R>::v2;
    using V4 = typename VT<R>::v4;
    R nbp, nbT, Sp, ST;
    gather<R, DIM, CF, USE_U>(L, i, j, k, me, nbp, nbT, Sp, ST);
    const V2 f = L.f[me];
    const V4 b = sweep_B(L, me);
    const R gp = f.x + nbp, gT = f.y + nbT;
    const R a = b.x + Sp, d = b.w + ST;
    const R inv = quot(R(1), a * d - b.y * b.z);
    V2 o;
    o.x = (d * gp - b.y * gT) * inv;
    o.y = (a * gT - b.z * gp) * inv;
    if (L.omega != R(1)) {
        V2 old;
        old.x = old.y = R(0);
        if (USE_U && !old_zero) old = L.u[me];
        o = relax(L.omega, o, old);
    }
    L.u[me] = o;
}

// Residual f - A u at one cell.
template <typename R, int DIM, bool CF>
__device__ __forceinline__ typename VT<R>::v2 residual_cell(const Lvl<R> &F, int i, int j, int k,
                                                            long long me)
{
    using V2 = typename VT<R>::v2;
    using V4 = typename VT<R>::v4;
    R nbp, nbT, Sp, ST;
    gather<R, DIM, CF, true>(F, i, j, k, me, nbp, nbT, Sp, ST);
    const V2 u = F.u[me];
    const V2 f = F.f[me];
    const V4 b = sweep_B(F, me);
    const R Ap = Sp * u.x - nbp + b.x * u.x + b.y * u.y;
    const R AT = ST * u.y - nbT + b.z * u.x + b.w * u.y;
    V2 r;
    r.x = f.x - Ap;
    r.y = f.y - AT;
    return r;
}

// Coarse right-hand side at coarse cell (I, J, K): mean over the children.
template <typename R, int DIM, bool CF>
__device__ __forceinline__ void restrict_cell(const Lvl<R> &F, const Lvl<R> &C, int I, int J, int K,
                                              long long t)
{
    using V2 = typename VT<R>::v2;
    R sp = R(0), sT = R(0);
#pragma unroll
    for (int m = 0; m < (1 << DIM); m++) {
        const int i = 2 * I + (m & 1), j = 2 * J + ((m >> 1) & 1);
        const int k = DIM == 3 ? 2 * K + ((m >> 2) & 1) : 0;
        const long long me = i + (long long)F.nx * (j + (long long)F.ny * k);
        const V2 r = residual_cell<R, DIM, CF>(F, i, j, k, me);
        sp += r.x;
        sT += r.y;
    }
    const R sc = R(1) / R(1 << DIM);
    V2 o;
    o.x = sp * sc;
    o.y = sT * sc;
    C.f[t] = o;
}

// P e at fine cell (i, j, k): along each axis weight 3/4 on the parent and
// 1/4 on the parent's neighbour on the fine cell's side (the parent at a
// boundary).
template <typename R, int DIM, typename Get>
__device__ __forceinline__ void prolong_delta_from(int i, int j, int k, int cnx, int cny, int cnz,
                                                   const Get &get, R &vp, R &vT)
{
    using V2 = typename VT<R>::v2;
    int par[3] = {i >> 1, j >> 1, DIM == 3 ? k >> 1 : 0};
    int nbr[3];
    const int fi[3] = {i, j, k};
    const int cn[3] = {cnx, cny, cnz};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (a >= DIM) {
            nbr[a] = par[a];
            continue;
        }
        int q = par[a] + ((fi[a] & 1) ? 1 : -1);
        nbr[a] = (q < 0 || q >= cn[a]) ? par[a] : q;
    }
    vp = vT = R(0);
#pragma unroll
    for (int m = 0; m < (1 << DIM); m++) {
        R w = R(1);
        int c[3] = {par[0], par[1], par[2]};
#pragma unroll
        for (int a = 0; a < DIM; a++) {
            if ((m >> a) & 1) {
                c[a] = nbr[a];
                w *= R(0.25);
            } else {
                w *= R(0.75);
            }
        }
        const V2 e = get(c[0], c[1], c[2]);
        vp += w * e.x;
        vT += w * e.y;
    }
}

template <typename R, int DIM>
__device__ __forceinline__ void prolong_delta(const Lvl<R> &C, int i, int j, int k, R &vp, R &vT)
{
    auto get = [&](int a, int b, int c) {
        return C.u[a + (long long)C.nx * (b + (long long)C.ny * c)];
    };
    prolong_delta_from<R, DIM>(i, j, k, C.nx, C.ny, C.nz, get, vp, vT);
}

// u += P e at fine cell (i, j, k).
template <typename R, int DIM>
__device__ __forceinline__ void prolong_cell(const Lvl<R> &F, const Lvl<R> &C, int i, int j, int k,
                                             long long t)
{
    using V2 = typename VT<R>::v2;
    R vp, vT;
    prolong_delta<R, DIM>(C, i, j, k, vp, vT);
    V2 u = F.u[t];
    u.x += vp;
    u.y += vT;
    F.u[t] = u;
}

// One colour of a red-black 2x2-block Gauss-Seidel sweep: each cell of
// colour (i+j+k) mod 2 == color solves
//   (B + diag(S_p, S_T)) u = f + sum_faces w u_nbr
// by Cramer's rule.  zero_guess: the neighbours are taken as zero (first
// red pass from a zero initial guess; the stale values are never read).
template <typename R, int DIM, bool CF>
__global__ __launch_bounds__(kBlock) void k_rb_pass(Lvl<R> L, int color, int zero_guess)
{
    if (gated(L.gate)) return;
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    const int nxh = (L.nx + 1) >> 1;
    const long long tot = (long long)nxh * L.ny * L.nz;
    if (t >= tot) return;
    int ti, j, k;
    decode(t, nxh, L.ny, ti, j, k);
    const int i = 2 * ti + ((j + k + color) & 1);
    if (i >= L.nx) return;
    const long long me = i + (long long)L.nx * (j + (long long)L.ny * k);
    // zero_guess 1: the iterate is zero (first colour of a sweep from a zero
    // guess); 2: the other colour's new values are read, the cell's own old
    // value is zero (second colour of that sweep)
    if (zero_guess == 1) rb_cell<R, DIM, CF, false>(L, i, j, k, me);
    else rb_cell<R, DIM, CF, true>(L, i, j, k, me, zero_guess == 2);
}

template <typename R>
void launch_rb_pass(int dim, int level0, const Lvl<R> &L, int color, int zero_guess,
                    hipStream_t s)
{
    const long long tot = (long long)((L.nx + 1) >> 1) * L.ny * L.nz;
    dim3 g(nblk(tot)), b(kBlock);
    if (dim == 3) {
        if (level0) hipLaunchKernelGGL((k_rb_pass<R, 3, true>), g, b, 0, s, L, color, zero_guess);
        else hipLaunchKernelGGL((k_rb_pass<R, 3, false>), g, b, 0, s, L, color, zero_guess);
    } else {
        if (level0) hipLaunchKernelGGL((k_rb_pass<R, 2, true>), g, b, 0, s, L, color, zero_guess);
        else hipLaunchKernelGGL((k_rb_pass<R, 2, false>), g, b, 0, s, L, color, zero_guess);
    }
}
template void launch_rb_pass<float>(int, int, const Lvl<float> &, int, int, hipStream_t);
template void launch_rb_pass<double>(int, int, const Lvl<double> &, int, int, hipStream_t);

// ------------------------------------------------ residual + restriction
// Coarse right-hand side = mean over the 2^DIM children of f - A u.
template <typename R, int DIM, bool CF>
__global__ __launch_bounds__(kBlock) void k_restrict(Lvl<R> F, Lvl<R> C)
{
    if (gated(F.gate)) return;
    // neighbouring coarse cells share the fine halo: runs of them per XCD
    long long t = (long long)xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (t >= C.N) return;
    int I, J, K;
    decode(t, C.nx, C.ny, I, J, K);
    restrict_cell<R, DIM, CF>(F, C, I, J, K, t);
}

template <typename R>
void launch_restrict(int dim, int level0, const Lvl<R> &F, const Lvl<R> &C, hipStream_t s)
{
    dim3 g(nblk(C.N)), b(kBlock);
    if (dim == 3) {
        if (level0) hipLaunchKernelGGL((k_restrict<R, 3, true>), g, b, 0, s, F, C);
        else hipLaunchKernelGGL((k_restrict<R, 3, false>), g, b, 0, s, F, C);
    } else {
        if (level0) hipLaunchKernelGGL((k_restrict<R, 2, true>), g, b, 0, s, F, C);
        else hipLaunchKernelGGL((k_restrict<R, 2, false>), g, b, 0, s, F, C);
    }
}
template void launch_restrict<float>(int, int, const Lvl<float> &, const Lvl<float> &, hipStream_t);
template void launch_restrict<double>(int, int, const Lvl<double> &, const Lvl<double> &,
                                      hipStream_t);

// ------------------------------------------- prolongation + correction
template <typename R, int DIM>
__global__ __launch_bounds__(kBlock) void k_prolong(Lvl<R> F, Lvl<R> C)
{
    if (gated(F.gate)) return;
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= F.N) return;
    int i, j, k;
    decode(t, F.nx, F.ny, i, j, k);
    prolong_cell<R, DIM>(F, C, i, j, k, t);
}

// 3-D: a 32 x 8 x 8 fine tile per block, its coarse parents and their
// neighbours (18 x 6 x 6) staged in LDS once instead of eight global reads
// per fine cell; the arithmetic of prolong_cell.
template <typename R>
__global__ __launch_bounds__(1024) void k_prolong3t(Lvl<R> F, Lvl<R> C, int tiles_x, int tiles_y)
{
    if (gated(F.gate)) return;
    using V2 = typename VT<R>::v2;
    // a 32 x 8 x 8 fine tile: each thread adds the correction to the cells
    // of planes k and k + 4, whose values are loaded with the coarse
    // tile's, before the barrier
    constexpr int TX = 32, TY = 8, TZ = 8, ZH = TZ / 2;
    constexpr int CX = TX / 2 + 2, CY = TY / 2 + 2, CZ = TZ / 2 + 2;
    static_assert(CX * CY * CZ <= 1024, "one coarse cell per thread");
    __shared__ V2 sc[CX * CY * CZ];
    const int b = blockIdx.x;
    const int x0 = (b % tiles_x) * TX, y0 = ((b / tiles_x) % tiles_y) * TY;
    const int z0 = (b / tiles_x / tiles_y) * TZ;
    const int cx0 = x0 / 2 - 1, cy0 = y0 / 2 - 1, cz0 = z0 / 2 - 1;
    const int t = threadIdx.x;
    const int i = x0 + t % TX, j = y0 + (t / TX) % TY, k = z0 + t / (TX * TY);
    const bool in = i < F.nx && j < F.ny;
    const long long g = i + (long long)F.nx * (j + (long long)F.ny * k);
    const long long gh = g + (long long)F.nx * F.ny * ZH;
    V2 u0, u1;
    if (in && k < F.nz) u0 = F.u[g];
    if (in && k + ZH < F.nz) u1 = F.u[gh];
    if (t < CX * CY * CZ) {
        const int ci = cx0 + t % CX, cj = cy0 + (t / CX) % CY, ck = cz0 + t / (CX * CY);
        V2 v;
        v.x = v.y = R(0);
        if (ci >= 0 && ci < C.nx && cj >= 0 && cj < C.ny && ck >= 0 && ck < C.nz)
            v = C.u[ci + (long long)C.nx * (cj + (long long)C.ny * ck)];
        sc[t] = v;
    }
    __syncthreads();
    if (!in) return;
    auto get = [&](int a, int bb, int c) {
        return sc[(a - cx0) + CX * ((bb - cy0) + CY * (c - cz0))];
    };
    R vp, vT;
    if (k < F.nz) {
        prolong_delta_from<R, 3>(i, j, k, C.nx, C.ny, C.nz, get, vp, vT);
        u0.x += vp;
        u0.y += vT;
        F.u[g] = u0;
    }
    if (k + ZH < F.nz) {
        prolong_delta_from<R, 3>(i, j, k + ZH, C.nx, C.ny, C.nz, get, vp, vT);
        u1.x += vp;
        u1.y += vT;
        F.u[gh] = u1;
    }
}

template <typename R>
void launch_prolong(int dim, const Lvl<R> &F, const Lvl<R> &C, hipStream_t s)
{
    dim3 g(nblk(F.N)), b(kBlock);
    if (dim == 3) {
        const int tx = (F.nx + 31) / 32, ty = (F.ny + 7) / 8, tz = (F.nz + 7) / 8;
        hipLaunchKernelGGL((k_prolong3t<R>), dim3(tx * ty * tz), dim3(1024), 0, s, F, C, tx, ty);
        return;
    }
    hipLaunchKernelGGL((k_prolong<R, 2>), g, b, 0, s, F, C);
}
template void launch_prolong<float>(int, const Lvl<float> &, const Lvl<float> &, hipStream_t);
template void launch_prolong<double>(int, const Lvl<double> &, const Lvl<double> &, hipStream_t);

// ------------------------------------------------------ coarse operator
// Coarse face coefficient = mean of the 2^(DIM-1) fine faces that make up
// the coarse face; coarse block = mean of the 2^DIM children's blocks.
// Coarse cell t of a cnx x cny x cnz level from the fine level F.
template <typename RIN, typename ROUT, int DIM, bool CF>
__device__ __forceinline__ void coarsen_cell(const Lvl<RIN> &F, int cnx, int cny, int cnz,
                                             typename VT<ROUT>::v2 *fx,
                                             typename VT<ROUT>::v2 *fy,
                                             typename VT<ROUT>::v2 *fz,
                                             typename VT<ROUT>::v4 *Bo, long long t)
{
    using V2 = typename VT<RIN>::v2;
    using V4 = typename VT<RIN>::v4;
    using O2 = typename VT<ROUT>::v2;
    using O4 = typename VT<ROUT>::v4;
    int I, J, K;
    decode(t, cnx, cny, I, J, K);
    const int base[3] = {2 * I, 2 * J, DIM == 3 ? 2 * K : 0};
    const int Ci[3] = {I, J, K};
    const long long st[3] = {1, F.nx, (long long)F.nx * F.ny};
    double b4[4] = {0, 0, 0, 0};
    double fs[3][2] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll
    for (int m = 0; m < (1 << DIM); m++) {
        const int c[3] = {base[0] + (m & 1), base[1] + ((m >> 1) & 1),
                          DIM == 3 ? base[2] + ((m >> 2) & 1) : 0};
        const long long me = c[0] + (long long)F.nx * (c[1] + (long long)F.ny * c[2]);
        const V4 b = cell_B(F, me);
        if (CF && F.axm) {
            // r-z: level 1 holds the volume-weighted equations (blocks
            // times the cell radius, faces times the face area below)
            const double rc = (double)F.axm[c[1]].z;
            b4[0] += (double)b.x * rc;
            b4[1] += (double)b.y * rc;
            b4[2] += (double)b.z * rc;
            b4[3] += (double)b.w * rc;
        } else {
            b4[0] += (double)b.x;
            b4[1] += (double)b.y;
            b4[2] += (double)b.z;
            b4[3] += (double)b.w;
        }
#pragma unroll
        for (int a = 0; a < DIM; a++) {
            if (c[a] != base[a] || Ci[a] == 0) continue;
            V2 w;
            if (CF) {
                w = harm2(cell_ac(F, me), cell_ac(F, me - st[a]));
                if (F.axm) {
                    // axial faces: area ~ cell radius; radial: face radius
                    const auto ar = a == 0 ? F.axm[c[1]].z : F.axm[c[1]].w;
                    w.x *= ar;
                    w.y *= ar;
                }
            } else {
                const V2 *Fa = a == 0 ? F.fx : (a == 1 ? F.fy : F.fz);
                w = Fa[me];
            }
            fs[a][0] += (double)w.x;
            fs[a][1] += (double)w.y;
        }
    }
    const double inv_nc = 1.0 / (1 << DIM), inv_nf = 1.0 / (1 << (DIM - 1));
    O4 ob;
    ob.x = (ROUT)(b4[0] * inv_nc);
    ob.y = (ROUT)(b4[1] * inv_nc);
    ob.z = (ROUT)(b4[2] * inv_nc);
    ob.w = (ROUT)(b4[3] * inv_nc);
    Bo[t] = ob;
    O2 o;
    o.x = (ROUT)(fs[0][0] * inv_nf);
    o.y = (ROUT)(fs[0][1] * inv_nf);
    fx[t] = o;
    o.x = (ROUT)(fs[1][0] * inv_nf);
    o.y = (ROUT)(fs[1][1] * inv_nf);
    fy[t] = o;
    if (DIM == 3) {
        o.x = (ROUT)(fs[2][0] * inv_nf);
        o.y = (ROUT)(fs[2][1] * inv_nf);
        fz[t] = o;
    }
}

template <typename RIN, typename ROUT, int DIM, bool CF>
__global__ __launch_bounds__(kBlock) void k_coarsen(Lvl<RIN> F, int cnx, int cny, int cnz,
                                                    typename VT<ROUT>::v2 *fx,
                                                    typename VT<ROUT>::v2 *fy,
                                                    typename VT<ROUT>::v2 *fz,
                                                    typename VT<ROUT>::v4 *Bo)
{
    // the lower faces read the neighbours' children: runs of coarse cells
    // per XCD, so that those reads hit its L2
    long long t = (long long)xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const long long CN = (long long)cnx * cny * cnz;
    if (t >= CN) return;
    coarsen_cell<RIN, ROUT, DIM, CF>(F, cnx, cny, cnz, fx, fy, fz, Bo, t);
}

// Level 1 from a 3-D finest level (cell coefficients), plane-marching: a
// block takes a 64 x 4 tile of fine cells (32 x 2 coarse cells) down a
// chunk of plane pairs, one coarse plane per step, with the next pair's
// loads in flight while a pair computes.  Each thread forms its two fine
// cells' blocks and the lower faces on which a cell is a lower child (the
// harmonic mean with the neighbour below along that axis: in-plane from
// the pair's coefficients staged in LDS with a lower halo, along z from
// the cell below); the coarse cells' threads then sum their eight
// children in the order of coarsen_cell (the block over all eight, each
// face over the children on it), so the result is k_coarsen's bit for bit.
template <typename RIN, typename ROUT>
__global__ __launch_bounds__(256) void k_coarsen0_zm(Lvl<RIN> F, int zc, int tiles_x, int tiles_y,
                                                     int ntiles, typename VT<ROUT>::v2 *fx,
                                                     typename VT<ROUT>::v2 *fy,
                                                     typename VT<ROUT>::v2 *fz,
                                                     typename VT<ROUT>::v4 *Bo)
{
    using V2 = typename VT<RIN>::v2;
    using V4 = typename VT<RIN>::v4;
    using O2 = typename VT<ROUT>::v2;
    using O4 = typename VT<ROUT>::v4;
    constexpr int TX = 64, TY = 4, NT = TX * TY;
    constexpr int PX = TX + 1, PY = TY + 1, PS = PX * PY;   // the tile and its lower halo
    constexpr int NLD = (PS + NT - 1) / NT;
    constexpr int CX = TX / 2, CY = TY / 2;
    __shared__ V2 sac[2][PS];
    __shared__ V4 sB[2][NT];
    __shared__ V2 sf[2][3][NT];   // [plane of the pair][axis][cell]
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int t = threadIdx.x;
    const int txi = tile % tiles_x;
    const int rr = tile / tiles_x;
    const int x0 = txi * TX, y0 = (rr % tiles_y) * TY;
    const int z0 = (rr / tiles_y) * zc, z1 = min(z0 + zc, F.nz);   // z0, z1 even
    const long long nxy = (long long)F.nx * F.ny;
    const int lx = t % TX, ly = t / TX;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool mine = gx < F.nx && gy < F.ny;
    const long long g0 = gx + (long long)F.nx * gy;
    const int cnx = F.nx / 2, cny = F.ny / 2;
    const int cxl = t % CX, cyl = t / CX;
    const int gcx = x0 / 2 + cxl, gcy = y0 / 2 + cyl;
    const bool cmine = t < CX * CY && gcx < cnx && gcy < cny;
    V2 zero;
    zero.x = zero.y = RIN(0);
    // the loads of a pair (planes z, z+1), raw in registers
    V2 pa[2][NLD];
    V4 pb[2];
    auto load = [&](int z) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
#pragma unroll
            for (int i = 0; i < NLD; i++) {
                const int c = t + i * NT;
                const int hx = x0 - 1 + c % PX, hy = y0 - 1 + c / PX;
                pa[h][i] = zero;
                if (c < PS && hx >= 0 && hx < F.nx && hy >= 0 && hy < F.ny)
                    pa[h][i] = cell_ac(F, hx + (long long)F.nx * hy + nxy * (z + h));
            }
            if (mine) pb[h] = cell_B_raw(F, g0 + nxy * (z + h));
        }
    };
    V2 below = zero;   // coefficients of this thread's cell on the plane below the pair
    if (mine && z0 > 0) below = cell_ac(F, g0 + nxy * (z0 - 1));
    if (z0 < z1) load(z0);
    for (int z = z0; z < z1; z += 2) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
#pragma unroll
            for (int i = 0; i < NLD; i++) {
                const int c = t + i * NT;
                if (c < PS) sac[h][c] = pa[h][i];
            }
        }
        V4 bown[2];
        bown[0] = pb[0];
        bown[1] = pb[1];
        __syncthreads();
        if (z + 2 < z1) load(z + 2);
        if (mine) {
            const int c = (ly + 1) * PX + lx + 1;
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const V2 am = sac[h][c];
                V2 wx = zero, wy = zero, wz = zero;
                if ((gx & 1) == 0 && gx > 0) wx = harm2(am, sac[h][c - 1]);
                if ((gy & 1) == 0 && gy > 0) wy = harm2(am, sac[h][c - PX]);
                if (h == 0 && z > 0) wz = harm2(am, below);
                sB[h][t] = cell_B_fin(F, bown[h]);
                sf[h][0][t] = wx;
                sf[h][1][t] = wy;
                sf[h][2][t] = wz;
                if (h == 1) below = am;
            }
        }
        __syncthreads();
        if (cmine) {
            // children m = 4 h + 2 b + a: x, then y, then z order
            double b4[4] = {0, 0, 0, 0};
            double fs[3][2] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll
            for (int h = 0; h < 2; h++) {
#pragma unroll
                for (int b = 0; b < 2; b++) {
#pragma unroll
                    for (int a = 0; a < 2; a++) {
                        const int q = (2 * cyl + b) * TX + 2 * cxl + a;
                        const V4 bq = sB[h][q];
                        b4[0] += (double)bq.x;
                        b4[1] += (double)bq.y;
                        b4[2] += (double)bq.z;
                        b4[3] += (double)bq.w;
                        if (a == 0 && gcx > 0) {
                            fs[0][0] += (double)sf[h][0][q].x;
                            fs[0][1] += (double)sf[h][0][q].y;
                        }
                        if (b == 0 && gcy > 0) {
                            fs[1][0] += (double)sf[h][1][q].x;
                            fs[1][1] += (double)sf[h][1][q].y;
                        }
                        if (h == 0 && z > 0) {
                            fs[2][0] += (double)sf[h][2][q].x;
                            fs[2][1] += (double)sf[h][2][q].y;
                        }
                    }
                }
            }
            const long long o = gcx + (long long)cnx * gcy + (long long)cnx * cny * (z >> 1);
            const double inv_nc = 1.0 / 8, inv_nf = 1.0 / 4;
            O4 ob;
            ob.x = (ROUT)(b4[0] * inv_nc);
            ob.y = (ROUT)(b4[1] * inv_nc);
            ob.z = (ROUT)(b4[2] * inv_nc);
            ob.w = (ROUT)(b4[3] * inv_nc);
            Bo[o] = ob;
            O2 w;
            w.x = (ROUT)(fs[0][0] * inv_nf);
            w.y = (ROUT)(fs[0][1] * inv_nf);
            fx[o] = w;
            w.x = (ROUT)(fs[1][0] * inv_nf);
            w.y = (ROUT)(fs[1][1] * inv_nf);
            fy[o] = w;
            w.x = (ROUT)(fs[2][0] * inv_nf);
            w.y = (ROUT)(fs[2][1] * inv_nf);
            fz[o] = w;
        }
    }
}

template <typename RIN, typename ROUT>
void launch_coarsen(int dim, int level0, const Lvl<RIN> &F, typename VT<ROUT>::v2 *fx,
                    typename VT<ROUT>::v2 *fy, typename VT<ROUT>::v2 *fz,
                    typename VT<ROUT>::v4 *B, hipStream_t s, bool zm)
{
    const int cnx = F.nx / 2, cny = F.ny / 2, cnz = dim == 3 ? F.nz / 2 : 1;
    dim3 g(nblk((long long)cnx * cny * cnz)), b(kBlock);
    if (dim == 3 && level0 && zm && !F.axm) {
        const int tx = (F.nx + 63) / 64, ty = (F.ny + 3) / 4;
        int zc = F.nz;   // even (the grid coarsens), kept even below
        while (zc > 8 && (long long)tx * ty * ((F.nz + zc - 1) / zc) < 2048) zc = ((zc + 1) / 2 + 1) & ~1;
        const int nt = tx * ty * ((F.nz + zc - 1) / zc);
        hipLaunchKernelGGL((k_coarsen0_zm<RIN, ROUT>), dim3(nt), dim3(256), 0, s, F, zc, tx, ty, nt,
                           fx, fy, fz, B);
        return;
    }
    if (dim == 3) {
        if (level0)
            hipLaunchKernelGGL((k_coarsen<RIN, ROUT, 3, true>), g, b, 0, s, F, cnx, cny, cnz, fx,
                               fy, fz, B);
        else
            hipLaunchKernelGGL((k_coarsen<RIN, ROUT, 3, false>), g, b, 0, s, F, cnx, cny, cnz,
                               fx, fy, fz, B);
    } else {
        if (level0)
            hipLaunchKernelGGL((k_coarsen<RIN, ROUT, 2, true>), g, b, 0, s, F, cnx, cny, cnz, fx,
                               fy, fz, B);
        else
            hipLaunchKernelGGL((k_coarsen<RIN, ROUT, 2, false>), g, b, 0, s, F, cnx, cny, cnz,
                               fx, fy, fz, B);
    }
}
template void launch_coarsen<double, double>(int, int, const Lvl<double> &, double2 *, double2 *,
                                             double2 *, double4 *, hipStream_t, bool);
template void launch_coarsen<double, float>(int, int, const Lvl<double> &, float2 *, float2 *,
                                            float2 *, float4 *, hipStream_t, bool);
template void launch_coarsen<float, float>(int, int, const Lvl<float> &, float2 *, float2 *,
                                           float2 *, float4 *, hipStream_t, bool);

// ------------------------------------------------ coarsest-grid matrix
// Dense FP64 matrix of the level operator, unknown (2*cell + component).
// pin_mean: adds s_c = (diagonal of cell 0, component c) / N to every
// entry of each component block.  For a consistent pure-Neumann system
// (A 1 = 0, 1^T f = 0) the solution of (A + s 1 1^T) x = f is the
// zero-mean solution of A x = f, and A + s 1 1^T stays positive definite.
template <typename R, int DIM, bool CF>
__device__ double dense_row_diag(const Lvl<R> &L, long long cell, int c, double *row)
{
    using V2 = typename VT<R>::v2;
    int i, j, k;
    decode(cell, L.nx, L.ny, i, j, k);
    V2 am;
    if (CF) am = cell_ac(L, cell);
    const long long st[3] = {1, L.nx, (long long)L.nx * L.ny};
    const int ii[3] = {i, j, k};
    const int nn[3] = {L.nx, L.ny, L.nz};
    double S = 0.0;
    for (int a = 0; a < DIM; a++) {
        for (int up = 0; up < 2; up++) {
            if (up == 0 && ii[a] == 0) continue;
            if (up == 1 && ii[a] == nn[a] - 1) continue;
            const long long q = up ? cell + st[a] : cell - st[a];
            V2 w = face_coef<R, CF>(L, am, cell, q, a, up == 1);
            if (CF && a == 1 && L.axm) axi_face(w, L.axm[j], up == 1);
            double wc = (double)(c == 0 ? w.x : w.y) * L.inv_h2;
            S += wc;
            if (row) row[2 * q + c] -= wc;
        }
    }
    const typename VT<R>::v4 b = cell_B(L, cell);
    return S + (double)(c == 0 ? b.x : b.w);
}

// Row r of the dense matrix.
template <typename R, int DIM, bool CF>
__device__ __forceinline__ void dense_row(const Lvl<R> &L, int pin_mean, double *M, long long r)
{
    using V4 = typename VT<R>::v4;
    const long long m = 2 * L.N;
    const long long cell = r >> 1;
    const int c = (int)(r & 1);
    double *row = M + r * m;
    for (long long q = 0; q < m; q++) row[q] = 0.0;
    const double D = dense_row_diag<R, DIM, CF>(L, cell, c, row);
    const V4 b = cell_B(L, cell);
    row[r] += D;
    row[2 * cell + (1 - c)] += (double)(c == 0 ? b.y : b.z);
    if (pin_mean) {
        double d0 = dense_row_diag<R, DIM, CF>(L, 0, c, nullptr);
        if (!(d0 > 0.0)) d0 = L.inv_h2;
        const double sh = d0 / (double)L.N;
        for (long long q = 0; q < L.N; q++) row[2 * q + c] += sh;
    }
}

template <typename R, int DIM, bool CF>
__global__ __launch_bounds__(kBlock) void k_coarse_dense(Lvl<R> L, int pin_mean, double *M)
{
    long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (r >= 2 * L.N) return;
    dense_row<R, DIM, CF>(L, pin_mean, M, r);
}

template <typename R>
void launch_coarse_dense(int dim, int level0, const Lvl<R> &L, int pin_mean, double *M,
                         hipStream_t s)
{
    dim3 g(nblk(2 * L.N)), b(kBlock);
    if (dim == 3) {
        if (level0) hipLaunchKernelGGL((k_coarse_dense<R, 3, true>), g, b, 0, s, L, pin_mean, M);
        else hipLaunchKernelGGL((k_coarse_dense<R, 3, false>), g, b, 0, s, L, pin_mean, M);
    } else {
        if (level0) hipLaunchKernelGGL((k_coarse_dense<R, 2, true>), g, b, 0, s, L, pin_mean, M);
        else hipLaunchKernelGGL((k_coarse_dense<R, 2, false>), g, b, 0, s, L, pin_mean, M);
    }
}
template void launch_coarse_dense<float>(int, int, const Lvl<float> &, int, double *, hipStream_t);
template void launch_coarse_dense<double>(int, int, const Lvl<double> &, int, double *,
                                          hipStream_t);

// One Gauss-Jordan elimination step without pivoting (out of place):
// pivot p = A[k][k], q = 1/p; A'[k][k] = q; A'[k][j] = A[k][j] q;
// A'[i][k] = -A[i][k] q; A'[i][j] = A[i][j] - A[i][k] (A[k][j] q).
// After m steps the matrix holds its inverse.  Pivots of the coarse
// operator are positive (positive diagonals and det of every 2x2 block,
// block-diagonally dominant rows); a pivot that is not is flagged.
__global__ __launch_bounds__(kBlock) void k_gj_step(const double *A, double *Bm, int m, int k,
                                                    int *flags)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long long)m * m) return;
    const int i = (int)(t / m), j = (int)(t % m);
    const double p = A[(long long)k * m + k];
    const double q = 1.0 / p;
    double v;
    if (i == k && j == k) {
        v = q;
        if (!(p > 0.0) || !isfinite(p)) atomicOr(&flags[FLAG_PIVOT], 1);
    } else if (i == k) {
        v = A[(long long)k * m + j] * q;
    } else if (j == k) {
        v = -A[(long long)i * m + k] * q;
    } else {
        v = A[t] - A[(long long)i * m + k] * (A[(long long)k * m + j] * q);
    }
    Bm[t] = v;
}

void launch_gj_step(const double *A, double *Bm, int m, int k, int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_gj_step, dim3(nblk((long long)m * m)), dim3(kBlock), 0, s, A, Bm, m, k,
                       flags);
}

// u = Ainv f on the coarsest grid, FP64 accumulation; one wave per row.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_coarse_apply(const double *Ainv, int m, const R *f,
                                                         R *u, const int *gate)
{
    if (gated(gate)) return;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= m) return;
    const double *a = Ainv + (long long)row * m;
    double s = 0.0;
    for (int c = lane; c < m; c += 64) s += a[c] * (double)f[c];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) u[row] = (R)s;
}

template <typename R>
void launch_coarse_apply(const double *Ainv, int m, const R *f, R *u, hipStream_t s,
                         const int *gate)
{
    const int rows_per_block = kBlock / 64;
    hipLaunchKernelGGL((k_coarse_apply<R>), dim3((m + rows_per_block - 1) / rows_per_block),
                       dim3(kBlock), 0, s, Ainv, m, f, u, gate);
}
template void launch_coarse_apply<float>(const double *, int, const float *, float *, hipStream_t,
                                         const int *);
template void launch_coarse_apply<double>(const double *, int, const double *, double *,
                                          hipStream_t, const int *);

// ------------------------------------------------------ export / convert
template <typename R, int DIM, bool CF>
__global__ __launch_bounds__(kBlock) void k_export_op(Lvl<R> L, double *faces, double *Bout)
{
    using V2 = typename VT<R>::v2;
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= L.N) return;
    int i, j, k;
    decode(t, L.nx, L.ny, i, j, k);
    const int ii[3] = {i, j, k};
    const long long st[3] = {1, L.nx, (long long)L.nx * L.ny};
    V2 am;
    if (CF) am = cell_ac(L, t);
    for (int a = 0; a < 3; a++) {
        double wp = 0.0, wT = 0.0;
        if (a < DIM && ii[a] > 0) {
            V2 w = face_coef<R, CF>(L, am, t, t - st[a], a, false);
            wp = (double)w.x;
            wT = (double)w.y;
        }
        faces[(0 * 3 + a) * L.N + t] = wp;
        faces[(1 * 3 + a) * L.N + t] = wT;
    }
    const typename VT<R>::v4 b = cell_B(L, t);
    Bout[t] = (double)b.x;
    Bout[L.N + t] = (double)b.y;
    Bout[2 * L.N + t] = (double)b.z;
    Bout[3 * L.N + t] = (double)b.w;
}

template <typename R>
void launch_export_op(int dim, int level0, const Lvl<R> &L, double *faces, double *B,
                      hipStream_t s)
{
    dim3 g(nblk(L.N)), b(kBlock);
    if (dim == 3) {
        if (level0) hipLaunchKernelGGL((k_export_op<R, 3, true>), g, b, 0, s, L, faces, B);
        else hipLaunchKernelGGL((k_export_op<R, 3, false>), g, b, 0, s, L, faces, B);
    } else {
        if (level0) hipLaunchKernelGGL((k_export_op<R, 2, true>), g, b, 0, s, L, faces, B);
        else hipLaunchKernelGGL((k_export_op<R, 2, false>), g, b, 0, s, L, faces, B);
    }
}
template void launch_export_op<float>(int, int, const Lvl<float> &, double *, double *, hipStream_t);
template void launch_export_op<double>(int, int, const Lvl<double> &, double *, double *,
                                       hipStream_t);

template <typename R>
__global__ __launch_bounds__(kBlock) void k_pack(long long N, const double *p, const double *T,
                                                 typename VT<R>::v2 *out)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= N) return;
    typename VT<R>::v2 o;
    o.x = (R)p[t];
    o.y = (R)T[t];
    out[t] = o;
}

template <typename R>
void launch_pack(long long N, const double *p, const double *T, typename VT<R>::v2 *out,
                 hipStream_t s)
{
    hipLaunchKernelGGL((k_pack<R>), dim3(nblk(N)), dim3(kBlock), 0, s, N, p, T, out);
}
template void launch_pack<float>(long long, const double *, const double *, float2 *, hipStream_t);
template void launch_pack<double>(long long, const double *, const double *, double2 *,
                                  hipStream_t);

template <typename R>
__global__ __launch_bounds__(kBlock) void k_unpack(long long N, const typename VT<R>::v2 *in,
                                                   double *p, double *T)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= N) return;
    typename VT<R>::v2 v = in[t];
    p[t] = (double)v.x;
    T[t] = (double)v.y;
}

template <typename R>
void launch_unpack(long long N, const typename VT<R>::v2 *in, double *p, double *T, hipStream_t s)
{
    hipLaunchKernelGGL((k_unpack<R>), dim3(nblk(N)), dim3(kBlock), 0, s, N, in, p, T);
}
template void launch_unpack<float>(long long, const float2 *, double *, double *, hipStream_t);
template void launch_unpack<double>(long long, const double2 *, double *, double *, hipStream_t);

template <typename RIN, typename ROUT>
__global__ __launch_bounds__(kBlock) void k_convert(long long n, const RIN *in, ROUT *out)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) out[t] = (ROUT)in[t];
}

template <typename RIN, typename ROUT>
void launch_convert(long long n, const RIN *in, ROUT *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_convert<RIN, ROUT>), dim3(nblk(n)), dim3(kBlock), 0, s, n, in, out);
}
template void launch_convert<double, double>(long long, const double *, double *, hipStream_t);
template void launch_convert<double, float>(long long, const double *, float *, hipStream_t);
template void launch_convert<float, double>(long long, const float *, double *, hipStream_t);

// Plain copy (16-byte vectors, then a byte tail): bandwidth calibration.
__global__ __launch_bounds__(kBlock) void k_copy(uint4 *dst, const uint4 *src, long long nvec,
                                                 unsigned char *dtail, const unsigned char *stail,
                                                 int ntail)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long q = t; q < nvec; q += stride) dst[q] = src[q];
    if (t < ntail) dtail[t] = stail[t];
}

void launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const long long nvec = (long long)(bytes / 16);
    const int ntail = (int)(bytes % 16);
    long long blocks = (nvec + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kBlock), 0, s, (uint4 *)dst,
                       (const uint4 *)src, nvec, (unsigned char *)dst + nvec * 16,
                       (const unsigned char *)src + nvec * 16, ntail);
}

}  // namespace ptmg

namespace ptmg {

// Zero fill with vector stores (kept out of hipMemsetAsync so that the
// work can be captured in a graph).
__global__ __launch_bounds__(kBlock) void k_zero(uint4 *p, long long nvec, unsigned char *tail,
                                                 int ntail, const int *gate)
{
    if (gated(gate)) return;
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long q = t; q < nvec; q += stride) p[q] = make_uint4(0, 0, 0, 0);
    if (t < ntail) tail[t] = 0;
}

// Two zero fills in one launch (the zero initial guess of p and T).
__global__ __launch_bounds__(kBlock) void k_zero2(uint4 *p, uint4 *q, long long nvec,
                                                  unsigned char *tp, unsigned char *tq, int ntail)
{
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = t; i < nvec; i += stride) {
        p[i] = make_uint4(0, 0, 0, 0);
        q[i] = make_uint4(0, 0, 0, 0);
    }
    if (t < ntail) {
        tp[t] = 0;
        tq[t] = 0;
    }
}

void launch_zero2(void *p, void *q, size_t bytes, hipStream_t s)
{
    const long long nvec = (long long)(bytes / 16);
    const int ntail = (int)(bytes % 16);
    long long blocks = (nvec + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero2, dim3((unsigned)blocks), dim3(kBlock), 0, s, (uint4 *)p,
                       (uint4 *)q, nvec, (unsigned char *)p + nvec * 16,
                       (unsigned char *)q + nvec * 16, ntail);
}

// The assembly's error flags into the host's pinned copy (through its
// device address), ordered on the stream like any kernel.
__global__ void k_flags_out(const int *src, int *dst, int n)
{
    if ((int)threadIdx.x < n) dst[threadIdx.x] = src[threadIdx.x];
}

void launch_flags_out(const int *src, int *dst, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_flags_out, dim3(1), dim3(64), 0, s, src, dst, n);
}

// ------------------------------------------------ stream-ordered solve
// The stop test of outer iteration k (the host loop's, on the device): the
// paper-form relative residual of each component from the norms of its
// residual, recorded in the history; the solve stops when both meet rtol,
// when a norm is not finite, or at max_cycles.
__global__ void k_async_decide(const double *norms, int k, double rtol, int max_cycles, int *gate,
                               AsyncInfo *info)
{
    if (threadIdx.x != 0 || gate[0] != 0) return;
    const double rel0 = norms[2] > 0 ? sqrt(norms[0] / norms[2]) : sqrt(norms[0]);
    const double rel1 = norms[3] > 0 ? sqrt(norms[1] / norms[3]) : sqrt(norms[1]);
    if (info->hist_len < PT_MAX_HIST) {
        info->hist[2 * info->hist_len] = rel0;
        info->hist[2 * info->hist_len + 1] = rel1;
        info->hist_len++;
    }
    info->relres[0] = rel0;
    info->relres[1] = rel1;
    int status = -1;
    if (!isfinite(rel0) || !isfinite(rel1)) {
        status = PT_ERR_NOCONV;
        info->nonfinite = 1;
    } else if (rel0 <= rtol && rel1 <= rtol) {
        status = PT_OK;
    } else if (k >= max_cycles) {
        status = PT_ERR_NOCONV;
    }
    if (status != -1) {
        info->status = status;
        info->cycles = k;
        gate[1] = k;
        gate[0] = 1;
    }
}

void launch_async_decide(const double *norms, int k, double rtol, int max_cycles, int *gate,
                         AsyncInfo *info, hipStream_t s)
{
    hipLaunchKernelGGL(k_async_decide, dim3(1), dim3(64), 0, s, norms, k, rtol, max_cycles, gate,
                       info);
}

// Where u_k lives after the solve: the caller's arrays when k + parity is
// even, else (xp, xT); from a zero guess u_0 is never stored.
// k1 (non-null): where outer 1 keeps its iterate as FP32 pairs (it may be
// p's own memory: each element is read before it is written)
__global__ __launch_bounds__(kBlock) void k_async_final(const int *gate, int parity, int zero_guess,
                                                        const double *xp, const double *xT,
                                                        const float2 *k1, double *p, double *T,
                                                        long long N)
{
    const int k = gate[1];
    const bool zero = k == 0 && zero_guess;
    const bool one = k == 1 && k1;
    if (!zero && !one && (k + parity) % 2 == 0) return;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < N; i += stride) {
        if (one) {
            const float2 v = k1[i];
            p[i] = (double)v.x;
            T[i] = (double)v.y;
        } else {
            p[i] = zero ? 0.0 : xp[i];
            T[i] = zero ? 0.0 : xT[i];
        }
    }
}

void launch_async_final(const int *gate, int parity, int zero_guess, const double *xp,
                        const double *xT, const float2 *k1, double *p, double *T, long long N,
                        hipStream_t s)
{
    long long blocks = (N + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_async_final, dim3((unsigned)blocks), dim3(kBlock), 0, s, gate, parity,
                       zero_guess, xp, xT, k1, p, T, N);
}

// The FP32 pairs of outer 1's iterate as FP64 p, T (k1 may be p's own
// memory: each element is read before it is written).
__global__ __launch_bounds__(kBlock) void k_pairs_to_fp64(const float2 *k1, double *p, double *T,
                                                          long long N)
{
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < N; i += stride) {
        const float2 v = k1[i];
        p[i] = (double)v.x;
        T[i] = (double)v.y;
    }
}

void launch_pairs_to_fp64(const float2 *k1, double *p, double *T, long long N, hipStream_t s)
{
    long long blocks = (N + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_pairs_to_fp64, dim3((unsigned)blocks), dim3(kBlock), 0, s, k1, p, T, N);
}

__global__ void k_gate_reset(int *gate, AsyncInfo *info)
{
    if (threadIdx.x != 0) return;
    gate[0] = 0;
    gate[1] = 0;
    info->status = -1;
    info->cycles = 0;
    info->hist_len = 0;
    info->nonfinite = 0;
    info->relres[0] = info->relres[1] = 0.0;
}

void launch_gate_reset(int *gate, AsyncInfo *info, hipStream_t s)
{
    hipLaunchKernelGGL(k_gate_reset, dim3(1), dim3(64), 0, s, gate, info);
}

void launch_zero(void *p, size_t bytes, hipStream_t s, const int *gate)
{
    const long long nvec = (long long)(bytes / 16);
    const int ntail = (int)(bytes % 16);
    long long blocks = (nvec + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(kBlock), 0, s, (uint4 *)p, nvec,
                       (unsigned char *)p + nvec * 16, ntail, gate);
}

}  // namespace ptmg

namespace ptmg {

// ------------------------------------------------ fused red-black sweep
// One whole red-black sweep on the finest grid (cell coefficients) in a
// single pass over memory.  A block owns an x-y tile of TX x TY cells and a
// chunk of planes along the slowest axis (z in 3-D, y in 2-D), which it
// walks in order.  LDS keeps a rolling window of 4 planes of (p, T) and of
// the cell coefficients, each with a ring of 2 cells.  A red-black sweep
// never reads a red cell's old value, so one LDS array per plane holds old
// black and new red values.  At plane step k the block
//   loads plane k+2, updates red on plane k+1 over the tile and a ring of
//   one cell (reads old black on planes k..k+2), updates black on plane k
//   over the tile (reads new red on planes k-1..k+1), writes plane k.
// Cells outside the grid get zero coefficients, so the harmonic-mean face
// weight to them is zero (no flux through the boundary).  Tiles are
// assigned XCD-aware (xcd_tile).

template <typename R>
__device__ __forceinline__ void block_solve(typename VT<R>::v2 f, typename VT<R>::v4 b, R gp_nb,
                                            R gT_nb, R Sp, R ST, typename VT<R>::v2 &o)
{
    const R gp = f.x + gp_nb, gT = f.y + gT_nb;
    const R a = b.x + Sp, d = b.w + ST;
    const R inv = quot(R(1), a * d - b.y * b.z);
    o.x = (d * gp - b.y * gT) * inv;
    o.y = (a * gT - b.z * gp) * inv;
}

template <typename R, int TX, int TY, bool ZG, bool FACES>
__global__ __launch_bounds__(TX *TY) void k_rb_fused3(Lvl<R> L, typename VT<R>::v2 *__restrict__ uo,
                                                      int zc, int tiles_x, int tiles_y, int ntiles)
{
    if (gated(L.gate)) return;
    // FACES: a coarse level with stored lower-face coefficients (fx, fy,
    // fz) instead of cell coefficients; faces of plane z are needed while
    // planes z-1 .. z+1 update, so they live in a 4-slot ring.
    // Software-pipelined walk over a 5-plane LDS ring: while plane step k
    // computes, the global loads of steps k+1 and k+2 (planes k+3, k+4 and
    // the f, B of their red and black cells) are in flight in registers,
    // three register sets taken in turn (the loop is unrolled by three, so
    // no set is copied while its loads are outstanding).  Five slots let
    // the store of plane k+2 overwrite plane k-3, whose last reader
    // finished before the previous barrier, so each step needs two
    // barriers.
    using V2 = typename VT<R>::v2;
    using V4 = typename VT<R>::v4;
    constexpr int NT = TX * TY;
    constexpr int PX = TX + 4, PY = TY + 4, PS = PX * PY;
    constexpr int NLD = (PS + NT - 1) / NT;     // plane cells loaded per thread
    constexpr int RW = (TX + 2) / 2;            // red cells per row of the ring region
    constexpr int BW = TX / 2;                  // black cells per tile row
    // ring slots: 5 with stored faces; 7 with cell coefficients, whose
    // walk takes one barrier per plane step (below)
    constexpr int NS = FACES ? 5 : 7;
    constexpr int NA = FACES ? 1 : NS, PA = FACES ? 1 : PS;
    constexpr int NF = FACES ? 4 : 1, PF = FACES ? PS : 1, NLF = FACES ? NLD : 1;
    __shared__ V2 su[NS][PS];
    __shared__ V2 sa[NA][PA];
    __shared__ V2 sfx[NF][PF], sfy[NF][PF], sfz[NF][PF];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int txi = tile % tiles_x;
    const int rr = tile / tiles_x;
    const int tyi = rr % tiles_y;
    const int tzi = rr / tiles_y;
    const int x0 = txi * TX, y0 = tyi * TY;
    const int z0 = tzi * zc, z1 = min(z0 + zc, L.nz);
    const R ih2 = (R)L.inv_h2;
    const long long nxy = (long long)L.nx * L.ny;
    const int t = threadIdx.x;
    auto slot = [](int z) { return FACES ? (z + 10) % 5 : (z + 14) % 7; };   // z >= -3
    auto fslot = [](int z) { return (z + 8) & 3; };

    // ---- per-thread pieces of a plane step: the global loads of step k
    // (plane k+2, f and B of the red cell on plane k+1 and of the black
    // cell on plane k) in registers
    struct Step {
        V2 pu[NLD], pa[NLD], pfx[NLF], pfy[NLF], pfz[NLF];
        int rc, bc;
        V2 rf, bf;
        V4 rB, bB;
    };
    auto fetch_plane = [&](int z, Step &S) {
#pragma unroll
        for (int i = 0; i < NLD; i++) {
            const int c = t + i * NT;
            S.pu[i].x = S.pu[i].y = R(0);
            S.pa[i].x = S.pa[i].y = R(0);
            if (FACES) {
                S.pfx[i].x = S.pfx[i].y = R(0);
                S.pfy[i].x = S.pfy[i].y = R(0);
                S.pfz[i].x = S.pfz[i].y = R(0);
            }
            if (c < PS) {
                const int gx = x0 + c % PX - 2, gy = y0 + c / PX - 2;
                if (z >= 0 && z < L.nz && gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny) {
                    const long long g = gx + (long long)L.nx * gy + nxy * z;
                    if (FACES) {
                        S.pfx[i] = L.fx[g];
                        S.pfy[i] = L.fy[g];
                        S.pfz[i] = L.fz[g];
                    } else {
                        S.pa[i] = cell_ac(L, g);
                    }
                    if (!ZG) S.pu[i] = L.u[g];
                }
            }
        }
    };
    auto store_plane = [&](int z, const Step &S) {
        const int s = slot(z);
#pragma unroll
        for (int i = 0; i < NLD; i++) {
            const int c = t + i * NT;
            if (c < PS) {
                su[s][c] = S.pu[i];
                if (FACES) {
                    const int fs = fslot(z);
                    sfx[fs][c] = S.pfx[i];
                    sfy[fs][c] = S.pfy[i];
                    sfz[fs][c] = S.pfz[i];
                } else {
                    sa[s][c] = S.pa[i];
                }
            }
        }
    };
    // red cell of this thread on plane z: ring region [1, TX+2] x [1, TY+2]
    auto red_cell = [&](int z, int &c, long long &g) {
        c = -1;
        if (z < 0 || z >= L.nz || t >= RW * (TY + 2)) return;
        const int ly = 1 + t / RW;
        const int gy = y0 + ly - 2;
        const int lx = 1 + 2 * (t % RW) + ((x0 - 1 + gy + z) & 1);
        const int gx = x0 + lx - 2;
        if (gx < 0 || gx >= L.nx || gy < 0 || gy >= L.ny) return;
        c = ly * PX + lx;
        g = gx + (long long)L.nx * gy + nxy * z;
    };
    // black cell of this thread on plane z: tile interior
    auto black_cell = [&](int z, int &c, long long &g) {
        c = -1;
        if (z < 0 || z >= L.nz || t >= BW * TY) return;
        const int ly = 2 + t / BW;
        const int gy = y0 + ly - 2;
        const int lx = 2 + 2 * (t % BW) + (1 - ((x0 + gy + z) & 1));
        const int gx = x0 + lx - 2;
        if (gx >= L.nx || gy >= L.ny) return;
        c = ly * PX + lx;
        g = gx + (long long)L.nx * gy + nxy * z;
    };
    auto update = [&](int z, int c, V2 f, V4 b) {
        const int s = slot(z), sm = slot(z - 1), sp = slot(z + 1);
        R gp = R(0), gT = R(0), Sp = R(0), ST = R(0);
        auto accw = [&](V2 w, int ss, int q) {
            const R wp = w.x * ih2, wT = w.y * ih2;
            const V2 uq = su[ss][q];
            Sp += wp;
            ST += wT;
            gp += wp * uq.x;
            gT += wT * uq.y;
        };
        if (FACES) {
            const int fs = fslot(z), fsp = fslot(z + 1);
            accw(sfx[fs][c], s, c - 1);
            accw(sfx[fs][c + 1], s, c + 1);
            accw(sfy[fs][c], s, c - PX);
            accw(sfy[fs][c + PX], s, c + PX);
            accw(sfz[fs][c], sm, c);
            accw(sfz[fsp][c], sp, c);
        } else {
            const V2 am = sa[s][c];
            accw(harm2(am, sa[s][c - 1]), s, c - 1);
            accw(harm2(am, sa[s][c + 1]), s, c + 1);
            accw(harm2(am, sa[s][c - PX]), s, c - PX);
            accw(harm2(am, sa[s][c + PX]), s, c + PX);
            accw(harm2(am, sa[sm][c]), sm, c);
            accw(harm2(am, sa[sp][c]), sp, c);
        }
        V2 o;
        block_solve<R>(f, b, gp, gT, Sp, ST, o);
        su[s][c] = relax(L.omega, o, su[s][c]);
    };
    auto write_plane = [&](int z) {
        if (z < z0 || z >= z1) return;
        const int s = slot(z);
        const int lx = 2 + t % TX, ly = 2 + t / TX;
        const int gx = x0 + lx - 2, gy = y0 + ly - 2;
        if (gx < L.nx && gy < L.ny) {
            uo[gx + (long long)L.nx * gy + nxy * z] = su[s][ly * PX + lx];
        }
    };

    // the global loads of step k (none past the chunk's last step): with
    // stored faces plane k+2, red on k+1, black on k; with cell
    // coefficients plane k+3, red on k+1, black on k-1
    auto load_step = [&](int k, Step &S) {
        S.rc = S.bc = -1;
        if (FACES ? k >= z1 : k > z1 + 1) return;
        long long g;
        fetch_plane(FACES ? k + 2 : k + 3, S);
        if (FACES || k + 1 <= z1) red_cell(k + 1, S.rc, g);
        if (S.rc >= 0) {
            S.rf = L.f[g];
            S.rB = sweep_B_raw(L, g);
        }
        const int kb = FACES ? k : k - 1;
        if (kb >= z0 && kb < z1) black_cell(kb, S.bc, g);
        if (S.bc >= 0) {
            S.bf = L.f[g];
            S.bB = sweep_B_raw(L, g);
        }
    };
    // plane step k from the set `cur`; the loads of step k+2 go to `ahead`.
    // Stored faces: red on k+1, a barrier, black on k.  Cell coefficients:
    // red on k+1 and black on k-1 in one barrier phase (red on k+1 reads
    // black on planes k..k+2, all still old; black on k-1 reads red on
    // k-2..k, all final since the previous steps), so each step needs one
    // barrier; the store of plane k+3 overwrites plane k-4, last read two
    // steps before.
    auto body = [&](int k, const Step &cur, Step &ahead) {
        if constexpr (FACES) {
            store_plane(k + 2, cur);
            load_step(k + 2, ahead);
            __syncthreads();
            write_plane(k - 1);
            if (cur.rc >= 0) update(k + 1, cur.rc, cur.rf, sweep_B_fin(L, cur.rB));
            __syncthreads();
            if (cur.bc >= 0) update(k, cur.bc, cur.bf, sweep_B_fin(L, cur.bB));
        } else {
            store_plane(k + 3, cur);
            load_step(k + 2, ahead);
            __syncthreads();
            write_plane(k - 2);
            if (cur.rc >= 0) update(k + 1, cur.rc, cur.rf, sweep_B_fin(L, cur.rB));
            if (cur.bc >= 0) update(k - 1, cur.bc, cur.bf, sweep_B_fin(L, cur.bB));
        }
    };

    // ---- prologue: planes z0-2 .. z0+1 (stored faces) or z0+2 (cell
    // coefficients), red on z0-1 and z0
    {
        Step S;
        for (int z = z0 - 2; z <= z0 + (FACES ? 1 : 2); z++) {
            fetch_plane(z, S);
            store_plane(z, S);
        }
    }
    __syncthreads();
    for (int z = z0 - 1; z <= z0; z++) {
        int c;
        long long g;
        red_cell(z, c, g);
        if (c >= 0) update(z, c, L.f[g], sweep_B(L, g));
        if (FACES) __syncthreads();
    }
    // in flight for steps z0 and z0+1
    Step A, B, C;
    load_step(z0, A);
    load_step(z0 + 1, B);
    // stored faces: steps z0 .. z1-1 and a last write; cell coefficients:
    // steps z0 .. z1+1 (the last two finish black and the writes)
    const int kend = FACES ? z1 : z1 + 2;
    for (int k = z0; k < kend; k += 3) {
        body(k, A, C);
        if (k + 1 >= kend) break;
        body(k + 1, B, A);
        if (k + 2 >= kend) break;
        body(k + 2, C, B);
    }
    if constexpr (FACES) {
        __syncthreads();
        write_plane(z1 - 1);
    }
}

// The finest 3-D sweep with every harmonic face coefficient computed once.
// Same walk as k_rb_fused3 (cell coefficients, a ring of two cells, red on
// plane k+1 over the tile and a ring of one, black on plane k over the
// tile), but the threads own columns: the thread that updates black at
// (x, y, k) also updates red at (x, y, k+1), one step earlier red at
// (x, y, k-1), so the two z faces of its black cell are faces its own red
// updates computed (kept in registers), and the red update writes its four
// in-plane faces to LDS (two plane slots), where the black update reads
// them.  Every face borders one red and one black cell, so a red-black
// sweep evaluates each face once (ring cells aside) instead of once per
// colour; the harmonic mean is symmetric in its arguments bit for bit, so
// the black update sums the same values in the same order.  Black no longer
// reads the cell coefficients, which then need three plane slots instead of
// five.  Threads BW*TY onwards take the red cells of the ring.
template <typename R, int TX, int TY, bool ZG>
__global__ __launch_bounds__(TX *TY) void k_rb_fused3c(Lvl<R> L, typename VT<R>::v2 *__restrict__ uo,
                                                       int zc, int tiles_x, int tiles_y, int ntiles)
{
    if (gated(L.gate)) return;
    using V2 = typename VT<R>::v2;
    using V4 = typename VT<R>::v4;
    constexpr int NT = TX * TY;
    constexpr int PX = TX + 4, PY = TY + 4, PS = PX * PY;
    constexpr int NLD = (PS + NT - 1) / NT;
    constexpr int BW = TX / 2;                  // black cells per tile row
    constexpr int NCOL = BW * TY;               // column-owning threads
    constexpr int NRING = TX + TY + 2;          // red cells of the ring, per plane
    static_assert(NCOL + NRING <= NT && TX % 2 == 0 && TY % 2 == 0, "thread mapping");
    __shared__ V2 su[5][PS];
    __shared__ V2 sa[3][PS];
    __shared__ V2 sfx[2][PS], sfy[2][PS];       // lower x / y face of each cell
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int txi = tile % tiles_x;
    const int rr = tile / tiles_x;
    const int tyi = rr % tiles_y;
    const int tzi = rr / tiles_y;
    const int x0 = txi * TX, y0 = tyi * TY;
    const int z0 = tzi * zc, z1 = min(z0 + zc, L.nz);
    const R ih2 = (R)L.inv_h2;
    const long long nxy = (long long)L.nx * L.ny;
    const int t = threadIdx.x;
    auto slot = [](int z) { return (z + 10) % 5; };   // z >= -2
    auto aslot = [](int z) { return (z + 9) % 3; };
    auto fslot = [](int z) { return z & 1; };

    struct Step {
        V2 pu[NLD], pa[NLD];
        int rc, bc;
        V2 rf, bf;
        V4 rB, bB;
    };
    auto fetch_plane = [&](int z, Step &S) {
#pragma unroll
        for (int i = 0; i < NLD; i++) {
            const int c = t + i * NT;
            S.pu[i].x = S.pu[i].y = R(0);
            S.pa[i].x = S.pa[i].y = R(0);
            if (c < PS) {
                const int gx = x0 + c % PX - 2, gy = y0 + c / PX - 2;
                if (z >= 0 && z < L.nz && gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny) {
                    const long long g = gx + (long long)L.nx * gy + nxy * z;
                    S.pa[i] = cell_ac(L, g);
                    if (!ZG) S.pu[i] = L.u[g];
                }
            }
        }
    };
    auto store_plane = [&](int z, const Step &S) {
        const int s = slot(z), sa_ = aslot(z);
#pragma unroll
        for (int i = 0; i < NLD; i++) {
            const int c = t + i * NT;
            if (c < PS) {
                su[s][c] = S.pu[i];
                sa[sa_][c] = S.pa[i];
            }
        }
    };
    // red cell of this thread on plane z: a tile column (t < NCOL), the
    // column of its black cell on plane z - 1, or a red cell of the ring
    auto red_cell = [&](int z, int &c, long long &g) {
        c = -1;
        if (z < 0 || z >= L.nz || t >= NCOL + NRING) return;
        int lx, ly;
        if (t < NCOL) {
            ly = 2 + t / BW;
            lx = 2 + 2 * (t % BW) + ((x0 + y0 + ly + z) & 1);
        } else {
            const int q = t - NCOL;
            constexpr int HX = (TX + 2) / 2, HY = TY / 2;
            if (q < HX) {                       // row below the tile
                ly = 1;
                lx = 1 + 2 * q + ((x0 + y0 + z) & 1);
            } else if (q < 2 * HX) {            // row above the tile
                ly = TY + 2;
                lx = 1 + 2 * (q - HX) + ((x0 + y0 + z + 1) & 1);
            } else if (q < 2 * HX + HY) {       // column left of the tile
                lx = 1;
                ly = 2 + 2 * (q - 2 * HX) + ((x0 + y0 + z + 1) & 1);
            } else {                            // column right of the tile
                lx = TX + 2;
                ly = 2 + 2 * (q - 2 * HX - HY) + ((x0 + y0 + z) & 1);
            }
        }
        const int gx = x0 + lx - 2, gy = y0 + ly - 2;
        if (gx < 0 || gx >= L.nx || gy < 0 || gy >= L.ny) return;
        c = ly * PX + lx;
        g = gx + (long long)L.nx * gy + nxy * z;
    };
    // black cell of this thread on plane z (t < NCOL): a tile cell
    auto black_cell = [&](int z, int &c, long long &g) {
        c = -1;
        if (z < 0 || z >= L.nz || t >= NCOL) return;
        const int ly = 2 + t / BW;
        const int lx = 2 + 2 * (t % BW) + ((x0 + y0 + ly + z + 1) & 1);
        const int gx = x0 + lx - 2, gy = y0 + ly - 2;
        if (gx >= L.nx || gy >= L.ny) return;
        c = ly * PX + lx;
        g = gx + (long long)L.nx * gy + nxy * z;
    };
    auto accw = [&](R &gp, R &gT, R &Sp, R &ST, V2 w, int ss, int q) {
        const R wp = w.x * ih2, wT = w.y * ih2;
        const V2 uq = su[ss][q];
        Sp += wp;
        ST += wT;
        gp += wp * uq.x;
        gT += wT * uq.y;
    };
    // red update on plane z: computes its six faces, writes the four in
    // the plane to LDS, returns the two z faces
    auto update_red = [&](int z, int c, V2 f, V4 b, V2 &wzm, V2 &wzp) {
        const int s = slot(z), sm = slot(z - 1), sp = slot(z + 1);
        const int a0 = aslot(z), fs = fslot(z);
        R gp = R(0), gT = R(0), Sp = R(0), ST = R(0);
        const V2 am = sa[a0][c];
        const V2 wxm = harm2(am, sa[a0][c - 1]), wxp = harm2(am, sa[a0][c + 1]);
        const V2 wym = harm2(am, sa[a0][c - PX]), wyp = harm2(am, sa[a0][c + PX]);
        wzm = harm2(am, sa[aslot(z - 1)][c]);
        wzp = harm2(am, sa[aslot(z + 1)][c]);
        sfx[fs][c] = wxm;
        sfx[fs][c + 1] = wxp;
        sfy[fs][c] = wym;
        sfy[fs][c + PX] = wyp;
        accw(gp, gT, Sp, ST, wxm, s, c - 1);
        accw(gp, gT, Sp, ST, wxp, s, c + 1);
        accw(gp, gT, Sp, ST, wym, s, c - PX);
        accw(gp, gT, Sp, ST, wyp, s, c + PX);
        accw(gp, gT, Sp, ST, wzm, sm, c);
        accw(gp, gT, Sp, ST, wzp, sp, c);
        V2 o;
        block_solve<R>(f, b, gp, gT, Sp, ST, o);
        su[s][c] = relax(L.omega, o, su[s][c]);
    };
    // black update on plane z with the faces of its red neighbours
    auto update_black = [&](int z, int c, V2 f, V4 b, V2 wzm, V2 wzp) {
        const int s = slot(z), sm = slot(z - 1), sp = slot(z + 1), fs = fslot(z);
        R gp = R(0), gT = R(0), Sp = R(0), ST = R(0);
        accw(gp, gT, Sp, ST, sfx[fs][c], s, c - 1);
        accw(gp, gT, Sp, ST, sfx[fs][c + 1], s, c + 1);
        accw(gp, gT, Sp, ST, sfy[fs][c], s, c - PX);
        accw(gp, gT, Sp, ST, sfy[fs][c + PX], s, c + PX);
        accw(gp, gT, Sp, ST, wzm, sm, c);
        accw(gp, gT, Sp, ST, wzp, sp, c);
        V2 o;
        block_solve<R>(f, b, gp, gT, Sp, ST, o);
        su[s][c] = relax(L.omega, o, su[s][c]);
    };
    auto write_plane = [&](int z) {
        if (z < z0 || z >= z1) return;
        const int s = slot(z);
        const int lx = 2 + t % TX, ly = 2 + t / TX;
        const int gx = x0 + lx - 2, gy = y0 + ly - 2;
        if (gx < L.nx && gy < L.ny) {
            uo[gx + (long long)L.nx * gy + nxy * z] = su[s][ly * PX + lx];
        }
    };
    auto load_step = [&](int k, Step &S) {
        S.rc = S.bc = -1;
        if (k >= z1) return;
        long long g;
        fetch_plane(k + 2, S);
        red_cell(k + 1, S.rc, g);
        if (S.rc >= 0) {
            S.rf = L.f[g];
            S.rB = sweep_B_raw(L, g);
        }
        black_cell(k, S.bc, g);
        if (S.bc >= 0) {
            S.bf = L.f[g];
            S.bB = sweep_B_raw(L, g);
        }
    };
    // z faces of this thread's column: zq0 is the lower face of its black
    // cell at the current step (the upper face of its red cell two steps
    // back), zq1 the one for the next step
    V2 zq0, zq1;
    zq0.x = zq0.y = zq1.x = zq1.y = R(0);
    auto body = [&](int k, const Step &cur, Step &ahead) {
        store_plane(k + 2, cur);
        load_step(k + 2, ahead);
        __syncthreads();
        write_plane(k - 1);
        V2 wzm, wzp;
        wzm.x = wzm.y = wzp.x = wzp.y = R(0);
        if (cur.rc >= 0) update_red(k + 1, cur.rc, cur.rf, sweep_B_fin(L, cur.rB), wzm, wzp);
        __syncthreads();
        if (cur.bc >= 0) update_black(k, cur.bc, cur.bf, sweep_B_fin(L, cur.bB), zq0, wzm);
        zq0 = zq1;
        zq1 = wzp;
    };

    // a face whose red cell lies outside the grid is never written: zero
    // (no flux), and it stays zero, as a cell has the same colour on every
    // plane that uses the same face slot
    for (int c = t; c < PS; c += NT) {
        sfx[0][c].x = sfx[0][c].y = sfx[1][c].x = sfx[1][c].y = R(0);
        sfy[0][c].x = sfy[0][c].y = sfy[1][c].x = sfy[1][c].y = R(0);
    }
    // ---- prologue: planes z0-2 .. z0 (three coefficient slots), red on
    // z0-1, plane z0+1, red on z0
    {
        Step S;
        for (int z = z0 - 2; z <= z0; z++) {
            fetch_plane(z, S);
            store_plane(z, S);
        }
        __syncthreads();
        int c;
        long long g;
        V2 wzm, wzp;
        red_cell(z0 - 1, c, g);
        if (c >= 0) update_red(z0 - 1, c, L.f[g], sweep_B(L, g), wzm, wzp);
        if (c >= 0 && t < NCOL) zq0 = wzp;
        fetch_plane(z0 + 1, S);
        __syncthreads();
        store_plane(z0 + 1, S);
        __syncthreads();
        red_cell(z0, c, g);
        if (c >= 0) update_red(z0, c, L.f[g], sweep_B(L, g), wzm, wzp);
        if (c >= 0 && t < NCOL) zq1 = wzp;
        __syncthreads();
    }
    Step A, B, C;
    load_step(z0, A);
    load_step(z0 + 1, B);
    for (int k = z0; k < z1; k += 3) {
        body(k, A, C);
        if (k + 1 >= z1) break;
        body(k + 1, B, A);
        if (k + 2 >= z1) break;
        body(k + 2, C, B);
    }
    __syncthreads();
    write_plane(z1 - 1);
}

// The finest 3-D sweep with the residual and its restriction fused in
// (the last pre-smoothing sweep of a V-cycle).  The sweep is k_rb_fused3's
// (same per-cell arithmetic, same order), with a ring of three cells so
// that the block also finishes black on a ring of one and red on a ring of
// two: after the sweep every neighbour of a tile cell then holds its final
// value in LDS, and the residual f - A u of the tile can be formed without
// reading another block's output.  The chunk's black planes extend one
// plane below and above it for the same reason (only the chunk's own
// planes are written).  At plane step k (red on k+1, black on k) the
// residual of plane k-2, whose planes k-3 .. k-1 are final, is formed by
// one thread per tile cell (its own column's plane k-3 kept in registers,
// as the 5-slot ring no longer holds it) with the arithmetic and summation
// order of k_restrict_zm, and the 2 x 2 x 2 child means go to the coarse
// right-hand side.  One plane step ahead is loaded while a step computes
// (two register sets), to keep the registers of 1024 threads within one
// block per CU.  FP32 only: FP64 rings of three cells exceed the LDS.
template <typename R, int TX, int TY, bool ZG>
__global__ __launch_bounds__(TX *TY) void k_rb_fused3r(Lvl<R> L, Lvl<R> C,
                                                       typename VT<R>::v2 *__restrict__ uo, int zc,
                                                       int tiles_x, int tiles_y, int ntiles)
{
    if (gated(L.gate)) return;
    using V2 = typename VT<R>::v2;
    using V4 = typename VT<R>::v4;
    constexpr int G = 3;                         // loaded ring around the tile
    constexpr int NT = TX * TY;
    constexpr int PX = TX + 2 * G, PY = TY + 2 * G, PS = PX * PY;
    constexpr int NLD = (PS + NT - 1) / NT;      // plane cells loaded per thread
    constexpr int RW = (TX + 4) / 2, RH = TY + 4;   // red: tile and two rings
    constexpr int BW = (TX + 2) / 2, BH = TY + 2;   // black: tile and one ring
    constexpr int CX = TX / 2, CY = TY / 2;
    static_assert(RW * RH <= NT && BW * BH <= NT && TX % 2 == 0 && TY % 2 == 0,
                  "thread mapping");
    __shared__ V2 su[5][PS];
    __shared__ V2 sa[5][PS];
    __shared__ V2 sr[NT];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int txi = tile % tiles_x;
    const int rr = tile / tiles_x;
    const int tyi = rr % tiles_y;
    const int tzi = rr / tiles_y;
    const int x0 = txi * TX, y0 = tyi * TY;
    const int z0 = tzi * zc, z1 = min(z0 + zc, L.nz);
    const R ih2 = (R)L.inv_h2;
    const long long nxy = (long long)L.nx * L.ny;
    const int t = threadIdx.x;
    auto slot = [](int z) { return (z + 10) % 5; };   // z >= -3

    struct Step {
        V2 pu[NLD], pa[NLD];
        int rc, bc;
        V2 rf, bf;
        V4 rB, bB;
    };
    auto fetch_plane = [&](int z, Step &S) {
#pragma unroll
        for (int i = 0; i < NLD; i++) {
            const int c = t + i * NT;
            S.pu[i].x = S.pu[i].y = R(0);
            S.pa[i].x = S.pa[i].y = R(0);
            if (c < PS) {
                const int gx = x0 + c % PX - G, gy = y0 + c / PX - G;
                if (z >= 0 && z < L.nz && gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny) {
                    const long long g = gx + (long long)L.nx * gy + nxy * z;
                    S.pa[i] = cell_ac(L, g);
                    if (!ZG) S.pu[i] = L.u[g];
                }
            }
        }
    };
    auto store_plane = [&](int z, const Step &S) {
        const int s = slot(z);
#pragma unroll
        for (int i = 0; i < NLD; i++) {
            const int c = t + i * NT;
            if (c < PS) {
                su[s][c] = S.pu[i];
                sa[s][c] = S.pa[i];
            }
        }
    };
    // red cell of this thread on plane z: region [1, TX+5) x [1, TY+5)
    auto red_cell = [&](int z, int &c, long long &g) {
        c = -1;
        if (z < 0 || z >= L.nz || t >= RW * RH) return;
        const int ly = 1 + t / RW;
        const int gy = y0 + ly - G;
        const int lx = 1 + 2 * (t % RW) + ((x0 + 1 - G + gy + z) & 1);
        const int gx = x0 + lx - G;
        if (gx < 0 || gx >= L.nx || gy < 0 || gy >= L.ny) return;
        c = ly * PX + lx;
        g = gx + (long long)L.nx * gy + nxy * z;
    };
    // black cell of this thread on plane z: region [2, TX+4) x [2, TY+4)
    auto black_cell = [&](int z, int &c, long long &g) {
        c = -1;
        if (z < 0 || z >= L.nz || t >= BW * BH) return;
        const int ly = 2 + t / BW;
        const int gy = y0 + ly - G;
        const int lx = 2 + 2 * (t % BW) + ((x0 + 3 - G + gy + z) & 1);
        const int gx = x0 + lx - G;
        if (gx < 0 || gx >= L.nx || gy < 0 || gy >= L.ny) return;
        c = ly * PX + lx;
        g = gx + (long long)L.nx * gy + nxy * z;
    };
    // the red-black update of k_rb_fused3 (cell coefficients)
    auto update = [&](int z, int c, V2 f, V4 b) {
        const int s = slot(z), sm = slot(z - 1), sp = slot(z + 1);
        R gp = R(0), gT = R(0), Sp = R(0), ST = R(0);
        auto accw = [&](V2 w, int ss, int q) {
            const R wp = w.x * ih2, wT = w.y * ih2;
            const V2 uq = su[ss][q];
            Sp += wp;
            ST += wT;
            gp += wp * uq.x;
            gT += wT * uq.y;
        };
        const V2 am = sa[s][c];
        accw(harm2(am, sa[s][c - 1]), s, c - 1);
        accw(harm2(am, sa[s][c + 1]), s, c + 1);
        accw(harm2(am, sa[s][c - PX]), s, c - PX);
        accw(harm2(am, sa[s][c + PX]), s, c + PX);
        accw(harm2(am, sa[sm][c]), sm, c);
        accw(harm2(am, sa[sp][c]), sp, c);
        V2 o;
        block_solve<R>(f, b, gp, gT, Sp, ST, o);
        su[s][c] = relax(L.omega, o, su[s][c]);
    };
    // this thread's tile cell (residual) and coarse cell (restriction)
    const int lxr = G + t % TX, lyr = G + t / TX;
    const int gxr = x0 + lxr - G, gyr = y0 + lyr - G;
    const bool rmine = gxr < L.nx && gyr < L.ny;
    const int cr = lyr * PX + lxr;
    const int cxl = t % CX, cyl = t / CX;
    const int gcx = x0 / 2 + cxl, gcy = y0 / 2 + cyl;
    const bool cmine = t < CX * CY && gcx < C.nx && gcy < C.ny;
    V2 um_prev, am_prev;     // the thread's own cell on the plane below the residual's
    um_prev.x = um_prev.y = am_prev.x = am_prev.y = R(0);
    R accp = R(0), accT = R(0);
    // residual of plane q at the thread's tile cell, into sr; the own
    // cell of plane q becomes the z- neighbour of the next residual
    auto residual = [&](int q, bool want) {
        V2 r;
        r.x = r.y = R(0);
        const int s = slot(q), sp = slot(q + 1);
        const V2 um = su[s][cr], am = sa[s][cr];
        if (want && rmine) {
            const long long g = gxr + (long long)L.nx * gyr + nxy * q;
            const V2 f = L.f[g];
            const V4 B = sweep_B(L, g);
            R nbp = R(0), nbT = R(0), Sp = R(0), ST = R(0);
            auto nb = [&](V2 aq, V2 uq) {
                V2 w = harm2(am, aq);
                const R wp = w.x * ih2, wT = w.y * ih2;
                Sp += wp;
                ST += wT;
                nbp += wp * uq.x;
                nbT += wT * uq.y;
            };
            nb(sa[s][cr - 1], su[s][cr - 1]);
            nb(sa[s][cr + 1], su[s][cr + 1]);
            nb(sa[s][cr - PX], su[s][cr - PX]);
            nb(sa[s][cr + PX], su[s][cr + PX]);
            nb(am_prev, um_prev);
            nb(sa[sp][cr], su[sp][cr]);
            const R Ap = Sp * um.x - nbp + B.x * um.x + B.y * um.y;
            const R AT = ST * um.y - nbT + B.z * um.x + B.w * um.y;
            r.x = f.x - Ap;
            r.y = f.y - AT;
        }
        sr[t] = r;
        um_prev = um;
        am_prev = am;
    };
    // the 2 x 2 children of this thread's coarse cell on plane q (after a
    // barrier), summed as k_restrict_zm sums them; the coarse plane is
    // written after its odd fine plane
    auto restrict_plane = [&](int q) {
        if (!cmine) return;
        const int base = 2 * cyl * TX + 2 * cxl;
        const V2 r00 = sr[base], r10 = sr[base + 1];
        const V2 r01 = sr[base + TX], r11 = sr[base + TX + 1];
        R sp_ = r00.x + r10.x, sT_ = r00.y + r10.y;
        sp_ += r01.x + r11.x;
        sT_ += r01.y + r11.y;
        accp += sp_;
        accT += sT_;
        if (q & 1) {
            V2 o;
            o.x = accp * R(0.125);
            o.y = accT * R(0.125);
            C.f[gcx + (long long)C.nx * gcy + (long long)C.nx * C.ny * (q >> 1)] = o;
            accp = accT = R(0);
        }
    };
    auto write_plane = [&](int z) {
        if (z < z0 || z >= z1 || !rmine) return;
        uo[gxr + (long long)L.nx * gyr + nxy * z] = su[slot(z)][cr];
    };
    // the global loads of step k: plane k+2, f and B of the red cell on
    // plane k+1 and of the black cell on plane k (none past step z1)
    auto load_step = [&](int k, Step &S) {
        S.rc = S.bc = -1;
        if (k > z1) return;
        long long g;
        fetch_plane(k + 2, S);
        red_cell(k + 1, S.rc, g);
        if (S.rc >= 0) {
            S.rf = L.f[g];
            S.rB = sweep_B_raw(L, g);
        }
        black_cell(k, S.bc, g);
        if (S.bc >= 0) {
            S.bf = L.f[g];
            S.bB = sweep_B_raw(L, g);
        }
    };
    // plane step k from `cur`; the loads of step k+1 go to `ahead`
    auto body = [&](int k, const Step &cur, Step &ahead) {
        store_plane(k + 2, cur);
        load_step(k + 1, ahead);
        __syncthreads();
        write_plane(k - 1);
        if (cur.rc >= 0) update(k + 1, cur.rc, cur.rf, sweep_B_fin(L, cur.rB));
        if (k - 2 >= z0 - 1) residual(k - 2, k - 2 >= z0);
        __syncthreads();
        if (cur.bc >= 0) update(k, cur.bc, cur.bf, sweep_B_fin(L, cur.bB));
        if (k - 2 >= z0) restrict_plane(k - 2);
    };

    // ---- prologue: planes z0-3 .. z0, red on z0-2 and z0-1
    {
        Step S;
        for (int z = z0 - 3; z <= z0; z++) {
            fetch_plane(z, S);
            store_plane(z, S);
        }
    }
    __syncthreads();
    for (int z = z0 - 2; z <= z0 - 1; z++) {
        int c;
        long long g;
        red_cell(z, c, g);
        if (c >= 0) update(z, c, L.f[g], sweep_B(L, g));
        __syncthreads();
    }
    // steps z0-1 .. z1: black on z0-1 .. z1, red on z0 .. z1+1
    Step A, B;
    load_step(z0 - 1, A);
    for (int k = z0 - 1; k <= z1; k += 2) {
        body(k, A, B);
        if (k + 1 > z1) break;
        body(k + 1, B, A);
    }
    // the last residual plane, z1 - 1 (plane z1 finished by the last step)
    __syncthreads();
    residual(z1 - 1, true);
    __syncthreads();
    restrict_plane(z1 - 1);
}

template <typename R>
void launch_rb_fused3r(const Lvl<R> &L, const Lvl<R> &C, typename VT<R>::v2 *uo, int zero_guess,
                       hipStream_t s)
{
    if constexpr (sizeof(R) == 4) {
        constexpr int TX = 64, TY = 16;
        const int tx = (L.nx + TX - 1) / TX, ty = (L.ny + TY - 1) / TY;
        // chunks of an even number of planes (a coarse plane takes two)
        int zc = L.nz;
        while (zc > 16 && (long long)tx * ty * ((L.nz + zc - 1) / zc) < 256)
            zc = ((zc + 1) / 2 + 1) & ~1;
        const int nt = tx * ty * ((L.nz + zc - 1) / zc);
        if (zero_guess)
            hipLaunchKernelGGL((k_rb_fused3r<R, TX, TY, true>), dim3(nt), dim3(TX * TY), 0, s, L, C,
                               uo, zc, tx, ty, nt);
        else
            hipLaunchKernelGGL((k_rb_fused3r<R, TX, TY, false>), dim3(nt), dim3(TX * TY), 0, s, L,
                               C, uo, zc, tx, ty, nt);
    }
}
template void launch_rb_fused3r<float>(const Lvl<float> &, const Lvl<float> &, float2 *, int,
                                       hipStream_t);
template void launch_rb_fused3r<double>(const Lvl<double> &, const Lvl<double> &, double2 *, int,
                                        hipStream_t);

// 2-D: one whole red-black sweep per TX x TY tile, not marching: the tile
// and a ring of 2 cells (u and the cell coefficients, or the stored faces)
// in LDS, red over the tile and a ring of one, then black over the tile.
// 2-D levels are small enough that thousands of independent tiles fill
// the chip.  Cells outside the grid carry zero coefficients.
template <typename R, int TX, int TY, bool ZG, bool FACES>
__global__ __launch_bounds__(TX *TY) void k_rb_tile2(Lvl<R> L, typename VT<R>::v2 *__restrict__ uo,
                                                     int tiles_x, int ntiles)
{
    if (gated(L.gate)) return;
    using V2 = typename VT<R>::v2;
    using V4 = typename VT<R>::v4;
    constexpr int NT = TX * TY;
    constexpr int PX = TX + 4, PY = TY + 4, PS = PX * PY;
    constexpr int RW = (TX + 2) / 2, BW = TX / 2;
    constexpr int PA = FACES ? 1 : PS, PF = FACES ? PS : 1;
    __shared__ V2 su[PS];
    __shared__ V2 sa[PA];
    __shared__ V2 sfx[PF], sfy[PF];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
    const R ih2 = (R)L.inv_h2;
    const int t = threadIdx.x;
    for (int c = t; c < PS; c += NT) {
        const int gx = x0 + c % PX - 2, gy = y0 + c / PX - 2;
        V2 u, a, fx, fy;
        u.x = u.y = a.x = a.y = fx.x = fx.y = fy.x = fy.y = R(0);
        if (gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny) {
            const long long g = gx + (long long)L.nx * gy;
            if (FACES) {
                fx = L.fx[g];
                fy = L.fy[g];
            } else {
                a = cell_ac(L, g);
            }
            if (!ZG) u = L.u[g];
        }
        su[c] = u;
        if (FACES) {
            sfx[c] = fx;
            sfy[c] = fy;
        } else {
            sa[c] = a;
        }
    }
    __syncthreads();
    auto update = [&](int c, long long g, int gy) {
        R gp = R(0), gT = R(0), Sp = R(0), ST = R(0);
        auto accw = [&](V2 w, int q) {
            const R wp = w.x * ih2, wT = w.y * ih2;
            const V2 uq = su[q];
            Sp += wp;
            ST += wT;
            gp += wp * uq.x;
            gT += wT * uq.y;
        };
        if (FACES) {
            accw(sfx[c], c - 1);
            accw(sfx[c + 1], c + 1);
            accw(sfy[c], c - PX);
            accw(sfy[c + PX], c + PX);
        } else {
            const V2 am = sa[c];
            V2 ym = harm2(am, sa[c - PX]), yp = harm2(am, sa[c + PX]);
            if (L.axm) {
                const V4 mt = L.axm[gy];
                axi_face(ym, mt, false);
                axi_face(yp, mt, true);
            }
            accw(harm2(am, sa[c - 1]), c - 1);
            accw(harm2(am, sa[c + 1]), c + 1);
            accw(ym, c - PX);
            accw(yp, c + PX);
        }
        V2 o;
        block_solve<R>(L.f[g], sweep_B(L, g), gp, gT, Sp, ST, o);
        su[c] = relax(L.omega, o, su[c]);
    };
    if (t < RW * (TY + 2)) {   // red cells ((x+y) even) of the tile and a ring of one
        const int ly = 1 + t / RW;
        const int gy = y0 + ly - 2;
        const int lx = 1 + 2 * (t % RW) + ((x0 - 1 + gy) & 1);
        const int gx = x0 + lx - 2;
        if (gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny)
            update(ly * PX + lx, gx + (long long)L.nx * gy, gy);
    }
    __syncthreads();
    if (t < BW * TY) {         // black cells of the tile
        const int ly = 2 + t / BW;
        const int gy = y0 + ly - 2;
        const int lx = 2 + 2 * (t % BW) + (1 - ((x0 + gy) & 1));
        const int gx = x0 + lx - 2;
        if (gx < L.nx && gy < L.ny) update(ly * PX + lx, gx + (long long)L.nx * gy, gy);
    }
    __syncthreads();
    {
        const int lx = 2 + t % TX, ly = 2 + t / TX;
        const int gx = x0 + lx - 2, gy = y0 + ly - 2;
        if (gx < L.nx && gy < L.ny) uo[gx + (long long)L.nx * gy] = su[ly * PX + lx];
    }
}

// 2-D finest grid (cell coefficients), one sweep per TX x TY tile with
// optional fused transfers:
//  PRO: the prolonged coarse correction is added to the iterate as it is
//       loaded (the first sweep after the coarse-grid correction);
//  RES: after the sweep, the residual on the tile is restricted to the
//       next level's f (the last sweep before restriction); the tile then
//       carries a ring of 3 cells, so that black is final on a ring of one
//       around it.
// The per-cell arithmetic and the restriction's summation order are those
// of the separate kernels (k_rb_tile2, k_prolong, k_restrict_zm).
template <typename R, int TX, int TY, bool ZG, bool PRO, bool RES>
__global__ __launch_bounds__(TX *TY) void k_rb_tile2x(Lvl<R> L, Lvl<R> C,
                                                      typename VT<R>::v2 *__restrict__ uo,
                                                      int tiles_x, int ntiles)
{
    if (gated(L.gate)) return;
    using V2 = typename VT<R>::v2;
    using V4 = typename VT<R>::v4;
    constexpr int NT = TX * TY;
    constexpr int RG = RES ? 3 : 2;
    constexpr int PX = TX + 2 * RG, PY = TY + 2 * RG, PS = PX * PY;
    constexpr int RWR = TX / 2 + RG - 1, RYR = TY + 2 * (RG - 1);   // red: ring RG - 1
    constexpr int RWB = TX / 2 + RG - 2, RYB = TY + 2 * (RG - 2);   // black: ring RG - 2
    static_assert(RWR * RYR <= NT && RWB * RYB <= NT, "tile too small for its rings");
    // sw[c] = (x- face, y- face) harmonic coefficients of cell c; every
    // face of a black cell or of a tile cell borders a red cell of the red
    // region, so the red pass computes each face once and the black pass
    // and the residual read it (scaled by 1/h^2 where used, in the same
    // expressions as the other kernels, so that contractions match)
    __shared__ V2 su[PS], sa[PS];
    __shared__ V4 sw[PS];
    __shared__ V2 sr[RES ? NT : 1];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
    const int ox = x0 - RG, oy = y0 - RG;
    const R ih2 = (R)L.inv_h2;
    const int t = threadIdx.x;
#pragma unroll
    for (int it = 0; it < (PS + NT - 1) / NT; it++) {
        const int c = t + it * NT;
        if (c >= PS) break;
        const int gx = ox + c % PX, gy = oy + c / PX;
        V2 u, a;
        u.x = u.y = a.x = a.y = R(0);
        if (gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny) {
            const long long g = gx + (long long)L.nx * gy;
            a = cell_ac(L, g);
            if (!ZG) {
                u = L.u[g];
                if (PRO) {
                    R vp, vT;
                    prolong_delta<R, 2>(C, gx, gy, 0, vp, vT);
                    u.x += vp;
                    u.y += vT;
                }
            }
        }
        su[c] = u;
        sa[c] = a;
    }
    __syncthreads();
    // block solve of cell c from its four face weights
    auto solve = [&](int c, long long g, V2 wxm, V2 wxp, V2 wym, V2 wyp) {
        R gp = R(0), gT = R(0), Sp = R(0), ST = R(0);
        auto accw = [&](V2 w, int q) {
            const R wp = w.x * ih2, wT = w.y * ih2;
            const V2 uq = su[q];
            Sp += wp;
            ST += wT;
            gp += wp * uq.x;
            gT += wT * uq.y;
        };
        accw(wxm, c - 1);
        accw(wxp, c + 1);
        accw(wym, c - PX);
        accw(wyp, c + PX);
        V2 o;
        block_solve<R>(L.f[g], sweep_B(L, g), gp, gT, Sp, ST, o);
        su[c] = relax(L.omega, o, su[c]);
    };
    auto weight = [&](V2 am, int q) { return harm2(am, sa[q]); };
    auto wget = [&](int c, V2 &wxm, V2 &wxp, V2 &wym, V2 &wyp) {
        const V4 a = sw[c], b = sw[c + 1], d = sw[c + PX];
        wxm.x = a.x;
        wxm.y = a.y;
        wym.x = a.z;
        wym.y = a.w;
        wxp.x = b.x;
        wxp.y = b.y;
        wyp.x = d.z;
        wyp.y = d.w;
    };
    // red: cells within ring RG - 1 (faces computed and kept for everyone)
    if (t < RWR * RYR) {
        const int d = RG - 1;
        const int ly = RG - d + t / RWR;
        const int gy = oy + ly;
        const int xs = x0 - d;
        const int gx = xs + 2 * (t % RWR) + ((xs + gy) & 1);
        const int c = ly * PX + gx - ox;
        const V2 am = sa[c];
        const V2 wxm = weight(am, c - 1), wxp = weight(am, c + 1);
        const V2 wym = weight(am, c - PX), wyp = weight(am, c + PX);
        V4 w;
        w.x = wxm.x;
        w.y = wxm.y;
        w.z = wym.x;
        w.w = wym.y;
        sw[c] = w;
        w.x = wxp.x;
        w.y = wxp.y;
        w.z = R(0);
        w.w = R(0);
        // x+ face of c is the x- face of c + 1 (a black cell), the y+ face
        // the y- face of c + PX: written into their slots
        ((V2 *)&sw[c + 1])[0] = wxp;
        ((V2 *)&sw[c + PX])[1] = wyp;
        if (gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny) {
            V2 ym = wym, yp = wyp;
            if (L.axm) {
                const V4 mt = L.axm[gy];
                axi_face(ym, mt, false);
                axi_face(yp, mt, true);
            }
            solve(c, gx + (long long)L.nx * gy, wxm, wxp, ym, yp);
        }
    }
    __syncthreads();
    if (t < RWB * RYB) {
        const int d = RG - 2;
        const int ly = RG - d + t / RWB;
        const int gy = oy + ly;
        const int xs = x0 - d;
        const int gx = xs + 2 * (t % RWB) + ((xs + gy + 1) & 1);
        const int c = ly * PX + gx - ox;
        if (gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny) {
            V2 wxm, wxp, wym, wyp;
            wget(c, wxm, wxp, wym, wyp);
            if (L.axm) {
                const V4 mt = L.axm[gy];
                axi_face(wym, mt, false);
                axi_face(wyp, mt, true);
            }
            solve(c, gx + (long long)L.nx * gy, wxm, wxp, wym, wyp);
        }
    }
    __syncthreads();
    const int lx = RG + t % TX, ly = RG + t / TX;
    const int gx = x0 + t % TX, gy = y0 + t / TX;
    const bool mine = gx < L.nx && gy < L.ny;
    const int c = ly * PX + lx;
    if (mine) uo[gx + (long long)L.nx * gy] = su[c];
    if (!RES) return;
    // residual f - A u on the tile, then the mean of each 2 x 2 block
    V2 r;
    r.x = r.y = R(0);
    if (mine) {
        const long long g = gx + (long long)L.nx * gy;
        const V2 um = su[c];
        R nbp = R(0), nbT = R(0), Sp = R(0), ST = R(0);
        V2 wxm, wxp, wym, wyp;
        wget(c, wxm, wxp, wym, wyp);
        if (L.axm) {
            const V4 mt = L.axm[gy];
            axi_face(wym, mt, false);
            axi_face(wyp, mt, true);
        }
        auto nb = [&](V2 w, int q) {
            const R wp = w.x * ih2, wT = w.y * ih2;
            const V2 uq = su[q];
            Sp += wp;
            ST += wT;
            nbp += wp * uq.x;
            nbT += wT * uq.y;
        };
        nb(wxm, c - 1);
        nb(wxp, c + 1);
        nb(wym, c - PX);
        nb(wyp, c + PX);
        const V2 f = L.f[g];
        const V4 B = sweep_B(L, g);
        const R Ap = Sp * um.x - nbp + B.x * um.x + B.y * um.y;
        const R AT = ST * um.y - nbT + B.z * um.x + B.w * um.y;
        r.x = f.x - Ap;
        r.y = f.y - AT;
    }
    sr[t] = r;
    __syncthreads();
    if (t < (TX / 2) * (TY / 2)) {
        const int ci = t % (TX / 2), cj = t / (TX / 2);
        const int I = x0 / 2 + ci, J = y0 / 2 + cj;
        if (I < C.nx && J < C.ny) {
            const int b0 = 2 * cj * TX + 2 * ci;
            const V2 r00 = sr[b0], r10 = sr[b0 + 1], r01 = sr[b0 + TX], r11 = sr[b0 + TX + 1];
            // row pairs first, as the plane-marching restriction sums them;
            // on an r-z grid each row's pair is weighted by its cell radius
            // (level 1 holds the volume-weighted equations)
            R accp = R(0), accT = R(0);
            if (L.axm) {
                const R rc0 = L.axm[2 * J].z, rc1 = L.axm[2 * J + 1].z;
                accp = fmadd(r00.x + r10.x, rc0, accp);
                accT = fmadd(r00.y + r10.y, rc0, accT);
                accp = fmadd(r01.x + r11.x, rc1, accp);
                accT = fmadd(r01.y + r11.y, rc1, accT);
            } else {
                accp += r00.x + r10.x;
                accT += r00.y + r10.y;
                accp += r01.x + r11.x;
                accT += r01.y + r11.y;
            }
            const R sc = R(0.25);
            V2 o;
            o.x = accp * sc;
            o.y = accT * sc;
            C.f[I + (long long)C.nx * J] = o;
        }
    }
}

// The finest 2-D level: one sweep with its fused transfers (see
// k_rb_tile2x); C is level 1 (its u for pro, its f written for res).
template <typename R>
void launch_tile2x(const Lvl<R> &L, const Lvl<R> &C, typename VT<R>::v2 *uo, int zero_guess,
                   int pro, int res, hipStream_t s)
{
    constexpr int TX = 64, TY = 8;
    const int tx = (L.nx + TX - 1) / TX, ty = (L.ny + TY - 1) / TY;
    const int nt = tx * ty;
#define PTMG_TILE2X(ZGC, PC, RC)                                                                \
    hipLaunchKernelGGL((k_rb_tile2x<R, TX, TY, ZGC, PC, RC>), dim3(nt), dim3(TX * TY), 0, s, L, C, \
                       uo, tx, nt)
    if (res) {
        if (zero_guess) PTMG_TILE2X(true, false, true);
        else PTMG_TILE2X(false, false, true);
    } else if (pro) {
        PTMG_TILE2X(false, true, false);
    } else {
        if (zero_guess) PTMG_TILE2X(true, false, false);
        else PTMG_TILE2X(false, false, false);
    }
#undef PTMG_TILE2X
}
template void launch_tile2x<float>(const Lvl<float> &, const Lvl<float> &, float2 *, int, int, int,
                                   hipStream_t);
template void launch_tile2x<double>(const Lvl<double> &, const Lvl<double> &, double2 *, int, int,
                                    int, hipStream_t);

// ------------------------------------------ 2-D coarse-level half cycles
// On the coarse 2-D levels a V-cycle visits each level twice: on the way
// down (nu1 sweeps from a zero guess, then the residual restricted to the
// next level) and on the way up (the prolonged correction added, then nu2
// sweeps).  These levels are small, so as separate kernels each step is
// bound by launch and memory latency; here each half is one kernel.  A
// block owns a TX x TY tile and recomputes a ring of 2 nu cells around it
// in LDS (each sweep needs its input one red and one black cell further
// out), so no block reads another block's intermediate values.  The
// arithmetic is that of the separate kernels cell for cell: the same face
// order (x-, x+, y-, y+; faces outside the grid are zero, which adds
// exact zeros), the same block solve, residual, restriction sum and
// prolongation weights.
//
// Patch coordinates: (lx, ly) in [0, PX) x [0, PY) at global
// (x0 - RG + lx, y0 - RG + ly); cells at ring distance d from the tile are
// those with lx in [RG - d, RG + TX + d), ly in [RG - d, RG + TY + d).  The
// extra column pair and row on the upper side hold the upper faces of the
// outermost cells.  Thread t owns the cell pairs (2 px, 2 px + 1) of row
// ly for pair indices t, t + NT, ...; their f and B are read once, before
// the first sweep.
template <typename R, int TX, int TY, int NU> struct HalfTile {
    static constexpr int NT = TX * TY;
    static constexpr int RG = 2 * NU;
    static constexpr int PX = TX + 2 * RG + 2, PY = TY + 2 * RG + 1, PS = PX * PY;
    static constexpr int HP = PX / 2, NPAIR = HP * PY, QP = (NPAIR + NT - 1) / NT;
};

template <typename R, int TX, int TY, int NU, bool UP>
__device__ __forceinline__ void half_cycle2(const Lvl<R> &L, const Lvl<R> &C,
                                            typename VT<R>::v2 *__restrict__ uo, int tiles_x,
                                            int ntiles)
{
    using V2 = typename VT<R>::v2;
    using V4 = typename VT<R>::v4;
    using H = HalfTile<R, TX, TY, NU>;
    constexpr int NT = H::NT, RG = H::RG, PX = H::PX, PY = H::PY, PS = H::PS, HP = H::HP,
                  NPAIR = H::NPAIR, QP = H::QP;
    __shared__ V2 su[PS], sfx[PS], sfy[PS];
    __shared__ V2 sr[UP ? 1 : NT];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
    const int ox = x0 - RG, oy = y0 - RG;
    const R ih2 = (R)L.inv_h2;
    const int t = threadIdx.x;
    auto inside = [&](int gx, int gy) { return gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny; };
    auto in_ring = [&](int lx, int ly, int d) {
        return lx >= RG - d && lx < RG + TX + d && ly >= RG - d && ly < RG + TY + d;
    };
    // faces and the iterate (zero going down; u + P e going up); a constant
    // trip count lets the loads of all iterations issue before any wait
#pragma unroll
    for (int it = 0; it < (PS + NT - 1) / NT; it++) {
        const int c = t + it * NT;
        if (c >= PS) break;
        const int lx = c % PX, ly = c / PX;
        const int gx = ox + lx, gy = oy + ly;
        V2 fx, fy, u;
        fx.x = fx.y = fy.x = fy.y = u.x = u.y = R(0);
        if (inside(gx, gy)) {
            const long long g = gx + (long long)L.nx * gy;
            fx = L.fx[g];
            fy = L.fy[g];
            if (UP && in_ring(lx, ly, RG)) {
                R vp, vT;
                prolong_delta<R, 2>(C, gx, gy, 0, vp, vT);
                u = L.u[g];
                u.x += vp;
                u.y += vT;
            }
        }
        sfx[c] = fx;
        sfy[c] = fy;
        su[c] = u;
    }
    // f and B of the owned cells that some sweep updates
    constexpr int DMAX = UP ? RG - 1 : RG;
    V2 f[QP][2];
    V4 B[QP][2];
#pragma unroll
    for (int q = 0; q < QP; q++) {
        const int p = t + q * NT;
#pragma unroll
        for (int k = 0; k < 2; k++) {
            f[q][k].x = f[q][k].y = R(0);
            B[q][k].x = B[q][k].y = B[q][k].z = B[q][k].w = R(0);
            if (p < NPAIR) {
                const int ly = p / HP, lx = 2 * (p % HP) + k;
                const int gx = ox + lx, gy = oy + ly;
                if (in_ring(lx, ly, DMAX) && inside(gx, gy)) {
                    const long long g = gx + (long long)L.nx * gy;
                    f[q][k] = L.f[g];
                    B[q][k] = sweep_B(L, g);
                }
            }
        }
    }
    __syncthreads();
    auto update = [&](int c, const V2 &fc, const V4 &Bc, bool zg) {
        R gp = R(0), gT = R(0), Sp = R(0), ST = R(0);
        auto accw = [&](V2 w, int q) {
            const R wp = w.x * ih2, wT = w.y * ih2;
            Sp += wp;
            ST += wT;
            if (!zg) {
                const V2 uq = su[q];
                gp += wp * uq.x;
                gT += wT * uq.y;
            }
        };
        accw(sfx[c], c - 1);
        accw(sfx[c + 1], c + 1);
        accw(sfy[c], c - PX);
        accw(sfy[c + PX], c + PX);
        V2 o;
        block_solve<R>(fc, Bc, gp, gT, Sp, ST, o);
        su[c] = o;
    };
    // one colour over the cells within ring distance d
    auto phase = [&](int color, int d, bool zg) {
#pragma unroll
        for (int q = 0; q < QP; q++) {
            const int p = t + q * NT;
            if (p >= NPAIR) continue;
            const int ly = p / HP;
            const int k = (color + ly) & 1;
            const int lx = 2 * (p % HP) + k;
            if (!in_ring(lx, ly, d) || !inside(ox + lx, oy + ly)) continue;
            // (selects, not a dynamic index: the arrays stay in registers)
            update(ly * PX + lx, k ? f[q][1] : f[q][0], k ? B[q][1] : B[q][0], zg);
        }
        __syncthreads();
    };
    if (UP) {
        for (int s = 1; s <= NU; s++) {
            phase(0, 2 * (NU - s) + 1, false);
            phase(1, 2 * (NU - s), false);
        }
        const int lx = RG + t % TX, ly = RG + t / TX;
        const int gx = ox + lx, gy = oy + ly;
        if (gx < L.nx && gy < L.ny) uo[gx + (long long)L.nx * gy] = su[ly * PX + lx];
        return;
    }
    for (int s = 1; s <= NU; s++) {
        phase(0, 2 * (NU - s) + 2, s == 1);
        phase(1, 2 * (NU - s) + 1, false);
    }
    // residual f - A u on the tile (the owned cells in it), u written out
#pragma unroll
    for (int q = 0; q < QP; q++) {
        const int p = t + q * NT;
        if (p >= NPAIR) continue;
        const int ly = p / HP;
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int lx = 2 * (p % HP) + k;
            const int gx = ox + lx, gy = oy + ly;
            if (!in_ring(lx, ly, 0) || !inside(gx, gy)) continue;
            const int c = ly * PX + lx;
            R nbp = R(0), nbT = R(0), Sp = R(0), ST = R(0);
            auto acc = [&](V2 w, int qq) {
                const R wp = w.x * ih2, wT = w.y * ih2;
                Sp += wp;
                ST += wT;
                const V2 uq = su[qq];
                nbp += wp * uq.x;
                nbT += wT * uq.y;
            };
            acc(sfx[c], c - 1);
            acc(sfx[c + 1], c + 1);
            acc(sfy[c], c - PX);
            acc(sfy[c + PX], c + PX);
            const V2 u = su[c];
            const V4 b = B[q][k];
            const R Ap = Sp * u.x - nbp + b.x * u.x + b.y * u.y;
            const R AT = ST * u.y - nbT + b.z * u.x + b.w * u.y;
            V2 r;
            r.x = f[q][k].x - Ap;
            r.y = f[q][k].y - AT;
            sr[(ly - RG) * TX + (lx - RG)] = r;
            L.u[gx + (long long)L.nx * gy] = u;
        }
    }
    __syncthreads();
    // restriction: coarse f = mean of the four children, in child order
    if (t < (TX / 2) * (TY / 2)) {
        const int ci = t % (TX / 2), cj = t / (TX / 2);
        const int I = x0 / 2 + ci, J = y0 / 2 + cj;
        if (I < C.nx && J < C.ny) {
            const int b0 = 2 * cj * TX + 2 * ci;
            const V2 r00 = sr[b0], r10 = sr[b0 + 1], r01 = sr[b0 + TX], r11 = sr[b0 + TX + 1];
            R sp = R(0), sT = R(0);
            sp += r00.x;
            sT += r00.y;
            sp += r10.x;
            sT += r10.y;
            sp += r01.x;
            sT += r01.y;
            sp += r11.x;
            sT += r11.y;
            const R sc = R(1) / R(4);
            V2 o;
            o.x = sp * sc;
            o.y = sT * sc;
            C.f[I + (long long)C.nx * J] = o;
        }
    }
}

template <typename R, int TX, int TY, int NU>
__global__ __launch_bounds__(TX *TY) void k_down2(Lvl<R> L, Lvl<R> C, int tiles_x, int ntiles)
{
    if (gated(L.gate)) return;
    half_cycle2<R, TX, TY, NU, false>(L, C, nullptr, tiles_x, ntiles);
}

template <typename R, int TX, int TY, int NU>
__global__ __launch_bounds__(TX *TY) void k_up2(Lvl<R> L, Lvl<R> C,
                                                typename VT<R>::v2 *__restrict__ uo, int tiles_x,
                                                int ntiles)
{
    if (gated(L.gate)) return;
    half_cycle2<R, TX, TY, NU, true>(L, C, uo, tiles_x, ntiles);
}

// Down: u_L = nu sweeps from zero on f_L (written to L.u), C.f = restricted
// residual.  Up: L.u + P C.u, then nu sweeps, written to uo (another
// buffer).  nu is 1 or 2; L is a coarse 2-D level (stored faces) whose
// dimensions are even.
template <typename R>
void launch_half2(bool up, int nu, const Lvl<R> &L, const Lvl<R> &C, typename VT<R>::v2 *uo,
                  hipStream_t s)
{
    constexpr int TX = 64, TY = 8;
    const int tx = (L.nx + TX - 1) / TX, ty = (L.ny + TY - 1) / TY;
    const int nt = tx * ty;
    if (up) {
        if (nu == 1) hipLaunchKernelGGL((k_up2<R, TX, TY, 1>), dim3(nt), dim3(TX * TY), 0, s, L, C, uo, tx, nt);
        else hipLaunchKernelGGL((k_up2<R, TX, TY, 2>), dim3(nt), dim3(TX * TY), 0, s, L, C, uo, tx, nt);
    } else {
        if (nu == 1) hipLaunchKernelGGL((k_down2<R, TX, TY, 1>), dim3(nt), dim3(TX * TY), 0, s, L, C, tx, nt);
        else hipLaunchKernelGGL((k_down2<R, TX, TY, 2>), dim3(nt), dim3(TX * TY), 0, s, L, C, tx, nt);
    }
}
template void launch_half2<float>(bool, int, const Lvl<float> &, const Lvl<float> &, float2 *,
                                  hipStream_t);
template void launch_half2<double>(bool, int, const Lvl<double> &, const Lvl<double> &, double2 *,
                                   hipStream_t);

// Reads the old iterate from L.u and writes the swept one to uo (a
// different buffer: blocks read halo cells that other blocks update).
// faces = 0: the finest grid (cell coefficients); 1: a coarse level.
template <typename R>
void launch_rb_fused(int dim, const Lvl<R> &L, typename VT<R>::v2 *uo, int zero_guess, int faces,
                     hipStream_t s)
{
    if (dim == 3) {
        // tile 64 x TY.  The FP32 finest grid takes 64 x 16 tiles (1024
        // threads, one block per CU with its 109 KB of LDS rings): the
        // two-cell y halo of the iterate and coefficients is re-read 1.33x
        // instead of 1.59x at 64 x 8, and 256 blocks (one per CU) keep the
        // z chunks long, so the four ring planes each chunk re-reads stay a
        // small share.  FP64 cells take twice the LDS, so the FP64 finest
        // grid keeps 64 x 8 (two blocks per CU, 512 blocks); coarse levels
        // with stored faces hold three more rings and take 64 x 4.
        constexpr int TX = 64;
        const int TY = faces ? 4 : (sizeof(R) == 4 ? 16 : 8);
        const int tx = (L.nx + TX - 1) / TX, ty = (L.ny + TY - 1) / TY;
        const long long want = TY == 4 ? 2048 : (TY == 16 ? 256 : 512);
        int zc = L.nz;
        while (zc > 16 && (long long)tx * ty * ((L.nz + zc - 1) / zc) < want) zc = (zc + 1) / 2;
        const int tz = (L.nz + zc - 1) / zc;
        const int nt = tx * ty * tz;
#define PTMG_FUSED3(TYC, ZGC, FC)                                                              \
    hipLaunchKernelGGL((k_rb_fused3<R, TX, TYC, ZGC, FC>), dim3(nt), dim3(TX * TYC), 0, s, L, uo, \
                       zc, tx, ty, nt)
        if (faces) {
            if (zero_guess) PTMG_FUSED3(4, true, true);
            else PTMG_FUSED3(4, false, true);
        } else if (TY == 16) {
            if constexpr (sizeof(R) == 4) {
                if (zero_guess) PTMG_FUSED3(16, true, false);
                else PTMG_FUSED3(16, false, false);
            }
        } else if (TY == 8) {
            // FP64: each face coefficient once per sweep (its divisions
            // bound the FP64 sweep)
            if constexpr (sizeof(R) == 8) {
                if (zero_guess)
                    hipLaunchKernelGGL((k_rb_fused3c<R, TX, 8, true>), dim3(nt), dim3(TX * 8), 0, s,
                                       L, uo, zc, tx, ty, nt);
                else
                    hipLaunchKernelGGL((k_rb_fused3c<R, TX, 8, false>), dim3(nt), dim3(TX * 8), 0, s,
                                       L, uo, zc, tx, ty, nt);
            }
        } else {
            if (zero_guess) PTMG_FUSED3(4, true, false);
            else PTMG_FUSED3(4, false, false);
        }
#undef PTMG_FUSED3
    } else {
        constexpr int TX = 64, TY = 8;
        const int tx = (L.nx + TX - 1) / TX, ty = (L.ny + TY - 1) / TY;
        const int nt = tx * ty;
#define PTMG_TILE2(ZGC, FC) \
    hipLaunchKernelGGL((k_rb_tile2<R, TX, TY, ZGC, FC>), dim3(nt), dim3(TX * TY), 0, s, L, uo, tx, nt)
        if (faces) {
            if (zero_guess) PTMG_TILE2(true, true);
            else PTMG_TILE2(false, true);
        } else {
            if (zero_guess) PTMG_TILE2(true, false);
            else PTMG_TILE2(false, false);
        }
#undef PTMG_TILE2
    }
}
template void launch_rb_fused<float>(int, const Lvl<float> &, float2 *, int, int, hipStream_t);
template void launch_rb_fused<double>(int, const Lvl<double> &, double2 *, int, int, hipStream_t);

}  // namespace ptmg

namespace ptmg {

// Gauss-Jordan inversion without pivoting of an m x m matrix (m <= 128) in
// one block, the matrix resident in LDS: the same elimination as k_gj_step,
// with the pivot row and column copied aside before each update.
constexpr int kGJLdsMax = 128;
// The elimination by the first nt threads of the block (nt a multiple of m;
// every thread of the block reaches the barriers).
__device__ __forceinline__ void gj_lds_body(const double *A, double *Ainv, int m, int *flags,
                                            double *M, double *rowk, double *colk, int nt)
{
    const int mm = m * m;
    const bool act = (int)threadIdx.x < nt;
    for (int e = threadIdx.x; e < mm; e += blockDim.x) M[e] = A[e];
    __syncthreads();
    for (int k = 0; k < m; k++) {
        const double p = M[k * m + k];
        const double q = 1.0 / p;
        // scaled pivot row and the pivot column, as in k_gj_step
        for (int e = threadIdx.x; e < m; e += blockDim.x) {
            rowk[e] = M[k * m + e] * q;
            colk[e] = M[e * m + k];
        }
        if (threadIdx.x == 0 && (!(p > 0.0) || !isfinite(p))) atomicOr(&flags[FLAG_PIVOT], 1);
        __syncthreads();
        if (act) {
            for (int i = threadIdx.x / m; i < m; i += nt / m) {
                const int j = threadIdx.x % m;
                const int e = i * m + j;
                double v;
                if (i == k && j == k) v = q;
                else if (i == k) v = rowk[j];
                else if (j == k) v = -colk[i] * q;
                else v = M[e] - colk[i] * rowk[j];
                M[e] = v;
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < mm; e += blockDim.x) Ainv[e] = M[e];
}

__global__ __launch_bounds__(1024) void k_gj_lds(const double *A, double *Ainv, int m, int *flags)
{
    __shared__ double M[kGJLdsMax * kGJLdsMax];
    __shared__ double rowk[kGJLdsMax], colk[kGJLdsMax];
    gj_lds_body(A, Ainv, m, flags, M, rowk, colk, (int)blockDim.x);
}

// The small end of the hierarchy build in one block: the coarsening of
// levels g[0] -> g[1] -> ... -> g[nl-1] (at most a few thousand cells
// each), the dense matrix of the coarsest and its Gauss-Jordan inverse,
// with the arithmetic of k_coarsen, k_coarse_dense and k_gj_lds; as
// separate kernels each of these steps is a launch.  The level views are
// staged in LDS and read with a dynamic index, so every step has one copy
// of its code.
template <typename R, int DIM>
__global__ __launch_bounds__(1024) void k_hier_small(HierSmallArgs<R> A)
{
    using O2 = typename VT<R>::v2;
    using O4 = typename VT<R>::v4;
    __shared__ Lvl<R> sl[kMaxTail];
    __shared__ double M[kGJLdsMax * kGJLdsMax];
    __shared__ double rowk[kGJLdsMax], colk[kGJLdsMax];
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < kMaxTail; q++)
        if (t == q && q < A.nl) sl[q] = A.g[q];
    __syncthreads();
    for (int q = 0; q + 1 < A.nl; q++) {
        const Lvl<R> F = sl[q], C = sl[q + 1];
        for (long long c = t; c < C.N; c += blockDim.x)
            coarsen_cell<R, R, DIM, false>(F, C.nx, C.ny, C.nz, (O2 *)C.fx, (O2 *)C.fy,
                                           (O2 *)C.fz, (O4 *)C.B, c);
        __syncthreads();
    }
    const Lvl<R> L = sl[A.nl - 1];
    for (long long r = t; r < 2 * L.N; r += blockDim.x) dense_row<R, DIM, false>(L, A.pin, A.M0, r);
    __syncthreads();
    gj_lds_body(A.M0, A.Ainv, A.m, A.flags, M, rowk, colk, (int)(blockDim.x / A.m) * A.m);
}

template <typename R>
bool launch_hier_small(int dim, const HierSmallArgs<R> &a, hipStream_t s)
{
    if (a.m > kGJLdsMax || a.nl < 2 || a.nl > kMaxTail) return false;
    if (dim == 3) hipLaunchKernelGGL((k_hier_small<R, 3>), dim3(1), dim3(1024), 0, s, a);
    else hipLaunchKernelGGL((k_hier_small<R, 2>), dim3(1), dim3(1024), 0, s, a);
    return true;
}
template bool launch_hier_small<float>(int, const HierSmallArgs<float> &, hipStream_t);
template bool launch_hier_small<double>(int, const HierSmallArgs<double> &, hipStream_t);

bool launch_gj_lds(const double *A, double *Ainv, int m, int *flags, hipStream_t s)
{
    if (m > kGJLdsMax) return false;
    // threads per block: a multiple of m (each thread keeps one column j)
    const int nt = (1024 / m) * m;
    hipLaunchKernelGGL(k_gj_lds, dim3(1), dim3(nt), 0, s, A, Ainv, m, flags);
    return true;
}

}  // namespace ptmg

namespace ptmg {

// -------------------------------------------- plane-marching stencils
// The FP64 outer residual: u_new = u + du (when update), the residual of
// the mode-native form (paper form Eqs. 27-28 in phases and state mode,
// computed directly so that its rounding does not depend on the size of
// b), the canonical residual for the V-cycle (r_T = -res_T,
// r_p = -res_p + l4 res_T), and per-block sums of res_p^2, res_T^2, b_p^2,
// b_T^2 for the fixed-order norm reduction.
// The FP64 outer residual and the finest-grid residual + restriction as
// z-marching tiles: a 4-slot LDS ring of planes (tile + a ring of one
// cell) so that every array element is read from HBM once, with the next
// plane and the next cells' pointwise data prefetched into registers while
// the current plane computes (one barrier per plane).  A 2-D grid runs as a
// flat 3-D one (ny = 1, planes = rows, TY = 1, no y neighbours).
template <int TY> struct Flat { static constexpr bool v = TY == 1; };

// The right-hand side with the mean constraint's shift.
template <typename RV>
__device__ __forceinline__ void outer_b(const OuterArgs<RV> &a, double &bp, double &bT)
{
    if (a.bshift) {
        bp -= a.bshift_scale * a.bshift[0];
        bT -= a.bshift_scale * a.bshift[1];
    }
}
// The outputs of one cell of the outer residual and its terms of the
// norms (every sum written out, so the residual of a zero iterate below
// sums exactly as the stencil kernel does).
template <typename RV>
__device__ __forceinline__ void outer_out(const OuterArgs<RV> &a, long long g, double resp,
                                          double resT, double rp, double rT, double bp,
                                          double bT, double *acc)
{
    if (a.r) {
        typename VT<RV>::v2 o;
        o.x = (RV)rp;
        o.y = (RV)rT;
        a.r[g] = o;
    }
    if (a.res_p) a.res_p[g] = resp;
    if (a.res_T) a.res_T[g] = resT;
    if (a.r64_p) {
        a.r64_p[g] = rp;
        a.r64_T[g] = rT;
    }
    acc[0] = fmadd(resp, resp, acc[0]);
    acc[1] = fmadd(resT, resT, acc[1]);
    acc[2] = fmadd(bp, bp, acc[2]);
    acc[3] = fmadd(bT, bT, acc[3]);
}

template <int DIM, typename RV, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void k_outer_zm(OuterArgs<RV> a, int NX, int NY, int NZ,
                                                     int zc, int tiles_x, int tiles_y, int ntiles)
{
    if (gated(a.gate)) return;
    using V2 = typename VT<RV>::v2;
    constexpr bool FLAT = Flat<TY>::v;
    constexpr int NT = TX * TY;
    constexpr int PX = TX + 2, PY = FLAT ? 1 : TY + 2, PS = PX * PY;
    constexpr int NLD = (PS + NT - 1) / NT;
    __shared__ double2 su[4][PS];
    __shared__ double2 sa[4][PS];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int t = threadIdx.x;
    if (tile < ntiles) {
        const int txi = tile % tiles_x;
        const int rr = tile / tiles_x;
        const int x0 = txi * TX, y0 = (rr % tiles_y) * TY;
        const int z0 = (rr / tiles_y) * zc, z1 = min(z0 + zc, NZ);
        const long long nxy = (long long)NX * NY;
        const int oy = FLAT ? 0 : 1;
        // the loads of a plane stay raw in registers until the plane is
        // stored a step later (the update u + du is formed there), so that
        // they are in flight while the step between computes
        // with the compact block, pa holds (C, bb) of the cell and the cell
        // coefficients are formed from C when the plane is stored (bit i of
        // inb: cell i of the ring lies in the grid)
        double2 pu[NLD], pa[NLD];
        V2 pd[NLD], ps[NLD];
        unsigned inb = 0u;
        auto fetch = [&](int z) {
            inb = 0u;
#pragma unroll
            for (int i = 0; i < NLD; i++) {
                const int c = t + i * NT;
                pu[i] = make_double2(0.0, 0.0);
                pa[i] = make_double2(0.0, 0.0);
                pd[i].x = pd[i].y = RV(0);
                ps[i].x = ps[i].y = RV(0);
                const int gx = x0 + c % PX - 1, gy = y0 + c / PX - oy;
                if (c < PS && z >= 0 && z < NZ && gx >= 0 && gx < NX && gy >= 0 && gy < NY) {
                    const long long g = gx + (long long)NX * gy + nxy * z;
                    if (a.src_p) pu[i] = make_double2(a.src_p[g], a.src_T[g]);
                    if (a.src32) ps[i] = a.src32[g];
                    if (a.update) pd[i] = a.du[g];
                    pa[i] = a.cb ? a.cb[g] : a.ac[g];
                    inb |= 1u << i;
                }
            }
        };
        auto store = [&](int z) {
            const int s = z & 3;
#pragma unroll
            for (int i = 0; i < NLD; i++) {
                const int c = t + i * NT;
                if (c < PS) {
                    double2 v = pu[i];
                    if (a.src32) v = make_double2((double)ps[i].x, (double)ps[i].y);
                    if (a.update) {
                        v.x += (double)pd[i].x;
                        v.y += (double)pd[i].y;
                    }
                    su[s][c] = v;
                    double2 w = pa[i];
                    if (a.cb) w = ((inb >> i) & 1u) ? phases_ac(a.rho, a.kc, w.x) : make_double2(0.0, 0.0);
                    sa[s][c] = w;
                }
            }
        };
        // this thread's interior cell
        const int lx = 1 + t % TX, ly = oy + t / TX;
        const int gx = x0 + lx - 1, gy = y0 + ly - oy;
        const bool mine = gx < NX && gy < NY;
        const int c = ly * PX + lx;
        double4 Bn;
        double bpn = 0.0, bTn = 0.0;
        auto fetch_cell = [&](int z) {
            if (mine && z < z1) {
                const long long g = gx + (long long)NX * gy + nxy * z;
                Bn = op_B64_raw(a, g);
                bpn = a.b_p ? a.b_p[g] : 0.0;
                bTn = a.b_T ? a.b_T[g] : 0.0;
            }
        };
        fetch(z0 - 1);
        store(z0 - 1);
        fetch(z0);
        store(z0);
        fetch_cell(z0);
        double4 B = op_B64_fin(a, Bn);
        double bp0 = bpn, bT0 = bTn;
        fetch(z0 + 1);
        for (int k = z0; k < z1; k++) {
            store(k + 1);
            fetch(k + 2);
            fetch_cell(k + 1);
            __syncthreads();
            if (mine) {
                const int s = k & 3, sm = (k + 3) & 3, sp = (k + 1) & 3;
                const double2 um = su[s][c];
                const double2 am = sa[s][c];
                double nbp = 0.0, nbT = 0.0, Sp = 0.0, ST = 0.0;
                // mr: the r-z metric of a radial (marching-axis, 2-D) face
                auto nb = [&](int ss, int q, int mr = -1) {
                    double2 w = harm2_exact(am, sa[ss][q]);
                    if (FLAT && mr >= 0 && a.axm) axi_face(w, a.axm[k], mr == 1);
                    w.x *= a.inv_h2;
                    w.y *= a.inv_h2;
                    const double2 uq = su[ss][q];
                    Sp += w.x;
                    ST += w.y;
                    nbp += w.x * uq.x;
                    nbT += w.y * uq.y;
                };
                nb(s, c - 1);
                nb(s, c + 1);
                if (!FLAT) {
                    nb(s, c - PX);
                    nb(s, c + PX);
                }
                nb(sm, c, 0);
                nb(sp, c, 1);
                const double Lp = Sp * um.x - nbp;   // -div(a_p grad p)
                const double LT = ST * um.y - nbT;   // -div(a_T grad T)
                double bp = bp0, bT = bT0;
                outer_b(a, bp, bT);
                double resp, resT, rp, rT;
                if (a.phases) {
                    const double l1 = -B.w, l2 = -B.z, l4 = B.y / l1, l3 = -B.x + l4 * l2;
                    resT = bT - (-LT + l1 * um.y + l2 * um.x);
                    resp = bp - (-Lp + l3 * um.x + l4 * (-LT));
                    rT = -resT;
                    rp = fmadd(l4, resT, -resp);
                } else {
                    rp = bp - (Lp + B.x * um.x + B.y * um.y);
                    rT = bT - (LT + B.z * um.x + B.w * um.y);
                    resp = rp;
                    resT = rT;
                }
                const long long g = gx + (long long)NX * gy + nxy * k;
                if (a.update) {
                    if (a.dst32) {
                        V2 o;   // exact: the iterate is the correction itself
                        o.x = (RV)um.x;
                        o.y = (RV)um.y;
                        a.dst32[g] = o;
                    } else {
                        a.dst_p[g] = um.x;
                        a.dst_T[g] = um.y;
                    }
                }
                outer_out(a, g, resp, resT, rp, rT, bp, bT, acc);
            }
            B = op_B64_fin(a, Bn);
            bp0 = bpn;
            bT0 = bTn;
        }
    }
    block_reduce_store(acc, 4, a.partials + 4ll * blockIdx.x);
}

// The outer residual of a zero iterate (the first of a solve from a zero
// guess): the residual is b itself, so no stencil is applied; each thread
// walks the column of cells that is its own in k_outer_zm (the same
// blocks, tiles and z order), so that the partial sums, and with them the
// norms, are those of k_outer_zm bit for bit.  The block enters through
// l4 = B_pT / (-B_TT) alone (compact block: (C, bb) without T).
template <int DIM, typename RV, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void k_outer_zg(OuterArgs<RV> a, int NX, int NY, int NZ,
                                                     int zc, int tiles_x, int tiles_y, int ntiles)
{
    if (gated(a.gate)) return;
    constexpr int U = 4;   // cells whose loads are in flight together
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int t = threadIdx.x;
    if (tile < ntiles) {
        const int txi = tile % tiles_x;
        const int rr = tile / tiles_x;
        const int x0 = txi * TX, y0 = (rr % tiles_y) * TY;
        const int z0 = (rr / tiles_y) * zc, z1 = min(z0 + zc, NZ);
        const long long nxy = (long long)NX * NY;
        const int gx = x0 + t % TX, gy = y0 + t / TX;
        if (gx < NX && gy < NY) {
            const long long g0 = gx + (long long)NX * gy;
            for (int kb = z0; kb < z1; kb += U) {
                double2 cb[U];
                double4 Bs[U];
                double bps[U], bTs[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    if (kb + u < z1) {
                        const long long g = g0 + nxy * (kb + u);
                        if (a.phases) {
                            if (a.cb) cb[u] = a.cb[g];
                            else Bs[u] = a.B[g];
                        }
                        bps[u] = a.b_p ? a.b_p[g] : 0.0;
                        bTs[u] = a.b_T ? a.b_T[g] : 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; u++) {
                    if (kb + u < z1) {
                        double bp = bps[u], bT = bTs[u];
                        outer_b(a, bp, bT);
                        double rp, rT;
                        if (a.phases) {
                            const double4 B = a.cb ? compact_B(a.k, cb[u].x, cb[u].y, 0.0) : Bs[u];
                            const double l1 = -B.w, l4 = B.y / l1;
                            rT = -bT;
                            rp = fmadd(l4, bT, -bp);
                        } else {
                            rp = bp;
                            rT = bT;
                        }
                        outer_out(a, g0 + nxy * (kb + u), bp, bT, rp, rT, bp, bT, acc);
                    }
                }
            }
        }
    }
    block_reduce_store(acc, 4, a.partials + 4ll * blockIdx.x);
}

// Launch geometry of the plane-marching outer residual (shared with the
// host's partial-sum sizing).
struct ZmGeom {
    int NX, NY, NZ, tx, ty, zc, nt;
};

static ZmGeom outer_geom(int dim, int nx, int ny, int nz)
{
    ZmGeom g;
    if (dim == 3) {
        g.NX = nx; g.NY = ny; g.NZ = nz;
        g.tx = (nx + 63) / 64;
        g.ty = (ny + 3) / 4;
    } else {
        g.NX = nx; g.NY = 1; g.NZ = ny;
        g.tx = (nx + 255) / 256;
        g.ty = 1;
    }
    g.zc = g.NZ;
    while (g.zc > 8 && (long long)g.tx * g.ty * ((g.NZ + g.zc - 1) / g.zc) < 2048)
        g.zc = (g.zc + 1) / 2;
    g.nt = g.tx * g.ty * ((g.NZ + g.zc - 1) / g.zc);
    return g;
}

int outer_zm_blocks(int dim, int nx, int ny, int nz) { return outer_geom(dim, nx, ny, nz).nt; }

template <typename RV>
int launch_outer_zm(int dim, const OuterArgs<RV> &a, hipStream_t s)
{
    const ZmGeom g = outer_geom(dim, a.nx, a.ny, a.nz);
    if (!a.src_p && !a.src32 && !a.update) {
        // a zero iterate: the residual is b (same blocks and partials)
        if (dim == 3)
            hipLaunchKernelGGL((k_outer_zg<3, RV, 64, 4>), dim3(g.nt), dim3(256), 0, s, a, g.NX,
                               g.NY, g.NZ, g.zc, g.tx, g.ty, g.nt);
        else
            hipLaunchKernelGGL((k_outer_zg<2, RV, 256, 1>), dim3(g.nt), dim3(256), 0, s, a, g.NX,
                               g.NY, g.NZ, g.zc, g.tx, g.ty, g.nt);
        return g.nt;
    }
    if (dim == 3)
        hipLaunchKernelGGL((k_outer_zm<3, RV, 64, 4>), dim3(g.nt), dim3(256), 0, s, a, g.NX, g.NY,
                           g.NZ, g.zc, g.tx, g.ty, g.nt);
    else
        hipLaunchKernelGGL((k_outer_zm<2, RV, 256, 1>), dim3(g.nt), dim3(256), 0, s, a, g.NX, g.NY,
                           g.NZ, g.zc, g.tx, g.ty, g.nt);
    return g.nt;
}
template int launch_outer_zm<float>(int, const OuterArgs<float> &, hipStream_t);
template int launch_outer_zm<double>(int, const OuterArgs<double> &, hipStream_t);

// Residual f - A u and its restriction (mean of the 2^d children) to the
// coarse right-hand side, plane-marching like k_outer_zm: the finest grid
// (cell coefficients in the ring) or, FACES, a coarse level (each cell's
// six stored faces read with its f and block).  Coarse plane K collects
// fine planes 2K and 2K+1, so chunks start on even planes; the 2x2 (2-D:
// 2) in-plane sums go through LDS.  Faces and children are summed in the
// order of restrict_cell (zero faces and zero neighbours past the
// boundary add nothing), so the coarse levels' result is k_restrict's bit
// for bit.
template <typename R, int TX, int TY, bool FACES>
__global__ __launch_bounds__(TX *TY) void k_restrict_zm(Lvl<R> F, Lvl<R> C, int NX, int NY, int NZ,
                                                        int zc, int tiles_x, int tiles_y,
                                                        int ntiles)
{
    if (gated(F.gate)) return;
    using V2 = typename VT<R>::v2;
    using V4 = typename VT<R>::v4;
    constexpr bool FLAT = Flat<TY>::v;
    constexpr int NT = TX * TY;
    constexpr int PX = TX + 2, PY = FLAT ? 1 : TY + 2, PS = PX * PY;
    constexpr int NLD = (PS + NT - 1) / NT;
    constexpr int CX = TX / 2, CY = FLAT ? 1 : TY / 2;
    __shared__ V2 su[4][PS];
    __shared__ V2 sa[FACES ? 1 : 4][FACES ? 1 : PS];
    __shared__ V2 sr[NT];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int t = threadIdx.x;
    const int txi = tile % tiles_x;
    const int rr = tile / tiles_x;
    const int x0 = txi * TX, y0 = (rr % tiles_y) * TY;
    const int z0 = (rr / tiles_y) * zc, z1 = min(z0 + zc, NZ);
    const long long nxy = (long long)NX * NY;
    const int oy = FLAT ? 0 : 1;
    const R ih2 = (R)F.inv_h2;
    V2 pu[NLD], pa[NLD];
    auto fetch = [&](int z) {
#pragma unroll
        for (int i = 0; i < NLD; i++) {
            const int c = t + i * NT;
            pu[i].x = pu[i].y = R(0);
            pa[i].x = pa[i].y = R(0);
            const int gx = x0 + c % PX - 1, gy = y0 + c / PX - oy;
            if (c < PS && z >= 0 && z < NZ && gx >= 0 && gx < NX && gy >= 0 && gy < NY) {
                const long long g = gx + (long long)NX * gy + nxy * z;
                pu[i] = F.u[g];
                if (!FACES) pa[i] = cell_ac(F, g);
            }
        }
    };
    auto store = [&](int z) {
        const int s = z & 3;
#pragma unroll
        for (int i = 0; i < NLD; i++) {
            const int c = t + i * NT;
            if (c < PS) {
                su[s][c] = pu[i];
                if (!FACES) sa[s][c] = pa[i];
            }
        }
    };
    const int lx = 1 + t % TX, ly = oy + t / TX;
    const int gx = x0 + lx - 1, gy = y0 + ly - oy;
    const bool mine = gx < NX && gy < NY;
    const int c = ly * PX + lx;
    V2 fn;
    V4 Bn;
    V2 wn[6], w6[6];   // FACES: the cell's faces x-, x+, y-, y+, z-, z+
    auto fetch_cell = [&](int z) {
        if (mine && z < z1) {
            const long long g = gx + (long long)NX * gy + nxy * z;
            fn = F.f[g];
            Bn = sweep_B_raw(F, g);
            if (FACES) {
#pragma unroll
                for (int q = 0; q < 6; q++) wn[q].x = wn[q].y = R(0);
                wn[0] = F.fx[g];
                if (gx + 1 < NX) wn[1] = F.fx[g + 1];
                wn[2] = F.fy[g];
                if (gy + 1 < NY) wn[3] = F.fy[g + NX];
                wn[4] = F.fz[g];
                if (z + 1 < NZ) wn[5] = F.fz[g + nxy];
            }
        }
    };
    // coarse cell of this thread (t < CX * CY)
    const int cxl = t % CX, cyl = t / CX;
    const int CNX = NX / 2, CNY = FLAT ? 1 : NY / 2;
    const int gcx = x0 / 2 + cxl, gcy = FLAT ? 0 : y0 / 2 + cyl;
    const bool cmine = t < CX * CY && gcx < CNX && gcy < CNY;
    R accp = R(0), accT = R(0);

    fetch(z0 - 1);
    store(z0 - 1);
    fetch(z0);
    store(z0);
    fetch_cell(z0);
    V2 f = fn;
    V4 B = sweep_B_fin(F, Bn);
    if (FACES) {
#pragma unroll
        for (int q = 0; q < 6; q++) w6[q] = wn[q];
    }
    fetch(z0 + 1);
    for (int k = z0; k < z1; k++) {
        store(k + 1);
        fetch(k + 2);
        fetch_cell(k + 1);
        __syncthreads();
        V2 r;
        r.x = r.y = R(0);
        if (mine) {
            const int s = k & 3, sm = (k + 3) & 3, sp = (k + 1) & 3;
            const V2 um = su[s][c];
            V2 am;
            if constexpr (!FACES) am = sa[s][c];
            R nbp = R(0), nbT = R(0), Sp = R(0), ST = R(0);
            // mr: the r-z metric of a radial (marching-axis, 2-D) face
            int nf = 0;
            auto nb = [&](int ss, int q, int mr) {
                V2 w;
                if constexpr (FACES) w = w6[nf++];
                else w = harm2(am, sa[ss][q]);
                if (FLAT && mr >= 0 && F.axm) axi_face(w, F.axm[k], mr == 1);
                const R wp = w.x * ih2, wT = w.y * ih2;
                const V2 uq = su[ss][q];
                Sp += wp;
                ST += wT;
                nbp += wp * uq.x;
                nbT += wT * uq.y;
            };
            nb(s, c - 1, -1);
            nb(s, c + 1, -1);
            if (!FLAT) {
                nb(s, c - PX, -1);
                nb(s, c + PX, -1);
            }
            nb(sm, c, 0);
            nb(sp, c, 1);
            const R Ap = Sp * um.x - nbp + B.x * um.x + B.y * um.y;
            const R AT = ST * um.y - nbT + B.z * um.x + B.w * um.y;
            r.x = f.x - Ap;
            r.y = f.y - AT;
        }
        sr[t] = r;
        __syncthreads();
        if (cmine) {
            // children (2 cxl + a, 2 cyl + b) of the tile, in x then y order
            const int base = 2 * cyl * TX + 2 * cxl;
            const V2 r00 = sr[base], r10 = sr[base + 1];
            if (FLAT && F.axm) {
                // r-z: the row's pair weighted by its cell radius
                const R rc = F.axm[k].z;
                accp = fmadd(r00.x + r10.x, rc, accp);
                accT = fmadd(r00.y + r10.y, rc, accT);
            } else if (FACES) {
                // one child after the other, as restrict_cell
                const V2 r01 = sr[base + TX], r11 = sr[base + TX + 1];
                accp = accp + r00.x;
                accp = accp + r10.x;
                accp = accp + r01.x;
                accp = accp + r11.x;
                accT = accT + r00.y;
                accT = accT + r10.y;
                accT = accT + r01.y;
                accT = accT + r11.y;
            } else {
                R sp_ = r00.x + r10.x, sT_ = r00.y + r10.y;
                if (!FLAT) {
                    const V2 r01 = sr[base + TX], r11 = sr[base + TX + 1];
                    sp_ += r01.x + r11.x;
                    sT_ += r01.y + r11.y;
                }
                accp += sp_;
                accT += sT_;
            }
            if (k & 1) {
                const R sc = FACES ? R(1) / R(8) : (FLAT ? R(0.25) : R(0.125));
                V2 o;
                o.x = accp * sc;
                o.y = accT * sc;
                C.f[gcx + (long long)CNX * gcy + (long long)CNX * CNY * (k >> 1)] = o;
                accp = accT = R(0);
            }
        }
        f = fn;
        B = sweep_B_fin(F, Bn);
        if (FACES) {
#pragma unroll
            for (int q = 0; q < 6; q++) w6[q] = wn[q];
        }
    }
}

// faces: a 3-D coarse level (stored faces)
template <typename R>
void launch_restrict_zm(int dim, const Lvl<R> &F, const Lvl<R> &C, hipStream_t s, bool faces)
{
    int NX, NY, NZ, tx, ty;
    if (dim == 3) {
        NX = F.nx; NY = F.ny; NZ = F.nz;
        tx = (NX + 63) / 64;
        ty = (NY + 3) / 4;
    } else {
        NX = F.nx; NY = 1; NZ = F.ny;
        tx = (NX + 255) / 256;
        ty = 1;
    }
    int zc = NZ;   // even (the grid coarsens), kept even below
    while (zc > 8 && (long long)tx * ty * ((NZ + zc - 1) / zc) < 2048) zc = ((zc + 1) / 2 + 1) & ~1;
    const int nt = tx * ty * ((NZ + zc - 1) / zc);
    if (dim == 3 && faces)
        hipLaunchKernelGGL((k_restrict_zm<R, 64, 4, true>), dim3(nt), dim3(256), 0, s, F, C, NX, NY,
                           NZ, zc, tx, ty, nt);
    else if (dim == 3)
        hipLaunchKernelGGL((k_restrict_zm<R, 64, 4, false>), dim3(nt), dim3(256), 0, s, F, C, NX, NY,
                           NZ, zc, tx, ty, nt);
    else
        hipLaunchKernelGGL((k_restrict_zm<R, 256, 1, false>), dim3(nt), dim3(256), 0, s, F, C, NX,
                           NY, NZ, zc, tx, ty, nt);
}
template void launch_restrict_zm<float>(int, const Lvl<float> &, const Lvl<float> &, hipStream_t,
                                        bool);
template void launch_restrict_zm<double>(int, const Lvl<double> &, const Lvl<double> &, hipStream_t,
                                         bool);

}  // namespace ptmg

namespace ptmg {

// ------------------------------------------------- single-block tail cycle
// The V-cycle of the coarsest few levels (all with stored faces) in one
// block of 1024 threads, every array in LDS: these levels have tens to a
// few thousand cells, so as separate kernels they are bound by launch
// latency.  Same steps and arithmetic as the grid kernels (the same cell
// functions): red-black sweeps (zero guess on the first red pass),
// residual + restriction, the FP64 inverse on the coarsest grid (matrix
// read from global memory), prolongation + correction.  Input: f of the
// first tail level; output: its u.  The level loops are unrolled over
// kMaxTail (guarded by nl) so that every per-level constant is a static
// kernel argument and every level view is built from the LDS base.
template <int DIM>
__device__ __forceinline__ void decode32(int e, int nx, int ny, int &i, int &j, int &k)
{
    const int r = e / nx;
    i = e - r * nx;
    if (DIM == 2) {
        j = r;
        k = 0;
    } else {
        k = r / ny;
        j = r - k * ny;
    }
}

template <typename R, int DIM>
__global__ __launch_bounds__(DIM == 3 ? 512 : 1024) void k_tail(TailArgs<R> A)
{
    if (gated(A.g[0].gate)) return;
    using V2 = typename VT<R>::v2;
    using V4 = typename VT<R>::v4;
    extern __shared__ __align__(16) unsigned char lds[];
    // 3-D tails start at 8^3 cells or fewer (LDS), and half the threads
    // leave each twice the registers
    constexpr int NT = DIM == 3 ? 512 : 1024;
    const int t = threadIdx.x;
    const int nl = A.nl;
    auto view = [&](int q) {
        Lvl<R> v = A.g[q];
        v.u = (V2 *)(lds + A.off[q][0]);
        v.f = (V2 *)(lds + A.off[q][1]);
        v.fx = (const V2 *)(lds + A.off[q][2]);
        v.fy = (const V2 *)(lds + A.off[q][3]);
        v.fz = DIM == 3 ? (const V2 *)(lds + A.off[q][4]) : nullptr;
        v.B = (const V4 *)(lds + A.off[q][5]);
        return v;
    };
    // operators of every tail level, the right-hand side of the first and
    // the coarsest inverse.  Element t of five levels at a time is loaded
    // unconditionally (level and index clamped into range) before any is
    // stored, so a round costs one memory latency rather than one per
    // level; larger arrays loop on.
    {
        struct Cell {
            R fx0, fx1, fy0, fy1, fz0, fz1, f0, f1, b0, b1, b2, b3;
        };
        // a level past the last reads element 0 of level 0 (static indices
        // only: a dynamic one would copy A to scratch)
        auto ld = [&](int q) {
            const bool ok = q < nl;
            const int qq = q < kMaxTail ? q : 0;
            const V2 *gfx = ok ? A.g[qq].fx : A.g[0].fx;
            const V2 *gfy = ok ? A.g[qq].fy : A.g[0].fy;
            const V2 *gfz = ok ? A.g[qq].fz : A.g[0].fz;
            const V4 *gB = ok ? A.g[qq].B : A.g[0].B;
            const int e = ok ? min(t, (int)A.g[qq].N - 1) : 0;
            Cell c;
            const V2 a = gfx[e], b = gfy[e];
            const V4 B = gB[e];
            c.fx0 = a.x; c.fx1 = a.y;
            c.fy0 = b.x; c.fy1 = b.y;
            c.fz0 = c.fz1 = R(0);
            if (DIM == 3) {
                const V2 z = gfz[e];
                c.fz0 = z.x; c.fz1 = z.y;
            }
            c.b0 = B.x; c.b1 = B.y; c.b2 = B.z; c.b3 = B.w;
            c.f0 = c.f1 = R(0);
            if (q == 0) {
                const V2 f = A.g[0].f[e];
                c.f0 = f.x; c.f1 = f.y;
            }
            return c;
        };
        auto st = [&](int q, const Cell &c) {
            if (q >= nl || q >= kMaxTail || t >= (int)A.g[q < kMaxTail ? q : 0].N) return;
            const Lvl<R> V = view(q);
            V2 v;
            v.x = c.fx0; v.y = c.fx1;
            ((V2 *)V.fx)[t] = v;
            v.x = c.fy0; v.y = c.fy1;
            ((V2 *)V.fy)[t] = v;
            if (DIM == 3) {
                v.x = c.fz0; v.y = c.fz1;
                ((V2 *)V.fz)[t] = v;
            }
            V4 B;
            B.x = c.b0; B.y = c.b1; B.z = c.b2; B.w = c.b3;
            ((V4 *)V.B)[t] = B;
            if (q == 0) {
                v.x = c.f0; v.y = c.f1;
                V.f[t] = v;
            }
        };
        const double ainv = A.ainv_off >= 0 ? A.Ainv[min(t, A.m * A.m - 1)] : 0.0;
#pragma unroll
        for (int q0 = 0; q0 < kMaxTail; q0 += 5) {
            if (q0 >= nl) break;
            const Cell c0 = ld(q0), c1 = ld(q0 + 1), c2 = ld(q0 + 2), c3 = ld(q0 + 3),
                       c4 = ld(q0 + 4);
            st(q0, c0);
            st(q0 + 1, c1);
            st(q0 + 2, c2);
            st(q0 + 3, c3);
            st(q0 + 4, c4);
        }
        if (A.ainv_off >= 0 && t < A.m * A.m) ((double *)(lds + A.ainv_off))[t] = ainv;
    }
#pragma unroll
    for (int q = 0; q < kMaxTail; q++) {
        if (q >= nl) break;
        const Lvl<R> &G = A.g[q];
        const Lvl<R> V = view(q);
        for (int e = t + NT; e < (int)G.N; e += NT) {
            ((V2 *)V.fx)[e] = G.fx[e];
            ((V2 *)V.fy)[e] = G.fy[e];
            if (DIM == 3) ((V2 *)V.fz)[e] = G.fz[e];
            ((V4 *)V.B)[e] = G.B[e];
            if (q == 0) V.f[e] = G.f[e];
        }
    }
    if (A.ainv_off >= 0)
        for (int e = t + NT; e < A.m * A.m; e += NT)
            ((double *)(lds + A.ainv_off))[e] = A.Ainv[e];
    // Sizes and LDS offsets of every level, staged in LDS so that the level
    // loops below run over a dynamic level index with one copy of each
    // phase's code.  Unrolled over the levels, the kernel grows past the
    // instruction cache, and the single block then stalls on instruction
    // fetches at every phase.
    __shared__ int smeta[kMaxTail][10];
    __shared__ double sih2[kMaxTail];
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < kMaxTail; q++) {
            smeta[q][0] = A.g[q].nx;
            smeta[q][1] = A.g[q].ny;
            smeta[q][2] = A.g[q].nz;
            smeta[q][3] = (int)A.g[q].N;
#pragma unroll
            for (int i = 0; i < 6; i++) smeta[q][4 + i] = A.off[q][i];
            sih2[q] = A.g[q].inv_h2;
        }
    }
    __syncthreads();
    // the LDS view of level q (face levels: no cell coefficients, no r-z
    // metric)
    auto lview = [&](int q) {
        Lvl<R> v;
        v.nx = smeta[q][0];
        v.ny = smeta[q][1];
        v.nz = smeta[q][2];
        v.N = smeta[q][3];
        v.inv_h2 = sih2[q];
        v.ac = nullptr;
        v.axm = nullptr;
        v.cb = nullptr;                 // stored faces and block
        v.T0 = nullptr;
        v.tmask = 0;
        v.gate = nullptr;               // the launch checked it at entry
        v.omega = R(1);
        v.u = (V2 *)(lds + smeta[q][4]);
        v.f = (V2 *)(lds + smeta[q][5]);
        v.fx = (const V2 *)(lds + smeta[q][6]);
        v.fy = (const V2 *)(lds + smeta[q][7]);
        v.fz = DIM == 3 ? (const V2 *)(lds + smeta[q][8]) : nullptr;
        v.B = (const V4 *)(lds + smeta[q][9]);
        return v;
    };
    // Levels of at most 64 cells run in wavefront 0 alone: its lanes
    // exchange values through LDS in program order, so a wavefront-scope
    // fence replaces the block barrier between phases.
    int w0 = nl;   // first level of the wavefront part
#pragma unroll
    for (int q = kMaxTail - 1; q >= 0; q--)
        if (q < nl && A.g[q].N <= 64) w0 = q;
    auto sync = [&](bool wave) {
        if (wave) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        } else {
            __syncthreads();
        }
    };
    // one colour of a sweep: cells of colour c enumerated directly when nx
    // is even (half the index space), else by test
    auto colour = [&](const Lvl<R> &V, int c, bool zero_guess, bool wave) {
        const int N = (int)V.N, stride = wave ? 64 : NT;
        if ((V.nx & 1) == 0) {
            const int hx = V.nx >> 1, NH = N >> 1;
            for (int e2 = t; e2 < NH; e2 += stride) {
                const int row = e2 / hx, ii = e2 - row * hx;
                const int k = DIM == 2 ? 0 : row / V.ny;
                const int j = DIM == 2 ? row : row - k * V.ny;
                const int i = 2 * ii + ((j + k + c) & 1);
                const int me = i + V.nx * row;
                if (zero_guess) rb_cell<R, DIM, false, false>(V, i, j, k, me);
                else rb_cell<R, DIM, false, true>(V, i, j, k, me);
            }
        } else {
            for (int e = t; e < N; e += stride) {
                int i, j, k;
                decode32<DIM>(e, V.nx, V.ny, i, j, k);
                if (((i + j + k) & 1) != c) continue;
                if (zero_guess) rb_cell<R, DIM, false, false>(V, i, j, k, e);
                else rb_cell<R, DIM, false, true>(V, i, j, k, e);
            }
        }
        sync(wave);
    };
    // down on level q: smoothing from a zero guess, residual restricted
    auto down = [&](int q, bool wave) {
        const Lvl<R> V = lview(q), C = lview(q + 1);
        const int stride = wave ? 64 : NT;
        if (A.nu1 == 0) {
            for (int e = t; e < (int)V.N; e += stride) {
                V2 z;
                z.x = z.y = R(0);
                V.u[e] = z;
            }
            sync(wave);
        }
        for (int s = 0; s < A.nu1; s++) {
            colour(V, 0, s == 0, wave);
            colour(V, 1, false, wave);
        }
        for (int e = t; e < (int)C.N; e += stride) {
            int I, J, K;
            decode32<DIM>(e, C.nx, C.ny, I, J, K);
            restrict_cell<R, DIM, false>(V, C, I, J, K, e);
        }
        sync(wave);
    };
    // up on level q: prolongation + correction, then smoothing
    auto up = [&](int q, bool wave) {
        const Lvl<R> V = lview(q), C = lview(q + 1);
        const int stride = wave ? 64 : NT;
        for (int e = t; e < (int)V.N; e += stride) {
            int i, j, k;
            decode32<DIM>(e, V.nx, V.ny, i, j, k);
            prolong_cell<R, DIM>(V, C, i, j, k, e);
        }
        sync(wave);
        for (int s = 0; s < A.nu2; s++) {
            colour(V, 0, false, wave);
            colour(V, 1, false, wave);
        }
    };
    // coarsest grid: u = Ainv f in FP64.  Row sums in the order of the grid
    // kernel k_coarse_apply (a 64-lane butterfly over lane-strided partial
    // sums); for m <= 64 the products sit in groups of G = 2^ceil(log2 m)
    // lanes, 64 / G rows at a time, and the butterfly's first steps, which
    // only add zeros, are skipped.
    auto coarsest = [&](int q, bool wave) {
        const Lvl<R> C = lview(q);
        const R *f = (const R *)C.f;
        R *u = (R *)C.u;
        const int lane = t & 63, wv = t >> 6;
        const int nw = wave ? 1 : NT / 64;
        const int m = A.m;
        const double *Ainv_l = (const double *)(lds + (A.ainv_off >= 0 ? A.ainv_off : 0));
        if (m <= 64) {
            int G = 1;
            while (G < m) G <<= 1;
            const int rpp = 64 / G;
            const int c = lane & (G - 1);
            for (int row0 = wv * rpp; row0 < m; row0 += nw * rpp) {
                const int row = row0 + lane / G;
                double x = 0.0;
                if (row < m && c < m) {
                    const double a = A.ainv_off >= 0 ? Ainv_l[row * m + c]
                                                     : A.Ainv[(long long)row * m + c];
                    x += a * (double)f[c];
                }
                for (int off = G >> 1; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
                if (c == 0 && row < m) u[row] = (R)x;
            }
        } else {
            for (int row = wv; row < m; row += nw) {
                const double *a = A.Ainv + (long long)row * m;
                double sacc = 0.0;
                for (int c = lane; c < m; c += 64) sacc += a[c] * (double)f[c];
                for (int off = 32; off >= 1; off >>= 1) sacc += __shfl_xor(sacc, off, 64);
                if (lane == 0) u[row] = (R)sacc;
            }
        }
        sync(wave);
    };
    // levels 0 .. wb-1 run block-wide on the way down and up, levels
    // wb .. nl-2 in the wavefront part; the coarsest is level nl-1
    const int wb = min(w0, nl - 1);
#pragma unroll 1
    for (int q = 0; q < wb; q++) down(q, false);
    if (wb == nl - 1) {
        coarsest(nl - 1, false);   // no wavefront part: the coarsest block-wide
    } else {
        if (t < 64) {
#pragma unroll 1
            for (int q = wb; q < nl - 1; q++) down(q, true);
            coarsest(nl - 1, true);
#pragma unroll 1
            for (int q = nl - 2; q >= wb; q--) up(q, true);
        }
        __syncthreads();
    }
#pragma unroll 1
    for (int q = wb - 1; q >= 0; q--) up(q, false);
    {
        const Lvl<R> V = view(0);
        for (int e = t; e < (int)V.N; e += NT) A.g[0].u[e] = V.u[e];
    }
}

template <typename R>
size_t tail_level_lds(int dim, long long N)
{
    // u, f, faces (dim), block; each array 16-byte aligned
    auto al = [](size_t b) { return (b + 15) & ~size_t(15); };
    const size_t v2 = al(2 * sizeof(R) * N), v4 = al(4 * sizeof(R) * N);
    return v2 * (2 + dim) + v4;
}
template size_t tail_level_lds<float>(int, long long);
template size_t tail_level_lds<double>(int, long long);

template <typename R>
bool launch_tail(int dim, const TailArgs<R> &a, size_t lds_bytes, hipStream_t s)
{
    if (dim == 3)
        hipLaunchKernelGGL((k_tail<R, 3>), dim3(1), dim3(512), lds_bytes, s, a);
    else
        hipLaunchKernelGGL((k_tail<R, 2>), dim3(1), dim3(1024), lds_bytes, s, a);
    return true;
}
template bool launch_tail<float>(int, const TailArgs<float> &, size_t, hipStream_t);
template bool launch_tail<double>(int, const TailArgs<double> &, size_t, hipStream_t);

template <typename R>
void tail_set_lds_limit(int dim, size_t bytes)
{
    // the limit belongs to the kernel, shared by every handle of the
    // process: it only grows, so no handle's tail is left without its LDS
    static std::mutex mu;
    static size_t granted[2] = {0, 0};
    std::lock_guard<std::mutex> lock(mu);
    size_t &g = granted[dim == 3 ? 1 : 0];
    if (bytes <= g) return;
    g = bytes;
    if (dim == 3)
        (void)hipFuncSetAttribute((const void *)k_tail<R, 3>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    else
        (void)hipFuncSetAttribute((const void *)k_tail<R, 2>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
template void tail_set_lds_limit<float>(int, size_t);
template void tail_set_lds_limit<double>(int, size_t);

}  // namespace ptmg

namespace ptmg {

// ------------------------------------------------ end of the step
// Velocity correction and phase energies in one plane-marching pass: a
// 4-slot LDS ring of planes (tile + a ring of one cell) holds (p, T),
// (1/rho, k) and (C, sigma kappa), so every cell array is read from HBM
// once; each cell recomputes the corrected velocity of its 2*DIM faces
// (the expression is the same in both cells that share a face) and writes
// the lower ones (and the upper wall face at the end of an axis).  A 2-D
// grid marches along y with 1-row planes.
template <int DIM, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void k_down_zm(DownArgs a, int NX, int NY, int NZ, int zc,
                                                    int tiles_x, int tiles_y, int ntiles)
{
    constexpr bool FLAT = DIM == 2;
    constexpr int NT = TX * TY;
    constexpr int PX = TX + 2, PY = FLAT ? 1 : TY + 2, PS = PX * PY;
    constexpr int NLD = (PS + NT - 1) / NT;
    __shared__ double2 sq[4][PS];   // (p, T)
    __shared__ double2 sa[4][PS];   // (1/rho, k)
    __shared__ double2 sc[4][PS];   // (C, sigma kappa)
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;     // whole block: no barrier is skipped by part of it
    const int t = threadIdx.x;
    const int txi = tile % tiles_x;
    const int rr = tile / tiles_x;
    const int x0 = txi * TX, y0 = (rr % tiles_y) * TY;
    const int z0 = (rr / tiles_y) * zc, z1 = min(z0 + zc, NZ);
    const long long nxy = (long long)NX * NY;
    const int oy = FLAT ? 0 : 1;
    const double *Um = FLAT ? a.Uy : a.Uz;   // faces across the marching axis
    double *Vm = FLAT ? a.Vy : a.Vz;
    const double *um = FLAT ? a.uy : a.uz;
    double *vm = FLAT ? a.vy : a.vz;
    const bool cellv = a.ux != nullptr;
    const bool energy = a.E1a != nullptr;

    double2 pq[NLD], pa[NLD], pc[NLD];
    auto fetch = [&](int z) {
#pragma unroll
        for (int i = 0; i < NLD; i++) {
            const int c = t + i * NT;
            pq[i] = make_double2(0.0, 0.0);
            pa[i] = make_double2(0.0, 0.0);
            pc[i] = make_double2(0.0, 0.0);
            const int gx = x0 + c % PX - 1, gy = y0 + c / PX - oy;
            if (c < PS && z >= 0 && z < NZ && gx >= 0 && gx < NX && gy >= 0 && gy < NY) {
                const long long g = gx + (long long)NX * gy + nxy * z;
                pq[i] = make_double2(a.p[g], a.T[g]);
                pa[i] = a.ac[g];
                pc[i] = make_double2(a.C[g], a.kappa ? a.sigma * a.kappa[g] : 0.0);
            }
        }
    };
    auto store = [&](int z) {
        const int s = z & 3;
#pragma unroll
        for (int i = 0; i < NLD; i++) {
            const int c = t + i * NT;
            if (c < PS) {
                sq[s][c] = pq[i];
                sa[s][c] = pa[i];
                sc[s][c] = pc[i];
            }
        }
    };
    // this thread's cell column
    const int lx = 1 + t % TX, ly = oy + t / TX;
    const int gx = x0 + lx - 1, gy = y0 + ly - oy;
    const bool mine = gx < NX && gy < NY;
    const int c = ly * PX + lx;
    // pointwise inputs of the next cell (prefetched one plane ahead)
    struct CellIn {
        double e1, e2, u0, u1, u2;   // energies, cell velocities (x, in-plane y, march)
        double xl, xh, yl, yh, mh;   // provisional face velocities
    };
    CellIn nx_ = {}, cur;
    auto fetch_cell = [&](int z) {
        if (mine && z < z1) {
            const long long g = gx + (long long)NX * gy + nxy * z;
            if (energy) {
                nx_.e1 = a.E1a[g];
                nx_.e2 = a.E2a[g];
            }
            if (cellv) {
                nx_.u0 = a.ux[g];
                if (!FLAT) nx_.u1 = a.uy[g];
                nx_.u2 = um[g];
            }
            const long long fx = gx + (long long)(NX + 1) * (gy + (long long)NY * z);
            nx_.xl = a.Ux[fx];
            nx_.xh = a.Ux[fx + 1];
            if (!FLAT) {
                const long long fy = gx + (long long)NX * (gy + (long long)(NY + 1) * z);
                nx_.yl = a.Uy[fy];
                nx_.yh = a.Uy[fy + NX];
            }
            nx_.mh = Um[g + nxy];
        }
    };
    double ml = 0.0;   // provisional velocity on the lower face across the marching axis
    if (mine) ml = Um[gx + (long long)NX * gy + nxy * z0];
    fetch(z0 - 1);
    store(z0 - 1);
    fetch(z0);
    store(z0);
    fetch_cell(z0);
    cur = nx_;
    fetch(z0 + 1);
    for (int k = z0; k < z1; k++) {
        store(k + 1);
        fetch(k + 2);
        fetch_cell(k + 1);
        __syncthreads();
        if (mine) {
            const int s = k & 3, sm = (k + 3) & 3, sp = (k + 1) & 3;
            const double2 q = sq[s][c], am = sa[s][c], cm = sc[s][c];
            const double p1c = q.x + (1.0 - cm.x) * cm.y, p2c = q.x - cm.x * cm.y;
            // one face of this cell: corrected velocity, (1/rho) dp/dn, the
            // phase pressures on the face and the heat flux k dT/dn
            struct Face {
                double U, g, P1, P2, q;
            };
            auto face = [&](int ss, int qi, bool inside, bool upper, double Us) {
                Face f;
                if (!inside) {
                    f.U = Us;
                    f.g = 0.0;
                    f.P1 = p1c;
                    f.P2 = p2c;
                    f.q = 0.0;
                    return f;
                }
                const double2 qn = sq[ss][qi], an = sa[ss][qi], cn = sc[ss][qi];
                const double p1n = qn.x + (1.0 - cn.x) * cn.y, p2n = qn.x - cn.x * cn.y;
                if (upper) {
                    f.g = harm_exact(am.x, an.x) * ((qn.x - q.x) * a.inv_h);
                    f.q = harm_exact(am.y, an.y) * ((qn.y - q.y) * a.inv_h);
                    f.P1 = 0.5 * (p1c + p1n);
                    f.P2 = 0.5 * (p2c + p2n);
                } else {
                    f.g = harm_exact(an.x, am.x) * ((q.x - qn.x) * a.inv_h);
                    f.q = harm_exact(an.y, am.y) * ((q.y - qn.y) * a.inv_h);
                    f.P1 = 0.5 * (p1n + p1c);
                    f.P2 = 0.5 * (p2n + p2c);
                }
                f.U = Us - a.dt * f.g;
                return f;
            };
            double w1 = 0.0, w2 = 0.0, qs = 0.0;
            auto axis = [&](const Face &lo, const Face &hi) {
                w1 += (hi.P1 * hi.U - lo.P1 * lo.U) * a.inv_h;
                w2 += (hi.P2 * hi.U - lo.P2 * lo.U) * a.inv_h;
                qs += (hi.q - lo.q) * a.inv_h;
            };
            const long long g = gx + (long long)NX * gy + nxy * k;
            // x
            const Face xlo = face(s, c - 1, gx > 0, false, cur.xl);
            const Face xhi = face(s, c + 1, gx < NX - 1, true, cur.xh);
            axis(xlo, xhi);
            const long long fx = gx + (long long)(NX + 1) * (gy + (long long)NY * k);
            a.Vx[fx] = xlo.U;
            if (gx == NX - 1) a.Vx[fx + 1] = xhi.U;
            if (cellv) a.vx[g] = cur.u0 - a.dt * (0.5 * (xlo.g + xhi.g));
            // in-plane y (3-D)
            if (!FLAT) {
                const Face ylo = face(s, c - PX, gy > 0, false, cur.yl);
                const Face yhi = face(s, c + PX, gy < NY - 1, true, cur.yh);
                axis(ylo, yhi);
                const long long fy = gx + (long long)NX * (gy + (long long)(NY + 1) * k);
                a.Vy[fy] = ylo.U;
                if (gy == NY - 1) a.Vy[fy + NX] = yhi.U;
                if (cellv) a.vy[g] = cur.u1 - a.dt * (0.5 * (ylo.g + yhi.g));
            }
            // marching axis
            const Face mlo = face(sm, c, k > 0, false, ml);
            const Face mhi = face(sp, c, k < NZ - 1, true, cur.mh);
            if (FLAT && a.axm) {
                // r-z: radial flux differences per unit volume
                const double4 mt = a.axm[k];
                w1 += (mt.y * mhi.P1 * mhi.U - mt.x * mlo.P1 * mlo.U) * a.inv_h;
                w2 += (mt.y * mhi.P2 * mhi.U - mt.x * mlo.P2 * mlo.U) * a.inv_h;
                qs += (mt.y * mhi.q - mt.x * mlo.q) * a.inv_h;
            } else {
                axis(mlo, mhi);
            }
            Vm[g] = mlo.U;
            if (k == NZ - 1) Vm[g + nxy] = mhi.U;
            if (cellv) vm[g] = cur.u2 - a.dt * (0.5 * (mlo.g + mhi.g));
            if (energy) {
                const double C = cm.x;
                a.E1[g] = cur.e1 + a.dt * C * (-w1 + qs);
                a.E2[g] = cur.e2 + a.dt * (1.0 - C) * (-w2 + qs);
            }
            ml = cur.mh;
        }
        cur = nx_;
    }
}

void launch_downstream(int dim, const DownArgs &a, hipStream_t s)
{
    const ZmGeom g = outer_geom(dim, a.nx, a.ny, a.nz);
    if (dim == 3)
        hipLaunchKernelGGL((k_down_zm<3, 64, 4>), dim3(g.nt), dim3(256), 0, s, a, g.NX, g.NY,
                           g.NZ, g.zc, g.tx, g.ty, g.nt);
    else
        hipLaunchKernelGGL((k_down_zm<2, 256, 1>), dim3(g.nt), dim3(256), 0, s, a, g.NX, g.NY,
                           g.NZ, g.zc, g.tx, g.ty, g.nt);
}

// Viscous work of the phase energies (Eq. 39): W = div(mu (grad u + grad u^T)
// . u) of the end-of-step velocity, one value per cell, and E_i += dt C_i W
// (the phases share the one-fluid flux, so the total is conservative).
// The normal flux (tau . u)_a on the face between cells L and R across
// axis a takes the face velocity as the normal component and the mean of
// the two cells' velocities for the others; tau_aa = 2 mu (u_a,R -
// u_a,L)/h, tau_ab = mu ((u_b,R - u_b,L)/h + mean over L, R of the centred
// difference of u_a along b, mirrored at a wall); mu the mean of the two
// cells' C mu_1 + (1 - C) mu_2.  Wall faces carry no flux; r-z radial faces
// the metric.  One thread per cell; every face flux is evaluated by the
// same function from the face's own data, so both cells of a face take
// the same value and the fluxes cancel exactly in the sum over the grid.
template <int DIM>
__device__ __forceinline__ double visc_flux(const ViscArgs &a, int ax, int i, int j, int k)
{
    const long long sx = 1, sy = a.nx, sz = (long long)a.nx * a.ny;
    const long long st[3] = {sx, sy, sz};
    const int idx[3] = {i, j, k};
    const int n[3] = {a.nx, a.ny, a.nz};
    const long long R = i + sy * j + sz * k, L = R - st[ax];
    const double *u[3] = {a.ux, a.uy, a.uz};
    const double muL = a.C[L] * a.mu1 + (1.0 - a.C[L]) * a.mu2;
    const double muR = a.C[R] * a.mu1 + (1.0 - a.C[R]) * a.mu2;
    const double mu = 0.5 * (muL + muR);
    double flux = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; b++) {
        const double vR = u[b][R], vL = u[b][L];
        if (b == ax) {
            const double *U = ax == 0 ? a.Ux : (ax == 1 ? a.Uy : a.Uz);
            const long long f = i + (long long)(a.nx + (ax == 0)) *
                                        (j + (long long)(a.ny + (ax == 1)) * k);
            flux += 2.0 * mu * (vR - vL) * a.inv_h * U[f];
        } else {
            // centred differences of u_ax along b at L and R (mirrored at walls)
            const long long lo = idx[b] > 0 ? st[b] : 0, hi = idx[b] < n[b] - 1 ? st[b] : 0;
            const double *w = u[ax];
            const double gR = (w[R + hi] - w[R - lo]) * (0.5 * a.inv_h);
            const double gL = (w[L + hi] - w[L - lo]) * (0.5 * a.inv_h);
            const double tau = mu * ((vR - vL) * a.inv_h + 0.5 * (gL + gR));
            flux += tau * (0.5 * (vL + vR));
        }
    }
    return flux;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_viscous(ViscArgs a)
{
    const long long N = (long long)a.nx * a.ny * a.nz;
    for (long long t = blockIdx.x * 256ll + threadIdx.x; t < N; t += (long long)gridDim.x * 256) {
        int i, j, k;
        decode(t, a.nx, a.ny, i, j, k);
        const int idx[3] = {i, j, k};
        const int n[3] = {a.nx, a.ny, a.nz};
        double W = 0.0;
#pragma unroll
        for (int ax = 0; ax < DIM; ax++) {
            const double lo = idx[ax] > 0 ? visc_flux<DIM>(a, ax, i, j, k) : 0.0;
            double hi = 0.0;
            if (idx[ax] < n[ax] - 1)
                hi = visc_flux<DIM>(a, ax, i + (ax == 0), j + (ax == 1), k + (ax == 2));
            if (DIM == 2 && ax == 1 && a.axm) {
                const double4 m = a.axm[j];
                W += (m.y * hi - m.x * lo) * a.inv_h;
            } else {
                W += (hi - lo) * a.inv_h;
            }
        }
        const double c = a.C[t];
        a.E1[t] += a.dt * c * W;
        a.E2[t] += a.dt * (1.0 - c) * W;
    }
}

void launch_viscous(int dim, const ViscArgs &a, hipStream_t s)
{
    const long long N = (long long)a.nx * a.ny * a.nz;
    const unsigned nb = (unsigned)std::min<long long>((N + 255) / 256, 1 << 20);
    if (dim == 3) hipLaunchKernelGGL(k_viscous<3>, dim3(nb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_viscous<2>, dim3(nb), dim3(256), 0, s, a);
}

__global__ __launch_bounds__(256) void k_divergence(int dim, int nx, int ny, int nz, double inv_h,
                                                    const double *Ux, const double *Uy,
                                                    const double *Uz, const double4 *axm,
                                                    double *div)
{
    const long long N = (long long)nx * ny * nz;
    for (long long t = blockIdx.x * 256ll + threadIdx.x; t < N; t += (long long)gridDim.x * 256) {
        int i, j, k;
        decode(t, nx, ny, i, j, k);
        const long long fx = i + (long long)(nx + 1) * (j + (long long)ny * k);
        const long long fy = i + (long long)nx * (j + (long long)(ny + 1) * k);
        double d = (Ux[fx + 1] - Ux[fx]) * inv_h;
        if (axm) {
            const double4 m = axm[j];
            d += (m.y * Uy[fy + nx] - m.x * Uy[fy]) * inv_h;
        } else {
            d += (Uy[fy + nx] - Uy[fy]) * inv_h;
        }
        if (dim == 3) d += (Uz[t + (long long)nx * ny] - Uz[t]) * inv_h;
        div[t] = d;
    }
}

void launch_divergence(int dim, int nx, int ny, int nz, double inv_h, const double *Ux,
                       const double *Uy, const double *Uz, const double4 *axm, double *div,
                       hipStream_t s)
{
    const long long N = (long long)nx * ny * nz;
    const long long nb = std::min<long long>((N + 255) / 256, 65536);
    hipLaunchKernelGGL(k_divergence, dim3((unsigned)nb), dim3(256), 0, s, dim, nx, ny, nz, inv_h,
                       Ux, Uy, Uz, axm, div);
}

// The r-z metric per row j of the finest grid, in units of h: radial faces
// at r = j (lower) and j + 1 (upper), the cell centre at j + 1/2.
__global__ __launch_bounds__(256) void k_axi_metric(int ny, double4 *m64, float4 *m32)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= ny) return;
    const double rc = (double)j + 0.5;
    double4 m;
    m.x = (double)j / rc;
    m.y = ((double)j + 1.0) / rc;
    m.z = rc;
    m.w = (double)j;
    m64[j] = m;
    if (m32) m32[j] = make_float4((float)m.x, (float)m.y, (float)m.z, (float)m.w);
}

void launch_axi_metric(int ny, double4 *m64, float4 *m32, hipStream_t s)
{
    hipLaunchKernelGGL(k_axi_metric, dim3((ny + 255) / 256), dim3(256), 0, s, ny, m64, m32);
}

}  // namespace ptmg
