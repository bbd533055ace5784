// Host side of libptmg: the C ABI, handle and memory plan, assembly and
// hierarchy set-up, the defect-correction (iterative refinement) driver and
// the V-cycle schedule.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ptmg_internal.h"

using namespace ptmg;

namespace {

thread_local std::string g_thread_err = "no error";

// ------------------------------------------------------------ memory plan
struct LevelPlan {
    int n[3];
    long long N;
    double h;
    size_t o_u, o_u2, o_f, o_ac, o_fx, o_fy, o_fz, o_B;   // o_u2: second iterate buffer
};

struct Plan {
    int dim = 0, prec = 0, nlev = 0, m = 0, nblocks = 0;
    int n[3] = {1, 1, 1};
    long long N = 0;
    LevelPlan lv[kMaxLevels];
    size_t o_ac64, o_B64, o_xp, o_xT, o_partials, o_flags, o_gj0, o_gj1;
    // phases mode: the finest block is kept compact, (C, bb) and T
    bool compact = false;
    size_t o_gate = (size_t)-1;
    size_t o_cb64 = (size_t)-1, o_T64 = (size_t)-1, o_cb32 = (size_t)-1, o_T32 = (size_t)-1;
    size_t o_axm64 = (size_t)-1, o_axm32 = (size_t)-1;   // r-z metric per finest row
    size_t total = 0;
    size_t take(size_t bytes)
    {
        size_t o = total;
        total += (bytes + 255) & ~size_t(255);
        return o;
    }
};

constexpr long long kMaxCoarseCells = 2048;   // coarsest grid solved by a dense inverse

// Coarsen while every active axis is even and its half is at least 2.
bool can_coarsen(int dim, const int *n)
{
    for (int a = 0; a < dim; a++)
        if (n[a] % 2 != 0 || n[a] / 2 < 2) return false;
    return true;
}

const char *plan_problem(const pt_problem *p, int prec, Plan &P)
{
    if (!p) return "problem is NULL";
    if (p->dim != 2 && p->dim != 3) return "dim must be 2 or 3";
    if (prec != PT_PREC_FP64 && prec != PT_PREC_MIXED) return "unknown precision";
    for (int a = 0; a < 3; a++) {
        if (a < p->dim && p->n[a] < 2) return "n[a] must be >= 2 on active axes";
        if (a >= p->dim && p->n[a] != 1) return "n[2] must be 1 in 2-D";
        if (p->n[a] > (1 << 20)) return "grid too large";
    }
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return "h must be positive";
    if (p->axisymmetric != 0 && p->axisymmetric != 1) return "axisymmetric must be 0 or 1";
    if (p->axisymmetric && p->dim != 2) return "the axisymmetric metric needs a 2-D grid";
    if (p->mode != PT_COEF_EXPLICIT && p->mode != PT_COEF_PHASES && p->mode != PT_COEF_STATE)
        return "unknown mode";
    if (p->mode == PT_COEF_STATE) {
        if (!p->C || !p->m1 || !p->m2 || !p->p_adv || !p->T_adv)
            return "state mode needs C, m1, m2, p_adv and T_adv";
        if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return "dt must be positive";
        if (p->mean_constraint) return "mean_constraint only applies to B = 0 (explicit mode)";
        const pt_phase *ph[2] = {&p->liquid, &p->gas};
        for (int q = 0; q < 2; q++) {
            const pt_phase &f = *ph[q];
            if (!(f.k >= 0) || !(f.cp > 0) || !(f.gamma > 0) || !(f.Gamma > 1.0) || !(f.b >= 0))
                return "state-mode phase needs k >= 0, cp > 0, gamma > 0, Gamma > 1, b >= 0";
            if (!(f.beta > 0) && !((f.Gamma - 1.0) * f.cv > 0))
                return "phase needs beta > 0 or (Gamma-1) c_v > 0 for Eq. (10)";
        }
    }
    if (p->mode == PT_COEF_PHASES) {
        if (!p->C) return "phases mode needs C";
        if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return "dt must be positive";
        if (p->mean_constraint) return "mean_constraint only applies to B = 0 (explicit mode)";
        const pt_phase *ph[2] = {&p->liquid, &p->gas};
        for (int q = 0; q < 2; q++) {
            const pt_phase &f = *ph[q];
            if (!(f.rho > 0) || !(f.k >= 0) || !(f.cp > 0) || !(f.c > 0) || !(f.gamma > 0))
                return "phase properties must be positive (k >= 0)";
            if (!(f.beta > 0) && !((f.Gamma - 1.0) * f.cv > 0))
                return "phase needs beta > 0 or (Gamma-1) c_v > 0 for Eq. (10)";
        }
    }
    P = Plan();
    P.dim = p->dim;
    P.prec = prec;
    for (int a = 0; a < 3; a++) P.n[a] = p->n[a];
    P.N = (long long)p->n[0] * p->n[1] * p->n[2];
    const size_t R = prec == PT_PREC_MIXED ? 4 : 8;
    // finest grid FP64 operator: cell coefficients and the block (phases
    // mode in mixed precision: compact, (C, bb) and T, in both precisions;
    // the FP64 sweeps of an FP64 V-cycle are faster with the stored block),
    // FP64 ping-pong iterate
    P.compact = p->mode == PT_COEF_PHASES && prec == PT_PREC_MIXED;
    P.o_ac64 = P.take(16 * P.N);
    P.o_B64 = (size_t)-1;
    if (P.compact) {
        P.o_cb64 = P.take(16 * P.N);
        P.o_T64 = P.take(8 * P.N);
        P.o_cb32 = P.take(8 * P.N);
        P.o_T32 = P.take(4 * P.N);
    } else {
        P.o_B64 = P.take(32 * P.N);
    }
    P.o_xp = P.take(8 * P.N);
    P.o_xT = P.take(8 * P.N);
    P.o_gate = P.take(256);   // stream-ordered solve: stop flag, final k
    if (p->axisymmetric) {
        P.o_axm64 = P.take(32ull * p->n[1]);
        if (prec == PT_PREC_MIXED) P.o_axm32 = P.take(16ull * p->n[1]);
    }
    // hierarchy
    int n[3] = {p->n[0], p->n[1], p->n[2]};
    double h = p->h;
    int l = 0;
    for (;;) {
        LevelPlan &L = P.lv[l];
        for (int a = 0; a < 3; a++) L.n[a] = n[a];
        L.N = (long long)n[0] * n[1] * n[2];
        L.h = h;
        L.o_u = P.take(2 * R * L.N);
        L.o_f = P.take(2 * R * L.N);
        L.o_ac = L.o_fx = L.o_fy = L.o_fz = L.o_B = (size_t)-1;
        L.o_u2 = P.take(2 * R * L.N);   // the fused sweep writes to the other buffer
        if (l == 0) {
            if (prec == PT_PREC_MIXED) {
                L.o_ac = P.take(2 * R * L.N);
                if (!P.compact) L.o_B = P.take(4 * R * L.N);
            }
        } else {
            L.o_fx = P.take(2 * R * L.N);
            L.o_fy = P.take(2 * R * L.N);
            if (p->dim == 3) L.o_fz = P.take(2 * R * L.N);
            L.o_B = P.take(4 * R * L.N);
        }
        if (!can_coarsen(p->dim, n) || l + 1 >= kMaxLevels) break;
        for (int a = 0; a < p->dim; a++) n[a] /= 2;
        h *= 2.0;
        l++;
    }
    P.nlev = l + 1;
    const long long Nc = P.lv[l].N;
    if (Nc > kMaxCoarseCells)
        return "grid does not coarsen to at most 2048 cells (use sizes m*2^k with m <= 7)";
    P.m = (int)(2 * Nc);
    P.o_gj0 = P.take(8ull * P.m * P.m);
    P.o_gj1 = P.take(8ull * P.m * P.m);
    P.nblocks = std::max(sum2_blocks(P.N), outer_zm_blocks(p->dim, p->n[0], p->n[1], p->n[2]));
    P.o_partials = P.take(8ull * (4 * ((size_t)P.nblocks + reduce_scratch(P.nblocks)) + 16));
    P.o_flags = P.take(sizeof(int) * NFLAGS);
    return nullptr;
}

struct TimerRec {
    int cls;
    hipEvent_t a, b;
    long launches = 0;   // launches between a and b
    double bytes = 0;    // their algorithmic bytes
};

// A captured V-cycle of the coarse levels (1 .. L-1), with the counters its
// launches add (capture records them once; each replay adds them again).
struct CoarseGraph {
    int key = -1;
    unsigned state_in = 0, state_out = 0;   // iterate-buffer bits of levels >= 1
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    long launches[PT_K_COUNT] = {0};
    double bytes[PT_K_COUNT] = {0};
    long long updates = 0;
};

}  // namespace

// ------------------------------------------------------------------ handle
struct pt_mg_s {
    Plan P;
    pt_problem prob;             // copy; array pointers are not kept
    hipStream_t stream = nullptr;
    char *base = nullptr;
    double *norms_host = nullptr;   // pinned
    int *flags_host = nullptr;      // pinned
    std::string err = "no error";
    double *Ainv = nullptr;
    double *kry = nullptr;          // Krylov work vectors (allocated on first use)
    bool ready = false;
    bool owns_memory = true;        // false: device + pinned memory belong to a server arena
    bool p_field = false, T_field = false;   // phases mode: p_adv / T_adv given per cell
    CBK<double> cbk64 = {};         // compact block: the constants of the last assembly
    double ac_rho[2] = {}, ac_k[2] = {};  // phase densities and conductivities of the last assembly
    // the last assembly left the FP64 cell coefficients unwritten (the
    // compact block's C forms them where they are read); ensure_ac64 writes
    // them for the kernels that read the array
    bool ac64_lazy = false;
    CBK<float> cbk32 = {};
    int device = 0;                 // the GPU current at setup (its static scratch)
    hipEvent_t done_ev = nullptr;   // marks the end of the last enqueued step
    // asynchronous solve (pt_mg_solve drives it to the end; a server polls it)
    // Outer iteration k computes u_k (k >= 1: after V-cycle k-1) and the
    // norms of its residual into pinned slot k & 1, marked by norm_ev[k & 1].
    // u_k lives in the caller's (p, T) when k + parity is even and in the
    // handle's second FP64 pair otherwise; a zero-guess solve takes the
    // parity of the previous solve's last k, so that its answer most often
    // lands in (p, T) with no copy.  The host reads the norms of k_wait while
    // outer k_wait + 1 (and, when the contraction so far predicts that k_wait
    // + 1 cannot meet the tolerance, outer k_wait + 2) is already enqueued,
    // so the device does not idle while the host decides.
    hipEvent_t norm_ev[2] = {nullptr, nullptr};
    double *norms_devp = nullptr;   // device address of norms_host
    struct Solve {
        int phase = 0;              // 0 idle, 1 iterating (norms in flight), 2 finishing
        pt_solve_opts o;
        const double *b_p = nullptr, *b_T = nullptr;
        double *p = nullptr, *T = nullptr;
        const double *bshift = nullptr;
        int k_wait = 0, k_enq = -1;
        int status = PT_ERR_NOCONV;
        bool have_prev = false;
        double prev[2] = {0, 0};
        long long upd[2] = {0, 0};  // cell-updates enqueued up to outer k (slot k & 1)
        bool check_asm = false;     // the assembly of this step is checked with the first norms
        int parity = 0;             // u_k is in (p, T) when k + parity is even
        pt_solve_info inf;
        std::chrono::steady_clock::time_point t0;
    } sv;
    bool speculate = true;
    // from the last finished solve: the parity of its final k, and its last
    // contraction per component (the steady rate of later cycles)
    int hint_parity = 0;
    double rate_hint[2] = {0.0, 0.0};
    unsigned u_cur = 0;             // bit l: level l's current iterate is in its second buffer
    bool use_fused = true;          // false: two colour passes per sweep (reference path)
    // measurement
    unsigned timing = 0;            // bit c set: time launches of kernel class c
    int timing_every = 1;           // time one run in this many of a timed class
    long runs[PT_K_COUNT] = {0};
    std::vector<hipEvent_t> ev_free;
    std::vector<hipEvent_t> ev_all;
    std::vector<TimerRec> pending;
    long launches[PT_K_COUNT] = {0};
    double bytes[PT_K_COUNT] = {0};
    long timed_launches[PT_K_COUNT] = {0};
    double timed_bytes[PT_K_COUNT] = {0};
    double ms[PT_K_COUNT] = {0};
    long long updates = 0, last_updates = 0;
    std::vector<CoarseGraph> graphs;
    // the hierarchy build (coarsening chain, coarsest matrix and inverse)
    // as one graph, captured at the first assembly on a non-null stream
    hipGraph_t hier_graph = nullptr;
    hipGraphExec_t hier_exec = nullptr;
    bool hier_fused = true;         // use_fused when hier_graph was captured
    int hier_fields = 0;            // p_field + 2 T_field when hier_graph was captured
    CBK<double> hier_cbk64 = {};    // the compact block's constants when hier_graph was
    CBK<float> hier_cbk32 = {};     // captured (the graph holds them as kernel arguments)
    // off by default: with one kernel per coarse visit and the tail, a graph
    // replaces few launches, and its end costs more than they do
    bool use_graphs = false;
    // single-block tail cycle over levels tail_lt .. nlev-1 (0: not used)
    int tail_lt = 0;
    size_t tail_lds = 0;
    int tail_ainv_off = -1;
    bool use_tail = true;
    long long tail_max_cells = 0;   // largest level the tail may hold (0: LDS-limited only)
    // 16 nu1 + nu2 of the levels below the finest (0: as the finest).  One
    // sweep each way there saves time on acoustic steps but costs cycles on
    // diffusion-dominated ones, so the default keeps the solve's own counts.
    int coarse_nu = 0;
    // levels 1 .. w_levels (above the single-block tail) visit their coarse
    // level twice per visit (W-cycle there); 0: V-cycle
    int w_levels = 0;
    // over-relaxation of the finest level's block Gauss-Seidel sweeps, in
    // thousandths (1000: the plain update)
    int omega_milli = 1000;
    // stream-ordered solve: the stop flag every launch of it checks (null
    // otherwise), and its record in pinned host memory (made on first use)
    const int *gate_active = nullptr;
    AsyncInfo *async_host = nullptr, *async_devp = nullptr;

    template <typename T> T *at(size_t off) { return off == (size_t)-1 ? nullptr : (T *)(base + off); }
    double2 *ac64() { return at<double2>(P.o_ac64); }
    double4 *B64() { return at<double4>(P.o_B64); }
    double *partials() { return at<double>(P.o_partials); }
    int *flags() { return at<int>(P.o_flags); }

    // the compact block, its T and constants (null: stored block)
    template <typename R>
    void compact_view(const typename VT<R>::v2 *&cb, const R *&T, long long &tmask, CBK<R> &k)
    {
        cb = nullptr;
        T = nullptr;
        tmask = 0;
        std::memset(&k, 0, sizeof k);
        if (!P.compact) return;
        const bool f32 = sizeof(R) == 4;
        cb = at<typename VT<R>::v2>(f32 ? P.o_cb32 : P.o_cb64);
        T = at<R>(f32 ? P.o_T32 : P.o_T64);
        tmask = T_field ? -1ll : 0ll;
        if constexpr (sizeof(R) == 4) k = cbk32;
        else k = cbk64;
    }

    template <typename R> Lvl<R> level(int l)
    {
        const LevelPlan &L = P.lv[l];
        Lvl<R> o;
        o.nx = L.n[0];
        o.ny = L.n[1];
        o.nz = L.n[2];
        o.N = L.N;
        o.inv_h2 = 1.0 / (L.h * L.h);
        o.u = at<typename VT<R>::v2>(((u_cur >> l) & 1u) ? L.o_u2 : L.o_u);
        o.f = at<typename VT<R>::v2>(L.o_f);
        o.fx = at<typename VT<R>::v2>(L.o_fx);
        o.fy = at<typename VT<R>::v2>(L.o_fy);
        o.fz = at<typename VT<R>::v2>(L.o_fz);
        if (l == 0 && P.prec == PT_PREC_FP64) {
            o.ac = (const typename VT<R>::v2 *)ac64();
            o.B = (const typename VT<R>::v4 *)B64();
        } else {
            o.ac = at<typename VT<R>::v2>(L.o_ac);
            o.B = at<typename VT<R>::v4>(L.o_B);
        }
        o.axm = nullptr;
        o.cb = nullptr;
        o.T0 = nullptr;
        o.tmask = 0;
        std::memset(&o.k, 0, sizeof o.k);
        o.gate = gate_active;
        o.omega = R(1);
        if (l == 0) {
            o.omega = (R)(omega_milli / 1000.0);
            o.axm = (const typename VT<R>::v4 *)(sizeof(R) == 8 ? (void *)axm64()
                                                                : (void *)at<float4>(P.o_axm32));
            compact_view<R>(o.cb, o.T0, o.tmask, o.k);
        }
        return o;
    }
    // r-z metric of the finest rows (null on Cartesian grids)
    double4 *axm64() { return at<double4>(P.o_axm64); }
    // FP64 view of the finest-grid operator (coarsening source, exports).
    Lvl<double> level0_fp64()
    {
        Lvl<double> o = level<double>(0);
        o.u = nullptr;
        o.f = nullptr;
        o.ac = ac64();
        o.B = B64();
        o.axm = axm64();
        compact_view<double>(o.cb, o.T0, o.tmask, o.k);
        o.gate = nullptr;
        return o;
    }

    // --- timing --------------------------------------------------------
    // A run of back-to-back launches of one class shares one event pair
    // (opened by the first launch, closed by the last), so the per-launch
    // average carries the event overhead once per run; with timing_every
    // = n only one run in n of a class is timed at all.
    void begin(int cls, double nbytes, bool open = true)
    {
        launches[cls]++;
        bytes[cls] += nbytes;
        if (open) {
            timed_now = ((timing >> cls) & 1u) && (runs[cls]++ % timing_every) == 0;
            if (timed_now) {
                TimerRec r;
                r.cls = cls;
                r.a = event();
                r.b = event();
                (void)hipEventRecord(r.a, stream);
                pending.push_back(r);
            }
        }
        if (timed_now) {
            pending.back().launches++;
            pending.back().bytes += nbytes;
        }
    }
    bool timed_now = false;
    void end(bool close = true)
    {
        if (!timed_now || !close) return;
        (void)hipEventRecord(pending.back().b, stream);
        timed_now = false;
    }
    hipEvent_t event()
    {
        if (ev_free.empty()) {
            hipEvent_t e;
            (void)hipEventCreate(&e);
            ev_all.push_back(e);
            return e;
        }
        hipEvent_t e = ev_free.back();
        ev_free.pop_back();
        return e;
    }
    void flush_timing()   // takes the pairs whose launches have completed
    {
        size_t keep = 0;
        bool not_ready = false;
        for (size_t i = 0; i < pending.size(); i++) {
            TimerRec &r = pending[i];
            float t = 0.f;
            hipError_t e = hipEventElapsedTime(&t, r.a, r.b);
            if (e == hipErrorNotReady) {
                pending[keep++] = r;
                not_ready = true;
                continue;
            }
            if (e == hipSuccess) {
                ms[r.cls] += t;
                timed_launches[r.cls] += r.launches;
                timed_bytes[r.cls] += r.bytes;
            }
            ev_free.push_back(r.a);
            ev_free.push_back(r.b);
        }
        pending.resize(keep);
        if (not_ready) (void)hipGetLastError();   // not an error of the next call
    }
};

namespace {

int fail(pt_mg_t h, int code, const std::string &msg)
{
    if (h) h->err = msg;
    else g_thread_err = msg;
    return code;
}

// ------------------------------------------------------- static scratch
// Work memory of pt_mg_solve_noalloc (BiCGStab's eight FP64 vector pairs):
// one array per GPU, loaded with the library's code object, so that no
// call allocates.  In host code the name `scratch` only stands in for the
// device symbol: its address on each GPU comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address
// is passed to kernels.
static __device__ __align__(256) double scratch[16 * (size_t)PT_SCRATCH_MAX_CELLS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on GPU dev (looked up on first use).
int scratch_address(pt_mg_t h, int dev, double **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) return fail(h, PT_ERR_HIP, "device index out of range");
    if (!g_scratch_dev[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, PT_ERR_HIP, "hipGetDevice failed");
        }
        if (cur != dev && hipSetDevice(dev) != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, PT_ERR_HIP, "hipSetDevice failed");
        }
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(h, PT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                           hipGetErrorString(e));
        }
        g_scratch_dev[dev] = (double *)ptr;
    }
    *out = g_scratch_dev[dev];
    return PT_OK;
}

int check_hip(pt_mg_t h, hipError_t e, const char *what)
{
    if (e == hipSuccess) return PT_OK;
    return fail(h, PT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int sync(pt_mg_t h, const char *what)
{
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipGetLastError();
    h->flush_timing();
    return check_hip(h, e, what);
}

// Algorithmic bytes of one kernel launch (each array read or written once).
// The operator of level l per cell: cell (finest) or face coefficients and
// the block, stored or compact ((C, bb), and T where given per cell).
double op_bytes(pt_mg_t h, int l, double R)
{
    if (l == 0 && h->P.compact) return R * (2 + 2 + h->T_field);
    return ((l == 0 ? 2 : 2 * h->P.dim) + 4) * R;
}

double bytes_sweep_half(pt_mg_t h, int l, bool zero_guess)
{
    const double R = h->P.prec == PT_PREC_MIXED ? 4 : 8;
    const double N = (double)h->P.lv[l].N;
    // one colour: reads the other colour's u, its own f and block, all
    // coefficients (harmonic means need the neighbours'), writes its own u;
    // compact block: (C, bb) and T (where given per cell) of its own
    const double op = (l == 0 && h->P.compact)
                          ? R * (2 + 0.5 * (2 + h->T_field))
                          : 0.5 * 4 * R + (l == 0 ? 2 : 2 * h->P.dim) * R;
    return N * (0.5 * (zero_guess ? 0 : 2 * R) + 0.5 * 2 * R + op + 0.5 * 2 * R);
}

// One pass over memory per sweep pays off where a level has enough
// work for the whole chip: every 2-D level (independent tiles), 3-D
// levels of at least 2^20 cells (the plane-marching kernel).
bool fused_level(pt_mg_t h, int l)
{
    return h->use_fused && (h->P.dim == 2 || l == 0 || h->P.lv[l].N >= (1ll << 20));
}

// 3-D coarse levels of at least 2^20 cells restrict their residual with
// the plane-marching kernel (bitwise the gather kernel's result).
bool restrict_zm_level(pt_mg_t h, int l)
{
    return h->use_fused && h->P.dim == 3 && l >= 1 && h->P.lv[l].N >= (1ll << 20);
}

// 2-D coarse levels (not the coarsest) with nu1, nu2 in {1, 2}: each
// visit of the level in a V-cycle is a single kernel.
bool half_level(pt_mg_t h, int l, int nu1, int nu2)
{
    return h->use_fused && h->P.dim == 2 && l >= 1 && l + 1 < h->P.nlev && nu1 >= 1 && nu1 <= 2 &&
           nu2 >= 1 && nu2 <= 2;
}

// 3-D finest level in FP32: the last pre-smoothing sweep also forms the
// residual and restricts it to level 1 (one pass instead of two).
bool fused_restrict3(pt_mg_t h, int l, int nu1)
{
    return h->use_fused && h->P.dim == 3 && l == 0 && h->P.prec == PT_PREC_MIXED &&
           h->P.nlev > 1 && nu1 >= 1;
}

// `sweeps` sweeps on level l; with res (fused_restrict3) the last one also
// writes the restricted residual into level l+1's right-hand side.
template <typename R> void smooth(pt_mg_t h, int l, int sweeps, bool zero_guess, bool res = false)
{
    if (fused_level(h, l)) {
        // fused red-black sweeps (one pass over memory each), ping-ponging
        // the iterate between the level's two buffers
        const double Rb = sizeof(R);
        const int cls = l == 0 ? PT_K_SMOOTH_FINE : PT_K_SMOOTH_COARSE;
        for (int s = 0; s < sweeps; s++) {
            const bool zg = zero_guess && s == 0, r = res && s == sweeps - 1;
            Lvl<R> L = h->level<R>(l);
            h->u_cur ^= 1u << l;
            typename VT<R>::v2 *uo = h->level<R>(l).u;
            double nb = (double)L.N * ((zg ? 0 : 2 * Rb) + 2 * Rb + op_bytes(h, l, Rb) + 2 * Rb);
            if (r) nb += (double)h->P.lv[l + 1].N * 2 * Rb;            // coarse f written
            // the sweep that also restricts is a class of its own
            const bool next_r = res && s + 1 == sweeps - 1;
            if (r) h->begin(PT_K_SMOOTH_FINE_T, nb);
            else h->begin(cls, nb, s == 0);
            if (r)
                launch_rb_fused3r<R>(L, h->level<R>(l + 1), uo, zg ? 1 : 0, h->stream);
            else
                launch_rb_fused<R>(h->P.dim, L, uo, zg ? 1 : 0, l == 0 ? 0 : 1, h->stream);
            h->end(r || next_r || s == sweeps - 1);
            h->updates += L.N * (r ? 2 : 1);
        }
        return;
    }
    Lvl<R> L = h->level<R>(l);
    const int cls = l == 0 ? PT_K_SMOOTH_FINE : PT_K_SMOOTH_COARSE;
    for (int s = 0; s < sweeps; s++) {
        const bool zg = zero_guess && s == 0;
        h->begin(cls, bytes_sweep_half(h, l, zg));
        launch_rb_pass<R>(h->P.dim, l == 0, L, 0, zg ? 1 : 0, h->stream);
        h->end();
        h->begin(cls, bytes_sweep_half(h, l, false));
        launch_rb_pass<R>(h->P.dim, l == 0, L, 1, zg ? 2 : 0, h->stream);
        h->end();
        h->updates += L.N;
    }
}

// 2-D finest level with fused transfers: the first sweep after the coarse
// correction adds the prolonged correction as it loads the iterate (pro),
// the last sweep before the coarse cycle restricts its residual (res).
bool fused_transfers0(pt_mg_t h, int nu1, int nu2)
{
    return h->use_fused && h->P.dim == 2 && h->P.nlev > 1 && nu1 >= 1 && nu2 >= 1;
}

template <typename R> void smooth0_fused(pt_mg_t h, int sweeps, bool zero_guess, bool pro, bool res)
{
    const double Rb = sizeof(R);
    for (int s = 0; s < sweeps; s++) {
        const bool zg = zero_guess && s == 0, p = pro && s == 0, r = res && s == sweeps - 1;
        Lvl<R> L = h->level<R>(0), C = h->level<R>(1);
        h->u_cur ^= 1u;
        typename VT<R>::v2 *uo = h->level<R>(0).u;
        double nb = (double)L.N * ((zg ? 0 : 2 * Rb) + 2 * Rb + op_bytes(h, 0, Rb) + 2 * Rb);
        if (p || r) nb += (double)C.N * 2 * Rb;   // coarse u read, or coarse f written
        // a sweep with a transfer is a class of its own; the plain sweeps
        // between share one run
        const bool tr = p || r;
        const bool next_tr = s + 1 < sweeps && ((pro && s + 1 == 0) || (res && s + 1 == sweeps - 1));
        h->begin(tr ? PT_K_SMOOTH_FINE_T : PT_K_SMOOTH_FINE, nb, tr || s == 0 || (pro && s == 1));
        launch_tile2x<R>(L, C, uo, zg ? 1 : 0, p ? 1 : 0, r ? 1 : 0, h->stream);
        h->end(tr || next_tr || s == sweeps - 1);
        h->updates += L.N * (r ? 2 : 1);
    }
}

template <typename R> void restrict_level(pt_mg_t h, int l)
{
    Lvl<R> F = h->level<R>(l), C = h->level<R>(l + 1);
    const double Rb = sizeof(R);
    // u, f, the operator read; coarse f written
    h->begin(PT_K_RESTRICT, (double)F.N * (4 * Rb + op_bytes(h, l, Rb)) + (double)C.N * 2 * Rb);
    if (l == 0) launch_restrict_zm<R>(h->P.dim, F, C, h->stream);
    else if (restrict_zm_level(h, l)) launch_restrict_zm<R>(h->P.dim, F, C, h->stream, true);
    else launch_restrict<R>(h->P.dim, 0, F, C, h->stream);
    h->end();
    h->updates += F.N;
}

template <typename R> void prolong_level(pt_mg_t h, int l)
{
    Lvl<R> F = h->level<R>(l), C = h->level<R>(l + 1);
    const double Rb = sizeof(R);
    h->begin(PT_K_PROLONG, (double)F.N * 4 * Rb + (double)C.N * 2 * Rb);
    launch_prolong<R>(h->P.dim, F, C, h->stream);
    h->end();
}

template <typename R> void coarse_solve(pt_mg_t h)
{
    Lvl<R> L = h->level<R>(h->P.nlev - 1);
    const int m = h->P.m;
    h->begin(PT_K_COARSE_SOLVE, 8.0 * m * m + 2.0 * m * sizeof(R));
    launch_coarse_apply<R>(h->Ainv, m, (const R *)L.f, (R *)L.u, h->stream, h->gate_active);
    h->end();
}

template <typename R> void vcycle(pt_mg_t h, int l, int nu1, int nu2);

// Sweeps of the levels below the finest (PT_OPT_COARSE_SWEEPS).
int coarse_nu1(pt_mg_t h, int nu1) { return h->coarse_nu ? h->coarse_nu >> 4 : nu1; }
int coarse_nu2(pt_mg_t h, int nu2) { return h->coarse_nu ? h->coarse_nu & 15 : nu2; }

// Kernel classes launched by the coarse-level cycle.
constexpr unsigned kCoarseClasses =
    (1u << PT_K_SMOOTH_COARSE) | (1u << PT_K_RESTRICT) | (1u << PT_K_PROLONG) |
    (1u << PT_K_COARSE_SOLVE) | (1u << PT_K_OTHER);

// The V-cycle of levels 1 .. L-1 as one HIP graph launch (captured on first
// use per (nu1, nu2)): the coarse levels are small and their kernels are
// bound by launch submission.  Direct launches when the handle's stream is
// the null stream (it cannot be captured) or a coarse class is being timed.
template <typename R> void coarse_cycle(pt_mg_t h, int nu1, int nu2)
{
    if (!h->use_graphs || !h->stream || (h->timing & kCoarseClasses) || h->gate_active) {
        vcycle<R>(h, 1, nu1, nu2);
        return;
    }
    const int key = nu1 * 16 + nu2 + (h->use_fused ? 256 : 0) + (h->use_tail ? 512 : 0) +
                    (h->tail_lt << 10) + (std::min(h->w_levels, 63) << 16);
    const unsigned state = h->u_cur & ~1u;
    CoarseGraph *g = nullptr;
    for (auto &c : h->graphs)
        if (c.key == key && c.state_in == state) g = &c;
    if (!g) {
        CoarseGraph c;
        c.key = key;
        c.state_in = state;
        long l0[PT_K_COUNT];
        double b0[PT_K_COUNT];
        for (int q = 0; q < PT_K_COUNT; q++) {
            l0[q] = h->launches[q];
            b0[q] = h->bytes[q];
        }
        const long long u0 = h->updates;
        bool ok = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            vcycle<R>(h, 1, nu1, nu2);
            ok = hipStreamEndCapture(h->stream, &c.graph) == hipSuccess && c.graph;
        }
        if (ok) ok = hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0) == hipSuccess;
        for (int q = 0; q < PT_K_COUNT; q++) {
            c.launches[q] = h->launches[q] - l0[q];
            c.bytes[q] = h->bytes[q] - b0[q];
            h->launches[q] = l0[q];
            h->bytes[q] = b0[q];
        }
        c.updates = h->updates - u0;
        h->updates = u0;
        c.state_out = h->u_cur & ~1u;
        if (!ok) {
            (void)hipGetLastError();
            if (c.graph) (void)hipGraphDestroy(c.graph);
            h->use_graphs = false;   // fall back to direct launches for good
            vcycle<R>(h, 1, nu1, nu2);
            return;
        }
        h->graphs.push_back(c);
        g = &h->graphs.back();
    }
    (void)hipGraphLaunch(g->exec, h->stream);
    h->u_cur = (h->u_cur & 1u) | g->state_out;
    for (int q = 0; q < PT_K_COUNT; q++) {
        h->launches[q] += g->launches[q];
        h->bytes[q] += g->bytes[q];
    }
    h->updates += g->updates;
}

template <typename R> void tail_cycle(pt_mg_t h, int nu1, int nu2)
{
    const Plan &P = h->P;
    TailArgs<R> a;
    std::memset(&a, 0, sizeof a);
    a.nl = P.nlev - h->tail_lt;
    a.m = P.m;
    a.nu1 = nu1;
    a.nu2 = nu2;
    a.Ainv = h->Ainv;
    a.ainv_off = h->tail_ainv_off;
    size_t off = 0;
    double nbytes = 8.0 * P.m * P.m;
    for (int q = 0; q < a.nl; q++) {
        const int l = h->tail_lt + q;
        a.g[q] = h->level<R>(l);
        const long long N = P.lv[l].N;
        const size_t v2 = ((2 * sizeof(R) * N) + 15) & ~size_t(15);
        const size_t v4 = ((4 * sizeof(R) * N) + 15) & ~size_t(15);
        a.off[q][0] = (int)off; off += v2;
        a.off[q][1] = (int)off; off += v2;
        a.off[q][2] = (int)off; off += v2;
        a.off[q][3] = (int)off; off += v2;
        a.off[q][4] = (int)off; if (P.dim == 3) off += v2;
        a.off[q][5] = (int)off; off += v4;
        nbytes += (double)N * sizeof(R) * (4 + 2 * P.dim);
        if (q + 1 < a.nl) h->updates += (long long)(nu1 + nu2 + 1) * N;
    }
    nbytes += 4.0 * sizeof(R) * P.lv[h->tail_lt].N;   // f in, u out
    h->begin(PT_K_COARSE_SOLVE, nbytes);
    launch_tail<R>(P.dim, a, h->tail_lds, h->stream);
    h->end();
}

template <typename R> void vcycle_visit(pt_mg_t h, int l, int nu1, int nu2);

// The second coarse correction of a W visit of level l (from the iterate
// its first one left): sweeps, residual and restriction, the coarse cycle,
// prolongation, sweeps.  Separate kernels, with the arithmetic of the
// fused ones.
template <typename R> void w_repeat(pt_mg_t h, int l, int nu1, int nu2)
{
    smooth<R>(h, l, nu1, false);
    restrict_level<R>(h, l);
    vcycle<R>(h, l + 1, nu1, nu2);
    prolong_level<R>(h, l);
    smooth<R>(h, l, nu2, false);
}

// Multigrid cycle on level l for A e = f_l, e in u_l, from a zero guess:
// a V(nu1, nu2) cycle, with two coarse corrections per visit on levels
// 1 .. w_levels above the tail (PT_OPT_W_LEVELS).
template <typename R> void vcycle(pt_mg_t h, int l, int nu1, int nu2)
{
    vcycle_visit<R>(h, l, nu1, nu2);
    const bool tail = h->use_tail && h->tail_lt > 0 && l >= h->tail_lt;
    if (l >= 1 && l <= h->w_levels && !tail && l < h->P.nlev - 1) w_repeat<R>(h, l, nu1, nu2);
}

template <typename R> void vcycle_visit(pt_mg_t h, int l, int nu1, int nu2)
{
    if (h->use_tail && h->tail_lt > 0 && l == h->tail_lt) {
        tail_cycle<R>(h, nu1, nu2);
        return;
    }
    if (l == h->P.nlev - 1) {
        coarse_solve<R>(h);
        return;
    }
    if (l == 0 && fused_transfers0(h, nu1, nu2)) {
        smooth0_fused<R>(h, nu1, true, false, true);
        coarse_cycle<R>(h, coarse_nu1(h, nu1), coarse_nu2(h, nu2));
        smooth0_fused<R>(h, nu2, false, true, false);
        return;
    }
    if (half_level(h, l, nu1, nu2)) {
        // one kernel per visit: down (sweeps + residual + restriction) and
        // up (prolongation + sweeps)
        const double Rb = sizeof(R);
        Lvl<R> L = h->level<R>(l), C = h->level<R>(l + 1);
        h->begin(PT_K_SMOOTH_COARSE, (double)L.N * 12 * Rb + (double)C.N * 2 * Rb);
        launch_half2<R>(false, nu1, L, C, nullptr, h->stream);
        h->end();
        h->updates += (long long)(nu1 + 1) * L.N;
        vcycle<R>(h, l + 1, nu1, nu2);
        L = h->level<R>(l);
        C = h->level<R>(l + 1);
        h->u_cur ^= 1u << l;
        typename VT<R>::v2 *uo = h->level<R>(l).u;
        h->begin(PT_K_SMOOTH_COARSE, (double)L.N * 14 * Rb + (double)C.N * 2 * Rb);
        launch_half2<R>(true, nu2, L, C, uo, h->stream);
        h->end();
        h->updates += (long long)nu2 * L.N;
        return;
    }
    Lvl<R> L = h->level<R>(l);
    if (nu1 == 0) {
        h->begin(PT_K_OTHER, (double)L.N * 2 * sizeof(R));
        launch_zero(L.u, (size_t)L.N * 2 * sizeof(R), h->stream, h->gate_active);
        h->end();
    }
    const bool res = fused_restrict3(h, l, nu1);
    smooth<R>(h, l, nu1, true, res);
    if (!res) restrict_level<R>(h, l);
    if (l == 0) coarse_cycle<R>(h, coarse_nu1(h, nu1), coarse_nu2(h, nu2));
    else vcycle<R>(h, l + 1, nu1, nu2);
    prolong_level<R>(h, l);
    smooth<R>(h, l, nu2, false);
}

void vcycle_any(pt_mg_t h, int nu1, int nu2)
{
    if (h->P.prec == PT_PREC_MIXED) vcycle<float>(h, 0, nu1, nu2);
    else vcycle<double>(h, 0, nu1, nu2);
}

// ---- assembly + hierarchy + coarsest inverse --------------------------
// Levels of at most this many cells are built, with the coarsest inverse,
// by one single-block kernel (launch_hier_small) on the fused path.
constexpr long long kHierSmallCells = 1024;

template <typename R> void build_hierarchy(pt_mg_t h)
{
    const Plan &P = h->P;
    double *M0 = h->at<double>(P.o_gj0), *M1 = h->at<double>(P.o_gj1);
    const int pin = h->prob.mean_constraint ? 1 : 0;
    // b0: the first level the single-block kernel builds (its parent, a
    // face level, is the finest it reads)
    int b0 = P.nlev - 1;
    while (b0 - 1 >= 2 && P.lv[b0 - 1].N <= kHierSmallCells && P.nlev - b0 + 2 <= kMaxTail) b0--;
    const bool small = h->use_fused && P.nlev >= 3 && b0 >= 2 && P.m <= 128;
    if (P.nlev > 1) {
        Lvl<R> c1 = h->level<R>(1);
        // level 1 from the finest operator in the V-cycle's precision (the
        // FP32 copies in mixed precision: half the bytes of the FP64 one)
        launch_coarsen<R, R>(P.dim, 1, h->level<R>(0), (typename VT<R>::v2 *)c1.fx,
                             (typename VT<R>::v2 *)c1.fy, (typename VT<R>::v2 *)c1.fz,
                             (typename VT<R>::v4 *)c1.B, h->stream, h->use_fused);
        for (int l = 1; l + 1 < (small ? b0 : P.nlev); l++) {
            Lvl<R> f = h->level<R>(l), c = h->level<R>(l + 1);
            launch_coarsen<R, R>(P.dim, 0, f, (typename VT<R>::v2 *)c.fx,
                                 (typename VT<R>::v2 *)c.fy, (typename VT<R>::v2 *)c.fz,
                                 (typename VT<R>::v4 *)c.B, h->stream);
        }
    }
    if (small) {
        HierSmallArgs<R> a;
        std::memset(&a, 0, sizeof a);
        a.nl = P.nlev - b0 + 1;
        a.pin = pin;
        a.m = P.m;
        for (int q = 0; q < a.nl; q++) a.g[q] = h->level<R>(b0 - 1 + q);
        a.M0 = M0;
        a.Ainv = M1;
        a.flags = h->flags();
        if (launch_hier_small<R>(P.dim, a, h->stream)) {
            h->Ainv = M1;
            return;
        }
        for (int l = b0 - 1; l + 1 < P.nlev; l++) {
            Lvl<R> f = h->level<R>(l), c = h->level<R>(l + 1);
            launch_coarsen<R, R>(P.dim, 0, f, (typename VT<R>::v2 *)c.fx,
                                 (typename VT<R>::v2 *)c.fy, (typename VT<R>::v2 *)c.fz,
                                 (typename VT<R>::v4 *)c.B, h->stream);
        }
    }
    // dense coarsest matrix, inverted by Gauss-Jordan
    if (P.nlev == 1)
        launch_coarse_dense<double>(P.dim, 1, h->level0_fp64(), pin, M0, h->stream);
    else
        launch_coarse_dense<R>(P.dim, 0, h->level<R>(P.nlev - 1), pin, M0, h->stream);
    if (launch_gj_lds(M0, M1, P.m, h->flags(), h->stream)) {
        h->Ainv = M1;
    } else {
        double *src = M0, *dst = M1;
        for (int k = 0; k < P.m; k++) {
            launch_gj_step(src, dst, P.m, k, h->flags(), h->stream);
            std::swap(src, dst);
        }
        h->Ainv = src;
    }
}

// The hierarchy build replayed from a graph: its kernels read and write
// only the handle's memory, so one capture serves every update.  Direct
// launches on the null stream or if the capture fails.
template <typename R> void hierarchy(pt_mg_t h)
{
    if (!h->use_graphs || !h->stream) {
        build_hierarchy<R>(h);
        return;
    }
    const int fields = (int)h->p_field + 2 * (int)h->T_field;
    const bool same_k = std::memcmp(&h->hier_cbk64, &h->cbk64, sizeof h->cbk64) == 0 &&
                        std::memcmp(&h->hier_cbk32, &h->cbk32, sizeof h->cbk32) == 0;
    if (h->hier_exec && (h->hier_fused != h->use_fused || h->hier_fields != fields || !same_k)) {
        // PT_OPT_FUSED, which provisional fields are given per cell, or the
        // compact block's constants (dt, the phases) changed since the
        // capture: the graph holds other kernels or arguments, so capture
        // again
        (void)hipGraphExecDestroy(h->hier_exec);
        (void)hipGraphDestroy(h->hier_graph);
        h->hier_exec = nullptr;
        h->hier_graph = nullptr;
    }
    if (!h->hier_exec) {
        h->hier_fused = h->use_fused;
        h->hier_fields = fields;
        h->hier_cbk64 = h->cbk64;
        h->hier_cbk32 = h->cbk32;
        bool ok = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            build_hierarchy<R>(h);
            ok = hipStreamEndCapture(h->stream, &h->hier_graph) == hipSuccess && h->hier_graph;
        }
        if (ok) ok = hipGraphInstantiate(&h->hier_exec, h->hier_graph, nullptr, nullptr, 0) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            if (h->hier_graph) (void)hipGraphDestroy(h->hier_graph);
            h->hier_graph = nullptr;
            h->hier_exec = nullptr;
            build_hierarchy<R>(h);
            return;
        }
    }
    (void)hipGraphLaunch(h->hier_exec, h->stream);
}

// Enqueue assembly, hierarchy, coarsest inverse and the flag read-back on
// the handle's stream; done_ev marks the end.  With b_p, b_T (phases and
// state mode) the assembly also writes the paper right-hand side, as
// pt_mg_paper_rhs would with these p_adv, T_adv and div.
int assemble_enqueue(pt_mg_t h, const pt_problem *p, const double *div = nullptr,
                     double *b_p = nullptr, double *b_T = nullptr)
{
    const Plan &P = h->P;
    AsmArgs a;
    std::memset(&a, 0, sizeof a);
    a.N = P.N;
    a.mode = p->mode;
    a.alpha_p = p->alpha_p;
    a.alpha_T = p->alpha_T;
    a.alpha_p_const = p->alpha_p_const;
    a.alpha_T_const = p->alpha_T_const;
    a.B = p->B;
    for (int q = 0; q < 4; q++) a.B_const[q] = p->B_const[q];
    a.C = p->C;
    a.liq = p->liquid;
    a.gas = p->gas;
    a.dt = p->dt;
    a.p_adv = p->p_adv;
    a.T_adv = p->T_adv;
    a.p_adv_const = p->p_adv_const;
    a.T_adv_const = p->T_adv_const;
    a.m1 = p->m1;
    a.m2 = p->m2;
    a.ac64 = h->ac64();
    a.B64 = h->B64();
    h->ac64_lazy = false;
    if (P.prec == PT_PREC_MIXED) {
        a.ac32 = h->at<float2>(P.lv[0].o_ac);
        a.B32 = h->at<float4>(P.lv[0].o_B);
    }
    if (p->mode == PT_COEF_PHASES) {
        // the constants of this assembly (dt and the phases may change),
        // and where the block is kept compact, its arrays
        h->p_field = p->p_adv != nullptr;
        h->T_field = p->T_adv != nullptr;
        if (P.compact) {
            a.cb64 = h->at<double2>(P.o_cb64);
            a.T64 = h->at<double>(P.o_T64);
            a.cb32 = h->at<float2>(P.o_cb32);
            a.T32 = h->at<float>(P.o_T32);
            a.T_cells = h->T_field;
        }
        OpK k64;
        std::memset(&k64, 0, sizeof k64);
        const pt_phase *ph[2] = {&p->liquid, &p->gas};
        for (int q = 0; q < 2; q++) {
            const pt_phase &f = *ph[q];
            k64.rho[q] = f.rho;
            k64.k[q] = f.k;
            k64.blk.K1[q] = f.gamma / (f.rho * f.c * f.c) / (p->dt * p->dt);
            k64.blk.K2[q] = f.rho * f.cp / p->dt;
            k64.gcv[q] = (f.Gamma - 1.0) * f.cv;
            k64.b[q] = f.b;
            k64.Pi[q] = f.Pi;
            if (f.beta > 0.0) {
                k64.beta[q] = f.beta;
            } else if (f.b == 0.0 && !h->T_field) {
                // Eq. (10) without the covolume at the uniform T: as the kernels
                // would form it (gcv T + 0 is exact)
                k64.beta[q] = k64.gcv[q] / (k64.gcv[q] * p->T_adv_const);
            }
        }
        k64.blk.idt = 1.0 / p->dt;
        k64.blk.idt2 = 1.0 / (p->dt * p->dt);
        CBK<float> k32;
        for (int q = 0; q < 2; q++) {
            k32.K1[q] = (float)k64.blk.K1[q];
            k32.K2[q] = (float)k64.blk.K2[q];
        }
        k32.idt = (float)k64.blk.idt;
        k32.idt2 = (float)k64.blk.idt2;
        h->cbk64 = k64.blk;
        for (int q = 0; q < 2; q++) {
            h->ac_rho[q] = k64.rho[q];
            h->ac_k[q] = k64.k[q];
        }
        h->cbk32 = k32;
        a.k64 = k64;
        if (P.compact && P.nlev > 1) {
            // the V-cycle, the outer residual and the right-hand side read
            // the compact block alone (a single-level grid's coarsest
            // matrix reads the array)
            a.ac64 = nullptr;
            h->ac64_lazy = true;
        }
    }
    if (b_p && p->mode != PT_COEF_EXPLICIT) {
        a.div = div;
        a.b_p = b_p;
        a.b_T = b_T;
    }
    a.flags = h->flags();
    h->ready = false;
    // the handle keeps the scalars of the problem (not its array pointers)
    h->prob = *p;
    h->prob.alpha_p = h->prob.alpha_T = h->prob.B = h->prob.C = h->prob.p_adv = h->prob.T_adv = nullptr;
    launch_zero(h->flags(), sizeof(int) * NFLAGS, h->stream);
    launch_assemble(a, h->stream);
    if (P.prec == PT_PREC_MIXED) hierarchy<float>(h);
    else hierarchy<double>(h);
    // the flags go straight into the pinned host copy (its device address)
    launch_flags_out(h->flags(), (int *)(h->norms_devp + 16), NFLAGS, h->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(h->done_ev, h->stream);
    return check_hip(h, e, "setup enqueue");
}

// The FP64 cell coefficients of an assembly that left them to the
// compact block, written from its C (the assembly's arithmetic).
void ensure_ac64(pt_mg_t h)
{
    if (!h->ac64_lazy) return;
    h->begin(PT_K_OTHER, 32.0 * h->P.N);
    launch_fill_ac64(h->P.N, h->at<double2>(h->P.o_cb64), h->ac_rho, h->ac_k, h->ac64(), h->stream);
    h->end();
    h->ac64_lazy = false;
}

// After done_ev: interpret the flags of the assembly.
int assemble_check(pt_mg_t h)
{
    h->flush_timing();
    const int *f = h->flags_host;
    if (f[FLAG_ARG]) return fail(h, PT_ERR_ARG, "invalid input field (C outside [0,1], non-finite value, T <= 0 or negative coefficient)");
    if (h->prob.mean_constraint) {
        if (f[FLAG_BNONZERO]) return fail(h, PT_ERR_ARG, "mean_constraint requires B = 0 everywhere");
    } else if (f[FLAG_SINGULAR]) {
        return fail(h, PT_ERR_SINGULAR, "a cell block has det <= 0 or a non-positive diagonal");
    }
    if (f[FLAG_PIVOT]) return fail(h, PT_ERR_SINGULAR, "coarsest-grid elimination met a non-positive pivot");
    h->ready = true;
    return PT_OK;
}

int assemble(pt_mg_t h, const pt_problem *p)
{
    int rc = assemble_enqueue(h, p);
    if (rc) return rc;
    rc = check_hip(h, hipEventSynchronize(h->done_ev), "setup");
    if (rc == PT_OK) rc = check_hip(h, hipGetLastError(), "setup");
    if (rc) return rc;
    return assemble_check(h);
}

// The single-block tail covers the coarsest levels (at least two, none the
// finest) whose arrays fit together in one block's LDS.
void plan_tail(pt_mg_t h)
{
    const Plan &P = h->P;
    h->tail_lt = 0;
    if (P.nlev < 3) return;
    int dev = 0, lds_max = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        lds_max = 65536;
    const size_t budget = (size_t)std::max(0, lds_max - 4096);
    const bool f32 = P.prec == PT_PREC_MIXED;
    auto need = [&](int l) {
        return f32 ? tail_level_lds<float>(P.dim, P.lv[l].N) : tail_level_lds<double>(P.dim, P.lv[l].N);
    };
    size_t total = need(P.nlev - 1);
    int lt = P.nlev - 1;
    for (int l = P.nlev - 2; l >= 1; l--) {
        if (total + need(l) > budget || P.nlev - l > kMaxTail) break;
        if (h->tail_max_cells > 0 && P.lv[l].N > h->tail_max_cells) break;
        total += need(l);
        lt = l;
    }
    if (P.nlev - lt < 2) return;
    // a small coarsest inverse is copied into LDS with the levels
    h->tail_ainv_off = -1;
    const size_t ainv = ((size_t)8 * P.m * P.m + 15) & ~size_t(15);
    if (P.m <= 32 && total + ainv <= budget) {
        h->tail_ainv_off = (int)total;
        total += ainv;
    }
    h->tail_lt = lt;
    h->tail_lds = total;
    if (f32) tail_set_lds_limit<float>(P.dim, total);
    else tail_set_lds_limit<double>(P.dim, total);
}

bool same_grid(const pt_problem *a, const pt_problem *b)
{
    return a->dim == b->dim && a->n[0] == b->n[0] && a->n[1] == b->n[1] && a->n[2] == b->n[2] &&
           a->h == b->h && a->mode == b->mode && a->mean_constraint == b->mean_constraint &&
           a->axisymmetric == b->axisymmetric;
}

double elapsed(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// ================================================================== C ABI
// (the declarations in pt_mg.h give these definitions C linkage)

int pt_state_eval(const pt_state *st, void *hip_stream)
{
    if (!st) return fail(nullptr, PT_ERR_ARG, "state is NULL");
    if (st->dim != 2 && st->dim != 3) return fail(nullptr, PT_ERR_ARG, "dim must be 2 or 3");
    if (st->n < 1) return fail(nullptr, PT_ERR_ARG, "n must be >= 1");
    if (!st->C || !st->m1 || !st->m2 || !st->E || !st->p_adv || !st->T_adv)
        return fail(nullptr, PT_ERR_ARG, "NULL field");
    if (!(st->liquid.Gamma > 1.0) || !(st->gas.Gamma > 1.0))
        return fail(nullptr, PT_ERR_ARG, "Gamma must be > 1");
    launch_state(*st, (hipStream_t)hip_stream);
    return check_hip(nullptr, hipGetLastError(), "state kernel");
}

size_t pt_mg_footprint_bytes(const pt_problem *prob, int precision)
{
    Plan P;
    if (plan_problem(prob, precision, P)) return 0;
    return P.total;
}

namespace ptmg {

// A handle on caller-provided device memory (`bytes` >= the plan's total)
// and pinned host memory (16 doubles + 16 ints); with own_memory both are
// allocated here.  The assembly is enqueued, not waited for: the caller
// waits on handle_event and calls handle_setup_check.
int handle_create(const pt_problem *prob, int precision, hipStream_t stream, char *dev_mem,
                  size_t bytes, void *pinned, pt_mg_t *out, std::string *err)
{
    *out = nullptr;
    Plan P;
    if (const char *why = plan_problem(prob, precision, P)) {
        *err = why;
        return PT_ERR_ARG;
    }
    pt_mg_t h = new pt_mg_s();
    h->P = P;
    h->stream = stream;
    if (hipGetDevice(&h->device) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        *err = "hipGetDevice failed";
        return PT_ERR_HIP;
    }
    {
        // the static scratch's address on this GPU, taken at set-up so that
        // pt_mg_solve_noalloc's first call loads and looks up nothing (a
        // failure here is reported by that call, which retries)
        double *w = nullptr;
        if (scratch_address(nullptr, h->device, &w) != PT_OK) (void)hipGetLastError();
    }
    h->owns_memory = dev_mem == nullptr;
    if (h->owns_memory) {
        hipError_t e = hipMalloc(&h->base, P.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete h;
            *err = "hipMalloc of " + std::to_string(P.total) + " bytes failed";
            return PT_ERR_OOM;
        }
        e = hipHostMalloc(&h->norms_host, 16 * sizeof(double) + 16 * sizeof(int),
                          hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->norms_host = nullptr;
            pt_mg_destroy(h);
            *err = "pinned host allocation failed";
            return PT_ERR_OOM;
        }
    } else {
        if (bytes < P.total || !pinned) {
            delete h;
            *err = "external memory too small";
            return PT_ERR_ARG;
        }
        h->base = dev_mem;
        h->norms_host = (double *)pinned;
    }
    h->flags_host = (int *)(h->norms_host + 16);
    bool ok = hipEventCreateWithFlags(&h->done_ev, hipEventDisableTiming) == hipSuccess;
    for (int q = 0; q < 2 && ok; q++)
        ok = hipEventCreateWithFlags(&h->norm_ev[q], hipEventDisableTiming) == hipSuccess;
    // the reductions write the norms straight into the pinned slots
    ok = ok && hipHostGetDevicePointer((void **)&h->norms_devp, h->norms_host, 0) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        pt_mg_destroy(h);
        *err = "event creation or pinned mapping failed";
        return PT_ERR_HIP;
    }
    plan_tail(h);
    if (prob->axisymmetric)
        launch_axi_metric(P.n[1], h->axm64(), h->at<float4>(P.o_axm32), h->stream);
    int rc = assemble_enqueue(h, prob);
    if (rc != PT_OK) {
        *err = h->err;
        pt_mg_destroy(h);
        return rc;
    }
    *out = h;
    return PT_OK;
}

// Paper right-hand side (Eqs. 33-34) enqueued without waiting.
int handle_paper_rhs_async(pt_mg_t h, const double *p_adv, const double *T_adv,
                           const double *div_ustar, double *b_p, double *b_T)
{
    if (h->prob.mode == PT_COEF_EXPLICIT)
        return fail(h, PT_ERR_STATE, "paper_rhs needs phases or state mode");
    h->begin(PT_K_OTHER, 48.0 * h->P.N);
    launch_paper_rhs(h->level0_fp64(), p_adv, h->prob.p_adv_const, T_adv, h->prob.T_adv_const,
                     div_ustar, h->prob.dt, b_p, b_T, h->stream);
    h->end();
    return PT_OK;
}

const char *handle_error(pt_mg_t h) { return h->err.c_str(); }
int handle_setup_check(pt_mg_t h) { return assemble_check(h); }
size_t handle_plan_bytes(const pt_problem *prob, int precision)
{
    Plan P;
    if (plan_problem(prob, precision, P)) return 0;
    return P.total;
}

}  // namespace ptmg

int pt_mg_setup(const pt_problem *prob, int precision, void *hip_stream, pt_mg_t *out)
{
    if (!out) return fail(nullptr, PT_ERR_ARG, "out is NULL");
    *out = nullptr;
    pt_mg_t h = nullptr;
    std::string err;
    int rc = handle_create(prob, precision, (hipStream_t)hip_stream, nullptr, 0, nullptr, &h, &err);
    if (rc != PT_OK) return fail(nullptr, rc, err);
    rc = check_hip(h, hipEventSynchronize(h->done_ev), "setup");
    if (rc == PT_OK) rc = check_hip(h, hipGetLastError(), "setup");
    if (rc == PT_OK) rc = assemble_check(h);
    if (rc != PT_OK) {
        g_thread_err = h->err;
        pt_mg_destroy(h);
        return rc;
    }
    *out = h;
    return PT_OK;
}

int pt_mg_update(pt_mg_t h, const pt_problem *prob)
{
    if (!h) return fail(nullptr, PT_ERR_ARG, "handle is NULL");
    Plan P;
    if (const char *why = plan_problem(prob, h->P.prec, P)) return fail(h, PT_ERR_ARG, why);
    if (!same_grid(prob, &h->prob))
        return fail(h, PT_ERR_STATE, "update must keep dim, n, h, mode and mean_constraint");
    if (P.total != h->P.total) return fail(h, PT_ERR_STATE, "update changes the memory plan");
    return assemble(h, prob);
}

void pt_mg_destroy(pt_mg_t h)
{
    if (!h) return;
    if (h->stream || h->base) (void)hipStreamSynchronize(h->stream);
    if (h->done_ev) (void)hipEventDestroy(h->done_ev);
    for (auto ev : h->norm_ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto e : h->ev_all) (void)hipEventDestroy(e);
    for (auto &c : h->graphs) {
        if (c.exec) (void)hipGraphExecDestroy(c.exec);
        if (c.graph) (void)hipGraphDestroy(c.graph);
    }
    if (h->hier_exec) (void)hipGraphExecDestroy(h->hier_exec);
    if (h->hier_graph) (void)hipGraphDestroy(h->hier_graph);
    if (h->kry) (void)hipFree(h->kry);
    if (h->async_host) (void)hipHostFree(h->async_host);
    if (h->owns_memory) {
        if (h->base) (void)hipFree(h->base);
        if (h->norms_host) (void)hipHostFree(h->norms_host);
    }
    delete h;
}

const char *pt_mg_last_error(pt_mg_t h) { return h ? h->err.c_str() : g_thread_err.c_str(); }

int pt_mg_paper_rhs(pt_mg_t h, const double *p_adv, const double *T_adv, const double *div_ustar,
                    double *b_p, double *b_T)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (h->prob.mode == PT_COEF_EXPLICIT)
        return fail(h, PT_ERR_STATE, "paper_rhs needs phases or state mode");
    if (!b_p || !b_T) return fail(h, PT_ERR_ARG, "outputs are NULL");
    h->begin(PT_K_OTHER, 48.0 * h->P.N);
    launch_paper_rhs(h->level0_fp64(), p_adv, h->prob.p_adv_const, T_adv, h->prob.T_adv_const,
                     div_ustar, h->prob.dt, b_p, b_T, h->stream);
    h->end();
    return sync(h, "paper_rhs");
}

int pt_mg_divergence(pt_mg_t h, const double *const U[3], double *div)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    const Plan &P = h->P;
    const int dim = h->prob.dim;
    if (!U || !div) return fail(h, PT_ERR_ARG, "NULL array");
    for (int a = 0; a < dim; a++)
        if (!U[a]) return fail(h, PT_ERR_ARG, "NULL face velocity array");
    double faces = 0.0;
    for (int a = 0; a < dim; a++) faces += (double)P.N + (double)P.N / P.n[a];
    h->begin(PT_K_OTHER, 8.0 * (faces + P.N));
    launch_divergence(dim, P.n[0], P.n[1], P.n[2], 1.0 / h->prob.h, U[0], U[1],
                      dim == 3 ? U[2] : nullptr, h->axm64(), div, h->stream);
    h->end();
    return sync(h, "divergence");
}

int pt_mg_downstream(pt_mg_t h, const pt_downstream *d)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (h->prob.mode == PT_COEF_EXPLICIT)
        return fail(h, PT_ERR_STATE, "downstream needs phases or state mode");
    if (!d) return fail(h, PT_ERR_ARG, "NULL argument record");
    const Plan &P = h->P;
    const int dim = h->prob.dim;
    if (!d->p || !d->T || !d->C) return fail(h, PT_ERR_ARG, "p, T and C are required");
    int ncell = 0;
    for (int a = 0; a < dim; a++) {
        if (!d->U_star[a] || !d->U[a]) return fail(h, PT_ERR_ARG, "face velocities are required");
        if (d->U[a] == d->U_star[a])
            return fail(h, PT_ERR_ARG, "face velocities cannot be updated in place");
        if (!d->u_star[a] != !d->u[a])
            return fail(h, PT_ERR_ARG, "cell velocity needs both u_star and u");
        ncell += d->u[a] != nullptr;
    }
    if (ncell != 0 && ncell != dim)
        return fail(h, PT_ERR_ARG, "cell velocities for some axes only");
    const int ne = (d->E1_adv != nullptr) + (d->E2_adv != nullptr) + (d->E1 != nullptr) +
                   (d->E2 != nullptr);
    if (ne != 0 && ne != 4) return fail(h, PT_ERR_ARG, "energy update needs E1_adv, E2_adv, E1, E2");
    const double mu1 = h->prob.liquid.mu, mu2 = h->prob.gas.mu;
    const bool viscous = ne && (mu1 != 0.0 || mu2 != 0.0);
    if (viscous && !ncell)
        return fail(h, PT_ERR_ARG, "the viscous work needs the cell velocities u_star and u");
    ensure_ac64(h);
    DownArgs a = {};
    a.nx = P.n[0];
    a.ny = P.n[1];
    a.nz = P.n[2];
    a.inv_h = 1.0 / h->prob.h;
    a.dt = h->prob.dt;
    a.sigma = d->sigma;
    a.ac = h->ac64();
    a.axm = h->axm64();
    a.p = d->p;
    a.T = d->T;
    a.C = d->C;
    a.kappa = d->kappa;
    a.Ux = d->U_star[0];
    a.Uy = d->U_star[1];
    a.Vx = d->U[0];
    a.Vy = d->U[1];
    if (ncell) {
        a.ux = d->u_star[0];
        a.uy = d->u_star[1];
        a.vx = d->u[0];
        a.vy = d->u[1];
    }
    if (dim == 3) {
        a.Uz = d->U_star[2];
        a.Vz = d->U[2];
        if (ncell) {
            a.uz = d->u_star[2];
            a.vz = d->u[2];
        }
    }
    if (ne) {
        a.E1a = d->E1_adv;
        a.E2a = d->E2_adv;
        a.E1 = d->E1;
        a.E2 = d->E2;
    }
    // algorithmic bytes: every array read or written once
    const double N = (double)P.N;
    double faces = 0.0;
    for (int q = 0; q < dim; q++) faces += N + N / P.n[q];
    double bytes = 8.0 * (5.0 * N + 2.0 * faces);   // p, T, (1/rho, k), C; U*, U
    if (d->kappa) bytes += 8.0 * N;
    if (ncell) bytes += 16.0 * dim * N;
    if (ne) bytes += 32.0 * N;
    // the viscous pass: C, u, U read, E1 and E2 read and written
    if (viscous) bytes += 8.0 * (N + dim * N + faces + 4.0 * N);
    h->begin(PT_K_DOWNSTREAM, bytes);
    launch_downstream(dim, a, h->stream);
    if (viscous) {
        // second pass: needs the corrected velocities of the neighbours
        ViscArgs v = {};
        v.nx = a.nx;
        v.ny = a.ny;
        v.nz = a.nz;
        v.inv_h = a.inv_h;
        v.dt = a.dt;
        v.mu1 = mu1;
        v.mu2 = mu2;
        v.C = d->C;
        v.Ux = d->U[0];
        v.Uy = d->U[1];
        v.Uz = dim == 3 ? d->U[2] : nullptr;
        v.ux = d->u[0];
        v.uy = d->u[1];
        v.uz = dim == 3 ? d->u[2] : nullptr;
        v.axm = h->axm64();
        v.E1 = d->E1;
        v.E2 = d->E2;
        launch_viscous(dim, v, h->stream);
    }
    h->end();
    return sync(h, "downstream");
}

namespace {

// Outer residual on the finest grid; returns blocks of partial sums.
template <typename RV>
int outer(pt_mg_t h, const double *b_p, const double *b_T, const double *src_p,
          const double *src_T, double *dst_p, double *dst_T, bool update, bool want_r,
          double *res_p, double *res_T, const double *bshift, double *r64_p = nullptr,
          double *r64_T = nullptr, const void *src32 = nullptr, void *dst32 = nullptr)
{
    const Plan &P = h->P;
    OuterArgs<RV> a;
    a.src32 = (const typename VT<RV>::v2 *)src32;
    a.dst32 = (typename VT<RV>::v2 *)dst32;
    a.r64_p = r64_p;
    a.r64_T = r64_T;
    a.nx = P.n[0];
    a.ny = P.n[1];
    a.nz = P.n[2];
    a.N = P.N;
    a.inv_h2 = 1.0 / (h->prob.h * h->prob.h);
    a.axm = h->axm64();
    a.phases = h->prob.mode != PT_COEF_EXPLICIT;
    a.ac = h->ac64();
    a.B = h->B64();
    h->compact_view<double>(a.cb, a.T0, a.tmask, a.k);
    for (int q = 0; q < 2; q++) {
        a.rho[q] = h->ac_rho[q];
        a.kc[q] = h->ac_k[q];
    }
    a.b_p = b_p;
    a.b_T = b_T;
    a.bshift = bshift;
    a.bshift_scale = 1.0 / (double)P.N;
    a.src_p = src_p;
    a.src_T = src_T;
    a.dst_p = dst_p;
    a.dst_T = dst_T;
    a.du = h->level<RV>(0).u;
    a.r = want_r ? h->at<typename VT<RV>::v2>(P.lv[0].o_f) : nullptr;
    a.res_p = res_p;
    a.res_T = res_T;
    a.partials = h->partials();
    a.update = update ? 1 : 0;
    a.gate = h->gate_active;
    const double Rb = sizeof(RV);
    // iterate (unless zero), operator (a, block; the compact block alone,
    // a formed from its C), b
    double opb = P.compact ? 8.0 * (2 + h->T_field) : op_bytes(h, 0, 8);
    // a zero iterate: the residual is b, the block enters through l4 alone
    // ((C, bb) of the compact block, else the stored block; none without
    // the paper form)
    if (!src_p && !update) opb = !a.phases ? 0.0 : (P.compact ? 16.0 : 32.0);
    double nbytes = (double)P.N * ((src_p ? 16 : (src32 ? 2 * Rb : 0)) + opb + 16);
    if (update) nbytes += (double)P.N * (2 * Rb + (dst32 ? 2 * Rb : 16));
    if (want_r) nbytes += (double)P.N * 2 * Rb;
    if (res_p) nbytes += 8.0 * P.N;
    if (res_T) nbytes += 8.0 * P.N;
    h->begin(PT_K_OUTER_RESIDUAL, nbytes);
    int nb = launch_outer_zm<RV>(P.dim, a, h->stream);
    h->end();
    h->updates += P.N;
    return nb;
}

int outer_any(pt_mg_t h, const double *b_p, const double *b_T, const double *src_p,
              const double *src_T, double *dst_p, double *dst_T, bool update, bool want_r,
              double *res_p, double *res_T, const double *bshift, double *r64_p = nullptr,
              double *r64_T = nullptr, const void *src32 = nullptr, void *dst32 = nullptr)
{
    if (h->P.prec == PT_PREC_MIXED)
        return outer<float>(h, b_p, b_T, src_p, src_T, dst_p, dst_T, update, want_r, res_p, res_T,
                            bshift, r64_p, r64_T, src32, dst32);
    return outer<double>(h, b_p, b_T, src_p, src_T, dst_p, dst_T, update, want_r, res_p, res_T,
                         bshift, r64_p, r64_T, src32, dst32);
}

// Reduce the partial sums to 4 doubles written straight into pinned host
// slot `slot`; norm_ev[slot] marks their arrival.
int enqueue_norms(pt_mg_t h, int nb, int slot)
{
    h->begin(PT_K_OTHER, 32.0 * nb);
    launch_reduce4(h->partials(), nb, h->norms_devp + 4 * slot, h->stream, h->gate_active);
    h->end();
    return check_hip(h, hipEventRecord(h->norm_ev[slot], h->stream), "norm event");
}

int read_norms(pt_mg_t h, int nb, double out[4])
{
    int rc = enqueue_norms(h, nb, 0);
    if (rc) return rc;
    rc = sync(h, "residual");
    if (rc) return rc;
    for (int q = 0; q < 4; q++) out[q] = h->norms_host[q];
    return PT_OK;
}

// Sums of (x, y) over the grid (mean constraint), in fixed order; `slot`
// 0 or 1 selects one of two result pairs kept after the partial sums.
double *grid_sums(pt_mg_t h, const double *x, const double *y, int slot)
{
    const int nb = sum2_blocks(h->P.N);
    double *part = h->partials();
    double *out = part + 4ll * (h->P.nblocks + reduce_scratch(h->P.nblocks)) + 8 + 2 * slot;
    h->begin(PT_K_OTHER, 16.0 * h->P.N);
    launch_sum2(h->P.N, x, y, part, nb, out, h->stream);
    h->end();
    return out;
}

}  // namespace

int pt_mg_residual(pt_mg_t h, const double *b_p, const double *b_T, const double *p, const double *T,
                   double *r_p, double *r_T, double relres[2])
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (!b_p || !b_T || !p != !T) return fail(h, PT_ERR_ARG, "NULL field");
    int nb = outer_any(h, b_p, b_T, p, T, nullptr, nullptr, false, false, r_p, r_T, nullptr);
    double s[4];
    int rc = read_norms(h, nb, s);
    if (rc) return rc;
    if (relres) {
        relres[0] = s[2] > 0 ? std::sqrt(s[0] / s[2]) : std::sqrt(s[0]);
        relres[1] = s[3] > 0 ? std::sqrt(s[1] / s[3]) : std::sqrt(s[1]);
    }
    return PT_OK;
}

namespace {

// Where u_k lives (see pt_mg_s::Solve).
void iterate_at(pt_mg_t h, int k, double **p, double **T)
{
    if ((k + h->sv.parity) % 2 == 0) {
        *p = h->sv.p;
        *T = h->sv.T;
    } else {
        *p = h->at<double>(h->P.o_xp);
        *T = h->at<double>(h->P.o_xT);
    }
}

// From a zero guess in mixed precision the first iterate u_1 = du_1 is the
// FP32 correction itself: outer 1 keeps it as FP32 (p, T) pairs in the
// memory of its own iterate buffer's p array (8 bytes per cell, which the
// pairs fill), and outer 2 reads them from there and writes the other
// buffer pair; null where the iterate stays FP64.
void *first_pairs(pt_mg_t h)
{
    if (!h->sv.o.zero_guess || h->P.prec != PT_PREC_MIXED) return nullptr;
    double *p1, *T1;
    iterate_at(h, 1, &p1, &T1);
    return p1;
}

// Enqueue outer iteration k: V-cycle k-1 on r_{k-1} and the FP64 update
// u_k = u_{k-1} + du (k >= 1), the residual of u_k and its norms.
int enqueue_outer(pt_mg_t h, int k)
{
    auto &S = h->sv;
    int nb;
    // from a zero guess u_0 = 0 is never stored: outers 0 and 1 read no
    // source iterate
    if (k == 0) {
        double *sp = nullptr, *sT = nullptr;
        if (!S.o.zero_guess) iterate_at(h, 0, &sp, &sT);
        nb = outer_any(h, S.b_p, S.b_T, sp, sT, nullptr, nullptr, false, true, nullptr, nullptr,
                       S.bshift);
    } else {
        vcycle_any(h, S.o.nu1, S.o.nu2);
        double *sp = nullptr, *sT = nullptr, *dp, *dT;
        void *k1 = first_pairs(h);
        if (k > 1 || !S.o.zero_guess) iterate_at(h, k - 1, &sp, &sT);
        iterate_at(h, k, &dp, &dT);
        if (k1 && k == 1)   // u_1 = du_1: kept as FP32 pairs
            nb = outer_any(h, S.b_p, S.b_T, nullptr, nullptr, nullptr, nullptr, true, true,
                           nullptr, nullptr, S.bshift, nullptr, nullptr, nullptr, k1);
        else if (k1 && k == 2)
            nb = outer_any(h, S.b_p, S.b_T, nullptr, nullptr, dp, dT, true, true, nullptr,
                           nullptr, S.bshift, nullptr, nullptr, k1, nullptr);
        else
            nb = outer_any(h, S.b_p, S.b_T, sp, sT, dp, dT, true, true, nullptr, nullptr,
                           S.bshift);
    }
    S.k_enq = k;
    S.upd[k & 1] = h->updates;
    return enqueue_norms(h, nb, k & 1);
}

}  // namespace

namespace ptmg {

hipEvent_t handle_event(pt_mg_t h)
{
    return h->sv.phase == 1 ? h->norm_ev[h->sv.k_wait & 1] : h->done_ev;
}

// Start a solve: enqueue the initial residual and its norms (and, from a
// zero guess, whose relative residual is 1, the first cycle).  Returns an
// error, or PT_OK with the solve running (handle_event marks progress).
int solve_begin(pt_mg_t h, const double *b_p, const double *b_T, double *p, double *T,
                const pt_solve_opts *opts_in)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (!b_p || !b_T || !p || !T) return fail(h, PT_ERR_ARG, "NULL field");
    pt_solve_opts o = {1e-9, 50, 2, 2, 1, PT_SOLVE_DEFECT};
    if (opts_in) o = *opts_in;
    if (!(o.rtol >= 0) || o.max_cycles < 0 || o.nu1 < 0 || o.nu2 < 0 || o.nu1 > 8 || o.nu2 > 8 ||
        o.nu1 + o.nu2 == 0)
        return fail(h, PT_ERR_ARG, "bad solve options");
    if (o.method != PT_SOLVE_DEFECT)
        return fail(h, PT_ERR_ARG, "only the defect-correction loop runs asynchronously");
    auto &S = h->sv;
    S = pt_mg_s::Solve();
    S.t0 = std::chrono::steady_clock::now();
    S.o = o;
    S.b_p = b_p;
    S.b_T = b_T;
    S.p = p;
    S.T = T;
    std::memset(&S.inf, 0, sizeof S.inf);
    h->updates = 0;
    if (o.zero_guess) S.parity = h->hint_parity;
    // mean constraint: the right-hand side is used with its mean removed
    S.bshift = h->prob.mean_constraint ? grid_sums(h, b_p, b_T, 0) : nullptr;
    int rc = enqueue_outer(h, 0);
    if (rc == PT_OK && h->speculate && o.zero_guess && o.rtol < 0.5 && o.max_cycles >= 1)
        rc = enqueue_outer(h, 1);
    if (rc) return rc;
    S.k_wait = 0;
    S.phase = 1;
    return PT_OK;
}

// Advance a running solve once handle_event has completed: returns
// PT_RUNNING (-1) after enqueuing what follows, or the final status.
int solve_advance(pt_mg_t h, pt_solve_info *info)
{
    auto &S = h->sv;
    const Plan &P = h->P;
    hipError_t e;
    h->flush_timing();
    if (S.phase == 1 && S.check_asm) {
        // pt_mg_step: the assembly flags were copied before the first
        // residual, so they are in host memory now
        S.check_asm = false;
        h->ready = false;
        const int rc = assemble_check(h);   // ready again on success
        if (rc != PT_OK) {
            (void)hipStreamSynchronize(h->stream);   // let the enqueued cycles drain
            S.phase = 0;
            return rc;
        }
    }
    if (S.phase == 1) {
        const int k = S.k_wait;
        const double *s = h->norms_host + 4 * (k & 1);
        double rel[2] = {s[2] > 0 ? std::sqrt(s[0] / s[2]) : std::sqrt(s[0]),
                         s[3] > 0 ? std::sqrt(s[1] / s[3]) : std::sqrt(s[1])};
        auto &inf = S.inf;
        if (inf.hist_len < PT_MAX_HIST) {
            inf.relres_hist[2 * inf.hist_len] = rel[0];
            inf.relres_hist[2 * inf.hist_len + 1] = rel[1];
            inf.hist_len++;
        }
        inf.relres[0] = rel[0];
        inf.relres[1] = rel[1];
        bool finish = true;
        if (!std::isfinite(rel[0]) || !std::isfinite(rel[1])) {
            S.status = PT_ERR_NOCONV;
            h->err = "residual norm is not finite";
        } else if (rel[0] <= S.o.rtol && rel[1] <= S.o.rtol) {
            S.status = PT_OK;
        } else if (k >= S.o.max_cycles) {
            S.status = PT_ERR_NOCONV;
            h->err = "max_cycles reached";
        } else {
            finish = false;
        }
        if (!finish) {
            int rc = PT_OK;
            if (S.k_enq == k) rc = enqueue_outer(h, k + 1);
            // Outer k+2 ahead of the norms of k+1 when, at the last
            // contraction seen (0.1 before any), u_{k+1} still misses the
            // tolerance by a factor of 3.  The multigrid contracts at a
            // steady rate after its first cycle, which contracts far more
            // from a zero guess (so its rate under-predicts the next
            // residual and errs on the side of waiting); a wrong guess
            // costs one cycle of device time, never a different result.
            if (rc == PT_OK && h->speculate && S.k_enq == k + 1 && k + 2 <= S.o.max_cycles) {
                constexpr double kMargin = 3.0;
                bool ahead = false;
                for (int c = 0; c < 2; c++) {
                    double rate = S.have_prev && S.prev[c] > 0 ? rel[c] / S.prev[c] : 0.1;
                    // the first cycle from a zero guess contracts far more
                    // than the later ones: the previous solve's last rate
                    // predicts the next better
                    if (k == 1 && S.o.zero_guess) rate = std::max(rate, h->rate_hint[c]);
                    rate = std::min(rate, 1.0);
                    if (rel[c] * rate > kMargin * S.o.rtol) ahead = true;
                }
                if (ahead) rc = enqueue_outer(h, k + 2);
            }
            if (rc) {
                S.phase = 0;
                return rc;
            }
            S.prev[0] = rel[0];
            S.prev[1] = rel[1];
            S.have_prev = true;
            S.k_wait = k + 1;
            return PT_RUNNING;
        }
        // u_k is the answer; later speculative outers wrote only the other
        // buffer pair, and the copy below is ordered after them.
        S.k_wait = k;
        if (S.o.zero_guess) h->hint_parity = k % 2;
        if (inf.hist_len >= 3) {
            const double *hh = inf.relres_hist + 2 * (inf.hist_len - 2);
            for (int c = 0; c < 2; c++)
                h->rate_hint[c] = hh[c] > 0 && std::isfinite(hh[c + 2]) ? hh[c + 2] / hh[c] : 0.0;
        }
        if (k == 0 && S.o.zero_guess) {
            // the answer is the zero guess itself, never stored
            h->begin(PT_K_OTHER, 16.0 * P.N);
            launch_zero2(S.p, S.T, 8 * (size_t)P.N, h->stream);
            h->end();
        } else if (k == 1 && first_pairs(h)) {
            // u_1 as FP32 pairs (possibly in S.p's own memory)
            h->begin(PT_K_OTHER, 24.0 * P.N);
            launch_pairs_to_fp64((const float2 *)first_pairs(h), S.p, S.T, P.N, h->stream);
            h->end();
        } else if ((k + S.parity) % 2 == 1) {
            double *xp, *xT;
            iterate_at(h, k, &xp, &xT);
            h->begin(PT_K_OTHER, 32.0 * P.N);
            launch_convert<double, double>(P.N, xp, S.p, h->stream);
            launch_convert<double, double>(P.N, xT, S.T, h->stream);
            h->end();
        }
        if (h->prob.mean_constraint) {
            double *us = grid_sums(h, S.p, S.T, 1);
            launch_shift2(P.N, S.p, S.T, us, 1.0 / (double)P.N, h->stream);
        }
        e = hipEventRecord(h->done_ev, h->stream);
        if (e != hipSuccess) {
            S.phase = 0;
            return check_hip(h, e, "solve");
        }
        S.phase = 2;
        return PT_RUNNING;
    }
    // phase 2: the final copies are done
    S.phase = 0;
    h->last_updates = S.upd[S.k_wait & 1];
    S.inf.cycles = S.k_wait;
    S.inf.t_solve_s = elapsed(S.t0);
    S.inf.status = S.status;
    if (info) *info = S.inf;
    return S.status;
}

}  // namespace ptmg

static int krylov_solve(pt_mg_t h, const double *b_p, const double *b_T, double *p, double *T,
                        const pt_solve_opts &o, pt_solve_info *info, double *work);

// Argument checks of a BiCGStab solve.
static int krylov_check(pt_mg_t h, const double *b_p, const double *b_T, double *p, double *T,
                        const pt_solve_opts &o)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (!b_p || !b_T || !p || !T) return fail(h, PT_ERR_ARG, "NULL field");
    if (!(o.rtol >= 0) || o.max_cycles < 0 || o.nu1 < 0 || o.nu2 < 0 || o.nu1 > 8 ||
        o.nu2 > 8 || o.nu1 + o.nu2 == 0)
        return fail(h, PT_ERR_ARG, "bad solve options");
    return PT_OK;
}

int pt_mg_solve_noalloc(pt_mg_t h, const double *b_p, const double *b_T, double *p, double *T,
                        const pt_solve_opts *opts_in, pt_solve_info *info)
{
    if (opts_in && opts_in->async)
        return fail(h, PT_ERR_ARG, "the stream-ordered mode allocates; call pt_mg_solve");
    if (!opts_in || opts_in->method != PT_SOLVE_BICGSTAB)
        return pt_mg_solve(h, b_p, b_T, p, T, opts_in, info);   // allocates nothing
    int rc = krylov_check(h, b_p, b_T, p, T, *opts_in);
    if (rc != PT_OK) return rc;
    if (h->P.N > PT_SCRATCH_MAX_CELLS)
        return fail(h, PT_ERR_ARG, "grid of " + std::to_string(h->P.N) +
                                       " cells exceeds the static scratch (" +
                                       std::to_string((long long)PT_SCRATCH_MAX_CELLS) +
                                       " cells)");
    double *work = nullptr;
    rc = scratch_address(h, h->device, &work);
    if (rc != PT_OK) return rc;
    return krylov_solve(h, b_p, b_T, p, T, *opts_in, info, work);
}

namespace {

// The end of a stream-ordered solve, run by the stream after its last
// launch: the record the stop tests wrote, into the caller's info.
struct AsyncDone {
    const AsyncInfo *rec;
    pt_solve_info *info;
    std::chrono::steady_clock::time_point t0;
};

void async_done(void *user)
{
    AsyncDone *d = (AsyncDone *)user;
    if (d->info) {
        const AsyncInfo &a = *d->rec;
        pt_solve_info o;
        std::memset(&o, 0, sizeof o);
        o.cycles = a.cycles;
        o.relres[0] = a.relres[0];
        o.relres[1] = a.relres[1];
        o.hist_len = a.hist_len;
        for (int q = 0; q < 2 * a.hist_len && q < 2 * PT_MAX_HIST; q++) o.relres_hist[q] = a.hist[q];
        o.status = a.status;
        o.t_solve_s = elapsed(d->t0);
        *d->info = o;
    }
    delete d;
}

// The defect-correction loop with every outer iteration up to max_cycles
// enqueued at once: after each residual a one-thread launch takes the stop
// test on the device and, once it is met, sets the flag that turns every
// later launch of the solve into a no-op; a last launch moves u_k into
// (p, T), and a host function fills `info`.  Nothing waits on the host.
int solve_async(pt_mg_t h, const double *b_p, const double *b_T, double *p, double *T,
                const pt_solve_opts &o, pt_solve_info *info)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (!b_p || !b_T || !p || !T) return fail(h, PT_ERR_ARG, "NULL field");
    if (!(o.rtol >= 0) || o.max_cycles < 0 || o.nu1 < 0 || o.nu2 < 0 || o.nu1 > 8 || o.nu2 > 8 ||
        o.nu1 + o.nu2 == 0)
        return fail(h, PT_ERR_ARG, "bad solve options");
    if (o.method != PT_SOLVE_DEFECT)
        return fail(h, PT_ERR_ARG, "the stream-ordered solve runs the defect-correction loop");
    if (o.max_cycles > PT_MAX_HIST - 1)
        return fail(h, PT_ERR_ARG, "stream-ordered solve: max_cycles <= PT_MAX_HIST - 1");
    const Plan &P = h->P;
    if (!h->async_host) {
        void *mem = nullptr;
        hipError_t e = hipHostMalloc(&mem, sizeof(AsyncInfo), hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, PT_ERR_OOM, "pinned host allocation failed");
        }
        h->async_host = (AsyncInfo *)mem;
        e = hipHostGetDevicePointer((void **)&h->async_devp, mem, 0);
        if (e != hipSuccess) return check_hip(h, e, "pinned mapping");
    }
    int *gate = h->at<int>(P.o_gate);
    auto &S = h->sv;
    S = pt_mg_s::Solve();
    S.t0 = std::chrono::steady_clock::now();
    S.o = o;
    S.b_p = b_p;
    S.b_T = b_T;
    S.p = p;
    S.T = T;
    h->updates = 0;
    if (o.zero_guess) S.parity = h->hint_parity;
    launch_gate_reset(gate, h->async_devp, h->stream);
    S.bshift = h->prob.mean_constraint ? grid_sums(h, b_p, b_T, 0) : nullptr;
    int rc = PT_OK;
    h->gate_active = gate;
    for (int k = 0; k <= o.max_cycles && rc == PT_OK; k++) {
        rc = enqueue_outer(h, k);
        if (rc == PT_OK)
            launch_async_decide(h->norms_devp + 4 * (k & 1), k, o.rtol, o.max_cycles, gate,
                                h->async_devp, h->stream);
    }
    h->gate_active = nullptr;
    if (rc != PT_OK) {
        (void)hipStreamSynchronize(h->stream);
        return rc;
    }
    h->begin(PT_K_OTHER, 32.0 * P.N);
    launch_async_final(gate, S.parity, o.zero_guess, h->at<double>(P.o_xp),
                       h->at<double>(P.o_xT), (const float2 *)first_pairs(h), p, T, P.N,
                       h->stream);
    h->end();
    if (h->prob.mean_constraint) {
        double *us = grid_sums(h, p, T, 1);
        launch_shift2(P.N, p, T, us, 1.0 / (double)P.N, h->stream);
    }
    AsyncDone *d = new AsyncDone{h->async_host, info, S.t0};
    hipError_t e = hipLaunchHostFunc(h->stream, async_done, d);
    if (e != hipSuccess) {
        delete d;
        return check_hip(h, e, "stream-ordered solve");
    }
    h->last_updates = 0;   // not known on the host
    S.phase = 0;
    return check_hip(h, hipGetLastError(), "stream-ordered solve");
}

}  // namespace

int pt_mg_solve(pt_mg_t h, const double *b_p, const double *b_T, double *p, double *T,
                const pt_solve_opts *opts_in, pt_solve_info *info)
{
    if (opts_in && opts_in->async) return solve_async(h, b_p, b_T, p, T, *opts_in, info);
    if (opts_in && opts_in->method == PT_SOLVE_BICGSTAB) {
        int rc = krylov_check(h, b_p, b_T, p, T, *opts_in);
        if (rc != PT_OK) return rc;
        return krylov_solve(h, b_p, b_T, p, T, *opts_in, info, nullptr);
    }
    if (opts_in && opts_in->method != PT_SOLVE_DEFECT) return fail(h, PT_ERR_ARG, "unknown method");
    int rc = solve_begin(h, b_p, b_T, p, T, opts_in);
    if (rc != PT_OK) return rc;
    for (;;) {
        rc = check_hip(h, hipEventSynchronize(handle_event(h)), "solve");
        if (rc == PT_OK) rc = check_hip(h, hipGetLastError(), "solve");
        if (rc != PT_OK) {
            h->sv.phase = 0;
            return rc;
        }
        rc = solve_advance(h, info);
        if (rc != PT_RUNNING) return rc;
    }
}

int pt_mg_step(pt_mg_t h, const pt_problem *prob, const double *div_ustar, double *b_p,
               double *b_T, double *p, double *T, const pt_solve_opts *opts_in,
               pt_solve_info *info)
{
    if (!h) return fail(nullptr, PT_ERR_ARG, "handle is NULL");
    if (!prob) return fail(h, PT_ERR_ARG, "problem is NULL");
    if (prob->mode == PT_COEF_EXPLICIT)
        return fail(h, PT_ERR_STATE, "step needs phases or state mode");
    if (!b_p || !b_T || !p || !T) return fail(h, PT_ERR_ARG, "NULL field");
    if (opts_in && opts_in->async)
        return fail(h, PT_ERR_ARG, "the stream-ordered mode applies to pt_mg_solve");
    if (opts_in && opts_in->method != PT_SOLVE_DEFECT) {
        // the Krylov loop waits on every reduction anyway
        int rc = pt_mg_update(h, prob);
        if (rc == PT_OK) rc = pt_mg_paper_rhs(h, prob->p_adv, prob->T_adv, div_ustar, b_p, b_T);
        if (rc == PT_OK) rc = pt_mg_solve(h, b_p, b_T, p, T, opts_in, info);
        return rc;
    }
    Plan P;
    if (const char *why = plan_problem(prob, h->P.prec, P)) return fail(h, PT_ERR_ARG, why);
    if (!same_grid(prob, &h->prob))
        return fail(h, PT_ERR_STATE, "update must keep dim, n, h, mode and mean_constraint");
    if (P.total != h->P.total) return fail(h, PT_ERR_STATE, "update changes the memory plan");
    // the assembly forms the paper right-hand side with the block
    int rc = assemble_enqueue(h, prob, div_ustar, b_p, b_T);
    if (rc != PT_OK) {
        (void)hipStreamSynchronize(h->stream);
        return rc;
    }
    h->ready = true;   // provisionally: the flags are checked with the first norms
    rc = solve_begin(h, b_p, b_T, p, T, opts_in);
    if (rc != PT_OK) {
        (void)hipStreamSynchronize(h->stream);
        h->ready = false;
        const int arc = assemble_check(h);
        return arc != PT_OK ? arc : rc;
    }
    h->sv.check_asm = true;
    for (;;) {
        rc = check_hip(h, hipEventSynchronize(handle_event(h)), "step");
        if (rc == PT_OK) rc = check_hip(h, hipGetLastError(), "step");
        if (rc != PT_OK) {
            h->sv.phase = 0;
            h->ready = false;
            return rc;
        }
        rc = solve_advance(h, info);
        if (rc != PT_RUNNING) return rc;
    }
}

// ---------------------------------------------------------- step entries
int pt_mg_num_levels(pt_mg_t h) { return h ? h->P.nlev : 0; }

int pt_mg_level_dims(pt_mg_t h, int level, int n[3], double *hl)
{
    if (!h) return fail(nullptr, PT_ERR_ARG, "handle is NULL");
    if (level < 0 || level >= h->P.nlev) return fail(h, PT_ERR_ARG, "level out of range");
    for (int a = 0; a < 3; a++) n[a] = h->P.lv[level].n[a];
    if (hl) *hl = h->P.lv[level].h;
    return PT_OK;
}

namespace {
template <typename R> void export_level(pt_mg_t h, int level, double *faces, double *B)
{
    ensure_ac64(h);
    if (level == 0)
        launch_export_op<double>(h->P.dim, 1, h->level0_fp64(), faces, B, h->stream);
    else
        launch_export_op<R>(h->P.dim, 0, h->level<R>(level), faces, B, h->stream);
}
}  // namespace

int pt_mg_get_operator(pt_mg_t h, int level, double *faces, double *B)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (level < 0 || level >= h->P.nlev) return fail(h, PT_ERR_ARG, "level out of range");
    if (!faces || !B) return fail(h, PT_ERR_ARG, "NULL output");
    if (h->P.prec == PT_PREC_MIXED) export_level<float>(h, level, faces, B);
    else export_level<double>(h, level, faces, B);
    return sync(h, "get_operator");
}

namespace {
template <typename R> void pack_lv(pt_mg_t h, int l, bool f, const double *x, const double *y)
{
    Lvl<R> L = h->level<R>(l);
    launch_pack<R>(L.N, x, y, f ? L.f : L.u, h->stream);
}
template <typename R> void unpack_lv(pt_mg_t h, int l, bool f, double *x, double *y)
{
    Lvl<R> L = h->level<R>(l);
    launch_unpack<R>(L.N, f ? L.f : L.u, x, y, h->stream);
}
}  // namespace

#define PT_DISPATCH(h, CALL)                                    \
    do {                                                        \
        if ((h)->P.prec == PT_PREC_MIXED) { using R = float; CALL; } \
        else { using R = double; CALL; }                        \
    } while (0)

// BiCGStab (van der Vorst) on the canonical system A x = f with the
// V-cycle as right preconditioner.  The residual is recomputed from x in
// FP64 every iteration (the outer-residual kernel, which also gives the
// paper-row-form norms of the stop test).  Vectors are FP64 pairs (p, T)
// in `work` (16 N doubles; null: h->kry, allocated on first use); "neg"
// vectors hold -A y, as the residual kernel returns them for a zero
// right-hand side.  Every vector is written before it is read except PV
// and VN, which are cleared, so stale work contents never matter.  Dot
// products are fixed-order reductions.
static int krylov_solve(pt_mg_t h, const double *b_p, const double *b_T, double *p, double *T,
                        const pt_solve_opts &o, pt_solve_info *info, double *work)
{
    const Plan &P = h->P;
    const long long N = P.N;
    if (h->prob.mean_constraint)
        return fail(h, PT_ERR_ARG, "BiCGStab does not take the mean constraint");
    if (!work) {
        if (!h->owns_memory)
            return fail(h, PT_ERR_STATE, "BiCGStab needs a handle with its own memory");
        if (!h->kry) {
            hipError_t e = hipMalloc(&h->kry, sizeof(double) * 16 * (size_t)N);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                h->kry = nullptr;
                return fail(h, PT_ERR_OOM, "BiCGStab work vectors");
            }
        }
        work = h->kry;
    }
    enum { R = 0, RH, PV, VN, SV, TN, PH, SH };
    auto vp = [&](int k) { return work + 2 * N * k; };
    auto vT = [&](int k) { return work + 2 * N * k + N; };
    const auto t0 = std::chrono::steady_clock::now();
    pt_solve_info inf;
    std::memset(&inf, 0, sizeof inf);
    h->updates = 0;
    hipStream_t st = h->stream;
    if (o.zero_guess) {
        launch_zero(p, 8 * (size_t)N, st);
        launch_zero(T, 8 * (size_t)N, st);
    }
    int rc = PT_OK;
    double rel[2] = {0, 0};
    // r = f - A x in FP64 (canonical), paper-form relative norms
    auto true_residual = [&]() {
        int nb = outer_any(h, b_p, b_T, p, T, nullptr, nullptr, false, false, nullptr, nullptr,
                           nullptr, vp(R), vT(R));
        rc = enqueue_norms(h, nb, 0);
        if (rc == PT_OK) rc = sync(h, "BiCGStab residual");
        if (rc) return;
        const double *s = h->norms_host;
        rel[0] = s[2] > 0 ? std::sqrt(s[0] / s[2]) : std::sqrt(s[0]);
        rel[1] = s[3] > 0 ? std::sqrt(s[1] / s[3]) : std::sqrt(s[1]);
        if (inf.hist_len < PT_MAX_HIST) {
            inf.relres_hist[2 * inf.hist_len] = rel[0];
            inf.relres_hist[2 * inf.hist_len + 1] = rel[1];
            inf.hist_len++;
        }
    };
    double d[2];
    auto dot2 = [&](int x, int y, int z, int w) {
        h->begin(PT_K_OTHER, 8.0 * 4 * N * (z >= 0 ? 2 : 1));
        int nb = launch_dot2(N, vp(x), vT(x), vp(y), vT(y), z >= 0 ? vp(z) : nullptr,
                             z >= 0 ? vT(z) : nullptr, z >= 0 ? vp(w) : nullptr,
                             z >= 0 ? vT(w) : nullptr, h->partials(), st);
        launch_reduce4(h->partials(), nb, h->norms_devp + 8, st);
        h->end();
        rc = sync(h, "BiCGStab dot");
        d[0] = h->norms_host[8];
        d[1] = h->norms_host[9];
    };
    auto lin3 = [&](double *op, double *oT, double a, int x, double b, int y, double c, int z) {
        h->begin(PT_K_OTHER, 8.0 * 2 * N * (z >= 0 ? 4 : 3));
        launch_lin3(N, op, oT, a, vp(x), vT(x), b, vp(y), vT(y), c, z >= 0 ? vp(z) : nullptr,
                    z >= 0 ? vT(z) : nullptr, st);
        h->end();
    };
    auto precond = [&](int in, int out) {
        PT_DISPATCH(h, {
            pack_lv<R>(h, 0, true, vp(in), vT(in));
            vcycle<R>(h, 0, o.nu1, o.nu2);
            unpack_lv<R>(h, 0, false, vp(out), vT(out));
        });
        inf.cycles++;
    };
    auto matvec_neg = [&](int in, int out) {
        (void)outer_any(h, nullptr, nullptr, vp(in), vT(in), nullptr, nullptr, false, false,
                        nullptr, nullptr, nullptr, vp(out), vT(out));
    };
    auto done = [&]() {
        return rel[0] <= o.rtol && rel[1] <= o.rtol;
    };
    int status = PT_ERR_NOCONV;
    true_residual();
    if (rc) return rc;
    if (done()) status = PT_OK;
    if (status != PT_OK && std::isfinite(rel[0]) && std::isfinite(rel[1])) {
        lin3(vp(RH), vT(RH), 1.0, R, 0.0, R, 0.0, -1);
        launch_zero(vp(PV), 16 * (size_t)N, st);
        launch_zero(vp(VN), 16 * (size_t)N, st);
        double rho = 1.0, alpha = 1.0, omega = 1.0;
        for (;;) {
            if (inf.cycles + 2 > o.max_cycles) {
                h->err = "max_cycles reached";
                break;
            }
            dot2(RH, R, -1, -1);
            if (rc) return rc;
            const double rho1 = d[0];
            if (!(std::isfinite(rho1)) || rho1 == 0.0) {
                h->err = "BiCGStab breakdown (rho)";
                break;
            }
            const double beta = (rho1 / rho) * (alpha / omega);
            // p = r + beta (p - omega A p^), A p^ = -VN
            lin3(vp(PV), vT(PV), 1.0, R, beta, PV, beta * omega, VN);
            precond(PV, PH);
            matvec_neg(PH, VN);
            dot2(RH, VN, -1, -1);
            if (rc) return rc;
            const double rAp = -d[0];
            if (!(std::isfinite(rAp)) || rAp == 0.0) {
                h->err = "BiCGStab breakdown (r^ . A p)";
                break;
            }
            alpha = rho1 / rAp;
            lin3(vp(SV), vT(SV), 1.0, R, alpha, VN, 0.0, -1);   // s = r - alpha A p^
            precond(SV, SH);
            matvec_neg(SH, TN);
            dot2(TN, SV, TN, TN);
            if (rc) return rc;
            omega = d[1] > 0.0 ? -d[0] / d[1] : 0.0;             // (A s^ . s) / |A s^|^2
            // x += alpha p^ + omega s^
            h->begin(PT_K_OTHER, 8.0 * 2 * N * 4);
            launch_lin3(N, p, T, 1.0, p, T, alpha, vp(PH), vT(PH), omega, vp(SH), vT(SH), st);
            h->end();
            true_residual();
            if (rc) return rc;
            if (!std::isfinite(rel[0]) || !std::isfinite(rel[1])) {
                h->err = "residual norm is not finite";
                break;
            }
            if (done()) {
                status = PT_OK;
                break;
            }
            if (omega == 0.0) {
                h->err = "BiCGStab breakdown (omega)";
                break;
            }
            rho = rho1;
        }
    } else if (status != PT_OK) {
        h->err = "residual norm is not finite";
    }
    rc = sync(h, "BiCGStab");
    if (rc) return rc;
    h->last_updates = h->updates;
    inf.relres[0] = rel[0];
    inf.relres[1] = rel[1];
    inf.t_solve_s = elapsed(t0);
    inf.status = status;
    if (info) *info = inf;
    return status;
}

int pt_mg_smooth(pt_mg_t h, int level, const double *f_p, const double *f_T, double *u_p,
                 double *u_T, int sweeps)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (level < 0 || level >= h->P.nlev) return fail(h, PT_ERR_ARG, "level out of range");
    if (sweeps < 0 || !f_p || !f_T || !u_p || !u_T) return fail(h, PT_ERR_ARG, "bad arguments");
    PT_DISPATCH(h, {
        pack_lv<R>(h, level, true, f_p, f_T);
        pack_lv<R>(h, level, false, u_p, u_T);
        smooth<R>(h, level, sweeps, false);
        unpack_lv<R>(h, level, false, u_p, u_T);
    });
    return sync(h, "smooth");
}

int pt_mg_restrict_residual(pt_mg_t h, int level, const double *f_p, const double *f_T,
                            const double *u_p, const double *u_T, double *fc_p, double *fc_T)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (level < 0 || level + 1 >= h->P.nlev) return fail(h, PT_ERR_ARG, "level out of range");
    if (!f_p || !f_T || !u_p || !u_T || !fc_p || !fc_T) return fail(h, PT_ERR_ARG, "NULL field");
    PT_DISPATCH(h, {
        pack_lv<R>(h, level, true, f_p, f_T);
        pack_lv<R>(h, level, false, u_p, u_T);
        restrict_level<R>(h, level);
        unpack_lv<R>(h, level + 1, true, fc_p, fc_T);
    });
    return sync(h, "restrict_residual");
}

int pt_mg_prolong_add(pt_mg_t h, int level, const double *ec_p, const double *ec_T, double *u_p,
                      double *u_T)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (level < 0 || level + 1 >= h->P.nlev) return fail(h, PT_ERR_ARG, "level out of range");
    if (!ec_p || !ec_T || !u_p || !u_T) return fail(h, PT_ERR_ARG, "NULL field");
    PT_DISPATCH(h, {
        pack_lv<R>(h, level + 1, false, ec_p, ec_T);
        pack_lv<R>(h, level, false, u_p, u_T);
        prolong_level<R>(h, level);
        unpack_lv<R>(h, level, false, u_p, u_T);
    });
    return sync(h, "prolong_add");
}

int pt_mg_coarse_solve(pt_mg_t h, const double *f_p, const double *f_T, double *u_p, double *u_T)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (!f_p || !f_T || !u_p || !u_T) return fail(h, PT_ERR_ARG, "NULL field");
    const int l = h->P.nlev - 1;
    PT_DISPATCH(h, {
        pack_lv<R>(h, l, true, f_p, f_T);
        coarse_solve<R>(h);
        unpack_lv<R>(h, l, false, u_p, u_T);
    });
    return sync(h, "coarse_solve");
}

int pt_mg_vcycle(pt_mg_t h, const double *f_p, const double *f_T, double *e_p, double *e_T, int nu1,
                 int nu2)
{
    if (!h || !h->ready) return fail(h, PT_ERR_STATE, "handle not ready");
    if (!f_p || !f_T || !e_p || !e_T || nu1 < 0 || nu2 < 0 || nu1 > 8 || nu2 > 8)
        return fail(h, PT_ERR_ARG, "bad arguments");
    PT_DISPATCH(h, {
        pack_lv<R>(h, 0, true, f_p, f_T);
        vcycle<R>(h, 0, nu1, nu2);
        unpack_lv<R>(h, 0, false, e_p, e_T);
    });
    return sync(h, "vcycle");
}

// ------------------------------------------------------------ measurement
int pt_mg_set_timing(pt_mg_t h, int on)
{
    if (!h) return fail(nullptr, PT_ERR_ARG, "handle is NULL");
    h->timing = on == 0 ? 0u : (on == 1 ? (1u << PT_K_COUNT) - 1u : (unsigned)on >> 1);
    return PT_OK;
}

int pt_mg_kernel_stats(pt_mg_t h, int cls, long *launches, double *ms, double *bytes)
{
    if (!h) return fail(nullptr, PT_ERR_ARG, "handle is NULL");
    if (cls < 0 || cls >= PT_K_COUNT) return fail(h, PT_ERR_ARG, "kernel class out of range");
    if (launches) *launches = h->launches[cls];
    if (ms) *ms = h->ms[cls];
    if (bytes) *bytes = h->bytes[cls];
    return PT_OK;
}

int pt_mg_timed_stats(pt_mg_t h, int cls, long *launches, double *ms, double *bytes)
{
    if (!h) return fail(nullptr, PT_ERR_ARG, "handle is NULL");
    if (cls < 0 || cls >= PT_K_COUNT) return fail(h, PT_ERR_ARG, "kernel class out of range");
    h->flush_timing();
    if (launches) *launches = h->timed_launches[cls];
    if (ms) *ms = h->ms[cls];
    if (bytes) *bytes = h->timed_bytes[cls];
    return PT_OK;
}

int pt_mg_reset_stats(pt_mg_t h)
{
    if (!h) return fail(nullptr, PT_ERR_ARG, "handle is NULL");
    for (int c = 0; c < PT_K_COUNT; c++) {
        h->launches[c] = 0;
        h->ms[c] = 0;
        h->bytes[c] = 0;
        h->timed_launches[c] = 0;
        h->timed_bytes[c] = 0;
        h->runs[c] = 0;
    }
    return PT_OK;
}

long long pt_mg_last_cell_updates(pt_mg_t h) { return h ? h->last_updates : 0; }

int pt_mg_set_option(pt_mg_t h, int option, int value)
{
    if (!h) return fail(nullptr, PT_ERR_ARG, "handle is NULL");
    if (option == PT_OPT_GRAPHS) h->use_graphs = value != 0;
    else if (option == PT_OPT_TAIL) h->use_tail = value != 0;
    else if (option == PT_OPT_FUSED) h->use_fused = value != 0;
    else if (option == PT_OPT_SPECULATE) h->speculate = value != 0;
    else if (option == PT_OPT_COARSE_SWEEPS) {
        const int a = value >> 4, b = value & 15;
        if (value != 0 && (value < 0 || value > 255 || a > 8 || b > 8 || a + b == 0))
            return fail(h, PT_ERR_ARG, "PT_OPT_COARSE_SWEEPS: 16 nu1 + nu2 with nu <= 8, or 0");
        h->coarse_nu = value;
    } else if (option == PT_OPT_TAIL_CELLS) {
        if (value < 0) return fail(h, PT_ERR_ARG, "PT_OPT_TAIL_CELLS must be >= 0");
        h->tail_max_cells = value;
        plan_tail(h);
    }
    else if (option == PT_OPT_TIMING_EVERY) {
        if (value < 1) return fail(h, PT_ERR_ARG, "PT_OPT_TIMING_EVERY must be >= 1");
        h->timing_every = value;
    } else if (option == PT_OPT_W_LEVELS) {
        if (value < 0) return fail(h, PT_ERR_ARG, "PT_OPT_W_LEVELS must be >= 0");
        h->w_levels = value;
    } else if (option == PT_OPT_OMEGA) {
        if (value < 1 || value > 1999) return fail(h, PT_ERR_ARG, "PT_OPT_OMEGA must be in 1..1999");
        h->omega_milli = value;
    } else return fail(h, PT_ERR_ARG, "unknown option");
    return PT_OK;
}

int pt_mg_get_option(pt_mg_t h, int option)
{
    if (!h) return -1;
    if (option == PT_OPT_GRAPHS) return h->use_graphs ? 1 : 0;
    if (option == PT_OPT_FUSED) return h->use_fused ? 1 : 0;
    if (option == PT_OPT_TIMING_EVERY) return h->timing_every;
    if (option == PT_OPT_SPECULATE) return h->speculate ? 1 : 0;
    if (option == PT_OPT_TAIL) return (h->use_tail && h->tail_lt > 0) ? h->P.nlev - h->tail_lt : 0;
    if (option == PT_OPT_TAIL_CELLS) return (int)h->tail_max_cells;
    if (option == PT_OPT_COARSE_SWEEPS) return h->coarse_nu;
    if (option == PT_OPT_W_LEVELS) return h->w_levels;
    if (option == PT_OPT_OMEGA) return h->omega_milli;
    return -1;
}

int pt_copy_kernel(void *dst, const void *src, size_t bytes, void *hip_stream)
{
    if ((!dst || !src) && bytes) return fail(nullptr, PT_ERR_ARG, "NULL pointer");
    launch_copy(dst, src, bytes, (hipStream_t)hip_stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, PT_ERR_HIP, hipGetErrorString(e));
    return PT_OK;
}
