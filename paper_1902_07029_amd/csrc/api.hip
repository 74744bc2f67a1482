// C ABI of the lsmg library: hierarchy construction, the Newton / Crank-Nicolson
// driver (section 3.4), the V-cycle driver (section 3.5) and the component entry
// points used by the parity tests.  All device work is enqueued on the
// hierarchy's stream; host decisions (cycle and Newton stopping) read max-norms
// back through pinned memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hier.hpp"

namespace lsmg {

namespace {
thread_local std::string g_err;
}

lsmg_status fail(lsmg_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}


int ipow(int b, int e)
{
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

lsmg_status check_params(const lsmg_params *p)
{
    if (!p) return fail(LSMG_EINVAL, "params is NULL");
    if (!(p->tau_s > 0.0) || p->nu1 < 0 || p->nu2 < 0 || p->ghost_sweeps < 0 || p->ghost_sweeps_coarse < 0 ||
        !(p->sweeps_lambda >= 0.0) || p->band_steps < 0 ||
        p->band_steps > 3 || p->coarsest_n < 3 || p->newton_max < 1 || p->cycles_max < 1 ||
        !(p->lin_rtol > 0.0) || !(p->newton_tol > 0.0) || (p->precision != 0 && p->precision != 1) ||
        (p->bc != 0 && p->bc != 1) || p->cycle_gamma < 1 || p->cycle_gamma > 2 || p->fmg < 0 || p->fmg > 2 ||
        (p->fused_sweep != 0 && p->fused_sweep != 1) || p->krylov_m < 0 || p->krylov_m > 200)
        return fail(LSMG_EINVAL, "invalid solver parameters");
    return LSMG_OK;
}

// relaxation parameter of the ghost rows of level l: tau_s for Dirichlet rows
// (eq. CFLcond); for Neumann rows tau_s times the bound of eq. CFLcondN,
// 2 sqrt(2) h / 3, in 3-D the same bound over three axes, 4 h / (3 sqrt(3))
double tau_level(const lsmg_hierarchy *H, int l)
{
    const double h = H->L[l].h, t = H->p.tau_s;
    if (H->p.bc == 0) return t;
    return H->dim == 2 ? t * (2.0 * std::sqrt(2.0) * h / 3.0) : t * (4.0 * h / (3.0 * std::sqrt(3.0)));
}

void fill_desc_scalars(lsmg_hierarchy *H)
{
    const lsmg_params &p = H->p;
    for (int l = 0; l < H->nlev; ++l) {
        const Level &Lv = H->L[l];
        LevelDesc<double> &D = H->hd64[l];
        D.kap = p.d / (4.0 * Lv.h * Lv.h);
        D.d_half_h2 = p.d / (2.0 * Lv.h * Lv.h);
        D.alpha = p.alpha;
        D.beta = p.beta;
        D.dt_inv = H->dt > 0.0 ? 1.0 / H->dt : 0.0;
        D.ks_half = 0.5 * (p.a / p.m_c);
        D.kc_half = 0.5 * (p.a / p.m_s);
        D.tau_s = tau_level(H, l);
        D.ghost_c_new = p.ghost_c_new;
        if (H->have32) {
            LevelDesc<float> &E = H->hd32[l];
            E.kap = (float)D.kap;
            E.d_half_h2 = (float)D.d_half_h2;
            E.alpha = (float)D.alpha;
            E.beta = (float)D.beta;
            E.dt_inv = (float)D.dt_inv;
            E.ks_half = (float)D.ks_half;
            E.kc_half = (float)D.kc_half;
            E.tau_s = (float)D.tau_s;
            E.ghost_c_new = D.ghost_c_new;
        }
    }
}

lsmg_status push_desc(lsmg_hierarchy *H)
{
    fill_desc_scalars(H);
    HIPCHK(hipMemcpyAsync(H->d64, H->hd64.data(), sizeof(LevelDesc<double>) * H->nlev, hipMemcpyHostToDevice,
                          H->stream));
    if (H->have32)
        HIPCHK(hipMemcpyAsync(H->d32, H->hd32.data(), sizeof(LevelDesc<float>) * H->nlev, hipMemcpyHostToDevice,
                              H->stream));
    // the host copies must stay unchanged until the copies ran
    HIPCHK(hipStreamSynchronize(H->stream));
    return LSMG_OK;
}

// ghost relaxations per smoothing step on level l: ghost_sweeps, or
// ghost_sweeps_coarse where the level's diffusion number d dt / h^2 is below
// sweeps_lambda (mass-dominated levels, where the inside rows hardly couple to
// the ghosts and the boundary error is removed by the ghost relaxation alone)
int level_sweeps(const lsmg_hierarchy *H, int l)
{
    const double hl = H->L[l].h;
    if (H->dt > 0.0 && H->p.d * H->dt / (hl * hl) < H->p.sweeps_lambda) return H->p.ghost_sweeps_coarse;
    return H->p.ghost_sweeps;
}

lsmg_status build_ghost_ops(lsmg_hierarchy *H, int l);
void make_descs(lsmg_hierarchy *H);
lsmg_status upload_tail_args(lsmg_hierarchy *H);

// recomputes every level's sweep count (force: rebuild every composed map)
lsmg_status update_sweeps(lsmg_hierarchy *H, bool force)
{
    bool changed = false;
    for (int l = 0; l < H->nlev; ++l) {
        const int S = level_sweeps(H, l);
        if (!force && S == H->L[l].sweeps) continue;
        H->L[l].sweeps = S;
        LSMGCHK(build_ghost_ops(H, l));
        changed = true;
    }
    if (changed) {
        make_descs(H);
        LSMGCHK(upload_tail_args(H));
    }
    return LSMG_OK;
}

lsmg_status set_dt(lsmg_hierarchy *H, double dt)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(LSMG_EINVAL, "dt must be positive and finite");
    if (dt != H->dt) {
        H->dt = dt;
        LSMGCHK(update_sweeps(H, false));
        LSMGCHK(push_desc(H));
    }
    return LSMG_OK;
}

// norm k lives in kNormSlots partial slots starting at d_norms + k * kNormSlots
unsigned long long *norm_slot(lsmg_hierarchy *H, int k) { return H->d_norms + k * kNormSlots; }

void zero_norms(lsmg_hierarchy *H, int first, int count, hipStream_t s = nullptr)
{
    launch_zero_u64(norm_slot(H, first), count * kNormSlots, s ? s : H->stream);
}

lsmg_status read_norms(lsmg_hierarchy *H, int count)
{
    HIPCHK(hipMemcpyAsync(H->h_norms, H->d_norms, sizeof(unsigned long long) * count * kNormSlots,
                          hipMemcpyDeviceToHost, H->stream));
    HIPCHK(hipStreamSynchronize(H->stream));
    return LSMG_OK;
}

double norm_value(const lsmg_hierarchy *H, int k)
{
    unsigned long long m = 0;
    for (int i = 0; i < kNormSlots; ++i) m = H->h_norms[k * kNormSlots + i] > m ? H->h_norms[k * kNormSlots + i] : m;
    double v;
    std::memcpy(&v, &m, sizeof(double));
    return v;
}

// ---------------------------------------------------------------------------
// launch timing: each launch of the selected kernel class on the selected level
// carries a pair of events that its own dispatch records
// ---------------------------------------------------------------------------
inline bool prof_on(const lsmg_hierarchy *H, int kernel, int l)
{
    return H->prof_kernel == kernel && H->prof_level == l;
}

Exec prof_exec(lsmg_hierarchy *H, hipStream_t s, int kernel, int l)
{
    Exec x(s);
    if (!prof_on(H, kernel, l)) return x;
    while (H->prof_pool.size() < H->prof_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return x;
        H->prof_pool.push_back(e);
    }
    x.ev0 = H->prof_pool[H->prof_used++];
    x.ev1 = H->prof_pool[H->prof_used++];
    return x;
}

// sum of the event pairs [first, last) into the accumulators
void prof_collect(lsmg_hierarchy *H, size_t first, size_t last)
{
    for (size_t i = first; i + 1 < last; i += 2) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, H->prof_pool[i], H->prof_pool[i + 1]) == hipSuccess) {
            H->prof_acc_ms += ms;
            ++H->prof_acc_n;
        }
    }
}

// ---------------------------------------------------------------------------
// V-cycle
// ---------------------------------------------------------------------------
template <typename T>
const LevelDesc<T> *descs(const lsmg_hierarchy *H);
template <>
const LevelDesc<double> *descs<double>(const lsmg_hierarchy *H) { return H->d64; }
template <>
const LevelDesc<float> *descs<float>(const lsmg_hierarchy *H) { return H->d32; }

// `count` smoothing steps on level l (section 3.5.1: a collective red-black
// sweep, then the ghost relaxation)
template <typename T>
void smooth_level(lsmg_hierarchy *H, int l, hipStream_t s, int count)
{
    const Level &Lv = H->L[l];
    const LevelDesc<T> *d = descs<T>(H);
    if (Lv.gc_ptr) {
        // 2-D, folded ghost map.  Pairs of steps with fused sweeps (on levels small
        // enough for launch latency to dominate): the first reads the corrections'
        // first copy and writes the second, the folded map then works on the
        // second, and the next step returns to the first
        if (H->p.fused_sweep && Lv.tiles && fuse_sweep(Lv.na, sizeof(T))) {
            for (; count >= 2; count -= 2) {
                for (int flip = 0; flip < 2; ++flip) {
                    launch_smooth_rb<T>(d, Lv.tiles, Lv.ntile, Lv.w_gh(), Lv.nghc, flip,
                                        prof_exec(H, s, LSMG_KERNEL_SMOOTH, l));
                    launch_ghost_apply<T>(H->dim, d, Lv.w_gh4(), Lv.nghc4, 1 - flip,
                                          with_tail(prof_exec(H, s, LSMG_KERNEL_GHOST, l), Lv.nghc4));
                }
            }
        }
        // one launch per colour: the black launch also snapshots the ghosts' delta s
        // (its list is followed by the ghost items), then one launch applies the map
        for (; count > 0; --count) {
            launch_smooth_colour<T>(H->dim, d, Lv.w_seg(0), Lv.nseg[0], 0, prof_exec(H, s, LSMG_KERNEL_SMOOTH, l));
            launch_smooth_colour<T>(H->dim, d, Lv.w_seg(1), Lv.nseg[1] + Lv.nghc, 1,
                                    with_tail(prof_exec(H, s, LSMG_KERNEL_SMOOTH, l), Lv.nghc));
            launch_ghost_apply<T>(H->dim, d, Lv.w_gh4(), Lv.nghc4, 0,
                                  with_tail(prof_exec(H, s, LSMG_KERNEL_GHOST, l), Lv.nghc4));
        }
        return;
    }
    for (; count > 0; --count) {
        for (int colour = 0; colour < 2; ++colour)
            launch_smooth_colour<T>(H->dim, d, Lv.w_seg(colour), Lv.nseg[colour], colour,
                                    prof_exec(H, s, LSMG_KERNEL_SMOOTH, l));
        const Exec xb = prof_exec(H, s, LSMG_KERNEL_GHOST, l);
        const Exec xa = with_tail(prof_exec(H, s, LSMG_KERNEL_GHOST, l), Lv.nghc4);
        launch_ghost<T>(H->dim, d, l, Lv.w_gh(), Lv.nghc, Lv.w_gh4(), Lv.nghc4, Lv.ng, Lv.sweeps,
                        Lv.go_ptr != nullptr, xb, xa);
    }
}

TailArgs tail_args(const lsmg_hierarchy *H, int l0, int d0)
{
    TailArgs a{};
    a.d0 = d0;
    a.l0 = l0;
    a.nlev = H->nlev;
    a.nu1 = H->p.nu1;
    a.nu2 = H->p.nu2;
    a.gamma = H->p.cycle_gamma;
    a.c2s = H->L[H->nlev - 1].c2s;
    a.ainv = H->ainv;
    int off = 0;
    for (int l = 0; l < H->nlev; ++l) {
        const Level &Lv = H->L[l];
        a.lev[l].in_ijk = Lv.in_ijk;
        a.lev[l].nin0 = Lv.nin[0];
        a.lev[l].nin1 = Lv.nin[1];
        a.lev[l].sweeps = Lv.sweeps;
        a.lev[l].soff = l >= l0 ? off : 0;
        if (l >= l0) off += Lv.nin[0] + Lv.nin[1] + 2 * Lv.ng + 1;
    }
    a.nstage = off;
    if (H->tail_lds) {
        a.tab = H->tail_tab;
        a.tab_words = H->tail_sz.tab_words;
        a.nvals = H->tail_sz.nvals;
        a.nints = H->tail_sz.nints;
        a.ngmax = H->tail_sz.ngmax;
        a.ncoarse = H->tail_sz.ncoarse;
        for (int l = H->tail_l0; l < H->nlev; ++l) a.ll[l] = H->tail_ll[l];
    }
    // which tail kernel runs it (the same one alone and in a batch)
    a.lds = (tail_in_lds<double>(H) ? 1 : 0) | (tail_in_lds<float>(H) ? 2 : 0);
    return a;
}

template <typename T>
void vcycle_rec(lsmg_hierarchy *H, int l, hipStream_t s)
{
    const Level &Lv = H->L[l];
    const LevelDesc<T> *d = descs<T>(H);
    if (l >= H->tail_l0) {
        // the coarsest factorisation forked off in this captured cycle joins here
        if (H->join_pending) {
            (void)hipStreamWaitEvent(s, H->ev_join, 0);
            H->join_pending = false;
        }
        // this level and every coarser one in one workgroup
        if (tail_in_lds<T>(H))
            launch_tail_lds<T>(H->dim, d, H->d_tail + l, 1, H->tail_sz.bytes<T>(), Exec(s));
        else
            launch_tail<T>(H->dim, d, H->d_tail + l, 1, H->L[H->nlev - 1].na,
                           tail_args(H, l, 0).nstage <= kTailStageInts, Exec(s));
        return;
    }
    smooth_level<T>(H, l, s, H->p.nu1);
    launch_defect<T>(H->dim, d, Lv.w_act(), Lv.nw_act(), -1, with_tail(prof_exec(H, s, LSMG_KERNEL_DEFECT, l), Lv.nghc));
    launch_band<T>(d, Lv.w_band(), Lv.nbandc, Exec(s));
    const Level &C = H->L[l + 1];
    launch_restrict<T>(H->dim, d, C.w_act(), C.nw_act(), with_tail(prof_exec(H, s, LSMG_KERNEL_RESTRICT, l + 1), C.nghc));
    // W-cycle: a second cycle on the next level from the first one's result; the
    // coarsest solve is exact, so it is not repeated
    const int reps = l + 1 == H->nlev - 1 ? 1 : H->p.cycle_gamma;
    for (int i = 0; i < reps; ++i) vcycle_rec<T>(H, l + 1, s);
    launch_prolong<T>(H->dim, d, Lv.w_act(), Lv.nw_act(), with_tail(prof_exec(H, s, LSMG_KERNEL_PROLONG, l), Lv.nghc));
    smooth_level<T>(H, l, s, H->p.nu2);
}

// full multigrid from a zero correction on level 0: the right-hand side
// restricted level by level (the defect of a zero correction is the right-hand
// side; the restriction clears the coarser correction), the coarsest problem
// solved, then on every finer level the prolongated coarser solution is the
// start of one cycle
template <typename T>
void fmg_enqueue(lsmg_hierarchy *H, hipStream_t s)
{
    const LevelDesc<T> *d = descs<T>(H);
    const int L = H->nlev;
    for (int l = 0; l + 1 < L; ++l) {
        const Level &Lv = H->L[l], &C = H->L[l + 1];
        launch_defect<T>(H->dim, d, Lv.w_act(), Lv.nw_act(), -1, with_tail(Exec(s), Lv.nghc));
        launch_band<T>(d, Lv.w_band(), Lv.nbandc, Exec(s));
        launch_restrict<T>(H->dim, d, C.w_act(), C.nw_act(), with_tail(Exec(s), C.nghc));
    }
    vcycle_rec<T>(H, L - 1, s);
    for (int l = L - 2; l >= 0; --l) {
        launch_prolong<T>(H->dim, d, H->L[l].w_act(), H->L[l].nw_act(), with_tail(Exec(s), H->L[l].nghc));
        vcycle_rec<T>(H, l, s);
    }
}

// one linear-solve iteration on level 0: a V-cycle on the correction (FP64), or
// an FP32 V-cycle on the current FP64 defect added to the FP64 correction; then
// the FP64 defect and its norm in slot 1.  fmg: a full-multigrid pass instead of
// the cycle (the correction is zero then)
void cycle_enqueue(lsmg_hierarchy *H, bool mixed, hipStream_t s, bool fmg = false)
{
    const Level &L0 = H->L[0];
    zero_norms(H, 1, 1, s);
    if (!mixed) {
        if (fmg) fmg_enqueue<double>(H, s);
        else vcycle_rec<double>(H, 0, s);
    } else {
        // the FP32 right-hand side and zero correction were written by the FP64
        // defect that precedes every cycle
        if (fmg) fmg_enqueue<float>(H, s);
        else vcycle_rec<float>(H, 0, s);
        launch_add_f32(H->dim, H->d64, H->d32, L0.w_act(), L0.nw_act(), with_tail(Exec(s), L0.nghc));
    }
    launch_defect<double>(H->dim, H->d64, L0.w_act(), L0.nw_act(), 1, with_tail(Exec(s), L0.nghc),
                          mixed ? H->d32 : nullptr);
}

void invalidate_graphs(lsmg_hierarchy *H)
{
    for (int i = 0; i < 8; ++i) {
        if (H->gexec[i]) (void)hipGraphExecDestroy(H->gexec[i]);
        H->gexec[i] = nullptr;
    }
}

// capture the cycle of precision `mixed` (fmg: the full-multigrid iteration;
// factor: the first cycle after a linearisation, with the coarsest operator
// factorised on a side stream while the fine levels run, joined before the
// coarse tail) once; replays run on the hierarchy's stream
lsmg_status cycle_graph(lsmg_hierarchy *H, bool mixed, hipGraphExec_t *out, bool fmg = false, bool factor = false)
{
    const int gi = (mixed ? 1 : 0) + (fmg ? 2 : 0) + (factor ? 4 : 0);
    if (!H->gexec[gi]) {
        if (!H->cap) HIPCHK(hipStreamCreateWithFlags(&H->cap, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(H->cap, hipStreamCaptureModeThreadLocal));
        if (factor) {
            if (!H->side) HIPCHK(hipStreamCreateWithFlags(&H->side, hipStreamNonBlocking));
            if (!H->ev_fork) HIPCHK(hipEventCreateWithFlags(&H->ev_fork, hipEventDisableTiming));
            if (!H->ev_join) HIPCHK(hipEventCreateWithFlags(&H->ev_join, hipEventDisableTiming));
            HIPCHK(hipEventRecord(H->ev_fork, H->cap));
            HIPCHK(hipStreamWaitEvent(H->side, H->ev_fork, 0));
            launch_coarse_factor(H->dim, H->d64, H->d_coarse, 1, H->L[H->nlev - 1].na, Exec(H->side));
            HIPCHK(hipEventRecord(H->ev_join, H->side));
            H->join_pending = true;
        }
        cycle_enqueue(H, mixed, H->cap, fmg);
        if (H->join_pending) {
            // every cycle reaches the tail; joined here all the same before the capture ends
            HIPCHK(hipStreamWaitEvent(H->cap, H->ev_join, 0));
            H->join_pending = false;
        }
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamEndCapture(H->cap, &g));
        hipError_t e = hipGraphInstantiate(&H->gexec[gi], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(LSMG_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    *out = H->gexec[gi];
    return LSMG_OK;
}

// linearisation on every level from level 0's (s, c); factors the coarsest
// operator unless the caller's first cycle does it (factor = false)
lsmg_status linearize(lsmg_hierarchy *H, bool factor = true)
{
    for (int l = 1; l < H->nlev; ++l) {
        const Level &C = H->L[l];
        launch_inject<double>(H->dim, H->d64, C.w_act(), C.nw_act(), with_tail(Exec(H->stream), C.nghc));
    }
    if (H->have32)
        for (int l = 0; l < H->nlev; ++l) {
            const Level &Lv = H->L[l];
            launch_to_f32(H->dim, H->d64, H->d32, Lv.w_act(), Lv.nw_act(), 0, with_tail(Exec(H->stream), Lv.nghc));
        }
    if (factor) launch_coarse_factor(H->dim, H->d64, H->d_coarse, 1, H->L[H->nlev - 1].na, H->stream);
    H->lin_set = true;
    return LSMG_OK;
}

lsmg_status check_factor(lsmg_hierarchy *H)
{
    HIPCHK(hipMemcpyAsync(H->h_status, H->lu_status, sizeof(int), hipMemcpyDeviceToHost, H->stream));
    HIPCHK(hipStreamSynchronize(H->stream));
    if (*H->h_status != 0) return fail(LSMG_ENONFINITE, "coarsest operator is singular or not finite");
    return LSMG_OK;
}

// ---------------------------------------------------------------------------
// hierarchy construction
// ---------------------------------------------------------------------------
lsmg_status build_level_arrays(lsmg_hierarchy *H, int l, const double *phi, uint8_t *fin, uint8_t *fgh,
                               int64_t *scratch, int nscratch, int *err)
{
    Level &Lv = H->L[l];
    const int dim = H->dim;
    const long long nn = (long long)Lv.n * Lv.n * (dim == 3 ? Lv.n : 1);
    LSMGCHK(H->zalloc(&Lv.type, Lv.ssize));
    LSMGCHK(H->zalloc(&Lv.ext, Lv.ssize));
    LSMGCHK(H->alloc(&Lv.cmap, Lv.ssize));
    launch_fill<int>(Lv.cmap, Lv.ssize, -1, H->stream);
    launch_classify(dim, phi, Lv.n, Lv.Wp, Lv.cs, Lv.type, fin, fgh, err, H->stream);
    const int ni = compact_flags(fin, nn, nullptr, scratch, nscratch, H->stream);
    const int ng = compact_flags(fgh, nn, nullptr, scratch, nscratch, H->stream);
    if (ni < 0 || ng < 0) return fail(LSMG_EHIP, "compaction failed on level %d", l);
    Lv.ni = ni;
    Lv.ng = ng;
    Lv.na = ni + ng;
    LSMGCHK(H->alloc(&Lv.c2g, Lv.na));
    LSMGCHK(H->alloc(&Lv.c2s, Lv.na));
    if (ni > 0) compact_flags(fin, nn, Lv.c2g, scratch, nscratch, H->stream);
    if (ng > 0) compact_flags(fgh, nn, Lv.c2g + ni, scratch, nscratch, H->stream);
    launch_c2s(dim, Lv.c2g, Lv.na, Lv.n, Lv.Wp, Lv.cs, Lv.c2s, Lv.cmap, H->stream);
    LSMGCHK(H->alloc(&Lv.in_ijk, ni));
    if (build_inside_lists(dim, Lv.c2g, ni, Lv.n, Lv.in_ijk, Lv.nin, scratch, nscratch, H->mem, H->stream) != 0)
        return fail(LSMG_EHIP, "inside-node lists failed on level %d", l);
    // ghost geometry
    const int nst = H->nst;
    LSMGCHK(H->alloc(&Lv.g_idx, ng));
    LSMGCHK(H->alloc(&Lv.g_ijk, ng));
    LSMGCHK(H->alloc(&Lv.g_stg, (long long)ng * nst));
    LSMGCHK(H->alloc(&Lv.g_st, (long long)ng * nst));
    LSMGCHK(H->alloc(&Lv.g_stc, (long long)ng * nst));
    LSMGCHK(H->alloc(&Lv.g_w, (long long)ng * nst));
    LSMGCHK(H->alloc(&Lv.g_B, (long long)ng * dim));
    LSMGCHK(H->alloc(&Lv.g_nrm, (long long)ng * dim));
    LSMGCHK(H->alloc(&Lv.g_nrow, (long long)ng * dim));
    LSMGCHK(H->alloc(&Lv.g_order, ng));
    LSMGCHK(H->alloc(&Lv.g_bfall, ng));
    LSMGCHK(H->zalloc(&Lv.g_buf0, ng));
    LSMGCHK(H->zalloc(&Lv.g_buf1, ng));
    launch_ghost_geometry(dim, l, H->p.bc, phi, Lv.type, Lv.c2g + ni, Lv.cmap, ni, ng, Lv.n, Lv.Wp, Lv.cs, H->lo,
                          Lv.h, Lv.g_idx, Lv.g_ijk, Lv.g_st, Lv.g_stg, Lv.g_stc, Lv.g_w, Lv.g_B, Lv.g_nrm, Lv.g_nrow,
                          Lv.g_order, Lv.g_bfall, err, H->stream);
    launch_ghost_ext(ng, Lv.g_idx, Lv.ext, H->stream);
    // vectors
    LSMGCHK(H->zalloc(&Lv.s, Lv.ssize));
    LSMGCHK(H->zalloc(&Lv.c, Lv.ssize));
    LSMGCHK(H->zalloc(&Lv.rhs_s, Lv.ssize));
    LSMGCHK(H->zalloc(&Lv.rhs_c, Lv.ssize));
    LSMGCHK(H->zalloc(&Lv.x_s, Lv.ssize));
    LSMGCHK(H->zalloc(&Lv.x_c, Lv.ssize));
    LSMGCHK(H->zalloc(&Lv.r_s, Lv.ssize));
    LSMGCHK(H->zalloc(&Lv.r_c, Lv.ssize));
    if (dim == 2) {
        LSMGCHK(H->zalloc(&Lv.x2_s, Lv.ssize));
        LSMGCHK(H->zalloc(&Lv.x2_c, Lv.ssize));
    }
    return LSMG_OK;
}

lsmg_status build_band(lsmg_hierarchy *H, int l, const double *phi, uint8_t *flag, int64_t *scratch, int nscratch)
{
    Level &F = H->L[l];
    const Level &C = H->L[l + 1];
    const int dim = H->dim;
    const long long nn = (long long)F.n * F.n * (dim == 3 ? F.n : 1);
    HIPCHK(hipMemsetAsync(flag, 0, (size_t)nn, H->stream));
    launch_band_mark(dim, C.c2g + C.ni, C.ng, C.n, F.type, F.n, F.Wp, F.cs, flag, H->stream);
    const int nb = compact_flags(flag, nn, nullptr, scratch, nscratch, H->stream);
    if (nb < 0) return fail(LSMG_EHIP, "band compaction failed on level %d", l);
    F.nb = nb;
    F.bmax = ipow(dim, H->p.band_steps);
    if (nb == 0) return LSMG_OK;
    int64_t *band = nullptr;
    int *bandid = nullptr, *up_s = nullptr, *up_b = nullptr, *blayer = nullptr;
    double *up_w = nullptr;
    DevTemps tmp(H->mem, H->stream);
    LSMGCHK(tmp.get(&band, nb));
    LSMGCHK(tmp.get(&bandid, nn));
    LSMGCHK(tmp.get(&up_s, (long long)nb * dim));
    LSMGCHK(tmp.get(&up_b, (long long)nb * dim));
    LSMGCHK(tmp.get(&up_w, (long long)nb * dim));
    LSMGCHK(tmp.get(&blayer, nb));
    compact_flags(flag, nn, band, scratch, nscratch, H->stream);
    launch_fill<int>(bandid, nn, -1, H->stream);
    launch_fill_bandid(band, nb, bandid, H->stream);
    LSMGCHK(H->alloc(&F.b_idx, nb));
    LSMGCHK(H->zalloc(&F.b_cnt, nb));
    LSMGCHK(H->zalloc(&F.b_src, (long long)nb * (F.bmax > 0 ? F.bmax : 1)));
    LSMGCHK(H->zalloc(&F.b_wt, (long long)nb * (F.bmax > 0 ? F.bmax : 1)));
    HIPCHK(hipMemsetAsync(blayer, 0, sizeof(int) * nb, H->stream));
    launch_band_geometry(dim, phi, band, nb, F.type, bandid, F.n, F.Wp, F.cs, F.h, up_s, up_b, up_w, F.b_idx,
                         H->stream);
    for (int layer = 1; layer <= H->p.band_steps; ++layer)
        launch_band_layer(dim, layer, nb, F.bmax, up_s, up_b, up_w, blayer, F.b_cnt, F.b_src, F.b_wt, H->stream);
    launch_band_ext(nb, F.b_idx, blayer, F.ext, H->stream);
    HIPCHK(hipStreamSynchronize(H->stream));
    return LSMG_OK;
}

// tiles of the fused 2-D sweep: kRbRows rows x 64 positions holding an inside or
// ghost node of either colour
lsmg_status build_tiles(lsmg_hierarchy *H, int l)
{
    Level &Lv = H->L[l];
    std::vector<uint8_t> type((size_t)Lv.ssize);
    HIPCHK(hipMemcpyAsync(type.data(), Lv.type, type.size(), hipMemcpyDeviceToHost, H->stream));
    HIPCHK(hipStreamSynchronize(H->stream));
    std::vector<int4> tiles;
    for (long long y0 = 0; y0 < Lv.rows; y0 += kRbRows)
        for (int p0 = 0; p0 < Lv.Wp; p0 += kWave) {
            bool any = false;
            for (int c = 0; c < 2 && !any; ++c)
                for (long long y = y0; y < y0 + kRbRows && y < Lv.rows && !any; ++y)
                    for (int p = p0; p < p0 + kWave && p < Lv.Wp; ++p) {
                        const uint8_t t = type[(size_t)(c * Lv.cs + y * Lv.Wp + p)];
                        if (t == kIn || t == kGhost) {
                            any = true;
                            break;
                        }
                    }
            if (any) tiles.push_back(make_int4(l << 2, (int)y0, p0, 0));
        }
    Lv.ntile = (int)tiles.size();
    if (tiles.empty()) return LSMG_OK;
    LSMGCHK(H->alloc(&Lv.tiles, Lv.ntile));
    HIPCHK(hipMemcpyAsync(Lv.tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, H->stream));
    HIPCHK(hipStreamSynchronize(H->stream));
    return LSMG_OK;
}

lsmg_status build_items(lsmg_hierarchy *H, int l)
{
    Level &Lv = H->L[l];
    int4 *seg[2] = {nullptr, nullptr};
    int cnt[2] = {0, 0};
    // 3-D: items of two bricks of one colour (consecutive along x) holding an inside
    // node, with the bits of their inside nodes, so that a wavefront reads whole
    // 128-byte lines of the brick layout.  Items in Morton (Z) order of the pair's
    // (x, y, z) brick coordinates: a launch deals each XCD a contiguous eighth of
    // the list (logical_block), which is then a compact piece of the domain, and
    // the lines of the other colour that two XCDs both fetch are those along the
    // pieces' faces.  (In storage order the eighths are thin z slabs of the domain,
    // whose large faces made the torus's finest FP32 sweep fetch 1.4x its bytes.)
    std::vector<int4> bricks;
    if (H->dim == 3) {
        const int np = brick_np(Lv.Wp), nj = brick_nj(Lv.n), nk = brick_nk(Lv.n);
        if (np > 1024 || nj > 1024 || nk > 1024) return fail(LSMG_EINVAL, "3-D grids hold at most 2047 nodes per axis");
        std::vector<uint8_t> ty((size_t)Lv.ssize);
        HIPCHK(hipMemcpyAsync(ty.data(), Lv.type, ty.size(), hipMemcpyDeviceToHost, H->stream));
        HIPCHK(hipStreamSynchronize(H->stream));
        auto spread3 = [](unsigned v) {
            unsigned long long r = 0;
            for (int b = 0; b < 10; ++b) r |= (unsigned long long)((v >> b) & 1u) << (3 * b);
            return r;
        };
        for (int c = 0; c < 2; ++c) {
            std::vector<std::pair<unsigned long long, int4>> keyed;
            for (int kb = 0; kb < nk; ++kb)
                for (int jb = 0; jb < nj; ++jb)
                    for (int pb = 0; pb < np; pb += 2) {
                        unsigned m[2] = {0u, 0u};
                        for (int h = 0; h < 2 && pb + h < np; ++h) {
                            const size_t base = (size_t)(c * Lv.cs + ((((long long)kb * nj + jb) * np + pb + h) << 5));
                            for (int in = 0; in < 32; ++in)
                                if (ty[base + in] == kIn) m[h] |= 1u << in;
                        }
                        if (m[0] | m[1]) {
                            const unsigned long long key =
                                spread3((unsigned)(pb >> 1)) | spread3((unsigned)jb) << 1 | spread3((unsigned)kb) << 2;
                            keyed.push_back({key, make_int4((l << 2) | c, pb | (jb << 10) | (kb << 20), (int)m[0],
                                                            (int)m[1])});
                        }
                    }
            std::sort(keyed.begin(), keyed.end(),
                      [](const std::pair<unsigned long long, int4> &a, const std::pair<unsigned long long, int4> &b) {
                          return a.first < b.first;
                      });
            for (const auto &e : keyed) bricks.push_back(e.second);
            cnt[c] = (int)keyed.size();
        }
        if (Lv.ni > 0 && cnt[0] + cnt[1] == 0) return fail(LSMG_EHIP, "brick lists empty on level %d", l);
    } else {
        build_segments(H->dim, Lv.type, Lv.n, Lv.Wp, Lv.rows, Lv.cs, l, seg, cnt, H->mem, H->stream);
        if (Lv.ni > 0 && cnt[0] + cnt[1] == 0) return fail(LSMG_EHIP, "segment construction failed on level %d", l);
    }
    struct SegFree {
        const DevMem &m;
        int4 *p;
        ~SegFree() { m.put(p); }
    } seg_free{H->mem, seg[0]};
    Lv.nseg[0] = cnt[0];
    Lv.nseg[1] = cnt[1];
    Lv.nghc = (Lv.ng + kWave - 1) / kWave;
    Lv.nbandc = (Lv.nb + kWave - 1) / kWave;
    // the composed ghost map's rows are applied 4 rows per wavefront
    Lv.nghc4 = (Lv.ng + 3) / 4;
    const int total = cnt[0] + cnt[1] + Lv.nghc + Lv.nbandc + Lv.nghc4;
    LSMGCHK(H->alloc(&Lv.items, total));
    if (!bricks.empty())
        HIPCHK(hipMemcpyAsync(Lv.items, bricks.data(), sizeof(int4) * bricks.size(), hipMemcpyHostToDevice, H->stream));
    else if (cnt[0] + cnt[1] > 0)
        HIPCHK(hipMemcpyAsync(Lv.items, seg[0], sizeof(int4) * (cnt[0] + cnt[1]), hipMemcpyDeviceToDevice, H->stream));
    std::vector<int4> hv;
    for (int c = 0; c < Lv.nghc; ++c) {
        const int e = (c + 1) * kWave < Lv.ng ? (c + 1) * kWave : Lv.ng;
        hv.push_back(make_int4((l << 2) | 2, 0, c * kWave, e));
    }
    for (int c = 0; c < Lv.nbandc; ++c) {
        const int e = (c + 1) * kWave < Lv.nb ? (c + 1) * kWave : Lv.nb;
        hv.push_back(make_int4((l << 2) | 3, 0, c * kWave, e));
    }
    for (int c = 0; c < Lv.nghc4; ++c) {
        const int e = (c + 1) * 4 < Lv.ng ? (c + 1) * 4 : Lv.ng;
        hv.push_back(make_int4((l << 2) | 2, 0, c * 4, e));
    }
    if (!hv.empty())
        HIPCHK(hipMemcpyAsync(Lv.items + cnt[0] + cnt[1], hv.data(), sizeof(int4) * hv.size(), hipMemcpyHostToDevice,
                              H->stream));
    HIPCHK(hipStreamSynchronize(H->stream));
    if (H->dim == 2) LSMGCHK(build_tiles(H, l));
    return LSMG_OK;
}

lsmg_status build_f32(lsmg_hierarchy *H)
{
    for (int l = 0; l < H->nlev; ++l) {
        Level &Lv = H->L[l];
        LSMGCHK(H->zalloc(&Lv.s32, Lv.ssize));
        LSMGCHK(H->zalloc(&Lv.c32, Lv.ssize));
        LSMGCHK(H->zalloc(&Lv.rhs_s32, Lv.ssize));
        LSMGCHK(H->zalloc(&Lv.rhs_c32, Lv.ssize));
        LSMGCHK(H->zalloc(&Lv.x_s32, Lv.ssize));
        LSMGCHK(H->zalloc(&Lv.x_c32, Lv.ssize));
        LSMGCHK(H->zalloc(&Lv.r_s32, Lv.ssize));
        LSMGCHK(H->zalloc(&Lv.r_c32, Lv.ssize));
        if (H->dim == 2) {
            LSMGCHK(H->zalloc(&Lv.x2_s32, Lv.ssize));
            LSMGCHK(H->zalloc(&Lv.x2_c32, Lv.ssize));
        }
        LSMGCHK(H->alloc(&Lv.g_w32, (long long)Lv.ng * H->nst));
        LSMGCHK(H->zalloc(&Lv.g_buf0_32, Lv.ng));
        LSMGCHK(H->zalloc(&Lv.g_buf1_32, Lv.ng));
        launch_convert<float, double>(Lv.g_w32, Lv.g_w, (long long)Lv.ng * H->nst, H->stream);
        LSMGCHK(H->zalloc(&Lv.b_wt32, (long long)Lv.nb * (Lv.bmax > 0 ? Lv.bmax : 1)));
        if (Lv.nb > 0) launch_convert<float, double>(Lv.b_wt32, Lv.b_wt, (long long)Lv.nb * Lv.bmax, H->stream);
    }
    H->have32 = true;
    return LSMG_OK;
}

// ghost_sweeps Jacobi sweeps of eq. (RelGhost) with the inside values fixed are
// the linear map  ds <- M ds + tau b,  M = I - tau W_GG, W_GG the boundary-row
// weights between ghosts.  After S sweeps ds = M^S ds0 + tau sum_{i<S} M^i b.
// Both matrices depend on the geometry and tau only; their rows are composed
// here once and stored as one CSR table with two value arrays.
lsmg_status build_ghost_ops(lsmg_hierarchy *H, int l)
{
    Level &Lv = H->L[l];
    for (void *p : {(void *)Lv.go_ptr, (void *)Lv.go_col, (void *)Lv.go_a, (void *)Lv.go_b, (void *)Lv.go_a32,
                    (void *)Lv.go_b32, (void *)Lv.gc_ptr, (void *)Lv.gc_idx, (void *)Lv.gc_w, (void *)Lv.gc_w32,
                    (void *)Lv.go_sidx, (void *)Lv.ell_col, (void *)Lv.ell_six, (void *)Lv.ellf_idx,
                    (void *)Lv.ell_a, (void *)Lv.ell_b, (void *)Lv.ellf_w, (void *)Lv.ell_a32, (void *)Lv.ell_b32,
                    (void *)Lv.ellf_w32}) {
        if (!p) continue;
        // the tables may be in use by work still queued on the stream
        HIPCHK(hipStreamSynchronize(H->stream));
        H->mem.put(p);
        for (auto &q : H->ghost_ops)
            if (q == p) q = nullptr;
    }
    Lv.go_ptr = Lv.go_col = nullptr;
    Lv.go_a = Lv.go_b = nullptr;
    Lv.go_a32 = Lv.go_b32 = nullptr;
    Lv.gc_ptr = Lv.gc_idx = Lv.go_sidx = nullptr;
    Lv.ell_we = Lv.ell_wf = 0;
    Lv.ell_col = Lv.ell_six = Lv.ellf_idx = nullptr;
    Lv.ell_a = Lv.ell_b = Lv.ellf_w = nullptr;
    Lv.ell_a32 = Lv.ell_b32 = Lv.ellf_w32 = nullptr;
    Lv.gc_w = nullptr;
    Lv.gc_w32 = nullptr;
    Lv.go_bytes = 0;
    const int ng = Lv.ng, nst = H->nst, S = Lv.sweeps;
    if (ng == 0 || !H->p.ghost_c_new) return LSMG_OK;
    std::vector<int> stg((size_t)ng * nst);
    std::vector<double> w((size_t)ng * nst);
    HIPCHK(hipMemcpyAsync(stg.data(), Lv.g_stg, sizeof(int) * stg.size(), hipMemcpyDeviceToHost, H->stream));
    HIPCHK(hipMemcpyAsync(w.data(), Lv.g_w, sizeof(double) * w.size(), hipMemcpyDeviceToHost, H->stream));
    HIPCHK(hipStreamSynchronize(H->stream));
    const double tau = tau_level(H, l);
    std::vector<int> ptr(ng + 1, 0), col;
    std::vector<double> va, vb;
    std::vector<double> cur(ng, 0.0), nxt(ng, 0.0), acc(ng, 0.0);
    std::vector<char> in_cur(ng, 0), in_nxt(ng, 0), in_acc(ng, 0);
    std::vector<int> lcur, lnxt, lacc;
    for (int q = 0; q < ng; ++q) {
        lcur.assign(1, q);
        cur[q] = 1.0;
        in_cur[q] = 1;
        for (int it = 0; it < S; ++it) {
            for (int p : lcur) {
                if (!in_acc[p]) { in_acc[p] = 1; lacc.push_back(p); }
                acc[p] += cur[p];
            }
            // row vector times M: nxt = cur - tau cur W
            for (int p : lcur) {
                if (!in_nxt[p]) { in_nxt[p] = 1; lnxt.push_back(p); }
                nxt[p] += cur[p];
                for (int k = 0; k < nst; ++k) {
                    const int j = stg[(size_t)k * ng + p];
                    if (j < 0) continue;
                    if (!in_nxt[j]) { in_nxt[j] = 1; lnxt.push_back(j); }
                    nxt[j] -= tau * cur[p] * w[(size_t)k * ng + p];
                }
            }
            for (int p : lcur) { cur[p] = 0.0; in_cur[p] = 0; }
            lcur.swap(lnxt);
            lnxt.clear();
            for (int p : lcur) { cur[p] = nxt[p]; nxt[p] = 0.0; in_nxt[p] = 0; in_cur[p] = 1; }
        }
        // union of the supports, sorted by ghost index
        std::vector<int> cols(lcur);
        for (int p : lacc)
            if (!in_cur[p]) cols.push_back(p);
        std::sort(cols.begin(), cols.end());
        for (int c : cols) {
            col.push_back(c);
            va.push_back(in_cur[c] ? cur[c] : 0.0);
            vb.push_back(in_acc[c] ? tau * acc[c] : 0.0);
        }
        ptr[q + 1] = (int)col.size();
        for (int p : lcur) { cur[p] = 0.0; in_cur[p] = 0; }
        for (int p : lacc) { acc[p] = 0.0; in_acc[p] = 0; }
        lcur.clear();
        lacc.clear();
    }
    const size_t nnz = col.size();
    std::vector<float> va32(va.begin(), va.end()), vb32(vb.begin(), vb.end());
    auto up = [&](void **dst, const void *src, size_t bytes) -> lsmg_status {
        *dst = H->mem.get(bytes);
        if (!*dst) return fail(LSMG_EOOM, "ghost operator allocation");
        H->ghost_ops.push_back(*dst);
        Lv.go_bytes += bytes ? bytes : 1;
        if (bytes) HIPCHK(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, H->stream));
        return LSMG_OK;
    };
    LSMGCHK(up((void **)&Lv.go_ptr, ptr.data(), sizeof(int) * ptr.size()));
    LSMGCHK(up((void **)&Lv.go_col, col.data(), sizeof(int) * nnz));
    LSMGCHK(up((void **)&Lv.go_a, va.data(), sizeof(double) * nnz));
    LSMGCHK(up((void **)&Lv.go_b, vb.data(), sizeof(double) * nnz));
    LSMGCHK(up((void **)&Lv.go_a32, va32.data(), sizeof(float) * nnz));
    LSMGCHK(up((void **)&Lv.go_b32, vb32.data(), sizeof(float) * nnz));
    if (H->dim == 2) {
        // C = B W_GI: the inside-node part of the b-terms, over storage indices
        std::vector<int> st((size_t)ng * nst), gidx(ng);
        HIPCHK(hipMemcpyAsync(st.data(), Lv.g_st, sizeof(int) * st.size(), hipMemcpyDeviceToHost, H->stream));
        HIPCHK(hipMemcpyAsync(gidx.data(), Lv.g_idx, sizeof(int) * ng, hipMemcpyDeviceToHost, H->stream));
        HIPCHK(hipStreamSynchronize(H->stream));
        // per entry, the storage index of its ghost: the b-part's right-hand side is read
        // without going through g_idx
        std::vector<int> sx(nnz);
        for (size_t e = 0; e < nnz; ++e) sx[e] = gidx[col[e]];
        LSMGCHK(up((void **)&Lv.go_sidx, sx.data(), sizeof(int) * nnz));
        std::vector<int> cptr(ng + 1, 0), cidx;
        std::vector<double> cw;
        std::vector<std::pair<int, double>> rowv;
        for (int q = 0; q < ng; ++q) {
            rowv.clear();
            for (int e = ptr[q]; e < ptr[q + 1]; ++e) {
                const int c = col[e];
                const double bq = vb[e];
                if (bq == 0.0) continue;
                for (int k = 0; k < nst; ++k) {
                    const double wk = w[(size_t)k * ng + c];
                    if (wk == 0.0 || stg[(size_t)k * ng + c] >= 0) continue;
                    rowv.push_back({st[(size_t)k * ng + c], bq * wk});
                }
            }
            std::sort(rowv.begin(), rowv.end(),
                      [](const std::pair<int, double> &a, const std::pair<int, double> &b) { return a.first < b.first; });
            for (size_t i = 0; i < rowv.size(); ++i) {
                if (i > 0 && rowv[i].first == rowv[i - 1].first) {
                    cw.back() += rowv[i].second;
                } else {
                    cidx.push_back(rowv[i].first);
                    cw.push_back(rowv[i].second);
                }
            }
            cptr[q + 1] = (int)cidx.size();
        }
        const size_t cn = cidx.size();
        std::vector<float> cw32(cw.begin(), cw.end());
        LSMGCHK(up((void **)&Lv.gc_ptr, cptr.data(), sizeof(int) * cptr.size()));
        LSMGCHK(up((void **)&Lv.gc_idx, cidx.data(), sizeof(int) * cn));
        LSMGCHK(up((void **)&Lv.gc_w, cw.data(), sizeof(double) * cn));
        LSMGCHK(up((void **)&Lv.gc_w32, cw32.data(), sizeof(float) * cn));
        // the same rows padded to fixed widths (multiples of 16: the 16 lanes of a row),
        // where every row fits in 64 entries per part (one chunk of the apply kernel)
        int we = 16, wf = 16;
        for (int q = 0; q < ng; ++q) {
            we = std::max(we, (ptr[q + 1] - ptr[q] + 15) / 16 * 16);
            wf = std::max(wf, (cptr[q + 1] - cptr[q] + 15) / 16 * 16);
        }
        if (we > 64 || wf > 64) we = wf = 0;
        if (we > 0) {
        std::vector<int> ecol((size_t)ng * we), esix((size_t)ng * we), fidx((size_t)ng * wf);
        std::vector<double> ea((size_t)ng * we, 0.0), eb((size_t)ng * we, 0.0), fw((size_t)ng * wf, 0.0);
        for (int q = 0; q < ng; ++q) {
            for (int k = 0; k < we; ++k) {
                const int e = ptr[q] + k;
                const bool in = e < ptr[q + 1];
                ecol[(size_t)q * we + k] = in ? col[e] : q;
                esix[(size_t)q * we + k] = in ? sx[e] : gidx[q];
                if (in) {
                    ea[(size_t)q * we + k] = va[e];
                    eb[(size_t)q * we + k] = vb[e];
                }
            }
            for (int k = 0; k < wf; ++k) {
                const int f = cptr[q] + k;
                const bool in = f < cptr[q + 1];
                fidx[(size_t)q * wf + k] = in ? cidx[f] : gidx[q];
                if (in) fw[(size_t)q * wf + k] = cw[f];
            }
        }
        std::vector<float> ea32(ea.begin(), ea.end()), eb32(eb.begin(), eb.end()), fw32(fw.begin(), fw.end());
        Lv.ell_we = we;
        Lv.ell_wf = wf;
        LSMGCHK(up((void **)&Lv.ell_col, ecol.data(), sizeof(int) * ecol.size()));
        LSMGCHK(up((void **)&Lv.ell_six, esix.data(), sizeof(int) * esix.size()));
        LSMGCHK(up((void **)&Lv.ellf_idx, fidx.data(), sizeof(int) * fidx.size()));
        LSMGCHK(up((void **)&Lv.ell_a, ea.data(), sizeof(double) * ea.size()));
        LSMGCHK(up((void **)&Lv.ell_b, eb.data(), sizeof(double) * eb.size()));
        LSMGCHK(up((void **)&Lv.ellf_w, fw.data(), sizeof(double) * fw.size()));
        LSMGCHK(up((void **)&Lv.ell_a32, ea32.data(), sizeof(float) * ea32.size()));
        LSMGCHK(up((void **)&Lv.ell_b32, eb32.data(), sizeof(float) * eb32.size()));
        LSMGCHK(up((void **)&Lv.ellf_w32, fw32.data(), sizeof(float) * fw32.size()));
        }
    }
    HIPCHK(hipStreamSynchronize(H->stream));
    return LSMG_OK;
}

// the coarse-tail arguments of every start level (entry l starts at level l)
lsmg_status upload_tail_args(lsmg_hierarchy *H)
{
    std::vector<TailArgs> ta(H->nlev);
    for (int l = 0; l < H->nlev; ++l) ta[l] = tail_args(H, l, 0);
    HIPCHK(hipMemcpyAsync(H->d_tail, ta.data(), sizeof(TailArgs) * H->nlev, hipMemcpyHostToDevice, H->stream));
    HIPCHK(hipStreamSynchronize(H->stream));
    return LSMG_OK;
}

void make_descs(lsmg_hierarchy *H)
{
    H->hd64.assign(H->nlev, LevelDesc<double>{});
    H->hd32.assign(H->nlev, LevelDesc<float>{});
    for (int l = 0; l < H->nlev; ++l) {
        const Level &Lv = H->L[l];
        LevelDesc<double> &D = H->hd64[l];
        D.dim = H->dim; D.n = Lv.n; D.Wp = Lv.Wp; D.nst = H->nst;
        D.ni = Lv.ni; D.ng = Lv.ng; D.na = Lv.na; D.nb = Lv.nb; D.bmax = Lv.bmax; D.level = l;
        D.rows = Lv.rows; D.cs = Lv.cs; D.lo = H->lo; D.h = Lv.h;
        D.type = Lv.type; D.ext = Lv.ext; D.cmap = Lv.cmap;
        D.s = Lv.s; D.c = Lv.c; D.rhs_s = Lv.rhs_s; D.rhs_c = Lv.rhs_c; D.x_s = Lv.x_s; D.x_c = Lv.x_c;
        D.r_s = Lv.r_s; D.r_c = Lv.r_c; D.x2_s = Lv.x2_s; D.x2_c = Lv.x2_c;
        D.g_idx = Lv.g_idx; D.g_ijk = Lv.g_ijk; D.g_st = Lv.g_st; D.g_stg = Lv.g_stg; D.g_w = Lv.g_w;
        D.g_buf0 = Lv.g_buf0; D.g_buf1 = Lv.g_buf1;
        D.go_ptr = Lv.go_ptr; D.go_col = Lv.go_col; D.go_a = Lv.go_a; D.go_b = Lv.go_b;
        D.gc_ptr = Lv.gc_ptr; D.gc_idx = Lv.gc_idx; D.gc_w = Lv.gc_w; D.go_sidx = Lv.go_sidx;
        D.ell_we = Lv.ell_we; D.ell_wf = Lv.ell_wf; D.ell_col = Lv.ell_col; D.ell_six = Lv.ell_six;
        D.ellf_idx = Lv.ellf_idx; D.ell_a = Lv.ell_a; D.ell_b = Lv.ell_b; D.ellf_w = Lv.ellf_w;
        D.b_idx = Lv.b_idx; D.b_cnt = Lv.b_cnt; D.b_src = Lv.b_src; D.b_wt = Lv.b_wt;
        D.norms = H->d_norms; D.norm_stride = kNormSlots;
        if (l == 0) {
            D.sn = const_cast<double *>(H->step_sn); D.cn = const_cast<double *>(H->step_cn);
            D.bs = H->bs; D.bc = H->bc;
            D.fn = H->step_fn; D.fnp1 = H->step_fnp1; D.sb = H->step_sb; D.sb_const = H->step_sb_const;
        }
        LevelDesc<float> &E = H->hd32[l];
        E.dim = D.dim; E.n = D.n; E.Wp = D.Wp; E.nst = D.nst;
        E.ni = D.ni; E.ng = D.ng; E.na = D.na; E.nb = D.nb; E.bmax = D.bmax; E.level = l;
        E.rows = D.rows; E.cs = D.cs; E.lo = D.lo; E.h = D.h;
        E.type = D.type; E.ext = D.ext; E.cmap = D.cmap;
        E.s = Lv.s32; E.c = Lv.c32; E.rhs_s = Lv.rhs_s32; E.rhs_c = Lv.rhs_c32; E.x_s = Lv.x_s32; E.x_c = Lv.x_c32;
        E.r_s = Lv.r_s32; E.r_c = Lv.r_c32; E.x2_s = Lv.x2_s32; E.x2_c = Lv.x2_c32;
        E.g_idx = D.g_idx; E.g_ijk = D.g_ijk; E.g_st = D.g_st; E.g_stg = D.g_stg; E.g_w = Lv.g_w32;
        E.g_buf0 = Lv.g_buf0_32; E.g_buf1 = Lv.g_buf1_32;
        E.go_ptr = Lv.go_ptr; E.go_col = Lv.go_col; E.go_a = Lv.go_a32; E.go_b = Lv.go_b32;
        E.gc_ptr = Lv.gc_ptr; E.gc_idx = Lv.gc_idx; E.gc_w = Lv.gc_w32; E.go_sidx = Lv.go_sidx;
        E.ell_we = Lv.ell_we; E.ell_wf = Lv.ell_wf; E.ell_col = Lv.ell_col; E.ell_six = Lv.ell_six;
        E.ellf_idx = Lv.ellf_idx; E.ell_a = Lv.ell_a32; E.ell_b = Lv.ell_b32; E.ellf_w = Lv.ellf_w32;
        E.b_idx = D.b_idx; E.b_cnt = D.b_cnt; E.b_src = D.b_src; E.b_wt = Lv.b_wt32;
        E.norms = D.norms; E.norm_stride = D.norm_stride;
    }
}

lsmg_status build(lsmg_hierarchy *H, const double *d_phi, const lsmg_grid *g)
{
    const int dim = g->dim;
    H->dim = dim;
    H->nst = dim == 2 ? 9 : 27;
    H->lo = g->lo;
    H->hi = g->hi;
    int nlev = 1, nl = g->n;
    while (nl > H->p.coarsest_n) {
        if ((nl - 1) % 2) return fail(LSMG_EINVAL, "n - 1 must be (coarsest_n - 1) * 2^k");
        nl = (nl - 1) / 2 + 1;
        ++nlev;
        if (nlev > 16) return fail(LSMG_EINVAL, "too many levels");
    }
    if (nl != H->p.coarsest_n) return fail(LSMG_EINVAL, "n - 1 must be (coarsest_n - 1) * 2^k");
    if (g->n > (dim == 2 ? 2048 : 1024)) return fail(LSMG_EINVAL, "n too large (2-D: 2048, 3-D: 1024 at most)");
    H->nlev = nlev;
    H->L.assign(nlev, Level{});
    nl = g->n;
    for (int l = 0; l < nlev; ++l) {
        Level &Lv = H->L[l];
        Lv.n = nl;
        Lv.h = (g->hi - g->lo) / (nl - 1);
        Lv.rows = dim == 2 ? nl : (long long)nl * nl;
        if (dim == 2) {
            // rows of positions padded to 128 bytes of doubles
            Lv.Wp = ((nl + 1) / 2 + 15) / 16 * 16;
            Lv.cs = Lv.rows * Lv.Wp;
        } else {
            // bricks of 32 values (positions x rows x planes)
            const long long half = (nl + 1) / 2;
            Lv.Wp = (int)((half + (1 << kBP) - 1) >> kBP << kBP);
            Lv.cs = 32LL * brick_np(Lv.Wp) * brick_nj(nl) * brick_nk(nl);
        }
        Lv.ssize = 2 * Lv.cs;
        if (Lv.ssize > 0x7fffffffLL) return fail(LSMG_EINVAL, "grid too large for 32-bit storage indices");
        nl = (nl - 1) / 2 + 1;
    }
    const long long nn0 = (long long)g->n * g->n * (dim == 3 ? g->n : 1);
    // temporaries
    std::vector<double *> phis(nlev, nullptr);
    uint8_t *fin = nullptr, *fgh = nullptr;
    int64_t *scratch = nullptr;
    int *err = nullptr;
    const long long nscr = compact_scratch_size(nn0) + 1;
    lsmg_status st = LSMG_OK;
    int herr = 0;
    {  // the temporaries of the level construction, handed back at the end of the block
        DevTemps tmp(H->mem, H->stream);
        LSMGCHK(tmp.get(&fin, nn0));
        LSMGCHK(tmp.get(&fgh, nn0));
        LSMGCHK(tmp.get(&scratch, nscr));
        LSMGCHK(tmp.get(&err, 1));
        (void)hipMemsetAsync(err, 0, sizeof(int), H->stream);
        for (int l = 0; l < nlev && st == LSMG_OK; ++l) {
            const Level &Lv = H->L[l];
            const long long nn = (long long)Lv.n * Lv.n * (dim == 3 ? Lv.n : 1);
            st = tmp.get(&phis[l], nn);
            if (st != LSMG_OK) break;
            if (l == 0)
                (void)hipMemcpyAsync(phis[0], d_phi, sizeof(double) * nn, hipMemcpyDeviceToDevice, H->stream);
            else
                launch_inject_phi(dim, phis[l - 1], H->L[l - 1].n, phis[l], Lv.n, H->stream);
            st = build_level_arrays(H, l, phis[l], fin, fgh, scratch, (int)nscr, err);
        }
        for (int l = 0; l + 1 < nlev && st == LSMG_OK; ++l) st = build_band(H, l, phis[l], fin, scratch, (int)nscr);
        if (st == LSMG_OK) {
            (void)hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, H->stream);
            if (hipStreamSynchronize(H->stream) != hipSuccess) st = fail(LSMG_EHIP, "build synchronisation failed");
        }
    }
    if (st != LSMG_OK) return st;
    if (herr & 1) return fail(LSMG_EGEOM, "an inside node lies on the box edge");
    if (herr & 2) return fail(LSMG_EGEOM, "a ghost has no admissible Neumann row");
    for (int l = 0; l < nlev; ++l) LSMGCHK(build_items(H, l));
    for (int l = 0; l < nlev; ++l) {
        H->L[l].sweeps = level_sweeps(H, l);
        LSMGCHK(build_ghost_ops(H, l));
    }
    // Newton work arrays, coarsest LU, norms
    const Level &L0 = H->L[0];
    LSMGCHK(H->zalloc(&H->bs, L0.ssize));
    LSMGCHK(H->zalloc(&H->bc, L0.ssize));
    LSMGCHK(H->zalloc(&H->tmp_s, L0.ssize));
    LSMGCHK(H->zalloc(&H->tmp_c, L0.ssize));
    H->luN = 2 * H->L[nlev - 1].na;
    if (H->luN > 1024) return fail(LSMG_EINVAL, "coarsest grid has more than 512 active nodes; use a smaller coarsest_n");
    {
        // coarsest solve storage: Schur-complement scratch (global when it does not fit
        // in LDS) and [S^{-1} | J^sc | J^cs | J^cc]
        const long long na_c = H->L[nlev - 1].na;
        LSMGCHK(H->alloc(&H->lu, na_c * na_c));
        LSMGCHK(H->alloc(&H->ainv, 2 * na_c * na_c + 2 * na_c));
    }
    // the coarse tail: the levels with one active node per thread of its workgroup,
    // and the next finer ones of up to kTailMaxNodes nodes where the tail of the
    // working precision still fits in LDS (a level of that size run alone is a chain
    // of latency-bound launches)
    int l1 = nlev - 1;
    while (l1 > 0 && H->L[l1 - 1].na <= kTailNodes1) --l1;
    int l2 = l1;
    while (l2 > 0 && H->L[l2 - 1].na <= kTailMaxNodes) --l2;
    H->tail_l0 = l2;
    LSMGCHK(build_tail_tables(H));
    if (l2 < l1) {
        const size_t bytes = H->p.precision == 1 ? H->tail_sz.bytes<float>() : H->tail_sz.bytes<double>();
        if (!H->tail_lds || bytes > kTailLdsMax) {
            H->tail_l0 = l1;
            LSMGCHK(build_tail_tables(H));
        }
    }
    LSMGCHK(H->alloc(&H->piv, H->luN));
    LSMGCHK(H->zalloc(&H->lu_status, 1));
    LSMGCHK(H->zalloc(&H->d_norms, 4 * kNormSlots));
    HIPCHK(hipHostMalloc(&H->h_norms, sizeof(unsigned long long) * 4 * kNormSlots, hipHostMallocDefault));
    HIPCHK(hipHostMalloc(&H->h_status, sizeof(int), hipHostMallocDefault));
    if (H->p.precision == 1) LSMGCHK(build_f32(H));
    LSMGCHK(H->alloc(&H->d64, nlev));
    LSMGCHK(H->alloc(&H->d32, nlev));
    // coarse-tail and coarsest-operator arguments
    LSMGCHK(H->alloc(&H->d_tail, nlev));
    LSMGCHK(H->alloc(&H->d_coarse, 1));
    {
        const Level &Lc = H->L[nlev - 1];
        CoarseArgs ca{};
        ca.desc = nlev - 1;
        ca.c2s = Lc.c2s;
        ca.M = H->lu;
        ca.Ainv = H->ainv;
        ca.status = H->lu_status;
        HIPCHK(hipMemcpyAsync(H->d_coarse, &ca, sizeof(CoarseArgs), hipMemcpyHostToDevice, H->stream));
        LSMGCHK(upload_tail_args(H));
    }
    make_descs(H);
    LSMGCHK(push_desc(H));
    return LSMG_OK;
}

lsmg_status level_ok(const lsmg_hierarchy *H, int level)
{
    if (!H) return fail(LSMG_EINVAL, "hierarchy is NULL");
    if (level < 0 || level >= H->nlev) return fail(LSMG_EINVAL, "level %d out of range", level);
    return LSMG_OK;
}

// compact (device) -> split arrays of a level
template <typename T>
void scatter(lsmg_hierarchy *H, int l, const double *v, T *a, T *b)
{
    const Level &Lv = H->L[l];
    launch_scatter_compact<T>(Lv.c2s, Lv.na, v, a, b, H->stream);
}

template <typename T>
void gather(lsmg_hierarchy *H, int l, const T *a, const T *b, double *v)
{
    const Level &Lv = H->L[l];
    launch_gather_compact<T>(Lv.c2s, Lv.na, a, b, v, H->stream);
}

// x = 0 on the active nodes of a level (inactive positions are never written)
void zero_active_x(lsmg_hierarchy *H, int l)
{
    const Level &Lv = H->L[l];
    launch_zero_x<double>(H->dim, H->d64, Lv.w_act(), Lv.nw_act(), with_tail(Exec(H->stream), Lv.nghc));
}

// linear solve J dW = F on level 0 (rhs already in rhs_s / rhs_c) by V-cycles from zero;
// nF = |F|_inf.  Returns cycles run; rho statistics accumulate into the outs.
lsmg_status linear_solve(lsmg_hierarchy *H, double nF, int *cycles, double *rho_last, double *logsum, int *nrho,
                         bool fmg_first, bool factor_first)
{
    const Level &L0 = H->L[0];
    double rprev = nF;
    const bool mixed = H->p.precision == 1;
    if (mixed)   // x = 0; the FP32 cycle's right-hand side is r = F - J 0 = F
        launch_start_mixed(H->dim, H->d64, L0.w_act(), L0.nw_act(), with_tail(Exec(H->stream), L0.nghc), H->d32);
    else
        zero_active_x(H, 0);
    hipGraphExec_t ge = nullptr, gf = nullptr;
    // events recorded inside a graph cannot be timed: while launch timing is on,
    // cycles run as direct launches
    const bool graphs = H->use_graphs && H->prof_kernel < 0;
    if (graphs) LSMGCHK(cycle_graph(H, mixed, &ge));
    if (graphs && (fmg_first || factor_first)) LSMGCHK(cycle_graph(H, mixed, &gf, fmg_first, factor_first));
    if (!graphs && factor_first) launch_coarse_factor(H->dim, H->d64, H->d_coarse, 1, H->L[H->nlev - 1].na, H->stream);
    for (int q = 0; q < H->p.cycles_max; ++q) {
        if (rprev <= H->p.lin_rtol * nF) {
            // no cycle ran: the factorisation still has to be done and checked
            if (q == 0 && factor_first && graphs) {
                launch_coarse_factor(H->dim, H->d64, H->d_coarse, 1, H->L[H->nlev - 1].na, H->stream);
                LSMGCHK(check_factor(H));
            }
            break;
        }
        const size_t mark0 = H->prof_used;
        const bool first = q == 0 && (fmg_first || factor_first);
        if (graphs) HIPCHK(hipGraphLaunch(first ? gf : ge, H->stream));
        else cycle_enqueue(H, mixed, H->stream, q == 0 && fmg_first);
        if (q == 0 && factor_first)
            HIPCHK(hipMemcpyAsync(H->h_status, H->lu_status, sizeof(int), hipMemcpyDeviceToHost, H->stream));
        LSMGCHK(read_norms(H, 2));
        if (q == 0 && factor_first && *H->h_status != 0)
            return fail(LSMG_ENONFINITE, "coarsest operator is singular or not finite");
        if (!graphs) {
            prof_collect(H, mark0, H->prof_used);
            H->prof_used = mark0;
        }
        const double rq = norm_value(H, 1);
        ++*cycles;
        *rho_last = rprev > 0.0 ? rq / rprev : 0.0;
        if (*rho_last > 0.0) *logsum += std::log(*rho_last);
        ++*nrho;
        rprev = rq;
        if (!std::isfinite(rq)) break;
    }
    return LSMG_OK;
}

// Flexible GMRES(m) for the Newton system J dW = F on level 0 (krylov_m = m > 0),
// right-preconditioned by one V-cycle from zero (the FP32 cycle in mixed
// precision, which is why the preconditioned vectors Z_j are kept: Saad's
// flexible variant).  The vectors are compact (2 Na values) and enter the cycle
// and the operator through the level-0 storage arrays.  Each new direction is
// made orthogonal to V_0..V_j by classical Gram-Schmidt applied twice, on the
// device (inner products summed in a fixed order); its coefficients and norm
// come back to the host once per iteration for the Givens rotations of the
// small least-squares problem, whose last rotated entry is the 2-norm of the
// defect.  From x = 0, until that norm is at most lin_rtol |F|_2 or cycles_max
// cycles have run, restarting from the true defect every m iterations.  F is in
// the level-0 right-hand side on entry; the correction is left in the level-0
// correction arrays, as after linear_solve.
lsmg_status krylov_solve(lsmg_hierarchy *H, int *cycles, double *rho_last, double *logsum, int *nrho,
                         bool factor_first)
{
    const Level &L0 = H->L[0];
    const int m = H->p.krylov_m;
    const long long N = 2LL * L0.na;
    const bool mixed = H->p.precision == 1;
    hipStream_t s = H->stream;
    if (N == 0) {
        if (factor_first) {
            launch_coarse_factor(H->dim, H->d64, H->d_coarse, 1, H->L[H->nlev - 1].na, s);
            LSMGCHK(check_factor(H));
        }
        return LSMG_OK;
    }
    if (H->km < m) {
        // buffers for a larger m replace the earlier ones, which are kept until the
        // hierarchy is destroyed
        LSMGCHK(H->alloc(&H->kv, (long long)(m + 1) * N));
        LSMGCHK(H->alloc(&H->kz, (long long)m * N));
        LSMGCHK(H->alloc(&H->kf, N));
        LSMGCHK(H->alloc(&H->kx, N));
        LSMGCHK(H->alloc(&H->kw, N));
        LSMGCHK(H->alloc(&H->kpart, (long long)(m + 1) * kKvBlocks));
        LSMGCHK(H->alloc(&H->kres, 2LL * (m + 1) + 1));
        LSMGCHK(H->alloc(&H->kcoef, m));
        H->km = m;
    }
    double *V = H->kv, *Z = H->kz, *Fv = H->kf, *X = H->kx, *Wv = H->kw;
    auto vec = [&](double *b, int i) { return b + (size_t)i * N; };
    std::vector<double> hres(2 * (m + 1) + 1), Hh((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    auto read = [&](int count) -> lsmg_status {
        HIPCHK(hipMemcpyAsync(hres.data(), H->kres, sizeof(double) * count, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return LSMG_OK;
    };
    gather<double>(H, 0, L0.rhs_s, L0.rhs_c, Fv);
    launch_kv_div(X, X, N, 0.0, s);
    launch_kv_dots(Fv, Fv, N, 1, H->kpart, H->kres, s);
    LSMGCHK(read(1));
    const double target = H->p.lin_rtol * std::sqrt(hres[0]);
    double beta = std::sqrt(hres[0]);
    const double *r = Fv;   // the defect of x = 0
    int used = 0;
    // the coarsest factorisation runs on a side stream beside the first cycle's fine
    // levels, which joins it before its coarse tail; its status is read with the first
    // inner products (or at once, when no cycle runs)
    bool factor_pending = false;
    if (factor_first) {
        if (beta > target && H->p.cycles_max > 0 && H->prof_kernel < 0) {
            if (!H->side) HIPCHK(hipStreamCreateWithFlags(&H->side, hipStreamNonBlocking));
            if (!H->ev_fork) HIPCHK(hipEventCreateWithFlags(&H->ev_fork, hipEventDisableTiming));
            if (!H->ev_join) HIPCHK(hipEventCreateWithFlags(&H->ev_join, hipEventDisableTiming));
            HIPCHK(hipEventRecord(H->ev_fork, s));
            HIPCHK(hipStreamWaitEvent(H->side, H->ev_fork, 0));
            launch_coarse_factor(H->dim, H->d64, H->d_coarse, 1, H->L[H->nlev - 1].na, Exec(H->side));
            HIPCHK(hipEventRecord(H->ev_join, H->side));
            H->join_pending = true;
            factor_pending = true;
        } else {
            launch_coarse_factor(H->dim, H->d64, H->d_coarse, 1, H->L[H->nlev - 1].na, s);
            LSMGCHK(check_factor(H));
        }
    }
    while (beta > target && used < H->p.cycles_max) {
        launch_kv_div(vec(V, 0), r, N, beta, s);
        std::fill(Hh.begin(), Hh.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        double prev = beta;
        int k = 0;
        for (int j = 0; j < m && used < H->p.cycles_max; ++j) {
            const size_t mark0 = H->prof_used;
            // Z_j = M V_j: one cycle on the level-0 arrays from a zero correction
            scatter<double>(H, 0, vec(V, j), L0.rhs_s, L0.rhs_c);
            if (mixed) {
                launch_start_mixed(H->dim, H->d64, L0.w_act(), L0.nw_act(), with_tail(Exec(s), L0.nghc), H->d32);
                vcycle_rec<float>(H, 0, s);
                launch_add_f32(H->dim, H->d64, H->d32, L0.w_act(), L0.nw_act(), with_tail(Exec(s), L0.nghc));
            } else {
                zero_active_x(H, 0);
                vcycle_rec<double>(H, 0, s);
            }
            ++used;
            if (H->join_pending) {
                // (a cycle that did not reach the coarse tail) the factorisation joins here
                HIPCHK(hipStreamWaitEvent(s, H->ev_join, 0));
                H->join_pending = false;
            }
            gather<double>(H, 0, L0.x_s, L0.x_c, vec(Z, j));
            // J Z_j (the operator reads the level-0 correction, which holds Z_j)
            launch_apply_J<double>(H->dim, H->d64, L0.w_act(), L0.nw_act(), Exec(s));
            double *w = vec(V, j + 1);
            gather<double>(H, 0, L0.r_s, L0.r_c, w);
            launch_kv_dots(w, V, N, j + 1, H->kpart, H->kres, s);
            launch_kv_update(w, V, N, j + 1, H->kres, -1.0, s);
            launch_kv_dots(w, V, N, j + 1, H->kpart, H->kres + (m + 1), s);
            launch_kv_update(w, V, N, j + 1, H->kres + (m + 1), -1.0, s);
            launch_kv_dots(w, w, N, 1, H->kpart, H->kres + 2 * (m + 1), s);
            if (factor_pending)
                HIPCHK(hipMemcpyAsync(H->h_status, H->lu_status, sizeof(int), hipMemcpyDeviceToHost, s));
            LSMGCHK(read(2 * (m + 1) + 1));
            if (factor_pending) {
                factor_pending = false;
                if (*H->h_status != 0) return fail(LSMG_ENONFINITE, "coarsest operator is singular or not finite");
            }
            if (H->prof_kernel >= 0) {
                prof_collect(H, mark0, H->prof_used);
                H->prof_used = mark0;
            }
            for (int i = 0; i <= j; ++i) Hh[(size_t)i * m + j] = (0.0 + hres[i]) + hres[m + 1 + i];
            const double hn = std::sqrt(hres[2 * (m + 1)]);
            Hh[(size_t)(j + 1) * m + j] = hn;
            launch_kv_div(w, w, N, hn, s);
            // the earlier rotations on column j, then the one that zeroes its last entry
            for (int i = 0; i < j; ++i) {
                const double a = Hh[(size_t)i * m + j], b = Hh[(size_t)(i + 1) * m + j];
                Hh[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
                Hh[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            const double a = Hh[(size_t)j * m + j], b = Hh[(size_t)(j + 1) * m + j];
            const double d = std::sqrt(a * a + b * b);
            cs[j] = d > 0.0 ? a / d : 1.0;
            sn[j] = d > 0.0 ? b / d : 0.0;
            Hh[(size_t)j * m + j] = d;
            Hh[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            const double res = std::fabs(g[j + 1]);
            *rho_last = prev > 0.0 ? res / prev : 0.0;
            if (*rho_last > 0.0) *logsum += std::log(*rho_last);
            ++*nrho;
            prev = res;
            if (res <= target || hn == 0.0 || !std::isfinite(res)) break;
        }
        // x += Z y, R y = g with R the rotated k x k upper triangle
        for (int i = k - 1; i >= 0; --i) {
            double t = g[i];
            for (int q = i + 1; q < k; ++q) t -= Hh[(size_t)i * m + q] * y[q];
            y[i] = t / Hh[(size_t)i * m + i];
        }
        HIPCHK(hipMemcpyAsync(H->kcoef, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
        launch_kv_update(X, Z, N, k, H->kcoef, 1.0, s);
        // the true defect F - J x
        scatter<double>(H, 0, X, L0.x_s, L0.x_c);
        launch_apply_J<double>(H->dim, H->d64, L0.w_act(), L0.nw_act(), Exec(s));
        gather<double>(H, 0, L0.r_s, L0.r_c, Wv);
        launch_kv_rsub(Wv, Fv, N, s);
        launch_kv_dots(Wv, Wv, N, 1, H->kpart, H->kres, s);
        LSMGCHK(read(1));
        beta = std::sqrt(hres[0]);
        r = Wv;
        if (!std::isfinite(beta)) break;
    }
    scatter<double>(H, 0, X, L0.x_s, L0.x_c);
    *cycles += used;
    return LSMG_OK;
}

// names the Crank-Nicolson step's arrays in the level-0 descriptor (pushed
// only when they change)
lsmg_status set_step(lsmg_hierarchy *H, const double *sn, const double *cn, const double *sb, double sb_const,
                     const double *fn, const double *fnp1)
{
    if (!(fn && fnp1)) fn = fnp1 = nullptr;
    if (sn == H->step_sn && cn == H->step_cn && sb == H->step_sb && sb_const == H->step_sb_const &&
        fn == H->step_fn && fnp1 == H->step_fnp1)
        return LSMG_OK;
    H->step_sn = sn;
    H->step_cn = cn;
    H->step_sb = sb;
    H->step_sb_const = sb_const;
    H->step_fn = fn;
    H->step_fnp1 = fnp1;
    LevelDesc<double> &D = H->hd64[0];
    D.sn = const_cast<double *>(sn);
    D.cn = const_cast<double *>(cn);
    D.sb = sb;
    D.sb_const = sb_const;
    D.fn = fn;
    D.fnp1 = fnp1;
    return push_desc(H);
}

}  // namespace lsmg

// ===========================================================================
// C ABI
// ===========================================================================
using namespace lsmg;

extern "C" {

void lsmg_default_params(lsmg_params *p)
{
    if (!p) return;
    p->a = 1.0e4;
    p->d = 0.1;
    p->m_s = 64.06;
    p->m_c = 100.09;
    p->alpha = 0.01;
    p->beta = 0.1;
    p->tau_s = 0.9;
    p->nu1 = 2;
    p->nu2 = 2;
    p->ghost_sweeps = 0;
    p->ghost_sweeps_coarse = 0;
    p->sweeps_lambda = 0.0;
    p->band_steps = 3;
    p->ghost_c_new = 1;
    p->coarsest_n = 5;
    p->precision = 0;
    p->newton_tol = 1e-10;
    p->newton_max = 20;
    p->lin_rtol = 1e-3;
    p->cycles_max = 30;
    p->bc = 0;
    p->cycle_gamma = 1;
    p->fmg = 0;
    p->fused_sweep = 1;
    p->krylov_m = 0;
}

const char *lsmg_last_error(void) { return g_err.c_str(); }

lsmg_status lsmg_build_hierarchy(const double *d_levelset, const lsmg_grid *grid, const lsmg_params *params,
                                 const lsmg_allocator *allocator, void *stream, lsmg_hierarchy **out)
{
    if (!out) return fail(LSMG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d_levelset || !grid) return fail(LSMG_EINVAL, "levelset or grid is NULL");
    if (grid->dim != 2 && grid->dim != 3) return fail(LSMG_EINVAL, "dim must be 2 or 3");
    if (grid->n < 3 || !(grid->hi > grid->lo)) return fail(LSMG_EINVAL, "bad grid");
    LSMGCHK(check_params(params));
    lsmg_hierarchy *H = new (std::nothrow) lsmg_hierarchy();
    if (!H) return fail(LSMG_EOOM, "host allocation");
    H->p = *params;
    if (H->p.ghost_sweeps == 0) H->p.ghost_sweeps = grid->dim == 2 ? 5 : 15;
    if (H->p.ghost_sweeps_coarse == 0) H->p.ghost_sweeps_coarse = grid->dim == 2 ? 20 : 30;
    if (H->p.sweeps_lambda == 0.0) H->p.sweeps_lambda = grid->dim == 2 ? 0.3 : 0.1;
    H->stream = (hipStream_t)stream;
    if (allocator) {
        if (!allocator->alloc || !allocator->free) {
            delete H;
            return fail(LSMG_EINVAL, "allocator needs both alloc and free");
        }
        H->mem.alloc_fn = allocator->alloc;
        H->mem.free_fn = allocator->free;
        H->mem.ctx = allocator->ctx;
    }
    // LSMG_GRAPHS=0 replays the V-cycle as direct launches instead of a captured graph
    if (const char *e = std::getenv("LSMG_GRAPHS")) H->use_graphs = std::atoi(e) != 0;
    // LSMG_TAIL_LDS=0 runs the coarse tail from HBM instead of LDS
    if (const char *e = std::getenv("LSMG_TAIL_LDS")) H->tail_lds_use = std::atoi(e) != 0;
    lsmg_status st = build(H, d_levelset, grid);
    if (st != LSMG_OK) {
        (void)hipStreamSynchronize(H->stream);
        delete H;
        return st;
    }
    *out = H;
    return LSMG_OK;
}

void lsmg_destroy_hierarchy(lsmg_hierarchy *h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

lsmg_status lsmg_set_params(lsmg_hierarchy *h, const lsmg_params *params)
{
    if (!h) return fail(LSMG_EINVAL, "hierarchy is NULL");
    LSMGCHK(check_params(params));
    if (params->coarsest_n != h->p.coarsest_n || params->band_steps != h->p.band_steps || params->bc != h->p.bc)
        return fail(LSMG_EINVAL, "coarsest_n, band_steps and bc are fixed at build");
    lsmg_params np = *params;
    if (np.ghost_sweeps == 0) np.ghost_sweeps = h->dim == 2 ? 5 : 15;
    if (np.ghost_sweeps_coarse == 0) np.ghost_sweeps_coarse = h->dim == 2 ? 20 : 30;
    if (np.sweeps_lambda == 0.0) np.sweeps_lambda = h->dim == 2 ? 0.3 : 0.1;
    const bool ghost_ops_change = np.ghost_sweeps != h->p.ghost_sweeps ||
                                  np.ghost_sweeps_coarse != h->p.ghost_sweeps_coarse ||
                                  np.sweeps_lambda != h->p.sweeps_lambda || np.tau_s != h->p.tau_s ||
                                  np.ghost_c_new != h->p.ghost_c_new;
    invalidate_graphs(h);
    if (np.precision == 1 && !h->have32) {
        h->p.precision = 1;
        LSMGCHK(build_f32(h));
    }
    h->p = np;
    LSMGCHK(update_sweeps(h, ghost_ops_change));
    // the coarse tails read nu1, nu2 and the cycle index from their arguments
    LSMGCHK(upload_tail_args(h));
    make_descs(h);
    return push_desc(h);
}

lsmg_status lsmg_tail_in_lds(const lsmg_hierarchy *h, int precision, int *in_lds)
{
    if (!h || !in_lds || (precision != 0 && precision != 1)) return fail(LSMG_EINVAL, "bad argument");
    *in_lds = precision == 0 ? tail_in_lds<double>(h) : tail_in_lds<float>(h);
    return LSMG_OK;
}

lsmg_status lsmg_sweep_fused(const lsmg_hierarchy *h, int level, int precision, int *fused)
{
    LSMGCHK(level_ok(h, level));
    if (!fused || (precision != 0 && precision != 1)) return fail(LSMG_EINVAL, "bad argument");
    const Level &Lv = h->L[level];
    *fused = h->p.fused_sweep && Lv.tiles && Lv.gc_ptr &&
             fuse_sweep(Lv.na, precision == 0 ? sizeof(double) : sizeof(float));
    return LSMG_OK;
}

lsmg_status lsmg_set_dt(lsmg_hierarchy *h, double dt)
{
    if (!h) return fail(LSMG_EINVAL, "hierarchy is NULL");
    return set_dt(h, dt);
}

lsmg_status lsmg_get_params(const lsmg_hierarchy *h, lsmg_params *params)
{
    if (!h || !params) return fail(LSMG_EINVAL, "NULL argument");
    *params = h->p;
    return LSMG_OK;
}

lsmg_status lsmg_memory_bytes(const lsmg_hierarchy *h, size_t *hierarchy_bytes, size_t *state_bytes)
{
    if (!h) return fail(LSMG_EINVAL, "hierarchy is NULL");
    size_t b = h->alloc_bytes;
    for (const Level &Lv : h->L) b += Lv.go_bytes;
    if (hierarchy_bytes) *hierarchy_bytes = b;
    if (state_bytes) *state_bytes = 2 * sizeof(double) * (size_t)h->L[0].ssize;
    return LSMG_OK;
}

lsmg_status lsmg_estimate_bytes(const lsmg_grid *grid, const lsmg_params *params, size_t *hierarchy_bytes,
                                size_t *state_bytes)
{
    if (!grid || !params) return fail(LSMG_EINVAL, "NULL argument");
    if (grid->dim != 2 && grid->dim != 3) return fail(LSMG_EINVAL, "dim must be 2 or 3");
    // the storage-layout arrays of every level (as built), plus 10 % and 64 MiB for the
    // tables whose size depends on the geometry (ghosts, band, work lists, composed maps)
    size_t full = 0, ss0 = 0;
    int nl = grid->n;
    for (int l = 0; l < 16; ++l) {
        const long long half = (nl + 1) / 2;
        const size_t ss = grid->dim == 2
                              ? (size_t)(2 * (long long)nl * ((half + 15) / 16 * 16))
                              : (size_t)(2 * 32LL * brick_np((int)((half + (1 << kBP) - 1) >> kBP << kBP)) *
                                         brick_nj(nl) * brick_nk(nl));
        if (l == 0) ss0 = ss;
        // 2-D: a second copy of the corrections for the fused sweeps
        const size_t nv = grid->dim == 2 ? 10 : 8;
        full += ss * (2 + 4 + nv * sizeof(double) + (params->precision == 1 ? nv * sizeof(float) : 0));
        if (nl <= params->coarsest_n || (nl - 1) % 2) break;
        nl = (nl - 1) / 2 + 1;
    }
    full += 4 * sizeof(double) * ss0;
    if (hierarchy_bytes) *hierarchy_bytes = full + full / 10 + ((size_t)64 << 20);
    if (state_bytes) *state_bytes = 2 * sizeof(double) * ss0;
    return LSMG_OK;
}

lsmg_status lsmg_num_levels(const lsmg_hierarchy *h, int *nlev)
{
    if (!h || !nlev) return fail(LSMG_EINVAL, "NULL argument");
    *nlev = h->nlev;
    return LSMG_OK;
}

lsmg_status lsmg_level_info(const lsmg_hierarchy *h, int level, int *n, double *hh, int *n_inside, int *n_ghost,
                            int *n_band)
{
    LSMGCHK(level_ok(h, level));
    const Level &Lv = h->L[level];
    if (n) *n = Lv.n;
    if (hh) *hh = Lv.h;
    if (n_inside) *n_inside = Lv.ni;
    if (n_ghost) *n_ghost = Lv.ng;
    if (n_band) *n_band = Lv.nb;
    return LSMG_OK;
}

lsmg_status lsmg_compact_to_grid(lsmg_hierarchy *h, int level, int64_t *d_out)
{
    LSMGCHK(level_ok(h, level));
    if (!d_out) return fail(LSMG_EINVAL, "d_out is NULL");
    const Level &Lv = h->L[level];
    HIPCHK(hipMemcpyAsync(d_out, Lv.c2g, sizeof(int64_t) * Lv.na, hipMemcpyDeviceToDevice, h->stream));
    return LSMG_OK;
}

lsmg_status lsmg_ghost_table(lsmg_hierarchy *h, int level, int32_t *d_st, double *d_w, double *d_B, double *d_normal,
                             double *d_row_normal, int32_t *d_order, int32_t *d_bfallback)
{
    LSMGCHK(level_ok(h, level));
    const Level &Lv = h->L[level];
    const size_t ng = Lv.ng, nst = h->nst, dim = h->dim;
    if (ng == 0) return LSMG_OK;
    // stored structure-of-arrays (k * ng + q); returned row-major (q * nst + k)
    if (d_st || d_w) {
        std::vector<int> st(ng * nst), stT(ng * nst);
        std::vector<double> w(ng * nst), wT(ng * nst);
        HIPCHK(hipMemcpyAsync(st.data(), Lv.g_stc, sizeof(int) * ng * nst, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(w.data(), Lv.g_w, sizeof(double) * ng * nst, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (size_t q = 0; q < ng; ++q)
            for (size_t k = 0; k < nst; ++k) {
                stT[q * nst + k] = st[k * ng + q];
                wT[q * nst + k] = w[k * ng + q];
            }
        if (d_st) HIPCHK(hipMemcpyAsync(d_st, stT.data(), sizeof(int) * ng * nst, hipMemcpyHostToDevice, h->stream));
        if (d_w) HIPCHK(hipMemcpyAsync(d_w, wT.data(), sizeof(double) * ng * nst, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    if (d_B) HIPCHK(hipMemcpyAsync(d_B, Lv.g_B, sizeof(double) * ng * dim, hipMemcpyDeviceToDevice, h->stream));
    if (d_normal)
        HIPCHK(hipMemcpyAsync(d_normal, Lv.g_nrm, sizeof(double) * ng * dim, hipMemcpyDeviceToDevice, h->stream));
    if (d_row_normal)
        HIPCHK(hipMemcpyAsync(d_row_normal, Lv.g_nrow, sizeof(double) * ng * dim, hipMemcpyDeviceToDevice,
                              h->stream));
    if (d_order) HIPCHK(hipMemcpyAsync(d_order, Lv.g_order, sizeof(int) * ng, hipMemcpyDeviceToDevice, h->stream));
    if (d_bfallback)
        HIPCHK(hipMemcpyAsync(d_bfallback, Lv.g_bfall, sizeof(int) * ng, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return LSMG_OK;
}

lsmg_status lsmg_state_create(lsmg_hierarchy *h, lsmg_state **out)
{
    if (!h || !out) return fail(LSMG_EINVAL, "NULL argument");
    *out = nullptr;
    lsmg_state *st = new (std::nothrow) lsmg_state();
    if (!st) return fail(LSMG_EOOM, "host allocation");
    st->h = h;
    const Level &L0 = h->L[0];
    st->s = (double *)h->mem.get(sizeof(double) * L0.ssize);
    st->c = (double *)h->mem.get(sizeof(double) * L0.ssize);
    if (!st->s || !st->c) {
        delete st;
        return fail(LSMG_EOOM, "state allocation");
    }
    if (hipMemsetAsync(st->s, 0, sizeof(double) * L0.ssize, h->stream) != hipSuccess ||
        hipMemsetAsync(st->c, 0, sizeof(double) * L0.ssize, h->stream) != hipSuccess) {
        delete st;
        return fail(LSMG_EHIP, "state clear");
    }
    *out = st;
    return LSMG_OK;
}

void lsmg_state_destroy(lsmg_state *st)
{
    if (!st) return;
    (void)hipStreamSynchronize(st->h->stream);
    delete st;
}

lsmg_status lsmg_state_set(lsmg_state *st, const double *d_W)
{
    if (!st) return fail(LSMG_EINVAL, "NULL argument");
    if (st->h->L[0].na == 0) return LSMG_OK;  // an empty domain: the vector has no entries
    if (!d_W) return fail(LSMG_EINVAL, "NULL argument");
    scatter<double>(st->h, 0, d_W, st->s, st->c);
    return LSMG_OK;
}

lsmg_status lsmg_state_get(const lsmg_state *st, double *d_W)
{
    if (!st) return fail(LSMG_EINVAL, "NULL argument");
    if (st->h->L[0].na == 0) return LSMG_OK;  // an empty domain: the vector has no entries
    if (!d_W) return fail(LSMG_EINVAL, "NULL argument");
    gather<double>(st->h, 0, st->s, st->c, d_W);
    return LSMG_OK;
}

lsmg_status lsmg_state_set_grid(lsmg_state *st, const double *d_s, const double *d_c)
{
    if (!st || !d_s || !d_c) return fail(LSMG_EINVAL, "NULL argument");
    const Level &L0 = st->h->L[0];
    launch_grid_to_split(L0.c2g, L0.na, d_s, d_c, L0.c2s, st->s, st->c, st->h->stream);
    return LSMG_OK;
}

lsmg_status lsmg_state_get_grid(const lsmg_state *st, double *d_s, double *d_c)
{
    if (!st || !d_s || !d_c) return fail(LSMG_EINVAL, "NULL argument");
    const lsmg_hierarchy *h = st->h;
    const Level &L0 = h->L[0];
    const long long nn = (long long)L0.n * L0.n * (h->dim == 3 ? L0.n : 1);
    launch_fill<double>(d_s, nn, NAN, h->stream);
    launch_fill<double>(d_c, nn, NAN, h->stream);
    launch_compact_to_grid(L0.c2g, L0.na, st->s, st->c, L0.c2s, d_s, d_c, h->stream);
    return LSMG_OK;
}

lsmg_status lsmg_newton_cn_step(lsmg_hierarchy *h, lsmg_state *st, double dt, const double *d_sb, double sb_const,
                                const double *d_fn, const double *d_fnp1, lsmg_step_stats *stats)
{
    if (!h || !st || st->h != h) return fail(LSMG_EINVAL, "bad hierarchy or state");
    LSMGCHK(set_dt(h, dt));
    LSMGCHK(set_step(h, st->s, st->c, d_sb, sb_const, d_fn, d_fnp1));
    const Level &L0 = h->L[0];
    hipStream_t s = h->stream;
    // explicit half, and the first iterate W^{(n+1,0)} = W^n
    launch_explicit_half(h->dim, h->d64, L0.w_act(), L0.nw_act(), with_tail(Exec(s), L0.nghc));
    zero_norms(h, 0, 4);
    launch_residual(h->dim, h->d64, L0.w_act(), L0.nw_act(), 0, with_tail(Exec(s), L0.nghc));
    LSMGCHK(read_norms(h, 1));
    double nF = norm_value(h, 0);
    lsmg_status rc = LSMG_ENOCONV;
    int cycles = 0, nrho = 0, it;
    double rho_last = 0.0, logsum = 0.0, dwrel = 0.0;
    for (it = 1; it <= h->p.newton_max; ++it) {
        if (!std::isfinite(nF)) {
            rc = fail(LSMG_ENONFINITE, "residual is not finite");
            break;
        }
        // the coarsest factorisation runs inside the first cycle, and is checked with its norms
        LSMGCHK(linearize(h, false));
        if (h->p.krylov_m > 0)
            LSMGCHK(krylov_solve(h, &cycles, &rho_last, &logsum, &nrho, true));
        else
            LSMGCHK(linear_solve(h, nF, &cycles, &rho_last, &logsum, &nrho,
                                 h->p.fmg == 2 || (h->p.fmg == 1 && it == 1), true));
        zero_norms(h, 0, 4);
        launch_newton_update(h->dim, h->d64, L0.w_act(), L0.nw_act(), with_tail(Exec(s), L0.nghc));
        launch_residual(h->dim, h->d64, L0.w_act(), L0.nw_act(), 0, with_tail(Exec(s), L0.nghc));
        LSMGCHK(read_norms(h, 4));
        nF = norm_value(h, 0);
        const double nD = norm_value(h, 2), nW = norm_value(h, 3);
        dwrel = nW > 0.0 ? nD / nW : nD;
        if (!std::isfinite(nF) || !std::isfinite(dwrel)) {
            rc = fail(LSMG_ENONFINITE, "Newton iterate is not finite");
            break;
        }
        if ((nF < dwrel ? nF : dwrel) < h->p.newton_tol) {
            rc = LSMG_OK;
            break;
        }
    }
    if (rc == LSMG_ENOCONV) fail(LSMG_ENOCONV, "Newton did not converge in %d iterations", h->p.newton_max);
    if (stats) {
        stats->newton_iters = it > h->p.newton_max ? h->p.newton_max : it;
        stats->vcycles = cycles;
        stats->res_inf = nF;
        stats->rho_last = rho_last;
        stats->rho_geo = nrho > 0 ? std::exp(logsum / nrho) : 0.0;
        stats->dw_rel = dwrel;
    }
    if (rc == LSMG_OK) {
        launch_commit(h->dim, h->d64, L0.w_act(), L0.nw_act(), with_tail(Exec(s), L0.nghc));
        HIPCHK(hipStreamSynchronize(s));
    }
    h->lin_set = false;
    return rc;
}

lsmg_status lsmg_residual(lsmg_hierarchy *h, const double *d_W, const double *d_Wn, double dt, const double *d_sb,
                          double sb_const, const double *d_fn, const double *d_fnp1, double *d_F, double *res_inf)
{
    if (!h || !d_W || !d_Wn || !d_F) return fail(LSMG_EINVAL, "NULL argument");
    LSMGCHK(set_dt(h, dt));
    const Level &L0 = h->L[0];
    scatter<double>(h, 0, d_Wn, h->tmp_s, h->tmp_c);
    LSMGCHK(set_step(h, h->tmp_s, h->tmp_c, d_sb, sb_const, d_fn, d_fnp1));
    // the explicit half also sets the iterate to W^n; W replaces it afterwards
    launch_explicit_half(h->dim, h->d64, L0.w_act(), L0.nw_act(), with_tail(Exec(h->stream), L0.nghc));
    scatter<double>(h, 0, d_W, L0.s, L0.c);
    zero_norms(h, 0, 1);
    launch_residual(h->dim, h->d64, L0.w_act(), L0.nw_act(), 0, with_tail(Exec(h->stream), L0.nghc));
    gather<double>(h, 0, L0.rhs_s, L0.rhs_c, d_F);
    h->lin_set = false;
    if (res_inf) {
        LSMGCHK(read_norms(h, 1));
        *res_inf = norm_value(h, 0);
    }
    return LSMG_OK;
}

lsmg_status lsmg_set_linearization(lsmg_hierarchy *h, const double *d_W, double dt)
{
    if (!h || !d_W) return fail(LSMG_EINVAL, "NULL argument");
    LSMGCHK(set_dt(h, dt));
    const Level &L0 = h->L[0];
    scatter<double>(h, 0, d_W, L0.s, L0.c);
    LSMGCHK(linearize(h));
    return check_factor(h);
}

lsmg_status lsmg_level_state(lsmg_hierarchy *h, int level, double *d_W)
{
    LSMGCHK(level_ok(h, level));
    if (!d_W) return fail(LSMG_EINVAL, "NULL argument");
    gather<double>(h, level, h->L[level].s, h->L[level].c, d_W);
    return LSMG_OK;
}

lsmg_status lsmg_apply_J(lsmg_hierarchy *h, int level, const double *d_x, double *d_y)
{
    LSMGCHK(level_ok(h, level));
    if (!h->lin_set) return fail(LSMG_EINVAL, "no linearisation point set");
    const Level &Lv = h->L[level];
    scatter<double>(h, level, d_x, Lv.x_s, Lv.x_c);
    launch_apply_J<double>(h->dim, h->d64, Lv.w_act(), Lv.nw_act(), h->stream);
    gather<double>(h, level, Lv.r_s, Lv.r_c, d_y);
    return LSMG_OK;
}

lsmg_status lsmg_smooth(lsmg_hierarchy *h, int level, const double *d_rhs, double *d_x, int nsweeps)
{
    LSMGCHK(level_ok(h, level));
    if (!h->lin_set) return fail(LSMG_EINVAL, "no linearisation point set");
    const Level &Lv = h->L[level];
    scatter<double>(h, level, d_rhs, Lv.rhs_s, Lv.rhs_c);
    scatter<double>(h, level, d_x, Lv.x_s, Lv.x_c);
    smooth_level<double>(h, level, h->stream, nsweeps);
    gather<double>(h, level, Lv.x_s, Lv.x_c, d_x);
    return LSMG_OK;
}

lsmg_status lsmg_defect(lsmg_hierarchy *h, int level, const double *d_rhs, const double *d_x, double *d_r,
                        double *res_inf)
{
    LSMGCHK(level_ok(h, level));
    if (!h->lin_set) return fail(LSMG_EINVAL, "no linearisation point set");
    const Level &Lv = h->L[level];
    scatter<double>(h, level, d_rhs, Lv.rhs_s, Lv.rhs_c);
    scatter<double>(h, level, d_x, Lv.x_s, Lv.x_c);
    zero_norms(h, 1, 1);
    launch_defect<double>(h->dim, h->d64, Lv.w_act(), Lv.nw_act(), 1, h->stream);
    if (d_r) gather<double>(h, level, Lv.r_s, Lv.r_c, d_r);
    if (res_inf) {
        LSMGCHK(read_norms(h, 2));
        *res_inf = norm_value(h, 1);
    }
    return LSMG_OK;
}

lsmg_status lsmg_restrict(lsmg_hierarchy *h, int level, const double *d_r, double *d_rhs_coarse)
{
    LSMGCHK(level_ok(h, level));
    if (level + 1 >= h->nlev) return fail(LSMG_EINVAL, "no coarser level");
    const Level &F = h->L[level], &C = h->L[level + 1];
    launch_fill<double>(F.r_s, F.ssize, 0.0, h->stream);
    launch_fill<double>(F.r_c, F.ssize, 0.0, h->stream);
    scatter<double>(h, level, d_r, F.r_s, F.r_c);
    launch_band<double>(h->d64, F.w_band(), F.nbandc, h->stream);
    launch_restrict<double>(h->dim, h->d64, C.w_act(), C.nw_act(), h->stream);
    gather<double>(h, level + 1, C.rhs_s, C.rhs_c, d_rhs_coarse);
    return LSMG_OK;
}

lsmg_status lsmg_prolong_add(lsmg_hierarchy *h, int level, const double *d_e_coarse, double *d_x)
{
    LSMGCHK(level_ok(h, level));
    if (level + 1 >= h->nlev) return fail(LSMG_EINVAL, "no coarser level");
    const Level &F = h->L[level], &C = h->L[level + 1];
    scatter<double>(h, level + 1, d_e_coarse, C.x_s, C.x_c);
    scatter<double>(h, level, d_x, F.x_s, F.x_c);
    launch_prolong<double>(h->dim, h->d64, F.w_act(), F.nw_act(), h->stream);
    gather<double>(h, level, F.x_s, F.x_c, d_x);
    return LSMG_OK;
}

lsmg_status lsmg_coarse_solve(lsmg_hierarchy *h, const double *d_rhs, double *d_x)
{
    if (!h || !d_rhs || !d_x) return fail(LSMG_EINVAL, "NULL argument");
    if (!h->lin_set) return fail(LSMG_EINVAL, "no linearisation point set");
    const int lc = h->nlev - 1;
    const Level &Lc = h->L[lc];
    scatter<double>(h, lc, d_rhs, Lc.rhs_s, Lc.rhs_c);
    launch_coarse_apply<double>(h->d64, lc, Lc.na, Lc.c2s, h->ainv, h->stream);
    gather<double>(h, lc, Lc.x_s, Lc.x_c, d_x);
    return LSMG_OK;
}

lsmg_status lsmg_vcycle(lsmg_hierarchy *h, int level, const double *d_rhs, double *d_x, double *res_inf)
{
    LSMGCHK(level_ok(h, level));
    if (!h->lin_set) return fail(LSMG_EINVAL, "no linearisation point set");
    const Level &Lv = h->L[level];
    scatter<double>(h, level, d_rhs, Lv.rhs_s, Lv.rhs_c);
    scatter<double>(h, level, d_x, Lv.x_s, Lv.x_c);
    vcycle_rec<double>(h, level, h->stream);
    zero_norms(h, 1, 1);
    launch_defect<double>(h->dim, h->d64, Lv.w_act(), Lv.nw_act(), 1, h->stream);
    gather<double>(h, level, Lv.x_s, Lv.x_c, d_x);
    if (res_inf) {
        LSMGCHK(read_norms(h, 2));
        *res_inf = norm_value(h, 1);
    }
    return LSMG_OK;
}

lsmg_status lsmg_profile_start(lsmg_hierarchy *h, int kernel, int level)
{
    LSMGCHK(level_ok(h, level));
    if (kernel < LSMG_KERNEL_SMOOTH || kernel > LSMG_KERNEL_GHOST) return fail(LSMG_EINVAL, "unknown kernel class");
    HIPCHK(hipStreamSynchronize(h->stream));
    invalidate_graphs(h);
    h->prof_kernel = kernel;
    h->prof_level = level;
    h->prof_used = 0;
    h->prof_pending = 0;
    h->prof_acc_ms = 0.0;
    h->prof_acc_n = 0;
    return LSMG_OK;
}

lsmg_status lsmg_profile_stop(lsmg_hierarchy *h, int *launches, double *total_ms)
{
    if (!h) return fail(LSMG_EINVAL, "hierarchy is NULL");
    HIPCHK(hipStreamSynchronize(h->stream));
    prof_collect(h, h->prof_pending, h->prof_used);
    if (launches) *launches = (int)h->prof_acc_n;
    if (total_ms) *total_ms = h->prof_acc_ms;
    h->prof_kernel = -1;
    h->prof_level = -1;
    h->prof_used = 0;
    h->prof_pending = 0;
    invalidate_graphs(h);
    return LSMG_OK;
}

}  // extern "C"
