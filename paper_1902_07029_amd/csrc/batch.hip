// Batches: many hierarchies (domains of different shapes and grid sizes)
// advanced together, one launch per kernel and grid size covering every domain
// that has a level of that size.
//
// The batch concatenates its members' level descriptors and work lists
// (rebasing the descriptor index of every item).  Its V-cycle walks the grid
// sizes from the finest down: at each size it smooths, forms the defect and
// restricts for every member level of that size that is not part of the
// member's coarse tail, then one launch runs the coarse tails of all members
// (one workgroup each), and the walk back up prolongs and post-smooths.  Each
// member therefore sees exactly the operations of its own V-cycle, in the same
// order, on its own data, so its results are bitwise those of running it alone.
//
// Newton and the cycle loop run in lockstep on the host with the same stopping
// rules as a single hierarchy, evaluated per member; a member that has
// converged (or failed) is switched off through the per-descriptor flags the
// item kernels check, so the captured cycle graph stays valid for any subset.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <map>
#include <vector>

#include "hier.hpp"

using namespace lsmg;

namespace {

// kernel classes the autotuner picks a workgroup size for
enum { kTSmooth = 0, kTGhost = 1, kTDefect = 2, kTRestrict = 3, kTProlong = 4, kTBand = 5, kTClasses = 6 };
// rows of per-descriptor flags (see b_build)
enum { kFCycle = 0, kFStart = 1, kFLin = 2, kFUpdate = 3, kFCommit = 4, kFlagRows = 5 };

struct BList {
    int off = 0, n = 0;   // range in the batch's item pool
    int tail = 0;         // trailing ghost items, dealt to the XCDs in turn (Exec::tail)
};

struct BSize {
    int n = 0;                       // nodes per axis
    BList seg[2], gh, act, band;     // member levels of this size outside the coarse tails
    BList gh4;                       // their ghosts in items of 4 (the composed map)
    BList seg1g;                     // colour-1 segments of the members, then all their ghost items
    BList tiles;                     // 2-D: tiles of the fused sweep
    long long na = 0;                // active nodes of the member levels outside the coarse tails
    BList rcoarse;                   // their next coarser levels (restriction targets)
    BList icoarse;                   // next coarser levels of every member level of this size (injection)
    int ipb[kTClasses];
};

}  // namespace

struct lsmg_batch {
    int dim = 2, ndom = 0, ndesc = 0;
    lsmg_params p{};
    hipStream_t stream = nullptr, cap = nullptr;
    std::vector<lsmg_hierarchy *> mem;
    std::vector<int> d0;
    std::vector<LevelDesc<double>> hd64;
    std::vector<LevelDesc<float>> hd32;
    LevelDesc<double> *d64 = nullptr;
    LevelDesc<float> *d32 = nullptr;
    std::vector<BSize> sizes;       // descending n
    std::vector<int> zfin;          // per member: the size class of its finest level
    BList lev0, all;
    int4 *pool = nullptr;
    int npool = 0;
    TailArgs *d_tail = nullptr;
    int tail_na_max = 0;
    bool tail_stage = true;     // every member's tail node lists fit the LDS copy
    // a member's coarse tail runs in the kernel it runs in alone: the LDS tail where it
    // fits there, else the HBM tail; a launch of each covers the members of its kind
    bool any_lds64 = false, any_lds32 = false, all_lds64 = true, all_lds32 = true;
    size_t lds_bytes64 = 0, lds_bytes32 = 0;   // the LDS tail's dynamic LDS (largest member)
    CoarseArgs *d_coarse = nullptr;
    int coarse_n_max = 0;
    int *d_act = nullptr, *h_act = nullptr;
    std::vector<int> act_last;
    int *d_cstatus = nullptr, *h_cstatus = nullptr;
    unsigned long long *d_norms = nullptr, *d_nred = nullptr, *h_nred = nullptr;
    long long norm_stride = 0;
    std::vector<hipGraphExec_t> gexec[2];   // per precision, by first size class (b_vcycle)
    // linear solves in chunks of cycles with the stopping tests on the device:
    // per-member control, the norms of a chunk's cycles, (d0, nlev) per member,
    // the cycles each member's last solve took, and the cycle graph with the
    // device-side tests (one per precision; a chunk replays it)
    LinCtl *d_lctl = nullptr, *h_lctl = nullptr;
    double *d_hist = nullptr, *h_hist = nullptr;
    int2 *d_dlev = nullptr;
    std::vector<int> last_cycles;
    std::vector<hipGraphExec_t> gctl[2];
    bool use_graphs = true;
    int autotune = 1, tuned = 0;
    bool fused = false;         // 2-D, every member with fused sweeps
    double dt = 0.0;
    std::vector<const lsmg_state *> last_states;
    std::vector<const double *> last_sb;
    std::vector<double> last_sbc;
    DevMem dmem;  // device memory: the caller's allocator or hipMalloc
    std::vector<void *> allocs;
    std::vector<hipEvent_t> evpool;
    // launch timing of one kernel class at one grid size
    int prof_kernel = -1, prof_n = -1;
    std::vector<hipEvent_t> prof_pool;
    size_t prof_used = 0;
    double prof_acc_ms = 0.0;
    long long prof_acc_n = 0;
    ~lsmg_batch()
    {
        for (int i = 0; i < 2; ++i) {
            for (hipGraphExec_t g : gexec[i])
                if (g) (void)hipGraphExecDestroy(g);
            for (hipGraphExec_t g : gctl[i])
                if (g) (void)hipGraphExecDestroy(g);
        }
        if (cap) (void)hipStreamDestroy(cap);
        for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
        for (hipEvent_t e : prof_pool) (void)hipEventDestroy(e);
        for (void *q : allocs) dmem.put(q);
        if (h_act) (void)hipHostFree(h_act);
        if (h_cstatus) (void)hipHostFree(h_cstatus);
        if (h_nred) (void)hipHostFree(h_nred);
        if (h_lctl) (void)hipHostFree(h_lctl);
        if (h_hist) (void)hipHostFree(h_hist);
    }
    template <typename T>
    lsmg_status alloc(T **ptr, long long count)
    {
        *ptr = nullptr;
        if (count <= 0) count = 1;
        void *q = dmem.get(sizeof(T) * (size_t)count);
        if (!q) return fail(LSMG_EOOM, "batch allocation of %lld bytes failed", (long long)(sizeof(T) * count));
        allocs.push_back(q);
        *ptr = (T *)q;
        return LSMG_OK;
    }
};

namespace {

template <typename T>
const LevelDesc<T> *bdescs(const lsmg_batch *B);
template <>
const LevelDesc<double> *bdescs<double>(const lsmg_batch *B) { return B->d64; }
template <>
const LevelDesc<float> *bdescs<float>(const lsmg_batch *B) { return B->d32; }

inline const int4 *items(const lsmg_batch *B, const BList &l) { return B->pool + l.off; }

Exec bexec(const lsmg_batch *B, hipStream_t s, int ipb) { return Exec(s, B->d_act, ipb); }

// the same, with a pair of timing events when kernel class `kernel` at grid
// size n is being timed
Exec bexec_t(lsmg_batch *B, hipStream_t s, int ipb, int kernel, int n)
{
    Exec x(s, B->d_act, ipb);
    if (B->prof_kernel != kernel || B->prof_n != n) return x;
    while (B->prof_pool.size() < B->prof_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return x;
        B->prof_pool.push_back(e);
    }
    x.ev0 = B->prof_pool[B->prof_used++];
    x.ev1 = B->prof_pool[B->prof_used++];
    return x;
}

// adds the timed launches recorded so far (the stream has been synchronised)
void b_prof_collect(lsmg_batch *B)
{
    for (size_t i = 0; i + 1 < B->prof_used; i += 2) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, B->prof_pool[i], B->prof_pool[i + 1]) == hipSuccess) {
            B->prof_acc_ms += ms;
            ++B->prof_acc_n;
        }
    }
    B->prof_used = 0;
}

// ---------------------------------------------------------------------------
// descriptors
// ---------------------------------------------------------------------------
// the batch's descriptors: the members' own, with the norms moved to the
// batch's slots and the step arrays of the states being advanced
lsmg_status refresh_descs(lsmg_batch *B, lsmg_state *const *states, const double *const *sb, const double *sbc)
{
    for (int k = 0; k < B->ndom; ++k) {
        const lsmg_hierarchy *H = B->mem[k];
        for (int l = 0; l < H->nlev; ++l) {
            LevelDesc<double> D = H->hd64[l];
            D.norms = B->d_norms + (long long)k * kNormSlots;
            D.norm_stride = B->norm_stride;
            if (l == 0) {
                D.sn = states ? states[k]->s : nullptr;
                D.cn = states ? states[k]->c : nullptr;
                D.bs = H->bs;
                D.bc = H->bc;
                D.fn = D.fnp1 = nullptr;
                D.sb = sb ? sb[k] : nullptr;
                D.sb_const = sbc ? sbc[k] : 1.0;
            }
            B->hd64[B->d0[k] + l] = D;
            if (H->have32) {
                LevelDesc<float> E = H->hd32[l];
                E.norms = D.norms;
                E.norm_stride = D.norm_stride;
                B->hd32[B->d0[k] + l] = E;
            }
        }
    }
    // coarse tails (their per-level sweep counts follow dt)
    std::vector<TailArgs> ta(B->ndom);
    for (int k = 0; k < B->ndom; ++k) ta[k] = tail_args(B->mem[k], B->mem[k]->tail_l0, B->d0[k]);
    HIPCHK(hipMemcpyAsync(B->d_tail, ta.data(), sizeof(TailArgs) * B->ndom, hipMemcpyHostToDevice, B->stream));
    HIPCHK(hipMemcpyAsync(B->d64, B->hd64.data(), sizeof(LevelDesc<double>) * B->ndesc, hipMemcpyHostToDevice,
                          B->stream));
    if (B->p.precision == 1)
        HIPCHK(hipMemcpyAsync(B->d32, B->hd32.data(), sizeof(LevelDesc<float>) * B->ndesc, hipMemcpyHostToDevice,
                              B->stream));
    HIPCHK(hipStreamSynchronize(B->stream));
    return LSMG_OK;
}

// per-descriptor flags from per-member flags; the pinned staging buffer is
// rewritten only after the stream has been synchronised since its last copy
// (every caller reads norms or statuses back before changing the flags again)
lsmg_status set_flags(lsmg_batch *B, const std::vector<char> &on)
{
    std::vector<int> v(B->ndesc, 0);
    for (int k = 0; k < B->ndom; ++k)
        for (int l = 0; l < B->mem[k]->nlev; ++l) v[B->d0[k] + l] = on[k] ? 1 : 0;
    if (v == B->act_last) return LSMG_OK;
    HIPCHK(hipStreamSynchronize(B->stream));
    std::memcpy(B->h_act, v.data(), sizeof(int) * B->ndesc);
    HIPCHK(hipMemcpyAsync(B->d_act, B->h_act, sizeof(int) * B->ndesc, hipMemcpyHostToDevice, B->stream));
    B->act_last = v;
    return LSMG_OK;
}

// all flag rows at once (member flags per row); the stream is synchronised
// before the pinned staging buffer is rewritten
lsmg_status set_flag_rows(lsmg_batch *B, const std::vector<std::vector<char>> &rows)
{
    const int nd = B->ndesc;
    std::vector<int> v((size_t)kFlagRows * nd, 0);
    for (int r = 0; r < kFlagRows && r < (int)rows.size(); ++r)
        for (int k = 0; k < B->ndom; ++k)
            for (int l = 0; l < B->mem[k]->nlev; ++l) v[(size_t)r * nd + B->d0[k] + l] = rows[r][k] ? 1 : 0;
    HIPCHK(hipStreamSynchronize(B->stream));
    std::memcpy(B->h_act, v.data(), sizeof(int) * v.size());
    HIPCHK(hipMemcpyAsync(B->d_act, B->h_act, sizeof(int) * v.size(), hipMemcpyHostToDevice, B->stream));
    B->act_last.assign(v.begin(), v.begin() + nd);
    return LSMG_OK;
}

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

void zero_bnorms(lsmg_batch *B, int first, int count, hipStream_t s)
{
    launch_fill<unsigned long long>(B->d_norms + first * B->norm_stride, count * B->norm_stride, 0ull, s);
}

// per-member maxima of norms [first, first + count) into h_nred[k * 4 + norm]
lsmg_status read_bnorms(lsmg_batch *B, int first, int count)
{
    launch_norm_reduce(B->d_norms, B->norm_stride, B->ndom, first, count, B->d_nred, B->stream);
    HIPCHK(hipMemcpyAsync(B->h_nred, B->d_nred, sizeof(unsigned long long) * 4 * B->ndom, hipMemcpyDeviceToHost,
                          B->stream));
    HIPCHK(hipStreamSynchronize(B->stream));
    return LSMG_OK;
}

double bnorm(const lsmg_batch *B, int k, int norm)
{
    double v;
    std::memcpy(&v, &B->h_nred[k * 4 + norm], sizeof(double));
    return v;
}

// ---------------------------------------------------------------------------
// V-cycle over all members
// ---------------------------------------------------------------------------
// `count` smoothing steps of every member level of size S.n (as in the single-
// hierarchy driver: where the launch covers few nodes, pairs of fused 2-D sweeps
// alternating between the copies of the corrections, the rest one launch per colour)
template <typename T>
void b_smooth(lsmg_batch *B, const BSize &S, hipStream_t s, int count)
{
    const LevelDesc<T> *d = bdescs<T>(B);
    if (B->dim == 2) {
        if (B->fused && fuse_sweep(S.na, sizeof(T))) {
            for (; count >= 2; count -= 2) {
                for (int flip = 0; flip < 2; ++flip) {
                    launch_smooth_rb<T>(d, items(B, S.tiles), S.tiles.n, items(B, S.gh), S.gh.n, flip,
                                        bexec_t(B, s, 0, LSMG_KERNEL_SMOOTH, S.n));
                    launch_ghost_apply<T>(B->dim, d, items(B, S.gh4), S.gh4.n, 1 - flip,
                                          with_tail(bexec_t(B, s, S.ipb[kTGhost], LSMG_KERNEL_GHOST, S.n), S.gh4.tail));
                }
            }
        }
        // folded ghost relaxation: the black launch snapshots the ghosts, one apply launch
        for (; count > 0; --count) {
            launch_smooth_colour<T>(B->dim, d, items(B, S.seg[0]), S.seg[0].n, 0,
                                    bexec_t(B, s, S.ipb[kTSmooth], LSMG_KERNEL_SMOOTH, S.n));
            launch_smooth_colour<T>(B->dim, d, items(B, S.seg1g), S.seg1g.n, 1,
                                    with_tail(bexec_t(B, s, S.ipb[kTSmooth], LSMG_KERNEL_SMOOTH, S.n), S.seg1g.tail));
            launch_ghost_apply<T>(B->dim, d, items(B, S.gh4), S.gh4.n, 0,
                                  with_tail(bexec_t(B, s, S.ipb[kTGhost], LSMG_KERNEL_GHOST, S.n), S.gh4.tail));
        }
        return;
    }
    for (; count > 0; --count) {
        for (int colour = 0; colour < 2; ++colour)
            launch_smooth_colour<T>(B->dim, d, items(B, S.seg[colour]), S.seg[colour].n, colour,
                                    bexec_t(B, s, S.ipb[kTSmooth], LSMG_KERNEL_SMOOTH, S.n));
        const Exec xb = bexec_t(B, s, S.ipb[kTGhost], LSMG_KERNEL_GHOST, S.n);
        const Exec xa = with_tail(bexec_t(B, s, S.ipb[kTGhost], LSMG_KERNEL_GHOST, S.n), S.gh4.tail);
        launch_ghost<T>(B->dim, d, 0, items(B, S.gh), S.gh.n, items(B, S.gh4), S.gh4.n, 0, B->p.ghost_sweeps, true,
                        xb, xa);
    }
}

// The size classes from z0 on: a member's levels lie in the classes of its finest
// size and below, so when the cycle's active members all have their finest level in
// class z0 or a smaller one, the classes before z0 hold no active level and their
// launches (every item skipped by its flag) are left out.
template <typename T>
void b_vcycle(lsmg_batch *B, hipStream_t s, int z0 = 0)
{
    const LevelDesc<T> *d = bdescs<T>(B);
    const int nz = (int)B->sizes.size();
    for (int z = z0; z < nz; ++z) {
        const BSize &S = B->sizes[z];
        if (S.act.n == 0) continue;
        b_smooth<T>(B, S, s, B->p.nu1);
        launch_defect<T>(B->dim, d, items(B, S.act), S.act.n, -1,
                         with_tail(bexec_t(B, s, S.ipb[kTDefect], LSMG_KERNEL_DEFECT, S.n), S.act.tail));
        launch_band<T>(d, items(B, S.band), S.band.n, bexec(B, s, S.ipb[kTBand]));
        launch_restrict<T>(B->dim, d, items(B, S.rcoarse), S.rcoarse.n,
                           with_tail(bexec_t(B, s, S.ipb[kTRestrict], LSMG_KERNEL_RESTRICT, S.n), S.rcoarse.tail));
    }
    const bool f64 = sizeof(T) == 8;
    if (f64 ? B->any_lds64 : B->any_lds32)
        launch_tail_lds<T>(B->dim, d, B->d_tail, B->ndom, f64 ? B->lds_bytes64 : B->lds_bytes32, Exec(s, B->d_act));
    if (!(f64 ? B->all_lds64 : B->all_lds32))
        launch_tail<T>(B->dim, d, B->d_tail, B->ndom, B->tail_na_max, B->tail_stage, Exec(s, B->d_act));
    for (int z = nz - 1; z >= z0; --z) {
        const BSize &S = B->sizes[z];
        if (S.act.n == 0) continue;
        launch_prolong<T>(B->dim, d, items(B, S.act), S.act.n,
                          with_tail(bexec_t(B, s, S.ipb[kTProlong], LSMG_KERNEL_PROLONG, S.n), S.act.tail));
        b_smooth<T>(B, S, s, B->p.nu2);
    }
}

// one linear-solve iteration for every active member (see the single-hierarchy
// driver): V-cycle, or FP32 V-cycle on the FP64 defect; then the FP64 defect
// with its norm in slot 1
void b_cycle_enqueue(lsmg_batch *B, bool mixed, hipStream_t s, bool ctl = false, int z0 = 0)
{
    // (with the device-side tests the norm slots are left zero by the previous
    // cycle, and cleared before a chunk)
    if (!ctl) zero_bnorms(B, 1, 1, s);
    const Exec x0(s, B->d_act);
    if (!mixed) {
        b_vcycle<double>(B, s, z0);
    } else {
        // the FP32 right-hand side and zero correction were written by the FP64
        // defect that precedes every cycle
        b_vcycle<float>(B, s, z0);
        launch_add_f32(B->dim, B->d64, B->d32, items(B, B->lev0), B->lev0.n, with_tail(x0, B->lev0.tail));
    }
    launch_defect<double>(B->dim, B->d64, items(B, B->lev0), B->lev0.n, 1, with_tail(x0, B->lev0.tail),
                          mixed ? B->d32 : nullptr);
    if (!ctl)
        launch_norm_reduce(B->d_norms, B->norm_stride, B->ndom, 1, 1, B->d_nred, s);
    else
        launch_norm_ctl(B->d_norms, B->norm_stride, B->ndom, B->d_nred, B->d_lctl, B->d_dlev, B->d_act, B->d_hist, s);
}

void b_invalidate(lsmg_batch *B)
{
    for (int i = 0; i < 2; ++i) {
        for (hipGraphExec_t &g : B->gexec[i]) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
        for (hipGraphExec_t &g : B->gctl[i]) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    }
}

// the captured cycle from size class z0 on, with the plain norm reduction or (ctl)
// the device-side stopping tests
lsmg_status b_graph(lsmg_batch *B, bool mixed, hipGraphExec_t *out, bool ctl = false, int z0 = 0)
{
    const int gi = mixed ? 1 : 0;
    std::vector<hipGraphExec_t> &gv = ctl ? B->gctl[gi] : B->gexec[gi];
    if (gv.size() < B->sizes.size() + 1) gv.resize(B->sizes.size() + 1, nullptr);
    hipGraphExec_t &ge = gv[z0];
    if (!ge) {
        if (!B->cap) HIPCHK(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
        b_cycle_enqueue(B, mixed, B->cap, ctl, z0);
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamEndCapture(B->cap, &g));
        hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(LSMG_EHIP, "batch graph instantiation failed: %s", hipGetErrorString(e));
    }
    *out = ge;
    return LSMG_OK;
}

// ---------------------------------------------------------------------------
// autotuner: per grid size and kernel class, the workgroup size (work items
// per workgroup: 1, 2, 4 or 8 wavefronts) with the least launch time, measured
// on the batch's own lists with the launches' own dispatch events.  The
// kernels only touch scratch arrays (corrections, defects, coarse right-hand
// sides) that every cycle rewrites before reading, and the workgroup size does
// not change any result.
// ---------------------------------------------------------------------------
lsmg_status ensure_events(lsmg_batch *B, size_t n)
{
    while (B->evpool.size() < n) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        B->evpool.push_back(e);
    }
    return LSMG_OK;
}

template <typename T>
void tune_launch(lsmg_batch *B, const BSize &S, int cls, const Exec &x)
{
    const LevelDesc<T> *d = bdescs<T>(B);
    switch (cls) {
    case kTSmooth:
        launch_smooth_colour<T>(B->dim, d, items(B, S.seg[0]), S.seg[0].n, 0, x);
        break;
    case kTGhost:
        if (B->dim == 2) {
            launch_ghost_apply<T>(B->dim, d, items(B, S.gh4), S.gh4.n, 0, with_tail(x, S.gh4.tail));
            break;
        }
        launch_ghost<T>(B->dim, d, 0, items(B, S.gh), S.gh.n, items(B, S.gh4), S.gh4.n, 0, B->p.ghost_sweeps, true, x,
                        with_tail(Exec(x.s, x.act, x.ipb), S.gh4.tail));
        break;
    case kTDefect:
        launch_defect<T>(B->dim, d, items(B, S.act), S.act.n, -1, with_tail(x, S.act.tail));
        break;
    case kTRestrict:
        launch_restrict<T>(B->dim, d, items(B, S.rcoarse), S.rcoarse.n, with_tail(x, S.rcoarse.tail));
        break;
    case kTProlong:
        launch_prolong<T>(B->dim, d, items(B, S.act), S.act.n, with_tail(x, S.act.tail));
        break;
    default:
        launch_band<T>(d, items(B, S.band), S.band.n, x);
        break;
    }
}

template <typename T>
lsmg_status b_autotune(lsmg_batch *B, int reps)
{
    static const int cand[4] = {1, 2, 4, 8};
    constexpr int nc = 4;
    LSMGCHK(ensure_events(B, (size_t)2 * reps * nc));
    for (BSize &S : B->sizes) {
        if (S.act.n == 0) continue;
        for (int cls = 0; cls < kTClasses; ++cls) {
            // one untimed launch per candidate, then `reps` rounds that time every
            // candidate in turn (so that a drift of the clock or of the caches during
            // tuning does not favour one of them); each candidate scores its median
            for (int ci = 0; ci < nc; ++ci) tune_launch<T>(B, S, cls, bexec(B, B->stream, cand[ci]));
            for (int r = 0; r < reps; ++r)
                for (int ci = 0; ci < nc; ++ci) {
                    Exec x = bexec(B, B->stream, cand[ci]);
                    x.ev0 = B->evpool[2 * (r * nc + ci)];
                    x.ev1 = B->evpool[2 * (r * nc + ci) + 1];
                    tune_launch<T>(B, S, cls, x);
                }
            HIPCHK(hipStreamSynchronize(B->stream));
            double best = 1e300;
            int best_ipb = kItemsPerBlock;
            for (int ci = 0; ci < nc; ++ci) {
                std::vector<double> t(reps, 1e300);
                for (int r = 0; r < reps; ++r) {
                    float ms = 0.0f;
                    if (hipEventElapsedTime(&ms, B->evpool[2 * (r * nc + ci)], B->evpool[2 * (r * nc + ci) + 1]) ==
                        hipSuccess)
                        t[r] = ms;
                }
                std::sort(t.begin(), t.end());
                const double med = t[reps / 2];
                if (med < best) {
                    best = med;
                    best_ipb = cand[ci];
                }
            }
            S.ipb[cls] = best_ipb;
        }
    }
    B->tuned = 1;
    b_invalidate(B);
    return LSMG_OK;
}

// ---------------------------------------------------------------------------
// construction
// ---------------------------------------------------------------------------
struct Job {
    const int4 *src;
    int cnt, dshift;
};

lsmg_status build_lists(lsmg_batch *B)
{
    // grid sizes present in the batch, finest first
    std::vector<int> ns;
    for (lsmg_hierarchy *H : B->mem)
        for (int l = 0; l < H->nlev; ++l) ns.push_back(H->L[l].n);
    std::sort(ns.begin(), ns.end(), std::greater<int>());
    ns.erase(std::unique(ns.begin(), ns.end()), ns.end());
    B->sizes.assign(ns.size(), BSize{});
    std::map<int, int> zi;
    for (size_t z = 0; z < ns.size(); ++z) {
        zi[ns[z]] = (int)z;
        B->sizes[z].n = ns[z];
        for (int c = 0; c < kTClasses; ++c) B->sizes[z].ipb[c] = kItemsPerBlock;
    }
    B->zfin.resize(B->mem.size());
    for (size_t k = 0; k < B->mem.size(); ++k) B->zfin[k] = zi[B->mem[k]->L[0].n];
    std::vector<Job> jobs;
    int total = 0;
    auto add = [&](BList &L, const std::vector<Job> &js) {
        L.off = total;
        L.n = 0;
        L.tail = 0;
        for (const Job &j : js) {
            if (j.cnt <= 0) continue;
            jobs.push_back(j);
            L.n += j.cnt;
            total += j.cnt;
        }
    };
    // leading job lists, then trailing ones (ghost items) counted in L.tail
    auto add_tail = [&](BList &L, std::initializer_list<const std::vector<Job> *> lead, const std::vector<Job> &trail) {
        L.off = total;
        L.n = 0;
        for (const std::vector<Job> *js : lead)
            for (const Job &j : *js) {
                if (j.cnt <= 0) continue;
                jobs.push_back(j);
                L.n += j.cnt;
                total += j.cnt;
            }
        L.tail = 0;
        for (const Job &j : trail) {
            if (j.cnt <= 0) continue;
            jobs.push_back(j);
            L.n += j.cnt;
            L.tail += j.cnt;
            total += j.cnt;
        }
    };
    const int nk = B->ndom;
    for (size_t z = 0; z < ns.size(); ++z) {
        BSize &S = B->sizes[z];
        std::vector<Job> seg0, seg1, gh, gh4, band, til, rco, rco_gh, ico, ico_gh;
        for (int k = 0; k < nk; ++k) {
            const lsmg_hierarchy *H = B->mem[k];
            for (int l = 0; l < H->nlev; ++l) {
                const Level &Lv = H->L[l];
                if (Lv.n != ns[z]) continue;
                const int ds = B->d0[k];
                if (l + 1 < H->nlev) {
                    const Level &C = H->L[l + 1];
                    ico.push_back({C.w_seg(0), C.nseg[0] + C.nseg[1], ds});
                    ico_gh.push_back({C.w_gh(), C.nghc, ds});
                }
                if (l >= H->tail_l0) continue;
                seg0.push_back({Lv.w_seg(0), Lv.nseg[0], ds});
                seg1.push_back({Lv.w_seg(1), Lv.nseg[1], ds});
                if (Lv.tiles) til.push_back({Lv.tiles, Lv.ntile, ds});
                S.na += Lv.na;
                gh.push_back({Lv.w_gh(), Lv.nghc, ds});
                gh4.push_back({Lv.w_gh4(), Lv.nghc4, ds});
                band.push_back({Lv.w_band(), Lv.nbandc, ds});
                const Level &C = H->L[l + 1];
                rco.push_back({C.w_seg(0), C.nseg[0] + C.nseg[1], ds});
                rco_gh.push_back({C.w_gh(), C.nghc, ds});
            }
        }
        add(S.seg[0], seg0);
        add(S.seg[1], seg1);
        // the members' row segments first, then all their ghost items
        add_tail(S.seg1g, {&seg1}, gh);
        add(S.tiles, til);
        add(S.gh, gh);
        add_tail(S.gh4, {}, gh4);
        add_tail(S.act, {&seg0, &seg1}, gh);
        add(S.band, band);
        add_tail(S.rcoarse, {&rco}, rco_gh);
        add_tail(S.icoarse, {&ico}, ico_gh);
    }
    std::vector<Job> l0, l0_gh, al, al_gh;
    for (int k = 0; k < nk; ++k) {
        const lsmg_hierarchy *H = B->mem[k];
        const Level &L0 = H->L[0];
        l0.push_back({L0.w_seg(0), L0.nseg[0] + L0.nseg[1], B->d0[k]});
        l0_gh.push_back({L0.w_gh(), L0.nghc, B->d0[k]});
        for (int l = 0; l < H->nlev; ++l) {
            const Level &Lv = H->L[l];
            al.push_back({Lv.w_seg(0), Lv.nseg[0] + Lv.nseg[1], B->d0[k]});
            al_gh.push_back({Lv.w_gh(), Lv.nghc, B->d0[k]});
        }
    }
    add_tail(B->lev0, {&l0}, l0_gh);
    add_tail(B->all, {&al}, al_gh);
    B->npool = total;
    LSMGCHK(B->alloc(&B->pool, total));
    // one launch copies every block; the job table is freed after the copy
    std::vector<ItemCopy> hj(jobs.size());
    int off = 0;
    for (size_t i = 0; i < jobs.size(); ++i) {
        hj[i].src = jobs[i].src;
        hj[i].cnt = jobs[i].cnt;
        hj[i].off = off;
        hj[i].dshift = jobs[i].dshift;
        hj[i].pad = 0;
        off += jobs[i].cnt;
    }
    if (!hj.empty()) {
        ItemCopy *dj = nullptr;
        DevTemps tmp(B->dmem, B->stream);
        LSMGCHK(tmp.get(&dj, (long long)hj.size()));
        HIPCHK(hipMemcpyAsync(dj, hj.data(), sizeof(ItemCopy) * hj.size(), hipMemcpyHostToDevice, B->stream));
        launch_copy_items(dj, (int)hj.size(), B->pool, B->stream);
        HIPCHK(hipStreamSynchronize(B->stream));
    }
    return LSMG_OK;
}

bool same_params(const lsmg_params &a, const lsmg_params &b)
{
    return a.a == b.a && a.d == b.d && a.m_s == b.m_s && a.m_c == b.m_c && a.alpha == b.alpha && a.beta == b.beta &&
           a.tau_s == b.tau_s && a.nu1 == b.nu1 && a.nu2 == b.nu2 && a.ghost_sweeps == b.ghost_sweeps &&
           a.ghost_sweeps_coarse == b.ghost_sweeps_coarse && a.sweeps_lambda == b.sweeps_lambda &&
           a.band_steps == b.band_steps && a.ghost_c_new == b.ghost_c_new && a.coarsest_n == b.coarsest_n &&
           a.precision == b.precision && a.newton_tol == b.newton_tol && a.newton_max == b.newton_max &&
           a.lin_rtol == b.lin_rtol && a.cycles_max == b.cycles_max && a.bc == b.bc &&
           a.cycle_gamma == b.cycle_gamma && a.fmg == b.fmg;
}

lsmg_status b_build(lsmg_batch *B)
{
    const int nk = B->ndom;
    B->d0.assign(nk, 0);
    int nd = 0;
    for (int k = 0; k < nk; ++k) {
        B->d0[k] = nd;
        nd += B->mem[k]->nlev;
    }
    B->ndesc = nd;
    B->hd64.assign(nd, LevelDesc<double>{});
    B->hd32.assign(nd, LevelDesc<float>{});
    LSMGCHK(B->alloc(&B->d64, nd));
    LSMGCHK(B->alloc(&B->d32, nd));
    B->norm_stride = (long long)nk * kNormSlots;
    LSMGCHK(B->alloc(&B->d_norms, 4 * B->norm_stride));
    LSMGCHK(B->alloc(&B->d_nred, 4LL * nk));
    // flag rows: 0 the cycle (and every launch of lsmg_batch_step), 1 step starts,
    // 2 linearisations, 3 Newton updates, 4 commits (lsmg_batch_advance)
    LSMGCHK(B->alloc(&B->d_act, (long long)kFlagRows * nd));
    LSMGCHK(B->alloc(&B->d_cstatus, nk));
    HIPCHK(hipHostMalloc(&B->h_nred, sizeof(unsigned long long) * 4 * nk, hipHostMallocDefault));
    HIPCHK(hipHostMalloc(&B->h_act, sizeof(int) * kFlagRows * nd, hipHostMallocDefault));
    HIPCHK(hipHostMalloc(&B->h_cstatus, sizeof(int) * nk, hipHostMallocDefault));
    {
        const int cmax = std::max(B->p.cycles_max, 1);
        LSMGCHK(B->alloc(&B->d_lctl, nk));
        LSMGCHK(B->alloc(&B->d_hist, (long long)cmax * nk));
        LSMGCHK(B->alloc(&B->d_dlev, nk));
        HIPCHK(hipHostMalloc(&B->h_lctl, sizeof(LinCtl) * nk, hipHostMallocDefault));
        HIPCHK(hipHostMalloc(&B->h_hist, sizeof(double) * (size_t)cmax * nk, hipHostMallocDefault));
        std::vector<int2> dl(nk);
        for (int k = 0; k < nk; ++k) dl[k] = make_int2(B->d0[k], B->mem[k]->nlev);
        HIPCHK(hipMemcpyAsync(B->d_dlev, dl.data(), sizeof(int2) * nk, hipMemcpyHostToDevice, B->stream));
        HIPCHK(hipStreamSynchronize(B->stream));
        B->last_cycles.assign(nk, 0);
    }
    // coarse tails and coarsest operators, one workgroup per member
    std::vector<TailArgs> ta(nk);
    std::vector<CoarseArgs> ca(nk);
    for (int k = 0; k < nk; ++k) {
        const lsmg_hierarchy *H = B->mem[k];
        ta[k] = tail_args(H, H->tail_l0, B->d0[k]);
        B->tail_na_max = std::max(B->tail_na_max, H->L[H->nlev - 1].na);
        B->tail_stage = B->tail_stage && ta[k].nstage <= kTailStageInts;
        const bool l64 = tail_in_lds<double>(H), l32 = tail_in_lds<float>(H);
        B->any_lds64 = B->any_lds64 || l64;
        B->any_lds32 = B->any_lds32 || l32;
        B->all_lds64 = B->all_lds64 && l64;
        B->all_lds32 = B->all_lds32 && l32;
        if (l64) B->lds_bytes64 = std::max(B->lds_bytes64, H->tail_sz.bytes<double>());
        if (l32) B->lds_bytes32 = std::max(B->lds_bytes32, H->tail_sz.bytes<float>());
        ca[k] = CoarseArgs{};
        ca[k].desc = B->d0[k] + H->nlev - 1;
        ca[k].c2s = H->L[H->nlev - 1].c2s;
        ca[k].M = H->lu;
        ca[k].Ainv = H->ainv;
        ca[k].status = B->d_cstatus + k;
        B->coarse_n_max = std::max(B->coarse_n_max, H->L[H->nlev - 1].na);
    }
    LSMGCHK(B->alloc(&B->d_tail, nk));
    LSMGCHK(B->alloc(&B->d_coarse, nk));
    HIPCHK(hipMemcpyAsync(B->d_tail, ta.data(), sizeof(TailArgs) * nk, hipMemcpyHostToDevice, B->stream));
    HIPCHK(hipMemcpyAsync(B->d_coarse, ca.data(), sizeof(CoarseArgs) * nk, hipMemcpyHostToDevice, B->stream));
    LSMGCHK(build_lists(B));
    LSMGCHK(refresh_descs(B, nullptr, nullptr, nullptr));
    return LSMG_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

lsmg_status lsmg_batch_create(lsmg_hierarchy *const *members, int count, const lsmg_allocator *allocator,
                              void *stream, lsmg_batch **out)
{
    if (!out) return fail(LSMG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!members || count < 1) return fail(LSMG_EINVAL, "a batch needs at least one member");
    for (int k = 0; k < count; ++k) {
        if (!members[k]) return fail(LSMG_EINVAL, "member %d is NULL", k);
        for (int j = 0; j < k; ++j)
            if (members[j] == members[k]) return fail(LSMG_EINVAL, "member %d appears twice", k);
        if (members[k]->dim != members[0]->dim) return fail(LSMG_EINVAL, "members differ in dimension");
        if (!same_params(members[k]->p, members[0]->p)) return fail(LSMG_EINVAL, "members differ in parameters");
        if (members[k]->p.cycle_gamma != 1 || members[k]->p.fmg != 0)
            return fail(LSMG_ENOTIMPL, "batches run V-cycles (cycle_gamma = 1) without full multigrid (fmg = 0)");
        if (!members[k]->p.ghost_c_new)
            return fail(LSMG_ENOTIMPL, "batches use the composed ghost relaxation (ghost_c_new = 1)");
        if (members[k]->p.krylov_m != 0)
            return fail(LSMG_ENOTIMPL, "batches iterate V-cycles (krylov_m = 0)");
        if (members[k]->p.precision == 1 && !members[k]->have32) return fail(LSMG_EINVAL, "member %d has no FP32 copy", k);
    }
    lsmg_batch *B = new (std::nothrow) lsmg_batch();
    if (!B) return fail(LSMG_EOOM, "host allocation");
    if (allocator) {
        if (!allocator->alloc || !allocator->free) {
            delete B;
            return fail(LSMG_EINVAL, "allocator needs both alloc and free");
        }
        B->dmem.alloc_fn = allocator->alloc;
        B->dmem.free_fn = allocator->free;
        B->dmem.ctx = allocator->ctx;
    }
    B->dim = members[0]->dim;
    B->p = members[0]->p;
    B->fused = B->dim == 2;
    for (int k = 0; k < count; ++k) B->fused = B->fused && members[k]->p.fused_sweep;
    B->ndom = count;
    B->stream = (hipStream_t)stream;
    B->mem.assign(members, members + count);
    if (const char *e = std::getenv("LSMG_GRAPHS")) B->use_graphs = std::atoi(e) != 0;
    lsmg_status st = b_build(B);
    if (st != LSMG_OK) {
        (void)hipStreamSynchronize(B->stream);
        delete B;
        return st;
    }
    *out = B;
    return LSMG_OK;
}

void lsmg_batch_destroy(lsmg_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    delete b;
}

lsmg_status lsmg_batch_sweep_fused(const lsmg_batch *b, int n, int precision, int *fused)
{
    if (!b || !fused || (precision != 0 && precision != 1)) return fail(LSMG_EINVAL, "bad argument");
    *fused = 0;
    for (const BSize &S : b->sizes)
        if (S.n == n)
            *fused = b->fused && S.tiles.n > 0 && fuse_sweep(S.na, precision == 0 ? sizeof(double) : sizeof(float));
    return LSMG_OK;
}

lsmg_status lsmg_batch_set_autotune(lsmg_batch *b, int enable)
{
    if (!b) return fail(LSMG_EINVAL, "batch is NULL");
    b->autotune = enable ? 1 : 0;
    if (!enable && b->tuned) {
        for (BSize &S : b->sizes)
            for (int c = 0; c < kTClasses; ++c) S.ipb[c] = kItemsPerBlock;
        b->tuned = 0;
        b_invalidate(b);
    }
    return LSMG_OK;
}

lsmg_status lsmg_batch_tuning(const lsmg_batch *b, int cap, int *count, int *sizes, int *ipb)
{
    if (!b || !count) return fail(LSMG_EINVAL, "NULL argument");
    *count = (int)b->sizes.size();
    for (int z = 0; z < *count && z < cap; ++z) {
        if (sizes) sizes[z] = b->sizes[z].n;
        if (ipb)
            for (int c = 0; c < kTClasses; ++c) ipb[z * kTClasses + c] = b->sizes[z].ipb[c];
    }
    return LSMG_OK;
}

lsmg_status lsmg_batch_step(lsmg_batch *b, lsmg_state *const *states, double dt, const double *const *d_sb,
                            const double *sb_const, lsmg_status *status, lsmg_step_stats *stats)
{
    if (!b || !states) return fail(LSMG_EINVAL, "NULL argument");
    lsmg_batch *B = b;
    const int nk = B->ndom;
    for (int k = 0; k < nk; ++k)
        if (!states[k] || states[k]->h != B->mem[k]) return fail(LSMG_EINVAL, "state %d does not belong to member %d", k, k);
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(LSMG_EINVAL, "dt must be positive and finite");
    // descriptors: dt of every member and the arrays of this step
    bool changed = dt != B->dt;
    B->dt = dt;
    for (int k = 0; k < nk; ++k)
        if (B->mem[k]->dt != dt) {
            LSMGCHK(set_dt(B->mem[k], dt));
            changed = true;
        }
    std::vector<const lsmg_state *> sv(states, states + nk);
    std::vector<const double *> sbv(nk, nullptr);
    std::vector<double> sbc(nk, 1.0);
    for (int k = 0; k < nk; ++k) {
        if (d_sb) sbv[k] = d_sb[k];
        if (sb_const) sbc[k] = sb_const[k];
    }
    if (changed || sv != B->last_states || sbv != B->last_sb || sbc != B->last_sbc) {
        LSMGCHK(refresh_descs(B, states, sbv.data(), sbc.data()));
        B->last_states = sv;
        B->last_sb = sbv;
        B->last_sbc = sbc;
    }
    const bool mixed = B->p.precision == 1;
    hipStream_t s = B->stream;
    const Exec x0(s, B->d_act);
    std::vector<lsmg_status> rc(nk, LSMG_ENOCONV);
    std::vector<char> on(nk, 1), lin(nk, 0);
    std::vector<int> cycles(nk, 0), nrho(nk, 0), iters(nk, 0);
    std::vector<double> nF(nk, 0.0), rho_last(nk, 0.0), logsum(nk, 0.0), dwrel(nk, 0.0), rprev(nk, 0.0);
    LSMGCHK(set_flags(B, on));
    // explicit half, first iterate and F(W^n)
    launch_explicit_half(B->dim, B->d64, items(B, B->lev0), B->lev0.n, with_tail(x0, B->lev0.tail));
    zero_bnorms(B, 0, 4, s);
    launch_residual(B->dim, B->d64, items(B, B->lev0), B->lev0.n, 0, with_tail(x0, B->lev0.tail));
    LSMGCHK(read_bnorms(B, 0, 1));
    for (int k = 0; k < nk; ++k) nF[k] = bnorm(B, k, 0);
    for (int it = 1; it <= B->p.newton_max; ++it) {
        int nact = 0;
        for (int k = 0; k < nk; ++k) {
            if (!on[k]) continue;
            if (!std::isfinite(nF[k])) {
                rc[k] = LSMG_ENONFINITE;
                on[k] = 0;
                continue;
            }
            iters[k] = it;
            ++nact;
        }
        if (nact == 0) break;
        LSMGCHK(set_flags(B, on));
        // linearisation: coarse (s, c) level by level (from the first size class that
        // holds a level of an iterating member), FP32 copies, coarsest inverses
        int zl = (int)B->sizes.size();
        for (int k = 0; k < nk; ++k)
            if (on[k]) zl = std::min(zl, B->zfin[k]);
        for (int z = zl; z < (int)B->sizes.size(); ++z) {
            const BSize &S = B->sizes[z];
            launch_inject<double>(B->dim, B->d64, items(B, S.icoarse), S.icoarse.n, with_tail(x0, S.icoarse.tail));
        }
        if (mixed) launch_to_f32(B->dim, B->d64, B->d32, items(B, B->all), B->all.n, 0, with_tail(x0, B->all.tail));
        launch_coarse_factor(B->dim, B->d64, B->d_coarse, nk, B->coarse_n_max, x0);
        // the factorisations' status comes back with the first chunk's norms; a member
        // whose coarsest operator is singular or not finite leaves the step then (its
        // cycles until that point touch only its own arrays, and are not counted)
        HIPCHK(hipMemcpyAsync(B->h_cstatus, B->d_cstatus, sizeof(int) * nk, hipMemcpyDeviceToHost, s));
        bool status_read = false;
        auto take_status = [&]() {
            for (int k = 0; k < nk; ++k)
                if (on[k] && B->h_cstatus[k] != 0) {
                    rc[k] = LSMG_ENONFINITE;
                    on[k] = 0;
                    lin[k] = 0;
                }
            status_read = true;
        };
        LSMGCHK(set_flags(B, on));
        if (B->autotune && !B->tuned) {
            if (mixed) LSMGCHK(b_autotune<float>(B, 5));
            else LSMGCHK(b_autotune<double>(B, 5));
        }
        // linear solves J dW = F from dW = 0
        if (mixed)
            launch_start_mixed(B->dim, B->d64, items(B, B->lev0), B->lev0.n, with_tail(x0, B->lev0.tail), B->d32);
        else
            launch_zero_x<double>(B->dim, B->d64, items(B, B->lev0), B->lev0.n, with_tail(x0, B->lev0.tail));
        for (int k = 0; k < nk; ++k) {
            lin[k] = on[k];
            rprev[k] = nF[k];
        }
        // cycles in chunks: each member's stopping tests (|r| <= lin_rtol |F|, a
        // non-finite |r|) run on the device after every cycle of a chunk (the captured
        // cycle replayed back to back), and the norms come back once per chunk.  A chunk
        // ends one cycle before the longest of the solving members' previous solves would
        // (later chunks: one cycle each), so it rarely holds a cycle no member needs.  The
        // host replays the same tests on the norms, so members run exactly the cycles
        // they would with a round trip after each
        std::vector<int> solve_cycles(nk, 0);
        int q = 0;
        while (q < B->p.cycles_max) {
            int nlin = 0, kc = 1;
            for (int k = 0; k < nk; ++k) {
                if (lin[k] && rprev[k] <= B->p.lin_rtol * nF[k]) lin[k] = 0;
                if (!lin[k]) continue;
                ++nlin;
                kc = std::max(kc, B->last_cycles[k] - 1 - solve_cycles[k]);
            }
            if (nlin == 0) break;
            kc = std::min(kc, B->p.cycles_max - q);
            for (int k = 0; k < nk; ++k) B->h_lctl[k] = LinCtl{B->p.lin_rtol * nF[k], rprev[k], lin[k] ? 1 : 0, 0};
            HIPCHK(hipMemcpyAsync(B->d_lctl, B->h_lctl, sizeof(LinCtl) * nk, hipMemcpyHostToDevice, s));
            LSMGCHK(set_flags(B, lin));
            zero_bnorms(B, 1, 1, s);
            // the first size class holding a level of a solving member (members only
            // leave during a chunk)
            int z0 = (int)B->sizes.size();
            for (int k = 0; k < nk; ++k)
                if (lin[k]) z0 = std::min(z0, B->zfin[k]);
            hipGraphExec_t gc = nullptr;
            // timed launches run direct: events inside a graph cannot be timed
            if (B->use_graphs && B->prof_kernel < 0) LSMGCHK(b_graph(B, mixed, &gc, true, z0));
            for (int j = 0; j < kc; ++j) {
                if (gc) HIPCHK(hipGraphLaunch(gc, s));
                else b_cycle_enqueue(B, mixed, s, true, z0);
            }
            B->act_last.clear();   // the chunk cleared the flags of the members that stopped
            HIPCHK(hipMemcpyAsync(B->h_hist, B->d_hist, sizeof(double) * (size_t)kc * nk, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (!gc) b_prof_collect(B);
            if (!status_read) take_status();
            for (int j = 0; j < kc; ++j)
                for (int k = 0; k < nk; ++k) {
                    if (!lin[k]) continue;
                    if (j > 0 && rprev[k] <= B->p.lin_rtol * nF[k]) {
                        lin[k] = 0;
                        continue;
                    }
                    // a member records the norms of its cycles from the chunk's first on
                    const double rq = B->h_hist[(size_t)j * nk + k];
                    ++cycles[k];
                    ++solve_cycles[k];
                    rho_last[k] = rprev[k] > 0.0 ? rq / rprev[k] : 0.0;
                    if (rho_last[k] > 0.0) logsum[k] += std::log(rho_last[k]);
                    ++nrho[k];
                    rprev[k] = rq;
                    if (!std::isfinite(rq)) lin[k] = 0;
                }
            q += kc;
        }
        if (!status_read) {
            HIPCHK(hipStreamSynchronize(s));
            take_status();
        }
        for (int k = 0; k < nk; ++k)
            if (solve_cycles[k] > 0) B->last_cycles[k] = solve_cycles[k];
        // Newton update and the new residual
        LSMGCHK(set_flags(B, on));
        zero_bnorms(B, 0, 4, s);
        launch_newton_update(B->dim, B->d64, items(B, B->lev0), B->lev0.n, with_tail(x0, B->lev0.tail));
        launch_residual(B->dim, B->d64, items(B, B->lev0), B->lev0.n, 0, with_tail(x0, B->lev0.tail));
        LSMGCHK(read_bnorms(B, 0, 4));
        for (int k = 0; k < nk; ++k) {
            if (!on[k]) continue;
            nF[k] = bnorm(B, k, 0);
            const double nD = bnorm(B, k, 2), nW = bnorm(B, k, 3);
            dwrel[k] = nW > 0.0 ? nD / nW : nD;
            if (!std::isfinite(nF[k]) || !std::isfinite(dwrel[k])) {
                rc[k] = LSMG_ENONFINITE;
                on[k] = 0;
            } else if ((nF[k] < dwrel[k] ? nF[k] : dwrel[k]) < B->p.newton_tol) {
                rc[k] = LSMG_OK;
                on[k] = 0;
            }
        }
    }
    // commit the members that converged
    std::vector<char> ok(nk, 0);
    lsmg_status first_bad = LSMG_OK;
    for (int k = 0; k < nk; ++k) {
        ok[k] = rc[k] == LSMG_OK;
        if (!ok[k] && first_bad == LSMG_OK) first_bad = rc[k];
    }
    LSMGCHK(set_flags(B, ok));
    launch_commit(B->dim, B->d64, items(B, B->lev0), B->lev0.n, with_tail(x0, B->lev0.tail));
    HIPCHK(hipStreamSynchronize(s));
    for (int k = 0; k < nk; ++k) {
        if (status) status[k] = rc[k];
        if (stats) {
            stats[k].newton_iters = iters[k];
            stats[k].vcycles = cycles[k];
            stats[k].res_inf = nF[k];
            stats[k].rho_last = rho_last[k];
            stats[k].rho_geo = nrho[k] > 0 ? std::exp(logsum[k] / nrho[k]) : 0.0;
            stats[k].dw_rel = dwrel[k];
        }
        B->mem[k]->lin_set = false;
    }
    if (first_bad != LSMG_OK) {
        for (int k = 0; k < nk; ++k)
            if (rc[k] != LSMG_OK) {
                fail(rc[k], "member %d: %s", k,
                     rc[k] == LSMG_ENOCONV ? "Newton did not converge" : "non-finite iterate or singular coarsest operator");
                break;
            }
    }
    return first_bad;
}

lsmg_status lsmg_batch_advance(lsmg_batch *b, lsmg_state *const *states, double dt, const double *sb_const,
                               const int *remaining, int max_ticks, int *ended, lsmg_status *status,
                               lsmg_step_stats *stats, double *step_ms, int *ticks_run)
{
    if (!b || !states || !remaining) return fail(LSMG_EINVAL, "NULL argument");
    lsmg_batch *B = b;
    const int nk = B->ndom;
    for (int k = 0; k < nk; ++k)
        if (!states[k] || states[k]->h != B->mem[k]) return fail(LSMG_EINVAL, "state %d does not belong to member %d", k, k);
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(LSMG_EINVAL, "dt must be positive and finite");
    bool changed = dt != B->dt;
    B->dt = dt;
    for (int k = 0; k < nk; ++k)
        if (B->mem[k]->dt != dt) {
            LSMGCHK(set_dt(B->mem[k], dt));
            changed = true;
        }
    std::vector<const lsmg_state *> sv(states, states + nk);
    std::vector<const double *> sbv(nk, nullptr);
    std::vector<double> sbc(nk, 1.0);
    for (int k = 0; k < nk; ++k)
        if (sb_const) sbc[k] = sb_const[k];
    if (changed || sv != B->last_states || sbv != B->last_sb || sbc != B->last_sbc) {
        LSMGCHK(refresh_descs(B, states, sbv.data(), sbc.data()));
        B->last_states = sv;
        B->last_sb = sbv;
        B->last_sbc = sbc;
    }
    const bool mixed = B->p.precision == 1;
    hipStream_t s = B->stream;
    const int nd = B->ndesc;
    const Exec xs(s, B->d_act + (size_t)kFStart * nd), xl(s, B->d_act + (size_t)kFLin * nd),
        xu(s, B->d_act + (size_t)kFUpdate * nd), xm(s, B->d_act + (size_t)kFCommit * nd);
    for (int k = 0; k < nk; ++k) {
        if (ended) ended[k] = 0;
        if (status) status[k] = LSMG_OK;
        RunState &R = B->mem[k]->run;
        if (R.next == RunState::Idle && remaining[k] > 0) R.next = RunState::Start;
    }
    int ticks = 0;
    bool any_end = false;
    while (ticks < max_ticks && !any_end) {
        std::vector<std::vector<char>> rows(kFlagRows, std::vector<char>(nk, 0));
        std::vector<char> &fc = rows[kFCycle], &fs = rows[kFStart], &fl = rows[kFLin], &fu = rows[kFUpdate];
        int nwork = 0;
        for (int k = 0; k < nk; ++k) {
            RunState &R = B->mem[k]->run;
            switch (R.next) {
            case RunState::Start:
                fs[k] = fl[k] = 1;
                break;
            case RunState::Lin:
                fl[k] = 1;
                // the first cycle of the new linear solve runs unless |F| = 0
                if (!(R.nF <= B->p.lin_rtol * R.nF)) fc[k] = 1;
                break;
            case RunState::Solve:
                if (!R.force_update && R.q < B->p.cycles_max && !(R.rprev <= B->p.lin_rtol * R.nF)) fc[k] = 1;
                else fu[k] = 1;
                break;
            default:
                break;
            }
            nwork += fs[k] | fl[k] | fc[k] | fu[k];
        }
        if (nwork == 0) break;
        LSMGCHK(set_flag_rows(B, rows));
        const double t_tick = now_ms();
        for (int k = 0; k < nk; ++k)
            if (fs[k]) B->mem[k]->run.t_start = t_tick;
        zero_bnorms(B, 0, 4, s);
        bool has_s = false, has_l = false, has_c = false, has_u = false;
        for (int k = 0; k < nk; ++k) {
            has_s |= fs[k];
            has_l |= fl[k];
            has_c |= fc[k];
            has_u |= fu[k];
        }
        if (has_s) {
            launch_explicit_half(B->dim, B->d64, items(B, B->lev0), B->lev0.n, with_tail(xs, B->lev0.tail));
            launch_residual(B->dim, B->d64, items(B, B->lev0), B->lev0.n, 0, with_tail(xs, B->lev0.tail));
        }
        // the first size classes holding a level of a member being linearised, or cycled
        int zl = (int)B->sizes.size(), zc = zl;
        for (int k = 0; k < nk; ++k) {
            if (fl[k]) zl = std::min(zl, B->zfin[k]);
            if (fc[k]) zc = std::min(zc, B->zfin[k]);
        }
        if (has_l) {
            for (int z = zl; z < (int)B->sizes.size(); ++z) {
                const BSize &S = B->sizes[z];
                launch_inject<double>(B->dim, B->d64, items(B, S.icoarse), S.icoarse.n, with_tail(xl, S.icoarse.tail));
            }
            if (mixed) launch_to_f32(B->dim, B->d64, B->d32, items(B, B->all), B->all.n, 0, with_tail(xl, B->all.tail));
            launch_coarse_factor(B->dim, B->d64, B->d_coarse, nk, B->coarse_n_max, xl);
            if (B->autotune && !B->tuned) {
                // workgroup sizes, timed on the members being linearised (flag row 0 set to
                // them for the tuner's launches): their scratch arrays are reset below and
                // by their first cycle, and no other member's arrays are touched
                std::vector<std::vector<char>> trow = rows;
                trow[kFCycle] = fl;
                LSMGCHK(set_flag_rows(B, trow));
                if (mixed) LSMGCHK(b_autotune<float>(B, 5));
                else LSMGCHK(b_autotune<double>(B, 5));
                LSMGCHK(set_flag_rows(B, rows));
            }
            if (mixed)
                launch_start_mixed(B->dim, B->d64, items(B, B->lev0), B->lev0.n, with_tail(xl, B->lev0.tail), B->d32);
            else
                launch_zero_x<double>(B->dim, B->d64, items(B, B->lev0), B->lev0.n, with_tail(xl, B->lev0.tail));
        }
        if (has_c) {
            hipGraphExec_t ge = nullptr;
            if (B->use_graphs && B->prof_kernel < 0) LSMGCHK(b_graph(B, mixed, &ge, false, zc));
            if (ge) HIPCHK(hipGraphLaunch(ge, s));
            else b_cycle_enqueue(B, mixed, s, false, zc);
        }
        if (has_u) {
            launch_newton_update(B->dim, B->d64, items(B, B->lev0), B->lev0.n, with_tail(xu, B->lev0.tail));
            launch_residual(B->dim, B->d64, items(B, B->lev0), B->lev0.n, 0, with_tail(xu, B->lev0.tail));
        }
        launch_norm_reduce(B->d_norms, B->norm_stride, nk, 0, 4, B->d_nred, s);
        HIPCHK(hipMemcpyAsync(B->h_nred, B->d_nred, sizeof(unsigned long long) * 4 * nk, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(B->h_cstatus, B->d_cstatus, sizeof(int) * nk, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (B->prof_kernel >= 0) b_prof_collect(B);
        ++ticks;
        const double t_end = now_ms();
        std::vector<char> commit(nk, 0);
        for (int k = 0; k < nk; ++k) {
            RunState &R = B->mem[k]->run;
            lsmg_status rc = LSMG_OK;
            bool done = false;
            if (fs[k]) {
                R.nF = bnorm(B, k, 0);
                R.it = 1;
                R.cycles = R.nrho = 0;
                R.rho_last = R.logsum = R.dwrel = 0.0;
                if (!std::isfinite(R.nF)) rc = LSMG_ENONFINITE;
            }
            if (fl[k] && rc == LSMG_OK) {
                if (B->h_cstatus[k] != 0) rc = LSMG_ENONFINITE;
                R.q = 0;
                R.rprev = R.nF;
                R.force_update = false;
                R.next = RunState::Solve;
            }
            if (fc[k] && rc == LSMG_OK) {
                const double rq = bnorm(B, k, 1);
                ++R.q;
                ++R.cycles;
                R.rho_last = R.rprev > 0.0 ? rq / R.rprev : 0.0;
                if (R.rho_last > 0.0) R.logsum += std::log(R.rho_last);
                ++R.nrho;
                R.rprev = rq;
                if (!std::isfinite(rq)) R.force_update = true;
            }
            if (fu[k]) {
                R.nF = bnorm(B, k, 0);
                const double nD = bnorm(B, k, 2), nW = bnorm(B, k, 3);
                R.dwrel = nW > 0.0 ? nD / nW : nD;
                if (!std::isfinite(R.nF) || !std::isfinite(R.dwrel)) rc = LSMG_ENONFINITE;
                else if ((R.nF < R.dwrel ? R.nF : R.dwrel) < B->p.newton_tol) done = true;
                else if (R.it >= B->p.newton_max) rc = LSMG_ENOCONV;
                else {
                    ++R.it;
                    R.next = RunState::Lin;
                }
            }
            if (rc != LSMG_OK || done) {
                any_end = true;
                if (ended) ended[k] = 1;
                if (status) status[k] = rc;
                if (stats) {
                    stats[k].newton_iters = R.it;
                    stats[k].vcycles = R.cycles;
                    stats[k].res_inf = R.nF;
                    stats[k].rho_last = R.rho_last;
                    stats[k].rho_geo = R.nrho > 0 ? std::exp(R.logsum / R.nrho) : 0.0;
                    stats[k].dw_rel = R.dwrel;
                }
                if (step_ms) step_ms[k] = t_end - R.t_start;
                if (done) commit[k] = 1;
                // a failed step keeps W^n and ends the member's run; a finished one
                // starts the next step in the following call if steps remain
                R.next = RunState::Idle;
                B->mem[k]->lin_set = false;
            }
        }
        bool any_commit = false;
        for (int k = 0; k < nk; ++k) any_commit |= commit[k];
        if (any_commit) {
            std::vector<std::vector<char>> crow(kFlagRows, std::vector<char>(nk, 0));
            crow[kFCommit] = commit;
            LSMGCHK(set_flag_rows(B, crow));
            launch_commit(B->dim, B->d64, items(B, B->lev0), B->lev0.n, with_tail(xm, B->lev0.tail));
            HIPCHK(hipStreamSynchronize(s));
        }
    }
    if (ticks_run) *ticks_run = ticks;
    return LSMG_OK;
}

lsmg_status lsmg_batch_profile_start(lsmg_batch *b, int kernel, int n)
{
    if (!b) return fail(LSMG_EINVAL, "batch is NULL");
    if (kernel < LSMG_KERNEL_SMOOTH || kernel > LSMG_KERNEL_GHOST) return fail(LSMG_EINVAL, "unknown kernel class");
    HIPCHK(hipStreamSynchronize(b->stream));
    b->prof_kernel = kernel;
    b->prof_n = n;
    b->prof_used = 0;
    b->prof_acc_ms = 0.0;
    b->prof_acc_n = 0;
    return LSMG_OK;
}

lsmg_status lsmg_batch_profile_stop(lsmg_batch *b, int *launches, double *total_ms)
{
    if (!b) return fail(LSMG_EINVAL, "batch is NULL");
    HIPCHK(hipStreamSynchronize(b->stream));
    b_prof_collect(b);
    if (launches) *launches = (int)b->prof_acc_n;
    if (total_ms) *total_ms = b->prof_acc_ms;
    b->prof_kernel = -1;
    b->prof_n = -1;
    return LSMG_OK;
}

}  // extern "C"
