// Host-side state of the lsmg library shared by its translation units: the
// hierarchy and state objects behind the opaque C handles, error reporting and
// the helpers both the single-hierarchy and the batch drivers use.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lsmg.h"
#include "lsmg_dev.hpp"
#include "lsmg_host.hpp"

namespace lsmg {

// records the message of a failing call (thread-local) and returns its status
lsmg_status fail(lsmg_status st, const char *fmt, ...);

#define HIPCHK(x)                                                                                      \
    do {                                                                                               \
        hipError_t e_ = (x);                                                                           \
        if (e_ != hipSuccess) return ::lsmg::fail(LSMG_EHIP, "%s failed: %s", #x, hipGetErrorString(e_)); \
    } while (0)

#define LSMGCHK(x)                        \
    do {                                  \
        lsmg_status s_ = (x);             \
        if (s_ != LSMG_OK) return s_;     \
    } while (0)

struct Level {
    int n = 0, Wp = 0;
    long long rows = 0, cs = 0, ssize = 0;
    double h = 0.0;
    int ni = 0, ng = 0, na = 0, nb = 0, bmax = 0;
    uint8_t *type = nullptr, *ext = nullptr;
    int *cmap = nullptr, *c2s = nullptr;
    int64_t *c2g = nullptr;
    double *s = nullptr, *c = nullptr, *rhs_s = nullptr, *rhs_c = nullptr, *x_s = nullptr, *x_c = nullptr,
           *r_s = nullptr, *r_c = nullptr;
    int *g_idx = nullptr, *g_ijk = nullptr, *g_st = nullptr, *g_stg = nullptr, *g_stc = nullptr, *g_order = nullptr,
        *g_bfall = nullptr;
    double *g_w = nullptr, *g_B = nullptr, *g_nrm = nullptr, *g_nrow = nullptr, *g_buf0 = nullptr, *g_buf1 = nullptr;
    int *b_idx = nullptr, *b_cnt = nullptr, *b_src = nullptr;
    double *b_wt = nullptr;
    float *s32 = nullptr, *c32 = nullptr, *rhs_s32 = nullptr, *rhs_c32 = nullptr, *x_s32 = nullptr, *x_c32 = nullptr,
          *r_s32 = nullptr, *r_c32 = nullptr, *g_w32 = nullptr, *g_buf0_32 = nullptr, *g_buf1_32 = nullptr,
          *b_wt32 = nullptr;
    double *x2_s = nullptr, *x2_c = nullptr;    // 2-D: second copy of the corrections
    float *x2_s32 = nullptr, *x2_c32 = nullptr;
    int4 *tiles = nullptr;                      // 2-D: tiles of the fused sweep (rows x 64 positions)
    int ntile = 0;
    int sweeps = 0;                             // ghost relaxations per smoothing step
    size_t go_bytes = 0;                        // device bytes of the composed ghost relaxation
    int *in_ijk = nullptr;                      // packed coordinates of inside nodes, colour 0 then 1
    int nin[2] = {0, 0};
    int *go_ptr = nullptr, *go_col = nullptr;   // composed ghost relaxation (CSR over ghosts)
    double *go_a = nullptr, *go_b = nullptr;
    float *go_a32 = nullptr, *go_b32 = nullptr;
    int *gc_ptr = nullptr, *gc_idx = nullptr;   // 2-D: the folded b-part (C = B W_GI)
    int *go_sidx = nullptr;                     // 2-D: storage index of each entry's ghost
    // 2-D: the folded rows again, padded to a fixed width per level (ELL): entry k of
    // ghost q at q * we + k (b-part) and q * wf + k (C-part); padding has zero weights
    int ell_we = 0, ell_wf = 0;
    int *ell_col = nullptr, *ell_six = nullptr, *ellf_idx = nullptr;
    double *ell_a = nullptr, *ell_b = nullptr, *ellf_w = nullptr;
    float *ell_a32 = nullptr, *ell_b32 = nullptr, *ellf_w32 = nullptr;
    double *gc_w = nullptr;
    float *gc_w32 = nullptr;
    // [seg colour 0 | seg colour 1 | ghost chunks of 64 | band chunks | ghost chunks of 4 (3-D)]
    int4 *items = nullptr;
    int nseg[2] = {0, 0}, nghc = 0, nbandc = 0, nghc4 = 0;
    const int4 *w_seg(int colour) const { return items + (colour ? nseg[0] : 0); }
    const int4 *w_act() const { return items; }
    int nw_act() const { return nseg[0] + nseg[1] + nghc; }
    const int4 *w_gh() const { return items + nseg[0] + nseg[1]; }
    const int4 *w_band() const { return items + nseg[0] + nseg[1] + nghc; }
    const int4 *w_gh4() const { return items + nseg[0] + nseg[1] + nghc + nbandc; }
};

// Progress of one hierarchy's Crank-Nicolson step inside a batch advanced at
// V-cycle granularity (lsmg_batch_advance): the stopping state of the Newton
// and linear-solve loops.  It lives with the hierarchy so that a step in
// progress survives a change of batch membership.
struct RunState {
    enum Next { Idle = 0, Start, Solve, Lin } next = Idle;
    int it = 0, q = 0, cycles = 0, nrho = 0;
    bool force_update = false;
    double nF = 0.0, rprev = 0.0, rho_last = 0.0, logsum = 0.0, dwrel = 0.0;
    double t_start = 0.0;   // host clock (ms) when the step's first launch was issued
};

}  // namespace lsmg

using namespace lsmg;

struct lsmg_hierarchy {
    int dim = 2, nst = 9, nlev = 0;
    double lo = -1.0, hi = 1.0;
    lsmg_params p{};
    hipStream_t stream = nullptr;
    std::vector<lsmg::Level> L;
    std::vector<LevelDesc<double>> hd64;
    std::vector<LevelDesc<float>> hd32;
    LevelDesc<double> *d64 = nullptr;
    LevelDesc<float> *d32 = nullptr;
    bool have32 = false;
    RunState run;
    double dt = 0.0;
    bool lin_set = false;
    double *bs = nullptr, *bc = nullptr, *tmp_s = nullptr, *tmp_c = nullptr;
    double *lu = nullptr, *ainv = nullptr;
    int *piv = nullptr, *lu_status = nullptr;
    int luN = 0;
    int tail_l0 = 0;   // first level handled by the coarse-tail kernel
    // coarse tail held in LDS: table image (device), per-level layout, sizes
    uint32_t *tail_tab = nullptr;
    std::vector<TailLdsLevel> tail_ll;
    TailLdsSize tail_sz{};
    bool tail_lds = false;     // tables built (the tail's levels fit the table encoding)
    bool tail_lds_use = true;  // LSMG_TAIL_LDS=0 turns the LDS tail off
    unsigned long long *d_norms = nullptr, *h_norms = nullptr;
    TailArgs *d_tail = nullptr;      // coarse-tail arguments, entry l for a tail starting at level l
    CoarseArgs *d_coarse = nullptr;  // coarsest-operator arguments
    // the Crank-Nicolson step's arrays currently named by the level-0 descriptor
    const double *step_sn = nullptr, *step_cn = nullptr, *step_fn = nullptr, *step_fnp1 = nullptr,
                 *step_sb = nullptr;
    double step_sb_const = 0.0;
    int *h_status = nullptr;
    // Krylov solve (krylov_m > 0): m + 1 basis vectors, m preconditioned vectors, F,
    // the iterate and a work vector (compact, 2 Na each), inner-product partial sums
    // and results, and the least-squares coefficients; allocated at the first solve
    // for its m (km)
    int km = 0;
    double *kv = nullptr, *kz = nullptr, *kf = nullptr, *kx = nullptr, *kw = nullptr, *kpart = nullptr,
           *kres = nullptr, *kcoef = nullptr;
    DevMem mem;              // device memory: the caller's allocator or hipMalloc
    std::vector<void *> allocs;
    size_t alloc_bytes = 0;  // device bytes held through alloc()
    // launch timing of one kernel class on one level (HIP events on the stream)
    int prof_kernel = -1, prof_level = -1;
    std::vector<hipEvent_t> prof_pool;
    size_t prof_used = 0;
    double prof_acc_ms = 0.0;
    long long prof_acc_n = 0;
    // V-cycle graphs (0: FP64 cycle, 1: mixed-precision refinement step), captured on a private stream
    bool use_graphs = true;
    hipStream_t cap = nullptr;
    // captured cycles, index mixed + 2 fmg + 4 factor: the full-multigrid first iteration, and the first
    // cycle of a linearisation with the coarsest factorisation forked onto a side stream
    hipGraphExec_t gexec[8] = {};
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool join_pending = false;       // during capture: the next tail launch waits for ev_join
    size_t prof_pending = 0;
    // composed ghost relaxation tables (CSR over ghosts), owned separately: rebuilt with the parameters
    std::vector<void *> ghost_ops;
    ~lsmg_hierarchy()
    {
        for (int i = 0; i < 8; ++i)
            if (gexec[i]) (void)hipGraphExecDestroy(gexec[i]);
        if (side) (void)hipStreamDestroy(side);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (cap) (void)hipStreamDestroy(cap);
        for (void *p : ghost_ops) mem.put(p);
        for (hipEvent_t e : prof_pool) (void)hipEventDestroy(e);
        for (void *p : allocs) mem.put(p);
        if (h_norms) (void)hipHostFree(h_norms);
        if (h_status) (void)hipHostFree(h_status);
    }
    template <typename T>
    lsmg_status alloc(T **ptr, long long count)
    {
        *ptr = nullptr;
        if (count <= 0) count = 1;
        void *p = mem.get(sizeof(T) * (size_t)count);
        if (!p) return fail(LSMG_EOOM, "device allocation of %lld bytes failed", (long long)(sizeof(T) * count));
        allocs.push_back(p);
        alloc_bytes += sizeof(T) * (size_t)count;
        *ptr = (T *)p;
        return LSMG_OK;
    }
    template <typename T>
    lsmg_status zalloc(T **ptr, long long count)
    {
        LSMGCHK(alloc(ptr, count));
        HIPCHK(hipMemsetAsync(*ptr, 0, sizeof(T) * (size_t)(count > 0 ? count : 1), stream));
        return LSMG_OK;
    }
};

// temporaries of one call, taken from a hierarchy's or batch's device memory
// and handed back on every exit path, after their stream has been synchronised
struct DevTemps {
    const lsmg::DevMem &m;
    hipStream_t s;
    std::vector<void *> p;
    DevTemps(const lsmg::DevMem &mm, hipStream_t ss) : m(mm), s(ss) {}
    template <typename T>
    lsmg_status get(T **out, long long count)
    {
        void *q = m.get(sizeof(T) * (size_t)(count > 0 ? count : 1));
        *out = (T *)q;
        if (!q) return lsmg::fail(LSMG_EOOM, "device allocation of %lld bytes failed", (long long)(sizeof(T) * count));
        p.push_back(q);
        return LSMG_OK;
    }
    ~DevTemps()
    {
        if (p.empty()) return;
        (void)hipStreamSynchronize(s);
        for (void *q : p) m.put(q);
    }
};

struct lsmg_state {
    lsmg_hierarchy *h = nullptr;
    double *s = nullptr, *c = nullptr;
    ~lsmg_state()
    {
        if (h) {
            h->mem.put(s);
            h->mem.put(c);
        }
    }
};


namespace lsmg {

// sets dt (and the descriptor scalars that depend on it) on a hierarchy
lsmg_status set_dt(lsmg_hierarchy *H, double dt);
// fills the model and solver scalars of the host copies of the descriptors
void fill_desc_scalars(lsmg_hierarchy *H);
// FP32 copies of every level (mixed precision)
lsmg_status build_f32(lsmg_hierarchy *H);
// the coarse-tail arguments of hierarchy H for a tail starting at level l0,
// its descriptors starting at d0 in the descriptor array the launch uses
TailArgs tail_args(const lsmg_hierarchy *H, int l0, int d0);
// index tables of the coarse tail held in LDS (tail.hip); leaves tail_lds false
// where the tail's levels do not fit the tables' encoding
lsmg_status build_tail_tables(lsmg_hierarchy *H);
// whether the coarse tail of H runs in LDS in precision T
template <typename T>
bool tail_in_lds(const lsmg_hierarchy *H)
{
    return H->tail_lds && H->tail_lds_use && H->p.ghost_c_new && H->tail_sz.bytes<T>() <= kTailLdsMax;
}

}  // namespace lsmg
