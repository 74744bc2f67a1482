// Host-side launchers of the lsmg kernels (implemented in kernels.hip and
// build.hip) and the structures the C ABI layer shares with them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lsmg_dev.hpp"

namespace lsmg {

// Device memory of a hierarchy or batch: the caller's allocator where one was
// given at creation (callbacks with a context), else hipMalloc / hipFree.
// put() is called only after the stream the block was used on has been
// synchronised.
struct DevMem {
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *ctx = nullptr;
    void *get(size_t bytes) const
    {
        if (bytes == 0) bytes = 1;
        if (alloc_fn) return alloc_fn(bytes, ctx);
        void *p = nullptr;
        return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
    }
    void put(void *p) const
    {
        if (!p) return;
        if (free_fn) free_fn(p, ctx);
        else (void)hipFree(p);
    }
};

// ghost sets up to this size are relaxed by one workgroup per smoothing step
constexpr int kGhostFusedMax = 256;
// levels with at most this many active nodes run inside the coarse-tail kernel
// tiles of the fused 2-D sweep: kRbRows rows x 64 positions; the red half-sweep
// covers the tile and a one-node halo (kRbSlots nodes, one per thread)
constexpr int kRbRows = 4;
constexpr int kRbCols = 64 + 2;
constexpr int kRbSlots = (kRbRows + 2) * kRbCols;
constexpr int kRbThreads = (kRbSlots + 63) / 64 * 64;
constexpr int kRbWaves = kRbThreads / 64;
// the fused sweep recomputes the red halo and reads every node of its tiles, which
// costs bandwidth but saves a launch: it is used where a sweep's launch moves
// little data (latency-bound), i.e. active nodes x sizeof(T) up to this many bytes
constexpr long long kFusedMaxBytes = 1 << 20;
inline bool fuse_sweep(long long active_nodes, size_t value_bytes)
{
    return active_nodes * (long long)value_bytes <= kFusedMaxBytes;
}
// the coarse tail: levels of at most kTailNodes1 active nodes (one per thread of
// its workgroup), and those of up to kTailMaxNodes where the tail still fits in LDS
constexpr int kTailNodes1 = 1024;
constexpr int kTailMaxNodes = 2048;
constexpr int kMaxLevels = 16;
// the coarse tail copies its levels' node lists into LDS when they fit in this many ints
constexpr int kTailStageInts = 6144;

struct TailLevel {
    gptr<const int> in_ijk;  // packed coordinates of the inside nodes, colour 0 then colour 1
    int nin0, nin1;
    int sweeps;          // ghost relaxations per smoothing step on this level
    int soff;            // offset of the level's node lists in the tail's LDS copy:
                         // inside coordinates, ghost coordinates, composed-map row pointers
};

// coarse tail held in LDS: where a level's index tables sit in the tail's table
// image (16-bit entries, offsets in entries) and its values in the value region
// (offsets in values: s, c, x_s, x_c, rhs_s, rhs_c, r_c with na entries each,
// then r_s with na + nb + 1: the band nodes and a zero)
struct TailLdsLevel {
    int nbr;     // inside nodes: tail indices of the 2 dim axis neighbours
    int gst;     // ghosts: tail indices of the stencil nodes, bit 15 set where the node
                 // is a ghost with nonzero weight
    int bcnt;    // band nodes: number of sources
    int bsrc;    // band nodes: tail indices of the source ghosts (entry j at j * nb + b)
    int pro;     // active nodes: the 2^dim coarse corners (tail index, kSkip, kOff) and the
                 // number of odd coordinates
    int rst;     // active nodes of the next coarser level: their 3^dim fine neighbours
                 // (slot | type << 12 | ext << 14 | in-box << 15)
    int perm;    // coarsest level: tail index of compact node r
    int gop;     // composed-map row pointers (ints, copied from the level at entry)
    int v;       // first value of the level
    int na, nb, pad;
};

// one hierarchy's coarse tail (levels l0 .. nlev-1), its descriptors starting at d0
struct TailArgs {
    int d0, l0, nlev, nu1, nu2;
    int nstage;          // ints of the LDS copy of the node lists (sum over the tail's levels)
    int gamma, pad;      // cycle index (1 V, 2 W)
    gptr<const int> c2s;      // coarsest level: compact -> storage
    gptr<const double> ainv;  // coarsest level: explicit inverse (FP64, 2Na x 2Na)
    TailLevel lev[kMaxLevels];
    // coarse tail held in LDS (when the hierarchy's tail fits)
    gptr<const uint32_t> tab;   // table image
    int tab_words, nvals, nints, ngmax;
    int ncoarse;         // active nodes of the coarsest level (4 ncoarse doubles of LDS)
    int lds;             // bit 0: this tail runs in LDS in FP64 cycles, bit 1: in FP32 cycles
    TailLdsLevel ll[kMaxLevels];
};

// one hierarchy's coarsest operator: descriptor, compact -> storage map, global
// scratch (used when the matrix does not fit in LDS), inverse and status word
struct CoarseArgs {
    int desc, pad;
    const int *c2s;
    double *M, *Ainv;
    int *status;
};

// one block of a work-list concatenation
struct ItemCopy {
    const int4 *src;
    int cnt, off, dshift, pad;
};

// launch configuration of the item kernels: stream, optional per-descriptor
// active flags, work items (wavefronts) per workgroup, optional timing events
struct Exec {
    hipStream_t s = nullptr;
    const int *act = nullptr;
    int ipb = kItemsPerBlock;
    // trailing items of the list (a level's ghost chunks) that are dealt to the
    // XCDs in turn and started first; the leading items go to the XCDs in
    // contiguous chunks
    int tail = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    Exec(hipStream_t s_ = nullptr) : s(s_) {}
    Exec(hipStream_t s_, const int *a, int ipb_ = kItemsPerBlock) : s(s_), act(a), ipb(ipb_) {}
};

inline Exec with_tail(Exec x, int tail)
{
    x.tail = tail;
    return x;
}

// ---- V-cycle and Newton kernels (kernels.hip) ----
template <typename T> void launch_smooth_colour(int dim, const LevelDesc<T> *d, const int4 *w, int nw, int colour, const Exec &x);
template <typename T> void launch_ghost(int dim, const LevelDesc<T> *d, int desc, const int4 *w, int nw, const int4 *w4,
                                        int nw4, int ng, int sweeps, bool composed, const Exec &xb, const Exec &xa);
template <typename T> void launch_tail(int dim, const LevelDesc<T> *d, const TailArgs *args, int nblocks, int ncoarse_max,
                                       bool stage, const Exec &x);
// the same tail with every tail level held in LDS (tail.hip); sizes are the
// maxima over the blocks' TailArgs
struct TailLdsSize {
    int ncoarse, ngmax, nvals, nints, tab_words;
    template <typename T> size_t bytes() const
    {
        return (size_t)4 * ncoarse * sizeof(double) + (size_t)(2 * ngmax + nvals) * sizeof(T) +
               (size_t)(nints + tab_words) * sizeof(int);
    }
};
// (each block lays out its LDS from its own arguments; shm bytes cover the largest;
// blocks whose lds bit for T is clear return, and k_tail skips the blocks whose bit is set)
template <typename T> void launch_tail_lds(int dim, const LevelDesc<T> *d, const TailArgs *args, int nblocks,
                                           size_t shm, const Exec &x);
constexpr size_t kTailLdsMax = 158 * 1024;   // of the 160 KiB of a gfx950 CU
template <typename T> void launch_ghost_apply(int dim, const LevelDesc<T> *d, const int4 *w, int nw, int alt,
                                             const Exec &x);
// both colours of a 2-D sweep in one launch over tiles of rows (corrections read from
// one copy, written to the other; flip selects which), with the ghost items after
template <typename T> void launch_smooth_rb(const LevelDesc<T> *d, const int4 *tiles, int ntile, const int4 *gh,
                                           int ngh, int flip, const Exec &x);
// rhs32: when given (the FP64 defect of a mixed-precision solve), the defect rounded
// to FP32 also goes to the FP32 right-hand side, with a zero FP32 correction
template <typename T> void launch_defect(int dim, const LevelDesc<T> *d, const int4 *w, int nw, int norm_k, const Exec &x,
                                         const LevelDesc<float> *rhs32 = nullptr);
template <typename T> void launch_apply_J(int dim, const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x);
template <typename T> void launch_band(const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x);
template <typename T> void launch_restrict(int dim, const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x);
template <typename T> void launch_prolong(int dim, const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x);
template <typename T> void launch_inject(int dim, const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x);
template <typename T> void launch_zero_x(int dim, const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x);
// x = 0 in FP64, and the FP32 right-hand side and correction of a mixed-precision solve's
// first cycle (its defect from x = 0), on the items' nodes
void launch_start_mixed(int dim, const LevelDesc<double> *d, const int4 *w, int nw, const Exec &x,
                        const LevelDesc<float> *d32);
void launch_explicit_half(int dim, const LevelDesc<double> *d, const int4 *w, int nw, const Exec &x);
void launch_residual(int dim, const LevelDesc<double> *d, const int4 *w, int nw, int norm_k, const Exec &x);
void launch_newton_update(int dim, const LevelDesc<double> *d, const int4 *w, int nw, const Exec &x);
void launch_commit(int dim, const LevelDesc<double> *d, const int4 *w, int nw, const Exec &x);
void launch_to_f32(int dim, const LevelDesc<double> *d64, const LevelDesc<float> *d32, const int4 *w, int nw, int what,
                   const Exec &x);
void launch_add_f32(int dim, const LevelDesc<double> *d64, const LevelDesc<float> *d32, const int4 *w, int nw,
                    const Exec &x);
template <typename T> void launch_gather_compact(const int *c2s, int na, const T *a, const T *b, double *out, hipStream_t s);
template <typename T> void launch_scatter_compact(const int *c2s, int na, const double *v, T *a, T *b, hipStream_t s);
template <typename T> void launch_fill(T *p, long long n, T v, hipStream_t s);
void launch_zero_u64(unsigned long long *p, int n, hipStream_t s);
// vectors of the Krylov solve: inner products <w, v_i> (i < nv, v_i = vb + i N) into
// out[0..nv) through part (kKvBlocks per vector), summed in a fixed order;
// w += sign sum coef[i] v_i; y = x / a (y = 0 for a = 0); y = x - y
constexpr int kKvBlocks = 512;
void launch_kv_dots(const double *w, const double *vb, long long N, int nv, double *part, double *out, hipStream_t s);
void launch_kv_update(double *w, const double *vb, long long N, int nv, const double *coef, double sign, hipStream_t s);
void launch_kv_div(double *y, const double *x, long long N, double a, hipStream_t s);
void launch_kv_rsub(double *y, const double *x, long long N, hipStream_t s);
void launch_norm_reduce(const unsigned long long *base, long long stride, int ndom, int first, int count,
                        unsigned long long *out, hipStream_t s);
// linear-solve control of one domain of a batch whose cycles run in chunks on the
// device: tol = lin_rtol |F|, the last defect norm, whether it still solves, and
// how many norms it has recorded in the chunk
struct LinCtl {
    double tol, rprev;
    int lin, n;
};
// norm 1 reduced per domain (as launch_norm_reduce), then each solving domain's
// control: the norm stored at hist[n * ndom + dom], n counted up; a domain that
// stops clears the flags act[d0 .. d0 + nlev) of its levels (dlev[dom] = (d0, nlev)).
// Norm 1's slots are left zero
void launch_norm_ctl(unsigned long long *base, long long stride, int ndom, unsigned long long *out, LinCtl *ctl,
                     const int2 *dlev, int *act, double *hist, hipStream_t s);
void launch_copy_items(const ItemCopy *jobs, int njobs, int4 *dst, hipStream_t s);
void launch_compact_to_grid(const int64_t *c2g, int na, const double *a, const double *b, const int *c2s, double *gs,
                            double *gc, hipStream_t s);
void launch_grid_to_split(const int64_t *c2g, int na, const double *gs, const double *gc, const int *c2s, double *a,
                          double *b, hipStream_t s);
// builds the coarsest operators' Schur complements and their inverses (FP64), one
// workgroup per args entry; n_max: the largest number of coarsest active nodes
void launch_coarse_factor(int dim, const LevelDesc<double> *d, const CoarseArgs *args, int nblocks, int n_max,
                          const Exec &x);
template <typename T> void launch_coarse_apply(const LevelDesc<T> *d, int lev, int N, const int *c2s, const double *Ainv,
                                               hipStream_t s);

// ---- hierarchy build (build.hip) ----
struct BuildLevel {
    int n, Wp;
    long long rows, cs;
    double lo, h;
    const double *phi;   // level set on this level, n^dim, lexicographic
    uint8_t *type;       // split layout (out)
    uint8_t *ext;        // split layout (out)
};

void launch_inject_phi(int dim, const double *phi_f, int nf, double *phi_c, int nc, hipStream_t s);
void launch_classify(int dim, const double *phi, int n, int Wp, long long cs, uint8_t *type_split, uint8_t *flag_in,
                     uint8_t *flag_gh, int *err, hipStream_t s);
// stream compaction of a byte flag array in index order; returns the count (synchronises)
int compact_flags(const uint8_t *flags, long long N, int64_t *out, int64_t *scratch_counts, int nscratch, hipStream_t s);
long long compact_scratch_size(long long N);
void launch_c2s(int dim, const int64_t *c2g, int na, int n, int Wp, long long cs, int *c2s, int *cmap, hipStream_t s);
// inside-segment work items of a level: returns the item count per colour (synchronises)
void build_segments(int dim, const uint8_t *type_split, int n, int Wp, long long rows, long long cs, int desc,
                    int4 **out_items, int *out_count, const DevMem &mem, hipStream_t s);
// packed coordinates of the inside nodes of each colour (out: ni ints, colour 0 then 1)
int build_inside_lists(int dim, const int64_t *c2g, int ni, int n, int *out, int *count, int64_t *scratch,
                       int nscratch, const DevMem &mem, hipStream_t s);
void launch_ghost_geometry(int dim, int level, int bc, const double *phi, const uint8_t *type_split,
                           const int64_t *c2g_ghost, const int *cmap, int ni, int ng, int n, int Wp, long long cs,
                           double lo, double h, int *g_idx, int *g_ijk, int *g_st, int *g_stg, int *g_stc, double *g_w,
                           double *g_B, double *g_nrm, double *g_nrow, int *g_order, int *g_bfall, int *err,
                           hipStream_t s);
void launch_band_mark(int dim, const int64_t *c2g_cghost, int ngc, int nc, const uint8_t *ftype_split, int nf, int fWp,
                      long long fcs, uint8_t *flag_lin, hipStream_t s);
void launch_band_geometry(int dim, const double *phi, const int64_t *band_lin, int nb, const uint8_t *type_split,
                          const int *bandid_lin, int n, int Wp, long long cs, double h, int *up_s, int *up_b,
                          double *up_w, int *b_idx, hipStream_t s);
void launch_band_layer(int dim, int layer, int nb, int maxc, const int *up_s, const int *up_b, const double *up_w,
                       int *blayer, int *b_cnt, int *b_src, double *b_wt, hipStream_t s);
void launch_band_ext(int nb, const int *b_idx, const int *blayer, uint8_t *ext, hipStream_t s);
void launch_ghost_ext(int ng, const int *g_idx, uint8_t *ext, hipStream_t s);
void launch_fill_bandid(const int64_t *band_lin, int nb, int *bandid_lin, hipStream_t s);
template <typename D, typename S> void launch_convert(D *dst, const S *src, long long n, hipStream_t s);

}  // namespace lsmg
