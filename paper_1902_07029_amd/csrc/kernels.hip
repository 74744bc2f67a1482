// Hot-path kernels of the level-set multigrid V-cycle and of the Newton /
// Crank-Nicolson step (gfx950, 64-lane wavefronts).
//
// Each operation is a per-node device function ("element") applied to a work
// item and a lane.  Fine levels launch one wavefront per work item; the coarse
// tail of the hierarchy (levels small enough for one workgroup) runs as a
// single 1024-thread workgroup that walks its work lists with workgroup
// barriers between phases, so the whole lower part of a V-cycle is one launch.
//
// Every element is templated on the working precision T (double, or float for
// the mixed-precision V-cycle) and on the dimension.  Jacobian entries are never
// stored: each element evaluates the rows it needs from the linearisation point
// (s, c), so a sweep moves only s, c, the right-hand side and the correction.
#include <hip/hip_ext.h>

#include "lsmg_dev.hpp"
#include "lsmg_host.hpp"
#include "rows.hpp"

namespace lsmg {

// ---------------------------------------------------------------------------
// rows read from a level in HBM (arithmetic in rows.hpp)
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__device__ __forceinline__ InsideRow<T> inside_row(const LevelDesc<T> *D, long long idx, const long long *nb)
{
    const T sr = D->s[idx], cr = D->c[idx];
    T se[2 * DIM], ce[2 * DIM], xse[2 * DIM], xce[2 * DIM];
#pragma unroll
    for (int e = 0; e < 2 * DIM; ++e) {
        se[e] = D->s[nb[e]];
        ce[e] = D->c[nb[e]];
        xse[e] = D->x_s[nb[e]];
        xce[e] = D->x_c[nb[e]];
    }
    return inside_row_vals<T, DIM>(D, sr, cr, se, ce, xse, xce);
}

// c-row diagonal entries of a node (inside or ghost)
template <typename T>
__device__ __forceinline__ void c_row(const LevelDesc<T> *D, long long idx, T &cs_d, T &cc_d)
{
    c_row_vals<T>(D, D->s[idx], D->c[idx], cs_d, cc_d);
}

// node of (item, lane): inside node of a segment (kinds 0/1) or a ghost (kind 2)
template <typename T, int DIM>
__device__ __forceinline__ bool node_of(const LevelDesc<T> *D, int4 w, int lane, long long &idx, int &i, int &j,
                                        int &k)
{
    const int kind = item_kind(w);
    if (kind < 2) {
        // segments (2-D) and bricks (3-D) hold inside nodes only
        if (DIM == 3) return brick_lane(D->n, D->Wp, D->cs, kind, w, lane, idx, i, j, k);
        int row, p;
        if (!seg_lane(w, lane, row, p)) return false;
        node_coords<DIM>(D->n, kind, row, p, i, j, k);
        idx = sidx_at<DIM>(D->n, D->Wp, D->cs, kind, p, j, k);
    } else {
        const int q = w.z + lane;
        if (q >= w.w) return false;
        idx = D->g_idx[q];
        unpack_ijk(D->g_ijk[q], i, j, k);
    }
    return true;
}

// ---------------------------------------------------------------------------
// elements
// ---------------------------------------------------------------------------

// collective red-black Gauss-Seidel on one inside node (section 3.5.1): the 2x2
// block of eq. (matrixP) is solved for (delta s, delta c) with the neighbours
// (the other colour) fixed
template <typename T, int DIM>
__device__ __forceinline__ void smooth_node(const LevelDesc<T> *D, long long idx, int i, int j, int k, int colour)
{
    long long nb[2 * DIM];
    neighbours<DIM>(D->n, D->Wp, D->cs, colour, i, j, k, nb);
    const InsideRow<T> R = inside_row<T, DIM>(D, idx, nb);
    T xs, xc;
    block_solve<T>(R, D->rhs_s[idx], D->rhs_c[idx], xs, xc);
    D->x_s[idx] = xs;
    D->x_c[idx] = xc;
}

template <typename T, int DIM>
__device__ __forceinline__ void smooth_elem(const LevelDesc<T> *D, int4 w, int lane, int colour)
{
    long long idx;
    int i, j, k;
    if (DIM == 3) {
        if (!brick_lane(D->n, D->Wp, D->cs, colour, w, lane, idx, i, j, k)) return;
    } else {
        int row, p;
        if (!seg_lane(w, lane, row, p)) return;
        node_coords<DIM>(D->n, colour, row, p, i, j, k);
        idx = sidx_at<DIM>(D->n, D->Wp, D->cs, colour, p, j, k);
    }
    smooth_node<T, DIM>(D, idx, i, j, k, colour);
}

// ghost relaxation of eq. (RelGhost), Jacobi over the ghosts of a level with the
// ghost values of delta s double-buffered by ghost index: load, sweeps, final
template <typename T>
__device__ __forceinline__ void ghost_load_elem(const LevelDesc<T> *D, int q)
{
    D->g_buf0[q] = D->x_s[D->g_idx[q]];
}

template <typename T, int NST>
__device__ __forceinline__ void ghost_sweep_elem(const LevelDesc<T> *D, int q, gptr<T> bin, gptr<T> bout)
{
    const int ng = D->ng;
    const long long g = D->g_idx[q];
    T val[NST];
#pragma unroll
    for (int k = 0; k < NST; ++k) {
        const int gq = D->g_stg[k * ng + q];
        val[k] = gq >= 0 ? bin[gq] : D->x_s[D->g_st[k * ng + q]];
    }
    T v = 0;
#pragma unroll
    for (int k = 0; k < NST; ++k) v += D->g_w[k * ng + q] * val[k];
    bout[q] = bin[q] + D->tau_s * (D->rhs_s[g] - v);
}

template <typename T>
__device__ __forceinline__ void ghost_final_elem(const LevelDesc<T> *D, int q, gptr<T> bfin, gptr<T> bprev)
{
    const long long g = D->g_idx[q];
    const T ns = bfin[q];
    D->x_s[g] = ns;
    T cs_d, cc_d;
    c_row<T>(D, g, cs_d, cc_d);
    const T dsv = D->ghost_c_new ? ns : bprev[q];
    D->x_c[g] = ghost_c_update<T>(cs_d, cc_d, D->rhs_c[g], dsv, D->x_c[g]);
}

// composed form of the same sweeps: phase 1 stores the ghost's current delta s
// and b = rhs - (its stencil terms on non-ghost nodes); phase 2 applies the
// composed map and relaxes the c-row with the new delta s
template <typename T, int NST>
__device__ __forceinline__ void ghost_b_elem(const LevelDesc<T> *D, int q)
{
    const int ng = D->ng;
    const long long g = D->g_idx[q];
    // every stencil entry names a valid node (zero-weight entries the ghost itself), so all
    // gathers are issued unconditionally and the ghost entries are dropped afterwards
    int st[NST];
    bool gh[NST];
#pragma unroll
    for (int k = 0; k < NST; ++k) {
        st[k] = D->g_st[k * ng + q];
        gh[k] = D->g_stg[k * ng + q] >= 0;
    }
    T val[NST];
#pragma unroll
    for (int k = 0; k < NST; ++k) {
        const T xv = D->x_s[st[k]];
        val[k] = gh[k] ? T(0) : xv;
    }
    T v = 0;
#pragma unroll
    for (int k = 0; k < NST; ++k) v += D->g_w[k * ng + q] * val[k];
    D->g_buf0[q] = D->rhs_s[g] - v;
    D->g_buf1[q] = D->x_s[g];
}

template <typename T>
__device__ __forceinline__ void ghost_apply_elem(const LevelDesc<T> *D, int q)
{
    const long long g = D->g_idx[q];
    const int e0 = D->go_ptr[q], e1 = D->go_ptr[q + 1];
    T v = 0;
    // b-values from ghost_b_elem (the folded rows serve the 16-lane kernel only)
    for (int e = e0; e < e1; ++e) {
        const int c = D->go_col[e];
        v += D->go_a[e] * D->g_buf1[c] + D->go_b[e] * D->g_buf0[c];
    }
    D->x_s[g] = v;
    T cs_d, cc_d;
    c_row<T>(D, g, cs_d, cc_d);
    D->x_c[g] = ghost_c_update<T>(cs_d, cc_d, D->rhs_c[g], v, D->x_c[g]);
}

// defect r = rhs - J x on one active row pair (section 3.5.2); returns |r| bits
// (a mixed-precision cycle's FP32 right-hand side: E, when given, takes the
// defect rounded to FP32 and a zero FP32 correction at the same node; the FP64
// defect itself is then not stored, since no later kernel of a mixed-precision
// solve reads it, only its norm)
__device__ __forceinline__ void defect_to_f32(const LevelDesc<float> *E, long long idx, double rs, double rc)
{
    E->rhs_s[idx] = (float)rs;
    E->rhs_c[idx] = (float)rc;
    E->x_s[idx] = 0.0f;
    E->x_c[idx] = 0.0f;
}

template <typename T, int DIM>
__device__ __forceinline__ unsigned long long defect_inside(const LevelDesc<T> *D, long long idx, int i, int j, int k,
                                                            const LevelDesc<float> *E)
{
    long long nb[2 * DIM];
    neighbours<DIM>(D->n, D->Wp, D->cs, (i + j + k) & 1, i, j, k, nb);
    const InsideRow<T> R = inside_row<T, DIM>(D, idx, nb);
    T rs, rc;
    inside_defect_vals<T>(R, D->rhs_s[idx], D->rhs_c[idx], D->x_s[idx], D->x_c[idx], rs, rc);
    if (E) {
        defect_to_f32(E, idx, (double)rs, (double)rc);
    } else {
        D->r_s[idx] = rs;
        D->r_c[idx] = rc;
    }
    const unsigned long long a = abs_bits((double)rs), b = abs_bits((double)rc);
    return a > b ? a : b;
}

template <typename T, int NST>
__device__ __forceinline__ unsigned long long defect_ghost(const LevelDesc<T> *D, int q, const LevelDesc<float> *E)
{
    const int ng = D->ng;
    const long long idx = D->g_idx[q];
    T val[NST];
#pragma unroll
    for (int kk = 0; kk < NST; ++kk) val[kk] = D->x_s[D->g_st[kk * ng + q]];
    T v = 0;
#pragma unroll
    for (int kk = 0; kk < NST; ++kk) v += D->g_w[kk * ng + q] * val[kk];
    T cs_d, cc_d;
    c_row<T>(D, idx, cs_d, cc_d);
    const T rs = D->rhs_s[idx] - v;
    const T rc = D->rhs_c[idx] - (cs_d * D->x_s[idx] + cc_d * D->x_c[idx]);
    if (E) {
        defect_to_f32(E, idx, (double)rs, (double)rc);
    } else {
        D->r_s[idx] = rs;
        D->r_c[idx] = rc;
    }
    const unsigned long long a = abs_bits((double)rs), b = abs_bits((double)rc);
    return a > b ? a : b;
}

template <typename T, int DIM, int NST>
__device__ __forceinline__ unsigned long long defect_elem(const LevelDesc<T> *D, int4 w, int lane,
                                                          const LevelDesc<float> *E)
{
    if (item_kind(w) == 2) {
        const int q = w.z + lane;
        return q < w.w ? defect_ghost<T, NST>(D, q, E) : 0ull;
    }
    long long idx;
    int i, j, k;
    if (!node_of<T, DIM>(D, w, lane, idx, i, j, k)) return 0ull;
    return defect_inside<T, DIM>(D, idx, i, j, k, E);
}

// y = J x on one active row pair (into r)
template <typename T, int DIM, int NST>
__device__ __forceinline__ void apply_J_elem(const LevelDesc<T> *D, int4 w, int lane)
{
    long long idx;
    int i, j, k;
    if (!node_of<T, DIM>(D, w, lane, idx, i, j, k)) return;
    if (item_kind(w) < 2) {
        long long nb[2 * DIM];
        neighbours<DIM>(D->n, D->Wp, D->cs, item_kind(w), i, j, k, nb);
        const InsideRow<T> R = inside_row<T, DIM>(D, idx, nb);
        const T xs = D->x_s[idx], xc = D->x_c[idx];
        D->r_s[idx] = R.ss_d * xs + R.sc_d * xc + R.off_s;
        D->r_c[idx] = R.cs_d * xs + R.cc_d * xc;
    } else {
        const int q = w.z + lane, ng = D->ng;
        T v = 0;
#pragma unroll
        for (int kk = 0; kk < NST; ++kk) v += D->g_w[kk * ng + q] * D->x_s[D->g_st[kk * ng + q]];
        T cs_d, cc_d;
        c_row<T>(D, idx, cs_d, cc_d);
        D->r_s[idx] = v;
        D->r_c[idx] = cs_d * D->x_s[idx] + cc_d * D->x_c[idx];
    }
}

// boundary-defect band: each reached band node is a fixed linear combination
// of ghost defects (the layered upwind extension of section 3.5.2, composed at
// build time)
template <typename T>
__device__ __forceinline__ void band_elem(const LevelDesc<T> *D, int b)
{
    const int cnt = D->b_cnt[b];
    if (cnt == 0) return;
    const int nb = D->nb;
    T v = 0;
    // sources fetched eight at a time (past the count: the last source again, not
    // summed), summed in order
    for (int j0 = 0; j0 < cnt; j0 += 8) {
        int src[8];
        T wt[8], r[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int ju = min(j0 + u, cnt - 1);
            src[u] = D->b_src[ju * nb + b];
            wt[u] = D->b_wt[ju * nb + b];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) r[u] = D->r_s[src[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const T t = fma(wt[u], r[u], v);
            v = j0 + u < cnt ? t : v;
        }
    }
    D->r_s[D->b_idx[b]] = v;
}

// restriction onto one coarse node (section 3.5.2, Fig. Neigh): modified full
// weighting; inside rows read inside fine defects, boundary rows read ghost and
// reached band defects, c-rows use full weighting renormalised over active fine
// nodes.  Also clears the coarse correction.
template <typename T, int DIM, bool INSIDE>
__device__ __forceinline__ void restrict_node(const LevelDesc<T> *C, long long cidx, int ci, int cj, int ck)
{
    const LevelDesc<T> *F = C - 1;
    constexpr int NST = DIM == 2 ? 9 : 27;
    const int fn = F->n, fWp = F->Wp;
    const long long fcs = F->cs;
    const int fc0 = 2 * ci, fc1 = 2 * cj, fc2 = 2 * ck;
    const long long fcentre = sidx(DIM, fn, fWp, fcs, fc0, fc1, fc2);
    // gather the 3^d fine neighbourhood (out-of-box entries read the centre with type "excluded")
    uint8_t ex[NST], act[NST];
    T rs[NST], rc[NST];
#pragma unroll
    for (int kk = 0; kk < NST; ++kk) {
        const int id0 = fc0 + kk % 3 - 1, id1 = fc1 + (kk / 3) % 3 - 1, id2 = DIM == 3 ? fc2 + kk / 9 - 1 : 0;
        const bool inb = id0 >= 0 && id0 < fn && id1 >= 0 && id1 < fn && (DIM == 2 || (id2 >= 0 && id2 < fn));
        const long long q = inb ? sidx(DIM, fn, fWp, fcs, id0, id1, id2) : fcentre;
        const uint8_t t = F->type[q];
        // boundary rows (INSIDE false) also need the extension flag; it is combined
        // without short-circuit so that its load is issued with the type's
        const uint8_t e = INSIDE ? 0 : F->ext[q];
        rs[kk] = F->r_s[q];
        rc[kk] = F->r_c[q];
        const bool tin = t == kIn, tout = t == kOut, ext = e != 0;
        const bool excl = INSIDE ? !tin : (tin | (tout & !ext));
        ex[kk] = inb ? (uint8_t)excl : (uint8_t)1;
        act[kk] = inb & !tout;
    }
    T vs, vc;
    restrict_vals<T, DIM>(ex, act, rs, rc, vs, vc);
    C->rhs_s[cidx] = vs;
    C->rhs_c[cidx] = vc;
    C->x_s[cidx] = T(0);
    C->x_c[cidx] = T(0);
}

template <typename T, int DIM>
__device__ __forceinline__ void restrict_elem(const LevelDesc<T> *C, int4 w, int lane)
{
    long long cidx;
    int ci, cj, ck;
    if (!node_of<T, DIM>(C, w, lane, cidx, ci, cj, ck)) return;
    if (item_kind(w) < 2) restrict_node<T, DIM, true>(C, cidx, ci, cj, ck);
    else restrict_node<T, DIM, false>(C, cidx, ci, cj, ck);
}

// bilinear (trilinear) prolongation onto one fine node (section 3.5.3), over
// active coarse nodes and renormalised, added to x
template <typename T, int DIM>
__device__ __forceinline__ void prolong_node(const LevelDesc<T> *F, long long idx, int i, int j, int k)
{
    const LevelDesc<T> *C = F + 1;
    const int fi[3] = {i, j, k};
    constexpr int NC = 1 << DIM;
    // the corners of the fine node's coarse cell; on an axis where the fine
    // coordinate is even only the corners with bit 0 exist, and the others (not
    // summed) re-read that corner, so that every load is issued at once
    long long cq[NC];
    T wq[NC];
    bool use[NC];
#pragma unroll
    for (int corner = 0; corner < NC; ++corner) {
        int id[3] = {0, 0, 0};
        T wk = 1;
        bool skip = false;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int bit = (corner >> a) & 1;
            if ((fi[a] & 1) == 0) {
                skip |= bit != 0;
                id[a] = fi[a] >> 1;
            } else {
                id[a] = (fi[a] >> 1) + bit;
                wk *= T(0.5);
            }
        }
        cq[corner] = sidx(DIM, C->n, C->Wp, C->cs, id[0], id[1], id[2]);
        wq[corner] = wk;
        use[corner] = !skip;
    }
    // the corrections are read with the node type and the fine node's own
    // correction (one round trip); an inactive corner adds +0, which leaves the
    // sums unchanged (they are never -0)
    bool on[NC];
    T xs[NC], xc[NC];
#pragma unroll
    for (int corner = 0; corner < NC; ++corner) {
        on[corner] = C->type[cq[corner]] != kOut;
        xs[corner] = C->x_s[cq[corner]];
        xc[corner] = C->x_c[cq[corner]];
    }
    const T fxs = F->x_s[idx], fxc = F->x_c[idx];
    T ws = 0, es = 0, ec = 0;
#pragma unroll
    for (int corner = 0; corner < NC; ++corner) {
        const T wk = wq[corner];
        const T ws1 = ws + (on[corner] ? wk : T(0));
        const T es1 = es + (on[corner] ? wk * xs[corner] : T(0));
        const T ec1 = ec + (on[corner] ? wk * xc[corner] : T(0));
        ws = use[corner] ? ws1 : ws;
        es = use[corner] ? es1 : es;
        ec = use[corner] ? ec1 : ec;
    }
    if (ws > T(0)) {
        F->x_s[idx] = fxs + es / ws;
        F->x_c[idx] = fxc + ec / ws;
    }
}

template <typename T, int DIM>
__device__ __forceinline__ void prolong_elem(const LevelDesc<T> *F, int4 w, int lane)
{
    long long idx;
    int i, j, k;
    if (!node_of<T, DIM>(F, w, lane, idx, i, j, k)) return;
    prolong_node<T, DIM>(F, idx, i, j, k);
}

// coarse linearisation point on one coarse node: injection where the fine centre
// is active, otherwise full weighting over the active fine neighbours
template <typename T, int DIM>
__device__ __forceinline__ void inject_elem(const LevelDesc<T> *C, int4 w, int lane)
{
    const LevelDesc<T> *F = C - 1;
    long long cidx;
    int ci[3];
    if (!node_of<T, DIM>(C, w, lane, cidx, ci[0], ci[1], ci[2])) return;
    const int fn = F->n;
    const int fc[3] = {2 * ci[0], 2 * ci[1], 2 * ci[2]};
    if (item_kind(w) < 2) {
        // a coarse inside node's fine centre has the same level-set value: inside
        const long long fq = sidx(DIM, fn, F->Wp, F->cs, fc[0], fc[1], fc[2]);
        C->s[cidx] = F->s[fq];
        C->c[cidx] = F->c[fq];
        return;
    }
    constexpr int NST = DIM == 2 ? 9 : 27;
    constexpr int CEN = DIM == 2 ? 4 : 13;
    // the whole fine neighbourhood is read at once (out-of-box entries read the
    // centre and are dropped), then combined in order with selects
    uint8_t t[NST];
    T sv[NST], cv[NST];
    bool inb[NST];
#pragma unroll
    for (int kk = 0; kk < NST; ++kk) {
        const int d[3] = {kk % 3 - 1, (kk / 3) % 3 - 1, DIM == 3 ? kk / 9 - 1 : 0};
        int id[3];
        bool in = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            id[a] = fc[a] + (a < DIM ? d[a] : 0);
            if (a < DIM && (id[a] < 0 || id[a] >= fn)) in = false;
        }
        const long long q = in ? sidx(DIM, fn, F->Wp, F->cs, id[0], id[1], id[2])
                               : sidx(DIM, fn, F->Wp, F->cs, fc[0], fc[1], fc[2]);
        inb[kk] = in;
        t[kk] = F->type[q];
        sv[kk] = F->s[q];
        cv[kk] = F->c[q];
    }
    if (t[CEN] != kOut) {
        C->s[cidx] = sv[CEN];
        C->c[cidx] = cv[CEN];
        return;
    }
    T ws = 0, vs = 0, vc = 0;
#pragma unroll
    for (int kk = 0; kk < NST; ++kk) {
        const int d[3] = {kk % 3 - 1, (kk / 3) % 3 - 1, DIM == 3 ? kk / 9 - 1 : 0};
        T wk = 1;
#pragma unroll
        for (int a = 0; a < DIM; ++a) wk *= d[a] == 0 ? T(0.5) : T(0.25);
        const bool use = inb[kk] && t[kk] != kOut;
        const T ws1 = ws + wk, vs1 = vs + wk * sv[kk], vc1 = vc + wk * cv[kk];
        ws = use ? ws1 : ws;
        vs = use ? vs1 : vs;
        vc = use ? vc1 : vc;
    }
    C->s[cidx] = vs / ws;
    C->c[cidx] = vc / ws;
}

// ---------------------------------------------------------------------------
// per-item kernels (fine levels): one wavefront per work item
// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// The logical block number gives XCD x a contiguous range of work items, so the
// rows above and below an item (its y and z neighbours) are mostly processed by
// the same XCD and found in its L2.
__device__ __forceinline__ int logical_block(int tb = 0)
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
    // the last tb logical blocks are dealt to the XCDs in turn and run first on
    // each; the others form one contiguous chunk per XCD
    const int tq = tb >> 3, tr = tb & 7, tx = tq + (x < tr ? 1 : 0);
    const int lead = x * q + (x < r ? x : r) - (x * tq + (x < tr ? x : tr)) + (i - tx);
    return i < tx ? nb - tb + b : lead;   // a select: no branch ahead of the item's loads
}

// Every item kernel ends with `ntb`, the number of blocks that hold trailing
// items only (logical_block deals them to the XCDs in turn; the launcher counts
// them from Exec::tail), and `act`, per-descriptor flags (null: all active);
// the items of a descriptor whose flag is 0 are skipped.  A wavefront returns
// as a whole, so the wavefront reductions that follow never see part of one.
// The item number is made wavefront-uniform explicitly (readfirstlane of the
// wavefront index), so the item, its descriptor and the descriptor's pointers
// are read with scalar loads and every data load of a lane can be issued at once.
#define LSMG_ITEM_PROLOGUE                                                                   \
    const int it = logical_block(ntb) * (int)(blockDim.x >> 6) +                            \
                   __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));                  \
    if (it >= nwork) return;                                                                \
    const int4 w = work[it];                                                                \
    if (act && !act[item_desc(w)]) return;                                                  \
    const int lane = threadIdx.x & 63;

#define LSMG_ITEMS const int4 *__restrict__ work, int nwork
#define LSMG_ACT int ntb, const int *__restrict__ act

template <typename T, int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_smooth_colour(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS,
                                                             int colour, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<T> *D = descs + item_desc(w);
    if (item_kind(w) == 2) {
        // ghost items after the segments: snapshot the ghosts' delta s for the folded
        // ghost relaxation (ghost values do not change during the colour sweeps)
        const int q = w.z + lane;
        if (q < w.w) D->g_buf1[q] = D->x_s[D->g_idx[q]];
        return;
    }
    smooth_elem<T, DIM>(D, w, lane, colour);
}

// ---------------------------------------------------------------------------
// fused red-black sweep (2-D): one workgroup per tile of kRbRows rows x 64
// positions, both colours, reading the corrections from one copy (x) and
// writing every active node of the tile to the other (x2), flip 1 the reverse.
// The red half-sweep is computed on the tile and a one-node halo around it
// (rows y0 - 1 .. y0 + kRbRows, positions p0 - 1 .. p0 + 64) from the black
// corrections of the read copy, which no workgroup of the launch writes; the
// black half-sweep reads every red neighbour (s, c and the new correction) from
// LDS.  A halo red node is computed with the same arithmetic as in the tile that
// owns it, so a sweep gives the bits of one launch per colour.  Ghosts of the
// tile are copied to the write copy unchanged.  Blocks after the tiles take the
// ghost items (the snapshot of the ghosts' delta s for the folded ghost map).
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kRbThreads) void k_smooth_rb(const LevelDesc<T> *__restrict__ descs,
                                                          const int4 *__restrict__ tiles, int ntile,
                                                          const int4 *__restrict__ gh, int ngh, int flip, LSMG_ACT)
{
    __shared__ T ls[kRbSlots], lc[kRbSlots], lxs[kRbSlots], lxc[kRbSlots];
    const int b = logical_block();
    const int tid = threadIdx.x;
    if (b >= ntile) {
        const int it = (b - ntile) * kRbWaves + __builtin_amdgcn_readfirstlane(tid >> 6);
        if (it >= ngh) return;
        const int4 w = gh[it];
        if (act && !act[item_desc(w)]) return;
        const LevelDesc<T> *D = descs + item_desc(w);
        const gptr<T> XS = flip ? D->x2_s : D->x_s;
        const int q = w.z + (tid & (kWave - 1));
        if (q < w.w) D->g_buf1[q] = XS[D->g_idx[q]];
        return;
    }
    const int4 w = tiles[b];
    if (act && !act[item_desc(w)]) return;
    const LevelDesc<T> *D = descs + item_desc(w);
    const gptr<T> XS = flip ? D->x2_s : D->x_s, XC = flip ? D->x2_c : D->x_c;
    const gptr<T> YS = flip ? D->x_s : D->x2_s, YC = flip ? D->x_c : D->x2_c;
    const int n = D->n, Wp = D->Wp;
    const long long cs = D->cs;
    const int y0 = w.y, p0 = w.z;
    // threads below 64 kRbRows own a black node (row y0 + tid / 64, position
    // p0 + tid % 64), whose values are fetched before the red half-sweep
    const int by = y0 + (tid >> 6), bp = p0 + (tid & (kWave - 1));
    const int bi = 2 * bp + ((1 + by) & 1);
    const bool bvalid = tid < kWave * kRbRows && by < n && bi < n;
    const long long bidx = bvalid ? cs + (long long)by * Wp + bp : 0;
    const uint8_t bt = D->type[bidx];
    const T bs = D->s[bidx], bc = D->c[bidx], brs = D->rhs_s[bidx], brc = D->rhs_c[bidx];
    const T bxs = XS[bidx], bxc = XC[bidx];
    for (int t = tid; t < kRbSlots; t += kRbThreads) {
        const int rr = t / kRbCols, pc = t - rr * kRbCols;
        const int y = y0 - 1 + rr, p = p0 - 1 + pc;
        const int i = 2 * p + (y & 1);
        const bool valid = y >= 0 && y < n && p >= 0 && i < n;
        // inside nodes never lie on the box edge, so only interior slots need neighbours
        const bool interior = valid && y > 0 && y < n - 1 && i > 0 && i < n - 1;
        const long long idx = valid ? (long long)y * Wp + p : 0;
        long long nb[4];
        if (interior) {
            neighbours<2>(n, Wp, cs, 0, i, y, 0, nb);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) nb[e] = idx;
        }
        const uint8_t ty = D->type[idx];
        const T sr = D->s[idx], cr = D->c[idx], rhs_s = D->rhs_s[idx], rhs_c = D->rhs_c[idx];
        const T xs0 = XS[idx], xc0 = XC[idx];
        T se[4], ce[4], xse[4], xce[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            se[e] = D->s[nb[e]];
            ce[e] = D->c[nb[e]];
            xse[e] = XS[nb[e]];
            xce[e] = XC[nb[e]];
        }
        // solved on every slot and kept on inside nodes only: the neighbour loads
        // then never wait for the type
        const InsideRow<T> R = inside_row_vals<T, 2>(D, sr, cr, se, ce, xse, xce);
        T nxs, nxc;
        block_solve<T>(R, rhs_s, rhs_c, nxs, nxc);
        const bool in = interior && ty == kIn;
        const T xs = in ? nxs : xs0, xc = in ? nxc : xc0;
        if (valid && ty != kOut && rr >= 1 && rr <= kRbRows && pc >= 1 && pc <= kWave) {
            YS[idx] = xs;
            YC[idx] = xc;
        }
        ls[t] = sr;
        lc[t] = cr;
        lxs[t] = xs;
        lxc[t] = xc;
    }
    __syncthreads();
    if (!bvalid || bt == kOut) return;
    if (bt != kIn) {
        YS[bidx] = bxs;
        YC[bidx] = bxc;
        return;
    }
    // red neighbours x-, x+, y-, y+ (LDS slots of the row above, this row and the row below)
    const int r0 = (tid >> 6) + 1, c0 = (tid & (kWave - 1)) + 1;
    const int sl[4] = {r0 * kRbCols + ((bi - 1) >> 1) - p0 + 1, r0 * kRbCols + ((bi + 1) >> 1) - p0 + 1,
                       (r0 - 1) * kRbCols + c0, (r0 + 1) * kRbCols + c0};
    T se[4], ce[4], xse[4], xce[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        se[e] = ls[sl[e]];
        ce[e] = lc[sl[e]];
        xse[e] = lxs[sl[e]];
        xce[e] = lxc[sl[e]];
    }
    const InsideRow<T> R = inside_row_vals<T, 2>(D, bs, bc, se, ce, xse, xce);
    T xs, xc;
    block_solve<T>(R, brs, brc, xs, xc);
    YS[bidx] = xs;
    YC[bidx] = xc;
}

template <typename T>
__global__ __launch_bounds__(kMaxBlock) void k_ghost_load(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const int q = w.z + lane;
    if (q < w.w) ghost_load_elem<T>(descs + item_desc(w), q);
}

template <typename T, int NST>
__global__ __launch_bounds__(kMaxBlock) void k_ghost_sweep(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS,
                                                           int parity, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<T> *D = descs + item_desc(w);
    const int q = w.z + lane;
    if (q < w.w) ghost_sweep_elem<T, NST>(D, q, parity ? D->g_buf1 : D->g_buf0, parity ? D->g_buf0 : D->g_buf1);
}

template <typename T>
__global__ __launch_bounds__(kMaxBlock) void k_ghost_final(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS,
                                                           int parity, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<T> *D = descs + item_desc(w);
    const int q = w.z + lane;
    if (q < w.w) ghost_final_elem<T>(D, q, parity ? D->g_buf1 : D->g_buf0, parity ? D->g_buf0 : D->g_buf1);
}

template <typename T, int NST>
__global__ __launch_bounds__(kMaxBlock) void k_ghost_b(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const int q = w.z + lane;
    if (q < w.w) ghost_b_elem<T, NST>(descs + item_desc(w), q);
}

template <typename T>
__global__ __launch_bounds__(kMaxBlock) void k_ghost_apply(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const int q = w.z + lane;
    if (q < w.w) ghost_apply_elem<T>(descs + item_desc(w), q);
}

// the same with 16 lanes per row (items of 4 ghosts: one row per 16-lane group),
// for the long composed rows; FOLD: the rows carry the folded b-part (2-D).  A
// lane takes the entries e0 + sub, e0 + sub + 16, ... of its row.  The entries
// of kApplyChunk strides are fetched (indices, then values) before they are
// summed, in the same order; the first chunk of both parts and the ghost's own
// values are fetched together, so that a row of up to 16 kApplyChunk entries
// per part costs two dependent round trips after the row pointers.
constexpr int kApplyChunk = 4;

template <typename T, bool FOLD>
struct ApplyChunk {
    int col[kApplyChunk], six[kApplyChunk];
    T a[kApplyChunk], b[kApplyChunk];
    T u[kApplyChunk], r[kApplyChunk];
    // entries past the row end re-read the row's last entry and are not summed
    __device__ __forceinline__ void fetch_index(const LevelDesc<T> *D, int e, int e1)
    {
#pragma unroll
        for (int k = 0; k < kApplyChunk; ++k) {
            const int ek = min(e + 16 * k, e1 - 1);
            col[k] = D->go_col[ek];
            six[k] = FOLD ? D->go_sidx[ek] : 0;
            a[k] = D->go_a[ek];
            b[k] = D->go_b[ek];
        }
    }
    __device__ __forceinline__ void fetch_values(const LevelDesc<T> *D)
    {
#pragma unroll
        for (int k = 0; k < kApplyChunk; ++k) {
            u[k] = D->g_buf1[col[k]];
            r[k] = FOLD ? D->rhs_s[six[k]] : D->g_buf0[col[k]];
        }
    }
    __device__ __forceinline__ T sum(T v, int e, int e1) const
    {
#pragma unroll
        for (int k = 0; k < kApplyChunk; ++k) {
            const T t = v + (a[k] * u[k] + b[k] * r[k]);
            v = e + 16 * k < e1 ? t : v;
        }
        return v;
    }
};

template <typename T>
struct FoldChunk {
    int ix[kApplyChunk];
    T w[kApplyChunk], x[kApplyChunk];
    __device__ __forceinline__ void fetch_index(const LevelDesc<T> *D, int f, int f1)
    {
#pragma unroll
        for (int k = 0; k < kApplyChunk; ++k) {
            const int fk = min(f + 16 * k, f1 - 1);
            ix[k] = D->gc_idx[fk];
            w[k] = D->gc_w[fk];
        }
    }
    __device__ __forceinline__ void fetch_values(gptr<T> XS)
    {
#pragma unroll
        for (int k = 0; k < kApplyChunk; ++k) x[k] = XS[ix[k]];
    }
    __device__ __forceinline__ T sum(T v, int f, int f1) const
    {
#pragma unroll
        for (int k = 0; k < kApplyChunk; ++k) {
            const T t = v - w[k] * x[k];
            v = f + 16 * k < f1 ? t : v;
        }
        return v;
    }
};

// Sum over each row of 16 lanes by DPP row rotations (VALU moves, no LDS).
// After a rotation by 8 a lane's value depends only on its lane number mod 8, so
// the next rotation by 4 pairs it with lane l ^ 4, and so on: every lane adds
// the same pairs, in the same order, as an xor butterfly over 8, 4, 2, 1, and the
// row's first lane ends with its sum ((v0 + v8) + (v4 + v12)) + ...  Called with
// every lane active.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <typename T>
__device__ __forceinline__ T row16_sum_lane0(T v)
{
    v += dpp_mov<0x128>(v);   // row_ror:8
    v += dpp_mov<0x124>(v);   // row_ror:4
    v += dpp_mov<0x122>(v);   // row_ror:2
    v += dpp_mov<0x121>(v);   // row_ror:1
    return v;
}

template <typename T, bool FOLD>
__global__ __launch_bounds__(kMaxBlock) void k_ghost_apply_grouped(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS,
                                                                   int alt, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<T> *D = descs + item_desc(w);
    // alt: the corrections live in the second copy (after a fused 2-D sweep)
    const gptr<T> XS = alt ? D->x2_s : D->x_s, XC = alt ? D->x2_c : D->x_c;
    const int sub = lane & 15, grp = lane >> 4;
    constexpr int kStride = 16 * kApplyChunk;
    for (int q0 = w.z; q0 < w.w; q0 += 4) {
        const int q = q0 + grp;
        const bool on = q < w.w;
        T v = 0, sg = 0, cg = 0, xcg = 0, rcg = 0;
        long long g = 0;
        const int ne = FOLD ? D->ell_we >> 4 : 0, nf = FOLD ? D->ell_wf >> 4 : 0;
        if (FOLD && on && ne >= 1 && ne <= kApplyChunk && nf <= kApplyChunk) {
            // the padded rows (each part within one chunk): no row pointers to wait for;
            // lane sub takes the entries sub, sub + 16, ... of each part, in order (b-part,
            // then C-part), and the padding adds exact zeros
            const long long eb = (long long)q * D->ell_we + sub, fb = (long long)q * D->ell_wf + sub;
            {
                // one chunk per part: the row's entries and the ghost's index in one round
                // trip, then every value in a second
                int col[kApplyChunk], six[kApplyChunk], ix[kApplyChunk];
                T a[kApplyChunk], b[kApplyChunk], cw[kApplyChunk];
#pragma unroll
                for (int k = 0; k < kApplyChunk; ++k) {
                    const long long ek = eb + 16 * min(k, ne - 1), fk = fb + 16 * min(k, nf - 1);
                    col[k] = D->ell_col[ek];
                    six[k] = D->ell_six[ek];
                    a[k] = D->ell_a[ek];
                    b[k] = D->ell_b[ek];
                    ix[k] = D->ellf_idx[fk];
                    cw[k] = D->ellf_w[fk];
                }
                g = D->g_idx[q];
                sg = D->s[g];
                cg = D->c[g];
                xcg = XC[g];
                rcg = D->rhs_c[g];
                T u[kApplyChunk], r[kApplyChunk], xv[kApplyChunk];
#pragma unroll
                for (int k = 0; k < kApplyChunk; ++k) {
                    u[k] = D->g_buf1[col[k]];
                    r[k] = D->rhs_s[six[k]];
                    xv[k] = XS[ix[k]];
                }
#pragma unroll
                for (int k = 0; k < kApplyChunk; ++k) {
                    const T t = v + (a[k] * u[k] + b[k] * r[k]);
                    v = k < ne ? t : v;
                }
#pragma unroll
                for (int k = 0; k < kApplyChunk; ++k) {
                    const T t = v - cw[k] * xv[k];
                    v = k < nf ? t : v;
                }
            }
        } else if (on) {
            g = D->g_idx[q];
            int e = D->go_ptr[q] + sub, f = FOLD ? D->gc_ptr[q] + sub : 0;
            const int e1 = D->go_ptr[q + 1], f1 = FOLD ? D->gc_ptr[q + 1] : 0;
            sg = D->s[g];
            cg = D->c[g];
            xcg = XC[g];
            rcg = D->rhs_c[g];
            ApplyChunk<T, FOLD> A;
            FoldChunk<T> F;
            const bool has_e = e < e1, has_f = FOLD && f < f1;
            if (has_e) A.fetch_index(D, e, e1);
            if (has_f) F.fetch_index(D, f, f1);
            if (has_e) A.fetch_values(D);
            if (has_f) F.fetch_values(XS);
            if (has_e) {
                v = A.sum(v, e, e1);
                for (e += kStride; e < e1; e += kStride) {
                    A.fetch_index(D, e, e1);
                    A.fetch_values(D);
                    v = A.sum(v, e, e1);
                }
            }
            if (has_f) {
                v = F.sum(v, f, f1);
                for (f += kStride; f < f1; f += kStride) {
                    F.fetch_index(D, f, f1);
                    F.fetch_values(XS);
                    v = F.sum(v, f, f1);
                }
            }
        }
        v = row16_sum_lane0(v);
        if (on && sub == 0) {
            XS[g] = v;
            T cs_d, cc_d;
            c_row_vals<T>(D, sg, cg, cs_d, cc_d);
            XC[g] = ghost_c_update<T>(cs_d, cc_d, rcg, v, xcg);
        }
    }
}

// all ghost sweeps of one level in one workgroup (sweep by sweep)
template <typename T, int NST>
__global__ __launch_bounds__(1024) void k_ghost_fused(const LevelDesc<T> *__restrict__ descs, int desc, int sweeps)
{
    const LevelDesc<T> *D = descs + desc;
    const int ng = D->ng;
    for (int q = threadIdx.x; q < ng; q += blockDim.x) ghost_load_elem<T>(D, q);
    __syncthreads();
    for (int sw = 0; sw < sweeps; ++sw) {
        const gptr<T> bin = (sw & 1) ? D->g_buf1 : D->g_buf0;
        const gptr<T> bout = (sw & 1) ? D->g_buf0 : D->g_buf1;
        for (int q = threadIdx.x; q < ng; q += blockDim.x) ghost_sweep_elem<T, NST>(D, q, bin, bout);
        __syncthreads();
    }
    const gptr<T> bfin = (sweeps & 1) ? D->g_buf1 : D->g_buf0;
    const gptr<T> bprev = (sweeps & 1) ? D->g_buf0 : D->g_buf1;
    for (int q = threadIdx.x; q < ng; q += blockDim.x) ghost_final_elem<T>(D, q, bfin, bprev);
}

// defect on the items' rows; norm_k >= 0 also accumulates |r|_inf into that norm
template <typename T, int DIM, int NST>
__global__ __launch_bounds__(kMaxBlock) void k_defect(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS, int norm_k,
                                                      const LevelDesc<float> *__restrict__ rhs32, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<T> *D = descs + item_desc(w);
    const unsigned long long bits = defect_elem<T, DIM, NST>(D, w, lane, rhs32 ? rhs32 + item_desc(w) : nullptr);
    if (norm_k >= 0) norm_accumulate(D, norm_k, bits);
}

template <typename T, int DIM, int NST>
__global__ __launch_bounds__(kMaxBlock) void k_apply_J(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    apply_J_elem<T, DIM, NST>(descs + item_desc(w), w, lane);
}

template <typename T>
__global__ __launch_bounds__(kMaxBlock) void k_band(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const int b = w.z + lane;
    if (b < w.w) band_elem<T>(descs + item_desc(w), b);
}

template <typename T, int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_restrict(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    restrict_elem<T, DIM>(descs + item_desc(w), w, lane);
}

template <typename T, int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_prolong(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    prolong_elem<T, DIM>(descs + item_desc(w), w, lane);
}

template <typename T, int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_inject(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    inject_elem<T, DIM>(descs + item_desc(w), w, lane);
}

// zero correction on the items' nodes
template <typename T, int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_zero_x(const LevelDesc<T> *__restrict__ descs, LSMG_ITEMS, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<T> *D = descs + item_desc(w);
    long long idx;
    int i, j, k;
    if (!node_of<T, DIM>(D, w, lane, idx, i, j, k)) return;
    D->x_s[idx] = T(0);
    D->x_c[idx] = T(0);
}

// start of a mixed-precision linear solve on the items' nodes: the FP64 correction
// is zero, so the first defect F - J 0 is F itself; it goes to the FP32 right-hand
// side with a zero FP32 correction (the effect of the defect from x = 0, without
// reading the rows)
template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_start_mixed(const LevelDesc<double> *__restrict__ descs, LSMG_ITEMS,
                                                           const LevelDesc<float> *__restrict__ rhs32, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<double> *D = descs + item_desc(w);
    long long idx;
    int i, j, k;
    if (!node_of<double, DIM>(D, w, lane, idx, i, j, k)) return;
    D->x_s[idx] = 0.0;
    D->x_c[idx] = 0.0;
    defect_to_f32(rhs32 + item_desc(w), idx, D->rhs_s[idx], D->rhs_c[idx]);
}

// ---------------------------------------------------------------------------
// coarse tail: levels l0 .. L-1 of a V-cycle in one workgroup, walking packed
// node lists (one node per thread and pass) with barriers between phases.
// Workgroup b runs the tail of the hierarchy described by args[b].
//
// Each phase costs about the latency of its chain of dependent loads, so the
// chains are kept short: the levels' node lists and composed-map row pointers
// are copied to LDS first (STAGE), the ghost relaxation keeps its per-ghost
// values in LDS, and row entries are fetched in groups before they are summed
// in their original order (the arithmetic, and so the result, is unchanged).
// LDS: [4 ncoarse_max doubles: coarsest solve][2 x kTailMaxNodes T: ghost values]
//      [nstage ints: node lists, STAGE only]
// ---------------------------------------------------------------------------
template <typename T>
struct TailLds {
    double *coarse;
    T *gb0, *gb1;    // per ghost: b = rhs - non-ghost stencil terms, and the old delta s
    int *si;         // per level at soff: inside coordinates, ghost coordinates, map row pointers
};

// packed coordinates of node t of a level's active list: inside nodes (colour 0,
// colour 1), then ghosts
template <typename T, bool STAGE>
__device__ __forceinline__ int tail_ijk(const LevelDesc<T> *D, const TailLevel &TL, const int *si, int t)
{
    if (STAGE) return si[TL.soff + t];
    const int nin = TL.nin0 + TL.nin1;
    return t < nin ? TL.in_ijk[t] : D->g_ijk[t - nin];
}

template <typename T, bool STAGE>
__device__ __forceinline__ void tail_node(const LevelDesc<T> *D, const TailLevel &TL, const int *si, int t,
                                          long long &idx, int &i, int &j, int &k)
{
    unpack_ijk(tail_ijk<T, STAGE>(D, TL, si, t), i, j, k);
    idx = sidx(D->dim, D->n, D->Wp, D->cs, i, j, k);
}

template <typename T, bool STAGE>
__device__ __forceinline__ int tail_goptr(const LevelDesc<T> *D, const TailLevel &TL, const int *si, int q)
{
    return STAGE ? si[TL.soff + TL.nin0 + TL.nin1 + D->ng + q] : D->go_ptr[q];
}

// composed ghost relaxation, phase 1 (as ghost_b_elem, values into LDS)
template <typename T, int NST>
__device__ __forceinline__ void tail_ghost_b(const LevelDesc<T> *D, int q, long long g, T *gb0, T *gb1)
{
    const int ng = D->ng;
    T val[NST];
#pragma unroll
    for (int k = 0; k < NST; ++k) {
        const T xv = D->x_s[D->g_st[k * ng + q]];
        val[k] = D->g_stg[k * ng + q] >= 0 ? T(0) : xv;
    }
    T v = 0;
#pragma unroll
    for (int k = 0; k < NST; ++k) v += D->g_w[k * ng + q] * val[k];
    gb0[q] = D->rhs_s[g] - v;
    gb1[q] = D->x_s[g];
}

// composed ghost relaxation, phase 2 (as ghost_apply_elem, row entries [e0, e1))
template <typename T, int DIM, int NST, bool STAGE>
__device__ void wg_smooth(const LevelDesc<T> *D, const TailLevel &TL, const TailLds<T> &S)
{
    for (int colour = 0; colour < 2; ++colour) {
        const int off = colour ? TL.nin0 : 0, cnt = colour ? TL.nin1 : TL.nin0;
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
            long long idx;
            int i, j, k;
            tail_node<T, STAGE>(D, TL, S.si, off + t, idx, i, j, k);
            smooth_node<T, DIM>(D, idx, i, j, k, colour);
        }
        __syncthreads();
    }
    const int ng = D->ng, nin = TL.nin0 + TL.nin1;
    if (D->go_ptr) {
        for (int q = threadIdx.x; q < ng; q += blockDim.x) {
            long long g;
            int i, j, k;
            tail_node<T, STAGE>(D, TL, S.si, nin + q, g, i, j, k);
            tail_ghost_b<T, NST>(D, q, g, S.gb0, S.gb1);
        }
        __syncthreads();
        // the composed rows, kRowGroup lanes per row
        const int sub = threadIdx.x % kRowGroup, grp = threadIdx.x / kRowGroup, ngrp = blockDim.x / kRowGroup;
        for (int q0 = 0; q0 < ng; q0 += ngrp) {
            const int q = q0 + grp;
            const bool on = q < ng;
            long long g = 0;
            int i, j, k, e0 = 0, e1 = 0;
            if (on) {
                tail_node<T, STAGE>(D, TL, S.si, nin + q, g, i, j, k);
                e0 = tail_goptr<T, STAGE>(D, TL, S.si, q);
                e1 = tail_goptr<T, STAGE>(D, TL, S.si, q + 1);
            }
            const T v = group_ghost_row<T>(D->go_col, D->go_a, D->go_b, S.gb0, S.gb1, e0, e1, sub);
            if (on && sub == 0) {
                T cs_d, cc_d;
                c_row<T>(D, g, cs_d, cc_d);
                const T xc = D->x_c[g], rc = D->rhs_c[g];
                D->x_s[g] = v;
                D->x_c[g] = ghost_c_update<T>(cs_d, cc_d, rc, v, xc);
            }
        }
        __syncthreads();
        return;
    }
    const int sweeps = TL.sweeps;
    for (int q = threadIdx.x; q < ng; q += blockDim.x) ghost_load_elem<T>(D, q);
    __syncthreads();
    for (int sw = 0; sw < sweeps; ++sw) {
        const gptr<T> bin = (sw & 1) ? D->g_buf1 : D->g_buf0;
        const gptr<T> bout = (sw & 1) ? D->g_buf0 : D->g_buf1;
        for (int q = threadIdx.x; q < ng; q += blockDim.x) ghost_sweep_elem<T, NST>(D, q, bin, bout);
        __syncthreads();
    }
    const gptr<T> bfin = (sweeps & 1) ? D->g_buf1 : D->g_buf0;
    const gptr<T> bprev = (sweeps & 1) ? D->g_buf0 : D->g_buf1;
    for (int q = threadIdx.x; q < ng; q += blockDim.x) ghost_final_elem<T>(D, q, bfin, bprev);
    __syncthreads();
}

// x = A^{-1} rhs on the coarsest level (FP64).  The c-rows couple a node only to
// itself (J^cs and J^cc are diagonal), so A^{-1} rhs is applied through the
// Schur complement S = J^ss - J^sc diag(J^cs / J^cc) of the c-block:
//     t = r_s - J^sc (r_c / J^cc),   x_s = S^{-1} t,   x_c = (r_c - J^cs x_s) / J^cc.
// Coarse storage (from k_coarse_invert): [S^{-1} | J^sc | J^cs | J^cc], Na x Na,
// Na x Na, Na, Na doubles.  b: 4 Na doubles of LDS.
template <typename T>
__device__ void wg_coarse_apply(const LevelDesc<T> *D, gptr<const int> c2s, gptr<const double> Ainv,
                                double *b)
{
    const int na = D->na;
    const gptr<const double> Sinv = Ainv, Jsc = Ainv + (long long)na * na, cs = Ainv + 2LL * na * na, cc = cs + na;
    double *rs = b, *rc = b + na, *t = b + 2 * na, *u = b + 3 * na;
    for (int r = threadIdx.x; r < na; r += blockDim.x) {
        const long long node = c2s[r];
        const double vc = (double)D->rhs_c[node];
        rs[r] = (double)D->rhs_s[node];
        rc[r] = vc;
        u[r] = vc / cc[r];
    }
    __syncthreads();
    // rows by groups of kRowGroup lanes (a group past the last row computes row 0 and drops it)
    const int sub = threadIdx.x % kRowGroup, grp = threadIdx.x / kRowGroup, ngrp = blockDim.x / kRowGroup;
    for (int r0 = 0; r0 < na; r0 += ngrp) {
        const int r = r0 + grp;
        const double d = group_row_dot(Jsc + (long long)(r < na ? r : 0) * na, u, na, sub);
        if (r < na && sub == 0) t[r] = rs[r] - d;
    }
    __syncthreads();
    for (int r0 = 0; r0 < na; r0 += ngrp) {
        const int r = r0 + grp;
        const double v = group_row_dot(Sinv + (long long)(r < na ? r : 0) * na, t, na, sub);
        if (r < na && sub == 0) {
            const long long node = c2s[r];
            const double csr = cs[r], ccr = cc[r];
            D->x_s[node] = (T)v;
            D->x_c[node] = (T)((rc[r] - csr * v) / ccr);
        }
    }
    __syncthreads();
}

template <typename T, int DIM, int NST, bool STAGE>
__global__ __launch_bounds__(1024) void k_tail(const LevelDesc<T> *__restrict__ descs,
                                               const TailArgs *__restrict__ args, int ncoarse_max, LSMG_ACT)
{
    extern __shared__ double sb[];
    const TailArgs &A = args[blockIdx.x];
    if (act && !act[A.d0]) return;
    // tails held in LDS run in k_tail_lds
    if (A.lds & (sizeof(T) == 8 ? 1 : 2)) return;
    TailLds<T> S;
    S.coarse = sb;
    S.gb0 = reinterpret_cast<T *>(sb + 4 * ncoarse_max);
    S.gb1 = S.gb0 + kTailMaxNodes;
    S.si = reinterpret_cast<int *>(S.gb1 + kTailMaxNodes);
    const LevelDesc<T> *base = descs + A.d0;
    const int L = A.nlev;
    if (STAGE) {
        for (int l = A.l0; l < L; ++l) {
            const LevelDesc<T> *D = base + l;
            const TailLevel &TL = A.lev[l];
            const int nin = TL.nin0 + TL.nin1, ng = D->ng;
            int *dst = S.si + TL.soff;
            for (int t = threadIdx.x; t < nin; t += blockDim.x) dst[t] = TL.in_ijk[t];
            for (int t = threadIdx.x; t < ng; t += blockDim.x) dst[nin + t] = D->g_ijk[t];
            if (D->go_ptr)
                for (int t = threadIdx.x; t <= ng; t += blockDim.x) dst[nin + ng + t] = D->go_ptr[t];
        }
        __syncthreads();
    }
    // cycle(l): pre-smoothing, defect, band, restriction to l + 1 (which clears
    // the coarse correction), gamma cycles on l + 1 (the second one from the
    // first one's result; the coarsest solve is exact and runs once),
    // prolongation, post-smoothing.  Walked without recursion: `done` holds, per
    // level p, whether one child cycle of p has finished.  Every thread takes the
    // same path.
    int l = A.l0;
    unsigned done = 0u;
    bool down = true;
    while (true) {
        if (down) {
            if (l == L - 1) {
                wg_coarse_apply<T>(base + l, A.c2s, A.ainv, S.coarse);
                down = false;
                continue;
            }
            const LevelDesc<T> *D = base + l;
            const TailLevel &TL = A.lev[l];
            for (int it = 0; it < A.nu1; ++it) wg_smooth<T, DIM, NST, STAGE>(D, TL, S);
            const int nin = TL.nin0 + TL.nin1;
            for (int t = threadIdx.x; t < nin + D->ng; t += blockDim.x) {
                if (t < nin) {
                    long long idx;
                    int i, j, k;
                    tail_node<T, STAGE>(D, TL, S.si, t, idx, i, j, k);
                    (void)defect_inside<T, DIM>(D, idx, i, j, k, nullptr);
                } else {
                    (void)defect_ghost<T, NST>(D, t - nin, nullptr);
                }
            }
            __syncthreads();
            for (int b = threadIdx.x; b < D->nb; b += blockDim.x) band_elem<T>(D, b);
            __syncthreads();
            const TailLevel &TC = A.lev[l + 1];
            const LevelDesc<T> *C = D + 1;
            const int ninc = TC.nin0 + TC.nin1;
            for (int t = threadIdx.x; t < ninc + C->ng; t += blockDim.x) {
                long long idx;
                int i, j, k;
                tail_node<T, STAGE>(C, TC, S.si, t, idx, i, j, k);
                if (t < ninc) restrict_node<T, DIM, true>(C, idx, i, j, k);
                else restrict_node<T, DIM, false>(C, idx, i, j, k);
            }
            __syncthreads();
            done &= ~(1u << l);
            ++l;
            continue;
        }
        // cycle(l) has finished
        if (l == A.l0) break;
        const int p = l - 1;
        if (A.gamma == 2 && l != L - 1 && !(done & (1u << p))) {
            done |= 1u << p;
            down = true;   // the second cycle on level l
            continue;
        }
        const LevelDesc<T> *D = base + p;
        const TailLevel &TL = A.lev[p];
        const int nin = TL.nin0 + TL.nin1;
        for (int t = threadIdx.x; t < nin + D->ng; t += blockDim.x) {
            long long idx;
            int i, j, k;
            tail_node<T, STAGE>(D, TL, S.si, t, idx, i, j, k);
            prolong_node<T, DIM>(D, idx, i, j, k);
        }
        __syncthreads();
        for (int it = 0; it < A.nu2; ++it) wg_smooth<T, DIM, NST, STAGE>(D, TL, S);
        l = p;
    }
}

// ---------------------------------------------------------------------------
// finest level, FP64: explicit half of the Crank-Nicolson step (section 3.1,
// eq. discTime), the Newton residual (eqs. FDs, FDc, BCs), the Newton update
// and the commit of W^{n+1}; the step's arrays are named by the level-0
// descriptor
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ double Ls_h(const LevelDesc<double> *D, gptr<double> s, gptr<double> c, long long idx,
                                       const long long *nb)
{
    const double phg = D->alpha * c[idx] + D->beta;
    double diff = 0.0;
#pragma unroll
    for (int e = 0; e < 2 * DIM; ++e) diff += ((D->alpha * c[nb[e]] + D->beta) + phg) * (s[nb[e]] - s[idx]);
    return -(2.0 * D->ks_half) * phg * s[idx] * c[idx] + D->d_half_h2 * diff;
}

__device__ __forceinline__ double Lc_h(const LevelDesc<double> *D, gptr<double> s, gptr<double> c, long long idx)
{
    return -(2.0 * D->kc_half) * (D->alpha * c[idx] + D->beta) * s[idx] * c[idx];
}

// b = W^n / dt + L_h(W^n) / 2 (+ source average), and the first Newton iterate W = W^n
template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_explicit_half(const LevelDesc<double> *__restrict__ descs, LSMG_ITEMS,
                                                             LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<double> *D = descs + item_desc(w);
    long long idx;
    int i, j, k;
    if (!node_of<double, DIM>(D, w, lane, idx, i, j, k)) return;
    const gptr<double> sn = D->sn, cn = D->cn;
    const int r = D->cmap[idx];
    const int na = D->na;
    if (item_kind(w) < 2) {
        long long nb[2 * DIM];
        neighbours<DIM>(D->n, D->Wp, D->cs, item_kind(w), i, j, k, nb);
        double bsv = (D->alpha * cn[idx] + D->beta) * sn[idx] * D->dt_inv + 0.5 * Ls_h<DIM>(D, sn, cn, idx, nb);
        if (D->fn) bsv += 0.5 * (D->fn[r] + D->fnp1[r]);
        D->bs[idx] = bsv;
    } else {
        D->bs[idx] = 0.0;
    }
    double bcv = cn[idx] * D->dt_inv + 0.5 * Lc_h(D, sn, cn, idx);
    if (D->fn) bcv += 0.5 * (D->fn[na + r] + D->fnp1[na + r]);
    D->bc[idx] = bcv;
    D->s[idx] = sn[idx];
    D->c[idx] = cn[idx];
}

// F(W) at the linearisation point (s, c) of level 0, written to rhs_s / rhs_c;
// norm_k >= 0 also accumulates |F|_inf
template <int DIM, int NST>
__global__ __launch_bounds__(kMaxBlock) void k_residual(const LevelDesc<double> *__restrict__ descs, LSMG_ITEMS,
                                                        int norm_k, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<double> *D = descs + item_desc(w);
    long long idx;
    int i, j, k;
    unsigned long long bits = 0;
    if (node_of<double, DIM>(D, w, lane, idx, i, j, k)) {
        const gptr<double> s = D->s, c = D->c;
        double fs;
        if (item_kind(w) < 2) {
            long long nb[2 * DIM];
            neighbours<DIM>(D->n, D->Wp, D->cs, item_kind(w), i, j, k, nb);
            fs = (D->alpha * c[idx] + D->beta) * s[idx] * D->dt_inv - 0.5 * Ls_h<DIM>(D, s, c, idx, nb) - D->bs[idx];
        } else {
            const int q = w.z + lane;
            const int ng = D->ng;
            double v = 0.0;
#pragma unroll
            for (int kk = 0; kk < NST; ++kk) v += D->g_w[kk * ng + q] * s[D->g_st[kk * ng + q]];
            fs = v - (D->sb ? D->sb[q] : D->sb_const);
        }
        const double fc = c[idx] * D->dt_inv - 0.5 * Lc_h(D, s, c, idx) - D->bc[idx];
        D->rhs_s[idx] = fs;
        D->rhs_c[idx] = fc;
        const unsigned long long a = abs_bits(fs), b = abs_bits(fc);
        bits = a > b ? a : b;
    }
    if (norm_k >= 0) norm_accumulate(D, norm_k, bits);
}

// W <- W - dW on active nodes, with |dW|_inf into norm 2 and |W_old|_inf into norm 3
template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_newton_update(const LevelDesc<double> *__restrict__ descs, LSMG_ITEMS,
                                                             LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<double> *D = descs + item_desc(w);
    long long idx;
    int i, j, k;
    unsigned long long bd = 0, bw = 0;
    if (node_of<double, DIM>(D, w, lane, idx, i, j, k)) {
        const double s = D->s[idx], c = D->c[idx], xs = D->x_s[idx], xc = D->x_c[idx];
        unsigned long long a = abs_bits(xs), b = abs_bits(xc);
        bd = a > b ? a : b;
        a = abs_bits(s);
        b = abs_bits(c);
        bw = a > b ? a : b;
        D->s[idx] = s - xs;
        D->c[idx] = c - xc;
    }
    norm_accumulate(D, 2, bd);
    norm_accumulate(D, 3, bw);
}

// W^{n+1} = W on active nodes
template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_commit(const LevelDesc<double> *__restrict__ descs, LSMG_ITEMS, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<double> *D = descs + item_desc(w);
    long long idx;
    int i, j, k;
    if (!node_of<double, DIM>(D, w, lane, idx, i, j, k)) return;
    D->sn[idx] = D->s[idx];
    D->cn[idx] = D->c[idx];
}

// ---------------------------------------------------------------------------
// mixed precision: FP64 <-> FP32 transfers on a level
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_to_f32(const LevelDesc<double> *__restrict__ d64,
                                                      const LevelDesc<float> *__restrict__ d32, LSMG_ITEMS, int what,
                                                      LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<double> *D = d64 + item_desc(w);
    const LevelDesc<float> *E = d32 + item_desc(w);
    long long idx;
    int i, j, k;
    if (!node_of<double, DIM>(D, w, lane, idx, i, j, k)) return;
    if (what == 0) {            // linearisation point
        E->s[idx] = (float)D->s[idx];
        E->c[idx] = (float)D->c[idx];
    } else {                    // defect -> rhs, zero correction
        E->rhs_s[idx] = (float)D->r_s[idx];
        E->rhs_c[idx] = (float)D->r_c[idx];
        E->x_s[idx] = 0.0f;
        E->x_c[idx] = 0.0f;
    }
}

template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_add_f32(const LevelDesc<double> *__restrict__ d64,
                                                       const LevelDesc<float> *__restrict__ d32, LSMG_ITEMS, LSMG_ACT)
{
    LSMG_ITEM_PROLOGUE
    const LevelDesc<double> *D = d64 + item_desc(w);
    const LevelDesc<float> *E = d32 + item_desc(w);
    long long idx;
    int i, j, k;
    if (!node_of<double, DIM>(D, w, lane, idx, i, j, k)) return;
    D->x_s[idx] += (double)E->x_s[idx];
    D->x_c[idx] += (double)E->x_c[idx];
}

// ---------------------------------------------------------------------------
// compact <-> split layout
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_gather_compact(const int *__restrict__ c2s, int na, const T *__restrict__ a,
                                 const T *__restrict__ b, double *__restrict__ out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= na) return;
    const int q = c2s[r];
    out[r] = (double)a[q];
    out[na + r] = (double)b[q];
}

template <typename T>
__global__ void k_scatter_compact(const int *__restrict__ c2s, int na, const double *__restrict__ v,
                                  T *__restrict__ a, T *__restrict__ b)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= na) return;
    const int q = c2s[r];
    a[q] = (T)v[r];
    b[q] = (T)v[na + r];
}

template <typename T>
__global__ void k_fill(T *__restrict__ p, long long n, T v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

// grid form of a compact vector pair: NaN at inactive nodes
__global__ void k_compact_to_grid(const int64_t *__restrict__ c2g, int na, const double *__restrict__ a,
                                  const double *__restrict__ b, const int *__restrict__ c2s, double *__restrict__ gs,
                                  double *__restrict__ gc)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= na) return;
    const long long g = c2g[r];
    const int q = c2s[r];
    gs[g] = a[q];
    gc[g] = b[q];
}

__global__ void k_grid_to_split(const int64_t *__restrict__ c2g, int na, const double *__restrict__ gs,
                                const double *__restrict__ gc, const int *__restrict__ c2s, double *__restrict__ a,
                                double *__restrict__ b)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= na) return;
    const long long g = c2g[r];
    const int q = c2s[r];
    a[q] = gs[g];
    b[q] = gc[g];
}

// ---------------------------------------------------------------------------
// batches: per-domain norm reduction and work-list assembly
// ---------------------------------------------------------------------------
// out[dom * 4 + k] = max over the kNormSlots slots of norm k of domain dom, for
// k in [first, first + count); one 256-thread workgroup per domain
__global__ __launch_bounds__(kNormSlots) void k_norm_reduce(const unsigned long long *__restrict__ base,
                                                            long long stride, int first, int count,
                                                            unsigned long long *__restrict__ out)
{
    __shared__ unsigned long long part[kNormSlots / kWave];
    const int dom = blockIdx.x;
    for (int k = first; k < first + count; ++k) {
        unsigned long long v = base[k * stride + (long long)dom * kNormSlots + threadIdx.x];
        v = wave_max_u64(v);
        if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long m = 0;
            for (int i = 0; i < kNormSlots / kWave; ++i) m = part[i] > m ? part[i] : m;
            out[dom * 4 + k] = m;
        }
        __syncthreads();
    }
}

// norm 1 (a cycle's FP64 defect) reduced per domain as in k_norm_reduce, then the
// domain's linear-solve control for cycles run without a host round trip: a
// domain still solving records the norm as the next of its chunk, and stops on a
// non-finite norm or once the norm is at most its tolerance (the tests the host
// makes between cycles); a domain that stops clears the cycle flags of its levels.
// The slots are cleared after they are read, for the next cycle's defect
__global__ __launch_bounds__(kNormSlots) void k_norm_ctl(unsigned long long *__restrict__ base, long long stride,
                                                         unsigned long long *__restrict__ out, LinCtl *__restrict__ ctl,
                                                         const int2 *__restrict__ dlev, int *__restrict__ act,
                                                         double *__restrict__ hist, int ndom)
{
    __shared__ unsigned long long part[kNormSlots / kWave];
    const int dom = blockIdx.x;
    const long long slot = stride + (long long)dom * kNormSlots + threadIdx.x;
    unsigned long long v = base[slot];
    base[slot] = 0ull;
    v = wave_max_u64(v);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x != 0) return;
    unsigned long long m = 0;
    for (int i = 0; i < kNormSlots / kWave; ++i) m = part[i] > m ? part[i] : m;
    out[dom * 4 + 1] = m;
    LinCtl c = ctl[dom];
    if (!c.lin) return;
    const double rq = __longlong_as_double((long long)m);
    hist[(long long)c.n * ndom + dom] = rq;
    ++c.n;
    c.rprev = rq;
    c.lin = (isfinite(rq) && !(rq <= c.tol)) ? 1 : 0;
    ctl[dom] = c;
    if (!c.lin) {
        const int2 dl = dlev[dom];
        for (int l = 0; l < dl.y; ++l) act[dl.x + l] = 0;
    }
}

// concatenation of work lists: job b copies cnt items from src to dst + off,
// adding dshift to each item's descriptor index
__global__ void k_copy_items(const ItemCopy *__restrict__ jobs, int4 *__restrict__ dst)
{
    const ItemCopy J = jobs[blockIdx.x];
    for (int t = threadIdx.x; t < J.cnt; t += blockDim.x) {
        int4 v = J.src[t];
        v.x += J.dshift << 2;
        dst[J.off + t] = v;
    }
}

// ---------------------------------------------------------------------------
// coarsest level (FP64): the operator assembled from the same rows as the
// smoother's, reduced to the Na x Na Schur complement S = J^ss - J^sc diag(J^cs /
// J^cc) of its diagonal c-block (the exact solve needs only S^{-1}, J^sc and the
// c-row diagonals, see wg_coarse_apply), and S inverted in place by Gauss-Jordan
// elimination with partial (row) pivoting, in LDS when it fits, in one workgroup;
// the row interchanges are undone as column interchanges at the end.  Workgroup
// b works on the operator described by args[b].
// ---------------------------------------------------------------------------
constexpr int kMaxCoarseN = 1024;

template <int DIM, int NST>
__global__ __launch_bounds__(1024) void k_coarse_invert(const LevelDesc<double> *__restrict__ descs,
                                                        const CoarseArgs *__restrict__ args, int use_lds, LSMG_ACT)
{
    extern __shared__ double Mlds[];
    const CoarseArgs &CA = args[blockIdx.x];
    if (act && !act[CA.desc]) return;
    const LevelDesc<double> *D = descs + CA.desc;
    const int *__restrict__ c2s = CA.c2s;
    double *__restrict__ Ainv = CA.Ainv;
    const int na = D->na, ni = D->ni, N = na;
    double *M = use_lds ? Mlds : CA.M;      // row-major N x N: the Schur complement S
    double *Jsc = Ainv + (long long)na * na, *csv = Ainv + 2LL * na * na, *ccv = csv + na;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & (kWave - 1), wv = tid >> 6, nwv = nt >> 6;
    __shared__ double fac[kMaxCoarseN];
    __shared__ int piv[kMaxCoarseN];
    __shared__ int s_pr, s_bad;
    for (int r = wv; r < N; r += nwv)
        for (int c = lane; c < N; c += kWave) {
            M[r * N + c] = 0.0;
            Jsc[(long long)r * N + c] = 0.0;
        }
    // c-row diagonals J^cs, J^cc of every node
    for (int r = tid; r < na; r += nt) c_row<double>(D, c2s[r], csv[r], ccv[r]);
    if (tid == 0) s_bad = 0;
    __syncthreads();
    // s-rows of the Jacobian on the coarsest level (section 3.4): J^ss into S, J^sc kept
    for (int r = tid; r < na; r += nt) {
        const long long idx = c2s[r];
        double *Rs = M + r * N, *Rsc = Jsc + (long long)r * N;
        if (r < ni) {
            int i, j, k;
            sidx_node<DIM>(D->n, D->Wp, D->cs, idx, i, j, k);
            long long nb[2 * DIM];
            neighbours<DIM>(D->n, D->Wp, D->cs, (i + j + k) & 1, i, j, k, nb);
            const double sr = D->s[idx], cr = D->c[idx];
            const double al = D->alpha, be = D->beta, kap = D->kap;
            const double phr = al * cr + be;
            double sum_ss = 0.0, sum_sc = 0.0;
            for (int e = 0; e < 2 * DIM; ++e) {
                const double se = D->s[nb[e]], ce = D->c[nb[e]];
                const double a_ss = (al * ce + be) + phr, a_sc = sr - se;
                sum_ss += a_ss;
                sum_sc += a_sc;
                const int q = D->cmap[nb[e]];
                Rs[q] += -kap * a_ss;
                Rsc[q] += kap * al * a_sc;
            }
            Rs[r] += phr * D->dt_inv + D->ks_half * phr * cr + kap * sum_ss;
            Rsc[r] += al * sr * D->dt_inv + D->ks_half * (al * sr * cr + phr * sr) + kap * al * sum_sc;
        } else {
            const int q = r - ni, ng = D->ng;
            for (int kk = 0; kk < NST; ++kk) {
                const double wk = D->g_w[kk * ng + q];
                if (wk == 0.0) continue;
                Rs[D->cmap[D->g_st[kk * ng + q]]] += wk;
            }
        }
    }
    __syncthreads();
    // S = J^ss - J^sc diag(J^cs / J^cc)
    for (int r = wv; r < N; r += nwv)
        for (int c = lane; c < N; c += kWave) M[r * N + c] -= Jsc[(long long)r * N + c] * (csv[c] / ccv[c]);
    __syncthreads();
    for (int kc = 0; kc < N; ++kc) {
        // pivot: largest |M[i][kc]|, i >= kc, first index on ties (one wavefront)
        if (tid < kWave) {
            double best = -1.0;
            int bi = N;
            for (int i2 = kc + tid; i2 < N; i2 += kWave) {
                const double v = fabs(M[i2 * N + kc]);
                if (v > best) { best = v; bi = i2; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(best, off, kWave);
                const int oi = __shfl_xor(bi, off, kWave);
                if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
            }
            if (tid == 0) {
                s_pr = bi;
                piv[kc] = bi;
                if (!(best > 0.0) || bi >= N) s_bad = 1;
            }
        }
        __syncthreads();
        if (s_bad) break;
        const int pr = s_pr;
        if (pr != kc)
            for (int c = tid; c < N; c += nt) {
                const double t = M[kc * N + c];
                M[kc * N + c] = M[pr * N + c];
                M[pr * N + c] = t;
            }
        __syncthreads();
        const double inv = 1.0 / M[kc * N + kc];
        for (int i2 = tid; i2 < N; i2 += nt) fac[i2] = M[i2 * N + kc];
        __syncthreads();
        // pivot row: column kc becomes 1/pivot, the rest is scaled
        for (int c = tid; c < N; c += nt) M[kc * N + c] = (c == kc ? 1.0 : M[kc * N + c]) * inv;
        __syncthreads();
        // other rows: column kc becomes -f/pivot, the rest loses f times the pivot row
        for (int i2 = wv; i2 < N; i2 += nwv) {
            if (i2 == kc) continue;
            const double f = fac[i2];
            double *Ri = M + i2 * N;
            const double *Rk = M + kc * N;
            for (int c = lane; c < N; c += kWave) Ri[c] = (c == kc ? 0.0 : Ri[c]) - f * Rk[c];
        }
        __syncthreads();
    }
    // undo the row interchanges as column interchanges, last first
    if (!s_bad)
        for (int kc = N - 1; kc >= 0; --kc) {
            const int pr = piv[kc];
            if (pr != kc)
                for (int r = tid; r < N; r += nt) {
                    const double t = M[r * N + kc];
                    M[r * N + kc] = M[r * N + pr];
                    M[r * N + pr] = t;
                }
            __syncthreads();
        }
    for (int r = wv; r < N; r += nwv)
        for (int c = lane; c < N; c += kWave) Ainv[(long long)r * N + c] = M[r * N + c];
    if (tid == 0) *CA.status = s_bad ? 1 : 0;
}

// One DPP step of a wavefront argmax: each lane takes the (value, index, payload)
// of the lane the control names when that value is larger or equal with a smaller
// index (lanes of rows the mask leaves out compare with themselves).
template <int CTRL, int ROWS>
__device__ __forceinline__ void argmax_dpp_step(double &a, int &i, double &pay)
{
    const long long ab = __double_as_longlong(a), pb = __double_as_longlong(pay);
    const int alo = __builtin_amdgcn_update_dpp((int)ab, (int)ab, CTRL, ROWS, 0xf, false);
    const int ahi = __builtin_amdgcn_update_dpp((int)(ab >> 32), (int)(ab >> 32), CTRL, ROWS, 0xf, false);
    const int plo = __builtin_amdgcn_update_dpp((int)pb, (int)pb, CTRL, ROWS, 0xf, false);
    const int phi = __builtin_amdgcn_update_dpp((int)(pb >> 32), (int)(pb >> 32), CTRL, ROWS, 0xf, false);
    const int oi = __builtin_amdgcn_update_dpp(i, i, CTRL, ROWS, 0xf, false);
    const double oa = __longlong_as_double(((long long)ahi << 32) | (unsigned)alo);
    const double op = __longlong_as_double(((long long)phi << 32) | (unsigned)plo);
    const bool take = oa > a || (oa == a && oi < i);
    a = take ? oa : a;
    i = take ? oi : i;
    pay = take ? op : pay;
}

// Wavefront argmax of a with ties to the smaller index, payload carried along, in
// every lane: pairs within quads, half rows and rows, then the two row broadcasts
// (rows 1 and 3 take row 0 and row 2, rows 2 and 3 take lane 31), which leave the
// result in lane 63.  The combine is associative and commutative, so the result is
// the one of any other reduction order.  Called with every lane active.
__device__ __forceinline__ void wave_argmax(double &a, int &i, double &pay)
{
    argmax_dpp_step<0xB1, 0xf>(a, i, pay);    // quad_perm [1, 0, 3, 2]
    argmax_dpp_step<0x4E, 0xf>(a, i, pay);    // quad_perm [2, 3, 0, 1]
    argmax_dpp_step<0x141, 0xf>(a, i, pay);   // row_half_mirror
    argmax_dpp_step<0x140, 0xf>(a, i, pay);   // row_mirror
    argmax_dpp_step<0x142, 0xa>(a, i, pay);   // row_bcast:15
    argmax_dpp_step<0x143, 0xc>(a, i, pay);   // row_bcast:31
    const long long ab = __double_as_longlong(a), pb = __double_as_longlong(pay);
    const int alo = __builtin_amdgcn_readlane((int)ab, 63), ahi = __builtin_amdgcn_readlane((int)(ab >> 32), 63);
    const int plo = __builtin_amdgcn_readlane((int)pb, 63), phi = __builtin_amdgcn_readlane((int)(pb >> 32), 63);
    i = __builtin_amdgcn_readlane(i, 63);
    a = __longlong_as_double(((long long)ahi << 32) | (unsigned)alo);
    pay = __longlong_as_double(((long long)phi << 32) | (unsigned)plo);
}

// The same factorisation for operators of at most kSmallCoarseN unknowns, with
// one barrier per pivot instead of five: S and J^sc are assembled in LDS, and the
// elimination writes each step's matrix into the other of two LDS copies.  Every
// wavefront finds the pivot of the step by itself (the same search and tie rule,
// so all agree), and every thread computes its entries of the next copy from the
// previous one: the pivot row scaled by the reciprocal pivot, every other row less
// its factor times that row, with the interchange of the pivot row and row kc
// folded into which source row is read.  Each entry is computed by the same
// operations as in the in-place elimination above.  The interchanges are composed
// into one column permutation that is applied while the inverse is written out.
constexpr int kSmallCoarseN = 96;
constexpr int kSmallEpt = (kSmallCoarseN * kSmallCoarseN + 1023) / 1024;

// Gauss-Jordan steps of the small-operator factorisation with EPT entries of the
// matrix per thread (entry tid + u blockDim); step kc reads copy kc & 1 of the two
// in lds and writes the other.  Returns the number of steps done: N, or the step
// whose pivot was not positive (the matrix is then left as it was before it).
template <int EPT>
__device__ __forceinline__ int small_eliminate(double *lds, int N, int *piv)
{
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (kWave - 1), NN = N * N;
    int ei[EPT], ec[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = tid + u * nt;
        ei[u] = e < NN ? e / N : -1;
        ec[u] = e < NN ? e - ei[u] * N : 0;
    }
    for (int kc = 0; kc < N; ++kc) {
        double *P = lds + (kc & 1) * NN, *Q = lds + ((kc & 1) ^ 1) * NN;
        // pivot: largest |P[i][kc]|, i >= kc, first index on ties
        double best = -1.0, bval = 0.0;
        int bi = N;
        for (int i2 = kc + lane; i2 < N; i2 += kWave) {
            const double v = P[i2 * N + kc];
            if (fabs(v) > best) {
                best = fabs(v);
                bval = v;
                bi = i2;
            }
        }
        wave_argmax(best, bi, bval);
        if (!(best > 0.0) || bi >= N) return kc;
        const int pr = bi;
        if (tid == 0) piv[kc] = pr;
        const double inv = 1.0 / bval;
        // every load of the step is issued before the first new entry is stored
        double nv[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int i = ei[u] < 0 ? 0 : ei[u], c = ec[u];
            const int src = i == pr ? kc : i;
            const double prc = P[pr * N + c], f = P[src * N + kc], a = P[src * N + c];
            const double pk = (c == kc ? 1.0 : prc) * inv;
            nv[u] = i == kc ? pk : (c == kc ? 0.0 : a) - f * pk;
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u)
            if (ei[u] >= 0) Q[ei[u] * N + ec[u]] = nv[u];
        __syncthreads();
    }
    return N;
}

template <int DIM, int NST>
__global__ __launch_bounds__(1024) void k_coarse_invert_small(const LevelDesc<double> *__restrict__ descs,
                                                              const CoarseArgs *__restrict__ args, LSMG_ACT)
{
    extern __shared__ double lds[];
    __shared__ double csl[kSmallCoarseN], ccl[kSmallCoarseN];
    __shared__ int piv[kSmallCoarseN], col[kSmallCoarseN];
    const CoarseArgs &CA = args[blockIdx.x];
    if (act && !act[CA.desc]) return;
    const LevelDesc<double> *D = descs + CA.desc;
    const int *__restrict__ c2s = CA.c2s;
    double *__restrict__ Ainv = CA.Ainv;
    const int na = D->na, ni = D->ni, N = na, NN = na * na;
    double *Jsc = Ainv + (long long)NN, *csv = Ainv + 2LL * NN, *ccv = csv + na;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (kWave - 1);
    double *P = lds, *Q = lds + NN;   // S in P, J^sc in Q; then the elimination's two copies
    for (int e = tid; e < 2 * NN; e += nt) lds[e] = 0.0;
    if (tid < na) {
        double a, b;
        c_row<double>(D, c2s[tid], a, b);
        csv[tid] = a;
        ccv[tid] = b;
        csl[tid] = a;
        ccl[tid] = b;
    }
    __syncthreads();
    // s-rows (section 3.4): every value of a row is loaded before its entries are added
    if (tid < ni) {
        const int r = tid;
        const long long idx = c2s[r];
        int i, j, k;
        sidx_node<DIM>(D->n, D->Wp, D->cs, idx, i, j, k);
        long long nb[2 * DIM];
        neighbours<DIM>(D->n, D->Wp, D->cs, (i + j + k) & 1, i, j, k, nb);
        double se[2 * DIM], ce[2 * DIM];
        int q[2 * DIM];
#pragma unroll
        for (int e = 0; e < 2 * DIM; ++e) {
            se[e] = D->s[nb[e]];
            ce[e] = D->c[nb[e]];
            q[e] = D->cmap[nb[e]];
        }
        const double sr = D->s[idx], cr = D->c[idx];
        const double al = D->alpha, be = D->beta, kap = D->kap;
        const double phr = al * cr + be;
        double *Rs = P + r * N, *Rsc = Q + r * N;
        double sum_ss = 0.0, sum_sc = 0.0;
#pragma unroll
        for (int e = 0; e < 2 * DIM; ++e) {
            const double a_ss = (al * ce[e] + be) + phr, a_sc = sr - se[e];
            sum_ss += a_ss;
            sum_sc += a_sc;
            Rs[q[e]] += -kap * a_ss;
            Rsc[q[e]] += kap * al * a_sc;
        }
        Rs[r] += phr * D->dt_inv + D->ks_half * phr * cr + kap * sum_ss;
        Rsc[r] += al * sr * D->dt_inv + D->ks_half * (al * sr * cr + phr * sr) + kap * al * sum_sc;
    } else if (tid < na) {
        const int r = tid, g = r - ni, ng = D->ng;
        double w[NST];
        int cm[NST];
#pragma unroll
        for (int kk = 0; kk < NST; ++kk) {
            w[kk] = D->g_w[kk * ng + g];
            cm[kk] = D->cmap[D->g_st[kk * ng + g]];
        }
        double *Rs = P + r * N;
#pragma unroll
        for (int kk = 0; kk < NST; ++kk)
            if (w[kk] != 0.0) Rs[cm[kk]] += w[kk];
    }
    __syncthreads();
    // S = J^ss - J^sc diag(J^cs / J^cc); J^sc goes out
    for (int e = tid; e < NN; e += nt) {
        const int c = e % N;
        P[e] -= Q[e] * (csl[c] / ccl[c]);
        Jsc[e] = Q[e];
    }
    __syncthreads();
    // entries per thread: a compile-time count, so that every load of a step is in flight at once
    int steps;
    switch ((NN + nt - 1) / nt) {
    case 1: steps = small_eliminate<1>(lds, N, piv); break;
    case 2: steps = small_eliminate<2>(lds, N, piv); break;
    case 3: steps = small_eliminate<3>(lds, N, piv); break;
    case 4: steps = small_eliminate<4>(lds, N, piv); break;
    case 5: steps = small_eliminate<5>(lds, N, piv); break;
    case 6: steps = small_eliminate<6>(lds, N, piv); break;
    case 7: steps = small_eliminate<7>(lds, N, piv); break;
    case 8: steps = small_eliminate<8>(lds, N, piv); break;
    default: steps = small_eliminate<kSmallEpt>(lds, N, piv); break;
    }
    const bool bad = steps < N;
    P = lds + (steps & 1) * NN;
    // the row interchanges, undone as column interchanges last first, as one permutation
    if (tid == 0) {
        for (int c = 0; c < N; ++c) col[c] = c;
        if (!bad)
            for (int kc = N - 1; kc >= 0; --kc) {
                const int pr = piv[kc], t = col[kc];
                col[kc] = col[pr];
                col[pr] = t;
            }
    }
    __syncthreads();
    for (int e = tid; e < NN; e += nt) {
        const int r = e / N, c = e - r * N;
        Ainv[e] = P[r * N + col[c]];
    }
    if (tid == 0) *CA.status = bad ? 1 : 0;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_coarse_apply(const LevelDesc<T> *__restrict__ descs, int lev,
                                                       const int *__restrict__ c2s, const double *__restrict__ Ainv)
{
    extern __shared__ double b[];
    wg_coarse_apply<T>(descs + lev, gptr<const int>{c2s}, gptr<const double>{Ainv}, b);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned grid_of(int nwork, int ipb) { return (unsigned)((nwork + ipb - 1) / ipb); }

// one wavefront per item, x.ipb items per workgroup, `act` appended; with a
// pair of events the launch is timed by its own dispatch
template <auto KERN, typename... Args>
static void item_launch(int nw, const Exec &x, Args... args)
{
    const int ipb = x.ipb >= 1 && x.ipb <= kMaxItemsPerBlock ? x.ipb : kItemsPerBlock;
    const dim3 g(grid_of(nw, ipb)), b(kWave * ipb);
    // blocks that hold trailing items only (see logical_block)
    const int tail = x.tail < 0 ? 0 : (x.tail > nw ? nw : x.tail);
    const int tb = (int)g.x - (int)grid_of(nw - tail, ipb);
    if (x.ev0) hipExtLaunchKernelGGL(KERN, g, b, 0, x.s, x.ev0, x.ev1, 0, args..., tb, x.act);
    else KERN<<<g, b, 0, x.s>>>(args..., tb, x.act);
}

#define LSMG_DISPATCH_DIM(dim, ...) \
    do { if ((dim) == 2) { constexpr int DIM = 2; constexpr int NST = 9; __VA_ARGS__; } \
         else { constexpr int DIM = 3; constexpr int NST = 27; __VA_ARGS__; } } while (0)

template <typename T>
void launch_smooth_colour(int dim, const LevelDesc<T> *d, const int4 *w, int nw, int colour, const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; item_launch<k_smooth_colour<T, DIM>>(nw, x, d, w, nw, colour));
}

// one fused 2-D sweep over the tiles, then the ghost items (kRbWaves per block)
template <typename T>
void launch_smooth_rb(const LevelDesc<T> *d, const int4 *tiles, int ntile, const int4 *gh, int ngh, int flip,
                      const Exec &x)
{
    if (ntile <= 0 && ngh <= 0) return;
    const dim3 g(ntile + (ngh + kRbWaves - 1) / kRbWaves), b(kRbThreads);
    if (x.ev0) hipExtLaunchKernelGGL(k_smooth_rb<T>, g, b, 0, x.s, x.ev0, x.ev1, 0, d, tiles, ntile, gh, ngh, flip, 0, x.act);
    else k_smooth_rb<T><<<g, b, 0, x.s>>>(d, tiles, ntile, gh, ngh, flip, 0, x.act);
}

// the ghost relaxation of one smoothing step: the composed map (two launches,
// xb and xa; in 3-D the map is applied over w4, items of 4 ghosts), or the sweeps
// one by one (timed as a whole with xb's events)
template <typename T>
void launch_ghost(int dim, const LevelDesc<T> *d, int desc, const int4 *w, int nw, const int4 *w4, int nw4, int ng,
                  int sweeps, bool composed, const Exec &xb, const Exec &xa)
{
    if (nw <= 0) return;
    if (composed) {
        LSMG_DISPATCH_DIM(dim, (void)DIM; item_launch<k_ghost_b<T, NST>>(nw, xb, d, w, nw));
        if (dim == 3) item_launch<k_ghost_apply_grouped<T, false>>(nw4, xa, d, w4, nw4, 0);
        else item_launch<k_ghost_apply<T>>(nw, xa, d, w, nw);
        return;
    }
    Exec x = xb;
    const hipEvent_t e0 = x.ev0, e1 = x.ev1;
    x.ev0 = x.ev1 = nullptr;
    if (e0) (void)hipEventRecord(e0, x.s);
    if (ng <= kGhostFusedMax) {
        LSMG_DISPATCH_DIM(dim, (void)DIM; k_ghost_fused<T, NST><<<1, 1024, 0, x.s>>>(d, desc, sweeps));
    } else {
        item_launch<k_ghost_load<T>>(nw, x, d, w, nw);
        for (int sw = 0; sw < sweeps; ++sw)
            LSMG_DISPATCH_DIM(dim, (void)DIM; item_launch<k_ghost_sweep<T, NST>>(nw, x, d, w, nw, sw & 1));
        item_launch<k_ghost_final<T>>(nw, x, d, w, nw, sweeps & 1);
    }
    if (e1) (void)hipEventRecord(e1, x.s);
}

// the folded composed ghost map alone (2-D), 16 lanes per row over items of 4
// ghosts, on the corrections' first copy (alt 0) or second (alt 1)
template <typename T>
void launch_ghost_apply(int dim, const LevelDesc<T> *d, const int4 *w4, int nw4, int alt, const Exec &x)
{
    (void)dim;
    if (nw4 <= 0) return;
    item_launch<k_ghost_apply_grouped<T, true>>(nw4, x, d, w4, nw4, alt);
}

template <typename T>
void launch_defect(int dim, const LevelDesc<T> *d, const int4 *w, int nw, int norm_k, const Exec &x,
                   const LevelDesc<float> *rhs32)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, item_launch<k_defect<T, DIM, NST>>(nw, x, d, w, nw, norm_k, rhs32));
}

template <typename T>
void launch_apply_J(int dim, const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, item_launch<k_apply_J<T, DIM, NST>>(nw, x, d, w, nw));
}

template <typename T>
void launch_band(const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x)
{
    if (nw <= 0) return;
    item_launch<k_band<T>>(nw, x, d, w, nw);
}

template <typename T>
void launch_restrict(int dim, const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; item_launch<k_restrict<T, DIM>>(nw, x, d, w, nw));
}

template <typename T>
void launch_prolong(int dim, const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; item_launch<k_prolong<T, DIM>>(nw, x, d, w, nw));
}

template <typename T>
void launch_inject(int dim, const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; item_launch<k_inject<T, DIM>>(nw, x, d, w, nw));
}

template <typename T>
void launch_zero_x(int dim, const LevelDesc<T> *d, const int4 *w, int nw, const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; item_launch<k_zero_x<T, DIM>>(nw, x, d, w, nw));
}

void launch_start_mixed(int dim, const LevelDesc<double> *d, const int4 *w, int nw, const Exec &x,
                        const LevelDesc<float> *d32)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; item_launch<k_start_mixed<DIM>>(nw, x, d, w, nw, d32));
}

template <typename T>
void launch_tail(int dim, const LevelDesc<T> *d, const TailArgs *args, int nblocks, int ncoarse_max, bool stage,
                 const Exec &x)
{
    if (nblocks <= 0) return;
    const size_t shm = (size_t)4 * ncoarse_max * sizeof(double) + 2 * kTailMaxNodes * sizeof(T) +
                       (stage ? kTailStageInts * sizeof(int) : 0);
    // above 64 KiB of dynamic LDS the kernel has to be allowed it
    static bool attr[2][2] = {{false, false}, {false, false}};
    bool &done = attr[dim == 3][stage];
    if (!done) {
        if (stage)
            LSMG_DISPATCH_DIM(dim, (void)hipFuncSetAttribute((const void *)k_tail<T, DIM, NST, true>,
                                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTailLdsMax));
        else
            LSMG_DISPATCH_DIM(dim, (void)hipFuncSetAttribute((const void *)k_tail<T, DIM, NST, false>,
                                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTailLdsMax));
        done = true;
    }
    if (stage)
        LSMG_DISPATCH_DIM(dim, k_tail<T, DIM, NST, true><<<nblocks, 1024, shm, x.s>>>(d, args, ncoarse_max, 0, x.act));
    else
        LSMG_DISPATCH_DIM(dim, k_tail<T, DIM, NST, false><<<nblocks, 1024, shm, x.s>>>(d, args, ncoarse_max, 0, x.act));
}

void launch_explicit_half(int dim, const LevelDesc<double> *d, const int4 *w, int nw, const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; item_launch<k_explicit_half<DIM>>(nw, x, d, w, nw));
}

void launch_residual(int dim, const LevelDesc<double> *d, const int4 *w, int nw, int norm_k, const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, item_launch<k_residual<DIM, NST>>(nw, x, d, w, nw, norm_k));
}

void launch_newton_update(int dim, const LevelDesc<double> *d, const int4 *w, int nw, const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; item_launch<k_newton_update<DIM>>(nw, x, d, w, nw));
}

void launch_commit(int dim, const LevelDesc<double> *d, const int4 *w, int nw, const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; item_launch<k_commit<DIM>>(nw, x, d, w, nw));
}

void launch_to_f32(int dim, const LevelDesc<double> *d64, const LevelDesc<float> *d32, const int4 *w, int nw,
                   int what, const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; item_launch<k_to_f32<DIM>>(nw, x, d64, d32, w, nw, what));
}

void launch_add_f32(int dim, const LevelDesc<double> *d64, const LevelDesc<float> *d32, const int4 *w, int nw,
                    const Exec &x)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; item_launch<k_add_f32<DIM>>(nw, x, d64, d32, w, nw));
}

template <typename T>
void launch_gather_compact(const int *c2s, int na, const T *a, const T *b, double *out, hipStream_t s)
{
    if (na <= 0) return;
    k_gather_compact<T><<<(na + 255) / 256, 256, 0, s>>>(c2s, na, a, b, out);
}

template <typename T>
void launch_scatter_compact(const int *c2s, int na, const double *v, T *a, T *b, hipStream_t s)
{
    if (na <= 0) return;
    k_scatter_compact<T><<<(na + 255) / 256, 256, 0, s>>>(c2s, na, v, a, b);
}

template <typename T>
void launch_fill(T *p, long long n, T v, hipStream_t s)
{
    if (n <= 0) return;
    k_fill<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
}

void launch_zero_u64(unsigned long long *p, int n, hipStream_t s) { k_zero_u64<<<1, 256, 0, s>>>(p, n); }

// ---------------------------------------------------------------------------
// vectors of the Krylov solve (compact level-0 vectors of N values).  Inner
// products are summed in a fixed order, so that a result does not depend on
// timing: block b sums, for each thread, the elements b * kKvThreads + t +
// k * kKvBlocks * kKvThreads in order of k, then the block's threads by a fixed
// tree; a second kernel sums the blocks' partial sums the same way.
// ---------------------------------------------------------------------------
constexpr int kKvThreads = 256;

__device__ __forceinline__ double block_tree_sum(double *sh, double t)
{
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int st = kKvThreads / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// part[i * kKvBlocks + b] = block b's share of <w, v_i>, v_i = vb + i N, i < nv
__global__ __launch_bounds__(kKvThreads) void k_kv_dots(const double *__restrict__ w, const double *__restrict__ vb,
                                                        long long N, int nv, double *__restrict__ part)
{
    __shared__ double sh[kKvThreads];
    const long long stride = (long long)kKvBlocks * kKvThreads;
    for (int i = 0; i < nv; ++i) {
        const double *v = vb + (long long)i * N;
        double t = 0.0;
        for (long long q = (long long)blockIdx.x * kKvThreads + threadIdx.x; q < N; q += stride)
            t = fma(w[q], v[q], t);
        const double r = block_tree_sum(sh, t);
        if (threadIdx.x == 0) part[(long long)i * kKvBlocks + blockIdx.x] = r;
    }
}

// out[i] = sum of the kKvBlocks partial sums of vector i (block i)
__global__ __launch_bounds__(kKvThreads) void k_kv_final(const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double sh[kKvThreads];
    double t = 0.0;
    for (int b = threadIdx.x; b < kKvBlocks; b += kKvThreads) t += part[(long long)blockIdx.x * kKvBlocks + b];
    const double r = block_tree_sum(sh, t);
    if (threadIdx.x == 0) out[blockIdx.x] = r;
}

// w += sign sum_{i < nv} coef[i] v_i, the terms taken in order of i
__global__ void k_kv_update(double *__restrict__ w, const double *__restrict__ vb, long long N, int nv,
                            const double *__restrict__ coef, double sign)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    double t = w[q];
    for (int i = 0; i < nv; ++i) t += sign * (coef[i] * vb[(long long)i * N + q]);
    w[q] = t;
}

// y = x / a (a != 0), or y = 0 (a == 0, x not read)
__global__ void k_kv_div(double *__restrict__ y, const double *__restrict__ x, long long N, double a)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    y[q] = a != 0.0 ? x[q] / a : 0.0;
}

// y = x - y
__global__ void k_kv_rsub(double *__restrict__ y, const double *__restrict__ x, long long N)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    y[q] = x[q] - y[q];
}

void launch_kv_dots(const double *w, const double *vb, long long N, int nv, double *part, double *out, hipStream_t s)
{
    if (nv <= 0) return;
    k_kv_dots<<<kKvBlocks, kKvThreads, 0, s>>>(w, vb, N, nv, part);
    k_kv_final<<<nv, kKvThreads, 0, s>>>(part, out);
}

void launch_kv_update(double *w, const double *vb, long long N, int nv, const double *coef, double sign, hipStream_t s)
{
    if (N <= 0 || nv <= 0) return;
    k_kv_update<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(w, vb, N, nv, coef, sign);
}

void launch_kv_div(double *y, const double *x, long long N, double a, hipStream_t s)
{
    if (N <= 0) return;
    k_kv_div<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(y, x, N, a);
}

void launch_kv_rsub(double *y, const double *x, long long N, hipStream_t s)
{
    if (N <= 0) return;
    k_kv_rsub<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(y, x, N);
}

void launch_norm_reduce(const unsigned long long *base, long long stride, int ndom, int first, int count,
                        unsigned long long *out, hipStream_t s)
{
    if (ndom <= 0) return;
    k_norm_reduce<<<ndom, kNormSlots, 0, s>>>(base, stride, first, count, out);
}

void launch_norm_ctl(unsigned long long *base, long long stride, int ndom, unsigned long long *out, LinCtl *ctl,
                     const int2 *dlev, int *act, double *hist, hipStream_t s)
{
    if (ndom <= 0) return;
    k_norm_ctl<<<ndom, kNormSlots, 0, s>>>(base, stride, out, ctl, dlev, act, hist, ndom);
}

void launch_copy_items(const ItemCopy *jobs, int njobs, int4 *dst, hipStream_t s)
{
    if (njobs <= 0) return;
    k_copy_items<<<njobs, 256, 0, s>>>(jobs, dst);
}

void launch_compact_to_grid(const int64_t *c2g, int na, const double *a, const double *b, const int *c2s,
                            double *gs, double *gc, hipStream_t s)
{
    if (na <= 0) return;
    k_compact_to_grid<<<(na + 255) / 256, 256, 0, s>>>(c2g, na, a, b, c2s, gs, gc);
}

void launch_grid_to_split(const int64_t *c2g, int na, const double *gs, const double *gc, const int *c2s, double *a,
                          double *b, hipStream_t s)
{
    if (na <= 0) return;
    k_grid_to_split<<<(na + 255) / 256, 256, 0, s>>>(c2g, na, gs, gc, c2s, a, b);
}

// dynamic LDS for the coarsest matrix: 147 KiB of the 160 KiB of a gfx950 CU
// (the kernels' own shared arrays take at most 12 KiB); operators of at most
// kSmallCoarseN unknowns take the one-barrier-per-pivot kernel with two copies
constexpr size_t kCoarseLdsMax = 147 * 1024;
static_assert(2 * kSmallCoarseN * kSmallCoarseN * sizeof(double) <= kCoarseLdsMax, "two copies of S fit");

void launch_coarse_factor(int dim, const LevelDesc<double> *d, const CoarseArgs *args, int nblocks, int n_max,
                          const Exec &x)
{
    if (nblocks <= 0) return;
    if (n_max <= kSmallCoarseN) {
        const size_t two = (size_t)2 * n_max * n_max * sizeof(double);
        LSMG_DISPATCH_DIM(dim, {
            static bool attr_set = false;
            if (two > 64 * 1024 && !attr_set) {
                (void)hipFuncSetAttribute((const void *)k_coarse_invert_small<DIM, NST>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCoarseLdsMax);
                attr_set = true;
            }
            k_coarse_invert_small<DIM, NST><<<nblocks, 1024, two, x.s>>>(d, args, 0, x.act);
        });
        return;
    }
    const size_t bytes = (size_t)n_max * n_max * sizeof(double);
    const int use_lds = bytes <= kCoarseLdsMax;
    LSMG_DISPATCH_DIM(dim, {
        static bool attr_set = false;
        if (use_lds && bytes > 64 * 1024 && !attr_set) {
            (void)hipFuncSetAttribute((const void *)k_coarse_invert<DIM, NST>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCoarseLdsMax);
            attr_set = true;
        }
        k_coarse_invert<DIM, NST><<<nblocks, 1024, use_lds ? bytes : 0, x.s>>>(d, args, use_lds, 0, x.act);
    });
}

template <typename T>
void launch_coarse_apply(const LevelDesc<T> *d, int lev, int N, const int *c2s, const double *Ainv, hipStream_t s)
{
    k_coarse_apply<T><<<1, 1024, (size_t)4 * N * sizeof(double), s>>>(d, lev, c2s, Ainv);
}

#define LSMG_INST(T) \
    template void launch_smooth_colour<T>(int, const LevelDesc<T> *, const int4 *, int, int, const Exec &); \
    template void launch_ghost<T>(int, const LevelDesc<T> *, int, const int4 *, int, const int4 *, int, int, int, bool, \
                                  const Exec &, const Exec &); \
    template void launch_defect<T>(int, const LevelDesc<T> *, const int4 *, int, int, const Exec &,              \
                                   const LevelDesc<float> *);                                                   \
    template void launch_ghost_apply<T>(int, const LevelDesc<T> *, const int4 *, int, int, const Exec &); \
    template void launch_smooth_rb<T>(const LevelDesc<T> *, const int4 *, int, const int4 *, int, int, const Exec &); \
    template void launch_apply_J<T>(int, const LevelDesc<T> *, const int4 *, int, const Exec &); \
    template void launch_band<T>(const LevelDesc<T> *, const int4 *, int, const Exec &); \
    template void launch_restrict<T>(int, const LevelDesc<T> *, const int4 *, int, const Exec &); \
    template void launch_prolong<T>(int, const LevelDesc<T> *, const int4 *, int, const Exec &); \
    template void launch_inject<T>(int, const LevelDesc<T> *, const int4 *, int, const Exec &); \
    template void launch_zero_x<T>(int, const LevelDesc<T> *, const int4 *, int, const Exec &); \
    template void launch_tail<T>(int, const LevelDesc<T> *, const TailArgs *, int, int, bool, const Exec &); \
    template void launch_gather_compact<T>(const int *, int, const T *, const T *, double *, hipStream_t); \
    template void launch_scatter_compact<T>(const int *, int, const double *, T *, T *, hipStream_t); \
    template void launch_fill<T>(T *, long long, T, hipStream_t); \
    template void launch_coarse_apply<T>(const LevelDesc<T> *, int, int, const int *, const double *, hipStream_t);
LSMG_INST(double)
LSMG_INST(float)
template void launch_fill<int>(int *, long long, int, hipStream_t);
template void launch_fill<uint8_t>(uint8_t *, long long, uint8_t, hipStream_t);
template void launch_fill<unsigned long long>(unsigned long long *, long long, unsigned long long, hipStream_t);

}  // namespace lsmg
