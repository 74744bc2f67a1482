// Hot-path kernels of the level-set multigrid V-cycle and of the Newton /
// Crank-Nicolson step (gfx950, 64-lane wavefronts, one work item per wavefront).
//
// Every kernel is templated on the working precision T (double, or float for the
// mixed-precision V-cycle) and on the dimension.  Jacobian entries are never
// stored: each kernel evaluates the rows it needs from the linearisation point
// (s, c) held in registers, so a sweep moves only s, c, the right-hand side and
// the correction.
#include "lsmg_dev.hpp"
#include "lsmg_host.hpp"

namespace lsmg {

// ---------------------------------------------------------------------------
// inside-row Jacobian (section 3.4, exact derivatives of eqs. FDs and FDc;
// the printed forms of eqs. JssI, JscI, JcsI, JccI are garbled)
// ---------------------------------------------------------------------------
template <typename T, int DIM>
struct InsideRow {
    T ss_d, sc_d, cs_d, cc_d;   // diagonal 2x2 block P (eq. matrixP)
    T off_s;                    // sum over neighbours of J^ss x_s + J^sc x_c
};

template <typename T, int DIM>
__device__ __forceinline__ InsideRow<T, DIM> inside_row(const LevelDesc<T> *D, long long idx, const long long *nb,
                                                        const T *xs, const T *xc)
{
    const T sr = D->s[idx], cr = D->c[idx];
    const T al = D->alpha, be = D->beta, kap = D->kap;
    const T phr = al * cr + be;
    T sum_ss = 0, sum_sc = 0, off = 0;
#pragma unroll
    for (int e = 0; e < 2 * DIM; ++e) {
        const T se = D->s[nb[e]], ce = D->c[nb[e]];
        const T a_ss = (al * ce + be) + phr;
        const T a_sc = sr - se;
        sum_ss += a_ss;
        sum_sc += a_sc;
        off += -kap * a_ss * xs[nb[e]] + kap * al * a_sc * xc[nb[e]];
    }
    InsideRow<T, DIM> R;
    R.ss_d = phr * D->dt_inv + D->ks_half * phr * cr + kap * sum_ss;
    R.sc_d = al * sr * D->dt_inv + D->ks_half * (al * sr * cr + phr * sr) + kap * al * sum_sc;
    R.cs_d = D->kc_half * phr * cr;
    R.cc_d = D->dt_inv + D->kc_half * (al * sr * cr + phr * sr);
    R.off_s = off;
    return R;
}

// c-row diagonal entries of a node (inside or ghost)
template <typename T>
__device__ __forceinline__ void c_row(const LevelDesc<T> *D, long long idx, T &cs_d, T &cc_d)
{
    const T sr = D->s[idx], cr = D->c[idx];
    const T phr = D->alpha * cr + D->beta;
    cs_d = D->kc_half * phr * cr;
    cc_d = D->dt_inv + D->kc_half * (D->alpha * sr * cr + phr * sr);
}

// ---------------------------------------------------------------------------
// collective red-black Gauss-Seidel on inside nodes (section 3.5.1): the 2x2
// block of eq. (matrixP) is solved for the node's (delta s, delta c) with its
// neighbours (the other colour) fixed
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_smooth_colour(const LevelDesc<T> *__restrict__ descs,
                                                          const int4 *__restrict__ work, int nwork, int colour)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<T> *D = descs + item_desc(w);
    const int p = w.z + (threadIdx.x & 63);
    if (p >= w.w) return;
    const long long row = w.y;
    const long long idx = colour * D->cs + row * D->Wp + p;
    if (D->type[idx] != kIn) return;
    int i, j, k;
    node_coords<DIM>(D->n, colour, row, p, i, j, k);
    long long nb[2 * DIM];
    neighbours<DIM>(D->n, D->Wp, D->cs, colour, row, i, p, nb);
    const InsideRow<T, DIM> R = inside_row<T, DIM>(D, idx, nb, D->x_s, D->x_c);
    const T rs = D->rhs_s[idx] - R.off_s;
    const T rc = D->rhs_c[idx];
    const T det = R.ss_d * R.cc_d - R.sc_d * R.cs_d;
    D->x_s[idx] = (R.cc_d * rs - R.sc_d * rc) / det;
    D->x_c[idx] = (R.ss_d * rc - R.cs_d * rs) / det;
}

// ---------------------------------------------------------------------------
// ghost relaxation (eq. RelGhost), Jacobi over the ghosts of a level:
// phase A computes delta s_g + tau (rhs_g - sum_k w_k delta s_k) for all ghosts,
// phase B writes it back and relaxes the ghost c-row with the new (or old)
// delta s_g
// ---------------------------------------------------------------------------
template <typename T, int NST>
__global__ __launch_bounds__(kBlock) void k_ghost_a(const LevelDesc<T> *__restrict__ descs,
                                                    const int4 *__restrict__ work, int nwork)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<T> *D = descs + item_desc(w);
    const int q = w.z + (threadIdx.x & 63);
    if (q >= w.w) return;
    const int ng = D->ng;
    const long long g = D->g_idx[q];
    T v = 0;
#pragma unroll
    for (int k = 0; k < NST; ++k) v += D->g_w[k * ng + q] * D->x_s[D->g_st[k * ng + q]];
    const T old = D->x_s[g];
    D->g_old[q] = old;
    D->g_tmp[q] = old + D->tau_s * (D->rhs_s[g] - v);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_ghost_b(const LevelDesc<T> *__restrict__ descs,
                                                    const int4 *__restrict__ work, int nwork)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<T> *D = descs + item_desc(w);
    const int q = w.z + (threadIdx.x & 63);
    if (q >= w.w) return;
    const long long g = D->g_idx[q];
    const T ns = D->g_tmp[q];
    D->x_s[g] = ns;
    T cs_d, cc_d;
    c_row<T>(D, g, cs_d, cc_d);
    const T dsv = D->ghost_c_new ? ns : D->g_old[q];
    const T xc = D->x_c[g];
    D->x_c[g] = xc + (D->rhs_c[g] - (cs_d * dsv + cc_d * xc)) / cc_d;
}

// ---------------------------------------------------------------------------
// defect r = rhs - J x on all active rows (section 3.5.2), with its max norm
// ---------------------------------------------------------------------------
template <typename T, int DIM, int NST>
__global__ __launch_bounds__(kBlock) void k_defect(const LevelDesc<T> *__restrict__ descs,
                                                   const int4 *__restrict__ work, int nwork,
                                                   unsigned long long *norm_slot)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<T> *D = descs + item_desc(w);
    const int kind = item_kind(w);
    const int lane = threadIdx.x & 63;
    unsigned long long bits = 0;
    if (kind < 2) {
        const int p = w.z + lane;
        const long long row = w.y;
        const long long idx = kind * D->cs + row * D->Wp + p;
        if (p < w.w && D->type[idx] == kIn) {
            int i, j, k;
            node_coords<DIM>(D->n, kind, row, p, i, j, k);
            long long nb[2 * DIM];
            neighbours<DIM>(D->n, D->Wp, D->cs, kind, row, i, p, nb);
            const InsideRow<T, DIM> R = inside_row<T, DIM>(D, idx, nb, D->x_s, D->x_c);
            const T xs = D->x_s[idx], xc = D->x_c[idx];
            const T rs = D->rhs_s[idx] - (R.ss_d * xs + R.sc_d * xc + R.off_s);
            const T rc = D->rhs_c[idx] - (R.cs_d * xs + R.cc_d * xc);
            D->r_s[idx] = rs;
            D->r_c[idx] = rc;
            if (norm_slot) {
                unsigned long long a = abs_bits((double)rs), b = abs_bits((double)rc);
                bits = a > b ? a : b;
            }
        }
    } else {
        const int q = w.z + lane;
        if (q < w.w) {
            const int ng = D->ng;
            const long long g = D->g_idx[q];
            T v = 0;
#pragma unroll
            for (int k = 0; k < NST; ++k) v += D->g_w[k * ng + q] * D->x_s[D->g_st[k * ng + q]];
            T cs_d, cc_d;
            c_row<T>(D, g, cs_d, cc_d);
            const T rs = D->rhs_s[g] - v;
            const T rc = D->rhs_c[g] - (cs_d * D->x_s[g] + cc_d * D->x_c[g]);
            D->r_s[g] = rs;
            D->r_c[g] = rc;
            if (norm_slot) {
                unsigned long long a = abs_bits((double)rs), b = abs_bits((double)rc);
                bits = a > b ? a : b;
            }
        }
    }
    if (norm_slot) norm_accumulate(norm_slot, bits);
}

// y = J x on all active rows
template <typename T, int DIM, int NST>
__global__ __launch_bounds__(kBlock) void k_apply_J(const LevelDesc<T> *__restrict__ descs,
                                                    const int4 *__restrict__ work, int nwork)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<T> *D = descs + item_desc(w);
    const int kind = item_kind(w);
    const int lane = threadIdx.x & 63;
    if (kind < 2) {
        const int p = w.z + lane;
        if (p >= w.w) return;
        const long long row = w.y;
        const long long idx = kind * D->cs + row * D->Wp + p;
        if (D->type[idx] != kIn) return;
        int i, j, k;
        node_coords<DIM>(D->n, kind, row, p, i, j, k);
        long long nb[2 * DIM];
        neighbours<DIM>(D->n, D->Wp, D->cs, kind, row, i, p, nb);
        const InsideRow<T, DIM> R = inside_row<T, DIM>(D, idx, nb, D->x_s, D->x_c);
        const T xs = D->x_s[idx], xc = D->x_c[idx];
        D->r_s[idx] = R.ss_d * xs + R.sc_d * xc + R.off_s;
        D->r_c[idx] = R.cs_d * xs + R.cc_d * xc;
    } else {
        const int q = w.z + lane;
        if (q >= w.w) return;
        const int ng = D->ng;
        const long long g = D->g_idx[q];
        T v = 0;
#pragma unroll
        for (int k = 0; k < NST; ++k) v += D->g_w[k * ng + q] * D->x_s[D->g_st[k * ng + q]];
        T cs_d, cc_d;
        c_row<T>(D, g, cs_d, cc_d);
        D->r_s[g] = v;
        D->r_c[g] = cs_d * D->x_s[g] + cc_d * D->x_c[g];
    }
}

// ---------------------------------------------------------------------------
// boundary-defect band: value of each reached band node as its fixed linear
// combination of ghost defects (the layered upwind extension of section 3.5.2
// composed at build time)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_band(const LevelDesc<T> *__restrict__ descs,
                                                 const int4 *__restrict__ work, int nwork)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<T> *D = descs + item_desc(w);
    const int b = w.z + (threadIdx.x & 63);
    if (b >= w.w) return;
    const int cnt = D->b_cnt[b];
    if (cnt == 0) return;
    const int nb = D->nb;
    T v = 0;
    for (int j = 0; j < cnt; ++j) v += D->b_wt[j * nb + b] * D->r_s[D->b_src[j * nb + b]];
    D->r_s[D->b_idx[b]] = v;
}

// ---------------------------------------------------------------------------
// restriction to the next coarser level (section 3.5.2, Fig. Neigh): modified
// full weighting; inside rows read inside fine defects, boundary rows read
// ghost and reached band defects, c-rows use full weighting renormalised over
// active fine nodes.  Also clears the coarse correction.
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_restrict(const LevelDesc<T> *__restrict__ descs,
                                                     const int4 *__restrict__ work, int nwork)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<T> *C = descs + item_desc(w);
    const LevelDesc<T> *F = C - 1;
    const int kind = item_kind(w);
    const int lane = threadIdx.x & 63;
    long long cidx;
    int ci, cj, ck;
    bool coarse_inside;
    if (kind < 2) {
        const int p = w.z + lane;
        if (p >= w.w) return;
        cidx = kind * C->cs + (long long)w.y * C->Wp + p;
        if (C->type[cidx] != kIn) return;
        node_coords<DIM>(C->n, kind, w.y, p, ci, cj, ck);
        coarse_inside = true;
    } else {
        const int q = w.z + lane;
        if (q >= w.w) return;
        cidx = C->g_idx[q];
        // coordinates of the ghost from its storage index
        const long long colour = cidx / C->cs;
        const long long rem = cidx - colour * C->cs;
        const long long row = rem / C->Wp;
        const int p = (int)(rem - row * C->Wp);
        node_coords<DIM>(C->n, (int)colour, row, p, ci, cj, ck);
        coarse_inside = false;
    }
    const int fn = F->n, fWp = F->Wp;
    const long long fcs = F->cs;
    const int fc[3] = {2 * ci, 2 * cj, 2 * ck};
    T wa[3][3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        bool ex[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            int id[3] = {fc[0], fc[1], fc[2]};
            id[a] += e ? 1 : -1;
            if (id[a] < 0 || id[a] >= fn) {
                ex[e] = true;
                continue;
            }
            const long long q = sidx(fn, fWp, fcs, id[0], id[1], id[2]);
            const uint8_t t = F->type[q];
            ex[e] = coarse_inside ? (t != kIn) : (t == kIn || (t == kOut && !F->ext[q]));
        }
        if (!ex[0] && !ex[1]) { wa[a][0] = T(0.25); wa[a][1] = T(0.5); wa[a][2] = T(0.25); }
        else if (!ex[0] && ex[1]) { wa[a][0] = T(0.5); wa[a][1] = T(0.5); wa[a][2] = T(0); }
        else if (ex[0] && !ex[1]) { wa[a][0] = T(0); wa[a][1] = T(0.5); wa[a][2] = T(0.5); }
        else { wa[a][0] = T(0); wa[a][1] = T(1); wa[a][2] = T(0); }
    }
    const long long fcentre = sidx(fn, fWp, fcs, fc[0], fc[1], fc[2]);
    T vs = 0, wcen = 0, vc = 0, wcs = 0;
    constexpr int NST = DIM == 2 ? 9 : 27;
#pragma unroll
    for (int kk = 0; kk < NST; ++kk) {
        const int d0 = kk % 3 - 1, d1 = (kk / 3) % 3 - 1, d2 = DIM == 3 ? kk / 9 - 1 : 0;
        const int id0 = fc[0] + d0, id1 = fc[1] + d1, id2 = fc[2] + d2;
        T wk = wa[0][d0 + 1] * wa[1][d1 + 1];
        T wf = (d0 == 0 ? T(0.5) : T(0.25)) * (d1 == 0 ? T(0.5) : T(0.25));
        if (DIM == 3) {
            wk *= wa[2][d2 + 1];
            wf *= (d2 == 0 ? T(0.5) : T(0.25));
        }
        if (id0 < 0 || id0 >= fn || id1 < 0 || id1 >= fn || (DIM == 3 && (id2 < 0 || id2 >= fn))) {
            wcen += wk;
            continue;
        }
        const long long q = sidx(fn, fWp, fcs, id0, id1, id2);
        const uint8_t t = F->type[q];
        bool excluded = coarse_inside ? (t != kIn) : (t == kIn || (t == kOut && !F->ext[q]));
        if (q == fcentre) excluded = false;
        if (excluded) wcen += wk;
        else if (wk != T(0)) vs += wk * F->r_s[q];
        if (t != kOut) {
            vc += wf * F->r_c[q];
            wcs += wf;
        }
    }
    vs += wcen * F->r_s[fcentre];
    C->rhs_s[cidx] = vs;
    C->rhs_c[cidx] = wcs > T(0) ? vc / wcs : T(0);
    C->x_s[cidx] = T(0);
    C->x_c[cidx] = T(0);
}

// ---------------------------------------------------------------------------
// prolongation (section 3.5.3): bilinear (trilinear) interpolation of the
// coarse correction over active coarse nodes, renormalised, added to x
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__device__ __forceinline__ void node_from_item(const LevelDesc<T> *D, int4 w, int lane, bool &ok, long long &idx,
                                               int &i, int &j, int &k)
{
    const int kind = item_kind(w);
    ok = false;
    if (kind < 2) {
        const int p = w.z + lane;
        if (p >= w.w) return;
        idx = kind * D->cs + (long long)w.y * D->Wp + p;
        if (D->type[idx] != kIn) return;
        node_coords<DIM>(D->n, kind, w.y, p, i, j, k);
    } else {
        const int q = w.z + lane;
        if (q >= w.w) return;
        idx = D->g_idx[q];
        const long long colour = idx / D->cs;
        const long long rem = idx - colour * D->cs;
        const long long row = rem / D->Wp;
        node_coords<DIM>(D->n, (int)colour, row, (int)(rem - row * D->Wp), i, j, k);
    }
    ok = true;
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_prolong(const LevelDesc<T> *__restrict__ descs,
                                                    const int4 *__restrict__ work, int nwork)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<T> *F = descs + item_desc(w);
    const LevelDesc<T> *C = F + 1;
    bool ok;
    long long idx;
    int fi[3];
    node_from_item<T, DIM>(F, w, threadIdx.x & 63, ok, idx, fi[0], fi[1], fi[2]);
    if (!ok) return;
    T ws = 0, es = 0, ec = 0;
#pragma unroll
    for (int corner = 0; corner < (1 << DIM); ++corner) {
        int id[3] = {0, 0, 0};
        T wk = 1;
        bool skip = false;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int bit = (corner >> a) & 1;
            if ((fi[a] & 1) == 0) {
                if (bit) skip = true;
                id[a] = fi[a] >> 1;
            } else {
                id[a] = (fi[a] >> 1) + bit;
                wk *= T(0.5);
            }
        }
        if (skip) continue;
        const long long q = sidx(C->n, C->Wp, C->cs, id[0], id[1], id[2]);
        if (C->type[q] == kOut) continue;
        ws += wk;
        es += wk * C->x_s[q];
        ec += wk * C->x_c[q];
    }
    if (ws > T(0)) {
        F->x_s[idx] += es / ws;
        F->x_c[idx] += ec / ws;
    }
}

// ---------------------------------------------------------------------------
// coarse linearisation point: injection where the fine centre is active,
// otherwise full weighting over the active fine neighbours
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_inject(const LevelDesc<T> *__restrict__ descs,
                                                   const int4 *__restrict__ work, int nwork)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<T> *C = descs + item_desc(w);
    const LevelDesc<T> *F = C - 1;
    bool ok;
    long long cidx;
    int ci[3];
    node_from_item<T, DIM>(C, w, threadIdx.x & 63, ok, cidx, ci[0], ci[1], ci[2]);
    if (!ok) return;
    const int fn = F->n;
    const int fc[3] = {2 * ci[0], 2 * ci[1], 2 * ci[2]};
    const long long fq = sidx(fn, F->Wp, F->cs, fc[0], fc[1], fc[2]);
    if (F->type[fq] != kOut) {
        C->s[cidx] = F->s[fq];
        C->c[cidx] = F->c[fq];
        return;
    }
    T ws = 0, vs = 0, vc = 0;
    constexpr int NST = DIM == 2 ? 9 : 27;
    for (int kk = 0; kk < NST; ++kk) {
        const int d[3] = {kk % 3 - 1, (kk / 3) % 3 - 1, DIM == 3 ? kk / 9 - 1 : 0};
        int id[3];
        T wk = 1;
        bool in = true;
        for (int a = 0; a < 3; ++a) {
            id[a] = fc[a] + d[a];
            if (a < DIM) {
                wk *= d[a] == 0 ? T(0.5) : T(0.25);
                if (id[a] < 0 || id[a] >= fn) in = false;
            }
        }
        if (!in) continue;
        const long long q = sidx(fn, F->Wp, F->cs, id[0], id[1], id[2]);
        if (F->type[q] == kOut) continue;
        ws += wk;
        vs += wk * F->s[q];
        vc += wk * F->c[q];
    }
    C->s[cidx] = vs / ws;
    C->c[cidx] = vc / ws;
}

// ---------------------------------------------------------------------------
// finest level, FP64: explicit half of the Crank-Nicolson step (section 3.1,
// eq. discTime) and the Newton residual (eqs. FDs, FDc, BCs)
// ---------------------------------------------------------------------------
struct StepArgs {
    const double *sn, *cn;          // W^n (split layout)
    double *bs, *bc;                // explicit half (split layout)
    const double *fn, *fnp1;        // compact [f1 | f2] or null
    const double *sb;               // per-ghost boundary values or null
    double sb_const;
};

template <int DIM>
__device__ __forceinline__ double Ls_h(const LevelDesc<double> *D, const double *s, const double *c, long long idx,
                                       const long long *nb)
{
    const double phg = D->alpha * c[idx] + D->beta;
    double diff = 0.0;
#pragma unroll
    for (int e = 0; e < 2 * DIM; ++e) diff += ((D->alpha * c[nb[e]] + D->beta) + phg) * (s[nb[e]] - s[idx]);
    return -(2.0 * D->ks_half) * phg * s[idx] * c[idx] + D->d_half_h2 * diff;
}

__device__ __forceinline__ double Lc_h(const LevelDesc<double> *D, const double *s, const double *c, long long idx)
{
    return -(2.0 * D->kc_half) * (D->alpha * c[idx] + D->beta) * s[idx] * c[idx];
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_explicit_half(const LevelDesc<double> *__restrict__ descs,
                                                          const int4 *__restrict__ work, int nwork, StepArgs A)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<double> *D = descs + item_desc(w);
    bool ok;
    long long idx;
    int i, j, k;
    node_from_item<double, DIM>(D, w, threadIdx.x & 63, ok, idx, i, j, k);
    if (!ok) return;
    const bool inside = item_kind(w) < 2;
    const int r = D->cmap[idx];
    const int na = D->na;
    if (inside) {
        long long nb[2 * DIM];
        neighbours<DIM>(D->n, D->Wp, D->cs, item_kind(w), (long long)j + (long long)D->n * k, i, i >> 1, nb);
        double bsv = (D->alpha * A.cn[idx] + D->beta) * A.sn[idx] * D->dt_inv + 0.5 * Ls_h<DIM>(D, A.sn, A.cn, idx, nb);
        if (A.fn) bsv += 0.5 * (A.fn[r] + A.fnp1[r]);
        A.bs[idx] = bsv;
    } else {
        A.bs[idx] = 0.0;
    }
    double bcv = A.cn[idx] * D->dt_inv + 0.5 * Lc_h(D, A.sn, A.cn, idx);
    if (A.fn) bcv += 0.5 * (A.fn[na + r] + A.fnp1[na + r]);
    A.bc[idx] = bcv;
}

// F(W) at the linearisation point (s, c) of level 0, written to rhs_s / rhs_c
template <int DIM, int NST>
__global__ __launch_bounds__(kBlock) void k_residual(const LevelDesc<double> *__restrict__ descs,
                                                     const int4 *__restrict__ work, int nwork, StepArgs A,
                                                     unsigned long long *norm_slot)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<double> *D = descs + item_desc(w);
    bool ok;
    long long idx;
    int i, j, k;
    const int lane = threadIdx.x & 63;
    node_from_item<double, DIM>(D, w, lane, ok, idx, i, j, k);
    unsigned long long bits = 0;
    if (ok) {
        const double *s = D->s, *c = D->c;
        double fs;
        if (item_kind(w) < 2) {
            long long nb[2 * DIM];
            neighbours<DIM>(D->n, D->Wp, D->cs, item_kind(w), (long long)j + (long long)D->n * k, i, i >> 1, nb);
            fs = (D->alpha * c[idx] + D->beta) * s[idx] * D->dt_inv - 0.5 * Ls_h<DIM>(D, s, c, idx, nb) - A.bs[idx];
        } else {
            const int q = w.z + lane;
            const int ng = D->ng;
            double v = 0.0;
#pragma unroll
            for (int kk = 0; kk < NST; ++kk) v += D->g_w[kk * ng + q] * s[D->g_st[kk * ng + q]];
            fs = v - (A.sb ? A.sb[q] : A.sb_const);
        }
        const double fc = c[idx] * D->dt_inv - 0.5 * Lc_h(D, s, c, idx) - A.bc[idx];
        D->rhs_s[idx] = fs;
        D->rhs_c[idx] = fc;
        if (norm_slot) {
            unsigned long long a = abs_bits(fs), b = abs_bits(fc);
            bits = a > b ? a : b;
        }
    }
    if (norm_slot) norm_accumulate(norm_slot, bits);
}

// W <- W - dW on active nodes, with |dW|_inf and |W_old|_inf
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_newton_update(const LevelDesc<double> *__restrict__ descs,
                                                          const int4 *__restrict__ work, int nwork,
                                                          unsigned long long *norm_dw, unsigned long long *norm_w)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<double> *D = descs + item_desc(w);
    bool ok;
    long long idx;
    int i, j, k;
    node_from_item<double, DIM>(D, w, threadIdx.x & 63, ok, idx, i, j, k);
    unsigned long long bd = 0, bw = 0;
    if (ok) {
        const double s = D->s[idx], c = D->c[idx], xs = D->x_s[idx], xc = D->x_c[idx];
        unsigned long long a = abs_bits(xs), b = abs_bits(xc);
        bd = a > b ? a : b;
        a = abs_bits(s);
        b = abs_bits(c);
        bw = a > b ? a : b;
        D->s[idx] = s - xs;
        D->c[idx] = c - xc;
    }
    norm_accumulate(norm_dw, bd);
    norm_accumulate(norm_w, bw);
}

// ---------------------------------------------------------------------------
// mixed precision: FP64 <-> FP32 transfers on a level
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_to_f32(const LevelDesc<double> *__restrict__ d64,
                                                   const LevelDesc<float> *__restrict__ d32,
                                                   const int4 *__restrict__ work, int nwork, int what)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<double> *D = d64 + item_desc(w);
    const LevelDesc<float> *E = d32 + item_desc(w);
    bool ok;
    long long idx;
    int i, j, k;
    node_from_item<double, DIM>(D, w, threadIdx.x & 63, ok, idx, i, j, k);
    if (!ok) return;
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
__global__ __launch_bounds__(kBlock) void k_add_f32(const LevelDesc<double> *__restrict__ d64,
                                                    const LevelDesc<float> *__restrict__ d32,
                                                    const int4 *__restrict__ work, int nwork)
{
    const int it = blockIdx.x * kItemsPerBlock + (threadIdx.x >> 6);
    if (it >= nwork) return;
    const int4 w = work[it];
    const LevelDesc<double> *D = d64 + item_desc(w);
    const LevelDesc<float> *E = d32 + item_desc(w);
    bool ok;
    long long idx;
    int i, j, k;
    node_from_item<double, DIM>(D, w, threadIdx.x & 63, ok, idx, i, j, k);
    if (!ok) return;
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
    const int i = threadIdx.x;
    if (i < n) p[i] = 0ull;
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
// coarsest level: dense LU with partial pivoting in one workgroup (FP64)
// ---------------------------------------------------------------------------
template <int DIM, int NST>
__global__ __launch_bounds__(1024) void k_coarse_factor(const LevelDesc<double> *__restrict__ descs, int lev,
                                                        const int *__restrict__ c2s, double *__restrict__ A,
                                                        int *__restrict__ piv, int *__restrict__ status)
{
    const LevelDesc<double> *D = descs + lev;
    const int na = D->na, ni = D->ni, N = 2 * na;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (long long e = tid; e < (long long)N * N; e += nt) A[e] = 0.0;
    __syncthreads();
    for (int r = tid; r < na; r += nt) {
        const long long idx = c2s[r];
        const long long colour = idx / D->cs;
        const long long rem = idx - colour * D->cs;
        const long long row = rem / D->Wp;
        const int p = (int)(rem - row * D->Wp);
        int i, j, k;
        node_coords<DIM>(D->n, (int)colour, row, p, i, j, k);
        double cs_d, cc_d;
        c_row<double>(D, idx, cs_d, cc_d);
        if (r < ni) {
            long long nb[2 * DIM];
            neighbours<DIM>(D->n, D->Wp, D->cs, (int)colour, row, i, p, nb);
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
                A[(long long)r * N + q] += -kap * a_ss;
                A[(long long)r * N + na + q] += kap * al * a_sc;
            }
            A[(long long)r * N + r] += phr * D->dt_inv + D->ks_half * phr * cr + kap * sum_ss;
            A[(long long)r * N + na + r] += al * sr * D->dt_inv + D->ks_half * (al * sr * cr + phr * sr) + kap * al * sum_sc;
        } else {
            const int q = r - ni, ng = D->ng;
            for (int kk = 0; kk < NST; ++kk) {
                const double wk = D->g_w[kk * ng + q];
                if (wk == 0.0) continue;
                A[(long long)r * N + D->cmap[D->g_st[kk * ng + q]]] += wk;
            }
        }
        A[(long long)(na + r) * N + r] += cs_d;
        A[(long long)(na + r) * N + na + r] += cc_d;
    }
    __syncthreads();
    __shared__ double red_v[1024];
    __shared__ int red_i[1024];
    __shared__ int s_bad;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int kc = 0; kc < N; ++kc) {
        // pivot: largest |A[i][kc]| for i >= kc, first index on ties
        double best = -1.0;
        int bi = N;
        for (int i2 = kc + tid; i2 < N; i2 += nt) {
            const double v = fabs(A[(long long)i2 * N + kc]);
            if (v > best) { best = v; bi = i2; }
        }
        red_v[tid] = best;
        red_i[tid] = bi;
        __syncthreads();
        for (int off = nt >> 1; off > 0; off >>= 1) {
            if (tid < off) {
                const double ov = red_v[tid + off];
                const int oi = red_i[tid + off];
                if (ov > red_v[tid] || (ov == red_v[tid] && oi < red_i[tid])) { red_v[tid] = ov; red_i[tid] = oi; }
            }
            __syncthreads();
        }
        const int pr = red_i[0];
        const double pv = red_v[0];
        if (tid == 0) {
            piv[kc] = pr;
            if (!(pv > 0.0) || pv != pv || pr >= N) s_bad = 1;
        }
        __syncthreads();
        if (s_bad) break;
        if (pr != kc)
            for (int jj = tid; jj < N; jj += nt) {
                const double t = A[(long long)kc * N + jj];
                A[(long long)kc * N + jj] = A[(long long)pr * N + jj];
                A[(long long)pr * N + jj] = t;
            }
        __syncthreads();
        const double dk = A[(long long)kc * N + kc];
        for (int i2 = kc + 1 + tid; i2 < N; i2 += nt) A[(long long)i2 * N + kc] /= dk;
        __syncthreads();
        const int m = N - kc - 1;
        for (long long e = tid; e < (long long)m * m; e += nt) {
            const int i2 = kc + 1 + (int)(e / m), jj = kc + 1 + (int)(e % m);
            A[(long long)i2 * N + jj] -= A[(long long)i2 * N + kc] * A[(long long)kc * N + jj];
        }
        __syncthreads();
    }
    if (tid == 0) *status = s_bad ? 1 : 0;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_coarse_solve(const LevelDesc<T> *__restrict__ descs, int lev,
                                                       const int *__restrict__ c2s, const double *__restrict__ A,
                                                       const int *__restrict__ piv)
{
    extern __shared__ double b[];
    const LevelDesc<T> *D = descs + lev;
    const int na = D->na, N = 2 * na;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int r = tid; r < na; r += nt) {
        b[r] = (double)D->rhs_s[c2s[r]];
        b[na + r] = (double)D->rhs_c[c2s[r]];
    }
    __syncthreads();
    if (tid == 0)
        for (int kc = 0; kc < N; ++kc) {
            const int p = piv[kc];
            if (p != kc) { const double t = b[kc]; b[kc] = b[p]; b[p] = t; }
        }
    __syncthreads();
    for (int jj = 0; jj < N; ++jj) {
        const double bj = b[jj];
        for (int i2 = jj + 1 + tid; i2 < N; i2 += nt) b[i2] -= A[(long long)i2 * N + jj] * bj;
        __syncthreads();
    }
    for (int jj = N - 1; jj >= 0; --jj) {
        if (tid == 0) b[jj] /= A[(long long)jj * N + jj];
        __syncthreads();
        const double bj = b[jj];
        for (int i2 = tid; i2 < jj; i2 += nt) b[i2] -= A[(long long)i2 * N + jj] * bj;
        __syncthreads();
    }
    for (int r = tid; r < na; r += nt) {
        D->x_s[c2s[r]] = (T)b[r];
        D->x_c[c2s[r]] = (T)b[na + r];
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned grid_of(int nwork) { return (unsigned)((nwork + kItemsPerBlock - 1) / kItemsPerBlock); }

#define LSMG_DISPATCH_DIM(dim, ...) \
    do { if ((dim) == 2) { constexpr int DIM = 2; constexpr int NST = 9; __VA_ARGS__; } \
         else { constexpr int DIM = 3; constexpr int NST = 27; __VA_ARGS__; } } while (0)

template <typename T>
void launch_smooth_colour(int dim, const LevelDesc<T> *d, const int4 *w, int nw, int colour, hipStream_t s)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; k_smooth_colour<T, DIM><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw, colour));
}

template <typename T>
void launch_ghost(int dim, const LevelDesc<T> *d, const int4 *w, int nw, hipStream_t s)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)DIM; k_ghost_a<T, NST><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw));
    k_ghost_b<T><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw);
}

template <typename T>
void launch_defect(int dim, const LevelDesc<T> *d, const int4 *w, int nw, unsigned long long *slot, hipStream_t s)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, k_defect<T, DIM, NST><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw, slot));
}

template <typename T>
void launch_apply_J(int dim, const LevelDesc<T> *d, const int4 *w, int nw, hipStream_t s)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, k_apply_J<T, DIM, NST><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw));
}

template <typename T>
void launch_band(const LevelDesc<T> *d, const int4 *w, int nw, hipStream_t s)
{
    if (nw <= 0) return;
    k_band<T><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw);
}

template <typename T>
void launch_restrict(int dim, const LevelDesc<T> *d, const int4 *w, int nw, hipStream_t s)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; k_restrict<T, DIM><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw));
}

template <typename T>
void launch_prolong(int dim, const LevelDesc<T> *d, const int4 *w, int nw, hipStream_t s)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; k_prolong<T, DIM><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw));
}

template <typename T>
void launch_inject(int dim, const LevelDesc<T> *d, const int4 *w, int nw, hipStream_t s)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; k_inject<T, DIM><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw));
}

void launch_explicit_half(int dim, const LevelDesc<double> *d, const int4 *w, int nw, const StepArgsHost &a,
                          hipStream_t s)
{
    if (nw <= 0) return;
    StepArgs A{a.sn, a.cn, a.bs, a.bc, a.fn, a.fnp1, a.sb, a.sb_const};
    LSMG_DISPATCH_DIM(dim, (void)NST; k_explicit_half<DIM><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw, A));
}

void launch_residual(int dim, const LevelDesc<double> *d, const int4 *w, int nw, const StepArgsHost &a,
                     unsigned long long *slot, hipStream_t s)
{
    if (nw <= 0) return;
    StepArgs A{a.sn, a.cn, a.bs, a.bc, a.fn, a.fnp1, a.sb, a.sb_const};
    LSMG_DISPATCH_DIM(dim, k_residual<DIM, NST><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw, A, slot));
}

void launch_newton_update(int dim, const LevelDesc<double> *d, const int4 *w, int nw, unsigned long long *ndw,
                          unsigned long long *nw_slot, hipStream_t s)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; k_newton_update<DIM><<<grid_of(nw), kBlock, 0, s>>>(d, w, nw, ndw, nw_slot));
}

void launch_to_f32(int dim, const LevelDesc<double> *d64, const LevelDesc<float> *d32, const int4 *w, int nw,
                   int what, hipStream_t s)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; k_to_f32<DIM><<<grid_of(nw), kBlock, 0, s>>>(d64, d32, w, nw, what));
}

void launch_add_f32(int dim, const LevelDesc<double> *d64, const LevelDesc<float> *d32, const int4 *w, int nw,
                    hipStream_t s)
{
    if (nw <= 0) return;
    LSMG_DISPATCH_DIM(dim, (void)NST; k_add_f32<DIM><<<grid_of(nw), kBlock, 0, s>>>(d64, d32, w, nw));
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

void launch_zero_u64(unsigned long long *p, int n, hipStream_t s) { k_zero_u64<<<1, 64, 0, s>>>(p, n); }

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

void launch_coarse_factor(int dim, const LevelDesc<double> *d, int lev, const int *c2s, double *A, int *piv,
                          int *status, hipStream_t s)
{
    LSMG_DISPATCH_DIM(dim, k_coarse_factor<DIM, NST><<<1, 1024, 0, s>>>(d, lev, c2s, A, piv, status));
}

template <typename T>
void launch_coarse_solve(const LevelDesc<T> *d, int lev, int N, const int *c2s, const double *A, const int *piv,
                         hipStream_t s)
{
    k_coarse_solve<T><<<1, 1024, (size_t)N * sizeof(double), s>>>(d, lev, c2s, A, piv);
}

#define LSMG_INST(T) \
    template void launch_smooth_colour<T>(int, const LevelDesc<T> *, const int4 *, int, int, hipStream_t); \
    template void launch_ghost<T>(int, const LevelDesc<T> *, const int4 *, int, hipStream_t); \
    template void launch_defect<T>(int, const LevelDesc<T> *, const int4 *, int, unsigned long long *, hipStream_t); \
    template void launch_apply_J<T>(int, const LevelDesc<T> *, const int4 *, int, hipStream_t); \
    template void launch_band<T>(const LevelDesc<T> *, const int4 *, int, hipStream_t); \
    template void launch_restrict<T>(int, const LevelDesc<T> *, const int4 *, int, hipStream_t); \
    template void launch_prolong<T>(int, const LevelDesc<T> *, const int4 *, int, hipStream_t); \
    template void launch_inject<T>(int, const LevelDesc<T> *, const int4 *, int, hipStream_t); \
    template void launch_gather_compact<T>(const int *, int, const T *, const T *, double *, hipStream_t); \
    template void launch_scatter_compact<T>(const int *, int, const double *, T *, T *, hipStream_t); \
    template void launch_fill<T>(T *, long long, T, hipStream_t); \
    template void launch_coarse_solve<T>(const LevelDesc<T> *, int, int, const int *, const double *, const int *, \
                                         hipStream_t);
LSMG_INST(double)
LSMG_INST(float)
template void launch_fill<int>(int *, long long, int, hipStream_t);
template void launch_fill<uint8_t>(uint8_t *, long long, uint8_t, hipStream_t);

}  // namespace lsmg
