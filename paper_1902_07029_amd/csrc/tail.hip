// Coarse tail of the V- or W-cycle held in LDS (gfx950, one 1024-thread
// workgroup per hierarchy).
//
// The coarsest levels (up to kTailMaxNodes active nodes) run in one workgroup with
// a barrier between phases (smoothing colours, ghost relaxation, defect, band,
// restriction, coarsest solve, prolongation).  Reading them from HBM makes each
// phase cost a few dependent memory round trips.  Here every value of those
// levels (s, c, corrections, right-hand sides, defects) is gathered into LDS
// once at entry, as compact arrays in the tail's node order (inside nodes of
// colour 0, of colour 1, then ghosts), and the tables that connect the nodes
// (axis neighbours, ghost stencils, band sources, restriction neighbourhoods,
// prolongation corners) were built once per hierarchy.  Only the correction of
// the entry level goes back to HBM.  The row arithmetic is the one of
// rows.hpp, applied to the same values in the same order as the HBM tail, so
// the two tails give the same bits.
#include <hip/hip_runtime.h>

#include <vector>

#include "hier.hpp"
#include "lsmg_dev.hpp"
#include "lsmg_host.hpp"
#include "rows.hpp"

namespace lsmg {

constexpr uint16_t kSkip = 0xFFFF;   // prolongation corner not used (even coordinate)
constexpr uint16_t kOff = 0xFFFE;    // prolongation corner on an inactive coarse node
constexpr int kSlotBits = 12;        // restriction entries: fine slot in the low 12 bits

// ---------------------------------------------------------------------------
// host: table image of a hierarchy's tail (levels tail_l0 .. nlev-1)
// ---------------------------------------------------------------------------
namespace {

template <typename V>
lsmg_status down(lsmg_hierarchy *H, std::vector<V> &h, const V *d, long long n)
{
    h.assign((size_t)(n > 0 ? n : 0), V());
    if (n > 0) HIPCHK(hipMemcpyAsync(h.data(), d, sizeof(V) * (size_t)n, hipMemcpyDeviceToHost, H->stream));
    return LSMG_OK;
}

struct HostLevel {
    std::vector<int> ijk, st, stg, bidx, bcnt, bsrc, c2s;
    std::vector<uint8_t> type, ext;
    std::vector<int> inv, binv;   // storage -> tail index / band index
};

void unpack(int v, int &i, int &j, int &k)
{
    i = v & 2047;
    j = (v >> 11) & 2047;
    k = (v >> 22) & 1023;
}

long long sidx_h(int dim, const Level &L, int i, int j, int k)
{
    return sidx(dim, L.n, L.Wp, L.cs, i, j, k);
}

}  // namespace

lsmg_status build_tail_tables(lsmg_hierarchy *H)
{
    H->tail_lds = false;
    const int dim = H->dim, nst = H->nst, L = H->nlev, l0 = H->tail_l0, nc = 1 << dim;
    std::vector<HostLevel> hl(L);
    for (int l = l0; l < L; ++l) {
        const Level &Lv = H->L[l];
        HostLevel &h = hl[l];
        std::vector<int> in;
        LSMGCHK(down(H, in, Lv.in_ijk, Lv.ni));
        std::vector<int> gi;
        LSMGCHK(down(H, gi, Lv.g_ijk, Lv.ng));
        LSMGCHK(down(H, h.st, Lv.g_st, (long long)Lv.ng * nst));
        LSMGCHK(down(H, h.stg, Lv.g_stg, (long long)Lv.ng * nst));
        LSMGCHK(down(H, h.bidx, Lv.b_idx, Lv.nb));
        LSMGCHK(down(H, h.bcnt, Lv.b_cnt, Lv.nb));
        LSMGCHK(down(H, h.bsrc, Lv.b_src, (long long)Lv.nb * Lv.bmax));
        LSMGCHK(down(H, h.type, Lv.type, Lv.ssize));
        LSMGCHK(down(H, h.ext, Lv.ext, Lv.ssize));
        if (l == L - 1) LSMGCHK(down(H, h.c2s, Lv.c2s, Lv.na));
        HIPCHK(hipStreamSynchronize(H->stream));
        h.ijk = in;
        h.ijk.insert(h.ijk.end(), gi.begin(), gi.end());
        h.inv.assign((size_t)Lv.ssize, -1);
        for (int t = 0; t < Lv.na; ++t) {
            int i, j, k;
            unpack(h.ijk[t], i, j, k);
            h.inv[(size_t)sidx_h(dim, Lv, i, j, k)] = t;
        }
        h.binv.assign((size_t)Lv.ssize, -1);
        for (int b = 0; b < Lv.nb; ++b) h.binv[(size_t)h.bidx[b]] = b;
    }
    std::vector<uint16_t> tab;
    std::vector<TailLdsLevel> ll(L);
    int nvals = 0, nints = 0, ngmax = 1;
    auto fits = [](int v) { return v >= 0 && v < 0x7FFF; };
    for (int l = l0; l < L; ++l) {
        const Level &Lv = H->L[l];
        HostLevel &h = hl[l];
        TailLdsLevel &d = ll[l];
        d.na = Lv.na;
        d.nb = l < L - 1 ? Lv.nb : 0;
        d.v = nvals;
        nvals += 8 * Lv.na + d.nb + 1;
        if (Lv.na + d.nb + 1 >= (1 << kSlotBits)) return LSMG_OK;
        const int nin = Lv.nin[0] + Lv.nin[1];
        if (l < L - 1) {
            ngmax = std::max(ngmax, Lv.ng);
            d.gop = nints;
            nints += Lv.ng + 1;
            // axis neighbours of the inside nodes (x-, x+, y-, y+[, z-, z+])
            d.nbr = (int)tab.size();
            for (int t = 0; t < nin; ++t) {
                int i, j, k;
                unpack(h.ijk[t], i, j, k);
                // axis neighbours: inside nodes never lie on the box edge
                const long long nb[6] = {sidx_h(dim, Lv, i - 1, j, k), sidx_h(dim, Lv, i + 1, j, k),
                                         sidx_h(dim, Lv, i, j - 1, k), sidx_h(dim, Lv, i, j + 1, k),
                                         dim == 3 ? sidx_h(dim, Lv, i, j, k - 1) : 0,
                                         dim == 3 ? sidx_h(dim, Lv, i, j, k + 1) : 0};
                for (int e = 0; e < 2 * dim; ++e) {
                    const int v = h.inv[(size_t)nb[e]];
                    if (!fits(v)) return LSMG_OK;
                    tab.push_back((uint16_t)v);
                }
            }
            // ghost stencils
            d.gst = (int)tab.size();
            for (int q = 0; q < Lv.ng; ++q)
                for (int k = 0; k < nst; ++k) {
                    const int v = h.inv[(size_t)h.st[(size_t)k * Lv.ng + q]];
                    if (!fits(v)) return LSMG_OK;
                    tab.push_back((uint16_t)(v | (h.stg[(size_t)k * Lv.ng + q] >= 0 ? 0x8000 : 0)));
                }
            // band sources
            d.bcnt = (int)tab.size();
            for (int b = 0; b < Lv.nb; ++b) tab.push_back((uint16_t)h.bcnt[b]);
            d.bsrc = (int)tab.size();
            for (int j = 0; j < Lv.bmax; ++j)
                for (int b = 0; b < Lv.nb; ++b) {
                    int v = 0;
                    if (j < h.bcnt[b]) {
                        v = h.inv[(size_t)h.bsrc[(size_t)j * Lv.nb + b]];
                        if (!fits(v)) return LSMG_OK;
                    }
                    tab.push_back((uint16_t)v);
                }
            // prolongation corners of every active node from level l + 1
            const Level &Cv = H->L[l + 1];
            const HostLevel &hc = hl[l + 1];
            d.pro = (int)tab.size();
            for (int t = 0; t < Lv.na; ++t) {
                int f[3];
                unpack(h.ijk[t], f[0], f[1], f[2]);
                int odd = 0;
                for (int a = 0; a < dim; ++a) odd += f[a] & 1;
                for (int corner = 0; corner < nc; ++corner) {
                    int id[3] = {0, 0, 0};
                    bool skip = false;
                    for (int a = 0; a < dim; ++a) {
                        const int bit = (corner >> a) & 1;
                        if ((f[a] & 1) == 0) {
                            if (bit) skip = true;
                            id[a] = f[a] >> 1;
                        } else {
                            id[a] = (f[a] >> 1) + bit;
                        }
                    }
                    if (skip) {
                        tab.push_back(kSkip);
                        continue;
                    }
                    const long long q = sidx_h(dim, Cv, id[0], id[1], id[2]);
                    if (hc.type[(size_t)q] == kOut) {
                        tab.push_back(kOff);
                        continue;
                    }
                    const int v = hc.inv[(size_t)q];
                    if (!fits(v)) return LSMG_OK;
                    tab.push_back((uint16_t)v);
                }
                tab.push_back((uint16_t)odd);
            }
            // restriction neighbourhoods of the active nodes of level l + 1
            d.rst = (int)tab.size();
            for (int tc = 0; tc < Cv.na; ++tc) {
                int c[3];
                unpack(hc.ijk[tc], c[0], c[1], c[2]);
                const long long fcentre = sidx_h(dim, Lv, 2 * c[0], 2 * c[1], 2 * c[2]);
                for (int kk = 0; kk < nst; ++kk) {
                    const int id0 = 2 * c[0] + kk % 3 - 1, id1 = 2 * c[1] + (kk / 3) % 3 - 1,
                              id2 = dim == 3 ? 2 * c[2] + kk / 9 - 1 : 0;
                    const bool inb = id0 >= 0 && id0 < Lv.n && id1 >= 0 && id1 < Lv.n &&
                                     (dim == 2 || (id2 >= 0 && id2 < Lv.n));
                    const long long q = inb ? sidx_h(dim, Lv, id0, id1, id2) : fcentre;
                    const uint8_t ty = h.type[(size_t)q], ex = h.ext[(size_t)q];
                    int slot;
                    if (ty != kOut) slot = h.inv[(size_t)q];
                    else if (ex) slot = h.binv[(size_t)q] >= 0 ? Lv.na + h.binv[(size_t)q] : -1;
                    else slot = Lv.na + d.nb;   // holds zero
                    if (slot < 0 || slot >= (1 << kSlotBits)) return LSMG_OK;
                    tab.push_back((uint16_t)(slot | (ty << 12) | ((ex ? 1 : 0) << 14) | ((inb ? 1 : 0) << 15)));
                }
            }
        } else {
            // the coarsest solve: compact order of the coarse matrix -> tail order
            d.perm = (int)tab.size();
            for (int r = 0; r < Lv.na; ++r) {
                const int v = h.inv[(size_t)h.c2s[r]];
                if (!fits(v)) return LSMG_OK;
                tab.push_back((uint16_t)v);
            }
        }
        if (tab.size() & 1) tab.push_back(0);
    }
    if (tab.empty()) tab.push_back(0);
    if (tab.size() & 1) tab.push_back(0);
    const int words = (int)(tab.size() / 2);
    uint32_t *dtab = nullptr;
    LSMGCHK(H->alloc(&dtab, words));
    HIPCHK(hipMemcpyAsync(dtab, tab.data(), sizeof(uint32_t) * (size_t)words, hipMemcpyHostToDevice, H->stream));
    HIPCHK(hipStreamSynchronize(H->stream));
    H->tail_tab = dtab;
    H->tail_ll = ll;
    H->tail_sz = TailLdsSize{H->L[L - 1].na, ngmax, nvals, nints, words};
    H->tail_lds = true;
    return LSMG_OK;
}

// ---------------------------------------------------------------------------
// device
// ---------------------------------------------------------------------------
template <typename T>
struct LdsLevel {
    T *s, *c, *xs, *xc, *rhs_s, *rhs_c, *r_c, *r_s;
    const uint16_t *nbr, *gst, *bcnt, *bsrc, *pro, *rst, *perm;
    const int *gop;
    int na, nb, nin;
};

template <typename T>
__device__ __forceinline__ LdsLevel<T> lds_level(const TailArgs &A, int l, T *V, const uint16_t *tab, const int *gop)
{
    const TailLdsLevel &d = A.ll[l];
    LdsLevel<T> Z;
    const int na = d.na;
    T *b = V + d.v;
    Z.s = b;
    Z.c = b + na;
    Z.xs = b + 2 * na;
    Z.xc = b + 3 * na;
    Z.rhs_s = b + 4 * na;
    Z.rhs_c = b + 5 * na;
    Z.r_c = b + 6 * na;
    Z.r_s = b + 7 * na;
    Z.nbr = tab + d.nbr;
    Z.gst = tab + d.gst;
    Z.bcnt = tab + d.bcnt;
    Z.bsrc = tab + d.bsrc;
    Z.pro = tab + d.pro;
    Z.rst = tab + d.rst;
    Z.perm = tab + d.perm;
    Z.gop = gop + d.gop;
    Z.na = na;
    Z.nb = d.nb;
    Z.nin = A.lev[l].nin0 + A.lev[l].nin1;
    return Z;
}

template <typename T, int DIM>
__device__ __forceinline__ InsideRow<T> lds_inside_row(const LevelDesc<T> *D, const LdsLevel<T> &Z, int t)
{
    const uint16_t *nb = Z.nbr + t * 2 * DIM;
    T se[2 * DIM], ce[2 * DIM], xse[2 * DIM], xce[2 * DIM];
#pragma unroll
    for (int e = 0; e < 2 * DIM; ++e) {
        se[e] = Z.s[nb[e]];
        ce[e] = Z.c[nb[e]];
        xse[e] = Z.xs[nb[e]];
        xce[e] = Z.xc[nb[e]];
    }
    return inside_row_vals<T, DIM>(D, Z.s[t], Z.c[t], se, ce, xse, xce);
}

// one smoothing step: colour 0, colour 1, then the composed ghost relaxation
template <typename T, int DIM, int NST>
__device__ void lds_smooth(const LevelDesc<T> *D, const TailLevel &TL, const LdsLevel<T> &Z, T *gb0, T *gb1)
{
    for (int colour = 0; colour < 2; ++colour) {
        const int off = colour ? TL.nin0 : 0, cnt = colour ? TL.nin1 : TL.nin0;
        for (int u = threadIdx.x; u < cnt; u += blockDim.x) {
            const int t = off + u;
            const InsideRow<T> R = lds_inside_row<T, DIM>(D, Z, t);
            T xs, xc;
            block_solve<T>(R, Z.rhs_s[t], Z.rhs_c[t], xs, xc);
            Z.xs[t] = xs;
            Z.xc[t] = xc;
        }
        __syncthreads();
    }
    const int ng = D->ng;
    for (int q = threadIdx.x; q < ng; q += blockDim.x) {
        const uint16_t *gs = Z.gst + q * NST;
        T val[NST];
#pragma unroll
        for (int k = 0; k < NST; ++k) {
            const T xv = Z.xs[gs[k] & 0x7FFF];
            val[k] = (gs[k] & 0x8000) ? T(0) : xv;
        }
        T v = 0;
#pragma unroll
        for (int k = 0; k < NST; ++k) v += D->g_w[k * ng + q] * val[k];
        const int g = Z.nin + q;
        gb0[q] = Z.rhs_s[g] - v;
        gb1[q] = Z.xs[g];
    }
    __syncthreads();
    // the composed rows, kRowGroup lanes per row
    const int sub = threadIdx.x % kRowGroup, grp = threadIdx.x / kRowGroup, ngrp = blockDim.x / kRowGroup;
    for (int q0 = 0; q0 < ng; q0 += ngrp) {
        const int q = q0 + grp;
        const bool on = q < ng;
        const int e0 = on ? Z.gop[q] : 0, e1 = on ? Z.gop[q + 1] : 0;
        const T v = group_ghost_row<T>(D->go_col, D->go_a, D->go_b, gb0, gb1, e0, e1, sub);
        if (on && sub == 0) {
            const int g = Z.nin + q;
            T cs_d, cc_d;
            c_row_vals<T>(D, Z.s[g], Z.c[g], cs_d, cc_d);
            const T xc = Z.xc[g], rc = Z.rhs_c[g];
            Z.xs[g] = v;
            Z.xc[g] = ghost_c_update<T>(cs_d, cc_d, rc, v, xc);
        }
    }
    __syncthreads();
}

template <typename T, int DIM, int NST>
__device__ void lds_defect(const LevelDesc<T> *D, const LdsLevel<T> &Z)
{
    const int ng = D->ng;
    for (int t = threadIdx.x; t < Z.nin + ng; t += blockDim.x) {
        if (t < Z.nin) {
            const InsideRow<T> R = lds_inside_row<T, DIM>(D, Z, t);
            T rs, rc;
            inside_defect_vals<T>(R, Z.rhs_s[t], Z.rhs_c[t], Z.xs[t], Z.xc[t], rs, rc);
            Z.r_s[t] = rs;
            Z.r_c[t] = rc;
        } else {
            const int q = t - Z.nin;
            const uint16_t *gs = Z.gst + q * NST;
            T val[NST];
#pragma unroll
            for (int k = 0; k < NST; ++k) val[k] = Z.xs[gs[k] & 0x7FFF];
            T v = 0;
#pragma unroll
            for (int k = 0; k < NST; ++k) v += D->g_w[k * ng + q] * val[k];
            T cs_d, cc_d;
            c_row_vals<T>(D, Z.s[t], Z.c[t], cs_d, cc_d);
            Z.r_s[t] = Z.rhs_s[t] - v;
            Z.r_c[t] = Z.rhs_c[t] - (cs_d * Z.xs[t] + cc_d * Z.xc[t]);
        }
    }
    __syncthreads();
}

template <typename T>
__device__ void lds_band(const LevelDesc<T> *D, const LdsLevel<T> &Z)
{
    const int nb = Z.nb;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const int cnt = Z.bcnt[b];
        if (cnt == 0) continue;
        T v = 0;
        // sources fetched eight at a time (past the count: the last source again, not
        // summed), summed in order
        for (int j0 = 0; j0 < cnt; j0 += 8) {
            int src[8];
            T wt[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int ju = min(j0 + u, cnt - 1);
                src[u] = Z.bsrc[ju * nb + b];
                wt[u] = D->b_wt[ju * nb + b];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const T t = fma(wt[u], Z.r_s[src[u]], v);
                v = j0 + u < cnt ? t : v;
            }
        }
        Z.r_s[Z.na + b] = v;
    }
    __syncthreads();
}

// restriction from fine level Z onto the active nodes of the coarser level C;
// also clears C's correction
template <typename T, int DIM, int NST>
__device__ void lds_restrict(const LdsLevel<T> &Z, const LdsLevel<T> &C)
{
    for (int tc = threadIdx.x; tc < C.na; tc += blockDim.x) {
        const uint16_t *rt = Z.rst + tc * NST;
        const bool coarse_inside = tc < C.nin;
        uint8_t ex[NST], act[NST];
        T rs[NST], rc[NST];
#pragma unroll
        for (int kk = 0; kk < NST; ++kk) {
            const int e = rt[kk];
            const int slot = e & ((1 << kSlotBits) - 1), ty = (e >> 12) & 3;
            const bool ext = (e >> 14) & 1, inb = (e >> 15) & 1;
            rs[kk] = Z.r_s[slot];
            rc[kk] = slot < Z.na ? Z.r_c[slot] : T(0);
            const bool excl = coarse_inside ? (ty != kIn) : (ty == kIn || (ty == kOut && !ext));
            ex[kk] = inb ? (uint8_t)excl : (uint8_t)1;
            act[kk] = inb && ty != kOut;
        }
        T vs, vc;
        restrict_vals<T, DIM>(ex, act, rs, rc, vs, vc);
        C.rhs_s[tc] = vs;
        C.rhs_c[tc] = vc;
        C.xs[tc] = T(0);
        C.xc[tc] = T(0);
    }
    __syncthreads();
}

// bilinear (trilinear) prolongation from C onto the active nodes of Z, added
template <typename T, int DIM>
__device__ void lds_prolong(const LdsLevel<T> &Z, const LdsLevel<T> &C)
{
    constexpr int NC = 1 << DIM;
    for (int t = threadIdx.x; t < Z.na; t += blockDim.x) {
        const uint16_t *pr = Z.pro + t * (NC + 1);
        T wk = 1;
        for (int a = 0; a < pr[NC]; ++a) wk *= T(0.5);
        T ws = 0, es = 0, ec = 0;
#pragma unroll
        for (int corner = 0; corner < NC; ++corner) {
            const uint16_t e = pr[corner];
            if (e == kSkip) continue;
            const bool on = e != kOff;
            const T xs = on ? C.xs[e] : T(0), xc = on ? C.xc[e] : T(0);
            ws += on ? wk : T(0);
            es += on ? wk * xs : T(0);
            ec += on ? wk * xc : T(0);
        }
        if (ws > T(0)) {
            Z.xs[t] += es / ws;
            Z.xc[t] += ec / ws;
        }
    }
    __syncthreads();
}

// x = A^{-1} rhs on the coarsest level through the Schur complement (as the HBM tail)
template <typename T>
__device__ void lds_coarse(const LevelDesc<T> *D, const LdsLevel<T> &Z, gptr<const double> Ainv, double *b)
{
    const int na = D->na;
    const gptr<const double> Sinv = Ainv, Jsc = Ainv + (long long)na * na, cs = Ainv + 2LL * na * na, cc = cs + na;
    double *rs = b, *rc = b + na, *t = b + 2 * na, *u = b + 3 * na;
    for (int r = threadIdx.x; r < na; r += blockDim.x) {
        const int p = Z.perm[r];
        const double vc = (double)Z.rhs_c[p];
        rs[r] = (double)Z.rhs_s[p];
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
            const int p = Z.perm[r];
            const double csr = cs[r], ccr = cc[r];
            Z.xs[p] = (T)v;
            Z.xc[p] = (T)((rc[r] - csr * v) / ccr);
        }
    }
    __syncthreads();
}

// LDS: [4 ncoarse doubles][ngmax T][ngmax T][nvals T][nints int][tab_words uint32]
template <typename T, int DIM, int NST>
__global__ __launch_bounds__(1024) void k_tail_lds(const LevelDesc<T> *__restrict__ descs,
                                                   const TailArgs *__restrict__ args,
                                                   const int *__restrict__ act)
{
    extern __shared__ double sb[];
    const TailArgs &A = args[blockIdx.x];
    if (act && !act[A.d0]) return;
    if (!(A.lds & (sizeof(T) == 8 ? 1 : 2))) return;
    double *coarse = sb;
    T *gb0 = reinterpret_cast<T *>(sb + 4 * A.ncoarse);
    T *gb1 = gb0 + A.ngmax;
    T *V = gb1 + A.ngmax;
    int *gop = reinterpret_cast<int *>(V + A.nvals);
    uint32_t *tab32 = reinterpret_cast<uint32_t *>(gop + A.nints);
    const uint16_t *tab = reinterpret_cast<const uint16_t *>(tab32);
    const LevelDesc<T> *base = descs + A.d0;
    const int L = A.nlev;
    // the table image, kTabChunk words per thread fetched before they are stored
    constexpr int kTabChunk = 8;
    for (int i0 = threadIdx.x; i0 < A.tab_words; i0 += kTabChunk * blockDim.x) {
        uint32_t w[kTabChunk];
#pragma unroll
        for (int k = 0; k < kTabChunk; ++k) w[k] = A.tab[min(i0 + k * (int)blockDim.x, A.tab_words - 1)];
#pragma unroll
        for (int k = 0; k < kTabChunk; ++k)
            if (i0 + k * (int)blockDim.x < A.tab_words) tab32[i0 + k * blockDim.x] = w[k];
    }
    // every level's values: where each tail level has at most one active node per
    // thread, the node codes of all levels are fetched first, then all their values
    constexpr int kLev = 8;
    bool one_per_thread = L - A.l0 <= kLev;
    for (int l = A.l0; l < L; ++l) one_per_thread = one_per_thread && A.ll[l].na <= (int)blockDim.x;
    if (one_per_thread) {
        const int t = threadIdx.x;
        int code[kLev];
#pragma unroll
        for (int m = 0; m < kLev; ++m) {
            const int l = A.l0 + m;
            code[m] = 0;
            if (l < L) {
                const TailLevel &TL = A.lev[l];
                const int na = A.ll[l].na, nin = TL.nin0 + TL.nin1;
                if (t < na) code[m] = t < nin ? TL.in_ijk[t] : base[l].g_ijk[t - nin];
            }
        }
        T sv[kLev], cv[kLev];
        long long q0 = 0;
#pragma unroll
        for (int m = 0; m < kLev; ++m) {
            const int l = A.l0 + m;
            sv[m] = cv[m] = T(0);
            if (l < L && t < A.ll[l].na) {
                const LevelDesc<T> *D = base + l;
                int i, j, k;
                unpack_ijk(code[m], i, j, k);
                const long long q = sidx(DIM, D->n, D->Wp, D->cs, i, j, k);
                if (m == 0) q0 = q;
                sv[m] = D->s[q];
                cv[m] = D->c[q];
            }
        }
        if (t < A.ll[A.l0].na) {
            const LevelDesc<T> *D = base + A.l0;
            T *b = V + A.ll[A.l0].v;
            const int na = A.ll[A.l0].na;
            b[2 * na + t] = D->x_s[q0];
            b[3 * na + t] = D->x_c[q0];
            b[4 * na + t] = D->rhs_s[q0];
            b[5 * na + t] = D->rhs_c[q0];
        }
#pragma unroll
        for (int m = 0; m < kLev; ++m) {
            const int l = A.l0 + m;
            if (l < L && t < A.ll[l].na) {
                T *b = V + A.ll[l].v;
                b[t] = sv[m];
                b[A.ll[l].na + t] = cv[m];
            }
        }
    } else {
        for (int l = A.l0; l < L; ++l) {
            const LevelDesc<T> *D = base + l;
            const TailLevel &TL = A.lev[l];
            const TailLdsLevel &d = A.ll[l];
            T *b = V + d.v;
            const int na = d.na, nin = TL.nin0 + TL.nin1;
            for (int t = threadIdx.x; t < na; t += blockDim.x) {
                int i, j, k;
                unpack_ijk(t < nin ? TL.in_ijk[t] : D->g_ijk[t - nin], i, j, k);
                const long long q = sidx(DIM, D->n, D->Wp, D->cs, i, j, k);
                b[t] = D->s[q];
                b[na + t] = D->c[q];
                if (l == A.l0) {
                    b[2 * na + t] = D->x_s[q];
                    b[3 * na + t] = D->x_c[q];
                    b[4 * na + t] = D->rhs_s[q];
                    b[5 * na + t] = D->rhs_c[q];
                }
            }
        }
    }
    for (int l = A.l0; l < L; ++l) {
        const LevelDesc<T> *D = base + l;
        const TailLdsLevel &d = A.ll[l];
        T *b = V + d.v;
        // band slots that the extension does not reach stay zero, as in HBM; the
        // last slot is the zero read for inactive fine nodes
        for (int t = threadIdx.x; t <= d.nb; t += blockDim.x) b[8 * d.na + t] = T(0);
        if (l < L - 1 && D->go_ptr)
            for (int q = threadIdx.x; q <= D->ng; q += blockDim.x) gop[d.gop + q] = D->go_ptr[q];
    }
    __syncthreads();
    // the cycle over levels l0 .. L-1 without recursion, as in the HBM tail
    int l = A.l0;
    unsigned done = 0u;
    bool down = true;
    while (true) {
        if (down) {
            if (l == L - 1) {
                lds_coarse<T>(base + l, lds_level<T>(A, l, V, tab, gop), A.ainv, coarse);
                down = false;
                continue;
            }
            const LevelDesc<T> *D = base + l;
            const LdsLevel<T> Z = lds_level<T>(A, l, V, tab, gop);
            for (int it = 0; it < A.nu1; ++it) lds_smooth<T, DIM, NST>(D, A.lev[l], Z, gb0, gb1);
            lds_defect<T, DIM, NST>(D, Z);
            lds_band<T>(D, Z);
            lds_restrict<T, DIM, NST>(Z, lds_level<T>(A, l + 1, V, tab, gop));
            done &= ~(1u << l);
            ++l;
            continue;
        }
        if (l == A.l0) break;
        const int p = l - 1;
        if (A.gamma == 2 && l != L - 1 && !(done & (1u << p))) {
            done |= 1u << p;
            down = true;
            continue;
        }
        const LdsLevel<T> Z = lds_level<T>(A, p, V, tab, gop);
        lds_prolong<T, DIM>(Z, lds_level<T>(A, l, V, tab, gop));
        for (int it = 0; it < A.nu2; ++it) lds_smooth<T, DIM, NST>(base + p, A.lev[p], Z, gb0, gb1);
        l = p;
    }
    // the entry level's correction back to HBM
    {
        const LevelDesc<T> *D = base + A.l0;
        const TailLevel &TL = A.lev[A.l0];
        const TailLdsLevel &d = A.ll[A.l0];
        const T *b = V + d.v;
        const int na = d.na, nin = TL.nin0 + TL.nin1;
        for (int t = threadIdx.x; t < na; t += blockDim.x) {
            int i, j, k;
            unpack_ijk(t < nin ? TL.in_ijk[t] : D->g_ijk[t - nin], i, j, k);
            const long long q = sidx(DIM, D->n, D->Wp, D->cs, i, j, k);
            D->x_s[q] = b[2 * na + t];
            D->x_c[q] = b[3 * na + t];
        }
    }
}

template <typename T>
void launch_tail_lds(int dim, const LevelDesc<T> *d, const TailArgs *args, int nblocks, size_t shm, const Exec &x)
{
    if (nblocks <= 0) return;
    if (dim == 2) {
        static bool attr = false;
        if (!attr) {
            (void)hipFuncSetAttribute((const void *)k_tail_lds<T, 2, 9>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)kTailLdsMax);
            attr = true;
        }
        k_tail_lds<T, 2, 9><<<nblocks, 1024, shm, x.s>>>(d, args, x.act);
    } else {
        static bool attr = false;
        if (!attr) {
            (void)hipFuncSetAttribute((const void *)k_tail_lds<T, 3, 27>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)kTailLdsMax);
            attr = true;
        }
        k_tail_lds<T, 3, 27><<<nblocks, 1024, shm, x.s>>>(d, args, x.act);
    }
}

template void launch_tail_lds<double>(int, const LevelDesc<double> *, const TailArgs *, int, size_t,
                                      const Exec &);
template void launch_tail_lds<float>(int, const LevelDesc<float> *, const TailArgs *, int, size_t,
                                     const Exec &);

}  // namespace lsmg
