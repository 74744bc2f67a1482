// Row arithmetic of the linearised Crank-Nicolson system (section 3.4), shared
// by every kernel that evaluates a row: the per-item kernels that read a level
// from HBM and the coarse tail that holds its levels in LDS call this same code
// on the same values, so they produce the same bits.
#pragma once

#include "lsmg_dev.hpp"

namespace lsmg {

// inside-row Jacobian (exact derivatives of eqs. FDs and FDc; the printed
// forms of eqs. JssI, JscI, JcsI, JccI are garbled)
template <typename T>
struct InsideRow {
    T ss_d, sc_d, cs_d, cc_d;   // diagonal 2x2 block P (eq. matrixP)
    T off_s;                    // sum over the axis neighbours of J^ss x_s + J^sc x_c
};

// the rows of an inside node from its (s, c) and (s, c, x_s, x_c) of its 2 DIM
// axis neighbours, ordered x-, x+, y-, y+[, z-, z+]
template <typename T, int DIM>
__device__ __forceinline__ InsideRow<T> inside_row_vals(const LevelDesc<T> *D, T sr, T cr, const T *se, const T *ce,
                                                        const T *xse, const T *xce)
{
    const T al = D->alpha, be = D->beta, kap = D->kap;
    const T phr = al * cr + be;
    T sum_ss = 0, sum_sc = 0, off = 0;
#pragma unroll
    for (int e = 0; e < 2 * DIM; ++e) {
        const T a_ss = (al * ce[e] + be) + phr;
        const T a_sc = sr - se[e];
        sum_ss += a_ss;
        sum_sc += a_sc;
        off += -kap * a_ss * xse[e] + kap * al * a_sc * xce[e];
    }
    InsideRow<T> R;
    R.ss_d = phr * D->dt_inv + D->ks_half * phr * cr + kap * sum_ss;
    R.sc_d = al * sr * D->dt_inv + D->ks_half * (al * sr * cr + phr * sr) + kap * al * sum_sc;
    R.cs_d = D->kc_half * phr * cr;
    R.cc_d = D->dt_inv + D->kc_half * (al * sr * cr + phr * sr);
    R.off_s = off;
    return R;
}

// c-row diagonal entries of a node (inside or ghost) from its (s, c)
template <typename T>
__device__ __forceinline__ void c_row_vals(const LevelDesc<T> *D, T sr, T cr, T &cs_d, T &cc_d)
{
    const T phr = D->alpha * cr + D->beta;
    cs_d = D->kc_half * phr * cr;
    cc_d = D->dt_inv + D->kc_half * (D->alpha * sr * cr + phr * sr);
}

// collective Gauss-Seidel update of an inside node (section 3.5.1): the 2x2
// block of eq. (matrixP) solved with the neighbours fixed
template <typename T>
__device__ __forceinline__ void block_solve(const InsideRow<T> &R, T rhs_s, T rhs_c, T &xs, T &xc)
{
    const T rs = rhs_s - R.off_s;
    const T rc = rhs_c;
    const T det = R.ss_d * R.cc_d - R.sc_d * R.cs_d;
    xs = (R.cc_d * rs - R.sc_d * rc) / det;
    xc = (R.ss_d * rc - R.cs_d * rs) / det;
}

// defect r = rhs - J x of an inside row pair
template <typename T>
__device__ __forceinline__ void inside_defect_vals(const InsideRow<T> &R, T rhs_s, T rhs_c, T xs, T xc, T &rs, T &rc)
{
    rs = rhs_s - (R.ss_d * xs + R.sc_d * xc + R.off_s);
    rc = rhs_c - (R.cs_d * xs + R.cc_d * xc);
}

// ghost c-row relaxation with the new delta s of the ghost (eq. RelGhost)
template <typename T>
__device__ __forceinline__ T ghost_c_update(T cs_d, T cc_d, T rhs_c, T ds, T xc)
{
    return xc + (rhs_c - (cs_d * ds + cc_d * xc)) / cc_d;
}

// restriction onto one coarse node (section 3.5.2, Fig. Neigh) from the 3^d fine
// neighbourhood (x fastest, centre at index 4 or 13): ex[k] marks the fine nodes
// the s-row excludes, act[k] the active ones, rs / rc their defects.  Modified
// full weighting per axis, [1,2,1]/4, [2,2,0]/4 if +1 is excluded, [0,2,2]/4 if
// -1 is, [0,4,0]/4 if both, tensor product, weight on excluded corners moved to
// the centre; the c-row takes full weighting renormalised over active nodes.
template <typename T, int DIM>
__device__ __forceinline__ void restrict_vals(uint8_t *ex, const uint8_t *act, const T *rs, const T *rc, T &out_s,
                                              T &out_c)
{
    constexpr int NST = DIM == 2 ? 9 : 27;
    constexpr int CEN = DIM == 2 ? 4 : 13;
    ex[CEN] = 0;
    T wa[3][3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int st = a == 0 ? 1 : (a == 1 ? 3 : 9);
        const bool em = ex[CEN - st], ep = ex[CEN + st];
        wa[a][0] = em ? T(0) : (ep ? T(0.5) : T(0.25));
        wa[a][1] = (em && ep) ? T(1) : T(0.5);
        wa[a][2] = ep ? T(0) : (em ? T(0.5) : T(0.25));
    }
    T vs = 0, wcen = 0, vc = 0, wcs = 0;
#pragma unroll
    for (int kk = 0; kk < NST; ++kk) {
        const int d0 = kk % 3, d1 = (kk / 3) % 3, d2 = kk / 9;
        T wk = wa[0][d0] * wa[1][d1];
        T wf = (d0 == 1 ? T(0.5) : T(0.25)) * (d1 == 1 ? T(0.5) : T(0.25));
        if (DIM == 3) {
            wk *= wa[2][d2];
            wf *= (d2 == 1 ? T(0.5) : T(0.25));
        }
        if (ex[kk]) wcen += wk;
        else vs += wk * rs[kk];
        if (act[kk]) {
            vc += wf * rc[kk];
            wcs += wf;
        }
    }
    vs += wcen * rs[CEN];
    out_s = vs;
    out_c = wcs > T(0) ? vc / wcs : T(0);
}

// Rows evaluated by a group of kRowGroup lanes (the coarse tail and the coarsest
// solve): lane sub sums the entries sub, sub + G, sub + 2G, ... of the row in
// order, fetching kRowChunk strides before summing them (entries past the row's
// end re-read its last entry and are dropped by a select); then the lanes' sums
// are added pairwise by xor shuffles, and every lane of the group gets the total.
// Every kernel that evaluates these rows uses this order, and the fused
// multiply-adds are written out (contraction left to the compiler may pair the
// products differently in different kernels), so they give the same bits.
constexpr int kRowGroup = 8;
constexpr int kRowChunk = 4;

// sum_q M[r][q] v[q] of one row
template <typename P>
__device__ __forceinline__ double group_row_dot(P row, const double *v, int na, int sub)
{
    double acc = 0.0;
    for (int q0 = sub; q0 < na; q0 += kRowChunk * kRowGroup) {
        double m[kRowChunk], x[kRowChunk];
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {
            const int q = min(q0 + k * kRowGroup, na - 1);
            m[k] = row[q];
            x[k] = v[q];
        }
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {
            const double t = fma(m[k], x[k], acc);
            acc = q0 + k * kRowGroup < na ? t : acc;
        }
    }
    for (int off = kRowGroup / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kRowGroup);
    return acc;
}

// one composed ghost-map row, sum_e a[e] gb1[col[e]] + b[e] gb0[col[e]] over e in
// [e0, e1) (the map's entries from HBM, the ghost values in LDS)
template <typename T, typename PC, typename PV>
__device__ __forceinline__ T group_ghost_row(PC col, PV a, PV b, const T *gb0, const T *gb1, int e0, int e1, int sub)
{
    T acc = 0;
    for (int e = e0 + sub; e < e1; e += kRowChunk * kRowGroup) {
        int c[kRowChunk];
        T av[kRowChunk], bv[kRowChunk];
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {
            const int ek = min(e + k * kRowGroup, e1 - 1);
            c[k] = col[ek];
            av[k] = a[ek];
            bv[k] = b[ek];
        }
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {
            const T t = acc + fma(av[k], gb1[c[k]], bv[k] * gb0[c[k]]);
            acc = e + k * kRowGroup < e1 ? t : acc;
        }
    }
    for (int off = kRowGroup / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kRowGroup);
    return acc;
}

}  // namespace lsmg
