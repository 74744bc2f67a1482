// Hierarchy build kernels: node classification and compaction (section 3.3,
// eq. ghostdef, map M of eq. maprij), inside-row work segments, ghost geometry
// (eq. nij, the upwind stencil ST, the boundary point B by bisection and the
// weights of eq. JssD) and the tables of the boundary-defect extension used by
// the restriction (section 3.5.2).
//
// This file is compiled with -ffp-contract=off: the geometry is a discrete
// definition (which stencil nodes carry an exactly-zero weight, which side of
// the level set a bisection midpoint falls on), so it is evaluated with plain
// IEEE double operations in a fixed order.
#include <hip/hip_runtime.h>

#include <vector>

#include "lsmg_dev.hpp"
#include "lsmg_host.hpp"

namespace lsmg {

// ---------------------------------------------------------------------------
// level set on the coarser grids: injection phi_c(I) = phi_f(2 I)
// ---------------------------------------------------------------------------
__global__ void k_inject_phi(int dim, const double *__restrict__ pf, int nf, double *__restrict__ pc, int nc)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long nn = (long long)nc * nc * (dim == 3 ? nc : 1);
    if (g >= nn) return;
    const int i = (int)(g % nc), j = (int)((g / nc) % nc), k = dim == 3 ? (int)(g / ((long long)nc * nc)) : 0;
    const long long gf = (long long)(2 * i) + (long long)nf * ((long long)(2 * j) + (long long)nf * (2 * k));
    pc[g] = pf[gf];
}

// ---------------------------------------------------------------------------
// classification: inside where phi < 0; ghost where not inside and an axis
// neighbour is inside; an inside node on the box edge is a geometry error
// ---------------------------------------------------------------------------
__global__ void k_classify(int dim, const double *__restrict__ phi, int n, int Wp, long long cs,
                           uint8_t *__restrict__ type, uint8_t *__restrict__ fin, uint8_t *__restrict__ fgh,
                           int *__restrict__ err)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nn = (long long)n * n * (dim == 3 ? n : 1);
    if (g >= nn) return;
    int id[3] = {(int)(g % n), (int)((g / n) % n), dim == 3 ? (int)(g / ((long long)n * n)) : 0};
    const bool inside = phi[g] < 0.0;
    bool ghost = false;
    if (inside) {
        for (int a = 0; a < dim; ++a)
            if (id[a] == 0 || id[a] == n - 1) atomicOr(err, 1);
    } else {
        long long st = 1;
        for (int a = 0; a < dim; ++a) {
            if (id[a] > 0 && phi[g - st] < 0.0) ghost = true;
            if (id[a] < n - 1 && phi[g + st] < 0.0) ghost = true;
            st *= n;
        }
    }
    const uint8_t t = inside ? kIn : (ghost ? kGhost : kOut);
    type[sidx(dim, n, Wp, cs, id[0], id[1], id[2])] = t;
    fin[g] = inside;
    fgh[g] = ghost;
}

// ---------------------------------------------------------------------------
// ordered stream compaction of a byte flag array
// ---------------------------------------------------------------------------
constexpr int kTileThreads = 256, kTilePer = 16, kTile = kTileThreads * kTilePer;

__global__ __launch_bounds__(kTileThreads) void k_tile_count(const uint8_t *__restrict__ f, long long N,
                                                             int64_t *__restrict__ counts)
{
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kTilePer;
    int c = 0;
    for (int e = 0; e < kTilePer; ++e)
        if (base + e < N) c += f[base + e] != 0;
    __shared__ int sh[kTileThreads];
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = kTileThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = sh[0];
}

// exclusive scan of M int64 values in place by one 1024-thread workgroup; total in a[M]
__global__ __launch_bounds__(1024) void k_scan_single(int64_t *__restrict__ a, long long M)
{
    __shared__ int64_t sh[1024];
    const int t = threadIdx.x;
    const long long chunk = (M + 1023) / 1024;
    const long long b = t * chunk, e = b + chunk < M ? b + chunk : M;
    int64_t s = 0;
    for (long long i = b; i < e; ++i) s += a[i];
    sh[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int64_t run = t > 0 ? sh[t - 1] : 0;
    for (long long i = b; i < e; ++i) {
        const int64_t v = a[i];
        a[i] = run;
        run += v;
    }
    if (t == 1023) a[M] = sh[1023];
}

__global__ __launch_bounds__(kTileThreads) void k_tile_emit(const uint8_t *__restrict__ f, long long N,
                                                            const int64_t *__restrict__ offs, int64_t *__restrict__ out)
{
    const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kTilePer;
    int c = 0;
    for (int e = 0; e < kTilePer; ++e)
        if (base + e < N) c += f[base + e] != 0;
    __shared__ int sh[kTileThreads];
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < kTileThreads; off <<= 1) {
        int v = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    long long pos = offs[blockIdx.x] + (threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0);
    for (int e = 0; e < kTilePer; ++e)
        if (base + e < N && f[base + e]) out[pos++] = base + e;
}

long long compact_scratch_size(long long N) { return (N + kTile - 1) / kTile + 1; }

int compact_flags(const uint8_t *flags, long long N, int64_t *out, int64_t *scratch, int nscratch, hipStream_t s)
{
    const long long nt = (N + kTile - 1) / kTile;
    if (nt + 1 > nscratch || N <= 0) return N <= 0 ? 0 : -1;
    k_tile_count<<<(unsigned)nt, kTileThreads, 0, s>>>(flags, N, scratch);
    k_scan_single<<<1, 1024, 0, s>>>(scratch, nt);
    if (out) k_tile_emit<<<(unsigned)nt, kTileThreads, 0, s>>>(flags, N, scratch, out);
    int64_t total = 0;
    if (hipMemcpyAsync(&total, scratch + nt, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    return (int)total;
}

// compact index -> storage index, and storage -> compact
__global__ void k_c2s(int dim, const int64_t *__restrict__ c2g, int na, int n, int Wp, long long cs,
                      int *__restrict__ c2s, int *__restrict__ cmap)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= na) return;
    const long long g = c2g[r];
    const int i = (int)(g % n), j = (int)((g / n) % n), k = dim == 3 ? (int)(g / ((long long)n * n)) : 0;
    const long long q = sidx(dim, n, Wp, cs, i, j, k);
    c2s[r] = (int)q;
    cmap[q] = r;
}

// ---------------------------------------------------------------------------
// work segments of inside nodes: per (colour, row) every maximal run of
// consecutive inside positions, cut into pieces of at most 64, so a segment
// holds inside nodes only
// ---------------------------------------------------------------------------
// type of position p of a row of one colour
struct RowType {
    const uint8_t *type;
    int dim, n, Wp, j, k, colour;
    long long cs, base;
    __device__ RowType(const uint8_t *t, int dim_, int n_, int Wp_, long long cs_, int colour_, long long row)
        : type(t), dim(dim_), n(n_), Wp(Wp_), colour(colour_), cs(cs_)
    {
        k = dim == 3 ? (int)(row / n) : 0;
        j = (int)(row - (long long)k * n);
        base = colour * cs + row * Wp;
    }
    __device__ uint8_t operator[](int p) const
    {
        return dim == 3 ? type[sidx3(n, Wp, cs, colour, p, j, k)] : type[base + p];
    }
};

__global__ void k_seg_count(const uint8_t *__restrict__ type, int dim, int n, long long rows, int Wp, long long cs,
                            int64_t *__restrict__ cnt)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * rows) return;
    const long long colour = t / rows, row = t - colour * rows;
    const RowType rp(type, dim, n, Wp, cs, (int)colour, row);
    long long c = 0;
    int p = 0;
    while (p < Wp) {
        if (rp[p] != kIn) { ++p; continue; }
        int e = p;
        while (e < Wp && rp[e] == kIn) ++e;
        c += (e - p + kWave - 1) / kWave;
        p = e;
    }
    cnt[t] = c;
}

__global__ void k_seg_emit(const uint8_t *__restrict__ type, int dim, int n, long long rows, int Wp, long long cs,
                           const int64_t *__restrict__ offs, int desc, int4 *__restrict__ items)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * rows) return;
    const long long colour = t / rows, row = t - colour * rows;
    const RowType rp(type, dim, n, Wp, cs, (int)colour, row);
    long long o = offs[t];
    int p = 0;
    while (p < Wp) {
        if (rp[p] != kIn) { ++p; continue; }
        int e = p;
        while (e < Wp && rp[e] == kIn) ++e;
        for (int b = p; b < e; b += kWave) items[o++] = make_int4((desc << 2) | (int)colour, (int)row, b, b + kWave < e ? b + kWave : e);
        p = e;
    }
}

// packed coordinates i | j << 11 | k << 22 of the inside nodes of one colour,
// in lexicographic order
__global__ void k_colour_flags(const int64_t *__restrict__ c2g, int ni, int n, int dim, int colour,
                               uint8_t *__restrict__ flags)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ni) return;
    const long long g = c2g[r];
    const int i = (int)(g % n), j = (int)((g / n) % n), k = dim == 3 ? (int)(g / ((long long)n * n)) : 0;
    flags[r] = ((i + j + k) & 1) == colour;
}

__global__ void k_pack_ijk(const int64_t *__restrict__ c2g, const int64_t *__restrict__ sel, int cnt, int n, int dim,
                           int *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const long long g = c2g[sel[t]];
    const int i = (int)(g % n), j = (int)((g / n) % n), k = dim == 3 ? (int)(g / ((long long)n * n)) : 0;
    out[t] = i | (j << 11) | (k << 22);
}

int build_inside_lists(int dim, const int64_t *c2g, int ni, int n, int *out, int *count, int64_t *scratch,
                       int nscratch, const DevMem &mem, hipStream_t s)
{
    count[0] = count[1] = 0;
    if (ni <= 0) return 0;
    uint8_t *flags = (uint8_t *)mem.get(ni);
    int64_t *sel = (int64_t *)mem.get(sizeof(int64_t) * ni);
    if (!flags || !sel) {
        mem.put(flags);
        mem.put(sel);
        return -1;
    }
    int off = 0;
    for (int colour = 0; colour < 2; ++colour) {
        k_colour_flags<<<(ni + 255) / 256, 256, 0, s>>>(c2g, ni, n, dim, colour, flags);
        const int c = compact_flags(flags, ni, sel, scratch, nscratch, s);
        if (c < 0) { off = -1; break; }
        if (c > 0) k_pack_ijk<<<(c + 255) / 256, 256, 0, s>>>(c2g, sel, c, n, dim, out + off);
        count[colour] = c;
        off += c;
    }
    (void)hipStreamSynchronize(s);
    mem.put(flags);
    mem.put(sel);
    return off < 0 ? -1 : 0;
}

void build_segments(int dim, const uint8_t *type, int n, int Wp, long long rows, long long cs, int desc,
                    int4 **out_items, int *out_count, const DevMem &mem, hipStream_t s)
{
    out_items[0] = out_items[1] = nullptr;
    out_count[0] = out_count[1] = 0;
    int64_t *cnt = (int64_t *)mem.get(sizeof(int64_t) * (2 * rows + 1));
    if (!cnt) return;
    const unsigned nb = (unsigned)((2 * rows + 255) / 256);
    k_seg_count<<<nb, 256, 0, s>>>(type, dim, n, rows, Wp, cs, cnt);
    // per-colour totals come from the exclusive scan at rows and 2 rows
    k_scan_single<<<1, 1024, 0, s>>>(cnt, 2 * rows);
    int64_t h[2] = {0, 0};
    (void)hipMemcpyAsync(&h[0], cnt + rows, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(&h[1], cnt + 2 * rows, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    const long long total = h[1];
    int4 *items = total > 0 ? (int4 *)mem.get(sizeof(int4) * total) : nullptr;
    if (items) {
        k_seg_emit<<<nb, 256, 0, s>>>(type, dim, n, rows, Wp, cs, cnt, desc, items);
        (void)hipStreamSynchronize(s);
        out_items[0] = items;
        out_items[1] = items + h[0];
        out_count[0] = (int)h[0];
        out_count[1] = (int)(total - h[0]);
    }
    (void)hipStreamSynchronize(s);
    mem.put(cnt);
}

// ---------------------------------------------------------------------------
// ghost geometry (section 3.3): normal by central differences (one-sided at
// the box edge), upwind stencil ST, boundary point B by full-precision
// bisection of the biquadratic (triquadratic) interpolant of phi on the
// segment P = G - 2 h n -> G, the tensor weights of eq. (JssD) and the order
// fallback (quadratic -> linear) where a nonzero weight falls on an inactive or
// out-of-box node; where no order is admissible, the ghost's own weight would be
// negative or B lies outside the stencil, the axis rule in 2-D and the constant
// rule in 3-D.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lag2(int k, double t)
{
    if (k == 0) return t * (1.0 + t) / 2.0;
    if (k == 1) return (1.0 - t) * (1.0 + t);
    return t * (t - 1.0) / 2.0;
}

__device__ __forceinline__ double lag1(int k, double t)
{
    if (k == 0) return t;
    if (k == 1) return 1.0 - t;
    return 0.0;
}

// d/dt of the quadratic weights (eq. intcoeffsN times h) and of the linear ones
__device__ __forceinline__ double dlag2(int k, double t)
{
    if (k == 0) return t + 0.5;
    if (k == 1) return -2.0 * t;
    return t - 0.5;
}

__device__ __forceinline__ double dlag1(int k)
{
    if (k == 0) return 1.0;
    if (k == 1) return -1.0;
    return 0.0;
}

// Neumann boundary row (section 3.6, eqs. BCsN, Neumanntilde, JccN): the
// derivative at B of the interpolant of s on ST along nr, the unit gradient at
// B of the interpolant of phi on ST (the central-difference normal where ST
// leaves the box, theta is out of range or that gradient vanishes);
// d/dx_a = (m_a / h) d/dt_a.  Rules in order: quadratic, bilinear gradient on
// the nodes k in {0,1}^d, one-sided differences s_G - s_{G - m_a e_a} on the
// axes with nr_a m_a > 0 whose inward neighbour is active.  A rule is taken
// only where its nonzero weights sit on active nodes and its own weight w_G
// lies in (0, 2 / tau_max] (eq. CFLcondN).  Returns false if no rule is
// admissible.  The operations follow the same order as the CPU reference,
// so that equal inputs give equal rows.
template <int DIM>
__device__ bool neumann_row(const double *phi, const uint8_t *type, const long long *stl, const long long *sts,
                            const bool *oob, bool any_oob, const double *th, bool bad, const int *m,
                            const double *nrm, double h, double *w, double *nr, int &order)
{
    constexpr int NST = DIM == 2 ? 9 : 27;
    for (int a = 0; a < DIM; ++a) nr[a] = nrm[a];
    if (!any_oob && !bad) {
        double gr[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < DIM; ++a) {
            double v = 0.0;
            for (int k = 0; k < NST; ++k) {
                int kk = k;
                double wk = 1.0;
                for (int b = 0; b < DIM; ++b) {
                    wk *= (b == a) ? dlag2(kk % 3, th[b]) : lag2(kk % 3, th[b]);
                    kk /= 3;
                }
                v += wk * phi[stl[k]];
            }
            gr[a] = (double)m[a] * v / h;
        }
        double g2 = 0.0;
        for (int a = 0; a < DIM; ++a) g2 += gr[a] * gr[a];
        if (g2 > 0.0) {
            const double gl = sqrt(g2);
            for (int a = 0; a < DIM; ++a) nr[a] = gr[a] / gl;
        }
    }
    const double wmax = DIM == 2 ? 3.0 / (sqrt(2.0) * h) : 3.0 * sqrt(3.0) / (2.0 * h);
    for (int o = 2; o >= 1 && !bad; --o) {
        for (int k = 0; k < NST; ++k) {
            double v = 0.0;
            for (int a = 0; a < DIM; ++a) {
                int kk = k;
                double wk = 1.0;
                for (int b = 0; b < DIM; ++b) {
                    const int kb = kk % 3;
                    if (o == 2) wk *= (b == a) ? dlag2(kb, th[b]) : lag2(kb, th[b]);
                    else wk *= (b == a) ? dlag1(kb) : lag1(kb, th[b]);
                    kk /= 3;
                }
                v += nr[a] * (double)m[a] * wk / h;
            }
            w[k] = v;
        }
        bool ok = w[0] > 0.0 && w[0] <= wmax;
        for (int k = 0; k < NST; ++k)
            if (w[k] != 0.0 && (oob[k] || type[sts[k]] == kOut)) ok = false;
        if (ok) {
            order = o;
            return true;
        }
    }
    for (int k = 0; k < NST; ++k) w[k] = 0.0;
    double wg = 0.0;
    for (int a = 0; a < DIM; ++a) {
        const int k = a == 0 ? 1 : (a == 1 ? 3 : 9);   // stencil entry of G - m_a e_a
        const double c = nr[a] * (double)m[a];
        if (!(c > 0.0) || oob[k] || type[sts[k]] == kOut) continue;
        w[k] = -c / h;
        wg += c / h;
    }
    order = 0;
    if (!(wg > 0.0)) return false;
    w[0] = wg;
    return true;
}

template <int DIM>
__device__ double phi_interp(const double *phi, const long long *stl, const int *gi, const int *m, const double *X,
                             double lo, double h)
{
    constexpr int NST = DIM == 2 ? 9 : 27;
    double t[3];
    for (int a = 0; a < DIM; ++a) t[a] = (double)m[a] * (X[a] - (lo + (double)(gi[a] - m[a]) * h)) / h;
    double v = 0.0;
    for (int k = 0; k < NST; ++k) {
        int kk = k;
        double wk = 1.0;
        for (int a = 0; a < DIM; ++a) {
            wk *= lag2(kk % 3, t[a]);
            kk /= 3;
        }
        v += wk * phi[stl[k]];
    }
    return v;
}

// axis rule (2-D), taken where the row would otherwise take the constant rule:
// among the inside axis neighbours G + sgn e_a (axes in order, sgn = -1 then
// +1), the line giving the ghost the largest self-weight; on it the stencil is
// oriented so that G - m_a e_a is that neighbour, B is the zero of the quadratic
// interpolant of phi through G and the next two nodes of the line (linear
// through two where the third leaves the box), bisected in t in (0, 1], and
// theta = t on the axis, 1 on the other.  The weights are those of the 1-D
// quadratic (linear where the third node is inactive).  Same operations in
// the same order as the CPU reference.  Returns false if G has no inside axis
// neighbour.
template <int DIM>
__device__ bool axis_row(const double *phi, const uint8_t *type, long long g, const int *gi, int n, int Wp,
                         long long cs, double lo, double h, int *m, long long *stl, long long *sts, bool *oob,
                         double *Bp, double *th, double *w, int &order)
{
    constexpr int NST = DIM == 2 ? 9 : 27;
    int best = -1, bsgn = 0;
    double bw = -1.0, bt = 0.0;
    long long sa = 1;
    for (int a = 0; a < DIM; ++a, sa *= n)
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            const int k1 = gi[a] + sgn, k2 = gi[a] + 2 * sgn;
            if (k1 < 0 || k1 >= n || !(phi[g + sgn * sa] < 0.0)) continue;
            const bool q2 = k2 >= 0 && k2 < n;
            const double f0 = phi[g], f1 = phi[g + sgn * sa], f2 = q2 ? phi[g + 2 * sgn * sa] : 0.0;
            double tlo = 0.0, thi = 1.0;
            for (int it = 0; it < 200; ++it) {
                const double t = 0.5 * (tlo + thi);
                if (t <= tlo || t >= thi) break;
                const double v = q2 ? lag2(0, t) * f0 + lag2(1, t) * f1 + lag2(2, t) * f2 : t * f0 + (1.0 - t) * f1;
                if (v < 0.0) tlo = t;
                else thi = t;
            }
            bool act2 = false;
            if (q2) {
                int id[3] = {gi[0], gi[1], gi[2]};
                id[a] = k2;
                act2 = type[sidx(DIM, n, Wp, cs, id[0], id[1], id[2])] != kOut;
            }
            const double wg = act2 ? lag2(0, thi) : lag1(0, thi);
            if (wg > bw) {
                bw = wg;
                best = a;
                bsgn = sgn;
                bt = thi;
            }
        }
    if (best < 0) return false;
    m[best] = -bsgn;
    const long long g0 = stl[0];
    const long long gs = sts[0];
    for (int k = 0; k < NST; ++k) {
        int kk = k, id[3] = {0, 0, 0};
        bool o = false;
        for (int a = 0; a < DIM; ++a) {
            id[a] = gi[a] - m[a] * (kk % 3);
            kk /= 3;
            if (id[a] < 0 || id[a] >= n) o = true;
        }
        oob[k] = o;
        stl[k] = o ? g0 : (long long)id[0] + (long long)n * ((long long)id[1] + (long long)n * id[2]);
        sts[k] = o ? gs : sidx(DIM, n, Wp, cs, id[0], id[1], id[2]);
    }
    for (int a = 0; a < DIM; ++a) {
        Bp[a] = lo + (double)gi[a] * h;
        th[a] = 1.0;
    }
    th[best] = bt;
    Bp[best] = (lo + (double)gi[best] * h) - (double)m[best] * h * (1.0 - bt);
    order = 2;
    for (int k = 0; k < NST; ++k) {
        int kk = k;
        double wk = 1.0;
        for (int a = 0; a < DIM; ++a) {
            wk *= lag2(kk % 3, th[a]);
            kk /= 3;
        }
        w[k] = wk;
    }
    for (int k = 0; k < NST; ++k)
        if (w[k] != 0.0 && (oob[k] || type[sts[k]] == kOut)) order = 1;
    if (order == 1)
        for (int k = 0; k < NST; ++k) {
            int kk = k;
            double wk = 1.0;
            for (int a = 0; a < DIM; ++a) {
                wk *= lag1(kk % 3, th[a]);
                kk /= 3;
            }
            w[k] = wk;
        }
    return true;
}

template <int DIM>
__global__ void k_ghost_geometry(int level, int bc, const double *__restrict__ phi, const uint8_t *__restrict__ type,
                                 const int64_t *__restrict__ c2g_gh, const int *__restrict__ cmap, int ni, int ng, int n,
                                 int Wp, long long cs, double lo, double h, int *__restrict__ g_idx,
                                 int *__restrict__ g_ijk, int *__restrict__ g_st, int *__restrict__ g_stg,
                                 int *__restrict__ g_stc, double *__restrict__ g_w, double *__restrict__ g_B,
                                 double *__restrict__ g_nrm, double *__restrict__ g_nrow,
                                 int *__restrict__ g_order, int *__restrict__ g_bfall, int *__restrict__ err)
{
    constexpr int NST = DIM == 2 ? 9 : 27;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ng) return;
    const long long g = c2g_gh[q];
    int gi[3] = {(int)(g % n), (int)((g / n) % n), DIM == 3 ? (int)(g / ((long long)n * n)) : 0};
    double G[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < DIM; ++a) G[a] = lo + (double)gi[a] * h;
    // normal
    double nt[3] = {0.0, 0.0, 0.0}, nrm[3] = {0.0, 0.0, 0.0};
    long long sa = 1;
    for (int a = 0; a < DIM; ++a) {
        if (gi[a] > 0 && gi[a] < n - 1) nt[a] = (phi[g + sa] - phi[g - sa]) / (2.0 * h);
        else if (gi[a] == 0) nt[a] = (phi[g + sa] - phi[g]) / h;
        else nt[a] = (phi[g] - phi[g - sa]) / h;
        sa *= n;
    }
    double len2 = 0.0;
    for (int a = 0; a < DIM; ++a) len2 += nt[a] * nt[a];
    const double len = sqrt(len2);
    int m[3] = {1, 1, 1};
    if (len > 0.0)
        for (int a = 0; a < DIM; ++a) nrm[a] = nt[a] / len;
    for (int a = 0; a < DIM; ++a) m[a] = nrm[a] >= 0.0 ? 1 : -1;
    // upwind stencil
    long long stl[NST];
    long long sts[NST];
    bool oob[NST];
    bool any_oob = false;
    const long long gs = sidx(DIM, n, Wp, cs, gi[0], gi[1], gi[2]);
    for (int k = 0; k < NST; ++k) {
        int kk = k, id[3] = {0, 0, 0};
        bool o = false;
        for (int a = 0; a < DIM; ++a) {
            id[a] = gi[a] - m[a] * (kk % 3);
            kk /= 3;
            if (id[a] < 0 || id[a] >= n) o = true;
        }
        oob[k] = o;
        any_oob |= o;
        stl[k] = o ? g : (long long)id[0] + (long long)n * ((long long)id[1] + (long long)n * id[2]);
        sts[k] = o ? gs : sidx(DIM, n, Wp, cs, id[0], id[1], id[2]);
    }
    // boundary point
    double Bp[3] = {G[0], G[1], G[2]};
    int bfall = 0;
    if (len > 0.0 && any_oob) {
        bfall = 1;
        for (int a = 0; a < DIM; ++a) Bp[a] = G[a] - phi[g] * nt[a] / len2;
    } else if (len > 0.0) {
        double P[3] = {0.0, 0.0, 0.0}, X[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < DIM; ++a) P[a] = G[a] - 2.0 * h * nrm[a];
        const double f0 = phi_interp<DIM>(phi, stl, gi, m, P, lo, h);
        if (f0 < 0.0) {
            double alo = 0.0, ahi = 1.0;
            for (int it = 0; it < 200; ++it) {
                const double am = 0.5 * (alo + ahi);
                if (am <= alo || am >= ahi) break;
                for (int a = 0; a < DIM; ++a) X[a] = P[a] + am * (G[a] - P[a]);
                if (phi_interp<DIM>(phi, stl, gi, m, X, lo, h) < 0.0) alo = am;
                else ahi = am;
            }
            for (int a = 0; a < DIM; ++a) Bp[a] = P[a] + ahi * (G[a] - P[a]);
        } else {
            bfall = 1;
            for (int a = 0; a < DIM; ++a) Bp[a] = G[a] - phi[g] * nt[a] / len2;
        }
    }
    double th[3] = {1.0, 1.0, 1.0};
    for (int a = 0; a < DIM; ++a) th[a] = (double)m[a] * (Bp[a] - (lo + (double)(gi[a] - m[a]) * h)) / h;
    bool bad = false;
    for (int a = 0; a < DIM; ++a)
        if (!(th[a] >= -1.0 && th[a] <= 2.0)) bad = true;
    // theta outside [-1, 2] (B from the first-order projection far from G, e.g. at a
    // crease of the level set): the constant rule below, on every level
    double w[NST];
    double nr[3] = {nrm[0], nrm[1], nrm[2]};
    int order = 2;
    if (bc == 1) {
        if (!neumann_row<DIM>(phi, type, stl, sts, oob, any_oob, th, bad, m, nrm, h, w, nr, order)) atomicOr(err, 2);
    } else if (!bad) {
        for (int k = 0; k < NST; ++k) {
            int kk = k;
            double wk = 1.0;
            for (int a = 0; a < DIM; ++a) {
                wk *= lag2(kk % 3, th[a]);
                kk /= 3;
            }
            w[k] = wk;
        }
        for (int k = 0; k < NST; ++k)
            if (w[k] != 0.0 && (oob[k] || type[sts[k]] == kOut)) order = 1;
        if (order == 1) {
            for (int k = 0; k < NST; ++k) {
                int kk = k;
                double wk = 1.0;
                for (int a = 0; a < DIM; ++a) {
                    wk *= lag1(kk % 3, th[a]);
                    kk /= 3;
                }
                w[k] = wk;
            }
            for (int k = 0; k < NST; ++k)
                if (w[k] != 0.0 && (oob[k] || type[sts[k]] == kOut)) order = 0;
        }
    } else {
        order = 0;
    }
    if (bc != 1) {
        // a negative weight of the ghost itself (theta outside [0, 1] on an axis)
        // cannot meet eq. CFLcond with 0 < tau < 1: in 2-D the row takes the axis
        // rule, in 3-D (and without an inside axis neighbour) the constant rule
        if (!bad && w[0] < 0.0) order = 0;
        if (order == 0 && DIM == 2 &&
            axis_row<DIM>(phi, type, g, gi, n, Wp, cs, lo, h, m, stl, sts, oob, Bp, th, w, order))
            bfall = 2;
        else if (order == 0)
            for (int k = 0; k < NST; ++k) w[k] = k == 0 ? 1.0 : 0.0;
    }
    g_idx[q] = (int)gs;
    g_ijk[q] = gi[0] | (gi[1] << 11) | (gi[2] << 22);
    for (int k = 0; k < NST; ++k) {
        // zero-weight entries point at the ghost itself, which is always active
        const long long tgt = w[k] != 0.0 ? sts[k] : gs;
        const int cm = cmap[sts[k]];
        g_st[k * ng + q] = (int)tgt;
        g_stg[k * ng + q] = (w[k] != 0.0 && cm >= ni) ? cm - ni : -1;
        g_stc[k * ng + q] = cm;
        g_w[k * ng + q] = w[k];
    }
    for (int a = 0; a < DIM; ++a) {
        g_B[q * DIM + a] = Bp[a];
        g_nrm[q * DIM + a] = nrm[a];
        g_nrow[q * DIM + a] = nr[a];
    }
    g_order[q] = order;
    g_bfall[q] = bfall;
}

// ---------------------------------------------------------------------------
// boundary band: inactive fine nodes in the 3^d neighbourhood of the fine
// centre 2I of every coarse ghost I
// ---------------------------------------------------------------------------
__global__ void k_band_mark(int dim, const int64_t *__restrict__ c2g_cg, int ngc, int nc,
                            const uint8_t *__restrict__ ftype, int nf, int fWp, long long fcs,
                            uint8_t *__restrict__ flag)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ngc) return;
    const long long g = c2g_cg[q];
    const int ci[3] = {(int)(g % nc), (int)((g / nc) % nc), dim == 3 ? (int)(g / ((long long)nc * nc)) : 0};
    const int nst = dim == 3 ? 27 : 9;
    for (int k = 0; k < nst; ++k) {
        int kk = k, id[3] = {0, 0, 0};
        bool in = true;
        for (int a = 0; a < dim; ++a) {
            id[a] = 2 * ci[a] + kk % 3 - 1;
            kk /= 3;
            if (id[a] < 0 || id[a] >= nf) in = false;
        }
        if (!in) continue;
        if (ftype[sidx(dim, nf, fWp, fcs, id[0], id[1], id[2])] == kOut)
            flag[(long long)id[0] + (long long)nf * ((long long)id[1] + (long long)nf * id[2])] = 1;
    }
}

__global__ void k_fill_bandid(const int64_t *__restrict__ band, int nb, int *__restrict__ bandid)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) bandid[band[b]] = b;
}

// upwind neighbours q - m_a e_a of each band node that are ghosts or band nodes,
// with weights |n_a| of the central-difference normal at the band node
__global__ void k_band_geometry(int dim, const double *__restrict__ phi, const int64_t *__restrict__ band, int nb,
                                const uint8_t *__restrict__ type, const int *__restrict__ bandid, int n, int Wp,
                                long long cs, double h, int *__restrict__ up_s, int *__restrict__ up_b,
                                double *__restrict__ up_w, int *__restrict__ b_idx)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const long long g = band[b];
    const int gi[3] = {(int)(g % n), (int)((g / n) % n), dim == 3 ? (int)(g / ((long long)n * n)) : 0};
    double nt[3] = {0.0, 0.0, 0.0};
    long long sa = 1;
    for (int a = 0; a < dim; ++a) {
        if (gi[a] > 0 && gi[a] < n - 1) nt[a] = (phi[g + sa] - phi[g - sa]) / (2.0 * h);
        else if (gi[a] == 0) nt[a] = (phi[g + sa] - phi[g]) / h;
        else nt[a] = (phi[g] - phi[g - sa]) / h;
        sa *= n;
    }
    double len2 = 0.0;
    for (int a = 0; a < dim; ++a) len2 += nt[a] * nt[a];
    const double len = sqrt(len2);
    b_idx[b] = (int)sidx(dim, n, Wp, cs, gi[0], gi[1], gi[2]);
    sa = 1;
    for (int a = 0; a < dim; ++a) {
        const double na = len > 0.0 ? nt[a] / len : 0.0;
        const int ma = na >= 0.0 ? 1 : -1;
        int up[3] = {gi[0], gi[1], gi[2]};
        up[a] -= ma;
        up_s[a * nb + b] = -1;
        up_b[a * nb + b] = -1;
        up_w[a * nb + b] = 0.0;
        if (up[a] >= 0 && up[a] < n) {
            const long long gu = g - ma * sa;
            const long long su = sidx(dim, n, Wp, cs, up[0], up[1], up[2]);
            const int bid = bandid[gu];
            if (type[su] == kGhost || bid >= 0) {
                up_s[a * nb + b] = (int)su;
                up_b[a * nb + b] = type[su] == kGhost ? -1 : bid;
                up_w[a * nb + b] = fabs(na);
            }
        }
        sa *= n;
    }
}

// one layer of the extension: an unassigned band node with assigned upwind
// neighbours (ghosts, or band nodes of earlier layers) becomes the normalised
// |n_a|-weighted combination of them, composed down to ghost sources
__global__ void k_band_layer(int dim, int layer, int nb, int maxc, const int *__restrict__ up_s,
                             const int *__restrict__ up_b, const double *__restrict__ up_w, int *__restrict__ blayer,
                             int *__restrict__ b_cnt, int *__restrict__ b_src, double *__restrict__ b_wt)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb || blayer[b] != 0) return;
    bool asg[3] = {false, false, false};
    double ws = 0.0;
    int cnt = 0;
    for (int a = 0; a < dim; ++a) {
        const int su = up_s[a * nb + b];
        if (su < 0) continue;
        const int bb = up_b[a * nb + b];
        bool ok = bb < 0;
        if (!ok) {
            const int lb = blayer[bb];
            ok = lb > 0 && lb < layer;
        }
        if (!ok) continue;
        asg[a] = true;
        ws += up_w[a * nb + b];
        ++cnt;
    }
    if (cnt == 0) return;
    int e = 0;
    for (int a = 0; a < dim; ++a) {
        if (!asg[a]) continue;
        const double wa = ws > 0.0 ? up_w[a * nb + b] / ws : 1.0 / cnt;
        const int bb = up_b[a * nb + b];
        if (bb < 0) {
            if (e < maxc) {
                b_src[e * nb + b] = up_s[a * nb + b];
                b_wt[e * nb + b] = wa;
                ++e;
            }
        } else {
            const int cb = b_cnt[bb];
            for (int j = 0; j < cb && e < maxc; ++j) {
                b_src[e * nb + b] = b_src[j * nb + bb];
                b_wt[e * nb + b] = wa * b_wt[j * nb + bb];
                ++e;
            }
        }
    }
    b_cnt[b] = e;
    blayer[b] = layer;
}

__global__ void k_band_ext(int nb, const int *__restrict__ b_idx, const int *__restrict__ blayer, uint8_t *ext)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb && blayer[b] > 0) ext[b_idx[b]] = 1;
}

__global__ void k_ghost_ext(int ng, const int *__restrict__ g_idx, uint8_t *ext)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < ng) ext[g_idx[q]] = 1;
}

template <typename D, typename S>
__global__ void k_convert(D *__restrict__ dst, const S *__restrict__ src, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (D)src[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

void launch_inject_phi(int dim, const double *pf, int nf, double *pc, int nc, hipStream_t s)
{
    const long long nn = (long long)nc * nc * (dim == 3 ? nc : 1);
    k_inject_phi<<<blocks(nn), 256, 0, s>>>(dim, pf, nf, pc, nc);
}

void launch_classify(int dim, const double *phi, int n, int Wp, long long cs, uint8_t *type, uint8_t *fin,
                     uint8_t *fgh, int *err, hipStream_t s)
{
    const long long nn = (long long)n * n * (dim == 3 ? n : 1);
    k_classify<<<blocks(nn), 256, 0, s>>>(dim, phi, n, Wp, cs, type, fin, fgh, err);
}

void launch_c2s(int dim, const int64_t *c2g, int na, int n, int Wp, long long cs, int *c2s, int *cmap, hipStream_t s)
{
    if (na > 0) k_c2s<<<blocks(na), 256, 0, s>>>(dim, c2g, na, n, Wp, cs, c2s, cmap);
}

void launch_ghost_geometry(int dim, int level, int bc, const double *phi, const uint8_t *type, const int64_t *c2g_gh,
                           const int *cmap, int ni, int ng, int n, int Wp, long long cs, double lo, double h, int *g_idx,
                           int *g_ijk, int *g_st, int *g_stg, int *g_stc, double *g_w, double *g_B, double *g_nrm,
                           double *g_nrow, int *g_order, int *g_bfall, int *err, hipStream_t s)
{
    if (ng <= 0) return;
    if (dim == 2)
        k_ghost_geometry<2><<<blocks(ng, 64), 64, 0, s>>>(level, bc, phi, type, c2g_gh, cmap, ni, ng, n, Wp, cs, lo, h,
                                                          g_idx, g_ijk, g_st, g_stg, g_stc, g_w, g_B, g_nrm, g_nrow,
                                                          g_order, g_bfall, err);
    else
        k_ghost_geometry<3><<<blocks(ng, 64), 64, 0, s>>>(level, bc, phi, type, c2g_gh, cmap, ni, ng, n, Wp, cs, lo, h,
                                                          g_idx, g_ijk, g_st, g_stg, g_stc, g_w, g_B, g_nrm, g_nrow,
                                                          g_order, g_bfall, err);
}

void launch_band_mark(int dim, const int64_t *c2g_cg, int ngc, int nc, const uint8_t *ftype, int nf, int fWp,
                      long long fcs, uint8_t *flag, hipStream_t s)
{
    if (ngc > 0) k_band_mark<<<blocks(ngc), 256, 0, s>>>(dim, c2g_cg, ngc, nc, ftype, nf, fWp, fcs, flag);
}

void launch_fill_bandid(const int64_t *band, int nb, int *bandid, hipStream_t s)
{
    if (nb > 0) k_fill_bandid<<<blocks(nb), 256, 0, s>>>(band, nb, bandid);
}

void launch_band_geometry(int dim, const double *phi, const int64_t *band, int nb, const uint8_t *type,
                          const int *bandid, int n, int Wp, long long cs, double h, int *up_s, int *up_b,
                          double *up_w, int *b_idx, hipStream_t s)
{
    if (nb > 0)
        k_band_geometry<<<blocks(nb), 256, 0, s>>>(dim, phi, band, nb, type, bandid, n, Wp, cs, h, up_s, up_b, up_w,
                                                   b_idx);
}

void launch_band_layer(int dim, int layer, int nb, int maxc, const int *up_s, const int *up_b, const double *up_w,
                       int *blayer, int *b_cnt, int *b_src, double *b_wt, hipStream_t s)
{
    if (nb > 0)
        k_band_layer<<<blocks(nb), 256, 0, s>>>(dim, layer, nb, maxc, up_s, up_b, up_w, blayer, b_cnt, b_src, b_wt);
}

void launch_band_ext(int nb, const int *b_idx, const int *blayer, uint8_t *ext, hipStream_t s)
{
    if (nb > 0) k_band_ext<<<blocks(nb), 256, 0, s>>>(nb, b_idx, blayer, ext);
}

void launch_ghost_ext(int ng, const int *g_idx, uint8_t *ext, hipStream_t s)
{
    if (ng > 0) k_ghost_ext<<<blocks(ng), 256, 0, s>>>(ng, g_idx, ext);
}

template <typename D, typename S>
void launch_convert(D *dst, const S *src, long long n, hipStream_t s)
{
    if (n > 0) k_convert<D, S><<<blocks(n), 256, 0, s>>>(dst, src, n);
}
template void launch_convert<float, double>(float *, const double *, long long, hipStream_t);

}  // namespace lsmg
