// Internal device-side definitions of the lsmg GPU library (gfx950).
//
// Storage of a level: every per-node array is a full grid held in red/black
// split form.  Node (i, j[, k]) has colour c = (i + j + k) & 1, row
// r = j + n k and position p = i >> 1.
//   2-D: its storage index is c * cs + r * Wp + p, cs = n * Wp, with Wp >=
//   (n + 1) / 2 rounded up to 16 doubles (128 bytes).  A red or black half-sweep
//   reads and writes contiguous memory, and the four axis neighbours of a node
//   are the other colour in the same row (x) or at the same position in the rows
//   above and below (y).
//   3-D: each colour is stored in bricks of 32 consecutive values (one 128-byte
//   line in FP32, two in FP64) covering 2^kBP positions x 2^kBJ rows (y) x 2^kBK
//   planes (z), bricks in (position, y, z) order: a run of inside nodes along a
//   row then shares its lines with the runs of the next rows and planes instead
//   of ending in partial lines of its own (a row crosses a 3-D domain in short
//   runs).  Wp is the position count rounded up to 2^kBP, and cs = 32 x the
//   number of bricks of a colour.
//
// Work is described by lists of int4 work items, one 64-lane wavefront per
// item: x = (descriptor index << 2) | kind, then
//   kind 0 / 1: inside nodes of colour 0 / 1: in 2-D row y, positions [z, w);
//   in 3-D two consecutive bricks of the colour (see brick_lane);
//   kind 2: ghosts [z, w) of the level's ghost list;
//   kind 3: band nodes [z, w) of the level's boundary band.
// Descriptors of one hierarchy are contiguous by level (finest first), so the
// next coarser level of descriptor d is d + 1 and the next finer is d - 1.
// A batch of hierarchies concatenates their descriptor arrays; its work lists
// carry the rebased descriptor indices, and an optional array of per-descriptor
// flags lets a launch skip the items of domains that have already converged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// 3-D brick shape (log2 of positions and of rows per brick; planes take the rest of 32)
#ifndef LSMG_BRICK_P
#define LSMG_BRICK_P 2
#endif
#ifndef LSMG_BRICK_J
#define LSMG_BRICK_J 2
#endif

namespace lsmg {

constexpr int kWave = 64;
constexpr int kItemsPerBlock = 4;          // default: 256-thread workgroups, one item per wavefront
constexpr int kBlock = kWave * kItemsPerBlock;
constexpr int kMaxItemsPerBlock = 8;       // workgroup sizes 64 .. 512 (chosen per launch)
constexpr int kMaxBlock = kWave * kMaxItemsPerBlock;
constexpr int kMaxBandEntries2 = 8;        // 2^band_steps with band_steps <= 3 (2-D)
constexpr int kMaxBandEntries3 = 27;       // 3^band_steps (3-D)

enum : uint8_t { kOut = 0, kIn = 1, kGhost = 2 };

// A device pointer held in a descriptor or an argument block.  On the device,
// subscripts go through the global address space, so that loads and stores
// through it compile to global (not flat) memory instructions: these take a
// scalar base address and are counted apart from the scalar loads of the
// descriptor itself.  Offsetting keeps the type; converting to T * gives a
// generic pointer (flat accesses).
template <typename T>
struct gptr {
    T *p;
    __host__ __device__ gptr &operator=(T *q)
    {
        p = q;
        return *this;
    }
    __host__ __device__ operator T *() const { return p; }
    __host__ __device__ gptr operator+(long long i) const { return gptr{p + i}; }
    __device__ __attribute__((address_space(1))) T &operator[](long long i) const
    {
        return ((__attribute__((address_space(1))) T *)p)[i];
    }
};

template <typename T>
struct LevelDesc {
    int dim, n, Wp, nst;
    int ni, ng, na, nb, bmax;
    int level, pad0;
    long long rows, cs;
    double lo, h;
    // model and solver scalars in the working precision
    T kap;       // d / (4 h^2)
    T alpha, beta, dt_inv, ks_half, kc_half, tau_s;
    T d_half_h2; // d / (2 h^2)
    int ghost_c_new, pad1;
    // per-node arrays (split layout)
    gptr<const uint8_t> type;     // kOut / kIn / kGhost
    gptr<const uint8_t> ext;      // 1 for ghosts and band nodes reached by the extension
    gptr<const int> cmap;         // storage -> compact index, -1 if inactive
    gptr<T> s, c;                // linearisation point
    gptr<T> rhs_s, rhs_c;
    gptr<T> x_s, x_c;
    gptr<T> r_s, r_c;
    gptr<T> x2_s, x2_c;          // 2-D: second copy of the corrections (fused sweeps alternate)
    // ghost table (structure of arrays, entry k of ghost q at k * ng + q)
    gptr<const int> g_idx;        // storage index of ghost q
    gptr<const int> g_ijk;        // packed grid coordinates i | j << 11 | k << 22
    gptr<const int> g_st;         // storage index of stencil node k
    gptr<const int> g_stg;        // ghost index of stencil node k if it is a ghost with nonzero weight, else -1
    gptr<const T> g_w;            // boundary-row weight of stencil node k
    gptr<T> g_buf0, g_buf1;      // Jacobi buffers of the ghost values of delta s
    // ghost_sweeps Jacobi sweeps composed into one linear map (CSR over ghosts):
    // delta s_q <- sum_e go_a[e] delta s_{go_col[e]} + go_b[e] b_{go_col[e]}, b the
    // ghost rows' right-hand sides minus their non-ghost stencil terms
    gptr<const int> go_ptr, go_col;
    gptr<const T> go_a, go_b;
    // 2-D: the b-part folded into the map, b = rhs - W_GI x_I, so that
    // delta s_q <- sum_e go_a[e] s_old + go_b[e] rhs_s[ghost go_col[e]] - sum_f gc_w[f] x_s[gc_idx[f]],
    // with C = B W_GI composed over inside storage indices (null in 3-D)
    gptr<const int> gc_ptr, gc_idx;
    gptr<const T> gc_w;
    gptr<const int> go_sidx;      // 2-D: g_idx[go_col[e]], the storage index of entry e's ghost
    // 2-D: the folded rows padded to widths ell_we / ell_wf (entry k of ghost q at
    // q * width + k; padding: zero weights on the ghost itself), read without row pointers
    int ell_we, ell_wf;
    gptr<const int> ell_col, ell_six, ellf_idx;
    gptr<const T> ell_a, ell_b, ellf_w;
    // band of inactive nodes used by the boundary-defect restriction
    gptr<const int> b_idx;        // storage index of band node b
    gptr<const int> b_cnt;        // number of ghost sources
    gptr<const int> b_src;        // entry j at j * nb + b: storage index of a ghost
    gptr<const T> b_wt;           // its weight
    // max-norm slots of this domain: norm k occupies kNormSlots words at norms + k * norm_stride
    gptr<unsigned long long> norms;
    long long norm_stride;
    // level 0 only: data of the Crank-Nicolson step (section 3.1)
    gptr<double> sn, cn;         // W^n (split layout); W^{n+1} is written back on commit
    gptr<double> bs, bc;         // explicit half of the step
    gptr<const double> fn, fnp1; // compact [f1 | f2] source terms at t_n and t_{n+1}, or null
    gptr<const double> sb;        // per-ghost boundary values at t_{n+1}, or null (then sb_const)
    double sb_const;
};

__device__ __forceinline__ int item_desc(int4 w) { return w.x >> 2; }
__device__ __forceinline__ int item_kind(int4 w) { return w.x & 3; }

// row and position of lane `lane` of a 2-D segment item (kinds 0 and 1): positions
// [w.z, w.w) of row w.y; false past its end
__device__ __forceinline__ bool seg_lane(int4 w, int lane, int &row, int &p)
{
    p = w.z + lane;
    row = w.y;
    return p < w.w;
}

// 3-D brick shape: 2^kBP positions x 2^kBJ rows (y) x 2^kBK planes (z) of one
// colour, 32 values
constexpr int kBP = LSMG_BRICK_P, kBJ = LSMG_BRICK_J, kBK = 5 - LSMG_BRICK_P - LSMG_BRICK_J;

// bricks per row of positions, per plane of rows and per grid of planes
__host__ __device__ __forceinline__ int brick_np(int Wp) { return Wp >> kBP; }
__host__ __device__ __forceinline__ int brick_nj(int n) { return (n + (1 << kBJ) - 1) >> kBJ; }
__host__ __device__ __forceinline__ int brick_nk(int n) { return (n + (1 << kBK) - 1) >> kBK; }

// node of lane `lane` of a 3-D brick item (kinds 0 and 1 = colour): two bricks
// of the colour, consecutive along x, lanes 0-31 the first and 32-63 the second;
// value v = l & 31 of a brick lies at position (v mod 2^kBP), y offset
// (v >> kBP) mod 2^kBJ and z offset v >> (kBP + kBJ) within it.  w.y = pb | jb << 10
// | kb << 20 of the first brick; w.z, w.w: the bits of the inside nodes of each
// brick (false for the other lanes)
__host__ __device__ __forceinline__ bool brick_lane(int n, int Wp, long long cs, int colour, int4 w, int lane,
                                                    long long &idx, int &i, int &j, int &k)
{
    const int hi = lane >> 5, in = lane & 31;
    const unsigned mask = (unsigned)(hi ? w.w : w.z);
    const int pb = (w.y & 1023) + hi, jb = (w.y >> 10) & 1023, kb = (w.y >> 20) & 1023;
    const long long brick = ((long long)kb * brick_nj(n) + jb) * brick_np(Wp) + pb;
    idx = colour * cs + (brick << 5) + in;
    const int p = (pb << kBP) + (in & ((1 << kBP) - 1));
    j = (jb << kBJ) + ((in >> kBP) & ((1 << kBJ) - 1));
    k = (kb << kBK) + (in >> (kBP + kBJ));
    i = 2 * p + ((colour + j + k) & 1);
    return (mask >> in) & 1u;
}

// grid coordinates of the node at (colour, row, position)
template <int DIM>
__device__ __forceinline__ void node_coords(int n, int colour, long long row, int p, int &i, int &j, int &k)
{
    if (DIM == 2) {
        j = (int)row;
        k = 0;
    } else {
        const int r = (int)row;
        k = r / n;
        j = r - k * n;
    }
    i = 2 * p + ((colour + j + k) & 1);
}

__device__ __forceinline__ void unpack_ijk(int v, int &i, int &j, int &k)
{
    i = v & 2047;
    j = (v >> 11) & 2047;
    k = (v >> 22) & 1023;
}

// 3-D storage index of (colour, position p, y index j, z index k)
__host__ __device__ __forceinline__ long long sidx3(int n, int Wp, long long cs, int colour, int p, int j, int k)
{
    const long long brick = ((long long)(k >> kBK) * brick_nj(n) + (j >> kBJ)) * brick_np(Wp) + (p >> kBP);
    const int in = ((((k & ((1 << kBK) - 1)) << kBJ) | (j & ((1 << kBJ) - 1))) << kBP) | (p & ((1 << kBP) - 1));
    return colour * cs + (brick << 5) + in;
}

// storage index of node (colour, p, j, k) on a level of dimension DIM
template <int DIM>
__host__ __device__ __forceinline__ long long sidx_at(int n, int Wp, long long cs, int colour, int p, int j, int k)
{
    if (DIM == 3) return sidx3(n, Wp, cs, colour, p, j, k);
    return colour * cs + (long long)j * Wp + p;
}

// storage index of grid node (i, j, k) (k = 0 in 2-D)
__host__ __device__ __forceinline__ long long sidx(int dim, int n, int Wp, long long cs, int i, int j, int k)
{
    const int colour = (i + j + k) & 1;
    return dim == 3 ? sidx3(n, Wp, cs, colour, i >> 1, j, k) : colour * cs + (long long)j * Wp + (i >> 1);
}

// grid node (i, j, k) of storage index idx
template <int DIM>
__host__ __device__ __forceinline__ void sidx_node(int n, int Wp, long long cs, long long idx, int &i, int &j, int &k)
{
    const int colour = (int)(idx / cs);
    const long long rem = idx - colour * cs;
    int p;
    if (DIM == 3) {
        const long long brick = rem >> 5;
        const int in = (int)(rem & 31), np = brick_np(Wp), nj = brick_nj(n);
        const long long jk = brick / np;
        p = ((int)(brick - jk * np) << kBP) + (in & ((1 << kBP) - 1));
        const int kb = (int)(jk / nj);
        j = ((int)(jk - (long long)kb * nj) << kBJ) + ((in >> kBP) & ((1 << kBJ) - 1));
        k = (kb << kBK) + (in >> (kBP + kBJ));
    } else {
        j = (int)(rem / Wp);
        p = (int)(rem - (long long)j * Wp);
        k = 0;
    }
    i = 2 * p + ((colour + j + k) & 1);
}

// storage indices of the axis neighbours of node (i, j, k) of colour `colour`
// (an inside node: never on the box edge), ordered x-, x+, y-, y+[, z-, z+]
template <int DIM>
__device__ __forceinline__ void neighbours(int n, int Wp, long long cs, int colour, int i, int j, int k, long long *nb)
{
    const int o = colour ^ 1, p = i >> 1;
    if (DIM == 3) {
        nb[0] = sidx3(n, Wp, cs, o, (i - 1) >> 1, j, k);
        nb[1] = sidx3(n, Wp, cs, o, (i + 1) >> 1, j, k);
        nb[2] = sidx3(n, Wp, cs, o, p, j - 1, k);
        nb[3] = sidx3(n, Wp, cs, o, p, j + 1, k);
        nb[4] = sidx3(n, Wp, cs, o, p, j, k - 1);
        nb[5] = sidx3(n, Wp, cs, o, p, j, k + 1);
        return;
    }
    const long long ob = o * cs + (long long)j * Wp;
    nb[0] = ob + ((i - 1) >> 1);
    nb[1] = ob + ((i + 1) >> 1);
    nb[2] = ob - Wp + p;
    nb[3] = ob + Wp + p;
}

// max of non-negative doubles as ordered bit patterns; NaN (any payload, sign
// cleared) orders above +inf, so the maximum propagates NaN
__device__ __forceinline__ unsigned long long abs_bits(double v)
{
    return (unsigned long long)__double_as_longlong(v) & 0x7fffffffffffffffull;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// A norm is kept in kNormSlots partial slots (the host takes their max): each
// wavefront folds its lanes and one lane updates the slot of its wavefront
// number, which keeps the atomics on any one address few.
constexpr int kNormSlots = 256;

// one DPP step of a wavefront max: each lane takes the larger of its value and
// the value of the lane the control names (lanes of rows the mask leaves out
// compare with themselves)
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long max_dpp_u64(unsigned long long v)
{
    const int lo = __builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(v >> 32), (int)(v >> 32), CTRL, ROWS, 0xf, false);
    const unsigned long long o = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
    return o > v ? o : v;
}

// the wavefront max by VALU data-parallel moves (no LDS traffic): pairs within
// quads, half rows and rows, then the two row broadcasts; the result is in lane 63.
// Called with every lane active.
__device__ __forceinline__ unsigned long long wave_max_u64_last(unsigned long long v)
{
    v = max_dpp_u64<0xB1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
    v = max_dpp_u64<0x4E, 0xf>(v);    // quad_perm [2, 3, 0, 1]
    v = max_dpp_u64<0x141, 0xf>(v);   // row_half_mirror
    v = max_dpp_u64<0x140, 0xf>(v);   // row_mirror
    v = max_dpp_u64<0x142, 0xa>(v);   // row_bcast:15
    v = max_dpp_u64<0x143, 0xc>(v);   // row_bcast:31
    return v;
}

__device__ __forceinline__ void norm_accumulate(unsigned long long *slot, unsigned long long bits)
{
    bits = wave_max_u64_last(bits);
    const int wslot = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & (kNormSlots - 1);
    if ((threadIdx.x & (kWave - 1)) == kWave - 1 && bits != 0ull) atomicMax(slot + wslot, bits);
}

// norm k of the domain that owns descriptor D
template <typename T>
__device__ __forceinline__ void norm_accumulate(const LevelDesc<T> *D, int k, unsigned long long bits)
{
    norm_accumulate(D->norms + k * D->norm_stride, bits);
}

}  // namespace lsmg
