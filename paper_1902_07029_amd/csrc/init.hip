// Preparation of a domain's inputs on a full grid, before its hierarchy is built
// (sections 2 and 3.3): re-initialisation of a level set towards the signed
// distance, a level set from a mask (the paper's treatment of image data), and
// the second-order extrapolation of initial data from the inside to the ghost
// nodes.  One thread per grid node (x fastest), compiled without FMA
// contraction and in the same operation order as the CPU reference, so that
// both give the same bits.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <utility>
#include <vector>

#include "hier.hpp"

namespace lsmg {
namespace {

struct Grid3 {
    int dim, n;
    long long nn;
    double h;
};

__device__ __forceinline__ void unravel3(long long g, int n, int dim, int *gi)
{
    gi[0] = (int)(g % n);
    gi[1] = (int)((g / n) % n);
    gi[2] = dim == 3 ? (int)(g / ((long long)n * n)) : 0;
}

__device__ __forceinline__ long long stride_of(int n, int a)
{
    return a == 0 ? 1LL : (a == 1 ? (long long)n : (long long)n * n);
}

// value of v at the neighbour of g along axis a on side s, or at g outside the box
__device__ __forceinline__ double nbv(const double *v, long long g, const int *gi, int n, int a, int s)
{
    const int k = gi[a] + s;
    if (k < 0 || k >= n) return v[g];
    return v[g + s * stride_of(n, a)];
}

// re-initialisation (subcell fix of Russo and Smereka): the nodes next to a sign
// change of phi0 and their target D = h phi0 / dphi0
__global__ void k_reinit_prep(Grid3 G, const double *__restrict__ phi0, uint8_t *__restrict__ near,
                              double *__restrict__ D)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G.nn) return;
    int gi[3];
    unravel3(g, G.n, G.dim, gi);
    const double p0 = phi0[g];
    double c2 = 0.0, f2 = 0.0, b2 = 0.0;
    bool nr = false;
    for (int a = 0; a < G.dim; ++a) {
        const double pm = nbv(phi0, g, gi, G.n, a, -1), pp = nbv(phi0, g, gi, G.n, a, +1);
        if (p0 * pm <= 0.0 || p0 * pp <= 0.0) nr = true;
        const double c = (pp - pm) / 2.0, f = pp - p0, bk = p0 - pm;
        c2 += c * c;
        f2 += f * f;
        b2 += bk * bk;
    }
    double dp = sqrt(c2);
    if (sqrt(f2) > dp) dp = sqrt(f2);
    if (sqrt(b2) > dp) dp = sqrt(b2);
    if (dp < 1e-300) dp = 1e-300;
    near[g] = nr;
    D[g] = G.h * p0 / dp;
}

__global__ void k_reinit_step(Grid3 G, const double *__restrict__ phi0, const uint8_t *__restrict__ near,
                              const double *__restrict__ D, const double *__restrict__ cur, double *__restrict__ nxt)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G.nn) return;
    const double h = G.h, p0 = phi0[g], dmu = h / G.dim;
    const double sg = p0 > 0.0 ? 1.0 : (p0 < 0.0 ? -1.0 : 0.0);
    if (near[g]) {
        nxt[g] = cur[g] - (dmu / h) * (sg * fabs(cur[g]) - D[g]);
        return;
    }
    int gi[3];
    unravel3(g, G.n, G.dim, gi);
    double g2 = 0.0;
    for (int a = 0; a < G.dim; ++a) {
        const double dm = (cur[g] - nbv(cur, g, gi, G.n, a, -1)) / h;
        const double dpp = (nbv(cur, g, gi, G.n, a, +1) - cur[g]) / h;
        double u, w;
        if (p0 > 0.0) {
            u = dm > 0.0 ? dm : 0.0;
            w = dpp < 0.0 ? dpp : 0.0;
        } else {
            u = dm < 0.0 ? dm : 0.0;
            w = dpp > 0.0 ? dpp : 0.0;
        }
        const double m = u * u > w * w ? u * u : w * w;
        g2 += m;
    }
    nxt[g] = cur[g] - dmu * sg * (sqrt(g2) - 1.0);
}

__global__ void k_mask_init(Grid3 G, const uint8_t *__restrict__ mask, double *__restrict__ phi)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < G.nn) phi[g] = mask[g] ? -1.0 : 1.0;
}

__global__ void k_heat_step(Grid3 G, const double *__restrict__ cur, double *__restrict__ nxt)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G.nn) return;
    int gi[3];
    unravel3(g, G.n, G.dim, gi);
    double lap = 0.0;
    for (int a = 0; a < G.dim; ++a) lap += nbv(cur, g, gi, G.n, a, -1) - 2.0 * cur[g] + nbv(cur, g, gi, G.n, a, +1);
    nxt[g] = cur[g] + (1.0 / (2.0 * G.dim)) * lap;
}

// unit normals by central differences (one-sided at the box edge) and the inside flags
__global__ void k_normals(Grid3 G, const double *__restrict__ phi, double *__restrict__ nrm, uint8_t *__restrict__ k0)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G.nn) return;
    int gi[3];
    unravel3(g, G.n, G.dim, gi);
    const double h = G.h;
    double gr[3] = {0.0, 0.0, 0.0}, l2 = 0.0;
    for (int a = 0; a < G.dim; ++a) {
        const long long sa = stride_of(G.n, a);
        if (gi[a] > 0 && gi[a] < G.n - 1) gr[a] = (phi[g + sa] - phi[g - sa]) / (2.0 * h);
        else if (gi[a] == 0) gr[a] = (phi[g + sa] - phi[g]) / h;
        else gr[a] = (phi[g] - phi[g - sa]) / h;
        l2 += gr[a] * gr[a];
    }
    const double l = sqrt(l2);
    for (int a = 0; a < G.dim; ++a) nrm[g * G.dim + a] = l > 0.0 ? gr[a] / l : 0.0;
    k0[g] = phi[g] < 0.0;
}

// v_out = n . grad v_in by central differences where the node and its axis
// neighbours are known (kout = 1 there), else 0
__global__ void k_normal_derivative(Grid3 G, const double *__restrict__ nrm, const uint8_t *__restrict__ kin,
                                    const double *__restrict__ vin, uint8_t *__restrict__ kout,
                                    double *__restrict__ vout)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G.nn) return;
    int gi[3];
    unravel3(g, G.n, G.dim, gi);
    bool ok = kin[g];
    for (int a = 0; a < G.dim && ok; ++a) {
        const long long sa = stride_of(G.n, a);
        if (gi[a] == 0 || gi[a] == G.n - 1 || !kin[g - sa] || !kin[g + sa]) ok = false;
    }
    kout[g] = ok;
    double v = 0.0;
    if (ok)
        for (int a = 0; a < G.dim; ++a) {
            const long long sa = stride_of(G.n, a);
            v += nrm[g * G.dim + a] * (vin[g + sa] - vin[g - sa]) / (2.0 * G.h);
        }
    vout[g] = v;
}

__global__ void k_keep_known(Grid3 G, const uint8_t *__restrict__ k0, const double *__restrict__ q,
                             double *__restrict__ out)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < G.nn) out[g] = k0[g] ? q[g] : 0.0;
}

// one pseudo-time step of the extension along n where known == 0:
// v <- v - dtau (n . grad_up v - src)
__global__ void k_extend_step(Grid3 G, const double *__restrict__ nrm, const uint8_t *__restrict__ known,
                              const double *__restrict__ src, const double *__restrict__ v, double *__restrict__ nxt)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G.nn) return;
    if (known[g]) {
        nxt[g] = v[g];
        return;
    }
    int gi[3];
    unravel3(g, G.n, G.dim, gi);
    const double h = G.h;
    double adv = 0.0;
    for (int a = 0; a < G.dim; ++a) {
        const double na = nrm[g * G.dim + a];
        double d;
        if (na > 0.0) d = (v[g] - nbv(v, g, gi, G.n, a, -1)) / h;
        else if (na < 0.0) d = (nbv(v, g, gi, G.n, a, +1) - v[g]) / h;
        else d = 0.0;
        adv += na * d;
    }
    nxt[g] = v[g] - (h / G.dim) * (adv - (src ? src[g] : 0.0));
}

unsigned blocks_of(long long n) { return (unsigned)((n + 255) / 256); }

lsmg_status grid3(const lsmg_grid *grid, Grid3 &G)
{
    if (!grid || (grid->dim != 2 && grid->dim != 3) || grid->n < 3 || !(grid->hi > grid->lo))
        return fail(LSMG_EINVAL, "bad grid");
    G.dim = grid->dim;
    G.n = grid->n;
    G.nn = (long long)grid->n * grid->n * (grid->dim == 3 ? grid->n : 1);
    G.h = (grid->hi - grid->lo) / (grid->n - 1);
    return LSMG_OK;
}

// device scratch of one call, freed on every exit path
struct Scratch {
    std::vector<void *> p;
    template <typename V>
    lsmg_status get(V **out, long long count)
    {
        void *q = nullptr;
        if (hipMalloc(&q, sizeof(V) * (size_t)(count > 0 ? count : 1)) != hipSuccess)
            return fail(LSMG_EOOM, "device allocation failed");
        p.push_back(q);
        *out = (V *)q;
        return LSMG_OK;
    }
    ~Scratch()
    {
        for (void *q : p) (void)hipFree(q);
    }
};

// re-initialisation on caller streams and buffers: phi0, D and the second
// copy of phi (n^dim doubles each), then the near-interface flags (n^dim bytes)
void reinit_run(const Grid3 &G, double *d_phi, int iterations, hipStream_t s, double *phi0, double *tmp, double *D,
                uint8_t *near)
{
    (void)hipMemcpyAsync(phi0, d_phi, sizeof(double) * G.nn, hipMemcpyDeviceToDevice, s);
    k_reinit_prep<<<blocks_of(G.nn), 256, 0, s>>>(G, phi0, near, D);
    double *cur = d_phi, *nxt = tmp;
    for (int it = 0; it < iterations; ++it) {
        k_reinit_step<<<blocks_of(G.nn), 256, 0, s>>>(G, phi0, near, D, cur, nxt);
        std::swap(cur, nxt);
    }
    if (cur != d_phi) (void)hipMemcpyAsync(d_phi, cur, sizeof(double) * G.nn, hipMemcpyDeviceToDevice, s);
}

// Scratch of the allocation-free re-initialisation: one array per device,
// sized for grids of up to kNoAllocNodes nodes (1025^2 in 2-D, 127^3 in 3-D),
// 25 bytes per node (three doubles and a flag), 52.4 MB in all.  Each device
// holds its copy until the process ends.
constexpr long long kNoAllocNodes = 1LL << 21;
constexpr size_t kNoAllocBytes = (size_t)kNoAllocNodes * (3 * sizeof(double) + 1);
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// the device address of `scratch` on each device, looked up once per device
// with that device current (the array's host-side name is not a device address)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

lsmg_status scratch_ptr(void **out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LSMG_EINVAL, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LSMG_EHIP, "no device address for the re-initialisation scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LSMG_OK;
}

}  // namespace
}  // namespace lsmg

using namespace lsmg;

extern "C" {

lsmg_status lsmg_reinitialize(double *d_phi, const lsmg_grid *grid, int iterations, void *stream)
{
    Grid3 G;
    LSMGCHK(grid3(grid, G));
    if (!d_phi || iterations < 0) return fail(LSMG_EINVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    Scratch S;
    double *phi0, *tmp, *D;
    uint8_t *near;
    LSMGCHK(S.get(&phi0, G.nn));
    LSMGCHK(S.get(&tmp, G.nn));
    LSMGCHK(S.get(&D, G.nn));
    LSMGCHK(S.get(&near, G.nn));
    reinit_run(G, d_phi, iterations, s, phi0, tmp, D, near);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return LSMG_OK;
}

lsmg_status lsmg_reinitialize_noalloc(double *d_phi, const lsmg_grid *grid, int iterations, void *stream)
{
    Grid3 G;
    LSMGCHK(grid3(grid, G));
    if (G.nn > kNoAllocNodes)
        return fail(LSMG_EINVAL, "grid of %lld nodes exceeds the %lld nodes of the allocation-free scratch",
                    G.nn, kNoAllocNodes);
    if (!d_phi || iterations < 0) return fail(LSMG_EINVAL, "bad argument");
    void *p = nullptr;
    LSMGCHK(scratch_ptr(&p));
    // the regions are laid out for the largest grid, so their offsets never move
    unsigned char *base = (unsigned char *)p;
    double *phi0 = (double *)base;
    double *tmp = phi0 + kNoAllocNodes;
    double *D = tmp + kNoAllocNodes;
    uint8_t *near = (uint8_t *)(D + kNoAllocNodes);
    hipStream_t s = (hipStream_t)stream;
    reinit_run(G, d_phi, iterations, s, phi0, tmp, D, near);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return LSMG_OK;
}

lsmg_status lsmg_levelset_from_mask(const uint8_t *d_mask, const lsmg_grid *grid, int iterations, double *d_phi,
                                    void *stream)
{
    Grid3 G;
    LSMGCHK(grid3(grid, G));
    if (!d_mask || !d_phi || iterations < 0) return fail(LSMG_EINVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    Scratch S;
    double *tmp;
    LSMGCHK(S.get(&tmp, G.nn));
    k_mask_init<<<blocks_of(G.nn), 256, 0, s>>>(G, d_mask, d_phi);
    double *cur = d_phi, *nxt = tmp;
    for (int it = 0; it < iterations; ++it) {
        k_heat_step<<<blocks_of(G.nn), 256, 0, s>>>(G, cur, nxt);
        std::swap(cur, nxt);
    }
    if (cur != d_phi) HIPCHK(hipMemcpyAsync(d_phi, cur, sizeof(double) * G.nn, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return LSMG_OK;
}

lsmg_status lsmg_extrapolate(const double *d_phi, const lsmg_grid *grid, double *d_q, int iterations, void *stream)
{
    Grid3 G;
    LSMGCHK(grid3(grid, G));
    if (!d_phi || !d_q || iterations < 0) return fail(LSMG_EINVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    const unsigned nb = blocks_of(G.nn);
    Scratch S;
    double *nrm, *qn, *qnn, *tmp, *out;
    uint8_t *k0, *k1, *k2;
    LSMGCHK(S.get(&nrm, G.nn * G.dim));
    LSMGCHK(S.get(&qn, G.nn));
    LSMGCHK(S.get(&qnn, G.nn));
    LSMGCHK(S.get(&tmp, G.nn));
    LSMGCHK(S.get(&out, G.nn));
    LSMGCHK(S.get(&k0, G.nn));
    LSMGCHK(S.get(&k1, G.nn));
    LSMGCHK(S.get(&k2, G.nn));
    k_normals<<<nb, 256, 0, s>>>(G, d_phi, nrm, k0);
    k_normal_derivative<<<nb, 256, 0, s>>>(G, nrm, k0, d_q, k1, qn);
    k_normal_derivative<<<nb, 256, 0, s>>>(G, nrm, k1, qn, k2, qnn);
    k_keep_known<<<nb, 256, 0, s>>>(G, k0, d_q, out);
    // q_nn, then q_n, then q, each extended over `iterations` pseudo-time steps
    struct Stage {
        const uint8_t *known;
        const double *src;
        double *v;
    } stages[3] = {{k2, nullptr, qnn}, {k1, qnn, qn}, {k0, qn, out}};
    for (const Stage &st : stages) {
        double *cur = st.v, *nxt = tmp;
        for (int it = 0; it < iterations; ++it) {
            k_extend_step<<<nb, 256, 0, s>>>(G, nrm, st.known, st.src, cur, nxt);
            std::swap(cur, nxt);
        }
        if (cur != st.v) HIPCHK(hipMemcpyAsync(st.v, cur, sizeof(double) * G.nn, hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipMemcpyAsync(d_q, out, sizeof(double) * G.nn, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return LSMG_OK;
}

}  // extern "C"
