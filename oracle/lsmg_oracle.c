/*
 * Serial FP64 CPU oracle for the level-set multigrid method of Coco, Semplice
 * and Serra Capizzano, "A level-set multigrid technique for nonlinear diffusion
 * in the numerical simulation of marble degradation under chemical pollutants"
 * (arXiv 1902.07029).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or table with the GPU
 * library.
 *
 * Everything is plain C99 in double precision, one node at a time, on
 * full-grid arrays indexed by the lexicographic grid index g = i + n*(j + n*k)
 * (x fastest).  Public vectors use the compact ordering of §3.3 (eq. maprij):
 * inside nodes in lexicographic order, then ghost nodes in lexicographic
 * order; a vector of a level is [s-block (Na) | c-block (Na)], Na = Ni + Ng.
 *
 * Readings of points the paper leaves open are marked READING and listed in
 * the design notes of the repository.  Parity status of each function is
 * stated in its comment; "parity unpinned" marks rules that no paper value or
 * closed form fixes (coarse-level choices that affect only the convergence
 * factor).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_EGEOM -2
#define OR_ENOCONV -3
#define OR_ENONFINITE -4
#define OR_EOOM -5

#define MAXLEV 16

typedef struct {
    int n;           /* nodes per axis */
    double h;        /* grid step */
    long nn;         /* n^dim */
    double *phi;     /* level set at the nodes of this level (injected) */
    signed char *type; /* 0 outside/inactive, 1 inside, 2 ghost */
    int ni, ng, na;
    long *c2g;       /* compact -> grid */
    int *g2c;        /* grid -> compact, -1 if inactive */
    /* ghost geometry, ghost q has compact index ni + q */
    long *st;        /* ng * nst grid indices of the upwind stencil ST */
    double *w;       /* ng * nst boundary-row weights */
    double *B;       /* ng * dim boundary points */
    double *nrm;     /* ng * dim unit outward normals (central differences, eq. nij) */
    double *nrow;    /* ng * dim normal of the boundary row: nrm (Dirichlet), or the unit
                        gradient of the interpolated level set at B (Neumann, eq. Neumanntilde) */
    int *order;      /* 2 biquadratic, 1 bilinear, 0 constant (Neumann: one-sided) */
    int *bfall;      /* B from: 0 bisection along the normal, 1 the first-order projection, 2 the axis rule */
    /* band of inactive nodes around coarse ghost centres (for the BC defect) */
    int nb;
    long *band;      /* grid indices */
    long *bup;       /* nb * dim upwind neighbour grid indices (-1 = none) */
    double *bwt;     /* nb * dim normalised upwind weights */
    /* linearisation point and work vectors, full grid */
    double *s, *c, *rhs_s, *rhs_c, *x_s, *x_c, *r_s, *r_c;
} OLevel;

typedef struct {
    double a, d, m_s, m_c, alpha, beta, tau_s;
    int nu1, nu2, ghost_c_new, band_steps, ghost_sweeps;
    /* READING (sweeps per smoothing step): levels whose diffusion number
     * d dt / h^2 is below sweeps_lambda use ghost_sweeps_coarse */
    int ghost_sweeps_coarse;
    double sweeps_lambda;
    int gamma;         /* cycle index: 1 V-cycle, 2 W-cycle (the paper's cycle, §4) */
    int lex;           /* 1: inside nodes relaxed in lexicographic order (the paper's
                          collective Gauss-Seidel, §3.5.1); 0: red-black */
    int fmg;           /* full multigrid as the first iteration of the linear solves:
                          0 never, 1 in the first Newton iteration of a step, 2 in every one */
    int krylov_m;      /* 0: the linear solves iterate V-cycles (the paper); m > 0: flexible
                          GMRES(m) preconditioned by one V-cycle (not in the paper) */
} OPar;

typedef struct or_hier {
    int dim, nlev, nst;
    int bctype;        /* boundary condition for s: 0 Dirichlet (eq. BCs), 1 Neumann (eq. BCsN) */
    double lo, hi;
    OLevel L[MAXLEV];
    OPar p;
    double dt;
    int lin_set;
    /* dense LU of the coarsest operator */
    int lu_n;
    double *lu;
    int *piv;
    int lu_ok;
    /* step state (finest level, full grid) */
    double *bs, *bc;   /* explicit Crank-Nicolson half */
    int *egeom_level;
} or_hier;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static void unravel(long g, int n, int dim, int *idx)
{
    for (int a = 0; a < dim; ++a) { idx[a] = (int)(g % n); g /= n; }
    for (int a = dim; a < 3; ++a) idx[a] = 0;
}

static long ravel(const int *idx, int n, int dim)
{
    long g = 0;
    for (int a = dim - 1; a >= 0; --a) g = g * n + idx[a];
    return g;
}

static int in_box(const int *idx, int n, int dim)
{
    for (int a = 0; a < dim; ++a) if (idx[a] < 0 || idx[a] >= n) return 0;
    return 1;
}

static long stride_of(int n, int a)
{
    long s = 1;
    for (int b = 0; b < a; ++b) s *= n;
    return s;
}

static int ipow3(int d) { return d == 1 ? 3 : d == 2 ? 9 : 27; }

static double phi_por(const OPar *p, double c) { return p->alpha * c + p->beta; }  /* §2, porosity law */

/* 1-D quadratic Lagrange weights at local coordinate t for the three stencil
 * nodes k = 0 (t = 1, the ghost), k = 1 (t = 0), k = 2 (t = -1): §3.4,
 * eq. (intcoeffsD), with the paper's theta equal to t. */
static double lag2(int k, double t)
{
    if (k == 0) return t * (1.0 + t) / 2.0;
    if (k == 1) return (1.0 - t) * (1.0 + t);
    return t * (t - 1.0) / 2.0;
}

/* 1-D linear weights on the two nodes nearest the ghost (READING: order
 * fallback when the biquadratic stencil touches an inactive node). */
static double lag1(int k, double t)
{
    if (k == 0) return t;
    if (k == 1) return 1.0 - t;
    return 0.0;
}

/* derivatives d/dt of the quadratic weights, the coefficients of eq.
 * (intcoeffsN) times h: theta + 1/2, -2 theta, theta - 1/2 for k = 0, 1, 2 */
static double dlag2(int k, double t)
{
    if (k == 0) return t + 0.5;
    if (k == 1) return -2.0 * t;
    return t - 0.5;
}

/* derivatives d/dt of the linear weights */
static double dlag1(int k)
{
    if (k == 0) return 1.0;
    if (k == 1) return -1.0;
    return 0.0;
}

/* relaxation parameter of the ghost rows on a level: tau_s for the Dirichlet
 * row (eq. CFLcond); for the Neumann row tau_s times the bound of eq.
 * CFLcondN, 2 sqrt(2) h / 3 (READING in 3-D: 4 h / (3 sqrt(3)), the same
 * bound taken over three axes) */
static double tau_level(const struct or_hier *H, const OLevel *L);

/* ------------------------------------------------------------------ */
/* hierarchy: classification (§3.3, eq. ghostdef) and ghost geometry    */
/* ------------------------------------------------------------------ */

static double xcoord(const or_hier *H, const OLevel *L, int i) { return H->lo + i * L->h; }

/* biquadratic (triquadratic) interpolant of phi on the stencil ST of a ghost,
 * evaluated at point X (§3.3, bisection step). */
static double phi_tilde(const or_hier *H, const OLevel *L, const long *st, const int *gi,
                        const int *m, const double *X)
{
    int dim = H->dim;
    double t[3];
    for (int a = 0; a < dim; ++a) t[a] = m[a] * (X[a] - xcoord(H, L, gi[a] - m[a])) / L->h;
    double v = 0.0;
    for (int k = 0; k < H->nst; ++k) {
        int kk = k;
        double wk = 1.0;
        for (int a = 0; a < dim; ++a) { wk *= lag2(kk % 3, t[a]); kk /= 3; }
        v += wk * L->phi[st[k]];
    }
    return v;
}

/* normal by central differences of phi (§3.3, eq. nij); one-sided at the box edge */
static void grad_phi(const or_hier *H, const OLevel *L, const int *gi, double *nt)
{
    int dim = H->dim, n = L->n;
    long g = ravel(gi, n, dim);
    for (int a = 0; a < dim; ++a) {
        long sa = stride_of(n, a);
        if (gi[a] > 0 && gi[a] < n - 1)
            nt[a] = (L->phi[g + sa] - L->phi[g - sa]) / (2.0 * L->h);
        else if (gi[a] == 0)
            nt[a] = (L->phi[g + sa] - L->phi[g]) / L->h;
        else
            nt[a] = (L->phi[g] - L->phi[g - sa]) / L->h;
    }
}

static double tau_level(const or_hier *H, const OLevel *L)
{
    if (H->bctype == 0) return H->p.tau_s;
    if (H->dim == 2) return H->p.tau_s * (2.0 * sqrt(2.0) * L->h / 3.0);
    return H->p.tau_s * (4.0 * L->h / (3.0 * sqrt(3.0)));
}

/* Neumann boundary row of a ghost (§3.6, eqs. BCsN, Neumanntilde, JccN): the
 * derivative at B of the biquadratic (triquadratic) interpolant of s on ST
 * along the row normal, the unit gradient at B of the interpolant of phi on
 * ST (the central-difference normal where ST leaves the box, theta is out of
 * range or that gradient vanishes).  With the local coordinate t_a of the
 * stencil, d/dx_a = (m_a / h) d/dt_a.
 * READING (order fallback, as for the Dirichlet row): the quadratic rule, else
 * the gradient of the bilinear interpolant on the box of the nodes k in
 * {0,1}^d, else one-sided differences s_G - s_{G - m_a e_a} on the axes with
 * n_a m_a > 0 whose inward neighbour is active (the bilinear rule at theta = 1
 * without the other axes).  A rule is taken only if its nonzero weights sit on
 * active nodes and its self weight w_G lies in (0, 2 / tau_max], tau_max the
 * bound of eq. CFLcondN, so that the relaxation factor stays below 1 in
 * modulus.  No admissible rule (no such axis): EGEOM. */
static int neumann_row(const or_hier *H, const OLevel *L, const int *m, const long *st, const char *oob,
                       int any_oob, const double *th, int bad_theta, const double *nrm, double *w,
                       double *nr, int *order_out)
{
    int dim = H->dim, nst = H->nst;
    double h = L->h;
    for (int a = 0; a < dim; ++a) nr[a] = nrm[a];
    if (!any_oob && !bad_theta) {
        double gr[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) {
            double v = 0.0;
            for (int k = 0; k < nst; ++k) {
                int kk = k;
                double wk = 1.0;
                for (int b = 0; b < dim; ++b) {
                    wk *= (b == a) ? dlag2(kk % 3, th[b]) : lag2(kk % 3, th[b]);
                    kk /= 3;
                }
                v += wk * L->phi[st[k]];
            }
            gr[a] = m[a] * v / h;
        }
        double g2 = 0.0;
        for (int a = 0; a < dim; ++a) g2 += gr[a] * gr[a];
        if (g2 > 0.0) {
            double gl = sqrt(g2);
            for (int a = 0; a < dim; ++a) nr[a] = gr[a] / gl;
        }
    }
    double wmax = (dim == 2) ? 3.0 / (sqrt(2.0) * h) : 3.0 * sqrt(3.0) / (2.0 * h);
    for (int order = 2; order >= 1 && !bad_theta; --order) {
        for (int k = 0; k < nst; ++k) {
            double v = 0.0;
            for (int a = 0; a < dim; ++a) {
                int kk = k;
                double wk = 1.0;
                for (int b = 0; b < dim; ++b) {
                    int kb = kk % 3;
                    if (order == 2) wk *= (b == a) ? dlag2(kb, th[b]) : lag2(kb, th[b]);
                    else wk *= (b == a) ? dlag1(kb) : lag1(kb, th[b]);
                    kk /= 3;
                }
                v += nr[a] * m[a] * wk / h;
            }
            w[k] = v;
        }
        int ok = w[0] > 0.0 && w[0] <= wmax;
        for (int k = 0; k < nst; ++k) if (w[k] != 0.0 && (oob[k] || L->type[st[k]] == 0)) ok = 0;
        if (ok) { *order_out = order; return OR_OK; }
    }
    for (int k = 0; k < nst; ++k) w[k] = 0.0;
    double wg = 0.0;
    for (int a = 0; a < dim; ++a) {
        int k = (a == 0) ? 1 : (a == 1) ? 3 : 9;   /* stencil entry of G - m_a e_a */
        double c = nr[a] * m[a];
        if (!(c > 0.0) || oob[k] || L->type[st[k]] == 0) continue;
        w[k] = -c / h;
        wg += c / h;
    }
    if (!(wg > 0.0)) return OR_EGEOM;
    w[0] = wg;
    *order_out = 0;
    return OR_OK;
}

/* READING (axis rule, 2-D): where the row of eq. BCs would take the constant
 * rule (a negative self-weight, B outside the stencil, or no admissible order),
 * the boundary point is taken on a grid line instead.  Among the axis
 * neighbours G + sgn e_a that are inside (axes in order, sgn = -1 then +1), the
 * one whose line gives the ghost the largest self-weight is chosen: on that line
 * the stencil is oriented so that G - m_a e_a is the neighbour (m_a = -sgn), B
 * is the zero of the quadratic interpolant of phi through G, G - m_a e_a and
 * G - 2 m_a e_a (linear through the first two where the third leaves the box),
 * found by bisection of t in (0, 1], and theta = t on that axis, 1 on the
 * other.  The row is the quadratic interpolation along the line (linear where
 * G - 2 m_a e_a is inactive): second order, with self-weight t (1 + t) / 2 (or
 * t) in (0, 1].  Returns 0 if G has no inside axis neighbour. */
static int axis_row(const or_hier *H, const OLevel *L, long g, const int *gi, int *m, long *st, char *oob,
                    double *Bp, double *th, double *w, int *order)
{
    int dim = H->dim, n = L->n, nst = H->nst;
    int best = -1, bsgn = 0;
    double bw = -1.0, bt = 0.0;
    for (int a = 0; a < dim; ++a)
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            int n1[3] = {gi[0], gi[1], gi[2]}, n2[3] = {gi[0], gi[1], gi[2]};
            n1[a] += sgn;
            n2[a] += 2 * sgn;
            if (!in_box(n1, n, dim) || !(L->phi[ravel(n1, n, dim)] < 0.0)) continue;
            int q2 = in_box(n2, n, dim);
            double f0 = L->phi[g], f1 = L->phi[ravel(n1, n, dim)], f2 = q2 ? L->phi[ravel(n2, n, dim)] : 0.0;
            double lo = 0.0, hi = 1.0;
            for (int it = 0; it < 200; ++it) {
                double t = 0.5 * (lo + hi);
                if (t <= lo || t >= hi) break;
                double v = q2 ? lag2(0, t) * f0 + lag2(1, t) * f1 + lag2(2, t) * f2 : t * f0 + (1.0 - t) * f1;
                if (v < 0.0) lo = t; else hi = t;
            }
            double wg = (q2 && L->type[ravel(n2, n, dim)] != 0) ? lag2(0, hi) : lag1(0, hi);
            if (wg > bw) { bw = wg; best = a; bsgn = sgn; bt = hi; }
        }
    if (best < 0) return 0;
    m[best] = -bsgn;
    for (int k = 0; k < nst; ++k) {
        int kk = k, idx[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) { idx[a] = gi[a] - m[a] * (kk % 3); kk /= 3; }
        oob[k] = !in_box(idx, n, dim);
        st[k] = oob[k] ? g : ravel(idx, n, dim);
    }
    for (int a = 0; a < dim; ++a) { Bp[a] = xcoord(H, L, gi[a]); th[a] = 1.0; }
    th[best] = bt;
    Bp[best] = xcoord(H, L, gi[best]) - m[best] * L->h * (1.0 - bt);
    *order = 2;
    for (int k = 0; k < nst; ++k) {
        int kk = k; double wk = 1.0;
        for (int a = 0; a < dim; ++a) { wk *= lag2(kk % 3, th[a]); kk /= 3; }
        w[k] = wk;
    }
    for (int k = 0; k < nst; ++k) if (w[k] != 0.0 && (oob[k] || L->type[st[k]] == 0)) *order = 1;
    if (*order == 1)
        for (int k = 0; k < nst; ++k) {
            int kk = k; double wk = 1.0;
            for (int a = 0; a < dim; ++a) { wk *= lag1(kk % 3, th[a]); kk /= 3; }
            w[k] = wk;
        }
    return 1;
}

static int build_level_geometry(or_hier *H, int l)
{
    OLevel *L = &H->L[l];
    int dim = H->dim, n = L->n, nst = H->nst;
    long nn = L->nn;
    /* classification */
    for (long g = 0; g < nn; ++g) L->type[g] = (L->phi[g] < 0.0) ? 1 : 0;
    for (long g = 0; g < nn; ++g) {
        int gi[3];
        unravel(g, n, dim, gi);
        if (L->type[g] == 1) {
            for (int a = 0; a < dim; ++a)
                if (gi[a] == 0 || gi[a] == n - 1) return OR_EGEOM;  /* 5-point row would leave the box */
            continue;
        }
        for (int a = 0; a < dim && L->type[g] == 0; ++a) {
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                int nb[3] = {gi[0], gi[1], gi[2]};
                nb[a] += sgn;
                if (!in_box(nb, n, dim)) continue;
                long q = ravel(nb, n, dim);
                if (L->phi[q] < 0.0) { L->type[g] = 2; break; }
            }
        }
    }
    /* compact ordering: inside nodes then ghosts, each lexicographic (eq. maprij) */
    int ni = 0, ng = 0;
    for (long g = 0; g < nn; ++g) { if (L->type[g] == 1) ++ni; else if (L->type[g] == 2) ++ng; }
    L->ni = ni; L->ng = ng; L->na = ni + ng;
    L->c2g = (long *)malloc(sizeof(long) * (L->na > 0 ? L->na : 1));
    L->g2c = (int *)malloc(sizeof(int) * nn);
    int ci = 0, cg = ni;
    for (long g = 0; g < nn; ++g) {
        L->g2c[g] = -1;
        if (L->type[g] == 1) { L->c2g[ci] = g; L->g2c[g] = ci++; }
    }
    for (long g = 0; g < nn; ++g)
        if (L->type[g] == 2) { L->c2g[cg] = g; L->g2c[g] = cg++; }

    /* ghost geometry */
    L->st = (long *)malloc(sizeof(long) * nst * (ng > 0 ? ng : 1));
    L->w = (double *)malloc(sizeof(double) * nst * (ng > 0 ? ng : 1));
    L->B = (double *)malloc(sizeof(double) * dim * (ng > 0 ? ng : 1));
    L->nrm = (double *)malloc(sizeof(double) * dim * (ng > 0 ? ng : 1));
    L->nrow = (double *)malloc(sizeof(double) * dim * (ng > 0 ? ng : 1));
    L->order = (int *)malloc(sizeof(int) * (ng > 0 ? ng : 1));
    L->bfall = (int *)malloc(sizeof(int) * (ng > 0 ? ng : 1));
    for (int q = 0; q < ng; ++q) {
        long g = L->c2g[ni + q];
        int gi[3];
        unravel(g, n, dim, gi);
        double G[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) G[a] = xcoord(H, L, gi[a]);
        double nt[3] = {0, 0, 0}, nrm[3] = {0, 0, 0};
        grad_phi(H, L, gi, nt);
        double len2 = 0.0;
        for (int a = 0; a < dim; ++a) len2 += nt[a] * nt[a];
        double len = sqrt(len2);
        int m[3] = {1, 1, 1};
        if (len > 0.0)
            for (int a = 0; a < dim; ++a) nrm[a] = nt[a] / len;
        for (int a = 0; a < dim; ++a) m[a] = (nrm[a] >= 0.0) ? 1 : -1;  /* SIGN(0) = +1 */
        for (int a = 0; a < dim; ++a) L->nrm[q * dim + a] = nrm[a];
        /* upwind stencil ST = {G - h (m_x k_x, m_y k_y[, m_z k_z])}, k in {0,1,2}^d */
        /* stencil nodes outside the box keep the ghost's own index and count as
         * inactive (READING: the paper assumes the box is large enough) */
        long *st = &L->st[(long)q * nst];
        char oob[27];
        int any_oob = 0;
        for (int k = 0; k < nst; ++k) {
            int kk = k, idx[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) { idx[a] = gi[a] - m[a] * (kk % 3); kk /= 3; }
            oob[k] = !in_box(idx, n, dim);
            any_oob |= oob[k];
            st[k] = oob[k] ? g : ravel(idx, n, dim);
        }
        /* boundary point B: bisection on the segment P -> G, P = G - 2h n */
        double Bp[3] = {G[0], G[1], G[2]};
        int bfall = 0;
        if (len > 0.0 && any_oob) {
            bfall = 1;
            for (int a = 0; a < dim; ++a) Bp[a] = G[a] - L->phi[g] * nt[a] / len2;
        } else if (len > 0.0) {
            double P[3] = {0, 0, 0}, X[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) P[a] = G[a] - 2.0 * L->h * nrm[a];
            double f0 = phi_tilde(H, L, st, gi, m, P);
            if (f0 < 0.0) {
                /* READING: bisect to full double precision (no early stop) */
                double alo = 0.0, ahi = 1.0;
                for (int it = 0; it < 200; ++it) {
                    double am = 0.5 * (alo + ahi);
                    if (am <= alo || am >= ahi) break;
                    for (int a = 0; a < dim; ++a) X[a] = P[a] + am * (G[a] - P[a]);
                    if (phi_tilde(H, L, st, gi, m, X) < 0.0) alo = am; else ahi = am;
                }
                for (int a = 0; a < dim; ++a) Bp[a] = P[a] + ahi * (G[a] - P[a]);
            } else {
                /* READING: no sign change on PG -> first-order projection along the gradient */
                bfall = 1;
                for (int a = 0; a < dim; ++a) Bp[a] = G[a] - L->phi[g] * nt[a] / len2;
            }
        }
        for (int a = 0; a < dim; ++a) L->B[q * dim + a] = Bp[a];
        L->bfall[q] = bfall;
        double th[3] = {1, 1, 1};
        for (int a = 0; a < dim; ++a) th[a] = m[a] * (Bp[a] - xcoord(H, L, gi[a] - m[a])) / L->h;
        int bad_theta = 0;
        for (int a = 0; a < dim; ++a) if (!(th[a] >= -1.0 && th[a] <= 2.0)) bad_theta = 1;
        /* READING: theta outside [-1, 2] (B found by the first-order projection far from G,
         * e.g. where the level set has a crease): the constant rule, on every level */
        double *w = &L->w[(long)q * nst];
        int order = 2;
        if (H->bctype == 1) {
            int rc = neumann_row(H, L, m, st, oob, any_oob, th, bad_theta, nrm, w, &L->nrow[q * dim], &order);
            if (rc != OR_OK) return rc;
            L->order[q] = order;
            continue;
        }
        for (int a = 0; a < dim; ++a) L->nrow[q * dim + a] = nrm[a];
        /* boundary-row weights (eq. JssD) with the order fallback */
        if (!bad_theta) {
            for (int k = 0; k < nst; ++k) {
                int kk = k; double wk = 1.0;
                for (int a = 0; a < dim; ++a) { wk *= lag2(kk % 3, th[a]); kk /= 3; }
                w[k] = wk;
            }
            for (int k = 0; k < nst; ++k) if (w[k] != 0.0 && (oob[k] || L->type[st[k]] == 0)) order = 1;
            if (order == 1) {
                for (int k = 0; k < nst; ++k) {
                    int kk = k; double wk = 1.0;
                    for (int a = 0; a < dim; ++a) { wk *= lag1(kk % 3, th[a]); kk /= 3; }
                    w[k] = wk;
                }
                for (int k = 0; k < nst; ++k) if (w[k] != 0.0 && (oob[k] || L->type[st[k]] == 0)) order = 0;
            }
        } else {
            order = 0;
        }
        /* READING: a ghost whose own weight w[0] is negative (theta outside
         * [0, 1] on an axis, outside the paper's analysis) cannot meet eq.
         * CFLcond with 0 < tau < 1: in 2-D its row takes the axis rule above,
         * in 3-D (and in 2-D without an inside axis neighbour) the constant rule */
        if (w[0] < 0.0) order = 0;
        if (order == 0 && dim == 2 && axis_row(H, L, g, gi, m, st, oob, Bp, th, w, &order)) {
            for (int a = 0; a < dim; ++a) L->B[q * dim + a] = Bp[a];
            L->bfall[q] = 2;
        } else if (order == 0) {
            for (int k = 0; k < nst; ++k) w[k] = (k == 0) ? 1.0 : 0.0;
        }
        L->order[q] = order;
    }
    return OR_OK;
}

/* Band of inactive fine nodes that the boundary-defect restriction reads:
 * the 3^d neighbourhood of every fine node 2I with I a coarse ghost.
 * For each band node the upwind neighbours q - m_a e_a (m = SIGN of the
 * central-difference normal) that are ghosts or band nodes, with weights
 * |n_a| (READING of the transport-equation extension of the ghost defect
 * along the normal, §3.5.2). */
static int build_band(or_hier *H, int l)
{
    OLevel *F = &H->L[l], *C = &H->L[l + 1];
    int dim = H->dim, n = F->n, nst = H->nst;
    char *flag = (char *)calloc(F->nn, 1);
    for (int q = 0; q < C->ng; ++q) {
        long gc = C->c2g[C->ni + q];
        int ci[3];
        unravel(gc, C->n, dim, ci);
        for (int k = 0; k < nst; ++k) {
            int kk = k, fi[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) { fi[a] = 2 * ci[a] + (kk % 3) - 1; kk /= 3; }
            if (!in_box(fi, n, dim)) continue;
            long gf = ravel(fi, n, dim);
            if (F->type[gf] == 0) flag[gf] = 1;
        }
    }
    int nb = 0;
    for (long g = 0; g < F->nn; ++g) nb += flag[g];
    F->nb = nb;
    F->band = (long *)malloc(sizeof(long) * (nb > 0 ? nb : 1));
    F->bup = (long *)malloc(sizeof(long) * dim * (nb > 0 ? nb : 1));
    F->bwt = (double *)malloc(sizeof(double) * dim * (nb > 0 ? nb : 1));
    int b = 0;
    for (long g = 0; g < F->nn; ++g) if (flag[g]) F->band[b++] = g;
    for (b = 0; b < nb; ++b) {
        long g = F->band[b];
        int gi[3];
        unravel(g, n, dim, gi);
        double nt[3] = {0, 0, 0};
        grad_phi(H, F, gi, nt);
        double len2 = 0.0;
        for (int a = 0; a < dim; ++a) len2 += nt[a] * nt[a];
        double len = sqrt(len2);
        double wsum = 0.0;
        for (int a = 0; a < dim; ++a) {
            double na = len > 0.0 ? nt[a] / len : 0.0;
            int ma = na >= 0.0 ? 1 : -1;
            int up[3] = {gi[0], gi[1], gi[2]};
            up[a] -= ma;
            F->bup[b * dim + a] = -1;
            F->bwt[b * dim + a] = 0.0;
            if (!in_box(up, n, dim)) continue;
            long gu = ravel(up, n, dim);
            if (F->type[gu] == 2 || flag[gu]) {
                F->bup[b * dim + a] = gu;
                F->bwt[b * dim + a] = fabs(na);
                wsum += fabs(na);
            }
        }
        (void)wsum;
    }
    free(flag);
    return OR_OK;
}

static double *dalloc(long n) { return (double *)calloc(n > 0 ? n : 1, sizeof(double)); }

void or_free(or_hier *H);

int or_build(const double *phi, int dim, int n, double lo, double hi, int coarsest_n, int bc, or_hier **out)
{
    *out = NULL;
    if (dim < 2 || dim > 3 || n < 3 || coarsest_n < 3 || !(hi > lo) || bc < 0 || bc > 1) return OR_EINVAL;
    int nlev = 1, nl = n;
    while (nl > coarsest_n) {
        if ((nl - 1) % 2) return OR_EINVAL;
        nl = (nl - 1) / 2 + 1;
        ++nlev;
        if (nlev > MAXLEV) return OR_EINVAL;
    }
    if (nl != coarsest_n) return OR_EINVAL;
    or_hier *H = (or_hier *)calloc(1, sizeof(or_hier));
    H->dim = dim; H->nlev = nlev; H->nst = ipow3(dim); H->lo = lo; H->hi = hi; H->bctype = bc;
    H->p.a = 1e4; H->p.d = 0.1; H->p.m_s = 64.06; H->p.m_c = 100.09;
    H->p.alpha = 0.01; H->p.beta = 0.1; H->p.tau_s = 0.9;
    H->p.nu1 = 2; H->p.nu2 = 2; H->p.ghost_c_new = 1; H->p.band_steps = 3; H->p.ghost_sweeps = 1;
    H->p.ghost_sweeps_coarse = 1; H->p.sweeps_lambda = 0.3;
    H->p.gamma = 1; H->p.lex = 0; H->p.fmg = 0; H->p.krylov_m = 0;
    nl = n;
    for (int l = 0; l < nlev; ++l) {
        OLevel *L = &H->L[l];
        L->n = nl;
        L->h = (hi - lo) / (nl - 1);
        L->nn = 1;
        for (int a = 0; a < dim; ++a) L->nn *= nl;
        L->phi = dalloc(L->nn);
        L->type = (signed char *)calloc(L->nn, 1);
        if (l == 0) {
            memcpy(L->phi, phi, sizeof(double) * L->nn);
        } else {
            OLevel *Fn = &H->L[l - 1];
            for (long g = 0; g < L->nn; ++g) {
                int ci[3], fi[3];
                unravel(g, nl, dim, ci);
                for (int a = 0; a < 3; ++a) fi[a] = 2 * ci[a];
                L->phi[g] = Fn->phi[ravel(fi, Fn->n, dim)];  /* injection of the level set */
            }
        }
        int rc = build_level_geometry(H, l);
        if (rc != OR_OK) { H->nlev = l + 1; or_free(H); return rc; }
        L->s = dalloc(L->nn); L->c = dalloc(L->nn);
        L->rhs_s = dalloc(L->nn); L->rhs_c = dalloc(L->nn);
        L->x_s = dalloc(L->nn); L->x_c = dalloc(L->nn);
        L->r_s = dalloc(L->nn); L->r_c = dalloc(L->nn);
        nl = (nl - 1) / 2 + 1;
    }
    for (int l = 0; l + 1 < nlev; ++l) build_band(H, l);
    H->bs = dalloc(H->L[0].nn);
    H->bc = dalloc(H->L[0].nn);
    *out = H;
    return OR_OK;
}

void or_free(or_hier *H)
{
    if (!H) return;
    for (int l = 0; l < H->nlev; ++l) {
        OLevel *L = &H->L[l];
        free(L->phi); free(L->type); free(L->c2g); free(L->g2c);
        free(L->st); free(L->w); free(L->B); free(L->nrm); free(L->nrow); free(L->order); free(L->bfall);
        free(L->band); free(L->bup); free(L->bwt);
        free(L->s); free(L->c); free(L->rhs_s); free(L->rhs_c);
        free(L->x_s); free(L->x_c); free(L->r_s); free(L->r_c);
    }
    free(H->lu); free(H->piv); free(H->bs); free(H->bc);
    free(H);
}

int or_set_params(or_hier *H, double a, double d, double m_s, double m_c, double alpha, double beta,
                  double tau_s, int nu1, int nu2, int ghost_c_new, int band_steps, int ghost_sweeps,
                  int ghost_sweeps_coarse, double sweeps_lambda, int gamma, int lex, int fmg,
                  int krylov_m)
{
    if (gamma < 1 || gamma > 2 || lex < 0 || lex > 1 || fmg < 0 || fmg > 2 || krylov_m < 0 || krylov_m > 200)
        return OR_EINVAL;
    H->p.fmg = fmg;
    H->p.krylov_m = krylov_m;
    H->p.gamma = gamma;
    H->p.lex = lex;
    H->p.ghost_sweeps = ghost_sweeps;
    H->p.ghost_sweeps_coarse = ghost_sweeps_coarse;
    H->p.sweeps_lambda = sweeps_lambda;
    H->p.a = a; H->p.d = d; H->p.m_s = m_s; H->p.m_c = m_c;
    H->p.alpha = alpha; H->p.beta = beta; H->p.tau_s = tau_s;
    H->p.nu1 = nu1; H->p.nu2 = nu2; H->p.ghost_c_new = ghost_c_new; H->p.band_steps = band_steps;
    return OR_OK;
}

int or_num_levels(const or_hier *H) { return H->nlev; }

int or_level_info(const or_hier *H, int l, int *n, double *h, int *ni, int *ng, int *nb)
{
    if (l < 0 || l >= H->nlev) return OR_EINVAL;
    *n = H->L[l].n; *h = H->L[l].h; *ni = H->L[l].ni; *ng = H->L[l].ng; *nb = H->L[l].nb;
    return OR_OK;
}

int or_compact_to_grid(const or_hier *H, int l, long *out)
{
    if (l < 0 || l >= H->nlev) return OR_EINVAL;
    memcpy(out, H->L[l].c2g, sizeof(long) * H->L[l].na);
    return OR_OK;
}

/* ghost table of level l: ST entries as compact indices (-1 for inactive nodes),
 * weights, boundary points, normals, order, fallback flags */
int or_ghost_table(const or_hier *H, int l, int *st_compact, double *w, double *B, double *nrm,
                   double *nrow, int *order, int *bfall)
{
    if (l < 0 || l >= H->nlev) return OR_EINVAL;
    const OLevel *L = &H->L[l];
    int nst = H->nst, dim = H->dim;
    for (long k = 0; k < (long)L->ng * nst; ++k) { st_compact[k] = L->g2c[L->st[k]]; w[k] = L->w[k]; }
    for (long k = 0; k < (long)L->ng * dim; ++k) { B[k] = L->B[k]; nrm[k] = L->nrm[k]; nrow[k] = L->nrow[k]; }
    for (int q = 0; q < L->ng; ++q) { order[q] = L->order[q]; bfall[q] = L->bfall[q]; }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* discrete operators (§3.3 eqs. FDs, FDc, BCs; §3.4 Jacobian)          */
/* ------------------------------------------------------------------ */

/* L^s_h(s,c) at inside node g: reaction plus the 5/7-point nonlinear diffusion
 * with the 1/h^2 factor (READING: the printed operator omits it). */
static double Ls_h(const or_hier *H, const OLevel *L, const double *s, const double *c, long g)
{
    const OPar *p = &H->p;
    double phg = phi_por(p, c[g]);
    double diff = 0.0;
    for (int a = 0; a < H->dim; ++a) {
        long sa = stride_of(L->n, a);
        long nb[2] = {g - sa, g + sa};
        for (int e = 0; e < 2; ++e)
            diff += (phi_por(p, c[nb[e]]) + phg) * (s[nb[e]] - s[g]);
    }
    return -(p->a / p->m_c) * phg * s[g] * c[g] + p->d / (2.0 * L->h * L->h) * diff;
}

static double Lc_h(const or_hier *H, const double *s, const double *c, long g)
{
    const OPar *p = &H->p;
    return -(p->a / p->m_s) * phi_por(p, c[g]) * s[g] * c[g];
}

/* Jacobian entries of an inside row (exact derivatives of FDs/FDc; READINGs
 * fix the garbled printed forms of eqs. JssI, JscI, JcsI, JccI).
 * Neighbour e = 2a + (0: minus, 1: plus). */
typedef struct { double ss_d, sc_d, cs_d, cc_d; double ss_n[6], sc_n[6]; long nb[6]; } JRow;

static void jrow_inside(const or_hier *H, const OLevel *L, long g, JRow *J)
{
    const OPar *p = &H->p;
    const double *s = L->s, *c = L->c;
    double dt = H->dt;
    double kap = p->d / (4.0 * L->h * L->h);
    double ks = p->a / p->m_c, kc = p->a / p->m_s;
    double phg = phi_por(p, c[g]);
    double sum_ss = 0.0, sum_sc = 0.0;
    for (int a = 0; a < H->dim; ++a) {
        long sa = stride_of(L->n, a);
        for (int e = 0; e < 2; ++e) {
            long q = e ? g + sa : g - sa;
            double phq = phi_por(p, c[q]);
            J->nb[2 * a + e] = q;
            J->ss_n[2 * a + e] = -kap * (phq + phg);
            J->sc_n[2 * a + e] = kap * p->alpha * (s[g] - s[q]);
            sum_ss += phq + phg;
            sum_sc += s[g] - s[q];
        }
    }
    J->ss_d = phg / dt + 0.5 * ks * phg * c[g] + kap * sum_ss;
    J->sc_d = p->alpha * s[g] / dt + 0.5 * ks * (p->alpha * s[g] * c[g] + phg * s[g]) + kap * p->alpha * sum_sc;
    J->cs_d = 0.5 * kc * phg * c[g];
    J->cc_d = 1.0 / dt + 0.5 * kc * (p->alpha * s[g] * c[g] + phg * s[g]);
}

/* c-row diagonal entries (inside and ghost rows) */
static void jrow_c(const or_hier *H, const OLevel *L, long g, double *cs_d, double *cc_d)
{
    const OPar *p = &H->p;
    double kc = p->a / p->m_s;
    double phg = phi_por(p, L->c[g]);
    *cs_d = 0.5 * kc * phg * L->c[g];
    *cc_d = 1.0 / H->dt + 0.5 * kc * (p->alpha * L->s[g] * L->c[g] + phg * L->s[g]);
}

/* y = J x on level l (full-grid vectors), all active rows */
static void apply_J_grid(const or_hier *H, int l, const double *xs, const double *xc, double *ys, double *yc)
{
    const OLevel *L = &H->L[l];
    int nd = 2 * H->dim;
    for (int r = 0; r < L->ni; ++r) {
        long g = L->c2g[r];
        JRow J;
        jrow_inside(H, L, g, &J);
        double v = J.ss_d * xs[g] + J.sc_d * xc[g];
        for (int e = 0; e < nd; ++e) v += J.ss_n[e] * xs[J.nb[e]] + J.sc_n[e] * xc[J.nb[e]];
        ys[g] = v;
        yc[g] = J.cs_d * xs[g] + J.cc_d * xc[g];
    }
    for (int q = 0; q < L->ng; ++q) {
        long g = L->c2g[L->ni + q];
        double v = 0.0;
        for (int k = 0; k < H->nst; ++k) v += L->w[(long)q * H->nst + k] * xs[L->st[(long)q * H->nst + k]];
        ys[g] = v;
        double cs, cc;
        jrow_c(H, L, g, &cs, &cc);
        yc[g] = cs * xs[g] + cc * xc[g];
    }
}

/* ------------------------------------------------------------------ */
/* compact <-> grid                                                    */
/* ------------------------------------------------------------------ */

static void to_grid(const OLevel *L, const double *v, double *gs, double *gc)
{
    for (int r = 0; r < L->na; ++r) { gs[L->c2g[r]] = v[r]; gc[L->c2g[r]] = v[L->na + r]; }
}

static void from_grid(const OLevel *L, const double *gs, const double *gc, double *v)
{
    for (int r = 0; r < L->na; ++r) { v[r] = gs[L->c2g[r]]; v[L->na + r] = gc[L->c2g[r]]; }
}

static double norm_inf_grid(const OLevel *L, const double *a, const double *b)
{
    double m = 0.0;
    for (int r = 0; r < L->na; ++r) {
        long g = L->c2g[r];
        double x = fabs(a[g]), y = fabs(b[g]);
        if (x > m || x != x) m = x;
        if (y > m || y != y) m = y;
        if (m != m) return m;
    }
    return m;
}

/* ------------------------------------------------------------------ */
/* linearisation point on every level                                  */
/* ------------------------------------------------------------------ */

/* coarse (s, c) from the next finer level: injection where the fine centre
 * is active, otherwise the full-weighting average over active fine
 * neighbours (READING: the paper only says the coarse operator is built
 * "with the same technique"; parity unpinned, affects the convergence factor
 * only). */
static void inject_state(or_hier *H, int l)
{
    OLevel *F = &H->L[l], *C = &H->L[l + 1];
    int dim = H->dim, nst = H->nst;
    for (long g = 0; g < C->nn; ++g) { C->s[g] = 0.0; C->c[g] = 0.0; }
    for (int r = 0; r < C->na; ++r) {
        long gc = C->c2g[r];
        int ci[3], fi[3] = {0, 0, 0};
        unravel(gc, C->n, dim, ci);
        for (int a = 0; a < dim; ++a) fi[a] = 2 * ci[a];
        long gf = ravel(fi, F->n, dim);
        if (F->type[gf] != 0) { C->s[gc] = F->s[gf]; C->c[gc] = F->c[gf]; continue; }
        double ws = 0.0, vs = 0.0, vc = 0.0;
        for (int k = 0; k < nst; ++k) {
            int kk = k, idx[3] = {0, 0, 0};
            double wk = 1.0;
            for (int a = 0; a < dim; ++a) { int dlt = kk % 3 - 1; kk /= 3; idx[a] = fi[a] + dlt; wk *= (dlt == 0) ? 0.5 : 0.25; }
            if (!in_box(idx, F->n, dim)) continue;
            long q = ravel(idx, F->n, dim);
            if (F->type[q] == 0) continue;
            ws += wk; vs += wk * F->s[q]; vc += wk * F->c[q];
        }
        C->s[gc] = vs / ws; C->c[gc] = vc / ws;
    }
}

static int lu_factor(double *A, int *piv, int n);

static int assemble_dense(const or_hier *H, int l, double *A)
{
    const OLevel *L = &H->L[l];
    int na = L->na, N = 2 * na;
    for (long k = 0; k < (long)N * N; ++k) A[k] = 0.0;
    int nd = 2 * H->dim;
    for (int r = 0; r < L->ni; ++r) {
        long g = L->c2g[r];
        JRow J;
        jrow_inside(H, L, g, &J);
        A[(long)r * N + r] += J.ss_d;
        A[(long)r * N + na + r] += J.sc_d;
        for (int e = 0; e < nd; ++e) {
            int q = L->g2c[J.nb[e]];
            A[(long)r * N + q] += J.ss_n[e];
            A[(long)r * N + na + q] += J.sc_n[e];
        }
        A[(long)(na + r) * N + r] += J.cs_d;
        A[(long)(na + r) * N + na + r] += J.cc_d;
    }
    for (int q = 0; q < L->ng; ++q) {
        int r = L->ni + q;
        long g = L->c2g[r];
        for (int k = 0; k < H->nst; ++k) {
            double wk = L->w[(long)q * H->nst + k];
            if (wk == 0.0) continue;
            A[(long)r * N + L->g2c[L->st[(long)q * H->nst + k]]] += wk;
        }
        double cs, cc;
        jrow_c(H, L, g, &cs, &cc);
        A[(long)(na + r) * N + r] += cs;
        A[(long)(na + r) * N + na + r] += cc;
    }
    return OR_OK;
}

/* set the linearisation point W (finest, compact) and the time step; builds
 * the coarse coefficients and factors the coarsest operator */
int or_set_linearization(or_hier *H, const double *W, double dt)
{
    OLevel *L0 = &H->L[0];
    H->dt = dt;
    for (long g = 0; g < L0->nn; ++g) { L0->s[g] = 0.0; L0->c[g] = 0.0; }
    to_grid(L0, W, L0->s, L0->c);
    for (int l = 0; l + 1 < H->nlev; ++l) inject_state(H, l);
    int lc = H->nlev - 1;
    int N = 2 * H->L[lc].na;
    free(H->lu); free(H->piv);
    H->lu = dalloc((long)N * N);
    H->piv = (int *)malloc(sizeof(int) * (N > 0 ? N : 1));
    H->lu_n = N;
    assemble_dense(H, lc, H->lu);
    H->lu_ok = (lu_factor(H->lu, H->piv, N) == 0);
    H->lin_set = 1;
    return H->lu_ok ? OR_OK : OR_ENONFINITE;
}

/* ------------------------------------------------------------------ */
/* dense LU with partial pivoting (coarsest solve; READING: the paper    */
/* does not name the coarsest solver)                                  */
/* ------------------------------------------------------------------ */

static int lu_factor(double *A, int *piv, int n)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[(long)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(A[(long)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (best == 0.0 || best != best) return -1;
        if (p != k)
            for (int j = 0; j < n; ++j) { double t = A[(long)k * n + j]; A[(long)k * n + j] = A[(long)p * n + j]; A[(long)p * n + j] = t; }
        for (int i = k + 1; i < n; ++i) {
            double f = A[(long)i * n + k] / A[(long)k * n + k];
            A[(long)i * n + k] = f;
            for (int j = k + 1; j < n; ++j) A[(long)i * n + j] -= f * A[(long)k * n + j];
        }
    }
    return 0;
}

static void lu_solve(const double *A, const int *piv, int n, double *b)
{
    for (int k = 0; k < n; ++k) {
        int p = piv[k];
        if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
    }
    for (int i = 0; i < n; ++i) {
        double v = b[i];
        for (int j = 0; j < i; ++j) v -= A[(long)i * n + j] * b[j];
        b[i] = v;
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = b[i];
        for (int j = i + 1; j < n; ++j) v -= A[(long)i * n + j] * b[j];
        b[i] = v / A[(long)i * n + i];
    }
}

int or_lu_solve_dense(double *A, double *b, int n)
{
    int *piv = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int rc = lu_factor(A, piv, n);
    if (rc == 0) lu_solve(A, piv, n, b);
    free(piv);
    return rc == 0 ? OR_OK : OR_ENONFINITE;
}

/* ------------------------------------------------------------------ */
/* multigrid components (§3.5)                                         */
/* ------------------------------------------------------------------ */

/* number of ghost relaxations per smoothing step on a level (READING; the
 * paper relaxes the ghosts once): ghost_sweeps, or ghost_sweeps_coarse where
 * the level's diffusion number d dt / h^2 is below sweeps_lambda.  On such
 * mass-dominated levels the inside rows hardly couple to the ghosts and the
 * boundary error is removed by the ghost relaxation alone. */
static int level_sweeps(const or_hier *H, const OLevel *L)
{
    const double lam = H->p.d * H->dt / (L->h * L->h);
    return lam < H->p.sweeps_lambda ? H->p.ghost_sweeps_coarse : H->p.ghost_sweeps;
}

/* one smoothing step on level l (§3.5.1): collective Gauss-Seidel on the
 * inside nodes in red-black order, or in the lexicographic order of the map
 * (eq. maprij) with lex = 1 (2x2 block solve with P of eq. matrixP), then the
 * ghost relaxation of eq. RelGhost on all ghosts at once. */
static void smooth_level(or_hier *H, int l)
{
    OLevel *L = &H->L[l];
    int nd = 2 * H->dim, dim = H->dim;
    double *xs = L->x_s, *xc = L->x_c;
    const int passes = H->p.lex ? 1 : 2;
    for (int colour = 0; colour < passes; ++colour) {
        for (int r = 0; r < L->ni; ++r) {
            long g = L->c2g[r];
            int gi[3];
            unravel(g, L->n, dim, gi);
            if (!H->p.lex && ((gi[0] + gi[1] + gi[2]) & 1) != colour) continue;
            JRow J;
            jrow_inside(H, L, g, &J);
            double rs = L->rhs_s[g] - (J.ss_d * xs[g] + J.sc_d * xc[g]);
            for (int e = 0; e < nd; ++e) rs -= J.ss_n[e] * xs[J.nb[e]] + J.sc_n[e] * xc[J.nb[e]];
            double rc = L->rhs_c[g] - (J.cs_d * xs[g] + J.cc_d * xc[g]);
            double det = J.ss_d * J.cc_d - J.sc_d * J.cs_d;
            double ds = (J.cc_d * rs - J.sc_d * rc) / det;
            double dc = (J.ss_d * rc - J.cs_d * rs) / det;
            xs[g] += ds;
            xc[g] += dc;
        }
    }
    /* ghosts: s-row relaxation with tau^s (Jacobi over the ghost set), then
     * the c-row with the updated (READING) or previous delta s */
    int ng = L->ng, nst = H->nst;
    double *news = dalloc(ng), *olds = dalloc(ng);
    const int sweeps = level_sweeps(H, L);
    for (int gs = 0; gs < sweeps; ++gs) {
    for (int q = 0; q < ng; ++q) {
        long g = L->c2g[L->ni + q];
        double v = 0.0;
        for (int k = 0; k < nst; ++k) v += L->w[(long)q * nst + k] * xs[L->st[(long)q * nst + k]];
        olds[q] = xs[g];
        news[q] = xs[g] + tau_level(H, L) * (L->rhs_s[g] - v);
    }
    for (int q = 0; q < ng; ++q) xs[L->c2g[L->ni + q]] = news[q];
    for (int q = 0; q < ng; ++q) {
        long g = L->c2g[L->ni + q];
        double cs, cc;
        jrow_c(H, L, g, &cs, &cc);
        double dsv = H->p.ghost_c_new ? xs[g] : olds[q];
        xc[g] += (L->rhs_c[g] - (cs * dsv + cc * xc[g])) / cc;
    }
    }
    free(news); free(olds);
}

/* defect r = rhs - J x on level l (§3.5.2); returns its infinity norm */
static double defect_level(or_hier *H, int l)
{
    OLevel *L = &H->L[l];
    for (long g = 0; g < L->nn; ++g) { L->r_s[g] = 0.0; L->r_c[g] = 0.0; }
    double *ys = dalloc(L->nn), *yc = dalloc(L->nn);
    apply_J_grid(H, l, L->x_s, L->x_c, ys, yc);
    for (int r = 0; r < L->na; ++r) {
        long g = L->c2g[r];
        L->r_s[g] = L->rhs_s[g] - ys[g];
        L->r_c[g] = L->rhs_c[g] - yc[g];
    }
    free(ys); free(yc);
    return norm_inf_grid(L, L->r_s, L->r_c);
}

/* extension of the ghost defect r^s to the band of inactive nodes (§3.5.2):
 * the ghost value is carried outward along the normal, the steady state of
 * d r/d tau + n . grad r = 0 with upwind differences, built in band_steps
 * layers (READING of "a few steps"; parity unpinned).  Ghosts start
 * assigned; in each layer an unassigned band node with at least one assigned
 * upwind neighbour takes the |n_a|-weighted mean of those neighbours (the
 * plain mean if all their |n_a| vanish) and becomes assigned for the next
 * layer.  ext[g] marks ghosts and assigned band nodes. */
static void extend_band(or_hier *H, int l, char *ext)
{
    OLevel *L = &H->L[l];
    int nb = L->nb, dim = H->dim;
    double *nxt = dalloc(nb);
    char *newly = (char *)calloc(nb > 0 ? nb : 1, 1);
    for (long g = 0; g < L->nn; ++g) ext[g] = (L->type[g] == 2);
    for (int b = 0; b < nb; ++b) L->r_s[L->band[b]] = 0.0;
    for (int step = 0; step < H->p.band_steps; ++step) {
        for (int b = 0; b < nb; ++b) {
            newly[b] = 0;
            if (ext[L->band[b]]) continue;
            double v = 0.0, ws = 0.0, vm = 0.0;
            int cnt = 0;
            for (int a = 0; a < dim; ++a) {
                long gu = L->bup[b * dim + a];
                if (gu < 0 || !ext[gu]) continue;
                v += L->bwt[b * dim + a] * L->r_s[gu];
                ws += L->bwt[b * dim + a];
                vm += L->r_s[gu];
                ++cnt;
            }
            if (cnt == 0) continue;
            nxt[b] = ws > 0.0 ? v / ws : vm / cnt;
            newly[b] = 1;
        }
        for (int b = 0; b < nb; ++b)
            if (newly[b]) { L->r_s[L->band[b]] = nxt[b]; ext[L->band[b]] = 1; }
    }
    free(nxt); free(newly);
}

/* restriction of the defect from level l to level l+1 (§3.5.2, eqs. Fstencil,
 * Fstencilgen and Fig. Neigh): full weighting modified near the boundary.
 * Per axis the weights [1,2,1]/4 become [2,2,0]/4 ([0,2,2]/4) when the fine
 * axis neighbour at +1 (-1) is excluded and [0,4,0]/4 when both are; the
 * stencil is the tensor product and any weight that lands on an excluded
 * fine node goes to the centre.  Inside equations exclude non-inside fine
 * nodes; boundary equations exclude inside fine nodes and inactive nodes the
 * band extension did not reach; the c-defect uses full weighting renormalised over active fine
 * nodes (READINGs; the three printed stencils pin the inside rule). */
static void restrict_level(or_hier *H, int l, const char *ext)
{
    OLevel *F = &H->L[l], *C = &H->L[l + 1];
    int dim = H->dim, nst = H->nst;
    for (long g = 0; g < C->nn; ++g) { C->rhs_s[g] = 0.0; C->rhs_c[g] = 0.0; }
    for (int r = 0; r < C->na; ++r) {
        long gc = C->c2g[r];
        int ci[3], fc[3] = {0, 0, 0};
        unravel(gc, C->n, dim, ci);
        for (int a = 0; a < dim; ++a) fc[a] = 2 * ci[a];
        long gfc = ravel(fc, F->n, dim);
        int coarse_inside = (C->type[gc] == 1);
        /* per-axis weights for the s-defect */
        double wa[3][3];
        for (int a = 0; a < dim; ++a) {
            int ex[2];
            for (int e = 0; e < 2; ++e) {
                int idx[3] = {fc[0], fc[1], fc[2]};
                idx[a] += e ? 1 : -1;
                if (!in_box(idx, F->n, dim)) { ex[e] = 1; continue; }
                long qe = ravel(idx, F->n, dim);
                int t = F->type[qe];
                ex[e] = coarse_inside ? (t != 1) : (t == 1 || (t == 0 && !ext[qe]));
            }
            /* index 0: -1, 1: centre, 2: +1 */
            if (!ex[0] && !ex[1]) { wa[a][0] = 0.25; wa[a][1] = 0.5; wa[a][2] = 0.25; }
            else if (!ex[0] && ex[1]) { wa[a][0] = 0.5; wa[a][1] = 0.5; wa[a][2] = 0.0; }
            else if (ex[0] && !ex[1]) { wa[a][0] = 0.0; wa[a][1] = 0.5; wa[a][2] = 0.5; }
            else { wa[a][0] = 0.0; wa[a][1] = 1.0; wa[a][2] = 0.0; }
        }
        double vs = 0.0, wcentre = 0.0;
        double vc = 0.0, wcs = 0.0;
        for (int k = 0; k < nst; ++k) {
            int kk = k, idx[3] = {0, 0, 0};
            double wk = 1.0, wf = 1.0;
            for (int a = 0; a < dim; ++a) {
                int dlt = kk % 3 - 1; kk /= 3;
                idx[a] = fc[a] + dlt;
                wk *= wa[a][dlt + 1];
                wf *= (dlt == 0) ? 0.5 : 0.25;
            }
            if (!in_box(idx, F->n, dim)) { wcentre += wk; continue; }
            long q = ravel(idx, F->n, dim);
            int t = F->type[q];
            int excluded = coarse_inside ? (t != 1) : (t == 1 || (t == 0 && !ext[q]));
            if (q == gfc) excluded = 0;
            if (excluded) wcentre += wk;
            else vs += wk * F->r_s[q];
            if (t != 0) { vc += wf * F->r_c[q]; wcs += wf; }
        }
        vs += wcentre * F->r_s[gfc];
        C->rhs_s[gc] = vs;
        C->rhs_c[gc] = wcs > 0.0 ? vc / wcs : 0.0;
    }
}

/* bilinear (trilinear) prolongation of the coarse correction onto the
 * active fine nodes, renormalised over active coarse nodes (§3.5.3;
 * READING near inactive coarse nodes), added to x */
static void prolong_add_level(or_hier *H, int l)
{
    OLevel *F = &H->L[l], *C = &H->L[l + 1];
    int dim = H->dim;
    int ncorner = 1 << dim;
    for (int r = 0; r < F->na; ++r) {
        long gf = F->c2g[r];
        int fi[3];
        unravel(gf, F->n, dim, fi);
        double ws = 0.0, es = 0.0, ec = 0.0;
        for (int k = 0; k < ncorner; ++k) {
            int idx[3] = {0, 0, 0};
            double wk = 1.0;
            int skip = 0;
            for (int a = 0; a < dim; ++a) {
                int bit = (k >> a) & 1;
                if (fi[a] % 2 == 0) { if (bit) { skip = 1; break; } idx[a] = fi[a] / 2; }
                else { idx[a] = (fi[a] - 1) / 2 + bit; wk *= 0.5; }
            }
            if (skip) continue;
            long q = ravel(idx, C->n, dim);
            if (C->type[q] == 0) continue;
            ws += wk; es += wk * C->x_s[q]; ec += wk * C->x_c[q];
        }
        if (ws > 0.0) { F->x_s[gf] += es / ws; F->x_c[gf] += ec / ws; }
    }
}

static void coarse_solve_level(or_hier *H)
{
    int lc = H->nlev - 1;
    OLevel *L = &H->L[lc];
    int na = L->na, N = 2 * na;
    double *b = dalloc(N);
    from_grid(L, L->rhs_s, L->rhs_c, b);
    lu_solve(H->lu, H->piv, N, b);
    for (long g = 0; g < L->nn; ++g) { L->x_s[g] = 0.0; L->x_c[g] = 0.0; }
    to_grid(L, b, L->x_s, L->x_c);
    free(b);
}

/* one V(nu1, nu2) cycle (gamma = 1) or W(nu1, nu2) cycle (gamma = 2: the
 * coarse-grid correction is two cycles on the next level, the second from the
 * first one's result) on level l with the level's rhs and x (§3.5, §4) */
static void vcycle_rec(or_hier *H, int l)
{
    if (l == H->nlev - 1) { coarse_solve_level(H); return; }
    OLevel *F = &H->L[l], *C = &H->L[l + 1];
    for (int i = 0; i < H->p.nu1; ++i) smooth_level(H, l);
    defect_level(H, l);
    char *ext = (char *)malloc(F->nn);
    extend_band(H, l, ext);
    restrict_level(H, l, ext);
    free(ext);
    for (long g = 0; g < C->nn; ++g) { C->x_s[g] = 0.0; C->x_c[g] = 0.0; }
    for (int i = 0; i < H->p.gamma; ++i) vcycle_rec(H, l + 1);
    prolong_add_level(H, l);
    for (int i = 0; i < H->p.nu2; ++i) smooth_level(H, l);
}

/* full multigrid (the paper names it as a first solver, §3.5; READING of how):
 * with x = 0 on level 0 the right-hand side is restricted level by level with
 * the same boundary-aware restriction as the cycle's defect; the coarsest
 * problem is solved; on every finer level the prolongated coarser solution is
 * the start of one cycle on that level */
static void fmg_level0(or_hier *H)
{
    int L = H->nlev;
    for (int l = 0; l + 1 < L; ++l) {
        OLevel *F = &H->L[l], *C = &H->L[l + 1];
        defect_level(H, l);          /* x_l = 0: the defect is the right-hand side */
        char *ext = (char *)malloc(F->nn);
        extend_band(H, l, ext);
        restrict_level(H, l, ext);
        free(ext);
        for (long g = 0; g < C->nn; ++g) { C->x_s[g] = 0.0; C->x_c[g] = 0.0; }
    }
    coarse_solve_level(H);
    for (int l = L - 2; l >= 0; --l) {
        prolong_add_level(H, l);
        vcycle_rec(H, l);
    }
}

/* ------------------------------------------------------------------ */
/* public per-component entry points (compact vectors)                 */
/* ------------------------------------------------------------------ */

static void load_rhs_x(or_hier *H, int l, const double *rhs, const double *x)
{
    OLevel *L = &H->L[l];
    for (long g = 0; g < L->nn; ++g) { L->rhs_s[g] = L->rhs_c[g] = L->x_s[g] = L->x_c[g] = 0.0; }
    if (rhs) to_grid(L, rhs, L->rhs_s, L->rhs_c);
    if (x) to_grid(L, x, L->x_s, L->x_c);
}

int or_apply_J(or_hier *H, int l, const double *x, double *y)
{
    if (!H->lin_set || l < 0 || l >= H->nlev) return OR_EINVAL;
    OLevel *L = &H->L[l];
    double *xs = dalloc(L->nn), *xc = dalloc(L->nn), *ys = dalloc(L->nn), *yc = dalloc(L->nn);
    to_grid(L, x, xs, xc);
    apply_J_grid(H, l, xs, xc, ys, yc);
    from_grid(L, ys, yc, y);
    free(xs); free(xc); free(ys); free(yc);
    return OR_OK;
}

int or_smooth(or_hier *H, int l, const double *rhs, double *x, int nsweeps)
{
    if (!H->lin_set || l < 0 || l >= H->nlev) return OR_EINVAL;
    OLevel *L = &H->L[l];
    load_rhs_x(H, l, rhs, x);
    for (int i = 0; i < nsweeps; ++i) smooth_level(H, l);
    from_grid(L, L->x_s, L->x_c, x);
    return OR_OK;
}

int or_defect(or_hier *H, int l, const double *rhs, const double *x, double *r, double *nrm)
{
    if (!H->lin_set || l < 0 || l >= H->nlev) return OR_EINVAL;
    OLevel *L = &H->L[l];
    load_rhs_x(H, l, rhs, x);
    double v = defect_level(H, l);
    if (r) from_grid(L, L->r_s, L->r_c, r);
    if (nrm) *nrm = v;
    return OR_OK;
}

/* restriction of a fine defect r (compact, level l) to the coarse rhs (level l+1);
 * band values (full-grid indices) are returned for inspection if requested */
int or_restrict(or_hier *H, int l, const double *r, double *rc, double *band_out)
{
    if (l < 0 || l + 1 >= H->nlev) return OR_EINVAL;
    OLevel *F = &H->L[l], *C = &H->L[l + 1];
    for (long g = 0; g < F->nn; ++g) { F->r_s[g] = 0.0; F->r_c[g] = 0.0; }
    to_grid(F, r, F->r_s, F->r_c);
    char *ext = (char *)malloc(F->nn);
    extend_band(H, l, ext);
    if (band_out) for (int b = 0; b < F->nb; ++b) band_out[b] = ext[F->band[b]] ? F->r_s[F->band[b]] : NAN;
    restrict_level(H, l, ext);
    free(ext);
    from_grid(C, C->rhs_s, C->rhs_c, rc);
    return OR_OK;
}

int or_band_nodes(const or_hier *H, int l, long *band)
{
    if (l < 0 || l >= H->nlev) return OR_EINVAL;
    memcpy(band, H->L[l].band, sizeof(long) * H->L[l].nb);
    return OR_OK;
}

int or_prolong_add(or_hier *H, int l, const double *ec, double *x)
{
    if (l < 0 || l + 1 >= H->nlev) return OR_EINVAL;
    OLevel *F = &H->L[l], *C = &H->L[l + 1];
    for (long g = 0; g < C->nn; ++g) { C->x_s[g] = 0.0; C->x_c[g] = 0.0; }
    to_grid(C, ec, C->x_s, C->x_c);
    for (long g = 0; g < F->nn; ++g) { F->x_s[g] = 0.0; F->x_c[g] = 0.0; }
    to_grid(F, x, F->x_s, F->x_c);
    prolong_add_level(H, l);
    from_grid(F, F->x_s, F->x_c, x);
    return OR_OK;
}

/* linearisation point of level l (compact), for inspection */
int or_level_state(const or_hier *H, int l, double *W)
{
    if (l < 0 || l >= H->nlev) return OR_EINVAL;
    from_grid(&H->L[l], H->L[l].s, H->L[l].c, W);
    return OR_OK;
}

int or_coarse_solve(or_hier *H, const double *rhs, double *x)
{
    if (!H->lin_set || !H->lu_ok) return OR_EINVAL;
    int lc = H->nlev - 1;
    load_rhs_x(H, lc, rhs, NULL);
    coarse_solve_level(H);
    from_grid(&H->L[lc], H->L[lc].x_s, H->L[lc].x_c, x);
    return OR_OK;
}

int or_vcycle(or_hier *H, int l, const double *rhs, double *x, double *res)
{
    if (!H->lin_set || !H->lu_ok || l < 0 || l >= H->nlev) return OR_EINVAL;
    OLevel *L = &H->L[l];
    load_rhs_x(H, l, rhs, x);
    vcycle_rec(H, l);
    double v = defect_level(H, l);
    from_grid(L, L->x_s, L->x_c, x);
    if (res) *res = v;
    return OR_OK;
}

/* dense matrix of level l (2Na x 2Na, row-major), for direct-solve checks */
int or_assemble_dense(or_hier *H, int l, double *A)
{
    if (!H->lin_set || l < 0 || l >= H->nlev) return OR_EINVAL;
    return assemble_dense(H, l, A);
}

/* sparse matrix of level l in COO form (row, col, value); *nnz in: capacity, out: count */
int or_assemble_coo(or_hier *H, int l, int *rows, int *cols, double *vals, long *nnz)
{
    if (!H->lin_set || l < 0 || l >= H->nlev) return OR_EINVAL;
    const OLevel *L = &H->L[l];
    int na = L->na, nd = 2 * H->dim;
    long cap = *nnz, k = 0;
#define PUSH(R, Cc, V) do { if (k < cap) { rows[k] = (R); cols[k] = (Cc); vals[k] = (V); } ++k; } while (0)
    for (int r = 0; r < L->ni; ++r) {
        long g = L->c2g[r];
        JRow J;
        jrow_inside(H, L, g, &J);
        PUSH(r, r, J.ss_d);
        PUSH(r, na + r, J.sc_d);
        for (int e = 0; e < nd; ++e) {
            int q = L->g2c[J.nb[e]];
            PUSH(r, q, J.ss_n[e]);
            PUSH(r, na + q, J.sc_n[e]);
        }
        PUSH(na + r, r, J.cs_d);
        PUSH(na + r, na + r, J.cc_d);
    }
    for (int q = 0; q < L->ng; ++q) {
        int r = L->ni + q;
        long g = L->c2g[r];
        for (int kk = 0; kk < H->nst; ++kk) {
            double wk = L->w[(long)q * H->nst + kk];
            if (wk == 0.0) continue;
            PUSH(r, L->g2c[L->st[(long)q * H->nst + kk]], wk);
        }
        double cs, cc;
        jrow_c(H, L, g, &cs, &cc);
        PUSH(na + r, r, cs);
        PUSH(na + r, na + r, cc);
    }
#undef PUSH
    int rc = (k <= cap) ? OR_OK : OR_EINVAL;
    *nnz = k;
    return rc;
}

/* ------------------------------------------------------------------ */
/* Crank-Nicolson step with Newton-Raphson (§3.1, §3.4)                */
/* ------------------------------------------------------------------ */

/* explicit half of the Crank-Nicolson step at W^n (§3.1 eq. discTime,
 * §3.3 eqs. FDs, FDc): b^s = phi(c^n) s^n / dt + L^s_h(W^n)/2 on inside
 * nodes, b^c = c^n / dt + L^c_h(W^n)/2 on inside and ghost nodes, plus the
 * trapezoidal average of the source terms of §4.1 when given (compact
 * [f1 | f2] vectors at t_n and t_{n+1}). */
static void explicit_half(or_hier *H, const double *Wn, const double *fn, const double *fnp1)
{
    OLevel *L = &H->L[0];
    double dt = H->dt;
    double *s = dalloc(L->nn), *c = dalloc(L->nn);
    to_grid(L, Wn, s, c);
    for (long g = 0; g < L->nn; ++g) { H->bs[g] = 0.0; H->bc[g] = 0.0; }
    int na = L->na;
    for (int r = 0; r < na; ++r) {
        long g = L->c2g[r];
        if (r < L->ni)
            H->bs[g] = phi_por(&H->p, c[g]) * s[g] / dt + 0.5 * Ls_h(H, L, s, c, g);
        H->bc[g] = c[g] / dt + 0.5 * Lc_h(H, s, c, g);
        if (fn && fnp1) {
            if (r < L->ni) H->bs[g] += 0.5 * (fn[r] + fnp1[r]);
            H->bc[g] += 0.5 * (fn[na + r] + fnp1[na + r]);
        }
    }
    free(s); free(c);
}

/* Newton residual F(W) (eqs. FDs, FDc on inside nodes, FDc and the boundary
 * row on ghosts; READING: the boundary row is s~(B) - s_b so that its
 * derivative is the +weights of eq. JssD) */
static double residual_F(or_hier *H, const double *W, const double *sb, double *Fv)
{
    OLevel *L = &H->L[0];
    double dt = H->dt;
    double *s = dalloc(L->nn), *c = dalloc(L->nn);
    to_grid(L, W, s, c);
    int na = L->na;
    double m = 0.0;
    for (int r = 0; r < na; ++r) {
        long g = L->c2g[r];
        double fs;
        if (r < L->ni) {
            fs = phi_por(&H->p, c[g]) * s[g] / dt - 0.5 * Ls_h(H, L, s, c, g) - H->bs[g];
        } else {
            int q = r - L->ni;
            double v = 0.0;
            for (int k = 0; k < H->nst; ++k) v += L->w[(long)q * H->nst + k] * s[L->st[(long)q * H->nst + k]];
            fs = v - sb[q];
        }
        double fc = c[g] / dt - 0.5 * Lc_h(H, s, c, g) - H->bc[g];
        Fv[r] = fs;
        Fv[na + r] = fc;
        double x = fabs(fs), y = fabs(fc);
        if (x > m || x != x) m = x;
        if (y > m || y != y) m = y;
    }
    free(s); free(c);
    return m;
}

int or_residual(or_hier *H, const double *W, const double *Wn, double dt, const double *sb,
                const double *fn, const double *fnp1, double *Fv, double *nrm)
{
    H->dt = dt;
    explicit_half(H, Wn, fn, fnp1);
    double v = residual_F(H, W, sb, Fv);
    if (nrm) *nrm = v;
    return OR_OK;
}

typedef struct {
    int newton_iters, vcycles;
    double res_inf, rho_last, rho_geo, dw_rel;
} or_stats;

/* one Crank-Nicolson step: W (compact) holds W^n on entry and W^{n+1} on
 * OR_OK; it is left unchanged on failure.  Newton stops when
 * min(||F||_inf, ||dW||_inf/||W||_inf) < newton_tol after at least one
 * iteration (§3.4); each linear system is solved by V-cycles from zero until
 * the defect drops below lin_rtol * ||F||_inf or cycles_max cycles ran
 * (READING: the paper gives no inner tolerance).  rho_hist (optional,
 * capacity rho_cap) receives the convergence factor of every cycle. */
/* ------------------------------------------------------------------ */
/* Krylov acceleration of the linear solves (krylov_m > 0)             */
/* ------------------------------------------------------------------ */

static double dot(const double *a, const double *b, int N)
{
    double t = 0.0;
    for (int r = 0; r < N; ++r) t += a[r] * b[r];
    return t;
}

/* z = one V-cycle on level 0 from a zero correction with right-hand side v
 * (compact vectors) */
static void precondition(or_hier *H, const double *v, double *z)
{
    OLevel *L = &H->L[0];
    for (long g = 0; g < L->nn; ++g) { L->rhs_s[g] = L->rhs_c[g] = L->x_s[g] = L->x_c[g] = 0.0; }
    to_grid(L, v, L->rhs_s, L->rhs_c);
    vcycle_rec(H, 0);
    from_grid(L, L->x_s, L->x_c, z);
}

/* Flexible GMRES(m) for J x = F on level 0 (Saad's flexible variant: the
 * preconditioned vectors Z_j = M(V_j) are kept, so the preconditioner need not
 * be a fixed linear map), M one V-cycle from zero.  The new direction is made
 * orthogonal to V_0..V_j by classical Gram-Schmidt applied twice (all inner
 * products of a pass taken before the pass subtracts them); the small
 * least-squares problem is reduced by Givens rotations, whose last rotated
 * entry |g_{j+1}| is the 2-norm of the defect F - J x_j.  The solve starts
 * from x = 0, stops when that norm is at most rtol |F|_2 or after cycles_max
 * V-cycles, and restarts from its current x every m iterations.  x: N values
 * on exit; cycles, rho: V-cycles taken and the last ratio of consecutive
 * defect norms (the caller's statistics).  Pinned against a sparse direct
 * solve of the assembled Jacobian, with and without restarts. */
static void krylov_solve(or_hier *H, const double *F, double *x, int m, double rtol, int cycles_max,
                         int *cycles, double *rho_last, double *logsum, int *nrho, double *rho_hist,
                         int rho_cap)
{
    const int N = 2 * H->L[0].na;
    double *V = dalloc((long)(m + 1) * N), *Z = dalloc((long)m * N), *w = dalloc(N), *r = dalloc(N);
    double *Hh = dalloc((long)(m + 1) * m), *cs = dalloc(m), *sn = dalloc(m), *g = dalloc(m + 1),
           *y = dalloc(m), *hp = dalloc(m + 1);
    for (int i = 0; i < N; ++i) { x[i] = 0.0; r[i] = F[i]; }
    const double target = rtol * sqrt(dot(F, F, N));
    double beta = sqrt(dot(r, r, N));
    int used = 0;
    while (beta > target && used < cycles_max) {
        for (int i = 0; i < N; ++i) V[i] = r[i] / beta;
        for (long e = 0; e < (long)(m + 1) * m; ++e) Hh[e] = 0.0;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        double prev = beta;
        int k = 0;
        for (int j = 0; j < m && used < cycles_max; ++j) {
            precondition(H, V + (long)j * N, Z + (long)j * N);
            ++used;
            or_apply_J(H, 0, Z + (long)j * N, w);
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = 0; i <= j; ++i) hp[i] = dot(w, V + (long)i * N, N);
                for (int i = 0; i <= j; ++i) {
                    Hh[(long)i * m + j] += hp[i];
                    for (int q = 0; q < N; ++q) w[q] -= hp[i] * V[(long)i * N + q];
                }
            }
            const double hn = sqrt(dot(w, w, N));
            Hh[(long)(j + 1) * m + j] = hn;
            for (int q = 0; q < N; ++q) V[(long)(j + 1) * N + q] = hn > 0.0 ? w[q] / hn : 0.0;
            /* the earlier rotations on column j, then the one that zeroes its last entry */
            for (int i = 0; i < j; ++i) {
                const double a = Hh[(long)i * m + j], b = Hh[(long)(i + 1) * m + j];
                Hh[(long)i * m + j] = cs[i] * a + sn[i] * b;
                Hh[(long)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            const double a = Hh[(long)j * m + j], b = Hh[(long)(j + 1) * m + j];
            const double d = sqrt(a * a + b * b);
            cs[j] = d > 0.0 ? a / d : 1.0;
            sn[j] = d > 0.0 ? b / d : 0.0;
            Hh[(long)j * m + j] = d;
            Hh[(long)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            const double res = fabs(g[j + 1]);
            *rho_last = prev > 0.0 ? res / prev : 0.0;
            if (*rho_last > 0.0) *logsum += log(*rho_last);
            if (rho_hist && *nrho < rho_cap) rho_hist[*nrho] = *rho_last;
            ++*nrho;
            prev = res;
            if (res <= target || hn == 0.0 || !(res == res)) break;
        }
        /* x += Z y with R y = g, R the rotated k x k upper triangle */
        for (int i = k - 1; i >= 0; --i) {
            double t = g[i];
            for (int q = i + 1; q < k; ++q) t -= Hh[(long)i * m + q] * y[q];
            y[i] = t / Hh[(long)i * m + i];
        }
        for (int i = 0; i < k; ++i)
            for (int q = 0; q < N; ++q) x[q] += y[i] * Z[(long)i * N + q];
        or_apply_J(H, 0, x, w);
        for (int q = 0; q < N; ++q) r[q] = F[q] - w[q];
        beta = sqrt(dot(r, r, N));
        if (!(beta == beta)) break;
    }
    *cycles += used;
    free(V); free(Z); free(w); free(r); free(Hh); free(cs); free(sn); free(g); free(y); free(hp);
}

/* the Krylov solve alone, for its tests: x (compact) from F at the current
 * linearisation point; returns the V-cycles taken */
int or_krylov_solve(or_hier *H, const double *F, double *x, int m, double rtol, int cycles_max)
{
    if (!H->lin_set || m < 1 || m > 200 || cycles_max < 0) return OR_EINVAL;
    int cycles = 0, nrho = 0;
    double rho = 0.0, logsum = 0.0;
    krylov_solve(H, F, x, m, rtol, cycles_max, &cycles, &rho, &logsum, &nrho, NULL, 0);
    return cycles;
}

int or_newton_cn_step(or_hier *H, double *W, double dt, const double *sb, const double *fn,
                      const double *fnp1, double newton_tol, int newton_max, double lin_rtol,
                      int cycles_max, or_stats *st, double *rho_hist, int rho_cap)
{
    OLevel *L = &H->L[0];
    int na = L->na, N = 2 * na;
    H->dt = dt;
    double *Wk = dalloc(N), *Fv = dalloc(N), *Dx = dalloc(N);
    memcpy(Wk, W, sizeof(double) * N);
    explicit_half(H, W, fn, fnp1);
    double nF = residual_F(H, Wk, sb, Fv);
    int rc = OR_ENOCONV, cycles = 0, nrho = 0;
    double rho_last = 0.0, logsum = 0.0, dwrel = 0.0;
    int it;
    for (it = 1; it <= newton_max; ++it) {
        if (!(nF == nF) || isinf(nF)) { rc = OR_ENONFINITE; break; }
        if (or_set_linearization(H, Wk, dt) != OR_OK) { rc = OR_ENONFINITE; break; }
        if (H->p.krylov_m > 0) {
            krylov_solve(H, Fv, Dx, H->p.krylov_m, lin_rtol, cycles_max, &cycles, &rho_last, &logsum, &nrho,
                         rho_hist, rho_cap);
            goto update;
        }
        /* J dW = F by V-cycles from dW = 0 */
        for (long g = 0; g < L->nn; ++g) { L->rhs_s[g] = L->rhs_c[g] = L->x_s[g] = L->x_c[g] = 0.0; }
        to_grid(L, Fv, L->rhs_s, L->rhs_c);
        double rprev = nF;
        for (int q = 0; q < cycles_max; ++q) {
            if (rprev <= lin_rtol * nF) break;
            if (q == 0 && (H->p.fmg == 2 || (H->p.fmg == 1 && it == 1))) fmg_level0(H);
            else vcycle_rec(H, 0);
            double rq = defect_level(H, 0);
            ++cycles;
            rho_last = rprev > 0.0 ? rq / rprev : 0.0;
            if (rho_last > 0.0) logsum += log(rho_last);
            if (rho_hist && nrho < rho_cap) rho_hist[nrho] = rho_last;
            ++nrho;
            rprev = rq;
            if (!(rq == rq) || isinf(rq)) break;
        }
        from_grid(L, L->x_s, L->x_c, Dx);
    update:;
        double nW = 0.0, nD = 0.0;
        for (int r = 0; r < N; ++r) {
            double a = fabs(Wk[r]), b = fabs(Dx[r]);
            if (a > nW) nW = a;
            if (b > nD || b != b) nD = b;
        }
        for (int r = 0; r < N; ++r) Wk[r] -= Dx[r];
        nF = residual_F(H, Wk, sb, Fv);
        dwrel = nW > 0.0 ? nD / nW : nD;
        if (!(nF == nF) || isinf(nF) || !(dwrel == dwrel)) { rc = OR_ENONFINITE; break; }
        if ((nF < dwrel ? nF : dwrel) < newton_tol) { rc = OR_OK; break; }
    }
    if (st) {
        st->newton_iters = it > newton_max ? newton_max : it;
        st->vcycles = cycles;
        st->res_inf = nF;
        st->rho_last = rho_last;
        st->rho_geo = nrho > 0 ? exp(logsum / nrho) : 0.0;
        st->dw_rel = dwrel;
    }
    if (rc == OR_OK) memcpy(W, Wk, sizeof(double) * N);
    free(Wk); free(Fv); free(Dx);
    return rc;
}

/* Newton step with an externally supplied exact linear solve is done in the
 * tests (scipy) through or_residual and or_assemble_coo. */

/* ------------------------------------------------------------------ */
/* level-set and initial-data preparation on a full grid (§2, §3.3)    */
/* ------------------------------------------------------------------ */

/* value of array v at node g shifted by s (+-1) along axis a; the node itself
 * where the neighbour leaves the box (zero one-sided difference there) */
static double nbv(const double *v, long g, const int *gi, int n, int a, long sa, int s)
{
    int k = gi[a] + s;
    if (k < 0 || k >= n) return v[g];
    return v[g + s * sa];
}

/* Re-initialisation of a level set towards the signed distance (§2): the
 * pseudo-time equation d phi/d mu = sgn(phi0) (1 - |grad phi|) from phi = phi0,
 * forward Euler with d mu = h / dim.  READING (the paper cites the PDE only):
 * the scheme with the subcell fix of Russo and Smereka, which keeps the zero
 * level set where phi0 puts it.  Nodes with a sign change of phi0 towards an
 * axis neighbour relax to D = h phi0 / dphi0, their distance estimated from
 * phi0, with dphi0 the largest of the central, forward and backward undivided
 * gradient norms of phi0:
 *     phi <- phi - (d mu / h) (sgn(phi0) |phi| - D);
 * every other node takes the upwind (Godunov) update
 *     phi <- phi - d mu sgn(phi0) (|grad phi| - 1).
 * One-sided differences vanish at the box edge.  iters steps. */
int or_reinitialize(const double *phi0, int dim, int n, double h, int iters, double *phi)
{
    if (dim < 2 || dim > 3 || n < 2 || !(h > 0.0) || iters < 0) return OR_EINVAL;
    long nn = 1;
    for (int a = 0; a < dim; ++a) nn *= n;
    double *cur = dalloc(nn), *nxt = dalloc(nn), *D = dalloc(nn);
    char *near = (char *)calloc(nn, 1);
    for (long g = 0; g < nn; ++g) {
        int gi[3];
        unravel(g, n, dim, gi);
        double p0 = phi0[g], c2 = 0.0, f2 = 0.0, b2 = 0.0;
        int nr = 0;
        for (int a = 0; a < dim; ++a) {
            long sa = stride_of(n, a);
            double pm = nbv(phi0, g, gi, n, a, sa, -1), pp = nbv(phi0, g, gi, n, a, sa, +1);
            if (p0 * pm <= 0.0 || p0 * pp <= 0.0) nr = 1;
            double c = (pp - pm) / 2.0, f = pp - p0, bk = p0 - pm;
            c2 += c * c;
            f2 += f * f;
            b2 += bk * bk;
        }
        double dp = sqrt(c2);
        if (sqrt(f2) > dp) dp = sqrt(f2);
        if (sqrt(b2) > dp) dp = sqrt(b2);
        if (dp < 1e-300) dp = 1e-300;
        near[g] = (char)nr;
        D[g] = h * p0 / dp;
    }
    memcpy(cur, phi0, sizeof(double) * nn);
    double dmu = h / dim;
    for (int it = 0; it < iters; ++it) {
        for (long g = 0; g < nn; ++g) {
            double p0 = phi0[g];
            double sg = p0 > 0.0 ? 1.0 : (p0 < 0.0 ? -1.0 : 0.0);
            if (near[g]) {
                nxt[g] = cur[g] - (dmu / h) * (sg * fabs(cur[g]) - D[g]);
                continue;
            }
            int gi[3];
            unravel(g, n, dim, gi);
            double g2 = 0.0;
            for (int a = 0; a < dim; ++a) {
                long sa = stride_of(n, a);
                double dm = (cur[g] - nbv(cur, g, gi, n, a, sa, -1)) / h;   /* backward */
                double dpp = (nbv(cur, g, gi, n, a, sa, +1) - cur[g]) / h;  /* forward */
                double u, w;
                if (p0 > 0.0) { u = dm > 0.0 ? dm : 0.0; w = dpp < 0.0 ? dpp : 0.0; }
                else { u = dm < 0.0 ? dm : 0.0; w = dpp > 0.0 ? dpp : 0.0; }
                double m = u * u > w * w ? u * u : w * w;
                g2 += m;
            }
            nxt[g] = cur[g] - dmu * sg * (sqrt(g2) - 1.0);
        }
        double *tt = cur; cur = nxt; nxt = tt;
    }
    memcpy(phi, cur, sizeof(double) * nn);
    free(cur); free(nxt); free(D); free(near);
    return OR_OK;
}

/* Level set from a mask (§2, the paper's treatment of image data): phi = -1
 * where mask != 0 (inside), +1 elsewhere, then iters explicit steps of the
 * heat equation, phi += (1 / (2 dim)) sum over the axes of the second
 * difference (READING: the step size, the largest stable one for the
 * five/seven-point Laplacian; the paper says "a few iterations"). */
int or_levelset_from_mask(const unsigned char *mask, int dim, int n, int iters, double *phi)
{
    if (dim < 2 || dim > 3 || n < 2 || iters < 0) return OR_EINVAL;
    long nn = 1;
    for (int a = 0; a < dim; ++a) nn *= n;
    double *cur = dalloc(nn), *nxt = dalloc(nn);
    for (long g = 0; g < nn; ++g) cur[g] = mask[g] ? -1.0 : 1.0;
    double k = 1.0 / (2.0 * dim);
    for (int it = 0; it < iters; ++it) {
        for (long g = 0; g < nn; ++g) {
            int gi[3];
            unravel(g, n, dim, gi);
            double lap = 0.0;
            for (int a = 0; a < dim; ++a) {
                long sa = stride_of(n, a);
                lap += nbv(cur, g, gi, n, a, sa, -1) - 2.0 * cur[g] + nbv(cur, g, gi, n, a, sa, +1);
            }
            nxt[g] = cur[g] + k * lap;
        }
        double *t = cur; cur = nxt; nxt = t;
    }
    memcpy(phi, cur, sizeof(double) * nn);
    free(cur); free(nxt);
    return OR_OK;
}

/* one pseudo-time stage of the extension along the outward normal: where
 * known[g] is 0, v <- v - dtau (n . grad_up v - src), grad_up the one-sided
 * difference against the normal component (upwind: information flows out of
 * the domain along n); src = NULL for 0 */
static void extend_stage(const double *nrm, const char *known, const double *src, int dim, int n, long nn, double h,
                         int iters, double *v)
{
    double *nxt = dalloc(nn);
    double dtau = h / dim;
    for (int it = 0; it < iters; ++it) {
        for (long g = 0; g < nn; ++g) {
            if (known[g]) { nxt[g] = v[g]; continue; }
            int gi[3];
            unravel(g, n, dim, gi);
            double adv = 0.0;
            for (int a = 0; a < dim; ++a) {
                long sa = stride_of(n, a);
                double na = nrm[g * dim + a], d;
                if (na > 0.0) d = (v[g] - nbv(v, g, gi, n, a, sa, -1)) / h;
                else if (na < 0.0) d = (nbv(v, g, gi, n, a, sa, +1) - v[g]) / h;
                else d = 0.0;
                adv += na * d;
            }
            nxt[g] = v[g] - dtau * (adv - (src ? src[g] : 0.0));
        }
        memcpy(v, nxt, sizeof(double) * nn);
    }
    free(nxt);
}

/* Second-order extrapolation of data q from the inside (phi < 0) to the rest
 * of the grid (§3.3: initial data at the ghosts), by the PDE approach the paper
 * cites (Aslam): with n = grad phi / |grad phi| (central differences),
 *   q_n = n . grad q and q_nn = n . grad q_n by central differences where their
 *   stencils are known, then, each over iters pseudo-time steps,
 *   q_nn extended constantly along n   (d/dtau q_nn + n . grad q_nn = 0),
 *   q_n  extended linearly              (d/dtau q_n + n . grad q_n = q_nn),
 *   q    extended                       (d/dtau q + n . grad q = q_n).
 * Values at phi < 0 are returned unchanged. */
int or_extrapolate(const double *phi, int dim, int n, double h, const double *q, int iters, double *out)
{
    if (dim < 2 || dim > 3 || n < 3 || !(h > 0.0) || iters < 0) return OR_EINVAL;
    long nn = 1;
    for (int a = 0; a < dim; ++a) nn *= n;
    double *nrm = dalloc(nn * dim), *qn = dalloc(nn), *qnn = dalloc(nn);
    char *k0 = (char *)calloc(nn, 1), *k1 = (char *)calloc(nn, 1), *k2 = (char *)calloc(nn, 1);
    for (long g = 0; g < nn; ++g) {
        int gi[3];
        unravel(g, n, dim, gi);
        double gr[3] = {0, 0, 0}, l2 = 0.0;
        for (int a = 0; a < dim; ++a) {
            long sa = stride_of(n, a);
            if (gi[a] > 0 && gi[a] < n - 1) gr[a] = (phi[g + sa] - phi[g - sa]) / (2.0 * h);
            else if (gi[a] == 0) gr[a] = (phi[g + sa] - phi[g]) / h;
            else gr[a] = (phi[g] - phi[g - sa]) / h;
            l2 += gr[a] * gr[a];
        }
        double l = sqrt(l2);
        for (int a = 0; a < dim; ++a) nrm[g * dim + a] = l > 0.0 ? gr[a] / l : 0.0;
        k0[g] = phi[g] < 0.0;
    }
    /* known set of a derived quantity: a known node whose axis neighbours are all known and in the box */
    for (int pass = 0; pass < 2; ++pass) {
        const char *kin = pass ? k1 : k0;
        char *kout = pass ? k2 : k1;
        const double *vin = pass ? qn : q;
        double *vout = pass ? qnn : qn;
        for (long g = 0; g < nn; ++g) {
            int gi[3];
            unravel(g, n, dim, gi);
            int ok = kin[g];
            for (int a = 0; a < dim && ok; ++a) {
                long sa = stride_of(n, a);
                if (gi[a] == 0 || gi[a] == n - 1 || !kin[g - sa] || !kin[g + sa]) ok = 0;
            }
            kout[g] = (char)ok;
            double v = 0.0;
            if (ok)
                for (int a = 0; a < dim; ++a) {
                    long sa = stride_of(n, a);
                    v += nrm[g * dim + a] * (vin[g + sa] - vin[g - sa]) / (2.0 * h);
                }
            vout[g] = v;
        }
    }
    for (long g = 0; g < nn; ++g) out[g] = k0[g] ? q[g] : 0.0;
    extend_stage(nrm, k2, NULL, dim, n, nn, h, iters, qnn);
    extend_stage(nrm, k1, qnn, dim, n, nn, h, iters, qn);
    extend_stage(nrm, k0, qn, dim, n, nn, h, iters, out);
    free(nrm); free(qn); free(qnn); free(k0); free(k1); free(k2);
    return OR_OK;
}
