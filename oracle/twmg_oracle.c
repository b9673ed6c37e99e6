/*
 * twmg oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 CPU implementation of geometric multigrid
 * with tweed / wireframe / checkerboard / zebra block Gauss-Seidel smoothing for
 * the nonuniform-grid Poisson problem of Bewley, Mashayek, Cavaglieri & Luchini,
 * "Tweed and wireframe: accelerated relaxation algorithms for multigrid solution
 * of elliptic PDEs on stretched structured grids" (arXiv 2110.08389).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  It shares no code, header, table or constant with the
 * GPU library; nothing in the product path may call it.
 *
 * Everything is double precision.  Build with -O2 -ffp-contract=off so that the
 * arithmetic is exactly the order written here.
 *
 * Threads (OpenMP, orc_set_threads): the only parallel loops are over the
 * blocks of one colour inside a half-sweep (uncoupled: each reads the other
 * colour and writes only its own points) and over the nodes of the operator,
 * defect, transfer and norm loops (each output written by one iteration; the
 * maximum is exact in any order).  Every value is computed by the same
 * expression in the same order whatever the thread count, so the results are
 * bitwise identical to one thread.
 *
 * Conventions (readings of the paper that it leaves open are marked READING):
 *  - nodes are 0-based, i = 0..n (n = number of cells on that axis); interior
 *    unknowns are 1..n-1 on every axis; node arrays are row-major with x fastest:
 *    idx = (l*(ny+1) + j)*(nx+1) + i.                       (READING: index base)
 *  - the operator is the paper's five-point (seven-point in 3D) nonuniform
 *    difference form of Section 2 (problem DP): row p reads
 *        W_i u_{i-1} + E_i u_{i+1} + S_j u_{j-1} + N_j u_{j+1} (+ B, T) + C u_p = f_p
 *    with C = -(sum of the off-diagonal coefficients).  It is not symmetric on a
 *    stretched grid; the adjoint uses the exact transpose of the interior block.
 *  - the coarse operators are re-discretised on the coarse coordinates
 *    x^{l-1}_I = x^l_{2I} (Section 4), not Galerkin products.   (READING)
 *  - coarsening stops once an axis has an odd number of cells or only 2 cells,
 *    so the usual coarsest grid is 3 nodes per axis (one unknown).  (READING)
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_MAXLEV 32
#define ORC_SLOTS 3 /* sweeps per relaxation: 3 for 3D alternating-direction zebra */

/* number of OpenMP threads of the parallel loops (1 = the plain serial order) */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }

/* smoother kinds */
enum { ORC_TWEED = 0, ORC_WIREFRAME = 1, ORC_CHECKER = 2, ORC_ZEBRA_X = 3, ORC_ZEBRA_Y = 4,
       ORC_ZEBRA_Z = 5, ORC_ADZ = 6, ORC_ALT_TW = 7 };
/* stretching kinds */
enum { ORC_UNIFORM = 0, ORC_TANH_WALL = 1, ORC_TANH_CENTRE = 2, ORC_SINH_CENTRE = 3, ORC_EXPLICIT = 4 };
/* block shapes */
enum { BLK_POINT = 0, BLK_PATH = 1, BLK_SPIDER = 2, BLK_RING = 3 };

/* ------------------------------------------------------------------------ */
/* Geometry: Section 5, equations (tanh) and (tanh_inv); sinh centre clustering */
/* ------------------------------------------------------------------------ */

/* Node coordinates x_0..x_n on [0, L].
 *  ORC_TANH_WALL  : eq. (tanh),     x_i = (L/2){1 + tanh[c(2i/n - 1)]/tanh c}
 *  ORC_TANH_CENTRE: eq. (tanh_inv), two shifted tanh halves meeting at the centre
 *  ORC_SINH_CENTRE: x_i = L{1/2 + sinh[b(2i/n - 1)]/(2 sinh b)}  (centre clustering)
 *  ORC_UNIFORM    : x_i = L i/n */
int orc_coords(int kind, double c, int n, double L, double *x)
{
    if (n < 1) return -1;
    for (int i = 0; i <= n; ++i) {
        double s = (double)i / (double)n;
        switch (kind) {
        case ORC_UNIFORM: x[i] = L * s; break;
        case ORC_TANH_WALL: x[i] = (L / 2.0) * (1.0 + tanh(c * (2.0 * s - 1.0)) / tanh(c)); break;
        case ORC_TANH_CENTRE:
            if (2 * i <= n) x[i] = (L / 2.0) * tanh(2.0 * c * s) / tanh(c);
            else x[i] = (L / 2.0) * (2.0 - tanh(c * (2.0 - 2.0 * s)) / tanh(c));
            break;
        case ORC_SINH_CENTRE: x[i] = L * (0.5 + sinh(c * (2.0 * s - 1.0)) / (2.0 * sinh(c))); break;
        default: return -1;
        }
    }
    /* pin the end points exactly */
    x[0] = 0.0;
    x[n] = L;
    return 0;
}

/* Section 2: with dxm = x_i - x_{i-1} (Delta x_{i-1/2}), dxp = x_{i+1} - x_i
 * (Delta x_{i+1/2}) and dx = (x_{i+1} - x_{i-1})/2 (Delta x_i):
 *     W_i = 1/(dx dxm),  E_i = 1/(dx dxp).   Defined for interior i = 1..n-1. */
void orc_coefs(int n, const double *x, double *lo, double *hi)
{
    for (int i = 0; i <= n; ++i) { lo[i] = 0.0; hi[i] = 0.0; }
    for (int i = 1; i < n; ++i) {
        double dxm = x[i] - x[i - 1];
        double dxp = x[i + 1] - x[i];
        double dx = (x[i + 1] - x[i - 1]) / 2.0;
        lo[i] = 1.0 / (dx * dxm);
        hi[i] = 1.0 / (dx * dxp);
    }
}

/* The axis-wise heterogeneous, anisotropic form of problem (CP) (Section 2)
 * with a diagonal conductivity whose a-th entry depends on x_a only,
 * sigma_aa = s_a(x_a): the flux form of the same three-point difference,
 *     W_i = s_{i-1/2}/(dx dxm),  E_i = s_{i+1/2}/(dx dxp),
 * with sig[k] = s_{k+1/2}, the value on cell k = [x_k, x_{k+1}] (n values).
 * sig == NULL is s = 1 (orc_coefs).                        (READING: extension) */
void orc_coefs_sigma(int n, const double *x, const double *sig, double *lo, double *hi)
{
    orc_coefs(n, x, lo, hi);
    if (!sig) return;
    for (int i = 1; i < n; ++i) {
        double dxm = x[i] - x[i - 1];
        double dxp = x[i + 1] - x[i];
        double dx = (x[i + 1] - x[i - 1]) / 2.0;
        lo[i] = sig[i - 1] / (dx * dxm);
        hi[i] = sig[i] / (dx * dxp);
    }
}

/* Coarse-cell conductivity (READING: the paper re-discretises on the coarse
 * coordinates and leaves heterogeneous media to standard methods): coarse cell
 * I covers fine cells 2I and 2I+1 in series, so its value is their
 * length-weighted harmonic mean, (h0 + h1)/(h0/s0 + h1/s1) -- the conductance
 * of the two cells in series, which keeps the coarse flux of a piecewise
 * linear-in-1/s profile exact. */
static void coarse_sigma(int nc, const double *xf, const double *sf, double *sc)
{
    for (int I = 0; I < nc; ++I) {
        double h0 = xf[2 * I + 1] - xf[2 * I], h1 = xf[2 * I + 2] - xf[2 * I + 1];
        sc[I] = (h0 + h1) / (h0 / sf[2 * I] + h1 / sf[2 * I + 1]);
    }
}

/* ------------------------------------------------------------------------ */
/* Grid hierarchy                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n[3];          /* cells per axis (n[2] = 0 in 2D)       */
    int np[3];         /* nodes per axis = n+1 (np[2] = 1 in 2D) */
    long nn;           /* total nodes                            */
    double *x[3];      /* coordinates                            */
    double *sig[3];    /* per-cell conductivity along each axis (NULL: 1) */
    double *lo[3], *hi[3];
    /* block partition for up to three smoother motifs (slots 0, 1, 2: the
     * sweeps of one relaxation, in order) */
    int nblk[ORC_SLOTS];
    int *bstart[ORC_SLOTS];    /* block b occupies pts[bstart[b] .. bstart[b+1]) */
    int *bpts[ORC_SLOTS];      /* node indices, ordered per the block shape      */
    int *bshape[ORC_SLOTS];    /* BLK_*                                          */
    int *bcolour[ORC_SLOTS];   /* 0 = red, 1 = black                             */
    int *bnleg[ORC_SLOTS];     /* spider: number of legs                         */
    int *blegstart[ORC_SLOTS]; /* spider: offset into blegs                      */
    int *blegs[ORC_SLOTS];     /* spider: leg lengths (points, excl. branch)     */
    int kind[ORC_SLOTS];       /* motif kind of each slot (-1 = unused)          */
    /* coarsest direct solve (banded LU, no pivoting) */
    double *band;      /* factorised band                                */
    int bw;            /* half bandwidth                                 */
    long nunk;         /* interior unknowns                              */
} orc_level;

typedef struct {
    int dim;
    int nlev;          /* level 0 = finest here (reverse of the paper's p..0 numbering) */
    int smoother;
    int transpose;     /* 1: operate with the transposed interior operator (adjoint) */
    orc_level lev[ORC_MAXLEV];
} orc_mg;

static inline long nid(const orc_level *L, int i, int j, int l)
{
    return ((long)l * L->np[1] + j) * L->np[0] + i;
}
static inline void ncoord(const orc_level *L, long p, int *c)
{
    c[0] = (int)(p % L->np[0]);
    c[1] = (int)((p / L->np[0]) % L->np[1]);
    c[2] = (int)(p / ((long)L->np[0] * L->np[1]));
}
static inline int is_interior(const orc_level *L, int dim, const int *c)
{
    for (int a = 0; a < dim; ++a)
        if (c[a] < 1 || c[a] > L->n[a] - 1) return 0;
    return 1;
}
static inline long stride(const orc_level *L, int a)
{
    return a == 0 ? 1 : (a == 1 ? L->np[0] : (long)L->np[0] * L->np[1]);
}

/* Coefficient of row c (interior) toward its neighbour c + dir*e_a.
 * Forward operator: W/S/B toward -1, E/N/T toward +1.
 * Transposed operator (adjoint): entry A[p, p+e] of A^T is A[p+e, p], i.e. the
 * neighbour's coefficient pointing back at p; couplings to boundary nodes are
 * dropped because the adjoint unknowns vanish there. */
static inline double coef(const orc_mg *M, const orc_level *L, int a, int ia, int dir)
{
    if (!M->transpose) return dir < 0 ? L->lo[a][ia] : L->hi[a][ia];
    int nb = ia + dir;
    if (nb < 1 || nb > L->n[a] - 1) return 0.0;
    return dir < 0 ? L->hi[a][nb] : L->lo[a][nb];
}
/* C_{ij} = -(W_i + E_i + S_j + N_j) (Section 2); the same diagonal for A^T. */
static inline double diagc(const orc_mg *M, const orc_level *L, const int *c)
{
    double s = 0.0;
    for (int a = 0; a < M->dim; ++a) s += L->lo[a][c[a]] + L->hi[a][c[a]];
    return -s;
}

/* ------------------------------------------------------------------------ */
/* Block labels (Section 3 motifs; Section 7 for 3D tweed)                   */
/* ------------------------------------------------------------------------ */
/* A block is a connected set of interior points with equal label; colour 0
 * (red) is relaxed first.  READING (figures are absent from the source):
 *  tweed 2D   : k = max(i',j'), i' = min(i, nx-i), j' = min(j, ny-j);
 *               red iff k odd (the corners, k = 1, are red).
 *  wireframe  : r = min(i',j'); red iff r odd (the outermost box is red).
 *  checker    : each point its own block; red iff i+j(+l) even.
 *  zebra x/y/z: lines along that axis; red iff the first interior line (2D: j odd;
 *               3D: sum of the two cross indices even).
 *  tweed 3D   : sort (i',j',l') -> s1<=s2<=s3; label (s2,s3); red iff s2+s3 even. */
static void label_of(int kind, int dim, const orc_level *L, const int *c, long *lab, int *col)
{
    int p[3] = { 0, 0, 0 };
    for (int a = 0; a < dim; ++a) {
        int v = c[a], w = L->n[a] - c[a];
        p[a] = v < w ? v : w;
    }
    switch (kind) {
    case ORC_TWEED:
        if (dim == 2) {
            int k = p[0] > p[1] ? p[0] : p[1];
            *lab = k;
            *col = (k % 2 == 1) ? 0 : 1;
        } else {
            int s[3] = { p[0], p[1], p[2] };
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2 - a; ++b)
                    if (s[b] > s[b + 1]) { int t = s[b]; s[b] = s[b + 1]; s[b + 1] = t; }
            *lab = (long)s[1] * 100000L + s[2];
            *col = ((s[1] + s[2]) % 2 == 0) ? 0 : 1;
        }
        break;
    case ORC_WIREFRAME: {
        int r = p[0] < p[1] ? p[0] : p[1];
        *lab = r;
        *col = (r % 2 == 1) ? 0 : 1;
        break;
    }
    case ORC_CHECKER: {
        *lab = nid(L, c[0], c[1], dim == 3 ? c[2] : 0);
        int s = c[0] + c[1] + (dim == 3 ? c[2] : 0);
        *col = (s % 2 == 0) ? 0 : 1;
        break;
    }
    case ORC_ZEBRA_X:
        if (dim == 2) { *lab = c[1]; *col = (c[1] % 2 == 1) ? 0 : 1; }
        else { *lab = (long)c[1] * 100000L + c[2]; *col = ((c[1] + c[2]) % 2 == 0) ? 0 : 1; }
        break;
    case ORC_ZEBRA_Y:
        if (dim == 2) { *lab = c[0]; *col = (c[0] % 2 == 1) ? 0 : 1; }
        else { *lab = (long)c[0] * 100000L + c[2]; *col = ((c[0] + c[2]) % 2 == 0) ? 0 : 1; }
        break;
    case ORC_ZEBRA_Z:
        *lab = (long)c[0] * 100000L + c[1];
        *col = ((c[0] + c[1]) % 2 == 0) ? 0 : 1;
        break;
    default: *lab = -1; *col = 0;
    }
}

/* ------------------------------------------------------------------------ */
/* Block extraction: connected components of equal label, then each block is */
/* ordered as a point, a path, a spider (legs tip -> branch) or a ring.      */
/* ------------------------------------------------------------------------ */

static int build_blocks(orc_mg *M, orc_level *L, int slot, int kind)
{
    int dim = M->dim;
    long nn = L->nn;
    long *lab = (long *)malloc(sizeof(long) * nn);
    int *col = (int *)malloc(sizeof(int) * nn);
    int *bid = (int *)malloc(sizeof(int) * nn);
    long *queue = (long *)malloc(sizeof(long) * nn);
    if (!lab || !col || !bid || !queue) return -1;
    long nint = 0;
    for (long p = 0; p < nn; ++p) {
        int c[3];
        ncoord(L, p, c);
        bid[p] = -1;
        if (is_interior(L, dim, c)) { label_of(kind, dim, L, c, &lab[p], &col[p]); ++nint; }
        else { lab[p] = -1; col[p] = -1; }
    }
    /* components */
    int cap = 1024, nb = 0;
    int *bstart = (int *)malloc(sizeof(int) * (cap + 1));
    int *comp = (int *)malloc(sizeof(int) * nint); /* points grouped by component, BFS order */
    long ncomp = 0;
    bstart[0] = 0;
    for (long p = 0; p < nn; ++p) {
        if (lab[p] < 0 || bid[p] >= 0) continue;
        long qh = 0, qt = 0;
        queue[qt++] = p;
        bid[p] = nb;
        while (qh < qt) {
            long q = queue[qh++];
            comp[ncomp++] = (int)q;
            int c[3];
            ncoord(L, q, c);
            for (int a = 0; a < dim; ++a)
                for (int d = -1; d <= 1; d += 2) {
                    int cc[3] = { c[0], c[1], c[2] };
                    cc[a] += d;
                    if (!is_interior(L, dim, cc)) continue;
                    long r = q + d * stride(L, a);
                    if (bid[r] < 0 && lab[r] == lab[q]) { bid[r] = nb; queue[qt++] = r; }
                }
        }
        ++nb;
        if (nb >= cap) { cap *= 2; bstart = (int *)realloc(bstart, sizeof(int) * (cap + 1)); }
        bstart[nb] = (int)ncomp;
    }
    /* order each block */
    int *bpts = (int *)malloc(sizeof(int) * nint);
    int *bshape = (int *)malloc(sizeof(int) * nb);
    int *bcolour = (int *)malloc(sizeof(int) * nb);
    int *bnleg = (int *)calloc(nb, sizeof(int));
    int *blegstart = (int *)calloc(nb + 1, sizeof(int));
    int legcap = 1024, nlegs = 0;
    int *blegs = (int *)malloc(sizeof(int) * legcap);
    int *deg = (int *)calloc(nn, sizeof(int)); /* scratch, indexed by node */
    char *seen = (char *)calloc(nn, 1);
    int err = 0;
    for (int b = 0; b < nb && !err; ++b) {
        int s = bstart[b], e = bstart[b + 1], sz = e - s;
        bcolour[b] = col[comp[s]];
        blegstart[b] = nlegs;
        long nedge2 = 0;
        int maxdeg = 0, nmax = 0, branch = -1;
        for (int t = s; t < e; ++t) {
            long q = comp[t];
            int c[3], dg = 0;
            ncoord(L, q, c);
            for (int a = 0; a < dim; ++a)
                for (int d = -1; d <= 1; d += 2) {
                    int cc[3] = { c[0], c[1], c[2] };
                    cc[a] += d;
                    if (!is_interior(L, dim, cc)) continue;
                    if (bid[q + d * stride(L, a)] == b) ++dg;
                }
            deg[q] = dg;
            nedge2 += dg;
            if (dg > maxdeg) { maxdeg = dg; nmax = 1; branch = (int)q; }
            else if (dg == maxdeg) ++nmax;
        }
        long nedge = nedge2 / 2;
        /* walk helper: next in-block neighbour of q that is not 'prev' */
#define NEXT_OF(q, prev, out)                                                        \
        do {                                                                         \
            int c_[3]; ncoord(L, (q), c_); (out) = -1;                               \
            for (int a_ = 0; a_ < dim && (out) < 0; ++a_)                            \
                for (int d_ = -1; d_ <= 1 && (out) < 0; d_ += 2) {                   \
                    int cc_[3] = { c_[0], c_[1], c_[2] }; cc_[a_] += d_;             \
                    if (!is_interior(L, dim, cc_)) continue;                         \
                    long r_ = (q) + d_ * stride(L, a_);                              \
                    if (bid[r_] == b && r_ != (prev) && !seen[r_]) (out) = r_;       \
                }                                                                    \
        } while (0)
        if (sz == 1) {
            bshape[b] = BLK_POINT;
            bpts[s] = comp[s];
        } else if (nedge == sz - 1 && maxdeg <= 2) {
            /* path: start at an end point (degree 1) */
            long start = -1;
            for (int t = s; t < e; ++t) if (deg[comp[t]] == 1) { start = comp[t]; break; }
            long prev = -1, q = start;
            int t = s;
            while (q >= 0) { bpts[t++] = (int)q; seen[q] = 1; long nx_; NEXT_OF(q, prev, nx_); prev = q; q = nx_; }
            if (t != e) err = 2;
            bshape[b] = BLK_PATH;
        } else if (nedge == sz - 1 && nmax == 1 && maxdeg >= 3) {
            /* spider: every other point must have degree <= 2 */
            for (int t = s; t < e; ++t) if (comp[t] != branch && deg[comp[t]] > 2) err = 3;
            seen[branch] = 1;
            int t = s;
            int c[3];
            ncoord(L, branch, c);
            for (int a = 0; a < dim; ++a)
                for (int d = -1; d <= 1; d += 2) {
                    int cc[3] = { c[0], c[1], c[2] };
                    cc[a] += d;
                    if (!is_interior(L, dim, cc)) continue;
                    long r = branch + d * stride(L, a);
                    if (bid[r] != b) continue;
                    /* walk outward from the branch, then store tip -> branch */
                    int t0 = t;
                    long prev = branch, q = r;
                    while (q >= 0) { bpts[t++] = (int)q; seen[q] = 1; long nx_; NEXT_OF(q, prev, nx_); prev = q; q = nx_; }
                    for (int u = t0, v = t - 1; u < v; ++u, --v) { int tmp = bpts[u]; bpts[u] = bpts[v]; bpts[v] = tmp; }
                    if (nlegs >= legcap) { legcap *= 2; blegs = (int *)realloc(blegs, sizeof(int) * legcap); }
                    blegs[nlegs++] = t - t0;
                    bnleg[b]++;
                }
            bpts[t++] = branch;
            if (t != e) err = 4;
            bshape[b] = BLK_SPIDER;
        } else if (nedge == sz && maxdeg == 2 && nmax == sz) {
            /* ring */
            long prev = -1, q = comp[s];
            int t = s;
            while (q >= 0) { bpts[t++] = (int)q; seen[q] = 1; long nx_; NEXT_OF(q, prev, nx_); prev = q; q = nx_; }
            if (t != e) err = 5;
            bshape[b] = BLK_RING;
        } else {
            err = 6;
        }
#undef NEXT_OF
        blegstart[b + 1] = nlegs;
    }
    free(deg); free(seen); free(lab); free(col); free(bid); free(queue); free(comp);
    if (err) {
        free(bpts); free(bshape); free(bcolour); free(bnleg); free(blegstart); free(blegs); free(bstart);
        return -err;
    }
    L->nblk[slot] = nb;
    L->bstart[slot] = bstart;
    L->bpts[slot] = bpts;
    L->bshape[slot] = bshape;
    L->bcolour[slot] = bcolour;
    L->bnleg[slot] = bnleg;
    L->blegstart[slot] = blegstart;
    L->blegs[slot] = blegs;
    L->kind[slot] = kind;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exact block solvers                                                       */
/* ------------------------------------------------------------------------ */

/* Tridiagonal (Thomas) solve of a_k x_{k-1} + b_k x_k + c_k x_{k+1} = r_k,
 * k = 0..m-1, a_0 = c_{m-1} = 0.  x may alias r. */
static void thomas(int m, const double *a, const double *b, const double *c, const double *r, double *x,
                   double *g, double *d)
{
    g[0] = c[0] / b[0];
    d[0] = r[0] / b[0];
    for (int k = 1; k < m; ++k) {
        double den = b[k] - a[k] * g[k - 1];
        g[k] = c[k] / den;
        d[k] = (r[k] - a[k] * d[k - 1]) / den;
    }
    x[m - 1] = d[m - 1];
    for (int k = m - 2; k >= 0; --k) x[k] = d[k] - g[k] * x[k + 1];
}

/* m-legged Thomas (eq. mLThomas).  Leg i holds points 1..p_i ordered from its
 * tip to the point next to the branch; row k of leg i reads
 *     a_k x_{k-1} + b_k x_k + c_k x_{k+1} = r_k,  x_{p_i+1} = x_centre,
 * and the branch row reads sum_i d_i x_{p_i}^{(i)} + d_{m+1} x_centre = r_centre.
 * Forward sweep from each tip toward the branch gives x_{p} = delta_p - gamma_p x_c;
 * the branch solve then gives x_c; back substitution runs out to the tips. */
static void mlthomas(int m, const int *p, double **a, double **b, double **c, double **r,
                     const double *d, double dm1, double rc, double **x, double **g, double **dl, double *xc)
{
    double num = rc, den = dm1;
    for (int i = 0; i < m; ++i) {
        int P = p[i];
        g[i][0] = c[i][0] / b[i][0];
        dl[i][0] = r[i][0] / b[i][0];
        for (int k = 1; k < P; ++k) {
            double q = b[i][k] - a[i][k] * g[i][k - 1];
            g[i][k] = c[i][k] / q;
            dl[i][k] = (r[i][k] - a[i][k] * dl[i][k - 1]) / q;
        }
        num -= d[i] * dl[i][P - 1];
        den -= d[i] * g[i][P - 1];
    }
    *xc = num / den;
    for (int i = 0; i < m; ++i) {
        int P = p[i];
        x[i][P - 1] = dl[i][P - 1] - g[i][P - 1] * (*xc);
        for (int k = P - 2; k >= 0; --k) x[i][k] = dl[i][k] - g[i][k] * x[i][k + 1];
    }
}

/* Circulant (periodic) tridiagonal solve of eq. (CircTri): row 1 couples to x_m
 * through a_1 and row m couples to x_1 through c_m.  Bordering on x_m: solve the
 * open tridiagonal rows 1..m-1 once for r and once for the column of x_m
 * (a_1 e_1 + c_{m-1} e_{m-1}), then close with row m.   READING: the periodic
 * Thomas algorithm is cited, not printed; this is its bordered form. */
static void circ_thomas(int m, const double *a, const double *b, const double *c, const double *r, double *x)
{
    int q = m - 1;
    double *aa = (double *)malloc(sizeof(double) * q), *cc = (double *)malloc(sizeof(double) * q);
    double *y = (double *)malloc(sizeof(double) * q), *z = (double *)malloc(sizeof(double) * q);
    double *col = (double *)malloc(sizeof(double) * q);
    double *g = (double *)malloc(sizeof(double) * q), *d = (double *)malloc(sizeof(double) * q);
    /* open system in rows 0..q-1 (0-based): drop a_1 (couples to x_m) and c_{m-1} */
    for (int k = 0; k < q; ++k) { aa[k] = (k == 0) ? 0.0 : a[k]; cc[k] = (k == q - 1) ? 0.0 : c[k]; }
    thomas(q, aa, b, cc, r, y, g, d);
    /* column of x_m inside rows 0..q-1 */
    for (int k = 0; k < q; ++k) col[k] = 0.0;
    col[0] += a[0];
    col[q - 1] += c[q - 1];
    thomas(q, aa, b, cc, col, z, g, d);
    /* row m (index q): c_m x_1 + a_m x_{m-1} + b_m x_m = r_m, with x_k = y_k - x_m z_k */
    double xm = (r[q] - c[q] * y[0] - a[q] * y[q - 1]) / (b[q] - c[q] * z[0] - a[q] * z[q - 1]);
    for (int k = 0; k < q; ++k) x[k] = y[k] - xm * z[k];
    x[q] = xm;
    free(aa); free(cc); free(y); free(z); free(col); free(g); free(d);
}

/* Dense Gaussian elimination with partial pivoting, used only by the debug
 * "dense" block solver that pins the structured solvers. A is n*n row-major. */
static int dense_solve(int n, double *A, double *bvec)
{
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i) if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
        if (A[piv * n + k] == 0.0) return -1;
        if (piv != k) {
            for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
            double t = bvec[k]; bvec[k] = bvec[piv]; bvec[piv] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            if (f == 0.0) continue;
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            bvec[i] -= f * bvec[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = bvec[k];
        for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * bvec[j];
        bvec[k] = s / A[k * n + k];
    }
    return 0;
}

/* Right-hand side of point q inside its block:  f_q - sum over neighbours
 * outside the block (other colour, or boundary nodes) of A[q, nb] u_nb. */
static double block_rhs(const orc_mg *M, const orc_level *L, const int *bid, int b, long q, const double *u,
                        const double *f)
{
    int c[3];
    ncoord(L, q, c);
    double r = f[q];
    for (int a = 0; a < M->dim; ++a)
        for (int d = -1; d <= 1; d += 2) {
            int cc[3] = { c[0], c[1], c[2] };
            cc[a] += d;
            long nb = q + d * stride(L, a);
            int inblock = is_interior(L, M->dim, cc) && bid[nb] == b;
            if (!inblock) r -= coef(M, L, a, c[a], d) * u[nb];
        }
    return r;
}
/* A[q, nb] for two distinct adjacent points q, nb */
static double pair_coef(const orc_mg *M, const orc_level *L, long q, long nb)
{
    int c[3], e[3];
    ncoord(L, q, c);
    ncoord(L, nb, e);
    for (int a = 0; a < M->dim; ++a)
        if (c[a] != e[a]) return coef(M, L, a, c[a], e[a] - c[a]);
    return 0.0;
}
static double pt_diag(const orc_mg *M, const orc_level *L, long q)
{
    int c[3];
    ncoord(L, q, c);
    return diagc(M, L, c);
}

/* block id per node, recomputed on demand for one motif slot */
static int *block_ids(const orc_level *L, int slot)
{
    int *bid = (int *)malloc(sizeof(int) * L->nn);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < L->nn; ++p) bid[p] = -1;
    for (int b = 0; b < L->nblk[slot]; ++b)
        for (int t = L->bstart[slot][b]; t < L->bstart[slot][b + 1]; ++t) bid[L->bpts[slot][t]] = b;
    return bid;
}

/* Solve block b of motif slot exactly, reading u outside the block, writing u
 * inside it.  dense != 0 uses Gaussian elimination on A[B,B] instead. */
static int solve_block(const orc_mg *M, const orc_level *L, int slot, const int *bid, int b, double *u,
                       const double *f, int dense, double *work)
{
    const int *pts = L->bpts[slot] + L->bstart[slot][b];
    int sz = L->bstart[slot][b + 1] - L->bstart[slot][b];
    int shape = L->bshape[slot][b];
    if (dense) {
        double *A = work, *rv = work + (long)sz * sz;
        for (int s = 0; s < sz; ++s) {
            for (int t = 0; t < sz; ++t) A[(long)s * sz + t] = 0.0;
            A[(long)s * sz + s] = pt_diag(M, L, pts[s]);
            rv[s] = block_rhs(M, L, bid, b, pts[s], u, f);
        }
        for (int s = 0; s < sz; ++s)
            for (int t = 0; t < sz; ++t) {
                if (s == t) continue;
                int c[3], e[3], dist = 0;
                ncoord(L, pts[s], c);
                ncoord(L, pts[t], e);
                for (int a = 0; a < M->dim; ++a) dist += abs(c[a] - e[a]);
                if (dist == 1) A[(long)s * sz + t] = pair_coef(M, L, pts[s], pts[t]);
            }
        if (dense_solve(sz, A, rv)) return -1;
        for (int s = 0; s < sz; ++s) u[pts[s]] = rv[s];
        return 0;
    }
    double *a = work, *bb = work + sz, *c = work + 2 * sz, *r = work + 3 * sz, *x = work + 4 * sz;
    double *g = work + 5 * sz, *d = work + 6 * sz;
    if (shape == BLK_POINT) {
        u[pts[0]] = block_rhs(M, L, bid, b, pts[0], u, f) / pt_diag(M, L, pts[0]);
        return 0;
    }
    for (int s = 0; s < sz; ++s) {
        bb[s] = pt_diag(M, L, pts[s]);
        r[s] = block_rhs(M, L, bid, b, pts[s], u, f);
    }
    if (shape == BLK_PATH) {
        for (int s = 0; s < sz; ++s) {
            a[s] = s > 0 ? pair_coef(M, L, pts[s], pts[s - 1]) : 0.0;
            c[s] = s < sz - 1 ? pair_coef(M, L, pts[s], pts[s + 1]) : 0.0;
        }
        thomas(sz, a, bb, c, r, x, g, d);
    } else if (shape == BLK_RING) {
        /* eq. CircTri ordering: a_k couples to the previous point (cyclically),
         * c_k to the next; a_1 -> x_m and c_m -> x_1 close the ring. */
        for (int s = 0; s < sz; ++s) {
            a[s] = pair_coef(M, L, pts[s], pts[(s - 1 + sz) % sz]);
            c[s] = pair_coef(M, L, pts[s], pts[(s + 1) % sz]);
        }
        circ_thomas(sz, a, bb, c, r, x);
    } else { /* spider */
        int m = L->bnleg[slot][b];
        const int *legs = L->blegs[slot] + L->blegstart[slot][b];
        double *pa[8], *pb[8], *pc[8], *pr[8], *px[8], *pg[8], *pd[8], dv[8];
        int p[8];
        long branch = pts[sz - 1];
        int off = 0;
        for (int i = 0; i < m; ++i) {
            p[i] = legs[i];
            pa[i] = a + off; pb[i] = bb + off; pc[i] = c + off; pr[i] = r + off;
            px[i] = x + off; pg[i] = g + off; pd[i] = d + off;
            for (int k = 0; k < p[i]; ++k) {
                long q = pts[off + k];
                long qn = (k < p[i] - 1) ? pts[off + k + 1] : branch;
                pa[i][k] = k > 0 ? pair_coef(M, L, q, pts[off + k - 1]) : 0.0;
                pc[i][k] = pair_coef(M, L, q, qn);
            }
            dv[i] = pair_coef(M, L, branch, pts[off + p[i] - 1]);
            off += p[i];
        }
        double xc;
        mlthomas(m, p, pa, pb, pc, pr, dv, bb[sz - 1], r[sz - 1], px, pg, pd, &xc);
        x[sz - 1] = xc;
    }
    for (int s = 0; s < sz; ++s) u[pts[s]] = x[s];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Operator, residual, transfers                                            */
/* ------------------------------------------------------------------------ */

/* out_p = (L u)_p at interior p (Section 2, problem DP); boundary entries 0. */
static void apply_op(const orc_mg *M, const orc_level *L, const double *u, double *out)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < L->nn; ++p) {
        int c[3];
        ncoord(L, p, c);
        if (!is_interior(L, M->dim, c)) { out[p] = 0.0; continue; }
        double s = diagc(M, L, c) * u[p];
        for (int a = 0; a < M->dim; ++a)
            for (int d = -1; d <= 1; d += 2) s += coef(M, L, a, c[a], d) * u[p + d * stride(L, a)];
        out[p] = s;
    }
}
/* defect d = f - L u at interior nodes, 0 at boundary nodes (Section 4 step 3). */
static void residual(const orc_mg *M, const orc_level *L, const double *u, const double *f, double *d)
{
    apply_op(M, L, u, d);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < L->nn; ++p) {
        int c[3];
        ncoord(L, p, c);
        d[p] = is_interior(L, M->dim, c) ? f[p] - d[p] : 0.0;
    }
}

/* Full weighting (Section 4): tensor product of (1/4, 1/2, 1/4) centred on fine
 * node 2I in index space; in 2D this is the printed 1/4, 1/8, 1/16 stencil.
 * Half weighting (2D only): 1/2 at the centre, 1/8 at each of the 4 neighbours.
 * Writes the coarse interior; coarse boundary entries are set to 0. */
static void restrict_op(int dim, const orc_level *F, const orc_level *Cl, const double *d, double *fc, int half)
{
    static const double w3[3] = { 0.25, 0.5, 0.25 };
#pragma omp parallel for schedule(static)
    for (long q = 0; q < Cl->nn; ++q) {
        int c[3];
        ncoord(Cl, q, c);
        if (!is_interior(Cl, dim, c)) { fc[q] = 0.0; continue; }
        double s = 0.0;
        if (half) {
            long p = nid(F, 2 * c[0], 2 * c[1], 0);
            s = 0.5 * d[p] + 0.125 * (d[p - 1] + d[p + 1] + d[p - F->np[0]] + d[p + F->np[0]]);
        } else {
            int lz = dim == 3 ? 1 : 0;
            for (int cz = -lz; cz <= lz; ++cz)
                for (int cy = -1; cy <= 1; ++cy)
                    for (int cx = -1; cx <= 1; ++cx) {
                        double w = w3[cx + 1] * w3[cy + 1] * (dim == 3 ? w3[cz + 1] : 1.0);
                        s += w * d[nid(F, 2 * c[0] + cx, 2 * c[1] + cy, dim == 3 ? 2 * c[2] + cz : 0)];
                    }
        }
        fc[q] = s;
    }
}

/* Bilinear (trilinear) interpolation in index space (Section 4): fine node i takes
 * coarse i/2 (even i) or the mean of (i-1)/2 and (i+1)/2 (odd i), tensor product
 * over the axes; coarse boundary values are taken as 0.  u_f += P e_c at fine
 * interior nodes (step 5). */
static void prolong_add(int dim, const orc_level *F, const orc_level *Cl, const double *ec, double *uf)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < F->nn; ++p) {
        int c[3];
        ncoord(F, p, c);
        if (!is_interior(F, dim, c)) continue;
        int lo[3], hi[3];
        double wl[3], wh[3];
        for (int a = 0; a < 3; ++a) {
            if (a >= dim) { lo[a] = hi[a] = 0; wl[a] = 1.0; wh[a] = 0.0; continue; }
            if (c[a] % 2 == 0) { lo[a] = hi[a] = c[a] / 2; wl[a] = 1.0; wh[a] = 0.0; }
            else { lo[a] = (c[a] - 1) / 2; hi[a] = (c[a] + 1) / 2; wl[a] = 0.5; wh[a] = 0.5; }
        }
        double v = 0.0;
        for (int sz = 0; sz < (dim == 3 ? 2 : 1); ++sz)
            for (int sy = 0; sy < 2; ++sy)
                for (int sx = 0; sx < 2; ++sx) {
                    double w = (sx ? wh[0] : wl[0]) * (sy ? wh[1] : wl[1]) * (dim == 3 ? (sz ? wh[2] : wl[2]) : 1.0);
                    if (w == 0.0) continue;
                    int I = sx ? hi[0] : lo[0], J = sy ? hi[1] : lo[1], K = sz ? hi[2] : lo[2];
                    int cc[3] = { I, J, K };
                    if (!is_interior(Cl, dim, cc)) continue; /* coarse boundary correction is 0 */
                    v += w * ec[nid(Cl, I, J, K)];
                }
        uf[p] += v;
    }
}

/* ------------------------------------------------------------------------ */
/* Coarsest-grid direct solve: banded LU without pivoting (the interior      */
/* matrix is diagonally dominant), natural ordering of interior unknowns.   */
/* ------------------------------------------------------------------------ */

static long unk_index(const orc_level *L, int dim, const int *c)
{
    long nx = L->n[0] - 1, ny = L->n[1] - 1;
    return (dim == 3 ? ((long)(c[2] - 1) * ny + (c[1] - 1)) * nx : (long)(c[1] - 1) * nx) + (c[0] - 1);
}

static int band_factor(const orc_mg *M, orc_level *L)
{
    int dim = M->dim;
    long nx = L->n[0] - 1, ny = L->n[1] - 1, nz = dim == 3 ? L->n[2] - 1 : 1;
    long n = nx * ny * nz;
    int bw = (int)(dim == 3 ? nx * ny : nx);
    int w = 2 * bw + 1;
    double *B = (double *)calloc((size_t)n * w, sizeof(double)); /* B[r*w + (col - r + bw)] */
    if (!B) return -1;
    for (long p = 0; p < L->nn; ++p) {
        int c[3];
        ncoord(L, p, c);
        if (!is_interior(L, dim, c)) continue;
        long r = unk_index(L, dim, c);
        B[r * w + bw] = diagc(M, L, c);
        for (int a = 0; a < dim; ++a)
            for (int d = -1; d <= 1; d += 2) {
                int cc[3] = { c[0], c[1], c[2] };
                cc[a] += d;
                if (!is_interior(L, dim, cc)) continue;
                long col = unk_index(L, dim, cc);
                B[r * w + (col - r + bw)] = coef(M, L, a, c[a], d);
            }
    }
    for (long k = 0; k < n; ++k) {
        double piv = B[k * w + bw];
        if (piv == 0.0) { free(B); return -2; }
        long iend = k + bw < n - 1 ? k + bw : n - 1;
        for (long i = k + 1; i <= iend; ++i) {
            double l = B[i * w + (k - i + bw)] / piv;
            B[i * w + (k - i + bw)] = l;
            if (l == 0.0) continue;
            long jend = k + bw < n - 1 ? k + bw : n - 1;
            for (long j = k + 1; j <= jend; ++j) B[i * w + (j - i + bw)] -= l * B[k * w + (j - k + bw)];
        }
    }
    L->band = B;
    L->bw = bw;
    L->nunk = n;
    return 0;
}

/* u_I = A_II^{-1} (f_I - A_IB u_B): boundary values of u are used as given. */
static void band_solve(const orc_mg *M, const orc_level *L, double *u, const double *f)
{
    if (!L->band && band_factor(M, (orc_level *)L)) { fprintf(stderr, "oracle: banded LU failed\n"); abort(); }
    int dim = M->dim;
    long n = L->nunk;
    int bw = L->bw, w = 2 * bw + 1;
    double *y = (double *)malloc(sizeof(double) * n);
    long *map = (long *)malloc(sizeof(long) * n);
    for (long p = 0; p < L->nn; ++p) {
        int c[3];
        ncoord(L, p, c);
        if (!is_interior(L, dim, c)) continue;
        long r = unk_index(L, dim, c);
        map[r] = p;
        double s = f[p];
        for (int a = 0; a < dim; ++a)
            for (int d = -1; d <= 1; d += 2) {
                int cc[3] = { c[0], c[1], c[2] };
                cc[a] += d;
                if (!is_interior(L, dim, cc)) s -= coef(M, L, a, c[a], d) * u[p + d * stride(L, a)];
            }
        y[r] = s;
    }
    const double *B = L->band;
    for (long i = 0; i < n; ++i) {
        long j0 = i - bw > 0 ? i - bw : 0;
        double s = y[i];
        for (long j = j0; j < i; ++j) s -= B[i * w + (j - i + bw)] * y[j];
        y[i] = s;
    }
    for (long i = n - 1; i >= 0; --i) {
        long j1 = i + bw < n - 1 ? i + bw : n - 1;
        double s = y[i];
        for (long j = i + 1; j <= j1; ++j) s -= B[i * w + (j - i + bw)] * y[j];
        y[i] = s / B[i * w + bw];
    }
    for (long r = 0; r < n; ++r) u[map[r]] = y[r];
    free(y);
    free(map);
}

/* ------------------------------------------------------------------------ */
/* Construction                                                              */
/* ------------------------------------------------------------------------ */

/* The motifs of one relaxation, in sweep order.  Alternating-direction zebra
 * is a zebra sweep along each axis in turn, x then y (then z in 3D: Section 7
 * compares 3D tweed with these three sweeps); alternating tweed/wireframe is
 * a tweed sweep then a wireframe sweep. */
static int motif_slots(int smoother, int dim, int *k)
{
    for (int s = 0; s < ORC_SLOTS; ++s) k[s] = -1;
    switch (smoother) {
    case ORC_TWEED: case ORC_WIREFRAME: case ORC_CHECKER: case ORC_ZEBRA_X: case ORC_ZEBRA_Y: case ORC_ZEBRA_Z:
        k[0] = smoother; return 0;
    case ORC_ADZ:
        k[0] = ORC_ZEBRA_X; k[1] = ORC_ZEBRA_Y;
        if (dim == 3) k[2] = ORC_ZEBRA_Z;
        return 0;
    case ORC_ALT_TW: k[0] = ORC_TWEED; k[1] = ORC_WIREFRAME; return 0;
    default: return -1;
    }
}

/* Create the hierarchy.  dim = 2 or 3; n[a] cells per axis; coords[a] = finest
 * node coordinates (n[a]+1 values each).  maxlev <= 0 means "as deep as the
 * coarsening rule allows"; otherwise at most maxlev levels (2 gives the
 * two-grid pair used for the spectral radii of Section 5). */
void *orc_create(int dim, const int *n, double *const *coords, double *const *sigma, int smoother, int transpose,
                 int maxlev)
{
    if (dim != 2 && dim != 3) return NULL;
    orc_mg *M = (orc_mg *)calloc(1, sizeof(orc_mg));
    M->dim = dim;
    M->smoother = smoother;
    M->transpose = transpose;
    int km[ORC_SLOTS];
    if (motif_slots(smoother, dim, km)) { free(M); return NULL; }
    int cur[3] = { n[0], n[1], dim == 3 ? n[2] : 0 };
    int lv = 0;
    for (;;) {
        orc_level *L = &M->lev[lv];
        for (int a = 0; a < 3; ++a) {
            L->n[a] = a < dim ? cur[a] : 0;
            L->np[a] = a < dim ? cur[a] + 1 : 1;
        }
        L->nn = (long)L->np[0] * L->np[1] * L->np[2];
        for (int a = 0; a < dim; ++a) {
            L->x[a] = (double *)malloc(sizeof(double) * (L->n[a] + 1));
            L->lo[a] = (double *)malloc(sizeof(double) * (L->n[a] + 1));
            L->hi[a] = (double *)malloc(sizeof(double) * (L->n[a] + 1));
            if (lv == 0) memcpy(L->x[a], coords[a], sizeof(double) * (L->n[a] + 1));
            else for (int i = 0; i <= L->n[a]; ++i) L->x[a][i] = M->lev[lv - 1].x[a][2 * i];
            L->sig[a] = NULL;
            if (sigma && sigma[a]) {
                L->sig[a] = (double *)malloc(sizeof(double) * L->n[a]);
                if (lv == 0) memcpy(L->sig[a], sigma[a], sizeof(double) * L->n[a]);
                else coarse_sigma(L->n[a], M->lev[lv - 1].x[a], M->lev[lv - 1].sig[a], L->sig[a]);
            }
            orc_coefs_sigma(L->n[a], L->x[a], L->sig[a], L->lo[a], L->hi[a]);
        }
        for (int s = 0; s < ORC_SLOTS; ++s) L->kind[s] = -1;
        ++lv;
        int can = 1;
        for (int a = 0; a < dim; ++a) if (cur[a] % 2 != 0 || cur[a] < 4) can = 0;
        if (!can || lv >= ORC_MAXLEV || (maxlev > 0 && lv >= maxlev)) break;
        for (int a = 0; a < dim; ++a) cur[a] /= 2;
    }
    M->nlev = lv;
    for (int l = 0; l < M->nlev; ++l) {
        orc_level *L = &M->lev[l];
        int bad = 0;
        for (int a = 0; a < dim; ++a) if (L->n[a] < 2) bad = 1;
        if (bad) { free(M); return NULL; }
        /* the motifs are defined for an even number of cells per axis (Section 3);
         * a coarsest level with an odd count is only ever solved directly */
        int odd = 0;
        for (int a = 0; a < dim; ++a) if (L->n[a] % 2) odd = 1;
        if (odd && l == M->nlev - 1 && l > 0) continue;
        for (int s = 0; s < ORC_SLOTS; ++s)
            if (km[s] >= 0 && build_blocks(M, L, s, km[s])) { free(M); return NULL; }
    }
    /* the coarsest level's banded LU is built on first use (band_solve) */
    return M;
}

void orc_destroy(void *h)
{
    orc_mg *M = (orc_mg *)h;
    if (!M) return;
    for (int l = 0; l < M->nlev; ++l) {
        orc_level *L = &M->lev[l];
        for (int a = 0; a < 3; ++a) { free(L->x[a]); free(L->lo[a]); free(L->hi[a]); free(L->sig[a]); }
        for (int s = 0; s < ORC_SLOTS; ++s) {
            free(L->bstart[s]); free(L->bpts[s]); free(L->bshape[s]); free(L->bcolour[s]);
            free(L->bnleg[s]); free(L->blegstart[s]); free(L->blegs[s]);
        }
        free(L->band);
    }
    free(M);
}

int orc_nlevels(void *h) { return ((orc_mg *)h)->nlev; }
void orc_level_shape(void *h, int lv, int *n) { for (int a = 0; a < 3; ++a) n[a] = ((orc_mg *)h)->lev[lv].n[a]; }
void orc_level_coefs(void *h, int lv, int axis, double *x, double *lo, double *hi)
{
    orc_level *L = &((orc_mg *)h)->lev[lv];
    int n = L->n[axis];
    memcpy(x, L->x[axis], sizeof(double) * (n + 1));
    memcpy(lo, L->lo[axis], sizeof(double) * (n + 1));
    memcpy(hi, L->hi[axis], sizeof(double) * (n + 1));
}

/* ------------------------------------------------------------------------ */
/* Smoothing                                                                 */
/* ------------------------------------------------------------------------ */

static size_t max_block(const orc_level *L, int slot)
{
    size_t m = 1;
    for (int b = 0; b < L->nblk[slot]; ++b) {
        size_t s = (size_t)(L->bstart[slot][b + 1] - L->bstart[slot][b]);
        if (s > m) m = s;
    }
    return m;
}

/* One sweep of block Gauss-Seidel with the motif in 'slot' (Section 3): every
 * red block is solved exactly with black values frozen, then every black block.
 * The adjoint (transposed) smoother runs the colours in reverse order so that the
 * adjoint cycle is the transpose of the forward cycle.  'order' != 0 visits the
 * blocks of a colour in reverse order (they are independent; used by a test). */
static int sweep(const orc_mg *M, const orc_level *L, int slot, double *u, const double *f, int dense, int order)
{
    int *bid = block_ids(L, slot);
    size_t mb = max_block(L, slot);
    const size_t wsz = dense ? mb * mb + mb : 12 * mb + 8;
    const int nb = L->nblk[slot];
    int rc = 0;
    for (int pass = 0; pass < 2 && !rc; ++pass) {
        int colour = M->transpose ? 1 - pass : pass;
        /* the blocks of one colour are uncoupled: any order (and any split
         * over threads) gives the same values */
#pragma omp parallel reduction(| : rc)
        {
            double *work = (double *)malloc(sizeof(double) * wsz);
#pragma omp for schedule(dynamic, 8)
            for (int t = 0; t < nb; ++t) {
                int b = order ? nb - 1 - t : t;
                if (L->bcolour[slot][b] != colour || rc) continue;
                if (solve_block(M, L, slot, bid, b, u, f, dense, work)) rc = 1;
            }
            free(work);
        }
    }
    free(bid);
    return rc ? -1 : 0;
}

/* One relaxation of the chosen smoother: for the alternating schemes (ADZ and
 * alternating tweed/wireframe) one relaxation is the pair (in 3D ADZ, the
 * triple) of sweeps, which is how the paper counts nu for them.  The adjoint
 * runs the sweeps in reverse order. */
static int relax(const orc_mg *M, const orc_level *L, double *u, const double *f, int dense, int order)
{
    int ns = 0;
    while (ns < ORC_SLOTS && L->kind[ns] >= 0) ++ns;
    for (int k = 0; k < ns; ++k) {
        int s = M->transpose ? ns - 1 - k : k;
        int rc = sweep(M, L, s, u, f, dense, order);
        if (rc) return rc;
    }
    return 0;
}

int orc_smooth(void *h, int lv, double *u, const double *f, int nu, int dense, int order)
{
    orc_mg *M = (orc_mg *)h;
    for (int s = 0; s < nu; ++s) {
        int rc = relax(M, &M->lev[lv], u, f, dense, order);
        if (rc) return rc;
    }
    return 0;
}

void orc_apply(void *h, int lv, const double *u, double *out)
{
    orc_mg *M = (orc_mg *)h;
    apply_op(M, &M->lev[lv], u, out);
}
void orc_residual(void *h, int lv, const double *u, const double *f, double *d)
{
    orc_mg *M = (orc_mg *)h;
    residual(M, &M->lev[lv], u, f, d);
}
void orc_restrict(void *h, int lv, const double *d, double *fc, int half)
{
    orc_mg *M = (orc_mg *)h;
    restrict_op(M->dim, &M->lev[lv], &M->lev[lv + 1], d, fc, half);
}
void orc_prolong_add(void *h, int lv, const double *ec, double *uf)
{
    orc_mg *M = (orc_mg *)h;
    prolong_add(M->dim, &M->lev[lv], &M->lev[lv + 1], ec, uf);
}
/* direct solve on the coarsest level (boundary values of u are used) */
void orc_coarse_solve(void *h, double *u, const double *f)
{
    orc_mg *M = (orc_mg *)h;
    band_solve(M, &M->lev[M->nlev - 1], u, f);
}

/* ------------------------------------------------------------------------ */
/* Cycles (Section 4, steps (1)-(6))                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *u[ORC_MAXLEV], *f[ORC_MAXLEV], *d[ORC_MAXLEV];
} orc_ws;

static int cycle(const orc_mg *M, orc_ws *W, int lv, int nu1, int nu2, int gamma, int half)
{
    const orc_level *L = &M->lev[lv];
    if (lv == M->nlev - 1) { band_solve(M, L, W->u[lv], W->f[lv]); return 0; }
    int rc;
    for (int s = 0; s < nu1; ++s) if ((rc = relax(M, L, W->u[lv], W->f[lv], 0, 0))) return rc;   /* step 2 */
    residual(M, L, W->u[lv], W->f[lv], W->d[lv]);                                                /* step 3 */
    restrict_op(M->dim, L, &M->lev[lv + 1], W->d[lv], W->f[lv + 1], half);
    memset(W->u[lv + 1], 0, sizeof(double) * M->lev[lv + 1].nn);                                 /* step 4 */
    for (int g = 0; g < gamma; ++g)
        if ((rc = cycle(M, W, lv + 1, nu1, nu2, gamma, half))) return rc;
    prolong_add(M->dim, L, &M->lev[lv + 1], W->u[lv + 1], W->u[lv]);                             /* step 5 */
    for (int s = 0; s < nu2; ++s) if ((rc = relax(M, L, W->u[lv], W->f[lv], 0, 0))) return rc;   /* step 6 */
    return 0;
}

static orc_ws *ws_alloc(const orc_mg *M)
{
    orc_ws *W = (orc_ws *)calloc(1, sizeof(orc_ws));
    for (int l = 0; l < M->nlev; ++l) {
        long nn = M->lev[l].nn;
        if (l > 0) { W->u[l] = (double *)calloc(nn, sizeof(double)); W->f[l] = (double *)calloc(nn, sizeof(double)); }
        W->d[l] = (double *)calloc(nn, sizeof(double));
    }
    return W;
}
static void ws_free(const orc_mg *M, orc_ws *W)
{
    for (int l = 0; l < M->nlev; ++l) { if (l > 0) { free(W->u[l]); free(W->f[l]); } free(W->d[l]); }
    free(W);
}

/* One gamma-cycle (gamma = 1: V, 2: W) on the finest level, in place on u
 * (its boundary entries are the Dirichlet data and are never written). */
int orc_cycle(void *h, double *u, const double *f, int nu1, int nu2, int gamma, int half)
{
    orc_mg *M = (orc_mg *)h;
    orc_ws *W = ws_alloc(M);
    W->u[0] = u;
    W->f[0] = (double *)f;
    int rc = cycle(M, W, 0, nu1, nu2, gamma, half);
    ws_free(M, W);
    return rc;
}

static double maxabs_interior(const orc_mg *M, const orc_level *L, const double *d)
{
    double m = 0.0;
    int nan = 0;
#pragma omp parallel for schedule(static) reduction(max : m) reduction(| : nan)
    for (long p = 0; p < L->nn; ++p) {
        int c[3];
        ncoord(L, p, c);
        if (!is_interior(L, M->dim, c)) continue;
        double a = fabs(d[p]);
        if (a != a) nan = 1;
        else if (a > m) m = a;
    }
    return nan ? NAN : m; /* NaN propagates */
}

/* Relative infinity-norm of the defect, ||f - L u||_inf over interior nodes. */
double orc_resnorm(void *h, const double *u, const double *f)
{
    orc_mg *M = (orc_mg *)h;
    const orc_level *L = &M->lev[0];
    double *d = (double *)malloc(sizeof(double) * L->nn);
    residual(M, L, u, f, d);
    double m = maxabs_interior(M, L, d);
    free(d);
    return m;
}

/* Section 4: repeat cycles until ||f - L u||_inf / ||d_0||_inf < tol, where d_0
 * is the defect of the initial u (its interior is used as given; callers pass
 * zeros for the paper's u = 0 start, step 1).  history[k] = relative defect after
 * cycle k+1.  Returns the number of cycles; *status: 0 converged, 1 not
 * converged within max_cycles, 2 diverged (NaN/Inf or defect > 1e6 d_0). */
int orc_solve(void *h, double *u, const double *f, int nu1, int nu2, int gamma, double tol, int max_cycles,
              double *history, int *status)
{
    orc_mg *M = (orc_mg *)h;
    const orc_level *L = &M->lev[0];
    orc_ws *W = ws_alloc(M);
    W->u[0] = u;
    W->f[0] = (double *)f;
    residual(M, L, u, f, W->d[0]);
    double d0 = maxabs_interior(M, L, W->d[0]);
    int k = 0;
    *status = 1;
    if (d0 == 0.0) { *status = 0; ws_free(M, W); return 0; }
    while (k < max_cycles) {
        if (cycle(M, W, 0, nu1, nu2, gamma, 0)) { *status = 3; break; }
        residual(M, L, u, f, W->d[0]);
        double rel = maxabs_interior(M, L, W->d[0]) / d0;
        if (history) history[k] = rel;
        ++k;
        if (!(rel == rel) || rel > 1e6) { *status = 2; break; }
        if (rel < tol) { *status = 0; break; }
    }
    ws_free(M, W);
    return k;
}

/* Direct solve of the finest level by banded LU (the limit the cycles must reach). */
int orc_direct(void *h, double *u, const double *f)
{
    orc_mg *M = (orc_mg *)h;
    orc_level tmp = M->lev[0];
    tmp.band = NULL;
    if (band_factor(M, &tmp)) return -1;
    band_solve(M, &tmp, u, f);
    free(tmp.band);
    return 0;
}

/* Two-grid error propagation of Section 5 (eq. Mh2h) with nu1 = nu, nu2 = 0:
 * e <- S^nu e (homogeneous problem), then e <- e + P L_c^{-1} R (-L e).
 * Requires a hierarchy built with maxlev = 2; e has zero boundary entries. */
int orc_twogrid(void *h, double *e, int nu, int half)
{
    orc_mg *M = (orc_mg *)h;
    if (M->nlev != 2) return -1;
    const orc_level *F = &M->lev[0], *Cl = &M->lev[1];
    double *zero = (double *)calloc(F->nn, sizeof(double));
    double *d = (double *)malloc(sizeof(double) * F->nn);
    double *fc = (double *)calloc(Cl->nn, sizeof(double));
    double *ec = (double *)calloc(Cl->nn, sizeof(double));
    int rc = 0;
    for (int s = 0; s < nu && !rc; ++s) rc = relax(M, F, e, zero, 0, 0);
    residual(M, F, e, zero, d);
    restrict_op(M->dim, F, Cl, d, fc, half);
    band_solve(M, Cl, ec, fc);
    prolong_add(M->dim, F, Cl, ec, e);
    free(zero); free(d); free(fc); free(ec);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Introspection used by the tests                                           */
/* ------------------------------------------------------------------------ */

int orc_nblocks(void *h, int lv, int slot) { return ((orc_mg *)h)->lev[lv].nblk[slot]; }
/* info = {size, shape, colour, nlegs}; legs receives the leg lengths. */
void orc_block_info(void *h, int lv, int slot, int b, int *info, int *legs)
{
    orc_level *L = &((orc_mg *)h)->lev[lv];
    info[0] = L->bstart[slot][b + 1] - L->bstart[slot][b];
    info[1] = L->bshape[slot][b];
    info[2] = L->bcolour[slot][b];
    info[3] = L->bnleg[slot][b];
    for (int i = 0; i < info[3]; ++i) legs[i] = L->blegs[slot][L->blegstart[slot][b] + i];
}
void orc_block_points(void *h, int lv, int slot, int b, int *pts)
{
    orc_level *L = &((orc_mg *)h)->lev[lv];
    int s = L->bstart[slot][b], e = L->bstart[slot][b + 1];
    for (int t = s; t < e; ++t) pts[t - s] = L->bpts[slot][t];
}
/* Dense block system A[B,B] x = f_B - A[B,Bbar] u_Bbar for block b (points in
 * the stored order); A is size*size row-major. */
void orc_block_system(void *h, int lv, int slot, int b, const double *u, const double *f, double *A, double *rhs)
{
    orc_mg *M = (orc_mg *)h;
    orc_level *L = &M->lev[lv];
    int *bid = block_ids(L, slot);
    const int *pts = L->bpts[slot] + L->bstart[slot][b];
    int sz = L->bstart[slot][b + 1] - L->bstart[slot][b];
    for (int s = 0; s < sz; ++s) {
        for (int t = 0; t < sz; ++t) A[(long)s * sz + t] = 0.0;
        A[(long)s * sz + s] = pt_diag(M, L, pts[s]);
        rhs[s] = block_rhs(M, L, bid, b, pts[s], u, f);
        for (int t = 0; t < sz; ++t) {
            if (s == t) continue;
            int c[3], e[3], dist = 0;
            ncoord(L, pts[s], c);
            ncoord(L, pts[t], e);
            for (int a = 0; a < M->dim; ++a) dist += abs(c[a] - e[a]);
            if (dist == 1) A[(long)s * sz + t] = pair_coef(M, L, pts[s], pts[t]);
        }
    }
    free(bid);
}
/* Solve one block in place (dense != 0: Gaussian elimination on A[B,B]). */
int orc_solve_block(void *h, int lv, int slot, int b, double *u, const double *f, int dense)
{
    orc_mg *M = (orc_mg *)h;
    orc_level *L = &M->lev[lv];
    int *bid = block_ids(L, slot);
    size_t mb = max_block(L, slot);
    double *work = (double *)malloc(sizeof(double) * (dense ? mb * mb + mb : 12 * mb + 8));
    int rc = solve_block(M, L, slot, bid, b, u, f, dense, work);
    free(work);
    free(bid);
    return rc;
}
