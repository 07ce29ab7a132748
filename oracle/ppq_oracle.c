/*
 * ppq_oracle.c -- plain FP64 CPU reference of dynamically pruned wavepacket
 * propagation (Larsson, Hartke & Tannor, J. Chem. Phys. 2016, arXiv:1606.04004).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the HIP implementation and is deliberately slow and literal.
 *
 * Built with -O2 -ffp-contract=off: no fused multiply-add anywhere, so the
 * threshold predicate |c|^2 >= eps^2 is evaluated as fl(fl(re*re)+fl(im*im)).
 *
 * What each routine follows:
 *   orc_apply_def   -- the plain definition of the pruned operator P H P on an
 *                      active set (Sec. II.B.2, Eq. matvecprod_sequential and
 *                      the pruned sums that follow it; DVR potential diagonal,
 *                      Sec. II.A).  Product terms with two non-diagonal factors
 *                      are applied sequentially with truncation to the active
 *                      set between factors, innermost (higher) dimension first.
 *   orc_fib_*       -- the appendix algorithm: permute so the transformed
 *                      dimension is last, contract each fiber with the 1D
 *                      matrix over the index ranges J(i), permute back; the
 *                      permutations are kept until the basis changes.
 *   orc_sil_step    -- short-iterative Lanczos (Hermitian) / Arnoldi
 *                      (non-Hermitian) propagator (Sec. III.A), Krylov order m,
 *                      classical Gram-Schmidt applied twice.
 *   orc_prune       -- basis adaption (Sec. II.E): keep |a| >= theta, add the
 *                      2D nearest neighbours (phase-space ball radius 1,
 *                      Sec. III.A; radius sqrt(2) and 2 on request), hash set
 *                      of used functions, then sort.
 *   orc_observe     -- norm, energy, autocorrelation C(t) (Eq. acorr),
 *                      number of used / above-threshold functions.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXD 8
typedef double complex zd;

/* ------------------------------------------------------------------------ */
/* model                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct orc_model {
    int D;
    int n[ORC_MAXD];
    int nmax;
    uint64_t stride[ORC_MAXD];
    uint64_t total;
    zd *h[ORC_MAXD];            /* single-dimension operator per dim (n_k x n_k), or NULL */
    int nv;                     /* diagonal potential terms */
    double *vcoef;
    int *vuse;                  /* [nv][D] */
    double *vtab;               /* [nv][D][nmax] */
    int np;                     /* product terms with dense factors */
    zd *pcoef;
    int *pnf;                   /* [np] number of factors */
    int *pk;                    /* [np][ORC_MAXD] their dimensions, increasing */
    zd **ph;                    /* [np][ORC_MAXD] their n_k x n_k matrices; applied
                                   coef * P h_0 P h_1 ... P h_{nf-1} P x, the last
                                   (highest) dimension first */
    int lat_s[ORC_MAXD], lat_l[ORC_MAXD]; /* phase-space lattice shape per dim; 0 = line */
    int stencil;                /* adaption neighbours: 1 = ball radius 1, 2 = radius sqrt(2), 3 = radius 2 */
    double krylov_tol;          /* > 0: SIL order chosen per step by the error estimate */
    int max_substeps;           /* > 1 (with krylov_tol > 0): step size control, see controlled_step */
} orc_model;

orc_model *orc_new(int D, const int32_t *n)
{
    if (D < 1 || D > ORC_MAXD) return NULL;
    orc_model *m = calloc(1, sizeof(*m));
    m->D = D;
    m->stencil = 1;
    m->nmax = 0;
    for (int k = 0; k < D; ++k) {
        m->n[k] = n[k];
        if (n[k] > m->nmax) m->nmax = n[k];
    }
    m->total = 1;
    for (int k = D - 1; k >= 0; --k) {
        m->stride[k] = m->total;
        m->total *= (uint64_t)n[k];
    }
    return m;
}

void orc_free(orc_model *m)
{
    if (!m) return;
    for (int k = 0; k < m->D; ++k) free(m->h[k]);
    free(m->vcoef); free(m->vuse); free(m->vtab);
    for (int t = 0; t < m->np; ++t)
        for (int f = 0; f < m->pnf[t]; ++f) free(m->ph[t * ORC_MAXD + f]);
    free(m->pcoef); free(m->pnf); free(m->pk); free(m->ph);
    free(m);
}

static zd *copy_cmat(const double *src, int nk)
{
    zd *h = malloc(sizeof(zd) * (size_t)nk * nk);
    for (int i = 0; i < nk * nk; ++i) h[i] = src[2 * i] + I * src[2 * i + 1];
    return h;
}

/* Adds a dense complex operator (interleaved re,im; row-major) on dim k. */
int orc_add_h(orc_model *m, int k, const double *h)
{
    if (k < 0 || k >= m->D) return -1;
    int nk = m->n[k];
    if (!m->h[k]) {
        m->h[k] = calloc((size_t)nk * nk, sizeof(zd));
    }
    for (int i = 0; i < nk * nk; ++i) m->h[k][i] += h[2 * i] + I * h[2 * i + 1];
    return 0;
}

/* Diagonal potential term coef * prod_{k: use[k]} tab[k][i_k]; tab is [D][nmax]. */
int orc_add_vterm(orc_model *m, double coef, const int32_t *use, const double *tab)
{
    int t = m->nv++;
    int D = m->D, nm = m->nmax;
    m->vcoef = realloc(m->vcoef, sizeof(double) * m->nv);
    m->vuse = realloc(m->vuse, sizeof(int) * m->nv * D);
    m->vtab = realloc(m->vtab, sizeof(double) * (size_t)m->nv * D * nm);
    m->vcoef[t] = coef;
    for (int k = 0; k < D; ++k) {
        m->vuse[t * D + k] = use[k] ? 1 : 0;
        for (int i = 0; i < nm; ++i)
            m->vtab[((size_t)t * D + k) * nm + i] = (use[k] && i < m->n[k]) ? tab[k * nm + i] : 0.0;
    }
    return 0;
}

/* Product term (cre + i cim) * h_0(dims[0]) (x) ... (x) h_{nf-1}(dims[nf-1]) of a
   sum-of-products operator (Sec. II.B.2), dims strictly increasing, each h_f
   a dense complex n_k x n_k matrix (interleaved re,im; row-major), the
   matrices concatenated in factor order.  On an active set it is applied as
   the sequential product of Eq. matvecprod_sequential with every
   intermediate truncated to the set: the factor of the highest dimension
   first (the innermost sum runs over the last index), then the next lower. */
int orc_add_prod(orc_model *m, double cre, double cim, int nf, const int32_t *dims, const double *mats)
{
    if (nf < 1 || nf > m->D) return -1;
    for (int f = 0; f < nf; ++f) {
        if (dims[f] < 0 || dims[f] >= m->D) return -1;
        if (f > 0 && dims[f] <= dims[f - 1]) return -1;
    }
    int t = m->np++;
    m->pcoef = realloc(m->pcoef, sizeof(zd) * m->np);
    m->pnf = realloc(m->pnf, sizeof(int) * m->np);
    m->pk = realloc(m->pk, sizeof(int) * ORC_MAXD * m->np);
    m->ph = realloc(m->ph, sizeof(zd *) * ORC_MAXD * m->np);
    m->pcoef[t] = cre + I * cim;
    m->pnf[t] = nf;
    size_t off = 0;
    for (int f = 0; f < nf; ++f) {
        int nk = m->n[dims[f]];
        m->pk[t * ORC_MAXD + f] = dims[f];
        m->ph[t * ORC_MAXD + f] = copy_cmat(mats + off, nk);
        off += 2 * (size_t)nk * nk;
    }
    return 0;
}

/* Two-factor product term coef * h1(k1) (x) h2(k2), k1 < k2. */
int orc_add_pair(orc_model *m, double cre, double cim, int k1, int k2, const double *h1, const double *h2)
{
    if (k1 < 0 || k2 < 0 || k1 >= m->D || k2 >= m->D || k1 >= k2) return -1;
    size_t n1 = 2 * (size_t)m->n[k1] * m->n[k1], n2 = 2 * (size_t)m->n[k2] * m->n[k2];
    double *mats = malloc(sizeof(double) * (n1 + n2));
    memcpy(mats, h1, sizeof(double) * n1);
    memcpy(mats + n1, h2, sizeof(double) * n2);
    int32_t dims[2] = {k1, k2};
    int r = orc_add_prod(m, cre, cim, 2, dims, mats);
    free(mats);
    return r;
}

int orc_set_lattice(orc_model *m, int k, int ns, int nl)
{
    if (k < 0 || k >= m->D || ns * nl != m->n[k]) return -1;
    m->lat_s[k] = ns;
    m->lat_l[k] = nl;
    return 0;
}

static inline int digit(const orc_model *m, uint64_t key, int k)
{
    return (int)((key / m->stride[k]) % (uint64_t)m->n[k]);
}

static double potential_at(const orc_model *m, uint64_t key)
{
    int d[ORC_MAXD];
    for (int k = 0; k < m->D; ++k) d[k] = digit(m, key, k);
    double v = 0.0;
    for (int t = 0; t < m->nv; ++t) {
        double f = m->vcoef[t];
        for (int k = 0; k < m->D; ++k)
            if (m->vuse[t * m->D + k]) f *= m->vtab[((size_t)t * m->D + k) * m->nmax + d[k]];
        v += f;
    }
    return v;
}

/* ------------------------------------------------------------------------ */
/* O-def: plain definition with a lookup in the sorted key list             */
/* ------------------------------------------------------------------------ */
static int64_t find_key(const uint64_t *keys, int64_t n, uint64_t key)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] == key) return mid;
        if (keys[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* out[p] = sum_j h[d_k(p)][j] x[I(p) with digit k -> j], restricted to the set */
static void def_dim(const orc_model *m, int k, const zd *h, int64_t n, const uint64_t *keys,
                    const zd *x, zd *out)
{
    int nk = m->n[k];
    for (int64_t p = 0; p < n; ++p) {
        uint64_t key = keys[p];
        int dk = digit(m, key, k);
        uint64_t base = key - (uint64_t)dk * m->stride[k];
        zd acc = 0.0;
        for (int j = 0; j < nk; ++j) {
            int64_t q = find_key(keys, n, base + (uint64_t)j * m->stride[k]);
            if (q >= 0) acc += h[(size_t)dk * nk + j] * x[q];
        }
        out[p] = acc;
    }
}

int orc_apply_def(const orc_model *m, int64_t n, const uint64_t *keys, const double *xin, double *yout)
{
    const zd *x = (const zd *)xin;
    zd *y = (zd *)yout;
    zd *tmp = malloc(sizeof(zd) * (size_t)(n > 0 ? n : 1));
    zd *z = malloc(sizeof(zd) * (size_t)(n > 0 ? n : 1));
    for (int64_t p = 0; p < n; ++p) y[p] = potential_at(m, keys[p]) * x[p];
    for (int k = 0; k < m->D; ++k) {
        if (!m->h[k]) continue;
        def_dim(m, k, m->h[k], n, keys, x, tmp);
        for (int64_t p = 0; p < n; ++p) y[p] += tmp[p];
    }
    for (int t = 0; t < m->np; ++t) {
        /* P h_{nf-1} P x first, then each lower factor on the truncated result */
        for (int64_t p = 0; p < n; ++p) z[p] = x[p];
        for (int f = m->pnf[t] - 1; f >= 0; --f) {
            def_dim(m, m->pk[t * ORC_MAXD + f], m->ph[t * ORC_MAXD + f], n, keys, z, tmp);
            for (int64_t p = 0; p < n; ++p) z[p] = tmp[p];
        }
        for (int64_t p = 0; p < n; ++p) y[p] += m->pcoef[t] * z[p];
    }
    free(tmp);
    free(z);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O-fib: the appendix algorithm                                            */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t rk; int64_t p; } rk_pair;

static int cmp_rk(const void *a, const void *b)
{
    const rk_pair *x = a, *y = b;
    return (x->rk > y->rk) - (x->rk < y->rk);
}

typedef struct orc_fib {
    int64_t n;
    int D;
    /* per dim: perm[q] = position of the q-th entry in "dim k last" order,
       dig[q] = its digit i_k; fibers = maximal runs with equal remaining
       digits, given by fstart[f]..fstart[f+1]; within each fiber the index
       set J(i) is stored as ranges [rlo, rhi] of digits with the member
       offset of the first digit in each range. */
    int64_t *perm[ORC_MAXD];
    int *dig[ORC_MAXD];
    int64_t nfib[ORC_MAXD];
    int64_t *fstart[ORC_MAXD];
    int64_t *rstart[ORC_MAXD];  /* per fiber: first range index */
    int *rlo[ORC_MAXD], *rhi[ORC_MAXD];
    int64_t *roff[ORC_MAXD];    /* member offset (within the fiber) of digit rlo */
    double *vdiag;              /* potential cached on the set */
} orc_fib;

static void fib_free_parts(orc_fib *f)
{
    for (int k = 0; k < f->D; ++k) {
        free(f->perm[k]); free(f->dig[k]); free(f->fstart[k]); free(f->rstart[k]);
        free(f->rlo[k]); free(f->rhi[k]); free(f->roff[k]);
    }
    free(f->vdiag);
}

void orc_fib_free(orc_fib *f)
{
    if (!f) return;
    fib_free_parts(f);
    free(f);
}

orc_fib *orc_fib_build(const orc_model *m, int64_t n, const uint64_t *keys)
{
    orc_fib *f = calloc(1, sizeof(*f));
    f->n = n;
    f->D = m->D;
    size_t nn = (size_t)(n > 0 ? n : 1);
    rk_pair *tmp = malloc(sizeof(rk_pair) * nn);
    for (int k = 0; k < m->D; ++k) {
        uint64_t nk = (uint64_t)m->n[k], sk = m->stride[k];
        /* rotated key: digit k moved to the last (fastest) position */
        for (int64_t p = 0; p < n; ++p) {
            uint64_t key = keys[p];
            uint64_t hi = key / (sk * nk), d = (key / sk) % nk, lo = key % sk;
            tmp[p].rk = (hi * sk + lo) * nk + d;
            tmp[p].p = p;
        }
        qsort(tmp, (size_t)n, sizeof(rk_pair), cmp_rk);
        f->perm[k] = malloc(sizeof(int64_t) * nn);
        f->dig[k] = malloc(sizeof(int) * nn);
        f->fstart[k] = malloc(sizeof(int64_t) * (nn + 1));
        f->rstart[k] = malloc(sizeof(int64_t) * (nn + 1));
        f->rlo[k] = malloc(sizeof(int) * nn);
        f->rhi[k] = malloc(sizeof(int) * nn);
        f->roff[k] = malloc(sizeof(int64_t) * nn);
        int64_t nf = 0, nr = 0;
        for (int64_t q = 0; q < n; ++q) {
            f->perm[k][q] = tmp[q].p;
            int d = (int)(tmp[q].rk % nk);
            f->dig[k][q] = d;
            int newfib = (q == 0) || (tmp[q].rk / nk != tmp[q - 1].rk / nk);
            if (newfib) {
                f->fstart[k][nf] = q;
                f->rstart[k][nf] = nr;
                ++nf;
            }
            if (newfib || d != f->dig[k][q - 1] + 1) {
                f->rlo[k][nr] = d;
                f->rhi[k][nr] = d;
                f->roff[k][nr] = q - f->fstart[k][nf - 1];
                ++nr;
            } else {
                f->rhi[k][nr - 1] = d;
            }
        }
        f->fstart[k][nf] = n;
        f->rstart[k][nf] = nr;
        f->nfib[k] = nf;
    }
    free(tmp);
    f->vdiag = malloc(sizeof(double) * nn);
    for (int64_t p = 0; p < n; ++p) f->vdiag[p] = potential_at(m, keys[p]);
    return f;
}

/* out (+)= P h P x along dim k, by permuting dim k to the last position,
   looping over fibers and their digit ranges, and permuting back. */
static void fib_dim(const orc_model *m, const orc_fib *f, int k, const zd *h, const zd *x,
                    zd *out, int accumulate, zd *xp, zd *yp)
{
    int64_t n = f->n;
    int nk = m->n[k];
    const int64_t *perm = f->perm[k];
    for (int64_t q = 0; q < n; ++q) { xp[q] = x[perm[q]]; yp[q] = 0.0; }  /* permute */
    for (int64_t fi = 0; fi < f->nfib[k]; ++fi) {
        int64_t base = f->fstart[k][fi];
        for (int64_t rl = f->rstart[k][fi]; rl < f->rstart[k][fi + 1]; ++rl) {
            for (int l = f->rlo[k][rl]; l <= f->rhi[k][rl]; ++l) {
                int64_t ql = base + f->roff[k][rl] + (l - f->rlo[k][rl]);
                zd acc = 0.0;
                for (int64_t rj = f->rstart[k][fi]; rj < f->rstart[k][fi + 1]; ++rj) {
                    for (int j = f->rlo[k][rj]; j <= f->rhi[k][rj]; ++j) {
                        int64_t qj = base + f->roff[k][rj] + (j - f->rlo[k][rj]);
                        acc += h[(size_t)l * nk + j] * xp[qj];
                    }
                }
                yp[ql] = acc;
            }
        }
    }
    for (int64_t q = 0; q < n; ++q) {                                       /* permute back */
        if (accumulate) out[perm[q]] += yp[q]; else out[perm[q]] = yp[q];
    }
}

int orc_apply_fib(const orc_model *m, const orc_fib *f, const double *xin, double *yout)
{
    int64_t n = f->n;
    size_t nn = (size_t)(n > 0 ? n : 1);
    const zd *x = (const zd *)xin;
    zd *y = (zd *)yout;
    zd *xp = malloc(sizeof(zd) * nn), *yp = malloc(sizeof(zd) * nn);
    for (int64_t p = 0; p < n; ++p) y[p] = f->vdiag[p] * x[p];
    for (int k = 0; k < m->D; ++k)
        if (m->h[k]) fib_dim(m, f, k, m->h[k], x, y, 1, xp, yp);
    if (m->np) {
        zd *z = malloc(sizeof(zd) * nn), *t2 = malloc(sizeof(zd) * nn);
        for (int t = 0; t < m->np; ++t) {
            for (int64_t p = 0; p < n; ++p) z[p] = x[p];
            for (int g = m->pnf[t] - 1; g >= 0; --g) {
                fib_dim(m, f, m->pk[t * ORC_MAXD + g], m->ph[t * ORC_MAXD + g], z, t2, 0, xp, yp);
                for (int64_t p = 0; p < n; ++p) z[p] = t2[p];
            }
            for (int64_t p = 0; p < n; ++p) y[p] += m->pcoef[t] * z[p];
        }
        free(z);
        free(t2);
    }
    free(xp);
    free(yp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* small dense linear algebra (m x m, m <= 64)                              */
/* ------------------------------------------------------------------------ */

/* Cyclic Jacobi eigen-decomposition of a real symmetric matrix a (n x n,
   row-major, destroyed).  On return lam[i] are eigenvalues and column i of z
   the eigenvector. */
static void jacobi_eig(int n, double *a, double *lam, double *z)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) z[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += a[i * n + j] * a[i * n + j];
                if (i != j) off += a[i * n + j] * a[i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double apq = a[p * n + q];
                if (apq == 0.0) continue;
                double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {       /* rotate columns p, q */
                    double akp = a[k * n + p], akq = a[k * n + q];
                    a[k * n + p] = c * akp - s * akq;
                    a[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {       /* rotate rows p, q */
                    double apk = a[p * n + k], aqk = a[q * n + k];
                    a[p * n + k] = c * apk - s * aqk;
                    a[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double zkp = z[k * n + p], zkq = z[k * n + q];
                    z[k * n + p] = c * zkp - s * zkq;
                    z[k * n + q] = s * zkp + c * zkq;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) lam[i] = a[i * n + i];
}

/* exp(A) for a complex n x n matrix by scaling and squaring of a Taylor series. */
static void cexpm(int n, const zd *a, zd *out)
{
    double norm = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = 0.0;
        for (int j = 0; j < n; ++j) r += cabs(a[i * n + j]);
        if (r > norm) norm = r;
    }
    int s = 0;
    while (norm > 0.25) { norm *= 0.5; ++s; }
    double scale = ldexp(1.0, -s);
    zd *b = malloc(sizeof(zd) * n * n), *term = malloc(sizeof(zd) * n * n), *tmp = malloc(sizeof(zd) * n * n);
    for (int i = 0; i < n * n; ++i) b[i] = a[i] * scale;
    for (int i = 0; i < n * n; ++i) { out[i] = 0.0; term[i] = 0.0; }
    for (int i = 0; i < n; ++i) { out[i * n + i] = 1.0; term[i * n + i] = 1.0; }
    for (int kterm = 1; kterm <= 30; ++kterm) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                zd acc = 0.0;
                for (int l = 0; l < n; ++l) acc += term[i * n + l] * b[l * n + j];
                tmp[i * n + j] = acc / (double)kterm;
            }
        memcpy(term, tmp, sizeof(zd) * n * n);
        for (int i = 0; i < n * n; ++i) out[i] += term[i];
    }
    for (int r = 0; r < s; ++r) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                zd acc = 0.0;
                for (int l = 0; l < n; ++l) acc += out[i * n + l] * out[l * n + j];
                tmp[i * n + j] = acc;
            }
        memcpy(out, tmp, sizeof(zd) * n * n);
    }
    free(b); free(term); free(tmp);
}

/* exposed for the tests: y = exp(-i dt T) e_1 for a real symmetric tridiagonal T */
int orc_tridiag_expv(int n, const double *alpha, const double *beta, double dt, double *yout)
{
    double *a = calloc((size_t)n * n, sizeof(double));
    double *lam = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n * n);
    for (int i = 0; i < n; ++i) {
        a[i * n + i] = alpha[i];
        if (i + 1 < n) { a[i * n + i + 1] = beta[i]; a[(i + 1) * n + i] = beta[i]; }
    }
    jacobi_eig(n, a, lam, z);
    zd *y = (zd *)yout;
    for (int j = 0; j < n; ++j) {
        zd acc = 0.0;
        for (int i = 0; i < n; ++i) acc += z[j * n + i] * cexp(-I * lam[i] * dt) * z[0 * n + i];
        y[j] = acc;
    }
    free(a); free(lam); free(z);
    return 0;
}

int orc_cexpm(int n, const double *ain, double *out)
{
    cexpm(n, (const zd *)ain, (zd *)out);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* state                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct orc_state {
    int64_t n;
    uint64_t *keys;
    zd *c;
    int nsub;                   /* substeps the next controlled step starts with */
} orc_state;

orc_state *orc_state_new(void) { return calloc(1, sizeof(orc_state)); }

void orc_state_free(orc_state *s)
{
    if (!s) return;
    free(s->keys);
    free(s->c);
    free(s);
}

int orc_state_set(orc_state *s, int64_t n, const uint64_t *keys, const double *c)
{
    for (int64_t p = 1; p < n; ++p)
        if (keys[p] <= keys[p - 1]) return -1;
    free(s->keys);
    free(s->c);
    s->n = n;
    s->nsub = 1;
    s->keys = malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    s->c = malloc(sizeof(zd) * (size_t)(n > 0 ? n : 1));
    if (n) {
        memcpy(s->keys, keys, sizeof(uint64_t) * (size_t)n);
        memcpy(s->c, c, sizeof(zd) * (size_t)n);
    }
    return 0;
}

int64_t orc_state_count(const orc_state *s) { return s->n; }

void orc_state_get(const orc_state *s, uint64_t *keys, double *c)
{
    if (!s->n) return;
    memcpy(keys, s->keys, sizeof(uint64_t) * (size_t)s->n);
    memcpy(c, s->c, sizeof(zd) * (size_t)s->n);
}

/* ------------------------------------------------------------------------ */
/* SIL: short-iterative Lanczos / Arnoldi                                   */
/* ------------------------------------------------------------------------ */
static zd cdot(int64_t n, const zd *a, const zd *b)   /* <a|b> */
{
    zd acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += conj(a[i]) * b[i];
    return acc;
}

/* One step psi <- exp(-i H dt) psi in the order-m Krylov space; returns the
   Krylov dimension actually used.  alpha0 (if not NULL) receives <v0|H v0>. */
int orc_sil_step(const orc_model *m, const orc_fib *f, orc_state *s, double dt, int mk, int arnoldi,
                 double *alpha0)
{
    int64_t n = s->n;
    if (n == 0) return 0;
    zd **V = malloc(sizeof(zd *) * (mk + 1));
    for (int j = 0; j <= mk; ++j) V[j] = malloc(sizeof(zd) * (size_t)n);
    zd *w = malloc(sizeof(zd) * (size_t)n);
    zd *hk = calloc((size_t)(mk + 1) * mk, sizeof(zd));   /* Hessenberg (Arnoldi) */
    double *alpha = calloc(mk, sizeof(double)), *beta = calloc(mk, sizeof(double));
    zd *h1 = malloc(sizeof(zd) * mk), *h2 = malloc(sizeof(zd) * mk);

    double n0 = sqrt(creal(cdot(n, s->c, s->c)));
    for (int64_t i = 0; i < n; ++i) V[0][i] = s->c[i] / n0;
    int meff = mk;
    /* error estimate of the order-k step, the first Taylor term the Krylov
       space leaves out: n0 |dt|^k / k! prod_{i<k} beta_i (Park and Light's
       estimate for the short-iterative Lanczos; a magnitude, so a backward
       step is judged like a forward one); with a tolerance set, the step
       stops at the first order whose estimate is within it */
    double est = n0;
    for (int j = 0; j < mk; ++j) {
        orc_apply_fib(m, f, (const double *)V[j], (double *)w);
        for (int i = 0; i <= j; ++i) h1[i] = cdot(n, V[i], w);
        for (int i = 0; i <= j; ++i)
            for (int64_t p = 0; p < n; ++p) w[p] -= h1[i] * V[i][p];
        for (int i = 0; i <= j; ++i) h2[i] = cdot(n, V[i], w);
        for (int i = 0; i <= j; ++i)
            for (int64_t p = 0; p < n; ++p) w[p] -= h2[i] * V[i][p];
        alpha[j] = creal(h1[j]);
        if (j == 0 && alpha0) *alpha0 = alpha[0];
        for (int i = 0; i <= j; ++i) hk[i * mk + j] = h1[i] + h2[i];
        double b = sqrt(creal(cdot(n, w, w)));
        beta[j] = b;
        if (j < mk - 1) {
            if (b < 1e-13) { meff = j + 1; break; }
            est = est * fabs(dt) * b / (double)(j + 1);
            if (m->krylov_tol > 0.0 && est <= m->krylov_tol) { meff = j + 1; break; }
            hk[(j + 1) * mk + j] = b;
            for (int64_t p = 0; p < n; ++p) V[j + 1][p] = w[p] / b;
        }
    }
    zd *y = malloc(sizeof(zd) * meff);
    if (!arnoldi) {
        orc_tridiag_expv(meff, alpha, beta, dt, (double *)y);
    } else {
        zd *a = calloc((size_t)meff * meff, sizeof(zd)), *e = calloc((size_t)meff * meff, sizeof(zd));
        for (int i = 0; i < meff; ++i)
            for (int j = 0; j < meff; ++j) a[i * meff + j] = -I * dt * hk[i * mk + j];
        cexpm(meff, a, e);
        for (int j = 0; j < meff; ++j) y[j] = e[j * meff + 0];
        free(a);
        free(e);
    }
    for (int64_t p = 0; p < n; ++p) {
        zd acc = 0.0;
        for (int j = 0; j < meff; ++j) acc += y[j] * V[j][p];
        s->c[p] = n0 * acc;
    }
    for (int j = 0; j <= mk; ++j) free(V[j]);
    free(V); free(w); free(hk); free(alpha); free(beta); free(h1); free(h2); free(y);
    return meff;
}

/* ------------------------------------------------------------------------ */
/* adaption: hash set of used functions                                     */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t *slot; uint64_t cap; uint64_t count; } keyset;
#define EMPTY_SLOT UINT64_MAX

static uint64_t mix64(uint64_t x)
{
    x ^= x >> 30; x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27; x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}

static void ks_init(keyset *s, uint64_t expect)
{
    uint64_t cap = 16;
    while (cap < 2 * expect + 16) cap <<= 1;
    s->cap = cap;
    s->count = 0;
    s->slot = malloc(sizeof(uint64_t) * cap);
    for (uint64_t i = 0; i < cap; ++i) s->slot[i] = EMPTY_SLOT;
}

static void ks_insert(keyset *s, uint64_t key);

static void ks_grow(keyset *s)
{
    keyset t;
    t.cap = s->cap * 2;
    t.count = 0;
    t.slot = malloc(sizeof(uint64_t) * t.cap);
    for (uint64_t i = 0; i < t.cap; ++i) t.slot[i] = EMPTY_SLOT;
    for (uint64_t i = 0; i < s->cap; ++i)
        if (s->slot[i] != EMPTY_SLOT) ks_insert(&t, s->slot[i]);
    free(s->slot);
    *s = t;
}

static void ks_insert(keyset *s, uint64_t key)
{
    if (2 * (s->count + 1) > s->cap) ks_grow(s);
    uint64_t i = mix64(key) & (s->cap - 1);
    while (s->slot[i] != EMPTY_SLOT) {
        if (s->slot[i] == key) return;
        i = (i + 1) & (s->cap - 1);
    }
    s->slot[i] = key;
    s->count++;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

static int above(zd c, double eps2)
{
    double re = creal(c), im = cimag(c);
    double s = re * re + im * im;   /* no contraction: built with -ffp-contract=off */
    return s >= eps2;
}

/* Phase-space axes of a function: one per DVR dimension (its grid index),
   two per lattice dimension (the cell index s and the level l of its (s, l)
   pair).  Fills each axis' index, extent and key stride; returns the count. */
static int phase_axes(const orc_model *m, uint64_t key, int *idx, int *ext, int64_t *str)
{
    int na = 0;
    for (int k = 0; k < m->D; ++k) {
        int d = digit(m, key, k);
        if (m->lat_s[k] == 0) {
            idx[na] = d;
            ext[na] = m->n[k];
            str[na++] = (int64_t)m->stride[k];
        } else {
            int nl = m->lat_l[k];
            idx[na] = d / nl;
            ext[na] = m->lat_s[k];
            str[na++] = (int64_t)nl * (int64_t)m->stride[k];
            idx[na] = d % nl;
            ext[na] = nl;
            str[na++] = (int64_t)m->stride[k];
        }
    }
    return na;
}

/* inserts key and its nearest neighbours (line: +-1; lattice: (s+-1,l), (s,l+-1)) */
static void insert_with_neighbours(const orc_model *m, keyset *set, uint64_t key)
{
    ks_insert(set, key);
    for (int k = 0; k < m->D; ++k) {
        int d = digit(m, key, k);
        uint64_t sk = m->stride[k];
        if (m->lat_s[k] == 0) {
            if (d - 1 >= 0) ks_insert(set, key - sk);
            if (d + 1 < m->n[k]) ks_insert(set, key + sk);
        } else {
            int nl = m->lat_l[k], ns = m->lat_s[k];
            int sidx = d / nl, l = d % nl;
            if (sidx - 1 >= 0) ks_insert(set, key - (uint64_t)nl * sk);
            if (sidx + 1 < ns) ks_insert(set, key + (uint64_t)nl * sk);
            if (l - 1 >= 0) ks_insert(set, key - sk);
            if (l + 1 < nl) ks_insert(set, key + sk);
        }
    }
    if (m->stencil == 1) return;
    /* the wider balls of Sec. III.A count index changes in phase space: the
       grid index of each DVR dimension and the cell and level indices of
       each lattice dimension are separate axes */
    int idx[2 * ORC_MAXD], ext[2 * ORC_MAXD];
    int64_t str[2 * ORC_MAXD];
    int na = phase_axes(m, key, idx, ext, str);
    /* ball radius sqrt(2): +-1 on two axes at once as well (2D^2 neighbours
       on a DVR grid) */
    if (m->stencil == 2)
        for (int a = 0; a < na; ++a)
            for (int b = a + 1; b < na; ++b)
                for (int da = -1; da <= 1; da += 2)
                    for (int db = -1; db <= 1; db += 2) {
                        if (idx[a] + da < 0 || idx[a] + da >= ext[a] || idx[b] + db < 0 || idx[b] + db >= ext[b])
                            continue;
                        ks_insert(set, (uint64_t)((int64_t)key + da * str[a] + db * str[b]));
                    }
    /* ball radius 2: every combination of -1/0/+1 changes over the axes
       (3^D - 1 neighbours on a DVR grid); combinations counted in base 3 */
    if (m->stencil == 3) {
        int ncomb = 1;
        for (int a = 0; a < na; ++a) ncomb *= 3;
        for (int c = 0; c < ncomb; ++c) {
            int rest = c, inside = 1;
            int64_t shift = 0;
            for (int a = 0; a < na; ++a) {
                int da = rest % 3 - 1;
                rest /= 3;
                if (idx[a] + da < 0 || idx[a] + da >= ext[a]) inside = 0;
                shift += da * str[a];
            }
            if (inside) ks_insert(set, (uint64_t)((int64_t)key + shift));
        }
    }
}

/* Tolerance of the adaptive SIL order (0: always the full order). */
int orc_set_krylov_tol(orc_model *m, double tol)
{
    if (!(tol >= 0.0)) return -1;
    m->krylov_tol = tol;
    return 0;
}

/* Step size control: with a Krylov tolerance set, each step of length dt runs
   as s substeps of dt/s (s <= max_substeps; 1 = off). */
int orc_set_max_substeps(orc_model *m, int smax)
{
    if (smax < 1 || smax > 1024) return -1;
    m->max_substeps = smax;
    return 0;
}

/* Selects the adaption stencil (1: radius 1; 2: radius sqrt(2); 3: radius 2). */
int orc_set_stencil(orc_model *m, int stencil)
{
    if (stencil < 1 || stencil > 3) return -1;
    m->stencil = stencil;
    return 0;
}

static void set_from_keyset(keyset *set, uint64_t **out, int64_t *nout)
{
    uint64_t *keys = malloc(sizeof(uint64_t) * (set->count ? set->count : 1));
    int64_t c = 0;
    for (uint64_t i = 0; i < set->cap; ++i)
        if (set->slot[i] != EMPTY_SLOT) keys[c++] = set->slot[i];
    qsort(keys, (size_t)c, sizeof(uint64_t), cmp_u64);
    *out = keys;
    *nout = c;
}

/* Adapts the set; returns |S| (number of coefficients at or above eps).
   rel_excl: functions are dropped only if more than rel_excl*|A| would go. */
int64_t orc_prune(const orc_model *m, orc_state *s, double eps, double rel_excl)
{
    double eps2 = eps * eps;
    keyset set;
    ks_init(&set, (uint64_t)s->n * 2 + 16);
    int64_t nabove = 0;
    for (int64_t p = 0; p < s->n; ++p) {
        if (above(s->c[p], eps2)) {
            ++nabove;
            insert_with_neighbours(m, &set, s->keys[p]);
        }
    }
    if (rel_excl > 0.0) {
        int64_t kept = 0;
        for (int64_t p = 0; p < s->n; ++p) {
            uint64_t key = s->keys[p];
            uint64_t i = mix64(key) & (set.cap - 1);
            while (set.slot[i] != EMPTY_SLOT && set.slot[i] != key) i = (i + 1) & (set.cap - 1);
            if (set.slot[i] == key) ++kept;
        }
        if ((double)(s->n - kept) <= rel_excl * (double)s->n)
            for (int64_t p = 0; p < s->n; ++p) ks_insert(&set, s->keys[p]);
    }
    uint64_t *nk;
    int64_t nn;
    set_from_keyset(&set, &nk, &nn);
    free(set.slot);
    zd *nc = malloc(sizeof(zd) * (size_t)(nn ? nn : 1));
    for (int64_t q = 0; q < nn; ++q) {
        int64_t p = find_key(s->keys, s->n, nk[q]);
        nc[q] = (p >= 0) ? s->c[p] : 0.0;
    }
    free(s->keys);
    free(s->c);
    s->keys = nk;
    s->c = nc;
    s->n = nn;
    return nabove;
}

/* Value of the product state prod_k tab_k[i_k] (complex, product taken in
   dimension order); tabs is [D][nmax] complex interleaved. */
static zd product_value(const orc_model *m, const zd *tabs, uint64_t key)
{
    zd v = 1.0;
    for (int k = 0; k < m->D; ++k) v *= tabs[(size_t)k * m->nmax + digit(m, key, k)];
    return v;
}

/* Initial state: A0 = neighbours of {I : |psi0_I| >= eps} over the full grid,
   coefficients psi0 on A0.  Returns |S0|. */
int64_t orc_init_product(const orc_model *m, orc_state *s, const double *tabs_in, double eps)
{
    const zd *tabs = (const zd *)tabs_in;
    double eps2 = eps * eps;
    keyset set;
    ks_init(&set, 1024);
    int64_t nabove = 0;
    for (uint64_t key = 0; key < m->total; ++key) {
        zd v = product_value(m, tabs, key);
        if (above(v, eps2)) {
            ++nabove;
            insert_with_neighbours(m, &set, key);
        }
    }
    uint64_t *nk;
    int64_t nn;
    set_from_keyset(&set, &nk, &nn);
    free(set.slot);
    free(s->keys);
    free(s->c);
    s->keys = nk;
    s->n = nn;
    s->c = malloc(sizeof(zd) * (size_t)(nn ? nn : 1));
    for (int64_t q = 0; q < nn; ++q) s->c[q] = product_value(m, tabs, nk[q]);
    return nabove;
}

/* ------------------------------------------------------------------------ */
/* observables                                                              */
/* ------------------------------------------------------------------------ */
enum { OBS_T, OBS_NORM2, OBS_ENERGY, OBS_ACF_RE, OBS_ACF_IM, OBS_NACT, OBS_NABOVE, OBS_MEFF, OBS_NSUB, OBS_N };

/* One step of length dt on the current set with the integrator's accuracy
   tied to the tolerance (Sec. III.A adapts it to the amplitude threshold; the
   reading here adapts the Krylov order and, with max_substeps > 1, the step
   size).  Without control: one SIL step of order mk.  With control: s
   substeps of dt/s, s starting at the state's nsub; every substep must meet
   the tolerance at an order below mk (the adaptive order stopped early);
   if one does not, the step is redone from its start with 2s substeps (error
   -1 beyond max_substeps).  After a step whose substeps all stopped at order
   mk/2 or below, the next starts with half as many.  *meff_out: the largest
   order of the accepted substeps; *nsub_out: their number. */
static int controlled_step(const orc_model *m, const orc_fib *f, orc_state *s, double dt, int mk, int arnoldi,
                           int *meff_out, int *nsub_out)
{
    if (m->max_substeps <= 1 || !(m->krylov_tol > 0.0)) {
        *meff_out = orc_sil_step(m, f, s, dt, mk, arnoldi, NULL);
        *nsub_out = 1;
        return 0;
    }
    int sub = s->nsub < 1 ? 1 : s->nsub;
    if (sub > m->max_substeps) sub = m->max_substeps;
    zd *save = malloc(sizeof(zd) * (size_t)(s->n > 0 ? s->n : 1));
    memcpy(save, s->c, sizeof(zd) * (size_t)s->n);
    int mo = 0;
    for (;;) {
        int ok = 1;
        mo = 0;
        const double h = dt / (double)sub;
        for (int j = 0; j < sub && ok; ++j) {
            int me = orc_sil_step(m, f, s, h, mk, arnoldi, NULL);
            if (me > mo) mo = me;
            if (me >= mk) ok = 0;
        }
        if (ok) break;
        memcpy(s->c, save, sizeof(zd) * (size_t)s->n);
        sub *= 2;
        if (sub > m->max_substeps) {
            free(save);
            return -1;
        }
    }
    free(save);
    *meff_out = mo;
    *nsub_out = sub;
    s->nsub = (mo <= mk / 2 && sub > 1) ? sub / 2 : sub;
    return 0;
}

/* out: [norm2, energy, acf_re, acf_im, n_active, n_above]; bra is [D][nmax] complex */
int orc_observe(const orc_model *m, const orc_fib *f, const orc_state *s, const double *bra_in,
                double eps, double *out)
{
    const zd *bra = (const zd *)bra_in;
    double eps2 = eps * eps;
    double norm2 = 0.0;
    zd acf = 0.0;
    int64_t nab = 0;
    for (int64_t p = 0; p < s->n; ++p) {
        norm2 += creal(conj(s->c[p]) * s->c[p]);
        acf += conj(product_value(m, bra, s->keys[p])) * s->c[p];
        nab += above(s->c[p], eps2);
    }
    double energy = 0.0;
    if (s->n && norm2 > 0.0) {
        zd *y = malloc(sizeof(zd) * (size_t)s->n);
        orc_apply_fib(m, f, (const double *)s->c, (double *)y);
        energy = creal(cdot(s->n, s->c, y)) / norm2;
        free(y);
    }
    out[0] = norm2;
    out[1] = energy;
    out[2] = creal(acf);
    out[3] = cimag(acf);
    out[4] = (double)s->n;
    out[5] = (double)nab;
    return 0;
}

/* FNV-1a over the little-endian bytes of the sorted keys (active-set fingerprint). */
uint64_t orc_set_hash(int64_t n, const uint64_t *keys)
{
    uint64_t h = 0xcbf29ce484222325ULL;
    for (int64_t p = 0; p < n; ++p) {
        uint64_t k = keys[p];
        for (int b = 0; b < 8; ++b) {
            h ^= (k >> (8 * b)) & 0xffu;
            h *= 0x100000001b3ULL;
        }
    }
    return h;
}

/* Full run: record obs(0); repeat nsteps: SIL step on A, adapt, record obs.
   trace: (nsteps+1) x OBS_N doubles [t, norm2, energy, acf_re, acf_im, n_active,
   n_above, krylov_used]; hashes: (nsteps+1) set fingerprints.  eps < 0 disables
   adaption (unpruned run on the given set). */
int orc_propagate(const orc_model *m, orc_state *s, int nsteps, double dt, int mk, double eps, int arnoldi,
                  const double *bra, double *trace, uint64_t *hashes)
{
    orc_fib *f = orc_fib_build(m, s->n, s->keys);
    double o[6];
    double eps_obs = eps < 0 ? 0.0 : eps;
    orc_observe(m, f, s, bra, eps_obs, o);
    trace[OBS_T] = 0.0;
    for (int i = 0; i < 6; ++i) trace[1 + i] = o[i];
    trace[OBS_MEFF] = 0.0;
    trace[OBS_NSUB] = 0.0;
    if (hashes) hashes[0] = orc_set_hash(s->n, s->keys);
    for (int st = 1; st <= nsteps; ++st) {
        int meff, nsub;
        if (controlled_step(m, f, s, dt, mk, arnoldi, &meff, &nsub) != 0) {
            orc_fib_free(f);
            return -1;
        }
        if (eps >= 0.0) {
            orc_prune(m, s, eps, 0.0);
            orc_fib_free(f);
            f = orc_fib_build(m, s->n, s->keys);
        }
        orc_observe(m, f, s, bra, eps_obs, o);
        double *r = trace + (size_t)st * OBS_N;
        r[OBS_T] = st * dt;
        for (int i = 0; i < 6; ++i) r[1 + i] = o[i];
        r[OBS_MEFF] = meff;
        r[OBS_NSUB] = nsub;
        if (hashes) hashes[st] = orc_set_hash(s->n, s->keys);
    }
    orc_fib_free(f);
    return 0;
}

/* Test access to the stored fiber structure of dim k: number of fibers, and
   for fiber fi its member count and digit ranges (rlo/rhi, up to cap). */
int64_t orc_fib_count(const orc_fib *f, int k) { return f->nfib[k]; }

int orc_fib_ranges(const orc_fib *f, int k, int64_t fi, int cap, int32_t *lo, int32_t *hi)
{
    if (fi < 0 || fi >= f->nfib[k]) return -1;
    int nr = 0;
    for (int64_t r = f->rstart[k][fi]; r < f->rstart[k][fi + 1]; ++r, ++nr)
        if (nr < cap) { lo[nr] = f->rlo[k][r]; hi[nr] = f->rhi[k][r]; }
    return nr;
}

/* O-def at selected output positions only: out[s] = (P H P x)[idx[s]].
   Used to check very large sets on a sample of outputs. */
int orc_apply_def_at(const orc_model *m, int64_t n, const uint64_t *keys, const double *xin, int64_t ns,
                     const int64_t *idx, double *yout)
{
    const zd *x = (const zd *)xin;
    zd *y = (zd *)yout;
    if (m->np) return -1;  /* product terms need the full intermediate */
    for (int64_t s = 0; s < ns; ++s) {
        int64_t p = idx[s];
        uint64_t key = keys[p];
        zd acc = potential_at(m, key) * x[p];
        for (int k = 0; k < m->D; ++k) {
            if (!m->h[k]) continue;
            int nk = m->n[k];
            int dk = digit(m, key, k);
            uint64_t base = key - (uint64_t)dk * m->stride[k];
            for (int j = 0; j < nk; ++j) {
                int64_t q = find_key(keys, n, base + (uint64_t)j * m->stride[k]);
                if (q >= 0) acc += m->h[k][(size_t)dk * nk + j] * x[q];
            }
        }
        y[s] = acc;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* frozen active-set trajectories (reference of the adjoint gradient)       */
/* ------------------------------------------------------------------------ */
/* Remaps the state onto the given sorted set (coefficients carried over on
   the intersection, zero elsewhere): the restriction R of one adaption. */
static void remap_to(orc_state *s, int64_t n, const uint64_t *keys)
{
    zd *nc = malloc(sizeof(zd) * (size_t)(n ? n : 1));
    for (int64_t q = 0; q < n; ++q) {
        int64_t p = find_key(s->keys, s->n, keys[q]);
        nc[q] = (p >= 0) ? s->c[p] : 0.0;
    }
    free(s->keys);
    free(s->c);
    s->keys = malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    if (n) memcpy(s->keys, keys, sizeof(uint64_t) * (size_t)n);
    s->c = nc;
    s->n = n;
}

/* Pruned forward run that records the active sets: set_sizes[0..nsteps],
   keys appended to *keys_out (malloc'd; caller frees with orc_free_buffer). */
int orc_propagate_record(const orc_model *m, orc_state *s, int nsteps, double dt, int mk, double eps,
                         int64_t *set_sizes, uint64_t **keys_out)
{
    int64_t cap = 1024, used = 0;
    uint64_t *buf = malloc(sizeof(uint64_t) * cap);
    for (int st = 0; st <= nsteps; ++st) {
        if (st > 0) {
            orc_fib *f = orc_fib_build(m, s->n, s->keys);
            int meff, nsub;
            int r = controlled_step(m, f, s, dt, mk, 0, &meff, &nsub);
            orc_fib_free(f);
            if (r != 0) {
                free(buf);
                return -1;
            }
            orc_prune(m, s, eps, 0.0);
        }
        set_sizes[st] = s->n;
        if (used + s->n > cap) {
            while (used + s->n > cap) cap *= 2;
            buf = realloc(buf, sizeof(uint64_t) * cap);
        }
        memcpy(buf + used, s->keys, sizeof(uint64_t) * (size_t)s->n);
        used += s->n;
    }
    *keys_out = buf;
    return 0;
}

void orc_free_buffer(void *p) { free(p); }

/* Forward map with frozen sets: the state (on set 0) takes nsteps SIL steps,
   each followed by the restriction to the next recorded set. */
int orc_propagate_frozen(const orc_model *m, orc_state *s, int nsteps, double dt, int mk, const int64_t *set_sizes,
                         const uint64_t *keys)
{
    int64_t off = set_sizes[0];
    for (int st = 1; st <= nsteps; ++st) {
        orc_fib *f = orc_fib_build(m, s->n, s->keys);
        int meff, nsub;
        int r = controlled_step(m, f, s, dt, mk, 0, &meff, &nsub);
        orc_fib_free(f);
        if (r != 0) return -1;
        remap_to(s, set_sizes[st], keys + off);
        off += set_sizes[st];
    }
    return 0;
}
