// C ABI (include/ppq.h): context, operator assembly, state, and the
// orchestration of one propagation step on one HIP stream.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "ppq_internal.hpp"
#include "ppq_model.hpp"

using namespace ppq;

namespace {

struct Factor {
    int dim;
    int kind;
    double p0, p1;
    std::vector<double> table;
};
struct Term {
    double coef;
    double coef_im = 0.0;  // imaginary part of the coefficient (ppq_add_term)
    std::vector<Factor> f;
};

// a product term with two dense factors and no diagonal ones, grouped with
// the others sharing its inner factor for evaluation
struct PairTerm {
    double cre, cim;  // coefficient
    int k1, f1;  // outer factor (lower dimension), index into dense factor list
    int k2, f2;  // inner factor (applied first)
};

// any other product term: diagonal factors (DVR dimensions in `use`, values
// in a [D][nmax] table) scale the input, then the dense factors act from the
// highest dimension down, each result truncated to the set
struct ProdTerm {
    double cre, cim;
    int nf = 0;        // dense factors, dimensions increasing
    int k[MAXD]{};
    int fid[MAXD]{};   // index into the dense factor list
    unsigned use = 0;  // dimensions with a diagonal factor
    int diag = -1;     // index of the diagonal table (ctx->PD64)
};

inline bool dense_kind(int kind) { return kind == PPQ_FAC_DENSE_REAL || kind == PPQ_FAC_DENSE_COMPLEX; }

int bucket(int n)
{
    if (n <= 8) return 8;
    if (n <= 16) return 16;
    if (n <= 24) return 24;
    if (n <= 32) return 32;
    if (n <= 48) return 48;
    if (n <= 64) return 64;
    return n;  // a long dimension: its factor is stored unpadded
}

struct HipError {
    hipError_t e;
    const char *what;
};

inline void ck(hipError_t e, const char *what)
{
    if (e != hipSuccess) throw HipError{e, what};
}

template <class T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

template <class T>
T *dalloc(int64_t count)
{
    void *p = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc(&p, (size_t)count * sizeof(T));
    if (e != hipSuccess) throw std::bad_alloc();
    return (T *)p;
}

}  // namespace

struct ppq_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int precision = PPQ_FP64;
    std::string err;
    bool poisoned = false;

    // grid
    bool has_grid = false;
    GridDesc g{};
    double lo[MAXD]{}, hi[MAXD]{}, mass = 1.0;
    int nb[MAXD]{};  // padded 1D size per dimension
    bool lattice[MAXD]{};
    bool weylets[MAXD]{};   // lattice dimension built from projected Weylets (else projected von Neumann)
    bool fgh[MAXD]{};       // periodic Fourier-grid dimension (else sine-DVR)
    bool any_lattice = false;
    int64_t nwords = 0;

    // operator (host description)
    std::vector<Term> terms;
    bool op_dirty = true;
    // built operator (device)
    double *T64[MAXD]{};   // real factor per DVR dimension (kinetic), nb x nb
    float *T32[MAXD]{};
    float *T32p[MAXD]{};   // factors zero-padded to 64 x 64 (matrix-core tiles)
    double *T64p[MAXD]{};
    double2 *H64p[MAXD]{};
    float2 *H32p[MAXD]{};
    std::vector<double2 *> F64p;
    std::vector<float2 *> F32p;
    double2 *H64[MAXD]{};  // complex factor per lattice dimension
    float2 *H32[MAXD]{};
    std::vector<double2 *> F64;  // distinct dense factors of product terms
    std::vector<float2 *> F32;
    std::vector<int> Fdim;
    std::vector<PairTerm> pairs;
    std::vector<ProdTerm> chains;
    std::vector<double *> PD64;   // diagonal tables of chain terms, [D][pd_nmax]
    int pd_nmax = 0;
    bool hermitian = true;        // P H P Hermitian: Lanczos (else Arnoldi)
    bool real_sym = true;         // ... and real symmetric (C(2t) from the state at t)
    bool dvr_real_sym = true;     // the operator in the DVR basis is real symmetric
                                  // (lattice bases: a similarity of it)
    double2 *full[2]{};           // full-grid tensors of C(2t) on lattice bases
    int64_t full_cap = 0;
    double *pot_coef = nullptr;
    int *pot_tab = nullptr;
    double *pot_tabs = nullptr;
    int pot_nterm = 0;
    int pot_nmax = 0;
    int pot_ntab = 0;

    // state
    int64_t cap = 0;
    int64_t nact = 0;
    bool has_state = false;
    int cur = 0;
    uint32_t *keys[2]{};
    double2 *psi[2]{};
    double2 *psi_tmp = nullptr;
    double *V64 = nullptr;
    float *V32 = nullptr;
    double *Vt64 = nullptr;  // the previous set's potential while it is carried over
    float *Vt32 = nullptr;
    bool derived_valid = false;  // fibers + potential cache match the set
    bool v_valid = false;        // V matches the current set and operator
    bool v_partial = false;      // V holds the carried-over values, NaN where new

    // fiber tables
    uint32_t *pi[MAXD]{};
    uint32_t *off[MAXD]{};
    uint64_t *mask[MAXD]{};
    uint8_t *info[MAXD]{};
    int64_t nf[MAXD]{};
    int hpsi_variant = 2;  // H*psi layout (PPQ_HPSI overrides; 4, 5 = block-fused, 6 = plane passes,
                           // 7 = the last two dimensions in one pass)
    uint32_t blk_window = BLOCK_WINDOW;  // chunk window of the block layouts (PPQ_BLOCK_WINDOW)
    int blk_unroll = 1;                  // one-lane-per-fiber block pass: row loop unrolled (PPQ_BLOCK_UNROLL)
    bool acc_stage = false;              // lane-per-fiber passes stage pi in LDS (PPQ_ACC_STAGE;
                                         // faster back to back in FP32, slower within steps)

    // block-fused H*psi: outer dimensions [0, split) through the inner-first
    // frame, inner dimensions [split, D) in the row-major frame
    int split = 0;
    bool block_ok = false;    // the operator and grid admit the block form
    bool block_mode = false;  // the current set's tables are built for it
    uint32_t *P_R = nullptr, *inv_R = nullptr;
    uint32_t *chunk[2]{}, *big[2]{};
    uint32_t *fch[MAXD]{};  // first fiber of each chunk, per dimension
    uint32_t nch[2]{}, nbig[2]{}, maxch[2]{};

    // plane passes: pairs of adjacent dimensions (D-2, D-1), (D-4, D-3), ...;
    // an odd first dimension keeps its own pass
    bool plane_ok = false;    // the operator and grid admit them
    bool plane_mode = false;  // the current set's plane tables are built
    int npl = 0;
    int pl_a[MAXD]{};         // first dimension of each pair
    uint32_t *plP[MAXD]{}, *pltask[MAXD]{};
    uint16_t *pldig[MAXD]{};
    uint32_t *pl_poff = nullptr;  // plane starts while the tables are built
    int64_t pl_cap = 0;

    // pair pass: the last two dimensions in one pass (whole planes per task)
    bool pair_ok = false;          // the operator and grid admit it
    uint32_t *pair_task = nullptr;  // task starts of the current set
    int64_t pair_cap = 0;

    // <x|y> of a product fused into its last pass (Hermitian Krylov steps)
    bool dot_want = false;  // the caller asks for it
    int dot_nb = 0;         // blocks whose partials the last product stored (0: not fused)

    // work
    uint32_t *flags = nullptr, *fidx = nullptr;
    uint64_t *tmpmask = nullptr;
    uint32_t *scan_tmp = nullptr;
    int64_t scan_tmp_n = 0;
    uint64_t *bm = nullptr;
    uint32_t *prefix = nullptr;
    uint64_t *kbm = nullptr;  // adaption: the functions above the threshold (word-parallel dilation)
    int64_t kbm_words = 0;
    int dilate_mode = 0;      // 0: by the sizes, 1: per function (atomics), 2: word by word (PPQ_DILATE)
    uint32_t *small = nullptr;            // device counters
    unsigned long long *count = nullptr;  // device counter
    uint32_t *h_small = nullptr;          // pinned mirrors
    unsigned long long *h_count = nullptr;

    // Krylov
    int kv_m = 0;
    int64_t kv_cap = 0;
    void *Vk = nullptr;
    void *wk = nullptr;
    std::vector<void *> zbuf;  // intermediates of product terms
    KState *ks = nullptr;
    double2 *partial = nullptr;
    unsigned *counter = nullptr;

    // reference packet
    bool has_ref = false;
    double2 *init_tabs = nullptr;
    double2 *bra_tabs = nullptr;
    int tab_nmax = 0;
    double *qtab = nullptr;  // grid points [MAXD][NMAX_FIBER], then MAXD results (position expectations)
    double rel_excl = 0.0;   // relative exclusion threshold of adaption
    double krylov_tol = 0.0; // > 0: SIL order chosen per step by its error estimate
    int max_substeps = 1;    // > 1 (with krylov_tol > 0): step size control
    int nsub = 1;            // substeps the next controlled step starts with
    double *sub_meff = nullptr;    // device: Krylov order of each substep of an attempt
    double *h_sub_meff = nullptr;  // pinned mirror
    int sub_cap = 0;
    double2 *psi_save = nullptr;   // the state at the start of a controlled step
    int64_t psi_save_cap = 0;
    double2 *acf2 = nullptr;  // C(2t) result (device)
    std::vector<double> factor[MAXD];  // caller's 1D factor per dimension (empty: sine-DVR kinetic)
    // fiber tables of all non-last dimensions at once (see fiber_tables_all)
    uint64_t *bmB = nullptr;
    uint32_t *pfxB = nullptr, *scanB = nullptr, *cntB = nullptr;
    uint64_t *occB = nullptr;  // fiber-slot bitmaps of the non-last dimensions
    uint32_t *opfxB = nullptr;
    int64_t bat_cap = 0;     // capacity the batched work space was sized for (0: not allocated)

    // records
    double *rec = nullptr;
    int64_t rec_cap = 0;

    // measurement
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ev_nf = nullptr;    // fiber counts of the last table build copied to h_small
    bool nf_pending = false;       // nf[] not yet read from h_small (see ensure_nf)
    int64_t nf_n = 0;              // set size of that build
    // opt-in phase timing: events recorded at phase boundaries
    bool timing = false;
    std::vector<hipEvent_t> tev;
    std::vector<int> tlabel;  // phase started at each recorded event (-1: none)
    size_t tcount = 0;
    double tms[PPQ_PHASE_N] = {};

    // adjoint: derivative terms dV/dtheta_p, recorded trajectory, work buffers
    std::vector<Term> dterms;
    std::vector<int> dparam;
    int nparam = 0;
    int *d_param = nullptr, *d_dtab = nullptr;
    double *d_dcoef = nullptr, *d_dtabs = nullptr;
    int d_nterm = 0, d_ntab = 0;
    double2 *dtabs = nullptr;  // [2D][nmax]: d psi0 factor / d centre_k, d momentum_k
    double pk_centre[MAXD]{}, pk_momentum[MAXD]{}, pk_width[MAXD]{};
    double rec_centre[MAXD]{}, rec_momentum[MAXD]{};
    bool recorded = false;
    int rec_steps = 0, rec_m = 0, rec_every = 0;
    double rec_tol = 0.0;          // Krylov tolerance of the recorded steps
    std::vector<int> rec_sub;      // substeps of each recorded step
    double rec_dt = 0.0;
    double2 rec_C = make_double2(0.0, 0.0);
    uint32_t *rec_keys = nullptr;
    int64_t rec_keys_cap = 0;
    std::vector<int64_t> rec_off, rec_n;
    std::vector<double2 *> ckpt;
    double2 *seg = nullptr;
    int64_t seg_cap = 0;
    void *Wk = nullptr;
    int64_t wk_cap = 0;
    KState *ks_b = nullptr;
    double2 *Qd = nullptr, *dC = nullptr, *lam = nullptr, *mu = nullptr;
    int64_t adj_cap = 0;
};

namespace {

int fail(ppq_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_fail(ppq_ctx *c, const HipError &e)
{
    c->poisoned = true;
    c->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
    return PPQ_E_HIP;
}

void free_state_buffers(ppq_ctx *c)
{
    for (int i = 0; i < 2; ++i) {
        dfree(c->keys[i]);
        dfree(c->psi[i]);
    }
    dfree(c->psi_tmp);
    dfree(c->psi_save);
    c->psi_save_cap = 0;
    dfree(c->V64);
    dfree(c->V32);
    dfree(c->Vt64);
    dfree(c->Vt32);
    for (int k = 0; k < MAXD; ++k) {
        dfree(c->pi[k]);
        dfree(c->off[k]);
        dfree(c->mask[k]);
        dfree(c->info[k]);
    }
    dfree(c->flags);
    dfree(c->fidx);
    dfree(c->tmpmask);
    dfree(c->scan_tmp);
    dfree(c->P_R);
    dfree(c->inv_R);
    for (int i = 0; i < 2; ++i) {
        dfree(c->chunk[i]);
        dfree(c->big[i]);
    }
    for (int k = 0; k < MAXD; ++k) dfree(c->fch[k]);
    dfree(c->bmB);
    dfree(c->pfxB);
    dfree(c->scanB);
    dfree(c->cntB);
    dfree(c->occB);
    dfree(c->opfxB);
    c->bat_cap = 0;
    for (int i = 0; i < MAXD; ++i) {
        dfree(c->plP[i]);
        dfree(c->pltask[i]);
        dfree(c->pldig[i]);
    }
    dfree(c->pl_poff);
    c->pl_cap = 0;
    c->plane_mode = false;
    dfree(c->pair_task);
    c->pair_cap = 0;
    c->cap = 0;
}

void free_krylov(ppq_ctx *c)
{
    dfree(c->Vk);
    dfree(c->wk);
    for (auto &z : c->zbuf) dfree(z);
    c->zbuf.clear();
    c->kv_m = 0;
    c->kv_cap = 0;
}

void free_operator(ppq_ctx *c)
{
    for (int k = 0; k < MAXD; ++k) {
        dfree(c->T64[k]);
        dfree(c->T32[k]);
        dfree(c->T32p[k]);
        dfree(c->T64p[k]);
        dfree(c->H64p[k]);
        dfree(c->H32p[k]);
        dfree(c->H64[k]);
        dfree(c->H32[k]);
    }
    for (auto &p : c->F64) dfree(p);
    for (auto &p : c->F32) dfree(p);
    for (auto &p : c->F64p) dfree(p);
    for (auto &p : c->F32p) dfree(p);
    c->F64.clear();
    c->F32.clear();
    c->F64p.clear();
    c->F32p.clear();
    c->Fdim.clear();
    c->pairs.clear();
    for (auto &p : c->PD64) dfree(p);
    c->PD64.clear();
    c->chains.clear();
    dfree(c->pot_coef);
    dfree(c->pot_tab);
    dfree(c->pot_tabs);
    c->pot_nterm = 0;
    c->op_dirty = true;
}

// (Re)allocates every per-point buffer for at least n points, keeping the
// current keys and coefficients. A growing set doubles the capacity (never
// past the grid size, which bounds the active set): each growth frees and
// allocates every table, so a set that spreads over a few steps should pay
// for that once or twice, not at every step.
void ensure_capacity(ppq_ctx *c, int64_t n)
{
    if (n <= c->cap) return;
    int64_t nc = std::max<int64_t>(n, std::min<int64_t>(2 * c->cap, (int64_t)c->g.total));
    nc = std::max<int64_t>(nc, 1024);
    uint32_t *nk = dalloc<uint32_t>(nc);
    double2 *np = dalloc<double2>(nc);
    if (c->has_state && c->nact > 0) {
        ck(hipMemcpyAsync(nk, c->keys[c->cur], c->nact * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream),
           "copy keys");
        ck(hipMemcpyAsync(np, c->psi[c->cur], c->nact * sizeof(double2), hipMemcpyDeviceToDevice, c->stream),
           "copy psi");
    }
    ck(hipStreamSynchronize(c->stream), "sync");
    free_state_buffers(c);
    c->cap = nc;
    c->cur = 0;
    c->keys[0] = nk;
    c->psi[0] = np;
    c->keys[1] = dalloc<uint32_t>(nc);
    c->psi[1] = dalloc<double2>(nc);
    c->psi_tmp = dalloc<double2>(nc);
    if (c->precision == PPQ_FP64) {
        c->V64 = dalloc<double>(nc);
        c->Vt64 = dalloc<double>(nc);
    } else {
        c->V32 = dalloc<float>(nc);
        c->Vt32 = dalloc<float>(nc);
    }
    for (int k = 0; k < c->g.D; ++k) {
        if (k < c->g.D - 1) c->pi[k] = dalloc<uint32_t>(nc);
        c->off[k] = dalloc<uint32_t>(nc + 1);
        c->mask[k] = dalloc<uint64_t>(nc);
        c->info[k] = dalloc<uint8_t>(nc);
    }
    c->flags = dalloc<uint32_t>(nc);
    c->fidx = dalloc<uint32_t>(nc);
    c->tmpmask = dalloc<uint64_t>(nc);
    c->scan_tmp_n = std::max(scan_tmp_words(nc), scan_tmp_words(c->nwords));
    c->scan_tmp = dalloc<uint32_t>(c->scan_tmp_n);
    c->P_R = dalloc<uint32_t>(nc);
    c->inv_R = dalloc<uint32_t>(nc);
    for (int i = 0; i < 2; ++i) {
        c->chunk[i] = dalloc<uint32_t>(nc / BLOCK_WINDOW + 2);
        c->big[i] = dalloc<uint32_t>(nc / BLOCK_WINDOW + 2);
    }
    for (int k = 0; k < c->g.D; ++k) c->fch[k] = dalloc<uint32_t>(nc / BLOCK_WINDOW + 2);
    c->derived_valid = false;
    c->v_valid = false;
    c->v_partial = false;
    free_krylov(c);
}

void ensure_krylov(ppq_ctx *c, int m)
{
    if (c->Vk && c->kv_m >= m && c->kv_cap == c->cap) return;
    free_krylov(c);
    size_t es = c->precision == PPQ_FP64 ? sizeof(double2) : sizeof(float2);
    void *p = nullptr;
    if (hipMalloc(&p, es * (size_t)(m + 1) * (size_t)c->cap) != hipSuccess) throw std::bad_alloc();
    c->Vk = p;
    if (hipMalloc(&p, es * (size_t)c->cap) != hipSuccess) throw std::bad_alloc();
    c->wk = p;
    c->kv_m = m;
    c->kv_cap = c->cap;
}

void ensure_zbuf(ppq_ctx *c)
{
    size_t need = std::max(c->F64.size(), c->chains.empty() ? (size_t)0 : (size_t)3);
    if (c->zbuf.size() >= need && c->kv_cap == c->cap && c->Vk) return;
    size_t es = c->precision == PPQ_FP64 ? sizeof(double2) : sizeof(float2);
    while (c->zbuf.size() < need) {
        void *p = nullptr;
        if (hipMalloc(&p, es * (size_t)c->cap) != hipSuccess) throw std::bad_alloc();
        c->zbuf.push_back(p);
    }
}

// ---- operator assembly -------------------------------------------------------
// Grid points of dimension k: sine-DVR interior points of the box, or the
// periodic Fourier grid x_j = lo + j (hi - lo) / n, j = 0..n-1.
// (written into q[0..n_k), no allocation)
void dim_points_into(const ppq_ctx *c, int k, double *q)
{
    const int n = c->g.n[k];
    const double lo = c->lo[k], hi = c->hi[k];
    if (!c->fgh[k]) {
        const double dx = (hi - lo) / (n + 1);
        for (int i = 0; i < n; ++i) q[i] = lo + (i + 1) * dx;
    } else {
        for (int j = 0; j < n; ++j) q[j] = lo + j * (hi - lo) / n;
    }
}

std::vector<double> dim_points(const ppq_ctx *c, int k)
{
    std::vector<double> q(c->g.n[k]);
    dim_points_into(c, k, q.data());
    return q;
}

// Quadrature weight of dimension k's grid: the spacing (hi - lo) / (n + 1) of
// the sine-DVR, (hi - lo) / n of the periodic Fourier grid.
double dim_weight(const ppq_ctx *c, int k)
{
    const int n = c->g.n[k];
    return (c->hi[k] - c->lo[k]) / (c->fgh[k] ? n : n + 1);
}

std::vector<double> factor_values(const ppq_ctx *c, const Factor &f)
{
    int k = f.dim;
    int n = c->g.n[k];
    std::vector<double> q = dim_points(c, k);
    std::vector<double> v(n);
    for (int i = 0; i < n; ++i) {
        if (f.kind == PPQ_FAC_POWER) {
            int p = (int)f.p0;
            double r = 1.0;
            for (int e = 0; e < p; ++e) r *= q[i];
            v[i] = r;
        } else if (f.kind == PPQ_FAC_MORSE) {
            double e = 1.0 - std::exp(-f.p0 * (q[i] - f.p1));
            v[i] = e * e;
        } else if (f.kind == PPQ_FAC_MORSE_DA) {
            double ex = std::exp(-f.p0 * (q[i] - f.p1));
            v[i] = 2.0 * (1.0 - ex) * ex * (q[i] - f.p1);
        } else {
            v[i] = f.table[i];
        }
    }
    return v;
}

// Copies a host table to a new device buffer.  Waits for the copy: the
// callers' host vectors go out of scope on return (set-up paths only).
template <class T>
T *upload(const std::vector<T> &h, hipStream_t s)
{
    T *d = dalloc<T>((int64_t)h.size());
    ck(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
    ck(hipStreamSynchronize(s), "upload");
    return d;
}

// Dense factor on a lattice dimension: G^+ h G^{-+} (padded to nb x nb, complex).
struct LatticeMaps {
    std::vector<cd> G, Gadj, GinvAdj, Ginv;
};

LatticeMaps lattice_maps(const ppq_ctx *c, int k)
{
    LatticeMaps L;
    int n = c->g.n[k];
    const std::vector<double> q = dim_points(c, k);
    L.G = c->weylets[k] ? weylet_projection(q, dim_weight(c, k), c->lo[k], c->hi[k], c->g.lat_s[k], c->g.lat_l[k])
                        : pvb_projection(q, dim_weight(c, k), c->lo[k], c->hi[k], c->g.lat_s[k], c->g.lat_l[k]);
    L.Gadj = adjoint(L.G, n);
    L.GinvAdj = L.Gadj;
    if (!invert(L.GinvAdj, n)) throw std::runtime_error("singular lattice projection");
    L.Ginv = adjoint(L.GinvAdj, n);
    return L;
}

std::vector<cd> similarity(const LatticeMaps &L, const std::vector<cd> &h, int n)
{
    return matmul(matmul(L.Gadj, h, n), L.GinvAdj, n);
}

// The one-dimensional operator of dimension k in its DVR basis: the caller's
// factor when one was set, else the kinetic energy of its grid (Fourier grid
// or sine-DVR).
std::vector<double> dim_factor(const ppq_ctx *c, int k)
{
    if (!c->factor[k].empty()) return c->factor[k];
    if (c->fgh[k]) return fgh_kinetic(c->g.n[k], c->lo[k], c->hi[k], c->mass);
    return sine_dvr_kinetic(c->g.n[k], c->lo[k], c->hi[k], c->mass);
}

// A term applied as a product of matrices (Sec. II.B.2): on a DVR basis one
// with a dense factor or a complex coefficient; on a lattice basis, where
// every factor is dense, one on two or more dimensions (single-dimension terms
// are summed into that dimension's operator).
bool is_product(const ppq_ctx *c, const Term &t)
{
    if (c->any_lattice) {
        unsigned used = 0;
        for (const Factor &f : t.f) used |= 1u << f.dim;
        return __builtin_popcount(used) > 1;
    }
    if (t.coef_im != 0.0) return true;
    for (const Factor &f : t.f)
        if (dense_kind(f.kind)) return true;
    return false;
}

// A factor as an n_k x n_k complex matrix in its dimension's DVR basis
// (diagonal kinds on the diagonal).
std::vector<cd> factor_matrix(const ppq_ctx *c, const Factor &f)
{
    const int n = c->g.n[f.dim];
    std::vector<cd> h((size_t)n * n, cd(0.0, 0.0));
    if (f.kind == PPQ_FAC_DENSE_REAL) {
        for (size_t i = 0; i < h.size(); ++i) h[i] = cd(f.table[i], 0.0);
    } else if (f.kind == PPQ_FAC_DENSE_COMPLEX) {
        for (size_t i = 0; i < h.size(); ++i) h[i] = cd(f.table[2 * i], f.table[2 * i + 1]);
    } else {
        const std::vector<double> v = factor_values(c, f);
        for (int i = 0; i < n; ++i) h[(size_t)i * n + i] = cd(v[i], 0.0);
    }
    return h;
}

void build_operator(ppq_ctx *c)
{
    if (!c->op_dirty) return;
    for (int k = 0; k < MAXD; ++k) {
        dfree(c->T64[k]);
        dfree(c->T32[k]);
        dfree(c->T32p[k]);
        dfree(c->T64p[k]);
        dfree(c->H64p[k]);
        dfree(c->H32p[k]);
        dfree(c->H64[k]);
        dfree(c->H32[k]);
    }
    for (auto &p : c->F64) dfree(p);
    for (auto &p : c->F32) dfree(p);
    for (auto &p : c->F64p) dfree(p);
    for (auto &p : c->F32p) dfree(p);
    c->F64.clear();
    c->F32.clear();
    c->F64p.clear();
    c->F32p.clear();
    c->Fdim.clear();
    c->pairs.clear();
    for (auto &p : c->PD64) dfree(p);
    c->PD64.clear();
    c->chains.clear();
    dfree(c->pot_coef);
    dfree(c->pot_tab);
    dfree(c->pot_tabs);
    const int D = c->g.D;
    hipStream_t s = c->stream;
    auto pad_upload = [&](const std::vector<cd> &h, int n, int b, double2 **d64, float2 **d32) {
        std::vector<double2> P((size_t)b * b, make_double2(0.0, 0.0));
        std::vector<float2> Pf((size_t)b * b, make_float2(0.f, 0.f));
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                cd v = h[(size_t)i * n + j];
                P[(size_t)i * b + j] = make_double2(v.real(), v.imag());
                Pf[(size_t)i * b + j] = make_float2((float)v.real(), (float)v.imag());
            }
        *d64 = upload(P, s);
        *d32 = upload(Pf, s);
    };
    // distinct dense factors of product terms, keyed by (dim, matrix), as they
    // act on the coefficients (transformed on lattice dimensions)
    std::vector<std::vector<cd>> fmats;
    auto factor_id = [&](int k, const std::vector<cd> &m) {
        for (size_t i = 0; i < fmats.size(); ++i)
            if (c->Fdim[i] == k && fmats[i] == m) return (int)i;
        fmats.push_back(m);
        c->Fdim.push_back(k);
        return (int)fmats.size() - 1;
    };
    int pd_nmax = 1;
    for (int k = 0; k < D; ++k) pd_nmax = std::max(pd_nmax, c->g.n[k]);
    c->pd_nmax = pd_nmax;
    // Registers a product term given its dense factors (dimensions increasing)
    // and, on DVR dimensions, the values of its diagonal factors per dimension.
    auto add_product = [&](double cre, double cim, const std::vector<int> &dk,
                           const std::vector<std::vector<cd>> &dm, const std::vector<std::vector<double>> &diag) {
        unsigned use = 0;
        for (int k = 0; k < D; ++k)
            if (!diag[k].empty()) use |= 1u << k;
        if (use == 0 && dk.size() == 2) {
            PairTerm p;
            p.cre = cre;
            p.cim = cim;
            p.k1 = dk[0];
            p.k2 = dk[1];
            p.f1 = factor_id(dk[0], dm[0]);
            p.f2 = factor_id(dk[1], dm[1]);
            c->pairs.push_back(p);
            return;
        }
        ProdTerm pt;
        pt.cre = cre;
        pt.cim = cim;
        pt.nf = (int)dk.size();
        for (int f = 0; f < pt.nf; ++f) {
            pt.k[f] = dk[f];
            pt.fid[f] = factor_id(dk[f], dm[f]);
        }
        pt.use = use;
        if (use) {
            std::vector<double> tab((size_t)D * pd_nmax, 1.0);
            for (int k = 0; k < D; ++k)
                for (size_t i = 0; i < diag[k].size(); ++i) tab[(size_t)k * pd_nmax + i] = diag[k][i];
            pt.diag = (int)c->PD64.size();
            c->PD64.push_back(upload(tab, s));
        }
        c->chains.push_back(pt);
    };
    c->hermitian = !c->any_lattice;
    c->real_sym = !c->any_lattice;
    // in the DVR basis: real coefficients and real symmetric dense factors
    c->dvr_real_sym = true;
    for (const Term &t : c->terms) {
        c->dvr_real_sym = c->dvr_real_sym && t.coef_im == 0.0;
        for (const Factor &f : t.f) {
            if (f.kind == PPQ_FAC_DENSE_COMPLEX) c->dvr_real_sym = false;
            if (f.kind == PPQ_FAC_DENSE_REAL) {
                const int n = c->g.n[f.dim];
                for (int i = 0; i < n && c->dvr_real_sym; ++i)
                    for (int j = 0; j < i; ++j)
                        if (f.table[(size_t)i * n + j] != f.table[(size_t)j * n + i]) {
                            c->dvr_real_sym = false;
                            break;
                        }
            }
        }
    }
    if (!c->any_lattice) {
        for (int k = 0; k < D; ++k) {
            int n = c->g.n[k], b = c->nb[k];
            std::vector<double> T = dim_factor(c, k);
            std::vector<double> P((size_t)b * b, 0.0);
            std::vector<float> Pf((size_t)b * b, 0.0f);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    P[(size_t)i * b + j] = T[(size_t)i * n + j];
                    Pf[(size_t)i * b + j] = (float)T[(size_t)i * n + j];
                }
            c->T64[k] = upload(P, s);
            c->T32[k] = upload(Pf, s);
            if (n > NMAX_MASK) continue;  // long dimensions take no matrix-core tiles
            std::vector<float> P64((size_t)64 * 64, 0.0f);
            std::vector<double> D64((size_t)64 * 64, 0.0);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    P64[(size_t)i * 64 + j] = (float)T[(size_t)i * n + j];
                    D64[(size_t)i * 64 + j] = T[(size_t)i * n + j];
                }
            c->T32p[k] = upload(P64, s);
            c->T64p[k] = upload(D64, s);
        }
        // diagonal potential: one table per factor
        int nmax = 0;
        for (int k = 0; k < D; ++k) nmax = std::max(nmax, c->g.n[k]);
        std::vector<double> coef, tabs;
        std::vector<int> tab;
        for (const Term &t : c->terms) {
            if (is_product(c, t)) continue;
            std::vector<int> idx(D, -1);
            std::vector<std::vector<double>> per(D);
            for (const Factor &f : t.f) {
                std::vector<double> v = factor_values(c, f);
                if (per[f.dim].empty()) per[f.dim] = v;
                else
                    for (size_t i = 0; i < v.size(); ++i) per[f.dim][i] *= v[i];
            }
            for (int k = 0; k < D; ++k) {
                if (per[k].empty()) continue;
                per[k].resize(nmax, 0.0);
                // identical tables (q, q^2, ... on equal grids) are stored once
                int found = -1;
                for (size_t t0 = 0; t0 < tabs.size() / nmax && found < 0; ++t0)
                    if (std::equal(per[k].begin(), per[k].end(), tabs.begin() + t0 * nmax)) found = (int)t0;
                if (found < 0) {
                    found = (int)(tabs.size() / nmax);
                    tabs.insert(tabs.end(), per[k].begin(), per[k].end());
                }
                idx[k] = found;
            }
            coef.push_back(t.coef);
            tab.insert(tab.end(), idx.begin(), idx.end());
        }
        c->pot_nterm = (int)coef.size();
        c->pot_nmax = nmax;
        c->pot_ntab = (int)(tabs.size() / nmax);
        int maxf = 0;
        for (int t = 0; t < c->pot_nterm; ++t) {
            int nf = 0;
            for (int k = 0; k < D; ++k) nf += tab[(size_t)t * D + k] >= 0;
            maxf = std::max(maxf, nf);
        }
        if (c->pot_nterm > 256 || (int64_t)tabs.size() > 2048 || maxf > 4)
            throw std::invalid_argument("potential: at most 256 terms of at most 4 factors, 2048 distinct table values");
        if (coef.empty()) {
            coef.push_back(0.0);
            tab.assign(D, -1);
            tabs.assign(nmax, 0.0);
        }
        if (tabs.empty()) tabs.assign(nmax, 0.0);
        c->pot_coef = upload(coef, s);
        c->pot_tab = upload(tab, s);
        c->pot_tabs = upload(tabs, s);
        // derivative terms of the trainable parameters, same table layout
        {
            std::vector<double> dcoef, dtabsv;
            std::vector<int> dtab, dpar;
            for (size_t ti = 0; ti < c->dterms.size(); ++ti) {
                const Term &t = c->dterms[ti];
                std::vector<std::vector<double>> per(D);
                for (const Factor &f : t.f) {
                    std::vector<double> v = factor_values(c, f);
                    if (per[f.dim].empty()) per[f.dim] = v;
                    else
                        for (size_t i = 0; i < v.size(); ++i) per[f.dim][i] *= v[i];
                }
                std::vector<int> idx(D, -1);
                for (int k = 0; k < D; ++k) {
                    if (per[k].empty()) continue;
                    per[k].resize(nmax, 0.0);
                    int found = -1;
                    for (size_t t0 = 0; t0 < dtabsv.size() / nmax && found < 0; ++t0)
                        if (std::equal(per[k].begin(), per[k].end(), dtabsv.begin() + t0 * nmax)) found = (int)t0;
                    if (found < 0) {
                        found = (int)(dtabsv.size() / nmax);
                        dtabsv.insert(dtabsv.end(), per[k].begin(), per[k].end());
                    }
                    idx[k] = found;
                }
                dcoef.push_back(t.coef);
                dpar.push_back(c->dparam[ti]);
                dtab.insert(dtab.end(), idx.begin(), idx.end());
            }
            c->d_nterm = (int)dcoef.size();
            c->d_ntab = (int)(dtabsv.size() / nmax);
            if (c->d_nterm > 256 || (int64_t)dtabsv.size() > 2048)
                throw std::invalid_argument("derivative terms: at most 256 terms, 2048 distinct table values");
            if (dcoef.empty()) {
                dcoef.push_back(0.0);
                dpar.push_back(0);
                dtab.assign(D, -1);
            }
            if (dtabsv.empty()) dtabsv.assign(nmax, 0.0);
            dfree(c->d_dcoef);
            dfree(c->d_param);
            dfree(c->d_dtab);
            dfree(c->d_dtabs);
            c->d_dcoef = upload(dcoef, s);
            c->d_param = upload(dpar, s);
            c->d_dtab = upload(dtab, s);
            c->d_dtabs = upload(dtabsv, s);
        }
        // product terms: dense factors as matrices, diagonal ones as values.
        // The operator stays Hermitian with one Hermitian dense factor and a
        // real coefficient per term (the diagonal factors commute with it and
        // with the truncation); real symmetric when that factor is real.
        for (const Term &t : c->terms) {
            if (!is_product(c, t)) continue;
            std::vector<int> dk;
            std::vector<std::vector<cd>> dm;
            std::vector<std::vector<double>> diag(D);
            for (const Factor &f : t.f) {
                if (dense_kind(f.kind)) {
                    dk.push_back(f.dim);
                    dm.push_back(factor_matrix(c, f));
                } else {
                    std::vector<double> v = factor_values(c, f);
                    if (diag[f.dim].empty()) diag[f.dim] = v;
                    else
                        for (size_t i = 0; i < v.size(); ++i) diag[f.dim][i] *= v[i];
                }
            }
            std::vector<size_t> order(dk.size());
            for (size_t i = 0; i < order.size(); ++i) order[i] = i;
            std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return dk[a] < dk[b]; });
            std::vector<int> dks;
            std::vector<std::vector<cd>> dms;
            for (size_t i : order) {
                dks.push_back(dk[i]);
                dms.push_back(dm[i]);
            }
            bool herm = t.coef_im == 0.0 && dks.size() == 1, real = herm;
            if (herm) {
                const int n = c->g.n[dks[0]];
                const std::vector<cd> &h = dms[0];
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        herm = herm && h[(size_t)i * n + j] == std::conj(h[(size_t)j * n + i]);
                        real = real && h[(size_t)i * n + j].imag() == 0.0;
                    }
            }
            c->hermitian = c->hermitian && herm;
            c->real_sym = c->real_sym && herm && real;
            add_product(t.coef, t.coef_im, dks, dms, diag);
        }
    } else {
        std::vector<LatticeMaps> L(D);
        for (int k = 0; k < D; ++k) L[k] = lattice_maps(c, k);
        std::vector<std::vector<cd>> Hk(D);
        for (int k = 0; k < D; ++k) {
            int n = c->g.n[k];
            std::vector<double> T = dim_factor(c, k);
            std::vector<cd> h((size_t)n * n);
            for (size_t i = 0; i < h.size(); ++i) h[i] = T[i];
            Hk[k] = h;  // DVR-space sum, transformed at the end
        }
        for (const Term &t : c->terms) {
            // per dimension, the product of the term's factors on it (several
            // diagonal factors multiply; a dense factor is alone on its dimension)
            std::vector<std::vector<cd>> per(D);
            for (const Factor &f : t.f) {
                std::vector<cd> m = factor_matrix(c, f);
                per[f.dim] = per[f.dim].empty() ? m : matmul(per[f.dim], m, c->g.n[f.dim]);
            }
            std::vector<int> dims;
            for (int k = 0; k < D; ++k)
                if (!per[k].empty()) dims.push_back(k);
            const cd coef(t.coef, t.coef_im);
            if (dims.empty()) {
                // a constant term: coef times the identity, carried by dimension 0
                const int n0 = c->g.n[0];
                for (int i = 0; i < n0; ++i) Hk[0][(size_t)i * n0 + i] += coef;
            } else if (dims.size() == 1) {
                const int k = dims[0];
                for (size_t i = 0; i < Hk[k].size(); ++i) Hk[k][i] += coef * per[k][i];
            } else {
                std::vector<std::vector<cd>> dms;
                for (int k : dims) dms.push_back(similarity(L[k], per[k], c->g.n[k]));
                add_product(t.coef, t.coef_im, dims, dms, std::vector<std::vector<double>>(D));
            }
        }
        for (int k = 0; k < D; ++k) {
            int n = c->g.n[k];
            std::vector<cd> ht = similarity(L[k], Hk[k], n);
            pad_upload(ht, n, c->nb[k], &c->H64[k], &c->H32[k]);
            if (n <= NMAX_MASK) pad_upload(ht, n, 64, &c->H64p[k], &c->H32p[k]);
        }
    }
    // dense factors of the product terms, unpadded (nb x nb) and as 64 x 64
    // matrix-core tiles
    for (size_t i = 0; i < fmats.size(); ++i) {
        const int k = c->Fdim[i], n = c->g.n[k];
        double2 *d64;
        float2 *d32;
        pad_upload(fmats[i], n, c->nb[k], &d64, &d32);
        c->F64.push_back(d64);
        c->F32.push_back(d32);
        d64 = nullptr;
        d32 = nullptr;
        if (n <= NMAX_MASK) pad_upload(fmats[i], n, 64, &d64, &d32);
        c->F64p.push_back(d64);
        c->F32p.push_back(d32);
    }
    ck(hipStreamSynchronize(s), "operator upload");
    c->op_dirty = false;
    c->v_valid = false;  // a carried potential belongs to the previous operator
    c->v_partial = false;
}

void ensure_nf(ppq_ctx *c);

// Dimensions longer than a fiber-mask word take the long-fiber tables and pass.
bool is_long(const ppq_ctx *c, int k) { return c->g.n[k] > NMAX_MASK; }

bool any_long(const ppq_ctx *c)
{
    for (int k = 0; k < c->g.D; ++k)
        if (is_long(c, k)) return true;
    return false;
}

// ---- derived tables of the current set --------------------------------------
// Row-major fiber tables of dimension k (k < D - 1): pi_k, off_k, mask_k, info_k.
void build_row_major(ppq_ctx *c, int k)
{
    const int64_t n = c->nact;
    hipStream_t s = c->stream;
    const uint32_t *keys = c->keys[c->cur];
    const RotFrame fr = row_major_rot(c->g, k);
    fill_u64(c->bm, c->nwords + 2, 0ull, s);
    rot_set(keys, n, fr, c->bm, s);
    scan_popcount(c->bm, c->nwords, c->prefix, &c->small[MAXD], c->scan_tmp, s);
    // the per-point fiber info of dimensions other than the last is read only
    // by the point-parallel-everywhere layout and (as plain digits) by the
    // long-fiber pass of dimensions longer than a mask word
    const bool lng = is_long(c, k);
    rot_rank(keys, n, fr, c->bm, c->prefix, nullptr, c->pi[k], nullptr, c->flags, c->tmpmask,
             (c->hpsi_variant == 1 || lng) ? c->info[k] : nullptr, s);
    scan_u32(c->flags, n, c->fidx, &c->small[k], c->scan_tmp, s);
    fib_fill(c->flags, c->fidx, c->tmpmask, n, &c->small[k], c->off[k], lng ? nullptr : c->mask[k], s);
}

// Tables of the outer dimensions [0, split) in the inner-first frame (digit
// order: inner digits, then outer digits): P_R (frame rank -> position) and,
// per outer dimension, fibers in frame ranks (the last outer dimension is the
// frame's last digit, so its fibers are contiguous runs of the frame).
void build_inner_first(ppq_ctx *c)
{
    const int64_t n = c->nact;
    hipStream_t s = c->stream;
    const uint32_t *keys = c->keys[c->cur];
    const int sp = c->split;
    const uint32_t sin = c->g.stride[sp - 1];
    const uint32_t sout = c->g.total / sin;
    for (int k = sp - 1; k >= 0; --k) {
        const RotFrame fr{c->g.stride[k] / sin, (uint32_t)c->g.n[k], sin, sout};
        const bool frame = (k == sp - 1);
        fill_u64(c->bm, c->nwords + 2, 0ull, s);
        rot_set(keys, n, fr, c->bm, s);
        scan_popcount(c->bm, c->nwords, c->prefix, &c->small[MAXD], c->scan_tmp, s);
        rot_rank(keys, n, fr, c->bm, c->prefix, frame ? nullptr : c->inv_R, frame ? c->P_R : c->pi[k],
                 frame ? c->inv_R : nullptr, c->flags, c->tmpmask, nullptr, s);
        scan_u32(c->flags, n, c->fidx, &c->small[k], c->scan_tmp, s);
        fib_fill(c->flags, c->fidx, c->tmpmask, n, &c->small[k], c->off[k], c->mask[k], s);
        if (frame)
            make_chunks(keys, c->P_R, n, sin, true, c->blk_window,
                        c->hpsi_variant == 5 ? block2_cap_small(c->precision) : block_cap_small(c->precision), c->chunk[1],
                        c->big[1], c->small + 2 * MAXD + 2, s);
        chunk_fibers(c->chunk[1], n, c->blk_window, c->fidx, &c->small[k], c->fch[k], s);
    }
}

// Device memory the one-pass tables of all non-last dimensions need, or 0 if
// they do not apply (one dimension; concatenated ranks beyond 32 bits).
constexpr int64_t BATCH_BYTES_MAX = 8ll << 30;
// Words of the fiber-slot bitmaps of the non-last dimensions, concatenated
// (offsets in owoff[0..nd]): one bit per key with digit k removed.
int64_t occ_words(const ppq_ctx *c, int64_t *owoff)
{
    const int nd = c->g.D - 1;
    int64_t w = 0;
    for (int k = 0; k < nd; ++k) {
        if (owoff) owoff[k] = w;
        w += ((int64_t)c->g.total / c->g.n[k] + 63) / 64;
    }
    if (owoff) owoff[nd] = w;
    return w;
}

int64_t batched_bytes(const ppq_ctx *c)
{
    const int64_t nd = c->g.D - 1;
    // ranks of the concatenated bitmaps are offset by k |A| in 32 bits
    if (nd < 1 || (nd + 1) * c->cap >= (1ll << 32)) return 0;
    const int64_t words = (nd + 1) * c->nwords + 2, owords = occ_words(c, nullptr) + 2;
    return (words + owords) * 12 + scan_tmp_words(std::max(words, owords)) * 4;
}

bool ensure_batched(ppq_ctx *c)
{
    // the one-pass tables describe fibers by masks: dimensions of at most 64 points
    if (any_long(c)) return false;
    const int64_t bytes = batched_bytes(c);
    if (bytes == 0 || bytes > BATCH_BYTES_MAX) return false;
    if (c->bat_cap == c->cap) return true;
    const int64_t nd = c->g.D - 1, words = (nd + 1) * c->nwords + 2, owords = occ_words(c, nullptr) + 2;
    dfree(c->bmB);
    dfree(c->pfxB);
    dfree(c->scanB);
    dfree(c->cntB);
    dfree(c->occB);
    dfree(c->opfxB);
    c->bat_cap = 0;
    c->bmB = dalloc<uint64_t>(words);
    c->pfxB = dalloc<uint32_t>(words);
    c->occB = dalloc<uint64_t>(owords);
    c->opfxB = dalloc<uint32_t>(owords);
    c->scanB = dalloc<uint32_t>(scan_tmp_words(std::max(words, owords)));
    c->cntB = dalloc<uint32_t>(2 + MAXD);
    c->bat_cap = c->cap;
    return true;
}

// Plane tables of every pair (allocated on first use at the current capacity).
void ensure_planes(ppq_ctx *c)
{
    if (c->pl_cap == c->cap) return;
    const int64_t nc = c->cap;
    for (int i = 0; i < c->npl; ++i) {
        dfree(c->plP[i]);
        dfree(c->pltask[i]);
        dfree(c->pldig[i]);
        if (c->pl_a[i] + 2 < c->g.D) c->plP[i] = dalloc<uint32_t>(nc);
        c->pldig[i] = dalloc<uint16_t>(nc);
        c->pltask[i] = dalloc<uint32_t>(nc / PLANE_WINDOW + 2);
    }
    dfree(c->pl_poff);
    c->pl_poff = dalloc<uint32_t>(nc + 1);
    c->pl_cap = nc;
}

PairPass pair_pass_of(const ppq_ctx *c)
{
    const int D = c->g.D;
    PairPass pp;
    pp.keys = c->keys[c->cur];
    pp.pi_a = c->pi[D - 2];
    pp.tstart = c->pair_task;
    pp.ntask = (uint32_t)((c->nact + PAIR_WINDOW - 1) / PAIR_WINDOW);
    pp.n_a = c->g.n[D - 2];
    pp.n_b = c->g.n[D - 1];
    pp.lda = c->nb[D - 2];
    pp.ldb = c->nb[D - 1];
    return pp;
}

PlanePass plane_pass_of(const ppq_ctx *c, int i)
{
    PlanePass pp;
    const int a = c->pl_a[i];
    pp.P = c->plP[i];
    pp.dig = c->pldig[i];
    pp.tstart = c->pltask[i];
    pp.ntask = (uint32_t)((c->nact + PLANE_WINDOW - 1) / PLANE_WINDOW);
    pp.na = c->nb[a];
    pp.nb = c->nb[a + 1];
    return pp;
}

void build_derived(ppq_ctx *c)
{
    if (c->derived_valid) return;
    build_operator(c);
    c->plane_mode = false;
    {
        const int D = c->g.D;
        bool ok = c->hpsi_variant == 6 && !c->any_lattice && !any_long(c) && D >= 2 && c->pairs.empty() &&
                  c->chains.empty();
        for (int k = 0; k < D; ++k) ok = ok && c->nb[k] <= PLANE_NMAX;
        // a task holds whole planes: a plane must fit a task's span
        for (int a = D - 2; ok && a >= 0; a -= 2) ok = c->g.n[a] * c->g.n[a + 1] < PLANE_SPAN;
        c->plane_ok = ok;
        c->npl = ok ? D / 2 : 0;
        for (int i = 0; i < c->npl; ++i) c->pl_a[i] = D - 2 - 2 * i;
        // pair pass: the last two dimensions' factors in LDS, their digits in
        // 6 bits, a plane within a task's span; dimension 0 keeps its own
        // pass (it carries the fused <x|y>)
        c->pair_ok = c->hpsi_variant == 7 && !c->any_lattice && !any_long(c) && D >= 3 && c->pairs.empty() &&
                     c->chains.empty() && c->nb[D - 2] <= 32 && c->nb[D - 1] <= 32 &&
                     (uint32_t)(c->g.n[D - 2] * c->g.n[D - 1]) <= PAIR_NAB_MAX;
    }
    const int D = c->g.D;
    const int64_t n = c->nact;
    hipStream_t s = c->stream;
    const uint32_t *keys = c->keys[c->cur];
    const bool try_block = c->block_ok && (c->hpsi_variant == 4 || c->hpsi_variant == 5) && n > 0 &&
                           c->pairs.empty() && c->chains.empty();
    const uint32_t cap_s = c->hpsi_variant == 5 ? block2_cap_small(c->precision) : block_cap_small(c->precision);
    if (try_block) {
        fill_u32(c->small + 2 * MAXD, 4, 0u, s);
        make_chunks(keys, nullptr, n, c->g.stride[c->split - 1], false, c->blk_window, cap_s,
                    c->chunk[0], c->big[0], c->small + 2 * MAXD, s);
    }
    // last dimension: contiguous runs
    last_flags(keys, n, c->g.n[D - 1], c->flags, s);
    scan_u32(c->flags, n, c->fidx, &c->small[D - 1], c->scan_tmp, s);
    last_fill(keys, n, c->g.n[D - 1], c->flags, c->fidx, &c->small[D - 1], c->off[D - 1], c->mask[D - 1], s);
    last_info(keys, n, c->g.n[D - 1], c->info[D - 1], s);
    if (try_block) chunk_fibers(c->chunk[0], n, c->blk_window, c->fidx, &c->small[D - 1], c->fch[D - 1], s);
    // the per-point fiber info of dimensions other than the last is read only
    // by the point-parallel-everywhere layout, which takes the per-dimension path
    if (!try_block && c->hpsi_variant != 1 && n > 0 && D > 1 && ensure_batched(c)) {
        RotAll r{};
        TabPtrs t{};
        r.nd = D - 1;
        r.nwords = c->nwords;
        occ_words(c, r.owoff);
        for (int k = 0; k < D - 1; ++k) {
            r.sk[k] = c->g.stride[k];
            r.nk[k] = (uint32_t)c->g.n[k];
            t.pi[k] = c->pi[k];
            t.off[k] = c->off[k];
            t.mask[k] = c->mask[k];
        }
        fiber_tables_all(keys, n, r, c->bmB, c->pfxB, c->occB, c->opfxB, t, c->scanB, c->cntB, c->small, s);
    } else {
        for (int k = try_block ? c->split : 0; k < D - 1; ++k) {
            build_row_major(c, k);
            if (try_block) chunk_fibers(c->chunk[0], n, c->blk_window, c->fidx, &c->small[k], c->fch[k], s);
        }
    }
    if (try_block) build_inner_first(c);
    if (c->pair_ok && n > 0) {
        if (c->pair_cap != c->cap) {
            dfree(c->pair_task);
            c->pair_task = dalloc<uint32_t>(c->cap / PAIR_WINDOW + 2);
            c->pair_cap = c->cap;
        }
        pair_tasks(keys, n, (uint32_t)(c->g.n[D - 2] * c->g.n[D - 1]), c->pair_task, s);
    }
    if (c->plane_ok && n > 0) {
        ensure_planes(c);
        for (int i = 0; i < c->npl; ++i)
            plane_tables(keys, n, c->g, c->pl_a[i], c->bm, c->prefix, c->nwords, c->plP[i], c->pldig[i],
                         c->pltask[i], c->pl_poff, reinterpret_cast<uint32_t *>(c->tmpmask), c->flags, c->fidx,
                         c->scan_tmp, c->small + 3 * MAXD, s);
        c->plane_mode = true;
    }
    if (!c->any_lattice) {
        PotDesc pd{c->pot_nterm, D, c->pot_nmax, c->pot_coef, c->pot_tab, c->pot_tabs, c->pot_ntab};
        // flags is free once the fiber tables are built
        potential(keys, n, c->g, pd, c->V64, c->V32, c->v_partial ? c->flags : nullptr,
                  reinterpret_cast<unsigned *>(c->small + 2 * MAXD + 4), s);
        c->v_valid = true;
        c->v_partial = false;
    }
    // The fiber counts size the H*psi launches only: the host reads them when
    // the first product is issued (ensure_nf), so the work queued in between
    // (observables, the next step's normalisation) hides the round trip.
    ck(hipMemcpyAsync(c->h_small, c->small, sizeof(uint32_t) * (2 * MAXD + 4), hipMemcpyDeviceToHost, s), "nf");
    ck(hipEventRecord(c->ev_nf, s), "nf");
    c->nf_pending = true;
    c->nf_n = n;
    c->block_mode = false;
    if (try_block) {
        ensure_nf(c);
        const uint32_t *cnt = c->h_small + 2 * MAXD;
        for (int i = 0; i < 2; ++i) {
            c->nch[i] = (uint32_t)((n + c->blk_window - 1) / c->blk_window);
            c->nbig[i] = cnt[2 * i];
            c->maxch[i] = cnt[2 * i + 1];
        }
        const int npi_inner = D - c->split - 1, npi_outer = c->split - 1;
        c->block_mode = c->maxch[0] <= block_cap_max(c->precision, npi_inner) &&
                        c->maxch[1] <= block_cap_max(c->precision, npi_outer);
        if (std::getenv("PPQ_BLOCK_STATS"))
            std::fprintf(stderr, "[ppq] block chunks: inner nbig %u max %u, outer nbig %u max %u, mode %d\n",
                         c->nbig[0], c->maxch[0], c->nbig[1], c->maxch[1], (int)c->block_mode);
        if (!c->block_mode) {
            // a chunk too long for LDS: row-major tables for the outer dimensions
            for (int k = 0; k < c->split; ++k) build_row_major(c, k);
            ck(hipStreamSynchronize(s), "fibers");
        }
    }
    c->derived_valid = true;
}

BlockPass block_pass(const ppq_ctx *c, int which)
{
    BlockPass bp{};
    const int D = c->g.D, sp = c->split;
    const int k0 = which == 0 ? sp : 0, k1 = which == 0 ? D : sp;
    bp.ndim = k1 - k0;
    for (int i = 0; i < bp.ndim; ++i) {
        const int k = k0 + i;
        bp.dim[i] = k;
        bp.pi[i] = (k == k1 - 1) ? nullptr : c->pi[k];
        bp.off[i] = c->off[k];
        bp.mask[i] = c->mask[k];
        bp.fch[i] = c->fch[k];
        bp.nf[i] = c->nf[k];
        bp.nb[i] = c->nb[k];
    }
    bp.chunk = c->chunk[which];
    bp.nch = c->nch[which];
    bp.P = which == 0 ? nullptr : c->P_R;
    bp.big = c->big[which];
    bp.nbig = c->nbig[which];
    bp.cap_small = c->hpsi_variant == 5 ? block2_cap_small(c->precision) : block_cap_small(c->precision);
    bp.unroll = c->blk_unroll;
    bp.cap_big = bp.nbig ? (c->maxch[which] + 63u) / 64u * 64u : 0u;
    return bp;
}

LongPass long_pass_of(const ppq_ctx *c, int k)
{
    LongPass lp;
    lp.pi = (k == c->g.D - 1) ? nullptr : c->pi[k];
    lp.off = c->off[k];
    lp.dig = c->info[k];
    lp.nf = c->nf[k];
    lp.n = c->g.n[k];
    return lp;
}

FiberPass pass_of(const ppq_ctx *c, int k)
{
    FiberPass fp;
    fp.pi = (k == c->g.D - 1) ? nullptr : c->pi[k];
    fp.off = c->off[k];
    fp.mask = c->mask[k];
    fp.nf = c->nf[k];
    fp.nmax = c->nb[k];
    fp.stage = c->acc_stage;
    return fp;
}

// The partial buffer for a dot fused into the last pass of a product, or
// nullptr when the caller did not ask for one or the pass has more blocks
// than the buffer holds (dimension 0's fiber pass launches nf_0 / 256 blocks).
double2 *fused_dot_partial(const ppq_ctx *c)
{
    if (!c->dot_want || c->g.D < 2) return nullptr;
    const int64_t nb = (c->nf[0] + 255) / 256;
    return nb <= DOT_BLOCKS_MAX ? c->partial : nullptr;
}

// y = P H_1 P x: the one-dimensional factors and the diagonal potential
void apply_single(ppq_ctx *c, const void *xv, void *yv, const int *skip_if, int skip_j)
{
    ensure_nf(c);
    const int D = c->g.D;
    hipStream_t s = c->stream;
    if (c->nact == 0) return;
    if (!c->any_lattice && any_long(c)) {
        // dimensions longer than a mask word: the long-fiber pass; the others
        // one lane per fiber; the last dimension's pass writes y with V fused
        for (int k = D - 1; k >= 0; --k) {
            const bool first = k == D - 1;
            if (c->precision == PPQ_FP64) {
                const double2 *x = (const double2 *)xv;
                double2 *y = (double2 *)yv;
                if (is_long(c, k))
                    hpsi_long_real_f64(long_pass_of(c, k), c->T64[k], x, first ? c->V64 : nullptr, y, first, skip_if,
                                       skip_j, s);
                else
                    hpsi_real_f64(pass_of(c, k), c->T64[k], x, first ? c->V64 : nullptr, y, first, skip_if, skip_j, s);
            } else {
                const float2 *x = (const float2 *)xv;
                float2 *y = (float2 *)yv;
                if (is_long(c, k))
                    hpsi_long_real_f32(long_pass_of(c, k), c->T32[k], x, first ? c->V32 : nullptr, y, first, skip_if,
                                       skip_j, s);
                else
                    hpsi_real_f32(pass_of(c, k), c->T32[k], x, first ? c->V32 : nullptr, y, first, skip_if, skip_j, s);
            }
        }
        return;
    }
    if (!c->any_lattice) {
        if (c->plane_mode) {
            // pairs of dimensions; the last pair's pass writes y with V fused
            for (int i = 0; i < c->npl; ++i) {
                const PlanePass pp = plane_pass_of(c, i);
                const int a = c->pl_a[i];
                if (c->precision == PPQ_FP64)
                    hpsi_plane_f64(pp, c->T64[a], c->T64[a + 1], (const double2 *)xv, i == 0 ? c->V64 : nullptr,
                                   (double2 *)yv, i == 0, skip_if, skip_j, s);
                else
                    hpsi_plane_f32(pp, c->T32[a], c->T32[a + 1], (const float2 *)xv, i == 0 ? c->V32 : nullptr,
                                   (float2 *)yv, i == 0, skip_if, skip_j, s);
            }
            if (D % 2 == 1) {
                if (c->precision == PPQ_FP64)
                    hpsi_acc_f64(pass_of(c, 0), c->T64[0], (const double2 *)xv, (double2 *)yv, skip_if, skip_j, s);
                else
                    hpsi_acc_f32(pass_of(c, 0), c->T32[0], (const float2 *)xv, (float2 *)yv, skip_if, skip_j, s);
            }
            return;
        }
        if (c->block_mode) {
            // inner-first pass over the outer dimensions writes y, the row-major
            // pass over the inner dimensions adds to it with the potential fused
            const BlockPass outer = block_pass(c, 1), inner = block_pass(c, 0);
            if (c->precision == PPQ_FP64) {
                const double *To[BLOCK_MAXDIM], *Ti[BLOCK_MAXDIM];
                for (int i = 0; i < outer.ndim; ++i) To[i] = c->T64[outer.dim[i]];
                for (int i = 0; i < inner.ndim; ++i) Ti[i] = c->T64[inner.dim[i]];
                auto run = c->hpsi_variant == 5 ? hpsi_block2_f64 : hpsi_block_f64;
                run(outer, To, (const double2 *)xv, nullptr, (double2 *)yv, false, skip_if, skip_j, s);
                run(inner, Ti, (const double2 *)xv, c->V64, (double2 *)yv, true, skip_if, skip_j, s);
            } else {
                const float *To[BLOCK_MAXDIM], *Ti[BLOCK_MAXDIM];
                for (int i = 0; i < outer.ndim; ++i) To[i] = c->T32[outer.dim[i]];
                for (int i = 0; i < inner.ndim; ++i) Ti[i] = c->T32[inner.dim[i]];
                auto run = c->hpsi_variant == 5 ? hpsi_block2_f32 : hpsi_block_f32;
                run(outer, To, (const float2 *)xv, nullptr, (float2 *)yv, false, skip_if, skip_j, s);
                run(inner, Ti, (const float2 *)xv, c->V32, (float2 *)yv, true, skip_if, skip_j, s);
            }
            return;
        }
        if (c->hpsi_variant == 3) {
            const int64_t n = c->nact;
            if (c->precision == PPQ_FP64) {
                const double2 *x = (const double2 *)xv;
                double2 *y = (double2 *)yv;
                hpsi_pt_f64(nullptr, c->info[D - 1], n, c->nb[D - 1], c->T64[D - 1], x, c->V64, y, true, skip_if,
                            skip_j, s);
                for (int k = D - 2; k >= 0; --k) hpsi_acc_f64(pass_of(c, k), c->T64[k], x, y, skip_if, skip_j, s);
            } else {
                const float2 *x = (const float2 *)xv;
                float2 *y = (float2 *)yv;
                hpsi_pt_f32(nullptr, c->info[D - 1], n, c->nb[D - 1], c->T32[D - 1], x, c->V32, y, true, skip_if,
                            skip_j, s);
                for (int k = D - 2; k >= 0; --k) hpsi_acc_f32(pass_of(c, k), c->T32[k], x, y, skip_if, skip_j, s);
            }
            return;
        }
        if (c->hpsi_variant == 2 || c->hpsi_variant == 4 || c->hpsi_variant == 7) {
            // point-parallel last dimension and lane-per-fiber passes while
            // fibers are short (gather-bound, no dense tile forms); fibers
            // averaging more than 16 points form dense tiles: matrix cores.
            // Layout 7 takes the last two dimensions in one pass while both
            // have short fibers.
            const int64_t n = c->nact;
            auto longf = [&](int k) { return c->nf[k] > 0 && n > 16 * c->nf[k]; };
            const bool pair = c->pair_ok && !longf(D - 1) && !longf(D - 2);
            if (c->precision == PPQ_FP64) {
                const double2 *x = (const double2 *)xv;
                double2 *y = (double2 *)yv;
                if (pair)
                    hpsi_pair_f64(pair_pass_of(c), c->T64[D - 2], c->T64[D - 1], x, c->V64, y, skip_if, skip_j, s);
                else if (longf(D - 1))
                    hpsi_mfma_f64(pass_of(c, D - 1), c->T64p[D - 1], x, c->V64, y, true, skip_if, skip_j, s);
                else
                    hpsi_pt_f64(nullptr, c->info[D - 1], n, c->nb[D - 1], c->T64[D - 1], x, c->V64, y, true,
                                skip_if, skip_j, s);
                for (int k = pair ? D - 3 : D - 2; k >= 0; --k) {
                    if (longf(k)) hpsi_mfma_f64(pass_of(c, k), c->T64p[k], x, nullptr, y, false, skip_if, skip_j, s);
                    else if (c->nb[k] <= 32)
                        c->dot_nb = hpsi_acc_f64(pass_of(c, k), c->T64[k], x, y, skip_if, skip_j, s,
                                                 k == 0 ? fused_dot_partial(c) : nullptr);
                    else hpsi_real_f64(pass_of(c, k), c->T64[k], x, nullptr, y, false, skip_if, skip_j, s);
                }
            } else {
                const float2 *x = (const float2 *)xv;
                float2 *y = (float2 *)yv;
                // the last dimension's fibers are contiguous runs, which the
                // matrix-core pass gathers with coalesced loads: in FP32 it beats
                // the point-parallel pass even on short fibers (25.6 against
                // 41.2 us on the 6D snapshot; in FP64 the two are level)
                if (pair)
                    hpsi_pair_f32(pair_pass_of(c), c->T32[D - 2], c->T32[D - 1], x, c->V32, y, skip_if, skip_j, s);
                else
                    hpsi_mfma_f32(pass_of(c, D - 1), c->T32p[D - 1], x, c->V32, y, true, skip_if, skip_j, s);
                for (int k = pair ? D - 3 : D - 2; k >= 0; --k) {
                    if (longf(k)) hpsi_mfma_f32(pass_of(c, k), c->T32p[k], x, nullptr, y, false, skip_if, skip_j, s);
                    else if (c->nb[k] <= 32)
                        c->dot_nb = hpsi_acc_f32(pass_of(c, k), c->T32[k], x, y, skip_if, skip_j, s,
                                                 k == 0 ? fused_dot_partial(c) : nullptr);
                    else hpsi_real_f32(pass_of(c, k), c->T32[k], x, nullptr, y, false, skip_if, skip_j, s);
                }
            }
            return;
        }
        if (c->hpsi_variant == 1) {
            const int64_t n = c->nact;
            if (c->precision == PPQ_FP64) {
                const double2 *x = (const double2 *)xv;
                double2 *y = (double2 *)yv;
                hpsi_pt_f64(nullptr, c->info[D - 1], n, c->nb[D - 1], c->T64[D - 1], x, c->V64, y, true, skip_if,
                            skip_j, s);
                for (int k = D - 2; k >= 0; --k)
                    hpsi_pt_f64(c->pi[k], c->info[k], n, c->nb[k], c->T64[k], x, nullptr, y, false, skip_if, skip_j, s);
            } else {
                const float2 *x = (const float2 *)xv;
                float2 *y = (float2 *)yv;
                hpsi_pt_f32(nullptr, c->info[D - 1], n, c->nb[D - 1], c->T32[D - 1], x, c->V32, y, true, skip_if,
                            skip_j, s);
                for (int k = D - 2; k >= 0; --k)
                    hpsi_pt_f32(c->pi[k], c->info[k], n, c->nb[k], c->T32[k], x, nullptr, y, false, skip_if, skip_j, s);
            }
            return;
        }
        if (c->precision == PPQ_FP64) {
            const double2 *x = (const double2 *)xv;
            double2 *y = (double2 *)yv;
            hpsi_real_f64(pass_of(c, D - 1), c->T64[D - 1], x, c->V64, y, true, skip_if, skip_j, s);
            for (int k = D - 2; k >= 0; --k)
                hpsi_real_f64(pass_of(c, k), c->T64[k], x, nullptr, y, false, skip_if, skip_j, s);
        } else {
            const float2 *x = (const float2 *)xv;
            float2 *y = (float2 *)yv;
            hpsi_real_f32(pass_of(c, D - 1), c->T32[D - 1], x, c->V32, y, true, skip_if, skip_j, s);
            for (int k = D - 2; k >= 0; --k)
                hpsi_real_f32(pass_of(c, k), c->T32[k], x, nullptr, y, false, skip_if, skip_j, s);
        }
        return;
    }
    // lattice: the single-dimension factors (complex; product terms follow)
    const bool mf = c->hpsi_variant != 3;
    if (c->precision == PPQ_FP64) {
        const double2 *x = (const double2 *)xv;
        double2 *y = (double2 *)yv;
        CInput in{};
        in.nin = 1;
        in.x[0] = x;
        in.c[0] = make_double2(1.0, 0.0);
        for (int k = D - 1; k >= 0; --k) {
            if (is_long(c, k)) hpsi_long_cplx_f64(long_pass_of(c, k), c->H64[k], in, y, k < D - 1, skip_if, skip_j, s);
            else if (mf) hpsi_cmfma_f64(pass_of(c, k), c->H64p[k], in, y, k < D - 1, skip_if, skip_j, s);
            else hpsi_cplx_f64(pass_of(c, k), c->H64[k], in, y, k < D - 1, nullptr, skip_if, skip_j, s);
        }
    } else {
        const float2 *x = (const float2 *)xv;
        float2 *y = (float2 *)yv;
        CInput32 in{};
        in.nin = 1;
        in.x[0] = x;
        in.c[0] = make_float2(1.f, 0.f);
        for (int k = D - 1; k >= 0; --k) {
            if (is_long(c, k)) hpsi_long_cplx_f32(long_pass_of(c, k), c->H32[k], in, y, k < D - 1, skip_if, skip_j, s);
            else if (mf) hpsi_cmfma_f32(pass_of(c, k), c->H32p[k], in, y, k < D - 1, skip_if, skip_j, s);
            else hpsi_cplx_f32(pass_of(c, k), c->H32[k], in, y, k < D - 1, nullptr, skip_if, skip_j, s);
        }
    }
}

// y += the product terms (Sec. II.B.2; each intermediate truncated to the
// set).  Two-factor terms without diagonal factors are grouped by their inner
// factor: it is applied once per distinct factor, and each outer factor acts
// on a weighted sum (the coefficients) of up to four inner results.  Other
// terms go one at a time: their diagonal factors scale the input (diagonal
// matrices commute with the truncation), then the dense factors act from the
// highest dimension down, the last one adding coef times its result to y.
template <class C, class CIn, class W>
void apply_products_t(ppq_ctx *c, const C *x, C *y, const int *skip_if, int skip_j,
                      const std::vector<const void *> &Fn, const std::vector<const void *> &Fp,
                      W (*mk)(double, double))
{
    hipStream_t s = c->stream;
    const bool mf = c->hpsi_variant != 3;
    auto cpass = [&](int k, int f, const CIn &in, C *out, bool acc) {
        if constexpr (std::is_same<C, double2>::value) {
            if (is_long(c, k))
                hpsi_long_cplx_f64(long_pass_of(c, k), (const double2 *)Fn[f], in, out, acc, skip_if, skip_j, s);
            else if (mf) hpsi_cmfma_f64(pass_of(c, k), (const double2 *)Fp[f], in, out, acc, skip_if, skip_j, s);
            else hpsi_cplx_f64(pass_of(c, k), (const double2 *)Fn[f], in, out, acc, nullptr, skip_if, skip_j, s);
        } else {
            if (is_long(c, k))
                hpsi_long_cplx_f32(long_pass_of(c, k), (const float2 *)Fn[f], in, out, acc, skip_if, skip_j, s);
            else if (mf) hpsi_cmfma_f32(pass_of(c, k), (const float2 *)Fp[f], in, out, acc, skip_if, skip_j, s);
            else hpsi_cplx_f32(pass_of(c, k), (const float2 *)Fn[f], in, out, acc, nullptr, skip_if, skip_j, s);
        }
    };
    C **z = (C **)c->zbuf.data();
    std::vector<int> inner_ids, outer_ids;
    for (const PairTerm &p : c->pairs) {
        if (std::find(inner_ids.begin(), inner_ids.end(), p.f2) == inner_ids.end()) inner_ids.push_back(p.f2);
        if (std::find(outer_ids.begin(), outer_ids.end(), p.f1) == outer_ids.end()) outer_ids.push_back(p.f1);
    }
    CIn one{};
    one.nin = 1;
    one.x[0] = x;
    one.c[0] = mk(1.0, 0.0);
    for (size_t i = 0; i < inner_ids.size(); ++i) cpass(c->Fdim[inner_ids[i]], inner_ids[i], one, z[i], false);
    for (int f : outer_ids) {
        CIn acc{};
        for (const PairTerm &p : c->pairs) {
            if (p.f1 != f) continue;
            const int zi = (int)(std::find(inner_ids.begin(), inner_ids.end(), p.f2) - inner_ids.begin());
            acc.x[acc.nin] = z[zi];
            acc.c[acc.nin] = mk(p.cre, p.cim);
            if (++acc.nin == 4) {
                cpass(c->Fdim[f], f, acc, y, true);
                acc.nin = 0;
            }
        }
        if (acc.nin) cpass(c->Fdim[f], f, acc, y, true);
    }
    for (const ProdTerm &t : c->chains) {
        const C *src = x;
        if (t.use || t.nf == 0) {
            // the diagonal factors (none: a constant term): straight into y for a
            // term without dense ones
            const bool alone = t.nf == 0;
            diag_scale<C>(c->keys[c->cur], x, c->nact, c->g, t.use ? c->PD64[t.diag] : nullptr, c->pd_nmax, t.use,
                          alone ? make_double2(t.cre, t.cim) : make_double2(1.0, 0.0), alone ? y : z[0], alone,
                          skip_if, skip_j, s);
            if (alone) continue;
            src = z[0];
        }
        for (int f = t.nf - 1; f >= 0; --f) {
            CIn in{};
            in.nin = 1;
            in.x[0] = src;
            if (f == 0) {
                in.c[0] = mk(t.cre, t.cim);
                cpass(t.k[f], t.fid[f], in, y, true);
            } else {
                in.c[0] = mk(1.0, 0.0);
                C *dst = (src == z[1]) ? z[2] : z[1];
                cpass(t.k[f], t.fid[f], in, dst, false);
                src = dst;
            }
        }
    }
}

inline double2 mk64(double r, double i) { return make_double2(r, i); }
inline float2 mk32(double r, double i) { return make_float2((float)r, (float)i); }

void apply_products(ppq_ctx *c, const void *xv, void *yv, const int *skip_if, int skip_j)
{
    if (c->pairs.empty() && c->chains.empty()) return;
    ensure_zbuf(c);
    if (c->precision == PPQ_FP64) {
        std::vector<const void *> Fn(c->F64.begin(), c->F64.end()), Fp(c->F64p.begin(), c->F64p.end());
        apply_products_t<double2, CInput, double2>(c, (const double2 *)xv, (double2 *)yv, skip_if, skip_j, Fn, Fp,
                                                   mk64);
    } else {
        std::vector<const void *> Fn(c->F32.begin(), c->F32.end()), Fp(c->F32p.begin(), c->F32p.end());
        apply_products_t<float2, CInput32, float2>(c, (const float2 *)xv, (float2 *)yv, skip_if, skip_j, Fn, Fp,
                                                   mk32);
    }
}

// y = P H P x on the current set (device vectors of the context precision)
void apply_launches(ppq_ctx *c, const void *xv, void *yv, const int *skip_if, int skip_j)
{
    // a fused <x|y> needs the single-factor passes to write y last
    const bool want = c->dot_want;
    c->dot_want = want && c->pairs.empty() && c->chains.empty();
    c->dot_nb = 0;
    apply_single(c, xv, yv, skip_if, skip_j);
    c->dot_want = want;
    if (c->nact > 0) apply_products(c, xv, yv, skip_if, skip_j);
}

// Launch errors (a configuration the device refuses) surface here rather than
// as a silently skipped pass.
void apply_internal(ppq_ctx *c, const void *xv, void *yv, const int *skip_if, int skip_j)
{
    apply_launches(c, xv, yv, skip_if, skip_j);
    ck(hipGetLastError(), "H*psi launch");
}

// Host copy of the fiber counts of the last table build (waits for its copy).
void ensure_nf(ppq_ctx *c)
{
    if (!c->nf_pending) return;
    ck(hipEventSynchronize(c->ev_nf), "fibers");
    for (int k = 0; k < c->g.D; ++k) c->nf[k] = c->nf_n > 0 ? c->h_small[k] : 0;
    c->nf_pending = false;
}

// ---- opt-in phase timing ------------------------------------------------------
constexpr size_t TIMING_EVENTS = 4096;
constexpr int PHASE_NONE = -1;

// Adds the intervals between the recorded events to their phases and keeps
// the last event as the start of the next interval.  The last event must have
// completed.
void timing_flush(ppq_ctx *c)
{
    for (size_t i = 0; i + 1 < c->tcount; ++i) {
        float ms = 0.0f;
        ck(hipEventElapsedTime(&ms, c->tev[i], c->tev[i + 1]), "elapsed");
        if (c->tlabel[i] >= 0) c->tms[c->tlabel[i]] += ms;
    }
    if (c->tcount > 1) {
        std::swap(c->tev[0], c->tev[c->tcount - 1]);
        c->tlabel[0] = c->tlabel[c->tcount - 1];
        c->tcount = 1;
    }
}

// Records a phase boundary: `phase` starts now (PHASE_NONE: nothing runs).
void mark(ppq_ctx *c, int phase)
{
    if (!c->timing) return;
    if (c->tcount == c->tev.size()) {
        if (c->tev.size() < TIMING_EVENTS) {
            hipEvent_t e;
            ck(hipEventCreate(&e), "event");
            c->tev.push_back(e);
            c->tlabel.push_back(PHASE_NONE);
        } else {
            ck(hipEventSynchronize(c->tev[c->tcount - 1]), "event sync");
            timing_flush(c);
        }
    }
    ck(hipEventRecord(c->tev[c->tcount], c->stream), "event");
    c->tlabel[c->tcount] = phase;
    ++c->tcount;
}

// Lanczos/Arnoldi basis of `src` (FP64 master vector on the current set) in
// Vb with the small matrix and norm in ks; m H-applications, CGS2.
// tol > 0: the order is chosen per step by the error estimate (the adjoint's
// recorded steps use the full order)
template <class C>
// fix_last: leave every basis vector corrected in memory (the adjoint reads the
// basis); otherwise a full-order step's last vector stays provisional and
// lanczos_coef folds its correction into the coefficients.
void krylov_build(ppq_ctx *c, const double2 *src, C *Vb, KState *ks, int m, double dt = 0.0, double tol = 0.0,
                  bool fix_last = true)
{
    hipStream_t s = c->stream;
    const int64_t n = c->nact;
    const int64_t ld = c->cap;
    C *w = (C *)c->wk;
    const int *meff = &ks->meff;
    const bool herm = c->hermitian;
    norm0<C>(src, n, c->partial, c->counter, ks, m, dt, tol, s);
    normalise_from_master<C>(src, n, ks, Vb, s);
    if (herm) {
        // Lanczos with the second Gram-Schmidt pass of each vector applied in
        // the next step's sweep: H is applied to the provisional q_j in slot
        // j, <q_j|H q_j> comes from the product's last pass where it can,
        // and one sweep per step corrects v_j and forms q_{j+1}
        for (int j = 0; j < m; ++j) {
            C *qj = Vb + (int64_t)j * ld;
            mark(c, PPQ_PHASE_HPSI);
            c->dot_want = true;
            apply_internal(c, qj, w, meff, j);
            c->dot_want = false;
            const int fused = c->dot_nb;
            mark(c, PPQ_PHASE_KRYLOV);
            if (fused) finalize_dot(c->partial, fused, ks, j, m, RED_DELAY, s);
            else cgs_dots<C>(qj, ld, 1, w, n, c->partial, c->counter, ks, j, m, j, s, RED_DELAY);
            if (j == m - 1) {
                if (j > 0 && fix_last) lanczos_fix<C>(Vb, ld, n, ks, j, s);
                break;
            }
            lanczos_sweep<C>(Vb, ld, w, n, c->partial, c->counter, ks, j, m, s);
        }
        return;
    }
    // Arnoldi with the same delayed second pass: H is applied to the
    // provisional q_j, the first-pass column of H v_j follows from the Arnoldi
    // relation, and one sweep corrects v_j and forms q_{j+1}
    for (int j = 0; j < m; ++j) {
        const C *qj = Vb + (int64_t)j * ld;
        mark(c, PPQ_PHASE_HPSI);
        apply_internal(c, qj, w, meff, j);
        mark(c, PPQ_PHASE_KRYLOV);
        const bool last = (j == m - 1);
        arnoldi_step<C>(Vb, ld, w, n, c->partial, c->counter, ks, j, m, last, s);
        if (last && j > 0 && fix_last) lanczos_fix<C>(Vb, ld, n, ks, j, s);
    }
}

template <class C>
void step_impl(ppq_ctx *c, double dt, int m, double tol)
{
    mark(c, PPQ_PHASE_KRYLOV);
    C *Vb = (C *)c->Vk;
    krylov_build<C>(c, c->psi[c->cur], Vb, c->ks, m, dt, tol, false);
    krylov_expv(c->ks, m, dt, c->hermitian ? 1 : 0, c->stream);
    lanczos_coef(c->ks, m, c->stream);
    lincomb<C>(Vb, c->cap, c->psi[c->cur], c->nact, c->ks, c->psi_tmp, c->stream);
    std::swap(c->psi[c->cur], c->psi_tmp);
}

// Outcome of one step: the Krylov order (-1: only on the device, in ks) and
// the number of substeps.
struct StepInfo {
    int meff = -1;
    int nsub = 1;
};

void step_any(ppq_ctx *c, double dt, int m)
{
    if (c->precision == PPQ_FP64) step_impl<double2>(c, dt, m, c->krylov_tol);
    else step_impl<float2>(c, dt, m, c->krylov_tol);
}

// One step of length dt on the current set (tables built).  Without step
// control one SIL step.  With control (max_substeps > 1 and a Krylov
// tolerance) s substeps of dt/s, s from the previous step; each substep's
// order goes to sub_meff and the host reads them once per attempt: an order
// of m means the tolerance was not met below m, and the step is redone from
// its saved start with 2s substeps.  alpha0_dst (device, may be NULL)
// receives alpha_0 of the first substep: the energy of the state at the start.
StepInfo advance(ppq_ctx *c, double dt, int m, double *alpha0_dst)
{
    StepInfo info;
    hipStream_t s = c->stream;
    if (c->nact == 0) return info;
    if (c->max_substeps <= 1 || !(c->krylov_tol > 0.0)) {
        step_any(c, dt, m);
        if (alpha0_dst) copy_alpha0(c->ks, alpha0_dst, s);
        return info;
    }
    if (c->sub_cap < c->max_substeps) {
        dfree(c->sub_meff);
        if (c->h_sub_meff) (void)hipHostFree(c->h_sub_meff);
        c->h_sub_meff = nullptr;
        c->sub_meff = dalloc<double>(c->max_substeps);
        ck(hipHostMalloc((void **)&c->h_sub_meff, sizeof(double) * c->max_substeps, hipHostMallocDefault),
           "pinned");
        c->sub_cap = c->max_substeps;
    }
    if (c->psi_save_cap < c->cap) {
        dfree(c->psi_save);
        c->psi_save = dalloc<double2>(c->cap);
        c->psi_save_cap = c->cap;
    }
    ck(hipMemcpyAsync(c->psi_save, c->psi[c->cur], c->nact * sizeof(double2), hipMemcpyDeviceToDevice, s), "save");
    int sub = std::min(std::max(c->nsub, 1), c->max_substeps);
    for (;;) {
        const double h = dt / (double)sub;
        for (int j = 0; j < sub; ++j) {
            step_any(c, h, m);
            if (j == 0 && alpha0_dst) copy_alpha0(c->ks, alpha0_dst, s);
            copy_meff(c->ks, c->sub_meff + j, s);
        }
        ck(hipMemcpyAsync(c->h_sub_meff, c->sub_meff, sizeof(double) * sub, hipMemcpyDeviceToHost, s), "orders");
        ck(hipStreamSynchronize(s), "orders");
        int mo = 0;
        bool ok = true;
        for (int j = 0; j < sub; ++j) {
            const int me = (int)c->h_sub_meff[j];
            mo = std::max(mo, me);
            ok = ok && me < m;
        }
        if (ok) {
            info.meff = mo;
            info.nsub = sub;
            c->nsub = (mo <= m / 2 && sub > 1) ? sub / 2 : sub;
            return info;
        }
        ck(hipMemcpyAsync(c->psi[c->cur], c->psi_save, c->nact * sizeof(double2), hipMemcpyDeviceToDevice, s),
           "restore");
        sub *= 2;
        if (sub > c->max_substeps) {
            ck(hipStreamSynchronize(s), "restore");
            throw std::runtime_error("a step does not meet the Krylov tolerance within the allowed substeps");
        }
    }
}

StepInfo do_step(ppq_ctx *c, double dt, int m)
{
    mark(c, PPQ_PHASE_TABLES);
    build_derived(c);
    ensure_krylov(c, m);
    return advance(c, dt, m, nullptr);
}

// adaption; returns false (state untouched) only on allocation failure
void do_prune(ppq_ctx *c, double eps, int64_t *nabove_out)
{
    mark(c, PPQ_PHASE_ADAPT);
    hipStream_t s = c->stream;
    const int64_t n_old = c->nact;
    double eps2 = eps * eps;
    fill_u64((uint64_t *)c->count, 1, 0ull, s);
    // the +-1 stencil on DVR axes word by word while the grid's bitmap is not
    // much larger than the set (every word is visited); else per function
    const bool words = c->g.pairs == 0 && !c->any_lattice && c->dilate_mode != 1 &&
                       (c->dilate_mode == 2 || c->nwords <= 4 * n_old + 4096);
    if (words) {
        if (c->kbm_words != c->nwords) {
            dfree(c->kbm);
            c->kbm = dalloc<uint64_t>(c->nwords);
            c->kbm_words = c->nwords;
        }
        dilate_words(c->keys[c->cur], c->psi[c->cur], n_old, c->g, eps2, c->kbm, c->bm, c->nwords, c->count,
                     c->flags, s);
    } else {
        fill_u64(c->bm, c->nwords + 2, 0ull, s);
        dilate(c->keys[c->cur], c->psi[c->cur], n_old, c->g, eps2, c->bm, c->count, c->flags, s);
    }
    if (c->rel_excl > 0.0)
        keep_all_if_few_dropped(c->keys[c->cur], n_old, c->bm, c->rel_excl, c->flags, c->count + 1, s);
    scan_popcount(c->bm, c->nwords, c->prefix, &c->small[MAXD], c->scan_tmp, s);
    ck(hipMemcpyAsync(c->h_small + MAXD, c->small + MAXD, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "count");
    ck(hipMemcpyAsync(c->h_count, c->count, sizeof(unsigned long long), hipMemcpyDeviceToHost, s), "count");
    ck(hipStreamSynchronize(s), "prune count");
    int64_t n_new = c->h_small[MAXD];
    if (nabove_out) *nabove_out = (int64_t)*c->h_count;
    if (n_new > c->cap) ensure_capacity(c, n_new);  // keeps keys/psi of the current set
    int nxt = 1 - c->cur;
    compact(c->bm, c->prefix, c->nwords, c->keys[nxt], s);
    fill_zero_bytes(c->psi[nxt], n_new * (int64_t)sizeof(double2), s);
    remap(c->keys[c->cur], c->psi[c->cur], n_old, c->bm, c->prefix, c->psi[nxt], s);
    // The diagonal potential of the functions that stay is carried over;
    // only the added ones are evaluated again (NaN marks them).
    const bool carry = c->v_valid && !c->any_lattice;
    if (carry) {
        if (c->precision == PPQ_FP64) {
            std::swap(c->V64, c->Vt64);
            fill_u64(reinterpret_cast<uint64_t *>(c->V64), n_new, 0x7ff8000000000000ull, s);
            remap_values(c->keys[c->cur], c->Vt64, n_old, c->bm, c->prefix, c->V64, s);
        } else {
            std::swap(c->V32, c->Vt32);
            fill_u32(reinterpret_cast<uint32_t *>(c->V32), n_new, 0x7fc00000u, s);
            remap_values(c->keys[c->cur], c->Vt32, n_old, c->bm, c->prefix, c->V32, s);
        }
    }
    c->cur = nxt;
    c->nact = n_new;
    c->derived_valid = false;
    c->v_valid = false;
    c->v_partial = carry;
}

void set_record_host(ppq_ctx *c, int64_t r, double t, int krylov, int nsub = 1)
{
    // t, |A|, the Krylov dimension and the substeps are host-known: kernel
    // arguments, no sync
    set_record(c->rec + r * PPQ_OBS_N, t, (double)c->nact, (double)krylov, (double)nsub, c->stream);
}

void ensure_records(ppq_ctx *c, int64_t nrec)
{
    if (c->rec_cap >= nrec) return;
    dfree(c->rec);
    c->rec = dalloc<double>(nrec * PPQ_OBS_N);
    c->rec_cap = nrec;
    fill_zero_bytes(c->rec, nrec * PPQ_OBS_N * (int64_t)sizeof(double), c->stream);
}

// observables of the current set into record r (energy left to the caller)
void observe_into(ppq_ctx *c, int64_t r, double eps)
{
    double *rec = c->rec + r * PPQ_OBS_N;
    // without a reference packet the tables are zero and C(t) reads 0
    const double2 *bra = c->bra_tabs;
    obs_partial(c->keys[c->cur], c->psi[c->cur], c->nact, c->g, bra, c->tab_nmax, eps * eps, c->partial,
                c->stream);
    obs_final(c->partial, RED_BLOCKS, rec, c->stream);
}

// energy of the current state by one explicit application (FP64 master in, precision of the context)
void energy_into(ppq_ctx *c, int64_t r)
{
    double *rec = c->rec + r * PPQ_OBS_N;
    if (c->nact == 0) return;
    ensure_krylov(c, std::max(c->kv_m, 1));
    if (c->precision == PPQ_FP64) {
        apply_internal(c, c->psi[c->cur], c->wk, nullptr, 0);
        dot_partial(c->psi[c->cur], (const double2 *)c->wk, c->nact, c->partial, c->stream);
    } else {
        // FP32 form: H acts on the FP32 copy; the inner product is accumulated in FP64
        float2 *x32 = (float2 *)c->Vk;
        KState *ks = c->ks;
        norm0<float2>(c->psi[c->cur], c->nact, c->partial, c->counter, ks, 1, 0.0, 0.0, c->stream);
        normalise_from_master<float2>(c->psi[c->cur], c->nact, ks, x32, c->stream);
        apply_internal(c, x32, c->wk, nullptr, 0);
        cgs_dots<float2>(x32, c->cap, 1, (const float2 *)c->wk, c->nact, c->partial, c->counter, ks, 0, 1, 0,
                         c->stream);
        copy_alpha0(ks, rec + PPQ_OBS_ENERGY, c->stream);
        return;
    }
    energy_from_dot(c->partial, RED_BLOCKS, rec, c->stream);
}

// Packet tables: init (coefficients of psi0 per dimension), bra (its dual,
// giving C(t)) and, for DVR dimensions, the derivatives of the normalised 1D
// factors with respect to the centre and the momentum.
// Packet tables of a product Gaussian: the initial-state tables (and their
// centre/momentum derivatives, for the adjoint) and the C(t) reference.  With
// reference_only, only the C(t) reference is replaced.
void set_packet_tables(ppq_ctx *c, const double *centre, const double *momentum, const double *width,
                       bool reference_only = false)
{
    const int D = c->g.D;
    int nmax = 0;
    for (int k = 0; k < D; ++k) nmax = std::max(nmax, c->g.n[k]);
    std::vector<double2> it((size_t)D * nmax, make_double2(0.0, 0.0)), bt = it;
    std::vector<double2> dt((size_t)2 * D * nmax, make_double2(0.0, 0.0));
    for (int k = 0; k < D; ++k) {
        int n = c->g.n[k];
        std::vector<double> q = dim_points(c, k);
        std::vector<cd> gk(n), dc(n), dp(n);
        double nrm2 = 0.0;
        for (int i = 0; i < n; ++i) {
            double d = q[i] - centre[k];
            gk[i] = std::exp(-d * d / (2.0 * width[k] * width[k])) * std::exp(cd(0.0, momentum[k] * d));
            dc[i] = gk[i] * cd(d / (width[k] * width[k]), -momentum[k]);
            dp[i] = gk[i] * cd(0.0, d);
            nrm2 += std::norm(gk[i]);
        }
        const double nrm = std::sqrt(nrm2);
        double rc = 0.0, rp = 0.0;  // Re <g|dg>
        for (int i = 0; i < n; ++i) {
            rc += (std::conj(gk[i]) * dc[i]).real();
            rp += (std::conj(gk[i]) * dp[i]).real();
        }
        for (int i = 0; i < n; ++i) {
            cd dci = dc[i] / nrm - gk[i] * (rc / (nrm * nrm2));
            cd dpi = dp[i] / nrm - gk[i] * (rp / (nrm * nrm2));
            dt[(size_t)(2 * k) * nmax + i] = make_double2(dci.real(), dci.imag());
            dt[(size_t)(2 * k + 1) * nmax + i] = make_double2(dpi.real(), dpi.imag());
        }
        for (int i = 0; i < n; ++i) gk[i] /= nrm;
        std::vector<cd> a = gk, b = gk;
        if (c->lattice[k]) {
            LatticeMaps L = lattice_maps(c, k);
            a.assign(n, cd(0.0, 0.0));
            b.assign(n, cd(0.0, 0.0));
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    a[i] += L.Gadj[(size_t)i * n + j] * gk[j];
                    b[i] += L.Ginv[(size_t)i * n + j] * gk[j];
                }
        }
        for (int i = 0; i < n; ++i) {
            it[(size_t)k * nmax + i] = make_double2(a[i].real(), a[i].imag());
            bt[(size_t)k * nmax + i] = make_double2(b[i].real(), b[i].imag());
        }
        if (!reference_only) {
            c->pk_centre[k] = centre[k];
            c->pk_momentum[k] = momentum[k];
            c->pk_width[k] = width[k];
        }
    }
    ck(hipStreamSynchronize(c->stream), "sync");
    dfree(c->bra_tabs);
    c->bra_tabs = upload(bt, c->stream);
    if (!reference_only) {
        dfree(c->init_tabs);
        dfree(c->dtabs);
        c->init_tabs = upload(it, c->stream);
        c->dtabs = upload(dt, c->stream);
    }
    c->tab_nmax = nmax;
    c->has_ref = true;
}

bool keys_valid(const ppq_ctx *c, int64_t n, const uint64_t *keys)
{
    for (int64_t i = 0; i < n; ++i) {
        if (keys[i] >= c->g.total) return false;
        if (i && keys[i] <= keys[i - 1]) return false;
    }
    return true;
}


// ---- adjoint helpers -----------------------------------------------------------
void set_current_set(ppq_ctx *c, const uint32_t *keys_dev, int64_t n)
{
    if (n > c->cap) throw std::runtime_error("set larger than the reserved capacity");
    if (n) ck(hipMemcpyAsync(c->keys[c->cur], keys_dev, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream),
              "set keys");
    c->nact = n;
    c->has_state = true;
    c->nsub = 1;
    c->derived_valid = false;
    c->v_valid = false;
    c->v_partial = false;
}

// restriction of the current state to a recorded set (one frozen adaption)
void frozen_remap(ppq_ctx *c, const uint32_t *next_keys, int64_t n_next)
{
    hipStream_t s = c->stream;
    if (n_next > c->cap) throw std::runtime_error("set larger than the reserved capacity");
    fill_u64(c->bm, c->nwords + 2, 0ull, s);
    mark_keys_wave(next_keys, n_next, c->bm, s);
    scan_popcount(c->bm, c->nwords, c->prefix, &c->small[MAXD], c->scan_tmp, s);
    const int nxt = 1 - c->cur;
    if (n_next)
        ck(hipMemcpyAsync(c->keys[nxt], next_keys, n_next * sizeof(uint32_t), hipMemcpyDeviceToDevice, s), "keys");
    fill_zero_bytes(c->psi[nxt], n_next * (int64_t)sizeof(double2), s);
    remap(c->keys[c->cur], c->psi[c->cur], c->nact, c->bm, c->prefix, c->psi[nxt], s);
    c->cur = nxt;
    c->nact = n_next;
    c->derived_valid = false;
    c->v_valid = false;
    c->v_partial = false;
}

void record_append(ppq_ctx *c)
{
    int64_t used = c->rec_off.empty() ? 0 : c->rec_off.back() + c->rec_n.back();
    if (used + c->nact > c->rec_keys_cap) {
        int64_t nc = std::max<int64_t>(2 * c->rec_keys_cap, used + c->nact + (1 << 20));
        uint32_t *nb = dalloc<uint32_t>(nc);
        if (used) ck(hipMemcpyAsync(nb, c->rec_keys, used * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream),
                     "record grow");
        ck(hipStreamSynchronize(c->stream), "record grow");
        dfree(c->rec_keys);
        c->rec_keys = nb;
        c->rec_keys_cap = nc;
    }
    if (c->nact)
        ck(hipMemcpyAsync(c->rec_keys + used, c->keys[c->cur], c->nact * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                          c->stream),
           "record keys");
    c->rec_off.push_back(used);
    c->rec_n.push_back(c->nact);
}

void clear_record(ppq_ctx *c)
{
    for (auto &p : c->ckpt) dfree(p);
    c->ckpt.clear();
    c->rec_off.clear();
    c->rec_n.clear();
    c->rec_sub.clear();
    c->recorded = false;
}

void checkpoint_now(ppq_ctx *c)
{
    double2 *b = dalloc<double2>(std::max<int64_t>(c->nact, 1));
    if (c->nact)
        ck(hipMemcpyAsync(b, c->psi[c->cur], c->nact * sizeof(double2), hipMemcpyDeviceToDevice, c->stream), "ckpt");
    c->ckpt.push_back(b);
}

// C = <psi0|psi> on the current set (the autocorrelation through the bra tables)
double2 overlap_with_packet(ppq_ctx *c)
{
    ensure_records(c, 1);
    obs_partial(c->keys[c->cur], c->psi[c->cur], c->nact, c->g, c->bra_tabs, c->tab_nmax, 0.0, c->partial, c->stream);
    obs_final(c->partial, RED_BLOCKS, c->rec, c->stream);
    double r[PPQ_OBS_N];
    ck(hipMemcpyAsync(r, c->rec, sizeof(r), hipMemcpyDeviceToHost, c->stream), "C");
    ck(hipStreamSynchronize(c->stream), "C");
    return make_double2(r[PPQ_OBS_ACF_RE], r[PPQ_OBS_ACF_IM]);
}

// K: the most states one recomputed segment holds (its steps' substeps)
void ensure_adjoint_buffers(ppq_ctx *c, int m, int K)
{
    const size_t es = c->precision == PPQ_FP64 ? sizeof(double2) : sizeof(float2);
    if (!c->Wk || c->wk_cap != c->cap) {
        dfree(c->Wk);
        void *p = nullptr;
        if (hipMalloc(&p, es * (size_t)(m + 1) * (size_t)c->cap) != hipSuccess) throw std::bad_alloc();
        c->Wk = p;
        c->wk_cap = c->cap;
    }
    if (!c->ks_b) {
        void *p = nullptr;
        ck(hipMalloc(&p, sizeof(KState)), "kstate");
        c->ks_b = (KState *)p;
        c->Qd = dalloc<double2>(MAXM * MAXM);
        c->dC = dalloc<double2>(ADJ_MAXP + 2 * MAXD);
    }
    if (c->adj_cap != c->cap || !c->lam) {
        dfree(c->lam);
        dfree(c->mu);
        c->lam = dalloc<double2>(c->cap);
        c->mu = dalloc<double2>(c->cap);
        c->adj_cap = c->cap;
    }
    if (c->seg_cap < (int64_t)K * c->cap) {
        dfree(c->seg);
        c->seg = dalloc<double2>((int64_t)K * c->cap);
        c->seg_cap = (int64_t)K * c->cap;
    }
}

template <class C>
void adjoint_backward(ppq_ctx *c, double2 C_N)
{
    hipStream_t s = c->stream;
    const int N = c->rec_steps, K = c->rec_every, m = c->rec_m;
    const double dt = c->rec_dt;
    const int D = c->g.D;
    DerivDesc dd{c->nparam, c->d_nterm, c->pot_nmax, c->d_param, c->d_dcoef, c->d_dtab, c->d_dtabs, c->d_ntab};
    fill_zero_bytes(c->dC, (ADJ_MAXP + 2 * MAXD) * (int64_t)sizeof(double2), s);
    auto keys_of = [&](int st) { return c->rec_keys + c->rec_off[st]; };
    // lambda_N = psi0 restricted to A_N
    product_values(keys_of(N), c->rec_n[N], c->g, c->bra_tabs, c->tab_nmax, c->lam, s);
    const int nseg = (N + K - 1) / K;
    std::vector<int> slot(N + 1, 0);  // first segment state of each step
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int a = sg * K, e = std::min(a + K, N);
        set_current_set(c, keys_of(a), c->rec_n[a]);
        if (c->rec_n[a])
            ck(hipMemcpyAsync(c->psi[c->cur], c->ckpt[sg], c->rec_n[a] * sizeof(double2), hipMemcpyDeviceToDevice, s),
               "restore");
        // recompute the segment, keeping the state at the start of every substep
        int idx = 0;
        for (int st = a; st < e; ++st) {
            const int ns = c->rec_sub[st];
            const double h = dt / (double)ns;
            slot[st] = idx;
            build_derived(c);
            for (int j = 0; j < ns; ++j, ++idx) {
                if (c->nact)
                    ck(hipMemcpyAsync(c->seg + (int64_t)idx * c->cap, c->psi[c->cur], c->nact * sizeof(double2),
                                      hipMemcpyDeviceToDevice, s),
                       "segment");
                if (c->nact) step_impl<C>(c, h, m, c->rec_tol);
            }
            frozen_remap(c, keys_of(st + 1), c->rec_n[st + 1]);
        }
        if (e == N) {
            // <d psi0 / d theta | psi_N>
            adj_packet(keys_of(N), c->rec_n[N], c->g, c->init_tabs, c->dtabs, c->tab_nmax, c->psi[c->cur], 1,
                       c->partial, s);
            adj_accumulate(c->partial, 2 * D, make_double2(1.0, 0.0), c->dC + c->nparam, s);
        } else {
            // the recomputation must reproduce the stored checkpoint bit for bit
            unsigned long long nd =
                count_diff(c->psi[c->cur], c->ckpt[sg + 1], c->nact, c->count, c->h_count, s);
            if (nd) throw std::runtime_error("recomputed segment differs from the stored checkpoint");
        }
        for (int st = e - 1; st >= a; --st) {
            const int64_t nn = c->rec_n[st];
            // mu = R^dagger lambda_{st+1}
            fill_u64(c->bm, c->nwords + 2, 0ull, s);
            mark_keys_wave(keys_of(st + 1), c->rec_n[st + 1], c->bm, s);
            scan_popcount(c->bm, c->nwords, c->prefix, &c->small[MAXD], c->scan_tmp, s);
            gather_remap(keys_of(st), nn, c->bm, c->prefix, c->lam, c->mu, s);
            set_current_set(c, keys_of(st), nn);
            build_derived(c);
            if (nn == 0) continue;
            // the substeps of the step, last first: each is a step map exp(-i H h)
            // on the same set, so the recursion runs through them as through steps
            const int ns = c->rec_sub[st];
            const double h = dt / (double)ns;
            for (int j = ns - 1; j >= 0; --j) {
                const double2 *psi_n = c->seg + (int64_t)(slot[st] + j) * c->cap;
                krylov_build<C>(c, psi_n, (C *)c->Vk, c->ks, m);
                krylov_build<C>(c, c->mu, (C *)c->Wk, c->ks_b, m);
                adj_q(c->ks, c->ks_b, h, c->Qd, s);
                if (c->nparam > 0) {
                    adj_reduce<C>((const C *)c->Vk, (const C *)c->Wk, c->cap, psi_n, c->mu, c->ks, c->ks_b, c->Qd,
                                  keys_of(st), nn, c->g, dd, c->partial, s);
                    adj_accumulate(c->partial, c->nparam, make_double2(0.0, -h), c->dC, s);
                }
                // lambda = exp(+i H h) mu
                krylov_expv(c->ks_b, m, -h, 1, s);
                lincomb<C>((const C *)c->Wk, c->cap, c->mu, nn, c->ks_b, c->lam, s);
                if (j > 0) std::swap(c->mu, c->lam);
            }
        }
    }
    // <lambda_0 | d psi0 / d theta>
    adj_packet(keys_of(0), c->rec_n[0], c->g, c->init_tabs, c->dtabs, c->tab_nmax, c->lam, 0, c->partial, s);
    adj_accumulate(c->partial, 2 * D, make_double2(1.0, 0.0), c->dC + c->nparam, s);
    ck(hipStreamSynchronize(s), "adjoint");
    (void)C_N;
}

// the most states a recomputed segment holds
int max_segment_states(const ppq_ctx *c)
{
    int best = 1;
    for (int a = 0; a < c->rec_steps; a += c->rec_every) {
        int t = 0;
        for (int st = a; st < std::min(a + c->rec_every, c->rec_steps); ++st) t += c->rec_sub[st];
        best = std::max(best, t);
    }
    return best;
}

}  // namespace

// =============================================================================
extern "C" {

// ---- device scratch of the no-allocation entry point ------------------------
// ppq_expect_q_noalloc keeps its grid-point table, its per-block partial sums
// and its result in this file-scope array instead of context buffers, so it
// allocates nothing.  Each device that runs the library holds its own copy
// until the process ends.  In host code the array's name is only a host-side
// stand-in: every host use goes through the device address taken once per
// device with hipGetSymbolAddress (scratch_setup, called by ppq_create with
// the device current).
constexpr size_t NOALLOC_SCRATCH_BYTES = 256u * 1024u;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES];
hipError_t g_scratch_err[NOALLOC_MAX_DEVICES];
bool g_scratch_done[NOALLOC_MAX_DEVICES];

// Address of this device's scratch (the current device must be `device`).
void scratch_setup(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_done[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
    g_scratch_done[device] = true;
}

void *scratch_of(int device, hipError_t *err)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    *err = g_scratch_done[device] ? g_scratch_err[device] : hipErrorNotInitialized;
    return g_scratch_ptr[device];
}

// Bytes of scratch ppq_expect_q_noalloc needs: the D x nmax grid-point table
// and the D results (rounded up to 256 bytes), then the (1 + MAXD) x
// RED_BLOCKS complex partial sums of the fixed-shape reduction.
size_t expect_q_scratch_bytes(int D, int nmax, size_t *off_out, size_t *off_partial)
{
    const size_t tab = sizeof(double) * (size_t)D * (size_t)nmax;
    *off_out = tab;
    const size_t head = (tab + sizeof(double) * MAXD + 255u) / 256u * 256u;
    *off_partial = head;
    return head + sizeof(double2) * (size_t)(1 + MAXD) * RED_BLOCKS;
}
}  // namespace

int ppq_create(ppq_ctx **out, int device, void *hip_stream, int precision)
{
    if (!out) return PPQ_E_ARG;
    *out = nullptr;
    if (precision != PPQ_FP64 && precision != PPQ_FP32) return PPQ_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PPQ_E_ARG;
    ppq_ctx *c = new (std::nothrow) ppq_ctx();
    if (!c) return PPQ_E_OOM;
    c->device = device;
    c->precision = precision;
    if (const char *v = std::getenv("PPQ_HPSI")) {
        const int h = std::atoi(v);
        if (h >= 0 && h <= 7) c->hpsi_variant = h;  // other values keep the default layout
    }
    if (const char *v = std::getenv("PPQ_BLOCK_UNROLL")) c->blk_unroll = std::atoi(v) != 0;
    if (const char *v = std::getenv("PPQ_ACC_STAGE")) c->acc_stage = std::atoi(v) != 0;
    if (const char *v = std::getenv("PPQ_DILATE")) {
        const int d = std::atoi(v);
        if (d >= 0 && d <= 2) c->dilate_mode = d;
    }
    if (const char *v = std::getenv("PPQ_BLOCK_WINDOW")) {
        const long w = std::atol(v);
        if (w >= (long)BLOCK_WINDOW && w <= (1l << 20)) c->blk_window = (uint32_t)w;
    }
    try {
        ck(hipSetDevice(device), "hipSetDevice");
        scratch_setup(device);  // once per device; a failure is reported by the entry point that needs it
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
        } else {
            ck(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "stream");
            c->own_stream = true;
        }
        void *p = nullptr;
        ck(hipMalloc(&p, sizeof(KState)), "kstate");
        c->ks = (KState *)p;
        c->partial = dalloc<double2>((int64_t)RED_BLOCKS * PSTRIDE_H);
        c->counter = dalloc<unsigned>(4);
        ck(hipMemset(c->counter, 0, 4 * sizeof(unsigned)), "counter");
        c->small = dalloc<uint32_t>(4 * MAXD);  // fiber counts, scan totals, block counters
        c->count = dalloc<unsigned long long>(2);
        ck(hipHostMalloc((void **)&c->h_small, sizeof(uint32_t) * 4 * MAXD, hipHostMallocDefault), "pinned");
        ck(hipHostMalloc((void **)&c->h_count, sizeof(unsigned long long) * 2, hipHostMallocDefault), "pinned");
        ck(hipEventCreateWithFlags(&c->ev_nf, hipEventDisableTiming), "event");
        ck(hipEventCreate(&c->ev0), "event");
        ck(hipEventCreate(&c->ev1), "event");
    } catch (const HipError &e) {
        ppq_destroy(c);
        return PPQ_E_HIP;
    } catch (const std::bad_alloc &) {
        ppq_destroy(c);
        return PPQ_E_OOM;
    }
    *out = c;
    return PPQ_OK;
}

void ppq_destroy(ppq_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_state_buffers(c);
    free_krylov(c);
    free_operator(c);
    dfree(c->bm);
    dfree(c->prefix);
    dfree(c->kbm);
    dfree(c->ks);
    dfree(c->partial);
    dfree(c->counter);
    for (auto &p : c->full) dfree(p);
    dfree(c->sub_meff);
    if (c->h_sub_meff) (void)hipHostFree(c->h_sub_meff);
    dfree(c->small);
    dfree(c->count);
    dfree(c->init_tabs);
    dfree(c->bra_tabs);
    dfree(c->qtab);
    dfree(c->acf2);
    dfree(c->rec);
    clear_record(c);
    dfree(c->rec_keys);
    dfree(c->seg);
    dfree(c->Wk);
    dfree(c->ks_b);
    dfree(c->Qd);
    dfree(c->dC);
    dfree(c->lam);
    dfree(c->mu);
    dfree(c->dtabs);
    dfree(c->d_param);
    dfree(c->d_dcoef);
    dfree(c->d_dtab);
    dfree(c->d_dtabs);
    if (c->h_small) (void)hipHostFree(c->h_small);
    if (c->h_count) (void)hipHostFree(c->h_count);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev_nf) (void)hipEventDestroy(c->ev_nf);
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *ppq_last_error(const ppq_ctx *c) { return c ? c->err.c_str() : "null context"; }

#define PPQ_GUARD(c)                                                       \
    if (!(c)) return PPQ_E_ARG;                                            \
    if ((c)->poisoned) return fail((c), PPQ_E_HIP, "context poisoned");    \
    (void)hipSetDevice((c)->device);

#define PPQ_TRY(c, ...)                                                    \
    try {                                                                  \
        __VA_ARGS__                                                        \
    } catch (const HipError &e) {                                          \
        return hip_fail((c), e);                                           \
    } catch (const std::bad_alloc &) {                                     \
        return fail((c), PPQ_E_OOM, "device allocation failed");           \
    } catch (const std::invalid_argument &e) {                             \
        return fail((c), PPQ_E_UNSUPPORTED, e.what());                     \
    } catch (const std::exception &e) {                                    \
        return fail((c), PPQ_E_NUMERIC, e.what());                         \
    }

int ppq_set_grid(ppq_ctx *c, int D, const int32_t *n, const double *lo, const double *hi, double mass)
{
    PPQ_GUARD(c)
    if (D < 1 || D > MAXD || !n || !lo || !hi || !(mass > 0.0)) return fail(c, PPQ_E_ARG, "bad grid arguments");
    uint64_t total = 1;
    for (int k = 0; k < D; ++k) {
        if (n[k] < 2 || n[k] > NMAX_FIBER) return fail(c, PPQ_E_ARG, "n[k] must be in [2, 256]");
        if (!(hi[k] > lo[k])) return fail(c, PPQ_E_ARG, "box must have hi > lo");
        total *= (uint64_t)n[k];
        if (total >= (1ull << 32)) return fail(c, PPQ_E_CAPACITY, "grid size must be < 2^32");
    }
    PPQ_TRY(c, {
        ck(hipStreamSynchronize(c->stream), "sync");
        free_state_buffers(c);
        free_krylov(c);
        free_operator(c);
        dfree(c->bm);
        dfree(c->prefix);
        dfree(c->kbm);
        c->kbm_words = 0;
        c->terms.clear();
        c->has_state = false;
        c->nact = 0;
        c->has_ref = false;
        GridDesc g{};
        g.D = D;
        uint32_t st = 1;
        for (int k = D - 1; k >= 0; --k) {
            g.n[k] = n[k];
            g.stride[k] = st;
            st *= (uint32_t)n[k];
        }
        g.total = (uint32_t)total;
        c->g = g;
        c->any_lattice = false;
        for (int k = 0; k < D; ++k) {
            c->lo[k] = lo[k];
            c->hi[k] = hi[k];
            c->nb[k] = bucket(n[k]);
            c->lattice[k] = false;
            c->weylets[k] = false;
            c->fgh[k] = false;
            c->factor[k].clear();
        }
        c->mass = mass;
        c->split = D / 2;
        c->block_ok = D >= 2 && D - c->split <= BLOCK_MAXDIM;
        for (int k = 0; k < D; ++k) c->block_ok = c->block_ok && c->nb[k] <= BLOCK_MAXNB;
        int nmax = 0;
        for (int k = 0; k < D; ++k) nmax = std::max(nmax, n[k]);
        std::vector<double2> zt((size_t)D * nmax, make_double2(0.0, 0.0));
        dfree(c->init_tabs);
        dfree(c->bra_tabs);
        c->init_tabs = upload(zt, c->stream);
        c->bra_tabs = upload(zt, c->stream);
        c->tab_nmax = nmax;
        c->nwords = (int64_t)((total + 63) / 64);
        c->bm = dalloc<uint64_t>(c->nwords + 2);
        c->prefix = dalloc<uint32_t>(c->nwords + 2);
        c->has_grid = true;
        c->op_dirty = true;
    })
    return PPQ_OK;
}

int ppq_get_grid(const ppq_ctx *c, int k, double *q)
{
    if (!c || !q) return PPQ_E_ARG;
    if (!c->has_grid || k < 0 || k >= c->g.D) return PPQ_E_ARG;
    std::vector<double> v = dim_points(c, k);
    std::memcpy(q, v.data(), v.size() * sizeof(double));
    return PPQ_OK;
}

static int set_lattice_kind(ppq_ctx *c, int k, int ns, int nl, bool weylets)
{
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    if (k < 0 || k >= c->g.D || ns < 1 || nl < 1 || ns * nl != c->g.n[k])
        return fail(c, PPQ_E_ARG, "lattice shape must satisfy n_s * n_l == n[k]");
    if (!c->terms.empty()) return fail(c, PPQ_E_STATE, "set lattices before adding terms");
    if (weylets) {
        // fails early on a lattice whose symmetrized Gaussians are linearly dependent
        PPQ_TRY(c, { (void)weylet_projection(dim_points(c, k), dim_weight(c, k), c->lo[k], c->hi[k], ns, nl); })
    }
    c->g.lat_s[k] = ns;
    c->g.lat_l[k] = nl;
    c->lattice[k] = true;
    c->weylets[k] = weylets;
    c->any_lattice = true;
    c->block_ok = false;
    c->op_dirty = true;
    c->derived_valid = false;
    c->v_valid = false;
    c->v_partial = false;
    return PPQ_OK;
}

int ppq_set_lattice(ppq_ctx *c, int k, int ns, int nl)
{
    PPQ_GUARD(c)
    return set_lattice_kind(c, k, ns, nl, false);
}

int ppq_set_weylets(ppq_ctx *c, int k, int nx, int np)
{
    PPQ_GUARD(c)
    return set_lattice_kind(c, k, nx, np, true);
}

namespace {
// Parses the factors of one term (layout of ppq_add_term); dense kinds only
// when allow_dense.  Returns PPQ_OK or the error (message set).
int parse_term(ppq_ctx *c, double cre, double cim, int nfac, const int32_t *dims, const int32_t *kinds,
               const double *params, const double *data, bool allow_dense, Term &t)
{
    if (nfac < 0 || nfac > 4 * MAXD || (nfac > 0 && (!dims || !kinds))) return fail(c, PPQ_E_ARG, "bad factors");
    if (!std::isfinite(cre) || !std::isfinite(cim)) return fail(c, PPQ_E_NUMERIC, "non-finite coefficient");
    t.coef = cre;
    t.coef_im = cim;
    int64_t toff = 0;
    unsigned dense_dims = 0, all_dims = 0;
    for (int f = 0; f < nfac; ++f) {
        Factor fa;
        fa.dim = dims[f];
        fa.kind = kinds[f];
        if (fa.dim < 0 || fa.dim >= c->g.D) return fail(c, PPQ_E_ARG, "factor dimension out of range");
        fa.p0 = params ? params[2 * f] : 0.0;
        fa.p1 = params ? params[2 * f + 1] : 0.0;
        const int64_t n = c->g.n[fa.dim];
        if (fa.kind == PPQ_FAC_POWER) {
            if (fa.p0 < 0 || fa.p0 > 16 || fa.p0 != std::floor(fa.p0))
                return fail(c, PPQ_E_ARG, "power must be an integer in [0, 16]");
        } else if (fa.kind == PPQ_FAC_MORSE || fa.kind == PPQ_FAC_MORSE_DA) {
        } else if (fa.kind == PPQ_FAC_TABLE || (allow_dense && dense_kind(fa.kind))) {
            const int64_t len = fa.kind == PPQ_FAC_TABLE ? n : fa.kind == PPQ_FAC_DENSE_REAL ? n * n : 2 * n * n;
            if (!data) return fail(c, PPQ_E_ARG, "table or dense factor without data");
            fa.table.assign(data + toff, data + toff + len);
            toff += len;
            for (double v : fa.table)
                if (!std::isfinite(v)) return fail(c, PPQ_E_NUMERIC, "non-finite factor entry");
            if (dense_kind(fa.kind)) {
                if ((dense_dims | all_dims) >> fa.dim & 1u)
                    return fail(c, PPQ_E_ARG, "a dense factor must be the only factor on its dimension");
                dense_dims |= 1u << fa.dim;
            }
        } else {
            return fail(c, PPQ_E_ARG, "unknown factor kind");
        }
        if (!dense_kind(fa.kind) && (dense_dims >> fa.dim & 1u))
            return fail(c, PPQ_E_ARG, "a dense factor must be the only factor on its dimension");
        all_dims |= 1u << fa.dim;
        t.f.push_back(fa);
    }
    return PPQ_OK;
}

void operator_changed(ppq_ctx *c)
{
    c->op_dirty = true;
    c->derived_valid = false;
    c->v_valid = false;
    c->v_partial = false;
}
}  // namespace

int ppq_add_potential_term(ppq_ctx *c, double coef, int nfac, const int32_t *dims, const int32_t *kinds,
                           const double *params, const double *tables)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    Term t;
    const int r = parse_term(c, coef, 0.0, nfac, dims, kinds, params, tables, false, t);
    if (r != PPQ_OK) return r;
    c->terms.push_back(t);
    operator_changed(c);
    return PPQ_OK;
}

int ppq_add_term(ppq_ctx *c, double c_re, double c_im, int nfac, const int32_t *dims, const int32_t *kinds,
                 const double *params, const double *data)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    Term t;
    const int r = parse_term(c, c_re, c_im, nfac, dims, kinds, params, data, true, t);
    if (r != PPQ_OK) return r;
    c->terms.push_back(t);
    operator_changed(c);
    return PPQ_OK;
}

int ppq_set_factor(ppq_ctx *c, int k, const double *h)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    if (k < 0 || k >= c->g.D) return fail(c, PPQ_E_ARG, "dimension out of range");
    const int n = c->g.n[k];
    if (h) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double v = h[(size_t)i * n + j];
                if (!std::isfinite(v)) return fail(c, PPQ_E_NUMERIC, "non-finite factor entry");
                if (v != h[(size_t)j * n + i]) return fail(c, PPQ_E_ARG, "factor must be symmetric");
            }
        c->factor[k].assign(h, h + (size_t)n * n);
    } else {
        c->factor[k].clear();
    }
    c->op_dirty = true;
    c->derived_valid = false;
    c->v_valid = false;
    c->v_partial = false;
    return PPQ_OK;
}

int ppq_set_stencil(ppq_ctx *c, int stencil)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    if (stencil < 1 || stencil > 3) return fail(c, PPQ_E_ARG, "stencil must be 1, 2 or 3");
    c->g.pairs = stencil - 1;
    return PPQ_OK;
}

int ppq_set_fgh(ppq_ctx *c, int k)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    if (k < 0 || k >= c->g.D) return fail(c, PPQ_E_ARG, "dimension out of range");
    if (c->g.n[k] % 2 == 0) return fail(c, PPQ_E_ARG, "the Fourier grid needs an odd number of points");
    if (c->lattice[k]) return fail(c, PPQ_E_STATE, "set Fourier grids before lattices");
    if (!c->terms.empty()) return fail(c, PPQ_E_STATE, "set Fourier grids before adding terms");
    c->fgh[k] = true;
    c->op_dirty = true;
    c->derived_valid = false;
    c->v_valid = false;
    c->v_partial = false;
    return PPQ_OK;
}

int ppq_clear_potential(ppq_ctx *c)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    c->terms.clear();
    c->op_dirty = true;
    c->derived_valid = false;
    c->v_valid = false;
    c->v_partial = false;
    return PPQ_OK;
}

int ppq_reserve(ppq_ctx *c, int64_t max_active)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    if (max_active < 1 || max_active > (int64_t)c->g.total) return fail(c, PPQ_E_ARG, "bad capacity");
    PPQ_TRY(c, { ensure_capacity(c, max_active); })
    return PPQ_OK;
}

int ppq_init_gaussian(ppq_ctx *c, const double *centre, const double *momentum, const double *width, double eps,
                      int64_t *n_active)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    if (!centre || !momentum || !width || !(eps >= 0.0)) return fail(c, PPQ_E_ARG, "bad packet");
    for (int k = 0; k < c->g.D; ++k)
        if (!(width[k] > 0.0)) return fail(c, PPQ_E_ARG, "width must be positive");
    PPQ_TRY(c, {
        set_packet_tables(c, centre, momentum, width);
        const int nmax = c->tab_nmax;
        // flag the full grid, dilate, compact
        hipStream_t s = c->stream;
        if (!c->scan_tmp) ensure_capacity(c, 1024);
        fill_u64(c->bm, c->nwords + 2, 0ull, s);
        fill_u64((uint64_t *)c->count, 1, 0ull, s);
        init_flag(c->g, c->init_tabs, nmax, eps * eps, c->bm, c->count, s);
        scan_popcount(c->bm, c->nwords, c->prefix, &c->small[MAXD], c->scan_tmp, s);
        ck(hipMemcpyAsync(c->h_small + MAXD, c->small + MAXD, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "n");
        ck(hipStreamSynchronize(s), "init count");
        int64_t n0 = c->h_small[MAXD];
        c->has_state = false;
        c->nact = 0;
        ensure_capacity(c, std::max<int64_t>(n0, 1));
        compact(c->bm, c->prefix, c->nwords, c->keys[c->cur], s);
        product_values(c->keys[c->cur], n0, c->g, c->init_tabs, nmax, c->psi[c->cur], s);
        c->nact = n0;
        c->has_state = true;
        c->nsub = 1;
        c->derived_valid = false;
        c->v_valid = false;
        c->v_partial = false;
        ck(hipStreamSynchronize(s), "init");
        if (n_active) *n_active = n0;
    })
    return PPQ_OK;
}

int ppq_set_reference(ppq_ctx *c, const double *centre, const double *momentum, const double *width)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    if (!centre || !momentum || !width) return fail(c, PPQ_E_ARG, "bad packet");
    for (int k = 0; k < c->g.D; ++k)
        if (!(width[k] > 0.0) || !std::isfinite(centre[k]) || !std::isfinite(momentum[k]))
            return fail(c, PPQ_E_ARG, "bad packet");
    PPQ_TRY(c, {
        set_packet_tables(c, centre, momentum, width, true);
        ck(hipStreamSynchronize(c->stream), "reference");
    })
    return PPQ_OK;
}

int ppq_set_state(ppq_ctx *c, int64_t count, const uint64_t *keys, const double *coeff)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    if (count < 0 || (count > 0 && (!keys || !coeff))) return fail(c, PPQ_E_ARG, "bad state arguments");
    if (!keys_valid(c, count, keys)) return fail(c, PPQ_E_ARG, "keys must be strictly ascending and in range");
    for (int64_t i = 0; i < 2 * count; ++i)
        if (!std::isfinite(coeff[i])) return fail(c, PPQ_E_NUMERIC, "non-finite coefficient");
    PPQ_TRY(c, {
        c->has_state = false;
        c->nact = 0;
        ensure_capacity(c, std::max<int64_t>(count, 1));
        std::vector<uint32_t> k32(count);
        for (int64_t i = 0; i < count; ++i) k32[i] = (uint32_t)keys[i];
        if (count) {
            ck(hipMemcpyAsync(c->keys[c->cur], k32.data(), count * sizeof(uint32_t), hipMemcpyHostToDevice,
                              c->stream),
               "set keys");
            ck(hipMemcpyAsync(c->psi[c->cur], coeff, count * sizeof(double2), hipMemcpyHostToDevice, c->stream),
               "set psi");
        }
        ck(hipStreamSynchronize(c->stream), "set state");
        c->nact = count;
        c->has_state = true;
        c->nsub = 1;
        c->derived_valid = false;
        c->v_valid = false;
        c->v_partial = false;
    })
    return PPQ_OK;
}

int ppq_active_count(const ppq_ctx *c, int64_t *count)
{
    if (!c || !count) return PPQ_E_ARG;
    if (!c->has_state) return PPQ_E_STATE;
    *count = c->nact;
    return PPQ_OK;
}

int ppq_get_state(ppq_ctx *c, int64_t cap, int64_t *count, uint64_t *keys, double *coeff)
{
    PPQ_GUARD(c)
    if (!count) return fail(c, PPQ_E_ARG, "count is NULL");
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    *count = c->nact;
    if (cap < c->nact) return fail(c, PPQ_E_ARG, "buffer too small");
    if (c->nact && (!keys || !coeff)) return fail(c, PPQ_E_ARG, "null buffers");
    PPQ_TRY(c, {
        std::vector<uint32_t> k32(c->nact);
        if (c->nact) {
            ck(hipMemcpyAsync(k32.data(), c->keys[c->cur], c->nact * sizeof(uint32_t), hipMemcpyDeviceToHost,
                              c->stream),
               "get keys");
            ck(hipMemcpyAsync(coeff, c->psi[c->cur], c->nact * sizeof(double2), hipMemcpyDeviceToHost, c->stream),
               "get psi");
        }
        ck(hipStreamSynchronize(c->stream), "get state");
        for (int64_t i = 0; i < c->nact; ++i) keys[i] = k32[i];
    })
    return PPQ_OK;
}

// True for memory the device can address as device memory (a hipMalloc'ed or
// managed allocation); a plain host pointer would fault a kernel.
bool device_pointer(const void *p)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

int ppq_set_state_device(ppq_ctx *c, int64_t count, const uint64_t *keys, const double *coeff)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    if (count < 0 || count > (int64_t)c->g.total || (count > 0 && (!keys || !coeff)))
        return fail(c, PPQ_E_ARG, "bad state arguments");
    if (count > 0 && (!device_pointer(keys) || !device_pointer(coeff)))
        return fail(c, PPQ_E_ARG, "keys and coefficients must be device memory");
    int status = PPQ_OK;
    PPQ_TRY(c, {
        ensure_capacity(c, std::max<int64_t>(count, 1));  // keeps the current state
        const int nxt = 1 - c->cur;
        take_state(keys, reinterpret_cast<const double2 *>(coeff), count, c->g.total, c->keys[nxt], c->psi[nxt],
                   c->flags, c->count, c->stream);
        unsigned long long bad[2] = {0, 0};
        if (count > 0) {
            ck(hipMemcpyAsync(c->h_count, c->count, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                              c->stream),
               "state check");
            ck(hipStreamSynchronize(c->stream), "state check");
            bad[0] = c->h_count[0];
            bad[1] = c->h_count[1];
        }
        if (bad[0]) {
            status = fail(c, PPQ_E_ARG, "keys must be strictly ascending and in range");
        } else if (bad[1]) {
            status = fail(c, PPQ_E_NUMERIC, "non-finite coefficient");
        } else {
            // the checked copy becomes the state (the previous one is dropped)
            c->cur = nxt;
            c->nact = count;
            c->has_state = true;
            c->nsub = 1;
            c->derived_valid = false;
            c->v_valid = false;
            c->v_partial = false;
        }
    })
    return status;
}

int ppq_get_state_device(ppq_ctx *c, int64_t cap, int64_t *count, uint64_t *keys, double *coeff)
{
    PPQ_GUARD(c)
    if (!count) return fail(c, PPQ_E_ARG, "count is NULL");
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    *count = c->nact;
    if (cap < c->nact) return fail(c, PPQ_E_ARG, "buffer too small");
    if (c->nact && (!keys || !coeff)) return fail(c, PPQ_E_ARG, "null buffers");
    if (c->nact && (!device_pointer(keys) || !device_pointer(coeff)))
        return fail(c, PPQ_E_ARG, "keys and coefficients must be device memory");
    PPQ_TRY(c, {
        give_keys(c->keys[c->cur], c->nact, keys, c->stream);
        if (c->nact)
            ck(hipMemcpyAsync(coeff, c->psi[c->cur], c->nact * sizeof(double2), hipMemcpyDeviceToDevice, c->stream),
               "get psi");
        ck(hipGetLastError(), "get state");
    })
    return PPQ_OK;
}

int ppq_apply_h(ppq_ctx *c, const void *x, void *y)
{
    PPQ_GUARD(c)
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    if (c->nact && (!x || !y || x == y)) return fail(c, PPQ_E_ARG, "x and y must be distinct device pointers");
    if (c->nact && (!device_pointer(x) || !device_pointer(y))) return fail(c, PPQ_E_ARG, "x and y must be device memory");
    PPQ_TRY(c, {
        build_derived(c);
        apply_internal(c, x, y, nullptr, 0);
    })
    return PPQ_OK;
}

int ppq_step(ppq_ctx *c, double dt, int m)
{
    PPQ_GUARD(c)
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    if (m < 1 || m > MAXM || !std::isfinite(dt)) return fail(c, PPQ_E_ARG, "1 <= m <= 16, finite dt");
    PPQ_TRY(c, {
        do_step(c, dt, m);
        mark(c, PHASE_NONE);
    })
    return PPQ_OK;
}

int ppq_prune(ppq_ctx *c, double eps, int64_t *n_active, int64_t *n_above)
{
    PPQ_GUARD(c)
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    if (!(eps >= 0.0)) return fail(c, PPQ_E_ARG, "eps must be >= 0");
    PPQ_TRY(c, {
        if (!c->scan_tmp) ensure_capacity(c, 1024);
        int64_t nab = 0;
        do_prune(c, eps, &nab);
        mark(c, PHASE_NONE);
        ck(hipStreamSynchronize(c->stream), "prune");
        if (n_active) *n_active = c->nact;
        if (n_above) *n_above = nab;
    })
    return PPQ_OK;
}

int ppq_enable_timings(ppq_ctx *c, int on)
{
    PPQ_GUARD(c)
    PPQ_TRY(c, {
        ck(hipStreamSynchronize(c->stream), "timings");
        if (c->timing) timing_flush(c);  // keep what the recorded events measured
        c->timing = on != 0;
        c->tcount = 0;
        if (c->timing)
            for (double &v : c->tms) v = 0.0;
    })
    return PPQ_OK;
}

int ppq_timings(ppq_ctx *c, double *ms)
{
    PPQ_GUARD(c)
    if (!ms) return fail(c, PPQ_E_ARG, "null argument");
    PPQ_TRY(c, {
        ck(hipStreamSynchronize(c->stream), "timings");
        timing_flush(c);
        for (int i = 0; i < PPQ_PHASE_N; ++i) ms[i] = c->tms[i];
    })
    return PPQ_OK;
}

int ppq_set_krylov_tolerance(ppq_ctx *c, double tol)
{
    PPQ_GUARD(c)
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(c, PPQ_E_ARG, "Krylov tolerance must be finite and >= 0");
    c->krylov_tol = tol;
    return PPQ_OK;
}

int ppq_set_step_control(ppq_ctx *c, int max_substeps)
{
    PPQ_GUARD(c)
    if (max_substeps < 1 || max_substeps > 1024) return fail(c, PPQ_E_ARG, "max_substeps must be in [1, 1024]");
    c->max_substeps = max_substeps;
    return PPQ_OK;
}

int ppq_set_relative_exclusion(ppq_ctx *c, double r)
{
    PPQ_GUARD(c)
    if (!(r >= 0.0) || !std::isfinite(r)) return fail(c, PPQ_E_ARG, "relative exclusion must be finite and >= 0");
    c->rel_excl = r;
    return PPQ_OK;
}

int ppq_propagate(ppq_ctx *c, int nsteps, double dt, int m, double eps, double *trace)
{
    PPQ_GUARD(c)
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    if (nsteps < 0 || m < 1 || m > MAXM || !std::isfinite(dt)) return fail(c, PPQ_E_ARG, "bad propagate arguments");
    PPQ_TRY(c, {
        if (!c->scan_tmp) ensure_capacity(c, 1024);
        ensure_records(c, (int64_t)nsteps + 1);
        double eps_obs = eps < 0 ? 0.0 : eps;
        mark(c, PPQ_PHASE_TABLES);
        build_derived(c);
        mark(c, PPQ_PHASE_OBS);
        observe_into(c, 0, eps_obs);
        set_record_host(c, 0, 0.0, 0, 0);
        for (int st = 1; st <= nsteps; ++st) {
            mark(c, PPQ_PHASE_TABLES);
            build_derived(c);
            ensure_krylov(c, m);
            // energy of the previous record = alpha_0 of this step
            const bool had = c->nact > 0;
            const StepInfo info = advance(c, dt, m, c->rec + (int64_t)(st - 1) * PPQ_OBS_N + PPQ_OBS_ENERGY);
            if (eps >= 0.0) do_prune(c, eps, nullptr);
            mark(c, PPQ_PHASE_TABLES);
            build_derived(c);
            mark(c, PPQ_PHASE_OBS);
            observe_into(c, st, eps_obs);
            set_record_host(c, st, st * dt, info.meff >= 0 ? info.meff : m, info.nsub);
            if (had && info.meff < 0) copy_meff(c->ks, c->rec + (int64_t)st * PPQ_OBS_N + PPQ_OBS_KRYLOV, c->stream);
        }
        energy_into(c, nsteps);
        mark(c, PHASE_NONE);
        ck(hipStreamSynchronize(c->stream), "propagate");
        if (trace) {
            ck(hipMemcpy(trace, c->rec, sizeof(double) * PPQ_OBS_N * ((int64_t)nsteps + 1), hipMemcpyDeviceToHost),
               "trace");
            // Krylov dimension actually used
        }
    })
    return PPQ_OK;
}

int ppq_observables(ppq_ctx *c, double eps, double *out)
{
    PPQ_GUARD(c)
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    if (!out || !(eps >= 0.0)) return fail(c, PPQ_E_ARG, "bad arguments");
    PPQ_TRY(c, {
        if (!c->scan_tmp) ensure_capacity(c, 1024);
        ensure_records(c, 1);
        build_derived(c);
        observe_into(c, 0, eps);
        set_record_host(c, 0, 0.0, 0, 0);
        energy_into(c, 0);
        ck(hipStreamSynchronize(c->stream), "observables");
        ck(hipMemcpy(out, c->rec, sizeof(double) * PPQ_OBS_N, hipMemcpyDeviceToHost), "obs");
    })
    return PPQ_OK;
}


int ppq_expect_q(ppq_ctx *c, double *q)
{
    PPQ_GUARD(c)
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    if (!q) return fail(c, PPQ_E_ARG, "bad arguments");
    PPQ_TRY(c, {
        const int D = c->g.D;
        std::vector<double> tab((size_t)MAXD * NMAX_FIBER + MAXD, 0.0);
        unsigned nan_mask = 0;
        for (int k = 0; k < D; ++k) {
            if (c->lattice[k]) {
                nan_mask |= 1u << k;
                continue;
            }
            std::vector<double> pts = dim_points(c, k);
            std::copy(pts.begin(), pts.end(), tab.begin() + (size_t)k * NMAX_FIBER);
        }
        if (!c->qtab) c->qtab = dalloc<double>((int64_t)tab.size());
        double *res = c->qtab + (size_t)MAXD * NMAX_FIBER;
        ck(hipMemcpyAsync(c->qtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, c->stream),
           "grid points");
        expect_q(c->keys[c->cur], c->psi[c->cur], c->nact, c->g, c->qtab, NMAX_FIBER, nan_mask, c->partial, res,
                 c->stream);
        ck(hipGetLastError(), "expect_q launch");
        ck(hipStreamSynchronize(c->stream), "expect_q");
        ck(hipMemcpy(q, res, sizeof(double) * D, hipMemcpyDeviceToHost), "expect_q result");
    })
    return PPQ_OK;
}

int ppq_expect_q_noalloc(ppq_ctx *c, double *q)
{
    PPQ_GUARD(c)
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    if (!q) return fail(c, PPQ_E_ARG, "bad arguments");
    hipError_t serr;
    unsigned char *base = (unsigned char *)scratch_of(c->device, &serr);
    if (!base) return fail(c, PPQ_E_STATE, "device scratch unavailable (hipGetSymbolAddress failed)");
    const int D = c->g.D;
    int nmax = 1;
    for (int k = 0; k < D; ++k) nmax = std::max(nmax, c->g.n[k]);
    size_t off_out, off_partial;
    const size_t need = expect_q_scratch_bytes(D, nmax, &off_out, &off_partial);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(c, PPQ_E_CAPACITY, "grid-point table exceeds the no-allocation scratch");
    PPQ_TRY(c, {
        // host staging of the table on the stack; the copy is waited for below
        double tab[MAXD * NMAX_FIBER];
        unsigned nan_mask = 0;
        for (int k = 0; k < D; ++k) {
            if (c->lattice[k]) {
                nan_mask |= 1u << k;
                for (int i = 0; i < nmax; ++i) tab[(size_t)k * nmax + i] = 0.0;
                continue;
            }
            dim_points_into(c, k, tab + (size_t)k * nmax);
            for (int i = c->g.n[k]; i < nmax; ++i) tab[(size_t)k * nmax + i] = 0.0;
        }
        double *dtab = (double *)base;
        double *res = (double *)(base + off_out);
        double2 *partial = (double2 *)(base + off_partial);
        ck(hipMemcpyAsync(dtab, tab, sizeof(double) * (size_t)D * nmax, hipMemcpyHostToDevice, c->stream),
           "grid points");
        expect_q(c->keys[c->cur], c->psi[c->cur], c->nact, c->g, dtab, nmax, nan_mask, partial, res, c->stream);
        ck(hipGetLastError(), "expect_q launch");
        ck(hipStreamSynchronize(c->stream), "expect_q");
        ck(hipMemcpy(q, res, sizeof(double) * D, hipMemcpyDeviceToHost), "expect_q result");
    })
    return PPQ_OK;
}

int ppq_acf_doubled(ppq_ctx *c, double *c2t)
{
    PPQ_GUARD(c)
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    if (!c2t) return fail(c, PPQ_E_ARG, "bad arguments");
    PPQ_TRY(c, { build_operator(c); })
    if (!c->any_lattice && !c->real_sym) return fail(c, PPQ_E_UNSUPPORTED, "C(2t) needs a real symmetric operator");
    if (c->any_lattice && !c->dvr_real_sym)
        return fail(c, PPQ_E_UNSUPPORTED, "C(2t) needs an operator real symmetric in the DVR basis");
    if (c->any_lattice && c->g.total > ACF2_MAX_FULL)
        return fail(c, PPQ_E_CAPACITY, "C(2t) on a lattice basis transforms the full grid: at most 2^28 points");
    PPQ_TRY(c, {
        if (!c->acf2) c->acf2 = dalloc<double2>(1);
        if (!c->any_lattice) {
            sum_of_squares(c->psi[c->cur], c->nact, c->partial, c->acf2, c->stream);
        } else {
            // DVR coefficients on the full grid, c = (x)_k B_k a with B_k =
            // G_k^{-+} (a = G^+ c), then C(2t) = c^T c = a^T B^T B a
            const int64_t total = c->g.total;
            if (c->full_cap < total) {
                for (auto &p : c->full) dfree(p);
                c->full[0] = dalloc<double2>(total);
                c->full[1] = dalloc<double2>(total);
                c->full_cap = total;
            }
            hipStream_t s = c->stream;
            fill_zero_bytes(c->full[0], total * (int64_t)sizeof(double2), s);
            scatter_full(c->keys[c->cur], c->psi[c->cur], c->nact, c->full[0], s);
            int cur = 0;
            for (int k = 0; k < c->g.D; ++k) {
                if (!c->lattice[k]) continue;
                const int n = c->g.n[k];
                const LatticeMaps L = lattice_maps(c, k);
                std::vector<double2> B((size_t)n * n);
                for (size_t i = 0; i < B.size(); ++i) B[i] = make_double2(L.GinvAdj[i].real(), L.GinvAdj[i].imag());
                double2 *dB = upload(B, s);
                transform_full(c->full[cur], c->full[1 - cur], total, (int64_t)c->g.stride[k], n, dB, s);
                ck(hipStreamSynchronize(s), "C(2t) transform");
                dfree(dB);
                cur = 1 - cur;
            }
            sum_of_squares(c->full[cur], total, c->partial, c->acf2, s);
        }
        ck(hipGetLastError(), "C(2t) launch");
        ck(hipStreamSynchronize(c->stream), "C(2t)");
        double2 v;
        ck(hipMemcpy(&v, c->acf2, sizeof(double2), hipMemcpyDeviceToHost), "C(2t) result");
        c2t[0] = v.x;
        c2t[1] = v.y;
    })
    return PPQ_OK;
}

int ppq_set_potential_term(ppq_ctx *c, int term, double coef, const double *params)
{
    PPQ_GUARD(c)
    if (term < 0 || term >= (int)c->terms.size()) return fail(c, PPQ_E_ARG, "term index out of range");
    Term &t = c->terms[term];
    t.coef = coef;
    if (params)
        for (size_t f = 0; f < t.f.size(); ++f) {
            t.f[f].p0 = params[2 * f];
            t.f[f].p1 = params[2 * f + 1];
        }
    c->op_dirty = true;
    c->derived_valid = false;
    c->v_valid = false;
    c->v_partial = false;
    return PPQ_OK;
}

int ppq_add_potential_derivative(ppq_ctx *c, int param, double coef, int nfac, const int32_t *dims,
                                 const int32_t *kinds, const double *params, const double *tables)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    if (param < 0 || param >= ADJ_MAXP) return fail(c, PPQ_E_ARG, "parameter index must be in [0, 32)");
    if (c->any_lattice) return fail(c, PPQ_E_UNSUPPORTED, "adjoint gradients are built for DVR dimensions");
    size_t before = c->terms.size();
    int r = ppq_add_potential_term(c, coef, nfac, dims, kinds, params, tables);
    if (r != PPQ_OK) return r;
    // move the parsed term from the potential to the derivative list
    c->dterms.push_back(c->terms.back());
    c->terms.resize(before);
    c->dparam.push_back(param);
    c->nparam = std::max(c->nparam, param + 1);
    c->op_dirty = true;
    return PPQ_OK;
}

int ppq_adjoint_record(ppq_ctx *c, const double *centre, const double *momentum, const double *width, double eps,
                       int nsteps, double dt, int m, int checkpoint_every, double *J)
{
    PPQ_GUARD(c)
    if (!c->has_grid) return fail(c, PPQ_E_STATE, "no grid");
    if (c->any_lattice) return fail(c, PPQ_E_UNSUPPORTED, "adjoint gradients are built for DVR dimensions");
    for (const Term &t : c->terms)
        if (is_product(c, t))
            return fail(c, PPQ_E_UNSUPPORTED, "adjoint gradients are built for diagonal potential terms");
    if (nsteps < 1 || m < 2 || m > MAXM || checkpoint_every < 1 || !(eps >= 0.0) || !std::isfinite(dt))
        return fail(c, PPQ_E_ARG, "bad adjoint recording arguments");
    int r = ppq_init_gaussian(c, centre, momentum, width, eps, nullptr);
    if (r != PPQ_OK) return r;
    // the recorded steps follow exp(-i H dt) to the tolerance: adaptive order
    // below m and step control (the settings are restored afterwards)
    const double tau = c->krylov_tol > 0.0 ? c->krylov_tol : ADJ_KRYLOV_TOL;
    const double tol_keep = c->krylov_tol;
    const int sub_keep = c->max_substeps;
    c->krylov_tol = tau;
    c->max_substeps = sub_keep > 1 ? sub_keep : 1024;
    int rc = PPQ_OK;
    try {
        clear_record(c);
        record_append(c);
        checkpoint_now(c);
        for (int st = 1; st <= nsteps; ++st) {
            const StepInfo info = do_step(c, dt, m);
            c->rec_sub.push_back(info.nsub);
            do_prune(c, eps, nullptr);
            record_append(c);
            if (st % checkpoint_every == 0 && st < nsteps) checkpoint_now(c);
        }
    } catch (const HipError &e) {
        rc = hip_fail(c, e);
    } catch (const std::bad_alloc &) {
        rc = fail(c, PPQ_E_OOM, "device allocation failed");
    } catch (const std::exception &e) {
        rc = fail(c, PPQ_E_NUMERIC, e.what());
    }
    c->krylov_tol = tol_keep;
    c->max_substeps = sub_keep;
    if (rc != PPQ_OK) {
        clear_record(c);
        return rc;
    }
    PPQ_TRY(c, {
        c->rec_C = overlap_with_packet(c);
        for (int k = 0; k < c->g.D; ++k) {
            c->rec_centre[k] = centre[k];
            c->rec_momentum[k] = momentum[k];
        }
        c->rec_steps = nsteps;
        c->rec_m = m;
        c->rec_dt = dt;
        c->rec_tol = tau;
        c->rec_every = checkpoint_every;
        c->recorded = true;
        mark(c, PHASE_NONE);
        if (J) *J = c->rec_C.x * c->rec_C.x + c->rec_C.y * c->rec_C.y;
    })
    return PPQ_OK;
}

int ppq_adjoint_frozen(ppq_ctx *c, const double *centre, const double *momentum, double *J)
{
    PPQ_GUARD(c)
    if (!c->recorded) return fail(c, PPQ_E_STATE, "no recorded trajectory");
    if (!centre || !momentum || !J) return fail(c, PPQ_E_ARG, "null argument");
    PPQ_TRY(c, {
        int64_t nmax_set = *std::max_element(c->rec_n.begin(), c->rec_n.end());
        ensure_capacity(c, std::max<int64_t>(nmax_set, 1));
        double w[MAXD];
        for (int k = 0; k < c->g.D; ++k) w[k] = c->pk_width[k];
        set_packet_tables(c, centre, momentum, w);
        auto keys_of = [&](int st) { return c->rec_keys + c->rec_off[st]; };
        set_current_set(c, keys_of(0), c->rec_n[0]);
        product_values(c->keys[c->cur], c->nact, c->g, c->init_tabs, c->tab_nmax, c->psi[c->cur], c->stream);
        for (int st = 1; st <= c->rec_steps; ++st) {
            build_derived(c);
            ensure_krylov(c, c->rec_m);
            // the recording's substeps, each at its tolerance
            const int ns = c->rec_sub[st - 1];
            const double h = c->rec_dt / (double)ns;
            for (int j = 0; j < ns && c->nact; ++j) {
                if (c->precision == PPQ_FP64) step_impl<double2>(c, h, c->rec_m, c->rec_tol);
                else step_impl<float2>(c, h, c->rec_m, c->rec_tol);
            }
            frozen_remap(c, keys_of(st), c->rec_n[st]);
        }
        double2 C = overlap_with_packet(c);
        *J = C.x * C.x + C.y * C.y;
        mark(c, PHASE_NONE);
    })
    return PPQ_OK;
}

int ppq_adjoint_gradient(ppq_ctx *c, double *dJ_dparam, double *dJ_dcentre, double *dJ_dmomentum)
{
    PPQ_GUARD(c)
    if (!c->recorded) return fail(c, PPQ_E_STATE, "no recorded trajectory");
    PPQ_TRY(c, {
        const int D = c->g.D;
        int64_t nmax_set = *std::max_element(c->rec_n.begin(), c->rec_n.end());
        ensure_capacity(c, std::max<int64_t>(nmax_set, 1));
        // the packet of the recording (ppq_adjoint_frozen may have changed the tables)
        double w[MAXD];
        for (int k = 0; k < D; ++k) w[k] = c->pk_width[k];
        set_packet_tables(c, c->rec_centre, c->rec_momentum, w);
        build_operator(c);
        ensure_krylov(c, c->rec_m);
        ensure_adjoint_buffers(c, c->rec_m, max_segment_states(c));
        if (c->precision == PPQ_FP64) adjoint_backward<double2>(c, c->rec_C);
        else adjoint_backward<float2>(c, c->rec_C);
        std::vector<double2> dC(ADJ_MAXP + 2 * MAXD);
        ck(hipMemcpy(dC.data(), c->dC, dC.size() * sizeof(double2), hipMemcpyDeviceToHost), "dC");
        const double2 Cn = c->rec_C;
        auto grad = [&](double2 d) { return 2.0 * (Cn.x * d.x + Cn.y * d.y); };  // 2 Re(conj(C) dC)
        if (dJ_dparam)
            for (int p = 0; p < c->nparam; ++p) dJ_dparam[p] = grad(dC[p]);
        for (int k = 0; k < D; ++k) {
            if (dJ_dcentre) dJ_dcentre[k] = grad(dC[c->nparam + 2 * k]);
            if (dJ_dmomentum) dJ_dmomentum[k] = grad(dC[c->nparam + 2 * k + 1]);
        }
        mark(c, PHASE_NONE);
    })
    return PPQ_OK;
}

int ppq_time_apply(ppq_ctx *c, int nrep, double *ms_median, double *ms_mean)
{
    PPQ_GUARD(c)
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    if (nrep < 1 || nrep > 100000 || !ms_median) return fail(c, PPQ_E_ARG, "1 <= nrep <= 100000");
    PPQ_TRY(c, {
        build_derived(c);
        ensure_krylov(c, std::max(c->kv_m, 1));
        const void *x = c->psi[c->cur];
        if (c->precision == PPQ_FP32) {
            norm0<float2>(c->psi[c->cur], c->nact, c->partial, c->counter, c->ks, 1, 0.0, 0.0, c->stream);
            normalise_from_master<float2>(c->psi[c->cur], c->nact, c->ks, (float2 *)c->Vk, c->stream);
            x = c->Vk;
        }
        apply_internal(c, x, c->wk, nullptr, 0);
        // one event between consecutive applications: nrep intervals
        std::vector<hipEvent_t> ev(nrep + 1, nullptr);
        int made = 0;
        try {
            for (; made <= nrep; ++made) ck(hipEventCreate(&ev[made]), "event");
            for (int r = 0; r < nrep; ++r) {
                ck(hipEventRecord(ev[r], c->stream), "event");
                apply_internal(c, x, c->wk, nullptr, 0);
            }
            ck(hipEventRecord(ev[nrep], c->stream), "event");
            ck(hipEventSynchronize(ev[nrep]), "event sync");
            std::vector<double> t(nrep);
            for (int r = 0; r < nrep; ++r) {
                float ms = 0.f;
                ck(hipEventElapsedTime(&ms, ev[r], ev[r + 1]), "elapsed");
                t[r] = ms;
            }
            float total = 0.f;
            ck(hipEventElapsedTime(&total, ev[0], ev[nrep]), "elapsed");
            std::sort(t.begin(), t.end());
            *ms_median = nrep % 2 ? t[nrep / 2] : 0.5 * (t[nrep / 2 - 1] + t[nrep / 2]);
            if (ms_mean) *ms_mean = (double)total / nrep;
        } catch (...) {
            for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
            throw;
        }
        for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    })
    return PPQ_OK;
}

int ppq_fiber_counts(ppq_ctx *c, int64_t *nf)
{
    PPQ_GUARD(c)
    if (!c->has_state) return fail(c, PPQ_E_STATE, "no state");
    if (!nf) return fail(c, PPQ_E_ARG, "nf is NULL");
    PPQ_TRY(c, {
        build_derived(c);
        ensure_nf(c);
        for (int k = 0; k < c->g.D; ++k) nf[k] = c->nf[k];
    })
    return PPQ_OK;
}

}  // extern "C"
