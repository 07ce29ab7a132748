// Internal declarations of the gfx950 library behind include/ppq.h.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ppq.h"

namespace ppq {

constexpr int MAXD = 8;
constexpr int MAXM = 16;        // largest Krylov order
constexpr int NMAX_FIBER = 256;  // largest 1D basis (digits are 8-bit in the fiber tables)
constexpr int NMAX_MASK = 64;    // largest 1D basis with fiber masks (one 64-bit word) and
                                 // the mask-driven kernels; longer dimensions keep a digit
                                 // per fiber entry and take the long-fiber pass
constexpr int RED_BLOCKS = 1024;  // blocks of the fixed-shape reductions
constexpr int PSTRIDE_H = 36;  // partial sums per block (matches the kernels)
constexpr int64_t ACF2_MAX_FULL = int64_t(1) << 28;  // full grid of C(2t) on lattice bases

// Grid geometry passed by value to kernels.
struct GridDesc {
    int D;
    int n[MAXD];
    uint32_t stride[MAXD];  // row-major, last dimension fastest
    int lat_s[MAXD];        // phase-space lattice shape; lat_s == 0 -> +-1 line stencil
    int lat_l[MAXD];
    uint32_t total;
    int pairs;              // adaption stencil over the phase-space axes (one per DVR
                            // dimension, cell and level per lattice one): 0 = +-1 on one
                            // axis, 1 = also +-1 on two axes at once, 2 = every
                            // combination of -1/0/+1 changes
};

// Diagonal potential as a sum of products of 1D tables.
struct PotDesc {
    int nterm;
    int D;
    int nmax;
    const double *coef;   // [nterm]
    const int *tab;       // [nterm][D]: table index or -1
    const double *tabs;   // [ntab][nmax]
    int ntab;
};

// Device state of one Krylov step.
struct KState {
    double n0;                 // |psi|
    double alpha[MAXM];        // Re <v_j|H v_j>
    double beta[MAXM];         // |w_j| after reorthogonalisation
    double2 h1[MAXM * MAXM];   // Hessenberg, first Gram-Schmidt pass  [i*MAXM + j]
    double2 h2[MAXM * MAXM];   // second pass
    double2 y[MAXM];           // coefficients of the propagated vector
    double2 cc[MAXM];          // delayed correction: H v_j = (H q_j - sum_k cc_k v_k) / beta_{j-1}
    double inv_b;              // 1 / beta_{j-1} for the provisional q_j
    double est;                // error estimate of the current order: n0 dt^k/k! prod beta_i
    double kdt, ktol;          // step and order tolerance of this step (ktol 0: full order)
    int meff;                  // Krylov dimension actually built
    int pad;
};

// ---- launchers (ppq_kernels.hip) ------------------------------------------
void fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);
void fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
void fill_zero_bytes(void *p, int64_t nbytes, hipStream_t s);

// exclusive scans; *total receives the sum; tmp holds >= scan_tmp_words(n) words
int64_t scan_tmp_words(int64_t n);
void scan_popcount(const uint64_t *words, int64_t nwords, uint32_t *prefix, uint32_t *total, uint32_t *tmp,
                   hipStream_t s);
void scan_u32(const uint32_t *in, int64_t n, uint32_t *out, uint32_t *total, uint32_t *tmp, hipStream_t s);

void init_flag(const GridDesc &g, const double2 *tabs, int nmax, double eps2, uint64_t *bm,
               unsigned long long *nabove, hipStream_t s);
void product_values(const uint32_t *keys, int64_t n, const GridDesc &g, const double2 *tabs, int nmax,
                    double2 *out, hipStream_t s);
// block_counts: work space of at least n / 256 + 1 entries
void dilate(const uint32_t *keys, const double2 *psi, int64_t n, const GridDesc &g, double eps2, uint64_t *bm,
            unsigned long long *nabove, unsigned *block_counts, hipStream_t s);
// The same dilation for the +-1 stencil on a grid without lattice axes, word
// by word: K (nwords words of work space) gets one bit per function above the
// threshold, then every word of bm (nwords + 2 words) is written from K and
// its shifts by the strides.  Costs O(nwords) instead of O(n) atomics.
void dilate_words(const uint32_t *keys, const double2 *psi, int64_t n, const GridDesc &g, double eps2, uint64_t *K,
                  uint64_t *bm, int64_t nwords, unsigned long long *nabove, unsigned *block_counts, hipStream_t s);
void compact(const uint64_t *bm, const uint32_t *prefix, int64_t nwords, uint32_t *keys_out, hipStream_t s);
void remap(const uint32_t *okeys, const double2 *opsi, int64_t n_old, const uint64_t *bm, const uint32_t *prefix,
           double2 *npsi, hipStream_t s);
// relative exclusion: sets the bits of all n keys when at most rel * n of them
// are clear (block_counts: nblocks(n) entries; dropped: one device counter)
void keep_all_if_few_dropped(const uint32_t *keys, int64_t n, uint64_t *bm, double rel, unsigned *block_counts,
                             unsigned long long *dropped, hipStream_t s);
void mark_keys(const uint32_t *keys, int64_t n, uint64_t *bm, hipStream_t s);

// fiber tables
void last_flags(const uint32_t *keys, int64_t n, int nlast, uint32_t *flags, hipStream_t s);
void last_info(const uint32_t *keys, int64_t n, int nlast, uint8_t *info, hipStream_t s);
void last_fill(const uint32_t *keys, int64_t n, int nlast, const uint32_t *flags, const uint32_t *fidx,
               const uint32_t *nf, uint32_t *off, uint64_t *mask, hipStream_t s);
// Rotated order: the frame key (see RotFrame) with the digit of stride sk and
// size nk moved to the last place.
struct RotFrame {
    uint32_t sk, nk;    // stride and size of the digit moved last, within the frame key
    uint32_t rin, rout;  // inner-first frame (S_in, total / S_in); rin == 0: row-major frame
};
inline RotFrame row_major_rot(const GridDesc &g, int k) { return RotFrame{g.stride[k], (uint32_t)g.n[k], 0u, 0u}; }
// fiber tables of dimensions 0..nd-1 (row-major frames) in one set of launches
struct RotAll {
    int nd;                 // dimensions 0..nd-1 (all but the last)
    uint32_t sk[MAXD];      // stride of the digit moved last
    uint32_t nk[MAXD];      // its size
    int64_t nwords;         // words per rotated bitmap
    int64_t owoff[MAXD + 1];  // word offsets of the fiber-slot bitmaps (one bit per key without digit k)
};
struct TabPtrs {
    uint32_t *pi[MAXD];
    uint32_t *off[MAXD];
    uint64_t *mask[MAXD];
};
// bm, prefix: (nd+1)*nwords + 2 words (nd rotated segments, then the row-major
// one); occ, oprefix: owoff[nd] + 2 words (per dimension a bit for every
// fiber slot that holds a point; their ranks number the fibers); counters: 2
// entries of scratch; nf[k] receives dimension k's fiber count.
void fiber_tables_all(const uint32_t *keys, int64_t n, const RotAll &r, uint64_t *bm, uint32_t *prefix,
                      uint64_t *occ, uint32_t *oprefix, const TabPtrs &t, uint32_t *scan_tmp, uint32_t *counters,
                      uint32_t *nf, hipStream_t s);
void rot_set(const uint32_t *keys, int64_t n, const RotFrame &f, uint64_t *bm, hipStream_t s);
void rot_rank(const uint32_t *keys, int64_t n, const RotFrame &f, const uint64_t *bm, const uint32_t *prefix,
              const uint32_t *map, uint32_t *pi, uint32_t *inv, uint32_t *flags, uint64_t *tmpmask, uint8_t *info,
              hipStream_t s);
// chunk starts of whole blocks (see the block-fused H*psi); chunk has
// ceil(n / S) + 1 entries
void make_chunks(const uint32_t *keys, const uint32_t *P, int64_t n, uint32_t sin, bool inner, uint32_t S,
                 uint32_t cap, uint32_t *chunk, uint32_t *big, uint32_t *counters, hipStream_t s);
// out[t] = index of the first fiber of chunk t (fidx: exclusive scan of the
// fiber start flags in the dimension's fiber order; chunk starts are fiber starts)
void chunk_fibers(const uint32_t *chunk, int64_t n, uint32_t S, const uint32_t *fidx, const uint32_t *nf,
                  uint32_t *out, hipStream_t s);
void fib_fill(const uint32_t *flags, const uint32_t *fidx, const uint64_t *tmpmask, int64_t n,
              const uint32_t *nf, uint32_t *off, uint64_t *mask, hipStream_t s);

// V (or Vf) of every point; with `list` (uint32[n] work space) and `count`
// (one device counter) only where V holds NaN, the rest is kept
void potential(const uint32_t *keys, int64_t n, const GridDesc &g, const PotDesc &pd, double *V, float *Vf,
               uint32_t *list, unsigned *count, hipStream_t s);
// nv[rank of okeys[p] in the bitmap] = ov[p] for the keys that stay
template <class T>
void remap_values(const uint32_t *okeys, const T *ov, int64_t n_old, const uint64_t *bm, const uint32_t *prefix,
                  T *nv, hipStream_t s);

// fiber contraction y (+)= P h_k P x along one dimension
struct FiberPass {
    const uint32_t *pi;     // nullptr for the last dimension (identity)
    const uint32_t *off;
    const uint64_t *mask;
    int64_t nf;
    int nmax;               // padded 1D size (matrix leading dimension)
    bool stage = false;     // lane-per-fiber pass: stage each wavefront's ranks of pi in LDS
};
// a pass over a dimension longer than NMAX_MASK: fibers as (off) runs of the
// dimension's order with the digit of every entry (no masks)
struct LongPass {
    const uint32_t *pi;     // nullptr for the last dimension (identity)
    const uint32_t *off;    // [nf + 1]
    const uint8_t *dig;     // digit of each entry in the dimension's order
    int64_t nf;
    int n;                  // size of the dimension (leading dimension of h)
};
void hpsi_long_real_f64(const LongPass &lp, const double *T, const double2 *x, const double *V, double2 *y,
                        bool first, const int *skip_if, int skip_j, hipStream_t s);
void hpsi_long_real_f32(const LongPass &lp, const float *T, const float2 *x, const float *V, float2 *y, bool first,
                        const int *skip_if, int skip_j, hipStream_t s);
struct CInput;
struct CInput32;
void hpsi_long_cplx_f64(const LongPass &lp, const double2 *H, const CInput &in, double2 *y, bool accumulate,
                        const int *skip_if, int skip_j, hipStream_t s);
void hpsi_long_cplx_f32(const LongPass &lp, const float2 *H, const CInput32 &in, float2 *y, bool accumulate,
                        const int *skip_if, int skip_j, hipStream_t s);
// real factor (DVR), FP64; first==true writes y = (T + V) x, else y += T x
void hpsi_real_f64(const FiberPass &fp, const double *T, const double2 *x, const double *V, double2 *y,
                   bool first, const int *skip_if, int skip_j, hipStream_t s);
// complex factor, FP64: y (= or +=) coef * h * (sum_i c_i x_i)  (up to 4 inputs)
struct CInput {
    int nin;
    const double2 *x[4];
    double2 c[4];
};
void hpsi_cplx_f64(const FiberPass &fp, const double2 *H, const CInput &in, double2 *y, bool accumulate,
                   const double *V, const int *skip_if, int skip_j, hipStream_t s);
// point-parallel form: info[q] = digit | 0x80 at the first member of each fiber
void hpsi_pt_f64(const uint32_t *pi, const uint8_t *info, int64_t n, int nmax, const double *T, const double2 *x,
                 const double *V, double2 *y, bool first, const int *skip_if, int skip_j, hipStream_t s);
void hpsi_pt_f32(const uint32_t *pi, const uint8_t *info, int64_t n, int nmax, const float *T, const float2 *x,
                 const float *V, float2 *y, bool first, const int *skip_if, int skip_j, hipStream_t s);
// accumulating pass (y += P h P x) with all loads issued before the contraction;
// with dotp, every block also stores its share of <x|y> (the y it leaves) in
// dotp[block] and the number of blocks is returned (0 without dotp)
int hpsi_acc_f64(const FiberPass &fp, const double *T, const double2 *x, double2 *y, const int *skip_if, int skip_j,
                 hipStream_t s, double2 *dotp = nullptr);
int hpsi_acc_f32(const FiberPass &fp, const float *T, const float2 *x, float2 *y, const int *skip_if, int skip_j,
                 hipStream_t s, double2 *dotp = nullptr);
// blocks of a fused <x|y> the shared partial buffer holds (RED_BLOCKS * PSTRIDE_H)
constexpr int64_t DOT_BLOCKS_MAX = (int64_t)RED_BLOCKS * PSTRIDE_H;
// Krylov reduction of nb per-block partials of one value (mode RED_H1 or RED_DELAY)
void finalize_dot(const double2 *partial, int nb, KState *ks, int j, int m, int mode, hipStream_t s);
// matrix-core forms (v_mfma_*_16x16x4); T64 / H64 are h zero-padded to 64 x 64
void hpsi_mfma_f32(const FiberPass &fp, const float *T64, const float2 *x, const float *V, float2 *y, bool first,
                   const int *skip_if, int skip_j, hipStream_t s);
void hpsi_mfma_f64(const FiberPass &fp, const double *T64, const double2 *x, const double *V, double2 *y, bool first,
                   const int *skip_if, int skip_j, hipStream_t s);
// block-fused form: one pass applies the 1D factors of up to 4 dimensions to
// chunks of whole blocks staged in LDS (see ppq_hpsi.hip)
constexpr int BLOCK_MAXDIM = 4;
constexpr int BLOCK_MAXNB = 32;
constexpr uint32_t BLOCK_WINDOW = 512;  // chunk t starts at the first block start >= t * window;
                                        // window >= BLOCK_WINDOW (chunk tables are sized for it)
constexpr uint32_t LDS_BYTES = 160u * 1024u;
// LDS per staged point: x and y (complex) and a 16-bit local rank per
// dimension with a permutation
inline uint32_t block_point_bytes(int precision, int npi)
{
    return (precision == PPQ_FP64 ? 32u : 16u) + 2u * (uint32_t)npi;
}
// capacity of the main launch (two 512-thread workgroups per CU: 4 or 8
// points per thread); chunks above it go to the 1024-thread launch, which
// holds up to 5 (FP64) or 8 (FP32) points per thread
inline uint32_t block_cap_small(int precision) { return precision == PPQ_FP64 ? 2048u : 4032u; }
inline uint32_t block_cap_max(int precision, int npi)
{
    const uint32_t lds = LDS_BYTES / block_point_bytes(precision, npi) / 64u * 64u;
    const uint32_t thr = precision == PPQ_FP64 ? 5u * 1024u : 8u * 1024u;
    return lds < thr ? lds : thr;
}
// the one-lane-per-fiber block pass: 256-thread workgroups with 8 (FP64) or
// 16 (FP32) points per thread
inline uint32_t block2_cap_small(int precision) { return precision == PPQ_FP64 ? 2048u : 4096u; }
struct BlockPass {
    int ndim;
    int dim[BLOCK_MAXDIM];
    const uint32_t *pi[BLOCK_MAXDIM];    // fiber-order rank -> frame rank; nullptr = identity
    const uint32_t *off[BLOCK_MAXDIM];   // fiber starts in fiber-order ranks, off[nf] = n
    const uint64_t *mask[BLOCK_MAXDIM];
    const uint32_t *fch[BLOCK_MAXDIM];   // [nch + 1] first fiber of each chunk
    int64_t nf[BLOCK_MAXDIM];
    int nb[BLOCK_MAXDIM];                // leading dimension of the factor table
    const uint32_t *chunk;               // [nch + 1] chunk starts (frame ranks)
    uint32_t nch;
    const uint32_t *P;                   // frame rank -> storage position; nullptr = identity
    const uint32_t *big;                 // chunks longer than cap_small
    uint32_t nbig;
    uint32_t cap_small, cap_big;         // LDS capacity (points) of the two launches
    int unroll = 1;                      // one-lane-per-fiber pass: unrolled row loop
};
void hpsi_block_f64(const BlockPass &bp, const double *const *T, const double2 *x, const double *V, double2 *y,
                    bool accumulate, const int *skip_if, int skip_j, hipStream_t s);
void hpsi_block_f32(const BlockPass &bp, const float *const *T, const float2 *x, const float *V, float2 *y,
                    bool accumulate, const int *skip_if, int skip_j, hipStream_t s);
// the same passes with one lane per fiber over the whole window (see ppq_hpsi.hip)
void hpsi_block2_f64(const BlockPass &bp, const double *const *T, const double2 *x, const double *V, double2 *y,
                     bool accumulate, const int *skip_if, int skip_j, hipStream_t s);
void hpsi_block2_f32(const BlockPass &bp, const float *const *T, const float2 *x, const float *V, float2 *y,
                     bool accumulate, const int *skip_if, int skip_j, hipStream_t s);

// ---- plane pass: two adjacent dimensions (a, a+1) per pass ------------------
// Frame: every other digit in row-major order, then the pair's merged digit
// d_a n_{a+1} + d_{a+1}; the points sharing every other digit (a plane) are a
// contiguous run of it.  For the last two dimensions the frame is the key
// order itself (P == nullptr).
constexpr int PLANE_SPAN = 768;        // members one wavefront holds at once (a round)
constexpr uint32_t PLANE_WINDOW = 512;  // task t: the planes starting in [t W, (t + 1) W)
constexpr int PLANE_NMAX = 32;         // largest size of either dimension of a pair
struct PlanePass {
    const uint32_t *P;       // frame rank -> storage position; nullptr = identity
    const uint16_t *dig;     // (d_a << 8) | d_{a+1} per frame rank; bit 15 marks a plane's last member
    const uint32_t *tstart;  // first frame rank of each task (a plane start) [ntask + 1], tstart[ntask] = n
    uint32_t ntask;          // ceil(n / PLANE_WINDOW)
    int na, nb;              // tile shape: the two factors' padded sizes (leading dimensions)
};
// Builds a pair's frame tables.  bm/prefix: a bitmap of the grid (nwords + 2
// words) and its prefix (rotated frames only); poff (n + 1), pkey, flags,
// pidx (n each): work space; counter: one device word of work space.  A plane
// must hold fewer than PLANE_SPAN points (n_a n_{a+1} < PLANE_SPAN).
void plane_tables(const uint32_t *keys, int64_t n, const GridDesc &g, int a, uint64_t *bm, uint32_t *prefix,
                  int64_t nwords, uint32_t *P, uint16_t *dig, uint32_t *tstart, uint32_t *poff, uint32_t *pkey,
                  uint32_t *flags, uint32_t *pidx, uint32_t *scan_tmp, uint32_t *counter, hipStream_t s);
// y (+)= (h_a (x) 1 + 1 (x) h_{a+1}) x over every plane; first == true writes
// y = ... + V x.  Ta, Tb: the factors (na x na, nb x nb, row-major).
void hpsi_plane_f64(const PlanePass &pp, const double *Ta, const double *Tb, const double2 *x, const double *V,
                    double2 *y, bool first, const int *skip_if, int skip_j, hipStream_t s);
void hpsi_plane_f32(const PlanePass &pp, const float *Ta, const float *Tb, const float2 *x, const float *V,
                    float2 *y, bool first, const int *skip_if, int skip_j, hipStream_t s);
// ---- pair pass: the last two dimensions (a = D-2, b = D-1) in one pass -------
// A plane (every digit but the last two fixed) is a contiguous run of the
// sorted state and, in the rotated order of dimension a (digit a moved last),
// occupies the same range of ranks.  Task t holds the planes that start in
// [t PAIR_WINDOW, (t + 1) PAIR_WINDOW); a plane holds at most n_a n_b points.
constexpr uint32_t PAIR_WINDOW = 256;
constexpr uint32_t PAIR_NAB_MAX = 1024;  // largest n_a n_b the pass takes
struct PairPass {
    const uint32_t *keys;    // sorted keys of the set
    const uint32_t *pi_a;    // dimension a's permutation: rank -> position
    const uint32_t *tstart;  // first position of each task [ntask + 1], tstart[ntask] = n
    uint32_t ntask;          // ceil(n / PAIR_WINDOW)
    int n_a, n_b;            // grid sizes of the two dimensions (digit extraction)
    int lda, ldb;            // padded sizes: row strides of the two factors
};
// tstart of the pair pass (ntask + 1 words)
void pair_tasks(const uint32_t *keys, int64_t n, uint32_t nab, uint32_t *tstart, hipStream_t s);
// y = (V + h_a (x) 1 + 1 (x) h_b) x over the last two dimensions (writes y)
void hpsi_pair_f64(const PairPass &pp, const double *Ta, const double *Tb, const double2 *x, const double *V,
                   double2 *y, const int *skip_if, int skip_j, hipStream_t s);
void hpsi_pair_f32(const PairPass &pp, const float *Ta, const float *Tb, const float2 *x, const float *V, float2 *y,
                   const int *skip_if, int skip_j, hipStream_t s);
// FP32 forms
void hpsi_real_f32(const FiberPass &fp, const float *T, const float2 *x, const float *V, float2 *y, bool first,
                   const int *skip_if, int skip_j, hipStream_t s);
struct CInput32 {
    int nin;
    const float2 *x[4];
    float2 c[4];
};
void hpsi_cplx_f32(const FiberPass &fp, const float2 *H, const CInput32 &in, float2 *y, bool accumulate,
                   const float *V, const int *skip_if, int skip_j, hipStream_t s);
// complex factors on the matrix cores: y (= or +=) h (sum_i c_i x_i), h padded to 64 x 64
void hpsi_cmfma_f64(const FiberPass &fp, const double2 *H64, const CInput &in, double2 *y, bool accumulate,
                    const int *skip_if, int skip_j, hipStream_t s);
void hpsi_cmfma_f32(const FiberPass &fp, const float2 *H64, const CInput32 &in, float2 *y, bool accumulate,
                    const int *skip_if, int skip_j, hipStream_t s);

// full-grid tensors (C(2t) on lattice bases): full[keys[p]] = psi[p]; and
// y = B applied along the digit of the given stride (size nk, B nk x nk)
void scatter_full(const uint32_t *keys, const double2 *psi, int64_t n, double2 *full, hipStream_t s);
void transform_full(const double2 *x, double2 *y, int64_t total, int64_t stride, int nk, const double2 *B,
                    hipStream_t s);

// y (= or +=) w D(I) x with D(I) = prod_{k in use} tab[k * nmax + i_k] (the
// diagonal factors of a product term); C is double2 or float2
template <class C>
void diag_scale(const uint32_t *keys, const C *x, int64_t n, const GridDesc &g, const double *tab, int nmax,
                unsigned use, double2 w, C *y, bool acc, const int *skip_if, int skip_j, hipStream_t s);

// Krylov vector kernels. V_i = Vb + i*ld (elements); C is double2 or float2.
// Reductions write per-block partials; one finalising block sums them in a
// fixed order (run-to-run deterministic) and updates KState.
// RED_H1: first-pass dots into h1[.][j] (alpha_j from the diagonal one).
// RED_BETA: second-pass dots into h2[.][j], then beta_j from the last value,
// |q_{j+1}|^2, less their squares, and the order's error estimate.
// RED_DELAY: Hermitian step with delayed correction, r[0] = <q_j|H q_j> of the
// provisional vector; sets alpha_j, cc and inv_b (see k_lanczos_sweep).
// RED_ADELAY: the same for an Arnoldi step, r[i] = <v_i|H q_j> (i < j) and
// r[j] = <q_j|H q_j>; sets the first-pass column h1[.][j], cc and inv_b.
enum ReduceMode { RED_NORM0 = 0, RED_H1 = 1, RED_BETA = 2, RED_DELAY = 3, RED_ADELAY = 4 };
template <class C>
void norm0(const double2 *psi, int64_t n, double2 *partial, unsigned *counter, KState *ks, int m, double dt,
           double tol, hipStream_t s);
template <class C>
void cgs_dots(const C *Vb, int64_t ld, int nv, const C *w, int64_t n, double2 *partial, unsigned *counter, KState *ks,
              int j, int m, int ioff, hipStream_t s, int mode = RED_H1);
// Hermitian Lanczos step j with the second Gram-Schmidt pass delayed by one
// step (see k_lanczos_sweep): corrects v_j in its slot, writes the provisional
// q_{j+1} to slot j+1 and reduces <v_i|q_{j+1}> (i <= j) and |q_{j+1}|^2
// into h2[.][j] and beta_j.  lanczos_fix corrects the last vector alone.
template <class C>
void lanczos_sweep(C *Vb, int64_t ld, const C *z, int64_t n, double2 *partial, unsigned *counter, KState *ks, int j,
                   int m, hipStream_t s);
template <class C>
void lanczos_fix(C *Vb, int64_t ld, int64_t n, const KState *ks, int j, hipStream_t s);
// Arnoldi step j with the second pass delayed: the dots <v_i|z> (i < j) and
// <q_j|z> of z = H q_j (RED_ADELAY), then one sweep that corrects v_j, forms
// q_{j+1} = H v_j - sum_{i<=j} h1_ij v_i and reduces its second-pass dots and
// norm (RED_BETA); `last`: the first reduction only (the step's last column)
template <class C>
void arnoldi_step(C *Vb, int64_t ld, const C *z, int64_t n, double2 *partial, unsigned *counter, KState *ks, int j,
                  int m, bool last, hipStream_t s);
// after the exponential: fold the last vector's pending correction into the
// coefficients y of a step that ran to its full order m (for a recombination
// that reads the provisional last vector)
void lanczos_coef(KState *ks, int m, hipStream_t s);
template <class C>
void normalise_from_master(const double2 *psi, int64_t n, KState *ks, C *v0, hipStream_t s);
template <class C>
void lincomb(const C *Vb, int64_t ld, const double2 *psi_master, int64_t n, const KState *ks, double2 *psi_out,
             hipStream_t s);
void krylov_expv(KState *ks, int m, double dt, int hermitian, hipStream_t s);

// observables
void obs_partial(const uint32_t *keys, const double2 *psi, int64_t n, const GridDesc &g, const double2 *bra,
                 int nmax, double eps2, double2 *partial, hipStream_t s);
void obs_final(const double2 *partial, int nblocks, double *rec, hipStream_t s);
void copy_alpha0(const KState *ks, double *dst, hipStream_t s);
void set_record(double *rec, double t, double nact, double krylov, double nsub, hipStream_t s);
// *out = sum_I psi_I^2 (device), fixed-order; partials in `partial`
void sum_of_squares(const double2 *psi, int64_t n, double2 *partial, double2 *out, hipStream_t s);
// device state transfer: caller keys/coefficients into the context's buffers,
// with violation counts bad[0] (keys) and bad[1] (non-finite values);
// block_counts holds 2 * nblocks(n) entries
void take_state(const uint64_t *keys, const double2 *coeff, int64_t n, uint64_t total, uint32_t *k32, double2 *psi,
                unsigned *block_counts, unsigned long long *bad, hipStream_t s);
void give_keys(const uint32_t *k32, int64_t n, uint64_t *keys, hipStream_t s);
// position expectations out[D] (device): two launches, partials in `partial`
void expect_q(const uint32_t *keys, const double2 *psi, int64_t n, const GridDesc &g, const double *q, int nmax,
              unsigned nan_mask, double2 *partial, double *out, hipStream_t s);

// adjoint
struct DerivDesc {
    int nparam;
    int nterm;
    int nmax;
    const int *param;     // [nterm]
    const double *coef;   // [nterm]
    const int *tab;       // [nterm][D] table index or -1
    const double *tabs;   // [ntab][nmax]
    int ntab;
};
constexpr int ADJ_MAXP = 32;
// Krylov tolerance of the adjoint's recorded steps unless the context sets one
constexpr double ADJ_KRYLOV_TOL = 1e-12;
void gather_remap(const uint32_t *keys, int64_t n, const uint64_t *bm, const uint32_t *prefix, const double2 *lam,
                  double2 *mu, hipStream_t s);
void mark_keys_wave(const uint32_t *keys, int64_t n, uint64_t *bm, hipStream_t s);
void adj_q(const KState *kf, const KState *kb, double dt, double2 *Q, hipStream_t s);
template <class C>
void adj_reduce(const C *Vb, const C *Wb, int64_t ld, const double2 *psi, const double2 *mu, const KState *kf,
                const KState *kb, const double2 *Q, const uint32_t *keys, int64_t n, const GridDesc &g,
                const DerivDesc &dd, double2 *partial, hipStream_t s);
void adj_accumulate(const double2 *partial, int nparam, double2 coef, double2 *dC, hipStream_t s);
void adj_packet(const uint32_t *keys, int64_t n, const GridDesc &g, const double2 *tabs, const double2 *dtabs,
                int nmax, const double2 *vec, int bra, double2 *partial, hipStream_t s);
unsigned long long count_diff(const double2 *a, const double2 *b, int64_t n, unsigned long long *dcount,
                              unsigned long long *hcount, hipStream_t s);
void copy_meff(const KState *ks, double *dst, hipStream_t s);
void energy_from_dot(const double2 *partial, int nblocks, double *rec, hipStream_t s);
void dot_partial(const double2 *a, const double2 *b, int64_t n, double2 *partial, hipStream_t s);

}  // namespace ppq
