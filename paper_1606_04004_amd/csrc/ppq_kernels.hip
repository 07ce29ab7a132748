// gfx950 kernels: scans, adaption (flag / dilate / compact / remap), fiber
// tables, potential cache, Krylov vector work, small exponential, observables.
// The fiber contraction kernels live in ppq_hpsi.hip.
#include <algorithm>

#include "ppq_internal.hpp"

namespace ppq {

namespace {

constexpr int TB = 256;  // threads per block for streaming kernels
constexpr int PSTRIDE = 36;  // partial sums per block (Krylov values, adjoint parameters)
// Per-block partial sums are stored value-major, [value][block]: the one-block
// final reductions then read every value's partials as contiguous runs, one
// 1 KB line group per wavefront load, instead of one cache line per lane.
__device__ inline int64_t pidx(int64_t b, int i) { return (int64_t)i * RED_BLOCKS + b; }

__device__ inline int64_t gid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

inline unsigned nblocks(int64_t n, int tb = TB)
{
    int64_t b = (n + tb - 1) / tb;
    return (unsigned)(b < 1 ? 1 : b);
}

// complex product without contraction: (ac - bd) + i(ad + bc)
__device__ inline double2 cmul_rn(double2 a, double2 b)
{
    return make_double2(__dsub_rn(__dmul_rn(a.x, b.x), __dmul_rn(a.y, b.y)),
                        __dadd_rn(__dmul_rn(a.x, b.y), __dmul_rn(a.y, b.x)));
}

__device__ inline bool above_eps(double2 c, double eps2)
{
    return __dadd_rn(__dmul_rn(c.x, c.x), __dmul_rn(c.y, c.y)) >= eps2;
}

__device__ inline void set_bit(uint64_t *bm, uint32_t key)
{
    atomicOr((unsigned long long *)&bm[key >> 6], 1ull << (key & 63));
}

// Sets bit `key` for every lane with `valid`; all 64 lanes of the wavefront
// must call it together.  Lanes that target the same word are merged by a
// segmented OR across neighbouring lanes, so one atomic per run of lanes
// hitting one word is issued (sorted keys put most of a wavefront's targets
// in a few words).
__device__ inline void set_bit_wave(uint64_t *bm, uint32_t key, bool valid)
{
    const int lane = threadIdx.x & 63;
    uint32_t w = valid ? (key >> 6) : 0xffffffffu;
    uint64_t bits = valid ? (1ull << (key & 63)) : 0ull;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t ow = __shfl_up(w, d, 64);
        uint32_t olo = __shfl_up((uint32_t)bits, d, 64);
        uint32_t ohi = __shfl_up((uint32_t)(bits >> 32), d, 64);
        if (lane >= d && ow == w) bits |= ((uint64_t)ohi << 32) | olo;
    }
    uint32_t nw = __shfl_down(w, 1, 64);
    bool last = (lane == 63) || (nw != w);
    if (valid && last) atomicOr((unsigned long long *)&bm[w], (unsigned long long)bits);
}

// Phase-space axis `part` of dimension k for `key`: the grid index of a DVR
// dimension (part 0), or the cell (part 0) and level (part 1) index of a
// lattice dimension; its index, extent and key stride.
__device__ inline void phase_axis(const GridDesc &g, uint32_t key, int k, int part, int &idx, int &ext, int64_t &str)
{
    const int d = (int)((key / g.stride[k]) % (uint32_t)g.n[k]);
    if (g.lat_s[k] == 0) {
        idx = d;
        ext = g.n[k];
        str = g.stride[k];
    } else if (part == 0) {
        idx = d / g.lat_l[k];
        ext = g.lat_s[k];
        str = (int64_t)g.lat_l[k] * g.stride[k];
    } else {
        idx = d % g.lat_l[k];
        ext = g.lat_l[k];
        str = g.stride[k];
    }
}

// Marks `key` and its neighbours of the selected stencil for lanes with `keep`
// (wave-collective: every lane runs the same loop bounds, which depend on the
// grid alone).  The wider balls of Sec. III.A count index changes over the
// phase-space axes: one per DVR dimension, two (cell, level) per lattice one.
__device__ inline void set_with_neighbours(const GridDesc &g, uint64_t *bm, uint32_t key, bool keep)
{
    if (g.pairs == 2) {
        // ball radius 2: every combination of -1/0/+1 changes over the axes,
        // the key itself included; the combinations are counted in base 3,
        // one digit per axis.  A wavefront with nothing to keep skips them
        // (the test is uniform across its lanes, so the collective calls
        // stay in step).
        if (__ballot(keep) == 0) return;
        int naxes = 0;
        for (int k = 0; k < g.D; ++k) naxes += g.lat_s[k] ? 2 : 1;
        int ncomb = 1;
        for (int a = 0; a < naxes; ++a) ncomb *= 3;
        for (int cmb = 0; cmb < ncomb; ++cmb) {
            int rest = cmb;
            bool inside = keep;
            int64_t shift = 0;
            for (int k = 0; k < g.D; ++k) {
                for (int part = 0; part < (g.lat_s[k] ? 2 : 1); ++part) {
                    int idx, ext;
                    int64_t str;
                    phase_axis(g, key, k, part, idx, ext, str);
                    const int a = rest % 3 - 1;
                    rest /= 3;
                    inside = inside && idx + a >= 0 && idx + a < ext;
                    shift += a * str;
                }
            }
            set_bit_wave(bm, (uint32_t)((int64_t)key + shift), inside);
        }
        return;
    }
    set_bit_wave(bm, key, keep);
    for (int k = 0; k < g.D; ++k) {
        uint32_t sk = g.stride[k];
        int d = (int)((key / sk) % (uint32_t)g.n[k]);
        if (g.lat_s[k] == 0) {
            set_bit_wave(bm, key - sk, keep && d > 0);
            set_bit_wave(bm, key + sk, keep && d + 1 < g.n[k]);
        } else {
            int nl = g.lat_l[k];
            int si = d / nl, l = d % nl;
            set_bit_wave(bm, key - (uint32_t)nl * sk, keep && si > 0);
            set_bit_wave(bm, key + (uint32_t)nl * sk, keep && si + 1 < g.lat_s[k]);
            set_bit_wave(bm, key - sk, keep && l > 0);
            set_bit_wave(bm, key + sk, keep && l + 1 < nl);
        }
    }
    // ball radius sqrt(2): also every change of +-1 on two axes at once
    if (g.pairs == 1) {
        for (int k = 0; k < g.D; ++k) {
            for (int pk = 0; pk < (g.lat_s[k] ? 2 : 1); ++pk) {
                int ia, ea;
                int64_t sa;
                phase_axis(g, key, k, pk, ia, ea, sa);
                for (int l = k; l < g.D; ++l) {
                    for (int pl = (l == k ? pk + 1 : 0); pl < (g.lat_s[l] ? 2 : 1); ++pl) {
                        int ib, eb;
                        int64_t sb;
                        phase_axis(g, key, l, pl, ib, eb, sb);
                        const bool ad = ia > 0, au = ia + 1 < ea, bd = ib > 0, bu = ib + 1 < eb;
                        set_bit_wave(bm, (uint32_t)((int64_t)key - sa - sb), keep && ad && bd);
                        set_bit_wave(bm, (uint32_t)((int64_t)key - sa + sb), keep && ad && bu);
                        set_bit_wave(bm, (uint32_t)((int64_t)key + sa - sb), keep && au && bd);
                        set_bit_wave(bm, (uint32_t)((int64_t)key + sa + sb), keep && au && bu);
                    }
                }
            }
        }
    }
}

// Counts `pred` over the block and adds the block's total with one atomic
// (integer, so the sum is order-independent).  Block-collective.
__device__ inline void count_ballot(bool pred, unsigned long long *counter)
{
    __shared__ unsigned s_cnt;
    if (threadIdx.x == 0) s_cnt = 0u;
    __syncthreads();
    uint64_t b = __ballot(pred);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&s_cnt, (unsigned)__popcll(b));
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(counter, (unsigned long long)s_cnt);
}

// Counts `pred` over the block into block_counts[blockIdx.x] (a plain store:
// thousands of blocks adding to one address serialise).  Block-collective.
__device__ inline void count_block(bool pred, unsigned *block_counts)
{
    __shared__ unsigned s_cnt;
    if (threadIdx.x == 0) s_cnt = 0u;
    __syncthreads();
    uint64_t b = __ballot(pred);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&s_cnt, (unsigned)__popcll(b));
    __syncthreads();
    if (threadIdx.x == 0) block_counts[blockIdx.x] = s_cnt;
}

// *out = sum of nb block counts (one block, fixed order)
__global__ __launch_bounds__(1024) void k_sum_counts(const unsigned *bc, int64_t nb, unsigned long long *out)
{
    __shared__ unsigned long long s_part[16];
    unsigned long long c = 0;
    for (int64_t i = threadIdx.x; i < nb; i += 1024) c += bc[i];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < 16; ++i) t += s_part[i];
        *out = t;
    }
}

// ---- scan ------------------------------------------------------------------
constexpr int SB = 256;
constexpr int SI = 8;
constexpr int STILE = SB * SI;

__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[NT / 64];
    uint32_t inc = wave_incl_scan(v);
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        uint32_t s = wsum[i];
        if (i < w) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

struct PopLoad {
    const uint64_t *w;
    __device__ uint32_t operator()(int64_t i) const { return (uint32_t)__popcll(w[i]); }
};
struct U32Load {
    const uint32_t *a;
    __device__ uint32_t operator()(int64_t i) const { return a[i]; }
};

template <class L>
__global__ __launch_bounds__(SB) void k_scan_reduce(L ld, int64_t n, uint32_t *tile_sums)
{
    int64_t base = (int64_t)blockIdx.x * STILE;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        int64_t idx = base + (int64_t)i * SB + threadIdx.x;
        if (idx < n) s += ld(idx);
    }
    uint32_t tot;
    block_excl_scan<SB>(s, &tot);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t *tile, int64_t ntiles, uint32_t *total)
{
    int64_t per = (ntiles + 1023) / 1024;
    int64_t lo = threadIdx.x * per, hi = lo + per < ntiles ? lo + per : ntiles;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += tile[i];
    uint32_t tot;
    uint32_t off = block_excl_scan<1024>(s, &tot);
    for (int64_t i = lo; i < hi; ++i) {
        uint32_t v = tile[i];
        tile[i] = off;
        off += v;
    }
    if (threadIdx.x == 0) *total = tot;
}

// The tile's SI rows of SB consecutive elements, each row read and written by
// the whole block (coalesced): a wavefront scan per row and wave, then every
// thread adds the totals of the (row, wave) pieces before its own.
template <class L>
__global__ __launch_bounds__(SB) void k_scan_apply(L ld, int64_t n, const uint32_t *tile_off, uint32_t *out)
{
    constexpr int NW = SB / 64;
    __shared__ uint32_t wsum[SI * NW];
    const int64_t base = (int64_t)blockIdx.x * STILE + threadIdx.x;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t v[SI], inc[SI];
#pragma unroll
    for (int i = 0; i < SI; ++i) v[i] = (base + (int64_t)i * SB < n) ? ld(base + (int64_t)i * SB) : 0u;
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        inc[i] = wave_incl_scan(v[i]);
        if (lane == 63) wsum[i * NW + w] = inc[i];
    }
    __syncthreads();
    uint32_t off = tile_off[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SI; ++i) {
        uint32_t before = 0, row = 0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            const uint32_t t = wsum[i * NW + ww];
            before += ww < w ? t : 0u;
            row += t;
        }
        const int64_t idx = base + (int64_t)i * SB;
        if (idx < n) out[idx] = off + before + inc[i] - v[i];
        off += row;
    }
}

template <class L>
void scan_impl(L ld, int64_t n, uint32_t *out, uint32_t *total, uint32_t *tmp, hipStream_t s)
{
    int64_t ntiles = (n + STILE - 1) / STILE;
    if (ntiles < 1) ntiles = 1;
    hipLaunchKernelGGL(k_scan_reduce<L>, dim3((unsigned)ntiles), dim3(SB), 0, s, ld, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, ntiles, total);
    hipLaunchKernelGGL(k_scan_apply<L>, dim3((unsigned)ntiles), dim3(SB), 0, s, ld, n, tmp, out);
}

// ---- fills -----------------------------------------------------------------
template <class T>
__global__ void k_fill(T *p, int64_t n, T v)
{
    for (int64_t i = gid(); i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---- adaption ----------------------------------------------------------------
__global__ void k_init_flag(GridDesc g, const double2 *tabs, int nmax, double eps2, uint64_t *bm,
                            unsigned long long *nabove)
{
    // wave-uniform trip count: every lane runs every iteration
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < (int64_t)g.total;
         base += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = base + threadIdx.x;
        bool inside = i < (int64_t)g.total;
        uint32_t key = inside ? (uint32_t)i : 0u;
        double2 v = make_double2(1.0, 0.0);
        for (int k = 0; k < g.D; ++k) {
            int d = (int)((key / g.stride[k]) % (uint32_t)g.n[k]);
            v = cmul_rn(v, tabs[k * nmax + d]);
        }
        bool keep = inside && above_eps(v, eps2);
        set_with_neighbours(g, bm, key, keep);
        count_ballot(keep, nabove);
    }
}

__global__ void k_product_values(const uint32_t *keys, int64_t n, GridDesc g, const double2 *tabs, int nmax,
                                 double2 *out)
{
    int64_t p = gid();
    if (p >= n) return;
    uint32_t key = keys[p];
    double2 v = make_double2(1.0, 0.0);
    for (int k = 0; k < g.D; ++k) {
        int d = (int)((key / g.stride[k]) % (uint32_t)g.n[k]);
        v = cmul_rn(v, tabs[k * nmax + d]);
    }
    out[p] = v;
}

__global__ void k_dilate(const uint32_t *keys, const double2 *psi, int64_t n, GridDesc g, double eps2,
                         uint64_t *bm, unsigned *block_counts)
{
    int64_t p = gid();
    bool keep = false;
    uint32_t key = 0;
    if (p < n) {
        key = keys[p];
        keep = above_eps(psi[p], eps2);
    }
    set_with_neighbours(g, bm, key, keep);
    count_block(keep, block_counts);
}

// ---- word-parallel dilation (the +-1 stencil on DVR axes) ---------------------
__device__ inline int64_t i64min(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ inline int64_t i64max(int64_t a, int64_t b) { return a > b ? a : b; }

// bits [lo, hi) of a word (0 <= lo, hi <= 64)
__device__ inline uint64_t bit_range(int lo, int hi)
{
    if (hi <= lo) return 0ull;
    const uint64_t up = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
    return up & ~((1ull << lo) - 1ull);
}

// the 64 bits of K from bit b on (bits outside the nwords words read 0)
__device__ inline uint64_t bit_window(const uint64_t *K, int64_t nwords, int64_t b)
{
    const int64_t q = b >> 6;  // rounds down for negative b
    const int r = (int)(b & 63);
    const uint64_t lo = (q >= 0 && q < nwords) ? K[q] : 0ull;
    if (r == 0) return lo;
    const uint64_t hi = (q + 1 >= 0 && q + 1 < nwords) ? K[q + 1] : 0ull;
    return (lo >> r) | (hi << (64 - r));
}

// K: one bit per function above the threshold (and the block counts of them)
__global__ void k_mark_kept(const uint32_t *keys, const double2 *psi, int64_t n, double eps2, uint64_t *K,
                            unsigned *block_counts)
{
    int64_t p = gid();
    bool keep = false;
    uint32_t key = 0;
    if (p < n) {
        key = keys[p];
        keep = above_eps(psi[p], eps2);
    }
    set_bit_wave(K, key, keep);
    count_block(keep, block_counts);
}

// bm = K with every +-1 neighbour on one axis: the neighbours one stride s_k
// below are K read s_k bits earlier, kept where the key's digit k is not 0
// (one stride above: not n_k - 1).  With P = s_k n_k, digit k is 0 on the
// runs [m P, m P + s_k) and n_k - 1 on [(m + 1) P - s_k, (m + 1) P).  A
// wavefront takes DW_ITER rows of 64 consecutive words; each lane keeps, per
// dimension, the position of its word's first bit within the period and
// advances it by 64 words' worth per row (no division per word).  Every word
// is written, the grid's tail bits cleared.
constexpr int DW_ITER = 8;
__global__ void k_dilate_words(const uint64_t *K, int64_t nwords, GridDesc g, uint64_t *bm)
{
    const int lane = threadIdx.x & 63;
    const int64_t wbase = (gid() >> 6) * 64 * DW_ITER;
    if (wbase >= nwords) return;
    const int64_t w0 = wbase + lane;
    int64_t pos[MAXD], inc[MAXD];
#pragma unroll
    for (int k = 0; k < MAXD; ++k) {
        pos[k] = 0;
        inc[k] = 0;
        if (k < g.D) {
            const int64_t P = (int64_t)g.stride[k] * g.n[k];
            pos[k] = (w0 * 64) % P;
            inc[k] = (int64_t)(64 * 64) % P;
        }
    }
    for (int it = 0; it < DW_ITER; ++it) {
        const int64_t w = w0 + (int64_t)it * 64;
        if (w >= nwords) break;
        const int64_t a = w * 64;
        uint64_t acc = K[w];
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
            if (k < g.D) {
                const int64_t st = g.stride[k], P = st * g.n[k];
                uint64_t zm = 0ull, tm = 0ull;
                for (int64_t r0 = -pos[k]; r0 < 64; r0 += P) {
                    if (r0 + st > 0) zm |= bit_range((int)i64max(r0, 0), (int)i64min(r0 + st, 64));
                    const int64_t ts = r0 + P - st;
                    if (r0 + P > 0 && ts < 64) tm |= bit_range((int)i64max(ts, 0), (int)i64min(r0 + P, 64));
                }
                acc |= (bit_window(K, nwords, a - st) & ~zm) | (bit_window(K, nwords, a + st) & ~tm);
                pos[k] += inc[k];
                if (pos[k] >= P) pos[k] -= P;
            }
        }
        const int64_t tail = (int64_t)g.total - a;
        if (tail < 64) acc &= tail > 0 ? ((1ull << tail) - 1ull) : 0ull;
        bm[w] = acc;
    }
}

// Relative exclusion (Sec. II.E): counts the current functions whose bit the
// dilated set leaves clear, i.e. those adaption would drop (block counts).
__global__ void k_count_dropped(const uint32_t *keys, int64_t n, const uint64_t *bm, unsigned *block_counts)
{
    int64_t p = gid();
    bool drop = false;
    if (p < n) {
        uint32_t key = keys[p];
        drop = ((bm[key >> 6] >> (key & 63)) & 1ull) == 0ull;
    }
    count_block(drop, block_counts);
}

// Keeps every current function when no more than rel * n of them would be
// dropped: functions go only if more than that fraction goes.  The test reads
// one device value, so it is uniform over the grid.
__global__ void k_keep_all_if(const uint32_t *keys, int64_t n, uint64_t *bm, const unsigned long long *dropped,
                              double rel)
{
    if ((double)*dropped > rel * (double)n) return;
    int64_t p = gid();
    set_bit_wave(bm, p < n ? keys[p] : 0u, p < n);
}

__global__ void k_mark(const uint32_t *keys, int64_t n, uint64_t *bm)
{
    int64_t p = gid();
    if (p < n) set_bit(bm, keys[p]);
}

__global__ void k_compact(const uint64_t *bm, const uint32_t *prefix, int64_t nwords, uint32_t *keys_out)
{
    int64_t w = gid();
    if (w >= nwords) return;
    uint64_t word = bm[w];
    if (!word) return;
    uint32_t q = prefix[w];
    while (word) {
        int b = __ffsll((unsigned long long)word) - 1;
        keys_out[q++] = (uint32_t)(w * 64 + b);
        word &= word - 1;
    }
}

__global__ void k_remap(const uint32_t *okeys, const double2 *opsi, int64_t n_old, const uint64_t *bm,
                        const uint32_t *prefix, double2 *npsi)
{
    int64_t p = gid();
    if (p >= n_old) return;
    uint32_t key = okeys[p];
    uint64_t word = bm[key >> 6];
    uint32_t b = key & 63;
    if ((word >> b) & 1ull) {
        uint32_t q = prefix[key >> 6] + (uint32_t)__popcll(word & ((1ull << b) - 1ull));
        npsi[q] = opsi[p];
    }
}

// ---- fiber tables ------------------------------------------------------------
__global__ void k_last_flags(const uint32_t *keys, int64_t n, int nl, uint32_t *flags)
{
    int64_t p = gid();
    if (p >= n) return;
    flags[p] = (p == 0 || keys[p] / (uint32_t)nl != keys[p - 1] / (uint32_t)nl) ? 1u : 0u;
}

// info[p] = the digit, with the fiber-start flag in bit 7 (dimensions of at
// most 64 points); a longer dimension (up to 256 points) keeps the digit alone
__global__ void k_last_info(const uint32_t *keys, int64_t n, int nl, uint8_t *info)
{
    int64_t p = gid();
    if (p >= n) return;
    bool start = (p == 0 || keys[p] / (uint32_t)nl != keys[p - 1] / (uint32_t)nl);
    const uint32_t flag = (start && nl <= NMAX_MASK) ? 0x80u : 0u;
    info[p] = (uint8_t)((keys[p] % (uint32_t)nl) | flag);
}

// mask[0, *nf) = 0 (the fiber count is on the device)
__global__ void k_zero_masks(uint64_t *mask, const uint32_t *nf)
{
    const int64_t m = *nf;
    for (int64_t i = gid(); i < m; i += (int64_t)gridDim.x * blockDim.x) mask[i] = 0ull;
}

// One thread per point: the fiber start writes off; every point's digit bit
// is ORed over the wavefront's consecutive lanes of its fiber and the
// segment's last lane adds it to the (zeroed) mask, so a fiber costs one or
// two atomics however its points fall over the wavefronts.  A dimension
// longer than a mask word keeps no mask.
__global__ void k_last_fill(const uint32_t *keys, int64_t n, int nl, const uint32_t *flags, const uint32_t *fidx,
                            const uint32_t *nf, uint32_t *off, uint64_t *mask)
{
    const int64_t p = gid();
    const int lane = threadIdx.x & 63;
    if (p == 0) off[*nf] = (uint32_t)n;
    const bool valid = p < n;
    uint32_t f = 0xffffffffu;
    uint64_t bits = 0ull;
    if (valid) {
        const uint32_t st = flags[p];
        f = fidx[p] - (st ? 0u : 1u);  // fidx counts the starts before p
        if (st) off[f] = (uint32_t)p;
        if (nl <= NMAX_MASK) bits = 1ull << (keys[p] % (uint32_t)nl);
    }
    if (nl > NMAX_MASK) return;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t of = __shfl_up(f, d, 64);
        const uint32_t lo = __shfl_up((uint32_t)bits, d, 64), hi = __shfl_up((uint32_t)(bits >> 32), d, 64);
        if (lane >= d && of == f) bits |= ((uint64_t)hi << 32) | lo;
    }
    const uint32_t nxt = __shfl_down(f, 1, 64);
    if (valid && (lane == 63 || nxt != f)) atomicOr((unsigned long long *)&mask[f], (unsigned long long)bits);
}

__device__ inline uint32_t rotate_key(uint32_t key, uint32_t sk, uint32_t nk, uint32_t *dig)
{
    uint32_t hi = key / (sk * nk);
    uint32_t rem = key - hi * sk * nk;
    uint32_t d = rem / sk, lo = rem - d * sk;
    *dig = d;
    return (hi * sk + lo) * nk + d;
}

// bits [base, base+len) of the bitmap, len <= 64
__device__ inline uint64_t extract_bits(const uint64_t *bm, uint32_t base, int len)
{
    uint32_t w0 = base >> 6, sh = base & 63;
    uint64_t v = bm[w0] >> sh;
    if (sh != 0 && sh + (uint32_t)len > 64) v |= bm[w0 + 1] << (64 - sh);
    return len == 64 ? v : (v & ((1ull << len) - 1ull));
}

// Key of a point in the frame whose digit order is (inner digits, outer
// digits): with S_in the product of the inner sizes and N_out = total / S_in,
// the frame key is (key mod S_in) * N_out + key / S_in.  rin == 0 keeps the
// row-major frame.
__device__ inline uint32_t frame_key(uint32_t key, uint32_t rin, uint32_t rout)
{
    return rin ? (key % rin) * rout + key / rin : key;
}

__global__ void k_rot_set(const uint32_t *keys, int64_t n, uint32_t sk, uint32_t nk, uint32_t rin, uint32_t rout,
                          uint64_t *bm)
{
    int64_t p = gid();
    uint32_t d, rk = 0;
    if (p < n) rk = rotate_key(frame_key(keys[p], rin, rout), sk, nk, &d);
    set_bit_wave(bm, rk, p < n);
}

// q = rank of the point in the rotated order.  pi[q] receives map[p] (p when
// map is null); inv[p] = q when inv is given.  flags/tmpmask/info describe the
// fibers along the rotated (last) digit (info may be null).
__global__ void k_rot_rank(const uint32_t *keys, int64_t n, uint32_t sk, uint32_t nk, uint32_t rin, uint32_t rout,
                           const uint64_t *bm, const uint32_t *prefix, const uint32_t *map, uint32_t *pi,
                           uint32_t *inv, uint32_t *flags, uint64_t *tmpmask, uint8_t *info)
{
    int64_t p = gid();
    if (p >= n) return;
    uint32_t d;
    uint32_t rk = rotate_key(frame_key(keys[p], rin, rout), sk, nk, &d);
    uint64_t word = bm[rk >> 6];
    uint32_t q = prefix[rk >> 6] + (uint32_t)__popcll(word & ((1ull << (rk & 63)) - 1ull));
    pi[q] = map ? map[p] : (uint32_t)p;
    if (inv) inv[p] = q;
    if (nk > (uint32_t)NMAX_MASK) {
        // a dimension longer than a mask word: the entry starts a fiber when no
        // bit of its fiber lies below it; info keeps the digit alone
        bool start = true;
        for (uint32_t b = rk - d; b < rk && start; b = (b | 63u) + 1u) {
            const uint32_t e = (b | 63u) + 1u < rk ? (b | 63u) + 1u : rk;
            const uint64_t w = bm[b >> 6] >> (b & 63u);
            const uint32_t len = e - b;
            start = (len >= 64 ? w : (w & ((1ull << len) - 1ull))) == 0;
        }
        flags[q] = start ? 1u : 0u;
        if (info) info[q] = (uint8_t)d;
        return;
    }
    uint64_t m = extract_bits(bm, rk - d, (int)nk);
    bool start = (m & ((1ull << d) - 1ull)) == 0;
    flags[q] = start ? 1u : 0u;
    if (start) tmpmask[q] = m;
    if (info) info[q] = (uint8_t)(d | (start ? 0x80u : 0u));
}

// ---- fiber tables of every non-last dimension in one set of launches ----------
// The D-1 rotated bitmaps (digit k moved last, k < D-1) and the row-major
// bitmap of the set are concatenated, each nwords long.  Every bitmap holds
// exactly n bits (rotation permutes the keys), so one exclusive prefix over the
// concatenation gives bitmap k's ranks offset by k n, and one scan over the
// concatenated fiber-start flags gives dimension k's fiber numbers offset by
// the count of the earlier dimensions.
__global__ void k_rot_set_all(const uint32_t *keys, int64_t n, RotAll r, uint64_t *bm, uint64_t *occ)
{
    int64_t p = gid();
    const bool valid = p < n;
    const uint32_t key = valid ? keys[p] : 0u;
    for (int k = 0; k < r.nd; ++k) {
        uint32_t d, rk = 0;
        if (valid) rk = rotate_key(key, r.sk[k], r.nk[k], &d);
        set_bit_wave(bm + (int64_t)k * r.nwords, rk, valid);
        // the point's fiber slot (the rotated key without its last digit)
        set_bit_wave(occ + r.owoff[k], rk / r.nk[k], valid);
    }
    // segment nd: the row-major bitmap of the set itself (point positions)
    set_bit_wave(bm + (int64_t)r.nd * r.nwords, key, valid);
}

// The r-th (0-based) set bit of v (r < popcount(v)): six halving steps.
__device__ inline int select_bit(uint64_t v, int r)
{
    int pos = 0;
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) {
        const int c = __popcll(v & ((1ull << sh) - 1ull));
        if (r >= c) {
            r -= c;
            v >>= sh;
            pos += sh;
        }
    }
    return pos;
}

// Rank order gather: the rotated bitmaps are walked word by word, so the
// points of dimension k come out in rank order q and every table write is
// contiguous.  A wavefront takes 64 consecutive words of the concatenated
// rotated segments; their set bits are dealt out to the lanes 64 at a time
// (a dense word's bits spread over the wavefront instead of one lane).  For
// the bit of rotated key rk: q from the segment's prefix, the point's
// position p from the row-major segment (rank of the un-rotated key), the
// fiber start and mask from the n_k-bit window holding rk, and the fiber's
// number from the rank of its slot among the occupied ones.
__global__ __launch_bounds__(TB) void k_rank_gather(int64_t n, RotAll r, const uint64_t *bm, const uint32_t *prefix,
                                                    const uint64_t *occ, const uint32_t *oprefix, TabPtrs t)
{
    __shared__ uint64_t s_word[TB];
    __shared__ uint32_t s_off[TB];
    __shared__ uint32_t s_q0[TB];
    __shared__ uint32_t s_w[TB];
    const int lane = threadIdx.x & 63, wbase = threadIdx.x & ~63;
    const int64_t nw = (int64_t)r.nd * r.nwords;
    const int64_t w = (int64_t)blockIdx.x * TB + threadIdx.x;
    uint64_t word = 0;
    uint32_t q0 = 0;
    if (w < nw) {
        word = bm[w];
        const int k = (int)(w / r.nwords);
        q0 = prefix[w] - (uint32_t)((int64_t)k * n);
    }
    const uint32_t cnt = (uint32_t)__popcll(word);
    // exclusive prefix of the counts over the wavefront
    uint32_t incl = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    const uint32_t total = __shfl(incl, 63, 64);
    s_word[threadIdx.x] = word;
    s_off[threadIdx.x] = incl - cnt;
    s_q0[threadIdx.x] = q0;
    s_w[threadIdx.x] = (uint32_t)(w < nw ? w % r.nwords : 0);
    __syncthreads();
    const uint64_t *rowm = bm + nw;            // row-major segment
    const uint32_t *rowp = prefix + nw;
    const uint32_t rbase = (uint32_t)((int64_t)r.nd * n);
    for (uint32_t b0 = 0; b0 < total; b0 += 64) {
        const uint32_t b = b0 + lane;
        if (b >= total) break;
        // source lane: the last lane whose offset is <= b (offsets ascend)
        int lo = 0, hi = 63;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[wbase + mid] <= b) lo = mid;
            else hi = mid - 1;
        }
        const int src = wbase + lo;
        const int rr = (int)(b - s_off[src]);
        const uint64_t sw = s_word[src];
        const int pos = select_bit(sw, rr);
        const int64_t wg = (int64_t)blockIdx.x * TB + src;  // global word index
        const int k = (int)(wg / r.nwords);
        const uint32_t rk = s_w[src] * 64u + (uint32_t)pos;
        const uint32_t q = s_q0[src] + (uint32_t)rr;
        // un-rotate: rk = (hi * sk + lo) * nk + d  ->  key = (hi * nk + d) * sk + lo
        const uint32_t nk = r.nk[k], sk = r.sk[k];
        const uint32_t d = rk % nk, tq = rk / nk;
        const uint32_t khi = tq / sk, klo = tq - khi * sk;
        const uint32_t key = (khi * nk + d) * sk + klo;
        const uint32_t p = rowp[key >> 6] - rbase +
                           (uint32_t)__popcll(rowm[key >> 6] & ((1ull << (key & 63)) - 1ull));
        t.pi[k][q] = p;
        const uint64_t *seg = bm + (int64_t)k * r.nwords;
        const uint64_t m = extract_bits(seg, rk - d, (int)nk);
        if ((m & ((1ull << d) - 1ull)) == 0) {
            // the fiber's first point: its slot tq's rank among the occupied slots
            const int64_t o0 = r.owoff[k], ow = o0 + (tq >> 6);
            const uint32_t f = oprefix[ow] - oprefix[o0] + (uint32_t)__popcll(occ[ow] & ((1ull << (tq & 63)) - 1ull));
            t.off[k][f] = q;
            t.mask[k][f] = m;
        }
    }
}

// Per dimension: the fiber count (occupied slots) and the end sentinel
// off_k[nf_k] = n.  `total` is the occupancy scan's total over all dimensions.
__global__ void k_occ_counts(const uint32_t *oprefix, int64_t n, RotAll r, const uint32_t *total, TabPtrs t,
                             uint32_t *nf)
{
    const int k = threadIdx.x;
    if (k >= r.nd) return;
    const uint32_t b0 = oprefix[r.owoff[k]];
    const uint32_t b1 = (k + 1 < r.nd) ? oprefix[r.owoff[k + 1]] : *total;
    nf[k] = b1 - b0;
    t.off[k][b1 - b0] = (uint32_t)n;
}

// Chunks of whole blocks for the block-fused H*psi.  A block is a maximal run
// of frame positions with the same block id (key / S_in in the row-major frame,
// key mod S_in in the inner-first frame, both non-decreasing along the frame).
// Chunk t starts at the first block start at or after t * S, so every chunk
// holds whole blocks; chunk[nch] = n.  counters[0] counts the chunks longer
// than cap (their indices go to big), counters[1] is the longest chunk.
__device__ inline uint32_t block_id(const uint32_t *keys, const uint32_t *P, uint32_t r, uint32_t sin, int inner)
{
    uint32_t k = keys[P ? P[r] : r];
    return inner ? k % sin : k / sin;
}

__device__ uint32_t chunk_start(const uint32_t *keys, const uint32_t *P, uint32_t n, uint32_t sin, int inner,
                                uint64_t st)
{
    if (st >= n) return n;
    uint32_t r = (uint32_t)st;
    uint32_t id = block_id(keys, P, r, sin, inner);
    if (r == 0 || block_id(keys, P, r - 1, sin, inner) != id) return r;
    uint32_t lo = r + 1, hi = n;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (block_id(keys, P, mid, sin, inner) == id) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void k_chunks(const uint32_t *keys, const uint32_t *P, uint32_t n, uint32_t sin, int inner, uint32_t S,
                         uint32_t nch, uint32_t cap, uint32_t *chunk, uint32_t *big, uint32_t *counters)
{
    int64_t t = gid();
    if (t > nch) return;
    uint32_t a = chunk_start(keys, P, n, sin, inner, (uint64_t)t * S);
    chunk[t] = a;
    if (t == nch) return;
    uint32_t b = chunk_start(keys, P, n, sin, inner, (uint64_t)(t + 1) * S);
    uint32_t len = b - a;
    if (len > 0) atomicMax(&counters[1], len);
    if (len > cap) big[atomicAdd(&counters[0], 1u)] = (uint32_t)t;
}

// ---- plane tables (two adjacent dimensions merged into one digit) ------------
// q = the point's rank in the pair's frame (its own position in the identity
// frame, bm == nullptr); P[q] = p, the pair's two digits and the plane key
// (the frame key without the merged digit).
__global__ void k_plane_rank(const uint32_t *keys, int64_t n, uint32_t sk, uint32_t na, uint32_t nb,
                             const uint64_t *bm, const uint32_t *prefix, uint32_t *P, uint16_t *dig, uint32_t *pkey)
{
    int64_t p = gid();
    if (p >= n) return;
    const uint32_t nk = na * nb;
    uint32_t d;
    const uint32_t rk = rotate_key(keys[p], sk, nk, &d);
    uint32_t q = (uint32_t)p;
    if (bm) {
        q = prefix[rk >> 6] + (uint32_t)__popcll(bm[rk >> 6] & ((1ull << (rk & 63)) - 1ull));
        P[q] = (uint32_t)p;
    }
    dig[q] = (uint16_t)(((d / nb) << 8) | (d % nb));
    pkey[q] = rk / nk;
}

// Marks the last member of every plane (bit 15 of its digits).
__global__ void k_plane_flags(const uint32_t *pkey, int64_t n, uint32_t *flags, uint16_t *dig)
{
    int64_t q = gid();
    if (q >= n) return;
    const uint32_t k = pkey[q];
    flags[q] = (q == 0 || k != pkey[q - 1]) ? 1u : 0u;
    if (q == n - 1 || k != pkey[q + 1]) dig[q] = (uint16_t)(dig[q] | 0x8000u);
}

__global__ void k_plane_fill(const uint32_t *flags, const uint32_t *pidx, int64_t n, const uint32_t *np,
                             uint32_t *poff)
{
    int64_t q = gid();
    if (q == 0) poff[*np] = (uint32_t)n;
    if (q < n && flags[q]) poff[pidx[q]] = (uint32_t)q;
}

// Task t starts at the first plane start at or after t S (n for none):
// plane pl starts the tasks t with poff[pl - 1] < t S <= poff[pl].
__global__ void k_plane_tasks(const uint32_t *poff, const uint32_t *np, int64_t n, uint32_t S, uint32_t ntask,
                              uint32_t *tstart)
{
    int64_t pl = gid();
    const uint32_t npl = *np;
    if (pl > (int64_t)npl) return;
    const uint32_t lo = pl == 0 ? 0u : poff[pl - 1] / S + 1u;
    const uint32_t hi = pl == (int64_t)npl ? ntask : poff[pl] / S;
    const uint32_t st = pl == (int64_t)npl ? (uint32_t)n : poff[pl];
    for (uint32_t t = lo; t <= hi && t <= ntask; ++t) tstart[t] = st;
}

// Pair-pass tasks: task t starts at the first plane start at or after t W (n
// if none).  The plane holding position t W ends within nab positions, so one
// wavefront per task looks at positions [t W, t W + nab] only.
__global__ void k_pair_tasks(const uint32_t *keys, int64_t n, uint32_t nab, uint32_t W, uint32_t ntask,
                             uint32_t *tstart)
{
    const int64_t t = gid() >> 6;
    const int lane = threadIdx.x & 63;
    if (t > (int64_t)ntask) return;
    uint32_t st = (uint32_t)n;
    if (t < (int64_t)ntask) {
        const int64_t q0 = t * W, qe = q0 + (int64_t)nab < n - 1 ? q0 + (int64_t)nab : n - 1;
        for (int64_t b = q0; b <= qe; b += 64) {
            const int64_t q = b + lane;
            const bool start = q <= qe && (q == 0 || keys[q] / nab != keys[q - 1] / nab);
            const uint64_t m = __ballot(start);
            if (m) {
                st = (uint32_t)(b + __ffsll((unsigned long long)m) - 1);
                break;
            }
        }
    }
    if (lane == 0) tstart[t] = st;
}

__global__ void k_fib_fill(const uint32_t *flags, const uint32_t *fidx, const uint64_t *tmpmask, int64_t n,
                           const uint32_t *nf, uint32_t *off, uint64_t *mask)
{
    int64_t q = gid();
    if (q == 0) off[*nf] = (uint32_t)n;
    if (q >= n || !flags[q]) return;
    uint32_t f = fidx[q];
    off[f] = (uint32_t)q;
    if (mask) mask[f] = tmpmask[q];
}

// ---- potential cache -----------------------------------------------------------
// Potential cache: V_I = sum_t coef_t prod_f tab_{t,f}[digit_{dim_{t,f}}(I)].
// Term descriptors and the (deduplicated) 1D tables are staged in LDS.
constexpr int POT_MAX_TERMS = 256;
constexpr int POT_MAX_TAB = 2048;
constexpr int POT_MAX_FAC = 4;

__device__ inline int select_digit(const int (&d)[MAXD], int k)
{
    int r = d[0];
#pragma unroll
    for (int i = 1; i < MAXD; ++i) r = (k == i) ? d[i] : r;
    return r;
}

// Grid-stride over the points (or over a list of them): the term
// descriptors and tables are staged in LDS once per block.
__global__ __launch_bounds__(TB) void k_potential(const uint32_t *keys, int64_t n, GridDesc g, PotDesc pd, double *V,
                                                  float *Vf, const uint32_t *list, const unsigned *count)
{
    __shared__ double s_coef[POT_MAX_TERMS];
    __shared__ int s_nf[POT_MAX_TERMS];
    __shared__ int s_fac[POT_MAX_TERMS][POT_MAX_FAC];  // (table index << 4) | dim
    __shared__ double s_tab[POT_MAX_TAB];
    for (int t = threadIdx.x; t < pd.nterm; t += TB) {
        int ti[MAXD];
#pragma unroll
        for (int k = 0; k < MAXD; ++k) ti[k] = k < g.D ? pd.tab[t * pd.D + k] : -1;
        s_coef[t] = pd.coef[t];
        int nf = 0;
#pragma unroll
        for (int k = 0; k < MAXD; ++k)
            if (ti[k] >= 0 && nf < POT_MAX_FAC) s_fac[t][nf++] = (ti[k] << 4) | k;
        s_nf[t] = nf;
    }
    for (int i = threadIdx.x; i < pd.ntab * pd.nmax; i += TB) s_tab[i] = pd.tabs[i];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * TB;
    const int64_t m = list ? (int64_t)*count : n;
    for (int64_t i = gid(); i < m; i += stride) {
        const int64_t p = list ? (int64_t)list[i] : i;
        uint32_t key = keys[p];
        int d[MAXD];
#pragma unroll
        for (int k = 0; k < MAXD; ++k) d[k] = (k < g.D) ? (int)((key / g.stride[k]) % (uint32_t)g.n[k]) : 0;
        double v = 0.0;
        for (int t = 0; t < pd.nterm; ++t) {
            double f = s_coef[t];
            const int nf = s_nf[t];
#pragma unroll
            for (int j = 0; j < POT_MAX_FAC; ++j) {
                if (j < nf) {
                    int e = s_fac[t][j];
                    f *= s_tab[(e >> 4) * pd.nmax + select_digit(d, e & 15)];
                }
            }
            v += f;
        }
        if (V) V[p] = v;
        if (Vf) Vf[p] = (float)v;
    }
}

// Positions whose potential is missing (NaN) into list.  Each block takes a
// contiguous range: it counts, reserves its segment with one atomic (block
// segments in any order), then writes its positions in order.
template <class T>
__global__ __launch_bounds__(TB) void k_missing(const T *V, int64_t n, uint32_t *list, unsigned *count)
{
    __shared__ unsigned s_w[TB / 64];
    __shared__ unsigned s_base, s_run;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    unsigned c = 0;
    for (int64_t p = lo + threadIdx.x; p < hi; p += TB) c += (V[p] == V[p]) ? 0u : 1u;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if (lane == 0) s_w[w] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned tot = 0;
        for (int i = 0; i < TB / 64; ++i) tot += s_w[i];
        s_base = tot ? atomicAdd(count, tot) : 0u;
        s_run = 0u;
    }
    __syncthreads();
    for (int64_t p0 = lo; p0 < hi; p0 += TB) {
        const int64_t p = p0 + threadIdx.x;
        const bool miss = p < hi && !(V[p] == V[p]);
        const uint64_t b = __ballot(miss);
        if (lane == 0) s_w[w] = (unsigned)__popcll(b);
        __syncthreads();
        unsigned off = s_base + s_run;
        for (int i = 0; i < w; ++i) off += s_w[i];
        if (miss) list[off + (unsigned)__popcll(b & ((1ull << lane) - 1ull))] = (uint32_t)p;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int i = 0; i < TB / 64; ++i) s_run += s_w[i];
        __syncthreads();
    }
}

// ---- Krylov vectors ---------------------------------------------------------------
__device__ inline double2 ld2(const double2 *p, int64_t i) { return p[i]; }
__device__ inline double2 ld2(const float2 *p, int64_t i)
{
    float2 v = p[i];
    return make_double2((double)v.x, (double)v.y);
}
__device__ inline void st2(double2 *p, int64_t i, double2 v) { p[i] = v; }
__device__ inline void st2(float2 *p, int64_t i, double2 v) { p[i] = make_float2((float)v.x, (float)v.y); }
// Streaming forms for the Krylov basis: the sweeps and the recombination
// stream every earlier basis vector (more than the last-level cache holds),
// so their loads and the corrected vectors' stores carry the non-temporal
// hint and leave the cache to the product's tables and vectors.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
__device__ inline double2 ld2nt(const double2 *p, int64_t i)
{
    const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(p) + i);
    return make_double2(v.x, v.y);
}
__device__ inline double2 ld2nt(const float2 *p, int64_t i)
{
    const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2 *>(p) + i);
    return make_double2((double)v.x, (double)v.y);
}
__device__ inline void st2nt(double2 *p, int64_t i, double2 v)
{
    const nt_d2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_d2 *>(p) + i);
}
__device__ inline void st2nt(float2 *p, int64_t i, double2 v)
{
    const nt_f2 w = {(float)v.x, (float)v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_f2 *>(p) + i);
}
// the value a store of v into a C vector holds, without reading it back
__device__ inline double2 stored(const double2 *, double2 v) { return v; }
__device__ inline double2 stored(const float2 *, double2 v) { return make_double2((float)v.x, (float)v.y); }

// conj(a) * b accumulated
__device__ inline void cdot_acc(double2 &acc, double2 a, double2 b)
{
    acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}

template <int NV>
__device__ inline void block_reduce_store(double2 (&acc)[NV], double2 *partial)
{
    __shared__ double2 red[TB / 64][NV];
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double2 v = acc[i];
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            v.x += __shfl_xor(v.x, s, 64);
            v.y += __shfl_xor(v.y, s, 64);
        }
        if (lane == 0) red[w][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double2 s = red[0][threadIdx.x];
        for (int ww = 1; ww < TB / 64; ++ww) {
            s.x += red[ww][threadIdx.x].x;
            s.y += red[ww][threadIdx.x].y;
        }
        partial[pidx(blockIdx.x, threadIdx.x)] = s;
    }
}

// Final reduction of the per-block partials [value][block] by one block: every
// value at once, each thread a fixed subset of blocks, then a fixed tree
// (run-to-run deterministic); then the finaliser `mode` updates KState.
// (A separate launch: a device-scope fence per block to let the last block
// finish the sum would write back the L2 of every XCD.)
template <int NV>
__global__ __launch_bounds__(TB) void k_finalize(const double2 *partial, int nb, KState *ks, int j, int mode, int m,
                                                 int ioff, int nvals, double dt, double tol)
{
    if (mode != RED_NORM0 && j >= ks->meff) return;
    // the partials were just written from every XCD: issue all of this
    // thread's loads before summing them (blocks t, t + TB, ... in order)
    double2 tot[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) tot[i] = make_double2(0.0, 0.0);
    constexpr int PER = RED_BLOCKS / TB;
    static_assert(RED_BLOCKS % TB == 0, "partials per thread");
    if (nb == RED_BLOCKS) {
        double2 v[PER][NV];
#pragma unroll
        for (int u = 0; u < PER; ++u)
#pragma unroll
            for (int i = 0; i < NV; ++i) v[u][i] = partial[pidx(threadIdx.x + u * TB, i)];
#pragma unroll
        for (int u = 0; u < PER; ++u)
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                tot[i].x += v[u][i].x;
                tot[i].y += v[u][i].y;
            }
    } else {
        for (int b = threadIdx.x; b < nb; b += TB) {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                double2 v = partial[pidx(b, i)];
                tot[i].x += v.x;
                tot[i].y += v.y;
            }
        }
    }
    __shared__ double2 vals[TB / 64][NV];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double2 v = tot[i];
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            v.x += __shfl_xor(v.x, s, 64);
            v.y += __shfl_xor(v.y, s, 64);
        }
        if (lane == 0) vals[wv][i] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    // Every loop over r runs to the compile-time NV with a predicate: an index
    // known only at run time would put r in scratch memory.
    double2 r[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        r[i] = vals[0][i];
#pragma unroll
        for (int w2 = 1; w2 < TB / 64; ++w2) {
            r[i].x += vals[w2][i].x;
            r[i].y += vals[w2][i].y;
        }
    }
    if (mode == RED_NORM0) {
        ks->n0 = sqrt(r[0].x);
        ks->meff = m;
        ks->est = ks->n0;
        ks->kdt = fabs(dt);  // the estimate is a magnitude: |dt|^k
        ks->ktol = tol;
    } else if (mode == RED_H1) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if (i < nvals) {
                ks->h1[(i + ioff) * MAXM + j] = r[i];
                if (i + ioff == j) ks->alpha[j] = r[i].x;
            }
        }
    } else if (mode == RED_DELAY) {
        // The provisional q_j = beta_{j-1} v_j + sum_{i<j} h_i v_i with
        // h_i = h2[i][j-1] (the second pass's coefficients, not yet applied).
        // From mu = <q_j|H q_j>, using H v_i = beta_i v_{i+1} + alpha_i v_i +
        // beta_{i-1} v_{i-1} for i < j (all terms beyond O(h^2) kept):
        //   g_i = <v_i|H q_j> = beta_i <v_{i+1}|q_j> + alpha_i h_i + beta_{i-1} h_{i-1}
        //   alpha_j = (mu - 2 Re sum conj(h_i) g_i + sum conj(h_i) T_ik h_k) / beta_{j-1}^2
        //   cc_k = sum_{i<j} T_ki h_i  (k <= j), so H v_j = (H q_j - sum cc_k v_k) / beta_{j-1}
        // (the step's scalars are loaded at once and cc is summed in registers:
        // loops run to MAXM with a predicate, so nothing goes to scratch)
        const double2 mu = r[0];
        double2 cc[MAXM];
#pragma unroll
        for (int k = 0; k < MAXM; ++k) cc[k] = make_double2(0.0, 0.0);
        if (j == 0) {
            ks->alpha[0] = mu.x;
            ks->inv_b = 1.0;
        } else {
            const double b = ks->beta[j - 1];
            const double2 *hh = ks->h2 + (j - 1);  // hh[i * MAXM] = h_i
            double2 h[MAXM];
            double al[MAXM], be[MAXM];
#pragma unroll
            for (int i = 0; i < MAXM; ++i) {
                h[i] = i < j ? hh[i * MAXM] : make_double2(0.0, 0.0);
                al[i] = i < j ? ks->alpha[i] : 0.0;
                be[i] = i < j ? ks->beta[i] : 0.0;
            }
            double s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int i = 0; i < MAXM; ++i) {
                if (i < j) {
                    const double2 hi = h[i];
                    const double2 hn = (i + 1 < j) ? h[(i + 1) % MAXM] : make_double2(b, 0.0);
                    const double2 hp = (i >= 1) ? h[(i + MAXM - 1) % MAXM] : make_double2(0.0, 0.0);
                    const double bp = (i >= 1) ? be[(i + MAXM - 1) % MAXM] : 0.0;
                    const double2 g = make_double2(be[i] * hn.x + al[i] * hi.x + bp * hp.x,
                                                   be[i] * hn.y + al[i] * hi.y + bp * hp.y);
                    s1 += hi.x * g.x + hi.y * g.y;  // Re(conj(h_i) g_i)
                    s2 += al[i] * (hi.x * hi.x + hi.y * hi.y);
                    if (i + 1 < j) s2 += 2.0 * be[i] * (hi.x * hn.x + hi.y * hn.y);
                    // cc_k = alpha_k h_k + beta_k h_{k+1} + beta_{k-1} h_{k-1}, gathered per h_i
                    cc[i].x += al[i] * hi.x;
                    cc[i].y += al[i] * hi.y;
                    if (i + 1 < MAXM) {
                        cc[(i + 1) % MAXM].x += be[i] * hi.x;
                        cc[(i + 1) % MAXM].y += be[i] * hi.y;
                    }
                    if (i >= 1) {
                        cc[(i + MAXM - 1) % MAXM].x += bp * hi.x;
                        cc[(i + MAXM - 1) % MAXM].y += bp * hi.y;
                    }
                }
            }
            ks->alpha[j] = (mu.x - 2.0 * s1 + s2) / (b * b);
            ks->inv_b = 1.0 / b;
        }
#pragma unroll
        for (int k = 0; k < MAXM; ++k) ks->cc[k] = cc[k];
    } else if (mode == RED_ADELAY) {
        // Arnoldi: q_j = beta_{j-1} v_j + sum_{i<j} h_i v_i (h_i = h2[i][j-1]);
        // H v_i = sum_{k<=i+1} H_ki v_k with H_ki = h1 + h2 (k <= i), beta_i (k = i+1):
        //   cc_k = sum_{i<j} H_ki h_i, so H v_j = (z - sum_{k<=j} cc_k v_k) / beta_{j-1}
        //   <v_j|z> = (<q_j|z> - sum_{i<j} conj(h_i) <v_i|z>) / beta_{j-1}
        //   h1_ij = <v_i|H v_j> = (<v_i|z> - cc_i) / beta_{j-1}   (i <= j)
        // column j's second-pass terms come from this step's sweep (RED_BETA);
        // a step's last column keeps only its first pass
        // (cc is summed in registers; loops run to MAXM with a predicate)
        double2 cc[MAXM];
#pragma unroll
        for (int k = 0; k < MAXM; ++k) {
            cc[k] = make_double2(0.0, 0.0);
            ks->h2[k * MAXM + j] = make_double2(0.0, 0.0);
        }
        if (j == 0) {
            ks->h1[0] = r[0];
            ks->alpha[0] = r[0].x;
            ks->inv_b = 1.0;
        } else {
            const double b = ks->beta[j - 1], ib = 1.0 / b;
            const double2 *hh = ks->h2 + (j - 1);
#pragma unroll
            for (int i = 0; i < MAXM; ++i) {
                if (i < j) {
                    const double2 hi = hh[i * MAXM];
#pragma unroll
                    for (int k = 0; k <= i; ++k) {
                        const double2 a1 = ks->h1[k * MAXM + i], a2 = ks->h2[k * MAXM + i];
                        const double2 hk = make_double2(a1.x + a2.x, a1.y + a2.y);
                        cc[k].x += hk.x * hi.x - hk.y * hi.y;
                        cc[k].y += hk.x * hi.y + hk.y * hi.x;
                    }
                    if (i + 1 < MAXM) {
                        const double bi = ks->beta[i];
                        cc[(i + 1) % MAXM].x += bi * hi.x;
                        cc[(i + 1) % MAXM].y += bi * hi.y;
                    }
                }
            }
            // <v_j|z>, r[i] = <v_i|z> for i < j, r[j] = <q_j|z> (loops to NV with a predicate)
            double2 vz = make_double2(0.0, 0.0);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                if (i < j) {
                    const double2 hi = hh[i * MAXM];
                    vz.x += hi.x * r[i].x + hi.y * r[i].y;  // conj(h_i) r_i
                    vz.y += hi.x * r[i].y - hi.y * r[i].x;
                } else if (i == j) {
                    vz = make_double2((r[i].x - vz.x) * ib, (r[i].y - vz.y) * ib);
                }
            }
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                if (i < j) {
                    ks->h1[i * MAXM + j] = make_double2((r[i].x - cc[i % MAXM].x) * ib, (r[i].y - cc[i % MAXM].y) * ib);
                } else if (i == j) {
                    const double2 g = make_double2((vz.x - cc[i % MAXM].x) * ib, (vz.y - cc[i % MAXM].y) * ib);
                    ks->h1[j * MAXM + j] = g;
                    ks->alpha[j] = g.x;
                }
            }
            ks->inv_b = ib;
        }
#pragma unroll
        for (int k = 0; k < MAXM; ++k) ks->cc[k] = cc[k];
    } else {  // RED_BETA: h2[.][j] and beta_j from |q_{j+1}|^2 - sum |h2_i|^2
        const int nh = nvals - 1;
        double hh = 0.0, last = 0.0;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if (i < nh) {
                ks->h2[i * MAXM + j] = r[i];
                hh += r[i].x * r[i].x + r[i].y * r[i].y;
            } else if (i == nh) {
                last = r[i].x;
            }
        }
        double b2 = last - hh;
        double b = sqrt(b2 > 0.0 ? b2 : 0.0);
        ks->beta[j] = b;
        if (j < m - 1) {
            if (b < 1e-13) {
                ks->meff = j + 1;
            } else {
                // Park and Light's estimate of the order-(j+1) step: the
                // first Taylor term the Krylov space leaves out; with a
                // tolerance, the step stops at the first order within it
                const double est = ks->est * ks->kdt * b / (double)(j + 1);
                ks->est = est;
                if (ks->ktol > 0.0 && est <= ks->ktol) ks->meff = j + 1;
            }
        }
    }
}

template <class C>
__global__ __launch_bounds__(TB) void k_norm0(const double2 *psi, int64_t n, double2 *partial, unsigned *counter,
                                              KState *ks, int m)
{
    double2 acc[1] = {make_double2(0.0, 0.0)};
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * TB) {
        double2 a = psi[p];
        acc[0].x = fma(a.x, a.x, fma(a.y, a.y, acc[0].x));
    }
    block_reduce_store<1>(acc, partial);
}

template <class C, int NV>
__global__ __launch_bounds__(TB) void k_cgs_dots(const C *Vb, int64_t ld, const C *w, int64_t n, double2 *partial,
                                                 unsigned *counter, KState *ks, int j, int m, int ioff)
{
    if (j >= ks->meff) return;
    double2 acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * TB) {
        double2 wv = ld2(w, p);
#pragma unroll
        for (int i = 0; i < NV; ++i) cdot_acc(acc[i], ld2(Vb, (int64_t)i * ld + p), wv);
    }
    block_reduce_store<NV>(acc, partial);
}

// Hermitian Lanczos step j with the second Gram-Schmidt pass of each vector
// delayed to the next step's sweep.  Slot j holds the provisional
// q_j = beta_{j-1} v_j + sum_{i<j} h_i v_i (first pass only, unnormalised) and
// z = H q_j; with h_i = h2[i][j-1] and alpha_j, cc from RED_DELAY, one pass
//   v_j     = (q_j - sum_{i<j} h_i v_i) / beta_{j-1}           -> slot j
//   H v_j   = (z - sum_{k<j} cc_k v_k - cc_j v_j) / beta_{j-1}
//   q_{j+1} = H v_j - alpha_j v_j - beta_{j-1} v_{j-1}          -> slot j+1
// with the partial sums of <v_i|q_{j+1}> (i <= j) and |q_{j+1}|^2: the next
// second pass's coefficients and, after RED_BETA, beta_j.  In exact arithmetic
// h = 0 and this is the three-term recurrence; with rounding it applies the
// same second projection as two separate sweeps would, one step later.
template <class C, int NV>
__global__ __launch_bounds__(TB) void k_lanczos_sweep(C *Vb, int64_t ld, const C *z, int64_t n, double2 *partial,
                                                      unsigned *counter, KState *ks, int j)
{
    if (j >= ks->meff) return;
    constexpr int NH = NV > 0 ? NV : 1;
    double2 hq[NH], cc[NV + 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) hq[i] = ks->h2[i * MAXM + (j - 1)];
#pragma unroll
    for (int k = 0; k <= NV; ++k) cc[k] = ks->cc[k];
    const double ib = ks->inv_b, al = ks->alpha[j], bm = NV > 0 ? ks->beta[j - 1] : 0.0;
    C *qs = Vb + (int64_t)j * ld;
    C *qn = Vb + (int64_t)(j + 1) * ld;
    double2 acc[NV + 2];
#pragma unroll
    for (int i = 0; i < NV + 2; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * TB) {
        double2 qv = ld2nt(qs, p), hv = ld2nt(z, p);
        double2 vv[NH];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            vv[i] = ld2nt(Vb, (int64_t)i * ld + p);
            qv.x -= hq[i].x * vv[i].x - hq[i].y * vv[i].y;
            qv.y -= hq[i].x * vv[i].y + hq[i].y * vv[i].x;
            hv.x -= cc[i].x * vv[i].x - cc[i].y * vv[i].y;
            hv.y -= cc[i].x * vv[i].y + cc[i].y * vv[i].x;
        }
        st2nt(qs, p, make_double2(qv.x * ib, qv.y * ib));
        const double2 vj = stored(qs, make_double2(qv.x * ib, qv.y * ib));
        hv.x -= cc[NV].x * vj.x - cc[NV].y * vj.y;
        hv.y -= cc[NV].x * vj.y + cc[NV].y * vj.x;
        double2 wp = make_double2(hv.x * ib - al * vj.x, hv.y * ib - al * vj.y);
        if (NV > 0) {
            wp.x -= bm * vv[NV - 1].x;
            wp.y -= bm * vv[NV - 1].y;
        }
        st2(qn, p, wp);
        const double2 ws = stored(qn, wp);
#pragma unroll
        for (int i = 0; i < NV; ++i) cdot_acc(acc[i], vv[i], ws);
        cdot_acc(acc[NV], vj, ws);
        acc[NV + 1].x = fma(ws.x, ws.x, fma(ws.y, ws.y, acc[NV + 1].x));
    }
    block_reduce_store<NV + 2>(acc, partial);
}

// Arnoldi step j, first reduction: <v_i|z> for i < j and <q_j|z> (slot j
// holds the provisional q_j, z = H q_j).
template <class C, int NV>
__global__ __launch_bounds__(TB) void k_arnoldi_dots(const C *Vb, int64_t ld, const C *z, int64_t n,
                                                     double2 *partial, unsigned *counter, KState *ks, int j)
{
    if (j >= ks->meff) return;
    const C *qs = Vb + (int64_t)j * ld;
    double2 acc[NV + 1];
#pragma unroll
    for (int i = 0; i <= NV; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * TB) {
        const double2 zv = ld2(z, p);
#pragma unroll
        for (int i = 0; i < NV; ++i) cdot_acc(acc[i], ld2nt(Vb, (int64_t)i * ld + p), zv);
        cdot_acc(acc[NV], ld2(qs, p), zv);
    }
    block_reduce_store<NV + 1>(acc, partial);
}

// Arnoldi step j, the sweep: with h_i = h2[i][j-1], cc, inv_b and the
// first-pass column h1[.][j] from RED_ADELAY,
//   v_j     = (q_j - sum_{i<j} h_i v_i) / beta_{j-1}           -> slot j
//   H v_j   = (z - sum_{k<=j} cc_k v_k) / beta_{j-1}
//   q_{j+1} = H v_j - sum_{i<=j} h1_ij v_i                       -> slot j+1
// and the partial sums of <v_i|q_{j+1}> (i <= j) and |q_{j+1}|^2.
template <class C, int NV>
__global__ __launch_bounds__(TB) void k_arnoldi_sweep(C *Vb, int64_t ld, const C *z, int64_t n, double2 *partial,
                                                      unsigned *counter, KState *ks, int j)
{
    if (j >= ks->meff) return;
    constexpr int NH = NV > 0 ? NV : 1;
    double2 hq[NH], cc[NV + 1], g1[NV + 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) hq[i] = ks->h2[i * MAXM + (j - 1)];
#pragma unroll
    for (int k = 0; k <= NV; ++k) {
        cc[k] = ks->cc[k];
        g1[k] = ks->h1[k * MAXM + j];
    }
    const double ib = ks->inv_b;
    C *qs = Vb + (int64_t)j * ld;
    C *qn = Vb + (int64_t)(j + 1) * ld;
    double2 acc[NV + 2];
#pragma unroll
    for (int i = 0; i < NV + 2; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * TB) {
        double2 qv = ld2nt(qs, p), hv = ld2nt(z, p);
        double2 vv[NH];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            vv[i] = ld2nt(Vb, (int64_t)i * ld + p);
            qv.x -= hq[i].x * vv[i].x - hq[i].y * vv[i].y;
            qv.y -= hq[i].x * vv[i].y + hq[i].y * vv[i].x;
            hv.x -= cc[i].x * vv[i].x - cc[i].y * vv[i].y;
            hv.y -= cc[i].x * vv[i].y + cc[i].y * vv[i].x;
        }
        st2nt(qs, p, make_double2(qv.x * ib, qv.y * ib));
        const double2 vj = stored(qs, make_double2(qv.x * ib, qv.y * ib));
        hv.x -= cc[NV].x * vj.x - cc[NV].y * vj.y;
        hv.y -= cc[NV].x * vj.y + cc[NV].y * vj.x;
        double2 wp = make_double2(hv.x * ib, hv.y * ib);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            wp.x -= g1[i].x * vv[i].x - g1[i].y * vv[i].y;
            wp.y -= g1[i].x * vv[i].y + g1[i].y * vv[i].x;
        }
        wp.x -= g1[NV].x * vj.x - g1[NV].y * vj.y;
        wp.y -= g1[NV].x * vj.y + g1[NV].y * vj.x;
        st2(qn, p, wp);
        const double2 ws = stored(qn, wp);
#pragma unroll
        for (int i = 0; i < NV; ++i) cdot_acc(acc[i], vv[i], ws);
        cdot_acc(acc[NV], vj, ws);
        acc[NV + 1].x = fma(ws.x, ws.x, fma(ws.y, ws.y, acc[NV + 1].x));
    }
    block_reduce_store<NV + 2>(acc, partial);
}

// v_j = (q_j - sum_{i<j} h_i v_i) / beta_{j-1} in slot j: the last vector of a
// step that ran to its full order (no later sweep corrects it).
template <class C, int NV>
__global__ __launch_bounds__(TB) void k_lanczos_fix(C *Vb, int64_t ld, int64_t n, const KState *ks, int j)
{
    if (j >= ks->meff) return;
    double2 hq[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) hq[i] = ks->h2[i * MAXM + (j - 1)];
    const double ib = ks->inv_b;
    C *qs = Vb + (int64_t)j * ld;
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * TB) {
        double2 qv = ld2(qs, p);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double2 v = ld2nt(Vb, (int64_t)i * ld + p);
            qv.x -= hq[i].x * v.x - hq[i].y * v.y;
            qv.y -= hq[i].x * v.y + hq[i].y * v.x;
        }
        st2(qs, p, make_double2(qv.x * ib, qv.y * ib));
    }
}

// A step that ran to its full order m leaves its last vector provisional:
// v_L = (q_L - sum_{i<L} h_i v_i) / beta_{L-1}, L = m - 1.  The propagated
// vector sum_k y_k v_k is then sum_{k<L} (y_k - y_L h_k / beta_{L-1}) v_k +
// (y_L / beta_{L-1}) q_L: the coefficients absorb the correction.
__global__ void k_lanczos_coef(KState *ks, int m)
{
    if (threadIdx.x != 0 || ks->meff != m || m < 2) return;
    const int L = m - 1;
    const double2 yl = ks->y[L];
    const double ib = ks->inv_b;
    for (int k = 0; k < L; ++k) {
        const double2 h = ks->h2[k * MAXM + (L - 1)];
        ks->y[k].x -= ib * (yl.x * h.x - yl.y * h.y);
        ks->y[k].y -= ib * (yl.x * h.y + yl.y * h.x);
    }
    ks->y[L] = make_double2(yl.x * ib, yl.y * ib);
}

template <class C>
__global__ void k_normalise(const double2 *psi, int64_t n, const KState *ks, C *v0)
{
    double s = 1.0 / ks->n0;
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * blockDim.x) {
        double2 a = ld2nt(psi, p);
        st2(v0, p, make_double2(a.x * s, a.y * s));
    }
}

template <class C>
__global__ void k_lincomb(const C *Vb, int64_t ld, const double2 *psi_master, int64_t n, const KState *ks,
                          double2 *out)
{
    int meff = ks->meff;
    double2 y[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) y[i] = ks->y[i];
    double inv_n0 = 1.0 / ks->n0;
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * blockDim.x) {
        // j = 0 from the FP64 master copy (exact v_0 direction, its last use), j >= 1 from the basis
        double2 v = ld2nt(psi_master, p);
        v.x *= inv_n0;
        v.y *= inv_n0;
        double2 acc = make_double2(y[0].x * v.x - y[0].y * v.y, y[0].x * v.y + y[0].y * v.x);
#pragma unroll
        for (int i = 1; i < MAXM; ++i) {
            if (i < meff) {
                double2 b = ld2nt(Vb, (int64_t)i * ld + p);
                acc.x += y[i].x * b.x - y[i].y * b.y;
                acc.y += y[i].x * b.y + y[i].y * b.x;
            }
        }
        out[p] = acc;
    }
}

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// y = n0 * exp(-i dt Hk) e_1 for the meff x meff Krylov matrix, by scaling and
// squaring of a truncated Taylor series; one workgroup of 256 lanes, lane
// (r, c) owns entry (r, c) of the 16 x 16 matrices.
__global__ __launch_bounds__(256) void k_krylov_expv(KState *ks, double dt, int hermitian)
{
    __shared__ double2 A[MAXM][MAXM], P[MAXM][MAXM], E[MAXM][MAXM];
    __shared__ double rown[MAXM];
    __shared__ int s_sq;
    int meff = ks->meff;
    int r = threadIdx.x / MAXM, c = threadIdx.x % MAXM;
    double2 h = make_double2(0.0, 0.0);
    if (r < meff && c < meff) {
        if (hermitian) {
            if (r == c) h = make_double2(ks->alpha[r], 0.0);
            else if (r == c + 1) h = make_double2(ks->beta[c], 0.0);
            else if (c == r + 1) h = make_double2(ks->beta[r], 0.0);
        } else {
            if (r <= c) {
                double2 a = ks->h1[r * MAXM + c], b = ks->h2[r * MAXM + c];
                h = make_double2(a.x + b.x, a.y + b.y);
            } else if (r == c + 1) {
                h = make_double2(ks->beta[c], 0.0);
            }
        }
    }
    // A = -i dt H
    A[r][c] = make_double2(dt * h.y, -dt * h.x);
    __syncthreads();
    if (threadIdx.x < MAXM) {
        double s = 0.0;
        for (int cc = 0; cc < MAXM; ++cc)
            s += sqrt(A[threadIdx.x][cc].x * A[threadIdx.x][cc].x + A[threadIdx.x][cc].y * A[threadIdx.x][cc].y);
        rown[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double nrm = 0.0;
        for (int i = 0; i < MAXM; ++i) nrm = rown[i] > nrm ? rown[i] : nrm;
        int sq = 0;
        while (nrm > 0.125) {
            nrm *= 0.5;
            ++sq;
        }
        s_sq = sq;
    }
    __syncthreads();
    int sq = s_sq;
    double scale = ldexp(1.0, -sq);
    A[r][c] = make_double2(A[r][c].x * scale, A[r][c].y * scale);
    P[r][c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    E[r][c] = P[r][c];
    __syncthreads();
    for (int kt = 1; kt <= 18; ++kt) {
        double2 acc = make_double2(0.0, 0.0);
        for (int l = 0; l < MAXM; ++l) {
            double2 t = cmul(P[r][l], A[l][c]);
            acc.x += t.x;
            acc.y += t.y;
        }
        __syncthreads();
        P[r][c] = make_double2(acc.x / kt, acc.y / kt);
        E[r][c] = make_double2(E[r][c].x + acc.x / kt, E[r][c].y + acc.y / kt);
        __syncthreads();
    }
    for (int q = 0; q < sq; ++q) {
        double2 acc = make_double2(0.0, 0.0);
        for (int l = 0; l < MAXM; ++l) {
            double2 t = cmul(E[r][l], E[l][c]);
            acc.x += t.x;
            acc.y += t.y;
        }
        __syncthreads();
        E[r][c] = acc;
        __syncthreads();
    }
    if (c == 0 && r < MAXM) {
        double n0 = ks->n0;
        ks->y[r] = (r < meff) ? make_double2(n0 * E[r][0].x, n0 * E[r][0].y) : make_double2(0.0, 0.0);
    }
}

__global__ __launch_bounds__(TB) void k_dot_partial(const double2 *a, const double2 *b, int64_t n,
                                                    double2 *partial)
{
    double2 acc[1] = {make_double2(0.0, 0.0)};
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * TB) cdot_acc(acc[0], a[p], b[p]);
    block_reduce_store<1>(acc, partial);
}

// ---- autocorrelation at twice the time --------------------------------------------
// sum_I c_I^2 (no conjugate): C(2t) = <psi(t)*|psi(t)> when the initial packet
// is real and the operator real symmetric (Eq. acorr and the text after it).
__global__ __launch_bounds__(TB) void k_sq_partial(const double2 *psi, int64_t n, double2 *partial)
{
    double2 acc[1] = {make_double2(0.0, 0.0)};
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * TB) {
        const double2 c = psi[p];
        acc[0].x = fma(c.x, c.x, fma(-c.y, c.y, acc[0].x));
        acc[0].y = fma(2.0 * c.x, c.y, acc[0].y);
    }
    block_reduce_store<1>(acc, partial);
}

// fixed-order sum of the first partial of nb blocks into *out
__global__ __launch_bounds__(TB) void k_sum_partial1(const double2 *partial, int nb, double2 *out)
{
    __shared__ double2 red[TB];
    double2 s = make_double2(0.0, 0.0);
    for (int b = threadIdx.x; b < nb; b += TB) {
        s.x += partial[pidx(b, 0)].x;
        s.y += partial[pidx(b, 0)].y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = TB / 2; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) {
            red[threadIdx.x].x += red[threadIdx.x + st].x;
            red[threadIdx.x].y += red[threadIdx.x + st].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// ---- observables ------------------------------------------------------------------
__global__ __launch_bounds__(TB) void k_obs_partial(const uint32_t *keys, const double2 *psi, int64_t n, GridDesc g,
                                                    const double2 *bra, int nmax, double eps2, double2 *partial)
{
    // the 1D tables of the reference packet (at most MAXD x 64 entries) in LDS
    __shared__ double2 sbra[MAXD * NMAX_FIBER];
    for (int i = threadIdx.x; i < g.D * nmax; i += TB) sbra[i] = bra[i];
    __syncthreads();
    double2 acc[3] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    // OBS_U points per thread and pass, every load issued before the first
    // use (one memory latency per pass instead of one per point)
    constexpr int OBS_U = 4;
    const int64_t stride = (int64_t)gridDim.x * TB;
    for (int64_t p0 = gid(); p0 < n; p0 += stride * OBS_U) {
        double2 c[OBS_U];
        uint32_t key[OBS_U];
#pragma unroll
        for (int u = 0; u < OBS_U; ++u) {
            const int64_t p = p0 + u * stride;
            c[u] = p < n ? psi[p] : make_double2(0.0, 0.0);
            key[u] = p < n ? keys[p] : 0u;
        }
        double2 v[OBS_U];
#pragma unroll
        for (int u = 0; u < OBS_U; ++u) v[u] = make_double2(1.0, 0.0);
        for (int k = 0; k < g.D; ++k) {
#pragma unroll
            for (int u = 0; u < OBS_U; ++u) {
                const int d = (int)((key[u] / g.stride[k]) % (uint32_t)g.n[k]);
                v[u] = cmul(v[u], sbra[k * nmax + d]);
            }
        }
#pragma unroll
        for (int u = 0; u < OBS_U; ++u) {
            if (p0 + u * stride >= n) continue;
            acc[0].x = fma(c[u].x, c[u].x, fma(c[u].y, c[u].y, acc[0].x));
            cdot_acc(acc[1], v[u], c[u]);
            if (above_eps(c[u], eps2)) acc[2].x += 1.0;
        }
    }
    block_reduce_store<3>(acc, partial);
}

__global__ __launch_bounds__(TB) void k_obs_final(const double2 *partial, int nb, double *rec)
{
    __shared__ double2 red[TB];
    for (int i = 0; i < 3; ++i) {
        double2 s = make_double2(0.0, 0.0);
        for (int b = threadIdx.x; b < nb; b += TB) {
            s.x += partial[pidx(b, i)].x;
            s.y += partial[pidx(b, i)].y;
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int st = TB / 2; st >= 1; st >>= 1) {
            if ((int)threadIdx.x < st) {
                red[threadIdx.x].x += red[threadIdx.x + st].x;
                red[threadIdx.x].y += red[threadIdx.x + st].y;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (i == 0) rec[PPQ_OBS_NORM2] = red[0].x;
            if (i == 1) {
                rec[PPQ_OBS_ACF_RE] = red[0].x;
                rec[PPQ_OBS_ACF_IM] = red[0].y;
            }
            if (i == 2) rec[PPQ_OBS_NABOVE] = red[0].x;
        }
        __syncthreads();
    }
}

// ---- position expectations ---------------------------------------------------------
// Per block: sum |c|^2 and, per dimension, sum |c|^2 q_k(i_k); the DVR position
// is diagonal in the grid index with the grid point as eigenvalue (Sec. II.A).
// q holds the grid points [D][nmax].
__global__ __launch_bounds__(TB) void k_expq_partial(const uint32_t *keys, const double2 *psi, int64_t n, GridDesc g,
                                                     const double *q, int nmax, double2 *partial)
{
    double2 acc[1 + MAXD];
#pragma unroll
    for (int i = 0; i <= MAXD; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * TB) {
        double2 c = psi[p];
        double w = fma(c.x, c.x, c.y * c.y);
        acc[0].x += w;
        uint32_t key = keys[p];
#pragma unroll
        for (int k = 0; k < MAXD; ++k)
            if (k < g.D) {
                int d = (int)((key / g.stride[k]) % (uint32_t)g.n[k]);
                acc[1 + k].x = fma(w, q[k * nmax + d], acc[1 + k].x);
            }
    }
    block_reduce_store<1 + MAXD>(acc, partial);
}

// Fixed-order sum of the partials; out[k] = sum_k / sum_0, NaN where bit k of
// `nan_mask` is set (dimensions without a diagonal position) or the sum is 0.
__global__ __launch_bounds__(TB) void k_expq_final(const double2 *partial, int nb, int D, unsigned nan_mask,
                                                   double *out)
{
    __shared__ double red[TB];
    __shared__ double norm2;
    for (int i = 0; i <= D; ++i) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += TB) s += partial[pidx(b, i)].x;
        red[threadIdx.x] = s;
        __syncthreads();
        for (int st = TB / 2; st >= 1; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (i == 0) norm2 = red[0];
            else
                out[i - 1] = ((nan_mask >> (i - 1)) & 1u) || !(norm2 > 0.0) ? __builtin_nan("") : red[0] / norm2;
        }
        __syncthreads();
    }
}

// ---- device-side state transfer ---------------------------------------------------
// Checks caller keys (strictly ascending, below the grid size) and coefficients
// (finite) while converting them: bad[0] counts key violations, bad[1]
// non-finite coefficients (per-block counts summed by one fixed-order kernel).
__global__ void k_take_state(const uint64_t *keys, const double2 *coeff, int64_t n, uint64_t total, uint32_t *k32,
                             double2 *psi, unsigned *block_bad_keys, unsigned *block_bad_vals)
{
    int64_t p = gid();
    bool bad_key = false, bad_val = false;
    if (p < n) {
        const uint64_t k = keys[p];
        bad_key = k >= total || (p > 0 && keys[p - 1] >= k);
        const double2 c = coeff[p];
        bad_val = !isfinite(c.x) || !isfinite(c.y);
        k32[p] = (uint32_t)k;
        psi[p] = c;
    }
    count_block(bad_key, block_bad_keys);
    count_block(bad_val, block_bad_vals);
}

__global__ void k_give_keys(const uint32_t *k32, int64_t n, uint64_t *keys)
{
    int64_t p = gid();
    if (p < n) keys[p] = k32[p];
}

// host-known fields of one observable record
__global__ void k_set_record(double *rec, double t, double nact, double krylov, double nsub)
{
    rec[PPQ_OBS_T] = t;
    rec[PPQ_OBS_NACTIVE] = nact;
    rec[PPQ_OBS_KRYLOV] = krylov;
    rec[PPQ_OBS_SUBSTEPS] = nsub;
}

__global__ void k_copy_alpha0(const KState *ks, double *dst) { *dst = ks->alpha[0]; }
__global__ void k_copy_meff(const KState *ks, double *dst) { *dst = (double)ks->meff; }

__global__ __launch_bounds__(TB) void k_energy_from_dot(const double2 *partial, int nb, double *rec)
{
    __shared__ double red[TB];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += TB) s += partial[pidx(b, 0)].x;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = TB / 2; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double n2 = rec[PPQ_OBS_NORM2];
        rec[PPQ_OBS_ENERGY] = n2 > 0.0 ? red[0] / n2 : 0.0;
    }
}

// ---- adjoint ----------------------------------------------------------------------
// R^dagger of one adaption: mu (on the earlier set) from lambda (on the later
// set): mu_I = lambda_I for I in both sets, zero otherwise.
__global__ void k_gather_remap(const uint32_t *keys, int64_t n, const uint64_t *bm, const uint32_t *prefix,
                               const double2 *lam, double2 *mu)
{
    int64_t p = gid();
    if (p >= n) return;
    uint32_t key = keys[p];
    uint64_t word = bm[key >> 6];
    uint32_t b = key & 63;
    mu[p] = ((word >> b) & 1ull) ? lam[prefix[key >> 6] + (uint32_t)__popcll(word & ((1ull << b) - 1ull))]
                                 : make_double2(0.0, 0.0);
}

__global__ void k_count_diff(const double2 *a, const double2 *b, int64_t n, unsigned long long *cnt)
{
    int64_t p = gid();
    bool diff = false;
    if (p < n) {
        double2 x = a[p], y = b[p];
        diff = (__double_as_longlong(x.x) != __double_as_longlong(y.x)) ||
               (__double_as_longlong(x.y) != __double_as_longlong(y.y));
    }
    count_ballot(diff, cnt);
}

__global__ void k_mark_wave(const uint32_t *keys, int64_t n, uint64_t *bm)
{
    int64_t p = gid();
    uint32_t key = p < n ? keys[p] : 0u;
    set_bit_wave(bm, key, p < n);
}

// Time integral of the Krylov-projected Frechet derivative:
//   Q = m0 n0 [exp([[-i dt T_b, e1 e1^T], [0, -i dt T_f]])]_{12}
// (the block-triangular exponential gives int_0^1 e^{A(1-s)} X e^{Bs} ds),
// T_f, T_b the Lanczos matrices of psi_n (forward) and mu (adjoint), both of
// dimension m; 1024 lanes, one per entry of the 32 x 32 block matrix.
constexpr int M2 = 2 * MAXM;
__global__ __launch_bounds__(1024) void k_adj_q(const KState *kf, const KState *kb, double dt, double2 *Q)
{
    __shared__ double2 A[M2][M2], P[M2][M2], E[M2][M2];
    __shared__ double rown[M2];
    __shared__ int s_sq;
    const int mf = kf->meff, mb = kb->meff;
    const int r = threadIdx.x / M2, c = threadIdx.x % M2;
    double h = 0.0;
    double2 x = make_double2(0.0, 0.0);
    // top-left: T_b (mb x mb) at [0, MAXM); bottom-right: T_f at [MAXM, 2 MAXM)
    auto tri = [](const KState *k, int mm, int i, int j) -> double {
        if (i >= mm || j >= mm) return 0.0;
        if (i == j) return k->alpha[i];
        if (i == j + 1) return k->beta[j];
        if (j == i + 1) return k->beta[i];
        return 0.0;
    };
    if (r < MAXM && c < MAXM) h = tri(kb, mb, r, c);
    else if (r >= MAXM && c >= MAXM) h = tri(kf, mf, r - MAXM, c - MAXM);
    A[r][c] = make_double2(0.0, -dt * h);
    if (r == 0 && c == MAXM) A[r][c] = make_double2(1.0, 0.0);
    (void)x;
    __syncthreads();
    if (threadIdx.x < M2) {
        double s = 0.0;
        for (int cc = 0; cc < M2; ++cc) s += sqrt(A[threadIdx.x][cc].x * A[threadIdx.x][cc].x + A[threadIdx.x][cc].y * A[threadIdx.x][cc].y);
        rown[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double nrm = 0.0;
        for (int i = 0; i < M2; ++i) nrm = rown[i] > nrm ? rown[i] : nrm;
        int sq = 0;
        while (nrm > 0.125) {
            nrm *= 0.5;
            ++sq;
        }
        s_sq = sq;
    }
    __syncthreads();
    const int sq = s_sq;
    const double scale = ldexp(1.0, -sq);
    A[r][c] = make_double2(A[r][c].x * scale, A[r][c].y * scale);
    P[r][c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    E[r][c] = P[r][c];
    __syncthreads();
    for (int kt = 1; kt <= 18; ++kt) {
        double2 acc = make_double2(0.0, 0.0);
        for (int l = 0; l < M2; ++l) {
            double2 a = P[r][l], b = A[l][c];
            acc.x += a.x * b.x - a.y * b.y;
            acc.y += a.x * b.y + a.y * b.x;
        }
        __syncthreads();
        P[r][c] = make_double2(acc.x / kt, acc.y / kt);
        E[r][c] = make_double2(E[r][c].x + acc.x / kt, E[r][c].y + acc.y / kt);
        __syncthreads();
    }
    for (int q = 0; q < sq; ++q) {
        double2 acc = make_double2(0.0, 0.0);
        for (int l = 0; l < M2; ++l) {
            double2 a = E[r][l], b = E[l][c];
            acc.x += a.x * b.x - a.y * b.y;
            acc.y += a.x * b.y + a.y * b.x;
        }
        __syncthreads();
        E[r][c] = acc;
        __syncthreads();
    }
    if (r < MAXM && c >= MAXM) {
        const double s2 = kf->n0 * kb->n0;
        double2 e = E[r][c];
        Q[r * MAXM + (c - MAXM)] = (r < mb && c - MAXM < mf) ? make_double2(s2 * e.x, s2 * e.y) : make_double2(0.0, 0.0);
    }
}

// Per point S = sum_ab Q_ab conj(W_a) V_b, then for every parameter p the
// partial sums of S * G_p(I), G_p = dV/dtheta_p as a sum of products of 1D
// tables (staged in LDS).  V_0 / W_0 come from the FP64 master vectors
// (psi_n / n0 and mu / m0), like the propagated vectors.
template <class C>
__global__ __launch_bounds__(TB) void k_adj_reduce(const C *Vb, const C *Wb, int64_t ld, const double2 *psi,
                                                   const double2 *mu, const KState *kf, const KState *kb,
                                                   const double2 *Q, const uint32_t *keys, int64_t n, GridDesc g,
                                                   DerivDesc dd, double2 *partial)
{
    __shared__ double2 sQ[MAXM * MAXM];
    __shared__ double s_coef[POT_MAX_TERMS];
    __shared__ int s_par[POT_MAX_TERMS];
    __shared__ int s_nf[POT_MAX_TERMS];
    __shared__ int s_fac[POT_MAX_TERMS][POT_MAX_FAC];
    __shared__ double s_tab[POT_MAX_TAB];
    for (int i = threadIdx.x; i < MAXM * MAXM; i += TB) sQ[i] = Q[i];
    for (int t = threadIdx.x; t < dd.nterm; t += TB) {
        s_coef[t] = dd.coef[t];
        s_par[t] = dd.param[t];
        int nf = 0;
        for (int k = 0; k < g.D; ++k) {
            int ti = dd.tab[t * g.D + k];
            if (ti >= 0 && nf < POT_MAX_FAC) s_fac[t][nf++] = (ti << 4) | k;
        }
        s_nf[t] = nf;
    }
    for (int i = threadIdx.x; i < dd.ntab * dd.nmax; i += TB) s_tab[i] = dd.tabs[i];
    __syncthreads();
    const int mf = kf->meff, mb = kb->meff;
    const double inv_n0 = 1.0 / kf->n0, inv_m0 = 1.0 / kb->n0;
    double2 acc[ADJ_MAXP];
#pragma unroll
    for (int i = 0; i < ADJ_MAXP; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * TB) {
        double2 v[MAXM];
        double2 a0 = psi[p];
        v[0] = make_double2(a0.x * inv_n0, a0.y * inv_n0);
#pragma unroll
        for (int b = 1; b < MAXM; ++b) v[b] = (b < mf) ? ld2(Vb, (int64_t)b * ld + p) : make_double2(0.0, 0.0);
        double2 S = make_double2(0.0, 0.0);
        for (int a = 0; a < mb; ++a) {
            double2 t = make_double2(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < MAXM; ++b) {
                double2 q = sQ[a * MAXM + b];
                t.x += q.x * v[b].x - q.y * v[b].y;
                t.y += q.x * v[b].y + q.y * v[b].x;
            }
            double2 wa;
            if (a == 0) {
                double2 m0v = mu[p];
                wa = make_double2(m0v.x * inv_m0, m0v.y * inv_m0);
            } else {
                wa = ld2(Wb, (int64_t)a * ld + p);
            }
            cdot_acc(S, wa, t);
        }
        uint32_t key = keys[p];
        int d[MAXD];
#pragma unroll
        for (int k = 0; k < MAXD; ++k) d[k] = (k < g.D) ? (int)((key / g.stride[k]) % (uint32_t)g.n[k]) : 0;
        for (int t = 0; t < dd.nterm; ++t) {
            double f = s_coef[t];
            const int nf = s_nf[t];
#pragma unroll
            for (int j = 0; j < POT_MAX_FAC; ++j) {
                if (j < nf) {
                    int e = s_fac[t][j];
                    f *= s_tab[(e >> 4) * dd.nmax + select_digit(d, e & 15)];
                }
            }
            const int pp = s_par[t];
#pragma unroll
            for (int i = 0; i < ADJ_MAXP; ++i) {
                if (i == pp) {
                    acc[i].x += f * S.x;
                    acc[i].y += f * S.y;
                }
            }
        }
    }
    block_reduce_store<ADJ_MAXP>(acc, partial);
}

// dC[p] += coef * sum over blocks (fixed order), coef = -i dt
__global__ __launch_bounds__(TB) void k_adj_accumulate(const double2 *partial, int nb, int nparam,
                                                       double2 coef, double2 *dC)
{
    __shared__ double2 red[TB];
    for (int i = 0; i < nparam; ++i) {
        double2 s = make_double2(0.0, 0.0);
        for (int b = threadIdx.x; b < nb; b += TB) {
            s.x += partial[pidx(b, i)].x;
            s.y += partial[pidx(b, i)].y;
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int st = TB / 2; st >= 1; st >>= 1) {
            if ((int)threadIdx.x < st) {
                red[threadIdx.x].x += red[threadIdx.x + st].x;
                red[threadIdx.x].y += red[threadIdx.x + st].y;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double2 r = red[0];
            dC[i].x += coef.x * r.x - coef.y * r.y;
            dC[i].y += coef.x * r.y + coef.y * r.x;
        }
        __syncthreads();
    }
}

// Packet-parameter terms.  For each dimension k and each of the two packet
// parameters (centre, momentum) the derivative of psi0_I is the product of
// the 1D tables with factor k replaced by its derivative table.
//   bra = 1: accumulates conj(dpsi0_I) vec_I      (<d psi0 | psi_N>)
//   bra = 0: accumulates conj(vec_I) dpsi0_I      (<lambda_0 | d psi0>)
constexpr int ADJ_MAXQ = 2 * MAXD;
__global__ __launch_bounds__(TB) void k_adj_packet(const uint32_t *keys, int64_t n, GridDesc g, const double2 *tabs,
                                                   const double2 *dtabs, int nmax, const double2 *vec, int bra,
                                                   double2 *partial)
{
    double2 acc[ADJ_MAXQ];
#pragma unroll
    for (int i = 0; i < ADJ_MAXQ; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int64_t p = gid(); p < n; p += (int64_t)gridDim.x * TB) {
        uint32_t key = keys[p];
        double2 v = vec[p];
        for (int kd = 0; kd < g.D; ++kd) {
            for (int which = 0; which < 2; ++which) {
                double2 prod = make_double2(1.0, 0.0);
                for (int k = 0; k < g.D; ++k) {
                    int d = (int)((key / g.stride[k]) % (uint32_t)g.n[k]);
                    double2 f = (k == kd) ? dtabs[(2 * k + which) * nmax + d] : tabs[k * nmax + d];
                    prod = cmul(prod, f);
                }
                double2 r = make_double2(0.0, 0.0);
                if (bra) cdot_acc(r, prod, v);
                else cdot_acc(r, v, prod);
                int slot = 2 * kd + which;
#pragma unroll
                for (int i = 0; i < ADJ_MAXQ; ++i)
                    if (i == slot) {
                        acc[i].x += r.x;
                        acc[i].y += r.y;
                    }
            }
        }
    }
    block_reduce_store<ADJ_MAXQ>(acc, partial);
}

}  // namespace

// ---- launchers -------------------------------------------------------------------
void fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s)
{
    if (n <= 0) return;
    unsigned b = nblocks(n);
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL(k_fill<uint64_t>, dim3(b), dim3(TB), 0, s, p, n, v);
}
void fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n <= 0) return;
    unsigned b = nblocks(n);
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(b), dim3(TB), 0, s, p, n, v);
}
void fill_zero_bytes(void *p, int64_t nbytes, hipStream_t s)
{
    // callers pass 8-byte multiples
    fill_u64((uint64_t *)p, nbytes / 8, 0ull, s);
}

int64_t scan_tmp_words(int64_t n) { return (n + STILE - 1) / STILE + 16; }

void scan_popcount(const uint64_t *words, int64_t nwords, uint32_t *prefix, uint32_t *total, uint32_t *tmp,
                   hipStream_t s)
{
    scan_impl(PopLoad{words}, nwords, prefix, total, tmp, s);
}
void scan_u32(const uint32_t *in, int64_t n, uint32_t *out, uint32_t *total, uint32_t *tmp, hipStream_t s)
{
    scan_impl(U32Load{in}, n, out, total, tmp, s);
}

void init_flag(const GridDesc &g, const double2 *tabs, int nmax, double eps2, uint64_t *bm,
               unsigned long long *nabove, hipStream_t s)
{
    unsigned b = nblocks(g.total);
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL(k_init_flag, dim3(b), dim3(TB), 0, s, g, tabs, nmax, eps2, bm, nabove);
}
void product_values(const uint32_t *keys, int64_t n, const GridDesc &g, const double2 *tabs, int nmax,
                    double2 *out, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_product_values, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, g, tabs, nmax, out);
}
void dilate(const uint32_t *keys, const double2 *psi, int64_t n, const GridDesc &g, double eps2, uint64_t *bm,
            unsigned long long *nabove, unsigned *block_counts, hipStream_t s)
{
    if (n <= 0) return;
    const unsigned nb = nblocks(n);
    hipLaunchKernelGGL(k_dilate, dim3(nb), dim3(TB), 0, s, keys, psi, n, g, eps2, bm, block_counts);
    hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(1024), 0, s, block_counts, (int64_t)nb, nabove);
}
void dilate_words(const uint32_t *keys, const double2 *psi, int64_t n, const GridDesc &g, double eps2, uint64_t *K,
                  uint64_t *bm, int64_t nwords, unsigned long long *nabove, unsigned *block_counts, hipStream_t s)
{
    fill_u64(K, nwords, 0ull, s);
    if (n > 0) {
        const unsigned nb = nblocks(n);
        hipLaunchKernelGGL(k_mark_kept, dim3(nb), dim3(TB), 0, s, keys, psi, n, eps2, K, block_counts);
        hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(1024), 0, s, block_counts, (int64_t)nb, nabove);
    }
    const int64_t waves = (nwords + 64 * DW_ITER - 1) / (64 * DW_ITER);
    hipLaunchKernelGGL(k_dilate_words, dim3((unsigned)((waves * 64 + TB - 1) / TB)), dim3(TB), 0, s, K, nwords, g, bm);
    fill_u64(bm + nwords, 2, 0ull, s);
}
void keep_all_if_few_dropped(const uint32_t *keys, int64_t n, uint64_t *bm, double rel, unsigned *block_counts,
                             unsigned long long *dropped, hipStream_t s)
{
    if (n <= 0) return;
    const unsigned nb = nblocks(n);
    hipLaunchKernelGGL(k_count_dropped, dim3(nb), dim3(TB), 0, s, keys, n, bm, block_counts);
    hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(1024), 0, s, block_counts, (int64_t)nb, dropped);
    hipLaunchKernelGGL(k_keep_all_if, dim3(nb), dim3(TB), 0, s, keys, n, bm, dropped, rel);
}
void mark_keys(const uint32_t *keys, int64_t n, uint64_t *bm, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mark, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, bm);
}
void compact(const uint64_t *bm, const uint32_t *prefix, int64_t nwords, uint32_t *keys_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_compact, dim3(nblocks(nwords)), dim3(TB), 0, s, bm, prefix, nwords, keys_out);
}
void remap(const uint32_t *okeys, const double2 *opsi, int64_t n_old, const uint64_t *bm, const uint32_t *prefix,
           double2 *npsi, hipStream_t s)
{
    if (n_old <= 0) return;
    hipLaunchKernelGGL(k_remap, dim3(nblocks(n_old)), dim3(TB), 0, s, okeys, opsi, n_old, bm, prefix, npsi);
}

void last_flags(const uint32_t *keys, int64_t n, int nlast, uint32_t *flags, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_last_flags, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, nlast, flags);
}
void last_fill(const uint32_t *keys, int64_t n, int nlast, const uint32_t *flags, const uint32_t *fidx,
               const uint32_t *nf, uint32_t *off, uint64_t *mask, hipStream_t s)
{
    if (nlast <= NMAX_MASK)
        hipLaunchKernelGGL(k_zero_masks, dim3(std::min<unsigned>(nblocks(n), 2048u)), dim3(TB), 0, s, mask, nf);
    hipLaunchKernelGGL(k_last_fill, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, nlast, flags, fidx, nf, off, mask);
}
void rot_set(const uint32_t *keys, int64_t n, const RotFrame &f, uint64_t *bm, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rot_set, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, f.sk, f.nk, f.rin, f.rout, bm);
}
void rot_rank(const uint32_t *keys, int64_t n, const RotFrame &f, const uint64_t *bm, const uint32_t *prefix,
              const uint32_t *map, uint32_t *pi, uint32_t *inv, uint32_t *flags, uint64_t *tmpmask, uint8_t *info,
              hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rot_rank, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, f.sk, f.nk, f.rin, f.rout, bm, prefix,
                       map, pi, inv, flags, tmpmask, info);
}
__global__ void k_chunk_fibers(const uint32_t *chunk, uint32_t nch, const uint32_t *fidx, const uint32_t *nf,
                               uint32_t n, uint32_t *out)
{
    int64_t t = gid();
    if (t > nch) return;
    const uint32_t c = chunk[t];
    out[t] = c < n ? fidx[c] : *nf;
}

void chunk_fibers(const uint32_t *chunk, int64_t n, uint32_t S, const uint32_t *fidx, const uint32_t *nf,
                  uint32_t *out, hipStream_t s)
{
    uint32_t nch = (uint32_t)((n + S - 1) / S);
    hipLaunchKernelGGL(k_chunk_fibers, dim3(nblocks((int64_t)nch + 1)), dim3(TB), 0, s, chunk, nch, fidx, nf,
                       (uint32_t)n, out);
}

void make_chunks(const uint32_t *keys, const uint32_t *P, int64_t n, uint32_t sin, bool inner, uint32_t S,
                 uint32_t cap, uint32_t *chunk, uint32_t *big, uint32_t *counters, hipStream_t s)
{
    uint32_t nch = (uint32_t)((n + S - 1) / S);
    hipLaunchKernelGGL(k_chunks, dim3(nblocks((int64_t)nch + 1)), dim3(TB), 0, s, keys, P, (uint32_t)n, sin,
                       inner ? 1 : 0, S, nch, cap, chunk, big, counters);
}
void last_info(const uint32_t *keys, int64_t n, int nlast, uint8_t *info, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_last_info, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, nlast, info);
}
void fiber_tables_all(const uint32_t *keys, int64_t n, const RotAll &r, uint64_t *bm, uint32_t *prefix,
                      uint64_t *occ, uint32_t *oprefix, const TabPtrs &t, uint32_t *scan_tmp, uint32_t *counters,
                      uint32_t *nf, hipStream_t s)
{
    if (n <= 0 || r.nd <= 0) return;
    const int64_t words = (int64_t)(r.nd + 1) * r.nwords;  // nd rotated segments + the row-major one
    const int64_t owords = r.owoff[r.nd];
    fill_u64(bm, words + 2, 0ull, s);
    fill_u64(occ, owords + 2, 0ull, s);
    hipLaunchKernelGGL(k_rot_set_all, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, r, bm, occ);
    scan_popcount(bm, words, prefix, &counters[0], scan_tmp, s);
    scan_popcount(occ, owords, oprefix, &counters[1], scan_tmp, s);
    hipLaunchKernelGGL(k_occ_counts, dim3(1), dim3(64), 0, s, oprefix, n, r, &counters[1], t, nf);
    hipLaunchKernelGGL(k_rank_gather, dim3(nblocks((int64_t)r.nd * r.nwords)), dim3(TB), 0, s, n, r, bm, prefix, occ,
                       oprefix, t);
}
void plane_tables(const uint32_t *keys, int64_t n, const GridDesc &g, int a, uint64_t *bm, uint32_t *prefix,
                  int64_t nwords, uint32_t *P, uint16_t *dig, uint32_t *tstart, uint32_t *poff, uint32_t *pkey,
                  uint32_t *flags, uint32_t *pidx, uint32_t *scan_tmp, uint32_t *counter, hipStream_t s)
{
    if (n <= 0) return;
    const uint32_t na = (uint32_t)g.n[a], nb = (uint32_t)g.n[a + 1];
    const bool ident = (a + 2 == g.D);
    const uint32_t sk = g.stride[a + 1];
    if (!ident) {
        fill_u64(bm, nwords + 2, 0ull, s);
        hipLaunchKernelGGL(k_rot_set, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, sk, na * nb, 0u, 0u, bm);
        scan_popcount(bm, nwords, prefix, counter, scan_tmp, s);
    }
    hipLaunchKernelGGL(k_plane_rank, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, ident ? 1u : sk, na, nb,
                       ident ? nullptr : bm, ident ? nullptr : prefix, ident ? nullptr : P, dig, pkey);
    hipLaunchKernelGGL(k_plane_flags, dim3(nblocks(n)), dim3(TB), 0, s, pkey, n, flags, dig);
    scan_u32(flags, n, pidx, counter, scan_tmp, s);
    hipLaunchKernelGGL(k_plane_fill, dim3(nblocks(n)), dim3(TB), 0, s, flags, pidx, n, counter, poff);
    const uint32_t ntask = (uint32_t)((n + PLANE_WINDOW - 1) / PLANE_WINDOW);
    hipLaunchKernelGGL(k_plane_tasks, dim3(nblocks(n + 1)), dim3(TB), 0, s, poff, counter, n, PLANE_WINDOW, ntask,
                       tstart);
}

void pair_tasks(const uint32_t *keys, int64_t n, uint32_t nab, uint32_t *tstart, hipStream_t s)
{
    if (n <= 0) return;
    const uint32_t ntask = (uint32_t)((n + PAIR_WINDOW - 1) / PAIR_WINDOW);
    const int64_t threads = ((int64_t)ntask + 1) * 64;
    hipLaunchKernelGGL(k_pair_tasks, dim3((unsigned)((threads + TB - 1) / TB)), dim3(TB), 0, s, keys, n, nab,
                       PAIR_WINDOW, ntask, tstart);
}

void fib_fill(const uint32_t *flags, const uint32_t *fidx, const uint64_t *tmpmask, int64_t n, const uint32_t *nf,
              uint32_t *off, uint64_t *mask, hipStream_t s)
{
    hipLaunchKernelGGL(k_fib_fill, dim3(nblocks(n)), dim3(TB), 0, s, flags, fidx, tmpmask, n, nf, off, mask);
}

void potential(const uint32_t *keys, int64_t n, const GridDesc &g, const PotDesc &pd, double *V, float *Vf,
               uint32_t *list, unsigned *count, hipStream_t s)
{
    if (n <= 0) return;
    const unsigned nb = std::min<unsigned>(nblocks(n), 2048u);
    if (list) {
        fill_u32(count, 1, 0u, s);
        const unsigned mb = std::min<unsigned>(nblocks(n), 1024u);
        if (V) hipLaunchKernelGGL(k_missing<double>, dim3(mb), dim3(TB), 0, s, V, n, list, count);
        else hipLaunchKernelGGL(k_missing<float>, dim3(mb), dim3(TB), 0, s, Vf, n, list, count);
    }
    hipLaunchKernelGGL(k_potential, dim3(nb), dim3(TB), 0, s, keys, n, g, pd, V, Vf, list, count);
}

template <class T>
__global__ void k_remap_values(const uint32_t *okeys, const T *ov, int64_t n_old, const uint64_t *bm,
                               const uint32_t *prefix, T *nv)
{
    int64_t p = gid();
    if (p >= n_old) return;
    uint32_t key = okeys[p];
    uint64_t word = bm[key >> 6];
    uint32_t b = key & 63;
    if ((word >> b) & 1ull) {
        uint32_t q = prefix[key >> 6] + (uint32_t)__popcll(word & ((1ull << b) - 1ull));
        nv[q] = ov[p];
    }
}

template <class T>
void remap_values(const uint32_t *okeys, const T *ov, int64_t n_old, const uint64_t *bm, const uint32_t *prefix,
                  T *nv, hipStream_t s)
{
    if (n_old <= 0) return;
    hipLaunchKernelGGL(k_remap_values<T>, dim3(nblocks(n_old)), dim3(TB), 0, s, okeys, ov, n_old, bm, prefix, nv);
}
template void remap_values<double>(const uint32_t *, const double *, int64_t, const uint64_t *, const uint32_t *,
                                   double *, hipStream_t);
template void remap_values<float>(const uint32_t *, const float *, int64_t, const uint64_t *, const uint32_t *,
                                  float *, hipStream_t);

static unsigned red_blocks(int64_t n)
{
    int64_t b = (n + TB - 1) / TB;
    if (b > RED_BLOCKS) b = RED_BLOCKS;
    return (unsigned)(b < 1 ? 1 : b);
}

#define PPQ_NV_SWITCH(nv, CALL) \
    switch (nv) {               \
    case 1: CALL(1); break;     \
    case 2: CALL(2); break;     \
    case 3: CALL(3); break;     \
    case 4: CALL(4); break;     \
    case 5: CALL(5); break;     \
    case 6: CALL(6); break;     \
    case 7: CALL(7); break;     \
    case 8: CALL(8); break;     \
    case 9: CALL(9); break;     \
    case 10: CALL(10); break;   \
    case 11: CALL(11); break;   \
    case 12: CALL(12); break;   \
    case 13: CALL(13); break;   \
    case 14: CALL(14); break;   \
    case 15: CALL(15); break;   \
    case 16: CALL(16); break;   \
    default: break;             \
    }

template <class C>
void norm0(const double2 *psi, int64_t n, double2 *partial, unsigned *counter, KState *ks, int m, double dt,
           double tol, hipStream_t s)
{
    hipLaunchKernelGGL(k_norm0<C>, dim3(RED_BLOCKS), dim3(TB), 0, s, psi, n, partial, counter, ks, m);
    hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(TB), 0, s, partial, RED_BLOCKS, ks, 0, (int)RED_NORM0, m, 0, 1,
                       dt, tol);
}
template <class C>
void cgs_dots(const C *Vb, int64_t ld, int nv, const C *w, int64_t n, double2 *partial, unsigned *counter, KState *ks,
              int j, int m, int ioff, hipStream_t s, int mode)
{
#define CALL(NV)                                                                                                  \
    hipLaunchKernelGGL((k_cgs_dots<C, NV>), dim3(RED_BLOCKS), dim3(TB), 0, s, Vb, ld, w, n, partial, counter, ks, j, \
                       m, ioff);                                                                              \
    hipLaunchKernelGGL(k_finalize<NV>, dim3(1), dim3(TB), 0, s, partial, RED_BLOCKS, ks, j, mode, m, ioff, NV, 0.0, \
                       0.0)
    PPQ_NV_SWITCH(nv, CALL)
#undef CALL
}
void finalize_dot(const double2 *partial, int nb, KState *ks, int j, int m, int mode, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(TB), 0, s, partial, nb, ks, j, mode, m, j, 1, 0.0, 0.0);
}
template <class C>
void lanczos_sweep(C *Vb, int64_t ld, const C *z, int64_t n, double2 *partial, unsigned *counter, KState *ks, int j,
                   int m, hipStream_t s)
{
#define CALL(NV)                                                                                                    \
    hipLaunchKernelGGL((k_lanczos_sweep<C, NV>), dim3(RED_BLOCKS), dim3(TB), 0, s, Vb, ld, z, n, partial, counter, \
                       ks, j);                                                                                   \
    hipLaunchKernelGGL(k_finalize<NV + 2>, dim3(1), dim3(TB), 0, s, partial, RED_BLOCKS, ks, j, (int)RED_BETA, m, 0, \
                       NV + 2, 0.0, 0.0)
    switch (j) {
    case 0: CALL(0); break;
    case 1: CALL(1); break;
    case 2: CALL(2); break;
    case 3: CALL(3); break;
    case 4: CALL(4); break;
    case 5: CALL(5); break;
    case 6: CALL(6); break;
    case 7: CALL(7); break;
    case 8: CALL(8); break;
    case 9: CALL(9); break;
    case 10: CALL(10); break;
    case 11: CALL(11); break;
    case 12: CALL(12); break;
    case 13: CALL(13); break;
    case 14: CALL(14); break;
    default: break;
    }
#undef CALL
}
template <class C>
void arnoldi_step(C *Vb, int64_t ld, const C *z, int64_t n, double2 *partial, unsigned *counter, KState *ks, int j,
                  int m, bool last, hipStream_t s)
{
#define CALL(NV)                                                                                                   \
    hipLaunchKernelGGL((k_arnoldi_dots<C, NV>), dim3(RED_BLOCKS), dim3(TB), 0, s, Vb, ld, z, n, partial, counter, \
                       ks, j);                                                                                  \
    hipLaunchKernelGGL(k_finalize<NV + 1>, dim3(1), dim3(TB), 0, s, partial, RED_BLOCKS, ks, j, (int)RED_ADELAY, m, \
                       0, NV + 1, 0.0, 0.0);                                                                    \
    if (!last) {                                                                                               \
        hipLaunchKernelGGL((k_arnoldi_sweep<C, NV>), dim3(RED_BLOCKS), dim3(TB), 0, s, Vb, ld, z, n, partial,   \
                           counter, ks, j);                                                                     \
        hipLaunchKernelGGL(k_finalize<NV + 2>, dim3(1), dim3(TB), 0, s, partial, RED_BLOCKS, ks, j, (int)RED_BETA, \
                           m, 0, NV + 2, 0.0, 0.0);                                                            \
    }
    switch (j) {
    case 0: CALL(0); break;
    case 1: CALL(1); break;
    case 2: CALL(2); break;
    case 3: CALL(3); break;
    case 4: CALL(4); break;
    case 5: CALL(5); break;
    case 6: CALL(6); break;
    case 7: CALL(7); break;
    case 8: CALL(8); break;
    case 9: CALL(9); break;
    case 10: CALL(10); break;
    case 11: CALL(11); break;
    case 12: CALL(12); break;
    case 13: CALL(13); break;
    case 14: CALL(14); break;
    case 15: CALL(15); break;
    default: break;
    }
#undef CALL
}
void lanczos_coef(KState *ks, int m, hipStream_t s)
{
    hipLaunchKernelGGL(k_lanczos_coef, dim3(1), dim3(64), 0, s, ks, m);
}
template <class C>
void lanczos_fix(C *Vb, int64_t ld, int64_t n, const KState *ks, int j, hipStream_t s)
{
    unsigned b = red_blocks(n) * 4;
#define CALL(NV) hipLaunchKernelGGL((k_lanczos_fix<C, NV>), dim3(b), dim3(TB), 0, s, Vb, ld, n, ks, j)
    PPQ_NV_SWITCH(j, CALL)
#undef CALL
}
template <class C>
void normalise_from_master(const double2 *psi, int64_t n, KState *ks, C *v0, hipStream_t s)
{
    unsigned b = red_blocks(n) * 4;
    hipLaunchKernelGGL(k_normalise<C>, dim3(b), dim3(TB), 0, s, psi, n, ks, v0);
}
template <class C>
void lincomb(const C *Vb, int64_t ld, const double2 *psi_master, int64_t n, const KState *ks, double2 *psi_out,
             hipStream_t s)
{
    unsigned b = red_blocks(n) * 4;
    hipLaunchKernelGGL(k_lincomb<C>, dim3(b), dim3(TB), 0, s, Vb, ld, psi_master, n, ks, psi_out);
}

#define PPQ_INST(C)                                                                                               \
    template void norm0<C>(const double2 *, int64_t, double2 *, unsigned *, KState *, int, double, double,        \
                           hipStream_t);                                                                         \
    template void cgs_dots<C>(const C *, int64_t, int, const C *, int64_t, double2 *, unsigned *, KState *, int,  \
                              int, int, hipStream_t, int);                                                      \
    template void lanczos_sweep<C>(C *, int64_t, const C *, int64_t, double2 *, unsigned *, KState *, int, int,   \
                                   hipStream_t);                                                                \
    template void lanczos_fix<C>(C *, int64_t, int64_t, const KState *, int, hipStream_t);                        \
    template void arnoldi_step<C>(C *, int64_t, const C *, int64_t, double2 *, unsigned *, KState *, int, int,    \
                                  bool, hipStream_t);                                                           \
    template void normalise_from_master<C>(const double2 *, int64_t, KState *, C *, hipStream_t);                 \
    template void lincomb<C>(const C *, int64_t, const double2 *, int64_t, const KState *, double2 *, hipStream_t);
PPQ_INST(double2)
PPQ_INST(float2)
#undef PPQ_INST

void krylov_expv(KState *ks, int m, double dt, int hermitian, hipStream_t s)
{
    (void)m;
    hipLaunchKernelGGL(k_krylov_expv, dim3(1), dim3(256), 0, s, ks, dt, hermitian);
}
void dot_partial(const double2 *a, const double2 *b, int64_t n, double2 *partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partial, dim3(RED_BLOCKS), dim3(TB), 0, s, a, b, n, partial);
}
void obs_partial(const uint32_t *keys, const double2 *psi, int64_t n, const GridDesc &g, const double2 *bra,
                 int nmax, double eps2, double2 *partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_obs_partial, dim3(RED_BLOCKS), dim3(TB), 0, s, keys, psi, n, g, bra, nmax, eps2, partial);
}
void obs_final(const double2 *partial, int nb, double *rec, hipStream_t s)
{
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(TB), 0, s, partial, nb, rec);
}
void expect_q(const uint32_t *keys, const double2 *psi, int64_t n, const GridDesc &g, const double *q, int nmax,
              unsigned nan_mask, double2 *partial, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_expq_partial, dim3(RED_BLOCKS), dim3(TB), 0, s, keys, psi, n, g, q, nmax, partial);
    hipLaunchKernelGGL(k_expq_final, dim3(1), dim3(TB), 0, s, partial, RED_BLOCKS, g.D, nan_mask, out);
}
void take_state(const uint64_t *keys, const double2 *coeff, int64_t n, uint64_t total, uint32_t *k32, double2 *psi,
                unsigned *block_counts, unsigned long long *bad, hipStream_t s)
{
    if (n <= 0) return;
    const unsigned nb = nblocks(n);
    hipLaunchKernelGGL(k_take_state, dim3(nb), dim3(TB), 0, s, keys, coeff, n, total, k32, psi, block_counts,
                       block_counts + nb);
    hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(1024), 0, s, block_counts, (int64_t)nb, bad);
    hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(1024), 0, s, block_counts + nb, (int64_t)nb, bad + 1);
}
void give_keys(const uint32_t *k32, int64_t n, uint64_t *keys, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_give_keys, dim3(nblocks(n)), dim3(TB), 0, s, k32, n, keys);
}
void sum_of_squares(const double2 *psi, int64_t n, double2 *partial, double2 *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sq_partial, dim3(RED_BLOCKS), dim3(TB), 0, s, psi, n, partial);
    hipLaunchKernelGGL(k_sum_partial1, dim3(1), dim3(TB), 0, s, partial, RED_BLOCKS, out);
}
void set_record(double *rec, double t, double nact, double krylov, double nsub, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_record, dim3(1), dim3(1), 0, s, rec, t, nact, krylov, nsub);
}
void copy_alpha0(const KState *ks, double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_alpha0, dim3(1), dim3(1), 0, s, ks, dst);
}
void gather_remap(const uint32_t *keys, int64_t n, const uint64_t *bm, const uint32_t *prefix, const double2 *lam,
                  double2 *mu, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_remap, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, bm, prefix, lam, mu);
}
unsigned long long count_diff(const double2 *a, const double2 *b, int64_t n, unsigned long long *dcount,
                              unsigned long long *hcount, hipStream_t s)
{
    fill_u64((uint64_t *)dcount, 1, 0ull, s);
    if (n > 0) hipLaunchKernelGGL(k_count_diff, dim3(nblocks(n)), dim3(TB), 0, s, a, b, n, dcount);
    (void)hipMemcpyAsync(hcount, dcount, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    return *hcount;
}
void mark_keys_wave(const uint32_t *keys, int64_t n, uint64_t *bm, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mark_wave, dim3(nblocks(n)), dim3(TB), 0, s, keys, n, bm);
}
void adj_q(const KState *kf, const KState *kb, double dt, double2 *Q, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_q, dim3(1), dim3(1024), 0, s, kf, kb, dt, Q);
}
template <class C>
void adj_reduce(const C *Vb, const C *Wb, int64_t ld, const double2 *psi, const double2 *mu, const KState *kf,
                const KState *kb, const double2 *Q, const uint32_t *keys, int64_t n, const GridDesc &g,
                const DerivDesc &dd, double2 *partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_reduce<C>, dim3(RED_BLOCKS), dim3(TB), 0, s, Vb, Wb, ld, psi, mu, kf, kb, Q, keys, n, g,
                       dd, partial);
}
template void adj_reduce<double2>(const double2 *, const double2 *, int64_t, const double2 *, const double2 *,
                                  const KState *, const KState *, const double2 *, const uint32_t *, int64_t,
                                  const GridDesc &, const DerivDesc &, double2 *, hipStream_t);
template void adj_reduce<float2>(const float2 *, const float2 *, int64_t, const double2 *, const double2 *,
                                 const KState *, const KState *, const double2 *, const uint32_t *, int64_t,
                                 const GridDesc &, const DerivDesc &, double2 *, hipStream_t);
void adj_accumulate(const double2 *partial, int nparam, double2 coef, double2 *dC, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_accumulate, dim3(1), dim3(TB), 0, s, partial, RED_BLOCKS, nparam, coef, dC);
}
void adj_packet(const uint32_t *keys, int64_t n, const GridDesc &g, const double2 *tabs, const double2 *dtabs,
                int nmax, const double2 *vec, int bra, double2 *partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_packet, dim3(RED_BLOCKS), dim3(TB), 0, s, keys, n, g, tabs, dtabs, nmax, vec, bra,
                       partial);
}

// ---- full-grid transform (C(2t) on lattice bases) ---------------------------
// y[I] = sum_j B[l][j] x[I with digit k -> j], l = i_k: the dense transform of
// a full-grid tensor along dimension k (stride of digit k, nk its size).
__global__ void k_modek(const double2 *__restrict__ x, double2 *__restrict__ y, int64_t total, int64_t stride, int nk,
                        const double2 *__restrict__ B)
{
    for (int64_t I = gid(); I < total; I += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)((I / stride) % nk);
        const int64_t base = I - (int64_t)l * stride;
        double re = 0.0, im = 0.0;
        for (int j = 0; j < nk; ++j) {
            const double2 b = B[l * nk + j], v = x[base + (int64_t)j * stride];
            re += b.x * v.x - b.y * v.y;
            im += b.x * v.y + b.y * v.x;
        }
        y[I] = make_double2(re, im);
    }
}

__global__ void k_scatter_full(const uint32_t *keys, const double2 *psi, int64_t n, double2 *full)
{
    const int64_t p = gid();
    if (p < n) full[keys[p]] = psi[p];
}

void scatter_full(const uint32_t *keys, const double2 *psi, int64_t n, double2 *full, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter_full, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, psi, n, full);
}

void transform_full(const double2 *x, double2 *y, int64_t total, int64_t stride, int nk, const double2 *B,
                    hipStream_t s)
{
    const int64_t nb = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_modek, dim3((unsigned)nb), dim3(256), 0, s, x, y, total, stride, nk, B);
}

// ---- diagonal factors of a product term -------------------------------------
// y (= or +=) w D(I) x_I with D(I) = prod over the dimensions in `use` of
// tab[k][i_k]: the diagonal (DVR) factors of a sum-of-products term.  They
// commute with the truncation to the active set, so they act on the input of
// the term's chain of dense factors.  D is formed in FP64 in increasing k.
template <class C>
__global__ void k_diag_scale(const uint32_t *keys, const C *x, int64_t n, GridDesc g, const double *tab, int nmax,
                             unsigned use, double2 w, C *y, int acc, const int *skip_if, int skip_j)
{
    if (skip_if && skip_j >= *skip_if) return;
    const int64_t p = gid();
    if (p >= n) return;
    const uint32_t key = keys[p];
    double d = 1.0;
#pragma unroll
    for (int k = 0; k < MAXD; ++k)
        if (k < g.D && ((use >> k) & 1u)) d *= tab[k * nmax + (int)((key / g.stride[k]) % (uint32_t)g.n[k])];
    const double wr = w.x * d, wi = w.y * d;
    const C v = x[p];
    const double vr = v.x, vi = v.y;
    double r = wr * vr - wi * vi, i = wr * vi + wi * vr;
    if (acc) {
        r += y[p].x;
        i += y[p].y;
    }
    C o;
    o.x = r;
    o.y = i;
    y[p] = o;
}

template <class C>
void diag_scale(const uint32_t *keys, const C *x, int64_t n, const GridDesc &g, const double *tab, int nmax,
                unsigned use, double2 w, C *y, bool acc, const int *skip_if, int skip_j, hipStream_t s)
{
    if (n <= 0) return;
    const int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_diag_scale<C>, dim3(nb), dim3(256), 0, s, keys, x, n, g, tab, nmax, use, w, y, acc ? 1 : 0,
                       skip_if, skip_j);
}
template void diag_scale<double2>(const uint32_t *, const double2 *, int64_t, const GridDesc &, const double *, int,
                                  unsigned, double2, double2 *, bool, const int *, int, hipStream_t);
template void diag_scale<float2>(const uint32_t *, const float2 *, int64_t, const GridDesc &, const double *, int,
                                 unsigned, double2, float2 *, bool, const int *, int, hipStream_t);

void copy_meff(const KState *ks, double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_meff, dim3(1), dim3(1), 0, s, ks, dst);
}
void energy_from_dot(const double2 *partial, int nb, double *rec, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy_from_dot, dim3(1), dim3(TB), 0, s, partial, nb, rec);
}

}  // namespace ppq
