// Pruned tensor transformation along one dimension (the appendix's
// last-dimension fiber product, generalised through per-dimension fiber
// tables instead of a materialised permutation):
//
//   for every fiber f of dimension k (points sharing all digits but i_k) and
//   every digit l present in f:  y[p_l] (+)= sum_{j in f} h_k[l][j] x[p_j]
//
// Layout.  A fiber is (off, mask): mask has bit d set when digit d is
// present; the member with digit d sits at entry off + popcount(mask & (2^d - 1))
// of the dimension's permutation pi_k (identity for the last dimension,
// whose fibers are contiguous runs of the key-sorted state).
//
// Mapping.  One lane per fiber.  Consecutive fibers differ in their lowest
// remaining digit, so at a given digit j neighbouring lanes read neighbouring
// positions: the digit-synchronised gather below is close to coalesced for
// every dimension.  The wavefront's union of masks fixes a window of W
// digits (W from a few width buckets); the window's W x W block of h_k is
// wave-uniform and is read through the scalar cache, so the contraction is
// W^2 FMA pairs per lane with no LDS traffic.  Output positions are
// recomputed per row (they hit in cache) so the row loop can stay rolled.
#include <algorithm>
#include <mutex>

#include "ppq_internal.hpp"

namespace ppq {
namespace {

constexpr int HB = 256;

__device__ inline uint64_t wave_or64(uint64_t v)
{
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        uint32_t lo = __shfl_xor((uint32_t)v, s, 64);
        uint32_t hi = __shfl_xor((uint32_t)(v >> 32), s, 64);
        v |= ((uint64_t)hi << 32) | lo;
    }
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <class R>
struct Cx;
template <>
struct Cx<double> {
    using T = double2;
    __device__ static T make(double a, double b) { return make_double2(a, b); }
};
template <>
struct Cx<float> {
    using T = float2;
    __device__ static T make(float a, float b) { return make_float2(a, b); }
};

// ---- real factor (DVR kinetic), first pass fuses the diagonal potential -----
template <class R, int W, int NMAX, bool FIRST, bool IDENT>
__device__ __forceinline__ void body_real(uint32_t o, uint64_t m, int ws, const uint32_t *__restrict__ pi,
                                          const R *__restrict__ T, const typename Cx<R>::T *__restrict__ x,
                                          const R *__restrict__ V, typename Cx<R>::T *__restrict__ y)
{
    using C = typename Cx<R>::T;
    C xw[W];
#pragma unroll
    for (int jj = 0; jj < W; ++jj) {
        int j = ws + jj;
        xw[jj] = Cx<R>::make(0, 0);
        if ((m >> j) & 1ull) {
            uint32_t pos = o + (uint32_t)__popcll(m & ((1ull << j) - 1ull));
            uint32_t p = IDENT ? pos : pi[pos];
            xw[jj] = x[p];
        }
    }
    const R *Tw = T + ws * NMAX + ws;
    // output rows: rolled loop; the W-wide contraction of each row is unrolled
    // and reads the row of h from the scalar cache
    for (int ll = 0; ll < W; ++ll) {
        R ar = 0, ai = 0;
        const R *Tr = Tw + ll * NMAX;
#pragma unroll
        for (int jj = 0; jj < W; ++jj) {
            R t = Tr[jj];
            ar = fma(t, xw[jj].x, ar);
            ai = fma(t, xw[jj].y, ai);
        }
        int l = ws + ll;
        if ((m >> l) & 1ull) {
            uint32_t pos = o + (uint32_t)__popcll(m & ((1ull << l) - 1ull));
            uint32_t p = IDENT ? pos : pi[pos];
            if (FIRST) {
                R v = V[p];
                C xl = x[p];
                y[p] = Cx<R>::make(fma(v, xl.x, ar), fma(v, xl.y, ai));
            } else {
                C o2 = y[p];
                y[p] = Cx<R>::make(o2.x + ar, o2.y + ai);
            }
        }
    }
}

template <class R, int NMAX, bool FIRST, bool IDENT>
__global__ __launch_bounds__(HB) void k_hpsi_real(const uint32_t *__restrict__ pi, const uint32_t *__restrict__ off,
                                                  const uint64_t *__restrict__ mask, int64_t nf,
                                                  const R *__restrict__ T, const typename Cx<R>::T *__restrict__ x,
                                                  const R *__restrict__ V, typename Cx<R>::T *__restrict__ y,
                                                  const int *skip_if, int skip_j)
{
    if (skip_if && skip_j >= *skip_if) return;
    int64_t f = (int64_t)blockIdx.x * HB + threadIdx.x;
    uint64_t m = 0;
    uint32_t o = 0;
    if (f < nf) {
        m = mask[f];
        o = off[f];
    }
    uint64_t wm = wave_or64(m);
    if (wm == 0) return;
    int wlo = __ffsll((unsigned long long)wm) - 1;
    int whi = 63 - __clzll((long long)wm);
    int width = whi - wlo + 1;
#define PPQ_BODY(W)                                                                        \
    {                                                                                      \
        int ws = wlo < NMAX - (W) ? wlo : NMAX - (W);                                      \
        body_real<R, W, NMAX, FIRST, IDENT>(o, m, ws, pi, T, x, V, y);                     \
        return;                                                                            \
    }
    if constexpr (NMAX >= 8) {
        if (width <= 8) PPQ_BODY(8)
    }
    if constexpr (NMAX >= 16) {
        if (width <= 16) PPQ_BODY(16)
    }
    if constexpr (NMAX >= 24) {
        if (width <= 24) PPQ_BODY(24)
    }
    if constexpr (NMAX >= 32) {
        if (width <= 32) PPQ_BODY(32)
    }
    if constexpr (NMAX >= 48) {
        if (width <= 48) PPQ_BODY(48)
    }
    PPQ_BODY(NMAX)
#undef PPQ_BODY
}

// Accumulating pass with every memory access of the wavefront issued up
// front: positions, x and the old y of all window digits are loaded before the
// contraction, so the output loop has no dependent loads.
// DOT: also returns sum_p conj(x_p) y_p over the fiber (the stored y), the
// lane's share of <x|y> when this pass writes y last.
// STAGE: the positions come from the wavefront's copy of its rank range of
// pi in LDS (sp[rank - r0]) instead of scattered global loads.
template <class R, int W, int NMAX, bool IDENT, bool DOT, bool STAGE = false>
__device__ __forceinline__ double2 body_real_acc(uint32_t o, uint64_t m, int ws, const uint32_t *__restrict__ pi,
                                                 const R *__restrict__ T, const typename Cx<R>::T *__restrict__ x,
                                                 typename Cx<R>::T *__restrict__ y, const uint32_t *sp = nullptr,
                                                 uint32_t r0 = 0)
{
    using C = typename Cx<R>::T;
    C xw[W], yw[W];
    uint32_t pw[W];
#pragma unroll
    for (int jj = 0; jj < W; ++jj) {
        int j = ws + jj;
        pw[jj] = 0;
        if ((m >> j) & 1ull) {
            uint32_t pos = o + (uint32_t)__popcll(m & ((1ull << j) - 1ull));
            pw[jj] = IDENT ? pos : (STAGE ? sp[pos - r0] : pi[pos]);
        }
    }
#pragma unroll
    for (int jj = 0; jj < W; ++jj) {
        xw[jj] = Cx<R>::make(0, 0);
        yw[jj] = Cx<R>::make(0, 0);
        if ((m >> (ws + jj)) & 1ull) {
            xw[jj] = x[pw[jj]];
            yw[jj] = y[pw[jj]];
        }
    }
    const R *Tw = T + ws * NMAX + ws;
    double2 dot = make_double2(0.0, 0.0);
#pragma unroll
    for (int ll = 0; ll < W; ++ll) {
        R ar = yw[ll].x, ai = yw[ll].y;
        const R *Tr = Tw + ll * NMAX;
#pragma unroll
        for (int jj = 0; jj < W; ++jj) {
            R t = Tr[jj];
            ar = fma(t, xw[jj].x, ar);
            ai = fma(t, xw[jj].y, ai);
        }
        if ((m >> (ws + ll)) & 1ull) {
            y[pw[ll]] = Cx<R>::make(ar, ai);
            if (DOT) {
                const double xr = (double)xw[ll].x, xi = (double)xw[ll].y;
                dot.x = fma(xr, (double)ar, fma(xi, (double)ai, dot.x));
                dot.y = fma(xr, (double)ai, fma(-xi, (double)ar, dot.y));
            }
        }
    }
    return dot;
}

// DOT: every block also stores its share of <x|y> (the y this pass leaves)
// in dotp[blockIdx.x], summed over the block in a fixed order.
// STAGE: a wavefront's 64 consecutive fibers cover one contiguous range of
// ranks; it copies that range of pi into LDS with coalesced loads first, so
// the per-digit position lookups read LDS (a lane's lookups otherwise touch
// a cache line of their own for every window digit).
template <class R, int NMAX, bool IDENT, bool DOT, bool STAGE = false>
__global__ __launch_bounds__(HB) void k_hpsi_acc(const uint32_t *__restrict__ pi, const uint32_t *__restrict__ off,
                                                 const uint64_t *__restrict__ mask, int64_t nf,
                                                 const R *__restrict__ T, const typename Cx<R>::T *__restrict__ x,
                                                 typename Cx<R>::T *__restrict__ y, const int *skip_if, int skip_j,
                                                 double2 *__restrict__ dotp)
{
    if (skip_if && skip_j >= *skip_if) return;
    int64_t f = (int64_t)blockIdx.x * HB + threadIdx.x;
    uint64_t m = 0;
    uint32_t o = 0;
    if (f < nf) {
        m = mask[f];
        o = off[f];
    }
    uint64_t wm = wave_or64(m);
    constexpr int SPW = STAGE ? 64 * NMAX : 1;  // a wavefront's ranks: 64 fibers of at most NMAX points
    __shared__ uint32_t s_pi[STAGE ? HB / 64 : 1][SPW];
    uint32_t r0 = 0;
    if constexpr (STAGE) {
        const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
        // the valid fibers are the wavefront's first lanes; their ranks are
        // [o of lane 0, end of the last valid lane)
        const uint64_t valid = __ballot(f < nf);
        uint32_t span = 0;
        if (valid) {
            const int last = 63 - __clzll((long long)valid);
            r0 = (uint32_t)__shfl((int)o, 0, 64);
            span = (uint32_t)__shfl((int)(o + (uint32_t)__popcll(m)), last, 64) - r0;
        }
        for (uint32_t i = (uint32_t)lane; i < span; i += 64) s_pi[wv][i] = pi[r0 + i];
        __syncthreads();
    }
    double2 dot = make_double2(0.0, 0.0);
    if (wm != 0) {
        int wlo = __ffsll((unsigned long long)wm) - 1;
        int whi = 63 - __clzll((long long)wm);
        int width = whi - wlo + 1;
#define PPQ_BODY(W)                                                                                   \
    {                                                                                                 \
        int ws = wlo < NMAX - (W) ? wlo : NMAX - (W);                                                 \
        dot = body_real_acc<R, W, NMAX, IDENT, DOT, STAGE>(o, m, ws, pi, T, x, y,                     \
                                                           STAGE ? s_pi[threadIdx.x >> 6] : nullptr, r0); \
        goto done;                                                                                    \
    }
        if constexpr (NMAX >= 8) {
            if (width <= 8) PPQ_BODY(8)
        }
        if constexpr (NMAX >= 12) {
            if (width <= 12) PPQ_BODY(12)
        }
        if constexpr (NMAX >= 16) {
            if (width <= 16) PPQ_BODY(16)
        }
        if constexpr (NMAX >= 24) {
            if (width <= 24) PPQ_BODY(24)
        }
        if constexpr (NMAX >= 32) {
            if (width <= 32) PPQ_BODY(32)
        }
        PPQ_BODY(NMAX)
#undef PPQ_BODY
    }
done:
    if constexpr (DOT) {
        __shared__ double2 wsum[HB / 64];
#pragma unroll
        for (int s2 = 32; s2 >= 1; s2 >>= 1) {
            dot.x += __shfl_xor(dot.x, s2, 64);
            dot.y += __shfl_xor(dot.y, s2, 64);
        }
        if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = dot;
        __syncthreads();
        if (threadIdx.x == 0) {
            double2 t = wsum[0];
#pragma unroll
            for (int w2 = 1; w2 < HB / 64; ++w2) {
                t.x += wsum[w2].x;
                t.y += wsum[w2].y;
            }
            dotp[blockIdx.x] = t;
        }
    }
}

// ---- complex factor (lattice bases), input a linear combination -----------------
template <class R>
struct CArgs {
    int nin;
    const typename Cx<R>::T *x[4];
    typename Cx<R>::T c[4];
};

template <class R, int W, int NMAX, bool IDENT>
__device__ __forceinline__ void body_cplx(uint32_t o, uint64_t m, int ws, const uint32_t *__restrict__ pi,
                                          const typename Cx<R>::T *__restrict__ H, const CArgs<R> &in,
                                          typename Cx<R>::T *__restrict__ y, bool accumulate)
{
    using C = typename Cx<R>::T;
    C xw[W];
#pragma unroll
    for (int jj = 0; jj < W; ++jj) {
        int j = ws + jj;
        xw[jj] = Cx<R>::make(0, 0);
        if ((m >> j) & 1ull) {
            uint32_t pos = o + (uint32_t)__popcll(m & ((1ull << j) - 1ull));
            uint32_t p = IDENT ? pos : pi[pos];
            C acc = Cx<R>::make(0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i < in.nin) {
                    C v = in.x[i][p];
                    C c = in.c[i];
                    acc.x = fma(c.x, v.x, fma(-c.y, v.y, acc.x));
                    acc.y = fma(c.x, v.y, fma(c.y, v.x, acc.y));
                }
            }
            xw[jj] = acc;
        }
    }
    const C *Hw = H + ws * NMAX + ws;
    for (int ll = 0; ll < W; ++ll) {
        R ar = 0, ai = 0;
        const C *Hr = Hw + ll * NMAX;
#pragma unroll
        for (int jj = 0; jj < W; ++jj) {
            C t = Hr[jj];
            ar = fma(t.x, xw[jj].x, fma(-t.y, xw[jj].y, ar));
            ai = fma(t.x, xw[jj].y, fma(t.y, xw[jj].x, ai));
        }
        int l = ws + ll;
        if ((m >> l) & 1ull) {
            uint32_t pos = o + (uint32_t)__popcll(m & ((1ull << l) - 1ull));
            uint32_t p = IDENT ? pos : pi[pos];
            if (accumulate) {
                C o2 = y[p];
                y[p] = Cx<R>::make(o2.x + ar, o2.y + ai);
            } else {
                y[p] = Cx<R>::make(ar, ai);
            }
        }
    }
}

template <class R, int NMAX, bool IDENT>
__global__ __launch_bounds__(HB) void k_hpsi_cplx(const uint32_t *__restrict__ pi, const uint32_t *__restrict__ off,
                                                  const uint64_t *__restrict__ mask, int64_t nf,
                                                  const typename Cx<R>::T *__restrict__ H, CArgs<R> in,
                                                  typename Cx<R>::T *__restrict__ y, int accumulate,
                                                  const int *skip_if, int skip_j)
{
    if (skip_if && skip_j >= *skip_if) return;
    int64_t f = (int64_t)blockIdx.x * HB + threadIdx.x;
    uint64_t m = 0;
    uint32_t o = 0;
    if (f < nf) {
        m = mask[f];
        o = off[f];
    }
    uint64_t wm = wave_or64(m);
    if (wm == 0) return;
    int wlo = __ffsll((unsigned long long)wm) - 1;
    int whi = 63 - __clzll((long long)wm);
    int width = whi - wlo + 1;
#define PPQ_BODY(W)                                                                               \
    {                                                                                             \
        int ws = wlo < NMAX - (W) ? wlo : NMAX - (W);                                             \
        body_cplx<R, W, NMAX, IDENT>(o, m, ws, pi, H, in, y, accumulate != 0);         \
        return;                                                                                   \
    }
    if constexpr (NMAX >= 8) {
        if (width <= 8) PPQ_BODY(8)
    }
    if constexpr (NMAX >= 16) {
        if (width <= 16) PPQ_BODY(16)
    }
    if constexpr (NMAX >= 24) {
        if (width <= 24) PPQ_BODY(24)
    }
    if constexpr (NMAX >= 32) {
        if (width <= 32) PPQ_BODY(32)
    }
    PPQ_BODY(NMAX)
#undef PPQ_BODY
}

// ---- point-parallel form ----------------------------------------------------
// One thread per entry of the dimension's permutation (= one output point).
// A block owns entries [B0, B0+PB); the fibers that straddle its ends are
// completed from a halo on each side (at least NMAX - 1 entries, since a
// fiber has at most n_k members).  The tile and its halos are staged in LDS
// with all their loads issued together, and each thread contracts its own
// row of h_k with its fiber: exactly L^2 multiply-adds per fiber.
constexpr int PB = 256;
constexpr int PH = 64;

template <class R, int NMAX, bool FIRST, bool IDENT>
__global__ __launch_bounds__(PB) void k_hpsi_pt(const uint32_t *__restrict__ pi, const uint8_t *__restrict__ info,
                                                int64_t n, const R *__restrict__ T,
                                                const typename Cx<R>::T *__restrict__ x, const R *__restrict__ V,
                                                typename Cx<R>::T *__restrict__ y, const int *skip_if, int skip_j)
{
    using C = typename Cx<R>::T;
    if (skip_if && skip_j >= *skip_if) return;
    // halo: a fiber has at most NMAX members, so NMAX - 1 entries suffice
    constexpr int PHN = NMAX <= 32 ? 32 : PH;
    constexpr int NW = PB + 2 * PHN;
    __shared__ R sT[NMAX * NMAX];
    __shared__ uint8_t sinfo[NW];
    __shared__ C sx[NW];
    __shared__ uint32_t sp[NW];
    __shared__ int sE;
    const int tid = threadIdx.x;
    const int64_t B0 = (int64_t)blockIdx.x * PB;
    const int64_t W0 = B0 - PHN;
    // every global load of the tile and its halos at once: positions, fiber
    // info, x, and V for the tile's own points
    uint32_t pw[2];
    uint8_t iw[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = tid + u * PB;
        const int64_t q = W0 + i;
        const bool in = i < NW && q >= 0 && q < n;
        iw[u] = in ? info[q] : (uint8_t)0x80;
        pw[u] = in ? (IDENT ? (uint32_t)q : pi[q]) : 0xffffffffu;
    }
    C xw[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) xw[u] = pw[u] != 0xffffffffu ? x[pw[u]] : Cx<R>::make(0, 0);
    const int64_t qo = B0 + tid;
    R vv = 0;
    if (FIRST && qo < n) vv = V[IDENT ? (uint32_t)qo : pi[qo]];
    for (int i = tid; i < NMAX * NMAX; i += PB) sT[i] = T[i];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = tid + u * PB;
        if (i < NW) {
            sinfo[i] = iw[u];
            sp[i] = pw[u];
            sx[i] = xw[u];
        }
    }
    __syncthreads();
    // end of the tile's last fiber: the first fiber start in the upper halo
    // (one ballot of the second wavefront)
    if ((tid >> 6) == 1) {
        const int e = PHN + PB + (tid & 63);
        const uint64_t b = __ballot(e >= NW || (sinfo[e] & 0x80) != 0);
        if ((tid & 63) == 0) sE = b ? PHN + PB + (__ffsll((unsigned long long)b) - 1) : NW;
    }
    __syncthreads();
    if (qo >= n) return;
    const int E = sE;
    const int i = PHN + tid;
    int fs = i;
    while (!(sinfo[fs] & 0x80)) --fs;
    int fe = i + 1;
    while (fe < E && !(sinfo[fe] & 0x80)) ++fe;
    const R *Tr = sT + (sinfo[i] & 63) * NMAX;
    R ar = 0, ai = 0;
    for (int j = fs; j < fe; ++j) {
        R t = Tr[sinfo[j] & 63];
        C v = sx[j];
        ar = fma(t, v.x, ar);
        ai = fma(t, v.y, ai);
    }
    const uint32_t p = sp[i];
    if (FIRST) {
        C xv = sx[i];
        y[p] = Cx<R>::make(fma(vv, xv.x, ar), fma(vv, xv.y, ai));
    } else {
        C o2 = y[p];
        y[p] = Cx<R>::make(o2.x + ar, o2.y + ai);
    }
}

template <class R>
void launch_pt(const uint32_t *pi, const uint8_t *info, int64_t n, int nmax, const R *T, const typename Cx<R>::T *x,
               const R *V, typename Cx<R>::T *y, bool first, const int *skip_if, int skip_j, hipStream_t s)
{
    if (n <= 0) return;
    unsigned nb = (unsigned)((n + PB - 1) / PB);
    bool ident = pi == nullptr;
#define L(NM, F, I) \
    hipLaunchKernelGGL((k_hpsi_pt<R, NM, F, I>), dim3(nb), dim3(PB), 0, s, pi, info, n, T, x, V, y, skip_if, skip_j)
#define DISPATCH(NM)                   \
    if (first) {                       \
        if (ident) L(NM, true, true);  \
        else L(NM, true, false);       \
    } else {                           \
        if (ident) L(NM, false, true); \
        else L(NM, false, false);      \
    }
    switch (nmax) {
    case 8: DISPATCH(8) break;
    case 16: DISPATCH(16) break;
    case 24: DISPATCH(24) break;
    case 32: DISPATCH(32) break;
    case 48: DISPATCH(48) break;
    default: DISPATCH(64) break;
    }
#undef DISPATCH
#undef L
}

// ---- matrix-core form -------------------------------------------------------
// A wavefront takes 16 consecutive fibers.  Their union of digits fixes a
// window of 16*NT digits; the contraction Y = h_window X is a 16*NT x 16*NT
// by 16*NT x 16 dense product, issued as 16x16x4 tiles
// (v_mfma_f32_16x16x4f32 or v_mfma_f64_16x16x4f64): A = a 16x4 block of h
// (lane i + 16 k holds h[row i][column k]), B = the fibers' values at 4
// digits (lane j + 16 k holds fiber j at the k-th digit of the step).  The
// accumulator holds D[4 (l/16) + r][l % 16] (FP32) or D[l/16 + 4 r][l % 16]
// (FP64) in element r of lane l.  A real factor takes one product per part
// (re, im); a complex factor four.  h is stored zero-padded to 64 x 64.
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int MFB = 256;  // 4 wavefronts, 64 fibers per block
constexpr int MFP = 64;   // padded size of h

template <class R>
struct Mma;
template <>
struct Mma<float> {
    using V4 = floatx4;
    __device__ static V4 op(float a, float b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // row of the accumulator's element r in lane group kr, and the digit fed
    // by lane group k at step kb: the same map, so a lane holds outputs at
    // exactly the digits it feeds
    __device__ static int row(int k, int r) { return 4 * k + r; }
};
template <>
struct Mma<double> {
    using V4 = doublex4;
    __device__ static V4 op(double a, double b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int k, int r) { return k + 4 * r; }
};

// Inputs of a matrix-core pass: x = sum_i c_i x_i (one unweighted input for
// real factors).
template <class R>
struct MfIn {
    int nin;
    const typename Cx<R>::T *x[4];
    typename Cx<R>::T c[4];
};

// MODE 0: y = h x; 1: y += h x; 2: y = h x + V x (first pass, potential fused)
template <class R, bool CPLX, int NT, int MODE, bool IDENT>
__device__ __forceinline__ void body_mf(uint32_t o, uint64_t m, int ws, int lane, const uint32_t *__restrict__ pi,
                                        const void *__restrict__ Hv, const MfIn<R> &in, const R *__restrict__ V,
                                        typename Cx<R>::T *__restrict__ y)
{
    using C = typename Cx<R>::T;
    using M = Mma<R>;
    const int col = lane & 15, kr = lane >> 4;
    constexpr int NK = 4 * NT;
    uint32_t pp[NK];
    C xin[NK], yold[NK];
    R vv[NK];
#pragma unroll
    for (int kb = 0; kb < NK; ++kb) {
        const int d = ws + 16 * (kb >> 2) + M::row(kr, kb & 3);
        pp[kb] = 0xffffffffu;
        if ((m >> d) & 1ull) {
            const uint32_t pos = o + (uint32_t)__popcll(m & ((1ull << d) - 1ull));
            pp[kb] = IDENT ? pos : pi[pos];
        }
    }
#pragma unroll
    for (int kb = 0; kb < NK; ++kb) {
        xin[kb] = Cx<R>::make(0, 0);
        yold[kb] = Cx<R>::make(0, 0);
        vv[kb] = 0;
        if (pp[kb] != 0xffffffffu) {
            if (CPLX) {
                C acc = Cx<R>::make(0, 0);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (i < in.nin) {
                        const C v = in.x[i][pp[kb]];
                        const C c = in.c[i];
                        acc.x = fma(c.x, v.x, fma(-c.y, v.y, acc.x));
                        acc.y = fma(c.x, v.y, fma(c.y, v.x, acc.y));
                    }
                }
                xin[kb] = acc;
            } else {
                xin[kb] = in.x[0][pp[kb]];
            }
            if (MODE == 2) vv[kb] = V[pp[kb]];
            if (MODE == 1) yold[kb] = y[pp[kb]];
        }
    }
    typename M::V4 accr[NT], acci[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        accr[t] = typename M::V4{0, 0, 0, 0};
        acci[t] = typename M::V4{0, 0, 0, 0};
    }
#pragma unroll
    for (int kb = 0; kb < NK; ++kb) {
        const int j = ws + 16 * (kb >> 2) + M::row(kr, kb & 3);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int hi = (ws + 16 * t + col) * MFP + j;
            if (CPLX) {
                const C h = reinterpret_cast<const C *>(Hv)[hi];
                accr[t] = M::op(h.x, xin[kb].x, accr[t]);
                accr[t] = M::op(-h.y, xin[kb].y, accr[t]);
                acci[t] = M::op(h.x, xin[kb].y, acci[t]);
                acci[t] = M::op(h.y, xin[kb].x, acci[t]);
            } else {
                const R a = reinterpret_cast<const R *>(Hv)[hi];
                accr[t] = M::op(a, xin[kb].x, accr[t]);
                acci[t] = M::op(a, xin[kb].y, acci[t]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int kb = 4 * t + r;  // element r of tile t sits at the digit of step kb
            if (pp[kb] != 0xffffffffu) {
                const R ar = accr[t][r], ai = acci[t][r];
                if (MODE == 2) y[pp[kb]] = Cx<R>::make(fma(vv[kb], xin[kb].x, ar), fma(vv[kb], xin[kb].y, ai));
                else if (MODE == 1) y[pp[kb]] = Cx<R>::make(yold[kb].x + ar, yold[kb].y + ai);
                else y[pp[kb]] = Cx<R>::make(ar, ai);
            }
        }
    }
}

template <class R, bool CPLX, int MODE, bool IDENT>
__global__ __launch_bounds__(MFB) void k_hpsi_mf(const uint32_t *__restrict__ pi, const uint32_t *__restrict__ off,
                                                 const uint64_t *__restrict__ mask, int64_t nf,
                                                 const void *__restrict__ H, MfIn<R> in, const R *__restrict__ V,
                                                 typename Cx<R>::T *__restrict__ y, const int *skip_if, int skip_j)
{
    if (skip_if && skip_j >= *skip_if) return;
    const int lane = threadIdx.x & 63;
    const int64_t f = ((int64_t)blockIdx.x * (MFB / 64) + (threadIdx.x >> 6)) * 16 + (lane & 15);
    uint64_t m = 0;
    uint32_t o = 0;
    if (f < nf) {
        m = mask[f];
        o = off[f];
    }
    const uint64_t wm = wave_or64(m);
    if (wm == 0) return;
    const int wlo = __ffsll((unsigned long long)wm) - 1;
    const int whi = 63 - __clzll((long long)wm);
    const int width = whi - wlo + 1;
#define PPQ_MF(NT)                                                              \
    {                                                                           \
        const int ws = wlo < MFP - 16 * (NT) ? wlo : MFP - 16 * (NT);           \
        body_mf<R, CPLX, NT, MODE, IDENT>(o, m, ws, lane, pi, H, in, V, y);     \
        return;                                                                 \
    }
    if (width <= 16) PPQ_MF(1)
    if (width <= 32) PPQ_MF(2)
    if (width <= 48) PPQ_MF(3)
    PPQ_MF(4)
#undef PPQ_MF
}

inline unsigned fblocks(int64_t nf)
{
    int64_t b = (nf + HB - 1) / HB;
    return (unsigned)(b < 1 ? 1 : b);
}

template <class R>
void launch_real(const FiberPass &fp, const R *T, const typename Cx<R>::T *x, const R *V, typename Cx<R>::T *y,
                 bool first, const int *skip_if, int skip_j, hipStream_t s)
{
    if (fp.nf <= 0) return;
    bool ident = fp.pi == nullptr;
#define L(NM, F, I)                                                                                        \
    hipLaunchKernelGGL((k_hpsi_real<R, NM, F, I>), dim3(fblocks(fp.nf)), dim3(HB), 0, s, fp.pi, fp.off, fp.mask, \
                       fp.nf, T, x, V, y, skip_if, skip_j)
#define DISPATCH(NM)                       \
    if (first) {                           \
        if (ident) L(NM, true, true);      \
        else L(NM, true, false);           \
    } else {                               \
        if (ident) L(NM, false, true);     \
        else L(NM, false, false);          \
    }
    switch (fp.nmax) {
    case 8: DISPATCH(8) break;
    case 16: DISPATCH(16) break;
    case 24: DISPATCH(24) break;
    case 32: DISPATCH(32) break;
    case 48: DISPATCH(48) break;
    default: DISPATCH(64) break;
    }
#undef DISPATCH
#undef L
}

template <class R>
void launch_cplx(const FiberPass &fp, const typename Cx<R>::T *H, const CArgs<R> &in, typename Cx<R>::T *y,
                 bool accumulate, const int *skip_if, int skip_j, hipStream_t s)
{
    if (fp.nf <= 0) return;
    bool ident = fp.pi == nullptr;
#define L(NM, I)                                                                                             \
    hipLaunchKernelGGL((k_hpsi_cplx<R, NM, I>), dim3(fblocks(fp.nf)), dim3(HB), 0, s, fp.pi, fp.off, fp.mask, \
                       fp.nf, H, in, y, accumulate ? 1 : 0, skip_if, skip_j)
#define DISPATCH(NM)        \
    if (ident) L(NM, true); \
    else L(NM, false);
    switch (fp.nmax) {
    case 8: DISPATCH(8) break;
    case 16: DISPATCH(16) break;
    case 24: DISPATCH(24) break;
    case 32: DISPATCH(32) break;
    case 48: DISPATCH(48) break;
    default: DISPATCH(64) break;
    }
#undef DISPATCH
#undef L
}


// ---- block-fused form ----------------------------------------------------------
// The state is cut into blocks of points that share the digits of the
// dimensions NOT handled by the pass; a block then holds every fiber of the
// pass's dimensions through its points.  In the row-major frame the blocks
// are contiguous runs of the key-sorted state (the pass over the inner
// dimensions); in the inner-first frame they are reached through the
// permutation P (the pass over the outer dimensions).  Each dimension's
// fiber order keeps the block's leading digits first, so a block occupies the
// same rank range in the frame and in every fiber order of the pass.
//
// A workgroup takes a chunk of whole blocks, stages x (and y when
// accumulating, plus V x when the potential is fused) in LDS, applies the
// pass's 1D factors one dimension after the other with one lane per fiber
// (x and y from LDS, the factor's window block through the scalar cache),
// and writes y back once: x is read once and y written once per pass instead
// of once per dimension.

template <class R>
struct BlockArgs {
    int ndim;
    const uint32_t *pi[4];
    const uint32_t *off[4];
    const uint64_t *mask[4];
    const uint32_t *fch[4];
    const R *T[4];
    int nb[4];
    const uint32_t *chunk;
    uint32_t nch;
    const uint32_t *P;
    const uint32_t *list;
    uint32_t cap;
    int accumulate;
    const R *V;
    int unroll;  // k_hpsi_blk2: unrolled row loop (1) or rolled with wave-uniform skips (0)
};

// One fiber, one group of 8 output rows: rows ws + 8g .. ws + 8g + 7 of the
// window [ws, ws + W), summed over the window's columns in blocks of 8
// inputs (the factor's entries are wave-uniform and come through the scalar
// cache); the 8 row sums stay in registers and are added to y in LDS once.
constexpr int RG = 4;  // output rows per wave task
constexpr int CB = 8;  // window columns per register block

template <class R, int W>
__device__ __forceinline__ void body_block(uint32_t o, uint64_t m, int ws, int g, uint32_t last, const uint16_t *lp,
                                           const R *__restrict__ T, int nb, const typename Cx<R>::T *xs,
                                           typename Cx<R>::T *ys)
{
    using C = typename Cx<R>::T;
    R ar[RG], ai[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) {
        ar[r] = 0;
        ai[r] = 0;
    }
    // the factor is read-only for the kernel's lifetime: constant address
    // space, so the wave-uniform entries load through the scalar cache
    using CR = __attribute__((address_space(4))) const R;
    CR *Tg = (CR *)(T + (ws + g * RG) * nb + ws);
    // member loads without branches: absent digits read a valid slot and are
    // zeroed, so each group of 8 LDS reads is issued back to back
#pragma unroll 1
    for (int cb = 0; cb < W / CB; ++cb) {
        uint32_t q[CB];
        bool on[CB];
#pragma unroll
        for (int jj = 0; jj < CB; ++jj) {
            const int j = ws + cb * CB + jj;
            on[jj] = (m >> j) & 1ull;
            const uint32_t pos = o + (uint32_t)__popcll(m & ((1ull << j) - 1ull));
            q[jj] = on[jj] ? pos : (o < last ? o : last);
        }
        if (lp) {
#pragma unroll
            for (int jj = 0; jj < CB; ++jj) q[jj] = lp[q[jj]];
        }
        C xw[CB];
#pragma unroll
        for (int jj = 0; jj < CB; ++jj) {
            const C v = xs[q[jj]];
            xw[jj] = on[jj] ? v : Cx<R>::make(0, 0);
        }
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            CR *Tr = Tg + r * nb + cb * CB;
#pragma unroll
            for (int jj = 0; jj < CB; ++jj) {
                const R t = Tr[jj];
                ar[r] = fma(t, xw[jj].x, ar[r]);
                ai[r] = fma(t, xw[jj].y, ai[r]);
            }
        }
    }
    uint32_t q[RG];
    bool on[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) {
        const int l = ws + g * RG + r;
        on[r] = (m >> l) & 1ull;
        const uint32_t pos = o + (uint32_t)__popcll(m & ((1ull << l) - 1ull));
        q[r] = on[r] ? pos : (o < last ? o : last);
    }
    if (lp) {
#pragma unroll
        for (int r = 0; r < RG; ++r) q[r] = lp[q[r]];
    }
    C v[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) v[r] = ys[q[r]];
#pragma unroll
    for (int r = 0; r < RG; ++r)
        if (on[r]) ys[q[r]] = Cx<R>::make(v[r].x + ar[r], v[r].y + ai[r]);
}

template <class T4>
__device__ __forceinline__ T4 pick4(const T4 (&v)[4], int d)
{
    return d == 0 ? v[0] : d == 1 ? v[1] : d == 2 ? v[2] : v[3];
}

// Every global load of a chunk (P, the fiber-order ranks of each dimension,
// each wave's first fiber batch per dimension, then x, y and V through P) is
// issued before the first LDS store, so a chunk waits for memory about three
// times instead of three times per dimension.  NT * SU >= the launch's cap.
template <class R, int NBMAX, int NT, int SU>
__global__ __launch_bounds__(NT) void k_hpsi_block(BlockArgs<R> a, const typename Cx<R>::T *__restrict__ x,
                                                   typename Cx<R>::T *__restrict__ y, const int *skip_if, int skip_j)
{
    using C = typename Cx<R>::T;
    if (skip_if && skip_j >= *skip_if) return;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t ci;
    if (a.list) {
        ci = a.list[blockIdx.x];
    } else {
        // consecutive chunks on one XCD (workgroups are dealt round-robin over 8)
        const uint32_t per = (a.nch + 7) / 8, i = blockIdx.x >> 3;
        ci = (blockIdx.x & 7) * per + i;
        if (i >= per || ci >= a.nch) return;
    }
    const uint32_t c0 = a.chunk[ci], c1 = a.chunk[ci + 1], len = c1 - c0;
    if (len == 0 || len > a.cap) return;
    C *xs = reinterpret_cast<C *>(smem);
    C *ys = xs + a.cap;
    uint16_t *lpb = reinterpret_cast<uint16_t *>(ys + a.cap);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int nd = a.ndim;

    uint32_t p[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
        const uint32_t i = u * NT + tid;
        p[u] = i < len ? (a.P ? a.P[c0 + i] : c0 + i) : 0xffffffffu;
    }
    // fiber-order ranks -> local frame ranks, dimensions with a permutation
    uint32_t q[3][SU];
    int slot[4];
    int ns = 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        slot[d] = -1;
        if (d < nd && a.pi[d]) {
            slot[d] = ns;
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const uint32_t i = u * NT + tid;
                if (ns == 0) q[0][u] = i < len ? a.pi[d][c0 + i] - c0 : 0u;
                else if (ns == 1) q[1][u] = i < len ? a.pi[d][c0 + i] - c0 : 0u;
                else q[2][u] = i < len ? a.pi[d][c0 + i] - c0 : 0u;
            }
            ++ns;
        }
    }
    // first fiber batch of this wave in every dimension
    uint32_t fa[4], fb[4], o0[4];
    uint64_t m0[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        fa[d] = fb[d] = 0;
        m0[d] = 0;
        o0[d] = 0;
        if (d < nd) {
            fa[d] = a.fch[d][ci];
            fb[d] = a.fch[d][ci + 1];
            const uint32_t f = fa[d] + (uint32_t)(wave / (a.nb[d] / RG)) * 64 + (uint32_t)lane;
            if (f < fb[d]) {
                m0[d] = a.mask[d][f];
                o0[d] = a.off[d][f] - c0;
            }
        }
    }
    {
        C xv[SU], yv[SU];
        R vv[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            xv[u] = Cx<R>::make(0, 0);
            yv[u] = Cx<R>::make(0, 0);
            vv[u] = 0;
            if (p[u] != 0xffffffffu) {
                xv[u] = x[p[u]];
                if (a.accumulate) yv[u] = y[p[u]];
                if (a.V) vv[u] = a.V[p[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const uint32_t i = u * NT + tid;
            if (i < len) {
                xs[i] = xv[u];
                ys[i] = a.V ? Cx<R>::make(fma(vv[u], xv[u].x, yv[u].x), fma(vv[u], xv[u].y, yv[u].y)) : yv[u];
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (k < ns) lpb[k * a.cap + i] = (uint16_t)q[k][u];
            }
        }
    }
    __syncthreads();
    for (int d = 0; d < nd; ++d) {
        const uint32_t *off = a.off[d];
        const int sl = d == 0 ? slot[0] : d == 1 ? slot[1] : d == 2 ? slot[2] : slot[3];
        const uint16_t *lq = sl >= 0 ? lpb + sl * a.cap : nullptr;
        const uint32_t f0 = pick4(fa, d), f1 = pick4(fb, d);
        const R *T = a.T[d];
        const int nb = a.nb[d];
        const int G = nb / RG;
        const uint64_t *mk = a.mask[d];
        // wave tasks: (batch of 64 consecutive fibers, group of 8 output rows)
        const uint32_t ntask = (f1 - f0 + 63) / 64 * (uint32_t)G;
        for (uint32_t task = (uint32_t)wave; task < ntask; task += NT / 64) {
            const uint32_t batch = task / (uint32_t)G;
            const int g = (int)(task - batch * (uint32_t)G);
            uint64_t m;
            uint32_t o;
            if (batch == (uint32_t)(wave / G)) {
                m = pick4(m0, d);
                o = pick4(o0, d);
            } else {
                const uint32_t f = f0 + batch * 64 + (uint32_t)lane;
                m = 0;
                o = 0;
                if (f < f1) {
                    m = mk[f];
                    o = off[f] - c0;
                }
            }
            const uint64_t wm = wave_or64(m);
            const int wlo = __ffsll((unsigned long long)wm) - 1;
            const int whi = 63 - __clzll((long long)wm);
            const int width = whi - wlo + 1;
#define PPQ_BLK(W)                                                          \
    {                                                                       \
        if (g * RG >= (W)) continue;                                        \
        const int ws = wlo < nb - (W) ? wlo : nb - (W);                     \
        body_block<R, W>(o, m, ws, g, len - 1, lq, T, nb, xs, ys);          \
        continue;                                                           \
    }
            if (width <= 8) PPQ_BLK(8)
            if constexpr (NBMAX >= 16) {
                if (width <= 16) PPQ_BLK(16)
            }
            if constexpr (NBMAX >= 24) {
                if (width <= 24) PPQ_BLK(24)
            }
            if constexpr (NBMAX >= 32) {
                if (width <= 32) PPQ_BLK(32)
            }
#undef PPQ_BLK
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
        const uint32_t i = u * NT + tid;
        if (i < len) y[p[u]] = ys[i];
    }
}

// ---- long fibers (dimensions of more than 64 points) --------------------------
// One wavefront per fiber (a one-wave workgroup).  The fiber's members (their
// positions, digits and input values, up to 256) are staged in LDS; each lane
// then computes the output of members lane, lane + 64, ...: the row of h at
// the member's digit against the members' values, exactly L^2 products per
// fiber.  h is the unpadded n x n factor (real, or complex interleaved).
// MODE 0: y = h x; 1: y += h x; 2: y = h x + V x.  x is the weighted sum of
// up to four inputs (one unweighted input for real factors).
constexpr int LB = 64;

template <class R, bool CPLX, int MODE>
__global__ __launch_bounds__(LB) void k_hpsi_long(const uint32_t *__restrict__ pi, const uint32_t *__restrict__ off,
                                                  const uint8_t *__restrict__ dig, int64_t nf, int n,
                                                  const void *__restrict__ Hv, MfIn<R> in, const R *__restrict__ V,
                                                  typename Cx<R>::T *__restrict__ y, const int *skip_if, int skip_j)
{
    using C = typename Cx<R>::T;
    if (skip_if && skip_j >= *skip_if) return;
    const int64_t f = blockIdx.x;
    if (f >= nf) return;
    __shared__ C sx[NMAX_FIBER];
    __shared__ uint32_t sp[NMAX_FIBER];
    __shared__ int sd[NMAX_FIBER];
    const uint32_t q0 = off[f];
    const int L = (int)(off[f + 1] - q0);
    const int lane = threadIdx.x;
    for (int t = lane; t < L; t += LB) {
        const uint32_t q = q0 + (uint32_t)t;
        const uint32_t p = pi ? pi[q] : q;
        C v;
        if (CPLX) {
            v = Cx<R>::make(0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i < in.nin) {
                    const C u = in.x[i][p];
                    const C c = in.c[i];
                    v.x = fma(c.x, u.x, fma(-c.y, u.y, v.x));
                    v.y = fma(c.x, u.y, fma(c.y, u.x, v.y));
                }
            }
        } else {
            v = in.x[0][p];
        }
        sx[t] = v;
        sp[t] = p;
        sd[t] = dig[q];
    }
    __syncthreads();
    for (int t = lane; t < L; t += LB) {
        const int l = sd[t];
        R ar = 0, ai = 0;
        if (CPLX) {
            const C *Hr = reinterpret_cast<const C *>(Hv) + (size_t)l * n;
            for (int u = 0; u < L; ++u) {
                const C h = Hr[sd[u]];
                const C v = sx[u];
                ar = fma(h.x, v.x, fma(-h.y, v.y, ar));
                ai = fma(h.x, v.y, fma(h.y, v.x, ai));
            }
        } else {
            const R *Hr = reinterpret_cast<const R *>(Hv) + (size_t)l * n;
            for (int u = 0; u < L; ++u) {
                const R h = Hr[sd[u]];
                const C v = sx[u];
                ar = fma(h, v.x, ar);
                ai = fma(h, v.y, ai);
            }
        }
        const uint32_t p = sp[t];
        if (MODE == 2) {
            const R vv = V[p];
            const C xv = sx[t];
            y[p] = Cx<R>::make(fma(vv, xv.x, ar), fma(vv, xv.y, ai));
        } else if (MODE == 1) {
            const C o2 = y[p];
            y[p] = Cx<R>::make(o2.x + ar, o2.y + ai);
        } else {
            y[p] = Cx<R>::make(ar, ai);
        }
    }
}

template <class R, bool CPLX>
void launch_long(const LongPass &lp, const void *H, const MfIn<R> &in, const R *V, typename Cx<R>::T *y, int mode,
                 const int *skip_if, int skip_j, hipStream_t s)
{
    if (lp.nf <= 0) return;
#define L(MD)                                                                                                     \
    hipLaunchKernelGGL((k_hpsi_long<R, CPLX, MD>), dim3((unsigned)lp.nf), dim3(LB), 0, s, lp.pi, lp.off, lp.dig, \
                       lp.nf, lp.n, H, in, V, y, skip_if, skip_j)
    if (mode == 2) L(2);
    else if (mode == 1) L(1);
    else L(0);
#undef L
}

// ---- block-fused form, one lane per fiber over the whole window -------------
// Same chunks as k_hpsi_block (whole blocks of the pass, x and y staged in
// LDS, y written once), but each lane loads its fiber's window of x from LDS
// once and computes every output row of the window (rolled loop; rows no
// lane of the wavefront holds are skipped), adding each to y in LDS.  A
// wave task is a batch of 64 fibers, so a chunk should hold a few hundred
// fibers per dimension for every wavefront of the workgroup to get work.
template <class R, int W>
__device__ __forceinline__ void body_blk2(uint32_t o, uint64_t m, uint64_t wm, int ws, const uint16_t *lq,
                                          const R *__restrict__ T, int nb, const typename Cx<R>::T *xs,
                                          typename Cx<R>::T *ys)
{
    using C = typename Cx<R>::T;
    using CR = __attribute__((address_space(4))) const R;
    C xw[W];
    {
        uint32_t q[W];
        bool on[W];
#pragma unroll
        for (int jj = 0; jj < W; ++jj) {
            const int j = ws + jj;
            on[jj] = (m >> j) & 1ull;
            q[jj] = on[jj] ? o + (uint32_t)__popcll(m & ((1ull << j) - 1ull)) : o;
        }
        if (lq) {
#pragma unroll
            for (int jj = 0; jj < W; ++jj) q[jj] = lq[q[jj]];
        }
#pragma unroll
        for (int jj = 0; jj < W; ++jj) {
            const C v = xs[q[jj]];
            xw[jj] = on[jj] ? v : Cx<R>::make(0, 0);
        }
    }
    CR *Tw = (CR *)(T + ws * nb + ws);
#pragma unroll 1
    for (int ll = 0; ll < W; ++ll) {
        const int l = ws + ll;
        if (!((wm >> l) & 1ull)) continue;  // wave-uniform
        CR *Tr = Tw + ll * nb;
        R ar = 0, ai = 0;
#pragma unroll
        for (int jj = 0; jj < W; ++jj) {
            const R t = Tr[jj];
            ar = fma(t, xw[jj].x, ar);
            ai = fma(t, xw[jj].y, ai);
        }
        if ((m >> l) & 1ull) {
            uint32_t q = o + (uint32_t)__popcll(m & ((1ull << l) - 1ull));
            if (lq) q = lq[q];
            const C v = ys[q];
            ys[q] = Cx<R>::make(v.x + ar, v.y + ai);
        }
    }
}

// The same contraction with the row loop unrolled: the factor's window comes
// through the scalar cache for every row at once, so the loads of later rows
// overlap the arithmetic of earlier ones; absent rows are predicated off.
template <class R, int W>
__device__ __forceinline__ void body_blk2u(uint32_t o, uint64_t m, int ws, const uint16_t *lq,
                                           const R *__restrict__ T, int nb, const typename Cx<R>::T *xs,
                                           typename Cx<R>::T *ys)
{
    using C = typename Cx<R>::T;
    using CR = __attribute__((address_space(4))) const R;
    C xw[W];
    uint32_t q[W];
    bool on[W];
#pragma unroll
    for (int jj = 0; jj < W; ++jj) {
        const int j = ws + jj;
        on[jj] = (m >> j) & 1ull;
        q[jj] = on[jj] ? o + (uint32_t)__popcll(m & ((1ull << j) - 1ull)) : o;
    }
    if (lq) {
#pragma unroll
        for (int jj = 0; jj < W; ++jj) q[jj] = lq[q[jj]];
    }
#pragma unroll
    for (int jj = 0; jj < W; ++jj) {
        const C v = xs[q[jj]];
        xw[jj] = on[jj] ? v : Cx<R>::make(0, 0);
    }
    CR *Tw = (CR *)(T + ws * nb + ws);
#pragma unroll
    for (int ll = 0; ll < W; ++ll) {
        CR *Tr = Tw + ll * nb;
        R ar = 0, ai = 0;
#pragma unroll
        for (int jj = 0; jj < W; ++jj) {
            const R t = Tr[jj];
            ar = fma(t, xw[jj].x, ar);
            ai = fma(t, xw[jj].y, ai);
        }
        if (on[ll]) {
            const C v = ys[q[ll]];
            ys[q[ll]] = Cx<R>::make(v.x + ar, v.y + ai);
        }
    }
}

template <class R, int NBMAX, int NT, int SU>
__global__ __launch_bounds__(NT) void k_hpsi_blk2(BlockArgs<R> a, const typename Cx<R>::T *__restrict__ x,
                                                  typename Cx<R>::T *__restrict__ y, const int *skip_if, int skip_j)
{
    using C = typename Cx<R>::T;
    if (skip_if && skip_j >= *skip_if) return;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t ci;
    if (a.list) {
        ci = a.list[blockIdx.x];
    } else {
        // consecutive chunks on one XCD (workgroups are dealt round-robin over 8)
        const uint32_t per = (a.nch + 7) / 8, i = blockIdx.x >> 3;
        ci = (blockIdx.x & 7) * per + i;
        if (i >= per || ci >= a.nch) return;
    }
    const uint32_t c0 = a.chunk[ci], c1 = a.chunk[ci + 1], len = c1 - c0;
    if (len == 0 || len > a.cap) return;
    C *xs = reinterpret_cast<C *>(smem);
    C *ys = xs + a.cap;
    uint16_t *lpb = reinterpret_cast<uint16_t *>(ys + a.cap);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int nd = a.ndim;
    // stage the chunk: positions, x, y or V x, and the local frame rank of
    // every fiber-order rank of the permuted dimensions; all loads first
    uint32_t p[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
        const uint32_t i = u * NT + tid;
        p[u] = i < len ? (a.P ? a.P[c0 + i] : c0 + i) : 0xffffffffu;
    }
    int slot[4];
    int ns = 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        slot[d] = -1;
        if (d < nd && a.pi[d]) slot[d] = ns++;
    }
    {
        C xv[SU], yv[SU];
        R vv[SU];
        uint16_t lr[3][SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            xv[u] = Cx<R>::make(0, 0);
            yv[u] = Cx<R>::make(0, 0);
            vv[u] = 0;
            const uint32_t i = u * NT + tid;
            if (p[u] != 0xffffffffu) {
                xv[u] = x[p[u]];
                if (a.accumulate) yv[u] = y[p[u]];
                if (a.V) vv[u] = a.V[p[u]];
            }
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int sl = slot[d];
                if (sl >= 0 && sl < 3) lr[sl][u] = i < len ? (uint16_t)(a.pi[d][c0 + i] - c0) : (uint16_t)0;
            }
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const uint32_t i = u * NT + tid;
            if (i < len) {
                xs[i] = xv[u];
                ys[i] = a.V ? Cx<R>::make(fma(vv[u], xv[u].x, yv[u].x), fma(vv[u], xv[u].y, yv[u].y)) : yv[u];
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (k < ns) lpb[k * a.cap + i] = lr[k][u];
            }
        }
    }
    __syncthreads();
    for (int d = 0; d < nd; ++d) {
        const int sl = d == 0 ? slot[0] : d == 1 ? slot[1] : d == 2 ? slot[2] : slot[3];
        const uint16_t *lq = sl >= 0 ? lpb + sl * a.cap : nullptr;
        const uint32_t f0 = a.fch[d][ci], f1 = a.fch[d][ci + 1];
        const uint32_t *off = a.off[d];
        const uint64_t *mk = a.mask[d];
        const R *T = a.T[d];
        const int nb = a.nb[d];
        const uint32_t nbatch = (f1 - f0 + 63) / 64;
        for (uint32_t b = (uint32_t)wave; b < nbatch; b += NT / 64) {
            const uint32_t f = f0 + b * 64 + (uint32_t)lane;
            uint64_t m = 0;
            uint32_t o = 0;
            if (f < f1) {
                m = mk[f];
                o = off[f] - c0;
            }
            const uint64_t wm = wave_or64(m);
            if (wm == 0) continue;
            const int wlo = __ffsll((unsigned long long)wm) - 1;
            const int whi = 63 - __clzll((long long)wm);
            const int width = whi - wlo + 1;
#define PPQ_B2(WW)                                                          \
    {                                                                       \
        const int ws = wlo < nb - (WW) ? wlo : nb - (WW);                   \
        if (a.unroll) body_blk2u<R, WW>(o, m, ws, lq, T, nb, xs, ys);      \
        else body_blk2<R, WW>(o, m, wm, ws, lq, T, nb, xs, ys);             \
        continue;                                                           \
    }
            if (width <= 8) PPQ_B2(8)
            if constexpr (NBMAX >= 16) {
                if (width <= 16) PPQ_B2(16)
            }
            if constexpr (NBMAX >= 24) {
                if (width <= 24) PPQ_B2(24)
            }
            if constexpr (NBMAX >= 32) {
                if (width <= 32) PPQ_B2(32)
            }
#undef PPQ_B2
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
        const uint32_t i = u * NT + tid;
        if (i < len) y[p[u]] = ys[i];
    }
}

// ---- plane pass: two adjacent dimensions per pass ----------------------------
// In the pair's frame a plane (every digit but d_a, d_b fixed) is a run of
// frame ranks sorted by (d_a, d_b).  A wavefront takes a task, the planes
// that start in one window of PLANE_WINDOW frame ranks, in rounds of at most
// PLANE_SPAN ranks:
//   1. every member of the round is loaded at once, 12 per lane (digits and
//      position, then x and the base value: y, or V x on the first pass);
//   2. plane by plane over the planes the round holds whole (bit 15 of the
//      digits marks a plane's last member), the members scatter x into a dense
//      n_a x n_b tile in the wavefront's own LDS region (absent cells are
//      zero), the bounding box comes from two wavefront reductions, and
//        Y[i][l] = sum_k h_a[i][k] X[k][l] + sum_j X[i][j] h_b[l][j]
//      is formed over the box with 16x16x4 matrix-core steps: both products
//      accumulate into the same 16 x 16 blocks (rows d_a, columns d_b), real
//      and imaginary parts apart.  The blocks go back over the box, every
//      member adds its cell to its base value, and the box is cleared;
//   3. the members of those planes store y; a plane cut by the round's end
//      starts the next round.
// The two factors sit in LDS once per workgroup.  A point's x and base value
// are read once and its y written once per pair of dimensions, where the
// per-dimension passes read and write y once per dimension.
__device__ inline uint32_t min2_u16(uint32_t u, uint32_t v)
{
    return (min(u >> 16, v >> 16) << 16) | min(u & 0xffffu, v & 0xffffu);
}
__device__ inline uint32_t max2_u16(uint32_t u, uint32_t v)
{
    return (max(u >> 16, v >> 16) << 16) | max(u & 0xffffu, v & 0xffffu);
}
__device__ inline uint32_t wave_min2_u16(uint32_t v)
{
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v = min2_u16(v, (uint32_t)__shfl_xor((int)v, s, 64));
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ inline uint32_t wave_max2_u16(uint32_t v)
{
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v = max2_u16(v, (uint32_t)__shfl_xor((int)v, s, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

constexpr int PLB = 256;               // 4 wavefronts per workgroup, one task each
constexpr int PLU = PLANE_SPAN / 64;   // round members per lane
constexpr uint32_t PL_END = 0x8000u;   // last member of its plane

// Y over the box, one 16 x 16 block (rows d_a, columns d_b) at a time: the
// block goes to the wavefront's block buffer Yr/Yi ([row][column]) and every
// member of the plane (round slots [r0, r1)) whose cell lies in it adds it to
// its base value.  X stays intact until the whole box is done.
template <class R>
__device__ __forceinline__ void plane_blocks(int a0, int a1, int b0, int b1, int na, int nb, int lane, int r0,
                                             int r1, const uint32_t (&dg)[PLU], typename Cx<R>::T (&base)[PLU],
                                             const R *__restrict__ sTa, const R *__restrict__ sTb, const R *Xr,
                                             const R *Xi, R *Yr, R *Yi)
{
    using M = Mma<R>;
    const int col = lane & 15, kr = lane >> 4;
    const int Ra = a1 - a0 + 1, Rb = b1 - b0 + 1;
    for (int i0 = a0; i0 <= a1; i0 += 16) {
        for (int l0 = b0; l0 <= b1; l0 += 16) {
            typename M::V4 accr{0, 0, 0, 0}, acci{0, 0, 0, 0};
            const int i = i0 + col, l = l0 + col;
            // dimension b: A = X[i][j] (rows of the tile), B = h_b[l][j]
            for (int s = 0; s < (Rb + 3) >> 2; ++s) {
                const int j = b0 + 4 * s + kr;
                const bool ok = i < na && j < nb;
                const R xr = ok ? Xr[i * nb + j] : R(0), xi = ok ? Xi[i * nb + j] : R(0);
                const R tb = (l < nb && j < nb) ? sTb[l * nb + j] : R(0);
                accr = M::op(xr, tb, accr);
                acci = M::op(xi, tb, acci);
            }
            // dimension a: A = h_a[i][k], B = X[k][l] (columns of the tile)
            for (int s = 0; s < (Ra + 3) >> 2; ++s) {
                const int k = a0 + 4 * s + kr;
                const R ta = (i < na && k < na) ? sTa[i * na + k] : R(0);
                const bool ok = l < nb && k < na;
                const R xr = ok ? Xr[k * nb + l] : R(0), xi = ok ? Xi[k * nb + l] : R(0);
                accr = M::op(ta, xr, accr);
                acci = M::op(ta, xi, acci);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Yr[M::row(kr, r) * 16 + col] = accr[r];
                Yi[M::row(kr, r) * 16 + col] = acci[r];
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int u = 0; u < PLU; ++u) {
                if (u * 64 >= r1 || u * 64 + 64 <= r0) continue;
                const int m = u * 64 + lane;
                const int di = (int)((dg[u] >> 8) & 0x7fu) - i0, dl = (int)(dg[u] & 0xffu) - l0;
                if (m >= r0 && m < r1 && di >= 0 && di < 16 && dl >= 0 && dl < 16)
                    base[u] = Cx<R>::make(base[u].x + Yr[di * 16 + dl], base[u].y + Yi[di * 16 + dl]);
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

template <class R>
__global__ __launch_bounds__(PLB, 2) void k_hpsi_plane(PlanePass pp, const R *__restrict__ Ta,
                                                       const R *__restrict__ Tb,
                                                       const typename Cx<R>::T *__restrict__ x,
                                                       const R *__restrict__ V, typename Cx<R>::T *__restrict__ y,
                                                       int first, const int *skip_if, int skip_j)
{
    using C = typename Cx<R>::T;
    if (skip_if && skip_j >= *skip_if) return;
    // consecutive tasks on one XCD (workgroups are dealt round-robin over 8)
    const uint32_t nwg = (pp.ntask + PLB / 64 - 1) / (PLB / 64);
    const uint32_t per = (nwg + 7) / 8, bi = blockIdx.x >> 3;
    const uint32_t wg = (blockIdx.x & 7) * per + bi;
    if (bi >= per || wg >= nwg) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int na = pp.na, nb = pp.nb, cells = na * nb;
    R *sTa = reinterpret_cast<R *>(smem);
    R *sTb = sTa + na * na;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    R *Xr = sTb + nb * nb + (size_t)wave * (2 * cells + 512);
    R *Xi = Xr + cells;
    R *Yr = Xi + cells;
    R *Yi = Yr + 256;
    const uint32_t t = wg * (PLB / 64) + (uint32_t)wave;
    const bool has = t < pp.ntask;
    const uint32_t T0 = has ? pp.tstart[t] : 0u, T1 = has ? pp.tstart[t + 1] : 0u;
    for (int i = threadIdx.x; i < na * na; i += PLB) sTa[i] = Ta[i];
    for (int i = threadIdx.x; i < nb * nb; i += PLB) sTb[i] = Tb[i];
    for (int i = lane; i < 2 * cells; i += 64) Xr[i] = 0;
    __syncthreads();
    for (uint32_t c = T0; c < T1;) {
        const int len = (int)min(T1 - c, (uint32_t)PLANE_SPAN);
        // 1. the round's members
        uint32_t pos[PLU], dg[PLU];
#pragma unroll
        for (int u = 0; u < PLU; ++u) {
            const int i = u * 64 + lane;
            pos[u] = 0xffffffffu;
            dg[u] = 0;
            if (u * 64 < len && i < len) {
                const uint32_t q = c + (uint32_t)i;
                dg[u] = pp.dig[q];
                pos[u] = pp.P ? pp.P[q] : q;
            }
        }
        C xv[PLU], base[PLU];
#pragma unroll
        for (int u = 0; u < PLU; ++u) {
            xv[u] = Cx<R>::make(0, 0);
            base[u] = Cx<R>::make(0, 0);
            if (pos[u] != 0xffffffffu) {
                xv[u] = x[pos[u]];
                if (first) base[u].x = V[pos[u]];
                else base[u] = y[pos[u]];
            }
        }
        if (first) {
#pragma unroll
            for (int u = 0; u < PLU; ++u) base[u] = Cx<R>::make(base[u].x * xv[u].x, base[u].x * xv[u].y);
        }
        // `done` = members of the planes the round holds whole
        int done = 0;
#pragma unroll
        for (int u = 0; u < PLU; ++u) {
            const uint64_t e = __ballot(pos[u] != 0xffffffffu && (dg[u] & PL_END));
            if (e) done = u * 64 + 64 - __clzll((long long)e);
        }
        if (done == 0) break;  // no whole plane (planes are shorter than a round: not reached)
        // 2. plane by plane
        for (int r0 = 0; r0 < done;) {
            int r1 = done;
#pragma unroll
            for (int u = PLU - 1; u >= 0; --u) {
                if (u * 64 + 63 < r0 || u * 64 >= r1) continue;
                uint64_t e = __ballot(pos[u] != 0xffffffffu && (dg[u] & PL_END));
                if (u * 64 < r0) e &= ~0ull << (r0 - u * 64);
                if (e) r1 = u * 64 + __ffsll((unsigned long long)e);
            }
            uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll
            for (int u = 0; u < PLU; ++u) {
                if (u * 64 >= r1 || u * 64 + 64 <= r0) continue;
                const int i = u * 64 + lane;
                if (i >= r0 && i < r1) {
                    const uint32_t da = (dg[u] >> 8) & 0x7fu, db = dg[u] & 0xffu;
                    lo = min2_u16(lo, (da << 16) | db);
                    hi = max2_u16(hi, (da << 16) | db);
                    Xr[da * nb + db] = xv[u].x;
                    Xi[da * nb + db] = xv[u].y;
                }
            }
            lo = wave_min2_u16(lo);
            hi = wave_max2_u16(hi);
            const int a0 = (int)(lo >> 16), b0 = (int)(lo & 0xffffu), a1 = (int)(hi >> 16), b1 = (int)(hi & 0xffffu);
            __builtin_amdgcn_wave_barrier();
            plane_blocks<R>(a0, a1, b0, b1, na, nb, lane, r0, r1, dg, base, sTa, sTb, Xr, Xi, Yr, Yi);
            // clear the plane's cells
#pragma unroll
            for (int u = 0; u < PLU; ++u) {
                if (u * 64 >= r1 || u * 64 + 64 <= r0) continue;
                const int i = u * 64 + lane;
                if (i >= r0 && i < r1) {
                    const uint32_t cell = ((dg[u] >> 8) & 0x7fu) * nb + (dg[u] & 0xffu);
                    Xr[cell] = 0;
                    Xi[cell] = 0;
                }
            }
            __builtin_amdgcn_wave_barrier();
            r0 = r1;
        }
        // 3. store the planes done
#pragma unroll
        for (int u = 0; u < PLU; ++u)
            if (pos[u] != 0xffffffffu && u * 64 + lane < done) y[pos[u]] = base[u];
        c += (uint32_t)done;
    }
}

template <class R>
void launch_plane(const PlanePass &pp, const R *Ta, const R *Tb, const typename Cx<R>::T *x, const R *V,
                  typename Cx<R>::T *y, bool first, const int *skip_if, int skip_j, hipStream_t s)
{
    if (pp.ntask == 0) return;
    const int cells = pp.na * pp.nb;
    const size_t lds = (size_t)(pp.na * pp.na + pp.nb * pp.nb + (PLB / 64) * (2 * cells + 512)) * sizeof(R);
    const uint32_t nwg = (pp.ntask + PLB / 64 - 1) / (PLB / 64);
    const dim3 grid(8 * ((nwg + 7) / 8));
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_hpsi_plane<R>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BYTES) != hipSuccess)
            (void)hipGetLastError();
    });
    hipLaunchKernelGGL((k_hpsi_plane<R>), grid, dim3(PLB), lds, s, pp, Ta, Tb, x, V, y, first ? 1 : 0, skip_if,
                       skip_j);
}

// ---- pair pass: the last two dimensions in one pass ---------------------------
// A workgroup takes one task (whole planes, contiguous in the sorted state),
// stages x in LDS and gives every point one thread, which sums its row run
// (dimension b = D-1: the points of its plane with its digit a, contiguous) and
// its column run (dimension a: the points of its plane with its digit b,
// contiguous in dimension a's rotated order, whose ranks the permutation maps
// onto the task's own positions) and writes y = V x + both sums once.  The
// per-dimension layout writes y in both passes and reads it in the second.
// LDS: x [span], the two factors, then per entry its digits and run flags
// (dg: d_a << 8 | d_b, bit 15 starts a row run, bit 14 a plane), rank ->
// position (pil), position -> rank (rpos) and per rank its digit a with bit
// 15 starting a column run (rinfo).
constexpr int PRB = 256;
constexpr int PRU = (int)((PAIR_WINDOW + PAIR_NAB_MAX + PRB - 1) / PRB);  // positions per thread
constexpr uint16_t PR_ROW = 0x8000u, PR_PLANE = 0x4000u;

template <class R>
__global__ __launch_bounds__(PRB) void k_hpsi_pair(PairPass pp, const R *__restrict__ Ta, const R *__restrict__ Tb,
                                                   const typename Cx<R>::T *__restrict__ x, const R *__restrict__ V,
                                                   typename Cx<R>::T *__restrict__ y, int span, const int *skip_if,
                                                   int skip_j)
{
    using C = typename Cx<R>::T;
    if (skip_if && skip_j >= *skip_if) return;
    const uint32_t T0 = pp.tstart[blockIdx.x], T1 = pp.tstart[blockIdx.x + 1];
    if (T0 >= T1) return;  // the whole workgroup: no barrier is left waiting
    const int len = (int)(T1 - T0);
    extern __shared__ __align__(16) unsigned char smem[];
    const int lda = pp.lda, ldb = pp.ldb;
    C *xs = reinterpret_cast<C *>(smem);
    R *sTa = reinterpret_cast<R *>(xs + span);
    R *sTb = sTa + lda * lda;
    uint16_t *dg = reinterpret_cast<uint16_t *>(sTb + ldb * ldb);
    uint16_t *pil = dg + span;
    uint16_t *rpos = pil + span;
    uint16_t *rinfo = rpos + span;
    const int tid = threadIdx.x;
    const uint32_t nb = (uint32_t)pp.n_b, na = (uint32_t)pp.n_a;
    // 1. the task's keys, x, V and rank -> position, all loads at once
    R vr[PRU];
#pragma unroll
    for (int u = 0; u < PRU; ++u) {
        const int i = tid + u * PRB;
        vr[u] = 0;
        if (i < len) {
            const uint32_t q = T0 + (uint32_t)i;
            const uint32_t k = pp.keys[q];
            const uint32_t kp = i > 0 ? pp.keys[q - 1] : 0u;
            const uint32_t kb = k / nb, db = k - kb * nb, ka = kb / na, da = kb - ka * na;
            const uint32_t kpb = kp / nb;
            const bool plane = i == 0 || kpb / na != ka;
            const bool row = plane || kpb != kb;
            dg[i] = (uint16_t)((da << 8) | db | (row ? PR_ROW : 0u) | (plane ? PR_PLANE : 0u));
            xs[i] = x[q];
            pil[i] = (uint16_t)(pp.pi_a[q] - T0);
            vr[u] = V[q];
        }
    }
    for (int i = tid; i < lda * lda; i += PRB) sTa[i] = Ta[i];
    for (int i = tid; i < ldb * ldb; i += PRB) sTb[i] = Tb[i];
    __syncthreads();
    // 2. per rank: its position's rank, digit a and column-run start (a plane
    // starts at the same index in both orders)
#pragma unroll
    for (int u = 0; u < PRU; ++u) {
        const int r = tid + u * PRB;
        if (r < len) {
            const int p = pil[r];
            rpos[p] = (uint16_t)r;
            const uint16_t dp = dg[p];
            const bool col = (dg[r] & PR_PLANE) || ((dg[pil[r - 1]] ^ dp) & 0x3fu);
            rinfo[r] = (uint16_t)(((dp >> 8) & 0x3fu) | (col ? PR_ROW : 0u));
        }
    }
    __syncthreads();
    // 3. one thread per point: row run, column run, V x; y written once
#pragma unroll
    for (int u = 0; u < PRU; ++u) {
        const int i = tid + u * PRB;
        if (i >= len) continue;
        const uint16_t d = dg[i];
        const R *rb = sTb + (d & 0x3fu) * ldb;
        R ar = 0, ai = 0;
        for (int j = i;; --j) {
            const uint16_t e = dg[j];
            const R t = rb[e & 0x3fu];
            const C v = xs[j];
            ar = fma(t, v.x, ar);
            ai = fma(t, v.y, ai);
            if (e & PR_ROW) break;
        }
        for (int j = i + 1; j < len; ++j) {
            const uint16_t e = dg[j];
            if (e & PR_ROW) break;
            const R t = rb[e & 0x3fu];
            const C v = xs[j];
            ar = fma(t, v.x, ar);
            ai = fma(t, v.y, ai);
        }
        const R *ra = sTa + ((d >> 8) & 0x3fu) * lda;
        const int r = rpos[i];
        for (int q = r;; --q) {
            const uint16_t e = rinfo[q];
            const R t = ra[e & 0x3fu];
            const C v = xs[pil[q]];
            ar = fma(t, v.x, ar);
            ai = fma(t, v.y, ai);
            if (e & PR_ROW) break;
        }
        for (int q = r + 1; q < len; ++q) {
            const uint16_t e = rinfo[q];
            if (e & PR_ROW) break;
            const R t = ra[e & 0x3fu];
            const C v = xs[pil[q]];
            ar = fma(t, v.x, ar);
            ai = fma(t, v.y, ai);
        }
        const C xv = xs[i];
        y[T0 + i] = Cx<R>::make(fma(vr[u], xv.x, ar), fma(vr[u], xv.y, ai));
    }
}

template <class R>
void launch_pair(const PairPass &pp, const R *Ta, const R *Tb, const typename Cx<R>::T *x, const R *V,
                 typename Cx<R>::T *y, const int *skip_if, int skip_j, hipStream_t s)
{
    if (pp.ntask == 0) return;
    const int span = (int)PAIR_WINDOW + pp.n_a * pp.n_b;
    const size_t lds = (size_t)span * sizeof(typename Cx<R>::T) +
                       (size_t)(pp.lda * pp.lda + pp.ldb * pp.ldb) * sizeof(R) + (size_t)span * 4 * sizeof(uint16_t);
    hipLaunchKernelGGL((k_hpsi_pair<R>), dim3(pp.ntask), dim3(PRB), lds, s, pp, Ta, Tb, x, V, y, span, skip_if,
                       skip_j);
}

}  // namespace

void hpsi_pair_f64(const PairPass &pp, const double *Ta, const double *Tb, const double2 *x, const double *V,
                   double2 *y, const int *skip_if, int skip_j, hipStream_t s)
{
    launch_pair<double>(pp, Ta, Tb, x, V, y, skip_if, skip_j, s);
}

void hpsi_pair_f32(const PairPass &pp, const float *Ta, const float *Tb, const float2 *x, const float *V, float2 *y,
                   const int *skip_if, int skip_j, hipStream_t s)
{
    launch_pair<float>(pp, Ta, Tb, x, V, y, skip_if, skip_j, s);
}

void hpsi_real_f64(const FiberPass &fp, const double *T, const double2 *x, const double *V, double2 *y, bool first,
                   const int *skip_if, int skip_j, hipStream_t s)
{
    launch_real<double>(fp, T, x, V, y, first, skip_if, skip_j, s);
}

void hpsi_pt_f64(const uint32_t *pi, const uint8_t *info, int64_t n, int nmax, const double *T, const double2 *x,
                 const double *V, double2 *y, bool first, const int *skip_if, int skip_j, hipStream_t s)
{
    launch_pt<double>(pi, info, n, nmax, T, x, V, y, first, skip_if, skip_j, s);
}

void hpsi_pt_f32(const uint32_t *pi, const uint8_t *info, int64_t n, int nmax, const float *T, const float2 *x,
                 const float *V, float2 *y, bool first, const int *skip_if, int skip_j, hipStream_t s)
{
    launch_pt<float>(pi, info, n, nmax, T, x, V, y, first, skip_if, skip_j, s);
}

template <class R>
int launch_acc(const FiberPass &fp, const R *T, const typename Cx<R>::T *x, typename Cx<R>::T *y, const int *skip_if,
               int skip_j, double2 *dotp, hipStream_t s)
{
    if (fp.nf <= 0) return 0;
    const unsigned nb = (unsigned)((fp.nf + HB - 1) / HB);
#define L(NM, ST)                                                                                                  \
    do {                                                                                                           \
        if (dotp)                                                                                                  \
            hipLaunchKernelGGL((k_hpsi_acc<R, NM, false, true, ST>), dim3(nb), dim3(HB), 0, s, fp.pi, fp.off,      \
                               fp.mask, fp.nf, T, x, y, skip_if, skip_j, dotp);                                    \
        else                                                                                                       \
            hipLaunchKernelGGL((k_hpsi_acc<R, NM, false, false, ST>), dim3(nb), dim3(HB), 0, s, fp.pi, fp.off,     \
                               fp.mask, fp.nf, T, x, y, skip_if, skip_j, dotp);                                    \
    } while (0)
    const bool st = fp.stage && fp.pi != nullptr && !dotp;  // the pass with the fused <x|y> keeps global loads
    switch (fp.nmax) {
    case 8: if (st) L(8, true); else L(8, false); break;
    case 16: if (st) L(16, true); else L(16, false); break;
    case 24: if (st) L(24, true); else L(24, false); break;
    case 32: if (st) L(32, true); else L(32, false); break;
    case 48: L(48, false); break;
    default: L(64, false); break;
    }
#undef L
    return dotp ? (int)nb : 0;
}

int hpsi_acc_f64(const FiberPass &fp, const double *T, const double2 *x, double2 *y, const int *skip_if, int skip_j,
                 hipStream_t s, double2 *dotp)
{
    return launch_acc<double>(fp, T, x, y, skip_if, skip_j, dotp, s);
}

int hpsi_acc_f32(const FiberPass &fp, const float *T, const float2 *x, float2 *y, const int *skip_if, int skip_j,
                 hipStream_t s, double2 *dotp)
{
    return launch_acc<float>(fp, T, x, y, skip_if, skip_j, dotp, s);
}

template <class R, bool CPLX>
void launch_mf(const FiberPass &fp, const void *H64, const MfIn<R> &in, const R *V, typename Cx<R>::T *y, int mode,
               const int *skip_if, int skip_j, hipStream_t s)
{
    if (fp.nf <= 0) return;
    const unsigned nb = (unsigned)((fp.nf + 63) / 64);
    const bool ident = fp.pi == nullptr;
#define L(MD, I)                                                                                                     \
    hipLaunchKernelGGL((k_hpsi_mf<R, CPLX, MD, I>), dim3(nb), dim3(MFB), 0, s, fp.pi, fp.off, fp.mask, fp.nf, H64, in, \
                       V, y, skip_if, skip_j)
    if (mode == 2) {
        if (ident) L(2, true);
        else L(2, false);
    } else if (mode == 1) {
        if (ident) L(1, true);
        else L(1, false);
    } else {
        if (ident) L(0, true);
        else L(0, false);
    }
#undef L
}

void hpsi_mfma_f32(const FiberPass &fp, const float *T64, const float2 *x, const float *V, float2 *y, bool first,
                   const int *skip_if, int skip_j, hipStream_t s)
{
    MfIn<float> in{};
    in.nin = 1;
    in.x[0] = x;
    in.c[0] = make_float2(1.f, 0.f);
    launch_mf<float, false>(fp, T64, in, V, y, first ? 2 : 1, skip_if, skip_j, s);
}

void hpsi_mfma_f64(const FiberPass &fp, const double *T64, const double2 *x, const double *V, double2 *y, bool first,
                   const int *skip_if, int skip_j, hipStream_t s)
{
    MfIn<double> in{};
    in.nin = 1;
    in.x[0] = x;
    in.c[0] = make_double2(1.0, 0.0);
    launch_mf<double, false>(fp, T64, in, V, y, first ? 2 : 1, skip_if, skip_j, s);
}

void hpsi_cmfma_f64(const FiberPass &fp, const double2 *H64, const CInput &in, double2 *y, bool accumulate,
                    const int *skip_if, int skip_j, hipStream_t s)
{
    MfIn<double> a{};
    a.nin = in.nin;
    for (int i = 0; i < 4; ++i) {
        a.x[i] = in.x[i];
        a.c[i] = in.c[i];
    }
    launch_mf<double, true>(fp, H64, a, nullptr, y, accumulate ? 1 : 0, skip_if, skip_j, s);
}

void hpsi_cmfma_f32(const FiberPass &fp, const float2 *H64, const CInput32 &in, float2 *y, bool accumulate,
                    const int *skip_if, int skip_j, hipStream_t s)
{
    MfIn<float> a{};
    a.nin = in.nin;
    for (int i = 0; i < 4; ++i) {
        a.x[i] = in.x[i];
        a.c[i] = in.c[i];
    }
    launch_mf<float, true>(fp, H64, a, nullptr, y, accumulate ? 1 : 0, skip_if, skip_j, s);
}

void hpsi_real_f32(const FiberPass &fp, const float *T, const float2 *x, const float *V, float2 *y, bool first,
                   const int *skip_if, int skip_j, hipStream_t s)
{
    launch_real<float>(fp, T, x, V, y, first, skip_if, skip_j, s);
}

void hpsi_cplx_f64(const FiberPass &fp, const double2 *H, const CInput &in, double2 *y, bool accumulate,
                   const double *V, const int *skip_if, int skip_j, hipStream_t s)
{
    (void)V;
    CArgs<double> a;
    a.nin = in.nin;
    for (int i = 0; i < 4; ++i) {
        a.x[i] = in.x[i];
        a.c[i] = in.c[i];
    }
    launch_cplx<double>(fp, H, a, y, accumulate, skip_if, skip_j, s);
}

void hpsi_cplx_f32(const FiberPass &fp, const float2 *H, const CInput32 &in, float2 *y, bool accumulate,
                   const float *V, const int *skip_if, int skip_j, hipStream_t s)
{
    (void)V;
    CArgs<float> a;
    a.nin = in.nin;
    for (int i = 0; i < 4; ++i) {
        a.x[i] = in.x[i];
        a.c[i] = in.c[i];
    }
    launch_cplx<float>(fp, H, a, y, accumulate, skip_if, skip_j, s);
}


template <class R>
void launch_block(const BlockPass &bp, const R *const *T, const typename Cx<R>::T *x, const R *V,
                  typename Cx<R>::T *y, bool accumulate, const int *skip_if, int skip_j, hipStream_t s)
{
    using C = typename Cx<R>::T;
    if (bp.nch == 0) return;
    BlockArgs<R> a{};
    a.ndim = bp.ndim;
    int nbmax = 8;
    for (int d = 0; d < bp.ndim; ++d) {
        a.pi[d] = bp.pi[d];
        a.off[d] = bp.off[d];
        a.mask[d] = bp.mask[d];
        a.fch[d] = bp.fch[d];
        a.T[d] = T[d];
        a.nb[d] = bp.nb[d];
        nbmax = std::max(nbmax, bp.nb[d]);
    }
    a.chunk = bp.chunk;
    a.nch = bp.nch;
    a.P = bp.P;
    a.accumulate = accumulate ? 1 : 0;
    a.V = V;
    int npi = 0;
    for (int d = 0; d < bp.ndim; ++d) npi += bp.pi[d] ? 1 : 0;
    const size_t bpp = 2 * sizeof(C) + sizeof(uint16_t) * (size_t)npi;
    // points per thread of the two launches (NT * SU >= cap)
    constexpr int SU_S = sizeof(R) == 8 ? 4 : 8, SU_B = sizeof(R) == 8 ? 5 : 8;
    // dynamic LDS above 64 KB: raise each instantiation's limit once per process
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        const void *fns[] = {
            reinterpret_cast<const void *>(&k_hpsi_block<R, 8, 512, SU_S>),
            reinterpret_cast<const void *>(&k_hpsi_block<R, 16, 512, SU_S>),
            reinterpret_cast<const void *>(&k_hpsi_block<R, 24, 512, SU_S>),
            reinterpret_cast<const void *>(&k_hpsi_block<R, 32, 512, SU_S>),
            reinterpret_cast<const void *>(&k_hpsi_block<R, 8, 1024, SU_B>),
            reinterpret_cast<const void *>(&k_hpsi_block<R, 16, 1024, SU_B>),
            reinterpret_cast<const void *>(&k_hpsi_block<R, 24, 1024, SU_B>),
            reinterpret_cast<const void *>(&k_hpsi_block<R, 32, 1024, SU_B>),
        };
        for (const void *f : fns)
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BYTES) != hipSuccess)
                (void)hipGetLastError();  // the launch itself then reports the LDS request
    });
    // main launch: two 512-thread workgroups per CU; long chunks: one
    // 1024-thread workgroup per CU
    auto go = [&](dim3 grid, uint32_t cap, bool wide) {
        a.cap = cap;
        const size_t lds = (size_t)cap * bpp;
#define PPQ_GO(NB, NT, SU) \
    hipLaunchKernelGGL((k_hpsi_block<R, NB, NT, SU>), grid, dim3(NT), lds, s, a, x, y, skip_if, skip_j)
        if (wide) {
            if (nbmax <= 8) PPQ_GO(8, 1024, SU_B);
            else if (nbmax <= 16) PPQ_GO(16, 1024, SU_B);
            else if (nbmax <= 24) PPQ_GO(24, 1024, SU_B);
            else PPQ_GO(32, 1024, SU_B);
        } else {
            if (nbmax <= 8) PPQ_GO(8, 512, SU_S);
            else if (nbmax <= 16) PPQ_GO(16, 512, SU_S);
            else if (nbmax <= 24) PPQ_GO(24, 512, SU_S);
            else PPQ_GO(32, 512, SU_S);
        }
#undef PPQ_GO
    };
    a.list = nullptr;
    go(dim3(8 * ((bp.nch + 7) / 8)), bp.cap_small, false);
    if (bp.nbig > 0) {
        a.list = bp.big;
        go(dim3(bp.nbig), bp.cap_big, true);
    }
}

// The one-lane-per-fiber block pass: 256-thread workgroups for chunks up to
// cap_small points, 512-thread ones (one per chunk) for the longer chunks.
template <class R>
void launch_block2(const BlockPass &bp, const R *const *T, const typename Cx<R>::T *x, const R *V,
                   typename Cx<R>::T *y, bool accumulate, const int *skip_if, int skip_j, hipStream_t s)
{
    using C = typename Cx<R>::T;
    if (bp.nch == 0) return;
    BlockArgs<R> a{};
    a.ndim = bp.ndim;
    int nbmax = 8;
    for (int d = 0; d < bp.ndim; ++d) {
        a.pi[d] = bp.pi[d];
        a.off[d] = bp.off[d];
        a.mask[d] = bp.mask[d];
        a.fch[d] = bp.fch[d];
        a.T[d] = T[d];
        a.nb[d] = bp.nb[d];
        nbmax = std::max(nbmax, bp.nb[d]);
    }
    a.chunk = bp.chunk;
    a.nch = bp.nch;
    a.P = bp.P;
    a.accumulate = accumulate ? 1 : 0;
    a.V = V;
    a.unroll = bp.unroll;
    int npi = 0;
    for (int d = 0; d < bp.ndim; ++d) npi += bp.pi[d] ? 1 : 0;
    const size_t bpp = 2 * sizeof(C) + sizeof(uint16_t) * (size_t)npi;
    // points per thread of the two launches: NT * SU covers their capacity
    // (the main launch's cap_small; the LDS limit for the long chunks)
    constexpr int SU_S = sizeof(R) == 8 ? 8 : 16, SU_B = sizeof(R) == 8 ? 10 : 16;
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        const void *fns[] = {
            reinterpret_cast<const void *>(&k_hpsi_blk2<R, 8, 256, SU_S>),
            reinterpret_cast<const void *>(&k_hpsi_blk2<R, 16, 256, SU_S>),
            reinterpret_cast<const void *>(&k_hpsi_blk2<R, 24, 256, SU_S>),
            reinterpret_cast<const void *>(&k_hpsi_blk2<R, 32, 256, SU_S>),
            reinterpret_cast<const void *>(&k_hpsi_blk2<R, 8, 512, SU_B>),
            reinterpret_cast<const void *>(&k_hpsi_blk2<R, 16, 512, SU_B>),
            reinterpret_cast<const void *>(&k_hpsi_blk2<R, 24, 512, SU_B>),
            reinterpret_cast<const void *>(&k_hpsi_blk2<R, 32, 512, SU_B>),
        };
        for (const void *f : fns)
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BYTES) != hipSuccess)
                (void)hipGetLastError();
    });
    auto go = [&](dim3 grid, uint32_t cap, bool wide) {
        a.cap = cap;
        const size_t lds = (size_t)cap * bpp;
#define PPQ_GO(NB, NT, SU) \
    hipLaunchKernelGGL((k_hpsi_blk2<R, NB, NT, SU>), grid, dim3(NT), lds, s, a, x, y, skip_if, skip_j)
        if (wide) {
            if (nbmax <= 8) PPQ_GO(8, 512, SU_B);
            else if (nbmax <= 16) PPQ_GO(16, 512, SU_B);
            else if (nbmax <= 24) PPQ_GO(24, 512, SU_B);
            else PPQ_GO(32, 512, SU_B);
        } else {
            if (nbmax <= 8) PPQ_GO(8, 256, SU_S);
            else if (nbmax <= 16) PPQ_GO(16, 256, SU_S);
            else if (nbmax <= 24) PPQ_GO(24, 256, SU_S);
            else PPQ_GO(32, 256, SU_S);
        }
#undef PPQ_GO
    };
    a.list = nullptr;
    go(dim3(8 * ((bp.nch + 7) / 8)), bp.cap_small, false);
    if (bp.nbig > 0) {
        a.list = bp.big;
        go(dim3(bp.nbig), bp.cap_big, true);
    }
}

void hpsi_block2_f64(const BlockPass &bp, const double *const *T, const double2 *x, const double *V, double2 *y,
                     bool accumulate, const int *skip_if, int skip_j, hipStream_t s)
{
    launch_block2<double>(bp, T, x, V, y, accumulate, skip_if, skip_j, s);
}

void hpsi_block2_f32(const BlockPass &bp, const float *const *T, const float2 *x, const float *V, float2 *y,
                     bool accumulate, const int *skip_if, int skip_j, hipStream_t s)
{
    launch_block2<float>(bp, T, x, V, y, accumulate, skip_if, skip_j, s);
}

void hpsi_long_real_f64(const LongPass &lp, const double *T, const double2 *x, const double *V, double2 *y,
                        bool first, const int *skip_if, int skip_j, hipStream_t s)
{
    MfIn<double> in{};
    in.nin = 1;
    in.x[0] = x;
    in.c[0] = make_double2(1.0, 0.0);
    launch_long<double, false>(lp, T, in, V, y, first ? 2 : 1, skip_if, skip_j, s);
}

void hpsi_long_real_f32(const LongPass &lp, const float *T, const float2 *x, const float *V, float2 *y, bool first,
                        const int *skip_if, int skip_j, hipStream_t s)
{
    MfIn<float> in{};
    in.nin = 1;
    in.x[0] = x;
    in.c[0] = make_float2(1.f, 0.f);
    launch_long<float, false>(lp, T, in, V, y, first ? 2 : 1, skip_if, skip_j, s);
}

void hpsi_long_cplx_f64(const LongPass &lp, const double2 *H, const CInput &in, double2 *y, bool accumulate,
                        const int *skip_if, int skip_j, hipStream_t s)
{
    MfIn<double> a{};
    a.nin = in.nin;
    for (int i = 0; i < 4; ++i) {
        a.x[i] = in.x[i];
        a.c[i] = in.c[i];
    }
    launch_long<double, true>(lp, H, a, nullptr, y, accumulate ? 1 : 0, skip_if, skip_j, s);
}

void hpsi_long_cplx_f32(const LongPass &lp, const float2 *H, const CInput32 &in, float2 *y, bool accumulate,
                        const int *skip_if, int skip_j, hipStream_t s)
{
    MfIn<float> a{};
    a.nin = in.nin;
    for (int i = 0; i < 4; ++i) {
        a.x[i] = in.x[i];
        a.c[i] = in.c[i];
    }
    launch_long<float, true>(lp, H, a, nullptr, y, accumulate ? 1 : 0, skip_if, skip_j, s);
}

void hpsi_plane_f64(const PlanePass &pp, const double *Ta, const double *Tb, const double2 *x, const double *V,
                    double2 *y, bool first, const int *skip_if, int skip_j, hipStream_t s)
{
    launch_plane<double>(pp, Ta, Tb, x, V, y, first, skip_if, skip_j, s);
}

void hpsi_plane_f32(const PlanePass &pp, const float *Ta, const float *Tb, const float2 *x, const float *V,
                    float2 *y, bool first, const int *skip_if, int skip_j, hipStream_t s)
{
    launch_plane<float>(pp, Ta, Tb, x, V, y, first, skip_if, skip_j, s);
}

void hpsi_block_f64(const BlockPass &bp, const double *const *T, const double2 *x, const double *V, double2 *y,
                    bool accumulate, const int *skip_if, int skip_j, hipStream_t s)
{
    launch_block<double>(bp, T, x, V, y, accumulate, skip_if, skip_j, s);
}

void hpsi_block_f32(const BlockPass &bp, const float *const *T, const float2 *x, const float *V, float2 *y,
                    bool accumulate, const int *skip_if, int skip_j, hipStream_t s)
{
    launch_block<float>(bp, T, x, V, y, accumulate, skip_if, skip_j, s);
}

}  // namespace ppq
