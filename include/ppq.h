/*
 * ppq.h -- C ABI of the MI355X (gfx950) library for dynamically pruned
 * wavepacket propagation in a direct-product basis (Larsson, Hartke & Tannor,
 * J. Chem. Phys. 2016, arXiv:1606.04004).
 *
 * The state is a coefficient vector held only on an active set A of
 * multi-indices I = (i_0, ..., i_{D-1}) of a direct-product basis (Sec. II.A,
 * Eq. wavepacket_form).  Each time step applies a sum-of-products operator
 * (Sec. II.B.2): one dense 1D matrix per dimension (sine-DVR kinetic energy,
 * or the similarity-transformed factors of a phase-space lattice basis,
 * Sec. II.B.1 and II.D) plus a diagonal sum-of-products potential (Sec. II.A,
 * II.E), restricted to A (the pruned transformation of Sec. II.B.2 and the
 * appendix), propagates with a short-iterative Lanczos / Arnoldi step
 * (Sec. III.A), and then adapts A with the amplitude threshold theta
 * (Sec. II.E): keep |c| >= theta, add the nearest neighbours of every kept
 * function (ball radius 1, Sec. III.A), drop the rest, compact.
 *
 * Conventions for every call
 *   - Return value: PPQ_OK (0) or a negative ppq_status.  On an error the
 *     context's state is unchanged unless stated otherwise; ppq_last_error()
 *     gives a message.  PPQ_E_HIP means a HIP runtime call failed: the context
 *     is then unusable and must be destroyed.
 *   - Keys: a multi-index is linearised row-major, last dimension fastest,
 *     key = sum_k i_k * prod_{k' > k} n_k'  (the layout of the appendix).
 *     Keys cross the ABI as uint64_t; the grid size prod n_k must be < 2^32.
 *   - Coefficients cross the ABI as interleaved complex FP64 (re, im) on the
 *     host, whatever the context precision.  ppq_apply_h takes device vectors
 *     of the context precision (see there).
 *   - Matrices are row-major, complex interleaved.
 *   - Host pointers are read during the call only (inputs copied in); device
 *     pointers are used in stream order on the context stream and must stay
 *     valid until that work has run.  The library never frees caller memory.
 *   - A context is used by one host thread at a time.
 *
 * Environment (read at ppq_create; for measurement and comparison only)
 *   PPQ_HPSI=2  (default) per-dimension fiber passes: matrix cores for long
 *               fibers (mean length > 16), for complex lattice factors and
 *               for the FP32 last-dimension pass; vector FMA for the other
 *               short-fiber passes.
 *   PPQ_HPSI=3  vector FMA in every pass (comparison).
 *   PPQ_HPSI=1  point-parallel in every pass; PPQ_HPSI=0 lane per fiber in
 *               every pass (earlier layouts, for comparison).
 *   PPQ_HPSI=4  block-fused layout: two LDS-staged passes over chunks of
 *               blocks (falls back to 2 when a chunk exceeds LDS); 5 the
 *               same chunks with one lane per fiber in each.
 *   PPQ_HPSI=6  plane passes: two adjacent dimensions per pass through
 *               matrix-core tiles (dimensions of at most 32 points).
 *   PPQ_HPSI=7  the last two dimensions in one pass (whole planes per
 *               workgroup), the others as in 2.
 *   PPQ_BLOCK_STATS=1  report the block layout's chunk statistics on stderr.
 *   PPQ_ACC_STAGE=1  lane-per-fiber passes (but the one with the fused
 *               <x|y>) read the permutation from each wavefront's copy of its
 *               rank range in LDS instead of scattered global loads.
 *   PPQ_DILATE=1 / 2  adaption's dilation per function (atomics) / word by
 *               word from the bitmap of the functions kept (the +-1 stencil
 *               on DVR axes only); 0 (default) chooses by the grid-to-set
 *               size ratio.  Both give the same set.
 *   Every layout computes the same product; only the summation order of
 *   the dimensions' contributions differs.
 */
#ifndef PPQ_H
#define PPQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ppq_ctx ppq_ctx;

typedef enum {
    PPQ_OK = 0,
    PPQ_E_ARG = -1,          /* invalid argument (state unchanged) */
    PPQ_E_STATE = -2,        /* call not valid in the current state (no grid / no set) */
    PPQ_E_OOM = -3,          /* device allocation failed */
    PPQ_E_CAPACITY = -4,     /* a size limit of this build was exceeded */
    PPQ_E_HIP = -5,          /* HIP runtime error; context poisoned */
    PPQ_E_NUMERIC = -6,      /* non-finite norm or coefficients */
    PPQ_E_UNSUPPORTED = -7   /* valid request this build does not implement */
} ppq_status;

typedef enum {
    PPQ_FP64 = 0,            /* all arithmetic in FP64 */
    PPQ_FP32 = 1             /* operator products and Krylov vectors in complex FP32
                                (matrix cores where fibers form dense tiles); inner
                                products, norms, the small exponential and the
                                coefficient master copy in FP64 */
} ppq_precision;

typedef enum {
    PPQ_FAC_POWER = 0,       /* q_k^p on the grid points;           params = {p, unused} */
    PPQ_FAC_MORSE = 1,       /* (1 - exp(-a (q_k - q0)))^2;          params = {a, q0}   */
    PPQ_FAC_TABLE = 2,       /* caller-supplied values at the n_k grid points          */
    PPQ_FAC_MORSE_DA = 3,    /* 2 (1 - e) e (q_k - q0), e = exp(-a (q_k - q0)): the
                                derivative of the Morse factor with respect to a;
                                params = {a, q0}                                       */
    PPQ_FAC_DENSE_REAL = 4,  /* dense real n_k x n_k matrix in the dimension's DVR
                                basis, row-major (ppq_add_term only)                   */
    PPQ_FAC_DENSE_COMPLEX = 5 /* dense complex n_k x n_k matrix, row-major, (re, im)
                                interleaved (ppq_add_term only)                        */
} ppq_factor_kind;

/* Fields of one observable record (ppq_observables, ppq_propagate). */
enum {
    PPQ_OBS_T = 0,           /* time */
    PPQ_OBS_NORM2 = 1,       /* sum |c_I|^2 over A */
    PPQ_OBS_ENERGY = 2,      /* <psi|H_A|psi> / <psi|psi> */
    PPQ_OBS_ACF_RE = 3,      /* autocorrelation C(t) = <psi(0)|psi(t)> (Eq. acorr), real */
    PPQ_OBS_ACF_IM = 4,      /* imaginary part */
    PPQ_OBS_NACTIVE = 5,     /* |A| */
    PPQ_OBS_NABOVE = 6,      /* |{I in A : |c_I| >= theta}| (1 - this/|A| is the wasted fraction, Sec. III.A) */
    PPQ_OBS_KRYLOV = 7,      /* Krylov dimension used by the step that produced the record
                                (the largest of its substeps under step control) */
    PPQ_OBS_SUBSTEPS = 8,    /* substeps of that step (1 without step control; 0 in a
                                record no step produced) */
    PPQ_OBS_N = 9
};

/* Creates a context on HIP device `device`.  `hip_stream` is a hipStream_t to
   run on (NULL: the library creates its own).  `precision` is a ppq_precision. */
int ppq_create(ppq_ctx **out, int device, void *hip_stream, int precision);
void ppq_destroy(ppq_ctx *ctx);
/* Message of the last error on this context; valid until the next call. */
const char *ppq_last_error(const ppq_ctx *ctx);

/* Direct-product sine-DVR grid (particle-in-a-box DVR of the DVR family,
   Sec. II.A): per dimension n[k] interior points of the box (lo[k], hi[k]),
   q_i = lo + i (hi-lo)/(n+1), i = 1..n.  Sets the kinetic operator
   -1/(2 mass) d^2/dq^2 on every dimension.  1 <= D <= 8, 2 <= n[k] <= 256,
   prod n < 2^32.  Dimensions of up to 64 points keep their fibers as 64-bit
   digit masks and take the matrix-core and mask-driven passes; longer ones
   keep a digit per fiber entry and take a long-fiber pass (one wavefront per
   fiber; the block-fused layout is then off).  Clears any operator and
   state. */
int ppq_set_grid(ppq_ctx *ctx, int D, const int32_t *n, const double *lo, const double *hi, double mass);

/* Grid points of dimension k (n[k] doubles, host). */
int ppq_get_grid(const ppq_ctx *ctx, int k, double *q);

/* Makes dimension k a periodic Fourier grid (the FGH DVR the paper uses
   under its lattices, Sec. III.A): points x_j = lo + j (hi-lo)/n, j = 0..n-1,
   over the period hi - lo, and kinetic energy -1/(2 mass) d^2/dx^2 from its
   spectral definition with |k| <= (n-1) pi/(hi-lo).  n[k] must be odd
   (PPQ_E_ARG).  A lattice on the dimension (ppq_set_lattice /
   ppq_set_weylets) is then projected on these points with weight
   (hi-lo)/n; the Fourier grid must be set first (PPQ_E_STATE after a
   lattice), and before adding terms. */
int ppq_set_fgh(ppq_ctx *ctx, int k);

/* Makes dimension k a phase-space lattice basis: n_s x n_l von Neumann
   Gaussians projected on the DVR grid and used biorthogonally (Sec. II.B.1,
   Eqs. pvN_def, pvb_def, psi_exp_pvb), n_s * n_l == n[k].  Cells are centred
   at x_s = lo + (s + 1/2) dx, dx = (hi-lo)/n_s, with momenta
   p_l = (l - (n_l-1)/2) dp, dp = 2 pi / dx.  Coefficients on this dimension
   are the overlaps a = G^+ c; every 1D factor on it acts as G^+ h G^{-+}
   (non-Hermitian, so steps use Arnoldi); its neighbours in adaption are the
   lattice cells (s+-1, l), (s, l+-1).  Must be called before adding terms. */
int ppq_set_lattice(ppq_ctx *ctx, int k, int n_s, int n_l);

/* Makes dimension k a projected-Weylet basis (Sec. II.D): the
   momentum-symmetrized Gaussians of Eq. sG_def on a doubly dense lattice of
   n_x cells (x_s = lo + (s + 1/2) dx, dx = (hi-lo)/n_x) and n_p momenta
   (p_l = (l + 1/2) dp > 0, dp = pi / dx, alpha = dp / (2 dx)), projected on
   the DVR grid (Eq. psG_def) and orthogonalised, W = Phi S^{-1/2}:
   a real orthogonal basis used like the lattice of ppq_set_lattice (a = W^T c,
   factors W^T h W, Arnoldi steps, lattice-cell neighbours in adaption).
   n_x * n_p == n[k].  PPQ_E_NUMERIC if the lattice's functions are linearly
   dependent.  Must be called before adding terms. */
int ppq_set_weylets(ppq_ctx *ctx, int k, int n_x, int n_p);

/* Adds the potential term coef * prod_f factor_f(q_{dims[f]}) (a product of
   diagonal 1D factors: Sec. II.E, potential as a sum of products of diagonal
   matrices).  kinds[f] is a ppq_factor_kind, params holds 2 doubles per
   factor, tables holds n[dims[f]] doubles per PPQ_FAC_TABLE factor (in factor
   order; may be NULL otherwise).  On DVR dimensions the term stays diagonal;
   a term touching lattice dimensions becomes a product of dense factors
   (applied as ppq_add_term describes). */
int ppq_add_potential_term(ppq_ctx *ctx, double coef, int nfac, const int32_t *dims, const int32_t *kinds,
                           const double *params, const double *tables);

/* Adds the general sum-of-products term (c_re + i c_im) prod_f h_f, one
   factor h_f acting on dimension dims[f] (Sec. II.B.2: the operator is a sum
   of products of one-dimensional operators).  kinds[f] is a ppq_factor_kind:
   the diagonal kinds of ppq_add_potential_term, or a dense matrix
   (PPQ_FAC_DENSE_REAL: n_k^2 doubles, PPQ_FAC_DENSE_COMPLEX: 2 n_k^2 doubles)
   in the dimension's DVR basis.  params: 2 doubles per factor (as for
   ppq_add_potential_term; ignored for dense and table kinds); data: the
   table (n_k doubles) and dense (n_k^2 or 2 n_k^2 doubles) factors one after
   the other in factor order (host, copied; may be NULL without such
   factors).  A dense factor must be the only factor on its dimension; a
   term of no factors is a constant.
   A term of diagonal factors with c_im = 0 is a potential term (as
   ppq_add_potential_term).  Any other term acts on a vector on the active
   set as the sequential pruned product of Sec. II.B.2 (Eq.
   matvecprod_sequential): its factors one at a time from the highest
   dimension down, each result truncated to the active set before the next,
   then times the coefficient; diagonal factors commute with the truncation
   and are applied to the input.  On lattice dimensions every factor is
   transformed like the kinetic matrix (G^+ h G^{-+}, W^T h W).  The operator
   stays Hermitian (Lanczos steps) while every such term on DVR dimensions
   has one dense factor, Hermitian, and a real coefficient; two or more dense
   factors in one term, a complex coefficient or a non-Hermitian factor make
   steps use Arnoldi.  PPQ_E_ARG for bad dimensions, kinds or layout,
   PPQ_E_NUMERIC for non-finite values (state unchanged). */
int ppq_add_term(ppq_ctx *ctx, double c_re, double c_im, int nfac, const int32_t *dims, const int32_t *kinds,
                 const double *params, const double *data);

/* Replaces the one-dimensional operator of dimension k (by default the
   sine-DVR kinetic energy of ppq_set_grid) by h, a real symmetric n_k x n_k
   matrix in the dimension's DVR basis, row-major (host, copied): any 1D
   factor of the sum-of-products operator (Sec. II.A, Eq. matvecprod_sequential),
   e.g. the kinetic matrix of another DVR.  On a phase-space lattice
   dimension it is transformed like the kinetic matrix.  h = NULL restores
   the sine-DVR kinetic energy.  PPQ_E_ARG unless h is exactly symmetric;
   PPQ_E_NUMERIC for non-finite entries. */
int ppq_set_factor(ppq_ctx *ctx, int k, const double *h);

/* Removes every potential and product term (ppq_add_potential_term,
   ppq_add_term; the kinetic factors stay), so that a new sum-of-products
   operator can be added term by term (Sec. II.A, II.E); the state and its
   active set are kept.  The derivative terms of the adjoint are not
   touched. */
int ppq_clear_potential(ppq_ctx *ctx);

/* Capacity of the active set (number of functions).  Grows automatically when
   adaption needs more, doubling each time (never past the grid size); each
   growth reallocates every per-point buffer, so reserving ahead avoids
   reallocation inside a run.  PPQ_E_ARG unless 1 <= max_active <= the grid
   size; PPQ_E_STATE without a grid. */
int ppq_reserve(ppq_ctx *ctx, int64_t max_active);

/* Initial state: product Gaussian psi0(q) = prod_k g_k(q_k),
   g_k = exp(-(q-centre_k)^2/(2 width_k^2) + i momentum_k (q-centre_k)),
   sampled on the grid and normalised per dimension; on lattice dimensions
   taken to coefficients a = G^+ g.  The active set is every function with
   |psi0_I| >= eps plus its nearest neighbours (the adaption rule applied to
   the full-grid packet).  psi0 also becomes the reference of C(t).
   n_active (may be NULL) receives |A|. */
int ppq_init_gaussian(ppq_ctx *ctx, const double *centre, const double *momentum, const double *width,
                      double eps, int64_t *n_active);

/* Replaces the state: `count` strictly ascending keys in range, coefficients
   interleaved complex FP64 (host).  PPQ_E_ARG if keys are unsorted, repeated
   or out of range. */
int ppq_set_state(ppq_ctx *ctx, int64_t count, const uint64_t *keys, const double *coeff);

/* Replaces the reference packet psi0 of C(t) (Eq. acorr) by the normalised
   product Gaussian of ppq_init_gaussian (same centre/momentum/width layout,
   D doubles each, host) without touching the state; e.g. for a state given by
   ppq_set_state.  ppq_init_gaussian and the adjoint calls also set the
   reference (to their own packet).  PPQ_E_ARG for a non-positive width or
   non-finite values. */
int ppq_set_reference(ppq_ctx *ctx, const double *centre, const double *momentum, const double *width);

/* Number of functions in the active set (no synchronisation needed). */
int ppq_active_count(const ppq_ctx *ctx, int64_t *count);

/* Copies the state to the host: *count = |A|; keys and coeff (2*|A| doubles)
   are written when cap >= |A| (else PPQ_E_ARG with *count set). */
int ppq_get_state(ppq_ctx *ctx, int64_t cap, int64_t *count, uint64_t *keys, double *coeff);

/* Device forms of ppq_set_state / ppq_get_state: keys (uint64) and
   coefficients (interleaved complex FP64) are device pointers, so a state
   moves between the library and device tensors without crossing PCIe.
   ppq_set_state_device checks the keys (strictly ascending, in range) and the
   coefficients (finite) on the device while copying them into a spare buffer
   and synchronises; on a violation it returns PPQ_E_ARG (keys) or
   PPQ_E_NUMERIC (coefficients) and the state is unchanged.
   ppq_get_state_device writes *count = |A| on the host and, when cap >= |A|,
   the keys and coefficients in stream order on the context stream (no
   synchronisation; the buffers must stay valid until that work has run).
   Pointers that are not device (or managed) memory give PPQ_E_ARG. */
int ppq_set_state_device(ppq_ctx *ctx, int64_t count, const uint64_t *keys, const double *coeff);
int ppq_get_state_device(ppq_ctx *ctx, int64_t cap, int64_t *count, uint64_t *keys, double *coeff);

/* y = P_A H P_A x on the current active set (the pruned product of Sec. II.B.2
   computed fiber by fiber as in the appendix).  x, y: device arrays of |A|
   complex values in key order -- interleaved FP64 for PPQ_FP64 contexts,
   interleaved FP32 for PPQ_FP32 contexts; x and y must not overlap.
   Enqueued on the context stream; no synchronisation.  PPQ_E_ARG when x or y
   is not device (or managed) memory. */
int ppq_apply_h(ppq_ctx *ctx, const void *x, void *y);

/* One short-iterative Lanczos (Arnoldi if any lattice dimension) step of
   length dt with Krylov order m (m H-applications, full reorthogonalisation
   by classical Gram-Schmidt applied twice; in the Lanczos case the first
   pass subtracts only the three-term recurrence's two projections and the
   second pass all of them), on the current set; no adaption.  1 <= m <= 16. */
int ppq_step(ppq_ctx *ctx, double dt, int m);

/* Adaptive SIL order (Sec. III.A adapts the integrator's accuracy to the
   amplitude threshold).  With tol > 0 every later step (ppq_step,
   ppq_propagate) stops its Krylov recurrence at the first order k <= m whose
   estimate n0 |dt|^k / k! prod_{i<k} beta_i (Park and Light's estimate of the
   first term the space leaves out; n0 = |psi|) is <= tol; the order used is
   recorded per step.  0 (default) keeps the full order m.  The decision is
   taken on the device, with no host wait.  PPQ_E_ARG unless tol is finite
   and >= 0.  The adjoint entry points need tolerance 0 (PPQ_E_UNSUPPORTED). */
int ppq_set_krylov_tolerance(ppq_ctx *ctx, double tol);

/* Step size control, tied like the adaptive order to the Krylov tolerance
   (Sec. III.A adapts the integrator's accuracy to the amplitude threshold;
   with tolerance 0 it has no effect).  With max_substeps > 1 every later step
   of length dt (ppq_step, ppq_propagate) runs as s substeps of dt/s on the
   current set: s starts at the previous step's count (1 after a new state);
   every substep must meet the tolerance at a Krylov order below m, else the
   step is redone from its start with 2s substeps, and a step needing more
   than max_substeps fails with PPQ_E_NUMERIC (the state keeps the values
   from before the step).  After a step whose substeps all stopped at order
   m/2 or below, the next starts with s/2.  Each attempt waits once for the
   orders on the host.  The record's PPQ_OBS_SUBSTEPS field gives s.
   PPQ_E_ARG unless 1 <= max_substeps <= 1024 (1 = off, the default). */
int ppq_set_step_control(ppq_ctx *ctx, int max_substeps);

/* Adaption with threshold eps (Sec. II.E, radius-1 stencil of Sec. III.A):
   A' = {I in A : |c_I| >= eps} plus their nearest neighbours inside the grid;
   coefficients carried over on A cap A', zero on new functions.  |c|^2 is
   compared as fl(fl(re^2) + fl(im^2)) >= fl(eps^2) (no fused multiply-add).
   n_active / n_above (may be NULL) receive |A'| and the kept count. */
int ppq_prune(ppq_ctx *ctx, double eps, int64_t *n_active, int64_t *n_above);

/* Neighbour stencil of every later adaption and of the initial set
   (Sec. III.A), counted over the phase-space axes: one per DVR dimension
   (its grid index), two per lattice dimension (the cell and the level of
   its (s, l) pair).  1 (default) adds +-1 on one axis (ball radius 1: 2D
   neighbours on a DVR grid, (s+-1, l) and (s, l+-1) on a lattice); 2 also
   adds every change of +-1 on two axes at once (ball radius sqrt(2), 2A^2
   neighbours for A axes); 3 adds every combination of -1/0/+1 changes over
   all axes, 3^A - 1 neighbours (ball radius 2).  The paper finds radius 1
   best and uses it throughout.  PPQ_E_ARG for other values. */
int ppq_set_stencil(ppq_ctx *ctx, int stencil);

/* Relative exclusion threshold r >= 0 of every later adaption (ppq_prune,
   ppq_propagate, the adjoint recording), Sec. II.E: functions are excluded
   only when more than r * |A| of them would go; otherwise the new set is
   A' united with A (all current functions stay, with their coefficients).
   r = 0 (the default) excludes whatever the threshold rule drops.
   PPQ_E_ARG for negative or non-finite r. */
int ppq_set_relative_exclusion(ppq_ctx *ctx, double r);

/* nsteps x {ppq_step(dt, m); ppq_prune(eps)} (eps < 0: no adaption), recording
   an observable record (PPQ_OBS_N doubles) before the first step and after
   every adaption into trace ((nsteps+1) * PPQ_OBS_N doubles, host; may be
   NULL).  Synchronises once at the end. */
int ppq_propagate(ppq_ctx *ctx, int nsteps, double dt, int m, double eps, double *trace);

/* Observable record of the current state (synchronises).  eps is the
   threshold used for PPQ_OBS_NABOVE. */
int ppq_observables(ppq_ctx *ctx, double eps, double *out);

/* Position expectation per dimension of the current state (synchronises):
   q[k] = sum_I |c_I|^2 q_k(i_k) / sum_I |c_I|^2 over the active set, with
   q_k(i) the sine-DVR grid point of index i; the DVR position operator is
   diagonal with the grid points as eigenvalues (Sec. II.A).  q is a host
   array of D doubles owned by the caller.  Phase-space lattice dimensions,
   where position is not diagonal in the cell index, and an empty or zero
   state give NaN.  PPQ_E_STATE without a state. */
int ppq_expect_q(ppq_ctx *ctx, double *q);

/* No-allocation form of ppq_expect_q, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops, hosts
   that forbid allocation): the same kernels and the same result, bit for
   bit, but the grid-point table, the per-block partial sums and the result
   live in a library-wide device array of 256 KiB (one per GPU, held until
   the process ends) instead of context buffers; the call makes no device
   allocation.  Needs D * max n_k doubles of table (always within the array
   under this build's grid limits; PPQ_E_CAPACITY otherwise).  Every call on
   one GPU uses that GPU's array: calls that overlap on one GPU (two host
   threads, or contexts on different streams) race and must be serialised by
   the caller.  Synchronises the context stream.  q: host array of D doubles.
   PPQ_E_STATE without a state or when the array's device address could not
   be obtained. */
int ppq_expect_q_noalloc(ppq_ctx *ctx, double *q);

/* Autocorrelation at twice the current time, C(2t) = <psi(t)*|psi(t)>, no
   complex conjugate (the identity after Eq. acorr): valid when the initial
   packet is real (zero momentum) and the operator real symmetric, so that
   one propagation to t gives C up to 2t.  On DVR dimensions it is
   sum_I c_I^2 over the active set.  On a phase-space lattice basis the
   coefficients a are not orthonormal: C(2t) = a^T B^T B a with B =
   (x)_k G_k^{-+} (c = B a the DVR coefficients; B = W for projected
   Weylets), evaluated by transforming a to the full DVR grid (two full-grid
   work tensors, at most 2^28 points, PPQ_E_CAPACITY beyond).  c2t: 2
   doubles (re, im), host.  Synchronises.  PPQ_E_UNSUPPORTED when a complex
   coefficient or a complex or non-symmetric dense factor (ppq_add_term)
   makes the operator other than real symmetric (in the DVR basis). */
int ppq_acf_doubled(ppq_ctx *ctx, double *c2t);

/* ---- adjoint gradient of the survival probability (added form) ----------
   J(theta) = |<psi0(centre, momentum)|psi(T)>|^2 after nsteps steps of the
   pruned propagation.  The active-set trajectory {A_n} of the recording run
   is frozen (adaption is not differentiable); each step map is taken as the
   exact exponential exp(-i H_{A_n} dt), evaluated in its Krylov space.  The
   gradient is computed by the adjoint recursion lambda_n = E_n^+ R_n^+
   lambda_{n+1} from lambda_N = psi0 on A_N, with the step derivative
   obtained in closed form in the two Krylov spaces (block-triangular
   exponential), psi recomputed from checkpoints every K steps (each
   recomputed segment must reproduce the next checkpoint bit for bit).
   DVR dimensions and diagonal potential terms only (PPQ_E_UNSUPPORTED on
   lattice dimensions or with product terms of ppq_add_term). */

/* Replaces coefficient and factor parameters (2 per factor, layout of
   ppq_add_potential_term; params may be NULL) of potential term `term`
   (0-based, in order of addition).  For finite-difference checks. */
int ppq_set_potential_term(ppq_ctx *ctx, int term, double coef, const double *params);

/* Declares one term of dV/dtheta_param (a trainable potential parameter,
   0 <= param < 32), a sum-of-products term in the layout of
   ppq_add_potential_term; a parameter may have several terms. */
int ppq_add_potential_derivative(ppq_ctx *ctx, int param, double coef, int nfac, const int32_t *dims,
                                 const int32_t *kinds, const double *params, const double *tables);

/* Recording run: initial packet (as ppq_init_gaussian), nsteps of step +
   adaption, active sets kept on the device, psi checkpointed every
   checkpoint_every steps.  J (may be NULL) receives the survival probability. */
int ppq_adjoint_record(ppq_ctx *ctx, const double *centre, const double *momentum, const double *width,
                       double eps, int nsteps, double dt, int m, int checkpoint_every, double *J);

/* Forward map on the recorded (frozen) sets from a packet with the given
   centre and momentum (width of the recording) and the current potential:
   J for finite differences.  Leaves the recording intact. */
int ppq_adjoint_frozen(ppq_ctx *ctx, const double *centre, const double *momentum, double *J);

/* Gradient of J at the recording's packet and the current potential:
   dJ_dparam[nparam] (parameters declared by ppq_add_potential_derivative),
   dJ_dcentre[D], dJ_dmomentum[D] (any may be NULL).  Synchronises. */
int ppq_adjoint_gradient(ppq_ctx *ctx, double *dJ_dparam, double *dJ_dcentre, double *dJ_dmomentum);

/* Measurement helper: applies H to the current state `nrep` times (after
   one untimed application), with a HIP event recorded on the context stream
   before each application and after the last, and returns the median time
   of one application in ms (all passes of one P_A H P_A product) and, when
   ms_mean is not NULL, the mean over the nrep back-to-back applications.
   The input is the state (FP64 contexts) or its normalised FP32 copy (FP32
   contexts); the output goes to an internal work vector.  Synchronises.
   PPQ_E_ARG unless 1 <= nrep <= 100000. */
int ppq_time_apply(ppq_ctx *ctx, int nrep, double *ms_median, double *ms_mean);

/* Fiber counts of the current set: nf[k] = number of dimension-k fibers
   (lines of the set along dimension k), k < D.  Synchronises. */
int ppq_fiber_counts(ppq_ctx *ctx, int64_t *nf);

/* Phases of a propagation step, for ppq_timings. */
enum {
    PPQ_PHASE_HPSI = 0,      /* the m products H_A v_j of the Krylov build (Sec. II.B.2) */
    PPQ_PHASE_KRYLOV = 1,    /* normalisation, CGS2 dot products and updates, small exponential, recombination */
    PPQ_PHASE_ADAPT = 2,     /* threshold, neighbours, compaction and coefficient carry (Sec. II.E) */
    PPQ_PHASE_TABLES = 3,    /* fiber tables of the new set and its potential cache (appendix) */
    PPQ_PHASE_OBS = 4,       /* observable records */
    PPQ_PHASE_N = 5
};

/* Turns per-phase timing on (on != 0: accumulators reset) or off.  While on,
   ppq_step, ppq_prune and ppq_propagate record a HIP event on the context
   stream at every phase boundary; the time between consecutive events goes to
   the phase that started at the first (GPU time line, so host waits inside a
   phase count for it).  Off by default: no events are recorded. */
int ppq_enable_timings(ppq_ctx *ctx, int on);

/* Milliseconds per phase accumulated since timing was turned on:
   ms[PPQ_PHASE_N] (host).  Synchronises. */
int ppq_timings(ppq_ctx *ctx, double *ms);

#ifdef __cplusplus
}
#endif
#endif
