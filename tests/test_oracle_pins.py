"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these compare the oracle with itself: every expected value comes from
a closed form, a textbook/library routine applied to the plain dense problem
(Kronecker products, scipy's expm / eigh), brute force on tiny inputs, or a
worked example printed in the paper (tests/golden).
"""
import ctypes
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import oracle as orc
from oracle.model import Model, sine_dvr_grid, sine_dvr_kinetic, pvb_projection
from workloads import card, random_active_set, random_complex, random_dense_factor
from workloads.cards import _power

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# dense references
# ---------------------------------------------------------------------------
def kron_dim(n, k, h):
    """I x ... x h (at k) x ... x I as a dense matrix."""
    out = np.ones((1, 1), dtype=np.complex128)
    for j, nj in enumerate(n):
        out = np.kron(out, h if j == k else np.eye(nj))
    return out


def dense_h(model):
    n = model.n
    N = int(np.prod(n))
    H = np.zeros((N, N), dtype=np.complex128)
    for k, h in enumerate(model.single_dim_ops()):
        H += kron_dim(n, k, h)
    if not model.pvb:
        H += np.diag(model.potential_full().ravel())
    return H


class RandomOp:
    """Random non-Hermitian SoP operator made directly in the C oracle."""

    def __init__(self, n, seed, nv=3, npair=2, ntriple=1):
        L = orc.lib()
        rng = np.random.default_rng(seed)
        self.n = list(n)
        D = len(n)
        nmax = max(n)
        self.m = L.orc_new(D, orc._ip(np.array(n, dtype=np.int32)))
        self.h = []
        for k in range(D):
            h = random_dense_factor(n[k], seed + 10 + k)
            self.h.append(h)
            L.orc_add_h(self.m, k, orc._dp(np.ascontiguousarray(h).view(np.float64)))
        self.v = []
        for t in range(nv):
            use = (rng.random(D) < 0.6).astype(np.int32)
            tab = rng.standard_normal((D, nmax))
            coef = float(rng.standard_normal())
            self.v.append((coef, use.copy(), tab.copy()))
            L.orc_add_vterm(self.m, coef, orc._ip(use), orc._dp(tab))
        self.pairs = []
        for t in range(npair if D > 1 else 0):
            k1, k2 = sorted(rng.choice(D, size=2, replace=False))
            h1 = random_dense_factor(n[k1], seed + 100 + t)
            h2 = random_dense_factor(n[k2], seed + 200 + t)
            c = complex(rng.standard_normal(), rng.standard_normal())
            self.pairs.append((c, k1, h1, k2, h2))
            L.orc_add_pair(self.m, c.real, c.imag, int(k1), int(k2),
                           orc._dp(np.ascontiguousarray(h1).view(np.float64)),
                           orc._dp(np.ascontiguousarray(h2).view(np.float64)))
        # products of three dense factors (general sum-of-products terms)
        self.prods = []
        for t in range(ntriple if D > 2 else 0):
            ks = sorted(int(v) for v in rng.choice(D, size=3, replace=False))
            hs = [random_dense_factor(n[k], seed + 300 + 10 * t + i) for i, k in enumerate(ks)]
            c = complex(rng.standard_normal(), rng.standard_normal())
            self.prods.append((c, ks, hs))
            flat = np.concatenate([np.ascontiguousarray(h).ravel() for h in hs])
            assert L.orc_add_prod(self.m, c.real, c.imag, 3, orc._ip(np.array(ks, dtype=np.int32)),
                                  orc._dp(flat.view(np.float64))) == 0

    def __del__(self):
        orc.lib().orc_free(self.m)

    def dense_pruned(self, keys):
        """Dense P H P with sequential truncated products, restricted to keys."""
        n = self.n
        N = int(np.prod(n))
        idx = np.asarray(keys, dtype=np.int64)
        H = np.zeros((N, N), dtype=np.complex128)
        for k, h in enumerate(self.h):
            H += kron_dim(n, k, h)
        V = np.zeros(N)
        digits = np.unravel_index(np.arange(N), n)
        for coef, use, tab in self.v:
            term = np.full(N, coef)
            for k in range(len(n)):
                if use[k]:
                    term = term * tab[k][digits[k]]
            V += term
        H += np.diag(V)
        Hr = H[np.ix_(idx, idx)]
        for c, k1, h1, k2, h2 in self.pairs:
            A = kron_dim(n, k1, h1)[np.ix_(idx, idx)]
            B = kron_dim(n, k2, h2)[np.ix_(idx, idx)]
            Hr = Hr + c * (A @ B)
        for c, ks, hs in self.prods:
            P = np.eye(idx.size, dtype=np.complex128)
            for k, h in zip(ks, hs):
                P = P @ kron_dim(n, k, h)[np.ix_(idx, idx)]
            Hr = Hr + c * P
        return Hr

    def apply_def(self, keys, x):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        x = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.zeros_like(x)
        orc.lib().orc_apply_def(self.m, keys.size, orc._up(keys), orc._dp(x.view(np.float64)),
                                orc._dp(y.view(np.float64)))
        return y

    def apply_fib(self, keys, x):
        L = orc.lib()
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        x = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.zeros_like(x)
        f = L.orc_fib_build(self.m, keys.size, orc._up(keys))
        L.orc_apply_fib(self.m, f, orc._dp(x.view(np.float64)), orc._dp(y.view(np.float64)))
        L.orc_fib_free(f)
        return y


# ---------------------------------------------------------------------------
# 1D builders
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,lo,hi,mass", [(48, -8.0, 8.0, 1.0), (24, -6.5, 6.5, 1.0), (7, -2.0, 3.0, 1.3)])
def test_sine_dvr_kinetic_eigenvalues(n, lo, hi, mass):
    """Particle in a box: the sine-DVR kinetic matrix has eigenvalues (k pi/L)^2/(2m) exactly."""
    T = sine_dvr_kinetic(n, lo, hi, mass)
    ev = np.linalg.eigvalsh(T)
    exact = (np.arange(1, n + 1) * np.pi / (hi - lo)) ** 2 / (2.0 * mass)
    assert np.allclose(T, T.T, atol=0, rtol=0)
    assert np.max(np.abs(ev - exact) / exact) < 1e-12


def test_harmonic_oscillator_eigenvalues_on_hh2d_grid():
    """H = (-d^2 + x^2)/2 (Fig. 1's oscillator) on the 48-point grid: E_k = k + 1/2 for low k."""
    q, _ = sine_dvr_grid(48, -8.0, 8.0)
    H = sine_dvr_kinetic(48, -8.0, 8.0, 1.0) + np.diag(0.5 * q * q)
    ev = np.linalg.eigvalsh(H)[:10]
    assert np.max(np.abs(ev - (np.arange(10) + 0.5))) < 1e-12


# ---------------------------------------------------------------------------
# pruned operator
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed", [((5,), 1), ((4, 6), 2), ((3, 5, 4), 3), ((3, 2, 4, 3), 4)])
def test_apply_def_full_fill_equals_kronecker(n, seed):
    op = RandomOp(n, seed)
    keys = np.arange(int(np.prod(n)), dtype=np.uint64)
    x = random_complex(keys.size, seed)
    y = op.apply_def(keys, x)
    ref = op.dense_pruned(keys) @ x
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,seed,fill", [((6, 7), 5, 0.4), ((5, 4, 6), 6, 0.3), ((4, 5, 3, 4), 7, 0.25),
                                         ((9, 8), 8, 0.05)])
def test_apply_def_pruned_equals_restricted_kronecker(n, seed, fill):
    op = RandomOp(n, seed)
    for blob in (True, False):
        keys = random_active_set(n, fill, seed, blob=blob)
        x = random_complex(keys.size, seed + 1)
        y = op.apply_def(keys, x)
        ref = op.dense_pruned(keys) @ x
        assert np.max(np.abs(y - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [5, 15, 33])
def test_fgh_kinetic_equals_spectral_definition(n):
    """The closed-form periodic FGH kinetic matrix equals (1/n) sum_k
    k^2/(2m) exp(i k (x_i - x_j)) over |k| <= (n-1) pi / L."""
    from oracle.model import fgh_grid, fgh_kinetic
    lo, hi, mass = -2.0, 3.5, 1.7
    x, _ = fgh_grid(n, lo, hi)
    L = hi - lo
    ks = 2.0 * np.pi * np.arange(-(n - 1) // 2, (n - 1) // 2 + 1) / L
    ref = np.real(np.exp(1j * ks[None, None, :] * (x[:, None, None] - x[None, :, None]))
                  @ (ks ** 2 / (2.0 * mass))) / n
    assert np.max(np.abs(fgh_kinetic(n, lo, hi, mass) - ref)) < 1e-12 * np.max(np.abs(ref))


def test_fgh_harmonic_eigenvalues():
    """Harmonic oscillator on a 41-point periodic Fourier grid over [-9, 9):
    the lowest eigenvalues are k + 1/2."""
    from oracle.model import fgh_grid, fgh_kinetic
    x, _ = fgh_grid(41, -9.0, 9.0)
    w = np.linalg.eigvalsh(fgh_kinetic(41, -9.0, 9.0, 1.0) + np.diag(0.5 * x * x))
    assert np.max(np.abs(w[:8] - (np.arange(8) + 0.5))) < 1e-9


def custom_factor_card(seed, terms=True):
    """small_3d with its own symmetric 1D matrices on dimensions 0 and 2."""
    cd = card("small_3d")
    if not terms:
        cd["terms"] = []
    rng = np.random.default_rng(seed)
    fac = {}
    for k in (0, 2):
        n = cd["n"][k]
        m = sine_dvr_kinetic(n, cd["lo"][k], cd["hi"][k], cd["mass"]) + 0.3 * rng.standard_normal((n, n)) / n
        fac[k] = ((m + m.T) / 2.0).tolist()
    cd["dim_factors"] = fac
    return cd


def test_card_dim_factors_equal_kronecker_sum():
    """A card's own 1D matrices: with no potential, O-def on the full grid is
    the Kronecker sum of the per-dimension matrices (dense)."""
    cd = custom_factor_card(5, terms=False)
    o = orc.Oracle(cd)
    n = cd["n"]
    hs = [np.array(cd["dim_factors"][k]) if k in cd["dim_factors"]
          else sine_dvr_kinetic(n[k], cd["lo"][k], cd["hi"][k], cd["mass"]) for k in range(3)]
    H = sum(kron_dim(n, k, hs[k]) for k in range(3))
    keys = o.full_keys()
    x = random_complex(keys.size, 6)
    assert np.max(np.abs(o.apply_def(keys, x) - H @ x)) < 1e-12 * np.max(np.abs(H @ x))


@pytest.mark.parametrize("n,seed", [((6, 7), 11), ((5, 4, 6), 12), ((4, 5, 3, 4), 13), ((3, 3, 3, 3, 3, 3), 14)])
def test_apply_fib_equals_def(n, seed):
    op = RandomOp(n, seed)
    for fill, blob in ((0.5, True), (0.2, False), (1.0, False)):
        keys = random_active_set(n, fill, seed, blob=blob)
        x = random_complex(keys.size, seed + 2)
        yd = op.apply_def(keys, x)
        yf = op.apply_fib(keys, x)
        assert np.max(np.abs(yd - yf)) <= 1e-12 * max(1.0, np.max(np.abs(yd)))


def _card_dense_pruned(cd, keys):
    """Dense reference of a card's pruned operator on a set, built here from
    the card's matrices: the kinetic Kronecker sum and the diagonal potential
    restricted to the set, plus every product term as the product of its
    factors' restricted Kronecker matrices (lowest dimension leftmost, so the
    highest acts first, each intermediate truncated to the set)."""
    from oracle.model import dense_matrix, factor_values, sine_dvr_grid, sine_dvr_kinetic
    n = cd["n"]
    D = len(n)
    idx = np.asarray(keys, dtype=np.int64)
    q = [sine_dvr_grid(n[k], cd["lo"][k], cd["hi"][k])[0] for k in range(D)]
    H = np.zeros((idx.size, idx.size), dtype=np.complex128)
    for k in range(D):
        H += kron_dim(n, k, sine_dvr_kinetic(n[k], cd["lo"][k], cd["hi"][k], cd["mass"]))[np.ix_(idx, idx)]
    digits = np.unravel_index(idx, n)
    for t in cd["terms"]:
        coef = complex(t["coef"], t.get("coef_im", 0.0))
        fs = sorted(t["factors"], key=lambda f: f["dim"])
        if all(f["kind"] != "dense" for f in fs) and coef.imag == 0.0:
            v = np.full(idx.size, coef.real)
            for f in fs:
                v = v * factor_values(f, q[f["dim"]])[digits[f["dim"]]]
            H += np.diag(v)
            continue
        P = np.eye(idx.size, dtype=np.complex128)
        for f in fs:
            h = dense_matrix(f) if f["kind"] == "dense" else np.diag(factor_values(f, q[f["dim"]]))
            P = P @ kron_dim(n, f["dim"], h)[np.ix_(idx, idx)]
        H += coef * P
    return H


@pytest.mark.parametrize("fill,seed", [(1.0, 1), (0.45, 2), (0.2, 3)])
def test_card_product_terms_match_dense(fill, seed):
    """General sum-of-products terms of a card (dense real and complex
    factors, complex coefficients, a three-factor product, diagonal factors
    in a product): O-def and O-fib equal the dense restricted products."""
    cd = card("sop3d")
    o = orc.Oracle(cd)
    keys = np.arange(int(np.prod(cd["n"]))) if fill == 1.0 else random_active_set(cd["n"], fill, seed)
    x = random_complex(keys.size, seed + 40)
    ref = _card_dense_pruned(cd, keys) @ x
    y_def = o.apply_def(keys, x)
    assert np.max(np.abs(y_def - ref)) < 1e-13 * np.max(np.abs(ref))
    y_fib = o.apply_fib(keys, x)
    assert np.max(np.abs(y_fib - ref)) < 1e-13 * np.max(np.abs(ref))


def test_product_terms_hermiticity_and_arnoldi():
    """A product term keeps the pruned operator Hermitian only with one dense
    Hermitian factor and a real coefficient (diagonal factors commute with
    the truncation); then the oracle steps with Lanczos, else Arnoldi, and
    one step of either equals exp(-i H dt) psi on the full grid (scipy)."""
    base = card("small_3d")
    sop = card("sop3d")
    herm = dict(base, terms=base["terms"] + sop["terms"][6:7])   # symmetric dense x diagonal
    cases = [(base, True), (herm, True), (sop, False),
             (dict(base, terms=base["terms"] + sop["terms"][7:8]), False),   # complex pair
             (dict(base, terms=base["terms"] + sop["terms"][9:10]), False)]  # complex diagonal
    for cd, want in cases:
        o = orc.Oracle(cd)
        assert o.model.hermitian() == want
        assert o.arnoldi == (0 if want else 1)
        keys = np.arange(int(np.prod(cd["n"])))
        c0 = random_complex(keys.size, 5)
        c0 /= np.linalg.norm(c0)
        H = _card_dense_pruned(cd, keys)
        if want:
            assert np.max(np.abs(H - H.conj().T)) < 1e-13
        o.set_state(keys, c0)
        o.sil_step(dt=0.05, m=16)
        _, c1 = o.state()
        assert np.max(np.abs(c1 - sla.expm(-0.05j * H) @ c0)) < 1e-11


def test_apply_single_point_and_empty():
    op = RandomOp((4, 5), 21)
    keys = np.array([7], dtype=np.uint64)
    x = np.array([1.5 - 0.5j])
    ref = op.dense_pruned(keys) @ x
    assert np.allclose(op.apply_def(keys, x), ref, rtol=1e-14, atol=0)
    assert np.allclose(op.apply_fib(keys, x), ref, rtol=1e-14, atol=0)
    empty = np.zeros(0, dtype=np.uint64)
    assert op.apply_def(empty, np.zeros(0, complex)).size == 0
    assert op.apply_fib(empty, np.zeros(0, complex)).size == 0


def test_card_operator_is_hermitian_and_matches_kronecker():
    o = orc.Oracle(card("small_3d"))
    H = dense_h(o.model)
    assert np.allclose(H, H.conj().T, atol=1e-13)
    keys = random_active_set(o.n, 0.4, 31)
    x = random_complex(keys.size, 32)
    idx = keys.astype(np.int64)
    ref = H[np.ix_(idx, idx)] @ x
    for y in (o.apply_def(keys, x), o.apply_fib(keys, x)):
        assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_appendix_range_example():
    """Ranges of a fiber's index set follow the appendix's worked example."""
    g = json.load(open(os.path.join(GOLDEN, "appendix_ranges.json")))
    o = orc.Oracle(card("small_2d"))
    n1 = o.n[1]
    # a fiber of dimension 1 at i_0 = 3 holding exactly the example digits
    keys = np.array([3 * n1 + d for d in g["digits"]], dtype=np.uint64)
    ranges = o.fiber_ranges(keys, 1)
    assert ranges == [[tuple(r) for r in g["ranges"]]]
    # and in the permuted (dimension 0) direction as well
    n0 = o.n[0]
    keys0 = np.array(sorted(d * n1 + 5 for d in g["digits"] if d < n0), dtype=np.uint64)
    r0 = o.fiber_ranges(keys0, 0)
    expect = [[(a, min(b, n0 - 1)) for a, b in g["ranges"] if a < n0]]
    assert r0 == expect


# ---------------------------------------------------------------------------
# small exponentials
# ---------------------------------------------------------------------------
def test_tridiag_expv_matches_expm():
    rng = np.random.default_rng(3)
    for m in (1, 2, 5, 10, 16):
        a = rng.standard_normal(m) * 3
        b = np.abs(rng.standard_normal(m - 1))
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        dt = 0.37
        ref = sla.expm(-1j * dt * T)[:, 0]
        y = orc.tridiag_expv(a, b, dt)
        assert np.max(np.abs(y - ref)) < 1e-13


def test_complex_expm_matches_scipy():
    rng = np.random.default_rng(4)
    for m in (1, 3, 10):
        A = (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) * 2.0
        assert np.max(np.abs(orc.cexpm(A) - sla.expm(A))) < 1e-12 * np.max(np.abs(sla.expm(A)))


# ---------------------------------------------------------------------------
# propagation
# ---------------------------------------------------------------------------
def _full_state(o):
    keys = o.full_keys()
    return keys, o.psi0_on(keys)


def test_sil_step_matches_dense_exponential():
    """Lanczos m=16 on a full tiny grid equals exp(-iH dt) psi (dense expm)."""
    o = orc.Oracle(card("small_2d"))
    keys, c0 = _full_state(o)
    o.set_state(keys, c0)
    H = dense_h(o.model)
    U = sla.expm(-1j * 0.05 * H)
    c = c0.copy()
    for _ in range(10):
        o.sil_step(dt=0.05, m=16)
        c = U @ c
    _, cg = o.state()
    assert np.max(np.abs(cg - c)) < 1e-12



def lanczos_betas(H, c0, m):
    """beta_0 .. beta_{m-2} of the Lanczos recurrence on a dense H, with a
    full reorthogonalisation by numpy's QR-free projections."""
    V = [c0 / np.linalg.norm(c0)]
    betas = []
    for j in range(m - 1):
        w = H @ V[j]
        for _ in range(2):
            for v in V:
                w = w - np.vdot(v, w) * v
        b = np.linalg.norm(w)
        betas.append(b)
        V.append(w / b)
    return betas


def test_adaptive_sil_order():
    """Adaptive SIL order (the integrator's accuracy tied to a tolerance,
    Sec. III.A) on a full tiny grid: the order picked is the first k whose
    estimate n0 dt^k / k! prod_{i<k} beta_i (betas from an independent dense
    Lanczos) is within the tolerance; the step is then within 10x the
    tolerance of exp(-iH dt) psi (dense expm); smaller tolerances never pick
    lower orders; tolerance 0 keeps the full order."""
    import math
    o = orc.Oracle(card("small_2d"))
    keys, c0 = _full_state(o)
    H = dense_h(o.model)
    dt, m = 0.05, 16
    U = sla.expm(-1j * dt * H)
    betas = lanczos_betas(H, c0, m)
    n0 = np.linalg.norm(c0)
    prev = 0
    for tol in (1e-4, 1e-7, 1e-10):
        want = m
        for k in range(1, m):
            est = n0 * dt ** k / math.factorial(k) * np.prod(betas[:k])
            if est <= tol:
                want = k
                break
        oo = orc.Oracle(card("small_2d", krylov_tol=tol))
        oo.set_state(keys, c0)
        used, _ = oo.sil_step(dt=dt, m=m)
        _, c1 = oo.state()
        assert used == want, (tol, used, want)
        assert 1 < used < m
        assert np.linalg.norm(c1 - U @ c0) <= 10 * tol
        assert used >= prev
        prev = used
    o.set_state(keys, c0)
    assert o.sil_step(dt=dt, m=m)[0] == m
    with pytest.raises(ValueError):
        orc.Oracle(card("small_2d", krylov_tol=-1.0))

def test_arnoldi_step_matches_dense_exponential():
    """Arnoldi on a non-Hermitian operator: matches expm of the dense restricted operator."""
    n = (4, 5)
    op = RandomOp(n, 41, nv=2, npair=1)
    keys = random_active_set(n, 0.6, 42)
    x = random_complex(keys.size, 43)
    x /= np.linalg.norm(x)
    A = op.dense_pruned(keys)
    A = A / np.max(np.abs(np.linalg.eigvals(A)))   # scale to unit spectral radius
    # rebuild the same operator scaled: easier to scale dt instead
    s = orc.lib().orc_state_new()
    orc.lib().orc_state_set(s, keys.size, orc._up(np.ascontiguousarray(keys)), orc._dp(x.view(np.float64)))
    f = orc.lib().orc_fib_build(op.m, keys.size, orc._up(np.ascontiguousarray(keys)))
    B = op.dense_pruned(keys)
    dt = 0.02
    used = orc.lib().orc_sil_step(op.m, f, s, dt, keys.size, 1, None)
    y = np.zeros_like(x)
    kk = np.zeros(keys.size, dtype=np.uint64)
    orc.lib().orc_state_get(s, orc._up(kk), orc._dp(y.view(np.float64)))
    orc.lib().orc_fib_free(f)
    orc.lib().orc_state_free(s)
    ref = sla.expm(-1j * dt * B) @ x
    assert used >= 1
    assert np.max(np.abs(y - ref)) < 1e-10


def _coherent_card():
    c = card("hh2d")
    c["terms"] = [t for t in c["terms"] if len(t["factors"]) == 1 and t["factors"][0]["p"] == 2]
    return c


def test_coherent_state_closed_form():
    """Uncoupled 2D oscillator: C(t) = prod_k exp(-it/2) exp(-|a_k|^2 (1 - exp(-it)))."""
    cd = _coherent_card()
    o = orc.Oracle(cd)
    keys, c0 = _full_state(o)
    o.set_state(keys, c0)
    tr, _ = o.propagate(nsteps=60, dt=0.05, m=16, prune=False)
    t = tr[:, 0]
    C = tr[:, 3] + 1j * tr[:, 4]
    ref = np.ones_like(C)
    for k in range(2):
        a = (cd["psi0"]["centre"][k] + 1j * cd["psi0"]["momentum"][k]) / np.sqrt(2.0)
        ref = ref * np.exp(-0.5j * t) * np.exp(-abs(a) ** 2 * (1.0 - np.exp(-1j * t)))
    assert np.max(np.abs(C - ref)) < 1e-10
    assert np.max(np.abs(tr[:, 2] - tr[0, 2])) < 1e-10        # energy conserved
    E = sum(0.5 + 0.5 * (cd["psi0"]["centre"][k] ** 2 + cd["psi0"]["momentum"][k] ** 2) for k in range(2))
    assert abs(tr[0, 2] - E) < 1e-10


def test_expect_q_follows_classical_trajectory():
    """Uncoupled harmonic oscillator (m = omega = 1): Ehrenfest's theorem is exact,
    <q_k>(t) = q0_k cos t + p0_k sin t, whatever the packet's shape."""
    cd = _coherent_card()
    o = orc.Oracle(cd)
    keys, c0 = _full_state(o)
    o.set_state(keys, c0)
    q0 = np.array(cd["psi0"]["centre"])
    p0 = np.array(cd["psi0"]["momentum"])
    dt = 0.05
    assert np.max(np.abs(o.expect_q() - q0)) < 1e-10
    for st in range(1, 41):
        o.sil_step(dt=dt, m=16)
        t = st * dt
        assert np.max(np.abs(o.expect_q() - (q0 * np.cos(t) + p0 * np.sin(t)))) < 1e-9


def test_acf_doubled_closed_form():
    """Real packet (zero momentum) on the uncoupled oscillator: sum c^2 after
    propagating to t is the closed-form C(2t)."""
    cd = _coherent_card()
    cd["psi0"] = dict(cd["psi0"], momentum=[0.0, 0.0])
    o = orc.Oracle(cd)
    keys, c0 = _full_state(o)
    o.set_state(keys, c0)
    dt = 0.05
    for st in range(1, 31):
        o.sil_step(dt=dt, m=16)
        if st % 10:
            continue
        t2 = 2 * st * dt
        ref = 1.0 + 0j
        for k in range(2):
            a = cd["psi0"]["centre"][k] / np.sqrt(2.0)
            ref *= np.exp(-0.5j * t2) * np.exp(-abs(a) ** 2 * (1.0 - np.exp(-1j * t2)))
        assert abs(o.acf_doubled() - ref) < 1e-9


@pytest.mark.parametrize("basis", ["pvb", "pw"])
def test_acf_doubled_on_lattices(basis):
    """C(2t) on a phase-space lattice basis is a^T B^T B a with B the map
    from the lattice coefficients to the DVR ones (the form after Eq. acorr):
    for a real packet, unpruned, it equals the C(t) record at twice the time
    (the dual-bra overlap) and the DVR run's sum of squares at t."""
    base = card("small_4d", n=[12, 12, 12, 12])
    base["terms"] = base["terms"][:2] + base["terms"][4:6]
    base["psi0"] = dict(base["psi0"], momentum=[0.0] * 4)
    lat = dict(base, basis=basis, lattice=[3, 4])
    ol = orc.Oracle(lat)
    od = orc.Oracle(base)
    for o in (ol, od):
        k, c0 = _full_state(o)
        o.set_state(k, c0)
    tr, _ = ol.propagate(nsteps=12, dt=0.05, m=14, prune=False)
    for o in (ol, od):
        k, c0 = _full_state(o)
        o.set_state(k, c0)
        o.propagate(nsteps=6, dt=0.05, m=14, prune=False)
    c2 = ol.acf_doubled()
    assert abs(c2 - complex(tr[12, 3], tr[12, 4])) < 1e-9
    assert abs(c2 - od.acf_doubled()) < 1e-9
    # the plain sum of squares of the lattice coefficients is not it (B^T B != I for pvb)
    if basis == "pvb":
        _, a = ol.state()
        assert abs(complex(np.sum(a * a)) - c2) > 1e-3


def test_expect_q_special_cases():
    """One grid point: <q_k> is that point's coordinate for any weight; a state
    mirror-symmetric in dimension k on a symmetric box: <q_k> = 0; lattice
    dimensions and the empty state: NaN."""
    cd = card("small_3d")
    o = orc.Oracle(cd)
    n = cd["n"]
    idx = (3, 7, 2)
    key = np.ravel_multi_index(idx, n)
    o.set_state(np.array([key], dtype=np.uint64), np.array([3.0 - 4.0j]))
    want = [sine_dvr_grid(n[k], cd["lo"][k], cd["hi"][k])[0][idx[k]] for k in range(3)]
    assert np.array_equal(o.expect_q(), np.array(want))
    # two points mirrored in dimension 0 (box symmetric about 0), equal weight
    lo, hi = cd["lo"][0], cd["hi"][0]
    assert lo == -hi
    a = (1, 4, 5)
    b = (n[0] - 2, 4, 5)
    keys = np.array(sorted([np.ravel_multi_index(a, n), np.ravel_multi_index(b, n)]), dtype=np.uint64)
    o.set_state(keys, np.array([0.6j, -0.6]))
    q = o.expect_q()
    assert abs(q[0]) < 1e-15
    assert q[1] == sine_dvr_grid(n[1], cd["lo"][1], cd["hi"][1])[0][4]
    o.set_state(np.zeros(0, dtype=np.uint64), np.zeros(0, dtype=np.complex128))
    assert np.all(np.isnan(o.expect_q()))
    op = orc.Oracle(card("small_2d", n=[12, 12], basis="pvb", lattice=[3, 4], lo=[-5.0, -5.0], hi=[5.0, 5.0]))
    op.init_state()
    assert np.all(np.isnan(op.expect_q()))


def test_unpruned_norm_and_energy_conserved():
    o = orc.Oracle(card("small_3d"))
    keys, c0 = _full_state(o)
    o.set_state(keys, c0)
    tr, h = o.propagate(nsteps=40, prune=False)
    assert np.max(np.abs(tr[:, 1] - tr[0, 1])) < 1e-13
    assert np.max(np.abs(tr[:, 2] - tr[0, 2])) < 1e-9
    assert len(set(h.tolist())) == 1


def test_pruned_norm_accounting():
    """SIL conserves the norm; adaption removes exactly the dropped |c|^2."""
    o = orc.Oracle(card("small_3d"))
    o.init_state()
    for _ in range(15):
        o.sil_step()
        k_before, c_before = o.state()
        n_before = np.sum(np.abs(c_before) ** 2)
        o.prune()
        k_after, c_after = o.state()
        kept = np.isin(k_before, k_after)
        dropped = np.sum(np.abs(c_before[~kept]) ** 2)
        assert abs(np.sum(np.abs(c_after) ** 2) - (n_before - dropped)) < 1e-14
        # retained coefficients are carried over untouched, new ones are zero
        pos = np.searchsorted(k_before, k_after)
        pos = np.minimum(pos, k_before.size - 1)
        old = k_before[pos] == k_after
        assert np.array_equal(c_after[old], c_before[pos[old]])
        assert np.all(c_after[~old] == 0)


def test_eps_zero_reproduces_unpruned():
    cd = card("small_3d")
    a = orc.Oracle(cd)
    b = orc.Oracle(cd)
    keys, c0 = _full_state(a)
    a.set_state(keys, c0)
    b.set_state(keys, c0)
    ta, _ = a.propagate(nsteps=20, eps=0.0)
    tb, _ = b.propagate(nsteps=20, prune=False)
    assert np.max(np.abs(ta[:, 1:5] - tb[:, 1:5])) < 1e-13
    assert np.all(ta[:, 5] == keys.size)


def test_adaptive_order_backward_step():
    """The adaptive order's estimate is a magnitude (|dt|^k): a backward step
    of the same length picks the same orders as a forward one, and a run
    forward then backward with a tolerance returns to the start (time
    reversal) within the accumulated tolerance."""
    tol = 1e-12
    o = orc.Oracle(card("small_2d", krylov_tol=tol))
    keys, c0 = _full_state(o)
    o.set_state(keys, c0)
    fwd = [o.sil_step(dt=0.05, m=16)[0] for _ in range(20)]
    bwd = [o.sil_step(dt=-0.05, m=16)[0] for _ in range(20)]
    assert all(1 < k < 16 for k in fwd + bwd)
    assert sorted(bwd) == sorted(fwd) or max(abs(a - b) for a, b in zip(sorted(fwd), sorted(bwd))) <= 1
    _, c = o.state()
    assert np.max(np.abs(c - c0)) < 100 * tol
    # the same state stepped forward and backward picks the same order
    for dt in (0.05, 0.02):
        used = []
        for sgn in (1.0, -1.0):
            oo = orc.Oracle(card("small_2d", krylov_tol=1e-8))
            oo.set_state(keys, c0)
            used.append(oo.sil_step(dt=sgn * dt, m=16)[0])
        assert used[0] == used[1] and 1 < used[0] < 16


def test_step_control_substeps():
    """Step size control (the integrator's accuracy tied to the tolerance,
    Sec. III.A): a step too long for the Krylov order at the tolerance runs
    as substeps, each meeting the tolerance below the order, and the step is
    then within a few times the tolerance of exp(-i H dt) (dense expm);
    without control the same order misses it by far.  The count follows the
    rule: doubled until every substep stops early, halved after a step whose
    substeps all stopped at order m/2 or below."""
    cd0 = card("small_2d")
    o = orc.Oracle(cd0)
    keys, c0 = _full_state(o)
    H = dense_h(o.model)
    dt, m, tol = 0.4, 10, 1e-10
    U = sla.expm(-1j * dt * H)
    plain = orc.Oracle(card("small_2d"))
    plain.set_state(keys, c0)
    plain.sil_step(dt=dt, m=m)
    err_plain = np.linalg.norm(plain.state()[1] - U @ c0)
    ctl = orc.Oracle(card("small_2d", krylov_tol=tol, max_substeps=64))
    ctl.set_state(keys, c0)
    tr, _ = ctl.propagate(nsteps=1, dt=dt, m=m, prune=False)
    err_ctl = np.linalg.norm(ctl.state()[1] - U @ c0)
    nsub = int(tr[1, 8])
    assert nsub > 1 and nsub & (nsub - 1) == 0          # a power of two
    assert tr[1, 7] < m
    assert err_ctl < 10 * nsub * tol < err_plain
    # a long run keeps every step within its substeps' tolerance
    ctl.set_state(keys, c0)
    tr, _ = ctl.propagate(nsteps=6, dt=dt, m=m, prune=False)
    U6 = np.linalg.matrix_power(U, 6)
    assert np.linalg.norm(ctl.state()[1] - U6 @ c0) < 60 * int(tr[1:, 8].max()) * tol
    assert np.all(tr[1:, 7] < m)
    # a short step needs one substep; too few allowed substeps is an error
    ctl.set_state(keys, c0)
    tr, _ = ctl.propagate(nsteps=1, dt=0.01, m=m, prune=False)
    assert tr[1, 8] == 1
    tight = orc.Oracle(card("small_2d", krylov_tol=1e-14, max_substeps=2))
    tight.set_state(keys, c0)
    with pytest.raises(RuntimeError):
        tight.propagate(nsteps=1, dt=2.0, m=6, prune=False)


def test_reversibility():
    o = orc.Oracle(card("small_2d"))
    keys, c0 = _full_state(o)
    o.set_state(keys, c0)
    for _ in range(20):
        o.sil_step(dt=0.05)
    for _ in range(20):
        o.sil_step(dt=-0.05)
    _, c = o.state()
    assert np.max(np.abs(c - c0)) < 1e-10


# ---------------------------------------------------------------------------
# adaption
# ---------------------------------------------------------------------------
def brute_adapt(n, keys, c, eps, lattice=None):
    n = list(n)
    total = int(np.prod(n))
    out = set()
    for key, v in zip(keys.tolist(), c):
        if v.real * v.real + v.imag * v.imag >= eps * eps:
            d = list(np.unravel_index(key, n))
            out.add(key)
            for k in range(len(n)):
                moves = []
                if lattice is None:
                    moves = [-1, 1]
                    ok = [0 <= d[k] + s < n[k] for s in moves]
                else:
                    ns, nl = lattice
                    s_, l_ = divmod(d[k], nl)
                    moves, ok = [], []
                    for ds, dl in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                        moves.append(ds * nl + dl)
                        ok.append(0 <= s_ + ds < ns and 0 <= l_ + dl < nl)
                for s, good in zip(moves, ok):
                    if good:
                        e = d.copy()
                        e[k] += s
                        out.add(int(np.ravel_multi_index(e, n)))
    assert all(0 <= k < total for k in out)
    return np.array(sorted(out), dtype=np.uint64)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_prune_matches_bruteforce(seed):
    cd = card("small_3d")
    o = orc.Oracle(cd)
    keys = random_active_set(o.n, 0.35, seed)
    rng = np.random.default_rng(seed)
    c = random_complex(keys.size, seed) * np.exp(rng.uniform(-12, 0, keys.size))
    eps = 1e-3
    # exact ties at |c| = eps (representable: re = eps, im = 0) and zeros
    c[::17] = eps
    c[5::23] = 0.0
    o.set_state(keys, c)
    nab = o.prune(eps=eps)
    k2, c2 = o.state()
    ref = brute_adapt(o.n, keys, c, eps)
    assert np.array_equal(k2, ref)
    assert nab == int(np.sum(c.real * c.real + c.imag * c.imag >= eps * eps))
    lookup = dict(zip(keys.tolist(), c))
    assert np.array_equal(c2, np.array([lookup.get(k, 0j) for k in k2.tolist()]))


def adversarial_prune_state(o, seed, eps=1e-3):
    keys = random_active_set(o.n, 0.35, seed)
    rng = np.random.default_rng(seed)
    c = random_complex(keys.size, seed) * np.exp(rng.uniform(-12, 0, keys.size))
    c[::17] = eps
    c[5::23] = 0.0
    return keys, c


@pytest.mark.parametrize("seed", [1, 2])
def test_prune_relative_exclusion_matches_bruteforce(seed):
    """Sec. II.E: functions are excluded only if more than r |A| of them would
    go; otherwise A' is united with A.  Thresholds just below, at and just
    above the dropped count."""
    cd = card("small_3d")
    o = orc.Oracle(cd)
    eps = 1e-3
    keys, c = adversarial_prune_state(o, seed, eps)
    plain = brute_adapt(o.n, keys, c, eps)
    dropped = np.setdiff1d(keys, plain).size
    n = keys.size
    assert 0 < dropped < n
    union = np.union1d(plain, keys).astype(np.uint64)
    cases = [(0.0, plain), ((dropped - 0.5) / n, plain), ((dropped + 0.5) / n, union), (1.0, union)]
    r_eq = dropped / n
    if r_eq * n == dropped:
        cases.append((r_eq, union))
    lookup = dict(zip(keys.tolist(), c))
    for r, want in cases:
        o.set_state(keys, c)
        o.prune(eps=eps, rel_excl=r)
        k2, c2 = o.state()
        assert np.array_equal(k2, want), r
        assert np.array_equal(c2, np.array([lookup.get(k, 0j) for k in k2.tolist()]))


def brute_adapt_pairs(n, keys, c, eps):
    """Ball radius sqrt(2): the radius-1 set plus every +-1 change in two
    dimensions at once (brute force over the kept points)."""
    n = list(n)
    out = set(brute_adapt(n, keys, c, eps).tolist())
    for key, v in zip(keys.tolist(), c):
        if v.real * v.real + v.imag * v.imag >= eps * eps:
            d = list(np.unravel_index(key, n))
            for k in range(len(n)):
                for l in range(k + 1, len(n)):
                    for a in (-1, 1):
                        for b in (-1, 1):
                            e = d.copy()
                            e[k] += a
                            e[l] += b
                            if 0 <= e[k] < n[k] and 0 <= e[l] < n[l]:
                                out.add(int(np.ravel_multi_index(e, n)))
    return np.array(sorted(out), dtype=np.uint64)


def test_prune_radius_sqrt2_stencil():
    """Sec. III.A's intermediate stencil: 2D^2 neighbours of an interior point,
    D + D(D-1)/2 of a corner, and brute force on adversarial states."""
    for name in ("small_3d", "small_4d"):
        cd = card(name, stencil=2)
        o = orc.Oracle(cd)
        n = cd["n"]
        D = len(n)
        for idx, want in (([v // 2 for v in n], 1 + 2 * D * D), ([0] * D, 1 + D + D * (D - 1) // 2)):
            key = np.ravel_multi_index(idx, n)
            o.set_state(np.array([key], dtype=np.uint64), np.array([1.0 + 0j]))
            o.prune(eps=0.5)
            assert o.state()[0].size == want, (name, idx)
    cd = card("small_3d", stencil=2)
    o = orc.Oracle(cd)
    for seed in (1, 2):
        keys, c = adversarial_prune_state(o, seed)
        o.set_state(keys, c)
        o.prune(eps=1e-3)
        assert np.array_equal(o.state()[0], brute_adapt_pairs(o.n, keys, c, 1e-3))



def dilate_moore(n, keys, c, eps):
    """Ball radius 2 by morphology: the kept functions as a boolean grid,
    dilated with the full 3^D structuring element (scipy), i.e. every grid
    point within Chebyshev distance 1 of a kept one."""
    from scipy.ndimage import binary_dilation
    kept = np.zeros(int(np.prod(n)), dtype=bool)
    k2 = c.real * c.real + c.imag * c.imag
    kept[keys[k2 >= eps * eps].astype(np.int64)] = True
    grown = binary_dilation(kept.reshape(n), structure=np.ones((3,) * len(n), dtype=bool))
    return np.flatnonzero(grown.ravel()).astype(np.uint64)


def test_prune_radius2_stencil():
    """Sec. III.A's most conservative stencil (ball radius 2): every
    combination of index changes, 3^D - 1 neighbours of an interior point,
    2^D - 1 of a corner; adversarial states against a morphological dilation
    of the kept set by the full 3^D block (scipy)."""
    for name in ("small_3d", "small_4d"):
        cd = card(name, stencil=3)
        o = orc.Oracle(cd)
        n = cd["n"]
        D = len(n)
        for idx, want in (([v // 2 for v in n], 3 ** D), ([0] * D, 2 ** D), ([v - 1 for v in n], 2 ** D)):
            key = np.ravel_multi_index(idx, n)
            o.set_state(np.array([key], dtype=np.uint64), np.array([1.0 + 0j]))
            o.prune(eps=0.5)
            assert o.state()[0].size == want, (name, idx)
    cd = card("small_3d", stencil=3)
    o = orc.Oracle(cd)
    for seed in (1, 2):
        keys, c = adversarial_prune_state(o, seed)
        o.set_state(keys, c)
        o.prune(eps=1e-3)
        k2, c2 = o.state()
        assert np.array_equal(k2, dilate_moore(o.n, keys, c, 1e-3))
        lookup = dict(zip(keys.tolist(), c))
        assert np.array_equal(c2, np.array([lookup.get(k, 0j) for k in k2.tolist()]))
    # radius 2 contains radius sqrt(2), which contains radius 1
    keys, c = adversarial_prune_state(o, 3)
    sets = []
    for st in (1, 2, 3):
        oo = orc.Oracle(card("small_3d", stencil=st))
        oo.set_state(keys, c)
        oo.prune(eps=1e-3)
        sets.append(set(oo.state()[0].tolist()))
    assert sets[0] < sets[1] < sets[2]
    for bad in (0, 4):
        with pytest.raises(ValueError):
            orc.Oracle(card("small_3d", stencil=bad))


def dilate_phase_space(shape, keys, c, eps, max_changes):
    """Adaption in phase space by morphology: the kept functions as a boolean
    array over the phase-space axes (the flat key reshaped to `shape`, which
    splits each lattice dimension into its cell and level indices), dilated
    by the block {-1, 0, 1}^axes restricted to at most `max_changes` nonzero
    entries (1: radius 1, 2: radius sqrt(2), all axes: radius 2)."""
    import itertools
    from scipy.ndimage import binary_dilation
    na = len(shape)
    st = np.zeros((3,) * na, dtype=bool)
    for off in itertools.product((0, 1, 2), repeat=na):
        if sum(o != 1 for o in off) <= max_changes:
            st[off] = True
    kept = np.zeros(int(np.prod(shape)), dtype=bool)
    k2 = c.real * c.real + c.imag * c.imag
    kept[keys[k2 >= eps * eps].astype(np.int64)] = True
    grown = binary_dilation(kept.reshape(shape), structure=st)
    return np.flatnonzero(grown.ravel()).astype(np.uint64)


@pytest.mark.parametrize("stencil", [1, 2, 3])
def test_prune_stencils_on_lattices(stencil):
    """The three balls of Sec. III.A counted in phase space: on 2D lattices
    (3 cells x 4 levels, and 4 x 3, per dimension) the adapted set equals a
    scipy dilation over the four phase-space axes, with carried
    coefficients; a single interior function gets 1 + 2A, 1 + 2A^2 and 3^A
    functions for A = 4 axes."""
    for ns, nl in ((3, 4), (4, 3)):
        cd = card("small_2d", n=[12, 12], basis="pvb", lattice=[ns, nl], lo=[-5.0, -5.0], hi=[5.0, 5.0],
                  stencil=stencil)
        o = orc.Oracle(cd)
        shape = [ns, nl, ns, nl]
        na = len(shape)
        for seed in (1, 2):
            keys = random_active_set(o.n, 0.3, seed)
            rng = np.random.default_rng(seed)
            c = random_complex(keys.size, seed) * np.exp(rng.uniform(-12, 0, keys.size))
            o.set_state(keys, c)
            o.prune(eps=1e-3)
            k2, c2 = o.state()
            assert np.array_equal(k2, dilate_phase_space(shape, keys, c, 1e-3, {1: 1, 2: 2, 3: na}[stencil]))
            lookup = dict(zip(keys.tolist(), c))
            assert np.array_equal(c2, np.array([lookup.get(k, 0j) for k in k2.tolist()]))
        centre = np.ravel_multi_index([1, 1, 1, 1], shape)
        o.set_state(np.array([centre], dtype=np.uint64), np.array([1.0 + 0j]))
        o.prune(eps=0.5)
        assert o.state()[0].size == {1: 1 + 2 * na, 2: 1 + 2 * na * na, 3: 3 ** na}[stencil]


def test_prune_edge_cases():
    o = orc.Oracle(card("small_2d"))
    total = int(np.prod(o.n))
    # empty S: everything below threshold -> empty set
    keys = np.arange(0, total, 3, dtype=np.uint64)
    o.set_state(keys, np.full(keys.size, 1e-9 + 0j))
    assert o.prune(eps=1e-3) == 0
    assert o.state()[0].size == 0
    # S = full grid -> full grid
    keys = np.arange(total, dtype=np.uint64)
    o.set_state(keys, np.ones(total, complex))
    o.prune(eps=0.5)
    assert o.state()[0].size == total
    # grid corners: neighbours outside the box are dropped, no wrap-around
    o.set_state(np.array([0, total - 1], dtype=np.uint64), np.ones(2, complex))
    o.prune(eps=0.5)
    n0, n1 = o.n
    expect = sorted({0, 1, n1, total - 1, total - 2, total - 1 - n1})
    assert o.state()[0].tolist() == expect


def test_neighbour_counts_golden():
    """One function above threshold in a 16-function mode adds 2 (line) or 4 (4x4 lattice) neighbours."""
    g = json.load(open(os.path.join(GOLDEN, "neighbour_counts.json")))
    m = g["mode_size"]
    line = orc.Oracle(card("small_2d", n=[m, 3], lo=[-4.0, -1.0], hi=[4.0, 1.0]))
    lat = orc.Oracle(card("small_2d", n=[m, m], basis="pvb", lattice=g["lattice"], lo=[-4.0, -4.0],
                          hi=[4.0, 4.0]))
    # interior function of mode 0 (digit 5 = lattice cell (1,1)); second dim at the box edge
    for o, added, frac in ((line, g["added_line"], g["fraction_line"]),
                           (lat, g["added_lattice"], g["fraction_lattice"])):
        n1 = o.n[1]
        key = 5 * n1 + 0
        o.set_state(np.array([key], dtype=np.uint64), np.array([1.0 + 0j]))
        o.prune(eps=0.5)
        k2, _ = o.state()
        d = np.array(np.unravel_index(k2.astype(np.int64), o.n))
        along0 = int(np.sum(d[1] == 0)) - 1
        assert along0 == added
        assert along0 / m == frac


def test_initial_set_matches_bruteforce():
    cd = card("small_3d")
    o = orc.Oracle(cd)
    nab = o.init_state()
    keys, c = o.state()
    full = o.full_keys()
    psi0 = o.psi0_on(full)
    ref = brute_adapt(o.n, full, psi0, cd["eps"])
    assert np.array_equal(keys, ref)
    assert nab == int(np.sum(psi0.real ** 2 + psi0.imag ** 2 >= cd["eps"] ** 2))
    assert np.allclose(c, o.psi0_on(keys), rtol=1e-14, atol=0)
    assert abs(np.sum(np.abs(psi0) ** 2) - 1.0) < 1e-14


# ---------------------------------------------------------------------------
# phase-space lattice (projected von Neumann, biorthogonal)
# ---------------------------------------------------------------------------
def test_pvb_unpruned_dynamics_is_similarity_of_dvr():
    """a = G^+ c: unpruned lattice dynamics maps back to the DVR dynamics exactly."""
    base = card("small_4d", n=[12, 12, 12, 12])
    base["terms"] = base["terms"][:2] + base["terms"][4:6]     # two Morse + two couplings
    lat = dict(base, basis="pvb", lattice=[3, 4])
    od = orc.Oracle(base)
    ol = orc.Oracle(lat)
    kd, cd0 = _full_state(od)
    kl, cl0 = _full_state(ol)
    od.set_state(kd, cd0)
    ol.set_state(kl, cl0)
    td, _ = od.propagate(nsteps=8, dt=0.05, m=12, prune=False)
    tl, _ = ol.propagate(nsteps=8, dt=0.05, m=12, prune=False)
    # autocorrelation through the dual bra tables equals the DVR one
    assert np.max(np.abs((td[:, 3] + 1j * td[:, 4]) - (tl[:, 3] + 1j * tl[:, 4]))) < 1e-9
    _, cdv = od.state()
    _, clat = ol.state()
    c_back = clat.reshape(ol.n)
    for k in range(4):
        c_back = np.moveaxis(np.tensordot(ol.model.GinvH[k], c_back, axes=([1], [k])), 0, k)
    assert np.max(np.abs(c_back.ravel() - cdv)) < 1e-9


@pytest.mark.parametrize("basis", ["pvb", "pw"])
def test_lattice_three_factor_terms_are_similarity_of_dvr(basis):
    """A three-factor product term (the 6D model's q_k q_l q_m couplings) and
    a dense factor in a phase-space lattice basis: the unpruned lattice
    dynamics maps back to the DVR dynamics (a similarity, every factor
    transformed as G^+ h G^{-+}; W^T h W for Weylets)."""
    base = card("small_3d", n=[12, 12, 12])
    rng = np.random.default_rng(4)
    sym = 0.02 * rng.standard_normal((12, 12))
    base["terms"] = base["terms"] + [
        {"coef": 0.004, "factors": [_power(0, 1), _power(1, 1), _power(2, 1)]},
        {"coef": 0.1, "factors": [{"dim": 1, "kind": "dense", "re": (sym + sym.T).tolist()}, _power(0, 1)]},
    ]
    lat = dict(base, basis=basis, lattice=[3, 4])
    od = orc.Oracle(base)
    ol = orc.Oracle(lat)
    kd, cd0 = _full_state(od)
    kl, cl0 = _full_state(ol)
    od.set_state(kd, cd0)
    ol.set_state(kl, cl0)
    td, _ = od.propagate(nsteps=6, dt=0.05, m=14, prune=False)
    tl, _ = ol.propagate(nsteps=6, dt=0.05, m=14, prune=False)
    assert np.max(np.abs((td[:, 3] + 1j * td[:, 4]) - (tl[:, 3] + 1j * tl[:, 4]))) < 1e-9
    _, cdv = od.state()
    _, clat = ol.state()
    c_back = clat.reshape(ol.n)
    for k in range(3):
        c_back = np.moveaxis(np.tensordot(ol.model.GinvH[k], c_back, axes=([1], [k])), 0, k)
    assert np.max(np.abs(c_back.ravel() - cdv)) < 1e-9


def test_pw_basis_is_orthogonal():
    """Projected Weylets (Sec. II.D): W = Phi S^{-1/2} is real and orthogonal,
    and its columns span the DVR space (W W^T = I as well)."""
    from oracle.model import pw_projection
    for n, lo, hi, nx, npm in ((12, -5.0, 5.0, 3, 4), (48, -3.0, 9.0, 6, 8)):
        q, dx = sine_dvr_grid(n, lo, hi)
        W = pw_projection(q, dx, lo, hi, nx, npm)
        assert np.max(np.abs(W.imag)) == 0.0
        assert np.max(np.abs(W.conj().T @ W - np.eye(n))) < 1e-12
        assert np.max(np.abs(W @ W.conj().T - np.eye(n))) < 1e-12


def test_pw_unpruned_dynamics_is_similarity_of_dvr():
    """a = W^T c: unpruned projected-Weylet dynamics maps back to the DVR
    dynamics exactly, and C(t) agrees."""
    base = card("small_4d", n=[12, 12, 12, 12])
    base["terms"] = base["terms"][:2] + base["terms"][4:6]
    lat = dict(base, basis="pw", lattice=[3, 4])
    od = orc.Oracle(base)
    ol = orc.Oracle(lat)
    kd, cd0 = _full_state(od)
    kl, cl0 = _full_state(ol)
    od.set_state(kd, cd0)
    ol.set_state(kl, cl0)
    td, _ = od.propagate(nsteps=8, dt=0.05, m=12, prune=False)
    tl, _ = ol.propagate(nsteps=8, dt=0.05, m=12, prune=False)
    assert np.max(np.abs((td[:, 3] + 1j * td[:, 4]) - (tl[:, 3] + 1j * tl[:, 4]))) < 1e-9
    _, cdv = od.state()
    _, clat = ol.state()
    c_back = clat.reshape(ol.n)
    for k in range(4):
        c_back = np.moveaxis(np.tensordot(ol.model.G[k], c_back, axes=([1], [k])), 0, k)
    assert np.max(np.abs(c_back.ravel() - cdv)) < 1e-9



@pytest.mark.parametrize("basis", ["pvb", "pw"])
def test_lattices_on_fourier_grids_are_similarity_of_fgh(basis):
    """Lattices projected on periodic Fourier grids (the paper's setting for
    its double well, Sec. III.A): the unpruned lattice dynamics maps back to
    the FGH DVR dynamics exactly, C(t) included, on a 15 x 15 grid with a
    3 x 5 lattice per dimension. The projection uses the FGH points and
    weight (hi - lo) / n: the middle cell's projected Gaussians have unit
    norm on the grid (the sine-DVR weight (hi - lo) / (n + 1) would give
    n / (n + 1))."""
    base = card("small_2d", n=[15, 15], fgh=[0, 1])
    lat = dict(base, basis=basis, lattice=[3, 5])
    od = orc.Oracle(base)
    ol = orc.Oracle(lat)
    assert np.allclose(ol.model.q[0], od.model.q[0], rtol=0, atol=0)
    if basis == "pvb":
        norms = np.sum(np.abs(ol.model.G[0]) ** 2, axis=0).reshape(3, 5)
        assert np.max(np.abs(norms[1] - 1.0)) < 1e-3
    kd, cd0 = _full_state(od)
    kl, cl0 = _full_state(ol)
    od.set_state(kd, cd0)
    ol.set_state(kl, cl0)
    td, _ = od.propagate(nsteps=8, dt=0.05, m=14, prune=False)
    tl, _ = ol.propagate(nsteps=8, dt=0.05, m=14, prune=False)
    assert np.max(np.abs((td[:, 3] + 1j * td[:, 4]) - (tl[:, 3] + 1j * tl[:, 4]))) < 1e-9
    _, cdv = od.state()
    _, clat = ol.state()
    back = ol.model.G if basis == "pw" else ol.model.GinvH
    c_back = clat.reshape(ol.n)
    for k in range(2):
        c_back = np.moveaxis(np.tensordot(back[k], c_back, axes=([1], [k])), 0, k)
    assert np.max(np.abs(c_back.ravel() - cdv)) < 1e-9

@pytest.mark.parametrize("s", [2, 3])
def test_pvb_lattice_geometry(s):
    """Sec. II.B.1: the von Neumann lattice's cells have width dx = (hi-lo)/n_s
    and centres x_s = lo + (s+1/2) dx; its momenta p_l are spaced dp with
    dx dp = 2 pi and centred on zero; the Gaussians have alpha = dp/(2 dx).
    Checked through the moments of the projected functions on a fine grid:
    <x> = x_s, Var x = 1/(4 alpha) (|g|^2 ~ exp(-2 alpha (x-x_s)^2)), and from
    the Fourier transform <p> = p_l, Var p = alpha."""
    lo, hi, ns, nl = -3.0, 9.0, 6, 8
    q, dxg = sine_dvr_grid(1201, lo, hi)
    G = pvb_projection(q, dxg, lo, hi, ns, nl)
    dX = (hi - lo) / ns
    dP = 2.0 * np.pi / dX
    alpha = dP / (2.0 * dX)
    k = 2.0 * np.pi * np.fft.fftfreq(q.size, dxg)
    for l in range(nl):
        g = G[:, s * nl + l] / np.sqrt(dxg)
        w = np.abs(g) ** 2
        assert abs(np.sum(w) * dxg - 1.0) < 1e-9          # normalised Gaussians
        mx = np.sum(w * q) / np.sum(w)
        vx = np.sum(w * (q - mx) ** 2) / np.sum(w)
        ghat = np.abs(np.fft.fft(g)) ** 2
        mp = np.sum(ghat * k) / np.sum(ghat)
        vp = np.sum(ghat * (k - mp) ** 2) / np.sum(ghat)
        assert abs(mx - (lo + (s + 0.5) * dX)) < 1e-9
        assert abs(mp - (l - 0.5 * (nl - 1)) * dP) < 1e-8
        assert abs(vx * 4.0 * alpha - 1.0) < 1e-8
        assert abs(vp / alpha - 1.0) < 1e-8
    # neighbouring momenta differ by dp = 2 pi / dx: the lattice has one function per phase-space cell of area 2 pi
    assert abs(dX * dP - 2.0 * np.pi) < 1e-14


def test_factor_values_closed_forms():
    """Diagonal potential factors at points where their closed forms are
    known: the Morse factor (1 - e^{-a (q - q0)})^2 is 0 at the minimum q0,
    1/4 at q0 + ln 2 / a, 1 at q0 - ln 2 / a and tends to 1 (the
    dissociation limit) far out; q^p is the plain power."""
    from oracle.model import factor_values
    a, q0 = 1.3, 0.4
    q = np.array([q0, q0 + np.log(2.0) / a, q0 - np.log(2.0) / a, q0 + 40.0])
    v = factor_values({"kind": "morse", "a": a, "q0": q0}, q)
    assert np.allclose(v, [0.0, 0.25, 1.0, 1.0], rtol=0, atol=1e-14)
    qq = np.array([-2.0, 0.5, 3.0])
    assert np.allclose(factor_values({"kind": "power", "p": 3}, qq), [-8.0, 0.125, 27.0], rtol=0, atol=0)


def test_pvb_coefficients_are_overlaps():
    """Eq. psi_exp_pvb: lattice coefficients are G^+ c_chi; G's columns are the projected Gaussians."""
    q, dx = sine_dvr_grid(16, -6.0, 6.0)
    G = pvb_projection(q, dx, -6.0, 6.0, 4, 4)
    # each projected Gaussian is (almost) normalised on the grid: sum_j w_j |g(x_j)|^2 ~ 1
    norms = np.sum(np.abs(G) ** 2, axis=0)
    assert np.all(np.abs(norms[4:12] - 1.0) < 0.05)     # interior cells; edges leak out of the box
    assert np.linalg.cond(G) < 10.0


# ---------------------------------------------------------------------------
# frozen-set forward map (reference of the adjoint gradient)
# ---------------------------------------------------------------------------
def test_frozen_forward_equals_dense_exponentials():
    """psi_{n+1} = R_{n+1} exp(-i H_{A_n} dt) psi_n with dense restricted H, scipy expm."""
    from oracle import adjoint as adj
    cd = card("small_2d", eps=2e-3)
    o = orc.Oracle(cd)
    o.init_state()
    sizes, keys = o.propagate_record(12, m=16)
    assert len(set(sizes.tolist())) > 1            # the set really changes
    offs = np.concatenate([[0], np.cumsum(sizes)])
    H = dense_h(o.model)
    k0 = keys[: sizes[0]].astype(np.int64)
    psi = o.psi0_on(k0)
    for st in range(12):
        ka = keys[offs[st]: offs[st + 1]].astype(np.int64)
        kb = keys[offs[st + 1]: offs[st + 2]].astype(np.int64)
        psi = sla.expm(-1j * cd["dt"] * H[np.ix_(ka, ka)]) @ psi
        pos = {int(k): i for i, k in enumerate(ka)}
        psi = np.array([psi[pos[int(k)]] if int(k) in pos else 0j for k in kb])
    f = orc.Oracle(cd)
    f.set_state(keys[: sizes[0]], f.psi0_on(keys[: sizes[0]]))
    f.propagate_frozen(sizes, keys, m=16)
    kf, cf = f.state()
    assert np.array_equal(kf.astype(np.int64), keys[offs[12]: offs[13]].astype(np.int64))
    assert np.max(np.abs(cf - psi)) < 1e-11


def test_fd_gradient_is_converged():
    """Central differences at two step sizes agree (the reference is smooth and resolved)."""
    from oracle import adjoint as adj
    cd = card("small_adjoint4d", nsteps=6)
    sizes, keys = adj.record_sets(cd)
    names = ["D0", "a1", "lam01", "centre0", "momentum2"]
    g1 = adj.fd_gradient(cd, names, sizes, keys, rel=1e-5)
    g2 = adj.fd_gradient(cd, names, sizes, keys, rel=1e-4)
    scale = max(abs(v) for v in g1.values())
    for nm in names:
        assert abs(g1[nm] - g2[nm]) < 1e-6 * scale, nm


@pytest.mark.parametrize("name", ["dwell2d", "dwell2d_literal"])
def test_double_well_potential_closed_form(name):
    """The double well's sum-of-products terms (Eq. ex_dwell written out in
    powers) equal 6.4 (x-1)^2 (x-2)^2 + 37.5 (y-2)^2 + c(x, y) on its Fourier
    grids, with the coupling c = 10 x^2 (y-2) of the card's reading or the
    printed 10 x^2 y.  The reading keeps the double well the paper names:
    along y = 2 the minima sit at x = 1 and 2 (V = 0) with a 0.4 barrier at
    x = 1.5; the printed form has one minimum near x = 0.49 and puts the
    packet's centre (2.1, 2.05) about 80 units above it."""
    from oracle.model import factor_values, fgh_grid, term_coef
    cd = card(name)
    x, _ = fgh_grid(cd["n"][0], cd["lo"][0], cd["hi"][0])
    y, _ = fgh_grid(cd["n"][1], cd["lo"][1], cd["hi"][1])

    def sop(xv, yv):
        q = (np.asarray(xv, float), np.asarray(yv, float))
        tot = np.zeros(np.broadcast(*q).shape, complex)
        for t in cd["terms"]:
            v = term_coef(t) * np.ones_like(tot)
            for f in t["factors"]:
                v = v * factor_values(f, q[f["dim"]])
            tot = tot + v
        return tot.real

    X, Y = np.meshgrid(x, y, indexing="ij")
    coupling = 10.0 * X ** 2 * (Y if name == "dwell2d_literal" else Y - 2.0)
    ref = 6.4 * (X - 1) ** 2 * (X - 2) ** 2 + 37.5 * (Y - 2) ** 2 + coupling
    assert np.max(np.abs(sop(X, Y) - ref)) < 1e-10 * np.max(np.abs(ref))
    xs = np.linspace(-0.5, 3.7, 42001)
    vline = sop(xs, 2.0 * np.ones_like(xs))
    if name == "dwell2d":
        assert abs(sop(1.0, 2.0)) < 1e-12 and abs(sop(2.0, 2.0)) < 1e-12
        assert abs(sop(1.5, 2.0) - 0.4) < 1e-12
        left, right = xs < 1.5, xs > 1.5
        assert abs(xs[left][np.argmin(vline[left])] - 1.0) < 1e-3
        assert abs(xs[right][np.argmin(vline[right])] - 2.0) < 1e-3
    else:
        assert abs(xs[np.argmin(vline)] - 0.493) < 2e-3
        assert sop(2.1, 2.05) - vline.min() > 75.0


@pytest.mark.parametrize("basis", ["pvb", "pw"])
def test_lattice_constant_and_same_dimension_terms(basis):
    """A reduced double well (15 x 9 Fourier grid, lattices 5 x 3 and 3 x 3)
    with its constant term (175.6) and an added two-factor term on one
    dimension (0.3 x * x): the unpruned lattice dynamics is the similarity
    of the FGH dynamics, C(t) included, so a dropped constant (a phase
    e^{-i 175.6 t}) or a dropped term fails it."""
    base = card("dwell2d", n=[15, 9], lattice=[[5, 3], [3, 3]])
    base["terms"] = base["terms"] + [{"coef": 0.3, "factors": [{"dim": 0, "kind": "power", "p": 1},
                                                               {"dim": 0, "kind": "power", "p": 1}]}]
    lat = dict(base, basis=basis)
    od = orc.Oracle(base)
    ol = orc.Oracle(lat)
    kd, cd0 = _full_state(od)
    kl, cl0 = _full_state(ol)
    od.set_state(kd, cd0)
    ol.set_state(kl, cl0)
    td, _ = od.propagate(nsteps=6, dt=0.02, m=16, prune=False)
    tl, _ = ol.propagate(nsteps=6, dt=0.02, m=16, prune=False)
    cdt = td[:, 3] + 1j * td[:, 4]
    clt = tl[:, 3] + 1j * tl[:, 4]
    assert np.max(np.abs(cdt - clt)) < 1e-9
    # the constant enters as a phase: without it C(t) turns by 175.6 t
    assert abs(np.angle(cdt[-1] / clt[-1])) < 1e-8
