"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only tests, the package smoke check and the benchmark's CPU-baseline leg
import this module.  It loads ``liboracle.so`` built from ``ppq_oracle.c``
(``python -m oracle.build``) and assembles the model from ``oracle.model``.
"""
import ctypes
import os

import numpy as np

from .model import Model

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OBS_FIELDS = ("t", "norm2", "energy", "acf_re", "acf_im", "n_active", "n_above", "krylov_used", "substeps")

_c_int64_p = ctypes.POINTER(ctypes.c_int64)
_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_u64_p = ctypes.POINTER(ctypes.c_uint64)
_c_i32_p = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from .build import build
            build()
        L = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        L.orc_new.restype = vp
        L.orc_new.argtypes = [ctypes.c_int, _c_i32_p]
        L.orc_free.argtypes = [vp]
        L.orc_add_h.argtypes = [vp, ctypes.c_int, _c_double_p]
        L.orc_add_vterm.argtypes = [vp, ctypes.c_double, _c_i32_p, _c_double_p]
        L.orc_add_pair.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   _c_double_p, _c_double_p]
        L.orc_add_prod.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _c_i32_p, _c_double_p]
        L.orc_set_lattice.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_apply_def.argtypes = [vp, ctypes.c_int64, _c_u64_p, _c_double_p, _c_double_p]
        L.orc_fib_build.restype = vp
        L.orc_fib_build.argtypes = [vp, ctypes.c_int64, _c_u64_p]
        L.orc_fib_free.argtypes = [vp]
        L.orc_apply_fib.argtypes = [vp, vp, _c_double_p, _c_double_p]
        L.orc_tridiag_expv.argtypes = [ctypes.c_int, _c_double_p, _c_double_p, ctypes.c_double, _c_double_p]
        L.orc_cexpm.argtypes = [ctypes.c_int, _c_double_p, _c_double_p]
        L.orc_state_new.restype = vp
        L.orc_state_free.argtypes = [vp]
        L.orc_state_set.argtypes = [vp, ctypes.c_int64, _c_u64_p, _c_double_p]
        L.orc_state_count.restype = ctypes.c_int64
        L.orc_state_count.argtypes = [vp]
        L.orc_state_get.argtypes = [vp, _c_u64_p, _c_double_p]
        L.orc_sil_step.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, _c_double_p]
        L.orc_set_stencil.argtypes = [vp, ctypes.c_int]
        L.orc_set_krylov_tol.argtypes = [vp, ctypes.c_double]
        L.orc_set_max_substeps.argtypes = [vp, ctypes.c_int]
        L.orc_prune.restype = ctypes.c_int64
        L.orc_prune.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double]
        L.orc_init_product.restype = ctypes.c_int64
        L.orc_init_product.argtypes = [vp, vp, _c_double_p, ctypes.c_double]
        L.orc_observe.argtypes = [vp, vp, vp, _c_double_p, ctypes.c_double, _c_double_p]
        L.orc_set_hash.restype = ctypes.c_uint64
        L.orc_set_hash.argtypes = [ctypes.c_int64, _c_u64_p]
        L.orc_propagate.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, _c_double_p, _c_double_p, _c_u64_p]
        L.orc_fib_count.restype = ctypes.c_int64
        L.orc_fib_count.argtypes = [vp, ctypes.c_int]
        L.orc_fib_ranges.argtypes = [vp, ctypes.c_int, ctypes.c_int64, ctypes.c_int, _c_i32_p, _c_i32_p]
        L.orc_apply_def_at.argtypes = [vp, ctypes.c_int64, _c_u64_p, _c_double_p, ctypes.c_int64, _c_int64_p,
                                       _c_double_p]
        L.orc_propagate_record.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                           _c_int64_p, ctypes.POINTER(_c_u64_p)]
        L.orc_free_buffer.argtypes = [vp]
        L.orc_propagate_frozen.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _c_int64_p,
                                           _c_u64_p]
        _LIB = L
    return _LIB


def _dp(a):
    return a.ctypes.data_as(_c_double_p)


def _up(a):
    return a.ctypes.data_as(_c_u64_p)


def _ip(a):
    return a.ctypes.data_as(_c_i32_p)


def _cplx(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def set_hash(keys):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    return int(lib().orc_set_hash(keys.size, _up(keys)))


def tridiag_expv(alpha, beta, dt):
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    n = alpha.size
    b = np.zeros(max(n, 1))
    b[: beta.size] = beta
    y = np.zeros(n, dtype=np.complex128)
    lib().orc_tridiag_expv(n, _dp(alpha), _dp(b), dt, _dp(y.view(np.float64)))
    return y


def cexpm(a):
    a = _cplx(a)
    out = np.zeros_like(a)
    lib().orc_cexpm(a.shape[0], _dp(a.view(np.float64)), _dp(out.view(np.float64)))
    return out


class Oracle:
    """A model card made into the C oracle's operator, plus a state."""

    def __init__(self, card):
        self.card = card
        self.model = Model(card)
        m = self.model
        self.D = m.D
        self.n = m.n
        self.nmax = max(m.n)
        L = lib()
        self._m = L.orc_new(self.D, _ip(np.array(m.n, dtype=np.int32)))
        for k, h in enumerate(m.single_dim_ops()):
            hh = _cplx(h)
            L.orc_add_h(self._m, k, _dp(hh.view(np.float64)))
        for coef, tabs in m.diag_terms():
            use = np.zeros(self.D, dtype=np.int32)
            tab = np.zeros((self.D, self.nmax))
            for k, v in tabs.items():
                use[k] = 1
                tab[k, : v.size] = v
            L.orc_add_vterm(self._m, float(coef), _ip(use), _dp(tab))
        for coef, dims, mats in m.product_terms():
            flat = np.concatenate([_cplx(h).ravel() for h in mats])
            if L.orc_add_prod(self._m, float(np.real(coef)), float(np.imag(coef)), len(dims),
                              _ip(np.array(dims, dtype=np.int32)), _dp(flat.view(np.float64))) != 0:
                raise ValueError("bad product term")
        if m.pvb:
            for k in range(self.D):
                ns, nl = m.lattices[k]
                L.orc_set_lattice(self._m, k, ns, nl)
        if card.get("krylov_tol", 0.0) and L.orc_set_krylov_tol(self._m, float(card["krylov_tol"])) != 0:
            raise ValueError("krylov_tol must be >= 0")
        if card.get("max_substeps", 1) != 1 and L.orc_set_max_substeps(self._m, int(card["max_substeps"])) != 0:
            raise ValueError("max_substeps must be in [1, 1024]")
        if card.get("stencil", 1) != 1 and L.orc_set_stencil(self._m, int(card["stencil"])) != 0:
            raise ValueError("stencil must be 1, 2 or 3")
        self.arnoldi = 0 if m.hermitian() else 1
        self._init_tabs = self._pack(m.init_tables())
        self._bra_tabs = self._pack(m.bra_tables())
        self._s = L.orc_state_new()
        self._fib = None

    def _pack(self, tables):
        out = np.zeros((self.D, self.nmax), dtype=np.complex128)
        for k, t in enumerate(tables):
            out[k, : t.size] = t
        return out

    def __del__(self):
        try:
            L = lib()
            if self._fib:
                L.orc_fib_free(self._fib)
            L.orc_state_free(self._s)
            L.orc_free(self._m)
        except Exception:
            pass

    # --- state -------------------------------------------------------------
    def set_state(self, keys, coeff):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        c = _cplx(coeff)
        if lib().orc_state_set(self._s, keys.size, _up(keys), _dp(c.view(np.float64))) != 0:
            raise ValueError("keys must be strictly ascending")
        self._drop_fib()

    def state(self):
        L = lib()
        n = L.orc_state_count(self._s)
        keys = np.zeros(n, dtype=np.uint64)
        c = np.zeros(n, dtype=np.complex128)
        L.orc_state_get(self._s, _up(keys), _dp(c.view(np.float64)))
        return keys, c

    def init_state(self, eps=None):
        eps = self.card["eps"] if eps is None else eps
        nab = lib().orc_init_product(self._m, self._s, _dp(self._init_tabs.view(np.float64)), eps)
        self._drop_fib()
        return int(nab)

    def _drop_fib(self):
        if self._fib:
            lib().orc_fib_free(self._fib)
            self._fib = None

    def _fib_now(self):
        if not self._fib:
            keys, _ = self.state()
            self._fib_keys = keys
            self._fib = lib().orc_fib_build(self._m, keys.size, _up(keys))
        return self._fib

    # --- operator ----------------------------------------------------------
    def apply_def(self, keys, x):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        x = _cplx(x)
        y = np.zeros_like(x)
        lib().orc_apply_def(self._m, keys.size, _up(keys), _dp(x.view(np.float64)), _dp(y.view(np.float64)))
        return y

    def apply_def_at(self, keys, x, idx):
        """(P H P x) at the positions idx only (plain definition)."""
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        x = _cplx(x)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        y = np.zeros(idx.size, dtype=np.complex128)
        if lib().orc_apply_def_at(self._m, keys.size, _up(keys), _dp(x.view(np.float64)), idx.size,
                                  idx.ctypes.data_as(_c_int64_p), _dp(y.view(np.float64))) != 0:
            raise ValueError("sampled application needs a model without product terms")
        return y

    def apply_fib(self, keys, x):
        L = lib()
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        x = _cplx(x)
        y = np.zeros_like(x)
        f = L.orc_fib_build(self._m, keys.size, _up(keys))
        L.orc_apply_fib(self._m, f, _dp(x.view(np.float64)), _dp(y.view(np.float64)))
        L.orc_fib_free(f)
        return y

    def fiber_ranges(self, keys, k):
        """Digit ranges J(i) of every dim-k fiber of the set (appendix range storage)."""
        L = lib()
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        f = L.orc_fib_build(self._m, keys.size, _up(keys))
        out = []
        lo = np.zeros(64, dtype=np.int32)
        hi = np.zeros(64, dtype=np.int32)
        for fi in range(L.orc_fib_count(f, k)):
            nr = L.orc_fib_ranges(f, k, fi, 64, _ip(lo), _ip(hi))
            out.append([(int(a), int(b)) for a, b in zip(lo[:nr], hi[:nr])])
        L.orc_fib_free(f)
        return out

    def apply_current(self, x):
        """O-fib on the current state's set with the cached fiber tables."""
        x = _cplx(x)
        y = np.zeros_like(x)
        lib().orc_apply_fib(self._m, self._fib_now(), _dp(x.view(np.float64)), _dp(y.view(np.float64)))
        return y

    # --- propagation -------------------------------------------------------
    def sil_step(self, dt=None, m=None):
        dt = self.card["dt"] if dt is None else dt
        m = self.card["krylov"] if m is None else m
        a0 = ctypes.c_double(0.0)
        used = lib().orc_sil_step(self._m, self._fib_now(), self._s, dt, m, self.arnoldi, ctypes.byref(a0))
        return used, a0.value

    def prune(self, eps=None, rel_excl=0.0):
        eps = self.card["eps"] if eps is None else eps
        nab = lib().orc_prune(self._m, self._s, eps, rel_excl)
        self._drop_fib()
        return int(nab)

    def observe(self, eps=None):
        eps = self.card["eps"] if eps is None else eps
        out = np.zeros(6)
        lib().orc_observe(self._m, self._fib_now(), self._s, _dp(self._bra_tabs.view(np.float64)), eps, _dp(out))
        return dict(zip(OBS_FIELDS[1:7], out))

    def acf_doubled(self):
        """C(2t) = <psi(t)*|psi(t)> (no conjugate), the autocorrelation at
        twice the time for a real initial packet and a real symmetric operator
        (the identity after Eq. acorr): sum_I c_I^2 on a DVR basis; on a
        lattice basis a^T B^T B a with B the map from the lattice coefficients
        to the DVR ones, c = (x)_k G_k^{-+} a, evaluated on the full grid."""
        keys, c = self.state()
        if not self.model.pvb:
            return complex(np.sum(c * c))
        full = np.zeros(int(np.prod(self.n)), dtype=np.complex128)
        full[keys.astype(np.int64)] = c
        full = full.reshape(self.n)
        for k in range(self.D):
            full = np.moveaxis(np.tensordot(self.model.GinvH[k], full, axes=([1], [k])), 0, k)
        return complex(np.sum(full * full))

    def expect_q(self):
        """Position expectation per dimension of the current state,
        <q_k> = sum_I |c_I|^2 q_k(i_k) / sum_I |c_I|^2.

        The DVR position operator is diagonal in the grid index, with the grid
        point as its eigenvalue (Sec. II.A), so this is the definition written
        out.  On a phase-space lattice dimension position is not diagonal in
        the cell index: NaN.  An empty state gives NaN everywhere.
        """
        keys, c = self.state()
        out = np.full(self.D, np.nan)
        if keys.size == 0:
            return out
        w = np.abs(c) ** 2
        norm2 = np.sum(w)
        digits = np.unravel_index(keys.astype(np.int64), self.n)
        for k in range(self.D):
            if not self.model.pvb:
                out[k] = np.sum(w * self.model.q[k][digits[k]]) / norm2
        return out

    def propagate(self, nsteps=None, dt=None, m=None, eps=None, prune=True):
        """Returns (trace[nsteps+1, 9], hashes[nsteps+1]); eps<0 or prune=False: no adaption."""
        nsteps = self.card["nsteps"] if nsteps is None else nsteps
        dt = self.card["dt"] if dt is None else dt
        m = self.card["krylov"] if m is None else m
        eps = self.card["eps"] if eps is None else eps
        if not prune:
            eps = -1.0
        trace = np.zeros((nsteps + 1, len(OBS_FIELDS)))
        hashes = np.zeros(nsteps + 1, dtype=np.uint64)
        self._drop_fib()
        if lib().orc_propagate(self._m, self._s, nsteps, dt, m, eps, self.arnoldi,
                               _dp(self._bra_tabs.view(np.float64)), _dp(trace), _up(hashes)) != 0:
            raise RuntimeError("a step did not meet the Krylov tolerance within max_substeps substeps")
        return trace, hashes

    # --- frozen-set trajectories (adjoint reference) ----------------------------
    def propagate_record(self, nsteps, dt=None, m=None, eps=None):
        """Pruned run from the current state; returns (set_sizes, concatenated keys)."""
        dt = self.card["dt"] if dt is None else dt
        m = self.card["krylov"] if m is None else m
        eps = self.card["eps"] if eps is None else eps
        sizes = np.zeros(nsteps + 1, dtype=np.int64)
        buf = _c_u64_p()
        if lib().orc_propagate_record(self._m, self._s, nsteps, dt, m, eps, sizes.ctypes.data_as(_c_int64_p),
                                      ctypes.byref(buf)) != 0:
            raise RuntimeError("a step did not meet the Krylov tolerance within max_substeps substeps")
        total = int(sizes.sum())
        keys = np.ctypeslib.as_array(buf, shape=(total,)).copy() if total else np.zeros(0, np.uint64)
        lib().orc_free_buffer(ctypes.cast(buf, ctypes.c_void_p))
        self._drop_fib()
        return sizes, keys

    def propagate_frozen(self, sizes, keys, dt=None, m=None):
        dt = self.card["dt"] if dt is None else dt
        m = self.card["krylov"] if m is None else m
        sizes = np.ascontiguousarray(sizes, dtype=np.int64)
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        if lib().orc_propagate_frozen(self._m, self._s, sizes.size - 1, dt, m, sizes.ctypes.data_as(_c_int64_p),
                                      _up(keys)) != 0:
            raise RuntimeError("a step did not meet the Krylov tolerance within max_substeps substeps")
        self._drop_fib()

    # --- helpers for tests ---------------------------------------------------
    def full_keys(self):
        return np.arange(int(np.prod(self.n)), dtype=np.uint64)

    def psi0_on(self, keys):
        """Initial coefficients (product of the 1D tables) at the given keys."""
        keys = np.asarray(keys, dtype=np.uint64).astype(np.int64)
        digits = np.unravel_index(keys, self.n)
        v = np.ones(keys.size, dtype=np.complex128)
        tabs = self.model.init_tables()
        for k in range(self.D):
            v = v * tabs[k][digits[k]]
        return v
