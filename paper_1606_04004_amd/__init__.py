"""Dynamically pruned wavepacket propagation on AMD MI355X (gfx950).

Thin Python front end of libppq.so (include/ppq.h).  It only marshals
arguments: every step of the propagation runs in the library's HIP kernels.
PyTorch is used for device memory and streams when the caller passes tensors.
"""
import ctypes

import numpy as np

from . import _ppq
from ._ppq import OBS_FIELDS, OBS_N, PHASES, PPQ_FP32, PPQ_FP64, PPQError  # noqa: F401

__all__ = ["Propagator", "PPQError", "PPQ_FP64", "PPQ_FP32", "OBS_FIELDS"]

_KIND = {"power": _ppq.PPQ_FAC_POWER, "morse": _ppq.PPQ_FAC_MORSE, "table": _ppq.PPQ_FAC_TABLE,
         "morse_da": _ppq.PPQ_FAC_MORSE_DA, "dense": _ppq.PPQ_FAC_DENSE_REAL}


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Propagator:
    """One library context holding a model card's operator and a state.

    precision: PPQ_FP64 or PPQ_FP32; device: HIP device index; stream: a
    torch.cuda.Stream (or raw hipStream_t int) to run on, None for the
    library's own stream.
    """

    def __init__(self, card, precision=PPQ_FP64, device=0, stream=None):
        self.lib = _ppq.load()
        self.card = card
        self.precision = precision
        self.D = int(card["D"])
        self.n = [int(v) for v in card["n"]]
        handle = None
        if stream is not None:
            handle = getattr(stream, "cuda_stream", stream)
        ctx = ctypes.c_void_p()
        _ppq.check(None, self.lib.ppq_create(ctypes.byref(ctx), int(device),
                                             ctypes.c_void_p(handle) if handle else None, int(precision)))
        self.ctx = ctx
        n, pn = _i32(self.n)
        lo, plo = _d(card["lo"])
        hi, phi = _d(card["hi"])
        self._call("ppq_set_grid", self.D, pn, plo, phi, float(card["mass"]))
        for k in card.get("fgh", []):
            self._call("ppq_set_fgh", int(k))
        if card.get("basis", "dvr") in ("pvb", "pw"):
            lat = card["lattice"]
            shapes = lat if isinstance(lat[0], (list, tuple)) else [lat] * self.D
            call = "ppq_set_weylets" if card["basis"] == "pw" else "ppq_set_lattice"
            for k in range(self.D):
                self._call(call, k, int(shapes[k][0]), int(shapes[k][1]))
        for k, h in card.get("dim_factors", {}).items():
            self.set_factor(int(k), h)
        if card.get("stencil", 1) != 1:
            self.set_stencil(card["stencil"])
        if card.get("krylov_tol", 0.0):
            self.set_krylov_tolerance(card["krylov_tol"])
        if card.get("max_substeps", 1) != 1:
            self.set_step_control(card["max_substeps"])
        for t in card["terms"]:
            self.add_term(t["coef"], t["factors"], t.get("coef_im", 0.0))

    # ---- plumbing -----------------------------------------------------------
    def _call(self, name, *args):
        return _ppq.check(self.ctx, getattr(self.lib, name)(self.ctx, *args))

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.ppq_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- model --------------------------------------------------------------
    @staticmethod
    def _factors(factors):
        dims, kinds, params, tables = [], [], [], []
        for f in factors:
            dims.append(int(f["dim"]))
            kinds.append(_KIND[f["kind"]])
            if f["kind"] == "power":
                params += [float(f["p"]), 0.0]
            elif f["kind"] in ("morse", "morse_da"):
                params += [float(f["a"]), float(f["q0"])]
            elif f["kind"] == "dense":
                params += [0.0, 0.0]
                re = np.asarray(f["re"], dtype=np.float64)
                if "im" in f:
                    kinds[-1] = _ppq.PPQ_FAC_DENSE_COMPLEX
                    m = re + 1j * np.asarray(f["im"], dtype=np.float64)
                    tables += list(np.ascontiguousarray(m, dtype=np.complex128).view(np.float64).ravel())
                else:
                    kinds[-1] = _ppq.PPQ_FAC_DENSE_REAL
                    tables += list(re.ravel())
            else:
                params += [0.0, 0.0]
                tables += list(f["values"])
        return dims, kinds, params, tables

    def set_stencil(self, stencil):
        """Adaption stencil: 1 (ball radius 1, 2D neighbours), 2 (radius
        sqrt(2), 2D^2 neighbours) or 3 (radius 2, 3^D - 1 neighbours)."""
        self._call("ppq_set_stencil", int(stencil))

    def set_factor(self, k, h):
        """1D operator of dimension k (real symmetric n_k x n_k); None restores
        the sine-DVR kinetic energy."""
        if h is None:
            self._call("ppq_set_factor", int(k), None)
            return
        a, pa = _d(np.asarray(h, dtype=np.float64).reshape(-1))
        self._call("ppq_set_factor", int(k), pa)

    def clear_potential(self):
        """Removes every potential term (add_term adds new ones)."""
        self._call("ppq_clear_potential")

    def add_term(self, coef, factors, coef_im=0.0):
        """A sum-of-products term (ppq_add_term): diagonal factors and dense
        matrices ({"kind": "dense", "re": ..., "im": ...}), complex coefficient."""
        dims, kinds, params, tables = self._factors(factors)
        d, pd = _i32(dims or [0])
        k, pk = _i32(kinds or [0])
        p, pp = _d(params or [0.0])
        tb, ptb = _d(tables or [0.0])
        self._call("ppq_add_term", float(coef), float(coef_im), len(factors), pd, pk, pp, ptb if tables else None)

    def add_potential_term(self, coef, factors):
        """A diagonal potential term (ppq_add_potential_term)."""
        dims, kinds, params, tables = self._factors(factors)
        d, pd = _i32(dims or [0])
        k, pk = _i32(kinds or [0])
        p, pp = _d(params or [0.0])
        tb, ptb = _d(tables or [0.0])
        self._call("ppq_add_potential_term", float(coef), len(factors), pd, pk, pp, ptb if tables else None)

    def add_derivative(self, param, coef, factors):
        dims, kinds, params, tables = self._factors(factors)
        d, pd = _i32(dims or [0])
        k, pk = _i32(kinds or [0])
        p, pp = _d(params or [0.0])
        tb, ptb = _d(tables or [0.0])
        self._call("ppq_add_potential_derivative", int(param), float(coef), len(factors), pd, pk, pp,
                   ptb if tables else None)

    def set_term(self, term, coef, params):
        p, pp = _d(params or [0.0])
        self._call("ppq_set_potential_term", int(term), float(coef), pp if params else None)

    # ---- adjoint ----------------------------------------------------------------
    def adjoint_record(self, centre=None, momentum=None, eps=None, nsteps=None, dt=None, m=None, every=None):
        ps = self.card["psi0"]
        c, pc = _d(ps["centre"] if centre is None else centre)
        mo, pm = _d(ps["momentum"] if momentum is None else momentum)
        w, pw = _d(ps["width"])
        J = ctypes.c_double(0.0)
        self._call("ppq_adjoint_record", pc, pm, pw,
                   float(self.card["eps"] if eps is None else eps),
                   int(self.card["nsteps"] if nsteps is None else nsteps),
                   float(self.card["dt"] if dt is None else dt),
                   int(self.card["krylov"] if m is None else m),
                   int(self.card.get("checkpoint_every", 50) if every is None else every), ctypes.byref(J))
        return J.value

    def adjoint_frozen(self, centre, momentum):
        c, pc = _d(centre)
        mo, pm = _d(momentum)
        J = ctypes.c_double(0.0)
        self._call("ppq_adjoint_frozen", pc, pm, ctypes.byref(J))
        return J.value

    def adjoint_gradient(self):
        npar = len(self.card.get("trainable", []))
        dp = np.zeros(max(npar, 1))
        dc = np.zeros(self.D)
        dm = np.zeros(self.D)
        self._call("ppq_adjoint_gradient", dp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   dc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   dm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return dp[:npar], dc, dm

    def grid(self, k):
        q = np.zeros(self.n[k])
        _ppq.check(self.ctx, self.lib.ppq_get_grid(self.ctx, k, q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return q

    def reserve(self, cap):
        self._call("ppq_reserve", int(cap))

    # ---- state --------------------------------------------------------------
    def init_state(self, eps=None):
        ps = self.card["psi0"]
        eps = self.card["eps"] if eps is None else eps
        c, pc = _d(ps["centre"])
        m, pm = _d(ps["momentum"])
        w, pw = _d(ps["width"])
        na = ctypes.c_int64(0)
        self._call("ppq_init_gaussian", pc, pm, pw, float(eps), ctypes.byref(na))
        return na.value

    def set_state(self, keys, coeff):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        c = np.ascontiguousarray(coeff, dtype=np.complex128)
        self._call("ppq_set_state", keys.size, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                   c.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)))

    def set_reference(self, centre=None, momentum=None, width=None):
        """C(t) reference packet; defaults to the card's psi0."""
        ps = self.card["psi0"]
        c, pc = _d(ps["centre"] if centre is None else centre)
        m, pm = _d(ps["momentum"] if momentum is None else momentum)
        w, pw = _d(ps["width"] if width is None else width)
        self._call("ppq_set_reference", pc, pm, pw)

    def set_state_device(self, keys, coeff):
        """State from device tensors: keys (int64/uint64 view, ascending) and
        coefficients (complex128), both on the context's device."""
        if keys.numel() != coeff.numel() or keys.element_size() != 8 or coeff.element_size() != 16:
            raise ValueError("keys: 8-byte integers, coeff: complex128, of one length")
        if not (keys.is_contiguous() and coeff.is_contiguous()):
            raise ValueError("keys and coeff must be contiguous")
        n = int(keys.numel())
        self._call("ppq_set_state_device", n, ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(coeff.data_ptr()))

    def state_device(self, keys, coeff):
        """Writes the state into device tensors (int64 keys, complex128
        coefficients, each at least |A| long, stream-ordered); returns |A|."""
        if keys.element_size() != 8 or coeff.element_size() != 16:
            raise ValueError("keys: 8-byte integers, coeff: complex128")
        if not (keys.is_contiguous() and coeff.is_contiguous()):
            raise ValueError("keys and coeff must be contiguous")
        cnt = ctypes.c_int64(0)
        self._call("ppq_get_state_device", int(min(keys.numel(), coeff.numel())), ctypes.byref(cnt),
                   ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(coeff.data_ptr()))
        return cnt.value

    def active_count(self):
        n = ctypes.c_int64(0)
        self._call("ppq_active_count", ctypes.byref(n))
        return n.value

    def state(self):
        cnt = ctypes.c_int64(0)
        code = self.lib.ppq_get_state(self.ctx, 0, ctypes.byref(cnt), None, None)
        if code not in (0, -1):
            _ppq.check(self.ctx, code)
        n = cnt.value
        keys = np.zeros(n, dtype=np.uint64)
        c = np.zeros(n, dtype=np.complex128)
        self._call("ppq_get_state", n, ctypes.byref(cnt), keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                   c.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return keys, c

    # ---- operator and propagation ---------------------------------------------
    def apply_h(self, x, y):
        """y = P H P x for device tensors/pointers of the context precision (complex interleaved)."""
        px = x.data_ptr() if hasattr(x, "data_ptr") else int(x)
        py = y.data_ptr() if hasattr(y, "data_ptr") else int(y)
        self._call("ppq_apply_h", ctypes.c_void_p(px), ctypes.c_void_p(py))

    def step(self, dt=None, m=None):
        dt = self.card["dt"] if dt is None else dt
        m = self.card["krylov"] if m is None else m
        self._call("ppq_step", float(dt), int(m))

    def prune(self, eps=None):
        eps = self.card["eps"] if eps is None else eps
        na, nb = ctypes.c_int64(0), ctypes.c_int64(0)
        self._call("ppq_prune", float(eps), ctypes.byref(na), ctypes.byref(nb))
        return na.value, nb.value

    def set_relative_exclusion(self, r):
        self._call("ppq_set_relative_exclusion", float(r))

    def set_krylov_tolerance(self, tol):
        """Adaptive SIL order: each step stops at the first order whose error
        estimate is within tol (0: the full order)."""
        self._call("ppq_set_krylov_tolerance", float(tol))

    def set_step_control(self, max_substeps):
        """Step size control under the Krylov tolerance: each step as up to
        max_substeps substeps (1 = off)."""
        self._call("ppq_set_step_control", int(max_substeps))

    def propagate(self, nsteps=None, dt=None, m=None, eps=None, prune=True):
        nsteps = self.card["nsteps"] if nsteps is None else nsteps
        dt = self.card["dt"] if dt is None else dt
        m = self.card["krylov"] if m is None else m
        eps = self.card["eps"] if eps is None else eps
        if not prune:
            eps = -1.0
        trace = np.zeros((nsteps + 1, OBS_N))
        self._call("ppq_propagate", int(nsteps), float(dt), int(m), float(eps),
                   trace.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return trace

    def observables(self, eps=None):
        eps = self.card["eps"] if eps is None else eps
        out = np.zeros(OBS_N)
        self._call("ppq_observables", float(eps), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return dict(zip(OBS_FIELDS[1:7], out[1:7]))

    def acf_doubled(self):
        """C(2t) = sum_I c_I^2 of the current state (real packet, real symmetric operator)."""
        out = np.zeros(2)
        self._call("ppq_acf_doubled", out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return complex(out[0], out[1])

    def expect_q(self):
        """<q_k> per dimension of the current state (NaN on lattice dimensions)."""
        out = np.zeros(self.D)
        self._call("ppq_expect_q", out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out

    def expect_q_noalloc(self):
        """expect_q through the entry point that allocates no device memory."""
        out = np.zeros(self.D)
        self._call("ppq_expect_q_noalloc", out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out

    def time_apply(self, nrep, mean=False):
        """Median ms of one H application over nrep (with mean=True: (median, mean))."""
        med = ctypes.c_double(0.0)
        avg = ctypes.c_double(0.0)
        self._call("ppq_time_apply", int(nrep), ctypes.byref(med), ctypes.byref(avg))
        return (med.value, avg.value) if mean else med.value

    def enable_timings(self, on=True):
        self._call("ppq_enable_timings", 1 if on else 0)

    def timings(self):
        """Milliseconds per phase since timing was turned on (dict by phase name)."""
        ms = np.zeros(len(PHASES))
        self._call("ppq_timings", ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return dict(zip(PHASES, ms.tolist()))

    def fiber_counts(self):
        nf = np.zeros(self.D, dtype=np.int64)
        self._call("ppq_fiber_counts", nf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        return nf
