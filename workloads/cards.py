"""Model cards: symbolic, seeded descriptions of the synthetic workloads.

A card is a plain dict:

  name, D, n[D], lo[D], hi[D]     sine-DVR grid per dimension (box walls lo, hi;
                                  n interior points)
  mass                            kinetic mass (hbar = 1); a kinetic term is
                                  present on every dimension
  terms                           diagonal potential as a sum of products:
                                  [{"coef": c, "factors": [f, ...]}, ...] with
                                  f = {"dim": k, "kind": "power", "p": p}     (q_k**p)
                                   or {"dim": k, "kind": "morse", "a": a, "q0": q0}
                                                                  ((1-exp(-a(q_k-q0)))**2)
                                   or {"dim": k, "kind": "dense", "re": [[..]], "im": [[..]]}
                                      (an n_k x n_k matrix in the DVR basis, "im" optional);
                                  "coef_im" (optional) makes the coefficient complex
  fgh (optional)                  dimensions on a periodic Fourier grid (odd n_k) instead
                                  of the sine-DVR
  dim_factors (optional)          {k: n_k x n_k real symmetric matrix} replacing the
                                  sine-DVR kinetic matrix of dimension k
  psi0                            product Gaussian: centre, momentum, width per dim
  eps, dt, nsteps, krylov         threshold, time step, steps, Krylov order
  basis                           "dvr", "pvb" or "pw" (phase-space lattice per dim, see
                                  "lattice": [n_s, n_l] with n_s*n_l == n, or one such
                                  pair per dimension)
  krylov_tol, max_substeps        (optional) integrator accuracy: adaptive order and
                                  step control
  params (adjoint card only)      names of the trainable coefficients

Random model coefficients are drawn here once with numpy's PCG64 generator
from a fixed seed and written out in full double precision; neither side
re-draws them.  Nothing in this module evaluates a model quantity.
"""
import copy

import numpy as np

CARD_NAMES = ("hh2d", "morse4d", "quartic6d", "pvb4d", "adjoint4d", "dwell2d")

_SEED_MORSE = 1606
_SEED_QUARTIC = 4004


def _power(k, p):
    return {"dim": k, "kind": "power", "p": int(p)}


def _morse(k, a, q0):
    return {"dim": k, "kind": "morse", "a": float(a), "q0": float(q0)}


def _hh2d():
    # 2D Henon-Heiles-type model on a 48x48 sine-DVR, x, y in [-8, 8].
    c = 0.111
    terms = [
        {"coef": 0.5, "factors": [_power(0, 2)]},
        {"coef": 0.5, "factors": [_power(1, 2)]},
        {"coef": c, "factors": [_power(0, 2), _power(1, 1)]},
        {"coef": -c / 3.0, "factors": [_power(1, 3)]},
    ]
    return {
        "name": "hh2d", "D": 2, "n": [48, 48], "lo": [-8.0, -8.0], "hi": [8.0, 8.0],
        "mass": 1.0, "terms": terms, "basis": "dvr",
        "psi0": {"centre": [2.0, 1.0], "momentum": [0.0, 0.5], "width": [1.0, 1.0]},
        "eps": 1e-5, "dt": 0.05, "nsteps": 200, "krylov": 10,
    }


def morse_lambdas():
    """The six coupling constants lambda_kl (k<l, row-major) of the 4D Morse model."""
    rng = np.random.default_rng(_SEED_MORSE)
    return [float(v) for v in rng.uniform(-0.01, 0.01, size=6)]


def _pairs(D):
    return [(k, l) for k in range(D) for l in range(k + 1, D)]


def _morse4d(n=32):
    lam = morse_lambdas()
    terms = [{"coef": 0.2, "factors": [_morse(k, 1.0, 0.0)]} for k in range(4)]
    for (k, l), v in zip(_pairs(4), lam):
        terms.append({"coef": v, "factors": [_power(k, 1), _power(l, 1)]})
    return {
        "name": "morse4d", "D": 4, "n": [n] * 4, "lo": [-3.0] * 4, "hi": [9.0] * 4,
        "mass": 1.0, "terms": terms, "basis": "dvr", "lambda": lam,
        "psi0": {"centre": [0.5, 0.0, 0.0, 0.0], "momentum": [0.0] * 4, "width": [0.5] * 4},
        "eps": 1e-6, "dt": 0.1, "nsteps": 1000, "krylov": 10,
    }


def quartic_params():
    rng = np.random.default_rng(_SEED_QUARTIC)
    omega = [float(v) for v in rng.uniform(0.8, 1.2, size=6)]
    c = [float(v) for v in rng.normal(0.0, 0.005, size=15)]
    d = [float(v) for v in rng.normal(0.0, 0.002, size=20)]
    return omega, c, d


def _quartic6d(n=24):
    omega, c, d = quartic_params()
    terms = [{"coef": 0.5 * w * w, "factors": [_power(k, 2)]} for k, w in enumerate(omega)]
    for (k, l), v in zip(_pairs(6), c):
        terms.append({"coef": v, "factors": [_power(k, 2), _power(l, 2)]})
    triples = [(k, l, m) for k in range(6) for l in range(k + 1, 6) for m in range(l + 1, 6)]
    for (k, l, m), v in zip(triples, d):
        terms.append({"coef": v, "factors": [_power(k, 1), _power(l, 1), _power(m, 1)]})
    width = [float(w) ** -0.5 for w in omega]
    return {
        "name": "quartic6d", "D": 6, "n": [n] * 6, "lo": [-6.5] * 6, "hi": [6.5] * 6,
        "mass": 1.0, "terms": terms, "basis": "dvr", "omega": omega,
        "psi0": {"centre": [1.5, 0.0, 0.0, 0.0, 0.0, 0.0], "momentum": [0.0] * 6, "width": width},
        "eps": 1e-6, "dt": 0.05, "nsteps": 500, "krylov": 10,
    }


def _pvb4d():
    base = _morse4d(n=48)
    base.update({"name": "pvb4d", "basis": "pvb", "lattice": [6, 8], "nsteps": 1000, "dt": 0.1})
    return base


def _adjoint4d():
    """4D Morse model with 20 trainable coefficients plus the packet centre and momentum.

    The coupling is written over ordered pairs k != l with lambda_kl = lambda_lk =
    lambda^{(k<l)} / 2, so the operator equals the 4D Morse model's.
    """
    lam = morse_lambdas()
    half = {}
    for (k, l), v in zip(_pairs(4), lam):
        half[(k, l)] = 0.5 * v
        half[(l, k)] = 0.5 * v
    terms, params = [], []
    for k in range(4):
        terms.append({"coef": 0.2, "factors": [_morse(k, 1.0, 0.0)]})
    ordered = [(k, l) for k in range(4) for l in range(4) if k != l]
    for (k, l) in ordered:
        terms.append({"coef": half[(k, l)], "factors": [_power(k, 1), _power(l, 1)]})
    params = ([f"D{k}" for k in range(4)] + [f"a{k}" for k in range(4)]
              + [f"lam{k}{l}" for (k, l) in ordered]
              + [f"centre{k}" for k in range(4)] + [f"momentum{k}" for k in range(4)])
    # where each potential parameter sits in the term list
    trainable = ([{"name": f"D{k}", "term": k, "what": "coef"} for k in range(4)]
                 + [{"name": f"a{k}", "term": k, "what": "a", "factor": 0} for k in range(4)]
                 + [{"name": f"lam{k}{l}", "term": 4 + i, "what": "coef"} for i, (k, l) in enumerate(ordered)])
    return {
        "name": "adjoint4d", "D": 4, "n": [32] * 4, "lo": [-3.0] * 4, "hi": [9.0] * 4,
        "mass": 1.0, "terms": terms, "basis": "dvr", "params": params, "trainable": trainable,
        "psi0": {"centre": [0.5, 0.0, 0.0, 0.0], "momentum": [0.0] * 4, "width": [0.5] * 4},
        "eps": 1e-6, "dt": 0.05, "nsteps": 2000, "krylov": 16, "checkpoint_every": 50,
    }


def _dense(k, rng, n, scale, kind):
    """A seeded dense factor on dimension k: "sym" real symmetric, "real"
    real, "complex" complex (re and im parts drawn independently)."""
    a = scale * rng.standard_normal((n, n))
    f = {"dim": k, "kind": "dense"}
    if kind == "sym":
        a = 0.5 * (a + a.T)
    f["re"] = a.tolist()
    if kind == "complex":
        f["im"] = (scale * rng.standard_normal((n, n))).tolist()
    return f


def _sop3d():
    """small_3d's model plus general sum-of-products terms: a real symmetric
    dense factor times a diagonal one, a complex two-factor product with a
    complex coefficient, a three-factor real product and a diagonal term
    with a complex coefficient (drawn once, seed 77)."""
    c = card("small_3d")
    rng = np.random.default_rng(77)
    n = c["n"]
    c["terms"] = c["terms"] + [
        {"coef": 0.3, "factors": [_dense(0, rng, n[0], 0.05, "sym"), _power(2, 1)]},
        {"coef": 0.05, "coef_im": 0.02, "factors": [_dense(1, rng, n[1], 0.1, "complex"),
                                                    _dense(2, rng, n[2], 0.1, "real")]},
        {"coef": 0.02, "factors": [_dense(0, rng, n[0], 0.1, "real"), _dense(1, rng, n[1], 0.1, "real"),
                                   _dense(2, rng, n[2], 0.1, "real")]},
        {"coef": 0.01, "coef_im": -0.003, "factors": [_power(0, 2)]},
    ]
    c["name"] = "sop3d"
    return c


def _dwell2d(literal=False):
    """The paper's two-dimensional double well (Sec. III.A, Eqs. ex_dwell and
    ex_dwell_psiInitial): mass 200, V = 6.4 (x-1)^2 (x-2)^2 + 37.5 (y-2)^2 +
    10 x^2 (y-2), written out in powers of x and y (sum-of-products terms plus
    a constant), the real Gaussian exp(-(x-2.1)^2/0.04 - (y-2.05)^2/0.02)
    (widths sqrt(0.02) and 0.1 in exp(-(q-c)^2/(2 w^2))), Fourier grids of
    165 x 81 points on x in [-0.5, 3.7], y in [1.0, 2.9] (the phase-space
    lattices take 15 x 11 and 9 x 9 on them), propagated to t_e = 24.6.

    The coupling is read as 10 x^2 (y-2): the printed 10 x^2 y adds 20 x^2 at
    the y minimum, which leaves a single well near x = 0.5 with the packet
    about 80 energy units up its wall, where it gains momenta beyond the
    grid's |p| <= pi/dx.  ``literal=True`` gives the printed form."""
    terms = [
        {"coef": 6.4, "factors": [_power(0, 4)]},
        {"coef": -38.4, "factors": [_power(0, 3)]},
        {"coef": 83.2 if literal else 63.2, "factors": [_power(0, 2)]},
        {"coef": -76.8, "factors": [_power(0, 1)]},
        {"coef": 37.5, "factors": [_power(1, 2)]},
        {"coef": -150.0, "factors": [_power(1, 1)]},
        {"coef": 10.0, "factors": [_power(0, 2), _power(1, 1)]},
        {"coef": 175.6, "factors": []},
    ]
    return {
        "name": "dwell2d_literal" if literal else "dwell2d", "D": 2, "n": [165, 81], "lo": [-0.5, 1.0],
        "hi": [3.7, 2.9], "fgh": [0, 1],
        "mass": 200.0, "terms": terms, "basis": "dvr", "lattice": [[15, 11], [9, 9]],
        "psi0": {"centre": [2.1, 2.05], "momentum": [0.0, 0.0], "width": [0.02 ** 0.5, 0.1]},
        "eps": 1e-5, "dt": 0.1, "nsteps": 246, "krylov": 16, "krylov_tol": 1e-10, "max_substeps": 64,
    }


_BUILDERS = {
    "hh2d": _hh2d, "morse4d": _morse4d, "quartic6d": _quartic6d,
    "pvb4d": _pvb4d, "adjoint4d": _adjoint4d, "dwell2d": _dwell2d,
    "dwell2d_literal": lambda: _dwell2d(literal=True),
}


def card(name, **overrides):
    """Return a fresh copy of the named card, with top-level keys overridden.

    Besides the five workload cards, ``small_<D>d`` names give reduced grids of
    the same model families for tests:
      small_2d  -> hh2d on 16x14 points
      small_3d  -> a 3D coupled anharmonic model on 9x11x10 points
      small_4d  -> the 4D Morse model on 10 points per dimension
      small_6d  -> the 6D quartic model on 7 points per dimension
      small_adjoint4d -> the adjoint card on 10 points per dimension, 20 steps
      sop3d     -> small_3d with general sum-of-products terms (dense factors,
                   complex coefficients, a three-factor product)
      dwell2d_literal -> the double well with the coupling as printed (10 x^2 y)
    """
    if name in _BUILDERS:
        c = _BUILDERS[name]()
    elif name == "small_2d":
        c = _hh2d()
        c.update({"name": "small_2d", "n": [16, 14], "lo": [-6.0, -5.0], "hi": [6.0, 5.5]})
    elif name == "small_3d":
        terms = [
            {"coef": 0.5, "factors": [_power(0, 2)]},
            {"coef": 0.7, "factors": [_power(1, 2)]},
            {"coef": 0.45, "factors": [_power(2, 2)]},
            {"coef": 0.05, "factors": [_power(0, 1), _power(1, 1)]},
            {"coef": -0.02, "factors": [_power(1, 2), _power(2, 1)]},
            {"coef": 0.01, "factors": [_power(0, 4)]},
        ]
        c = {
            "name": "small_3d", "D": 3, "n": [9, 11, 10], "lo": [-5.0, -4.5, -5.5],
            "hi": [5.0, 4.0, 5.0], "mass": 1.3, "terms": terms, "basis": "dvr",
            "psi0": {"centre": [0.8, -0.3, 0.2], "momentum": [0.3, 0.0, -0.4],
                     "width": [1.0, 0.9, 1.1]},
            "eps": 1e-4, "dt": 0.05, "nsteps": 40, "krylov": 10,
        }
    elif name == "small_4d":
        c = _morse4d(n=10)
        c.update({"name": "small_4d", "eps": 1e-4, "nsteps": 30})
    elif name == "small_adjoint4d":
        c = _adjoint4d()
        c.update({"name": "small_adjoint4d", "n": [10] * 4, "eps": 1e-4, "nsteps": 20, "checkpoint_every": 5})
    elif name == "sop3d":
        c = _sop3d()
    elif name == "small_6d":
        c = _quartic6d(n=7)
        c.update({"name": "small_6d", "eps": 1e-4, "nsteps": 10})
    else:
        raise KeyError(f"unknown card {name!r}")
    c = copy.deepcopy(c)
    c.update(copy.deepcopy(overrides))
    return c
