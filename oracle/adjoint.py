"""Finite-difference reference of the adjoint gradient (test infrastructure only).

J(theta) = |<psi0(theta)|psi_N(theta)>|^2 with the active-set trajectory
frozen at the sets of the pruned run at the reference parameters; psi_N is
the oracle's forward map (SIL steps, restriction to the next recorded set).
The recording runs with the adjoint's settings (the card's Krylov order as
the largest, its tolerance or 1e-12, step control), so its sets are those of
the library's recording; the finite differences differentiate the exact
step map exp(-i H dt) on those sets, evaluated with Krylov order up to 30 at
tolerance 1e-15 under step control.  Central differences with
h_p = rel * max(1, |theta_p|).
"""
import copy

import numpy as np

from .oracle import Oracle


def param_value(card, name):
    for t in card.get("trainable", []):
        if t["name"] == name:
            term = card["terms"][t["term"]]
            return term["coef"] if t["what"] == "coef" else term["factors"][t["factor"]][t["what"]]
    if name.startswith("centre"):
        return card["psi0"]["centre"][int(name[6:])]
    if name.startswith("momentum"):
        return card["psi0"]["momentum"][int(name[8:])]
    raise KeyError(name)


def card_with(card, name, value):
    c = copy.deepcopy(card)
    for t in c.get("trainable", []):
        if t["name"] == name:
            term = c["terms"][t["term"]]
            if t["what"] == "coef":
                term["coef"] = value
            else:
                term["factors"][t["factor"]][t["what"]] = value
            return c
    if name.startswith("centre"):
        c["psi0"]["centre"][int(name[6:])] = value
    elif name.startswith("momentum"):
        c["psi0"]["momentum"][int(name[8:])] = value
    else:
        raise KeyError(name)
    return c


ADJ_TOL = 1e-12


def recording_card(card):
    """The card with the adjoint recording's integrator settings."""
    c = copy.deepcopy(card)
    c["krylov_tol"] = card.get("krylov_tol", 0.0) or ADJ_TOL
    c["max_substeps"] = 1024
    return c


def exact_card(card):
    """The card with the step map evaluated to the exact exponential."""
    c = copy.deepcopy(card)
    c.update({"krylov": 30, "krylov_tol": 1e-15, "max_substeps": 1024})
    return c


def record_sets(card, nsteps=None):
    o = Oracle(recording_card(card))
    o.init_state()
    nsteps = card["nsteps"] if nsteps is None else nsteps
    return o.propagate_record(nsteps)


def survival_frozen(card, sizes, keys, exact=False):
    """J on the frozen sets: the recording's map, or (exact) exp(-i H dt) per step."""
    o = Oracle(exact_card(card) if exact else recording_card(card))
    k0 = keys[: sizes[0]]
    o.set_state(k0, o.psi0_on(k0))
    o.propagate_frozen(sizes, keys)
    kN, cN = o.state()
    C = np.sum(np.conj(o.psi0_on(kN)) * cN)
    return float(abs(C) ** 2)


def fd_gradient(card, names, sizes, keys, rel=1e-5):
    g = {}
    for nm in names:
        v = param_value(card, nm)
        h = rel * max(1.0, abs(v))
        jp = survival_frozen(card_with(card, nm, v + h), sizes, keys, exact=True)
        jm = survival_frozen(card_with(card, nm, v - h), sizes, keys, exact=True)
        g[nm] = (jp - jm) / (2 * h)
    return g
