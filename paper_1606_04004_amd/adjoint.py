"""Adjoint gradient of the survival probability behind torch.autograd.

SurvivalProbability.apply(theta, prop) returns J = |<psi0|psi(T)>|^2 for the
parameter vector theta = [trainable potential parameters..., centre[D],
momentum[D]] of a Propagator built from a card with a "trainable" list; the
backward pass is the library's adjoint recursion over the recorded
(frozen) active-set trajectory.  Argument marshalling only.
"""
import numpy as np
import torch


def declare_trainable(prop, card):
    """Declares dV/dtheta for every trainable parameter of the card (symbolic
    derivative of the card's term: coefficient -> the term's factors; Morse
    steepness a -> coefficient times the a-derivative factor)."""
    for i, t in enumerate(card["trainable"]):
        term = card["terms"][t["term"]]
        if t["what"] == "coef":
            prop.add_derivative(i, 1.0, term["factors"])
        elif t["what"] == "a":
            facs = []
            for j, f in enumerate(term["factors"]):
                if j == t["factor"]:
                    assert f["kind"] == "morse"
                    facs.append({"dim": f["dim"], "kind": "morse_da", "a": f["a"], "q0": f["q0"]})
                else:
                    facs.append(f)
            prop.add_derivative(i, term["coef"], facs)
        else:
            raise ValueError(f"unsupported trainable {t['what']!r}")


def apply_parameters(prop, card, values):
    """Writes potential parameter values into the library's terms."""
    for t, v in zip(card["trainable"], values):
        term = card["terms"][t["term"]]
        coef = term["coef"]
        params = []
        for j, f in enumerate(term["factors"]):
            if f["kind"] == "power":
                params += [float(f["p"]), 0.0]
            else:
                params += [float(f["a"]), float(f["q0"])]
        if t["what"] == "coef":
            coef = v
        else:
            params[2 * t["factor"]] = v
        prop.set_term(t["term"], coef, params)


class SurvivalProbability(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, prop):
        card = prop.card
        npar = len(card["trainable"])
        D = card["D"]
        th = theta.detach().cpu().double().numpy()
        apply_parameters(prop, card, th[:npar])
        centre, momentum = th[npar:npar + D], th[npar + D:npar + 2 * D]
        J = prop.adjoint_record(centre=centre, momentum=momentum)
        ctx.prop = prop
        ctx.shape = theta.shape
        return theta.new_tensor(J)

    @staticmethod
    def backward(ctx, gJ):
        dpar, dcen, dmom = ctx.prop.adjoint_gradient()
        g = np.concatenate([dpar, dcen, dmom])
        return gJ * torch.as_tensor(g, dtype=gJ.dtype, device=gJ.device).reshape(ctx.shape), None
