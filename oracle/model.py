"""Oracle-side model construction in FP64 numpy (test infrastructure only).

Everything here is the oracle's own reading of the paper's definitions; the
HIP library builds the same quantities with separate C++ code.

* Sine-DVR (particle-in-a-box DVR; the DVR family of Sec. II.A): box walls
  lo, hi and n interior points q_i = lo + i*dx, dx = (hi-lo)/(n+1), i = 1..n,
  DVR weight dx (Eq. pvN_def's omega_j).  The kinetic matrix is written in
  the closed form of the sine DVR (Colbert & Miller's box result), not via
  its spectral decomposition; its eigenvalues (k pi/L)^2/(2m) are a pin.
* Diagonal potential factors: q^p and Morse (1-exp(-a(q-q0)))^2 sampled on
  the grid (DVR potential is diagonal, Sec. II.A).
* Initial packet: product Gaussian exp(-(q-c)^2/(2 w^2) + i p (q-c)) sampled
  on the grid and normalised per dimension in the discrete 2-norm.
* Projected von Neumann basis (Sec. II.B, Eqs. pvN_def, psi_exp_pvb):
  lattice Gaussians g_{sl}(x) = (2a/pi)^{1/4} exp(-a(x-x_s)^2 + i p_l (x-x_s)),
  a = dp/(2dx), dx*dp = 2 pi, projected G_{j,(s,l)} = sqrt(w_j) g_{sl}(q_j).
  Coefficients a = G^dagger c; the operator acting on them is the similarity
  transform G^dagger h G^{-dagger} of every 1D DVR factor (the full-basis
  form of S^{-1} H, Sec. II.B.2 last paragraph).
"""
import numpy as np


def sine_dvr_grid(n, lo, hi):
    dx = (hi - lo) / (n + 1)
    return lo + dx * np.arange(1, n + 1), dx


def fgh_grid(n, lo, hi):
    """Periodic Fourier grid: x_j = lo + j L / n, j = 0..n-1, L = hi - lo."""
    dx = (hi - lo) / n
    return lo + dx * np.arange(n), dx


def fgh_kinetic(n, lo, hi, mass):
    """-1/(2 mass) d^2/dx^2 on the periodic Fourier grid of odd n, in closed
    form: T_ii = (pi/L)^2 (n^2 - 1) / (6 mass),
    T_ij = (pi/L)^2 (-1)^(i-j) cos(pi (i-j)/n) / (mass sin^2(pi (i-j)/n))."""
    L = hi - lo
    d = np.arange(n)[:, None] - np.arange(n)[None, :]
    T = np.empty((n, n))
    off = d != 0
    dd = d[off]
    T[off] = (np.pi / L) ** 2 * (-1.0) ** dd * np.cos(np.pi * dd / n) / (mass * np.sin(np.pi * dd / n) ** 2)
    np.fill_diagonal(T, (np.pi / L) ** 2 * (n * n - 1) / (6.0 * mass))
    return T


def sine_dvr_kinetic(n, lo, hi, mass):
    """Closed-form sine-DVR kinetic matrix (hbar = 1)."""
    L = hi - lo
    K = n + 1
    pref = np.pi ** 2 / (4.0 * mass * L ** 2)
    T = np.empty((n, n))
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            if i == j:
                T[i - 1, j - 1] = pref * ((2.0 * K * K + 1.0) / 3.0 - 1.0 / np.sin(np.pi * i / K) ** 2)
            else:
                T[i - 1, j - 1] = pref * (-1.0) ** (i - j) * (
                    1.0 / np.sin(np.pi * (i - j) / (2.0 * K)) ** 2
                    - 1.0 / np.sin(np.pi * (i + j) / (2.0 * K)) ** 2)
    return T


def lattice_shapes(card):
    """Per dimension (n_s, n_l): the card's "lattice" is one pair for every
    dimension or a list of pairs, one per dimension."""
    lat = card["lattice"]
    if isinstance(lat[0], (list, tuple)):
        return [tuple(int(v) for v in p) for p in lat]
    return [(int(lat[0]), int(lat[1]))] * card["D"]


def is_dense(f):
    return f["kind"] == "dense"


def dense_matrix(f):
    """A dense factor's matrix in the dimension's DVR basis: "re" plus i "im"."""
    h = np.array(f["re"], dtype=np.float64)
    if "im" in f:
        h = h + 1j * np.array(f["im"], dtype=np.float64)
    return np.asarray(h, dtype=np.complex128)


def term_coef(t):
    return complex(t["coef"], t.get("coef_im", 0.0))


def factor_values(f, q):
    if f["kind"] == "power":
        return q ** f["p"]
    if f["kind"] == "morse":
        return (1.0 - np.exp(-f["a"] * (q - f["q0"]))) ** 2
    raise ValueError(f"unknown factor kind {f['kind']!r}")


def gaussian_1d(q, c, p, w):
    g = np.exp(-((q - c) ** 2) / (2.0 * w * w)) * np.exp(1j * p * (q - c))
    return g / np.sqrt(np.sum(np.abs(g) ** 2))


def pvb_projection(q, dx_grid, lo, hi, ns, nl):
    """G[j, s*nl+l] = sqrt(dx_grid) * g_{sl}(q_j)."""
    dX = (hi - lo) / ns
    dP = 2.0 * np.pi / dX
    alpha = dP / (2.0 * dX)
    xs = lo + (np.arange(ns) + 0.5) * dX
    pl = (np.arange(nl) - 0.5 * (nl - 1)) * dP
    G = np.empty((q.size, ns * nl), dtype=np.complex128)
    for s in range(ns):
        for l in range(nl):
            G[:, s * nl + l] = np.sqrt(dx_grid) * (2.0 * alpha / np.pi) ** 0.25 * np.exp(
                -alpha * (q - xs[s]) ** 2 + 1j * pl[l] * (q - xs[s]))
    return G


def pw_projection(q, dx_grid, lo, hi, nx, npm):
    """Projected Weylets (Sec. II.D): W = Phi S^{-1/2}, Phi[j, s*npm+l] =
    sqrt(dx_grid) phi_sl(q_j) with the momentum-symmetrized Gaussians of
    Eq. sG_def on a doubly dense lattice (dX dP = pi, p_l = (l + 1/2) dP > 0),
    S = Phi^T Phi (Loewdin)."""
    dX = (hi - lo) / nx
    dP = np.pi / dX
    alpha = dP / (2.0 * dX)
    xs = lo + (np.arange(nx) + 0.5) * dX
    pl = (np.arange(npm) + 0.5) * dP
    shift = np.sqrt(np.pi / (8.0 * alpha))
    Phi = np.empty((q.size, nx * npm))
    for s in range(nx):
        for l in range(npm):
            d = q - xs[s]
            Phi[:, s * npm + l] = (np.sqrt(dx_grid) * (8.0 * alpha / np.pi) ** 0.25 * np.exp(-alpha * d * d)
                                   * np.sin(pl[l] * (d - shift)))
    w, V = np.linalg.eigh(Phi.T @ Phi)
    return (Phi @ (V * w ** -0.5) @ V.T).astype(np.complex128)


class Model:
    """All 1D ingredients of a card, in the oracle's own FP64 construction."""

    def __init__(self, card):
        self.card = card
        D = card["D"]
        self.D = D
        self.n = [int(v) for v in card["n"]]
        self.q, self.dx, self.T = [], [], []
        fgh = set(int(k) for k in card.get("fgh", []))
        for k in range(D):
            grid, kin = (fgh_grid, fgh_kinetic) if k in fgh else (sine_dvr_grid, sine_dvr_kinetic)
            qk, dxk = grid(self.n[k], card["lo"][k], card["hi"][k])
            self.q.append(qk)
            self.dx.append(dxk)
            self.T.append(kin(self.n[k], card["lo"][k], card["hi"][k], card["mass"]))
        # a card may replace the 1D operator of a dimension by its own matrix
        for k, h in card.get("dim_factors", {}).items():
            self.T[int(k)] = np.array(h, dtype=np.float64).reshape(self.n[int(k)], self.n[int(k)])
        ps = card["psi0"]
        self.g0 = [gaussian_1d(self.q[k], ps["centre"][k], ps["momentum"][k], ps["width"][k])
                   for k in range(D)]
        # phase-space lattice bases: projected von Neumann ("pvb", biorthogonal)
        # or projected Weylets ("pw", orthogonal); both act as a = G^+ c
        self.pvb = card.get("basis", "dvr") in ("pvb", "pw")
        if self.pvb:
            self.lattices = lattice_shapes(card)
            self.lattice = self.lattices[0]
            proj = pw_projection if card["basis"] == "pw" else pvb_projection
            self.G = [proj(self.q[k], self.dx[k], card["lo"][k], card["hi"][k], *self.lattices[k])
                      for k in range(D)]
            self.Ginv = [np.linalg.inv(G) for G in self.G]
            self.GinvH = [np.linalg.inv(G.conj().T) for G in self.G]

    # --- operator pieces -------------------------------------------------
    def transform(self, k, h):
        """Matrix acting on dim-k coefficients: h itself (DVR) or G^+ h G^-+ (lattice)."""
        if not self.pvb:
            return np.asarray(h, dtype=np.complex128)
        return self.G[k].conj().T @ h @ self.GinvH[k]

    def factor_matrix(self, f):
        """A factor as a matrix in its dimension's DVR basis (diagonal kinds on the diagonal)."""
        if is_dense(f):
            return dense_matrix(f)
        return np.diag(factor_values(f, self.q[f["dim"]])).astype(np.complex128)

    def is_product_term(self, t):
        """True for a term applied as a product of matrices: any dense factor
        or a complex coefficient (DVR), any term on two or more dimensions
        (lattice, where every factor is dense)."""
        if self.pvb:
            return len(set(f["dim"] for f in t["factors"])) > 1
        return any(is_dense(f) for f in t["factors"]) or t.get("coef_im", 0.0) != 0.0

    def single_dim_ops(self):
        """Per dim: kinetic plus, in a lattice basis, every term on that one
        dimension (the product of its factors' matrices, dense there) and, on
        dimension 0, every constant term times the identity."""
        ops = [self.transform(k, self.T[k]) for k in range(self.D)]
        if self.pvb:
            for t in self.card["terms"]:
                dims = set(f["dim"] for f in t["factors"])
                if not dims:
                    ops[0] = ops[0] + term_coef(t) * np.eye(self.n[0])
                elif len(dims) == 1:
                    k = dims.pop()
                    m = np.eye(self.n[k])
                    for f in t["factors"]:
                        m = m @ self.factor_matrix(f)
                    ops[k] = ops[k] + term_coef(t) * self.transform(k, m)
        return ops

    def diag_terms(self):
        """Diagonal potential terms (DVR): list of (coef, {dim: values})."""
        out = []
        if self.pvb:
            return out
        for t in self.card["terms"]:
            if self.is_product_term(t):
                continue
            tabs = {}
            coef = t["coef"]
            for f in t["factors"]:
                k = f["dim"]
                v = factor_values(f, self.q[k])
                tabs[k] = tabs[k] * v if k in tabs else v
            out.append((coef, tabs))
        return out

    def product_terms(self):
        """Terms applied as products of matrices (Sec. II.B.2), as
        (coef, dims increasing, matrices acting on the coefficients): the
        factors on distinct dimensions, each the factor's matrix (lattice:
        transformed like the kinetic matrix)."""
        out = []
        for t in self.card["terms"]:
            if not self.is_product_term(t):
                continue
            fs = sorted(t["factors"], key=lambda f: f["dim"])
            dims = [f["dim"] for f in fs]
            if len(set(dims)) != len(dims):
                raise ValueError("a product term takes one factor per dimension")
            mats = [self.transform(f["dim"], self.factor_matrix(f)) for f in fs]
            out.append((term_coef(t), dims, mats))
        return out

    def hermitian(self):
        """True when the pruned operator is Hermitian, so the propagator may be
        Lanczos: a DVR basis whose product terms each have one dense factor,
        Hermitian, and a real coefficient (diagonal factors commute with the
        truncation).  Two or more dense factors truncated in sequence, a
        complex coefficient or a lattice basis make it non-Hermitian."""
        if self.pvb:
            return False
        for t in self.card["terms"]:
            if not self.is_product_term(t):
                continue
            dense = [f for f in t["factors"] if is_dense(f)]
            if t.get("coef_im", 0.0) != 0.0 or len(dense) != 1:
                return False
            h = dense_matrix(dense[0])
            if not np.array_equal(h, h.conj().T):
                return False
        return True

    def potential_full(self):
        """V on the full grid (DVR cards; tiny grids only)."""
        V = np.zeros(self.n)
        for coef, tabs in self.diag_terms():
            term = np.full(self.n, coef)
            for k, v in tabs.items():
                shape = [1] * self.D
                shape[k] = self.n[k]
                term = term * v.reshape(shape)
            V = V + term
        return V

    # --- packet tables -----------------------------------------------------
    def init_tables(self):
        """1D factors of the initial coefficients (DVR values or lattice a = G^+ c)."""
        if not self.pvb:
            return [g.copy() for g in self.g0]
        return [self.G[k].conj().T @ self.g0[k] for k in range(self.D)]

    def bra_tables(self):
        """1D factors of the bra that gives C(t) = <psi0|psi(t)> from the coefficients."""
        if not self.pvb:
            return [g.copy() for g in self.g0]
        return [self.Ginv[k] @ self.g0[k] for k in range(self.D)]
