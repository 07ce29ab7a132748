"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: integer/index work (active sets, fiber counts, carried-over
coefficients) bit-exact; FP64 operator products within 1e-13 relative;
FP64 trajectories within 1e-10 on every observable with identical active
sets at every step.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from workloads import card, random_active_set, random_complex

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "needs a GPU"
    return t


def make(cd, torch, precision=0):
    import paper_1606_04004_amd as ppq
    return ppq.Propagator(cd, precision=precision, device=0, stream=torch.cuda.current_stream())


def lattice_card(n=12, ns=3, nl=4, **kw):
    base = card("small_4d", n=[n, n, n, n], **kw)
    return dict(base, name="small_lattice4d", basis="pvb", lattice=[ns, nl])


# ---------------------------------------------------------------------------
# operator
# ---------------------------------------------------------------------------
APPLY_CASES = [
    ("small_2d", 0.5, True, 1), ("small_3d", 0.35, True, 2), ("small_4d", 0.25, True, 3),
    ("small_6d", 0.08, True, 4), ("small_3d", 1.0, False, 5), ("small_4d", 0.05, False, 6),
    ("hh2d", 0.3, True, 7), ("morse4d", 0.02, True, 8),
]


@pytest.mark.parametrize("name,fill,blob,seed", APPLY_CASES)
def test_apply_h_fp64(name, fill, blob, seed, torch):
    cd = card(name)
    say(f"apply_h fp64 {name} fill={fill} blob={blob} seed={seed}")
    keys = random_active_set(cd["n"], fill, seed, blob=blob)
    x = random_complex(keys.size, seed + 100)
    ref = Oracle(cd).apply_def(keys, x)
    g = make(cd, torch)
    g.set_state(keys, x)
    xt = torch.from_numpy(x).cuda()
    yt = torch.zeros_like(xt)
    g.apply_h(xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy()
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    say(f"  |A|={keys.size} rel err {err:.2e}")
    assert err < 1e-13


def test_apply_h_tiny_sets(torch):
    cd = card("small_3d")
    o = Oracle(cd)
    for keys in (np.array([0], np.uint64), np.array([5, 6, 7], np.uint64),
                 np.array([int(np.prod(cd["n"])) - 1], np.uint64)):
        say(f"apply_h tiny set {keys.tolist()}")
        x = random_complex(keys.size, 3)
        g = make(cd, torch)
        g.set_state(keys, x)
        xt = torch.from_numpy(x).cuda()
        yt = torch.zeros_like(xt)
        g.apply_h(xt, yt)
        torch.cuda.synchronize()
        assert np.allclose(yt.cpu().numpy(), o.apply_def(keys, x), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("name", ["hh2d", "morse4d", "quartic6d"])
def test_apply_h_full_size_sampled(name, torch):
    """Full workload size (the initial active set of each card), outputs sampled."""
    cd = card(name)
    say(f"apply_h sampled {name}")
    o = Oracle(cd)
    o.init_state()
    keys, _ = o.state()
    n = keys.size
    g = make(cd, torch)
    x = random_complex(n, 11)
    g.set_state(keys, x)
    xt = torch.from_numpy(x).cuda()
    yt = torch.zeros_like(xt)
    g.apply_h(xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy()
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([rng.integers(0, n, 1500), [0, n - 1]]))
    ref = o.apply_def_at(keys, x, idx)
    err = np.max(np.abs(y[idx] - ref)) / np.max(np.abs(ref))
    say(f"  |A|={n} sampled={idx.size} rel err {err:.2e}")
    assert err < 1e-13


def test_fiber_counts_match_oracle(torch):
    cd = card("small_4d")
    keys = random_active_set(cd["n"], 0.3, 17)
    g = make(cd, torch)
    g.set_state(keys, np.ones(keys.size, complex))
    nf = g.fiber_counts()
    o = Oracle(cd)
    ref = [len(o.fiber_ranges(keys, k)) for k in range(cd["D"])]
    assert nf.tolist() == ref


# ---------------------------------------------------------------------------
# adaption
# ---------------------------------------------------------------------------
def adversarial_state(n, seed, eps):
    keys = random_active_set(n, 0.4, seed)
    rng = np.random.default_rng(seed)
    c = random_complex(keys.size, seed) * np.exp(rng.uniform(-14, 0, keys.size))
    c[::13] = eps                       # |c|^2 == eps^2 exactly
    c[3::29] = eps * (1 - 2 ** -52)     # just below
    c[7::31] = 0.0
    c[11::37] = 1e-310                  # subnormal
    c[2::41] = 1j * eps                 # tie on the imaginary axis
    return keys, c


@pytest.mark.parametrize("name,seed", [("small_2d", 1), ("small_3d", 2), ("small_4d", 3), ("small_6d", 4)])
def test_prune_bit_exact(name, seed, torch):
    cd = card(name)
    eps = 2.0 ** -10
    keys, c = adversarial_state(cd["n"], seed, eps)
    say(f"prune {name} |A|={keys.size}")
    o = Oracle(cd)
    o.set_state(keys, c)
    nab_o = o.prune(eps=eps)
    ko, co = o.state()
    g = make(cd, torch)
    g.set_state(keys, c)
    na, nab_g = g.prune(eps=eps)
    kg, cg = g.state()
    assert np.array_equal(kg, ko)
    assert np.array_equal(cg.view(np.uint64), co.view(np.uint64))
    assert nab_g == nab_o and na == ko.size


@pytest.mark.parametrize("name,n", [("small_3d", [24, 24, 24]), ("small_3d", [5, 2, 7]), ("small_3d", [2, 9, 70]),
                                    ("small_2d", [130, 3]), ("small_6d", [4, 4, 4, 4, 4, 4])])
@pytest.mark.parametrize("fill", [0.01, 0.3])
def test_dilation_word_and_point_forms_agree(name, n, fill, torch):
    """Adaption's two dilation forms (per function with atomics, and word by
    word from the bitmap of the functions above the threshold, chosen by the
    grid-to-set size ratio) give the oracle's set: grids whose size is not a
    multiple of 64, axes of 2 points, strides below and above a word."""
    import os
    cd = card(name, n=n)
    eps = 2.0 ** -10
    keys = random_active_set(n, fill, 51, blob=False)
    c = random_complex(keys.size, 52) * 2.0 ** -9
    o = Oracle(cd)
    o.set_state(keys, c)
    nab_o = o.prune(eps=eps)
    ko, _ = o.state()
    old = os.environ.get("PPQ_DILATE")
    try:
        for mode in ("1", "2"):
            os.environ["PPQ_DILATE"] = mode
            g = make(cd, torch)
            g.set_state(keys, c)
            na, nab_g = g.prune(eps=eps)
            kg, _ = g.state()
            say(f"  dilation form {mode}, n={n}, fill {fill}: |A| {keys.size} -> {kg.size}")
            assert np.array_equal(kg, ko) and nab_g == nab_o and na == ko.size
    finally:
        if old is None:
            del os.environ["PPQ_DILATE"]
        else:
            os.environ["PPQ_DILATE"] = old


def test_prune_edge_cases(torch):
    cd = card("small_3d")
    total = int(np.prod(cd["n"]))
    g = make(cd, torch)
    say("prune: empty S")
    keys = np.arange(0, total, 7, dtype=np.uint64)
    g.set_state(keys, np.full(keys.size, 1e-9 + 0j))
    assert g.prune(eps=1e-3) == (0, 0)
    assert g.state()[0].size == 0
    say("prune: from empty set")
    assert g.prune(eps=1e-3) == (0, 0)
    say("prune: S = full grid")
    keys = np.arange(total, dtype=np.uint64)
    g.set_state(keys, np.ones(total, complex))
    assert g.prune(eps=0.5) == (total, total)
    say("prune: lattice stencil")
    lc = lattice_card()
    o = Oracle(lc)
    keys = random_active_set(lc["n"], 0.05, 3)
    c = random_complex(keys.size, 3) * 1e-3
    o.set_state(keys, c)
    o.prune(eps=1e-3)
    gl = make(lc, torch)
    gl.set_state(keys, c)
    gl.prune(eps=1e-3)
    assert np.array_equal(gl.state()[0], o.state()[0])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_prune_relative_exclusion_bit_exact(seed, torch):
    """Relative exclusion threshold (Sec. II.E) below, at and above the dropped
    fraction: identical sets and carried coefficients."""
    cd = card("small_4d")
    o = Oracle(cd)
    eps = 1e-3
    keys = random_active_set(o.n, 0.35, seed)
    rng = np.random.default_rng(seed)
    c = random_complex(keys.size, seed) * np.exp(rng.uniform(-12, 0, keys.size))
    c[::17] = eps
    o.set_state(keys, c)
    o.prune(eps=eps)
    dropped = np.setdiff1d(keys, o.state()[0]).size
    n = keys.size
    g = make(cd, torch)
    for r in (0.0, (dropped - 0.5) / n, dropped / n, (dropped + 0.5) / n, 1.0):
        say(f"relative exclusion seed {seed} r={r:.6f} (dropped {dropped} of {n})")
        o.set_state(keys, c)
        nab = o.prune(eps=eps, rel_excl=r)
        g.set_state(keys, c)
        g.set_relative_exclusion(r)
        assert g.prune(eps=eps)[1] == nab
        kg, cg = g.state()
        ko, co = o.state()
        assert np.array_equal(kg, ko)
        assert np.array_equal(cg, co)


def test_relative_exclusion_trajectory(torch):
    """small_3d, 40 steps with r = 0.05 against the oracle's step/adapt loop."""
    cd = card("small_3d")
    r = 0.05
    o = Oracle(cd)
    g = make(cd, torch)
    o.init_state()
    g.init_state()
    g.set_relative_exclusion(r)
    tg = g.propagate(nsteps=40)
    for st in range(1, 41):
        o.sil_step()
        o.prune(rel_excl=r)
        ob = o.observe()
        assert int(ob["n_active"]) == int(tg[st, 5]), st
        for col, nm in ((1, "norm2"), (3, "acf_re"), (4, "acf_im"), (6, "n_above")):
            assert abs(tg[st, col] - ob[nm]) < 1e-10, (st, nm)
    assert np.array_equal(g.state()[0], o.state()[0])
    say(f"  |A| at the end {int(tg[-1, 5])}")


@pytest.mark.parametrize("name", ["hh2d", "small_3d", "morse4d", "quartic6d"])
def test_initial_state(name, torch):
    cd = card(name)
    say(f"init {name}")
    g = make(cd, torch)
    n = g.init_state()
    o = Oracle(cd)
    o.init_state()
    kg, cg = g.state()
    ko, co = o.state()
    say(f"  |A0| gpu={n} oracle={ko.size}")
    assert np.array_equal(kg, ko)
    assert np.max(np.abs(cg - co)) < 1e-15


# ---------------------------------------------------------------------------
# propagation
# ---------------------------------------------------------------------------
def test_single_step(torch):
    cd = card("small_4d")
    o = Oracle(cd)
    o.init_state()
    keys, c = o.state()
    g = make(cd, torch)
    g.set_state(keys, c)
    say("single SIL step small_4d")
    g.step()
    o.sil_step()
    kg, cg = g.state()
    _, co = o.state()
    assert np.max(np.abs(cg - co)) < 1e-13



@pytest.mark.parametrize("m", [1, 2, 3, 16])
def test_single_step_krylov_orders(m, torch):
    """One SIL step at the extreme Krylov orders (Sec. III.A): m = 1 is the
    bare alpha_0 phase, m = 2 the first Lanczos recurrence, 16 the largest
    order the library takes. The Hermitian first Gram-Schmidt pass takes
    beta_{j-1} from the recurrence; the result must still be the oracle's."""
    cd = card("small_4d")
    o = Oracle(cd)
    o.init_state()
    keys, c = o.state()
    g = make(cd, torch)
    g.set_state(keys, c)
    say(f"single SIL step small_4d, m = {m}")
    g.step(m=m)
    o.sil_step(m=m)
    _, cg = g.state()
    _, co = o.state()
    assert np.max(np.abs(cg - co)) < 1e-13


@pytest.mark.parametrize("prec", [0, 1])
def test_krylov_space_exhausted(prec, torch):
    """A set of 5 functions holds at most a 5-dimensional Krylov space: with
    m = 16 the recurrence breaks down (beta below 1e-13) and the space is
    truncated. Whatever the order at which either side stops, the coupling
    left out is of the size of the breakdown threshold, so the steps agree
    to 1e-12 (FP64), and to the FP32 form's 1e-6."""
    cd = card("small_4d")
    o = Oracle(cd)
    o.init_state()
    keys, c = o.state()
    sel = np.argsort(-np.abs(c))[:5]
    sel.sort()
    k5, c5 = keys[sel].copy(), c[sel].copy()
    o.set_state(k5, c5)
    g = make(cd, torch, precision=prec)
    g.set_state(k5, c5)
    say(f"exhausted Krylov space: 5 functions, m = 16, precision {prec}")
    for _ in range(3):
        g.step(m=16)
        o.sil_step(m=16)
    kg, cg = g.state()
    ko, co = o.state()
    assert np.array_equal(kg, ko)
    assert np.all(np.isfinite(cg))
    assert abs(np.vdot(co, co).real - np.vdot(c5, c5).real) < 1e-12  # unitary on the set
    assert np.max(np.abs(cg - co)) < (1e-12 if prec == 0 else 1e-6)

@pytest.mark.parametrize("m", [1, 2, 3, 16])
def test_arnoldi_single_step_krylov_orders(m, torch):
    """One SIL step on a phase-space lattice (non-Hermitian P S^-1 H P, so
    Arnoldi) at the extreme Krylov orders: m = 1 and 2 reach the first
    Hessenberg column without and with a correction of the provisional
    vector, m = 16 the largest order, whose last column keeps its first
    Gram-Schmidt pass only. Coefficients within 1e-12 of the largest."""
    cd = lattice_card(eps=1e-4)
    o = Oracle(cd)
    o.init_state()
    keys, c = o.state()
    g = make(cd, torch)
    g.set_state(keys, c)
    say(f"single Arnoldi step small_lattice4d, m = {m}")
    g.step(dt=0.05, m=m)
    o.sil_step(dt=0.05, m=m)
    _, cg = g.state()
    _, co = o.state()
    assert np.max(np.abs(cg - co)) < 1e-12 * np.max(np.abs(co))


@pytest.mark.parametrize("prec", [0, 1])
def test_arnoldi_space_exhausted(prec, torch):
    """Five lattice functions hold at most a 5-dimensional Krylov space: at
    m = 16 the Arnoldi process breaks down (beta below 1e-13) and the space
    is truncated; the steps agree to 1e-12 (FP64), 1e-6 in the FP32 form,
    relative to the largest coefficient."""
    cd = lattice_card(eps=1e-4)
    o = Oracle(cd)
    o.init_state()
    keys, c = o.state()
    sel = np.argsort(-np.abs(c))[:5]
    sel.sort()
    k5, c5 = keys[sel].copy(), c[sel].copy()
    o.set_state(k5, c5)
    g = make(cd, torch, precision=prec)
    g.set_state(k5, c5)
    say(f"exhausted Arnoldi space: 5 lattice functions, m = 16, precision {prec}")
    for _ in range(3):
        g.step(dt=0.05, m=16)
        o.sil_step(dt=0.05, m=16)
    kg, cg = g.state()
    ko, co = o.state()
    assert np.array_equal(kg, ko)
    assert np.all(np.isfinite(cg))
    assert np.max(np.abs(cg - co)) < (1e-12 if prec == 0 else 1e-6) * np.max(np.abs(co))


def test_hh2d_trajectory_sets_every_step(torch):
    """Config 1 (2D, 48x48, eps=1e-5): identical active set after every step, 200 steps."""
    cd = card("hh2d")
    o = Oracle(cd)
    o.init_state()
    g = make(cd, torch)
    g.init_state()
    worst = 0.0
    for st in range(cd["nsteps"]):
        g.step()
        g.prune()
        o.sil_step()
        o.prune()
        kg, cg = g.state()
        ko, co = o.state()
        assert np.array_equal(kg, ko), f"active sets differ after step {st + 1}"
        worst = max(worst, float(np.max(np.abs(cg - co))))
    say(f"  hh2d 200 steps: max coefficient difference {worst:.2e}")
    assert worst < 1e-10


# The 4D Morse card (dt = 0.1, m = 10) is numerically sensitive: a 1e-15
# relative perturbation of the oracle's own initial state reaches 1.4e-10 in
# C(t) after 30 steps, so the free-running comparison stops at 25 steps and
# test_shadow_steps_morse4d checks the step map itself over a longer run.
@pytest.mark.parametrize("name,nsteps,prune", [("hh2d", 200, True), ("hh2d", 200, False), ("small_3d", 40, True),
                                               ("morse4d", 25, True), ("small_6d", 10, True)])
def test_trajectory_observables(name, nsteps, prune, torch):
    cd = card(name)
    say(f"trajectory {name} {nsteps} steps prune={prune}")
    o = Oracle(cd)
    g = make(cd, torch)
    if prune:
        o.init_state()
        g.init_state()
    else:
        # full grid holding the packet; eps = 0 keeps every function
        keys = np.arange(int(np.prod(cd["n"])), dtype=np.uint64)
        o.set_state(keys, o.psi0_on(keys))
        g.init_state(eps=0.0)
    tr, _ = o.propagate(nsteps=nsteps, prune=prune)
    tg = g.propagate(nsteps=nsteps, prune=prune)
    assert np.array_equal(tg[:, 5], tr[:, 5]), "active-set sizes differ"
    for col, nm in ((1, "norm2"), (2, "energy"), (3, "acf_re"), (4, "acf_im"), (6, "n_above")):
        d = np.max(np.abs(tg[:, col] - tr[:, col]))
        say(f"  {nm}: max diff {d:.2e}")
        assert d < 1e-10, nm


# ---------------------------------------------------------------------------
# position expectations
# ---------------------------------------------------------------------------
def _box_scale(cd):
    return max(max(abs(v) for v in cd["lo"]), max(abs(v) for v in cd["hi"]))


@pytest.mark.parametrize("name,nsteps", [("hh2d", 40), ("small_3d", 20), ("morse4d", 10), ("small_6d", 5)])
def test_expect_q_trajectory(name, nsteps, torch):
    """<q_k> of the GPU state equals the oracle's on the same state (1e-13 of the
    box size) and the oracle's along its own trajectory (1e-10), twice in a row."""
    cd = card(name)
    o = Oracle(cd)
    ref = Oracle(cd)
    g = make(cd, torch)
    o.init_state()
    g.init_state()
    scale = _box_scale(cd)
    for rep in range(2):
        say(f"expect_q {name}: steps {rep * nsteps}..{(rep + 1) * nsteps}")
        o.propagate(nsteps=nsteps)
        g.propagate(nsteps=nsteps)
        qg = g.expect_q()
        kg, _ = g.state()
        # the same state: the oracle's, given to a second context
        ko, co = o.state()
        h = make(cd, torch)
        h.set_state(ko, co)
        d_same = np.max(np.abs(h.expect_q() - o.expect_q()))
        d_traj = np.max(np.abs(qg - o.expect_q()))
        say(f"  |A|={kg.size} same-state diff {d_same:.2e} trajectory diff {d_traj:.2e}")
        assert d_same < 1e-13 * scale
        assert d_traj < 1e-10


@pytest.mark.parametrize("fill,seed", [(1.0, 21), (0.7, 22)])
def test_expect_q_large_sets(fill, seed, torch):
    """32^4 grid, full and with a ragged random fill: several grid-stride passes."""
    cd = card("morse4d")
    keys = random_active_set(cd["n"], fill, seed, blob=False)
    c = random_complex(keys.size, seed + 1)
    say(f"expect_q large set |A|={keys.size}")
    g = make(cd, torch)
    g.set_state(keys, c)
    o = Oracle(cd)
    o.set_state(keys, c)
    d = np.max(np.abs(g.expect_q() - o.expect_q()))
    say(f"  diff {d:.2e}")
    assert d < 1e-13 * _box_scale(cd)


def test_expect_q_edge_cases(torch):
    cd = card("small_3d")
    n = cd["n"]
    o = Oracle(cd)
    g = make(cd, torch)
    for idx in ((0, 0, 0), (3, 7, 2), (n[0] - 1, n[1] - 1, n[2] - 1)):
        say(f"expect_q one point {idx}")
        keys = np.array([np.ravel_multi_index(idx, n)], dtype=np.uint64)
        c = np.array([3.0 - 4.0j])
        g.set_state(keys, c)
        o.set_state(keys, c)
        assert np.allclose(g.expect_q(), o.expect_q(), rtol=1e-15, atol=1e-15)
    say("expect_q empty set")
    g.set_state(np.zeros(0, np.uint64), np.zeros(0, complex))
    assert np.all(np.isnan(g.expect_q()))
    say("expect_q lattice dimensions")
    lc = lattice_card()
    gl = make(lc, torch)
    gl.init_state()
    assert np.all(np.isnan(gl.expect_q()))


def test_phase_timings(torch):
    """Phase events leave the trajectory bit-identical; every phase of a step
    takes time; the phases add up to at most the host's wall time."""
    import time
    cd = card("morse4d")
    a = make(cd, torch)
    b = make(cd, torch)
    a.init_state()
    b.init_state()
    ta = a.propagate(nsteps=10)
    b.enable_timings(True)
    t0 = time.perf_counter()
    tb = b.propagate(nsteps=10)
    wall = (time.perf_counter() - t0) * 1e3
    ph = b.timings()
    say(f"phases (ms): {ph}, wall {wall:.2f} ms")
    assert np.array_equal(ta, tb)
    assert np.array_equal(a.state()[1], b.state()[1])
    assert all(v > 0.0 for v in ph.values())
    assert sum(ph.values()) <= wall
    b.enable_timings(False)
    b.propagate(nsteps=2)
    assert b.timings() == ph
    b.enable_timings(True)
    b.step()
    b.prune()
    ph2 = b.timings()
    assert ph2["hpsi"] > 0 and ph2["krylov"] > 0 and ph2["adapt"] > 0 and ph2["obs"] == 0.0


def test_fp32_form_expect_q_and_relative_exclusion(torch):
    """The FP32 form keeps the FP64 master state: its position expectations
    match the oracle's on the same state, and its adaption (with a relative
    exclusion threshold) is bit-exact."""
    cd = card("small_4d")
    o = Oracle(cd)
    g = make(cd, torch, precision=1)
    o.init_state()
    o.propagate(nsteps=5)
    ko, co = o.state()
    g.set_state(ko, co)
    assert np.max(np.abs(g.expect_q() - o.expect_q())) < 1e-13 * _box_scale(cd)
    eps = 1e-3
    keys = random_active_set(o.n, 0.35, 7)
    c = random_complex(keys.size, 7) * np.exp(np.random.default_rng(7).uniform(-12, 0, keys.size))
    o.set_state(keys, c)
    o.prune(eps=eps)
    dropped = np.setdiff1d(keys, o.state()[0]).size
    for r in (0.0, (dropped + 0.5) / keys.size):
        say(f"fp32 form adaption, relative exclusion {r:.5f}")
        o.set_state(keys, c)
        nab = o.prune(eps=eps, rel_excl=r)
        g.set_state(keys, c)
        g.set_relative_exclusion(r)
        assert g.prune(eps=eps)[1] == nab
        assert np.array_equal(g.state()[0], o.state()[0])
        assert np.array_equal(g.state()[1], o.state()[1])


def test_lattice_reference_and_expect_q(torch):
    """Lattice card: C(t) from a state set on the host, with the reference
    packet given separately, equals the initial-packet run; position
    expectations are NaN on lattice dimensions."""
    cd = lattice_card(eps=1e-4)
    a = make(cd, torch)
    a.init_state()
    keys, c = a.state()
    b = make(cd, torch)
    b.set_state(keys, c)
    b.set_reference()
    ta = a.propagate(nsteps=5, dt=0.05)
    tb = b.propagate(nsteps=5, dt=0.05)
    assert np.array_equal(ta, tb)
    assert np.all(np.isnan(b.expect_q()))


def test_shadow_steps_morse4d(torch):
    """Each step of the GPU map from the oracle's state equals the oracle's step:
    identical adapted set, coefficients within 1e-12 (relative to the largest)."""
    cd = card("morse4d")
    o = Oracle(cd)
    o.init_state()
    g = make(cd, torch)
    worst = 0.0
    for st in range(40):
        keys, c = o.state()
        g.set_state(keys, c)
        g.step()
        g.prune()
        o.sil_step()
        o.prune()
        kg, cg = g.state()
        ko, co = o.state()
        assert np.array_equal(kg, ko), f"sets differ at step {st + 1}"
        worst = max(worst, float(np.max(np.abs(cg - co)) / np.max(np.abs(co))))
    say(f"  morse4d 40 shadowed steps: |A|={ko.size}, worst rel coefficient diff {worst:.2e}")
    assert worst < 1e-12


def test_lattice_full_card(torch):
    """4D lattice card at full size (48^4 functions, 6x8 lattice per dimension,
    dense complex 48x48 factors, Arnoldi): identical sets and observables."""
    cd = card("pvb4d")
    say("pvb4d: 3 steps")
    o = Oracle(cd)
    o.init_state()
    g = make(cd, torch)
    n = g.init_state()
    assert np.array_equal(g.state()[0], o.state()[0])
    tr, _ = o.propagate(nsteps=3)
    tg = g.propagate(nsteps=3)
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 2, 3, 4, 6):
        d = np.max(np.abs(tg[:, col] - tr[:, col]))
        say(f"  col {col}: {d:.2e}")
        assert d < 1e-10
    kg, cg = g.state()
    ko, co = o.state()
    assert np.array_equal(kg, ko)
    assert np.max(np.abs(cg - co)) < 1e-11


def test_lattice_trajectory(torch):
    """Phase-space lattice (biorthogonal projected von Neumann), Arnoldi, lattice stencil."""
    cd = lattice_card(eps=1e-4)
    say("lattice trajectory")
    o = Oracle(cd)
    o.init_state()
    g = make(cd, torch)
    g.init_state()
    assert np.array_equal(g.state()[0], o.state()[0])
    tr, _ = o.propagate(nsteps=10, dt=0.05)
    tg = g.propagate(nsteps=10, dt=0.05)
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 3, 4, 6):
        d = np.max(np.abs(tg[:, col] - tr[:, col]))
        say(f"  col {col}: {d:.2e}")
        assert d < 1e-10


# Stated error of the FP32 form (complex-FP32 operator and Krylov vectors,
# FP64 reductions, exponential and master copy) against the FP64 oracle, on
# the cards whose trajectories are well conditioned.
FP32_BOUNDS = {"norm2": 1e-6, "acf_re": 1e-6, "acf_im": 1e-6, "energy_rel": 1e-6}


@pytest.mark.parametrize("name,nsteps", [("hh2d", 200), ("small_3d", 40), ("small_6d", 10)])
def test_fp32_form_error(name, nsteps, torch):
    import paper_1606_04004_amd as ppq
    cd = card(name)
    say(f"fp32 form {name}")
    o = Oracle(cd)
    o.init_state()
    tr, _ = o.propagate(nsteps=nsteps)
    g = make(cd, torch, precision=ppq.PPQ_FP32)
    g.init_state()
    tg = g.propagate(nsteps=nsteps)
    errs = {nm: float(np.max(np.abs(tg[:, c] - tr[:, c]))) for c, nm in ((1, "norm2"), (3, "acf_re"),
                                                                      (4, "acf_im"))}
    errs["energy_rel"] = float(np.max(np.abs(tg[:, 2] - tr[:, 2]) / np.abs(tr[:, 2])))
    rel_n = float(np.max(np.abs(tg[:, 5] - tr[:, 5]) / tr[:, 5]))
    say(f"  errors {errs} |A| rel {rel_n:.2e}")
    for nm, bound in FP32_BOUNDS.items():
        assert errs[nm] < bound, nm


@pytest.mark.parametrize("name,nsteps", [("morse4d", 15), ("pvb4d", 2), ("hh2d", 10)])
def test_fp32_shadow_steps(name, nsteps, torch):
    """The FP32 form against the FP64 oracle, one step + adaption at a time
    from the oracle's state (shadowed: on the chaotic 4D Morse card a free
    run's own error would grow; the lattice card at its full 48^4 size):
    norm^2, C(t) and the relative energy within 1e-6 at every step; the
    active-set size within 1e-3 relative (the FP32 coefficients can cross
    the threshold where the FP64 ones do not: one function in 10^5 on the
    lattice card); the coefficients within 1e-5 relative to the largest
    where the sets agree."""
    import paper_1606_04004_amd as ppq
    cd = card(name)
    o = Oracle(cd)
    o.init_state()
    g = make(cd, torch, precision=ppq.PPQ_FP32)
    g.set_reference()
    worst = {"norm2": 0.0, "acf": 0.0, "energy_rel": 0.0, "n_active_rel": 0.0, "coef_rel": 0.0}
    for st in range(nsteps):
        keys, c = o.state()
        g.set_state(keys, c)
        t32 = g.propagate(nsteps=1)
        tr, _ = o.propagate(nsteps=1)
        worst["norm2"] = max(worst["norm2"], abs(t32[1, 1] - tr[1, 1]))
        worst["acf"] = max(worst["acf"], abs(complex(t32[1, 3], t32[1, 4]) - complex(tr[1, 3], tr[1, 4])))
        worst["energy_rel"] = max(worst["energy_rel"], abs(t32[0, 2] - tr[0, 2]) / abs(tr[0, 2]))
        worst["n_active_rel"] = max(worst["n_active_rel"], abs(t32[1, 5] - tr[1, 5]) / tr[1, 5])
        kg, cg = g.state()
        kr, cr = o.state()
        if np.array_equal(kg, kr):
            worst["coef_rel"] = max(worst["coef_rel"], float(np.max(np.abs(cg - cr)) / np.max(np.abs(cr))))
    say(f"  {name} FP32 shadowed steps vs oracle: {worst}")
    assert worst["norm2"] < 1e-6 and worst["acf"] < 1e-6 and worst["energy_rel"] < 1e-6
    assert worst["n_active_rel"] < 1e-3 and worst["coef_rel"] < 1e-5


# ---------------------------------------------------------------------------
# fused layouts (selected per context with PPQ_HPSI): the same products and
# trajectories as the per-dimension layout
# ---------------------------------------------------------------------------
# 4, 5: block-fused (row groups per wave task; one lane per fiber);
# 6: plane passes (two dimensions per pass through matrix-core tiles; a card
# with a dimension above 32 points keeps the per-dimension layout);
# 7: the last two dimensions in one pass (one thread per point, whole planes
# per workgroup), the others one lane per fiber
BLOCK_VARIANTS = ["4", "5", "6", "7"]


def make_block(cd, torch, precision=0, variant="4"):
    import os
    old = os.environ.get("PPQ_HPSI")
    os.environ["PPQ_HPSI"] = variant
    try:
        return make(cd, torch, precision)
    finally:
        if old is None:
            del os.environ["PPQ_HPSI"]
        else:
            os.environ["PPQ_HPSI"] = old


@pytest.mark.parametrize("variant", BLOCK_VARIANTS)
@pytest.mark.parametrize("name,fill,blob,seed", APPLY_CASES + [("small_6d", 0.6, True, 9)])
def test_block_layout_apply_h(name, fill, blob, seed, variant, torch):
    cd = card(name)
    say(f"block layout {variant} apply_h {name} fill={fill} seed={seed}")
    keys = random_active_set(cd["n"], fill, seed, blob=blob)
    x = random_complex(keys.size, seed + 100)
    ref = Oracle(cd).apply_def(keys, x)
    for prec in (0, 1):
        g = make_block(cd, torch, prec, variant)
        g.set_state(keys, x)
        xt = torch.from_numpy(x).cuda()
        if prec == 1:
            xt = xt.to(torch.complex64)
        yt = torch.zeros_like(xt)
        g.apply_h(xt, yt)
        torch.cuda.synchronize()
        r = ref if prec == 0 else Oracle(cd).apply_def(keys, x.astype(np.complex64).astype(np.complex128))
        err = np.max(np.abs(yt.cpu().numpy().astype(np.complex128) - r)) / np.max(np.abs(r))
        say(f"  prec {prec} |A|={keys.size} rel err {err:.2e}")
        assert err < (1e-13 if prec == 0 else 1e-6)


@pytest.mark.parametrize("variant", BLOCK_VARIANTS)
def test_block_layout_full_size_sampled(variant, torch):
    """6D quartic initial set (3.5M points): chunks above the main launch's
    capacity go through the second launch."""
    cd = card("quartic6d")
    o = Oracle(cd)
    o.init_state()
    keys, _ = o.state()
    n = keys.size
    g = make_block(cd, torch, 0, variant)
    x = random_complex(n, 12)
    g.set_state(keys, x)
    xt = torch.from_numpy(x).cuda()
    yt = torch.zeros_like(xt)
    g.apply_h(xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy()
    idx = np.unique(np.concatenate([np.random.default_rng(6).integers(0, n, 1500), [0, n - 1]]))
    ref = o.apply_def_at(keys, x, idx)
    err = np.max(np.abs(y[idx] - ref)) / np.max(np.abs(ref))
    say(f"  block layout |A|={n} rel err {err:.2e}")
    assert err < 1e-13


@pytest.mark.parametrize("variant", BLOCK_VARIANTS)
def test_block_layout_oversized_blocks_fall_back(variant, torch):
    """A full 2x2x2x20x20x20 grid has 8000-point inner blocks, more than one
    workgroup's LDS holds: the context uses the per-dimension layout."""
    cd = card("small_6d", n=[2, 2, 2, 20, 20, 20])
    keys = np.arange(int(np.prod(cd["n"])), dtype=np.uint64)
    x = random_complex(keys.size, 13)
    ref = Oracle(cd).apply_def(keys, x)
    g = make_block(cd, torch, 0, variant)
    g.set_state(keys, x)
    xt = torch.from_numpy(x).cuda()
    yt = torch.zeros_like(xt)
    g.apply_h(xt, yt)
    torch.cuda.synchronize()
    err = np.max(np.abs(yt.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err < 1e-13


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("fill", [1.0, 0.3])
def test_plane_pass_largest_planes(fill, prec, torch):
    """Plane passes at the largest planes a task holds: a 6 x 27 x 28 grid,
    full (756-point planes of the pair (1, 2), one per task, in 32 x 32
    tiles; dimension 0 keeps its own pass) and a random subset."""
    cd = card("small_3d", n=[6, 27, 28])
    n = cd["n"]
    keys = np.arange(int(np.prod(n)), dtype=np.uint64) if fill == 1.0 else random_active_set(n, fill, 31)
    x = random_complex(keys.size, 32)
    xin = x if prec == 0 else x.astype(np.complex64).astype(np.complex128)
    ref = Oracle(cd).apply_def(keys, xin)
    g = make_block(cd, torch, prec, "6")
    g.set_state(keys, x)
    xt = torch.from_numpy(x).cuda()
    if prec == 1:
        xt = xt.to(torch.complex64)
    yt = torch.zeros_like(xt)
    g.apply_h(xt, yt)
    torch.cuda.synchronize()
    err = np.max(np.abs(yt.cpu().numpy().astype(np.complex128) - ref)) / np.max(np.abs(ref))
    say(f"  plane passes 6x27x28 fill {fill} prec {prec}: rel err {err:.2e}")
    assert err < (1e-13 if prec == 0 else 1e-6)


@pytest.mark.parametrize("prec", [0, 1])
def test_staged_permutation_same_results(prec, torch):
    """The lane-per-fiber passes read the permutation either from scattered
    global loads or from a wavefront's copy of its rank range in LDS
    (PPQ_ACC_STAGE=1): the same arithmetic, so the products, and 5 steps
    (whose Krylov iterations also take the fused <x|y> pass), are bitwise
    identical; the product also matches the oracle."""
    import os
    cd = card("small_6d")
    keys = random_active_set(cd["n"], 0.5, 61)
    x = random_complex(keys.size, 62)
    xin = x if prec == 0 else x.astype(np.complex64).astype(np.complex128)
    ref = Oracle(cd).apply_def(keys, xin)
    old = os.environ.get("PPQ_ACC_STAGE")
    out, traj = {}, {}
    try:
        for st in ("0", "1"):
            os.environ["PPQ_ACC_STAGE"] = st
            g = make(cd, torch, precision=prec)
            g.set_state(keys, x)
            xt = torch.from_numpy(x).cuda()
            if prec == 1:
                xt = xt.to(torch.complex64)
            yt = torch.zeros_like(xt)
            g.apply_h(xt, yt)
            torch.cuda.synchronize()
            out[st] = yt.cpu().numpy().astype(np.complex128)
            g.init_state()
            traj[st] = g.propagate(nsteps=5)
    finally:
        if old is None:
            del os.environ["PPQ_ACC_STAGE"]
        else:
            os.environ["PPQ_ACC_STAGE"] = old
    assert np.array_equal(out["0"], out["1"])
    assert np.array_equal(traj["0"], traj["1"])
    err = np.max(np.abs(out["1"] - ref)) / np.max(np.abs(ref))
    say(f"  staged permutation, prec {prec}: identical; rel err vs oracle {err:.2e}")
    assert err < (1e-13 if prec == 0 else 1e-6)


@pytest.mark.parametrize("prec", [0, 1])
def test_pair_pass_largest_plane(prec, torch):
    """Layout 7 with a task at its largest span: on a 5 x 32 x 32 grid one
    plane is full (1024 points, the most a plane may hold) and the others
    hold 5% of their points, so the mean fibers stay short and the pass is
    taken; the full plane shares its task with the planes around it."""
    cd = card("small_3d", n=[5, 32, 32])
    n = cd["n"]
    sparse = random_active_set(n, 0.05, 41, blob=False)
    keys = np.union1d(sparse, np.arange(2 * 1024, 3 * 1024, dtype=np.uint64)).astype(np.uint64)
    x = random_complex(keys.size, 42)
    xin = x if prec == 0 else x.astype(np.complex64).astype(np.complex128)
    ref = Oracle(cd).apply_def(keys, xin)
    g = make_block(cd, torch, prec, "7")
    g.set_state(keys, x)
    nf = g.fiber_counts()
    assert keys.size <= 16 * min(nf[1], nf[2]), "fibers too long for the pair pass"
    xt = torch.from_numpy(x).cuda()
    if prec == 1:
        xt = xt.to(torch.complex64)
    yt = torch.zeros_like(xt)
    g.apply_h(xt, yt)
    torch.cuda.synchronize()
    err = np.max(np.abs(yt.cpu().numpy().astype(np.complex128) - ref)) / np.max(np.abs(ref))
    say(f"  pair pass 5x32x32, |A| {keys.size}, prec {prec}: rel err {err:.2e}")
    assert err < (1e-13 if prec == 0 else 1e-6)


@pytest.mark.parametrize("variant", BLOCK_VARIANTS)
@pytest.mark.parametrize("name,nsteps", [("small_6d", 10), ("small_4d", 30), ("morse4d", 25)])
def test_block_layout_trajectory(name, nsteps, variant, torch):
    cd = card(name)
    say(f"block layout {variant} trajectory {name} {nsteps} steps")
    o = Oracle(cd)
    o.init_state()
    g = make_block(cd, torch, 0, variant)
    g.init_state()
    tr, _ = o.propagate(nsteps=nsteps)
    tg = g.propagate(nsteps=nsteps)
    assert np.array_equal(tg[:, 5], tr[:, 5]), "active-set sizes differ"
    for col in (1, 2, 3, 4, 6):
        assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10


@pytest.mark.parametrize("n,prec", [([24, 20, 18], 0), ([24, 20, 18], 1), ([17, 33, 40], 0)])
def test_apply_h_long_fibers(n, prec, torch):
    """Full grids: every fiber is longer than 16 points, so FP64 takes the
    matrix-core passes (windows of 1-3 tiles), as the FP32 form always does."""
    cd = card("small_3d", n=n)
    keys = np.arange(int(np.prod(n)), dtype=np.uint64)
    x = random_complex(keys.size, 21)
    ref = Oracle(cd).apply_def(keys, x)
    g = make(cd, torch, precision=prec)
    g.set_state(keys, x)
    xt = torch.from_numpy(x).cuda()
    if prec == 1:
        xt = xt.to(torch.complex64)
    yt = torch.zeros_like(xt)
    g.apply_h(xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy().astype(np.complex128)
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    say(f"  long fibers n={n} prec={prec} rel err {err:.2e}")
    assert err < (1e-13 if prec == 0 else 1e-6)


def test_quartic6d_full_size_shadowed(torch):
    """The 6D quartic card at full size (24^6 grid, the oracle's 3.52M-point
    initial state, the size of the timed step-250 snapshot): two step +
    adaption cycles, each started from the oracle's state, give the oracle's
    sets bit for bit and its coefficients within 1e-12; the FP32 form, from
    the same states, stays within 1e-6 of the oracle on norm^2, C(t), |A|
    and (relative) energy."""
    cd = card("quartic6d")
    o = Oracle(cd)
    o.init_state()
    g = make(cd, torch)
    g.reserve(16_000_000)
    g32 = make(cd, torch, precision=1)
    g32.reserve(16_000_000)
    for h in (g, g32):
        h.set_reference()  # C(t) against the card's packet, as the oracle's
    worst32 = {"norm2": 0.0, "acf": 0.0, "energy_rel": 0.0, "n_active_rel": 0.0}
    for cyc in range(2):
        ko, co = o.state()
        say(f"6D shadowed cycle {cyc}: |A| = {ko.size}")
        g.set_state(ko, co)
        g32.set_state(ko, co)
        tr, _ = o.propagate(nsteps=1)
        tg = g.propagate(nsteps=1)
        t32 = g32.propagate(nsteps=1)
        kr, cr = o.state()
        kg, cg = g.state()
        assert np.array_equal(kg, kr), f"sets differ in cycle {cyc}"
        err = np.max(np.abs(cg - cr))
        say(f"  |A'| = {kr.size}, max coefficient difference {err:.2e}")
        assert err < 1e-12
        for col in (1, 2, 3, 4, 6):
            assert abs(tg[1, col] - tr[1, col]) < 1e-10
        worst32["norm2"] = max(worst32["norm2"], abs(t32[1, 1] - tr[1, 1]))
        worst32["acf"] = max(worst32["acf"], abs(complex(t32[1, 3], t32[1, 4]) - complex(tr[1, 3], tr[1, 4])))
        worst32["energy_rel"] = max(worst32["energy_rel"], abs(t32[0, 2] - tr[0, 2]) / abs(tr[0, 2]))
        worst32["n_active_rel"] = max(worst32["n_active_rel"], abs(t32[1, 5] - tr[1, 5]) / tr[1, 5])
    say(f"  FP32 form vs oracle: {worst32}")
    assert worst32["norm2"] < 1e-6 and worst32["acf"] < 1e-6 and worst32["energy_rel"] < 1e-6
    assert worst32["n_active_rel"] < 1e-6


# ---------------------------------------------------------------------------
# extreme shapes: one dimension, eight dimensions (the most the context takes),
# two-point and 64-point (largest) bases, a grid near the 2^32 key limit
# ---------------------------------------------------------------------------
def shape_card(n, lo=-4.0, hi=4.0):
    D = len(n)
    terms = [{"coef": 0.5, "factors": [{"dim": k, "kind": "power", "p": 2}]} for k in range(D)]
    terms += [{"coef": 0.05, "factors": [{"dim": k, "kind": "power", "p": 1}, {"dim": k + 1, "kind": "power", "p": 1}]}
              for k in range(D - 1)]
    return {"name": f"shape_{'x'.join(map(str, n))}", "D": D, "n": list(n), "lo": [lo] * D, "hi": [hi] * D,
            "mass": 1.0, "terms": terms, "basis": "dvr",
            "psi0": {"centre": [0.5] * D, "momentum": [0.3] * D, "width": [0.8] * D},
            "eps": 1e-4, "dt": 0.05, "nsteps": 10, "krylov": 8}


SHAPES = [[64], [2] * 6, [4] * 8, [3, 5, 4, 6, 3, 5, 4, 2], [64, 64, 64], [2, 64, 3]]


@pytest.mark.parametrize("n", SHAPES, ids=lambda n: "x".join(map(str, n)))
@pytest.mark.parametrize("prec", [0, 1])
def test_extreme_shapes_apply_h(n, prec, torch):
    cd = shape_card(n)
    o = Oracle(cd)
    for fill, seed in ((1.0, 1), (0.45, 2)):
        keys = (np.arange(int(np.prod(n)), dtype=np.uint64) if fill == 1.0
                else random_active_set(n, fill, seed, blob=False))
        say(f"extreme shape {n} prec {prec} |A|={keys.size}")
        x = random_complex(keys.size, seed + 10)
        ref = o.apply_def(keys, x)
        g = make(cd, torch, precision=prec)
        g.set_state(keys, x)
        if prec == 0:
            xt = torch.from_numpy(x).cuda()
        else:
            xt = torch.from_numpy(x.astype(np.complex64)).cuda()
        yt = torch.zeros_like(xt)
        g.apply_h(xt, yt)
        torch.cuda.synchronize()
        y = yt.cpu().numpy().astype(np.complex128)
        if prec == 1:
            ref = o.apply_def(keys, x.astype(np.complex64).astype(np.complex128))
        err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
        say(f"  rel err {err:.2e}")
        assert err < (1e-13 if prec == 0 else 2e-6)


@pytest.mark.parametrize("n", SHAPES, ids=lambda n: "x".join(map(str, n)))
def test_extreme_shapes_trajectory(n, torch):
    cd = shape_card(n)
    say(f"extreme shape trajectory {n}")
    o = Oracle(cd)
    g = make(cd, torch)
    o.init_state()
    g.init_state()
    assert np.array_equal(g.state()[0], o.state()[0])
    tr, _ = o.propagate(nsteps=10)
    tg = g.propagate(nsteps=10)
    assert np.array_equal(tg[:, 5], tr[:, 5]), "active-set sizes differ"
    for col in (1, 2, 3, 4, 6):
        assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10
    assert np.array_equal(g.state()[0], o.state()[0])
    assert np.max(np.abs(g.expect_q() - o.expect_q())) < 1e-10


def test_grid_near_key_limit(torch):
    """64^5 x 3 = 3.2e9 grid points (keys above 2^31): a blob of ~10^5 functions
    inside; product, adaption and three steps against the oracle."""
    n = [64, 64, 64, 64, 64, 3]
    assert 2 ** 31 < int(np.prod(n)) < 2 ** 32
    cd = shape_card(n, lo=-8.0, hi=8.0)
    rng = np.random.default_rng(5)
    sub = np.stack(np.meshgrid(*[np.arange(40, 48)] * 5, np.arange(3), indexing="ij"), -1).reshape(-1, 6)
    sub = sub[rng.random(sub.shape[0]) > 0.2]
    keys = np.sort(np.ravel_multi_index(tuple(sub.T), n)).astype(np.uint64)
    assert keys[-1] > 2 ** 31
    x = random_complex(keys.size, 6) / np.sqrt(keys.size)
    say(f"grid near key limit |A|={keys.size}")
    o = Oracle(cd)
    ref = o.apply_def(keys, x)
    g = make(cd, torch)
    g.set_state(keys, x)
    g.set_reference()
    xt = torch.from_numpy(x).cuda()
    yt = torch.zeros_like(xt)
    g.apply_h(xt, yt)
    torch.cuda.synchronize()
    err = np.max(np.abs(yt.cpu().numpy() - ref)) / np.max(np.abs(ref))
    say(f"  product rel err {err:.2e}")
    assert err < 1e-13
    o.set_state(keys, x)
    eps = 2e-3
    assert g.prune(eps=eps)[1] == o.prune(eps=eps)
    assert np.array_equal(g.state()[0], o.state()[0])
    say(f"  after adaption |A|={g.state()[0].size}")
    tr, _ = o.propagate(nsteps=3, eps=eps)
    tg = g.propagate(nsteps=3, eps=eps)
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 2, 3, 4, 6):
        assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10
    assert np.array_equal(g.state()[0], o.state()[0])


# ---------------------------------------------------------------------------
# argument and state errors: each is refused with its code and leaves the
# context's state as it was (host-side validation, no kernel sees the input)
# ---------------------------------------------------------------------------
def test_errors_leave_state_unchanged(torch):
    from paper_1606_04004_amd import PPQError
    from paper_1606_04004_amd._ppq import STATUS
    code_of = {v: k for k, v in STATUS.items()}
    E_ARG, E_STATE, E_NUMERIC = code_of["PPQ_E_ARG"], code_of["PPQ_E_STATE"], code_of["PPQ_E_NUMERIC"]
    cd = card("small_3d")
    g = make(cd, torch)
    say("errors: no state yet")
    for fn in (g.expect_q, g.step, lambda: g.prune(eps=1e-3), lambda: g.observables()):
        with pytest.raises(PPQError) as e:
            fn()
        assert e.value.code == E_STATE
    g.init_state()
    k0, c0 = g.state()
    total = int(np.prod(cd["n"]))
    bad = [
        ("unsorted keys", lambda: g.set_state(k0[::-1].copy(), c0[::-1].copy()), E_ARG),
        ("key beyond the grid", lambda: g.set_state(np.array([0, total], np.uint64), np.ones(2, complex)),
         E_ARG),
        ("non-finite coefficient", lambda: g.set_state(k0, np.where(np.arange(k0.size) == 3, np.nan, c0)),
         E_NUMERIC),
        ("Krylov order 0", lambda: g.step(m=0), E_ARG),
        ("Krylov order 17", lambda: g.step(m=17), E_ARG),
        ("non-finite dt", lambda: g.step(dt=float("inf")), E_ARG),
        ("negative threshold", lambda: g.prune(eps=-1.0), E_ARG),
        ("negative relative exclusion", lambda: g.set_relative_exclusion(-0.1), E_ARG),
        ("NaN relative exclusion", lambda: g.set_relative_exclusion(float("nan")), E_ARG),
        ("zero reference width", lambda: g.set_reference(width=[0.0, 1.0, 1.0]), E_ARG),
        ("capacity beyond the grid", lambda: g.reserve(total + 1), E_ARG),
    ]
    for what, fn, code in bad:
        say(f"errors: {what}")
        with pytest.raises(PPQError) as e:
            fn()
        assert e.value.code == code, what
        k1, c1 = g.state()
        assert np.array_equal(k1, k0) and np.array_equal(c1, c0), what
    # the context still works, and matches a fresh one
    o = Oracle(cd)
    o.init_state()
    tr, _ = o.propagate(nsteps=5)
    tg = g.propagate(nsteps=5)
    assert np.array_equal(tg[:, 5], tr[:, 5])
    assert np.max(np.abs(tg[:, 1] - tr[:, 1])) < 1e-10


def test_clear_potential(torch):
    """Clearing the potential and adding the same terms again reproduces the
    run bit for bit; with no terms left the run matches the oracle's
    kinetic-only model."""
    cd = card("small_3d")
    a = make(cd, torch)
    a.init_state()
    ta = a.propagate(nsteps=5)
    b = make(cd, torch)
    b.clear_potential()
    for t in cd["terms"]:
        b.add_term(t["coef"], t["factors"])
    b.init_state()
    tb = b.propagate(nsteps=5)
    assert np.array_equal(ta, tb)
    free = dict(cd, terms=[])
    o = Oracle(free)
    o.init_state()
    g = make(cd, torch)
    g.clear_potential()
    g.init_state()
    tr, _ = o.propagate(nsteps=5)
    tg = g.propagate(nsteps=5)
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 2, 3, 4, 6):
        assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10


def test_device_state_transfer(torch):
    """State to and from device tensors: identical to the host path; bad keys,
    non-finite values and host pointers are refused with the state unchanged."""
    from paper_1606_04004_amd import PPQError
    from paper_1606_04004_amd._ppq import STATUS
    code_of = {v: k for k, v in STATUS.items()}
    cd = card("small_3d")
    total = int(np.prod(cd["n"]))
    g = make(cd, torch)
    g.init_state()
    k_host, c_host = g.state()
    n = k_host.size
    kt = torch.zeros(n + 5, dtype=torch.int64, device="cuda")
    ct = torch.zeros(n + 5, dtype=torch.complex128, device="cuda")
    assert g.state_device(kt, ct) == n
    torch.cuda.synchronize()
    assert np.array_equal(kt[:n].cpu().numpy().astype(np.uint64), k_host)
    assert np.array_equal(ct[:n].cpu().numpy(), c_host)
    h = make(cd, torch)
    h.set_state_device(kt[:n], ct[:n])
    kh, ch = h.state()
    assert np.array_equal(kh, k_host) and np.array_equal(ch, c_host)
    bad_keys = kt[:n].flip(0).contiguous()
    beyond = kt[:n].clone()
    beyond[-1] = total
    nan_c = ct[:n].clone()
    nan_c[3] = complex(float("nan"), 0.0)
    for what, args, code in (("descending keys", (bad_keys, ct[:n]), "PPQ_E_ARG"),
                             ("key beyond the grid", (beyond, ct[:n]), "PPQ_E_ARG"),
                             ("non-finite coefficient", (kt[:n], nan_c), "PPQ_E_NUMERIC"),
                             ("host tensors", (kt[:n].cpu(), ct[:n].cpu()), "PPQ_E_ARG")):
        say(f"device state: {what}")
        with pytest.raises(PPQError) as e:
            h.set_state_device(*args)
        assert e.value.code == code_of[code], what
        kh, ch = h.state()
        assert np.array_equal(kh, k_host) and np.array_equal(ch, c_host), what
    ta = g.propagate(nsteps=5)
    h.set_reference()
    tb = h.propagate(nsteps=5)
    assert np.array_equal(ta, tb)


def _custom_factor_card(seed):
    from oracle.model import sine_dvr_kinetic
    cd = card("small_3d")
    rng = np.random.default_rng(seed)
    fac = {}
    for k in (0, 2):
        n = cd["n"][k]
        m = sine_dvr_kinetic(n, cd["lo"][k], cd["hi"][k], cd["mass"]) + 0.3 * rng.standard_normal((n, n)) / n
        fac[k] = ((m + m.T) / 2.0).tolist()
    cd["dim_factors"] = fac
    return cd


@pytest.mark.parametrize("prec", [0, 1])
def test_custom_dim_factors(prec, torch):
    """The caller's own 1D matrices on two dimensions: products against the
    oracle (FP64 1e-13, FP32 2e-6), a 10-step trajectory (FP64), restoring
    the sine-DVR matrix, and refusal of a non-symmetric matrix."""
    from paper_1606_04004_amd import PPQError
    cd = _custom_factor_card(3)
    o = Oracle(cd)
    g = make(cd, torch, precision=prec)
    for fill, seed in ((1.0, 1), (0.4, 2)):
        keys = (np.arange(int(np.prod(cd["n"])), dtype=np.uint64) if fill == 1.0
                else random_active_set(cd["n"], fill, seed))
        x = random_complex(keys.size, seed + 20)
        say(f"custom factors prec {prec} |A|={keys.size}")
        g.set_state(keys, x)
        if prec == 0:
            xt = torch.from_numpy(x).cuda()
            ref = o.apply_def(keys, x)
        else:
            xt = torch.from_numpy(x.astype(np.complex64)).cuda()
            ref = o.apply_def(keys, x.astype(np.complex64).astype(np.complex128))
        yt = torch.zeros_like(xt)
        g.apply_h(xt, yt)
        torch.cuda.synchronize()
        err = np.max(np.abs(yt.cpu().numpy().astype(np.complex128) - ref)) / np.max(np.abs(ref))
        say(f"  rel err {err:.2e}")
        assert err < (1e-13 if prec == 0 else 2e-6)
    if prec == 0:
        o.init_state()
        g.init_state()
        tr, _ = o.propagate(nsteps=10)
        tg = g.propagate(nsteps=10)
        assert np.array_equal(tg[:, 5], tr[:, 5])
        for col in (1, 2, 3, 4, 6):
            assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10
    # restoring the sine-DVR matrices gives the plain card's product
    plain = card("small_3d")
    op = Oracle(plain)
    g.set_factor(0, None)
    g.set_factor(2, None)
    keys = random_active_set(plain["n"], 0.4, 9)
    x = random_complex(keys.size, 9)
    g.set_state(keys, x)
    xt = torch.from_numpy(x if prec == 0 else x.astype(np.complex64)).cuda()
    yt = torch.zeros_like(xt)
    g.apply_h(xt, yt)
    torch.cuda.synchronize()
    ref = op.apply_def(keys, x if prec == 0 else x.astype(np.complex64).astype(np.complex128))
    assert np.max(np.abs(yt.cpu().numpy().astype(np.complex128) - ref)) / np.max(np.abs(ref)) < (
        1e-13 if prec == 0 else 2e-6)
    h = np.array(cd["dim_factors"][0])
    h[0, 1] += 1e-9
    with pytest.raises(PPQError):
        g.set_factor(0, h)


@pytest.mark.parametrize("name", ["small_3d", "small_4d", "small_6d"])
def test_radius_sqrt2_stencil(name, torch):
    """Ball radius sqrt(2) (2D^2 neighbours): adaption bit-exact on adversarial
    states, the same initial set, and a 10-step trajectory."""
    cd = card(name, stencil=2)
    o = Oracle(cd)
    g = make(cd, torch)
    for seed in (1, 2):
        keys = random_active_set(o.n, 0.3, seed)
        rng = np.random.default_rng(seed)
        c = random_complex(keys.size, seed) * np.exp(rng.uniform(-12, 0, keys.size))
        c[::17] = 1e-3
        say(f"radius sqrt2 {name} seed {seed} |A|={keys.size}")
        o.set_state(keys, c)
        nab = o.prune(eps=1e-3)
        g.set_state(keys, c)
        assert g.prune(eps=1e-3)[1] == nab
        assert np.array_equal(g.state()[0], o.state()[0])
        assert np.array_equal(g.state()[1], o.state()[1])
    o.init_state()
    g.init_state()
    assert np.array_equal(g.state()[0], o.state()[0])
    tr, _ = o.propagate(nsteps=10)
    tg = g.propagate(nsteps=10)
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 2, 3, 4, 6):
        assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10



@pytest.mark.parametrize("name", ["small_3d", "small_4d", "small_6d"])
def test_radius2_stencil(name, torch):
    """Ball radius 2 (every combination of -1/0/+1 changes, 3^D - 1
    neighbours): adaption bit-exact on adversarial states, the same initial
    set, a 10-step trajectory; stencils outside 1..3 are refused."""
    from paper_1606_04004_amd import PPQError
    cd = card(name, stencil=3)
    o = Oracle(cd)
    g = make(cd, torch)
    for seed in (1, 2):
        keys = random_active_set(o.n, 0.3, seed)
        rng = np.random.default_rng(seed)
        c = random_complex(keys.size, seed) * np.exp(rng.uniform(-12, 0, keys.size))
        c[::17] = 1e-3
        say(f"radius 2 {name} seed {seed} |A|={keys.size}")
        o.set_state(keys, c)
        nab = o.prune(eps=1e-3)
        g.set_state(keys, c)
        assert g.prune(eps=1e-3)[1] == nab
        assert np.array_equal(g.state()[0], o.state()[0])
        assert np.array_equal(g.state()[1], o.state()[1])
    o.init_state()
    g.init_state()
    assert np.array_equal(g.state()[0], o.state()[0])
    tr, _ = o.propagate(nsteps=10)
    tg = g.propagate(nsteps=10)
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 2, 3, 4, 6):
        assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10
    for bad in (0, 4):
        with pytest.raises(PPQError):
            g.set_stencil(bad)


@pytest.mark.parametrize("stencil", [2, 3])
def test_wide_stencils_on_lattices(stencil, torch):
    """Radius sqrt(2) and 2 counted over the phase-space axes (cell and level
    of each lattice dimension): adaption bit-exact against the oracle on a
    2D lattice card and a 4D one (3 x 4 per dimension), and a 5-step
    trajectory with the same sets."""
    for cd in (dict(card("small_2d", n=[12, 12], lo=[-5.0, -5.0], hi=[5.0, 5.0]), name="small_lattice2d",
                    basis="pvb", lattice=[3, 4], stencil=stencil),
               dict(lattice_card(), stencil=stencil)):
        o = Oracle(cd)
        g = make(cd, torch)
        for seed in (1, 2):
            keys = random_active_set(o.n, 0.3, seed)
            rng = np.random.default_rng(seed)
            c = random_complex(keys.size, seed) * np.exp(rng.uniform(-12, 0, keys.size))
            c[::17] = 1e-3
            say(f"stencil {stencil} on {cd['name']} seed {seed} |A|={keys.size}")
            o.set_state(keys, c)
            nab = o.prune(eps=1e-3)
            g.set_state(keys, c)
            assert g.prune(eps=1e-3)[1] == nab
            assert np.array_equal(g.state()[0], o.state()[0])
            assert np.array_equal(g.state()[1], o.state()[1])
        o.init_state()
        g.init_state()
        assert np.array_equal(g.state()[0], o.state()[0])
        tr, _ = o.propagate(nsteps=5)
        tg = g.propagate(nsteps=5)
        assert np.array_equal(tg[:, 5], tr[:, 5])
        for col in (1, 2, 3, 4, 6):
            assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10


@pytest.mark.parametrize("which,tol,nsteps,dt", [("hh2d", 1e-8, 25, None), ("small_4d", 1e-6, 15, None),
                                                  ("lattice", 1e-6, 8, None), ("hh2d", 1e-8, 25, -0.05),
                                                  ("small_4d", 1e-6, 15, -0.1)])
def test_adaptive_krylov_order(which, tol, nsteps, dt, torch):
    """Adaptive SIL order (each step stops at the first order whose estimate
    is within the tolerance): the order used per step (an integer the device
    decides) equals the oracle's, and so do the sets and observables, on
    the 2D and 4D DVR cards and a lattice (Arnoldi) card, forward and
    backward in time (the estimate takes |dt|); the FP32 form stays within
    its bound; bad tolerances are refused."""
    from paper_1606_04004_amd import PPQError
    cd = lattice_card() if which == "lattice" else card(which)
    cd = dict(cd, krylov_tol=tol)
    if dt is not None:
        cd["dt"] = dt
    o = Oracle(cd)
    g = make(cd, torch)
    o.init_state()
    g.init_state()
    tr, _ = o.propagate(nsteps=nsteps)
    tg = g.propagate(nsteps=nsteps)
    say(f"adaptive order {which} tol {tol}: orders {tg[1:, 7].astype(int).tolist()}")
    assert np.array_equal(tg[:, 7], tr[:, 7])
    assert np.min(tr[1:, 7]) < cd["krylov"]   # the tolerance did truncate
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 2, 3, 4, 6):
        assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10
    g32 = make(cd, torch, precision=1)
    g32.init_state()
    t32 = g32.propagate(nsteps=nsteps)
    for col in (1, 3, 4):
        assert np.max(np.abs(t32[:, col] - tr[:, col])) < 1e-6
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(PPQError):
            g.set_krylov_tolerance(bad)
    g.set_krylov_tolerance(0.0)
    g.init_state()
    assert np.all(g.propagate(nsteps=2)[1:, 7] == cd["krylov"])


@pytest.mark.parametrize("which,dt,nsteps", [("hh2d", 0.25, 20), ("small_4d", 0.3, 12), ("lattice", 0.3, 6)])
def test_step_control(which, dt, nsteps, torch):
    """Step size control under the Krylov tolerance: the substeps of every
    step and the orders (integers the host reads back) equal the oracle's,
    and so do the sets and observables; a limit too small for a step fails
    with the state as it was before that step."""
    from paper_1606_04004_amd import PPQError
    cd = lattice_card() if which == "lattice" else card(which)
    cd = dict(cd, krylov_tol=1e-10, max_substeps=64, dt=dt)
    o = Oracle(cd)
    g = make(cd, torch)
    o.init_state()
    g.init_state()
    tr, _ = o.propagate(nsteps=nsteps)
    tg = g.propagate(nsteps=nsteps)
    say(f"step control {which} dt {dt}: substeps {tg[1:, 8].astype(int).tolist()} "
        f"orders {tg[1:, 7].astype(int).tolist()}")
    assert np.max(tr[1:, 8]) > 1
    assert np.array_equal(tg[:, 8], tr[:, 8])
    assert np.array_equal(tg[:, 7], tr[:, 7])
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 2, 3, 4, 6):
        assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10
    kg, cg = g.state()
    kr, cr = o.state()
    assert np.array_equal(kg, kr) and np.max(np.abs(cg - cr)) < 1e-10
    g.set_step_control(2)
    g.set_krylov_tolerance(1e-14)
    with pytest.raises(PPQError):
        g.propagate(nsteps=1, dt=2.0, m=6)
    k2, c2 = g.state()
    assert np.array_equal(k2, kg) and np.array_equal(c2, cg)
    for bad in (0, 2000):
        with pytest.raises(PPQError):
            g.set_step_control(bad)


@pytest.mark.parametrize("basis", ["pvb", "pw"])
def test_lattices_on_fourier_grids(basis, torch):
    """Lattice bases projected on periodic Fourier grids (15 x 15, 3 x 5
    cells and momenta per dimension): products against the oracle's on a
    random set, the initial set, and a 10-step pruned trajectory; a Fourier
    grid set after the lattice is refused."""
    from paper_1606_04004_amd import PPQError
    cd = dict(card("small_2d", n=[15, 15], fgh=[0, 1]), name="fgh_lattice2d", basis=basis, lattice=[3, 5])
    o = Oracle(cd)
    g = make(cd, torch)
    keys = random_active_set(o.n, 0.6, 3)
    x = random_complex(keys.size, 4)
    g.set_state(keys, x)
    xt = torch.from_numpy(x).cuda()
    yt = torch.zeros_like(xt)
    g.apply_h(xt, yt)
    torch.cuda.synchronize()
    ref = o.apply_def(keys, x)
    say(f"{basis} on Fourier grids: product error {np.max(np.abs(yt.cpu().numpy() - ref)):.2e}")
    assert np.max(np.abs(yt.cpu().numpy() - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))
    o.init_state()
    g.init_state()
    assert np.array_equal(g.state()[0], o.state()[0])
    tr, _ = o.propagate(nsteps=10)
    tg = g.propagate(nsteps=10)
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 2, 3, 4, 6):
        assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10
    with pytest.raises(PPQError):
        g._call("ppq_set_fgh", 0)


@pytest.mark.parametrize("stencil", [2, 3])
def test_options_together(stencil, torch):
    """The adaption and integrator options at once on the 3D card: a wider
    stencil, a relative exclusion threshold and an adaptive SIL order;
    per-step sets, Krylov orders and observables equal the oracle's over 20
    steps, and the position expectations agree at the end."""
    cd = dict(card("small_3d"), stencil=stencil, krylov_tol=1e-7)
    o = Oracle(cd)
    g = make(cd, torch)
    g.set_relative_exclusion(0.02)
    o.init_state()
    g.init_state()
    recs_o, recs_g = [], []
    for _ in range(20):
        used, _ = o.sil_step()
        nab = o.prune(rel_excl=0.02)
        recs_o.append((used, nab, o.state()[0].size))
        g.step()
        na, nb = g.prune()
        recs_g.append((None, nb, na))
        assert np.array_equal(g.state()[0], o.state()[0])
    assert [r[1:] for r in recs_g] == [r[1:] for r in recs_o]
    assert min(r[0] for r in recs_o) < cd["krylov"]
    _, cg = g.state()
    _, co = o.state()
    assert np.max(np.abs(cg - co)) < 1e-10
    assert np.max(np.abs(g.expect_q() - o.expect_q())) < 1e-10

def test_acf_doubled(torch):
    """C(2t) with a real packet: on DVR dimensions sum c^2 and on lattice
    bases (projected von Neumann and projected Weylets) a^T B^T B a through
    the full-grid transform; each equals the oracle's on its own state after
    the same pruned steps (identical sets), and, unpruned, the C(t) record at
    twice the time."""
    from paper_1606_04004_amd import PPQError
    base = card("small_3d")
    base["psi0"] = dict(base["psi0"], momentum=[0.0, 0.0, 0.0])
    lat = dict(card("small_4d", n=[12, 12, 12, 12]), name="small_lattice4d", lattice=[3, 4])
    lat["psi0"] = dict(lat["psi0"], momentum=[0.0] * 4)
    for cd in (base, dict(lat, basis="pvb"), dict(lat, basis="pw")):
        o = Oracle(cd)
        g = make(cd, torch)
        o.init_state()
        g.init_state()
        o.propagate(nsteps=6)
        g.propagate(nsteps=6)
        assert np.array_equal(g.state()[0], o.state()[0])
        d = abs(g.acf_doubled() - o.acf_doubled())
        say(f"C(2t) {cd.get('basis')}: gpu vs oracle {d:.2e}")
        assert d < 1e-10
        g.init_state(eps=0.0)
        tr = g.propagate(nsteps=12, prune=False)
        g.init_state(eps=0.0)
        g.propagate(nsteps=6, prune=False)
        c2 = g.acf_doubled()
        say(f"  C(2t) {c2} record {tr[12, 3]} {tr[12, 4]}")
        assert abs(c2 - complex(tr[12, 3], tr[12, 4])) < 1e-9
    # refused for an operator that is not real symmetric
    g = make(base, torch)
    g.init_state()
    g.add_term(0.01, [{"dim": 0, "kind": "power", "p": 2}], coef_im=0.01)
    with pytest.raises(PPQError):
        g.acf_doubled()


def weylet_card(n=12, nx=3, npm=4, **kw):
    base = card("small_4d", n=[n, n, n, n], **kw)
    return dict(base, name="small_weylet4d", basis="pw", lattice=[nx, npm])


def test_weylet_products(torch):
    """Projected Weylets (real orthogonal W, dense factors W^T h W and the
    truncated pair terms): products on random sets against the oracle."""
    cd = weylet_card()
    o = Oracle(cd)
    g = make(cd, torch)
    for fill, seed in ((1.0, 1), (0.3, 2), (0.05, 3)):
        keys = (np.arange(int(np.prod(cd["n"])), dtype=np.uint64) if fill == 1.0
                else random_active_set(cd["n"], fill, seed))
        x = random_complex(keys.size, seed + 30)
        say(f"weylet product |A|={keys.size}")
        g.set_state(keys, x)
        xt = torch.from_numpy(x).cuda()
        yt = torch.zeros_like(xt)
        g.apply_h(xt, yt)
        torch.cuda.synchronize()
        ref = o.apply_def(keys, x)
        err = np.max(np.abs(yt.cpu().numpy() - ref)) / np.max(np.abs(ref))
        say(f"  rel err {err:.2e}")
        assert err < 1e-13


def test_weylet_trajectory(torch):
    """Projected Weylets: identical initial set, sets and observables over 10
    steps (Arnoldi, lattice-cell stencil)."""
    cd = weylet_card(eps=1e-4)
    o = Oracle(cd)
    o.init_state()
    g = make(cd, torch)
    g.init_state()
    assert np.array_equal(g.state()[0], o.state()[0])
    tr, _ = o.propagate(nsteps=10, dt=0.05)
    tg = g.propagate(nsteps=10, dt=0.05)
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 2, 3, 4, 6):
        d = np.max(np.abs(tg[:, col] - tr[:, col]))
        say(f"  col {col}: {d:.2e}")
        assert d < 1e-10


def test_weylet_full_size_card(torch):
    """The 4D lattice card's size (48^4) with projected Weylets on a 6 x 8
    doubly dense lattice: identical initial set and two steps."""
    cd = dict(card("pvb4d"), basis="pw")
    say("pw 48^4: 2 steps")
    o = Oracle(cd)
    o.init_state()
    g = make(cd, torch)
    g.init_state()
    assert np.array_equal(g.state()[0], o.state()[0])
    tr, _ = o.propagate(nsteps=2)
    tg = g.propagate(nsteps=2)
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 2, 3, 4, 6):
        d = np.max(np.abs(tg[:, col] - tr[:, col]))
        say(f"  col {col}: {d:.2e}")
        assert d < 1e-10


@pytest.mark.parametrize("prec", [0, 1])
def test_fgh_dimensions(prec, torch):
    """Periodic Fourier grids on two dimensions (points, kinetic matrix,
    potential and packet on those points): products against the oracle, the
    initial set and a 10-step trajectory; even sizes are refused."""
    import ctypes
    from paper_1606_04004_amd import PPQError
    cd = card("small_3d", fgh=[0, 1])
    o = Oracle(cd)
    g = make(cd, torch, precision=prec)
    q = np.zeros(cd["n"][0])
    g.lib.ppq_get_grid(g.ctx, 0, q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert np.allclose(q, o.model.q[0], rtol=0, atol=1e-14)
    for fill, seed in ((1.0, 1), (0.4, 2)):
        keys = (np.arange(int(np.prod(cd["n"])), dtype=np.uint64) if fill == 1.0
                else random_active_set(cd["n"], fill, seed))
        x = random_complex(keys.size, seed + 40)
        g.set_state(keys, x)
        xs = x if prec == 0 else x.astype(np.complex64)
        xt = torch.from_numpy(xs).cuda()
        yt = torch.zeros_like(xt)
        g.apply_h(xt, yt)
        torch.cuda.synchronize()
        ref = o.apply_def(keys, xs.astype(np.complex128))
        err = np.max(np.abs(yt.cpu().numpy().astype(np.complex128) - ref)) / np.max(np.abs(ref))
        say(f"fgh prec {prec} |A|={keys.size} rel err {err:.2e}")
        assert err < (1e-13 if prec == 0 else 2e-6)
    if prec == 0:
        o.init_state()
        g.init_state()
        assert np.array_equal(g.state()[0], o.state()[0])
        tr, _ = o.propagate(nsteps=10)
        tg = g.propagate(nsteps=10)
        assert np.array_equal(tg[:, 5], tr[:, 5])
        for col in (1, 2, 3, 4, 6):
            assert np.max(np.abs(tg[:, col] - tr[:, col])) < 1e-10
    with pytest.raises(PPQError):
        make(card("small_3d", fgh=[2]), torch)
