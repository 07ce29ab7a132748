"""The entry point that allocates no device memory (ppq_expect_q_noalloc):
its result equals ppq_expect_q's bit for bit and the oracle's definition of
the position expectation within 1e-12, on two calls in a row, the second
with a smaller state (and on a card with a Fourier-grid dimension and one
with lattice dimensions, where position is not diagonal: NaN)."""
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


def _same(a, b):
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_expect_q_two_calls(prec, torch):
    cd = card("morse4d")
    g = make(cd, torch, precision=prec)
    o = Oracle(cd)
    # first call: a large blob-shaped set; second: a smaller one
    for ncall, (fill, seed) in enumerate(((0.3, 1), (0.02, 2))):
        keys = random_active_set(cd["n"], fill, seed, blob=True)
        c = random_complex(keys.size, seed + 100)
        say(f"noalloc expect_q prec {prec} call {ncall}: |A| = {keys.size}")
        g.set_state(keys, c)
        o.set_state(keys, c)
        q_ref = g.expect_q()
        q_na = g.expect_q_noalloc()
        assert _same(q_na, q_ref), (q_na, q_ref)
        q_or = o.expect_q()
        assert np.max(np.abs(q_na - q_or)) < 1e-12


def test_noalloc_expect_q_fgh_and_lattice(torch):
    cd = card("small_3d", fgh=[1], n=[9, 11, 10])
    g = make(cd, torch)
    o = Oracle(cd)
    g.init_state()
    o.init_state()
    g.propagate(nsteps=5)
    o.propagate(nsteps=5)
    q_na = g.expect_q_noalloc()
    assert _same(q_na, g.expect_q())
    assert np.max(np.abs(q_na - o.expect_q())) < 1e-10
    base = card("small_4d", n=[12, 12, 12, 12])
    lat = dict(base, name="small_lattice4d", basis="pvb", lattice=[3, 4])
    gl = make(lat, torch)
    gl.init_state()
    q_lat = gl.expect_q_noalloc()
    assert np.all(np.isnan(q_lat)) and _same(q_lat, gl.expect_q())
    # and back on the first context after the lattice call
    assert _same(g.expect_q_noalloc(), g.expect_q())


def test_noalloc_expect_q_refuses_without_state(torch):
    from paper_1606_04004_amd import PPQError
    g = make(card("small_2d"), torch)
    with pytest.raises(PPQError):
        g.expect_q_noalloc()
