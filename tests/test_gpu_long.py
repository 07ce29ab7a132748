"""Dimensions longer than 64 points (long fibers, up to 256) on the GPU
against the oracle, and the paper's two-dimensional double well (Sec. III.A):
165 x 81 Fourier grids, and its projected von Neumann (15 x 11, 9 x 9) and
projected-Weylet lattices.  Bars as in test_gpu_parity: products 1e-13
relative (FP32 1e-6), identical active sets, observables within 1e-10."""
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


def long3d():
    """A 3D sine-DVR card with a long first and last dimension around a short one."""
    cd = card("small_3d", n=[70, 9, 130])
    return dict(cd, name="long3d")


CASES = [("dwell2d", "dvr", 1.0, 1), ("dwell2d", "dvr", 0.3, 2), ("long3d", "dvr", 0.2, 3),
         ("long3d", "dvr", 0.02, 4), ("dwell2d", "pvb", 0.3, 5), ("dwell2d", "pw", 0.25, 6)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name,basis,fill,seed", CASES)
def test_long_dimension_products(name, basis, fill, seed, prec, torch):
    cd = long3d() if name == "long3d" else card(name, basis=basis)
    n = cd["n"]
    keys = np.arange(int(np.prod(n)), dtype=np.uint64) if fill == 1.0 else random_active_set(n, fill, seed)
    x = random_complex(keys.size, seed + 50)
    say(f"long dims {name} {basis} fill {fill} prec {prec}: |A| = {keys.size}")
    o = Oracle(cd)
    xin = x if prec == 0 else x.astype(np.complex64).astype(np.complex128)
    ref = o.apply_def(keys, xin)
    g = make(cd, torch, prec)
    g.set_state(keys, x)
    xt = torch.from_numpy(x).cuda()
    if prec == 1:
        xt = xt.to(torch.complex64)
    yt = torch.zeros_like(xt)
    g.apply_h(xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy().astype(np.complex128)
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    say(f"  rel err {err:.2e}")
    assert err < (1e-13 if prec == 0 else 1e-6)
    # fiber counts of every dimension equal the oracle's
    assert g.fiber_counts().tolist() == [len(o.fiber_ranges(keys, k)) for k in range(cd["D"])]


@pytest.mark.parametrize("basis,nsteps", [("dvr", 40), ("pw", 12), ("pvb", 6)])
def test_double_well_trajectory(basis, nsteps, torch):
    """The paper's double well in each basis: step control (tolerance 1e-10,
    substeps, orders up to 15) and adaption every step; the substeps and
    orders of every step, the active sets and the observables equal the
    oracle's."""
    cd = card("dwell2d", basis=basis)
    o = Oracle(cd)
    g = make(cd, torch)
    o.init_state()
    g.init_state()
    tr, _ = o.propagate(nsteps=nsteps)
    tg = g.propagate(nsteps=nsteps)
    say(f"double well {basis}: |A| {tg[0, 5]:.0f} -> {tg[-1, 5]:.0f}, substeps "
        f"{sorted(set(tg[1:, 8].astype(int).tolist()))}, orders {sorted(set(tg[1:, 7].astype(int).tolist()))}")
    assert np.array_equal(tg[:, 8], tr[:, 8])
    assert np.array_equal(tg[:, 7], tr[:, 7])
    assert np.array_equal(tg[:, 5], tr[:, 5])
    for col in (1, 2, 3, 4, 6):
        d = np.max(np.abs(tg[:, col] - tr[:, col]))
        assert d < 1e-10 * max(1.0, np.max(np.abs(tr[:, col]))), (col, d)
    kg, cg = g.state()
    kr, cr = o.state()
    assert np.array_equal(kg, kr)
    assert np.max(np.abs(cg - cr)) < 1e-10


def test_double_well_acf_doubled(torch):
    """The double well's packet is real: C(2t) from the state at t (FGH grid
    and projected Weylets) equals the oracle's on the same trajectory."""
    for basis in ("dvr", "pw"):
        cd = card("dwell2d", basis=basis)
        o = Oracle(cd)
        g = make(cd, torch)
        o.init_state()
        g.init_state()
        o.propagate(nsteps=10)
        g.propagate(nsteps=10)
        d = abs(g.acf_doubled() - o.acf_doubled())
        say(f"double well {basis} C(2t) gpu vs oracle {d:.2e}")
        assert d < 1e-10
