"""Benchmark: pruned H*psi active-point updates/s and steps/s on one MI355X.

Workload: the 6D SoP quartic model (sine-DVR 24^6 = 191,102,976-function
grid, eps = 1e-6, dt = 0.05, Lanczos order 10), started from its Gaussian
packet and propagated to a mid-trajectory snapshot (step 250) before timing.
A step is one pass of the whole hot path: one short-iterative Lanczos step
(10 pruned H*psi products with the fused diagonal potential, full
reorthogonalisation, the small exponential, the linear combination), the
adaption (flag, dilate, compact, remap), the rebuild of the fiber tables and
the potential cache, and the observables.

value = total H*psi point updates in the K timed steps (sum over steps of
m * |A|) / wall time of those K steps.  The isolated H*psi rate, the
roofline of the H*psi kernels and the FP32 form are reported beside it, and
secondary lines (not the headline) time the other workloads: the 4D coupled
Morse model (FP64 and FP32), its phase-space lattice form, and the adjoint
gradient of the survival probability (FP64 and FP32).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# adaptive SIL order: tolerance = this factor x eps (on the 2D card it keeps
# the infidelity of the fixed order; eps itself lets the integrator error
# dominate over 200 steps)
ADAPTIVE_TOL_FACTOR = 1e-2
SNAPSHOT_STEP = 250
# Measured fabric-side bytes per active point of one FP64 product on this
# workload's snapshot (FETCH_SIZE x 2 + WRITE_SIZE, calibrated on a 1 GiB
# copy; profiles/hpsi_quartic6d_24pow6_traffic.md).  Valid for the
# per-dimension layout's kernels as measured there.
TRAFFIC_BYTES_PER_POINT_FP64 = 322.5
TRAFFIC_SOURCE = "profiles/hpsi_quartic6d_24pow6_traffic.md"


def bytes_per_point(D, precision):
    """Algorithmic bytes of one pruned H*psi per active point: read x once,
    write y once, one 32-bit fiber/permutation entry per dimension."""
    sc = 16 if precision == 0 else 8
    return 2 * sc + 4 * D


def describe(cd):
    names = {"quartic6d": "6D SoP quartic", "morse4d": "4D coupled Morse", "hh2d": "2D Henon-Heiles",
             "pvb4d": "4D coupled Morse in a 6x8 phase-space lattice basis per dimension",
             "adjoint4d": "4D coupled Morse (adjoint card)"}
    n = cd["n"]
    return (f"{cd['name']}: {names.get(cd['name'], cd['name'])}, sine-DVR {n[0]}^{cd['D']} on "
            f"[{cd['lo'][0]},{cd['hi'][0]}]^{cd['D']}, eps={cd['eps']}, dt={cd['dt']}, m={cd['krylov']}")


def cpu_baseline(cd, reps=9, max_threads=16):
    """The FP64 oracle as it stands (O-fib, the appendix algorithm, serial C)
    on its own initial set of the card, which stands in for the GPU's
    step-250 snapshot (3.52M against 3.60M functions; the oracle would need
    about 20 minutes to propagate there, and its inputs never come from the
    GPU path).  One thread: the median of `reps` products, and one whole step
    (SIL step of the card's order, adaption, rebuild of the permutations).
    All cores: that many threads each applying H to the same set at once (the
    oracle's tables are read-only, and ctypes releases the GIL during the
    call), aggregate rate."""
    import threading
    from oracle.oracle import Oracle
    o = Oracle(cd)
    o.init_state()
    keys, c = o.state()
    n = keys.size
    o.apply_current(c)  # builds the stored permutations (not timed)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        o.apply_current(c)
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    nthreads = max(1, min(os.cpu_count() or 1, max_threads))
    per_thread = 3
    xs = [c.copy() for _ in range(nthreads)]

    def work(i):
        for _ in range(per_thread):
            o.apply_current(xs[i])
    th = [threading.Thread(target=work, args=(i,)) for i in range(nthreads)]
    t0 = time.perf_counter()
    for t in th:
        t.start()
    for t in th:
        t.join()
    wall = time.perf_counter() - t0
    agg = n * nthreads * per_thread / wall
    t0 = time.perf_counter()
    o.sil_step()
    o.prune()
    o.apply_current(o.state()[1])  # rebuilds the permutations of the new set
    step_s = time.perf_counter() - t0
    try:
        cpu_model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except (OSError, IndexError):
        cpu_model = "unknown"
    return {"value": agg, "unit": "active-point updates/s", "cores": nthreads, "kind": "oracle",
            "sample": f"O-fib H*psi on the oracle's initial set of the 6D quartic card (|A0| = {n}): "
                      f"{nthreads} threads x {per_thread} products at once ({wall:.1f} s); one thread: median of "
                      f"{reps} products and one whole step",
            "one_thread": {"hpsi_median_s": med, "updates_per_s": n / med, "step_s": step_s,
                           "step_updates_per_s": cd["krylov"] * n / step_s},
            "host": {"nproc": os.cpu_count(), "cpu": cpu_model}}


def timed_steps(g, steps, warmup):
    """Whole-path steps through the library's propagation loop (SIL step,
    adaption, fiber tables and potential cache of the new set, observable
    record), one call for all steps.  Returns (updates/s, ms per step, trace);
    an update is one active point through one H*psi product, so step s counts
    its Krylov dimension times the size of the set it acted on."""
    import torch
    if warmup:
        g.propagate(nsteps=warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = g.propagate(nsteps=steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    upd = float(np.sum(tr[1:, 7] * tr[:-1, 5]))
    return upd / wall, wall * 1e3 / steps, tr


def secondary(stream, steps, warmup, adjoint_steps):
    """Other workloads, each from its own seeded start (not the headline)."""
    import torch
    import paper_1606_04004_amd as ppq
    from paper_1606_04004_amd.adjoint import declare_trainable
    from workloads import card
    out = {}
    cd = card("morse4d")
    for prec, tag in ((ppq.PPQ_FP64, "fp64"), (ppq.PPQ_FP32, "fp32")):
        g = ppq.Propagator(cd, precision=prec, device=0, stream=stream)
        g.reserve(min(16_000_000, int(np.prod(cd["n"]))))  # as for the headline
        g.init_state()
        g.propagate(nsteps=20)
        ms_h = g.time_apply(100)
        na = g.active_count()
        rate, ms, _ = timed_steps(g, steps, warmup)
        out[f"morse4d_{tag}"] = {"active_points": int(na), "hpsi_ms": ms_h, "hpsi_updates_per_s": na / (ms_h * 1e-3),
                                 "updates_per_s": rate, "ms_per_step": ms,
                                 "from": "step 20 of the 4D coupled Morse card (32^4, eps 1e-6, dt 0.1, m 10)"}
        del g
    cd = card("pvb4d")
    for prec, tag in ((ppq.PPQ_FP64, "fp64"), (ppq.PPQ_FP32, "fp32")):
        g = ppq.Propagator(cd, precision=prec, device=0, stream=stream)
        g.reserve(min(16_000_000, int(np.prod(cd["n"]))))  # as for the headline
        g.init_state()
        # algorithmic flops of one product: a complex factor application costs
        # 8 L flops per point for fibers of mean length L = |A| / nf_k; one per
        # dimension for the single-dimension factors and two per pair term
        apps = [k for k in range(cd["D"])]
        for t in cd["terms"]:
            dims = sorted(set(f["dim"] for f in t["factors"]))
            if len(dims) > 1:
                apps += dims

        def product_flops():
            n_act, nf = g.active_count(), g.fiber_counts()
            return n_act, float(sum(8.0 * n_act * (n_act / nf[k]) for k in apps))

        ms_h = g.time_apply(100)
        na, alg = product_flops()
        rate, ms, _ = timed_steps(g, steps, warmup)
        # the same product on the set the timed steps grew to (near the full grid)
        ms_g = g.time_apply(20)
        na_g, alg_g = product_flops()
        out[f"pvb4d_{tag}"] = {"active_points": int(na), "hpsi_ms": ms_h, "updates_per_s": rate, "ms_per_step": ms,
                               "factor_applications": len(apps),
                               "algorithmic_gflop_per_product": alg / 1e9,
                               "algorithmic_tflops": alg / (ms_h * 1e-3) / 1e12,
                               "grown_active_points": int(na_g), "grown_hpsi_ms": ms_g,
                               "grown_algorithmic_tflops": alg_g / (ms_g * 1e-3) / 1e12,
                               "from": "initial set of the 4D phase-space lattice card (48^4, 6x8 lattice per "
                                       "dimension), complex factors on the matrix cores; grown_*: the set after "
                                       "the timed steps"}
        del g
    cd = dict(card("pvb4d"), basis="pw")
    for prec, tag in ((ppq.PPQ_FP64, "fp64"), (ppq.PPQ_FP32, "fp32")):
        g = ppq.Propagator(cd, precision=prec, device=0, stream=stream)
        g.reserve(min(16_000_000, int(np.prod(cd["n"]))))  # as for the headline
        g.init_state()
        na = g.active_count()
        ms_h = g.time_apply(100)
        rate, ms, _ = timed_steps(g, steps, warmup)
        out[f"pw4d_{tag}"] = {"active_points": int(na), "hpsi_ms": ms_h, "updates_per_s": rate, "ms_per_step": ms,
                              "from": "initial set of the 4D Morse model in projected Weylets (48^4, 6x8 "
                                      "doubly dense lattice per dimension)"}
        del g
    cd = card("adjoint4d", nsteps=adjoint_steps)
    grads = {}
    for prec, tag in ((ppq.PPQ_FP64, "fp64"), (ppq.PPQ_FP32, "fp32")):
        g = ppq.Propagator(cd, precision=prec, device=0, stream=stream)
        declare_trainable(g, cd)
        print(f"[bench] adjoint {tag}: {adjoint_steps} steps ...", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = g.adjoint_record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dp, dc, dm = g.adjoint_gradient()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        grads[tag] = np.concatenate([dp, dc, dm])
        out[f"adjoint4d_{tag}"] = {"steps": adjoint_steps, "checkpoint_every": cd["checkpoint_every"],
                                   "dt": cd["dt"], "max_krylov_order": cd["krylov"],
                                   "step_tolerance": 1e-12, "J": J, "forward_record_s": t1 - t0,
                                   "backward_s": t2 - t1, "final_active": int(g.active_count()),
                                   "gradient_components": int(grads[tag].size),
                                   "grad_norm": float(np.linalg.norm(grads[tag]))}
        del g
    out["adjoint4d_fp32"]["grad_max_rel_err_vs_fp64"] = float(
        np.max(np.abs(grads["fp32"] - grads["fp64"])) / np.max(np.abs(grads["fp64"])))
    out["adjoint4d_fp32"]["J_rel_err_vs_fp64"] = abs(out["adjoint4d_fp32"]["J"] - out["adjoint4d_fp64"]["J"]) / \
        abs(out["adjoint4d_fp64"]["J"])
    out["hh2d_accuracy"] = accuracy_sweep(stream)
    out["dwell2d_accuracy"] = dwell_sweep(stream)
    return out


def accuracy_sweep(stream):
    """The paper's accuracy measure on the 2D card (Sec. III.A): the
    infidelity of C(t), sqrt(sum_n |C_pruned(t_n) - C_exact(t_n)|^2) over all
    201 records, against the mean number of functions used (percent of the
    48^2 grid), per threshold, for the DVR with each of the three neighbour
    stencils (ball radius 1, sqrt(2), 2), for the projected von Neumann
    lattice with each stencil (counted over its phase-space axes) and for the
    projected Weylet lattice (6 x 8 per
    dimension), and for the DVR with the SIL order adapted to a tolerance
    of eps / 100; the exact run keeps the full DVR grid without adaption (all
    three bases are similarity transforms of it)."""
    import torch
    import paper_1606_04004_amd as ppq
    from workloads import card
    cd = card("hh2d")
    total = int(np.prod(cd["n"]))
    g = ppq.Propagator(cd, precision=ppq.PPQ_FP64, device=0, stream=stream)
    g.init_state(eps=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = g.propagate(prune=False)
    torch.cuda.synchronize()
    ms_exact = (time.perf_counter() - t0) * 1e3 / (ref.shape[0] - 1)
    c_ref = ref[:, 3] + 1j * ref[:, 4]
    del g
    rows = []
    pvb = {"basis": "pvb", "lattice": [6, 8]}
    variants = (("dvr", 1, {}), ("dvr", 2, {"stencil": 2}), ("dvr", 3, {"stencil": 3}),
                ("pvb", 1, pvb), ("pvb", 2, dict(pvb, stencil=2)), ("pvb", 3, dict(pvb, stencil=3)),
                ("pw", 1, {"basis": "pw", "lattice": [6, 8]}),
                ("dvr_adaptive_order", 1, {"krylov_tol": None}))
    for basis, stencil, extra in variants:
        for eps in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
            # the adaptive variant ties the SIL order's tolerance to eps
            ex = {k: (ADAPTIVE_TOL_FACTOR * eps if v is None else v) for k, v in extra.items()}
            g = ppq.Propagator(dict(cd, **ex), precision=ppq.PPQ_FP64, device=0, stream=stream)
            g.init_state(eps=eps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tr = g.propagate(eps=eps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            c = tr[:, 3] + 1j * tr[:, 4]
            rows.append({"basis": basis, "stencil": stencil, "eps": eps,
                         "mean_basis_percent": float(100.0 * np.mean(tr[:, 5]) / total),
                         "mean_krylov_order": float(np.mean(tr[1:, 7])),
                         "infidelity": float(np.sqrt(np.sum(np.abs(c - c_ref) ** 2))),
                         "ms_per_step": wall * 1e3 / (tr.shape[0] - 1)})
            del g
    return {"exact_ms_per_step": ms_exact, "runs": rows}


def dwell_sweep(stream):
    """The paper's 2D double well (Sec. III.A, Figs. 3 and 4): for the pruned
    Fourier-grid DVR, the projected von Neumann lattice (15 x 11 and 9 x 9)
    and projected Weylets, per threshold the infidelity of C(t) over the run
    to t_e = 24.6 against the unpruned 165 x 81 Fourier-grid run, the mean
    share of the 13365-function basis used and the time per step.  Every run
    keeps the integrator within 1e-10 per step (adaptive order up to 15,
    substeps as needed), so the infidelity is the pruning error.  The card
    reads the coupling as 10 x^2 (y-2) (the printed 10 x^2 y leaves no double
    well; see workloads/cards.py)."""
    import torch
    import paper_1606_04004_amd as ppq
    from workloads import card
    base = card("dwell2d")
    total = int(np.prod(base["n"]))
    g = ppq.Propagator(base, precision=ppq.PPQ_FP64, device=0, stream=stream)
    g.init_state(eps=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = g.propagate(prune=False)
    torch.cuda.synchronize()
    ms_exact = (time.perf_counter() - t0) * 1e3 / (ref.shape[0] - 1)
    c_ref = ref[:, 3] + 1j * ref[:, 4]
    del g
    rows = []
    for basis in ("dvr", "pw", "pvb"):
        for eps in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-8):
            cd = card("dwell2d", basis=basis)
            g = ppq.Propagator(cd, precision=ppq.PPQ_FP64, device=0, stream=stream)
            g.init_state(eps=eps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tr = g.propagate(eps=eps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            c = tr[:, 3] + 1j * tr[:, 4]
            rows.append({"basis": basis, "eps": eps,
                         "mean_basis_percent": float(100.0 * np.mean(tr[:, 5]) / total),
                         "infidelity": float(np.sqrt(np.sum(np.abs(c - c_ref) ** 2))),
                         "mean_substeps": float(np.mean(tr[1:, 8])),
                         "ms_per_step": wall * 1e3 / (tr.shape[0] - 1), "wall_s": wall})
            print(f"[bench] double well {basis} eps {eps}: {rows[-1]}", file=sys.stderr, flush=True)
            del g
    return {"card": base["name"], "exact_ms_per_step": ms_exact, "exact_wall_s": ms_exact * (ref.shape[0] - 1) / 1e3,
            "t_end": base["dt"] * base["nsteps"], "runs": rows}


def traffic_probe(stream):
    """A plain device copy of known size, the calibration dispatch for the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    return {"copy_bytes": nbytes}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--snapshot", type=int, default=SNAPSHOT_STEP)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--workload", default="quartic6d")
    ap.add_argument("--no-secondary", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--traffic-probe", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1606_04004_amd as ppq
    from workloads import card

    cd = card(args.workload)
    D, m, dt, eps = cd["D"], cd["krylov"], cd["dt"], cd["eps"]
    print(f"[bench] workload {cd['name']} D={D} n={cd['n'][0]} eps={eps}", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    total = int(np.prod(cd["n"]))
    cap = min(16_000_000, total)
    g = ppq.Propagator(cd, precision=ppq.PPQ_FP64, device=0, stream=stream)
    g.reserve(cap)
    n0 = g.init_state()
    t0 = time.perf_counter()
    g.propagate(nsteps=args.snapshot)
    torch.cuda.synchronize()
    print(f"[bench] |A0|={n0}; reached step {args.snapshot} in {time.perf_counter() - t0:.2f} s",
          file=sys.stderr, flush=True)

    # snapshot (kept for the FP32 leg)
    snap_keys, snap_c = g.state()
    # isolated H*psi timing on the snapshot (HIP events on the context stream)
    n_snap = snap_keys.size
    ms_h, ms_h_mean = g.time_apply(100, mean=True)
    hpsi_rate = n_snap / (ms_h * 1e-3)
    bpp = bytes_per_point(D, 0)
    achieved = bpp * n_snap / (ms_h * 1e-3) / 1e9

    # whole-path steps
    value, ms_step, _ = timed_steps(g, args.steps, args.warmup)
    obs64 = g.observables()      # the FP32 leg is compared with this state
    # where a step's time goes: a few more steps with the phase events on
    # (outside the timed region; the events cost a few us per step)
    g.enable_timings(True)
    nph = min(args.steps, 5)
    g.propagate(nsteps=nph)
    phases = {k: v / nph for k, v in g.timings().items()}
    g.enable_timings(False)
    # the integrator's accuracy tied to the threshold: the adaptive SIL order
    # with tolerance eps and eps / 100 against the full order, each from the
    # snapshot over the same steps (outside the headline figure)
    g.set_state(snap_keys, snap_c)
    _, ms_full, tr_full = timed_steps(g, args.steps, 0)
    acf = lambda tr: tr[:, 3] + 1j * tr[:, 4]
    adaptive = {"ms_per_step_full_order": ms_full, "steps": args.steps, "runs": []}
    for tol in (eps, ADAPTIVE_TOL_FACTOR * eps):
        g.set_state(snap_keys, snap_c)
        g.set_krylov_tolerance(tol)
        _, ms_ad, tr_ad = timed_steps(g, args.steps, 0)
        adaptive["runs"].append({
            "tolerance": tol, "ms_per_step": ms_ad,
            "orders_used": sorted(set(tr_ad[1:, 7].astype(int).tolist())),
            "acf_max_diff_vs_full_order": float(np.max(np.abs(acf(tr_ad) - acf(tr_full)))),
            "norm2_max_diff_vs_full_order": float(np.max(np.abs(tr_ad[:, 1] - tr_full[:, 1])))})
    g.set_krylov_tolerance(0.0)

    out = {
        "metric": "pruned H*psi active-point updates/s (whole step) + steps/s",
        "value": value,
        "unit": "active-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "steps_per_s": 1e3 / ms_step,
        "hpsi_updates_per_s": hpsi_rate,
        "hpsi_ms": ms_h,
        "hpsi_ms_mean": ms_h_mean,
        "hpsi_timing": "median of 100 back-to-back products (HIP events on the context stream)",
        "active_points_at_snapshot": int(n_snap),
        "phase_ms_per_step": phases,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": describe(cd) + f", timed from the step-{args.snapshot} snapshot",
                   "grid": total, "D": D, "krylov": m, "eps": eps, "dt": dt},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (TRAFFIC_BYTES_PER_POINT_FP64 * n_snap
                                 if args.workload == "quartic6d" and args.snapshot == SNAPSHOT_STEP else None),
                     "traffic_unit": "bytes per product (fabric side, counter-calibrated)",
                     "traffic_source": TRAFFIC_SOURCE,
                     "kernel": "pruned H*psi (D fiber passes, potential fused in the first)",
                     "bytes_per_point": bpp},
    }

    out["adaptive_order"] = adaptive

    if not args.no_fp32:
        g32 = ppq.Propagator(cd, precision=ppq.PPQ_FP32, device=0, stream=stream)
        g32.reserve(cap)
        g32.init_state()
        g32.set_state(snap_keys, snap_c)
        ms32 = g32.time_apply(100)
        value32, ms_step32, _ = timed_steps(g32, args.steps, args.warmup)
        bpp32 = bytes_per_point(D, 1)
        obs32 = g32.observables()
        g32.enable_timings(True)
        g32.propagate(nsteps=nph)
        phases32 = {k: v / nph for k, v in g32.timings().items()}
        g32.enable_timings(False)
        err = {k: abs(obs32[k] - obs64[k]) for k in ("norm2", "acf_re", "acf_im")}
        err["energy_rel"] = abs(obs32["energy"] - obs64["energy"]) / abs(obs64["energy"])
        err["n_active_rel"] = abs(obs32["n_active"] - obs64["n_active"]) / obs64["n_active"]
        out["fp32"] = {"value": value32, "ms_per_step": ms_step32, "phase_ms_per_step": phases32,
                       "error_vs_fp64_after_steps": err,
                       "hpsi_updates_per_s": n_snap / (ms32 * 1e-3), "hpsi_ms": ms32,
                       "roofline_frac": bpp32 * n_snap / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "bytes_per_point": bpp32}

    if not args.no_secondary:
        print("[bench] secondary workloads ...", file=sys.stderr, flush=True)
        out["secondary"] = secondary(stream, args.steps, args.warmup, args.adjoint_steps)
    if args.traffic_probe:
        out["traffic_probe"] = traffic_probe(stream)

    if not args.no_cpu:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cd)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
