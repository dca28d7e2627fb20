"""GPU CG-SENSE against the FP64 oracle CG, through the C ABI.

Tolerances (relative L2 per batch element):
* 1e-5 wherever fp32 storage allows it: the 64x64 / 4-coil / R=2 solve
  (20 iterations) and the first 10 iterations of the 256x256 / 12-coil /
  VD R=4 solve;
* for the full 30-iteration 256x256 solve, K_FLOOR times the
  complex64-storage floor computed here for the same problem (the oracle's
  own loop with every CG vector rounded to complex64, oracle.cg(vec32=True)):
  CG on that problem amplifies rounding, so no fp32-storage implementation
  can meet 1e-5 there.  The objective ||E x - y||^2, which is well
  conditioned, is checked at 1e-6 too.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import K_FLOOR, TOL_FP32, c64, log, rel_l2, to_dev, to_host
from paper_1807_11830_amd import sense, synth

pytestmark = pytest.mark.gpu


def _problem(w, batch=1, per_slice_maps=False, seed=synth.SEED_PHANTOM):
    imgs, maps, mask = synth.slice_inputs(w, batch, seed=seed, per_slice_maps=per_slice_maps)
    maps = c64(maps)
    y = oracle.E(imgs, maps, mask)
    y = c64(y + synth.complex_noise(y.shape) * mask[None, None, :, None])
    return imgs, maps, mask, y


def _objective(x, maps, mask, y):
    r = oracle.E(x, maps, mask) - y * mask[None, None, :, None]
    return np.array([np.vdot(r[b].ravel(), r[b].ravel()).real for b in range(r.shape[0])])


def test_cg_small64_matches_oracle():
    w = synth.SMALL_64
    imgs, maps, mask, y = _problem(w)
    xo, it, st, hist = oracle.cg(y, maps, mask, w.iters)
    with sense.Plan(to_dev(maps), mask, batch=1) as plan:
        res = plan.cg(to_dev(y), w.iters, history=True)
    err = rel_l2(to_host(res.x), xo)
    log(f"64x64 CG rel-L2 {err:.3e}, iters {res.iters}, status {res.status}")
    assert err <= TOL_FP32
    assert res.iters[0] == w.iters and res.status[0] == sense.MAXITER
    h = res.rho_hist.cpu().numpy()[0]
    assert np.allclose(h[:5], hist[0, :5], rtol=1e-5)
    assert abs(res.rho0[0] - hist[0, 0]) <= 1e-6 * hist[0, 0]


@pytest.mark.parametrize("iters", [10, 30])
def test_cg_slice256_matches_oracle(iters):
    w = synth.SLICE_256
    imgs, maps, mask, y = _problem(w)
    xo, it, st, hist = oracle.cg(y, maps, mask, iters)
    if iters <= 10:
        bar, floor = TOL_FP32, None
    else:
        floor = rel_l2(oracle.cg(y, maps, mask, iters, vec32=True)[0], xo)
        bar = K_FLOOR * floor
    with sense.Plan(to_dev(maps), mask, batch=1) as plan:
        res = plan.cg(to_dev(y), iters, history=True)
    xg = to_host(res.x)
    err = rel_l2(xg, xo)
    fo, fg = _objective(xo, maps, mask, y), _objective(xg, maps, mask, y)
    log(f"256x256 CG K={iters} rel-L2 {err:.3e} (bar {bar:.3e}, floor {floor}); "
        f"objective {fg[0]:.6e} vs {fo[0]:.6e}")
    assert err <= bar
    assert abs(fg[0] - fo[0]) <= 1e-6 * fo[0]
    # the rho history follows the oracle's (every entry the true <r, r>)
    h = res.rho_hist.cpu().numpy()[0]
    assert np.all(np.abs(h - hist[0]) <= 1e-4 * hist[0])


@pytest.mark.parametrize("G", [1, 2])
def test_cg_coil_groups(G):
    """The 64x64 / 4-coil solve with the coils split into G groups (the
    workspace holds 2; the default for so small a slice is 1) matches the
    oracle; the same G is bitwise reproducible."""
    w = synth.SMALL_64
    imgs, maps, mask, y = _problem(w)
    xo, it, st, hist = oracle.cg(y, maps, mask, w.iters)
    with sense.Plan(to_dev(maps), mask, batch=1) as plan:
        assert plan.coil_groups() == (1, 2)
        plan.set_coil_groups(G)
        r1 = plan.cg(to_dev(y), w.iters).x.clone()
        r2 = plan.cg(to_dev(y), w.iters).x
    err = rel_l2(to_host(r1), xo)
    log(f"64x64 CG G={G} rel-L2 {err:.3e}")
    assert err <= TOL_FP32
    assert torch.equal(r1, r2)


@pytest.mark.parametrize("G", [1, 2])
def test_cg_tikhonov_matches_oracle(G):
    """Regularised CG-SENSE (lambda = 0.05) on the 64x64 / 4-coil problem,
    with and without coil groups, against the oracle's CG on E^H E + lambda I;
    also the rho history and a tolerance stop."""
    w = synth.SMALL_64
    imgs, maps, mask, y = _problem(w)
    lam = 0.05
    xo, it, st, hist = oracle.cg(y, maps, mask, w.iters, lam=lam)
    xt, itt, stt, _ = oracle.cg(y, maps, mask, 50, tol=1e-3, lam=lam)
    with sense.Plan(to_dev(maps), mask, batch=1) as plan:
        plan.set_coil_groups(G)
        res = plan.cg(to_dev(y), w.iters, lam=lam, history=True)
        rt = plan.cg(to_dev(y), 50, tol=1e-3, lam=lam)
    err = rel_l2(to_host(res.x), xo)
    log(f"64x64 CG lambda={lam} G={G} rel-L2 {err:.3e}; tol stop at {rt.iters[0]} (oracle {itt[0]})")
    assert err <= TOL_FP32
    assert np.allclose(res.rho_hist.cpu().numpy()[0, :6], hist[0, :6], rtol=1e-5)
    assert rt.status[0] == sense.CONVERGED == stt[0]
    assert abs(int(rt.iters[0]) - int(itt[0])) <= 1
    if int(rt.iters[0]) == int(itt[0]):  # the same number of updates
        assert rel_l2(to_host(rt.x), xt) <= TOL_FP32


def test_cg_batch_per_slice_maps():
    w = synth.SMALL_64
    imgs, maps, mask, y = _problem(w, batch=3, per_slice_maps=True)
    xo, it, st, hist = oracle.cg(y, maps, mask, 12)
    with sense.Plan(to_dev(maps), mask, batch=3) as plan:
        res = plan.cg(to_dev(y), 12)
    assert rel_l2(to_host(res.x), xo) <= TOL_FP32
    assert list(res.iters) == [12, 12, 12]


@pytest.mark.parametrize("split", [False, True])
def test_cg_batch_mixed_stops(split):
    """A batch whose slices stop at different iterations and for different
    reasons (a tolerance reached at each slice's own iteration, zero data:
    EXACT before the first update), on the whole-solve kernel of small
    slices and on the per-iteration fused launches: per-slice iteration
    counts, statuses and iterates against the oracle."""
    w = synth.SMALL_64
    imgs, maps, mask, y = _problem(w, batch=3, per_slice_maps=True)
    y = y.copy()
    y[1] = 0
    # slice 2: scaled-down data plus noise, which converges more slowly
    y[2] *= 1e-3
    y[2] += c64(1e-4 * synth.complex_normal(y[2].shape, 71)) * mask[None, :, None]
    K, tol = 40, 2e-3  # stops at 5 and 8 iterations, 13-22% clear of tol on either side
    xo, ito, sto, _ = oracle.cg(y, maps, mask, K, tol=tol)
    assert sto[1] == oracle.EXACT and ito[1] == 0
    assert len({int(i) for i in ito}) == 3  # three different stop iterations
    with _split(sense.Plan(to_dev(maps), mask, batch=3), split) as plan:
        res = plan.cg(to_dev(y), K, tol=tol)
    log(f"mixed stops (split={split}): oracle iters {list(ito)} status {list(sto)}, "
        f"GPU {list(res.iters)} {list(res.status)}")
    assert list(res.iters) == [int(i) for i in ito]
    assert list(res.status) == [int(v) for v in sto]
    xg = to_host(res.x)
    assert np.count_nonzero(xg[1]) == 0
    for b in (0, 2):
        assert rel_l2(xg[b:b + 1], xo[b:b + 1]) <= TOL_FP32


def _split(plan, split):
    """With split, force the workspace's largest coil-group count, which
    takes the per-iteration fused launches instead of the whole-solve
    kernel of small slices."""
    if split:
        gmax = plan.coil_groups()[1]
        assert gmax > 1
        plan.set_coil_groups(gmax)
    return plan


@pytest.mark.parametrize("split", [False, True])
def test_cg_statuses(split):
    """Every stop status, on the whole-solve kernel of small slices and on
    the per-iteration fused launches."""
    n, nc = 32, 4
    maps = c64(synth.coil_maps2d(n, nc))
    mask = synth.mask_regular(n, 2, 4)
    full = np.ones(n, np.uint8)
    x_true = synth.phantom2d(n, seed=3)[None]
    # zero data: EXACT before the first update
    with _split(sense.Plan(to_dev(maps), mask), split) as plan:
        res = plan.cg(torch.zeros((1, nc, n, n), dtype=torch.complex64, device="cuda:0"), 5)
        assert res.status[0] == sense.EXACT and res.iters[0] == 0
        assert torch.count_nonzero(res.x) == 0
        # tolerance: same stop iteration as the oracle
        y = c64(oracle.E(x_true, maps, mask))
        xo, ito, sto, _ = oracle.cg(y, maps, mask, 50, tol=1e-3)
        res = plan.cg(to_dev(y), 50, tol=1e-3)
        assert sto[0] == oracle.CONVERGED
        assert res.status[0] == sense.CONVERGED and res.iters[0] == ito[0]
        # NaN input
        yn = y.copy()
        yn[0, 0, 0, 0] = np.nan
        res = plan.cg(to_dev(yn), 5)
        assert res.status[0] == sense.NONFINITE and res.iters[0] == 0
    # A = 0 (lambda = -1 with full sampling and sum |S|^2 = 1): breakdown
    with _split(sense.Plan(to_dev(maps), full), split) as plan:
        y = c64(oracle.E(x_true, maps, full))
        res = plan.cg(to_dev(y), 5, lam=-1.0)
        assert res.status[0] == sense.BREAKDOWN and res.iters[0] == 0
        # full sampling: one iteration recovers x (alpha = 1)
        res = plan.cg(to_dev(y), 1)
        assert rel_l2(to_host(res.x), x_true) <= TOL_FP32


def test_cg_zero_iterations_and_repeat():
    w = synth.SMALL_64
    imgs, maps, mask, y = _problem(w)
    with sense.Plan(to_dev(maps), mask) as plan:
        res = plan.cg(to_dev(y), 0)
        assert res.iters[0] == 0 and res.status[0] == sense.MAXITER
        assert torch.count_nonzero(res.x) == 0
        a = plan.cg(to_dev(y), 7).x.clone()
        b = plan.cg(to_dev(y), 7).x
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_cg_full_size_batch_sampled():
    """The benchmark's launch configuration: 160 slices of 256x256, 12 coils,
    per-slice maps, 30 iterations; sampled slices against the oracle."""
    w = synth.SLICE_256
    B = 160
    imgs, maps, mask = synth.slice_inputs(w, B, per_slice_maps=True)
    maps = c64(maps)
    picks = [0, 97, 159]
    # k-space of the checked slices from the oracle's forward model; the
    # other slices get masked random data (cheap, and checked only for the
    # iteration count)
    y = 0.05 * synth.complex_normal((B, w.ncoils, w.n, w.n), 999) * mask[None, None, :, None]
    for b in picks:
        yb = oracle.E(imgs[b:b + 1], maps[b], mask)
        y[b] = (yb + synth.complex_noise(yb.shape, seed=1000 + b) * mask[None, None, :, None])[0]
    y = c64(y)
    with sense.Plan(to_dev(maps), mask, batch=B) as plan:
        res = plan.cg(to_dev(y), w.iters)
        pd = to_dev(imgs)
        q = plan.EHE(pd)
        torch.cuda.synchronize()
    assert list(np.unique(res.iters)) == [w.iters]
    xg = to_host(res.x)
    qg = to_host(q)
    for b in picks:
        qo = oracle.A(imgs[b:b + 1], maps[b], mask)
        assert rel_l2(qg[b:b + 1], qo) <= TOL_FP32
        xo, _, _, _ = oracle.cg(y[b:b + 1], maps[b], mask, w.iters)
        floor = rel_l2(oracle.cg(y[b:b + 1], maps[b], mask, w.iters, vec32=True)[0], xo)
        err = rel_l2(xg[b:b + 1], xo)
        log(f"slice {b}: CG rel-L2 {err:.3e}, complex64 floor {floor:.3e} (bar {K_FLOOR * floor:.3e})")
        assert err <= K_FLOOR * floor


def test_cg_full_size_batch_bf16_maps():
    """The benchmark's launch with BF16 maps (`--maps-storage bf16`: the
    streaming instantiation with the maps staged through LDS): sampled
    slices against the oracle on the same quantised maps (K_FLOOR times the
    complex64 floor) and on the unquantised ones (the 1e-2 bar)."""
    from gpu_common import quantise
    w = synth.SLICE_256
    B = 160
    imgs, maps, mask = synth.slice_inputs(w, B, per_slice_maps=True)
    maps = c64(maps)
    picks = [0, 159]
    y = 0.05 * synth.complex_normal((B, w.ncoils, w.n, w.n), 998) * mask[None, None, :, None]
    for b in picks:
        yb = oracle.E(imgs[b:b + 1], maps[b], mask)
        y[b] = (yb + synth.complex_noise(yb.shape, seed=1000 + b) * mask[None, None, :, None])[0]
    y = c64(y)
    with sense.Plan(to_dev(maps), mask, batch=B, maps_storage="bf16") as plan:
        assert plan.coil_groups()[0] == 1
        res = plan.cg(to_dev(y), w.iters)
        torch.cuda.synchronize()
    assert list(np.unique(res.iters)) == [w.iters]
    xg = to_host(res.x)
    for b in picks:
        mq = quantise(maps[b], "bf16")
        xq, _, _, _ = oracle.cg(y[b:b + 1], mq, mask, w.iters)
        floor = rel_l2(oracle.cg(y[b:b + 1], mq, mask, w.iters, vec32=True)[0], xq)
        xo, _, _, _ = oracle.cg(y[b:b + 1], maps[b], mask, w.iters)
        e_arith, e_total = rel_l2(xg[b:b + 1], xq), rel_l2(xg[b:b + 1], xo)
        log(f"slice {b} bf16 maps: vs oracle on quantised maps {e_arith:.3e} (bar {K_FLOOR * floor:.3e}), "
            f"vs oracle {e_total:.3e}")
        assert e_arith <= K_FLOOR * floor
        assert e_total <= 1e-2


def test_cg_graph_replay_matches_eager():
    """Whole-solve graph replays, interleaved with eager work and
    synchronisations, reproduce the eager solve bitwise every time; changed
    arguments re-capture."""
    w = synth.SMALL_64
    imgs, maps, mask, y = _problem(w, batch=2, per_slice_maps=True)
    with sense.Plan(to_dev(maps), mask, batch=2) as plan:
        yd = to_dev(y)
        plan.set_graphs(False)
        ref = plan.cg(yd, 15).x.clone()
        ref_tol = plan.cg(yd, 15, tol=1e-3).x.clone()
        plan.set_graphs(True)
        out = torch.empty_like(ref)
        p = to_dev(imgs)
        for rep in range(4):
            res = plan.cg(yd, 15, out=out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), rep
            assert list(res.iters) == [15, 15]
            plan.EHE(p)  # eager work between replays
            (p * 2.0).sum().item()
            torch.cuda.synchronize()
        res = plan.cg(yd, 15, tol=1e-3, out=out)
        assert torch.equal(out, ref_tol)
        res = plan.cg(yd, 15, out=out)
        assert torch.equal(out, ref)


# Widths below 64 leave part of the 64-column workgroup idle (ragged tile);
# CG needs a supported readout length for E^H y.
SMALL_CASES = [  # ny, nx, coils, batch, per-slice maps, storage
    (8, 8, 2, 2, True, "c64"),
    (16, 48, 3, 1, False, "c64"),
    (32, 64, 4, 3, True, "c64"),
    (48, 16, 3, 1, False, "c64"),
    (64, 64, 8, 2, False, "bf16"),
    (64, 32, 4, 1, True, "c64"),
    (64, 48, 6, 2, True, "c64"),   # maps re-read per iteration, block layout
    (32, 16, 4, 2, False, "fp16"),  # maps held in registers, 16-bit storage
    (32, 48, 7, 2, True, "c64"),    # 7 of 8 register coil slots
    (48, 32, 2, 1, True, "bf16"),   # 48 rows: two coils in registers
]


@pytest.mark.parametrize("ny,nx,nc,b,per,st", SMALL_CASES)
def test_small_whole_solve_matches_oracle(ny, nx, nc, b, per, st):
    """Slices of at most 64 x 64 run the whole solve in one workgroup per
    batch element (every supported length, ragged widths, batches, 16-bit
    maps): x, the iteration count, the status and the rho history against
    the oracle's CG on the same (quantised) inputs."""
    from gpu_common import quantise
    maps = c64(0.5 * synth.complex_normal((b, nc, ny, nx) if per else (nc, ny, nx), ny + nx))
    mask = synth.mask_variable_density(ny, 2.0, max(2, ny // 8), seed=ny)
    xt = c64(synth.complex_normal((b, ny, nx), 7))
    mq = quantise(maps, st)
    y = np.concatenate([oracle.E(xt[i:i + 1], mq[i] if per else mq, mask) for i in range(b)])
    y = c64(y + 1e-3 * synth.complex_normal(y.shape, 8) * mask[None, None, :, None])
    K = 12
    xo = np.empty_like(xt)
    ho = np.empty((b, K + 1))
    for i in range(b):
        xo[i:i + 1], _, _, ho[i:i + 1] = oracle.cg(y[i:i + 1], mq[i] if per else mq, mask, K)
    with sense.Plan(to_dev(maps), mask, batch=b, maps_storage=st) as plan:
        assert plan.coil_groups()[0] == 1
        res = plan.cg(to_dev(y), K, history=True)
    err = rel_l2(to_host(res.x), xo)
    log(f"small {ny}x{nx} C={nc} B={b} {st}: rel-L2 {err:.3e}")
    assert err <= TOL_FP32
    assert list(res.iters) == [K] * b and list(res.status) == [sense.MAXITER] * b
    assert np.allclose(res.rho_hist.cpu().numpy(), ho, rtol=1e-4)
    assert np.allclose(res.rho0, ho[:, 0], rtol=1e-5)


def test_small_whole_solve_equals_graph_replay_and_engine():
    """A small solve gives the same bits with graphs on (where it still
    launches eagerly) and off, and a small request in the serving engine
    (run whole at admission) equals the plain solve bitwise."""
    w = synth.SMALL_64
    imgs, maps, mask, y = _problem(w)
    with sense.Plan(to_dev(maps), mask) as plan, sense.Plan(to_dev(maps), mask) as pe:
        yd = to_dev(y)
        plan.set_graphs(False)
        ref = plan.cg(yd, w.iters).x.clone()
        plan.set_graphs(True)
        for _ in range(3):
            assert torch.equal(plan.cg(yd, w.iters).x, ref)
        x = torch.empty_like(ref)
        with sense.Engine(budget_bytes=1 << 30, max_slots=2) as eng:
            assert eng.admit(pe, yd, x, w.iters) == 0
            done = []
            while not done:
                eng.step()
                done = eng.poll()
        torch.cuda.synchronize()
        assert torch.equal(x, ref)
