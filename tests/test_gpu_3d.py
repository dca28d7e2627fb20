"""3D operators, 3D CG and the autograd wrapper on the GPU, against the FP64
oracle, through the C ABI.  Relative L2 <= 1e-5 per batch element for
single applies and small solves; finite differences of ||E x - y||^2 at
1e-3 (fp32 forward evaluations)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import TOL_FP32, c64, log, rel_l2, to_dev, to_host
from paper_1807_11830_amd import sense, synth
from paper_1807_11830_amd.autograd import sense_E

pytestmark = pytest.mark.gpu


def _case3d(nz, ny, nx, nc, b, per, seed=0, accel=3.0):
    maps_shape = (b, nc, nz, ny, nx) if per else (nc, nz, ny, nx)
    maps = c64(0.5 * synth.complex_normal(maps_shape, seed + 1))
    x = c64(synth.complex_normal((b, nz, ny, nx), seed + 2))
    cy, cz = max(2, ny // 8), max(2, nz // 8)
    mask = synth.mask_variable_density_2d(ny, nz, accel, (cy, cz), seed=seed + 3)
    return maps, x, mask


CASES = [  # nz, ny, nx, ncoils, batch, per_batch_maps
    (8, 16, 16, 2, 1, False),
    (16, 32, 48, 3, 2, True),
    (8, 64, 64, 4, 1, False),
    (32, 16, 80, 2, 1, False),
]


@pytest.mark.parametrize("nz,ny,nx,nc,b,per", CASES)
def test_3d_operators_match_oracle(nz, ny, nx, nc, b, per):
    log(f"3D nz={nz} ny={ny} nx={nx} C={nc} B={b}")
    maps, x, mask = _case3d(nz, ny, nx, nc, b, per, seed=nz + ny + nx)
    yin = c64(synth.complex_normal((b, nc, nz, ny, nx), 5))
    with sense.Plan(to_dev(maps), mask, batch=b) as plan:
        assert plan.ndim == 3
        y = to_host(plan.E(to_dev(x)))
        xh = to_host(plan.EH(to_dev(yin)))
        q = to_host(plan.EHE(to_dev(x), lam=0.25))
    e1 = rel_l2(y, oracle.E(x, maps, mask, ndim=3))
    e2 = rel_l2(xh, oracle.EH(yin, maps, mask, ndim=3))
    e3 = rel_l2(q, oracle.A(x, maps, mask, lam=0.25, ndim=3))
    log(f"  E {e1:.3e} EH {e2:.3e} EHE {e3:.3e}")
    assert max(e1, e2, e3) <= TOL_FP32
    m = mask.astype(bool)
    assert np.all(y[:, :, ~m, :] == 0)


def test_3d_rss_matches_oracle():
    """Zero-filled RSS of a volume: x rows, z pass, y combine."""
    maps, _, mask = _case3d(16, 32, 48, 3, 2, False, seed=21)
    y = c64(synth.complex_normal((2, 3, 16, 32, 48), 22))
    ref = oracle.rss(y * mask[None, None, :, :, None], ndim=3)
    with sense.Plan(to_dev(maps), mask, batch=2) as plan:
        got = plan.rss(to_dev(y)).cpu().numpy().astype(np.float64)
    err = rel_l2(got, ref)
    log(f"3D RSS rel-L2 {err:.3e}")
    assert err <= TOL_FP32


def test_3d_compact_kspace_equals_full_grid():
    maps, x, mask = _case3d(16, 32, 48, 3, 1, False, seed=41)
    lines = np.flatnonzero(mask.ravel())
    with sense.Plan(to_dev(maps), mask) as pf, sense.Plan(to_dev(maps), mask, kspace_compact=True) as pc:
        assert pc.kspace_shape == (1, 3, len(lines), 48)
        yf = pf.E(to_dev(x))
        yc = pc.E(to_dev(x))
        assert torch.equal(yc, yf.reshape(1, 3, 16 * 32, 48)[:, :, lines].contiguous())
        assert torch.equal(pc.EH(yc), pf.EH(yf))
        assert torch.equal(pc.rss(yc), pf.rss(yf))
        assert torch.equal(pc.cg(yc, 4).x, pf.cg(yf, 4).x)


def test_3d_ehe_ragged_readout():
    maps, x, mask = _case3d(8, 32, 40, 3, 2, False, seed=9)
    with sense.Plan(to_dev(maps), mask, batch=2) as plan:
        q = to_host(plan.EHE(to_dev(x)))
    assert rel_l2(q, oracle.A(x, maps, mask, ndim=3)) <= TOL_FP32


def test_3d_adjoint_identity():
    maps, x, mask = _case3d(16, 32, 32, 3, 1, False, seed=4)
    yin = c64(synth.complex_normal((1, 3, 16, 32, 32), 6))
    with sense.Plan(to_dev(maps), mask) as plan:
        ex = to_host(plan.E(to_dev(x)))
        ehy = to_host(plan.EH(to_dev(yin)))
    lhs = np.vdot(ex.ravel(), (yin * mask[None, None, :, :, None]).ravel())
    rhs = np.vdot(x.ravel(), ehy.ravel())
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_3d_cg_matches_oracle():
    nz, ny, nx, nc = 16, 32, 32, 4
    maps = c64(synth.coil_maps3d(nx, ny, nz, nc))
    mask = synth.mask_variable_density_2d(ny, nz, 3.0, (8, 4))
    xt = synth.phantom3d(nx, ny, nz)[None]
    y = oracle.E(xt, maps, mask, ndim=3)
    y = c64(y + synth.complex_noise(y.shape) * mask[None, None, :, :, None])
    xo, it, st, hist = oracle.cg(y, maps, mask, 8, ndim=3)
    with sense.Plan(to_dev(maps), mask) as plan:
        res = plan.cg(to_dev(y), 8, history=True)
    err = rel_l2(to_host(res.x), xo)
    log(f"3D CG rel-L2 {err:.3e}")
    assert err <= TOL_FP32
    assert res.iters[0] == 8
    assert np.allclose(res.rho_hist.cpu().numpy()[0, :4], hist[0, :4], rtol=1e-5)


def test_3d_cg_tolerance_stop_and_batch():
    """3D CG with a relative tolerance on a batch of two problems (per-slice
    maps): the iteration count and status of each element, its rho history
    and x against the oracle's loop; and the same problem with a zero
    right-hand side in the second element stops with EXACT at iteration 0."""
    nz, ny, nx, nc, B = 8, 32, 16, 4, 2
    base = synth.coil_maps3d(nx, ny, nz, nc)
    maps = c64(np.stack([base * np.exp(0.3j * b * np.arange(1, nc + 1))[:, None, None, None] for b in range(B)]))
    mask = synth.mask_variable_density_2d(ny, nz, 2.5, (8, 4))
    xt = np.concatenate([synth.phantom3d(nx, ny, nz, seed=20 + b)[None] for b in range(B)])
    y = np.concatenate([oracle.E(xt[b:b + 1], maps[b], mask, ndim=3) for b in range(B)])
    y = c64(y + synth.complex_noise(y.shape) * mask[None, None, :, :, None])
    tol, K = 3.4e-3, 40  # both elements cross it with a margin of at least 10%
    with sense.Plan(to_dev(maps), mask, batch=B) as plan:
        res = plan.cg(to_dev(y), K, tol=tol, history=True)
        for b in range(B):
            xo, it, st, hist = oracle.cg(y[b:b + 1], maps[b], mask, K, tol=tol, ndim=3)
            err = rel_l2(to_host(res.x[b:b + 1]), xo)
            log(f"3D CG tol: element {b} iters {res.iters[b]} (oracle {it[0]}), status {res.status[b]}, rel-L2 {err:.3e}")
            assert res.iters[b] == it[0] < K and res.status[b] == st[0] == sense.CONVERGED
            n = int(it[0]) + 1
            assert np.allclose(res.rho_hist.cpu().numpy()[b, :n], hist[0, :n], rtol=1e-4)
            assert err <= 1e-4
        y0 = y.copy()
        y0[1] = 0
        res0 = plan.cg(to_dev(y0), K, tol=tol)
    assert res0.status[1] == sense.EXACT and res0.iters[1] == 0
    assert not np.any(to_host(res0.x[1:2]))
    assert res0.iters[0] == res.iters[0] and res0.status[0] == sense.CONVERGED


def _loss_and_grad(plan, x, y):
    xt = to_dev(x).requires_grad_(True)
    r = sense_E(xt, plan) - to_dev(y)
    loss = (r.real.double() ** 2 + r.imag.double() ** 2).sum()
    loss.backward()
    return float(loss.detach()), to_host(xt.grad)


@pytest.mark.parametrize("shape", [(16, 16, 8), (64, 64, 1)])
def test_autograd_gradient(shape):
    """x.grad of ||E x - y||^2 equals the oracle's 2 E^H (E x - y) and
    central differences of the GPU loss.  (16, 16, 8) with 2 coils is the
    small 3D instance of the differentiation workload."""
    nx, ny, nz = shape
    nc = 2
    ndim = 3 if nz > 1 else 2
    grid = (nz, ny, nx) if ndim == 3 else (ny, nx)
    maps = c64(0.5 * synth.complex_normal((nc,) + grid, 30))
    if ndim == 3:
        mask = synth.mask_variable_density_2d(ny, nz, 6.0, (4, 4), seed=31)
    else:
        mask = synth.mask_regular(ny, 2, 8)
    x = c64(synth.complex_normal((1,) + grid, 32))
    y = c64(synth.complex_normal((1, nc) + grid, 33))
    bshape = (1, 1) + mask.shape + ((1,) if True else ())
    y = c64(y * mask.reshape(bshape))
    with sense.Plan(to_dev(maps), mask, ndim=ndim) as plan:
        loss, g = _loss_and_grad(plan, x, y)
        r = oracle.E(x, maps, mask, ndim=ndim) - y
        g_ref = 2.0 * oracle.EH(r, maps, mask, ndim=ndim)
        assert rel_l2(g, g_ref) <= TOL_FP32
        for s in range(3):
            d = c64(synth.complex_normal(x.shape, 40 + s))
            eps = 1e-2
            lp, _ = _loss_and_grad(plan, x + eps * d, y)
            lm, _ = _loss_and_grad(plan, x - eps * d, y)
            fd = (lp - lm) / (2 * eps)
            an = float(np.vdot(g.ravel(), d.ravel()).real)
            log(f"FD {fd:.6e} analytic {an:.6e}")
            assert abs(fd - an) <= 1e-3 * abs(an)


def test_3d_full_transform_lengths_match_oracle():
    """The differentiation workload's transform lengths (ny = 256, nz = 128,
    (ky, kz) mask R = 6 with a 32 x 32 centre) on a narrow readout (nx = 16)
    and 2 coils: E, E^H, E^H E and a 4-iteration CG against the oracle, so
    the 256-point y passes and the 128-point z passes that the full volume
    runs are all compared."""
    nz, ny, nx, nc = 128, 256, 16, 2
    maps = c64(synth.coil_maps3d(nx, ny, nz, nc))
    mask = synth.mask_variable_density_2d(ny, nz, 6.0, (32, 32))
    xt = c64(synth.phantom3d(nx, ny, nz)[None])
    yin = c64(synth.complex_normal((1, nc, nz, ny, nx), 51))
    log(f"3D full lengths nz={nz} ny={ny} nx={nx} C={nc}")
    with sense.Plan(to_dev(maps), mask) as plan:
        y = to_host(plan.E(to_dev(xt)))
        xh = to_host(plan.EH(to_dev(yin)))
        q = to_host(plan.EHE(to_dev(xt)))
        yo = oracle.E(xt, maps, mask, ndim=3)
        e1 = rel_l2(y, yo)
        e2 = rel_l2(xh, oracle.EH(yin, maps, mask, ndim=3))
        e3 = rel_l2(q, oracle.A(xt, maps, mask, ndim=3))
        log(f"  E {e1:.3e} EH {e2:.3e} EHE {e3:.3e}")
        assert max(e1, e2, e3) <= TOL_FP32
        assert np.all(y[:, :, mask == 0, :] == 0)
        yd = c64(yo + synth.complex_noise(yo.shape) * mask[None, None, :, :, None])
        xo, it, st, hist = oracle.cg(yd, maps, mask, 4, ndim=3)
        res = plan.cg(to_dev(yd), 4, history=True)
    err = rel_l2(to_host(res.x), xo)
    log(f"  CG (4 iterations) rel-L2 {err:.3e}")
    assert err <= TOL_FP32 and res.iters[0] == 4
    assert np.allclose(res.rho_hist.cpu().numpy()[0], hist[0], rtol=1e-5)


def test_3d_full_size_sampled_coil_and_composition():
    """The 3D workload at its full size (256 x 256 x 128, 16 coils, (ky, kz)
    mask R = 6 with a 32 x 32 centre: the launches the autograd benchmark
    times).  Sampled outputs against the oracle: coil 0 of E x (the oracle's
    forward model with that coil's map alone) and E^H of k-space that is
    zero outside coil 0.  The normal operator against E^H(E p) and the
    adjoint identity, on the GPU: properties that hold at any size."""
    nx, ny, nz, nc = 256, 256, 128, 16
    maps = c64(synth.coil_maps3d(nx, ny, nz, nc))
    mask = synth.mask_variable_density_2d(ny, nz, 6.0, (32, 32))
    xt = c64(synth.phantom3d(nx, ny, nz)[None])
    y0 = np.zeros((1, nc, nz, ny, nx), np.complex64)
    y0[:, 0] = c64(synth.complex_normal((1, nz, ny, nx), 61))
    log(f"3D full size {nx}x{ny}x{nz}, C={nc}")
    with sense.Plan(to_dev(maps), mask) as plan:
        xd = to_dev(xt)
        yd = plan.E(xd)
        ye = to_host(yd[:, 0:1])
        xh = to_host(plan.EH(to_dev(y0)))
        q = plan.EHE(xd)
        qc = plan.EH(yd)
        yr = to_dev(c64(synth.complex_normal((1, nc, nz, ny, nx), 62)))
        lhs = torch.vdot(yd.flatten().to(torch.complex128), yr.flatten().to(torch.complex128))
        rhs = torch.vdot(xd.flatten().to(torch.complex128), plan.EH(yr).flatten().to(torch.complex128))
        e_comp = (torch.linalg.vector_norm(q - qc) / torch.linalg.vector_norm(qc)).item()
        e_adj = (abs(lhs - rhs) / (torch.linalg.vector_norm(yd) * torch.linalg.vector_norm(yr))).item()
        del yd, q, qc, yr
    e1 = rel_l2(ye, oracle.E(xt, maps[0:1], mask, ndim=3))
    e2 = rel_l2(xh, oracle.EH(y0[:, 0:1], maps[0:1], mask, ndim=3))
    log(f"  E coil 0 {e1:.3e}, EH coil 0 {e2:.3e}, EHE vs EH(E) {e_comp:.3e}, adjoint {e_adj:.3e}")
    assert max(e1, e2, e_comp) <= TOL_FP32
    assert e_adj <= 1e-6
