"""The allocation-free CG-SENSE entry point (sense_cg_solve_static) against
the plan-based sense_cg_solve, through the C ABI.

Two calls in a row on the same GPU, the second with a smaller problem, so
the second runs on a static workspace that still holds the first call's
values.  Each result is compared with sense_cg_solve on a plan with the
same descriptor, maps and mask: relative L2 per batch element within the
fp32 bar (1e-5), and with the FP64 oracle at the same bar for the small
20-iteration solve.  Both paths run the same kernels on the same tables,
so the results are also expected to agree bitwise; the test reports it.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_common import DEV, TOL_FP32, c64, log, rel_l2, to_dev, to_host
from paper_1807_11830_amd import sense, synth

pytestmark = pytest.mark.gpu


def _case(w, batch, seed):
    imgs, maps, mask = synth.slice_inputs(w, batch, seed=seed)
    maps = c64(maps)
    y = oracle.E(imgs, maps, mask)
    y = c64(y + synth.complex_noise(y.shape) * mask[None, None, :, None])
    return maps, mask, y


def _solve_both(maps, mask, y, iters, batch, lam=0.0):
    dmaps, dy = to_dev(maps), to_dev(y)
    ny, nx = maps.shape[-2:]
    x_static = torch.empty((batch, ny, nx), dtype=torch.complex64, device=DEV)
    info = torch.zeros(24 * batch, dtype=torch.uint8, device=DEV)
    hist = torch.zeros((batch, iters + 1), dtype=torch.float64, device=DEV)
    sense.cg_solve_static(dmaps, mask, dy, x_static, iters, lam=lam, batch=batch, info=info, rho_hist=hist)
    torch.cuda.synchronize()
    with sense.Plan(dmaps, mask, batch=batch) as plan:
        res = plan.cg(dy, iters, lam=lam, history=True)
    raw = info.cpu().numpy().tobytes()
    infos = (sense.CgInfo * batch).from_buffer_copy(raw)
    return to_host(x_static), hist.cpu().numpy(), infos, res


@pytest.mark.parametrize("first,second", [(("slice256", 2), ("small64", 1))])
def test_static_solve_matches_plan_twice(first, second):
    cases = {"slice256": (synth.SLICE_256, 10), "small64": (synth.SMALL_64, synth.SMALL_64.iters)}
    for n, (name, batch) in enumerate((first, second)):
        w, iters = cases[name]
        maps, mask, y = _case(w, batch, seed=synth.SEED_PHANTOM + 5 * n)
        log(f"static solve call {n}: {name} batch {batch}, {iters} iterations")
        x_static, hist, infos, res = _solve_both(maps, mask, y, iters, batch)
        x_plan = to_host(res.x)
        err = rel_l2(x_static, x_plan)
        same = bool(np.array_equal(x_static, x_plan))
        log(f"  static vs plan rel-L2 {err:.3e} (bitwise equal: {same})")
        assert err <= TOL_FP32
        for b in range(batch):
            assert infos[b].iters_run == res.iters[b] == iters
            assert infos[b].status == res.status[b] == sense.MAXITER
            assert abs(infos[b].rho0 - res.rho0[b]) <= 1e-6 * res.rho0[b]
        assert np.allclose(hist, res.rho_hist.cpu().numpy(), rtol=1e-5, atol=0.0)
        if name == "small64":
            xo, _, _, _ = oracle.cg(y, maps, mask, iters)
            err_o = rel_l2(x_static, xo)
            log(f"  static vs FP64 oracle rel-L2 {err_o:.3e}")
            assert err_o <= TOL_FP32


def test_static_solve_compact_kspace_and_bf16():
    """Compact k-space (the sampled lines only) in BF16 storage, with BF16
    maps, on the small-slice path: the static solve against the plan with
    the same descriptor, bitwise."""
    w = synth.SMALL_64
    maps, mask, y = _case(w, 2, seed=synth.SEED_PHANTOM + 11)
    rows = np.flatnonzero(mask)
    mq = sense.to_storage(to_dev(maps), "bf16")
    yq = sense.to_storage(to_dev(y[:, :, rows]).contiguous(), "bf16")
    x_static = torch.empty((2, w.n, w.n), dtype=torch.complex64, device=DEV)
    sense.cg_solve_static(mq, mask, yq, x_static, w.iters, batch=2, maps_storage="bf16",
                          kspace_storage="bf16", kspace_compact=True)
    torch.cuda.synchronize()
    with sense.Plan(to_dev(maps), mask, batch=2, maps_storage="bf16", kspace_storage="bf16",
                    kspace_compact=True) as plan:
        x_plan = plan.cg(yq, w.iters).x
        torch.cuda.synchronize()
    log(f"static compact BF16 vs plan: bitwise {torch.equal(x_static, x_plan)}")
    assert torch.equal(x_static, x_plan)


def test_static_solve_rejects_oversize():
    # 384^2 x 32 coils x 8 slices needs far more than the 64 MiB workspace
    maps = torch.zeros((8, 32, 384, 384), dtype=torch.complex64, device=DEV)
    y = torch.zeros((8, 32, 384, 384), dtype=torch.complex64, device=DEV)
    x = torch.empty((8, 384, 384), dtype=torch.complex64, device=DEV)
    mask = np.ones(384, np.uint8)
    with pytest.raises(sense.SenseError) as ei:
        sense.cg_solve_static(maps, mask, y, x, 5, batch=8)
    assert ei.value.code == 2 and "bytes of workspace" in str(ei.value)
