"""Serving engine on the GPU: each request's result is bitwise the same
solved alone (Plan.cg) and in a continuously batched mix of sizes, coil
counts and accelerations; budget and slot admission; plans in a slot are
locked; admission is ordered after the caller's stream; mixed requests of
different sizes and coil counts, each with its own seeded inputs, against
the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import TOL_FP32, log, rel_l2, to_host
from paper_1807_11830_amd import sense
from paper_1807_11830_amd.serving import (EngineExecutor, InputBank, Request, Scheduler, SerialExecutor,
                                          make_requests)

pytestmark = pytest.mark.gpu

CLASSES = [(128, 8, 2), (192, 16, 3), (256, 8, 4), (128, 8, 2), (320, 16, 2), (192, 32, 4), (256, 16, 3)]


def _alone(bank, r):
    maps, y = bank.inputs(r)
    with sense.Plan(maps, bank.mask(r.n, r.accel)) as p:
        res = p.cg(y, r.iters)
        return res.x.clone(), res.iters[0], res.status[0]


def test_alone_equals_mixed_bitwise():
    bank = InputBank()
    reqs = [Request(i, 0.0005 * i, n, c, a, 12) for i, (n, c, a) in enumerate(CLASSES)]
    bank.prepare(reqs)
    alone = {r.id: _alone(bank, r) for r in reqs}
    ex = EngineExecutor(bank, budget_bytes=8 << 30, max_slots=8)
    st = Scheduler(ex).run(reqs)
    ex.close()
    log(f"mixed run: max in flight {st.max_inflight}, steps {st.steps}")
    assert st.max_inflight >= 2
    for r in reqs:
        assert torch.equal(r.result, alone[r.id][0]), r
    # serial executor (plain path) gives the same results too
    reqs2 = [Request(i, 0.0, n, c, a, 12) for i, (n, c, a) in enumerate(CLASSES)]
    ex2 = SerialExecutor(bank)
    Scheduler(ex2).run(reqs2)
    ex2.close()
    for r in reqs2:
        assert torch.equal(r.result, alone[r.id][0])


def test_large_group_uses_device_table_bitwise():
    """20 same-size requests in flight: one group larger than a kernel-argument
    table, so the step reads a device copy of the table; results are still
    bitwise those of the plain solve."""
    bank = InputBank()
    reqs = [Request(i, 0.0, 128, 8, 2 + i % 3, 10) for i in range(20)]
    bank.prepare(reqs)
    alone = {r.id: _alone(bank, r) for r in reqs}
    ex = EngineExecutor(bank, budget_bytes=8 << 30, max_slots=32)
    st = Scheduler(ex).run(reqs)
    ex.close()
    log(f"large group: max in flight {st.max_inflight}")
    assert st.max_inflight > 16
    for r in reqs:
        assert torch.equal(r.result, alone[r.id][0]), r


def test_mixed_storage_groups_bitwise():
    """Plans with complex64 and BF16 maps of the same size form separate
    groups in a step; each result is bitwise its plain solve."""
    bank = InputBank()
    reqs = [Request(i, 0.0, 192, 8, 3, 8) for i in range(6)]
    bank.prepare(reqs)
    maps, mask = bank.coil_maps(192, 8), bank.mask(192, 3)
    y = bank.kspace(192, 8, 3)
    plans = [sense.Plan(maps, mask, maps_storage="bf16" if i % 2 else "c64") for i in range(6)]
    outs = [torch.empty((1, 192, 192), dtype=torch.complex64, device="cuda:0") for _ in range(6)]
    with sense.Engine(budget_bytes=1 << 32, max_slots=8) as eng:
        for i, p in enumerate(plans):
            assert eng.admit(p, y, outs[i], 8) == i
        done = []
        while len(done) < 6:
            eng.step()
            done += eng.poll()
    for i, p in enumerate(plans):
        ref = p.cg(y, 8).x
        assert torch.equal(outs[i], ref), i
        p.close()
    assert not torch.equal(outs[0], outs[1])  # the storages really differ


def test_shared_lanes_and_device_tables_bitwise():
    """More group keys than the engine has lanes, two of them larger than a
    kernel-argument table and sharing a lane (both read their rows of that
    lane's device table in the same step); every result is bitwise its
    plain solve."""
    bank = InputBank()
    spec = [(128, "c64")] * 17 + [(128, "bf16"), (192, "c64"), (192, "bf16")] + [(256, "c64")] * 17
    reqs = [Request(i, 0.0, n, 8, 3, 6) for i, (n, _) in enumerate(spec)]
    bank.prepare(reqs)
    plans, ys, outs = [], [], []
    for (n, st), r in zip(spec, reqs):
        plans.append(sense.Plan(bank.coil_maps(n, 8), bank.mask(n, 3), maps_storage=st))
        ys.append(bank.kspace(n, 8, 3))
        outs.append(torch.empty((1, n, n), dtype=torch.complex64, device="cuda:0"))
    with sense.Engine(budget_bytes=1 << 34, max_slots=48) as eng:
        for i, p in enumerate(plans):
            assert eng.admit(p, ys[i], outs[i], 6) == i
        done = []
        while len(done) < len(plans):
            eng.step()
            done += eng.poll()
    for i, p in enumerate(plans):
        ref = p.cg(ys[i], 6).x
        assert torch.equal(outs[i], ref), (i, spec[i])
        p.close()


def test_mixed_requests_match_oracle():
    """A continuously batched stream of seeded requests (every request with
    its own maps, image and noise); three of them with different sizes and
    coil counts are checked against the oracle's CG, and every request is
    bitwise its plain solve."""
    bank = InputBank()
    reqs = make_requests(14, rate=4000.0, iters=10, sizes=(128, 192, 256), coils=(8, 16), accels=(2, 3, 4))
    bank.prepare(reqs)
    # distinct inputs per request: no two requests share a maps or k-space buffer
    ptrs = {bank.inputs(r)[0].data_ptr() for r in reqs} | {bank.inputs(r)[1].data_ptr() for r in reqs}
    assert len(ptrs) == 2 * len(reqs)
    alone = {r.id: _alone(bank, r)[0] for r in reqs}
    ex = EngineExecutor(bank, budget_bytes=4 << 30, max_slots=8)
    st = Scheduler(ex).run(reqs)
    ex.close()
    assert st.max_inflight >= 2
    for r in reqs:
        assert torch.equal(r.result, alone[r.id]), r
    picks, seen = [], set()
    for r in reversed(reqs):
        if (r.n, r.ncoils) not in seen:
            seen.add((r.n, r.ncoils))
            picks.append(r)
    picks = picks[:3]
    assert len({p.n for p in picks}) >= 2 and len({p.ncoils for p in picks}) >= 2, picks
    for r in picks:
        maps, y = bank.inputs(r)
        xo, _, _, _ = oracle.cg(to_host(y), maps.cpu().numpy().astype(np.complex128), bank.mask(r.n, r.accel),
                                r.iters)
        err = rel_l2(to_host(r.result), xo)
        log(f"request {r.id} ({r.n}, {r.ncoils} coils, R{r.accel}) vs oracle {err:.3e}")
        assert err <= TOL_FP32


def test_engine_admission_limits():
    bank = InputBank()
    r = Request(0, 0.0, 128, 8, 2, 5)
    bank.prepare([r])
    (maps, y), mask = bank.inputs(r), bank.mask(128, 2)
    with sense.Engine(budget_bytes=1000, max_slots=2) as eng, sense.Plan(maps, mask) as p1, \
            sense.Plan(maps, mask) as p2, sense.Plan(maps, mask) as p3:
        x1, x2, x3 = (torch.empty((1, 128, 128), dtype=torch.complex64, device="cuda:0") for _ in range(3))
        assert eng.admit(p1, y, x1, 5, footprint=2000) is None  # over budget
        assert eng.admit(p1, y, x1, 5, footprint=400) == 0
        with pytest.raises(sense.SenseError, match="slot"):
            eng.admit(p1, y, x2, 5, footprint=1)  # plan already in a slot
        with pytest.raises(sense.SenseError, match="slot"):
            p1.cg(y, 5)
        assert eng.admit(p2, y, x2, 5, footprint=400) == 1
        assert eng.admit(p3, y, x3, 5, footprint=100) is None  # no free slot
        done = []
        while len(done) < 2:
            eng.step()
            done += eng.poll()
        assert sorted(done) == [0, 1]
        assert eng.stats()["used"] == 0
        ref = p3.cg(y, 5).x
        assert torch.equal(x1, ref) and torch.equal(x2, ref)


def test_admit_waits_for_the_callers_stream():
    """k-space produced on the caller's stream immediately before admission
    (no synchronisation in between, on a non-default stream behind a long
    queue of work) is what the engine solves: the result is bitwise the
    plain solve's."""
    bank = InputBank()
    r = Request(0, 0.0, 256, 16, 3, 8)
    bank.prepare([r])
    maps, mask = bank.coil_maps(256, 16), bank.mask(256, 3)
    img = torch.from_numpy(np.stack([bank.synth.phantom2d(256, seed=5)]).astype(np.complex64)).to("cuda:0")
    with sense.Plan(maps, mask) as pe, sense.Plan(maps, mask) as pref:
        yref = pref.E(img)
        ref = pref.cg(yref, 8).x.clone()
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        x = torch.empty((1, 256, 256), dtype=torch.complex64, device="cuda:0")
        with sense.Engine(budget_bytes=1 << 32, max_slots=2) as eng:
            with torch.cuda.stream(s):
                busy = torch.randn((4096, 4096), device="cuda:0")
                for _ in range(8):
                    busy = busy @ busy * 1e-3  # keep the caller's stream busy
                y = torch.zeros_like(yref)
                y += yref  # y is ready only after the queue above
                assert eng.admit(pe, y, x, 8) == 0
            done = []
            while not done:
                eng.step()
                done = eng.poll()
            eng.sync()
        torch.cuda.synchronize()
    assert torch.equal(x, ref)


def test_engine_holds_inputs_until_polled():
    """The caller may drop a request's k-space right after admission: the
    engine binding holds it (with the plan and x) until poll reports the
    slot, so torch's allocator cannot hand that memory to a tensor written
    meanwhile on the caller's stream.  The result is bitwise the plain
    solve's."""
    bank = InputBank()
    r = Request(0, 0.0, 256, 16, 3, 8)
    bank.prepare([r])
    maps, mask = bank.coil_maps(256, 16), bank.mask(256, 3)
    img = torch.from_numpy(np.stack([bank.synth.phantom2d(256, seed=6)]).astype(np.complex64)).to("cuda:0")
    with sense.Plan(maps, mask) as pe, sense.Plan(maps, mask) as pref:
        yref = pref.E(img)
        ref = pref.cg(yref, 8).x.clone()
        torch.cuda.synchronize()
        x = torch.empty((1, 256, 256), dtype=torch.complex64, device="cuda:0")
        s = torch.cuda.Stream()
        with sense.Engine(budget_bytes=1 << 32, max_slots=2) as eng:
            with torch.cuda.stream(s):
                busy = torch.randn((4096, 4096), device="cuda:0")
                for _ in range(8):
                    busy = busy @ busy * 1e-3  # keep the caller's stream busy
                # the clone's only reference after this line is the engine's
                assert eng.admit(pe, yref.clone(), x, 8) == 0
                junk = [torch.full_like(yref, 1e3) for _ in range(4)]
            assert len(eng._held) == 1
            done = []
            while not done:
                eng.step()
                done = eng.poll()
            assert done == [0] and eng._held == {}
            eng.sync()
        torch.cuda.synchronize()
        del junk
    assert torch.equal(x, ref)
