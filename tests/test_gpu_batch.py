"""A batch of independent problems (members of the c5 batch), one context
and one stream each, with deferred errors so that no call waits for the
device: the members' kernels overlap on the GPU, and every member's
pressure and flux equal those of a one-at-a-time solve bit for bit.  The
gradient equals the one-at-a-time gradient to rounding (the adjoint sums the
overlapping boxes' contributions with atomic adds, whose order varies).  A
device-side error of one member is reported by mrcm_wait of that member
only, and clears with it."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from inputs import make_workload  # noqa: E402

pytestmark = pytest.mark.gpu

NMEM = 4


def _weights(wl, torch):
    """Outflow through the +x side as flux weights; 16 observation cells."""
    nx, ny = wl.ncell
    n = nx * ny
    fw = torch.zeros(n, 4, dtype=torch.float64, device="cuda")
    fw[torch.arange(nx - 1, n, nx, device="cuda"), 1] = wl.h
    obs = torch.as_tensor(np.arange(0, n, n // 16)[:16], device="cuda")
    return fw.reshape(-1), obs


def _round(m, ctx, wl, fw, obs, adjoint=True):
    import torch
    m.build_basis(ctx)
    m.solve_interface(ctx)
    m.smooth(ctx, wl.nsmooth)
    p, fl = m.get_solution(ctx)
    g = None
    if adjoint:
        dJdp = torch.zeros_like(p)
        dJdp[obs] = p[obs] - 0.1
        g = m.adjoint(ctx, dJdp, fw)
    return p, fl, g


def _open(m, api, wl, deferred):
    ctx = m.create(wl.dim, wl.ncell, wl.h)
    api.configure(ctx, wl, "fp64")
    m.set_checkpointing(ctx, True)
    if deferred:
        m.set_deferred_errors(ctx, True)
    return ctx


def test_batch_on_streams_matches_one_at_a_time():
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    wls = [make_workload("c5", member=k) for k in range(NMEM)]
    fw, obs = _weights(wls[0], torch)
    torch.cuda.synchronize()
    ref = []
    for wl in wls:
        ctx = _open(m, api, wl, False)
        try:
            p, fl, g = _round(m, ctx, wl, fw, obs)
            ref.append((p.cpu().numpy(), fl.cpu().numpy(), g.cpu().numpy()))
        finally:
            m.destroy(ctx)
    streams = [torch.cuda.Stream() for _ in wls]
    ctxs = []
    try:
        for wl, s in zip(wls, streams):
            with torch.cuda.stream(s):
                ctxs.append(_open(m, api, wl, True))
        for rep in range(2):  # the second round reuses plans and graphs
            outs = []
            for ctx, wl, s in zip(ctxs, wls, streams):
                with torch.cuda.stream(s):
                    outs.append(_round(m, ctx, wl, fw, obs))
            for ctx in ctxs:
                m.wait(ctx)
            for k, (p, fl, g) in enumerate(outs):
                rp, rf, rg = ref[k]
                print("round", rep, "member", k, flush=True)
                assert np.array_equal(p.cpu().numpy(), rp)
                assert np.array_equal(fl.cpu().numpy(), rf)
                gg = g.cpu().numpy()
                assert np.linalg.norm(gg - rg) <= 1e-13 * np.linalg.norm(rg)
    finally:
        for ctx in ctxs:
            m.destroy(ctx)


def test_deferred_error_reported_by_wait_of_its_member():
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    wls = [make_workload("c5", member=k) for k in range(3)]
    fw, obs = _weights(wls[0], torch)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in wls]
    ctxs = []
    try:
        for wl, s in zip(wls, streams):
            with torch.cuda.stream(s):
                ctxs.append(_open(m, api, wl, True))
        good = torch.as_tensor(wls[1].logk.ravel(), dtype=torch.float64, device="cuda").contiguous()
        bad = good.clone()
        bad[37] = float("nan")
        torch.cuda.synchronize()

        def batch(k_adj):
            outs = []
            for k, (ctx, wl, s) in enumerate(zip(ctxs, wls, streams)):
                with torch.cuda.stream(s):
                    outs.append(_round(m, ctx, wl, fw, obs, adjoint=k != k_adj))
            return outs

        first = batch(-1)
        for ctx in ctxs:
            m.wait(ctx)
        first = [(p.cpu().numpy(), fl.cpu().numpy()) for p, fl, _ in first]
        with torch.cuda.stream(streams[1]):
            m.set_permeability(ctxs[1], bad)
        # every member runs its adjoint too, the bad one included: the
        # adjoint must leave the forward solve's unread error flag in place
        second = batch(-1)
        m.wait(ctxs[0])
        with pytest.raises(m.MRCMError) as err:
            m.wait(ctxs[1])
        assert err.value.status == 1  # MRCM_EINVAL
        m.wait(ctxs[2])
        for k in (0, 2):
            assert np.array_equal(second[k][0].cpu().numpy(), first[k][0])
        with torch.cuda.stream(streams[1]):
            m.set_permeability(ctxs[1], good)
        third = batch(-1)
        for ctx in ctxs:
            m.wait(ctx)  # the error was cleared by the wait that reported it
        for k in range(3):
            assert np.array_equal(third[k][0].cpu().numpy(), first[k][0])
            assert np.array_equal(third[k][1].cpu().numpy(), first[k][1])
    finally:
        for ctx in ctxs:
            m.destroy(ctx)


def test_back_to_back_deferred_solves_equal_a_synchronous_solve():
    """The benchmark's timed form (c2 at full size, overlap 4, linear spaces):
    solves enqueued back to back with one mrcm_wait at the end give the
    pressure and flux of a solve that waits for its own error read-back."""
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    wl = make_workload("c2")
    ctx = m.create(wl.dim, wl.ncell, wl.h)
    try:
        api.configure(ctx, wl, "fp64")

        def solve():
            m.build_basis(ctx)
            m.solve_interface(ctx)
            m.smooth(ctx, wl.nsmooth)
            return m.get_solution(ctx)

        p0, f0 = solve()
        p0, f0 = p0.cpu().numpy(), f0.cpu().numpy()
        m.set_deferred_errors(ctx, True)
        outs = [solve() for _ in range(3)]
        m.wait(ctx)
        m.set_deferred_errors(ctx, False)
        for p, fl in outs:
            assert np.array_equal(p.cpu().numpy(), p0)
            assert np.array_equal(fl.cpu().numpy(), f0)
    finally:
        m.destroy(ctx)


def test_deferred_errors_from_the_first_call_of_a_new_context():
    """A context whose first solve runs with deferred errors reports only
    its own errors: its device flags start clear, whatever the memory it
    was given held before (here: device memory filled with all bits set and
    handed back to the driver just before the context is created)."""
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    wl = make_workload("c5", scale=4)
    for _ in range(3):
        junk = torch.full((1 << 24,), -1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        del junk
        torch.cuda.empty_cache()
        ctx = m.create(wl.dim, wl.ncell, wl.h)
        try:
            api.configure(ctx, wl, "fp64")
            m.set_deferred_errors(ctx, True)
            m.build_basis(ctx)
            m.solve_interface(ctx)
            m.smooth(ctx, 2)
            m.get_solution(ctx)
            m.wait(ctx)
        finally:
            m.destroy(ctx)
