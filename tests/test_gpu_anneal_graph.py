"""Runs of annealing steps (lpf_anneal_run: hipGraph replays of 32 captured steps plus the
remainder) against the same chains stepped one call at a time, bit for bit.  Graph replays are
interleaved with eager steps, other device work and synchronisations."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_04359_amd import Context
    c = Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pair(ctx, kind, seed=5):
    from paper_1601_04359_amd import Anneal
    side, c = 24, 6
    if kind == "s2":
        tgt = wl.square_particles(48, 48, 4, 23, 3)
        target = oracle.s2(tgt, c, c, 3)
    else:
        tgt = wl.boolean_disks(48, 48, 3.0, 0.4, 3)
        target = oracle.lpf(tgt, c, c, 3)
    cell = wl.random_cell(side, side, int(round(tgt.mean() * side * side)), 4)
    kw = {}
    if kind == "s2":
        kw["descriptor"] = "s2"
    if kind == "sampled":
        Xt = wl.sample_positions(48, 48, 500, 6)
        target = oracle.lpf_sampled(tgt, c, c, Xt, 3)
        kw["sample"] = ctx.pack(_dev(wl.sample_positions(side, side, 150, 7)))
    Nt = 500 if kind == "sampled" else tgt.size
    chains = []
    for _ in range(2):
        ch = Anneal(ctx, ctx.pack(_dev(cell)), side, side, c, c, 3, _dev(target.astype(np.int32)),
                    Nt, seed, **kw)
        chains.append(ch)
    if kind in ("recount", "records"):
        from paper_1601_04359_amd import LPF_DELTA_RECORDS, LPF_DELTA_RECOUNT
        m = LPF_DELTA_RECOUNT if kind == "recount" else LPF_DELTA_RECORDS
        for ch in chains:
            ch.set_method(m)
    return chains


@pytest.mark.parametrize("kind,proposal,K", [("records", 0, 256), ("recount", 0, 64),
                                             ("records", 1, 200), ("s2", 0, 128),
                                             ("sampled", 0, 100)])
def test_run_equals_stepwise(ctx, kind, proposal, K):
    import torch
    from paper_1601_04359_amd import step_records
    print(f"[gpu] anneal run graph {kind} proposal={proposal} K={K}", flush=True)
    a, b = _pair(ctx, kind)
    Ts = 2e-4 * 0.97 ** np.arange(120)
    ra = [step_records(a.run_schedule(K, Ts[:40], proposal))]
    torch.cuda.synchronize()
    junk = torch.arange(1 << 16, device="cuda").float().sum()  # other eager work in between
    ra.append(step_records(a.run(K, Ts[40:50], proposal)))
    torch.cuda.synchronize()
    ra.append(step_records(a.run_schedule(K, Ts[50:120], proposal)))
    torch.cuda.synchronize()
    ra = np.concatenate(ra)
    rb = step_records(b.run(K, Ts, proposal))
    torch.cuda.synchronize()
    assert float(junk) > 0
    assert np.array_equal(ra, rb)
    assert np.array_equal(ra["step"], np.arange(120))
    assert (ra["k"] >= 0).sum() > 10
    assert torch.equal(a.bits, b.bits) and torch.equal(a.counts, b.counts)
    assert torch.equal(a.e, b.e)
    # a fresh graph each call: a later run continues the chain
    rc = step_records(a.run_schedule(K, Ts[:64], proposal))
    rd = step_records(b.run(K, Ts[:64], proposal))
    torch.cuda.synchronize()
    assert np.array_equal(rc, rd)
    a.close()
    b.close()


@pytest.mark.parametrize("refresh,use_net", [(3, False), (4, False), (4, True), (1, True)])
def test_run_learned_proposals(ctx, refresh, use_net):
    # learned proposals: captured when refresh divides 32 (the re-scoring pattern repeats in
    # every replay), else enqueued one by one; either way the chain of anneal_step
    import torch
    from paper_1601_04359_amd import LPF_PROP_LEARNED, ProposalNet, learn, step_records
    print(f"[gpu] anneal run learned refresh={refresh} net={use_net}", flush=True)
    a, b = _pair(ctx, "records", seed=9)
    net = None
    if use_net:
        net = ProposalNet(ctx, 24, 24, 1, 16, learn.init_params(4, torch.device("cuda:0")))
    sc = _dev(np.random.default_rng(2).standard_normal(24 * 24).astype(np.float32))
    for ch in (a, b):
        if net is not None:
            ch.set_proposal(net=net, beta=1.5, eps_uniform=0.2, refresh=refresh, rank=True)
        else:
            ch.set_proposal(scores=sc, beta=1.5, eps_uniform=0.2, refresh=refresh, rank=True)
    Ts = 1e-4 * np.ones(100)
    ra = [step_records(a.run_schedule(128, Ts[:70], LPF_PROP_LEARNED))]
    torch.cuda.synchronize()
    ra.append(step_records(a.run(128, Ts[70:75], LPF_PROP_LEARNED)))
    ra.append(step_records(a.run_schedule(128, Ts[75:], LPF_PROP_LEARNED)))
    rb = step_records(b.run(128, Ts, LPF_PROP_LEARNED))
    torch.cuda.synchronize()
    assert np.array_equal(np.concatenate(ra), rb)
    assert torch.equal(a.bits, b.bits)
    a.close()
    b.close()
    if net is not None:
        net.close()
