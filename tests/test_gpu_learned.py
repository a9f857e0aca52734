"""Learned proposals (anneal_step with LPF_PROP_LEARNED) and exact energy labels."""
from __future__ import annotations

from fractions import Fraction

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


def _chain(ctx, cell, cx, mask, target, Nt, seed):
    import torch
    from paper_1601_04359_amd import Anneal
    H, W = cell.shape
    bits = ctx.pack(torch.from_numpy(cell).cuda())
    return Anneal(ctx, bits, W, H, cx, cx, mask, torch.from_numpy(target.astype(np.int32)).cuda(),
                  Nt, seed)


def _problem(side=24, cx=5, mask=3, seed=3):
    tgt = wl.boolean_disks(64, 64, 3.0, 0.4, seed)
    target = oracle.lpf(tgt, cx, cx, mask)
    cell = wl.random_cell(side, side, int(round(0.4 * side * side)), seed + 1)
    return tgt, target, cell


@pytest.mark.parametrize("method", [1, 2])
def test_delta_energy_exact(ctx, method):
    # de of given interchanges equals the exact rational change of eq. (LSE)
    import torch
    print(f"[gpu] delta energy exact, method {method}", flush=True)
    tgt, target, cell = _problem()
    ch = _chain(ctx, cell, 5, 3, target, tgt.size, 1)
    ch.set_method(method)
    g = np.random.default_rng(0)
    ones = np.flatnonzero(cell.ravel() == 1)
    zeros = np.flatnonzero(cell.ravel() == 0)
    sw = np.stack([g.choice(ones, 40), g.choice(zeros, 40)], 1).astype(np.int32)
    sw[0] = [ones[0], ones[1]]  # same phase: zero
    de = ch.delta_energy(torch.from_numpy(sw).cuda()).cpu().numpy()
    N, Nt = cell.size, tgt.size
    L0 = oracle.lpf(cell, 5, 5, 3).astype(np.int64)
    dl = oracle.delta_swap(cell, 5, 5, sw, 3).astype(np.int64)

    def lse(L):
        return sum((Fraction(int(t), Nt) - Fraction(int(c), N)) ** 2
                   for c, t in zip(L.ravel(), target.ravel()))
    e0 = lse(L0)
    for i in range(len(sw)):
        assert de[i] == float(lse(L0 + dl[i]) - e0), i
    ch.close()


def test_learned_draws_follow_scores(ctx):
    # with a fixed score field, draws of a follow exp(beta * score) over the phase-1 pixels
    import torch
    tgt, target, cell = _problem(side=32)
    ch = _chain(ctx, cell, 5, 3, target, tgt.size, 2)
    W = H = 32
    score = np.zeros((H, W), np.float32)
    score[:, : W // 2] = 1.0   # left half preferred
    sc = torch.from_numpy(score.ravel()).cuda()
    beta = 1.5
    ch.set_proposal(scores=sc, beta=beta, eps_uniform=0.0)
    K = 65536
    cand = ch.propose(K, 2).cpu().numpy()
    flat = cell.ravel()
    assert np.all(flat[cand[:, 0]] == 1) and np.all(flat[cand[:, 1]] == 0)
    left = (np.arange(W * H) % W) < W // 2
    for col, ph in ((0, 1), (1, 0)):
        w = np.exp(beta * score.ravel())[flat == ph]
        p_left = w[left[flat == ph]].sum() / w.sum()
        emp = left[cand[:, col]].mean()
        assert abs(emp - p_left) < 5 * np.sqrt(p_left * (1 - p_left) / K), (emp, p_left)
    # eps = 1 falls back to uniform draws: the same candidates as LPF_PROP_UNIFORM
    ch.set_proposal(scores=sc, beta=beta, eps_uniform=1.0)
    assert torch.equal(ch.propose(256, 2), ch.propose(256, 0))
    ch.close()


@pytest.mark.parametrize("refresh", [1, 4])
def test_learned_chain_stays_exact(ctx, refresh):
    # learned steps keep counts equal to a full recount and e equal to eq. (LSE)
    import torch
    from paper_1601_04359_amd import ProposalNet, step_records
    from oracle import cnn
    print(f"[gpu] learned chain refresh {refresh}", flush=True)
    tgt, target, cell = _problem(side=32)
    ch = _chain(ctx, cell, 5, 3, target, tgt.size, 3)
    net = ProposalNet(ctx, 32, 32, 1, 4, torch.from_numpy(cnn.init_params(9)).cuda())
    ch.set_proposal(net=net, beta=1.0, eps_uniform=0.2, refresh=refresh)
    recs = step_records(ch.run(64, np.full(80, 5e-5), 2))
    torch.cuda.synchronize()
    assert (recs["k"] >= 0).sum() > 5
    fresh = ctx.full(ch.bits, 32, 32, 5, 5, 3)
    assert torch.equal(fresh, ch.counts)
    e = oracle.lse(ch.counts.cpu().numpy(), target, 32 * 32, tgt.size)
    assert abs(float(ch.e.cpu()[0]) - e) <= 1e-12 * max(e, 1e-30)
    ch.close()
    net.close()
