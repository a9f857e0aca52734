"""What the trained proposal network gains over uniform proposals (everything seeded: the chains,
the training data and the training are deterministic, and every move is still judged by the
exact energy change).

Problem: a 64 x 64 cell matching the LPF (|dx|,|dy| <= 12, both phases) of a 512 x 512 Boolean
disk image (phi 0.35, r 4); 256 candidates per step, T_s = 1e-3 * 0.01^(s/S) over S = 1500 steps.
The plain chain's final error is E*.  The network is trained on labelled interchanges of an
independent plain chain; the learned chain (beta 8, same seed and start cell) must reach E* in
at most 0.6 of the plain chain's steps, while an untrained network (same architecture, its
initial weights) needs more than 0.8 of them."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def test_trained_network_reaches_plain_error_in_half_the_steps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_04359_amd import (Anneal, Context, LPF_PROP_LEARNED, LPF_PROP_UNIFORM,
                                      ProposalNet, learn, step_records)
    print("[gpu] learned gain 64x64 c=12", flush=True)
    dev = torch.device("cuda:0")
    side, tside, c, K, S = 64, 512, 12, 256, 1500
    ctx = Context(0)
    tgt = wl.anneal_target(tside, 0.35, 4.0, 77)
    target = ctx.full(ctx.pack(torch.from_numpy(tgt).to(dev)), tside, tside, c, c, 3)
    cell = wl.random_cell(side, side, int(round(float(tgt.mean()) * side * side)), 5)
    Ts = 1e-3 * (0.01 ** (1.0 / S)) ** np.arange(S)

    def chain(seed):
        return Anneal(ctx, ctx.pack(torch.from_numpy(cell).to(dev)), side, side, c, c, 3, target,
                      tside * tside, seed)

    def steps_to(e_star, net):
        ch = chain(1)
        ch.set_proposal(net=net, beta=8.0, eps_uniform=0.1)
        r = step_records(ch.run(K, Ts, LPF_PROP_LEARNED))
        ch.close()
        hit = np.flatnonzero(r["e"] <= e_star)
        return int(hit[0]) + 1 if len(hit) else None

    plain = chain(1)
    rp = step_records(plain.run(K, Ts, LPF_PROP_UNIFORM))
    plain.close()
    e_star = float(rp["e"][-1])
    assert e_star < float(rp["e"][0])

    src = chain(99)
    data = learn.collect(src, 48, S // 48, 1024, K, Ts, seed=7)
    src.close()
    p0 = learn.init_params(11, dev)
    untrained = ProposalNet(ctx, side, side, 8, 8 * 1024, p0)
    net = ProposalNet(ctx, side, side, 8, 8 * 1024, p0)
    losses = learn.train(net, data, 300, 8, 2e-3, seed=3)
    assert losses[-1] < 0.6 * losses[0], losses[::30]

    s_learned = steps_to(e_star, net)
    s_untrained = steps_to(e_star, untrained)
    print(f"[gpu] steps to E*: plain {S}, learned {s_learned}, untrained {s_untrained}", flush=True)
    assert s_learned is not None and s_learned <= 0.6 * S, s_learned
    assert s_untrained is None or s_untrained > 0.8 * S, s_untrained
    net.close()
    untrained.close()
    ctx.close()
