"""Training data and training loop of the swap-proposal network (orchestration only).

Samples are (cell state, interchange (a, b), exact energy change de) triples taken from plain
annealing runs: the chain is advanced with uniform proposals, its state is copied every few
steps, random phase-preserving interchanges of that state are labelled with their exact de by
lpf_anneal_delta_energy, and the network is fitted so that S[a] + S[b] predicts -de / sigma.
The annealing, the exact labels, the network's forward and backward passes and Adam run in
liblpf's kernels.  This module does the data bookkeeping on the host with numpy: it draws the
labelled interchanges from an unpacked copy of each snapshot, takes sigma as the standard
deviation of the collected labels, scales them, and picks the mini-batches.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import Anneal, Context, ProposalNet, cnn_samples, _abi


@dataclass
class Dataset:
    bits: torch.Tensor      # [S][H][ceil(W/64)] packed snapshots (device)
    img: np.ndarray         # [n] snapshot index of each sample
    a: np.ndarray           # [n] phase-1 pixel
    b: np.ndarray           # [n] phase-0 pixel
    de: np.ndarray          # [n] exact energy change of the interchange
    sigma: float            # label scale: y = -de / sigma
    W: int
    H: int


def init_params(seed: int, device) -> torch.Tensor:
    """Initial network parameters (packed like LPF_CNN_PARAMS): weights uniform in
    +-sqrt(6 / fan_in) (He initialisation), biases zero, drawn from PCG64(seed)."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, shape in ((18, (9, 16, 2)), (0, (16,)), (144, (9, 16, 16)), (0, (16,)),
                          (144, (9, 16, 16)), (0, (16,)), (16, (16,)), (0, (1,))):
        if fan_in:
            lim = np.sqrt(6.0 / fan_in)
            parts.append(g.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == _abi.LPF_CNN_PARAMS
    return torch.from_numpy(p).to(device)


def unpack_bits(bits: torch.Tensor, W: int, H: int) -> np.ndarray:
    b = bits.detach().cpu().numpy().view(np.uint64).reshape(H, -1)
    out = np.zeros((H, W), np.uint8)
    for x in range(W):
        out[:, x] = (b[:, x // 64] >> np.uint64(x % 64)) & np.uint64(1)
    return out


def collect(chain: Anneal, n_snapshots: int, every: int, per_snapshot: int, K: int, Ts,
            seed: int) -> Dataset:
    """Advance `chain` (uniform proposals) and label `per_snapshot` random interchanges of its
    state every `every` steps.  Ts: temperature of each step (len >= n_snapshots * every)."""
    g = np.random.Generator(np.random.PCG64(seed))
    W, H = chain.W, chain.H
    snaps, imgs, aa, bb, des = [], [], [], [], []
    step = 0
    for s in range(n_snapshots):
        chain.run(K, Ts[step:step + every])
        step += every
        snaps.append(chain.bits.clone())
        cell = unpack_bits(chain.bits, W, H).ravel()
        ones = np.flatnonzero(cell == 1)
        zeros = np.flatnonzero(cell == 0)
        a = g.choice(ones, per_snapshot)
        b = g.choice(zeros, per_snapshot)
        sw = torch.from_numpy(np.stack([a, b], 1).astype(np.int32)).to(chain.bits.device)
        de = chain.delta_energy(sw).cpu().numpy()
        imgs.append(np.full(per_snapshot, s, np.int32))
        aa.append(a.astype(np.int32))
        bb.append(b.astype(np.int32))
        des.append(de)
    de = np.concatenate(des)
    sigma = float(np.std(de)) or 1.0
    return Dataset(torch.stack(snaps), np.concatenate(imgs), np.concatenate(aa),
                   np.concatenate(bb), de, sigma, W, H)


def train(net: ProposalNet, data: Dataset, steps: int, batch_images: int, lr: float,
          seed: int = 0, log_every: int = 0):
    """Adam on mini-batches of `batch_images` snapshots with all their samples; returns the
    loss history (host floats)."""
    g = np.random.Generator(np.random.PCG64(seed))
    n_snap = data.bits.shape[0]
    by_img = [np.flatnonzero(data.img == s) for s in range(n_snap)]
    y_all = (-data.de / data.sigma).astype(np.float32)
    dev = data.bits.device
    losses = []
    for it in range(steps):
        sel = g.choice(n_snap, min(batch_images, n_snap), replace=False)
        idx = np.concatenate([by_img[s] for s in sel])
        local = np.concatenate([np.full(len(by_img[s]), i, np.int32) for i, s in enumerate(sel)])
        bits = data.bits[torch.from_numpy(sel).to(dev)].reshape(-1)
        smp = cnn_samples(local, data.a[idx], data.b[idx], y_all[idx], dev)
        grad, loss = net.grad(bits, len(sel), smp)
        net.adam(grad, lr)
        losses.append(loss)
        if log_every and (it + 1) % log_every == 0:
            print(f"  train step {it + 1}: loss {float(loss.cpu()[0]):.4f}", flush=True)
    return [float(l.cpu()[0]) for l in losses]
