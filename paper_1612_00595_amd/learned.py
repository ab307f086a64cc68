"""The learned birth proposal end to end: train the mixture-density network
on pairs from the forward simulator, then turn an instance's trace into the
anchor mixture table and weights that the sampler's learned births read.

Every step runs in the library's kernels (pair simulation, features, BF16
MFMA forward/backward, Adam, table construction); this module only
sequences the calls and owns the device buffers.
"""
from __future__ import annotations

import dataclasses
import time

from . import chromh
from .workloads import ModelSpec


@dataclasses.dataclass
class TrainResult:
    net: "chromh.MDN"
    steps: int
    pairs: int
    seconds: float
    losses: list            # (step, mean batch loss) every log_every steps
    held_out: float         # mean loss on pairs never trained on


def train(model: ModelSpec, pairs: int = 10_000_000, batch: int = 8192, lr: float = 1e-3,
          seed: int = 0, init_seed: int = 1, log_every: int = 100, held_out: int = 8192,
          device="cuda") -> TrainResult:
    """One epoch over `pairs` fresh simulator pairs (pair indices 0 ..
    pairs - 1 of stream `seed`), Adam at learning rate lr; the held-out loss
    uses pairs from index 2^40 on."""
    import torch
    net = chromh.MDN(device=device, seed=init_seed)
    steps = max(1, pairs // batch)
    losses = []
    loss_buf = torch.empty(batch, dtype=torch.float32, device=device)
    pairs_buf = (torch.empty((batch, 576), dtype=torch.bfloat16, device=device),
                 torch.empty((batch, 3), dtype=torch.float32, device=device))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chunk = log_every if log_every else steps
    step = 1
    while step <= steps:
        # pairs and steps step .. step + n - 1 in one library call; the stream
        # orders each step's pairs after the previous step's use of the buffers
        n = min(chunk, steps - step + 1)
        net.train(model, seed, (step - 1) * batch, n, batch, step, lr, pairs_buf, loss=loss_buf)
        step += n
        if log_every:
            losses.append((step - 1, float(loss_buf.mean())))
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    Xh, Zh = chromh.mdn_pairs(model, seed, 1 << 40, held_out, device)
    lh, _ = net.gradients(Xh, Zh)
    return TrainResult(net=net, steps=steps, pairs=steps * batch, seconds=seconds, losses=losses,
                       held_out=float(lh.mean()))


def anchor_table(net: "chromh.MDN", model: ModelSpec, trace, chunk: int = 65536):
    """(table [anchors, 8, 8] float64, weights [anchors] float64, n_tau) on the
    trace's device, anchors processed `chunk` at a time."""
    import torch
    na, ntau = chromh.anchor_count(model)
    table = torch.empty((na, 8, 8), dtype=torch.float64, device=trace.device)
    weights = torch.empty(na, dtype=torch.float64, device=trace.device)
    for first in range(0, na, chunk):
        cnt = min(chunk, na - first)
        X, w = chromh.anchor_features(model, trace, first, cnt)
        head = net.infer(X)
        table[first:first + cnt] = chromh.mixture_table(model, head, first)
        weights[first:first + cnt] = w
    return table, weights, ntau
