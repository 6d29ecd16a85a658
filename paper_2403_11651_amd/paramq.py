"""Choice of the decoder's parameter quantisation steps.

Section II: once an image is encoded, its network parameters are quantised
and entropy coded; their rate adds to the latents' rate in the
rate-distortion cost of Eq. (1).  Each module (ARM, upsampling, synthesis)
gets one step 2^-k.  `quantize_decoder` picks the steps greedily, module by
module (the others held at their current choice, starting from the finest
step): for every candidate k it quantises the parameters with
coolchic_param_quantize, evaluates Eq. (1) with coolchic_forward on the
quantised decoder, and keeps the k with the smallest total cost
    D + lambda (R_latents + R_parameters) / (H W).
All the arithmetic runs in the library's kernels; this module only drives
the search and reads the losses back.
"""
from __future__ import annotations

import torch

from . import binding as B

DEFAULT_STEPS = tuple(range(4, 15))   # candidate k: steps 2^-4 .. 2^-14


def quantize_decoder(p: "B.Problem", img, y, arm, ups, syn, candidates=DEFAULT_STEPS, u=None):
    """Returns a dict: steps (k per module), the quantised arm / ups / syn
    tensors, bits of each module, the loss terms of the quantised decoder
    (loss4 = {loss without the parameter rate, D, R_latents, flag}), and
    total = D + lambda (R_latents + R_parameters) / (H W) with every
    candidate's total in `tried`."""
    dev = y.device
    q = [torch.empty_like(t) if t is not None and t.numel() else None for t in (arm, ups, syn)]
    bits = torch.zeros(3, device=dev)
    loss4 = torch.zeros(4, device=dev)
    hw = float(p.H * p.W)
    steps = [max(candidates)] * 3
    tried = {}

    def evaluate(ks):
        B.coolchic_param_quantize(p.arch, arm, ups, syn, ks, q[0], q[1], q[2], bits)
        B.coolchic_forward(p, img, y, u, q[0], q[1], q[2], loss4)
        l4 = loss4.cpu().tolist()
        b = bits.cpu().tolist()
        total = l4[1] + p.lam * (l4[2] + sum(b)) / hw
        tried[tuple(ks)] = total
        return total, l4, b

    for m in range(3):
        if m == 1 and (ups is None or ups.numel() == 0):
            continue
        best_k, best_total = steps[m], None
        for k in candidates:
            ks = list(steps)
            ks[m] = k
            total, _, _ = evaluate(ks)
            if best_total is None or total < best_total:
                best_k, best_total = k, total
        steps[m] = best_k
    total, l4, b = evaluate(steps)
    return dict(steps=tuple(steps), arm=q[0].clone(), ups=None if q[1] is None else q[1].clone(), syn=q[2].clone(),
                bits=b, loss4=l4, total=total, tried=tried)
