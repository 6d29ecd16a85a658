"""GPU: the allocation-free training step (coolchic_train_step_noalloc,
workspace in the library's static device scratch) against
coolchic_train_step with a caller workspace, through the C ABI.

Two calls in a row on the same device, the second on a smaller problem (so
the scratch still holds the first call's contents), each as two training
iterations: latents and parameters, gradients, both Adam moments, the loss
and the step counter must be bit-identical (the same kernels in the same
dependency order, every reduction in a fixed order).
"""
import numpy as np
import pytest
import torch

from tests import cases as CS

pytestmark = pytest.mark.gpu




def _state(c, B):
    dev = torch.device("cuda", 0)
    theta = torch.from_numpy(np.concatenate([c.y, c.arm, c.ups, c.syn]).astype(np.float32)).to(dev)
    z = lambda: torch.zeros_like(theta)  # noqa: E731
    return dict(theta=theta, grad=z(), m=z(), v=z(), step=torch.zeros(2, dtype=torch.int32, device=dev),
                loss4=torch.zeros(4, device=dev))


def _run(B, c, noalloc, iters=2):
    p = B.Problem(c.H, c.W, B.Arch(*c.arch), B.CC_QUANT_NOISE if c.u is not None else B.CC_QUANT_ROUND, c.lam)
    s = _state(c, B)
    img = torch.from_numpy(c.img).cuda().reshape(-1)
    u = None if c.u is None else torch.from_numpy(c.u).cuda()
    losses = []
    for _ in range(iters):
        args = (p, img, u, 1.0, s["loss4"], s["theta"], s["grad"], s["m"], s["v"], s["step"])
        if noalloc:
            B.coolchic_train_step_noalloc(*args)
        else:
            B.coolchic_train_step(*args)
        losses.append(s["loss4"].clone())
    torch.cuda.synchronize()
    out = {k: t.cpu().numpy() for k, t in s.items()}
    out["losses"] = np.stack([x.cpu().numpy() for x in losses])
    return out


def test_noalloc_matches_train_step_two_calls_shrinking():
    from paper_2403_11651_amd import binding as B
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    big = CS.full()                                        # 768x512, full decoder: 31.8 MiB of scratch
    small = CS.make("tiny64_noise", 64, 64, CS.TINY, seeds=(0, 1, 2, 4), noise=True)
    assert B.workspace_bytes(B.Problem(big.H, big.W, B.Arch(*big.arch)), B.CC_WS_BACKWARD) \
        <= B.CC_NOALLOC_SCRATCH_BYTES
    for c in (big, small):
        print(f"noalloc vs train_step: {c.name} {c.H}x{c.W} arch {c.arch}", flush=True)
        got = _run(B, c, noalloc=True)
        ref = _run(B, c, noalloc=False)
        for k in ("theta", "grad", "m", "v", "losses", "step"):
            assert np.array_equal(got[k], ref[k]), (c.name, k)
        assert np.all(got["losses"][:, 3] == 0.0) and np.all(np.isfinite(got["losses"][:, 0])), c.name
        assert got["step"].tolist() == [2, 0]
