"""GPU parity of Table I's decoders and the 4-tap upsamplers: the HIP path
through the C ABI against the FP64 oracle, at the bars of the other parity
tests (loss 1e-5 relative, per-latent rate, every gradient tensor 1e-3).

Table I ("1-1-TConv-K"): one non-separable K x K transposed convolution
shared by every upsampling step, K = 4 for the 300, 545 and 1079 rows and 8
for the 2300 row; the separable per-step upsampler with K = 4 as well.
"""
import numpy as np
import pytest
import torch

import oracle as O
from tests import cases as CS
from tests.test_gpu_parity import check_backward, check_forward, gpu_backward, _dev, _problem

pytestmark = pytest.mark.gpu

ROW300 = (7, 8, 1, 4, 8, 1, 1)
ROW545 = (7, 8, 2, 4, 16, 2, 1)
ROW1079 = (7, 16, 2, 4, 16, 2, 1)
ROW2300 = (7, 24, 2, 8, 40, 2, 1)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_11651_amd import binding
    return binding


CASES = [
    ("row300_64x64", 64, 64, ROW300, False),
    ("row545_96x160_L6_noise", 96, 160, (6,) + ROW545[1:], True),
    ("row1079_64x192", 64, 192, ROW1079, False),
    ("row2300_64x64", 64, 64, ROW2300, False),
    ("row2300_40x72_L4_noise", 40, 72, (4,) + ROW2300[1:], True),
    ("shared4_L2_8x24", 8, 24, (2, 8, 1, 4, 8, 1, 1), False),
    ("separable4_64x64", 64, 64, (7, 8, 2, 4, 16, 1, 0), False),
    ("separable4_L4_40x72_noise", 40, 72, (4, 16, 2, 4, 32, 2, 0), True),
]


def _case(name, H, W, arch, noise, seed=60):
    return CS.make(name, H, W, arch, seeds=(seed, seed + 1, seed + 2, seed + 3), n_blobs=max(3, H * W // 400),
                   noise=noise)


@pytest.mark.parametrize("name,H,W,arch,noise", CASES, ids=[c[0] for c in CASES])
def test_table1_variants_vs_oracle(B, name, H, W, arch, noise):
    c = _case(name, H, W, arch, noise)
    check_forward(B, c)
    check_backward(B, c)


@pytest.mark.parametrize("row", [ROW1079, ROW2300], ids=["row1079", "row2300"])
def test_table1_768x512_vs_oracle(B, row):
    c = CS.make("t1_768x512", 512, 768, row, seeds=(10, 11, 12, 13), n_blobs=200)
    check_forward(B, c)
    check_backward(B, c)


def test_decode_synth_shared(B):
    c = _case("row545_64x64", 64, 64, ROW545, False)
    p = _problem(B, c)
    yq = np.rint(c.y)
    xhat = torch.zeros(3 * c.H * c.W, device="cuda")
    B.coolchic_decode_synth(p, _dev(yq), _dev(c.ups), _dev(c.syn), xhat)
    torch.cuda.synchronize()
    ref = O.forward(O.Arch(*c.arch), c.img, yq, c.arm, c.ups, c.syn, c.lam)["xhat"]
    got = xhat.cpu().numpy().reshape(3, c.H, c.W)
    assert np.allclose(got, ref, rtol=0, atol=1e-5 * max(1.0, np.max(np.abs(ref))))


@pytest.mark.parametrize("arch", [ROW300, (7, 8, 2, 4, 16, 1, 0), ROW2300], ids=["shared4", "separable4", "shared8"])
def test_train_step_matches_backward_then_adam(B, arch):
    """The fused training step with the shared / 4-tap upsampler (its tap
    gradient reduced from the padded 8-tap partials) against
    coolchic_backward + coolchic_adam_step, bit for bit, over two steps."""
    c = _case("ts", 64, 64, arch, False)
    p = _problem(B, c)
    n = CS.n_latents(c.H, c.W, c.arch[0])
    na, nu, ns = CS.sizes(c.arch)
    theta0 = np.concatenate([c.y, c.arm, c.ups, c.syn]).astype(np.float32)
    img = _dev(c.img)
    st = [dict(th=_dev(theta0), g=torch.zeros(theta0.size, device="cuda"), m=torch.zeros(theta0.size, device="cuda"),
               v=torch.zeros(theta0.size, device="cuda"), step=torch.zeros(2, dtype=torch.int32, device="cuda"),
               loss=torch.zeros(4, device="cuda")) for _ in range(2)]
    for _ in range(2):
        a = st[0]
        B.coolchic_train_step(p, img, None, 1.0, a["loss"], a["th"], a["g"], a["m"], a["v"], a["step"])
        b = st[1]
        th = b["th"]
        views = lambda t: (t[:n], t[n:n + na], t[n + na:n + na + nu], t[n + na + nu:])  # noqa: E731
        y, arm, ups, syn = views(th)
        gy, ga, gu, gs = views(b["g"])
        B.coolchic_backward(p, img, y.clone(), None, arm.clone(), ups.clone(), syn.clone(), 1.0, b["loss"], gy, ga,
                            gu, gs)
        B.coolchic_adam_step(th, b["g"], b["m"], b["v"], b["step"])
    torch.cuda.synchronize()
    for k in ("th", "g", "m", "v", "loss", "step"):
        assert torch.equal(st[0][k], st[1][k]), k
    # and the first iteration's gradient is the oracle's
    ref = O.backward(O.Arch(*c.arch), c.img, c.y, c.arm, c.ups, c.syn, c.lam)
    out = gpu_backward(B, c)
    assert np.linalg.norm(out["g_ups"] - ref["g_ups"]) <= 1e-3 * np.linalg.norm(ref["g_ups"])


def test_batch_shared_matches_single_images(B):
    """The batched pass with the shared 8 x 8 upsampler gives, image by image,
    what coolchic_backward gives (default launch shape: bit-identical)."""
    arch = ROW2300
    sizes = [(64, 64), (128, 64), (64, 192)]
    cs = [_case(f"b{k}", H, W, arch, False, seed=70 + 4 * k) for k, (H, W) in enumerate(sizes)]
    probs = [_problem(B, c) for c in cs]
    io, outs = [], []
    for c in cs:
        n = CS.n_latents(c.H, c.W, c.arch[0])
        na, nu, ns = CS.sizes(c.arch)
        d = dict(img=_dev(c.img), y=_dev(c.y), arm_w=_dev(c.arm), ups_w=_dev(c.ups), syn_w=_dev(c.syn),
                 loss4=torch.zeros(4, device="cuda"), g_y=torch.zeros(n, device="cuda"),
                 g_arm=torch.zeros(na, device="cuda"), g_ups=torch.zeros(nu, device="cuda"),
                 g_syn=torch.zeros(ns, device="cuda"))
        io.append(d)
    plan = B.BatchPlan(probs, io)
    plan.backward()
    torch.cuda.synchronize()
    for c, d in zip(cs, io):
        ref = gpu_backward(B, c)
        for k, key in (("g_y", "g_y"), ("g_arm", "g_arm"), ("g_ups", "g_ups"), ("g_syn", "g_syn")):
            assert np.array_equal(d[k].cpu().numpy(), ref[key]), (c.name, k)
        assert np.array_equal(d["loss4"].cpu().numpy(), ref["loss4"])
