"""GPU parity of C3's quantisation proxy (CC_QUANT_SOFT): y_hat = s(s(y) +
u), s the soft rounding of sharpness alpha stored after the noise, through
the C ABI against the FP64 oracle at the bars of the other parity tests
(y_hat within FP32 rounding, per-latent rate, loss 1e-5, every gradient
tensor and latent level 1e-3), and the fused training step against
backward + Adam, bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
from tests import cases as CS
from tests.test_gpu_parity import assert_grad_close, assert_rate_close, _dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_11651_amd import binding
    return binding


def _case(which):
    if which == "tiny":
        return CS.make("soft64", 64, 64, CS.TINY, seeds=(0, 1, 2, 4), noise=True), 3.0
    if which == "ragged_c24":
        return CS.make("soft_r", 64, 192, (7, 24, 2, 8, 40, 2), seeds=(20, 21, 22, 23), noise=True), 10.0
    if which == "L1":
        return CS.make("soft_l1", 16, 40, (1, 8, 2, 8, 16, 1), seeds=(40, 41, 42, 43), n_blobs=3, noise=True), 5.0
    if which == "row1079":
        return CS.make("soft_t1", 64, 64, (7, 16, 2, 4, 16, 2, 1), seeds=(50, 51, 52, 53), noise=True), 4.0
    return CS.make("soft768", 512, 768, CS.FULL, seeds=(10, 11, 12, 13), n_blobs=200, noise=True), 5.0


def _u(c, alpha):
    return _dev(np.concatenate([c.u, [alpha]]))


@pytest.mark.parametrize("which", ["tiny", "ragged_c24", "L1", "row1079", "full768x512"])
def test_soft_forward_backward_vs_oracle(B, which):
    c, a = _case(which)
    p = B.Problem(c.H, c.W, B.Arch(*c.arch), B.CC_QUANT_SOFT, c.lam)
    n = CS.n_latents(c.H, c.W, c.arch[0])
    na, nu, ns = CS.sizes(c.arch)
    u = _u(c, a)
    loss4 = torch.zeros(4, device="cuda")
    rate = torch.zeros(n, device="cuda")
    yq = torch.zeros(n, device="cuda")
    B.coolchic_forward(p, _dev(c.img), _dev(c.y), u, _dev(c.arm), _dev(c.ups), _dev(c.syn), loss4, rate, yq)
    g = [torch.full((k,), float("nan"), device="cuda") for k in (n, na, nu, ns)]
    l4b = torch.zeros(4, device="cuda")
    B.coolchic_backward(p, _dev(c.img), _dev(c.y), u, _dev(c.arm), _dev(c.ups), _dev(c.syn), 1.0, l4b, *g)
    torch.cuda.synchronize()
    ref = O.backward(O.Arch(*c.arch), c.img, c.y, c.arm, c.ups, c.syn, c.lam, u=c.u, soft_alpha=a)
    assert np.allclose(yq.cpu().numpy(), ref["yq"], rtol=0, atol=2e-6 * max(1.0, np.max(np.abs(ref["yq"]))))
    assert_rate_close(rate.cpu().numpy(), ref)
    for l4 in (loss4.cpu().numpy(), l4b.cpu().numpy()):
        assert l4[3] == 0.0 and abs(l4[0] - ref["loss"]) <= 1e-5 * abs(ref["loss"]), (l4, ref["loss"])
    for k, t in zip(("g_y", "g_arm", "g_ups", "g_syn"), g):
        assert_grad_close(k, t.cpu().numpy(), ref[k])
    o = 0
    gy = g[0].cpu().numpy()
    for lv in range(c.arch[0]):
        m = (c.H >> lv) * (c.W >> lv)
        assert_grad_close(f"g_y[{lv}]", gy[o:o + m], ref["g_y"][o:o + m])
        o += m


def test_soft_train_step_matches_backward_then_adam(B):
    c, a = _case("tiny")
    p = B.Problem(c.H, c.W, B.Arch(*c.arch), B.CC_QUANT_SOFT, c.lam)
    n = CS.n_latents(c.H, c.W, c.arch[0])
    na, nu, ns = CS.sizes(c.arch)
    theta0 = np.concatenate([c.y, c.arm, c.ups, c.syn]).astype(np.float32)
    img, u = _dev(c.img), _u(c, a)
    st = [dict(th=_dev(theta0), g=torch.zeros(theta0.size, device="cuda"), m=torch.zeros(theta0.size, device="cuda"),
               v=torch.zeros(theta0.size, device="cuda"), step=torch.zeros(2, dtype=torch.int32, device="cuda"),
               loss=torch.zeros(4, device="cuda")) for _ in range(2)]
    for _ in range(2):
        x = st[0]
        B.coolchic_train_step(p, img, u, 1.0, x["loss"], x["th"], x["g"], x["m"], x["v"], x["step"])
        x = st[1]
        views = lambda t: (t[:n], t[n:n + na], t[n + na:n + na + nu], t[n + na + nu:])  # noqa: E731
        y, arm, ups, syn = views(x["th"])
        B.coolchic_backward(p, img, y.clone(), u, arm.clone(), ups.clone(), syn.clone(), 1.0, x["loss"],
                            *views(x["g"]))
        B.coolchic_adam_step(x["th"], x["g"], x["m"], x["v"], x["step"])
    torch.cuda.synchronize()
    for k in ("th", "g", "m", "v", "loss", "step"):
        assert torch.equal(st[0][k], st[1][k]), k
