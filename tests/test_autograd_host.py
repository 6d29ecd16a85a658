"""CPU check of the CoolChicFn wrapper's plumbing (argument order, the scale
of the incoming gradient, which inputs get gradients) with
torch.autograd.gradcheck.  The library calls it makes are replaced, inside
this test only, by stand-ins that evaluate the FP64 oracle, so gradcheck
compares the wrapper's backward with central differences of its forward on
the 16x16, 5-level instance in the noise mode."""
import numpy as np
import pytest
import torch

import oracle as O
from tests import cases as CS


@pytest.fixture()
def fn(monkeypatch):
    from paper_2403_11651_amd import autograd as AG

    def arch_of(p):
        a = p.arch
        return O.Arch(a.n_levels, a.arm_ctx, a.arm_layers, a.ups_taps, a.syn_hidden, a.syn_res)

    def img3(p, img):
        return img.detach().numpy().reshape(3, p.H, p.W)

    def fake_forward(p, img, y, u, arm, ups, syn, loss4, *rest, **kw):
        r = O.forward(arch_of(p), img3(p, img), y.detach().numpy(), arm.detach().numpy(), ups.detach().numpy(),
                      syn.detach().numpy(), p.lam, u=None if u is None else u.numpy())
        loss4.copy_(torch.tensor([r["loss"], r["D"], r["R"], 0.0], dtype=loss4.dtype))

    def fake_backward(p, img, y, u, arm, ups, syn, dloss, loss4, g_y, g_arm, g_ups, g_syn, *rest, **kw):
        r = O.backward(arch_of(p), img3(p, img), y.numpy(), arm.numpy(), ups.numpy(), syn.numpy(), p.lam,
                       u=None if u is None else u.numpy(), dloss=dloss)
        loss4.copy_(torch.tensor([r["loss"], r["D"], r["R"], 0.0], dtype=loss4.dtype))
        for dst, key in ((g_y, "g_y"), (g_arm, "g_arm"), (g_ups, "g_ups"), (g_syn, "g_syn")):
            dst.copy_(torch.from_numpy(r[key]))

    monkeypatch.setattr(AG.B, "coolchic_forward", fake_forward)
    monkeypatch.setattr(AG.B, "coolchic_backward", fake_backward)
    monkeypatch.setattr(AG, "_f32", lambda t, name: t.contiguous())
    return AG


def test_coolchicfn_gradcheck_against_finite_differences(fn):
    from paper_2403_11651_amd import binding as B
    c = CS.small_variants()[0]  # 16x16, 5 levels, noise mode (the loss is smooth in y)
    p = B.Problem(c.H, c.W, B.Arch(*c.arch), B.CC_QUANT_NOISE, c.lam)
    t = lambda a, g=True: torch.tensor(np.asarray(a, np.float64), requires_grad=g)  # noqa: E731
    img, u = t(c.img.ravel(), False), t(c.u, False)
    y, arm, ups, syn = t(c.y), t(c.arm), t(c.ups), t(c.syn)

    def f(y, arm, ups, syn):
        return 2.5 * fn.CoolChicFn.apply(p, img, u, y, arm, ups, syn)

    assert torch.autograd.gradcheck(f, (y, arm, ups, syn), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_coolchicfn_round_mode_passes_no_noise(fn):
    """Rounding mode: u is ignored (None reaches the library), and the image
    and noise receive no gradient."""
    from paper_2403_11651_amd import binding as B
    c = CS.tiny()
    p = B.Problem(c.H, c.W, B.Arch(*c.arch), B.CC_QUANT_ROUND, c.lam)
    t = lambda a, g=True: torch.tensor(np.asarray(a, np.float64), requires_grad=g)  # noqa: E731
    img = t(c.img.ravel())
    y, arm, ups, syn = t(c.y), t(c.arm), t(c.ups), t(c.syn)
    loss = fn.coolchic_loss(p, img, y, arm, ups, syn, u=t(np.zeros(c.y.size)))
    loss.backward()
    ref = O.backward(O.Arch(*c.arch), c.img, c.y, c.arm, c.ups, c.syn, c.lam)
    assert abs(float(loss) - ref["loss"]) < 1e-12
    assert img.grad is None
    assert np.array_equal(y.grad.numpy(), ref["g_y"])
