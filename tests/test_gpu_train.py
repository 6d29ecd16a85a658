"""GPU: the optimiser and the autograd wrapper against the FP64 oracle.

* coolchic_adam_step over several steps of changing gradients, with the
  default and with other betas: parameters, both moments and the step
  counter (the betas only show from the second step on).
* coolchic_train_step (Adam fused into the gradient reductions) over three
  iterations in the noise mode against the oracle's backward + Adam: the
  gradients then depend on the parameters, so a large eps keeps the update
  Lipschitz in the gradient and the comparison well conditioned.
* A ten-iteration trajectory of the 64x64 workload (rounding, default Adam):
  the loss of every iteration within 1e-3 relative of the oracle's.
* CoolChicFn: loss.backward() through the torch.autograd.Function gives the
  oracle's gradients at the 1e-3 bar.
"""
import numpy as np
import pytest
import torch

import oracle as O
from tests import cases as CS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_11651_amd import binding
    return binding


def _dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _problem(B, c):
    return B.Problem(c.H, c.W, B.Arch(*c.arch), B.CC_QUANT_NOISE if c.u is not None else B.CC_QUANT_ROUND, c.lam)


def _rel_close(name, a, ref, tol):
    a = np.asarray(a, np.float64)
    nrm = np.linalg.norm(ref)
    assert np.linalg.norm(a - ref) <= tol * nrm + 1e-30, (name, np.linalg.norm(a - ref) / max(nrm, 1e-30))
    assert np.max(np.abs(a - ref)) <= tol * np.max(np.abs(ref)) + 1e-30, (name, np.max(np.abs(a - ref)))


@pytest.mark.parametrize("betas", [(0.9, 0.999), (0.8, 0.95)])
@pytest.mark.parametrize("offset", [0, 1])
def test_adam_step_several_steps_vs_oracle(B, betas, offset):
    """Four steps with a new gradient each step; offset 1 makes the arrays
    16-byte misaligned (the kernel's scalar path), offset 0 takes the vector
    path with a ragged tail (n = 1003)."""
    rng = np.random.default_rng(31)
    n = 1003
    th0 = rng.normal(size=n).astype(np.float32)
    buf = [torch.zeros(n + offset, device="cuda") for _ in range(4)]
    th, g, m, v = (t[offset:] for t in buf)
    th.copy_(_dev(th0))
    step = torch.zeros(2, dtype=torch.int32, device="cuda")
    th_o, m_o, v_o = th0.astype(np.float64), np.zeros(n), np.zeros(n)
    lr, eps = 1e-2, 1e-8
    # the oracle takes the hyperparameters as the kernel sees them (FP32)
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    for t in range(1, 5):
        gv = (rng.normal(size=n) * (0.5 + t)).astype(np.float32)
        g.copy_(_dev(gv))
        B.coolchic_adam_step(th, g, m, v, step, lr=lr, beta1=betas[0], beta2=betas[1], eps=eps)
        th_o, m_o, v_o = O.adam_step(th_o, gv, m_o, v_o, t, lr=f32(lr), beta1=f32(betas[0]), beta2=f32(betas[1]),
                                     eps=f32(eps))
        torch.cuda.synchronize()
        assert np.allclose(m.cpu().numpy(), m_o, rtol=2e-6, atol=1e-7), t
        assert np.allclose(v.cpu().numpy(), v_o, rtol=2e-6, atol=1e-7), t
        # the update is lr * O(1): its FP32 error is a few 1e-7 of lr
        assert np.max(np.abs(th.cpu().numpy() - th_o)) <= 1e-6, t
        assert step.cpu().tolist() == [t, 0]


def test_train_step_three_iterations_vs_oracle(B):
    """coolchic_train_step x 3 on the 64x64 workload with the noise proxy and
    betas (0.8, 0.95), eps 0.1: latents and every parameter block, both
    moments, the loss of each iteration and the step counter.  The moments
    and the parameter updates are held to the gradient bar; a latent update
    can be below the FP32 resolution of the latent, so the parameters also
    get four FP32 spacings of slack."""
    c = CS.make("tiny64_noise", 64, 64, CS.TINY, seeds=(0, 1, 2, 4), noise=True)
    p = _problem(B, c)
    n = CS.n_latents(c.H, c.W, c.arch[0])
    na, nu, ns = CS.sizes(c.arch)
    theta0 = np.concatenate([c.y, c.arm, c.ups, c.syn]).astype(np.float32)
    lr, b1, b2, eps = (float(np.float32(x)) for x in (1e-2, 0.8, 0.95, 0.1))
    th = _dev(theta0)
    g = torch.zeros_like(th)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    step = torch.zeros(2, dtype=torch.int32, device="cuda")
    loss4 = torch.zeros(4, device="cuda")
    img, u = _dev(c.img), _dev(c.u)
    th_o, m_o, v_o = theta0.astype(np.float64), np.zeros(theta0.size), np.zeros(theta0.size)
    A = O.Arch(*c.arch)
    for t in range(1, 4):
        B.coolchic_train_step(p, img, u, 1.0, loss4, th, g, m, v, step, lr=lr, beta1=b1, beta2=b2, eps=eps)
        ref = O.backward(A, c.img, th_o[:n], th_o[n:n + na], th_o[n + na:n + na + nu], th_o[n + na + nu:], c.lam,
                         u=c.u)
        go = np.concatenate([ref["g_y"], ref["g_arm"], ref["g_ups"], ref["g_syn"]])
        th_new, m_o, v_o = O.adam_step(th_o, go, m_o, v_o, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
        torch.cuda.synchronize()
        l4 = loss4.cpu().numpy()
        assert l4[3] == 0.0 and abs(l4[0] - ref["loss"]) <= 1e-5 * abs(ref["loss"]), (t, l4, ref["loss"])
        got = {k: x.cpu().numpy() for k, x in (("theta", th), ("m", m), ("v", v))}
        for lo, hi, blk in ((0, n, "y"), (n, n + na, "arm"), (n + na, n + na + nu, "ups"),
                            (n + na + nu, theta0.size, "syn")):
            # the parameters (against the size of their update), and the
            # moments, block by block
            upd = np.max(np.abs(th_new[lo:hi] - theta0[lo:hi]))
            slack = 4.0 * np.spacing(np.abs(th_new[lo:hi]).astype(np.float32)).astype(np.float64)
            dth = np.abs(got["theta"][lo:hi] - th_new[lo:hi])
            assert np.all(dth <= 2e-3 * upd + slack), (t, blk, float(np.max(dth - slack)), upd)
            _rel_close(f"t{t} m {blk}", got["m"][lo:hi], m_o[lo:hi], 2e-3)
            _rel_close(f"t{t} v {blk}", got["v"][lo:hi], v_o[lo:hi], 2e-3)
        th_o = th_new
    assert step.cpu().tolist() == [3, 0]


def test_ten_iteration_trajectory_64x64(B):
    """Ten training iterations of the 64x64 workload (rounding with the
    straight-through gradient, Adam lr 1e-2, betas (0.9, 0.999)): the loss of
    each iteration within 1e-3 relative of the oracle's trajectory."""
    c = CS.tiny()
    p = _problem(B, c)
    n = CS.n_latents(c.H, c.W, c.arch[0])
    na, nu, ns = CS.sizes(c.arch)
    theta0 = np.concatenate([c.y, c.arm, c.ups, c.syn]).astype(np.float32)
    th = _dev(theta0)
    g, m, v = torch.zeros_like(th), torch.zeros_like(th), torch.zeros_like(th)
    step = torch.zeros(2, dtype=torch.int32, device="cuda")
    loss4 = torch.zeros(4, device="cuda")
    img = _dev(c.img)
    A = O.Arch(*c.arch)
    th_o, m_o, v_o = theta0.astype(np.float64), np.zeros(theta0.size), np.zeros(theta0.size)
    losses, ref_losses = [], []
    for t in range(1, 11):
        B.coolchic_train_step(p, img, None, 1.0, loss4, th, g, m, v, step)
        losses.append(loss4.clone())
        ref = O.backward(A, c.img, th_o[:n], th_o[n:n + na], th_o[n + na:n + na + nu], th_o[n + na + nu:], c.lam)
        ref_losses.append(ref["loss"])
        go = np.concatenate([ref["g_y"], ref["g_arm"], ref["g_ups"], ref["g_syn"]])
        th_o, m_o, v_o = O.adam_step(th_o, go, m_o, v_o, t)
    torch.cuda.synchronize()
    got = np.array([float(x[0]) for x in losses])
    ref = np.array(ref_losses)
    assert np.all(np.abs(got - ref) <= 1e-3 * np.abs(ref)), (got, ref)
    assert ref[-1] < ref[0]


@pytest.mark.parametrize("which", ["fd16_L5_noise", "tiny64_round"])
def test_coolchicfn_backward_matches_oracle(B, which):
    from paper_2403_11651_amd.autograd import CoolChicFn, coolchic_loss
    c = CS.small_variants()[0] if which == "fd16_L5_noise" else CS.tiny()
    p = _problem(B, c)
    y, arm, ups, syn = (_dev(a).requires_grad_(True) for a in (c.y, c.arm, c.ups, c.syn))
    loss = coolchic_loss(p, _dev(c.img), y, arm, ups, syn, u=_dev(c.u))
    (3.0 * loss).backward()
    ref = O.backward(O.Arch(*c.arch), c.img, c.y, c.arm, c.ups, c.syn, c.lam, u=c.u, dloss=3.0)
    assert abs(float(loss) - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    for name, t in (("g_y", y), ("g_arm", arm), ("g_ups", ups), ("g_syn", syn)):
        _rel_close(name, t.grad.cpu().numpy(), ref[name], 1e-3)
    assert CoolChicFn is not None


def test_train_step_graph_replay_matches_eager(B):
    """coolchic_train_step captured in a graph (under capture the ARM is forked
    after the head backward) and replayed: every replay equals the same
    number of eager steps bit for bit, with unrelated eager work and
    synchronisations between the replays (24-wide ARM, ragged 64x192)."""
    c = CS.make("ragged_L7_64x192", 64, 192, CS.FULL, seeds=(20, 21, 22, 23), noise=True)
    p = _problem(B, c)
    theta0 = np.concatenate([c.y, c.arm, c.ups, c.syn]).astype(np.float32)
    img, u = _dev(c.img), _dev(c.u)

    def state():
        th = _dev(theta0)
        return [th, torch.zeros_like(th), torch.zeros_like(th), torch.zeros_like(th),
                torch.zeros(2, dtype=torch.int32, device="cuda"), torch.zeros(4, device="cuda")]

    def step(sv):
        th, g, m, v, st, l4 = sv
        B.coolchic_train_step(p, img, u, 1.0, l4, th, g, m, v, st, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8)

    eager, graphed = state(), state()
    step(eager)  # the first calls on the device run eagerly (side stream set-up)
    step(graphed)
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        step(graphed)
        step(graphed)
    scratch = torch.randn(1 << 16, device="cuda")
    for r in range(3):
        step(eager)
        step(eager)
        gr.replay()
        scratch = torch.tanh(scratch * 1.01) + scratch.sum() * 0.0
        torch.cuda.synchronize()
        for a, b in zip(eager, graphed):
            assert torch.equal(a, b), r
    assert eager[4].cpu().tolist()[0] == 7


def test_train_steps_on_two_streams_run_concurrently_and_match(B):
    """Two problems trained on two streams, their calls interleaved without
    synchronisation (each stream has its own side stream and events): every
    state equals that of the same steps run one problem after the other.
    Then a graph captured on a fresh, prepared stream replays bit-identically
    to eager steps."""
    cases = [CS.make("ragged_L7_64x192", 64, 192, CS.FULL, seeds=(30, 31, 32, 33), noise=True),
             CS.make("small_64x128", 64, 128, CS.LOW, seeds=(34, 35, 36, 37), noise=True)]

    def state(c):
        th = _dev(np.concatenate([c.y, c.arm, c.ups, c.syn]).astype(np.float32))
        return [th, torch.zeros_like(th), torch.zeros_like(th), torch.zeros_like(th),
                torch.zeros(2, dtype=torch.int32, device="cuda"), torch.zeros(4, device="cuda")]

    probs = [_problem(B, c) for c in cases]
    inputs = [(_dev(c.img), _dev(c.u)) for c in cases]

    def step(k, sv, stream=None):
        th, g, m, v, st, l4 = sv
        B.coolchic_train_step(probs[k], inputs[k][0], inputs[k][1], 1.0, l4, th, g, m, v, st, lr=1e-2, beta1=0.9,
                              beta2=0.999, eps=1e-8, stream=stream)

    seq = [state(c) for c in cases]
    for k in range(2):
        for _ in range(4):
            step(k, seq[k])
    torch.cuda.synchronize()
    conc = [state(c) for c in cases]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for _ in range(4):
        for k in range(2):
            step(k, conc[k], streams[k])
    torch.cuda.synchronize()
    for k in range(2):
        for a, b in zip(seq[k], conc[k]):
            assert torch.equal(a, b), k

    # capture on a stream prepared beforehand (no eager call on it first)
    cap = torch.cuda.Stream()
    B.coolchic_stream_prepare(cap)
    eager, graphed = state(cases[0]), state(cases[0])
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr, stream=cap):
        step(0, graphed)
    for r in range(2):
        step(0, eager)
        gr.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, graphed):
            assert torch.equal(a, b), r
