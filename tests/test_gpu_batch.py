"""Batched overfitting on the GPU: the batched C ABI against single-image calls
and the FP64 oracle, HIP-graph replay against eager iterations, and the
autotuner."""
import numpy as np
import pytest
import torch

import oracle as O
from tests import cases as CS
from tests.test_gpu_parity import assert_grad_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_11651_amd import binding
    return binding


@pytest.fixture(scope="module")
def BT():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_11651_amd import batch
    return batch


SMALL_SIZES = [(64, 128), (128, 64), (192, 128), (64, 64)]


def batch_cases(arch, sizes, seed0=100):
    return [CS.make(f"b{k}", H, W, arch, seeds=(seed0 + 4 * k, seed0 + 4 * k + 1, seed0 + 4 * k + 2, 0),
                    n_blobs=max(3, H * W // 2048)) for k, (H, W) in enumerate(sizes)]


def make_encoder(B, BT, cs, tune=(0, 0, 0, 0)):
    probs = [B.Problem(c.H, c.W, B.Arch(*c.arch), B.CC_QUANT_ROUND, c.lam) for c in cs]
    return BT.BatchEncoder(probs, [c.img for c in cs], [c.y for c in cs], [(c.arm, c.ups, c.syn) for c in cs],
                           tune=tune)


def single(B, c):
    p = B.Problem(c.H, c.W, B.Arch(*c.arch), B.CC_QUANT_ROUND, c.lam)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    na, nu, ns = CS.sizes(c.arch)
    loss4 = torch.zeros(4, device="cuda")
    g = [torch.full((k,), float("nan"), device="cuda") for k in (c.y.size, na, nu, ns)]
    B.coolchic_backward(p, d(c.img), d(c.y), None, d(c.arm), d(c.ups), d(c.syn), 1.0, loss4, *g)
    torch.cuda.synchronize()
    return loss4.cpu().numpy(), [t.cpu().numpy() for t in g]


def check_vs_oracle(c, loss4, grads):
    ref = O.backward(O.Arch(*c.arch), c.img, c.y, c.arm, c.ups, c.syn, c.lam)
    assert loss4[3] == 0.0
    assert abs(loss4[0] - ref["loss"]) <= 1e-5 * abs(ref["loss"]), (loss4, ref["loss"])
    for name, g in zip(("g_y", "g_arm", "g_ups", "g_syn"), grads):
        assert_grad_close(f"{c.name}.{name}", g, ref[name])


def coarse_masks(c):
    """Masks of g_y and g_ups over what a single image's coarse upsampling
    adjoint sums in another order than the batch's step-by-step chain: with
    a separable upsampler and L >= 5 levels, coolchic_backward takes the
    gradients at the outputs of steps 3 .. L-2 from the composed adjoint of
    steps 1 .. s-1, so latent levels >= 4 and the taps of steps >= 3 differ
    by rounding only."""
    L, taps = c.arch[0], c.arch[3]
    my = np.zeros(c.y.size, bool)
    mu = np.zeros(CS.sizes(c.arch)[1], bool)
    if L >= 5:
        off = sum((c.H >> l) * (c.W >> l) for l in range(4))
        my[off:] = True
        mu[3 * 2 * taps:] = True
    return my, mu


@pytest.mark.parametrize("arch,tile", [(CS.LOW, 0), (CS.FULL, 0), (CS.LOW, 16)], ids=["low", "full", "low_tile16"])
def test_batch_default_equals_single_calls(B, BT, arch, tile):
    """With the default launch shape the batched pass runs the same blocks
    over the same tiles as one coolchic_backward per image: bit-identical,
    except where the single image's composed coarse adjoint sums in another
    order (coarse_masks): there within 1e-5 of the gradient's 2-norm.  The
    upsampling forward's tile side only changes which work-group computes
    an output, not its arithmetic: bit-identical too."""
    cs = batch_cases(arch, SMALL_SIZES)
    enc = make_encoder(B, BT, cs, tune=(0, 0, 0, tile))
    enc.backward()
    torch.cuda.synchronize()
    L = enc.loss.cpu().numpy()
    for k, c in enumerate(cs):
        l4, g = single(B, c)
        assert np.array_equal(L[k], l4), (k, L[k], l4)
        my, mu = coarse_masks(c)
        for name, a, b, msk in zip(("g_y", "g_arm", "g_ups", "g_syn"), enc.grads(k), g,
                                   (my, None, mu, None)):
            if msk is None:
                assert np.array_equal(a, b), (k, name)
                continue
            assert np.array_equal(a[~msk], b[~msk]), (k, name)
            d = np.linalg.norm((a - b)[msk].astype(np.float64))
            assert d <= 1e-5 * np.linalg.norm(b[msk].astype(np.float64)), (k, name, d)


@pytest.mark.parametrize("tune", [(0, 0, 0), (7, 5, 0), (4096, 4096, 0), (0, 0, 1), (512, 2048, 1), (0, 0, 2),
                                  (1024, 512, 2), (7, 5, 1, 16), (0, 0, 2, 32)])
def test_batch_vs_oracle(B, BT, tune):
    cs = batch_cases(CS.LOW, SMALL_SIZES, seed0=200)
    enc = make_encoder(B, BT, cs, tune=tune)
    enc.backward()
    torch.cuda.synchronize()
    L = enc.loss.cpu().numpy()
    for k, c in enumerate(cs):
        check_vs_oracle(c, L[k], enc.grads(k))


@pytest.mark.parametrize("tune", [(0, 0, 3), (0, 0, 0, 24), (0, 0, 0, 64)])
def test_batch_rejects_unknown_arm_order_or_tile(B, BT, tune):
    cs = batch_cases(CS.LOW, SMALL_SIZES[:2], seed0=210)
    with pytest.raises(B.CoolChicError):
        make_encoder(B, BT, cs, tune=tune)


def test_batch_full_arch_vs_oracle(B, BT):
    cs = batch_cases(CS.FULL, [(64, 192), (128, 128)], seed0=300)
    enc = make_encoder(B, BT, cs, tune=(37, 11, 1))
    enc.backward()
    torch.cuda.synchronize()
    L = enc.loss.cpu().numpy()
    for k, c in enumerate(cs):
        check_vs_oracle(c, L[k], enc.grads(k))


def test_batch_adam_step_matches_oracle(B, BT):
    """One batched iteration (backward + one Adam launch over every image):
    the gradients against the oracle's, and the updated parameters against
    the oracle's Adam applied to those gradients."""
    cs = batch_cases(CS.LOW, SMALL_SIZES[:2], seed0=400)
    enc = make_encoder(B, BT, cs)
    enc.step()
    torch.cuda.synchronize()
    L = enc.loss.cpu().numpy()
    for k, c in enumerate(cs):
        grads = enc.grads(k)
        check_vs_oracle(c, L[k], grads)
        th = np.concatenate([c.y, c.arm, c.ups, c.syn]).astype(np.float64)
        g = np.concatenate(grads).astype(np.float64)
        z = np.zeros_like(th)
        th1, _, _ = O.adam_step(th, g, z, z.copy(), 1)
        got = np.concatenate(enc.params(k)).astype(np.float64)
        assert np.max(np.abs(got - th1)) <= 1e-6 + 2e-7 * np.max(np.abs(th)), k


def test_noise_kernel_matches_oracle_philox(B):
    from oracle import noise as NZ
    u = torch.full((1001,), float("nan"), device="cuda")
    step = torch.tensor([7, 0], dtype=torch.int32, device="cuda")
    B.coolchic_uniform_noise(u, (5 << 32) | 123, step=step, stream_id=3)
    ref = NZ.uniform_noise(1001, (5 << 32) | 123, it=7, stream_id=3)
    assert np.array_equal(u.cpu().numpy(), ref)
    B.coolchic_uniform_noise(u, 9)
    assert np.array_equal(u.cpu().numpy(), NZ.uniform_noise(1001, 9))


def test_batch_noise_mode_vs_oracle(B, BT):
    """Noise proxy: the batched pass draws u on the device; the oracle takes
    the same u from its own Philox generator."""
    from oracle import noise as NZ
    cs = batch_cases(CS.LOW, SMALL_SIZES[:3], seed0=800)
    enc = make_encoder(B, BT, cs)
    enc.noise_seed = 77
    enc.set_mode(B.CC_QUANT_NOISE)
    enc.backward()
    torch.cuda.synchronize()
    # the encoder's noise buffer: each image's noise, then one float (the
    # soft proxy's sharpness slot)
    u_all = NZ.uniform_noise(sum(c.y.size + 1 for c in cs), 77, it=0)
    L = enc.loss.cpu().numpy()
    o = 0
    for k, c in enumerate(cs):
        u = u_all[o:o + c.y.size]
        o += c.y.size + 1
        ref = O.backward(O.Arch(*c.arch), c.img, c.y, c.arm, c.ups, c.syn, c.lam, u=u)
        assert abs(L[k, 0] - ref["loss"]) <= 1e-5 * abs(ref["loss"])
        for name, g in zip(("g_y", "g_arm", "g_ups", "g_syn"), enc.grads(k)):
            assert_grad_close(f"{k}.{name}", g, ref[name])


@pytest.mark.parametrize("mode", ["round", "noise"])
def test_graph_replays_match_eager(B, BT, mode):
    """Every replay of a captured block of iterations equals the same number of
    eager iterations, with unrelated eager work and synchronisations between
    the replays (noise mode: fresh noise every iteration from the device step
    counter)."""
    cs = batch_cases(CS.LOW, SMALL_SIZES[:3], seed0=500)
    eager = make_encoder(B, BT, cs)
    graphed = make_encoder(B, BT, cs)
    if mode == "noise":
        eager.set_mode(B.CC_QUANT_NOISE)
        graphed.set_mode(B.CC_QUANT_NOISE)
    g = graphed.capture(3)
    scratch = torch.randn(1 << 16, device="cuda")
    for r in range(4):
        for _ in range(3):
            eager.step()
        g.replay()
        scratch = torch.tanh(scratch * 1.01) + scratch.sum() * 0.0  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(eager.theta, graphed.theta), r
        assert torch.equal(eager.loss, graphed.loss), r
        assert torch.equal(eager.step_ctr, graphed.step_ctr), r
    assert int(graphed.step_ctr[0]) == 12


def test_training_lowers_every_loss(B, BT):
    cs = batch_cases(CS.LOW, SMALL_SIZES, seed0=600)
    enc = make_encoder(B, BT, cs)
    enc.backward()
    torch.cuda.synchronize()
    l0 = enc.loss[:, 0].cpu().numpy().copy()
    enc.fit(100, noise_frac=0.6, graph_steps=20)
    assert enc.mode == B.CC_QUANT_ROUND and int(enc.step_ctr[0]) == 100
    enc.backward()
    torch.cuda.synchronize()
    l1 = enc.loss.cpu().numpy()
    assert np.all(l1[:, 3] == 0.0)
    assert np.all(l1[:, 0] < 0.8 * l0), (l0, l1[:, 0])


def test_autotune_restores_state_and_caches(B, BT, tmp_path, monkeypatch):
    monkeypatch.setenv("COOLCHIC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    cs = batch_cases(CS.LOW, SMALL_SIZES, seed0=700)
    enc = make_encoder(B, BT, cs)
    before = enc.theta.clone()
    res = BT.autotune(enc, iters=2, reps=1)
    assert not res["cached"]
    assert tuple(res["tune"]) in {(a, s, f, t) for a in BT.ARM_CANDIDATES for s in BT.SYN_CANDIDATES
                                  for f in BT.ARM_FIRST_CANDIDATES for t in BT.UPS_TILE_CANDIDATES}
    assert enc.tune == tuple(res["tune"])
    assert torch.equal(enc.theta, before)
    assert int(enc.step_ctr[0]) == 0
    again = BT.autotune(enc)
    assert again["cached"] and again["tune"] == res["tune"]
    # the tuned plan still matches the oracle
    enc.backward()
    torch.cuda.synchronize()
    check_vs_oracle(cs[3], enc.loss[3].cpu().numpy(), enc.grads(3))


def test_bench_batch_sampled(B, BT):
    """At the benchmark's size (32 images, 256x256 .. 1024x768, low-complexity
    decoder) under an explicit tuned launch shape: every image's loss and
    gradient against its own single-image call (reordered sums only), and
    the smallest image against the oracle."""
    from bench import batch_inputs
    probs, images, y0, params0 = batch_inputs(B)
    enc = BT.BatchEncoder(probs, images, y0, params0, tune=(2048, 1024))
    enc.backward()
    torch.cuda.synchronize()
    L = enc.loss.cpu().numpy()
    assert np.all(L[:, 3] == 0.0)
    k_small = int(np.argmin([p.H * p.W for p in probs]))
    for k, p in enumerate(probs):
        a, u, s = params0[k]
        c = CS.Case(f"bench{k}", p.H, p.W, CS.LOW, images[k], y0[k], None, a, u, s, p.lam)
        l4, g = single(B, c)
        assert abs(L[k, 0] - l4[0]) <= 1e-6 * abs(l4[0]), k
        for name, ga, gb in zip(("g_y", "g_arm", "g_ups", "g_syn"), enc.grads(k), g):
            assert_grad_close(f"{k}.{name}", ga, gb.astype(np.float64), tol=1e-4)
        if k == k_small:
            check_vs_oracle(c, L[k], enc.grads(k))


def test_batch_soft_mode_vs_oracle(B, BT):
    """C3's soft proxy in the batch: the device noise, the sharpness from
    the encoder's device scalar, against the oracle with the same noise."""
    from oracle import noise as NZ
    cs = batch_cases(CS.LOW, SMALL_SIZES[:3], seed0=820)
    enc = make_encoder(B, BT, cs)
    enc.noise_seed = 78
    enc.set_mode(B.CC_QUANT_SOFT)
    enc.alpha.fill_(4.0)
    enc.backward()
    torch.cuda.synchronize()
    u_all = NZ.uniform_noise(sum(c.y.size + 1 for c in cs), 78, it=0)
    L = enc.loss.cpu().numpy()
    o = 0
    for k, c in enumerate(cs):
        u = u_all[o:o + c.y.size]
        o += c.y.size + 1
        ref = O.backward(O.Arch(*c.arch), c.img, c.y, c.arm, c.ups, c.syn, c.lam, u=u, soft_alpha=4.0)
        assert abs(L[k, 0] - ref["loss"]) <= 1e-5 * abs(ref["loss"])
        for name, g in zip(("g_y", "g_arm", "g_ups", "g_syn"), enc.grads(k)):
            assert_grad_close(f"{k}.{name}", g, ref[name])


def test_fit_soft_schedule_runs_and_lowers_the_loss(B, BT):
    """The soft-proxy schedule (annealed sharpness in graph replays, then
    rounding) trains: the rounding-mode loss falls, and stays finite."""
    cs = batch_cases(CS.LOW, SMALL_SIZES[:3], seed0=840)
    enc = make_encoder(B, BT, cs)
    enc.probe()
    torch.cuda.synchronize()
    l0 = enc.loss.cpu().numpy()[:, 0].copy()
    enc.fit(100, noise_frac=0.6, graph_steps=20, proxy="soft")
    enc.probe()
    torch.cuda.synchronize()
    l1 = enc.loss.cpu().numpy()
    assert np.all(np.isfinite(l1[:, 0])) and np.all(l1[:, 3] == 0.0)
    assert np.all(l1[:, 0] < l0)
