"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/coolchic.h declares, and rejects invalid arguments with
the documented codes before anything is enqueued."""
import ctypes
import os
import re

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_2403_11651_amd import binding
    return binding


def test_exports_every_declared_symbol(B):
    hdr = open(os.path.join(ROOT, "include", "coolchic.h")).read()
    declared = set(re.findall(r"\b(coolchic_\w+)\s*\(", hdr))
    assert declared == set(B.EXPORTS)
    for name in declared:
        assert hasattr(B.lib, name), name


def test_param_counts_match_oracle(B):
    for arch in [(7, 24, 2, 8, 40, 2), (7, 8, 2, 8, 16, 1), (5, 16, 3, 8, 48, 2), (2, 8, 1, 8, 8, 1)]:
        assert B.param_count(B.Arch(*arch)) == O.param_sizes(O.Arch(*arch))


def test_table1_param_counts_through_the_c_abi(B):
    """Table I's four decoders (shared K x K upsampler): 281 / 525 / 941 /
    1925 parameters, as the oracle counts them from the paper's layers."""
    rows = {300: (7, 8, 1, 4, 8, 1, 1), 545: (7, 8, 2, 4, 16, 2, 1), 1079: (7, 16, 2, 4, 16, 2, 1),
            2300: (7, 24, 2, 8, 40, 2, 1)}
    expect = {300: 281, 545: 525, 1079: 941, 2300: 1925}
    for k, arch in rows.items():
        assert sum(B.param_count(B.Arch(*arch))) == expect[k], k
        o = O.TABLE1[k]
        assert B.param_count(B.Arch(*arch)) == O.param_sizes(o)
    # separable 4-tap upsampler: [L-1][2][4]
    assert B.param_count(B.Arch(7, 8, 2, 4, 16, 1))[1] == 6 * 2 * 4


def test_latent_count_and_workspace(B):
    p = B.Problem(512, 768)
    assert B.latent_count(p) == 524256
    f, b, d = (B.workspace_bytes(p, w) for w in (0, 1, 2))
    assert 0 < d <= f < b
    assert B.workspace_bytes(p, 7) == 0


@pytest.mark.parametrize("H,W,arch,quant,code", [
    (100, 768, (7, 24, 2, 8, 40, 2), 0, -1),   # H not a multiple of 2^(L-1)
    (512, 760, (7, 24, 2, 8, 40, 2), 0, -1),
    (0, 768, (7, 24, 2, 8, 40, 2), 0, -1),
    (512, 768, (7, 24, 2, 8, 40, 2), 5, -1),   # unknown quantiser
    (512, 768, (7, 12, 2, 8, 40, 2), 0, -2),   # context width not compiled
    (512, 768, (7, 24, 2, 6, 40, 2), 0, -2),   # 6-tap upsampler not compiled
    (512, 768, (7, 24, 2, 8, 44, 2), 0, -2),   # hidden width not a multiple of 8
    (512, 768, (7, 24, 2, 8, 40, 3), 0, -2),   # three residual convs
    (1024, 1024, (9, 24, 2, 8, 40, 2), 0, -2),  # more than 7 levels
])
def test_invalid_problems_rejected(B, H, W, arch, quant, code):
    p = B.Problem(H, W, B.Arch(*arch), quant)
    pc = p.c()
    assert B.lib.coolchic_workspace_bytes(ctypes.byref(pc), 1) == 0
    dummy = ctypes.c_void_p(0x1000)
    rc = B.lib.coolchic_forward(ctypes.byref(pc), dummy, dummy, dummy, dummy, dummy, dummy, dummy, None, None, None,
                                dummy, 1 << 30, None)
    assert rc == code


def test_null_pointers_and_small_workspace(B):
    p = B.Problem(64, 64, B.LOW)
    pc = p.c()
    d = ctypes.c_void_p(0x1000)
    need = B.workspace_bytes(p, 0)
    # null image
    assert B.lib.coolchic_forward(ctypes.byref(pc), None, d, None, d, d, d, d, None, None, None, d, need, None) == -1
    # workspace too small
    assert B.lib.coolchic_forward(ctypes.byref(pc), d, d, None, d, d, d, d, None, None, None, d, need - 4, None) == -3
    # noise quantiser without u
    pn = B.Problem(64, 64, B.LOW, B.CC_QUANT_NOISE).c()
    assert B.lib.coolchic_forward(ctypes.byref(pn), d, d, None, d, d, d, d, None, None, None, d, need, None) == -1
    needb = B.workspace_bytes(p, 1)
    assert B.lib.coolchic_backward(ctypes.byref(pc), d, d, None, d, d, d, 1.0, d, d, d, d, d, d, needb - 1, None) == -3
    assert B.lib.coolchic_backward(ctypes.byref(pc), d, d, None, d, d, d, 1.0, d, None, d, d, d, d, needb, None) == -1
    assert B.lib.coolchic_decode_synth(ctypes.byref(pc), d, d, d, None, d, B.workspace_bytes(p, 2), None) == -1
    assert B.lib.coolchic_decode_synth(None, d, d, d, d, d, 1 << 20, None) == -1
    assert B.lib.coolchic_adam_step(d, d, d, d, 0, d, 0.01, 0.9, 0.999, 1e-8, None) == -1
    assert B.lib.coolchic_adam_step(d, d, d, d, 10, d, 0.01, 1.0, 0.999, 1e-8, None) == -1
    assert B.strerror(-3).startswith("workspace")


def _batch(B, probs):
    arr = (B.CCProblem * len(probs))(*[p.c() for p in probs])
    return arr, B.CCBatchTuning(0, 0, 0, 0)


def test_batch_workspace_bytes(B):
    a = B.Problem(256, 320, B.LOW)
    b = B.Problem(512, 768, B.LOW)
    one = B.batch_workspace_bytes([a])
    two = B.batch_workspace_bytes([a, b])
    # every image brings its own backward workspace, plus argument blocks
    assert one >= B.workspace_bytes(a, 1)
    assert two >= one + B.workspace_bytes(b, 1)
    # a larger persistent grid needs more partial-sum rows
    assert B.batch_workspace_bytes([a, b], (4096, 4096)) > B.batch_workspace_bytes([a, b], (64, 64))
    assert B.batch_workspace_bytes([a, B.Problem(512, 768, B.FULL)]) == 0  # architectures differ
    assert B.batch_workspace_bytes([a, B.Problem(100, 768, B.LOW)]) == 0  # invalid size
    arr, t = _batch(B, [a])
    assert B.lib.coolchic_batch_workspace_bytes(0, arr, ctypes.byref(t)) == 0
    assert B.lib.coolchic_batch_workspace_bytes(1, None, ctypes.byref(t)) == 0
    assert B.lib.coolchic_batch_workspace_bytes(1, arr, None) == one  # NULL tuning = default shapes
    # the upsampling forward's tile side: 16 means four times the work items of 32; others are invalid
    assert B.batch_workspace_bytes([a, b], (0, 0, 0, 32)) == two
    assert B.batch_workspace_bytes([a, b], (0, 0, 0, 16)) >= two
    for bad in (8, 24, 64, -16):
        assert B.batch_workspace_bytes([a, b], (0, 0, 0, bad)) == 0
    assert B.batch_workspace_bytes([a, b], (0, 0, 3)) == 0


def test_batch_create_argument_checks(B):
    probs = [B.Problem(64, 128, B.LOW), B.Problem(128, 64, B.LOW)]
    arr, t = _batch(B, probs)
    need = B.batch_workspace_bytes(probs)
    io = (B.CCImageIO * 2)()
    for k in range(2):
        for name, _ in B.CCImageIO._fields_:
            if name != "u":
                setattr(io[k], name, 0x1000)
    out = ctypes.c_void_p(0x1)
    ws = ctypes.c_void_p(0x1000)
    rc = B.lib.coolchic_batch_create(2, arr, io, ctypes.byref(t), 1.0, None, need, ctypes.byref(out))
    assert rc == B.CC_EINVAL and not out.value
    rc = B.lib.coolchic_batch_create(2, arr, io, ctypes.byref(t), 1.0, ws, need - 1, ctypes.byref(out))
    assert rc == B.CC_EWORKSPACE
    io[1].g_syn = None
    rc = B.lib.coolchic_batch_create(2, arr, io, ctypes.byref(t), 1.0, ws, need, ctypes.byref(out))
    assert rc == B.CC_EINVAL
    assert B.lib.coolchic_batch_create(2, arr, None, ctypes.byref(t), 1.0, ws, need, ctypes.byref(out)) == B.CC_EINVAL
    assert B.lib.coolchic_batch_backward(None, None) == B.CC_EINVAL
    B.lib.coolchic_batch_destroy(None)  # no-op


def test_warm_param_count_matches_oracle(B):
    from oracle import warmstart as WS
    for arch in (B.LOW, B.FULL, B.Arch(7, 16, 1, 8, 24, 1)):
        n_theta = sum(B.param_count(arch))
        assert B.warm_param_count(arch) == WS.WarmLayout(n_theta).size
    assert B.lib.coolchic_warm_param_count(ctypes.byref(B.Arch(7, 12, 2, 8, 16, 1).c())) == -1


def test_warm_workspace_and_invalid_problems(B):
    ws = lambda wp, w: B.lib.coolchic_warm_workspace_bytes(ctypes.byref(wp.c()), w)
    ok = B.WarmProblem(512, 768, 4)
    f, b = ws(ok, 0), ws(ok, 1)
    assert 0 < f < b
    assert ws(B.WarmProblem(512, 768, 8), 1) > b
    for bad in (B.WarmProblem(500, 768, 1), B.WarmProblem(512, 760, 1), B.WarmProblem(512, 768, 0),
                B.WarmProblem(512, 768, 1, B.Arch(6, 8, 2, 8, 16, 1)), B.WarmProblem(8192, 8192, 64)):
        assert ws(bad, 1) == 0
    assert ws(ok, 2) == 0
    d = ctypes.c_void_p(0x1000)
    pc = ok.c()
    assert B.lib.coolchic_warm_forward(ctypes.byref(pc), d, d, d, None, d, f, None) == B.CC_EINVAL
    assert B.lib.coolchic_warm_forward(ctypes.byref(pc), d, d, d, d, d, f - 1, None) == B.CC_EWORKSPACE
    assert B.lib.coolchic_warm_backward(ctypes.byref(pc), d, d, d, d, d, None, d, b, None) == B.CC_EINVAL
    assert B.lib.coolchic_warm_backward(ctypes.byref(pc), d, d, d, d, d, d, d, b - 1, None) == B.CC_EWORKSPACE


def test_timing_event_null_arguments(B):
    d = ctypes.c_void_p(0x1000)
    ms = ctypes.c_float()
    assert B.lib.coolchic_timing_event_create(None) == -1
    assert B.lib.coolchic_timing_event_elapsed(None, d, ctypes.byref(ms)) == -1
    assert B.lib.coolchic_timing_event_elapsed(d, d, None) == -1
    assert B.lib.coolchic_timing_event_destroy(None) == -1


def test_train_step_rejects_invalid_arguments(B):
    p = B.Problem(64, 64, B.LOW)
    pc = p.c()
    d = ctypes.c_void_p(0x1000)
    need = B.workspace_bytes(p, 1)
    args = lambda theta, b1: (ctypes.byref(pc), d, None, ctypes.c_float(1.0), d, theta, d, d, d, d,
                              ctypes.c_float(0.01), ctypes.c_float(b1), ctypes.c_float(0.999), ctypes.c_float(1e-8),
                              d, need, None)
    assert B.lib.coolchic_train_step(*args(None, 0.9)) == -1     # null theta
    assert B.lib.coolchic_train_step(*args(d, 1.0)) == -1        # beta1 outside [0, 1)
    assert B.lib.coolchic_train_step(None, *args(d, 0.9)[1:]) == -1
    small = list(args(d, 0.9))
    small[15] = need - 4                                          # workspace too small
    assert B.lib.coolchic_train_step(*small) == -3


def test_train_step_noalloc_rejects_before_touching_the_device(B):
    """The allocation-free training step refuses, with the documented codes
    and before any HIP call, a problem whose backward workspace exceeds the
    static scratch (CC_ESCRATCH), an invalid problem and bad arguments."""
    d = ctypes.c_void_p(0x1000)

    def call(p, theta=d, b1=0.9):
        pc = p.c() if p is not None else None
        return B.lib.coolchic_train_step_noalloc(None if pc is None else ctypes.byref(pc), d, None,
                                                 ctypes.c_float(1.0), d, theta, d, d, d, d, ctypes.c_float(0.01),
                                                 ctypes.c_float(b1), ctypes.c_float(0.999), ctypes.c_float(1e-8), None)

    big = B.Problem(2048, 2048, B.FULL)
    assert B.workspace_bytes(big, 1) > B.CC_NOALLOC_SCRATCH_BYTES
    assert call(big) == B.CC_ESCRATCH
    assert "static scratch" in B.strerror(B.CC_ESCRATCH)
    assert call(None) == -1
    assert call(B.Problem(100, 768, B.FULL)) == -1                 # H not a multiple of 2^(L-1)
    assert call(B.Problem(512, 768, B.Arch(7, 12, 2, 8, 40, 2))) == -2
    fits = B.Problem(512, 768, B.FULL)
    assert B.workspace_bytes(fits, 1) <= B.CC_NOALLOC_SCRATCH_BYTES
    assert call(fits, theta=None) == -1
    assert call(fits, b1=1.0) == -1


def test_batch_refuses_four_tap_upsamplers(B):
    """The batched entry points run 8-tap upsamplers only: a 4-tap
    architecture gets no workspace size and no plan."""
    p = B.Problem(64, 64, B.Arch(7, 8, 1, 4, 8, 1, 1))
    assert B.batch_workspace_bytes([p]) == 0
    q = B.Problem(64, 64, B.Arch(7, 24, 2, 8, 40, 2, 1))
    assert B.batch_workspace_bytes([q]) > 0


def test_analysis_sizes_and_argument_checks(B):
    """The analysis transform's host checks (no device work): parameter count
    of the oracle's layout, workspace sizes, and the sizes it refuses."""
    import oracle.analysis as A
    assert B._lib.coolchic_analysis_param_count() == A.param_count()
    one = B._lib.coolchic_analysis_workspace_bytes(512, 768, 1)
    assert one > 2 * 512 * 768 * 64 * 2  # two bfloat16 feature buffers at level-0 size
    assert B._lib.coolchic_analysis_workspace_bytes(512, 768, 8) > 7 * one
    for H, W, n in [(64, 96, 1), (96, 64, 1), (0, 64, 1), (64, 64, 0), (64, 64, -1), (32768, 32768, 2)]:
        assert B._lib.coolchic_analysis_workspace_bytes(H, W, n) == 0, (H, W, n)
    assert B._lib.coolchic_analysis_workspace_bytes(32768, 32704, 2) > 0  # n H W just below 2^31
    d = 0x1000
    assert B._lib.coolchic_analysis_forward(64, 64, 1, None, d, d, d, 1 << 30, None) == B.CC_EINVAL
    assert B._lib.coolchic_analysis_forward(64, 64, 1, d, d, d, None, 1 << 30, None) == B.CC_EINVAL
    assert B._lib.coolchic_analysis_forward(32768, 32768, 2, d, d, d, d, 1 << 62, None) == B.CC_EINVAL
    assert B._lib.coolchic_analysis_forward(64, 64, 1, d, d, d, d, 16, None) == B.CC_EWORKSPACE
