"""ctypes binding of libcoolchic.so (include/coolchic.h).

Argument marshalling only: every function passes device pointers of torch
tensors and the current HIP stream to the C ABI of the same name; all the
arithmetic runs in the library's HIP kernels.  Importing this module fails
loudly when the library has not been built.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
from dataclasses import dataclass

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcoolchic.so")

CC_OK, CC_EINVAL, CC_EUNSUPPORTED, CC_EWORKSPACE, CC_EHIP, CC_ESCRATCH = 0, -1, -2, -3, -4, -5
CC_NOALLOC_SCRATCH_BYTES = 64 << 20
CC_QUANT_ROUND, CC_QUANT_NOISE, CC_QUANT_SOFT = 0, 1, 2
CC_WS_FORWARD, CC_WS_BACKWARD, CC_WS_DECODE = 0, 1, 2

# every symbol the header declares
EXPORTS = ("coolchic_param_count", "coolchic_latent_count", "coolchic_workspace_bytes", "coolchic_forward",
           "coolchic_backward", "coolchic_decode_synth", "coolchic_adam_step", "coolchic_set_stage_events",
           "coolchic_strerror", "coolchic_batch_workspace_bytes", "coolchic_batch_create",
           "coolchic_batch_backward", "coolchic_batch_destroy", "coolchic_warm_param_count",
           "coolchic_warm_workspace_bytes", "coolchic_warm_forward", "coolchic_warm_backward",
           "coolchic_uniform_noise", "coolchic_warm_backward_grad", "coolchic_timing_event_create",
           "coolchic_timing_event_elapsed", "coolchic_timing_event_destroy", "coolchic_train_step",
           "coolchic_train_step_noalloc", "coolchic_entropy_workspace_bytes", "coolchic_entropy_bound",
           "coolchic_entropy_tables", "coolchic_entropy_encode", "coolchic_entropy_decode",
           "coolchic_param_quantize", "coolchic_analysis_param_count", "coolchic_analysis_workspace_bytes",
           "coolchic_analysis_forward", "coolchic_stream_prepare")
CC_STAGE_NONE, CC_STAGE_ARM, CC_STAGE_SYNTHESIS = 0, 1, 2


class CCArch(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("arm_ctx", ctypes.c_int32), ("arm_layers", ctypes.c_int32),
                ("ups_taps", ctypes.c_int32), ("syn_hidden", ctypes.c_int32), ("syn_res", ctypes.c_int32),
                ("ups_shared", ctypes.c_int32)]


class CCProblem(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("arch", CCArch), ("quant", ctypes.c_int32),
                ("lam", ctypes.c_float)]


class CCWarmProblem(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("batch", ctypes.c_int32), ("arch", CCArch)]


class CCImageIO(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("img", "y", "u", "arm_w", "ups_w", "syn_w", "loss4", "g_y", "g_arm", "g_ups", "g_syn")]


class CCBatchTuning(ctypes.Structure):
    _fields_ = [("arm_blocks", ctypes.c_int32), ("syn_blocks", ctypes.c_int32), ("arm_first", ctypes.c_int32),
                ("ups_tile", ctypes.c_int32)]


class CoolChicError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {strerror(code)} (code {code})")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2403_11651_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, SZ, F, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float, ctypes.c_int
    pa, pp = ctypes.POINTER(CCArch), ctypes.POINTER(CCProblem)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "coolchic_param_count": (I64, [pa, pi64, pi64, pi64]),
        "coolchic_latent_count": (I64, [pp]),
        "coolchic_workspace_bytes": (SZ, [pp, I]),
        "coolchic_forward": (I, [pp, P, P, P, P, P, P, P, P, P, P, P, SZ, P]),
        "coolchic_backward": (I, [pp, P, P, P, P, P, P, F, P, P, P, P, P, P, SZ, P]),
        "coolchic_decode_synth": (I, [pp, P, P, P, P, P, SZ, P]),
        "coolchic_adam_step": (I, [P, P, P, P, I64, P, F, F, F, F, P]),
        "coolchic_train_step": (I, [pp, P, P, F, P, P, P, P, P, P, F, F, F, F, P, SZ, P]),
        "coolchic_train_step_noalloc": (I, [pp, P, P, F, P, P, P, P, P, P, F, F, F, F, P]),
        "coolchic_set_stage_events": (I, [I, P, P]),
        "coolchic_stream_prepare": (I, [P]),
        "coolchic_timing_event_create": (I, [ctypes.POINTER(P)]),
        "coolchic_timing_event_elapsed": (I, [P, P, ctypes.POINTER(F)]),
        "coolchic_timing_event_destroy": (I, [P]),
        "coolchic_strerror": (ctypes.c_char_p, [I]),
        "coolchic_batch_workspace_bytes": (SZ, [I, pp, ctypes.POINTER(CCBatchTuning)]),
        "coolchic_batch_create": (I, [I, pp, ctypes.POINTER(CCImageIO), ctypes.POINTER(CCBatchTuning), F, P, SZ,
                                      ctypes.POINTER(P)]),
        "coolchic_batch_backward": (I, [P, P]),
        "coolchic_batch_destroy": (None, [P]),
        "coolchic_uniform_noise": (I, [P, I64, ctypes.c_uint64, P, ctypes.c_uint32, P]),
        "coolchic_param_quantize": (I, [pa, P, P, P, ctypes.POINTER(ctypes.c_int32), P, P, P, P, P]),
        "coolchic_entropy_workspace_bytes": (SZ, [pp]),
        "coolchic_entropy_bound": (I64, [pp]),
        "coolchic_entropy_tables": (I, [P, P]),
        "coolchic_entropy_encode": (I, [pp, P, P, P, SZ, P, P, SZ, P]),
        "coolchic_entropy_decode": (I, [pp, P, SZ, P, P, P, P, SZ, P]),
        "coolchic_warm_param_count": (I64, [pa]),
        "coolchic_analysis_param_count": (I64, []),
        "coolchic_analysis_workspace_bytes": (SZ, [I, I, I]),
        "coolchic_analysis_forward": (I, [I, I, I, P, P, P, P, SZ, P]),
        "coolchic_warm_workspace_bytes": (SZ, [ctypes.POINTER(CCWarmProblem), I]),
        "coolchic_warm_forward": (I, [ctypes.POINTER(CCWarmProblem), P, P, P, P, P, SZ, P]),
        "coolchic_warm_backward": (I, [ctypes.POINTER(CCWarmProblem), P, P, P, P, P, P, P, SZ, P]),
        "coolchic_warm_backward_grad": (I, [ctypes.POINTER(CCWarmProblem), P, P, P, P, P, P, P, SZ, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype, fn.argtypes = res, args
    return lib


_lib = _load()


def strerror(code: int) -> str:
    return _lib.coolchic_strerror(int(code)).decode()


@dataclass(frozen=True)
class Arch:
    """Table I style architecture (see include/coolchic.h, cc_arch)."""
    n_levels: int = 7
    arm_ctx: int = 24
    arm_layers: int = 2
    ups_taps: int = 8
    syn_hidden: int = 40
    syn_res: int = 2
    ups_shared: int = 0

    def c(self) -> CCArch:
        return CCArch(self.n_levels, self.arm_ctx, self.arm_layers, self.ups_taps, self.syn_hidden, self.syn_res,
                      int(self.ups_shared))


FULL = Arch(7, 24, 2, 8, 40, 2)
LOW = Arch(7, 8, 2, 8, 16, 1)


@dataclass(frozen=True)
class Problem:
    H: int
    W: int
    arch: Arch = FULL
    quant: int = CC_QUANT_ROUND
    lam: float = 1e-3

    def c(self) -> CCProblem:
        return CCProblem(self.H, self.W, self.arch.c(), self.quant, self.lam)


def param_count(arch: Arch):
    a, u, s = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    tot = _lib.coolchic_param_count(ctypes.byref(arch.c()), ctypes.byref(a), ctypes.byref(u), ctypes.byref(s))
    if tot < 0:
        raise CoolChicError(CC_EUNSUPPORTED, "coolchic_param_count")
    return a.value, u.value, s.value


def latent_count(p: Problem) -> int:
    n = _lib.coolchic_latent_count(ctypes.byref(p.c()))
    if n < 0:
        raise CoolChicError(CC_EINVAL, "coolchic_latent_count")
    return n


def workspace_bytes(p: Problem, which: int) -> int:
    return int(_lib.coolchic_workspace_bytes(ctypes.byref(p.c()), int(which)))


def workspace(p: Problem, which: int, device="cuda") -> torch.Tensor:
    n = workspace_bytes(p, which)
    if n == 0:
        raise CoolChicError(CC_EINVAL, "coolchic_workspace_bytes")
    return torch.empty(n, dtype=torch.uint8, device=device)


def _ptr(t, n=None, name="tensor"):
    """Device pointer of a contiguous float32 GPU tensor (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype not in (torch.float32, torch.int32, torch.int64, torch.uint8) or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _on(stream):
    """Context in which a temporary workspace is allocated for a call on
    `stream`: torch's caching allocator ties a block to the stream that was
    current when it was allocated, and may hand it out again on that stream
    as soon as it is freed; allocating it on the call's own stream keeps a
    later allocation from overwriting it while the call's kernels run."""
    if stream is None:
        return contextlib.nullcontext()
    if not isinstance(stream, torch.cuda.Stream):
        stream = torch.cuda.ExternalStream(_stream(stream))
    return torch.cuda.stream(stream)


def _check(rc, where):
    if rc != CC_OK:
        raise CoolChicError(rc, where)


def _n_noise(p: Problem, n_lat: int) -> int:
    """Floats of the noise buffer: the soft proxy stores its sharpness after
    the noise."""
    return n_lat + 1 if p.quant == CC_QUANT_SOFT else n_lat


def coolchic_forward(p: Problem, img, y, u, arm_w, ups_w, syn_w, loss4, rate_map=None, yq_out=None, xhat_out=None,
                     ws=None, stream=None):
    n_lat = latent_count(p)
    na, nu, ns = param_count(p.arch)
    hw3 = 3 * p.H * p.W
    if ws is None:
        with _on(stream):
            ws = workspace(p, CC_WS_FORWARD, device=y.device)
    rc = _lib.coolchic_forward(ctypes.byref(p.c()), _ptr(img, hw3, "img"), _ptr(y, n_lat, "y"),
                               _ptr(u, _n_noise(p, n_lat), "u"),
                               _ptr(arm_w, na, "arm_w"), _ptr(ups_w, nu, "ups_w"), _ptr(syn_w, ns, "syn_w"),
                               _ptr(loss4, 4, "loss4"), _ptr(rate_map, n_lat, "rate_map"),
                               _ptr(yq_out, n_lat, "yq_out"), _ptr(xhat_out, hw3, "xhat_out"),
                               _ptr(ws, None, "ws"), ws.numel(), _stream(stream))
    _check(rc, "coolchic_forward")


def coolchic_backward(p: Problem, img, y, u, arm_w, ups_w, syn_w, dloss, loss4, g_y, g_arm, g_ups, g_syn, ws=None,
                      stream=None):
    n_lat = latent_count(p)
    na, nu, ns = param_count(p.arch)
    hw3 = 3 * p.H * p.W
    if ws is None:
        with _on(stream):
            ws = workspace(p, CC_WS_BACKWARD, device=y.device)
    rc = _lib.coolchic_backward(ctypes.byref(p.c()), _ptr(img, hw3, "img"), _ptr(y, n_lat, "y"),
                                _ptr(u, _n_noise(p, n_lat), "u"),
                                _ptr(arm_w, na, "arm_w"), _ptr(ups_w, nu, "ups_w"), _ptr(syn_w, ns, "syn_w"),
                                float(dloss), _ptr(loss4, 4, "loss4"), _ptr(g_y, n_lat, "g_y"),
                                _ptr(g_arm, na, "g_arm"), _ptr(g_ups, nu, "g_ups"), _ptr(g_syn, ns, "g_syn"),
                                _ptr(ws, None, "ws"), ws.numel(), _stream(stream))
    _check(rc, "coolchic_backward")


def coolchic_decode_synth(p: Problem, yq, ups_w, syn_w, xhat, ws=None, stream=None):
    n_lat = latent_count(p)
    _, nu, ns = param_count(p.arch)
    if ws is None:
        with _on(stream):
            ws = workspace(p, CC_WS_DECODE, device=yq.device)
    rc = _lib.coolchic_decode_synth(ctypes.byref(p.c()), _ptr(yq, n_lat, "yq"), _ptr(ups_w, nu, "ups_w"),
                                    _ptr(syn_w, ns, "syn_w"), _ptr(xhat, 3 * p.H * p.W, "xhat"),
                                    _ptr(ws, None, "ws"), ws.numel(), _stream(stream))
    _check(rc, "coolchic_decode_synth")


def coolchic_adam_step(theta, grad, m, v, step, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    n = theta.numel()
    if step.dtype != torch.int32 or step.numel() != 2:
        raise TypeError("step must be a device int32 tensor of 2 elements: steps taken, completion counter (0)")
    rc = _lib.coolchic_adam_step(_ptr(theta, n, "theta"), _ptr(grad, n, "grad"), _ptr(m, n, "m"), _ptr(v, n, "v"),
                                 n, _ptr(step, 2, "step"), lr, beta1, beta2, eps, _stream(stream))
    _check(rc, "coolchic_adam_step")


def coolchic_train_step(p: Problem, img, u, dloss, loss4, theta, grad, m, v, step, lr=1e-2, beta1=0.9, beta2=0.999,
                        eps=1e-8, ws=None, stream=None):
    """coolchic_backward then coolchic_adam_step on the packed vectors
    theta = [y | arm_w | ups_w | syn_w] (grad, m, v alike), in one pass."""
    n_lat = latent_count(p)
    na, nu, ns = param_count(p.arch)
    n = n_lat + na + nu + ns
    if step.dtype != torch.int32 or step.numel() != 2:
        raise TypeError("step must be a device int32 tensor of 2 elements: steps taken, completion counter (0)")
    if ws is None:
        with _on(stream):
            ws = workspace(p, CC_WS_BACKWARD, device=theta.device)
    rc = _lib.coolchic_train_step(ctypes.byref(p.c()), _ptr(img, 3 * p.H * p.W, "img"), _ptr(u, _n_noise(p, n_lat), "u"),
                                  float(dloss), _ptr(loss4, 4, "loss4"), _ptr(theta, n, "theta"),
                                  _ptr(grad, n, "grad"), _ptr(m, n, "m"), _ptr(v, n, "v"), _ptr(step, 2, "step"),
                                  lr, beta1, beta2, eps, _ptr(ws, None, "ws"), ws.numel(), _stream(stream))
    _check(rc, "coolchic_train_step")


def coolchic_train_step_noalloc(p: Problem, img, u, dloss, loss4, theta, grad, m, v, step, lr=1e-2, beta1=0.9,
                                beta2=0.999, eps=1e-8, stream=None):
    """coolchic_train_step with the library's static device scratch as its
    workspace (no allocation by the library or here)."""
    n_lat = latent_count(p)
    na, nu, ns = param_count(p.arch)
    n = n_lat + na + nu + ns
    if step.dtype != torch.int32 or step.numel() != 2:
        raise TypeError("step must be a device int32 tensor of 2 elements: steps taken, completion counter (0)")
    rc = _lib.coolchic_train_step_noalloc(ctypes.byref(p.c()), _ptr(img, 3 * p.H * p.W, "img"),
                                          _ptr(u, _n_noise(p, n_lat), "u"),
                                          float(dloss), _ptr(loss4, 4, "loss4"), _ptr(theta, n, "theta"),
                                          _ptr(grad, n, "grad"), _ptr(m, n, "m"), _ptr(v, n, "v"),
                                          _ptr(step, 2, "step"), lr, beta1, beta2, eps, _stream(stream))
    _check(rc, "coolchic_train_step_noalloc")


def coolchic_param_quantize(arch: Arch, arm_w, ups_w, syn_w, step_log2, arm_q, ups_q, syn_q, bits, stream=None):
    """Each module on a grid of step 2^-k (k from step_log2, three ints);
    quantised values into *_q, the modules' rates (bits) into the device
    float tensor bits [3]."""
    na, nu, ns = param_count(arch)
    ks = (ctypes.c_int32 * 3)(*[int(k) for k in step_log2])
    rc = _lib.coolchic_param_quantize(ctypes.byref(arch.c()), _ptr(arm_w, na, "arm_w"), _ptr(ups_w, nu, "ups_w"),
                                      _ptr(syn_w, ns, "syn_w"), ks, _ptr(arm_q, na, "arm_q"),
                                      _ptr(ups_q, nu, "ups_q"), _ptr(syn_q, ns, "syn_q"), _ptr(bits, 3, "bits"),
                                      _stream(stream))
    _check(rc, "coolchic_param_quantize")


def entropy_workspace(p: Problem, device="cuda") -> torch.Tensor:
    n = int(_lib.coolchic_entropy_workspace_bytes(ctypes.byref(p.c())))
    if n == 0:
        raise CoolChicError(CC_EUNSUPPORTED, "coolchic_entropy_workspace_bytes")
    return torch.empty(n, dtype=torch.uint8, device=device)


def entropy_bound(p: Problem) -> int:
    n = int(_lib.coolchic_entropy_bound(ctypes.byref(p.c())))
    if n < 0:
        raise CoolChicError(CC_EINVAL, "coolchic_entropy_bound")
    return n


def coolchic_entropy_tables(cum, stream=None):
    """cum: device int32 tensor of 75 * 16 * 99 elements (read as uint32)."""
    _check(_lib.coolchic_entropy_tables(_ptr(cum, 75 * 16 * 99, "cum"), _stream(stream)), "coolchic_entropy_tables")


def coolchic_entropy_encode(p: Problem, yq, arm_w, out, out_nbytes, ws=None, stream=None):
    """Bitstream of the integer latents yq into the device uint8 tensor out;
    out_nbytes: device int64 tensor of one element (size, 0, or -size)."""
    n_lat = latent_count(p)
    na, _, _ = param_count(p.arch)
    if ws is None:
        with _on(stream):
            ws = entropy_workspace(p, device=yq.device)
    rc = _lib.coolchic_entropy_encode(ctypes.byref(p.c()), _ptr(yq, n_lat, "yq"), _ptr(arm_w, na, "arm_w"),
                                      _ptr(out, None, "out"), out.numel(), _ptr(out_nbytes, 1, "out_nbytes"),
                                      _ptr(ws, None, "ws"), ws.numel(), _stream(stream))
    _check(rc, "coolchic_entropy_encode")


def coolchic_entropy_decode(p: Problem, data, nbytes: int, arm_w, yq_out, status, ws=None, stream=None):
    """Latents from the first nbytes bytes of the device uint8 tensor data;
    status: device int32 tensor of two elements (one per set of grids)."""
    n_lat = latent_count(p)
    na, _, _ = param_count(p.arch)
    if ws is None:
        with _on(stream):
            ws = entropy_workspace(p, device=yq_out.device)
    if nbytes > data.numel():
        raise ValueError("nbytes exceeds the data tensor")
    rc = _lib.coolchic_entropy_decode(ctypes.byref(p.c()), _ptr(data, None, "data"), int(nbytes),
                                      _ptr(arm_w, na, "arm_w"), _ptr(yq_out, n_lat, "yq_out"),
                                      _ptr(status, 2, "status"), _ptr(ws, None, "ws"), ws.numel(), _stream(stream))
    _check(rc, "coolchic_entropy_decode")


def coolchic_uniform_noise(u, seed: int, step=None, stream_id: int = 0, stream=None):
    """Fill u (device float32) with Philox uniform noise in [-1/2, 1/2);
    step: device int32 tensor whose first element is the iteration, or None."""
    if step is not None and (step.dtype != torch.int32 or not step.is_cuda):
        raise TypeError("step must be a device int32 tensor")
    rc = _lib.coolchic_uniform_noise(_ptr(u, None, "u"), u.numel(), int(seed) & ((1 << 64) - 1),
                                     None if step is None else step.data_ptr(), int(stream_id) & 0xffffffff,
                                     _stream(stream))
    _check(rc, "coolchic_uniform_noise")


def coolchic_stream_prepare(stream=None):
    """Creates the library's side stream and events for `stream` (default:
    the current torch stream) on the current device ahead of time."""
    _check(_lib.coolchic_stream_prepare(_stream(stream)), "coolchic_stream_prepare")


def coolchic_set_stage_events(stage: int, ev_begin=None, ev_end=None):
    """ev_begin / ev_end: raw hipEvent_t handles (ints) or None."""
    _check(_lib.coolchic_set_stage_events(int(stage), ev_begin, ev_end), "coolchic_set_stage_events")


class TimingEvent:
    """A fence-free timing event of the library (coolchic_timing_event_*);
    .handle is the raw hipEvent_t for coolchic_set_stage_events."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(_lib.coolchic_timing_event_create(ctypes.byref(h)), "coolchic_timing_event_create")
        self.handle = h.value

    def elapsed_ms(self, end: "TimingEvent") -> float:
        ms = ctypes.c_float()
        _check(_lib.coolchic_timing_event_elapsed(self.handle, end.handle, ctypes.byref(ms)),
               "coolchic_timing_event_elapsed")
        return ms.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.coolchic_timing_event_destroy(self.handle)
            self.handle = None


def _tuning(tune):
    """cc_batch_tuning from a tuple (arm_blocks, syn_blocks, arm_first,
    ups_tile); missing trailing entries are 0 (the defaults)."""
    tune = tuple(int(t) for t in tune)
    if len(tune) > 4:
        raise ValueError("tune has at most 4 entries")
    return CCBatchTuning(*(tune + (0,) * (4 - len(tune))))


def batch_workspace_bytes(probs, tune=(0, 0, 0, 0)) -> int:
    arr = (CCProblem * len(probs))(*[p.c() for p in probs])
    t = _tuning(tune)
    return int(_lib.coolchic_batch_workspace_bytes(len(probs), arr, ctypes.byref(t)))


class BatchPlan:
    """Owner of a coolchic_batch_create plan.  `io` is a list of dicts with the
    device tensors of each image (keys of CCImageIO; "u" may be None); the plan
    keeps references to them and to its workspace so the pointers it holds stay
    valid."""

    def __init__(self, probs, io, tune=(0, 0, 0, 0), dloss=1.0, device="cuda"):
        n = len(probs)
        if n == 0 or len(io) != n:
            raise ValueError("probs and io must be non-empty lists of equal length")
        self.probs, self.io, self.tune = list(probs), list(io), tuple(int(t) for t in tune)
        arr = (CCProblem * n)(*[p.c() for p in probs])
        ios = (CCImageIO * n)()
        for k, (p, d) in enumerate(zip(probs, io)):
            n_lat = latent_count(p)
            na, nu, ns = param_count(p.arch)
            sizes = {"img": 3 * p.H * p.W, "y": n_lat, "u": _n_noise(p, n_lat), "arm_w": na, "ups_w": nu, "syn_w": ns,
                     "loss4": 4, "g_y": n_lat, "g_arm": na, "g_ups": nu, "g_syn": ns}
            for name, size in sizes.items():
                setattr(ios[k], name, _ptr(d.get(name), size, f"io[{k}].{name}"))
        t = _tuning(self.tune)
        nbytes = int(_lib.coolchic_batch_workspace_bytes(n, arr, ctypes.byref(t)))
        if nbytes == 0:
            raise CoolChicError(CC_EINVAL, "coolchic_batch_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        rc = _lib.coolchic_batch_create(n, arr, ios, ctypes.byref(t), float(dloss), self.ws.data_ptr(), nbytes,
                                        ctypes.byref(h))
        _check(rc, "coolchic_batch_create")
        self._h = h

    def backward(self, stream=None):
        _check(_lib.coolchic_batch_backward(self._h, _stream(stream)), "coolchic_batch_backward")

    def close(self):
        # (at interpreter exit the module globals may already be gone)
        if getattr(self, "_h", None) and _lib is not None:
            _lib.coolchic_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


@dataclass(frozen=True)
class WarmProblem:
    H: int
    W: int
    batch: int
    arch: Arch = LOW

    def c(self) -> CCWarmProblem:
        return CCWarmProblem(self.H, self.W, self.batch, self.arch.c())


def warm_param_count(arch: Arch) -> int:
    n = _lib.coolchic_warm_param_count(ctypes.byref(arch.c()))
    if n < 0:
        raise CoolChicError(CC_EUNSUPPORTED, "coolchic_warm_param_count")
    return int(n)


def analysis_param_count() -> int:
    return int(_lib.coolchic_analysis_param_count())


def analysis_workspace(H: int, W: int, n: int, device="cuda") -> torch.Tensor:
    nb = int(_lib.coolchic_analysis_workspace_bytes(int(H), int(W), int(n)))
    if nb == 0:
        raise CoolChicError(CC_EINVAL, "coolchic_analysis_workspace_bytes")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def coolchic_analysis_forward(H: int, W: int, n: int, x, theta, y, ws=None, stream=None):
    """Non-overfitted analysis transform: x [n][3][H][W] -> y [n][N_lat]."""
    n_lat = sum((H >> l) * (W >> l) for l in range(7))
    if ws is None:
        with _on(stream):
            ws = analysis_workspace(H, W, n, device=x.device)
    rc = _lib.coolchic_analysis_forward(int(H), int(W), int(n), _ptr(x, n * 3 * H * W, "x"),
                                        _ptr(theta, analysis_param_count(), "theta"), _ptr(y, n * n_lat, "y"),
                                        _ptr(ws, None, "ws"), ws.numel(), _stream(stream))
    _check(rc, "coolchic_analysis_forward")


def warm_workspace(wp: WarmProblem, which: int, device="cuda") -> torch.Tensor:
    n = int(_lib.coolchic_warm_workspace_bytes(ctypes.byref(wp.c()), int(which)))
    if n == 0:
        raise CoolChicError(CC_EINVAL, "coolchic_warm_workspace_bytes")
    return torch.empty(n, dtype=torch.uint8, device=device)


def coolchic_warm_forward(wp: WarmProblem, x, net, y_out, theta_out, ws=None, stream=None):
    n_lat = latent_count(Problem(wp.H, wp.W, wp.arch))
    n_theta = sum(param_count(wp.arch))
    if ws is None:
        with _on(stream):
            ws = warm_workspace(wp, CC_WS_FORWARD, device=x.device)
    rc = _lib.coolchic_warm_forward(ctypes.byref(wp.c()), _ptr(x, wp.batch * 3 * wp.H * wp.W, "x"),
                                    _ptr(net, warm_param_count(wp.arch), "net"),
                                    _ptr(y_out, wp.batch * n_lat, "y_out"),
                                    _ptr(theta_out, wp.batch * n_theta, "theta_out"), _ptr(ws, None, "ws"),
                                    ws.numel(), _stream(stream))
    _check(rc, "coolchic_warm_forward")


def coolchic_warm_backward(wp: WarmProblem, x, net, y_target, theta_target, loss4, g_net, ws=None, stream=None):
    n_lat = latent_count(Problem(wp.H, wp.W, wp.arch))
    n_theta = sum(param_count(wp.arch))
    nn = warm_param_count(wp.arch)
    if ws is None:
        with _on(stream):
            ws = warm_workspace(wp, CC_WS_BACKWARD, device=x.device)
    rc = _lib.coolchic_warm_backward(ctypes.byref(wp.c()), _ptr(x, wp.batch * 3 * wp.H * wp.W, "x"),
                                     _ptr(net, nn, "net"), _ptr(y_target, wp.batch * n_lat, "y_target"),
                                     _ptr(theta_target, wp.batch * n_theta, "theta_target"),
                                     _ptr(loss4, 4, "loss4"), _ptr(g_net, nn, "g_net"), _ptr(ws, None, "ws"),
                                     ws.numel(), _stream(stream))
    _check(rc, "coolchic_warm_backward")


def coolchic_warm_backward_grad(wp: WarmProblem, x, net, g_y, g_theta, loss4, g_net, ws=None, stream=None):
    n_lat = latent_count(Problem(wp.H, wp.W, wp.arch))
    n_theta = sum(param_count(wp.arch))
    nn = warm_param_count(wp.arch)
    if ws is None:
        with _on(stream):
            ws = warm_workspace(wp, CC_WS_BACKWARD, device=x.device)
    rc = _lib.coolchic_warm_backward_grad(ctypes.byref(wp.c()), _ptr(x, wp.batch * 3 * wp.H * wp.W, "x"),
                                          _ptr(net, nn, "net"), _ptr(g_y, wp.batch * n_lat, "g_y"),
                                          _ptr(g_theta, wp.batch * n_theta, "g_theta"), _ptr(loss4, 4, "loss4"),
                                          _ptr(g_net, nn, "g_net"), _ptr(ws, None, "ws"), ws.numel(),
                                          _stream(stream))
    _check(rc, "coolchic_warm_backward_grad")


# raw access for tests of the C ABI itself
lib = _lib
