"""Batched overfitting: many images of uneven sizes trained together.

Every image keeps its own latent pyramid and its own ARM / upsampling /
synthesis parameters (Section III: each image gets its own overfitted
decoder); they share only the architecture.  One training iteration of the
whole batch is the batched backward pass of the HIP library (one launch per
stage for all images) plus one Adam launch over the parameters of every
image, so a block of iterations is captured once in a HIP graph and replayed.

The persistent kernels' launch shapes (work-groups of the ARM and of the
synthesis-backward launch, spread over the images in proportion to their
tiles) are picked by `autotune`, which times candidates on the device and
caches the choice per device, architecture and image-size list.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import os
import threading

import numpy as np
import torch

from . import binding as B


class BatchEncoder:
    """Overfits n images at once.  `images[k]` is planar [3][H][W] float32;
    `y0[k]` the packed initial latent pyramid; `params0[k]` the initial
    (arm, ups, syn) blocks.

    Parameters of image k live in one flat buffer, segment k = [y | arm | ups |
    syn], with matching gradient and Adam moment buffers, so a single Adam
    launch updates every image.  The quantisation proxy is a mode: rounding
    with a straight-through gradient (CC_QUANT_ROUND, the default) or additive
    uniform noise (CC_QUANT_NOISE), drawn on the device every iteration from
    the Philox generator keyed by `noise_seed` and the step counter."""

    def __init__(self, problems, images, y0, params0, lr=1e-2, tune=(0, 0), noise_seed=0, device="cuda"):
        """The noise buffer holds, per image, its latents' noise followed by one
        float: the soft proxy's sharpness (CC_QUANT_SOFT reads it there), copied
        from the device scalar self.alpha after every draw."""
        n = len(problems)
        if not (n and len(images) == n and len(y0) == n and len(params0) == n):
            raise ValueError("problems, images, y0 and params0 must be equally long and non-empty")
        arch = problems[0].arch
        for p in problems:
            if p.arch != arch:
                raise ValueError("every image must share one architecture")
        self.device = torch.device(device)
        self.problems = [dataclasses.replace(p, quant=B.CC_QUANT_ROUND) for p in problems]
        self.lr = float(lr)
        self.noise_seed = int(noise_seed)
        na, nu, ns = B.param_count(arch)
        self.seg = []  # (offset, n_lat, offset in the noise buffer) per image
        off = uoff = 0
        for p in problems:
            n_lat = B.latent_count(p)
            self.seg.append((off, n_lat, uoff))
            off += n_lat + na + nu + ns
            uoff += n_lat + 1
        self.n_params = off
        flat = np.empty(off, np.float32)
        for (o, n_lat, _), y, (a, u, s) in zip(self.seg, y0, params0):
            flat[o:o + n_lat] = y
            flat[o + n_lat:o + n_lat + na] = a
            flat[o + n_lat + na:o + n_lat + na + nu] = u
            flat[o + n_lat + na + nu:o + n_lat + na + nu + ns] = s
        dev = self.device
        self.theta = torch.from_numpy(flat).to(dev)
        self.grad = torch.zeros_like(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.u = torch.zeros(uoff, device=dev)
        self.alpha = torch.ones(1, device=dev)
        self._alpha_idx = torch.tensor([uo + n for _, n, uo in self.seg], dtype=torch.int64, device=dev)
        self.step_ctr = torch.zeros(2, dtype=torch.int32, device=dev)
        self.loss = torch.zeros(n, 4, device=dev)
        self.images = [torch.from_numpy(np.ascontiguousarray(x, np.float32).reshape(-1)).to(dev) for x in images]
        self._na, self._nu, self._ns = na, nu, ns
        self.plans = {}
        self.mode = B.CC_QUANT_ROUND
        self.tune = tuple(int(t) for t in tune) + (0,) * (4 - len(tune))
        self.plan = self._plan(self.mode)

    # -- views of image k's parameters and gradients
    def _views(self, buf, k):
        o, n_lat, _ = self.seg[k]
        na, nu, ns = self._na, self._nu, self._ns
        return (buf[o:o + n_lat], buf[o + n_lat:o + n_lat + na], buf[o + n_lat + na:o + n_lat + na + nu],
                buf[o + n_lat + na + nu:o + n_lat + na + nu + ns])

    def params(self, k):
        return tuple(t.detach().cpu().numpy() for t in self._views(self.theta, k))

    def grads(self, k):
        return tuple(t.detach().cpu().numpy() for t in self._views(self.grad, k))

    def _plan(self, mode):
        if mode not in self.plans:
            io = []
            for k in range(len(self.problems)):
                y, a, u, s = self._views(self.theta, k)
                gy, ga, gu, gs = self._views(self.grad, k)
                _, n_lat, uo = self.seg[k]
                noise = {B.CC_QUANT_NOISE: n_lat, B.CC_QUANT_SOFT: n_lat + 1}.get(mode)
                io.append(dict(img=self.images[k], y=y, u=self.u[uo:uo + noise] if noise else None,
                               arm_w=a, ups_w=u, syn_w=s, loss4=self.loss[k], g_y=gy, g_arm=ga, g_ups=gu, g_syn=gs))
            probs = [dataclasses.replace(p, quant=mode) for p in self.problems]
            self.plans[mode] = B.BatchPlan(probs, io, tune=self.tune, device=self.device)
        return self.plans[mode]

    def set_tuning(self, tune):
        tune = tuple(int(t) for t in tune) + (0,) * (4 - len(tune))
        if tune != self.tune:
            for p in self.plans.values():
                p.close()
            self.plans = {}
            self.tune = tune
        self.plan = self._plan(self.mode)

    def set_mode(self, mode):
        """CC_QUANT_ROUND, CC_QUANT_NOISE or CC_QUANT_SOFT for the following
        iterations."""
        if mode not in (B.CC_QUANT_ROUND, B.CC_QUANT_NOISE, B.CC_QUANT_SOFT):
            raise ValueError("unknown quantisation mode")
        self.mode = mode
        self.plan = self._plan(mode)

    def _draw(self, stream=None):
        B.coolchic_uniform_noise(self.u, self.noise_seed, step=self.step_ctr, stream=stream)
        if self.mode == B.CC_QUANT_SOFT:
            # the sharpness after each image's noise (a device copy: a graph
            # replay reads the current self.alpha)
            self.u.index_copy_(0, self._alpha_idx, self.alpha.expand(len(self.seg)))

    def backward(self, stream=None):
        """Loss and gradients of every image (written to self.loss, self.grad)
        at the current parameters, in the current mode."""
        if self.mode in (B.CC_QUANT_NOISE, B.CC_QUANT_SOFT):
            self._draw(stream)
        self.plan.backward(stream)

    def step(self, stream=None):
        """One training iteration of every image."""
        self.backward(stream)
        B.coolchic_adam_step(self.theta, self.grad, self.m, self.v, self.step_ctr, lr=self.lr, stream=stream)

    def probe(self, stream=None):
        """Loss (and gradients) of the current parameters with the rounding
        quantiser, whatever the training mode: the rate-distortion cost the
        decoder will actually see."""
        self._plan(B.CC_QUANT_ROUND).backward(stream)

    def capture(self, k, probe=False):
        """A HIP graph of k training iterations in the current mode (then, with
        probe, the rounding-mode loss of the result).  Runs one backward pass
        first (outside the graph; it leaves the parameters unchanged) so that
        every stream and event the library uses exists before capture."""
        self.backward()
        torch.cuda.synchronize(self.device)
        g = torch.cuda.CUDAGraph()
        if probe:
            self.probe()
        torch.cuda.synchronize(self.device)
        with torch.cuda.graph(g):
            for _ in range(k):
                self.step()
            if probe:
                self.probe()
        return g

    def run(self, iters, graph_steps=50):
        """iters training iterations in the current mode, replaying a captured
        graph of graph_steps iterations (the remainder eagerly)."""
        if iters >= graph_steps > 0:
            g = self.capture(graph_steps)
            for _ in range(iters // graph_steps):
                g.replay()
            rem = iters % graph_steps
        else:
            rem = iters
        for _ in range(rem):
            self.step()

    def fit(self, iters, noise_frac=0.8, graph_steps=50, proxy="noise", t_start=1.0, t_end=0.1):
        """The two-phase schedule: a differentiable proxy for the first
        noise_frac of the iterations, then rounding with the straight-through
        gradient.  proxy "noise": y + u; "soft": C3's soft rounding s(s(y) +
        u) with the temperature 1 / alpha annealed linearly from t_start to
        t_end over the first phase (stepped once per graph of graph_steps
        iterations)."""
        n_noise = int(round(iters * noise_frac))
        if proxy == "soft":
            self.set_mode(B.CC_QUANT_SOFT)
            g = self.capture(graph_steps) if n_noise >= graph_steps > 0 else None
            done = 0
            while done < n_noise:
                k = graph_steps if g is not None and n_noise - done >= graph_steps else 1
                frac = (done + 0.5 * k) / max(n_noise, 1)
                self.alpha.fill_(1.0 / (t_start + (t_end - t_start) * frac))
                if k == graph_steps and g is not None:
                    g.replay()
                else:
                    self.step()
                done += k
        elif proxy == "noise":
            self.set_mode(B.CC_QUANT_NOISE)
            self.run(n_noise, graph_steps)
        else:
            raise ValueError("proxy is 'noise' or 'soft'")
        self.set_mode(B.CC_QUANT_ROUND)
        self.run(iters - n_noise, graph_steps)

    def save(self):
        return [t.clone() for t in (self.theta, self.m, self.v, self.step_ctr, self.loss)]

    def load(self, state):
        for dst, src in zip((self.theta, self.m, self.v, self.step_ctr, self.loss), state):
            dst.copy_(src)


# ---- autotuner -----------------------------------------------------------

ARM_CANDIDATES = (0, 512, 1024, 2048, 4096)
ARM_FIRST_CANDIDATES = (0, 1, 2)
SYN_CANDIDATES = (0, 512, 1024, 2048, 4096)
UPS_TILE_CANDIDATES = (32, 16)  # level-1 tile side of the upsampling forward
_cache_lock = threading.Lock()


def cache_path():
    return os.environ.get("COOLCHIC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "coolchic", "autotune.json"))


_LIB_DIGEST = None


def _library_digest():
    """Hash of the built library: a tuned choice is only reused with the
    kernels it was timed on."""
    global _LIB_DIGEST
    if _LIB_DIGEST is None:
        with open(B.LIB_PATH, "rb") as f:
            _LIB_DIGEST = hashlib.sha256(f.read()).hexdigest()[:16]
    return _LIB_DIGEST


def tuning_key(enc: BatchEncoder):
    a = enc.problems[0].arch
    sizes = ",".join(f"{p.H}x{p.W}" for p in enc.problems)
    dev = torch.cuda.get_device_name(enc.device)
    return f"{dev}|{_library_digest()}|{a.n_levels},{a.arm_ctx},{a.arm_layers},{a.ups_taps},{a.syn_hidden}," \
           f"{a.syn_res}|{hashlib.sha256(sizes.encode()).hexdigest()[:16]}"


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path, key, value):
    with _cache_lock:
        data = _load_cache(path)
        data[key] = value
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = f"{path}.{os.getpid()}.tmp"
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass  # a read-only home: the choice is simply not remembered


def time_iteration(enc: BatchEncoder, iters=10, reps=3):
    """Median device time (ms) of one training iteration, from HIP events
    around `iters` eager iterations, over `reps` repetitions."""
    stream = torch.cuda.current_stream(enc.device)
    enc.step()
    enc.step()
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(iters):
            enc.step()
        e1.record(stream)
        e1.synchronize()
        out.append(e0.elapsed_time(e1) / iters)
    return float(np.median(out))


def autotune(enc: BatchEncoder, use_cache=True, iters=10, reps=3, log=None):
    """Chooses (arm_blocks, syn_blocks, arm_first, ups_tile) for enc by
    coordinate search over the candidate lists (the ARM's launch position,
    then its grid with the default synthesis shape, then the synthesis
    shape, then the upsampling forward's tile side), timing whole training
    iterations.  The encoder's state is restored afterwards;
    the choice is applied and returned, with the timings, and cached."""
    path = cache_path()
    key = tuning_key(enc)
    if use_cache:
        hit = _load_cache(path).get(key)
        if hit:
            enc.set_tuning(tuple(hit["tune"]))
            return dict(hit, cached=True)
    state = enc.save()
    timings = {}

    def measure(t):
        if t not in timings:
            enc.set_tuning(t)
            timings[t] = time_iteration(enc, iters, reps)
            if log:
                log(f"autotune {t}: {timings[t]:.4f} ms/iter")
        return timings[t]

    t0 = UPS_TILE_CANDIDATES[0]
    best_f = min(ARM_FIRST_CANDIDATES, key=lambda f: measure((0, 0, f, t0)))
    best_a = min(ARM_CANDIDATES, key=lambda a: measure((a, 0, best_f, t0)))
    best_s = min(SYN_CANDIDATES, key=lambda s: measure((best_a, s, best_f, t0)))
    best = min(((best_a, best_s, best_f, t) for t in UPS_TILE_CANDIDATES), key=measure)
    enc.load(state)
    enc.set_tuning(best)
    result = dict(tune=list(best), ms_per_iter=timings[best],
                  timings={",".join(str(x) for x in t): v for t, v in timings.items()})
    _store_cache(path, key, result)
    return dict(result, cached=False)
