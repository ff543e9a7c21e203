"""Learned initial guess: the network's parameters, its training on solves of
the method itself, and weight files.

Every forward/backward/optimizer step runs in the HIP kernels of the C ABI
(np_net_*); torch only allocates device memory and provides the stream.

Network (see include/nested_poisson.h): conv3x3x3(2->16) -> ReLU ->
conv3x3x3(16->16) -> ReLU -> conv3x3x3(16->1).  Input: f/||f|| and the
residual of the interpolated guess / ||f|| on Gamma^l; target: the error of the
interpolated guess, (Phi_converged - Phi_interp) / (||f|| dx^2).
"""
import ctypes
import math
import os

import numpy as np
import torch

from . import _lib
from . import workloads as W

LAYERS = [(2, 16), (16, 16), (16, 1)]
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "guess_net_multi_plummer_3lev_128.npy")


def n_params():
    return sum(27 * ci * co + co for ci, co in LAYERS)


def init_params(seed=0):
    """He-style initialisation (weights ~ N(0, 2/fan_in)), zero biases; the last
    layer starts small so the untrained network's guess is near the interpolant."""
    rng = np.random.default_rng(seed)
    out = []
    for k, (ci, co) in enumerate(LAYERS):
        std = math.sqrt(2.0 / (27 * ci)) * (0.1 if k == len(LAYERS) - 1 else 1.0)
        out.append(rng.standard_normal(27 * co * ci).astype(np.float32) * std)
        out.append(np.zeros(co, dtype=np.float32))
    return np.concatenate(out)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _chk(rc, what):
    if rc:
        raise _lib.NestedPoissonError(rc, what)


class GuessNet:
    """Parameters on the device (FP32 master + bfloat16 copies) with training state."""

    def __init__(self, theta=None, device="cuda"):
        self.dev = torch.device(device)
        theta = init_params() if theta is None else np.asarray(theta, dtype=np.float32)
        assert theta.size == n_params()
        self.theta = torch.tensor(theta, device=self.dev)
        self.grad = torch.zeros_like(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.wbf = torch.zeros(self.theta.numel(), dtype=torch.int16, device=self.dev)
        self.step = 0
        self.st = torch.cuda.current_stream(self.dev).cuda_stream
        self._sync_bf16()
        # views per layer: (w, b, w_bf16, gw, gb)
        self.views = []
        k = 0
        for ci, co in LAYERS:
            nw = 27 * ci * co
            self.views.append((slice(k, k + nw), slice(k + nw, k + nw + co)))
            k += nw + co

    def _sync_bf16(self):
        _chk(_lib.lib().np_net_to_bf16(_p(self.theta), _p(self.wbf), self.theta.numel(), ctypes.c_void_p(self.st)),
             "to_bf16")

    def params(self):
        return self.theta.detach().cpu().numpy().copy()

    def _w(self, k):
        sw, sb = self.views[k]
        return self.wbf[sw], self.theta[sb]

    # -------------------------------------------------------------- forward / backward (FP32 activations)
    def _round_bf16(self, t):
        _chk(_lib.lib().np_net_round_bf16(_p(t), t.numel(), ctypes.c_void_p(self.st)), "round bf16")

    def forward(self, x, bf16_acts=True):
        """x: [B, Z, Y, X, 2] FP32.  Returns the list of activations (input first).
        With bf16_acts the input and the hidden activations are rounded to
        bfloat16 (in place for the input), as the solver's inference path
        stores them; the output stays FP32 there too."""
        B, Z, Y, X, _ = x.shape
        if bf16_acts:
            self._round_bf16(x)
        acts = [x]
        h = x
        for k, (ci, co) in enumerate(LAYERS):
            w, b = self._w(k)
            out = torch.empty((B, Z, Y, X, co), dtype=torch.float32, device=self.dev)
            _chk(_lib.lib().np_net_conv3d_fwd(_p(h), ci, _p(w), _p(b), co, int(k < len(LAYERS) - 1), B, Z, Y, X,
                                              _p(out), ctypes.c_void_p(self.st)), "conv fwd")
            if bf16_acts and k < len(LAYERS) - 1:
                self._round_bf16(out)
            acts.append(out)
            h = out
        return acts

    def backward(self, acts, gy):
        """Accumulates parameter gradients into self.grad (overwrites); returns d loss / d input."""
        B, Z, Y, X, _ = acts[0].shape
        g = gy
        for k in range(len(LAYERS) - 1, -1, -1):
            ci, co = LAYERS[k]
            sw, sb = self.views[k]
            ws = _lib.lib().np_net_workspace_bytes(ci, co, 0)
            work = torch.empty(ws // 4 + 1, dtype=torch.float32, device=self.dev)
            gw = self.grad[sw]
            gb = self.grad[sb]
            _chk(_lib.lib().np_net_conv3d_bwd_weight(_p(acts[k]), ci, _p(g), co, B, Z, Y, X, _p(gw), _p(gb), _p(work),
                                                     ws, ctypes.c_void_p(self.st)), "conv bwd weight")
            gin = torch.empty((B, Z, Y, X, ci), dtype=torch.float32, device=self.dev)
            w, _ = self._w(k)
            _chk(_lib.lib().np_net_conv3d_bwd_data(_p(g), co, _p(w), ci, B, Z, Y, X, _p(gin), ctypes.c_void_p(self.st)),
                 "conv bwd data")
            if k > 0:
                _chk(_lib.lib().np_net_relu_bwd(_p(acts[k]), _p(gin), gin.numel(), ctypes.c_void_p(self.st)),
                     "relu bwd")
            g = gin
        return g

    def loss_grad(self, pred, target, mask=None):
        n = pred.numel()
        count = float(mask.sum().item()) if mask is not None else float(n)
        ws = _lib.lib().np_net_workspace_bytes(1, 1, n)
        work = torch.empty(ws // 4 + 1, dtype=torch.float32, device=self.dev)
        grad = torch.empty_like(pred)
        loss = torch.empty(1, dtype=torch.float32, device=self.dev)
        _chk(_lib.lib().np_net_mse(_p(pred), _p(target), _p(mask), n, count, _p(grad), _p(loss), _p(work), ws,
                                   ctypes.c_void_p(self.st)), "mse")
        return loss, grad

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        _chk(_lib.lib().np_net_adam(_p(self.theta), _p(self.grad), _p(self.m), _p(self.v), self.theta.numel(), lr, b1,
                                    b2, eps, self.step, _p(self.wbf), ctypes.c_void_p(self.st)), "adam")

    def train_step(self, x, target, mask=None, lr=1e-3):
        """Error objective: mean (y - target)^2."""
        acts = self.forward(x)
        loss, gy = self.loss_grad(acts[-1], target, mask)
        self.backward(acts, gy)
        self.adam_step(lr)
        return loss

    def _lap7(self, a, out):
        B, Z, Y, X, _ = a.shape
        _chk(_lib.lib().np_net_lap7(_p(a), B, Z, Y, X, _p(out), ctypes.c_void_p(self.st)), "lap7")

    def train_step_residual(self, x, lr=1e-3):
        """Residual objective: mean (r0/||f|| - L y)^2, the max-norm-relevant
        residual left by the corrected guess (L = the library's 7-point stencil
        without 1/dx^2, zero outside Gamma; the input's second channel is r0/||f||)."""
        acts = self.forward(x)
        ly = torch.empty_like(acts[-1])
        self._lap7(acts[-1], ly)
        r = x[..., 1:2].contiguous()
        loss, gl = self.loss_grad(ly, r)
        gy = torch.empty_like(gl)
        self._lap7(gl, gy)  # the stencil is its own adjoint
        self.backward(acts, gy)
        self.adam_step(lr)
        return loss


# ------------------------------------------------------------------ data and training
def level_samples(solver, nlevels):
    """(x, target) of every level >= 1 of the last solve, as [1, Z, Y, X, C] tensors."""
    out = []
    for l in range(1, nlevels):
        x, t = solver.guess_features(l)
        out.append((x.unsqueeze(0), t.unsqueeze(0).unsqueeze(-1)))
    return out


def train(seeds, N=128, nlevels=3, epochs=1, lr=2e-3, lr_final=2e-4, log=None, net=None, objective="error"):
    """Train on FP64 solves of the seeded multi-Plummer workload (one solve per
    seed, every refined level a sample).  Returns (net, loss history)."""
    from .solver import NestedPoissonSolver
    dev = torch.device("cuda")
    wl0 = W.c4_multi_plummer(seeds[0], N=N, nlevels=nlevels)
    solver = NestedPoissonSolver(wl0.geom)
    net = net or GuessNet()
    hist = []
    total = epochs * len(seeds) * (nlevels - 1)
    it = 0
    for ep in range(epochs):
        for si, seed in enumerate(seeds):
            wl = W.c4_multi_plummer(seed, N=N, nlevels=nlevels)
            rho, po = W.make_inputs(wl.geom, wl.prob, device=dev)
            solver.solve(rho, po)
            for x, t in level_samples(solver, nlevels):
                frac = it / max(total - 1, 1)
                cur_lr = lr * (lr_final / lr) ** frac
                if objective == "residual":
                    loss = net.train_step_residual(x, lr=cur_lr)
                else:
                    loss = net.train_step(x, t, lr=cur_lr)
                it += 1
                if it % 50 == 0 or it == total:
                    hist.append((it, float(loss.item())))
                    if log:
                        log("step %d/%d seed %d loss %.4e lr %.2e" % (it, total, seed, hist[-1][1], cur_lr))
    solver.close()
    return net, hist


def save_weights(theta, path=DEFAULT_WEIGHTS):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, np.asarray(theta, dtype=np.float32))


def load_weights(path=DEFAULT_WEIGHTS):
    return np.load(path, allow_pickle=False)
