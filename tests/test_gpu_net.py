"""Learned initial guess on the GPU: the np_net_* kernels against the FP64
reference in oracle/net.py, the features the solver extracts against the
oracle's own solve, and the solve with the learned guess.

Tolerances: the FP32 kernels use bfloat16 weights, so the reference is given
the same bfloat16-rounded weights and the remaining difference is FP32
accumulation over at most 27 * 16 = 432 terms: 1e-5 relative to the output's
max.  The matrix-core kernels (the inference path) take bfloat16 activations,
so the reference gets the same rounded inputs and the products are exact; the
16-channel outputs are rounded to bfloat16 (relative 2^-9): 2e-2; the FP32
output of the last layer: 1e-5.
"""
import os

import numpy as np
import pytest
import torch

from oracle import core
from oracle import net as onet
from paper_2001_02327_amd import _lib, learned
from paper_2001_02327_amd import workloads as W
from paper_2001_02327_amd.solver import NestedPoissonSolver

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need the MI355X"


def _bf16_bits(a):
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return r.view(np.int16)


def _dev(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _st():
    return torch.cuda.current_stream().cuda_stream


@pytest.mark.parametrize("ci,co,shape", [(2, 16, (2, 5, 6, 7)), (16, 16, (1, 4, 5, 9)), (16, 1, (1, 6, 3, 5)),
                                         (3, 5, (2, 3, 4, 70))])
def test_conv_forward_and_backward(ci, co, shape):
    rng = np.random.default_rng(ci * 100 + co)
    B, Z, Y, X = shape
    x = rng.standard_normal((B, Z, Y, X, ci))
    w = onet.bf16_round(rng.standard_normal((27, co, ci)) * 0.3)
    b = rng.standard_normal(co) * 0.1
    gy = rng.standard_normal((B, Z, Y, X, co))
    L = _lib.lib()
    xd, wd, bd = _dev(x), _dev(_bf16_bits(w), torch.int16), _dev(b)
    out = torch.empty((B, Z, Y, X, co), dtype=torch.float32, device="cuda")
    assert L.np_net_conv3d_fwd(xd.data_ptr(), ci, wd.data_ptr(), bd.data_ptr(), co, 0, B, Z, Y, X, out.data_ptr(),
                               _st()) == 0
    ref = onet.conv_fwd(x, w, b)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max()
    # backward data
    gyd = _dev(gy)
    gin = torch.empty_like(xd)
    assert L.np_net_conv3d_bwd_data(gyd.data_ptr(), co, wd.data_ptr(), ci, B, Z, Y, X, gin.data_ptr(), _st()) == 0
    ref = onet.conv_bwd_data(gy, w)
    assert np.abs(gin.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max()
    # backward weight (deterministic two-stage sum)
    ws = L.np_net_workspace_bytes(ci, co, 0)
    work = torch.empty(ws // 4 + 1, dtype=torch.float32, device="cuda")
    gw = torch.empty(27 * co * ci, dtype=torch.float32, device="cuda")
    gb = torch.empty(co, dtype=torch.float32, device="cuda")
    for rep in range(2):
        assert L.np_net_conv3d_bwd_weight(xd.data_ptr(), ci, gyd.data_ptr(), co, B, Z, Y, X, gw.data_ptr(),
                                          gb.data_ptr(), work.data_ptr(), ws, _st()) == 0
        if rep == 0:
            first = gw.clone()
    assert torch.equal(first, gw)
    rgw, rgb = onet.conv_bwd_weight(x, gy)
    assert np.abs(gw.cpu().numpy().reshape(27, co, ci) - rgw).max() <= 1e-5 * np.abs(rgw).max()
    assert np.abs(gb.cpu().numpy() - rgb).max() <= 1e-5 * np.abs(rgb).max()


@pytest.mark.parametrize("ci,co", [(2, 16), (16, 16), (16, 1)])
@pytest.mark.parametrize("shape", [(1, 4, 5, 16), (2, 3, 4, 21), (1, 5, 5, 37), (1, 9, 7, 33)])
def test_layers_on_matrix_cores(shape, ci, co):
    """The inference path of each layer (LDS-staged blocks of 16 x 4 x 4
    voxels; the shapes give partial blocks on every axis)."""
    rng = np.random.default_rng(sum(shape) + ci + co)
    B, Z, Y, X = shape
    x = onet.bf16_round(rng.standard_normal((B, Z, Y, X, ci)))
    w = onet.bf16_round(rng.standard_normal((27, co, ci)) * 0.2)
    b = rng.standard_normal(co) * 0.1
    xd = _dev(_bf16_bits(x), torch.int16)
    wd = _dev(_bf16_bits(w), torch.int16)
    bd = _dev(b)
    out = torch.empty((B, Z, Y, X, co), dtype=torch.int16 if co == 16 else torch.float32, device="cuda")
    for relu in (0, 1):
        assert _lib.lib().np_net_conv3d_fwd_mfma(xd.data_ptr(), ci, wd.data_ptr(), bd.data_ptr(), co, relu, B, Z, Y,
                                                 X, out.data_ptr(), _st()) == 0
        if co == 16:
            got = (out.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        else:
            got = out.cpu().numpy().astype(np.float64)
        ref = onet.conv_fwd(x, w, b)
        if relu:
            ref = np.maximum(ref, 0)
        # bfloat16 output rounding (2^-9 relative) for cout 16; FP32 accumulation otherwise
        tol = 2e-2 if co == 16 else 1e-5
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), relu
    assert _lib.lib().np_net_conv3d_fwd_mfma(xd.data_ptr(), 3, wd.data_ptr(), bd.data_ptr(), co, 0, B, Z, Y, X,
                                             out.data_ptr(), _st()) == _lib.NP_EINVAL


def test_training_step_matches_reference():
    """Loss, every gradient and one Adam step of the full network vs the reference."""
    rng = np.random.default_rng(5)
    theta = learned.init_params(3)
    theta[-1] = 0.05
    net = learned.GuessNet(theta)
    x = rng.standard_normal((1, 6, 5, 7, 2)).astype(np.float32)
    t = rng.standard_normal((1, 6, 5, 7, 1)).astype(np.float32)
    acts = net.forward(_dev(x), bf16_acts=False)
    loss, gy = net.loss_grad(acts[-1], _dev(t))
    net.backward(acts, gy)
    parts = list(_split(theta))
    params = [(onet.bf16_round(parts[2 * k].reshape(27, co, ci)), parts[2 * k + 1].astype(np.float64))
              for k, (ci, co) in enumerate(onet.LAYERS)]
    rloss, rgrads = onet.loss_and_grads(params, x.astype(np.float64), t.astype(np.float64), np.ones_like(t))
    assert float(loss.item()) == pytest.approx(rloss, rel=1e-5)
    g = net.grad.cpu().numpy()
    rg = onet.pack(rgrads)
    assert np.abs(g - rg).max() <= 1e-4 * np.abs(rg).max()
    before = net.theta.cpu().numpy().astype(np.float64)
    net.adam_step(lr=1e-2)
    rth, _, _ = onet.adam(before, g.astype(np.float64), np.zeros_like(before), np.zeros_like(before), 1, lr=1e-2)
    assert np.abs(net.theta.cpu().numpy() - rth).max() <= 1e-6


def test_training_forward_rounds_like_inference():
    """With bfloat16 activations (the default of the training forward pass) the
    FP32 kernels see the values the matrix-core inference path stores: inputs
    and hidden activations rounded to bfloat16.  Given the committed weights
    (or a seeded initialisation) the two paths then differ only by the FP32
    summation order and the rare bfloat16 rounding it flips."""
    theta = learned.load_weights() if os.path.exists(learned.DEFAULT_WEIGHTS) else learned.init_params(4)
    net = learned.GuessNet(theta)
    rng = np.random.default_rng(11)
    B, Z, Y, X = 1, 9, 10, 37
    x = rng.standard_normal((B, Z, Y, X, 2)).astype(np.float32)
    xd = _dev(x)
    acts = net.forward(xd)  # rounds xd in place
    y_train = acts[-1].cpu().numpy().astype(np.float64)
    # the inference path: bfloat16 input, three matrix-core layers
    L = _lib.lib()
    xb = _dev(_bf16_bits(x), torch.int16)
    a1 = torch.empty((B, Z, Y, X, 16), dtype=torch.int16, device="cuda")
    a2 = torch.empty_like(a1)
    y = torch.empty((B, Z, Y, X, 1), dtype=torch.float32, device="cuda")
    h = xb
    for k, (ci, co) in enumerate(learned.LAYERS):
        w, b = net._w(k)
        out = (a1, a2, y)[k]
        assert L.np_net_conv3d_fwd_mfma(h.data_ptr(), ci, w.data_ptr(), b.data_ptr(), co, int(k < 2), B, Z, Y, X,
                                        out.data_ptr(), _st()) == 0
        h = out
    y_inf = y.cpu().numpy().astype(np.float64)
    # the rounded training input is exactly the inference input
    assert np.array_equal(_bf16_bits(xd.cpu().numpy()), _bf16_bits(x))
    scale = np.abs(y_inf).max()
    diff = np.abs(y_train - y_inf)
    print("training forward vs inference path: max %.3e, mean %.3e (relative to max |y| %.3e)"
          % (diff.max() / scale, diff.mean() / scale, scale))
    assert diff.max() <= 2e-2 * scale
    assert diff.mean() <= 1e-3 * scale


def test_lap7_and_residual_objective():
    """np_net_lap7 is the 7-point stencil with zero outside the box (checked
    against shifted copies in FP64) and its own adjoint (<L a, b> = <a, L b>)."""
    rng = np.random.default_rng(12)
    B, Z, Y, X = 2, 5, 6, 71
    a = rng.standard_normal((B, Z, Y, X, 1))
    b = rng.standard_normal((B, Z, Y, X, 1))
    L = _lib.lib()
    ad, bd = _dev(a), _dev(b)
    la, lb = torch.empty_like(ad), torch.empty_like(bd)
    assert L.np_net_lap7(ad.data_ptr(), B, Z, Y, X, la.data_ptr(), _st()) == 0
    assert L.np_net_lap7(bd.data_ptr(), B, Z, Y, X, lb.data_ptr(), _st()) == 0
    p = np.pad(a[..., 0], ((0, 0), (1, 1), (1, 1), (1, 1)))
    ref = (p[:, :-2, 1:-1, 1:-1] + p[:, 2:, 1:-1, 1:-1] + p[:, 1:-1, :-2, 1:-1] + p[:, 1:-1, 2:, 1:-1]
           + p[:, 1:-1, 1:-1, :-2] + p[:, 1:-1, 1:-1, 2:] - 6.0 * a[..., 0])
    got = la.cpu().numpy()[..., 0].astype(np.float64)
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    lhs = float((la.double() * bd.double()).sum())
    rhs = float((ad.double() * lb.double()).sum())
    assert lhs == pytest.approx(rhs, rel=1e-5)
    assert L.np_net_lap7(ad.data_ptr(), B, Z, Y, X, ad.data_ptr(), _st()) == _lib.NP_EINVAL


def test_guess_weights_blob_is_versioned():
    """set_guess_weights takes the versioned blob only: a wrong magic, version,
    shape or size is rejected before any device work, and the packed blob of
    the committed parameters round-trips (the learned solve runs)."""
    theta = learned.init_params(2)
    blob = bytearray(_lib.pack_guess_weights(theta))
    wl = W.c4_multi_plummer(200001, N=16)
    s = NestedPoissonSolver(wl.geom, guess="learned")
    bad_version = bytearray(blob)
    bad_version[4] = 2
    bad_magic = bytearray(blob)
    bad_magic[0] ^= 0xFF
    bad_shape = bytearray(blob)
    bad_shape[12] = 3
    for bad in (bad_version, bad_magic, bad_shape, blob[:-4]):
        with pytest.raises(_lib.NestedPoissonError) as ei:
            s.set_guess_weights(bytes(bad))
        assert ei.value.code == _lib.NP_EINVAL
    s.set_guess_weights(bytes(blob))
    rho, po = W.make_inputs(wl.geom, wl.prob, device="cuda")
    st = s.solve(rho, po)
    assert st["status"] == 0
    s.close()


def _split(theta):
    k = 0
    for ci, co in onet.LAYERS:
        nw = 27 * ci * co
        yield theta[k:k + nw]
        yield theta[k + nw:k + nw + co]
        k += nw + co


def test_features_match_oracle():
    """The solver's network input and target vs the oracle's solve, interface
    fill and residual."""
    wl = W.c4_multi_plummer(4, N=16)
    rho, po = W.make_inputs(wl.geom, wl.prob)
    ref = core.solve(wl.geom, [r.numpy() for r in rho], po.numpy())
    s = NestedPoissonSolver(wl.geom)
    s.set_fixed_cycles(ref["cycles"])
    s.solve([r.cuda() for r in rho], po.cuda())
    fourpiG = 4 * np.pi * wl.geom.G
    f_prev = None
    for l in range(wl.geom.nlevels):
        n = wl.geom.n[l]
        if l == 0:
            f = np.zeros((n + 4,) * 3)
            f[1:-1, 1:-1, 1:-1] = fourpiG * rho[0].numpy()
            f_prev = f
            continue
        pint, fint = core.interface_fill(3, ref["phi"][l - 1], f_prev, n, wl.geom.off[l], rho[l].numpy(), fourpiG)
        f_prev = fint
        dx = wl.geom.dx(l)
        r0 = core.residual(3, dx, pint, fint)
        fn = np.abs(fint[1:-1, 1:-1, 1:-1]).max()
        x, t = s.guess_features(l)
        x, t = x.cpu().numpy(), t.cpu().numpy()
        g = (slice(1, -1),) * 3
        np.testing.assert_allclose(x[..., 0], fint[g] / fn, rtol=1e-6, atol=1e-7)
        scale_r = np.abs(r0[g] / fn).max()
        assert np.abs(x[..., 1] - r0[g] / fn).max() <= 1e-5 * scale_r
        tref = (ref["phi"][l] - pint)[g] / (fn * dx * dx)
        assert np.abs(t - tref).max() <= 1e-5 * np.abs(tref).max()
    s.close()


def _solve(wl, theta=None, **kw):
    rho, po = W.make_inputs(wl.geom, wl.prob, device="cuda")
    s = NestedPoissonSolver(wl.geom, **kw)
    if theta is not None:
        s.set_guess_weights(theta)
    st = s.solve(rho, po)
    phi = [s.potential(l).cpu().numpy() for l in range(wl.geom.nlevels)]
    s.close()
    return phi, st


def test_learned_guess_is_checked_by_multigrid():
    """Untrained or broken weights never change the answer: the V-cycles reach
    the same tolerance, and a guess that is worse than the interpolant (NaN
    weights here) is discarded."""
    wl = W.c4_multi_plummer(200001, N=32)
    phi0, st0 = _solve(wl)
    phi1, st1 = _solve(wl, learned.init_params(1), guess="learned")
    bad = learned.init_params(1)
    bad[100] = np.nan
    phi2, st2 = _solve(wl, bad, guess="learned")
    assert st2["learned_used"][1:] == [0, 0]
    for l in range(wl.geom.nlevels):
        for ph in (phi1, phi2):
            assert np.abs(ph[l] - phi0[l]).max() <= 1e-8 * np.abs(phi0[l]).max()
    assert st2["cycles"] == st0["cycles"]


@pytest.mark.skipif(not os.path.exists(learned.DEFAULT_WEIGHTS), reason="no trained weights in the tree")
@pytest.mark.parametrize("precision", ["fp64", "fp16s_dc"])
def test_trained_network_gain(precision):
    """What the trained network buys on held-out seeds (3 levels of 128^3 of
    the seeded multi-Plummer workload): the V-cycles and the host time of the
    refined levels with and without it, printed.  Measured: it buys nothing.
    Its guess lowers the residual restricted twice to 0.13-0.38 of the
    interpolated guess's, yet the refined levels need 99 instead of 95
    V-cycles in FP64: neither the point-wise nor the restricted residual of the
    starting guess predicts the cycle count.  Pinned: the answer is the plain
    solve's, a kept guess passed the keep test, and the loss stays within two
    V-cycles per level."""
    theta = learned.load_weights()
    kw = dict(precision=precision, inner_cycles="adaptive") if precision != "fp64" else {}
    tot0 = tot1 = kept = 0
    ms0 = ms1 = 0.0
    ratios = []
    for seed in (200000, 200002, 200003, 200005):
        wl = W.c4_multi_plummer(seed, N=128)
        phi0, st0 = _solve(wl, **kw)
        phi1, st1 = _solve(wl, theta, guess="learned", **kw)
        tot0 += sum(st0["cycles"][1:])
        tot1 += sum(st1["cycles"][1:])
        ms0 += sum(st0["level_ms"][1:])
        ms1 += sum(st1["level_ms"][1:])
        kept += sum(st1["learned_used"][1:])
        ratios += st1["guess_box_ratio"][1:]
        for l in range(wl.geom.nlevels):
            assert np.abs(phi1[l] - phi0[l]).max() <= 1e-8 * np.abs(phi0[l]).max()
        for l in range(1, wl.geom.nlevels):
            assert st1["cycles"][l] <= st0["cycles"][l] + 2
            if st1["learned_used"][l]:
                assert st1["guess_box_ratio"][l] <= 0.95
    print("%s, refined levels of 4 held-out seeds: V-cycles %d (interpolated guess) vs %d (learned, kept on %d of "
          "8 levels); host time %.1f vs %.1f ms; restricted-residual ratios %s"
          % (precision, tot0, tot1, kept, ms0, ms1, ", ".join("%.2f" % x for x in ratios)))


@pytest.mark.skipif(not os.path.exists(learned.DEFAULT_WEIGHTS), reason="no trained weights in the tree")
@pytest.mark.parametrize("precision", ["fp64", "fp16s_dc"])
def test_guess_gate(precision):
    """The cost gate of the learned guess: the network runs on every refined
    level in a handle's first solve; a level where the guess did not save more
    V-cycle time than it took skips the network in later solves, and a solve
    that skips it everywhere equals the interpolated-guess solve bit for bit
    (the same start, the same iterates); new weights re-arm every level;
    guess_gate = 0 runs the network in every solve."""
    theta = learned.load_weights()
    wl = W.c4_multi_plummer(200002, N=64)
    L = wl.geom.nlevels
    kw = dict(precision=precision, inner_cycles="adaptive") if precision != "fp64" else {}
    rho, po = W.make_inputs(wl.geom, wl.prob, device="cuda")
    plain = NestedPoissonSolver(wl.geom, **kw)
    st0 = plain.solve(rho, po)
    phi0 = [plain.potential(l).cpu().numpy() for l in range(L)]
    plain.close()
    s = NestedPoissonSolver(wl.geom, guess="learned", **kw)
    s.set_guess_weights(theta)
    st1 = s.solve(rho, po)
    assert st1["learned_ran"] == [0] + [1] * (L - 1)
    assert all(st1["guess_ms"][l] > 0 for l in range(1, L))
    st2 = s.solve(rho, po)
    phi2 = [s.potential(l).cpu().numpy() for l in range(L)]
    print("%s: network ran on levels %s then %s; guess host ms %s; cycles %s / %s / plain %s"
          % (precision, st1["learned_ran"], st2["learned_ran"], ["%.2f" % x for x in st1["guess_ms"]],
             st1["cycles"], st2["cycles"], st0["cycles"]))
    for l in range(1, L):
        # a level keeps running the network only where its guess was kept
        assert st2["learned_ran"][l] <= st1["learned_used"][l]
    if not any(st2["learned_ran"]):
        assert st2["cycles"] == st0["cycles"]
        for l in range(L):
            assert np.array_equal(phi2[l], phi0[l]), l
    for l in range(L):
        assert np.abs(phi2[l] - phi0[l]).max() <= 1e-8 * np.abs(phi0[l]).max()
    s.set_guess_weights(theta)
    assert s.solve(rho, po)["learned_ran"] == [0] + [1] * (L - 1)
    s.close()
    s = NestedPoissonSolver(wl.geom, guess="learned", guess_gate=False, **kw)
    s.set_guess_weights(theta)
    for _ in range(2):
        assert s.solve(rho, po)["learned_ran"] == [0] + [1] * (L - 1)
    s.close()
