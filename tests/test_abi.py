"""The C-ABI library on the host (no GPU): it loads, exports every function
include/nested_poisson.h declares, validates geometry before touching a
device, and plans the same multigrid hierarchy as the oracle."""
import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT
from oracle import core
from paper_2001_02327_amd import _lib
from paper_2001_02327_amd import workloads as W


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(nested_poisson_\w+|np_\w+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    declared = _declared()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(L, name), name
    # the binding declares exactly the header's functions
    assert declared == set(_lib.SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (\w+)", out))
    assert declared <= exported


def test_library_links_no_oracle():
    out = subprocess.run(["nm", "-D", _lib.LIB_PATH], capture_output=True, text=True).stdout
    assert "orc_" not in out
    ldd = subprocess.run(["ldd", _lib.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in ldd


def _check_plan(wl, interp_buffer=False):
    cfg = _lib.make_config(wl.geom, buffer="interp" if interp_buffer else "relaxed")
    plan = _lib.plan(cfg)
    d = wl.geom.dim
    for l, p in enumerate(plan):
        N0 = tuple(v + (0 if (interp_buffer and l > 0) else 2) for v in wl.geom.ext(l))
        assert p["N"] == core.plan3(d, N0)
        for L in range(1, len(p["N"])):
            for a in range(d):
                one, c = core.ghost_rule(N0[a], L, p["N"][L][a])
                assert bool(p["xn_is_one"][L][a]) == one
                if not one:
                    assert p["coef"][L][a] == c  # same rational, one rounding


@pytest.mark.parametrize("wl", [W.c1_gaussian_2d(64), W.c2_plummer(128), W.c3_plummer_offset(256),
                                W.c5_two_plummer(512), W.paper2d(1024), W.paper3d(10 * 4), W.box_plummer_3d(1),
                                W.box_plummer_3d(8), W.box_gaussian_2d(4)],
                         ids=lambda w: w.name)
def test_host_plan_matches_oracle(wl):
    _check_plan(wl)


@pytest.mark.parametrize("wl", [W.c2_plummer(128), W.paper2d(64), W.c5_two_plummer(512), W.box_plummer_3d(2)],
                         ids=lambda w: w.name)
def test_host_plan_interp_buffer(wl):
    """With the interpolated buffer, levels l >= 1 plan their hierarchy from
    N^0 = n (Omega^l alone), level 0 from n + 2 as before."""
    _check_plan(wl, interp_buffer=True)


def test_host_plan_refuses_steep_ghost_lines():
    """A hierarchy whose right-ghost gain |c| / (2d) exceeds NP_MAX_GHOST_GAIN
    (N^0 = 194: c = -63 on multigrid level 7) is refused with a message, as
    the oracle refuses it; one just inside the bound is accepted."""
    bad = W.box_geometry(2, (192, 200), (8, 16), (2, 4), dx0=1.0 / 16)
    with pytest.raises(_lib.NestedPoissonError) as ei:
        _lib.plan(_lib.make_config(bad))
    assert ei.value.code == _lib.NP_EINVAL
    assert "right-ghost coefficient" in str(ei.value)
    assert not core.plan_stable(2, (194, 202))
    ok = W.box_geometry(2, (196, 200), (8, 16), (2, 4), dx0=1.0 / 16)
    _lib.plan(_lib.make_config(ok))
    assert core.plan_stable(2, (198, 202))


def _bad(**kw):
    g = W.centred_geometry(3, 3, 16, 0.5, 1.0)
    cfg = _lib.make_config(g)
    for k, v in kw.items():
        if k == "n":
            cfg.n[v[0]] = v[1]
        elif k == "off":
            cfg.offset[v[0]][v[1]] = v[2]
        else:
            setattr(cfg, k, v)
    return cfg


@pytest.mark.parametrize("kw", [
    dict(dim=4), dict(nlevels=0), dict(nlevels=9), dict(nlevels=17), dict(n=(1, 7)), dict(n=(0, 2)), dict(off=(1, 0, 0)),
    dict(off=(2, 2, 9)), dict(dx0=0.0), dict(tol=-1.0), dict(max_cycles=0), dict(max_cycles=100000),
    dict(n_pre=-1), dict(stop_rule=7), dict(inner_cycles=-1), dict(inner_cycles=9), dict(buffer=2),
    dict(buffer=1, precision=1), dict(buffer=1, precision=2), dict(buffer=1, guess=1), dict(buffer=1, stop_rule=1),
    dict(sweep=4), dict(sweep=-1), dict(batch=2), dict(guess_gate=2), dict(guess_gate=-1), dict(coarse_post=-2), dict(coarse_post=17),
], ids=lambda k: ",".join("%s=%s" % kv for kv in k.items()))
def test_invalid_geometry_rejected_before_any_device_call(kw):
    cfg = _bad(**kw)
    p = _lib.NpPlan()
    assert _lib.lib().nested_poisson_plan(ctypes.byref(cfg), ctypes.byref(p)) == _lib.NP_EINVAL
    assert _lib.lib().nested_poisson_last_error(None)
    h = ctypes.c_void_p()
    assert _lib.lib().nested_poisson_create(ctypes.byref(cfg), None, ctypes.byref(h)) == _lib.NP_EINVAL
    assert not h.value


def test_margin_rule_matches_oracle():
    for off in range(0, 12):
        g = W.Geometry(dim=2, n=[16, 12], off=[(0, 0, 0), (off, off, 0)], lo0=(0, 0, 0), dx0=1.0)
        cfg = _lib.make_config(g)
        ok = _lib.lib().nested_poisson_plan(ctypes.byref(cfg), ctypes.byref(_lib.NpPlan())) == 0
        assert ok == core.validate(g), off


def test_null_handle_calls_are_safe():
    L = _lib.lib()
    assert L.nested_poisson_forces(None, 0, None, None, None) == _lib.NP_EINVAL
    assert L.nested_poisson_potential(None, 0, None) == _lib.NP_EINVAL
    assert L.nested_poisson_set_fixed_cycles(None, None) == _lib.NP_EINVAL
    L.nested_poisson_destroy(None)
    assert L.nested_poisson_strerror(_lib.NP_ENOTCONV) == b"not converged"


def test_plan_accepts_every_even_patch_size():
    """Every even n (so every N^0 = n + 2) plans within the index bounds the
    kernels rely on (checked inside nested_poisson_plan), unless a level's
    right-ghost gain is beyond the bound, exactly where the oracle refuses it
    too (297 of the 2998 sizes, 192, 320, 384, ... among them; none of the
    paper's or the benchmark's)."""
    refused = []
    for n in range(4, 6000, 2):
        g = W.Geometry(dim=3, n=[n], off=[(0, 0, 0)], lo0=(0, 0, 0), dx0=1.0)
        cfg = _lib.make_config(g)
        rc = _lib.lib().nested_poisson_plan(ctypes.byref(cfg), ctypes.byref(_lib.NpPlan()))
        stable = core.plan_stable(3, (n + 2,) * 3)
        assert (rc == 0) == stable, n
        if rc:
            assert b"right-ghost coefficient" in _lib.lib().nested_poisson_last_error(None), n
            refused.append(n)
    assert len(refused) == 297
    for n in (16, 32, 64, 128, 256, 512, 1020, 1024):
        assert n not in refused


def _tree_cfg(parent=None, off=None):
    g = W.two_patch_geometry(3, 32)
    cfg = _lib.make_config(g)
    if parent is not None:
        for l, p in enumerate(parent):
            cfg.parent[l] = p
    if off is not None:
        l, o = off
        for a in range(3):
            cfg.offset[l][a] = o[a]
    return cfg


def test_default_parents_are_the_stack():
    cfg = _lib.NpConfig()
    _lib.lib().nested_poisson_default_config(ctypes.byref(cfg))
    assert [cfg.parent[l] for l in range(_lib.NP_MAX_LEVELS)] == list(range(-1, _lib.NP_MAX_LEVELS - 1))


def test_default_settings():
    """The defaults the header states: the paper's V(2,1) on every level, tol
    1e-10, 50 cycles, FP64, full sweeps, batched patches and the learned guess's
    cost gate on."""
    cfg = _lib.NpConfig()
    _lib.lib().nested_poisson_default_config(ctypes.byref(cfg))
    assert (cfg.n_pre, cfg.n_post, cfg.tol, cfg.max_cycles) == (2, 1, 1e-10, 50)
    assert (cfg.precision, cfg.sweep, cfg.batch, cfg.guess_gate, cfg.coarse_post) == (0, _lib.SWEEPS["full"], 1, 1, -1)
    assert _lib.make_config(W.c2_plummer(16).geom).guess_gate == 1
    assert _lib.make_config(W.c2_plummer(16).geom, guess_gate=False).guess_gate == 0


def test_patch_tree_plans_and_validates_like_the_oracle():
    cfg = _tree_cfg()
    assert _lib.lib().nested_poisson_plan(ctypes.byref(cfg), ctypes.byref(_lib.NpPlan())) == 0
    assert core.validate(W.two_patch_geometry(3, 32))
    plan = _lib.plan(cfg)
    assert [p["N"][0] for p in plan] == [(34, 34, 34)] + [(18, 18, 18)] * 3


@pytest.mark.parametrize("bad", [
    dict(parent=[-1, 0, 2, 1]),            # parent not an earlier entry
    dict(parent=[-1, -1, 0, 1]),           # negative parent
    dict(parent=[-1, 0, 0, 0], off=(3, (5, 13, 13))),  # grandchild moved under the base, onto patch A
    dict(off=(2, (6, 10, 12))),            # patch B moved onto patch A
    dict(off=(3, (1, 1, 9))),              # grandchild beyond its parent's margin
], ids=["later_parent", "negative_parent", "overlap_base", "overlap_sibling", "margin"])
def test_invalid_patch_trees_rejected(bad):
    cfg = _tree_cfg(**bad)
    assert _lib.lib().nested_poisson_plan(ctypes.byref(cfg), ctypes.byref(_lib.NpPlan())) == _lib.NP_EINVAL
    g = W.two_patch_geometry(3, 32)
    if "parent" in bad:
        g.parent = bad["parent"]
    if "off" in bad:
        l, o = bad["off"]
        g.off = list(g.off)
        g.off[l] = o
    assert not core.validate(g)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library every entry point raises (no CPU fallback)."""
    from paper_2001_02327_amd.solver import NestedPoissonSolver
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.lib()
    g = W.centred_geometry(3, 2, 16, 0.5, 1.0)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.plan(_lib.make_config(g))
    # the solver refuses too (here, without a device, before it reaches the library)
    with pytest.raises(RuntimeError):
        NestedPoissonSolver(g)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU and says so for --gpus N > 1 (before touching a device)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr


def test_guess_weight_blob_on_the_host():
    """The versioned parameter blob: packing rounds the weights to bfloat16
    (nearest even) and copies the FP32 biases; the check refuses a wrong
    magic, version, layer shape, size or a non-finite bias.  Host only."""
    import numpy as np
    from paper_2001_02327_amd import learned
    theta = learned.init_params(7)
    theta[-1] = 0.25
    blob = _lib.pack_guess_weights(theta)
    assert len(blob) == _lib.NP_GUESS_BLOB_BYTES
    L = _lib.lib()
    hdr = np.frombuffer(blob[:_lib.NP_GUESS_BLOB_HEADER], dtype="<u4")
    assert list(hdr) == [_lib.NP_GUESS_BLOB_MAGIC, _lib.NP_GUESS_BLOB_VERSION, 3, 2, 16, 16, 16, 16, 1, 0]
    # layer 1 weights: bfloat16 round-to-nearest-even of the FP32 values
    nw = 27 * 2 * 16
    w = np.frombuffer(blob[_lib.NP_GUESS_BLOB_HEADER:_lib.NP_GUESS_BLOB_HEADER + 2 * nw], dtype="<u2")
    u = theta[:nw].astype(np.float32).view(np.uint32).astype(np.uint64)
    assert np.array_equal(w, ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16))
    b = np.frombuffer(blob[_lib.NP_GUESS_BLOB_HEADER + 2 * nw:_lib.NP_GUESS_BLOB_HEADER + 2 * nw + 64], dtype="<f4")
    assert np.array_equal(b, theta[nw:nw + 16])
    last = np.frombuffer(blob[-4:], dtype="<f4")
    assert last[0] == np.float32(0.25)

    def check(bb):
        buf = ctypes.create_string_buffer(bytes(bb), len(bb))
        return L.nested_poisson_check_guess_weights(buf, len(bb))

    assert check(blob) == 0
    for pos, val in ((0, 0x00), (4, 2), (8, 4), (12, 3), (32, 2)):
        bad = bytearray(blob)
        bad[pos] = val
        assert check(bad) == _lib.NP_EINVAL, pos
    assert check(blob[:-1]) == _lib.NP_EINVAL
    assert check(blob + b"\0") == _lib.NP_EINVAL
    bad = bytearray(blob)
    bad[-4:] = np.array([np.nan], dtype="<f4").tobytes()
    assert check(bad) == _lib.NP_EINVAL
    assert b"non-finite" in L.nested_poisson_last_error(None)
    # wrong parameter count
    short = np.zeros(100, dtype=np.float32)
    buf = ctypes.create_string_buffer(_lib.NP_GUESS_BLOB_BYTES)
    assert L.nested_poisson_pack_guess_weights(short.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), 100, buf,
                                               _lib.NP_GUESS_BLOB_BYTES) == _lib.NP_EINVAL


def test_profile_classes_match_the_header():
    """The ctypes mirror of np_profile and the class names follow the header's
    NP_KCLASS_* numbering (no device needed)."""
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                            "nested_poisson.h")).read()
    classes = {int(v): k for k, v in re.findall(r"#define NP_KCLASS_(\w+) (\d+)", hdr)}
    n = int(re.search(r"#define NP_NKCLASS (\d+)", hdr).group(1))
    assert n == _lib.NP_NKCLASS and len(classes) <= n
    assert [classes[i].lower() for i in range(len(classes))] == _lib.KCLASSES
    assert ctypes.sizeof(_lib.NpProfile) == n * (ctypes.sizeof(ctypes.c_long) + ctypes.sizeof(ctypes.c_double))
    sweeps = dict(re.findall(r"#define NP_SWEEP_(\w+) (\d+)", hdr))
    assert {k.lower(): int(v) for k, v in sweeps.items()} == _lib.SWEEPS
