"""ctypes declarations of the C ABI in include/nested_poisson.h.

Loads paper_2001_02327_amd/libnested_poisson.so (built in-tree by
paper_2001_02327_amd/build.py).  There is no fallback: if the library is
missing every entry point raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnested_poisson.so")

NP_MAX_LEVELS = 16
NP_MAX_MG = 32

NP_OK = 0
NP_EINVAL = -1
NP_ENOMEM = -2
NP_EHIP = -3
NP_ENONFINITE = -4
NP_ENOTCONV = -5
NP_EDIVERGED = -6
NP_ESTATE = -7
NP_ENODEV = -8

STOP_RULES = {"residual": 0, "force_delta": 1}
PRECISIONS = {"fp64": 0, "fp32_dc": 1, "fp16s_dc": 2}
GUESSES = {"interp": 0, "learned": 1}
BUFFERS = {"relaxed": 0, "interp": 1}
SWEEPS = {"full": 0, "half": 1, "fused": 2, "full_all": 3}


class NpConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("nlevels", ctypes.c_int),
        ("n", ctypes.c_int * NP_MAX_LEVELS),
        ("offset", (ctypes.c_int * 3) * NP_MAX_LEVELS),
        ("dx0", ctypes.c_double),
        ("G", ctypes.c_double),
        ("n_pre", ctypes.c_int),
        ("n_post", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("max_cycles", ctypes.c_int),
        ("stop_rule", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("inner_cycles", ctypes.c_int),
        ("guess", ctypes.c_int),
        ("buffer", ctypes.c_int),
        ("parent", ctypes.c_int * NP_MAX_LEVELS),
        ("extent", (ctypes.c_int * 3) * NP_MAX_LEVELS),
        ("batch", ctypes.c_int),
        ("sweep", ctypes.c_int),
        ("guess_gate", ctypes.c_int),
        ("coarse_post", ctypes.c_int),
    ]


class NpPlan(ctypes.Structure):
    _fields_ = [
        ("nmg", ctypes.c_int * NP_MAX_LEVELS),
        ("N", ((ctypes.c_int * 3) * NP_MAX_MG) * NP_MAX_LEVELS),
        ("xn_is_one", ((ctypes.c_int * 3) * NP_MAX_MG) * NP_MAX_LEVELS),
        ("ghost_coef", ((ctypes.c_double * 3) * NP_MAX_MG) * NP_MAX_LEVELS),
    ]


class NpStats(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int * NP_MAX_LEVELS),
        ("initial_rel_residual", ctypes.c_double * NP_MAX_LEVELS),
        ("final_rel_residual", ctypes.c_double * NP_MAX_LEVELS),
        ("scale", ctypes.c_double * NP_MAX_LEVELS),
        ("level_ms", ctypes.c_double * NP_MAX_LEVELS),
        ("total_ms", ctypes.c_double),
        ("learned_used", ctypes.c_int * NP_MAX_LEVELS),
        ("interp_rel_residual", ctypes.c_double * NP_MAX_LEVELS),
        ("outer_steps", ctypes.c_int * NP_MAX_LEVELS),
        ("guess_box_ratio", ctypes.c_double * NP_MAX_LEVELS),
        ("learned_ran", ctypes.c_int * NP_MAX_LEVELS),
        ("guess_ms", ctypes.c_double * NP_MAX_LEVELS),
    ]


NP_NKCLASS = 16
KCLASSES = ["smooth", "restrict", "prolong", "coarse", "norm", "fill", "forces", "dc", "guess", "seeded", "full",
            "full_res", "dc_scale", "black_restrict"]
NP_NET_PARAMS = 8241
NP_NET_MSE_NOALLOC_MAX = 1 << 28
NP_GUESS_BLOB_MAGIC = 0x5747504E
NP_GUESS_BLOB_VERSION = 1
NP_GUESS_BLOB_HEADER = 40
NP_GUESS_BLOB_BYTES = NP_GUESS_BLOB_HEADER + 2 * 27 * (2 * 16 + 16 * 16 + 16 * 1) + 4 * (16 + 16 + 1)


class NpProfile(ctypes.Structure):
    _fields_ = [("count", ctypes.c_long * NP_NKCLASS), ("ms", ctypes.c_double * NP_NKCLASS)]


# every symbol the header declares, with its signature
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "nested_poisson_default_config": (None, [ctypes.POINTER(NpConfig)]),
    "nested_poisson_plan": (ctypes.c_int, [ctypes.POINTER(NpConfig), ctypes.POINTER(NpPlan)]),
    "nested_poisson_create": (ctypes.c_int, [ctypes.POINTER(NpConfig), _vp, ctypes.POINTER(_vp)]),
    "nested_poisson_solve": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), _vp, ctypes.POINTER(NpStats)]),
    "nested_poisson_set_fixed_cycles": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    "nested_poisson_history": (ctypes.c_int, [_vp, ctypes.c_int, _dp, ctypes.c_int]),
    "nested_poisson_forces": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
    "nested_poisson_potential": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
    "nested_poisson_set_profiling": (ctypes.c_int, [_vp, ctypes.c_int]),
    "nested_poisson_get_profile": (ctypes.c_int, [_vp, ctypes.POINTER(NpProfile)]),
    "nested_poisson_pack_guess_weights": (ctypes.c_int, [ctypes.POINTER(ctypes.c_float), ctypes.c_size_t, _vp,
                                                          ctypes.c_size_t]),
    "nested_poisson_check_guess_weights": (ctypes.c_int, [_vp, ctypes.c_size_t]),
    "nested_poisson_set_guess_weights": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "nested_poisson_guess_features": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp]),
    "np_net_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_long]),
    "np_net_conv3d_fwd": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "np_net_conv3d_fwd_mfma": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "np_net_conv3d_bwd_data": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "np_net_conv3d_bwd_weight": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "np_net_relu_bwd": (ctypes.c_int, [_vp, _vp, ctypes.c_long, _vp]),
    "np_net_mse": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_long, ctypes.c_float, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "np_net_mse_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_long, ctypes.c_float, _vp, _vp, _vp]),
    "np_net_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_long, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_int, _vp, _vp]),
    "np_net_to_bf16": (ctypes.c_int, [_vp, _vp, ctypes.c_long, _vp]),
    "np_net_round_bf16": (ctypes.c_int, [_vp, ctypes.c_long, _vp]),
    "np_net_lap7": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "nested_poisson_destroy": (None, [_vp]),
    "nested_poisson_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "nested_poisson_last_error": (ctypes.c_char_p, [_vp]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built; run `python -m paper_2001_02327_amd.build` "
                               "(there is no CPU fallback)" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class NestedPoissonError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (lib().nested_poisson_strerror(code).decode(), code, msg))
        self.code = code


def make_config(geom, n_pre=2, n_post=1, tol=1e-10, max_cycles=50, stop_rule="residual", precision="fp64",
                inner_cycles=1, guess="interp", buffer="relaxed", batch=True, sweep="full", guess_gate=True,
                coarse_post=None):
    """np_config from a geometry (attributes dim, n, off, dx0, G) and solver settings."""
    c = NpConfig()
    lib().nested_poisson_default_config(ctypes.byref(c))
    c.dim = int(geom.dim)
    c.nlevels = len(geom.n)
    for l, n in enumerate(geom.n):
        if isinstance(n, (tuple, list)):
            # a box: cells per axis (n[l] unused)
            for a in range(3):
                c.extent[l][a] = int(n[a]) if a < len(n) else 0
        else:
            c.n[l] = int(n)
        off = list(geom.off[l]) + [0, 0, 0]
        for a in range(3):
            c.offset[l][a] = int(off[a])
    c.dx0 = float(geom.dx0)
    c.G = float(geom.G)
    c.n_pre, c.n_post = int(n_pre), int(n_post)
    c.tol = float(tol)
    c.max_cycles = int(max_cycles)
    c.stop_rule = STOP_RULES[stop_rule] if isinstance(stop_rule, str) else int(stop_rule)
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.inner_cycles = 0 if inner_cycles == "adaptive" else int(inner_cycles)
    c.guess = GUESSES[guess] if isinstance(guess, str) else int(guess)
    c.buffer = BUFFERS[buffer] if isinstance(buffer, str) else int(buffer)
    c.batch = 1 if batch else 0
    c.sweep = SWEEPS[sweep] if isinstance(sweep, str) else int(sweep)
    c.guess_gate = 1 if guess_gate else 0
    c.coarse_post = -1 if coarse_post is None else int(coarse_post)
    parent = getattr(geom, "parent", None)
    if parent is not None:
        for l, p in enumerate(parent):
            c.parent[l] = int(p)
    return c


def plan(cfg):
    """Validate and plan on the host (no device needed)."""
    p = NpPlan()
    rc = lib().nested_poisson_plan(ctypes.byref(cfg), ctypes.byref(p))
    if rc:
        raise NestedPoissonError(rc, lib().nested_poisson_last_error(None).decode())
    out = []
    d = cfg.dim
    for l in range(cfg.nlevels):
        m = p.nmg[l]
        out.append(dict(N=[tuple(p.N[l][L][a] for a in range(d)) for L in range(m)],
                        xn_is_one=[tuple(p.xn_is_one[l][L][a] for a in range(d)) for L in range(m)],
                        coef=[tuple(p.ghost_coef[l][L][a] for a in range(d)) for L in range(m)]))
    return out


def pack_guess_weights(theta):
    """The library's versioned parameter blob (bytes) of an FP32 parameter vector."""
    import numpy as np
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).reshape(-1))
    buf = ctypes.create_string_buffer(NP_GUESS_BLOB_BYTES)
    rc = lib().nested_poisson_pack_guess_weights(th.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), th.size, buf,
                                                 NP_GUESS_BLOB_BYTES)
    if rc:
        raise NestedPoissonError(rc, lib().nested_poisson_last_error(None).decode())
    return buf.raw
