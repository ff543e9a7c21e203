"""Python handle over the C ABI (argument marshalling only).

Device memory comes from torch (ROCm) tensors; every step of the solve runs
in the HIP library.  Inputs are float64 tensors on the solver's device,
indexed [k, j, i] (x fastest), shapes per axis from the geometry:
    rho[0]: n0_a + 2, rho[l>=1]: n_l,a, phi_outer: n0_a + 4.
"""
import ctypes

import torch

from . import _lib


class NestedPoissonSolver:
    def __init__(self, geom, stream=None, **settings):
        if not torch.cuda.is_available():
            raise RuntimeError("NestedPoissonSolver needs a HIP device")
        self.geom = geom
        self.dim = int(geom.dim)
        self.n = list(geom.n)
        self.cfg = _lib.make_config(geom, **settings)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        rc = _lib.lib().nested_poisson_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                              ctypes.byref(self._h))
        if rc:
            raise _lib.NestedPoissonError(rc, _lib.lib().nested_poisson_last_error(None).decode())
        self.last_stats = None

    # ------------------------------------------------------------------
    def _check(self, rc, allow=()):
        if rc and rc not in allow:
            raise _lib.NestedPoissonError(rc, _lib.lib().nested_poisson_last_error(self._h).decode())
        return rc

    def _shape(self, l, pad):
        """[k, j, i] shape of level l's cells with `pad` extra cells on every side."""
        n = self.n[l]
        ext = tuple(n) if isinstance(n, (tuple, list)) else (int(n),) * self.dim
        return tuple(v + 2 * pad for v in reversed(ext))

    def _tensor(self, t, shape, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device:
            raise TypeError("%s must be a float64 tensor on %s" % (name, self.device))
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError("%s must be contiguous with shape %s (got %s)" % (name, tuple(shape), tuple(t.shape)))
        return t

    def solve(self, rho, phi_outer, allow_notconv=False):
        d = self.dim
        if len(rho) != len(self.n):
            raise ValueError("need one density array per level")
        rho = [self._tensor(rho[0], self._shape(0, 1), "rho[0]")] + \
              [self._tensor(rho[l], self._shape(l, 0), "rho[%d]" % l) for l in range(1, len(self.n))]
        phi_outer = self._tensor(phi_outer, self._shape(0, 2), "phi_outer")
        ptrs = (ctypes.c_void_p * len(rho))(*[r.data_ptr() for r in rho])
        st = _lib.NpStats()
        rc = _lib.lib().nested_poisson_solve(self._h, ptrs, ctypes.c_void_p(phi_outer.data_ptr()), ctypes.byref(st))
        self._check(rc, allow=(_lib.NP_ENOTCONV,) if allow_notconv else ())
        L = len(self.n)
        self.last_stats = dict(
            status=rc,
            cycles=[st.cycles[l] for l in range(L)],
            initial_rel_residual=[st.initial_rel_residual[l] for l in range(L)],
            final_rel_residual=[st.final_rel_residual[l] for l in range(L)],
            scale=[st.scale[l] for l in range(L)],
            level_ms=[st.level_ms[l] for l in range(L)],
            total_ms=st.total_ms,
            learned_used=[st.learned_used[l] for l in range(L)],
            interp_rel_residual=[st.interp_rel_residual[l] for l in range(L)],
            outer_steps=[st.outer_steps[l] for l in range(L)],
            guess_box_ratio=[st.guess_box_ratio[l] for l in range(L)],
            learned_ran=[st.learned_ran[l] for l in range(L)],
            guess_ms=[st.guess_ms[l] for l in range(L)],
        )
        return self.last_stats

    def set_fixed_cycles(self, cycles):
        if cycles is None:
            self._check(_lib.lib().nested_poisson_set_fixed_cycles(self._h, None))
            return
        arr = (ctypes.c_int * len(self.n))(*[int(c) for c in cycles])
        self._check(_lib.lib().nested_poisson_set_fixed_cycles(self._h, arr))

    def history(self, level):
        buf = (ctypes.c_double * 256)()
        m = _lib.lib().nested_poisson_history(self._h, level, buf, 256)
        self._check(m if m < 0 else 0)
        return [buf[i] for i in range(m)]

    def forces(self, level, out=None):
        d = self.dim
        shp = self._shape(level, 0)
        if out is None:
            out = [torch.empty(shp, dtype=torch.float64, device=self.device) for _ in range(d)]
        for a, t in enumerate(out):
            self._tensor(t, shp, "force[%d]" % a)
        fz = out[2].data_ptr() if d == 3 else None
        self._check(_lib.lib().nested_poisson_forces(self._h, level, ctypes.c_void_p(out[0].data_ptr()),
                                                     ctypes.c_void_p(out[1].data_ptr()), ctypes.c_void_p(fz)))
        return tuple(out)

    def potential(self, level, out=None):
        shp = self._shape(level, 2)
        if out is None:
            out = torch.empty(shp, dtype=torch.float64, device=self.device)
        self._tensor(out, shp, "phi")
        self._check(_lib.lib().nested_poisson_potential(self._h, level, ctypes.c_void_p(out.data_ptr())))
        return out

    def set_guess_weights(self, theta):
        """Network parameters: an FP32 vector of NP_NET_PARAMS values (packed into
        the library's versioned blob) or such a blob (bytes)."""
        blob = theta if isinstance(theta, (bytes, bytearray)) else _lib.pack_guess_weights(theta)
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        self._check(_lib.lib().nested_poisson_set_guess_weights(self._h, buf, len(blob)))

    def guess_features(self, level, with_target=True):
        """(x, target) of the learned guess for a level >= 1 after a solve:
        x is Gamma^l's shape x 2 channel-last, target Gamma^l's shape (FP32 device tensors)."""
        shp = self._shape(level, 1)
        x = torch.empty(shp + (2,), dtype=torch.float32, device=self.device)
        t = torch.empty(shp, dtype=torch.float32, device=self.device) if with_target else None
        self._check(_lib.lib().nested_poisson_guess_features(self._h, level, ctypes.c_void_p(x.data_ptr()),
                                                             ctypes.c_void_p(t.data_ptr() if t is not None else 0)))
        return x, t

    def set_profiling(self, enable=True):
        self._check(_lib.lib().nested_poisson_set_profiling(self._h, int(bool(enable))))

    def profile(self):
        """{class: (launches, device ms)} since profiling was enabled."""
        p = _lib.NpProfile()
        self._check(_lib.lib().nested_poisson_get_profile(self._h, ctypes.byref(p)))
        return {name: (p.count[i], p.ms[i]) for i, name in enumerate(_lib.KCLASSES)}

    def close(self):
        if self._h:
            _lib.lib().nested_poisson_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
