"""Thin Python binding over the libsgm C ABI (argument marshalling only).

Arrays are torch tensors on the current HIP device; every call is enqueued on
torch's current stream.  All arithmetic happens in the HIP kernels.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import PlanDesc, check, load

BASES = {"dirichlet": _lib.SGM_SHEN_DIRICHLET, "biharmonic": _lib.SGM_SHEN_BIHARMONIC,
         "chebyshev": _lib.SGM_CHEBYSHEV, "neumann": _lib.SGM_SHEN_NEUMANN,
         "legendre": _lib.SGM_LEGENDRE, "leg_dirichlet": _lib.SGM_LEG_DIRICHLET,
         "leg_neumann": _lib.SGM_LEG_NEUMANN, "leg_biharmonic": _lib.SGM_LEG_BIHARMONIC}
KINDS = {"r2c": _lib.SGM_R2C, "c2c": _lib.SGM_C2C}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous {dtype} of shape {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")


class Plan:
    """TensorProductSpace V(x) x V^p(y) [x V^p(z)] with x the Chebyshev/Shen axis."""

    def __init__(self, basis, N, M1, M2=None, kind_last="r2c", Ly=0.0, Lz=0.0, autotune=False, generic=False,
                 variant=None):
        lib = load()
        self._lib = lib
        ndim = 2 if M2 is None else 3
        d = PlanDesc(ndim, BASES[basis], int(N), int(M1), int(M2 or 1), KINDS[kind_last], float(Ly), float(Lz),
                     2 if generic else (16 + int(variant)) if variant is not None else int(bool(autotune)))
        h = ctypes.c_void_p()
        check(lib.sgm_plan_create(ctypes.byref(d), _stream(), ctypes.byref(h)), "sgm_plan_create")
        self._h = h
        phys = (ctypes.c_int64 * 3)()
        spec = (ctypes.c_int64 * 3)()
        check(lib.sgm_plan_shapes(h, phys, spec), "sgm_plan_shapes")
        self.basis, self.kind_last, self.ndim = basis, kind_last, ndim
        self.Ly, self.Lz = float(Ly), float(Lz)
        self.phys_shape = tuple(phys[:ndim])
        self.spec_shape = tuple(spec[:ndim])
        self.phys_dtype = torch.float64 if kind_last == "r2c" else torch.complex128

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sgm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, enable=True, passes=None):
        """Bracket pass kernels of this plan with hipEvents (diagnostics): all of
        them, or only the named passes (see PASS_NAMES)."""
        if enable and passes is not None:
            bits = 0
            for name in passes:
                bits |= 1 << _lib.PASS_NAMES.index(name)
            flag = _lib.SGM_TIMING_ONLY | bits
        else:
            flag = int(bool(enable))
        check(self._lib.sgm_plan_timing(self._h, flag), "sgm_plan_timing")

    def points(self):
        """The N points of the x axis (numpy array)."""
        x = (ctypes.c_double * self.phys_shape[0])()
        check(self._lib.sgm_plan_points(self._h, x), "sgm_plan_points")
        return np.array(x[:], dtype=np.float64)

    def variants(self):
        """Register-kernel variant per axis (x, y, z); -1 = generic kernels."""
        v = (ctypes.c_int * 3)()
        check(self._lib.sgm_plan_variants(self._h, v), "sgm_plan_variants")
        return list(v)

    def solve_layout(self):
        """(lanes per chain, rows per lane) of the segmented solves; (0, 0) if none."""
        k, r = ctypes.c_int(), ctypes.c_int()
        check(self._lib.sgm_plan_solve_layout(self._h, ctypes.byref(k), ctypes.byref(r)), "sgm_plan_solve_layout")
        return k.value, r.value

    def set_solve_rows(self, rows):
        check(self._lib.sgm_plan_set_solve_rows(self._h, int(rows)), "sgm_plan_set_solve_rows")

    def pass_times(self, reset=False):
        """{pass name: (total ms, launches)} accumulated since the last reset."""
        ms = (ctypes.c_double * _lib.NPASS)()
        cnt = (ctypes.c_int64 * _lib.NPASS)()
        check(self._lib.sgm_plan_pass_times(self._h, ms, cnt, int(bool(reset))), "sgm_plan_pass_times")
        return {n: (ms[i], cnt[i]) for i, n in enumerate(_lib.PASS_NAMES) if cnt[i]}

    def _out(self, out, shape, dtype, dev):
        return torch.empty(shape, dtype=dtype, device=dev) if out is None else out

    def forward(self, u, out=None):
        _need(u, self.phys_dtype, self.phys_shape, "u")
        out = self._out(out, self.spec_shape, torch.complex128, u.device)
        _need(out, torch.complex128, self.spec_shape, "u_hat")
        check(self._lib.sgm_forward(self._h, _ptr(u), _ptr(out), _stream()), "sgm_forward")
        return out

    def backward(self, uh, out=None):
        _need(uh, torch.complex128, self.spec_shape, "u_hat")
        out = self._out(out, self.phys_shape, self.phys_dtype, uh.device)
        _need(out, self.phys_dtype, self.phys_shape, "u")
        check(self._lib.sgm_backward(self._h, _ptr(uh), _ptr(out), _stream()), "sgm_backward")
        return out

    def backward_noalloc(self, uh, out=None):
        """backward() through the allocation-free entry point (static workspace)."""
        _need(uh, torch.complex128, self.spec_shape, "u_hat")
        out = self._out(out, self.phys_shape, self.phys_dtype, uh.device)
        _need(out, self.phys_dtype, self.phys_shape, "u")
        check(self._lib.sgm_backward_noalloc(self._h, _ptr(uh), _ptr(out), _stream()), "sgm_backward_noalloc")
        return out

    def project_derivative(self, uh, order, target=None, out=None):
        """Coefficients in `target`'s space (a Plan on the same grid with the
        "chebyshev", "dirichlet" or "neumann" basis, or for a Legendre-family plan
        "legendre", "leg_dirichlet" or "leg_neumann"; default: the regular space of
        this plan's family, made here) of the projection of d^(ox+oy+oz) u / dx^ox dy^oy dz^oz, where u has
        the coefficients uh in this plan's space.  order = (ox, oy[, oz])."""
        _need(uh, torch.complex128, self.spec_shape, "u_hat")
        if target is None:
            target = self._cheb_target()
        out = self._out(out, self.spec_shape, torch.complex128, uh.device)
        _need(out, torch.complex128, self.spec_shape, "du_hat")
        o = list(order) + [0] * (3 - len(order))
        arr = (ctypes.c_int * 3)(*[int(v) for v in o])
        check(self._lib.sgm_project_derivative(self._h, target._h, arr, _ptr(uh), _ptr(out), _stream()),
              "sgm_project_derivative")
        return out

    def _cheb_target(self):
        if getattr(self, "_cheb", None) is None:
            M2 = self.phys_shape[2] if self.ndim == 3 else None
            regular = "legendre" if self.basis.startswith("leg") else "chebyshev"
            self._cheb = Plan(regular, self.phys_shape[0], self.phys_shape[1], M2, kind_last=self.kind_last,
                              Ly=self.Ly, Lz=self.Lz)
        return self._cheb

    def scalar_product(self, f, out=None):
        _need(f, self.phys_dtype, self.phys_shape, "f")
        out = self._out(out, self.spec_shape, torch.complex128, f.device)
        _need(out, torch.complex128, self.spec_shape, "f_tilde")
        check(self._lib.sgm_scalar_product(self._h, _ptr(f), _ptr(out), _stream()), "sgm_scalar_product")
        return out

    def helmholtz_solve(self, f_tilde, alpha=0.0, out=None):
        _need(f_tilde, torch.complex128, self.spec_shape, "f_tilde")
        out = self._out(out, self.spec_shape, torch.complex128, f_tilde.device)
        _need(out, torch.complex128, self.spec_shape, "u_hat")
        check(self._lib.sgm_helmholtz_solve(self._h, float(alpha), _ptr(f_tilde), _ptr(out), _stream()),
              "sgm_helmholtz_solve")
        return out

    def helmholtz_solve_physical(self, f, alpha=0.0, out=None):
        """alpha u - lap u = f from the physical right-hand side (scalar product
        and solve; one fused pass where the plan allows)."""
        _need(f, self.phys_dtype, self.phys_shape, "f")
        out = self._out(out, self.spec_shape, torch.complex128, f.device)
        _need(out, torch.complex128, self.spec_shape, "u_hat")
        check(self._lib.sgm_helmholtz_solve_physical(self._h, float(alpha), _ptr(f), _ptr(out), _stream()),
              "sgm_helmholtz_solve_physical")
        return out

    def biharmonic_solve(self, f_tilde, out=None):
        _need(f_tilde, torch.complex128, self.spec_shape, "f_tilde")
        out = self._out(out, self.spec_shape, torch.complex128, f_tilde.device)
        _need(out, torch.complex128, self.spec_shape, "u_hat")
        check(self._lib.sgm_biharmonic_solve(self._h, _ptr(f_tilde), _ptr(out), _stream()), "sgm_biharmonic_solve")
        return out


class GLBatch:
    """Ragged batch of complex Ginzburg-Landau problems on [-L/2, L/2)^2.

    All arrays are packed complex128 device vectors of length `total`; problem i
    occupies [offsets[i], offsets[i+1]) as an N_i x N_i C-ordered array.

    tune: False (default launch configuration), True (time every candidate at
    creation, keep the fastest) or an int 0 <= k < 6 pinning candidate k
    (2 * FFT tiling + grid mode)."""

    def __init__(self, sizes, L=100.0, b=0.0, c=1.5, dt=0.025, scheme="rk4", graph=True, tune=False):
        lib = load()
        self._lib = lib
        self.sizes = [int(n) for n in sizes]
        arr = (ctypes.c_int * len(self.sizes))(*self.sizes)
        d = _lib.GLDesc(len(self.sizes), arr, float(L), float(b), float(c), float(dt),
                        _lib.SGM_IFRK4 if scheme == "ifrk4" else _lib.SGM_RK4, int(bool(graph)),
                        1 if tune is True else 0 if tune is False else 16 + int(tune))
        h = ctypes.c_void_p()
        check(lib.sgm_gl_create(ctypes.byref(d), _stream(), ctypes.byref(h)), "sgm_gl_create")
        self._h = h
        offs = (ctypes.c_int64 * (len(self.sizes) + 1))()
        check(lib.sgm_gl_offsets(h, offs), "sgm_gl_offsets")
        self.offsets = list(offs)
        self.total = self.offsets[-1]

    @property
    def variant(self):
        """Launch configuration in use: 2 * FFT tiling + grid mode."""
        v = ctypes.c_int()
        check(self._lib.sgm_gl_variant(self._h, ctypes.byref(v)), "sgm_gl_variant")
        return v.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sgm_gl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, arrays, device="cuda"):
        """Concatenate N_i x N_i arrays (numpy or torch) into one packed device vector."""
        parts = [torch.as_tensor(a, dtype=torch.complex128).reshape(-1) for a in arrays]
        return torch.cat(parts).to(device).contiguous()

    def unpack(self, packed):
        """Split a packed vector into a list of N_i x N_i tensors (views)."""
        return [packed[self.offsets[i]:self.offsets[i + 1]].view(n, n) for i, n in enumerate(self.sizes)]

    def _vec(self, t, name):
        _need(t, torch.complex128, (self.total,), name)

    def forward(self, u, out=None):
        self._vec(u, "u")
        out = torch.empty_like(u) if out is None else out
        self._vec(out, "u_hat")
        check(self._lib.sgm_gl_forward(self._h, _ptr(u), _ptr(out), _stream()), "sgm_gl_forward")
        return out

    def backward(self, uh, out=None):
        self._vec(uh, "u_hat")
        out = torch.empty_like(uh) if out is None else out
        self._vec(out, "u")
        check(self._lib.sgm_gl_backward(self._h, _ptr(uh), _ptr(out), _stream()), "sgm_gl_backward")
        return out

    def rhs(self, uh, out=None):
        self._vec(uh, "u_hat")
        out = torch.empty_like(uh) if out is None else out
        self._vec(out, "rhs")
        check(self._lib.sgm_gl_rhs(self._h, _ptr(uh), _ptr(out), _stream()), "sgm_gl_rhs")
        return out

    def step(self, uh, nsteps=1):
        """Advance the packed state in place by nsteps time steps."""
        self._vec(uh, "u_hat")
        check(self._lib.sgm_gl_step(self._h, _ptr(uh), int(nsteps), _stream()), "sgm_gl_step")
        return uh


class FNO:
    """FNO-style surrogate u(t) -> u(t + s dt) with hand-written training and inference kernels.

    Inputs and outputs are fp32 device tensors [B, H, W, 2] (Re, Im channels)."""

    def __init__(self, H, W, width=32, modes=16, layers=4, hidden=128, max_batch=16, seed=0):
        lib = load()
        self._lib = lib
        d = _lib.FNODesc(int(H), int(W), int(width), int(modes), int(layers), int(hidden), int(max_batch))
        h = ctypes.c_void_p()
        check(lib.sgm_fno_create(ctypes.byref(d), ctypes.c_uint64(seed), ctypes.byref(h)), "sgm_fno_create")
        self._h = h
        n = ctypes.c_int64()
        check(lib.sgm_fno_num_params(h, ctypes.byref(n)), "sgm_fno_num_params")
        self.num_params = n.value
        self.H, self.W, self.C, self.K, self.nl, self.P, self.max_batch = H, W, width, modes, layers, hidden, max_batch
        self.ensemble = 1

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sgm_fno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # flat parameter vector <-> dict in the documented order
    def param_shapes(self):
        C, K, P = self.C, self.K, self.P
        sh = [("Wl", (2, C)), ("bl", (C,))]
        for l in range(self.nl):
            sh += [(f"Rr{l}", (2 * K, K, C, C)), (f"Ri{l}", (2 * K, K, C, C)), (f"Wp{l}", (C, C)), (f"bp{l}", (C,))]
        sh += [("W1", (C, P)), ("b1", (P,)), ("W2", (P, 2)), ("b2", (2,))]
        return sh

    def flatten(self, params):
        return np.concatenate([np.asarray(params[k], dtype=np.float32).reshape(-1) for k, _ in self.param_shapes()])

    def unflatten(self, flat):
        out, o = {}, 0
        for k, shp in self.param_shapes():
            n = int(np.prod(shp))
            out[k] = np.asarray(flat[o:o + n]).reshape(shp)
            o += n
        return out

    def set_params(self, params):
        flat = np.ascontiguousarray(self.flatten(params) if isinstance(params, dict) else params, dtype=np.float32)
        assert flat.size == self.num_params
        check(self._lib.sgm_fno_set_params(self._h, flat.ctypes.data_as(ctypes.c_void_p)), "sgm_fno_set_params")

    def get_params(self):
        flat = np.empty(self.num_params, dtype=np.float32)
        check(self._lib.sgm_fno_get_params(self._h, flat.ctypes.data_as(ctypes.c_void_p)), "sgm_fno_get_params")
        return self.unflatten(flat)

    def _x(self, x, name):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
                and x.dim() == 4 and tuple(x.shape[1:]) == (self.H, self.W, 2)):
            raise ValueError(f"{name}: expected contiguous float32 device tensor [B, {self.H}, {self.W}, 2]")
        if not 1 <= x.shape[0] <= self.max_batch:
            raise ValueError(f"{name}: batch must be in 1..{self.max_batch}")

    def set_ensemble(self, members):
        """Average inference over 1, 2, 4 or 8 reflections of the periodic grid
        (sgm_fno_set_ensemble); applies to infer() and advance_checked()."""
        check(self._lib.sgm_fno_set_ensemble(self._h, int(members)), "sgm_fno_set_ensemble")
        self.ensemble = int(members)

    def infer(self, x, out=None):
        self._x(x, "x")
        out = torch.empty_like(x) if out is None else out
        check(self._lib.sgm_fno_infer(self._h, _ptr(x), _ptr(out), x.shape[0], _stream()), "sgm_fno_infer")
        return out

    def grads(self, x, target):
        self._x(x, "x")
        self._x(target, "target")
        g = np.empty(self.num_params, dtype=np.float32)
        loss = ctypes.c_float()
        check(self._lib.sgm_fno_grads(self._h, _ptr(x), _ptr(target), x.shape[0], g.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(loss), _stream()), "sgm_fno_grads")
        return self.unflatten(g), loss.value

    def train_step(self, x, target, lr, want_loss=True):
        self._x(x, "x")
        self._x(target, "target")
        loss = ctypes.c_float()
        check(self._lib.sgm_fno_train_step(self._h, _ptr(x), _ptr(target), x.shape[0], float(lr),
                                           ctypes.byref(loss) if want_loss else None, _stream()), "sgm_fno_train_step")
        return loss.value if want_loss else None

    def rel_l2(self, pred, target):
        self._x(pred, "pred")
        self._x(target, "target")
        out = torch.empty(pred.shape[0], dtype=torch.float32, device=pred.device)
        check(self._lib.sgm_fno_rel_l2(self._h, _ptr(pred), _ptr(target), pred.shape[0], _ptr(out), _stream()),
              "sgm_fno_rel_l2")
        return out

    def advance_checked(self, gl, gl_check, u_hat, nsur, steps_per, tol=1e-2, seed=0, max_fail_frac=0.0):
        """Advance the packed GL state u_hat by nsur surrogate macro-steps with the FP64
        check/fallback on gl_check.count samples per macro-step (the whole batch is
        re-advanced by the FP64 solver when more than max_fail_frac of the checks
        fail); returns the stats dict."""
        gl._vec(u_hat, "u_hat")
        st = _lib.FNOStats(0, 0, 0.0, 0.0, 0, 0)
        check(self._lib.sgm_fno_advance_checked(self._h, gl._h, gl_check._h, _ptr(u_hat), int(nsur), int(steps_per),
                                                float(tol), float(max_fail_frac), ctypes.c_uint64(seed),
                                                ctypes.byref(st), _stream()),
              "sgm_fno_advance_checked")
        return {"n_checked": st.n_checked, "n_fallback": st.n_fallback, "max_rel_l2": st.max_rel_l2,
                "mean_rel_l2": st.mean_rel_l2, "n_batch_fallback": st.n_batch_fallback,
                "n_replaced": st.n_replaced}

    def save(self, path):
        check(self._lib.sgm_fno_save(self._h, str(path).encode()), "sgm_fno_save")

    def load(self, path):
        check(self._lib.sgm_fno_load(self._h, str(path).encode()), "sgm_fno_load")


def pack_states(u_c128, out=None):
    """complex128 device tensor (..., H, W) -> fp32 (..., H, W, 2) with the library kernel."""
    lib = load()
    if out is None:
        out = torch.empty(tuple(u_c128.shape) + (2,), dtype=torch.float32, device=u_c128.device)
    check(lib.sgm_fno_pack(_ptr(u_c128), _ptr(out), u_c128.numel(), _stream()), "sgm_fno_pack")
    return out


def unpack_states(x, out=None):
    lib = load()
    if out is None:
        out = torch.empty(tuple(x.shape[:-1]), dtype=torch.complex128, device=x.device)
    check(lib.sgm_fno_unpack(_ptr(x), _ptr(out), out.numel(), _stream()), "sgm_fno_unpack")
    return out


def autotune_forget():
    """Clear the library's in-process memory of autotuned choices (the cache file stays)."""
    check(load().sgm_autotune_forget(), "sgm_autotune_forget")


def autotune_cache_path():
    """Path of the autotuner's cache file ("" if none)."""
    buf = ctypes.create_string_buffer(4096)
    check(load().sgm_autotune_cache_path(buf, 4096), "sgm_autotune_cache_path")
    return buf.value.decode()
