"""Thin Python binding over the libsgm C ABI (argument marshalling only).

Arrays are torch tensors on the current HIP device; every call is enqueued on
torch's current stream.  All arithmetic happens in the HIP kernels.
"""
import ctypes

import torch

from . import _lib
from ._lib import PlanDesc, check, load

BASES = {"dirichlet": _lib.SGM_SHEN_DIRICHLET, "biharmonic": _lib.SGM_SHEN_BIHARMONIC,
         "chebyshev": _lib.SGM_CHEBYSHEV}
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
        check(lib.sgm_plan_create(ctypes.byref(d), ctypes.byref(h)), "sgm_plan_create")
        self._h = h
        phys = (ctypes.c_int64 * 3)()
        spec = (ctypes.c_int64 * 3)()
        check(lib.sgm_plan_shapes(h, phys, spec), "sgm_plan_shapes")
        self.basis, self.kind_last, self.ndim = basis, kind_last, ndim
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

    def set_timing(self, enable=True):
        """Bracket every pass kernel of this plan with hipEvents (diagnostics)."""
        check(self._lib.sgm_plan_timing(self._h, int(bool(enable))), "sgm_plan_timing")

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

    def biharmonic_solve(self, f_tilde, out=None):
        _need(f_tilde, torch.complex128, self.spec_shape, "f_tilde")
        out = self._out(out, self.spec_shape, torch.complex128, f_tilde.device)
        _need(out, torch.complex128, self.spec_shape, "u_hat")
        check(self._lib.sgm_biharmonic_solve(self._h, _ptr(f_tilde), _ptr(out), _stream()), "sgm_biharmonic_solve")
        return out


class GLBatch:
    """Ragged batch of complex Ginzburg-Landau problems on [-L/2, L/2)^2.

    All arrays are packed complex128 device vectors of length `total`; problem i
    occupies [offsets[i], offsets[i+1]) as an N_i x N_i C-ordered array."""

    def __init__(self, sizes, L=100.0, b=0.0, c=1.5, dt=0.025, scheme="rk4", graph=True):
        lib = load()
        self._lib = lib
        self.sizes = [int(n) for n in sizes]
        arr = (ctypes.c_int * len(self.sizes))(*self.sizes)
        d = _lib.GLDesc(len(self.sizes), arr, float(L), float(b), float(c), float(dt),
                        _lib.SGM_IFRK4 if scheme == "ifrk4" else _lib.SGM_RK4, int(bool(graph)))
        h = ctypes.c_void_p()
        check(lib.sgm_gl_create(ctypes.byref(d), ctypes.byref(h)), "sgm_gl_create")
        self._h = h
        offs = (ctypes.c_int64 * (len(self.sizes) + 1))()
        check(lib.sgm_gl_offsets(h, offs), "sgm_gl_offsets")
        self.offsets = list(offs)
        self.total = self.offsets[-1]

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
