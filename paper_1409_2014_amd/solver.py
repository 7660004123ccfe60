"""Python face of the C ABI: plans, solves and the autograd wrapper.

PyTorch only provides device memory and the current stream; every step of a
solve runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _binding as B

__all__ = ["Plan", "BatchPlan", "PhiSolve", "phi_solve", "describe", "host_gauss_legendre",
           "host_es_kernel", "host_es_transform", "host_polar_nodes", "make_params"]

_DTYPES = {torch.float64: B.PHI_F64, torch.float32: B.PHI_F32}


def _dtype_code(dtype) -> int:
    if isinstance(dtype, str):
        dtype = {"float64": torch.float64, "f64": torch.float64, "float32": torch.float32,
                 "f32": torch.float32}[dtype]
    if dtype not in _DTYPES:
        raise ValueError(f"unsupported dtype {dtype}")
    return _DTYPES[dtype]


def make_params(n: int, h: float, *, dtype=torch.float64, n_r: int = 64, n_theta: int = 128,
                tol: float | None = None, sigma: float | None = None, cutoff: float | None = None,
                component: str = "x", pad: int = 2, bin: int = 0, sub_nodes: int = 0,
                autotune: bool = False, radial: str = "legendre", kernel: str = "es",
                two_streams: bool = False, partition: str | None = None) -> B.PhiParams:
    code = _dtype_code(dtype)
    p = B.PhiParams()
    B.check(B.lib().phi_params_default(ctypes.byref(p), int(n), float(h), code))
    p.n_r = int(n_r)
    p.n_theta = int(n_theta)
    if tol is not None:
        p.tol = float(tol)
    p.pad = int(pad)
    p.sigma = float(sigma) if sigma else 0.0
    p.cutoff = float(cutoff) if cutoff else 0.0
    comp_flags = {"x": 0, "xx": 0, "y": B.PHI_COMPONENT_Y, "yy": B.PHI_COMPONENT_Y, "xy": B.PHI_COMPONENT_XY,
                  "coulomb": B.PHI_COMPONENT_COULOMB}
    if component not in comp_flags:
        raise ValueError(f"component must be one of {sorted(comp_flags)}, got {component!r}")
    if radial not in ("legendre", "jacobi"):
        raise ValueError(f"radial must be 'legendre' or 'jacobi', got {radial!r}")
    if kernel not in ("es", "gaussian"):
        raise ValueError(f"kernel must be 'es' or 'gaussian', got {kernel!r}")
    if partition not in (None, "erfc", "gauss"):
        raise ValueError(f"partition must be 'erfc' or 'gauss', got {partition!r}")
    if partition == "erfc" and component != "coulomb":
        raise ValueError("the erfc partition is for the Coulomb multiplier only")
    p.flags = (comp_flags[component] | (B.PHI_AUTOTUNE if autotune else 0)
               | (B.PHI_PARTITION_GAUSS if partition == "gauss" and component == "coulomb" else 0)
               | (B.PHI_RADIAL_JACOBI if radial == "jacobi" else 0)
               | (B.PHI_KERNEL_GAUSSIAN if kernel == "gaussian" else 0)
               | (B.PHI_TWO_STREAMS if two_streams else 0))
    p.bin = int(bin)
    p.sub_nodes = int(sub_nodes)
    return p


def _info_dict(info: B.PhiPlanInfo) -> dict:
    return {name: getattr(info, name) for name, _ in B.PhiPlanInfo._fields_}


def describe(**kwargs) -> dict:
    """Derived plan quantities for make_params(**kwargs), computed on the host."""
    p = make_params(**kwargs)
    info = B.PhiPlanInfo()
    B.check(B.lib().phi_describe(ctypes.byref(p), ctypes.byref(info)))
    return _info_dict(info)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def host_gauss_legendre(n: int):
    x = np.empty(n)
    w = np.empty(n)
    B.check(B.lib().phi_host_gauss_legendre(int(n), _dptr(x), _dptr(w)))
    return x, w


def host_gauss_jacobi01(n: int):
    x = np.empty(n)
    w = np.empty(n)
    B.check(B.lib().phi_host_gauss_jacobi01(int(n), _dptr(x), _dptr(w)))
    return x, w


def host_es_kernel(z, beta: float):
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty_like(z)
    B.check(B.lib().phi_host_es_kernel(z.size, _dptr(z), float(beta), _dptr(out)))
    return out


def host_es_transform(omega, beta: float):
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.empty_like(omega)
    B.check(B.lib().phi_host_es_transform(omega.size, _dptr(omega), float(beta), _dptr(out)))
    return out


def host_polar_nodes(**kwargs):
    p = make_params(**kwargs)
    m = p.n_r * p.n_theta
    kx, ky, q = np.empty(m), np.empty(m), np.empty(m)
    B.check(B.lib().phi_host_polar_nodes(ctypes.byref(p), _dptr(kx), _dptr(ky), _dptr(q)))
    return kx, ky, q


def _stream_handle(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_disjoint(src: torch.Tensor, dst: torch.Tensor) -> None:
    """The library reads its input while other kernels of the same call write
    the output, so the two must not share memory."""
    s0, d0 = src.data_ptr(), dst.data_ptr()
    if s0 < d0 + dst.numel() * dst.element_size() and d0 < s0 + src.numel() * src.element_size():
        raise ValueError("input and output must not overlap")


class Plan:
    """A solve plan on one GPU (tables + workspace live on the device).

    Plan(n, h, dtype=torch.float32|float64, n_r=64, n_theta=128, tol=None,
         sigma=None, cutoff=None, component="x", bin=0, sub_nodes=0, autotune=False)

    component selects the multiplier: "x" -kx^2/|k|^2 (the DS potential), "y"
    -ky^2/|k|^2, "xy" -kx ky/|k|^2, "coulomb" 1/|k| (the 2-D Coulomb potential;
    partition "erfc" (default) or "gauss", the paper's e^{-|k|^2/sigma^2},
    which leaves a cone in the I1 integrand); radial "legendre" or "jacobi" the radial
    rule; kernel "es" or "gaussian" (Greengard-Lee gridding) the NUFFT kernel.  bin / sub_nodes set the node sort (0: 4
    cells, 64 nodes); autotune=True times the candidates on the device at plan
    time (as eager solves) and keeps the fastest; under graph replay the
    default has measured as fast or faster."""

    def __init__(self, n: int, h: float, *, dtype=torch.float64, device=None, **kwargs):
        if not torch.cuda.is_available():
            raise RuntimeError("phisolve needs a ROCm GPU (torch.cuda is not available)")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.dtype = dtype if not isinstance(dtype, str) else {
            "float64": torch.float64, "float32": torch.float32}[dtype]
        self.n = int(n)
        self.h = float(h)
        self.params = make_params(n, h, dtype=self.dtype, **kwargs)
        self._handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            B.check(B.lib().phi_plan(ctypes.byref(self.params), _stream_handle(self.device),
                                     ctypes.byref(self._handle)))
        info = B.PhiPlanInfo()
        B.check(B.lib().phi_plan_get_info(self._handle, ctypes.byref(info)), self._handle)
        self.info = _info_dict(info)

    # -- lifetime -------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_handle", None) and self._handle.value:
            with torch.cuda.device(self.device):
                B.check(B.lib().phi_destroy(self._handle))
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers --------------------------------------------------------------
    def _check_grid(self, t: torch.Tensor, name: str, output: bool = False) -> torch.Tensor:
        if t.device != self.device or t.dtype != self.dtype or tuple(t.shape) != (self.n, self.n):
            raise ValueError(f"{name} must be a {self.n}x{self.n} {self.dtype} tensor on {self.device}, "
                             f"got {tuple(t.shape)} {t.dtype} on {t.device}")
        if output:
            # written in place: a contiguous copy would leave the caller's tensor untouched
            if not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous")
            return t
        return t.contiguous()

    def _call(self, fn, src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
        _check_disjoint(src, dst)
        with torch.cuda.device(self.device):
            B.check(fn(self._handle, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                       _stream_handle(self.device)), self._handle)
        return dst

    def _grid_out(self, out):
        if out is None:
            return torch.empty((self.n, self.n), dtype=self.dtype, device=self.device)
        return self._check_grid(out, "out", output=True)

    # -- entry points ---------------------------------------------------------
    def solve(self, rho: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Phi = I1 + I2 for the density rho (N x N, on the plan's device)."""
        return self._call(B.lib().phi_solve, self._check_grid(rho, "rho"), self._grid_out(out))

    def solve_adjoint(self, g_phi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        return self._call(B.lib().phi_solve_adjoint, self._check_grid(g_phi, "g_phi"), self._grid_out(out))

    def highfreq(self, rho: torch.Tensor, out=None) -> torch.Tensor:
        return self._call(B.lib().phi_solve_highfreq, self._check_grid(rho, "rho"), self._grid_out(out))

    def lowfreq(self, rho: torch.Tensor, out=None) -> torch.Tensor:
        return self._call(B.lib().phi_solve_lowfreq, self._check_grid(rho, "rho"), self._grid_out(out))

    def periodic(self, rho: torch.Tensor, out=None) -> torch.Tensor:
        """The standard periodic FFT solver on the same grid (the paper's baseline)."""
        return self._call(B.lib().phi_solve_periodic, self._check_grid(rho, "rho"), self._grid_out(out))

    def type2(self, rho: torch.Tensor) -> torch.Tensor:
        """rho_hat at the plan's polar nodes (complex, plan order)."""
        m = self.info["n_nodes"]
        out = torch.empty((m, 2), dtype=self.dtype, device=self.device)
        self._call(B.lib().phi_nodes_type2, self._check_grid(rho, "rho"), out)
        return torch.view_as_complex(out)

    def type1(self, coef: torch.Tensor, out=None) -> torch.Tensor:
        """Re sum_j coef_j e^{+2 pi i k_j.x_n} on the grid (coef complex, plan order)."""
        m = self.info["n_nodes"]
        cdt = torch.complex128 if self.dtype == torch.float64 else torch.complex64
        if coef.device != self.device or coef.dtype != cdt or tuple(coef.shape) != (m,):
            raise ValueError(f"coef must be a ({m},) {cdt} tensor on {self.device}")
        src = torch.view_as_real(coef.contiguous())
        return self._call(B.lib().phi_nodes_type1, src, self._grid_out(out))

    def solve_timed(self, src: torch.Tensor, out: torch.Tensor, adjoint: bool = False):
        """Run one solve (or transposed solve) with HIP events around every
        kernel on the current stream; returns [(kernel name, ms), ...].
        Blocks until the solve has finished (measurement only)."""
        cap = 16
        ms = (ctypes.c_float * cap)()
        names = (ctypes.c_char_p * cap)()
        count = ctypes.c_int32(0)
        src = self._check_grid(src, "input")
        out = self._check_grid(out, "out", output=True)
        _check_disjoint(src, out)
        with torch.cuda.device(self.device):
            B.check(B.lib().phi_solve_timed(self._handle, ctypes.c_void_p(src.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), int(bool(adjoint)),
                                            _stream_handle(self.device), ms, names, cap,
                                            ctypes.byref(count)), self._handle)
        return [(names[i].decode(), float(ms[i])) for i in range(min(count.value, cap))]

    def nodes(self):
        """(kx, ky, q) of the plan's polar nodes as float64 numpy arrays, plan order."""
        m = self.info["n_nodes"]
        kx, ky, q = np.empty(m), np.empty(m), np.empty(m)
        B.check(B.lib().phi_plan_nodes(self._handle, _dptr(kx), _dptr(ky), _dptr(q)), self._handle)
        return kx, ky, q


class BatchPlan:
    """Independent solves of several densities, possibly of different sizes, as
    one chain of launches (one per stage over all members).

    BatchPlan(members, dtype=torch.float32) where members is a list of dicts of
    make_params keyword arguments (n, h, n_r, n_theta, tol, ...).  Inputs and
    outputs are packed 1-D tensors: member i occupies
    [offsets[i], offsets[i+1]) as an n_i x n_i row-major grid."""

    def __init__(self, members, *, dtype=torch.float32, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("phisolve needs a ROCm GPU (torch.cuda is not available)")
        if len(members) == 0:
            raise ValueError("a batch needs at least one member")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.dtype = dtype
        self.sizes = [int(m["n"]) for m in members]
        arr = (B.PhiParams * len(members))()
        for i, m in enumerate(members):
            kw = dict(m)
            kw["dtype"] = dtype
            arr[i] = make_params(**kw)
        self._handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            B.check(B.lib().phi_plan_batch(arr, len(members), _stream_handle(self.device),
                                           ctypes.byref(self._handle)))
        count = ctypes.c_int32(0)
        offs = (ctypes.c_int64 * (len(members) + 1))()
        B.check(B.lib().phi_batch_layout(self._handle, ctypes.byref(count), offs), self._handle)
        self.offsets = [int(offs[i]) for i in range(count.value + 1)]
        self.total = self.offsets[-1]
        info = B.PhiPlanInfo()
        B.check(B.lib().phi_plan_get_info(self._handle, ctypes.byref(info)), self._handle)
        self.device_bytes = int(info.device_bytes)

    def close(self) -> None:
        if getattr(self, "_handle", None) and self._handle.value:
            with torch.cuda.device(self.device):
                B.check(B.lib().phi_destroy(self._handle))
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def member_info(self, i: int) -> dict:
        """Derived plan quantities of member i (bin / sub_nodes as chosen, ...)."""
        info = B.PhiPlanInfo()
        B.check(B.lib().phi_batch_member_info(self._handle, int(i), ctypes.byref(info)), self._handle)
        return _info_dict(info)

    def pack(self, grids) -> torch.Tensor:
        """One packed device tensor from a list of n_i x n_i tensors or arrays."""
        out = torch.empty(self.total, dtype=self.dtype, device=self.device)
        for i, g in enumerate(grids):
            t = torch.as_tensor(g, dtype=self.dtype, device=self.device)
            out[self.offsets[i]:self.offsets[i + 1]].copy_(t.reshape(-1))
        return out

    def unpack(self, packed: torch.Tensor):
        """Views of the members' n_i x n_i grids in a packed tensor."""
        return [packed[self.offsets[i]:self.offsets[i + 1]].view(n, n) for i, n in enumerate(self.sizes)]

    def _check_packed(self, t: torch.Tensor, name: str, output: bool = False) -> torch.Tensor:
        if t.device != self.device or t.dtype != self.dtype or t.numel() != self.total:
            raise ValueError(f"{name} must be a packed {self.dtype} tensor of {self.total} elements on "
                             f"{self.device}, got {tuple(t.shape)} {t.dtype} on {t.device}")
        if output:
            if not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous")
            return t
        return t.contiguous()

    def _call(self, fn, src, out):
        src = self._check_packed(src, "input")
        out = (torch.empty(self.total, dtype=self.dtype, device=self.device) if out is None
               else self._check_packed(out, "out", output=True))
        _check_disjoint(src, out)
        with torch.cuda.device(self.device):
            B.check(fn(self._handle, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                       _stream_handle(self.device)), self._handle)
        return out

    def solve(self, rho: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        return self._call(B.lib().phi_solve, rho, out)

    def solve_adjoint(self, g_phi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        return self._call(B.lib().phi_solve_adjoint, g_phi, out)

    def solve_timed(self, src: torch.Tensor, out: torch.Tensor, adjoint: bool = False):
        cap = 16
        ms = (ctypes.c_float * cap)()
        names = (ctypes.c_char_p * cap)()
        count = ctypes.c_int32(0)
        src = self._check_packed(src, "input")
        out = self._check_packed(out, "out", output=True)
        _check_disjoint(src, out)
        with torch.cuda.device(self.device):
            B.check(B.lib().phi_solve_timed(self._handle, ctypes.c_void_p(src.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), int(bool(adjoint)),
                                            _stream_handle(self.device), ms, names, cap,
                                            ctypes.byref(count)), self._handle)
        return [(names[i].decode(), float(ms[i])) for i in range(min(count.value, cap))]


class PhiSolve(torch.autograd.Function):
    """Phi = A rho with the hand-written transposed solve as its backward."""

    @staticmethod
    def forward(ctx, rho: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.solve(rho.detach())

    @staticmethod
    def backward(ctx, grad_phi: torch.Tensor):
        return ctx.plan.solve_adjoint(grad_phi.contiguous()), None


def phi_solve(rho: torch.Tensor, plan: Plan) -> torch.Tensor:
    return PhiSolve.apply(rho, plan)
