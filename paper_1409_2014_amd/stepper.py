"""Python face of the DS time stepper (include/phi_ds.h): split-step time
integration with one potential solve per step, its reverse pass, and
checkpointed backpropagation through many steps.

Every step runs in the library's HIP kernels; this module allocates fields and
stores and sequences the calls.  Gradients of a real loss with respect to a
complex field follow PyTorch's convention dJ/dRe(u) + i dJ/dIm(u), which is
also the library's.
"""
from __future__ import annotations

import ctypes

import torch

from . import _binding as B
from .solver import _info_dict, _stream_handle, make_params

__all__ = ["DSStepper", "DSEvolve", "ds_evolve"]

_COMPLEX = {torch.float64: torch.complex128, torch.float32: torch.complex64}


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


class DSStepper:
    """Split-step integrator of the DS system on an n x n periodic grid of
    spacing h (Sec. 2.3):

        DSStepper(n, h, alpha=1.0, beta=1.0, tau=1e-3, dtype=torch.float64,
                  scheme="strang" | "yoshida4", potential="split" | "periodic",
                  c_local=None, c_potential=None, n_r=64, n_theta=128, tol=None, ...)

    The nonlinear substep's phase is s (c_local |u|^2 + c_potential Phi), by
    default c_local = 2 beta and c_potential = 4 beta (eq. 1).

    The remaining keyword arguments configure the potential solve (as Plan).
    Fields are complex tensors (complex128 for float64, complex64 for float32)
    of shape (n, n), indexed [y][x]."""

    def __init__(self, n: int, h: float, *, alpha: float = 1.0, beta: float = 1.0, tau: float = 1e-3,
                 dtype=torch.float64, device=None, scheme: str = "strang", potential: str = "split",
                 c_local: float | None = None, c_potential: float | None = None, **solve_kwargs):
        if not torch.cuda.is_available():
            raise RuntimeError("the DS stepper needs a ROCm GPU (torch.cuda is not available)")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.dtype = dtype
        self.cdtype = _COMPLEX[dtype]
        self.n = int(n)
        self.h = float(h)
        self.alpha, self.beta, self.tau = float(alpha), float(beta), float(tau)
        self.scheme, self.potential = scheme, potential
        params = make_params(n, h, dtype=dtype, **solve_kwargs)
        self.c_local = 2.0 * self.beta if c_local is None else float(c_local)
        self.c_potential = 4.0 * self.beta if c_potential is None else float(c_potential)
        opts = B.PhiDsOptions(self.alpha, self.c_local, self.c_potential, self.tau, B.PHI_DS_SCHEMES[scheme],
                              B.PHI_DS_POTENTIALS[potential])
        self._handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            B.check(B.lib().phi_ds_create(ctypes.byref(params), ctypes.byref(opts),
                                          _stream_handle(self.device), ctypes.byref(self._handle)))
        k = ctypes.c_int32(0)
        B.check(B.lib().phi_ds_substeps(self._handle, ctypes.byref(k)))
        self.substeps = int(k.value)
        plan = ctypes.c_void_p()
        B.check(B.lib().phi_ds_plan(self._handle, ctypes.byref(plan)))
        info = B.PhiPlanInfo()
        B.check(B.lib().phi_plan_get_info(plan, ctypes.byref(info)))
        self.solve_info = _info_dict(info)

    def close(self) -> None:
        if getattr(self, "_handle", None) and self._handle.value:
            with torch.cuda.device(self.device):
                B.check(B.lib().phi_ds_destroy(self._handle))
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ----------------------------------------------------------------
    def _check_field(self, u: torch.Tensor, name: str) -> None:
        if (u.device != self.device or u.dtype != self.cdtype or tuple(u.shape) != (self.n, self.n)
                or not u.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {self.n}x{self.n} {self.cdtype} tensor on "
                             f"{self.device}, got {tuple(u.shape)} {u.dtype} on {u.device}")

    def new_store(self, steps: int):
        """(v_store, phi_store) for `steps` steps: the inputs and potentials of
        their steps * substeps nonlinear substeps, which the reverse pass reads."""
        k = steps * self.substeps
        v = torch.empty((k, self.n, self.n), dtype=self.cdtype, device=self.device)
        p = torch.empty((k, self.n, self.n), dtype=self.dtype, device=self.device)
        return v, p

    def _call(self, name, *args):
        with torch.cuda.device(self.device):
            B.check(getattr(B.lib(), name)(self._handle, *args, _stream_handle(self.device)))

    # -- entry points -------------------------------------------------------------
    def forward(self, u: torch.Tensor, steps: int, store=None) -> torch.Tensor:
        """Advances u in place by `steps` steps; fills `store` (from new_store)
        for a later reverse pass when given."""
        self._check_field(u, "u")
        v, p = (None, None) if store is None else store
        if store is not None and (v.shape[0] < steps * self.substeps or p.shape[0] < steps * self.substeps):
            raise ValueError("store holds fewer steps than requested")
        self._call("phi_ds_forward", _ptr(u), int(steps), _ptr(v), _ptr(p))
        return u

    def backward(self, g: torch.Tensor, steps: int, store) -> torch.Tensor:
        """In place: gradient after `steps` steps -> gradient before them, with
        the store a forward of the same steps filled."""
        self._check_field(g, "g")
        v, p = store
        if v.shape[0] < steps * self.substeps or p.shape[0] < steps * self.substeps:
            raise ValueError("store holds fewer steps than requested")
        self._call("phi_ds_backward", _ptr(g), int(steps), _ptr(v), _ptr(p))
        return g

    def moments(self, u: torch.Tensor) -> torch.Tensor:
        """Device tensor (h^2 sum |u|^2, h^2 sum |u|^4), float64."""
        self._check_field(u, "u")
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        self._call("phi_ds_moments", _ptr(u), _ptr(out))
        return out

    def loss_grad(self, u: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """4 h^2 |u|^2 u, the gradient of h^2 sum |u|^4."""
        self._check_field(u, "u")
        g = torch.empty_like(u) if out is None else out
        self._check_field(g, "out")
        self._call("phi_ds_loss_grad", _ptr(u), _ptr(g))
        return g

    def segments(self, steps: int, checkpoint_every: int):
        if checkpoint_every < 1:
            raise ValueError("checkpoint_every must be >= 1")
        lens = [checkpoint_every] * (steps // checkpoint_every)
        if steps % checkpoint_every:
            lens.append(steps % checkpoint_every)
        return lens

    def loss_and_grad(self, u0: torch.Tensor, steps: int, checkpoint_every: int = 50):
        """J = h^2 sum |u(T)|^4 after `steps` steps from u0, and dJ/du0 by the
        reverse pass with checkpoints: the states at segment starts are kept,
        each segment but the last is run again with its store before its
        reverse pass (the last keeps the store of the first run).

        Returns (J as a 0-d float64 device tensor, gradient, counts of forward,
        recomputed and transposed potential solves: substeps per step each)."""
        lens = self.segments(steps, checkpoint_every)
        store = self.new_store(max(lens)) if lens else None
        u = u0.clone()
        starts = []
        for k, m in enumerate(lens):
            starts.append(u.clone())
            self.forward(u, m, store if k == len(lens) - 1 else None)
        loss = self.moments(u)[1]
        g = self.loss_grad(u)
        recomputed = 0
        for k in range(len(lens) - 1, -1, -1):
            if k != len(lens) - 1:
                w = starts[k].clone()
                self.forward(w, lens[k], store)
                recomputed += lens[k]
            self.backward(g, lens[k], store)
        k = self.substeps
        counts = {"forward_solves": k * steps, "recomputed_solves": k * recomputed, "adjoint_solves": k * steps}
        return loss, g, counts


class DSEvolve(torch.autograd.Function):
    """u(T) = the stepper's `steps` steps from u0, differentiable in u0 with
    checkpointed recomputation (a checkpoint every `checkpoint_every` steps)."""

    @staticmethod
    def forward(ctx, u0: torch.Tensor, stepper: DSStepper, steps: int, checkpoint_every: int):
        lens = stepper.segments(steps, checkpoint_every)
        u = u0.detach().clone().contiguous()
        starts = []
        for m in lens:
            starts.append(u.clone())
            stepper.forward(u, m)
        ctx.stepper, ctx.lens, ctx.starts = stepper, lens, starts
        return u

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        stepper, lens = ctx.stepper, ctx.lens
        g = grad_u.detach().clone().contiguous()
        store = stepper.new_store(max(lens)) if lens else None
        for k in range(len(lens) - 1, -1, -1):
            w = ctx.starts[k].clone()
            stepper.forward(w, lens[k], store)
            stepper.backward(g, lens[k], store)
        ctx.starts = None
        return g, None, None, None


def ds_evolve(u0: torch.Tensor, stepper: DSStepper, steps: int, checkpoint_every: int = 50) -> torch.Tensor:
    return DSEvolve.apply(u0, stepper, int(steps), int(checkpoint_every))

