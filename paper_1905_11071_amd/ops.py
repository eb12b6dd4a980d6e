"""PyTorch binding of the Step-LISTA library: argument marshalling only.

Every computation runs in libslista's HIP kernels; torch provides device
memory (the tensors and the workspace) and the current stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import torch

from ._lib import SlistaError, check, lib  # noqa: F401

PRECISIONS = {"fp32": 0, "bf16": 1}


def bf16_fp32_tail(tail: int) -> int:
    """Precision schedule: BF16 contractions, then FP32 in the last `tail`
    layers (SLISTA_BF16_FP32_TAIL)."""
    if tail < 0:
        raise ValueError("tail must be >= 0")
    return PRECISIONS["bf16"] | (int(tail) << 8)


def _prec(prec) -> int:
    if isinstance(prec, int):
        return prec
    try:
        return PRECISIONS[prec]
    except KeyError:
        raise ValueError(f"precision must be one of {list(PRECISIONS)}") from None


def _stream(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dev_f32(t: torch.Tensor, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.contiguous()


class Dictionary:
    """Per-dictionary device state: G = D^T D (FP32 and BF16) and D^T."""

    def __init__(self, D: torch.Tensor):
        D = _dev_f32(D, "D")
        if D.dim() != 2:
            raise ValueError("D must be [n, m]")
        self.device = D.device
        self.n, self.m = int(D.shape[0]), int(D.shape[1])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().slista_dict_create(D.data_ptr(), self.n, self.m, _stream(self.device), ctypes.byref(h)))
        self._h = h
        mp = ctypes.c_int()
        check(lib().slista_dict_dims(self._h, None, None, ctypes.byref(mp)))
        self.m_pad = mp.value

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def gram(self) -> torch.Tensor:
        G = torch.empty(self.m, self.m, device=self.device, dtype=torch.float32)
        check(lib().slista_dict_gram(self._h, G.data_ptr(), _stream(self.device)))
        return G

    def lipschitz(self, max_iter: int = 100_000, rtol: float = 1e-13) -> Tuple[float, int]:
        """(L, iterations): FP64 power iteration on G. Raises if rtol is not met."""
        L = ctypes.c_double()
        it = ctypes.c_int()
        with torch.cuda.device(self.device):
            check(lib().slista_dict_lipschitz(self._h, max_iter, rtol, ctypes.byref(L), ctypes.byref(it),
                                              _stream(self.device)))
        return L.value, it.value

    def workspace_bytes(self, N: int, T: int, prec="fp32", ckpt_every: int = 0) -> int:
        b = ctypes.c_size_t()
        check(lib().slista_workspace_size(self._h, N, T, _prec(prec), ckpt_every, ctypes.byref(b)))
        return b.value

    def workspace(self, N: int, T: int, prec="fp32", ckpt_every: int = 0) -> torch.Tensor:
        nbytes = self.workspace_bytes(N, T, prec, ckpt_every)
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)

    def ckpt_for_budget(self, N: int, T: int, prec="fp32", budget: Optional[int] = None) -> int:
        """The smallest checkpoint spacing whose workspace fits `budget` bytes
        (default: 90 % of the device's free memory)."""
        if budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget = int(0.9 * free)
        k = ctypes.c_int()
        check(lib().slista_ckpt_for_budget(self._h, N, T, _prec(prec), int(budget), ctypes.byref(k), None))
        return k.value

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().slista_dict_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_inputs(d: Dictionary, X: torch.Tensor, alpha: torch.Tensor):
    X = _dev_f32(X, "X")
    if X.dim() != 2 or X.shape[1] != d.n:
        raise ValueError(f"X must be [N, {d.n}]")
    alpha = _dev_f32(alpha, "alpha")
    if alpha.dim() != 1:
        raise ValueError("alpha must be [T]")
    return X, alpha


def forward(d: Dictionary, X: torch.Tensor, lam: float, alpha: torch.Tensor, prec="fp32",
            f_trace: bool = False, want_f: bool = True, want_loss: bool = True, ckpt_every: int = 0,
            ws: Optional[torch.Tensor] = None):
    """z^(T) for every sample, plus F (per sample, or the [T+1, N] trace) and
    the mean loss. Returns (Z, F or None, loss or None, ws)."""
    X, alpha = _check_inputs(d, X, alpha)
    N, T = int(X.shape[0]), int(alpha.shape[0])
    p = _prec(prec)
    if ws is None:
        ws = d.workspace(N, T, p, ckpt_every)
    Z = torch.empty(N, d.m, device=d.device, dtype=torch.float32)
    F = None
    if want_f:
        F = torch.empty((T + 1, N) if f_trace else (N,), device=d.device, dtype=torch.float32)
    loss = torch.empty(1, device=d.device, dtype=torch.float32) if want_loss else None
    check(lib().slista_forward(d.handle, X.data_ptr(), N, float(lam), alpha.data_ptr(), T, p, Z.data_ptr(),
                               _ptr(F), int(bool(f_trace)), _ptr(loss), ckpt_every, ws.data_ptr(), ws.numel(),
                               _stream(d.device)))
    return Z, F, loss, ws


def objective(d: Dictionary, X: torch.Tensor, lam: float, Z: torch.Tensor) -> torch.Tensor:
    """F_i = 1/2 ||x_i - D z_i||^2 + lam ||z_i||_1 for given codes (FP32 residual,
    FP64 sums), independent of the precision that produced Z."""
    X = _dev_f32(X, "X")
    Z = _dev_f32(Z, "Z", (X.shape[0], d.m))
    F = torch.empty(X.shape[0], device=d.device, dtype=torch.float32)
    check(lib().slista_objective(d.handle, X.data_ptr(), int(X.shape[0]), float(lam), Z.data_ptr(), F.data_ptr(),
                                 _stream(d.device)))
    return F


def forward_f64(d: Dictionary, X: torch.Tensor, lam: float, alpha: torch.Tensor, f_trace: bool = False,
                want_loss: bool = True):
    """T layers in double precision (slista_forward_f64): X [N, n] and alpha
    [T] float64 device tensors. Returns (Z [N, m], F ([T+1, N] with f_trace,
    else [N]), loss (0-d tensor or None)), all float64."""
    for t, name in ((X, "X"), (alpha, "alpha")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
            raise ValueError(f"{name} must be a float64 CUDA (HIP) tensor")
    X, alpha = X.contiguous(), alpha.contiguous()
    if X.dim() != 2 or X.shape[1] != d.n:
        raise ValueError(f"X has shape {tuple(X.shape)}, expected (N, {d.n})")
    N, T = int(X.shape[0]), int(alpha.numel())
    Z = torch.empty(N, d.m, device=d.device, dtype=torch.float64)
    F = torch.empty((T + 1, N) if f_trace else (N,), device=d.device, dtype=torch.float64)
    loss = torch.empty((), device=d.device, dtype=torch.float64) if want_loss else None
    check(lib().slista_forward_f64(d.handle, X.data_ptr(), N, float(lam), alpha.data_ptr(), T, Z.data_ptr(),
                                   F.data_ptr(), int(f_trace), loss.data_ptr() if loss is not None else None,
                                   None, 0, _stream(d.device)))
    return Z, F, loss


def kkt(d: Dictionary, X: torch.Tensor, lam: float, Z: torch.Tensor):
    """(kkt, F): per sample, in FP64 on the device, the largest violation of
    the Lasso optimality conditions (Lemma 2.1) by the codes Z, and F(z)."""
    X = _dev_f32(X, "X")
    Z = _dev_f32(Z, "Z", (X.shape[0], d.m))
    N = int(X.shape[0])
    k = torch.empty(N, device=d.device, dtype=torch.float64)
    F = torch.empty(N, device=d.device, dtype=torch.float64)
    check(lib().slista_kkt(d.handle, X.data_ptr(), N, float(lam), Z.data_ptr(), k.data_ptr(), F.data_ptr(),
                           _stream(d.device)))
    return k, F


def lambda_max(d: Dictionary, X: torch.Tensor):
    """(max_i ||D^T x_i||_inf as a Python float, the per-sample values [N])
    from the forward pass's own correlation product."""
    X = _dev_f32(X, "X")
    N = int(X.shape[0])
    nbytes = ctypes.c_size_t()
    check(lib().slista_lambda_max_workspace_size(d.handle, N, ctypes.byref(nbytes)))
    ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=d.device)
    out = torch.empty(1, device=d.device, dtype=torch.float32)
    rows = torch.empty(max(N, 1), device=d.device, dtype=torch.float32)
    check(lib().slista_lambda_max(d.handle, X.data_ptr(), N, out.data_ptr(), rows.data_ptr(), ws.data_ptr(),
                                  ws.numel(), _stream(d.device)))
    return float(out.item()), rows[:N]


def backward(d: Dictionary, X: torch.Tensor, lam: float, alpha: torch.Tensor, ws: torch.Tensor,
             dZ: Optional[torch.Tensor] = None, dF: Optional[torch.Tensor] = None, prec="fp32",
             ckpt_every: int = 1) -> torch.Tensor:
    """d J / d alpha for J = sum dF_i F_i(z^T) + <dZ, Z^T>, from the tape a
    forward() call with the same arguments left in ws."""
    X, alpha = _check_inputs(d, X, alpha)
    N, T = int(X.shape[0]), int(alpha.shape[0])
    if dZ is not None:
        dZ = _dev_f32(dZ, "dZ", (N, d.m))
    if dF is not None:
        dF = _dev_f32(dF, "dF", (N,))
    dalpha = torch.empty(T, device=d.device, dtype=torch.float32)
    check(lib().slista_backward(d.handle, X.data_ptr(), N, float(lam), alpha.data_ptr(), T, _prec(prec),
                                _ptr(dZ), _ptr(dF), dalpha.data_ptr(), ckpt_every, ws.data_ptr(), ws.numel(),
                                _stream(d.device)))
    return dalpha


def forward_backward(d: Dictionary, X: torch.Tensor, lam: float, alpha: torch.Tensor, prec="fp32",
                     ckpt_every: int = 1, ws: Optional[torch.Tensor] = None, want_f: bool = True):
    """Forward plus d(mean F)/d alpha in one call. Returns (Z, F, loss, dalpha, ws)."""
    X, alpha = _check_inputs(d, X, alpha)
    N, T = int(X.shape[0]), int(alpha.shape[0])
    p = _prec(prec)
    if ws is None:
        ws = d.workspace(N, T, p, ckpt_every)
    Z = torch.empty(N, d.m, device=d.device, dtype=torch.float32)
    F = torch.empty(N, device=d.device, dtype=torch.float32) if want_f else None
    loss = torch.empty(1, device=d.device, dtype=torch.float32)
    dalpha = torch.empty(T, device=d.device, dtype=torch.float32)
    check(lib().slista_forward_backward(d.handle, X.data_ptr(), N, float(lam), alpha.data_ptr(), T, p,
                                        Z.data_ptr(), _ptr(F), loss.data_ptr(), dalpha.data_ptr(), ckpt_every,
                                        ws.data_ptr(), ws.numel(), _stream(d.device)))
    return Z, F, loss, dalpha, ws


def autotune(d: Dictionary, X: torch.Tensor, lam: float, alpha: torch.Tensor, prec="fp32", ckpt_every: int = 1):
    """Time every tile variant of the persistent kernels on this problem and
    make the fastest the default for its (precision, m, N) class. Returns
    (best variant, [ms per call of variants 1..4; 0 where a variant does not apply])."""
    X, alpha = _check_inputs(d, X, alpha)
    N, T = int(X.shape[0]), int(alpha.shape[0])
    p = _prec(prec)
    ws = d.workspace(N, T, p, ckpt_every)
    Z = torch.empty(N, d.m, device=d.device, dtype=torch.float32)
    da = torch.empty(T, device=d.device, dtype=torch.float32)
    best = ctypes.c_int()
    ms = (ctypes.c_double * 4)()
    check(lib().slista_autotune(d.handle, X.data_ptr(), N, float(lam), alpha.data_ptr(), T, p, ckpt_every,
                                Z.data_ptr(), da.data_ptr(), ws.data_ptr(), ws.numel(), _stream(d.device),
                                ctypes.byref(best), ms))
    return best.value, list(ms)


def fista(d: Dictionary, X: torch.Tensor, lam: float, alpha: torch.Tensor, prec="fp32"):
    """T layers of FISTA (forward only). Returns (Z, F of z^T, mean loss)."""
    X, alpha = _check_inputs(d, X, alpha)
    N, T = int(X.shape[0]), int(alpha.shape[0])
    p = _prec(prec)
    nbytes = ctypes.c_size_t()
    check(lib().slista_fista_workspace_size(d.handle, N, T, p, ctypes.byref(nbytes)))
    ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=d.device)
    Z = torch.empty(N, d.m, device=d.device, dtype=torch.float32)
    F = torch.empty(N, device=d.device, dtype=torch.float32)
    loss = torch.empty(1, device=d.device, dtype=torch.float32)
    check(lib().slista_fista(d.handle, X.data_ptr(), N, float(lam), alpha.data_ptr(), T, p, Z.data_ptr(),
                             F.data_ptr(), loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream(d.device)))
    return Z, F, loss


def oista(d: Dictionary, X: torch.Tensor, lam: float, L: float, T: int, prec="fp32", max_power_iter: int = 5000,
          power_rtol: float = 1e-12):
    """T layers of Oracle-ISTA. Returns (Z, F of z^T, mean loss, steps [T, N])."""
    X = _dev_f32(X, "X")
    if X.dim() != 2 or X.shape[1] != d.n:
        raise ValueError(f"X must be [N, {d.n}]")
    N = int(X.shape[0])
    p = _prec(prec)
    nbytes = ctypes.c_size_t()
    check(lib().slista_oista_workspace_size(d.handle, N, T, p, ctypes.byref(nbytes)))
    ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=d.device)
    Z = torch.empty(N, d.m, device=d.device, dtype=torch.float32)
    F = torch.empty(N, device=d.device, dtype=torch.float32)
    loss = torch.empty(1, device=d.device, dtype=torch.float32)
    steps = torch.empty(max(T, 1), N, device=d.device, dtype=torch.float32)
    check(lib().slista_oista(d.handle, X.data_ptr(), N, float(lam), float(L), int(T), p, int(max_power_iter),
                             float(power_rtol), Z.data_ptr(), F.data_ptr(), loss.data_ptr(), steps.data_ptr(),
                             ws.data_ptr(), ws.numel(), _stream(d.device)))
    return Z, F, loss, steps[:T]


def train(d: Dictionary, X: torch.Tensor, lam: float, alpha: torch.Tensor, iters: int, lr: float,
          prec="fp32", max_halvings: int = 30):
    """Learn the step sizes in place (alpha, a device float32 [T] tensor) by
    full-batch sub-gradient descent with a backtracking learning rate on the
    mean loss. Returns (losses [accepted + 1] as a list, final learning rate)."""
    target = alpha
    X, alpha = _check_inputs(d, X, alpha)
    N, T = int(X.shape[0]), int(alpha.shape[0])
    p = _prec(prec)
    nbytes = ctypes.c_size_t()
    check(lib().slista_train_workspace_size(d.handle, N, T, p, ctypes.byref(nbytes)))
    ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=d.device)
    Z = torch.empty(N, d.m, device=d.device, dtype=torch.float32)
    losses = (ctypes.c_double * (iters + 1))()
    acc = ctypes.c_int()
    lr_out = ctypes.c_double()
    check(lib().slista_train(d.handle, X.data_ptr(), N, float(lam), alpha.data_ptr(), T, p, int(iters), float(lr),
                             int(max_halvings), Z.data_ptr(), losses, ctypes.byref(acc), ctypes.byref(lr_out),
                             ws.data_ptr(), ws.numel(), _stream(d.device)))
    if alpha.data_ptr() != target.data_ptr():
        target.copy_(alpha)
    return [losses[i] for i in range(acc.value + 1)], lr_out.value


def tune_save(path: str) -> None:
    check(lib().slista_tune_save(path.encode()))


def tune_load(path: str) -> None:
    check(lib().slista_tune_load(path.encode()))


class Batch:
    """Forward + backward of many independent Lasso problems (own dictionary,
    n, m, N, lambda and steps; common T) in grouped persistent launches, with
    an optional captured HIP graph.

    problems: list of (Dictionary, X [N, n], lam, alpha [T]). Outputs per
    problem after run()/replay(): Z[i], F[i], loss[i], dalpha[i]."""

    def __init__(self, problems, prec="fp32", ckpt_every: int = 1):
        from ._lib import Problem
        if not problems:
            raise ValueError("empty batch")
        T = int(problems[0][3].shape[0])
        self.device = problems[0][0].device
        self._keep = []
        self.Z, self.F, self.loss, self.dalpha = [], [], [], []
        arr = (Problem * len(problems))()
        for i, (d, X, lam, alpha) in enumerate(problems):
            X, alpha = _check_inputs(d, X, alpha)
            if int(alpha.shape[0]) != T:
                raise ValueError("all problems of a batch share T")
            N = int(X.shape[0])
            Z = torch.empty(N, d.m, device=d.device, dtype=torch.float32)
            F = torch.empty(N, device=d.device, dtype=torch.float32)
            loss = torch.empty(1, device=d.device, dtype=torch.float32)
            da = torch.empty(T, device=d.device, dtype=torch.float32)
            self._keep += [d, X, alpha]
            self.Z.append(Z)
            self.F.append(F)
            self.loss.append(loss)
            self.dalpha.append(da)
            arr[i] = Problem(d.handle.value, X.data_ptr(), N, float(lam), alpha.data_ptr(), Z.data_ptr(),
                             F.data_ptr(), loss.data_ptr(), da.data_ptr())
        h = ctypes.c_void_p()
        check(lib().slista_batch_create(ctypes.cast(arr, ctypes.c_void_p), len(problems), T, _prec(prec),
                                        ckpt_every, ctypes.byref(h)))
        self._h = h
        nbytes = ctypes.c_size_t()
        check(lib().slista_batch_workspace_size(self._h, ctypes.byref(nbytes)))
        self.ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            check(lib().slista_batch_bind(self._h, self.ws.data_ptr(), self.ws.numel(), _stream(self.device)))

    def run(self) -> None:
        check(lib().slista_batch_run(self._h, _stream(self.device)))

    def capture(self) -> None:
        """Record run() into a HIP graph (on a side stream, as capture requires)."""
        s = torch.cuda.Stream(self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        check(lib().slista_batch_capture(self._h, ctypes.c_void_p(s.cuda_stream)))
        torch.cuda.current_stream(self.device).wait_stream(s)

    def replay(self) -> None:
        check(lib().slista_batch_replay(self._h, _stream(self.device)))

    def autotune(self) -> dict:
        """Pick each bucket's tile variant by timing whole-batch runs; returns
        {column passes: variant}. Drops a captured graph."""
        v = (ctypes.c_int * 4)()
        check(lib().slista_batch_autotune(self._h, _stream(self.device), v))
        return {np_: v[i] for i, np_ in enumerate((1, 2, 4, 8)) if v[i]}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().slista_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedCall:
    """The one-call batch entry point (slista_batched_fwd_bwd): the library
    plans the batch on the first call (and captures a HIP graph if asked) and
    replays it on later calls. Same inputs and outputs as Batch."""

    def __init__(self, problems, prec="fp32", ckpt_every: int = 1):
        from ._lib import Problem
        if not problems:
            raise ValueError("empty batch")
        self.T = int(problems[0][3].shape[0])
        self.device = problems[0][0].device
        self.prec, self.ckpt = _prec(prec), int(ckpt_every)
        self._keep = []
        self.Z, self.F, self.loss, self.dalpha = [], [], [], []
        self._arr = (Problem * len(problems))()
        for i, (d, X, lam, alpha) in enumerate(problems):
            X, alpha = _check_inputs(d, X, alpha)
            N = int(X.shape[0])
            out = (torch.empty(N, d.m, device=d.device, dtype=torch.float32),
                   torch.empty(N, device=d.device, dtype=torch.float32),
                   torch.empty(1, device=d.device, dtype=torch.float32),
                   torch.empty(self.T, device=d.device, dtype=torch.float32))
            self._keep += [d, X, alpha]
            for lst, t in zip((self.Z, self.F, self.loss, self.dalpha), out):
                lst.append(t)
            self._arr[i] = Problem(d.handle.value, X.data_ptr(), N, float(lam), alpha.data_ptr(),
                                   out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(), out[3].data_ptr())
        nbytes = ctypes.c_size_t()
        check(lib().slista_batched_workspace_size(ctypes.cast(self._arr, ctypes.c_void_p), len(problems), self.T,
                                                  self.prec, self.ckpt, ctypes.byref(nbytes)))
        self.ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)

    def __call__(self, use_graph: bool = True) -> None:
        check(lib().slista_batched_fwd_bwd(ctypes.cast(self._arr, ctypes.c_void_p), len(self._arr), self.T,
                                           self.prec, self.ckpt, self.ws.data_ptr(), self.ws.numel(),
                                           _stream(self.device), int(bool(use_graph))))


def batched_release() -> None:
    """Drop every plan slista_batched_fwd_bwd keeps (synchronises the device)."""
    check(lib().slista_batched_release())


KERNEL_FAMILIES = {"auto": 0, "layer": 1, "persistent": 2}


def set_check_finite(on: bool) -> None:
    """Count NaN / Inf in the inputs and outputs of the dictionary, forward
    and backward calls (synchronising); raise SLISTA_ENONFINITE if any."""
    check(lib().slista_set_option(3, int(bool(on))))


def set_kernel_family(name: str) -> None:
    """Select the layer kernels: 'auto', 'layer' (one launch per layer) or
    'persistent' (one workgroup per sample tile through all layers)."""
    check(lib().slista_set_option(1, KERNEL_FAMILIES[name]))


def set_tile_variant(v: int) -> None:
    """Tile configuration of the persistent kernels (0 = library default, 1..4)."""
    check(lib().slista_set_option(2, int(v)))


def profile_begin() -> None:
    """Start recording HIP-event timings of every library launch."""
    check(lib().slista_profile_begin())


def profile_end() -> dict:
    """Stop recording; {kernel class: (launches, total milliseconds)}."""
    from ._lib import PROFILE_KINDS
    n = len(PROFILE_KINDS)
    launches = (ctypes.c_int * n)()
    total = (ctypes.c_double * n)()
    dropped = ctypes.c_int()
    check(lib().slista_profile_end(launches, total, ctypes.byref(dropped)))
    out = {k: (launches[i], total[i]) for i, k in enumerate(PROFILE_KINDS)}
    out["dropped"] = (dropped.value, 0.0)
    return out


class SlistaFunction(torch.autograd.Function):
    """Step-LISTA as an autograd node: alpha -> (z^(T), F(z^(T))).

    Only the step sizes are learned (Section 4, Step-LISTA); the backward
    runs the library's hand-written adjoint kernels over the tape the
    forward kept in its workspace."""

    @staticmethod
    def forward(ctx, alpha, d: Dictionary, X, lam, prec="fp32", ckpt_every=1):
        if ckpt_every == "auto":  # keep every layer if it fits, else checkpoint
            ckpt_every = d.ckpt_for_budget(int(X.shape[0]), int(alpha.shape[0]), prec)
        Z, F, _, ws = forward(d, X, lam, alpha, prec=prec, want_loss=False, ckpt_every=ckpt_every)
        ctx.save_for_backward(alpha, X)
        ctx.d, ctx.lam, ctx.prec, ctx.ckpt, ctx.ws = d, lam, prec, ckpt_every, ws
        return Z, F

    @staticmethod
    def backward(ctx, gZ, gF):
        alpha, X = ctx.saved_tensors
        dalpha = backward(ctx.d, X, ctx.lam, alpha, ctx.ws, dZ=None if gZ is None else gZ.contiguous(),
                          dF=None if gF is None else gF.contiguous(), prec=ctx.prec, ckpt_every=ctx.ckpt)
        return dalpha, None, None, None, None, None


def slista(alpha: torch.Tensor, d: Dictionary, X: torch.Tensor, lam: float, prec="fp32", ckpt_every=1):
    """Differentiable Step-LISTA network: returns (Z, F) with gradients to alpha.
    ckpt_every: checkpoint spacing of the tape (1 = keep every layer), or
    "auto" for the smallest spacing whose workspace fits the free memory."""
    return SlistaFunction.apply(alpha, d, X, lam, prec, ckpt_every)


# --------------------------------------------------------------- coupled LISTA

def _check_lista(d: Dictionary, W: torch.Tensor, alpha: torch.Tensor, beta: torch.Tensor):
    alpha = _dev_f32(alpha, "alpha")
    if alpha.dim() != 1:
        raise ValueError("alpha must be [T]")
    T = int(alpha.shape[0])
    beta = _dev_f32(beta, "beta", (T,))
    W = _dev_f32(W, "W", (T, d.n, d.m))
    return W, alpha, beta


def lista_workspace(d: Dictionary, N: int, T: int, prec="fp32", tape: bool = False) -> torch.Tensor:
    nbytes = ctypes.c_size_t()
    check(lib().slista_lista_workspace_size(d.handle, int(N), int(T), _prec(prec), int(bool(tape)),
                                            ctypes.byref(nbytes)))
    return torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=d.device)


def lista_forward(d: Dictionary, X: torch.Tensor, lam: float, W: torch.Tensor, alpha: torch.Tensor,
                  beta: torch.Tensor, prec="fp32", tape: bool = False, ws: Optional[torch.Tensor] = None):
    """T coupled LISTA layers (per-layer W_t [n, m], alpha_t, beta_t; W is
    [T, n, m]). Returns (Z, F of z^T, mean loss, ws); with tape the workspace
    keeps what lista_backward reads."""
    X = _dev_f32(X, "X")
    if X.dim() != 2 or X.shape[1] != d.n:
        raise ValueError(f"X must be [N, {d.n}]")
    W, alpha, beta = _check_lista(d, W, alpha, beta)
    N, T = int(X.shape[0]), int(alpha.shape[0])
    p = _prec(prec)
    if ws is None:
        ws = lista_workspace(d, N, T, p, tape)
    Z = torch.empty(N, d.m, device=d.device, dtype=torch.float32)
    F = torch.empty(N, device=d.device, dtype=torch.float32)
    loss = torch.empty(1, device=d.device, dtype=torch.float32)
    check(lib().slista_lista_forward(d.handle, X.data_ptr(), N, float(lam), W.data_ptr(), alpha.data_ptr(),
                                     beta.data_ptr(), T, p, Z.data_ptr(), F.data_ptr(), loss.data_ptr(),
                                     int(bool(tape)), ws.data_ptr(), ws.numel(), _stream(d.device)))
    return Z, F, loss, ws


def lista_backward(d: Dictionary, N: int, lam: float, alpha: torch.Tensor, beta: torch.Tensor, ws: torch.Tensor,
                   dZ: Optional[torch.Tensor] = None, dF: Optional[torch.Tensor] = None, prec="fp32",
                   want_dW: bool = True):
    """(dW [T, n, m] or None, dalpha [T], dbeta [T]) of J = sum dF_i F_i(z^T) +
    <dZ, Z^T>, from the tape of a lista_forward(tape=True) call in ws."""
    alpha = _dev_f32(alpha, "alpha")
    T = int(alpha.shape[0])
    beta = _dev_f32(beta, "beta", (T,))
    if dZ is not None:
        dZ = _dev_f32(dZ, "dZ", (N, d.m))
    if dF is not None:
        dF = _dev_f32(dF, "dF", (N,))
    dW = torch.empty(T, d.n, d.m, device=d.device, dtype=torch.float32) if want_dW else None
    dalpha = torch.empty(T, device=d.device, dtype=torch.float32)
    dbeta = torch.empty(T, device=d.device, dtype=torch.float32)
    check(lib().slista_lista_backward(d.handle, int(N), float(lam), alpha.data_ptr(), beta.data_ptr(), T,
                                      _prec(prec), _ptr(dZ), _ptr(dF), _ptr(dW), dalpha.data_ptr(),
                                      dbeta.data_ptr(), ws.data_ptr(), ws.numel(), _stream(d.device)))
    return dW, dalpha, dbeta


def lista_forward_backward(d: Dictionary, X: torch.Tensor, lam: float, W: torch.Tensor, alpha: torch.Tensor,
                           beta: torch.Tensor, prec="fp32", want_dW: bool = True, ws: Optional[torch.Tensor] = None):
    """Forward plus the gradient of the mean loss (Eq. (15)) in every layer's
    parameters. Returns (Z, F, loss, dW or None, dalpha, dbeta, ws)."""
    X = _dev_f32(X, "X")
    if X.dim() != 2 or X.shape[1] != d.n:
        raise ValueError(f"X must be [N, {d.n}]")
    W, alpha, beta = _check_lista(d, W, alpha, beta)
    N, T = int(X.shape[0]), int(alpha.shape[0])
    p = _prec(prec)
    if ws is None:
        ws = lista_workspace(d, N, T, p, True)
    Z = torch.empty(N, d.m, device=d.device, dtype=torch.float32)
    F = torch.empty(N, device=d.device, dtype=torch.float32)
    loss = torch.empty(1, device=d.device, dtype=torch.float32)
    dW = torch.empty(T, d.n, d.m, device=d.device, dtype=torch.float32) if want_dW else None
    dalpha = torch.empty(T, device=d.device, dtype=torch.float32)
    dbeta = torch.empty(T, device=d.device, dtype=torch.float32)
    check(lib().slista_lista_forward_backward(d.handle, X.data_ptr(), N, float(lam), W.data_ptr(), alpha.data_ptr(),
                                              beta.data_ptr(), T, p, Z.data_ptr(), F.data_ptr(), loss.data_ptr(),
                                              _ptr(dW), dalpha.data_ptr(), dbeta.data_ptr(), ws.data_ptr(),
                                              ws.numel(), _stream(d.device)))
    return Z, F, loss, dW, dalpha, dbeta, ws


class ListaFunction(torch.autograd.Function):
    """Coupled LISTA as an autograd node: (W, alpha, beta) -> (z^(T), F(z^(T))),
    differentiated by the library's hand-written adjoint over the tape the
    forward kept in its workspace."""

    @staticmethod
    def forward(ctx, W, alpha, beta, d: Dictionary, X, lam, prec="fp32"):
        Z, F, _, ws = lista_forward(d, X, lam, W, alpha, beta, prec=prec, tape=True)
        ctx.save_for_backward(alpha, beta)
        ctx.d, ctx.lam, ctx.prec, ctx.ws, ctx.N = d, lam, prec, ws, int(X.shape[0])
        return Z, F

    @staticmethod
    def backward(ctx, gZ, gF):
        alpha, beta = ctx.saved_tensors
        if gZ is None and gF is None:
            return None, None, None, None, None, None, None
        dW, dalpha, dbeta = lista_backward(ctx.d, ctx.N, ctx.lam, alpha, beta, ctx.ws,
                                           dZ=None if gZ is None else gZ.contiguous(),
                                           dF=None if gF is None else gF.contiguous(), prec=ctx.prec,
                                           want_dW=ctx.needs_input_grad[0])
        return dW, dalpha, dbeta, None, None, None, None


def lista(W: torch.Tensor, alpha: torch.Tensor, beta: torch.Tensor, d: Dictionary, X: torch.Tensor, lam: float,
          prec="fp32"):
    """Differentiable coupled LISTA network: returns (Z, F) with gradients to
    W [T, n, m], alpha [T] and beta [T]."""
    return ListaFunction.apply(W, alpha, beta, d, X, lam, prec)
