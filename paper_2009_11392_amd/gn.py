"""Python binding of libgn: the C entry points with the same names, taking torch
tensors for device memory and torch's current HIP stream.  Argument marshalling
only: every step of the computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import dataclasses
from dataclasses import dataclass

import torch

from . import _capi as C
from ._capi import GNError  # noqa: F401  (re-export)

MODES = {"f64": C.GN_MODE_F64, "f32": C.GN_MODE_F32, "bf16": C.GN_MODE_BF16_BS,
         "f16": C.GN_MODE_F16_BS}
KINDS = {"gaussian": C.GN_SKETCH_GAUSSIAN, "srht": C.GN_SKETCH_SRHT, "user": C.GN_SKETCH_USER}
CORE_METHODS = {"qr": C.GN_CORE_QR, "svd": C.GN_CORE_SVD, "lift_svd": C.GN_CORE_LIFT_SVD,
                "lift_rrqr": C.GN_CORE_LIFT_RRQR, "lift_diag": C.GN_CORE_LIFT_DIAG}
SKETCH_TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
                "f16": torch.float16}
ACCUM_TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32,
               "f16": torch.float32}
DT_OF_TORCH = {torch.float64: C.GN_DT_F64, torch.float32: C.GN_DT_F32, torch.bfloat16: C.GN_DT_BF16,
               torch.float16: C.GN_DT_F16}


@dataclass
class Problem:
    """The problem statement of Algorithm 2.1: shape of A, r, l, eps, sketch kinds,
    seed, and the pass precision."""
    m: int
    n: int
    r: int
    l: int = -1              # < 0: ceil(r/2)
    kind_x: str = "gaussian"
    kind_y: str = "gaussian"
    seed: int = 0
    mode: str = "f64"
    eps: float = 0.0         # absolute; <= 0: plain GN
    nu_x: float = 0.0
    nu_y: float = 0.0
    core_method: str = "qr"  # Section 5.1.1: qr, svd, lift_svd, lift_rrqr, lift_diag

    @property
    def l_eff(self) -> int:
        return (self.r + 1) // 2 if self.l < 0 else self.l

    @property
    def rl(self) -> int:
        return self.r + self.l_eff

    def c(self) -> C.GnProblem:
        return C.GnProblem(self.m, self.n, self.r, self.l, KINDS[self.kind_x], KINDS[self.kind_y],
                           self.seed & ((1 << 64) - 1), MODES[self.mode],
                           CORE_METHODS[self.core_method], self.eps, self.nu_x, self.nu_y)


def _ptr(t):
    return ctypes.c_void_p(0) if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libgn takes device tensors")


def gn_workspace_size(p: Problem, op: int, kcols: int = 0) -> int:
    out = ctypes.c_size_t(0)
    pc = p.c()
    C.check(C.lib().gn_workspace_size(ctypes.byref(pc), op, kcols, ctypes.byref(out)),
            "gn_workspace_size")
    return int(out.value)


def workspace(p: Problem, op: int, kcols: int = 0, device="cuda") -> torch.Tensor:
    return torch.empty(max(gn_workspace_size(p, op, kcols), 256), dtype=torch.uint8, device=device)


def gn_generate_gaussian(seed: int, stream: int, rows: int, cols: int, dtype=torch.float64,
                         layout: int = 0, row0: int = 0, col0: int = 0, out=None):
    shape = (rows, cols) if layout == 0 else (cols, rows)
    if out is None:
        out = torch.empty(shape, dtype=dtype, device="cuda")
    _need_cuda(out)
    C.check(C.lib().gn_generate_gaussian(seed & ((1 << 64) - 1), stream, row0, col0, rows, cols,
                                         DT_OF_TORCH[out.dtype], layout, _ptr(out), out.stride(0),
                                         _stream()), "gn_generate_gaussian")
    return out


def gn_srht_generate(seed: int, n: int, r: int):
    npad = 1 << max(0, (n - 1).bit_length())
    signs = torch.empty(npad, dtype=torch.int8, device="cuda")
    idx = torch.empty(r, dtype=torch.int32, device="cuda")
    # the workspace depends on n' only; any valid problem with this n sizes it
    ws = workspace(Problem(n, n, max(1, min(r, n)), kind_x="srht"), C.GN_OP_SRHT)
    C.check(C.lib().gn_srht_generate(seed & ((1 << 64) - 1), n, r, _ptr(signs), _ptr(idx), _ptr(ws),
                                     ws.numel(), _stream()), "gn_srht_generate")
    return signs, idx


def gn_sketch_prepare(p: Problem, ws: torch.Tensor, X_user=None, Y_user=None,
                      want_srht: bool = False):
    """Draw (or take) the sketches into the workspace ws; returns SRHT signs/idx
    copies when asked."""
    _need_cuda(ws, X_user, Y_user)
    signs = idx = None
    if want_srht and p.kind_x == "srht":
        npad = 1 << max(0, (p.n - 1).bit_length())
        signs = torch.empty(npad, dtype=torch.int8, device=ws.device)
        idx = torch.empty(p.r, dtype=torch.int32, device=ws.device)
    pc = p.c()
    C.check(C.lib().gn_sketch_prepare(
        ctypes.byref(pc), _ptr(X_user), X_user.stride(0) if X_user is not None else 0,
        _ptr(Y_user), Y_user.stride(0) if Y_user is not None else 0, _ptr(signs), _ptr(idx),
        _ptr(ws), ws.numel(), _stream()), "gn_sketch_prepare")
    return signs, idx


def gn_sketch_pass(p: Problem, A: torch.Tensor, ws: torch.Tensor, scales=None, AX=None, YtA=None):
    """The single pass over A: AX and Y^T A from the sketches in a prepared ws."""
    _need_cuda(A, ws, scales)
    acc = ACCUM_TORCH[p.mode]
    AX = torch.empty(p.m, p.r, dtype=acc, device=A.device) if AX is None else AX
    YtA = torch.empty(p.rl, p.n, dtype=acc, device=A.device) if YtA is None else YtA
    pc = p.c()
    C.check(C.lib().gn_sketch_pass(ctypes.byref(pc), _ptr(A), A.stride(0), _ptr(scales), _ptr(AX),
                                   AX.stride(0), _ptr(YtA), YtA.stride(0), _ptr(ws), ws.numel(),
                                   _stream()), "gn_sketch_pass")
    return AX, YtA


def gn_sketch(p: Problem, A: torch.Tensor, scales=None, X_user=None, Y_user=None, AX=None,
              YtA=None, want_srht: bool = False, ws=None):
    """AX (m x r) and Y^T A ((r+l) x n); optionally the SRHT signs and sample."""
    _need_cuda(A, scales, X_user, Y_user)
    acc = ACCUM_TORCH[p.mode]
    AX = torch.empty(p.m, p.r, dtype=acc, device=A.device) if AX is None else AX
    YtA = torch.empty(p.rl, p.n, dtype=acc, device=A.device) if YtA is None else YtA
    signs = idx = None
    if want_srht and p.kind_x == "srht":
        npad = 1 << max(0, (p.n - 1).bit_length())
        signs = torch.empty(npad, dtype=torch.int8, device=A.device)
        idx = torch.empty(p.r, dtype=torch.int32, device=A.device)
    ws = workspace(p, C.GN_OP_SKETCH) if ws is None else ws
    pc = p.c()
    C.check(C.lib().gn_sketch(
        ctypes.byref(pc), _ptr(A), A.stride(0), _ptr(scales),
        _ptr(X_user), X_user.stride(0) if X_user is not None else 0,
        _ptr(Y_user), Y_user.stride(0) if Y_user is not None else 0,
        _ptr(AX), AX.stride(0), _ptr(YtA), YtA.stride(0), _ptr(signs), _ptr(idx),
        _ptr(ws), ws.numel(), _stream()), "gn_sketch")
    return AX, YtA, signs, idx


@dataclass
class CoreResult:
    k: torch.Tensor       # int32[1] on device
    status: torch.Tensor  # int32[1] on device
    Q1: torch.Tensor
    R: torch.Tensor
    Q2: torch.Tensor
    R2: torch.Tensor

    def c(self) -> C.GnCoreOut:
        return C.GnCoreOut(self.k.data_ptr(), self.status.data_ptr(), self.Q1.data_ptr(),
                           self.R.data_ptr(), self.Q2.data_ptr(), self.R2.data_ptr())

    def rank(self) -> int:
        return int(self.k.item())

    def flags(self) -> int:
        return int(self.status.item())


def new_core(p: Problem, device="cuda") -> CoreResult:
    f = dict(dtype=torch.float64, device=device)
    i = dict(dtype=torch.int32, device=device)
    return CoreResult(torch.zeros(1, **i), torch.zeros(1, **i), torch.empty(p.rl, p.r, **f),
                      torch.empty(p.r, p.r, **f), torch.empty(p.r, p.r, **f),
                      torch.empty(p.r, p.r, **f))


def gn_core(p: Problem, AX: torch.Tensor, Y_user=None, out: CoreResult | None = None, ws=None,
            YtA: torch.Tensor | None = None):
    """The core from AX (and Y^T A: with an SRHT X in FP32 / BF16 mode the core
    matrix is then (Y^T A) X, see gn.h)."""
    _need_cuda(AX, Y_user, YtA)
    out = new_core(p, AX.device) if out is None else out
    ws = workspace(p, C.GN_OP_CORE) if ws is None else ws
    pc, oc = p.c(), out.c()
    C.check(C.lib().gn_core(ctypes.byref(pc), _ptr(AX), AX.stride(0), _ptr(YtA),
                            YtA.stride(0) if YtA is not None else 0, _ptr(Y_user),
                            Y_user.stride(0) if Y_user is not None else 0, ctypes.byref(oc),
                            _ptr(ws), ws.numel(), _stream()), "gn_core")
    return out


def gn_core_check(p: Problem, core: CoreResult, delta: float = 0.0, nv: int = 8, iters: int = 4,
                  est: torch.Tensor | None = None) -> torch.Tensor:
    """Section 5.1.2 power-method check of a core: returns the estimate of the
    2-norm of the inverse triangular factor (device double); sets bit 8 of
    core.status when estimate * delta * nu_x * nu_y > 1 (delta <= 0: p.eps)."""
    est = torch.zeros(1, dtype=torch.float64, device=core.R.device) if est is None else est
    ws = workspace(p, C.GN_OP_CHECK, nv, device=core.R.device)
    pc, oc = p.c(), core.c()
    C.check(C.lib().gn_core_check(ctypes.byref(pc), ctypes.byref(oc), float(delta), nv, iters,
                                  _ptr(est), _ptr(ws), ws.numel(), _stream()), "gn_core_check")
    return est


def gn_core_checked(p: Problem, AX: torch.Tensor, delta: float, nv: int = 8, iters: int = 4,
                    Y_user=None):
    """Plain GN's core, checked (Section 5.1.2); when the check flags it, the
    core is recomputed as SGN with eps = delta.  Synchronizes to read the flag.
    Returns (problem used, core, estimate, flagged)."""
    plain = dataclasses.replace(p, eps=0.0, core_method="qr")
    core = gn_core(plain, AX, Y_user)
    est = gn_core_check(plain, core, delta, nv, iters)
    flagged = bool(core.flags() & 8)
    if not flagged:
        return plain, core, est, False
    sgn = dataclasses.replace(p, eps=delta, core_method="qr")
    return sgn, gn_core(sgn, AX, Y_user), est, True


def gn_factors(p: Problem, AX, YtA, core: CoreResult, F=None, G=None):
    F = torch.empty(p.m, p.r, dtype=torch.float64, device=AX.device) if F is None else F
    G = torch.empty(p.r, p.n, dtype=torch.float64, device=AX.device) if G is None else G
    pc, oc = p.c(), core.c()
    ws = torch.empty(256, dtype=torch.uint8, device=AX.device)
    C.check(C.lib().gn_factors(ctypes.byref(pc), _ptr(AX), AX.stride(0), _ptr(YtA), YtA.stride(0),
                               ctypes.byref(oc), _ptr(F), F.stride(0), _ptr(G), G.stride(0),
                               _ptr(ws), ws.numel(), _stream()), "gn_factors")
    return F, G


def gn_apply(p: Problem, side: int, AX, YtA, core: CoreResult, W: torch.Tensor, out=None):
    """side 0: A_hat W (W n x k); side 1: W A_hat (W k x m)."""
    kc = W.shape[1] if side == 0 else W.shape[0]
    shape = (p.m, kc) if side == 0 else (kc, p.n)
    out = torch.empty(shape, dtype=torch.float64, device=W.device) if out is None else out
    ws = workspace(p, C.GN_OP_APPLY, kc)
    pc, oc = p.c(), core.c()
    C.check(C.lib().gn_apply(ctypes.byref(pc), side, _ptr(AX), AX.stride(0), _ptr(YtA),
                             YtA.stride(0), ctypes.byref(oc), _ptr(W), W.stride(0), kc, _ptr(out),
                             out.stride(0), _ptr(ws), ws.numel(), _stream()), "gn_apply")
    return out


def gn_residual(A: torch.Tensor, F: torch.Tensor, G: torch.Tensor, k: int | None = None,
                scales=None) -> torch.Tensor:
    """||A - F[:, :k] G[:k]||_F^2 as a device double (fixed-order reduction)."""
    m, n = A.shape
    k = F.shape[1] if k is None else k
    out = torch.empty(1, dtype=torch.float64, device=A.device)
    nt = ((m + 63) // 64) * ((n + 63) // 64)
    ws = torch.empty(max(8 * nt + 256, 256), dtype=torch.uint8, device=A.device)
    C.check(C.lib().gn_residual(m, n, k, _ptr(A), A.stride(0), DT_OF_TORCH[A.dtype], _ptr(scales),
                                _ptr(F), F.stride(0), _ptr(G), G.stride(0), _ptr(out), _ptr(ws),
                                ws.numel(), _stream()), "gn_residual")
    return out


def gn_residual_noalloc(A: torch.Tensor, F: torch.Tensor, G: torch.Tensor, k: int | None = None,
                        scales=None, out: torch.Tensor | None = None) -> torch.Tensor:
    """gn_residual with the library's fixed device scratch array (no workspace);
    `out` (a device double) may be given so that the call allocates nothing."""
    m, n = A.shape
    k = F.shape[1] if k is None else k
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=A.device)
    C.check(C.lib().gn_residual_noalloc(m, n, k, _ptr(A), A.stride(0), DT_OF_TORCH[A.dtype],
                                        _ptr(scales), _ptr(F), F.stride(0), _ptr(G), G.stride(0),
                                        _ptr(out), _stream()), "gn_residual_noalloc")
    return out


def gn_quantize_bf16_bs(A: torch.Tensor):
    m, n = A.shape
    out = torch.empty(m, n, dtype=torch.bfloat16, device=A.device)
    scales = torch.empty((m + 127) // 128, (n + 127) // 128, dtype=torch.float32, device=A.device)
    C.check(C.lib().gn_quantize_bf16_bs(m, n, _ptr(A), A.stride(0), DT_OF_TORCH[A.dtype], _ptr(out),
                                        out.stride(0), _ptr(scales), _stream()),
            "gn_quantize_bf16_bs")
    return out, scales


def gn_quantize_f16_bs(A: torch.Tensor):
    """binary16 storage of A with the power-of-two 128 x 128 block scales."""
    m, n = A.shape
    out = torch.empty(m, n, dtype=torch.float16, device=A.device)
    scales = torch.empty((m + 127) // 128, (n + 127) // 128, dtype=torch.float32, device=A.device)
    C.check(C.lib().gn_quantize_f16_bs(m, n, _ptr(A), A.stride(0), DT_OF_TORCH[A.dtype], _ptr(out),
                                       out.stride(0), _ptr(scales), _stream()),
            "gn_quantize_f16_bs")
    return out, scales


def solve(p: Problem, A: torch.Tensor, scales=None, X_user=None, Y_user=None):
    """Sketch pass + core: returns (AX, YtA, core)."""
    AX, YtA, _, _ = gn_sketch(p, A, scales=scales, X_user=X_user, Y_user=Y_user)
    core = gn_core(p, AX, Y_user=Y_user, YtA=YtA)
    return AX, YtA, core


def gn_materialize(p: Problem, AX, YtA, core: CoreResult, out=None):
    """A_hat (m x n) in the mode's accumulation dtype (gn_apply side 2)."""
    out = torch.empty(p.m, p.n, dtype=ACCUM_TORCH[p.mode], device=AX.device) if out is None else out
    ws = workspace(p, C.GN_OP_MATERIALIZE)
    pc, oc = p.c(), core.c()
    C.check(C.lib().gn_apply(ctypes.byref(pc), 2, _ptr(AX), AX.stride(0), _ptr(YtA), YtA.stride(0),
                             ctypes.byref(oc), None, 0, 0, _ptr(out), out.stride(0), _ptr(ws),
                             ws.numel(), _stream()), "gn_apply(side 2)")
    return out


def gn_backward(p: Problem, Gbar: torch.Tensor, YtA: torch.Tensor, core: CoreResult,
                AX: torch.Tensor | None = None, A: torch.Tensor | None = None, dA=None, ws=None):
    """dL/dA from dL/dA_hat = Gbar, with the forward's kept rank held fixed.
    AX None: recomputed from A."""
    _need_cuda(Gbar, YtA, AX, A)
    dA = torch.empty(p.m, p.n, dtype=ACCUM_TORCH[p.mode], device=Gbar.device) if dA is None else dA
    ws = workspace(p, C.GN_OP_BACKWARD) if ws is None else ws
    pc, oc = p.c(), core.c()
    C.check(C.lib().gn_backward(ctypes.byref(pc), _ptr(A), A.stride(0) if A is not None else 0,
                                _ptr(Gbar), Gbar.stride(0), _ptr(AX),
                                AX.stride(0) if AX is not None else 0, _ptr(YtA), YtA.stride(0),
                                ctypes.byref(oc), _ptr(dA), dA.stride(0), _ptr(ws), ws.numel(),
                                _stream()), "gn_backward")
    return dA


def gn_sketch_extend(p_old: Problem, p_new: Problem, A, AX, YtA, ws=None):
    """Resampling r -> r + dr (Section 6): AX (m x r_new) and YtA (rl_new x n) hold
    the old products in their leading columns / rows; the new ones are filled in."""
    _need_cuda(A, AX, YtA)
    ws = workspace(p_new, C.GN_OP_UPDATE) if ws is None else ws
    po, pn = p_old.c(), p_new.c()
    C.check(C.lib().gn_sketch_extend(ctypes.byref(po), ctypes.byref(pn), _ptr(A), A.stride(0),
                                     _ptr(AX), AX.stride(0), _ptr(YtA), YtA.stride(0), _ptr(ws),
                                     ws.numel(), _stream()), "gn_sketch_extend")
    return AX, YtA


def gn_sketch_append(p: Problem, axis: int, old_size: int, B, AX, YtA, ws=None):
    """Appended rows (axis 0) or columns (axis 1) B (Section 6); p is the enlarged
    problem, AX / YtA its buffers holding the old products in place."""
    _need_cuda(B, AX, YtA)
    ws = workspace(p, C.GN_OP_UPDATE) if ws is None else ws
    pc = p.c()
    C.check(C.lib().gn_sketch_append(ctypes.byref(pc), axis, old_size, _ptr(B), B.stride(0),
                                     _ptr(AX), AX.stride(0), _ptr(YtA), YtA.stride(0), _ptr(ws),
                                     ws.numel(), _stream()), "gn_sketch_append")
    return AX, YtA


def gn_sketch_update(p: Problem, E, AX, YtA, ws=None):
    """A -> A + E (Section 6): AX += E X, Y^T A += Y^T E in place."""
    _need_cuda(E, AX, YtA)
    ws = workspace(p, C.GN_OP_UPDATE) if ws is None else ws
    pc = p.c()
    C.check(C.lib().gn_sketch_update(ctypes.byref(pc), _ptr(E), E.stride(0), _ptr(AX), AX.stride(0),
                                     _ptr(YtA), YtA.stride(0), _ptr(ws), ws.numel(), _stream()),
            "gn_sketch_update")
    return AX, YtA


class GNApprox(torch.autograd.Function):
    """A -> A_hat = AX (Y^T A X)_eps^+ Y^T A as a differentiable torch op.

    forward runs the sketch pass, the core and materializes A_hat; backward calls
    gn_backward with the kept rank of this forward held fixed.  With
    store_ax=False the forward keeps A instead of AX and the backward recomputes
    AX = A X (less memory when r is large relative to the batch of saved tensors).
    """

    @staticmethod
    def forward(ctx, A, p: Problem, store_ax: bool = True):
        AX, YtA, core = solve(p, A)
        Ahat = gn_materialize(p, AX, YtA, core)
        ctx.p, ctx.core, ctx.store_ax = p, core, store_ax
        if store_ax:
            ctx.save_for_backward(AX, YtA)
        else:
            ctx.save_for_backward(A, YtA)
        return Ahat

    @staticmethod
    def backward(ctx, gout):
        first, YtA = ctx.saved_tensors
        gout = gout.contiguous()
        if ctx.store_ax:
            dA = gn_backward(ctx.p, gout, YtA, ctx.core, AX=first)
        else:
            dA = gn_backward(ctx.p, gout, YtA, ctx.core, A=first)
        return dA, None, None


def gn_approx(A: torch.Tensor, p: Problem, store_ax: bool = True) -> torch.Tensor:
    """Differentiable A_hat (see GNApprox)."""
    return GNApprox.apply(A, p, store_ax)


class Batch:
    """Many independent FP32 problems (Gaussian X and Y) solved by gn_batch_solve.

    problems: list of (Problem, A) with Problem.mode "f32"; A float32 (m x n, row
    stride a multiple of 4).  Allocates AX, YtA and the core outputs of every
    problem and the workspace, then calls gn_batch_prepare.  solve() enqueues the
    passes and cores of all problems (graph-capturable).
    """

    def __init__(self, problems, tile_policy=None, device="cuda"):
        if tile_policy is None:   # the autotuner's table, when one has been written
            from .autotune import load_policy
            tile_policy = load_policy("batch_f32")
        self.problems = [p for p, _ in problems]
        self.A = [a for _, a in problems]
        self.AX, self.YtA, self.core = [], [], []
        arr = (C.GnBatchProblem * len(problems))()
        for i, (p, A) in enumerate(problems):
            if p.mode != "f32" or p.kind_x != "gaussian" or p.kind_y != "gaussian":
                raise ValueError("batches are FP32 with Gaussian X and Y")
            _need_cuda(A)
            if A.dtype != torch.float32:
                raise ValueError("A must be float32")
            ldax = (p.r + 3) // 4 * 4
            AX = torch.empty(p.m, ldax, dtype=torch.float32, device=device)[:, :p.r]
            YtA = torch.empty(p.rl, p.n, dtype=torch.float32, device=device)
            core = new_core(p, device)
            self.AX.append(AX)
            self.YtA.append(YtA)
            self.core.append(core)
            arr[i] = C.GnBatchProblem(p.m, p.n, p.r, p.l, p.seed & ((1 << 64) - 1), p.eps,
                                      A.data_ptr(), A.stride(0), AX.data_ptr(), AX.stride(0),
                                      YtA.data_ptr(), YtA.stride(0), core.c())
        self._arr = arr
        nbytes = ctypes.c_size_t(0)
        C.check(C.lib().gn_batch_workspace_size(arr, len(problems), ctypes.byref(nbytes)),
                "gn_batch_workspace_size")
        self.ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=device)
        self.plan = C.GnBatchPlan()
        pol = None if tile_policy is None else (ctypes.c_int32 * 4)(*tile_policy)
        C.check(C.lib().gn_batch_prepare(arr, len(problems), pol, ctypes.byref(self.plan),
                                         _ptr(self.ws), self.ws.numel(), _stream()),
                "gn_batch_prepare")

    def solve(self, stages: int = C.GN_BATCH_ALL):
        C.check(C.lib().gn_batch_solve(ctypes.byref(self.plan), stages, _ptr(self.ws),
                                       self.ws.numel(), _stream()), "gn_batch_solve")
