"""Python API over libbds: tensors and streams from PyTorch, all arithmetic in the HIP library.

    F = factor(Ad, As, prec="f64")      # recursive factorisation (the paper's Alg. 4)
    X = F.solve(B)                      # recursive solve (Alg. 5-7), refined if prec != "f64"
    F.tune(B)                           # autotuner: crossover nstar and tile shapes for this shape
    X = solve(Ad, As, B)                # differentiable: torch.autograd.Function

Shapes (float64, CUDA/HIP device, C-contiguous): Ad (N, n, n) with only the
lower triangle read, As (N-1, n, n) with As[i] = A[i+1, i], B (N, n, d).
"""
from __future__ import annotations

import ctypes

import torch

from . import _binding as bb

PRECISIONS = {"f64": bb.BDS_F64, "f32": bb.BDS_F32, "bf16": bb.BDS_BF16}


class BdsError(RuntimeError):
    def __init__(self, code: int, what: str, info: dict | None = None):
        self.code = code
        self.info = info
        super().__init__(f"{what}: {bb.STATUS_NAMES.get(code, code)}" + (f" {info}" if info else ""))


def _stream_handle(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_tensor(t: torch.Tensor, name: str, shape: tuple, device: torch.device | None = None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() > 0 else 0)


def _info_dict(info: torch.Tensor) -> dict:
    v = info.cpu().tolist()
    keys = ("status", "level", "position", "orig_block", "column", "iters", "converged", "reserved")
    return dict(zip(keys, v))


class Factor:
    """Factor hierarchy of one SPD block-tridiagonal matrix, held in a device workspace."""

    def __init__(self, Ad: torch.Tensor, As: torch.Tensor | None, prec: str = "f64", nstar: int = 0,
                 check: bool = True, tiles: int = 0):
        if Ad.dim() != 3:
            raise ValueError("Ad must have shape (N, n, n)")
        N, n, _ = Ad.shape
        self.device = Ad.device
        _check_tensor(Ad, "Ad", (N, n, n))
        if N > 1:
            _check_tensor(As, "As", (N - 1, n, n), self.device)
        self.N, self.n = int(N), int(n)
        self.prec = prec
        self.nstar = int(nstar)
        self.tiles = int(tiles)
        self.Ad, self.As = Ad, (As if N > 1 else None)
        self._solve_ws = {}
        self.info_t = torch.zeros(8, dtype=torch.int32, device=self.device)
        self._alloc_factor()
        self.refactor(check=check)

    def _alloc_factor(self):
        rc, fbytes, _ = bb.workspace_size(self._desc(1))
        if rc != bb.BDS_OK:
            raise BdsError(rc, "bds_workspace_size")
        self.fbytes = fbytes
        self.fws = torch.empty(max(fbytes, 1), dtype=torch.uint8, device=self.device)

    def refactor(self, check: bool = False):
        """Run bds_factor again on the same Ad/As into the existing workspace (no allocation)."""
        desc = self._desc(1)
        rc = bb.load().bds_factor(ctypes.byref(desc), _ptr(self.Ad), _ptr(self.As), _ptr(self.fws), self.fbytes,
                                  _ptr(self.info_t), _stream_handle(self.device))
        if rc != bb.BDS_OK:
            raise BdsError(rc, "bds_factor")
        if check:
            self.check("bds_factor")

    def _desc(self, d: int, max_refine: int = 0, refine_tol: float = 0.0) -> bb.BdsDesc:
        if self.prec not in PRECISIONS:
            raise ValueError(f"prec must be one of {list(PRECISIONS)}")
        return bb.BdsDesc(self.N, self.n, int(d), PRECISIONS[self.prec], self.nstar, int(max_refine),
                          self.tiles, float(refine_tol))

    def info(self) -> dict:
        """Synchronise and read the device info record of the last call."""
        return _info_dict(self.info_t)

    def check(self, what: str = "bds"):
        inf = self.info()
        if inf["status"] != bb.BDS_OK:
            raise BdsError(inf["status"], what, inf)
        return inf

    def _workspace(self, d: int, desc: bb.BdsDesc):
        ws = self._solve_ws.get(d)
        if ws is None:
            rc, _, sbytes = bb.workspace_size(desc)
            if rc != bb.BDS_OK:
                raise BdsError(rc, "bds_workspace_size")
            ws = torch.empty(max(sbytes, 1), dtype=torch.uint8, device=self.device)
            self._solve_ws[d] = ws
        return ws

    def solve(self, B: torch.Tensor, out: torch.Tensor | None = None, max_refine: int = 0,
              refine_tol: float = 0.0, check: bool = True) -> torch.Tensor:
        if B.dim() != 3:
            raise ValueError("B must have shape (N, n, d)")
        d = int(B.shape[2])
        _check_tensor(B, "B", (self.N, self.n, d), self.device)
        X = torch.empty_like(B) if out is None else out
        _check_tensor(X, "out", (self.N, self.n, d), self.device)
        desc = self._desc(d, max_refine, refine_tol)
        ws = self._workspace(d, desc)
        rc = bb.load().bds_solve(ctypes.byref(desc), _ptr(self.fws), self.fbytes, _ptr(self.Ad), _ptr(self.As),
                                 _ptr(B), _ptr(X), _ptr(ws), ws.numel(), _ptr(self.info_t),
                                 _stream_handle(self.device))
        if rc != bb.BDS_OK:
            raise BdsError(rc, "bds_solve")
        if check and self.prec != "f64":
            self.check("bds_solve")
        return X

    def tune(self, B: torch.Tensor, reps: int = 3, max_refine: int = 0, refine_tol: float = 0.0) -> dict:
        """Run the library's autotuner (bds_tune) on this system with right-hand side B.

        The fields left to the library (nstar == 0, zero tile fields) are searched; the factor is then
        rebuilt with the winner, which later solves use.  Returns the chosen nstar and tile shapes.
        """
        d = int(B.shape[2])
        _check_tensor(B, "B", (self.N, self.n, d), self.device)
        desc = self._desc(d, max_refine, refine_tol)
        rc, fbytes, sbytes = bb.tune_workspace_size(desc)
        if rc != bb.BDS_OK:
            raise BdsError(rc, "bds_tune_workspace_size")
        fws = torch.empty(max(fbytes, 1), dtype=torch.uint8, device=self.device)
        sws = torch.empty(max(sbytes, 1), dtype=torch.uint8, device=self.device)
        X = torch.empty_like(B)
        best = bb.BdsDesc()
        rc = bb.load().bds_tune(ctypes.byref(desc), _ptr(self.Ad), _ptr(self.As), _ptr(B), _ptr(X), _ptr(fws),
                                fbytes, _ptr(sws), sbytes, _ptr(self.info_t), int(reps),
                                _stream_handle(self.device), ctypes.byref(best))
        if rc != bb.BDS_OK:
            raise BdsError(rc, "bds_tune")
        self.check("bds_tune")
        del fws, sws
        self.nstar, self.tiles = int(best.nstar), int(best.tiles)
        self._solve_ws = {}
        self._alloc_factor()
        self.refactor(check=True)
        return {"nstar": self.nstar, "tiles": self.tiles, **bb.tiles_fields(self.tiles)}

    def backward(self, X: torch.Tensor, dX: torch.Tensor, check: bool = True):
        """Gradients (dAd, dAs, dB) of a loss with dL/dX = dX, for X = A^-1 B."""
        d = int(X.shape[2])
        _check_tensor(X, "X", (self.N, self.n, d), self.device)
        _check_tensor(dX, "dX", (self.N, self.n, d), self.device)
        desc = self._desc(d)
        ws = self._workspace(d, desc)
        dAd = torch.empty((self.N, self.n, self.n), dtype=torch.float64, device=self.device)
        dAs = torch.empty((max(self.N - 1, 0), self.n, self.n), dtype=torch.float64, device=self.device)
        dB = torch.empty_like(X)
        rc = bb.load().bds_backward(ctypes.byref(desc), _ptr(self.fws), self.fbytes, _ptr(self.Ad), _ptr(self.As),
                                    _ptr(X), _ptr(dX), _ptr(dAd), _ptr(dAs), _ptr(dB), _ptr(ws), ws.numel(),
                                    _ptr(self.info_t), _stream_handle(self.device))
        if rc != bb.BDS_OK:
            raise BdsError(rc, "bds_backward")
        if check and self.prec != "f64":
            self.check("bds_backward")
        return dAd, dAs, dB


def _ptr_array(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() if t is not None and t.numel() > 0 else 0 for t in ts])


class BatchedFactor:
    """Factor hierarchies of K independent systems of uneven size, built by one launch per kernel and level."""

    def __init__(self, Ads, Ass, prec: str = "f64", nstar: int = 0, check: bool = True, tiles=None):
        if len(Ads) != len(Ass) or len(Ads) == 0:
            raise ValueError("need equally many (>= 1) Ad and As tensors")
        self.K = len(Ads)
        self.device = Ads[0].device
        self.prec, self.nstar = prec, int(nstar)
        self.tiles = [0] * self.K if tiles is None else [int(t) for t in tiles]
        if len(self.tiles) != self.K:
            raise ValueError("tiles needs one entry per system")
        self.shapes = []
        for k, (Ad, As) in enumerate(zip(Ads, Ass)):
            if Ad.dim() != 3:
                raise ValueError(f"Ad[{k}] must have shape (N, n, n)")
            N, n, _ = Ad.shape
            _check_tensor(Ad, f"Ad[{k}]", (N, n, n), self.device)
            if N > 1:
                _check_tensor(As, f"As[{k}]", (N - 1, n, n), self.device)
            self.shapes.append((int(N), int(n)))
        self.Ads = list(Ads)
        self.Ass = [As if N > 1 else None for As, (N, _) in zip(Ass, self.shapes)]
        self._solve_ws = {}
        self.info_t = torch.zeros((self.K, 8), dtype=torch.int32, device=self.device)
        self._Ad_p = _ptr_array(self.Ads)
        self._As_p = _ptr_array(self.Ass)
        self._alloc_factor()
        self.refactor(check=check)

    def _sizes(self, descs):
        f = ctypes.c_size_t(0)
        sb = ctypes.c_size_t(0)
        rc = bb.load().bds_batched_workspace_size(self.K, descs, ctypes.byref(f), ctypes.byref(sb))
        if rc != bb.BDS_OK:
            raise BdsError(rc, "bds_batched_workspace_size")
        return f.value, sb.value

    def _alloc_factor(self):
        self.fbytes, _ = self._sizes(self._descs([1] * self.K))
        self.fws = torch.empty(max(self.fbytes, 1), dtype=torch.uint8, device=self.device)

    def _descs(self, ds, max_refine: int = 0, refine_tol: float = 0.0):
        arr = (bb.BdsDesc * self.K)()
        for k, ((N, n), d) in enumerate(zip(self.shapes, ds)):
            arr[k] = bb.BdsDesc(N, n, int(d), PRECISIONS[self.prec], self.nstar, int(max_refine), self.tiles[k],
                                float(refine_tol))
        return arr

    def tune(self, Bs, reps: int = 3, max_refine: int = 0, refine_tol: float = 0.0) -> dict:
        """Run the batched autotuner (bds_tune_batched): tile shapes per padded block size, chosen by
        timing factor + solve of the whole batch.  The factor is rebuilt with the winner.  Returns
        {np: {"couple": .., "schur": .., "solve": ..}}."""
        ds = [int(B.shape[2]) for B in Bs]
        descs = self._descs(ds, max_refine, refine_tol)
        fbytes, sbytes = self._sizes(descs)
        fws = torch.empty(max(fbytes, 1), dtype=torch.uint8, device=self.device)
        sws = torch.empty(max(sbytes, 1), dtype=torch.uint8, device=self.device)
        Xs = [torch.empty_like(B) for B in Bs]
        best = (bb.BdsDesc * self.K)()
        rc = bb.load().bds_tune_batched(self.K, descs, self._Ad_p, self._As_p, _ptr_array(Bs), _ptr_array(Xs),
                                        _ptr(fws), fbytes, _ptr(sws), sbytes, _ptr(self.info_t), int(reps),
                                        _stream_handle(self.device), best)
        if rc != bb.BDS_OK:
            raise BdsError(rc, "bds_tune_batched")
        self.check("bds_tune_batched")
        del fws, sws
        self.tiles = [int(best[k].tiles) for k in range(self.K)]
        self._solve_ws = {}
        self._alloc_factor()
        self.refactor(check=True)
        out = {}
        for (N, n), t in zip(self.shapes, self.tiles):
            out[(n + 15) // 16 * 16] = bb.tiles_fields(t)
        return out

    def refactor(self, check: bool = False):
        descs = self._descs([1] * self.K)
        rc = bb.load().bds_factor_batched(self.K, descs, self._Ad_p, self._As_p, _ptr(self.fws), self.fbytes,
                                          _ptr(self.info_t), _stream_handle(self.device))
        if rc != bb.BDS_OK:
            raise BdsError(rc, "bds_factor_batched")
        if check:
            self.check("bds_factor_batched")

    def info(self) -> list:
        keys = ("status", "level", "position", "orig_block", "column", "iters", "converged", "reserved")
        return [dict(zip(keys, row)) for row in self.info_t.cpu().tolist()]

    def check(self, what: str = "bds"):
        infos = self.info()
        for k, inf in enumerate(infos):
            if inf["status"] != bb.BDS_OK:
                raise BdsError(inf["status"], f"{what} (system {k})", inf)
        return infos

    def solve(self, Bs, outs=None, max_refine: int = 0, refine_tol: float = 0.0, check: bool = True):
        if len(Bs) != self.K:
            raise ValueError(f"expected {self.K} right-hand sides")
        ds = []
        for k, (B, (N, n)) in enumerate(zip(Bs, self.shapes)):
            if B.dim() != 3:
                raise ValueError(f"B[{k}] must have shape (N, n, d)")
            _check_tensor(B, f"B[{k}]", (N, n, int(B.shape[2])), self.device)
            ds.append(int(B.shape[2]))
        Xs = [torch.empty_like(B) for B in Bs] if outs is None else list(outs)
        for k, X in enumerate(Xs):
            _check_tensor(X, f"out[{k}]", tuple(Bs[k].shape), self.device)
        descs = self._descs(ds, max_refine, refine_tol)
        key = tuple(ds)
        ws = self._solve_ws.get(key)
        if ws is None:
            _, sb = self._sizes(descs)
            ws = torch.empty(max(sb, 1), dtype=torch.uint8, device=self.device)
            self._solve_ws[key] = ws
        rc = bb.load().bds_solve_batched(self.K, descs, _ptr(self.fws), self.fbytes, self._Ad_p, self._As_p,
                                         _ptr_array(Bs), _ptr_array(Xs), _ptr(ws), ws.numel(), _ptr(self.info_t),
                                         _stream_handle(self.device))
        if rc != bb.BDS_OK:
            raise BdsError(rc, "bds_solve_batched")
        if check and self.prec != "f64":
            self.check("bds_solve_batched")
        return Xs


def factor_batched(Ads, Ass, prec: str = "f64", nstar: int = 0, check: bool = True, tiles=None) -> BatchedFactor:
    return BatchedFactor(Ads, Ass, prec=prec, nstar=nstar, check=check, tiles=tiles)


def factor(Ad: torch.Tensor, As: torch.Tensor | None, prec: str = "f64", nstar: int = 0,
           check: bool = True, tiles: int = 0) -> Factor:
    return Factor(Ad, As, prec=prec, nstar=nstar, check=check, tiles=tiles)


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Ad, As, B, prec, nstar):
        F = Factor(Ad.detach(), As.detach() if As is not None else None, prec=prec, nstar=nstar)
        X = F.solve(B.detach())
        ctx.F = F
        ctx.save_for_backward(X)
        return X

    @staticmethod
    def backward(ctx, dX):
        (X,) = ctx.saved_tensors
        dAd, dAs, dB = ctx.F.backward(X, dX.contiguous())
        return dAd, dAs, dB, None, None


def solve(Ad: torch.Tensor, As: torch.Tensor, B: torch.Tensor, prec: str = "f64", nstar: int = 0) -> torch.Tensor:
    """X = A^-1 B, differentiable in Ad (as a symmetric block), As and B."""
    return _Solve.apply(Ad, As, B, prec, nstar)
