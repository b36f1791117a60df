"""Convenience wrapper over the C ABI for torch device tensors.

Argument marshalling only: the points stay in the caller's tensor (borrowed,
kept alive by this object) and every step runs in ``libscpmwu.so``.
"""
from __future__ import annotations

from . import _lib as L

_DTYPES = None


def _dtype_code(t):
    import torch
    global _DTYPES
    if _DTYPES is None:
        _DTYPES = {torch.float32: L.SCP_MWU_F32, torch.bfloat16: L.SCP_MWU_BF16,
                   torch.float64: L.SCP_MWU_F64}
    if t.dtype not in _DTYPES:
        raise TypeError(f"points must be float32, bfloat16 or float64, not {t.dtype}")
    return _DTYPES[t.dtype]


class MWU:
    """One SES or SVM problem on the GPU.

    points   device tensor n x d (row stride >= d, unit column stride); SVM rows
             [0, n_pos) are class +1 and the rest class -1.
    storage  None (stream the points as given), "bf16" (round FP32 points
             once into a library-owned BF16 copy) or "fp8" (quantize FP32
             points once into library-owned per-row scaled FP8 E4M3 codes).
    """

    def __init__(self, points, problem: str = "ses", *, n_pos: int | None = None, radii=None,
                 v1: int = 0, eps: float = 1e-3, delta: float = 1e-4, patience: int = 10,
                 flags: int = 0, t_cap: int = 0, max_iters: int = 0, storage: str | None = None,
                 chunk: int = 0, grid: int = 0, stream=None):
        import torch
        L.load()
        if not points.is_cuda:
            raise ValueError("points must be a device (HIP) tensor")
        if points.dim() != 2 or points.stride(1) != 1:
            raise ValueError("points must be 2-D with unit column stride")
        self.points = points
        self.radii = radii
        self.problem = problem
        self.n, self.d = points.shape
        self.svm = problem == "svm"
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        self.stream = stream
        desc = L.scp_mwu_desc()
        desc.struct_size = __import__("ctypes").sizeof(L.scp_mwu_desc)
        desc.problem = L.SCP_MWU_PROBLEM_SVM if self.svm else L.SCP_MWU_PROBLEM_SES
        desc.dtype = _dtype_code(points)
        desc.storage = {None: 0, "bf16": L.SCP_MWU_BF16, "fp8": L.SCP_MWU_FP8}[storage]
        desc.n, desc.d, desc.ld = self.n, self.d, points.stride(0)
        desc.points = points.data_ptr()
        if radii is not None:
            if radii.dtype != torch.float64 or not radii.is_cuda or radii.numel() != self.n:
                raise ValueError("radii must be a device float64 tensor of length n")
            desc.radii = radii.data_ptr()
        desc.n_pos = int(n_pos or 0)
        desc.v1_index = int(v1)
        desc.eps, desc.delta, desc.patience = float(eps), float(delta), int(patience)
        desc.flags, desc.t_cap, desc.max_iters = int(flags), int(t_cap), int(max_iters)
        desc.stream = stream.cuda_stream
        desc.chunk, desc.grid = int(chunk), int(grid)
        with torch.cuda.device(points.device):
            self.ctx = L.scp_mwu_init(desc)
        self.D = L.scp_mwu_get_D(self.ctx)

    # -- lifetime
    def close(self):
        if getattr(self, "ctx", None):
            L.scp_mwu_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls
    def step(self, alpha: float, T: int, k: int, reset: bool = False) -> dict:
        info = L.scp_mwu_step(self.ctx, float(alpha), int(T), int(k), int(reset))
        out = {f: getattr(info, f) for f, _ in L.scp_mwu_stepinfo._fields_}
        out["outcome_name"] = L.OUTCOME_NAMES[info.outcome]
        return out

    def solve(self) -> dict:
        code, res, y = L.scp_mwu_solve(self.ctx, self.d)
        out = {f: getattr(res, f) for f, _ in L.scp_mwu_result._fields_}
        out["code"] = code
        if self.svm:
            out["w"], out["s1"], out["s2"] = y[: self.d], y[self.d], y[self.d + 1]
        else:
            out["center"], out["radius"] = y[: self.d], y[self.d]
        return out

    def get_state(self):
        return L.scp_mwu_get_state(self.ctx, self.d, self.svm)

    def set_state(self, alpha: float, T: int, t: int, sums) -> None:
        L.scp_mwu_set_state(self.ctx, float(alpha), int(T), int(t), list(sums))

    def vector(self, which: int):
        return L.scp_mwu_get_vector(self.ctx, which, self.d, self.svm)

    def time_passes(self, k: int):
        """(pass-kernel ms, whole-iteration ms): HIP-event means over k further iterations."""
        return L.scp_mwu_time_passes(self.ctx, int(k))

    def backward(self, grad_value: float = 1.0, out=None, checkpoint_every: int = 50):
        """(R, grad_value * dR/dV) of the T-iteration map at the current
        test's alpha and T: R = max_i ||v_i - ubar_T||, the gradient an
        n x d float32 device tensor (written into `out` when given).
        checkpoint_every: K in 1..50 keeps the running sum every K iterations
        and recomputes segments; 0 keeps the whole tape."""
        import torch
        if out is None:
            out = torch.empty(self.n, self.d, dtype=torch.float32, device=self.points.device)
        if out.dtype != torch.float32 or out.shape != (self.n, self.d) or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 n x d tensor")
        with torch.cuda.device(self.points.device):
            R = L.scp_mwu_backward(self.ctx, float(grad_value), out.data_ptr(), int(checkpoint_every))
        return R, out

    def radius(self, checkpoint_every: int = 50) -> float:
        """R of the T-iteration map at the current test's alpha and T (the
        forward iterations of backward() without the reverse pass)."""
        import torch
        with torch.cuda.device(self.points.device):
            return L.scp_mwu_backward(self.ctx, 1.0, None, int(checkpoint_every))


class MWUBatch:
    """Many independent SES point sets solved together (one streaming pass per
    column layout and one epilogue launch per MWU iteration of the batch).

    points   device float32 tensor holding every instance's rows back to back
             (instance k: n[k] dense rows of d[k] values from element
             offset[k]; offsets default to the packed layout).
    storage  None or "bf16" (library-owned BF16 copy).
    """

    def __init__(self, points, n, d, offset=None, *, eps: float = 1e-3, delta: float = 1e-4,
                 patience: int = 10, flags: int = 0, t_cap: int = 0, max_iters: int = 0,
                 storage: str | None = None, chunk: int = 0, rows_per_group: int = 0, stream=None):
        import ctypes
        import torch
        L.load()
        if not points.is_cuda or points.dtype != torch.float32 or not points.is_contiguous():
            raise ValueError("points must be a contiguous float32 device tensor")
        self.points = points
        self.n = [int(v) for v in n]
        self.d = [int(v) for v in d]
        self.m = len(self.n)
        if offset is None:
            offset, o = [], 0
            for nk, dk in zip(self.n, self.d):
                offset.append(o)
                o += nk * dk
        self.offset = [int(v) for v in offset]
        self.d_total = sum(self.d)
        if stream is None:
            stream = torch.cuda.current_stream(points.device)
        self.stream = stream
        I64 = ctypes.c_int64 * self.m
        self._arrays = (I64(*self.n), I64(*self.d), I64(*self.offset))
        desc = L.scp_mwu_batch_desc()
        desc.struct_size = ctypes.sizeof(L.scp_mwu_batch_desc)
        desc.dtype = L.SCP_MWU_F32
        desc.storage = {None: 0, "bf16": L.SCP_MWU_BF16}[storage]
        desc.count = self.m
        desc.n, desc.d, desc.offset = self._arrays
        desc.points = points.data_ptr()
        desc.eps, desc.delta, desc.patience = float(eps), float(delta), int(patience)
        desc.flags, desc.t_cap, desc.max_iters = int(flags), int(t_cap), int(max_iters)
        desc.stream = stream.cuda_stream
        desc.chunk, desc.rows_per_group = int(chunk), int(rows_per_group)
        with torch.cuda.device(points.device):
            self.b = L.scp_mwu_batch_init(desc)
        self.D = L.scp_mwu_batch_get_D(self.b, self.m)

    def close(self):
        if getattr(self, "b", None):
            L.scp_mwu_batch_destroy(self.b)
            self.b = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _split(self, flat, extra=0):
        out, o = [], 0
        for dk in self.d:
            out.append(flat[o:o + dk + extra])
            o += dk + extra
        return out

    def step(self, alpha, T, k: int, reset: bool = False) -> list:
        infos = L.scp_mwu_batch_step(self.b, list(alpha), list(T), int(k), int(reset))
        out = []
        for info in infos:
            r = {f: getattr(info, f) for f, _ in L.scp_mwu_stepinfo._fields_}
            r["outcome_name"] = L.OUTCOME_NAMES[info.outcome]
            out.append(r)
        return out

    def solve(self):
        code, res, y = L.scp_mwu_batch_solve(self.b, self.m, self.d_total)
        out = []
        for r, yk in zip(res, self._split(y, 1)):
            o = {f: getattr(r, f) for f, _ in L.scp_mwu_result._fields_}
            o["center"], o["radius"] = yk[:-1], yk[-1]
            out.append(o)
        return code, out

    def solve_kway(self):
        """k-way alpha search over one point set: the batch's k instances must
        be that point set (see MWUBatch.kway)."""
        code, res, y = L.scp_mwu_batch_solve_kway(self.b, self.d[0])
        out = {f: getattr(res, f) for f, _ in L.scp_mwu_result._fields_}
        out["code"], out["center"], out["radius"] = code, y[:-1], y[-1]
        return out

    @classmethod
    def kway(cls, points, k: int, **kw):
        """A batch of k test slots over one n x d point set (a 2-D float32
        device tensor) for solve_kway."""
        n, d = points.shape
        return cls(points.reshape(-1), [n] * k, [d] * k, [0] * k, **kw)

    def vectors(self, which: int) -> list:
        return self._split(L.scp_mwu_batch_get_vector(self.b, which, self.d_total))

    def time_iters(self, k: int):
        """(pass ms, whole-iteration ms): HIP-event means over k further iterations."""
        return L.scp_mwu_batch_time_iters(self.b, int(k))


class ProductCone:
    """A product cone R^{n_orth}_+ (+) Q^{d+1} for each d in dims, validated once
    (its block offsets resident on the device, its workspace owned by the
    library); exp() computes the SCMWU iterate exp(-eta m) / Tr(...) of a
    float64 device vector m laid out as the orthant coordinates, then each
    block's vector part and scalar part."""

    def __init__(self, n_orth: int, dims, device=None, stream=None):
        import numpy as np
        import torch
        L.load()
        dims = np.asarray(dims, dtype=np.int64).reshape(-1)
        offsets = np.empty(dims.size + 1, dtype=np.int64)
        offsets[0] = int(n_orth)
        np.cumsum(dims + 1, out=offsets[1:])
        offsets[1:] += int(n_orth)
        self.n_orth, self.nblocks = int(n_orth), int(dims.size)
        self.length = int(offsets[-1])
        self.device = torch.device("cuda") if device is None else torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        with torch.cuda.device(self.device):
            self.handle = L.scp_mwu_product_init(self.n_orth, offsets if dims.size else [], self.length,
                                                 stream.cuda_stream)

    def exp(self, m, eta: float, out=None, log_trace: bool = True):
        """(p, ln Tr); with log_trace=False the launches are only enqueued on
        the stream and ln Tr is None."""
        import torch
        if (not m.is_cuda or m.dtype != torch.float64 or m.dim() != 1 or not m.is_contiguous()
                or m.numel() != self.length):
            raise ValueError("m must be a contiguous float64 device vector of the cone's length")
        if out is None:
            out = torch.empty_like(m)
        if out.shape != m.shape or out.dtype != m.dtype or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 vector of m's length")
        with torch.cuda.device(m.device):
            lt = L.scp_mwu_product_exp(self.handle, m.data_ptr(), float(eta), out.data_ptr(), log_trace)
        return out, lt

    def close(self):
        if getattr(self, "handle", None):
            L.scp_mwu_product_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def product_exp(m, n_orth: int, dims, eta: float, out=None):
    """One-off SCMWU iterate exp(-eta m) / Tr(...) over R^{n_orth}_+ (+) Q^{d+1}
    for each d in dims (a ProductCone made and released for the call).
    Returns (p, ln Tr)."""
    import torch
    if not m.is_cuda or m.dtype != torch.float64 or m.dim() != 1:
        raise ValueError("m must be a float64 device vector")
    with ProductCone(n_orth, dims, device=m.device) as pc:
        if m.numel() != pc.length:
            raise ValueError("m's length does not match n_orth and dims")
        return pc.exp(m, eta, out)


def _radius_function():
    import torch

    class _Radius(torch.autograd.Function):
        @staticmethod
        def forward(ctx, points, alpha, T):
            m = MWU(points.detach(), "ses", flags=L.SCP_MWU_FLAG_NO_EARLY_STOP)
            m.step(alpha, T, 0, reset=True)       # starts the test that fixes alpha and T
            R = m.radius()                        # the forward map only
            if ctx.needs_input_grad[0]:            # the points require grad and grad mode is on
                ctx.mwu = m                       # the reverse pass runs in backward()
            else:
                m.close()
                ctx.mwu = None
            ctx.points_dtype = points.dtype
            return torch.tensor(R, dtype=torch.float64, device=points.device)

        @staticmethod
        def backward(ctx, grad_out):
            m, ctx.mwu = ctx.mwu, None
            if m is None:
                raise RuntimeError("ses_radius: backward through a forward run without gradients")
            try:
                _, g = m.backward(float(grad_out))
            finally:
                m.close()
            return g.to(ctx.points_dtype), None, None

    return _Radius


_RADIUS = None


def ses_radius(points, alpha: float, T: int):
    """R = max_i ||v_i - ubar_T|| after T fixed-alpha SES iterations on the
    points (float32 or float64 device tensor, n x d) as a differentiable
    torch scalar (float64).  The forward call runs the T iterations only; the
    reverse pass runs in backward, scaled by the incoming gradient."""
    global _RADIUS
    if _RADIUS is None:
        _RADIUS = _radius_function()
    return _RADIUS.apply(points, float(alpha), int(T))


def autotune_rows_per_group(points, n, d, offset=None, candidates=(2048, 4096, 8192, 16384, 32768),
                            iters: int = 10, storage: str | None = None):
    """Pick the workgroup share (rows per workgroup) of a batch's streaming
    pass by timing `iters` iterations of a running test (alpha = D, the
    points' own enclosing radius) for each candidate with the library's HIP
    event timer.  Returns (best, {candidate: pass ms})."""
    times = {}
    for rpg in candidates:
        with MWUBatch(points, n, d, offset, flags=L.SCP_MWU_FLAG_NO_EARLY_STOP, storage=storage,
                      rows_per_group=int(rpg)) as b:
            b.step(b.D, [20000] * b.m, 2, reset=True)
            times[int(rpg)] = b.time_iters(iters)[0]
    best = min(times, key=times.get)
    return best, times
