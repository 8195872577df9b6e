"""Python binding of the HIP library: argument marshalling only.

Every step of the sweep runs in the library's kernels; torch provides device
memory and the stream.  Arrays are dimension-major ([n][Q]) float32 CUDA
tensors, as in include/hjg.h.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check


@dataclass
class ProblemSpec:
    """Python view of struct hjg_problem (see include/hjg.h for each field)."""
    n: int
    ham: str = "quadratic"
    datum: str = "ball"
    nu: float = 0.05
    ham_p: Sequence[float] = (1.0, 1.0, 1.0, 1.0)
    datum_p: Sequence[float] = ()
    datum_aux: Optional[torch.Tensor] = None
    eta: float = 1e-2
    c_min: float = 1e-2
    c_max: float = 1e4
    tilt: bool = False
    sample_mode: str = "crn_step"
    sample_bf16: bool = False
    grad_cv: bool = False
    seed: int = 0
    problem_id: int = 0
    tube: bool = False

    def to_c(self) -> _lib.Problem:
        p = _lib.Problem()
        p.n = self.n
        p.ham = _lib.HAMILTONIANS[self.ham]
        p.datum = _lib.DATUMS[self.datum]
        if len(self.ham_p) > 8 or len(self.datum_p) > 4:
            raise ValueError("at most 8 Hamiltonian and 4 datum parameters")
        hp = list(self.ham_p) + [0.0] * (8 - len(self.ham_p))
        dp = list(self.datum_p) + [0.0] * (4 - len(self.datum_p))
        for i in range(8):
            p.ham_p[i] = float(hp[i])
        for i in range(4):
            p.datum_p[i] = float(dp[i])
        if self.datum_aux is not None:
            _require_cuda(self.datum_aux, "datum_aux")
            p.datum_aux = self.datum_aux.data_ptr()
        else:
            p.datum_aux = None
        p.nu, p.eta, p.c_min, p.c_max = float(self.nu), float(self.eta), float(self.c_min), float(self.c_max)
        p.tilt = int(bool(self.tilt))
        p.sample_mode = _lib.SAMPLE_MODES[self.sample_mode]
        p.sample_bf16 = int(bool(self.sample_bf16))
        p.grad_cv = int(bool(self.grad_cv))
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        p.problem_id = int(self.problem_id)
        p.tube = int(bool(self.tube))
        return p


def _require_cuda(t: torch.Tensor, name: str, dtype=torch.float32):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream or None


class Context:
    """An hjg_ctx on one device (workspace, draw-table cache, recorded graphs)."""

    def __init__(self, device: int = 0):
        L = _lib.lib()
        h = C.c_void_p()
        check(L.hjg_ctx_create(int(device), C.byref(h)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def set_timing(self, enable: bool):
        """Bracket every pair-loop kernel launch with HIP events."""
        check(_lib.lib().hjg_set_timing(self._h, int(bool(enable))))

    def sweep_time(self):
        """(total ms, launches) of the pair-loop kernels of the last call; waits for it."""
        ms, n = C.c_double(0.0), C.c_int32(0)
        check(_lib.lib().hjg_sweep_time(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def save_tuning(self, path: str):
        check(_lib.lib().hjg_tuning_save(self._h, str(path).encode()))

    def load_tuning(self, path: str):
        check(_lib.lib().hjg_tuning_load(self._h, str(path).encode()))

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().hjg_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def philox_words(seed: int, c1: int, c2: int, c3: int, G: int, device="cuda", stream=None) -> np.ndarray:
    """Raw Philox4x32-10 words for counters (g, c1, c2, c3), g < G, as uint32 [G, 4]."""
    out = torch.empty(4 * G, dtype=torch.int32, device=device)
    check(_lib.lib().hjg_philox4x32_10(int(seed) & (2 ** 64 - 1), c1, c2, c3, G, _ptr(out), _stream(stream)))
    return out.cpu().numpy().view(np.uint32).reshape(G, 4)


def sample_table(ctx: Context, spec: ProblemSpec, N: int, time_step: int = 0, stream=None) -> torch.Tensor:
    """The common draw table z[n][N]: float32, or bfloat16 when spec.sample_bf16."""
    dtype = torch.bfloat16 if spec.sample_bf16 else torch.float32
    out = torch.empty((spec.n, N), dtype=dtype, device=f"cuda:{ctx.device}")
    p = spec.to_c()
    check(_lib.lib().hjg_sample_table(ctx.handle, C.byref(p), int(N), int(time_step), _ptr(out), _stream(stream)))
    return out


def value_grad(ctx: Context, spec: ProblemSpec, x: torch.Tensor, t: float, N: int, c: torch.Tensor,
               theta: Optional[torch.Tensor] = None, time_step: int = 0, iteration: int = 0,
               check_finite: bool = False, out=None, stream=None):
    """One frozen-coefficient sweep; returns (v [Q], grad [n][Q], ess [Q])."""
    _require_cuda(x, "x")
    n, Q = x.shape
    if n != spec.n:
        raise ValueError("x must have shape [n, Q]")
    _require_cuda(c, "c")
    if theta is not None:
        _require_cuda(theta, "theta")
    if out is None:
        v = torch.empty(Q, dtype=torch.float32, device=x.device)
        grad = torch.empty((n, Q), dtype=torch.float32, device=x.device)
        ess = torch.empty(Q, dtype=torch.float32, device=x.device)
    else:
        v, grad, ess = out
    p = spec.to_c()
    check(_lib.lib().hjg_value_grad(ctx.handle, C.byref(p), Q, _ptr(x), float(t), int(N), int(time_step),
                                    int(iteration), _ptr(c), _ptr(theta), _ptr(v), _ptr(grad), _ptr(ess),
                                    int(bool(check_finite)), _stream(stream)))
    return v, grad, ess


def value_grad_noalloc(ctx: Context, spec: ProblemSpec, x: torch.Tensor, t: float, N: int, c: torch.Tensor,
                       theta: Optional[torch.Tensor] = None, time_step: int = 0, iteration: int = 0, out=None,
                       stream=None):
    """hjg_value_grad_noalloc: the sweep of value_grad with its scratch in the
    library's fixed per-GPU array (the C call allocates nothing and does not
    synchronise).  Pass out = (v, grad, ess) to allocate nothing here either."""
    _require_cuda(x, "x")
    n, Q = x.shape
    if n != spec.n:
        raise ValueError("x must have shape [n, Q]")
    _require_cuda(c, "c")
    if theta is not None:
        _require_cuda(theta, "theta")
    if out is None:
        v = torch.empty(Q, dtype=torch.float32, device=x.device)
        grad = torch.empty((n, Q), dtype=torch.float32, device=x.device)
        ess = torch.empty(Q, dtype=torch.float32, device=x.device)
    else:
        v, grad, ess = out
    p = spec.to_c()
    check(_lib.lib().hjg_value_grad_noalloc(ctx.handle, C.byref(p), Q, _ptr(x), float(t), int(N), int(time_step),
                                            int(iteration), _ptr(c), _ptr(theta), _ptr(v), _ptr(grad), _ptr(ess),
                                            _stream(stream)))
    return v, grad, ess


@dataclass
class PicardOut:
    v: torch.Tensor
    grad: torch.Tensor
    c: torch.Tensor
    ess: torch.Tensor
    flags: torch.Tensor
    resid_hist: np.ndarray
    iters_done: int
    status: int


def picard_sweep(ctx: Context, spec: ProblemSpec, x: torch.Tensor, t: float, N: int, K: int, tol: float = 0.0,
                 time_step: int = 0, p0: Optional[torch.Tensor] = None, v0: Optional[torch.Tensor] = None,
                 host_outputs: bool = True, out: Optional[PicardOut] = None, stream=None) -> PicardOut:
    """Algorithm 1 at the states x [n][Q]; see hjg_picard_sweep."""
    _require_cuda(x, "x")
    n, Q = x.shape
    if n != spec.n:
        raise ValueError("x must have shape [n, Q]")
    if p0 is not None:
        _require_cuda(p0, "p0")
    if v0 is not None:
        _require_cuda(v0, "v0")
    dev = x.device
    if out is None:
        out = PicardOut(torch.empty(Q, dtype=torch.float32, device=dev),
                        torch.empty((n, Q), dtype=torch.float32, device=dev),
                        torch.empty(Q, dtype=torch.float32, device=dev),
                        torch.empty(Q, dtype=torch.float32, device=dev),
                        torch.empty(Q, dtype=torch.uint8, device=dev),
                        np.zeros(K), 0, 0)
    hist = (C.c_double * K)() if host_outputs else None
    iters = C.c_int32(0)
    p = spec.to_c()
    code = _lib.lib().hjg_picard_sweep(ctx.handle, C.byref(p), Q, _ptr(x), float(t), int(N), int(K), float(tol),
                                       int(time_step), _ptr(p0), _ptr(v0), _ptr(out.v), _ptr(out.grad), _ptr(out.c),
                                       _ptr(out.ess), _ptr(out.flags), hist,
                                       C.byref(iters) if host_outputs else None, _stream(stream))
    check(code, allow=(_lib.HJG_OK, _lib.HJG_ENOTCONVERGED))
    out.status = code
    if host_outputs:
        out.resid_hist = np.array(list(hist))
        out.iters_done = int(iters.value)
    return out


# ------------------------------------------------------------------- batched
@dataclass
class BatchOut:
    v: torch.Tensor           # [sum Q]
    grad: torch.Tensor        # concatenated [n_p][Q_p] blocks
    resid_hist: np.ndarray    # [P][max K]
    iters: np.ndarray         # [P]
    q_off: np.ndarray         # [P+1]
    x_off: np.ndarray         # [P+1] element offsets of the [n_p][Q_p] blocks


def picard_sweep_batched(ctx: Context, specs, xs, N, K, t, tol: float = 0.0, host_outputs: bool = True,
                         x_all: Optional[torch.Tensor] = None, out: Optional[BatchOut] = None, stream=None):
    """Algorithm 1 for several problems in one call (hjg_picard_sweep_batched).

    specs: list of ProblemSpec; xs: list of [n_p][Q_p] CUDA tensors (or x_all
    with the concatenated blocks); N, K, t: per-problem sequences.
    """
    P = len(specs)
    if x_all is None:
        for i, x in enumerate(xs):
            _require_cuda(x, f"xs[{i}]")
            if x.shape[0] != specs[i].n:
                raise ValueError(f"xs[{i}] must have shape [n, Q]")
        x_all = torch.cat([x.reshape(-1) for x in xs]).contiguous()
        Qs = [x.shape[1] for x in xs]
    else:
        _require_cuda(x_all, "x_all")
        Qs = [x.shape[1] if hasattr(x, "shape") else int(x) for x in xs]
    q_off = np.zeros(P + 1, dtype=np.int64)
    q_off[1:] = np.cumsum(Qs)
    x_off = np.zeros(P + 1, dtype=np.int64)
    x_off[1:] = np.cumsum([s.n * q for s, q in zip(specs, Qs)])
    if out is None:
        out = BatchOut(torch.empty(int(q_off[-1]), dtype=torch.float32, device=x_all.device),
                       torch.empty(int(x_off[-1]), dtype=torch.float32, device=x_all.device),
                       np.zeros((P, max(K))), np.zeros(P, dtype=np.int32), q_off, x_off)
    probs = (_lib.Problem * P)(*[s.to_c() for s in specs])
    qo = (C.c_int64 * (P + 1))(*q_off.tolist())
    Na = (C.c_int32 * P)(*[int(v) for v in N])
    Ka = (C.c_int32 * P)(*[int(v) for v in K])
    ta = (C.c_double * P)(*[float(v) for v in t])
    hist = (C.c_double * (P * max(K)))() if host_outputs else None
    it = (C.c_int32 * P)() if host_outputs else None
    check(_lib.lib().hjg_picard_sweep_batched(ctx.handle, P, probs, qo, Na, Ka, ta, float(tol), _ptr(x_all),
                                              _ptr(out.v), _ptr(out.grad), hist, it, _stream(stream)))
    if host_outputs:
        out.resid_hist = np.array(list(hist)).reshape(P, max(K))
        out.iters = np.array(list(it), dtype=np.int32)
    return out


def knn_grid(ctx: Context, pos: torch.Tensor, box_lo, box_hi, cell: float, k: int = 7, want_idx: bool = True,
             stream=None):
    """k nearest other agents of each agent via the hash grid.

    pos: device float32 [3, M].  Returns (idx [k, M] int32 or None,
    nbr [k, 3, M] float32) -- nbr is the datum_aux of the knn_balls datum.
    """
    _require_cuda(pos, "pos")
    if pos.dim() != 2 or pos.shape[0] != 3:
        raise ValueError("pos must have shape [3, M]")
    M = pos.shape[1]
    idx = torch.empty((k, M), dtype=torch.int32, device=pos.device) if want_idx else None
    nbr = torch.empty((k, 3, M), dtype=torch.float32, device=pos.device)
    lo = (C.c_float * 3)(*[float(v) for v in box_lo])
    hi = (C.c_float * 3)(*[float(v) for v in box_hi])
    check(_lib.lib().hjg_knn_grid(ctx.handle, M, _ptr(pos), lo, hi, float(cell), int(k), _ptr(idx), _ptr(nbr),
                                  _stream(stream)))
    return idx, nbr


def autotune_sweep(ctx: Context, spec: ProblemSpec, x: torch.Tensor, t: float, N: int, c: torch.Tensor,
                   theta: Optional[torch.Tensor] = None, stream=None):
    """Tune the sample-split target of this sweep's bucket; returns (blocks, ms)."""
    _require_cuda(x, "x")
    _require_cuda(c, "c")
    n, Q = x.shape
    b, ms = C.c_int32(0), C.c_double(0.0)
    p = spec.to_c()
    check(_lib.lib().hjg_autotune_sweep(ctx.handle, C.byref(p), Q, _ptr(x), float(t), int(N), _ptr(c),
                                        _ptr(theta), C.byref(b), C.byref(ms), _stream(stream)))
    return int(b.value), float(ms.value)


def probe_valu_rate(waves_per_simd: int, iters: int = 20000, form: int = 0, stream=None):
    """Issue rate of independent unpacked float32 operations at waves_per_simd
    resident waves per SIMD (form 0: FMA with a scalar operand, 1: accumulating
    FMA, 2: multiply, ... 7: forms 0 and 1 on alternate chains, 8-10: fixed
    sequences with different dependences; include/hjg.h lists all thirteen): (wave-level VALU instructions per compute-unit clock,
    shader clock in GHz).  A measurement helper for the vector-ALU roofline."""
    r, g = C.c_double(0.0), C.c_double(0.0)
    check(_lib.lib().hjg_probe_valu_rate(int(waves_per_simd), int(iters), int(form), C.byref(r), C.byref(g),
                                         _stream(stream)))
    return r.value, g.value


def autotune_batched(ctx: Context, specs, xs, N, K, t, tol: float = 0.0, stream=None):
    """Tune the samples per split of the batched sweep on this batch; returns (split, ms)."""
    P = len(specs)
    x_all = torch.cat([x.reshape(-1) for x in xs]).contiguous()
    Qs = [x.shape[1] for x in xs]
    q_off = np.zeros(P + 1, dtype=np.int64)
    q_off[1:] = np.cumsum(Qs)
    nx = sum(s.n * q for s, q in zip(specs, Qs))
    v = torch.empty(int(q_off[-1]), dtype=torch.float32, device=x_all.device)
    g = torch.empty(nx, dtype=torch.float32, device=x_all.device)
    probs = (_lib.Problem * P)(*[s.to_c() for s in specs])
    qo = (C.c_int64 * (P + 1))(*q_off.tolist())
    Na = (C.c_int32 * P)(*[int(v) for v in N])
    Ka = (C.c_int32 * P)(*[int(v) for v in K])
    ta = (C.c_double * P)(*[float(v) for v in t])
    b, ms = C.c_int32(0), C.c_double(0.0)
    check(_lib.lib().hjg_autotune_batched(ctx.handle, P, probs, qo, Na, Ka, ta, float(tol), _ptr(x_all), _ptr(v),
                                          _ptr(g), C.byref(b), C.byref(ms), _stream(stream)))
    return int(b.value), float(ms.value)


# ----------------------------------------------------------------- surrogate
@dataclass
class TrainConfig:
    """Training settings (struct hjg_train_cfg)."""
    epochs: int = 20
    batch: int = 4096
    lr: float = 1e-3
    lr_min: float = 1e-5
    weight_decay: float = 1e-4
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    grad_weight: float = 1.0
    seed: int = 0

    def to_c(self) -> _lib.TrainCfg:
        c = _lib.TrainCfg()
        c.epochs, c.batch = int(self.epochs), int(self.batch)
        c.lr, c.lr_min, c.weight_decay = float(self.lr), float(self.lr_min), float(self.weight_decay)
        c.beta1, c.beta2, c.eps = float(self.beta1), float(self.beta2), float(self.eps)
        c.grad_weight, c.seed = float(self.grad_weight), int(self.seed) & 0xFFFFFFFFFFFFFFFF
        return c


def _host_f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


class Surrogate:
    """The library's surrogate network (x, t) -> (v, Dv) on the context's device."""

    def __init__(self, ctx: Context, n: int, width: int = 256, depth: int = 4, seed: int = 0):
        h = C.c_void_p()
        check(_lib.lib().hjg_surrogate_create(ctx.handle, int(n), int(width), int(depth),
                                              int(seed) & 0xFFFFFFFFFFFFFFFF, C.byref(h)))
        self._h, self.n, self.width, self.depth, self.ctx = h, n, width, depth, ctx

    @property
    def handle(self):
        return self._h

    def save(self, path: str):
        """Write shape, parameters and normalisation to a file (hjg_surrogate_save)."""
        check(_lib.lib().hjg_surrogate_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, ctx: Context, path: str) -> "Surrogate":
        """A surrogate from a file written by save (hjg_surrogate_load)."""
        h = C.c_void_p()
        check(_lib.lib().hjg_surrogate_load(ctx.handle, os.fsencode(path), C.byref(h)))
        obj = cls.__new__(cls)
        obj._h, obj.ctx = h, ctx
        with open(path, "rb") as f:
            hdr = np.frombuffer(f.read(24)[8:24], dtype=np.int32)
        obj.n, obj.width, obj.depth = int(hdr[0]), int(hdr[1]), int(hdr[2])
        return obj

    def param_count(self) -> int:
        c = C.c_int64(0)
        check(_lib.lib().hjg_surrogate_param_count(self._h, C.byref(c)))
        return int(c.value)

    def set_params(self, params, norm):
        p, nm = _host_f32(params), _host_f32(norm)
        if p.size != self.param_count() or nm.shape != (4, self.n + 1):
            raise ValueError("params or norm has the wrong size")
        check(_lib.lib().hjg_surrogate_set_params(self._h, p.ctypes.data, nm.ctypes.data))

    def get_params(self):
        p = np.zeros(self.param_count(), dtype=np.float32)
        nm = np.zeros((4, self.n + 1), dtype=np.float32)
        check(_lib.lib().hjg_surrogate_get_params(self._h, p.ctypes.data, nm.ctypes.data))
        return p, nm

    def predict(self, x: torch.Tensor, t, stream=None):
        _require_cuda(x, "x")
        n, Q = x.shape
        tq = t if isinstance(t, torch.Tensor) else torch.full((Q,), float(t), dtype=torch.float32, device=x.device)
        _require_cuda(tq, "t")
        v = torch.empty(Q, dtype=torch.float32, device=x.device)
        g = torch.empty((n, Q), dtype=torch.float32, device=x.device)
        check(_lib.lib().hjg_surrogate_predict(self._h, Q, _ptr(x), _ptr(tq), _ptr(v), _ptr(g), _stream(stream)))
        return v, g

    def loss_grad(self, x, t, v, grad, grad_weight: float = 1.0, stream=None):
        for name, a in (("x", x), ("t", t), ("v", v), ("grad", grad)):
            _require_cuda(a, name)
        B = x.shape[1]
        loss = C.c_double(0.0)
        g = np.zeros(self.param_count(), dtype=np.float32)
        check(_lib.lib().hjg_surrogate_loss_grad(self._h, B, _ptr(x), _ptr(t), _ptr(v), _ptr(grad),
                                                 float(grad_weight), C.byref(loss), g.ctypes.data, _stream(stream)))
        return loss.value, g

    def train(self, x, t, v, grad, cfg: TrainConfig = TrainConfig(), stream=None) -> np.ndarray:
        for name, a in (("x", x), ("t", t), ("v", v), ("grad", grad)):
            _require_cuda(a, name)
        M = x.shape[1]
        hist = np.zeros(cfg.epochs, dtype=np.float64)
        c = cfg.to_c()
        check(_lib.lib().hjg_surrogate_train(self._h, M, _ptr(x), _ptr(t), _ptr(v), _ptr(grad), C.byref(c),
                                             hist.ctypes.data, _stream(stream)))
        return hist

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().hjg_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def surrogate_sweep(ctx: Context, sur: Surrogate, spec: ProblemSpec, x: torch.Tensor, t: float, N_s: int, K_s: int,
                    N_fb: int, K_fb: int, tol: float = 1e-3, time_step: int = 0, stream=None):
    """Surrogate-accelerated sweep; returns (v, grad, fell_back, n_fallback)."""
    _require_cuda(x, "x")
    n, Q = x.shape
    v = torch.empty(Q, dtype=torch.float32, device=x.device)
    g = torch.empty((n, Q), dtype=torch.float32, device=x.device)
    fb = torch.empty(Q, dtype=torch.uint8, device=x.device)
    nfb = C.c_int64(0)
    p = spec.to_c()
    check(_lib.lib().hjg_surrogate_sweep(ctx.handle, sur.handle, C.byref(p), Q, _ptr(x), float(t), int(N_s),
                                         int(K_s), int(N_fb), int(K_fb), float(tol), int(time_step), _ptr(v),
                                         _ptr(g), _ptr(fb), C.byref(nfb), _stream(stream)))
    return v, g, fb, int(nfb.value)


def surrogate_tube_step(ctx: Context, sur: Surrogate, spec: ProblemSpec, x: torch.Tensor, t_prev: float, dt: float,
                        N: int, K: int, tol: float = 0.0, time_step: int = 0, stream=None) -> PicardOut:
    """One time-marching step with the surrogate as the datum (hjg_surrogate_tube_step):
    the value at t_prev + dt from v_S(., t_prev).  Returns a PicardOut (flags unused)."""
    _require_cuda(x, "x")
    n, Q = x.shape
    if n != spec.n:
        raise ValueError("x must have shape [n, Q]")
    dev = x.device
    out = PicardOut(torch.empty(Q, dtype=torch.float32, device=dev), torch.empty((n, Q), dtype=torch.float32, device=dev),
                    torch.empty(Q, dtype=torch.float32, device=dev), torch.empty(Q, dtype=torch.float32, device=dev),
                    torch.zeros(Q, dtype=torch.uint8, device=dev), np.zeros(K), 0, 0)
    hist = (C.c_double * K)()
    iters = C.c_int32(0)
    p = spec.to_c()
    check(_lib.lib().hjg_surrogate_tube_step(ctx.handle, sur.handle, C.byref(p), Q, _ptr(x), float(t_prev), float(dt),
                                             int(N), int(K), float(tol), int(time_step), _ptr(out.v), _ptr(out.grad),
                                             _ptr(out.c), _ptr(out.ess), hist, C.byref(iters), _stream(stream)))
    out.resid_hist = np.array(list(hist))
    out.iters_done = int(iters.value)
    return out


# ------------------------------------------------------------- certification
def error_budget(C1: float, rho: float, K: int, C2: float, N: int, delta_p: float, eps_ql: float = 0.0,
                 C3: float = 0.0, delta: float = 0.0) -> float:
    """E = C1 rho^K + C2 sqrt(log(1/delta_p)/N) + eps_ql + C3 sqrt(delta) (hjg_error_budget)."""
    b = _lib.Budget(C1=C1, rho=rho, K=K, C2=C2, N=N, delta_p=delta_p, eps_ql=eps_ql, C3=C3, delta=delta)
    E = C.c_double(0.0)
    check(_lib.lib().hjg_error_budget(C.byref(b), C.byref(E)))
    return float(E.value)


def mc_margin(v: torch.Tensor, c: torch.Tensor, N: int, delta_p: float, g_min: float, g_max: float = float("inf"),
              ess: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Per-state sampling margin: the concentration theorem (Hoeffding), or with
    ess the empirical Bernstein form (hjg_mc_margin)."""
    _require_cuda(v, "v")
    _require_cuda(c, "c")
    if ess is not None:
        _require_cuda(ess, "ess")
    out = torch.empty_like(v)
    check(_lib.lib().hjg_mc_margin(v.numel(), _ptr(v), _ptr(c), _ptr(ess), int(N), float(delta_p), float(g_min),
                                   float(g_max), _ptr(out), _stream(stream)))
    return out


def certify(v: torch.Tensor, E: float = 0.0, margin: Optional[torch.Tensor] = None, stream=None):
    """Labels (+1 SAFE, -1 UNSAFE, 0 UNDETERMINED) and the counts (unsafe, undetermined, safe)."""
    _require_cuda(v, "v")
    if margin is not None:
        _require_cuda(margin, "margin")
    label = torch.empty(v.numel(), dtype=torch.int8, device=v.device)
    counts = torch.empty(3, dtype=torch.int64, device=v.device)
    check(_lib.lib().hjg_certify(v.numel(), _ptr(v), _ptr(margin), float(E), _ptr(label), _ptr(counts),
                                 _stream(stream)))
    return label, counts


# ------------------------------------------------------------------ reach-avoid
def avoid_project(obstacle: ProblemSpec, x: torch.Tensor, v: torch.Tensor, grad: Optional[torch.Tensor] = None,
                  want_active: bool = False, stream=None) -> Optional[torch.Tensor]:
    """Obstacle projection of the reach-avoid tube, in place: v <- max(v, -l_A(x)) and grad <- -D l_A(x) where
    the obstacle wins; l_A is the datum of `obstacle` (only n and its datum fields are used).  x [n, Q], v [Q],
    grad [n, Q] float32 device tensors.  Returns the uint8 flags of the replaced states when asked."""
    _require_cuda(x, "x")
    _require_cuda(v, "v")
    if grad is not None:
        _require_cuda(grad, "grad")
        if grad.shape != x.shape:
            raise ValueError("grad must have the shape of x")
    if x.dim() != 2 or x.shape[0] != obstacle.n or v.numel() != x.shape[1]:
        raise ValueError("need x [n, Q] and v [Q] with n = obstacle.n")
    active = torch.empty(v.numel(), dtype=torch.uint8, device=v.device) if want_active else None
    p = obstacle.to_c()
    check(_lib.lib().hjg_avoid_project(C.byref(p), v.numel(), _ptr(x), _ptr(v), _ptr(grad), _ptr(active),
                                       _stream(stream)))
    return active


# ------------------------------------------------------------------ topology
def topology(v: torch.Tensor, stream=None):
    """Markers of {v <= 0} on slices v [B, ny, nx] (or [ny, nx]): (n_comp, beta1, chi) int32 tensors [B]."""
    _require_cuda(v, "v")
    if v.dim() == 2:
        v = v.unsqueeze(0)
    B, ny, nx = v.shape
    out = [torch.empty(B, dtype=torch.int32, device=v.device) for _ in range(3)]
    check(_lib.lib().hjg_topology(B, ny, nx, _ptr(v), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _stream(stream)))
    return tuple(out)


def topology_events(chi, beta1, n_comp) -> np.ndarray:
    """Event bits per step (1 vacuole nucleation, 2 cordon formation, 4 fragmentation)."""
    chi, beta1, n_comp = (np.ascontiguousarray(np.asarray(a, dtype=np.int32)) for a in (chi, beta1, n_comp))
    T = len(chi)
    ev = np.zeros(T, dtype=np.int32)
    check(_lib.lib().hjg_topology_events(T, chi.ctypes.data, beta1.ctypes.data, n_comp.ctypes.data,
                                         ev.ctypes.data))
    return ev


def isocontour(v: torch.Tensor, level: float = 0.0, max_seg: Optional[int] = None, stream=None):
    """Marching-squares segments of v = level on slices v [B, ny, nx] (or [ny, nx]):
    (seg [S, 4] as (x0, y0, x1, y1) in grid units, slice [S]); grows the buffer and
    repeats if more than max_seg were found."""
    _require_cuda(v, "v")
    if v.dim() == 2:
        v = v.unsqueeze(0)
    B, ny, nx = v.shape
    cap = int(max_seg) if max_seg is not None else max(1024, 4 * B * (ny + nx))
    count = torch.zeros(1, dtype=torch.int64, device=v.device)
    while True:
        seg = torch.empty((cap, 4), dtype=torch.float32, device=v.device)
        sl = torch.empty(cap, dtype=torch.int32, device=v.device)
        check(_lib.lib().hjg_isocontour(B, ny, nx, _ptr(v), float(level), _ptr(seg), _ptr(sl), cap, _ptr(count),
                                        _stream(stream)))
        n = int(count.item())
        if n <= cap:
            return seg[:n], sl[:n]
        cap = n


def smooth_slices(v: torch.Tensor, sigma: float, stream=None) -> torch.Tensor:
    """Gaussian smoothing (sigma in cells) of slices v [B, ny, nx] (or [ny, nx])."""
    _require_cuda(v, "v")
    squeeze = v.dim() == 2
    if squeeze:
        v = v.unsqueeze(0)
    B, ny, nx = v.shape
    out = torch.empty_like(v)
    check(_lib.lib().hjg_smooth_slices(B, ny, nx, _ptr(v), float(sigma), _ptr(out), _stream(stream)))
    return out[0] if squeeze else out
