"""Thin Python binding of libqtthom.so (argument marshalling only).

Every computation runs in the HIP library; this module only moves cores
between numpy and PyTorch device tensors, fills the C descriptors and calls the
C ABI declared in include/qtthom.h.  There is no CPU fallback: loading fails
loudly when the library or a GPU is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqtthom.so")

QT_OK, QT_NOT_CONVERGED = 0, 1
ROUND_SVD, ROUND_SKETCH, ROUND_LEARNED, ROUND_POLAR = 0, 1, 2, 3
PREC_F64, PREC_F32 = 0, 1

EXPORTS = ["qt_ctx_create", "qt_ctx_destroy", "qt_last_error", "qt_ctx_sync",
           "qt_ctx_counters", "qt_ctx_profile", "qt_ctx_profile_read", "qt_ctx_autotune",
           "tt_hadamard",
           "tt_mpo_apply", "tt_add", "tt_round", "tt_round_noalloc", "tt_dot", "tt_sketch_round", "tt_sandwich", "tt_amen_mv",
           "ls_iterate", "homogenize", "qt_mlp_num_params", "qt_mlp_train_step", "qt_mlp_infer",
           "qt_ranklog_enable", "qt_ranklog_get", "qt_set_predictor", "qt_learn_reset",
           "qt_learn_log_enable", "qt_learn_log_get", "qt_ctx_fixed_bytes",
           "qt_ctx_create_with_memory", "qt_workspace_query", "qt_ls_workspace_query"]


class QtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"qtthom status {status}: {msg}")
        self.status = status


class TTDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("batch", C.c_int32), ("modes", C.POINTER(C.c_int32)),
                ("cap", C.POINTER(C.c_int32)), ("offsets", C.POINTER(C.c_int64)),
                ("inst_stride", C.c_int64), ("ranks", C.c_void_p), ("data", C.c_void_p)]


class MPODesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("modes_out", C.POINTER(C.c_int32)),
                ("modes_in", C.POINTER(C.c_int32)), ("ranks", C.POINTER(C.c_int32)),
                ("diag", C.POINTER(C.c_int32)), ("offsets", C.POINTER(C.c_int64)),
                ("data", C.c_void_p), ("inst_stride", C.c_int64), ("inst_group", C.c_int32)]


class RoundOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_rank", C.c_int32), ("mode", C.c_int32),
                ("jacobi_max_sweeps", C.c_int32), ("precision", C.c_int32),
                ("oversample", C.c_int32), ("seed", C.c_uint64)]


class Operands(C.Structure):
    _fields_ = [("L", C.c_int32), ("kp", TTDesc), ("Kp", MPODesc), ("K2", MPODesc),
                ("k0", C.c_double), ("S", MPODesc), ("Sinv", MPODesc), ("G", MPODesc),
                ("E", TTDesc), ("E_norm", C.POINTER(C.c_double)), ("SE", TTDesc),
                ("G2", MPODesc)]


class SolveOpts(C.Structure):
    _fields_ = [("round", RoundOpts), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("graph", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libqtthom.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: run __graft_entry__.build() first")
    lib = C.CDLL(path)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    lib.qt_ctx_create.argtypes = [C.c_int, vp, C.c_size_t, C.POINTER(vp)]
    lib.qt_ctx_destroy.argtypes = [vp]
    lib.qt_ctx_destroy.restype = None
    lib.qt_last_error.restype = C.c_char_p
    lib.qt_ctx_sync.argtypes = [vp]
    lib.qt_ctx_counters.argtypes = [vp, C.POINTER(C.c_int64), i32, i32]
    lib.qt_ctx_profile.argtypes = [vp, i32]
    lib.qt_ctx_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.qt_ctx_autotune.argtypes = [vp, i32, C.POINTER(C.c_int32)]
    lib.tt_hadamard.argtypes = [vp, C.POINTER(TTDesc), C.POINTER(TTDesc), C.POINTER(TTDesc)]
    lib.tt_mpo_apply.argtypes = [vp, C.POINTER(MPODesc), C.POINTER(TTDesc), C.POINTER(TTDesc)]
    lib.tt_add.argtypes = [vp, dbl, dbl, C.POINTER(TTDesc), dbl, dbl, C.POINTER(TTDesc),
                           C.POINTER(TTDesc)]
    lib.tt_round.argtypes = [vp, C.POINTER(TTDesc), C.POINTER(RoundOpts), vp, vp]
    lib.tt_round_noalloc.argtypes = [vp, C.POINTER(TTDesc), C.POINTER(RoundOpts), vp, vp]
    lib.tt_dot.argtypes = [vp, C.POINTER(TTDesc), C.POINTER(TTDesc), vp]
    lib.tt_sketch_round.argtypes = [vp, C.POINTER(MPODesc), C.POINTER(TTDesc), C.POINTER(TTDesc),
                                    C.POINTER(RoundOpts), vp, C.POINTER(TTDesc), vp, vp]
    lib.tt_sandwich.argtypes = [vp, C.POINTER(MPODesc), C.POINTER(TTDesc), dbl, vp]
    lib.tt_amen_mv.argtypes = [vp, C.POINTER(MPODesc), C.POINTER(TTDesc), C.POINTER(TTDesc),
                               C.POINTER(TTDesc), dbl, i32, i32, vp]
    lib.ls_iterate.argtypes = [vp, C.POINTER(Operands), C.POINTER(TTDesc), C.POINTER(SolveOpts),
                               i32, vp]
    lib.homogenize.argtypes = [vp, C.POINTER(Operands), C.POINTER(TTDesc), C.POINTER(TTDesc),
                               C.POINTER(SolveOpts), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                               C.POINTER(C.c_double)]
    lib.qt_mlp_num_params.argtypes = [i32, i32]
    f32 = C.c_float
    lib.qt_mlp_train_step.argtypes = [vp, vp, vp, vp, i32, vp, vp, i32, i32, i32, f32, f32, f32,
                                      vp, vp]
    lib.qt_mlp_infer.argtypes = [vp, vp, vp, i32, i32, i32, f32, vp, vp, vp]
    lib.qt_ranklog_enable.argtypes = [vp, i32, i32]
    lib.qt_ranklog_get.argtypes = [vp, vp, vp, i32, C.POINTER(C.c_int32)]
    lib.qt_set_predictor.argtypes = [vp, vp, i32, f32, f32]
    lib.qt_learn_reset.argtypes = [vp]
    lib.qt_learn_log_enable.argtypes = [vp, i32]
    lib.qt_learn_log_get.argtypes = [vp, vp, i32, C.POINTER(C.c_int32)]
    lib.qt_ctx_fixed_bytes.argtypes = []
    lib.qt_ctx_create_with_memory.argtypes = [C.c_int, vp, vp, C.c_size_t, C.POINTER(vp)]
    lib.qt_workspace_query.argtypes = [C.POINTER(TTDesc), C.POINTER(RoundOpts),
                                       C.POINTER(C.c_size_t)]
    lib.qt_ls_workspace_query.argtypes = [C.POINTER(Operands), C.POINTER(TTDesc),
                                          C.POINTER(TTDesc), C.POINTER(SolveOpts),
                                          C.POINTER(C.c_size_t)]
    for name in EXPORTS:
        if name not in ("qt_ctx_destroy", "qt_last_error", "qt_ctx_fixed_bytes"):
            getattr(lib, name).restype = C.c_int32
    lib.qt_ctx_fixed_bytes.restype = C.c_size_t
    _lib = lib
    return lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("qtthom needs a HIP device (torch.cuda.is_available() is False)")
    return torch


def _check(status):
    if status < 0:
        raise QtError(status, load_library().qt_last_error().decode())
    return status


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _i64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _p32(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _p64(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


class Context:
    """A library context bound to torch's current stream on `device`."""

    def __init__(self, device: int = 0, ws_bytes: int = 0, memory=None):
        """memory: optional caller-owned device block (a uint8 torch tensor on
        `device`, 256-byte aligned) holding all of the context's device state
        (qt_ctx_create_with_memory); the context keeps a reference to it."""
        torch = _torch()
        self.lib = load_library()
        self.device = device
        torch.cuda.set_device(device)
        self.stream = torch.cuda.current_stream(device)
        h = C.c_void_p()
        self.memory = memory
        if memory is None:
            _check(self.lib.qt_ctx_create(device, C.c_void_p(self.stream.cuda_stream), ws_bytes,
                                          C.byref(h)))
        else:
            nbytes = memory.numel() * memory.element_size()
            _check(self.lib.qt_ctx_create_with_memory(
                device, C.c_void_p(self.stream.cuda_stream), C.c_void_p(memory.data_ptr()),
                nbytes, C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.qt_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(self.lib.qt_ctx_sync(self.h))

    def counters(self, reset: bool = False) -> dict:
        """Device event counters (see qt_ctx_counters in include/qtthom.h)."""
        out = (C.c_int64 * 8)()
        _check(self.lib.qt_ctx_counters(self.h, out, 8, 1 if reset else 0))
        return {"svd_calls": out[0], "svd_sweeps": out[1], "sketch_over_budget": out[2],
                "learned_fallbacks": out[3], "gemm_flops": out[4], "gemm_bytes": out[5],
                "learned_roundings": out[6]}

    PROF_GEMM, PROF_QR, PROF_SVD = 1, 2, 4

    def profile(self, classes: int):
        """Start live event timing of kernel classes (bit mask; 0 stops)."""
        _check(self.lib.qt_ctx_profile(self.h, classes))

    def autotune(self, mode: int = 1) -> int:
        """GEMM tile-shape mode (0 fixed 64x64, 1 autotune, 2..5 forced shape);
        returns the number of tuned call signatures so far."""
        n = C.c_int32()
        _check(self.lib.qt_ctx_autotune(self.h, mode, C.byref(n)))
        return n.value

    def profile_read(self):
        """(summed kernel time in ms, number of timed launches) since the last read."""
        ms = C.c_double()
        n = C.c_int64()
        _check(self.lib.qt_ctx_profile_read(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value


def natural_caps(modes):
    n = len(modes)
    nat = [1] * (n + 1)
    for k in range(1, n):
        nat[k] = int(min(np.prod(modes[:k], dtype=float), np.prod(modes[k:], dtype=float), 2 ** 30))
    return nat


@dataclass
class DeviceTT:
    """A batch of trains in device memory with fixed rank capacities."""
    modes: np.ndarray
    cap: np.ndarray
    offsets: np.ndarray
    stride: int
    batch: int
    data: object          # torch complex128 tensor [batch * stride]
    ranks: object         # torch int32 tensor [batch, n+1]
    _desc: TTDesc = field(default=None, repr=False)

    @property
    def n(self):
        return len(self.modes)

    @staticmethod
    def empty(modes, cap, batch: int = 1, device: int = 0):
        torch = _torch()
        modes = _i32(modes)
        cap = _i32(cap)
        off = []
        o = 0
        for k in range(len(modes)):
            off.append(o)
            s = int(cap[k]) * int(modes[k]) * int(cap[k + 1])
            o += (s + 31) & ~31
        stride = max(o, 1)
        data = torch.zeros(batch * stride, dtype=torch.complex128, device=f"cuda:{device}")
        ranks = torch.ones((batch, len(modes) + 1), dtype=torch.int32, device=f"cuda:{device}")
        return DeviceTT(modes, cap, _i64(off), stride, batch, data, ranks)

    @staticmethod
    def from_cores(cores_list, cap=None, device: int = 0):
        """cores_list: one list of cores per instance (all with equal modes)."""
        torch = _torch()
        if cores_list and not isinstance(cores_list[0], (list, tuple)):
            cores_list = [cores_list]
        modes = [c.shape[1] for c in cores_list[0]]
        n = len(modes)
        rk = np.array([[c.shape[0] for c in cs] + [1] for cs in cores_list], dtype=np.int32)
        if cap is None:
            cap = rk.max(axis=0)
        cap = _i32(cap)
        if np.any(rk > cap[None, :]):
            raise ValueError("ranks exceed capacities")
        t = DeviceTT.empty(modes, cap, len(cores_list), device)
        host = np.zeros(t.batch * t.stride, dtype=np.complex128)
        for b, cs in enumerate(cores_list):
            for k, c in enumerate(cs):
                o = b * t.stride + int(t.offsets[k])
                host[o:o + c.size] = np.ascontiguousarray(c, dtype=np.complex128).reshape(-1)
        t.data.copy_(torch.from_numpy(host))
        t.ranks.copy_(torch.from_numpy(rk))
        return t

    def desc(self) -> TTDesc:
        d = TTDesc(self.n, self.batch, _p32(self.modes), _p32(self.cap), _p64(self.offsets),
                   self.stride, C.c_void_p(self.ranks.data_ptr()), C.c_void_p(self.data.data_ptr()))
        self._desc = d
        return d

    def rank_array(self):
        return self.ranks.cpu().numpy()

    def to_cores(self):
        rk = self.rank_array()
        host = self.data.cpu().numpy()
        out = []
        for b in range(self.batch):
            cs = []
            for k in range(self.n):
                r0, r1, p = int(rk[b, k]), int(rk[b, k + 1]), int(self.modes[k])
                o = b * self.stride + int(self.offsets[k])
                cs.append(host[o:o + r0 * p * r1].reshape(r0, p, r1).copy())
            out.append(cs)
        return out


@dataclass
class DeviceMPO:
    modes_out: np.ndarray
    modes_in: np.ndarray
    ranks: np.ndarray
    diag: np.ndarray
    offsets: np.ndarray
    data: object
    _desc: MPODesc = field(default=None, repr=False)

    @property
    def n(self):
        return len(self.ranks) - 1

    inst_stride: int = 0
    inst_group: int = 1

    @staticmethod
    def from_cores(cores, diag_flags=None, device: int = 0, inst_group: int = 1):
        """cores: (r, p_out, p_in, r') arrays, or (r, p, r') where diag_flags[k] is set;
        or a list of such lists (one operator instance per microstructure), which
        are zero-padded to common ranks; field b then uses instance b // inst_group."""
        torch = _torch()
        multi = isinstance(cores[0], (list, tuple))
        insts = cores if multi else [cores]
        n = len(insts[0])
        diag_flags = [0] * n if diag_flags is None else [int(d) for d in diag_flags]
        rk = [max(cs[k].shape[0] for cs in insts) for k in range(n)]
        rk.append(max(cs[-1].shape[-1] for cs in insts))
        mo, mi, off, shapes = [], [], [], []
        o = 0
        for k, d in enumerate(diag_flags):
            c = insts[0][k]
            if d:
                mo.append(c.shape[1]); mi.append(c.shape[1])
                shp = (rk[k], c.shape[1], rk[k + 1])
            else:
                mo.append(c.shape[1]); mi.append(c.shape[2])
                shp = (rk[k], c.shape[1], c.shape[2], rk[k + 1])
            shapes.append(shp)
            off.append(o)
            o += (int(np.prod(shp)) + 31) & ~31
        stride = max(o, 1)
        host = np.zeros(stride * len(insts), dtype=np.complex128)
        for i, cs in enumerate(insts):
            for k, (c, s0) in enumerate(zip(cs, off)):
                padded = np.zeros(shapes[k], dtype=np.complex128)
                padded[tuple(slice(0, m) for m in c.shape)] = c
                host[i * stride + s0:i * stride + s0 + padded.size] = padded.reshape(-1)
        data = torch.from_numpy(host).to(f"cuda:{device}")
        return DeviceMPO(_i32(mo), _i32(mi), _i32(rk), _i32(diag_flags), _i64(off), data,
                         inst_stride=stride if multi else 0, inst_group=int(inst_group))

    def desc(self) -> MPODesc:
        d = MPODesc(self.n, _p32(self.modes_out), _p32(self.modes_in), _p32(self.ranks),
                    _p32(self.diag), _p64(self.offsets), C.c_void_p(self.data.data_ptr()),
                    self.inst_stride, self.inst_group)
        self._desc = d
        return d


def round_opts(eps=0.0, max_rank=0, mode=ROUND_SVD, jacobi_max_sweeps=0, precision=PREC_F64,
               oversample=0, seed=0):
    return RoundOpts(eps, max_rank, mode, jacobi_max_sweeps, precision, oversample, seed)


# ------------------------------------------------------------- entry points

def tt_hadamard(ctx: Context, a: DeviceTT, b: DeviceTT, out: DeviceTT = None) -> DeviceTT:
    if out is None:
        out = DeviceTT.empty(b.modes, a.cap * b.cap, b.batch, ctx.device)
    _check(ctx.lib.tt_hadamard(ctx.h, C.byref(a.desc()), C.byref(b.desc()), C.byref(out.desc())))
    return out


def tt_mpo_apply(ctx: Context, A: DeviceMPO, x: DeviceTT, out: DeviceTT = None) -> DeviceTT:
    if out is None:
        out = DeviceTT.empty(A.modes_out, A.ranks * x.cap, x.batch, ctx.device)
    _check(ctx.lib.tt_mpo_apply(ctx.h, C.byref(A.desc()), C.byref(x.desc()), C.byref(out.desc())))
    return out


def tt_add(ctx: Context, alpha, x: DeviceTT, beta, y: DeviceTT, out: DeviceTT = None) -> DeviceTT:
    if out is None:
        cap = x.cap + y.cap
        cap[0] = cap[-1] = 1
        out = DeviceTT.empty(x.modes, cap, x.batch, ctx.device)
    alpha, beta = complex(alpha), complex(beta)
    _check(ctx.lib.tt_add(ctx.h, alpha.real, alpha.imag, C.byref(x.desc()), beta.real, beta.imag,
                          C.byref(y.desc()), C.byref(out.desc())))
    return out


def tt_round(ctx: Context, x: DeviceTT, eps: float, max_rank: int = 0, **kw):
    """In-place rounding; returns (err, norm) as device tensors of shape [batch]."""
    torch = _torch()
    err = torch.zeros(x.batch, dtype=torch.float64, device=x.data.device)
    nrm = torch.zeros(x.batch, dtype=torch.float64, device=x.data.device)
    o = round_opts(eps, max_rank, **kw)
    _check(ctx.lib.tt_round(ctx.h, C.byref(x.desc()), C.byref(o), C.c_void_p(err.data_ptr()),
                            C.c_void_p(nrm.data_ptr())))
    return err, nrm


def ctx_fixed_bytes() -> int:
    """Bytes of the fixed head of a caller-owned context block."""
    return int(load_library().qt_ctx_fixed_bytes())


def workspace_query(x: DeviceTT, eps: float = 0.0, max_rank: int = 0, **kw) -> int:
    """Workspace bytes of tt_round on x with these options (host only)."""
    o = round_opts(eps, max_rank, **kw)
    b = C.c_size_t()
    _check(load_library().qt_workspace_query(C.byref(x.desc()), C.byref(o), C.byref(b)))
    return b.value


def ls_workspace_query(ops: "DeviceOperands", e: DeviceTT, opts: "SolveOpts",
                       homogenize: bool = False) -> int:
    """Workspace bytes of ls_iterate (or homogenize) on this batch (host only)."""
    b = C.c_size_t()
    st = ops.struct()
    ksel = (TTDesc * len(ops.k_sel))(*[t.desc() for t in ops.k_sel]) if homogenize else None
    _check(load_library().qt_ls_workspace_query(C.byref(st), ksel, C.byref(e.desc()),
                                                C.byref(opts), C.byref(b)))
    return b.value


def tt_round_noalloc(ctx: Context, x: DeviceTT, eps: float, err, nrm, max_rank: int = 0, **kw):
    """tt_round with the library's static scratch (no device allocation in the
    call); err and nrm are caller-owned float64 device tensors [batch]."""
    o = round_opts(eps, max_rank, **kw)
    _check(ctx.lib.tt_round_noalloc(ctx.h, C.byref(x.desc()), C.byref(o),
                                    C.c_void_p(err.data_ptr()), C.c_void_p(nrm.data_ptr())))


def tt_dot(ctx: Context, a: DeviceTT, b: DeviceTT):
    """sum conj(a) b per instance, as a complex128 device tensor [batch]."""
    torch = _torch()
    out = torch.zeros(2 * b.batch, dtype=torch.float64, device=b.data.device)
    _check(ctx.lib.tt_dot(ctx.h, C.byref(a.desc()), C.byref(b.desc()), C.c_void_p(out.data_ptr())))
    return torch.view_as_complex(out.view(b.batch, 2))


def tt_sandwich(ctx: Context, Q: DeviceMPO, y: DeviceTT, scale: float = 1.0):
    """scale * Re <y, Q y> per instance (device float64 tensor [batch])."""
    torch = _torch()
    out = torch.zeros(y.batch, dtype=torch.float64, device=y.data.device)
    _check(ctx.lib.tt_sandwich(ctx.h, C.byref(Q.desc()), C.byref(y.desc()), scale,
                               C.c_void_p(out.data_ptr())))
    return out


def tt_sketch_round(ctx: Context, A: DeviceMPO, y: DeviceTT, xnorm2, out: DeviceTT,
                    omega: DeviceTT = None, eps: float = 0.0, max_rank: int = 0,
                    mode: int = ROUND_SKETCH, oversample: int = 8, seed: int = 1,
                    precision: int = PREC_F64):
    """Product-aware rounding of A y into out; returns (err, fail) device tensors [batch]."""
    torch = _torch()
    err = torch.zeros(y.batch, dtype=torch.float64, device=y.data.device)
    fail = torch.zeros(y.batch, dtype=torch.int32, device=y.data.device)
    o = round_opts(eps, max_rank, mode, 0, precision, oversample, seed)
    om = C.byref(omega.desc()) if omega is not None else None
    _check(ctx.lib.tt_sketch_round(ctx.h, C.byref(A.desc()), C.byref(y.desc()), om, C.byref(o),
                                   C.c_void_p(xnorm2.data_ptr()), C.byref(out.desc()),
                                   C.c_void_p(err.data_ptr()), C.c_void_p(fail.data_ptr())))
    return err, fail


def tt_amen_mv(ctx: Context, A: DeviceMPO, x: DeviceTT, y: DeviceTT, z: DeviceTT, eps: float,
               max_rank: int = 0, sweeps: int = 2):
    """AMEn approximation y ~ A x in place (y: initial guess in, result out; z:
    residual guess in and out); returns the last sweep's rounding error [batch]."""
    torch = _torch()
    err = torch.zeros(x.batch, dtype=torch.float64, device=x.data.device)
    _check(ctx.lib.tt_amen_mv(ctx.h, C.byref(A.desc()), C.byref(x.desc()), C.byref(y.desc()),
                              C.byref(z.desc()), float(eps), int(max_rank), int(sweeps),
                              C.c_void_p(err.data_ptr())))
    return err


@dataclass
class DeviceOperands:
    L: int
    kp: DeviceTT
    Kp: DeviceMPO
    K2: DeviceMPO
    k0: float
    S: DeviceMPO
    Sinv: DeviceMPO
    G: DeviceMPO
    E: DeviceTT
    E_norm: np.ndarray
    k_sel: list
    SE: DeviceTT
    G2: DeviceMPO = None          # G^H G (elasticity); None: conductivity identity
    _struct: Operands = field(default=None, repr=False)

    def struct(self) -> Operands:
        kp = self.kp.desc() if self.kp is not None else TTDesc()
        g2 = self.G2.desc() if self.G2 is not None else MPODesc()
        s = Operands(self.L, kp, self.Kp.desc(), self.K2.desc(), self.k0,
                     self.S.desc(), self.Sinv.desc(), self.G.desc(), self.E.desc(),
                     self.E_norm.ctypes.data_as(C.POINTER(C.c_double)), self.SE.desc(), g2)
        self._struct = s
        return s


def field_capacity(L: int, max_rank: int, d: int = 3):
    modes = [d] + [2] * (3 * L)
    nat = natural_caps(modes)
    return modes, [min(r, max_rank) if max_rank > 0 else r for r in nat]


def solve_opts(eps, max_rank, tol=1e-8, max_iter=200, mode=ROUND_SVD, graph=False, **kw):
    return SolveOpts(round_opts(eps, max_rank, mode, **kw), tol, max_iter, 1 if graph else 0)


def ls_iterate(ctx: Context, ops: DeviceOperands, e: DeviceTT, opts: SolveOpts, n_iter: int):
    torch = _torch()
    res = torch.zeros(max(n_iter, 1) * e.batch, dtype=torch.float64, device=e.data.device)
    st = ops.struct()
    _check(ctx.lib.ls_iterate(ctx.h, C.byref(st), C.byref(e.desc()), C.byref(opts), n_iter,
                              C.c_void_p(res.data_ptr())))
    return res.view(-1, e.batch)[:n_iter]


def homogenize(ctx: Context, ops: DeviceOperands, e: DeviceTT, opts: SolveOpts):
    """Returns (A_eff [batch, d] (mean flux or stress per field), iterations [batch],
    residuals [max_iter, batch], status); d = the field's component mode."""
    B = e.batch
    d = int(e.modes[0])
    A = np.zeros((B, d))
    its = np.zeros(B, dtype=np.int32)
    res = np.full((opts.max_iter, B), np.nan)
    ksel = (TTDesc * d)(*[t.desc() for t in ops.k_sel])
    st = ops.struct()
    s = _check(ctx.lib.homogenize(ctx.h, C.byref(st), ksel, C.byref(e.desc()), C.byref(opts),
                                  A.ctypes.data_as(C.POINTER(C.c_double)),
                                  its.ctypes.data_as(C.POINTER(C.c_int32)),
                                  res.ctypes.data_as(C.POINTER(C.c_double))))
    return A, its, res, s


# ---------------------------------------------------------------------------
# Learned-rank rounding: MLP kernels, rank logs and the predictor.

RANK_FEATURES = 24


def mlp_num_params(n_in: int, n_cls: int) -> int:
    return int(load_library().qt_mlp_num_params(n_in, n_cls))


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def mlp_train_step(ctx: Context, params, m, v, step: int, X, labels, n_cls: int, lr: float,
                   beta: float, gamma: float, loss=None, grad=None):
    """One full-batch MLP step on device tensors (params/m/v float32, X [n, F] float32,
    labels [n] int32); loss (float32 [1]) and grad (float32 [P]) are optional outputs."""
    n, F = X.shape
    _check(ctx.lib.qt_mlp_train_step(ctx.h, _ptr(params), _ptr(m), _ptr(v), step, _ptr(X),
                                     _ptr(labels), n, F, n_cls, lr, beta, gamma, _ptr(loss),
                                     _ptr(grad)))


def mlp_infer(ctx: Context, params, X, n_cls: int, quantile: float = 0.9, rank_cap=None):
    """(logits [n, n_cls] float32, ranks [n] int32) on the device."""
    torch = _torch()
    n, F = X.shape
    logits = torch.empty((n, n_cls), dtype=torch.float32, device=X.device)
    ranks = torch.empty(n, dtype=torch.int32, device=X.device)
    _check(ctx.lib.qt_mlp_infer(ctx.h, _ptr(params), _ptr(X), n, F, n_cls, quantile,
                                _ptr(logits), _ptr(ranks), _ptr(rank_cap)))
    return logits, ranks


def ranklog_enable(ctx: Context, capacity: int, n_cls: int):
    _check(ctx.lib.qt_ranklog_enable(ctx.h, capacity, n_cls))


def ranklog_get(ctx: Context):
    """The logged (features [count, 24] float32, labels [count] int32) as device tensors."""
    torch = _torch()
    cnt = C.c_int32()
    _check(ctx.lib.qt_ranklog_get(ctx.h, None, None, 0, C.byref(cnt)))
    n = cnt.value
    X = torch.empty((n, RANK_FEATURES), dtype=torch.float32, device="cuda")
    Y = torch.empty(n, dtype=torch.int32, device="cuda")
    if n:
        _check(ctx.lib.qt_ranklog_get(ctx.h, _ptr(X), _ptr(Y), n, C.byref(cnt)))
        ctx.sync()
    return X, Y


def set_predictor(ctx: Context, params, n_cls: int, quantile: float = 0.9,
                  accept_factor: float = 1.0):
    _check(ctx.lib.qt_set_predictor(ctx.h, _ptr(params), n_cls, quantile, accept_factor))


def learn_reset(ctx: Context):
    _check(ctx.lib.qt_learn_reset(ctx.h))


LEARN_LOG_COLS = 6


def learn_log_enable(ctx: Context, capacity: int):
    _check(ctx.lib.qt_learn_log_enable(ctx.h, capacity))


def learn_log_get(ctx: Context):
    """Rows (iteration, step, instance, error, reference, kept) of the learned-
    rounding log as a host float64 array [count, 6]."""
    cnt = C.c_int32()
    _check(ctx.lib.qt_learn_log_get(ctx.h, None, 0, C.byref(cnt)))
    rows = np.zeros((max(cnt.value, 1), LEARN_LOG_COLS), dtype=np.float64)
    if cnt.value:
        _check(ctx.lib.qt_learn_log_get(ctx.h, rows.ctypes.data_as(C.c_void_p), cnt.value,
                                        C.byref(cnt)))
    return rows[:cnt.value]
