"""ctypes binding of libgbs (include/gbs.h): the same entry points under the same
names, argument marshalling only.  Device buffers are torch tensors; every
compute step runs in the library's HIP kernels.  There is no fallback: if
libgbs.so has not been built, loading raises."""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# GBS_LIBRARY may name another build of the same library (same ABI)
LIB_PATH = os.environ.get("GBS_LIBRARY") or os.path.join(_HERE, "libgbs.so")

GBS_OK = 0
GBS_E_INVALID_ARG = 1
GBS_E_NOT_SPD = 2
GBS_E_OUT_OF_MEMORY = 3
GBS_E_DEVICE = 4
GBS_E_UNSUPPORTED = 5
GBS_E_SCRATCH_LIMIT = 6
GBS_NOALLOC_SCRATCH_BYTES = 160 * 1024 * 1024

GBS_CLICK = 0
GBS_PARITY = 1
GBS_FP64 = 0
GBS_MIXED = 2
GBS_ASYNC = 4
GBS_TIMING = 8
GBS_ALL_MINORS = 16

GBS_STAGE_BUILD_Q = 0
GBS_STAGE_NORMALISE = 1
GBS_STAGE_FORWARD = 2
GBS_STAGE_ADJOINT = 3
GBS_STAGE_BATCHED = 4
GBS_STAGE_SAMPLE = 5
GBS_STAGE_ESTIMATE = 6
STAGE_NAMES = {0: "build_q", 1: "normalise", 2: "forward", 3: "adjoint", 4: "batched", 5: "sample",
               6: "estimate"}

GBS_MAX_ORDER = 5
GBS_MAX_MODES = 2048

# every symbol declared in include/gbs.h
EXPORTS = (
    "gbs_num_subsets", "gbs_order_offset", "gbs_total_outputs", "gbs_colex_rank",
    "gbs_colex_unrank", "gbs_correlators", "gbs_cumulants", "gbs_cumulants_displaced",
    "gbs_cumulants_shard",
    "gbs_cumulant_grad",
    "gbs_cumulants_batched", "gbs_autotune_batched", "gbs_set_tuning", "gbs_sample",
    "gbs_sample_cumulants", "gbs_pearson", "gbs_last_error",
    "gbs_last_timings", "gbs_status_string", "gbs_cumulants_noalloc",
)


class GBSError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {gbs_status_string(status)} (status {status})")


class gbs_instance(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sigma", ctypes.c_void_p), ("corr", ctypes.c_void_p), ("cum", ctypes.c_void_p)]


class gbs_tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("unroll", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("group_wpc", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class gbs_kernel_time(ctypes.Structure):
    _fields_ = [("stage", ctypes.c_int32), ("order", ctypes.c_int32), ("ms", ctypes.c_float)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libgbs.so (raises if it is missing: there is no other implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2511_14923_amd/build.py` "
                          "or __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.gbs_num_subsets.argtypes = [i32, i32]
    L.gbs_num_subsets.restype = i64
    L.gbs_order_offset.argtypes = [i32, i32]
    L.gbs_order_offset.restype = i64
    L.gbs_total_outputs.argtypes = [i32, i32]
    L.gbs_total_outputs.restype = i64
    L.gbs_colex_rank.argtypes = [i32, ctypes.POINTER(i32)]
    L.gbs_colex_rank.restype = i64
    L.gbs_colex_unrank.argtypes = [i32, i64, ctypes.POINTER(i32)]
    L.gbs_colex_unrank.restype = i32
    L.gbs_correlators.argtypes = [i32, vp, i32, i32, vp, vp]
    L.gbs_correlators.restype = i32
    L.gbs_cumulants.argtypes = [i32, vp, i32, i32, vp, vp, vp]
    L.gbs_cumulants.restype = i32
    L.gbs_cumulants_noalloc.argtypes = [i32, vp, i32, i32, vp, vp, vp]
    L.gbs_cumulants_noalloc.restype = i32
    L.gbs_cumulants_displaced.argtypes = [i32, vp, vp, i32, i32, vp, vp, vp]
    L.gbs_cumulants_displaced.restype = i32
    L.gbs_cumulants_shard.argtypes = [i32, vp, i32, i64, i64, i32, vp, vp, vp]
    L.gbs_cumulants_shard.restype = i32
    L.gbs_cumulant_grad.argtypes = [i32, vp, i32, i32, vp, vp, vp, vp]
    L.gbs_cumulant_grad.restype = i32
    L.gbs_cumulants_batched.argtypes = [i32, ctypes.POINTER(gbs_instance), i32, i32, vp]
    L.gbs_cumulants_batched.restype = i32
    L.gbs_autotune_batched.argtypes = [i32, ctypes.POINTER(gbs_instance), i32, i32, vp,
                                       ctypes.POINTER(gbs_tuning)]
    L.gbs_autotune_batched.restype = i32
    L.gbs_set_tuning.argtypes = [i32, i32, ctypes.POINTER(gbs_tuning)]
    L.gbs_set_tuning.restype = i32
    L.gbs_sample.argtypes = [i32, vp, i32, i64, vp, vp, vp, vp, i64, i32, vp]
    L.gbs_sample.restype = i32
    L.gbs_sample_cumulants.argtypes = [i32, i64, vp, i32, vp, i32, vp]
    L.gbs_sample_cumulants.restype = i32
    L.gbs_pearson.argtypes = [i64, vp, vp, vp, i32, vp]
    L.gbs_pearson.restype = i32
    L.gbs_last_error.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.gbs_last_error.restype = i32
    L.gbs_last_timings.argtypes = [i32, ctypes.POINTER(gbs_kernel_time)]
    L.gbs_last_timings.restype = i32
    L.gbs_status_string.argtypes = [i32]
    L.gbs_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int, where: str):
    if status != GBS_OK:
        raise GBSError(status, where)


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("device tensor required")
    if t.dtype != torch.float64:
        raise ValueError("float64 tensor required")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor required")
    return ctypes.c_void_p(t.data_ptr())


# The C ABI receives bare pointers and cannot see buffer sizes, so every size,
# dtype and device is checked here, before the call: an undersized buffer would
# otherwise be read or written out of bounds by the kernels.

def _need(t, name, numel, dtype=torch.float64, shape=None, optional=False):
    """Check that t is a contiguous tensor of `dtype` with `numel` elements (and
    `shape` if given); None is accepted when optional."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name}: {dtype} tensor required, got {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{name}: {numel} elements required, got {t.numel()}")
    if shape is not None and tuple(t.shape) not in (tuple(shape), (numel,)):
        raise ValueError(f"{name}: shape {tuple(shape)} required, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: contiguous tensor required")


def _same_device(*named):
    """All given tensors (None skipped) on one GPU."""
    dev = None
    for name, t in named:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError(f"{name}: device tensor required")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError(f"{name} is on {t.device}, expected {dev}")


def _outputs(M, max_order):
    """N(M, K), or ValueError for arguments the library would reject anyway."""
    n = gbs_total_outputs(M, max_order)
    if n < 0:
        raise ValueError(f"invalid M = {M} / max_order = {max_order}")
    return n


def _sigma(M, sigma, name="sigma"):
    _need(sigma, name, 4 * M * M, shape=(2 * M, 2 * M))


def _stream(stream, device):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


# ---- host helpers -----------------------------------------------------------

def gbs_num_subsets(M: int, d: int) -> int:
    return int(lib().gbs_num_subsets(M, d))


def gbs_order_offset(M: int, d: int) -> int:
    return int(lib().gbs_order_offset(M, d))


def gbs_total_outputs(M: int, max_order: int) -> int:
    return int(lib().gbs_total_outputs(M, max_order))


def gbs_colex_rank(S) -> int:
    arr = (ctypes.c_int32 * len(S))(*[int(x) for x in S])
    return int(lib().gbs_colex_rank(len(S), arr))


def gbs_colex_unrank(d: int, r: int) -> tuple:
    arr = (ctypes.c_int32 * max(d, 1))()
    _check(lib().gbs_colex_unrank(d, r, arr), "gbs_colex_unrank")
    return tuple(arr[:d])


def gbs_last_error() -> tuple:
    o, r = ctypes.c_int32(), ctypes.c_int64()
    st = lib().gbs_last_error(ctypes.byref(o), ctypes.byref(r))
    return st, o.value, r.value


def gbs_last_timings(capacity: int = 64) -> list:
    """[(stage name, order, ms), ...] of this thread's last GBS_TIMING call."""
    buf = (gbs_kernel_time * capacity)()
    n = int(lib().gbs_last_timings(capacity, buf))
    if n < 0:
        raise GBSError(GBS_E_DEVICE, "gbs_last_timings")
    return [(STAGE_NAMES.get(buf[i].stage, str(buf[i].stage)), buf[i].order, float(buf[i].ms))
            for i in range(min(n, capacity))]


def gbs_status_string(status: int) -> str:
    return lib().gbs_status_string(status).decode()


# ---- device entry points ----------------------------------------------------

def _out(buf, n, like):
    if buf is None:
        return torch.empty(n, dtype=torch.float64, device=like.device)
    return buf


def gbs_correlators(M: int, sigma: torch.Tensor, max_order: int, flags: int = 0, corr=None,
                    stream=None) -> torch.Tensor:
    n = _outputs(M, max_order)
    _sigma(M, sigma)
    corr = _out(corr, n, sigma)
    _need(corr, "corr", n)
    _same_device(("sigma", sigma), ("corr", corr))
    with torch.cuda.device(sigma.device):
        st = lib().gbs_correlators(M, _ptr(sigma), max_order, flags, _ptr(corr),
                                   _stream(stream, sigma.device))
    _check(st, "gbs_correlators")
    return corr


def gbs_cumulants(M: int, sigma: torch.Tensor, max_order: int, flags: int = 0, corr=None, cum=None,
                  stream=None, want_corr: bool = True) -> tuple:
    n = _outputs(M, max_order)
    _sigma(M, sigma)
    if want_corr:
        corr = _out(corr, n, sigma)
    cum = _out(cum, n, sigma)
    _need(corr, "corr", n, optional=True)
    _need(cum, "cum", n)
    _same_device(("sigma", sigma), ("corr", corr), ("cum", cum))
    with torch.cuda.device(sigma.device):
        st = lib().gbs_cumulants(M, _ptr(sigma), max_order, flags, _ptr(corr), _ptr(cum),
                                 _stream(stream, sigma.device))
    _check(st, "gbs_cumulants")
    return corr, cum


def gbs_cumulants_noalloc(M: int, sigma: torch.Tensor, max_order: int, flags: int, corr, cum,
                          stream=None) -> tuple:
    """gbs_cumulants through the allocation-free entry point: the caller passes
    every output buffer (corr may be None), nothing is allocated here either."""
    n = _outputs(M, max_order)
    _sigma(M, sigma)
    _need(corr, "corr", n, optional=True)
    _need(cum, "cum", n)
    _same_device(("sigma", sigma), ("corr", corr), ("cum", cum))
    with torch.cuda.device(sigma.device):
        st = lib().gbs_cumulants_noalloc(M, _ptr(sigma), max_order, flags, _ptr(corr), _ptr(cum),
                                         _stream(stream, sigma.device))
    _check(st, "gbs_cumulants_noalloc")
    return corr, cum


def gbs_cumulants_displaced(M: int, sigma: torch.Tensor, mu: torch.Tensor, max_order: int,
                            flags: int = 0, corr=None, cum=None, stream=None,
                            want_corr: bool = True) -> tuple:
    n = _outputs(M, max_order)
    _sigma(M, sigma)
    _need(mu, "mu", 2 * M)
    if want_corr:
        corr = _out(corr, n, sigma)
    cum = _out(cum, n, sigma)
    _need(corr, "corr", n, optional=True)
    _need(cum, "cum", n)
    _same_device(("sigma", sigma), ("mu", mu), ("corr", corr), ("cum", cum))
    with torch.cuda.device(sigma.device):
        st = lib().gbs_cumulants_displaced(M, _ptr(sigma), _ptr(mu), max_order, flags, _ptr(corr),
                                           _ptr(cum), _stream(stream, sigma.device))
    _check(st, "gbs_cumulants_displaced")
    return corr, cum


def gbs_cumulants_shard(M: int, sigma: torch.Tensor, order: int, rank0: int, count: int,
                        flags: int = 0, corr=None, cum=None, stream=None,
                        want_corr: bool = True) -> tuple:
    if not (1 <= M <= GBS_MAX_MODES and 1 <= order <= min(GBS_MAX_ORDER, M)):
        raise ValueError(f"invalid M = {M} / order = {order}")
    if rank0 < 0 or count < 0 or rank0 + count > gbs_num_subsets(M, order):
        raise ValueError(f"rank range [{rank0}, {rank0} + {count}) outside C({M}, {order})")
    _sigma(M, sigma)
    if want_corr:
        corr = _out(corr, count, sigma)
    cum = _out(cum, count, sigma)
    _need(corr, "corr", count, optional=True)
    _need(cum, "cum", count, optional=True)
    _same_device(("sigma", sigma), ("corr", corr), ("cum", cum))
    with torch.cuda.device(sigma.device):
        st = lib().gbs_cumulants_shard(M, _ptr(sigma), order, rank0, count, flags, _ptr(corr),
                                       _ptr(cum), _stream(stream, sigma.device))
    _check(st, "gbs_cumulants_shard")
    return corr, cum


def _ptr_u8(t):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.uint8 \
            or not t.is_contiguous():
        raise ValueError("contiguous uint8 device tensor required")
    return ctypes.c_void_p(t.data_ptr())


def gbs_sample(M: int, kappa: torch.Tensor, max_order: int, uniforms: torch.Tensor, bits=None,
               prob=None, cond=None, batch: int = 0, flags: int = 0, stream=None,
               want_prob: bool = True, want_cond: bool = False) -> tuple:
    """Sampler: uniforms is (M, n) FP64; returns (bits (n, M) uint8, prob (n,) or
    None, cond (M, n) or None)."""
    if M < 1:
        raise ValueError(f"invalid M = {M}")
    if uniforms.dim() == 2:
        if uniforms.shape[0] != M:
            raise ValueError(f"uniforms: shape ({M}, n) required, got {tuple(uniforms.shape)}")
        n = uniforms.shape[1]
    else:
        if uniforms.numel() % M:
            raise ValueError(f"uniforms: a multiple of M = {M} elements required")
        n = uniforms.numel() // M
    _need(kappa, "kappa", _outputs(M, max_order))
    _need(uniforms, "uniforms", M * n)
    dev = kappa.device
    if bits is None:
        bits = torch.empty((n, M), dtype=torch.uint8, device=dev)
    if prob is None and want_prob:
        prob = torch.empty(n, dtype=torch.float64, device=dev)
    if cond is None and want_cond:
        cond = torch.empty((M, n), dtype=torch.float64, device=dev)
    _need(bits, "bits", n * M, dtype=torch.uint8)
    _need(prob, "prob", n, optional=True)
    _need(cond, "cond", M * n, optional=True)
    _same_device(("kappa", kappa), ("uniforms", uniforms), ("bits", bits), ("prob", prob),
                 ("cond", cond))
    with torch.cuda.device(dev):
        st = lib().gbs_sample(M, _ptr(kappa), max_order, n, _ptr(uniforms), _ptr_u8(bits),
                              _ptr(prob), _ptr(cond), batch, flags, _stream(stream, dev))
    _check(st, "gbs_sample")
    return bits, prob, cond


def gbs_sample_cumulants(bits: torch.Tensor, max_order: int, cum=None, flags: int = 0,
                         stream=None) -> torch.Tensor:
    """Unbiased click cumulants of orders 1..max_order from samples (n, M) uint8."""
    if bits.dim() != 2:
        raise ValueError("bits: shape (nsamples, M) required")
    n, M = bits.shape
    _need(bits, "bits", n * M, dtype=torch.uint8)
    nout = _outputs(M, max_order)
    cum = _out(cum, nout, bits)
    _need(cum, "cum", nout)
    _same_device(("bits", bits), ("cum", cum))
    with torch.cuda.device(bits.device):
        st = lib().gbs_sample_cumulants(M, n, _ptr_u8(bits), max_order, _ptr(cum), flags,
                                        _stream(stream, bits.device))
    _check(st, "gbs_sample_cumulants")
    return cum


def gbs_pearson(x: torch.Tensor, y: torch.Tensor, r=None, flags: int = 0, stream=None) -> torch.Tensor:
    """Pearson coefficient of two device FP64 vectors (a one-element tensor)."""
    _need(x, "x", x.numel() if isinstance(x, torch.Tensor) else -1)
    _need(y, "y", x.numel())
    if r is None:
        r = torch.empty(1, dtype=torch.float64, device=x.device)
    _need(r, "r", 1)
    _same_device(("x", x), ("y", y), ("r", r))
    with torch.cuda.device(x.device):
        st = lib().gbs_pearson(x.numel(), _ptr(x), _ptr(y), _ptr(r), flags, _stream(stream, x.device))
    _check(st, "gbs_pearson")
    return r


def gbs_cumulant_grad(M: int, sigma: torch.Tensor, max_order: int, flags: int = 0,
                      grad_corr=None, grad_cum=None, grad_sigma=None, stream=None) -> torch.Tensor:
    n = _outputs(M, max_order)
    _sigma(M, sigma)
    _need(grad_corr, "grad_corr", n, optional=True)
    _need(grad_cum, "grad_cum", n, optional=True)
    if grad_sigma is None:
        grad_sigma = torch.empty_like(sigma)
    _sigma(M, grad_sigma, "grad_sigma")
    _same_device(("sigma", sigma), ("grad_corr", grad_corr), ("grad_cum", grad_cum),
                 ("grad_sigma", grad_sigma))
    with torch.cuda.device(sigma.device):
        st = lib().gbs_cumulant_grad(M, _ptr(sigma), max_order, flags, _ptr(grad_corr),
                                     _ptr(grad_cum), _ptr(grad_sigma), _stream(stream, sigma.device))
    _check(st, "gbs_cumulant_grad")
    return grad_sigma


def _instances(instances, max_order):
    if len(instances) == 0:
        raise ValueError("at least one instance is required")
    for i, (M, sigma, corr, cum) in enumerate(instances):
        n = _outputs(M, max_order)
        _sigma(M, sigma, f"instance {i} sigma")
        _need(corr, f"instance {i} corr", n, optional=True)
        _need(cum, f"instance {i} cum", n)
    for i, (M, sigma, corr, cum) in enumerate(instances):
        _same_device(("instance 0 sigma", instances[0][1]), (f"instance {i} sigma", sigma),
                     (f"instance {i} corr", corr), (f"instance {i} cum", cum))
    arr = (gbs_instance * len(instances))()
    for i, (M, sigma, corr, cum) in enumerate(instances):
        arr[i].M = M
        arr[i].reserved = 0
        arr[i].sigma = _ptr(sigma).value
        arr[i].corr = _ptr(corr).value if corr is not None else None
        arr[i].cum = _ptr(cum).value
    return arr


def gbs_cumulants_batched(instances, max_order: int, flags: int = 0, stream=None) -> None:
    """instances: list of (M, sigma, corr or None, cum) with device tensors."""
    arr = _instances(instances, max_order)
    dev = instances[0][1].device
    with torch.cuda.device(dev):
        st = lib().gbs_cumulants_batched(len(instances), arr, max_order, flags, _stream(stream, dev))
    _check(st, "gbs_cumulants_batched")


def gbs_autotune_batched(instances, max_order: int, flags: int = 0, stream=None) -> dict:
    arr = _instances(instances, max_order)
    dev = instances[0][1].device
    best = gbs_tuning()
    with torch.cuda.device(dev):
        st = lib().gbs_autotune_batched(len(instances), arr, max_order, flags, _stream(stream, dev),
                                        ctypes.byref(best))
    _check(st, "gbs_autotune_batched")
    return best.as_dict()


def gbs_set_tuning(max_order: int, flags: int, tuning: dict | None) -> None:
    if tuning is None:
        _check(lib().gbs_set_tuning(max_order, flags, None), "gbs_set_tuning")
        return
    t = gbs_tuning(**tuning)
    _check(lib().gbs_set_tuning(max_order, flags, ctypes.byref(t)), "gbs_set_tuning")
