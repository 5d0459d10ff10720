"""MI355X (gfx950) sort library: thin Python binding of ``libak.so``.

Every function marshals torch tensors into the C ABI declared in
``include/ak.h`` (device pointers and the current HIP stream); all work runs
in the library's HIP kernels.  There is no fallback: if ``libak.so`` is
missing or a tensor is not on a GPU, the call raises.

The operations are the paper's sorting primitives (AcceleratedKernels.jl,
Sec. II-B): ``sort_`` (in place, stable, Julia Base order: NaN last, -0.0
before +0.0), ``sortperm`` (stable 0-based uint32 permutation), the batched
``segmented_sort_`` and the learned-CDF partition sort ``sort_learned_``.
Unsigned keys are passed in signed storage of the same width with an
explicit ``dtype`` ("u32" / "u64").
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libak.so")

DTYPE_CODE = {"i32": 1, "i64": 2, "u32": 3, "u64": 4, "f32": 5, "f64": 6,
              "i16": 7, "u16": 8, "i128": 9, "u128": 10}
_TORCH_DEFAULT = {torch.int32: "i32", torch.int64: "i64", torch.float32: "f32",
                  torch.float64: "f64", torch.int16: "i16"}
for _name, _dt in (("uint16", "u16"), ("uint32", "u32"), ("uint64", "u64")):
    if hasattr(torch, _name):
        _TORCH_DEFAULT[getattr(torch, _name)] = _dt
# bytes per key; 128-bit keys (no torch dtype) are held as int64 pairs,
# e.g. an (n, 2) int64 tensor, low word first
_WIDTH = {"i32": 4, "u32": 4, "f32": 4, "i64": 8, "u64": 8, "f64": 8, "i16": 2, "u16": 2,
          "i128": 16, "u128": 16}
OPS = {"sort": 0, "sortperm": 1, "segmented": 2, "learned": 3, "accumulate": 4, "sort_by_key": 5,
       "sortperm_lowmem": 6}


class AKError(RuntimeError):
    """A library call returned a non-zero ak_status."""

    def __init__(self, status: int, what: str, detail: str):
        super().__init__(f"{what}: status {status} ({detail})")
        self.status = status


class LearnedCfg(ctypes.Structure):
    _fields_ = [("leaves", ctypes.c_int32), ("buckets_log2", ctypes.c_int32),
                ("sample_frac", ctypes.c_float), ("train_iters", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("untrained", ctypes.c_int32),
                ("model", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class LearnedStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sample_size", ctypes.c_int64),
                ("leaves", ctypes.c_int32), ("code_bits", ctypes.c_int32),
                ("max_bucket", ctypes.c_int64), ("imbalance", ctypes.c_double),
                ("fallback_keys", ctypes.c_int64), ("constant_keys", ctypes.c_int64),
                ("fallback_runs", ctypes.c_int64), ("chunks", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libak.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2507_16710_amd.build` "
                          "or __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    sig = {
        "ak_sort": [vp, i64, i32, vp],
        "ak_sort_noalloc": [vp, i64, i32, vp],
        "ak_sortperm_lowmem": [vp, vp, i64, i32, vp],
        "ak_segmented_sort_n": [vp, i64, vp, i64, i32, vp],
        "ak_sort_by_key": [vp, vp, i64, i32, i32, vp],
        "ak_sortperm": [vp, vp, i64, i32, vp],
        "ak_segmented_sort": [vp, vp, i64, i32, vp],
        "ak_check_device_error": [vp],
        "ak_sort_learned": [vp, i64, i32, vp, vp, vp],
        "ak_learned_sample": [vp, i64, i32, u64, i64, vp, vp],
        "ak_rmi_fit": [vp, i64, i32, i32, i32, vp, vp],
        "ak_rmi_leaf_grad": [vp, i64, i32, vp, vp, vp],
        "ak_rmi_codes": [vp, i64, i32, vp, i32, vp, vp],
        "ak_mlp_loss_grad": [vp, vp, i64, vp, vp, vp],
        "ak_mlp_fit": [vp, i64, i32, i32, i32, vp, vp, vp],
        "ak_release_workspace": [],
        "ak_set_workspace": [vp, ctypes.c_size_t, vp],
        "ak_sort_route": [vp, vp],
        "ak_accumulate": [vp, vp, i64, i32, i32, vp],
        "ak_searchsortedfirst": [vp, i64, vp, i64, i32, vp, vp],
        "ak_searchsortedlast": [vp, i64, vp, i64, i32, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = i32
    for suf in ("i32", "i64", "u32", "u64", "f32", "f64"):
        getattr(lib, f"ak_sortperm_{suf}").argtypes = [vp, vp, i64, vp]
        getattr(lib, f"ak_sortperm_{suf}").restype = i32
        getattr(lib, f"ak_segmented_sort_{suf}").argtypes = [vp, vp, i64, vp]
        getattr(lib, f"ak_segmented_sort_{suf}").restype = i32
    lib.ak_temp_bytes.argtypes = [i32, i64, i32]
    lib.ak_temp_bytes.restype = ctypes.c_size_t
    lib.ak_temp_bytes_segmented.argtypes = [i64, i64, i32]
    lib.ak_temp_bytes_segmented.restype = ctypes.c_size_t
    lib.ak_rmi_model_floats.argtypes = [i32]
    lib.ak_rmi_model_floats.restype = ctypes.c_size_t
    lib.ak_profile_enable.argtypes = [i32]
    lib.ak_profile_enable.restype = i32
    lib.ak_profile_read.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    lib.ak_profile_read.restype = ctypes.c_size_t
    lib.ak_seg_set_tuning.argtypes = [i32, i32, i32, i32, i32, i32]
    lib.ak_seg_set_tuning.restype = i32
    lib.ak_last_error.restype = ctypes.c_char_p
    lib.ak_status_string.argtypes = [i32]
    lib.ak_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, what: str) -> None:
    if status != 0:
        lib = load_library()
        detail = lib.ak_last_error().decode() or lib.ak_status_string(status).decode()
        raise AKError(status, what, detail)


def _dtype(t: torch.Tensor, dtype: str | None) -> str:
    dt = dtype or _TORCH_DEFAULT.get(t.dtype)
    if dt not in DTYPE_CODE:
        raise TypeError(f"unsupported key dtype {t.dtype} (pass dtype=...)")
    if dt in ("i128", "u128"):
        if t.element_size() != 8 or t.numel() % 2:
            raise TypeError("128-bit keys are held as pairs of 64-bit words (an even number of int64 elements)")
    elif t.element_size() != _WIDTH[dt]:
        raise TypeError(f"dtype {dt} needs {_WIDTH[dt]}-byte elements, got {t.dtype}")
    return dt


def _count(t: torch.Tensor, dt: str) -> int:
    """Number of keys a tensor of dtype `dt` holds."""
    return t.numel() * t.element_size() // _WIDTH[dt]


def _gpu(t: torch.Tensor, name: str) -> None:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def sort_(keys: torch.Tensor, dtype: str | None = None) -> torch.Tensor:
    """Sorts ``keys`` in place (ak_sort); returns it."""
    _gpu(keys, "keys")
    dt = _dtype(keys, dtype)
    with torch.cuda.device(keys.device):
        _check(load_library().ak_sort(keys.data_ptr(), _count(keys, dt), DTYPE_CODE[dt], _stream(keys)), "ak_sort")
    return keys


def sortperm(keys: torch.Tensor, dtype: str | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Stable 0-based permutation (uint32 bits in an int32 tensor)."""
    _gpu(keys, "keys")
    dt = _dtype(keys, dtype)
    n = _count(keys, dt)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=keys.device)
    _gpu(out, "out")
    if out.numel() != n or out.element_size() != 4:
        raise ValueError("out must hold one 4-byte index per key")
    with torch.cuda.device(keys.device):
        _check(load_library().ak_sortperm(keys.data_ptr(), out.data_ptr(), n, DTYPE_CODE[dt], _stream(keys)),
               "ak_sortperm")
    return out


def sortperm_lowmem(keys: torch.Tensor, dtype: str | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """The permutation of ``sortperm`` with scratch for the indices only
    (ak_sortperm_lowmem)."""
    _gpu(keys, "keys")
    dt = _dtype(keys, dtype)
    n = _count(keys, dt)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=keys.device)
    _gpu(out, "out")
    if out.numel() != n or out.element_size() != 4:
        raise ValueError("out must hold one 4-byte index per key")
    with torch.cuda.device(keys.device):
        _check(load_library().ak_sortperm_lowmem(keys.data_ptr(), out.data_ptr(), n, DTYPE_CODE[dt], _stream(keys)),
               "ak_sortperm_lowmem")
    return out


def sort_by_key_(keys: torch.Tensor, vals: torch.Tensor, dtype: str | None = None):
    """Sorts ``keys`` in place and reorders ``vals`` (one 4- or 8-byte
    payload per key, any dtype: its bits are moved) the same way
    (ak_sort_by_key); returns (keys, vals)."""
    _gpu(keys, "keys")
    _gpu(vals, "vals")
    dt = _dtype(keys, dtype)
    n = _count(keys, dt)
    vb = vals.numel() * vals.element_size() // max(n, 1) if n else 4
    if vals.numel() * vals.element_size() != n * vb or vb not in (4, 8):
        raise ValueError("vals must hold one 4- or 8-byte payload per key")
    with torch.cuda.device(keys.device):
        _check(load_library().ak_sort_by_key(keys.data_ptr(), vals.data_ptr(), n, DTYPE_CODE[dt], vb, _stream(keys)),
               "ak_sort_by_key")
    return keys, vals


def segmented_sort_(keys: torch.Tensor, offsets: torch.Tensor, dtype: str | None = None,
                    check: bool = True) -> torch.Tensor:
    """Sorts every segment [offsets[s], offsets[s+1]) of ``keys`` in place
    (ak_segmented_sort_n: asynchronous, the offsets are checked against
    len(keys) on the device).  With check=True the call then waits and
    raises if the device found offsets outside [0, len(keys)] or
    decreasing; check=False returns at once (ak.check_device_error reports
    such offsets later)."""
    _gpu(keys, "keys")
    _gpu(offsets, "offsets")
    if offsets.dtype != torch.int64:
        raise TypeError("offsets must be int64")
    dt = _dtype(keys, dtype)
    with torch.cuda.device(keys.device):
        _check(load_library().ak_segmented_sort_n(keys.data_ptr(), keys.numel(), offsets.data_ptr(),
                                                  offsets.numel() - 1, DTYPE_CODE[dt], _stream(keys)),
               "ak_segmented_sort_n")
    if check:
        check_device_error(keys.device)
    return keys


def check_device_error(device=None) -> None:
    dev = torch.device("cuda" if device is None else device)
    with torch.cuda.device(dev):
        _check(load_library().ak_check_device_error(torch.cuda.current_stream(dev).cuda_stream),
               "ak_check_device_error")


MODELS = {"rmi": 0, "mlp": 1}
MLP_PARAMS = 4353


def make_cfg(leaves=0, buckets_log2=0, sample_frac=0.0, train_iters=0, seed=0, untrained=False,
             model: str = "rmi") -> LearnedCfg:
    c = LearnedCfg()
    c.leaves, c.buckets_log2, c.sample_frac = leaves, buckets_log2, sample_frac
    c.train_iters, c.seed, c.untrained = train_iters, seed, int(bool(untrained))
    c.model = MODELS[model]
    return c


def sort_learned_(keys: torch.Tensor, dtype: str | None = None, cfg: LearnedCfg | None = None,
                  stats: bool = False):
    """Learned-CDF partition sort in place.  With stats=True returns
    (keys, stats dict) and synchronises the stream."""
    _gpu(keys, "keys")
    dt = _dtype(keys, dtype)
    st = LearnedStats() if stats else None
    with torch.cuda.device(keys.device):
        _check(load_library().ak_sort_learned(
            keys.data_ptr(), keys.numel(), DTYPE_CODE[dt],
            ctypes.byref(cfg) if cfg is not None else None,
            ctypes.byref(st) if st is not None else None, _stream(keys)), "ak_sort_learned")
    return (keys, st.as_dict()) if stats else keys


def learned_sample(keys: torch.Tensor, m: int, seed: int = 0, dtype: str | None = None) -> torch.Tensor:
    _gpu(keys, "keys")
    dt = _dtype(keys, dtype)
    out = torch.empty(m, dtype=keys.dtype, device=keys.device)
    with torch.cuda.device(keys.device):
        _check(load_library().ak_learned_sample(keys.data_ptr(), keys.numel(), DTYPE_CODE[dt], seed, m,
                                                out.data_ptr(), _stream(keys)), "ak_learned_sample")
    return out


def model_floats(leaves: int) -> int:
    return int(load_library().ak_rmi_model_floats(leaves))


def rmi_fit(sorted_sample: torch.Tensor, leaves: int = 4096, iters: int = 3, dtype: str | None = None) -> torch.Tensor:
    _gpu(sorted_sample, "sorted_sample")
    dt = _dtype(sorted_sample, dtype)
    model = torch.zeros(model_floats(leaves), dtype=torch.float32, device=sorted_sample.device)
    with torch.cuda.device(sorted_sample.device):
        _check(load_library().ak_rmi_fit(sorted_sample.data_ptr(), sorted_sample.numel(), DTYPE_CODE[dt],
                                         leaves, iters, model.data_ptr(), _stream(sorted_sample)), "ak_rmi_fit")
    return model


def rmi_leaf_grad(sorted_sample: torch.Tensor, model: torch.Tensor, dtype: str | None = None) -> torch.Tensor:
    _gpu(sorted_sample, "sorted_sample")
    _gpu(model, "model")
    dt = _dtype(sorted_sample, dtype)
    leaves = int(round(float(model[3].item())))
    out = torch.zeros(leaves, 8, dtype=torch.float32, device=model.device)
    with torch.cuda.device(model.device):
        _check(load_library().ak_rmi_leaf_grad(sorted_sample.data_ptr(), sorted_sample.numel(), DTYPE_CODE[dt],
                                               model.data_ptr(), out.data_ptr(), _stream(model)),
               "ak_rmi_leaf_grad")
    return out


def rmi_codes(keys: torch.Tensor, model: torch.Tensor, code_bits: int, dtype: str | None = None) -> torch.Tensor:
    _gpu(keys, "keys")
    _gpu(model, "model")
    dt = _dtype(keys, dtype)
    out = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
    with torch.cuda.device(keys.device):
        _check(load_library().ak_rmi_codes(keys.data_ptr(), keys.numel(), DTYPE_CODE[dt], model.data_ptr(),
                                           code_bits, out.data_ptr(), _stream(keys)), "ak_rmi_codes")
    return out


def mlp_loss_grad(u: torch.Tensor, y: torch.Tensor, params: torch.Tensor) -> torch.Tensor:
    """Loss and gradient of the MLP CDF model over the points (u, y) at the
    raw parameters: returns MLP_PARAMS gradient entries, then the loss."""
    for t, name in ((u, "u"), (y, "y"), (params, "params")):
        _gpu(t, name)
        if t.dtype != torch.float32:
            raise TypeError(f"{name} must be float32")
    if u.numel() != y.numel() or params.numel() != MLP_PARAMS:
        raise ValueError("u and y need one value per point; params needs MLP_PARAMS values")
    out = torch.empty(MLP_PARAMS + 1, dtype=torch.float32, device=u.device)
    with torch.cuda.device(u.device):
        _check(load_library().ak_mlp_loss_grad(u.data_ptr(), y.data_ptr(), u.numel(), params.data_ptr(),
                                               out.data_ptr(), _stream(u)), "ak_mlp_loss_grad")
    return out


def mlp_fit(sorted_sample: torch.Tensor, iters: int = 300, leaves: int = 4096, dtype: str | None = None):
    """Trains the MLP CDF model on an ascending sample and tabulates it:
    returns (raw parameters, model table in the two-level format)."""
    _gpu(sorted_sample, "sorted_sample")
    dt = _dtype(sorted_sample, dtype)
    params = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=sorted_sample.device)
    model = torch.zeros(model_floats(leaves), dtype=torch.float32, device=sorted_sample.device)
    with torch.cuda.device(sorted_sample.device):
        _check(load_library().ak_mlp_fit(sorted_sample.data_ptr(), sorted_sample.numel(), DTYPE_CODE[dt], iters,
                                         leaves, params.data_ptr(), model.data_ptr(), _stream(sorted_sample)),
               "ak_mlp_fit")
    return params, model


def profile_enable(on: bool = True) -> None:
    """Start / stop per-kernel event timing inside the library."""
    _check(load_library().ak_profile_enable(int(on)), "ak_profile_enable")


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} since the last read."""
    lib = load_library()
    buf = ctypes.create_string_buffer(1 << 20)
    lib.ak_profile_read(buf, len(buf))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


def _search(fn: str, sorted_keys: torch.Tensor, keys: torch.Tensor, dtype: str | None,
            out: torch.Tensor | None) -> torch.Tensor:
    _gpu(sorted_keys, "sorted_keys")
    _gpu(keys, "keys")
    dt = _dtype(sorted_keys, dtype)
    if _dtype(keys, dt) != dt or keys.dtype != sorted_keys.dtype:
        raise TypeError("keys and sorted_keys must have the same dtype")
    if out is None:
        out = torch.empty(keys.numel(), dtype=torch.int64, device=keys.device)
    _gpu(out, "out")
    if out.dtype != torch.int64 or out.numel() != keys.numel():
        raise ValueError("out must be an int64 tensor with one element per key")
    with torch.cuda.device(keys.device):
        _check(getattr(load_library(), fn)(sorted_keys.data_ptr(), sorted_keys.numel(), keys.data_ptr(),
                                           keys.numel(), DTYPE_CODE[dt], out.data_ptr(), _stream(keys)), fn)
    return out


def accumulate(x: torch.Tensor, inclusive: bool = True, dtype: str | None = None,
               out: torch.Tensor | None = None) -> torch.Tensor:
    """Prefix sums of ``x`` (ak_accumulate): a new tensor, or ``out`` (which
    may be ``x`` itself for the in-place form)."""
    _gpu(x, "x")
    dt = _dtype(x, dtype)
    if out is None:
        out = torch.empty_like(x)
    _gpu(out, "out")
    if out.dtype != x.dtype or out.numel() != x.numel():
        raise ValueError("out must match x in dtype and size")
    with torch.cuda.device(x.device):
        _check(load_library().ak_accumulate(x.data_ptr(), out.data_ptr(), x.numel(), DTYPE_CODE[dt],
                                            1 if inclusive else 0, _stream(x)), "ak_accumulate")
    return out


def accumulate_(x: torch.Tensor, inclusive: bool = True, dtype: str | None = None) -> torch.Tensor:
    """In-place prefix sums of ``x``."""
    return accumulate(x, inclusive, dtype, out=x)


def searchsortedfirst(sorted_keys: torch.Tensor, keys: torch.Tensor, dtype: str | None = None,
                      out: torch.Tensor | None = None) -> torch.Tensor:
    """0-based index of the first element of ``sorted_keys`` not below each
    key (len if none), as int64 (ak_searchsortedfirst)."""
    return _search("ak_searchsortedfirst", sorted_keys, keys, dtype, out)


def searchsortedlast(sorted_keys: torch.Tensor, keys: torch.Tensor, dtype: str | None = None,
                     out: torch.Tensor | None = None) -> torch.Tensor:
    """0-based index of the last element of ``sorted_keys`` not above each
    key (-1 if none), as int64 (ak_searchsortedlast)."""
    return _search("ak_searchsortedlast", sorted_keys, keys, dtype, out)


def sort_route() -> dict:
    """How the last sort_ / sortperm call on the current stream ordered its
    keys: {"prefix_places", "passes", "chunks", "fallback_runs",
    "fallback_keys"} (waits for the stream)."""
    info = (ctypes.c_int64 * 5)()
    _check(load_library().ak_sort_route(info, torch.cuda.current_stream().cuda_stream), "ak_sort_route")
    return dict(zip(("prefix_places", "passes", "chunks", "fallback_runs", "fallback_keys"), list(info)))


def seg_set_tuning(key_bits: int, ipt_a: int, ipt_b: int, grid_mult: int = 4, b_max: int = 0,
                   xl_min: int = 32768) -> None:
    """Override the segmented-sort tuning for 32- or 64-bit keys."""
    _check(load_library().ak_seg_set_tuning(key_bits, ipt_a, ipt_b, grid_mult, b_max, xl_min),
           "ak_seg_set_tuning")


def temp_bytes(op: str, n: int, dtype: str) -> int:
    return int(load_library().ak_temp_bytes(OPS[op], n, DTYPE_CODE[dtype]))


def temp_bytes_segmented(n: int, nseg: int, dtype: str) -> int:
    return int(load_library().ak_temp_bytes_segmented(n, nseg, DTYPE_CODE[dtype]))


def set_workspace(arena=None) -> None:
    """Binds a caller-owned uint8 CUDA tensor as the scratch arena of the
    current stream (None unbinds).  The caller keeps the tensor alive while
    it is bound."""
    if arena is None:
        _check(load_library().ak_set_workspace(None, 0, torch.cuda.current_stream().cuda_stream),
               "ak_set_workspace")
        return
    if not arena.is_cuda or not arena.is_contiguous():
        raise ValueError("the arena must be a contiguous CUDA tensor")
    nbytes = arena.numel() * arena.element_size()
    _check(load_library().ak_set_workspace(arena.data_ptr(), nbytes, _stream(arena)), "ak_set_workspace")


def release_workspace() -> None:
    _check(load_library().ak_release_workspace(), "ak_release_workspace")
