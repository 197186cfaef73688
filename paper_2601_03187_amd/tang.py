"""ctypes binding of libtang.so (include/tang.h). Argument marshalling only.

Every function keeps the C name. Device buffers may be passed as integers (device
addresses, unchecked) or as torch tensors (checked: on a GPU, contiguous, and large
enough for the call's n, so a wrong n raises instead of reaching past a buffer's end);
streams as integers or
objects with a ``cuda_stream`` attribute (torch streams). A non-zero return code raises
``TangError`` carrying the library's message. Nothing here computes any part of the
classification: if the library is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .synth import HDR_DTYPE, RULE_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtang.so")

TANG_NO_MATCH = 0xFFFFFFFF
TANG_HOST_ONLY = -1
TANG_MAX_TUPLES = 512
TANG_NOALLOC_MAX_HEADERS = 262144
TANG_FP32, TANG_BF16, TANG_FP8 = 0, 1, 2
PRECISIONS = {"fp32": TANG_FP32, "bf16": TANG_BF16, "fp8": TANG_FP8}
ERRORS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ENOTFOUND", -4: "EEXIST", -5: "EDEVICE",
          -6: "EBUSY", -7: "ETIMEOUT"}


class TangError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class tang_mlp_desc_t(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_uint32), ("dims", ctypes.c_uint32 * 9), ("topk", ctypes.c_uint32)]


class tang_resnet_desc_t(ctypes.Structure):
    _fields_ = [("width", ctypes.c_uint32), ("n_blocks", ctypes.c_uint32), ("n_out", ctypes.c_uint32),
                ("topk", ctypes.c_uint32)]


class tang_stats_t(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in
                ("packets", "probes", "slots", "records", "top1_hits", "fallbacks", "no_match",
                 "filter_checks", "wave_steps", "wave_rounds")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class tang_server_cfg_t(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_size_t), ("max_inflight_packets", ctypes.c_uint32),
                ("n_streams", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("use_graphs", ctypes.c_uint32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_03187_amd.build`")
# One HIP runtime per process: torch ships its own libamdhip64 (soname libamdhip64.so.7),
# which its libraries load by an unversioned name. Importing torch first makes the
# library's libamdhip64.so.7 dependency bind to that already-loaded runtime instead of
# loading a second HIP/HSA runtime from /opt/rocm next to it.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is only plumbing for device buffers
    torch = None
_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
# tang_alloc_fn / tang_free_fn
ALLOC_FN = ctypes.CFUNCTYPE(_P, ctypes.c_size_t, ctypes.c_int, _P)
FREE_FN = ctypes.CFUNCTYPE(None, _P, ctypes.c_int, _P)
_sigs = {
    "tang_set_allocator": (ctypes.c_int, [ALLOC_FN, FREE_FN, _P]),
    "tang_ruleset_create": (ctypes.c_int, [ctypes.c_int, _P, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "tang_ruleset_destroy": (None, [_P]),
    "tang_ruleset_num_tuples": (ctypes.c_uint32, [_P]),
    "tang_ruleset_tuple": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint8),
                                          ctypes.POINTER(ctypes.c_uint8)]),
    "tang_ruleset_num_rules": (ctypes.c_size_t, [_P]),
    "tang_ruleset_rule_tuple": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
    "tang_ruleset_conflict_mask": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
    "tang_ruleset_conflict_mask_words": (ctypes.c_int, [_P, ctypes.c_uint32, _P, ctypes.c_uint32]),
    "tang_ruleset_device_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "tang_ruleset_set_stream": (ctypes.c_int, [_P, _P]),
    "tang_model_load": (ctypes.c_int, [_P, ctypes.POINTER(tang_mlp_desc_t), _P, _P, ctypes.c_int, _P]),
    "tang_model_load_resnet": (ctypes.c_int, [_P, ctypes.POINTER(tang_resnet_desc_t), _P, _P, ctypes.c_int]),
    "tang_ruleset_coarse_rules": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "tang_search_host": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_size_t, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_int, ctypes.POINTER(tang_stats_t)]),
    "tang_ruleset_export": (ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "tang_model_unload": (ctypes.c_int, [_P]),
    "tang_classify": (ctypes.c_int, [_P, _P, _P, ctypes.c_size_t, _P, ctypes.POINTER(tang_stats_t)]),
    "tang_predict": (ctypes.c_int, [_P, _P, _P, ctypes.c_size_t, _P]),
    "tang_search": (ctypes.c_int, [_P, _P, _P, ctypes.c_size_t, _P, ctypes.POINTER(tang_stats_t)]),
    "tang_classify_host": (ctypes.c_int, [_P, _P, _P, ctypes.c_size_t, ctypes.POINTER(tang_stats_t)]),
    "tang_classify_host_noalloc": (ctypes.c_int, [_P, _P, _P, ctypes.c_size_t,
                                                  ctypes.POINTER(tang_stats_t)]),
    "tang_mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, _P, _P]),
    "tang_insert": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "tang_delete": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "tang_last_error": (ctypes.c_char_p, []),
    "tang_server_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(tang_server_cfg_t), ctypes.POINTER(_P)]),
    "tang_server_add_ruleset": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_uint32)]),
    "tang_server_prepare": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "tang_server_submit": (ctypes.c_int, [_P, ctypes.c_uint32, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "tang_server_wait": (ctypes.c_int, [_P, ctypes.c_int64]),
    "tang_server_poll": (ctypes.c_int, [_P]),
    "tang_server_req_times": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    "tang_server_req_free": (None, [_P]),
    "tang_server_destroy": (ctypes.c_int, [_P]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sigs)


def _check(rc: int):
    if rc != 0:
        raise TangError(rc, _lib.tang_last_error().decode())


def _dbuf(x, nbytes: int, what: str):
    """Device pointer for a call that reads or writes nbytes through it. A torch tensor is
    checked (on a GPU, contiguous, large enough) so that a wrong n cannot send a kernel
    past the buffer's end; an int is taken as the caller's own device pointer; None goes
    through (the library rejects it when n > 0)."""
    if x is None or isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if not x.is_cuda:
            raise ValueError(f"{what}: a device tensor is needed")
        if not x.is_contiguous():
            raise ValueError(f"{what}: the tensor must be contiguous")
        have = x.numel() * x.element_size()
        if have < nbytes:
            raise ValueError(f"{what}: {have} bytes, the call needs {nbytes}")
        return x.data_ptr()
    raise TypeError(f"{what}: a device tensor or an int device pointer is needed, not {type(x)}")


_model_topk = {}  # ruleset handle -> candidates per header of its loaded model


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _rules(rules) -> np.ndarray:
    r = np.ascontiguousarray(rules)
    if r.dtype != RULE_DTYPE:
        raise TypeError("rules must use RULE_DTYPE")
    return r


# --- rulesets ---------------------------------------------------------------------------

def tang_ruleset_create(device: int, rules) -> int:
    r = _rules(rules)
    out = _P()
    _check(_lib.tang_ruleset_create(device, r.ctypes.data if len(r) else None, len(r), ctypes.byref(out)))
    return out.value


def tang_ruleset_destroy(rs: int) -> None:
    _lib.tang_ruleset_destroy(rs)
    _model_topk.pop(rs, None)


def tang_ruleset_num_tuples(rs: int) -> int:
    return int(_lib.tang_ruleset_num_tuples(rs))


def tang_ruleset_tuple(rs: int, t: int):
    a, b = ctypes.c_uint8(), ctypes.c_uint8()
    _check(_lib.tang_ruleset_tuple(rs, t, ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def tang_ruleset_num_rules(rs: int) -> int:
    return int(_lib.tang_ruleset_num_rules(rs))


def tang_ruleset_rule_tuple(rs: int, rule_id: int) -> int:
    t = ctypes.c_uint32()
    _check(_lib.tang_ruleset_rule_tuple(rs, rule_id, ctypes.byref(t)))
    return int(t.value)


def tang_ruleset_conflict_mask(rs: int, rule_id: int) -> int:
    """The whole conflict mask as a Python int (bit t = tuple t, up to TANG_MAX_TUPLES)."""
    nw = TANG_MAX_TUPLES // 32
    words = (ctypes.c_uint32 * nw)()
    _check(_lib.tang_ruleset_conflict_mask_words(rs, rule_id, ctypes.cast(words, _P), nw))
    return sum(int(w) << (32 * i) for i, w in enumerate(words))


def tang_ruleset_device_bytes(rs: int) -> int:
    b = ctypes.c_size_t()
    _check(_lib.tang_ruleset_device_bytes(rs, ctypes.byref(b)))
    return int(b.value)


def tang_ruleset_set_stream(rs: int, stream) -> None:
    _check(_lib.tang_ruleset_set_stream(rs, _stream(stream)))


# --- model ------------------------------------------------------------------------------

def tang_model_load(rs: int, Ws, bs, precision="fp32", topk: int = 1, act_scales=None) -> None:
    """Ws[l]: [out][in] float32 arrays (nn.Linear.weight layout); bs[l]: [out]."""
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    Ws = [np.ascontiguousarray(np.asarray(w, dtype=np.float32)) for w in Ws]
    bs = [np.ascontiguousarray(np.asarray(b, dtype=np.float32)) for b in bs]
    d = tang_mlp_desc_t()
    d.n_layers = len(Ws)
    dims = [Ws[0].shape[1]] + [w.shape[0] for w in Ws]
    for i, v in enumerate(dims):
        d.dims[i] = v
    d.topk = topk
    wp = (ctypes.c_void_p * len(Ws))(*[w.ctypes.data for w in Ws])
    bp = (ctypes.c_void_p * len(bs))(*[b.ctypes.data for b in bs])
    sc = None
    if act_scales is not None:
        sc = np.ascontiguousarray(np.asarray(act_scales, dtype=np.float32))
    _check(_lib.tang_model_load(rs, ctypes.byref(d), ctypes.cast(wp, _P), ctypes.cast(bp, _P), p,
                                sc.ctypes.data if sc is not None else None))
    _model_topk[rs] = int(topk)


def tang_search_host(rs: int, hdr: np.ndarray, cand=None, kcand: int = 0, threads: int = 1,
                     exact: bool = True, out=None, want_stats: bool = False):
    """Host search (the paper's CPU side); hdr: HDR_DTYPE array, cand: uint32 candidate
    words or None. Returns the rule ids (and the stats dict when asked). The call releases
    the GIL (ctypes), so a Python thread can run it beside GPU work."""
    hdr = np.ascontiguousarray(hdr)
    if hdr.dtype != HDR_DTYPE:
        raise TypeError("headers must use HDR_DTYPE")
    out = np.empty(len(hdr), dtype=np.uint32) if out is None else out
    c = None if cand is None else np.ascontiguousarray(cand, dtype=np.uint32)
    st = tang_stats_t() if want_stats else None
    _check(_lib.tang_search_host(rs, hdr.ctypes.data if len(hdr) else None,
                                 c.ctypes.data if c is not None and len(c) else None,
                                 out.ctypes.data if len(out) else None, len(hdr),
                                 kcand if c is not None else 0, threads, 1 if exact else 0,
                                 ctypes.byref(st) if st is not None else None))
    return (out, st.as_dict()) if want_stats else out


def tang_ruleset_coarse_rules(rs: int) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib.tang_ruleset_coarse_rules(rs, ctypes.byref(n)))
    return int(n.value)


def tang_ruleset_export(rs: int) -> np.ndarray:
    """Live rules (RULE_DTYPE), normalised, in ascending (priority, id) order."""
    n = ctypes.c_size_t(0)
    _check(_lib.tang_ruleset_export(rs, None, 0, ctypes.byref(n)))
    out = np.zeros(int(n.value), dtype=RULE_DTYPE)
    if len(out):
        _check(_lib.tang_ruleset_export(rs, out.ctypes.data, len(out), ctypes.byref(n)))
    return out


def tang_model_load_resnet(rs: int, Ws, bs, precision="bf16", topk: int = 1) -> None:
    """The residual predictor: Ws = [W_in (width x 7), then two width x width matrices per
    block, W_out (C x width)], nn.Linear layout; bs likewise."""
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    Ws = [np.ascontiguousarray(np.asarray(w, dtype=np.float32)) for w in Ws]
    bs = [np.ascontiguousarray(np.asarray(b, dtype=np.float32)) for b in bs]
    d = tang_resnet_desc_t(Ws[0].shape[0], (len(Ws) - 2) // 2, Ws[-1].shape[0], topk)
    wp = (ctypes.c_void_p * len(Ws))(*[w.ctypes.data for w in Ws])
    bp = (ctypes.c_void_p * len(bs))(*[b.ctypes.data for b in bs])
    _check(_lib.tang_model_load_resnet(rs, ctypes.byref(d), ctypes.cast(wp, _P), ctypes.cast(bp, _P), p))
    _model_topk[rs] = int(topk)


def tang_model_unload(rs: int) -> None:
    _check(_lib.tang_model_unload(rs))
    _model_topk.pop(rs, None)


# --- classify ---------------------------------------------------------------------------

def tang_classify(rs: int, d_hdr, d_rule_id, n: int, stream=None, want_stats: bool = False):
    st = tang_stats_t() if want_stats else None
    _check(_lib.tang_classify(rs, _dbuf(d_hdr, 16 * n, "d_hdr"), _dbuf(d_rule_id, 4 * n, "d_rule_id"),
                              n, _stream(stream),
                              ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def tang_predict(rs: int, d_hdr, d_io, n: int, stream=None) -> None:
    _check(_lib.tang_predict(rs, _dbuf(d_hdr, 16 * n, "d_hdr"), _dbuf(d_io, 4 * n, "d_io"), n,
                             _stream(stream)))


def tang_search(rs: int, d_hdr, d_io, n: int, stream=None, want_stats: bool = False):
    st = tang_stats_t() if want_stats else None
    _check(_lib.tang_search(rs, _dbuf(d_hdr, 16 * n, "d_hdr"), _dbuf(d_io, 4 * n, "d_io"), n,
                            _stream(stream),
                            ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def tang_classify_host(rs: int, hdr: np.ndarray, want_stats: bool = False):
    h = np.ascontiguousarray(hdr)
    if h.dtype != HDR_DTYPE:
        raise TypeError("headers must use HDR_DTYPE")
    out = np.empty(len(h), dtype=np.uint32)
    st = tang_stats_t() if want_stats else None
    _check(_lib.tang_classify_host(rs, h.ctypes.data if len(h) else None,
                                   out.ctypes.data if len(h) else None, len(h),
                                   ctypes.byref(st) if st is not None else None))
    return (out, st.as_dict()) if want_stats else out


def tang_classify_host_noalloc(rs: int, hdr: np.ndarray, want_stats: bool = False):
    """tang_classify_host staged through the library's static device array (no device
    allocation; at most TANG_NOALLOC_MAX_HEADERS headers per call)."""
    h = np.ascontiguousarray(hdr)
    if h.dtype != HDR_DTYPE:
        raise TypeError("headers must use HDR_DTYPE")
    out = np.empty(len(h), dtype=np.uint32)
    st = tang_stats_t() if want_stats else None
    _check(_lib.tang_classify_host_noalloc(rs, h.ctypes.data if len(h) else None,
                                           out.ctypes.data if len(h) else None, len(h),
                                           ctypes.byref(st) if st is not None else None))
    return (out, st.as_dict()) if want_stats else out


def tang_mlp_forward(rs: int, d_hdr, n: int, d_logits=None, d_cand=None, stream=None) -> None:
    C = tang_ruleset_num_tuples(rs)
    k = _model_topk.get(rs, 1)
    _check(_lib.tang_mlp_forward(rs, _dbuf(d_hdr, 16 * n, "d_hdr"), n,
                                 _dbuf(d_logits, 4 * n * C, "d_logits"),
                                 _dbuf(d_cand, 2 * n * k, "d_cand"), _stream(stream)))


# --- updates ----------------------------------------------------------------------------

def tang_insert(rs: int, rules) -> None:
    r = _rules(rules)
    _check(_lib.tang_insert(rs, r.ctypes.data if len(r) else None, len(r)))


def tang_delete(rs: int, ids) -> None:
    a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
    _check(_lib.tang_delete(rs, a.ctypes.data if len(a) else None, len(a)))


_allocator_refs = None  # the ctypes callbacks in use (kept alive while installed)


def tang_set_allocator(alloc=None, free=None) -> None:
    """Route the library's internal device memory through alloc(bytes, device) -> int
    pointer (0 on failure) and free(ptr, device); tang_set_allocator() restores hipMalloc."""
    global _allocator_refs
    if alloc is None and free is None:
        _check(_lib.tang_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return
    if alloc is None or free is None:
        _check(_lib.tang_set_allocator(ALLOC_FN(alloc) if alloc else ALLOC_FN(),
                                       FREE_FN(free) if free else FREE_FN(), None))
        return
    a = ALLOC_FN(lambda nbytes, dev, ctx: alloc(nbytes, dev) or None)
    f = FREE_FN(lambda ptr, dev, ctx: free(ptr, dev))
    _check(_lib.tang_set_allocator(a, f, None))
    _allocator_refs = (a, f)


def torch_allocator():
    """(alloc, free) over torch's caching allocator, for tang_set_allocator."""
    import torch

    def alloc(nbytes, dev):
        try:
            return torch.cuda.caching_allocator_alloc(max(int(nbytes), 1), device=dev)
        except RuntimeError:
            return 0

    def free(ptr, dev):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, free


def tang_last_error() -> str:
    return _lib.tang_last_error().decode()


# --- serving ----------------------------------------------------------------------------

def tang_server_create(device: int, mem_budget_bytes=0, max_inflight_packets=0, n_streams=0,
                       max_batch=0, use_graphs=1) -> int:
    c = tang_server_cfg_t(mem_budget_bytes, max_inflight_packets, n_streams, max_batch, use_graphs)
    out = _P()
    _check(_lib.tang_server_create(device, ctypes.byref(c), ctypes.byref(out)))
    return out.value


def tang_server_add_ruleset(srv: int, rs: int) -> int:
    t = ctypes.c_uint32()
    _check(_lib.tang_server_add_ruleset(srv, rs, ctypes.byref(t)))
    return int(t.value)


def tang_server_prepare(srv: int, tag: int) -> None:
    """Record every (size class, slot) graph of ruleset `tag` now (blocks until done)."""
    _check(_lib.tang_server_prepare(srv, tag))


def tang_server_submit(srv: int, tag: int, hdr: np.ndarray, out: np.ndarray) -> int:
    """hdr (HDR_DTYPE) and out (uint32) are host arrays that must outlive the request."""
    assert hdr.dtype == HDR_DTYPE and out.dtype == np.uint32 and hdr.flags.c_contiguous
    req = _P()
    _check(_lib.tang_server_submit(srv, tag, hdr.ctypes.data if len(hdr) else None, len(hdr),
                                   out.ctypes.data if len(out) else None, ctypes.byref(req)))
    return req.value


def tang_server_wait(req: int, timeout_us: int = -1) -> None:
    _check(_lib.tang_server_wait(req, timeout_us))


def tang_server_poll(req: int) -> bool:
    return bool(_lib.tang_server_poll(req))


def tang_server_req_times(req: int):
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(_lib.tang_server_req_times(req, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return int(a.value), int(b.value), int(c.value)


def tang_server_req_free(req: int) -> None:
    _lib.tang_server_req_free(req)


def tang_server_destroy(srv: int) -> None:
    _check(_lib.tang_server_destroy(srv))
