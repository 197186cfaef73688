"""Helpers for the GPU tests: device buffers (torch) around the C-ABI calls."""
import numpy as np

from paper_2601_03187_amd import synth
from paper_2601_03187_amd import tang as T


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def to_dev(arr: np.ndarray):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(arr).view(np.uint8).reshape(-1).copy()).cuda()


def classify_dev(rs, hdr: np.ndarray, stats: bool = False):
    """tang_classify on device buffers with torch's current stream."""
    torch = torch_cuda()
    d_hdr = to_dev(hdr) if len(hdr) else torch.empty(16, dtype=torch.uint8, device="cuda")
    d_out = torch.full((max(1, len(hdr)),), -7, dtype=torch.int32, device="cuda")
    st = T.tang_classify(rs, d_hdr, d_out, len(hdr), torch.cuda.current_stream(), want_stats=stats)
    torch.cuda.synchronize()
    got = d_out.cpu().numpy().view(np.uint32)[: len(hdr)].copy()
    return (got, st) if stats else got


def mlp_dev(rs, hdr: np.ndarray, n_out: int, topk: int = 1):
    torch = torch_cuda()
    n = len(hdr)
    d_hdr = to_dev(hdr)
    logits = torch.full((n * n_out,), float("nan"), dtype=torch.float32, device="cuda")
    cand = torch.full((n * topk,), -1, dtype=torch.int16, device="cuda")
    T.tang_mlp_forward(rs, d_hdr, n, logits, cand, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return logits.cpu().numpy().reshape(n, n_out), cand.cpu().numpy().view(np.uint16).reshape(n, topk)


def keys_of(rules: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """(priority << 32 | id) of the given rule ids (no-match -> 2^64-1)."""
    order = np.argsort(rules["id"])
    sid = rules["id"][order]
    pos = np.searchsorted(sid, ids)
    pos = np.minimum(pos, len(sid) - 1)
    found = sid[pos] == ids
    r = rules[order[pos]]
    k = (r["priority"].astype(np.uint64) << np.uint64(32)) | r["id"].astype(np.uint64)
    return np.where(found, k, np.uint64(0xFFFFFFFFFFFFFFFF))
