"""Launch-shape autotuning for the batched float-float reductions.

The search runs natively: ``ff_dot_batched_autotune`` (C ABI) times every
candidate shape with HIP events on the caller's stream.  This module only
keys the winners by device (architecture, compute-unit count) and by a
coarse batch shape class, and keeps them in a JSON file so that later runs
reuse them without searching.

Cache file: ``$FF_AUTOTUNE_CACHE`` or ``~/.cache/libff/autotune.json``.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import threading

import torch

from ._lib import DotCfg, check, lib

_LOCK = threading.Lock()
_MEMO: dict | None = None


def cache_path() -> str:
    return os.environ.get("FF_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "libff", "autotune.json"))


def device_key(device) -> str:
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", "unknown").split(":")[0]
    return f"{arch}-cu{props.multi_processor_count}"


# Version of the launch-shape format (block, chunk, grid, unroll) the entries
# hold: entries of another version are not reused.
SHAPE_FORMAT = 2


def shape_class(total_len: int, nvec: int) -> str:
    """Batches whose total length and vector count agree to a factor of two
    share one entry."""
    return (f"dot{SHAPE_FORMAT}-t{int(math.log2(total_len + 1))}"
            f"-v{int(math.log2(nvec + 1))}")


def _load() -> dict:
    global _MEMO
    if _MEMO is None:
        try:
            with open(cache_path()) as f:
                _MEMO = json.load(f)
        except (OSError, ValueError):
            _MEMO = {}
    return _MEMO


def _store(entries: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(entries, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass   # an unwritable cache only costs a new search next time


def tune_dot(x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor, reps: int = 3,
             stream=None):
    """Search the launch shape of ``ff_dot_batched`` on this batch.
    Returns ((block, chunk, grid, unroll), mean milliseconds)."""
    nvec = offsets.numel() - 1
    total = x.numel()
    smallest = DotCfg(64, 256, 0, 4)   # the search's smallest chunk
    nbytes = int(lib.ff_dot_batched_workspace_size(total, nvec, ctypes.byref(smallest)))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=x.device)
    out = torch.empty((2, nvec), dtype=torch.float32, device=x.device)
    best = DotCfg()
    best_ms = ctypes.c_float()
    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    with torch.cuda.device(x.device):
        check("ff_dot_batched_autotune", lib.ff_dot_batched_autotune(
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
            ctypes.c_void_p(offsets.data_ptr()), nvec, total, ctypes.c_void_p(ws.data_ptr()),
            ws.numel(), ctypes.c_void_p(out[0].data_ptr()), ctypes.c_void_p(out[1].data_ptr()),
            int(reps), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(best),
            ctypes.byref(best_ms)))
    return best.as_tuple(), float(best_ms.value)


def dot_cfg(x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor, search: bool = True):
    """Cached launch shape for this batch's class, searched on a miss when
    ``search`` is true (else None on a miss)."""
    key = f"{device_key(x.device)}/{shape_class(x.numel(), offsets.numel() - 1)}"
    with _LOCK:
        entries = _load()
        hit = entries.get(key)
    if hit is not None:
        return tuple(hit["cfg"])
    if not search:
        return None
    cfg, ms = tune_dot(x, y, offsets)
    with _LOCK:
        entries = _load()
        entries[key] = {"cfg": list(cfg), "ms": ms, "total_len": int(x.numel()),
                        "nvec": int(offsets.numel() - 1)}
        _store(entries)
    return cfg
