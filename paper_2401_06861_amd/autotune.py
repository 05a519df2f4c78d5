"""Autotuned launch shapes, cached per device and state shape.

`tune(handle)` runs the library's autotuner (nwq_autotune) once per
(device, state kind, qubit count) and stores the chosen launch shape of each
kernel class and target bucket in a JSON file; later calls apply the cached shapes with
nwq_set_launch without timing again.
"""
from __future__ import annotations

import json
import os
from typing import Optional

from . import nwq

DEFAULT_CACHE = os.environ.get("NWQ_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "nwq_tune.json"))
CLASS_IDS = {name: i for i, name in enumerate(nwq.TIMING_CLASSES)}


def _device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', p.name)}|cu{p.multi_processor_count}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(h: int, reps: int = 3, cache_path: Optional[str] = DEFAULT_CACHE, force: bool = False) -> dict:
    """Launch shapes for handle h: {class name: {bucket: [ppt, flags, ms or None]}}
    (flags: bit 0 the non-temporal hint, bit 1 the XCD-contiguous workgroup order)
    (buckets "low", "mid" and "high" of the lowest target bit: 0-2, 3-10, 11 and up).
    The per-target shapes the tuner picks are cached too (under "targets") and
    applied on a cache hit."""
    kind, n, _ = nwq.nwq_info(h)
    key = f"{_device_key()}|{'sv' if kind == nwq.KIND_SV else 'dm'}|n{n}|targets2"
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        for name, per_bucket in cache[key]["buckets"].items():
            for bname, (ppt, nt, _) in per_bucket.items():
                nwq.nwq_set_launch(h, CLASS_IDS[name], nwq.LAUNCH_BUCKETS.index(bname), int(ppt), int(nt))
        for name, per_bit in cache[key]["targets"].items():
            for bit, (ppt, nt) in enumerate(per_bit):
                nwq.nwq_set_launch_target(h, CLASS_IDS[name], bit, int(ppt), int(nt))
        return cache[key]["buckets"]
    ms = nwq.nwq_autotune(h, reps)
    entry = {}
    targets = {}
    for name, per_bucket in ms.items():
        for bname, t in per_bucket.items():
            ppt, nt = nwq.nwq_get_launch(h, CLASS_IDS[name], nwq.LAUNCH_BUCKETS.index(bname))
            entry.setdefault(name, {})[bname] = [ppt, nt, t]
        # per lowest target qubit (the superoperator classes are looked up by qubit too)
        targets[name] = [list(nwq.nwq_get_launch_target(h, CLASS_IDS[name], b)) for b in range(n)]
    if cache_path:
        cache = _load(cache_path)
        cache[key] = {"buckets": entry, "targets": targets}
        os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return entry
