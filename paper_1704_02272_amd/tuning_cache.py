"""JSON cache of autotuned launch choices.

The autotuner (``pfac_tune`` in the library) measures a sample workload; its result
depends on the pattern set, the alphabet, the workload's shape and the device, so the
cache keys on exactly those. A hit applies the stored tuning with ``pfac_set_tuning``
and skips the measurement.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import pfac


def cache_key(patterns, alphabet: int, n_bytes: int, n_pkts: int, device_name: str) -> str:
    h = hashlib.sha256()
    for p in patterns:
        h.update(len(p).to_bytes(4, "little"))
        h.update(bytes(p))
    return "%s|a%d|n%d|p%d|%s|v%d" % (h.hexdigest()[:24], alphabet, n_bytes, n_pkts, device_name,
                                      pfac.pfac_version())


def _load(path: str) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def tune_cached(a, patterns, alphabet: int, data, offsets=None, path: str = "", reps: int = 5,
                stream=None) -> dict:
    """Tuning for this automaton and workload shape: from the cache at ``path`` when
    present, else measured with ``pfac_tune`` and stored there."""
    import torch
    n_pk = offsets.numel() - 1 if offsets is not None else 0
    key = cache_key(patterns, alphabet, data.numel(), n_pk, torch.cuda.get_device_name(data.device))
    table = _load(path)
    if key in table:
        t = table[key]
        pfac.pfac_set_tuning(a, **{k: t[k] for k in pfac.TUNING_FIELDS})
        return dict(t, cached=True)
    t = pfac.pfac_tune(a, data, offsets, reps=reps, stream=stream)
    if path:
        table[key] = t
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return dict(t, cached=False)
