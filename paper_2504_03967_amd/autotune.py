"""Autotuned tile shapes, cached per (device, qubit count, precision).

The search itself is the library's qg_autotune (timed single-gate passes per pass
class, then per target qubit); this module only stores and re-applies its result:
the class table and the per-target entries.  The cache is a JSON file at
$QG_AUTOTUNE_CACHE (default ~/.cache/qgear-mi355x/autotune.json).
"""
from __future__ import annotations

import json
import os
from typing import List

import torch

from . import qg

N_CLASSES = 5
N_TARGETS = 64
TARGET_FIELDS = ("tile", "reg", "swz", "xcd")


def cache_path() -> str:
    return os.environ.get("QG_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "qgear-mi355x", "autotune.json"))


def apply(table, dtype: str) -> None:
    for cls, (tile, reg, swz) in enumerate(table):
        qg.set_tuning(f"cls{cls}_tile_{dtype}", int(tile))
        qg.set_tuning(f"cls{cls}_reg_{dtype}", int(reg))
        qg.set_tuning(f"cls{cls}_swz_{dtype}", int(swz))


def current(dtype: str) -> List[List[int]]:
    return [[qg.get_tuning(f"cls{c}_{w}_{dtype}") for w in ("tile", "reg", "swz")] for c in range(N_CLASSES)]


def current_targets(dtype: str) -> List[List[int]]:
    """Per target qubit: [tile, reg, swz, xcd]; tile 0 = the class's shape."""
    return [[qg.get_tuning(f"tgt{q}_{w}_{dtype}") for w in TARGET_FIELDS] for q in range(N_TARGETS)]


def apply_targets(targets, dtype: str) -> None:
    for q, entry in enumerate(targets):
        for w, v in zip(TARGET_FIELDS, entry):
            qg.set_tuning(f"tgt{q}_{w}_{dtype}", int(v))


def snapshot(dtype: str):
    """Everything the autotuner sets for dtype (to restore it afterwards)."""
    return current(dtype), current_targets(dtype)


def restore(snap, dtype: str) -> None:
    apply(snap[0], dtype)
    apply_targets(snap[1], dtype)


def tuned(n: int, dtype: str = "c128", reps: int = 3, use_cache: bool = True):
    """(table, source): the class table for (device, n, dtype), from the cache or a fresh
    search; the per-target entries are installed as well."""
    key = f"{torch.cuda.get_device_name(0)}|{qg.version()}|n={n}|{dtype}"
    path = cache_path()
    data = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                data = json.load(f)
        except (OSError, ValueError):
            data = {}
    entry = data.get(key)
    if isinstance(entry, dict) and "classes" in entry and "targets" in entry:
        apply(entry["classes"], dtype)
        apply_targets(entry["targets"], dtype)
        return entry["classes"], "cache"
    st = qg.State(n, dtype)
    table = st.autotune(reps).tolist()
    st.close()
    data[key] = {"classes": table, "targets": current_targets(dtype)}
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(data, f, indent=1)
        except OSError:
            pass
    return table, "search"
