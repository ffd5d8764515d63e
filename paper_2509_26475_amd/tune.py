"""Autotuner of batched launches: the cost model of a plan (the constants of
one Taylor term's time, phicomb_batch_model) is fitted by the library from
the device clocks of every run; this module keeps the fitted constants in an
on-disk cache, keyed by device and operator kind, so that a new plan starts
from the schedule the earlier runs found instead of the built-in constants.

    b = tuned_batch_create(items, precision)         # cached model if any
    tune_batch(b, count, runs=2)                      # runs; refits; caches

Plain marshalling around the C ABI plus a JSON file; no kernel code."""
from __future__ import annotations

import json
import os
from typing import Optional

from . import (FP64, phicomb_batch_create, phicomb_batch_fit, phicomb_batch_model,
               phicomb_batch_run, OK, PhicombError)

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "phicomb", "batch_models.json")


def _device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"


def cache_key(kind: str, precision: int) -> str:
    return f"{_device_key()}|{kind}|{'fp64' if precision == FP64 else 'mixed'}"


def load_cache(path: Optional[str] = None) -> dict:
    path = path or DEFAULT_CACHE
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: Optional[str] = None) -> None:
    path = path or DEFAULT_CACHE
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned_batch_create(items, precision: int, kind: str, cache_path: Optional[str] = None):
    """phicomb_batch_create, then the cached model for (device, kind,
    precision) if one exists.  Returns (plan, whether a cached model was
    applied)."""
    b = phicomb_batch_create(items, precision)
    model = load_cache(cache_path).get(cache_key(kind, precision))
    if model is not None:
        try:
            phicomb_batch_model(b, model)
            return b, True
        except PhicombError:
            pass
    return b, False


def tune_batch(b, count: int, kind: str, precision: int, runs: int = 2,
               cache_path: Optional[str] = None) -> dict:
    """Runs the plan `runs` times (each run refits the model and may rebuild
    the schedule), stores the final model in the cache and returns the fit
    record of the last run."""
    fit = None
    for _ in range(runs):
        st, _stats = phicomb_batch_run(b, count)
        if st != OK:
            raise PhicombError(st, "phicomb_batch_run")
        fit = phicomb_batch_fit(b)
    cache = load_cache(cache_path)
    cache[cache_key(kind, precision)] = phicomb_batch_model(b)
    save_cache(cache, cache_path)
    return fit
