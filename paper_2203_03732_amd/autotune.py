"""Persistent choices of the batch autotuner.

`prot_batch_autotune` (C++) times every configuration of a batched solve
(LDS engine or teams of 1..8 workgroups per instance, and for d >= 16 both
cost paths) on real inputs. This module keeps the winner per device and
workload class in a JSON file, so a later batch of the same class is planned
without timing again:

    key = arch | n_max bucket | mean-n bucket | batch bucket | d | eps | mode | origin

Buckets are the next power of two. The file is PROT_TUNE_CACHE, else
~/.cache/paper_2203_03732_amd/batch_tuning.json.
"""
from __future__ import annotations

import json
import os


def _bucket(x: float) -> int:
    b = 1
    while b < x:
        b *= 2
    return b


def cache_key(arch: str, ns, d: int, eps: float, eps_mode: str = "algorithmic",
              origin: str = "diag") -> str:
    ns = [int(v) for v in ns]
    n_max = max(ns) if ns else 0
    mean = sum(ns) / len(ns) if ns else 0.0
    return (f"{arch.split(':')[0]}|nmax{_bucket(n_max)}|nmean{_bucket(mean)}|"
            f"batch{_bucket(len(ns))}|d{int(d)}|eps{float(eps)!r}|{eps_mode}|{origin}")


def cache_path() -> str:
    return os.environ.get("PROT_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2203_03732_amd", "batch_tuning.json")


def load(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key: str, entry: dict, path: str | None = None) -> None:
    path = path or cache_path()
    data = load(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned_batch(ctx, ns, d: int, eps: float, X, Y, *, reps: int = 3, path: str | None = None,
                eps_mode: str = "algorithmic", origin: str = "diag", arch: str | None = None,
                **kw):
    """A Batch planned with the cached best configuration for this workload
    class, timing the candidates on X, Y first when the class is new."""
    if arch is None:
        import torch
        arch = torch.cuda.get_device_properties(ctx.device).gcnArchName
    key = cache_key(arch, ns, d, eps, eps_mode, origin)
    entry = load(path).get(key)
    if entry is None:
        cfg, ms, tried = ctx.autotune_batch(ns, d, eps, X, Y, reps=reps, eps_mode=eps_mode,
                                            origin=origin)
        entry = dict(cfg, ms=ms, tried=tried)
        store(key, entry, path)
    config = {k: entry[k] for k in ("engine", "team", "cost_path")}
    return ctx.batch(ns, d, eps, eps_mode=eps_mode, origin=origin, config=config, **kw)
