"""Autotuned batch schedules, cached on disk.

jxlr_autotune (native) times the candidate workgroup counts and tile orders
of each persistent stage kernel for one prepared batch.  The choice depends
on the device and on the batch's shape (how many tiles, how many EPF passes),
not on its pixel values, so it is cached under a key made of the device
(architecture and compute-unit count), the tile count rounded to a power of
two and the largest EPF pass count.
The cache is a JSON file at $JXLR_TUNE_CACHE, else ~/.cache/jxlr/schedules.json.
"""
import json
import math
import os

from . import jxlr as J


def cache_path():
    return os.environ.get("JXLR_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "jxlr", "schedules.json"))


def batch_key(device_name, plan):
    bucket = 1 << max(0, round(math.log2(max(1, plan.total_tiles))))
    return f"{device_name}|tiles~{bucket}|epf{plan.max_epf_iters}"


def _load(path):
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path, cache):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned_config(ctx, plan, stream=None, reps=5, path=None, retune=False):
    """Returns (LaunchConfig, info dict).  Tunes on a cache miss (or when
    retune is set) and records the result."""
    import torch
    path = path or cache_path()
    # the architecture and compute-unit count name the device (the marketing
    # name can read differently under a profiler)
    props = torch.cuda.get_device_properties(ctx.device)
    name = f"{props.gcnArchName.split(':')[0]}x{props.multi_processor_count}"
    key = batch_key(name, plan)
    cache = _load(path)
    ent = cache.get(key)
    if ent and not retune:
        cfg = J.LaunchConfig(**{k: int(ent[k]) for k, _ in J.LaunchConfig._fields_})
        return cfg, dict(key=key, cached=True, tuned_ms=ent.get("tuned_ms"))
    cfg, ms = ctx.autotune(plan, reps=reps, stream=stream)
    ent = cfg.as_dict()
    ent["tuned_ms"] = ms
    cache[key] = ent
    try:
        _store(path, cache)
    except OSError:
        pass  # a read-only home only loses the cache
    return cfg, dict(key=key, cached=False, tuned_ms=ms)
