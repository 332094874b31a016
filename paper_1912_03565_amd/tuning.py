"""Persistent autotune cache: the launch-shape choices found by cs3d_autotune /
cs3d_batch_autotune, stored as JSON keyed by device, problem shape, scheme,
precision and number of right-hand sides.

    plan = Plan(...); tuned_plan(plan, f)         # look up, or tune and store
    batch = Batch(members); tuned_batch(batch, fs)

The cache file is CS3D_TUNE_CACHE, else ~/.cache/cs3d/tuning.json.  CS3D_AUTOTUNE=0
turns tuning off (the defaults are kept and nothing is written).  The choices change
launch shapes: results are bitwise the same for every entry, except that another radix
split of a y-line (ywpl, plans) and packed lines (pack, batches) change the rounding only.
"""
import hashlib
import json
import os
import tempfile

import torch


def cache_path():
    return os.environ.get("CS3D_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "cs3d",
                                                              "tuning.json")


def enabled():
    return os.environ.get("CS3D_AUTOTUNE", "1") not in ("0", "off", "false")


def _device_name(device):
    try:
        return torch.cuda.get_device_name(device)
    except Exception:
        return "unknown"


def plan_key(plan, nrhs):
    return "|".join([_device_name(plan.device), "plan", f"{plan.nx}x{plan.ny}x{plan.nz}", plan.scheme,
                     plan.precision, f"rhs{nrhs}"])


def batch_key(batch, schemes):
    desc = ";".join(f"{nx}x{ny}x{nz}:{s}" for (nx, ny, nz), s in zip(batch.shapes, schemes))
    return "|".join([_device_name(batch.device), "batch", f"n{len(batch)}",
                     hashlib.sha1(desc.encode()).hexdigest()[:16]])


def load(path=None):
    path = path or cache_path()
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key, entry, path=None):
    """Add one entry; the file is replaced atomically."""
    path = path or cache_path()
    data = load(path)
    data[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned_plan(plan, f, out=None, reps=2, path=None):
    """Apply the cached choice for this plan and right-hand-side count, or autotune on f
    and cache the result.  Returns the tuning in use."""
    nrhs = f.shape[0]
    if not enabled():
        return plan.tuning()
    key = plan_key(plan, nrhs)
    hit = load(path).get(key)
    if hit:
        plan.set_tuning(hit["tuning"])
        return plan.tuning()
    t, ms = plan.autotune(f, out=out, reps=reps)
    store(key, {"tuning": t, "ms": ms}, path)
    return t


def tuned_batch(batch, fs, schemes, us=None, reps=2, path=None):
    """As tuned_plan for a Batch (schemes: the members' scheme names, part of the key)."""
    if not enabled():
        return batch.tuning()
    key = batch_key(batch, schemes)
    hit = load(path).get(key)
    if hit:
        batch.set_tuning(hit["tuning"])
        return batch.tuning()
    t, ms = batch.autotune(fs, us=us, reps=reps)
    store(key, {"tuning": t, "ms": ms}, path)
    return t
