"""Tile autotuning of the reward kernels with a JSON cache.

A cache entry is keyed by the GPU architecture, a hash of the kernel
sources, the dynamics, team size and horizon (and records the sample count it
was tuned at).  `tune` runs d4_autotune for shapes not in the cache and
installs the result; `install_cache` re-installs every cached tile of this
architecture and source version in the current process.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os

import torch

from . import _lib as L

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "d4orm_mi355x_tiles.json")

_I = ctypes.POINTER(ctypes.c_int32)
L.lib().d4_tile_set.argtypes = [ctypes.c_int32] * 6
L.lib().d4_tile_set.restype = ctypes.c_int32
L.lib().d4_tile_get.argtypes = [ctypes.POINTER(L.D4Problem), ctypes.c_int32, _I, _I, _I]
L.lib().d4_tile_get.restype = ctypes.c_int32
L.lib().d4_autotune.argtypes = [ctypes.POINTER(L.D4Problem), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                _I, _I, _I, ctypes.POINTER(ctypes.c_float)]
L.lib().d4_autotune.restype = ctypes.c_int32


def source_version():
    h = hashlib.sha256()
    for f in ("d4_device.hpp", "d4_kernels.hpp", "d4_host.hpp", "d4_api.hip"):
        with open(os.path.join(_HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _arch():
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName


def _key(p):
    return f"{_arch()}|{source_version()}|{p.dyn}|{p.n_robots}|{p.horizon}"


def _load(path):
    if os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def set_tile(dyn, n, horizon, samples_per_group, steps_per_block, replicas=1):
    L._check(L.lib().d4_tile_set(dyn, n, horizon, samples_per_group, steps_per_block, replicas))


def clear_tile(dyn, n, horizon):
    L._check(L.lib().d4_tile_set(dyn, n, horizon, 0, 0, 0))


def get_tile(p, batched=False):
    """(samples per group, steps per block, replicas) the library uses for p."""
    S, Tb, R = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    c = L.to_c(p)
    L._check(L.lib().d4_tile_get(ctypes.byref(c), int(batched), ctypes.byref(S), ctypes.byref(Tb), ctypes.byref(R)))
    return S.value, Tb.value, R.value


def tune(p, x0, goal, path=DEFAULT_CACHE, reps=5, force=False):
    """Tile for problem p: from the cache, else measured now on the start
    states x0 [n][d_x] and goals [n][d_p] (and cached).  The cost of the pair
    checks depends on how close the robots come, so tune on a representative
    instance of the shape."""
    cache = _load(path)
    key = _key(p)
    if key in cache and not force:
        e = cache[key]
        set_tile(p.dyn, p.n_robots, p.horizon, e["S"], e["Tb"], e.get("R", 1))
        return e
    S, Tb, R, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
    c = L.to_c(p)
    x0_d = L._f32(x0).reshape(p.n_robots, p.dx).contiguous()
    g_d = L._f32(goal).reshape(p.n_robots, p.dp).contiguous()
    L._check(L.lib().d4_autotune(ctypes.byref(c), ctypes.c_void_p(x0_d.data_ptr()), ctypes.c_void_p(g_d.data_ptr()),
                                 reps, ctypes.byref(S), ctypes.byref(Tb), ctypes.byref(R), ctypes.byref(us)))
    e = {"S": S.value, "Tb": Tb.value, "R": R.value, "us": us.value, "n_samples": p.n_samples}
    cache[key] = e
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return e


def install_cache(path=DEFAULT_CACHE):
    """Install every cached tile of this architecture and source version; returns how many."""
    prefix = f"{_arch()}|{source_version()}|"
    k = 0
    for key, e in _load(path).items():
        if key.startswith(prefix):
            dyn, n, T = (int(v) for v in key[len(prefix):].split("|"))
            set_tile(dyn, n, T, e["S"], e["Tb"], e.get("R", 1))
            k += 1
    return k


# ------------------------------------------------------------ batched form
L.lib().d4_batch_tile_set.argtypes = [ctypes.c_int32] * 7
L.lib().d4_batch_tile_set.restype = ctypes.c_int32

N_BUCKETS = ((1, 4), (5, 8), (9, 16), (17, 32))
T_BUCKETS = ((1, 80), (81, 120), (121, 100000))


def batch_bucket(p):
    """(dyn, n_lo, n_hi, t_lo, t_hi) of the bucket holding problem p."""
    nb = next(b for b in N_BUCKETS if b[0] <= p.n_robots <= b[1])
    tb = next(b for b in T_BUCKETS if b[0] <= p.horizon <= b[1])
    return (p.dyn, nb[0], nb[1], tb[0], tb[1])


def set_batch_tile(bucket, samples_per_group, steps_per_block):
    L._check(L.lib().d4_batch_tile_set(*bucket, samples_per_group, steps_per_block))


def clear_batch_tile(bucket):
    L._check(L.lib().d4_batch_tile_set(*bucket, 0, 0))


def _candidates(bucket):
    dyn, n_lo, n_hi = bucket[0], bucket[1], bucket[2]
    cs = 4 if dyn == 1 else 2
    S0 = min(64, 256 // n_hi)
    out = []
    for S in sorted({S0, max(1, S0 // 2)}):
        for Tb in (4, 8, 12, 16, 24):
            if Tb % cs == 0:
                out.append((S, Tb))
    return out


def tune_batch(probs, x0s, goals, path=DEFAULT_CACHE, steps=10, min_tiles=1024, force=False, log=None):
    """Tile of every (dynamics, team-size, horizon) bucket of a batch, chosen by
    timing short whole batched iterations (`steps` denoising steps, so the
    timing covers the step sequence and not one step) of a sub-batch of the
    batch's own instances in that bucket, repeated under new instance ids
    until one launch holds at least `min_tiles` reward tiles (so that the
    sub-batch fills the GPU as the whole batch does), with each candidate
    tile; cached per architecture and kernel source version, and installed
    with d4_batch_tile_set, which refuses tiles whose LDS would lower the
    whole batch's occupancy.  A tile changes only speed.  Returns
    {bucket: entry}."""
    import time
    import numpy as np
    cache = _load(path)
    groups = {}
    for j, p in enumerate(probs):
        groups.setdefault(batch_bucket(p), []).append(j)
    chosen = {}
    for bucket, idx in sorted(groups.items()):
        key = f"{_arch()}|{source_version()}|batch|" + "|".join(str(v) for v in bucket) + f"|M{probs[0].n_samples}"
        if key in cache and not force:
            e = cache[key]
            set_batch_tile(bucket, e["S"], e["Tb"])
            chosen[bucket] = e
            continue
        S_rule = min(64, 256 // bucket[2])
        tiles_each = -(-probs[0].n_samples // S_rule)
        reps = -(-min_tiles // (tiles_each * len(idx)))
        sel = [idx[i % len(idx)] for i in range(len(idx) * max(1, reps))]
        sub = [probs[j].replace(n_steps=steps, instance_id=r) for r, j in enumerate(sel)]
        best = None
        for S, Tb in _candidates(bucket):
            try:
                set_batch_tile(bucket, S, Tb)
            except L.D4Error:
                continue
            bc = L.BatchContext(sub, [x0s[j] for j in sel], [goals[j] for j in sel])
            bc.iterate(0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(2):
                bc.iterate(1 + k, sync=False)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / 2 * 1e3
            bc.close()
            if best is None or ms < best["ms"]:
                best = {"S": S, "Tb": Tb, "ms": ms, "instances": len(sel)}
        set_batch_tile(bucket, best["S"], best["Tb"])
        chosen[bucket] = best
        cache[key] = best
        if log:
            log(f"bucket {bucket}: S={best['S']} Tb={best['Tb']} ({best['ms']:.2f} ms for {len(sel)} instances)")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return chosen
