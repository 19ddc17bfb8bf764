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


def tune(p, x0, goal, path=DEFAULT_CACHE, reps=2, force=False):
    """Tile for problem p: from the cache, else measured now by d4_autotune
    on the start states x0 [n][d_x] and goals [n][d_p] (and cached).
    d4_autotune times whole iterations from a plan one iteration old and keeps
    the rule's tile unless a candidate is at least 1 % faster; the entry's
    "us" is the chosen tile's time per denoising step.  The cost of the pair
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


def _batch_cost(p):
    """Relative cost of one instance: its pair checks and its draws."""
    return p.n_robots * p.horizon * p.n_samples * (p.n_robots + 40 * p.du)


def tune_batch(probs, x0s, goals, path=DEFAULT_CACHE, steps=None, reps=1, min_gain=0.01, min_share=0.05,
               force=False, log=None):
    """Tiles of the (dynamics, team-size, horizon) buckets of a batch, chosen
    by coordinate descent on the time of the whole batch: starting from the
    shared rule (which sizes each instance's sample tile by its own team), each
    bucket holding at least `min_share` of the batch's work tries every
    admissible candidate tile in turn, the others held fixed, and keeps one
    only when a batched iteration (the least of `reps` timed iterations, after
    one untimed) runs at least `min_gain` faster than the best so far.  The
    iterations keep the problems' own denoising steps unless `steps` is
    given: a shorter schedule changes how close the sampled trajectories come,
    and with it the share of the pair checks, so it ranks tiles differently.  The result can therefore not be slower than the rule by more than the
    timing noise.  A tile changes only speed (d4_batch_tile_set refuses tiles
    whose LDS would lower the whole batch's occupancy).  Cached per
    architecture, kernel source version and batch composition.  Returns
    {bucket: entry} for the buckets that left the rule."""
    import time
    groups = {}
    for j, p in enumerate(probs):
        groups.setdefault(batch_bucket(p), []).append(j)
    comp = hashlib.sha256(json.dumps(sorted((list(b), len(v)) for b, v in groups.items())).encode()).hexdigest()[:16]
    key = f"{_arch()}|{source_version()}|batch|{comp}|M{probs[0].n_samples}|N{steps or probs[0].n_steps}"
    cache = _load(path)
    for b in groups:
        clear_batch_tile(b)
    if key in cache and not force:
        chosen = {tuple(e["bucket"]): e for e in cache[key]}
        for b, e in chosen.items():
            set_batch_tile(b, e["S"], e["Tb"])
        return chosen
    sub = [p.replace(n_steps=steps) for p in probs] if steps else list(probs)

    def measure():
        bc = L.BatchContext(sub, x0s, goals)
        bc.iterate(0)
        torch.cuda.synchronize()
        best_t = None
        for k in range(reps):
            t0 = time.perf_counter()
            bc.iterate(1 + k)
            dt = time.perf_counter() - t0
            best_t = dt if best_t is None else min(best_t, dt)
        bc.close()
        return best_t

    total = sum(_batch_cost(p) for p in probs)
    share = {b: sum(_batch_cost(probs[j]) for j in idx) / total for b, idx in groups.items()}
    best = measure()
    if log:
        log(f"batch tuner: rule tiles {best * 1e3:.2f} ms per iteration")
    chosen = {}
    for b in sorted(groups, key=lambda b: -share[b]):
        if share[b] < min_share:
            continue
        for S, Tb in _candidates(b):
            try:
                set_batch_tile(b, S, Tb)
            except L.D4Error:
                continue
            t = measure()
            kept = t < best * (1.0 - min_gain)
            if kept:
                best = t
                chosen[b] = {"bucket": list(b), "S": S, "Tb": Tb, "ms": t * 1e3, "share": share[b]}
            if log:
                log(f"batch tuner: bucket {b} S={S} Tb={Tb}: {t * 1e3:.2f} ms{' (kept)' if kept else ''}")
        if b in chosen:
            set_batch_tile(b, chosen[b]["S"], chosen[b]["Tb"])
        else:
            clear_batch_tile(b)
    cache[key] = list(chosen.values())
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return chosen
