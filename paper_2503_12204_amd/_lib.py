"""ctypes binding of libd4.so (include/d4.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Torch tensors supply device memory and the current HIP stream.
If the library is missing this module raises at import time; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int32, c_uint32, c_uint64, c_void_p

import torch

from .workloads import Problem

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libd4.so")

D4_OK, D4_EINVAL, D4_ENOMEM, D4_EHIP, D4_ENONFINITE, D4_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
MAX_OBSTACLES = 16
OPTIONS = {"graphs": 0, "aligned_draws": 1, "update_grid": 2, "batch_persistent": 3, "gemm_tile": 4}


class D4Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"d4 error {code}: {msg}")
        self.code = code


class D4Problem(ctypes.Structure):
    _fields_ = [
        ("dyn", c_int32), ("n_robots", c_int32), ("horizon", c_int32), ("n_samples", c_int32),
        ("n_steps", c_int32), ("dt", c_float), ("robot_radius", c_float), ("safety_margin", c_float),
        ("w_safe", c_float), ("temperature", c_float), ("beta_min", c_float), ("beta_max", c_float),
        ("u_lo", c_float * 3), ("u_hi", c_float * 3), ("v_max", c_float), ("goal_tol", c_float),
        ("d0_floor", c_float), ("flags", c_uint32), ("instance_id", c_uint32), ("seed", c_uint64),
        ("n_obstacles", c_int32), ("obstacles", (c_float * 4) * MAX_OBSTACLES),
    ]


class D4Stats(ctypes.Structure):
    _fields_ = [("reward", c_float), ("objective", c_float), ("hits", c_int32),
                ("robots_hit", c_int32), ("success", c_int32), ("at_goal", c_int32), ("obstacle_hits", c_int32),
                ("status", c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2503_12204_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = POINTER(D4Problem)
    fp = c_void_p
    sig = {
        "d4_last_error": ([], ctypes.c_char_p),
        "d4_set_option": ([c_int32, c_int32], c_int32),
        "d4_get_option": ([c_int32, POINTER(c_int32)], c_int32),
        "d4_noise": ([P, c_uint32, c_uint32, fp, c_void_p], c_int32),
        "d4_box_muller": ([fp, ctypes.c_int64, fp, c_void_p], c_int32),
        "d4_rollout": ([P, fp, fp, fp, c_void_p], c_int32),
        "d4_fitness": ([P, fp, fp, fp, fp, fp, c_void_p], c_int32),
        "d4_sample_rollout_fitness": ([P, fp, fp, fp, fp, c_uint32, c_uint32, fp, fp, fp, c_void_p], c_int32),
        "d4_score_update": ([P, fp, fp, fp, c_int32, fp, fp, c_void_p], c_int32),
        "d4_ctx_create": ([P, POINTER(c_void_p)], c_int32),
        "d4_ctx_destroy": ([c_void_p], c_int32),
        "d4_denoise_iter": ([c_void_p, P, fp, fp, fp, c_uint32, fp, POINTER(D4Stats), c_void_p], c_int32),
        "d4_denoise_iter_noalloc": ([P, fp, fp, fp, c_uint32, fp, POINTER(D4Stats), c_void_p], c_int32),
        "d4_batch_create": ([P, c_int32, POINTER(c_void_p)], c_int32),
        "d4_batch_layout": ([c_void_p, fp, fp, fp, fp], c_int32),
        "d4_batch_iter": ([c_void_p, fp, fp, fp, c_uint32, POINTER(D4Stats), c_void_p], c_int32),
        "d4_batch_destroy": ([c_void_p], c_int32),
        "d4_batch_work_list": ([P, c_int32, c_int32, c_int32, fp, fp], c_int32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def _check(rc):
    if rc != D4_OK:
        raise D4Error(rc, _lib.d4_last_error().decode())


def set_option(name: str, value: int):
    """d4_set_option by name: graphs, aligned_draws, update_grid."""
    _check(_lib.d4_set_option(OPTIONS[name], int(value)))


def get_option(name: str) -> int:
    v = c_int32()
    _check(_lib.d4_get_option(OPTIONS[name], ctypes.byref(v)))
    return v.value


class option:
    """Context manager that sets a launch option and restores it on exit."""

    def __init__(self, name: str, value: int):
        self.name, self.value = name, value

    def __enter__(self):
        self.old = get_option(self.name)
        set_option(self.name, self.value)
        return self

    def __exit__(self, *exc):
        set_option(self.name, self.old)
        return False


def to_c(p: Problem) -> D4Problem:
    c = D4Problem()
    for f in ("dyn", "n_robots", "horizon", "n_samples", "n_steps", "flags", "instance_id", "seed"):
        setattr(c, f, int(getattr(p, f)))
    for f in ("dt", "robot_radius", "safety_margin", "w_safe", "temperature", "beta_min", "beta_max",
              "v_max", "goal_tol", "d0_floor"):
        setattr(c, f, float(getattr(p, f)))
    for i in range(3):
        c.u_lo[i] = float(p.u_lo[i])
        c.u_hi[i] = float(p.u_hi[i])
    obs = list(p.obstacles)
    if len(obs) > MAX_OBSTACLES:
        raise ValueError(f"at most {MAX_OBSTACLES} obstacles")
    c.n_obstacles = len(obs)
    for i, o in enumerate(obs):
        for j in range(4):
            c.obstacles[i][j] = float(o[j])
    return c


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, shape=None, dtype=torch.float32, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return c_void_p(t.data_ptr())


def _f32(a, device="cuda"):
    return torch.as_tensor(a, dtype=torch.float32, device=device).contiguous()


# ------------------------------------------------------------------ calls
def noise(p: Problem, iteration: int, step: int, out=None):
    """eps [D][M] of denoising step `step` of iteration `iteration`."""
    c = to_c(p)
    eps = out if out is not None else torch.empty((p.D, p.n_samples), dtype=torch.float32, device="cuda")
    _check(_lib.d4_noise(ctypes.byref(c), iteration, step, _dev(eps, (p.D, p.n_samples), name="eps"), _stream()))
    return eps


def box_muller(words):
    """Box-Muller stage of the draw recipe on generator words [2*count] (int32
    or uint32 bits): z[2i] = rho cos, z[2i+1] = rho sin."""
    if not isinstance(words, torch.Tensor) or not words.is_cuda or words.dim() != 1 or words.numel() % 2:
        raise TypeError("words must be a 1-D CUDA tensor of even length")
    if words.dtype not in (torch.int32, torch.uint32) or not words.is_contiguous():
        raise TypeError("words must be contiguous int32 or uint32")
    z = torch.empty(words.numel(), dtype=torch.float32, device=words.device)
    _check(_lib.d4_box_muller(c_void_p(words.data_ptr()), words.numel() // 2, _dev(z, name="z"), _stream()))
    return z


def rollout(p: Problem, x0, u):
    """x [M][n][T+1][d_x] from x0 [n][d_x] and controls u [M][n][T][d_u]."""
    c = to_c(p)
    M = u.shape[0]
    q = p.replace(n_samples=M)
    c = to_c(q)
    x = torch.empty((M, p.n_robots, p.horizon + 1, p.dx), dtype=torch.float32, device="cuda")
    _check(_lib.d4_rollout(ctypes.byref(c), _dev(x0, (p.n_robots, p.dx), name="x0"),
                           _dev(u, (M, p.n_robots, p.horizon, p.du), name="u"), _dev(x, name="x"), _stream()))
    return x


def fitness(p: Problem, x, goal):
    """(r [M], hits [M], robots_hit [M]) of trajectories x [M][n][T+1][d_x]."""
    M = x.shape[0]
    c = to_c(p.replace(n_samples=M))
    r = torch.empty(M, dtype=torch.float32, device="cuda")
    hits = torch.empty(M, dtype=torch.int32, device="cuda")
    rh = torch.empty(M, dtype=torch.int32, device="cuda")
    _check(_lib.d4_fitness(ctypes.byref(c), _dev(x, (M, p.n_robots, p.horizon + 1, p.dx), name="x"),
                           _dev(goal, (p.n_robots, p.dp), name="goal"), _dev(r), _dev(hits, dtype=torch.int32),
                           _dev(rh, dtype=torch.int32), _stream()))
    return r, hits, rh


def sample_rollout_fitness(p: Problem, x0, goal, u_base, du_in, iteration: int, step: int,
                           eps=None, r=None, hits=None):
    """Fused sampling, rollout and reward of one denoising step -> (eps, r, hits)."""
    c = to_c(p)
    if eps is None:
        eps = torch.empty((p.D, p.n_samples), dtype=torch.float32, device="cuda")
    if r is None:
        r = torch.empty(p.n_samples, dtype=torch.float32, device="cuda")
    if hits is None:
        hits = torch.empty(p.n_samples, dtype=torch.int32, device="cuda")
    _check(_lib.d4_sample_rollout_fitness(
        ctypes.byref(c), _dev(x0, (p.n_robots, p.dx), name="x0"), _dev(goal, (p.n_robots, p.dp), name="goal"),
        _dev(u_base, (p.D,), name="u_base"), _dev(du_in, (p.D,), name="du_in"), iteration, step,
        _dev(eps, (p.D, p.n_samples), name="eps"), _dev(r, (p.n_samples,), name="r"),
        _dev(hits, (p.n_samples,), dtype=torch.int32, name="hits"), _stream()))
    return eps, r, hits


def score_update(p: Problem, r, eps, du_in, step: int, du_out=None, w_out=None):
    """Softmax weights and the one-step update -> (du_out [D], w [M])."""
    c = to_c(p)
    if du_out is None:
        du_out = torch.empty(p.D, dtype=torch.float32, device="cuda")
    if w_out is None:
        w_out = torch.empty(p.n_samples, dtype=torch.float32, device="cuda")
    _check(_lib.d4_score_update(ctypes.byref(c), _dev(r, (p.n_samples,), name="r"),
                                _dev(eps, (p.D, p.n_samples), name="eps"), _dev(du_in, (p.D,), name="du_in"),
                                step, _dev(du_out, (p.D,), name="du_out"), _dev(w_out, (p.n_samples,), name="w"),
                                _stream()))
    return du_out, w_out


class Context:
    """Owns a d4_ctx (workspace + captured graph) for one problem shape."""

    def __init__(self, p: Problem):
        self.p = p
        self._c = to_c(p)
        h = c_void_p()
        _check(_lib.d4_ctx_create(ctypes.byref(self._c), ctypes.byref(h)))
        self._h = h
        self._stats = D4Stats()

    def close(self):
        if self._h:
            _lib.d4_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def denoise_iter(self, x0, goal, u_base, iteration: int, traj=None, sync=True, p: Problem = None):
        """One iteration of Algorithm 2; u_base [n][T][d_u] is updated in place."""
        if p is not None:
            self._c = to_c(p)
            self.p = p
        p = self.p
        tr = _dev(traj, (p.n_robots, p.horizon + 1, p.dx), name="traj") if traj is not None else None
        _check(_lib.d4_denoise_iter(self._h, ctypes.byref(self._c), _dev(x0, (p.n_robots, p.dx), name="x0"),
                                    _dev(goal, (p.n_robots, p.dp), name="goal"),
                                    _dev(u_base, (p.n_robots, p.horizon, p.du), name="u_base"),
                                    iteration, tr, ctypes.byref(self._stats) if sync else None, _stream()))
        if not sync:
            return None
        torch.cuda.current_stream().synchronize()
        s = self._stats
        return dict(reward=s.reward, objective=s.objective, hits=s.hits, robots_hit=s.robots_hit,
                    success=bool(s.success), at_goal=bool(s.at_goal), obstacle_hits=s.obstacle_hits,
                    status=s.status)


def denoise_iter_noalloc(p: Problem, x0, goal, u_base, iteration: int, traj=None):
    """One iteration through d4_denoise_iter_noalloc (static workspace, no
    allocation, no graph); u_base [n][T][d_u] is updated in place."""
    c = to_c(p)
    st = D4Stats()
    tr = _dev(traj, (p.n_robots, p.horizon + 1, p.dx), name="traj") if traj is not None else None
    _check(_lib.d4_denoise_iter_noalloc(ctypes.byref(c), _dev(x0, (p.n_robots, p.dx), name="x0"),
                                        _dev(goal, (p.n_robots, p.dp), name="goal"),
                                        _dev(u_base, (p.n_robots, p.horizon, p.du), name="u_base"), iteration, tr,
                                        ctypes.byref(st), _stream()))
    torch.cuda.current_stream().synchronize()
    return _stats_dict(st)


def plan(p: Problem, x0, goal, iterations: int, u_init=None, stop_on_success=False):
    """Algorithm 2 from zero controls (or u_init): returns (u [n][T][d_u], per-iteration stats)."""
    x0 = _f32(x0)
    goal = _f32(goal)
    u = torch.zeros((p.n_robots, p.horizon, p.du), dtype=torch.float32, device="cuda") if u_init is None \
        else _f32(u_init).reshape(p.n_robots, p.horizon, p.du).clone()
    ctx = Context(p)
    hist = []
    try:
        for k in range(iterations):
            st = ctx.denoise_iter(x0, goal, u, k)
            hist.append(st)
            if stop_on_success and st["success"]:
                break
    finally:
        ctx.close()
    return u, hist


def batch_work_list(probs, lag):
    """The persistent step's work list for these problems (host only):
    int32 array [items][4] of (kind, instance, a, b)."""
    import numpy as np
    arr = (D4Problem * len(probs))(*[to_c(p) for p in probs])
    n = c_int32()
    _lib.d4_batch_work_list(arr, len(probs), int(lag), 0, None, ctypes.byref(n))
    out = np.zeros((max(n.value, 1), 4), dtype=np.int32)
    _check(_lib.d4_batch_work_list(arr, len(probs), int(lag), n.value, c_void_p(out.ctypes.data), ctypes.byref(n)))
    return out[:n.value]


def _stats_dict(s):
    return dict(reward=s.reward, objective=s.objective, hits=s.hits, robots_hit=s.robots_hit,
                success=bool(s.success), at_goal=bool(s.at_goal), obstacle_hits=s.obstacle_hits,
                status=s.status)


class BatchContext:
    """Owns a d4_batch: many problems sharing the sampler settings, advanced together.

    Inputs are lists of per-instance arrays; they are packed into device
    arrays in the library's layout (offsets from d4_batch_layout)."""

    def __init__(self, probs, x0s, goals):
        import numpy as np
        self.probs = list(probs)
        n = len(self.probs)
        arr = (D4Problem * n)(*[to_c(p) for p in self.probs])
        self._arr = arr
        h = c_void_p()
        _check(_lib.d4_batch_create(arr, n, ctypes.byref(h)))
        self._h = h
        off = [np.zeros(n, dtype=np.int64) for _ in range(3)]
        tot = np.zeros(3, dtype=np.int64)
        _check(_lib.d4_batch_layout(h, *[c_void_p(o.ctypes.data) for o in off], c_void_p(tot.ctypes.data)))
        self.x0_off, self.goal_off, self.u_off = off
        self.totals = tot
        self.x0 = self._pack(x0s, self.x0_off, tot[0])
        self.goal = self._pack(goals, self.goal_off, tot[1])
        self.u = torch.zeros(int(tot[2]), dtype=torch.float32, device="cuda")
        self._stats = (D4Stats * n)()

    @staticmethod
    def _pack(arrays, offsets, total):
        import numpy as np
        flat = np.zeros(int(total), dtype=np.float32)
        for a, o in zip(arrays, offsets):
            a = np.asarray(a, dtype=np.float32).ravel()
            flat[int(o):int(o) + a.size] = a
        return torch.as_tensor(flat, device="cuda")

    def plan_of(self, j):
        """Instance j's plan [n][T][d_u] as a view of the packed device array."""
        p = self.probs[j]
        o = int(self.u_off[j])
        return self.u[o:o + p.D].view(p.n_robots, p.horizon, p.du)

    def set_plans(self, plans):
        import numpy as np
        self.u.copy_(self._pack(plans, self.u_off, self.totals[2]))

    def iterate(self, iteration: int, sync=True):
        """One iteration of every instance; returns per-instance stats when sync."""
        _check(_lib.d4_batch_iter(self._h, _dev(self.x0), _dev(self.goal), _dev(self.u), iteration,
                                  self._stats if sync else None, _stream()))
        if not sync:
            return None
        torch.cuda.current_stream().synchronize()
        return [_stats_dict(s) for s in self._stats]

    def close(self):
        if self._h:
            _lib.d4_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ learned proposal
class D4PConfig(ctypes.Structure):
    _fields_ = [("d_in", c_int32), ("width", c_int32), ("hidden", c_int32), ("layers", c_int32),
                ("d_out", c_int32), ("max_rows", c_int32), ("max_batch", c_int32), ("seed", c_uint64)]


def _load_proposal():
    fp = c_void_p
    sig = {
        "d4p_create": ([POINTER(D4PConfig), POINTER(c_void_p)], c_int32),
        "d4p_destroy": ([c_void_p], c_int32),
        "d4p_num_params": ([c_void_p, POINTER(ctypes.c_int64)], c_int32),
        "d4p_set_params": ([c_void_p, fp, c_void_p], c_int32),
        "d4p_get_params": ([c_void_p, fp, c_void_p], c_int32),
        "d4p_forward": ([c_void_p, fp, fp, c_int32, c_int32, fp, c_void_p], c_int32),
        "d4p_gradients": ([c_void_p, fp, fp, c_int32, c_int32, fp, fp, fp, fp, c_void_p], c_int32),
        "d4p_train_step": ([c_void_p, fp, fp, c_int32, c_int32, fp, fp, c_float, fp, c_void_p], c_int32),
        "d4p_gemm_bf16": ([c_int32, c_int32, fp, fp, fp, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32,
                           c_float, c_void_p], c_int32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(_lib, name)
        fn.argtypes = args
        fn.restype = res


_load_proposal()


def gemm_bf16(A, B, M, N, K, trans_a=False, trans_b=False, C=None, beta=0.0):
    """C[M][N] (+)= op(A) op(B) on the BF16 MFMA kernel; A, B bfloat16 CUDA tensors."""
    if C is None:
        C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    lda = M if trans_a else K
    ldb = K if trans_b else N
    _check(_lib.d4p_gemm_bf16(int(trans_a), int(trans_b), _dev(A, dtype=torch.bfloat16, name="A"),
                              _dev(B, dtype=torch.bfloat16, name="B"), _dev(C, name="C"), M, N, K, lda, ldb, N,
                              float(beta), _stream()))
    return C


class ProposalNet:
    """The set network of d4p_* (weights, Adam state and workspace on the GPU)."""

    def __init__(self, d_in=6, width=256, hidden=512, layers=4, d_out=200, max_rows=4096, max_batch=512, seed=0):
        self.cfg = D4PConfig(d_in, width, hidden, layers, d_out, max_rows, max_batch, seed)
        h = c_void_p()
        _check(_lib.d4p_create(ctypes.byref(self.cfg), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64()
        _check(_lib.d4p_num_params(h, ctypes.byref(n)))
        self.n_params = int(n.value)
        self._loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def set_params(self, flat):
        flat = _f32(flat)
        _check(_lib.d4p_set_params(self._h, _dev(flat, (self.n_params,), name="params"), _stream()))

    def get_params(self):
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(_lib.d4p_get_params(self._h, _dev(out), _stream()))
        return out

    def forward(self, x, seg):
        R, B = x.shape[0], seg.shape[0] - 1
        y = torch.empty((R, self.cfg.d_out), dtype=torch.float32, device="cuda")
        _check(_lib.d4p_forward(self._h, _dev(x, (R, self.cfg.d_in), name="x"),
                                _dev(seg, dtype=torch.int32, name="seg"), R, B, _dev(y), _stream()))
        return y

    def gradients(self, x, seg, target, mask):
        R, B = x.shape[0], seg.shape[0] - 1
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(_lib.d4p_gradients(self._h, _dev(x, (R, self.cfg.d_in), name="x"),
                                  _dev(seg, dtype=torch.int32, name="seg"), R, B,
                                  _dev(target, (R, self.cfg.d_out), name="target"), _dev(mask, (R,), name="mask"),
                                  _dev(self._loss), _dev(g), _stream()))
        return self._loss.clone(), g

    def train_step(self, x, seg, target, mask, lr):
        R, B = x.shape[0], seg.shape[0] - 1
        _check(_lib.d4p_train_step(self._h, _dev(x, (R, self.cfg.d_in), name="x"),
                                   _dev(seg, dtype=torch.int32, name="seg"), R, B,
                                   _dev(target, (R, self.cfg.d_out), name="target"),
                                   _dev(mask, (R,), name="mask"), float(lr), _dev(self._loss), _stream()))
        return self._loss

    def close(self):
        if self._h:
            _lib.d4p_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
