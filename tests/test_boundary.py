"""The C-ABI library without a GPU: it loads, exports every declared symbol,
its structs match the Python mirror, and bad arguments fail before any launch."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "d4.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|const char\*)\s+(d4\w*)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2503_12204_amd import _lib
    return _lib


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L.lib(), n), n


def test_struct_layout_matches_header(L, tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "d4.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(d4_problem), offsetof(d4_problem, u_lo),
         offsetof(d4_problem, flags), offsetof(d4_problem, seed), sizeof(d4_stats),
         offsetof(d4_stats, status));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    P, S = L.D4Problem, L.D4Stats
    assert got == [ctypes.sizeof(P), P.u_lo.offset, P.flags.offset, P.seed.offset, ctypes.sizeof(S), S.status.offset]


def _bad(L, **kw):
    from paper_2503_12204_amd import workloads as W
    p, _, _ = W.holo2d_circle()
    return L.to_c(p.replace(**kw))


@pytest.mark.parametrize("kw", [dict(n_robots=0), dict(n_robots=33), dict(horizon=0), dict(n_samples=0),
                                dict(n_steps=0), dict(n_steps=70000), dict(dt=0.0), dict(temperature=-1.0),
                                dict(dyn=7), dict(beta_min=0.0), dict(beta_max=1.0), dict(d0_floor=0.0),
                                dict(u_lo=(1.0, 1.0, 1.0), u_hi=(-1.0, -1.0, -1.0)), dict(robot_radius=-0.1)])
def test_invalid_problem_rejected_without_launch(L, kw):
    c = _bad(L, **kw)
    buf = (ctypes.c_float * 4)()
    rc = L.lib().d4_noise(ctypes.byref(c), 0, 1, ctypes.cast(buf, ctypes.c_void_p), None)
    assert rc == L.D4_EINVAL
    assert L.lib().d4_last_error().decode()


def test_null_and_misaligned_pointers_rejected(L):
    from paper_2503_12204_amd import workloads as W
    p, _, _ = W.holo2d_circle()
    c = L.to_c(p)
    assert L.lib().d4_noise(ctypes.byref(c), 0, 1, None, None) == L.D4_EINVAL
    buf = (ctypes.c_float * 8)()
    odd = ctypes.c_void_p(ctypes.addressof(buf) + 2)
    assert L.lib().d4_noise(ctypes.byref(c), 0, 1, odd, None) == L.D4_EINVAL
    assert L.lib().d4_noise(ctypes.byref(c), 0, 0, ctypes.cast(buf, ctypes.c_void_p), None) == L.D4_EINVAL
    assert L.lib().d4_noise(ctypes.byref(c), 70000, 1, ctypes.cast(buf, ctypes.c_void_p), None) == L.D4_EINVAL
    assert L.lib().d4_denoise_iter(None, ctypes.byref(c), None, None, None, 0, None, None, None) == L.D4_EINVAL
    assert L.lib().d4_ctx_create(ctypes.byref(c), None) == L.D4_EINVAL
    # the transform entry: negative counts and NULL arrays fail, an empty call launches nothing
    assert L.lib().d4_box_muller(None, -1, None, None) == L.D4_EINVAL
    assert L.lib().d4_box_muller(None, 4, ctypes.cast(buf, ctypes.c_void_p), None) == L.D4_EINVAL
    assert L.lib().d4_box_muller(ctypes.cast(buf, ctypes.c_void_p), 4, odd, None) == L.D4_EINVAL
    assert L.lib().d4_box_muller(None, 0, None, None) == L.D4_OK


def test_invalid_obstacles_rejected_without_launch(L):
    """Obstacles (appendix penalty): a count outside 0..16, a non-finite
    centre or a negative radius fail before any launch."""
    from paper_2503_12204_amd import workloads as W
    p, _, _ = W.holo2d_circle_obstacles(n=4, n_obs=2)
    buf = (ctypes.c_float * 4)()
    out = ctypes.cast(buf, ctypes.c_void_p)
    for mutate in (lambda c: setattr(c, "n_obstacles", L.MAX_OBSTACLES + 1),
                   lambda c: setattr(c, "n_obstacles", -1),
                   lambda c: c.obstacles[1].__setitem__(0, float("nan")),
                   lambda c: c.obstacles[0].__setitem__(3, -0.5)):
        c = L.to_c(p)
        mutate(c)
        assert L.lib().d4_noise(ctypes.byref(c), 0, 1, out, None) == L.D4_EINVAL
        assert L.lib().d4_last_error().decode()


def test_tile_rule_without_a_gpu():
    """The launch-shape rule is host code (d4_tile_get makes no GPU call).
    S = min(64, 256 / n), halved until M / S >= 256; with the full S the time
    block keeps the positions near 32 KiB (2D, 8-byte slots), or near 48 KiB
    for a single 3D problem (16-byte slots); with a halved S, R = min(16,
    1024 / (S n)) replica lanes, and time blocks of about a fifth of the
    horizon (at least 16 steps) when replica 0 fills whole waves (n S a
    multiple of 64, the pipelined schedule), else the longest block that
    fits (up to 64)."""
    import bench
    from paper_2503_12204_amd import autotune as AT
    expect = {
        # name: (single problem, batched rule)
        "holo3d_sphere_swap": ((16, 12, 1), (16, 8, 1)),     # 48 KiB / (16 * 16 * 16 B) = 12
        "unicycle_random": ((8, 20, 16), (32, 16, 1)),       # M = 2048: S 32 -> 8, R = 1024 / 64, T / 5
        "holo2d_circle_swap": ((1, 64, 16), (64, 16, 1)),    # M = 256: S 64 -> 1, R = 16
        "diffdrive_circle_swap": ((16, 16, 1), (16, 16, 1)),  # 32 KiB / (16 * 16 * 8 B) = 16
        "holo2d_circle_obstacles": ((16, 16, 1), (16, 16, 1)),
    }
    for name, (single, batched) in expect.items():
        p, _, _ = bench.make_workload(name)
        assert AT.get_tile(p) == single, name
        assert AT.get_tile(p, batched=True) == batched, name


def test_launch_options_without_a_gpu(L):
    """Launch options are explicit calls of the C ABI (no environment
    switches): defaults, round trip, and invalid options or values rejected."""
    lib = L.lib()
    v = ctypes.c_int32()
    for name, default in (("graphs", 1), ("aligned_draws", 1), ("update_grid", 0)):
        assert L.get_option(name) == default, name
    with L.option("graphs", 0):
        assert L.get_option("graphs") == 0
    assert L.get_option("graphs") == 1
    with L.option("update_grid", 256):
        assert L.get_option("update_grid") == 256
    assert L.get_option("update_grid") == 0
    assert lib.d4_set_option(0, 2) == L.D4_EINVAL
    assert lib.d4_set_option(1, -1) == L.D4_EINVAL
    assert lib.d4_set_option(2, -5) == L.D4_EINVAL
    assert L.get_option("gemm_tile") == 0
    with L.option("gemm_tile", 128):
        assert L.get_option("gemm_tile") == 128
    assert L.get_option("gemm_tile") == 0
    assert lib.d4_set_option(4, 96) == L.D4_EINVAL
    assert lib.d4_set_option(9, 0) == L.D4_EINVAL
    assert lib.d4_get_option(9, ctypes.byref(v)) == L.D4_EINVAL
    assert lib.d4_get_option(0, None) == L.D4_EINVAL
    assert L.get_option("graphs") == 1 and L.get_option("aligned_draws") == 1
    # the persistent batched step is switched off: the two-launch form is the default and stays
    assert L.get_option("batch_persistent") == 0
    assert lib.d4_set_option(3, 1) == L.D4_EUNSUPPORTED
    assert lib.d4_set_option(3, 0) == L.D4_OK


def test_noalloc_entry_rejects_before_any_launch(L):
    """The allocation-free iteration validates its arguments and its 64 MiB
    workspace limit on the host: a problem whose draws alone exceed it fails
    with D4_EUNSUPPORTED, NULL or misaligned pointers with D4_EINVAL."""
    from paper_2503_12204_amd import workloads as W
    lib = L.lib()
    p, _, _ = W.holo3d_sphere()      # 16 x 100 x 3 x 8192 draws: 157 MB
    c = L.to_c(p)
    buf = (ctypes.c_float * 64)()
    ptr = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.d4_denoise_iter_noalloc(ctypes.byref(c), ptr, ptr, ptr, 0, None, None, None) == L.D4_EUNSUPPORTED
    assert "workspace" in lib.d4_last_error().decode()
    q, _, _ = W.holo2d_circle()
    cq = L.to_c(q)
    assert lib.d4_denoise_iter_noalloc(ctypes.byref(cq), None, ptr, ptr, 0, None, None, None) == L.D4_EINVAL
    odd = ctypes.c_void_p(ctypes.addressof(buf) + 2)
    assert lib.d4_denoise_iter_noalloc(ctypes.byref(cq), ptr, ptr, odd, 0, None, None, None) == L.D4_EINVAL
    assert lib.d4_denoise_iter_noalloc(ctypes.byref(cq), ptr, ptr, ptr, 70000, None, None, None) == L.D4_EINVAL
    bad = L.to_c(q.replace(n_robots=0))
    assert lib.d4_denoise_iter_noalloc(ctypes.byref(bad), ptr, ptr, ptr, 0, None, None, None) == L.D4_EINVAL


def test_bench_measures_one_gpu_and_reports_its_source_hash():
    """bench.py refuses a multi-GPU run with a message, before touching a
    device, and --source-hash prints the hash that keys the stored traffic."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, cwd=ROOT, timeout=300)
    assert res.returncode != 0 and "one GPU" in (res.stdout + res.stderr)
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--source-hash"], capture_output=True,
                         text=True, cwd=ROOT, timeout=300)
    assert res.returncode == 0
    h = res.stdout.strip().splitlines()[-1]
    assert re.fullmatch(r"[0-9a-f]{16}", h) and h == bench.kernel_source_hash()
