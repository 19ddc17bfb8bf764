// Host-side helpers shared by the C-ABI sources: error reporting, argument
// validation, the noise schedule and the launch shapes of the reward kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "d4.h"
#include "d4_kernels.hpp"

namespace d4host {

using namespace d4;

inline thread_local std::string g_err;

// Process-wide launch options (d4_set_option): iterations replay a captured
// graph; the whole-block draw window serves problems whose horizons start
// every robot on a Philox block; the update kernel's grid follows its rule
// (0) or a given workgroup count.
inline std::atomic<int> g_opt_graphs{1};
inline std::atomic<int> g_opt_aligned_draws{1};
inline std::atomic<int> g_opt_update_grid{0};
inline std::atomic<int> g_opt_batch_persistent{0};
inline std::atomic<int> g_opt_gemm_tile{0};

inline int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(D4_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

#define HIP_LAUNCH_CHECK(name)                                                         \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return fail(D4_EHIP, "launch of %s failed: %s", name, hipGetErrorString(e_)); \
    } while (0)

// LDS a reward kernel may request dynamically: 160 KiB per CU less room for
// the kernels' static arrays (staged obstacles, reductions).
constexpr size_t LDS_DYNAMIC_MAX = 160 * 1024 - 1024;

// Dynamic LDS every reward workgroup of the batched form requests: room for
// two on a CU, not three (the batched kernel carries every model's code, and
// three workgroups per CU ran a mixed batch 45 % slower).  A bucket tile
// must fit under it, since the largest request sets every workgroup's.
constexpr size_t LDS_TWO_PER_CU = 56 * 1024;

struct Shape {
    int dx, du, dp;
};

inline Shape shape_of(int dyn) {
    switch (dyn) {
        case HOLO2D: return {4, 2, 2};
        case HOLO3D: return {6, 3, 3};
        case UNICYCLE: return {3, 2, 2};
        default: return {4, 2, 2};
    }
}

inline bool finite_f(float v) { return std::isfinite(v); }

inline int validate(const d4_problem* p) {
    if (!p) return fail(D4_EINVAL, "problem is NULL");
    if (p->dyn < 0 || p->dyn > 3) return fail(D4_EINVAL, "dyn %d is not a known model", p->dyn);
    if (p->n_robots < 1 || p->n_robots > 32)
        return fail(D4_EINVAL, "n_robots %d outside 1..32", p->n_robots);
    if (p->horizon < 1) return fail(D4_EINVAL, "horizon %d < 1", p->horizon);
    if (p->n_samples < 1) return fail(D4_EINVAL, "n_samples %d < 1", p->n_samples);
    if (p->n_steps < 1 || p->n_steps > 65535)
        return fail(D4_EINVAL, "n_steps %d outside 1..65535", p->n_steps);
    if (!(p->dt > 0.0f) || !finite_f(p->dt)) return fail(D4_EINVAL, "dt must be positive");
    if (!(p->temperature > 0.0f) || !finite_f(p->temperature))
        return fail(D4_EINVAL, "temperature must be positive");
    if (!(p->robot_radius >= 0.0f) || !(p->safety_margin >= 0.0f) || !finite_f(p->robot_radius) ||
        !finite_f(p->safety_margin))
        return fail(D4_EINVAL, "robot_radius and safety_margin must be >= 0");
    if (!(p->d0_floor > 0.0f)) return fail(D4_EINVAL, "d0_floor must be positive");
    if (!finite_f(p->w_safe) || !finite_f(p->beta_min) || !finite_f(p->beta_max))
        return fail(D4_EINVAL, "non-finite weight or schedule");
    if (!(p->beta_min > 0.0f) || !(p->beta_max < 1.0f) || p->beta_min > p->beta_max)
        return fail(D4_EINVAL, "need 0 < beta_min <= beta_max < 1");
    const Shape s = shape_of(p->dyn);
    for (int d = 0; d < s.du; ++d)
        if (!(p->u_lo[d] <= p->u_hi[d]) || !finite_f(p->u_lo[d]) || !finite_f(p->u_hi[d]))
            return fail(D4_EINVAL, "control box %d is empty or non-finite", d);
    if (p->dyn != UNICYCLE && !(p->v_max >= 0.0f)) return fail(D4_EINVAL, "v_max must be >= 0");
    if (p->n_obstacles < 0 || p->n_obstacles > D4_MAX_OBSTACLES)
        return fail(D4_EINVAL, "n_obstacles %d outside 0..%d", p->n_obstacles, D4_MAX_OBSTACLES);
    for (int o = 0; o < p->n_obstacles; ++o) {
        for (int c = 0; c < 4; ++c)
            if (!finite_f(p->obstacles[o][c])) return fail(D4_EINVAL, "obstacle %d is not finite", o);
        if (!(p->obstacles[o][3] >= 0.0f)) return fail(D4_EINVAL, "obstacle %d has a negative radius", o);
    }
    const double D = (double)p->n_robots * p->horizon * s.du;
    if (D * p->n_samples > 4.0e9) return fail(D4_EUNSUPPORTED, "D*M = %.0f too large", D * p->n_samples);
    if ((D + 3) / 4 > 65535.0) return fail(D4_EUNSUPPORTED, "D = %.0f too large for one launch", D);
    return D4_OK;
}

inline int need(const void* ptr, const char* name) {
    if (!ptr) return fail(D4_EINVAL, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(ptr) & 3u) return fail(D4_EINVAL, "%s is not 4-byte aligned", name);
    return D4_OK;
}

#define NEED(ptr)                                \
    do {                                         \
        int rc_ = need((ptr), #ptr);             \
        if (rc_) return rc_;                     \
    } while (0)

struct Schedule {
    std::vector<float> ms, sigma, os;  // index 0..N
};

// Linear betas over i = 1..N (both ends included), alpha-bar products in FP64.
inline Schedule make_schedule(const d4_problem* p) {
    const int N = p->n_steps;
    Schedule s;
    s.ms.assign(N + 1, 0.0f);
    s.sigma.assign(N + 1, 0.0f);
    s.os.assign(N + 1, 0.0f);
    double ab_prev = 1.0;
    for (int i = 1; i <= N; ++i) {
        const double beta = N == 1 ? (double)p->beta_min
                                   : (double)p->beta_min +
                                         ((double)p->beta_max - (double)p->beta_min) * (i - 1) / (N - 1);
        const double ab = ab_prev * (1.0 - beta);
        s.ms[i] = (float)(1.0 / std::sqrt(ab));
        s.sigma[i] = (float)std::sqrt(1.0 / ab - 1.0);
        s.os[i] = (float)std::sqrt(ab_prev);
        ab_prev = ab;
    }
    return s;
}

inline float thr2_reward(const d4_problem* p) {
    const double thr = 2.0 * (double)p->robot_radius + (double)p->safety_margin;
    return (float)(thr * thr);
}

// Obstacle o as (centre, (R_a + r_o + epsilon)^2) for the reward, and its
// squared safety distance (R_a + r_o)^2 for success; squares formed in FP64
// from the FP32 parameters, then rounded.
inline float4 obstacle_reward(const d4_problem* p, int o) {
    const double thr = (double)p->robot_radius + (double)p->obstacles[o][3] + (double)p->safety_margin;
    return make_float4(p->obstacles[o][0], p->obstacles[o][1], p->obstacles[o][2], (float)(thr * thr));
}
inline float obstacle_safe2(const d4_problem* p, int o) {
    const double s = (double)p->robot_radius + (double)p->obstacles[o][3];
    return (float)(s * s);
}

inline StepConsts step_consts(const d4_problem* p) {
    StepConsts c;
    c.dt = p->dt;
    c.hdt = (float)(0.5 * p->dt);
    c.hdt2 = (float)(0.5 * (double)p->dt * (double)p->dt);
    c.dt6 = (float)((double)p->dt / 6.0);
    c.vmax = p->v_max;
    return c;
}

struct Tile {
    int S, Tb;
    int R = 1;  // replica lanes per (sample, robot); R > 1 selects the cooperative kernel
};

// Samples per workgroup and time-block length of the reward kernels.  One
// rule serves the single-problem and the batched kernels (workgroups of at most
// 256 lanes), so a batched instance reproduces its single-problem run bit for
// bit: S = min(64, floor(256 / n)) samples, and a time block that keeps the
// positions near 32 KiB, in whole draw chunks, so that three workgroups share
// a CU's 160 KiB of LDS.
inline Tile default_tile(int dyn, int n) {
    int S = std::min(64, 256 / n);
    const int slot = shape_of(dyn).dp == 3 ? 16 : 8;
    const int per_step = n * S * slot;
    int Tb = (32 * 1024) / per_step;
    const int cs = shape_of(dyn).du == 2 ? 2 : 4;
    Tb = std::max(cs, std::min(16, Tb / cs * cs));
    return {S, Tb};
}

// Tuned tile of a problem shape installed by d4_tile_set / d4_autotune, if any.
bool tile_override(int dyn, int n, int T, Tile* out);

// Tile of an instance of the batched form: the tile installed for its
// (dynamics, team-size range, horizon range) bucket by d4_batch_tile_set, if
// any, else the shared rule.
Tile batch_tile(int dyn, int n, int T);

// Dynamic LDS of the cooperative kernel: double-buffered controls
// [2][n][G][4][S] (G = Tb d_u / 4 + 1 Philox blocks per robot and time block,
// plus two of padding for the rollout's read-ahead)
// and positions [2][Tb][2n-1][S], triple-buffered masks [3][Tb][S]; the final
// reductions reuse the space.
inline size_t coop_lds(int dyn, size_t n, size_t S, size_t Tb, size_t R) {
    const Shape s = shape_of(dyn);
    const size_t slot = s.dp == 3 ? 16 : 8;
    const size_t G = Tb * s.du / 4 + 3;
    const size_t a = 2 * n * G * 4 * S * 4 + 2 * Tb * (2 * n - 1) * S * slot + 3 * Tb * S * 4;
    const size_t b = (3 + R) * n * S * 4;
    return a > b ? a : b;
}

// Single-problem default: halve the samples per workgroup until there are at
// least 256 workgroups (one per CU), then add replica lanes (cooperative
// kernel), up to 16 and 1024 lanes per workgroup, when a workgroup would be
// smaller.  When the cooperative kernel pipelines its stages (replica 0 fills
// whole waves) a horizon is cut into about five time blocks; otherwise its
// stages run one after another and its time blocks are as long as the LDS
// allows (up to 64 steps).
// A single 3D problem with the full sample tile takes positions near 48 KiB
// instead of 32 (at 16 robots Tb = 12 runs 0.7 % faster than 8); the batched
// kernel keeps the shared rule, under which its mixed batches run fastest.
inline Tile single_tile(int dyn, int n, int M, int T) {
    Tile t = default_tile(dyn, n);
    int S = t.S;
    while (S > 1 && (M + S - 1) / S < 256) S >>= 1;
    if (S == t.S) {
        if (shape_of(dyn).dp == 3) {
            const int cs = shape_of(dyn).du == 2 ? 2 : 4;
            t.Tb = std::max(cs, std::min(16, ((48 * 1024) / (n * S * 16)) / cs * cs));
        }
        return t;
    }
    const int R = std::max(1, std::min(16, 1024 / (S * n)));
    const int cs = shape_of(dyn).du == 2 ? 2 : 4;
    const int slot = shape_of(dyn).dp == 3 ? 16 : 8;
    int Tb = std::max(cs, std::min(16, ((32 * 1024) / (n * S * slot)) / cs * cs));
    if (R > 1) {
        if ((n * S) % 64 == 0) {
            // pipelined stages: about five time blocks, of at least 16 steps
            Tb = std::max(16, ((T + 4) / 5 + cs - 1) / cs * cs);
        } else {
            // sequential stages: time blocks as long as the LDS allows
            Tb = 64;
        }
        while (Tb > cs && coop_lds(dyn, n, S, Tb, R) > LDS_DYNAMIC_MAX) Tb -= cs;
    }
    Tile out;
    out.S = S;
    out.Tb = Tb;
    out.R = R;
    return out;
}

inline Tile pick_tile(const d4_problem* p) {
    const int n = p->n_robots;
    Tile t = single_tile(p->dyn, n, p->n_samples, p->horizon);
    Tile o;
    if (tile_override(p->dyn, n, p->horizon, &o)) t = o;
    int S = t.S, Tb = t.Tb;
    int R = t.R;
    if (R * S * n > 1024) R = std::max(1, 1024 / (S * n));
    Tile out;
    out.S = S;
    out.Tb = Tb;
    out.R = R;
    return out;
}

inline size_t rollfit_lds(const d4_problem* p, Tile t) {
    const Shape s = shape_of(p->dyn);
    const size_t n = p->n_robots;
    const size_t slot = s.dp == 3 ? 16 : 8;
    if (t.R > 1) return coop_lds(p->dyn, n, t.S, t.Tb, t.R);
    // one-lane kernel: positions [Tb][n][S], boxes [n][S][2], masks [2][Tb][S], flags [2][S],
    // hit counters [S], then per wave a list of 64 floor(n/2) 16-bit narrow-phase triples
    const size_t waves = (n * t.S + 63) / 64;
    const size_t a = (size_t)t.Tb * n * t.S * slot + (size_t)2 * n * t.S * slot +
                     (size_t)2 * t.Tb * t.S * 4 + (size_t)2 * t.S * 4 + (size_t)t.S * 4 +
                     waves * 64 * (n / 2) * 2;
    const size_t b = (size_t)3 * n * t.S * 4;
    return a > b ? a : b;
}

// Float4 columns per lane of the register form of the update kernel (the
// smallest power of two with 1024 J >= M), or 0 for the LDS form: the sample
// count must be a multiple of 4 and the draws and rewards 16-byte aligned.
inline int upd_reg_j(int M, const void* eps, const void* r) {
    if (M % 4 || M > 16384 || (reinterpret_cast<uintptr_t>(eps) & 15u) || (reinterpret_cast<uintptr_t>(r) & 15u))
        return 0;
    int J = 1;
    while (J * 1024 < M) J <<= 1;
    return J;
}

// Whether every robot's draws start on a Philox block boundary.
inline bool draws_aligned(const d4_problem* p) { return (p->horizon * shape_of(p->dyn).du) % 4 == 0; }

inline RollFitArgs base_args(const d4_problem* p, Tile tile) {
    RollFitArgs a;
    std::memset(&a, 0, sizeof a);
    a.n = p->n_robots;
    a.T = p->horizon;
    a.M = p->n_samples;
    a.S = tile.S;
    a.Tb = tile.Tb;
    a.thr2 = thr2_reward(p);
    a.w_safe = p->w_safe;
    a.d0_floor = p->d0_floor;
    for (int d = 0; d < 3; ++d) {
        a.ulo[d] = p->u_lo[d];
        a.uhi[d] = p->u_hi[d];
    }
    a.sc = step_consts(p);
    a.key0 = (uint32_t)(p->seed & 0xFFFFFFFFull);
    a.key1 = (uint32_t)(p->seed >> 32);
    a.inst = p->instance_id;
    a.flags = p->flags;
    a.n_obs = p->n_obstacles;
    a.obs = nullptr;
    for (int o = 0; o < p->n_obstacles; ++o) a.obs_inline[o] = obstacle_reward(p, o);
    return a;
}

// Dynamic LDS above 64 KiB must be enabled per kernel (gfx950: 160 KiB per CU).
template <typename K>
inline void allow_lds(K kernel, size_t lds) {
    if (lds > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace d4host
