// Host side of the C ABI declared in include/d4.h: argument validation, the
// noise schedule, launch shapes, the per-problem workspace and the captured
// HIP graph of one deformation iteration (Algorithm 2 loop body).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "d4.h"
#include "d4_host.hpp"

using namespace d4;

namespace {

using namespace d4host;

template <int DYN>
void launch_rollfit_dyn(bool from_x, bool aligned, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                        const RollFitArgs& a) {
    if (!from_x && aligned) {
        allow_lds(k_rollfit<DYN, MODE_FUSED_ALIGNED>, lds);
        hipLaunchKernelGGL((k_rollfit<DYN, MODE_FUSED_ALIGNED>), grid, block, lds, st, a);
    } else if (!from_x) {
        allow_lds(k_rollfit<DYN, MODE_FUSED>, lds);
        hipLaunchKernelGGL((k_rollfit<DYN, MODE_FUSED>), grid, block, lds, st, a);
    } else {
        allow_lds(k_rollfit<DYN, MODE_FROM_X>, lds);
        hipLaunchKernelGGL((k_rollfit<DYN, MODE_FROM_X>), grid, block, lds, st, a);
    }
}

template <bool FROM_X>
int launch_rollfit(const d4_problem* p, const RollFitArgs& a, Tile tile, hipStream_t st) {
    const dim3 grid((p->n_samples + tile.S - 1) / tile.S);
    if (FROM_X) tile.R = 1;
    const dim3 block(tile.R * tile.S * p->n_robots);
    const size_t lds = rollfit_lds(p, tile);
    if (lds > LDS_DYNAMIC_MAX) return fail(D4_EUNSUPPORTED, "reward kernel needs %zu bytes of LDS", lds);
    if (tile.S * p->n_robots > 256 || tile.R * tile.S * p->n_robots > 1024)
        return fail(D4_EINVAL, "workgroup of %d x %d x %d lanes too large", tile.R, tile.S, p->n_robots);
    if (tile.R > 1) {
        switch (p->dyn) {
            case HOLO2D:
                allow_lds(k_rollfit_coop<HOLO2D>, lds);
                hipLaunchKernelGGL(k_rollfit_coop<HOLO2D>, grid, block, lds, st, a, tile.R);
                break;
            case HOLO3D:
                allow_lds(k_rollfit_coop<HOLO3D>, lds);
                hipLaunchKernelGGL(k_rollfit_coop<HOLO3D>, grid, block, lds, st, a, tile.R);
                break;
            case UNICYCLE:
                allow_lds(k_rollfit_coop<UNICYCLE>, lds);
                hipLaunchKernelGGL(k_rollfit_coop<UNICYCLE>, grid, block, lds, st, a, tile.R);
                break;
            default:
                allow_lds(k_rollfit_coop<DIFFDRIVE>, lds);
                hipLaunchKernelGGL(k_rollfit_coop<DIFFDRIVE>, grid, block, lds, st, a, tile.R);
                break;
        }
        HIP_LAUNCH_CHECK("k_rollfit_coop");
        return D4_OK;
    }
    const bool al = draws_aligned(p) && g_opt_aligned_draws.load() != 0;
    switch (p->dyn) {
        case HOLO2D: launch_rollfit_dyn<HOLO2D>(FROM_X, al, grid, block, lds, st, a); break;
        case HOLO3D: launch_rollfit_dyn<HOLO3D>(FROM_X, al, grid, block, lds, st, a); break;
        case UNICYCLE: launch_rollfit_dyn<UNICYCLE>(FROM_X, al, grid, block, lds, st, a); break;
        default: launch_rollfit_dyn<DIFFDRIVE>(FROM_X, al, grid, block, lds, st, a); break;
    }
    HIP_LAUNCH_CHECK("k_rollfit");
    return D4_OK;
}

// Weighted update of step i: softmax weights from the reward statistics, the
// weighted sum of the draws and the rescaled deformation.
int launch_update(const d4_problem* p, const float* eps, const float* r, const float* du_in, float* du_out,
                  float* w_out, int* status, float ms, float sigma, float os, hipStream_t st) {
    const int D = p->n_robots * p->horizon * shape_of(p->dyn).du;
    const int M = p->n_samples;
    if (M > 16384) return fail(D4_EUNSUPPORTED, "n_samples %d above the 16384 weights one workgroup stages", M);
    UpdateArgs a;
    a.eps = eps;
    a.r = r;
    a.du_in = du_in;
    a.du_out = du_out;
    a.w_out = w_out;
    a.status = status;
    a.D = D;
    a.M = M;
    a.inv_lam = 1.0f / p->temperature;
    a.normalize = (p->flags & FLAG_NORMALIZE) ? 1 : 0;
    a.ms = ms;
    a.sigma = sigma;
    a.os = os;
    // register form when the rows are whole float4s; LDS form otherwise
    const int J = upd_reg_j(M, eps, r);
    if (J > 0) {
        // at most 512 workgroups, of two rows each when D is small
        int grid = std::max(1, std::min(512, (D + 1) / 2));
        if (const int g = g_opt_update_grid.load()) grid = std::max(1, std::min(D, g));
        switch (J) {
            case 1:
                // up to 256 samples fit one wave's float4 columns
                if (M <= 256) hipLaunchKernelGGL(k_softmax_update_wave, dim3(grid), dim3(64), 0, st, a);
                else hipLaunchKernelGGL(k_softmax_update_reg<1>, dim3(grid), dim3(256), 0, st, a);
                break;
            case 2: hipLaunchKernelGGL(k_softmax_update_reg<2>, dim3(grid), dim3(256), 0, st, a); break;
            case 4: hipLaunchKernelGGL(k_softmax_update_reg<4>, dim3(grid), dim3(256), 0, st, a); break;
            case 8: hipLaunchKernelGGL(k_softmax_update_reg<8>, dim3(grid), dim3(256), 0, st, a); break;
            default: hipLaunchKernelGGL(k_softmax_update_reg<16>, dim3(grid), dim3(256), 0, st, a); break;
        }
    } else {
        const int waves = 4;
        int grid = std::min(1024, (D + waves - 1) / waves);
        hipLaunchKernelGGL(k_softmax_update, dim3(grid), dim3(64 * waves), (size_t)M * 4, st, a);
    }
    HIP_LAUNCH_CHECK("k_softmax_update");
    return D4_OK;
}

}  // namespace

// ------------------------------------------------------------------ context
struct d4_ctx {
    d4_problem prob;
    bool captured;
    int device;
    hipStream_t cap_stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
    float *eps, *r, *w, *du_a, *du_b, *x0, *goal, *ubase, *traj, *stats;
    int* hits;
    int* status;
    uint32_t* iter;
};

namespace {

void free_ctx_buffers(d4_ctx* c) {
    float* fb[] = {c->eps, c->r, c->w, c->du_a, c->du_b, c->x0, c->goal, c->ubase, c->traj, c->stats};
    for (float* f : fb)
        if (f) (void)hipFree(f);
    if (c->hits) (void)hipFree(c->hits);
    if (c->status) (void)hipFree(c->status);
    if (c->iter) (void)hipFree(c->iter);
}

// Field by field (a byte compare would also compare padding, which C callers
// need not initialise).  Floats compare by value; obstacles past n_obstacles
// are ignored.
bool same_problem(const d4_problem& a, const d4_problem& b) {
    bool eq = a.dyn == b.dyn && a.n_robots == b.n_robots && a.horizon == b.horizon && a.n_samples == b.n_samples &&
              a.n_steps == b.n_steps && a.dt == b.dt && a.robot_radius == b.robot_radius &&
              a.safety_margin == b.safety_margin && a.w_safe == b.w_safe && a.temperature == b.temperature &&
              a.beta_min == b.beta_min && a.beta_max == b.beta_max && a.v_max == b.v_max &&
              a.goal_tol == b.goal_tol && a.d0_floor == b.d0_floor && a.flags == b.flags &&
              a.instance_id == b.instance_id && a.seed == b.seed && a.n_obstacles == b.n_obstacles;
    for (int d = 0; d < 3 && eq; ++d) eq = a.u_lo[d] == b.u_lo[d] && a.u_hi[d] == b.u_hi[d];
    for (int o = 0; o < a.n_obstacles && eq; ++o)
        for (int c = 0; c < 4; ++c) eq = eq && a.obstacles[o][c] == b.obstacles[o][c];
    return eq;
}

bool same_shape(const d4_problem& a, const d4_problem& b) {
    return a.dyn == b.dyn && a.n_robots == b.n_robots && a.horizon == b.horizon &&
           a.n_samples == b.n_samples && a.n_steps == b.n_steps;
}

// Device buffers of one iteration: problem inputs, the plan (updated in
// place), the workspace and the outputs.
struct IterBuffers {
    const float* x0;
    const float* goal;
    float* ubase;
    float *eps, *r, *du_a, *du_b, *traj, *stats;
    int *hits, *status;
    uint32_t* iter;
};

// Enqueue one full iteration of problem p on `st`.
int enqueue_iteration(const d4_problem* p, const IterBuffers& c_, hipStream_t st) {
    const IterBuffers* c = &c_;
    const Shape s = shape_of(p->dyn);
    const int D = p->n_robots * p->horizon * s.du;
    const Schedule sc = make_schedule(p);
    const Tile tile = pick_tile(p);
    hipLaunchKernelGGL(k_fill, dim3((D + 255) / 256), dim3(256), 0, st, c->du_a, D, 0.0f);
    HIP_LAUNCH_CHECK("k_fill");
    float* du_cur = c->du_a;
    float* du_nxt = c->du_b;
    RollFitArgs a = base_args(p, tile);
    a.x0 = c->x0;
    a.goal = c->goal;
    a.u_base = c->ubase;
    a.eps = c->eps;
    a.r = c->r;
    a.hits = c->hits;
    a.robots_hit = nullptr;
    a.iter_dev = c->iter;
    for (int i = p->n_steps; i >= 1; --i) {
        a.du_in = du_cur;
        a.step = (uint32_t)i;
        a.mean_scale = sc.ms[i];
        a.sigma = sc.sigma[i];
        int rc = launch_rollfit<false>(p, a, tile, st);
        if (rc) return rc;
        rc = launch_update(p, c->eps, c->r, du_cur, du_nxt, nullptr, c->status, sc.ms[i],
                           sc.sigma[i], sc.os[i], st);
        if (rc) return rc;
        float* t = du_cur;
        du_cur = du_nxt;
        du_nxt = t;
    }
    FinalArgs f;
    std::memset(&f, 0, sizeof f);
    f.u_base = c->ubase;
    f.du0 = du_cur;
    f.x0 = c->x0;
    f.goal = c->goal;
    f.traj = c->traj;
    f.stats = c->stats;
    f.status = c->status;
    f.n = p->n_robots;
    f.T = p->horizon;
    for (int d = 0; d < 3; ++d) {
        f.ulo[d] = p->u_lo[d];
        f.uhi[d] = p->u_hi[d];
    }
    f.sc = step_consts(p);
    f.thr2 = thr2_reward(p);
    const double s2 = 2.0 * (double)p->robot_radius;
    f.safe2 = (float)(s2 * s2);
    f.goal_tol = p->goal_tol;
    f.w_safe = p->w_safe;
    f.d0_floor = p->d0_floor;
    f.flags = p->flags;
    f.n_obs = p->n_obstacles;
    f.obs = nullptr;
    f.obs_safe2 = nullptr;
    for (int o = 0; o < p->n_obstacles; ++o) {
        f.obs_inline[o] = obstacle_reward(p, o);
        f.safe2_inline[o] = obstacle_safe2(p, o);
    }
    switch (p->dyn) {
        case HOLO2D: hipLaunchKernelGGL(k_apply_final<HOLO2D>, dim3(1), dim3(256), 0, st, f); break;
        case HOLO3D: hipLaunchKernelGGL(k_apply_final<HOLO3D>, dim3(1), dim3(256), 0, st, f); break;
        case UNICYCLE: hipLaunchKernelGGL(k_apply_final<UNICYCLE>, dim3(1), dim3(256), 0, st, f); break;
        default: hipLaunchKernelGGL(k_apply_final<DIFFDRIVE>, dim3(1), dim3(256), 0, st, f); break;
    }
    HIP_LAUNCH_CHECK("k_apply_final");
    return D4_OK;
}

IterBuffers ctx_buffers(d4_ctx* c) {
    IterBuffers b;
    b.x0 = c->x0;
    b.goal = c->goal;
    b.ubase = c->ubase;
    b.eps = c->eps;
    b.r = c->r;
    b.du_a = c->du_a;
    b.du_b = c->du_b;
    b.traj = c->traj;
    b.stats = c->stats;
    b.hits = c->hits;
    b.status = c->status;
    b.iter = c->iter;
    return b;
}

bool graphs_disabled() { return g_opt_graphs.load() == 0; }

}  // namespace

// ------------------------------------------ workspace of the allocation-free entry point
// Every GPU the library runs on holds one copy of this array until the
// process ends.  Host code never uses the array's name as an address: each
// device's copy is reached through the pointer hipGetSymbolAddress returns
// on that device (scratch_on_device).
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[MAX_DEVICES] = {};

// The device address of the current device's scratch array, looked up once
// per device with that device current.
int scratch_on_device(int dev, unsigned char** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(D4_EUNSUPPORTED, "device %d beyond %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(D4_EHIP, "hipGetSymbolAddress of the static workspace failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return D4_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* d4_last_error(void) { return g_err.c_str(); }

int32_t d4_set_option(int32_t option, int32_t value) {
    switch (option) {
        case D4_OPT_GRAPHS:
            if (value != 0 && value != 1) return fail(D4_EINVAL, "D4_OPT_GRAPHS takes 0 or 1, not %d", value);
            g_opt_graphs.store(value);
            return D4_OK;
        case D4_OPT_ALIGNED_DRAWS:
            if (value != 0 && value != 1) return fail(D4_EINVAL, "D4_OPT_ALIGNED_DRAWS takes 0 or 1, not %d", value);
            g_opt_aligned_draws.store(value);
            return D4_OK;
        case D4_OPT_UPDATE_GRID:
            if (value < 0 || value > 65535) return fail(D4_EINVAL, "D4_OPT_UPDATE_GRID %d outside 0..65535", value);
            g_opt_update_grid.store(value);
            return D4_OK;
        case D4_OPT_BATCH_PERSISTENT:
            if (value != 0 && value != 1) return fail(D4_EINVAL, "D4_OPT_BATCH_PERSISTENT takes 0 or 1, not %d", value);
            // the persistent step did not finish on the GPU and is switched off
            // until the cause is found (the two-launch form serves every batch)
            if (value == 1) return fail(D4_EUNSUPPORTED, "the persistent batched step is switched off");
            g_opt_batch_persistent.store(value);
            return D4_OK;
        case D4_OPT_GEMM_TILE:
            if (value != 0 && value != 64 && value != 128)
                return fail(D4_EINVAL, "D4_OPT_GEMM_TILE takes 0, 64 or 128, not %d", value);
            g_opt_gemm_tile.store(value);
            return D4_OK;
        default: return fail(D4_EINVAL, "unknown option %d", option);
    }
}

int32_t d4_get_option(int32_t option, int32_t* value) {
    if (!value) return fail(D4_EINVAL, "value is NULL");
    switch (option) {
        case D4_OPT_GRAPHS: *value = g_opt_graphs.load(); return D4_OK;
        case D4_OPT_ALIGNED_DRAWS: *value = g_opt_aligned_draws.load(); return D4_OK;
        case D4_OPT_UPDATE_GRID: *value = g_opt_update_grid.load(); return D4_OK;
        case D4_OPT_BATCH_PERSISTENT: *value = g_opt_batch_persistent.load(); return D4_OK;
        case D4_OPT_GEMM_TILE: *value = g_opt_gemm_tile.load(); return D4_OK;
        default: return fail(D4_EINVAL, "unknown option %d", option);
    }
}

int32_t d4_noise(const d4_problem* p, uint32_t iter, uint32_t step, float* eps, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    NEED(eps);
    if (iter > 65535u || step < 1u || step > 65535u)
        return fail(D4_EINVAL, "iter %u / step %u outside the 16-bit counter fields", iter, step);
    const int D = p->n_robots * p->horizon * shape_of(p->dyn).du;
    const int M = p->n_samples;
    const dim3 grid((M + 255) / 256, (D + 3) / 4);
    hipLaunchKernelGGL(k_noise, grid, dim3(256), 0, (hipStream_t)stream, eps, D, M,
                       (iter << 16) | step, p->instance_id, (uint32_t)(p->seed & 0xFFFFFFFFull),
                       (uint32_t)(p->seed >> 32));
    HIP_LAUNCH_CHECK("k_noise");
    return D4_OK;
}

int32_t d4_box_muller(const uint32_t* words, int64_t count, float* z, void* stream) {
    if (count < 0) return fail(D4_EINVAL, "count %lld < 0", (long long)count);
    if (count == 0) return D4_OK;
    NEED(words);
    NEED(z);
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(k_box_muller, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, words, count, z);
    HIP_LAUNCH_CHECK("k_box_muller");
    return D4_OK;
}

int32_t d4_rollout(const d4_problem* p, const float* x0, const float* u, float* x, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    NEED(x0);
    NEED(u);
    NEED(x);
    const int total = p->n_samples * p->n_robots;
    const dim3 grid((total + 255) / 256);
    const StepConsts sc = step_consts(p);
    hipStream_t st = (hipStream_t)stream;
#define D4_ROLL(DY)                                                                              \
    hipLaunchKernelGGL(k_rollout<DY>, grid, dim3(256), 0, st, x0, u, x, p->n_robots, p->horizon, \
                       p->n_samples, sc, p->u_lo[0], p->u_lo[1], p->u_lo[2], p->u_hi[0],         \
                       p->u_hi[1], p->u_hi[2])
    switch (p->dyn) {
        case HOLO2D: D4_ROLL(HOLO2D); break;
        case HOLO3D: D4_ROLL(HOLO3D); break;
        case UNICYCLE: D4_ROLL(UNICYCLE); break;
        default: D4_ROLL(DIFFDRIVE); break;
    }
#undef D4_ROLL
    HIP_LAUNCH_CHECK("k_rollout");
    return D4_OK;
}

int32_t d4_fitness(const d4_problem* p, const float* x, const float* goal, float* r, int32_t* hits,
                   int32_t* robots_hit, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    NEED(x);
    NEED(goal);
    NEED(r);
    NEED(hits);
    if (robots_hit) NEED(robots_hit);
    const Tile tile = pick_tile(p);
    RollFitArgs a = base_args(p, tile);
    a.xs = x;
    a.goal = goal;
    a.r = r;
    a.hits = hits;
    a.robots_hit = robots_hit;
    return launch_rollfit<true>(p, a, tile, (hipStream_t)stream);
}

int32_t d4_sample_rollout_fitness(const d4_problem* p, const float* x0, const float* goal,
                                  const float* u_base, const float* du_in, uint32_t iter,
                                  uint32_t step, float* eps, float* r, int32_t* hits, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    NEED(x0);
    NEED(goal);
    NEED(u_base);
    NEED(du_in);
    NEED(eps);
    NEED(r);
    NEED(hits);
    if (iter > 65535u || step < 1u || step > (uint32_t)p->n_steps)
        return fail(D4_EINVAL, "iter %u or step %u out of range", iter, step);
    const Schedule sc = make_schedule(p);
    const Tile tile = pick_tile(p);
    RollFitArgs a = base_args(p, tile);
    a.x0 = x0;
    a.goal = goal;
    a.u_base = u_base;
    a.du_in = du_in;
    a.eps = eps;
    a.r = r;
    a.hits = hits;
    a.iter = iter;
    a.step = step;
    a.mean_scale = sc.ms[step];
    a.sigma = sc.sigma[step];
    return launch_rollfit<false>(p, a, tile, (hipStream_t)stream);
}

int32_t d4_score_update(const d4_problem* p, const float* r, const float* eps, const float* du_in,
                        int32_t step, float* du_out, float* w_out, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    NEED(r);
    NEED(eps);
    NEED(du_in);
    NEED(du_out);
    if (step < 1 || step > p->n_steps) return fail(D4_EINVAL, "step %d outside 1..N", step);
    if (du_out == du_in) return fail(D4_EINVAL, "du_out must not alias du_in");
    hipStream_t st = (hipStream_t)stream;
    if (w_out) NEED(w_out);
    if (p->n_samples > 16384)
        return fail(D4_EUNSUPPORTED, "n_samples %d above the 16384 weights one workgroup stages", p->n_samples);
    const Schedule sc = make_schedule(p);
    return launch_update(p, eps, r, du_in, du_out, w_out, nullptr, sc.ms[step], sc.sigma[step], sc.os[step], st);
}

int32_t d4_ctx_create(const d4_problem* p, d4_ctx** out) {
    int rc = validate(p);
    if (rc) return rc;
    if (!out) return fail(D4_EINVAL, "ctx out-pointer is NULL");
    if (p->n_samples > 16384)
        return fail(D4_EUNSUPPORTED, "n_samples %d above the 16384 weights one workgroup stages", p->n_samples);
    d4_ctx* c = new (std::nothrow) d4_ctx;
    if (!c) return fail(D4_ENOMEM, "host allocation failed");
    std::memset(c, 0, sizeof *c);
    c->prob = *p;
    HIP_TRY(hipGetDevice(&c->device));
    const Shape s = shape_of(p->dyn);
    const size_t n = p->n_robots, T = p->horizon, M = p->n_samples;
    const size_t D = n * T * s.du;
    struct {
        void** ptr;
        size_t bytes;
    } allocs[] = {
        {(void**)&c->eps, 4 * D * M}, {(void**)&c->r, 4 * M},       {(void**)&c->w, 4 * M},
        {(void**)&c->du_a, 4 * D},    {(void**)&c->du_b, 4 * D},    {(void**)&c->x0, 4 * n * s.dx},
        {(void**)&c->goal, 4 * n * s.dp}, {(void**)&c->ubase, 4 * D}, {(void**)&c->traj, 4 * n * (T + 1) * s.dx},
        {(void**)&c->stats, sizeof(d4_stats)}, {(void**)&c->hits, 4 * M}, {(void**)&c->status, 4},
        {(void**)&c->iter, 4},
    };
    for (auto& a : allocs) {
        if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
            free_ctx_buffers(c);
            delete c;
            return fail(D4_ENOMEM, "hipMalloc of %zu bytes failed", a.bytes);
        }
    }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        free_ctx_buffers(c);
        delete c;
        return fail(D4_EHIP, "stream creation failed");
    }
    *out = c;
    return D4_OK;
}

int32_t d4_ctx_destroy(d4_ctx* c) {
    if (!c) return D4_OK;
    (void)hipDeviceSynchronize();
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    free_ctx_buffers(c);
    delete c;
    return D4_OK;
}

int32_t d4_denoise_iter(d4_ctx* c, const d4_problem* p, const float* x0, const float* goal,
                        float* u_base, uint32_t iter, float* traj_out, d4_stats* stats,
                        void* stream) {
    if (!c) return fail(D4_EINVAL, "ctx is NULL");
    int rc = validate(p);
    if (rc) return rc;
    NEED(x0);
    NEED(goal);
    NEED(u_base);
    if (traj_out) NEED(traj_out);
    if (iter > 65535u) return fail(D4_EINVAL, "iter %u does not fit 16 bits", iter);
    if (!same_shape(*p, c->prob)) return fail(D4_EINVAL, "problem shape differs from the ctx's");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != c->device) return fail(D4_EINVAL, "ctx was created on device %d, current is %d", c->device, dev);
    hipStream_t st = (hipStream_t)stream;
    if (!same_problem(*p, c->prob)) {
        // scalars baked into the graph changed: capture again
        c->prob = *p;
        if (c->exec) (void)hipGraphExecDestroy(c->exec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        c->exec = nullptr;
        c->graph = nullptr;
        c->captured = false;
    }
    const Shape s = shape_of(p->dyn);
    const size_t n = p->n_robots, T = p->horizon;
    const size_t D = n * T * s.du;
    HIP_TRY(hipMemcpyAsync(c->x0, x0, 4 * n * s.dx, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->goal, goal, 4 * n * s.dp, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->ubase, u_base, 4 * D, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_set_iter, dim3(1), dim3(1), 0, st, c->iter, iter, c->status);
    HIP_LAUNCH_CHECK("k_set_iter");
    if (graphs_disabled()) {
        rc = enqueue_iteration(&c->prob, ctx_buffers(c), st);
        if (rc) return rc;
    } else {
        if (!c->captured) {
            HIP_TRY(hipStreamSynchronize(st));
            HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            rc = enqueue_iteration(&c->prob, ctx_buffers(c), c->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (ec != hipSuccess) return fail(D4_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
            c->graph = g;
            HIP_TRY(hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0));
            c->captured = true;
        }
        HIP_TRY(hipGraphLaunch(c->exec, st));
    }
    HIP_TRY(hipMemcpyAsync(u_base, c->ubase, 4 * D, hipMemcpyDeviceToDevice, st));
    if (traj_out)
        HIP_TRY(hipMemcpyAsync(traj_out, c->traj, 4 * n * (T + 1) * s.dx, hipMemcpyDeviceToDevice, st));
    if (stats) HIP_TRY(hipMemcpyAsync(stats, c->stats, sizeof(d4_stats), hipMemcpyDeviceToHost, st));
    return D4_OK;
}

int32_t d4_denoise_iter_noalloc(const d4_problem* p, const float* x0, const float* goal, float* u_base,
                                uint32_t iter, float* traj_out, d4_stats* stats, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    NEED(x0);
    NEED(goal);
    NEED(u_base);
    if (traj_out) NEED(traj_out);
    if (iter > 65535u) return fail(D4_EINVAL, "iter %u does not fit 16 bits", iter);
    if (p->n_samples > 16384)
        return fail(D4_EUNSUPPORTED, "n_samples %d above the 16384 weights one workgroup stages", p->n_samples);
    const Shape s = shape_of(p->dyn);
    const size_t n = p->n_robots, T = p->horizon, M = p->n_samples, D = n * T * s.du;
    // workspace layout: eps [D][M], r [M], hits [M], Delta U ping-pong, trajectory, stats, status, iteration
    const size_t o_eps = 0, o_r = o_eps + align256(4 * D * M), o_hits = o_r + align256(4 * M),
                 o_dua = o_hits + align256(4 * M), o_dub = o_dua + align256(4 * D),
                 o_traj = o_dub + align256(4 * D), o_stats = o_traj + align256(4 * n * (T + 1) * s.dx),
                 o_status = o_stats + align256(sizeof(d4_stats)), o_iter = o_status + 256, total = o_iter + 256;
    if (total > STATIC_SCRATCH_BYTES)
        return fail(D4_EUNSUPPORTED, "problem needs %zu bytes of workspace, above the %zu of the static array", total,
                    STATIC_SCRATCH_BYTES);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    unsigned char* base = nullptr;
    rc = scratch_on_device(dev, &base);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    IterBuffers b;
    b.x0 = x0;
    b.goal = goal;
    b.ubase = u_base;
    b.eps = reinterpret_cast<float*>(base + o_eps);
    b.r = reinterpret_cast<float*>(base + o_r);
    b.hits = reinterpret_cast<int*>(base + o_hits);
    b.du_a = reinterpret_cast<float*>(base + o_dua);
    b.du_b = reinterpret_cast<float*>(base + o_dub);
    b.traj = traj_out ? traj_out : reinterpret_cast<float*>(base + o_traj);
    b.stats = reinterpret_cast<float*>(base + o_stats);
    b.status = reinterpret_cast<int*>(base + o_status);
    b.iter = reinterpret_cast<uint32_t*>(base + o_iter);
    // the iteration index and the status word, written by a kernel (the
    // previous call's values stay in the array)
    hipLaunchKernelGGL(k_set_iter, dim3(1), dim3(1), 0, st, b.iter, iter, b.status);
    HIP_LAUNCH_CHECK("k_set_iter");
    rc = enqueue_iteration(p, b, st);
    if (rc) return rc;
    if (stats) HIP_TRY(hipMemcpyAsync(stats, b.stats, sizeof(d4_stats), hipMemcpyDeviceToHost, st));
    return D4_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ tuning
namespace d4host {

namespace {
std::mutex g_tile_mu;
std::map<std::tuple<int, int, int>, Tile> g_tiles;
}  // namespace

bool tile_override(int dyn, int n, int T, Tile* out) {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tiles.find(std::make_tuple(dyn, n, T));
    if (it == g_tiles.end()) return false;
    *out = it->second;
    return true;
}

namespace {
struct BatchBucket {
    int dyn, n_lo, n_hi, t_lo, t_hi;
    Tile tile;
};
std::vector<BatchBucket> g_batch_buckets;
}  // namespace

Tile batch_tile(int dyn, int n, int T) {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    for (const BatchBucket& b : g_batch_buckets)
        if (b.dyn == dyn && n >= b.n_lo && n <= b.n_hi && T >= b.t_lo && T <= b.t_hi) return b.tile;
    return default_tile(dyn, n);
}

}  // namespace d4host

namespace {

int tile_ok(const d4_problem* p, Tile t) {
    const int cs = shape_of(p->dyn).du == 2 ? 2 : 4;
    // a workgroup holds S samples of all n robots (times R replicas): at most 256 lanes
    // for the one-lane kernel, 1024 for the cooperative one
    if (t.S < 1 || t.S > 64 || t.S * p->n_robots > 256) return fail(D4_EINVAL, "samples per group %d invalid", t.S);
    if (t.R < 1 || t.R > 16 || t.R * t.S * p->n_robots > 1024) return fail(D4_EINVAL, "replicas %d invalid", t.R);
    if (t.Tb < cs || t.Tb > 64 || t.Tb % cs) return fail(D4_EINVAL, "steps per block %d invalid", t.Tb);
    if (rollfit_lds(p, t) > LDS_DYNAMIC_MAX) return fail(D4_EUNSUPPORTED, "tile needs too much LDS");
    return D4_OK;
}

}  // namespace

extern "C" {

int32_t d4_tile_set(int32_t dyn, int32_t n_robots, int32_t horizon, int32_t samples_per_group,
                    int32_t steps_per_block, int32_t replicas) {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    const auto key = std::make_tuple((int)dyn, (int)n_robots, (int)horizon);
    if (samples_per_group == 0) {
        g_tiles.erase(key);
        return D4_OK;
    }
    d4_problem p;
    std::memset(&p, 0, sizeof p);
    p.dyn = dyn;
    p.n_robots = n_robots;
    p.horizon = horizon;
    if (dyn < 0 || dyn > 3 || n_robots < 1 || n_robots > 32 || horizon < 1)
        return fail(D4_EINVAL, "bad problem shape");
    Tile t;
    t.S = samples_per_group;
    t.Tb = steps_per_block;
    t.R = replicas;
    int rc = tile_ok(&p, t);
    if (rc) return rc;
    g_tiles[key] = t;
    return D4_OK;
}

int32_t d4_batch_tile_set(int32_t dyn, int32_t n_lo, int32_t n_hi, int32_t t_lo, int32_t t_hi,
                          int32_t samples_per_group, int32_t steps_per_block) {
    if (dyn < 0 || dyn > 3 || n_lo < 1 || n_hi < n_lo || n_hi > 32 || t_lo < 1 || t_hi < t_lo)
        return fail(D4_EINVAL, "bad bucket");
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto same = [&](const BatchBucket& b) {
        return b.dyn == dyn && b.n_lo == n_lo && b.n_hi == n_hi && b.t_lo == t_lo && b.t_hi == t_hi;
    };
    g_batch_buckets.erase(std::remove_if(g_batch_buckets.begin(), g_batch_buckets.end(), same),
                          g_batch_buckets.end());
    if (samples_per_group == 0) return D4_OK;
    // the tile must be admissible for the bucket's largest team
    d4_problem p;
    std::memset(&p, 0, sizeof p);
    p.dyn = dyn;
    p.n_robots = n_hi;
    p.horizon = t_hi;
    Tile t;
    t.S = samples_per_group;
    t.Tb = steps_per_block;
    t.R = 1;
    int rc = tile_ok(&p, t);
    if (rc) return rc;
    if (rollfit_lds(&p, t) > LDS_TWO_PER_CU)
        return fail(D4_EUNSUPPORTED, "bucket tile needs %zu bytes of LDS, above the %zu of two workgroups per CU",
                    rollfit_lds(&p, t), LDS_TWO_PER_CU);
    for (const BatchBucket& b : g_batch_buckets)
        if (b.dyn == dyn && n_lo <= b.n_hi && b.n_lo <= n_hi && t_lo <= b.t_hi && b.t_lo <= t_hi)
            return fail(D4_EINVAL, "bucket overlaps an installed one");
    g_batch_buckets.push_back(BatchBucket{dyn, n_lo, n_hi, t_lo, t_hi, t});
    return D4_OK;
}

int32_t d4_tile_get(const d4_problem* p, int32_t batched, int32_t* samples_per_group, int32_t* steps_per_block,
                    int32_t* replicas) {
    int rc = validate(p);
    if (rc) return rc;
    const Tile t = batched ? batch_tile(p->dyn, p->n_robots, p->horizon) : pick_tile(p);
    if (samples_per_group) *samples_per_group = t.S;
    if (steps_per_block) *steps_per_block = t.Tb;
    if (replicas) *replicas = t.R;
    return D4_OK;
}

int32_t d4_autotune(const d4_problem* p, const float* x0, const float* goal, int32_t reps,
                    int32_t* samples_per_group, int32_t* steps_per_block, int32_t* replicas, float* best_us) {
    int rc = validate(p);
    if (rc) return rc;
    NEED(x0);
    NEED(goal);
    if (reps < 1) reps = 2;
    if (p->n_samples > 16384)
        return fail(D4_EUNSUPPORTED, "n_samples %d above the 16384 weights one workgroup stages", p->n_samples);
    const Shape s = shape_of(p->dyn);
    const int n = p->n_robots, cs = s.du == 2 ? 2 : 4;
    const size_t D = (size_t)n * p->horizon * s.du;
    d4_ctx* c = nullptr;
    rc = d4_ctx_create(p, &c);
    if (rc) return rc;
    float* u1 = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    Tile prev;
    const bool had_prev = tile_override(p->dyn, n, p->horizon, &prev);
    auto set_override = [&](const Tile* t) {
        std::lock_guard<std::mutex> lk(g_tile_mu);
        const auto key = std::make_tuple((int)p->dyn, n, (int)p->horizon);
        if (t) g_tiles[key] = *t;
        else g_tiles.erase(key);
    };
    auto release = [&]() {
        if (u1) (void)hipFree(u1);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)d4_ctx_destroy(c);
    };
    auto give_up = [&](int code, const char* what) {
        set_override(had_prev ? &prev : nullptr);
        release();
        return fail(code, "autotune: %s", what);
    };
    if (hipMalloc(&u1, 4 * D) != hipSuccess) return give_up(D4_ENOMEM, "plan buffer allocation failed");
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return give_up(D4_EHIP, "could not create its timing events");
    hipStream_t st = c->cap_stream;
    const IterBuffers b = ctx_buffers(c);
    const Shape sh = shape_of(p->dyn);
    if (hipMemcpyAsync(c->x0, x0, 4 * n * sh.dx, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(c->goal, goal, 4 * n * sh.dp, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemsetAsync(c->ubase, 0, 4 * D, st) != hipSuccess)
        return give_up(D4_EHIP, "could not stage its inputs");
    // a representative plan: one iteration from zero controls under the rule
    set_override(nullptr);
    const Tile rule = pick_tile(p);
    hipLaunchKernelGGL(k_set_iter, dim3(1), dim3(1), 0, st, c->iter, 0u, c->status);
    if (enqueue_iteration(p, b, st) != D4_OK) return give_up(D4_EHIP, "the first iteration failed");
    if (hipMemcpyAsync(u1, c->ubase, 4 * D, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return give_up(D4_EHIP, "the first iteration failed");
    // time of the iteration from that plan with tile t installed (the rule when
    // t is null): one untimed run, then the least of `reps`
    auto time_tile = [&](const Tile* t) -> float {
        set_override(t);
        float best = 1e30f;
        for (int k = 0; k <= reps; ++k) {
            if (hipMemcpyAsync(c->ubase, u1, 4 * D, hipMemcpyDeviceToDevice, st) != hipSuccess) return 1e30f;
            hipLaunchKernelGGL(k_set_iter, dim3(1), dim3(1), 0, st, c->iter, 1u, c->status);
            (void)hipEventRecord(e0, st);
            if (enqueue_iteration(p, b, st) != D4_OK) return 1e30f;
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) return 1e30f;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (k > 0 && ms < best) best = ms;
        }
        return best;
    };
    const float t_rule = time_tile(nullptr);
    if (t_rule >= 1e30f) return give_up(D4_EHIP, "the rule's tile could not be timed");
    float t_best = t_rule;
    Tile best_t = rule;
    for (int S : {rule.S / 2, rule.S, rule.S * 2}) {
        if (S < 1 || S > 64) continue;
        for (int R : {1, 2, 4, 8, 16}) {
            if (R > 1 && S * n * R < 64) continue;  // a cooperative workgroup below one wave
            for (int Tb : {4, 8, 12, 16, 20, 24, 32, 48, 64}) {
                Tile t;
                t.S = S;
                t.Tb = Tb;
                t.R = R;
                if (Tb % cs || (t.S == rule.S && t.Tb == rule.Tb && t.R == rule.R)) continue;
                if (S * n > 256 || R * S * n > 1024 || rollfit_lds(p, t) > LDS_DYNAMIC_MAX) continue;
                const float tm = time_tile(&t);
                if (tm < t_best) {
                    t_best = tm;
                    best_t = t;
                }
            }
        }
    }
    // a tile other than the rule's is kept only when it is at least 1 % faster
    if (t_best > 0.99f * t_rule) {
        best_t = rule;
        t_best = t_rule;
        set_override(nullptr);
    } else {
        set_override(&best_t);
    }
    release();
    if (samples_per_group) *samples_per_group = best_t.S;
    if (steps_per_block) *steps_per_block = best_t.Tb;
    if (replicas) *replicas = best_t.R;
    if (best_us) *best_us = t_best * 1000.0f / (float)p->n_steps;
    return D4_OK;
}

}  // extern "C"
