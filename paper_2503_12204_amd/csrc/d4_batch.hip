// Host side of the batched form: many independent planning problems of
// uneven team size, horizon and dynamics advanced together, one graph per
// iteration.  Each denoising step is one reward launch and one update launch.
// The persistent form (one launch per step over a work list of reward and
// update tiles, k_batch_persist) is built but switched off: it did not
// finish on the GPU, and d4_set_option refuses to select it.
#include "d4.h"
#include "d4_host.hpp"

using namespace d4;
using namespace d4host;

struct d4_batch {
    int count;
    int device;
    std::vector<d4_problem> probs;
    std::vector<BatchInst> insts;
    std::vector<BatchTile> tiles;
    std::vector<BatchRows> rows;
    long long tot_x0, tot_goal, tot_u, tot_eps, tot_r, tot_traj;
    size_t lds_rollfit;
    // device buffers
    BatchInst* d_insts;
    BatchTile* d_tiles;
    BatchRows* d_rows;
    float *x0, *goal, *u, *du_a, *du_b, *eps, *r, *traj, *stats;
    int *hits, *status;
    uint32_t* iter;
    // persistent step: work list, reward tiles per instance, two counter sets
    std::vector<BatchWork> work;
    BatchWork* d_work;
    int* d_tiles_of;
    int* d_cnt;
    int persist_grid;
    int captured_form;
    bool captured;
    hipStream_t cap_stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {


bool same_sampler(const d4_problem& a, const d4_problem& b) {
    return a.n_samples == b.n_samples && a.n_steps == b.n_steps && a.temperature == b.temperature &&
           a.beta_min == b.beta_min && a.beta_max == b.beta_max && a.flags == b.flags && a.seed == b.seed;
}

// Relative cost of one reward tile: steps times the per-lane work of a step.
double tile_cost(const d4_problem& p) {
    const Shape s = shape_of(p.dyn);
    const double dyn_ops = p.dyn == UNICYCLE ? 13 : p.dyn == DIFFDRIVE ? 17 : 5 * s.dp;
    return (double)p.horizon * (s.du * 66.0 + dyn_ops + (2 * s.dp + 3) * (1 + (p.n_robots - 1) / 2.0) + 4);
}

void free_batch(d4_batch* b) {
    void* ptrs[] = {b->d_insts, b->d_tiles, b->d_rows, b->x0,     b->goal,  b->u,      b->du_a,
                    b->du_b,    b->eps,     b->r,      b->traj,   b->stats, b->hits,   b->status,
                    b->iter,    b->d_work,  b->d_tiles_of, b->d_cnt};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

constexpr int ROWS_PER_TILE = 64;

// Polls of an update tile's wait before the persistent step gives up on it:
// each poll is one device-scope load (about a microsecond) and a sleep of
// about 512 cycles, some 0.1 s in all, against reward tiles of well under a
// millisecond.
constexpr int SPIN_LIMIT = 1 << 16;

struct InstPlan {
    int S, D;
    double cost;
};

// Work list of the persistent step.  Instances in descending tile cost; the
// reward tiles of each instance in turn; the update tiles of instance j
// follow once `lag` further reward tiles have been listed after its last one
// (by the time a workgroup takes them, instance j's tiles have most likely
// finished, and its draws are still in the Infinity Cache), and the update
// tiles still pending close the list.  Every reward tile of an instance
// precedes every update tile of it.
std::vector<BatchWork> batch_work_list(const std::vector<InstPlan>& ip, int M, int lag) {
    const int count = (int)ip.size();
    std::vector<int> order(count);
    for (int j = 0; j < count; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return ip[x].cost > ip[y].cost; });
    std::vector<BatchWork> out;
    std::vector<std::pair<long long, int>> pending;  // (reward tiles listed when j's last one was, j)
    size_t head = 0;
    long long rewards = 0;
    auto emit_updates = [&](int j) {
        for (int e0 = 0; e0 < ip[j].D; e0 += ROWS_PER_TILE)
            out.push_back(BatchWork{1, j, e0, std::min(ip[j].D, e0 + ROWS_PER_TILE)});
    };
    for (int j : order) {
        for (int m0 = 0; m0 < M; m0 += ip[j].S) {
            out.push_back(BatchWork{0, j, m0, 0});
            ++rewards;
            while (head < pending.size() && pending[head].first + lag <= rewards) emit_updates(pending[head++].second);
        }
        pending.push_back({rewards, j});
    }
    while (head < pending.size()) emit_updates(pending[head++].second);
    return out;
}

InstPlan plan_of(const d4_problem& p) {
    const Tile t = batch_tile(p.dyn, p.n_robots, p.horizon);
    return InstPlan{t.S, p.n_robots * p.horizon * shape_of(p.dyn).du, tile_cost(p)};
}

int enqueue_batch_iteration(d4_batch* b, hipStream_t st) {
    const d4_problem& p0 = b->probs[0];
    const Schedule sc = make_schedule(&p0);
    const int M = p0.n_samples;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((b->tot_u + 255) / 256)), dim3(256), 0, st, b->du_a,
                       (int)b->tot_u, 0.0f);
    HIP_LAUNCH_CHECK("k_fill");
    float* du_cur = b->du_a;
    float* du_nxt = b->du_b;
    BatchStepArgs a;
    std::memset(&a, 0, sizeof a);
    a.insts = b->d_insts;
    a.tiles = b->d_tiles;
    a.x0 = b->x0;
    a.goal = b->goal;
    a.u = b->u;
    a.eps = b->eps;
    a.r = b->r;
    a.hits = b->hits;
    a.iter_dev = b->iter;
    a.M = M;
    a.key0 = (uint32_t)(p0.seed & 0xFFFFFFFFull);
    a.key1 = (uint32_t)(p0.seed >> 32);
    a.flags = p0.flags;
    BatchUpdArgs ua;
    std::memset(&ua, 0, sizeof ua);
    ua.insts = b->d_insts;
    ua.rows = b->d_rows;
    ua.eps = b->eps;
    ua.r = b->r;
    ua.status = b->status;
    ua.M = M;
    ua.inv_lam = 1.0f / p0.temperature;
    ua.normalize = (p0.flags & FLAG_NORMALIZE) ? 1 : 0;
    allow_lds(k_batch_rollfit, b->lds_rollfit);
    const bool persist = g_opt_batch_persistent.load() != 0;
    const int J = upd_reg_j(M, b->eps, b->r);
    const int cnt_stride = CNT_DONE + b->count;
    if (persist) {
        // both counter sets start from zero (a kernel, not a memset, so that
        // the captured graph holds no memset node)
        hipLaunchKernelGGL(k_fill_int, dim3((2 * cnt_stride + 255) / 256), dim3(256), 0, st, b->d_cnt,
                           2 * cnt_stride, 0);
        HIP_LAUNCH_CHECK("k_fill_int");
    }
    for (int i = p0.n_steps; i >= 1; --i) {
        a.du_in = du_cur;
        a.step = (uint32_t)i;
        a.mean_scale = sc.ms[i];
        a.sigma = sc.sigma[i];
        ua.du_in = du_cur;
        ua.du_out = du_nxt;
        ua.ms = sc.ms[i];
        ua.sigma = sc.sigma[i];
        ua.os = sc.os[i];
        if (persist) {
            BatchPersistArgs pa;
            pa.s = a;
            pa.u = ua;
            pa.work = b->d_work;
            pa.tiles_of = b->d_tiles_of;
            pa.cnt = b->d_cnt + (i & 1) * cnt_stride;
            pa.n_work = (int)b->work.size();
            pa.count = b->count;
            pa.spin_limit = SPIN_LIMIT;
            const dim3 g((unsigned)b->persist_grid);
            switch (J) {
                case 0: hipLaunchKernelGGL(k_batch_persist<0>, g, dim3(256), b->lds_rollfit, st, pa); break;
                case 1: hipLaunchKernelGGL(k_batch_persist<1>, g, dim3(256), b->lds_rollfit, st, pa); break;
                case 2: hipLaunchKernelGGL(k_batch_persist<2>, g, dim3(256), b->lds_rollfit, st, pa); break;
                case 4: hipLaunchKernelGGL(k_batch_persist<4>, g, dim3(256), b->lds_rollfit, st, pa); break;
                case 8: hipLaunchKernelGGL(k_batch_persist<8>, g, dim3(256), b->lds_rollfit, st, pa); break;
                default: hipLaunchKernelGGL(k_batch_persist<16>, g, dim3(256), b->lds_rollfit, st, pa); break;
            }
            HIP_LAUNCH_CHECK("k_batch_persist");
            std::swap(du_cur, du_nxt);
            continue;
        }
        hipLaunchKernelGGL(k_batch_rollfit, dim3((unsigned)b->tiles.size()), dim3(256), b->lds_rollfit, st, a);
        HIP_LAUNCH_CHECK("k_batch_rollfit");
        const dim3 ng((unsigned)b->rows.size());
        switch (J) {
            case 0: hipLaunchKernelGGL(k_batch_update<0>, ng, dim3(256), (size_t)M * 4, st, ua); break;
            case 1: hipLaunchKernelGGL(k_batch_update<1>, ng, dim3(256), 0, st, ua); break;
            case 2: hipLaunchKernelGGL(k_batch_update<2>, ng, dim3(256), 0, st, ua); break;
            case 4: hipLaunchKernelGGL(k_batch_update<4>, ng, dim3(256), 0, st, ua); break;
            case 8: hipLaunchKernelGGL(k_batch_update<8>, ng, dim3(256), 0, st, ua); break;
            default: hipLaunchKernelGGL(k_batch_update<16>, ng, dim3(256), 0, st, ua); break;
        }
        HIP_LAUNCH_CHECK("k_batch_update");
        std::swap(du_cur, du_nxt);
    }
    BatchFinalArgs f;
    f.wait_error = persist ? b->d_cnt + CNT_ERROR : nullptr;
    f.cnt_stride = cnt_stride;
    f.insts = b->d_insts;
    f.u = b->u;
    f.du0 = du_cur;
    f.x0 = b->x0;
    f.goal = b->goal;
    f.traj = b->traj;
    f.stats = b->stats;
    f.status = b->status;
    f.flags = p0.flags;
    hipLaunchKernelGGL(k_batch_final, dim3((unsigned)b->count), dim3(256), 0, st, f);
    HIP_LAUNCH_CHECK("k_batch_final");
    return D4_OK;
}

}  // namespace

extern "C" {

int32_t d4_batch_create(const d4_problem* probs, int32_t count, d4_batch** out) {
    if (!probs || count < 1) return fail(D4_EINVAL, "need at least one problem");
    if (!out) return fail(D4_EINVAL, "batch out-pointer is NULL");
    for (int j = 0; j < count; ++j) {
        int rc = validate(&probs[j]);
        if (rc) return fail(rc, "instance %d: %s", j, g_err.c_str());
        if (!same_sampler(probs[j], probs[0]))
            return fail(D4_EINVAL, "instance %d: sampler settings differ from instance 0", j);
    }
    if (probs[0].n_samples > 16384)
        return fail(D4_EUNSUPPORTED, "n_samples %d above the 16384 weights one workgroup stages", probs[0].n_samples);
    d4_batch* b = new (std::nothrow) d4_batch();
    if (!b) return fail(D4_ENOMEM, "host allocation failed");
    b->count = count;
    b->probs.assign(probs, probs + count);
    HIP_TRY(hipGetDevice(&b->device));
    const long long M = probs[0].n_samples;
    long long ox = 0, og = 0, ou = 0, oe = 0, orr = 0, ot = 0;
    size_t lds = 0;
    std::vector<std::pair<double, BatchTile>> tl;
    for (int j = 0; j < count; ++j) {
        const d4_problem& p = probs[j];
        const Shape s = shape_of(p.dyn);
        const Tile t = batch_tile(p.dyn, p.n_robots, p.horizon);
        BatchInst in;
        std::memset(&in, 0, sizeof in);
        in.n = p.n_robots;
        in.T = p.horizon;
        in.dyn = p.dyn;
        in.S = t.S;
        in.Tb = t.Tb;
        in.mode = draws_aligned(&p) ? MODE_FUSED_ALIGNED : MODE_FUSED;
        in.D = p.n_robots * p.horizon * s.du;
        in.x0 = ox;
        in.goal = og;
        in.u = ou;
        in.eps = oe;
        in.r = orr;
        in.traj = ot;
        in.thr2 = thr2_reward(&p);
        const double s2 = 2.0 * (double)p.robot_radius;
        in.safe2 = (float)(s2 * s2);
        in.w_safe = p.w_safe;
        in.d0_floor = p.d0_floor;
        in.goal_tol = p.goal_tol;
        for (int d = 0; d < 3; ++d) {
            in.ulo[d] = p.u_lo[d];
            in.uhi[d] = p.u_hi[d];
        }
        in.sc = step_consts(&p);
        in.inst_id = p.instance_id;
        in.n_obs = p.n_obstacles;
        for (int o = 0; o < p.n_obstacles; ++o) {
            in.obs[o] = obstacle_reward(&p, o);
            in.obs_safe2[o] = obstacle_safe2(&p, o);
        }
        b->insts.push_back(in);
        const double cost = tile_cost(p);
        for (long long m0 = 0; m0 < M; m0 += t.S) tl.push_back({cost, BatchTile{j, (int)m0}});
        for (int e0 = 0; e0 < in.D; e0 += ROWS_PER_TILE)
            b->rows.push_back(BatchRows{j, e0, std::min(in.D, e0 + ROWS_PER_TILE)});
        lds = std::max(lds, rollfit_lds(&p, t));
        ox += (long long)p.n_robots * s.dx;
        og += (long long)p.n_robots * s.dp;
        ou += in.D;
        oe += (long long)in.D * M;
        orr += M;
        ot += (long long)p.n_robots * (p.horizon + 1) * s.dx;
    }
    if (lds > LDS_DYNAMIC_MAX) {
        delete b;
        return fail(D4_EUNSUPPORTED, "reward tiles need %zu bytes of LDS", lds);
    }
    // longest tiles first: the dispatcher hands workgroups out in order
    std::stable_sort(tl.begin(), tl.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    for (auto& t : tl) b->tiles.push_back(t.second);
    b->tot_x0 = ox;
    b->tot_goal = og;
    b->tot_u = ou;
    b->tot_eps = oe;
    b->tot_r = orr;
    b->tot_traj = ot;
    // At most two reward workgroups per CU: the batched kernel carries every
    // dynamics and draw alignment, and three workgroups of a mixed batch on a
    // CU ran 45 % slower than two (one per CU ran slower still).  Requesting
    // more than a third of the CU's LDS enforces the limit.
    b->lds_rollfit = std::max(lds, LDS_TWO_PER_CU);
    if (ou >= (1ll << 31) || oe >= (1ll << 40)) {
        delete b;
        return fail(D4_EUNSUPPORTED, "batch too large");
    }
    struct {
        void** ptr;
        size_t bytes;
    } allocs[] = {
        {(void**)&b->d_insts, sizeof(BatchInst) * b->insts.size()},
        {(void**)&b->d_tiles, sizeof(BatchTile) * b->tiles.size()},
        {(void**)&b->d_rows, sizeof(BatchRows) * b->rows.size()},
        {(void**)&b->x0, 4 * (size_t)ox},
        {(void**)&b->goal, 4 * (size_t)og},
        {(void**)&b->u, 4 * (size_t)ou},
        {(void**)&b->du_a, 4 * (size_t)ou},
        {(void**)&b->du_b, 4 * (size_t)ou},
        {(void**)&b->eps, 4 * (size_t)oe},
        {(void**)&b->r, 4 * (size_t)orr},
        {(void**)&b->hits, 4 * (size_t)orr},
        {(void**)&b->traj, 4 * (size_t)ot},
        {(void**)&b->stats, sizeof(d4_stats) * (size_t)count},
        {(void**)&b->status, 4 * (size_t)count},
        {(void**)&b->iter, 4},
        {(void**)&b->d_tiles_of, 4 * (size_t)count},
        {(void**)&b->d_cnt, 4 * 2 * (size_t)(CNT_DONE + count)},
    };
    for (auto& a : allocs) {
        if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
            free_batch(b);
            delete b;
            return fail(D4_ENOMEM, "hipMalloc of %zu bytes failed", a.bytes);
        }
    }
    // persistent step: occupancy-sized grid, work list, per-instance tile counts
    {
        std::vector<InstPlan> ip;
        std::vector<int> tiles_of;
        for (int j = 0; j < count; ++j) {
            ip.push_back(plan_of(probs[j]));
            tiles_of.push_back((int)((M + ip.back().S - 1) / ip.back().S));
        }
        int cus = 0, per_cu = 0;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
        allow_lds(k_batch_persist<1>, b->lds_rollfit);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_batch_persist<1>),
                                                         256, b->lds_rollfit) != hipSuccess)
            per_cu = 1;
        b->persist_grid = std::max(1, std::max(1, per_cu) * std::max(1, cus));
        b->work = batch_work_list(ip, (int)M, b->persist_grid);
        b->persist_grid = std::min<int>(b->persist_grid, (int)b->work.size());
        if (hipMalloc(&b->d_work, sizeof(BatchWork) * b->work.size()) != hipSuccess ||
            hipMemcpy(b->d_work, b->work.data(), sizeof(BatchWork) * b->work.size(), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(b->d_tiles_of, tiles_of.data(), 4 * (size_t)count, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(b->d_cnt, 0, 4 * 2 * (size_t)(CNT_DONE + count)) != hipSuccess) {
            free_batch(b);
            delete b;
            return fail(D4_ENOMEM, "persistent-step work list set-up failed");
        }
    }
    hipError_t e1 = hipMemcpy(b->d_insts, b->insts.data(), sizeof(BatchInst) * b->insts.size(), hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(b->d_tiles, b->tiles.data(), sizeof(BatchTile) * b->tiles.size(), hipMemcpyHostToDevice);
    hipError_t e3 = hipMemcpy(b->d_rows, b->rows.data(), sizeof(BatchRows) * b->rows.size(), hipMemcpyHostToDevice);
    hipError_t e4 = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
        free_batch(b);
        delete b;
        return fail(D4_EHIP, "batch set-up copies failed");
    }
    *out = b;
    return D4_OK;
}

int32_t d4_batch_layout(const d4_batch* b, int64_t* x0_off, int64_t* goal_off, int64_t* u_off, int64_t* totals) {
    if (!b) return fail(D4_EINVAL, "batch is NULL");
    for (int j = 0; j < b->count; ++j) {
        if (x0_off) x0_off[j] = b->insts[j].x0;
        if (goal_off) goal_off[j] = b->insts[j].goal;
        if (u_off) u_off[j] = b->insts[j].u;
    }
    if (totals) {
        totals[0] = b->tot_x0;
        totals[1] = b->tot_goal;
        totals[2] = b->tot_u;
    }
    return D4_OK;
}

int32_t d4_batch_iter(d4_batch* b, const float* x0_all, const float* goal_all, float* u_all, uint32_t iter,
                      d4_stats* stats, void* stream) {
    if (!b) return fail(D4_EINVAL, "batch is NULL");
    NEED(x0_all);
    NEED(goal_all);
    NEED(u_all);
    if (iter > 65535u) return fail(D4_EINVAL, "iter %u does not fit 16 bits", iter);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != b->device) return fail(D4_EINVAL, "batch was created on device %d, current is %d", b->device, dev);
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(b->x0, x0_all, 4 * (size_t)b->tot_x0, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(b->goal, goal_all, 4 * (size_t)b->tot_goal, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(b->u, u_all, 4 * (size_t)b->tot_u, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_fill_int, dim3((b->count + 255) / 256), dim3(256), 0, st, b->status, b->count, 0);
    HIP_LAUNCH_CHECK("k_fill_int");
    hipLaunchKernelGGL(k_set_iter, dim3(1), dim3(1), 0, st, b->iter, iter, b->status);
    HIP_LAUNCH_CHECK("k_set_iter");
    const int form = g_opt_batch_persistent.load();
    if (b->captured && b->captured_form != form) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        b->captured = false;
    }
    if (g_opt_graphs.load() == 0) {
        int rc = enqueue_batch_iteration(b, st);
        if (rc) return rc;
    } else {
        if (!b->captured) {
            b->captured_form = form;
            HIP_TRY(hipStreamSynchronize(st));
            HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_batch_iteration(b, b->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(b->cap_stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (ec != hipSuccess) return fail(D4_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
            b->graph = g;
            HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            b->captured = true;
        }
        HIP_TRY(hipGraphLaunch(b->exec, st));
    }
    HIP_TRY(hipMemcpyAsync(u_all, b->u, 4 * (size_t)b->tot_u, hipMemcpyDeviceToDevice, st));
    if (stats)
        HIP_TRY(hipMemcpyAsync(stats, b->stats, sizeof(d4_stats) * (size_t)b->count, hipMemcpyDeviceToHost, st));
    return D4_OK;
}

int32_t d4_batch_work_list(const d4_problem* probs, int32_t count, int32_t lag, int32_t capacity, int32_t* items,
                           int32_t* n_items) {
    if (!probs || count < 1) return fail(D4_EINVAL, "need at least one problem");
    if (lag < 0 || capacity < 0 || !n_items || (capacity > 0 && !items))
        return fail(D4_EINVAL, "bad lag, capacity or output");
    std::vector<InstPlan> ip;
    for (int j = 0; j < count; ++j) {
        int rc = validate(&probs[j]);
        if (rc) return fail(rc, "instance %d: %s", j, g_err.c_str());
        if (!same_sampler(probs[j], probs[0]))
            return fail(D4_EINVAL, "instance %d: sampler settings differ from instance 0", j);
        ip.push_back(plan_of(probs[j]));
    }
    const std::vector<BatchWork> w = batch_work_list(ip, probs[0].n_samples, lag);
    *n_items = (int32_t)w.size();
    if ((int64_t)w.size() > capacity) return fail(D4_EINVAL, "work list of %zu items exceeds capacity %d", w.size(), capacity);
    for (size_t i = 0; i < w.size(); ++i) {
        items[4 * i] = w[i].kind;
        items[4 * i + 1] = w[i].inst;
        items[4 * i + 2] = w[i].a;
        items[4 * i + 3] = w[i].b;
    }
    return D4_OK;
}

int32_t d4_batch_destroy(d4_batch* b) {
    if (!b) return D4_OK;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    free_batch(b);
    delete b;
    return D4_OK;
}

}  // extern "C"
