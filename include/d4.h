/*
 * d4.h - C ABI of the MI355X (gfx950) denoising hot path of D4orm
 * ("Multi-Robot Trajectories with Dynamics-aware Diffusion Denoised
 * Deformations", Zhang et al., 2025).
 *
 * Conventions shared by every entry point:
 *  - Every array argument is a DEVICE pointer unless marked "host".  The
 *    caller allocates and owns it; the library never frees caller memory.
 *  - Arrays are FP32 (int32 where stated), row-major, contiguous, and
 *    4-byte aligned at least; index orders are given per argument.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls only enqueue work on it and return; results are ready once the
 *    stream has synchronised.
 *  - Return value: D4_OK or a negative status.  On error nothing was
 *    enqueued, and d4_last_error() (thread-local) holds a message.  No C++
 *    exception crosses this boundary.
 *  - Device-side numerical failures (a non-finite reward) are reported in
 *    d4_stats.status after the stream has synchronised.
 *
 * Symbols: n robots, T horizon steps (controls u[0..T-1], states x[0..T]),
 * M Monte Carlo samples, N denoising steps, d_x/d_u/d_p state, control and
 * position dimensions, D = n*T*d_u, element e = (k*T + t)*d_u + d.
 */
#ifndef D4_H
#define D4_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    D4_OK = 0,
    D4_EINVAL = -1,        /* bad argument, nothing enqueued */
    D4_ENOMEM = -2,        /* device allocation failed */
    D4_EHIP = -3,          /* a HIP runtime call failed */
    D4_ENONFINITE = -4,    /* a reward was NaN or infinite (stats.status) */
    D4_EUNSUPPORTED = -5   /* shape or form beyond the library's limits */
};

/* Robot models (Section V).  HOLO2D/HOLO3D: x = [p, v], u = a.  UNICYCLE:
 * x = [p_x, p_y, theta], u = [v, omega].  DIFFDRIVE, the paper's differential
 * drive: x = [p_x, p_y, theta, v], u = [omega, a], speed clipped to v_max. */
enum { D4_HOLO2D = 0, D4_HOLO3D = 1, D4_UNICYCLE = 2, D4_DIFFDRIVE = 3 };

/* Flag bits of d4_problem.flags. */
enum {
    D4_NORMALIZE = 1,   /* z-score the batch rewards before the softmax */
    D4_SAFE_PAIRS = 2   /* r_safe = -(number of colliding partners) instead of -1 */
};

/* Most static obstacles of one problem. */
#define D4_MAX_OBSTACLES 16

/*
 * One planning problem and its sampler settings.  Problem data follow the
 * problem definition of Section III (team size, radius R_a, dynamics, horizon,
 * time step); reward weights follow Eq. generic-reward and the r_goal/r_safe
 * definitions of Section IV-A; temperature and schedule follow Section IV-B
 * and Algorithm 1.
 */
typedef struct d4_problem {
    int32_t dyn;            /* D4_HOLO2D, D4_HOLO3D, D4_UNICYCLE or D4_DIFFDRIVE */
    int32_t n_robots;       /* n, 1..32 */
    int32_t horizon;        /* T, >= 1 */
    int32_t n_samples;      /* M, >= 1 */
    int32_t n_steps;        /* N, 1..65535 */
    float dt;               /* > 0 */
    float robot_radius;     /* R_a >= 0: safety condition uses 2 R_a */
    float safety_margin;    /* epsilon >= 0: r_safe uses 2 R_a + epsilon */
    float w_safe;           /* weight of r_safe */
    float temperature;      /* lambda > 0 */
    float beta_min;         /* linear beta schedule, step 1 */
    float beta_max;         /* linear beta schedule, step N */
    float u_lo[3];          /* per-component control box */
    float u_hi[3];
    float v_max;            /* speed bound: per component (holonomic), |v| (DIFFDRIVE) */
    float goal_tol;         /* terminal-condition tolerance */
    float d0_floor;         /* floor of the r_goal denominator */
    uint32_t flags;         /* D4_NORMALIZE | D4_SAFE_PAIRS */
    uint32_t instance_id;   /* fourth Philox counter word */
    uint64_t seed;          /* Philox key */
    /* Static circular (spherical in 3D) obstacles of the appendix: each state
     * within R_a + radius + epsilon of any obstacle costs a binary penalty -1
     * in the team reward, weighted like r_safe; success also requires every
     * state farther than R_a + radius from every obstacle. */
    int32_t n_obstacles;                      /* 0..D4_MAX_OBSTACLES */
    float obstacles[D4_MAX_OBSTACLES][4];     /* centre x, y, z (z unused in 2D), radius >= 0 */
} d4_problem;

/* Outcome of one iteration, written by d4_denoise_iter (host memory). */
typedef struct d4_stats {
    float reward;           /* r(tau) of the updated plan (Eq. generic-reward) */
    float objective;        /* Eq. objective: fraction of robot-steps at the goal */
    int32_t hits;           /* colliding pairs (reward threshold) summed over t */
    int32_t robots_hit;     /* robot-steps with r_safe != 0 */
    int32_t success;        /* conflict-free: every pair farther apart than 2 R_a at t = 1..T
                               (feasibility holds by construction; Sec. V-A reads success as
                               feasible and conflict-free) */
    int32_t at_goal;        /* terminal condition: every robot within goal_tol of its goal at t = T */
    int32_t obstacle_hits;  /* robot-steps within an obstacle's reward distance (t = 1..T) */
    int32_t status;         /* D4_OK or D4_ENONFINITE */
} d4_stats;

typedef struct d4_ctx d4_ctx;

/* Message of the last failed call on this thread ("" if none). */
const char* d4_last_error(void);

/* Process-wide launch options.  None changes a result; each exists so that
 * tests can check that two launch forms agree bit for bit.
 *  D4_OPT_GRAPHS        1 (default): d4_denoise_iter and d4_batch_iter replay a
 *                       HIP graph captured on their first call; 0: they enqueue
 *                       the same launches directly on the caller's stream.
 *  D4_OPT_ALIGNED_DRAWS 1 (default): problems whose robots' draws start on a
 *                       Philox block (T d_u a multiple of 4) use the fused
 *                       kernel's whole-block draw window; 0: every problem uses
 *                       the general window.
 *  D4_OPT_UPDATE_GRID   0 (default): the update kernel's grid follows its rule
 *                       (at most 512 workgroups of two rows each); n > 0: n
 *                       workgroups (capped at D).
 *  D4_OPT_BATCH_PERSISTENT 0 (default): d4_batch_iter runs each denoising step
 *                       as one reward launch and one update launch; 1 would run
 *                       it as one persistent launch over a work list of reward
 *                       and update tiles, but that form is switched off in this
 *                       build (it did not finish on the GPU): setting 1 returns
 *                       D4_EUNSUPPORTED.
 *  D4_OPT_GEMM_TILE     0 (default): d4p_gemm_bf16 and the proposal's products
 *                       use 128x128 workgroup tiles when those still give at
 *                       least 256 workgroups, else 64x64; 64 or 128 fixes the
 *                       tile.
 * d4_set_option returns D4_EINVAL for an unknown option or a value outside the
 * ranges above; d4_get_option writes the current value to *value (host). */
enum {
    D4_OPT_GRAPHS = 0,
    D4_OPT_ALIGNED_DRAWS = 1,
    D4_OPT_UPDATE_GRID = 2,
    D4_OPT_BATCH_PERSISTENT = 3,
    D4_OPT_GEMM_TILE = 4
};
int32_t d4_set_option(int32_t option, int32_t value);
int32_t d4_get_option(int32_t option, int32_t* value);

/*
 * Standard normal draws of one denoising step (the sampling step of
 * Algorithm 1, Eq. mc).  eps[e][m], e < D, m < M, [D][M] layout.
 * Counter-based Philox4x32-10 with key (lo32(seed), hi32(seed)) and counter
 * (e>>2, m, (iter<<16)|step, instance_id); words pair into Box-Muller
 * normals with an FP32 ln and sin/cos evaluated one correctly rounded
 * operation at a time, so every implementation of the recipe draws the same
 * bits.  iter < 65536, 1 <= step < 65536.
 */
int32_t d4_noise(const d4_problem* p, uint32_t iter, uint32_t step, float* eps, void* stream);

/*
 * The Box-Muller stage of the d4_noise recipe on given generator words
 * (sampling step of Algorithm 1): for i < count, words[2i] feeds the radius
 * and words[2i+1] the angle; z[2i] = rho cos, z[2i+1] = rho sin.  words and
 * z are device arrays of 2*count elements; count >= 0 (0 launches nothing).
 * Lets a caller check the transform on every input it can receive.
 */
int32_t d4_box_muller(const uint32_t* words, int64_t count, float* z, void* stream);

/*
 * Rollout (Section III feasibility, Section IV-C): x[m][k][0] = x0[k];
 * x[m][k][t+1] = RK4(x[m][k][t], clip(u[m][k][t])) with holonomic speeds
 * clipped per component after each step.
 * x0 [n][d_x], u [M][n][T][d_u], x [M][n][T+1][d_x] (written).
 */
int32_t d4_rollout(const d4_problem* p, const float* x0, const float* u, float* x, void* stream);

/*
 * Team reward of trajectories (Eq. generic-reward with r_goal and r_safe of
 * Section IV-A).  x [M][n][T+1][d_x], goal [n][d_p]; writes r [M],
 * hits [M] (colliding pairs k<l summed over t=1..T, FP32 predicate
 * ((dx*dx + dy*dy) + dz*dz) <= RN32((2 R_a + epsilon)^2)), and, unless NULL,
 * robots_hit [M] (robot-steps with r_safe != 0).
 */
int32_t d4_fitness(const d4_problem* p, const float* x, const float* goal, float* r,
                   int32_t* hits, int32_t* robots_hit, void* stream);

/*
 * Fused sampling + rollout + reward of denoising step `step` (Algorithm 1,
 * sample and rollout steps, in the deformation form of Section IV-D):
 * draws eps as d4_noise, forms Delta U^(m) = du_in / sqrt(abar_step)
 * + sqrt(1/abar_step - 1) eps^(m), rolls out clip(u_base + Delta U^(m)) and
 * scores it.  x0 [n][d_x], goal [n][d_p], u_base [D], du_in [D];
 * writes eps [D][M], r [M], hits [M].
 */
int32_t d4_sample_rollout_fitness(const d4_problem* p, const float* x0, const float* goal,
                                  const float* u_base, const float* du_in, uint32_t iter,
                                  uint32_t step, float* eps, float* r, int32_t* hits,
                                  void* stream);

/*
 * Softmax weights and the one-step update (Eq. mc and Eq. mbd-denoising,
 * Algorithm 1 MC-estimate and denoise steps) for step `step`:
 * w = softmax(normalise(r) / lambda), S[e] = sum_m w[m] eps[e][m],
 * du_out[e] = sqrt(abar_{step-1}) (du_in[e] / sqrt(abar_step)
 * + sqrt(1/abar_step - 1) S[e]).  r [M], eps [D][M], du_in [D] -> du_out [D];
 * w_out [M] unless NULL.  du_out must not alias du_in.
 */
int32_t d4_score_update(const d4_problem* p, const float* r, const float* eps,
                        const float* du_in, int32_t step, float* du_out, float* w_out,
                        void* stream);

/*
 * Library-owned workspace for d4_denoise_iter: eps [D][M], r, hits, w,
 * the Delta U ping-pong, stats and the captured HIP graph.  The shape
 * (dyn, n, T, M, N) of later calls must match the one it was created for.
 */
int32_t d4_ctx_create(const d4_problem* p, d4_ctx** ctx);
int32_t d4_ctx_destroy(d4_ctx* ctx);

/*
 * One iteration of Algorithm 2: Delta U_N = 0, denoising steps N..1 of
 * Algorithm 1, then u_base <- clip(u_base + Delta U_0) and a rollout of the
 * updated plan.  x0 [n][d_x], goal [n][d_p], u_base [n][T][d_u] (read and
 * written); traj_out [n][T+1][d_x] unless NULL; stats (host memory, pinned
 * for a truly asynchronous call) unless NULL.  The N steps replay one HIP
 * graph captured on the first call.  Calls on one ctx must not overlap.
 */
int32_t d4_denoise_iter(d4_ctx* ctx, const d4_problem* p, const float* x0, const float* goal,
                        float* u_base, uint32_t iter, float* traj_out, d4_stats* stats,
                        void* stream);

/*
 * d4_denoise_iter for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels with the same results, but no d4_ctx, no graph and no
 * allocation of any kind.  The workspace (draws, rewards, counts, the Delta U
 * ping-pong, trajectory, stats, status) lives in one static device array of
 * 64 MiB that every GPU the library runs on holds until the process ends:
 * problems whose workspace (about 4 D M bytes plus small arrays) exceeds it
 * return D4_EUNSUPPORTED before any launch.  Arguments as d4_denoise_iter;
 * u_base is updated in place and x0, goal are read where they are.  Calls on
 * one GPU share the array, so calls that overlap on one GPU (concurrent
 * streams or threads) race; the array keeps the last call's contents.
 */
int32_t d4_denoise_iter_noalloc(const d4_problem* p, const float* x0, const float* goal, float* u_base,
                                uint32_t iter, float* traj_out, d4_stats* stats, void* stream);

/* ------------------------------------------------------------------------
 * Launch-shape tuning of the reward kernels (d4_sample_rollout_fitness,
 * d4_fitness, d4_denoise_iter).  A tile is the number of samples per
 * workgroup S (1..64), the number of steps per LDS time block (a multiple of
 * 2 for d_u = 2, of 4 for d_u = 3) and the replica lanes R per (sample,
 * robot) (1..16; R > 1 lets R lanes share the draws and pair checks of one
 * lane, for problems with too few lanes to fill the GPU; when S * n_robots is
 * a multiple of 64 the replicas also pipeline the serial rollout of one time
 * block against the draws of the next and the pair checks of the previous
 * one), with S * n_robots <= 256 and R * S * n_robots <= 1024.  A tile
 * changes only speed: every admissible tile gives the same bits.  The
 * batched form uses its own rule or the bucket tiles of d4_batch_tile_set
 * (R = 1).
 * ------------------------------------------------------------------------ */

/* Install (or, with samples_per_group = 0, remove) a process-wide tile for
 * problems of this (dyn, n_robots, horizon). */
int32_t d4_tile_set(int32_t dyn, int32_t n_robots, int32_t horizon, int32_t samples_per_group,
                    int32_t steps_per_block, int32_t replicas);

/* Install (or, with samples_per_group = 0, remove) the tile of the batched
 * form for instances of dynamics dyn with n_lo <= n_robots <= n_hi and
 * t_lo <= horizon <= t_hi (one replica lane; admissible for n_hi, and within
 * the 56 KiB of LDS that keeps two reward workgroups per CU, else
 * D4_EUNSUPPORTED: the largest request sets every workgroup's; buckets of one
 * dynamics must not overlap).  Batches created afterwards use it
 * (d4_batch_create reads the buckets); a tile changes only speed. */
int32_t d4_batch_tile_set(int32_t dyn, int32_t n_lo, int32_t n_hi, int32_t t_lo, int32_t t_hi,
                          int32_t samples_per_group, int32_t steps_per_block);

/* The tile the library uses for p: the batched form's bucket tile or rule
 * when batched is non-zero, else the single-problem choice (installed tile or
 * default).  Outputs are host pointers, each may be NULL. */
int32_t d4_tile_get(const d4_problem* p, int32_t batched, int32_t* samples_per_group, int32_t* steps_per_block,
                    int32_t* replicas);

/* Choose the launch tile of problem p on the current device by timing whole
 * iterations (Algorithm 2's loop body: N denoising steps and the apply step).
 * One iteration from zero controls under the rule gives a representative
 * plan; the iteration from that plan is then timed (one untimed run, the
 * least of reps, reps < 1 meaning 2) with the rule's tile and with each
 * candidate around it: samples per group S/2, S and 2S of the rule's S,
 * 1..16 replica lanes and 4..64 steps per block, when admissible.  x0 [n][d_x]
 * and goal [n][d_p] are device arrays: the broad phase of the pair checks
 * makes the cost depend on where the robots are.  A tile other than the
 * rule's is installed (as by d4_tile_set) only when it is at least 1 % faster;
 * otherwise the rule stays and any tile installed for this shape is removed.
 * Reports the chosen tile and its time per denoising step in microseconds
 * (outputs are host pointers, each may be NULL).  Allocates a context and a
 * plan buffer, frees them before returning, and synchronises its own stream.
 * Tiles change speed, never results.  The library keeps installed tiles in
 * memory only: the persistent cache of tuned tiles (keyed by architecture,
 * kernel source version and problem shape) is the Python layer's
 * (paper_2503_12204_amd/autotune.py), which reinstalls them with
 * d4_tile_set, so this call takes no cache path.  Errors: D4_EINVAL for a bad
 * problem or NULL inputs, D4_EUNSUPPORTED above 16384 samples, D4_ENOMEM or
 * D4_EHIP when its buffers or timings fail (any tile installed before the
 * call is then left as it was). */
int32_t d4_autotune(const d4_problem* p, const float* x0, const float* goal, int32_t reps,
                    int32_t* samples_per_group, int32_t* steps_per_block, int32_t* replicas, float* best_us);

/* ------------------------------------------------------------------------
 * Batched form: many independent problems advanced together.  Each instance
 * runs exactly the iteration of d4_denoise_iter (Algorithm 2 loop body over
 * Algorithm 1), with its own team size, horizon, dynamics, limits, start and
 * goal; every instance must share n_samples, n_steps, temperature,
 * beta_min/beta_max, flags and seed (instance_id tells their draws apart).
 * Each denoising step is one reward launch over all (instance, sample block)
 * tiles, longest first, and one update launch over all (instance, row range)
 * tiles; the iteration replays one captured HIP graph.  (A persistent form,
 * one launch per step taking reward and update tiles from the work list of
 * d4_batch_work_list, is built but switched off: see D4_OPT_BATCH_PERSISTENT.)
 * With the default launch shapes an instance's results equal its own
 * d4_denoise_iter run bit for bit.
 * ------------------------------------------------------------------------ */
typedef struct d4_batch d4_batch;

/* probs: host array of `count` problems (copied).  Allocates the workspace:
 * sum_j D_j * M floats of draws dominate.  D4_EINVAL if sampler settings
 * differ between instances.  There is no options argument: launch shapes come
 * from the shared tile rule and d4_set_option. */
int32_t d4_batch_create(const d4_problem* probs, int32_t count, d4_batch** batch);

/* Host outputs (each may be NULL): per-instance float offsets of the packed
 * start states (x0_off, [n_j][d_x]), goals (goal_off, [n_j][d_p]) and plans
 * (u_off, [n_j][T_j][d_u]) in instance order, and totals[3] = their lengths. */
int32_t d4_batch_layout(const d4_batch* batch, int64_t* x0_off, int64_t* goal_off, int64_t* u_off,
                        int64_t* totals);

/* One iteration for every instance.  x0_all, goal_all, u_all are packed
 * device arrays laid out as d4_batch_layout reports; u_all is updated in
 * place.  stats: host array of `count` entries, or NULL.  Calls on one batch
 * must not overlap. */
int32_t d4_batch_iter(d4_batch* batch, const float* x0_all, const float* goal_all, float* u_all,
                      uint32_t iter, d4_stats* stats, void* stream);

int32_t d4_batch_destroy(d4_batch* batch);

/* The work list of the persistent step for these problems, computed on the
 * host (no GPU call), as d4_batch_create builds it with lag = the launch's
 * workgroup count: items (host, [capacity][4]) receives (kind, instance, a, b)
 * per item in list order, kind 0 a reward tile of samples a .. a+S-1, kind 1
 * an update tile of rows a .. b-1; *n_items (host) the list length.
 * D4_EINVAL if the list needs more than `capacity` items (n_items still set).
 * Every reward tile of an instance precedes every update tile of it, which
 * is what bounds the persistent kernel's waits; the CPU tests check that. */
int32_t d4_batch_work_list(const d4_problem* probs, int32_t count, int32_t lag, int32_t capacity, int32_t* items,
                           int32_t* n_items);

/* ------------------------------------------------------------------------
 * Learned proposal: a permutation-equivariant set network that predicts the
 * initial plan tau.u from which Algorithm 2 starts (the paper initialises tau
 * without learning; the planner still judges and refines the prediction).
 * Per robot r of instance b:
 *   h_0 = x_r W_e + b_e
 *   h_{l+1} = h_l + relu(h_l W1_l + b1_l) W2_l + b2_l + mean_{r' in b}(h_l,r') Wp_l
 *   y_r = h_L W_h + b_h            (y_r: the robot's T*d_u controls)
 * Weights are FP32 master copies rounded to BF16 for every product; products
 * run on the BF16 MFMA with FP32 accumulation.  Loss: sum_r mask_r
 * |y_r - t_r|^2 / (2 d_out sum_r mask_r); optimiser Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8) with bias correction.  Flat parameter order: W_e [d_in][W],
 * b_e [W], then per layer W1 [W][H], b1 [H], W2 [H][W], b2 [W], Wp [W][W],
 * then W_h [W][d_out], b_h [d_out] (row-major).
 * ------------------------------------------------------------------------ */
typedef struct d4p_config {
    int32_t d_in;       /* per-robot features, 1..8 */
    int32_t width;      /* W */
    int32_t hidden;     /* H */
    int32_t layers;     /* L */
    int32_t d_out;      /* T * d_u */
    int32_t max_rows;   /* most robots in one call (sum over instances) */
    int32_t max_batch;  /* most instances in one call */
    uint64_t seed;      /* initialisation: uniform(+-1/sqrt(fan_in)) weights, zero biases */
} d4p_config;

typedef struct d4p_net d4p_net;

int32_t d4p_create(const d4p_config* cfg, d4p_net** net);
int32_t d4p_destroy(d4p_net* net);
int32_t d4p_num_params(const d4p_net* net, int64_t* count);       /* count: host */
/* params: device [count] FP32 in the flat order above; set also resets Adam.
 * These two calls are the network's save and load: the library writes no
 * files, so a caller stores the flat vector (with the d4p_config that shapes
 * it) in its own format and sets it back into a network of the same config. */
int32_t d4p_set_params(d4p_net* net, const float* params, void* stream);
int32_t d4p_get_params(const d4p_net* net, float* params, void* stream);

/* x [rows][d_in] features, seg [batch+1] device int32 row offsets of the
 * instances (seg[0] = 0, seg[batch] = rows, every instance non-empty);
 * writes y [rows][d_out]. */
int32_t d4p_forward(d4p_net* net, const float* x, const int32_t* seg, int32_t rows, int32_t batch, float* y,
                    void* stream);

/* Forward and backward: loss (device [1]) and grads (device [count], flat
 * order) unless NULL.  target [rows][d_out], mask [rows] (0 or 1). */
int32_t d4p_gradients(d4p_net* net, const float* x, const int32_t* seg, int32_t rows, int32_t batch,
                      const float* target, const float* mask, float* loss, float* grads, void* stream);

/* d4p_gradients followed by one Adam step with learning rate lr > 0. */
int32_t d4p_train_step(d4p_net* net, const float* x, const int32_t* seg, int32_t rows, int32_t batch,
                       const float* target, const float* mask, float lr, float* loss, void* stream);

/* The network's product kernel on its own: C[M][N] = op(A) op(B) + beta C,
 * A and B BF16 (bit patterns in uint16), C FP32 row-major; op(A) = A [M][K]
 * (lda >= K) or, with trans_a, A^T for A stored [K][M] (lda >= M); likewise
 * op(B) = B [K][N] or B^T for B stored [N][K]. */
int32_t d4p_gemm_bf16(int32_t trans_a, int32_t trans_b, const uint16_t* A, const uint16_t* B, float* C, int32_t M,
                      int32_t N, int32_t K, int32_t lda, int32_t ldb, int32_t ldc, float beta, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* D4_H */
