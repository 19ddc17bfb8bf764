// Kernels of the denoising hot path.
//
//  k_noise             - standard normal draws eps[e][m] (sampling step of Algorithm 1)
//  k_rollout           - RK4 rollout of given controls (Section III, Section IV-C)
//  k_rollfit<DYN,MODE> - reward of trajectories (Eq. generic-reward): the fused sample +
//                        rollout + reward of one denoising step (draws streamed per element,
//                        or generated in whole Philox blocks when aligned), or the reward of
//                        trajectories read from memory
//  k_softmax_update    - batch normalisation, softmax weights (p_0 of Section IV-B),
//                        S[e] = sum_m w_m eps[e][m] and the one-step update (Eq. mbd-denoising)
//  k_apply_final       - tau.u <- clip(tau.u + Delta U_0), rollout and stats (Algorithm 2)
//
// Lane mapping of k_rollfit: one lane per (sample m, robot k) with the sample
// index fastest, S samples per workgroup (blockDim = n*S).  A lane keeps its
// robot's state in registers and walks t = 0..T-1; positions of a block of Tb
// steps go to LDS as [Tb][n][S] float2/float4 slots, one per robot and step
// (a small footprint: two or three 256-lane workgroups share a CU at 16
// robots in space), and the pair checks of one step read consecutive slots
// across a wave.  Lane k checks partners (k + j) mod n
// for j = 1..floor((n-1)/2), plus j = n/2 for k < n/2 when n is even: every
// unordered pair exactly once, spread evenly.  Each lane also keeps the
// bounding box of its positions over the block; a partner is checked step by
// step only when the two boxes come within the threshold (exact in FP32, see
// box_gap2), which skips nearly all pairs of robots that stay apart, and the
// kept partners' steps are read from LDS NARROW_STEPS at a time.  The
// per-(m, t) "robot k hit anything" bits are OR-ed into an LDS word; masks are
// double buffered, so each time block costs two barriers.
#pragma once

#include "d4_device.hpp"

namespace d4 {

// ------------------------------------------------------------- reductions
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

struct RollFitArgs {
    const float* x0;      // [n][dx]
    const float* goal;    // [n][dp]
    const float* u_base;  // [D]
    const float* du_in;   // [D]
    const float* xs;      // [M][n][T+1][dx] (trajectory input mode)
    float* eps;           // [D][M] (fused mode)
    float* r;             // [M]
    int* hits;            // [M]
    int* robots_hit;      // [M] or null
    const uint32_t* iter_dev;  // iteration index in device memory, or null
    int n, T, M, S, Tb;
    float mean_scale, sigma;
    float thr2, w_safe, d0_floor;
    float ulo[3], uhi[3];
    StepConsts sc;
    uint32_t key0, key1, step, iter, inst;
    uint32_t flags;
    // static obstacles (appendix): centre and squared reward distance
    // (R_a + r_o + epsilon)^2 each, from device memory (obs) or, when obs is
    // null, from the kernel arguments themselves
    int n_obs;
    const float4* obs;
    float4 obs_inline[MAX_OBS];
};

// Stage a problem's obstacles in LDS (static, MAX_OBS slots); the caller
// synchronises the workgroup before the first use.  Workgroups can be
// smaller than the obstacle count (a tile of one sample of two robots has two
// lanes), so the lanes stride over the obstacles.
__device__ __forceinline__ void stage_obstacles(const RollFitArgs& a, float4* obs_l) {
    for (int o = threadIdx.x; o < a.n_obs; o += blockDim.x) obs_l[o] = a.obs ? a.obs[o] : a.obs_inline[o];
}

// Binary obstacle hit of a position: within the reward distance of any obstacle.
template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};
template <int V>
struct IntTag {
    static constexpr int value = V;
};

template <int DP>
__device__ __forceinline__ int obstacle_hit(const float* x, const float4* obs_l, int n_obs) {
    int hit = 0;
    for (int o = 0; o < n_obs; ++o) {
        const float4 c = obs_l[o];
        const float cc[3] = {c.x, c.y, c.z};
        hit |= pair_d2<DP>(x, cc) <= c.w ? 1 : 0;
    }
    return hit;
}

// Position slot of one robot in LDS: float2 in the plane, float4 (w unused) in space.
template <int DP>
struct PosSlot;
template <>
struct PosSlot<2> {
    using T = float2;
    __device__ __forceinline__ static T pack(const float* x) { return make_float2(x[0], x[1]); }
    __device__ __forceinline__ static void unpack(const T& v, float* p) {
        p[0] = v.x;
        p[1] = v.y;
    }
};
template <>
struct PosSlot<3> {
    using T = float4;
    __device__ __forceinline__ static T pack(const float* x) { return make_float4(x[0], x[1], x[2], 0.0f); }
    __device__ __forceinline__ static void unpack(const T& v, float* p) {
        p[0] = v.x;
        p[1] = v.y;
        p[2] = v.z;
    }
};

// MODE_FUSED_ALIGNED: every robot's first draw element is a multiple of 4
// (T * d_u % 4 == 0), so the draw window needs no phase selection.
enum { MODE_FUSED = 1, MODE_FROM_X = 2, MODE_FUSED_ALIGNED = 3 };

// Collision bits of robot k at one step: bit l set when partner l = k + j
// (mod n), j = 1..jmax, is within the reward threshold.  pb points at slot 0
// of this sample's step; the step holds 2n - 1 slots (robots 0..n-1, then
// 0..n-2 again, S apart: the cooperative kernel's layout), so the partners
// are contiguous.  Hits are collected
// at unwrapped positions k + j < 2n and folded back modulo n.
template <int DP>
__device__ __forceinline__ uint32_t pair_bits(const typename PosSlot<DP>::T* pb, int n, int S, int k, int jmax,
                                              float thr2) {
    using PS = PosSlot<DP>;
    float pk[DP];
    PS::unpack(pb[k * S], pk);
    const typename PS::T* q = pb + (k + 1) * S;
    const uint32_t low = n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
    if (n <= 16) {
        uint32_t bits = 0u, bit = 2u << k;
#pragma unroll 4
        for (int j = 0; j < jmax; ++j) {
            float pl[DP];
            PS::unpack(*q, pl);
            bits |= (pair_d2<DP>(pk, pl) <= thr2) ? bit : 0u;
            q += S;
            bit <<= 1;
        }
        return (bits | (bits >> n)) & low;
    }
    uint64_t bits = 0ull, bit = 2ull << k;
#pragma unroll 4
    for (int j = 0; j < jmax; ++j) {
        float pl[DP];
        PS::unpack(*q, pl);
        bits |= (pair_d2<DP>(pk, pl) <= thr2) ? bit : 0ull;
        q += S;
        bit <<= 1;
    }
    return (uint32_t)((bits | (bits >> n)) & low);
}

// Steps of a time block whose narrow-phase checks are read from LDS together
// (the batched kernel, which holds every model's code, takes one at a time:
// the unrolled form grows each copy and slowed a mixed batch by 14 %).
constexpr int NARROW_STEPS = 4;

// Steps per noise chunk (a whole number of Philox blocks) and blocks per chunk.
template <int DU>
struct Chunk {
    static constexpr int STEPS = (DU == 2) ? 2 : 4;
    static constexpr int GROUPS = STEPS * DU / 4;
};

// Reward of one (sample, robot) lane per step block; see the mapping notes above.
// MODE_FUSED draws, samples and rolls out; it requires Tb to be a multiple of
// Chunk::STEPS.  MODE_FROM_X reads trajectories instead.
// One tile: samples m0 .. m0+S-1 of one problem, lanes tid < n*S (the rest of
// the workgroup idles through the barriers).
template <int DYN, int MODE, int NS = NARROW_STEPS, bool PRIO = true>
__device__ __forceinline__ void rollfit_tile(const RollFitArgs& a, int m0, float* lds) {
    using DY = Dyn<DYN>;
    constexpr int DX = DY::DX, DU = DY::DU, DP = DY::DP;
    using PS = PosSlot<DP>;
    using PT = typename PS::T;
    constexpr bool FROM_X = MODE == MODE_FROM_X;
    const int n = a.n, T = a.T, M = a.M, S = a.S, Tb = a.Tb;
    const int tid = threadIdx.x;
    const int k_raw = tid / S;
    const bool active = k_raw < n;
    const int k = active ? k_raw : n - 1;
    const int ms = tid - k_raw * S;
    const int m = m0 + ms;
    const bool live = active && m < M;
    const int mc = m < M ? m : M - 1;
    PT* pos = reinterpret_cast<PT*>(lds);                                        // [Tb][n][S]
    PT* box = pos + Tb * n * S;                                                  // [n][S][lo, hi]
    uint32_t* mask = reinterpret_cast<uint32_t*>(box + 2 * n * S);              // [2][Tb][S]
    uint32_t* anyhit = mask + 2 * Tb * S;                                        // [2][S]
    int* hitc = reinterpret_cast<int*>(anyhit + 2 * S);                          // [S] pair hits per sample
    const int wave = tid >> 6, lane = tid & 63;
    uint16_t* items = reinterpret_cast<uint16_t*>(hitc + S) + wave * (64 * (n >> 1));  // [waves][64 (n/2)]

    float x[DX], aux[DY::AUX], g[DP];
    if (FROM_X) {
        const float* xr = a.xs + ((size_t)mc * n + k) * (size_t)(T + 1) * DX;
#pragma unroll
        for (int c = 0; c < DX; ++c) x[c] = xr[c];
    } else {
#pragma unroll
        for (int c = 0; c < DX; ++c) x[c] = a.x0[k * DX + c];
        DY::init(x, aux);
    }
#pragma unroll
    for (int c = 0; c < DP; ++c) g[c] = a.goal[k * DP + c];
    const float inv_d0 = inv_start_dist(goal_d2<DP>(x, g), a.d0_floor);

    float goal_acc = 0.0f;
    int safe_cnt = 0, obs_cnt = 0;
    __shared__ float4 obs_l[MAX_OBS];
    // the obstacle count is uniform over the grid, so the barrier is too
    if (a.n_obs > 0) {
        stage_obstacles(a, obs_l);
        __syncthreads();
    }
    const int n_obs = a.n_obs;
    // pair-hit counters; the first block's barrier orders this before any update
    if (k_raw == 0) hitc[ms] = 0;

    const uint32_t iter = a.iter_dev ? *a.iter_dev : a.iter;
    const uint32_t c2 = (iter << 16) | a.step;
    // this robot's first draw element and its phase within a Philox block
    const uint32_t ebase = (uint32_t)(k * T * DU);
    const uint32_t phase = MODE == MODE_FUSED_ALIGNED ? 0u : (ebase & 3u);
    float left[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (!FROM_X) normal_block(ebase >> 2, (uint32_t)mc, c2, a.inst, a.key0, a.key1, left[0], left[1], left[2], left[3]);
    float ulo[DU], uhi[DU];
#pragma unroll
    for (int d = 0; d < DU; ++d) {
        ulo[d] = a.ulo[d];
        uhi[d] = a.uhi[d];
    }
    // the draw, sampling and dynamics loop reads its uniform operands from
    // VGPR copies (an SGPR operand keeps a VALU instruction from pairing)
    const float sigma = vgpr_copy(a.sigma), mscale = vgpr_copy(a.mean_scale);
#pragma unroll
    for (int d = 0; d < DU; ++d) {
        ulo[d] = vgpr_copy(ulo[d]);
        uhi[d] = vgpr_copy(uhi[d]);
    }
    StepConsts sc = a.sc;
    sc.dt = vgpr_copy(sc.dt);
    sc.hdt = vgpr_copy(sc.hdt);
    sc.hdt2 = vgpr_copy(sc.hdt2);
    sc.dt6 = vgpr_copy(sc.dt6);
    sc.vmax = vgpr_copy(sc.vmax);
    const PhiloxKey pk = PhiloxKey::make<true>(a.key0, a.key1);
    const int jmax = active ? ((n - 1) >> 1) + ((((n & 1) == 0) && (k < (n >> 1))) ? 1 : 0) : 0;
    const bool pairs_mode = (a.flags & FLAG_SAFE_PAIRS) != 0;
    const size_t Ms = (size_t)M;
    // eps stores go through a buffer resource with 32-bit offsets when the
    // whole [D][M] array (plus one chunk of rows) spans under 2 GiB
    const size_t Dt = (size_t)n * T * DU;
    const bool eps32 = (Dt + 64) * Ms * 4 <= 0x7FFFFFFFull;
    const int eps_voff = eps32 ? (int)(((size_t)k * T * DU * Ms + (size_t)m) * 4) : 0;

    // bounding box of this lane's positions over the current block
    float blo[DP], bhi[DP];
    const MinMaxInf mm;

    // goal term, LDS position and bounding box of the state after step tt of the block
    auto after_step = [&](int tt) {
        goal_acc += goal_term(fast_sqrt(goal_d2<DP>(x, g)), inv_d0);
        if (n_obs) obs_cnt += obstacle_hit<DP>(x, obs_l, n_obs);
#pragma unroll
        for (int c = 0; c < DP; ++c) {
            blo[c] = mm.min(blo[c], x[c]);
            bhi[c] = mm.max(bhi[c], x[c]);
        }
        if (active) {
            const PT v = PS::pack(x);
            pos[(tt * n + k) * S + ms] = v;
        }
    };

    // control bases (u_base, du_in) of the next draw chunk, loaded one chunk
    // ahead so that their latency hides behind the current chunk's draws.
    // Buffer loads are range-checked against the D-element arrays (reads past
    // the end return 0), so a chunk's loads need no guard: elements past the
    // robot's last step belong to the next robot or are zero, and go unused.
    constexpr int CS = Chunk<DU>::STEPS, CG = Chunk<DU>::GROUPS, NE = 4 * CG;
    float ub_nx[NE], du_nx[NE];
    const __amdgpu_buffer_rsrc_t ub_rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.u_base), (short)0, (int)(Dt * 4), 0x00020000);
    const __amdgpu_buffer_rsrc_t du_rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.du_in), (short)0, (int)(Dt * 4), 0x00020000);
    auto load_ctrl = [&](int t) {
        const int vo = (int)((ebase + (uint32_t)(t * DU)) * 4u);
#pragma unroll
        for (int j = 0; j < NE; ++j) {
            ub_nx[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ub_rs, vo + 4 * j, 0, 0));
            du_nx[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(du_rs, vo + 4 * j, 0, 0));
        }
    };
    if (!FROM_X) load_ctrl(0);

    const int nblk = (T + Tb - 1) / Tb;
    for (int b = 0; b < nblk; ++b) {
        // The draw-and-rollout loop runs at raised wave priority, the pair
        // phases at the default: when the two waves sharing a SIMD are in
        // different phases, the VALU-dense one issues first (c3 iterations
        // 3 % faster than with equal priorities; the results do not change).
        // The batched kernel, whose neighbouring tiles belong to different
        // instances, runs 1 % faster without it (PRIO = false).
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
        const int buf = b & 1;
        const int t0 = b * Tb;
        const int tcount = min(Tb, T - t0);
#pragma unroll
        for (int c = 0; c < DP; ++c) {
            blo[c] = INFINITY;
            bhi[c] = -INFINITY;
        }
        if (!FROM_X) {
            // Chunks of CS steps use CS*DU = 4*CG consecutive draws starting at
            // phase p of a Philox block; the window holds the block the
            // previous chunk ended in ("left") plus CG new blocks.
            for (int tc = 0; tc < tcount; tc += CS) {
                const int t = t0 + tc;
                const uint32_t e0 = ebase + (uint32_t)(t * DU);
                const uint32_t g0 = e0 >> 2;
                // sample means of this chunk, then the next chunk's loads
                float mean_c[NE];
#pragma unroll
                for (int j = 0; j < NE; ++j) mean_c[j] = sample_mean(ub_nx[j], du_nx[j], mscale);
                load_ctrl(t + CS);
                float win[4 + 4 * CG];
#pragma unroll
                for (int j = 0; j < 4; ++j) win[j] = left[j];
                normal_blocks<CG, true>(g0 + 1, (uint32_t)mc, c2, a.inst, pk, win + 4);
                float z[4 * CG];
#pragma unroll
                for (int j = 0; j < 4 * CG; ++j)
                    z[j] = phase == 0 ? win[j] : phase == 1 ? win[j + 1] : phase == 2 ? win[j + 2] : win[j + 3];
#pragma unroll
                for (int j = 0; j < 4; ++j) left[j] = win[4 * CG + j];
                const int steps = min(CS, T - t);
                if (live) {
                    if (eps32) {
                        // rows e0 .. e0+4CG-1 of eps: a uniform base for this chunk's
                        // steps, the lane's fixed offset and a uniform row offset
                        const uint32_t rows_left = (uint32_t)(Dt - (size_t)t * DU);
                        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                            a.eps + (size_t)t * DU * Ms, (short)0, (int)(rows_left * (uint32_t)M * 4u), 0x00020000);
#pragma unroll
                        for (int j = 0; j < 4 * CG; ++j)
                            if (j < steps * DU)
                                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(z[j]), rs, eps_voff, j * M * 4, 0);
                    } else {
                        float* ep = a.eps + (size_t)e0 * Ms + m;
#pragma unroll
                        for (int j = 0; j < 4 * CG; ++j)
                            if (j < steps * DU) ep[(size_t)j * Ms] = z[j];
                    }
                }
#pragma unroll
                for (int s = 0; s < CS; ++s) {
                    if (s < steps) {
                        float u[DU];
#pragma unroll
                        for (int d = 0; d < DU; ++d) {
                            u[d] = sample_from_mean(mean_c[s * DU + d], sigma, z[s * DU + d], ulo[d], uhi[d]);
                        }
                        DY::step(x, aux, u, sc);
                        after_step(tc + s);
                    }
                }
            }
        } else {
            for (int tt = 0; tt < tcount; ++tt) {
                const int t = t0 + tt;
                const float* xr = a.xs + (((size_t)mc * n + k) * (size_t)(T + 1) + (t + 1)) * DX;
#pragma unroll
                for (int c = 0; c < DP; ++c) x[c] = xr[c];
                after_step(tt);
            }
        }
        if (active) {
            box[(k * S + ms) * 2] = PS::pack(blo);
            box[(k * S + ms) * 2 + 1] = PS::pack(bhi);
        }
        if (k_raw == 0) {
            for (int tt = 0; tt < tcount; ++tt) mask[(buf * Tb + tt) * S + ms] = 0u;
            anyhit[buf * S + ms] = 0u;
        }
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        // broad phase: partners whose block boxes come within the threshold
        uint32_t near = 0u;
        {
            int l = k + 1 < n ? k + 1 : 0;
            for (int j = 0; j < jmax; ++j) {
                float llo[DP], lhi[DP];
                PS::unpack(box[(l * S + ms) * 2], llo);
                PS::unpack(box[(l * S + ms) * 2 + 1], lhi);
                near |= (box_gap2<DP>(blo, bhi, llo, lhi) <= a.thr2) ? (1u << j) : 0u;
                l = l + 1 < n ? l + 1 : 0;
            }
        }
        // narrow phase: exact checks of the kept partners at every step of the
        // block.  The wave lists its kept (robot, sample, partner) triples in
        // LDS, ordered by partner and lane (ballot and lane count per partner
        // index), and its lanes then take them in turn, so that the checks
        // are spread over the wave instead of waiting on the lane with the
        // most kept partners.  Each triple reads NS steps' positions from
        // LDS together before its compares.  Hits are OR-ed into the step's
        // collision mask for both robots and counted per sample; the order of
        // these integer updates does not change their result.
        if (__ballot(near != 0u)) {
            const int jw = n >> 1;
            int total = 0;
            for (int j = 0; j < jw; ++j) {
                const bool has = (near >> j) & 1u;
                const uint64_t bal = __ballot(has);
                if (bal) {
                    if (has) {
                        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                        items[total + (int)below] = (uint16_t)((k << 10) | (ms << 4) | j);
                    }
                    total += __popcll(bal);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // the last wave of a workgroup can hold fewer than 64 lanes
            const int wlanes = min(64, (int)blockDim.x - wave * 64);
            for (int i = lane; i < total; i += wlanes) {
                const uint32_t code = items[i];
                const int ki = (int)(code >> 10), mi = (int)((code >> 4) & 63u);
                int l = ki + 1 + (int)(code & 15u);
                l = l >= n ? l - n : l;
                const uint32_t pair = (1u << ki) | (1u << l);
                int cnt = 0;
                for (int tt0 = 0; tt0 < tcount; tt0 += NS) {
                    float pa[NS][DP], pb[NS][DP];
#pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        const int tt = tt0 + q < tcount ? tt0 + q : tcount - 1;
                        PS::unpack(pos[(tt * n + ki) * S + mi], pa[q]);
                        PS::unpack(pos[(tt * n + l) * S + mi], pb[q]);
                    }
#pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        if (tt0 + q < tcount && pair_d2<DP>(pa[q], pb[q]) <= a.thr2) {
                            atomicOr(&mask[(buf * Tb + tt0 + q) * S + mi], pair);
                            ++cnt;
                        }
                    }
                }
                if (cnt) {
                    atomicAdd(&hitc[mi], cnt);
                    atomicOr(&anyhit[buf * S + mi], 1u);
                }
            }
        }
        __syncthreads();
        if (active && anyhit[buf * S + ms])
            for (int tt = 0; tt < tcount; ++tt) safe_cnt += (mask[(buf * Tb + tt) * S + ms] >> k) & 1u;
    }

    __syncthreads();
    float* rg = lds;
    int* rs = reinterpret_cast<int*>(lds + n * S);
    int* ro = rs + n * S;
    if (active) {
        rg[k * S + ms] = goal_acc;
        rs[k * S + ms] = safe_cnt;
        ro[k * S + ms] = obs_cnt;
    }
    __syncthreads();
    if (k_raw == 0 && live) {
        float gs = 0.0f;
        int ss = 0, os = 0;
        const int hs = hitc[ms];
        for (int kk = 0; kk < n; ++kk) {
            gs += rg[kk * S + ms];
            ss += rs[kk * S + ms];
            os += ro[kk * S + ms];
        }
        const float pen = (float)((pairs_mode ? 2 * hs : ss) + os);
        const float rv = team_reward(gs, a.w_safe, pen, n * T);
        a.r[m] = rv;
        a.hits[m] = hs;
        if (a.robots_hit) a.robots_hit[m] = ss;
    }
}

template <int DYN, int MODE>
__global__ void __launch_bounds__(256) k_rollfit(const RollFitArgs a) {
    extern __shared__ float lds[];
    rollfit_tile<DYN, MODE>(a, blockIdx.x * a.S, lds);
}

// Cooperative variant of the fused kernel for problems with few (sample,
// robot) lanes: R >= 2 replica lanes per (sample, robot).  Per time block of
// Tb steps: (1) the draws of the robot's block, whole Philox blocks, go to
// eps and, as the block's sampled controls, to LDS; (2) replica 0 rolls the
// robot out over the block, reading its controls from LDS; (3) the pair
// checks, one step per replica in turn; (4) the collision masks are read.
// Only the rollout is serial, so when replica 0 fills whole waves the stages
// are pipelined over the blocks: the rollout of block i overlaps the draws of
// block i+1 and the pair checks of block i-1; otherwise the blocks' stages run
// one after another.  Every value is computed as in the one-lane kernel and
// every sum is taken in the same order, so the results are identical to it.
// Lanes: tid = rep * (n*S) + k * S + ms.  LDS: controls [2][n][G][4][S]
// floats with G = Tb*d_u/4 + 3, positions [2][Tb][2n-1][S] slots, masks
// [3][Tb][S].
template <int DYN, int MODE>
__device__ __forceinline__ void rollfit_coop_tile(const RollFitArgs& a, int R, int m0, float* lds) {
    using DY = Dyn<DYN>;
    constexpr int DX = DY::DX, DU = DY::DU, DP = DY::DP;
    using PS = PosSlot<DP>;
    using PT = typename PS::T;
    const int n = a.n, T = a.T, M = a.M, S = a.S, Tb = a.Tb;
    // Philox blocks per robot and time block, plus two of padding that the
    // rollout's read-ahead may touch (and never uses)
    const int G = Tb * DU / 4 + 3;
    const int tid = threadIdx.x;
    const int group = n * S;
    const int rep = tid / group;
    const int local = tid - rep * group;
    const bool active = rep < R;
    const int k = local / S;
    const int ms = local - k * S;
    const int m = m0 + ms;
    const bool live = active && m < M;
    const int mc = m < M ? m : M - 1;
    const int n2 = 2 * n - 1;
    const size_t NZB = (size_t)n * G * 4 * S, PB = (size_t)Tb * n2 * S;
    float* nz = lds;                                                     // [2][n][G][4][S]
    PT* pos = reinterpret_cast<PT*>(nz + 2 * NZB);                      // [2][Tb][2n-1][S]
    uint32_t* mask = reinterpret_cast<uint32_t*>(pos + 2 * PB);         // [3][Tb][S]

    float x[DX], aux[DY::AUX], g[DP];
#pragma unroll
    for (int c = 0; c < DX; ++c) x[c] = a.x0[k * DX + c];
    DY::init(x, aux);
#pragma unroll
    for (int c = 0; c < DP; ++c) g[c] = a.goal[k * DP + c];
    const float inv_d0 = inv_start_dist(goal_d2<DP>(x, g), a.d0_floor);
    float goal_acc = 0.0f;
    int safe_cnt = 0, hit_cnt = 0, obs_cnt = 0;
    __shared__ float4 obs_l[MAX_OBS];
    // the obstacle count is uniform over the grid, so the barrier is too
    if (a.n_obs > 0) {
        stage_obstacles(a, obs_l);
        __syncthreads();
    }
    const int n_obs = a.n_obs;
    const uint32_t iter = a.iter_dev ? *a.iter_dev : a.iter;
    const uint32_t c2 = (iter << 16) | a.step;
    const uint32_t ebase = (uint32_t)(k * T * DU);
    // the draw phase, on every replica, reads its uniform operands from VGPR
    // copies (an SGPR operand halves a VALU instruction's issue rate)
    float ulo[DU], uhi[DU];
#pragma unroll
    for (int d = 0; d < DU; ++d) {
        ulo[d] = vgpr_copy(a.ulo[d]);
        uhi[d] = vgpr_copy(a.uhi[d]);
    }
    const float sigma = vgpr_copy(a.sigma), mscale = vgpr_copy(a.mean_scale);
    // the key schedule stays in SGPRs: the draws here are bound by latency,
    // not by the half issue rate of an SGPR operand, and the kernel's 1024
    // lanes leave each 128 VGPRs
    const PhiloxKey pk = PhiloxKey::make<false>(a.key0, a.key1);
    const int jmax = active ? ((n - 1) >> 1) + ((((n & 1) == 0) && (k < (n >> 1))) ? 1 : 0) : 0;
    const bool pairs_mode = (a.flags & FLAG_SAFE_PAIRS) != 0;
    const size_t Ms = (size_t)M;
    const size_t nzk_off = (size_t)k * G * 4 * S + ms;

    const int nblk = (T + Tb - 1) / Tb;
    // (1) draws of time block bb into control buffer nzb, Philox blocks
    // r0, r0 + rstride, ... of the robot's block range: the block's sampled
    // controls go to LDS, its normals to eps.  The control bases of a Philox
    // block are loaded one block ahead (the first block's by draw_bases,
    // which the caller issues early), so their latency is covered.
    struct DrawBlock {
        uint32_t e_lo, e_hi, g_a;
        int G_b;
    };
    auto draw_span = [&](int bb) {
        DrawBlock db;
        const int t0 = bb * Tb;
        const int tcount = min(Tb, T - t0);
        db.e_lo = ebase + (uint32_t)(t0 * DU);
        db.e_hi = db.e_lo + (uint32_t)(tcount * DU);
        db.g_a = db.e_lo >> 2;
        db.G_b = (int)(((db.e_hi - 1) >> 2) - db.g_a) + 1;
        return db;
    };
    // control bases of Philox block gi (indices clamped into the time block;
    // the clamped values are not used)
    auto draw_bases = [&](const DrawBlock& db, int gi, float (&ubj)[4], float (&duj)[4]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t e = 4 * (db.g_a + (uint32_t)gi) + (uint32_t)j;
            const uint32_t ec = e < db.e_lo ? db.e_lo : e >= db.e_hi ? db.e_hi - 1 : e;
            ubj[j] = a.u_base[ec];
            duj[j] = a.du_in[ec];
        }
    };
    auto draw_block = [&](const DrawBlock& db, int nzb, int r0, int rstride, float (&ubj)[4], float (&duj)[4]) {
        float* nzk = nz + nzb * NZB + nzk_off;
        for (int gi = r0; gi < db.G_b; gi += rstride) {
            float ubn[4], dun[4];
            if (gi + rstride < db.G_b) draw_bases(db, gi + rstride, ubn, dun);
            float z[4];
            normal_blocks<1, true>(db.g_a + (uint32_t)gi, (uint32_t)mc, c2, a.inst, pk, z);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t e = 4 * (db.g_a + (uint32_t)gi) + (uint32_t)j;
                const bool in_blk = e >= db.e_lo && e < db.e_hi;
                float v = z[j];
                if (in_blk) {
                    const int d = (int)((e - ebase) % (uint32_t)DU);
                    // the bounds are chosen by selects of values (an indexed
                    // choice would put the two small arrays in scratch memory)
                    float lo = ulo[0], hi = uhi[0];
                    if constexpr (DU > 1) {
                        lo = d == 1 ? ulo[1] : lo;
                        hi = d == 1 ? uhi[1] : hi;
                    }
                    if constexpr (DU > 2) {
                        lo = d == 2 ? ulo[2] : lo;
                        hi = d == 2 ? uhi[2] : hi;
                    }
                    v = sample_control(ubj[j], duj[j], mscale, sigma, z[j], lo, hi);
                }
                nzk[(size_t)(gi * 4 + j) * S] = v;
                if (live && in_blk) a.eps[(size_t)e * Ms + m] = z[j];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                ubj[j] = ubn[j];
                duj[j] = dun[j];
            }
        }
    };
    // (2) rollout of time block bb from control buffer nzb into position
    // buffer pb.  Step tt's control d sits at nzk[(o + tt d_u + d) S] with
    // o = e_lo mod 4 (the block's draws start at Philox block e_lo / 4).  The
    // controls are read two steps ahead of their use (the two padding blocks
    // hold the reads past the block's end), before the position stores that
    // the compiler may not move them past, so no LDS round trip sits in the
    // state chain.  The loop body has no branch (robot n-1's second position
    // store repeats its first), so the unrolled steps are one block of
    // straight-line code that the scheduler can interleave.  The goal and
    // obstacle terms, which need the positions only, are left to another
    // replica.
    auto roll_block = [&](int bb, int nzb, int pb, auto score_tag) {
        // SCORE 0: positions only; 1: goal terms inline; 2: goal and obstacle terms inline
        constexpr int SCORE = decltype(score_tag)::value;
        const int t0 = bb * Tb;
        const int tcount = min(Tb, T - t0);
        const uint32_t e_lo = ebase + (uint32_t)(t0 * DU);
        const float* ub = nz + nzb * NZB + nzk_off + (size_t)(e_lo & 3u) * S;
        PT* slot = pos + pb * PB + k * S + ms;   // step tt at slot + tt (2n-1) S
        const int dup = k < n - 1 ? n * S : 0;
        float u1[DU], u2[DU];
#pragma unroll
        for (int d = 0; d < DU; ++d) {
            u1[d] = ub[(size_t)d * S];
            u2[d] = ub[(size_t)(DU + d) * S];
        }
        ub += (size_t)2 * DU * S;
        // four steps per unrolled body (two for the six-state 3D model, which
        // would otherwise exceed the 128 VGPRs of a 1024-lane workgroup)
        constexpr int RU = DX > 4 ? 2 : 4;
#pragma unroll RU
        for (int tt = 0; tt < tcount; ++tt) {
            float u[DU];
#pragma unroll
            for (int d = 0; d < DU; ++d) {
                u[d] = u1[d];
                u1[d] = u2[d];
                u2[d] = ub[(size_t)d * S];
            }
            ub += (size_t)DU * S;
            DY::step(x, aux, u, a.sc);
            if constexpr (SCORE >= 1) goal_acc += goal_term(fast_sqrt(goal_d2<DP>(x, g)), inv_d0);
            if constexpr (SCORE == 2) obs_cnt += obstacle_hit<DP>(x, obs_l, n_obs);
            const PT v = PS::pack(x);
            slot[0] = v;
            slot[dup] = v;
            slot += n2 * S;
        }
    };
    // goal and obstacle terms of time block bb from position buffer pb, in
    // step order (the goal sum is taken in the one-lane kernel's order); the
    // positions of four steps are read together
    auto score_block = [&](int bb, int pb, auto obs_tag) {
        constexpr bool OBS = decltype(obs_tag)::value;
        const int tcount = min(Tb, T - bb * Tb);
        const PT* slot = pos + pb * PB + k * S + ms;
        const int st = n2 * S;
        for (int tt0 = 0; tt0 < tcount; tt0 += 4) {
            float xp[4][DP];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int tt = tt0 + q < tcount ? tt0 + q : tcount - 1;
                PS::unpack(slot[tt * st], xp[q]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (tt0 + q < tcount) {
                    goal_acc += goal_term(fast_sqrt(goal_d2<DP>(xp[q], g)), inv_d0);
                    if constexpr (OBS) obs_cnt += obstacle_hit<DP>(xp[q], obs_l, n_obs);
                }
            }
        }
    };
    // (3) pair checks of time block bb on position buffer pb, steps r0,
    // r0 + rstride, ...: hits OR-ed into the step's collision mask in mask
    // buffer mb for both robots
    auto pair_block = [&](int bb, int pb, int mb, int r0, int rstride) {
        const int tcount = min(Tb, T - bb * Tb);
        for (int tt = r0; tt < tcount; tt += rstride) {
            const uint32_t bits = pair_bits<DP>(pos + pb * PB + tt * n2 * S + ms, n, S, k, jmax, a.thr2);
            hit_cnt += __popc(bits);
            if (bits) atomicOr(&mask[(mb * Tb + tt) * S + ms], bits | (1u << k));
        }
    };
    // (4) collision flags of robot k in time block bb
    auto mask_read = [&](int bb, int mb) {
        const int tcount = min(Tb, T - bb * Tb);
        for (int tt = 0; tt < tcount; ++tt) safe_cnt += (mask[(mb * Tb + tt) * S + ms] >> k) & 1u;
    };

    if ((group & 63) != 0) {
        // Sequential schedule, for workgroups whose replica 0 does not fill
        // whole waves (the roles would share waves, and a pipeline would only
        // add stages): per block, the draws on every replica, the rollout
        // with its goal and obstacle terms on replica 0, the pair checks on
        // every replica, the masks read by replica 1 (mask buffers alternate
        // so that clearing the next one does not race with that read).
        for (int b = 0; b < nblk; ++b) {
            if (active) {
                const DrawBlock db = draw_span(b);
                float ubj[4], duj[4];
                if (rep < db.G_b) draw_bases(db, rep, ubj, duj);
                draw_block(db, 0, rep, R, ubj, duj);
            }
            if (rep == 0 && k == 0 && active)
                for (int tt = 0; tt < Tb; ++tt) mask[((b & 1) * Tb + tt) * S + ms] = 0u;
            __syncthreads();
            if (rep == 0 && active) {
                if (n_obs) roll_block(b, 0, 0, IntTag<2>{});
                else roll_block(b, 0, 0, IntTag<1>{});
            }
            __syncthreads();
            if (active) pair_block(b, 0, b & 1, rep, R);
            __syncthreads();
            if (rep == 1 && active) mask_read(b, b & 1);
        }
    } else {
        // Software pipeline over the time blocks, one barrier per stage.  In
        // stage i replica 0 rolls block i out, at raised wave priority; the
        // workers (replicas 2..R-1, or replica 1 when R = 2) check the pairs
        // of block i-1 and draw block i+1; replica 1 scores block i-1, reads
        // the collision masks of block i-2 and clears the mask buffer read in
        // the stage before.  Controls and positions are double-buffered,
        // masks triple-buffered.
        if (active) {
            const DrawBlock db = draw_span(0);
            float ubj[4], duj[4];
            if (rep < db.G_b) draw_bases(db, rep, ubj, duj);
            draw_block(db, 0, rep, R, ubj, duj);
        }
        if (rep == 0 && k == 0 && active)
            for (int q = 0; q < 3 * Tb; ++q) mask[q * S + ms] = 0u;
        __syncthreads();
        const int w0 = R > 2 ? 2 : 1, workers = R - w0;
        for (int i = 0; i <= nblk + 1; ++i) {
            if (active) {
                if (rep == 0) {
                    if (i < nblk) {
                        __builtin_amdgcn_s_setprio(2);
                        roll_block(i, i & 1, i & 1, IntTag<0>{});
                        __builtin_amdgcn_s_setprio(0);
                    }
                } else {
                    if (rep >= w0) {
                        // the draws' first control bases are requested before
                        // the pair checks, which then cover their latency
                        const bool draw = i + 1 < nblk;
                        const DrawBlock db = draw_span(draw ? i + 1 : 0);
                        float ubj[4], duj[4];
                        if (draw && rep - w0 < db.G_b) draw_bases(db, rep - w0, ubj, duj);
                        if (i >= 1 && i <= nblk) pair_block(i - 1, (i - 1) & 1, (i - 1) % 3, rep - w0, workers);
                        if (draw) draw_block(db, (i + 1) & 1, rep - w0, workers, ubj, duj);
                    }
                    if (rep == 1) {
                        // the scorer's serial goal sum at a priority between the
                        // rollout's and the workers' (c2 1 % faster)
                        __builtin_amdgcn_s_setprio(1);
                        if (i >= 1 && i <= nblk) {
                            if (n_obs) score_block(i - 1, (i - 1) & 1, BoolTag<true>{});
                            else score_block(i - 1, (i - 1) & 1, BoolTag<false>{});
                        }
                        if (i >= 2) mask_read(i - 2, (i - 2) % 3);
                        if (i >= 3 && k == 0)
                            for (int tt = 0; tt < Tb; ++tt) mask[((i % 3) * Tb + tt) * S + ms] = 0u;
                        __builtin_amdgcn_s_setprio(0);
                    }
                }
            }
            __syncthreads();
        }
    }
    // The roles change only which lane evaluates a value, never its
    // operations or their order, so the results are those of the one-lane
    // kernel under either schedule.

    __syncthreads();
    float* rg = lds;
    int* rs = reinterpret_cast<int*>(lds + group);
    int* rh = rs + group;                  // [R][n][S]
    int* ro = rh + R * group;              // [n][S]
    if (active) {
        rh[rep * group + k * S + ms] = hit_cnt;
        // the goal and obstacle sums are replica 0's under the sequential
        // schedule and replica 1's under the pipeline; the masks are read by
        // replica 1 under both
        if (rep == ((group & 63) != 0 ? 0 : 1)) {
            rg[k * S + ms] = goal_acc;
            ro[k * S + ms] = obs_cnt;
        }
        if (rep == 1) rs[k * S + ms] = safe_cnt;
    }
    __syncthreads();
    if (rep == 0 && k == 0 && live) {
        float gs = 0.0f;
        int ss = 0, hs = 0, os = 0;
        for (int kk = 0; kk < n; ++kk) {
            gs += rg[kk * S + ms];
            ss += rs[kk * S + ms];
            os += ro[kk * S + ms];
            for (int rr = 0; rr < R; ++rr) hs += rh[rr * group + kk * S + ms];
        }
        const float pen = (float)((pairs_mode ? 2 * hs : ss) + os);
        const float rv = team_reward(gs, a.w_safe, pen, n * T);
        a.r[m] = rv;
        a.hits[m] = hs;
        if (a.robots_hit) a.robots_hit[m] = ss;
    }
}

template <int DYN>
__global__ void __launch_bounds__(1024) k_rollfit_coop(const RollFitArgs a, int R) {
    extern __shared__ float lds[];
    rollfit_coop_tile<DYN, MODE_FUSED>(a, R, blockIdx.x * a.S, lds);
}

// eps[e][m] for e < D, m < M; one lane per (Philox block, sample).
static __global__ void __launch_bounds__(256) k_box_muller(const uint32_t* words, int64_t count, float* z) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        float a, b;
        box_muller(words[2 * i], words[2 * i + 1], a, b);
        z[2 * i] = a;
        z[2 * i + 1] = b;
    }
}

static __global__ void __launch_bounds__(256) k_noise(float* eps, int D, int M, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (m >= M) return;
    float z[4];
    normal_block((uint32_t)g, (uint32_t)m, c2, c3, k0, k1, z[0], z[1], z[2], z[3]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = 4 * g + j;
        if (e < D) eps[(size_t)e * M + m] = z[j];
    }
}

// x[m][k][t+1] = RK4 step of x[m][k][t] under clip(u[m][k][t]).
template <int DYN>
__global__ void __launch_bounds__(256) k_rollout(const float* x0, const float* u, float* xs, int n,
                                                 int T, int M, StepConsts sc, float ulo0, float ulo1,
                                                 float ulo2, float uhi0, float uhi1, float uhi2) {
    using DY = Dyn<DYN>;
    constexpr int DX = DY::DX, DU = DY::DU;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * n) return;
    const int k = idx % n;
    const float lo[3] = {ulo0, ulo1, ulo2}, hi[3] = {uhi0, uhi1, uhi2};
    float x[DX], aux[DY::AUX];
#pragma unroll
    for (int c = 0; c < DX; ++c) x[c] = x0[k * DX + c];
    DY::init(x, aux);
    float* xo = xs + (size_t)idx * (T + 1) * DX;
    const float* ui = u + (size_t)idx * T * DU;
#pragma unroll
    for (int c = 0; c < DX; ++c) xo[c] = x[c];
    for (int t = 0; t < T; ++t) {
        float uu[DU];
#pragma unroll
        for (int d = 0; d < DU; ++d) uu[d] = fminf(fmaxf(ui[t * DU + d], lo[d]), hi[d]);
        DY::step(x, aux, uu, sc);
#pragma unroll
        for (int c = 0; c < DX; ++c) xo[(t + 1) * DX + c] = x[c];
    }
}

struct UpdateArgs {
    const float* eps;        // [D][M]
    const float* r;          // [M]
    const float* du_in;      // [D]
    float* du_out;           // [D]
    float* w_out;            // [M] or null (written by workgroup 0)
    int* status;             // set to D4_ENONFINITE on a non-finite reward, or null
    int D, M;
    float inv_lam;
    int normalize;
    float ms, sigma, os;
};

// Sum and maximum over the workgroup (256 lanes at most), the same bits in
// every lane and every workgroup of the same size.
__device__ __forceinline__ void block_sum_max(float& s, float& mx, float* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    s = wave_sum(s);
    mx = wave_max(mx);
    __syncthreads();
    if (lane == 0) {
        red[wave] = s;
        red[8 + wave] = mx;
    }
    __syncthreads();
    s = red[0];
    mx = red[8];
    for (int w = 1; w < nw; ++w) {
        s += red[w];
        mx = fmaxf(mx, red[8 + w]);
    }
}

// Softmax weights (Section IV-B, p_0 proportional to exp(r/lambda) of the
// batch-normalised rewards) and the one-step update (Eq. mbd-denoising), for
// any sample count: every workgroup stages the rewards in LDS, takes their
// mean, population variance and maximum in a fixed order (two passes),
// replaces them by the unnormalised weights exp(z_m - z_max) with their sum,
// then reduces rows of eps, one wave per row, and applies the normaliser
// once per row.  All workgroups of one launch (and of the batched form, which
// uses the same 256-lane workgroups) compute the same weights bit for bit.
__device__ __forceinline__ void softmax_update_rows(const UpdateArgs& a, int e_begin, int e_step, int e_end,
                                                    bool first, float* wl) {
#pragma clang fp contract(off)
    __shared__ float red[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, bd = blockDim.x;
    const int M = a.M;
    for (int i = tid; i < M; i += bd) wl[i] = a.r[i];
    __syncthreads();
    float sum = 0.0f, mx = -INFINITY;
    for (int i = tid; i < M; i += bd) {
        sum += wl[i];
        mx = fmaxf(mx, wl[i]);
    }
    block_sum_max(sum, mx, red);
    const float mean = sum / (float)M;
    float q = 0.0f, unused = -INFINITY;
    for (int i = tid; i < M; i += bd) {
        const float d = wl[i] - mean;
        q = __builtin_fmaf(d, d, q);
    }
    block_sum_max(q, unused, red);
    const bool bad = !isfinite(mean) || !isfinite(q) || !isfinite(mx);
    float mu = 0.0f, scale = a.inv_lam;
    if (a.normalize) {
        mu = mean;
        scale = a.inv_lam / fmaxf(sqrtf(q / (float)M), 1e-6f);
    }
    const float zmax = (mx - mu) * scale;
    float se = 0.0f;
    for (int i = tid; i < M; i += bd) {
        const float e = bad ? 1.0f : __expf(__builtin_fmaf(wl[i] - mu, scale, -zmax));
        wl[i] = e;
        se += e;
    }
    block_sum_max(se, unused, red);
    const float inv_se = 1.0f / se;
    if (first) {
        if (a.w_out)
            for (int i = tid; i < M; i += blockDim.x) a.w_out[i] = wl[i] * inv_se;
        if (bad && tid == 0 && a.status) *a.status = -4;
    }
    const float s_inv = a.sigma * inv_se;
    for (int e = e_begin + wave; e < e_end; e += e_step) {
        const float* row = a.eps + (size_t)e * M;
        float acc = 0.0f;
        for (int i = lane; i < M; i += 64) acc = __builtin_fmaf(row[i], wl[i], acc);
        acc = wave_sum(acc);
        if (lane == 0) a.du_out[e] = a.os * (a.du_in[e] * a.ms + s_inv * acc);
    }
}

static __global__ void __launch_bounds__(256) k_softmax_update(const UpdateArgs a) {
    extern __shared__ float wl[];
    const int nw = blockDim.x >> 6;
    softmax_update_rows(a, blockIdx.x * nw, gridDim.x * nw, a.D, blockIdx.x == 0, wl);
}

typedef float f4v __attribute__((ext_vector_type(4)));

// Range-checked 16-byte buffer load: bytes past num_records read as zero.
// AUX is the cache policy: 0 the default, CPOL_AGENT a load coherent at
// device scope (sc1), which reads what other workgroups of the same launch
// published with a device-scope release, whichever XCD's L2 they wrote through.
constexpr int CPOL_AGENT = 16;
template <int AUX = 0>
__device__ __forceinline__ f4v load4_checked(__amdgpu_buffer_rsrc_t rs, int byte_offset) {
    return __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(rs, byte_offset, 0, AUX));
}

// The same update for a sample count that is a multiple of 4, with the
// weights in registers: lane t of the 256-lane workgroup owns the float4
// columns t + 256 j (j < J, J * 1024 >= M) of the rewards, the weights and of
// every eps row.  The workgroup handles rows e0 .. e1-1, upd_rows(J) at a
// time (more rows per pass when a lane owns fewer columns, so that each pass
// keeps 8-32 KiB of loads in flight per workgroup); the first rows' loads are
// issued before the statistics so that their latency overlaps the softmax.  Loads are range-checked buffer loads (columns
// past M read as zero and carry weight zero), so no load needs a guard.
// Statistics are taken per lane over its columns in j order, then across the
// wave and the workgroup in a fixed order: every workgroup (of this launch
// and of the batched form) computes the same weights bit for bit.
constexpr int UPD_ROWS_MAX = 8;
constexpr int upd_rows(int J) { return J >= 4 ? 2 : J == 2 ? 4 : 8; }

// Workgroup (four waves) sum, and sum with maximum, through LDS slots that
// no other reduction of the same call reuses, so one barrier each suffices.
__device__ __forceinline__ float block_sum4(float s, float* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    s = wave_sum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}
__device__ __forceinline__ void block_sum_max4(float& s, float& m, float* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    s = wave_sum(s);
    m = wave_max(m);
    if (lane == 0) {
        red[wave] = s;
        red[4 + wave] = m;
    }
    __syncthreads();
    s = (red[0] + red[1]) + (red[2] + red[3]);
    m = fmaxf(fmaxf(red[4], red[5]), fmaxf(red[6], red[7]));
}

// NW = 1 is the one-wave form for up to 256 samples (J = 1): its reductions
// stay in the wave and take no barrier, and each adds the +0.0 that the
// idle waves of the four-wave form contribute, so both forms give the same
// bits.
template <int J, int AUX = 0, int NW = 4>
__device__ __forceinline__ void softmax_update_block(const UpdateArgs& a, int e0, int e1, bool first) {
#pragma clang fp contract(off)
    static_assert(NW == 4 || (NW == 1 && J == 1), "the one-wave form owns one float4 column per lane");
    // statistics slots: sum and maximum [0, 8), squares [8, 12), exponentials [12, 16)
    __shared__ float red[16];
    constexpr int UPD_ROWS = upd_rows(J);
    __shared__ float rowred[UPD_ROWS_MAX][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int M = a.M, M4 = M >> 2;
    const __amdgpu_buffer_rsrc_t r_rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.r), (short)0, M * 4, 0x00020000);
    f4v w[J];
#pragma unroll
    for (int j = 0; j < J; ++j) w[j] = load4_checked<AUX>(r_rs, (tid + 256 * j) * 16);
    f4v x[UPD_ROWS][J];
    // rows past e1 (the last pass of a short range) are not loaded; their
    // sums are formed from zeros and not written
    auto load_rows = [&](int e) {
#pragma unroll
        for (int q = 0; q < UPD_ROWS; ++q) {
            if (e + q < e1) {
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<float*>(a.eps + (size_t)(e + q) * M), (short)0, M * 4, 0x00020000);
#pragma unroll
                for (int j = 0; j < J; ++j) x[q][j] = load4_checked<AUX>(rs, (tid + 256 * j) * 16);
            } else {
#pragma unroll
                for (int j = 0; j < J; ++j) x[q][j] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
            }
        }
    };
    if (e0 < e1) load_rows(e0);
    float sum = 0.0f, mx = -INFINITY;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (tid + 256 * j < M4) {
            sum += w[j].x;
            sum += w[j].y;
            sum += w[j].z;
            sum += w[j].w;
            mx = fmaxf(fmaxf(mx, fmaxf(w[j].x, w[j].y)), fmaxf(w[j].z, w[j].w));
        }
    }
    if constexpr (NW == 4) {
        block_sum_max4(sum, mx, red);
    } else {
        sum = wave_sum(sum) + 0.0f;
        mx = fmaxf(wave_max(mx), -INFINITY);
    }
    const float mean = sum / (float)M;
    float q = 0.0f;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (tid + 256 * j < M4) {
            float d = w[j].x - mean;
            q = __builtin_fmaf(d, d, q);
            d = w[j].y - mean;
            q = __builtin_fmaf(d, d, q);
            d = w[j].z - mean;
            q = __builtin_fmaf(d, d, q);
            d = w[j].w - mean;
            q = __builtin_fmaf(d, d, q);
        }
    }
    q = NW == 4 ? block_sum4(q, red + 8) : wave_sum(q) + 0.0f;
    const bool bad = !isfinite(mean) || !isfinite(q) || !isfinite(mx);
    float mu = 0.0f, scale = a.inv_lam;
    if (a.normalize) {
        mu = mean;
        scale = a.inv_lam / fmaxf(sqrtf(q / (float)M), 1e-6f);
    }
    const float zmax = (mx - mu) * scale;
    float se = 0.0f;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const bool in = tid + 256 * j < M4;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float e = !in ? 0.0f : bad ? 1.0f : __expf(__builtin_fmaf(w[j][c] - mu, scale, -zmax));
            w[j][c] = e;
            se += e;
        }
    }
    se = NW == 4 ? block_sum4(se, red + 12) : wave_sum(se) + 0.0f;
    const float inv_se = 1.0f / se;
    if (first) {
        if (a.w_out) {
#pragma unroll
            for (int j = 0; j < J; ++j)
                if (tid + 256 * j < M4)
#pragma unroll
                    for (int c = 0; c < 4; ++c) a.w_out[4 * (tid + 256 * j) + c] = w[j][c] * inv_se;
        }
        if (bad && tid == 0 && a.status) *a.status = -4;
    }
    const float s_inv = a.sigma * inv_se;
    for (int e = e0; e < e1; e += UPD_ROWS) {
        if (e != e0) load_rows(e);
        float acc[UPD_ROWS];
#pragma unroll
        for (int rr = 0; rr < UPD_ROWS; ++rr) {
            float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, c3 = 0.0f;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                c0 = __builtin_fmaf(x[rr][j].x, w[j].x, c0);
                c1 = __builtin_fmaf(x[rr][j].y, w[j].y, c1);
                c2 = __builtin_fmaf(x[rr][j].z, w[j].z, c2);
                c3 = __builtin_fmaf(x[rr][j].w, w[j].w, c3);
            }
            acc[rr] = wave_sum((c0 + c1) + (c2 + c3));
        }
        if constexpr (NW == 4) {
            __syncthreads();
            if (lane == 0)
#pragma unroll
                for (int rr = 0; rr < UPD_ROWS; ++rr) rowred[rr][wave] = acc[rr];
            __syncthreads();
            if (tid < UPD_ROWS && e + tid < e1) {
                const float t = (rowred[tid][0] + rowred[tid][1]) + (rowred[tid][2] + rowred[tid][3]);
                a.du_out[e + tid] = a.os * (a.du_in[e + tid] * a.ms + s_inv * t);
            }
        } else {
            // every lane holds every row's sum; lane rr writes row e + rr
            float t = 0.0f;
#pragma unroll
            for (int rr = 0; rr < UPD_ROWS; ++rr) t = tid == rr ? acc[rr] : t;
            t = t + 0.0f;
            if (tid < UPD_ROWS && e + tid < e1) a.du_out[e + tid] = a.os * (a.du_in[e + tid] * a.ms + s_inv * t);
        }
    }
}

// Rows split evenly over the grid.
template <int J>
__global__ void __launch_bounds__(256) k_softmax_update_reg(const UpdateArgs a) {
    const int e0 = (int)((long long)a.D * blockIdx.x / gridDim.x);
    const int e1 = (int)((long long)a.D * (blockIdx.x + 1) / gridDim.x);
    softmax_update_block<J>(a, e0, e1, blockIdx.x == 0);
}

// The same with one wave per workgroup, for up to 256 samples.
static __global__ void __launch_bounds__(64) k_softmax_update_wave(const UpdateArgs a) {
    const int e0 = (int)((long long)a.D * blockIdx.x / gridDim.x);
    const int e1 = (int)((long long)a.D * (blockIdx.x + 1) / gridDim.x);
    softmax_update_block<1, 0, 1>(a, e0, e1, blockIdx.x == 0);
}

static __global__ void k_fill(float* p, int n, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static __global__ void k_set_iter(uint32_t* it, uint32_t v, int* status) {
    *it = v;
    *status = 0;
}

struct FinalArgs {
    float* u_base;        // [D] updated in place
    const float* du0;     // [D]
    const float* x0;      // [n][dx]
    const float* goal;    // [n][dp]
    float* traj;          // [n][T+1][dx]
    float* stats;         // d4_stats layout: reward, objective, hits, robots_hit, success, at_goal,
                          // obstacle_hits, status
    const int* status;    // sticky status of the iteration
    int n, T;
    float ulo[3], uhi[3];
    StepConsts sc;
    float thr2, safe2, goal_tol, w_safe, d0_floor;
    uint32_t flags;
    // obstacles: (centre, reward distance^2) and safety distance^2, from device
    // memory (obs, obs_safe2) or, when obs is null, from the arguments
    int n_obs;
    const float4* obs;
    const float* obs_safe2;
    float4 obs_inline[MAX_OBS];
    float safe2_inline[MAX_OBS];
};

// One block: apply the deformation, roll the plan out, score it.
template <int DYN>
__device__ __forceinline__ void apply_final_body(const FinalArgs& a) {
    using DY = Dyn<DYN>;
    constexpr int DX = DY::DX, DU = DY::DU, DP = DY::DP;
    __shared__ float red_g[256];
    __shared__ int red_s[256], red_h[256], red_o[256], red_bad[256], red_ob[256];
    const int n = a.n, T = a.T, D = n * T * DU;
    const int tid = threadIdx.x;
    for (int e = tid; e < D; e += blockDim.x) {
        const int d = e % DU;
        a.u_base[e] = fminf(fmaxf(a.u_base[e] + a.du0[e], a.ulo[d]), a.uhi[d]);
    }
    __syncthreads();
    float gacc = 0.0f;
    int at_goal = 0, term_bad = 0, obs_cnt = 0, obs_unsafe = 0;
    const float4* ob = a.obs ? a.obs : a.obs_inline;
    const float* ob_safe2 = a.obs ? a.obs_safe2 : a.safe2_inline;
    if (tid < n) {
        const int k = tid;
        float x[DX], aux[DY::AUX], g[DP];
#pragma unroll
        for (int c = 0; c < DX; ++c) x[c] = a.x0[k * DX + c];
        DY::init(x, aux);
#pragma unroll
        for (int c = 0; c < DP; ++c) g[c] = a.goal[k * DP + c];
        const float inv_d0 = inv_start_dist(goal_d2<DP>(x, g), a.d0_floor);
        float* tr = a.traj + (size_t)k * (T + 1) * DX;
#pragma unroll
        for (int c = 0; c < DX; ++c) tr[c] = x[c];
        for (int t = 0; t < T; ++t) {
            float u[DU];
#pragma unroll
            for (int d = 0; d < DU; ++d) u[d] = a.u_base[(k * T + t) * DU + d];
            DY::step(x, aux, u, a.sc);
#pragma unroll
            for (int c = 0; c < DX; ++c) tr[(t + 1) * DX + c] = x[c];
            const float dist = fast_sqrt(goal_d2<DP>(x, g));
            gacc += goal_term(dist, inv_d0);
            at_goal += dist <= a.goal_tol;
            if (t == T - 1) term_bad = dist > a.goal_tol;
            int hit = 0;
            for (int o = 0; o < a.n_obs; ++o) {
                const float4 c = ob[o];
                const float cc[3] = {c.x, c.y, c.z};
                const float d2 = pair_d2<DP>(x, cc);
                hit |= d2 <= c.w ? 1 : 0;
                obs_unsafe |= d2 <= ob_safe2[o] ? 1 : 0;
            }
            obs_cnt += hit;
        }
    }
    __syncthreads();
    // pair checks of every (step, robot) spread over the whole workgroup
    int safe_cnt = 0, hit_cnt = 0, unsafe = 0;
    for (int idx = tid; idx < T * n; idx += blockDim.x) {
        const int t = idx / n + 1, k = idx - (idx / n) * n;
        float pk[DP];
#pragma unroll
        for (int c = 0; c < DP; ++c) pk[c] = a.traj[((size_t)k * (T + 1) + t) * DX + c];
        int partners = 0;
        for (int l = 0; l < n; ++l) {
            if (l == k) continue;
            float pl[DP];
#pragma unroll
            for (int c = 0; c < DP; ++c) pl[c] = a.traj[((size_t)l * (T + 1) + t) * DX + c];
            const float d2 = pair_d2<DP>(pk, pl);
            if (d2 <= a.thr2) {
                ++partners;
                if (k < l) ++hit_cnt;
            }
            if (d2 <= a.safe2) unsafe = 1;
        }
        safe_cnt += partners > 0;
    }
    red_g[tid] = gacc;
    red_s[tid] = safe_cnt;
    red_h[tid] = hit_cnt;
    red_o[tid] = at_goal;
    red_bad[tid] = (unsafe | obs_unsafe) | (term_bad << 1);
    red_ob[tid] = obs_cnt;
    __syncthreads();
    if (tid == 0) {
        float gs = 0.0f;
        int ss = 0, hs = 0, os = 0, bad = 0, obt = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) {
            gs += red_g[i];
            ss += red_s[i];
            hs += red_h[i];
            os += red_o[i];
            bad |= red_bad[i];
            obt += red_ob[i];
        }
        const float pen = (float)(((a.flags & FLAG_SAFE_PAIRS) ? 2 * hs : ss) + obt);
        a.stats[0] = team_reward(gs, a.w_safe, pen, n * T);
        a.stats[1] = (float)os / (float)(n * T);
        int* si = reinterpret_cast<int*>(a.stats);
        si[2] = hs;
        si[3] = ss;
        si[4] = (bad & 1) ? 0 : 1;
        si[5] = (bad & 2) ? 0 : 1;
        si[6] = obt;
        si[7] = a.status ? *a.status : 0;
    }
}

template <int DYN>
__global__ void __launch_bounds__(256) k_apply_final(const FinalArgs a) {
    apply_final_body<DYN>(a);
}

// ------------------------------------------------------------- batched form
// Many independent problems per launch.  Every instance shares the sample
// count M, the schedule, the temperature, the flags and the Philox key; the
// team size, horizon, dynamics and limits are its own.  Offsets count floats
// (or samples) into packed arrays in instance order.
struct BatchInst {
    int n, T, dyn, S, Tb, mode, D, n_obs;
    float4 obs[MAX_OBS];        // centre, reward distance^2
    float obs_safe2[MAX_OBS];   // safety distance^2
    long long x0, goal, u, eps, r, traj;
    float thr2, safe2, w_safe, d0_floor, goal_tol;
    float ulo[3], uhi[3];
    StepConsts sc;
    uint32_t inst_id;
};
struct BatchTile {   // samples m0 .. m0+S-1 of one instance
    int inst, m0;
};
struct BatchRows {   // rows e0 .. e1-1 of one instance's update
    int inst, e0, e1;
};

struct BatchStepArgs {
    const BatchInst* insts;
    const BatchTile* tiles;
    const float* x0;
    const float* goal;
    const float* u;
    const float* du_in;
    float* eps;
    float* r;
    int* hits;
    const uint32_t* iter_dev;
    int M;
    uint32_t key0, key1, step, flags;
    float mean_scale, sigma;
};

// Sampling + rollout + reward of samples m0 .. m0+S-1 of instance inst (one
// 256-lane workgroup).
__device__ __forceinline__ void batch_reward_tile(const BatchStepArgs& b, int inst, int m0, float* lds) {
    const BatchTile tl{inst, m0};
    const BatchInst& in = b.insts[tl.inst];
    RollFitArgs a;
    a.x0 = b.x0 + in.x0;
    a.goal = b.goal + in.goal;
    a.u_base = b.u + in.u;
    a.du_in = b.du_in + in.u;
    a.xs = nullptr;
    a.eps = b.eps + in.eps;
    a.r = b.r + in.r;
    a.hits = b.hits + in.r;
    a.robots_hit = nullptr;
    a.iter_dev = b.iter_dev;
    a.n = in.n;
    a.T = in.T;
    a.M = b.M;
    a.S = in.S;
    a.Tb = in.Tb;
    a.mean_scale = b.mean_scale;
    a.sigma = b.sigma;
    a.thr2 = in.thr2;
    a.w_safe = in.w_safe;
    a.d0_floor = in.d0_floor;
    for (int d = 0; d < 3; ++d) {
        a.ulo[d] = in.ulo[d];
        a.uhi[d] = in.uhi[d];
    }
    a.sc = in.sc;
    a.key0 = b.key0;
    a.key1 = b.key1;
    a.step = b.step;
    a.iter = 0;
    a.inst = in.inst_id;
    a.flags = b.flags;
    a.n_obs = in.n_obs;
    a.obs = in.obs;
    const bool al = in.mode == MODE_FUSED_ALIGNED;
    switch (in.dyn) {
        case HOLO2D:
            if (al) rollfit_tile<HOLO2D, MODE_FUSED_ALIGNED, 1, false>(a, tl.m0, lds);
            else rollfit_tile<HOLO2D, MODE_FUSED, 1, false>(a, tl.m0, lds);
            break;
        case HOLO3D:
            if (al) rollfit_tile<HOLO3D, MODE_FUSED_ALIGNED, 1, false>(a, tl.m0, lds);
            else rollfit_tile<HOLO3D, MODE_FUSED, 1, false>(a, tl.m0, lds);
            break;
        case UNICYCLE:
            if (al) rollfit_tile<UNICYCLE, MODE_FUSED_ALIGNED, 1, false>(a, tl.m0, lds);
            else rollfit_tile<UNICYCLE, MODE_FUSED, 1, false>(a, tl.m0, lds);
            break;
        default:
            if (al) rollfit_tile<DIFFDRIVE, MODE_FUSED_ALIGNED, 1, false>(a, tl.m0, lds);
            else rollfit_tile<DIFFDRIVE, MODE_FUSED, 1, false>(a, tl.m0, lds);
            break;
    }
}

// One reward tile per workgroup, from the launch's tile list.
static __global__ void __launch_bounds__(256) k_batch_rollfit(const BatchStepArgs b) {
    extern __shared__ float lds[];
    const BatchTile tl = b.tiles[blockIdx.x];
    batch_reward_tile(b, tl.inst, tl.m0, lds);
}

struct BatchUpdArgs {
    const BatchInst* insts;
    const BatchRows* rows;
    const float* eps;
    const float* r;
    const float* du_in;
    float* du_out;
    int* status;  // [count]
    int M;
    float inv_lam;
    int normalize;
    float ms, sigma, os;
};

// Softmax weights and the update of rows e0 .. e1-1 of instance inst (one
// 256-lane workgroup): the register form (J > 0, sample count a multiple of
// 4) or the LDS form (J = 0, weights staged in wl).
template <int J, int AUX = 0>
__device__ __forceinline__ void batch_update_tile(const BatchUpdArgs& b, int inst, int e0, int e1, float* wl) {
    const BatchRows rt{inst, e0, e1};
    const BatchInst& in = b.insts[rt.inst];
    UpdateArgs a;
    a.eps = b.eps + in.eps;
    a.r = b.r + in.r;
    a.du_in = b.du_in + in.u;
    a.du_out = b.du_out + in.u;
    a.w_out = nullptr;
    a.status = b.status + rt.inst;
    a.D = in.D;
    a.M = b.M;
    a.inv_lam = b.inv_lam;
    a.normalize = b.normalize;
    a.ms = b.ms;
    a.sigma = b.sigma;
    a.os = b.os;
    if constexpr (J > 0)
        softmax_update_block<J, AUX>(a, rt.e0, rt.e1, rt.e0 == 0);
    else
        softmax_update_rows(a, rt.e0, blockDim.x >> 6, rt.e1, rt.e0 == 0, wl);
}

// One row range per workgroup, from the launch's row list.
template <int J>
__global__ void __launch_bounds__(256) k_batch_update(const BatchUpdArgs b) {
    extern __shared__ float wl[];
    const BatchRows rt = b.rows[blockIdx.x];
    batch_update_tile<J>(b, rt.inst, rt.e0, rt.e1, wl);
}

// ----------------------------------------------- persistent batched step
// Work item of the persistent step kernel: a reward tile (kind 0: samples
// a .. a+S-1 of instance inst) or an update tile (kind 1: rows a .. b-1).
struct BatchWork {
    int kind, inst, a, b;
};

// Per-step counters of the persistent kernel (ints): the next work item, the
// workgroups that have left, a wait-timeout flag, then per instance the
// number of its reward tiles completed.
enum { CNT_NEXT = 0, CNT_EXIT = 1, CNT_ERROR = 2, CNT_DONE = 3 };

struct BatchPersistArgs {
    BatchStepArgs s;
    BatchUpdArgs u;
    const BatchWork* work;
    const int* tiles_of;   // [count] reward tiles per instance
    int* cnt;              // this step's counter set: CNT_DONE + count ints
    int n_work, count, spin_limit;
};

// One denoising step of every instance in one launch.  Workgroups take work
// items in list order from an atomic counter.  A reward tile publishes its
// draws, rewards and counts with a device-scope release (each wave writes
// its stores back past its XCD's L2, then one lane counts the tile done for
// its instance); an update tile first waits until every reward tile of its
// instance is done, polling the count with relaxed device-scope loads (no
// cache invalidation per poll), and then reads the instance's rewards and
// draws with device-coherent (sc1) loads; the LDS form of the update, for
// sample counts that are not a multiple of 4, takes a device-scope acquire
// instead.  The list puts every reward tile of an instance before any of its
// update tiles, so an update tile only waits on reward tiles that running
// workgroups already hold: the wait always ends.  It is bounded all the same:
// past spin_limit polls, or once any workgroup has timed out, the workgroup
// sets the error flag, skips the tile and goes on, so every workgroup exits.
// The last workgroup to leave clears the counter set for its next use.
template <int J>
__global__ void __launch_bounds__(256) k_batch_persist(const BatchPersistArgs p) {
    extern __shared__ float lds[];
    __shared__ int s_item, s_ok;
    int* const done = p.cnt + CNT_DONE;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&p.cnt[CNT_NEXT], 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= p.n_work) break;
        const BatchWork w = p.work[it];
        if (w.kind == 0) {
            batch_reward_tile(p.s, w.inst, w.a, lds);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (threadIdx.x == 0) __hip_atomic_fetch_add(&done[w.inst], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (threadIdx.x == 0) {
                const int need = p.tiles_of[w.inst];
                int spins = 0, ok = 1;
                while (__hip_atomic_load(&done[w.inst], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (++spins > p.spin_limit ||
                        __hip_atomic_load(&p.cnt[CNT_ERROR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        ok = 0;
                        atomicExch(&p.cnt[CNT_ERROR], 1);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
                s_ok = ok;
            }
            __syncthreads();
            if (s_ok) {
                if constexpr (J > 0) {
                    batch_update_tile<J, CPOL_AGENT>(p.u, w.inst, w.a, w.b, lds);
                } else {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    batch_update_tile<0>(p.u, w.inst, w.a, w.b, lds);
                }
            }
            __syncthreads();
        }
    }
    __shared__ int s_last;
    if (threadIdx.x == 0) s_last = atomicAdd(&p.cnt[CNT_EXIT], 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (s_last) {
        __threadfence();
        for (int j = threadIdx.x; j < p.count; j += blockDim.x) done[j] = 0;
        if (threadIdx.x == 0) {
            p.cnt[CNT_NEXT] = 0;
            p.cnt[CNT_EXIT] = 0;
        }
    }
}

struct BatchFinalArgs {
    const int* wait_error;   // two counter sets' error flags (CNT_ERROR of each), or null
    int cnt_stride;
    const BatchInst* insts;
    float* u;
    const float* du0;
    const float* x0;
    const float* goal;
    float* traj;
    float* stats;        // [count][8], d4_stats layout
    const int* status;   // [count]
    uint32_t flags;
};

// Apply, roll out and score one instance per workgroup.
static __global__ void __launch_bounds__(256) k_batch_final(const BatchFinalArgs b) {
    const BatchInst& in = b.insts[blockIdx.x];
    FinalArgs a;
    a.u_base = b.u + in.u;
    a.du0 = b.du0 + in.u;
    a.x0 = b.x0 + in.x0;
    a.goal = b.goal + in.goal;
    a.traj = b.traj + in.traj;
    a.stats = b.stats + 8 * (size_t)blockIdx.x;
    a.status = b.status + blockIdx.x;
    a.n = in.n;
    a.T = in.T;
    for (int d = 0; d < 3; ++d) {
        a.ulo[d] = in.ulo[d];
        a.uhi[d] = in.uhi[d];
    }
    a.sc = in.sc;
    a.thr2 = in.thr2;
    a.safe2 = in.safe2;
    a.goal_tol = in.goal_tol;
    a.w_safe = in.w_safe;
    a.d0_floor = in.d0_floor;
    a.flags = b.flags;
    a.n_obs = in.n_obs;
    a.obs = in.obs;
    a.obs_safe2 = in.obs_safe2;
    switch (in.dyn) {
        case HOLO2D: apply_final_body<HOLO2D>(a); break;
        case HOLO3D: apply_final_body<HOLO3D>(a); break;
        case UNICYCLE: apply_final_body<UNICYCLE>(a); break;
        default: apply_final_body<DIFFDRIVE>(a); break;
    }
    // a persistent step whose wait timed out skipped update tiles: every
    // instance reports it (the stats' status word, thread 0 wrote it above)
    if (threadIdx.x == 0 && b.wait_error && (b.wait_error[0] | b.wait_error[b.cnt_stride]))
        reinterpret_cast<int*>(a.stats)[7] = -3;
}

static __global__ void k_fill_int(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace d4
