// Kernels of the denoising hot path.
//
//  k_noise             - standard normal draws eps[e][m] (sampling step of Algorithm 1)
//  k_rollout           - RK4 rollout of given controls (Section III, Section IV-C)
//  k_rollfit<DYN,X>    - reward of trajectories (Eq. generic-reward): with X = false the
//                        fused sample + rollout + reward of one denoising step, with X = true
//                        the reward of trajectories read from memory
//  k_softmax           - batch normalisation and softmax weights (p_0 of Section IV-B)
//  k_reduce_update     - S[e] = sum_m w_m eps[e][m] and the one-step update (Eq. mbd-denoising)
//  k_apply_final       - tau.u <- clip(tau.u + Delta U_0), rollout and stats (Algorithm 2)
//
// Lane mapping of k_rollfit: one lane per (sample m, robot k) with the sample
// index fastest, S samples per workgroup (blockDim = n*S).  A lane keeps its
// robot's state in registers and walks t = 0..T-1; positions of a block of Tb
// steps go to LDS as [Tb][d_p][n][S] so that the pair checks of one step read
// consecutive addresses across a wave.  Lane k checks partners (k + j) mod n
// for j = 1..floor((n-1)/2), plus j = n/2 for k < n/2 when n is even: every
// unordered pair exactly once, spread evenly.  The per-(m, t) "robot k hit
// anything" bits are OR-ed into an LDS word; positions and masks are double
// buffered, so each time block costs two barriers.
#pragma once

#include "d4_device.hpp"

namespace d4 {

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
};

template <int DYN, bool FROM_X>
__global__ void __launch_bounds__(1024) k_rollfit(const RollFitArgs a) {
    using DY = Dyn<DYN>;
    constexpr int DX = DY::DX, DU = DY::DU, DP = DY::DP;
    extern __shared__ float lds[];
    const int n = a.n, T = a.T, M = a.M, S = a.S, Tb = a.Tb;
    const int tid = threadIdx.x;
    const int k = tid / S;
    const int ms = tid - k * S;
    const int m = blockIdx.x * S + ms;
    const bool live = m < M;
    const int mc = live ? m : M - 1;
    float* pos = lds;                                                   // [2][Tb][DP][n][S]
    uint32_t* mask = reinterpret_cast<uint32_t*>(lds + 2 * Tb * DP * n * S);  // [2][Tb][S]

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
    float d0s = 0.0f;
#pragma unroll
    for (int c = 0; c < DP; ++c) d0s += (x[c] - g[c]) * (x[c] - g[c]);
    const float inv_d0 = 1.0f / fmaxf(sqrtf(d0s), a.d0_floor);

    float goal_acc = 0.0f;
    int safe_cnt = 0, hit_cnt = 0;

    NormalStream ns;
    const uint32_t iter = a.iter_dev ? *a.iter_dev : a.iter;
    ns.init((uint32_t)mc, (iter << 16) | a.step, a.inst, a.key0, a.key1);
    float ulo[DU], uhi[DU];
#pragma unroll
    for (int d = 0; d < DU; ++d) {
        ulo[d] = a.ulo[d];
        uhi[d] = a.uhi[d];
    }
    const int jhalf = (n - 1) >> 1;
    const bool extra = ((n & 1) == 0) && (k < (n >> 1));
    const bool pairs_mode = (a.flags & FLAG_SAFE_PAIRS) != 0;

    const int nblk = (T + Tb - 1) / Tb;
    for (int b = 0; b < nblk; ++b) {
        const int buf = b & 1;
        const int t0 = b * Tb;
        const int tcount = min(Tb, T - t0);
        for (int tt = 0; tt < tcount; ++tt) {
            const int t = t0 + tt;
            if (FROM_X) {
                const float* xr = a.xs + (((size_t)mc * n + k) * (size_t)(T + 1) + (t + 1)) * DX;
#pragma unroll
                for (int c = 0; c < DP; ++c) x[c] = xr[c];
            } else {
                float u[DU];
                const uint32_t e0 = (uint32_t)((k * T + t) * DU);
#pragma unroll
                for (int d = 0; d < DU; ++d) {
                    const uint32_t e = e0 + d;
                    const float z = ns.get(e);
                    if (live) a.eps[(size_t)e * M + m] = z;
                    const float cb = a.u_base[e] + a.du_in[e] * a.mean_scale;
                    u[d] = fminf(fmaxf(cb + a.sigma * z, ulo[d]), uhi[d]);
                }
                DY::step(x, aux, u, a.sc);
            }
            float dist2 = 0.0f;
#pragma unroll
            for (int c = 0; c < DP; ++c) dist2 += (x[c] - g[c]) * (x[c] - g[c]);
            goal_acc += 1.0f - sqrtf(dist2) * inv_d0;
#pragma unroll
            for (int c = 0; c < DP; ++c) pos[(((buf * Tb + tt) * DP + c) * n + k) * S + ms] = x[c];
        }
        if (k == 0)
            for (int tt = 0; tt < tcount; ++tt) mask[(buf * Tb + tt) * S + ms] = 0u;
        __syncthreads();
        for (int tt = 0; tt < tcount; ++tt) {
            const float* pb = pos + ((buf * Tb + tt) * DP) * n * S + ms;
            float pk[DP];
#pragma unroll
            for (int c = 0; c < DP; ++c) pk[c] = pb[(c * n + k) * S];
            uint32_t bits = 0u;
            const int jmax = jhalf + (extra ? 1 : 0);
            for (int j = 1; j <= jmax; ++j) {
                int l = k + j;
                if (l >= n) l -= n;
                float pl[DP];
#pragma unroll
                for (int c = 0; c < DP; ++c) pl[c] = pb[(c * n + l) * S];
                if (pair_d2<DP>(pk, pl) <= a.thr2) {
                    bits |= 1u << l;
                    ++hit_cnt;
                }
            }
            if (bits) atomicOr(&mask[(buf * Tb + tt) * S + ms], bits | (1u << k));
        }
        __syncthreads();
        for (int tt = 0; tt < tcount; ++tt) safe_cnt += (mask[(buf * Tb + tt) * S + ms] >> k) & 1u;
    }

    __syncthreads();
    float* rg = lds;
    int* rs = reinterpret_cast<int*>(lds + n * S);
    int* rh = rs + n * S;
    rg[k * S + ms] = goal_acc;
    rs[k * S + ms] = safe_cnt;
    rh[k * S + ms] = hit_cnt;
    __syncthreads();
    if (k == 0 && live) {
        float gs = 0.0f;
        int ss = 0, hs = 0;
        for (int kk = 0; kk < n; ++kk) {
            gs += rg[kk * S + ms];
            ss += rs[kk * S + ms];
            hs += rh[kk * S + ms];
        }
        const float pen = pairs_mode ? (float)(2 * hs) : (float)ss;
        a.r[m] = (gs - a.w_safe * pen) / (float)(n * T);
        a.hits[m] = hs;
        if (a.robots_hit) a.robots_hit[m] = ss;
    }
}

// eps[e][m] for e < D, m < M; one lane per (Philox block, sample).
__global__ void __launch_bounds__(256) k_noise(float* eps, int D, int M, uint32_t c2, uint32_t c3,
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

// Block-wide reduction for blockDim a multiple of 64 (<= 1024); all threads get the result.
template <bool MAX>
__device__ __forceinline__ float block_reduce(float v, float* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = MAX ? wave_max(v) : wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    float r = red[0];
    for (int i = 1; i < nw; ++i) r = MAX ? fmaxf(r, red[i]) : r + red[i];
    return r;
}

// Softmax weights of one batch of rewards; a non-finite reward sets *status
// and falls back to uniform weights.
__global__ void __launch_bounds__(1024) k_softmax(const float* r, float* w, int M, float inv_lam,
                                                  int normalize, int* status) {
    __shared__ float red[16];
    const int tid = threadIdx.x, nt = blockDim.x;
    float s = 0.0f;
    int bad = 0;
    for (int i = tid; i < M; i += nt) {
        const float v = r[i];
        bad |= !isfinite(v);
        s += v;
    }
    const float nbad = block_reduce<false>((float)bad, red);
    if (nbad > 0.0f) {
        for (int i = tid; i < M; i += nt) w[i] = 1.0f / (float)M;
        if (tid == 0 && status) *status = -4;
        return;
    }
    float mu = 0.0f, scale = inv_lam;
    if (normalize) {
        mu = block_reduce<false>(s, red) / (float)M;
        float q = 0.0f;
        for (int i = tid; i < M; i += nt) {
            const float d = r[i] - mu;
            q += d * d;
        }
        const float var = block_reduce<false>(q, red) / (float)M;
        scale = inv_lam / fmaxf(sqrtf(var), 1e-6f);
    }
    float mx = -INFINITY;
    for (int i = tid; i < M; i += nt) mx = fmaxf(mx, (r[i] - mu) * scale);
    mx = block_reduce<true>(mx, red);
    float se = 0.0f;
    for (int i = tid; i < M; i += nt) se += expf((r[i] - mu) * scale - mx);
    se = block_reduce<false>(se, red);
    const float inv = 1.0f / se;
    for (int i = tid; i < M; i += nt) w[i] = expf((r[i] - mu) * scale - mx) * inv;
}

// du_out[e] = os * (du_in[e] * ms + sigma * sum_m w[m] eps[e][m]); one wave per row.
template <bool STAGED, bool VEC>
__global__ void __launch_bounds__(256) k_reduce_update(const float* __restrict__ eps,
                                                       const float* __restrict__ w,
                                                       const float* __restrict__ du_in,
                                                       float* __restrict__ du_out, int D, int M,
                                                       float ms, float sigma, float os) {
    extern __shared__ float wl[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const float* wsrc = w;
    if (STAGED) {
        for (int i = tid; i < M; i += blockDim.x) wl[i] = w[i];
        __syncthreads();
        wsrc = wl;
    }
    for (int e = blockIdx.x * nw + wave; e < D; e += gridDim.x * nw) {
        const float* row = eps + (size_t)e * M;
        float acc = 0.0f;
        if (VEC) {
            const float4* r4 = reinterpret_cast<const float4*>(row);
            const float4* w4 = reinterpret_cast<const float4*>(wsrc);
            const int M4 = M >> 2;
#pragma unroll 4
            for (int i = lane; i < M4; i += 64) {
                const float4 a = r4[i], b = w4[i];
                acc += a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
            }
        } else {
            for (int i = lane; i < M; i += 64) acc += row[i] * wsrc[i];
        }
        acc = wave_sum(acc);
        if (lane == 0) du_out[e] = os * (du_in[e] * ms + sigma * acc);
    }
}

__global__ void k_fill(float* p, int n, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_set_iter(uint32_t* it, uint32_t v, int* status) {
    *it = v;
    *status = 0;
}

struct FinalArgs {
    float* u_base;        // [D] updated in place
    const float* du0;     // [D]
    const float* x0;      // [n][dx]
    const float* goal;    // [n][dp]
    float* traj;          // [n][T+1][dx]
    float* stats;         // d4_stats layout: reward, objective, hits, robots_hit, success, status
    const int* status;    // sticky status of the iteration
    int n, T;
    float ulo[3], uhi[3];
    StepConsts sc;
    float thr2, safe2, goal_tol, w_safe, d0_floor;
    uint32_t flags;
};

// One block: apply the deformation, roll the plan out, score it.
template <int DYN>
__global__ void __launch_bounds__(256) k_apply_final(const FinalArgs a) {
    using DY = Dyn<DYN>;
    constexpr int DX = DY::DX, DU = DY::DU, DP = DY::DP;
    __shared__ float red_g[256];
    __shared__ int red_s[256], red_h[256], red_o[256], red_bad[256];
    const int n = a.n, T = a.T, D = n * T * DU;
    const int tid = threadIdx.x;
    for (int e = tid; e < D; e += blockDim.x) {
        const int d = e % DU;
        a.u_base[e] = fminf(fmaxf(a.u_base[e] + a.du0[e], a.ulo[d]), a.uhi[d]);
    }
    __syncthreads();
    float gacc = 0.0f;
    int at_goal = 0, term_bad = 0;
    if (tid < n) {
        const int k = tid;
        float x[DX], aux[DY::AUX], g[DP];
#pragma unroll
        for (int c = 0; c < DX; ++c) x[c] = a.x0[k * DX + c];
        DY::init(x, aux);
#pragma unroll
        for (int c = 0; c < DP; ++c) g[c] = a.goal[k * DP + c];
        float d0s = 0.0f;
#pragma unroll
        for (int c = 0; c < DP; ++c) d0s += (x[c] - g[c]) * (x[c] - g[c]);
        const float inv_d0 = 1.0f / fmaxf(sqrtf(d0s), a.d0_floor);
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
            float d2 = 0.0f;
#pragma unroll
            for (int c = 0; c < DP; ++c) d2 += (x[c] - g[c]) * (x[c] - g[c]);
            const float dist = sqrtf(d2);
            gacc += 1.0f - dist * inv_d0;
            at_goal += dist <= a.goal_tol;
            if (t == T - 1) term_bad = dist > a.goal_tol;
        }
    }
    __syncthreads();
    int safe_cnt = 0, hit_cnt = 0, unsafe = 0;
    if (tid < n) {
        const int k = tid;
        for (int t = 1; t <= T; ++t) {
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
    }
    red_g[tid] = gacc;
    red_s[tid] = safe_cnt;
    red_h[tid] = hit_cnt;
    red_o[tid] = at_goal;
    red_bad[tid] = unsafe | term_bad;
    __syncthreads();
    if (tid == 0) {
        float gs = 0.0f;
        int ss = 0, hs = 0, os = 0, bad = 0;
        for (int i = 0; i < n; ++i) {
            gs += red_g[i];
            ss += red_s[i];
            hs += red_h[i];
            os += red_o[i];
            bad |= red_bad[i];
        }
        const float pen = (a.flags & FLAG_SAFE_PAIRS) ? (float)(2 * hs) : (float)ss;
        a.stats[0] = (gs - a.w_safe * pen) / (float)(n * T);
        a.stats[1] = (float)os / (float)(n * T);
        int* si = reinterpret_cast<int*>(a.stats);
        si[2] = hs;
        si[3] = ss;
        si[4] = bad ? 0 : 1;
        si[5] = a.status ? *a.status : 0;
    }
}

}  // namespace d4
