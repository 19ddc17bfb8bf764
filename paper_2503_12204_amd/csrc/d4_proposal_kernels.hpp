// Kernels of the learned proposal: a permutation-equivariant set network over
// the robots of each instance, trained on plans the planner solved.
//
//  k_gemm_bf16<TA,TB,WM,WN>  C = alpha op(A) op(B) + beta C with BF16 operands
//                      and FP32 accumulation on the 32x32x16 MFMA; op(X) = X or
//                      X^T.  64x64 or 128x128 workgroup tiles, four waves, K
//                      steps of 32 staged in LDS k-contiguous for both operands.
//  elementwise         embedding, bias + ReLU, instance mean / sum pooling and
//                      their broadcasts, residual sums, masked MSE, column sums,
//                      Adam with FP32 master weights, BF16 rounding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace d4p {

typedef uint16_t bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ bf16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int BK = 32, KPAD = 8;

// Eight consecutive BF16 values of one operand row (op = X) or of one stored
// row of a transposed operand, starting at (outer, inner0): one 16-byte
// global load when the whole group is in range and 16-byte aligned, element
// loads (zero past the edges) otherwise.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 load8_bf16(const bf16_t* __restrict__ X, int ld, int outer, int n_outer,
                                            int inner0, int n_inner) {
    u32x4 v = {0u, 0u, 0u, 0u};
    if (outer >= n_outer) return v;
    const bf16_t* p = X + (size_t)outer * ld + inner0;
    if (inner0 + 8 <= n_inner && (reinterpret_cast<uintptr_t>(p) & 15u) == 0)
        return *reinterpret_cast<const u32x4*>(p);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if (inner0 + i < n_inner) w[i >> 1] |= (uint32_t)p[i] << (16 * (i & 1));
    v[0] = w[0];
    v[1] = w[1];
    v[2] = w[2];
    v[3] = w[3];
    return v;
}

// C = alpha op(A) op(B) + beta C.  Workgroup tiles of (64 WM) x (64 WN), four
// waves in a 2 x 2 grid, each wave WM x WN blocks of 32x32 on
// v_mfma_f32_32x32x16_bf16, K in steps of 32: 64x64 tiles (WM = WN = 1) for the
// network's small products, 128x128 (WM = WN = 2) for large ones, where each
// operand element staged in LDS feeds twice as many MFMAs.  Each lane moves
// WM (A) and WN (B) groups of eight BF16 values per K step with 16-byte global
// loads (both operands are stored k-contiguous in LDS, so a transposed
// operand's group is scattered into its eight k rows on the way in).  The LDS
// tiles are double buffered: the loads of step k+1 go out before the MFMAs of
// step k, and one barrier per step separates the writes of one buffer from
// the reads of the other.  Every output element accumulates its K range in
// the same order (K steps in turn, 16 k per MFMA) whatever the tile, so both
// tiles give the same bits.
template <bool TA, bool TB, int WM, int WN>
__global__ void __launch_bounds__(256) k_gemm_bf16(const bf16_t* __restrict__ A, const bf16_t* __restrict__ B,
                                                   float* __restrict__ C, int M, int N, int K, int lda,
                                                   int ldb, int ldc, float alpha, float beta) {
    constexpr int TM = 64 * WM, TN = 64 * WN;
    __shared__ __attribute__((aligned(16))) bf16_t As[2][TM][BK + KPAD];
    __shared__ __attribute__((aligned(16))) bf16_t Bs[2][TN][BK + KPAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    // group q = tid + 256 g of an operand tile: non-transposed, row q/4 and k
    // (q%4)*8; transposed (stored [K][outer]), k row q%32 and outer (q/32)*8,
    // so that the 32 lanes writing one step of the scatter below fill 32
    // consecutive k of the same LDS row (two to a bank) instead of one k of
    // rows eight apart (which fall into two banks)
    auto load_a = [&](int k0, int g) {
        const int q = tid + 256 * g;
        return TA ? load8_bf16(A, lda, k0 + (q & 31), K, m0 + (q >> 5) * 8, M)
                  : load8_bf16(A, lda, m0 + (q >> 2), M, k0 + (q & 3) * 8, K);
    };
    auto load_b = [&](int k0, int g) {
        const int q = tid + 256 * g;
        return TB ? load8_bf16(B, ldb, n0 + (q >> 2), N, k0 + (q & 3) * 8, K)
                  : load8_bf16(B, ldb, k0 + (q & 31), K, n0 + (q >> 5) * 8, N);
    };
    auto store = [&](bf16_t (*T)[BK + KPAD], bool trans, int g, u32x4 v) {
        const int q = tid + 256 * g;
        if (!trans) {
            *reinterpret_cast<u32x4*>(&T[q >> 2][(q & 3) * 8]) = v;
        } else {
            const int kr = q & 31, o = (q >> 5) * 8;
#pragma unroll
            for (int i = 0; i < 8; ++i) T[o + i][kr] = (bf16_t)(v[i >> 1] >> (16 * (i & 1)));
        }
    };
    f32x16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
    u32x4 va[WM], vb[WN];
#pragma unroll
    for (int g = 0; g < WM; ++g) va[g] = load_a(0, g);
#pragma unroll
    for (int g = 0; g < WN; ++g) vb[g] = load_b(0, g);
#pragma unroll
    for (int g = 0; g < WM; ++g) store(As[0], TA, g, va[g]);
#pragma unroll
    for (int g = 0; g < WN; ++g) store(Bs[0], !TB, g, vb[g]);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += BK) {
        const bool more = k0 + BK < K;
        if (more) {
#pragma unroll
            for (int g = 0; g < WM; ++g) va[g] = load_a(k0 + BK, g);
#pragma unroll
            for (int g = 0; g < WN; ++g) vb[g] = load_b(k0 + BK, g);
        }
#pragma unroll
        for (int kb = 0; kb < BK; kb += 16) {
            const int r = lane & 31, kq = kb + (lane >> 5) * 8;
            bf16x8 a[WM], b[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i)
                a[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wm * 32 * WM + i * 32 + r][kq]);
#pragma unroll
            for (int j = 0; j < WN; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn * 32 * WN + j * 32 + r][kq]);
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) {
#pragma unroll
            for (int g = 0; g < WM; ++g) store(As[buf ^ 1], TA, g, va[g]);
#pragma unroll
            for (int g = 0; g < WN; ++g) store(Bs[buf ^ 1], !TB, g, vb[g]);
        }
        __syncthreads();
        buf ^= 1;
    }
    // lane l holds column l%32, rows 8*(v/4) + 4*(l/32) + v%4 of each 32x32 block
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            const int col = n0 + wn * 32 * WN + j * 32 + (lane & 31);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = m0 + wm * 32 * WM + i * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
                if (row < M && col < N) {
                    float* c = C + (size_t)row * ldc + col;
                    *c = beta == 0.0f ? alpha * acc[i][j][v] : alpha * acc[i][j][v] + beta * *c;
                }
            }
        }
}

__global__ void k_cast_bf16(const float* __restrict__ x, bf16_t* __restrict__ y, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = to_bf16(x[i]);
}

// instance index of every row from offsets seg[B+1]
__global__ void k_row_inst(const int* __restrict__ seg, int B, int* __restrict__ inst) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B)
        for (int r = seg[b]; r < seg[b + 1]; ++r) inst[r] = b;
}

// h = x W_e + b_e with W_e in BF16 (K = d_in is small: plain FMA)
__global__ void k_embed(const float* __restrict__ x, const bf16_t* __restrict__ We, const float* __restrict__ be,
                        float* __restrict__ h, bf16_t* __restrict__ hb, int R, int d_in, int W) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)R * W) return;
    const int r = (int)(i / W), c = (int)(i - (long long)r * W);
    float acc = be[c];
    for (int j = 0; j < d_in; ++j) acc += x[(size_t)r * d_in + j] * from_bf16(We[(size_t)j * W + c]);
    h[i] = acc;
    hb[i] = to_bf16(acc);
}

// z += b (in place), a = bf16(relu(z))
__global__ void k_bias_relu(float* __restrict__ z, const float* __restrict__ b, bf16_t* __restrict__ a, int R, int H) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)R * H) return;
    const int c = (int)(i % H);
    const float v = z[i] + b[c];
    z[i] = v;
    a[i] = to_bf16(fmaxf(v, 0.0f));
}

// per-instance mean (mean = true) or sum of rows; one thread per (instance, column)
__global__ void k_segment_reduce(const float* __restrict__ x, const int* __restrict__ seg, float* __restrict__ out,
                                 bf16_t* __restrict__ outb, int B, int W, int mean) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)B * W) return;
    const int b = (int)(i / W), c = (int)(i - (long long)b * W);
    const int r0 = seg[b], r1 = seg[b + 1];
    float s = 0.0f;
    for (int r = r0; r < r1; ++r) s += x[(size_t)r * W + c];
    if (mean) s /= (float)max(r1 - r0, 1);
    if (out) out[i] = s;
    outb[i] = to_bf16(s);
}

// h_next = h + z2 + b2 + q[inst]
__global__ void k_residual(const float* __restrict__ h, const float* __restrict__ z2, const float* __restrict__ b2,
                           const float* __restrict__ q, const int* __restrict__ inst, float* __restrict__ hn,
                           bf16_t* __restrict__ hnb, int R, int W) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)R * W) return;
    const int r = (int)(i / W), c = (int)(i - (long long)r * W);
    const float v = h[i] + z2[i] + b2[c] + q[(size_t)inst[r] * W + c];
    hn[i] = v;
    hnb[i] = to_bf16(v);
}

__global__ void k_add_bias(float* __restrict__ y, const float* __restrict__ b, int R, int N) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (long long)R * N) y[i] += b[i % N];
}

// dy = mask (y - t) / (N sum(mask)); per-block partial loss sums (FP32)
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             const float* __restrict__ mask, const float* __restrict__ msum,
                                             float* __restrict__ dy, bf16_t* __restrict__ dyb,
                                             float* __restrict__ partial, int R, int N) {
    __shared__ float red[256];
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (i < (long long)R * N) {
        const int r = (int)(i / N);
        const float cnt = (float)N * fmaxf(*msum, 1.0f);
        const float d = (y[i] - t[i]) * mask[r];
        l = d * (y[i] - t[i]);
        const float g = d / cnt;
        dy[i] = g;
        dyb[i] = to_bf16(g);
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_sum_partials(const float* __restrict__ partial, int n, float scale,
                                                      float* __restrict__ out) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// loss = sum(partial) / (2 N sum(mask))
__global__ void __launch_bounds__(256) k_loss_final(const float* __restrict__ partial, int n, int N,
                                                    const float* __restrict__ msum, float* __restrict__ out) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] / (2.0f * (float)N * fmaxf(*msum, 1.0f));
}

// Column reductions over all rows, parallel over rows: a workgroup of 256
// lanes takes 16 columns, lane (q, c) sums rows q, q + 16, ... of column c,
// and the 16 partial sums are added in a fixed order, so results do not
// depend on timing.  COLS_PER_GROUP columns per workgroup.
constexpr int COLS_PER_GROUP = 16, ROW_LANES = 16;

// out[c] = sum_r x[r][c]
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ x, float* __restrict__ out, int R, int N) {
    __shared__ float part[ROW_LANES][COLS_PER_GROUP];
    const int cl = threadIdx.x % COLS_PER_GROUP, q = threadIdx.x / COLS_PER_GROUP;
    const int c = blockIdx.x * COLS_PER_GROUP + cl;
    float s = 0.0f;
    if (c < N)
        for (int r = q; r < R; r += ROW_LANES) s += x[(size_t)r * N + c];
    part[q][cl] = s;
    __syncthreads();
    if (q == 0 && c < N) {
        float t = 0.0f;
        for (int i = 0; i < ROW_LANES; ++i) t += part[i][cl];
        out[c] = t;
    }
}

// dz = da * (z > 0), in place on da, plus its BF16 copy
__global__ void k_relu_bwd(float* __restrict__ da, const float* __restrict__ z, bf16_t* __restrict__ dzb, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = z[i] > 0.0f ? da[i] : 0.0f;
    da[i] = v;
    dzb[i] = to_bf16(v);
}

// dh[r] += dpm[inst r] / n_inst
__global__ void k_pool_bwd(float* __restrict__ dh, const float* __restrict__ dpm, const int* __restrict__ inst,
                           const int* __restrict__ seg, int R, int W) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)R * W) return;
    const int r = (int)(i / W), c = (int)(i - (long long)r * W);
    const int b = inst[r];
    dh[i] += dpm[(size_t)b * W + c] / (float)(seg[b + 1] - seg[b]);
}

// gWe[j][c] = sum_r x[r][j] dh[r][c], for d_in <= MAX_D_IN, rows in parallel as
// in k_colsum (the partial sums of the 16 row lanes added in a fixed order)
constexpr int MAX_D_IN = 8;
__global__ void __launch_bounds__(256) k_embed_grad(const float* __restrict__ x, const float* __restrict__ dh,
                                                    float* __restrict__ g, int R, int d_in, int W) {
    __shared__ float part[MAX_D_IN][ROW_LANES][COLS_PER_GROUP];
    const int cl = threadIdx.x % COLS_PER_GROUP, q = threadIdx.x / COLS_PER_GROUP;
    const int c = blockIdx.x * COLS_PER_GROUP + cl;
    float s[MAX_D_IN];
#pragma unroll
    for (int j = 0; j < MAX_D_IN; ++j) s[j] = 0.0f;
    if (c < W)
        for (int r = q; r < R; r += ROW_LANES) {
            const float d = dh[(size_t)r * W + c];
#pragma unroll
            for (int j = 0; j < MAX_D_IN; ++j)
                if (j < d_in) s[j] += x[(size_t)r * d_in + j] * d;
        }
#pragma unroll
    for (int j = 0; j < MAX_D_IN; ++j) part[j][q][cl] = s[j];
    __syncthreads();
    if (q == 0 && c < W)
        for (int j = 0; j < d_in; ++j) {
            float t = 0.0f;
            for (int i = 0; i < ROW_LANES; ++i) t += part[j][i][cl];
            g[(size_t)j * W + c] = t;
        }
}

// Adam with bias correction on FP32 master weights, then their BF16 copy
__global__ void k_adam(float* __restrict__ w, bf16_t* __restrict__ wb, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = to_bf16(wi);
}

__global__ void k_zero(float* __restrict__ p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

}  // namespace d4p
