// Host side of the learned proposal (d4p_* in include/d4.h): parameter
// layout, workspace, forward, backward and Adam training steps, every step
// running in the kernels of d4_proposal_kernels.hpp.
#include "d4.h"
#include "d4_host.hpp"
#include "d4_proposal_kernels.hpp"

using namespace d4host;
using namespace d4p;

struct d4p_net {
    d4p_config cfg;
    int device;
    long long n_params;
    // parameter offsets (floats) into the flat arrays
    long long oWe, obe, oWh, obh;
    std::vector<long long> oW1, ob1, oW2, ob2, oWp;
    float *w, *g, *m, *v;
    bf16_t* wb;
    int adam_t;
    // workspace
    int* inst;
    float *h, *z1, *z2, *q, *y, *dy, *dh0, *dh1, *da1, *dpm, *partial, *msum, *loss;
    bf16_t *hb, *a1b, *pmb, *dyb, *dhb, *dz1b, *dqb;
};

namespace {

inline unsigned blocks(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// 128x128 tiles when they still give at least 256 workgroups (one per CU),
// else 64x64; D4_OPT_GEMM_TILE fixes either (the results are the same bits)
template <bool TA, bool TB>
int gemm(const bf16_t* A, const bf16_t* B, float* C, int M, int N, int K, int lda, int ldb, int ldc, float beta,
         hipStream_t st) {
    if (M <= 0 || N <= 0) return D4_OK;
    int tile = g_opt_gemm_tile.load();
    if (tile == 0) tile = (long long)((M + 127) / 128) * ((N + 127) / 128) >= 256 ? 128 : 64;
    if (tile == 128) {
        const dim3 grid((N + 127) / 128, (M + 127) / 128);
        hipLaunchKernelGGL((k_gemm_bf16<TA, TB, 2, 2>), grid, dim3(256), 0, st, A, B, C, M, N, K, lda, ldb, ldc,
                           1.0f, beta);
    } else {
        const dim3 grid((N + 63) / 64, (M + 63) / 64);
        hipLaunchKernelGGL((k_gemm_bf16<TA, TB, 1, 1>), grid, dim3(256), 0, st, A, B, C, M, N, K, lda, ldb, ldc,
                           1.0f, beta);
    }
    HIP_LAUNCH_CHECK("k_gemm_bf16");
    return D4_OK;
}

#define TRY(x)              \
    do {                    \
        int rc_ = (x);      \
        if (rc_) return rc_; \
    } while (0)

// splitmix64: host-side initialisation stream
uint64_t mix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int check_rows(const d4p_net* n, int rows, int batch) {
    if (rows < 1 || rows > n->cfg.max_rows) return fail(D4_EINVAL, "rows %d outside 1..%d", rows, n->cfg.max_rows);
    if (batch < 1 || batch > n->cfg.max_batch)
        return fail(D4_EINVAL, "batch %d outside 1..%d", batch, n->cfg.max_batch);
    return D4_OK;
}

int forward_impl(d4p_net* n, const float* x, const int* seg, int R, int B, hipStream_t st) {
    const d4p_config& c = n->cfg;
    const int W = c.width, H = c.hidden, L = c.layers;
    const long long RW = (long long)R * W, RH = (long long)R * H;
    hipLaunchKernelGGL(k_row_inst, dim3(blocks(B)), dim3(256), 0, st, seg, B, n->inst);
    hipLaunchKernelGGL(k_embed, dim3(blocks(RW)), dim3(256), 0, st, x, n->wb + n->oWe, n->w + n->obe, n->h, n->hb,
                       R, c.d_in, W);
    HIP_LAUNCH_CHECK("k_embed");
    for (int l = 0; l < L; ++l) {
        const float* h = n->h + (size_t)l * c.max_rows * W;
        const bf16_t* hb = n->hb + (size_t)l * c.max_rows * W;
        float* z1 = n->z1 + (size_t)l * c.max_rows * H;
        bf16_t* a1b = n->a1b + (size_t)l * c.max_rows * H;
        bf16_t* pmb = n->pmb + (size_t)l * c.max_batch * W;
        TRY((gemm<false, false>(hb, n->wb + n->oW1[l], z1, R, H, W, W, H, H, 0.0f, st)));
        hipLaunchKernelGGL(k_bias_relu, dim3(blocks(RH)), dim3(256), 0, st, z1, n->w + n->ob1[l], a1b, R, H);
        TRY((gemm<false, false>(a1b, n->wb + n->oW2[l], n->z2, R, W, H, H, W, W, 0.0f, st)));
        hipLaunchKernelGGL(k_segment_reduce, dim3(blocks((long long)B * W)), dim3(256), 0, st, h, seg,
                           (float*)nullptr, pmb, B, W, 1);
        TRY((gemm<false, false>(pmb, n->wb + n->oWp[l], n->q, B, W, W, W, W, W, 0.0f, st)));
        hipLaunchKernelGGL(k_residual, dim3(blocks(RW)), dim3(256), 0, st, h, n->z2, n->w + n->ob2[l], n->q,
                           n->inst, n->h + (size_t)(l + 1) * c.max_rows * W, n->hb + (size_t)(l + 1) * c.max_rows * W,
                           R, W);
        HIP_LAUNCH_CHECK("k_residual");
    }
    const bf16_t* hL = n->hb + (size_t)L * c.max_rows * W;
    TRY((gemm<false, false>(hL, n->wb + n->oWh, n->y, R, c.d_out, W, W, c.d_out, c.d_out, 0.0f, st)));
    hipLaunchKernelGGL(k_add_bias, dim3(blocks((long long)R * c.d_out)), dim3(256), 0, st, n->y, n->w + n->obh, R,
                       c.d_out);
    HIP_LAUNCH_CHECK("k_add_bias");
    return D4_OK;
}

int backward_impl(d4p_net* n, const float* x, const int* seg, const float* target, const float* mask, int R, int B,
                  hipStream_t st) {
    const d4p_config& c = n->cfg;
    const int W = c.width, H = c.hidden, L = c.layers, N = c.d_out;
    const long long RW = (long long)R * W, RH = (long long)R * H, RN = (long long)R * N;
    // loss and dL/dy
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, mask, R, 1.0f, n->msum);
    hipLaunchKernelGGL(k_mse, dim3(blocks(RN)), dim3(256), 0, st, n->y, target, mask, n->msum, n->dy, n->dyb,
                       n->partial, R, N);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, n->partial, (int)blocks(RN), N, n->msum, n->loss);
    HIP_LAUNCH_CHECK("k_loss_final");
    // head
    const bf16_t* hL = n->hb + (size_t)L * c.max_rows * W;
    TRY((gemm<true, false>(hL, n->dyb, n->g + n->oWh, W, N, R, W, N, N, 0.0f, st)));
    hipLaunchKernelGGL(k_colsum, dim3(blocks(N, COLS_PER_GROUP)), dim3(256), 0, st, n->dy, n->g + n->obh, R, N);
    float* dh = n->dh0;
    float* dhn = n->dh1;
    TRY((gemm<false, true>(n->dyb, n->wb + n->oWh, dh, R, W, N, N, N, W, 0.0f, st)));
    for (int l = L - 1; l >= 0; --l) {
        const bf16_t* hb = n->hb + (size_t)l * c.max_rows * W;
        const float* z1 = n->z1 + (size_t)l * c.max_rows * H;
        const bf16_t* a1b = n->a1b + (size_t)l * c.max_rows * H;
        const bf16_t* pmb = n->pmb + (size_t)l * c.max_batch * W;
        hipLaunchKernelGGL(k_cast_bf16, dim3(blocks(RW)), dim3(256), 0, st, dh, n->dhb, RW);
        // branch relu(h W1 + b1) W2 + b2
        TRY((gemm<true, false>(a1b, n->dhb, n->g + n->oW2[l], H, W, R, H, W, W, 0.0f, st)));
        hipLaunchKernelGGL(k_colsum, dim3(blocks(W, COLS_PER_GROUP)), dim3(256), 0, st, dh, n->g + n->ob2[l], R, W);
        TRY((gemm<false, true>(n->dhb, n->wb + n->oW2[l], n->da1, R, H, W, W, W, H, 0.0f, st)));
        hipLaunchKernelGGL(k_relu_bwd, dim3(blocks(RH)), dim3(256), 0, st, n->da1, z1, n->dz1b, RH);
        TRY((gemm<true, false>(hb, n->dz1b, n->g + n->oW1[l], W, H, R, W, H, H, 0.0f, st)));
        hipLaunchKernelGGL(k_colsum, dim3(blocks(H, COLS_PER_GROUP)), dim3(256), 0, st, n->da1, n->g + n->ob1[l], R, H);
        HIP_TRY(hipMemcpyAsync(dhn, dh, sizeof(float) * RW, hipMemcpyDeviceToDevice, st));
        TRY((gemm<false, true>(n->dz1b, n->wb + n->oW1[l], dhn, R, W, H, H, H, W, 1.0f, st)));
        // pool mean_b(h) Wp
        hipLaunchKernelGGL(k_segment_reduce, dim3(blocks((long long)B * W)), dim3(256), 0, st, dh, seg,
                           (float*)nullptr, n->dqb, B, W, 0);
        TRY((gemm<true, false>(pmb, n->dqb, n->g + n->oWp[l], W, W, B, W, W, W, 0.0f, st)));
        TRY((gemm<false, true>(n->dqb, n->wb + n->oWp[l], n->dpm, B, W, W, W, W, W, 0.0f, st)));
        hipLaunchKernelGGL(k_pool_bwd, dim3(blocks(RW)), dim3(256), 0, st, dhn, n->dpm, n->inst, seg, R, W);
        HIP_LAUNCH_CHECK("k_pool_bwd");
        std::swap(dh, dhn);
    }
    hipLaunchKernelGGL(k_embed_grad, dim3(blocks(W, COLS_PER_GROUP)), dim3(256), 0, st, x, dh, n->g + n->oWe, R,
                       c.d_in, W);
    hipLaunchKernelGGL(k_colsum, dim3(blocks(W, COLS_PER_GROUP)), dim3(256), 0, st, dh, n->g + n->obe, R, W);
    HIP_LAUNCH_CHECK("k_colsum");
    return D4_OK;
}

void free_net(d4p_net* n) {
    void* ptrs[] = {n->w,   n->g,  n->m,  n->v,   n->wb,  n->inst, n->h,    n->z1,   n->z2,  n->q,
                    n->y,   n->dy, n->dh0, n->dh1, n->da1, n->dpm, n->partial, n->msum, n->loss, n->hb,
                    n->a1b, n->pmb, n->dyb, n->dhb, n->dz1b, n->dqb};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

}  // namespace

extern "C" {

int32_t d4p_create(const d4p_config* cfg, d4p_net** out) {
    if (!cfg || !out) return fail(D4_EINVAL, "config or out-pointer is NULL");
    const d4p_config& c = *cfg;
    if (c.d_in < 1 || c.width < 1 || c.hidden < 1 || c.layers < 0 || c.d_out < 1 || c.max_rows < 1 ||
        c.max_batch < 1 || c.layers > 64)
        return fail(D4_EINVAL, "bad network shape");
    if (c.d_in > MAX_D_IN) return fail(D4_EUNSUPPORTED, "d_in %d above %d", c.d_in, MAX_D_IN);
    d4p_net* n = new (std::nothrow) d4p_net();
    if (!n) return fail(D4_ENOMEM, "host allocation failed");
    n->cfg = c;
    HIP_TRY(hipGetDevice(&n->device));
    const long long W = c.width, H = c.hidden, Din = c.d_in, Dout = c.d_out;
    long long o = 0;
    n->oWe = o; o += Din * W;
    n->obe = o; o += W;
    for (int l = 0; l < c.layers; ++l) {
        n->oW1.push_back(o); o += W * H;
        n->ob1.push_back(o); o += H;
        n->oW2.push_back(o); o += H * W;
        n->ob2.push_back(o); o += W;
        n->oWp.push_back(o); o += W * W;
    }
    n->oWh = o; o += W * Dout;
    n->obh = o; o += Dout;
    n->n_params = o;
    const size_t R = c.max_rows, B = c.max_batch, L = c.layers;
    const size_t nparts = (R * Dout + 255) / 256 + 1;
    struct {
        void** ptr;
        size_t bytes;
    } allocs[] = {
        {(void**)&n->w, 4 * (size_t)o},           {(void**)&n->g, 4 * (size_t)o},
        {(void**)&n->m, 4 * (size_t)o},           {(void**)&n->v, 4 * (size_t)o},
        {(void**)&n->wb, 2 * (size_t)o},          {(void**)&n->inst, 4 * R},
        {(void**)&n->h, 4 * (L + 1) * R * W},     {(void**)&n->hb, 2 * (L + 1) * R * W},
        {(void**)&n->z1, 4 * std::max<size_t>(L, 1) * R * H}, {(void**)&n->a1b, 2 * std::max<size_t>(L, 1) * R * H},
        {(void**)&n->pmb, 2 * std::max<size_t>(L, 1) * B * W}, {(void**)&n->z2, 4 * R * W},
        {(void**)&n->q, 4 * B * W},               {(void**)&n->y, 4 * R * Dout},
        {(void**)&n->dy, 4 * R * Dout},           {(void**)&n->dyb, 2 * R * Dout},
        {(void**)&n->dh0, 4 * R * W},             {(void**)&n->dh1, 4 * R * W},
        {(void**)&n->dhb, 2 * R * W},             {(void**)&n->da1, 4 * R * H},
        {(void**)&n->dz1b, 2 * R * H},            {(void**)&n->dqb, 2 * B * W},
        {(void**)&n->dpm, 4 * B * W},             {(void**)&n->partial, 4 * nparts},
        {(void**)&n->msum, 4},                    {(void**)&n->loss, 4},
    };
    for (auto& a : allocs) {
        if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
            free_net(n);
            delete n;
            return fail(D4_ENOMEM, "hipMalloc of %zu bytes failed", a.bytes);
        }
    }
    // uniform(+-1/sqrt(fan_in)) weights, zero biases
    std::vector<float> w(o, 0.0f);
    uint64_t s = c.seed;
    auto fill = [&](long long off, long long rows, long long cols) {
        const double lim = 1.0 / std::sqrt((double)rows);
        for (long long i = 0; i < rows * cols; ++i) {
            const double u = (double)(mix(s) >> 11) * (1.0 / 9007199254740992.0);
            w[off + i] = (float)((2.0 * u - 1.0) * lim);
        }
    };
    fill(n->oWe, Din, W);
    for (int l = 0; l < c.layers; ++l) {
        fill(n->oW1[l], W, H);
        fill(n->oW2[l], H, W);
        fill(n->oWp[l], W, W);
    }
    fill(n->oWh, W, Dout);
    if (hipMemcpy(n->w, w.data(), 4 * (size_t)o, hipMemcpyHostToDevice) != hipSuccess) {
        free_net(n);
        delete n;
        return fail(D4_EHIP, "parameter upload failed");
    }
    hipLaunchKernelGGL(k_cast_bf16, dim3(blocks(o)), dim3(256), 0, 0, n->w, n->wb, (long long)o);
    hipLaunchKernelGGL(k_zero, dim3(blocks(o)), dim3(256), 0, 0, n->m, (long long)o);
    hipLaunchKernelGGL(k_zero, dim3(blocks(o)), dim3(256), 0, 0, n->v, (long long)o);
    if (hipDeviceSynchronize() != hipSuccess) {
        free_net(n);
        delete n;
        return fail(D4_EHIP, "parameter set-up failed");
    }
    *out = n;
    return D4_OK;
}

int32_t d4p_num_params(const d4p_net* n, int64_t* count) {
    if (!n || !count) return fail(D4_EINVAL, "NULL argument");
    *count = n->n_params;
    return D4_OK;
}

int32_t d4p_set_params(d4p_net* n, const float* params, void* stream) {
    if (!n) return fail(D4_EINVAL, "net is NULL");
    NEED(params);
    hipStream_t st = (hipStream_t)stream;
    const long long P = n->n_params;
    HIP_TRY(hipMemcpyAsync(n->w, params, 4 * (size_t)P, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_cast_bf16, dim3(blocks(P)), dim3(256), 0, st, n->w, n->wb, P);
    hipLaunchKernelGGL(k_zero, dim3(blocks(P)), dim3(256), 0, st, n->m, P);
    hipLaunchKernelGGL(k_zero, dim3(blocks(P)), dim3(256), 0, st, n->v, P);
    HIP_LAUNCH_CHECK("k_zero");
    n->adam_t = 0;
    return D4_OK;
}

int32_t d4p_get_params(const d4p_net* n, float* params, void* stream) {
    if (!n) return fail(D4_EINVAL, "net is NULL");
    NEED(params);
    HIP_TRY(hipMemcpyAsync(params, n->w, 4 * (size_t)n->n_params, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return D4_OK;
}

int32_t d4p_forward(d4p_net* n, const float* x, const int32_t* seg, int32_t rows, int32_t batch, float* y,
                    void* stream) {
    if (!n) return fail(D4_EINVAL, "net is NULL");
    NEED(x);
    NEED(seg);
    NEED(y);
    int rc = check_rows(n, rows, batch);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    rc = forward_impl(n, x, seg, rows, batch, st);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(y, n->y, 4 * (size_t)rows * n->cfg.d_out, hipMemcpyDeviceToDevice, st));
    return D4_OK;
}

int32_t d4p_gradients(d4p_net* n, const float* x, const int32_t* seg, int32_t rows, int32_t batch,
                      const float* target, const float* mask, float* loss, float* grads, void* stream) {
    if (!n) return fail(D4_EINVAL, "net is NULL");
    NEED(x);
    NEED(seg);
    NEED(target);
    NEED(mask);
    int rc = check_rows(n, rows, batch);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    rc = forward_impl(n, x, seg, rows, batch, st);
    if (!rc) rc = backward_impl(n, x, seg, target, mask, rows, batch, st);
    if (rc) return rc;
    if (loss) HIP_TRY(hipMemcpyAsync(loss, n->loss, 4, hipMemcpyDeviceToDevice, st));
    if (grads) HIP_TRY(hipMemcpyAsync(grads, n->g, 4 * (size_t)n->n_params, hipMemcpyDeviceToDevice, st));
    return D4_OK;
}

int32_t d4p_train_step(d4p_net* n, const float* x, const int32_t* seg, int32_t rows, int32_t batch,
                       const float* target, const float* mask, float lr, float* loss, void* stream) {
    int rc = d4p_gradients(n, x, seg, rows, batch, target, mask, loss, nullptr, stream);
    if (rc) return rc;
    if (!(lr > 0.0f)) return fail(D4_EINVAL, "learning rate must be positive");
    n->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, n->adam_t));
    const float c2 = (float)(1.0 - std::pow(0.999, n->adam_t));
    const long long P = n->n_params;
    hipLaunchKernelGGL(k_adam, dim3(blocks(P)), dim3(256), 0, (hipStream_t)stream, n->w, n->wb, n->g, n->m, n->v, P,
                       lr, b1, b2, 1e-8f, c1, c2);
    HIP_LAUNCH_CHECK("k_adam");
    return D4_OK;
}

int32_t d4p_gemm_bf16(int32_t trans_a, int32_t trans_b, const uint16_t* A, const uint16_t* B, float* C, int32_t M,
                      int32_t N, int32_t K, int32_t lda, int32_t ldb, int32_t ldc, float beta, void* stream) {
    if (!A || !B || !C) return fail(D4_EINVAL, "NULL operand");
    if (M < 0 || N < 0 || K < 0 || lda < 1 || ldb < 1 || ldc < 1) return fail(D4_EINVAL, "bad GEMM shape");
    if ((!trans_a && lda < K) || (trans_a && lda < M) || (!trans_b && ldb < N) || (trans_b && ldb < K) || ldc < N)
        return fail(D4_EINVAL, "leading dimension smaller than the row length");
    hipStream_t st = (hipStream_t)stream;
    const bf16_t* a = reinterpret_cast<const bf16_t*>(A);
    const bf16_t* b = reinterpret_cast<const bf16_t*>(B);
    if (!trans_a && !trans_b) return gemm<false, false>(a, b, C, M, N, K, lda, ldb, ldc, beta, st);
    if (!trans_a && trans_b) return gemm<false, true>(a, b, C, M, N, K, lda, ldb, ldc, beta, st);
    if (trans_a && !trans_b) return gemm<true, false>(a, b, C, M, N, K, lda, ldb, ldc, beta, st);
    return gemm<true, true>(a, b, C, M, N, K, lda, ldb, ldc, beta, st);
}

int32_t d4p_destroy(d4p_net* n) {
    if (!n) return D4_OK;
    (void)hipDeviceSynchronize();
    free_net(n);
    delete n;
    return D4_OK;
}

}  // extern "C"
