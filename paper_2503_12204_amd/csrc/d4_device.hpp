// Device math of the denoising hot path (gfx950, wave64).
//
//  - Counter-based normal draws for the sampling step of Algorithm 1
//    (Eq. mc): Philox4x32-10 (Salmon et al., SC'11) feeding a Box-Muller
//    transform whose ln and sin/cos are evaluated in FP32 one correctly
//    rounded operation (or fused multiply-add) at a time, in a fixed order
//    with no other contraction, so the draws are the same bits on every
//    implementation of the recipe.
//  - RK4 steps of the three robot models (Section III feasibility condition,
//    Section V models).  The double integrator's RK4 step is evaluated in
//    its exact closed form p + v dt + a dt^2/2, v + a dt (RK4 is exact when
//    A^2 = 0); the unicycle's RK4 step is evaluated as Simpson's rule on the
//    heading, which is what the four stages reduce to when theta is linear
//    in time, with the end-of-step sine/cosine reused as the next step's
//    first stage.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace d4 {

enum { HOLO2D = 0, HOLO3D = 1, UNICYCLE = 2, DIFFDRIVE = 3 };
constexpr int MAX_OBS = 16;   // static obstacles per problem
enum { FLAG_NORMALIZE = 1, FLAG_SAFE_PAIRS = 2 };

// ---------------------------------------------------- uniform values in VGPRs
// A VALU instruction that reads an SGPR operand issues in 4 cycles on gfx950,
// but one whose sources are all VGPRs (or inline constants) can pair with
// another wave's instruction and issue in about 2.5 (a probe of ours: FP32
// add and multiply, 4.4 against 2.45 cycles per wave64).  The hot loops
// therefore take their uniform operands from VGPR copies.  The empty asm
// ties the value to a VGPR and hides its origin, so the optimiser neither
// folds it back to the scalar register nor rematerialises it there.
__device__ __forceinline__ float vgpr_copy(float x) {
    float r;
    asm volatile("" : "=v"(r) : "0"(x));
    return r;
}
__device__ __forceinline__ uint32_t vgpr_copy(uint32_t x) {
    uint32_t r;
    asm volatile("" : "=v"(r) : "0"(x));
    return r;
}

// ------------------------------------------------------------------ Philox
// The constants of Philox4x32-10 under one key: the two round multipliers
// and the ten round keys (the key advanced by the Weyl constants), in VGPRs
// when IN_VGPRS.
struct PhiloxKey {
    uint32_t m0, m1, k0[10], k1[10];
    template <bool IN_VGPRS>
    __device__ __forceinline__ static PhiloxKey make(uint32_t key0, uint32_t key1) {
        PhiloxKey pk;
        pk.m0 = 0xD2511F53u;
        pk.m1 = 0xCD9E8D57u;
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            pk.k0[r] = key0 + (uint32_t)r * 0x9E3779B9u;
            pk.k1[r] = key1 + (uint32_t)r * 0xBB67AE85u;
        }
        if (IN_VGPRS) {
            pk.m0 = vgpr_copy(pk.m0);
            pk.m1 = vgpr_copy(pk.m1);
#pragma unroll
            for (int r = 0; r < 10; ++r) {
                pk.k0[r] = vgpr_copy(pk.k0[r]);
                pk.k1[r] = vgpr_copy(pk.k1[r]);
            }
        }
        return pk;
    }
};

// Philox4x32-10 on G independent counter blocks under one key.  The rounds
// run in lockstep across the blocks: each round is a short dependent chain
// (two 32x32->64 products feeding two three-input XORs), so interleaving
// the blocks keeps 2G products in flight instead of two.
template <int G>
__device__ __forceinline__ void philox4x32_10_n(uint32_t (&c)[G][4], const PhiloxKey& pk) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t k0 = pk.k0[r], k1 = pk.k1[r];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const uint64_t p0 = (uint64_t)pk.m0 * c[q][0];
            const uint64_t p1 = (uint64_t)pk.m1 * c[q][2];
            const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
            const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
            // three-input XORs (truth table 0x96) in one gfx950 instruction each
            const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c[q][1], k0, 0x96);
            const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c[q][3], k1, 0x96);
            c[q][0] = n0;
            c[q][1] = lo1;
            c[q][2] = n2;
            c[q][3] = lo0;
        }
    }
}

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
    uint32_t c[1][4] = {{c0, c1, c2, c3}};
    philox4x32_10_n<1>(c, PhiloxKey::make<false>(k0, k1));
    c0 = c[0][0];
    c1 = c[0][1];
    c2 = c[0][2];
    c3 = c[0][3];
}

// ------------------------------------------------ FP32 ln and sin/cos recipe
// Each function below works on P independent operands, one operation at a
// time across all of them (the per-operand sequence does not depend on P),
// so that P dependent chains are in flight together.

// Correctly rounded a / b for the operands of ln_unit (a in [-0.25, 0.5],
// b in [1.75, 2.5]): one Newton-Raphson refinement of the hardware
// reciprocal, then two quotient corrections from the exact FMA residual
// a - b q (Markstein, IBM J. Res. Dev. 34(1), 1990).  No range scaling or
// special-value handling is needed for finite operands of moderate exponent.
// Every reachable operand pair is checked against the correctly rounded
// quotient by the exhaustive transform test.
template <int P>
__device__ __forceinline__ void div_rn_moderate_n(const float (&a)[P], const float (&b)[P], float (&out)[P]) {
    float y[P], e[P], q[P], r[P];
#pragma unroll
    for (int i = 0; i < P; ++i) y[i] = __builtin_amdgcn_rcpf(b[i]);
#pragma unroll
    for (int i = 0; i < P; ++i) e[i] = __builtin_fmaf(-b[i], y[i], 1.0f);
#pragma unroll
    for (int i = 0; i < P; ++i) y[i] = __builtin_fmaf(e[i], y[i], y[i]);
#pragma unroll
    for (int i = 0; i < P; ++i) q[i] = a[i] * y[i];
#pragma unroll
    for (int i = 0; i < P; ++i) r[i] = __builtin_fmaf(-b[i], q[i], a[i]);
#pragma unroll
    for (int i = 0; i < P; ++i) q[i] = __builtin_fmaf(r[i], y[i], q[i]);
#pragma unroll
    for (int i = 0; i < P; ++i) r[i] = __builtin_fmaf(-b[i], q[i], a[i]);
#pragma unroll
    for (int i = 0; i < P; ++i) out[i] = __builtin_fmaf(r[i], y[i], q[i]);
}

__device__ __forceinline__ float div_rn_moderate(float a, float b) {
    const float av[1] = {a}, bv[1] = {b};
    float q[1];
    div_rn_moderate_n<1>(av, bv, q);
    return q[0];
}

// Correctly rounded sqrt(x) for finite normal x > 0 away from the denormal
// range: the hardware estimate (within 1 ulp) is moved to a neighbour when the
// exact FMA residual x - s' s says that the neighbour is nearer (the residual
// test of Markstein's method).
template <int P>
__device__ __forceinline__ void sqrt_rn_normal_n(const float (&x)[P], float (&out)[P]) {
    float sq[P];
#pragma unroll
    for (int i = 0; i < P; ++i) sq[i] = __builtin_amdgcn_sqrtf(x[i]);
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const float s = sq[i];
        const float s_dn = __uint_as_float(__float_as_uint(s) - 1u);
        const float s_up = __uint_as_float(__float_as_uint(s) + 1u);
        const float r_dn = __builtin_fmaf(-s_dn, s, x[i]);
        const float r_up = __builtin_fmaf(-s_up, s, x[i]);
        const float o = r_dn <= 0.0f ? s_dn : s;
        out[i] = r_up > 0.0f ? s_up : o;
    }
}

__device__ __forceinline__ float sqrt_rn_normal(float x) {
    const float xv[1] = {x};
    float o[1];
    sqrt_rn_normal_n<1>(xv, o);
    return o[0];
}

// Natural log of a uniform in (0, 1): u = 2^e f, f in [0.75, 1.5),
// ln f = 2 atanh(s), s = (f - 1)/(f + 1), atanh by its Taylor series in
// fused Horner form through s^9, e*ln2 split as 355/512 (exact products
// with e) plus the FP32 remainder.
// Within 2 ulp of ln u for every uniform the recipe produces.
template <int P>
__device__ __forceinline__ void ln_unit_n(const float (&u)[P], float (&out)[P]) {
#pragma clang fp contract(off)
    const float A3 = 1.0f / 3.0f, A5 = 1.0f / 5.0f, A7 = 1.0f / 7.0f, A9 = 1.0f / 9.0f;
    const float LN2_HI = 355.0f / 512.0f;
    const float LN2_LO = (float)(0.693147180559945309417232121458 - 355.0 / 512.0);
    float num[P], den[P], ef[P], s[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const uint32_t b = __float_as_uint(u[i]);
        int e = (int)(b >> 23) - 127;
        float f = __uint_as_float((b & 0x7FFFFFu) | 0x3F800000u);
        const bool big = f >= 1.5f;
        f = big ? f * 0.5f : f;
        e += big ? 1 : 0;
        num[i] = f - 1.0f;
        den[i] = f + 1.0f;
        ef[i] = (float)e;
    }
    div_rn_moderate_n<P>(num, den, s);
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const float s2 = s[i] * s[i];
        const float q = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(A9, s2, A7), s2, A5), s2, A3);
        const float t = __builtin_fmaf(s[i] * s2, q, s[i]);
        out[i] = __builtin_fmaf(ef[i], LN2_HI, __builtin_fmaf(ef[i], LN2_LO, 2.0f * t));
    }
}

__device__ __forceinline__ float ln_unit(float u) {
    const float uv[1] = {u};
    float o[1];
    ln_unit_n<1>(uv, o);
    return o[0];
}

// sin and cos of 2 pi u_b for u_b = (2j + 1) 2^-24, j = word >> 9: exact
// quarter-turn reduction in integers, then Taylor series on [-pi/4, pi/4]
// (sine through y^9, cosine through y^8; within 2 ulp, or 2^-23 absolute).
__device__ __forceinline__ void sincos_2pi_word(uint32_t word, float& sn_o, float& cs_o) {
#pragma clang fp contract(off)
    const float S3 = -1.0f / 6.0f, S5 = 1.0f / 120.0f, S7 = -1.0f / 5040.0f, S9 = 1.0f / 362880.0f;
    const float C2 = -1.0f / 2.0f, C4 = 1.0f / 24.0f, C6 = -1.0f / 720.0f, C8 = 1.0f / 40320.0f;
    const float PI_F = 3.14159265358979323846f;
    const int jj = (int)((word >> 9) << 1) + 1;
    const int q = (jj + (1 << 21)) >> 22;
    const int rn = jj - (q << 22);
    const float r = (float)rn * 0x1.0p-23f;
    const float y = r * PI_F;
    const float y2 = y * y;
    const float sp = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(S9, y2, S7), y2, S5), y2, S3);
    const float sn = __builtin_fmaf(y * y2, sp, y);
    const float cp = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(C8, y2, C6), y2, C4), y2, C2);
    const float cs = __builtin_fmaf(y2, cp, 1.0f);
    // rotate by q quarter turns: swap on odd q, then exact sign flips
    // (sin: q = 2, 3; cos: q = 1, 2)
    const uint32_t qq = (uint32_t)q & 3u;
    const float a = (qq & 1u) ? cs : sn;
    const float b = (qq & 1u) ? sn : cs;
    sn_o = __uint_as_float(__float_as_uint(a) ^ ((qq & 2u) << 30));
    cs_o = __uint_as_float(__float_as_uint(b) ^ (((qq + 1u) & 2u) << 30));
}

// Box-Muller on P word pairs: rho = sqrt(-2 ln u_a) lies in [3e-4, 5.8], so
// its square is a normal FP32 number and sqrt_rn_normal applies.  The
// sin/cos of each pair has no dependence on its ln and sqrt chain.
template <int P>
__device__ __forceinline__ void box_muller_n(const uint32_t (&wa)[P], const uint32_t (&wb)[P],
                                             float (&z_even)[P], float (&z_odd)[P]) {
#pragma clang fp contract(off)
    float u[P], l[P], rho[P], sn[P], cs[P];
#pragma unroll
    for (int i = 0; i < P; ++i) u[i] = (float)(((wa[i] >> 9) << 1) + 1u) * 0x1.0p-24f;
    ln_unit_n<P>(u, l);
#pragma unroll
    for (int i = 0; i < P; ++i) l[i] = -2.0f * l[i];
    sqrt_rn_normal_n<P>(l, rho);
#pragma unroll
    for (int i = 0; i < P; ++i) sincos_2pi_word(wb[i], sn[i], cs[i]);
#pragma unroll
    for (int i = 0; i < P; ++i) {
        z_even[i] = rho[i] * cs[i];
        z_odd[i] = rho[i] * sn[i];
    }
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& z_even, float& z_odd) {
    const uint32_t a[1] = {wa}, b[1] = {wb};
    float ze[1], zo[1];
    box_muller_n<1>(a, b, ze, zo);
    z_even = ze[0];
    z_odd = zo[0];
}

// The 4G normals of the consecutive Philox blocks group0 .. group0+G-1 of
// sample m, block q's four normals at z[4q .. 4q+3].  c2 and c3 (uniform)
// enter the first round's product and XOR, so they go in as VGPR copies too
// when the key does.
template <int G, bool IN_VGPRS>
__device__ __forceinline__ void normal_blocks(uint32_t group0, uint32_t m, uint32_t c2, uint32_t c3,
                                              const PhiloxKey& pk, float* z) {
    uint32_t w[G][4];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        w[q][0] = group0 + (uint32_t)q;
        w[q][1] = m;
        w[q][2] = IN_VGPRS ? vgpr_copy(c2) : c2;
        w[q][3] = IN_VGPRS ? vgpr_copy(c3) : c3;
    }
    philox4x32_10_n<G>(w, pk);
    uint32_t wa[2 * G], wb[2 * G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        wa[2 * q] = w[q][0];
        wb[2 * q] = w[q][1];
        wa[2 * q + 1] = w[q][2];
        wb[2 * q + 1] = w[q][3];
    }
    float ze[2 * G], zo[2 * G];
    box_muller_n<2 * G>(wa, wb, ze, zo);
#pragma unroll
    for (int j = 0; j < 2 * G; ++j) {
        z[2 * j] = ze[j];
        z[2 * j + 1] = zo[j];
    }
}

// The four normals of Philox block `group` for sample m.
__device__ __forceinline__ void normal_block(uint32_t group, uint32_t m, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1, float& z0, float& z1,
                                             float& z2, float& z3) {
    float z[4];
    normal_blocks<1, false>(group, m, c2, c3, PhiloxKey::make<false>(k0, k1), z);
    z0 = z[0];
    z1 = z[1];
    z2 = z[2];
    z3 = z[3];
}

// min(max(x, lo), hi) for lo <= hi: the median of the three, one v_med3_f32
// (fminf/fmaxf would first quiet each operand, as IEEE minNum/maxNum ask).
// Equal to the clamp for every finite x.
__device__ __forceinline__ float clamp_f(float x, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(x, lo, hi);
}
// Running min and max of finite values as medians with -inf and +inf (no
// operand quieting, unlike fminf/fmaxf).  The infinities are VGPR copies the
// optimiser cannot see through, which keeps it from folding the medians back
// into minnum/maxnum (and keeps SGPR operands out of the medians).
struct MinMaxInf {
    float ninf, pinf;
    __device__ __forceinline__ MinMaxInf() {
        ninf = vgpr_copy(-INFINITY);
        pinf = vgpr_copy(INFINITY);
    }
    __device__ __forceinline__ float min(float a, float b) const { return __builtin_amdgcn_fmed3f(a, b, ninf); }
    __device__ __forceinline__ float max(float a, float b) const { return __builtin_amdgcn_fmed3f(a, b, pinf); }
};

// Square root outside the bit-exact recipe (goal distances): one hardware
// v_sqrt_f32 (1 ulp) instead of the correctly rounded sequence.
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// ------------------------------------------------------------- scoring forms
// Every kernel that samples, rolls out or scores uses these FP32 forms (and
// the dynamics below), with explicit fused multiply-adds and no other
// contraction, so that all of them produce the same bits for the same
// trajectory whatever the surrounding code.

// Squared distance of a position to the goal.
template <int DP>
__device__ __forceinline__ float goal_d2(const float* x, const float* g) {
#pragma clang fp contract(off)
    const float d0 = x[0] - g[0];
    float acc = d0 * d0;
#pragma unroll
    for (int c = 1; c < DP; ++c) {
        const float dc = x[c] - g[c];
        acc = __builtin_fmaf(dc, dc, acc);
    }
    return acc;
}

// 1 / max(|p_0 - g|, d0_floor): the goal term's normaliser.
__device__ __forceinline__ float inv_start_dist(float d0_2, float d0_floor) {
    return 1.0f / fmaxf(__builtin_amdgcn_sqrtf(d0_2), d0_floor);
}

// Per-step goal reward 1 - |p_t - g| / d0 from the distance itself.
__device__ __forceinline__ float goal_term(float dist, float inv_d0) {
    return __builtin_fmaf(-dist, inv_d0, 1.0f);
}

// Sampled control clip(u_base + du * mean_scale + sigma * eps) of one element,
// in two parts: the sample mean u_base + du * mean_scale, then the draw.
__device__ __forceinline__ float sample_mean(float ub, float du, float mscale) {
    return __builtin_fmaf(du, mscale, ub);
}
__device__ __forceinline__ float sample_from_mean(float mean, float sigma, float z, float lo, float hi) {
    return clamp_f(__builtin_fmaf(sigma, z, mean), lo, hi);
}
__device__ __forceinline__ float sample_control(float ub, float du, float mscale, float sigma, float z, float lo,
                                                float hi) {
    return sample_from_mean(sample_mean(ub, du, mscale), sigma, z, lo, hi);
}

// Team reward (sum of goal terms - w_safe * penalty) / (n T).
__device__ __forceinline__ float team_reward(float goal_sum, float w_safe, float penalty, int nT) {
    return __builtin_fmaf(-w_safe, penalty, goal_sum) / (float)nT;
}

// ---------------------------------------------------------------- dynamics
struct StepConsts {
    float dt, hdt, hdt2, dt6, vmax;
};

template <int DYN>
struct Dyn;

template <>
struct Dyn<HOLO2D> {
    static constexpr int DX = 4, DU = 2, DP = 2, AUX = 1;
    __device__ __forceinline__ static void init(const float*, float*) {}
    __device__ __forceinline__ static void step(float* x, float*, const float* u, const StepConsts& c) {
#pragma clang fp contract(off)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float p = x[i], v = x[2 + i], a = u[i];
            x[i] = __builtin_fmaf(a, c.hdt2, __builtin_fmaf(v, c.dt, p));
            x[2 + i] = clamp_f(__builtin_fmaf(a, c.dt, v), -c.vmax, c.vmax);
        }
    }
};

template <>
struct Dyn<HOLO3D> {
    static constexpr int DX = 6, DU = 3, DP = 3, AUX = 1;
    __device__ __forceinline__ static void init(const float*, float*) {}
    __device__ __forceinline__ static void step(float* x, float*, const float* u, const StepConsts& c) {
#pragma clang fp contract(off)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float p = x[i], v = x[3 + i], a = u[i];
            x[i] = __builtin_fmaf(a, c.hdt2, __builtin_fmaf(v, c.dt, p));
            x[3 + i] = clamp_f(__builtin_fmaf(a, c.dt, v), -c.vmax, c.vmax);
        }
    }
};

template <>
struct Dyn<UNICYCLE> {
    static constexpr int DX = 3, DU = 2, DP = 2, AUX = 2;
    // aux = (cos theta, sin theta) of the current heading
    __device__ __forceinline__ static void init(const float* x, float* aux) {
        __sincosf(x[2], &aux[1], &aux[0]);
    }
    __device__ __forceinline__ static void step(float* x, float* aux, const float* u,
                                                const StepConsts& c) {
#pragma clang fp contract(off)
        const float v = u[0], om = u[1];
        const float th_h = __builtin_fmaf(om, c.hdt, x[2]);
        const float th_1 = __builtin_fmaf(om, c.dt, x[2]);
        float sh, ch, s1, c1;
        __sincosf(th_h, &sh, &ch);
        __sincosf(th_1, &s1, &c1);
        const float kv = v * c.dt6;
        x[0] = __builtin_fmaf(kv, __builtin_fmaf(4.0f, ch, aux[0]) + c1, x[0]);
        x[1] = __builtin_fmaf(kv, __builtin_fmaf(4.0f, sh, aux[1]) + s1, x[1]);
        x[2] = th_1;
        aux[0] = c1;
        aux[1] = s1;
    }
};

// The paper's differential drive (Section V): x = [p_x, p_y, theta, v],
// u = [omega, a].  Within a step theta and v are linear in time, so the RK4
// stages depend on time alone, k2 = k3, and the position update is Simpson's
// rule on v(s) [cos, sin](theta(s)); theta and v themselves advance exactly.
// The speed is clipped to [-v_max, v_max] after the step.
template <>
struct Dyn<DIFFDRIVE> {
    static constexpr int DX = 4, DU = 2, DP = 2, AUX = 2;
    // aux = (cos theta, sin theta) of the current heading
    __device__ __forceinline__ static void init(const float* x, float* aux) {
        __sincosf(x[2], &aux[1], &aux[0]);
    }
    __device__ __forceinline__ static void step(float* x, float* aux, const float* u,
                                                const StepConsts& c) {
#pragma clang fp contract(off)
        const float om = u[0], acc = u[1];
        const float th_h = __builtin_fmaf(om, c.hdt, x[2]);
        const float th_1 = __builtin_fmaf(om, c.dt, x[2]);
        float sh, ch, s1, c1;
        __sincosf(th_h, &sh, &ch);
        __sincosf(th_1, &s1, &c1);
        const float v0 = x[3];
        const float vh = __builtin_fmaf(acc, c.hdt, v0);
        const float v1 = __builtin_fmaf(acc, c.dt, v0);
        x[0] = __builtin_fmaf(c.dt6, __builtin_fmaf(4.0f * vh, ch, v0 * aux[0]) + v1 * c1, x[0]);
        x[1] = __builtin_fmaf(c.dt6, __builtin_fmaf(4.0f * vh, sh, v0 * aux[1]) + v1 * s1, x[1]);
        x[2] = th_1;
        x[3] = clamp_f(v1, -c.vmax, c.vmax);
        aux[0] = c1;
        aux[1] = s1;
    }
};

// Squared pair distance in the fixed FP32 order ((dx*dx + dy*dy) + dz*dz).
template <int DP>
__device__ __forceinline__ float pair_d2(const float* a, const float* b) {
#pragma clang fp contract(off)
    const float d0 = a[0] - b[0];
    float acc = d0 * d0;
#pragma unroll
    for (int c = 1; c < DP; ++c) {
        const float dc = a[c] - b[c];
        acc = acc + dc * dc;
    }
    return acc;
}

// Squared gap between two axis-aligned boxes [alo, ahi] and [blo, bhi] in the
// order of pair_d2, with per-axis gap g = max(alo - bhi, blo - ahi, 0).  For
// points a in the first box and b in the second, |fl(a - b)| >= fl-gap on
// every axis, because rounding is monotonic; squaring and adding in the same
// order keep the inequality, so pair_d2(a, b) >= box_gap2(...) holds exactly
// in FP32 and a box pair with gap above the threshold holds no hit.
template <int DP>
__device__ __forceinline__ float box_gap2(const float* alo, const float* ahi, const float* blo,
                                          const float* bhi) {
#pragma clang fp contract(off)
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < DP; ++c) {
        const float gc = fmaxf(fmaxf(alo[c] - bhi[c], blo[c] - ahi[c]), 0.0f);
        acc = c == 0 ? gc * gc : acc + gc * gc;
    }
    return acc;
}

}  // namespace d4
