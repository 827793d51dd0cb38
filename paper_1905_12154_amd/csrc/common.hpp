// Shared definitions of the HIP back-and-forth library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfm.h"

namespace bfm {

constexpr int kWave = 64;
constexpr int kRedBlock = 256;       // threads of every reduction-carrying kernel
constexpr int kMaxRedBlocks = 1024;  // grid size of the grid-stride reduction kernels

// Reduction slots: each kernel that contributes to a float64 sum writes one
// partial per block into partials[slot * slot_len + block] (slot_len is a
// property of the plan: at least the largest grid of a contributing kernel);
// a single controller block reduces them in a fixed order (deterministic).
enum Slot {
    S_P_TGT = 0,    // sum p * tgt            (head of a half-step)
    S_PC_SRC,       // sum p^c * src          (head)
    S_PRIMAL,       // sum src * |x - T|^2/2  (head)
    S_G,            // sum w_k X_k^2 / lambda_k (Poisson)
    S_Q_TGT,        // sum p_new * tgt        (after the gradient step)
    S_Q_SRC,        // sum q * src, q = p_new^c
    S_SUM_MU,
    S_SUM_NU,
    S_MAX_MU,
    S_MAX_NU,
    S_MIN_MU,
    S_MIN_NU,
    S_BAD,          // count of non-finite input values
    S_MEAN_A,
    S_MEAN_B,
    kNumSlots
};

// Device-resident solver state (float64 scalars, one per problem).
struct DevState {
    double sigma;
    double J_old, P, G, J_new;   // current half-step
    double gap;
    double mass_mu, mass_nu, max_mu, max_nu, min_mu, min_nu, bad;
    double mean_a, mean_b;
    double dual_head, primal_head, G_head;   // last phi-step head
    double q_src;                // sum q * src of the last step = sum p * tgt of the next head
    int32_t iter;                // completed full iterations
    int32_t done;                // 1: gap < tol reached, later kernels are no-ops
    int32_t nonfinite;           // 1: a non-finite scalar appeared
    int32_t ntrace;
    int32_t sigma_floor_hits;    // step-rule updates that held sigma at sigma_min
};

// One trace record per evaluated head of a phi-step.
struct TraceRec {
    double iter, dual, primal, G, gap, sigma, J_half, I_new;
};
constexpr int kMaxTrace = 4096;

template <typename T> struct cpx { T x, y; };

template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cpx<T> conj_(cpx<T> a) { return {a.x, -a.y}; }

// Line geometry of a separable sweep along one axis of a row-major field:
// line L starts at (L / inner) * n * inner + (L % inner), elements are `inner`
// apart (inner = product of the sizes of the later axes).
__device__ __forceinline__ long long line_base(long long L, int n, int inner) {
    return (L / inner) * (long long)n * inner + (L % inner);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}

// Block reductions for blockDim.x == kRedBlock; result valid in thread 0.
// `sh` holds kRedBlock / kWave doubles.
enum RedOp { R_SUM = 0, R_MAX = 1, R_MIN = 2 };
template <int OP> __device__ __forceinline__ double block_reduce(double v, double *sh) {
    v = OP == R_SUM ? wave_sum(v) : (OP == R_MAX ? wave_max(v) : wave_min(v));
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
    if (threadIdx.x == 0) {
        for (int i = 1; i < kRedBlock / kWave; ++i)
            r = OP == R_SUM ? r + sh[i] : (OP == R_MAX ? fmax(r, sh[i]) : fmin(r, sh[i]));
    }
    __syncthreads();
    return r;
}

// Grid-level shape of a field, handed to elementwise/stencil kernels by value.
struct Grid {
    int ndim;
    int n[3];
    long long stride[3];
    long long N;
    double vol;    // cell volume
    double pw[3];  // cost exponent per axis, h_a(z) = |z|^pw / pw (eq. p_costs); 2 = quadratic
};

}  // namespace bfm
