// Float64 reductions, elementwise helpers and the on-device step-size controller.
//
// The dual functionals J(phi) = int phi dnu + int phi^c dmu and
// I(psi) = int psi dmu + int psi^c dnu (eq. defJ / defI) are cell-volume
// weighted sums.  Every sum is accumulated in float64 from per-block partials
// reduced by one controller block in a fixed order, so results do not depend
// on scheduling.  The controller applies the Section 4.2 rule after each
// gradient step: with increase = J(p + sigma g) - J(p) and G = ||grad||^2_{H^1},
// keep sigma when beta1 sigma G <= increase <= beta2 sigma G, otherwise
// shrink by alpha2 (not below sigma_min) or grow by alpha1; no backtracking.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace bfm {

template <typename T>
__global__ void __launch_bounds__(kRedBlock)
dot2_kernel(const T *__restrict__ a1, const T *__restrict__ b1, const T *__restrict__ a2,
            const T *__restrict__ b2, long long N, double *__restrict__ part1, double *__restrict__ part2,
            const int32_t *__restrict__ done)
{
    if (done != nullptr && *done) return;
    __shared__ double sh[kRedBlock / kWave];
    double s1 = 0.0, s2 = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool vec = (N & 3) == 0 && ((((uintptr_t)a1 | (uintptr_t)(b1 ? b1 : a1) | (uintptr_t)(a2 ? a2 : a1) |
                                        (uintptr_t)(b2 ? b2 : a1)) & 15) == 0);
    if (vec) {
        using V = typename std::conditional<sizeof(T) == 4, float4, double4>::type;
        const long long N4 = N / 4;
        for (long long i = t0; i < N4; i += stride) {
            const V x = reinterpret_cast<const V *>(a1)[i];
            if (b1 != nullptr) {
                const V y = reinterpret_cast<const V *>(b1)[i];
                s1 += (double)x.x * (double)y.x + (double)x.y * (double)y.y + (double)x.z * (double)y.z +
                      (double)x.w * (double)y.w;
            } else {
                s1 += (double)x.x + (double)x.y + (double)x.z + (double)x.w;
            }
            if (a2 != nullptr) {
                const V u = reinterpret_cast<const V *>(a2)[i];
                const V v = reinterpret_cast<const V *>(b2)[i];
                s2 += (double)u.x * (double)v.x + (double)u.y * (double)v.y + (double)u.z * (double)v.z +
                      (double)u.w * (double)v.w;
            }
        }
    } else {
        for (long long i = t0; i < N; i += stride) {
            s1 += (double)a1[i] * (b1 != nullptr ? (double)b1[i] : 1.0);
            if (a2 != nullptr) s2 += (double)a2[i] * (double)b2[i];
        }
    }
    s1 = block_reduce<R_SUM>(s1, sh);
    if (threadIdx.x == 0) part1[blockIdx.x] = s1;
    if (a2 != nullptr) {
        s2 = block_reduce<R_SUM>(s2, sh);
        if (threadIdx.x == 0) part2[blockIdx.x] = s2;
    }
}

template <typename T>
hipError_t launch_dot2(const T *a1, const T *b1, const T *a2, const T *b2, long long N, double *part1,
                       double *part2, int nblocks, const int32_t *done, hipStream_t stream)
{
    hipLaunchKernelGGL((dot2_kernel<T>), dim3(nblocks), dim3(kRedBlock), 0, stream, a1, b1, a2, b2, N, part1,
                       part2, done);
    return hipGetLastError();
}

// Sums, extrema and a count of invalid (negative or non-finite) values of mu, nu.
template <typename T>
__global__ void __launch_bounds__(kRedBlock)
stats_kernel(const T *__restrict__ mu, const T *__restrict__ nu, long long N, double *__restrict__ partials,
             long long slot_len)
{
    __shared__ double sh[kRedBlock / kWave];
    double smu = 0, snu = 0, xmu = -INFINITY, xnu = -INFINITY, nmu = INFINITY, nnu = INFINITY, bad = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        const double a = (double)mu[i], b = (double)nu[i];
        if (!(isfinite(a) && a >= 0.0)) bad += 1.0;
        if (!(isfinite(b) && b >= 0.0)) bad += 1.0;
        smu += a;
        snu += b;
        xmu = fmax(xmu, a);
        xnu = fmax(xnu, b);
        nmu = fmin(nmu, a);
        nnu = fmin(nnu, b);
    }
    const double r0 = block_reduce<R_SUM>(smu, sh);
    const double r1 = block_reduce<R_SUM>(snu, sh);
    const double r2 = block_reduce<R_MAX>(xmu, sh);
    const double r3 = block_reduce<R_MAX>(xnu, sh);
    const double r4 = block_reduce<R_MIN>(nmu, sh);
    const double r5 = block_reduce<R_MIN>(nnu, sh);
    const double r6 = block_reduce<R_SUM>(bad, sh);
    if (threadIdx.x == 0) {
        const int b = blockIdx.x;
        partials[S_SUM_MU * slot_len + b] = r0;
        partials[S_SUM_NU * slot_len + b] = r1;
        partials[S_MAX_MU * slot_len + b] = r2;
        partials[S_MAX_NU * slot_len + b] = r3;
        partials[S_MIN_MU * slot_len + b] = r4;
        partials[S_MIN_NU * slot_len + b] = r5;
        partials[S_BAD * slot_len + b] = r6;
    }
}

template <typename T>
hipError_t launch_stats(const T *mu, const T *nu, long long N, double *partials, long long slot_len, int nblocks,
                        hipStream_t stream)
{
    hipLaunchKernelGGL((stats_kernel<T>), dim3(nblocks), dim3(kRedBlock), 0, stream, mu, nu, N, partials, slot_len);
    return hipGetLastError();
}

template <typename T>
__global__ void fill_kernel(T *x, long long N, T value)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = value;
}

template <typename T>
hipError_t launch_fill(T *x, long long N, T value, hipStream_t stream)
{
    const long long b = (N + 255) / 256;
    hipLaunchKernelGGL((fill_kernel<T>), dim3((unsigned)(b < 8192 ? b : 8192)), dim3(256), 0, stream, x, N,
                       value);
    return hipGetLastError();
}

// out = mul * (in + sign * (*shift)) for up to two fields; a null shift adds 0.
template <typename T>
__global__ void shift_scale_kernel(T *out_a, const T *in_a, const double *shift_a, double sign_a, T *out_b,
                                   const T *in_b, const double *shift_b, double sign_b, long long N, double mul)
{
    const T ca = shift_a != nullptr ? T(sign_a * *shift_a) : T(0);
    const T cb = shift_b != nullptr ? T(sign_b * *shift_b) : T(0);
    const T m = T(mul);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        if (out_a != nullptr) out_a[i] = m * (in_a[i] + ca);
        if (out_b != nullptr) out_b[i] = m * (in_b[i] + cb);
    }
}

template <typename T>
hipError_t launch_shift_scale(T *out_a, const T *in_a, const double *shift_a, double sign_a, T *out_b,
                              const T *in_b, const double *shift_b, double sign_b, long long N, double mul,
                              hipStream_t stream)
{
    const long long b = (N + 255) / 256;
    hipLaunchKernelGGL((shift_scale_kernel<T>), dim3((unsigned)(b < 8192 ? b : 8192)), dim3(256), 0, stream,
                       out_a, in_a, shift_a, sign_a, out_b, in_b, shift_b, sign_b, N, mul);
    return hipGetLastError();
}

// acc + x[t] + x[t + B] + x[t + 2B] + ... (t = threadIdx.x, B = blockDim.x,
// indices < n), added in that order; eight terms are loaded before they are
// added, so their load latencies overlap.
__device__ __forceinline__ double strided_sum(const double *__restrict__ x, int n, double acc)
{
    const int st = blockDim.x;
    int i = threadIdx.x;
    for (; i + 7 * st < n; i += 8 * st) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = x[i + k * st];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += v[k];
    }
    for (; i < n; i += st) acc += x[i];
    return acc;
}

__device__ double slot_reduce_sum(const double *partials, long long slot_len, int slot, int nb, double *sh)
{
    return block_reduce<R_SUM>(strided_sum(partials + slot * slot_len, nb, 0.0), sh);
}
__device__ double slot_reduce_max(const double *partials, long long slot_len, int slot, int nb, double *sh)
{
    double v = -INFINITY;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) v = fmax(v, partials[slot * slot_len + i]);
    return block_reduce<R_MAX>(v, sh);
}
__device__ double slot_reduce_min(const double *partials, long long slot_len, int slot, int nb, double *sh)
{
    double v = INFINITY;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) v = fmin(v, partials[slot * slot_len + i]);
    return block_reduce<R_MIN>(v, sh);
}

// K block sums at once (valid in thread 0), each in the order of
// slot_reduce_sum: per-thread strided partial, wave sum, waves in order.
// One pair of barriers for all K instead of one per sum.
template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double *sh)
{
    constexpr int NW = kRedBlock / kWave;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) sh[k * NW + w] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double r = sh[k * NW];
            for (int i = 1; i < NW; ++i) r += sh[k * NW + i];
            v[k] = r;
        }
    __syncthreads();
}

__device__ double step_rule(double sigma, double increase, double G, const CtrlParams &p)
{
    if (increase < p.beta1 * sigma * G) return fmax(p.alpha2 * sigma, p.sigma_min);
    if (increase > p.beta2 * sigma * G) return p.alpha1 * sigma;
    return sigma;
}

__device__ __forceinline__ void ctrl_body(DevState *st, const double *__restrict__ partials,
                                          const double *__restrict__ gpart, int mode, const CtrlParams &prm,
                                          TraceRec *trace)
{
    __shared__ double sh[4 * (kRedBlock / kWave)];
    const int nb = prm.nred, ns = prm.nsplat, ng = prm.ngpart;
    const long long sl = prm.slot_len;
    const bool reuse_dot = (mode & CTRL_REUSE_DOT) != 0;
    mode &= 0xff;
    if (mode == CTRL_INIT) {
        const double smu = slot_reduce_sum(partials, sl, S_SUM_MU, nb, sh);
        const double snu = slot_reduce_sum(partials, sl, S_SUM_NU, nb, sh);
        const double xmu = slot_reduce_max(partials, sl, S_MAX_MU, nb, sh);
        const double xnu = slot_reduce_max(partials, sl, S_MAX_NU, nb, sh);
        const double nmu = slot_reduce_min(partials, sl, S_MIN_MU, nb, sh);
        const double nnu = slot_reduce_min(partials, sl, S_MIN_NU, nb, sh);
        const double bad = slot_reduce_sum(partials, sl, S_BAD, nb, sh);
        if (threadIdx.x == 0) {
            st->mass_mu = prm.vol * smu;
            st->mass_nu = prm.vol * snu;
            st->max_mu = xmu;
            st->max_nu = xnu;
            st->min_mu = nmu;
            st->min_nu = nnu;
            st->bad = bad;
            st->sigma = prm.sigma0 > 0.0 ? prm.sigma0 : 8.0 * fmin(1.0 / xmu, 1.0 / xnu);
            st->J_old = st->P = st->G = st->J_new = st->gap = 0.0;
            st->q_src = 0.0;   // <phi_0, nu> of a start from phi_0 = 0 (a head reusing the step sum reads it)
            st->dual_head = st->primal_head = st->G_head = 0.0;
            st->mean_a = st->mean_b = 0.0;
            st->iter = 0;
            st->done = 0;
            st->nonfinite = 0;
            st->ntrace = 0;
            st->sigma_floor_hits = 0;
        }
        return;
    }
    if (mode == CTRL_MEANS) {
        const double a = slot_reduce_sum(partials, sl, S_MEAN_A, nb, sh);
        const double b = slot_reduce_sum(partials, sl, S_MEAN_B, nb, sh);
        if (threadIdx.x == 0) {
            st->mean_a = a * prm.inv_N;
            st->mean_b = b * prm.inv_N;
        }
        return;
    }
    if (st->done) return;
    if (mode == CTRL_HEAD_PHI || mode == CTRL_HEAD_PSI) {
        // sum p * tgt (unless reused), sum pc * src, the primal cost, G
        double acc[4];
        acc[0] = reuse_dot ? 0.0 : strided_sum(partials + S_P_TGT * sl, nb, 0.0);
        acc[1] = strided_sum(partials + S_PC_SRC * sl, ns, 0.0);
        acc[2] = strided_sum(partials + S_PRIMAL * sl, ns, 0.0);
        acc[3] = strided_sum(gpart, ng, 0.0);
        block_sums<4>(acc, sh);
        const double a = reuse_dot ? st->q_src : acc[0];
        const double b = acc[1], P = acc[2], G = acc[3];
        if (threadIdx.x == 0) {
            st->J_old = prm.vol * (a + b);
            st->P = prm.vol * P;
            st->G = prm.vol * G;
            if (!(isfinite(st->J_old) && isfinite(st->G) && isfinite(st->P))) {
                st->nonfinite = 1;
                st->done = 1;
                return;
            }
            if (mode == CTRL_HEAD_PHI) {
                st->gap = fmax(fabs(st->P - st->J_old), st->G);
                st->dual_head = st->J_old;
                st->primal_head = st->P;
                st->G_head = st->G;
                if (st->ntrace < kMaxTrace) {
                    TraceRec &r = trace[st->ntrace];
                    r.iter = st->iter;
                    r.dual = st->J_old;
                    r.primal = st->P;
                    r.G = st->G;
                    r.gap = st->gap;
                    r.sigma = st->sigma;
                    r.J_half = NAN;
                    r.I_new = NAN;
                }
                st->ntrace += 1;
                if (prm.tol > 0.0 && st->gap < prm.tol) st->done = 1;
            }
        }
        return;
    }
    if (mode == CTRL_GA_NEXT) {
        const double a = slot_reduce_sum(partials, sl, S_Q_TGT, prm.nqt, sh);
        if (threadIdx.x == 0) {
            if (!isfinite(a)) {
                st->nonfinite = 1;
                st->done = 1;
                return;
            }
            st->q_src = a;
            st->iter += 1;
        }
        return;
    }
    if (mode == CTRL_STEP_PHI || mode == CTRL_STEP_PSI) {
        double acc[2];
        acc[0] = strided_sum(partials + S_Q_TGT * sl, prm.nqt, 0.0);
        acc[1] = strided_sum(partials + S_Q_SRC * sl, prm.nqs, 0.0);
        block_sums<2>(acc, sh);
        const double a = acc[0], b = acc[1];
        if (threadIdx.x == 0) {
            st->q_src = b;
            st->J_new = prm.vol * (a + b);
            if (!isfinite(st->J_new)) {
                st->nonfinite = 1;
                st->done = 1;
                return;
            }
            const int tr = st->ntrace - 1;
            if (tr >= 0 && tr < kMaxTrace) {
                if (mode == CTRL_STEP_PHI)
                    trace[tr].J_half = st->J_new;
                else
                    trace[tr].I_new = st->J_new;
            }
            st->sigma = step_rule(st->sigma, st->J_new - st->J_old, st->G, prm);
            if (st->sigma == prm.sigma_min) st->sigma_floor_hits += 1;
            if (mode == CTRL_STEP_PSI) st->iter += 1;
        }
    }
}

__global__ void __launch_bounds__(kRedBlock)
ctrl_kernel(DevState *st, const double *__restrict__ partials, const double *__restrict__ gpart, int mode,
            CtrlParams prm, TraceRec *trace)
{
    ctrl_body(st, partials, gpart, mode, prm, trace);
}

// The controller of every pair of a batch: one workgroup per pair, each with
// its pair's state, partials and counts (the deposition's partial count is
// the number of its joint-list workgroups that visited the pair).
// A pair that stops here also sets its bit of the table's stop mask, which
// the other multi-pair kernels test (one load from the table head instead of
// a load of the pair's state pointer and then of its flag).
__global__ void __launch_bounds__(kRedBlock)
ctrl_multi_kernel(BatchHead *__restrict__ tab, int role, int mode)
{
    const PairDev &P = reinterpret_cast<const PairDev *>(tab + 1)[blockIdx.x];
    CtrlParams prm = P.cp;
    const int ent = (role ? P.tiles_nu : P.tiles_mu)[0];
    prm.nsplat = ent < tab->splat_grid ? ent : tab->splat_grid;
    ctrl_body(P.st, P.part, P.gpart, mode, prm, P.trace);
    __syncthreads();
    if (threadIdx.x == 0 && P.st->done) atomicOr(&tab->done_mask, 1ull << blockIdx.x);
}

// One wave, lane p for pair p (np <= kBatchChunk = 64): the stop flags as a
// bit mask, their count and whether all are set.
__global__ void __launch_bounds__(kWave) batch_done_kernel(BatchHead *tab)
{
    static_assert(kBatchChunk <= kWave, "one lane per pair");
    const PairDev *pairs = reinterpret_cast<const PairDev *>(tab + 1);
    const int np = tab->np;
    const int p = threadIdx.x;
    const bool stopped = p < np ? pairs[p].st->done != 0 : true;
    const unsigned long long mask = __ballot(stopped);
    if (p == 0) {
        const unsigned long long live = np >= 64 ? ~0ull : ((1ull << np) - 1);
        tab->done_mask = mask & live;
        tab->nactive = np - __popcll(mask & live);
        tab->all_done = (mask & live) == live;
    }
}

hipError_t launch_batch_done(BatchHead *tab, hipStream_t stream)
{
    hipLaunchKernelGGL(batch_done_kernel, dim3(1), dim3(kWave), 0, stream, tab);
    return hipGetLastError();
}

hipError_t launch_ctrl_multi(BatchHead *tab, int np, int role, int mode, hipStream_t stream)
{
    if (np < 1 || np > kBatchChunk) return hipErrorInvalidValue;
    hipLaunchKernelGGL(ctrl_multi_kernel, dim3(np), dim3(kRedBlock), 0, stream, tab, role, mode);
    return hipGetLastError();
}

// ------------------------------------------------------- batched gradient
__device__ __forceinline__ int grad_pair_of(const BatchIdx &bi)
{
    int lo = 0, hi = bi.np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bi.off[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ void __launch_bounds__(kRedBlock) grad_sums_kernel(const GradPair *__restrict__ tab, BatchIdx bi)
{
    __shared__ double sh[kRedBlock / kWave];
    const int p = grad_pair_of(bi);
    const GradPair &G = tab[p];
    const long long b = (long long)blockIdx.x - bi.off[p];
    const long long i0 = b * G.epb, i1 = i0 + G.epb < G.N ? i0 + G.epb : G.N;
    const T *phi = (const T *)G.phi, *psi = (const T *)G.psi;
    double sa = 0.0, sb = 0.0;
    for (long long i = i0 + threadIdx.x; i < i1; i += kRedBlock) {
        sa += (double)psi[i];
        sb += (double)phi[i];
    }
    sa = block_reduce<R_SUM>(sa, sh);
    sb = block_reduce<R_SUM>(sb, sh);
    if (threadIdx.x == 0) {
        G.part[S_MEAN_A * G.slot_len + b] = sa;
        G.part[S_MEAN_B * G.slot_len + b] = sb;
    }
}

__global__ void __launch_bounds__(kRedBlock) grad_means_kernel(const GradPair *__restrict__ tab)
{
    __shared__ double sh[4 * (kRedBlock / kWave)];
    const GradPair &G = tab[blockIdx.x];
    const double a = slot_reduce_sum(G.part, G.slot_len, S_MEAN_A, G.nb, sh);
    const double b = slot_reduce_sum(G.part, G.slot_len, S_MEAN_B, G.nb, sh);
    if (threadIdx.x == 0) {
        G.st->mean_a = a / (double)G.N;
        G.st->mean_b = b / (double)G.N;
    }
}

template <typename T>
__global__ void __launch_bounds__(kRedBlock) grad_apply_kernel(const GradPair *__restrict__ tab, BatchIdx bi)
{
    const int p = grad_pair_of(bi);
    const GradPair &G = tab[p];
    const long long b = (long long)blockIdx.x - bi.off[p];
    const long long i0 = b * G.epb, i1 = i0 + G.epb < G.N ? i0 + G.epb : G.N;
    const T ca = T(-G.st->mean_a), cb = T(-G.st->mean_b), m = T(G.mul);
    const T *phi = (const T *)G.phi, *psi = (const T *)G.psi;
    T *gmu = (T *)G.gmu, *gnu = (T *)G.gnu;
    for (long long i = i0 + threadIdx.x; i < i1; i += kRedBlock) {
        if (gmu != nullptr) gmu[i] = m * (psi[i] + ca);
        if (gnu != nullptr) gnu[i] = m * (phi[i] + cb);
    }
}

template <typename T>
hipError_t launch_grad_multi(const GradPair *tab, const GradPair *host, int np, hipStream_t stream)
{
    if (np < 1 || np > kBatchChunk) return hipErrorInvalidValue;
    BatchIdx bi{};
    bi.np = np;
    for (int p = 0; p < np; ++p) bi.off[p + 1] = bi.off[p] + host[p].nb;
    hipLaunchKernelGGL((grad_sums_kernel<T>), dim3((unsigned)bi.off[np]), dim3(kRedBlock), 0, stream, tab, bi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(grad_means_kernel, dim3(np), dim3(kRedBlock), 0, stream, tab);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((grad_apply_kernel<T>), dim3((unsigned)bi.off[np]), dim3(kRedBlock), 0, stream, tab, bi);
    return hipGetLastError();
}
template hipError_t launch_grad_multi<float>(const GradPair *, const GradPair *, int, hipStream_t);
template hipError_t launch_grad_multi<double>(const GradPair *, const GradPair *, int, hipStream_t);

// ------------------------------------------------------- batched finish
// After the last head of every pair: phi <- phi - mean(phi) and
// psi <- phi^c + mean(phi) (the outputs of a solve), for a chunk of pairs in
// three launches: per-workgroup sums of phi, the mean per pair, the shifts.
__device__ __forceinline__ void finish_range(const PairDev &P, long long b, long long epb, long long &i0,
                                             long long &i1)
{
    const long long N = (long long)P.n0 * P.n1;
    i0 = b * epb;
    i1 = i0 + epb < N ? i0 + epb : N;
}

template <typename T>
__global__ void __launch_bounds__(kRedBlock) finish_sums_kernel(const BatchHead *__restrict__ tab, BatchIdx bi,
                                                                long long epb)
{
    __shared__ double sh[kRedBlock / kWave];
    const int p = grad_pair_of(bi);
    const PairDev &P = reinterpret_cast<const PairDev *>(tab + 1)[p];
    const long long b = (long long)blockIdx.x - bi.off[p];
    long long i0, i1;
    finish_range(P, b, epb, i0, i1);
    const T *phi = (const T *)P.phi;
    double s = 0.0;
    for (long long i = i0 + threadIdx.x; i < i1; i += kRedBlock) s += (double)phi[i];
    s = block_reduce<R_SUM>(s, sh);
    if (threadIdx.x == 0) P.part[S_MEAN_A * P.slot_len + b] = s;
}

__global__ void __launch_bounds__(kRedBlock) finish_means_kernel(const BatchHead *__restrict__ tab, BatchIdx bi)
{
    __shared__ double sh[kRedBlock / kWave];
    const PairDev &P = reinterpret_cast<const PairDev *>(tab + 1)[blockIdx.x];
    const int nb = bi.off[blockIdx.x + 1] - bi.off[blockIdx.x];
    const double a = slot_reduce_sum(P.part, P.slot_len, S_MEAN_A, nb, sh);
    if (threadIdx.x == 0) P.st->mean_a = a / ((double)P.n0 * (double)P.n1);
}

template <typename T>
__global__ void __launch_bounds__(kRedBlock) finish_apply_kernel(const BatchHead *__restrict__ tab, BatchIdx bi,
                                                                 long long epb)
{
    const int p = grad_pair_of(bi);
    const PairDev &P = reinterpret_cast<const PairDev *>(tab + 1)[p];
    const long long b = (long long)blockIdx.x - bi.off[p];
    long long i0, i1;
    finish_range(P, b, epb, i0, i1);
    const T m = T(P.st->mean_a);
    T *phi = (T *)P.phi, *psi = (T *)P.psi;
    const T *pc = (const T *)P.pc;
    for (long long i = i0 + threadIdx.x; i < i1; i += kRedBlock) {
        phi[i] = phi[i] - m;
        psi[i] = pc[i] + m;
    }
}

template <typename T>
hipError_t launch_finish_multi(const BatchHead *tab, const int *n0s, const int *n1s, int np, long long epb,
                               hipStream_t stream)
{
    if (np < 1 || np > kBatchChunk || epb < 1) return hipErrorInvalidValue;
    BatchIdx bi{};
    bi.np = np;
    for (int p = 0; p < np; ++p) bi.off[p + 1] = bi.off[p] + (int)(((long long)n0s[p] * n1s[p] + epb - 1) / epb);
    hipLaunchKernelGGL((finish_sums_kernel<T>), dim3((unsigned)bi.off[np]), dim3(kRedBlock), 0, stream, tab, bi, epb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finish_means_kernel, dim3(np), dim3(kRedBlock), 0, stream, tab, bi);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((finish_apply_kernel<T>), dim3((unsigned)bi.off[np]), dim3(kRedBlock), 0, stream, tab, bi, epb);
    return hipGetLastError();
}
template hipError_t launch_finish_multi<float>(const BatchHead *, const int *, const int *, int, long long,
                                               hipStream_t);
template hipError_t launch_finish_multi<double>(const BatchHead *, const int *, const int *, int, long long,
                                                hipStream_t);

hipError_t launch_ctrl(DevState *st, const double *partials, const double *gpart, int mode, CtrlParams prm,
                       TraceRec *trace, hipStream_t stream)
{
    hipLaunchKernelGGL(ctrl_kernel, dim3(1), dim3(kRedBlock), 0, stream, st, partials, gpart, mode, prm, trace);
    return hipGetLastError();
}

#define BFM_INST_RED(T)                                                                                      \
    template hipError_t launch_dot2<T>(const T *, const T *, const T *, const T *, long long, double *,      \
                                       double *, int, const int32_t *, hipStream_t);                         \
    template hipError_t launch_stats<T>(const T *, const T *, long long, double *, long long, int, hipStream_t); \
    template hipError_t launch_fill<T>(T *, long long, T, hipStream_t);                                      \
    template hipError_t launch_shift_scale<T>(T *, const T *, const double *, double, T *, const T *,       \
                                              const double *, double, long long, double, hipStream_t);
BFM_INST_RED(float)
BFM_INST_RED(double)

}  // namespace bfm
