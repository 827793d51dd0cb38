// Map and pushforward of one density by the current potential.
//
// Paper: T_phi(x) = x - (grad h)^{-1}(grad phi^c(x)) (Lemma on c-transform
// properties (ii)), which for h = |.|^2/2 is x - grad phi^c(x); the first
// variation of J is nu - T#mu (Lemma fact:derivative-J), with the pushforward
// defined against test functions, int f d(T#mu) = int f(T(x)) dmu
// (Section 2.1).  On the grid:
//   * grad phi^c by central differences, one-sided on the two faces of each
//     axis; T clamped to the box of cell centres [h/2, 1 - h/2];
//   * T#mu with piecewise-multilinear test functions: the mass of cell x is
//     split over the 2^d cell centres around T(x) with the multilinear
//     weights (atomic adds; exact mass conservation up to rounding).
// Fused float64 partial sums: sum mu |x - T|^2 / 2 (primal cost of the map)
// and sum mu phi^c (the second term of J).
#include "common.hpp"
#include "launch.hpp"

namespace bfm {

template <typename T, int D>
__global__ void __launch_bounds__(kRedBlock)
splat_kernel(Grid g, const T *__restrict__ pc, const T *__restrict__ src, T *__restrict__ rho,
             T *__restrict__ Tout, double *__restrict__ part_primal, double *__restrict__ part_pcsrc,
             const int32_t *__restrict__ done)
{
    if (done != nullptr && *done) return;
    __shared__ double sh[kRedBlock / kWave];
    double accP = 0.0, accJ = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < g.N;
         idx += (long long)gridDim.x * blockDim.x) {
        const T s = src[idx];
        if (s == T(0) && Tout == nullptr) continue;   // no mass, nothing to write
        int ii[D];
        long long r = idx;
#pragma unroll
        for (int a = D - 1; a >= 0; --a) {
            ii[a] = (int)(r % g.n[a]);
            r /= g.n[a];
        }
        const T p0 = pc[idx];
        T wup[D];
        long long base = 0;
        T sq = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int n = g.n[a];
            const long long str = g.stride[a];
            const int i = ii[a];
            const T fn = T(n);
            T d;
            if (i == 0)
                d = (pc[idx + str] - p0) * fn;
            else if (i == n - 1)
                d = (p0 - pc[idx - str]) * fn;
            else
                d = (pc[idx + str] - pc[idx - str]) * (T(0.5) * fn);
            const T x = (T(i) + T(0.5)) / fn;
            const T lo = T(0.5) / fn;
            const T t = fmin(fmax(x - d, lo), T(1) - lo);
            if (Tout != nullptr) Tout[(long long)a * g.N + idx] = t;
            sq += (x - t) * (x - t);
            const T q = t * fn - T(0.5);
            int i0 = (int)floor(q);
            i0 = min(max(i0, 0), n - 2);
            wup[a] = q - T(i0);
            base += (long long)i0 * str;
        }
        if (s != T(0) && rho != nullptr) {
#pragma unroll
            for (int c = 0; c < (1 << D); ++c) {
                T w = s;
                long long off = base;
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    const int bit = (c >> (D - 1 - a)) & 1;
                    w *= bit ? wup[a] : T(1) - wup[a];
                    off += bit ? g.stride[a] : 0;
                }
                atomicAdd(rho + off, w);
            }
            accP += (double)s * 0.5 * (double)sq;
            accJ += (double)s * (double)p0;
        }
    }
    const double P = block_reduce<R_SUM>(accP, sh);
    const double J = block_reduce<R_SUM>(accJ, sh);
    if (threadIdx.x == 0) {
        if (part_primal != nullptr) part_primal[blockIdx.x] = P;
        if (part_pcsrc != nullptr) part_pcsrc[blockIdx.x] = J;
    }
}

template <typename T>
hipError_t launch_splat(const Grid &g, const T *pc, const T *src, T *rho, T *Tout, double *part_primal,
                        double *part_pcsrc, int nblocks, const int32_t *done, hipStream_t stream)
{
    if (g.ndim == 2)
        hipLaunchKernelGGL((splat_kernel<T, 2>), dim3(nblocks), dim3(kRedBlock), 0, stream, g, pc, src, rho,
                           Tout, part_primal, part_pcsrc, done);
    else if (g.ndim == 3)
        hipLaunchKernelGGL((splat_kernel<T, 3>), dim3(nblocks), dim3(kRedBlock), 0, stream, g, pc, src, rho,
                           Tout, part_primal, part_pcsrc, done);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template hipError_t launch_splat<float>(const Grid &, const float *, const float *, float *, float *, double *,
                                        double *, int, const int32_t *, hipStream_t);
template hipError_t launch_splat<double>(const Grid &, const double *, const double *, double *, double *,
                                         double *, double *, int, const int32_t *, hipStream_t);

}  // namespace bfm
