// Neumann Poisson solve on the grid: g = (-Laplacian)^{-1}(f - mean f).
//
// Paper: the H^1 gradient is (-Laplacian)^{-1} of the mean-free first
// variation with zero Neumann data (H^1-gradient lemma, eq. gradients_J_I);
// the Laplace inversion uses the FFT (Section 4.3).  On the cell-centred grid
// the second-difference Neumann Laplacian is diagonalised by the DCT-II, with
// eigenvalues lambda_k = sum_a 4 sin^2(pi k_a / (2 n_a)) n_a^2, so
//     g = DCT3( DCT2(f) / lambda ),   zero mode dropped.
//
// Transforms along one axis at a time (separable), unnormalised:
//   DCT2:  X_k = sum_j x_j cos(pi k (2j+1) / (2n))
//   DCT3:  x_j = (X_0 + 2 sum_{k>0} X_k cos(pi k (2j+1) / (2n))) / n  (exact inverse)
// Each line is reordered (even samples forward, odd samples backward) so the
// DCT becomes one length-n complex DFT plus a quarter-wave twiddle (Makhoul's
// method); two real lines share one complex DFT (real and imaginary parts).
// The DFT is a Stockham auto-sort FFT in LDS with radix 4, 2 and 3 stages
// (n = 2^a 3^b), twiddles from a per-axis table.
#include "common.hpp"
#include "launch.hpp"

namespace bfm {

template <typename T, int R>
__device__ __forceinline__ void small_dft(cpx<T> *x) {
    if constexpr (R == 2) {
        const cpx<T> a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const cpx<T> a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
        const cpx<T> c = cadd(x[1], x[3]), d = csub(x[1], x[3]);
        // forward transform: multiply d by -i
        const cpx<T> dmi = {d.y, -d.x};
        x[0] = cadd(a, c);
        x[1] = cadd(b, dmi);
        x[2] = csub(a, c);
        x[3] = csub(b, dmi);
    } else {  // R == 3, omega = exp(-2 pi i / 3)
        const T s3 = T(0.86602540378443864676);
        const cpx<T> a = x[0], b = x[1], c = x[2];
        const cpx<T> s = cadd(b, c), df = csub(b, c);
        const cpx<T> m = {a.x - T(0.5) * s.x, a.y - T(0.5) * s.y};
        // -i * s3 * (b - c)
        const cpx<T> r = {s3 * df.y, -s3 * df.x};
        x[0] = cadd(a, s);
        x[1] = cadd(m, r);
        x[2] = csub(m, r);
    }
}

// One Stockham stage: butterflies i = tid + q * blockDim (i < n/R), k = i mod p,
// inputs buf[i + t n/R], twiddle exp(-2 pi i t k / (p R)), outputs at
// (i - k) R + k + t p.  All reads complete before any write (barrier).
template <typename T, int VMAX, int R>
__device__ __forceinline__ void fft_stage(cpx<T> *buf, int n, int p, const cpx<T> *__restrict__ tw) {
    constexpr int NB = (VMAX + R - 1) / R;
    const int m = n / R;
    cpx<T> x[NB][R];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = threadIdx.x + q * blockDim.x;
        if (i < m) {
#pragma unroll
            for (int t = 0; t < R; ++t) x[q][t] = buf[i + t * m];
        }
    }
    __syncthreads();
    const int tstep = n / (p * R);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = threadIdx.x + q * blockDim.x;
        if (i < m) {
            const int k = i % p;
#pragma unroll
            for (int t = 1; t < R; ++t) x[q][t] = cmul(x[q][t], tw[t * k * tstep]);
            small_dft<T, R>(x[q]);
            const int j = (i - k) * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) buf[j + t * p] = x[q][t];
        }
    }
    __syncthreads();
}

template <typename T, int VMAX>
__device__ void fft_lds(cpx<T> *buf, int n, uint32_t radices, int nstages, const cpx<T> *__restrict__ tw) {
    int p = 1;
    for (int s = 0; s < nstages; ++s) {
        const int R = (radices >> (2 * s)) & 3;   // 0 -> 4
        if (R == 2) {
            fft_stage<T, VMAX, 2>(buf, n, p, tw);
            p *= 2;
        } else if (R == 3) {
            fft_stage<T, VMAX, 3>(buf, n, p, tw);
            p *= 3;
        } else {
            fft_stage<T, VMAX, 4>(buf, n, p, tw);
            p *= 4;
        }
    }
}

__device__ __forceinline__ int makhoul_src(int j, int n) {
    return j < (n + 1) / 2 ? 2 * j : 2 * (n - 1 - j) + 1;
}

struct AxisArgs {
    int n, inner;
    long long nlines;
    uint32_t radices;
    int nstages;
};

// Forward DCT-II along one axis for two lines per block.  The input is
// a - b when `b` is non-null (residual tgt - rho); when `zero_b` is set the
// consumed entries of b are cleared afterwards (rho is re-zeroed for the
// next deposition).
template <typename T, int VMAX>
__global__ void __launch_bounds__(256)
dct2_lines_kernel(const T *a, T *b, T *out, AxisArgs ax, const cpx<T> *__restrict__ tw,
                  const cpx<T> *__restrict__ qw, int zero_b, const int32_t *__restrict__ done)
{
    if (done != nullptr && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<T> *buf = reinterpret_cast<cpx<T> *>(smem);
    const int n = ax.n, inner = ax.inner;
    const long long La = 2LL * blockIdx.x, Lb = La + 1;
    const bool hasb = Lb < ax.nlines;
    const long long ba = line_base(La, n, inner), bb = hasb ? line_base(Lb, n, inner) : 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const long long s = (long long)makhoul_src(j, n) * inner;
        T xa = a[ba + s];
        T xb = hasb ? a[bb + s] : T(0);
        if (b != nullptr) {
            xa -= b[ba + s];
            if (hasb) xb -= b[bb + s];
        }
        buf[j] = {xa, xb};
    }
    __syncthreads();
    if (zero_b && b != nullptr) {
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            b[ba + (long long)j * inner] = T(0);
            if (hasb) b[bb + (long long)j * inner] = T(0);
        }
    }
    fft_lds<T, VMAX>(buf, n, ax.radices, ax.nstages, tw);
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const cpx<T> z = buf[k];
        const cpx<T> zc = conj_(buf[k == 0 ? 0 : n - k]);
        const cpx<T> va = {T(0.5) * (z.x + zc.x), T(0.5) * (z.y + zc.y)};
        const cpx<T> dd = csub(z, zc);
        const cpx<T> vb = {T(0.5) * dd.y, T(-0.5) * dd.x};
        const cpx<T> w = qw[k];   // exp(-i pi k / (2n))
        out[ba + (long long)k * inner] = w.x * va.x - w.y * va.y;
        if (hasb) out[bb + (long long)k * inner] = w.x * vb.x - w.y * vb.y;
    }
}

// Inverse (DCT-III / n) along one axis for two lines per block.  With
// `base` non-null the result is written as out = base + (*scale) * x (the
// gradient step p + sigma g, sigma read from device memory).
template <typename T, int VMAX>
__global__ void __launch_bounds__(256)
dct3_lines_kernel(const T *in, T *out, const T *base, const double *scale, AxisArgs ax,
                  const cpx<T> *__restrict__ tw, const cpx<T> *__restrict__ qw,
                  const int32_t *__restrict__ done)
{
    if (done != nullptr && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<T> *buf = reinterpret_cast<cpx<T> *>(smem);
    const int n = ax.n, inner = ax.inner;
    const long long La = 2LL * blockIdx.x, Lb = La + 1;
    const bool hasb = Lb < ax.nlines;
    const long long ba = line_base(La, n, inner), bb = hasb ? line_base(Lb, n, inner) : 0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const long long s = (long long)k * inner;
        buf[k] = {in[ba + s], hasb ? in[bb + s] : T(0)};
    }
    __syncthreads();
    // W_k = X_k - i X_{n-k} (X_n = 0), V_k = exp(+i pi k/(2n)) W_k, Z = V_a + i V_b;
    // the inverse DFT is conj(DFT(conj(Z))) / n, so conj(Z) is staged.
    constexpr int KMAX = VMAX;
    cpx<T> zr[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        const int k = threadIdx.x + q * blockDim.x;
        if (k < n) {
            const cpx<T> xk = buf[k];
            const cpx<T> xr = k == 0 ? cpx<T>{T(0), T(0)} : buf[n - k];
            const cpx<T> w = conj_(qw[k]);
            const cpx<T> wa = {xk.x, -xr.x}, wb = {xk.y, -xr.y};
            const cpx<T> va = cmul(w, wa), vb = cmul(w, wb);
            const cpx<T> z = {va.x - vb.y, va.y + vb.x};
            zr[q] = conj_(z);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        const int k = threadIdx.x + q * blockDim.x;
        if (k < n) buf[k] = zr[q];
    }
    __syncthreads();
    fft_lds<T, VMAX>(buf, n, ax.radices, ax.nstages, tw);
    const T inv_n = T(1) / T(n);
    const T sc = scale != nullptr ? T(*scale) : T(1);
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const cpx<T> z = buf[j];   // conj of the inverse transform times n
        const long long s = (long long)makhoul_src(j, n) * inner;
        const T xa = z.x * inv_n, xb = -z.y * inv_n;
        if (base != nullptr) {
            out[ba + s] = base[ba + s] + sc * xa;
            if (hasb) out[bb + s] = base[bb + s] + sc * xb;
        } else {
            out[ba + s] = xa;
            if (hasb) out[bb + s] = xb;
        }
    }
}

// X_k /= lambda_k (zero mode set to 0) and the partial of
// sum_k prod_a(w_a / n_a) X_k^2 / lambda_k, w = 1 at k_a = 0 and 2 otherwise.
template <typename T>
__global__ void __launch_bounds__(kRedBlock)
spectral_divide_kernel(T *X, Grid g, const T *__restrict__ lam0, const T *__restrict__ lam1,
                       const T *__restrict__ lam2, double *__restrict__ part, const int32_t *__restrict__ done)
{
    if (done != nullptr && *done) return;
    __shared__ double sh[kRedBlock / kWave];
    double acc = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < g.N;
         idx += (long long)gridDim.x * blockDim.x) {
        long long r = idx;
        int k[3] = {0, 0, 0};
        for (int a = g.ndim - 1; a >= 0; --a) {
            k[a] = (int)(r % g.n[a]);
            r /= g.n[a];
        }
        const T lam = lam0[k[0]] + lam1[k[1]] + (g.ndim == 3 ? lam2[k[2]] : T(0));
        const T x = X[idx];
        if (idx == 0) {
            X[idx] = T(0);
        } else {
            const T y = x / lam;
            X[idx] = y;
            double w = 1.0;
            for (int a = 0; a < g.ndim; ++a) w *= (k[a] == 0 ? 1.0 : 2.0) / g.n[a];
            acc += w * (double)x * (double)y;
        }
    }
    const double s = block_reduce<R_SUM>(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T> constexpr int dct_vmax() { return 16; }

static int dct_block(int n) {
    int bd = 64;
    while (bd * 16 < n) bd <<= 1;   // n / blockDim <= 16 complex values per lane
    return bd;
}

template <typename T>
hipError_t launch_dct2_axis(const T *a, T *b, T *out, const AxisPlan &ap, long long N, int zero_b,
                            const void *tw, const void *qw, const int32_t *done, hipStream_t stream)
{
    AxisArgs ax{ap.n, ap.inner, N / ap.n, ap.radices, ap.nstages};
    const long long blocks = (ax.nlines + 1) / 2;
    const int bd = dct_block(ap.n);
    if (bd > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL((dct2_lines_kernel<T, 16>), dim3((unsigned)blocks), dim3(bd),
                       (size_t)ap.n * sizeof(cpx<T>), stream, a, b, out, ax,
                       (const cpx<T> *)tw, (const cpx<T> *)qw, zero_b, done);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dct3_axis(const T *in, T *out, const T *base, const double *scale, const AxisPlan &ap,
                            long long N, const void *tw, const void *qw, const int32_t *done,
                            hipStream_t stream)
{
    AxisArgs ax{ap.n, ap.inner, N / ap.n, ap.radices, ap.nstages};
    const long long blocks = (ax.nlines + 1) / 2;
    const int bd = dct_block(ap.n);
    if (bd > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL((dct3_lines_kernel<T, 16>), dim3((unsigned)blocks), dim3(bd),
                       (size_t)ap.n * sizeof(cpx<T>), stream, in, out, base, scale, ax,
                       (const cpx<T> *)tw, (const cpx<T> *)qw, done);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spectral_divide(T *X, const Grid &g, const T *lam0, const T *lam1, const T *lam2,
                                  double *part, int nblocks, const int32_t *done, hipStream_t stream)
{
    hipLaunchKernelGGL((spectral_divide_kernel<T>), dim3(nblocks), dim3(kRedBlock), 0, stream, X, g,
                       lam0, lam1, lam2, part, done);
    return hipGetLastError();
}

#define BFM_INST_DCT(T)                                                                                     \
    template hipError_t launch_dct2_axis<T>(const T *, T *, T *, const AxisPlan &, long long, int,          \
                                            const void *, const void *, const int32_t *, hipStream_t);      \
    template hipError_t launch_dct3_axis<T>(const T *, T *, const T *, const double *, const AxisPlan &,    \
                                            long long, const void *, const void *, const int32_t *,         \
                                            hipStream_t);                                                   \
    template hipError_t launch_spectral_divide<T>(T *, const Grid &, const T *, const T *, const T *,       \
                                                  double *, int, const int32_t *, hipStream_t);
BFM_INST_DCT(float)
BFM_INST_DCT(double)

}  // namespace bfm
