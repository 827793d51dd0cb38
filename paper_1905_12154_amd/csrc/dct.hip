// Neumann Poisson solve on the grid: g = (-Laplacian)^{-1}(f - mean f).
//
// Paper: the H^1 gradient is (-Laplacian)^{-1} of the mean-free first
// variation with zero Neumann data (H^1-gradient lemma, eq. gradients_J_I);
// the Laplace inversion uses the FFT (Section 4.3).  On the cell-centred grid
// the second-difference Neumann Laplacian is diagonalised by the DCT-II, with
// eigenvalues lambda_k = sum_a 4 sin^2(pi k_a / (2 n_a)) n_a^2, so
//     g = DCT3( DCT2(f) / lambda ),   zero mode dropped,
// and ||f - mean f||^2_{H^-1} = sum_k prod_a(w_a / n_a) X_k^2 / lambda_k with
// w = 1 at k_a = 0 and 2 otherwise (Parseval for the unnormalised DCT-II).
//
// Transforms along one axis at a time (separable), unnormalised:
//   DCT2:  X_k = sum_j x_j cos(pi k (2j+1) / (2n))
//   DCT3:  x_j = (X_0 + 2 sum_{k>0} X_k cos(pi k (2j+1) / (2n))) / n  (exact inverse)
// Each line is reordered (even samples forward, odd samples backward) so the
// DCT becomes one length-n complex DFT plus a quarter-wave twiddle (Makhoul's
// method); two real lines share one complex DFT (real and imaginary parts).
// The DFT is a Stockham auto-sort FFT in LDS with radix 16, 8, 4, 2 and 3
// stages (n = 2^a 3^b; radix-16 and radix-8 butterflies are done in
// registers), twiddles from a per-axis table.
//
// Passes (2D): forward along rows (input tgt - rho, rho cleared for the next
// deposition) -> along columns forward, divide by lambda, inverse (one
// kernel, G accumulated) -> inverse along rows writing p + sigma g.  3D adds a
// forward and an inverse pass along the middle axis.  Contiguous axes move
// 16-byte vectors per lane; strided axes process four adjacent lines per
// workgroup so every grid row is one 16-byte vector.
#include "common.hpp"
#include "launch.hpp"

namespace bfm {

template <typename T> struct v4t;
template <> struct v4t<float> { using type = float4; };
template <> struct v4t<double> { using type = double4; };

__device__ __forceinline__ int padc(int j) { return j + (j >> 4); }
__host__ __device__ inline int padc_len(int n) { return n + (n >> 4) + 1; }

__device__ __forceinline__ long long xcd_map(long long b, long long nb) {
    const long long q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// exp(-2 pi i e / 16) for 0 <= e < 16, exact to the type's rounding
template <typename T>
__device__ __forceinline__ cpx<T> w16(int e) {
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, r2 = 0.70710678118654752440;
    constexpr double cs[16] = {1, c1, r2, s1, 0, -s1, -r2, -c1, -1, -c1, -r2, -s1, 0, s1, r2, c1};
    constexpr double sn[16] = {0, s1, r2, c1, 1, c1, r2, s1, 0, -s1, -r2, -c1, -1, -c1, -r2, -s1};
    return {T(cs[e & 15]), T(-sn[e & 15])};
}

template <typename T>
__device__ __forceinline__ void dft4_inplace(cpx<T> &x0, cpx<T> &x1, cpx<T> &x2, cpx<T> &x3) {
    const cpx<T> a = cadd(x0, x2), b = csub(x0, x2);
    const cpx<T> c = cadd(x1, x3), d = csub(x1, x3);
    const cpx<T> dmi = {d.y, -d.x};   // -i d
    x0 = cadd(a, c);
    x1 = cadd(b, dmi);
    x2 = csub(a, c);
    x3 = csub(b, dmi);
}

// Products by the constant twiddles of the register radix-8/16 transforms:
// multiplications by -i and exp(-i pi/4)-type factors are spelled out.
template <typename T>
__device__ __forceinline__ cpx<T> mul_w16(cpx<T> x, int e) {
    if (e == 0) return x;
    if (e == 4) return {x.y, -x.x};
    return cmul(x, w16<T>(e));
}

template <typename T, int R>
__device__ __forceinline__ void small_dft(cpx<T> *x) {
    if constexpr (R == 16) {
        // decimation in frequency, 16 = 4 x 4: row DFTs over s of x[j + 4 s],
        // twiddles w16^(j r), column DFTs over j; output X[4 m + r]
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            dft4_inplace(x[j], x[j + 4], x[j + 8], x[j + 12]);
#pragma unroll
            for (int r = 1; r < 4; ++r) x[j + 4 * r] = mul_w16(x[j + 4 * r], j * r);
        }
        cpx<T> y[16];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            cpx<T> u0 = x[4 * r], u1 = x[4 * r + 1], u2 = x[4 * r + 2], u3 = x[4 * r + 3];
            dft4_inplace(u0, u1, u2, u3);
            y[r] = u0;
            y[4 + r] = u1;
            y[8 + r] = u2;
            y[12 + r] = u3;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) x[k] = y[k];
    } else if constexpr (R == 8) {
        // decimation in frequency, 8 = 2 x 4
        cpx<T> a[4], b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = cadd(x[j], x[j + 4]);
            b[j] = mul_w16(csub(x[j], x[j + 4]), 2 * j);
        }
        dft4_inplace(a[0], a[1], a[2], a[3]);
        dft4_inplace(b[0], b[1], b[2], b[3]);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            x[2 * m] = a[m];
            x[2 * m + 1] = b[m];
        }
    } else if constexpr (R == 2) {
        const cpx<T> a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const cpx<T> a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
        const cpx<T> c = cadd(x[1], x[3]), d = csub(x[1], x[3]);
        const cpx<T> dmi = {d.y, -d.x};   // -i d
        x[0] = cadd(a, c);
        x[1] = cadd(b, dmi);
        x[2] = csub(a, c);
        x[3] = csub(b, dmi);
    } else {   // R == 3, omega = exp(-2 pi i / 3)
        const T s3 = T(0.86602540378443864676);
        const cpx<T> a = x[0], b = x[1], c = x[2];
        const cpx<T> s = cadd(b, c), df = csub(b, c);
        const cpx<T> m = {a.x - T(0.5) * s.x, a.y - T(0.5) * s.y};
        const cpx<T> r = {s3 * df.y, -s3 * df.x};   // -i s3 (b - c)
        x[0] = cadd(a, s);
        x[1] = cadd(m, r);
        x[2] = csub(m, r);
    }
}

// tab[i] of a table in global memory, read with a global (not flat) load: a
// pointer argument of an out-of-line function carries no address space.
template <typename T>
__device__ __forceinline__ cpx<T> global_cpx(const cpx<T> *tab, int i) {
    using G = const T __attribute__((address_space(1)));
    const G *q = (const G *)tab;
    return {q[2 * i], q[2 * i + 1]};
}

// One Stockham stage on a padded LDS line (kept out of line: inlining all
// stages of a transform into one body multiplies its register footprint).
// The line starts `off` complex values into the workgroup's dynamic LDS: a
// pointer argument would reach an out-of-line function as a generic address
// and every access would become a flat instruction instead of an LDS one.
// Butterflies i = lt + q * bd
// (i < n/R), k = i mod p, inputs buf[i + t n/R], twiddle exp(-2 pi i t k/(p R)),
// outputs at (i - k) R + k + t p.  All reads of the block complete before any
// write (barrier); lines of one workgroup advance together.  tstep = n / (p R)
// comes from the caller; the radix-3 stages run last, so p is a power of two
// in every other stage and k = i mod p is a mask there.
// Division of a coefficient by the Laplacian's eigenvalue: float32 takes the
// hardware reciprocal (1 ulp), which is within the rounding the float32
// coefficients already carry; float64 divides.
template <typename T> __device__ __forceinline__ T lap_div(T x, T l)
{
    if constexpr (sizeof(T) == 4)
        return x * __builtin_amdgcn_rcpf(l);
    else
        return x / l;
}

template <typename T, int VMAX, int R>
__device__ __attribute__((noinline)) void fft_stage(int off, int n, int p, int tstep, int lt, int bd,
                                                    const cpx<T> *__restrict__ tw) {
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<T> *buf = reinterpret_cast<cpx<T> *>(smem) + off;
    constexpr int NB = (VMAX + R - 1) / R;
    const int m = n / R;
    auto kmod = [p](int i) { return R == 3 ? i % p : (i & (p - 1)); };
    // twiddles w^t, w = exp(-2 pi i k / (p R)): for radix 4, 8 and 16 one
    // table load of w and powers by products (w^2t = (w^t)^2,
    // w^(t+1) = w^t w: at most 6 products deep); the first stage (p = 1)
    // needs none.  Loaded before the barrier so the latency overlaps.
    cpx<T> w1[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = lt + q * bd;
        w1[q] = {T(1), T(0)};
        if (R >= 4 && p > 1 && i < m) w1[q] = global_cpx(tw, kmod(i) * tstep);
    }
    cpx<T> x[NB][R];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = lt + q * bd;
        if (i < m) {
#pragma unroll
            for (int t = 0; t < R; ++t) x[q][t] = buf[padc(i + t * m)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = lt + q * bd;
        if (i < m) {
            const int k = kmod(i);
            if constexpr (R >= 4) {
                if (p > 1) {
                    cpx<T> wp[R];
                    wp[1] = w1[q];
#pragma unroll
                    for (int t = 2; t < R; ++t) wp[t] = (t & 1) ? cmul(wp[t - 1], wp[1]) : cmul(wp[t / 2], wp[t / 2]);
#pragma unroll
                    for (int t = 1; t < R; ++t) x[q][t] = cmul(x[q][t], wp[t]);
                }
            } else {
#pragma unroll
                for (int t = 1; t < R; ++t) x[q][t] = cmul(x[q][t], global_cpx(tw, t * k * tstep));
            }
            small_dft<T, R>(x[q]);
            const int j = (i - k) * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) buf[padc(j + t * p)] = x[q][t];
        }
    }
    __syncthreads();
}

// Stage counts are packed as radices = n16 | n8 << 6 | n4 << 12 | n2 << 18 |
// n3 << 24 (stages in that order); one loop per radix keeps each stage's
// register footprint separate.
template <typename T, int VMAX>
__device__ void fft_lds(int off, int n, uint32_t radices, int lt, int bd, const cpx<T> *__restrict__ tw) {
    const int n16 = radices & 63, n8 = (radices >> 6) & 63, n4 = (radices >> 12) & 63;
    const int n2 = (radices >> 18) & 63, n3 = (radices >> 24) & 63;
    int p = 1, rest = n;   // rest = n / p
#pragma unroll 1
    for (int s = 0; s < n16; ++s) {
        fft_stage<T, VMAX, 16>(off, n, p, rest / 16, lt, bd, tw);
        p *= 16;
        rest /= 16;
    }
#pragma unroll 1
    for (int s = 0; s < n8; ++s) {
        fft_stage<T, VMAX, 8>(off, n, p, rest / 8, lt, bd, tw);
        p *= 8;
        rest /= 8;
    }
#pragma unroll 1
    for (int s = 0; s < n4; ++s) {
        fft_stage<T, VMAX, 4>(off, n, p, rest / 4, lt, bd, tw);
        p *= 4;
        rest /= 4;
    }
#pragma unroll 1
    for (int s = 0; s < n2; ++s) {
        fft_stage<T, VMAX, 2>(off, n, p, rest / 2, lt, bd, tw);
        p *= 2;
        rest /= 2;
    }
#pragma unroll 1
    for (int s = 0; s < n3; ++s) {
        fft_stage<T, VMAX, 3>(off, n, p, rest / 3, lt, bd, tw);
        p *= 3;
        rest /= 3;
    }
}

__device__ __forceinline__ int makhoul_src(int j, int n) {
    return j < (n + 1) / 2 ? 2 * j : 2 * (n - 1 - j) + 1;
}

struct DctArgs {
    int n, inner;
    long long nlines;
    uint32_t radices;
    int nstages;
    // fused divide: other-axis eigenvalue tables and sizes (2D: A only)
    int nA, nB;              // sizes of the other axes in line-index order (nB = 1 in 2D)
    int innerB;              // line index = kA * nB + kB
};

enum DctMode { DM_FWD = kDctFwd, DM_INV = kDctInv, DM_FUSED = kDctFused };

// This lane's entries tab[k0 + q step] (q < Q; indices past the line clamp
// to its last entry): every load is issued before the first is used, so the
// lane waits for the table once rather than once per index.
template <typename V, int Q>
__device__ __forceinline__ void lane_table(V (&out)[Q], const V *__restrict__ tab, int k0, int step, int n) {
#pragma unroll
    for (int q = 0; q < Q; ++q) out[q] = tab[min(k0 + q * step, n - 1)];
}

// After a forward FFT of z = v_a + i v_b in buf, the DCT-II coefficients of
// lines a and b at index k.
// z = buf[k], zr = buf[n - k] (buf[0] for k = 0), w = qw[k].
template <typename T>
__device__ __forceinline__ void dct2_post_v(cpx<T> z, cpx<T> zr, cpx<T> w, T &Xa, T &Xb) {
    const cpx<T> zc = conj_(zr);
    const cpx<T> va = {T(0.5) * (z.x + zc.x), T(0.5) * (z.y + zc.y)};
    const cpx<T> dd = csub(z, zc);
    const cpx<T> vb = {T(0.5) * dd.y, T(-0.5) * dd.x};
    Xa = w.x * va.x - w.y * va.y;
    Xb = w.x * vb.x - w.y * vb.y;
}

template <typename T>
__device__ __forceinline__ void dct2_post(const cpx<T> *buf, int n, int k, cpx<T> w, T &Xa, T &Xb) {
    const cpx<T> z = buf[padc(k)];
    const cpx<T> zc = conj_(buf[padc(k == 0 ? 0 : n - k)]);
    const cpx<T> va = {T(0.5) * (z.x + zc.x), T(0.5) * (z.y + zc.y)};
    const cpx<T> dd = csub(z, zc);
    const cpx<T> vb = {T(0.5) * dd.y, T(-0.5) * dd.x};
    // w = qw[k] = exp(-i pi k / (2n))
    Xa = w.x * va.x - w.y * va.y;
    Xb = w.x * vb.x - w.y * vb.y;
}

// Before an inverse: from coefficients (X_a[k], X_b[k]) staged in buf, the
// conjugate of Z_k = e^{i pi k/(2n)} ((X_a[k] - i X_a[n-k]) + i (X_b[k] - i X_b[n-k])).
// xk = (X_a[k], X_b[k]), xr = (X_a[n-k], X_b[n-k]) (zero for k = 0), qk = qw[k].
template <typename T>
__device__ __forceinline__ cpx<T> dct3_pre_v(cpx<T> xk, cpx<T> xr, cpx<T> qk) {
    const cpx<T> w = conj_(qk);
    const cpx<T> wa = {xk.x, -xr.x}, wb = {xk.y, -xr.y};
    const cpx<T> va = cmul(w, wa), vb = cmul(w, wb);
    return conj_(cpx<T>{va.x - vb.y, va.y + vb.x});
}

template <typename T>
__device__ __forceinline__ cpx<T> dct3_pre(const cpx<T> *buf, int n, int k, cpx<T> qk) {
    const cpx<T> xk = buf[padc(k)];
    const cpx<T> xr = k == 0 ? cpx<T>{T(0), T(0)} : buf[padc(n - k)];
    const cpx<T> w = conj_(qk);   // qk = qw[k]
    const cpx<T> wa = {xk.x, -xr.x}, wb = {xk.y, -xr.y};
    const cpx<T> va = cmul(w, wa), vb = cmul(w, wb);
    return conj_(cpx<T>{va.x - vb.y, va.y + vb.x});
}

// Sum over the block (blockDim.x a multiple of 64, at most 512); valid in thread 0.
__device__ __forceinline__ double block_sum_any(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) r += sh[i];
    __syncthreads();
    return r;
}

// Line transforms along one axis.  NPAIR pairs of lines (2 NPAIR lines) per
// workgroup, bd lanes per pair.  CONTIG: lines are contiguous (axis ndim-1,
// NPAIR = 1); otherwise four adjacent lines are read/written as 16-byte vectors.
// The body of one workgroup: line group `blk` (2 NPAIR lines from line
// 2 NPAIR blk); the workgroup's float64 partial (G, or the sum with dotw)
// goes to *gslot.
template <typename T, int VMAX, int NPAIR, int MODE, bool CONTIG>
__device__ __forceinline__ void
dct_lines_body(const T *a, T *b, T *out, const T *base, const double *scale, const DctArgs &ax, int zero_b,
               const cpx<T> *__restrict__ tw, const cpx<T> *__restrict__ qw, const T *__restrict__ lam0,
               const T *__restrict__ lamA, const T *__restrict__ lamB, double *__restrict__ gslot,
               const T *__restrict__ dotw, long long blk)
{
    // Vector loads per thread (the launch guarantees n <= 16 bd): contiguous
    // lines take n / (4 bd) <= 4 per line, the two-pair strided form
    // n / (2 bd) <= 8.  Each load loop issues all of them before the first
    // LDS write, so their latencies overlap.
    constexpr int kContigIt = 4, kStridedIt = 8;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[8];
    const int n = ax.n, inner = ax.inner;
    const int NPC = padc_len(n);
    const int bd = blockDim.x / NPAIR;
    const int pr = threadIdx.x / bd, lt = threadIdx.x - pr * bd;
    cpx<T> *buf = reinterpret_cast<cpx<T> *>(smem) + (size_t)pr * NPC;
    const long long L0 = blk * (2 * NPAIR);          // first line of the workgroup
    const long long La = L0 + 2 * pr, Lb = La + 1;   // this pair
    const bool hasa = La < ax.nlines, hasb = Lb < ax.nlines;
    const bool al16 = (((uintptr_t)a | (uintptr_t)out | (uintptr_t)(b != nullptr ? b : a) |
                        (uintptr_t)(base != nullptr ? base : a)) & 15) == 0;

    // ---------------------------------------------------------------- load
    if (MODE == DM_INV) {
        // coefficients (X_a[k], X_b[k]) into buf
        if (CONTIG) {
            const long long ba = La * n, bbb = Lb * n;
            const bool vec = (n & 3) == 0 && al16;
            if (vec) {
                // every load of the thread is issued before its first LDS write
                typename v4t<T>::type xa[kContigIt], xb[kContigIt];
#pragma unroll
                for (int q = 0; q < kContigIt; ++q) {
                    const int k4 = (lt + q * bd) * 4;
                    if (k4 < n) {
                        xa[q] = *reinterpret_cast<const typename v4t<T>::type *>(a + ba + k4);
                        if (hasb) xb[q] = *reinterpret_cast<const typename v4t<T>::type *>(a + bbb + k4);
                        else xb[q].x = xb[q].y = xb[q].z = xb[q].w = T(0);
                    }
                }
#pragma unroll
                for (int q = 0; q < kContigIt; ++q) {
                    const int k4 = (lt + q * bd) * 4;
                    if (k4 < n) {
                        buf[padc(k4)] = {xa[q].x, xb[q].x};
                        buf[padc(k4 + 1)] = {xa[q].y, xb[q].y};
                        buf[padc(k4 + 2)] = {xa[q].z, xb[q].z};
                        buf[padc(k4 + 3)] = {xa[q].w, xb[q].w};
                    }
                }
            } else {
                for (int k4 = lt * 4; k4 < n; k4 += bd * 4)
                    for (int e = 0; e < 4; ++e)
                        if (k4 + e < n) buf[padc(k4 + e)] = {hasa ? a[ba + k4 + e] : T(0), hasb ? a[bbb + k4 + e] : T(0)};
            }
        } else {
            const bool vec = NPAIR == 2 && (inner & 3) == 0 && (L0 % inner) + 4 <= inner && L0 + 4 <= ax.nlines && al16;
            const long long b0 = line_base(L0, n, inner);
            cpx<T> *buf0 = reinterpret_cast<cpx<T> *>(smem);
            cpx<T> *buf1 = buf0 + NPC;
            if (vec) {
                typename v4t<T>::type xs[kStridedIt];
#pragma unroll
                for (int q = 0; q < kStridedIt; ++q) {
                    const int k = threadIdx.x + q * blockDim.x;
                    if (k < n) xs[q] = *reinterpret_cast<const typename v4t<T>::type *>(a + b0 + (long long)k * inner);
                }
#pragma unroll
                for (int q = 0; q < kStridedIt; ++q) {
                    const int k = threadIdx.x + q * blockDim.x;
                    if (k < n) {
                        buf0[padc(k)] = {xs[q].x, xs[q].y};
                        buf1[padc(k)] = {xs[q].z, xs[q].w};
                    }
                }
            } else {
                for (int k = lt; k < n; k += bd)
                    buf[padc(k)] = {hasa ? a[line_base(La, n, inner) + (long long)k * inner] : T(0),
                                    hasb ? a[line_base(Lb, n, inner) + (long long)k * inner] : T(0)};
            }
        }
        __syncthreads();
        cpx<T> wq[VMAX];
        lane_table(wq, qw, lt, bd, n);
        cpx<T> zr[VMAX];
#pragma unroll
        for (int q = 0; q < VMAX; ++q) {
            const int k = lt + q * bd;
            if (k < n) zr[q] = dct3_pre(buf, n, k, wq[q]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < VMAX; ++q) {
            const int k = lt + q * bd;
            if (k < n) buf[padc(k)] = zr[q];
        }
    } else {
        // real samples, reordered: v_j = x_{2j}, v_{n-1-j} = x_{2j+1}
        if (CONTIG) {
            const long long ba = La * n, bbb = Lb * n;
            const bool vec = (n & 3) == 0 && al16;
            if (vec) {
                // all loads of a chunk are issued before its first LDS write
                constexpr int QN = sizeof(T) == 4 ? kContigIt : kContigIt / 2;
#pragma unroll
                for (int q0 = 0; q0 < kContigIt; q0 += QN) {
                    typename v4t<T>::type va[QN], vb[QN], ra[QN], rb[QN];
#pragma unroll
                    for (int q = 0; q < QN; ++q) {
                        const int j4 = (lt + (q0 + q) * bd) * 4;
                        if (j4 < n) {
                            va[q] = *reinterpret_cast<const typename v4t<T>::type *>(a + ba + j4);
                            if (hasb) vb[q] = *reinterpret_cast<const typename v4t<T>::type *>(a + bbb + j4);
                            if (b != nullptr) {
                                ra[q] = *reinterpret_cast<const typename v4t<T>::type *>(b + ba + j4);
                                if (hasb) rb[q] = *reinterpret_cast<const typename v4t<T>::type *>(b + bbb + j4);
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < QN; ++q) {
                        const int j4 = (lt + (q0 + q) * bd) * 4;
                        if (j4 >= n) continue;
                        T xa[4] = {va[q].x, va[q].y, va[q].z, va[q].w};
                        T xb[4] = {T(0), T(0), T(0), T(0)};
                        if (hasb) {
                            xb[0] = vb[q].x; xb[1] = vb[q].y; xb[2] = vb[q].z; xb[3] = vb[q].w;
                        }
                        if (b != nullptr) {
                            xa[0] -= ra[q].x; xa[1] -= ra[q].y; xa[2] -= ra[q].z; xa[3] -= ra[q].w;
                            if (hasb) {
                                xb[0] -= rb[q].x; xb[1] -= rb[q].y; xb[2] -= rb[q].z; xb[3] -= rb[q].w;
                            }
                            if (zero_b) {
                                typename v4t<T>::type z;
                                z.x = z.y = z.z = z.w = T(0);
                                *reinterpret_cast<typename v4t<T>::type *>(b + ba + j4) = z;
                                if (hasb) *reinterpret_cast<typename v4t<T>::type *>(b + bbb + j4) = z;
                            }
                        }
                        // x_{j4}, x_{j4+2} are even samples, x_{j4+1}, x_{j4+3} odd
                        buf[padc(j4 / 2)] = {xa[0], xb[0]};
                        buf[padc(j4 / 2 + 1)] = {xa[2], xb[2]};
                        buf[padc(n - 1 - j4 / 2)] = {xa[1], xb[1]};
                        buf[padc(n - 2 - j4 / 2)] = {xa[3], xb[3]};
                    }
                }
            } else {
                for (int j4 = lt * 4; j4 < n; j4 += bd * 4) {
                    #pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (j4 + e >= n) break;
                        const int jj = j4 + e;
                        T ya = hasa ? a[ba + jj] : T(0), yb = hasb ? a[bbb + jj] : T(0);
                        if (b != nullptr) {
                            if (hasa) ya -= b[ba + jj];
                            if (hasb) yb -= b[bbb + jj];
                            if (zero_b) {
                                if (hasa) b[ba + jj] = T(0);
                                if (hasb) b[bbb + jj] = T(0);
                            }
                        }
                        const int pos = (jj & 1) ? n - 1 - (jj >> 1) : (jj >> 1);
                        buf[padc(pos)] = {ya, yb};
                    }
                }
            }
        } else {
            const bool vec = NPAIR == 2 && (inner & 3) == 0 && (L0 % inner) + 4 <= inner && L0 + 4 <= ax.nlines && al16;
            const long long b0 = line_base(L0, n, inner);
            cpx<T> *buf0 = reinterpret_cast<cpx<T> *>(smem);
            cpx<T> *buf1 = buf0 + NPC;
            if (vec) {
                typename v4t<T>::type xs[kStridedIt];
#pragma unroll
                for (int q = 0; q < kStridedIt; ++q) {
                    const int j = threadIdx.x + q * blockDim.x;
                    if (j < n)
                        xs[q] = *reinterpret_cast<const typename v4t<T>::type *>(
                            a + b0 + (long long)makhoul_src(j, n) * inner);
                }
#pragma unroll
                for (int q = 0; q < kStridedIt; ++q) {
                    const int j = threadIdx.x + q * blockDim.x;
                    if (j < n) {
                        buf0[padc(j)] = {xs[q].x, xs[q].y};
                        buf1[padc(j)] = {xs[q].z, xs[q].w};
                    }
                }
            } else {
                for (int j = lt; j < n; j += bd) {
                    const long long s = (long long)makhoul_src(j, n) * inner;
                    buf[padc(j)] = {hasa ? a[line_base(La, n, inner) + s] : T(0),
                                    hasb ? a[line_base(Lb, n, inner) + s] : T(0)};
                }
            }
        }
    }
    __syncthreads();
    fft_lds<T, VMAX>(pr * NPC, n, ax.radices, lt, bd, tw);

    double gacc = 0.0;
    if (MODE == DM_FUSED) {
        // coefficients along this axis, divided by lambda, and the inverse's
        // input: each lane takes index pairs {u, n - u} (u = 0 .. n/2), whose
        // two FFT values give the coefficients at both indices and whose two
        // divided coefficients give the inverse's input at both, so the
        // divided coefficients never pass through LDS
        // eigenvalue and weight of the other axes for lines a and b
        T lra = T(0), lrb = T(0);
        double wra = 1.0, wrb = 1.0;
        {
            const long long Ls[2] = {La, Lb};
            for (int s = 0; s < 2; ++s) {
                const long long Lx = Ls[s] < ax.nlines ? Ls[s] : 0;
                const int kA = ax.nB == 1 ? (int)Lx : (int)(Lx / ax.nB), kB = ax.nB == 1 ? 0 : (int)(Lx % ax.nB);
                const T lr = lamA[kA] + (ax.nB > 1 ? lamB[kB] : T(0));
                const double wr = ((kA == 0) ? 1.0 : 2.0) / ax.nA * (ax.nB > 1 ? ((kB == 0) ? 1.0 : 2.0) / ax.nB : 1.0);
                if (s == 0) { lra = lr; wra = wr; } else { lrb = lr; wrb = wr; }
            }
        }
        constexpr int QU = VMAX / 2 + 1;   // n <= VMAX bd: n/2 + 1 <= QU bd pairs
        const int half = n / 2;
        cpx<T> wq1[QU], wq2[QU];
        T l01[QU], l02[QU];
        lane_table(wq1, qw, lt, bd, n);
        lane_table(l01, lam0, lt, bd, n);
#pragma unroll
        for (int q = 0; q < QU; ++q) {   // partner indices n - u (u = 0: itself)
            const int u = min(lt + q * bd, half);
            const int k2 = u == 0 ? 0 : n - u;
            wq2[q] = qw[k2];
            l02[q] = lam0[k2];
        }
        const double inv_n = 1.0 / n;   // c / n == c * (1 / n) exactly for c = 1, 2
        // buf[u] and buf[n - u] are read and written by this lane alone:
        // each pair goes back in place without a barrier
#pragma unroll
        for (int q = 0; q < QU; ++q) {
            const int u = lt + q * bd;
            if (u <= half) {
                const bool self = u == 0 || 2 * u == n;   // n - u is u itself (or k = 0)
                const cpx<T> z1 = buf[padc(u)], z2 = buf[padc(u == 0 ? 0 : n - u)];
                T Xa1, Xb1, Xa2, Xb2;
                dct2_post_v(z1, z2, wq1[q], Xa1, Xb1);
                dct2_post_v(z2, z1, wq2[q], Xa2, Xb2);
                const T la1 = l01[q] + lra, lb1 = l01[q] + lrb;
                const T la2 = l02[q] + lra, lb2 = l02[q] + lrb;
                const T ya1 = la1 > T(0) ? lap_div(Xa1, la1) : T(0), yb1 = lb1 > T(0) ? lap_div(Xb1, lb1) : T(0);
                const T ya2 = la2 > T(0) ? lap_div(Xa2, la2) : T(0), yb2 = lb2 > T(0) ? lap_div(Xb2, lb2) : T(0);
                const double wk1 = (u == 0 ? 1.0 : 2.0) * inv_n, wk2 = 2.0 * inv_n;
                if (hasa) gacc += wk1 * wra * (double)Xa1 * (double)ya1;
                if (hasb) gacc += wk1 * wrb * (double)Xb1 * (double)yb1;
                if (!self) {
                    if (hasa) gacc += wk2 * wra * (double)Xa2 * (double)ya2;
                    if (hasb) gacc += wk2 * wrb * (double)Xb2 * (double)yb2;
                }
                const cpx<T> y1 = {ya1, yb1}, y2 = {ya2, yb2};
                // the inverse's input at u (no partner coefficient at k = 0)
                // and at n - u
                buf[padc(u)] = dct3_pre_v(y1, u == 0 ? cpx<T>{T(0), T(0)} : (self ? y1 : y2), wq1[q]);
                if (!self) buf[padc(n - u)] = dct3_pre_v(y2, y1, wq2[q]);
            }
        }
        __syncthreads();
        fft_lds<T, VMAX>(pr * NPC, n, ax.radices, lt, bd, tw);
    }

    // --------------------------------------------------------------- store
    if (MODE == DM_FWD) {
        if (CONTIG) {
            const long long ba = La * n, bbb = Lb * n;
            const bool vec = (n & 3) == 0 && al16;
            // n <= 16 bd: at most kContigIt groups of four per lane
            cpx<T> wq[kContigIt][4];
#pragma unroll
            for (int it = 0; it < kContigIt; ++it) lane_table(wq[it], qw, (lt + it * bd) * 4, 1, n);
#pragma unroll
            for (int it = 0; it < kContigIt; ++it) {
                const int k4 = (lt + it * bd) * 4;
                if (k4 >= n) break;
                T Xa[4], Xb[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    Xa[e] = Xb[e] = T(0);
                    if (k4 + e < n) dct2_post(buf, n, k4 + e, wq[it][e], Xa[e], Xb[e]);
                }
                if (vec) {
                    typename v4t<T>::type oa, ob;
                    oa.x = Xa[0]; oa.y = Xa[1]; oa.z = Xa[2]; oa.w = Xa[3];
                    ob.x = Xb[0]; ob.y = Xb[1]; ob.z = Xb[2]; ob.w = Xb[3];
                    if (hasa) *reinterpret_cast<typename v4t<T>::type *>(out + ba + k4) = oa;
                    if (hasb) *reinterpret_cast<typename v4t<T>::type *>(out + bbb + k4) = ob;
                } else {
                    #pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (k4 + e >= n) break;
                        if (hasa) out[ba + k4 + e] = Xa[e];
                        if (hasb) out[bbb + k4 + e] = Xb[e];
                    }
                }
            }
        } else {
            const bool vec = NPAIR == 2 && (inner & 3) == 0 && (L0 % inner) + 4 <= inner && L0 + 4 <= ax.nlines && al16;
            const long long b0 = line_base(L0, n, inner);
            if (vec) {
                // thread owns (pair, k): gather both pairs through registers
                cpx<T> *buf0 = reinterpret_cast<cpx<T> *>(smem);
                cpx<T> *buf1 = buf0 + NPC;
                // n <= 16 bd = 8 blockDim: at most kStridedIt indices per lane
                cpx<T> wq[kStridedIt];
                lane_table(wq, qw, (int)threadIdx.x, (int)blockDim.x, n);
#pragma unroll
                for (int it = 0; it < kStridedIt; ++it) {
                    const int k = threadIdx.x + it * blockDim.x;
                    if (k >= n) break;
                    T a0, b0v, a1, b1v;
                    dct2_post(buf0, n, k, wq[it], a0, b0v);
                    dct2_post(buf1, n, k, wq[it], a1, b1v);
                    typename v4t<T>::type o;
                    o.x = a0; o.y = b0v; o.z = a1; o.w = b1v;
                    *reinterpret_cast<typename v4t<T>::type *>(out + b0 + (long long)k * inner) = o;
                }
            } else {
                for (int k = lt; k < n; k += bd) {
                    T Xa, Xb;
                    dct2_post(buf, n, k, qw[k], Xa, Xb);
                    if (hasa) out[line_base(La, n, inner) + (long long)k * inner] = Xa;
                    if (hasb) out[line_base(Lb, n, inner) + (long long)k * inner] = Xb;
                }
            }
        }
    } else {
        // inverse result: buf_j = n conj(z_j); x[src(j)] = Re z_j (line a), Im z_j (line b)
        const T inv_n = T(1) / T(n);
        const T sc = scale != nullptr ? T(*scale) : T(1);
        if (CONTIG) {
            const long long ba = La * n, bbb = Lb * n;
            const bool vec = (n & 3) == 0 && al16;
            if (vec) {
                // the reads of p and of the weights are issued before the outputs are formed
                constexpr int QN = sizeof(T) == 4 ? kContigIt : kContigIt / 2;
#pragma unroll
                for (int q0 = 0; q0 < kContigIt; q0 += QN) {
                    typename v4t<T>::type pa[QN], pb[QN], wa[QN], wb[QN];
#pragma unroll
                    for (int q = 0; q < QN; ++q) {
                        const int j4 = (lt + (q0 + q) * bd) * 4;
                        if (j4 < n) {
                            if (base != nullptr) {
                                pa[q] = *reinterpret_cast<const typename v4t<T>::type *>(base + ba + j4);
                                if (hasb) pb[q] = *reinterpret_cast<const typename v4t<T>::type *>(base + bbb + j4);
                            }
                            if (dotw != nullptr) {
                                wa[q] = *reinterpret_cast<const typename v4t<T>::type *>(dotw + ba + j4);
                                if (hasb) wb[q] = *reinterpret_cast<const typename v4t<T>::type *>(dotw + bbb + j4);
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < QN; ++q) {
                        const int j4 = (lt + (q0 + q) * bd) * 4;
                        if (j4 >= n) continue;
                    T xa[4], xb[4];
                    #pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        xa[e] = xb[e] = T(0);
                        if (j4 + e >= n) break;
                        const int jj = j4 + e;
                        const int pos = (jj & 1) ? n - 1 - (jj >> 1) : (jj >> 1);
                        const cpx<T> z = buf[padc(pos)];
                        xa[e] = z.x * inv_n;
                        xb[e] = -z.y * inv_n;
                    }
                        typename v4t<T>::type oa, ob;
                        oa.x = xa[0]; oa.y = xa[1]; oa.z = xa[2]; oa.w = xa[3];
                        ob.x = xb[0]; ob.y = xb[1]; ob.z = xb[2]; ob.w = xb[3];
                        if (base != nullptr) {
                            oa.x = pa[q].x + sc * oa.x; oa.y = pa[q].y + sc * oa.y;
                            oa.z = pa[q].z + sc * oa.z; oa.w = pa[q].w + sc * oa.w;
                            if (hasb) {
                                ob.x = pb[q].x + sc * ob.x; ob.y = pb[q].y + sc * ob.y;
                                ob.z = pb[q].z + sc * ob.z; ob.w = pb[q].w + sc * ob.w;
                            }
                        }
                        if (hasa) *reinterpret_cast<typename v4t<T>::type *>(out + ba + j4) = oa;
                        if (hasb) *reinterpret_cast<typename v4t<T>::type *>(out + bbb + j4) = ob;
                        if (dotw != nullptr) {   // sum out * dotw of the written values
                            gacc += (double)oa.x * wa[q].x + (double)oa.y * wa[q].y + (double)oa.z * wa[q].z +
                                    (double)oa.w * wa[q].w;
                            if (hasb)
                                gacc += (double)ob.x * wb[q].x + (double)ob.y * wb[q].y + (double)ob.z * wb[q].z +
                                        (double)ob.w * wb[q].w;
                        }
                    }
                }
            } else {
                for (int j4 = lt * 4; j4 < n; j4 += bd * 4) {
                    T xa[4], xb[4];
                    #pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        xa[e] = xb[e] = T(0);
                        if (j4 + e >= n) break;
                        const int jj = j4 + e;
                        const int pos = (jj & 1) ? n - 1 - (jj >> 1) : (jj >> 1);
                        const cpx<T> z = buf[padc(pos)];
                        xa[e] = z.x * inv_n;
                        xb[e] = -z.y * inv_n;
                    }
                    #pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (j4 + e >= n) break;
                        const long long ia = ba + j4 + e, ib = bbb + j4 + e;
                        if (hasa) {
                            out[ia] = base != nullptr ? base[ia] + sc * xa[e] : xa[e];
                            if (dotw != nullptr) gacc += (double)out[ia] * dotw[ia];
                        }
                        if (hasb) {
                            out[ib] = base != nullptr ? base[ib] + sc * xb[e] : xb[e];
                            if (dotw != nullptr) gacc += (double)out[ib] * dotw[ib];
                        }
                    }
                }
            }
        } else {
            const bool vec = NPAIR == 2 && (inner & 3) == 0 && (L0 % inner) + 4 <= inner && L0 + 4 <= ax.nlines && al16;
            const long long b0 = line_base(L0, n, inner);
            if (vec) {
                cpx<T> *buf0 = reinterpret_cast<cpx<T> *>(smem);
                cpx<T> *buf1 = buf0 + NPC;
                for (int j = threadIdx.x; j < n; j += blockDim.x) {
                    const cpx<T> z0 = buf0[padc(j)], z1 = buf1[padc(j)];
                    typename v4t<T>::type o;
                    o.x = z0.x * inv_n; o.y = -z0.y * inv_n; o.z = z1.x * inv_n; o.w = -z1.y * inv_n;
                    const long long addr = b0 + (long long)makhoul_src(j, n) * inner;
                    if (base != nullptr) {
                        const typename v4t<T>::type p = *reinterpret_cast<const typename v4t<T>::type *>(base + addr);
                        o.x = p.x + sc * o.x; o.y = p.y + sc * o.y; o.z = p.z + sc * o.z; o.w = p.w + sc * o.w;
                    }
                    *reinterpret_cast<typename v4t<T>::type *>(out + addr) = o;
                }
            } else {
                for (int j = lt; j < n; j += bd) {
                    const cpx<T> z = buf[padc(j)];
                    const long long s = (long long)makhoul_src(j, n) * inner;
                    const T xa = z.x * inv_n, xb = -z.y * inv_n;
                    if (hasa) {
                        const long long ia = line_base(La, n, inner) + s;
                        out[ia] = base != nullptr ? base[ia] + sc * xa : xa;
                    }
                    if (hasb) {
                        const long long ib = line_base(Lb, n, inner) + s;
                        out[ib] = base != nullptr ? base[ib] + sc * xb : xb;
                    }
                }
            }
        }
    }
    if (MODE == DM_FUSED || (MODE == DM_INV && CONTIG && dotw != nullptr)) {   // uniform
        const double gs = block_sum_any(gacc, red);
        if (threadIdx.x == 0) *gslot = gs;
    }
}

template <typename T, int VMAX, int NPAIR, int MODE, bool CONTIG>
__global__ void __launch_bounds__(512)
dct_lines_kernel(const T *a, T *b, T *out, const T *base, const double *scale, DctArgs ax, int zero_b,
                 const cpx<T> *__restrict__ tw, const cpx<T> *__restrict__ qw, const T *__restrict__ lam0,
                 const T *__restrict__ lamA, const T *__restrict__ lamB, double *__restrict__ gpart,
                 const T *__restrict__ dotw, const int32_t *__restrict__ done)
{
    if (done != nullptr && *done) return;
    dct_lines_body<T, VMAX, NPAIR, MODE, CONTIG>(a, b, out, base, scale, ax, zero_b, tw, qw, lam0, lamA, lamB,
                                                 gpart != nullptr ? gpart + blockIdx.x : nullptr, dotw,
                                                 xcd_map(blockIdx.x, gridDim.x));
}

// ------------------------------------------------------------ multi-pair
// One pass of the 2D Poisson solve for every pair of a batch in one launch:
//   DM_FWD:   rows of tgt - rho into F (rho cleared), axis 1;
//   DM_FUSED: columns of F forward, divided by lambda, G partials, inverse;
//   DM_INV:   rows of F back, p += sigma g, partials of sum p * tgt.
// role 0 is the phi-step (p, tgt) = (phi, nu), role 1 the psi-step (psi, mu).
// Partials go to the pair's own slots at the workgroup's index inside the pair.
template <typename T, int NPAIR, int MODE, bool CONTIG>
__global__ void __launch_bounds__(512)
dct_multi_kernel(const BatchHead *__restrict__ tab, BatchIdx bi, int role)
{
    int lo = 0, hi = bi.np - 1;   // largest pair with off[pair] <= blockIdx.x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bi.off[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const PairDev &P = reinterpret_cast<const PairDev *>(tab + 1)[lo];
    if ((tab->done_mask >> lo) & 1ull) return;
    const long long blk = (long long)blockIdx.x - bi.off[lo];
    T *p = (T *)(role ? P.psi : P.phi);
    const T *tgt = (const T *)(role ? P.mu : P.nu);
    const int ax_ = MODE == DM_FUSED ? 0 : 1;
    DctArgs ax{};
    ax.n = ax_ == 0 ? P.n0 : P.n1;
    ax.inner = ax_ == 0 ? P.n1 : 1;
    ax.nlines = ax_ == 0 ? P.n1 : P.n0;
    ax.radices = P.radices[ax_];
    ax.nA = P.n1;
    ax.nB = 1;
    ax.innerB = 1;
    const cpx<T> *tw = (const cpx<T> *)(P.tables + P.tw[ax_]);
    const cpx<T> *qw = (const cpx<T> *)(P.tables + P.qw[ax_]);
    if (MODE == DM_FWD)
        dct_lines_body<T, 16, NPAIR, MODE, CONTIG>(tgt, (T *)P.rho, (T *)P.F, nullptr, nullptr, ax, 1, tw, qw, nullptr,
                                                   nullptr, nullptr, nullptr, nullptr, blk);
    else if (MODE == DM_FUSED)
        dct_lines_body<T, 16, NPAIR, MODE, CONTIG>((T *)P.F, nullptr, (T *)P.F, nullptr, nullptr, ax, 0, tw, qw,
                                                   (const T *)(P.tables + P.lam[0]), (const T *)(P.tables + P.lam[1]),
                                                   nullptr, P.gpart + blk, nullptr, blk);
    else
        dct_lines_body<T, 16, NPAIR, MODE, CONTIG>((T *)P.F, nullptr, p, p, &P.st->sigma, ax, 0, tw, qw, nullptr,
                                                   nullptr, nullptr, P.part + S_Q_TGT * P.slot_len + blk, tgt, blk);
}

long long dct_multi_inv_parts(int n0) { return (n0 + 1) / 2; }

static int dct_block(int n) {
    int bd = 64;
    while (bd * 16 < n) bd <<= 1;   // n / bd <= 16 complex values per lane
    return bd;
}

template <typename T, int NPAIR, int MODE, bool CONTIG>
static hipError_t launch_dct_impl(const T *a, T *b, T *out, const T *base, const double *scale, const DctArgs &ax,
                                  int zero_b, const void *tw, const void *qw, const T *lam0, const T *lamA,
                                  const T *lamB, double *gpart, const int32_t *done, hipStream_t stream,
                                  const T *dotw = nullptr)
{
    const int bd = dct_block(ax.n);
    if (bd * NPAIR > 512) return hipErrorInvalidValue;
    const size_t smem = (size_t)NPAIR * padc_len(ax.n) * sizeof(cpx<T>);
    const long long blocks = (ax.nlines + 2 * NPAIR - 1) / (2 * NPAIR);
    static size_t lds_limit[kMaxDevices] = {};
    hipError_t e = raise_dyn_lds((const void *)dct_lines_kernel<T, 16, NPAIR, MODE, CONTIG>, smem, lds_limit);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((dct_lines_kernel<T, 16, NPAIR, MODE, CONTIG>), dim3((unsigned)blocks), dim3(bd * NPAIR),
                       smem, stream, a, b, out, base, scale, ax, zero_b, (const cpx<T> *)tw, (const cpx<T> *)qw,
                       lam0, lamA, lamB, gpart, dotw, done);
    return hipGetLastError();
}

static DctArgs make_args(const AxisPlan &ap, long long N) {
    DctArgs ax{};
    ax.n = ap.n;
    ax.inner = ap.inner;
    ax.nlines = N / ap.n;
    ax.radices = ap.radices;
    ax.nstages = ap.nstages;
    ax.nA = 1;
    ax.nB = 1;
    ax.innerB = 1;
    return ax;
}

// Strided axes use two pairs (four lines) per workgroup when LDS allows.
template <typename T> static bool dct_two_pairs(int n) {
    return (size_t)2 * padc_len(n) * sizeof(cpx<T>) <= 150 * 1024;
}

template <typename T>
hipError_t launch_dct_fwd(const T *a, T *b, T *out, const AxisPlan &ap, long long N, int zero_b, const void *tw,
                          const void *qw, const int32_t *done, hipStream_t stream)
{
    const DctArgs ax = make_args(ap, N);
    if (ap.inner == 1)
        return launch_dct_impl<T, 1, DM_FWD, true>(a, b, out, nullptr, nullptr, ax, zero_b, tw, qw, nullptr, nullptr,
                                                   nullptr, nullptr, done, stream);
    if (b != nullptr) return hipErrorInvalidValue;
    if (dct_two_pairs<T>(ap.n))
        return launch_dct_impl<T, 2, DM_FWD, false>(a, nullptr, out, nullptr, nullptr, ax, 0, tw, qw, nullptr,
                                                    nullptr, nullptr, nullptr, done, stream);
    return launch_dct_impl<T, 1, DM_FWD, false>(a, nullptr, out, nullptr, nullptr, ax, 0, tw, qw, nullptr, nullptr,
                                                nullptr, nullptr, done, stream);
}

template <typename T>
hipError_t launch_dct_inv(const T *in, T *out, const T *base, const double *scale, const AxisPlan &ap, long long N,
                          const void *tw, const void *qw, const int32_t *done, hipStream_t stream, const T *dotw,
                          double *dotpart)
{
    const DctArgs ax = make_args(ap, N);
    if (ap.inner == 1)
        return launch_dct_impl<T, 1, DM_INV, true>(in, nullptr, out, base, scale, ax, 0, tw, qw, nullptr, nullptr,
                                                   nullptr, dotpart, done, stream, dotw);
    if (dotw != nullptr) return hipErrorInvalidValue;   // the sum is fused into contiguous passes only
    if (dct_two_pairs<T>(ap.n))
        return launch_dct_impl<T, 2, DM_INV, false>(in, nullptr, out, base, scale, ax, 0, tw, qw, nullptr, nullptr,
                                                    nullptr, nullptr, done, stream);
    return launch_dct_impl<T, 1, DM_INV, false>(in, nullptr, out, base, scale, ax, 0, tw, qw, nullptr, nullptr,
                                                nullptr, nullptr, done, stream);
}

// Along axis 0: forward, divide by lambda = lam0[k0] + lamA[kA] (+ lamB[kB]),
// inverse; per-workgroup partials of G into gpart (one per workgroup).
template <typename T>
hipError_t launch_dct_fused(T *X, const AxisPlan &ap0, long long N, int nA, int nB, const void *tw, const void *qw,
                            const T *lam0, const T *lamA, const T *lamB, double *gpart, int *nparts,
                            const int32_t *done, hipStream_t stream)
{
    DctArgs ax = make_args(ap0, N);
    ax.nA = nA;
    ax.nB = nB;
    const bool two = dct_two_pairs<T>(ap0.n) && ap0.inner > 1;
    const int per = two ? 4 : 2;
    *nparts = (int)((ax.nlines + per - 1) / per);
    if (ap0.inner == 1) return hipErrorInvalidValue;
    if (two)
        return launch_dct_impl<T, 2, DM_FUSED, false>(X, nullptr, X, nullptr, nullptr, ax, 0, tw, qw, lam0, lamA,
                                                      lamB, gpart, done, stream);
    return launch_dct_impl<T, 1, DM_FUSED, false>(X, nullptr, X, nullptr, nullptr, ax, 0, tw, qw, lam0, lamA, lamB,
                                                  gpart, done, stream);
}

long long dct_fused_parts(int n0, long long N, size_t esz)
{
    const bool two = (size_t)2 * padc_len(n0) * 2 * esz <= 150 * 1024;
    const long long nl = N / n0;
    return two ? (nl + 3) / 4 : (nl + 1) / 2;
}

template <typename T>
hipError_t launch_dct_multi(const BatchHead *tab, const int *n0s, const int *n1s, int np, int role, int mode,
                            hipStream_t stream)
{
    if (np < 1 || np > kBatchChunk) return hipErrorInvalidValue;
    BatchIdx bi{};
    bi.np = np;
    int bd = 64, nmax = 1;
    for (int p = 0; p < np; ++p) {
        const int n = mode == DM_FUSED ? n0s[p] : n1s[p];
        if ((n1s[p] & 3) != 0) return hipErrorInvalidValue;
        const int b = dct_block(n);
        bd = b > bd ? b : bd;
        nmax = n > nmax ? n : nmax;
        const long long lines = mode == DM_FUSED ? n1s[p] : n0s[p];
        bi.off[p + 1] = bi.off[p] + (int)(mode == DM_FUSED ? (lines + 3) / 4 : (lines + 1) / 2);
    }
    const int npair = mode == DM_FUSED ? 2 : 1;
    if (bd * npair > 512) return hipErrorInvalidValue;
    const size_t smem = (size_t)npair * padc_len(nmax) * sizeof(cpx<T>);
    static size_t lds_limit[3][kMaxDevices] = {};
    const dim3 grid((unsigned)bi.off[np]), block(bd * npair);
    hipError_t e = hipSuccess;
    if (mode == DM_FWD) {
        e = raise_dyn_lds((const void *)dct_multi_kernel<T, 1, DM_FWD, true>, smem, lds_limit[0]);
        if (e == hipSuccess)
            hipLaunchKernelGGL((dct_multi_kernel<T, 1, DM_FWD, true>), grid, block, smem, stream, tab, bi, role);
    } else if (mode == DM_FUSED) {
        e = raise_dyn_lds((const void *)dct_multi_kernel<T, 2, DM_FUSED, false>, smem, lds_limit[1]);
        if (e == hipSuccess)
            hipLaunchKernelGGL((dct_multi_kernel<T, 2, DM_FUSED, false>), grid, block, smem, stream, tab, bi, role);
    } else if (mode == DM_INV) {
        e = raise_dyn_lds((const void *)dct_multi_kernel<T, 1, DM_INV, true>, smem, lds_limit[2]);
        if (e == hipSuccess)
            hipLaunchKernelGGL((dct_multi_kernel<T, 1, DM_INV, true>), grid, block, smem, stream, tab, bi, role);
    } else {
        return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

#define BFM_INST_DCT(T)                                                                                       \
    template hipError_t launch_dct_fwd<T>(const T *, T *, T *, const AxisPlan &, long long, int, const void *, \
                                          const void *, const int32_t *, hipStream_t);                         \
    template hipError_t launch_dct_inv<T>(const T *, T *, const T *, const double *, const AxisPlan &,        \
                                          long long, const void *, const void *, const int32_t *,             \
                                          hipStream_t, const T *, double *);                                                       \
    template hipError_t launch_dct_fused<T>(T *, const AxisPlan &, long long, int, int, const void *,         \
                                            const void *, const T *, const T *, const T *, double *, int *,    \
                                            const int32_t *, hipStream_t);
BFM_INST_DCT(float)
BFM_INST_DCT(double)
template hipError_t launch_dct_multi<float>(const BatchHead *, const int *, const int *, int, int, int, hipStream_t);
template hipError_t launch_dct_multi<double>(const BatchHead *, const int *, const int *, int, int, int, hipStream_t);

}  // namespace bfm
