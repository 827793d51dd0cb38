// One-dimensional c-transform steps for the separable power cost
// h(z) = |z|^p / p, p > 1 (eq. p_costs), by the monotone divide and conquer
// of Section 4.1 (general costs).
//
// Along one line of n cell-centred points, out_i = min_j H_|i-j| + u_j with
// H_k = (k/n)^p / p and u = sgn * in.  Because h is strictly convex the
// matrix H_|i-j| + u_j has the Monge property, so the leftmost minimiser
// j*(i) is non-decreasing in i: the minimiser of a row is trapped between
// those of any two rows around it.  Row 0 is found by a full scan; then for
// s = 2^K, ..., 2, 1 (2^K the largest power of two below n) every row
// i = s (2m + 1) searches only [j*(i - s), j*(i + s)] (n - 1 when i + s >= n),
// rows whose neighbours at distance s were found at an earlier level.  A
// level costs at most n + (number of rows) evaluations, so a line costs
// O(n log n).
//
// GPU organisation: one line per workgroup at a time, persistent over
// lines.  A level is spread over the 256 lanes as one flattened run of
// (row, column) pairs: a block scan of the bracket lengths gives each row's
// offset, each lane walks one equal share of the run (finding its first row
// by binary search) and folds the minimum of every row piece it saw into
// the row's slot with an LDS atomic min on an order-preserving integer key.
// float32 packs (key << 32 | j), so one atomic yields the leftmost
// minimiser; float64 takes a second walk that offers j only where the value
// equals the row minimum.  Neighbouring lines of a strided axis are taken
// by workgroups on the same XCD at the same time, so their strided accesses
// meet in that XCD's L2.
#include <climits>

#include "common.hpp"
#include "launch.hpp"

namespace bfm {

constexpr int kDcBlock = 256;

__device__ __forceinline__ unsigned int order_key(float v) {
    const unsigned int b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ unsigned long long order_key(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// blocks on one XCD (b mod 8) take consecutive indices
__device__ __forceinline__ long long dc_xcd_block(long long b, long long nb) {
    const long long q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// LDS layout for a line of n points (rmax = n / 2 + 1 rows per level at most)
template <typename T> __host__ __device__ constexpr size_t dc_smem_bytes(int n) {
    const size_t rmax = (size_t)n / 2 + 1;
    return rmax * 8                                  // row keys
           + 2 * (size_t)n * sizeof(T)               // u, H
           + (rmax + 1) * 4                          // row offsets
           + (sizeof(T) == 8 ? rmax * 4 : 0)         // leftmost minimiser (float64)
           + (size_t)n * 2;                          // j*(i)
}

template <typename T>
__global__ void __launch_bounds__(kDcBlock)
ct_dc_kernel(const T *in, T *out, int n, int inner, long long nlines, T sgn, double p, const int32_t *done)
{
    if (done != nullptr && *done) return;
    extern __shared__ __align__(16) unsigned char dsm[];
    __shared__ int wtot[kDcBlock / kWave];
    const int rmax = n / 2 + 1;
    unsigned long long *key = (unsigned long long *)dsm;
    T *u = (T *)(key + rmax);
    T *H = u + n;
    int *pre = (int *)(H + n);
    int *amin = pre + rmax + 1;
    unsigned short *arg = (unsigned short *)(amin + (sizeof(T) == 8 ? rmax : 0));
    const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;

    // H_k = (k h)^p / p, evaluated in float64
    const double hh = 1.0 / n;
    for (int k = t; k < n; k += kDcBlock) H[k] = (T)(pow((double)k * hh, p) / p);
    int top = 1;
    while (2 * top < n) top *= 2;

    for (long long L = dc_xcd_block(blockIdx.x, gridDim.x); L < nlines; L += gridDim.x) {
        const long long base = (L / inner) * (long long)n * inner + (L % inner);
        __syncthreads();   // the previous line's last readers of u and arg
        for (int j = t; j < n; j += kDcBlock) u[j] = sgn * in[base + (long long)j * inner];
        __syncthreads();

        // level s = 0 is row 0 over [0, n - 1]; then s = top, ..., 1
        for (int s = 0;; s = (s == 0 ? top : s >> 1)) {
            const int R = s == 0 ? 1 : (n + s - 1) / (2 * s);
            auto row_i = [&](int m) { return s == 0 ? 0 : s * (2 * m + 1); };
            auto row_lo = [&](int m) { return s == 0 ? 0 : (int)arg[row_i(m) - s]; };
            auto row_hi = [&](int m) {
                const int i = row_i(m);
                return (s == 0 || i + s >= n) ? n - 1 : (int)arg[i + s];
            };
            // 1. bracket lengths and their exclusive scan (contiguous rows per lane)
            const int cpt = (R + kDcBlock - 1) / kDcBlock;
            const int m0 = t * cpt, m1 = min(R, m0 + cpt);
            int lsum = 0;
            for (int m = m0; m < m1; ++m) lsum += row_hi(m) - row_lo(m) + 1;
            int incl = lsum;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int y = __shfl_up(incl, o, kWave);
                if (lane >= o) incl += y;
            }
            if (lane == kWave - 1) wtot[wv] = incl;
            __syncthreads();
            int off = 0, W = 0;
#pragma unroll
            for (int w = 0; w < kDcBlock / kWave; ++w) {
                off += w < wv ? wtot[w] : 0;
                W += wtot[w];
            }
            int run = off + incl - lsum;
            for (int m = m0; m < m1; ++m) {
                pre[m] = run;
                run += row_hi(m) - row_lo(m) + 1;
                key[m] = ~0ull;
                if constexpr (sizeof(T) == 8) amin[m] = INT_MAX;
            }
            if (t == 0) pre[R] = W;
            __syncthreads();   // also: every lane has read wtot before the next level writes it

            // 2. walk an equal share of the flattened (row, column) run
            const int cw = (W + kDcBlock - 1) / kDcBlock;
            const int k0 = t * cw, k1 = min(W, k0 + cw);
            int mfirst = 0;
            if (k0 < k1) {
                int a = 0, b = R - 1;
                while (a < b) {
                    const int mid = (a + b + 1) >> 1;
                    if (pre[mid] <= k0) a = mid; else b = mid - 1;
                }
                mfirst = a;
                int m = a, i = row_i(m), jb = row_lo(m) - pre[m], kend = pre[m + 1];
                unsigned long long best = ~0ull;
                for (int k = k0; k < k1; ++k) {
                    if (k >= kend) {
                        atomicMin(&key[m], best);
                        best = ~0ull;
                        ++m;
                        i = row_i(m);
                        jb = row_lo(m) - pre[m];
                        kend = pre[m + 1];
                    }
                    const int j = jb + k;
                    const T v = H[abs(i - j)] + u[j];
                    unsigned long long kk;
                    if constexpr (sizeof(T) == 4)
                        kk = ((unsigned long long)order_key(v) << 32) | (unsigned int)j;
                    else
                        kk = order_key(v);
                    best = kk < best ? kk : best;
                }
                atomicMin(&key[m], best);
            }
            __syncthreads();
            if constexpr (sizeof(T) == 8) {
                // leftmost column attaining each row's minimum
                if (k0 < k1) {
                    int m = mfirst, i = row_i(m), jb = row_lo(m) - pre[m], kend = pre[m + 1];
                    unsigned long long target = key[m];
                    bool found = false;
                    for (int k = k0; k < k1; ++k) {
                        if (k >= kend) {
                            ++m;
                            i = row_i(m);
                            jb = row_lo(m) - pre[m];
                            kend = pre[m + 1];
                            target = key[m];
                            found = false;
                        }
                        if (found) continue;
                        const int j = jb + k;
                        if (order_key(H[abs(i - j)] + u[j]) == target) {
                            atomicMin(&amin[m], j);
                            found = true;
                        }
                    }
                }
                __syncthreads();
            }
            // 3. record the minimisers of this level's rows
            for (int m = t; m < R; m += kDcBlock) {
                int j;
                if constexpr (sizeof(T) == 4)
                    j = (int)(key[m] & 0xffffffffull);
                else
                    j = amin[m];
                arg[row_i(m)] = (unsigned short)j;
            }
            __syncthreads();
            if (s == 1) break;
        }
        for (int i = t; i < n; i += kDcBlock) {
            const int j = arg[i];
            out[base + (long long)i * inner] = H[abs(i - j)] + u[j];
        }
    }
}

template <typename T>
hipError_t launch_ct_dc(const T *in, T *out, int n, int inner, long long nlines, T sgn, double p,
                        const int32_t *done, hipStream_t stream)
{
    if (n < 2 || n > 4096 || nlines <= 0 || !(p > 1.0)) return hipErrorInvalidValue;
    const size_t smem = dc_smem_bytes<T>(n);
    static size_t lds_limit[kMaxDevices] = {};
    hipError_t e = raise_dyn_lds((const void *)ct_dc_kernel<T>, smem, lds_limit);
    if (e != hipSuccess) return e;
    const int ncu = device_cu_count();
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)ct_dc_kernel<T>, kDcBlock, smem) !=
            hipSuccess ||
        occ < 1)
        occ = 1;
    long long grid = (long long)occ * ncu;
    if (grid > nlines) grid = nlines;
    hipLaunchKernelGGL(ct_dc_kernel<T>, dim3((unsigned)grid), dim3(kDcBlock), smem, stream, in, out, n, inner, nlines,
                       sgn, p, done);
    return hipGetLastError();
}

template hipError_t launch_ct_dc<float>(const float *, float *, int, int, long long, float, double, const int32_t *,
                                        hipStream_t);
template hipError_t launch_ct_dc<double>(const double *, double *, int, int, long long, double, double,
                                         const int32_t *, hipStream_t);

}  // namespace bfm
