// One-dimensional quadratic c-transform along one axis of a grid field.
//
// Paper, Section 4.1: with c = |x-y|^2/2 the transform of a line is a Legendre
// transform, phi^c(x) = |x|^2/2 - varphi^*(x), varphi(y) = |y|^2/2 - phi(y)
// (eq. legendre), and varphi^* only needs the lower convex hull varphi^**:
// the optimal y for x is where x - (varphi^**)'(y) changes sign
// (eq. legendre_search).  The multi-dimensional transform repeats the line
// transform along every axis.
//
// For the line values u_j (j = 0..n-1, y_j = (j+1/2)h) a pass computes
//     out_i = min_j (i - j)^2 h^2 / 2 + u_j .
// In index units this is min_j (w_j - i j) + i^2/2 with w_j = j^2/2 + n^2 u_j,
// i.e. the Legendre transform of the points (j, w_j) at integer slopes i.
//
// GPU organisation (one workgroup of 256 lanes handles `lpb` lines, `tpl`
// lanes per line, C consecutive points per lane):
//   1. the line is staged in LDS;
//   2. each lane builds the lower hull of its own C points (sequential scan,
//      hull kept as prev/next links in LDS, popped points marked dead);
//   3. log2(tpl) merge rounds join neighbouring hulls: one lane walks the
//      seam (moving the left end left and the right end right until the
//      joining edge supports both hulls) and relinks;
//   4. every surviving vertex k, whose hull predecessor is p, is optimal for
//      the integer slopes i >= (w_k - w_p)/(k - p); it writes k at that start
//      index (atomic max), and a prefix maximum over i then gives the optimal
//      vertex of every output (the largest vertex whose range has begun);
//   5. the output is re-evaluated directly as (i-k)^2 h^2/2 + u_k.
// No step depends on the data being convex; ties (collinear points) are
// removed from the hull, which never changes a minimum value.
#include "common.hpp"
#include "launch.hpp"

namespace bfm {

constexpr short kNone = -1;
constexpr short kDead = -2;

// True when point k is on or above the chord from a to b (a < k < b) in the
// (j, j^2/2 + n^2 u_j) plane: k can be dropped from the lower hull.
template <typename T>
__device__ __forceinline__ bool above_chord(int a, int k, int b, T ua, T uk, T ub, T n2) {
    const T q = T(0.5) * T(b - a) * T(b - k) * T(k - a);
    const T r = T(k - a) * (ub - uk) - T(b - k) * (uk - ua);
    return q + n2 * r <= T(0);
}

template <typename T, int C>
__global__ void __launch_bounds__(256)
ct_lines_kernel(const T *__restrict__ in, T *__restrict__ out, int n, int inner, long long nlines,
                int tpl, int lpb, T sgn, T h, const int32_t *__restrict__ done)
{
    if (done != nullptr && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    T *vals = reinterpret_cast<T *>(smem);
    short *prv = reinterpret_cast<short *>(vals + (size_t)lpb * n);
    short *nxt = prv + (size_t)lpb * n;
    int *grp = reinterpret_cast<int *>(nxt + (size_t)lpb * n);   // [lpb][2][tpl]

    const int tid = threadIdx.x;
    const long long L0 = (long long)blockIdx.x * lpb;
    const int tot = lpb * n;

    // 1. stage the lines (u = sgn * in)
    if (inner == 1) {
        for (int e = tid; e < tot; e += blockDim.x) {
            const int l = e / n, j = e - l * n;
            const long long L = L0 + l;
            vals[e] = L < nlines ? sgn * in[L * n + j] : T(0);
        }
    } else {
        for (int e = tid; e < tot; e += blockDim.x) {
            const int l = e % lpb, j = e / lpb;
            const long long L = L0 + l;
            vals[l * n + j] = L < nlines ? sgn * in[line_base(L, n, inner) + (long long)j * inner] : T(0);
        }
    }
    __syncthreads();

    const int l = tid / tpl, t = tid - l * tpl;
    const T *v = vals + l * n;
    short *pv = prv + l * n;
    short *nx = nxt + l * n;
    int *GH = grp + l * 2 * tpl;
    int *GT = GH + tpl;
    const T n2 = T(n) * T(n);
    const int j0 = t * C, j1 = min(j0 + C, n);

    // 2. lane-local lower hull of points [j0, j1)
    if (j0 < j1) {
        int top = j0;
        T utop = v[j0];
        pv[j0] = kNone;
        for (int j = j0 + 1; j < j1; ++j) {
            const T uj = v[j];
            int a = pv[top];
            while (a >= 0) {
                const T ua = v[a];
                if (!above_chord(a, top, j, ua, utop, uj, n2)) break;
                pv[top] = kDead;
                top = a;
                utop = ua;
                a = pv[top];
            }
            pv[j] = (short)top;
            top = j;
            utop = uj;
        }
        int k = top;
        nx[k] = kNone;
        while (pv[k] >= 0) {
            const int p = pv[k];
            nx[p] = (short)k;
            k = p;
        }
        GH[t] = j0;
        GT[t] = top;
    } else {
        GH[t] = -1;
        GT[t] = -1;
    }
    __syncthreads();

    // 3. merge neighbouring hulls, doubling the group width each round
    for (int r = 1; r < tpl; r <<= 1) {
        if ((t & (2 * r - 1)) == 0 && t + r < tpl) {
            const int hL = GH[t], tL = GT[t], hR = GH[t + r], tR = GT[t + r];
            if (hR >= 0) {
                if (hL < 0) {
                    GH[t] = hR;
                    GT[t] = tR;
                } else {
                    int a = tL, b = hR;
                    T ua = v[a], ub = v[b];
                    for (;;) {
                        bool moved = false;
                        const int pa = pv[a];
                        if (pa >= 0) {
                            const T upa = v[pa];
                            if (above_chord(pa, a, b, upa, ua, ub, n2)) {
                                pv[a] = kDead;
                                a = pa;
                                ua = upa;
                                moved = true;
                            }
                        }
                        const int nb = nx[b];
                        if (nb >= 0) {
                            const T unb = v[nb];
                            if (above_chord(a, b, nb, ua, ub, unb, n2)) {
                                pv[b] = kDead;
                                b = nb;
                                ub = unb;
                                moved = true;
                            }
                        }
                        if (!moved) break;
                    }
                    nx[a] = (short)b;
                    pv[b] = (short)a;
                    GT[t] = tR;
                }
            }
        }
        __syncthreads();
    }

    // 4. start index of every surviving vertex (registers), then markers
    int st[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = j0 + c;
        st[c] = n;
        if (j < j1) {
            const int p = pv[j];
            if (p == kNone) {
                st[c] = 0;
            } else if (p >= 0) {
                T s = T(0.5) * T(j + p) + n2 * (v[j] - v[p]) / T(j - p);
                s = fmin(fmax(s, T(-1)), T(n));
                const int si = (int)ceil(s);
                st[c] = si < 0 ? 0 : si;
            }
        }
    }
    __syncthreads();
    int *mk = reinterpret_cast<int *>(prv) + l * n;   // aliases prv/nxt of this block's lines
    for (int j = j0; j < j1; ++j) mk[j] = -1;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (st[c] < n) atomicMax(&mk[st[c]], j0 + c);
    __syncthreads();

    // prefix maximum of the markers along the line
    int loc[C];
    int m = -1;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = j0 + c;
        if (j < j1) m = max(m, mk[j]);
        loc[c] = m;
    }
    GH[t] = m;
    __syncthreads();
    for (int off = 1; off < tpl; off <<= 1) {
        int val = GH[t];
        if (t >= off) val = max(val, GH[t - off]);
        __syncthreads();
        GH[t] = val;
        __syncthreads();
    }
    const int excl = t > 0 ? GH[t - 1] : -1;

    // 5. evaluate at the selected vertex
    T res[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = j0 + c;
        res[c] = T(0);
        if (j < j1) {
            const int k = max(excl, loc[c]);
            const T d = T(j - k) * h;
            res[c] = T(0.5) * d * d + v[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (j0 + c < j1) vals[l * n + j0 + c] = res[c];
    __syncthreads();

    if (inner == 1) {
        for (int e = tid; e < tot; e += blockDim.x) {
            const int ll = e / n, j = e - ll * n;
            const long long L = L0 + ll;
            if (L < nlines) out[L * n + j] = vals[e];
        }
    } else {
        for (int e = tid; e < tot; e += blockDim.x) {
            const int ll = e % lpb, j = e / lpb;
            const long long L = L0 + ll;
            if (L < nlines) out[line_base(L, n, inner) + (long long)j * inner] = vals[ll * n + j];
        }
    }
}

constexpr int kCtChunk = 16;

int ct_threads_per_line(int n) {
    int need = (n + kCtChunk - 1) / kCtChunk;
    int tpl = 1;
    while (tpl < need) tpl <<= 1;
    return tpl;
}

template <typename T>
size_t ct_smem_bytes(int n, int tpl, int lpb) {
    size_t b = (size_t)lpb * n * sizeof(T);
    b = (b + 3) & ~(size_t)3;
    b += (size_t)lpb * n * 2 * sizeof(short);
    b += (size_t)lpb * 2 * tpl * sizeof(int);
    return b;
}

template <typename T>
hipError_t launch_ct_axis(const T *in, T *out, int n, int inner, long long nlines, T sgn,
                          const int32_t *done, hipStream_t stream)
{
    const int tpl = ct_threads_per_line(n);
    if (tpl > 256) return hipErrorInvalidValue;
    const int lpb = 256 / tpl;
    const size_t smem = ct_smem_bytes<T>(n, tpl, lpb);
    const long long blocks = (nlines + lpb - 1) / lpb;
    const T h = T(1.0) / T(n);
    hipLaunchKernelGGL((ct_lines_kernel<T, kCtChunk>), dim3((unsigned)blocks), dim3(256), smem, stream,
                       in, out, n, inner, nlines, tpl, lpb, sgn, h, done);
    return hipGetLastError();
}

// Full c-transform of a field: out = in^c, axis ndim-1 first (u = -in), then
// each earlier axis on the running result.
template <typename T>
hipError_t ctransform_field(const Grid &g, const T *in, T *out, const int32_t *done, hipStream_t stream)
{
    for (int a = g.ndim - 1; a >= 0; --a) {
        const int n = g.n[a];
        const int inner = (int)g.stride[a];
        const long long nlines = g.N / n;
        hipError_t e = launch_ct_axis<T>(a == g.ndim - 1 ? in : out, out, n, inner, nlines,
                                         a == g.ndim - 1 ? T(-1) : T(1), done, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_ct_axis<float>(const float *, float *, int, int, long long, float, const int32_t *,
                                          hipStream_t);
template hipError_t launch_ct_axis<double>(const double *, double *, int, int, long long, double,
                                           const int32_t *, hipStream_t);
template hipError_t ctransform_field<float>(const Grid &, const float *, float *, const int32_t *, hipStream_t);
template hipError_t ctransform_field<double>(const Grid &, const double *, double *, const int32_t *, hipStream_t);
template size_t ct_smem_bytes<float>(int, int, int);
template size_t ct_smem_bytes<double>(int, int, int);

}  // namespace bfm
