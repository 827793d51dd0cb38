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
// GPU organisation: a workgroup handles LPB lines with TPL lanes per line and
// C consecutive points per lane:
//   1. the lane's C values are loaded into registers (vector loads along
//      contiguous lines; for strided axes LPB adjacent lines are read as one
//      vector per grid row) and staged in LDS;
//   2. each lane builds the lower hull of its own C points (sequential scan,
//      hull kept as prev/next links in LDS, popped points marked dead);
//   3. log2(TPL) merge rounds join neighbouring hulls: one lane walks the
//      seam (moving the left end left and the right end right until the
//      joining edge supports both hulls) and relinks;
//   4. every surviving vertex k, whose hull predecessor is p, is optimal for
//      the integer slopes i >= (w_k - w_p)/(k - p); it writes k at that start
//      index (atomic max), and a prefix maximum over i (DPP inside a wave) gives
//      the optimal vertex of every output;
//   5. the output is re-evaluated directly as (i-k)^2 h^2/2 + u_k.
// LDS rows are padded by one slot every 16 entries so that the lane-strided
// accesses of steps 2, 4 and 5 fall on distinct banks.  No step depends on
// the data being convex; ties (collinear points) are removed from the hull,
// which never changes a minimum value.
#include "common.hpp"
#include "launch.hpp"

namespace bfm {

constexpr short kNone = -1;
constexpr short kDead = -2;

__device__ __forceinline__ int padi(int j) { return j + (j >> 4); }
// padi(j0 + c) for the c-th of a lane's own C points (j0 = lane * C): with C
// a power of two up to 16 the lane's points share one pad count, so the
// index is padi(j0) + c and the C accesses differ only in their offsets.
template <int C> __device__ __forceinline__ int lane_padi(int pb, int j0, int c)
{
    if constexpr (C <= 16 && (C & (C - 1)) == 0) return pb + c;
    else return padi(j0 + c);
}
__host__ __device__ inline int padded_len(int n) { return n + (n >> 4) + 1; }

// True when point k is on or above the chord from a to b (a < k < b) in the
// (j, j^2/2 + n^2 u_j) plane: k can be dropped from the lower hull.
template <typename T>
__device__ __forceinline__ bool above_chord(int a, int k, int b, T ua, T uk, T ub, T n2) {
    const T q = T(0.5) * T(b - a) * T(b - k) * T(k - a);
    const T r = T(k - a) * (ub - uk) - T(b - k) * (uk - ua);
    return q + n2 * r <= T(0);
}

// XCD-aware block order: hardware dispatches consecutive block ids round-robin
// over the 8 XCDs; give each XCD a contiguous range of line groups so that
// groups sharing cache lines run under the same L2.
__device__ __forceinline__ long long xcd_block(long long b, long long nb) {
    const long long q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

template <typename T> struct vec4;
template <> struct vec4<float> { using type = float4; };
template <> struct vec4<double> { using type = double4; };

// W-wide vectors (W = 2 or 4) of the strided passes: one per grid row for W
// adjacent lines.
template <typename T, int W> struct vecw;
template <> struct vecw<float, 4> { using type = float4; };
template <> struct vecw<double, 4> { using type = double4; };
template <> struct vecw<float, 2> { using type = float2; };
template <> struct vecw<double, 2> { using type = double2; };
template <typename V> __device__ __forceinline__ auto vget(const V &x, int e) {
    if constexpr (sizeof(V) / sizeof(x.x) == 4) return e == 0 ? x.x : e == 1 ? x.y : e == 2 ? x.z : x.w;
    else return e == 0 ? x.x : x.y;
}
template <typename V, typename T> __device__ __forceinline__ void vset(V &x, int e, T val) {
    if constexpr (sizeof(V) / sizeof(x.x) == 4) {
        if (e == 0) x.x = val; else if (e == 1) x.y = val; else if (e == 2) x.z = val; else x.w = val;
    } else {
        if (e == 0) x.x = val; else x.y = val;
    }
}

// Largest workgroup a (C, LPB) instantiation is launched with: lines of at
// most 4096 points take tpl lanes, the next power of two >= 4096 / C.
constexpr int ct_pow2_at_least(int x) { return x <= 1 ? 1 : 2 * ct_pow2_at_least((x + 1) / 2); }
constexpr int ct_max_threads(int C, int LPB)
{
    return LPB * ct_pow2_at_least((4096 + C - 1) / C) < 1024 ? LPB * ct_pow2_at_least((4096 + C - 1) / C) : 1024;
}

// Wait for the lanes of one wave around LDS traffic, without a workgroup
// barrier: a wave's LDS operations are performed in issue order, so only the
// compiler has to be kept from moving accesses across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Synchronise the lanes of one line: a line of tpl <= 64 lanes lies inside
// one wave (lines start at multiples of tpl, a power of two).
__device__ __forceinline__ void line_sync(int tpl) {
    if (tpl <= kWave) wave_sync();
    else __syncthreads();
}

// Steps 2-5 for the line of this lane, whose values are staged in v (LDS)
// and, for the lane's points [j0, j1), in u; on return u holds the output.
// Touches only this line's LDS (v, pv/nx, GH/GT) and wave_tot; all lanes of
// the workgroup call it (its block barriers are uniform).
//
// FULL: every lane of the line holds all C of its points (n = tpl C), so the
// per-point range tests drop out.
template <typename T, int C, bool FULL = false>
__device__ __forceinline__ void ct_line_core(T (&u)[C], const T *v, short *pv, short *nx, int *GH, int *GT,
                                             int *wave_tot, int j0, int j1, int t, int tpl, int l, int n, T h)
{
    const T n2 = T(n) * T(n);
    const int pb = padi(j0);
    auto has = [&](int c) { return FULL || j0 + c < j1; };
    // 2. lane-local lower hull of points [j0, j1): a stack scan whose top two
    //    entries live in registers (u holds the lane's values), so only pops
    //    read LDS.  Each push also links the element below it forward
    //    (a later push over the same element overwrites a popped successor),
    //    so the forward links of the final stack need no second walk.
    if (FULL || j0 < j1) {
        int top = j0, a = -1;
        T utop = u[0], ua = T(0);
        pv[pb] = kNone;
#pragma unroll
        for (int c = 1; c < C; ++c) {
            const int j = j0 + c;
            if (has(c)) {
                const T uj = u[c];
                while (a >= 0 && above_chord(a, top, j, ua, utop, uj, n2)) {
                    pv[padi(top)] = kDead;
                    top = a;
                    utop = ua;
                    a = pv[padi(top)];
                    if (a >= 0) ua = v[padi(a)];
                }
                pv[lane_padi<C>(pb, j0, c)] = (short)top;
                nx[padi(top)] = (short)j;
                a = top;
                ua = utop;
                top = j;
                utop = uj;
            }
        }
        nx[padi(top)] = kNone;
        GH[t] = j0;
        GT[t] = top;
    } else {
        GH[t] = -1;
        GT[t] = -1;
    }

    // 3. merge neighbouring hulls, doubling the group width each round; a
    //    group of 2r <= 64 lanes lies in one wave and synchronises only it.
    //    The merges and the markers below are short chains of dependent LDS
    //    reads on few lanes, while other workgroups on the CU stream through
    //    their lines: these waves take issue priority until the markers are
    //    placed.
    __builtin_amdgcn_s_setprio(3);
    for (int r = 1; r < tpl; r <<= 1) {
        if (2 * r <= kWave) wave_sync();
        else __syncthreads();
        if ((t & (2 * r - 1)) == 0 && t + r < tpl) {
            const int hL = GH[t], tL = GT[t], hR = GH[t + r], tR = GT[t + r];
            // all four ends in one LDS round trip (the branches below would
            // otherwise make the compiler wait for them one after another)
            __asm__ volatile("" ::"v"(hL), "v"(tL), "v"(hR), "v"(tR));
            if (hR >= 0) {
                if (hL < 0) {
                    GH[t] = hR;
                    GT[t] = tR;
                } else {
                    int a = tL, b = hR;
                    T ua = v[padi(a)], ub = v[padi(b)];
                    for (;;) {
                        bool moved = false;
                        const int pa = pv[padi(a)];
                        if (pa >= 0) {
                            const T upa = v[padi(pa)];
                            if (above_chord(pa, a, b, upa, ua, ub, n2)) {
                                pv[padi(a)] = kDead;
                                a = pa;
                                ua = upa;
                                moved = true;
                            }
                        }
                        const int nb = nx[padi(b)];
                        if (nb >= 0) {
                            const T unb = v[padi(nb)];
                            if (above_chord(a, b, nb, ua, ub, unb, n2)) {
                                pv[padi(b)] = kDead;
                                b = nb;
                                ub = unb;
                                moved = true;
                            }
                        }
                        if (!moved) break;
                    }
                    nx[padi(a)] = (short)b;
                    pv[padi(b)] = (short)a;
                    GT[t] = tR;
                }
            }
        }
    }
    line_sync(tpl);

    // 4. start index of every surviving vertex (registers), then markers
    int st[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = j0 + c;
        st[c] = n;
        if (has(c)) {
            const int p = pv[lane_padi<C>(pb, j0, c)];
            if (p == kNone) {
                st[c] = 0;
            } else if (p >= 0) {
                // float32: the hardware reciprocal (1 ulp) instead of a
                // correctly rounded division; s is a rounded crossing slope
                // either way, and an output within rounding of it may take
                // either of two candidates whose values agree to rounding
                T s;
                if constexpr (sizeof(T) == 4)
                    s = T(0.5) * T(j + p) + n2 * (u[c] - v[padi(p)]) * __builtin_amdgcn_rcpf(T(j - p));
                else
                    s = T(0.5) * T(j + p) + n2 * (u[c] - v[padi(p)]) / T(j - p);
                s = fmin(fmax(s, T(-1)), T(n));
                const int si = (int)ceil(s);
                st[c] = si < 0 ? 0 : si;
            }
        }
    }
    line_sync(tpl);
    int *mk = reinterpret_cast<int *>(pv);   // NP ints over this line's prev/next links
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (has(c)) mk[lane_padi<C>(pb, j0, c)] = -1;
    line_sync(tpl);
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (st[c] < n) atomicMax(&mk[padi(st[c])], j0 + c);
    line_sync(tpl);

    __builtin_amdgcn_s_setprio(0);
    // prefix maximum of the markers along the line
    int loc[C];
    int m = -1;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (has(c)) m = max(m, mk[lane_padi<C>(pb, j0, c)]);
        loc[c] = m;
    }
    // inclusive scan over the lanes of this line: inside a whole wave by DPP
    // (row shifts by 1, 2, 4, 8 within rows of 16 lanes, then the broadcasts
    // of lane 15 and lane 31 into the following rows; lanes without a source
    // keep -1), in segments of tpl < 64 lanes by shuffles; wave totals through
    // LDS
    const int seg = tpl < kWave ? tpl : kWave;
    int incl = m;
    int excl;
    if (seg == kWave) {
        incl = max(incl, __builtin_amdgcn_update_dpp(-1, incl, 0x111, 0xf, 0xf, false));   // row_shr:1
        incl = max(incl, __builtin_amdgcn_update_dpp(-1, incl, 0x112, 0xf, 0xf, false));   // row_shr:2
        incl = max(incl, __builtin_amdgcn_update_dpp(-1, incl, 0x114, 0xf, 0xf, false));   // row_shr:4
        incl = max(incl, __builtin_amdgcn_update_dpp(-1, incl, 0x118, 0xf, 0xf, false));   // row_shr:8
        incl = max(incl, __builtin_amdgcn_update_dpp(-1, incl, 0x142, 0xa, 0xf, false));   // row_bcast:15
        incl = max(incl, __builtin_amdgcn_update_dpp(-1, incl, 0x143, 0xc, 0xf, false));   // row_bcast:31
        excl = __builtin_amdgcn_update_dpp(-1, incl, 0x138, 0xf, 0xf, false);              // wave_shr:1
    } else {
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int o = __shfl_up(incl, off, seg);
            if (off < seg && (t % seg) >= off) incl = max(incl, o);
        }
        excl = __shfl_up(incl, 1, seg);
        if (t % seg == 0) excl = -1;
    }
    if (tpl > kWave) {
        const int tid = threadIdx.x;
        const int w = tid / kWave;
        if ((tid & (kWave - 1)) == kWave - 1) wave_tot[w] = incl;
        __syncthreads();
        const int wl0 = (l * tpl) / kWave;   // first wave of this line
        for (int q = wl0; q < w; ++q) excl = max(excl, wave_tot[q]);
    }

    // 5. evaluate at the selected vertex
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = j0 + c;
        if (has(c)) {
            const int k = max(excl, loc[c]);
            const T d = T(j - k) * h;
            u[c] = T(0.5) * d * d + v[padi(k)];
        }
    }
}

// The same line transform for short lines, by the definition itself: the
// minimum over every point k of the line of (1/2)((j - k) h)^2 + v_k, each
// candidate in the arithmetic of the hull path's step 5.  Its cost is n
// candidates per output, but no step depends on an LDS result of the one
// before, where the hull scan and merges are chains of dependent LDS reads;
// for a line of a few hundred points the direct minimum finishes first.  The
// line's values must be staged in v and visible to this lane, and u must
// hold this lane's own values.
template <typename T, int C>
__device__ __forceinline__ void ct_line_direct(T (&u)[C], const T *v, int j0, int j1, int n, T h)
{
    T best[C];
#pragma unroll
    for (int c = 0; c < C; ++c) best[c] = T(INFINITY);
    for (int k0 = 0; k0 < n; k0 += 16) {       // padi: one pad slot after every 16 values
        const T *vk = v + padi(k0);
        const int kn = min(16, n - k0);
#pragma unroll 4
        for (int q = 0; q < kn; ++q) {
            const T val = vk[q];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T d = T(j0 + c - (k0 + q)) * h;
                best[c] = fmin(best[c], T(0.5) * d * d + val);
            }
        }
    }
    // u still holds this lane's inputs: a non-finite input stays visible in
    // its own outputs (the minimum alone would pass over a NaN)
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (j0 + c < j1) u[c] = best[c] + (u[c] - u[c]);
}

// One group of LPB lines per workgroup: any line length, stride or alignment.
template <typename T, int C, int LPB>
__global__ void __launch_bounds__(ct_max_threads(C, LPB))
ct_lines_kernel(const T *__restrict__ in, T *__restrict__ out, int n, int inner, long long nlines, int tpl,
                T sgn, T h, const int32_t *__restrict__ done)
{
    if (done != nullptr && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int NP = padded_len(n);
    T *vals = reinterpret_cast<T *>(smem);                                   // [LPB][NP]
    short *links = reinterpret_cast<short *>(vals + (size_t)LPB * NP);        // [LPB][2][NP]
    int *grp = reinterpret_cast<int *>(links + (size_t)LPB * 2 * NP);        // [LPB][2][tpl]
    __shared__ int wave_tot[16];

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const long long L0 = xcd_block(blockIdx.x, gridDim.x) * LPB;
    const int l = tid / tpl, t = tid - l * tpl;
    const long long L = L0 + l;
    const int j0 = t * C, j1 = min(j0 + C, n);
    T *v = vals + l * NP;
    short *pv = links + (size_t)l * 2 * NP;
    int *GH = grp + l * 2 * tpl;

    T u[C];
    // 1. stage the lines (u = sgn * in)
    const bool in_al = ((uintptr_t)in & 15) == 0, out_al = ((uintptr_t)out & 15) == 0;
    if (inner == 1) {
        const bool vec = (n & 3) == 0 && (C & 3) == 0 && in_al;
        if (L < nlines && j0 < j1) {
            const T *src = in + L * n;
#pragma unroll
            for (int q = 0; q < C; q += 4) {
                if (vec && j0 + q + 3 < n) {
                    const typename vec4<T>::type x = *reinterpret_cast<const typename vec4<T>::type *>(src + j0 + q);
                    u[q] = x.x; u[q + 1] = x.y; u[q + 2] = x.z; u[q + 3] = x.w;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) u[q + e] = (q + e < C && j0 + q + e < n) ? src[j0 + q + e] : T(0);
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) u[c] = T(0);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            u[c] *= sgn;
            if (j0 + c < j1) v[lane_padi<C>(padi(j0), j0, c)] = u[c];
        }
    } else {
        // LPB adjacent lines are adjacent in memory along every grid row
        const bool vec = LPB == 4 && (inner & 3) == 0 && (L0 % inner) + 4 <= inner && L0 + 4 <= nlines && in_al;
        const long long base0 = line_base(L0, n, inner);
        if (vec) {
            for (int j = tid; j < n; j += nthr) {
                const typename vec4<T>::type x =
                    *reinterpret_cast<const typename vec4<T>::type *>(in + base0 + (long long)j * inner);
                const int pj = padi(j);
                vals[0 * NP + pj] = sgn * x.x;
                vals[1 * NP + pj] = sgn * x.y;
                vals[2 * NP + pj] = sgn * x.z;
                vals[3 * NP + pj] = sgn * x.w;
            }
        } else {
            for (int e = tid; e < LPB * n; e += nthr) {
                const int ll = e % LPB, j = e / LPB;
                const long long LL = L0 + ll;
                vals[ll * NP + padi(j)] = LL < nlines ? sgn * in[line_base(LL, n, inner) + (long long)j * inner] : T(0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < C; ++c) u[c] = j0 + c < j1 ? v[lane_padi<C>(padi(j0), j0, c)] : T(0);
    }
    // rows: each lane staged only its own points, which the local hull reads
    // back itself; the merge rounds synchronise before reading other lanes'

    if (n == tpl * C)   // uniform
        ct_line_core<T, C, true>(u, v, pv, pv + NP, GH, GH + tpl, wave_tot, j0, j1, t, tpl, l, n, h);
    else
        ct_line_core<T, C>(u, v, pv, pv + NP, GH, GH + tpl, wave_tot, j0, j1, t, tpl, l, n, h);

    if (inner == 1) {
        const bool vec = (n & 3) == 0 && (C & 3) == 0 && out_al;
        if (L < nlines && j0 < j1) {
            T *dst = out + L * n;
#pragma unroll
            for (int q = 0; q < C; q += 4) {
                if (vec && j0 + q + 3 < n) {
                    typename vec4<T>::type x;
                    x.x = u[q]; x.y = u[q + 1]; x.z = u[q + 2]; x.w = u[q + 3];
                    *reinterpret_cast<typename vec4<T>::type *>(dst + j0 + q) = x;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (q + e < C && j0 + q + e < n) dst[j0 + q + e] = u[q + e];
                }
            }
        }
    } else {
        __syncthreads();
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (j0 + c < j1) v[lane_padi<C>(padi(j0), j0, c)] = u[c];
        __syncthreads();
        const bool vec = LPB == 4 && (inner & 3) == 0 && (L0 % inner) + 4 <= inner && L0 + 4 <= nlines && out_al;
        const long long base0 = line_base(L0, n, inner);
        if (vec) {
            for (int j = tid; j < n; j += nthr) {
                const int pj = padi(j);
                typename vec4<T>::type x;
                x.x = vals[0 * NP + pj]; x.y = vals[1 * NP + pj]; x.z = vals[2 * NP + pj]; x.w = vals[3 * NP + pj];
                *reinterpret_cast<typename vec4<T>::type *>(out + base0 + (long long)j * inner) = x;
            }
        } else {
            for (int e = tid; e < LPB * n; e += nthr) {
                const int ll = e % LPB, j = e / LPB;
                const long long LL = L0 + ll;
                if (LL < nlines) out[line_base(LL, n, inner) + (long long)j * inner] = vals[ll * NP + padi(j)];
            }
        }
    }
}

// Persistent workgroups with prefetch, for the aligned cases: contiguous
// lines with n % 4 == 0 (STRIDED = false), or four adjacent strided lines per
// group with inner % 4 == 0 (STRIDED = true, LPB = 4); both with 16-byte
// aligned fields.  Workgroup b takes the groups xcd_block(b) + k * gridDim;
// the C values each lane needs for the next group (tpl * C >= n, so a lane's
// share of LPB * n values is at most C) are loaded into registers while the
// current group is transformed from LDS.
//
// BLK selects the column-blocked layout of a 2D field (rows r < R, columns
// c < K, K % 4 == 0): element (r, c) at (c / 4) * 4 R + 4 r + c % 4, i.e. each
// group of four columns is one contiguous run of R 16-byte vectors.  The
// strided pass over the columns (nlines = inner = K, n = R) writes its output
// in that layout, so every group's output is one contiguous 16 R-byte run;
// the contiguous pass over the rows (nlines = R, n = K) reads it.
template <typename T, int C, int LPB, bool STRIDED, bool BLK>
__global__ void __launch_bounds__(ct_max_threads(C, LPB))
ct_lines_pf_kernel(const T *__restrict__ in, T *__restrict__ out, int n, int inner, long long nlines, int tpl,
                   T sgn, T h, const int32_t *__restrict__ done, const T *__restrict__ dotw,
                   double *__restrict__ dotpart)
{
    static_assert(C % 4 == 0 && (!STRIDED || LPB == 4 || LPB == 2) && (!BLK || !STRIDED || LPB == 4),
                  "vector layout");
    if (done != nullptr && *done) return;
    double dacc = 0.0;   // sum out * dotw over the written outputs (contiguous lines only)
    __shared__ double dred[16];
    using V4 = typename vec4<T>::type;
    constexpr int W = STRIDED ? LPB : 4;   // vector width of the global accesses
    using VW = typename vecw<T, W>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const int NP = padded_len(n);
    T *vals = reinterpret_cast<T *>(smem);
    short *links = reinterpret_cast<short *>(vals + (size_t)LPB * NP);
    int *grp = reinterpret_cast<int *>(links + (size_t)LPB * 2 * NP);
    __shared__ int wave_tot[16];

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int l = tid / tpl, t = tid - l * tpl;
    const int jb = t * C;
    T *v = vals + l * NP;
    short *pv = links + (size_t)l * 2 * NP;
    int *GH = grp + l * 2 * tpl;
    const long long step = (long long)gridDim.x * LPB;

    VW pf[C / W] = {};
    auto fetch = [&](long long G0) {
        if constexpr (!STRIDED) {
            const long long L = G0 + l;
            if (BLK) {   // row L of the column-blocked layout: vector q at (jb + 4q) R + 4L
#pragma unroll
                for (int q = 0; q < C / 4; ++q)
                    if (L < nlines && jb + 4 * q < n)
                        pf[q] = *reinterpret_cast<const V4 *>(in + (long long)(jb + 4 * q) * nlines + 4 * L);
            } else {
                const V4 *src = reinterpret_cast<const V4 *>(in + L * n + jb);
#pragma unroll
                for (int q = 0; q < C / 4; ++q)
                    if (L < nlines && jb + 4 * q < n) pf[q] = src[q];
            }
        } else {
            const T *src = in + line_base(G0, n, inner);
#pragma unroll
            for (int q = 0; q < C / W; ++q) {
                const int j = tid + q * nthr;
                if (j < n) pf[q] = *reinterpret_cast<const VW *>(src + (long long)j * inner);
            }
        }
    };

    long long G0 = xcd_block(blockIdx.x, gridDim.x) * LPB;
    if (G0 < nlines) fetch(G0);
    for (; G0 < nlines; G0 += step) {
        // the lane's first point, re-derived every pass so that the compiler
        // does not keep C precomputed LDS addresses per array over the loop
        int j0 = jb;
        __asm__ volatile("" : "+v"(j0));
        const int j1 = min(j0 + C, n);
        const long long L = G0 + l;
        T u[C];
        if constexpr (!STRIDED) {
#pragma unroll
            for (int q = 0; q < C / 4; ++q) {
                u[4 * q] = sgn * pf[q].x;
                u[4 * q + 1] = sgn * pf[q].y;
                u[4 * q + 2] = sgn * pf[q].z;
                u[4 * q + 3] = sgn * pf[q].w;
            }
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (j0 + c < j1) v[lane_padi<C>(padi(j0), j0, c)] = u[c];
            // no barrier: the local hull reads only the lane's own points and
            // the merge rounds synchronise before reading other lanes'
        } else {
#pragma unroll
            for (int q = 0; q < C / W; ++q) {
                const int j = tid + q * nthr;
                if (j < n) {
                    const int pj = padi(j);
#pragma unroll
                    for (int e = 0; e < W; ++e) vals[e * NP + pj] = sgn * vget(pf[q], e);
                }
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < C; ++c) u[c] = j0 + c < j1 ? v[lane_padi<C>(padi(j0), j0, c)] : T(0);
        }
        if (G0 + step < nlines) fetch(G0 + step);   // in flight during the transform

        if (n == tpl * C)   // uniform
            ct_line_core<T, C, true>(u, v, pv, pv + NP, GH, GH + tpl, wave_tot, j0, j1, t, tpl, l, n, h);
        else
            ct_line_core<T, C>(u, v, pv, pv + NP, GH, GH + tpl, wave_tot, j0, j1, t, tpl, l, n, h);

        if constexpr (!STRIDED) {
            if (L < nlines && j0 < j1) {
                V4 *dst = reinterpret_cast<V4 *>(out + L * n + j0);
#pragma unroll
                for (int q = 0; q < C / 4; ++q) {
                    if (j0 + 4 * q < n) {
                        V4 x;
                        x.x = u[4 * q]; x.y = u[4 * q + 1]; x.z = u[4 * q + 2]; x.w = u[4 * q + 3];
                        dst[q] = x;
                        if (dotw != nullptr) {
                            const V4 wv = *reinterpret_cast<const V4 *>(dotw + L * n + j0 + 4 * q);
                            dacc += (double)x.x * wv.x + (double)x.y * wv.y + (double)x.z * wv.z + (double)x.w * wv.w;
                        }
                    }
                }
            }
            line_sync(tpl);   // the next group restages this line's LDS
        } else {
            line_sync(tpl);
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (j0 + c < j1) v[lane_padi<C>(padi(j0), j0, c)] = u[c];
            __syncthreads();
            // plain: row j of the group at line_base + j * inner; blocked: the
            // group's run starts at G0 * n (G0 = 4 x group index), 4 per row
            T *dst = BLK ? out + G0 * n : out + line_base(G0, n, inner);
            const long long rs = BLK ? 4 : inner;
            for (int j = tid; j < n; j += nthr) {
                const int pj = padi(j);
                VW x;
#pragma unroll
                for (int e = 0; e < W; ++e) vset(x, e, vals[e * NP + pj]);
                *reinterpret_cast<VW *>(dst + (long long)j * rs) = x;
            }
            __syncthreads();
        }
    }
    if (dotw != nullptr) {   // uniform: one partial per workgroup, fixed order
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) dacc += __shfl_xor(dacc, o, kWave);
        if ((tid & (kWave - 1)) == 0) dred[tid / kWave] = dacc;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < nthr / kWave; ++w) sum += dred[w];
            dotpart[blockIdx.x] = sum;
        }
    }
}

// Launch shape per line length: C points per lane, TPL = next power of two
// >= n / C lanes per line, LPB lines per workgroup (4 for strided axes so
// that each grid row is read as one 16-byte vector).
struct CtShape {
    int C, tpl, lpb, threads;
};

static size_t ct_smem_for(int n, int tpl, int lpb, size_t esz)
{
    const size_t NP = (size_t)padded_len(n);
    size_t b = (size_t)lpb * NP * esz + (size_t)lpb * 2 * NP * sizeof(short);
    b = (b + 3) & ~(size_t)3;
    return b + (size_t)lpb * 2 * tpl * sizeof(int);
}

constexpr size_t kCtLdsBudget = 150 * 1024;   // gfx950: 160 KB of LDS per CU

static CtShape ct_shape(int n, bool strided, size_t esz, CtCfg cfg = CtCfg{})
{
    CtShape s;
    s.C = cfg.C > 0 ? cfg.C : (n > 1024 ? 16 : 8);
    const int need = (n + s.C - 1) / s.C;
    s.tpl = 1;
    while (s.tpl < need) s.tpl <<= 1;
    if (strided) {
        // the widest group of 4 or 2 lines that fits LDS and 1024 lanes (or the requested width)
        const int want = cfg.lpb > 0 ? cfg.lpb : 4;
        s.lpb = 1;
        for (int w = want; w > 1; w >>= 1)
            if (ct_smem_for(n, s.tpl, w, esz) <= kCtLdsBudget && w * s.tpl <= 1024) {
                s.lpb = w;
                break;
            }
    } else {
        s.lpb = s.tpl >= 256 ? 1 : 256 / s.tpl;
        if (s.lpb > 64) s.lpb = 64;
    }
    s.threads = s.tpl * s.lpb;
    if (s.threads < 64) {   // keep whole waves
        s.lpb *= 64 / s.threads;
        s.threads = 64;
    }
    return s;
}

int ct_threads_per_line(int n) { return ct_shape(n, false, 4).tpl; }

template <typename T>
size_t ct_smem_bytes(int n, int tpl, int lpb) { return ct_smem_for(n, tpl, lpb, sizeof(T)); }

// Workgroups resident at once for a kernel (the persistent grid size).
static long long resident_blocks(const void *fn, int threads, size_t smem)
{
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, threads, smem) != hipSuccess || occ < 1) occ = 1;
    return (long long)occ * device_cu_count();
}

template <typename T, int C, int LPB, bool STRIDED, bool BLK>
static hipError_t launch_pf(const T *in, T *out, int n, int inner, long long nlines, int tpl, int threads, T sgn,
                            const int32_t *done, hipStream_t stream, const T *dotw = nullptr,
                            double *dotpart = nullptr, int *ndot = nullptr)
{
    static size_t lds_limit[kMaxDevices] = {};
    const size_t smem = ct_smem_bytes<T>(n, tpl, LPB);
    const long long groups = (nlines + LPB - 1) / LPB;
    auto fn = ct_lines_pf_kernel<T, C, LPB, STRIDED, BLK>;
    hipError_t e = raise_dyn_lds((const void *)fn, smem, lds_limit);
    if (e != hipSuccess) return e;
    long long blocks = resident_blocks((const void *)fn, threads, smem);
    if (blocks > groups) blocks = groups;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(threads), smem, stream, in, out, n, inner, nlines, tpl, sgn,
                       T(1.0) / T(n), done, dotw, dotpart);
    if (ndot != nullptr) *ndot = dotw != nullptr ? (int)blocks : 0;
    return hipGetLastError();
}

// blk: the strided pass writes, the contiguous pass reads, the column-blocked
// layout of a 2D field (only with the persistent kernel).
template <typename T, int C, int LPB>
static hipError_t launch_ct_impl(const T *in, T *out, int n, int inner, long long nlines, int tpl, int threads,
                                 T sgn, const int32_t *done, hipStream_t stream, bool persistent, bool blk,
                                 const T *dotw, double *dotpart, int *ndot)
{
    if (ndot != nullptr) *ndot = 0;
    const size_t smem = ct_smem_bytes<T>(n, tpl, LPB);
    const long long groups = (nlines + LPB - 1) / LPB;
    const T h = T(1.0) / T(n);
    if (persistent) {
        if constexpr (LPB == 4) {
            if (inner > 1)
                return blk ? launch_pf<T, C, 4, true, true>(in, out, n, inner, nlines, tpl, threads, sgn, done, stream)
                           : launch_pf<T, C, 4, true, false>(in, out, n, inner, nlines, tpl, threads, sgn, done, stream);
        }
        if constexpr (LPB == 2) {
            if (inner > 1 && !blk)
                return launch_pf<T, C, 2, true, false>(in, out, n, inner, nlines, tpl, threads, sgn, done, stream);
        }
        if (inner == 1)
            return blk ? launch_pf<T, C, LPB, false, true>(in, out, n, inner, nlines, tpl, threads, sgn, done, stream,
                                                           dotw, dotpart, ndot)
                       : launch_pf<T, C, LPB, false, false>(in, out, n, inner, nlines, tpl, threads, sgn, done, stream,
                                                            dotw, dotpart, ndot);
        return hipErrorInvalidValue;
    }
    if (blk) return hipErrorInvalidValue;
    static size_t lds_limit[kMaxDevices] = {};
    hipError_t e = raise_dyn_lds((const void *)ct_lines_kernel<T, C, LPB>, smem, lds_limit);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ct_lines_kernel<T, C, LPB>), dim3((unsigned)groups), dim3(threads), smem, stream, in,
                       out, n, inner, nlines, tpl, sgn, h, done);
    return hipGetLastError();
}

// The persistent kernel applies where its vector layout does: contiguous
// lines of n % 4 == 0, or four strided lines per group with inner % 4 == 0,
// with 16-byte aligned fields.
static bool ct_persistent_ok(int n, int inner, int lpb, const void *in, const void *out)
{
    if ((((uintptr_t)in | (uintptr_t)out) & 15) != 0) return false;
    if (inner == 1) return (n & 3) == 0;
    return (lpb == 4 && (inner & 3) == 0) || (lpb == 2 && (inner & 1) == 0);
}

// Whether an axis pass runs the persistent kernel under `cfg`.
template <typename T>
static bool ct_uses_persistent(int n, int inner, const void *in, const void *out, CtCfg cfg)
{
    const CtShape s = ct_shape(n, inner > 1, sizeof(T), cfg);
    return ct_persistent_ok(n, inner, s.lpb, in, out) && (cfg.pers == 2 || (cfg.pers == 0 && sizeof(T) == 4));
}

template <typename T>
static hipError_t launch_ct_axis_blk(const T *in, T *out, int n, int inner, long long nlines, T sgn,
                                     const int32_t *done, hipStream_t stream, CtCfg cfg, bool blk,
                                     const T *dotw = nullptr, double *dotpart = nullptr, int *ndot = nullptr)
{
    const CtShape s = ct_shape(n, inner > 1, sizeof(T), cfg);
    if (s.tpl > 1024 || s.threads > ct_max_threads(s.C, s.lpb)) return hipErrorInvalidValue;
    const bool ok = ct_persistent_ok(n, inner, s.lpb, in, out);
    if (cfg.pers == 2 && !ok) return hipErrorInvalidValue;
    const bool pers = ok && (cfg.pers == 2 || (cfg.pers == 0 && sizeof(T) == 4));
    if (blk && !pers) return hipErrorInvalidValue;
#define BFM_CT_CASE(CC, LL)                                                                               \
    if (s.C == CC && s.lpb == LL)                                                                         \
        return launch_ct_impl<T, CC, LL>(in, out, n, inner, nlines, s.tpl, s.threads, sgn, done, stream, pers, blk, \
                                         dotw, dotpart, ndot);
    BFM_CT_CASE(16, 1) BFM_CT_CASE(16, 4) BFM_CT_CASE(8, 1) BFM_CT_CASE(8, 2) BFM_CT_CASE(8, 4)
    BFM_CT_CASE(8, 8) BFM_CT_CASE(8, 16) BFM_CT_CASE(8, 32) BFM_CT_CASE(8, 64) BFM_CT_CASE(16, 2)
    BFM_CT_CASE(16, 8) BFM_CT_CASE(16, 16) BFM_CT_CASE(16, 32) BFM_CT_CASE(16, 64) BFM_CT_CASE(4, 1)
    BFM_CT_CASE(4, 2) BFM_CT_CASE(4, 4) BFM_CT_CASE(4, 8) BFM_CT_CASE(4, 16) BFM_CT_CASE(4, 32) BFM_CT_CASE(4, 64)
    BFM_CT_CASE(12, 1) BFM_CT_CASE(12, 2) BFM_CT_CASE(12, 4) BFM_CT_CASE(12, 8) BFM_CT_CASE(12, 16)
    BFM_CT_CASE(12, 32) BFM_CT_CASE(12, 64)
#undef BFM_CT_CASE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_ct_axis(const T *in, T *out, int n, int inner, long long nlines, T sgn,
                          const int32_t *done, hipStream_t stream, CtCfg cfg)
{
    return launch_ct_axis_blk<T>(in, out, n, inner, nlines, sgn, done, stream, cfg, false);
}

// The column-blocked two-pass form of a 2D transform applies when both
// passes run the persistent kernel (four-column groups on the columns) with
// 16-byte aligned fields and a row length divisible by 4.
template <typename T>
bool ct_blocked_applies(const Grid &g, const void *in, const void *mid, const void *out, const CtCfg *cfg)
{
    const CtCfg c0 = cfg != nullptr ? cfg[0] : CtCfg{}, c1 = cfg != nullptr ? cfg[1] : CtCfg{};
    return g.ndim == 2 && grid_quadratic(g) && (g.n[1] & 3) == 0 && ct_uses_persistent<T>(g.n[0], g.n[1], in, mid, c0) &&
           ct_shape(g.n[0], true, sizeof(T), c0).lpb == 4 && ct_uses_persistent<T>(g.n[1], 1, mid, out, c1);
}

// One pass of that form: pass 0 transforms the columns of u = -in and
// writes the column-blocked layout; pass 1 transforms the rows of a
// column-blocked field and writes row-major output (with dotw, also the
// per-workgroup partials of sum out * dotw).
template <typename T>
hipError_t ct_blocked_pass(const Grid &g, int pass, const T *in, T *out, const int32_t *done, hipStream_t stream,
                           const CtCfg *cfg, const T *dotw, double *dotpart, int *ndot)
{
    const CtCfg c0 = cfg != nullptr ? cfg[0] : CtCfg{}, c1 = cfg != nullptr ? cfg[1] : CtCfg{};
    if (ndot != nullptr) *ndot = 0;
    if (pass == 0) return launch_ct_axis_blk<T>(in, out, g.n[0], g.n[1], g.n[1], T(-1), done, stream, c0, true);
    return launch_ct_axis_blk<T>(in, out, g.n[1], 1, g.n[0], T(1), done, stream, c1, true, dotw, dotpart, ndot);
}

// Full c-transform of a field: out = in^c.  The axes are independent
// minimisations, so any order gives the same minimum.  Default order: axis
// ndim-1 first (u = -in), then each earlier axis on the running result.  In
// 2D, when both passes run the persistent kernel and `scratch` (N words) is
// given, the columns go first and write the column-blocked layout into
// scratch, and the rows read it: both passes then write whole contiguous runs.
template <typename T>
hipError_t ctransform_field(const Grid &g, const T *in, T *out, const int32_t *done, hipStream_t stream,
                            const CtCfg *cfg, T *scratch, const T *dotw, double *dotpart, int *ndot)
{
    if (ndot != nullptr) *ndot = 0;
    if (scratch != nullptr && scratch != in && scratch != out && ct_blocked_applies<T>(g, in, scratch, out, cfg)) {
        hipError_t e = ct_blocked_pass<T>(g, 0, in, scratch, done, stream, cfg);
        if (e != hipSuccess) return e;
        return ct_blocked_pass<T>(g, 1, scratch, out, done, stream, cfg, dotw, dotpart, ndot);
    }
    for (int a = g.ndim - 1; a >= 0; --a) {
        const int n = g.n[a];
        const int inner = (int)g.stride[a];
        const long long nlines = g.N / n;
        const T *src = a == g.ndim - 1 ? in : out;
        const T sgn = a == g.ndim - 1 ? T(-1) : T(1);
        hipError_t e = g.pw[a] != 2.0
                           ? launch_ct_dc<T>(src, out, n, inner, nlines, sgn, g.pw[a], done, stream)
                           : launch_ct_axis<T>(src, out, n, inner, nlines, sgn, done, stream,
                                               cfg != nullptr ? cfg[a] : CtCfg{});
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------ multi-pair
// One pass of the 2D transform for every pair of a batch in one launch
// (rows: u = -p into F; columns: F into p^c or q, the latter with the fused
// sum of q * src).  Workgroups of 256 lanes, C points per lane (16 for lines
// longer than 256 points, 4 for shorter ones, whose workgroups would
// otherwise be few and long: a small pair's pass is a chain of dependent LDS
// steps whose length grows with C), tpl lanes per line (the next power of two
// >= n / C) and 256 / tpl lines per workgroup, so every pair's lines fill
// whole workgroups whatever its size.
constexpr int kMultiCtThreads = 256;
constexpr int kMultiCtC = 16;        // lines longer than kMultiCtShort points
constexpr int kMultiCtCShort = 4;    // lines of at most kMultiCtShort points
constexpr int kMultiCtShort = 256;
constexpr int kMultiCtDirect = 256;  // lines this short take the direct minimum
static_assert(kMultiCtDirect <= kMultiCtShort && kMultiCtShort <= kMultiCtCShort * kWave,
              "direct lines lie inside one wave (line_sync is a wave barrier)");

__host__ __device__ inline int multi_c(int n) { return n <= kMultiCtShort ? kMultiCtCShort : kMultiCtC; }

__host__ __device__ inline int multi_tpl(int n)
{
    const int C = multi_c(n);
    int tpl = 1;
    while (tpl * C < n) tpl <<= 1;
    return tpl;
}

int ct_multi_col_groups(int n0, int n1)
{
    const int lpb = kMultiCtThreads / multi_tpl(n0);
    return (n1 + lpb - 1) / lpb;
}

static int ct_multi_groups(int n0, int n1, bool strided)
{
    if (strided) return ct_multi_col_groups(n0, n1);
    const int lpb = kMultiCtThreads / multi_tpl(n1);
    return (n0 + lpb - 1) / lpb;
}

__device__ __forceinline__ int batch_pair(const BatchIdx &bi)
{
    int lo = 0, hi = bi.np - 1;   // largest p with off[p] <= blockIdx.x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bi.off[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// which: 0 head rows, 1 head columns, 2 step rows, 3 step columns (+ sum)
template <typename T, bool STRIDED, int C>
__device__ __forceinline__ void ct_multi_body(const PairDev &P, const BatchIdx &bi, int pr, int role, int which,
                                              unsigned char *smem, int *wave_tot, double *dred)
{
    using V4 = typename vec4<T>::type;
    const T *pfield = (const T *)(role ? P.psi : P.phi);
    const T *src = (const T *)(role ? P.nu : P.mu);
    const T *in = STRIDED ? (const T *)P.F : pfield;
    T *out = STRIDED ? (which == 3 ? (T *)(role ? P.phi : P.psi) : (T *)P.pc) : (T *)P.F;
    const T sgn = STRIDED ? T(1) : T(-1);
    const bool dot = STRIDED && which == 3;

    const int n = STRIDED ? P.n0 : P.n1;
    const int inner = STRIDED ? P.n1 : 1;
    const long long nlines = STRIDED ? P.n1 : P.n0;
    const int tpl = multi_tpl(n);
    const int lpb = kMultiCtThreads / tpl;
    const int NP = padded_len(n);
    T *vals = reinterpret_cast<T *>(smem);                                   // [lpb][NP]
    short *links = reinterpret_cast<short *>(vals + (size_t)lpb * NP);        // [lpb][2][NP]
    int *grp = reinterpret_cast<int *>(smem + ((((size_t)lpb * NP * sizeof(T) + (size_t)lpb * 2 * NP * sizeof(short)) + 3) & ~(size_t)3));

    const int tid = threadIdx.x;
    const long long L0 = (long long)(blockIdx.x - bi.off[pr]) * lpb;
    const int l = tid / tpl, t = tid - l * tpl;
    const long long L = L0 + l;
    const int j0 = t * C, j1 = min(j0 + C, n);
    T *v = vals + l * NP;
    short *pv = links + (size_t)l * 2 * NP;
    int *GH = grp + l * 2 * tpl;

    T u[C];
    if (!STRIDED) {
        const T *row = in + L * n;
#pragma unroll
        for (int q = 0; q < C; q += 4) {
            if (L < nlines && j0 + q < n) {   // n % 4 == 0
                const V4 x = *reinterpret_cast<const V4 *>(row + j0 + q);
                u[q] = x.x; u[q + 1] = x.y; u[q + 2] = x.z; u[q + 3] = x.w;
            } else {
                u[q] = u[q + 1] = u[q + 2] = u[q + 3] = T(0);
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            u[c] *= sgn;
            if (j0 + c < j1) v[lane_padi<C>(padi(j0), j0, c)] = u[c];
        }
    } else {
        // lines L0 .. L0 + lpb - 1 are adjacent columns: four per 16-byte
        // vector of a grid row (lpb >= 4), else element by element
        if (lpb >= 4) {
            const int nv = lpb / 4;
            for (int e = tid; e < nv * n; e += kMultiCtThreads) {
                const int vq = e % nv, j = e / nv;
                const long long c0 = L0 + 4 * vq;
                V4 x;
                if (c0 < nlines) x = *reinterpret_cast<const V4 *>(in + (long long)j * inner + c0);
                else x.x = x.y = x.z = x.w = T(0);
                const int pj = padi(j);
                vals[(4 * vq + 0) * NP + pj] = sgn * x.x;
                vals[(4 * vq + 1) * NP + pj] = sgn * x.y;
                vals[(4 * vq + 2) * NP + pj] = sgn * x.z;
                vals[(4 * vq + 3) * NP + pj] = sgn * x.w;
            }
        } else {
            for (int e = tid; e < lpb * n; e += kMultiCtThreads) {
                const int ll = e % lpb, j = e / lpb;
                const long long c = L0 + ll;
                vals[ll * NP + padi(j)] = c < nlines ? sgn * in[(long long)j * inner + c] : T(0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < C; ++c) u[c] = j0 + c < j1 ? v[lane_padi<C>(padi(j0), j0, c)] : T(0);
    }

    if (n <= kMultiCtDirect) {   // uniform: one pair per workgroup
        if (!STRIDED) line_sync(tpl);   // the line's values, staged by its other lanes
        ct_line_direct<T, C>(u, v, j0, j1, n, T(1.0) / T(n));
    } else {
        const T hn = T(1.0) / T(n);
        if (n == tpl * C)   // uniform: one pair per workgroup
            ct_line_core<T, C, true>(u, v, pv, pv + NP, GH, GH + tpl, wave_tot, j0, j1, t, tpl, l, n, hn);
        else
            ct_line_core<T, C>(u, v, pv, pv + NP, GH, GH + tpl, wave_tot, j0, j1, t, tpl, l, n, hn);
    }

    double dacc = 0.0;
    if (!STRIDED) {
        if (L < nlines && j0 < j1) {
            T *dst = out + L * n;
#pragma unroll
            for (int q = 0; q < C; q += 4) {
                if (j0 + q < n) {
                    V4 x;
                    x.x = u[q]; x.y = u[q + 1]; x.z = u[q + 2]; x.w = u[q + 3];
                    *reinterpret_cast<V4 *>(dst + j0 + q) = x;
                }
            }
        }
    } else {
        __syncthreads();
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (j0 + c < j1) v[lane_padi<C>(padi(j0), j0, c)] = u[c];
        __syncthreads();
        if (lpb >= 4) {
            const int nv = lpb / 4;
            for (int e = tid; e < nv * n; e += kMultiCtThreads) {
                const int vq = e % nv, j = e / nv;
                const long long c0 = L0 + 4 * vq;
                if (c0 >= nlines) continue;
                const int pj = padi(j);
                V4 x;
                x.x = vals[(4 * vq + 0) * NP + pj];
                x.y = vals[(4 * vq + 1) * NP + pj];
                x.z = vals[(4 * vq + 2) * NP + pj];
                x.w = vals[(4 * vq + 3) * NP + pj];
                const long long at = (long long)j * inner + c0;
                *reinterpret_cast<V4 *>(out + at) = x;
                if (dot) {
                    const V4 w = *reinterpret_cast<const V4 *>(src + at);
                    dacc += (double)x.x * w.x + (double)x.y * w.y + (double)x.z * w.z + (double)x.w * w.w;
                }
            }
        } else {
            for (int e = tid; e < lpb * n; e += kMultiCtThreads) {
                const int ll = e % lpb, j = e / lpb;
                const long long c = L0 + ll;
                if (c >= nlines) continue;
                const long long at = (long long)j * inner + c;
                const T x = vals[ll * NP + padi(j)];
                out[at] = x;
                if (dot) dacc += (double)x * src[at];
            }
        }
    }
    if (dot) {   // uniform: one partial per workgroup of the pair, in group order
        dacc = wave_sum(dacc);
        if ((tid & (kWave - 1)) == 0) dred[tid / kWave] = dacc;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < kMultiCtThreads / kWave; ++w) sum += dred[w];
            P.part[S_Q_SRC * P.slot_len + (blockIdx.x - bi.off[pr])] = sum;
        }
    }
}

template <typename T, bool STRIDED>
__global__ void __launch_bounds__(kMultiCtThreads)
ct_multi_kernel(const BatchHead *__restrict__ tab, BatchIdx bi, int role, int which)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int wave_tot[16];
    __shared__ double dred[kMultiCtThreads / kWave];
    const int pr = batch_pair(bi);
    const PairDev &P = reinterpret_cast<const PairDev *>(tab + 1)[pr];
    if ((tab->done_mask >> pr) & 1ull) return;
    if (multi_c(STRIDED ? P.n0 : P.n1) == kMultiCtCShort)
        ct_multi_body<T, STRIDED, kMultiCtCShort>(P, bi, pr, role, which, smem, wave_tot, dred);
    else
        ct_multi_body<T, STRIDED, kMultiCtC>(P, bi, pr, role, which, smem, wave_tot, dred);
}

template <typename T>
hipError_t launch_ct_multi(const BatchHead *tab, const int *n0s, const int *n1s, int np, int role, int which,
                           hipStream_t stream)
{
    if (np < 1 || np > kBatchChunk || which < 0 || which > 3) return hipErrorInvalidValue;
    const bool strided = (which & 1) != 0;
    BatchIdx bi{};
    bi.np = np;
    size_t smem = 0;
    for (int p = 0; p < np; ++p) {
        const int n = strided ? n0s[p] : n1s[p];
        if (n > kMultiCtC * kMultiCtThreads || (n1s[p] & 3) != 0) return hipErrorInvalidValue;
        const int tpl = multi_tpl(n);
        const size_t b = ct_smem_for(n, tpl, kMultiCtThreads / tpl, sizeof(T));
        smem = b > smem ? b : smem;
        bi.off[p + 1] = bi.off[p] + ct_multi_groups(n0s[p], n1s[p], strided);
    }
    static size_t lds_limit[2][kMaxDevices] = {};
    const void *fn = strided ? (const void *)ct_multi_kernel<T, true> : (const void *)ct_multi_kernel<T, false>;
    hipError_t e = raise_dyn_lds(fn, smem, lds_limit[strided ? 1 : 0]);
    if (e != hipSuccess) return e;
    if (strided)
        hipLaunchKernelGGL((ct_multi_kernel<T, true>), dim3((unsigned)bi.off[np]), dim3(kMultiCtThreads), smem, stream,
                           tab, bi, role, which);
    else
        hipLaunchKernelGGL((ct_multi_kernel<T, false>), dim3((unsigned)bi.off[np]), dim3(kMultiCtThreads), smem,
                           stream, tab, bi, role, which);
    return hipGetLastError();
}

template hipError_t launch_ct_multi<float>(const BatchHead *, const int *, const int *, int, int, int, hipStream_t);
template hipError_t launch_ct_multi<double>(const BatchHead *, const int *, const int *, int, int, int, hipStream_t);

template hipError_t launch_ct_axis<float>(const float *, float *, int, int, long long, float, const int32_t *,
                                          hipStream_t, CtCfg);
template hipError_t launch_ct_axis<double>(const double *, double *, int, int, long long, double,
                                           const int32_t *, hipStream_t, CtCfg);
template hipError_t ctransform_field<float>(const Grid &, const float *, float *, const int32_t *, hipStream_t,
                                            const CtCfg *, float *, const float *, double *, int *);
template hipError_t ctransform_field<double>(const Grid &, const double *, double *, const int32_t *, hipStream_t,
                                             const CtCfg *, double *, const double *, double *, int *);
template bool ct_blocked_applies<float>(const Grid &, const void *, const void *, const void *, const CtCfg *);
template bool ct_blocked_applies<double>(const Grid &, const void *, const void *, const void *, const CtCfg *);
template hipError_t ct_blocked_pass<float>(const Grid &, int, const float *, float *, const int32_t *, hipStream_t,
                                           const CtCfg *, const float *, double *, int *);
template hipError_t ct_blocked_pass<double>(const Grid &, int, const double *, double *, const int32_t *,
                                            hipStream_t, const CtCfg *, const double *, double *, int *);
template size_t ct_smem_bytes<float>(int, int, int);
template size_t ct_smem_bytes<double>(int, int, int);

}  // namespace bfm
