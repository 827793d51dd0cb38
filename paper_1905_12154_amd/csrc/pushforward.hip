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
//     weights (exact mass conservation up to rounding).
// For the power cost of eq. p_costs, h_a(z) = |z|^{p_a} / p_a, the inverse
// of h_a' is g -> sign(g) |g|^{1/(p_a - 1)}, so component a of the map is
// x_a - sign(g_a) |g_a|^{1/(p_a - 1)} with g = grad phi^c (GEN kernels).
// Fused float64 partial sums: sum mu c(x, T(x)) (primal cost of the map;
// |x - T|^2 / 2 for the quadratic cost) and sum mu phi^c (the second term
// of J).  With tmix != 1 the map is the
// displacement interpolant S_t(x) = t T(x) + (1 - t) x (Section 4.3,
// optimal transport of images), t = tmix.
//
// Deposition: source cells are processed by compact tiles (16 x 32 in 2D,
// 8 x 8 x 8 in 3D).  Where the map compresses mass, many sources of a tile
// land on few target cells, and global atomics on the same addresses
// serialise; so the workgroup first accumulates its deposits in an LDS box
// covering all its targets (LDS atomics) and then adds each non-zero box
// cell to the global density once.  Tiles whose targets spread over more
// than the LDS box holds deposit with global atomics directly (no
// contention there).  float32 boxes hold unsigned fixed-point sums (LDS
// integer atomics; see BoxCell), float64 boxes float64 sums.
#include <climits>

#include "common.hpp"
#include "launch.hpp"

namespace bfm {

// LDS box: 32 KB in 2D, 16 KB in 3D.  A 2D tile's targets overflow the box
// only where the map expands by more than about 4 per axis.  In 2D the box
// sets four workgroups per CU (registers would allow six), but smaller
// boxes overflow to global atomics more often and were slower; in 3D a
// larger box was slower.
template <typename T, int D> constexpr int box_cap() { return (D == 3 ? 16384 : 32768) / (int)sizeof(T); }

// Box cells: float32 deposits accumulate in unsigned 32-bit fixed point (an
// LDS integer atomic add is about 40 times cheaper on gfx950 than a float
// one), float64 deposits in float64.  Per tile the fixed-point unit is
// tile_mass / kFixOne, so no cell can exceed 2^32 even if all of the tile's
// mass lands in it; each deposit is rounded to that unit once (as precise as
// the float32 product it comes from), the integer sums are exact, and each
// flushed cell is converted back with one float32 product.
template <typename T> struct BoxCell { using type = T; };
template <> struct BoxCell<float> { using type = unsigned; };
constexpr float kFixOne = 4.29e9f;   // below 2^32 by more than the rounding of the deposits

template <int D> struct Tile;
// 2D: 16 x 32 tiles (two cells per lane) spread the tiles with mass of a
// compactly supported density over more workgroups than 32 x 32 did.
template <> struct Tile<2> { static constexpr int s[2] = {16, 32}; static constexpr int cells = 512; };
template <> struct Tile<3> { static constexpr int s[3] = {8, 8, 8}; static constexpr int cells = 512; };

// One float64 deposit per lane into the LDS box (key = box cell, or < 0 for
// none).
template <typename T>
__device__ __forceinline__ void box_deposit(T *box, int key, T w)
{
    if (key >= 0) atomicAdd(&box[key], w);
}

// Persistent workgroups walk the tiles in a grid-stride loop; a tile without
// mass is skipped after one vote.  With `tiles` (a count followed by tile
// indices, as tile_list_kernel writes them) only the listed tiles are walked:
// the sources of a solve do not change, so the tiles without mass are found
// once.  Partial sums are one per workgroup.
template <typename T> __device__ __forceinline__ T tpow(T x, T y) {
    if constexpr (sizeof(T) == 4)
        return powf(x, y);
    else
        return pow(x, y);
}

// One source tile: map, partial sums, deposition through the LDS box.  All
// lanes of the workgroup call it with the same tile (its barriers are
// uniform).  `box` is all zero on entry and on return; `bnd` holds the two
// alternating bound sets, `kused` counts the tiles with mass processed so far.
template <typename T, int D, bool GEN>
__device__ __forceinline__ void
splat_tile(const Grid &g, const int (&ntile)[D], const T (&pw)[D], const T (&ex)[D], const T (&hn)[D], long long tile,
           const T *__restrict__ pc, const T *__restrict__ src, T *__restrict__ rho, T *__restrict__ Tout, T tmix,
           typename BoxCell<T>::type *box, int (*bnd)[2 * D], float (*tmw)[kRedBlock / kWave], int &kused,
           double &accP, double &accJ)
{
    constexpr int PER = Tile<D>::cells / kRedBlock;   // cells per lane
    constexpr int kBoxCap = box_cap<T, D>();
    {
        int tc[D];
        long long rem = tile;
#pragma unroll
        for (int a = D - 1; a >= 0; --a) {
            tc[a] = (int)(rem % ntile[a]);
            rem /= ntile[a];
        }
        // source cells of this lane and their masses
        long long idx[PER];
        int ii[PER][D];
        T s[PER];
        bool any = false;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            int r = threadIdx.x + q * kRedBlock;   // inside the tile, last axis fastest
            bool inside = true;
            long long id = 0;
#pragma unroll
            for (int a = D - 1; a >= 0; --a) {
                ii[q][a] = tc[a] * Tile<D>::s[a] + r % Tile<D>::s[a];
                r /= Tile<D>::s[a];
                inside = inside && ii[q][a] < g.n[a];
                id += (long long)ii[q][a] * g.stride[a];
            }
            idx[q] = inside ? id : -1;
            s[q] = inside ? src[id] : T(0);
            any = any || s[q] != T(0);
        }
        if (!__syncthreads_or(any) && Tout == nullptr) return;
        // this tile's bounds; the other set was last read before the barrier
        // above, so it is reset here for the next tile
        int *bb = bnd[kused & 1];
        if (threadIdx.x < D) {
            bnd[(kused + 1) & 1][threadIdx.x] = 0x7fffffff;
            bnd[(kused + 1) & 1][D + threadIdx.x] = -1;
        }
        ++kused;

        T wup[PER][D];
        int lo[PER][D];
        long long base[PER];
        int bmin[D], bmax[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            bmin[a] = 0x7fffffff;
            bmax[a] = -1;
        }
        // phi^c at every source of the lane and its two neighbours per axis
        // (the face neighbour outside the grid replaced by the cell itself),
        // all loaded before any is used so that they are in flight together
        T pcv[PER][1 + 2 * D];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const bool ok = idx[q] >= 0;
            const long long id = ok ? idx[q] : 0;
            pcv[q][0] = pc[id];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int i = ii[q][a];
                const long long str = g.stride[a];
                pcv[q][1 + 2 * a] = pc[ok && i + 1 < g.n[a] ? id + str : id];
                pcv[q][2 + 2 * a] = pc[ok && i > 0 ? id - str : id];
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (idx[q] < 0 || (s[q] == T(0) && Tout == nullptr)) {
                s[q] = T(0);
                continue;
            }
            const long long id = idx[q];
            const T p0 = pcv[q][0];
            T sq = T(0);
            long long b = 0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int n = g.n[a];
                const long long str = g.stride[a];
                const int i = ii[q][a];
                const T fn = T(n);
                const T pp = pcv[q][1 + 2 * a], pm = pcv[q][2 + 2 * a];
                T d;
                if (i == 0)
                    d = (pp - p0) * fn;
                else if (i == n - 1)
                    d = (p0 - pm) * fn;
                else
                    d = (pp - pm) * (T(0.5) * fn);
                const T x = (T(i) + T(0.5)) * hn[a];   // cell centre (i + 1/2) h
                const T lo_t = T(0.5) * hn[a];
                if constexpr (GEN) {
                    if (pw[a] != T(2)) d = copysign(tpow(fabs(d), ex[a]), d);
                }
                T t = fmin(fmax(x - d, lo_t), T(1) - lo_t);
                if (tmix != T(1)) t = x + tmix * (t - x);   // displacement interpolation: t T(x) + (1 - t) x
                if (Tout != nullptr) Tout[(long long)a * g.N + id] = t;
                if constexpr (GEN)
                    sq += pw[a] == T(2) ? T(0.5) * (x - t) * (x - t) : tpow(fabs(x - t), pw[a]) / pw[a];
                else
                    sq += (x - t) * (x - t);
                const T qq = t * fn - T(0.5);
                int i0 = (int)floor(qq);
                i0 = min(max(i0, 0), n - 2);
                wup[q][a] = qq - T(i0);
                lo[q][a] = i0;
                b += (long long)i0 * str;
            }
            base[q] = b;
            if (s[q] != T(0) && rho != nullptr) {
                accP += (double)s[q] * (GEN ? 1.0 : 0.5) * (double)sq;
                accJ += (double)s[q] * (double)p0;
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    bmin[a] = min(bmin[a], lo[q][a]);
                    bmax[a] = max(bmax[a], lo[q][a] + 1);
                }
            } else {
                s[q] = T(0);
            }
        }
        // the tile's deposited mass (float32 fixed-point unit): per wave by
        // DPP row rotations and the four row sums, one LDS slot per wave
        if constexpr (sizeof(T) == 4) {
            float m = 0.f;
#pragma unroll
            for (int q = 0; q < PER; ++q) m += s[q];
            m += __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(m), __float_as_int(m), 0x121, 0xf, 0xf, false));
            m += __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(m), __float_as_int(m), 0x122, 0xf, 0xf, false));
            m += __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(m), __float_as_int(m), 0x124, 0xf, 0xf, false));
            m += __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(m), __float_as_int(m), 0x128, 0xf, 0xf, false));
            const float wm = (__int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 0)) +
                              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 16))) +
                             (__int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 32)) +
                              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 48)));
            if ((threadIdx.x & (kWave - 1)) == 0) tmw[kused & 1][threadIdx.x / kWave] = wm;
        }
        // box bounds: reduce across the wave first, one LDS atomic per wave
#pragma unroll
        for (int a = 0; a < D; ++a) {
            // rotations inside each 16-lane row (DPP), then the four row
            // results read out to scalars: no LDS permutes on this path
            int vmn = bmin[a], vmx = bmax[a];
            vmn = min(vmn, __builtin_amdgcn_update_dpp(vmn, vmn, 0x121, 0xf, 0xf, false));
            vmx = max(vmx, __builtin_amdgcn_update_dpp(vmx, vmx, 0x121, 0xf, 0xf, false));
            vmn = min(vmn, __builtin_amdgcn_update_dpp(vmn, vmn, 0x122, 0xf, 0xf, false));
            vmx = max(vmx, __builtin_amdgcn_update_dpp(vmx, vmx, 0x122, 0xf, 0xf, false));
            vmn = min(vmn, __builtin_amdgcn_update_dpp(vmn, vmn, 0x124, 0xf, 0xf, false));
            vmx = max(vmx, __builtin_amdgcn_update_dpp(vmx, vmx, 0x124, 0xf, 0xf, false));
            vmn = min(vmn, __builtin_amdgcn_update_dpp(vmn, vmn, 0x128, 0xf, 0xf, false));
            vmx = max(vmx, __builtin_amdgcn_update_dpp(vmx, vmx, 0x128, 0xf, 0xf, false));
            const int wmn = min(min(__builtin_amdgcn_readlane(vmn, 0), __builtin_amdgcn_readlane(vmn, 16)),
                                min(__builtin_amdgcn_readlane(vmn, 32), __builtin_amdgcn_readlane(vmn, 48)));
            const int wmx = max(max(__builtin_amdgcn_readlane(vmx, 0), __builtin_amdgcn_readlane(vmx, 16)),
                                max(__builtin_amdgcn_readlane(vmx, 32), __builtin_amdgcn_readlane(vmx, 48)));
            if ((threadIdx.x & (kWave - 1)) == 0 && wmx >= 0) {
                atomicMin(&bb[a], wmn);
                atomicMax(&bb[D + a], wmx);
            }
        }
        __syncthreads();
        if (rho == nullptr || bb[D] < 0) return;   // uniform: read after the barrier
        int bl[D], bs[D];
        long long area = 1;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            bl[a] = bb[a];
            bs[a] = bb[D + a] - bb[a] + 1;
            area *= bs[a];
        }
        // floor(r / bs) = umulhi(r, floor(2^32 / bs) + 1) whenever r * bs < 2^32
        // (here r < area <= 8192 and bs <= area); bs >= 2, since a box spans at
        // least two cells per axis, keeps the reciprocal within 32 bits
        unsigned bdiv[D];
#pragma unroll
        for (int a = 0; a < D; ++a) bdiv[a] = 0xffffffffu / (unsigned)bs[a] + 1u;
        float fix_scale = 0.f, fix_unit = 0.f;
        bool fits = area <= kBoxCap;
        if constexpr (sizeof(T) == 4) {
            float tm = 0.f;
#pragma unroll
            for (int w = 0; w < kRedBlock / kWave; ++w) tm += tmw[kused & 1][w];
            fits = fits && tm > 1e-30f;   // a unit too small for float32 goes to the global path
            fix_scale = kFixOne / tm;
            fix_unit = tm / kFixOne;
        }
        if (fits) {
            // the box is all zero here: cleared at the start and by every flush;
            // all lanes take part in each deposit (lanes without mass pass a
            // key of their own that is negative)
#pragma unroll
            for (int q = 0; q < PER; ++q) {
#pragma unroll
                for (int c = 0; c < (1 << D); ++c) {
                    T w = s[q];
                    int off = 0;
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        const int bit = (c >> (D - 1 - a)) & 1;
                        w *= bit ? wup[q][a] : T(1) - wup[q][a];
                        off = off * bs[a] + (lo[q][a] + bit - bl[a]);
                    }
                    if constexpr (sizeof(T) == 4) {
                        if (s[q] != T(0)) atomicAdd(&box[off], (unsigned)(w * fix_scale + 0.5f));
                    } else {
                        box_deposit(box, s[q] != T(0) ? off : -1 - (int)(threadIdx.x & (kWave - 1)), w);
                    }
                }
            }
            __syncthreads();
            for (int e = threadIdx.x; e < area; e += kRedBlock) {
                T v;
                if constexpr (sizeof(T) == 4) {
                    const unsigned qv = box[e];
                    box[e] = 0u;
                    v = qv != 0u ? (float)qv * fix_unit : 0.f;
                } else {
                    v = box[e];
                    box[e] = T(0);
                }
                if (v != T(0)) {
                    // box cell e -> grid index; division by the box sizes as a
                    // high product with a per-tile reciprocal
                    unsigned r = (unsigned)e;
                    long long gi = 0;
#pragma unroll
                    for (int a = D - 1; a >= 0; --a) {
                        const unsigned qd = __umulhi(r, bdiv[a]);
                        gi += (long long)(bl[a] + (int)(r - qd * (unsigned)bs[a])) * g.stride[a];
                        r = qd;
                    }
                    atomicAdd(rho + gi, v);
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                if (s[q] == T(0)) continue;
#pragma unroll
                for (int c = 0; c < (1 << D); ++c) {
                    T w = s[q];
                    long long off = base[q];
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        const int bit = (c >> (D - 1 - a)) & 1;
                        w *= bit ? wup[q][a] : T(1) - wup[q][a];
                        off += bit ? g.stride[a] : 0;
                    }
                    atomicAdd(rho + off, w);
                }
            }
        }
        // no barrier: the next tile deposits into the box only after its own
        // two barriers, which this flush precedes
    }
}

template <typename T, int D>
__device__ __forceinline__ void splat_setup(const Grid &g, int (&ntile)[D], T (&pw)[D], T (&ex)[D], T (&hn)[D])
{
#pragma unroll
    for (int a = 0; a < D; ++a) {
        ntile[a] = (g.n[a] + Tile<D>::s[a] - 1) / Tile<D>::s[a];
        pw[a] = T(g.pw[a]);
        ex[a] = T(1.0 / (g.pw[a] - 1.0));
        hn[a] = T(1) / T(g.n[a]);
    }
}

// First tile of workgroup b in the walk over a list of tiles with grid G:
// workgroups are dispatched round-robin over the 8 XCDs, so with G a
// multiple of 8 the XCD of b (b mod 8) takes a contiguous eighth of each
// round of G tiles.  Neighbouring tiles share cache lines (a 3D tile row is
// 32 bytes of a 128-byte line, and the deposits of neighbouring tiles
// overlap), which then meet in one XCD's L2.  Tile k + G follows tile k.
__device__ __forceinline__ long long splat_first_tile(long long b, long long G)
{
    return (G & 7) == 0 ? (b & 7) * (G >> 3) + (b >> 3) : b;
}

template <typename T, int D>
__device__ __forceinline__ void splat_clear(typename BoxCell<T>::type *box, int (*bnd)[2 * D])
{
    for (int e = threadIdx.x; e < box_cap<T, D>(); e += kRedBlock) box[e] = 0;
    if (threadIdx.x < 2 * D) {
        bnd[threadIdx.x / D][threadIdx.x % D] = 0x7fffffff;
        bnd[threadIdx.x / D][D + threadIdx.x % D] = -1;
    }
    __syncthreads();
}

template <typename T, int D, bool GEN>
__global__ void __launch_bounds__(kRedBlock)
splat_kernel(Grid g, long long ntiles_total, const T *__restrict__ pc, const T *__restrict__ src,
             T *__restrict__ rho, T *__restrict__ Tout, double *__restrict__ part_primal,
             double *__restrict__ part_pcsrc, const int32_t *__restrict__ done, T tmix,
             const int *__restrict__ tiles)
{
    if (done != nullptr && *done) return;
    __shared__ double sh[kRedBlock / kWave];
    __shared__ typename BoxCell<T>::type box[box_cap<T, D>()];
    __shared__ int bnd[2][2 * D];   // box bounds, alternating between consecutive tiles with mass
    __shared__ float tmw[2][kRedBlock / kWave];   // per-wave tile mass, same alternation
    int ntile[D];
    T pw[D], ex[D], hn[D];   // exponent p_a of the cost, 1 / (p_a - 1), 1 / n_a
    splat_setup<T, D>(g, ntile, pw, ex, hn);
    double accP = 0.0, accJ = 0.0;
    splat_clear<T, D>(box, bnd);
    int kused = 0;   // tiles with mass processed so far by this workgroup
    const long long count = tiles != nullptr ? (long long)tiles[0] : ntiles_total;
    for (long long k = splat_first_tile(blockIdx.x, gridDim.x); k < count; k += gridDim.x) {
        const long long tile = tiles != nullptr ? (long long)tiles[1 + k] : k;
        splat_tile<T, D, GEN>(g, ntile, pw, ex, hn, tile, pc, src, rho, Tout, tmix, box, bnd, tmw, kused, accP,
                              accJ);
    }
    const double P = block_reduce<R_SUM>(accP, sh);
    const double J = block_reduce<R_SUM>(accJ, sh);
    if (threadIdx.x == 0) {
        if (part_primal != nullptr) part_primal[blockIdx.x] = P;
        if (part_pcsrc != nullptr) part_pcsrc[blockIdx.x] = J;
    }
}

// ------------------------------------------------------------ multi-pair
// The deposition of every pair of a batch (2D, quadratic cost) in one launch:
// the pairs' lists of tiles with mass are walked as one joint list (pair p's
// entries start at ent_mu / ent_nu), splat_grid workgroups (at most
// kBatchSplatGrid, at most the pairs' tile count) striding over it.  A workgroup keeps its sums per pair and writes them when its walk
// leaves the pair, at index (first entry it visited - the pair's first
// entry): every workgroup walks one residue class modulo the grid, so the
// pair's partials are indices 0 .. min(grid, entries) - 1, one each.
template <typename T>
__global__ void __launch_bounds__(kRedBlock)
splat_multi_kernel(const BatchHead *__restrict__ tab, int role)
{
    constexpr int D = 2;
    __shared__ double sh[kRedBlock / kWave];
    __shared__ typename BoxCell<T>::type box[box_cap<T, D>()];
    __shared__ int bnd[2][2 * D];
    __shared__ float tmw[2][kRedBlock / kWave];
    const PairDev *pairs = reinterpret_cast<const PairDev *>(tab + 1);
    const int np = tab->np;
    const int total = role ? tab->ent_total_nu : tab->ent_total_mu;
    splat_clear<T, D>(box, bnd);
    int kused = 0, cur = -1;
    double accP = 0.0, accJ = 0.0;
    long long first = 0;
    Grid g{};
    int ntile[D];
    T pw[D], ex[D], hn[D];
    const T *pc = nullptr, *src = nullptr;
    T *rho = nullptr;
    const int *tiles = nullptr;
    bool skip = false;
    auto flush = [&]() {
        const double P = block_reduce<R_SUM>(accP, sh);
        const double J = block_reduce<R_SUM>(accJ, sh);
        if (threadIdx.x == 0 && !skip) {
            const PairDev &Q = pairs[cur];
            const long long i = first - (role ? Q.ent_nu : Q.ent_mu);
            Q.part[S_PRIMAL * Q.slot_len + i] = P;
            Q.part[S_PC_SRC * Q.slot_len + i] = J;
        }
        accP = accJ = 0.0;
    };
    for (long long k = splat_first_tile(blockIdx.x, gridDim.x); k < total; k += gridDim.x) {
        int p = cur < 0 ? 0 : cur;
        while (p + 1 < np && (role ? pairs[p + 1].ent_nu : pairs[p + 1].ent_mu) <= k) ++p;
        if (p != cur) {
            if (cur >= 0) flush();
            cur = p;
            first = k;
            const PairDev &Q = pairs[p];
            skip = ((tab->done_mask >> p) & 1ull) != 0;
            g.ndim = 2;
            g.n[0] = Q.n0;
            g.n[1] = Q.n1;
            g.n[2] = 1;
            g.stride[0] = Q.n1;
            g.stride[1] = 1;
            g.stride[2] = 0;
            g.N = (long long)Q.n0 * Q.n1;
            g.vol = 1.0 / (double)g.N;
            g.pw[0] = g.pw[1] = g.pw[2] = 2.0;
            splat_setup<T, D>(g, ntile, pw, ex, hn);
            pc = (const T *)Q.pc;
            src = (const T *)(role ? Q.nu : Q.mu);
            rho = (T *)Q.rho;
            tiles = role ? Q.tiles_nu : Q.tiles_mu;
        }
        if (skip) continue;   // uniform: the pair has stopped
        const long long tile = tiles[1 + (k - (role ? pairs[p].ent_nu : pairs[p].ent_mu))];
        splat_tile<T, D, false>(g, ntile, pw, ex, hn, tile, pc, src, rho, nullptr, T(1), box, bnd, tmw, kused,
                                accP, accJ);
    }
    if (cur >= 0) flush();
}

// The map of every pair of a batch that has a map output (2D, quadratic
// cost): T_a = x_a - d_a clamped to the cell-centre box, d by central
// differences of phi^c (one-sided on the faces), with the same operations as
// the deposition's map.  kMapCells cells per workgroup.
constexpr int kMapCells = 4 * kRedBlock;

template <typename T>
__global__ void __launch_bounds__(kRedBlock) map_multi_kernel(const BatchHead *__restrict__ tab, BatchIdx bi)
{
    int lo = 0, hi = bi.np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bi.off[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const PairDev &P = reinterpret_cast<const PairDev *>(tab + 1)[lo];
    const long long N = (long long)P.n0 * P.n1;
    const long long c0 = ((long long)blockIdx.x - bi.off[lo]) * kMapCells;
    const T *pc = (const T *)P.pc;
    T *Tout = (T *)P.Tmap;
    const int nn[2] = {P.n0, P.n1};
    const long long str[2] = {P.n1, 1};
    for (long long id = c0 + threadIdx.x; id < c0 + kMapCells && id < N; id += kRedBlock) {
        const int ii[2] = {(int)(id / P.n1), (int)(id % P.n1)};
        const T p0 = pc[id];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int n = nn[a], i = ii[a];
            const T fn = T(n);
            const T pp = pc[i + 1 < n ? id + str[a] : id], pm = pc[i > 0 ? id - str[a] : id];
            T d;
            if (i == 0)
                d = (pp - p0) * fn;
            else if (i == n - 1)
                d = (p0 - pm) * fn;
            else
                d = (pp - pm) * (T(0.5) * fn);
            const T hn = T(1) / fn;   // as the deposition: (i + 1/2) h with h = 1 / n
            const T x = (T(i) + T(0.5)) * hn;
            const T lo_t = T(0.5) * hn;
            Tout[(long long)a * N + id] = fmin(fmax(x - d, lo_t), T(1) - lo_t);
        }
    }
}

template <typename T>
hipError_t launch_map_multi(const BatchHead *tab, const int *n0s, const int *n1s, int np, hipStream_t stream)
{
    if (np < 1 || np > kBatchChunk) return hipErrorInvalidValue;
    BatchIdx bi{};
    bi.np = np;
    for (int p = 0; p < np; ++p)
        bi.off[p + 1] = bi.off[p] + (n0s[p] > 0 ? (int)(((long long)n0s[p] * n1s[p] + kMapCells - 1) / kMapCells) : 0);
    if (bi.off[np] == 0) return hipSuccess;
    hipLaunchKernelGGL((map_multi_kernel<T>), dim3((unsigned)bi.off[np]), dim3(kRedBlock), 0, stream, tab, bi);
    return hipGetLastError();
}

// Joint-list offsets of the pairs' deposition tiles (one lane: at most
// kBatchChunk pairs).
__global__ void batch_entries_kernel(BatchHead *tab)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    PairDev *pairs = reinterpret_cast<PairDev *>(tab + 1);
    int am = 0, an = 0;
    for (int p = 0; p < tab->np; ++p) {
        pairs[p].ent_mu = am;
        pairs[p].ent_nu = an;
        am += pairs[p].tiles_mu[0];
        an += pairs[p].tiles_nu[0];
    }
    tab->ent_total_mu = am;
    tab->ent_total_nu = an;
}

hipError_t launch_batch_entries(BatchHead *tab, hipStream_t stream)
{
    hipLaunchKernelGGL(batch_entries_kernel, dim3(1), dim3(64), 0, stream, tab);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_splat_multi(const BatchHead *tab, int np, int role, int grid, hipStream_t stream)
{
    if (np < 1 || np > kBatchChunk || grid < 1 || grid > kBatchSplatGrid) return hipErrorInvalidValue;
    hipLaunchKernelGGL((splat_multi_kernel<T>), dim3(grid), dim3(kRedBlock), 0, stream, tab, role);
    return hipGetLastError();
}

template <int D> long long splat_tiles(const Grid &g) {
    long long t = 1;
    for (int a = 0; a < D; ++a) t *= (g.n[a] + Tile<D>::s[a] - 1) / Tile<D>::s[a];
    return t;
}

static long long splat_ntiles(const Grid &g) { return g.ndim == 2 ? splat_tiles<2>(g) : splat_tiles<3>(g); }

// Workgroups of the deposition kernel: one per tile up to 2048 (eight per CU).
long long splat_blocks(const Grid &g) {
    const long long t = splat_ntiles(g);
    return t < 2048 ? t : 2048;
}

long long splat_tile_count(const Grid &g) { return splat_ntiles(g); }

// flags[tile] = 1 when some source cell of the tile holds mass
template <typename T, int D>
__global__ void __launch_bounds__(kRedBlock)
tile_flag_kernel(Grid g, long long ntiles, const T *__restrict__ src, int *__restrict__ flags)
{
    constexpr int PER = Tile<D>::cells / kRedBlock;
    int ntile[D];
#pragma unroll
    for (int a = 0; a < D; ++a) ntile[a] = (g.n[a] + Tile<D>::s[a] - 1) / Tile<D>::s[a];
    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int tc[D];
        long long rem = tile;
#pragma unroll
        for (int a = D - 1; a >= 0; --a) {
            tc[a] = (int)(rem % ntile[a]);
            rem /= ntile[a];
        }
        bool any = false;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            int r = threadIdx.x + q * kRedBlock;
            bool inside = true;
            long long id = 0;
#pragma unroll
            for (int a = D - 1; a >= 0; --a) {
                const int i = tc[a] * Tile<D>::s[a] + r % Tile<D>::s[a];
                r /= Tile<D>::s[a];
                inside = inside && i < g.n[a];
                id += (long long)i * g.stride[a];
            }
            any = any || (inside && src[id] != T(0));
        }
        const int f = __syncthreads_or(any);
        if (threadIdx.x == 0) flags[tile] = f;
    }
}

// list[0] = number of flagged tiles, list[1..] = their indices in tile order
// (one workgroup: contiguous runs of flags per lane and a block scan, so the
// order, and with it every partial sum of the deposition, is deterministic)
constexpr int kListBlock = 1024;
__global__ void __launch_bounds__(kListBlock)
tile_list_kernel(const int *__restrict__ flags, long long ntiles, int *__restrict__ list)
{
    __shared__ int wsum[kListBlock / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const long long per = (ntiles + kListBlock - 1) / kListBlock;
    const long long b0 = t * per, b1 = b0 + per < ntiles ? b0 + per : ntiles;
    int cnt = 0;
    for (long long i = b0; i < b1; ++i) cnt += flags[i] != 0;
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int off = 0, total = 0;
    for (int q = 0; q < kListBlock / kWave; ++q) {
        off += q < w ? wsum[q] : 0;
        total += wsum[q];
    }
    int pos = off + incl - cnt;
    for (long long i = b0; i < b1; ++i)
        if (flags[i] != 0) list[1 + pos++] = (int)i;
    if (t == 0) list[0] = total;
}

template <typename T>
hipError_t launch_tile_list(const Grid &g, const T *src, int *flags, int *list, hipStream_t stream)
{
    const long long nt = splat_ntiles(g);
    const long long nb = nt < 4096 ? nt : 4096;
    if (g.ndim == 2)
        hipLaunchKernelGGL((tile_flag_kernel<T, 2>), dim3((unsigned)nb), dim3(kRedBlock), 0, stream, g, nt, src, flags);
    else if (g.ndim == 3)
        hipLaunchKernelGGL((tile_flag_kernel<T, 3>), dim3((unsigned)nb), dim3(kRedBlock), 0, stream, g, nt, src, flags);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tile_list_kernel, dim3(1), dim3(kListBlock), 0, stream, flags, nt, list);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_splat(const Grid &g, const T *pc, const T *src, T *rho, T *Tout, double *part_primal,
                        double *part_pcsrc, int nblocks, const int32_t *done, hipStream_t stream, T tmix,
                        const int *tiles)
{
    const long long nb = nblocks > 0 ? nblocks : splat_blocks(g), nt = splat_ntiles(g);
    const bool gen = !grid_quadratic(g);
#define BFM_SPLAT(D_, G_)                                                                                        \
    hipLaunchKernelGGL((splat_kernel<T, D_, G_>), dim3((unsigned)nb), dim3(kRedBlock), 0, stream, g, nt, pc, src, \
                       rho, Tout, part_primal, part_pcsrc, done, tmix, tiles)
    if (g.ndim == 2 && !gen)
        BFM_SPLAT(2, false);
    else if (g.ndim == 2)
        BFM_SPLAT(2, true);
    else if (g.ndim == 3 && !gen)
        BFM_SPLAT(3, false);
    else if (g.ndim == 3)
        BFM_SPLAT(3, true);
    else
        return hipErrorInvalidValue;
#undef BFM_SPLAT
    return hipGetLastError();
}

template hipError_t launch_splat<float>(const Grid &, const float *, const float *, float *, float *, double *,
                                        double *, int, const int32_t *, hipStream_t, float, const int *);
template hipError_t launch_splat<double>(const Grid &, const double *, const double *, double *, double *,
                                         double *, double *, int, const int32_t *, hipStream_t, double, const int *);
template hipError_t launch_tile_list<float>(const Grid &, const float *, int *, int *, hipStream_t);
template hipError_t launch_splat_multi<float>(const BatchHead *, int, int, int, hipStream_t);
template hipError_t launch_map_multi<float>(const BatchHead *, const int *, const int *, int, hipStream_t);
template hipError_t launch_map_multi<double>(const BatchHead *, const int *, const int *, int, hipStream_t);
template hipError_t launch_splat_multi<double>(const BatchHead *, int, int, int, hipStream_t);
template hipError_t launch_tile_list<double>(const Grid &, const double *, int *, int *, hipStream_t);

}  // namespace bfm
