// Host-side launchers shared between the library's translation units.
#pragma once

#include "common.hpp"

namespace bfm {

// Per-axis spectral plan: FFT stage counts (n = 16^a 8^b 4^c 2^d 3^e packed
// as a | b << 6 | c << 12 | d << 18 | e << 24) and the stride of the axis.
struct AxisPlan {
    int n;
    int inner;
    uint32_t radices;
    int nstages;
};

// Launch facts kept per device (ids below kMaxDevices; for others they are
// looked up or set again at every call).
constexpr int kMaxDevices = 64;

// Compute units of the current device.
inline int device_cu_count()
{
    static int ncu[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    const bool known = dev >= 0 && dev < kMaxDevices;
    if (known && ncu[dev] > 0) return ncu[dev];
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    if (known) ncu[dev] = n;
    return n;
}

// Raises fn's dynamic LDS limit on the current device to `bytes` when that
// exceeds the 64 KB default and what was set before; `limit` (one array per
// kernel) records per device the largest value set so far.
inline hipError_t raise_dyn_lds(const void *fn, size_t bytes, size_t (&limit)[kMaxDevices])
{
    if (bytes <= 64 * 1024) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const bool known = dev >= 0 && dev < kMaxDevices;
    if (known && limit[dev] >= bytes) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess && known) limit[dev] = bytes;
    return e;
}

// c-transform (ctransform.hip).  CtCfg overrides the launch shape of one
// axis (0 = built-in choice): C points per lane, lines per workgroup on a
// strided axis (1, 2 or 4), pers = 1 one line group per workgroup, 2 persistent
// workgroups with prefetch (aligned layouts only).
struct CtCfg {
    int C = 0;
    int lpb = 0;
    int pers = 0;
};
template <typename T>
bool ct_blocked_applies(const Grid &g, const void *in, const void *mid, const void *out, const CtCfg *cfg);
template <typename T>
hipError_t ct_blocked_pass(const Grid &g, int pass, const T *in, T *out, const int32_t *done, hipStream_t stream,
                           const CtCfg *cfg, const T *dotw = nullptr, double *dotpart = nullptr, int *ndot = nullptr);
// With `scratch`, 2D fields may take the column-blocked two-pass form; when
// it does and dotw is given, its second pass also writes one float64 partial
// per workgroup of sum out * dotw into dotpart and sets *ndot to their count
// (otherwise *ndot = 0).
template <typename T>
hipError_t ctransform_field(const Grid &g, const T *in, T *out, const int32_t *done, hipStream_t stream,
                            const CtCfg *cfg = nullptr, T *scratch = nullptr, const T *dotw = nullptr,
                            double *dotpart = nullptr, int *ndot = nullptr);
template <typename T>
hipError_t launch_ct_axis(const T *in, T *out, int n, int inner, long long nlines, T sgn,
                          const int32_t *done, hipStream_t stream, CtCfg cfg = CtCfg{});
int ct_threads_per_line(int n);
// One axis of the c-transform for the power cost |z|^p / p, p != 2
// (ctransform_dc.hip): out = min_j |i - j|^p h^p / p + sgn * in_j per line.
template <typename T>
hipError_t launch_ct_dc(const T *in, T *out, int n, int inner, long long nlines, T sgn, double p,
                        const int32_t *done, hipStream_t stream);
// true when every axis of the grid has the quadratic cost
inline bool grid_quadratic(const Grid &g) {
    for (int a = 0; a < g.ndim; ++a)
        if (g.pw[a] != 2.0) return false;
    return true;
}
template <typename T> size_t ct_smem_bytes(int n, int tpl, int lpb);

// DCT Poisson (dct.hip)
template <typename T>
hipError_t launch_dct_fwd(const T *a, T *b, T *out, const AxisPlan &ap, long long N, int zero_b, const void *tw,
                          const void *qw, const int32_t *done, hipStream_t stream);
template <typename T>
// dotw (contiguous axis only): also one float64 partial per workgroup of
// sum out * dotw into dotpart[workgroup] ((lines + 1) / 2 workgroups).
hipError_t launch_dct_inv(const T *in, T *out, const T *base, const double *scale, const AxisPlan &ap, long long N,
                          const void *tw, const void *qw, const int32_t *done, hipStream_t stream,
                          const T *dotw = nullptr, double *dotpart = nullptr);
template <typename T>
hipError_t launch_dct_fused(T *X, const AxisPlan &ap0, long long N, int nA, int nB, const void *tw, const void *qw,
                            const T *lam0, const T *lamA, const T *lamB, double *gpart, int *nparts,
                            const int32_t *done, hipStream_t stream);
long long dct_fused_parts(int n0, long long N, size_t esz);

// map, pushforward, reductions, controller (pushforward.hip, reduce.hip)
// tiles (nullable): count followed by the indices of the source tiles with
// mass, from launch_tile_list; only those tiles are deposited.  nblocks:
// workgroups (0: splat_blocks); part_* receive one partial per workgroup.
template <typename T>
hipError_t launch_splat(const Grid &g, const T *pc, const T *src, T *rho, T *Tout, double *part_primal,
                        double *part_pcsrc, int nblocks, const int32_t *done, hipStream_t stream, T tmix = T(1),
                        const int *tiles = nullptr);
// list of the deposition tiles of src that hold mass (flags: splat_tile_count
// ints of scratch; list: splat_tile_count + 1 ints)
template <typename T>
hipError_t launch_tile_list(const Grid &g, const T *src, int *flags, int *list, hipStream_t stream);
long long splat_tile_count(const Grid &g);
template <typename T>
hipError_t launch_dot2(const T *a1, const T *b1, const T *a2, const T *b2, long long N, double *part1,
                       double *part2, int nblocks, const int32_t *done, hipStream_t stream);
template <typename T>
hipError_t launch_stats(const T *mu, const T *nu, long long N, double *partials, long long slot_len, int nblocks,
                        hipStream_t stream);
long long splat_blocks(const Grid &g);
constexpr int kMaxDepositGrid = 8192;   // most deposition workgroups a plan's slots hold
template <typename T>
hipError_t launch_fill(T *x, long long N, T value, hipStream_t stream);
template <typename T>
hipError_t launch_shift_scale(T *out_a, const T *in_a, const double *shift_a, double sign_a, T *out_b,
                              const T *in_b, const double *shift_b, double sign_b, long long N, double mul,
                              hipStream_t stream);

// Controller modes
enum CtrlMode {
    CTRL_INIT = 0,     // masses, extrema, sigma0
    CTRL_HEAD_PHI,     // J(phi_n), P_n, G_n, gap, stop test, trace
    CTRL_STEP_PHI,     // J(phi_{n+1/2}) and the sigma update
    CTRL_HEAD_PSI,     // I(psi_{n+1/2}), G
    CTRL_STEP_PSI,     // I(psi_{n+1}), sigma update, iteration count
    CTRL_MEANS,        // mean_a, mean_b from S_MEAN_A / S_MEAN_B
    CTRL_GA_NEXT       // gradient ascent: sum phi_{n+1} * nu from S_Q_TGT (prm.nqt partials)
                       // kept for the next head, iteration count
};
// Head modes OR'ed with this flag take sum p * tgt from the previous step's
// sum q * src (the same products: p of a head is q of the step before it),
// or, in gradient ascent, from the sum CTRL_GA_NEXT kept.
constexpr int CTRL_REUSE_DOT = 0x100;

struct CtrlParams {
    double tol, sigma0, sigma_min, beta1, beta2, alpha1, alpha2, vol, inv_N;
    long long slot_len;   // stride between reduction slots
    int nred;             // partials of the grid-stride kernels (dot products, statistics)
    int nsplat;           // partials of the deposition kernel (S_PRIMAL, S_PC_SRC)
    int ngpart;           // partials of G (separate array)
    int nqt, nqs;         // partials in S_Q_TGT and S_Q_SRC (fused sums or the dot kernel's)
};

hipError_t launch_ctrl(DevState *st, const double *partials, const double *gpart, int mode, CtrlParams prm,
                       TraceRec *trace, hipStream_t stream);

// ------------------------------------------------------------ multi-pair
// Batched form: many independent 2D problems advanced by one launch per pass.
// The pairs of one launch (at most kBatchChunk) are described by a device
// table of PairDev records (kept in the workspace of the chunk's first
// pair); each launch also takes, by value, the prefix of its workgroups per
// pair (BatchIdx), so a workgroup finds its pair by a binary search over
// kernel arguments.
constexpr int kBatchChunk = 64;
constexpr int kBatchSplatGrid = 2048;   // most workgroups of the joint deposition

struct PairDev {
    const void *mu, *nu;
    void *phi, *psi;
    void *pc, *rho, *F;
    DevState *st;
    TraceRec *trace;
    double *part;        // kNumSlots slots of slot_len float64 partials
    double *gpart;       // partials of G from the fused Poisson pass
    const unsigned char *tables;
    const int *tiles_mu, *tiles_nu;   // count, then the tiles of mu / nu that hold mass
    long long slot_len;
    int n0, n1;
    int tw[2], qw[2], lam[2];   // byte offsets of the axis tables in `tables`
    uint32_t radices[2];
    int ent_mu, ent_nu;         // first entry of the pair in the joint deposition lists (device-filled)
    CtrlParams cp;              // controller parameters with the multi-pair partial counts
    void *Tmap;                 // map output (2 planar fields) or null
};
// Table header in device memory, followed by the PairDev records.
struct BatchHead {
    int np;
    int ent_total_mu, ent_total_nu;   // lengths of the joint deposition lists (device-filled)
    int all_done;                     // 1 when every pair's stop flag is set (launch_batch_done)
    int splat_grid;                   // workgroups of the joint deposition launch (host-set)
    int nactive;                      // pairs whose stop flag is clear (launch_batch_done)
    unsigned long long done_mask;     // bit p: pair p has stopped (set by the controller, launch_batch_done)
};
static_assert(sizeof(BatchHead) % 8 == 0, "the pair table after the head stays 8-byte aligned");
constexpr size_t kBatchTableBytes = sizeof(BatchHead) + kBatchChunk * sizeof(PairDev);

struct BatchIdx {
    int np;
    int off[kBatchChunk + 1];   // first workgroup of each pair; off[np] = grid size
};

// role 0: the phi-step (p, src, tgt, q) = (phi, mu, nu, psi); role 1: the
// psi-step (psi, nu, mu, phi).  Every launch skips pairs whose stop flag is set.
enum MultiCt { MCT_HEAD = 0, MCT_STEP = 1 };
template <typename T>
hipError_t launch_ct_multi(const BatchHead *tab, const int *n0s, const int *n1s, int np, int role, int which,
                           hipStream_t stream);
template <typename T>
hipError_t launch_splat_multi(const BatchHead *tab, int np, int role, int grid, hipStream_t stream);
hipError_t launch_batch_entries(BatchHead *tab, hipStream_t stream);
// modes of launch_dct_multi (the DCT pass kinds of dct.hip)
constexpr int kDctFwd = 0, kDctInv = 1, kDctFused = 2;
template <typename T>
hipError_t launch_dct_multi(const BatchHead *tab, const int *n0s, const int *n1s, int np, int role, int mode,
                            hipStream_t stream);
hipError_t launch_ctrl_multi(BatchHead *tab, int np, int role, int mode, hipStream_t stream);
hipError_t launch_batch_done(BatchHead *tab, hipStream_t stream);
// Batched W2^2 gradient: per pair, the potentials' sums (one partial per
// workgroup into S_MEAN_A (psi) and S_MEAN_B (phi)), the means (one workgroup
// per pair), then gmu = mul (psi - mean psi), gnu = mul (phi - mean phi).
struct GradPair {
    const void *phi, *psi;
    void *gmu, *gnu;     // either may be null
    DevState *st;
    double *part;
    long long slot_len;
    long long N;
    long long epb;       // elements per workgroup (a multiple of 4 * kRedBlock)
    int nb;              // workgroups of the pair
    double mul;          // 2 cell_volume scale
};
constexpr size_t kGradTableBytes = kBatchChunk * sizeof(GradPair);
static_assert(kGradTableBytes <= kBatchTableBytes, "gradient table fits the batch region");
template <typename T>
hipError_t launch_grad_multi(const GradPair *tab, const GradPair *host, int np, hipStream_t stream);

// The outputs of every pair after its last head: phi - mean(phi) and
// phi^c + mean(phi) (three launches; epb elements per workgroup, chosen so
// that no pair has more workgroups than its slots hold).
template <typename T>
hipError_t launch_finish_multi(const BatchHead *tab, const int *n0s, const int *n1s, int np, long long epb,
                               hipStream_t stream);
// T = x - grad phi^c of every pair with a map output (PairDev::Tmap)
template <typename T>
hipError_t launch_map_multi(const BatchHead *tab, const int *n0s, const int *n1s, int np, hipStream_t stream);

// partial counts the multi-pair launches leave per pair (for CtrlParams)
int ct_multi_col_groups(int n0, int n1);
long long dct_multi_inv_parts(int n0);

}  // namespace bfm
