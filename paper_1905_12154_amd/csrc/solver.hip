// Host side of the C ABI: parameter validation, plans, workspace layout,
// spectral tables and the back-and-forth loop (Algorithm 1) enqueued on a
// HIP stream, with the step-size state kept on the device.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "launch.hpp"

using namespace bfm;

// ----------------------------------------------------------------- errors

static thread_local std::string g_last_error;

static bfm_status fail(bfm_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return fail(BFM_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                                  \
    } while (0)

extern "C" const char *bfm_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *bfm_version(void) { return "bfm-gfx950 0.1"; }

// ------------------------------------------------------------------ plan

struct bfm_plan_s {
    bfm_params prm;
    Grid g;
    size_t esz;
    AxisPlan ax[3];
    int red_blocks;
    int gparts;      // partial sums of G written by the fused Poisson pass
    int nsplat;      // workgroups of the deposition kernel
    long long slot_len;
    CtCfg ct_cfg[3];   // c-transform launch shape per axis (autotuned or built-in)
    // workspace layout (byte offsets from the workspace base)
    size_t off_state, off_trace, off_part, off_gpart, off_tables, off_pc, off_rho, off_f, total;
    size_t off_tiles_mu, off_tiles_nu;   // deposition tiles of mu and nu that hold mass
    size_t off_batch;                    // multi-pair table of a batch led by this pair
    long long ntiles;
    size_t tab_tw[3], tab_qw[3], tab_lam[3];   // offsets inside the table image
    std::vector<unsigned char> tables;         // host image of the spectral tables
};

static bool is_2a3b(int n)
{
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// FFT stage counts: n = 16^n16 8^n8 4^n4 2^n2 3^n3 with as many radix-16
// stages as the power of two allows and at most one of radix 8, 4 or 2;
// packed as n16 | n8 << 6 | n4 << 12 | n2 << 18 | n3 << 24.
static bool factor_radices(int n, uint32_t *code, int *nstages)
{
    uint32_t p2 = 0, n3 = 0;
    while (n % 2 == 0) { ++p2; n /= 2; }
    while (n % 3 == 0) { ++n3; n /= 3; }
    if (n != 1) return false;
    const uint32_t n16 = p2 / 4, r = p2 % 4;
    const uint32_t n8 = r == 3, n4 = r == 2, n2 = r == 1;
    *code = n16 | (n8 << 6) | (n4 << 12) | (n2 << 18) | (n3 << 24);
    *nstages = (int)(n16 + n8 + n4 + n2 + n3);
    return true;
}

static bfm_status check_params(const bfm_params *p)
{
    if (p == nullptr) return fail(BFM_EINVAL, "params is NULL");
    if (p->ndim != 2 && p->ndim != 3) return fail(BFM_EINVAL, "ndim must be 2 or 3 (got %d)", p->ndim);
    for (int a = 0; a < p->ndim; ++a) {
        const int n = p->shape[a];
        if (n < 4 || n > 4096 || !is_2a3b(n))
            return fail(BFM_EINVAL, "shape[%d] = %d: need 4 <= n <= 4096 and n = 2^a 3^b", a, n);
    }
    if (p->dtype != BFM_F32 && p->dtype != BFM_F64) return fail(BFM_EINVAL, "dtype must be BFM_F32 or BFM_F64");
    if (p->max_iters < 0) return fail(BFM_EINVAL, "max_iters must be >= 0");
    if (!(p->tol >= 0.0) || !isfinite(p->tol)) return fail(BFM_EINVAL, "tol must be finite and >= 0");
    if (!isfinite(p->sigma0)) return fail(BFM_EINVAL, "sigma0 must be finite");
    if (!(p->sigma_min > 0.0) || !isfinite(p->sigma_min)) return fail(BFM_EINVAL, "sigma_min must be > 0");
    if (!(0.0 < p->beta1 && p->beta1 < p->beta2 && p->beta2 < 1.0))
        return fail(BFM_EINVAL, "need 0 < beta1 < beta2 < 1");
    if (!(p->alpha1 > 1.0 && p->alpha2 > 0.0 && p->alpha2 < 1.0) || !isfinite(p->alpha1))
        return fail(BFM_EINVAL, "need alpha1 > 1 and 0 < alpha2 < 1");
    if (p->check_every < 1) return fail(BFM_EINVAL, "check_every must be >= 1");
    if (p->method != BFM_METHOD_BFM && p->method != BFM_METHOD_GA)
        return fail(BFM_EINVAL, "method must be BFM_METHOD_BFM or BFM_METHOD_GA (got %d)", p->method);
    for (int a = 0; a < p->ndim; ++a)
        if (!(p->power[a] >= 1.05 && p->power[a] <= 8.0))
            return fail(BFM_EINVAL, "power[%d] = %g: the cost exponent must lie in [1.05, 8]", a, p->power[a]);
    return BFM_OK;
}

extern "C" bfm_status bfm_params_init(bfm_params *p, int32_t ndim, const int32_t *shape, int32_t dtype)
{
    if (p == nullptr || shape == nullptr) return fail(BFM_EINVAL, "NULL argument");
    memset(p, 0, sizeof(*p));
    p->ndim = ndim;
    for (int a = 0; a < ndim && a < 3; ++a) p->shape[a] = shape[a];
    p->dtype = dtype;
    p->max_iters = 60;
    p->tol = 0.0;
    p->sigma0 = 0.0;
    p->sigma_min = 0.01;
    p->beta1 = 0.25;
    p->beta2 = 0.75;
    p->alpha1 = 1.25;
    p->alpha2 = 0.8;
    p->check_every = 8;
    p->method = BFM_METHOD_BFM;
    p->power[0] = p->power[1] = p->power[2] = 2.0;
    return check_params(p);
}

template <typename T>
static void put(std::vector<unsigned char> &img, size_t off, T v) { memcpy(img.data() + off, &v, sizeof(T)); }

static void build_tables(bfm_plan_s *P)
{
    const int d = P->g.ndim;
    const bool f64 = P->prm.dtype == BFM_F64;
    const size_t ce = 2 * P->esz;   // complex element
    size_t off = 0;
    for (int a = 0; a < d; ++a) {
        const int n = P->g.n[a];
        P->tab_tw[a] = off;  off = align256(off + (size_t)n * ce);
        P->tab_qw[a] = off;  off = align256(off + (size_t)n * ce);
        P->tab_lam[a] = off; off = align256(off + (size_t)n * P->esz);
    }
    P->tables.assign(off, 0);
    for (int a = 0; a < d; ++a) {
        const int n = P->g.n[a];
        for (int j = 0; j < n; ++j) {
            const double th = 2.0 * M_PI * (double)j / (double)n;     // exp(-2 pi i j / n)
            const double ph = M_PI * (double)j / (2.0 * (double)n);   // exp(-i pi j / (2n))
            const double s = sin(ph);
            const double lam = 4.0 * s * s * (double)n * (double)n;   // 4 sin^2(pi k/(2n)) n^2
            if (f64) {
                put<double>(P->tables, P->tab_tw[a] + j * ce, cos(th));
                put<double>(P->tables, P->tab_tw[a] + j * ce + 8, -sin(th));
                put<double>(P->tables, P->tab_qw[a] + j * ce, cos(ph));
                put<double>(P->tables, P->tab_qw[a] + j * ce + 8, -sin(ph));
                put<double>(P->tables, P->tab_lam[a] + j * 8, lam);
            } else {
                put<float>(P->tables, P->tab_tw[a] + j * ce, (float)cos(th));
                put<float>(P->tables, P->tab_tw[a] + j * ce + 4, (float)-sin(th));
                put<float>(P->tables, P->tab_qw[a] + j * ce, (float)cos(ph));
                put<float>(P->tables, P->tab_qw[a] + j * ce + 4, (float)-sin(ph));
                put<float>(P->tables, P->tab_lam[a] + j * 4, (float)lam);
            }
        }
    }
}

extern "C" bfm_status bfm_plan_create(const bfm_params *p, bfm_plan *out)
{
    if (out == nullptr) return fail(BFM_EINVAL, "out is NULL");
    *out = nullptr;
    bfm_status s = check_params(p);
    if (s != BFM_OK) return s;
    bfm_plan_s *P = new (std::nothrow) bfm_plan_s();
    if (P == nullptr) return fail(BFM_EINVAL, "out of host memory");
    P->prm = *p;
    P->esz = p->dtype == BFM_F64 ? 8 : 4;
    Grid &g = P->g;
    g.ndim = p->ndim;
    g.N = 1;
    for (int a = 0; a < 3; ++a) g.n[a] = a < p->ndim ? p->shape[a] : 1;
    for (int a = p->ndim - 1; a >= 0; --a) {
        g.stride[a] = g.N;
        g.N *= g.n[a];
    }
    for (int a = p->ndim; a < 3; ++a) g.stride[a] = 0;
    g.vol = 1.0;
    for (int a = 0; a < p->ndim; ++a) g.vol /= g.n[a];
    for (int a = 0; a < 3; ++a) g.pw[a] = a < p->ndim ? p->power[a] : 2.0;
    for (int a = 0; a < p->ndim; ++a) {
        AxisPlan &ap = P->ax[a];
        ap.n = g.n[a];
        ap.inner = (int)g.stride[a];
        if (!factor_radices(ap.n, &ap.radices, &ap.nstages)) {
            delete P;
            return fail(BFM_EINVAL, "axis %d: size %d has no radix-2/3/4 factorisation", a, ap.n);
        }
    }
    long long rb = (g.N + kRedBlock - 1) / kRedBlock;
    P->red_blocks = (int)(rb < kMaxRedBlocks ? rb : kMaxRedBlocks);
    build_tables(P);
    size_t off = 0;
    P->off_state = off;  off = align256(off + sizeof(DevState));
    P->off_trace = off;  off = align256(off + sizeof(TraceRec) * kMaxTrace);
    P->nsplat = (int)splat_blocks(g);
    // slots hold kMaxDepositGrid partials: the deposition's (any tuned grid),
    // the grid-stride reductions (1024), and the sums fused into the last
    // inverse DCT pass and the c-transform's second pass when their grids fit
    P->slot_len = kMaxDepositGrid;
    P->off_part = off;   off = align256(off + sizeof(double) * kNumSlots * (size_t)P->slot_len);
    P->gparts = (int)dct_fused_parts(g.n[0], g.N, P->esz);
    P->off_gpart = off;  off = align256(off + sizeof(double) * (size_t)P->gparts);
    P->off_tables = off; off = align256(off + P->tables.size());
    P->ntiles = splat_tile_count(g);
    P->off_tiles_mu = off; off = align256(off + sizeof(int) * (size_t)(P->ntiles + 1));
    P->off_tiles_nu = off; off = align256(off + sizeof(int) * (size_t)(P->ntiles + 1));
    P->off_batch = off;    off = align256(off + kBatchTableBytes);
    const size_t fb = align256((size_t)g.N * P->esz);
    P->off_pc = off;  off += fb;
    P->off_rho = off; off += fb;
    P->off_f = off;   off += fb;
    P->total = off;
    *out = P;
    return BFM_OK;
}

extern "C" void bfm_plan_destroy(bfm_plan plan) { delete plan; }

extern "C" bfm_status bfm_plan_workspace_bytes(bfm_plan plan, size_t *bytes)
{
    if (plan == nullptr || bytes == nullptr) return fail(BFM_EINVAL, "NULL argument");
    *bytes = plan->total;
    return BFM_OK;
}

// ------------------------------------------------------- device pointers

struct Ws {
    DevState *st;
    TraceRec *trace;
    double *part;
    double *gpart;
    unsigned char *tables;
    void *pc, *rho, *f;
    int *tiles_mu, *tiles_nu;   // filled by solve_begin
    BatchHead *batch;           // multi-pair table (batched solves led by this pair)
    long long slot_len;
    double *slot(int s) const { return part + (size_t)s * slot_len; }
};

static bfm_status check_ws(bfm_plan P, void *ws, size_t ws_bytes, Ws *w)
{
    if (ws == nullptr) return fail(BFM_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(BFM_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < P->total)
        return fail(BFM_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, P->total);
    unsigned char *b = (unsigned char *)ws;
    w->st = (DevState *)(b + P->off_state);
    w->trace = (TraceRec *)(b + P->off_trace);
    w->part = (double *)(b + P->off_part);
    w->gpart = (double *)(b + P->off_gpart);
    w->slot_len = P->slot_len;
    w->tables = b + P->off_tables;
    w->pc = b + P->off_pc;
    w->rho = b + P->off_rho;
    w->f = b + P->off_f;
    w->tiles_mu = (int *)(b + P->off_tiles_mu);
    w->tiles_nu = (int *)(b + P->off_tiles_nu);
    w->batch = (BatchHead *)(b + P->off_batch);
    return BFM_OK;
}

static hipError_t upload_tables(bfm_plan P, const Ws &w, hipStream_t s)
{
    return hipMemcpyAsync(w.tables, P->tables.data(), P->tables.size(), hipMemcpyHostToDevice, s);
}

static CtrlParams ctrl_params(bfm_plan P)
{
    CtrlParams c;
    c.tol = P->prm.tol;
    c.sigma0 = P->prm.sigma0;
    c.sigma_min = P->prm.sigma_min;
    c.beta1 = P->prm.beta1;
    c.beta2 = P->prm.beta2;
    c.alpha1 = P->prm.alpha1;
    c.alpha2 = P->prm.alpha2;
    c.vol = P->g.vol;
    c.inv_N = 1.0 / (double)P->g.N;
    c.slot_len = P->slot_len;
    c.nred = P->red_blocks;
    c.nsplat = P->nsplat;
    c.ngpart = P->gparts;
    c.nqt = c.nqs = P->red_blocks;
    return c;
}

static bfm_status check_inputs(const DevState &hs)
{
    if (hs.bad > 0) return fail(BFM_EINVAL, "mu/nu contain %.0f negative or non-finite values", hs.bad);
    if (fabs(hs.mass_mu - 1.0) > 1e-5 || fabs(hs.mass_nu - 1.0) > 1e-5)
        return fail(BFM_EINVAL, "densities must have unit mass (cell_volume*sum): mu %.9g, nu %.9g", hs.mass_mu,
                    hs.mass_nu);
    if (!(hs.max_mu > 0.0) || !(hs.max_nu > 0.0)) return fail(BFM_EINVAL, "a density is identically zero");
    return BFM_OK;
}

// Poisson solve of f = a - b (b may be null): forward transforms along the
// contiguous (and, in 3D, middle) axes, then one pass along axis 0 that
// transforms forward, divides by lambda (G partials into gpart) and
// transforms back; `b` is cleared as it is consumed when zero_b is set.  The
// remaining inverse passes run in poisson_inverse, the last one writing
// update = update + sigma * g when `update` is non-null.  All passes are
// no-ops once the device stop flag is set.
template <typename T>
static hipError_t poisson_forward(bfm_plan P, const Ws &w, const T *a, T *b, int zero_b, T *F,
                                  const int32_t *done, hipStream_t s)
{
    const Grid &g = P->g;
    const int d = g.ndim;
    hipError_t e;
    e = launch_dct_fwd<T>(a, b, F, P->ax[d - 1], g.N, zero_b, w.tables + P->tab_tw[d - 1],
                          w.tables + P->tab_qw[d - 1], done, s);
    if (e != hipSuccess) return e;
    if (d == 3) {
        e = launch_dct_fwd<T>(F, nullptr, F, P->ax[1], g.N, 0, w.tables + P->tab_tw[1], w.tables + P->tab_qw[1],
                              done, s);
        if (e != hipSuccess) return e;
    }
    const T *l0 = (const T *)(w.tables + P->tab_lam[0]);
    const T *lA = (const T *)(w.tables + P->tab_lam[1]);
    const T *lB = d == 3 ? (const T *)(w.tables + P->tab_lam[2]) : nullptr;
    int np = 0;
    e = launch_dct_fused<T>(F, P->ax[0], g.N, g.n[1], d == 3 ? g.n[2] : 1, w.tables + P->tab_tw[0],
                            w.tables + P->tab_qw[0], l0, lA, lB, w.gpart, &np, done, s);
    if (e == hipSuccess && np != P->gparts) return hipErrorInvalidValue;
    return e;
}

// dotw (with update): the last pass also sums update * dotw into dotpart
// when its grid fits a slot; *ndot = partial count, or 0 when not fused.
template <typename T>
static hipError_t poisson_inverse(bfm_plan P, const Ws &w, T *F, T *out, T *update, const int32_t *done,
                                  hipStream_t s, const T *dotw = nullptr, double *dotpart = nullptr,
                                  int *ndot = nullptr)
{
    const Grid &g = P->g;
    const int d = g.ndim;
    hipError_t e;
    if (ndot != nullptr) *ndot = 0;
    if (d == 3) {
        e = launch_dct_inv<T>(F, F, nullptr, nullptr, P->ax[1], g.N, w.tables + P->tab_tw[1], w.tables + P->tab_qw[1],
                              done, s);
        if (e != hipSuccess) return e;
    }
    T *dst = update != nullptr ? update : out;
    const long long nblk = (g.N / g.n[d - 1] + 1) / 2;   // workgroups of the contiguous inverse pass
    const bool fuse = dotw != nullptr && update != nullptr && ndot != nullptr && nblk <= P->slot_len;
    e = launch_dct_inv<T>(F, dst, update, update != nullptr ? &w.st->sigma : nullptr, P->ax[d - 1], g.N,
                          w.tables + P->tab_tw[d - 1], w.tables + P->tab_qw[d - 1], done, s,
                          fuse ? dotw : nullptr, fuse ? dotpart : nullptr);
    if (e == hipSuccess && fuse) *ndot = (int)nblk;
    return e;
}

// One half-step of Algorithm 1 on J(p) = <p, tgt> + <p^c, src>:
//   head:  pc = p^c, J(p), map + pushforward rho = T#src, primal cost,
//          H^1 gradient g of tgt - rho and G; controller `head_mode`;
//   step:  p <- p + sigma g, q = p^c, J(p), controller `step_mode`.
// head_ct = false takes pc as already holding p^c (gradient ascent, where
// the previous step left it there).
template <typename T>
static hipError_t half_step(bfm_plan P, const Ws &w, T *p, const T *src, const int *src_tiles, const T *tgt, T *q,
                            int head_mode, int step_mode, bool head_only, bool head_dot, hipStream_t s,
                            bool head_ct = true)
{
    const Grid &g = P->g;
    const int32_t *done = &w.st->done;
    const int nb = P->red_blocks;
    T *pc = (T *)w.pc, *rho = (T *)w.rho, *F = (T *)w.f;
    const CtrlParams cp = ctrl_params(P);
    hipError_t e;
    if (head_ct && (e = ctransform_field<T>(g, p, pc, done, s, P->ct_cfg, F)) != hipSuccess)
        return e;   // F is free here
    if (head_dot &&
        (e = launch_dot2<T>(p, tgt, nullptr, nullptr, g.N, w.slot(S_P_TGT), nullptr, nb, done, s)) != hipSuccess)
        return e;
    if ((e = launch_splat<T>(g, pc, src, rho, nullptr, w.slot(S_PRIMAL), w.slot(S_PC_SRC), P->nsplat, done, s, T(1),
                             src_tiles)) !=
        hipSuccess)
        return e;
    if ((e = poisson_forward<T>(P, w, tgt, rho, 1, F, done, s)) != hipSuccess) return e;
    if ((e = launch_ctrl(w.st, w.part, w.gpart, head_mode | (head_dot ? 0 : CTRL_REUSE_DOT), cp, w.trace, s)) !=
        hipSuccess)
        return e;
    if (head_only) return hipSuccess;
    // the two sums of J at the stepped potential, <p, tgt> and <q, src>,
    // fused into the passes that write p and q where possible
    int nqt = 0, nqs = 0;
    const bool al = ((((uintptr_t)tgt) | ((uintptr_t)src)) & 15) == 0;   // the fused passes read 16-byte vectors
    if ((e = poisson_inverse<T>(P, w, F, nullptr, p, done, s, al ? tgt : nullptr, w.slot(S_Q_TGT), &nqt)) !=
        hipSuccess)
        return e;
    if ((e = ctransform_field<T>(g, p, q, done, s, P->ct_cfg, F, al ? src : nullptr, w.slot(S_Q_SRC), &nqs)) !=
        hipSuccess)
        return e;   // F consumed above
    if (nqs > w.slot_len) return hipErrorInvalidValue;
    if (nqt == 0 && nqs == 0)
        e = launch_dot2<T>(p, tgt, q, src, g.N, w.slot(S_Q_TGT), w.slot(S_Q_SRC), nb, done, s);
    else if (nqt == 0)
        e = launch_dot2<T>(p, tgt, nullptr, nullptr, g.N, w.slot(S_Q_TGT), nullptr, nb, done, s);
    else if (nqs == 0)
        e = launch_dot2<T>(q, src, nullptr, nullptr, g.N, w.slot(S_Q_SRC), nullptr, nb, done, s);
    if (e != hipSuccess) return e;
    CtrlParams cs = cp;
    cs.nqt = nqt > 0 ? nqt : nb;
    cs.nqs = nqs > 0 ? nqs : nb;
    return launch_ctrl(w.st, w.part, w.gpart, step_mode, cs, w.trace, s);
}

// Solve in four parts so that the iterations can be enqueued without any host
// synchronisation (and captured in a graph):
//   begin:   tables, input statistics, sigma0, validation (synchronises),
//            rho = 0, phi = phi_init or 0;
//   iterate: full iterations it0 .. it0+count-1 (the head of iteration 0
//            computes <phi, nu>, later heads reuse the previous step's sum);
//   final:   the head of iteration `it` only (no-op once the stop flag is set);
//   finish:  T from the last head's phi^c, phi - mean, psi = phi^c + mean,
//            the result block (synchronises).
template <typename T>
static bfm_status solve_begin(bfm_plan P, const T *mu, const T *nu, const T *phi_init, T *phi, const Ws &w,
                              hipStream_t s, bool sync_check)
{
    const Grid &g = P->g;
    HIP_TRY(upload_tables(P, w, s));
    HIP_TRY(launch_stats<T>(mu, nu, g.N, w.part, P->slot_len, P->red_blocks, s));
    HIP_TRY(launch_ctrl(w.st, w.part, w.gpart, CTRL_INIT, ctrl_params(P), w.trace, s));
    HIP_TRY(launch_fill<T>((T *)w.rho, g.N, T(0), s));
    // the deposition walks only the tiles of mu (phi-steps) and nu (psi-steps)
    // that hold mass; F is free scratch here
    HIP_TRY(launch_tile_list<T>(g, mu, (int *)w.f, w.tiles_mu, s));
    HIP_TRY(launch_tile_list<T>(g, nu, (int *)w.f, w.tiles_nu, s));
    if (phi_init != nullptr)
        HIP_TRY(hipMemcpyAsync(phi, phi_init, (size_t)g.N * sizeof(T), hipMemcpyDeviceToDevice, s));
    else
        HIP_TRY(launch_fill<T>(phi, g.N, T(0), s));
    if (!sync_check) return BFM_OK;
    DevState hs;
    HIP_TRY(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return check_inputs(hs);
}

// One iteration of the plain H^1 gradient ascent of Section 4.3 (the scheme
// Tables 5 and 6 compare with): the phi half-step of Algorithm 1 with its
// c-transform written to pc (q = phi_{n+1/2}^c, the stepped J and the sigma
// update), then phi_{n+1} = q^c = phi_{n+1/2}^cc.  Since f^ccc = f^c, q is
// phi_{n+1}^c and serves the next head, which therefore computes no
// c-transform: 2 c-transforms and 1 Poisson solve per iteration.  The sum
// <phi_{n+1}, nu> of the next head is fused into the pass writing phi_{n+1}.
template <typename T>
static hipError_t ga_iteration(bfm_plan P, const Ws &w, const T *mu, const T *nu, T *phi, bool first, hipStream_t s)
{
    const Grid &g = P->g;
    const int32_t *done = &w.st->done;
    T *pc = (T *)w.pc, *F = (T *)w.f;
    hipError_t e;
    if ((e = half_step<T>(P, w, phi, mu, w.tiles_mu, nu, pc, CTRL_HEAD_PHI, CTRL_STEP_PHI, false, first, s,
                          first)) !=
        hipSuccess)
        return e;
    int nd = 0;
    const bool al = (((uintptr_t)nu) & 15) == 0;
    if ((e = ctransform_field<T>(g, pc, phi, done, s, P->ct_cfg, F, al ? nu : nullptr, w.slot(S_Q_TGT), &nd)) !=
        hipSuccess)
        return e;   // F is free after the step
    if (nd > w.slot_len) return hipErrorInvalidValue;
    if (nd == 0 &&
        (e = launch_dot2<T>(phi, nu, nullptr, nullptr, g.N, w.slot(S_Q_TGT), nullptr, P->red_blocks, done, s)) !=
            hipSuccess)
        return e;
    CtrlParams cs = ctrl_params(P);
    cs.nqt = nd > 0 ? nd : P->red_blocks;
    return launch_ctrl(w.st, w.part, w.gpart, CTRL_GA_NEXT, cs, w.trace, s);
}

template <typename T>
static hipError_t enqueue_iterations(bfm_plan P, const Ws &w, const T *mu, const T *nu, T *phi, T *psi, int it0,
                                     int count, hipStream_t s)
{
    hipError_t e;
    if (P->prm.method == BFM_METHOD_GA) {
        for (int it = it0; it < it0 + count; ++it)
            if ((e = ga_iteration<T>(P, w, mu, nu, phi, it == 0, s)) != hipSuccess) return e;
        return hipSuccess;
    }
    for (int it = it0; it < it0 + count; ++it) {
        if ((e = half_step<T>(P, w, phi, mu, w.tiles_mu, nu, psi, CTRL_HEAD_PHI, CTRL_STEP_PHI, false, it == 0,
                              s)) != hipSuccess)
            return e;
        if ((e = half_step<T>(P, w, psi, nu, w.tiles_nu, mu, phi, CTRL_HEAD_PSI, CTRL_STEP_PSI, false, false, s)) !=
            hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <typename T>
static hipError_t enqueue_final_head(bfm_plan P, const Ws &w, const T *mu, const T *nu, T *phi, T *psi, int it,
                                     hipStream_t s)
{
    // gradient ascent keeps phi^c in pc from the last step
    return half_step<T>(P, w, phi, mu, w.tiles_mu, nu, psi, CTRL_HEAD_PHI, CTRL_STEP_PHI, true, it == 0, s,
                        P->prm.method != BFM_METHOD_GA || it == 0);
}

template <typename T>
static hipError_t enqueue_finish(bfm_plan P, const Ws &w, const T *mu, T *phi, T *psi, T *Tmap, hipStream_t s)
{
    const Grid &g = P->g;
    const int nb = P->red_blocks;
    T *pc = (T *)w.pc;
    hipError_t e;
    if (Tmap != nullptr &&
        (e = launch_splat<T>(g, pc, mu, nullptr, Tmap, nullptr, nullptr, P->nsplat, nullptr, s)) != hipSuccess)
        return e;
    if ((e = launch_dot2<T>(phi, nullptr, nullptr, nullptr, g.N, w.slot(S_MEAN_A), nullptr, nb, nullptr, s)) !=
        hipSuccess)
        return e;
    if ((e = launch_dot2<T>(pc, nullptr, nullptr, nullptr, g.N, w.slot(S_MEAN_B), nullptr, nb, nullptr, s)) !=
        hipSuccess)
        return e;
    if ((e = launch_ctrl(w.st, w.part, w.gpart, CTRL_MEANS, ctrl_params(P), w.trace, s)) != hipSuccess) return e;
    return launch_shift_scale<T>(phi, phi, &w.st->mean_a, -1.0, psi, pc, &w.st->mean_a, 1.0, g.N, 1.0, s);
}

static bfm_status fill_result(const DevState &hs, bfm_result *res)
{
    if (res != nullptr) {
        memset(res, 0, sizeof(*res));
        res->iters = hs.iter;
        res->converged = (hs.done && !hs.nonfinite) ? 1 : 0;
        res->status = hs.nonfinite ? BFM_ENUMERIC : BFM_OK;
        res->sigma_floor_hits = hs.sigma_floor_hits;
        res->dual = hs.dual_head;
        res->primal = hs.primal_head;
        res->gap = hs.gap;
        res->G = hs.G_head;
        res->sigma = hs.sigma;
        res->mass_mu = hs.mass_mu;
        res->mass_nu = hs.mass_nu;
    }
    if (hs.nonfinite) return fail(BFM_ENUMERIC, "non-finite value in the dual, primal or gradient norm");
    return BFM_OK;
}

template <typename T>
static bfm_status solve_impl(bfm_plan P, const T *mu, const T *nu, const T *phi_init, T *phi, T *psi, T *Tmap,
                             const Ws &w, hipStream_t s, bfm_result *res)
{
    bfm_status st = solve_begin<T>(P, mu, nu, phi_init, phi, w, s, true);
    if (st != BFM_OK) return st;
    DevState hs;
    const int K = P->prm.check_every;
    int it = 0;
    while (it < P->prm.max_iters) {
        const int cnt = P->prm.max_iters - it < K ? P->prm.max_iters - it : K;
        HIP_TRY(enqueue_iterations<T>(P, w, mu, nu, phi, psi, it, cnt, s));
        it += cnt;
        HIP_TRY(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hs.done) break;
    }
    HIP_TRY(enqueue_final_head<T>(P, w, mu, nu, phi, psi, it, s));
    HIP_TRY(enqueue_finish<T>(P, w, mu, phi, psi, Tmap, s));
    HIP_TRY(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return fill_result(hs, res);
}

extern "C" bfm_status bfm_solve(bfm_plan plan, const void *mu, const void *nu, const void *phi_init, void *phi,
                                void *psi, void *T, void *workspace, size_t ws_bytes, void *stream,
                                bfm_result *result)
{
    if (plan == nullptr) return fail(BFM_EINVAL, "plan is NULL");
    if (mu == nullptr || nu == nullptr || phi == nullptr || psi == nullptr)
        return fail(BFM_EINVAL, "mu, nu, phi and psi must be non-NULL");
    if (phi == psi || phi == mu || phi == nu || psi == mu || psi == nu)
        return fail(BFM_EINVAL, "phi and psi must be distinct buffers, distinct from mu and nu");
    Ws w;
    bfm_status st = check_ws(plan, workspace, ws_bytes, &w);
    if (st != BFM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (plan->prm.dtype == BFM_F64)
        return solve_impl<double>(plan, (const double *)mu, (const double *)nu, (const double *)phi_init,
                                  (double *)phi, (double *)psi, (double *)T, w, s, result);
    return solve_impl<float>(plan, (const float *)mu, (const float *)nu, (const float *)phi_init, (float *)phi,
                             (float *)psi, (float *)T, w, s, result);
}

// ------------------------------------------------- allocation-free solve

// bfm_solve_noalloc keeps the workspace of a solve in this file-scope device
// array (one copy on every GPU the library runs on, held until the process
// ends) for callers that cannot allocate device memory.  In host code
// `scratch` names a host-side stand-in, not device memory: its device
// address is looked up once per device with hipGetSymbolAddress and only that
// address is handed to kernels and copies.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the calling thread's current device.
static bfm_status scratch_address(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(BFM_EDEVICE, "device id %d is outside 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[dev] == nullptr) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (p == nullptr || ((uintptr_t)p & 255) != 0)
            return fail(BFM_EDEVICE, "static scratch of device %d has no usable address", dev);
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return BFM_OK;
}

extern "C" bfm_status bfm_solve_noalloc(bfm_plan plan, const void *mu, const void *nu, const void *phi_init,
                                        void *phi, void *psi, void *T, void *stream, bfm_result *result)
{
    if (plan == nullptr) return fail(BFM_EINVAL, "plan is NULL");
    if (plan->total > kNoAllocScratchBytes)
        return fail(BFM_EWORKSPACE,
                    "bfm_solve_noalloc: this plan needs %zu bytes of scratch, more than the %zu bytes of the "
                    "static array; use bfm_solve with a caller workspace",
                    plan->total, kNoAllocScratchBytes);
    void *ws = nullptr;
    bfm_status st = scratch_address(&ws);
    if (st != BFM_OK) return st;
    return bfm_solve(plan, mu, nu, phi_init, phi, psi, T, ws, kNoAllocScratchBytes, stream, result);
}

// ------------------------------------------------------------- batched

// Many independent problems (each with its own plan, workspace and device
// step-size state) advanced together: the first iteration is enqueued
// directly, then `K` iterations of every problem are captured once into a
// graph whose branches run on up to eight streams and the graph is replayed;
// a problem whose stop flag is set turns into no-ops.  Stop flags are read
// between replays.
namespace {
struct BatchStreams {
    int nw = 0;
    hipStream_t w[8] = {};
    hipStream_t cap = nullptr;   // capture origin (the caller's stream may be the legacy null stream)
    hipEvent_t fork = nullptr, join[8] = {}, capev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchStreams() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (int i = 0; i < nw; ++i) {
            if (w[i]) (void)hipStreamDestroy(w[i]);
            if (join[i]) (void)hipEventDestroy(join[i]);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (capev) (void)hipEventDestroy(capev);
        if (cap) (void)hipStreamDestroy(cap);
    }
    hipError_t init(int n) {
        nw = n;
        hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&capev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        for (int i = 0; i < nw && e == hipSuccess; ++i) {
            e = hipStreamCreateWithFlags(&w[i], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
        }
        return e;
    }
    hipError_t begin(hipStream_t s) {
        hipError_t e = hipEventRecord(fork, s);
        for (int i = 0; i < nw && e == hipSuccess; ++i) e = hipStreamWaitEvent(w[i], fork, 0);
        return e;
    }
    hipError_t end(hipStream_t s) {
        hipError_t e = hipSuccess;
        for (int i = 0; i < nw && e == hipSuccess; ++i) {
            e = hipEventRecord(join[i], w[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, join[i], 0);
        }
        return e;
    }
};
}  // namespace

template <typename T>
static bfm_status batched_impl(int np, const bfm_plan *P, const void *const *mu_, const void *const *nu_,
                               void *const *phi_, void *const *psi_, void *const *T_, const std::vector<Ws> &w,
                               int K, hipStream_t s, bfm_result *res)
{
    auto MU = [&](int p) { return (const T *)mu_[p]; };
    auto NU = [&](int p) { return (const T *)nu_[p]; };
    auto PHI = [&](int p) { return (T *)phi_[p]; };
    auto PSI = [&](int p) { return (T *)psi_[p]; };
    std::vector<DevState> hs(np);
    for (int p = 0; p < np; ++p) {
        bfm_status st = solve_begin<T>(P[p], MU(p), NU(p), nullptr, PHI(p), w[p], s, false);
        if (st != BFM_OK) return st;
    }
    for (int p = 0; p < np; ++p)
        HIP_TRY(hipMemcpyAsync(&hs[p], w[p].st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int p = 0; p < np; ++p) {
        bfm_status st = check_inputs(hs[p]);
        if (st != BFM_OK) return fail(st, "pair %d: %s", p, g_last_error.c_str());
    }
    BatchStreams bs;
    HIP_TRY(bs.init(np < 8 ? np : 8));
    auto worker = [&](int p) { return bs.w[p % bs.nw]; };
    const int maxit = P[0]->prm.max_iters;
    int it = 0;
    if (maxit > 0) {
        HIP_TRY(bs.begin(s));
        for (int p = 0; p < np; ++p)
            HIP_TRY(enqueue_iterations<T>(P[p], w[p], MU(p), NU(p), PHI(p), PSI(p), 0, 1, worker(p)));
        HIP_TRY(bs.end(s));
        it = 1;
    }
    bool all_done = false;
    if (maxit - it >= K) {
        // capture on a private stream; the graph is then launched on `s`
        HIP_TRY(hipStreamBeginCapture(bs.cap, hipStreamCaptureModeThreadLocal));
        hipError_t ce = bs.begin(bs.cap);
        for (int p = 0; p < np && ce == hipSuccess; ++p)
            ce = enqueue_iterations<T>(P[p], w[p], MU(p), NU(p), PHI(p), PSI(p), it, K, worker(p));
        if (ce == hipSuccess) ce = bs.end(bs.cap);
        hipError_t ee = hipStreamEndCapture(bs.cap, &bs.graph);
        HIP_TRY(ce);
        HIP_TRY(ee);
        HIP_TRY(hipGraphInstantiate(&bs.exec, bs.graph, nullptr, nullptr, 0));
        while (maxit - it >= K) {
            HIP_TRY(hipGraphLaunch(bs.exec, s));
            it += K;
            for (int p = 0; p < np; ++p)
                HIP_TRY(hipMemcpyAsync(&hs[p], w[p].st, sizeof(DevState), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            all_done = true;
            for (int p = 0; p < np; ++p) all_done = all_done && hs[p].done;
            if (all_done) break;
        }
    }
    HIP_TRY(bs.begin(s));
    for (int p = 0; p < np; ++p) {
        if (!all_done && it < maxit)
            HIP_TRY(enqueue_iterations<T>(P[p], w[p], MU(p), NU(p), PHI(p), PSI(p), it, maxit - it, worker(p)));
        HIP_TRY(enqueue_final_head<T>(P[p], w[p], MU(p), NU(p), PHI(p), PSI(p), all_done ? it : maxit, worker(p)));
        HIP_TRY(enqueue_finish<T>(P[p], w[p], MU(p), PHI(p), PSI(p), T_ != nullptr ? (T *)T_[p] : nullptr,
                                  worker(p)));
    }
    HIP_TRY(bs.end(s));
    for (int p = 0; p < np; ++p)
        HIP_TRY(hipMemcpyAsync(&hs[p], w[p].st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bfm_status out = BFM_OK;
    for (int p = 0; p < np; ++p) {
        bfm_status st = fill_result(hs[p], res != nullptr ? &res[p] : nullptr);
        if (st != BFM_OK && out == BFM_OK) out = st;
    }
    return out;
}

// ------------------------------------------------- batched, one launch per pass
// 2D quadratic-cost batches: after the first iteration (enqueued per pair),
// every pass of a half-step runs as ONE launch over all pairs of a chunk of
// at most kBatchChunk pairs (c-transform rows and columns, deposition, the
// three Poisson passes, the controller), reading a device table of per-pair
// pointers and sizes; K iterations of these launches are captured once into
// a graph and replayed.  Each pair keeps its own step size, gap and stop
// flag; a stopped pair's workgroups return at once.
static bool multi_applies(int np, const bfm_plan *P)
{
    for (int p = 0; p < np; ++p) {
        const Grid &g = P[p]->g;
        if (g.ndim != 2 || !grid_quadratic(g) || P[p]->prm.method != BFM_METHOD_BFM) return false;
        if ((g.n[1] & 3) != 0) return false;
    }
    return true;
}

namespace {
struct MultiChunk {
    BatchHead *tab = nullptr;     // device table in the workspace of the chunk's first pair
    std::vector<int> pair;        // batch index of each entry
    std::vector<int> n0, n1;
    std::vector<int> n0map;       // n0 of the pairs with a map output, 0 for the others
    int splat_grid = 0;           // workgroups of the joint deposition
    long long epb = 0;            // elements per workgroup of the finishing passes
    std::vector<unsigned char> img;   // host image of the table
};
}  // namespace

// The head of a half-step for every pair of a chunk: p^c, the map and
// deposition, the forward Poisson passes, the controller (J, P, G, gap, stop
// test).  <p, tgt> is the previous step's <q, src> (CTRL_REUSE_DOT); at the
// first head phi_0 = 0 and the state holds 0 for it.
template <typename T>
static hipError_t multi_head(const MultiChunk &c, int role, hipStream_t s)
{
    const int np = (int)c.pair.size();
    const int head = role ? CTRL_HEAD_PSI : CTRL_HEAD_PHI;
    hipError_t e;
    if ((e = launch_ct_multi<T>(c.tab, c.n0.data(), c.n1.data(), np, role, 0, s)) != hipSuccess) return e;
    if ((e = launch_ct_multi<T>(c.tab, c.n0.data(), c.n1.data(), np, role, 1, s)) != hipSuccess) return e;
    if ((e = launch_splat_multi<T>(c.tab, np, role, c.splat_grid, s)) != hipSuccess) return e;
    if ((e = launch_dct_multi<T>(c.tab, c.n0.data(), c.n1.data(), np, role, kDctFwd, s)) != hipSuccess) return e;
    if ((e = launch_dct_multi<T>(c.tab, c.n0.data(), c.n1.data(), np, role, kDctFused, s)) != hipSuccess) return e;
    return launch_ctrl_multi(c.tab, np, role, head | CTRL_REUSE_DOT, s);
}

template <typename T>
static hipError_t multi_half_step(const MultiChunk &c, int role, hipStream_t s)
{
    const int np = (int)c.pair.size();
    const int step = role ? CTRL_STEP_PSI : CTRL_STEP_PHI;
    hipError_t e;
    if ((e = multi_head<T>(c, role, s)) != hipSuccess) return e;
    if ((e = launch_dct_multi<T>(c.tab, c.n0.data(), c.n1.data(), np, role, kDctInv, s)) != hipSuccess) return e;
    if ((e = launch_ct_multi<T>(c.tab, c.n0.data(), c.n1.data(), np, role, 2, s)) != hipSuccess) return e;
    if ((e = launch_ct_multi<T>(c.tab, c.n0.data(), c.n1.data(), np, role, 3, s)) != hipSuccess) return e;
    return launch_ctrl_multi(c.tab, np, role, step, s);
}

template <typename T>
static hipError_t multi_iterations(const std::vector<MultiChunk> &chunks, int count, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (int it = 0; it < count && e == hipSuccess; ++it)
        for (int role = 0; role < 2 && e == hipSuccess; ++role)
            for (const MultiChunk &c : chunks)
                if ((e = multi_half_step<T>(c, role, s)) != hipSuccess) break;
    for (const MultiChunk &c : chunks)
        if (e == hipSuccess) e = launch_batch_done(c.tab, s);
    return e;
}

template <typename T>
static bfm_status batched_multi_impl(int np, const bfm_plan *P, const void *const *mu_, const void *const *nu_,
                                     void *const *phi_, void *const *psi_, void *const *T_, const std::vector<Ws> &w,
                                     int K, hipStream_t s, bfm_result *res)
{
    auto MU = [&](int p) { return (const T *)mu_[p]; };
    auto NU = [&](int p) { return (const T *)nu_[p]; };
    auto PHI = [&](int p) { return (T *)phi_[p]; };
    std::vector<DevState> hs(np);
    for (int p = 0; p < np; ++p) {
        bfm_status st = solve_begin<T>(P[p], MU(p), NU(p), nullptr, PHI(p), w[p], s, false);
        if (st != BFM_OK) return st;
    }
    for (int p = 0; p < np; ++p)
        HIP_TRY(hipMemcpyAsync(&hs[p], w[p].st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int p = 0; p < np; ++p) {
        bfm_status st = check_inputs(hs[p]);
        if (st != BFM_OK) return fail(st, "pair %d: %s", p, g_last_error.c_str());
    }
    // device tables, one per chunk of at most kBatchChunk pairs of `ids`
    auto make_chunks = [&](const std::vector<int> &ids, std::vector<MultiChunk> &out) -> bfm_status {
        out.clear();
        for (size_t first = 0; first < ids.size(); first += kBatchChunk) {
            MultiChunk c;
            const int cnp = (int)(ids.size() - first < (size_t)kBatchChunk ? ids.size() - first : kBatchChunk);
            c.tab = w[ids[first]].batch;
            c.img.assign(sizeof(BatchHead) + (size_t)cnp * sizeof(PairDev), 0);
            long long tiles = 0;
            for (int k = 0; k < cnp; ++k) {
                const int p = ids[first + k];
                const bfm_plan_s *Q = P[p];
                const Ws &W = w[p];
                PairDev d{};
                d.mu = mu_[p];
                d.nu = nu_[p];
                d.phi = phi_[p];
                d.psi = psi_[p];
                d.pc = W.pc;
                d.rho = W.rho;
                d.F = W.f;
                d.st = W.st;
                d.trace = W.trace;
                d.part = W.part;
                d.gpart = W.gpart;
                d.tables = W.tables;
                d.tiles_mu = W.tiles_mu;
                d.tiles_nu = W.tiles_nu;
                d.slot_len = W.slot_len;
                d.n0 = Q->g.n[0];
                d.n1 = Q->g.n[1];
                for (int a = 0; a < 2; ++a) {
                    d.tw[a] = (int)Q->tab_tw[a];
                    d.qw[a] = (int)Q->tab_qw[a];
                    d.lam[a] = (int)Q->tab_lam[a];
                    d.radices[a] = Q->ax[a].radices;
                }
                d.Tmap = T_ != nullptr ? T_[p] : nullptr;
                d.cp = ctrl_params(const_cast<bfm_plan>(Q));
                d.cp.nqt = (int)dct_multi_inv_parts(d.n0);
                d.cp.nqs = ct_multi_col_groups(d.n0, d.n1);
                if (d.cp.nqt > W.slot_len || d.cp.nqs > W.slot_len || (d.n1 + 3) / 4 != Q->gparts)
                    return fail(BFM_EDEVICE, "pair %d: multi-pair partial counts exceed the workspace slots", p);
                memcpy(c.img.data() + sizeof(BatchHead) + (size_t)k * sizeof(PairDev), &d, sizeof(d));
                c.pair.push_back(p);
                c.n0.push_back(d.n0);
                c.n1.push_back(d.n1);
                c.n0map.push_back(d.Tmap != nullptr ? d.n0 : 0);
                tiles += splat_tile_count(Q->g);
            }
            c.splat_grid = (int)(tiles < kBatchSplatGrid ? tiles : kBatchSplatGrid);
            BatchHead hd{};
            hd.np = cnp;
            hd.splat_grid = c.splat_grid;
            memcpy(c.img.data(), &hd, sizeof(hd));
            out.push_back(std::move(c));
        }
        return BFM_OK;
    };
    auto upload = [&](const std::vector<MultiChunk> &cs) -> bfm_status {
        for (const MultiChunk &c : cs) {
            HIP_TRY(hipMemcpyAsync(c.tab, c.img.data(), c.img.size(), hipMemcpyHostToDevice, s));
            HIP_TRY(launch_batch_entries(c.tab, s));
        }
        return BFM_OK;
    };
    auto heads = [&](const std::vector<MultiChunk> &cs, std::vector<BatchHead> &h) -> bfm_status {
        h.resize(cs.size());
        for (size_t i = 0; i < cs.size(); ++i)
            HIP_TRY(hipMemcpyAsync(&h[i], cs[i].tab, sizeof(BatchHead), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return BFM_OK;
    };
    std::vector<int> ids(np);
    for (int p = 0; p < np; ++p) ids[p] = p;
    std::vector<MultiChunk> full;
    bfm_status bst = make_chunks(ids, full);
    if (bst != BFM_OK) return bst;
    for (MultiChunk &c : full) {   // finishing passes: no pair above its slot count of workgroups
        long long epb = 4 * kRedBlock;
        for (size_t k = 0; k < c.pair.size(); ++k) {
            const long long N = (long long)c.n0[k] * c.n1[k];
            while ((N + epb - 1) / epb > w[c.pair[k]].slot_len) epb += 4 * kRedBlock;
        }
        c.epb = epb;
    }
    if ((bst = upload(full)) != BFM_OK) return bst;
    // The iterations run on the chunks of the pairs still iterating: when at
    // most half of the pairs of the current chunks are still running after a
    // replay, the tables are rebuilt over those pairs alone and the graph is
    // captured again, so stopped pairs stop costing workgroups and the
    // deposition grid shrinks with the remaining tiles.
    std::vector<MultiChunk> cur = full;
    bool compacted = false;
    const int maxit = P[0]->prm.max_iters;
    int it = 0;
    bool done = false;
    if (maxit - it >= K) {
        hipStream_t cap = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        auto drop_graph = [&]() {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            exec = nullptr;
            graph = nullptr;
        };
        hipError_t ce = hipSuccess;
        std::vector<BatchHead> h;
        while (ce == hipSuccess && bst == BFM_OK && maxit - it >= K) {
            if (exec == nullptr) {
                ce = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
                if (ce == hipSuccess) {
                    ce = multi_iterations<T>(cur, K, cap);
                    hipError_t ee = hipStreamEndCapture(cap, &graph);
                    if (ce == hipSuccess) ce = ee;
                }
                if (ce == hipSuccess) ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                if (ce != hipSuccess) break;
            }
            ce = hipGraphLaunch(exec, s);
            if (ce != hipSuccess) break;
            it += K;
            if ((bst = heads(cur, h)) != BFM_OK) break;
            int running = 0, size = 0;
            for (size_t i = 0; i < cur.size(); ++i) {
                running += h[i].nactive;
                size += (int)cur[i].pair.size();
            }
            if (running == 0) {
                done = true;
                break;
            }
            if (2 * running <= size && maxit - it >= K) {
                std::vector<int> live;
                for (size_t i = 0; i < cur.size(); ++i)
                    for (size_t k = 0; k < cur[i].pair.size(); ++k)
                        if (!((h[i].done_mask >> k) & 1ull)) live.push_back(cur[i].pair[k]);
                std::vector<MultiChunk> next;
                if ((bst = make_chunks(live, next)) != BFM_OK) break;
                if ((bst = upload(next)) != BFM_OK) break;
                cur.swap(next);
                compacted = true;
                drop_graph();
            }
        }
        drop_graph();
        (void)hipStreamDestroy(cap);
        HIP_TRY(ce);
        if (bst != BFM_OK) return bst;
    }
    if (!done && it < maxit) {
        HIP_TRY(multi_iterations<T>(cur, maxit - it, s));
        it = maxit;
    }
    // the last head (no-op for stopped pairs), then the outputs, on the full tables
    // (their stop masks gathered again from the pairs' flags)
    if (compacted) {
        if ((bst = upload(full)) != BFM_OK) return bst;
        for (const MultiChunk &c : full) HIP_TRY(launch_batch_done(c.tab, s));
    }
    for (const MultiChunk &c : full) {
        const int cnp = (int)c.pair.size();
        HIP_TRY(multi_head<T>(c, 0, s));
        HIP_TRY(launch_map_multi<T>(c.tab, c.n0map.data(), c.n1.data(), cnp, s));
        HIP_TRY(launch_finish_multi<T>(c.tab, c.n0.data(), c.n1.data(), cnp, c.epb, s));
    }
    for (int p = 0; p < np; ++p)
        HIP_TRY(hipMemcpyAsync(&hs[p], w[p].st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bfm_status out = BFM_OK;
    for (int p = 0; p < np; ++p) {
        bfm_status st = fill_result(hs[p], res != nullptr ? &res[p] : nullptr);
        if (st != BFM_OK && out == BFM_OK) out = st;
    }
    return out;
}

extern "C" bfm_status bfm_solve_batched(int32_t npairs, const bfm_plan *plans, const void *const *mu,
                                        const void *const *nu, void *const *phi, void *const *psi, void *const *T,
                                        void *const *workspaces, const size_t *ws_bytes, int32_t iters_per_graph,
                                        void *stream, bfm_result *results)
{
    if (npairs < 1) return fail(BFM_EINVAL, "npairs must be >= 1");
    if (plans == nullptr || mu == nullptr || nu == nullptr || phi == nullptr || psi == nullptr ||
        workspaces == nullptr || ws_bytes == nullptr)
        return fail(BFM_EINVAL, "NULL argument");
    if (iters_per_graph < 1) return fail(BFM_EINVAL, "iters_per_graph must be >= 1");
    std::vector<Ws> w(npairs);
    for (int p = 0; p < npairs; ++p) {
        if (plans[p] == nullptr) return fail(BFM_EINVAL, "plan %d is NULL", p);
        if (plans[p]->prm.dtype != plans[0]->prm.dtype) return fail(BFM_EINVAL, "pair %d: dtype differs", p);
        if (plans[p]->prm.max_iters != plans[0]->prm.max_iters)
            return fail(BFM_EINVAL, "pair %d: max_iters differs (all pairs iterate together)", p);
        if (mu[p] == nullptr || nu[p] == nullptr || phi[p] == nullptr || psi[p] == nullptr)
            return fail(BFM_EINVAL, "pair %d: NULL field", p);
        if (phi[p] == psi[p]) return fail(BFM_EINVAL, "pair %d: phi and psi must be distinct", p);
        bfm_status st = check_ws(plans[p], workspaces[p], ws_bytes[p], &w[p]);
        if (st != BFM_OK) return fail(st, "pair %d: %s", p, g_last_error.c_str());
        for (int q = 0; q < p; ++q)
            if (workspaces[q] == workspaces[p]) return fail(BFM_EINVAL, "pairs %d and %d share a workspace", q, p);
    }
    hipStream_t s = (hipStream_t)stream;
    const bool multi = multi_applies(npairs, plans);
    if (plans[0]->prm.dtype == BFM_F64)
        return multi ? batched_multi_impl<double>(npairs, plans, mu, nu, phi, psi, T, w, iters_per_graph, s, results)
                     : batched_impl<double>(npairs, plans, mu, nu, phi, psi, T, w, iters_per_graph, s, results);
    return multi ? batched_multi_impl<float>(npairs, plans, mu, nu, phi, psi, T, w, iters_per_graph, s, results)
                 : batched_impl<float>(npairs, plans, mu, nu, phi, psi, T, w, iters_per_graph, s, results);
}

// ------------------------------------------------------- batched gradient

extern "C" bfm_status bfm_grad_batched(int32_t npairs, const bfm_plan *plans, const void *const *phi,
                                       const void *const *psi, const double *scale, void *const *grad_mu,
                                       void *const *grad_nu, void *const *workspaces, const size_t *ws_bytes,
                                       void *stream)
{
    if (npairs < 1) return fail(BFM_EINVAL, "npairs must be >= 1");
    if (plans == nullptr || phi == nullptr || psi == nullptr || scale == nullptr || workspaces == nullptr ||
        ws_bytes == nullptr)
        return fail(BFM_EINVAL, "NULL argument");
    std::vector<Ws> w(npairs);
    std::vector<GradPair> g(npairs);
    for (int p = 0; p < npairs; ++p) {
        if (plans[p] == nullptr) return fail(BFM_EINVAL, "plan %d is NULL", p);
        if (plans[p]->prm.dtype != plans[0]->prm.dtype) return fail(BFM_EINVAL, "pair %d: dtype differs", p);
        if (phi[p] == nullptr || psi[p] == nullptr) return fail(BFM_EINVAL, "pair %d: NULL potential", p);
        if (!isfinite(scale[p])) return fail(BFM_EINVAL, "pair %d: scale must be finite", p);
        bfm_status st = check_ws(plans[p], workspaces[p], ws_bytes[p], &w[p]);
        if (st != BFM_OK) return fail(st, "pair %d: %s", p, g_last_error.c_str());
        for (int q = 0; q < p; ++q)
            if (workspaces[q] == workspaces[p]) return fail(BFM_EINVAL, "pairs %d and %d share a workspace", q, p);
        const bfm_plan_s *P = plans[p];
        GradPair &G = g[p];
        G.phi = phi[p];
        G.psi = psi[p];
        G.gmu = grad_mu != nullptr ? grad_mu[p] : nullptr;
        G.gnu = grad_nu != nullptr ? grad_nu[p] : nullptr;
        G.st = w[p].st;
        G.part = w[p].part;
        G.slot_len = w[p].slot_len;
        G.N = P->g.N;
        long long epb = 4 * kRedBlock;
        while ((G.N + epb - 1) / epb > G.slot_len) epb += 4 * kRedBlock;
        G.epb = epb;
        G.nb = (int)((G.N + epb - 1) / epb);
        G.mul = 2.0 * P->g.vol * scale[p];
    }
    hipStream_t s = (hipStream_t)stream;
    for (int first = 0; first < npairs; first += kBatchChunk) {
        const int np = npairs - first < kBatchChunk ? npairs - first : kBatchChunk;
        GradPair *tab = reinterpret_cast<GradPair *>(w[first].batch);
        HIP_TRY(hipMemcpyAsync(tab, g.data() + first, (size_t)np * sizeof(GradPair), hipMemcpyHostToDevice, s));
        if (plans[0]->prm.dtype == BFM_F64)
            HIP_TRY(launch_grad_multi<double>(tab, g.data() + first, np, s));
        else
            HIP_TRY(launch_grad_multi<float>(tab, g.data() + first, np, s));
    }
    // the host table must outlive the copies above
    HIP_TRY(hipStreamSynchronize(s));
    return BFM_OK;
}

// ------------------------------------------------------------ autotuner

// Candidate c-transform launch shapes are timed per axis, in the order of a
// transform, on a caller's sample potential (or, without one, on a smooth
// test potential written into the workspace); the fastest is kept in the
// plan and in a process-wide table keyed by (line length, strided, dtype,
// lines) that later untuned requests of the same geometry reuse.
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, long long>, CtCfg> g_tune;
}

template <typename T>
__global__ void tune_field_kernel(T *f, Grid g)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N; i += (long long)gridDim.x * blockDim.x) {
        long long r = i;
        double v = 0.0;
        for (int a = g.ndim - 1; a >= 0; --a) {
            const double x = ((double)(r % g.n[a]) + 0.5) / g.n[a];
            r /= g.n[a];
            v += 0.35 * x * x - 0.1 * x + 0.01 * sin(23.0 * x + a);
        }
        f[i] = (T)v;
    }
}

template <typename T>
static bfm_status autotune_impl(bfm_plan P, const T *sample, const Ws &w, hipStream_t s, int reps)
{
    const Grid &g = P->g;
    T *f = (T *)w.f, *o = (T *)w.pc, *nxt = (T *)w.rho;
    if (sample != nullptr) {
        HIP_TRY(hipMemcpyAsync(f, sample, (size_t)g.N * sizeof(T), hipMemcpyDeviceToDevice, s));
    } else {
        hipLaunchKernelGGL((tune_field_kernel<T>), dim3(1024), dim3(256), 0, s, f, g);
        HIP_TRY(hipGetLastError());
    }
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    bfm_status out = BFM_OK;
    // axes in the order of a transform (last axis first, its input -sample),
    // each later axis timed on the previous pass's output
    for (int ax = g.ndim - 1; ax >= 0 && out == BFM_OK; --ax) {
        const int n = g.n[ax], inner = (int)g.stride[ax];
        const long long nl = g.N / n;
        const T sgn = ax == g.ndim - 1 ? T(-1) : T(1);
        const auto key = std::make_tuple(n, inner > 1 ? 1 : 0, (int)sizeof(T), nl);
        bool cached = false;
        if (sample == nullptr) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(key);
            if (it != g_tune.end()) {
                P->ct_cfg[ax] = it->second;
                cached = true;
            }
        }
        if (cached) {
            HIP_TRY(launch_ct_axis<T>(f, nxt, n, inner, nl, sgn, nullptr, s, P->ct_cfg[ax]));
            std::swap(f, nxt);
            continue;
        }
        std::vector<CtCfg> cand;
        for (int C : {4, 8, 12, 16})
            for (int lpb : inner > 1 ? std::vector<int>{1, 2, 4} : std::vector<int>{0})
                for (int pers : {1, 2}) {
                    if ((n + C - 1) / C > 1024) continue;
                    CtCfg c;
                    c.C = C;
                    c.lpb = lpb;
                    c.pers = pers;
                    cand.push_back(c);   // shapes that do not apply fail to launch and are skipped
                }
        float best = 1e30f;
        CtCfg bestc;
        for (const CtCfg &c : cand) {
            hipError_t e = launch_ct_axis<T>(f, o, n, inner, nl, sgn, nullptr, s, c);   // warm-up
            if (e != hipSuccess) continue;
            (void)hipEventRecord(a, s);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_ct_axis<T>(f, o, n, inner, nl, sgn, nullptr, s, c);
            (void)hipEventRecord(b, s);
            if (hipEventSynchronize(b) != hipSuccess || e != hipSuccess) continue;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, a, b);
            if (ms < best) {
                best = ms;
                bestc = c;
            }
        }
        if (best >= 1e30f) {
            out = fail(BFM_EDEVICE, "autotune: no c-transform shape launched for axis %d", ax);
            break;
        }
        P->ct_cfg[ax] = bestc;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[key] = bestc;
        }
        if (launch_ct_axis<T>(f, nxt, n, inner, nl, sgn, nullptr, s, bestc) != hipSuccess) {
            out = fail(BFM_EDEVICE, "autotune: chained pass failed on axis %d", ax);
            break;
        }
        std::swap(f, nxt);
    }
    // 2D: the per-axis choice against the column-blocked form (both axes on
    // the persistent kernel, four-column groups, which lets the transform
    // pass the column-blocked intermediate); timed as whole transforms
    if (out == BFM_OK && g.ndim == 2) {
        const T *src = sample;
        if (src == nullptr) {
            hipLaunchKernelGGL((tune_field_kernel<T>), dim3(1024), dim3(256), 0, s, (T *)w.f, g);
            HIP_TRY(hipGetLastError());
            src = (const T *)w.f;
        }
        // candidates: the per-axis choice, then the blocked form with the
        // tuned column width (and 16) and each row width
        CtCfg cand[8][3];
        int ncand = 0;
        for (int a = 0; a < 3; ++a) cand[0][a] = P->ct_cfg[a];
        ncand = 1;
        for (int C0 : {P->ct_cfg[0].C, 16}) {
            if (C0 == 0 || (C0 == 16 && P->ct_cfg[0].C == 16 && ncand > 1)) continue;
            for (int C : {8, 16}) {
                if ((g.n[1] + C - 1) / C > 1024 || (g.n[0] + C0 - 1) / C0 > 1024) continue;
                for (int a = 0; a < 3; ++a) cand[ncand][a] = P->ct_cfg[a];
                cand[ncand][0].C = C0;
                cand[ncand][0].lpb = 4;
                cand[ncand][0].pers = 2;
                cand[ncand][1].C = C;
                cand[ncand][1].pers = 2;
                ++ncand;
            }
        }
        T *scratch = src == (const T *)w.f ? (T *)w.rho : (T *)w.f;
        float best = 1e30f;
        int pick = -1;
        for (int c = 0; c < ncand; ++c) {
            const CtCfg *cf = cand[c];
            hipError_t e = ctransform_field<T>(g, src, o, nullptr, s, cf, scratch);   // warm-up
            if (e != hipSuccess) continue;
            (void)hipEventRecord(a, s);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = ctransform_field<T>(g, src, o, nullptr, s, cf, scratch);
            (void)hipEventRecord(b, s);
            if (hipEventSynchronize(b) != hipSuccess || e != hipSuccess) continue;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, a, b);
            // candidates in the blocked form are credited 5%: in a solve they
            // also fuse <q, src> into the row pass, which this timing does not see
            if (ct_blocked_applies<T>(g, src, scratch, o, cf)) ms *= 0.95f;
            if (ms < best) {
                best = ms;
                pick = c;
            }
        }
        if (pick > 0) {
            P->ct_cfg[0] = cand[pick][0];
            P->ct_cfg[1] = cand[pick][1];
        }
        (void)hipGetLastError();
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return out;
}

extern "C" bfm_status bfm_autotune(bfm_plan plan, const void *sample, void *workspace, size_t ws_bytes, void *stream)
{
    if (plan == nullptr) return fail(BFM_EINVAL, "plan is NULL");
    Ws w;
    bfm_status st = check_ws(plan, workspace, ws_bytes, &w);
    if (st != BFM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (plan->prm.dtype == BFM_F64) return autotune_impl<double>(plan, (const double *)sample, w, s, 5);
    return autotune_impl<float>(plan, (const float *)sample, w, s, 5);
}

extern "C" bfm_status bfm_plan_set_deposit_grid(bfm_plan plan, int32_t workgroups)
{
    if (plan == nullptr) return fail(BFM_EINVAL, "plan is NULL");
    if (workgroups != 0 && (workgroups < 8 || workgroups > kMaxDepositGrid || workgroups % 8 != 0))
        return fail(BFM_EINVAL, "deposition workgroups %d: 0, or a multiple of 8 from 8 to %d", workgroups,
                    kMaxDepositGrid);
    plan->nsplat = workgroups == 0 ? (int)splat_blocks(plan->g) : workgroups;
    return BFM_OK;
}

extern "C" bfm_status bfm_plan_deposit_grid(bfm_plan plan, int32_t *workgroups)
{
    if (plan == nullptr || workgroups == nullptr) return fail(BFM_EINVAL, "NULL argument");
    *workgroups = plan->nsplat;
    return BFM_OK;
}

template <typename T>
static bfm_status autotune_deposit_impl(bfm_plan P, const T *phi, const T *mass, const Ws &w, hipStream_t s, int reps)
{
    const Grid &g = P->g;
    T *pc = (T *)w.pc, *rho = (T *)w.rho;
    HIP_TRY(ctransform_field<T>(g, phi, pc, nullptr, s, P->ct_cfg, (T *)w.f));
    HIP_TRY(launch_tile_list<T>(g, mass, (int *)w.f, w.tiles_mu, s));
    HIP_TRY(launch_fill<T>(rho, g.N, T(0), s));   // the deposits accumulate over the timed calls
    const long long tiles8 = (splat_tile_count(g) + 7) / 8 * 8;
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    float best = 1e30f;
    int pick = 0;
    for (int G : {1024, 2048, 4096, kMaxDepositGrid}) {
        if (G > tiles8 && G != 1024) continue;
        const int Gc = (long long)G > tiles8 ? (int)tiles8 : G;
        hipError_t e = launch_splat<T>(g, pc, mass, rho, nullptr, w.slot(S_PRIMAL), w.slot(S_PC_SRC), Gc, nullptr,
                                       s, T(1), w.tiles_mu);   // warm-up
        if (e != hipSuccess) continue;
        // the least of three timed blocks of `reps` calls: the candidates differ
        // by a few percent, about as much as two blocks of one candidate can
        float ms = 1e30f;
        for (int blk = 0; blk < 3 && e == hipSuccess; ++blk) {
            (void)hipEventRecord(a, s);
            for (int r = 0; r < reps && e == hipSuccess; ++r)
                e = launch_splat<T>(g, pc, mass, rho, nullptr, w.slot(S_PRIMAL), w.slot(S_PC_SRC), Gc, nullptr, s,
                                    T(1), w.tiles_mu);
            (void)hipEventRecord(b, s);
            if (hipEventSynchronize(b) != hipSuccess || e != hipSuccess) break;
            float t = 0.f;
            (void)hipEventElapsedTime(&t, a, b);
            ms = t < ms ? t : ms;
        }
        if (e != hipSuccess) continue;
        if (ms < best) {
            best = ms;
            pick = Gc;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (pick == 0) return fail(BFM_EDEVICE, "autotune: no deposition grid launched");
    P->nsplat = pick;
    return BFM_OK;
}

extern "C" bfm_status bfm_autotune_deposit(bfm_plan plan, const void *phi, const void *mass, void *workspace,
                                           size_t ws_bytes, void *stream)
{
    if (plan == nullptr || phi == nullptr || mass == nullptr) return fail(BFM_EINVAL, "NULL argument");
    Ws w;
    bfm_status st = check_ws(plan, workspace, ws_bytes, &w);
    if (st != BFM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (plan->prm.dtype == BFM_F64)
        return autotune_deposit_impl<double>(plan, (const double *)phi, (const double *)mass, w, s, 5);
    return autotune_deposit_impl<float>(plan, (const float *)phi, (const float *)mass, w, s, 5);
}

extern "C" bfm_status bfm_plan_set_tuning(bfm_plan plan, const int32_t *cfg9)
{
    if (plan == nullptr || cfg9 == nullptr) return fail(BFM_EINVAL, "NULL argument");
    CtCfg c[3];
    for (int a = 0; a < 3; ++a) {
        const int C = cfg9[3 * a], lpb = cfg9[3 * a + 1], pers = cfg9[3 * a + 2];
        if ((C != 0 && C != 4 && C != 8 && C != 12 && C != 16) || (lpb != 0 && lpb != 1 && lpb != 2 && lpb != 4) ||
            pers < 0 || pers > 2)
            return fail(BFM_EINVAL,
                        "tuning of axis %d: points per lane %d (0, 4, 8, 12, 16), lines %d (0, 1, 2, 4), mode %d (0-2)", a, C,
                        lpb, pers);
        if (a < plan->g.ndim && C != 0 && (plan->g.n[a] + C - 1) / C > 1024)
            return fail(BFM_EINVAL, "tuning of axis %d: %d points per lane do not cover %d points", a, C, plan->g.n[a]);
        c[a].C = C;
        c[a].lpb = lpb;
        c[a].pers = pers;
    }
    for (int a = 0; a < 3; ++a) plan->ct_cfg[a] = c[a];
    return BFM_OK;
}

extern "C" bfm_status bfm_plan_tuning(bfm_plan plan, int32_t *cfg9)
{
    if (plan == nullptr || cfg9 == nullptr) return fail(BFM_EINVAL, "NULL argument");
    for (int a = 0; a < 3; ++a) {
        cfg9[3 * a] = plan->ct_cfg[a].C;
        cfg9[3 * a + 1] = plan->ct_cfg[a].lpb;
        cfg9[3 * a + 2] = plan->ct_cfg[a].pers;
    }
    return BFM_OK;
}

// ------------------------------------------------------------ primitives

extern "C" bfm_status bfm_ctransform(bfm_plan plan, const void *in, void *out, void *workspace, size_t ws_bytes,
                                     void *stream)
{
    if (plan == nullptr || in == nullptr || out == nullptr) return fail(BFM_EINVAL, "NULL argument");
    Ws w;
    bfm_status st = check_ws(plan, workspace, ws_bytes, &w);
    if (st != BFM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (plan->prm.dtype == BFM_F64)
        HIP_TRY(ctransform_field<double>(plan->g, (const double *)in, (double *)out, nullptr, s, plan->ct_cfg,
                                         (double *)w.f));
    else
        HIP_TRY(ctransform_field<float>(plan->g, (const float *)in, (float *)out, nullptr, s, plan->ct_cfg,
                                        (float *)w.f));
    return BFM_OK;
}

extern "C" bfm_status bfm_ctransform_axis(bfm_plan plan, int32_t axis, int32_t sign, const void *in, void *out,
                                          void *stream)
{
    if (plan == nullptr || in == nullptr || out == nullptr) return fail(BFM_EINVAL, "NULL argument");
    if (axis < 0 || axis >= plan->g.ndim) return fail(BFM_EINVAL, "axis %d out of range", axis);
    if (sign != 1 && sign != -1) return fail(BFM_EINVAL, "sign must be +1 or -1");
    const Grid &g = plan->g;
    hipStream_t s = (hipStream_t)stream;
    const int n = g.n[axis], inner = (int)g.stride[axis];
    if (g.pw[axis] != 2.0) {
        if (plan->prm.dtype == BFM_F64)
            HIP_TRY(launch_ct_dc<double>((const double *)in, (double *)out, n, inner, g.N / n, (double)sign,
                                         g.pw[axis], nullptr, s));
        else
            HIP_TRY(launch_ct_dc<float>((const float *)in, (float *)out, n, inner, g.N / n, (float)sign, g.pw[axis],
                                        nullptr, s));
        return BFM_OK;
    }
    if (plan->prm.dtype == BFM_F64)
        HIP_TRY(launch_ct_axis<double>((const double *)in, (double *)out, n, inner, g.N / n, (double)sign, nullptr,
                                       s, plan->ct_cfg[axis]));
    else
        HIP_TRY(launch_ct_axis<float>((const float *)in, (float *)out, n, inner, g.N / n, (float)sign, nullptr, s,
                                      plan->ct_cfg[axis]));
    return BFM_OK;
}

template <typename T>
static bfm_status ct_pass_impl(bfm_plan plan, int pass, const T *in, T *out, const T *weight, double *host_sum,
                               const Ws &w, hipStream_t s)
{
    const Grid &g = plan->g;
    const bool ok = pass == 0 ? ct_blocked_applies<T>(g, in, out, out, plan->ct_cfg)
                              : ct_blocked_applies<T>(g, in, in, out, plan->ct_cfg);
    if (!ok)
        return fail(BFM_EUNSUPPORTED, "the column-blocked two-pass transform does not apply to this plan "
                                      "(2D, last size a multiple of 4, persistent launch shapes, 16-byte aligned "
                                      "fields)");
    int nd = 0;
    HIP_TRY(ct_blocked_pass<T>(g, pass, in, out, nullptr, s, plan->ct_cfg, pass == 1 ? weight : nullptr,
                               w.slot(S_Q_SRC), &nd));
    if (nd > w.slot_len) return fail(BFM_EDEVICE, "c-transform pass: %d partials exceed the slot", nd);
    if (host_sum != nullptr) {
        std::vector<double> h(nd > 0 ? nd : 1);
        if (nd > 0) HIP_TRY(hipMemcpyAsync(h.data(), w.slot(S_Q_SRC), nd * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double sum = 0.0;
        for (int i = 0; i < nd; ++i) sum += h[i];
        *host_sum = sum;
    }
    return BFM_OK;
}

extern "C" bfm_status bfm_ctransform_pass(bfm_plan plan, int32_t pass, const void *in, void *out, const void *weight,
                                          double *host_sum, void *workspace, size_t ws_bytes, void *stream)
{
    if (plan == nullptr || in == nullptr || out == nullptr) return fail(BFM_EINVAL, "NULL argument");
    if (pass != 0 && pass != 1) return fail(BFM_EINVAL, "pass must be 0 or 1");
    if (in == out) return fail(BFM_EINVAL, "in and out must be distinct buffers");
    if (host_sum != nullptr && (pass != 1 || weight == nullptr))
        return fail(BFM_EINVAL, "host_sum needs pass 1 and a weight field");
    Ws w;
    bfm_status st = check_ws(plan, workspace, ws_bytes, &w);
    if (st != BFM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (plan->prm.dtype == BFM_F64)
        return ct_pass_impl<double>(plan, pass, (const double *)in, (double *)out, (const double *)weight, host_sum,
                                    w, s);
    return ct_pass_impl<float>(plan, pass, (const float *)in, (float *)out, (const float *)weight, host_sum, w, s);
}

template <typename T>
static bfm_status interp_impl(bfm_plan P, const T *phi, const T *mu, int nt, const double *times, T *rho,
                              const Ws &w, hipStream_t s)
{
    const Grid &g = P->g;
    T *pc = (T *)w.pc;
    HIP_TRY(ctransform_field<T>(g, phi, pc, nullptr, s, P->ct_cfg, (T *)w.f));
    for (int k = 0; k < nt; ++k) {
        T *r = rho + (size_t)k * g.N;
        HIP_TRY(launch_fill<T>(r, g.N, T(0), s));
        HIP_TRY(launch_splat<T>(g, pc, mu, r, nullptr, nullptr, nullptr, P->nsplat, nullptr, s, (T)times[k]));
    }
    return BFM_OK;
}

extern "C" bfm_status bfm_interpolate(bfm_plan plan, const void *phi, const void *mu, int32_t ntimes,
                                      const double *times, void *rho, void *workspace, size_t ws_bytes, void *stream)
{
    if (plan == nullptr || phi == nullptr || mu == nullptr || times == nullptr || rho == nullptr)
        return fail(BFM_EINVAL, "NULL argument");
    if (ntimes < 1) return fail(BFM_EINVAL, "ntimes = %d: need at least one time", ntimes);
    for (int k = 0; k < ntimes; ++k)
        if (!(times[k] >= 0.0 && times[k] <= 1.0)) return fail(BFM_EINVAL, "times[%d] = %g is not in [0, 1]", k, times[k]);
    if (rho == phi || rho == mu) return fail(BFM_EINVAL, "rho must not alias phi or mu");
    Ws w;
    bfm_status st = check_ws(plan, workspace, ws_bytes, &w);
    if (st != BFM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (plan->prm.dtype == BFM_F64)
        return interp_impl<double>(plan, (const double *)phi, (const double *)mu, ntimes, times, (double *)rho, w, s);
    return interp_impl<float>(plan, (const float *)phi, (const float *)mu, ntimes, times, (float *)rho, w, s);
}

extern "C" bfm_status bfm_trace(bfm_plan plan, const void *workspace, size_t ws_bytes, double *host,
                                int32_t max_records, int32_t *count, void *stream)
{
    if (plan == nullptr || count == nullptr || (host == nullptr && max_records > 0))
        return fail(BFM_EINVAL, "NULL argument");
    Ws w;
    bfm_status st = check_ws(plan, (void *)workspace, ws_bytes, &w);
    if (st != BFM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    DevState hs;
    HIP_TRY(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *count = hs.ntrace;
    int m = hs.ntrace < max_records ? hs.ntrace : max_records;
    if (m > kMaxTrace) m = kMaxTrace;
    if (m > 0) {
        HIP_TRY(hipMemcpyAsync(host, w.trace, (size_t)m * sizeof(TraceRec), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return BFM_OK;
}

static double host_slot_sum(const std::vector<double> &v) {
    double acc = 0.0;
    for (double x : v) acc += x;
    return acc;
}

template <typename T>
static bfm_status push_impl(bfm_plan P, const T *phic, const T *mass, T *rho, T *Tmap, double *primal,
                            const Ws &w, hipStream_t s)
{
    HIP_TRY(launch_fill<T>(rho, P->g.N, T(0), s));
    HIP_TRY(launch_splat<T>(P->g, phic, mass, rho, Tmap, w.slot(S_PRIMAL), w.slot(S_PC_SRC), P->nsplat, nullptr, s));
    if (primal != nullptr) {
        std::vector<double> h(P->nsplat);
        HIP_TRY(hipMemcpyAsync(h.data(), w.slot(S_PRIMAL), P->nsplat * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *primal = P->g.vol * host_slot_sum(h);
    }
    return BFM_OK;
}

extern "C" bfm_status bfm_pushforward(bfm_plan plan, const void *phic, const void *mass, void *rho, void *T,
                                      double *primal, void *workspace, size_t ws_bytes, void *stream)
{
    if (plan == nullptr || phic == nullptr || mass == nullptr || rho == nullptr)
        return fail(BFM_EINVAL, "NULL argument");
    Ws w;
    bfm_status st = check_ws(plan, workspace, ws_bytes, &w);
    if (st != BFM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (plan->prm.dtype == BFM_F64)
        return push_impl<double>(plan, (const double *)phic, (const double *)mass, (double *)rho, (double *)T,
                                 primal, w, s);
    return push_impl<float>(plan, (const float *)phic, (const float *)mass, (float *)rho, (float *)T, primal, w,
                            s);
}

template <typename T>
static bfm_status poisson_impl(bfm_plan P, const T *f, T *g, double *G, const Ws &w, hipStream_t s)
{
    HIP_TRY(upload_tables(P, w, s));
    HIP_TRY(poisson_forward<T>(P, w, f, nullptr, 0, g, nullptr, s));
    HIP_TRY(poisson_inverse<T>(P, w, g, g, nullptr, nullptr, s));
    if (G != nullptr) {
        std::vector<double> h(P->gparts);
        HIP_TRY(hipMemcpyAsync(h.data(), w.gpart, P->gparts * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *G = P->g.vol * host_slot_sum(h);
    }
    return BFM_OK;
}

extern "C" bfm_status bfm_poisson_neumann(bfm_plan plan, const void *f, void *g, double *G, void *workspace,
                                          size_t ws_bytes, void *stream)
{
    if (plan == nullptr || f == nullptr || g == nullptr) return fail(BFM_EINVAL, "NULL argument");
    Ws w;
    bfm_status st = check_ws(plan, workspace, ws_bytes, &w);
    if (st != BFM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (plan->prm.dtype == BFM_F64)
        return poisson_impl<double>(plan, (const double *)f, (double *)g, G, w, s);
    return poisson_impl<float>(plan, (const float *)f, (float *)g, G, w, s);
}

template <typename T>
static bfm_status grad_impl(bfm_plan P, const T *phi, const T *psi, double scale, T *gmu, T *gnu, const Ws &w,
                            hipStream_t s)
{
    const int nb = P->red_blocks;
    HIP_TRY(launch_dot2<T>(psi, nullptr, nullptr, nullptr, P->g.N, w.slot(S_MEAN_A), nullptr, nb, nullptr, s));
    HIP_TRY(launch_dot2<T>(phi, nullptr, nullptr, nullptr, P->g.N, w.slot(S_MEAN_B), nullptr, nb, nullptr, s));
    HIP_TRY(launch_ctrl(w.st, w.part, w.gpart, CTRL_MEANS, ctrl_params(P), w.trace, s));
    HIP_TRY(launch_shift_scale<T>(gmu, psi, &w.st->mean_a, -1.0, gnu, phi, &w.st->mean_b, -1.0, P->g.N,
                                  2.0 * P->g.vol * scale, s));
    return BFM_OK;
}

extern "C" bfm_status bfm_grad(bfm_plan plan, const void *phi, const void *psi, double scale, void *grad_mu,
                               void *grad_nu, void *workspace, size_t ws_bytes, void *stream)
{
    if (plan == nullptr || phi == nullptr || psi == nullptr) return fail(BFM_EINVAL, "NULL argument");
    if (!isfinite(scale)) return fail(BFM_EINVAL, "scale must be finite");
    Ws w;
    bfm_status st = check_ws(plan, workspace, ws_bytes, &w);
    if (st != BFM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (plan->prm.dtype == BFM_F64)
        return grad_impl<double>(plan, (const double *)phi, (const double *)psi, scale, (double *)grad_mu,
                                 (double *)grad_nu, w, s);
    return grad_impl<float>(plan, (const float *)phi, (const float *)psi, scale, (float *)grad_mu,
                            (float *)grad_nu, w, s);
}
