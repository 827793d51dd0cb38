/*
 * bfm.h -- C ABI of the MI355X (gfx950) back-and-forth optimal-transport library.
 *
 * Problem (paper: Jacobs & Leger, "A fast approach to optimal transport: the
 * back-and-forth method", Section 3, eq. dual): given two probability
 * densities mu, nu on the uniform grid of Omega = [0,1]^d (d = 2 or 3,
 * Section 4.3) and the quadratic cost c(x,y) = |x-y|^2 / 2, maximise the
 * Kantorovich dual J(phi) = int phi dnu + int phi^c dmu (eq. defJ) by the
 * back-and-forth iteration (Algorithm 1) with H^1 gradient steps
 * (eq. gradients_J_I) and the adaptive step size of Section 4.2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid:    shape[0..ndim-1] cells per axis, row-major, axis ndim-1 contiguous.
 *          Cells are centred: x = (i + 1/2) / n_a on axis a.  N = prod(shape).
 * Fields:  device arrays of N elements of the plan's dtype (float or double),
 *          owned and allocated by the caller.  A density f is given by its
 *          grid values with cell_volume * sum(f) = 1.
 * Maps:    T is ndim planar fields (T_0 then T_1 ...), each N elements, in
 *          physical coordinates, clamped to [h_a/2, 1 - h_a/2].
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 *          Work is enqueued asynchronously on it.  Entry points that return
 *          host scalars synchronise that stream before returning.
 * Memory:  the library never allocates device memory.  Every call that needs
 *          scratch takes a caller-owned device `workspace` of at least
 *          bfm_plan_workspace_bytes() bytes, 256-byte aligned, not shared
 *          between calls that may run concurrently.  A plan owns host memory
 *          only.
 * Errors:  every call returns a bfm_status; no exception crosses the ABI.
 *          Argument validation happens before any launch.  The message of the
 *          last failure on the calling thread is returned by bfm_last_error().
 */
#ifndef BFM_H
#define BFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BFM_OK = 0,
    BFM_EINVAL = 1,        /* invalid argument: null pointer, bad shape, bad density ... */
    BFM_EDEVICE = 2,       /* a HIP call failed (launch, copy, synchronise) */
    BFM_ENUMERIC = 3,      /* a non-finite value appeared in the device state */
    BFM_EWORKSPACE = 4,    /* workspace pointer null, misaligned or too small */
    BFM_EUNSUPPORTED = 5   /* valid request outside what the library implements */
} bfm_status;

typedef enum { BFM_F32 = 0, BFM_F64 = 1 } bfm_dtype;

/* Iteration scheme of bfm_solve / bfm_solve_batched.
 *   BFM_METHOD_BFM: the back-and-forth iteration of Algorithm 1: a gradient
 *     step on J in phi-space, a c-transform, a gradient step on I in
 *     psi-space, a c-transform (4 c-transforms, 2 Poisson solves per
 *     iteration).
 *   BFM_METHOD_GA: the plain H^1 gradient ascent on J that Section 4.3
 *     compares against (Tables 5 and 6): phi_{n+1/2} = phi_n + sigma grad J(phi_n),
 *     phi_{n+1} = (phi_{n+1/2})^cc.  The first c-transform of the double
 *     transform is phi_{n+1}^c itself (a c-transform is idempotent after two
 *     applications: f^ccc = f^c), so it serves the next head and an
 *     iteration costs 2 c-transforms and 1 Poisson solve.  Same step rule,
 *     gap and stopping test as the back-and-forth iteration. */
typedef enum { BFM_METHOD_BFM = 0, BFM_METHOD_GA = 1 } bfm_method;

/* Solver parameters.  Defaults (bfm_params_init) are the paper's Section 4.2
 * constants: sigma_min = 0.01, beta1 = 1/4, beta2 = 3/4, alpha1 = 5/4,
 * alpha2 = 4/5, and sigma0 <= 0 meaning 8 min(1/max mu, 1/max nu). */
typedef struct {
    int32_t ndim;          /* 2 or 3 */
    int32_t shape[3];      /* cells per axis, each 4 <= n <= 4096 and of the form 2^a 3^b */
    int32_t dtype;         /* bfm_dtype: storage and arithmetic type of fields; sums are float64 */
    int32_t max_iters;     /* full iterations (BFM: phi-step + psi-step; GA: one gradient step + cc) */
    double tol;            /* stop when gap < tol; 0 runs max_iters iterations */
    double sigma0;         /* initial step; <= 0 selects 8 min(1/max mu, 1/max nu) */
    double sigma_min;
    double beta1, beta2, alpha1, alpha2;
    int32_t check_every;   /* iterations enqueued between host reads of the stop flag (>= 1) */
    int32_t method;        /* bfm_method; default BFM_METHOD_BFM */
    double power[3];       /* cost exponent per axis, 1.05 <= p <= 8 (default 2: the quadratic cost).
                            * The cost is c(x, y) = sum_a |x_a - y_a|^p_a / p_a (Section 4.3,
                            * eq. p_costs); p_a = 2 on every axis is |x - y|^2 / 2.  An axis with
                            * p_a != 2 takes the monotone divide-and-conquer c-transform of
                            * Section 4.1 (O(n log n) per line) instead of the convex-hull one, and
                            * the map becomes T = x - (grad h)^{-1}(grad phi^c), component a being
                            * x_a - sign(g_a) |g_a|^{1/(p_a - 1)}. */
} bfm_params;

/* Per-solve report (host struct). gap = max(|primal - dual|, G) at the last
 * evaluated head, G = ||nu - T#mu||^2 in H^-1 (squared H^1 norm of the gradient). */
typedef struct {
    int32_t iters;         /* completed full iterations */
    int32_t converged;     /* 1 when gap < tol stopped the loop */
    int32_t status;        /* bfm_status of the solve */
    int32_t sigma_floor_hits;  /* step-size updates (Section 4.2 rule) that left sigma at sigma_min:
                                * the shrink branch was clamped there, or sigma stayed at it */
    double dual;           /* J(phi) = C(mu,nu) estimate = W2^2 / 2 */
    double primal;         /* int |x - T(x)|^2 / 2 dmu */
    double gap;
    double G;
    double sigma;          /* step size after the last update */
    double mass_mu, mass_nu;  /* cell_volume * sum, as read on the device */
} bfm_result;

typedef struct bfm_plan_s *bfm_plan;

/* Fill `p` with the defaults for a grid; returns BFM_EINVAL on a bad shape. */
bfm_status bfm_params_init(bfm_params *p, int32_t ndim, const int32_t *shape, int32_t dtype);

/* Validate parameters and build the host-side plan (spectral tables, launch
 * shapes).  Host only: no device call.  *out receives a plan to be released
 * with bfm_plan_destroy. */
bfm_status bfm_plan_create(const bfm_params *p, bfm_plan *out);
void bfm_plan_destroy(bfm_plan plan);

/* Bytes of device workspace every call on this plan needs. */
bfm_status bfm_plan_workspace_bytes(bfm_plan plan, size_t *bytes);

/* Back-and-forth solve (Algorithm 1, step rule of Section 4.2), or with
 * params.method = BFM_METHOD_GA the plain gradient ascent of Section 4.3.
 *   mu, nu     device, N elements each: source and target densities (read only).
 *              Rejected with BFM_EINVAL (before any iteration) if a value is
 *              negative or non-finite or |cell_volume*sum - 1| > 1e-5.
 *   phi_init   device, N elements or NULL (NULL: phi_0 = 0).  Warm start/resume.
 *   phi, psi   device outputs, N elements each: phi - mean(phi) and
 *              psi = phi^c + mean(phi), an exactly c-conjugate pair.
 *              Also used as working buffers during the solve.
 *   T          device output, ndim*N elements, or NULL: the map x - grad psi.
 *   result     host output (may be NULL).
 * Synchronises `stream` every check_every iterations to read the stop flag.
 * Not reaching tol within max_iters is not an error (converged = 0). */
bfm_status bfm_solve(bfm_plan plan, const void *mu, const void *nu, const void *phi_init,
                     void *phi, void *psi, void *T, void *workspace, size_t ws_bytes,
                     void *stream, bfm_result *result);

/* bfm_solve without a workspace argument, for callers that cannot allocate
 * device memory (code that must not call hipMalloc: tight serving loops,
 * harnesses that forbid allocation).  Same arguments, outputs, validation and
 * synchronisation as bfm_solve; the solve's scratch lives in a static device
 * array of 64 MiB (67108864 bytes) that the library holds on every GPU it runs
 * on until the process ends.  Plans whose bfm_plan_workspace_bytes exceeds
 * that size are rejected with BFM_EWORKSPACE before any device call (float32
 * 2048^2 and float64 1536^2 fit; float32 4096^2 does not).  The device is the
 * calling thread's current device, which must be the device of `stream`.
 * Every call on one GPU shares that array: calls that overlap in time on one
 * GPU (from several threads or streams) race and must be serialised by the
 * caller.  Each call re-initialises everything it reads from the array, so
 * nothing carries over from an earlier call. */
bfm_status bfm_solve_noalloc(bfm_plan plan, const void *mu, const void *nu, const void *phi_init,
                             void *phi, void *psi, void *T, void *stream, bfm_result *result);

/* Batched solve of `npairs` independent problems (Algorithm 1 for each),
 * advanced together: after the first iteration, iters_per_graph iterations of
 * every problem are captured once into a HIP graph (independent problems on
 * parallel branches) and the graph is replayed; each problem keeps its own
 * step size, gap and stop flag, and a problem that has stopped turns into
 * no-ops.  Stop flags are read on the host between replays.
 *   plans       npairs plans (any shapes; same dtype and max_iters; tol and method may differ).
 *   mu .. T     host arrays of npairs device pointers (T may be NULL, or
 *               hold NULL entries); same meaning as in bfm_solve.
 *   workspaces  host array of npairs distinct device workspaces;
 *   ws_bytes    their sizes.
 *   results     host array of npairs reports (may be NULL).
 * Synchronises `stream` between graph replays and at the end. */
bfm_status bfm_solve_batched(int32_t npairs, const bfm_plan *plans, const void *const *mu, const void *const *nu,
                             void *const *phi, void *const *psi, void *const *T, void *const *workspaces,
                             const size_t *ws_bytes, int32_t iters_per_graph, void *stream, bfm_result *results);

/* Gradients of W2^2 for a batch of converged pairs (the bfm_grad formula for
 * every pair: grad_mu = scale[p] * 2 cell_volume (psi - mean psi),
 * grad_nu = scale[p] * 2 cell_volume (phi - mean phi); first variation of J,
 * Lemma fact:derivative-J, envelope form), computed by three launches for the
 * whole batch (potential sums per workgroup, the means per pair, the scaled
 * differences) instead of four per pair.
 *   plans       npairs plans (any shapes, one dtype).
 *   phi, psi    host arrays of npairs device pointers: each pair's potentials,
 *               N elements each (e.g. the outputs of bfm_solve_batched).
 *   scale       host array of npairs factors (e.g. the upstream gradients).
 *   grad_mu, grad_nu  host arrays of npairs device outputs of N elements, or
 *               NULL (that gradient is not computed); NULL entries allowed.
 *   workspaces  host array of npairs distinct device workspaces (overwritten).
 * BFM_EINVAL for NULL arrays, mixed dtypes, a non-finite scale or shared
 * workspaces; BFM_EWORKSPACE as in bfm_solve.  Synchronises `stream`. */
bfm_status bfm_grad_batched(int32_t npairs, const bfm_plan *plans, const void *const *phi, const void *const *psi,
                            const double *scale, void *const *grad_mu, void *const *grad_nu,
                            void *const *workspaces, const size_t *ws_bytes, void *stream);

/* Autotuner: times the candidate launch shapes of the c-transform line
 * kernel for every axis of the plan (points per lane 4, 8, 12 or 16; on strided
 * axes one, two or four lines per workgroup; one line group per workgroup or
 * persistent prefetching workgroups), axis by axis in the order of a
 * transform, on `sample` (a device potential of N elements, e.g. the
 * current phi; NULL: a smooth test potential), and keeps the fastest in the
 * plan (and in a process-wide table).  In 2D it then times the whole
 * transform with that choice against both axes on the persistent kernel
 * (which passes a column-blocked intermediate between the two passes) and
 * keeps the faster.  Optional: untuned plans use built-in shapes.
 * Synchronises `stream`; overwrites the workspace. */
bfm_status bfm_autotune(bfm_plan plan, const void *sample, void *workspace, size_t ws_bytes, void *stream);

/* The launch shapes the plan uses, three int32 per axis a < 3:
 * cfg9[3a] = points per lane, cfg9[3a+1] = lines per workgroup on a strided
 * axis, cfg9[3a+2] = 1 one line group per workgroup, 2 persistent
 * workgroups (0 everywhere = built-in choice). */
bfm_status bfm_plan_tuning(bfm_plan plan, int32_t *cfg9);

/* Sets the launch shapes (same layout as bfm_plan_tuning), e.g. to reuse a
 * tuning from an earlier process.  BFM_EINVAL for values outside the listed
 * choices or too few points per lane for the axis (C * 1024 < n).  A mode-2
 * (persistent) choice on a layout it does not apply to (n % 4 != 0 on the
 * last axis; on a strided axis one line per workgroup, four lines with
 * inner % 4 != 0 or two with inner odd; fields not 16-byte aligned) makes
 * later calls fail with BFM_EDEVICE. */
bfm_status bfm_plan_set_tuning(bfm_plan plan, const int32_t *cfg9);

/* Deposition workgroups (the pushforward of Section 2.1 on the grid): the
 * deposition walks the source tiles that hold mass with this many
 * workgroups.  0 restores the built-in count (one per 8^3 or 16 x 32 tile, at
 * most 2048); otherwise a multiple of 8 from 8 to 8192.  BFM_EINVAL outside
 * that.  The count changes only the order of the float64 partial sums. */
bfm_status bfm_plan_set_deposit_grid(bfm_plan plan, int32_t workgroups);
bfm_status bfm_plan_deposit_grid(bfm_plan plan, int32_t *workgroups);

/* Times the deposition with 1024, 2048, 4096 and 8192 workgroups (those not
 * above the tile count rounded up to a multiple of 8) on phi^c of `phi` and
 * the density `mass` (N device elements each; mass as the solver walks it:
 * its tiles with mass only), and keeps the fastest in the plan.  The best
 * count depends on the density's support and the map, so the caller passes
 * the problem's own.  Synchronises `stream`; overwrites the workspace. */
bfm_status bfm_autotune_deposit(bfm_plan plan, const void *phi, const void *mass, void *workspace, size_t ws_bytes,
                                void *stream);

/* Displacement interpolation (Section 4.3, optimal transport of images):
 * for each time t_k in [0, 1],
 *   rho_k = S_t # mu,  S_t(x) = t T(x) + (1 - t) x,  T(x) = x - grad phi^c(x),
 * with the map and the multilinear deposition of bfm_pushforward (t = 0
 * gives mu, t = 1 the pushforward by T).  phi is a potential from bfm_solve
 * (T is then the computed map from mu to nu); phi and mu are device fields of
 * N elements; rho is a device array of ntimes * N elements (frame k at
 * offset k * N), written whole.  times is a host array of ntimes values.
 * BFM_EINVAL for NULL arguments, ntimes < 1, a time outside [0, 1] or rho
 * aliasing phi or mu.  Overwrites the workspace. */
bfm_status bfm_interpolate(bfm_plan plan, const void *phi, const void *mu, int32_t ntimes, const double *times,
                           void *rho, void *workspace, size_t ws_bytes, void *stream);

/* Primitive: c-transform on the grid for the plan's cost (Definition of the
 * c-transform; separable evaluation of Section 4.1):
 *   out(x) = min over grid points y of c(x, y) - in(y),
 * c = |x - y|^2 / 2 (per line the Legendre transform on the lower convex
 * hull, eq. legendre / legendre_search), or with params.power the sum over
 * axes of |x_a - y_a|^p_a / p_a (axes with p_a != 2 by the monotone divide and
 * conquer of Section 4.1).  in and out are device fields of N elements; out
 * may equal in. */
bfm_status bfm_ctransform(bfm_plan plan, const void *in, void *out, void *workspace,
                          size_t ws_bytes, void *stream);

/* Primitive: map and pushforward (Lemma on c-transform properties (ii);
 * pushforward of Section 2.1).  T = x - grad phic for h = |.|^2/2, or
 * component a of T = x_a - sign(g_a)|g_a|^{1/(p_a - 1)} with g = grad phic
 * for the power costs (central differences, one-sided at faces, clamped to
 * the cell-centre box) and
 * rho = T#mass by cloud-in-cell deposition (multilinear weights).
 *   phic, mass  device inputs, N elements.
 *   rho         device output density, N elements (overwritten).
 *   T           device output, ndim*N elements, or NULL.
 *   primal      host output or NULL: int c(x, T(x)) dmass (synchronises). */
bfm_status bfm_pushforward(bfm_plan plan, const void *phic, const void *mass, void *rho, void *T,
                           double *primal, void *workspace, size_t ws_bytes, void *stream);

/* Primitive: H^1 gradient (H^1-gradient lemma, eq. gradients_J_I):
 * g = (-Laplacian)^{-1}(f - mean f) with zero-flux Neumann data, the
 * Laplacian being the second-difference stencil diagonalised by the DCT-II
 * (inversion by FFT, Section 4.3).
 *   f  device input, N elements (read only); g device output, N elements.
 *   G  host output or NULL: cell_volume * sum(f g) = ||f - mean f||^2_{H^-1}
 *      (synchronises). */
bfm_status bfm_poisson_neumann(bfm_plan plan, const void *f, void *g, double *G,
                               void *workspace, size_t ws_bytes, void *stream);

/* Gradient of W2^2 = 2 C(mu,nu) with respect to the grid density values at a
 * converged pair (first variation of J, Lemma fact:derivative-J, envelope
 * form): grad_mu = scale * 2 cell_volume (psi - mean psi),
 * grad_nu = scale * 2 cell_volume (phi - mean phi).  Either output may be NULL. */
bfm_status bfm_grad(bfm_plan plan, const void *phi, const void *psi, double scale,
                    void *grad_mu, void *grad_nu, void *workspace, size_t ws_bytes, void *stream);

/* Primitive: one separable pass of the c-transform along `axis` (the
 * one-dimensional step of Section 4.1): for every grid line along that axis
 *   out_i = min_j h_axis(x_i - y_j) + sign * in_j ,
 * h_axis(z) = z^2 / 2, or |z|^p / p with p = params.power[axis].
 * sign is +1 or -1 (the first pass of a transform uses -1).  in/out are
 * device fields of N elements; out may equal in.  Exposed for measurement
 * and tests. */
bfm_status bfm_ctransform_axis(bfm_plan plan, int32_t axis, int32_t sign, const void *in, void *out,
                               void *stream);

/* Primitive: one pass of the two-pass form of a 2D c-transform that the
 * solver uses when it applies (Section 4.1, separable evaluation; the axes
 * are independent minimisations, so columns may go first):
 *   pass 0: out = the column pass of u = -in, written in the column-blocked
 *           layout: element (r, c) of the n0 x n1 result at
 *           (c / 4) * 4 n0 + 4 r + c % 4 (each group of four columns is one
 *           contiguous run);
 *   pass 1: in = a column-blocked field, out = its row pass, row-major, so
 *           pass 1 after pass 0 gives in^c.  With `weight` (a row-major
 *           field), also sum_x out(x) weight(x) in float64: its per-workgroup
 *           partials go to the workspace and, when host_sum is non-NULL, the
 *           fixed-order total to *host_sum (synchronises `stream`).
 * in, out (and weight) are distinct device fields of N elements, 16-byte
 * aligned.  BFM_EINVAL for a NULL or aliased field, pass not 0 or 1, or
 * host_sum without pass 1 and a weight.  BFM_EUNSUPPORTED when the form does
 * not apply: not 2D, n1 not a multiple of 4, or launch shapes that are not
 * persistent with four-column groups (the float32 default for large enough
 * grids; float64 plans need bfm_plan_set_tuning). */
bfm_status bfm_ctransform_pass(bfm_plan plan, int32_t pass, const void *in, void *out, const void *weight,
                               double *host_sum, void *workspace, size_t ws_bytes, void *stream);

/* Copy the per-iteration trace of the last bfm_solve run on `workspace`
 * to host memory: record r is 8 doubles (iteration, dual J(phi_n), primal
 * P_n, G_n, gap_n, sigma_n, J(phi_{n+1/2}), I(psi_{n+1})) taken at the head of
 * iteration n.  Up to max_records records are copied; *count receives the
 * number recorded (which may exceed max_records).  Synchronises `stream`. */
bfm_status bfm_trace(bfm_plan plan, const void *workspace, size_t ws_bytes, double *host, int32_t max_records,
                     int32_t *count, void *stream);

/* Message describing the last non-OK status returned on this thread. */
const char *bfm_last_error(void);

/* Library version string. */
const char *bfm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BFM_H */
