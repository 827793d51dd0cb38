/*
 * Test infrastructure only (CPU oracle): never linked into the product path.
 *
 * One-dimensional step of the separable c-transform for the quadratic cost,
 * written as its definition (paper, Definition of the c-transform and the
 * separable decomposition of Section 4.1): for every line l and every grid
 * point x_i,
 *
 *     out[l][i] = min over all j of  0.5 * (x_i - y_j)^2 + in[l][j],
 *
 * with cell-centred points x_i = (i + 1/2) h, y_j = (j + 1/2) h.  Plain
 * O(n^2) per line in float64; lines are independent and split over OpenMP
 * threads.  No hull, no search, no pruning.
 */
#include <math.h>
#include <stdint.h>

void oracle_line_min(const double *in, double *out, int64_t nlines, int64_t n, double h)
{
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < nlines; ++l) {
        const double *u = in + l * n;
        double *o = out + l * n;
        for (int64_t i = 0; i < n; ++i) {
            const double xi = ((double)i + 0.5) * h;
            double best = INFINITY;
            for (int64_t j = 0; j < n; ++j) {
                const double d = xi - ((double)j + 0.5) * h;
                const double v = 0.5 * d * d + u[j];
                best = v < best ? v : best;
            }
            o[i] = best;
        }
    }
}

/*
 * The same one-dimensional step for the separable power cost of eq. p_costs,
 * h(z) = |z|^p / p with p > 1 (Section 4.1 for general separable costs;
 * Section 4.3, optimal transport with general costs):
 *
 *     out[l][i] = min over all j of  |x_i - y_j|^p / p + in[l][j].
 *
 * Plain O(n^2) per line, from the definition, like oracle_line_min.
 */
void oracle_line_min_p(const double *in, double *out, int64_t nlines, int64_t n, double h, double p)
{
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < nlines; ++l) {
        const double *u = in + l * n;
        double *o = out + l * n;
        for (int64_t i = 0; i < n; ++i) {
            const double xi = ((double)i + 0.5) * h;
            double best = INFINITY;
            for (int64_t j = 0; j < n; ++j) {
                const double d = fabs(xi - ((double)j + 0.5) * h);
                const double v = pow(d, p) / p + u[j];
                best = v < best ? v : best;
            }
            o[i] = best;
        }
    }
}

int oracle_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}
