/*
 * FP64 CPU reference ("oracle") for the exact softened all-pairs gravity sum
 * of Fujiwara & Nakasato, "Fast Simulations of Gravitational Many-body
 * Problem on RV770 GPU" (arXiv:0904.3659).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg load this library.  It shares no code, header, table or
 * helper with the HIP library; it is the plain definition written out, slow
 * and obviously correct, so that the GPU path can be checked against it.
 *
 * Arithmetic: IEEE double, no fast-math, no FMA contraction (built with
 * -ffp-contract=off).  Inputs are float32 values upcast to double by the
 * caller, so every coordinate difference is exact.  For every output row the
 * j-sum runs sequentially in index order, so the result does not depend on
 * the number of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count for later calls (timing only: results do not depend on it). */
void oracle_set_num_threads(int threads)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

/*
 * Eq. (gravity), Sec. I.  For each requested row i:
 *     a_i = sum_{j != i} m_j (x_i - x_j) / (|x_i - x_j|^2 + eps^2)^(3/2)
 *     p_i = sum_{j != i} m_j / (|x_i - x_j|^2 + eps^2)^(1/2)
 * in the paper's sign (a points from x_j towards x_i, p is positive).
 * The term j == i is skipped by index, as the sum's bounds state.
 *
 * x: [n,3] row-major, m: [n], eps2 = eps^2.
 * rows: indices of the rows to evaluate (NULL means rows 0..nrows-1).
 * a: [nrows,3] and p: [nrows] receive row r = rows[r] (either may be NULL).
 */
void oracle_forces_rows(const double *x, const double *m, int64_t n, double eps2,
                        const int64_t *rows, int64_t nrows, double *a, double *p)
{
    int64_t r;
#pragma omp parallel for schedule(dynamic, 8)
    for (r = 0; r < nrows; ++r) {
        const int64_t i = rows ? rows[r] : r;
        double ax = 0.0, ay = 0.0, az = 0.0, pot = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            const double dx = x[3 * i + 0] - x[3 * j + 0];
            const double dy = x[3 * i + 1] - x[3 * j + 1];
            const double dz = x[3 * i + 2] - x[3 * j + 2];
            const double s = dx * dx + dy * dy + dz * dz + eps2;
            const double inv_r = 1.0 / sqrt(s);            /* s^(-1/2) */
            const double inv_r3 = inv_r * inv_r * inv_r;   /* s^(-3/2) */
            pot += m[j] * inv_r;
            ax += m[j] * dx * inv_r3;
            ay += m[j] * dy * inv_r3;
            az += m[j] * dz * inv_r3;
        }
        if (a) {
            a[3 * r + 0] = ax;
            a[3 * r + 1] = ay;
            a[3 * r + 2] = az;
        }
        if (p)
            p[r] = pot;
    }
}

/* All rows: the full N^2 evaluation of Eq. (gravity). */
void oracle_forces(const double *x, const double *m, int64_t n, double eps2,
                   double *a, double *p)
{
    oracle_forces_rows(x, m, n, eps2, NULL, n, a, p);
}

/*
 * Eq. (gravity) applied to independent systems: system s holds particles
 * [offsets[s], offsets[s+1]) and interacts only with itself.
 */
void oracle_forces_batched(const int64_t *offsets, int64_t num_systems,
                           const double *x, const double *m, double eps2,
                           double *a, double *p)
{
    for (int64_t s = 0; s < num_systems; ++s) {
        const int64_t lo = offsets[s], cnt = offsets[s + 1] - offsets[s];
        oracle_forces_rows(x + 3 * lo, m + lo, cnt, eps2, NULL, cnt,
                           a + 3 * lo, p + lo);
    }
}

/*
 * Vector-Jacobian product of Eq. (gravity).
 *
 * For upstream weights w_i (on a_i) and v_i (on p_i) the scalar
 *     L = sum_i w_i . a_i + v_i p_i = sum_{i != j} T_ij,
 *     T_ij = m_j [ (w_i . d_ij) s_ij^(-3/2) + v_i s_ij^(-1/2) ],
 *     d_ij = x_i - x_j,  s_ij = |d_ij|^2 + eps^2,
 * depends on x_k through d_ij (d/dx_i = +1, d/dx_j = -1) and on m_k through
 * the factor m_j of the terms with j == k.  The chain rule gives
 *     dT/dd = m_j [ w_i s^(-3/2) - 3 (w_i . d) s^(-5/2) d - v_i s^(-3/2) d ],
 *     dL/dx_k = sum_{j != k} dT_kj/dd  -  sum_{i != k} dT_ik/dd,
 *     dL/dm_k = sum_{i != k} [ (w_i . d_ik) s_ik^(-3/2) + v_i s_ik^(-1/2) ].
 * Each output row is gathered in index order (deterministic).
 *
 * w: [n,3] or NULL (zero), v: [n] or NULL (zero).
 * gx: [n,3] or NULL, gm: [n] or NULL.  Outputs are overwritten.
 */
static void pair_grad_d(const double *d, double inv_r, double mj, const double *wi,
                        double vi, double *out)
{
    const double inv_r3 = inv_r * inv_r * inv_r;
    const double inv_r5 = inv_r3 * inv_r * inv_r;
    const double wd = wi[0] * d[0] + wi[1] * d[1] + wi[2] * d[2];
    for (int c = 0; c < 3; ++c)
        out[c] = mj * (wi[c] * inv_r3 - 3.0 * wd * inv_r5 * d[c] - vi * inv_r3 * d[c]);
}

void oracle_forces_vjp(const double *x, const double *m, int64_t n, double eps2,
                       const double *w, const double *v, double *gx, double *gm)
{
    int64_t k;
#pragma omp parallel for schedule(dynamic, 8)
    for (k = 0; k < n; ++k) {
        double acc[3] = {0.0, 0.0, 0.0};
        double accm = 0.0;
        const double zero3[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == k)
                continue;
            double d[3], g[3];
            /* term T_kj: x_k enters as x_i (sign +1) */
            d[0] = x[3 * k + 0] - x[3 * j + 0];
            d[1] = x[3 * k + 1] - x[3 * j + 1];
            d[2] = x[3 * k + 2] - x[3 * j + 2];
            const double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
            const double inv_r = 1.0 / sqrt(s);
            pair_grad_d(d, inv_r, m[j], w ? w + 3 * k : zero3, v ? v[k] : 0.0, g);
            acc[0] += g[0];
            acc[1] += g[1];
            acc[2] += g[2];
            /* term T_jk: x_k enters as x_j (sign -1); d_jk = -d */
            double dj[3] = {-d[0], -d[1], -d[2]};
            pair_grad_d(dj, inv_r, m[k], w ? w + 3 * j : zero3, v ? v[j] : 0.0, g);
            acc[0] -= g[0];
            acc[1] -= g[1];
            acc[2] -= g[2];
            /* dT_jk/dm_k */
            const double *wj = w ? w + 3 * j : zero3;
            const double wd = wj[0] * dj[0] + wj[1] * dj[1] + wj[2] * dj[2];
            accm += wd * inv_r * inv_r * inv_r + (v ? v[j] : 0.0) * inv_r;
        }
        if (gx) {
            gx[3 * k + 0] = acc[0];
            gx[3 * k + 1] = acc[1];
            gx[3 * k + 2] = acc[2];
        }
        if (gm)
            gm[k] = accm;
    }
}

/* y += alpha * x over a flat array of len doubles. */
static void axpy(int64_t len, double alpha, const double *xv, double *y)
{
    for (int64_t t = 0; t < len; ++t)
        y[t] += alpha * xv[t];
}

/*
 * Leap-frog integration, Eqs. (1)-(3) with the algorithm of Sec. III
 * (one force evaluation per step, reused by the next step's first kick).
 * The paper's a of Eq. (gravity) points away from the attracting body, so
 * the physical acceleration fed to Eqs. (1) and (3) is g = -a.
 *     v_half = v + (dt/2) g(x);  x' = x + dt v_half;  v' = v_half + (dt/2) g(x')
 * (Eq. (2), x + v dt + a dt^2/2, equals x + dt v_half.)
 *
 * x, v: [n,3] in/out (state after `steps` steps).  traj: optional
 * [(steps+1), n, 3] receiving x at every step (x_0 first).  g_work: [n,3]
 * scratch; on return it holds g at the final positions.
 */
void oracle_leapfrog(double *x, double *v, const double *m, int64_t n, double eps2,
                     double dt, int64_t steps, double *traj, double *g_work)
{
    const int64_t len = 3 * n;
    oracle_forces(x, m, n, eps2, g_work, NULL);
    for (int64_t t = 0; t < len; ++t)
        g_work[t] = -g_work[t];
    if (traj)
        memcpy(traj, x, sizeof(double) * len);
    for (int64_t s = 0; s < steps; ++s) {
        axpy(len, 0.5 * dt, g_work, v);        /* Eq. (1) */
        axpy(len, dt, v, x);                   /* Eq. (2) */
        oracle_forces(x, m, n, eps2, g_work, NULL);
        for (int64_t t = 0; t < len; ++t)
            g_work[t] = -g_work[t];
        axpy(len, 0.5 * dt, g_work, v);        /* Eq. (3) */
        if (traj)
            memcpy(traj + (s + 1) * len, x, sizeof(double) * len);
    }
}
