/*
 * CPU oracle for the state-vector sweep (TEST INFRASTRUCTURE ONLY).
 *
 * Plain, slow, complex128 gate-by-gate simulator.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load this
 * library.  It shares no code, header or constant with the GPU library.
 *
 * What it follows:
 *  - Section 2 (preliminaries): a single-qubit gate U = [[a,b],[c,d]] on
 *    qubit k updates, for every index i whose bit k is 0, the pair
 *    (alpha_i, alpha_{i+2^k}) by the 2x2 matrix-vector product.  Qubit k is
 *    index bit k (U acts as I^{n-k-1} (x) U (x) I^{k}).
 *  - Section 2 (preliminaries): CZ is the controlled-Z; the target picks up
 *    the factor -1 exactly when control and target bits are both 1.
 *  - Norm: sum of |alpha|^2 with Neumaier's compensated summation.
 *
 * State layout: 2^n complex128 amplitudes as interleaved (re, im) doubles.
 */
#include <stddef.h>
#include <stdint.h>
#include <math.h>

/* Apply one single-qubit gate m = {a.re, a.im, b.re, b.im, c.re, c.im, d.re, d.im}. */
void oref_apply_1q(double *psi, int n, int k, const double *m)
{
    const int64_t dim = (int64_t)1 << n;
    const int64_t stride = (int64_t)1 << k;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        if (i & stride)
            continue;
        const int64_t j = i + stride;
        const double xr = psi[2 * i], xi = psi[2 * i + 1];
        const double yr = psi[2 * j], yi = psi[2 * j + 1];
        /* x' = a x + b y ; y' = c x + d y (complex) */
        psi[2 * i]     = m[0] * xr - m[1] * xi + m[2] * yr - m[3] * yi;
        psi[2 * i + 1] = m[0] * xi + m[1] * xr + m[2] * yi + m[3] * yr;
        psi[2 * j]     = m[4] * xr - m[5] * xi + m[6] * yr - m[7] * yi;
        psi[2 * j + 1] = m[4] * xi + m[5] * xr + m[6] * yi + m[7] * yr;
    }
}

/* Controlled-Z on qubits q0, q1: negate every amplitude with both bits set. */
void oref_apply_cz(double *psi, int n, int q0, int q1)
{
    const int64_t dim = (int64_t)1 << n;
    const int64_t m0 = (int64_t)1 << q0, m1 = (int64_t)1 << q1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        if ((i & m0) && (i & m1)) {
            psi[2 * i] = -psi[2 * i];
            psi[2 * i + 1] = -psi[2 * i + 1];
        }
    }
}

/*
 * Run a gate list in order.  Gate g acts on q0[g]; if q1[g] >= 0 it is a CZ
 * on (q0[g], q1[g]), otherwise the single-qubit matrix mats[8g .. 8g+7].
 */
void oref_run(double *psi, int n, int64_t n_gates, const int32_t *q0,
              const int32_t *q1, const double *mats)
{
    for (int64_t g = 0; g < n_gates; ++g) {
        if (q1[g] >= 0)
            oref_apply_cz(psi, n, q0[g], q1[g]);
        else
            oref_apply_1q(psi, n, q0[g], mats + 8 * g);
    }
}

/* Neumaier-compensated sum of |psi_i|^2 over len amplitudes. */
double oref_norm2(const double *psi, int64_t len)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        const double v = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        const double t = s + v;
        if (fabs(s) >= fabs(v))
            c += (s - t) + v;
        else
            c += (v - t) + s;
        s = t;
    }
    return s + c;
}

/* |0...0>: zero everything, amplitude 0 = 1. */
void oref_zero_state(double *psi, int n)
{
    const int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < 2 * dim; ++i)
        psi[i] = 0.0;
    psi[0] = 1.0;
}

/* Number of OpenMP threads a parallel region will use (for reporting). */
int oref_threads(void)
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
