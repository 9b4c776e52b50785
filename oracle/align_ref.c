/*
 * FP64 reference for the optimal starting point and rotation of two closed
 * planar curves (Dogan, Bernal, Hagwood, "FFT-based alignment of 2d closed
 * curves", section 2).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * library itself never links, calls or includes anything from here, and this
 * file includes nothing from the library.
 *
 * Notation follows section 2 of the paper:
 *   - a curve is given by n distinct nodes beta^l, l = 0..n-1, uniformly
 *     parametrized on [0,1) (the paper lists n+1 points with first == last
 *     and uses h = 1/(number of listed points - 1), i.e. h = 1/n here);
 *   - for a start index m (t0 = t_m = m/n) the shifted curve is
 *     beta2^{l (+) m} = beta2[(l + m) mod n]   (definition above Eq. disc-energy);
 *   - A_kj(t_m) = sum_l beta1_k^l beta2_j^{l (+) m}         (Eq. A-mtx);
 *   - R(theta) = [[cos, sin], [-sin, cos]]  (the rotation of section 2);
 *   - the optimal R for a fixed m maximizes tr(R A^T)  (Algorithm 1);
 *   - E^h(t_m, R) = h sum_l || beta1^l - R beta2^{l (+) m} ||^2  (Eq. disc-energy).
 *
 * The per-shift optimum is written out as the plain maximisation of
 * tr(R(theta) A^T) over theta: with R as above,
 *   tr(R A^T) = cos(theta) (A11 + A22) + sin(theta) (A12 - A21),
 * a linear form in (cos, sin) whose maximum over the circle is
 *   T = hypot(A11 + A22, A12 - A21)  at  theta = atan2(A12 - A21, A11 + A22).
 * The SVD route of Algorithm 1 reaches the same R; the tests pin this file
 * against a library SVD with the determinant test and against brute force
 * over a fine angle grid.
 *
 * The outer loop over every start index is the O(n^2) method described in
 * section 2 just before the convolution-theorem argument.  Algorithm 2 returns
 * the start index with the highest value and is silent on exact ties; this
 * oracle keeps, among indices whose values are exactly equal, the one whose
 * correlation shift s = (n - m) mod n is smallest (the library's convention
 * for reporting the optimum as a shift).  The scan therefore visits the
 * indices in the order m = 0, n-1, n-2, ..., 1 and keeps the first highest.
 *
 * Build: gcc -O3 -fopenmp -shared -fPIC align_ref.c -o liboracle_align.so -lm
 * (no fast-math: the reference must round like the plain formulas).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* A(t_m), Eq. A-mtx: four real sums over l of products of node coordinates. */
static void a_matrix(const double* b1, const double* b2, int n, int m,
                     double* a11, double* a12, double* a21, double* a22)
{
    double s11 = 0.0, s12 = 0.0, s21 = 0.0, s22 = 0.0;
    for (int l = 0; l < n; ++l) {
        int lm = (l + m) % n;
        double x1 = b1[2 * l], y1 = b1[2 * l + 1];
        double x2 = b2[2 * lm], y2 = b2[2 * lm + 1];
        s11 += x1 * x2;
        s12 += x1 * y2;
        s21 += y1 * x2;
        s22 += y1 * y2;
    }
    *a11 = s11; *a12 = s12; *a21 = s21; *a22 = s22;
}

/* Optimal rotation angle and the value of tr(R A^T) at the optimum. */
static void best_rotation(double a11, double a12, double a21, double a22,
                          double* theta, double* trace)
{
    double c = a11 + a22;      /* coefficient of cos(theta) */
    double s = a12 - a21;      /* coefficient of sin(theta) */
    *trace = hypot(c, s);
    *theta = (c == 0.0 && s == 0.0) ? 0.0 : atan2(s, c);
}

/*
 * Per-start-index scores.  For m = 0..n-1:
 *   T[m]     = max_R tr(R A(t_m)^T)
 *   theta[m] = the maximising angle, paper convention (R(theta) above)
 * b1, b2: interleaved (x, y) doubles, n nodes each.  Either output may be NULL.
 */
void oracle_shift_scores(const double* b1, const double* b2, int n,
                         double* T, double* theta)
{
    for (int m = 0; m < n; ++m) {
        double a11, a12, a21, a22, th, tr;
        a_matrix(b1, b2, n, m, &a11, &a12, &a21, &a22);
        best_rotation(a11, a12, a21, a22, &th, &tr);
        if (T) T[m] = tr;
        if (theta) theta[m] = th;
    }
}

/* The 2x2 matrix A(t_m) itself (row-major a11 a12 a21 a22). */
void oracle_a_matrix(const double* b1, const double* b2, int n, int m, double* a)
{
    a_matrix(b1, b2, n, m, &a[0], &a[1], &a[2], &a[3]);
}

/* E^h(t_m, R(theta)), Eq. disc-energy, summed directly (no expansion). */
double oracle_energy(const double* b1, const double* b2, int n, int m, double theta)
{
    double c = cos(theta), s = sin(theta);
    double e = 0.0;
    for (int l = 0; l < n; ++l) {
        int lm = (l + m) % n;
        double x2 = b2[2 * lm], y2 = b2[2 * lm + 1];
        /* R(theta) beta2 with R = [[c, s], [-s, c]] */
        double rx = c * x2 + s * y2;
        double ry = -s * x2 + c * y2;
        double dx = b1[2 * l] - rx, dy = b1[2 * l + 1] - ry;
        e += dx * dx + dy * dy;
    }
    return e / (double)n;
}

/* ||beta||^2 with the same trapezoid weight h = 1/n. */
double oracle_sqnorm(const double* b, int n)
{
    double e = 0.0;
    for (int l = 0; l < n; ++l) e += b[2 * l] * b[2 * l] + b[2 * l + 1] * b[2 * l + 1];
    return e / (double)n;
}

/*
 * Start index of the largest value among v[m], m = 0..n-1, visiting the
 * indices by increasing shift s = (n - m) mod n and keeping the first highest,
 * so that exact ties go to the smallest s.
 */
int oracle_best_index(const double* v, int n)
{
    int best = 0;
    for (int s = 1; s < n; ++s) {
        int m = n - s;
        if (v[m] > v[best]) best = m;
    }
    return best;
}

/*
 * The slow method for one pair: loop over every start index, optimal rotation
 * per index, keep the best, then evaluate E^h there.  Outputs (paper notation):
 *   *m_best, *theta_best, *e_best, *t_best; T and theta arrays optional.
 */
void oracle_align_pair(const double* b1, const double* b2, int n,
                       int* m_best, double* theta_best, double* e_best,
                       double* t_best, double* T, double* theta)
{
    double* Tloc = T ? T : (double*)malloc(sizeof(double) * (size_t)n);
    double* Hloc = theta ? theta : (double*)malloc(sizeof(double) * (size_t)n);
    oracle_shift_scores(b1, b2, n, Tloc, Hloc);
    int m = oracle_best_index(Tloc, n);
    *m_best = m;
    *theta_best = Hloc[m];
    *t_best = Tloc[m];
    *e_best = oracle_energy(b1, b2, n, m, Hloc[m]);
    if (!T) free(Tloc);
    if (!theta) free(Hloc);
}

/*
 * Batch of pairs given as complex64 (float x, float y) nodes, [num_pairs][n]
 * each, upcast to double before any arithmetic.  Pairs are independent; the
 * loop over pairs is spread over `nthreads` OpenMP threads (<= 0: runtime
 * default).  Returns the number of threads used.
 */
int oracle_align_batch_f32(const float* z1, const float* z2, int64_t num_pairs, int n,
                           int nthreads, int32_t* m_out, double* theta_out,
                           double* e_out, double* t_out)
{
    int used = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
        double* b1 = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        double* b2 = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        double* T = (double*)malloc(sizeof(double) * (size_t)n);
        double* H = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < num_pairs; ++p) {
            const float* s1 = z1 + (size_t)p * 2 * (size_t)n;
            const float* s2 = z2 + (size_t)p * 2 * (size_t)n;
            for (int i = 0; i < 2 * n; ++i) { b1[i] = (double)s1[i]; b2[i] = (double)s2[i]; }
            int m; double th, e, t;
            oracle_align_pair(b1, b2, n, &m, &th, &e, &t, T, H);
            m_out[p] = m; theta_out[p] = th; e_out[p] = e; if (t_out) t_out[p] = t;
        }
        free(b1); free(b2); free(T); free(H);
    }
#else
    (void)nthreads;
    double* b1 = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    double* b2 = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    double* T = (double*)malloc(sizeof(double) * (size_t)n);
    double* H = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t p = 0; p < num_pairs; ++p) {
        const float* s1 = z1 + (size_t)p * 2 * (size_t)n;
        const float* s2 = z2 + (size_t)p * 2 * (size_t)n;
        for (int i = 0; i < 2 * n; ++i) { b1[i] = (double)s1[i]; b2[i] = (double)s2[i]; }
        int m; double th, e, t;
        oracle_align_pair(b1, b2, n, &m, &th, &e, &t, T, H);
        m_out[p] = m; theta_out[p] = th; e_out[p] = e; if (t_out) t_out[p] = t;
    }
    free(b1); free(b2); free(T); free(H);
#endif
    return used;
}

/*
 * The slow method over a batch of complex64 pairs (as oracle_align_batch_f32)
 * that also evaluates each pair at a start index chosen elsewhere: for pair p
 * the start index m_at = (n - shift_in[p]) mod n (shift_in holds correlation
 * shifts s, the library's reporting form).  Outputs per pair: the best index
 * and its value, angle and energy, the largest value over the other indices
 * (t2_out), and at m_at the value, angle and energy of Eq. disc-energy
 * (t_at, theta_at, e_at).  Nothing here changes what the slow method
 * computes; the extra outputs are the same per-index quantities read at a
 * second index.  Returns the number of threads used.
 */
int oracle_check_batch_f32(const float* z1, const float* z2, int64_t num_pairs, int n,
                           int nthreads, const int32_t* shift_in, int32_t* m_out,
                           double* theta_out, double* e_out, double* t_out, double* t2_out,
                           double* t_at, double* theta_at, double* e_at)
{
    int used = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
#endif
        double* b1 = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        double* b2 = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        double* T = (double*)malloc(sizeof(double) * (size_t)n);
        double* H = (double*)malloc(sizeof(double) * (size_t)n);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t p = 0; p < num_pairs; ++p) {
            const float* s1 = z1 + (size_t)p * 2 * (size_t)n;
            const float* s2 = z2 + (size_t)p * 2 * (size_t)n;
            for (int i = 0; i < 2 * n; ++i) { b1[i] = (double)s1[i]; b2[i] = (double)s2[i]; }
            int m; double th, e, t;
            oracle_align_pair(b1, b2, n, &m, &th, &e, &t, T, H);
            m_out[p] = m; theta_out[p] = th; e_out[p] = e; t_out[p] = t;
            double t2 = -1.0;
            for (int k = 0; k < n; ++k)
                if (k != m && T[k] > t2) t2 = T[k];
            t2_out[p] = t2;
            int sh = shift_in[p] % n;
            if (sh < 0) sh += n;
            const int ma = (n - sh) % n;
            t_at[p] = T[ma];
            theta_at[p] = H[ma];
            e_at[p] = oracle_energy(b1, b2, n, ma, H[ma]);
        }
        free(b1); free(b2); free(T); free(H);
#ifdef _OPENMP
    }
#endif
    return used;
}
