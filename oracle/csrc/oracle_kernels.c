/*
 * ORACLE -- test infrastructure only. Plain FP64 C, no GPU code, shared with
 * nothing in the product library. Only tests/, the smoke check and the CPU
 * baseline leg of the benchmark call into it.
 *
 *   oracle_jacobi_eig      cyclic-by-row two-sided Jacobi eigensolver for a
 *                          dense symmetric matrix (Golub & Van Loan, Matrix
 *                          Computations, Sec. 8.5, symmetric Schur 2x2 step).
 *   oracle_project_jacobi  PSD projection by the closed form of Section 1,
 *                          eq. (3): Q diag(max(lambda_i, 0)) Q^T.
 *   oracle_efloat          the discretised error of Section 3.3, eq. (12):
 *                          maximum pointwise error of a composite odd filter
 *                          over every float32 value in [-1, 1].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* A (n*n, row-major, symmetric) is overwritten; on return its diagonal holds
 * the eigenvalues, copied to w. V (n*n row-major) receives the eigenvectors as
 * columns. Returns the number of sweeps used, or -1 if max_sweeps was hit. */
int oracle_jacobi_eig(int n, double *A, double *V, double *w, int max_sweeps,
                      double rel_tol) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    double fro2 = 0.0;
    for (size_t i = 0; i < (size_t)n * n; ++i) fro2 += A[i] * A[i];
    const double stop = rel_tol * sqrt(fro2);
    int sweep;
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        double off2 = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q)
                if (p != q) off2 += A[(size_t)p * n + q] * A[(size_t)p * n + q];
        if (sqrt(off2) <= stop) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p];
                const double aqq = A[(size_t)q * n + q];
                /* symmetric Schur decomposition of the (p,q) 2x2 block */
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                              : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                /* A <- A J  (columns p, q) */
                for (int k = 0; k < n; ++k) {
                    double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                /* A <- J^T A  (rows p, q) */
                for (int k = 0; k < n; ++k) {
                    double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                A[(size_t)p * n + q] = 0.0;
                A[(size_t)q * n + p] = 0.0;
                /* V <- V J */
                for (int k = 0; k < n; ++k) {
                    double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
    return sweep < max_sweeps ? sweep : -1;
}

/* out = Q diag(max(w,0)) Q^T for the symmetric X (n*n row-major, FP64).
 * Returns the Jacobi sweep count (or -1 when not converged). */
int oracle_project_jacobi(int n, const double *X, double *out, double *eigvals) {
    double *A = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *V = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    memcpy(A, X, sizeof(double) * (size_t)n * n);
    int sweeps = oracle_jacobi_eig(n, A, V, w, 60, 1e-15);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) {
                double lk = w[k] > 0.0 ? w[k] : 0.0;
                acc += V[(size_t)i * n + k] * lk * V[(size_t)j * n + k];
            }
            out[(size_t)i * n + j] = acc;
        }
    if (eigvals) memcpy(eigvals, w, sizeof(double) * (size_t)n);
    free(A); free(V); free(w);
    return sweeps;
}

/* Composite odd filter p(x) = f_T o ... o f_1 (x), f_t(x) = a x + b x^3 + c x^5,
 * coefficient rows abc[3t..3t+2] (rescale already folded in by the caller). */
static double composite(double x, int T, const double *abc) {
    for (int t = 0; t < T; ++t) {
        const double x2 = x * x;
        x = x * (abc[3 * t] + x2 * (abc[3 * t + 1] + x2 * abc[3 * t + 2]));
    }
    return x;
}

/* Largest |x p(x) - |x|| over every float32 x in [-1, 1]. By oddness of p the
 * error at -x equals the error at x, so only the 0x00000000..0x3F800000 bit
 * patterns are visited. x p(x) - |x| is twice the ReLU error of
 * f(x) = x (1 + p(x)) / 2; the caller halves it for the literal definition.
 * argmax_out receives the maximising x. */
double oracle_efloat(int T, const double *abc, double *argmax_out) {
    const uint32_t last = 0x3F800000u;
    double best = 0.0, best_x = 0.0;
#pragma omp parallel
    {
        double lb = 0.0, lx = 0.0;
#pragma omp for schedule(static)
        for (int64_t b = 0; b <= (int64_t)last; ++b) {
            uint32_t bits = (uint32_t)b;
            float xf;
            memcpy(&xf, &bits, 4);
            const double x = (double)xf;
            const double e = fabs(x * composite(x, T, abc) - x);
            if (e > lb) { lb = e; lx = x; }
        }
#pragma omp critical
        {
            if (lb > best || (lb == best && lx < best_x)) { best = lb; best_x = lx; }
        }
    }
    if (argmax_out) *argmax_out = best_x;
    return best;
}
