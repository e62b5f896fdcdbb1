/*
 * Plain C oracle: blocked right-looking LU with partial pivoting (FP64).
 *
 * TEST INFRASTRUCTURE ONLY.  Used by the tests for sizes the Python oracle is too
 * slow for, and timed as the CPU baseline.  Shares no code with the HIP library.
 *
 * Storage: row-major, element (i, j) at A[i*lda + j], lda >= n.
 * Algorithm: Fig. "LU" (right) of the paper, the blocked RL variant, with the
 * panel factored by the unblocked RL algorithm (Fig. "LU", left):
 *   RL1  [A11; A21] := LU_unb([A11; A21])   -- per column: first index of the
 *        largest |value| from the diagonal down, interchange of the panel rows,
 *        rl1 a21 := a21 / alpha11, rl2 A22 := A22 - a21 a12^T
 *        (the panel's interchanges are then applied to every other column)
 *   RL2  A12 := trilu(A11)^{-1} A12          -- forward substitution
 *   RL3  A22 := A22 - A21 A12
 * A zero pivot sets info to its 1-based column (first occurrence) and skips rl1.
 * ipiv receives 1-based row indices (LAPACK convention).
 * Loops are plain; OpenMP only splits independent rows or columns.
 */
#include <math.h>
#include <stdint.h>

static void swap_rows(double *A, long lda, int r, int p, int c0, int c1)
{
    if (r == p) return;
    double *x = A + (long)r * lda, *y = A + (long)p * lda;
    for (int c = c0; c < c1; ++c) {
        double t = x[c];
        x[c] = y[c];
        y[c] = t;
    }
}

int oracle_dgetrf_rl(int m, int n, double *A, int lda, int nb, int32_t *ipiv)
{
    int mn = m < n ? m : n;
    int info = 0;
    long ld = lda;
    if (nb < 1) nb = 1;
    for (int j = 0; j < mn; j += nb) {
        int b = mn - j < nb ? mn - j : nb;
        /* RL1: unblocked LU of the panel rows j..m-1, columns j..j+b-1 */
        for (int c = 0; c < b; ++c) {
            int col = j + c;
            int p = col;
            double best = fabs(A[col * ld + col]);
            for (int i = col + 1; i < m; ++i) {
                double v = fabs(A[i * ld + col]);
                if (v > best) { best = v; p = i; }
            }
            ipiv[col] = p + 1;
            swap_rows(A, ld, col, p, j, j + b);
            double alpha = A[col * ld + col];
            if (alpha != 0.0) {
                for (int i = col + 1; i < m; ++i) A[i * ld + col] = A[i * ld + col] / alpha;
            } else if (info == 0) {
                info = col + 1;
            }
            #pragma omp parallel for schedule(static) if ((long)(m - col) * (b - c) > 65536)
            for (int i = col + 1; i < m; ++i) {
                double l = A[i * ld + col];
                for (int cc = col + 1; cc < j + b; ++cc) A[i * ld + cc] -= l * A[col * ld + cc];
            }
        }
        /* the panel's interchanges, applied to the columns left and right of it */
        for (int c = 0; c < b; ++c) {
            int r = j + c, p = ipiv[j + c] - 1;
            swap_rows(A, ld, r, p, 0, j);
            swap_rows(A, ld, r, p, j + b, n);
        }
        /* RL2: forward substitution with trilu(A11) on A12 */
        #pragma omp parallel for schedule(static)
        for (int cc = j + b; cc < n; ++cc) {
            for (int r = 1; r < b; ++r) {
                double s = A[(long)(j + r) * ld + cc];
                for (int t = 0; t < r; ++t) s -= A[(long)(j + r) * ld + (j + t)] * A[(long)(j + t) * ld + cc];
                A[(long)(j + r) * ld + cc] = s;
            }
        }
        /* RL3: A22 -= A21 A12 */
        #pragma omp parallel for schedule(static)
        for (int i = j + b; i < m; ++i) {
            double *ci = A + (long)i * ld;
            for (int t = 0; t < b; ++t) {
                double a = ci[j + t];
                const double *bt = A + (long)(j + t) * ld;
                for (int cc = j + b; cc < n; ++cc) ci[cc] -= a * bt[cc];
            }
        }
    }
    return info;
}
