/* Largest singular value of many small square blocks, for the seeded input
 * generators: s = sqrt(lambda_max(J^T J)), lambda_max by the cyclic Jacobi
 * eigenvalue method (rotations until the off-diagonal mass is negligible).
 * OpenMP over blocks.  Input generation only; no solver arithmetic. */
#include <math.h>

static double lambda_max_sym(int n, double a[8][8])
{
    for (int sweep = 0; sweep < 64; sweep++) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < n; p++) {
            diag += a[p][p] * a[p][p];
            for (int q = p + 1; q < n; q++) off += a[p][q] * a[p][q];
        }
        if (off <= 1e-32 * diag || off == 0.0) break;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                if (a[p][q] == 0.0) continue;
                double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; k++) {           /* columns p, q */
                    double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; k++) {           /* rows p, q */
                    double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
            }
    }
    double m = a[0][0];
    for (int p = 1; p < n; p++) if (a[p][p] > m) m = a[p][p];
    return m;
}

void spectral_norms(long nb, int n, const double *J, double *out)
{
#pragma omp parallel for schedule(static)
    for (long f = 0; f < nb; f++) {
        const double *B = J + f * n * n;
        double g[8][8];
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                double s = 0.0;
                for (int k = 0; k < n; k++) s += B[k * n + i] * B[k * n + j];
                g[i][j] = s;
            }
        double l = lambda_max_sym(n, g);
        out[f] = sqrt(l > 0.0 ? l : 0.0);
    }
}
