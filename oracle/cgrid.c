/*
 * Fast-FCM spreading in plain C, FP64 -- TEST INFRASTRUCTURE ONLY.
 *
 * The same operator as oracle/fastfcm.py:spread, written as straight loops so
 * that the oracle can spread the particles of the largest request-stream
 * problems (10^5 particles, 432^3 grids, M_G = 16) in seconds rather than
 * minutes.  Nothing is blocked, fused or factorised: every support point of
 * every particle evaluates the kernels from their definitions.
 *
 *   J~^dagger[F] (Sec. 3.1, eq. force_kernel_mod): the modified kernel
 *     Delta~(d; Sigma) = Delta(d; Sigma) [1 + (sigma^2 - Sigma^2)/2
 *                         (|d|^2/Sigma^4 - 3/Sigma^2)]
 *     (the operator (1 + ((sigma^2 - Sigma^2)/2) lap) applied to the Gaussian,
 *     Sec. 3);
 *   N~^dagger[T] (Sec. 3.4, eq. torque_kernel_mod): -(1/2) T x grad Delta(d;
 *     Sigma_D) = (1 / (2 Sigma_D^2)) Delta(d; Sigma_D) (T x d);
 *   Delta(r; s) = (2 pi s^2)^(-3/2) exp(-r^2 / (2 s^2)) (Sec. 2).
 *
 * Grid conventions (the paper leaves them open; the same readings as the
 * numpy oracle): grid points at (i, j, k) dx on [0, L); the M_G support points
 * of a coordinate Y along an axis are start .. start + M_G - 1 (mod M) with
 * start = floor(Y/dx - M_G/2) + 1, displacement (start + j) dx - Y.
 *
 * Layout: positions, forces and torques are N x 3 (x, y, z interleaved); the
 * field is 3 components of Mx x My x Mz points with z fastest, i.e. the numpy
 * array of shape (3, Mx, My, Mz).  The field is accumulated into (the caller
 * clears it first).  T may be NULL (no torques).
 *
 * Built with gcc (no fast-math), loaded by oracle/cgrid.py through ctypes.
 */
#include <math.h>
#include <stdint.h>

static const double kPi = 3.14159265358979323846;

/* Python's float modulo: the result has the sign of the divisor. */
static double pymod(double a, double L) {
    double r = fmod(a, L);
    if (r != 0.0 && ((r < 0.0) != (L < 0.0))) r += L;
    return r;
}

static int64_t imod(int64_t j, int64_t M) {
    int64_t r = j % M;
    return r < 0 ? r + M : r;
}

/* Delta at squared distance r2 for width s, with norm = (2 pi s^2)^(-3/2) */
static double gaussian(double r2, double s, double norm) { return norm * exp(-r2 / (2.0 * s * s)); }

int oracle_spread(int64_t N, const double* Y, const double* F, const double* T, int Mx, int My,
                  int Mz, double Lx, double Ly, double Lz, int MG, double sigma, double Sigma,
                  double SigmaD, double* f) {
    if (N < 0 || Mx <= 0 || My <= 0 || Mz <= 0 || MG <= 0 || MG > 64) return -1;
    const double L[3] = {Lx, Ly, Lz};
    const int64_t Mv[3] = {Mx, My, Mz};
    const double dx = Lx / Mx;
    const int64_t M3 = (int64_t)Mx * My * Mz;
    const double S2 = Sigma * Sigma;
    const double c = 0.5 * (sigma * sigma - S2);
    const double normS = pow(2.0 * kPi * S2, -1.5);
    const double normD = pow(2.0 * kPi * SigmaD * SigmaD, -1.5);
    int64_t idx[3][64];
    double d[3][64];
    for (int64_t n = 0; n < N; ++n) {
        for (int a = 0; a < 3; ++a) {
            double y = pymod(Y[3 * n + a], L[a]);
            if (y >= L[a]) y = 0.0;
            const int64_t start = (int64_t)floor(y / dx - MG / 2.0) + 1;
            for (int j = 0; j < MG; ++j) {
                idx[a][j] = imod(start + j, Mv[a]);
                d[a][j] = (double)(start + j) * dx - y;
            }
        }
        const double* Fn = F + 3 * n;
        const double* Tn = T ? T + 3 * n : 0;
        for (int i = 0; i < MG; ++i)
            for (int j = 0; j < MG; ++j)
                for (int k = 0; k < MG; ++k) {
                    const double ddx = d[0][i], ddy = d[1][j], ddz = d[2][k];
                    const double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                    const double gS = gaussian(r2, Sigma, normS);
                    const double dmod = gS * (1.0 + c * (r2 / (S2 * S2) - 3.0 / S2));
                    double v0 = dmod * Fn[0], v1 = dmod * Fn[1], v2 = dmod * Fn[2];
                    if (Tn) {
                        /* one width for both kernels: the same Gaussian */
                        const double gD = SigmaD == Sigma ? gS : gaussian(r2, SigmaD, normD);
                        const double dtor = gD / (2.0 * SigmaD * SigmaD);
                        v0 += dtor * (Tn[1] * ddz - Tn[2] * ddy);
                        v1 += dtor * (Tn[2] * ddx - Tn[0] * ddz);
                        v2 += dtor * (Tn[0] * ddy - Tn[1] * ddx);
                    }
                    const int64_t g = (idx[0][i] * Mv[1] + idx[1][j]) * Mv[2] + idx[2][k];
                    f[g] += v0;
                    f[M3 + g] += v1;
                    f[2 * M3 + g] += v2;
                }
    }
    return 0;
}
