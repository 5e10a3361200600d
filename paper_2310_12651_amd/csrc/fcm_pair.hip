// Pairwise correction of fast FCM in FP64 (Sec. 4, pairwise correction;
// Sec. 3.2 eq. correction_VF; Sec. 3.4 eqs. correction_WF, correction_WT) and
// the self corrections of App. B.
//
// One thread per particle, in pair-cell order: it scans its own and the 26
// adjacent cells (cells are at least R_c wide, Sec. 4 spatial hashing),
// takes the minimum image of every candidate and, for r < R_c, adds
//   V_n     += C_VF(x) F_m + C_VT(x) T_m,   Omega_n += C_OF(x) F_m + C_OT(x) T_m
// with x = Y_n - Y_m.  Each ordered pair is evaluated by its own receiving
// particle, so no atomics are needed and the result is deterministic.
//
// The blocks, with xh = x/r and (-x cross) T = T x x:
//   C_VF = Avf I + Bvf xh xh^T    (S(sigma sqrt2) - S~ - (sigma^2-Sigma^2) Q(Sigma sqrt2)
//                                   - (sigma^2-Sigma^2)^2/4 T(Sigma sqrt2), Sec. 2.2, 3.2)
//   C_OF = C_VT = fof (-x cross)   (R(sqrt(sigma^2+sigma_D^2)) - R(sqrt(Sigma^2+Sigma_D^2))
//                                   - (sigma^2-Sigma^2)/2 K(sqrt(Sigma^2+Sigma_D^2)), Sec. 3.4)
//   C_OT = Aot I + Bot xh xh^T    ((P(sigma_D sqrt2) - P(Sigma_D sqrt2))/2, Sec. 3.4)
// The erf terms of the two widths are combined as erfc differences, which
// keeps their small difference accurate at large r.
#include "fcm_internal.h"

namespace fcm {

namespace {

__device__ inline double gauss3(double r2, double s2) {
    // (2 pi s2)^(-3/2) exp(-r2 / 2 s2)
    const double pi = 3.14159265358979323846;
    const double t = 2.0 * pi * s2;
    return exp(-0.5 * r2 / s2) / (t * sqrt(t));
}

struct Coef {
    double Avf, Bvf, fof, Aot, Bot;
};

__device__ inline Coef correction_coeffs(double r, const PairArgs& a) {
    const double pi = 3.14159265358979323846;
    const double eta = a.eta;
    const double sg2 = a.sigma * a.sigma, Sg2 = a.Sigma * a.Sigma;
    const double sD2 = a.sigmaD * a.sigmaD, SD2 = a.SigmaD * a.SigmaD;
    const double r2 = r * r, r3 = r2 * r;
    const double d = sg2 - Sg2;
    Coef c;
    // force-velocity: erf part = (E(r; sigma sqrt2) - E(r; Sigma sqrt2)) (G + sigma^2 lap G)
    {
        const double dE = erfc(r / (2.0 * a.Sigma)) - erfc(r / (2.0 * a.sigma));
        const double g1 = 1.0 / (8.0 * pi * eta * r);
        const double g3 = sg2 / (4.0 * pi * eta * r3);
        c.Avf = dE * (g1 + g3);
        c.Bvf = dE * (g1 - 3.0 * g3);
        const double s1 = 2.0 * sg2, s2 = 2.0 * Sg2;  // squared widths sigma sqrt2, Sigma sqrt2
        const double D1 = gauss3(r2, s1), D2 = gauss3(r2, s2);
        // S3(s1) - S3(s2), S3 = -(s^4 / 2 eta r^2) (I - 3 xh xh) Delta
        const double t3 = (s1 * s1 * D1 - s2 * s2 * D2) / (2.0 * eta * r2);
        c.Avf += -t3;
        c.Bvf += 3.0 * t3;
        // -(sigma^2 - Sigma^2) Q2(s2), Q2 = -(1/eta)[(1 + s^2/r^2) I - (1 + 3 s^2/r^2) xh xh] Delta
        c.Avf += d / eta * (1.0 + s2 / r2) * D2;
        c.Bvf += -d / eta * (1.0 + 3.0 * s2 / r2) * D2;
        // -(sigma^2 - Sigma^2)^2 / 4 T(s2), T = (1/eta s^2)[(2 - r^2/s^2) I + (r^2/s^2) xh xh] Delta
        const double tq = d * d / (4.0 * eta * s2) * D2;
        c.Avf += -tq * (2.0 - r2 / s2);
        c.Bvf += -tq * (r2 / s2);
    }
    // rotation-force: R(sa) - R(sb) - (d/2) K(sb)
    {
        const double sa = sg2 + sD2, sb = Sg2 + SD2;
        const double dE = erfc(r / sqrt(2.0 * sb)) - erfc(r / sqrt(2.0 * sa));
        const double Da = gauss3(r2, sa), Db = gauss3(r2, sb);
        c.fof = (dE - 4.0 * pi * r * (sa * Da - sb * Db)) / (8.0 * pi * eta * r3) +
                d * Db / (4.0 * eta * sb);
    }
    // rotation-torque: (P(sigma_D sqrt2) - P(Sigma_D sqrt2)) / 2
    {
        const double sc = 2.0 * sD2, sd = 2.0 * SD2;
        const double dE = erfc(r / (2.0 * a.SigmaD)) - erfc(r / (2.0 * a.sigmaD));
        const double Dc = gauss3(r2, sc), Dd = gauss3(r2, sd);
        c.Aot = 0.5 * (-dE / (8.0 * pi * eta * r3) + ((sc + r2) * Dc - (sd + r2) * Dd) / (2.0 * eta * r2));
        c.Bot = 0.5 * (3.0 * dE / (8.0 * pi * eta * r3) -
                       ((3.0 * sc + r2) * Dc - (3.0 * sd + r2) * Dd) / (2.0 * eta * r2));
    }
    return c;
}

constexpr int kPairThreads = 256;
constexpr int kHitBuf = 16;

// add the corrections from one neighbour m at x = Y_n - Y_m (r^2 = r2 < R_c^2)
__device__ inline void add_pair(double x0, double x1, double x2, double r2, const PairRec& o,
                                const PairArgs& a, double* v, double* w) {
    const double F0 = o.F[0], F1 = o.F[1], F2 = o.F[2];
    const double T0 = o.T[0], T1 = o.T[1], T2 = o.T[2];
    const double r = sqrt(r2);
    if (r < 1e-3 * a.sigma) {
        // coincident centres: the r -> 0 limits (App. B)
        v[0] += a.selfVF * F0;
        v[1] += a.selfVF * F1;
        v[2] += a.selfVF * F2;
        w[0] += a.selfOT * T0;
        w[1] += a.selfOT * T1;
        w[2] += a.selfOT * T2;
        return;
    }
    const Coef c = correction_coeffs(r, a);
    const double h0 = x0 / r, h1 = x1 / r, h2 = x2 / r;
    const double hF = h0 * F0 + h1 * F1 + h2 * F2;
    const double hT = h0 * T0 + h1 * T1 + h2 * T2;
    // V += Avf F + Bvf xh (xh.F) + fof (T x x)
    v[0] += c.Avf * F0 + c.Bvf * h0 * hF + c.fof * (T1 * x2 - T2 * x1);
    v[1] += c.Avf * F1 + c.Bvf * h1 * hF + c.fof * (T2 * x0 - T0 * x2);
    v[2] += c.Avf * F2 + c.Bvf * h2 * hF + c.fof * (T0 * x1 - T1 * x0);
    // Omega += fof (F x x) + Aot T + Bot xh (xh.T)
    w[0] += c.fof * (F1 * x2 - F2 * x1) + c.Aot * T0 + c.Bot * h0 * hT;
    w[1] += c.fof * (F2 * x0 - F0 * x2) + c.Aot * T1 + c.Bot * h1 * hT;
    w[2] += c.fof * (F0 * x1 - F1 * x0) + c.Aot * T2 + c.Bot * h2 * hT;
}

// The candidate scan touches only the compact positions; the pairs found are
// buffered per lane and evaluated together, so the expensive FP64 body runs
// with the wavefront converged instead of once per candidate position.
__global__ __launch_bounds__(kPairThreads) void k_pair(const double4* __restrict__ pos4,
                                                       const PairRec* __restrict__ rec,
                                                       const int* __restrict__ cell_start,
                                                       PairArgs a, double* __restrict__ V,
                                                       double* __restrict__ W) {
    __shared__ int hits[kPairThreads][kHitBuf + 1];
    const int j = xcd_remap(blockIdx.x, gridDim.x) * kPairThreads + threadIdx.x;
    if (j >= a.N) return;
    int* hb = hits[threadIdx.x];
    const PairRec me = rec[j];
    const double4 mp = pos4[j];
    double v[3] = {a.selfVF * me.F[0], a.selfVF * me.F[1], a.selfVF * me.F[2]};
    double w[3] = {a.selfOT * me.T[0], a.selfOT * me.T[1], a.selfOT * me.T[2]};
    const double L = a.L, iL = 1.0 / a.L;
    auto flush = [&](int n) {
        for (int h = 0; h < n; ++h) {
            const int q = hb[h];
            const double4 op = pos4[q];
            double x0 = mp.x - op.x, x1 = mp.y - op.y, x2 = mp.z - op.z;
            x0 -= L * rint(x0 * iL);
            x1 -= L * rint(x1 * iL);
            x2 -= L * rint(x2 * iL);
            add_pair(x0, x1, x2, x0 * x0 + x1 * x1 + x2 * x2, rec[q], a, v, w);
        }
    };
    if (a.with_pairs) {
        const int m = a.m;
        const int cx = me.cell % m, cy = (me.cell / m) % m, cz = me.cell / (m * m);
        int nh = 0;
        for (int oz = -1; oz <= 1; ++oz) {
            int nz = cz + oz;
            nz = nz < 0 ? nz + m : (nz >= m ? nz - m : nz);
            for (int oy = -1; oy <= 1; ++oy) {
                int ny = cy + oy;
                ny = ny < 0 ? ny + m : (ny >= m ? ny - m : ny);
                for (int ox = -1; ox <= 1; ++ox) {
                    int nx = cx + ox;
                    nx = nx < 0 ? nx + m : (nx >= m ? nx - m : nx);
                    const int nc = nx + m * (ny + m * nz);
                    const int b = cell_start[nc], e = cell_start[nc + 1];
                    for (int q = b; q < e; ++q) {
                        const double4 op = pos4[q];
                        double x0 = mp.x - op.x, x1 = mp.y - op.y, x2 = mp.z - op.z;
                        x0 -= L * rint(x0 * iL);
                        x1 -= L * rint(x1 * iL);
                        x2 -= L * rint(x2 * iL);
                        const double r2 = x0 * x0 + x1 * x1 + x2 * x2;
                        if (q != j && r2 < a.rc2) {
                            hb[nh++] = q;
                            if (nh == kHitBuf) {
                                flush(nh);
                                nh = 0;
                            }
                        }
                    }
                }
            }
        }
        flush(nh);
    }
    const int64_t n = me.orig;
    V[3 * n + 0] += v[0];
    V[3 * n + 1] += v[1];
    V[3 * n + 2] += v[2];
    if (W) {
        W[3 * n + 0] += w[0];
        W[3 * n + 1] += w[1];
        W[3 * n + 2] += w[2];
    }
}

}  // namespace

hipError_t launch_pair(const fcm_plan_impl* P, double* V, double* W, bool /*torque*/,
                       hipStream_t st) {
    PairArgs a;
    a.N = (int)P->N;
    a.m = P->m;
    a.L = P->L;
    a.cw = P->L / P->m;
    a.rc2 = P->rc * P->rc;
    a.eta = P->eta;
    a.sigma = P->sigma;
    a.sigmaD = P->sigmaD;
    a.Sigma = P->Sigma;
    a.SigmaD = P->SigmaD;
    a.selfVF = P->selfVF;
    a.selfOT = P->selfOT;
    a.with_pairs = P->rc > 0.0 ? 1 : 0;
    hipLaunchKernelGGL(k_pair, dim3((a.N + kPairThreads - 1) / kPairThreads), dim3(kPairThreads), 0,
                       st, P->ppos, P->prec, P->starts + P->nbins + 1, a, V, W);
    return hipGetLastError();
}

}  // namespace fcm
