// Pairwise correction of fast FCM in FP64 (Sec. 4, pairwise correction;
// Sec. 3.2 eq. correction_VF; Sec. 3.4 eqs. correction_WF, correction_WT) and
// the self corrections of App. B.
//
// Particles are in pair-cell order.  For every particle n and every neighbour
// m with r = |x| < R_c (x = Y_n - Y_m, minimum image; cells are at least R_c
// wide, Sec. 4 spatial hashing) the receiving particle gets
//   V_n     += C_VF(x) F_m + C_VT(x) T_m,   Omega_n += C_OF(x) F_m + C_OT(x) T_m.
// Each ordered pair is evaluated for its receiving particle, so no atomics are
// needed, and every sum is taken in a fixed order: the result is deterministic.
//
// Work split, two launches.  The scan runs one thread per (particle, z layer
// of the 3x3x3 neighbour cells); cells are numbered x fastest, so the three x
// neighbours of a cell row are one contiguous run of particles (two when the
// row wraps).  It touches only compact positions and records up to kPairCap
// neighbours per thread.  The evaluation takes kPairPerBlock consecutive
// particles per workgroup, queues their recorded pairs in LDS order and
// evaluates them with all threads, so the FP64 body (erfc, exp) runs with
// full wavefronts; threads whose layer had more neighbours than the scan
// recorded rescan it for the next few and queue those for further passes of
// the whole workgroup.
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

// The six Gaussian widths of the corrections (squared): s1 = 2 sigma^2,
// s2 = 2 Sigma^2 (force); sa = sigma^2 + sigma_D^2, sb = Sigma^2 + Sigma_D^2
// (rotation-force); sc = 2 sigma_D^2, sd = 2 Sigma_D^2 (rotation-torque).
// For each, E(r) = erfc(r / sqrt(2 s)) and D(r) = (2 pi s)^(-3/2) exp(-r^2 / 2 s),
// with the width constants computed on the host.  When Sigma_D = Sigma the
// widths sb and sd equal s2 and their terms are shared (SAME).
enum { W1 = 0, W2, WA, WB, WC, WD };

struct Coef {
    double Avf, Bvf, fof, Aot, Bot;
};

// erfcx(x) = exp(x^2) erfc(x) for x >= 0, as a Chebyshev series of degree 26 in
// u = (2 - x) / (2 + x) (the variable t = 2 / (2 + x) of the Chebyshev method for
// erfc, mapped to [-1, 1]), summed by Clenshaw's recurrence without branches.
// The coefficients are this function's Chebyshev interpolant at 27 nodes,
// computed by the discrete Chebyshev transform in extended precision
// (erfcx_coefficients.py prints them); against a reference erfcx the relative
// error is below 2e-15 on [0, 10].
__device__ inline double erfcx_series(double x) {
    constexpr double c[27] = {
        0.3773760996258595, 0.4825091196506808, 0.12232459533097707,
        0.01783114971927683, 0.00032117365249443295, -0.00035039525647959736,
        -2.2438806506199784e-05, 1.0537433119359262e-05, 5.671331132873462e-07,
        -4.2976815761618624e-07, 5.104952564337281e-09, 1.8899699349060554e-08,
        -2.242755493657211e-09, -6.855253690936841e-10, 2.1487969354753117e-10,
        5.5155076776774266e-12, -1.3477436015898652e-11, 2.086398602286235e-12,
        4.4816025217859236e-13, -2.2686840572348302e-13, 1.8504140791592736e-14,
        1.1513644659686387e-14, -4.008688904952689e-15, 1.5322006653606344e-16,
        2.967500820377109e-16, -5.229189908700497e-17, 2.7446934186569573e-18};
    const double u = (2.0 - x) / (2.0 + x);
    const double u2 = 2.0 * u;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int j = 26; j >= 1; --j) {
        const double b0 = fma(u2, b1, c[j] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(u, b1, c[0] - b2);
}

template <bool SAME>
__device__ inline Coef correction_coeffs(double r, double ir, const PairArgs& a) {
    const double pi = 3.14159265358979323846;
    const double r2 = r * r, ir2 = ir * ir;
    // E(w) = erfc(x) and D(w) = gnorm exp(-x^2), x = r / sqrt(2 s_w), share one
    // exponential: erfc(x) = exp(-x^2) erfcx(x)
    auto ED = [&](int w, double& E, double& D) {
        const double x = r * a.escale[w];
        const double g = exp(-x * x);
        E = g * erfcx_series(x);
        D = a.gnorm[w] * g;
    };
    double E2, D2, Eb, Db, Ed, Dd, E1, D1, Ea, Da, Ec, Dc;
    ED(W2, E2, D2);
    if (SAME) {
        Eb = Ed = E2;
        Db = Dd = D2;
    } else {
        ED(WB, Eb, Db);
        ED(WD, Ed, Dd);
    }
    ED(W1, E1, D1);
    ED(WA, Ea, Da);
    ED(WC, Ec, Dc);
    const double s1 = a.wsq[W1], s2 = a.wsq[W2], sa = a.wsq[WA], sb = a.wsq[WB];
    const double sc = a.wsq[WC], sd = a.wsq[WD];
    const double i8 = a.c8 * ir2 * ir;  // 1 / (8 pi eta r^3)
    const double ih = a.ch * ir2;       // 1 / (2 eta r^2)
    Coef c;
    // force-velocity: erf part = (E(r; sigma sqrt2) - E(r; Sigma sqrt2)) (G + sigma^2 lap G)
    {
        const double dE = E2 - E1;
        const double g1 = a.c8 * ir;                     // 1 / (8 pi eta r)
        const double g3 = 2.0 * a.sigma * a.sigma * i8;  // sigma^2 / (4 pi eta r^3)
        c.Avf = dE * (g1 + g3);
        c.Bvf = dE * (g1 - 3.0 * g3);
        // S3(s1) - S3(s2), S3 = -(s^4 / 2 eta r^2) (I - 3 xh xh) Delta
        const double t3 = (s1 * s1 * D1 - s2 * s2 * D2) * ih;
        c.Avf += -t3;
        c.Bvf += 3.0 * t3;
        // -(sigma^2 - Sigma^2) Q2(s2), Q2 = -(1/eta)[(1 + s^2/r^2) I - (1 + 3 s^2/r^2) xh xh] Delta
        c.Avf += a.deta * (1.0 + s2 * ir2) * D2;
        c.Bvf += -a.deta * (1.0 + 3.0 * s2 * ir2) * D2;
        // -(sigma^2 - Sigma^2)^2 / 4 T(s2), T = (1/eta s^2)[(2 - r^2/s^2) I + (r^2/s^2) xh xh] Delta
        const double tq = a.cq * D2;
        const double rs = r2 * a.is2;
        c.Avf += -tq * (2.0 - rs);
        c.Bvf += -tq * rs;
    }
    // rotation-force: R(sa) - R(sb) - (d/2) K(sb)
    {
        const double dE = Eb - Ea;
        c.fof = (dE - 4.0 * pi * r * (sa * Da - sb * Db)) * i8 + a.cfb * Db;
    }
    // rotation-torque: (P(sigma_D sqrt2) - P(Sigma_D sqrt2)) / 2
    {
        const double dE = Ed - Ec;
        c.Aot = 0.5 * (-dE * i8 + ((sc + r2) * Dc - (sd + r2) * Dd) * ih);
        c.Bot = 0.5 * (3.0 * dE * i8 - ((3.0 * sc + r2) * Dc - (3.0 * sd + r2) * Dd) * ih);
    }
    return c;
}

constexpr int kPairPerBlock = 85;                 // evaluation: particles per workgroup
constexpr int kPairThreads = 3 * kPairPerBlock;   // one thread per (particle, z layer)
constexpr int kPairBlock = 256;                   // launched threads (the last one idles)
constexpr int kScanBlock = 256;

// add the corrections from one neighbour m at x = Y_n - Y_m (r^2 = r2 < R_c^2)
template <bool SAME>
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
    const double ir = 1.0 / r;
    const Coef c = correction_coeffs<SAME>(r, ir, a);
    const double h0 = x0 * ir, h1 = x1 * ir, h2 = x2 * ir;
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

// r^2 with every product and sum rounded, (x0^2 + x1^2) + x2^2: the cut-off
// test r^2 < rc2 then decides as sqrt(r^2) < R_c does on that sum (rc2 is the
// smallest double whose square root reaches R_c), pairs within ulps of R_c
// included
__device__ inline double dist2_rounded(double x0, double x1, double x2) {
#pragma clang fp contract(off)
    return (x0 * x0 + x1 * x1) + x2 * x2;
}

// minimum image of p - o in the box of sides a.Lx, a.Ly, a.Lz
__device__ inline double4 min_image(double4 p, double4 o, const PairArgs& a) {
    double x0 = p.x - o.x, x1 = p.y - o.y, x2 = p.z - o.z;
    x0 -= a.Lx * rint(x0 * a.iLx);
    x1 -= a.Ly * rint(x1 * a.iLy);
    x2 -= a.Lz * rint(x2 * a.iLz);
    return make_double4(x0, x1, x2, dist2_rounded(x0, x1, x2));
}

// The candidates of particle j's z layer `layer` (0, 1, 2 = cz-1, cz, cz+1)
// of the 3x3x3 cells around `cell`: x neighbours cx-1, cx, cx+1 (mod m) of
// the three rows, one or two runs of cells each; run k is [rb[k], re[k]).
__device__ inline void layer_runs(const int* __restrict__ cell_start, const PairArgs& a, int cell,
                                  int layer, int* rb, int* re) {
    const int mx = a.mx, my = a.my, mz = a.mz;
    const int cx = cell % mx, cy = (cell / mx) % my, cz = cell / (mx * my);
    int nz = cz + layer - 1;
    nz = nz < 0 ? nz + mz : (nz >= mz ? nz - mz : nz);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        int ny = cy + r - 1;
        ny = ny < 0 ? ny + my : (ny >= my ? ny - my : ny);
        const int row = mx * (ny + my * nz);
        if (cx == 0) {
            rb[2 * r] = cell_start[row + mx - 1];
            re[2 * r] = cell_start[row + mx];
            rb[2 * r + 1] = cell_start[row];
            re[2 * r + 1] = cell_start[row + 2];
        } else if (cx == mx - 1) {
            rb[2 * r] = cell_start[row + mx - 2];
            re[2 * r] = cell_start[row + mx];
            rb[2 * r + 1] = cell_start[row];
            re[2 * r + 1] = cell_start[row + 1];
        } else {
            rb[2 * r] = cell_start[row + cx - 1];
            re[2 * r] = cell_start[row + cx + 2];
            rb[2 * r + 1] = 0;
            re[2 * r + 1] = 0;
        }
    }
}

// Neighbours of particle j (position mp, cell `cell`) in the z layer `layer`
// within R_c, q != j: hit(q) for each, in a fixed order (runs in turn,
// ascending q).  Candidate positions are loaded four at a time.
template <class Hit>
__device__ inline void scan_layer(const double4* __restrict__ pos4, const int* __restrict__ cell_start,
                                  const PairArgs& a, int j, double4 mp, int cell, int layer,
                                  Hit&& hit) {
    int rb[6], re[6];
    layer_runs(cell_start, a, cell, layer, rb, re);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int b = rb[k], e = re[k];
        for (int q0 = b; q0 < e; q0 += 4) {
            double4 c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) c[u] = pos4[min(q0 + u, e - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u;
                if (q < e) {
                    const double4 x = min_image(mp, c[u], a);
                    if (q != j && x.w < a.rc2) hit(q);
                }
            }
        }
    }
}

// The same scan, resumable: from candidate `pos` of run `run` (pos < 0: the
// run's start), skip the first `skip` neighbours, then store the next ones in
// out[] until `cap` are stored or the layer ends.  Returns the number stored;
// (run, pos) then name the first candidate not yet examined.
__device__ inline int scan_layer_resume(const double4* __restrict__ pos4,
                                        const int* __restrict__ cell_start, const PairArgs& a, int j,
                                        double4 mp, int cell, int layer, int& run, int& pos, int skip,
                                        int cap, int* out) {
    int rb[6], re[6];
    layer_runs(cell_start, a, cell, layer, rb, re);
    int got = 0;
    for (; run < 6; ++run, pos = -1) {
        const int e = re[run];
        if (pos < 0) pos = rb[run];
        for (; pos < e; pos += 4) {
            double4 c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) c[u] = pos4[min(pos + u, e - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = pos + u;
                if (q < e) {
                    const double4 x = min_image(mp, c[u], a);
                    if (q != j && x.w < a.rc2) {
                        if (skip > 0) {
                            --skip;
                        } else {
                            out[got++] = q;
                            if (got == cap) {
                                pos = q + 1;
                                if (pos >= e) {
                                    ++run;
                                    pos = -1;
                                }
                                return got;
                            }
                        }
                    }
                }
            }
        }
    }
    return got;
}

// thread t = 3 j + layer records the first kPairCap neighbours of particle j
// in its layer and their total count
__global__ __launch_bounds__(kScanBlock) void k_pair_scan(const double4* __restrict__ pos4,
                                                          const PairRec* __restrict__ rec,
                                                          const int* __restrict__ cell_start,
                                                          PairArgs a, int* __restrict__ hits,
                                                          int* __restrict__ count) {
    const int t = xcd_remap(blockIdx.x, gridDim.x) * kScanBlock + threadIdx.x;
    if (t >= 3 * a.N) return;
    const int j = t / 3, layer = t - 3 * j;
    int n = 0;
    int* h = hits + (size_t)t * kPairCap;
    scan_layer(pos4, cell_start, a, j, pos4[j], rec[j].cell, layer, [&](int q) {
        if (n < kPairCap) h[n] = q;
        ++n;
    });
    count[t] = n;
}

constexpr int kRefill = 24;   // evaluation: hits a thread queues per refill pass (LDS)

template <bool SAME>
__global__ __launch_bounds__(kPairBlock) void k_pair_eval(const double4* __restrict__ pos4,
                                                          const PairRec* __restrict__ rec,
                                                          const int* __restrict__ cell_start,
                                                          const int* __restrict__ hits,
                                                          const int* __restrict__ count,
                                                          PairArgs a, double* __restrict__ V,
                                                          double* __restrict__ W) {
    __shared__ int qoff[kPairBlock + 1];         // queue offset of each thread's pairs
    __shared__ int wsum[kPairBlock / 64];
    __shared__ double res[kPairBlock][6];        // evaluated pairs of one round
    __shared__ int rq[kPairBlock * kRefill];     // refill passes: each thread's next hits
    const int tid = threadIdx.x;
    const int base = xcd_remap(blockIdx.x, gridDim.x) * kPairPerBlock;
    const int pl = tid / 3, layer = tid - 3 * pl;  // local particle, z layer
    const int j = base + pl;
    const bool active = tid < kPairThreads && j < a.N;
    const size_t t0 = (size_t)3 * base;          // scan thread of local thread 0
    int ntrue = (active && a.with_pairs) ? count[t0 + tid] : 0;

    // Pass 0 evaluates the hits the scan recorded.  While a thread of the
    // block has more, each such thread rescans its layer for its next kRefill
    // hits into LDS and the block evaluates them in another pass, so long
    // neighbour lists keep every thread busy.  A particle's pairs are summed
    // pass by pass, layer by layer, in scan order.
    int nq = min(ntrue, kPairCap);               // this pass's hits of this thread
    int taken = 0;                               // hits consumed by earlier passes
    int srun = 0, spos = -1;                     // where the refill scan resumes
    double v[3] = {0, 0, 0}, w[3] = {0, 0, 0};
    for (int pass = 0;; ++pass) {
        // queue offsets: exclusive scan of the per-thread counts
        {
            const int lane = tid & 63, wid = tid >> 6;
            int inc = nq;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(inc, o, 64);
                if (lane >= o) inc += u;
            }
            if (lane == 63) wsum[wid] = inc;
            __syncthreads();
            int pre = 0;
            for (int k = 0; k < wid; ++k) pre += wsum[k];
            qoff[tid] = pre + inc - nq;
            if (tid == kPairBlock - 1) qoff[kPairBlock] = pre + inc;
            __syncthreads();
        }
        const int total = qoff[kPairBlock];

        // evaluate the queue in rounds of kPairBlock pairs; the layer-0 thread
        // of each particle adds its particle's results of the round in queue order
        for (int r0 = 0; r0 < total; r0 += kPairBlock) {
            const int e = r0 + tid;
            if (e < total) {
                // the thread that queued pair e: the last one whose offset is <= e
                int lo = 0, hi = kPairBlock - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (qoff[mid] <= e) lo = mid;
                    else hi = mid - 1;
                }
                const int q = pass == 0 ? hits[(t0 + lo) * kPairCap + (e - qoff[lo])]
                                        : rq[lo * kRefill + (e - qoff[lo])];
                const double4 y = min_image(pos4[base + lo / 3], pos4[q], a);
                double rv[3] = {0, 0, 0}, rw[3] = {0, 0, 0};
                add_pair<SAME>(y.x, y.y, y.z, y.w, rec[q], a, rv, rw);
                res[tid][0] = rv[0];
                res[tid][1] = rv[1];
                res[tid][2] = rv[2];
                res[tid][3] = rw[0];
                res[tid][4] = rw[1];
                res[tid][5] = rw[2];
            }
            __syncthreads();
            if (active && layer == 0) {
                const int lo = max(qoff[tid], r0), hi = min(qoff[tid + 3], r0 + kPairBlock);
                for (int k = lo; k < hi; ++k) {
                    const double* rr = res[k - r0];
                    v[0] += rr[0];
                    v[1] += rr[1];
                    v[2] += rr[2];
                    w[0] += rr[3];
                    w[1] += rr[4];
                    w[2] += rr[5];
                }
            }
            __syncthreads();
        }

        taken += nq;
        const int rem = ntrue - taken;
        if (!__syncthreads_or(rem > 0)) break;
        nq = min(rem, kRefill);
        if (nq > 0) {
            // the first refill skips the hits the scan recorded; later ones resume
            const int got = scan_layer_resume(pos4, cell_start, a, j, pos4[j], rec[j].cell, layer, srun,
                                              spos, pass == 0 ? taken : 0, nq, rq + tid * kRefill);
            // queue only what the rescan found (it repeats the scan's count)
            if (got < nq) {
                nq = got;
                ntrue = taken + got;
            }
        }
    }

    if (active && layer == 0) {
        const PairRec me = rec[j];
        const int64_t n = me.orig;
        const double c[6] = {a.selfVF * me.F[0] + v[0], a.selfVF * me.F[1] + v[1],
                             a.selfVF * me.F[2] + v[2], a.selfOT * me.T[0] + w[0],
                             a.selfOT * me.T[1] + w[1], a.selfOT * me.T[2] + w[2]};
        if (a.store) {
#pragma unroll
            for (int d = 0; d < 3; ++d) V[3 * n + d] = c[d];
            if (W) {
#pragma unroll
                for (int d = 0; d < 3; ++d) W[3 * n + d] = c[3 + d];
            }
        } else {
#pragma unroll
            for (int d = 0; d < 3; ++d) V[3 * n + d] += c[d];
            if (W) {
#pragma unroll
                for (int d = 0; d < 3; ++d) W[3 * n + d] += c[3 + d];
            }
        }
    }
}

}  // namespace

hipError_t launch_pair(const fcm_plan_impl* P, double* V, double* W, bool /*torque*/,
                       hipStream_t st, bool store, bool scan) {
    PairArgs a;
    a.N = (int)P->N;
    a.mx = P->m;
    a.my = P->mcy;
    a.mz = P->mcz;
    a.Lx = P->L;
    a.Ly = P->Ly;
    a.Lz = P->Lz;
    a.iLx = 1.0 / P->L;
    a.iLy = 1.0 / P->Ly;
    a.iLz = 1.0 / P->Lz;
    a.cwx = P->L / P->m;
    a.cwy = P->Ly / P->mcy;
    a.cwz = P->Lz / P->mcz;
    // the smallest double whose (correctly rounded) square root reaches R_c:
    // r2 < rc2 exactly when sqrt(r2) < R_c, as sqrt is monotone
    double t = P->rc * P->rc;
    while (t > 0.0 && sqrt(nextafter(t, 0.0)) >= P->rc) t = nextafter(t, 0.0);
    while (sqrt(t) < P->rc) t = nextafter(t, INFINITY);
    a.rc2 = t;
    a.eta = P->eta;
    a.sigma = P->sigma;
    a.sigmaD = P->sigmaD;
    a.Sigma = P->Sigma;
    a.SigmaD = P->SigmaD;
    a.selfVF = P->selfVF;
    a.selfOT = P->selfOT;
    a.with_pairs = P->rc > 0.0 ? 1 : 0;
    a.store = store ? 1 : 0;
    const int* cs = P->starts + P->nbins + 1;
    if (a.with_pairs && scan)
        hipLaunchKernelGGL(k_pair_scan, dim3((3 * a.N + kScanBlock - 1) / kScanBlock), dim3(kScanBlock),
                           0, st, P->ppos, P->prec, cs, a, P->pair_hits, P->pair_count);
    // width constants of the six Gaussians (see correction_coeffs)
    const double pi = 3.14159265358979323846;
    const double sg2 = P->sigma * P->sigma, Sg2 = P->Sigma * P->Sigma;
    const double sD2 = P->sigmaD * P->sigmaD, SD2 = P->SigmaD * P->SigmaD;
    const double wsq[6] = {2.0 * sg2, 2.0 * Sg2, sg2 + sD2, Sg2 + SD2, 2.0 * sD2, 2.0 * SD2};
    for (int k = 0; k < 6; ++k) {
        a.wsq[k] = wsq[k];
        a.escale[k] = 1.0 / sqrt(2.0 * wsq[k]);
        a.gnorm[k] = pow(2.0 * pi * wsq[k], -1.5);
    }
    const double d = sg2 - Sg2;
    a.c8 = 1.0 / (8.0 * pi * a.eta);
    a.ch = 1.0 / (2.0 * a.eta);
    a.deta = d / a.eta;
    a.cq = d * d / (4.0 * a.eta * wsq[1]);
    a.cfb = d / (4.0 * a.eta * wsq[3]);
    a.is2 = 1.0 / wsq[1];
    const dim3 ge((a.N + kPairPerBlock - 1) / kPairPerBlock), be(kPairBlock);
    if (P->SigmaD == P->Sigma)
        hipLaunchKernelGGL(k_pair_eval<true>, ge, be, 0, st, P->ppos, P->prec, cs, P->pair_hits,
                           P->pair_count, a, V, W);
    else
        hipLaunchKernelGGL(k_pair_eval<false>, ge, be, 0, st, P->ppos, P->prec, cs, P->pair_hits,
                           P->pair_count, a, V, W);
    return hipGetLastError();
}

}  // namespace fcm
