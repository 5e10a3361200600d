// Grid operators of fast FCM: spreading J~^dagger[F] + N~^dagger[T] and
// interpolation J~[u], N~[u] (Sec. 2.1, Sec. 3.1, Sec. 3.4).
//
// Spreading is done in gather form: one 64-lane wavefront owns a tile of
// TX x TY grid columns and TZ points along z, scans the particles of the grid
// bins whose supports can reach the tile (particles are sorted by the bin of
// their first support point), stages the contributing ones in LDS, and
// accumulates their kernel values in registers.  Every grid point is written
// exactly once, with one coalesced store per point: no global atomics.
//
// The modified force kernel is Delta~(d) = Delta(d; Sigma) (A + B |d|^2) with
// A = 1 - 3c/Sigma^2, B = c/Sigma^4, c = (sigma^2 - Sigma^2)/2 (the operator
// (1 + c lap) applied to the Gaussian), and the torque kernel is
// (1/2 Sigma_D^2) Delta(d; Sigma_D) (T x d) (Sec. 3.4).  Both are separable
// Gaussians times low-order polynomials, so along z the sum is factorised:
// each lane forms its (x, y) column factors once per particle and then needs
// only a few FMAs per z point.
//
// Interpolation is particle-major, with a factorised sum along z per lane: in
// general one wavefront per particle with lanes over the (x, y) columns of the
// M_G^3 support and a butterfly shuffle reduction; in FP32 with one width,
// lanes over support rows reading 16-byte quads of four x points (k_interp4:
// one particle a wavefront; k_interp8: several, for fields in the tiled
// layout).
#include "fcm_internal.h"

namespace fcm {

namespace {

constexpr int kChunk = 32;

template <typename R>
struct alignas(16) ZTab {
    R g;    // Gaussian of width Sigma along z (unnormalised)
    R gd2;  // g * dz^2
    R gD;   // Gaussian of width Sigma_D along z
    R gDd;  // gD * dz
};

// 2^x for x <= 0: the hardware exponential (results below the FP32 normal
// range flush towards 0, which only drops kernel tails beyond ~e^-87)
__device__ inline float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline double fexp2(double x) { return exp2(x); }

// Accumulation of the spread sums: ACC_PLAIN adds in the grid precision,
// ACC_KAHAN keeps a Kahan compensation term per value, ACC_WIDE accumulates
// FP32 contributions in FP64 registers.
enum { ACC_PLAIN = 0, ACC_KAHAN = 1, ACC_WIDE = 2 };

template <int MODE, typename R>
struct Acc {
    R s = 0, c = 0;
    __device__ inline void add(R v) {
        if (MODE == ACC_KAHAN) {
            const R y = v - c;
            const R t = s + y;
            c = (t - s) - y;
            s = t;
        } else {
            s += v;
        }
    }
    __device__ inline R value() const { return MODE == ACC_KAHAN ? s - c : s; }
};

template <>
struct Acc<ACC_WIDE, float> {
    double s = 0;
    __device__ inline void add(float v) { s += (double)v; }
    __device__ inline float value() const { return (float)s; }
};

// the n lowest bits set (0 <= n <= 32, 0 <= n <= 64)
__device__ inline unsigned low_bits(int n) { return n >= 32 ? 0xffffffffu : (1u << n) - 1u; }
__device__ inline unsigned long long low_bits64(int n) { return n >= 64 ? ~0ull : (1ull << n) - 1ull; }

// contributors staged for one round of the spread, one array per field:
// lm: the lanes (tile columns) within the support, as a 64-bit lane mask;
// km: the tile heights within it, as a bit mask; zo: the byte offset of the
// z-factor entry of the tile's first height; c (x, y): the offset of tile
// column 0 from the contributor's centre along the axis, in grid spacings
// (column i lies at (i + c) dx); fz: its z fraction; F, T: force and torque
template <typename R>
struct Stage {
    unsigned lm[2][kChunk];
    unsigned km[kChunk];
    int zo[kChunk];
    int dz[kChunk];      // folded z (support longer than the z axis): (Z0 - first point) mod Mz
    R c[2][kChunk];
    R fz[kChunk];
    R F[3][kChunk];
    R T[3][kChunk];
};

template <typename R, int TZ, int MODE, bool TORQUE, bool SAMEW>
__global__ __launch_bounds__(64) void k_spread(const GridRec<R>* __restrict__ rec,
                                               const int* __restrict__ bin_start,
                                               R* __restrict__ grid, GridArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    Stage<R>& stg = *reinterpret_cast<Stage<R>*>(smem);
    ZTab<R>* zt = reinterpret_cast<ZTab<R>*>(smem + sizeof(Stage<R>));

    const int lane = threadIdx.x;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int Mx = a.M, My = a.My, Mz = a.Mz, MG = a.MG;
    const int btx = tile % a.nbx;
    const int rem = tile / a.nbx;
    const int bty = rem % a.nby;
    const int btz = rem / a.nby;
    const int X0 = btx * a.TX, Y0 = bty * a.TY, Z0 = btz * TZ;
    const int li = lane % a.TX, lj = lane / a.TX;
    const bool lact = lj < a.TY;
    const int gxp = X0 + li, gyp = Y0 + (lact ? lj : 0);
    const R dx = a.dx;
    const R lif = (R)li, ljf = (R)lj;

    Acc<MODE, R> acc[3][TZ];

    // The bins that can reach the tile are bx in btx-backx .. btx (mod nbx)
    // for each (by, bz) row; bins are numbered x fastest and particles are
    // sorted by bin, so each row is one contiguous run of particles (two when
    // it wraps around the periodic x boundary).  One lane per row fetches the
    // row's bounds, so all of them arrive in one round trip.
    __shared__ int4 runs[64];
    const int nrows = (a.backy + 1) * (a.backz + 1);
    for (int rr = lane; rr < nrows; rr += 64) {
        const int oz = rr / (a.backy + 1), oy = rr - oz * (a.backy + 1);
        int bz = btz - oz;
        if (bz < 0) bz += a.nbz;
        int by = bty - oy;
        if (by < 0) by += a.nby;
        const int row = a.nbx * (by + a.nby * bz);
        const int bx0 = btx - a.backx;
        const bool wraps = bx0 < 0;
        int4 b;
        b.x = bin_start[row + (wraps ? bx0 + a.nbx : bx0)];
        b.y = bin_start[row + (wraps ? a.nbx : btx + 1)];
        b.z = wraps ? bin_start[row] : 0;
        b.w = wraps ? bin_start[row + btx + 1] : 0;
        if (rr < 64) runs[rr] = b;
    }
    // Contributors are staged until the next chunk of candidates would
    // overflow the stage, so short runs (a few bins of one row) share one
    // round of z factors and barriers; the summation order is that of the
    // runs, rows and lanes regardless of where a round ends.
    int cnt = 0;
    auto process = [&]() {
        __syncthreads();
        // their z factors, one table entry per lane
        if (!a.zfold) {
            for (int e = lane; e < cnt * MG; e += 64) {
                const int s = (e * a.mgmul) >> 16, t = e - s * MG;
                const R d = ((R)t - stg.fz[s]) * dx;
                const R d2 = d * d;
                ZTab<R> z;
                z.g = fexp2(-d2 * a.e2);
                z.gd2 = z.g * d2;
                z.gD = SAMEW ? z.g : fexp2(-d2 * a.e2D);
                z.gDd = z.gD * d;
                zt[e] = z;
            }
        } else {
            // support longer than the z axis (one tile spans it, TZ = Mz):
            // height k receives the support points t = k + dz (mod Mz),
            // t + Mz, ... below M_G; their factors are summed into entry k
            for (int e = lane; e < cnt * Mz; e += 64) {
                const int s = e / Mz, k = e - s * Mz;
                int t = k + stg.dz[s];
                if (t >= Mz) t -= Mz;
                ZTab<R> z = {0, 0, 0, 0};
                for (; t < MG; t += Mz) {
                    const R d = ((R)t - stg.fz[s]) * dx;
                    const R d2 = d * d;
                    const R g = fexp2(-d2 * a.e2);
                    const R gD = SAMEW ? g : fexp2(-d2 * a.e2D);
                    z.g += g;
                    z.gd2 += g * d2;
                    z.gD += gD;
                    z.gDd += gD * d;
                }
                zt[s * MG + k] = z;
            }
        }
        __syncthreads();
        for (int q = 0; q < cnt; ++q) {
            const unsigned lo = __builtin_amdgcn_readfirstlane(stg.lm[0][q]);
            const unsigned hi = __builtin_amdgcn_readfirstlane(stg.lm[1][q]);
            const bool in = __builtin_amdgcn_inverse_ballot_w64(((unsigned long long)hi << 32) | lo);
            const R dxv = (lif + stg.c[0][q]) * dx;
            const R dyv = (ljf + stg.c[1][q]) * dx;
            const R r2 = dxv * dxv + dyv * dyv;
            const R gxy = in ? fexp2(-r2 * a.e2) : (R)0;
            // Column coefficients: with g_z, d_z the z factors, the
            // contribution to component c at height z is
            //   g_z (P_c + d_z^2 Q_c) + gD_z (Pt_c + d_z S_c)
            // where P, Q carry the force kernel g_xy (A + B r_xy^2 +
            // B d_z^2) F_c and Pt, S the torque kernel's T x d split
            // into its d_z-free part and its d_z coefficient.
            const R wq = gxy * a.B;
            const R wf = wq * r2 + gxy * a.A;
            R P[3], Q[3], Pt[3] = {0, 0, 0}, S0 = 0, S1 = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                P[c] = wf * stg.F[c][q];
                Q[c] = wq * stg.F[c][q];
            }
            if (TORQUE) {
                const R gxyD = SAMEW ? gxy : (in ? fexp2(-r2 * a.e2D) : (R)0);
                const R g0 = gxyD * stg.T[0][q], g1 = gxyD * stg.T[1][q], g2 = gxyD * stg.T[2][q];
                // T x d = (T1 dz - T2 dy, T2 dx - T0 dz, T0 dy - T1 dx)
                Pt[0] = -g2 * dyv;
                Pt[1] = g2 * dxv;
                Pt[2] = g0 * dyv - g1 * dxv;
                S0 = g1;
                S1 = -g0;
                if (SAMEW) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) P[c] += Pt[c];
                }
            }
            const unsigned kmask = __builtin_amdgcn_readfirstlane(stg.km[q]);
            auto step = [&](const int k, const ZTab<R>& e) {
                if (MODE == ACC_PLAIN) {
                    R v0 = acc[0][k].s, v1 = acc[1][k].s, v2 = acc[2][k].s;
                    v0 = v0 + e.g * P[0] + e.gd2 * Q[0];
                    v1 = v1 + e.g * P[1] + e.gd2 * Q[1];
                    v2 = v2 + e.g * P[2] + e.gd2 * Q[2];
                    if (TORQUE) {
                        if (!SAMEW) {
                            v0 = v0 + e.gD * Pt[0];
                            v1 = v1 + e.gD * Pt[1];
                            v2 = v2 + e.gD * Pt[2];
                        }
                        v0 = v0 + e.gDd * S0;
                        v1 = v1 + e.gDd * S1;
                    }
                    acc[0][k].s = v0;
                    acc[1][k].s = v1;
                    acc[2][k].s = v2;
                } else {
                    R v0 = e.g * P[0] + e.gd2 * Q[0];
                    R v1 = e.g * P[1] + e.gd2 * Q[1];
                    R v2 = e.g * P[2] + e.gd2 * Q[2];
                    if (TORQUE) {
                        if (!SAMEW) {
                            v0 = v0 + e.gD * Pt[0];
                            v1 = v1 + e.gD * Pt[1];
                            v2 = v2 + e.gD * Pt[2];
                        }
                        v0 = v0 + e.gDd * S0;
                        v1 = v1 + e.gDd * S1;
                    }
                    acc[0][k].add(v0);
                    acc[1][k].add(v1);
                    acc[2][k].add(v2);
                }
            };
            // the table entry of height k is zb[k] (heights outside kmask
            // are not read)
            const ZTab<R>* zb = reinterpret_cast<const ZTab<R>*>(reinterpret_cast<const char*>(zt) + stg.zo[q]);
#pragma unroll
            for (int k = 0; k < TZ; ++k)
                if (kmask & (1u << k)) step(k, zb[k]);
        }
        __syncthreads();
    };
    __syncthreads();
    // One pass over the chunks of candidates of every run of every row, with
    // one place where the stage is processed (when the next chunk would
    // overflow it, and once at the end).
    auto row_runs = [&](int rr) {
        int4 b;
        if (rr < 64) {
            b = runs[rr];
        } else {
            const int oz = rr / (a.backy + 1), oy = rr - oz * (a.backy + 1);
            int bz = btz - oz;
            if (bz < 0) bz += a.nbz;
            int by = bty - oy;
            if (by < 0) by += a.nby;
            const int row = a.nbx * (by + a.nby * bz);
            const int bx0 = btx - a.backx;
            const bool wraps = bx0 < 0;
            b.x = bin_start[row + (wraps ? bx0 + a.nbx : bx0)];
            b.y = bin_start[row + (wraps ? a.nbx : btx + 1)];
            b.z = wraps ? bin_start[row] : 0;
            b.w = wraps ? bin_start[row + btx + 1] : 0;
        }
        b.x = __builtin_amdgcn_readfirstlane(b.x);
        b.y = __builtin_amdgcn_readfirstlane(b.y);
        b.z = __builtin_amdgcn_readfirstlane(b.z);
        b.w = __builtin_amdgcn_readfirstlane(b.w);
        return b;
    };
    int rr = 0, second = 0, base = 0, end = 0;
    int4 rb = make_int4(0, 0, 0, 0);
    for (;;) {
        // the next non-empty run: the first of row rr, then its second
        while (base >= end && rr < nrows) {
            if (!second) {
                rb = row_runs(rr);
                base = rb.x;
                end = rb.y;
                second = 1;
            } else {
                base = rb.z;
                end = rb.w;
                second = 0;
                ++rr;
            }
        }
        const bool done = base >= end;
        bool take = false;
        GridRec<R> r;
        // the contributors among this chunk of candidates
        const int p = base + lane;
        if (!done && lane < kChunk && p < end) {
            r = rec[p];
            int d0x = X0 - r.s[0];
            if (d0x < 0) d0x += Mx;
            int d0y = Y0 - r.s[1];
            if (d0y < 0) d0y += My;
            int d0z = Z0 - r.s[2];
            if (d0z < 0) d0z += Mz;
            take = (d0x < MG || d0x > Mx - a.TX) && (d0y < MG || d0y > My - a.TY) &&
                   (d0z < MG || d0z > Mz - TZ);
        }
        const unsigned long long mask = __ballot(take);
        const int n = __popcll(mask);
        if (done || cnt + n > kChunk) {
            process();
            cnt = 0;
        }
        if (done) break;
        if (take) {
            // Along x and y the tile's columns within the support form one
            // run (the plan keeps TX <= M - MG + 1, TY <= My - MG + 1): with
            // o the support index of the tile's first column (signed), lanes
            // i in [max(0, -o), min(T, MG - o)).  Along z, heights k with
            // (Z0 + k - sz) mod Mz < MG form one run too (TZ <= Mz - MG + 1).
            const int k = cnt + __popcll(mask & ((1ull << lane) - 1ull));
            int ox = X0 - r.s[0];
            if (ox < 0) ox += Mx;
            if (ox > Mx - a.TX) ox -= Mx;
            int oy = Y0 - r.s[1];
            if (oy < 0) oy += My;
            if (oy > My - a.TY) oy -= My;
            const int xlo = max(0, -ox), xhi = min(a.TX, MG - ox);
            const int ylo = max(0, -oy), yhi = min(a.TY, MG - oy);
            const unsigned long long lm = ((low_bits64(xhi) & ~low_bits64(xlo)) * a.rowrep) &
                                          (low_bits64(a.TX * yhi) & ~low_bits64(a.TX * ylo));
            int dz0 = Z0 - r.s[2];
            if (dz0 < 0) dz0 += Mz;
            const int hi1 = min(TZ, MG - dz0);
            const int lo2 = Mz - dz0;
            const int hi2 = min(TZ, Mz - dz0 + MG);
            unsigned km = hi1 > 0 ? low_bits(hi1) : 0u;
            if (lo2 < TZ) km |= low_bits(hi2) & ~low_bits(lo2);
            stg.lm[0][k] = (unsigned)lm;
            stg.lm[1][k] = (unsigned)(lm >> 32);
            if (a.zfold) {
                // every height of the tile (the whole z axis) is in the support;
                // the contributor's table holds one folded entry per height
                km = low_bits(TZ);
                stg.dz[k] = dz0;
                stg.zo[k] = k * MG * (int)sizeof(ZTab<R>);
            } else {
                stg.zo[k] = (k * MG + (hi1 > 0 ? dz0 : dz0 - Mz)) * (int)sizeof(ZTab<R>);
            }
            stg.km[k] = km;
            stg.c[0][k] = (R)ox - r.f[0];
            stg.c[1][k] = (R)oy - r.f[1];
            stg.fz[k] = r.f[2];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                stg.F[d][k] = r.F[d];
                stg.T[d][k] = r.T[d];
            }
        }
        cnt += n;
        base += kChunk;
    }
    if (lact) {
        const size_t M3 = (size_t)Mx * My * Mz;
        const size_t col = a.tiled ? (size_t)((gyp >> 2) * (Mx << 2) + ((gxp >> 3) << 5) + ((gyp & 3) << 3) +
                                              (gxp & 7))
                                   : (size_t)gyp * Mx + gxp;
#pragma unroll
        for (int k = 0; k < TZ; ++k) {
            const size_t idx = (size_t)(Z0 + k) * Mx * My + col;
#pragma unroll
            for (int c = 0; c < 3; ++c) grid[c * M3 + idx] = acc[c][k].value();
        }
    }
}

// element at byte offset `col` of the plane of n values starting at `plane` (a
// wavefront-uniform pointer)
__device__ inline float plane_load(const float* plane, int n, unsigned col) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(plane), (short)0, n * (int)sizeof(float), kBufferWord3);
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)col, 0, 0));
}
__device__ inline double plane_load(const double* plane, int n, unsigned col) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double*>(plane), (short)0, n * (int)sizeof(double), kBufferWord3);
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)col, 0, 0));
}

__device__ inline float uniform(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ inline double uniform(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

template <typename R>
__device__ inline R wave_sum(R v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename R, bool OMEGA, bool SAMEW>
__global__ __launch_bounds__(256) void k_interp(const GridRec<R>* __restrict__ rec,
                                                const R* __restrict__ grid, double* __restrict__ V,
                                                double* __restrict__ W, GridArgs<R> a,
                                                double scaleV, double scaleW,
                                                const double* __restrict__ corr) {
    __shared__ ZTab<R> zt[4][kMaxSupport];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int p = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    const bool live = p < a.N;
    const GridRec<R> rv = rec[live ? p : a.N - 1];
    // the record is the same for the whole wavefront: keep it in scalar registers
    GridRec<R> r;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r.s[d] = __builtin_amdgcn_readfirstlane(rv.s[d]);
        r.f[d] = uniform(rv.f[d]);
    }
    r.orig = __builtin_amdgcn_readfirstlane(rv.orig);
    const int Mx = a.M, My = a.My, Mz = a.Mz, MG = a.MG;
    const int nplane = Mx * My;
    const R dx = a.dx;
    if (lane < MG) {
        const R d = ((R)lane - r.f[2]) * dx;
        const R d2 = d * d;
        ZTab<R> e;
        e.g = fexp2(-d2 * a.e2);
        e.gd2 = e.g * d2;
        e.gD = SAMEW ? e.g : fexp2(-d2 * a.e2D);
        e.gDd = e.gD * d;
        zt[wave][lane] = e;
    }
    __syncthreads();
    const size_t M3 = (size_t)Mx * My * Mz;
    R v0 = 0, v1 = 0, v2 = 0, o0 = 0, o1 = 0, o2 = 0;
    const int ncol = MG * MG;
    for (int q0 = 0; q0 < ncol; q0 += 64) {
        const int q = q0 + lane;
        const bool ok = q < ncol;
        const int i = ok ? q % MG : 0;
        const int j = ok ? q / MG : 0;
        int x = r.s[0] + i;
        if (x >= Mx) x -= Mx;
        int y = r.s[1] + j;
        if (y >= My) y -= My;
        const R dxv = ((R)i - r.f[0]) * dx;
        const R dyv = ((R)j - r.f[1]) * dx;
        const R x2 = dxv * dxv, y2 = dyv * dyv;
        const R gxy = ok ? fexp2(-(x2 + y2) * a.e2) : (R)0;
        R A0[3] = {0, 0, 0}, A2[3] = {0, 0, 0}, D1[3] = {0, 0, 0}, D0[3] = {0, 0, 0};
        // per-lane byte offset of the column within a z plane (32 bits); the
        // plane and component bases are wavefront-uniform
        const unsigned col =
            (a.tiled ? (unsigned)((y >> 2) * (Mx << 2) + ((x >> 3) << 5) + ((y & 3) << 3) + (x & 7))
                     : (unsigned)y * (unsigned)Mx + (unsigned)x) *
            (unsigned)sizeof(R);
        for (int k = 0; k < MG; ++k) {
            int z = r.s[2] + k;
            while (z >= Mz) z -= Mz;   // the support may be longer than the z axis
            const ZTab<R> e = zt[wave][k];
            const R* pz = grid + (size_t)z * nplane;
            const R u0 = plane_load(pz, nplane, col);
            const R u1 = plane_load(pz + M3, nplane, col);
            const R u2 = plane_load(pz + 2 * M3, nplane, col);
            A0[0] += e.g * u0;
            A0[1] += e.g * u1;
            A0[2] += e.g * u2;
            A2[0] += e.gd2 * u0;
            A2[1] += e.gd2 * u1;
            A2[2] += e.gd2 * u2;
            if (OMEGA) {
                D1[0] += e.gDd * u0;
                D1[1] += e.gDd * u1;
                D1[2] += e.gDd * u2;
                if (!SAMEW) {
                    D0[0] += e.gD * u0;
                    D0[1] += e.gD * u1;
                    D0[2] += e.gD * u2;
                }
            }
        }
        const R cw = gxy * (a.A + a.B * (x2 + y2));
        const R cb = gxy * a.B;
        v0 += cw * A0[0] + cb * A2[0];
        v1 += cw * A0[1] + cb * A2[1];
        v2 += cw * A0[2] + cb * A2[2];
        if (OMEGA) {
            R gD = gxy;
            const R* S0 = A0;
            if (!SAMEW) {
                gD = ok ? fexp2(-(x2 + y2) * a.e2D) : (R)0;
                S0 = D0;
            }
            // (d x u): x: dy u_z - dz u_y ; y: dz u_x - dx u_z ; z: dx u_y - dy u_x
            o0 += gD * (dyv * S0[2] - D1[1]);
            o1 += gD * (D1[0] - dxv * S0[2]);
            o2 += gD * (dxv * S0[1] - dyv * S0[0]);
        }
    }
    v0 = wave_sum(v0);
    v1 = wave_sum(v1);
    v2 = wave_sum(v2);
    if (OMEGA) {
        o0 = wave_sum(o0);
        o1 = wave_sum(o1);
        o2 = wave_sum(o2);
    }
    if (live && lane == 0) {
        const int64_t n = r.orig;
        double cv[3] = {0, 0, 0}, cw[3] = {0, 0, 0};
        if (corr) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                cv[d] = corr[3 * n + d];
                cw[d] = corr[3 * (int64_t)a.N + 3 * n + d];
            }
        }
        V[3 * n + 0] = (double)v0 * scaleV + cv[0];
        V[3 * n + 1] = (double)v1 * scaleV + cv[1];
        V[3 * n + 2] = (double)v2 * scaleV + cv[2];
        if (OMEGA) {
            W[3 * n + 0] = (double)o0 * scaleW + cw[0];
            W[3 * n + 1] = (double)o1 * scaleW + cw[1];
            W[3 * n + 2] = (double)o2 * scaleW + cw[2];
        }
    }
}

__device__ inline float4 plane_load4(const float* plane, int n, unsigned col) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(plane), (short)0, n * (int)sizeof(float), kBufferWord3);
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)col, 0, 0));
}

// FP32 interpolation with 16-byte loads (M divisible by 4, M_G <= 13, Sigma_D =
// Sigma): lane (j, c) owns support row j and the aligned chunk c of four x
// points, so each load returns four values of one row and a wavefront covers a
// particle's support in one pass.  Per z plane the lane forms the x-weighted
// sums of its chunk; the z sums and the lane sums follow the factorisation
//   V_c     = (A + B dy^2) P_c + B (R_c + PD2_c)
//   Omega   = (dy P_z - PD_y, PD_x - Q_z, Q_y - dy P_x)
// with P_c = sum_z g_z sum_x g_xy u_c, R_c = sum_z g_z sum_x g_xy dx^2 u_c,
// PD2_c = sum_z g_z dz^2 sum_x g_xy u_c, PD_c = sum_z g_z dz sum_x g_xy u_c,
// Q_c = sum_z g_z sum_x g_xy dx u_c.
// WIDE (row-major layout, M_G <= 16): the chunks start at the support's first
// point x0 instead of x0 & ~3, so 16 rows x 4 chunks cover an M_G = 16 support
// exactly; the 16-byte loads are then only 4-byte aligned, and a chunk that
// crosses the end of a row is read as four single values.
template <bool OMEGA, bool WIDE = false>
__global__ __launch_bounds__(256) void k_interp4(const GridRec<float>* __restrict__ rec,
                                                 const float* __restrict__ grid, double* __restrict__ V,
                                                 double* __restrict__ W, GridArgs<float> a,
                                                 double scaleV, double scaleW,
                                                 const double* __restrict__ corr) {
    __shared__ ZTab<float> zt[4][kMaxSupport];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int p = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    const bool live = p < a.N;
    const GridRec<float> rv = rec[live ? p : a.N - 1];
    GridRec<float> r;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r.s[d] = __builtin_amdgcn_readfirstlane(rv.s[d]);
        r.f[d] = uniform(rv.f[d]);
    }
    r.orig = __builtin_amdgcn_readfirstlane(rv.orig);
    const int Mx = a.M, My = a.My, Mz = a.Mz, MG = a.MG;
    const int nplane = Mx * My;
    const float dx = a.dx;
    if (lane < MG) {
        const float d = ((float)lane - r.f[2]) * dx;
        const float d2 = d * d;
        ZTab<float> e;
        e.g = fexp2(-d2 * a.e2);
        e.gd2 = e.g * d2;
        e.gD = e.g;
        e.gDd = e.g * d;
        zt[wave][lane] = e;
    }
    // lane -> support row j, chunk c of four x points starting at the aligned x0 & ~3
    const int j = lane >> 2, c = lane & 3;
    const int x0 = r.s[0], off0 = WIDE ? 0 : x0 & 3;
    int xs = (x0 - off0) + 4 * c;
    if (xs >= Mx) xs -= Mx;
    // WIDE: a chunk running past the end of the row wraps to its start
    const bool split = WIDE && xs > Mx - 4;
    const bool rowok = j < MG;
    int yy = r.s[1] + (rowok ? j : 0);
    if (yy >= My) yy -= My;
    const float dyv = ((float)j - r.f[1]) * dx;
    const float gy = rowok ? fexp2(-dyv * dyv * a.e2) : 0.0f;
    float gw[4], gwd[4], gwd2[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int i = 4 * c + e - off0;
        const float dxe = ((float)i - r.f[0]) * dx;
        const float gx = (i >= 0 && i < MG) ? fexp2(-dxe * dxe * a.e2) : 0.0f;
        gw[e] = gx * gy;
        gwd[e] = gw[e] * dxe;
        gwd2[e] = gwd[e] * dxe;
    }
    const unsigned col =
        (a.tiled ? (unsigned)((yy >> 2) * (Mx << 2) + ((xs >> 3) << 5) + ((yy & 3) << 3) + (xs & 7))
                 : (unsigned)yy * (unsigned)Mx + (unsigned)xs) *
        4u;
    // lanes whose row or chunk lies outside the support load nothing
    const bool need = rowok && 4 * c - off0 < MG && 4 * c + 3 - off0 >= 0;
    __syncthreads();
    const size_t M3 = (size_t)Mx * My * Mz;
    float P[3] = {0, 0, 0}, Rr[3] = {0, 0, 0}, PD2[3] = {0, 0, 0}, PD[2] = {0, 0}, Q[2] = {0, 0};
    for (int k = 0; k < MG; ++k) {
        int z = r.s[2] + k;
        while (z >= Mz) z -= Mz;   // the support may be longer than the z axis
        const ZTab<float> e = zt[wave][k];
        const float* pz = grid + (size_t)z * nplane;
        float4 u[3] = {make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0)};
        if (need && !split) {
            u[0] = plane_load4(pz, nplane, col);
            u[1] = plane_load4(pz + M3, nplane, col);
            u[2] = plane_load4(pz + 2 * M3, nplane, col);
        } else if (need) {
            // xs + e past the row end wraps back by Mx points (4 Mx bytes)
            const unsigned cw = col - 4u * (unsigned)Mx;
            const unsigned c1 = xs + 1 < Mx ? col + 4u : cw + 4u;
            const unsigned c2 = xs + 2 < Mx ? col + 8u : cw + 8u;
            const unsigned c3 = xs + 3 < Mx ? col + 12u : cw + 12u;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const float* pc = pz + cc * M3;
                u[cc] = make_float4(plane_load(pc, nplane, col), plane_load(pc, nplane, c1),
                                    plane_load(pc, nplane, c2), plane_load(pc, nplane, c3));
            }
        }
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            const float pc = gw[0] * u[cc].x + gw[1] * u[cc].y + gw[2] * u[cc].z + gw[3] * u[cc].w;
            const float rc = gwd2[0] * u[cc].x + gwd2[1] * u[cc].y + gwd2[2] * u[cc].z + gwd2[3] * u[cc].w;
            P[cc] += e.g * pc;
            Rr[cc] += e.g * rc;
            PD2[cc] += e.gd2 * pc;
            if (OMEGA) {
                if (cc < 2) PD[cc] += e.gDd * pc;
                if (cc > 0) {
                    const float qc = gwd[0] * u[cc].x + gwd[1] * u[cc].y + gwd[2] * u[cc].z + gwd[3] * u[cc].w;
                    Q[cc - 1] += e.g * qc;
                }
            }
        }
    }
    const float cy = a.A + a.B * dyv * dyv;
    float v0 = cy * P[0] + a.B * (Rr[0] + PD2[0]);
    float v1 = cy * P[1] + a.B * (Rr[1] + PD2[1]);
    float v2 = cy * P[2] + a.B * (Rr[2] + PD2[2]);
    float o0 = 0, o1 = 0, o2 = 0;
    if (OMEGA) {
        o0 = dyv * P[2] - PD[1];
        o1 = PD[0] - Q[1];
        o2 = Q[0] - dyv * P[0];
    }
    v0 = wave_sum(v0);
    v1 = wave_sum(v1);
    v2 = wave_sum(v2);
    if (OMEGA) {
        o0 = wave_sum(o0);
        o1 = wave_sum(o1);
        o2 = wave_sum(o2);
    }
    if (live && lane == 0) {
        const int64_t n = r.orig;
        double cv[3] = {0, 0, 0}, cw[3] = {0, 0, 0};
        if (corr) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                cv[d] = corr[3 * n + d];
                cw[d] = corr[3 * (int64_t)a.N + 3 * n + d];
            }
        }
        V[3 * n + 0] = (double)v0 * scaleV + cv[0];
        V[3 * n + 1] = (double)v1 * scaleV + cv[1];
        V[3 * n + 2] = (double)v2 * scaleV + cv[2];
        if (OMEGA) {
            W[3 * n + 0] = (double)o0 * scaleW + cw[0];
            W[3 * n + 1] = (double)o1 * scaleW + cw[1];
            W[3 * n + 2] = (double)o2 * scaleW + cw[2];
        }
    }
}

// FP32 interpolation with several particles per wavefront (M divisible by 4,
// M_G <= 16, Sigma_D = Sigma, one field component addressable with 32-bit byte
// offsets).  Lane 32 h + M_G g + j serves particle slot g (g < 32 / M_G, at
// most four slots), support row j and NQ quads of four x points counted from
// x0 & ~3 (NQ 16-byte loads): quad 2 l + h, l < NQ, taken cyclically from the
// parity of x0 >> 2, so the two lanes of a row read the two halves of one 8 x 4
// tile in each load where they can.  NQ = 2 covers 16 points (M_G <= 13), NQ =
// 3 covers 24 (M_G <= 16, two particles per wavefront); at M_G = 10 three
// particles share a wavefront and 60 of its 64 lanes work.  The per-lane sums
// follow the factorisation of k_interp4; the two lanes of a row are combined by
// one lane exchange, the rows of each particle through LDS, in a fixed order.
template <bool OMEGA, int NQ>
__global__ __launch_bounds__(256) void k_interp8(const GridRec<float>* __restrict__ rec,
                                                 const float* __restrict__ grid, double* __restrict__ V,
                                                 double* __restrict__ W, GridArgs<float> a,
                                                 double scaleV, double scaleW,
                                                 const double* __restrict__ corr) {
    constexpr int kSlots = 4;
    constexpr int NV = OMEGA ? 6 : 3;
    constexpr int NX = 4 * NQ;
    __shared__ ZTab<float> zt[4][kSlots][kMaxSupport];
    __shared__ float red[4][NV][32];
    __shared__ int origs[4][kSlots];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int Mx = a.M, My = a.My, Mz = a.Mz, MG = a.MG;
    const int ppw = min(kSlots, 32 / MG);
    const int h = lane >> 5, r = lane & 31;
    const int g = r / MG, j = r - g * MG;
    const bool slot = g < ppw;
    const int64_t pb = ((int64_t)xcd_remap(blockIdx.x, gridDim.x) * 4 + wave) * ppw;
    const int64_t p = pb + g;
    const bool live = slot && p < a.N;
    const GridRec<float> rv = rec[live ? p : a.N - 1];
    const int gz = slot ? g : 0;
    const float dx = a.dx;
    if (slot && h == 0) {
        ZTab<float> e = {0.0f, 0.0f, 0.0f, 0.0f};
        if (live) {
            const float d = ((float)j - rv.f[2]) * dx;
            const float d2 = d * d;
            e.g = fexp2(-d2 * a.e2);
            e.gd2 = e.g * d2;
            e.gD = e.g;
            e.gDd = e.g * d;
        }
        zt[wave][g][j] = e;
        if (j == 0) origs[wave][g] = rv.orig;
    }
    const int x0 = rv.s[0], off0 = x0 & 3;
    const int odd = (x0 >> 2) & 1;
    int yy = rv.s[1] + j;
    if (yy >= My) yy -= My;
    const float dyv = ((float)j - rv.f[1]) * dx;
    const float gy = fexp2(-dyv * dyv * a.e2);
    float gw[NX], gwd[NX], gwd2[NX];
    unsigned col[NQ];
    bool need[NQ];
#pragma unroll
    for (int l = 0; l < NQ; ++l) {
        const int o = (2 * l + h + odd) % (2 * NQ);
        int x = (x0 - off0) + 4 * o;
        if (x >= Mx) x -= Mx;
        col[l] = (a.tiled ? (unsigned)((yy >> 2) * (Mx << 2) + ((x >> 3) << 5) + ((yy & 3) << 3) + (x & 7))
                          : (unsigned)yy * (unsigned)Mx + (unsigned)x) *
                 4u;
        // quads of four x points that meet the support [0, M_G)
        need[l] = live && 4 * o - off0 < MG;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 4 * o + e - off0;
            const float dxe = ((float)i - rv.f[0]) * dx;
            const float gx = (i >= 0 && i < MG) ? fexp2(-dxe * dxe * a.e2) : 0.0f;
            gw[4 * l + e] = gx * gy;
            gwd[4 * l + e] = gw[4 * l + e] * dxe;
            gwd2[4 * l + e] = gwd[4 * l + e] * dxe;
        }
    }
    const size_t M3 = (size_t)Mx * My * Mz;
    const int bytes = (int)(M3 * sizeof(float));
    const __amdgpu_buffer_rsrc_t rs0 = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(grid), (short)0, bytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rs1 = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(grid + M3), (short)0, bytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rs2 = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(grid + 2 * M3), (short)0, bytes, kBufferWord3);
    const unsigned plane = (unsigned)Mx * (unsigned)My * 4u;
    int z = rv.s[2];
    unsigned zoff = (unsigned)z * plane;
    __syncthreads();
    float P[3] = {0, 0, 0}, Rr[3] = {0, 0, 0}, PD2[3] = {0, 0, 0}, PD[2] = {0, 0}, Q[2] = {0, 0};
    for (int k = 0; k < MG; ++k) {
        const ZTab<float> e = zt[wave][gz][k];
        float u[3][NX];
#pragma unroll
        for (int l = 0; l < NQ; ++l) {
            float4 q[3] = {make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0)};
            if (need[l]) {
                q[0] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs0, (int)(zoff + col[l]), 0, 0));
                q[1] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs1, (int)(zoff + col[l]), 0, 0));
                q[2] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs2, (int)(zoff + col[l]), 0, 0));
            }
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                u[cc][4 * l + 0] = q[cc].x;
                u[cc][4 * l + 1] = q[cc].y;
                u[cc][4 * l + 2] = q[cc].z;
                u[cc][4 * l + 3] = q[cc].w;
            }
        }
        if (++z == Mz) {
            z = 0;
            zoff = 0;
        } else {
            zoff += plane;
        }
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            float pc = 0.0f, rc = 0.0f;
#pragma unroll
            for (int t = 0; t < NX; ++t) {
                pc += gw[t] * u[cc][t];
                rc += gwd2[t] * u[cc][t];
            }
            P[cc] += e.g * pc;
            Rr[cc] += e.g * rc;
            PD2[cc] += e.gd2 * pc;
            if (OMEGA) {
                if (cc < 2) PD[cc] += e.gDd * pc;
                if (cc > 0) {
                    float qc = 0.0f;
#pragma unroll
                    for (int t = 0; t < NX; ++t) qc += gwd[t] * u[cc][t];
                    Q[cc - 1] += e.g * qc;
                }
            }
        }
    }
    const float cy = a.A + a.B * dyv * dyv;
    float vals[NV];
    vals[0] = cy * P[0] + a.B * (Rr[0] + PD2[0]);
    vals[1] = cy * P[1] + a.B * (Rr[1] + PD2[1]);
    vals[2] = cy * P[2] + a.B * (Rr[2] + PD2[2]);
    if constexpr (OMEGA) {
        vals[3] = dyv * P[2] - PD[1];
        vals[4] = PD[0] - Q[1];
        vals[5] = Q[0] - dyv * P[0];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) vals[v] += __shfl_xor(vals[v], 32, 64);
    if (h == 0 && slot) {
#pragma unroll
        for (int v = 0; v < NV; ++v) red[wave][v][r] = vals[v];
    }
    __syncthreads();
    if (lane < ppw * NV) {
        const int gg = lane / NV, v = lane - gg * NV;
        if (pb + gg < a.N) {
            float sum = 0.0f;
            for (int jj = 0; jj < MG; ++jj) sum += red[wave][v][gg * MG + jj];
            const int64_t n = origs[wave][gg];
            if (v < 3) {
                V[3 * n + v] = (double)sum * scaleV + (corr ? corr[3 * n + v] : 0.0);
            } else {
                W[3 * n + v - 3] = (double)sum * scaleW + (corr ? corr[3 * (int64_t)a.N + 3 * n + v - 3] : 0.0);
            }
        }
    }
}

template <typename R>
GridArgs<R> make_args(const fcm_plan_impl* P) {
    GridArgs<R> a;
    a.M = P->M;
    a.My = P->My;
    a.Mz = P->Mz;
    a.MG = P->MG;
    a.N = (int)P->N;
    a.TX = P->TX;
    a.TY = P->TY;
    a.rowrep = 0;
    for (int j = 0; j < P->TY; ++j) a.rowrep |= 1ull << (P->TX * j);
    a.TZ = P->TZ;
    a.nbx = P->nbx;
    a.nby = P->nby;
    a.nbz = P->nbz;
    a.backx = P->backx;
    a.backy = P->backy;
    a.backz = P->backz;
    a.mgmul = 65536 / P->MG + 1;
    a.tiled = 0;
    a.zfold = P->MG > P->Mz ? 1 : 0;
    a.dx = (R)P->dx;
    const double log2e = 1.4426950408889634074;
    a.e2 = (R)(log2e / (2.0 * P->Sigma * P->Sigma));
    a.e2D = (R)(log2e / (2.0 * P->SigmaD * P->SigmaD));
    const double c = 0.5 * (P->sigma * P->sigma - P->Sigma * P->Sigma);
    const double S2 = P->Sigma * P->Sigma;
    a.A = (R)(1.0 - 3.0 * c / S2);
    a.B = (R)(c / (S2 * S2));
    a.dV = (R)(P->dx * P->dx * P->dx);
    a.same_width = (P->SigmaD == P->Sigma) ? 1 : 0;
    return a;
}

template <typename R, int TZ, int MODE, bool TORQUE>
hipError_t spread_tz(const fcm_plan_impl* P, R* grid, hipStream_t st, bool tiled) {
    GridArgs<R> a = make_args<R>(P);
    a.tiled = tiled ? 1 : 0;
    const size_t shm = sizeof(Stage<R>) + kChunk * (size_t)P->MG * sizeof(ZTab<R>);
    dim3 g(P->nbins), b(64);
    const GridRec<R>* rec = (const GridRec<R>*)P->grec;
    if (a.same_width)
        hipLaunchKernelGGL((k_spread<R, TZ, MODE, TORQUE, true>), g, b, shm, st, rec, P->starts, grid, a);
    else
        hipLaunchKernelGGL((k_spread<R, TZ, MODE, TORQUE, false>), g, b, shm, st, rec, P->starts, grid, a);
    return hipGetLastError();
}

template <typename R, int MODE, bool TORQUE>
hipError_t spread_m(const fcm_plan_impl* P, R* grid, hipStream_t st, bool tiled) {
    switch (P->TZ) {
        case 16: return spread_tz<R, 16, MODE, TORQUE>(P, grid, st, tiled);
        case 12: return spread_tz<R, 12, MODE, TORQUE>(P, grid, st, tiled);
        case 8: return spread_tz<R, 8, MODE, TORQUE>(P, grid, st, tiled);
        case 6: return spread_tz<R, 6, MODE, TORQUE>(P, grid, st, tiled);
        case 4: return spread_tz<R, 4, MODE, TORQUE>(P, grid, st, tiled);
        case 2: return spread_tz<R, 2, MODE, TORQUE>(P, grid, st, tiled);
        case 1: return spread_tz<R, 1, MODE, TORQUE>(P, grid, st, tiled);
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int MODE>
hipError_t spread_r(const fcm_plan_impl* P, bool torque, R* grid, hipStream_t st, bool tiled) {
    return torque ? spread_m<R, MODE, true>(P, grid, st, tiled)
                  : spread_m<R, MODE, false>(P, grid, st, tiled);
}

template <typename R>
hipError_t interp_r(const fcm_plan_impl* P, const R* grid, double* V, double* W, hipStream_t st,
                    bool tiled, const double* corr) {
    GridArgs<R> a = make_args<R>(P);
    a.tiled = tiled ? 1 : 0;
    const double pi = 3.14159265358979323846;
    const double dV = P->dx * P->dx * P->dx;
    const double scaleV = dV * pow(2.0 * pi * P->Sigma * P->Sigma, -1.5);
    const double scaleW =
        dV * pow(2.0 * pi * P->SigmaD * P->SigmaD, -1.5) / (2.0 * P->SigmaD * P->SigmaD);
    dim3 g((unsigned)((P->N + 3) / 4)), b(256);
    const GridRec<R>* rec = (const GridRec<R>*)P->grec;
    if constexpr (sizeof(R) == sizeof(float)) {
        // Packed kernels need one width.  In the tiled layout the two lanes of
        // a support row read one 8 x 4 tile's halves per load, so several
        // particles per wavefront pay (M_G <= 16); in the row-major layout rows
        // are a plane row apart and the four-lane form reads fewest cache lines
        // per byte: aligned quads for M divisible by 4 and M_G <= 13, quads from
        // the support's first point otherwise (M_G <= 16).
        if (P->M % 4 == 0 && a.same_width && tiled && P->MG <= 16 &&
            (size_t)P->M * P->My * P->Mz <= (size_t)512 * 512 * 512) {
            const int ppw = std::min(4, 32 / P->MG);
            dim3 g8((unsigned)((P->N + 4 * ppw - 1) / (4 * ppw)));
            if (P->MG <= 13) {
                if (W == nullptr)
                    hipLaunchKernelGGL((k_interp8<false, 2>), g8, b, 0, st, rec, grid, V, W, a, scaleV, scaleW, corr);
                else
                    hipLaunchKernelGGL((k_interp8<true, 2>), g8, b, 0, st, rec, grid, V, W, a, scaleV, scaleW, corr);
            } else {
                if (W == nullptr)
                    hipLaunchKernelGGL((k_interp8<false, 3>), g8, b, 0, st, rec, grid, V, W, a, scaleV, scaleW, corr);
                else
                    hipLaunchKernelGGL((k_interp8<true, 3>), g8, b, 0, st, rec, grid, V, W, a, scaleV, scaleW, corr);
            }
            return hipGetLastError();
        }
        if (P->M % 4 == 0 && a.same_width && P->MG <= 13) {
            if (W == nullptr)
                hipLaunchKernelGGL(k_interp4<false>, g, b, 0, st, rec, grid, V, W, a, scaleV, scaleW, corr);
            else
                hipLaunchKernelGGL(k_interp4<true>, g, b, 0, st, rec, grid, V, W, a, scaleV, scaleW, corr);
            return hipGetLastError();
        }
        if (!tiled && a.same_width && P->MG <= 16 && P->M >= 4) {
            if (W == nullptr)
                hipLaunchKernelGGL((k_interp4<false, true>), g, b, 0, st, rec, grid, V, W, a, scaleV, scaleW, corr);
            else
                hipLaunchKernelGGL((k_interp4<true, true>), g, b, 0, st, rec, grid, V, W, a, scaleV, scaleW, corr);
            return hipGetLastError();
        }
    }
    if (W == nullptr)
        hipLaunchKernelGGL((k_interp<R, false, true>), g, b, 0, st, rec, grid, V, W, a, scaleV, scaleW, corr);
    else if (a.same_width)
        hipLaunchKernelGGL((k_interp<R, true, true>), g, b, 0, st, rec, grid, V, W, a, scaleV, scaleW, corr);
    else
        hipLaunchKernelGGL((k_interp<R, true, false>), g, b, 0, st, rec, grid, V, W, a, scaleV, scaleW, corr);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_spread(const fcm_plan_impl* P, bool torque, void* grid, hipStream_t st,
                         bool tiled) {
    if (P->precision == FCM_FP64)
        return spread_r<double, ACC_PLAIN>(P, torque, (double*)grid, st, tiled);
    if (P->kahan == 1) return spread_r<float, ACC_KAHAN>(P, torque, (float*)grid, st, tiled);
    if (P->kahan == 2) return spread_r<float, ACC_WIDE>(P, torque, (float*)grid, st, tiled);
    return spread_r<float, ACC_PLAIN>(P, torque, (float*)grid, st, tiled);
}

hipError_t launch_interp(const fcm_plan_impl* P, const void* grid, double* V, double* W,
                         hipStream_t st, bool tiled, const double* corr) {
    if (P->precision == FCM_FP64)
        return interp_r<double>(P, (const double*)grid, V, W, st, tiled, corr);
    return interp_r<float>(P, (const float*)grid, V, W, st, tiled, corr);
}

}  // namespace fcm
