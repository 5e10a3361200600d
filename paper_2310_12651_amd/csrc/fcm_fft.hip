// The Fourier Stokes solve of fast FCM (Sec. 2.1 step 2, App. A):
//   f -> f^ (3-D real-to-complex FFT) -> u^ = (I - k k^T/k^2) f^ / (eta k^2),
//   u^(0) = 0, modes with index M/2 on any axis set to 0 -> u (complex-to-real).
//
// Five passes over the field, each a batch of 1-D transforms held in LDS:
//   x : real-to-complex along x (half-length complex FFT + split), in place;
//       the x-Nyquist coefficient is not stored (it is zeroed by the solve),
//       so the spectrum (M/2 x M x M complex) has exactly the field's size;
//   y : forward complex FFT along y;
//   z : forward FFT along z, the projection, and the inverse FFT along z,
//       all three components of a pencil at once (the fused middle pass);
//   y : inverse complex FFT along y;
//   x : complex-to-real along x.
// Each 1-D transform is a mixed-radix (2, 3, 4, 8) Stockham autosort FFT:
// stage s with radix R reads x[j + r n/R], twiddles by exp(+-2 pi i r k/(Ns R))
// with k = j mod Ns, applies an R-point DFT and writes
// y[(j div Ns) Ns R + k + r Ns].  Every thread holds its butterflies of a
// stage in registers between a barrier-separated read and write, so a tile
// is transformed in place.
#include <utility>

#include "fcm_internal.h"

namespace fcm {

namespace {

constexpr int kFFTThreads = 256;

template <typename R>
__device__ inline C2<R> cadd(C2<R> a, C2<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ inline C2<R> csub(C2<R> a, C2<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ inline C2<R> cmul(C2<R> a, C2<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by DIR * i
template <int DIR, typename R>
__device__ inline C2<R> mul_i(C2<R> a) {
    return DIR < 0 ? C2<R>{a.y, -a.x} : C2<R>{-a.y, a.x};
}

template <typename R, int RAD, int DIR>
struct DFT;

template <typename R, int DIR>
struct DFT<R, 2, DIR> {
    static __device__ inline void run(C2<R>* v) {
        C2<R> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename R, int DIR>
struct DFT<R, 3, DIR> {
    static __device__ inline void run(C2<R>* v) {
        const R h = (R)0.86602540378443864676;  // sqrt(3)/2
        C2<R> a = v[0], s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        C2<R> m = {a.x - (R)0.5 * s.x, a.y - (R)0.5 * s.y};
        C2<R> t = mul_i<DIR>(C2<R>{h * d.x, h * d.y});
        v[0] = cadd(a, s);
        v[1] = cadd(m, t);
        v[2] = csub(m, t);
    }
};

template <typename R, int DIR>
struct DFT<R, 4, DIR> {
    static __device__ inline void run(C2<R>* v) {
        C2<R> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        C2<R> t2 = cadd(v[1], v[3]), t3 = mul_i<DIR>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[1] = cadd(t1, t3);
        v[2] = csub(t0, t2);
        v[3] = csub(t1, t3);
    }
};

template <typename R, int DIR>
struct DFT<R, 8, DIR> {
    static __device__ inline void run(C2<R>* v) {
        C2<R> e[4] = {v[0], v[2], v[4], v[6]};
        C2<R> o[4] = {v[1], v[3], v[5], v[7]};
        DFT<R, 4, DIR>::run(e);
        DFT<R, 4, DIR>::run(o);
        const R c = (R)0.70710678118654752440;
        // W8^k = exp(DIR 2 pi i k / 8)
        C2<R> w1 = {c, DIR * c}, w3 = {-c, DIR * c};
        C2<R> o1 = cmul(o[1], w1), o2 = mul_i<DIR>(o[2]), o3 = cmul(o[3], w3);
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
};

// One Stockham stage on an LDS tile of W lines of length n; element (w, idx)
// lives at buf[w * sw + idx * sn].  tw[m] = exp(-2 pi i m / M), n divides M.
// With wfast the line index w is the fastest-varying thread index (W = 2^lw).
template <typename R, int RAD, int DIR, int MAXB>
__device__ void fft_stage(C2<R>* buf, const C2<R>* tw, const RadixPlan& rp, int s, int W, int lw,
                          int sw, int sn, bool wfast) {
    const int nb = rp.nb[s];
    const unsigned nbm = rp.nbm[s];
    const int Ns = rp.ns[s];
    const unsigned nsm = rp.nsm[s];
    const int tstep = rp.tstep[s];
    const int total = nb * W;
    const int tid = threadIdx.x;
    C2<R> v[MAXB][RAD];
    int jj[MAXB], ww[MAXB];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int t = tid + q * kFFTThreads;
        jj[q] = 0;
        ww[q] = 0;
        if (t < total) {
            int w, j;
            if (wfast) {
                w = t & (W - 1);
                j = t >> lw;
            } else {
                w = fast_div(t, nb, nbm);
                j = t - w * nb;
            }
            jj[q] = j;
            ww[q] = w;
#pragma unroll
            for (int r = 0; r < RAD; ++r) v[q][r] = buf[w * sw + (j + r * nb) * sn];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int t = tid + q * kFFTThreads;
        if (t < total) {
            const int j = jj[q], w = ww[q];
            const int jd = fast_div(j, Ns, nsm);
            const int k = j - jd * Ns;
#pragma unroll
            for (int r = 1; r < RAD; ++r) {
                C2<R> f = tw[r * k * tstep];
                if (DIR > 0) f.y = -f.y;
                v[q][r] = cmul(v[q][r], f);
            }
            DFT<R, RAD, DIR>::run(v[q]);
            const int o = jd * Ns * RAD + k;
#pragma unroll
            for (int r = 0; r < RAD; ++r) buf[w * sw + (o + r * Ns) * sn] = v[q][r];
        }
    }
    __syncthreads();
}

template <typename R, int DIR, int MAXE>
__device__ void fft_lines(C2<R>* buf, const C2<R>* tw, const RadixPlan& rp, int W, int lw, int sw,
                          int sn, bool wfast) {
    for (int s = 0; s < rp.nst; ++s) {
        switch (rp.rad[s]) {
            case 2: fft_stage<R, 2, DIR, (MAXE + 1) / 2>(buf, tw, rp, s, W, lw, sw, sn, wfast); break;
            case 3: fft_stage<R, 3, DIR, (MAXE + 2) / 3>(buf, tw, rp, s, W, lw, sw, sn, wfast); break;
            case 4: fft_stage<R, 4, DIR, (MAXE + 3) / 4>(buf, tw, rp, s, W, lw, sw, sn, wfast); break;
            default: fft_stage<R, 8, DIR, (MAXE + 7) / 8>(buf, tw, rp, s, W, lw, sw, sn, wfast); break;
        }
    }
}

template <typename R>
__device__ inline void load_twiddles(C2<R>* tw, const C2<R>* __restrict__ twg, int M) {
    for (int e = threadIdx.x; e < M; e += kFFTThreads) tw[e] = twg[e];
}

// x pass, forward: Wx real lines of length M per block -> M/2 complex each
template <typename R, int MAXE>
__global__ __launch_bounds__(kFFTThreads) void k_fft_x_r2c(R* __restrict__ grid,
                                                           const C2<R>* __restrict__ twg, int M,
                                                           RadixPlan rpH, int Wx, int nlines) {
    extern __shared__ __align__(16) unsigned char smem[];
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem);
    C2<R>* buf = tw + M;
    const int H = M / 2, sw = H + 1;
    const int line0 = xcd_remap(blockIdx.x, gridDim.x) * Wx;
    C2<R>* g = reinterpret_cast<C2<R>*>(grid);
    load_twiddles(tw, twg, M);
    for (int e = threadIdx.x; e < Wx * H; e += kFFTThreads) {
        const int w = fast_div(e, H, rpH.nm), m = e - w * H, l = line0 + w;
        buf[w * sw + m] = (l < nlines) ? g[(size_t)l * H + m] : C2<R>{0, 0};
    }
    __syncthreads();
    fft_lines<R, -1, MAXE>(buf, tw, rpH, Wx, 0, sw, 1, false);
    for (int e = threadIdx.x; e < Wx * H; e += kFFTThreads) {
        const int w = fast_div(e, H, rpH.nm), k = e - w * H, l = line0 + w;
        if (l >= nlines) continue;
        const C2<R> Z = buf[w * sw + k];
        C2<R> Zc = buf[w * sw + (k == 0 ? 0 : H - k)];
        Zc.y = -Zc.y;
        const C2<R> S = cadd(Z, Zc), D = csub(Z, Zc);
        const C2<R> WD = cmul(tw[k], D);  // exp(-2 pi i k/M) (Z_k - conj Z_{H-k})
        g[(size_t)l * H + k] = C2<R>{(R)0.5 * (S.x + WD.y), (R)0.5 * (S.y - WD.x)};
    }
}

// x pass, inverse: M/2 complex (x-Nyquist taken as 0) -> M reals, unnormalised
template <typename R, int MAXE>
__global__ __launch_bounds__(kFFTThreads) void k_fft_x_c2r(R* __restrict__ grid,
                                                           const C2<R>* __restrict__ twg, int M,
                                                           RadixPlan rpH, int Wx, int nlines) {
    extern __shared__ __align__(16) unsigned char smem[];
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem);
    C2<R>* buf = tw + M;
    const int H = M / 2, sw = H + 1;
    const int line0 = xcd_remap(blockIdx.x, gridDim.x) * Wx;
    C2<R>* g = reinterpret_cast<C2<R>*>(grid);
    load_twiddles(tw, twg, M);
    for (int e = threadIdx.x; e < Wx * H; e += kFFTThreads) {
        const int w = fast_div(e, H, rpH.nm), m = e - w * H, l = line0 + w;
        buf[w * sw + m] = (l < nlines) ? g[(size_t)l * H + m] : C2<R>{0, 0};
    }
    __syncthreads();
    C2<R> zr[MAXE];
#pragma unroll
    for (int q = 0; q < MAXE; ++q) {
        const int e = threadIdx.x + q * kFFTThreads;
        if (e < Wx * H) {
            const int w = fast_div(e, H, rpH.nm), k = e - w * H;
            const C2<R> X = buf[w * sw + k];
            C2<R> Xc = {0, 0};
            if (k > 0) {
                Xc = buf[w * sw + H - k];
                Xc.y = -Xc.y;
            }
            const C2<R> E = cadd(X, Xc);
            C2<R> wk = tw[k];
            wk.y = -wk.y;  // exp(+2 pi i k / M)
            const C2<R> O = cmul(csub(X, Xc), wk);
            zr[q] = C2<R>{E.x - O.y, E.y + O.x};
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXE; ++q) {
        const int e = threadIdx.x + q * kFFTThreads;
        if (e < Wx * H) {
            const int w = fast_div(e, H, rpH.nm);
            buf[w * sw + (e - w * H)] = zr[q];
        }
    }
    __syncthreads();
    fft_lines<R, 1, MAXE>(buf, tw, rpH, Wx, 0, sw, 1, false);
    for (int e = threadIdx.x; e < Wx * H; e += kFFTThreads) {
        const int w = fast_div(e, H, rpH.nm), m = e - w * H, l = line0 + w;
        if (l < nlines) g[(size_t)l * H + m] = buf[w * sw + m];
    }
}

// y pass: batches of W consecutive kx columns of one (component, z) plane
// (lines of length M = My; H = the x half-length, the number of kx columns)
template <typename R, int DIR, int MAXE>
__global__ __launch_bounds__(kFFTThreads) void k_fft_y(C2<R>* __restrict__ spec,
                                                       const C2<R>* __restrict__ twg, int M, int H,
                                                       RadixPlan rpM, int W, int lw) {
    extern __shared__ __align__(16) unsigned char smem[];
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem);
    C2<R>* buf = tw + M;
    const int ng = (H + W - 1) / W;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g = blk % ng;
    const int rest = blk / ng;  // c * Mz + z
    const int kx0 = g * W;
    const int Wv = min(W, H - kx0);
    C2<R>* base = spec + (size_t)rest * M * H + kx0;
    load_twiddles(tw, twg, M);
    for (int e = threadIdx.x; e < W * M; e += kFFTThreads) {
        const int w = e & (W - 1), y = e >> lw;
        buf[e] = (w < Wv) ? base[(size_t)y * H + w] : C2<R>{0, 0};
    }
    __syncthreads();
    fft_lines<R, DIR, MAXE>(buf, tw, rpM, W, lw, 1, W, true);
    for (int e = threadIdx.x; e < W * M; e += kFFTThreads) {
        const int w = e & (W - 1), y = e >> lw;
        if (w < Wv) base[(size_t)y * H + w] = buf[e];
    }
}

struct ProjArgs {
    double kux, kuy, kuz;   // 2 pi / L along x, y, z
    double scale;           // 1 / (eta Mx My Mz); square root: 1 / (sqrt(eta) Mx My Mz)
    int root;               // multiply by P(k) / sqrt(eta k^2) instead of P(k) / (eta k^2)
};

// z pass: forward FFT along z, projection / (eta k^2), inverse FFT along z
// (lines of length M = Mz over the H x My columns (kx, ky), H = Mx / 2)
template <typename R, int MAXE>
__global__ __launch_bounds__(kFFTThreads) void k_fft_z_solve(C2<R>* __restrict__ spec,
                                                             const C2<R>* __restrict__ twg, int M,
                                                             int H, int My, RadixPlan rpM, int W,
                                                             int lw, ProjArgs pa) {
    extern __shared__ __align__(16) unsigned char smem[];
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem);
    C2<R>* buf = tw + M;  // 3 components, each M x W
    const int ng = (H + W - 1) / W;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g = blk % ng;
    const int y = blk / ng;
    const int kx0 = g * W;
    const int Wv = min(W, H - kx0);
    const size_t cstride = (size_t)M * My * H;
    const size_t zstride = (size_t)My * H;
    C2<R>* base = spec + (size_t)y * H + kx0;
    load_twiddles(tw, twg, M);
    for (int e = threadIdx.x; e < W * M; e += kFFTThreads) {
        const int w = e & (W - 1), z = e >> lw;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            buf[c * M * W + e] = (w < Wv) ? base[c * cstride + (size_t)z * zstride + w] : C2<R>{0, 0};
    }
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < 3; ++c) fft_lines<R, -1, MAXE>(buf + c * M * W, tw, rpM, W, lw, 1, W, true);
    const R kux = (R)pa.kux, kuy = (R)pa.kuy, kuz = (R)pa.kuz;
    const R sc = (R)pa.scale;
    const int Hy = My / 2, Hz = M / 2;
    const int jy = y < Hy ? y : y - My;
    for (int e = threadIdx.x; e < W * M; e += kFFTThreads) {
        const int w = e & (W - 1), z = e >> lw;
        const int jx = kx0 + w;
        const int jz = z < Hz ? z : z - M;
        const bool zero = (w >= Wv) || (y == Hy) || (z == Hz) || (jx == 0 && jy == 0 && jz == 0);
        C2<R> f0 = buf[e], f1 = buf[M * W + e], f2 = buf[2 * M * W + e];
        C2<R> u0 = {0, 0}, u1 = {0, 0}, u2 = {0, 0};
        if (!zero) {
            const R kx = kux * (R)jx, ky = kuy * (R)jy, kz = kuz * (R)jz;
            const R k2 = kx * kx + ky * ky + kz * kz;
            const R ik2 = (R)1 / k2;
            const C2<R> kf = {(kx * f0.x + ky * f1.x + kz * f2.x) * ik2,
                              (kx * f0.y + ky * f1.y + kz * f2.y) * ik2};
            const R s = pa.root ? sc * sqrt(ik2) : sc * ik2;
            u0 = C2<R>{(f0.x - kx * kf.x) * s, (f0.y - kx * kf.y) * s};
            u1 = C2<R>{(f1.x - ky * kf.x) * s, (f1.y - ky * kf.y) * s};
            u2 = C2<R>{(f2.x - kz * kf.x) * s, (f2.y - kz * kf.y) * s};
        }
        buf[e] = u0;
        buf[M * W + e] = u1;
        buf[2 * M * W + e] = u2;
    }
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < 3; ++c) fft_lines<R, 1, MAXE>(buf + c * M * W, tw, rpM, W, lw, 1, W, true);
    for (int e = threadIdx.x; e < W * M; e += kFFTThreads) {
        const int w = e & (W - 1), z = e >> lw;
        if (w < Wv) {
#pragma unroll
            for (int c = 0; c < 3; ++c) base[c * cstride + (size_t)z * zstride + w] = buf[c * M * W + e];
        }
    }
}

// ---- register-resident transforms (FP32) ----
//
// A transform of length N = N1 N2 (N2 dividing N1, C = N1 / N2) is done by N2
// threads per line: thread p holds the N1 elements x[p + N2 j], transforms
// them in registers (an N1-point DFT), multiplies by exp(+-2 pi i p k1 / N),
// and one LDS exchange hands it the N2 values of each of the C indices
// k1 = p + N2 s; C N2-point DFTs in registers give X[k1 + N1 k2] = X[p + N2 i]
// with i = s + C k2 (four-step Cooley-Tukey).  Input and output share the
// layout "thread p holds the indices congruent to p modulo N2", so the same
// routine runs forward and inverse transforms in either pass order.  Each
// element crosses LDS once per transform instead of once per radix stage.

// cos and sin of 2 pi m / n at compile time: exact quadrant reduction, then
// Taylor series on [0, pi/2)
constexpr double ct_sin_q(double x) {
    double t = x, s = x;
    for (int i = 1; i < 16; ++i) {
        t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
        s += t;
    }
    return s;
}
constexpr double ct_cos_q(double x) {
    double t = 1.0, s = 1.0;
    for (int i = 1; i < 16; ++i) {
        t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        s += t;
    }
    return s;
}
constexpr double ct_cos(long m, long n) {
    m %= n;
    if (m < 0) m += n;
    const long q = (4 * m) / n, r = 4 * m - q * n;
    const double x = 1.57079632679489661923 * (double)r / (double)n;
    return q == 0 ? ct_cos_q(x) : q == 1 ? -ct_sin_q(x) : q == 2 ? -ct_cos_q(x) : ct_sin_q(x);
}
constexpr double ct_sin(long m, long n) {
    m %= n;
    if (m < 0) m += n;
    const long q = (4 * m) / n, r = 4 * m - q * n;
    const double x = 1.57079632679489661923 * (double)r / (double)n;
    return q == 0 ? ct_sin_q(x) : q == 1 ? ct_cos_q(x) : q == 2 ? -ct_sin_q(x) : -ct_cos_q(x);
}

// v * exp(DIR 2 pi i K / N), K and N compile-time
template <typename R, int N, int DIR, int K>
__device__ inline C2<R> twc(C2<R> v) {
    if constexpr (K % N == 0) {
        return v;
    } else {
        constexpr double c = ct_cos(K, N), sn = DIR * ct_sin(K, N);
        return C2<R>{v.x * (R)c - v.y * (R)sn, v.x * (R)sn + v.y * (R)c};
    }
}

template <int... I, typename F>
__device__ inline void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ inline void static_for(F&& f) {
    static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// in-register DFT of length N (natural order in and out)
template <typename R, int N, int DIR>
struct RDFT {
    static constexpr int P = (N % 4 == 0) ? 4 : ((N % 2 == 0) ? 2 : 3);
    static constexpr int S = N / P;
    static __device__ inline void run(C2<R>* x) {
        C2<R> e[P][S];
#pragma unroll
        for (int r = 0; r < P; ++r)
#pragma unroll
            for (int m = 0; m < S; ++m) e[r][m] = x[P * m + r];
#pragma unroll
        for (int r = 0; r < P; ++r) RDFT<R, S, DIR>::run(e[r]);
        static_for<S>([&](auto k) {
            C2<R> t[P];
            static_for<P>([&](auto r) {
                constexpr int rk = decltype(r)::value * decltype(k)::value;
                t[decltype(r)::value] = twc<R, N, DIR, rk>(e[decltype(r)::value][decltype(k)::value]);
            });
            DFT<R, P, DIR>::run(t);
#pragma unroll
            for (int q = 0; q < P; ++q) x[decltype(k)::value + S * q] = t[q];
        });
    }
};
template <typename R, int DIR>
struct RDFT<R, 1, DIR> {
    static __device__ inline void run(C2<R>*) {}
};
template <typename R, int DIR>
struct RDFT<R, 2, DIR> {
    static __device__ inline void run(C2<R>* x) { DFT<R, 2, DIR>::run(x); }
};
template <typename R, int DIR>
struct RDFT<R, 3, DIR> {
    static __device__ inline void run(C2<R>* x) { DFT<R, 3, DIR>::run(x); }
};
template <typename R, int DIR>
struct RDFT<R, 4, DIR> {
    static __device__ inline void run(C2<R>* x) { DFT<R, 4, DIR>::run(x); }
};
template <typename R, int DIR>
struct RDFT<R, 8, DIR> {
    static __device__ inline void run(C2<R>* x) { DFT<R, 8, DIR>::run(x); }
};

__device__ inline C2<float> buf_load(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    return __builtin_bit_cast(C2<float>, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}
__device__ inline void buf_store(C2<float> v, __amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), rs, voff, soff, 0);
}

// One four-step transform per thread group (see above).  v: in v[j] =
// x[p + N2 j], out v[i] = X[p + N2 i].  tw: table of exp(-2 pi i m / (N TS)).
// E: this group's exchange buffer; element (k1, p) at E[k1 ES + p EP].
template <int N1, int N2, int DIR, int TS>
__device__ inline void four_step(C2<float>* v, const C2<float>* tw, C2<float>* E, int p, int ES,
                                 int EP) {
    constexpr int C = N1 / N2;
    static_assert(C * N2 == N1, "N2 must divide N1");
    RDFT<float, N1, DIR>::run(v);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
        C2<float> t = tw[p * k1 * TS];
        if (DIR > 0) t.y = -t.y;
        v[k1] = cmul(v[k1], t);
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) E[k1 * ES + p * EP] = v[k1];
    __syncthreads();
    C2<float> u[C][N2];
#pragma unroll
    for (int s2 = 0; s2 < C; ++s2)
#pragma unroll
        for (int j2 = 0; j2 < N2; ++j2) u[s2][j2] = E[(p + N2 * s2) * ES + j2 * EP];
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < C; ++s2) RDFT<float, N2, DIR>::run(u[s2]);
#pragma unroll
    for (int i = 0; i < N1; ++i) v[i] = u[i % C][i / C];
}

// y and z passes: W adjacent kx columns per workgroup, N2 threads per column
template <int N1, int N2, int W>
struct ColGeom {
    static constexpr int M = N1 * N2;
    static constexpr int H = M / 2;
    static constexpr int NT = W * N2;        // threads per block
    static constexpr int PL = N2 * W + 8;    // exchange-buffer stride of k1 (complex)
    static constexpr int NG = H / W;         // column groups per kx row
    static_assert(H % W == 0, "W must divide M/2");
    static_assert(NT <= 256, "block size");
};

// y pass: one (component, z) plane and W kx columns per block
template <int N1, int N2, int W, int DIR>
__global__ __launch_bounds__(W * N2) void k_fft_y_reg(C2<float>* __restrict__ spec,
                                                      const C2<float>* __restrict__ twg) {
    using G = ColGeom<N1, N2, W>;
    __shared__ C2<float> tw[G::M];
    __shared__ C2<float> E[N1 * G::PL];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g = blk % G::NG, plane = blk / G::NG;
    const int w = threadIdx.x % W, p = threadIdx.x / W;
    char* base = (char*)(spec + (size_t)plane * G::M * G::H + g * W);
    const unsigned lo = ((unsigned)p * G::H + (unsigned)w) * 8u;
    auto at = [&](unsigned off) -> C2<float>& { return *(C2<float>*)(base + off); };
    for (int e = threadIdx.x; e < G::M; e += G::NT) tw[e] = twg[e];
    C2<float> v[N1];
#pragma unroll
    for (int j = 0; j < N1; ++j) v[j] = at(lo + j * N2 * G::H * 8u);
    __syncthreads();
    four_step<N1, N2, DIR, 1>(v, tw, E + w, p, G::PL, W);
#pragma unroll
    for (int i = 0; i < N1; ++i) at(lo + i * N2 * G::H * 8u) = v[i];
}

// z pass: forward FFT along z of the three components of W kx columns at one
// ky, the projection, and the inverse FFT along z
template <int N1, int N2, int W>
__global__ __launch_bounds__(W * N2) void k_fft_z_solve_reg(C2<float>* __restrict__ spec,
                                                            const C2<float>* __restrict__ twg,
                                                            ProjArgs pa) {
    using G = ColGeom<N1, N2, W>;
    constexpr int M = G::M, H = G::H;
    __shared__ C2<float> tw[M];
    __shared__ C2<float> E[N1 * G::PL];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g = blk % G::NG, y = blk / G::NG;
    const int w = threadIdx.x % W, p = threadIdx.x / W;
    // Buffer loads and stores: one 32-bit lane offset plus a scalar offset per
    // element, instead of a 64-bit address per element held in registers.
    static_assert((unsigned long long)3 * M * M * H * 8 < (1ull << 31), "offsets exceed 31 bits");
    constexpr int cstride = M * M * H * 8, zstride = M * H * 8;
    C2<float>* base = spec + (size_t)y * H + g * W;
    const int nbytes = (int)(((size_t)3 * M * M * H - ((size_t)y * H + g * W)) * 8);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, nbytes, kBufferWord3);
    const int lo = p * zstride + w * 8;
    for (int e = threadIdx.x; e < M; e += G::NT) tw[e] = twg[e];
    C2<float> v[3][N1];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < N1; ++j) v[c][j] = buf_load(rs, lo, c * cstride + j * N2 * zstride);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) four_step<N1, N2, -1, 1>(v[c], tw, E + w, p, G::PL, W);
    // projection: u^ = (I - k k^T / k^2) f^ / (eta k^2 M^3); k = 0 and index-H modes -> 0
    const float kux = (float)pa.kux, kuy = (float)pa.kuy, kuz = (float)pa.kuz, sc = (float)pa.scale;
    const int jx = g * W + w;
    const int jy = y < H ? y : y - M;
    const float kx = kux * (float)jx, ky = kuy * (float)jy;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
        const int iz = p + N2 * i;
        const int jz = iz < H ? iz : iz - M;
        const bool zero = (y == H) || (iz == H) || (jx == 0 && jy == 0 && jz == 0);
        const float kz = kuz * (float)jz;
        const float k2s = kx * kx + ky * ky + kz * kz;
        const float ik2 = zero ? 0.0f : 1.0f / k2s;
        const C2<float> f0 = v[0][i], f1 = v[1][i], f2 = v[2][i];
        const C2<float> kf = {(kx * f0.x + ky * f1.x + kz * f2.x) * ik2,
                              (kx * f0.y + ky * f1.y + kz * f2.y) * ik2};
        const float s = pa.root ? sc * sqrtf(ik2) : sc * ik2;
        v[0][i] = C2<float>{(f0.x - kx * kf.x) * s, (f0.y - kx * kf.y) * s};
        v[1][i] = C2<float>{(f1.x - ky * kf.x) * s, (f1.y - ky * kf.y) * s};
        v[2][i] = C2<float>{(f2.x - kz * kf.x) * s, (f2.y - kz * kf.y) * s};
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) four_step<N1, N2, 1, 1>(v[c], tw, E + w, p, G::PL, W);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < N1; ++i) buf_store(v[c][i], rs, lo, c * cstride + i * N2 * zstride);
}

// z pass with one thread group per component: W kx columns at one ky, N2
// threads per column and component (3 W N2 threads).  Each thread transforms
// one component's line; the projection runs on the tile in LDS with the
// arithmetic of k_fft_z_solve_reg for each element.  A thread holds N1
// values instead of 3 N1, so the lines of 216-432 points fit in registers.
template <int N1, int N2, int W>
struct ZGeom3 {
    static constexpr int M = N1 * N2;
    static constexpr int H = M / 2;
    static constexpr int GT = W * N2;        // threads per component group
    static constexpr int NT = 3 * GT;        // threads per block
    static constexpr int PL = N2 * W + 8;    // exchange-buffer stride of k1 (complex)
    static constexpr int EL = N1 * PL;       // one component's exchange buffer
    static constexpr int NG = H / W;         // column groups per kx row
    static_assert(H % W == 0, "W must divide M/2");
    static_assert(NT <= 1024, "block size");
};

template <int N1, int N2, int W>
__global__ __launch_bounds__(3 * W * N2) void k_fft_z_solve_3g(
    C2<float>* __restrict__ spec, const C2<float>* __restrict__ twg, ProjArgs pa) {
    using G = ZGeom3<N1, N2, W>;
    constexpr int M = G::M, H = G::H, PL = G::PL, EL = G::EL;
    __shared__ C2<float> tw[M];
    __shared__ C2<float> E[3 * EL];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g = blk % G::NG, y = blk / G::NG;
    const int c = threadIdx.x / G::GT;
    const int t = threadIdx.x - c * G::GT;
    const int w = t % W, p = t / W;
    static_assert((unsigned long long)3 * M * M * H * 8 < (1ull << 31), "offsets exceed 31 bits");
    constexpr int cstride = M * M * H * 8, zstride = M * H * 8;
    C2<float>* base = spec + (size_t)y * H + g * W;
    const int nbytes = (int)(((size_t)3 * M * M * H - ((size_t)y * H + g * W)) * 8);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, nbytes, kBufferWord3);
    const int lo = c * cstride + p * zstride + w * 8;
    for (int e = threadIdx.x; e < M; e += G::NT) tw[e] = twg[e];
    C2<float> v[N1];
#pragma unroll
    for (int j = 0; j < N1; ++j) v[j] = buf_load(rs, lo, j * N2 * zstride);
    __syncthreads();
    C2<float>* Ec = E + c * EL + w;
    four_step<N1, N2, -1, 1>(v, tw, Ec, p, PL, W);
    // projection: u^ = (I - k k^T / k^2) f^ / (eta k^2 M^3); k = 0 and index-H modes -> 0.
    // The coefficients go to LDS and every thread projects elements of the
    // tile, all three components at a time; the lines' registers are free
    // meanwhile.
#pragma unroll
    for (int i = 0; i < N1; ++i) Ec[i * PL + p * W] = v[i];
    __syncthreads();
    const float kux = (float)pa.kux, kuy = (float)pa.kuy, kuz = (float)pa.kuz, sc = (float)pa.scale;
    const int jy = y < H ? y : y - M;
    const float ky = kuy * (float)jy;
    constexpr int LW = N2 * W;   // elements of one k1 row of the tile
#pragma unroll 2
    for (int e = threadIdx.x; e < N1 * LW; e += G::NT) {
        const int i = e / LW, r = e - i * LW;
        const int pp = r / W, ww = r - pp * W;
        const int o = i * PL + pp * W + ww;
        const int jx = g * W + ww;
        const int iz = pp + N2 * i;
        const int jz = iz < H ? iz : iz - M;
        const bool zero = (y == H) || (iz == H) || (jx == 0 && jy == 0 && jz == 0);
        const float kx = kux * (float)jx, kz = kuz * (float)jz;
        const float k2s = kx * kx + ky * ky + kz * kz;
        const float ik2 = zero ? 0.0f : 1.0f / k2s;
        const C2<float> f0 = E[o], f1 = E[EL + o], f2 = E[2 * EL + o];
        const C2<float> kf = {(kx * f0.x + ky * f1.x + kz * f2.x) * ik2,
                              (kx * f0.y + ky * f1.y + kz * f2.y) * ik2};
        const float s = pa.root ? sc * sqrtf(ik2) : sc * ik2;
        E[o] = C2<float>{(f0.x - kx * kf.x) * s, (f0.y - kx * kf.y) * s};
        E[EL + o] = C2<float>{(f1.x - ky * kf.x) * s, (f1.y - ky * kf.y) * s};
        E[2 * EL + o] = C2<float>{(f2.x - kz * kf.x) * s, (f2.y - kz * kf.y) * s};
    }
    __syncthreads();
    // each thread reads back the slots its own exchange writes next: no barrier
#pragma unroll
    for (int i = 0; i < N1; ++i) v[i] = Ec[i * PL + p * W];
    four_step<N1, N2, 1, 1>(v, tw, Ec, p, PL, W);
#pragma unroll
    for (int i = 0; i < N1; ++i) buf_store(v[i], rs, lo, i * N2 * zstride);
}

// Four-step transform of length N = N1 N2 for any N1, N2 (N2 need not divide
// N1): a line has LT = max(N1, N2) threads t.  In: threads t < N2 hold
// r[j] = x[t + N2 j], j < N1; they do the N1-point DFTs and twiddle by
// exp(-+2 pi i t k1 / N), then threads t < N1 take the N2 values of k1 = t
// through LDS and do the N2-point DFTs.  Out: threads t < N1 hold
// r[k2] = X[t + N1 k2], k2 < N2.  E: element (k1, a) at E[k1 ES + a EP].
template <int N1, int N2, int DIR>
__device__ inline void four_step_split(C2<float>* r, const C2<float>* tw, C2<float>* E, int t, int ES,
                                       int EP) {
    if (t < N2) {
        RDFT<float, N1, DIR>::run(r);
#pragma unroll
        for (int k1 = 1; k1 < N1; ++k1) {
            C2<float> f = tw[t * k1];
            if (DIR > 0) f.y = -f.y;
            r[k1] = cmul(r[k1], f);
        }
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) E[k1 * ES + t * EP] = r[k1];
    }
    __syncthreads();
    if (t < N1) {
#pragma unroll
        for (int a = 0; a < N2; ++a) r[a] = E[t * ES + a * EP];
        RDFT<float, N2, DIR>::run(r);
    }
    __syncthreads();
}

// z pass with one thread group per component, each line split N = N1 N2 as
// in four_step_split (W kx columns at one ky; 3 W max(N1, N2) threads).  The
// forward coefficients go to a tile in LDS in natural z order, the projection
// runs on the tile with the arithmetic of k_fft_z_solve_reg, and each thread
// reads back the input layout of the (inverse) split transform.
template <int N1, int N2, int W>
struct ZGeomSplit {
    static constexpr int M = N1 * N2;
    static constexpr int H = M / 2;
    static constexpr int LT = N1 > N2 ? N1 : N2;   // threads per line
    static constexpr int GT = W * LT;               // threads per component group
    static constexpr int NT = 3 * GT;               // threads per block
    static constexpr int ES = N2 * W + 8;           // exchange: k1 stride (complex)
    static constexpr int EC = (N1 * ES > M * W ? N1 * ES : M * W);   // one component's LDS
    static constexpr int NG = H / W;
    static_assert(H % W == 0, "W must divide M/2");
    static_assert(NT <= 1024, "block size");
};

template <int N1, int N2, int W>
__global__ __launch_bounds__(3 * W * (N1 > N2 ? N1 : N2)) void k_fft_z_solve_split(
    C2<float>* __restrict__ spec, const C2<float>* __restrict__ twg, ProjArgs pa) {
    using G = ZGeomSplit<N1, N2, W>;
    constexpr int M = G::M, H = G::H, LT = G::LT, ES = G::ES, EC = G::EC;
    __shared__ C2<float> tw[M];
    __shared__ C2<float> E[3 * EC];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int g = blk % G::NG, y = blk / G::NG;
    const int c = threadIdx.x / G::GT;
    const int tt = threadIdx.x - c * G::GT;
    const int w = tt % W, t = tt / W;
    static_assert((unsigned long long)3 * M * M * H * 8 < (1ull << 31), "offsets exceed 31 bits");
    constexpr int cstride = M * M * H * 8, zstride = M * H * 8;
    C2<float>* base = spec + (size_t)y * H + g * W;
    const int nbytes = (int)(((size_t)3 * M * M * H - ((size_t)y * H + g * W)) * 8);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, nbytes, kBufferWord3);
    const int lo = c * cstride + t * zstride + w * 8;
    for (int e = threadIdx.x; e < M; e += G::NT) tw[e] = twg[e];
    C2<float> r[LT];
    if (t < N2) {
#pragma unroll
        for (int j = 0; j < N1; ++j) r[j] = buf_load(rs, lo, j * N2 * zstride);
    }
    __syncthreads();
    C2<float>* Ec = E + c * EC + w;
    four_step_split<N1, N2, -1>(r, tw, Ec, t, ES, W);
    // the coefficients in natural z order: (z, column) at Ec[z W]
    if (t < N1) {
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) Ec[(t + N1 * k2) * W] = r[k2];
    }
    __syncthreads();
    // projection: u^ = (I - k k^T / k^2) f^ / (eta k^2 M^3); k = 0 and index-H modes -> 0
    const float kux = (float)pa.kux, kuy = (float)pa.kuy, kuz = (float)pa.kuz, sc = (float)pa.scale;
    const int jy = y < H ? y : y - M;
    const float ky = kuy * (float)jy;
#pragma unroll 2
    for (int e = threadIdx.x; e < M * W; e += G::NT) {
        const int iz = e / W, ww = e - iz * W;
        const int jx = g * W + ww;
        const int jz = iz < H ? iz : iz - M;
        const bool zero = (y == H) || (iz == H) || (jx == 0 && jy == 0 && jz == 0);
        const float kx = kux * (float)jx, kz = kuz * (float)jz;
        const float k2s = kx * kx + ky * ky + kz * kz;
        const float ik2 = zero ? 0.0f : 1.0f / k2s;
        const C2<float> f0 = E[e], f1 = E[EC + e], f2 = E[2 * EC + e];
        const C2<float> kf = {(kx * f0.x + ky * f1.x + kz * f2.x) * ik2,
                              (kx * f0.y + ky * f1.y + kz * f2.y) * ik2};
        const float s = pa.root ? sc * sqrtf(ik2) : sc * ik2;
        E[e] = C2<float>{(f0.x - kx * kf.x) * s, (f0.y - kx * kf.y) * s};
        E[EC + e] = C2<float>{(f1.x - ky * kf.x) * s, (f1.y - ky * kf.y) * s};
        E[2 * EC + e] = C2<float>{(f2.x - kz * kf.x) * s, (f2.y - kz * kf.y) * s};
    }
    __syncthreads();
    if (t < N2) {
#pragma unroll
        for (int j = 0; j < N1; ++j) r[j] = Ec[(t + N2 * j) * W];
    }
    __syncthreads();
    four_step_split<N1, N2, 1>(r, tw, Ec, t, ES, W);
    if (t < N1) {
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) buf_store(r[k2], rs, lo, k2 * N1 * zstride);
    }
}

// z pass of a box with a short z axis (MZ points): one (kx, ky) column a
// thread, the three components' lines in registers (forward DFT, the
// projection, inverse DFT); consecutive threads take consecutive kx, so every
// load and store of a wavefront is one contiguous run.
template <int MZ>
__global__ __launch_bounds__(256) void k_fft_z_solve_col(C2<float>* __restrict__ spec, int H, int My,
                                                         ProjArgs pa) {
    const int t = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (t >= H * My) return;
    const int jx = t % H, y = t / H;
    const size_t zs = (size_t)My * H, cs = (size_t)MZ * zs;
    C2<float>* col = spec + t;
    C2<float> v[3][MZ];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int z = 0; z < MZ; ++z) v[c][z] = col[c * cs + z * zs];
#pragma unroll
    for (int c = 0; c < 3; ++c) RDFT<float, MZ, -1>::run(v[c]);
    // projection: u^ = (I - k k^T / k^2) f^ / (eta k^2 Mx My Mz); k = 0 and index-H modes -> 0
    const float kux = (float)pa.kux, kuy = (float)pa.kuy, kuz = (float)pa.kuz, sc = (float)pa.scale;
    const int Hy = My / 2;
    const int jy = y < Hy ? y : y - My;
    const float kx = kux * (float)jx, ky = kuy * (float)jy;
#pragma unroll
    for (int z = 0; z < MZ; ++z) {
        const int jz = z < MZ / 2 ? z : z - MZ;
        const bool zero = (y == Hy) || (z == MZ / 2) || (jx == 0 && jy == 0 && jz == 0);
        const float kz = kuz * (float)jz;
        const float k2s = kx * kx + ky * ky + kz * kz;
        const float ik2 = zero ? 0.0f : 1.0f / k2s;
        const C2<float> f0 = v[0][z], f1 = v[1][z], f2 = v[2][z];
        const C2<float> kf = {(kx * f0.x + ky * f1.x + kz * f2.x) * ik2,
                              (kx * f0.y + ky * f1.y + kz * f2.y) * ik2};
        const float s = pa.root ? sc * sqrtf(ik2) : sc * ik2;
        v[0][z] = C2<float>{(f0.x - kx * kf.x) * s, (f0.y - kx * kf.y) * s};
        v[1][z] = C2<float>{(f1.x - ky * kf.x) * s, (f1.y - ky * kf.y) * s};
        v[2][z] = C2<float>{(f2.x - kz * kf.x) * s, (f2.y - kz * kf.y) * s};
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) RDFT<float, MZ, 1>::run(v[c]);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int z = 0; z < MZ; ++z) col[c * cs + z * zs] = v[c][z];
}

// x passes for a half-length H = N1 N2: T = N2 threads per line hold the
// values of index congruent to their lane q modulo T, before and after the
// transform.  The real/complex split pairs index k with H - k, whose holder
// is lane T - q, register N1 - 1 - i (lane 0: itself, register (N1 - i) mod
// N1): exchanged by lane shuffles when T is a power of two dividing 64 (a
// line's lanes then share a wavefront), through LDS otherwise.
template <int N1, int N2>
struct XGeom {
    static constexpr int H = N1 * N2, M = 2 * H, T = N2;
    static constexpr int KS = N2 + 1;               // exchange: k1 stride (complex)
    static constexpr int LS = (N1 * KS + 31) / 32 * 32 + 8;   // exchange: line stride
    // lines per block: a multiple of 4, at most 32, exchange buffer within
    // 68 KiB (two blocks a CU; 32 lines of 432 points: 192 threads, three
    // full wavefronts)
    static constexpr int lpb(int l) { return (l > 4 && l * LS * 8 > 69632) ? lpb(l - 4) : l; }
    static constexpr int LPB = lpb((256 / T) / 4 * 4 > 32 ? 32 : (256 / T) / 4 * 4);
    static constexpr int NT = LPB * T;
    static constexpr bool SHFL = (T & (T - 1)) == 0 && 64 % T == 0;
    static_assert(LS >= H, "line buffer holds a line");
};

__device__ inline C2<float> shfl_c(C2<float> v, int src) {
    return C2<float>{__shfl(v.x, src, 64), __shfl(v.y, src, 64)};
}

// the values at H - k of a line held in the lane-modulo-T layout (index 0's
// partner, X_H, is returned as X_0; the callers treat it)
template <int N1, int N2>
__device__ inline void x_partners(const C2<float>* v, C2<float>* pv, C2<float>* Eline, int q) {
    using G = XGeom<N1, N2>;
    constexpr int T = G::T;
    if constexpr (G::SHFL) {
        const int lane = threadIdx.x & 63;
        const int partner = (lane & ~(T - 1)) | ((T - q) & (T - 1));
#pragma unroll
        for (int i = 0; i < N1; ++i) {
            const C2<float> a = shfl_c(v[N1 - 1 - i], partner);
            pv[i] = (q == 0) ? v[(N1 - i) % N1] : a;
        }
    } else {
#pragma unroll
        for (int i = 0; i < N1; ++i) Eline[q + T * i] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < N1; ++i) {
            const int k = q + T * i;
            pv[i] = Eline[k == 0 ? 0 : G::H - k];
        }
        __syncthreads();
    }
}

// Moves a block's LPB lines between HBM and its line buffers in LDS (line ll
// at E + ll LS, complex index k).  The lines of a block are the floats
// [line0 M, (line0 + LPB) M) of the grid in either layout (LPB and M are
// multiples of 4, so a block holds whole tile rows), so the block reads or
// writes them as one contiguous run of 16-byte vectors; nf of those floats
// belong to lines that exist.  TILED: tiles of 8 x by 4 y; otherwise line
// after line (the row-major real grid, or the spectrum's H complex a line).
// A 16-byte vector must not straddle two lines: M a multiple of 4.
template <int M, int LPB, int LS, int NT, bool TILED, bool LOAD>
__device__ inline void stage_lines(float* __restrict__ blk, C2<float>* E, int nf) {
    static_assert(M % 4 == 0 && LPB % 4 == 0, "whole vectors and tile rows a block");
    // every vector of the thread in flight at once (loads issued before any
    // LDS write, LDS reads before any store)
    constexpr int NV = (LPB * M / 4 + NT - 1) / NT;
    float4 buf[NV];
    const int f0 = 4 * (int)threadIdx.x;
    if (LOAD) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int f = f0 + 4 * NT * i;
            if (f < nf) buf[i] = *reinterpret_cast<const float4*>(blk + f);
        }
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int f = f0 + 4 * NT * i;
        if (f >= nf) continue;
        int ll, k;
        if (TILED) {
            const int r = f / (4 * M), rem = f - r * (4 * M);
            ll = 4 * r + ((rem >> 3) & 3);
            k = (((rem >> 5) << 3) + (rem & 7)) >> 1;
        } else {
            ll = f / M;
            k = (f - ll * M) >> 1;
        }
        C2<float>* d = E + ll * LS + k;
        if (LOAD) {
            d[0] = C2<float>{buf[i].x, buf[i].y};
            d[1] = C2<float>{buf[i].z, buf[i].w};
        } else {
            buf[i] = make_float4(d[0].x, d[0].y, d[1].x, d[1].y);
        }
    }
    if (!LOAD) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int f = f0 + 4 * NT * i;
            if (f < nf) *reinterpret_cast<float4*>(blk + f) = buf[i];
        }
    }
}

template <int N1, int N2, bool TILED>
__global__ __launch_bounds__((XGeom<N1, N2>::NT)) void k_fft_x_r2c_reg(float* __restrict__ grid,
                                                                     const C2<float>* __restrict__ twg,
                                                                     int nlines) {
    using G = XGeom<N1, N2>;
    constexpr int H = G::H, T = G::T;
    // The block's lines cross HBM as one contiguous run of 16-byte vectors,
    // staged through the line buffers, where such vectors tile a line (H
    // even); the output too where the registers allow (measured: faster for
    // N1 <= 18, slower for N1 = 24, 36).
    constexpr bool kStageIn = H % 2 == 0, kStageOut = kStageIn && N1 <= 18;
    __shared__ C2<float> tw[G::M];
    __shared__ C2<float> E[G::LPB * G::LS];
    const int tid = threadIdx.x, q = tid % T, ll = tid / T;
    const int line = xcd_remap(blockIdx.x, gridDim.x) * G::LPB + ll;
    const bool ok = line < nlines;
    C2<float>* g = reinterpret_cast<C2<float>*>(grid) + (size_t)(ok ? line : 0) * H;
    for (int e = tid; e < G::M; e += G::NT) tw[e] = twg[e];
    C2<float> v[N1];
    const int line0 = line - ll;
    float* blk = grid + (size_t)line0 * G::M;
    const int nf = (min(nlines - line0, G::LPB)) * G::M;
    if constexpr (kStageIn) {
        stage_lines<G::M, G::LPB, G::LS, G::NT, TILED, true>(blk, E, nf);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < N1; ++j) v[j] = E[ll * G::LS + j * T + q];
    } else if (TILED) {
        // tiles of 8 x by 4 y (as written by the spread); a block's lines are
        // groups of 4 consecutive y
        constexpr int M = G::M;
        const int y = line % M;
        const float* pl =
            grid + (size_t)(line / M) * M * M + (size_t)(y >> 2) * (M << 2) + ((y & 3) << 3);
#pragma unroll
        for (int j = 0; j < N1; ++j) {
            const int x = 2 * (j * T + q);
            v[j] = ok ? *reinterpret_cast<const C2<float>*>(pl + ((x >> 3) << 5) + (x & 7))
                      : C2<float>{0, 0};
        }
    } else {
#pragma unroll
        for (int j = 0; j < N1; ++j) v[j] = ok ? g[j * T + q] : C2<float>{0, 0};
    }
    __syncthreads();
    four_step<N1, N2, -1, 2>(v, tw, E + ll * G::LS, q, G::KS, 1);
    // split: X_k = (Z_k + conj Z_{H-k})/2 - (i/2) exp(-2 pi i k/M) (Z_k - conj Z_{H-k})
    C2<float> pv[N1];
    x_partners<N1, N2>(v, pv, E + ll * G::LS, q);
#pragma unroll
    for (int i = 0; i < N1; ++i) {
        C2<float> Zc = pv[i];
        Zc.y = -Zc.y;
        const int k = q + T * i;
        const C2<float> S = cadd(v[i], Zc), D = csub(v[i], Zc);
        const C2<float> WD = cmul(tw[k], D);
        const C2<float> X = {0.5f * (S.x + WD.y), 0.5f * (S.y - WD.x)};
        if constexpr (kStageOut)
            E[ll * G::LS + k] = X;
        else if (ok)
            g[k] = X;
    }
    if constexpr (kStageOut) {
        __syncthreads();
        stage_lines<G::M, G::LPB, G::LS, G::NT, false, false>(blk, E, nf);
    }
}

template <int N1, int N2, bool TILED>
__global__ __launch_bounds__((XGeom<N1, N2>::NT)) void k_fft_x_c2r_reg(float* __restrict__ grid,
                                                                     const C2<float>* __restrict__ twg,
                                                                     int nlines) {
    using G = XGeom<N1, N2>;
    constexpr int H = G::H, T = G::T;
    __shared__ C2<float> tw[G::M];
    __shared__ C2<float> E[G::LPB * G::LS];
    const int tid = threadIdx.x, q = tid % T, ll = tid / T;
    const int line = xcd_remap(blockIdx.x, gridDim.x) * G::LPB + ll;
    const bool ok = line < nlines;
    C2<float>* g = reinterpret_cast<C2<float>*>(grid) + (size_t)(ok ? line : 0) * H;
    for (int e = tid; e < G::M; e += G::NT) tw[e] = twg[e];
    C2<float> x[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) x[i] = ok ? g[q + T * i] : C2<float>{0, 0};
    __syncthreads();
    // Z_k = E + i O, E = X_k + conj X_{H-k}, O = exp(+2 pi i k/M) (X_k - conj X_{H-k}),
    // with the x-Nyquist coefficient X_H taken as 0
    C2<float> pv[N1];
    x_partners<N1, N2>(x, pv, E + ll * G::LS, q);
    C2<float> z[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) {
        const int k = q + T * i;
        C2<float> Xc = (k == 0) ? C2<float>{0, 0} : pv[i];
        Xc.y = -Xc.y;
        const C2<float> Ev = cadd(x[i], Xc);
        C2<float> wk = tw[k];
        wk.y = -wk.y;
        const C2<float> O = cmul(csub(x[i], Xc), wk);
        z[i] = C2<float>{Ev.x - O.y, Ev.y + O.x};
    }
    four_step<N1, N2, 1, 2>(z, tw, E + ll * G::LS, q, G::KS, 1);
    if (TILED) {
        // tiles of 8 x by 4 y; a block's lines are groups of 4 consecutive y
        constexpr int M = G::M;
        const int y = line % M;
        float* pl = grid + (size_t)(line / M) * M * M + (size_t)(y >> 2) * (M << 2) + ((y & 3) << 3);
#pragma unroll
        for (int i = 0; i < N1; ++i) {
            const int x = 2 * (q + T * i);
            if (ok) *reinterpret_cast<C2<float>*>(pl + ((x >> 3) << 5) + (x & 7)) = z[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < N1; ++i)
            if (ok) g[q + T * i] = z[i];
    }
}


// ---- x and y passes fused over one (component, z) plane (FP32) ----
//
// A workgroup holds a whole M x M plane in registers and does both in-plane
// transforms before writing it back, so the plane crosses HBM once each way
// instead of twice.  Forward: the x transforms of the M lines in RX rounds of
// LR (T threads a line: the register four-step and the real/complex split of
// the x pass), then the H kx columns in RY rounds of CW: each round's columns
// are transposed through LDS and transformed by YN2 threads a column (the
// register four-step of the y pass); the inverse runs the same steps
// backwards.  The x exchange, the transpose and the y exchange take turns in
// one LDS buffer; their strides put the lines or rows one wavefront writes at
// different bank offsets.  Sizes: 64, 96, 128 and 256 (whose x geometry
// exchanges partners by lane shuffles and whose plane fits one workgroup).
template <int M_, int XN1_, int XN2_, int YN1_, int YN2_, int NT_>
struct XYGeom {
    static constexpr int M = M_, H = M_ / 2, XN1 = XN1_, XN2 = XN2_, T = XN2_;
    static constexpr int YN1 = YN1_, YN2 = YN2_, NT = NT_;
    static constexpr int LR = NT / T, RX = M / LR;   // x: lines per round, rounds
    static constexpr int CW = NT / YN2, RY = H / CW;  // y: kx columns per round, rounds
    static constexpr int KS = XN2 + 1;               // x exchange: k1 stride (complex)
    // the smallest stride >= need that is congruent to r modulo 32 complex
    static constexpr int up_to(int need, int r) { return need + ((r - need % 32) % 32 + 32) % 32; }
    static constexpr int LS = up_to(KS * (XN1 - 1) + XN2, (3 * T) % 32);  // x exchange: line stride
    static constexpr int RS = up_to(CW, T % 32);                          // transpose: row stride
    static constexpr int PL = YN2 * CW + 8;                                // y exchange: k1 stride
    static constexpr int cmax(int a, int b) { return a > b ? a : b; }
    static constexpr int LDSN = cmax(LR * LS, cmax(M * RS, YN1 * PL));
    static_assert(XN1 * XN2 == H && YN1 * YN2 == M, "factorisations of the plane");
    static_assert(XN1 % XN2 == 0 && YN1 % YN2 == 0, "four-step: N2 divides N1");
    static_assert(LR * RX == M && CW * RY == H && CW % T == 0, "rounds cover the plane");
    static_assert(XGeom<XN1, XN2>::SHFL, "x partners by lane shuffles");
    static_assert((LDSN + M) * 8 <= 163840, "LDS of one workgroup");
};

// threads of the fused passes for an M x M plane (0: separate passes)
constexpr int fused_xy_threads(int M) {
    return M == 64 ? 256 : M == 96 ? 192 : M == 128 ? 512 : M == 192 ? 384 : M == 256 ? 1024 : 0;
}

// element x (even) of line y of a plane: its pair of reals (x, x + 1)
template <int M, bool TILED>
__device__ inline C2<float>* xy_pair(float* pg, int y, int x) {
    if (TILED)
        return reinterpret_cast<C2<float>*>(pg + (y >> 2) * (M << 2) + ((y & 3) << 3) +
                                            ((x >> 3) << 5) + (x & 7));
    return reinterpret_cast<C2<float>*>(pg + y * M + x);
}

template <class G, bool TILED>
__global__ __launch_bounds__(G::NT) void k_fft_xy_r2c(float* __restrict__ grid,
                                                     const C2<float>* __restrict__ twg) {
    constexpr int M = G::M, H = G::H, XN1 = G::XN1, XN2 = G::XN2, T = G::T, YN1 = G::YN1;
    constexpr int YN2 = G::YN2, NT = G::NT, LR = G::LR, RX = G::RX, CW = G::CW, RY = G::RY;
    __shared__ C2<float> tw[M];
    __shared__ C2<float> E[G::LDSN];
    const int plane = xcd_remap(blockIdx.x, gridDim.x);  // component * M + z
    const int tid = threadIdx.x;
    float* pg = grid + (size_t)plane * M * M;
    C2<float>* spec = reinterpret_cast<C2<float>*>(pg);   // the plane's M x H spectrum
    for (int e = tid; e < M; e += NT) tw[e] = twg[e];
    // x: thread (ll, q) holds lines ll + LR r, elements q + T j of each
    const int q = tid % T, ll = tid / T;
    C2<float> v[RX][XN1];
#pragma unroll
    for (int r = 0; r < RX; ++r)
#pragma unroll
        for (int j = 0; j < XN1; ++j) v[r][j] = *xy_pair<M, TILED>(pg, ll + LR * r, 2 * (j * T + q));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RX; ++r) {
        four_step<XN1, XN2, -1, 2>(v[r], tw, E + ll * G::LS, q, G::KS, 1);
        C2<float> pv[XN1];
        x_partners<XN1, XN2>(v[r], pv, nullptr, q);
        // X_k = (Z_k + conj Z_{H-k})/2 - (i/2) exp(-2 pi i k/M) (Z_k - conj Z_{H-k})
#pragma unroll
        for (int i = 0; i < XN1; ++i) {
            C2<float> Zc = pv[i];
            Zc.y = -Zc.y;
            const C2<float> S = cadd(v[r][i], Zc), D = csub(v[r][i], Zc);
            const C2<float> WD = cmul(tw[q + T * i], D);
            v[r][i] = C2<float>{0.5f * (S.x + WD.y), 0.5f * (S.y - WD.x)};
        }
    }
    // y: thread (p, w) transforms column CW h + w, elements p + YN2 j
    const int w = tid % CW, p = tid / CW;
#pragma unroll
    for (int h = 0; h < RY; ++h) {
        // kx = q + T i lies in [CW h, CW h + CW) for i = (CW / T) h + ii
#pragma unroll
        for (int r = 0; r < RX; ++r)
#pragma unroll
            for (int ii = 0; ii < CW / T; ++ii) E[(ll + LR * r) * G::RS + q + T * ii] = v[r][(CW / T) * h + ii];
        __syncthreads();
        C2<float> u[YN1];
#pragma unroll
        for (int j = 0; j < YN1; ++j) u[j] = E[(p + YN2 * j) * G::RS + w];
        __syncthreads();
        four_step<YN1, YN2, -1, 1>(u, tw, E + w, p, G::PL, CW);
#pragma unroll
        for (int i = 0; i < YN1; ++i) spec[(p + YN2 * i) * H + CW * h + w] = u[i];
    }
}

template <class G, bool TILED>
__global__ __launch_bounds__(G::NT) void k_fft_xy_c2r(float* __restrict__ grid,
                                                     const C2<float>* __restrict__ twg) {
    constexpr int M = G::M, H = G::H, XN1 = G::XN1, XN2 = G::XN2, T = G::T, YN1 = G::YN1;
    constexpr int YN2 = G::YN2, NT = G::NT, LR = G::LR, RX = G::RX, CW = G::CW, RY = G::RY;
    __shared__ C2<float> tw[M];
    __shared__ C2<float> E[G::LDSN];
    const int plane = xcd_remap(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x;
    float* pg = grid + (size_t)plane * M * M;
    const C2<float>* spec = reinterpret_cast<const C2<float>*>(pg);
    for (int e = tid; e < M; e += NT) tw[e] = twg[e];
    const int w = tid % CW, p = tid / CW;
    C2<float> u[RY][YN1];
#pragma unroll
    for (int h = 0; h < RY; ++h)
#pragma unroll
        for (int j = 0; j < YN1; ++j) u[h][j] = spec[(p + YN2 * j) * H + CW * h + w];
    __syncthreads();
    const int q = tid % T, ll = tid / T;
    C2<float> x[RX][XN1];
#pragma unroll
    for (int h = 0; h < RY; ++h) {
        four_step<YN1, YN2, 1, 1>(u[h], tw, E + w, p, G::PL, CW);
#pragma unroll
        for (int i = 0; i < YN1; ++i) E[(p + YN2 * i) * G::RS + w] = u[h][i];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RX; ++r)
#pragma unroll
            for (int ii = 0; ii < CW / T; ++ii) x[r][(CW / T) * h + ii] = E[(ll + LR * r) * G::RS + q + T * ii];
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RX; ++r) {
        // Z_k = E + i O, E = X_k + conj X_{H-k}, O = exp(+2 pi i k/M) (X_k - conj X_{H-k}),
        // with the x-Nyquist coefficient X_H taken as 0
        C2<float> pv[XN1];
        x_partners<XN1, XN2>(x[r], pv, nullptr, q);
#pragma unroll
        for (int i = 0; i < XN1; ++i) {
            const int k = q + T * i;
            C2<float> Xc = (k == 0) ? C2<float>{0, 0} : pv[i];
            Xc.y = -Xc.y;
            const C2<float> Ev = cadd(x[r][i], Xc);
            C2<float> wk = tw[k];
            wk.y = -wk.y;
            const C2<float> O = cmul(csub(x[r][i], Xc), wk);
            x[r][i] = C2<float>{Ev.x - O.y, Ev.y + O.x};
        }
        four_step<XN1, XN2, 1, 2>(x[r], tw, E + ll * G::LS, q, G::KS, 1);
#pragma unroll
        for (int i = 0; i < XN1; ++i) *xy_pair<M, TILED>(pg, ll + LR * r, 2 * (q + T * i)) = x[r][i];
    }
}

// the z pass in LDS (all sizes and precisions)
// twz: the twiddle table of length Mz
template <typename R, int MZ>
void z_lds(const fcm_plan_impl* P, C2<R>* spec, const C2<R>* twz, hipStream_t st, ProjArgs pa) {
    const int Mz = P->Mz, H = P->H;
    const int ngz = (H + P->Wz - 1) / P->Wz;
    const size_t shz = (Mz + 3 * (size_t)P->Wz * Mz) * sizeof(C2<R>);
    hipLaunchKernelGGL((k_fft_z_solve<R, MZ>), dim3(ngz * P->My), dim3(kFFTThreads), shz, st, spec,
                       twz, Mz, H, P->My, P->radZ, P->Wz, __builtin_ctz(P->Wz), pa);
}

// root: the square root of the solve's multiplier (Brownian grid part)
ProjArgs proj_args(const fcm_plan_impl* P, bool root) {
    const double twopi = 2.0 * 3.14159265358979323846;
    ProjArgs pa;
    pa.kux = twopi / P->L;
    pa.kuy = twopi / P->Ly;
    pa.kuz = twopi / P->Lz;
    pa.scale = 1.0 / ((root ? sqrt(P->eta) : P->eta) * (double)P->M * P->My * P->Mz);
    pa.root = root ? 1 : 0;
    return pa;
}

// how the z pass of a register size runs
constexpr int kZLds = 0, kZReg = 1, kZGroups = 2, kZSplit = 3;

// FP32 solve with register passes (RegPlan sizes)
template <int XN1, int XN2, int YN1, int YN2, int YW, int ZMODE, int ZW, int ZN1, int ZN2>
hipError_t solve_reg(const fcm_plan_impl* P, float* grid, hipStream_t st, hipEvent_t* ev, bool tiled,
                     bool root) {
    using X = XGeom<XN1, XN2>;
    using Y = ColGeom<YN1, YN2, YW>;
    static_assert(2 * X::H == Y::M, "x and y factorisations of the same M");
    auto mark = [&](int i) {
        if (ev && timing_event(P, i + 2)) (void)hipEventRecord(ev[i], st);
    };
    constexpr int M = Y::M;
    const C2<float>* tw = (const C2<float>*)P->twid;
    C2<float>* spec = (C2<float>*)grid;
    const int nlines = 3 * M * M;
    const dim3 gx((nlines + X::LPB - 1) / X::LPB), bx(X::NT);
    const bool tl = tiled && M % 8 == 0;
    // the x and y passes of a plane in one workgroup where it fits (stage
    // times: the fused pass is reported as the x pass, the y pass as empty)
    constexpr int FNT = fused_xy_threads(M);
    constexpr bool fused = FNT > 0;
    using XY = XYGeom<M, XN1, XN2, YN1, YN2, fused ? FNT : 2 * M>;
    mark(0);
    if constexpr (fused) {
        if (tl)
            hipLaunchKernelGGL((k_fft_xy_r2c<XY, true>), dim3(3 * M), dim3(FNT), 0, st, grid, tw);
        else
            hipLaunchKernelGGL((k_fft_xy_r2c<XY, false>), dim3(3 * M), dim3(FNT), 0, st, grid, tw);
        mark(1);
    } else {
        if (tl)
            hipLaunchKernelGGL((k_fft_x_r2c_reg<XN1, XN2, true>), gx, bx, 0, st, grid, tw, nlines);
        else
            hipLaunchKernelGGL((k_fft_x_r2c_reg<XN1, XN2, false>), gx, bx, 0, st, grid, tw, nlines);
        mark(1);
        hipLaunchKernelGGL((k_fft_y_reg<YN1, YN2, YW, -1>), dim3(Y::NG * 3 * M), dim3(Y::NT), 0, st,
                           spec, tw);
    }
    mark(2);
    if constexpr (ZMODE == kZReg)
        hipLaunchKernelGGL((k_fft_z_solve_reg<YN1, YN2, YW>), dim3(Y::NG * M), dim3(Y::NT), 0, st, spec,
                           tw, proj_args(P, root));
    else if constexpr (ZMODE == kZGroups) {
        using Z = ZGeom3<YN1, YN2, ZW>;
        hipLaunchKernelGGL((k_fft_z_solve_3g<YN1, YN2, ZW>), dim3(Z::NG * M), dim3(Z::NT), 0, st, spec,
                           tw, proj_args(P, root));
    } else if constexpr (ZMODE == kZSplit) {
        using Z = ZGeomSplit<ZN1, ZN2, ZW>;
        hipLaunchKernelGGL((k_fft_z_solve_split<ZN1, ZN2, ZW>), dim3(Z::NG * M), dim3(Z::NT), 0, st,
                           spec, tw, proj_args(P, root));
    } else {
        static_assert(ZMODE == kZLds, "z-pass mode");
        z_lds<float, 8>(P, spec, tw, st, proj_args(P, root));
    }
    mark(3);
    if constexpr (fused) {
        mark(4);
        if (tl)
            hipLaunchKernelGGL((k_fft_xy_c2r<XY, true>), dim3(3 * M), dim3(FNT), 0, st, grid, tw);
        else
            hipLaunchKernelGGL((k_fft_xy_c2r<XY, false>), dim3(3 * M), dim3(FNT), 0, st, grid, tw);
    } else {
        hipLaunchKernelGGL((k_fft_y_reg<YN1, YN2, YW, 1>), dim3(Y::NG * 3 * M), dim3(Y::NT), 0, st,
                           spec, tw);
        mark(4);
        if (tl)
            hipLaunchKernelGGL((k_fft_x_c2r_reg<XN1, XN2, true>), gx, bx, 0, st, grid, tw, nlines);
        else
            hipLaunchKernelGGL((k_fft_x_c2r_reg<XN1, XN2, false>), gx, bx, 0, st, grid, tw, nlines);
    }
    mark(5);
    return hipGetLastError();
}

// FP32 boxes with a square cross-section (Mx = My = M, a register size or
// 512) and a short z axis (4, 8, 12 or 16 points): the register x and y
// passes of M (fused where they fuse), in the row-major layout, around the
// one-column-a-thread z pass.
template <int MZ>
void z_col(const fcm_plan_impl* P, C2<float>* spec, hipStream_t st, ProjArgs pa) {
    const int H = P->H, My = P->My;
    hipLaunchKernelGGL((k_fft_z_solve_col<MZ>), dim3((H * My + 255) / 256), dim3(256), 0, st, spec, H, My,
                       pa);
}

bool box_zcol(int Mz) { return Mz == 4 || Mz == 8 || Mz == 12 || Mz == 16; }

template <int XN1, int XN2, int YN1, int YN2, int YW>
hipError_t solve_box(const fcm_plan_impl* P, float* grid, hipStream_t st, hipEvent_t* ev, bool root) {
    using X = XGeom<XN1, XN2>;
    using Y = ColGeom<YN1, YN2, YW>;
    static_assert(2 * X::H == Y::M, "x and y factorisations of the same M");
    auto mark = [&](int i) {
        if (ev && timing_event(P, i + 2)) (void)hipEventRecord(ev[i], st);
    };
    constexpr int M = Y::M;
    const int Mz = P->Mz;
    const C2<float>* tw = (const C2<float>*)P->twid;   // Mx = My: the x and y tables agree
    C2<float>* spec = (C2<float>*)grid;
    const int nlines = 3 * M * Mz;
    const dim3 gx((nlines + X::LPB - 1) / X::LPB), bx(X::NT);
    constexpr int FNT = fused_xy_threads(M);
    using XY = XYGeom<M, XN1, XN2, YN1, YN2, (FNT > 0 ? FNT : 2 * M)>;
    // the fused passes take one workgroup a plane: with fewer planes than
    // CUs the separate passes spread wider
    const bool fused = FNT > 0 && 3 * Mz >= 256;
    const ProjArgs pa = proj_args(P, root);
    mark(0);
    if constexpr (FNT > 0) {
        if (fused) hipLaunchKernelGGL((k_fft_xy_r2c<XY, false>), dim3(3 * Mz), dim3(FNT), 0, st, grid, tw);
    }
    if (!fused) {
        hipLaunchKernelGGL((k_fft_x_r2c_reg<XN1, XN2, false>), gx, bx, 0, st, grid, tw, nlines);
        mark(1);
        hipLaunchKernelGGL((k_fft_y_reg<YN1, YN2, YW, -1>), dim3(Y::NG * 3 * Mz), dim3(Y::NT), 0, st,
                           spec, tw);
    } else {
        mark(1);
    }
    mark(2);
    switch (Mz) {
        case 4: z_col<4>(P, spec, st, pa); break;
        case 8: z_col<8>(P, spec, st, pa); break;
        case 12: z_col<12>(P, spec, st, pa); break;
        default: z_col<16>(P, spec, st, pa); break;
    }
    mark(3);
    if (!fused) {
        hipLaunchKernelGGL((k_fft_y_reg<YN1, YN2, YW, 1>), dim3(Y::NG * 3 * Mz), dim3(Y::NT), 0, st,
                           spec, tw);
        mark(4);
        hipLaunchKernelGGL((k_fft_x_c2r_reg<XN1, XN2, false>), gx, bx, 0, st, grid, tw, nlines);
    } else {
        mark(4);
    }
    if constexpr (FNT > 0) {
        if (fused) hipLaunchKernelGGL((k_fft_xy_c2r<XY, false>), dim3(3 * Mz), dim3(FNT), 0, st, grid, tw);
    }
    mark(5);
    return hipGetLastError();
}

// The sizes with register passes: M -> (x: M/2 = XN1 XN2), (y: M = YN1 YN2 over
// YW columns), how the z pass runs and over how many columns ZW (kZReg: three
// components a thread over YW columns; kZGroups: one component a thread with
// the y factorisation; kZSplit: one component a thread, M = ZN1 ZN2 split as
// in four_step_split; kZLds: the LDS Stockham pass).
#define FCM_REG_SIZES(X)                                 \
    X(64, 8, 4, 8, 8, 32, kZReg, 0, 0, 0)            \
    X(72, 18, 2, 12, 6, 36, kZReg, 0, 0, 0)          \
    X(96, 12, 4, 24, 4, 48, kZSplit, 16, 12, 8)      \
    X(108, 18, 3, 18, 6, 27, kZSplit, 6, 12, 9)      \
    X(128, 8, 8, 16, 8, 32, kZGroups, 8, 0, 0)       \
    X(144, 12, 6, 12, 12, 18, kZSplit, 4, 16, 9)     \
    X(162, 9, 9, 18, 9, 27, kZGroups, 9, 0, 0)       \
    X(192, 24, 4, 24, 8, 32, kZSplit, 4, 16, 12)     \
    X(216, 18, 6, 36, 6, 18, kZSplit, 4, 18, 12)     \
    X(256, 16, 8, 16, 16, 16, kZReg, 0, 0, 0)        \
    X(288, 12, 12, 24, 12, 16, kZSplit, 4, 16, 18)   \
    X(324, 18, 9, 18, 18, 9, kZGroups, 9, 0, 0)      \
    X(384, 24, 8, 48, 8, 24, kZGroups, 16, 0, 0)   \
    X(432, 36, 6, 36, 12, 18, kZGroups, 4, 0, 0)

bool reg_size(int M) {
#define FCM_REG_CASE(m, a, b, c, d, e, f, g, h, i) \
    case m:                                        \
        return true;
    switch (M) {
        FCM_REG_SIZES(FCM_REG_CASE)
        default: return false;
    }
#undef FCM_REG_CASE
}

template <typename R, int MX, int MZ>
hipError_t solve_r(const fcm_plan_impl* P, R* grid, hipStream_t st, hipEvent_t* ev, bool tiled,
                   bool root) {
    if constexpr (sizeof(R) == sizeof(float)) {
#define FCM_REG_CASE(m, a, b, c, d, e, f, g, h, i) \
    case m:                                        \
        return solve_reg<a, b, c, d, e, f, g, h, i>(P, grid, st, ev, tiled, root);
        if (P->cubic) switch (P->M) {
                FCM_REG_SIZES(FCM_REG_CASE)
                default: break;
            }
#undef FCM_REG_CASE
#define FCM_BOX_CASE(m, a, b, c, d, e, f, g, h, i) \
    case m:                                        \
        return solve_box<a, b, c, d, e>(P, grid, st, ev, root);
        if (!P->cubic && P->M == P->My && box_zcol(P->Mz)) switch (P->M) {
                FCM_REG_SIZES(FCM_BOX_CASE)
                case 512: return solve_box<16, 16, 32, 16, 8>(P, grid, st, ev, root);
                default: break;
            }
#undef FCM_BOX_CASE
    }
    auto mark = [&](int i) {
        if (ev && timing_event(P, i + 2)) (void)hipEventRecord(ev[i], st);
    };
    const int M = P->M, H = P->H, My = P->My, Mz = P->Mz;
    // twiddle tables of lengths M, My, Mz, one after the other
    const C2<R>* tw = (const C2<R>*)P->twid;
    const C2<R>* twy = tw + M;
    const C2<R>* twz = twy + My;
    C2<R>* spec = (C2<R>*)grid;
    const int nlines = 3 * My * Mz;
    const size_t cs = sizeof(C2<R>);
    mark(0);
    {
        const size_t shm = (M + (size_t)P->Wx * (H + 1)) * cs;
        hipLaunchKernelGGL((k_fft_x_r2c<R, MX>), dim3((nlines + P->Wx - 1) / P->Wx),
                           dim3(kFFTThreads), shm, st, grid, tw, M, P->radH, P->Wx, nlines);
    }
    mark(1);
    const int ngy = (H + P->Wy - 1) / P->Wy;
    const size_t shy = (My + (size_t)P->Wy * My) * cs;
    const int lwy = __builtin_ctz(P->Wy);
    hipLaunchKernelGGL((k_fft_y<R, -1, MX>), dim3(ngy * 3 * Mz), dim3(kFFTThreads), shy, st, spec, twy,
                       My, H, P->radY, P->Wy, lwy);
    mark(2);
    z_lds<R, MZ>(P, spec, twz, st, proj_args(P, root));
    mark(3);
    hipLaunchKernelGGL((k_fft_y<R, 1, MX>), dim3(ngy * 3 * Mz), dim3(kFFTThreads), shy, st, spec, twy,
                       My, H, P->radY, P->Wy, lwy);
    mark(4);
    {
        const size_t shm = (M + (size_t)P->Wx * (H + 1)) * cs;
        hipLaunchKernelGGL((k_fft_x_c2r<R, MX>), dim3((nlines + P->Wx - 1) / P->Wx),
                           dim3(kFFTThreads), shm, st, grid, tw, M, P->radH, P->Wx, nlines);
    }
    mark(5);
    return hipGetLastError();
}

}  // namespace

// elements per thread of the x/y passes and of the z pass
int fft_maxe(int precision, bool zpass) {
    if (precision == FCM_FP64) return zpass ? 4 : 8;
    return zpass ? 8 : 16;
}

bool solve_tiles(const fcm_plan_impl* P) {
    return P->precision != FCM_FP64 && P->cubic && reg_size(P->M) && P->M % 8 == 0;
}

hipError_t launch_solve(const fcm_plan_impl* P, void* grid, hipStream_t st, hipEvent_t* ev,
                        bool tiled, bool root) {
    if (P->precision == FCM_FP64) return solve_r<double, 8, 4>(P, (double*)grid, st, ev, false, root);
    return solve_r<float, 16, 8>(P, (float*)grid, st, ev, tiled && solve_tiles(P), root);
}

}  // namespace fcm
