// Public C ABI of the fast-FCM library (include/fcm.h): plan construction,
// validation, and the orchestration of the hot path on one HIP stream:
//   hash -> sort -> spread -> Stokes solve (5 FFT passes) -> interpolate ->
//   pair correction (Sec. 4, steps 1-6).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "fcm_internal.h"

using namespace fcm;

// Device scratch of the allocation-free entry point fcm_mobility_static: one
// 64 MiB array per GPU the library runs on (uninitialised; the code object
// carries only its size).  Host code uses its device address, never its name.
constexpr int64_t kStaticScratchBytes = (int64_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr double kPi = 3.14159265358979323846;

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

bool is_smooth_even(int n) {
    if (n < 8 || n > kMaxGrid || (n & 1)) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// radices (8, 4, 2 for the power of two; 3 for each factor 3), largest first
RadixPlan make_radix_plan(int n) {
    RadixPlan rp;
    rp.n = n;
    rp.nst = 0;
    int m = n;
    int p2 = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++p2;
    }
    while (p2 >= 3) {
        rp.rad[rp.nst++] = 8;
        p2 -= 3;
    }
    if (p2 == 2) rp.rad[rp.nst++] = 4;
    if (p2 == 1) rp.rad[rp.nst++] = 2;
    while (m % 3 == 0) {
        rp.rad[rp.nst++] = 3;
        m /= 3;
    }
    return rp;
}

// fill the per-stage strides, divisors and twiddle steps (table length M)
void finish_radix_plan(RadixPlan& rp, int M) {
    int Ns = 1;
    for (int s = 0; s < rp.nst; ++s) {
        rp.ns[s] = Ns;
        rp.nsm[s] = div_magic((unsigned)Ns);
        rp.nb[s] = rp.n / rp.rad[s];
        rp.nbm[s] = div_magic((unsigned)rp.nb[s]);
        rp.tstep[s] = M / (Ns * rp.rad[s]);
        Ns *= rp.rad[s];
    }
    rp.nm = div_magic((unsigned)rp.n);
}

int pow2_floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

void choose_tiles(fcm_plan_impl* P) {
    const int M = P->M, My = P->My, Mz = P->Mz, MG = P->MG;
    double best = 1e300;
    int bx = 1, by = 1;
    // tx <= M - MG + 1 and ty <= My - MG + 1: a particle's support covers the
    // tile's columns in one run along x and along y
    for (int tx = 1; tx <= 64 && tx <= M - MG + 1; ++tx) {
        if (M % tx) continue;
        for (int ty = 1; tx * ty <= 64 && ty <= My - MG + 1; ++ty) {
            if (My % ty) continue;
            // candidate-scan work per grid point of a wavefront tile
            const double score = (double)(tx + MG - 1) * (ty + MG - 1) / (tx * ty) +
                                 (tx < 8 ? 0.01 : 0.0);
            if (score < best - 1e-12) {
                best = score;
                bx = tx;
                by = ty;
            }
        }
    }
    P->TX = bx;
    P->TY = by;
    // tile height: a divisor of Mz with TZ <= Mz - MG + 1, so that the heights
    // a particle's support covers within a tile form a single run
    const int tzs[] = {16, 12, 8, 6, 4, 2, 1};
    P->TZ = 1;
    for (int t : tzs)
        if (Mz % t == 0 && t <= Mz - MG + 1) {
            P->TZ = t;
            break;
        }
    // a support longer than the z axis: one tile spans the axis (Mz is one of
    // the tile heights, checked by plan_derive) and every height is covered
    if (MG > Mz) P->TZ = Mz;
    // One wavefront spreads a tile: with fewer than 8 tiles per SIMD (8192 on
    // the 1024 SIMDs) latency and crowded tiles are poorly hidden, and tiles
    // of height 8 pay less than their extra candidate scans (measured: 192^3
    // clustered rods and 128^3 dilute faster, 256^3 dense slower).
    if (P->TZ > 8 && Mz % 8 == 0 && (int64_t)(M / P->TX) * (My / P->TY) * (Mz / P->TZ) < 8192)
        P->TZ = 8;
    P->nbx = M / P->TX;
    P->nby = My / P->TY;
    P->nbz = Mz / P->TZ;
    P->nbins = P->nbx * P->nby * P->nbz;
    auto back = [&](int T, int nb) {
        int b = (MG - 1 + T - 1) / T;
        return b > nb - 1 ? nb - 1 : b;
    };
    P->backx = back(P->TX, P->nbx);
    P->backy = back(P->TY, P->nby);
    P->backz = back(P->TZ, P->nbz);
}

size_t real_size(int precision) { return precision == FCM_FP64 ? sizeof(double) : sizeof(float); }

size_t grid_rec_size(int precision) {
    return precision == FCM_FP64 ? sizeof(GridRec<double>) : sizeof(GridRec<float>);
}

constexpr int kMaxTimedCalls = 1024;
// events per call: stage boundaries 0..8 and the end of the call (9) on the call's
// stream, then the start and end of the pair correction (10, 11) on the side stream
constexpr int kEvPerCall = FCM_NUM_STAGES + 3;

void free_events(fcm_plan_impl* P) {
    if (!P->events) return;
    for (int i = 0; i < P->ev_cap * kEvPerCall; ++i)
        if (P->events[i]) (void)hipEventDestroy(P->events[i]);
    free(P->events);
    P->events = nullptr;
    P->ev_cap = 0;
    P->ev_calls = 0;
}

// the event set of the current call, or NULL when not timing / record full
hipEvent_t* call_events(fcm_plan_impl* P) {
    if (!P->timing || P->ev_calls >= P->ev_cap) return nullptr;
    return P->events + (size_t)(P->ev_calls++) * kEvPerCall;
}

void free_plan(fcm_plan_impl* P) {
    if (!P) return;
    free_events(P);
    void* bufs[] = {P->grid,  P->twid, P->counts, P->starts,    P->keys,       P->ranks,
                    P->perm,  P->scan_tmp, P->grec, P->prec,    P->ppos,       P->flag,
                    P->pair_hits, P->pair_count, P->corr, P->krylov, P->partial};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (P->fork) (void)hipEventDestroy(P->fork);
    if (P->join) (void)hipEventDestroy(P->join);
    if (P->side) (void)hipStreamDestroy(P->side);
    delete P;
}

int map_err(hipError_t e) {
    if (e == hipSuccess) return FCM_OK;
    if (e == hipErrorOutOfMemory) return FCM_ENOMEM;
    return FCM_EDEVICE;
}

// Counting sort into grid bins and pair cells.  The counts are all zero
// between calls (the scan clears them, and the segment sorts clear the work
// lists they keep there); after an allocation or a failed launch they are
// cleared here first.
hipError_t sort_particles(fcm_plan_impl* P, const double* pos, hipStream_t st) {
    hipError_t e;
    P->repeat_ok = 0;
    if (P->counts_dirty &&
        (e = launch_fill(P->counts, P->nbins + P->cells_cap, 0, st)) != hipSuccess)
        return e;
    P->counts_dirty = 1;
    if ((e = launch_hash(P, pos, st)) != hipSuccess) return e;
    if ((e = launch_scan(P, st)) != hipSuccess) return e;
    if ((e = launch_scatter(P, st)) != hipSuccess) return e;
    P->counts_dirty = 0;
    return hipSuccess;
}

bool needs_correction(const fcm_plan_impl* P) {
    return !(P->Sigma == P->sigma && P->SigmaD == P->sigmaD);
}

}  // namespace

namespace fcm {

// Validate the arguments and fill every scalar of a plan (no allocation).
// L and grid: box sides and grid points along x, y, z (one grid spacing).
int plan_derive(fcm_plan_impl* P, int64_t N, const double L[3], double a, double sigma_delta,
                const int grid[3], double r_cut, const fcm_options* opt_in) {
    memset(P, 0, sizeof(*P));  // no buffers, no events, no stream yet
    fcm_options opt;
    fcm_options_default(&opt);
    if (opt_in) opt = *opt_in;
    if (!L || !grid) return FCM_EINVAL;
    if (N <= 0 || N > (int64_t)1 << 29) return FCM_EINVAL;
    for (int d = 0; d < 3; ++d) {
        if (!(L[d] > 0.0) || !isfinite(L[d])) return FCM_EINVAL;
        if (!is_smooth_even(grid[d])) return FCM_EINVAL;
    }
    if (!(a > 0.0) || !isfinite(a)) return FCM_EINVAL;
    const double dx = L[0] / grid[0];
    for (int d = 1; d < 3; ++d)
        if (fabs(L[d] / grid[d] - dx) > 1e-12 * dx) return FCM_EINVAL;
    if (!(opt.eta > 0.0) || !isfinite(opt.eta)) return FCM_EINVAL;
    if (opt.precision != FCM_FP64 && opt.precision != FCM_FP32_BULK) return FCM_EINVAL;
    if (opt.kahan < 0 || opt.kahan > 2) return FCM_EINVAL;
    const double sigma = a / sqrt(kPi);
    const double sigmaD = a / cbrt(6.0 * sqrt(kPi));
    if (!(sigma_delta >= sigma * (1.0 - 1e-12)) || !isfinite(sigma_delta)) return FCM_EINVAL;
    // widths within 1e-12 (relative) of sigma and sigma_D are taken as equal to
    // them, so standard FCM is recognised whatever rounding the caller's
    // sqrt and cube root had
    const double Sigma = sigma_delta < sigma * (1.0 + 1e-12) ? sigma : sigma_delta;
    double SigmaD = opt.sigma_D_grid > 0.0 ? opt.sigma_D_grid : Sigma;
    if (!(SigmaD >= sigmaD * (1.0 - 1e-12)) || !isfinite(SigmaD)) return FCM_EINVAL;
    if (SigmaD < sigmaD * (1.0 + 1e-12)) SigmaD = sigmaD;
    if (!(r_cut >= 0.0) || !isfinite(r_cut)) return FCM_EINVAL;
    const double Lmin = fmin(L[0], fmin(L[1], L[2]));
    if (r_cut >= 0.5 * Lmin) return FCM_ERANGE;
    const int gmax = grid[0] > grid[1] ? (grid[0] > grid[2] ? grid[0] : grid[2])
                                       : (grid[1] > grid[2] ? grid[1] : grid[2]);
    int MG = opt.support;
    if (MG == 0) {
        const double wmax = Sigma > SigmaD ? Sigma : SigmaD;
        MG = (int)ceil(10.0 * wmax / dx - 1e-9);
        if (MG & 1) ++MG;
        if (MG < 8) MG = 8;
    }
    // Along x and y the support fits the axis.  Along z it may be longer (the
    // paper's rod runs use 8 z points, Sec. 6.3): the support then wraps onto
    // itself and its coinciding points add, which needs one spreading tile to
    // span the axis (Mz = 8, 12 or 16).
    const int gxy = grid[0] < grid[1] ? grid[0] : grid[1];
    if (MG < 2 || MG > kMaxSupport || MG > gxy) return FCM_EINVAL;
    if (MG > grid[2] && grid[2] != 8 && grid[2] != 12 && grid[2] != 16) return FCM_EINVAL;
    // FP64 spreading stages its particles with M_G-point tables in LDS
    if (opt.precision == FCM_FP64 && MG > 24) return FCM_EINVAL;
    const int mz = fft_maxe(opt.precision, true) * 256;
    if (gmax > mz) return FCM_EINVAL;

    P->N = N;
    P->L = L[0];
    P->Ly = L[1];
    P->Lz = L[2];
    P->a = a;
    P->eta = opt.eta;
    P->sigma = sigma;
    P->sigmaD = sigmaD;
    P->Sigma = Sigma;
    P->SigmaD = SigmaD;
    P->rc = r_cut;
    P->dx = dx;
    P->M = grid[0];
    P->My = grid[1];
    P->Mz = grid[2];
    P->H = grid[0] / 2;
    P->cubic = grid[0] == grid[1] && grid[1] == grid[2];
    P->MG = MG;
    P->precision = opt.precision;
    P->kahan = opt.kahan;
    choose_tiles(P);
    // pair cells per axis: m = max(int(L / R_c), 3) (at most kMaxCellsPerAxis);
    // R_c = 0: no pair search, one cell
    int mc[3] = {1, 1, 1};
    if (r_cut > 0.0) {
        for (int d = 0; d < 3; ++d) {
            const double q = L[d] / r_cut;
            mc[d] = q > (double)kMaxCellsPerAxis ? kMaxCellsPerAxis : (int)q;
            if (mc[d] < 3) mc[d] = 3;
        }
    }
    P->m = mc[0];
    P->mcy = mc[1];
    P->mcz = mc[2];
    P->ncells = mc[0] * mc[1] * mc[2];
    P->radH = make_radix_plan(grid[0] / 2);
    P->radY = make_radix_plan(grid[1]);
    P->radZ = make_radix_plan(grid[2]);
    finish_radix_plan(P->radH, grid[0]);
    finish_radix_plan(P->radY, grid[1]);
    finish_radix_plan(P->radZ, grid[2]);
    const int mxy = fft_maxe(P->precision, false) * 256;
    P->Wy = pow2_floor(mxy / P->My);
    if (P->Wy > 32) P->Wy = 32;
    P->Wz = pow2_floor(mz / P->Mz);
    if (P->Wz > 32) P->Wz = 32;
    // FP32 z passes in LDS (216^3, 384^3, 432^3 and the non-cubic boxes): half
    // the columns per workgroup gives more resident workgroups, which pays more
    // than the longer rows (216^3: 135 -> 110 us, 432^3: 1229 -> 1073 us; a
    // quarter, or twice the threads, is slower; FP64 keeps its width)
    if (P->precision == FCM_FP32_BULK && P->Mz >= 192 && P->Wz > 1) P->Wz /= 2;
    P->Wx = mxy / P->H;
    if (P->Wx > 64) P->Wx = 64;
    if (P->Wx < 1) P->Wx = 1;
    {
        const double sp = Sigma * sqrt(kPi);
        const double d = sigma * sigma - Sigma * Sigma;
        P->selfVF = 1.0 / (6.0 * kPi * P->eta * a) - 1.0 / (6.0 * kPi * P->eta * sp) +
                    d / (12.0 * P->eta * sp * sp * sp) -
                    d * d / (32.0 * P->eta * pow(Sigma, 5.0) * pow(kPi, 1.5));
        const double sd = SigmaD * sqrt(kPi);
        P->selfOT = 1.0 / (8.0 * kPi * P->eta * a * a * a) - 1.0 / (48.0 * P->eta * sd * sd * sd);
    }
    return FCM_OK;
}

// Allocate the device buffers of a derived plan for up to ncap particles and
// cellcap pair cells, and upload the twiddles.  No device-wide synchronisation.
int plan_allocate(fcm_plan_impl* P, int64_t ncap, int cellcap) {
    if (hipGetDevice(&P->device) != hipSuccess) return FCM_EDEVICE;
    P->Ncap = ncap;
    P->cells_cap = cellcap;
    P->counts_dirty = 1;
    const size_t rs = real_size(P->precision);
    const size_t M3 = (size_t)P->M * P->My * P->Mz;
    const int ntw = P->M + P->My + P->Mz;
    hipError_t e = hipSuccess;
#define FCM_ALLOC(ptr, bytes)                                        \
    do {                                                             \
        if (e == hipSuccess) e = hipMalloc((void**)&(ptr), (bytes)); \
    } while (0)
    FCM_ALLOC(P->grid, 3 * M3 * rs);
    FCM_ALLOC(P->twid, (size_t)ntw * 2 * rs);
    FCM_ALLOC(P->counts, (size_t)(P->nbins + cellcap) * sizeof(int));
    FCM_ALLOC(P->starts, (size_t)(P->nbins + 1 + cellcap + 1) * sizeof(int));
    FCM_ALLOC(P->keys, (size_t)2 * ncap * sizeof(int));
    FCM_ALLOC(P->ranks, (size_t)2 * ncap * sizeof(int));
    FCM_ALLOC(P->perm, (size_t)2 * ncap * sizeof(int));
    FCM_ALLOC(P->scan_tmp, kMaxScanTiles * sizeof(int));
    FCM_ALLOC(P->grec, (size_t)ncap * grid_rec_size(P->precision));
    FCM_ALLOC(P->prec, (size_t)ncap * sizeof(PairRec));
    FCM_ALLOC(P->ppos, (size_t)ncap * sizeof(double4));
    FCM_ALLOC(P->pair_hits, (size_t)3 * ncap * kPairCap * sizeof(int));
    FCM_ALLOC(P->pair_count, (size_t)3 * ncap * sizeof(int));
    FCM_ALLOC(P->corr, (size_t)6 * ncap * sizeof(double));
    FCM_ALLOC(P->partial, 1024 * sizeof(double));
    FCM_ALLOC(P->flag, 16 * sizeof(int));
#undef FCM_ALLOC
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->join, hipEventDisableTiming);
    if (e != hipSuccess) return map_err(e);
    // twiddles exp(-2 pi i m / n) for n = M, My, Mz in turn, in extended
    // precision, rounded once
    const size_t n = (size_t)ntw * 2;
    void* host = malloc(n * rs);
    if (!host) return FCM_ENOMEM;
    const int lens[3] = {P->M, P->My, P->Mz};
    int off = 0;
    for (int d = 0; d < 3; ++d) {
        const int len = lens[d];
        for (int mm = 0; mm < len; ++mm) {
            const long double ang = -2.0L * 3.141592653589793238462643383279502884L * mm / len;
            const long double c = cosl(ang), sn = sinl(ang);
            const size_t k = (size_t)(off + mm);
            if (P->precision == FCM_FP64) {
                ((double*)host)[2 * k] = (double)c;
                ((double*)host)[2 * k + 1] = (double)sn;
            } else {
                ((float*)host)[2 * k] = (float)c;
                ((float*)host)[2 * k + 1] = (float)sn;
            }
        }
        off += len;
    }
    e = hipMemcpy(P->twid, host, n * rs, hipMemcpyHostToDevice);
    free(host);
    if (e == hipSuccess) e = hipMemset(P->flag, 0, 16 * sizeof(int));
    return map_err(e);
}

// Re-parameterise an allocated plan with the scalars of `d` (derived for a new
// problem of the same grid, support, precision and accumulation mode).
int plan_rebind(fcm_plan_impl* P, const fcm_plan_impl* d) {
    if (d->M != P->M || d->My != P->My || d->Mz != P->Mz || d->MG != P->MG ||
        d->precision != P->precision || d->kahan != P->kahan || d->N > P->Ncap ||
        d->ncells > P->cells_cap)
        return FCM_EINVAL;
    P->repeat_ok = 0;
    P->N = d->N;
    P->L = d->L;
    P->Ly = d->Ly;
    P->Lz = d->Lz;
    P->a = d->a;
    P->eta = d->eta;
    P->sigma = d->sigma;
    P->sigmaD = d->sigmaD;
    P->Sigma = d->Sigma;
    P->SigmaD = d->SigmaD;
    P->rc = d->rc;
    P->dx = d->dx;
    P->m = d->m;
    P->mcy = d->mcy;
    P->mcz = d->mcz;
    P->ncells = d->ncells;
    P->selfVF = d->selfVF;
    P->selfOT = d->selfOT;
    return FCM_OK;
}

void plan_free(fcm_plan_impl* P) { free_plan(P); }

int64_t plan_bytes(int64_t ncap, const int grid[3], int precision, int cellcap, int nbins) {
    const int64_t rs = (int64_t)real_size(precision);
    int64_t b = 3 * (int64_t)grid[0] * grid[1] * grid[2] * rs +
                (int64_t)(grid[0] + grid[1] + grid[2]) * 2 * rs;
    b += 6 * ncap * (int64_t)sizeof(int);
    b += 3 * ncap * (int64_t)(kPairCap + 1) * (int64_t)sizeof(int);
    b += 6 * ncap * (int64_t)sizeof(double);
    b += ncap * (int64_t)(grid_rec_size(precision) + sizeof(PairRec) + sizeof(double4));
    // counts and starts of the bins and cells, the scan's block sums, the
    // reduction partials and the flags (the buffers of plan_allocate)
    b += (int64_t)(2 * (nbins + 1) + 2 * (cellcap + 1)) * (int64_t)sizeof(int);
    b += (int64_t)kMaxScanTiles * (int64_t)sizeof(int) + 1024 * (int64_t)sizeof(double) + 16 * (int64_t)sizeof(int);
    return b;
}

}  // namespace fcm

namespace {

// ---- the allocation-free entry point (fcm_mobility_static) ----------------
//
// Every buffer of its plan lives in `scratch`, one array per GPU the library
// runs on, held until the process ends.  Host code never passes the array's
// name to the device: it takes the array's device address once per device
// (hipGetSymbolAddress, with that device current) and uses that address.

constexpr int kMaxStaticDevices = 64;

std::mutex g_static_mu;
unsigned char* g_static_ptr[kMaxStaticDevices];

// the device address of this device's scratch (looked up on first use)
int static_scratch(unsigned char** out, int* device) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FCM_EDEVICE;
    if (dev < 0 || dev >= kMaxStaticDevices) return FCM_EDEVICE;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FCM_EDEVICE;
        g_static_ptr[dev] = (unsigned char*)ptr;
    }
    *out = g_static_ptr[dev];
    *device = dev;
    return FCM_OK;
}

// the buffers of plan_allocate, carved in the same order from `base` (each
// 256-byte aligned; plan_bytes(...) plus the alignment fits the scratch, see
// the size check at the call); no side stream, events or timing
void carve_static_plan(fcm_plan_impl* P, unsigned char* base) {
    const int64_t ncap = P->N;
    const int cellcap = P->ncells;
    P->Ncap = ncap;
    P->cells_cap = cellcap;
    const size_t rs = real_size(P->precision);
    const size_t M3 = (size_t)P->M * P->My * P->Mz;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void* p = base + off;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    P->grid = take(3 * M3 * rs);
    P->twid = take((size_t)(P->M + P->My + P->Mz) * 2 * rs);
    P->counts = (int*)take((size_t)(P->nbins + cellcap) * sizeof(int));
    P->starts = (int*)take((size_t)(P->nbins + 1 + cellcap + 1) * sizeof(int));
    P->keys = (int*)take((size_t)2 * ncap * sizeof(int));
    P->ranks = (int*)take((size_t)2 * ncap * sizeof(int));
    P->perm = (int*)take((size_t)2 * ncap * sizeof(int));
    P->scan_tmp = (int*)take(kMaxScanTiles * sizeof(int));
    P->grec = take((size_t)ncap * grid_rec_size(P->precision));
    P->prec = (PairRec*)take((size_t)ncap * sizeof(PairRec));
    P->ppos = (double4*)take((size_t)ncap * sizeof(double4));
    P->pair_hits = (int*)take((size_t)3 * ncap * kPairCap * sizeof(int));
    P->pair_count = (int*)take((size_t)3 * ncap * sizeof(int));
    P->corr = (double*)take((size_t)6 * ncap * sizeof(double));
    P->partial = (double*)take(1024 * sizeof(double));
    P->flag = (int*)take(16 * sizeof(int));
    P->side = nullptr;
    P->fork = P->join = nullptr;
    P->timing = 0;
    P->events = nullptr;
}

// twiddles exp(-2 pi i m / n) for n = M, My, Mz in turn (FP64 sincospi,
// rounded once to the grid precision)
template <typename R>
__global__ void k_static_twiddles(R* __restrict__ tw, int M, int My, int Mz) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M + My + Mz) return;
    int n = M, m = t;
    if (m >= M) {
        m -= M;
        n = My;
        if (m >= My) {
            m -= My;
            n = Mz;
        }
    }
    double sn, cs;
    sincospi(-2.0 * (double)m / (double)n, &sn, &cs);
    tw[2 * t] = (R)cs;
    tw[2 * t + 1] = (R)sn;
}

hipError_t launch_static_twiddles(const fcm_plan_impl* P, hipStream_t st) {
    const int n = P->M + P->My + P->Mz;
    const int blocks = (n + 255) / 256;
    if (P->precision == FCM_FP64)
        hipLaunchKernelGGL(k_static_twiddles<double>, dim3(blocks), dim3(256), 0, st, (double*)P->twid, P->M,
                           P->My, P->Mz);
    else
        hipLaunchKernelGGL(k_static_twiddles<float>, dim3(blocks), dim3(256), 0, st, (float*)P->twid, P->M,
                           P->My, P->Mz);
    return hipGetLastError();
}

}  // namespace

extern "C" {

int fcm_options_default(fcm_options* opt) {
    if (!opt) return FCM_EINVAL;
    opt->eta = 1.0;
    opt->support = 0;
    opt->sigma_D_grid = 0.0;
    opt->precision = FCM_FP32_BULK;
    opt->kahan = 0;
    return FCM_OK;
}

int fcm_plan_footprint(int64_t N, int grid, int precision, int64_t* bytes) {
    // An upper bound over every box, width, support and cut-off: at most one
    // grid bin per grid point (supports as long as the grid leave tiles of
    // one point) and kMaxCellsPerAxis^3 pair cells.
    if (!bytes || N <= 0 || N > (int64_t)1 << 29 || !is_smooth_even(grid)) return FCM_EINVAL;
    if (precision != FCM_FP64 && precision != FCM_FP32_BULK) return FCM_EINVAL;
    const int g3[3] = {grid, grid, grid};
    const int64_t nbins = (int64_t)grid * grid * grid;
    const int cells = kMaxCellsPerAxis * kMaxCellsPerAxis * kMaxCellsPerAxis;
    *bytes = plan_bytes(N, g3, precision, cells, (int)std::min<int64_t>(nbins, 1 << 30));
    return FCM_OK;
}

int fcm_plan_footprint_box(int64_t N, const double L[3], double a, double sigma_delta,
                           const int grid[3], double r_cut, const fcm_options* opt, int64_t* bytes) {
    if (!bytes) return FCM_EINVAL;
    fcm_plan_impl d;
    const int st = plan_derive(&d, N, L, a, sigma_delta, grid, r_cut, opt);
    if (st != FCM_OK) return st;
    const int g3[3] = {d.M, d.My, d.Mz};
    *bytes = plan_bytes(N, g3, d.precision, d.ncells, d.nbins);
    return FCM_OK;
}

int fcm_plan(fcm_plan_t* out, int64_t N, double L, double a, double sigma_delta, int grid,
             double r_cut) {
    return fcm_plan_ex(out, N, L, a, sigma_delta, grid, r_cut, nullptr);
}

int fcm_plan_ex(fcm_plan_t* out, int64_t N, double L, double a, double sigma_delta, int grid,
                double r_cut, const fcm_options* opt_in) {
    const double L3[3] = {L, L, L};
    const int g3[3] = {grid, grid, grid};
    return fcm_plan_box(out, N, L3, a, sigma_delta, g3, r_cut, opt_in);
}

int fcm_plan_box(fcm_plan_t* out, int64_t N, const double L[3], double a, double sigma_delta,
                 const int grid[3], double r_cut, const fcm_options* opt_in) {
    if (!out) return FCM_EINVAL;
    *out = nullptr;
    fcm_plan_impl* P = new (std::nothrow) fcm_plan_impl;
    if (!P) return FCM_ENOMEM;
    memset(P, 0, sizeof(*P));
    int st = fcm::plan_derive(P, N, L, a, sigma_delta, grid, r_cut, opt_in);
    if (st == FCM_OK) st = fcm::plan_allocate(P, N, P->ncells);
    if (st != FCM_OK) {
        free_plan(P);
        return st;
    }
    *out = P;
    return FCM_OK;
}

int fcm_plan_destroy(fcm_plan_t p) {
    if (!p) return FCM_EINVAL;
    DeviceGuard g(p->device);
    (void)hipDeviceSynchronize();
    free_plan(p);
    return FCM_OK;
}

int fcm_plan_info(fcm_plan_t p, int64_t* N, int* grid, int* support, int* precision,
                  int* cells_per_axis) {
    if (!p) return FCM_EINVAL;
    if (N) *N = p->N;
    if (grid) *grid = p->M;
    if (support) *support = p->MG;
    if (precision) *precision = p->precision;
    if (cells_per_axis) *cells_per_axis = p->m;
    return FCM_OK;
}

int fcm_plan_box_info(fcm_plan_t p, double L[3], int grid[3], int cells[3]) {
    if (!p) return FCM_EINVAL;
    if (L) {
        L[0] = p->L;
        L[1] = p->Ly;
        L[2] = p->Lz;
    }
    if (grid) {
        grid[0] = p->M;
        grid[1] = p->My;
        grid[2] = p->Mz;
    }
    if (cells) {
        cells[0] = p->m;
        cells[1] = p->mcy;
        cells[2] = p->mcz;
    }
    return FCM_OK;
}

namespace {

// The mobility after the records are in place (from a new sort, or refreshed
// forces at the last sort's positions): pair correction on the side stream
// (with a fresh neighbour search when `scan`), spread, solve, interpolation.
hipError_t mobility_from_records(fcm_plan_impl* p, const double* T, double* V, double* Omega,
                                 hipStream_t st, hipEvent_t* ev, bool scan) {
    const bool corr = needs_correction(p);
    hipError_t e = hipSuccess;
    // The pair correction depends only on the sorted records: it runs on the
    // plan's side stream while spread and FFT run here, into the plan's
    // correction buffer, which the interpolation adds to its results.
    if (corr && !p->side) {
        // a plan without a side stream (the static entry point) runs the pair
        // correction on the call's stream, before the grid part
        e = launch_pair(p, p->corr, Omega ? p->corr + 3 * p->N : nullptr, T != nullptr, st, true, scan);
    } else if (corr) {
        e = hipEventRecord(p->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->fork, 0);
        if (ev && e == hipSuccess && timing_event(p, 10)) (void)hipEventRecord(ev[10], p->side);
        if (e == hipSuccess)
            e = launch_pair(p, p->corr, Omega ? p->corr + 3 * p->N : nullptr, T != nullptr, p->side,
                            true, scan);
        if (ev && e == hipSuccess && timing_event(p, 11)) (void)hipEventRecord(ev[11], p->side);
        if (e == hipSuccess) e = hipEventRecord(p->join, p->side);
    } else if (ev && timing_event(p, 10)) {
        (void)hipEventRecord(ev[10], st);
        (void)hipEventRecord(ev[11], st);
    }
    // the field stays inside the call, so spread, solve and interpolation may
    // pass it along in the tiled layout
    const bool tiled = solve_tiles(p);
    if (e == hipSuccess) e = launch_spread(p, T != nullptr, p->grid, st, tiled);
    if (e == hipSuccess) e = launch_solve(p, p->grid, st, ev ? ev + 2 : nullptr, tiled);
    if (e == hipSuccess && corr && p->side) e = hipStreamWaitEvent(st, p->join, 0);
    if (e == hipSuccess) e = launch_interp(p, p->grid, V, Omega, st, tiled, corr ? p->corr : nullptr);
    return e;
}

}  // namespace

int fcm_mobility(fcm_plan_t p, const double* pos, const double* F, const double* T, double* V,
                 double* Omega, void* stream) {
    if (!p || !pos || !F || !V) return FCM_EINVAL;
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    p->last_stream = st;
    hipEvent_t* ev = call_events(p);
    auto mark = [&](int i) {
        if (ev && timing_event(p, i)) (void)hipEventRecord(ev[i], st);
    };
    mark(0);
    const bool corr = needs_correction(p);
    hipError_t e = sort_particles(p, pos, st);
    if (e == hipSuccess)
        e = corr ? launch_gather_both(p, pos, F, T, st) : launch_gather_grid(p, pos, F, T, st);
    mark(1);
    if (e == hipSuccess) e = mobility_from_records(p, T, V, Omega, st, ev, true);
    mark(8);
    mark(9);
    // the records (and the pair lists) now describe these positions
    if (e == hipSuccess) p->repeat_ok = 1;
    return map_err(e);
}

int fcm_mobility_repeat(fcm_plan_t p, const double* F, const double* T, double* V, double* Omega,
                        void* stream) {
    if (!p || !F || !V) return FCM_EINVAL;
    if (!p->repeat_ok) return FCM_EINVAL;
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    p->last_stream = st;
    hipEvent_t* ev = call_events(p);
    auto mark = [&](int i) {
        if (ev && timing_event(p, i)) (void)hipEventRecord(ev[i], st);
    };
    mark(0);
    const bool corr = needs_correction(p);
    // The pair records are read by the previous call's correction on the side
    // stream until its join, which this stream has already waited for.
    hipError_t e = launch_refresh_forces(p, F, T, corr, st);
    mark(1);
    if (e == hipSuccess) e = mobility_from_records(p, T, V, Omega, st, ev, false);
    mark(8);
    mark(9);
    if (e != hipSuccess) p->repeat_ok = 0;
    return map_err(e);
}

int fcm_brownian_reserve(fcm_plan_t p, int max_iter) {
    if (!p || max_iter < 1 || max_iter > 64) return FCM_EINVAL;
    DeviceGuard g(p->device);
    if (p->krylov && p->krylov_cap >= max_iter) return FCM_OK;
    if (p->krylov) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p->krylov);
        p->krylov = nullptr;
        p->krylov_cap = 0;
    }
    hipError_t e = hipMalloc((void**)&p->krylov, (size_t)(max_iter + 1) * 3 * p->Ncap * sizeof(double));
    if (e != hipSuccess) {
        p->krylov = nullptr;
        return map_err(e);
    }
    p->krylov_cap = max_iter;
    return FCM_OK;
}

int fcm_brownian(fcm_plan_t p, const double* pos, const void* xi_grid, const double* xi_pair,
                 double kT, double tol, double* V, int* iterations, void* stream) {
    if (!p || !pos || !xi_grid || !V || !(kT >= 0.0) || !isfinite(kT) || !(tol > 0.0))
        return FCM_EINVAL;
    const bool corr = needs_correction(p);
    if (corr && (!xi_pair || !p->krylov)) return FCM_EINVAL;
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    p->last_stream = st;
    const int n = (int)(3 * p->N);
    hipError_t e = sort_particles(p, pos, st);
    if (e == hipSuccess)
        e = corr ? launch_gather_both(p, pos, nullptr, nullptr, st)
                 : launch_gather_grid(p, pos, nullptr, nullptr, st);
    int it = 0;
    // grid part: J~ G^(1/2) xi_grid, with the noise copied into the plan's
    // grid, queued on the call's stream first so that it runs while the host
    // drives the Lanczos steps of the pair part on the side stream
    const size_t nb = (size_t)3 * p->M * p->My * p->Mz * real_size(p->precision);
    if (e == hipSuccess && corr) {
        e = hipEventRecord(p->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->fork, 0);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(p->grid, xi_grid, nb, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = launch_solve(p, p->grid, st, nullptr, false, true);
    if (e == hipSuccess) e = launch_interp(p, p->grid, V, nullptr, st, false, nullptr);
    // pair part y = C^(1/2) xi_pair into the correction buffer (side stream)
    if (e == hipSuccess && corr) {
        e = lanczos_sqrt_pair(p, xi_pair, p->corr, tol, &it, p->side);
        if (e == hipSuccess) e = hipEventRecord(p->join, p->side);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, p->join, 0);
    }
    // V = sqrt(2 kT / dV) J~ G^(1/2) xi_grid + sqrt(2 kT) y
    const double dV = p->dx * p->dx * p->dx;
    if (e == hipSuccess) {
        if (corr)
            e = launch_axpby(sqrt(2.0 * kT), p->corr, sqrt(2.0 * kT / dV), V, n, st);
        else
            e = launch_axpby(0.0, V, sqrt(2.0 * kT / dV), V, n, st);
    }
    if (iterations) *iterations = it;
    return map_err(e);
}

int fcm_plan_set_timing(fcm_plan_t p, int enable) {
    if (!p || enable < 0 || enable >= 2 + FCM_NUM_STAGES) return FCM_EINVAL;
    DeviceGuard g(p->device);
    if (enable && !p->events) {
        const int n = kMaxTimedCalls * kEvPerCall;
        p->events = (hipEvent_t*)calloc(n, sizeof(hipEvent_t));
        if (!p->events) return FCM_ENOMEM;
        p->ev_cap = kMaxTimedCalls;
        for (int i = 0; i < n; ++i) {
            hipError_t e = hipEventCreate(&p->events[i]);
            if (e != hipSuccess) {
                free_events(p);
                return map_err(e);
            }
        }
    }
    p->timing = enable;
    p->ev_calls = 0;
    return FCM_OK;
}

int fcm_plan_stage_times(fcm_plan_t p, double* ms_out, int* ncalls) {
    if (!p || !ms_out) return FCM_EINVAL;
    DeviceGuard g(p->device);
    for (int s = 0; s < FCM_NUM_STAGES; ++s) ms_out[s] = 0.0;
    const int n = p->events ? p->ev_calls : 0;
    if (n > 0) {
        const size_t last = (size_t)(n - 1) * kEvPerCall + timing_last_event(p);
        hipError_t e = hipEventSynchronize(p->events[last]);
        if (e != hipSuccess) return map_err(e);
    }
    for (int c = 0; c < n; ++c) {
        hipEvent_t* ev = p->events + (size_t)c * kEvPerCall;
        for (int s = 0; s < FCM_NUM_STAGES; ++s) {
            // the pair correction (last stage) is timed on the side stream
            const int b = s == FCM_NUM_STAGES - 1 ? 10 : s, t = s == FCM_NUM_STAGES - 1 ? 11 : s + 1;
            if (!timing_event(p, b) || !timing_event(p, t)) continue;   // stage not timed
            float ms = 0.0f;
            hipError_t e = hipEventElapsedTime(&ms, ev[b], ev[t]);
            if (e != hipSuccess) return map_err(e);
            ms_out[s] += ms;
        }
    }
    if (ncalls) *ncalls = n;
    p->ev_calls = 0;
    return FCM_OK;
}

int fcm_spread(fcm_plan_t p, const double* pos, const double* F, const double* T, void* grid_out,
               void* stream) {
    if (!p || !pos || !F || !grid_out) return FCM_EINVAL;
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    p->last_stream = st;
    hipError_t e = sort_particles(p, pos, st);
    if (e == hipSuccess) e = launch_gather_grid(p, pos, F, T, st);
    if (e == hipSuccess) e = launch_spread(p, T != nullptr, grid_out, st);
    return map_err(e);
}

int fcm_solve(fcm_plan_t p, void* grid_inout, void* stream) {
    if (!p || !grid_inout) return FCM_EINVAL;
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    p->last_stream = st;
    return map_err(launch_solve(p, grid_inout, st));
}

int fcm_interp(fcm_plan_t p, const double* pos, const void* grid_in, double* V, double* Omega,
               void* stream) {
    if (!p || !pos || !grid_in || !V) return FCM_EINVAL;
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    p->last_stream = st;
    hipError_t e = sort_particles(p, pos, st);
    if (e == hipSuccess) e = launch_gather_grid(p, pos, nullptr, nullptr, st);
    if (e == hipSuccess) e = launch_interp(p, grid_in, V, Omega, st);
    return map_err(e);
}

int fcm_correct(fcm_plan_t p, const double* pos, const double* F, const double* T, double* V,
                double* Omega, void* stream) {
    if (!p || !pos || !F || !V) return FCM_EINVAL;
    DeviceGuard g(p->device);
    hipStream_t st = (hipStream_t)stream;
    p->last_stream = st;
    if (!needs_correction(p)) return FCM_OK;
    hipError_t e = sort_particles(p, pos, st);
    if (e == hipSuccess) e = launch_gather_pair(p, pos, F, T, st);
    if (e == hipSuccess) e = launch_pair(p, V, Omega, T != nullptr, st);
    return map_err(e);
}

int fcm_plan_last_error(fcm_plan_t p) {
    if (!p) return FCM_EINVAL;
    DeviceGuard g(p->device);
    hipError_t e = hipStreamSynchronize(p->last_stream);
    if (e != hipSuccess) return map_err(e);
    int h = 0;
    e = hipMemcpy(&h, p->flag, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return map_err(e);
    if (h) {
        e = hipMemset(p->flag, 0, sizeof(int));
        if (e != hipSuccess) return map_err(e);
        return FCM_ENONFINITE;
    }
    return FCM_OK;
}

int fcm_mobility_static(int64_t N, double L, double a, double sigma_delta, int grid, double r_cut,
                        const fcm_options* opt, const double* pos, const double* F, const double* T,
                        double* V, double* Omega, void* stream) {
    if (!pos || !F || !V) return FCM_EINVAL;
    fcm_plan_impl P;
    const double L3[3] = {L, L, L};
    const int g3[3] = {grid, grid, grid};
    int st = plan_derive(&P, N, L3, a, sigma_delta, g3, r_cut, opt);
    if (st != FCM_OK) return st;
    // the buffers, each rounded up to 256 bytes, must fit the scratch
    if (plan_bytes(N, g3, P.precision, P.ncells, P.nbins) + 16 * 256 > kStaticScratchBytes)
        return FCM_ESCRATCH;
    unsigned char* base = nullptr;
    st = static_scratch(&base, &P.device);
    if (st != FCM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    carve_static_plan(&P, base);
    // The scratch keeps the last call's contents: the counters (cleared by the
    // sort, as after a plan's allocation) and the flags must start at zero, and
    // the twiddles are rebuilt for this grid.
    P.counts_dirty = 1;
    hipError_t e = launch_fill(P.flag, 16, 0, s);
    if (e == hipSuccess) e = launch_static_twiddles(&P, s);
    const bool corr = needs_correction(&P);
    if (e == hipSuccess) e = sort_particles(&P, pos, s);
    if (e == hipSuccess)
        e = corr ? launch_gather_both(&P, pos, F, T, s) : launch_gather_grid(&P, pos, F, T, s);
    if (e == hipSuccess) e = mobility_from_records(&P, T, V, Omega, s, nullptr, true);
    return map_err(e);
}

const char* fcm_status_string(int status) {
    switch (status) {
        case FCM_OK: return "ok";
        case FCM_EINVAL: return "invalid argument";
        case FCM_ENOMEM: return "out of memory";
        case FCM_EDEVICE: return "HIP runtime error";
        case FCM_ERANGE: return "cut-off radius must be below half the box";
        case FCM_ENONFINITE: return "non-finite position in the last call";
        case FCM_ESCRATCH: return "problem needs more than the static scratch of fcm_mobility_static (64 MiB per GPU)";
        default: return "unknown status";
    }
}

}  // extern "C"
