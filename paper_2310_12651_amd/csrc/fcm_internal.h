// Internal definitions shared by the translation units of the fast-FCM HIP
// library (plan layout, per-particle records, kernel argument blocks and
// launchers).  Not part of the public C ABI (include/fcm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fcm.h"

namespace fcm {

constexpr int kMaxRadixStages = 16;
constexpr int kMaxSupport = 32;      // largest M_G accepted
constexpr int kMaxGrid = 1024;       // largest grid per axis accepted
constexpr int kMaxCellsPerAxis = 128;
constexpr int kMaxScanTiles = 8192;     // block sums of the bin and cell scans (scan_tmp)
constexpr int kPairCap = 48;         // neighbours recorded per (particle, z layer)

template <typename R>
struct C2 {
    R x, y;
};

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each with
// its own L2.  Map the b-th dispatched block of nb to a logical block so that
// every XCD receives one contiguous run of logical blocks: neighbouring work
// (sorted particles, adjacent grid columns) then shares one L2.
__device__ inline int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, l = b >> 3;
    return x * q + (x < r ? x : r) + l;
}

// Per-particle record of the grid kernels, in grid-bin order.  s[] is the
// first support point along each axis (mod M), f[] the particle coordinate in
// grid units minus the unwrapped first support point (so the displacement of
// support point j is (j - f) dx), F and T are the force and the torque scaled
// by the kernel normalisation (and by 1/(2 Sigma_D^2) for T).
template <typename R>
struct alignas(16) GridRec {
    int s[3];
    int orig;
    R f[3];
    R F[3];
    R T[3];
};

// Per-particle record of the pair kernel, in pair-cell order.
struct alignas(16) PairRec {
    double y[3];
    int orig;
    int cell;
    double F[3];
    double T[3];
};

// A length-n mixed-radix Stockham plan.  Per stage s: radix rad[s], the
// product ns[s] of the radices before it, the butterflies per line nb[s] =
// n / rad[s], and the twiddle step tstep[s] = M / (ns[s] rad[s]) into the
// length-M table.  Divisions by ns and nb use multipliers m = 2^32/d + 1
// (exact for numerators and divisors below 2^16; d = 1 is special-cased).
struct RadixPlan {
    int n;                                 // transform length
    int nst;                               // number of stages
    int rad[kMaxRadixStages];
    int ns[kMaxRadixStages];
    unsigned nsm[kMaxRadixStages];
    int nb[kMaxRadixStages];
    unsigned nbm[kMaxRadixStages];
    int tstep[kMaxRadixStages];
    unsigned nm;                           // multiplier for division by n
};

__host__ __device__ inline unsigned div_magic(unsigned d) {
    return d <= 1 ? 0u : (unsigned)(0x100000000ull / d + 1ull);
}

// Word 3 of a raw buffer resource (32-bit data format, as for all gfx9-family
// raw buffers).  Buffer loads address with one 32-bit lane offset plus a
// scalar offset, so wavefront-uniform parts of an address stay in scalar
// registers; reads past num_records return 0.
constexpr int kBufferWord3 = 0x00020000;

__device__ inline int fast_div(int j, int d, unsigned m) {
    return d == 1 ? j : (int)__umulhi((unsigned)j, m);
}

// Scalars of the grid kernels (one plan).
template <typename R>
struct GridArgs {
    int M, My, Mz;                 // grid points along x, y, z
    int MG, N;
    int TX, TY, TZ;                // spread tile (points)
    unsigned long long rowrep;     // bit TX*j set for each tile row j < TY (lane = x + TX y)
    int nbx, nby, nbz;             // tiles (= bins) per axis
    int backx, backy, backz;       // bins scanned before the tile's own
    int mgmul;                     // 65536 / MG + 1: e / MG = (e * mgmul) >> 16 for e < 1024
    int tiled;                     // interp: field in the x-y tiled layout
    int zfold;                     // M_G > Mz: one tile spans z, support points folded
    R dx;                          // grid spacing
    R e2;                          // log2(e) / (2 Sigma^2)
    R e2D;                         // log2(e) / (2 Sigma_D^2)
    R A, B;                        // Delta~ = Delta (A + B r^2)
    R dV;                          // dx^3
    int same_width;                // Sigma_D == Sigma
};

struct PairArgs {
    int N;
    int mx, my, mz;                // pair cells per axis
    double Lx, Ly, Lz;             // box sides
    double iLx, iLy, iLz;          // and their reciprocals
    double cwx, cwy, cwz;          // cell widths
    double rc2;                    // smallest r^2 with sqrt(r^2) >= R_c (the cut-off test)
    double eta, sigma, sigmaD, Sigma, SigmaD;
    double selfVF, selfOT;
    int with_pairs;                // 0 = only self corrections (R_c = 0)
    int store;                     // 1 = write the corrections, 0 = add them
    // the six Gaussian widths of the corrections: squared width s, erfc
    // argument scale 1/sqrt(2 s), exponent scale -1/(2 s), norm (2 pi s)^(-3/2)
    double wsq[6], escale[6], gnorm[6];
    // constants of the correction blocks (d = sigma^2 - Sigma^2, s2 = 2 Sigma^2,
    // sb = Sigma^2 + Sigma_D^2): 1/(8 pi eta), 1/(2 eta), d/eta, d^2/(4 eta s2),
    // d/(4 eta sb), 1/s2
    double c8, ch, deta, cq, cfb, is2;
};

}  // namespace fcm

struct fcm_plan_impl {
    int device;
    int64_t N;
    int64_t Ncap;          // particles the buffers hold
    int cells_cap;         // pair cells the buffers hold
    double L, a, eta;      // L: box side along x
    double Ly, Lz;         // box sides along y and z (L for a cube)
    double sigma, sigmaD, Sigma, SigmaD;
    double rc, dx;         // dx: grid spacing, the same on all axes
    int M, H, MG;          // M: grid points along x, H = M / 2
    int My, Mz;            // grid points along y and z (M for a cube)
    int cubic;             // M == My == Mz
    int precision, kahan;
    // spread tiling / grid bins
    int TX, TY, TZ, nbx, nby, nbz, nbins;
    int backx, backy, backz;
    // pair cells: m along x, mcy and mcz along y and z
    int m, mcy, mcz, ncells;
    // FFT: radH (length M/2, the x pass), radY and radZ (lengths My and Mz);
    // twiddle tables of lengths M, My, Mz one after the other in twid
    fcm::RadixPlan radH, radY, radZ;
    int Wx, Wy, Wz;
    // closed-form constants
    double selfVF, selfOT;
    // device buffers
    void* grid;            // 3 M^3 reals (working field / spectrum)
    void* twid;            // M + My + Mz complex: exp(-2 pi i m / n) for n = M, My, Mz
    int* counts;           // nbins + ncells (+2) counters
    int* starts;           // exclusive scans: bins then cells
    int* keys;             // 2N keys (bin, cell)
    int* ranks;            // 2N ranks within key; after the sort, the inverse permutations
    int* perm;             // 2N: grid order then pair order
    int* scan_tmp;         // block sums of the scan
    void* grec;            // N GridRec
    fcm::PairRec* prec;    // N PairRec
    double4* ppos;         // N wrapped positions in pair order (w unused)
    int* pair_hits;        // 3N x kPairCap neighbours found by the pair scan
    int* pair_count;       // 3N neighbour counts
    double* corr;          // 6N: pair + self corrections of V (3N) then Omega (3N)
    double* krylov;        // Brownian pair part: (krylov_cap + 1) x 3N Lanczos basis, or NULL
    int krylov_cap;        // Lanczos steps the basis holds
    double* partial;       // 1024 partial sums of the vector reductions
    hipStream_t side;      // the pair correction runs here, beside spread and FFT
    hipEvent_t fork, join; // sorted records ready / corrections ready
    int* flag;             // [0] non-finite position seen; [1], [2] segment-sort work-list lengths
    hipStream_t last_stream;
    int counts_dirty;      // counts may be non-zero (cleared by the next sort)
    int repeat_ok;         // the sorted records and pair lists belong to the last
                           // fcm_mobility's positions (fcm_mobility_repeat may run)
    // per-stage timing
    int timing;             // 0 off, 1 every stage, 2 + s stage s only
    int ev_calls;           // calls recorded
    int ev_cap;             // event sets allocated
    hipEvent_t* events;     // ev_cap * (FCM_NUM_STAGES + 1)
};

// Whether event i of a timed call is recorded.  Events 0..8 are the stage
// boundaries on the call's stream (stage s runs from event s to s + 1), 9 the
// end of the call, 10 and 11 the start and end of the pair correction on the
// side stream (the last stage).  Timing mode 1 records all of them; mode 2 + s
// only stage s's two, so that a call timed for one kernel carries two events
// instead of twelve.
inline bool timing_event(const fcm_plan_impl* P, int i) {
    if (P->timing <= 1) return true;
    const int s = P->timing - 2;
    if (s == 8) return i == 10 || i == 11;
    return i == s || i == s + 1;
}

// The last event a timed call records (the one to wait for before reading).
inline int timing_last_event(const fcm_plan_impl* P) {
    if (P->timing <= 1) return 9;
    const int s = P->timing - 2;
    return s == 8 ? 11 : s + 1;
}

// ---- launchers (each enqueues on `st`; return hipError_t of the launch) ----
namespace fcm {

hipError_t launch_fill(int* p, int n, int v, hipStream_t st);
// wrap + hash (Sec. 4, spatial hashing) for the grid bins and the pair cells
hipError_t launch_hash(const fcm_plan_impl* P, const double* pos, hipStream_t st);
// exclusive scans of the bin and cell counts into starts (each with its total
// appended); clears the counts
hipError_t launch_scan(const fcm_plan_impl* P, hipStream_t st);
// counting-sort scatter and in-segment ordering by original index
hipError_t launch_scatter(const fcm_plan_impl* P, hipStream_t st);
// the per-particle records in sorted order (built from the caller's order)
hipError_t launch_gather_grid(const fcm_plan_impl* P, const double* pos, const double* F,
                              const double* T, hipStream_t st);
hipError_t launch_gather_pair(const fcm_plan_impl* P, const double* pos, const double* F,
                              const double* T, hipStream_t st);
// both of the above in one launch
hipError_t launch_gather_both(const fcm_plan_impl* P, const double* pos, const double* F,
                              const double* T, hipStream_t st);
// new forces and torques into the records of the last sort (grid records, and
// pair records when `pair`); T may be null (zero torques)
hipError_t launch_refresh_forces(const fcm_plan_impl* P, const double* F, const double* T,
                                 bool pair, hipStream_t st);

// tiled: write the field in the x-y tiled layout of launch_solve
hipError_t launch_spread(const fcm_plan_impl* P, bool torque, void* grid, hipStream_t st,
                         bool tiled = false);
// tiled: the field is in the x-y tiled layout written by launch_solve(..., tiled);
// corr: NULL, or corrections added to the results (V part, then Omega part at + 3N)
hipError_t launch_interp(const fcm_plan_impl* P, const void* grid, double* V, double* W,
                         hipStream_t st, bool tiled = false, const double* corr = nullptr);
// ev: NULL or 6 events recorded before/between/after the five FFT passes
// tiled: the force field arrives, and the velocity field leaves, in the x-y
// tiled layout (tiles of 8 x by 4 y, x fastest inside a tile, tiles x fastest,
// then tile rows, then z); only when the plan supports it (solve_tiles)
// root: multiply by the square root P(k) / sqrt(eta k^2) of the solve's
// Fourier multiplier instead (the grid part of Brownian velocities)
hipError_t launch_solve(const fcm_plan_impl* P, void* grid, hipStream_t st,
                        hipEvent_t* ev = nullptr, bool tiled = false, bool root = false);
bool solve_tiles(const fcm_plan_impl* P);
// store: write the corrections to V and W (else add them); scan: search the
// neighbours first (else reuse the lists of the last search, same positions)
hipError_t launch_pair(const fcm_plan_impl* P, double* V, double* W, bool torque,
                       hipStream_t st, bool store = false, bool scan = true);

// Brownian pair part: y = C^(1/2) xi (caller order, N x 3) for the VF
// correction matrix C, by Lanczos steps (at most the plan's krylov_cap) until
// the relative change of y is below tol; needs the sorted records of the
// positions; iters receives the steps taken.  Host-synchronous.
hipError_t lanczos_sqrt_pair(fcm_plan_impl* P, const double* xi, double* y, double tol,
                             int* iters, hipStream_t st);
// y = alpha x + beta y over n doubles
hipError_t launch_axpby(double alpha, const double* x, double beta, double* y, int n,
                        hipStream_t st);

// plan construction pieces (fcm_api.hip), shared with the request server
int fft_maxe(int precision, bool zpass);
int plan_derive(fcm_plan_impl* P, int64_t N, const double L[3], double a, double sigma_delta,
                const int grid[3], double r_cut, const fcm_options* opt);
int plan_allocate(fcm_plan_impl* P, int64_t ncap, int cellcap);
int plan_rebind(fcm_plan_impl* P, const fcm_plan_impl* derived);
void plan_free(fcm_plan_impl* P);
int64_t plan_bytes(int64_t ncap, const int grid[3], int precision, int cellcap, int nbins);

}  // namespace fcm
