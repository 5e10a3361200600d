/*
 * fcm.h -- C ABI of the fast force-coupling-method (fast FCM) mobility library
 * for AMD Instinct MI355X (gfx950).
 *
 * Fast FCM (Su & Keaveny, arXiv 2310.12651) applies the periodic FCM mobility
 * of N spheres of radius a: given positions Y_n, forces F_n and torques T_n in
 * the triply periodic box [0, L)^3 with viscosity eta, it returns the particle
 * velocities V_n and angular velocities Omega_n (Sec. 2, Sec. 3.4, eq.
 * symmetric_FFT_mod).  It spreads F and T onto a grid with kernels of the
 * widened width Sigma (Sec. 3, modified kernel Delta~; Sec. 3.4, eq.
 * torque_kernel_mod), solves Stokes flow in Fourier space (Sec. 2.1),
 * interpolates back (Sec. 3.1, eq. avg_particle_vel_mod; Sec. 3.4,
 * eq. avg_particle_rot_mod), and adds the pairwise correction M - M~ for pairs
 * closer than R_c plus the self correction (Sec. 3.2 eq. correction_VF,
 * Sec. 3.4 eqs. correction_WF and correction_WT, App. B), following the steps
 * of Sec. 4.
 *
 * Conventions (all calls):
 *  - Every call returns an int status: FCM_OK (0) or a negative FCM_E* code.
 *    No C++ exception crosses this interface.
 *  - Particle arrays are DEVICE pointers to N x 3 row-major FP64 values
 *    (x, y, z interleaved per particle) on the device the plan was created on.
 *    The caller owns them.  Outputs are written in the caller's particle order.
 *  - Positions may lie anywhere; they are wrapped into [0, L) by the exact
 *    floating-point remainder (plus L for negative values; a result that
 *    rounds to L becomes 0).  Non-finite positions are replaced by 0 and
 *    reported by fcm_plan_last_error().
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *    and return without waiting; results are ready when the stream reaches
 *    them.  A plan owns scratch buffers, so concurrent calls on one plan race:
 *    use one plan per concurrently used stream.
 *  - fcm_mobility and fcm_mobility_repeat allocate nothing and never wait on
 *    the host, so they may be captured into a HIP graph (stream capture on a
 *    non-null stream; the pair correction's side stream joins the capture
 *    through the plan's own events).  A replay reads the particle arrays named
 *    at capture, so new inputs are written into those arrays.  The graph refers
 *    to the plan's buffers, side stream and events: destroy every such graph
 *    before fcm_plan_destroy.
 *  - Grid fields exchanged by the stage calls are DEVICE buffers of
 *    3 * grid^3 values in the plan's grid precision (double for FCM_FP64,
 *    float for FCM_FP32_BULK), component-major, x fastest:
 *    field[c * grid^3 + i + grid * (j + grid * k)] is component c at the grid
 *    point (i, j, k) * L / grid.
 *  - Units: mobilities scale as 1/eta (default eta = 1).
 */
#ifndef FCM_H
#define FCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcm_plan_impl* fcm_plan_t;

enum {
    FCM_OK = 0,
    FCM_EINVAL = -1,      /* an argument is out of its documented range            */
    FCM_ENOMEM = -2,      /* device or host allocation failed                      */
    FCM_EDEVICE = -3,     /* a HIP runtime call failed                             */
    FCM_ERANGE = -4,      /* r_cut >= L/2: pairs would need more than one image    */
    FCM_ENONFINITE = -5,  /* non-finite input seen by the last call (see below)    */
    FCM_ESCRATCH = -7     /* too large for fcm_mobility_static's 64 MiB scratch    */
};

/* Precision of the grid part (spreading, FFT Stokes solve, interpolation).
 * The pair correction and the final V, Omega are FP64 in both modes. */
enum { FCM_FP64 = 0, FCM_FP32_BULK = 1 };

typedef struct {
    double eta;          /* viscosity; default 1                                        */
    int support;         /* M_G, grid points per direction of a kernel's support
                            (Sec. 2.1); 0 = smallest even >= 10 Sigma/dx, at least 8    */
    double sigma_D_grid; /* Sigma_D, width of the torque kernel on the grid (Sec. 3.4);
                            0 = Sigma, the paper's choice                                */
    int precision;       /* FCM_FP64 or FCM_FP32_BULK (default)                          */
    int kahan;           /* FP32 spreading sums: 0 plain FP32 (default: a grid point
                            receives a few tens of terms at most), 1 Kahan-compensated,
                            2 FP64 accumulators                                          */
} fcm_options;

/* Fill `opt` with the defaults listed above. */
int fcm_options_default(fcm_options* opt);

/*
 * Create a plan for N particles of radius a in the periodic cube [0, L)^3.
 *   sigma_delta : Sigma, width of the modified Gaussian (Sec. 3); Sigma >= sigma
 *                 = a / sqrt(pi).  Sigma == sigma is standard FCM (no correction);
 *                 widths within 1e-12 (relative) of sigma, and torque widths
 *                 (fcm_options.sigma_D_grid) within 1e-12 of sigma_D, count as
 *                 equal to them.
 *   grid        : grid points per axis, an even 2^p 3^q between 8 and 1024
 *                 (dx = L / grid).
 *   r_cut       : R_c, pair-correction cut-off (Sec. 4); 0 <= R_c < L/2.  R_c = 0:
 *                 no pair search (only the self corrections of App. B, which
 *                 vanish for standard FCM).
 * Allocates every device buffer the plan needs on the current HIP device;
 * later calls allocate nothing.
 * Errors: FCM_EINVAL if N <= 0, L <= 0, a <= 0, Sigma < sigma, the grid is not
 * an even 2^p 3^q in range, or the support exceeds the grid, 32, or (FP64) 24;
 * FCM_ERANGE if
 * r_cut >= L/2; FCM_ENOMEM / FCM_EDEVICE on allocation or runtime failure.
 */
int fcm_plan(fcm_plan_t* out, int64_t N, double L, double a, double sigma_delta,
             int grid, double r_cut);
/* As fcm_plan with options (NULL = defaults). */
int fcm_plan_ex(fcm_plan_t* out, int64_t N, double L, double a, double sigma_delta,
                int grid, double r_cut, const fcm_options* opt);
/*
 * As fcm_plan_ex for the rectangular periodic box [0, L[0]) x [0, L[1]) x
 * [0, L[2]) (host arrays, sides along x, y, z) on a grid of grid[0] x grid[1] x
 * grid[2] points (each an even 2^p 3^q between 8 and 1024).  The grid spacing
 * must be the same on all axes (|L[d]/grid[d] - L[0]/grid[0]| <= 1e-12 of it);
 * the Fourier wave numbers are 2 pi j / L[d] per axis (Sec. 2.1) and the pair
 * cells m_d = max(int(L[d]/R_c), 3) per axis (Sec. 4).  Grid buffers of the
 * stage calls hold 3 x grid[2] x grid[1] x grid[0] values (x fastest).
 * The support M_G may be longer than the z axis when grid[2] is 8, 12 or 16 (the
 * paper's rod runs use 512 x 512 x 8 points, Sec. 6.3): a particle's support
 * then wraps onto itself along z and its coinciding points add, as the
 * periodic sums of Sec. 2.1 read on such a grid.
 * Errors: as fcm_plan_ex; FCM_EINVAL also for unequal spacings, a support
 * longer than the x or y axis, or longer than a z axis other than 8, 12 or 16
 * points; FCM_ERANGE if r_cut >= min(L)/2.
 */
int fcm_plan_box(fcm_plan_t* out, int64_t N, const double L[3], double a, double sigma_delta,
                 const int grid[3], double r_cut, const fcm_options* opt);
/* Release a plan and its device buffers (synchronises the device first). */
int fcm_plan_destroy(fcm_plan_t p);

/*
 * The mobility (Sec. 4, all steps): V, Omega = M (F, T).
 *   pos, F : device, N x 3 FP64.   T : device N x 3 FP64 or NULL (zero torques).
 *   V      : device, N x 3 FP64, overwritten.
 *   Omega  : device, N x 3 FP64, overwritten; or NULL to skip angular velocities.
 */
int fcm_mobility(fcm_plan_t p, const double* pos, const double* F, const double* T,
                 double* V, double* Omega, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): fcm_mobility without a
 * plan.  The arguments are those of fcm_plan_ex followed by those of
 * fcm_mobility (opt may be NULL for the defaults); the results equal those of
 * fcm_mobility on a plan built with the same arguments, to rounding (1e-10
 * relative in FP64, 1e-5 in FP32 bulk).
 * Memory: no allocation of any kind.  Every buffer of the evaluation (field,
 * sort arrays, records, neighbour lists, corrections) lives in a static device
 * array of 64 MiB that each GPU the library runs on holds until the process
 * ends; the pair correction runs on `stream` itself (no side stream).  That
 * bounds the problem: e.g. 10^4 particles on a 128^3 FP32 grid fit.
 * Concurrency: every call on one GPU uses that GPU's single array, so calls
 * that overlap on one GPU (other streams, other threads) race; serialise them.
 * Errors: as fcm_plan_ex and fcm_mobility; FCM_ESCRATCH if the buffers the
 * problem needs exceed the array (nothing is launched then).
 */
int fcm_mobility_static(int64_t N, double L, double a, double sigma_delta, int grid, double r_cut,
                        const fcm_options* opt, const double* pos, const double* F, const double* T,
                        double* V, double* Omega, void* stream);

/*
 * The mobility again at the positions of this plan's last fcm_mobility call,
 * for new forces and torques: repeated applications of M at one configuration,
 * as in the iterative solves for the constraint forces of rigid rods (Sec. 6.1).
 * The particle sort, the sorted positions and the pair neighbour lists of the
 * last call are reused; only the forces and torques of the sorted records are
 * rewritten.  Same argument conventions and results as fcm_mobility with the
 * same pos (bitwise equal: the summation order does not change).
 * Errors: FCM_EINVAL if F or V is NULL, or if the plan's last position-taking
 * call was not a successful fcm_mobility (fcm_spread, fcm_interp and
 * fcm_correct sort again and end the reuse).
 */
int fcm_mobility_repeat(fcm_plan_t p, const double* F, const double* T, double* V,
                        double* Omega, void* stream);

/*
 * Brownian velocities (force-free particles): V = sqrt(2 kT) [M~^(1/2) xi_g +
 * (M - M~)^(1/2) xi_p], whose covariance is 2 kT M (the VF block), built on the
 * positive splitting of Sec. 3.3 as the paper proposes in Sec. 7: the grid part
 * by fluctuating FCM, sqrt(2 kT / dV) J~[G^(1/2) xi_g] with G^(1/2) the Fourier
 * multiplier P(k) / sqrt(eta k^2) (k = 0 and the Nyquist planes removed), the
 * pair part by Lanczos steps whose matrix products are the pair-correction pass.
 *   pos     : device N x 3 FP64 positions.
 *   xi_grid : device noise field, 3 x grid[2] x grid[1] x grid[0] values (x
 *             fastest) in the plan's grid precision, i.i.d. N(0, 1); not modified.
 *   xi_pair : device N x 3 FP64 i.i.d. N(0, 1) (unused, may be NULL, when the
 *             plan needs no correction: standard FCM).
 *   kT      : thermal energy (>= 0).
 *   tol     : Lanczos stops when the relative change of the pair part is below tol.
 *   V       : device N x 3 FP64, overwritten.  iterations: host, Lanczos steps taken.
 * The caller supplies every random number, so results are reproducible.  The
 * Lanczos recurrence runs on the plan's second stream and the host waits for it
 * at each step (the call returns when it has converged); the grid part runs on
 * `stream` meanwhile, and V is complete in stream order.  Requires
 * fcm_brownian_reserve first when a correction is needed (FCM_EINVAL otherwise).
 */
int fcm_brownian(fcm_plan_t p, const double* pos, const void* xi_grid, const double* xi_pair,
                 double kT, double tol, double* V, int* iterations, void* stream);
/* Allocates the Lanczos basis of fcm_brownian for up to max_iter steps (1..64):
 * (max_iter + 1) x 3N FP64.  The one call besides plan creation that allocates. */
int fcm_brownian_reserve(fcm_plan_t p, int max_iter);

/* Stage calls: the operators of Sec. 2.1 / 3.1 / 3.4 one at a time. */

/* grid_out = J~^dagger[F] + N~^dagger[T] on the grid (modified force kernel of
 * width Sigma, torque kernel of width Sigma_D, each truncated to M_G^3 points). */
int fcm_spread(fcm_plan_t p, const double* pos, const double* F, const double* T,
               void* grid_out, void* stream);
/* In place: field -> L^{-1} field, the Fourier Stokes solve (Sec. 2.1 step 2,
 * App. A): u^ = (I - k k^T/k^2) f^ / (eta k^2), u^(0) = 0, and every Fourier mode
 * with index grid/2 along any axis set to 0. */
int fcm_solve(fcm_plan_t p, void* grid_inout, void* stream);
/* V = J~[u], Omega = N~[u] by the trapezoid rule on each particle's support
 * (Omega may be NULL).  V and Omega are overwritten. */
int fcm_interp(fcm_plan_t p, const double* pos, const void* grid_in,
               double* V, double* Omega, void* stream);
/* Adds the pairwise corrections (M - M~)(F, T) for pairs with |Y_n - Y_m| < R_c
 * (minimum image) and the self corrections of App. B into V and Omega. */
int fcm_correct(fcm_plan_t p, const double* pos, const double* F, const double* T,
                double* V, double* Omega, void* stream);

/* Plan properties.  cells_per_axis: m = max(int(L/R_c), 3) pair cells per axis
 * (Sec. 4), at most 128; 1 when R_c = 0 (no pair search). */
int fcm_plan_info(fcm_plan_t p, int64_t* N, int* grid, int* support, int* precision,
                  int* cells_per_axis);
/* Box sides, grid points and pair cells per axis (x, y, z) of a plan; any of
 * the host arrays may be NULL.  For fcm_plan_info, grid and cells_per_axis are
 * those along x. */
int fcm_plan_box_info(fcm_plan_t p, double L[3], int grid[3], int cells[3]);
/* Device bytes an fcm_plan_box with these arguments allocates, exactly (the
 * sum of its buffers: field, twiddles, bin and cell counters, sort arrays,
 * particle records, neighbour lists, corrections; for admission control).
 * Returns the status fcm_plan_box would return for invalid arguments. */
int fcm_plan_footprint_box(int64_t N, const double L[3], double a, double sigma_delta,
                           const int grid[3], double r_cut, const fcm_options* opt, int64_t* bytes);
/* An upper bound of the device bytes of any plan with N particles on a cubic
 * grid of `grid` points in this precision, whatever its box, width, support and
 * cut-off (it counts one grid bin per grid point and the largest number of pair
 * cells).  FCM_EINVAL if N or grid is out of range. */
int fcm_plan_footprint(int64_t N, int grid, int precision, int64_t* bytes);
/* Synchronises the last call's stream and returns FCM_ENONFINITE if that call saw a
 * non-finite position, else FCM_OK; clears the flag. */
int fcm_plan_last_error(fcm_plan_t p);
/*
 * Per-stage timing with HIP events.  When enabled, every fcm_mobility call records
 * its stage boundaries (up to 1024 calls are kept): enable = 1 times every stage,
 * enable = 2 + s only stage s (two events a call instead of twelve, so the other
 * stages run without the events' gaps; the untimed stages read 0), enable = 0
 * stops; other values give FCM_EINVAL.  Changing the mode clears the record, so
 * read it first.  fcm_plan_stage_times
 * synchronises, adds the elapsed milliseconds of each stage over the recorded
 * calls into ms_out[0..FCM_NUM_STAGES), stores the number of calls in *ncalls, and
 * clears the record.  Stages, in order: sort (hash, scan, scatter, records),
 * spread, FFT x forward, FFT y forward, FFT z + projection, FFT y inverse, FFT x
 * inverse, interpolation, pair correction.  The pair correction runs on a second
 * stream of the plan, beside spread and FFT, so the first eight stages add up to
 * the call and the ninth overlaps them.
 */
#define FCM_NUM_STAGES 9
int fcm_plan_set_timing(fcm_plan_t p, int enable);
int fcm_plan_stage_times(fcm_plan_t p, double* ms_out, int* ncalls);

/* Static description of a status code. */
const char* fcm_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* FCM_H */
