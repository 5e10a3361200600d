// Particle bookkeeping of fast FCM (Sec. 4, spatial hashing and sorting):
// periodic wrap, hashing into grid bins (for the spreading tiles) and into
// pair cells of width >= R_c (m = max(int(L/R_c), 3) per axis), a counting
// sort by key, and the per-particle records in sorted order.
//
// The counting sort places particles with atomics and then orders every
// segment by original index, so the sorted order is (key, original index):
// deterministic from run to run.  Segments of up to 16 members are ordered by
// one thread each (in registers), up to 64 by a wavefront, longer ones (dense
// bins, large pair cells) by a workgroup each.  With
// no pair search (R_c = 0) the pair order is the caller's order.  The records are built in the caller's
// order (coalesced reads of positions, forces and torques) and stored at each
// particle's sorted position through the inverse permutation.
#include "fcm_internal.h"

namespace fcm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 4;
constexpr int kScanTile = kScanThreads * kScanPerThread;   // 1024
static_assert((int64_t)kMaxScanTiles * kScanTile >=
                  (int64_t)kMaxCellsPerAxis * kMaxCellsPerAxis * kMaxCellsPerAxis + (1 << 20),
              "scan tiles cover the largest cell grid and a million bins");

struct HashArgs {
    int N, MG;
    int Mv[3];                     // grid points per axis
    int TX, TY, TZ, nbx, nby, nbz, nbins;
    int mc[3];                     // pair cells per axis
    int ident;                     // pair order = caller's order (no cell search)
    double Lv[3], dx, cw[3];       // box sides, grid spacing, cell widths
};

constexpr int kThreadSegment = 16;     // ordered by one thread, in registers
constexpr int kWaveSegment = 64;       // ordered by one wavefront
constexpr int kLdsSegment = 8192;      // ordered by a workgroup's bitonic sort in LDS

// wrap into [0, L): the floating-point remainder (exact for every finite y),
// plus L when negative (one rounding, which may reach L: then 0).  Support
// starts are integers decided from the wrapped value at grid points, so the
// wrap must not round more than this: y - L floor(y / L) differs from it by
// ulps when y lies periods away, or when y / L rounds up to an integer.
// Non-finite values become 0 and raise the plan's flag; every index derived
// from the result is in range.
__device__ inline double wrap_coord(double y, double L, int* bad) {
    if (!isfinite(y)) {
        *bad = 1;
        return 0.0;
    }
    double w = fmod(y, L);
    if (w < 0.0) w += L;
    if (w >= L) w -= L;
    if (!(w < L) || w < 0.0) {   // unreachable for finite y and L > 0
        *bad = 1;
        w = 0.0;
    }
    return w;
}

// first support point (unwrapped) of a coordinate w in [0, L): floor(w/dx - M_G/2) + 1
__device__ inline int support_start(double w, double dx, int MG) {
    return (int)floor(w / dx - 0.5 * MG) + 1;
}

__device__ inline int wrap_index(int s, int M) {
    if (s < 0) s += M;
    if (s >= M) s -= M;
    return s;
}

__global__ void k_fill(int* __restrict__ p, int n, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_hash(const double* __restrict__ pos, HashArgs h, int* __restrict__ keys,
                       int* __restrict__ ranks, int* __restrict__ counts, int* __restrict__ flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= h.N) return;
    int bad = 0;
    int s[3], c[3];
    double y[3];
    // the three coordinates are loaded before the wrap's branches
#pragma unroll
    for (int a = 0; a < 3; ++a) y[a] = pos[3 * (int64_t)i + a];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double w = wrap_coord(y[a], h.Lv[a], &bad);
        s[a] = wrap_index(support_start(w, h.dx, h.MG), h.Mv[a]);
        int cc = (int)floor(w / h.cw[a]);
        c[a] = cc < 0 ? 0 : (cc >= h.mc[a] ? h.mc[a] - 1 : cc);
    }
    if (bad) atomicOr(flag, 1);
    if (i == 0) {
        flag[1] = 0;   // work-list lengths of the segment sorts
        flag[2] = 0;
    }
    int bin = s[0] / h.TX + h.nbx * (s[1] / h.TY + h.nby * (s[2] / h.TZ));
    int cell = c[0] + h.mc[0] * (c[1] + h.mc[1] * c[2]);
    keys[i] = bin;
    keys[h.N + i] = cell;
    // both counter increments are issued before either rank is stored, so
    // their round trips overlap
    const int rb = atomicAdd(&counts[bin], 1);
    const int rc = h.ident ? i : atomicAdd(&counts[h.nbins + cell], 1);
    if (h.ident && i == 0) counts[h.nbins] = h.N;
    ranks[i] = rb;
    ranks[h.N + i] = rc;
}

// block-wide inclusive scan of one int per thread (blockDim = NT)
template <int NT>
__device__ inline int block_inclusive_scan(int v, int* sh) {
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    if (lane == 63) sh[wid] = v;
    __syncthreads();
    if (wid == 0) {
        int t = lane < NT / 64 ? sh[lane] : 0;
#pragma unroll
        for (int o = 1; o < NT / 64; o <<= 1) {
            int u = __shfl_up(t, o, 64);
            if (lane >= o) t += u;
        }
        if (lane < NT / 64) sh[lane] = t;
    }
    __syncthreads();
    if (wid > 0) v += sh[wid - 1];
    __syncthreads();
    return v;
}

// Exclusive scans of two count arrays in two launches.  The arrays A (grid
// bins, nA entries) and B (pair cells, nB entries) are cut into tiles of
// kScanTile; block b < tA handles tile b of A, the others tile b - tA of B.
__device__ inline void scan2_tile(int b, int nA, int nB, int tA, int* n, int* base, int* first) {
    if (b < tA) {
        *n = nA;
        *base = b * kScanTile;
        *first = 0;
    } else {
        *n = nB;
        *base = (b - tA) * kScanTile;
        *first = tA;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan2_reduce(const int* __restrict__ counts,
                                                                int nA, int nB, int tA,
                                                                int* __restrict__ sums) {
    __shared__ int sh[kScanThreads / 64];
    int n, base, first;
    scan2_tile(blockIdx.x, nA, nB, tA, &n, &base, &first);
    const int b = (int)blockIdx.x;
    const int* in = b < tA ? counts : counts + nA;
    const int i0 = base + threadIdx.x * kScanPerThread;
    int v = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k)
        if (i0 + k < n) v += in[i0 + k];
    v = block_inclusive_scan<kScanThreads>(v, sh);
    if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = v;
}

// Writes out[0..n] (out[n] = total) for each array and clears the counts it
// read, so the next hash starts from zero.
__global__ __launch_bounds__(kScanThreads) void k_scan2_down(int* __restrict__ counts, int nA,
                                                              int nB, int tA, int tB,
                                                              const int* __restrict__ sums,
                                                              int* __restrict__ outA,
                                                              int* __restrict__ outB) {
    __shared__ int sh[kScanThreads / 64];
    int n, base, first;
    scan2_tile(blockIdx.x, nA, nB, tA, &n, &base, &first);
    const int b = (int)blockIdx.x;
    int* in = b < tA ? counts : counts + nA;
    int* out = b < tA ? outA : outB;
    const int last = b < tA ? tA - 1 : tA + tB - 1;
    // sum of the tiles before this one in its array
    __shared__ int tile_pre;
    int pre = 0;
    for (int t = first + threadIdx.x; t < (int)blockIdx.x; t += kScanThreads) pre += sums[t];
    pre = block_inclusive_scan<kScanThreads>(pre, sh);
    if (threadIdx.x == kScanThreads - 1) tile_pre = pre;
    __syncthreads();
    pre = tile_pre;
    const int i0 = base + threadIdx.x * kScanPerThread;
    int loc[kScanPerThread];
    int v = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        loc[k] = (i0 + k < n) ? in[i0 + k] : 0;
        v += loc[k];
    }
    const int inc = block_inclusive_scan<kScanThreads>(v, sh);
    int run = pre + inc - v;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        if (i0 + k < n) {
            out[i0 + k] = run;
            in[i0 + k] = 0;
        }
        run += loc[k];
    }
    if ((int)blockIdx.x == last && threadIdx.x == kScanThreads - 1) out[n] = run;
}

__global__ void k_scatter(const int* __restrict__ keys, const int* __restrict__ ranks,
                          const int* __restrict__ start_bin, const int* __restrict__ start_cell,
                          int* __restrict__ perm, int N) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    perm[start_bin[keys[i]] + ranks[i]] = i;
    perm[N + start_cell[keys[N + i]] + ranks[N + i]] = i;
}

// Segment s of the sort: grid bins 0..nbins-1 (perm[0..N)), then pair cells
// (perm[N..2N)).  Returns the bounds [b, e) and the arrays of its half.
__device__ inline void segment(int s, const int* starts, int nbins, int N, int* perm, int* inv,
                               int* b, int* e, int** pm, int** iv) {
    const int* start = starts;
    *pm = perm;
    *iv = inv;
    if (s >= nbins) {
        s -= nbins;
        start = starts + nbins + 1;
        *pm = perm + N;
        *iv = inv + N;
    }
    *b = start[s];
    *e = start[s + 1];
}

// n (2 <= n <= W) values of pm[b..b+n) sorted in registers by a bitonic
// network over W entries (the rest padded with INT_MAX), written back with
// the inverse permutation iv[pm[j]] = j
template <int W>
__device__ inline void thread_sort(int* pm, int* iv, int b, int n) {
    int v[W];
#pragma unroll
    for (int i = 0; i < W; ++i) v[i] = i < n ? pm[b + i] : 0x7fffffff;
#pragma unroll
    for (int k = 2; k <= W; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < W; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const int x = v[i], y = v[l];
                    const bool up = (i & k) == 0;
                    v[i] = up ? min(x, y) : max(x, y);
                    v[l] = up ? max(x, y) : min(x, y);
                }
            }
#pragma unroll
    for (int i = 0; i < W; ++i)
        if (i < n) {
            pm[b + i] = v[i];
            iv[v[i]] = b + i;
        }
}

// Append s to a work list with one atomic per wavefront (the lanes with
// `want` set); list entries go to list[idx] (dir > 0) or list[-idx] (dir < 0).
__device__ inline void wave_append(bool want, int s, int* counter, int* list, int dir) {
    const unsigned long long m = __ballot(want);
    if (m == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader, 64);
    if (want) {
        const int idx = base + __popcll(m & ((1ull << lane) - 1ull));
        list[dir > 0 ? idx : -idx] = s;
    }
}

// Order each segment of perm by value and record the inverse permutation
// inv[perm[j]] = j.  A thread orders a segment of up to kThreadSegment members
// in registers.  Longer segments go to two work lists for k_segment_wide:
// up to kWaveSegment members (one wavefront each), and beyond (one workgroup
// each).  The lists live in `lists` (the bin and cell counts, all zero
// between the scan and the next hash): wavefront entries from the front,
// workgroup entries from the back (index cap - 1 - i); their lengths in
// counters[0], counters[1] (cleared by the hash).
__global__ __launch_bounds__(256) void k_segment_order(const int* __restrict__ starts, int nbins,
                                                       int nseg, int N, int* __restrict__ perm,
                                                       int* __restrict__ inv, int* __restrict__ lists,
                                                       int cap, int* __restrict__ counters) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    int n = 0;
    if (s < nseg) {
        int b, e;
        int *pm, *iv;
        segment(s, starts, nbins, N, perm, inv, &b, &e, &pm, &iv);
        n = e - b;
        if (n == 1) {
            iv[pm[b]] = b;
        } else if (n > 1 && n <= 4) {
            thread_sort<4>(pm, iv, b, n);
        } else if (n > 4 && n <= kThreadSegment) {
            thread_sort<kThreadSegment>(pm, iv, b, n);
        }
    }
    wave_append(n > kThreadSegment && n <= kWaveSegment, s, counters, lists, 1);
    wave_append(n > kWaveSegment, s, counters + 1, lists + cap - 1, -1);
}

// The segments k_segment_order listed.  Wavefront items: a bitonic sort of
// one value per lane by lane exchanges.  Workgroup items: up to kLdsSegment
// members by a bitonic sort in LDS, beyond that by rank counting (a member's
// rank is the number of smaller members, counted against a copy of the
// segment staged through LDS; tmp holds the copy, indexed like perm).  Each
// list entry is cleared once read, so the counts are zero again for the next
// hash.
__global__ __launch_bounds__(256) void k_segment_wide(const int* __restrict__ starts, int nbins,
                                                      int N, int* __restrict__ perm,
                                                      int* __restrict__ inv, int* __restrict__ tmp,
                                                      int* __restrict__ lists, int cap,
                                                      const int* __restrict__ counters) {
    __shared__ int sh[kLdsSegment];
    __shared__ int item;
    const int t = threadIdx.x, nt = blockDim.x;
    const int lane = t & 63;
    const int nwave = counters[0], nblock = counters[1];
    const int waves = gridDim.x * (nt / 64);
    for (int it = blockIdx.x * (nt / 64) + (t >> 6); it < nwave; it += waves) {
        const int s = __builtin_amdgcn_readfirstlane(lists[it]);
        if (lane == 0) lists[it] = 0;
        int b, e;
        int *pm, *iv;
        segment(s, starts, nbins, N, perm, inv, &b, &e, &pm, &iv);
        const int n = e - b;
        int v = lane < n ? pm[b + lane] : 0x7fffffff;
#pragma unroll
        for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const int o = __shfl_xor(v, j, 64);
                const bool up = (lane & k) == 0, lower = (lane & j) == 0;
                v = (lower == up) ? min(v, o) : max(v, o);
            }
        if (lane < n) {
            pm[b + lane] = v;
            iv[v] = b + lane;
        }
    }
    for (int it = blockIdx.x; it < nblock; it += gridDim.x) {
        if (t == 0) {
            item = lists[cap - 1 - it];
            lists[cap - 1 - it] = 0;
        }
        __syncthreads();
        int b, e;
        int *pm, *iv;
        segment(item, starts, nbins, N, perm, inv, &b, &e, &pm, &iv);
        const int n = e - b;
        if (n <= kLdsSegment) {
            int p2 = 1;
            while (p2 < n) p2 <<= 1;
            for (int i = t; i < p2; i += nt) sh[i] = i < n ? pm[b + i] : 0x7fffffff;
            __syncthreads();
            for (int k = 2; k <= p2; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int i = t; i < p2; i += nt) {
                        const int l = i ^ j;
                        if (l > i) {
                            const int x = sh[i], y = sh[l];
                            const bool up = (i & k) == 0;
                            if ((x > y) == up) {
                                sh[i] = y;
                                sh[l] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (int i = t; i < n; i += nt) {
                const int v = sh[i];
                pm[b + i] = v;
                iv[v] = b + i;
            }
        } else {
            int* tp = tmp + (pm - perm);
            for (int i = t; i < n; i += nt) tp[b + i] = pm[b + i];
            __syncthreads();
            for (int r0 = 0; r0 < n; r0 += nt) {
                const int i = r0 + t;
                const int v = i < n ? tp[b + i] : 0x7fffffff;
                int rank = 0;
                for (int c0 = 0; c0 < n; c0 += kLdsSegment) {
                    const int cn = min(kLdsSegment, n - c0);
                    __syncthreads();
                    for (int k = t; k < cn; k += nt) sh[k] = tp[b + c0 + k];
                    __syncthreads();
                    for (int k = 0; k < cn; ++k) rank += sh[k] < v;
                }
                if (i < n) {
                    pm[b + rank] = v;
                    iv[v] = b + rank;
                }
            }
        }
        __syncthreads();
    }
}

// Per-particle records in sorted order, built in the caller's order: thread i
// reads particle i (coalesced) and writes its grid record to grec[inv[i]] and
// its pair record to prec[inv[N + i]] (either may be skipped: null).  F may be
// null (interpolation alone needs only positions).
template <typename R>
__global__ void k_place(const double* __restrict__ pos, const double* __restrict__ F,
                        const double* __restrict__ T, const int* __restrict__ inv,
                        const int* __restrict__ cellkey, int N, int3 Mv, int MG, double3 Lv,
                        double dx, double normF, double normT, GridRec<R>* __restrict__ grec,
                        PairRec* __restrict__ prec, double4* __restrict__ pos4) {
    const int Ma[3] = {Mv.x, Mv.y, Mv.z};
    const double La[3] = {Lv.x, Lv.y, Lv.z};
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int bad = 0;
    double w[3], f[3], t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        w[a] = wrap_coord(pos[3 * (int64_t)i + a], La[a], &bad);
        f[a] = F ? F[3 * (int64_t)i + a] : 0.0;
        t[a] = T ? T[3 * (int64_t)i + a] : 0.0;
    }
    if (grec) {
        GridRec<R> r;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int su = support_start(w[a], dx, MG);
            r.s[a] = wrap_index(su, Ma[a]);
            r.f[a] = (R)(w[a] / dx - (double)su);
            r.F[a] = (R)(f[a] * normF);
            r.T[a] = (R)(t[a] * normT);
        }
        r.orig = i;
        grec[inv[i]] = r;
    }
    if (prec) {
        PairRec r;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r.y[a] = w[a];
            r.F[a] = f[a];
            r.T[a] = t[a];
        }
        r.orig = i;
        r.cell = cellkey[i];
        const int j = inv[N + i];
        prec[j] = r;
        pos4[j] = make_double4(w[0], w[1], w[2], 0.0);
    }
}

inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

hipError_t launch_fill(int* p, int n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_hash(const fcm_plan_impl* P, const double* pos, hipStream_t st) {
    HashArgs h;
    h.N = (int)P->N;
    h.Mv[0] = P->M;
    h.Mv[1] = P->My;
    h.Mv[2] = P->Mz;
    h.MG = P->MG;
    h.TX = P->TX;
    h.TY = P->TY;
    h.TZ = P->TZ;
    h.nbx = P->nbx;
    h.nby = P->nby;
    h.nbz = P->nbz;
    h.nbins = P->nbins;
    h.mc[0] = P->m;
    h.mc[1] = P->mcy;
    h.mc[2] = P->mcz;
    h.ident = P->rc > 0.0 ? 0 : 1;
    h.Lv[0] = P->L;
    h.Lv[1] = P->Ly;
    h.Lv[2] = P->Lz;
    h.dx = P->dx;
    for (int d = 0; d < 3; ++d) h.cw[d] = h.Lv[d] / h.mc[d];
    hipLaunchKernelGGL(k_hash, dim3(blocks_for(h.N, 256)), dim3(256), 0, st, pos, h, P->keys,
                       P->ranks, P->counts, P->flag);
    return hipGetLastError();
}

hipError_t launch_scan(const fcm_plan_impl* P, hipStream_t st) {
    const int nA = P->nbins, nB = P->ncells;
    const int tA = blocks_for(nA, kScanTile), tB = blocks_for(nB, kScanTile);
    if (tA + tB > kMaxScanTiles) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan2_reduce, dim3(tA + tB), dim3(kScanThreads), 0, st, P->counts, nA, nB,
                       tA, P->scan_tmp);
    hipLaunchKernelGGL(k_scan2_down, dim3(tA + tB), dim3(kScanThreads), 0, st, P->counts, nA, nB,
                       tA, tB, P->scan_tmp, P->starts, P->starts + nA + 1);
    return hipGetLastError();
}

hipError_t launch_scatter(const fcm_plan_impl* P, hipStream_t st) {
    int N = (int)P->N;
    const int* sb = P->starts;
    const int* sc = P->starts + P->nbins + 1;
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(N, 256)), dim3(256), 0, st, P->keys, P->ranks, sb,
                       sc, P->perm, N);
    // The ranks are dead after the scatter: their buffer takes the inverse
    // permutation.  Without a pair search the pair order is the identity, which
    // the hash already wrote there.  pair_hits is free until the pair pass
    // (which runs after the records are built): it holds the copies of the
    // longest segments.
    const int nseg = P->nbins + (P->rc > 0.0 ? P->ncells : 0);
    const int cap = P->nbins + P->cells_cap;   // entries of the counts array (>= nseg)
    hipLaunchKernelGGL(k_segment_order, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, P->starts,
                       P->nbins, nseg, N, P->perm, P->ranks, P->counts, cap, P->flag + 1);
    const int wide = std::min(2048, std::max(1, nseg / 64));
    hipLaunchKernelGGL(k_segment_wide, dim3(wide), dim3(256), 0, st, P->starts, P->nbins, N,
                       P->perm, P->ranks, P->pair_hits, P->counts, cap, P->flag + 1);
    return hipGetLastError();
}

namespace {

// records of the particles in sorted order: grid (`grid`) and/or pair (`pair`)
hipError_t place(const fcm_plan_impl* P, const double* pos, const double* F, const double* T,
                 bool grid, bool pair, hipStream_t st) {
    const int N = (int)P->N;
    const double pi = 3.14159265358979323846;
    const double normF = pow(2.0 * pi * P->Sigma * P->Sigma, -1.5);
    const double normT =
        pow(2.0 * pi * P->SigmaD * P->SigmaD, -1.5) / (2.0 * P->SigmaD * P->SigmaD);
    const dim3 g(blocks_for(N, 256)), b(256);
    PairRec* pr = pair ? P->prec : nullptr;
    const int3 Mv = make_int3(P->M, P->My, P->Mz);
    const double3 Lv = make_double3(P->L, P->Ly, P->Lz);
    if (P->precision == FCM_FP64)
        hipLaunchKernelGGL(k_place<double>, g, b, 0, st, pos, F, T, P->ranks, P->keys + N, N, Mv,
                           P->MG, Lv, P->dx, normF, normT,
                           grid ? (GridRec<double>*)P->grec : nullptr, pr, P->ppos);
    else
        hipLaunchKernelGGL(k_place<float>, g, b, 0, st, pos, F, T, P->ranks, P->keys + N, N, Mv,
                           P->MG, Lv, P->dx, normF, normT,
                           grid ? (GridRec<float>*)P->grec : nullptr, pr, P->ppos);
    return hipGetLastError();
}

// New forces and torques for the records of the last sort: thread i reads
// particle i (coalesced) and rewrites the force and torque fields of its grid
// record (and pair record) in place; positions, supports and cells stay.
template <typename R>
__global__ void k_refresh(const double* __restrict__ F, const double* __restrict__ T,
                          const int* __restrict__ inv, int N, double normF, double normT,
                          GridRec<R>* __restrict__ grec, PairRec* __restrict__ prec) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double f[3], t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f[a] = F[3 * (int64_t)i + a];
        t[a] = T ? T[3 * (int64_t)i + a] : 0.0;
    }
    GridRec<R>& g = grec[inv[i]];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g.F[a] = (R)(f[a] * normF);
        g.T[a] = (R)(t[a] * normT);
    }
    if (prec) {
        PairRec& r = prec[inv[N + i]];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r.F[a] = f[a];
            r.T[a] = t[a];
        }
    }
}

}  // namespace

hipError_t launch_gather_grid(const fcm_plan_impl* P, const double* pos, const double* F,
                              const double* T, hipStream_t st) {
    return place(P, pos, F, T, true, false, st);
}

hipError_t launch_gather_pair(const fcm_plan_impl* P, const double* pos, const double* F,
                              const double* T, hipStream_t st) {
    return place(P, pos, F, T, false, true, st);
}

hipError_t launch_gather_both(const fcm_plan_impl* P, const double* pos, const double* F,
                              const double* T, hipStream_t st) {
    return place(P, pos, F, T, true, true, st);
}

hipError_t launch_refresh_forces(const fcm_plan_impl* P, const double* F, const double* T,
                                 bool pair, hipStream_t st) {
    const int N = (int)P->N;
    const double pi = 3.14159265358979323846;
    const double normF = pow(2.0 * pi * P->Sigma * P->Sigma, -1.5);
    const double normT =
        pow(2.0 * pi * P->SigmaD * P->SigmaD, -1.5) / (2.0 * P->SigmaD * P->SigmaD);
    const dim3 g(blocks_for(N, 256)), b(256);
    PairRec* pr = pair ? P->prec : nullptr;
    if (P->precision == FCM_FP64)
        hipLaunchKernelGGL(k_refresh<double>, g, b, 0, st, F, T, P->ranks, N, normF, normT,
                           (GridRec<double>*)P->grec, pr);
    else
        hipLaunchKernelGGL(k_refresh<float>, g, b, 0, st, F, T, P->ranks, N, normF, normT,
                           (GridRec<float>*)P->grec, pr);
    return hipGetLastError();
}

}  // namespace fcm
