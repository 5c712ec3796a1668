// Device-side types and helpers of the DUWP pipeline (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace duwp {

constexpr int KWIN = 16;             // a particle may move at most KWIN cells per step
constexpr int NBIN = 2 * KWIN + 1;   // destination bins per source cell
constexpr int WAVE = 64;
constexpr int BIG_N = 4096;          // a cell with at least this many particles ...
constexpr int BIG_M = 4096;          // ... and candidates collides in the block kernel

// Philox counter tags: one per kind of random draw.
enum : uint32_t { TAG_CLS = 1, TAG_RCNT = 2, TAG_RVEL = 3, TAG_NCNT = 4, TAG_PAIR = 5,
                  TAG_ICNT = 6, TAG_IVEL = 7 };

// Device error word bits.
enum : int32_t { ERR_CAPACITY = 1, ERR_RANGE = 2, ERR_STATE = 4 };

// Per-case constants, derived on the host once.
struct DCase {
    int32_t ncells, cell_base;
    int32_t bc_lo, bc_hi, law, eps_law, full_dt, flux2;   // flux2: MUSCL inviscid face states
    int32_t abs_stream;                                   // absorbed particles stream for t_f first
    uint32_t key0, key1;
    int64_t inj_base, inj_cap;       // slot range of this case's entrants in the injection buffer
    int64_t cand_base[2], cand_cap[2];  // injection candidate slots per side
    int64_t chunk_base[2];              // per-side entrant counts of INJ_CH-slot candidate chunks
    double x_lo, x_hi, dx, dt;
    double R, omega, T_ref, mu_ref, coll_k, ups, c_ref;
    double m_p, fac;                 // fac = m_p / dx
    double rho_L, u_L, T_L, rho_R, u_R, T_R;
    float dtdx_f, pad1;              // dt/dx for the cell-relative FP32 positions
};

// The constants a per-cell loop reads for every particle (free flight, random
// draws, sampling), held in registers: a reference into global memory is read
// again after each fence inside the loop.
struct CaseK {
    const DCase *pc;                 // the whole case, for the rare paths
    double x_lo, x_hi, dx, dt, R;
    float dtdx_f;
    int ncells;
    uint32_t key0, key1;
    __device__ explicit CaseK(const DCase &c)
        : pc(&c), x_lo(c.x_lo), x_hi(c.x_hi), dx(c.dx), dt(c.dt), R(c.R), dtdx_f(c.dtdx_f), ncells(c.ncells),
          key0(c.key0), key1(c.key1)
    {
    }
};
// The fields the free flight of one precision reads on its fast path, held in
// registers per lane by a kernel whose lanes may work on different cases.
template <typename T>
struct FlightK;
template <>
struct FlightK<float> {
    const DCase *pc;
    float dtdx_f;
    int ncells;
    __device__ FlightK() : pc(nullptr), dtdx_f(0.0f), ncells(0) {}
    __device__ explicit FlightK(const DCase &c) : pc(&c), dtdx_f(c.dtdx_f), ncells(c.ncells) {}
};
template <>
struct FlightK<double> {
    const DCase *pc;
    double x_lo, x_hi, dx, dt;
    int ncells;
    __device__ FlightK() : pc(nullptr), x_lo(0.0), x_hi(0.0), dx(1.0), dt(0.0), ncells(0) {}
    __device__ explicit FlightK(const DCase &c)
        : pc(&c), x_lo(c.x_lo), x_hi(c.x_hi), dx(c.dx), dt(c.dt), ncells(c.ncells)
    {
    }
};
__device__ __forceinline__ const DCase &case_of(const DCase &c) { return c; }
__device__ __forceinline__ const DCase &case_of(const CaseK &k) { return *k.pc; }
template <typename T>
__device__ __forceinline__ const DCase &case_of(const FlightK<T> &k) { return *k.pc; }

// Per-step, per-cell work arrays shared by the stage kernels.
struct Cells {
    double *psi_w;      // [G*5] wave part
    double *psi_p;      // [G*5] particle part of the canonical array
    double *wt;         // [G*5] (rho, U, V, W, T) of the total at step start
    double *pc;         // [G] absorbed fraction P
    double *tau;        // [G] mean collision time mu/p of the total state at step start
    int32_t *okc;       // [G] 1 unless vacuum
    double *cr_max;     // [G]
    int32_t *n_surv, *n_new, *n_int;   // [G] survivors, resampled, survivors+resampled
    int64_t *nstage;    // [1] staging records handed out this step (cleared at the end of each step)
    int64_t *seg;       // [G] start of the cell's intermediate segment
    int32_t *seg_stg;   // [G] 1: segment in the staging buffer, 0: in place in the canonical buffer
    int32_t *d_abs, *d_new, *d_cand, *d_coll;  // [G] diagnostics; d_cand is also the collide work size
    int32_t *ncand_w;   // [G] candidates in the wave kernel's list (0 for cells of the block kernel)
    int64_t *cbase;     // [G+1] first collision candidate of each cell in the step's candidate list
    int32_t *big_list;  // [G] cells that collide in the block kernel (unordered)
    int32_t *nbig;      // [1] their number (cleared at the end of each step)
    int32_t *touch_list;  // [G] cells that absorb or resample this step (any order)
    int32_t *ntouch;      // [1] their number (cleared at the end of each step)
    uint64_t *cr_seen;  // [G] largest relative speed seen this step (bits of a non-negative double)
    int32_t *hist;      // [G*NBIN] destination histogram of this step, then scatter bases
    int32_t *hist_nx;   // [G*NBIN] histogram predicted for the next step
    int32_t *cnt_new;   // [G]
    int32_t *inj_cnt;   // [G] injected entrants per destination cell
    int32_t *inj_ofs;   // [G] cell-sourced particles of each destination cell: where its entrants
                        // start, relative to the cell's start in the next array
    int32_t *cell_case; // [G]
    int32_t *order;     // [G] cells in the visiting order of the block-per-cell kernels
    double *avg;        // [G*5]
    double *mnear;      // [G*15] particle moment sums of a source cell per destination g-1, g, g+1
    double *mpart;      // [G*NBIN*5] sums from farther sources, by destination (zero unless far_in)
    int32_t *far_in;    // [G] 1: a farther source left sums in the cell's mpart row this step
    double *wabs;       // [G*NBIN*5] absorbed moments that streamed in from other cells, by
                        // source (absorb_stream cases only; zero unless wabs_in)
    int32_t *wabs_in;   // [G] 1: another cell's absorbed particles reached this one this step
};

// Injection buffers: candidates of every (case, side), then the entrants of
// every case in (side, slot) order with their destination and rank.
template <typename T>
struct Inj {
    T *x, *u, *v, *w;
    int32_t *dest;      // global destination cell of an entrant
    int32_t *rank;      // rank among injected entrants of the same destination
    int32_t *count;     // [ncases] entrants written this step
    T *cx, *cu, *cv, *cw;
    int32_t *cdest;     // local destination of a candidate, -1 if it does not enter
    int64_t *ncand;     // [ncases*2] candidates generated per side
    int32_t *cchunk;    // entrants per INJ_CH-slot candidate chunk (entrants compacted to the chunk front)
};

// Injection candidate slots per chunk: one wave's worth, so that any wave of
// any launch can generate and compact a chunk by itself.
constexpr int INJ_CH = WAVE;

// One particle: position and velocity in one record (16 B with FP32 particles,
// 32 B with FP64), so that a particle is one vector access and one cache line.
// With FP32 particles x is the position inside the cell, in cells.
template <typename T>
struct alignas(4 * sizeof(T) > 16 ? 16 : 4 * sizeof(T)) P4 {
    T x, u, v, w;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
struct U4 { uint32_t a, b, c, d; };

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        // one 32x32 -> 64-bit product per multiplier (its high and low words)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    return U4{c0, c1, c2, c3};
}

template <typename K>
__device__ __forceinline__ U4 draw(const K &cs, uint32_t step, uint32_t a, uint32_t b, uint32_t tag, uint32_t j)
{
    return philox(step, a, b, (tag << 16) | j, cs.key0, cs.key1);
}

// [0,1) with 2^-32 resolution (exact in FP64)
__device__ __forceinline__ double u01(uint32_t r) { return (double)r * 2.3283064365386962890625e-10; }

// uniform index in [0,n): floor(r n / 2^64)
__device__ __forceinline__ uint64_t mulhi64(uint64_t r, uint64_t n) { return __umul64hi(r, n); }

// ---------------------------------------------------------------------------
// Wave / block primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }
// index of this wave in its block, as a wave-uniform value
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }
// number of set bits of m below this lane
__device__ __forceinline__ int lane_rank_lt(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int l)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)(uint64_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    return __longlong_as_double(readlane64(__double_as_longlong(v), l));
}

// Orders this wave's LDS accesses (no barrier): LDS operations of one wave
// complete in issue order, so a later read by any lane sees an earlier write.
__device__ __forceinline__ void lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block barrier that orders LDS only: outstanding global loads (e.g. prefetches)
// stay in flight across it.  Use where no global memory written before the
// barrier is read by another thread after it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Deterministic block sum of N doubles per thread; the result is valid in every thread.
// red must hold N * (blockDim/64) doubles.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double *red)
{
    const int w = wave_id(), nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) red[k * nw + w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += red[k * nw + i];
        v[k] = s;
    }
    __syncthreads();
}

// Wave sums of N <= 16 doubles by recursive halving: at each of the steps 32,
// 16, 8, 4 a lane keeps the half of its values chosen by that bit of its index
// and adds the partner's copy, so the sum of value q ends in lanes 4q..4q+3
// (the last two steps add those four).  Returns the sum of value lane/4 (0 for
// q >= N).  17 exchanges instead of 6 per value.
// One halving step: lanes with bit O set keep the upper H values, the others the
// lower H, and each adds its partner's copy of the half it keeps.  H and O are
// template parameters so that every array index is a constant (an index that
// depends on the lane would turn each access into a chain of selects).
template <int H, int O>
__device__ __forceinline__ void spread_step(double (&a)[16], int lane)
{
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int q = 0; q < H; ++q) {
        const double lo = a[q], hi = a[H + q];
        const double keep = up ? hi : lo;
        const double send = up ? lo : hi;
        a[q] = keep + __shfl_xor(send, O, WAVE);
    }
}

template <int N>
__device__ __forceinline__ double wave_sum_spread(const double (&v)[N])
{
    static_assert(N <= 16, "at most 16 values");
    const int lane = lane_id();
    double a[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) a[q] = q < N ? v[q] : 0.0;
    spread_step<8, 32>(a, lane);
    spread_step<4, 16>(a, lane);
    spread_step<2, 8>(a, lane);
    spread_step<1, 4>(a, lane);
    double e = a[0];
    e += __shfl_xor(e, 2, WAVE);
    e += __shfl_xor(e, 1, WAVE);
    return e;
}

// Block sum of value q of N <= 16 doubles per thread, returned in thread q
// (q < N; other threads get 0).  red must hold N * (blockDim/64) doubles.
// Deterministic: a fixed tree inside each wave, then the waves in order.
template <int N>
__device__ __forceinline__ double block_sum_to_thread(const double (&v)[N], double *red)
{
    const int lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
    const double e = wave_sum_spread<N>(v);
    if (nw == 1) {
        const double r = __shfl(e, (lane & 15) * 4, WAVE);
        return lane < N ? r : 0.0;
    }
    __syncthreads();
    if ((lane & 3) == 0 && (lane >> 2) < N) red[(lane >> 2) * nw + w] = e;
    __syncthreads();
    double s = 0.0;
    if ((int)threadIdx.x < N)
        for (int i = 0; i < nw; ++i) s += red[threadIdx.x * nw + i];
    __syncthreads();
    return s;
}

// Exclusive block prefix of a 0/1 flag; returns this thread's prefix, *total the block total.
// scratch must hold blockDim/64 ints.
__device__ __forceinline__ int block_flag_prefix(bool f, int *scratch, int *total)
{
    const int w = wave_id(), nw = blockDim.x >> 6;
    uint64_t m = __ballot(f);
    int in_wave = __popcll(m & lanemask_lt());
    __syncthreads();
    if (lane_id() == 0) scratch[w] = __popcll(m);
    __syncthreads();
    int base = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        int c = scratch[i];
        if (i < w) base += c;
        tot += c;
    }
    *total = tot;
    return base + in_wave;
}

// Exclusive block prefix of a small per-thread count; returns this thread's
// prefix, *total the block total.  scratch must hold blockDim/64 ints.
__device__ __forceinline__ int block_count_prefix(int v, int *scratch, int *total)
{
    const int w = wave_id(), nw = blockDim.x >> 6, lane = lane_id();
    int incl = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const int t = __shfl_up(incl, o, WAVE);
        if (lane >= o) incl += t;
    }
    __syncthreads();
    if (lane == WAVE - 1) scratch[w] = incl;
    __syncthreads();
    int base = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        const int c = scratch[i];
        if (i < w) base += c;
        tot += c;
    }
    *total = tot;
    return base + incl - v;
}

}  // namespace duwp
