// Stage kernels of one DUWP time step (gfx950, wave64) and the step sequence.
//
// Data layout: cells of all cases are numbered case by case (global cell g);
// particles are structure-of-arrays sorted by global cell, so every case's
// particles are contiguous.  Two canonical buffers alternate with the step
// parity; a staging buffer holds the intermediate array of a step (per cell:
// survivors in order, then resampled particles by slot).  Cell arrays are FP64.
// Particle storage is FP64 with absolute positions, or FP32 with the position
// stored relative to the particle's cell (in cells, [0,1)).
//
// Per step (Sec. 3.4):
//   cellstate      Psi_t = Psi_w + Psi_p, (rho,U,T), tau = mu/p, P (Eq. p),
//                  absorbed count, resample count
//   scan           staging offsets
//   absorb_resample  classify, absorb into Psi_w, compact survivors,
//                  sample new particles (Eq. maxsample), subtract their moments
//   collide        NTC/VHS (Appendix A), one wave per cell, candidates in
//                  order with conflict-free rounds
//   inject         reservoir entrants, one wave per case
//   stream_hist    free flight + boundaries, histogram of destination cells
//   count/scan/bases  windowed stable counting-sort offsets
//   scatter        free flight again, stable scatter into the next canonical array
//   scatter_inj    entrants after the cell-sourced particles of their cell
//   wave           NS wave flux and update of Psi_w (Eq. r1)
//   moments        Psi_p of the new state, running average of Psi_t
#include <hip/hip_runtime.h>
#include <math.h>
#include <type_traits>

#include "duwp_ctx.hpp"
#include "duwp_device.hpp"

namespace duwp {

#define D_TWO_PI 6.283185307179586

// ---------------------------------------------------------------------------
// Gas physics
// ---------------------------------------------------------------------------
__device__ __forceinline__ double viscosity(const DCase &c, double T)
{
    return c.mu_ref * pow(T / c.T_ref, c.omega);
}

// Eq. p (law 0) or the QMC probability 1 - exp(-dt/tau) (law 1)
__device__ __forceinline__ double absorb_fraction(int law, double dt, double tau)
{
    if (law == 1) return -expm1(-dt / tau);
    return (dt > tau) ? 1.0 - tau / dt : 0.0;
}

// (rho,U,V,W,T) of a conserved vector; 0 for vacuum (rho <= 0, T <= 0 or not finite)
__device__ __forceinline__ int primitive(const double t[5], double R, double W[5])
{
    double rho = t[0];
    if (!(rho > 0.0)) { W[0] = rho; W[1] = W[2] = W[3] = W[4] = 0.0; return 0; }
    double U = t[1] / rho, V = t[2] / rho, Wv = t[3] / rho;
    double e = t[4] / rho;
    double T = (2.0 / (3.0 * R)) * (e - 0.5 * (U * U + V * V + Wv * Wv));
    W[0] = rho; W[1] = U; W[2] = V; W[3] = Wv; W[4] = T;
    return (T > 0.0) && isfinite(T);
}

__device__ __forceinline__ uint32_t pick(const U4 &r, uint32_t i)
{
    return i == 0 ? r.a : (i == 1 ? r.b : (i == 2 ? r.c : r.d));
}

// Maxwellian velocity, one (cos, log) pair of uniforms per component (Eq. maxsample)
__device__ __forceinline__ void maxwell(double U, double V, double W, double T, double R,
                                        const double uu[6], double out[3])
{
    double sd = sqrt(2.0 * R * T);
    double mean[3] = {U, V, W};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        out[d] = mean[d] + sd * cos(D_TWO_PI * uu[2 * d]) * sqrt(-log(1.0 - uu[2 * d + 1]));
}

// ---------------------------------------------------------------------------
// Free flight and boundaries.  Returns the local destination cell, -1 if the
// particle left through a reservoir side.
// ---------------------------------------------------------------------------

// FP64, absolute position.
__device__ __forceinline__ int bc_cell_abs(const DCase &c, double &x, double &u)
{
    for (int it = 0; it < 1000; ++it) {
        if (x < c.x_lo) {
            if (c.bc_lo == 0) return -1;
            x = 2.0 * c.x_lo - x;
            u = -u;
        } else if (x > c.x_hi) {
            if (c.bc_hi == 0) return -1;
            x = 2.0 * c.x_hi - x;
            u = -u;
        } else {
            double f = floor((x - c.x_lo) / c.dx);
            int64_t ci = (int64_t)f;
            if (f < 0.0) ci = 0;
            if (ci > c.ncells - 1) ci = c.ncells - 1;
            return (int)ci;
        }
    }
    return -1;
}

// FP32, position as (integer cell I, fraction f in [0,1)) relative to x_lo.
__device__ __forceinline__ int bc_cell_rel(const DCase &c, int I, float f, float &u, float &s)
{
    const int C = c.ncells;
    for (int it = 0; it < 1000; ++it) {
        if (I < 0) {
            if (c.bc_lo == 0) return -1;
            I = -I - 1;
            f = 1.0f - f;
            u = -u;
        } else if (I >= C) {
            if (c.bc_hi == 0) return -1;
            I = 2 * C - I - 1;
            f = 1.0f - f;
            u = -u;
        } else {
            if (f >= 1.0f) { f -= 1.0f; I += 1; continue; }
            s = f;
            return I;
        }
    }
    return -1;
}

template <typename T>
struct Flight;

template <>
struct Flight<double> {
    // stream a particle of local cell lc; x is absolute
    __device__ static int go(const DCase &c, int /*lc*/, double &x, double &u)
    {
        x = x + u * c.dt;
        return bc_cell_abs(c, x, u);
    }
};

template <>
struct Flight<float> {
    // stream a particle of local cell lc; x is the position inside the cell, in cells
    __device__ static int go(const DCase &c, int lc, float &s, float &u)
    {
        float X = s + u * c.dtdx_f;
        if (!(fabsf(X) < 1.0e9f)) return -1;
        float fl = floorf(X);
        return bc_cell_rel(c, lc + (int)fl, X - fl, u, s);
    }
};

// ---------------------------------------------------------------------------
// 1. Cell state at step start, absorbed and resampled counts
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024) k_cellstate(const DCase *__restrict__ cases, Cells cl,
                                                    const int64_t *__restrict__ off,
                                                    const uint32_t *__restrict__ d_step, int G,
                                                    int32_t *err, int64_t *d_nout, int64_t *d_ninj)
{
    __shared__ double red[16];
    const uint32_t step = *d_step;
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const int k = cl.cell_case[g];
        const DCase &c = cases[k];
        const int lc = g - c.cell_base;
        double t[5], W[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) t[i] = cl.psi_w[g * 5 + i] + cl.psi_p[g * 5 + i];
        const int ok = primitive(t, c.R, W);
        double P = 0.0;
        if (ok) {
            double tau = viscosity(c, W[4]) / (W[0] * c.R * W[4]);
            P = absorb_fraction(c.law, c.dt, tau);
        }
        const int64_t b = off[g], e = off[g + 1];
        const int64_t pbase = off[c.cell_base];
        double nabs[1] = {0.0};
        if (P > 0.0) {
            for (int64_t kk = b + threadIdx.x; kk < e; kk += blockDim.x) {
                uint32_t kl = (uint32_t)(kk - pbase);
                U4 r = draw(c, step, kl >> 2, 0, TAG_CLS, 0);
                nabs[0] += (u01(pick(r, kl & 3)) < P) ? 1.0 : 0.0;
            }
            block_sum<1>(nabs, red);
        }
        int32_t nnew = 0;
        if (ok) {
            double Mw = c.dx * cl.psi_w[g * 5 + 0];
            U4 r = draw(c, step, (uint32_t)lc, 0, TAG_RCNT, 0);
            double nf = floor((1.0 - P) * Mw / c.m_p + u01(r.a));
            double cap = floor((Mw > 0.0 ? Mw : 0.0) / c.m_p);
            if (nf > cap) nf = cap;
            if (nf < 0.0) nf = 0.0;
            if (nf > 2.0e9) { if (threadIdx.x == 0) atomicOr(err, ERR_CAPACITY); nf = 0.0; }
            nnew = (int32_t)nf;
        }
        if (threadIdx.x == 0) {
#pragma unroll
            for (int i = 0; i < 5; ++i) cl.wt[g * 5 + i] = W[i];
            cl.pc[g] = P;
            cl.okc[g] = ok;
            int32_t ns = (int32_t)(e - b) - (int32_t)nabs[0];
            cl.n_surv[g] = ns;
            cl.n_new[g] = nnew;
            cl.n_int[g] = ns + nnew;
            cl.inj_cnt[g] = 0;
            if (lc == 0) {
                d_nout[k] = 0;
                d_ninj[2 * k] = 0;
                d_ninj[2 * k + 1] = 0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of int32 counts into int64 offsets [G+1] (reduce, scan, scan)
// ---------------------------------------------------------------------------
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_TILE = SCAN_ITEMS * SCAN_BLOCK;

__device__ __forceinline__ int64_t block_exclusive_scan64(int64_t v, int64_t *lds, int64_t *total)
{
    const int lane = lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int64_t incl = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int64_t n = __shfl_up(incl, o, WAVE);
        if (lane >= o) incl += n;
    }
    __syncthreads();
    if (lane == WAVE - 1) lds[w] = incl;
    __syncthreads();
    int64_t base = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) base += lds[i];
        tot += lds[i];
    }
    *total = tot;
    return base + incl - v;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const int32_t *__restrict__ in, int G,
                                                            int64_t *__restrict__ part)
{
    __shared__ double red[8];
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    double s[1] = {0.0};
    int64_t si = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (t0 + i < G) si += in[t0 + i];
    s[0] = (double)si;   // exact: counts stay far below 2^53
    block_sum<1>(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = (int64_t)s[0];
}

__global__ void __launch_bounds__(1024) k_scan_partials(int64_t *part, int n)
{
    __shared__ int64_t lds[16];
    int64_t carry = 0;
    for (int i0 = 0; i0 < n; i0 += blockDim.x) {
        int i = i0 + threadIdx.x;
        int64_t v = i < n ? part[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan64(v, lds, &tot);
        if (i < n) part[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_apply(const int32_t *__restrict__ in, int G,
                                                           const int64_t *__restrict__ part,
                                                           int64_t *__restrict__ out, int64_t cap,
                                                           int64_t *total, int32_t *err)
{
    __shared__ int64_t lds[8];
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (t0 + i < G) ? in[t0 + i] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t run = part[blockIdx.x] + block_exclusive_scan64(s, lds, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        // offsets are clamped to the capacity so that later kernels stay in bounds
        if (t0 + i < G) out[t0 + i] = run < cap ? run : cap;
        run += v[i];
        if (t0 + i == G - 1) {
            out[G] = run < cap ? run : cap;
            *total = run;
            if (run > cap) atomicOr(err, ERR_CAPACITY);
        }
    }
}

static void enqueue_scan(duwp_ctx *ctx, const int32_t *in, int64_t *out, int64_t *total)
{
    const int G = ctx->G;
    hipLaunchKernelGGL(k_scan_reduce, dim3(ctx->ntiles), dim3(SCAN_BLOCK), 0, ctx->stream, in, G,
                       ctx->scan_part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, ctx->stream, ctx->scan_part,
                       ctx->ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3(ctx->ntiles), dim3(SCAN_BLOCK), 0, ctx->stream, in, G,
                       ctx->scan_part, out, ctx->cap, total, ctx->d_err);
}

// ---------------------------------------------------------------------------
// 3. Classify + absorb + compact survivors + resample (Step 2)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024) k_absorb_resample(const DCase *__restrict__ cases, Cells cl,
                                                          Soa<T> src, const int64_t *__restrict__ off,
                                                          Soa<T> stg, const int64_t *__restrict__ ibase,
                                                          const uint32_t *__restrict__ d_step, int G,
                                                          int64_t cap, int32_t *err)
{
    __shared__ double red[5 * 16];
    __shared__ int scr[16];
    const uint32_t step = *d_step;
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const int k = cl.cell_case[g];
        const DCase &c = cases[k];
        const int lc = g - c.cell_base;
        const double P = cl.pc[g];
        const int64_t b = off[g], e = off[g + 1];
        const int64_t pbase = off[c.cell_base];
        const int64_t ob = ibase[g];
        const int32_t nsurv = cl.n_surv[g];
        double sa[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        int64_t written = 0;
        if (P > 0.0) {
            for (int64_t k0 = b; k0 < e; k0 += blockDim.x) {
                const int64_t kk = k0 + threadIdx.x;
                const bool valid = kk < e;
                T x = 0, u = 0, v = 0, w = 0;
                bool absorbed = false;
                if (valid) {
                    x = src.x[kk]; u = src.u[kk]; v = src.v[kk]; w = src.w[kk];
                    uint32_t kl = (uint32_t)(kk - pbase);
                    U4 r = draw(c, step, kl >> 2, 0, TAG_CLS, 0);
                    absorbed = u01(pick(r, kl & 3)) < P;
                }
                if (absorbed) {
                    double du = u, dv = v, dw = w;
                    sa[0] += 1.0; sa[1] += du; sa[2] += dv; sa[3] += dw;
                    sa[4] += 0.5 * (du * du + dv * dv + dw * dw);
                }
                int tot;
                const bool keep = valid && !absorbed;
                int pre = block_flag_prefix(keep, scr, &tot);
                if (keep) {
                    int64_t d = ob + written + pre;
                    if (d < cap) { stg.x[d] = x; stg.u[d] = u; stg.v[d] = v; stg.w[d] = w; }
                    else atomicOr(err, ERR_CAPACITY);
                }
                written += tot;
            }
            block_sum<5>(sa, red);
        } else {
            // nothing is absorbed: a straight copy of the segment
            for (int64_t kk = b + threadIdx.x; kk < e; kk += blockDim.x) {
                int64_t d = ob + (kk - b);
                if (d < cap) { stg.x[d] = src.x[kk]; stg.u[d] = src.u[kk]; stg.v[d] = src.v[kk]; stg.w[d] = src.w[kk]; }
                else atomicOr(err, ERR_CAPACITY);
            }
        }
        // resample 1-P of the start-of-step wave mass at the total state
        const int32_t nnew = cl.n_new[g];
        double ss[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (nnew > 0) {
            const double *Wc = cl.wt + g * 5;
            for (int q = threadIdx.x; q < nnew; q += blockDim.x) {
                U4 a = draw(c, step, (uint32_t)lc, (uint32_t)q, TAG_RVEL, 0);
                U4 bb = draw(c, step, (uint32_t)lc, (uint32_t)q, TAG_RVEL, 1);
                double uu[6] = {u01(a.b), u01(a.c), u01(a.d), u01(bb.a), u01(bb.b), u01(bb.c)};
                double xi[3];
                maxwell(Wc[1], Wc[2], Wc[3], Wc[4], c.R, uu, xi);
                T px;
                if constexpr (std::is_same<T, double>::value) {
                    px = c.x_lo + ((double)lc + u01(a.a)) * c.dx;
                } else {
                    px = (float)u01(a.a);
                    if (px >= 1.0f) px = 0.99999994f;
                }
                T pu = (T)xi[0], pv = (T)xi[1], pw = (T)xi[2];
                int64_t d = ob + nsurv + q;
                if (d < cap) { stg.x[d] = px; stg.u[d] = pu; stg.v[d] = pv; stg.w[d] = pw; }
                else atomicOr(err, ERR_CAPACITY);
                // moments of the particle as stored, so Psi_t is unchanged exactly
                double du = pu, dv = pv, dw = pw;
                ss[0] += 1.0; ss[1] += du; ss[2] += dv; ss[3] += dw;
                ss[4] += 0.5 * (du * du + dv * dv + dw * dw);
            }
            block_sum<5>(ss, red);
        }
        if (threadIdx.x == 0) {
            const int32_t nabs = (int32_t)(e - b) - nsurv;
            if (nabs > 0)
#pragma unroll
                for (int i = 0; i < 5; ++i) cl.psi_w[g * 5 + i] += c.fac * sa[i];
            if (nnew > 0)
#pragma unroll
                for (int i = 0; i < 5; ++i) cl.psi_w[g * 5 + i] -= c.fac * ss[i];
            cl.d_abs[g] = nabs;
            cl.d_new[g] = nnew;
        }
    }
}

// ---------------------------------------------------------------------------
// 4. NTC / VHS collisions, one wave per cell.
//
// Candidates q = 0..M-1 are taken in chunks of 64, one per lane.  Pair indices
// depend only on the random stream, so each lane can see which earlier lanes
// of its chunk share a particle with it.  Lanes run in rounds: a lane runs
// once every earlier lane it shares a particle with has run, which gives the
// same result as running the candidates one after another.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool collide_pair(T *su, T *sv, T *sw, uint32_t i, uint32_t j, double cm,
                                             double accept_exp, double u2, double u3, double u4,
                                             double &seen)
{
    if constexpr (std::is_same<T, double>::value) {
        double ui = su[i], vi = sv[i], wi = sw[i];
        double uj = su[j], vj = sv[j], wj = sw[j];
        double d0 = ui - uj, d1 = vi - vj, d2 = wi - wj;
        double cr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        seen = fmax(seen, cr);
        double pa = pow(cr / cm, accept_exp);
        if (!(u2 < pa)) return false;
        double ct = 2.0 * u3 - 1.0;
        double st = sqrt(1.0 - ct * ct);
        double ph = D_TWO_PI * u4;
        double r0 = cr * st * cos(ph), r1 = cr * st * sin(ph), r2 = cr * ct;
        double m0 = 0.5 * (ui + uj), m1 = 0.5 * (vi + vj), m2 = 0.5 * (wi + wj);
        su[i] = m0 + 0.5 * r0; sv[i] = m1 + 0.5 * r1; sw[i] = m2 + 0.5 * r2;
        su[j] = m0 - 0.5 * r0; sv[j] = m1 - 0.5 * r1; sw[j] = m2 - 0.5 * r2;
        return true;
    } else {
        float ui = su[i], vi = sv[i], wi = sw[i];
        float uj = su[j], vj = sv[j], wj = sw[j];
        float d0 = ui - uj, d1 = vi - vj, d2 = wi - wj;
        float cr = sqrtf(__fmaf_rn(d0, d0, __fmaf_rn(d1, d1, d2 * d2)));
        seen = fmax(seen, (double)cr);
        float pa = powf(cr / (float)cm, (float)accept_exp);
        if (!(u2 < (double)pa)) return false;
        float ct = __fmaf_rn(2.0f, (float)u3, -1.0f);
        float st = sqrtf(fmaxf(__fmaf_rn(-ct, ct, 1.0f), 0.0f));
        float sp, cp;
        sincosf((float)D_TWO_PI * (float)u4, &sp, &cp);
        float h = 0.5f * cr;
        float r0 = h * st * cp, r1 = h * st * sp, r2 = h * ct;
        float m0 = 0.5f * (ui + uj), m1 = 0.5f * (vi + vj), m2 = 0.5f * (wi + wj);
        su[i] = m0 + r0; sv[i] = m1 + r1; sw[i] = m2 + r2;
        su[j] = m0 - r0; sv[j] = m1 - r1; sw[j] = m2 - r2;
        return true;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_collide(const DCase *__restrict__ cases, Cells cl, Soa<T> stg,
                                                 const int64_t *__restrict__ ibase,
                                                 const uint32_t *__restrict__ d_step, int G,
                                                 int64_t cap, int32_t *err)
{
    const uint32_t step = *d_step;
    const int wpb = blockDim.x >> 6, wid = threadIdx.x >> 6, lane = lane_id();
    for (int g = blockIdx.x * wpb + wid; g < G; g += gridDim.x * wpb) {
        const int k = cl.cell_case[g];
        const DCase &c = cases[k];
        const int lc = g - c.cell_base;
        const int32_t N = cl.n_int[g];
        int64_t M = 0;
        int ncoll = 0;
        double seen = 0.0;
        double cm = 0.0;
        if (cl.okc[g] && N >= 2 && ibase[g] + N <= cap) {
            const double P = cl.pc[g];
            const double dtc = c.full_dt ? c.dt : (1.0 - P) * c.dt;
            cm = cl.cr_max[g];
            double Mr = 0.5 * (double)(N - 1) * c.coll_k * cl.wt[g * 5 + 0] *
                        pow(c.c_ref / cm, 2.0 * c.ups) * cm * dtc;
            U4 r = draw(c, step, (uint32_t)lc, 0, TAG_NCNT, 0);
            double Mf = floor(Mr + u01(r.a));
            if (Mf > 2.0e9) { if (lane == 0) atomicOr(err, ERR_CAPACITY); Mf = 0.0; }
            M = (int64_t)Mf;
            const double aexp = 1.0 - 2.0 * c.ups;
            T *su = stg.u + ibase[g], *sv = stg.v + ibase[g], *sw = stg.w + ibase[g];
            for (int64_t q0 = 0; q0 < M; q0 += WAVE) {
                const int64_t q = q0 + lane;
                const bool act = q < M;
                uint32_t i = 0xffffffffu, j = 0xfffffffeu;
                double u2 = 0.0, u3 = 0.0, u4 = 0.0;
                if (act) {
                    U4 a = draw(c, step, (uint32_t)lc, (uint32_t)q, TAG_PAIR, 0);
                    U4 bb = draw(c, step, (uint32_t)lc, (uint32_t)q, TAG_PAIR, 1);
                    uint64_t r0 = ((uint64_t)a.a << 32) | a.b;
                    uint64_t r1 = ((uint64_t)a.c << 32) | a.d;
                    i = (uint32_t)mulhi64(r0, (uint64_t)N);
                    j = (uint32_t)mulhi64(r1, (uint64_t)(N - 1));
                    if (j >= i) j += 1;
                    u2 = u01(bb.a); u3 = u01(bb.b); u4 = u01(bb.c);
                }
                const uint64_t actm = __ballot(act);
                uint64_t dep = 0;
                const int nl = (int)min((int64_t)WAVE, M - q0);
                for (int l = 0; l < nl; ++l) {
                    uint32_t il = __builtin_amdgcn_readlane(i, l);
                    uint32_t jl = __builtin_amdgcn_readlane(j, l);
                    bool cf = (l < lane) && (il == i || il == j || jl == i || jl == j);
                    dep |= (uint64_t)cf << l;
                }
                uint64_t done = ~actm;
                while (done != ~0ull) {
                    const bool ready = act && !((done >> lane) & 1ull) && ((dep & ~done) == 0ull);
                    if (ready) {
                        if (collide_pair<T>(su, sv, sw, i, j, cm, aexp, u2, u3, u4, seen)) ++ncoll;
                    }
                    // this round's stores are complete before the next round loads
                    __threadfence_block();
                    done |= __ballot(ready);
                }
            }
        }
        seen = wave_max(seen);
        ncoll = wave_sum_i(ncoll);
        if (lane == 0) {
            cl.d_cand[g] = (int32_t)M;
            cl.d_coll[g] = ncoll;
            if (seen > cm && M > 0) cl.cr_max[g] = seen;
        }
    }
}

// ---------------------------------------------------------------------------
// 5. Reservoir injection, one wave per case.  Entrants are kept in (side,
// slot) order; each gets its rank among entrants of the same destination.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_inject(const DCase *__restrict__ cases, int ncases, Cells cl,
                                                Inj<T> inj, const uint32_t *__restrict__ d_step,
                                                int64_t *d_ninj, int32_t *err)
{
    const uint32_t step = *d_step;
    const int wpb = blockDim.x >> 6, wid = threadIdx.x >> 6, lane = lane_id();
    const int k = blockIdx.x * wpb + wid;
    if (k >= ncases) return;
    const DCase &c = cases[k];
    int64_t count = 0;
    for (int side = 0; side < 2; ++side) {
        if ((side == 0 ? c.bc_lo : c.bc_hi) != 0) continue;
        const double rho = side == 0 ? c.rho_L : c.rho_R;
        const double U = side == 0 ? c.u_L : c.u_R;
        const double Ts = side == 0 ? c.T_L : c.T_R;
        const double tau = viscosity(c, Ts) / (rho * c.R * Ts);
        const double Ps = absorb_fraction(c.law, c.dt, tau);
        const double Lg = c.dt * (fabs(U) + 8.0 * sqrt(c.R * Ts));
        U4 r = draw(c, step, (uint32_t)side, 0, TAG_ICNT, 0);
        double nf = floor((1.0 - Ps) * rho * Lg / c.m_p + u01(r.a));
        if (nf > 2.0e9) { if (lane == 0) atomicOr(err, ERR_CAPACITY); nf = 0.0; }
        const int64_t ng = (int64_t)nf;
        int64_t nside = 0;
        for (int64_t q0 = 0; q0 < ng; q0 += WAVE) {
            const int64_t q = q0 + lane;
            int dest = -1;
            T px = 0, pu = 0, pv = 0, pw = 0;
            if (q < ng) {
                U4 a = draw(c, step, (uint32_t)side, (uint32_t)q, TAG_IVEL, 0);
                U4 bb = draw(c, step, (uint32_t)side, (uint32_t)q, TAG_IVEL, 1);
                double uu[6] = {u01(a.b), u01(a.c), u01(a.d), u01(bb.a), u01(bb.b), u01(bb.c)};
                double xi[3];
                maxwell(U, 0.0, 0.0, Ts, c.R, uu, xi);
                if constexpr (std::is_same<T, double>::value) {
                    double x = side == 0 ? c.x_lo - u01(a.a) * Lg : c.x_hi + u01(a.a) * Lg;
                    double u = xi[0];
                    x = x + u * c.dt;
                    dest = bc_cell_abs(c, x, u);
                    px = x; pu = u;
                } else {
                    float u = (float)xi[0];
                    float lgc = (float)(Lg / c.dx);
                    float X0 = side == 0 ? -(float)u01(a.a) * lgc : (float)u01(a.a) * lgc;
                    float X = X0 + u * c.dtdx_f;
                    float fl = floorf(X);
                    int I = (side == 0 ? 0 : c.ncells) + (int)fl;
                    float s = 0.0f;
                    dest = bc_cell_rel(c, I, X - fl, u, s);
                    px = s; pu = u;
                }
                pv = (T)xi[1]; pw = (T)xi[2];
            }
            const bool ent = dest >= 0;
            const uint64_t m = __ballot(ent);
            const int64_t pos = count + __popcll(m & lanemask_lt());
            int rank = 0;
            uint64_t rem = m;
            while (rem) {
                const int leader = __ffsll((unsigned long long)rem) - 1;
                const int v = __builtin_amdgcn_readlane(dest, leader);
                const uint64_t mm = __ballot(ent && dest == v);
                int old = 0;
                if (lane == leader) old = atomicAdd(&cl.inj_cnt[c.cell_base + v], __popcll(mm));
                old = __builtin_amdgcn_readlane(old, leader);
                if (ent && dest == v) rank = old + __popcll(mm & lanemask_lt());
                rem &= ~mm;
            }
            if (ent) {
                if (pos < c.inj_cap) {
                    const int64_t sl = c.inj_base + pos;
                    inj.x[sl] = px; inj.u[sl] = pu; inj.v[sl] = pv; inj.w[sl] = pw;
                    inj.dest[sl] = c.cell_base + dest;
                    inj.rank[sl] = rank;
                } else {
                    atomicOr(err, ERR_CAPACITY);
                }
            }
            count += __popcll(m);
            nside += __popcll(m);
        }
        if (lane == 0) d_ninj[2 * k + side] = nside;
    }
    if (lane == 0) inj.count[k] = (int32_t)min(count, c.inj_cap);
}

// ---------------------------------------------------------------------------
// 6. Free flight of the staged particles: destination histogram per source cell
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024) k_stream_hist(const DCase *__restrict__ cases, Cells cl, Soa<T> stg,
                                                      const int64_t *__restrict__ ibase, int G, int64_t cap,
                                                      int32_t *err, int64_t *d_nout)
{
    __shared__ int h[NBIN];
    __shared__ int nout;
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const int k = cl.cell_case[g];
        const DCase &c = cases[k];
        const int lc = g - c.cell_base;
        for (int t = threadIdx.x; t < NBIN; t += blockDim.x) h[t] = 0;
        if (threadIdx.x == 0) nout = 0;
        __syncthreads();
        const int64_t b = ibase[g];
        const int32_t n = (int32_t)min((int64_t)cl.n_int[g], cap - b);
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            T x = stg.x[b + i], u = stg.u[b + i];
            int dest = Flight<T>::go(c, lc, x, u);
            if (dest < 0) {
                atomicAdd(&nout, 1);
            } else {
                int d = dest - lc;
                if (d < -KWIN || d > KWIN) atomicOr(err, ERR_RANGE);
                else atomicAdd(&h[d + KWIN], 1);
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < NBIN; t += blockDim.x) cl.hist[(int64_t)g * NBIN + t] = h[t];
        if (threadIdx.x == 0 && nout) atomicAdd((unsigned long long *)&d_nout[k], (unsigned long long)nout);
        __syncthreads();
    }
}

// 7. particles arriving in each destination cell
__global__ void k_count_new(Cells cl, int G)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= G) return;
    int32_t s = cl.inj_cnt[d];
#pragma unroll
    for (int dl = -KWIN; dl <= KWIN; ++dl) {
        const int src = d - dl;
        if (src >= 0 && src < G) s += cl.hist[(int64_t)src * NBIN + dl + KWIN];
    }
    cl.cnt_new[d] = s;
}

// 9. start of each (source cell, destination) group inside its destination segment,
// in source-cell order; entrants follow the cell-sourced particles.
__global__ void k_bases(Cells cl, const int64_t *__restrict__ off_new, int G)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= G) return;
    int32_t run = 0;
    for (int src = d - KWIN; src <= d + KWIN; ++src) {
        if (src < 0 || src >= G) continue;
        const int64_t idx = (int64_t)src * NBIN + (d - src) + KWIN;
        const int32_t h = cl.hist[idx];
        cl.hist[idx] = run;
        run += h;
    }
    cl.inj_start[d] = off_new[d] + run;
}

// ---------------------------------------------------------------------------
// 10. Stable scatter of the staged particles into the next canonical array
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024) k_scatter(const DCase *__restrict__ cases, Cells cl, Soa<T> stg,
                                                  const int64_t *__restrict__ ibase, Soa<T> dst,
                                                  const int64_t *__restrict__ off_new, int G, int64_t cap)
{
    __shared__ int binbase[NBIN];
    __shared__ int wcnt[16][NBIN];
    const int lane = lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const int k = cl.cell_case[g];
        const DCase &c = cases[k];
        const int lc = g - c.cell_base;
        for (int t = threadIdx.x; t < NBIN; t += blockDim.x) binbase[t] = cl.hist[(int64_t)g * NBIN + t];
        for (int t = threadIdx.x; t < 16 * NBIN; t += blockDim.x) (&wcnt[0][0])[t] = 0;
        __syncthreads();
        const int64_t b = ibase[g];
        const int32_t n = (int32_t)min((int64_t)cl.n_int[g], cap - b);
        for (int i0 = 0; i0 < n; i0 += blockDim.x) {
            const int i = i0 + threadIdx.x;
            T x = 0, u = 0, v = 0, ww = 0;
            int key = -1;
            if (i < n) {
                x = stg.x[b + i]; u = stg.u[b + i]; v = stg.v[b + i]; ww = stg.w[b + i];
                int dest = Flight<T>::go(c, lc, x, u);
                if (dest >= 0) {
                    int d = dest - lc;
                    if (d >= -KWIN && d <= KWIN) key = d + KWIN;
                }
            }
            int my = 0;
            uint64_t rem = __ballot(key >= 0);
            while (rem) {
                const int leader = __ffsll((unsigned long long)rem) - 1;
                const int v0 = __builtin_amdgcn_readlane(key, leader);
                const uint64_t mm = __ballot(key == v0);
                if (key == v0) my = __popcll(mm & lanemask_lt());
                if (lane == leader) wcnt[w][v0] = __popcll(mm);
                rem &= ~mm;
            }
            __syncthreads();
            if (key >= 0) {
                int r = binbase[key] + my;
                for (int w2 = 0; w2 < w; ++w2) r += wcnt[w2][key];
                const int64_t pos = off_new[g + key - KWIN] + r;
                if (pos < cap) { dst.x[pos] = x; dst.u[pos] = u; dst.v[pos] = v; dst.w[pos] = ww; }
            }
            __syncthreads();
            for (int t = threadIdx.x; t < NBIN; t += blockDim.x) {
                int s = 0;
                for (int w2 = 0; w2 < nw; ++w2) { s += wcnt[w2][t]; wcnt[w2][t] = 0; }
                binbase[t] += s;
            }
            __syncthreads();
        }
    }
}

// 11. entrants go after the cell-sourced particles of their destination cell
template <typename T>
__global__ void __launch_bounds__(256) k_scatter_inj(const DCase *__restrict__ cases, Cells cl, Inj<T> inj,
                                                     Soa<T> dst, int64_t cap)
{
    const int k = blockIdx.x;
    const DCase &c = cases[k];
    const int32_t n = inj.count[k];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t sl = c.inj_base + i;
        const int d = inj.dest[sl];
        const int64_t pos = cl.inj_start[d] + inj.rank[sl];
        if (pos < cap) { dst.x[pos] = inj.x[sl]; dst.u[pos] = inj.u[sl]; dst.v[pos] = inj.v[sl]; dst.w[pos] = inj.w[sl]; }
    }
}

// ---------------------------------------------------------------------------
// 12. Wave part: NS flux (KFVS inviscid + central viscous, eps-scaled
// viscosity, weighted by the interface absorption fraction) and update of
// Psi_w (Eq. r1).  One thread per cell computes both of its faces.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void kfvs_half(const double W[5], double R, int sign, double H[5])
{
    double U = W[1], V = W[2], Wv = W[3], th = R * W[4];
    double a = U / sqrt(2.0 * th);
    double A = 0.5 * erfc(-(double)sign * a);
    double B = sqrt(th / D_TWO_PI) * exp(-a * a);
    double sg = (double)sign;
    double M1 = U * A + sg * B;
    double M2 = (U * U + th) * A + sg * U * B;
    double M3 = (U * U * U + 3.0 * U * th) * A + sg * (U * U + 2.0 * th) * B;
    H[0] = M1;
    H[1] = M2;
    H[2] = V * M1;
    H[3] = Wv * M1;
    H[4] = 0.5 * M3 + 0.5 * (V * V + Wv * Wv + 2.0 * th) * M1;
}

__device__ __forceinline__ double eps_factor(int law, double x)
{
    switch (law) {
    case 1: return x / (2.0 + x);
    case 2: return 1.0;
    case 3: {
        double em = -expm1(-x);
        return (-2.0 * em + x * (1.0 + exp(-x))) / (x - em);
    }
    default: return 1.0 - x / expm1(x);
    }
}

__device__ __forceinline__ bool valid_state(const double W[5]) { return W[0] > 0.0 && W[4] > 0.0 && isfinite(W[4]); }

__device__ void face_flux(const DCase &c, const double Wl[5], const double Wr[5], double F[5])
{
#pragma unroll
    for (int k = 0; k < 5; ++k) F[k] = 0.0;
    if (!valid_state(Wl) || !valid_state(Wr)) return;
    double Wm[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) Wm[k] = 0.5 * (Wl[k] + Wr[k]);
    const double mu = viscosity(c, Wm[4]);
    const double tau = mu / (Wm[0] * c.R * Wm[4]);
    const double xr = c.dt / tau;
    const double Pm = absorb_fraction(c.law, c.dt, tau);
    if (!(Pm > 0.0)) return;
    double Hp[5], Hm[5];
    kfvs_half(Wl, c.R, +1, Hp);
    kfvs_half(Wr, c.R, -1, Hm);
    const double mue = eps_factor(c.eps_law, xr) * mu;
    const double dU = (Wr[1] - Wl[1]) / c.dx;
    const double dV = (Wr[2] - Wl[2]) / c.dx;
    const double dW = (Wr[3] - Wl[3]) / c.dx;
    const double dT = (Wr[4] - Wl[4]) / c.dx;
    const double sxx = (4.0 / 3.0) * mue * dU;
    const double sxy = mue * dV;
    const double sxz = mue * dW;
    const double q = -(15.0 / 4.0) * c.R * mue * dT;
    const double visc[5] = {0.0, sxx, sxy, sxz, Wm[1] * sxx + Wm[2] * sxy + Wm[3] * sxz - q};
#pragma unroll
    for (int k = 0; k < 5; ++k) F[k] = Pm * ((Wl[0] * Hp[k] + Wr[0] * Hm[k]) - visc[k]);
}

// flux through local face f (between local cells f-1 and f) of a case
__device__ void case_face_flux(const DCase &c, const Cells &cl, int f, double F[5])
{
    const int C = c.ncells, base = c.cell_base;
    double Wl[5], Wr[5];
    int okl, okr;
    if (f == 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) Wr[k] = cl.wt[(int64_t)base * 5 + k];
        if (c.bc_lo == 0) { Wl[0] = c.rho_L; Wl[1] = c.u_L; Wl[2] = 0.0; Wl[3] = 0.0; Wl[4] = c.T_L; }
        else {
#pragma unroll
            for (int k = 0; k < 5; ++k) Wl[k] = Wr[k];
            Wl[1] = -Wr[1];
        }
        okl = (c.bc_lo == 0) || cl.okc[base];
        okr = cl.okc[base];
    } else if (f == C) {
#pragma unroll
        for (int k = 0; k < 5; ++k) Wl[k] = cl.wt[(int64_t)(base + C - 1) * 5 + k];
        if (c.bc_hi == 0) { Wr[0] = c.rho_R; Wr[1] = c.u_R; Wr[2] = 0.0; Wr[3] = 0.0; Wr[4] = c.T_R; }
        else {
#pragma unroll
            for (int k = 0; k < 5; ++k) Wr[k] = Wl[k];
            Wr[1] = -Wl[1];
        }
        okl = cl.okc[base + C - 1];
        okr = (c.bc_hi == 0) || cl.okc[base + C - 1];
    } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            Wl[k] = cl.wt[(int64_t)(base + f - 1) * 5 + k];
            Wr[k] = cl.wt[(int64_t)(base + f) * 5 + k];
        }
        okl = cl.okc[base + f - 1];
        okr = cl.okc[base + f];
    }
    if (okl && okr) face_flux(c, Wl, Wr, F);
    else {
#pragma unroll
        for (int k = 0; k < 5; ++k) F[k] = 0.0;
    }
}

__global__ void __launch_bounds__(256) k_wave(const DCase *__restrict__ cases, Cells cl, int G)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const DCase &c = cases[cl.cell_case[g]];
    const int lc = g - c.cell_base;
    double Fl[5], Fr[5];
    case_face_flux(c, cl, lc, Fl);
    case_face_flux(c, cl, lc + 1, Fr);
    const double r = c.dt / c.dx;
#pragma unroll
    for (int k = 0; k < 5; ++k) cl.psi_w[(int64_t)g * 5 + k] -= r * (Fr[k] - Fl[k]);
}

// ---------------------------------------------------------------------------
// 13. Particle moments of the new canonical array (Eq. gkt_moment0), running
// average of Psi_t, finite-state check.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024) k_moments(const DCase *__restrict__ cases, Cells cl, Soa<T> a,
                                                  const int64_t *__restrict__ off, int G, int accumulate,
                                                  int32_t *err)
{
    __shared__ double red[5 * 16];
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const DCase &c = cases[cl.cell_case[g]];
        const int64_t b = off[g], e = off[g + 1];
        double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t kk = b + threadIdx.x; kk < e; kk += blockDim.x) {
            double u = a.u[kk], v = a.v[kk], w = a.w[kk];
            s[0] += 1.0; s[1] += u; s[2] += v; s[3] += w;
            s[4] += 0.5 * (u * u + v * v + w * w);
        }
        block_sum<5>(s, red);
        if (threadIdx.x == 0) {
            bool bad = false;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                double p = c.fac * s[k];
                cl.psi_p[(int64_t)g * 5 + k] = p;
                double t = cl.psi_w[(int64_t)g * 5 + k] + p;
                if (!isfinite(t)) bad = true;
                if (accumulate) cl.avg[(int64_t)g * 5 + k] += t;
            }
            if (bad) atomicOr(err, ERR_STATE);
        }
    }
}

// closes the step: particle-steps of this step (particles alive at its start), step index
__global__ void k_finish(uint32_t *d_step, const int64_t *__restrict__ off, int G, int64_t *d_psteps)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *d_psteps += off[G];
        *d_step += 1;
    }
}

// ---------------------------------------------------------------------------
// Step sequence
// ---------------------------------------------------------------------------
template <typename T>
static Soa<T> soa(void *const p[4])
{
    return Soa<T>{(T *)p[0], (T *)p[1], (T *)p[2], (T *)p[3]};
}

static inline int grid_cells(const duwp_ctx *ctx) { return ctx->G; }

struct Mark {
    duwp_ctx *ctx;
    const char *name;
    Mark(duwp_ctx *c, const char *n) : ctx(c), name(n)
    {
        KernelTimer &t = ctx->timer;
        if (t.on) (void)hipEventRecord(t.ev[2 * t.idx], ctx->stream);
    }
    ~Mark()
    {
        KernelTimer &t = ctx->timer;
        if (t.on) {
            (void)hipEventRecord(t.ev[2 * t.idx + 1], ctx->stream);
            if ((int)t.names.size() <= t.idx) t.names.push_back(name);
            t.idx++;
        }
    }
};

template <typename T>
static void step_impl(duwp_ctx *ctx)
{
    const int G = ctx->G, p = ctx->step & 1;
    const int bc = ctx->block_cells;
    hipStream_t st = ctx->stream;
    Soa<T> src = soa<T>(ctx->A[p]), dst = soa<T>(ctx->A[p ^ 1]), stg = soa<T>(ctx->S);
    Inj<T> inj{(T *)ctx->J[0], (T *)ctx->J[1], (T *)ctx->J[2], (T *)ctx->J[3], ctx->j_dest, ctx->j_rank,
               ctx->j_count};
    const int gc = grid_cells(ctx);
    const int gthreads = (G + 255) / 256;
    {
        Mark m(ctx, "cellstate");
        hipLaunchKernelGGL(k_cellstate<T>, dim3(gc), dim3(bc), 0, st, ctx->d_cases, ctx->cl, ctx->off[p],
                           ctx->d_step, G, ctx->d_err, ctx->d_nout, ctx->d_ninj);
    }
    {
        Mark m(ctx, "scan_staging");
        enqueue_scan(ctx, ctx->cl.n_int, ctx->ibase, ctx->d_total);
    }
    {
        Mark m(ctx, "absorb_resample");
        hipLaunchKernelGGL(k_absorb_resample<T>, dim3(gc), dim3(bc), 0, st, ctx->d_cases, ctx->cl, src,
                           ctx->off[p], stg, ctx->ibase, ctx->d_step, G, ctx->cap, ctx->d_err);
    }
    {
        Mark m(ctx, "collide");
        const int wpb = 4;
        hipLaunchKernelGGL(k_collide<T>, dim3((G + wpb - 1) / wpb), dim3(64 * wpb), 0, st, ctx->d_cases,
                           ctx->cl, stg, ctx->ibase, ctx->d_step, G, ctx->cap, ctx->d_err);
    }
    {
        Mark m(ctx, "inject");
        const int wpb = 4;
        hipLaunchKernelGGL(k_inject<T>, dim3((ctx->ncases + wpb - 1) / wpb), dim3(64 * wpb), 0, st,
                           ctx->d_cases, ctx->ncases, ctx->cl, inj, ctx->d_step, ctx->d_ninj, ctx->d_err);
    }
    {
        Mark m(ctx, "stream_hist");
        hipLaunchKernelGGL(k_stream_hist<T>, dim3(gc), dim3(bc), 0, st, ctx->d_cases, ctx->cl, stg,
                           ctx->ibase, G, ctx->cap, ctx->d_err, ctx->d_nout);
    }
    {
        Mark m(ctx, "count_new");
        hipLaunchKernelGGL(k_count_new, dim3(gthreads), dim3(256), 0, st, ctx->cl, G);
    }
    {
        Mark m(ctx, "scan_offsets");
        enqueue_scan(ctx, ctx->cl.cnt_new, ctx->off[p ^ 1], ctx->d_total + 1);
    }
    {
        Mark m(ctx, "bases");
        hipLaunchKernelGGL(k_bases, dim3(gthreads), dim3(256), 0, st, ctx->cl, ctx->off[p ^ 1], G);
    }
    {
        Mark m(ctx, "scatter");
        hipLaunchKernelGGL(k_scatter<T>, dim3(gc), dim3(bc), 0, st, ctx->d_cases, ctx->cl, stg, ctx->ibase,
                           dst, ctx->off[p ^ 1], G, ctx->cap);
    }
    {
        Mark m(ctx, "scatter_inj");
        hipLaunchKernelGGL(k_scatter_inj<T>, dim3(ctx->ncases), dim3(256), 0, st, ctx->d_cases, ctx->cl, inj,
                           dst, ctx->cap);
    }
    {
        Mark m(ctx, "wave");
        hipLaunchKernelGGL(k_wave, dim3(gthreads), dim3(256), 0, st, ctx->d_cases, ctx->cl, G);
    }
    {
        Mark m(ctx, "moments");
        hipLaunchKernelGGL(k_moments<T>, dim3(gc), dim3(bc), 0, st, ctx->d_cases, ctx->cl, dst, ctx->off[p ^ 1],
                           G, 1, ctx->d_err);
    }
    {
        Mark m(ctx, "finish");
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, ctx->d_step, ctx->off[p], G, ctx->d_psteps);
    }
}

void enqueue_step(duwp_ctx *ctx)
{
    if (ctx->precision == DUWP_MIXED) step_impl<float>(ctx);
    else step_impl<double>(ctx);
}

void enqueue_moments(duwp_ctx *ctx)
{
    const int p = ctx->step & 1;
    if (ctx->precision == DUWP_MIXED)
        hipLaunchKernelGGL(k_moments<float>, dim3(ctx->G), dim3(ctx->block_cells), 0, ctx->stream, ctx->d_cases,
                           ctx->cl, soa<float>(ctx->A[p]), ctx->off[p], ctx->G, 0, ctx->d_err);
    else
        hipLaunchKernelGGL(k_moments<double>, dim3(ctx->G), dim3(ctx->block_cells), 0, ctx->stream, ctx->d_cases,
                           ctx->cl, soa<double>(ctx->A[p]), ctx->off[p], ctx->G, 0, ctx->d_err);
}

}  // namespace duwp
