// Stage kernels of one DUWP time step (gfx950, wave64) and the step sequence.
//
// Data layout: cells of all cases are numbered case by case (global cell g);
// particles are structure-of-arrays sorted by global cell, so every case's
// particles are contiguous.  Two canonical buffers alternate with the step
// parity.  The intermediate array of a step (per cell: survivors in order,
// then resampled particles by slot) lives in place in the canonical buffer
// for a cell that neither absorbs nor resamples anything, and in a staging
// buffer otherwise.  Cell arrays are FP64.  Particle storage is FP64 with
// absolute positions, or FP32 with the position relative to the particle's
// cell (in cells, [0,1)).
//
// Per step (Sec. 3.4, Steps 2-3, Eq. r1):
//   cellstate        Psi_t = Psi_w + Psi_p, (rho,U,T), tau = mu/p, P (Eq. p),
//                    absorbed and resampled counts, staging segments of the
//                    cells that change; in extra blocks, the reservoir
//                    injection candidates
//   absorb_resample  classify, absorb into Psi_w, compact survivors, sample
//                    new particles (Eq. maxsample), subtract their moments
//   collide          NTC/VHS (Appendix A), candidates in order: a wave per
//                    cell or per work item with conflict-free rounds, or a
//                    block per big cell; in its first blocks (or a kernel of
//                    their own on large inflows), the entrants' ranks
//   count_bases/scan windowed stable counting-sort counts, group bases, offsets
//                    (one single-block kernel on small grids)
//   scatter          free flight again, stable scatter into the next canonical
//                    array, particle moment sums per destination; the
//                    entrants after the cell-sourced particles of their cell
//   gather_moments   Psi_p of the new state, NS wave flux and update of
//                    Psi_w, running average of Psi_t
#include <hip/hip_runtime.h>
#include <climits>
#include <math.h>

#include <type_traits>

#include "duwp_ctx.hpp"
#include "duwp_device.hpp"
#include "duwp_physics.hpp"
#include "duwp_scan.hpp"

namespace duwp {

constexpr int MB = 1;                  // destinations |d| <= MB get register moment sums
constexpr int NMB = 2 * MB + 1;
constexpr int NBI = 2 * (KWIN + 1);    // injection destination window (both ends)

template <typename T>
__device__ void inject_gen_wave(const DCase &c, int k, int side, const Inj<T> &inj, uint32_t step, int32_t *err,
                                int wi, int nwv);
template <typename T, int NT>
__device__ void inject_rank_block(const DCase &c, const Cells &cl, const Inj<T> &inj, int64_t *d_ninj, int32_t *err,
                                  int k, int y);

// ---------------------------------------------------------------------------
// 1. Cell state at step start, absorbed and resampled counts, collision
// candidate counts.  A block takes 64 cells, one lane of its first wave per
// cell; the absorbed particles of its cells with P > 0 are counted by all of
// its waves (cell l by wave l mod waves), so that cells with many particles
// keep the whole GPU busy.  The gen_b blocks per (case, side) after the cells'
// blocks generate the step's injection candidates (they read nothing the step
// computes).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024) k_cellstate(const DCase *__restrict__ cases, Cells cl,
                                                     const int64_t *__restrict__ off,
                                                     const uint32_t *__restrict__ d_step, int G,
                                                     int32_t *err, int64_t *d_nout, int64_t *d_ninj,
                                                     int abs_stream, int big_min_n, int big_min_m, int64_t cap,
                                                     Inj<T> inj, int gen_b)
{
    __shared__ double sP[WAVE];
    __shared__ int64_t sb[WAVE], se[WAVE], spb[WAVE];
    __shared__ int sk[WAVE], scnt[WAVE];
    const uint32_t step = *d_step;
    const int lane = lane_id(), wv = wave_id(), nw = blockDim.x >> 6;
    const int cblk = (G + WAVE - 1) / WAVE;
    if ((int)blockIdx.x >= cblk) {
        const int e = (int)blockIdx.x - cblk, ks = e / gen_b, sub = e - ks * gen_b;
        inject_gen_wave<T>(cases[ks >> 1], ks >> 1, ks & 1, inj, step, err, sub * nw + wv, gen_b * nw);
        return;
    }
    const int g0 = blockIdx.x * WAVE;
    const int nc = min(WAVE, G - g0);
    for (int t = threadIdx.x; t < nc * NBIN; t += blockDim.x) cl.hist_nx[(int64_t)g0 * NBIN + t] = 0;
    const int g = g0 + lane;
    const bool in = lane < nc;
    const int k = (in && wv == 0) ? cl.cell_case[g] : 0;
    const DCase &c = cases[k];
    double W[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int ok = 0;
    double P = 0.0, tau = 0.0;
    int64_t b = 0, e = 0, pbase = 0;
    if (in && wv == 0) {
        double t[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) t[i] = cl.psi_w[(int64_t)g * 5 + i] + cl.psi_p[(int64_t)g * 5 + i];
        ok = primitive(t, c.R, W);
        if (ok) {
            tau = viscosity(c, W[4]) / (W[0] * c.R * W[4]);
            P = absorb_fraction(c.law, c.dt, tau);
        }
        b = off[g];
        e = off[g + 1];
        pbase = off[c.cell_base];
    }
    // classification (one Philox block decides four consecutive particles of a
    // case): cell l of the block is counted by wave l mod nw
    if (wv == 0) {
        sP[lane] = (in && e > b) ? P : 0.0;
        sb[lane] = b; se[lane] = e; spb[lane] = pbase; sk[lane] = k;
        scnt[lane] = 0;
    }
    __syncthreads();
    for (int l = wv; l < nc; l += nw) {
        const double Pl = sP[l];
        if (!(Pl > 0.0)) continue;
        const int64_t bl = sb[l], el = se[l], pl = spb[l];
        const DCase &cc = cases[sk[l]];
        const int64_t q0 = (bl - pl) >> 2, q1 = (el - 1 - pl) >> 2;
        int cnt = 0;
        for (int64_t q = q0 + lane; q <= q1; q += WAVE) {
            const U4 r = draw(cc, step, (uint32_t)q, 0, TAG_CLS, 0);
            const int64_t i0 = pl + 4 * q;
            const uint32_t wd[4] = {r.a, r.b, r.c, r.d};
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (i0 + m >= bl && i0 + m < el && u01(wd[m]) < Pl) ++cnt;
        }
        cnt = wave_sum_i(cnt);
        if (lane == 0) scnt[l] = cnt;
    }
    __syncthreads();
    if (wv != 0) return;
    const int32_t nabs = in ? scnt[lane] : 0;
    const int lc = g - c.cell_base;
    int32_t nnew = 0, N = 0, M = 0, ns = 0;
    if (in) {
        if (ok) {
            const double Mw = c.dx * cl.psi_w[(int64_t)g * 5 + 0];
            const U4 r = draw(c, step, (uint32_t)lc, 0, TAG_RCNT, 0);
            double nf = floor((1.0 - P) * Mw / c.m_p + u01(r.a));
            const double capn = floor((Mw > 0.0 ? Mw : 0.0) / c.m_p);
            if (nf > capn) nf = capn;
            if (nf < 0.0) nf = 0.0;
            if (nf > 2.0e9) { atomicOr(err, ERR_CAPACITY); nf = 0.0; }
            nnew = (int32_t)nf;
        }
        ns = (int32_t)(e - b) - nabs;
        N = ns + nnew;
        // NTC candidate count (Appendix A) over the collision share of the step
        if (ok && N >= 2) {
            const double dtc = c.full_dt ? c.dt : (1.0 - P) * c.dt;
            const double cm = cl.cr_max[g];
            const double Mr = 0.5 * (double)(N - 1) * c.coll_k * W[0] * pow(c.c_ref / cm, 2.0 * c.ups) * cm * dtc;
            const U4 r = draw(c, step, (uint32_t)lc, 0, TAG_NCNT, 0);
            double Mf = floor(Mr + u01(r.a));
            if (Mf > 2.0e9) { atomicOr(err, ERR_CAPACITY); Mf = 0.0; }
            M = (int32_t)Mf;
        }
    }
    // cells with many particles and many candidates collide one block each
    // (k_collide_big); the others go to the wave kernel's candidate list
    const bool big = in && N >= big_min_n && M >= big_min_m;
    const uint64_t bm = __ballot(big);
    if (bm) {
        int base = 0;
        if (lane == 0) base = atomicAdd(cl.nbig, __popcll(bm));
        base = __shfl(base, 0, WAVE);
        if (big) cl.big_list[base + lane_rank_lt(bm)] = g;
    }
    // cells that absorb or resample are listed for k_absorb_resample; the others
    // keep their segment in place
    const bool touched = in && (nabs > 0 || nnew > 0);
    const uint64_t tm = __ballot(touched);
    if (tm) {
        int base = 0;
        if (lane == 0) base = atomicAdd(cl.ntouch, __popcll(tm));
        base = __shfl(base, 0, WAVE);
        if (touched) cl.touch_list[base + lane_rank_lt(tm)] = g;
    }
    // their segments in the staging array, handed out from a running count a
    // wave at a time (where a segment lies changes nothing that is computed
    // from it); past the capacity a cell is reported and skipped
    int64_t sseg = 0;
    if (tm) {
        const int64_t nst = touched ? (int64_t)N : 0;
        int64_t incl = nst;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const int64_t t = __shfl_up(incl, o, WAVE);
            if (lane >= o) incl += t;
        }
        const int64_t tot = readlane64(incl, WAVE - 1);
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd((unsigned long long *)cl.nstage, (unsigned long long)tot);
        sseg = readlane64(base, 0) + incl - nst;
        if (touched && sseg + N > cap) atomicOr(err, ERR_CAPACITY);
    }
    if (!in) return;
    if (!touched) {
        cl.seg[g] = b;
        cl.d_abs[g] = 0;
        cl.d_new[g] = 0;
    } else {
        cl.seg[g] = sseg;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) cl.wt[(int64_t)g * 5 + i] = W[i];
    cl.pc[g] = P;
    if (abs_stream) cl.tau[g] = tau;    // read only by streamed absorption
    cl.okc[g] = ok;
    cl.n_surv[g] = ns;
    cl.n_new[g] = nnew;
    cl.n_int[g] = N;
    cl.seg_stg[g] = touched ? 1 : 0;
    cl.inj_cnt[g] = 0;
    cl.d_cand[g] = M;
    cl.ncand_w[g] = big ? 0 : M;
    cl.d_coll[g] = 0;
    if (lc == 0) {
        d_nout[k] = 0;
        d_ninj[2 * k] = 0;
        d_ninj[2 * k + 1] = 0;
    }
}

static void enqueue_scan(duwp_ctx *ctx, const int32_t *in, int64_t *out, int64_t *total, int64_t cap)
{
    const int G = ctx->G;
    if (G <= SCAN1_MAX) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, ctx->stream, in, G, out, cap, total,
                           ctx->d_err);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(ctx->ntiles), dim3(SCAN_BLOCK), 0, ctx->stream, in, G,
                       ctx->scan_part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, ctx->stream, ctx->scan_part,
                       ctx->ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3(ctx->ntiles), dim3(SCAN_BLOCK), 0, ctx->stream, in, G,
                       ctx->scan_part, out, cap, total, ctx->d_err);
}

// Destination bin (d + KWIN) of a particle of local cell lc after free flight;
// -1 when it leaves through a reservoir or moves farther than the window.  The
// histograms count a particle in this bin and every change of its velocity
// moves it between bins, so one in no bin is in none when the scatter places
// the particles: if it still moves that far, the scatter reports the range
// error (a recount would give the same histogram).
template <typename T, typename K>
__device__ __forceinline__ int flight_bin(const K &c, int lc, T x, T u)
{
    const int dest = Flight<T>::go(c, lc, x, u);
    if (dest < 0) return -1;
    const int d = dest - lc;
    return (d < -KWIN || d > KWIN) ? -1 : d + KWIN;
}

// Cell segment of the intermediate array: staging buffer or in place.
template <typename T>
__device__ __forceinline__ P4<T> *segment(const Cells &cl, int g, P4<T> *src, P4<T> *stg, int64_t &base)
{
    base = cl.seg[g];
    return cl.seg_stg[g] ? stg : src;
}

// ---------------------------------------------------------------------------
// 3. Classify + absorb + compact survivors + resample (Step 2), for the cells
// that absorb or resample anything, into the staging segments the cell-state
// kernel handed out.
// ---------------------------------------------------------------------------
template <typename T, bool STRM>
__global__ void __launch_bounds__(512) k_absorb_resample(const DCase *__restrict__ cases, Cells cl,
                                                          const P4<T> *__restrict__ src,
                                                          const int64_t *__restrict__ off, P4<T> *__restrict__ stg,
                                                          const uint32_t *__restrict__ d_step, int G,
                                                          int64_t cap, int32_t *err, int64_t *d_nout)
{
    __shared__ double red[5 * 16];
    __shared__ int scr[16];
    __shared__ int dh[NBIN];
    __shared__ unsigned long long farland;   // landing bins |dd| >= 2 of absorbed particles
    const uint32_t step = *d_step;
    const int ntouch = *cl.ntouch;
    for (int e0 = blockIdx.x; e0 < ntouch; e0 += gridDim.x) {
        const int g = cl.touch_list[e0];
        const int k = cl.cell_case[g];
        const DCase &c = cases[k];
        const CaseK ck(c);
        const int lc = g - c.cell_base;
        const double P = cl.pc[g];
        const int64_t b = off[g], e = off[g + 1];
        const int64_t pbase = off[c.cell_base];
        const int64_t ob = cl.seg[g];
        const int32_t nsurv = cl.n_surv[g];
        double sa[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        // absorb_stream: moments of the absorbed particles landing in g-1 and g+1
        // (sa: in g), particles that leave through a reservoir
        // (STRM: the context has such a case; the other instantiation carries none of this)
        const bool strm = STRM && c.abs_stream != 0;
        const double tau = strm ? cl.tau[g] : 0.0;
        double sl[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, sr[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        bool hasl = false, hasr = false;
        int nleave = 0;
        int64_t written = 0;
        // the cell's destination histogram loses the absorbed and gains the resampled particles
        for (int t = threadIdx.x; t < NBIN; t += blockDim.x) dh[t] = 0;
        if (threadIdx.x == 0) farland = 0ull;
        __syncthreads();
        if (P > 0.0) {
            // one Philox block classifies the four particles of an aligned quad of
            // case-local indices: a thread takes one quad
            const int64_t qa = (b - pbase) >> 2, qb = (e - 1 - pbase) >> 2;
            for (int64_t q0 = qa; q0 <= qb; q0 += blockDim.x) {
                const int64_t qd = q0 + threadIdx.x;
                T xs[4], us[4], vs[4], ws[4];
                int keep = 0;
                if (qd <= qb) {
                    const U4 r = draw(ck, step, (uint32_t)qd, 0, TAG_CLS, 0);
                    const uint32_t wd[4] = {r.a, r.b, r.c, r.d};
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int64_t kk = pbase + 4 * qd + m;
                        xs[m] = 0; us[m] = 0; vs[m] = 0; ws[m] = 0;
                        if (kk < b || kk >= e) continue;
                        const P4<T> r = src[kk];
                        xs[m] = r.x; us[m] = r.u; vs[m] = r.v; ws[m] = r.w;
                        const double uu = u01(wd[m]);
                        if (uu < P) {
                            double du = us[m];
                            const double dv = vs[m], dw = ws[m];
                            int dd = 0;
                            if (strm) {
                                T uf = us[m];
                                const int dest = PartialFlight<T>::go(ck, lc, xs[m], uf,
                                                                      free_time(c.law, tau, uu));
                                dd = dest < 0 ? INT_MIN : dest - lc;
                                du = uf;
                            }
                            const double e2 = 0.5 * (du * du + dv * dv + dw * dw);
                            if (dd == 0) {
                                sa[0] += 1.0; sa[1] += du; sa[2] += dv; sa[3] += dw; sa[4] += e2;
                            } else if (dd == -1) {
                                sl[0] += 1.0; sl[1] += du; sl[2] += dv; sl[3] += dw; sl[4] += e2;
                                hasl = true;
                            } else if (dd == 1) {
                                sr[0] += 1.0; sr[1] += du; sr[2] += dv; sr[3] += dw; sr[4] += e2;
                                hasr = true;
                            } else if (dd == INT_MIN) {
                                ++nleave;
                            } else if (dd >= -KWIN && dd <= KWIN) {
                                atomicOr(&farland, 1ull << (dd + KWIN));
                            } else {
                                atomicOr(err, ERR_RANGE);
                            }
                            const int hb = flight_bin<T>(ck, lc, xs[m], us[m]);
                            if (hb >= 0) atomicSub(&dh[hb], 1);
                        } else {
                            keep |= 1 << m;
                        }
                    }
                }
                // survivors in index order: quads in thread order, then m
                int tot;
                int pre = block_count_prefix(__popc(keep), scr, &tot);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    if (!((keep >> m) & 1)) continue;
                    const int64_t d = ob + written + pre++;
                    if (d < cap) stg[d] = P4<T>{xs[m], us[m], vs[m], ws[m]};
                    else atomicOr(err, ERR_CAPACITY);
                }
                written += tot;
            }
            block_sum<5>(sa, red);
            if (strm) {
                // absorbed moments that landed in other cells go to those cells'
                // rows (slot KWIN - dd); the gather adds them to the wave part
                auto land = [&](int dd, const double (&v)[5]) {
                    if (threadIdx.x < 5) cl.wabs[((int64_t)(g + dd) * NBIN + (KWIN - dd)) * 5 + threadIdx.x] = v[threadIdx.x];
                    if (threadIdx.x == 0) cl.wabs_in[g + dd] = 1;
                };
                if (__syncthreads_or(hasl)) { block_sum<5>(sl, red); land(-1, sl); }
                if (__syncthreads_or(hasr)) { block_sum<5>(sr, red); land(1, sr); }
                int tot;
                (void)block_count_prefix(nleave, scr, &tot);
                if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long *)&d_nout[k], (unsigned long long)tot);
                // farther landings (rare): a pass over the cell per landing bin
                const unsigned long long fl = farland;
                for (int bin = 0; bin < NBIN; ++bin) {
                    if (!((fl >> bin) & 1ull)) continue;
                    const int dd = bin - KWIN;
                    double a2[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                    for (int64_t kk = b + threadIdx.x; kk < e; kk += blockDim.x) {
                        const int64_t li = kk - pbase;
                        const U4 r = draw(ck, step, (uint32_t)(li >> 2), 0, TAG_CLS, 0);
                        const int m = (int)(li & 3);
                        const uint32_t wdm = m == 0 ? r.a : (m == 1 ? r.b : (m == 2 ? r.c : r.d));
                        const double uu = u01(wdm);
                        if (!(uu < P)) continue;
                        const P4<T> rr = src[kk];
                        T uf = rr.u;
                        const int dest = PartialFlight<T>::go(ck, lc, rr.x, uf, free_time(c.law, tau, uu));
                        if (dest < 0 || dest - lc != dd) continue;
                        const double du = uf, dv = rr.v, dw = rr.w;
                        a2[0] += 1.0; a2[1] += du; a2[2] += dv; a2[3] += dw;
                        a2[4] += 0.5 * (du * du + dv * dv + dw * dw);
                    }
                    block_sum<5>(a2, red);
                    land(dd, a2);
                }
            }
        } else {
            for (int64_t kk = b + threadIdx.x; kk < e; kk += blockDim.x) {
                int64_t d = ob + (kk - b);
                if (d < cap) stg[d] = src[kk];
                else atomicOr(err, ERR_CAPACITY);
            }
        }
        // resample 1-P of the start-of-step wave mass at the total state
        const int32_t nnew = cl.n_new[g];
        double ss[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (nnew > 0) {
            const double *Wc = cl.wt + (int64_t)g * 5;
            const Maxwell<T> mw(Wc[1], Wc[2], Wc[3], Wc[4], ck.R);
            for (int q = threadIdx.x; q < nnew; q += blockDim.x) {
                U4 a = draw(ck, step, (uint32_t)lc, (uint32_t)q, TAG_RVEL, 0);
                U4 bb = draw(ck, step, (uint32_t)lc, (uint32_t)q, TAG_RVEL, 1);
                const uint32_t w6[6] = {a.b, a.c, a.d, bb.a, bb.b, bb.c};
                T xi[3];
                mw.sample(w6, xi);
                T px;
                if constexpr (std::is_same<T, double>::value) {
                    px = ck.x_lo + ((double)lc + u01(a.a)) * ck.dx;
                } else {
                    px = u01f(a.a);
                    if (px >= 1.0f) px = 0.99999994f;
                }
                T pu = xi[0], pv = xi[1], pw = xi[2];
                const int hb = flight_bin<T>(ck, lc, px, pu);
                if (hb >= 0) atomicAdd(&dh[hb], 1);
                int64_t d = ob + nsurv + q;
                if (d < cap) stg[d] = P4<T>{px, pu, pv, pw};
                else atomicOr(err, ERR_CAPACITY);
                // moments of the particle as stored, so Psi_t is unchanged exactly
                double du = pu, dv = pv, dw = pw;
                ss[0] += 1.0; ss[1] += du; ss[2] += dv; ss[3] += dw;
                ss[4] += 0.5 * (du * du + dv * dv + dw * dw);
            }
            block_sum<5>(ss, red);
        }
        __syncthreads();
        for (int t = threadIdx.x; t < NBIN; t += blockDim.x)
            if (dh[t]) cl.hist[(int64_t)g * NBIN + t] += dh[t];
        if (threadIdx.x == 0) {
            const int32_t nabs = (int32_t)(e - b) - nsurv;
            if (nabs > 0)
#pragma unroll
                for (int i = 0; i < 5; ++i) cl.psi_w[(int64_t)g * 5 + i] += c.fac * sa[i];
            if (nnew > 0)
#pragma unroll
                for (int i = 0; i < 5; ++i) cl.psi_w[(int64_t)g * 5 + i] -= c.fac * ss[i];
            cl.d_abs[g] = nabs;
            cl.d_new[g] = nnew;
        }
    }
}

// ---------------------------------------------------------------------------
// 4. NTC / VHS collisions (Appendix A).
//
// The candidates of all cells form one list in (cell, q) order; cbase[g] is
// the first candidate of cell g.  The list is cut into work items of S
// candidates: item w takes every cell whose first candidate lies in
// [w S, (w+1) S), so a cell belongs to exactly one item and one wave runs all
// of its candidates, 64 at a time (one per lane, several cells per chunk).
//
// Within a chunk, lane L must see particle p as the candidates before it left
// it.  An LDS table of lane masks hashed by (cell, particle) finds, for each of
// L's two particles, the last earlier lane that touched it; lanes run in rounds
// once those (at most two) lanes have run, and take the particle's velocity
// from that lane's LDS slot instead of memory.  Chunks of one item run in
// order with the earlier chunks' stores visible, so the result is the
// candidates' sequential result.
// ---------------------------------------------------------------------------
constexpr int COLL_HBITS = 8;
constexpr int COLL_WPB = 4;      // waves per block

// item_cell[w] = first cell of item w; d_items = {number of items, S}
__global__ void __launch_bounds__(256) k_items(const int64_t *__restrict__ cbase, int G, int32_t *item_cell,
                                               int64_t *d_items, int64_t items_cap)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g > G) return;
    const int64_t total = cbase[G];
    int64_t S = (total + items_cap - 2) / (items_cap - 1);   // at most items_cap - 1 items
    S = S < WAVE ? WAVE : (S + WAVE - 1) / WAVE * WAVE;
    const int64_t nitems = (total + S - 1) / S;
    if (g == 0) {
        d_items[0] = nitems;
        d_items[1] = S;
        if (nitems > 0) item_cell[0] = 0;
        return;
    }
    // items w >= 1 with cbase[g-1] < w S <= cbase[g] start at cell g
    const int64_t lo = cbase[g - 1], hi = cbase[g];
    for (int64_t w = lo / S + 1; w * S <= hi && w < nitems; ++w) item_cell[w] = g;
}

__device__ __forceinline__ uint32_t coll_slot(int g, uint32_t i)
{
    return ((uint32_t)g * 0x9E3779B1u ^ i * 0x85EBCA77u) * 0xC2B2AE3Du >> (32 - COLL_HBITS);
}

template <typename T>
__global__ void __launch_bounds__(256) k_collide(const DCase *__restrict__ cases, Cells cl, P4<T> *src,
                                                 P4<T> *stg, const uint32_t *__restrict__ d_step, int G,
                                                 int64_t cap, int32_t *err, const int32_t *__restrict__ item_cell,
                                                 const int64_t *__restrict__ d_items, int by_cell, Inj<T> inj,
                                                 int64_t *d_ninj, int nrk)
{
    // the first nrk blocks rank the step's entrants, two per case (the
    // collisions neither read nor write what they touch)
    if ((int)blockIdx.x < nrk) {
        const int kk = (int)blockIdx.x >> 1;
        inject_rank_block<T, WAVE * COLL_WPB>(cases[kk], cl, inj, d_ninj, err, kk, (int)blockIdx.x & 1);
        return;
    }
    const int bid = (int)blockIdx.x - nrk, nbk = (int)gridDim.x - nrk;
    __shared__ uint64_t hmask[COLL_WPB][1 << COLL_HBITS];
    __shared__ T fwd[COLL_WPB][6][WAVE];     // (u,v,w) of particle i, then of j, per lane
    const int wv = wave_id(), lane = lane_id();
    const uint32_t step = *d_step;
    for (int t = lane; t < (1 << COLL_HBITS); t += WAVE) hmask[wv][t] = 0ull;
    lds_fence();
    const uint64_t lt = lanemask_lt();
    // One chunk: lane l runs candidate q of cell g (act false: no candidate).
    // The cell's constants (CellRef) and the candidate's pair, words and records
    // (Cand) come first; run finds each lane's predecessors in the chunk, runs
    // the candidates in dependency rounds and adds the per-cell results.  more:
    // another chunk of the same work follows and reads what this one stored.
    struct CellRef {
        P4<T> *pr;
        int lc, k;
        double cm, aexp;
        // FP32: the case's flight constants in registers for the bin moves
        // inside the rounds (FP64 reads them from the case: its registers are
        // worth more than the loads)
        FlightK<T> fk;
    };
    struct Cand {
        uint32_t i, j, w2, w3, w4;
        T xi, ui, vi, wi, xj, uj, vj, wj;
    };
    // pair and words of candidate q of a cell with N >= 2 particles at pr, and
    // the two records
    auto pair = [&](const DCase &c, int lc, uint32_t q, int32_t N, P4<T> *pr, Cand &d) {
        const U4 ra = draw(c, step, (uint32_t)lc, q, TAG_PAIR, 0);
        const U4 rb = draw(c, step, (uint32_t)lc, q, TAG_PAIR, 1);
        const uint64_t r0 = ((uint64_t)ra.a << 32) | ra.b;
        const uint64_t r1 = ((uint64_t)ra.c << 32) | ra.d;
        d.i = (uint32_t)mulhi64(r0, (uint64_t)N);
        d.j = (uint32_t)mulhi64(r1, (uint64_t)(N - 1));
        if (d.j >= d.i) d.j += 1;
        d.w2 = rb.a; d.w3 = rb.b; d.w4 = rb.c;
        const P4<T> x = pr[d.i], y = pr[d.j];
        d.xi = x.x; d.ui = x.u; d.vi = x.v; d.wi = x.w;
        d.xj = y.x; d.uj = y.u; d.vj = y.v; d.wj = y.w;
    };
    auto run = [&](int g, bool act, bool more, const CellRef &cr, const Cand &d) {
        const uint32_t i = d.i, j = d.j;
        T ui = d.ui, vi = d.vi, wi = d.wi, uj = d.uj, vj = d.vj, wj = d.wj;
        const T xi = d.xi, xj = d.xj;
        if (!act) g = -1;
        // last earlier lane touching each of this lane's particles
        const uint32_t si = coll_slot(g, i), sj = coll_slot(g, j);
        if (act) {
            atomicOr(&hmask[wv][si], 1ull << lane);
            atomicOr(&hmask[wv][sj], 1ull << lane);
        }
        lds_fence();
        uint64_t ci = act ? (hmask[wv][si] & lt) : 0ull, cj = act ? (hmask[wv][sj] & lt) : 0ull;
        lds_fence();
        if (act) { hmask[wv][si] = 0ull; hmask[wv][sj] = 0ull; }
        int pi = -1, pj = -1, oi = 0, oj = 0;
        while (__ballot(ci != 0ull || cj != 0ull)) {
            const int li = ci ? 63 - __clzll((long long)ci) : lane;
            const int lj = cj ? 63 - __clzll((long long)cj) : lane;
            const int gli = __shfl(g, li, WAVE), glj = __shfl(g, lj, WAVE);
            const uint32_t ii = __shfl(i, li, WAVE), ji = __shfl(j, li, WAVE);
            const uint32_t ij = __shfl(i, lj, WAVE), jj = __shfl(j, lj, WAVE);
            if (ci) {
                if (gli == g && (ii == i || ji == i)) { pi = li; oi = ii == i ? 0 : 3; ci = 0ull; }
                else ci &= ~(1ull << li);
            }
            if (cj) {
                if (glj == g && (ij == j || jj == j)) { pj = lj; oj = ij == j ? 0 : 3; cj = 0ull; }
                else cj &= ~(1ull << lj);
            }
        }
        const uint64_t dep = (pi >= 0 ? 1ull << pi : 0ull) | (pj >= 0 ? 1ull << pj : 0ull);
        double seen = 0.0;
        int acc = 0;
        uint64_t done = ~__ballot(act);
        while (done != ~0ull) {
            const bool ready = !((done >> lane) & 1ull) && (dep & ~done) == 0ull;
            if (ready) {
                if (pi >= 0) { ui = fwd[wv][oi][pi]; vi = fwd[wv][oi + 1][pi]; wi = fwd[wv][oi + 2][pi]; }
                if (pj >= 0) { uj = fwd[wv][oj][pj]; vj = fwd[wv][oj + 1][pj]; wj = fwd[wv][oj + 2][pj]; }
                const T ui0 = ui, uj0 = uj;
                if (collide_vals<T>(ui, vi, wi, uj, vj, wj, cr.cm, cr.aexp, d.w2, d.w3, d.w4, seen)) {
                    acc = 1;
                    cr.pr[i] = P4<T>{xi, ui, vi, wi};
                    cr.pr[j] = P4<T>{xj, uj, vj, wj};
                    // move the pair between destination bins of this step's histogram
                    int32_t *hg = cl.hist + (int64_t)g * NBIN;
                    int a0, a1, b0, b1;
                    auto bins = [&](const auto &kc) {
                        a0 = flight_bin<T>(kc, cr.lc, xi, ui0);
                        a1 = flight_bin<T>(kc, cr.lc, xi, ui);
                        b0 = flight_bin<T>(kc, cr.lc, xj, uj0);
                        b1 = flight_bin<T>(kc, cr.lc, xj, uj);
                    };
                    if constexpr (std::is_same<T, float>::value) bins(cr.fk);
                    else bins(cases[cr.k]);
                    if (a0 != a1) {
                        if (a0 >= 0) atomicSub(&hg[a0], 1);
                        if (a1 >= 0) atomicAdd(&hg[a1], 1);
                    }
                    if (b0 != b1) {
                        if (b0 >= 0) atomicSub(&hg[b0], 1);
                        if (b1 >= 0) atomicAdd(&hg[b1], 1);
                    }
                }
                fwd[wv][0][lane] = ui; fwd[wv][1][lane] = vi; fwd[wv][2][lane] = wi;
                fwd[wv][3][lane] = uj; fwd[wv][4][lane] = vj; fwd[wv][5][lane] = wj;
            }
            lds_fence();
            done |= __ballot(ready);
        }
        // per-cell results: accepted collisions (segmented sum over the chunk's
        // lanes of one cell), largest relative speed, out-of-window flag
        int sacc = acc;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const int t = __shfl_up(sacc, o, WAVE);
            const int gu = __shfl_up(g, o, WAVE);
            if (lane >= o && gu == g) sacc += t;
        }
        const int gd = __shfl_down(g, 1, WAVE);
        if (g >= 0 && (lane == WAVE - 1 || gd != g) && sacc > 0) atomicAdd(&cl.d_coll[g], sacc);
        if (act && seen > cr.cm)
            atomicMax((unsigned long long *)&cl.cr_seen[g], (unsigned long long)__double_as_longlong(seen));
        // the next chunk of this work reads what this one stored
        if (more) __threadfence_block();
    };
    if (by_cell) {
        // a wave per cell, cells in visiting order (few cells with many
        // candidates); the cell's constants are read once, not per chunk
        for (int gi = bid * COLL_WPB + wv; gi < G; gi += nbk * COLL_WPB) {
            const int g = __builtin_amdgcn_readfirstlane(cl.order[gi]);
            const int32_t M = __builtin_amdgcn_readfirstlane(cl.ncand_w[g]);
            if (M <= 0) continue;
            const int32_t N = __builtin_amdgcn_readfirstlane(cl.n_int[g]);
            const int64_t sb = cl.seg[g];
            if (sb + N > cap) continue;   // capacity overflow, already reported
            CellRef cr;
            cr.k = __builtin_amdgcn_readfirstlane(cl.cell_case[g]);
            const DCase &c = cases[cr.k];
            cr.lc = g - c.cell_base;
            cr.pr = (cl.seg_stg[g] ? stg : src) + sb;
            cr.cm = cl.cr_max[g];
            cr.aexp = 1.0 - 2.0 * c.ups;
            if constexpr (std::is_same<T, float>::value) cr.fk = FlightK<T>(c);
            for (int32_t q0 = 0; q0 < M; q0 += WAVE) {
                const bool act = q0 + lane < M;
                Cand d{};
                if (act) pair(c, cr.lc, (uint32_t)(q0 + lane), N, cr.pr, d);
                run(g, act, q0 + WAVE < M, cr, d);
            }
        }
        return;
    }
    // work items of whole cells from the scanned candidate list
    const int64_t nitems = d_items[0];
    for (int64_t it = (int64_t)bid * COLL_WPB + wv; it < nitems; it += (int64_t)nbk * COLL_WPB) {
        const int ga = item_cell[it];
        const int gb = it + 1 < nitems ? item_cell[it + 1] : G;
        const int64_t qend = cl.cbase[gb];
        int gcur = ga;
        for (int64_t Q0 = cl.cbase[ga]; Q0 < qend; Q0 += WAVE) {
            const int64_t Q = Q0 + lane;
            bool act = Q < qend;
            // cell of candidate Q: gcur + number of cell starts <= Q after gcur
            int g = -1;
            int64_t gstart = 0;
            {
                bool need = act;
                int gw = gcur;
                int64_t prev = cl.cbase[gw];
                while (__ballot(need)) {
                    const int gl = gw + 1 + lane;
                    const int64_t cb = gl <= gb ? cl.cbase[gl] : INT64_MAX;
                    int n = 0;
#pragma unroll
                    for (int st2 = 32; st2 >= 1; st2 >>= 1) {
                        const int64_t v = __shfl(cb, n + st2 - 1, WAVE);
                        if (v <= Q) n += st2;
                    }
                    const int64_t last = readlane64(cb, WAVE - 1);
                    if (n == WAVE - 1 && last <= Q) n = WAVE;
                    const int64_t sprev = __shfl(cb, n > 0 ? n - 1 : 0, WAVE);
                    if (need && n < WAVE) {
                        g = gw + n;
                        gstart = n > 0 ? sprev : prev;
                        need = false;
                    }
                    prev = last;
                    gw += WAVE;
                }
            }
            const int gnext = __builtin_amdgcn_readlane(g, WAVE - 1);
            // the lane's cell and candidate (a cell beyond the capacity was
            // reported already)
            CellRef cr{nullptr, 0, 0, 1.0, 0.0, FlightK<T>()};
            Cand d{};
            if (act) {
                const int32_t N = cl.n_int[g];
                const int64_t sb = cl.seg[g];
                cr.k = cl.cell_case[g];
                const DCase &c = cases[cr.k];
                cr.lc = g - c.cell_base;
                if (sb + N > cap) {
                    act = false;
                } else {
                    cr.pr = (cl.seg_stg[g] ? stg : src) + sb;
                    cr.cm = cl.cr_max[g];
                    cr.aexp = 1.0 - 2.0 * c.ups;
                    if constexpr (std::is_same<T, float>::value) cr.fk = FlightK<T>(c);
                    pair(c, cr.lc, (uint32_t)(Q - gstart), N, cr.pr, d);
                }
            }
            run(g, act, Q0 + WAVE < qend, cr, d);
            gcur = gnext;
        }
    }
}

// ---------------------------------------------------------------------------
// 4b. NTC / VHS collisions of cells with many particles and candidates: one
// block per cell, BigCfg<T>::B candidates at a time (one per thread).
//
// For each of its particles a candidate needs the last earlier candidate of the
// chunk that touched it: an LDS hash table keyed exactly by particle index
// records up to BIG_LIST candidates per particle, and the largest one below the
// candidate's own index is its predecessor.  Candidates without predecessors
// (nearly all of a chunk in a big cell) run at once.  The others wait for their
// predecessors and take velocities from the predecessors' LDS slots: they are
// staged in LDS, BIG_DEPCAP at a time in candidate order, and run by one wave in
// wave-level rounds, so that the collision arithmetic of a chunk is issued about
// once per wave instead of once per round.  A particle drawn by more than
// BIG_LIST candidates of one chunk sends that chunk through a serial path: with
// 8 per list, about 4e-8 of the chunks of a cell of 1800 particles (one chunk
// in 40 with 4 per list, a serial chunk then costing as much as the rest).
//
// The random particle reads dominate: the block works on the cell's records in
// place (one cache line per access), two blocks share a compute unit, and the
// barriers inside a chunk order LDS only, so that the stores of the candidates
// that run first do not hold up the waiting ones.  Histogram moves of accepted
// collisions are summed in LDS and added once per cell.
// ---------------------------------------------------------------------------
constexpr int BIG_LIST = 8;
constexpr int BIG_DEPCAP = 64;

// B threads (candidates per chunk: 256, 512 or 1024), 2^HBITS hash slots (twice
// the particles a chunk draws)
template <int B>
struct BigCfg {
    static constexpr int HBITS = B == 256 ? 10 : (B == 512 ? 11 : 12);
    static constexpr int SLOTS = 1 << HBITS;
    static_assert(SLOTS == 4 * B, "hash slots: twice the 2B particles a chunk draws");
};


template <int HBITS>
__device__ __forceinline__ int big_insert(uint32_t *hkey, int *hcnt, uint16_t (*hlst)[BIG_LIST], uint32_t p,
                                          int t, int *ovf)
{
    uint32_t h = (p * 0x9E3779B1u) >> (32 - HBITS);
    while (true) {
        const uint32_t prev = atomicCAS(&hkey[h], 0xffffffffu, p);
        if (prev == 0xffffffffu || prev == p) break;
        h = (h + 1) & ((1u << HBITS) - 1);
    }
    const int k = atomicAdd(&hcnt[h], 1);
    if (k < BIG_LIST) hlst[h][k] = (uint16_t)t;
    else *ovf = 1;
    return (int)h;
}

// last candidate before t that touched the particle of slot s: its index, and
// 0 or 3 for its first or second particle
__device__ __forceinline__ void big_pred(const int *hcnt, const uint16_t (*hlst)[BIG_LIST], const uint32_t *ci,
                                         int s, uint32_t p, int t, int &pl, int &po)
{
    const int c = min(hcnt[s], BIG_LIST);
    int best = -1;
    for (int k = 0; k < c; ++k) {
        const int l = hlst[s][k];
        if (l < t && l > best) best = l;
    }
    pl = best;
    po = (best >= 0 && ci[best] != p) ? 3 : 0;
}

// particles of candidate q (its first draw) and its three uniforms (the second)
__device__ __forceinline__ void big_idx(const CaseK &c, uint32_t step, int lc, uint32_t q, int32_t N,
                                        uint32_t &i, uint32_t &j)
{
    const U4 ra = draw(c, step, (uint32_t)lc, q, TAG_PAIR, 0);
    const uint64_t r0 = ((uint64_t)ra.a << 32) | ra.b;
    const uint64_t r1 = ((uint64_t)ra.c << 32) | ra.d;
    i = (uint32_t)mulhi64(r0, (uint64_t)N);
    j = (uint32_t)mulhi64(r1, (uint64_t)(N - 1));
    if (j >= i) j += 1;
}

__device__ __forceinline__ void big_uni(const CaseK &c, uint32_t step, int lc, uint32_t q, uint32_t &w2,
                                        uint32_t &w3, uint32_t &w4)
{
    const U4 rb = draw(c, step, (uint32_t)lc, q, TAG_PAIR, 1);
    w2 = rb.a; w3 = rb.b; w4 = rb.c;
}

// move the pair between destination bins of this step's histogram (summed in hd)
template <typename T>
__device__ __forceinline__ void big_bins(const CaseK &c, int lc, T xi, T ui0, T ui, T xj, T uj0, T uj, int *hd)
{
    const int a0 = flight_bin<T>(c, lc, xi, ui0), a1 = flight_bin<T>(c, lc, xi, ui);
    const int b0 = flight_bin<T>(c, lc, xj, uj0), b1 = flight_bin<T>(c, lc, xj, uj);
    if (a0 != a1) {
        if (a0 >= 0) atomicSub(&hd[a0], 1);
        if (a1 >= 0) atomicAdd(&hd[a1], 1);
    }
    if (b0 != b1) {
        if (b0 >= 0) atomicSub(&hd[b0], 1);
        if (b1 >= 0) atomicAdd(&hd[b1], 1);
    }
}

// a candidate that waits for predecessors, staged for the wave that runs it
template <typename T>
struct BigDep {
    T x[2][BIG_DEPCAP], v[6][BIG_DEPCAP];
    uint32_t u[3][BIG_DEPCAP], p[2][BIG_DEPCAP];
    int t[BIG_DEPCAP], pred[2][BIG_DEPCAP];   // predecessor * 4 + (0 or 3), or -1
};

// 256 FP64 threads: registers capped for three waves per SIMD (three blocks per
// compute unit, which their LDS allows)
template <typename T, int B>
__global__ void __launch_bounds__(B, (sizeof(T) == 8 && B == 256) ? 3 : 1) k_collide_big(const DCase *__restrict__ cases, Cells cl,
                                                   P4<T> *src, P4<T> *stg,
                                                   const uint32_t *__restrict__ d_step, int64_t cap)
{
    constexpr int NW = B / WAVE;
    constexpr int SLOTS = BigCfg<B>::SLOTS;
    constexpr int HB = BigCfg<B>::HBITS;
    __shared__ uint32_t hkey[SLOTS];
    __shared__ int hcnt[SLOTS];
    __shared__ uint16_t hlst[SLOTS][BIG_LIST];
    __shared__ uint32_t ci[B];
    __shared__ int done[B];
    __shared__ T fwd[6][B];
    __shared__ BigDep<T> dq;
    __shared__ int hd[NBIN];
    __shared__ double redd[NW];
    __shared__ int redi[NW];
    __shared__ int ovf[2];           // by chunk parity
    __shared__ int wdep[NW];         // per-wave counts of waiting candidates
    const int t = threadIdx.x, lane = lane_id(), wv = wave_id();
    const int nbig = *cl.nbig;
    if ((int)blockIdx.x >= nbig) return;   // no cell for this block (often none at all)
    const uint32_t step = *d_step;
    for (int s = t; s < SLOTS; s += B) { hkey[s] = 0xffffffffu; hcnt[s] = 0; }
    for (int e = blockIdx.x; e < nbig; e += gridDim.x) {
        const int g = cl.big_list[e];
        const int k = cl.cell_case[g];
        const DCase &c = cases[k];
        const CaseK ck(c);
        const int lc = g - c.cell_base;
        const int32_t N = cl.n_int[g];
        const int64_t M = cl.d_cand[g];
        int64_t sb;
        P4<T> *sg = segment(cl, g, src, stg, sb);
        if (sb + N > cap) continue;   // capacity overflow, already reported (block-uniform)
        P4<T> *P = sg + sb;           // the cell's records
        const double cm = cl.cr_max[g];
        const double aexp = 1.0 - 2.0 * c.ups;
        if (t < NBIN) hd[t] = 0;
        if (t < 2) ovf[t] = 0;
        __syncthreads();
        double seen = 0.0;
        int acc = 0;
        // candidate tt on particles a and b with their current records; its
        // outgoing velocities go to its LDS slot
        auto run = [&](int tt, uint32_t a, uint32_t b, T xa, T ua, T va, T wa, T xb, T ub, T vb, T wb,
                       uint32_t v2, uint32_t v3, uint32_t v4) {
            const T ua0 = ua, ub0 = ub;
            if (collide_vals<T>(ua, va, wa, ub, vb, wb, cm, aexp, v2, v3, v4, seen)) {
                ++acc;
                P[a] = P4<T>{xa, ua, va, wa};
                P[b] = P4<T>{xb, ub, vb, wb};
                big_bins<T>(ck, lc, xa, ua0, ua, xb, ub0, ub, hd);
            }
            fwd[0][tt] = ua; fwd[1][tt] = va; fwd[2][tt] = wa;
            fwd[3][tt] = ub; fwd[4][tt] = vb; fwd[5][tt] = wb;
            done[tt] = 1;
        };
        int par = 0;
        for (int64_t q0 = 0; q0 < M; q0 += B, par ^= 1) {
            const int64_t q = q0 + t;
            const bool act = q < M;
            uint32_t i = 0, j = 0;
            T xi = 0, ui = 0, vi = 0, wi = 0, xj = 0, uj = 0, vj = 0, wj = 0;
            int si = 0, sj = 0;
            if (act) {
                big_idx(ck, step, lc, (uint32_t)q, N, i, j);
                const P4<T> a = P[i], bq = P[j];
                xi = a.x; ui = a.u; vi = a.v; wi = a.w;
                xj = bq.x; uj = bq.u; vj = bq.v; wj = bq.w;
                si = big_insert<HB>(hkey, hcnt, hlst, i, t, &ovf[par]);
                sj = big_insert<HB>(hkey, hcnt, hlst, j, t, &ovf[par]);
            }
            ci[t] = i;
            done[t] = act ? 0 : 1;
            lds_barrier();
            const bool serial = ovf[par] != 0;
            // the next chunk's flag: its last readers were in the previous chunk
            if (t == 0) ovf[par ^ 1] = 0;
            if (serial) {
                // serial path: the chunk's candidates one after another in thread 0,
                // reading and writing the particles in memory
                if (t == 0) {
                    const int nq = (int)min((int64_t)B, M - q0);
                    for (int l = 0; l < nq; ++l) {
                        uint32_t a, bq, v2, v3, v4;
                        big_idx(ck, step, lc, (uint32_t)(q0 + l), N, a, bq);
                        big_uni(ck, step, lc, (uint32_t)(q0 + l), v2, v3, v4);
                        P4<T> ra = P[a], rb = P[bq];
                        const T ua0 = ra.u, ub0 = rb.u;
                        if (collide_vals<T>(ra.u, ra.v, ra.w, rb.u, rb.v, rb.w, cm, aexp, v2, v3, v4, seen)) {
                            ++acc;
                            P[a] = ra;
                            P[bq] = rb;
                            big_bins<T>(ck, lc, ra.x, ua0, ra.u, rb.x, ub0, rb.u, hd);
                        }
                    }
                }
            } else {
                uint32_t u2 = 0, u3 = 0, u4 = 0;
                int pi = -1, pj = -1, oi = 0, oj = 0;
                if (act) {
                    big_uni(ck, step, lc, (uint32_t)q, u2, u3, u4);
                    big_pred(hcnt, hlst, ci, si, i, t, pi, oi);
                    big_pred(hcnt, hlst, ci, sj, j, t, pj, oj);
                }
                const bool waits = pi >= 0 || pj >= 0;
                // no predecessor: the records read above are current
                if (act && !waits) run(t, i, j, xi, ui, vi, wi, xj, uj, vj, wj, u2, u3, u4);
                const uint64_t wb = __ballot(act && waits);
                if (lane == 0) wdep[wv] = __popcll(wb);
                lds_barrier();
                int ndep = 0, before = 0;
#pragma unroll
                for (int w2 = 0; w2 < NW; ++w2) {
                    const int n2 = wdep[w2];
                    before += w2 < wv ? n2 : 0;
                    ndep += n2;
                }
                // the waiting candidates, BIG_DEPCAP at a time in candidate order, are
                // staged in LDS and run by wave 0 (their predecessors come earlier)
                for (int b0 = 0; b0 < ndep; b0 += BIG_DEPCAP) {
                    if (b0 > 0) lds_barrier();   // wave 0 is done with the previous batch
                    const int d = before + __popcll(wb & lanemask_lt()) - b0;
                    if (act && waits && d >= 0 && d < BIG_DEPCAP) {
                        dq.x[0][d] = xi; dq.x[1][d] = xj;
                        dq.v[0][d] = ui; dq.v[1][d] = vi; dq.v[2][d] = wi;
                        dq.v[3][d] = uj; dq.v[4][d] = vj; dq.v[5][d] = wj;
                        dq.u[0][d] = u2; dq.u[1][d] = u3; dq.u[2][d] = u4;
                        dq.p[0][d] = i; dq.p[1][d] = j;
                        dq.t[d] = t;
                        dq.pred[0][d] = pi < 0 ? -1 : pi * 4 + oi;
                        dq.pred[1][d] = pj < 0 ? -1 : pj * 4 + oj;
                    }
                    lds_barrier();
                    if (wv == 0) {
                        bool mine = lane < min(BIG_DEPCAP, ndep - b0);
                        const int e2 = mine ? lane : 0;
                        const int ti = dq.t[e2], ri = dq.pred[0][e2], rj = dq.pred[1][e2];
                        T a0 = dq.v[0][e2], a1 = dq.v[1][e2], a2 = dq.v[2][e2];
                        T c0 = dq.v[3][e2], c1 = dq.v[4][e2], c2 = dq.v[5][e2];
                        // wave-level rounds: LDS operations of one wave complete in order
                        while (true) {
                            const bool ready = mine && (ri < 0 || done[ri >> 2]) && (rj < 0 || done[rj >> 2]);
                            if (ready) {
                                if (ri >= 0) {
                                    const int l = ri >> 2, o = ri & 3;
                                    a0 = fwd[o][l]; a1 = fwd[o + 1][l]; a2 = fwd[o + 2][l];
                                }
                                if (rj >= 0) {
                                    const int l = rj >> 2, o = rj & 3;
                                    c0 = fwd[o][l]; c1 = fwd[o + 1][l]; c2 = fwd[o + 2][l];
                                }
                                run(ti, dq.p[0][e2], dq.p[1][e2], dq.x[0][e2], a0, a1, a2, dq.x[1][e2], c0, c1, c2,
                                    dq.u[0][e2], dq.u[1][e2], dq.u[2][e2]);
                                mine = false;
                            }
                            lds_fence();
                            if (__ballot(mine) == 0) break;
                        }
                    }
                }
            }
            // empty the table for the next chunk; make this chunk's stores visible to it
            if (act) {
                hkey[si] = 0xffffffffu; hcnt[si] = 0;
                hkey[sj] = 0xffffffffu; hcnt[sj] = 0;
            }
            __threadfence_block();
            __syncthreads();
        }
        // per-cell results
        int a = wave_sum_i(acc);
        double m = wave_max(seen);
        if (lane == 0) { redi[wv] = a; redd[wv] = m; }
        __syncthreads();
        if (t == 0) {
            int sa = 0;
            double sm = 0.0;
            for (int w2 = 0; w2 < NW; ++w2) { sa += redi[w2]; sm = fmax(sm, redd[w2]); }
            cl.d_coll[g] = sa;
            if (sm > cm) cl.cr_seen[g] = (uint64_t)__double_as_longlong(sm);
        }
        if (t < NBIN && hd[t]) cl.hist[(int64_t)g * NBIN + t] += hd[t];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 5a. Reservoir injection candidates, in parallel over (case, side, slot):
// a particle sampled in the ghost slab beyond a reservoir side, streamed over
// dt; it enters when it ends inside the domain.  Side `side` of case k, by
// wave wi of the nwv waves that take this side: chunk ci of INJ_CH slots goes
// to wave ci mod nwv, which compacts its entrants, in slot order, to the
// chunk's front.  (Run by extra blocks of the cell-state launch: the
// candidates depend on the step and the case alone.)
// ---------------------------------------------------------------------------
template <typename T>
__device__ void inject_gen_wave(const DCase &c, int k, int side, const Inj<T> &inj, uint32_t step, int32_t *err,
                                int wi, int nwv)
{
    const int lane = lane_id();
    if ((side == 0 ? c.bc_lo : c.bc_hi) != 0) {
        if (wi == 0 && lane == 0) inj.ncand[2 * k + side] = 0;
        return;
    }
    const double rho = side == 0 ? c.rho_L : c.rho_R;
    const double U = side == 0 ? c.u_L : c.u_R;
    const double Ts = side == 0 ? c.T_L : c.T_R;
    const double tau = viscosity(c, Ts) / (rho * c.R * Ts);
    const double Ps = absorb_fraction(c.law, c.dt, tau);
    const double Lg = c.dt * (fabs(U) + 8.0 * sqrt(c.R * Ts));
    U4 r = draw(c, step, (uint32_t)side, 0, TAG_ICNT, 0);
    double nf = floor((1.0 - Ps) * rho * Lg / c.m_p + u01(r.a));
    int64_t ng = (int64_t)fmin(nf, 4.0e9);
    if (ng > c.cand_cap[side]) {
        if (wi == 0 && lane == 0) atomicOr(err, ERR_CAPACITY);
        ng = c.cand_cap[side];
    }
    if (wi == 0 && lane == 0) inj.ncand[2 * k + side] = ng;
    const int64_t cb = c.cand_base[side];
    const Maxwell<T> mw(U, 0.0, 0.0, Ts, c.R);
    for (int64_t ci = wi; ci * INJ_CH < ng; ci += nwv) {
        const int64_t q = ci * INJ_CH + lane;
        int dest = -1;
        T px = 0, pu = 0, pv = 0, pw = 0;
        if (q < ng) {
            U4 a = draw(c, step, (uint32_t)side, (uint32_t)q, TAG_IVEL, 0);
            U4 bb = draw(c, step, (uint32_t)side, (uint32_t)q, TAG_IVEL, 1);
            const uint32_t w6[6] = {a.b, a.c, a.d, bb.a, bb.b, bb.c};
            T xi[3];
            mw.sample(w6, xi);
            if constexpr (std::is_same<T, double>::value) {
                double x = side == 0 ? c.x_lo - u01(a.a) * Lg : c.x_hi + u01(a.a) * Lg;
                double u = xi[0];
                x = x + u * c.dt;
                dest = bc_cell_abs(c, x, u);
                px = x; pu = u;
            } else {
                float u = xi[0];
                const float lgc = (float)(Lg / c.dx);
                const float X0 = side == 0 ? -u01f(a.a) * lgc : u01f(a.a) * lgc;
                const float X = X0 + u * c.dtdx_f;
                const float fl = floorf(X);
                float s = 0.0f;
                dest = (fabsf(X) < 1.0e9f) ? bc_cell_rel(c, (side == 0 ? 0 : c.ncells) + (int)fl, X - fl, u, s) : -1;
                px = s; pu = u;
            }
            pv = xi[1]; pw = xi[2];
        }
        const bool ent = dest >= 0;
        const uint64_t m = __ballot(ent);
        if (ent) {
            const int64_t sl = cb + ci * INJ_CH + lane_rank_lt(m);
            inj.cx[sl] = px; inj.cu[sl] = pu; inj.cv[sl] = pv; inj.cw[sl] = pw;
            inj.cdest[sl] = dest;
        }
        if (lane == 0) inj.cchunk[c.chunk_base[side] + ci] = __popcll(m);
    }
}

// Injection destination window: cells within KWIN of either end of the case.
__device__ __forceinline__ int inj_slot(int d, int C)
{
    if (C <= NBI) return d;
    if (d <= KWIN) return d;
    if (d >= C - 1 - KWIN) return KWIN + 1 + (C - 1 - d);
    return -1;
}
__device__ __forceinline__ int inj_cell(int slot, int C)
{
    if (C <= NBI) return slot < C ? slot : -1;
    if (slot <= KWIN) return slot;
    return C - 1 - (slot - KWIN - 1);
}

// Stable rank of per-thread keys in [0,NB) within one chunk of a block (one key
// per thread, in thread order), continuing the running counts binbase[];
// returns the rank, or -1 for a key < 0.  wcnt holds a row of NB ints per wave,
// zero on entry and on exit.
template <int NB>
__device__ __forceinline__ int block_stable_rank(int key, int *binbase, int (*wcnt)[NB])
{
    const int lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
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
    int r = -1;
    if (key >= 0) {
        r = binbase[key] + my;
        for (int w2 = 0; w2 < w; ++w2) r += wcnt[w2][key];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NB; t += blockDim.x) {
        int s = 0;
        for (int w2 = 0; w2 < nw; ++w2) { s += wcnt[w2][t]; wcnt[w2][t] = 0; }
        binbase[t] += s;
    }
    __syncthreads();
    return r;
}

// 5b. Entrants in (side, slot) order, with their rank among entrants of the
// same destination cell.  Only the compacted entrants of each candidate chunk
// are visited: a prefix over the chunk counts maps the e-th entrant of a side to
// its chunk.  A case of more than NBI cells has its sides ranked by two blocks:
// each side's entrants then land in that side's own bins (one landing in the
// other side's bins has crossed more than the sort window and is reported), and
// side 1's entrants follow side 0's.  An entrant that is reported keeps its place
// with destination -1 and is not scattered.  Block y of case k, RK_THREADS
// threads: the first blocks of the collision launch (the ranks are needed
// only by the scatter, and the collisions do not touch them), or, when a side
// may have many entrants, a kernel of its own with 1024 threads a block (a
// quarter of the rounds).
constexpr int RK_THREADS = 256;
static_assert(RK_THREADS == WAVE * COLL_WPB, "the entrants are ranked by blocks of the collision launch");
template <typename T, int NT>
__device__ void inject_rank_block(const DCase &c, const Cells &cl, const Inj<T> &inj, int64_t *d_ninj, int32_t *err,
                                  int k, int y)
{
    constexpr int RK_THREADS = NT;
    constexpr int MAXCH = 1024;                  // chunks per pass
    constexpr int RK_IT = MAXCH / RK_THREADS;    // chunk counts per thread in the prefix
    constexpr int NW = RK_THREADS / WAVE;
    __shared__ int binbase[NBI];
    __shared__ int wcnt[NW][NBI];
    __shared__ int pref[MAXCH + 1];
    __shared__ int red[NW];
    __shared__ int64_t lds[NW];
    const int C = c.ncells;
    const int lane = lane_id();
    const bool split = C > NBI;
    if (!split && y == 1) return;
    const int s0 = split ? y : 0, s1 = split ? s0 + 1 : 2;
    for (int t = threadIdx.x; t < NBI; t += RK_THREADS) binbase[t] = 0;
    for (int t = threadIdx.x; t < NW * NBI; t += RK_THREADS) (&wcnt[0][0])[t] = 0;
    int64_t count = 0;
    if (s0 == 1) {
        // side 1 follows the entrants of side 0: the sum of its chunk counts
        const int64_t nch0 = (inj.ncand[2 * k] + INJ_CH - 1) / INJ_CH;
        int sum = 0;
        for (int64_t i = threadIdx.x; i < nch0; i += RK_THREADS) sum += inj.cchunk[c.chunk_base[0] + i];
        sum = wave_sum_i(sum);
        if (lane == 0) red[wave_id()] = sum;
        __syncthreads();
        for (int w2 = 0; w2 < NW; ++w2) count += red[w2];
    }
    __syncthreads();
    for (int side = s0; side < s1; ++side) {
        const int64_t n = inj.ncand[2 * k + side];
        const int64_t cb = c.cand_base[side];
        const int64_t nch = (n + INJ_CH - 1) / INJ_CH;
        int64_t nside = 0;
        for (int64_t ch0 = 0; ch0 < nch; ch0 += MAXCH) {
            const int nb = (int)min((int64_t)MAXCH, nch - ch0);
            // exclusive prefix of the chunk counts: a thread loads RK_IT
            // consecutive counts at once, then one block scan
            int v[RK_IT];
            int sv = 0;
#pragma unroll
            for (int jj = 0; jj < RK_IT; ++jj) {
                const int i = threadIdx.x * RK_IT + jj;
                v[jj] = i < nb ? inj.cchunk[c.chunk_base[side] + ch0 + i] : 0;
                sv += v[jj];
            }
            int64_t tot;
            int64_t ex = block_exclusive_scan64(sv, lds, &tot);
#pragma unroll
            for (int jj = 0; jj < RK_IT; ++jj) {
                const int i = threadIdx.x * RK_IT + jj;
                if (i < nb) pref[i] = (int)ex;
                ex += v[jj];
            }
            if (threadIdx.x == 0) pref[nb] = (int)tot;
            __syncthreads();
            const int E = pref[nb];
            for (int e0 = 0; e0 < E; e0 += RK_THREADS) {
                const int e = e0 + threadIdx.x;
                int slot = -1, d = -1;
                int64_t slc = 0;
                if (e < E) {
                    int lo = 0, hi = nb - 1;          // last chunk with pref <= e
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (pref[mid] <= e) lo = mid; else hi = mid - 1;
                    }
                    slc = cb + (ch0 + lo) * INJ_CH + (e - pref[lo]);
                    d = inj.cdest[slc];
                    slot = inj_slot(d, C);
                    if (slot >= 0 && split && (slot <= KWIN ? 0 : 1) != side) slot = -1;
                    if (slot < 0) atomicOr(err, ERR_RANGE);
                }
                const int r = block_stable_rank<NBI>(slot, binbase, wcnt);
                if (e < E) {
                    const int64_t pos = count + e;
                    if (pos < c.inj_cap) {
                        const int64_t sl = c.inj_base + pos;
                        if (slot >= 0) {
                            inj.x[sl] = inj.cx[slc]; inj.u[sl] = inj.cu[slc];
                            inj.v[sl] = inj.cv[slc]; inj.w[sl] = inj.cw[slc];
                            inj.dest[sl] = c.cell_base + d;
                            inj.rank[sl] = r;
                        } else {
                            inj.dest[sl] = -1;
                        }
                    } else {
                        atomicOr(err, ERR_CAPACITY);
                    }
                }
            }
            count += E;
            nside += E;
            __syncthreads();
        }
        if (threadIdx.x == 0) d_ninj[2 * k + side] = nside;
    }
    // entrant counts of the bins of the sides ranked here
    for (int t = threadIdx.x; t < NBI; t += RK_THREADS) {
        const int d = inj_cell(t, C);
        if (d >= 0 && (!split || (t <= KWIN ? 0 : 1) == s0)) cl.inj_cnt[c.cell_base + d] = binbase[t];
    }
    if (threadIdx.x == 0 && s1 == 2) inj.count[k] = (int32_t)min(count, c.inj_cap);
}

template <typename T>
__global__ void __launch_bounds__(1024) k_inject_rank(const DCase *__restrict__ cases, Cells cl, Inj<T> inj,
                                                      int64_t *d_ninj, int32_t *err)
{
    inject_rank_block<T, 1024>(cases[blockIdx.x], cl, inj, d_ninj, err, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// 6. Free flight of the particles of a loaded canonical state: destination
// histogram per source cell (the steps keep it from then on: the scatter
// predicts the next step's, absorption, resampling and collisions move the
// particles they change between bins)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(512) k_hist_build(const DCase *__restrict__ cases, Cells cl,
                                                     const P4<T> *__restrict__ src,
                                                     const int64_t *__restrict__ off, int gbeg, int gend)
{
    // a block per cell of [gbeg, gend), in turn
    constexpr int IT = 4;
    __shared__ int h[NBIN];
    for (int g = gbeg + (int)blockIdx.x; g < gend; g += gridDim.x) {
        const DCase &c = cases[cl.cell_case[g]];
        const int lc = g - c.cell_base;
        for (int t = threadIdx.x; t < NBIN; t += blockDim.x) h[t] = 0;
        __syncthreads();
        const int64_t b = off[g];
        const int32_t n = (int32_t)(off[g + 1] - b);
        for (int i0 = 0; i0 < n; i0 += IT * blockDim.x) {
            T x[IT], u[IT];
#pragma unroll
            for (int j = 0; j < IT; ++j) {
                const int i = i0 + j * blockDim.x + threadIdx.x;
                x[j] = 0; u[j] = 0;
                if (i < n) {
                    const P4<T> r = src[b + i];
                    x[j] = r.x; u[j] = r.u;
                }
            }
#pragma unroll
            for (int j = 0; j < IT; ++j) {
                const int i = i0 + j * blockDim.x + threadIdx.x;
                if (i >= n) continue;
                const int hb = flight_bin<T>(c, lc, x[j], u[j]);
                if (hb >= 0) atomicAdd(&h[hb], 1);
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < NBIN; t += blockDim.x) cl.hist[(int64_t)g * NBIN + t] = h[t];
        __syncthreads();
    }
}

// Destination cells d of a block: [d0, d0 + nd), nd <= CN_D (fewer when the
// grid would otherwise be small); the histogram rows of their sources,
// [d0 - KWIN, d0 + nd + KWIN), are contiguous in memory and are read into LDS
// once (a destination's 33 sources are 33 different rows).
constexpr int CN_D = 256;   // destinations of a block on large grids: one per thread
constexpr int CN_ROWS = CN_D + 2 * KWIN;

__device__ __forceinline__ void load_hist_tile(const Cells &cl, int d0, int nd, int G, int *tile)
{
    const int s0 = d0 - KWIN;
    for (int t = threadIdx.x; t < (nd + 2 * KWIN) * NBIN; t += blockDim.x) {
        const int src = s0 + t / NBIN;
        tile[t] = (src >= 0 && src < G) ? cl.hist[(int64_t)s0 * NBIN + t] : 0;
    }
}

// 7. Per destination cell d, over its sources d + l - KWIN (l = 0..32, whose bin
// pointing at d is 2 KWIN - l): the start of each (source, d) group inside the
// segment of d, in source-cell order (an exclusive prefix, replacing the counts
// in place), the cell-sourced particles of d (where its entrants start) and its
// count for the next array with the entrants.  Large grids (nd > 4): the block's
// rows through LDS, a thread per destination (the block writes back the entries
// of its destinations); small grids (nd = 4): a wave per destination, lane l =
// source d + l - KWIN, in place.
__global__ void __launch_bounds__(256) k_count_bases(Cells cl, int G, int nd)
{
    __shared__ int tile[CN_ROWS * NBIN];
    const int d0 = blockIdx.x * nd;
    if (nd <= 4) {
        const int lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
        for (int dd = w; dd < nd && d0 + dd < G; dd += nw) {
            const int d = d0 + dd;
            const int src = d + lane - KWIN;
            const bool ok = lane < NBIN && src >= 0 && src < G;
            const int64_t gi = (int64_t)src * NBIN + (2 * KWIN - lane);
            const int h = ok ? cl.hist[gi] : 0;
            int incl = h;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                const int t = __shfl_up(incl, o, WAVE);
                if (lane >= o) incl += t;
            }
            if (ok) cl.hist[gi] = incl - h;
            const int run = __shfl(incl, WAVE - 1, WAVE);
            if (lane == 0) {
                cl.inj_ofs[d] = run;
                cl.cnt_new[d] = run + cl.inj_cnt[d];
            }
        }
        return;
    }
    load_hist_tile(cl, d0, nd, G, tile);
    __syncthreads();
    {
        const int dd = threadIdx.x, d = d0 + dd;
        if (dd < nd && d < G) {
            // (entries of sources outside the grid are zero in the tile and stay so)
            int run = 0;
#pragma unroll
            for (int l = 0; l < NBIN; ++l) {
                const int ti = (dd + l) * NBIN + (2 * KWIN - l);
                const int h = tile[ti];
                tile[ti] = run;
                run += h;
            }
            cl.inj_ofs[d] = run;
            cl.cnt_new[d] = run + cl.inj_cnt[d];
        }
    }
    __syncthreads();
    const int s0 = d0 - KWIN, dend = min(d0 + nd, G);
    for (int t = threadIdx.x; t < (nd + 2 * KWIN) * NBIN; t += blockDim.x) {
        const int src = s0 + t / NBIN;
        const int d = src + t % NBIN - KWIN;
        if (src >= 0 && src < G && d >= d0 && d < dend) cl.hist[(int64_t)s0 * NBIN + t] = tile[t];
    }
}

// 7+8 on small grids (G <= CS1_MAX): the same group bases and the offsets of
// the next array in one block, every histogram row in LDS and a thread per
// destination, then the block's scan of the destination counts (one launch
// instead of two on grids whose passes are all latency).
constexpr int CS1_MAX = 448;

__global__ void __launch_bounds__(1024) k_count_scan_small(Cells cl, int G, int64_t *__restrict__ out,
                                                           int64_t cap, int64_t *total, int32_t *err)
{
    __shared__ int tile[(CS1_MAX + 2 * KWIN) * NBIN];
    __shared__ int64_t lds[16];
    load_hist_tile(cl, 0, G, G, tile);
    __syncthreads();
    const int d = threadIdx.x;
    int64_t cnt = 0;
    if (d < G) {
        int run = 0;
#pragma unroll
        for (int l = 0; l < NBIN; ++l) {
            const int ti = (d + l) * NBIN + (2 * KWIN - l);
            const int h = tile[ti];
            tile[ti] = run;
            run += h;
        }
        cl.inj_ofs[d] = run;
        cnt = run + cl.inj_cnt[d];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < (G + 2 * KWIN) * NBIN; t += blockDim.x) {
        const int src = t / NBIN - KWIN;
        const int dd = src + t % NBIN - KWIN;
        if (src >= 0 && src < G && dd >= 0 && dd < G) cl.hist[(int64_t)src * NBIN + t % NBIN] = tile[t];
    }
    // offsets, clamped to the capacity like the other scans
    int64_t tot;
    const int64_t ex = block_exclusive_scan64(cnt, lds, &tot);
    if (d < G) out[d] = ex < cap ? ex : cap;
    if (d == G - 1) {
        const int64_t end = ex + cnt;
        out[G] = end < cap ? end : cap;
        *total = end;
        if (end > cap) atomicOr(err, ERR_CAPACITY);
    }
}

// Entrants go after the cell-sourced particles of their destination cell; their
// next-step destinations join the predicted histogram.  Part sub of nsub of the
// entrants of case k.
template <typename T>
__device__ __forceinline__ void scatter_entrants(const DCase &c, const Cells &cl, const Inj<T> &inj, P4<T> *dst,
                                              const int64_t *__restrict__ off_new, int64_t cap, int k, int sub,
                                              int nsub)
{
    const int32_t n = inj.count[k];
    const int lane = lane_id();
    for (int i0 = sub * blockDim.x; i0 < n; i0 += nsub * blockDim.x) {
        const int i = i0 + threadIdx.x;
        int key = -1;
        if (i < n) {
            const int64_t sl = c.inj_base + i;
            const int d = inj.dest[sl];
            if (d >= 0) {      // -1: an entrant reported out of range
                const int64_t pos = off_new[d] + cl.inj_ofs[d] + inj.rank[sl];
                const T x = inj.x[sl], u = inj.u[sl];
                if (pos < cap) dst[pos] = P4<T>{x, u, inj.v[sl], inj.w[sl]};
                const int hb = flight_bin<T>(c, d - c.cell_base, x, u);
                if (hb >= 0) key = d * NBIN + hb;
            }
        }
        uint64_t rem = __ballot(key >= 0);
        while (rem) {
            const int leader = __ffsll((unsigned long long)rem) - 1;
            const int v0 = __builtin_amdgcn_readlane(key, leader);
            const uint64_t mm = __ballot(key == v0);
            if (lane == leader) atomicAdd(&cl.hist_nx[v0], __popcll(mm));
            rem &= ~mm;
        }
    }
}

// 11. the entrants of case blockIdx.y, in gridDim.x parts (beside the one-wave
// scatter; the scatter of several-wave blocks places them itself)
template <typename T>
__global__ void __launch_bounds__(256) k_scatter_inj(const DCase *__restrict__ cases, Cells cl,
                                                     const Inj<T> *__restrict__ injp, P4<T> *dst,
                                                     const int64_t *__restrict__ off_new, int64_t cap)
{
    scatter_entrants<T>(cases[blockIdx.y], cl, *injp, dst, off_new, cap, blockIdx.y, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// 10. Stable scatter of the intermediate particles into the next canonical
// array, with the moment sums (1, xi, |xi|^2/2) of each (source, destination)
// group.  Destinations within MB cells keep their sums in registers; the rare
// farther ones are summed in a second pass over the cell.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void add_phi(double (&a)[5], double u, double v, double w)
{
    a[0] += 1.0; a[1] += u; a[2] += v; a[3] += w;
    a[4] += 0.5 * (u * u + v * v + w * w);
}


// Items per thread and chunk, and the waves per SIMD the register budget is cut
// for (FP32 particles): one-wave blocks (small cells) and blocks of several waves.
constexpr int SCAT_IT1 = 2, SCAT_W1 = 7;
constexpr int SCAT_WN = 1;
// blocks per case that place its entrants, after the cells' blocks
constexpr int SCAT_INJ_PARTS = 8;

template <typename T, int MAXW, int IT>
__global__ void __launch_bounds__(512, sizeof(T) == 8 ? 1 : (MAXW == 1 ? SCAT_W1 : SCAT_WN)) k_scatter(const DCase *__restrict__ cases, Cells cl, P4<T> *src,
                                                 P4<T> *stg, P4<T> *dst, const int64_t *__restrict__ off_new,
                                                 int G, int64_t cap, int32_t *err, int64_t *d_nout,
                                                 int by_order, const Inj<T> *__restrict__ injp, int inj_parts)
{
    // One block per cell (the first G blocks), in visiting order cl.order when by_order
    // is set (largest cells first: worth it when the grid runs in few rounds
    // of resident blocks), else in index order, which spares the first load
    // of the chain before a block's particle loads.  Besides placing
    // each particle, the scatter predicts where it goes next step (free flight
    // from its new place with its current velocity) and counts the next step's
    // destination histogram of its new cell in hn[] (new cell relative to this
    // one, next destination), flushed for the new cells that received particles.
    //
    // Each chunk holds IT*blockDim particles; wave w takes the contiguous
    // range of IT*64 particles at w*IT*64, lane l its items l, l+64, ...  Ranks
    // inside a wave come from ballots; the waves' counts are combined once per
    // chunk behind a single barrier.  Two register sets alternate: the next
    // chunk is loaded into one while the other is placed, with no copy between
    // them (a copy would wait for the loads just issued).
    // MAXW: the most waves a block has (blockDim <= 64 MAXW).  A one-wave block
    // keeps the bin bases in registers (lane b: bin b) and needs no barrier
    // inside the chunk loop; blocks of several waves combine their counts in
    // LDS.  IT: items per thread and chunk.
    //
    // Blocks of several waves: the inj_parts blocks per case after the first G
    // place the case's entrants after the cell-sourced particles of their
    // cells: their own places of the next array, and atomic adds to the next
    // histogram like the cells' blocks, so the two go in any order (and no
    // launch of their own).  One-wave blocks leave the entrants to
    // k_scatter_inj (their code would cost the one-wave instance registers).
    constexpr bool ONE = MAXW == 1;
    __shared__ int binbase[ONE ? 1 : 2][NBIN];     // by chunk parity
    __shared__ int bin0[NBIN];
    __shared__ int64_t offb[NBIN];
    __shared__ int wcnt[ONE ? 1 : 2][MAXW][NBIN];  // by chunk parity
    __shared__ double red[NMB * 5 * MAXW];
    __shared__ __attribute__((aligned(16))) int hn[(NBIN * NBIN + 3) / 4 * 4];
    __shared__ int nout;
    if ((int)blockIdx.x >= G) {
        if constexpr (!ONE) {
            const int e = (int)blockIdx.x - G, ke = e / inj_parts;
            scatter_entrants<T>(cases[ke], cl, *injp, dst, off_new, cap, ke, e - ke * inj_parts, inj_parts);
        }
        return;
    }
    const int lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
    for (int t = threadIdx.x; t < (NBIN * NBIN + 3) / 4; t += blockDim.x)
        reinterpret_cast<int4 *>(hn)[t] = int4{0, 0, 0, 0};
    if (threadIdx.x == 0) nout = 0;
    const int g = by_order ? cl.order[blockIdx.x] : (int)blockIdx.x;
    const int k = cl.cell_case[g];
    const DCase &c = cases[k];
    const int lc = g - c.cell_base;
    const CaseK fk(c);
    // lane b of a one-wave block: running base of bin b, its first value, and
    // the bin's destination start relative to lo (set once lo is known)
    int bbr = 0, bb0r = 0, obr = 0;
    int64_t offr = 0;
    if constexpr (ONE) {
        if (lane < NBIN) {
            bbr = cl.hist[(int64_t)g * NBIN + lane];
            bb0r = bbr;
            const int d = g + lane - KWIN;
            offr = (d >= 0 && d < G) ? off_new[d] : 0;
        }
    } else {
        for (int t = threadIdx.x; t < NBIN; t += blockDim.x) {
            binbase[0][t] = cl.hist[(int64_t)g * NBIN + t];
            bin0[t] = binbase[0][t];
            const int d = g + t - KWIN;
            offb[t] = (d >= 0 && d < G) ? off_new[d] : 0;
        }
    }
    __syncthreads();
    int64_t b;
    P4<T> *sg = segment(cl, g, src, stg, b);
    const int32_t n = (int32_t)min((int64_t)cl.n_int[g], cap - b);
    // cell-uniform base pointer: per-particle offsets are unsigned 32-bit
    const P4<T> *__restrict__ gp = sg + b;
    const int64_t lo = off_new[max(g - KWIN, 0)];     // no destination of this cell starts lower
    // record offsets from the uniform bases are 32-bit byte offsets: a block
    // whose source cell or destination window holds more records than that
    // addresses reports a capacity error instead
    constexpr int64_t LIM = ((int64_t)1 << 32) / (int64_t)sizeof(P4<T>);
    if ((int64_t)cl.n_int[g] >= LIM || off_new[min(g + KWIN + 1, G)] - lo >= LIM) {
        if (threadIdx.x == 0) atomicOr(err, ERR_CAPACITY);
        return;
    }
    // destination index relative to lo below which stores stay inside the capacity
    const int64_t dlim = min(cap - lo, (int64_t)INT32_MAX);
    if constexpr (ONE) obr = (int)(offr - lo);
    P4<T> *__restrict__ op = dst + lo;
    // moment sums of the particles moving |d| <= MB cells, per destination
    // (the counts as integers: exact, and half the registers of a double)
    double mb[NMB * 4];
    int mc[NMB];
#pragma unroll
    for (int i = 0; i < NMB * 4; ++i) mb[i] = 0.0;
#pragma unroll
    for (int i = 0; i < NMB; ++i) mc[i] = 0;
    bool far = false;
    const int CH = IT * (int)blockDim.x;
    const int wofs = w * IT * WAVE + lane;
    int cb = 0;

    // loads of a chunk: indices past the end are clamped to the last particle
    // (their values are loaded but not used), so the loads need no branches
    auto load = [&](T (&X)[IT], T (&U)[IT], T (&V)[IT], T (&W)[IT], int i0) {
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            // 32-bit byte offset from a wave-uniform base
            const uint32_t bo = (uint32_t)min(i0 + wofs + j * WAVE, n - 1) * (uint32_t)sizeof(P4<T>);
            const P4<T> r = *(const P4<T> *)((const char *)gp + bo);
            X[j] = r.x; U[j] = r.u; V[j] = r.v; W[j] = r.w;
        }
    };
    auto place = [&](T (&X)[IT], T (&U)[IT], T (&V)[IT], T (&W)[IT], int i0) {
        int key[IT], rk[IT];
        int gone = 0;
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            key[j] = -1;
            if (i0 + wofs + j * WAVE < n) {
                const int dest = Flight<T>::go(fk, lc, X[j], U[j]);
                if (dest >= 0) {
                    const int d = dest - lc;
                    if (d >= -KWIN && d <= KWIN) key[j] = d + KWIN;
                    else atomicOr(err, ERR_RANGE);
                } else {
                    ++gone;
                }
            }
            // next step's destination of the particle from its new place
            if (key[j] >= 0) {
                const int hb = flight_bin<T>(fk, lc + key[j] - KWIN, X[j], U[j]);
                if (hb >= 0) atomicAdd(&hn[key[j] * NBIN + hb], 1);
            }
        }
        if (gone) atomicAdd(&nout, gone);
        // wave-level stable ranks, items in order: one ballot per near bin
        // (wave-uniform counts cn), a loop over distinct keys for the farther
        // ones (lane b of wc counts far bin b); the counts then go to
        // wcnt[cb][w][b] for the cross-wave combine
        int cn0 = 0, cn1 = 0, cn2 = 0;
        int wc = 0;
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int kk = key[j];
            const uint64_t m0 = __ballot(kk == KWIN - 1);
            const uint64_t m1 = __ballot(kk == KWIN);
            const uint64_t m2 = __ballot(kk == KWIN + 1);
            // the three ranks with the masks as scalar operands, then one select
            // (selecting the masks first would copy them into vector registers)
            const int r0 = cn0 + lane_rank_lt(m0), r1 = cn1 + lane_rank_lt(m1), r2 = cn2 + lane_rank_lt(m2);
            rk[j] = kk == KWIN ? r1 : (kk == KWIN - 1 ? r0 : r2);
            cn0 += __popcll(m0);
            cn1 += __popcll(m1);
            cn2 += __popcll(m2);
            const bool kfar = kk >= 0 && (kk < KWIN - 1 || kk > KWIN + 1);
            uint64_t rem = __ballot(kfar);
            while (rem) {
                const int leader = __ffsll((unsigned long long)rem) - 1;
                const int v0 = __builtin_amdgcn_readlane(kk, leader);
                const uint64_t mm = __ballot(kfar && kk == v0);
                const int base = __builtin_amdgcn_readlane(wc, v0);
                if (kfar && kk == v0) rk[j] = base + lane_rank_lt(mm);
                if (lane == v0) wc += __popcll(mm);
                rem &= ~mm;
            }
        }
        const int cntl = lane == KWIN ? cn1 : (lane == KWIN - 1 ? cn0 : (lane == KWIN + 1 ? cn2 : wc));
        // this wave's first destination index of each bin, relative to lo, in
        // lane b for bin b: the bin's running base plus the earlier waves' counts
        int wb = 0;
        if constexpr (ONE) {
            wb = obr + bbr;
            if (lane < NBIN) bbr += cntl;
        } else {
            if (lane < NBIN) wcnt[cb][w][lane] = cntl;
            // the only barrier of the chunk: counts and bases are double-buffered
            lds_barrier();
            if (lane < NBIN) {
                int r = binbase[cb][lane];
                for (int w2 = 0; w2 < w; ++w2) r += wcnt[cb][w2][lane];
                wb = (int)(offb[lane] - lo) + r;
            }
        }
        int di[IT];
#pragma unroll
        for (int j = 0; j < IT; ++j) di[j] = __shfl(wb, max(key[j], 0), WAVE) + rk[j];
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            if (key[j] < 0) continue;
            if (di[j] < dlim) {
                // 32-bit byte offset from the block-uniform destination base
                const uint32_t bo = (uint32_t)di[j] * (uint32_t)sizeof(P4<T>);
                *(P4<T> *)((char *)op + bo) = P4<T>{X[j], U[j], V[j], W[j]};
            }
            const int dd = key[j] - KWIN;
            if (dd >= -MB && dd <= MB) {
                const double du = U[j], dv = V[j], dw = W[j];
                const double e2 = 0.5 * (du * du + dv * dv + dw * dw);
#pragma unroll
                for (int m = 0; m < NMB; ++m)
                    if (dd + MB == m) {
                        mc[m] += 1; mb[m * 4 + 0] += du; mb[m * 4 + 1] += dv; mb[m * 4 + 2] += dw;
                        mb[m * 4 + 3] += e2;
                    }
            } else {
                far = true;
            }
        }
        if constexpr (!ONE) {
            for (int t = threadIdx.x; t < NBIN; t += blockDim.x) {
                int s = 0;
                for (int w2 = 0; w2 < nw; ++w2) s += wcnt[cb][w2][t];
                binbase[cb ^ 1][t] = binbase[cb][t] + s;
            }
            cb ^= 1;
        }
    };

    if (n > 0) {
        T xa[IT], ua[IT], va[IT], wa[IT], xb[IT], ub[IT], vb[IT], wb[IT];
        // the loads past the end read the last particle again (one cache line)
        load(xa, ua, va, wa, 0);
        for (int i0 = 0; i0 < n; i0 += 2 * CH) {
            load(xb, ub, vb, wb, i0 + CH);
            place(xa, ua, va, wa, i0);
            if (i0 + CH >= n) break;
            load(xa, ua, va, wa, i0 + 2 * CH);
            place(xb, ub, vb, wb, i0 + CH);
        }
    }
    double ms[NMB * 5];
#pragma unroll
    for (int m = 0; m < NMB; ++m) {
        ms[m * 5] = (double)mc[m];
#pragma unroll
        for (int q = 0; q < 4; ++q) ms[m * 5 + 1 + q] = mb[m * 4 + q];
    }
    const double mnear_q = block_sum_to_thread<NMB * 5>(ms, red);
    const bool any_far = __syncthreads_or(far);
    // destinations (bins) that received particles, one bit each
    uint64_t rows;
    if constexpr (ONE) rows = __ballot(lane < NBIN && bbr != bb0r);
    else rows = __ballot(lane < NBIN && binbase[cb][lane] != bin0[lane]);
    // rows of the predicted histogram: only new cells that received particles
    for (uint64_t rm = rows; rm; rm &= rm - 1) {
        const int r = __ffsll((unsigned long long)rm) - 1;
        for (int t = threadIdx.x; t < NBIN; t += blockDim.x) {
            const int v0 = hn[r * NBIN + t];
            if (v0) atomicAdd(&cl.hist_nx[(int64_t)(g + r - KWIN) * NBIN + t], v0);
        }
    }
    if (threadIdx.x == 0 && nout) atomicAdd((unsigned long long *)&d_nout[k], (unsigned long long)nout);
    // near sums of this source cell: slot m is destination g + m - MB
    if (threadIdx.x < NMB * 5) cl.mnear[(int64_t)g * (NMB * 5) + threadIdx.x] = mnear_q;
    if (any_far) {
        // a second pass per farther destination that received particles; the
        // sums go to the destination's row, slot KWIN - dd
        for (int bin = 0; bin < NBIN; ++bin) {
            const int dd = bin - KWIN;
            if ((dd >= -MB && dd <= MB) || !((rows >> bin) & 1)) continue;
            double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const P4<T> r = gp[i];
                T x = r.x, u = r.u;
                const int dest = Flight<T>::go(c, lc, x, u);
                if (dest >= 0 && dest - lc == dd) add_phi(a, u, r.v, r.w);
            }
            const double aq = block_sum_to_thread<5>(a, red);
            if (threadIdx.x < 5) cl.mpart[((int64_t)(g + dd) * NBIN + (KWIN - dd)) * 5 + threadIdx.x] = aq;
            if (threadIdx.x == 0) cl.far_in[g + dd] = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// 12. Particle moments of the new state per cell (Eq. gkt_moment0): the sums of
// the near source cells, of farther sources if any, then the entrants; the wave
// part's flux update (Eq. r1); running average of Psi_t; largest relative speed
// of the collisions; finite-state check.
// Two lanes per destination cell: the even one owns the cell, each computes
// one of its two face fluxes (the odd lane's goes to the even one), so the
// transcendental chains of a cell's two faces run side by side.  The entrants
// of a cell are summed by the whole wave.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_gather_moments(const DCase *__restrict__ cases, Cells cl, const P4<T> *dst,
                                                        const int64_t *__restrict__ off_new, int G, int32_t *err,
                                                        uint32_t *d_step, const int64_t *__restrict__ off_old,
                                                        int64_t *d_psteps, int abs_stream)
{
    const int lane = lane_id();
    constexpr int CPW = WAVE / 2;    // cells per wave
    const int d0 = (blockIdx.x * (blockDim.x >> 6) + wave_id()) * CPW;
    const int d = d0 + (lane >> 1), h = lane & 1;
    // the step's close: particle-steps (particles alive at its start), step
    // index, and the big-cell list emptied for the next step
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *d_psteps += off_old[G];
        *d_step += 1;
        *cl.nbig = 0;
        *cl.ntouch = 0;
        *cl.nstage = 0;
    }
    if (d0 >= G) return;
    const bool in = d < G && h == 0;
    // What a lane reads depends on d alone: it is all issued here, before any
    // store and before the case is known (the face's two cells by global index),
    // so that a lane waits on its loads once instead of along a chain.
    const int dc = min(d, G - 1);
    const int kc = cl.cell_case[dc];
    const int g0 = max(dc - 1 + h, 0), g1 = min(dc + h, G - 1);
    double W0[5], W1[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        W0[q] = cl.wt[(int64_t)g0 * 5 + q];
        W1[q] = cl.wt[(int64_t)g1 * 5 + q];
    }
    const int ok0 = cl.okc[g0], ok1 = cl.okc[g1];
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double w0[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, av[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t ib = 0, ie = 0;
    int fin = 0, wain = 0;
    double seen = 0.0, crm = 0.0;
    if (in) {
        constexpr int R = NMB * 5;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            // sources d-1 (moved +1), d (stayed), d+1 (moved -1)
            const double a = d > 0 ? cl.mnear[(int64_t)(d - 1) * R + 2 * 5 + q] : 0.0;
            const double bq = cl.mnear[(int64_t)d * R + 1 * 5 + q];
            const double cq = d + 1 < G ? cl.mnear[(int64_t)(d + 1) * R + 0 * 5 + q] : 0.0;
            s[q] = (a + bq) + cq;
            w0[q] = cl.psi_w[(int64_t)d * 5 + q];
            av[q] = cl.avg[(int64_t)d * 5 + q];
        }
        fin = cl.far_in[d];
        wain = abs_stream ? cl.wabs_in[d] : 0;
        ib = off_new[d] + cl.inj_ofs[d];
        ie = off_new[d + 1];
        seen = __longlong_as_double((long long)cl.cr_seen[d]);
        crm = cl.cr_max[d];
    }
    if (in && fin) {
        double *row = cl.mpart + (int64_t)d * NBIN * 5;
        for (int t = 0; t < NBIN; ++t)
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                s[q] += row[t * 5 + q];
                row[t * 5 + q] = 0.0;
            }
        cl.far_in[d] = 0;
    }
    // the entrants, cell by cell: each lane sums its records in index order,
    // four loads in flight (a load past the end repeats the last record and adds
    // zeros: the loads and sums need no branches)
    uint64_t todo = __ballot(in && ie > ib);
    while (todo) {
        const int l = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const int64_t bl = readlane64(ib, l), el = readlane64(ie, l);
        double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t kk = bl + lane; kk < el; kk += 4 * WAVE) {
            P4<T> r[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) r[j] = dst[min(kk + j * WAVE, el - 1)];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool ok = kk + j * WAVE < el;
                const double u = ok ? (double)r[j].u : 0.0, v = ok ? (double)r[j].v : 0.0;
                const double w = ok ? (double)r[j].w : 0.0;
                a[0] += ok ? 1.0 : 0.0; a[1] += u; a[2] += v; a[3] += w;
                a[4] += 0.5 * (u * u + v * v + w * w);
            }
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            a[q] = wave_sum(a[q]);
            if (lane == l) s[q] += a[q];
        }
    }
    // wave part: the update with the NS flux of the start-of-step total state
    // (Eq. r1; the states cl.wt are those of the step's start), after the
    // absorbed and resampled moments.  Lane h of a cell takes its face lc + h.
    const DCase &c = cases[kc];
    double F[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (d < G) {
        const int f = d - c.cell_base + h;
        if (c.flux2) case_face_flux(c, cl, f, F);
        else case_face_flux1(c, f, W0, ok0, W1, ok1, F);
    }
    double Fr[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) Fr[q] = __shfl_down(F[q], 1, WAVE);
    if (!in) return;
    double pw[5];
    {
        // absorbed moments that streamed in from other cells (absorb_stream),
        // their sources in order, join the wave part before its flux update
        double wa[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        // (abs_stream: some case of the context streams absorbed particles)
        const bool win = abs_stream && c.abs_stream && wain;
        if (win) {
            double *row = cl.wabs + (int64_t)d * NBIN * 5;
            for (int t = 0; t < NBIN; ++t)
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    wa[q] += row[t * 5 + q];
                    row[t * 5 + q] = 0.0;
                }
            cl.wabs_in[d] = 0;
        }
        const double r = c.dt / c.dx;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const double w = win ? w0[q] + c.fac * wa[q] : w0[q];
            pw[q] = w - r * (Fr[q] - F[q]);
            cl.psi_w[(int64_t)d * 5 + q] = pw[q];
        }
    }
    // largest relative speed seen by this cell's collision candidates
    if (seen > crm) cl.cr_max[d] = seen;
    cl.cr_seen[d] = 0ull;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const double p = c.fac * s[q];
        cl.psi_p[(int64_t)d * 5 + q] = p;
        const double t = pw[q] + p;
        if (!isfinite(t)) bad = true;
        cl.avg[(int64_t)d * 5 + q] = av[q] + t;
    }
    if (bad) atomicOr(err, ERR_STATE);
}

// ---------------------------------------------------------------------------
// Diagnostics: normal stress and heat flux of the current state (Eq. gkt_moment1),
// per cell (Pi, Q, Pi_p, Q_p, rho_w/rho_t).  The particle part is taken about the
// total state's mean velocity; the wave part, a Maxwellian at that velocity plus
// the NS closure its flux carries (Sec. 3.3), adds -P (4/3) eps mu dU/dx and
// -P (15/4) R eps mu dT/dx with central differences (the flux's ghost states
// beyond the ends of a case).  Not part of the step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cell_prim(const Cells &cl, const DCase &c, int g, double W[5])
{
    double t[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) t[k] = cl.psi_w[(int64_t)g * 5 + k] + cl.psi_p[(int64_t)g * 5 + k];
    return primitive(t, c.R, W);
}

template <typename T>
__global__ void __launch_bounds__(256) k_stress_heat(const DCase *__restrict__ cases, Cells cl, const P4<T> *a,
                                                     const int64_t *__restrict__ off, int g0, int g1,
                                                     double *__restrict__ out)
{
    __shared__ double red[3 * 4];
    for (int g = g0 + blockIdx.x; g < g1; g += gridDim.x) {
        const DCase &c = cases[cl.cell_case[g]];
        const int lc = g - c.cell_base;
        double W[5], Wl[5], Wr[5];
        const int ok = cell_prim(cl, c, g, W);
        int okl, okr;
        if (lc == 0) {
            if (c.bc_lo == 0) { Wl[0] = c.rho_L; Wl[1] = c.u_L; Wl[2] = 0.0; Wl[3] = 0.0; Wl[4] = c.T_L; okl = 1; }
            else {
#pragma unroll
                for (int k = 0; k < 5; ++k) Wl[k] = W[k];
                Wl[1] = -W[1];
                okl = ok;
            }
        } else {
            okl = cell_prim(cl, c, g - 1, Wl);
        }
        if (lc == c.ncells - 1) {
            if (c.bc_hi == 0) { Wr[0] = c.rho_R; Wr[1] = c.u_R; Wr[2] = 0.0; Wr[3] = 0.0; Wr[4] = c.T_R; okr = 1; }
            else {
#pragma unroll
                for (int k = 0; k < 5; ++k) Wr[k] = W[k];
                Wr[1] = -W[1];
                okr = ok;
            }
        } else {
            okr = cell_prim(cl, c, g + 1, Wr);
        }
        double sm[3] = {0.0, 0.0, 0.0};
        if (ok) {
            for (int64_t kk = off[g] + threadIdx.x; kk < off[g + 1]; kk += blockDim.x) {
                const P4<T> r = a[kk];
                const double cx = (double)r.u - W[1], cy = (double)r.v - W[2], cz = (double)r.w - W[3];
                const double c2 = cx * cx + cy * cy + cz * cz;
                sm[0] += cx * cx;
                sm[1] += c2;
                sm[2] += cx * c2;
            }
        }
        block_sum<3>(sm, red);
        if (threadIdx.x == 0) {
            double o[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (ok) {
                const double pip = c.fac * (sm[0] - sm[1] / 3.0);
                const double qp = c.fac * 0.5 * sm[2];
                double piw = 0.0, qw = 0.0;
                if (okl && okr) {
                    const double mu = viscosity(c, W[4]);
                    const double tau = mu / (W[0] * c.R * W[4]);
                    const double P = absorb_fraction(c.law, c.dt, tau);
                    const double mue = eps_factor(c.eps_law, c.dt / tau) * mu;
                    const double dU = (Wr[1] - Wl[1]) / (2.0 * c.dx);
                    const double dT = (Wr[4] - Wl[4]) / (2.0 * c.dx);
                    piw = -P * (4.0 / 3.0) * mue * dU;
                    qw = -P * (15.0 / 4.0) * c.R * mue * dT;
                }
                o[0] = pip + piw;
                o[1] = qp + qw;
                o[2] = pip;
                o[3] = qp;
                o[4] = cl.psi_w[(int64_t)g * 5] / W[0];
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) out[(int64_t)g * 5 + k] = o[k];
        }
    }
}

// Particle moments of cells [g0, g1) recomputed from a canonical array (after a
// state is loaded), or kept as loaded; either way their totals are checked.
template <typename T>
__global__ void __launch_bounds__(512) k_moments(const DCase *__restrict__ cases, Cells cl, const P4<T> *a,
                                                  const int64_t *__restrict__ off, int g0, int g1,
                                                  int recompute, int32_t *err)
{
    __shared__ double red[5 * 16];
    for (int g = g0 + (int)blockIdx.x; g < g1; g += gridDim.x) {
        const DCase &c = cases[cl.cell_case[g]];
        double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (recompute) {
            const int64_t b = off[g], e = off[g + 1];
            for (int64_t kk = b + threadIdx.x; kk < e; kk += blockDim.x) {
                const P4<T> r = a[kk];
                add_phi(s, (double)r.u, (double)r.v, (double)r.w);
            }
            block_sum<5>(s, red);
        }
        if (threadIdx.x == 0) {
            bool bad = false;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                double p;
                if (recompute) {
                    p = c.fac * s[k];
                    cl.psi_p[(int64_t)g * 5 + k] = p;
                } else {
                    p = cl.psi_p[(int64_t)g * 5 + k];
                }
                if (!isfinite(cl.psi_w[(int64_t)g * 5 + k] + p)) bad = true;
            }
            if (bad) atomicOr(err, ERR_STATE);
        }
    }
}

// closes the step: particle-steps of this step (particles alive at its start), step index

// ---------------------------------------------------------------------------
// Step sequence
// ---------------------------------------------------------------------------
template <typename T>
static P4<T> *recs(void *p)
{
    return (P4<T> *)p;
}

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
    P4<T> *const src = recs<T>(ctx->A[p]), *const dst = recs<T>(ctx->A[p ^ 1]), *const stg = recs<T>(ctx->S);
    const Inj<T> inj{(T *)ctx->J[0], (T *)ctx->J[1], (T *)ctx->J[2], (T *)ctx->J[3], ctx->j_dest, ctx->j_rank,
                     ctx->j_count, (T *)ctx->K[0], (T *)ctx->K[1], (T *)ctx->K[2], (T *)ctx->K[3], ctx->k_dest,
                     ctx->k_n, ctx->k_chunk};
    Cells cl = ctx->cl;
    cl.hist = ctx->hist_buf[p];
    cl.hist_nx = ctx->hist_buf[p ^ 1];
    {
        Mark m(ctx, "cellstate");
        // 64 cells per block; enough waves in all (>= 8192) to count absorbed
        // particles of large cells at full occupancy, at most 16 per block
        const int cblk = (G + WAVE - 1) / WAVE;
        const int cw = std::max(1, std::min(16, (8192 + cblk - 1) / cblk));
        // then the injection candidates: at least four waves per 256 slots of
        // the largest side (up to 256 waves a side)
        const int gen_b = ctx->inj_blocks > 0 ? (4 * ctx->inj_blocks + cw - 1) / cw : 0;
        hipLaunchKernelGGL(k_cellstate<T>, dim3(cblk + 2 * ctx->ncases * gen_b), dim3(WAVE * cw), 0, st,
                           ctx->d_cases, cl, ctx->off[p], ctx->d_step, G, ctx->d_err, ctx->d_nout, ctx->d_ninj,
                           ctx->abs_stream, ctx->big_min_n, ctx->big_min_m, ctx->cap, inj, gen_b);
    }
    {
        Mark m(ctx, "absorb_resample");
        // the listed cells, by a grid of at most 16 blocks per compute unit
        if (ctx->abs_stream)
            hipLaunchKernelGGL((k_absorb_resample<T, true>), dim3(std::min(G, 16 * ctx->big_blocks)), dim3(bc), 0,
                               st, ctx->d_cases, cl, src, ctx->off[p], stg, ctx->d_step, G, ctx->cap,
                               ctx->d_err, ctx->d_nout);
        else
            hipLaunchKernelGGL((k_absorb_resample<T, false>), dim3(std::min(G, 16 * ctx->big_blocks)), dim3(bc), 0,
                               st, ctx->d_cases, cl, src, ctx->off[p], stg, ctx->d_step, G, ctx->cap,
                               ctx->d_err, ctx->d_nout);
    }
    // The big-cell collide does not depend on the small-cell collide: it goes
    // on a second stream (a parallel branch of the captured graph).  Kernel
    // timing keeps everything on one stream.
    const bool big = ctx->big_min_m < INT32_MAX;
    const bool fork = big && !ctx->timer.on && ctx->stream2 != nullptr;
    hipStream_t s2 = fork ? ctx->stream2 : st;
    if (fork) {
        (void)hipEventRecord(ctx->ev_fork, st);
        (void)hipStreamWaitEvent(s2, ctx->ev_fork, 0);
    }
    if (big) {
        // cells with many particles and candidates (their own list): disjoint
        // from the cells of k_collide, so the two run side by side (a threshold
        // no cell reaches leaves the kernel out)
        Mark m(ctx, "collide_big");
        const dim3 gb(ctx->big_blocks * ctx->big_per_cu);
        if (ctx->big_block == 256)
            hipLaunchKernelGGL((k_collide_big<T, 256>), gb, dim3(256), 0, s2, ctx->d_cases, cl, src, stg,
                               ctx->d_step, ctx->cap);
        else if (ctx->big_block == 512)
            hipLaunchKernelGGL((k_collide_big<T, 512>), gb, dim3(512), 0, s2, ctx->d_cases, cl, src, stg,
                               ctx->d_step, ctx->cap);
        else
            hipLaunchKernelGGL((k_collide_big<T, 1024>), gb, dim3(1024), 0, s2, ctx->d_cases, cl, src, stg,
                               ctx->d_step, ctx->cap);
    }
    if (fork) (void)hipEventRecord(ctx->ev_join, s2);
    if (ctx->rank_sep) {
        Mark m(ctx, "inject_rank");
        hipLaunchKernelGGL(k_inject_rank<T>, dim3(ctx->ncases, 2), dim3(1024), 0, st, ctx->d_cases, cl, inj,
                           ctx->d_ninj, ctx->d_err);
    }
    {
        Mark m(ctx, "collide");
        // few cells: a wave per cell; many (mostly small) cells: work items cut
        // from the scanned candidate list
        const int by_cell = G <= ctx->coll_by_cell_max;
        if (!by_cell) {
            enqueue_scan(ctx, ctx->cl.ncand_w, ctx->cl.cbase, ctx->d_total + 2, INT64_MAX);
            hipLaunchKernelGGL(k_items, dim3((G + 1 + 255) / 256), dim3(256), 0, st, ctx->cl.cbase, G,
                               ctx->item_cell, ctx->d_items, ctx->items_cap);
        }
        const int cblocks = by_cell ? std::min(ctx->coll_blocks, (G + COLL_WPB - 1) / COLL_WPB) : ctx->coll_blocks;
        // first, two blocks per case that rank the entrants (unless they have
        // a kernel of their own)
        const int nrk = ctx->rank_sep ? 0 : 2 * ctx->ncases;
        hipLaunchKernelGGL(k_collide<T>, dim3(nrk + cblocks), dim3(64 * COLL_WPB), 0, st, ctx->d_cases,
                           cl, src, stg, ctx->d_step, G, ctx->cap, ctx->d_err, ctx->item_cell, ctx->d_items,
                           by_cell, inj, ctx->d_ninj, nrk);
    }
    if (fork) (void)hipStreamWaitEvent(st, ctx->ev_join, 0);
    // destinations per block of the histogram pass before the scatter: 4 (a wave
    // each, small grids) or up to 256 (a thread each), so that its grid keeps
    // about 1000 blocks or more
    const int nd = std::max(4, std::min(std::min(CN_D, ctx->count_dests), G / 1024 / 4 * 4));
    if (G <= CS1_MAX) {
        Mark m(ctx, "count_scan");
        hipLaunchKernelGGL(k_count_scan_small, dim3(1), dim3(1024), 0, st, cl, G, ctx->off[p ^ 1], ctx->cap,
                           ctx->d_total + 1, ctx->d_err);
    } else {
        {
            Mark m(ctx, "count_bases");
            hipLaunchKernelGGL(k_count_bases, dim3((G + nd - 1) / nd), dim3(256), 0, st, cl, G, nd);
        }
        Mark m(ctx, "scan_offsets");
        enqueue_scan(ctx, ctx->cl.cnt_new, ctx->off[p ^ 1], ctx->d_total + 1, ctx->cap);
    }
    // one-wave scatter blocks: the entrants in a kernel of their own before it
    if (bc == WAVE) {
        Mark m(ctx, "scatter_inj");
        hipLaunchKernelGGL(k_scatter_inj<T>, dim3(SCAT_INJ_PARTS, ctx->ncases), dim3(256), 0, st, ctx->d_cases,
                           cl, (const Inj<T> *)ctx->d_inj, dst, ctx->off[p ^ 1], ctx->cap);
    }
    {
        Mark m(ctx, "scatter");
        if (bc == WAVE)
            hipLaunchKernelGGL((k_scatter<T, 1, SCAT_IT1>), dim3(G), dim3(bc), 0, st, ctx->d_cases, cl, src, stg,
                               dst, ctx->off[p ^ 1], G, ctx->cap, ctx->d_err, ctx->d_nout, ctx->scat_by_order,
                               (const Inj<T> *)ctx->d_inj, SCAT_INJ_PARTS);
        else if (ctx->scat_items == 2)
            hipLaunchKernelGGL((k_scatter<T, 8, 2>), dim3(G + SCAT_INJ_PARTS * ctx->ncases), dim3(bc), 0, st,
                               ctx->d_cases, cl, src, stg, dst, ctx->off[p ^ 1], G, ctx->cap, ctx->d_err,
                               ctx->d_nout, ctx->scat_by_order, (const Inj<T> *)ctx->d_inj, SCAT_INJ_PARTS);
        else
            hipLaunchKernelGGL((k_scatter<T, 8, 4>), dim3(G + SCAT_INJ_PARTS * ctx->ncases), dim3(bc), 0, st,
                               ctx->d_cases, cl, src, stg, dst, ctx->off[p ^ 1], G, ctx->cap, ctx->d_err,
                               ctx->d_nout, ctx->scat_by_order, (const Inj<T> *)ctx->d_inj, SCAT_INJ_PARTS);
    }
    {
        Mark m(ctx, "gather_moments");
        hipLaunchKernelGGL(k_gather_moments<T>, dim3((G + 127) / 128), dim3(256), 0, st, ctx->d_cases, cl, dst,
                           ctx->off[p ^ 1], G, ctx->d_err, ctx->d_step, ctx->off[p], ctx->d_psteps, ctx->abs_stream);
    }
}

// Scatter blocks that fit on one compute unit at once, for this precision, block size
// and items per thread.
int scatter_blocks_per_cu(int precision, int bc, int items)
{
    const void *f;
    if (precision == DUWP_MIXED)
        f = bc == WAVE ? (const void *)&k_scatter<float, 1, SCAT_IT1>
                       : (items == 2 ? (const void *)&k_scatter<float, 8, 2> : (const void *)&k_scatter<float, 8, 4>);
    else
        f = bc == WAVE ? (const void *)&k_scatter<double, 1, SCAT_IT1>
                       : (items == 2 ? (const void *)&k_scatter<double, 8, 2> : (const void *)&k_scatter<double, 8, 4>);
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, bc, 0) != hipSuccess || per <= 0) per = 1;
    return per;
}

void enqueue_step(duwp_ctx *ctx)
{
    if (ctx->precision == DUWP_MIXED) step_impl<float>(ctx);
    else step_impl<double>(ctx);
}

// Zero an int array (kernel, so it can sit in captured work too).
__global__ void k_zero_i32(int32_t *a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

template <typename T>
static void reload_impl(duwp_ctx *ctx, int g0, int g1, bool recompute)
{
    const int p = ctx->step & 1, n = g1 - g0;
    if (n <= 0) return;
    Cells cl = ctx->cl;
    cl.hist = ctx->hist_buf[p];
    P4<T> *const a = recs<T>(ctx->A[p]);
    hipLaunchKernelGGL(k_moments<T>, dim3(std::min(n, 65535)), dim3(ctx->block_cells), 0, ctx->stream, ctx->d_cases,
                       cl, a, ctx->off[p], g0, g1, recompute ? 1 : 0, ctx->d_err);
    hipLaunchKernelGGL(k_hist_build<T>, dim3(std::min(n, 65535)), dim3(ctx->block_cells), 0, ctx->stream,
                       ctx->d_cases, cl, a, ctx->off[p], g0, g1);
}

// Shift the canonical cell offsets of cells [g0, G] by delta (after a restore
// changed the particle count of an earlier case).
__global__ void k_shift_offsets(int64_t *off, int g0, int G, int64_t delta)
{
    const int g = g0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (g <= G) off[g] += delta;
}

void enqueue_shift_offsets(duwp_ctx *ctx, int64_t *off, int g0, int64_t delta)
{
    const int n = ctx->G + 1 - g0;
    if (n > 0 && delta != 0)
        hipLaunchKernelGGL(k_shift_offsets, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, off, g0, ctx->G, delta);
}

// Particle moments of cells [g0, g1) of a loaded canonical state (recomputed from
// the particles, or kept as loaded and only checked), and the destination
// histogram of the same cells.
void enqueue_moments(duwp_ctx *ctx, int g0, int g1, bool recompute)
{
    if (ctx->precision == DUWP_MIXED) reload_impl<float>(ctx, g0, g1, recompute);
    else reload_impl<double>(ctx, g0, g1, recompute);
}

// Normal stress and heat flux of cells [g0, g1) into out (device, [G*5] by global cell).
template <typename T>
static void stress_heat_impl(duwp_ctx *ctx, int g0, int g1, double *out)
{
    const int p = ctx->step & 1;
    P4<T> *const a = recs<T>(ctx->A[p]);
    const int n = g1 - g0;
    hipLaunchKernelGGL(k_stress_heat<T>, dim3(n < 65535 ? n : 65535), dim3(256), 0, ctx->stream, ctx->d_cases,
                       ctx->cl, a, ctx->off[p], g0, g1, out);
}

void enqueue_stress_heat(duwp_ctx *ctx, int g0, int g1, double *out)
{
    if (ctx->precision == DUWP_MIXED) stress_heat_impl<float>(ctx, g0, g1, out);
    else stress_heat_impl<double>(ctx, g0, g1, out);
}

}  // namespace duwp
