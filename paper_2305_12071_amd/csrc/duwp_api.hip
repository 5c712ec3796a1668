// C ABI of the DUWP library: context set-up, stepping, state access.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "duwp.h"
#include "duwp_ctx.hpp"

using duwp::DCase;

namespace {

constexpr double kPi = 3.14159265358979323846;

#define HIP_OK(expr)                                  \
    do {                                              \
        if ((expr) != hipSuccess) return DUWP_EDEVICE; \
    } while (0)

bool tune_valid(const duwp_tune &t, int precision)
{
    if (t.collide_blocks_per_cu < 0 || t.collide_blocks_per_cu > 256) return false;
    if (t.scatter_items != 0 && t.scatter_items != 2 && t.scatter_items != 4) return false;
    if (t.big_block != 0 && t.big_block != 256 && t.big_block != 512 && t.big_block != 1024) return false;
    if (t.big_blocks_per_cu < 0 || t.big_blocks_per_cu > 8) return false;
    (void)precision;
    if (t.big_min_particles < 0 || (t.big_min_particles > 0 && t.big_min_particles < 64)) return false;
    if (t.big_min_candidates < 0 || (t.big_min_candidates > 0 && t.big_min_candidates < 64)) return false;
    if (t.collide_by_cell_max < 0) return false;
    if (t.count_dests < 0 || t.count_dests % 4 || t.count_dests > 256) return false;
    return true;
}

bool case_valid(const duwp_case &c)
{
    if (c.ncells <= 0 || !(c.x_hi > c.x_lo) || !(c.m_particle > 0.0) || !(c.dt > 0.0)) return false;
    if (!(c.R > 0.0) || !(c.T_ref > 0.0) || !(c.omega > 0.0)) return false;
    if (!(c.x_split >= c.x_lo && c.x_split <= c.x_hi)) return false;
    if (!(c.rho_L > 0.0 && c.rho_R > 0.0 && c.T_L > 0.0 && c.T_R > 0.0)) return false;
    if (!(c.lambda_ref > 0.0 && c.rho_ref > 0.0) && !(c.m_mol > 0.0 && c.d_ref > 0.0)) return false;
    if (c.bc_lo < 0 || c.bc_lo > 1 || c.bc_hi < 0 || c.bc_hi > 1) return false;
    if (c.classify_law < 0 || c.classify_law > 1 || c.eps_law < 0 || c.eps_law > 3) return false;
    if (c.dsmc_full_dt < 0 || c.dsmc_full_dt > 1 || c.absorb_stream < 0 || c.absorb_stream > 1) return false;
    if (c.reserved_case != 0) return false;
    return true;
}

// Gas constants of a case.  beta: mean-free-path factor (Sec. 4.1, Eq. lambda,
// alpha = 1).  Lam = lambda_ref rho_ref = m/(sqrt(2) pi d_ref^2) (Appendix A).
// Matching the viscosity and diameter forms of the mean free path at T_ref gives
// mu_ref = beta Lam sqrt(2 pi R T_ref).  sigma_ref n = rho/(sqrt(2) Lam).
// VHS reference relative speed c_ref = sqrt(4 R T_ref)/Gamma(5/2-omega)^(1/(2 ups)).
DCase derive(const duwp_case &c, int cell_base, uint64_t seed, int case_id)
{
    DCase d{};
    d.ncells = c.ncells;
    d.cell_base = cell_base;
    d.bc_lo = c.bc_lo;
    d.bc_hi = c.bc_hi;
    d.law = c.classify_law;
    d.eps_law = c.eps_law;
    d.full_dt = c.dsmc_full_dt;
    d.flux2 = c.flux_order == 2;
    d.abs_stream = c.absorb_stream != 0;
    d.key0 = (uint32_t)seed;
    d.key1 = (uint32_t)(seed >> 32) + (uint32_t)case_id;
    d.x_lo = c.x_lo;
    d.x_hi = c.x_hi;
    d.dx = (c.x_hi - c.x_lo) / (double)c.ncells;
    d.dt = c.dt;
    d.R = c.R;
    d.omega = c.omega;
    d.T_ref = c.T_ref;
    const double beta = 30.0 / (4.0 * (5.0 - 2.0 * c.omega) * (7.0 - 2.0 * c.omega));
    const double lam = (c.lambda_ref > 0.0) ? c.lambda_ref * c.rho_ref
                                            : c.m_mol / (std::sqrt(2.0) * kPi * c.d_ref * c.d_ref);
    d.mu_ref = beta * lam * std::sqrt(2.0 * kPi * c.R * c.T_ref);
    d.coll_k = 1.0 / (std::sqrt(2.0) * lam);
    d.ups = c.omega - 0.5;
    d.c_ref = (d.ups != 0.0) ? std::sqrt(4.0 * c.R * c.T_ref) / std::pow(std::tgamma(2.5 - c.omega), 1.0 / (2.0 * d.ups))
                             : 1.0;
    d.m_p = c.m_particle;
    d.fac = c.m_particle / d.dx;
    d.rho_L = c.rho_L; d.u_L = c.u_L; d.T_L = c.T_L;
    d.rho_R = c.rho_R; d.u_R = c.u_R; d.T_R = c.T_R;
    d.dtdx_f = (float)(c.dt / d.dx);
    return d;
}

// Upper bound on the injection candidates of one side in one step:
// floor((1-P) rho Lg / m_p + u) <= rho Lg / m_p + 1.
int64_t inject_bound(const duwp_case &c, int side)
{
    if ((side == 0 ? c.bc_lo : c.bc_hi) != DUWP_BC_RESERVOIR) return 0;
    double rho = side == 0 ? c.rho_L : c.rho_R, U = side == 0 ? c.u_L : c.u_R, T = side == 0 ? c.T_L : c.T_R;
    double Lg = c.dt * (std::fabs(U) + 8.0 * std::sqrt(c.R * T));
    return (int64_t)std::ceil(rho * Lg / c.m_particle) + 2;
}

// one device buffer from the caller's allocator, or hipMalloc; every buffer is
// listed for duwp_destroy
template <typename P>
duwp_status dalloc(duwp_ctx *ctx, P **p, size_t bytes)
{
    void *q = nullptr;
    bytes = bytes ? (bytes + 255) / 256 * 256 : 256;
    if (ctx->alloc_fn) {
        q = ctx->alloc_fn(bytes, ctx->alloc_ctx);
        if (!q) return DUWP_ENOMEM;
        if (((uintptr_t)q & 255) != 0) {      // the records and histograms need the alignment
            ctx->free_fn(q, ctx->alloc_ctx);
            return DUWP_ENOMEM;
        }
    } else if (hipMalloc(&q, bytes) != hipSuccess) {
        return DUWP_ENOMEM;
    }
    ctx->allocs.push_back(q);
    *p = (P *)q;
    return DUWP_OK;
}

#define TRY(expr)                                \
    do {                                         \
        duwp_status s_ = (expr);                 \
        if (s_ != DUWP_OK) return s_;            \
    } while (0)

duwp_status alloc_all(duwp_ctx *ctx)
{
    const int G = ctx->G;
    const size_t es = ctx->precision == DUWP_MIXED ? sizeof(float) : sizeof(double);
    // particles as (x,u,v,w) records: one vector access and one cache line each
    for (int p = 0; p < 2; ++p) TRY(dalloc(ctx, &ctx->A[p], 4 * es * (size_t)ctx->cap));
    TRY(dalloc(ctx, &ctx->S, 4 * es * (size_t)ctx->cap));
    for (int a = 0; a < 4; ++a) TRY(dalloc(ctx, &ctx->J[a], es * (size_t)ctx->inj_total));
    TRY(dalloc(ctx, &ctx->j_dest, 4 * (size_t)ctx->inj_total));
    TRY(dalloc(ctx, &ctx->j_rank, 4 * (size_t)ctx->inj_total));
    TRY(dalloc(ctx, &ctx->j_count, 4 * (size_t)ctx->ncases));
    for (int a = 0; a < 4; ++a) TRY(dalloc(ctx, &ctx->K[a], es * (size_t)ctx->cand_total));
    TRY(dalloc(ctx, &ctx->k_dest, 4 * (size_t)ctx->cand_total));
    TRY(dalloc(ctx, &ctx->k_n, 16 * (size_t)ctx->ncases));
    TRY(dalloc(ctx, &ctx->k_chunk, 4 * (size_t)ctx->chunk_total));
    // the entrant buffers' addresses in device memory: the scatter reads them
    // there, which spares it fourteen argument registers
    TRY(dalloc(ctx, &ctx->d_inj, sizeof(duwp::Inj<double>)));
    if (ctx->precision == DUWP_MIXED) {
        const duwp::Inj<float> h{(float *)ctx->J[0], (float *)ctx->J[1], (float *)ctx->J[2], (float *)ctx->J[3],
                                 ctx->j_dest, ctx->j_rank, ctx->j_count, (float *)ctx->K[0], (float *)ctx->K[1],
                                 (float *)ctx->K[2], (float *)ctx->K[3], ctx->k_dest, ctx->k_n, ctx->k_chunk};
        HIP_OK(hipMemcpy(ctx->d_inj, &h, sizeof(h), hipMemcpyHostToDevice));
    } else {
        const duwp::Inj<double> h{(double *)ctx->J[0], (double *)ctx->J[1], (double *)ctx->J[2], (double *)ctx->J[3],
                                  ctx->j_dest, ctx->j_rank, ctx->j_count, (double *)ctx->K[0], (double *)ctx->K[1],
                                  (double *)ctx->K[2], (double *)ctx->K[3], ctx->k_dest, ctx->k_n, ctx->k_chunk};
        HIP_OK(hipMemcpy(ctx->d_inj, &h, sizeof(h), hipMemcpyHostToDevice));
    }
    for (int p = 0; p < 2; ++p) TRY(dalloc(ctx, &ctx->off[p], 8 * (size_t)(G + 1)));
    duwp::Cells &c = ctx->cl;
    TRY(dalloc(ctx, &c.psi_w, 8 * 5 * (size_t)G));
    TRY(dalloc(ctx, &c.psi_p, 8 * 5 * (size_t)G));
    TRY(dalloc(ctx, &c.wt, 8 * 5 * (size_t)G));
    TRY(dalloc(ctx, &c.pc, 8 * (size_t)G));
    TRY(dalloc(ctx, &c.tau, 8 * (size_t)G));
    TRY(dalloc(ctx, &c.okc, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.cr_max, 8 * (size_t)G));
    TRY(dalloc(ctx, &c.n_surv, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.n_new, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.n_int, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.nstage, 8));
    TRY(dalloc(ctx, &c.seg, 8 * (size_t)G));
    TRY(dalloc(ctx, &c.seg_stg, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.mpart, 8 * 5 * (size_t)G * duwp::NBIN));
    TRY(dalloc(ctx, &c.mnear, 8 * 15 * (size_t)G));
    TRY(dalloc(ctx, &c.far_in, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.wabs_in, 4 * (size_t)G));
    {
        // the table of absorbed moments that stream across cells, only when a case asks for it
        bool any = false;
        for (const DCase &d : ctx->hcases) any = any || d.abs_stream;
        ctx->abs_stream = any ? 1 : 0;
        if (any) TRY(dalloc(ctx, &c.wabs, 8 * 5 * (size_t)G * duwp::NBIN));
    }
    TRY(dalloc(ctx, &c.d_abs, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.d_new, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.d_cand, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.d_coll, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.cbase, 8 * (size_t)(G + 1)));
    TRY(dalloc(ctx, &c.cr_seen, 8 * (size_t)G));
    TRY(dalloc(ctx, &c.ncand_w, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.big_list, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.nbig, 4));
    TRY(dalloc(ctx, &c.touch_list, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.ntouch, 4));
    TRY(dalloc(ctx, &ctx->diag, 8 * 5 * (size_t)G));
    ctx->items_cap = std::max<int64_t>(1 << 20, 2 * (int64_t)G);
    TRY(dalloc(ctx, &ctx->item_cell, 4 * (size_t)ctx->items_cap));
    TRY(dalloc(ctx, &ctx->d_items, 16));
    for (int p = 0; p < 2; ++p) TRY(dalloc(ctx, &ctx->hist_buf[p], 4 * (size_t)G * duwp::NBIN));
    c.hist = ctx->hist_buf[0];
    TRY(dalloc(ctx, &c.cnt_new, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.inj_cnt, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.inj_ofs, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.cell_case, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.order, 4 * (size_t)G));
    TRY(dalloc(ctx, &c.avg, 8 * 5 * (size_t)G));
    ctx->ntiles = (G + 2047) / 2048;
    TRY(dalloc(ctx, &ctx->scan_part, 8 * (size_t)std::max(ctx->ntiles, 1)));
    TRY(dalloc(ctx, &ctx->d_step, 4));
    TRY(dalloc(ctx, &ctx->d_err, 4));
    TRY(dalloc(ctx, &ctx->d_nout, 8 * (size_t)ctx->ncases));
    TRY(dalloc(ctx, &ctx->d_ninj, 16 * (size_t)ctx->ncases));
    TRY(dalloc(ctx, &ctx->d_total, 24));
    TRY(dalloc(ctx, &ctx->d_psteps, 8));
    TRY(dalloc(ctx, &ctx->d_cases, sizeof(DCase) * (size_t)ctx->ncases));
    return DUWP_OK;
}

duwp_status upload_initial(duwp_ctx *ctx)
{
    const int G = ctx->G;
    std::vector<double> psi(5 * (size_t)G), cr(G), npc(G);
    std::vector<int32_t> cc(G);
    for (int k = 0; k < ctx->ncases; ++k) {
        const duwp_case &c = ctx->cases[k];
        const DCase &d = ctx->hcases[k];
        for (int i = 0; i < c.ncells; ++i) {
            const int g = d.cell_base + i;
            // all mass starts in the wave part at the cell-centre value of the step profile
            const double xc = c.x_lo + ((double)i + 0.5) * d.dx;
            const bool left = xc < c.x_split;
            const double rho = left ? c.rho_L : c.rho_R, U = left ? c.u_L : c.u_R, T = left ? c.T_L : c.T_R;
            psi[5 * g + 0] = rho;
            psi[5 * g + 1] = rho * U;
            psi[5 * g + 2] = 0.0;
            psi[5 * g + 3] = 0.0;
            psi[5 * g + 4] = rho * (0.5 * U * U + 1.5 * c.R * T);
            cr[g] = 6.0 * std::sqrt(c.R * T);
            cc[g] = k;
            npc[g] = rho * d.dx / c.m_particle;
        }
    }
    // Block-per-cell kernels visit the cells with the most particles first (by
    // the initial profile), so that the longest blocks do not start last.  The
    // order changes no result: every cell's work is independent.
    std::vector<int32_t> order(G);
    for (int g = 0; g < G; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return npc[a] > npc[b]; });
    hipStream_t s = ctx->stream;
    HIP_OK(hipMemcpyAsync(ctx->cl.psi_w, psi.data(), 8 * psi.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(ctx->cl.cr_max, cr.data(), 8 * cr.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(ctx->cl.cell_case, cc.data(), 4 * cc.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(ctx->cl.order, order.data(), 4 * order.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(ctx->d_cases, ctx->hcases.data(), sizeof(DCase) * ctx->hcases.size(),
                          hipMemcpyHostToDevice, s));
    HIP_OK(hipMemsetAsync(ctx->cl.psi_p, 0, 8 * 5 * (size_t)G, s));
    HIP_OK(hipMemsetAsync(ctx->cl.avg, 0, 8 * 5 * (size_t)G, s));
    HIP_OK(hipMemsetAsync(ctx->cl.cr_seen, 0, 8 * (size_t)G, s));
    HIP_OK(hipMemsetAsync(ctx->cl.mpart, 0, 8 * 5 * (size_t)G * duwp::NBIN, s));
    HIP_OK(hipMemsetAsync(ctx->cl.far_in, 0, 4 * (size_t)G, s));
    HIP_OK(hipMemsetAsync(ctx->cl.wabs_in, 0, 4 * (size_t)G, s));
    if (ctx->cl.wabs) HIP_OK(hipMemsetAsync(ctx->cl.wabs, 0, 8 * 5 * (size_t)G * duwp::NBIN, s));
    HIP_OK(hipMemsetAsync(ctx->cl.nbig, 0, 4, s));
    HIP_OK(hipMemsetAsync(ctx->cl.ntouch, 0, 4, s));
    HIP_OK(hipMemsetAsync(ctx->cl.nstage, 0, 8, s));
    for (int p = 0; p < 2; ++p) HIP_OK(hipMemsetAsync(ctx->off[p], 0, 8 * (size_t)(G + 1), s));
    HIP_OK(hipMemsetAsync(ctx->d_step, 0, 4, s));
    HIP_OK(hipMemsetAsync(ctx->d_err, 0, 4, s));
    HIP_OK(hipMemsetAsync(ctx->d_psteps, 0, 8, s));
    HIP_OK(hipMemsetAsync(ctx->d_nout, 0, 8 * (size_t)ctx->ncases, s));
    HIP_OK(hipMemsetAsync(ctx->d_ninj, 0, 16 * (size_t)ctx->ncases, s));
    HIP_OK(hipMemsetAsync(ctx->j_count, 0, 4 * (size_t)ctx->ncases, s));
    HIP_OK(hipMemsetAsync(ctx->k_n, 0, 16 * (size_t)ctx->ncases, s));
    for (int p = 0; p < 2; ++p) HIP_OK(hipMemsetAsync(ctx->hist_buf[p], 0, 4 * (size_t)G * duwp::NBIN, s));
    const duwp::Cells &c = ctx->cl;
    for (int32_t *p : {c.d_abs, c.d_new, c.d_cand, c.d_coll}) HIP_OK(hipMemsetAsync(p, 0, 4 * (size_t)G, s));
    HIP_OK(hipStreamSynchronize(s));
    return DUWP_OK;
}

duwp_status read_error(duwp_ctx *ctx)
{
    int32_t e = 0;
    HIP_OK(hipMemcpyAsync(&e, ctx->d_err, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    if (e & duwp::ERR_CAPACITY) return DUWP_ECAPACITY;
    if (e & duwp::ERR_RANGE) return DUWP_ERANGE;
    if (e & duwp::ERR_STATE) return DUWP_ESTATE;
    return DUWP_OK;
}

duwp_status build_graphs(duwp_ctx *ctx)
{
    for (int p = 0; p < 2; ++p) {
        if (ctx->graph[p]) continue;
        const uint32_t saved = ctx->step;
        ctx->step = (uint32_t)p;   // only the parity matters for the captured pointers
        hipGraph_t g = nullptr;
        (void)hipGetLastError();
        if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            ctx->step = saved;
            return DUWP_EDEVICE;
        }
        duwp::enqueue_step(ctx);
        hipError_t e = hipStreamEndCapture(ctx->stream, &g);
        ctx->step = saved;
        if (e != hipSuccess) return DUWP_EDEVICE;
        e = hipGraphInstantiate(&ctx->graph[p], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return DUWP_EDEVICE;
    }
    ctx->graph_ready = true;
    return DUWP_OK;
}

// host copy of the canonical offsets of one case's cells (ncells + 1 values) at the current parity
duwp_status case_offsets(duwp_ctx *ctx, const DCase &d, std::vector<int64_t> &off)
{
    off.resize((size_t)d.ncells + 1);
    HIP_OK(hipMemcpyAsync(off.data(), ctx->off[ctx->step & 1] + d.cell_base, 8 * off.size(), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return DUWP_OK;
}

// records [b, b+n) of the canonical array, as four host arrays x, u, v, w
template <typename T>
duwp_status download_particles(duwp_ctx *ctx, int64_t b, int64_t n, std::vector<T> (&out)[4])
{
    const int p = ctx->step & 1;
    std::vector<T> rec(4 * (size_t)n);
    if (n)
        HIP_OK(hipMemcpyAsync(rec.data(), (T *)ctx->A[p] + 4 * b, 4 * sizeof(T) * n, hipMemcpyDeviceToHost,
                              ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    for (int a = 0; a < 4; ++a) {
        out[a].resize((size_t)n);
        for (int64_t q = 0; q < n; ++q) out[a][q] = rec[4 * q + a];
    }
    return DUWP_OK;
}

}  // namespace

extern "C" {

const char *duwp_strerror(duwp_status s)
{
    switch (s) {
    case DUWP_OK: return "ok";
    case DUWP_EINVAL: return "invalid argument or case description";
    case DUWP_ENOMEM: return "device allocation failed";
    case DUWP_EDEVICE: return "HIP call failed";
    case DUWP_ECAPACITY: return "particle, staging or injection capacity exceeded";
    case DUWP_ESTATE: return "non-finite cell state";
    case DUWP_ERANGE: return "a particle crossed more cells in one step than the sort window allows";
    }
    return "unknown status";
}

void duwp_destroy(duwp_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->stream2) (void)hipStreamSynchronize(ctx->stream2);
    // The whole device, not only the context's streams: a replayed graph runs its
    // parallel branch on a stream of the runtime's own, and buffers freed while the
    // runtime still counted that branch as running were never released (measured:
    // two of the three particle buffers stayed allocated after each closed context).
    (void)hipDeviceSynchronize();
    for (auto &g : ctx->graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (hipEvent_t e : ctx->timer.ev) (void)hipEventDestroy(e);
    for (void *p : ctx->allocs) {
        if (ctx->free_fn) ctx->free_fn(p, ctx->alloc_ctx);
        else (void)hipFree(p);
    }
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->stream2) (void)hipStreamDestroy(ctx->stream2);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    delete ctx;
}

duwp_status duwp_init(duwp_ctx **out, const duwp_case *cases, int32_t ncases, const duwp_opts *opts)
{
    if (!out || !cases || ncases <= 0 || !opts) return DUWP_EINVAL;
    *out = nullptr;
    // every check on the arguments comes before the first device call
    if (opts->precision != DUWP_FP64 && opts->precision != DUWP_MIXED) return DUWP_EINVAL;
    if (opts->block_cells < 0 || (opts->block_cells > 0 && (opts->block_cells % 64 || opts->block_cells > 512)))
        return DUWP_EINVAL;
    if (opts->reserved != 0 || (opts->alloc != nullptr) != (opts->free != nullptr)) return DUWP_EINVAL;
    if (!tune_valid(opts->tune, opts->precision)) return DUWP_EINVAL;
    {
        int64_t cells = 0;
        for (int k = 0; k < ncases; ++k) {
            if (!case_valid(cases[k])) return DUWP_EINVAL;
            cells += cases[k].ncells;
        }
        if (cells > (int64_t)1 << 30) return DUWP_EINVAL;
    }
    duwp_ctx *ctx = new (std::nothrow) duwp_ctx();
    if (!ctx) return DUWP_ENOMEM;
    ctx->ncases = ncases;
    ctx->precision = opts->precision;
    ctx->use_graph = opts->use_graph;
    ctx->stream = (hipStream_t)opts->stream;
    if (!ctx->stream) {
        // the null stream cannot be captured into a graph: use a private stream
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return DUWP_EDEVICE;
        }
        ctx->own_stream = true;
    }
    ctx->seed = opts->seed;
    ctx->block_cells = opts->block_cells > 0 ? opts->block_cells : 256;
    ctx->alloc_fn = opts->alloc;
    ctx->free_fn = opts->free;
    ctx->alloc_ctx = opts->alloc_ctx;
    {
        const duwp_tune &t = opts->tune;
        ctx->scat_items = t.scatter_items ? t.scatter_items : 4;
        ctx->big_block = t.big_block ? t.big_block : (opts->precision == DUWP_MIXED ? 512 : 256);
        ctx->big_per_cu = t.big_blocks_per_cu ? t.big_blocks_per_cu : (ctx->big_block == 1024 ? 1 : 2);
        ctx->big_min_n = t.big_min_particles ? t.big_min_particles : duwp::BIG_N;
        ctx->big_min_m = t.big_min_candidates ? t.big_min_candidates : duwp::BIG_M;
        ctx->coll_by_cell_max = t.collide_by_cell_max ? t.collide_by_cell_max : 8192;
        ctx->count_dests = t.count_dests ? t.count_dests : 256;
    }
    if (hipStreamCreateWithFlags(&ctx->stream2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess) {
        duwp_destroy(ctx);
        return DUWP_EDEVICE;
    }
    const double head = opts->headroom > 0.0 ? opts->headroom : 1.5;
    int64_t G = 0, cap = 0, inj = 0, cand = 0, max_side = 0, chunks = 0;
    for (int k = 0; k < ncases; ++k) {
        const duwp_case &c = cases[k];
        ctx->cases.push_back(c);
        ctx->hcases.push_back(derive(c, (int)G, opts->seed, k));
        G += c.ncells;
        int64_t cc = c.capacity;
        if (cc <= 0) {
            const double mass = c.rho_L * (c.x_split - c.x_lo) + c.rho_R * (c.x_hi - c.x_split);
            cc = (int64_t)std::ceil(head * mass / c.m_particle) + 4096;
        }
        cap += cc;
        DCase &d = ctx->hcases.back();
        int64_t ib = 0;
        for (int side = 0; side < 2; ++side) {
            const int64_t nb = inject_bound(c, side);
            d.cand_base[side] = cand;
            d.cand_cap[side] = nb;
            d.chunk_base[side] = chunks;
            chunks += (nb + duwp::INJ_CH - 1) / duwp::INJ_CH;
            cand += nb;
            ib += nb;
            max_side = std::max(max_side, nb);
        }
        d.inj_base = inj;
        d.inj_cap = ib;
        inj += ib;
    }
    if (cap > ((int64_t)1 << 40)) { duwp_destroy(ctx); return DUWP_EINVAL; }
    ctx->G = (int)G;
    ctx->cap = cap;
    ctx->inj_total = std::max<int64_t>(inj, 1);
    ctx->cand_total = std::max<int64_t>(cand, 1);
    ctx->chunk_total = std::max<int64_t>(chunks, 1);
    ctx->inj_blocks = (int)std::min<int64_t>((max_side + 255) / 256, 64);
    // sides that may draw more than 2^18 candidates have their entrants ranked
    // by 1024-thread blocks of a kernel of their own rather than inside the
    // collision launch (a quarter of the rounds: 0.43 -> 0.05 ms on the Mach-10
    // shock, whose inflow brings 1.4e5 entrants a step)
    ctx->rank_sep = max_side > (1 << 18) ? 1 : 0;
    {
        // collision work items are taken by a fixed grid of 16 blocks (64 waves) per compute unit
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess) { duwp_destroy(ctx); return DUWP_EDEVICE; }
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            ncu = 256;
        // the allocation-free moments' staging array on this device
        if (duwp::noalloc_setup(dev, &ctx->scratch) != hipSuccess) { duwp_destroy(ctx); return DUWP_EDEVICE; }
        // work items: many waves in flight hide each chunk's load chain
        ctx->coll_blocks = (opts->tune.collide_blocks_per_cu ? opts->tune.collide_blocks_per_cu : 16) * ncu;
        ctx->big_blocks = ncu;
        // the scatter visits cells largest first only when its grid runs in
        // few rounds of resident blocks (the tail then matters); with many
        // rounds the order lookup would only lengthen each block's load chain
        const int64_t resident = (int64_t)duwp::scatter_blocks_per_cu(ctx->precision, ctx->block_cells, ctx->scat_items) * ncu;
        ctx->scat_by_order = G < 16 * resident ? 1 : 0;
    }
    duwp_status s = alloc_all(ctx);
    if (s == DUWP_OK) s = upload_initial(ctx);
    if (s != DUWP_OK) { duwp_destroy(ctx); return s; }
    *out = ctx;
    return DUWP_OK;
}

duwp_status duwp_step(duwp_ctx *ctx, int32_t nsteps)
{
    if (!ctx || nsteps < 0) return DUWP_EINVAL;
    if (ctx->use_graph && !ctx->graph_ready) {
        duwp_status s = build_graphs(ctx);
        if (s != DUWP_OK) return s;
    }
    (void)hipGetLastError();   // drop errors left by unrelated earlier calls
    for (int32_t i = 0; i < nsteps; ++i) {
        if (ctx->use_graph) {
            if (hipGraphLaunch(ctx->graph[ctx->step & 1], ctx->stream) != hipSuccess) return DUWP_EDEVICE;
        } else {
            duwp::enqueue_step(ctx);
            if (hipGetLastError() != hipSuccess) return DUWP_EDEVICE;
        }
        ctx->step += 1;
        ctx->avg_count += 1;
    }
    return read_error(ctx);
}

duwp_status duwp_sync(duwp_ctx *ctx)
{
    if (!ctx) return DUWP_EINVAL;
    return read_error(ctx);
}

duwp_status duwp_counts(duwp_ctx *ctx, int32_t case_id, int64_t *n_particles, int32_t *ncells, uint32_t *step)
{
    if (!ctx || case_id < 0 || case_id >= ctx->ncases) return DUWP_EINVAL;
    const DCase &d = ctx->hcases[case_id];
    if (n_particles) {
        int64_t v[2];
        HIP_OK(hipMemcpyAsync(&v[0], ctx->off[ctx->step & 1] + d.cell_base, 8, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipMemcpyAsync(&v[1], ctx->off[ctx->step & 1] + d.cell_base + d.ncells, 8, hipMemcpyDeviceToHost,
                              ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
        *n_particles = v[1] - v[0];
    }
    if (ncells) *ncells = d.ncells;
    if (step) *step = ctx->step;
    return DUWP_OK;
}

duwp_status duwp_moments(duwp_ctx *ctx, int32_t case_id, int32_t what, double *out, int64_t len,
                         int32_t out_on_device)
{
    if (!ctx || !out || case_id < 0 || case_id >= ctx->ncases || what < 0 || what > DUWP_M_STRESS_HEAT)
        return DUWP_EINVAL;
    const DCase &d = ctx->hcases[case_id];
    const int C = d.ncells;
    if (len < 5 * (int64_t)C) return DUWP_EINVAL;
    if (what == DUWP_M_STRESS_HEAT) {
        (void)hipGetLastError();
        duwp::enqueue_stress_heat(ctx, d.cell_base, d.cell_base + C, ctx->diag);
        if (hipGetLastError() != hipSuccess) return DUWP_EDEVICE;
        const double *src = ctx->diag + 5 * (size_t)d.cell_base;
        HIP_OK(hipMemcpyAsync(out, src, 8 * 5 * (size_t)C,
                              out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
        return read_error(ctx);
    }
    std::vector<double> w(5 * (size_t)C), p(5 * (size_t)C), a(5 * (size_t)C);
    const size_t o = 5 * (size_t)d.cell_base, nb = 8 * 5 * (size_t)C;
    HIP_OK(hipMemcpyAsync(w.data(), ctx->cl.psi_w + o, nb, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipMemcpyAsync(p.data(), ctx->cl.psi_p + o, nb, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipMemcpyAsync(a.data(), ctx->cl.avg + o, nb, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    std::vector<double> r(5 * (size_t)C);
    const double inv = ctx->avg_count > 0 ? 1.0 / (double)ctx->avg_count : 0.0;
    for (int i = 0; i < C; ++i) {
        double t[5];
        for (int k = 0; k < 5; ++k) {
            switch (what) {
            case DUWP_M_PSI_W: t[k] = w[5 * i + k]; break;
            case DUWP_M_PSI_P: t[k] = p[5 * i + k]; break;
            case DUWP_M_AVG_SUM: t[k] = a[5 * i + k]; break;
            case DUWP_M_AVG_PRIM: t[k] = a[5 * i + k] * inv; break;
            default: t[k] = w[5 * i + k] + p[5 * i + k]; break;
            }
        }
        if (what == DUWP_M_PRIM || what == DUWP_M_AVG_PRIM) {
            const double rho = t[0];
            double U = 0, V = 0, W = 0, T = 0;
            if (rho > 0.0) {
                U = t[1] / rho; V = t[2] / rho; W = t[3] / rho;
                T = (2.0 / (3.0 * d.R)) * (t[4] / rho - 0.5 * (U * U + V * V + W * W));
            }
            t[0] = rho; t[1] = U; t[2] = V; t[3] = W; t[4] = T;
        }
        for (int k = 0; k < 5; ++k) r[5 * i + k] = t[k];
    }
    if (out_on_device) {
        HIP_OK(hipMemcpyAsync(out, r.data(), 8 * r.size(), hipMemcpyHostToDevice, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
    } else {
        std::memcpy(out, r.data(), 8 * r.size());
    }
    return DUWP_OK;
}

int64_t duwp_avg_count(duwp_ctx *ctx) { return ctx ? ctx->avg_count : 0; }

duwp_status duwp_particle_steps(duwp_ctx *ctx, int64_t *psteps, int32_t reset)
{
    if (!ctx || !psteps) return DUWP_EINVAL;
    HIP_OK(hipMemcpyAsync(psteps, ctx->d_psteps, 8, hipMemcpyDeviceToHost, ctx->stream));
    if (reset) HIP_OK(hipMemsetAsync(ctx->d_psteps, 0, 8, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return DUWP_OK;
}

duwp_status duwp_reset_average(duwp_ctx *ctx)
{
    if (!ctx) return DUWP_EINVAL;
    HIP_OK(hipMemsetAsync(ctx->cl.avg, 0, 8 * 5 * (size_t)ctx->G, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    ctx->avg_count = 0;
    return DUWP_OK;
}

duwp_status duwp_diag(duwp_ctx *ctx, int32_t case_id, int32_t *n_abs, int32_t *n_new, int32_t *n_cand,
                      int32_t *n_coll, int64_t *n_inj, int64_t *n_out)
{
    if (!ctx || case_id < 0 || case_id >= ctx->ncases) return DUWP_EINVAL;
    const DCase &d = ctx->hcases[case_id];
    const size_t nb = 4 * (size_t)d.ncells;
    const duwp::Cells &c = ctx->cl;
    hipStream_t s = ctx->stream;
    if (n_abs) HIP_OK(hipMemcpyAsync(n_abs, c.d_abs + d.cell_base, nb, hipMemcpyDeviceToHost, s));
    if (n_new) HIP_OK(hipMemcpyAsync(n_new, c.d_new + d.cell_base, nb, hipMemcpyDeviceToHost, s));
    if (n_cand) HIP_OK(hipMemcpyAsync(n_cand, c.d_cand + d.cell_base, nb, hipMemcpyDeviceToHost, s));
    if (n_coll) HIP_OK(hipMemcpyAsync(n_coll, c.d_coll + d.cell_base, nb, hipMemcpyDeviceToHost, s));
    if (n_inj) HIP_OK(hipMemcpyAsync(n_inj, ctx->d_ninj + 2 * case_id, 16, hipMemcpyDeviceToHost, s));
    if (n_out) HIP_OK(hipMemcpyAsync(n_out, ctx->d_nout + case_id, 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return DUWP_OK;
}

duwp_status duwp_get_state(duwp_ctx *ctx, int32_t case_id, duwp_state *st)
{
    if (!ctx || !st || case_id < 0 || case_id >= ctx->ncases) return DUWP_EINVAL;
    const DCase &d = ctx->hcases[case_id];
    std::vector<int64_t> off;
    TRY(case_offsets(ctx, d, off));
    const int64_t b = off[0], n = off[d.ncells] - b;
    if (st->ncells != d.ncells || st->n_particles < n) return DUWP_EINVAL;
    st->n_particles = n;
    st->step = ctx->step;
    st->avg_count = ctx->avg_count;
    if (st->off)
        for (int i = 0; i <= d.ncells; ++i) st->off[i] = off[i] - b;
    if (ctx->precision == DUWP_MIXED) {
        std::vector<float> h[4];
        TRY(download_particles<float>(ctx, b, n, h));
        for (int i = 0; i < d.ncells; ++i)
            for (int64_t q = off[i] - b; q < off[i + 1] - b; ++q) {
                if (st->x) st->x[q] = d.x_lo + ((double)i + (double)h[0][q]) * d.dx;
                if (st->u) st->u[q] = h[1][q];
                if (st->v) st->v[q] = h[2][q];
                if (st->w) st->w[q] = h[3][q];
            }
    } else {
        std::vector<double> h[4];
        TRY(download_particles<double>(ctx, b, n, h));
        double *dst[4] = {st->x, st->u, st->v, st->w};
        for (int a = 0; a < 4; ++a)
            if (dst[a]) std::memcpy(dst[a], h[a].data(), 8 * (size_t)n);
    }
    hipStream_t s = ctx->stream;
    const size_t o5 = 5 * (size_t)d.cell_base, n5 = 8 * 5 * (size_t)d.ncells;
    if (st->psi_w) HIP_OK(hipMemcpyAsync(st->psi_w, ctx->cl.psi_w + o5, n5, hipMemcpyDeviceToHost, s));
    if (st->cr_max)
        HIP_OK(hipMemcpyAsync(st->cr_max, ctx->cl.cr_max + d.cell_base, 8 * (size_t)d.ncells, hipMemcpyDeviceToHost, s));
    if (st->psi_p) HIP_OK(hipMemcpyAsync(st->psi_p, ctx->cl.psi_p + o5, n5, hipMemcpyDeviceToHost, s));
    if (st->avg_sum) HIP_OK(hipMemcpyAsync(st->avg_sum, ctx->cl.avg + o5, n5, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return DUWP_OK;
}

duwp_status duwp_set_state(duwp_ctx *ctx, int32_t case_id, const duwp_state *st)
{
    if (!ctx || !st || case_id < 0 || case_id >= ctx->ncases) return DUWP_EINVAL;
    const DCase &d = ctx->hcases[case_id];
    if (st->ncells != d.ncells || !st->off || !st->psi_w || !st->cr_max || st->n_particles < 0) return DUWP_EINVAL;
    if (st->n_particles > 0 && (!st->x || !st->u || !st->v || !st->w)) return DUWP_EINVAL;
    if (st->off[0] != 0 || st->off[d.ncells] != st->n_particles) return DUWP_EINVAL;
    for (int i = 0; i < d.ncells; ++i)
        if (st->off[i + 1] < st->off[i]) return DUWP_EINVAL;
    if (st->avg_sum && st->avg_count < 0) return DUWP_EINVAL;
    const int G = ctx->G, p = ctx->step & 1;
    // the case's first offset and its end, and the end of the whole array
    int64_t b, e, endall;
    {
        hipStream_t s = ctx->stream;
        HIP_OK(hipMemcpyAsync(&b, ctx->off[p] + d.cell_base, 8, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(&e, ctx->off[p] + d.cell_base + d.ncells, 8, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(&endall, ctx->off[p] + G, 8, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    const int64_t nold = e - b, nnew = st->n_particles, delta = nnew - nold;
    const int64_t total = endall + delta;
    if (total > ctx->cap) return DUWP_ECAPACITY;
    const bool mixed = ctx->precision == DUWP_MIXED;
    const size_t es = mixed ? 4 : 8, rs = 4 * es;   // element and record sizes
    // the case's records in device layout, record q at out + rs q
    std::vector<char> hh(rs * (size_t)nnew);
    {
        const double *srcv[4] = {st->x, st->u, st->v, st->w};
        char *out = hh.data();
        for (int i = 0; i < d.ncells; ++i)
            for (int64_t q = st->off[i]; q < st->off[i + 1]; ++q)
                for (int a = 0; a < 4; ++a) {
                    double val = srcv[a][q];
                    char *slot = out + rs * (size_t)q + es * (size_t)a;
                    if (mixed) {
                        float f;
                        if (a == 0) {
                            double sv = (val - d.x_lo) / d.dx - (double)i;
                            f = (float)sv;
                            if (f < 0.0f) f = 0.0f;
                            if (f >= 1.0f) f = 0.99999994f;
                        } else {
                            f = (float)val;
                        }
                        std::memcpy(slot, &f, 4);
                    } else {
                        std::memcpy(slot, &val, 8);
                    }
                }
    }
    std::vector<int64_t> coff((size_t)d.ncells + 1);
    for (int i = 0; i <= d.ncells; ++i) coff[i] = b + st->off[i];
    hipStream_t s = ctx->stream;
    // a fresh error word: the context may be restored after a step reported one
    HIP_OK(hipMemsetAsync(ctx->d_err, 0, 4, s));
    char *A = (char *)ctx->A[p];
    if (delta != 0) {
        // the later cases' records move by delta, on the device, through the
        // staging buffer (source and destination overlap); their offsets follow
        const int64_t tail = endall - e;
        if (tail > 0) {
            HIP_OK(hipMemcpyAsync(ctx->S, A + rs * (size_t)e, rs * (size_t)tail, hipMemcpyDeviceToDevice, s));
            HIP_OK(hipMemcpyAsync(A + rs * (size_t)(e + delta), ctx->S, rs * (size_t)tail, hipMemcpyDeviceToDevice, s));
        }
        (void)hipGetLastError();
        duwp::enqueue_shift_offsets(ctx, ctx->off[p], d.cell_base + d.ncells + 1, delta);
        if (hipGetLastError() != hipSuccess) return DUWP_EDEVICE;
    }
    if (nnew) HIP_OK(hipMemcpyAsync(A + rs * (size_t)b, hh.data(), hh.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(ctx->off[p] + d.cell_base, coff.data(), 8 * coff.size(), hipMemcpyHostToDevice, s));
    const size_t o5 = 5 * (size_t)d.cell_base, n5 = 8 * 5 * (size_t)d.ncells;
    HIP_OK(hipMemcpyAsync(ctx->cl.psi_w + o5, st->psi_w, n5, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(ctx->cl.cr_max + d.cell_base, st->cr_max, 8 * (size_t)d.ncells, hipMemcpyHostToDevice, s));
    if (st->psi_p) HIP_OK(hipMemcpyAsync(ctx->cl.psi_p + o5, st->psi_p, n5, hipMemcpyHostToDevice, s));
    if (st->avg_sum) HIP_OK(hipMemcpyAsync(ctx->cl.avg + o5, st->avg_sum, n5, hipMemcpyHostToDevice, s));
    // the step index is shared by all cases; the buffers of the state follow its parity
    if ((st->step & 1u) != (ctx->step & 1u)) {
        if (total)
            HIP_OK(hipMemcpyAsync(ctx->A[p ^ 1], ctx->A[p], rs * (size_t)total, hipMemcpyDeviceToDevice, s));
        HIP_OK(hipMemcpyAsync(ctx->off[p ^ 1], ctx->off[p], 8 * (size_t)(G + 1), hipMemcpyDeviceToDevice, s));
        HIP_OK(hipMemcpyAsync(ctx->hist_buf[p ^ 1], ctx->hist_buf[p], 4 * (size_t)G * duwp::NBIN,
                              hipMemcpyDeviceToDevice, s));
    }
    ctx->step = st->step;
    if (st->avg_sum) ctx->avg_count = st->avg_count;
    uint32_t dstep = st->step;
    HIP_OK(hipMemcpyAsync(ctx->d_step, &dstep, 4, hipMemcpyHostToDevice, s));
    (void)hipGetLastError();
    // the case's particle moments (loaded or summed afresh) and its destination histograms
    duwp::enqueue_moments(ctx, d.cell_base, d.cell_base + d.ncells, st->psi_p == nullptr);
    if (hipGetLastError() != hipSuccess) return DUWP_EDEVICE;
    return read_error(ctx);
}

duwp_status duwp_profile(duwp_ctx *ctx, int32_t nsteps, const char **names, double *ms, int32_t cap,
                         int32_t *count)
{
    if (!ctx || nsteps <= 0) return DUWP_EINVAL;
    duwp::KernelTimer &t = ctx->timer;
    const int nk = 16;
    if (t.ev.empty()) {
        t.ev.resize(2 * nk);
        for (auto &e : t.ev) HIP_OK(hipEventCreate(&e));
    }
    std::vector<double> acc(nk, 0.0);
    int used = 0;
    for (int s = 0; s < nsteps; ++s) {
        t.on = true;
        t.idx = 0;
        duwp::enqueue_step(ctx);
        t.on = false;
        ctx->step += 1;
        ctx->avg_count += 1;
        HIP_OK(hipStreamSynchronize(ctx->stream));
        used = t.idx;
        for (int i = 0; i < used; ++i) {
            float m = 0.0f;
            HIP_OK(hipEventElapsedTime(&m, t.ev[2 * i], t.ev[2 * i + 1]));
            acc[i] += m;
        }
    }
    if (count) *count = used;
    for (int i = 0; i < used && i < cap; ++i) {
        if (names) names[i] = t.names[i].c_str();
        if (ms) ms[i] = acc[i] / nsteps;
    }
    return read_error(ctx);
}

}  // extern "C"
