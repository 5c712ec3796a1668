// Cell moments of one case into a caller's device buffer with nothing
// allocated, nothing copied to or from the host and no synchronization: the
// variant of duwp_moments for callers that cannot allocate (code under HIP
// graph capture, serving loops).
//
// The normal stress and heat flux take two passes through a file-scope device
// array (`scratch`, one copy per GPU): the first writes each cell's primitive
// state and the two ghost states of the case, the second the stress and heat
// flux of every cell from its own row and its neighbours'.  The other moments
// need no scratch and go straight to the output.
#include <hip/hip_runtime.h>

#include <mutex>

#include "duwp.h"
#include "duwp_ctx.hpp"
#include "duwp_device.hpp"
#include "duwp_physics.hpp"

namespace duwp {

// rows of (rho, U, V, W, T, ok) for the cells of one case (rows 1..C) and its
// ghost states (rows 0 and C+1)
constexpr int SCR_ROW = 6;
static __device__ __align__(256) double scratch[(DUWP_NOALLOC_MAX_CELLS + 2) * SCR_ROW];

// device address of `scratch` per device, taken once per device at set-up
constexpr int MAX_DEV = 64;
static double *g_scratch[MAX_DEV] = {nullptr};
static std::mutex g_scratch_mu;

hipError_t noalloc_setup(int dev, double **ptr)
{
    if (dev < 0 || dev >= MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = (double *)p;
    }
    *ptr = g_scratch[dev];
    return hipSuccess;
}

// pass 1: primitive state of every cell of the case and of its two ghosts
// (the reservoir state, or the mirror image of the boundary cell at a wall)
__global__ void __launch_bounds__(256) k_na_prim(const DCase *__restrict__ cases, Cells cl, int case_id,
                                                 double *__restrict__ scr)
{
    const DCase &c = cases[case_id];
    const int C = c.ncells;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > C + 1) return;
    double W[5];
    int ok;
    const int side = r == 0 ? 0 : (r == C + 1 ? 1 : -1);
    if (side < 0 || (side == 0 ? c.bc_lo : c.bc_hi) != 0) {
        // a cell, or the cell a wall mirrors
        const int lc = side < 0 ? r - 1 : (side == 0 ? 0 : C - 1);
        const int64_t g = c.cell_base + lc;
        double t[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) t[k] = cl.psi_w[g * 5 + k] + cl.psi_p[g * 5 + k];
        ok = primitive(t, c.R, W);
        if (side >= 0) W[1] = -W[1];
    } else {
        W[0] = side == 0 ? c.rho_L : c.rho_R;
        W[1] = side == 0 ? c.u_L : c.u_R;
        W[2] = 0.0;
        W[3] = 0.0;
        W[4] = side == 0 ? c.T_L : c.T_R;
        ok = 1;
    }
    double *row = scr + (int64_t)r * SCR_ROW;
#pragma unroll
    for (int k = 0; k < 5; ++k) row[k] = W[k];
    row[5] = (double)ok;
}

// pass 2: (Pi, Q, Pi_p, Q_p, rho_w/rho_t) of each cell (Eq. gkt_moment1, xx entry
// and x component), the particle part about the cell's total mean velocity, the
// wave part the NS closure its flux carries (Sec. 3.3), weighted by P
template <typename T>
__global__ void __launch_bounds__(256) k_na_stress_heat(const DCase *__restrict__ cases, Cells cl, const P4<T> *a,
                                                        const int64_t *__restrict__ off, int case_id,
                                                        const double *__restrict__ scr, double *__restrict__ out)
{
    __shared__ double red[3 * 4];
    const DCase &c = cases[case_id];
    for (int lc = blockIdx.x; lc < c.ncells; lc += gridDim.x) {
        const int64_t g = c.cell_base + lc;
        const double *Wl = scr + (int64_t)lc * SCR_ROW, *W = Wl + SCR_ROW, *Wr = W + SCR_ROW;
        const bool ok = W[5] != 0.0, okl = Wl[5] != 0.0, okr = Wr[5] != 0.0;
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
                o[4] = cl.psi_w[g * 5] / W[0];
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) out[(int64_t)lc * 5 + k] = o[k];
        }
    }
}

// every other moment: one thread per cell, straight into the output
__global__ void __launch_bounds__(256) k_na_moments(const DCase *__restrict__ cases, Cells cl, int case_id, int what,
                                                    double inv_count, double *__restrict__ out)
{
    const DCase &c = cases[case_id];
    const int lc = blockIdx.x * blockDim.x + threadIdx.x;
    if (lc >= c.ncells) return;
    const int64_t g = c.cell_base + lc;
    double t[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double w = cl.psi_w[g * 5 + k], p = cl.psi_p[g * 5 + k], s = cl.avg[g * 5 + k];
        switch (what) {
        case DUWP_M_PSI_W: t[k] = w; break;
        case DUWP_M_PSI_P: t[k] = p; break;
        case DUWP_M_AVG_SUM: t[k] = s; break;
        case DUWP_M_AVG_PRIM: t[k] = s * inv_count; break;
        default: t[k] = w + p; break;
        }
    }
    if (what == DUWP_M_PRIM || what == DUWP_M_AVG_PRIM) {
        const double rho = t[0];
        double U = 0.0, V = 0.0, Wv = 0.0, T = 0.0;
        if (rho > 0.0) {
            U = t[1] / rho;
            V = t[2] / rho;
            Wv = t[3] / rho;
            T = (2.0 / (3.0 * c.R)) * (t[4] / rho - 0.5 * (U * U + V * V + Wv * Wv));
        }
        t[0] = rho; t[1] = U; t[2] = V; t[3] = Wv; t[4] = T;
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) out[(int64_t)lc * 5 + k] = t[k];
}

template <typename T>
static void na_stress_heat(duwp_ctx *ctx, int case_id, int C, double *out)
{
    const int p = ctx->step & 1;
    const P4<T> *a = (const P4<T> *)ctx->A[p];
    hipLaunchKernelGGL(k_na_prim, dim3((C + 2 + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_cases, ctx->cl, case_id,
                       ctx->scratch);
    hipLaunchKernelGGL(k_na_stress_heat<T>, dim3(C < 65535 ? C : 65535), dim3(256), 0, ctx->stream, ctx->d_cases,
                       ctx->cl, a, ctx->off[p], case_id, ctx->scratch, out);
}

}  // namespace duwp

extern "C" duwp_status duwp_moments_noalloc(duwp_ctx *ctx, int32_t case_id, int32_t what, double *out, int64_t len)
{
    if (!ctx || !out || case_id < 0 || case_id >= ctx->ncases || what < 0 || what > DUWP_M_STRESS_HEAT)
        return DUWP_EINVAL;
    const int C = ctx->hcases[case_id].ncells;
    if (len < 5 * (int64_t)C) return DUWP_EINVAL;
    (void)hipGetLastError();
    if (what == DUWP_M_STRESS_HEAT) {
        if (C > DUWP_NOALLOC_MAX_CELLS) return DUWP_EINVAL;
        if (!ctx->scratch) return DUWP_EDEVICE;
        if (ctx->precision == DUWP_MIXED) duwp::na_stress_heat<float>(ctx, case_id, C, out);
        else duwp::na_stress_heat<double>(ctx, case_id, C, out);
    } else {
        const double inv = ctx->avg_count > 0 ? 1.0 / (double)ctx->avg_count : 0.0;
        hipLaunchKernelGGL(duwp::k_na_moments, dim3((C + 255) / 256), dim3(256), 0, ctx->stream, ctx->d_cases, ctx->cl,
                           case_id, what, inv, out);
    }
    return hipGetLastError() == hipSuccess ? DUWP_OK : DUWP_EDEVICE;
}
