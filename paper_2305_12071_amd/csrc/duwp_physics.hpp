// Device-side gas physics of the DUWP step: viscosity and relaxation time,
// absorption fraction (Eq. p), primitive state, Maxwellian sampling
// (Eq. maxsample), free flight with boundaries, and the wave flux (Sec. 3.3).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

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

// Maxwellian velocity, one (cos, log) pair of uniforms per component (Eq. maxsample):
// xi_d = U_d + sqrt(2 R T) cos(2 pi u) sqrt(-ln(1 - u')), the uniforms from the
// words w[2d] and w[2d+1].  The sampler of one state is set up once per cell.
template <typename T>
struct Maxwell;

template <>
struct Maxwell<double> {
    double mean[3], sd;
    __device__ Maxwell(double U, double V, double W, double T, double R) : mean{U, V, W}, sd(sqrt(2.0 * R * T)) {}
    __device__ __forceinline__ void sample(const uint32_t w[6], double out[3]) const
    {
#pragma unroll
        for (int d = 0; d < 3; ++d)
            out[d] = mean[d] + sd * cos(D_TWO_PI * u01(w[2 * d])) * sqrt(-log(1.0 - u01(w[2 * d + 1])));
    }
};

// FP32 particles: the velocity is stored in FP32, so it is computed in FP32.  The
// uniforms are the nearest floats to w 2^-32 and to 1 - w 2^-32 (formed from the
// integer 2^32 - w, so the tail keeps its 2^-32 resolution): the values of the
// exact FP64 uniforms rounded to FP32.  cos(2 pi u) is taken as cospi(2u), whose
// argument is exact.
__device__ __forceinline__ float u01f(uint32_t r) { return (float)r * 2.3283064365386962890625e-10f; }
__device__ __forceinline__ float one_minus_u01f(uint32_t r)
{
    return r == 0u ? 1.0f : (float)(0u - r) * 2.3283064365386962890625e-10f;
}

template <>
struct Maxwell<float> {
    float mean[3], sd;
    __device__ Maxwell(double U, double V, double W, double T, double R)
        : mean{(float)U, (float)V, (float)W}, sd(sqrtf((float)(2.0 * R * T)))
    {
    }
    __device__ __forceinline__ void sample(const uint32_t w[6], float out[3]) const
    {
#pragma unroll
        for (int d = 0; d < 3; ++d)
            out[d] = mean[d] + sd * cospif(2.0f * u01f(w[2 * d])) * sqrtf(-logf(one_minus_u01f(w[2 * d + 1])));
    }
};

// ---------------------------------------------------------------------------
// Free flight and boundaries.  Returns the local destination cell, -1 if the
// particle left through a reservoir side.
// ---------------------------------------------------------------------------

// FP64, absolute position.  A particle that ends inside [x_lo, x_hi] takes the
// short path; leaving the domain (reflection or deletion) takes the loop.
struct FlightD { double x, u; int dest; };
struct FlightF { float s, u; int dest; };

__device__ __noinline__ FlightD bc_cell_abs_slow(const DCase &c, double x, double u)
{
    for (int it = 0; it < 1000; ++it) {
        if (!isfinite(x)) return FlightD{x, u, -1};
        if (x < c.x_lo) {
            if (c.bc_lo == 0) return FlightD{x, u, -1};
            x = 2.0 * c.x_lo - x;
            u = -u;
        } else if (x > c.x_hi) {
            if (c.bc_hi == 0) return FlightD{x, u, -1};
            x = 2.0 * c.x_hi - x;
            u = -u;
        } else {
            double f = floor((x - c.x_lo) / c.dx);
            int64_t ci = (int64_t)f;
            if (f < 0.0) ci = 0;
            if (ci > c.ncells - 1) ci = c.ncells - 1;
            return FlightD{x, u, (int)ci};
        }
    }
    return FlightD{x, u, -1};
}

template <typename K>
__device__ __forceinline__ int bc_cell_abs(const K &c, double &x, double &u)
{
    if (x >= c.x_lo && x <= c.x_hi) {
        const double f = floor((x - c.x_lo) / c.dx);
        int ci = (int)f;
        if (ci > c.ncells - 1) ci = c.ncells - 1;
        return ci;
    }
    const FlightD r = bc_cell_abs_slow(case_of(c), x, u);
    x = r.x;
    u = r.u;
    return r.dest;
}

// FP32, position as (integer cell I, fraction f in [0,1)) relative to x_lo.
__device__ __noinline__ FlightF bc_cell_rel_slow(const DCase &c, int I, float f, float u)
{
    const int C = c.ncells;
    for (int it = 0; it < 1000; ++it) {
        if (I < 0) {
            if (c.bc_lo == 0) return FlightF{f, u, -1};
            I = -I - 1;
            f = 1.0f - f;
            u = -u;
        } else if (I >= C) {
            if (c.bc_hi == 0) return FlightF{f, u, -1};
            I = 2 * C - I - 1;
            f = 1.0f - f;
            u = -u;
        } else {
            if (f >= 1.0f) { f -= 1.0f; I += 1; continue; }
            return FlightF{f, u, I};
        }
    }
    return FlightF{f, u, -1};
}

template <typename K>
__device__ __forceinline__ int bc_cell_rel(const K &c, int I, float f, float &u, float &s)
{
    if (f >= 1.0f) { f -= 1.0f; I += 1; }
    if (I >= 0 && I < c.ncells) {
        s = f;
        return I;
    }
    const FlightF r = bc_cell_rel_slow(case_of(c), I, f, u);
    s = r.s;
    u = r.u;
    return r.dest;
}

template <typename T>
struct Flight;

template <>
struct Flight<double> {
    // stream a particle of local cell lc; x is absolute
    template <typename K>
    __device__ static int go(const K &c, int /*lc*/, double &x, double &u)
    {
        x = x + u * c.dt;
        return bc_cell_abs(c, x, u);
    }
};

template <>
struct Flight<float> {
    // stream a particle of local cell lc; x is the position inside the cell, in cells
    template <typename K>
    __device__ static int go(const K &c, int lc, float &s, float &u)
    {
        const float X = s + u * c.dtdx_f;
        if (!(fabsf(X) < 1.0e9f)) return -1;
        const float fl = floorf(X);
        return bc_cell_rel(c, lc + (int)fl, X - fl, u, s);
    }
};

// Free time of an absorbed particle (absorb_stream): the u of its classification
// draw gives t_f < dt with u < P: tau/(1-u) under Eq. p, -tau ln(1-u) under
// the exponential law.
__device__ __forceinline__ double free_time(int law, double tau, double u)
{
    return law == 1 ? -tau * log(1.0 - u) : tau / (1.0 - u);
}

// Flight of an absorbed particle over its free time tf < dt: its landing cell
// (local), or -1 when it leaves through a reservoir; u follows wall reflections.
template <typename T>
struct PartialFlight;

template <>
struct PartialFlight<double> {
    template <typename K>
    __device__ static int go(const K &c, int /*lc*/, double x, double &u, double tf)
    {
        x = x + u * tf;
        return bc_cell_abs(c, x, u);
    }
};

template <>
struct PartialFlight<float> {
    template <typename K>
    __device__ static int go(const K &c, int lc, float s, float &u, double tf)
    {
        const float X = s + u * (float)(tf / c.dx);
        if (!(fabsf(X) < 1.0e9f)) return -1;
        const float fl = floorf(X);
        return bc_cell_rel(c, lc + (int)fl, X - fl, u, s);
    }
};

// ---------------------------------------------------------------------------
// Wave part: NS flux (KFVS inviscid + central viscous, eps-scaled viscosity,
// weighted by the interface absorption fraction).
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

// Flux through a face with cell states (Wl, Wr): P_m, the viscosity and the
// central gradients come from them; the KFVS part takes the inviscid face
// states (ql, qr), which are (Wl, Wr) at first order.
__device__ inline void face_flux(const DCase &c, const double Wl[5], const double Wr[5], const double ql[5],
                                 const double qr[5], double F[5])
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
    kfvs_half(ql, c.R, +1, Hp);
    kfvs_half(qr, c.R, -1, Hm);
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
    for (int k = 0; k < 5; ++k) F[k] = Pm * ((ql[0] * Hp[k] + qr[0] * Hm[k]) - visc[k]);
}

// State of local cell lc of a case at step start, lc in [-1, C]: -1 and C are the
// ghost states (the reservoir state, or the mirror image of the boundary cell at
// a wall).  Returns 0 for a vacuum cell.
__device__ inline int case_cell_state(const DCase &c, const Cells &cl, int lc, double W[5])
{
    const int C = c.ncells, base = c.cell_base;
    if (lc >= 0 && lc < C) {
#pragma unroll
        for (int k = 0; k < 5; ++k) W[k] = cl.wt[(int64_t)(base + lc) * 5 + k];
        return cl.okc[base + lc];
    }
    const int side = lc < 0 ? 0 : 1;
    if ((side == 0 ? c.bc_lo : c.bc_hi) == 0) {
        W[0] = side == 0 ? c.rho_L : c.rho_R;
        W[1] = side == 0 ? c.u_L : c.u_R;
        W[2] = 0.0; W[3] = 0.0;
        W[4] = side == 0 ? c.T_L : c.T_R;
        return 1;
    }
    const int b = side == 0 ? base : base + C - 1;
#pragma unroll
    for (int k = 0; k < 5; ++k) W[k] = cl.wt[(int64_t)b * 5 + k];
    W[1] = -W[1];
    return cl.okc[b];
}

__device__ __forceinline__ double minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

// Minmod slope of the primitive state of local cell lc (zero for a ghost, or
// when the cell or a neighbour is vacuum)
__device__ inline void case_slope(const DCase &c, const Cells &cl, int lc, double D[5])
{
#pragma unroll
    for (int k = 0; k < 5; ++k) D[k] = 0.0;
    if (lc < 0 || lc >= c.ncells) return;
    double W[5], Wm[5], Wp[5];
    const int ok = case_cell_state(c, cl, lc, W);
    const int okm = case_cell_state(c, cl, lc - 1, Wm);
    const int okp = case_cell_state(c, cl, lc + 1, Wp);
    if (!(ok && okm && okp)) return;
#pragma unroll
    for (int k = 0; k < 5; ++k) D[k] = minmod(W[k] - Wm[k], Wp[k] - W[k]);
}

// flux through local face f (between local cells f-1 and f) of a case
__device__ inline void case_face_flux(const DCase &c, const Cells &cl, int f, double F[5])
{
    double Wl[5], Wr[5];
    const int okl = case_cell_state(c, cl, f - 1, Wl);
    const int okr = case_cell_state(c, cl, f, Wr);
    if (!(okl && okr)) {
#pragma unroll
        for (int k = 0; k < 5; ++k) F[k] = 0.0;
        return;
    }
    if (c.flux2) {
        double Dl[5], Dr[5], ql[5], qr[5];
        case_slope(c, cl, f - 1, Dl);
        case_slope(c, cl, f, Dr);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            ql[k] = Wl[k] + 0.5 * Dl[k];
            qr[k] = Wr[k] - 0.5 * Dr[k];
        }
        // at a wall the ghost's face state mirrors the boundary cell's (no mass or
        // energy through the wall); a reservoir ghost keeps its own state
        if (f == 0 && c.bc_lo != 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) ql[k] = qr[k];
            ql[1] = -qr[1];
        }
        if (f == c.ncells && c.bc_hi != 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) qr[k] = ql[k];
            qr[1] = -ql[1];
        }
        face_flux(c, Wl, Wr, ql, qr, F);
    } else {
        face_flux(c, Wl, Wr, Wl, Wr, F);
    }
}

// First-order flux through local face f of a case, from the start-of-step
// states of global cells g-1 and g (face f = g - cell_base) that the caller
// loaded beforehand, indices clamped to the grid: the same states and ghosts as
// case_face_flux takes (a wall's ghost mirrors the boundary cell, which is g at
// f = 0 and g-1 at f = ncells; a reservoir's is its own state).
__device__ inline void case_face_flux1(const DCase &c, int f, const double (&Wg0)[5], int ok0,
                                       const double (&Wg1)[5], int ok1, double F[5])
{
    double Wl[5], Wr[5];
    int okl = 1, okr = 1;
    if (f > 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) Wl[k] = Wg0[k];
        okl = ok0;
    } else if (c.bc_lo == 0) {
        Wl[0] = c.rho_L; Wl[1] = c.u_L; Wl[2] = 0.0; Wl[3] = 0.0; Wl[4] = c.T_L;
    } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) Wl[k] = Wg1[k];
        Wl[1] = -Wl[1];
        okl = ok1;
    }
    if (f < c.ncells) {
#pragma unroll
        for (int k = 0; k < 5; ++k) Wr[k] = Wg1[k];
        okr = ok1;
    } else if (c.bc_hi == 0) {
        Wr[0] = c.rho_R; Wr[1] = c.u_R; Wr[2] = 0.0; Wr[3] = 0.0; Wr[4] = c.T_R;
    } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) Wr[k] = Wg0[k];
        Wr[1] = -Wr[1];
        okr = ok0;
    }
    if (!(okl && okr)) {
#pragma unroll
        for (int k = 0; k < 5; ++k) F[k] = 0.0;
        return;
    }
    face_flux(c, Wl, Wr, Wl, Wr, F);
}

// ---------------------------------------------------------------------------
// Equal-mass VHS collision of a particle pair held in registers (Appendix A):
// acceptance (c_r/c_max)^(1-2 upsilon), isotropic scattering with
// cos(theta) = 2 u3 - 1, phi = 2 pi u4, the uniforms u_k = w_k 2^-32 from the
// candidate's words.  Returns true when accepted (the velocities are then
// replaced by the post-collision ones).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool collide_vals(T &ui, T &vi, T &wi, T &uj, T &vj, T &wj, double cm,
                                             double accept_exp, uint32_t w2, uint32_t w3, uint32_t w4,
                                             double &seen)
{
    if constexpr (std::is_same<T, double>::value) {
        const double u2 = u01(w2), u3 = u01(w3), u4 = u01(w4);
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
        ui = m0 + 0.5 * r0; vi = m1 + 0.5 * r1; wi = m2 + 0.5 * r2;
        uj = m0 - 0.5 * r0; vj = m1 - 0.5 * r1; wj = m2 - 0.5 * r2;
        return true;
    } else {
        float d0 = ui - uj, d1 = vi - vj, d2 = wi - wj;
        float cr = sqrtf(__fmaf_rn(d0, d0, __fmaf_rn(d1, d1, d2 * d2)));
        seen = fmax(seen, (double)cr);
        // (c_r/c_max)^a as 2^(a log2(c_r/c_max)); a = 1 (hard spheres) and a = 0
        // (Maxwell molecules) exactly
        const float rat = cr / (float)cm, ae = (float)accept_exp;
        const float pa = ae == 1.0f ? rat : (ae == 0.0f ? 1.0f : exp2f(ae * log2f(rat)));
        if (!(u01(w2) < (double)pa)) return false;
        float ct = __fmaf_rn(2.0f, u01f(w3), -1.0f);
        float st = sqrtf(fmaxf(__fmaf_rn(-ct, ct, 1.0f), 0.0f));
        // phi = 2 pi u4: sin and cos of pi (2 u4), whose argument is exact
        float sp, cp;
        sincospif(2.0f * u01f(w4), &sp, &cp);
        float h = 0.5f * cr;
        float r0 = h * st * cp, r1 = h * st * sp, r2 = h * ct;
        float m0 = 0.5f * (ui + uj), m1 = 0.5f * (vi + vj), m2 = 0.5f * (wi + wj);
        ui = m0 + r0; vi = m1 + r1; wi = m2 + r2;
        uj = m0 - r0; vj = m1 - r1; wj = m2 - r2;
        return true;
    }
}

}  // namespace duwp
