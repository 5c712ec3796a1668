/*
 * DUWP CPU oracle -- TEST INFRASTRUCTURE ONLY (see duwp_oracle.h).
 *
 * Plain serial FP64 loops, one stage after another in the order of the
 * paper's algorithm (Sec. 3.4, Steps 1-4), with the DSMC collision term of
 * Appendix A.  Where the paper leaves a choice open, the reading taken is
 * stated at the point of use.  Build with -ffp-contract=off so that every
 * product and sum rounds exactly as written.
 */
#include "duwp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define O_PI 3.14159265358979323846
#define O_TWO_PI 6.28318530717958647692

/* Philox counter tags, one per kind of random draw. */
enum { T_CLS = 1, T_RCNT = 2, T_RVEL = 3, T_NCNT = 4, T_PAIR = 5, T_ICNT = 6, T_IVEL = 7 };

struct orc_state {
    orc_case cs;
    uint32_t key[2];
    /* derived constants */
    double dx, beta, mu_ref, ups, c_ref, coll_k;
    /* canonical particle array, sorted by cell, and its cell offsets */
    int64_t n, cap;
    double *x, *u, *v, *w;
    int64_t *off;
    /* cell arrays */
    double *psi_w;   /* [C*5] wave part */
    double *psi_p;   /* [C*5] particle part of the current canonical array */
    double *cr_max;  /* [C] */
    uint32_t step;
    /* diagnostics of the last step */
    int32_t *d_abs, *d_new, *d_cand, *d_coll;
    int64_t d_inj[2], d_out;
    /* averaging */
    double *avg;
    int64_t avg_count;
};

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32
 * multiplies with Weyl-sequence key increments.                              */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(const orc_state *s, uint32_t a, uint32_t b, uint32_t tag, uint32_t j, uint32_t out[4])
{
    uint32_t ctr[4] = { s->step, a, b, (tag << 16) | j };
    orc_philox(ctr, s->key, out);
}

/* uniform on [0,1) from a 32-bit word */
static double u01(uint32_t r) { return (double)r * (1.0 / 4294967296.0); }

/* floor(r * n / 2^64): a uniform index in [0, n) from a 64-bit word */
static uint64_t mulhi64(uint64_t r, uint64_t n)
{
    return (uint64_t)(((unsigned __int128)r * (unsigned __int128)n) >> 64);
}

/* ------------------------------------------------------------------------ */
/* Gas constants.
 * beta: mean-free-path factor of Eq. lambda (Sec. 4.1) with alpha = 1.
 * Lambda = lambda_ref * rho_ref = m / (sqrt(2) pi d_ref^2): the reference mean
 * free path of Appendix A times its density.  Equating the viscosity form of
 * lambda (Eq. lambda) and the diameter form (Appendix A) at T_ref gives
 * mu_ref = beta * Lambda * sqrt(2 pi R T_ref).  The NTC number density times
 * reference cross-section is sigma_ref n = rho / (sqrt(2) Lambda) (App. A).
 * c_ref is the VHS reference relative speed sqrt(2kT_ref/m_r)/Gamma(2.5-omega)^(0.5/upsilon)
 * with m_r = m/2, i.e. sqrt(4 R T_ref)/Gamma(2.5-omega)^(1/(2 upsilon)).        */
static void derive(orc_state *s)
{
    const orc_case *c = &s->cs;
    s->dx = (c->x_hi - c->x_lo) / (double)c->ncells;
    s->beta = 5.0 * 2.0 * 3.0 / (4.0 * (5.0 - 2.0 * c->omega) * (7.0 - 2.0 * c->omega));
    double Lam;
    if (c->lambda_ref > 0.0) Lam = c->lambda_ref * c->rho_ref;
    else Lam = c->m_mol / (sqrt(2.0) * O_PI * c->d_ref * c->d_ref);
    s->mu_ref = s->beta * Lam * sqrt(O_TWO_PI * c->R * c->T_ref);
    s->coll_k = 1.0 / (sqrt(2.0) * Lam);
    s->ups = c->omega - 0.5;
    if (s->ups != 0.0)
        s->c_ref = sqrt(4.0 * c->R * c->T_ref) / pow(tgamma(2.5 - c->omega), 1.0 / (2.0 * s->ups));
    else
        s->c_ref = 1.0; /* hard spheres: the cross-section does not depend on c_r */
}

void orc_constants(const orc_state *s, double out[6])
{
    out[0] = s->dx; out[1] = s->beta; out[2] = s->mu_ref;
    out[3] = s->ups; out[4] = s->c_ref; out[5] = s->coll_k;
}

static double viscosity(const orc_state *s, double T)
{
    return s->mu_ref * pow(T / s->cs.T_ref, s->cs.omega);   /* mu ~ T^omega */
}

/* Absorption fraction for time step dt against relaxation time tau.
 * Law 0: Eq. p, P = 1 - tau/dt when dt > tau, else 0.
 * Law 1: the QMC probability of being a colliding molecule, 1 - exp(-dt/tau). */
static double absorb_fraction(int law, double dt, double tau)
{
    if (law == 1) return -expm1(-dt / tau);
    return (dt > tau) ? 1.0 - tau / dt : 0.0;
}

/* Primitive state (rho,U,V,W,T) of a conserved vector (rho, rho U, rho V, rho W, rho E)
 * with E = (U^2+V^2+W^2)/2 + 3RT/2 (Sec. 2, Eq. gkt_moment0 with D = 0).
 * Returns 0 for a vacuum cell (rho <= 0 or T <= 0 or not finite). */
static int primitive(const double psi[5], double R, double W[5])
{
    double rho = psi[0];
    if (!(rho > 0.0)) { W[0] = rho; W[1] = W[2] = W[3] = W[4] = 0.0; return 0; }
    double U = psi[1] / rho, V = psi[2] / rho, Wv = psi[3] / rho;
    double e = psi[4] / rho;
    double T = (2.0 / (3.0 * R)) * (e - 0.5 * (U * U + V * V + Wv * Wv));
    W[0] = rho; W[1] = U; W[2] = V; W[3] = Wv; W[4] = T;
    return (T > 0.0) && isfinite(T);
}

/* ------------------------------------------------------------------------ */
/* Wave flux (Sec. 3.3).  Inviscid part: kinetic flux-vector splitting, i.e.
 * the half-range moments of the left and right Maxwellians (the G|_0 term of
 * Eq. ce2).  Viscous part: Navier-Stokes stress and heat flux with the
 * viscosity scaled by the non-equilibrium factor eps, Pr = 2/3 so
 * kappa = (15/4) R mu, central gradients.  The whole flux is weighted by the
 * wave fraction of the interface state (the analogue of 1-exp(-dt/tau) in the
 * at-dt flux for the law used in classification).                            */
void orc_kfvs_half(const double W[5], double R, int32_t sign, double H[5])
{
    double U = W[1], V = W[2], Wv = W[3], th = R * W[4];
    double a = U / sqrt(2.0 * th);
    double A = 0.5 * erfc(-(double)sign * a);
    double B = sqrt(th / O_TWO_PI) * exp(-a * a);
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

double orc_eps(int32_t law, double x)
{
    switch (law) {
    case 1: return x / (2.0 + x);                           /* eps_12 */
    case 2: return 1.0;                                     /* eps_0 */
    case 3: {                                               /* Eq. vp */
        double em = -expm1(-x);                             /* 1 - e^-x */
        return (-2.0 * em + x * (1.0 + exp(-x))) / (x - em);
    }
    default: return 1.0 - x / expm1(x);                     /* eps_1, Eq. vp1 */
    }
}

static int valid_state(const double W[5]) { return W[0] > 0.0 && W[4] > 0.0 && isfinite(W[4]); }

void orc_wave_flux(const orc_state *s, const double Wl[5], const double Wr[5], double F[5])
{
    orc_wave_flux2(s, Wl, Wr, Wl, Wr, F);
}

/* The flux with separate inviscid face states: the KFVS part uses (ql, qr), the
 * weight P_m, the viscosity and the central gradients use the cell states
 * (Wl, Wr).  First order: ql = Wl, qr = Wr. */
void orc_wave_flux2(const orc_state *s, const double Wl[5], const double Wr[5], const double ql[5],
                    const double qr[5], double F[5])
{
    const orc_case *c = &s->cs;
    for (int k = 0; k < 5; ++k) F[k] = 0.0;
    if (!valid_state(Wl) || !valid_state(Wr)) return;
    double Wm[5];
    for (int k = 0; k < 5; ++k) Wm[k] = 0.5 * (Wl[k] + Wr[k]);
    double mu = viscosity(s, Wm[4]);
    double tau = mu / (Wm[0] * c->R * Wm[4]);
    double xr = c->dt / tau;
    double Pm = absorb_fraction(c->classify_law, c->dt, tau);
    if (!(Pm > 0.0)) return;
    double Hp[5], Hm[5];
    orc_kfvs_half(ql, c->R, +1, Hp);
    orc_kfvs_half(qr, c->R, -1, Hm);
    double mue = orc_eps(c->eps_law, xr) * mu;
    double dU = (Wr[1] - Wl[1]) / s->dx;
    double dV = (Wr[2] - Wl[2]) / s->dx;
    double dW = (Wr[3] - Wl[3]) / s->dx;
    double dT = (Wr[4] - Wl[4]) / s->dx;
    double sxx = (4.0 / 3.0) * mue * dU;
    double sxy = mue * dV;
    double sxz = mue * dW;
    double q = -(15.0 / 4.0) * c->R * mue * dT;
    double visc[5] = { 0.0, sxx, sxy, sxz, Wm[1] * sxx + Wm[2] * sxy + Wm[3] * sxz - q };
    for (int k = 0; k < 5; ++k)
        F[k] = Pm * ((ql[0] * Hp[k] + qr[0] * Hm[k]) - visc[k]);
}

static double minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

/* Ghost states beyond the two ends: the reservoir state, or the mirror image of
 * the boundary cell at a wall. */
static void ghost_state(const orc_case *cs, int side, const double Wb[5], double G[5])
{
    const int res = side == 0 ? cs->bc_lo == 0 : cs->bc_hi == 0;
    if (res) {
        G[0] = side == 0 ? cs->rho_L : cs->rho_R;
        G[1] = side == 0 ? cs->u_L : cs->u_R;
        G[2] = 0.0; G[3] = 0.0;
        G[4] = side == 0 ? cs->T_L : cs->T_R;
    } else {
        memcpy(G, Wb, 5 * sizeof(double));
        G[1] = -Wb[1];
    }
}

/* Equal-mass binary collision with isotropic scattering (Appendix A):
 * cos(theta) = 2 u3 - 1, phi = 2 pi u4, post-collision relative velocity of
 * the same magnitude along (theta, phi), centre-of-mass velocity unchanged. */
void orc_scatter_pair(const double xi_i[3], const double xi_j[3], double u3, double u4,
                      double out_i[3], double out_j[3])
{
    double d0 = xi_i[0] - xi_j[0], d1 = xi_i[1] - xi_j[1], d2 = xi_i[2] - xi_j[2];
    double cr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    double ct = 2.0 * u3 - 1.0;
    double st = sqrt(1.0 - ct * ct);
    double ph = O_TWO_PI * u4;
    double r[3] = { cr * st * cos(ph), cr * st * sin(ph), cr * ct };
    for (int k = 0; k < 3; ++k) {
        double m = 0.5 * (xi_i[k] + xi_j[k]);
        out_i[k] = m + 0.5 * r[k];
        out_j[k] = m - 0.5 * r[k];
    }
}

/* Maxwellian velocity by the paper's Eq. maxsample: one independent
 * (cos, log) pair per component, rand -> (1 - u) so the log argument is in (0,1]. */
static void maxwell_sample(double U, double V, double W, double T, double R,
                           const double uu[6], double out[3])
{
    double sd = sqrt(2.0 * R * T);
    double mean[3] = { U, V, W };
    for (int d = 0; d < 3; ++d)
        out[d] = mean[d] + sd * cos(O_TWO_PI * uu[2 * d]) * sqrt(-log(1.0 - uu[2 * d + 1]));
}

/* ------------------------------------------------------------------------ */
/* Grow *p to n doubles; on failure *p is left as it was (still owned by the caller). */
static int regrow(double **p, int64_t n)
{
    double *q = realloc(*p, (size_t)(n ? n : 1) * sizeof(double));
    if (!q) return -1;
    *p = q;
    return 0;
}

static int reserve(orc_state *s, int64_t need)
{
    if (need <= s->cap) return 0;
    int64_t nc = s->cap ? s->cap : 1024;
    while (nc < need) nc *= 2;
    if (regrow(&s->x, nc) || regrow(&s->u, nc) || regrow(&s->v, nc) || regrow(&s->w, nc)) return -1;
    s->cap = nc;
    return 0;
}

/* O1: particle moments per cell, Psi_p = (m_p/dx) sum (1, xi, |xi|^2/2)
 * (Eq. gkt_moment0 for a sum of delta functions), in canonical order. */
static void particle_moments(orc_state *s)
{
    int C = s->cs.ncells;
    double fac = s->cs.m_particle / s->dx;
    for (int c = 0; c < C; ++c) {
        double a[5] = { 0, 0, 0, 0, 0 };
        for (int64_t k = s->off[c]; k < s->off[c + 1]; ++k) {
            double u = s->u[k], v = s->v[k], w = s->w[k];
            a[0] += 1.0;
            a[1] += u;
            a[2] += v;
            a[3] += w;
            a[4] += 0.5 * (u * u + v * v + w * w);
        }
        for (int k = 0; k < 5; ++k) s->psi_p[c * 5 + k] = fac * a[k];
    }
}

static void accumulate_average(orc_state *s)
{
    int C = s->cs.ncells;
    for (int i = 0; i < C * 5; ++i) s->avg[i] += s->psi_w[i] + s->psi_p[i];
    s->avg_count += 1;
}

orc_state *orc_create(const orc_case *cs, uint64_t seed, int32_t case_id)
{
    if (!cs || cs->ncells <= 0 || !(cs->x_hi > cs->x_lo) || !(cs->m_particle > 0) || !(cs->dt > 0))
        return NULL;
    orc_state *s = calloc(1, sizeof(orc_state));
    if (!s) return NULL;
    s->cs = *cs;
    s->key[0] = (uint32_t)seed;
    s->key[1] = (uint32_t)(seed >> 32) + (uint32_t)case_id;
    derive(s);
    int C = cs->ncells;
    s->off = calloc((size_t)C + 1, sizeof(int64_t));
    s->psi_w = calloc((size_t)C * 5, sizeof(double));
    s->psi_p = calloc((size_t)C * 5, sizeof(double));
    s->cr_max = calloc((size_t)C, sizeof(double));
    s->avg = calloc((size_t)C * 5, sizeof(double));
    s->d_abs = calloc((size_t)C, sizeof(int32_t));
    s->d_new = calloc((size_t)C, sizeof(int32_t));
    s->d_cand = calloc((size_t)C, sizeof(int32_t));
    s->d_coll = calloc((size_t)C, sizeof(int32_t));
    if (!s->off || !s->psi_w || !s->psi_p || !s->cr_max || !s->avg || !s->d_abs ||
        !s->d_new || !s->d_cand || !s->d_coll || reserve(s, 1024)) {
        orc_destroy(s);
        return NULL;
    }
    /* Initial state: all mass in the wave part at the cell-centre value of
     * the step profile; no particles yet, so the first resampling creates
     * them.  cr_max starts at 6 sqrt(R T). */
    for (int c = 0; c < C; ++c) {
        double xc = cs->x_lo + ((double)c + 0.5) * s->dx;
        int left = xc < cs->x_split;
        double rho = left ? cs->rho_L : cs->rho_R;
        double U = left ? cs->u_L : cs->u_R;
        double T = left ? cs->T_L : cs->T_R;
        double *p = s->psi_w + c * 5;
        p[0] = rho;
        p[1] = rho * U;
        p[2] = 0.0;
        p[3] = 0.0;
        p[4] = rho * (0.5 * U * U + 1.5 * cs->R * T);
        s->cr_max[c] = 6.0 * sqrt(cs->R * T);
    }
    return s;
}

void orc_destroy(orc_state *s)
{
    if (!s) return;
    free(s->x); free(s->u); free(s->v); free(s->w);
    free(s->off); free(s->psi_w); free(s->psi_p); free(s->cr_max); free(s->avg);
    free(s->d_abs); free(s->d_new); free(s->d_cand); free(s->d_coll);
    free(s);
}

int64_t orc_num_particles(const orc_state *s) { return s->n; }
int32_t orc_num_cells(const orc_state *s) { return s->cs.ncells; }
uint32_t orc_get_step(const orc_state *s) { return s->step; }

int orc_get_state(const orc_state *s, double *x, double *u, double *v, double *w,
                  int64_t *off, double *psi_w, double *cr_max)
{
    int C = s->cs.ncells;
    if (x) memcpy(x, s->x, (size_t)s->n * sizeof(double));
    if (u) memcpy(u, s->u, (size_t)s->n * sizeof(double));
    if (v) memcpy(v, s->v, (size_t)s->n * sizeof(double));
    if (w) memcpy(w, s->w, (size_t)s->n * sizeof(double));
    if (off) memcpy(off, s->off, ((size_t)C + 1) * sizeof(int64_t));
    if (psi_w) memcpy(psi_w, s->psi_w, (size_t)C * 5 * sizeof(double));
    if (cr_max) memcpy(cr_max, s->cr_max, (size_t)C * sizeof(double));
    return 0;
}

int orc_set_state(orc_state *s, int64_t n, const double *x, const double *u,
                  const double *v, const double *w, const int64_t *off,
                  const double *psi_w, const double *cr_max, uint32_t step)
{
    int C = s->cs.ncells;
    if (n < 0 || off[0] != 0 || off[C] != n) return -1;
    for (int c = 0; c < C; ++c) if (off[c + 1] < off[c]) return -1;
    if (reserve(s, n)) return -1;
    s->n = n;
    memcpy(s->x, x, (size_t)n * sizeof(double));
    memcpy(s->u, u, (size_t)n * sizeof(double));
    memcpy(s->v, v, (size_t)n * sizeof(double));
    memcpy(s->w, w, (size_t)n * sizeof(double));
    memcpy(s->off, off, ((size_t)C + 1) * sizeof(int64_t));
    memcpy(s->psi_w, psi_w, (size_t)C * 5 * sizeof(double));
    memcpy(s->cr_max, cr_max, (size_t)C * sizeof(double));
    s->step = step;
    particle_moments(s);
    return 0;
}

void orc_get_diag(const orc_state *s, int32_t *n_abs, int32_t *n_new, int32_t *n_cand,
                  int32_t *n_coll, int64_t *n_inj, int64_t *n_out)
{
    int C = s->cs.ncells;
    if (n_abs) memcpy(n_abs, s->d_abs, (size_t)C * sizeof(int32_t));
    if (n_new) memcpy(n_new, s->d_new, (size_t)C * sizeof(int32_t));
    if (n_cand) memcpy(n_cand, s->d_cand, (size_t)C * sizeof(int32_t));
    if (n_coll) memcpy(n_coll, s->d_coll, (size_t)C * sizeof(int32_t));
    if (n_inj) { n_inj[0] = s->d_inj[0]; n_inj[1] = s->d_inj[1]; }
    if (n_out) *n_out = s->d_out;
}

void orc_get_cells(const orc_state *s, double *prim, double *psi_t, double *psi_p)
{
    int C = s->cs.ncells;
    for (int c = 0; c < C; ++c) {
        double t[5];
        for (int k = 0; k < 5; ++k) t[k] = s->psi_w[c * 5 + k] + s->psi_p[c * 5 + k];
        if (psi_t) memcpy(psi_t + c * 5, t, sizeof t);
        if (psi_p) memcpy(psi_p + c * 5, s->psi_p + c * 5, sizeof t);
        if (prim) primitive(t, s->cs.R, prim + c * 5);
    }
}

/* Normal stress and heat flux of the current state, per cell (Eq. gkt_moment1,
 * xx entry of S and x component of Q for the monatomic gas of the tests):
 * out[c*5 + 0..4] = (Pi, Q, Pi_p, Q_p, rho_w/rho_t).
 *
 * Particle part, about the total state's mean velocity U_t (c = xi - U_t):
 *   Pi_p = (m_p/dx) sum (c_x^2 - |c|^2/3),  Q_p = (m_p/dx) sum c_x |c|^2 / 2.
 * Pi_p is the xx entry of rho cc(f - g) for the particles with the trace
 * removed.  The wave part is taken as a Maxwellian at the cell's total
 * velocity (no deviatoric stress, no heat flux) plus the NS closure that its
 * flux carries (Sec. 3.3), weighted like that flux by the cell's absorbed
 * fraction P_c:
 *   Pi_w = -P_c (4/3) eps mu dU/dx,  Q_w = -P_c (15/4) R eps mu dT/dx,
 * with eps and P_c of the cell's state, and central differences over the
 * neighbouring cells (the flux's ghost states beyond the ends).  A vacuum cell,
 * or a vacuum neighbour, gives no wave term. */
int orc_stress_heat(const orc_state *s, double *out)
{
    const orc_case *cs = &s->cs;
    const int C = cs->ncells;
    const double fac = cs->m_particle / s->dx;
    double *W = malloc(((size_t)C + 2) * 5 * sizeof(double));
    int *ok = malloc(((size_t)C + 2) * sizeof(int));
    if (!W || !ok) { free(W); free(ok); return -1; }
    /* W[1..C] the cells, W[0] and W[C+1] the ghost states */
    for (int c = 0; c < C; ++c) {
        double t[5];
        for (int k = 0; k < 5; ++k) t[k] = s->psi_w[c * 5 + k] + s->psi_p[c * 5 + k];
        ok[c + 1] = primitive(t, cs->R, W + (c + 1) * 5);
    }
    if (cs->bc_lo == 0) {
        W[0] = cs->rho_L; W[1] = cs->u_L; W[2] = 0.0; W[3] = 0.0; W[4] = cs->T_L; ok[0] = 1;
    } else {
        memcpy(W, W + 5, 5 * sizeof(double)); W[1] = -W[6]; ok[0] = ok[1];
    }
    double *Wg = W + (C + 1) * 5, *Wl = W + C * 5;
    if (cs->bc_hi == 0) {
        Wg[0] = cs->rho_R; Wg[1] = cs->u_R; Wg[2] = 0.0; Wg[3] = 0.0; Wg[4] = cs->T_R; ok[C + 1] = 1;
    } else {
        memcpy(Wg, Wl, 5 * sizeof(double)); Wg[1] = -Wl[1]; ok[C + 1] = ok[C];
    }
    for (int c = 0; c < C; ++c) {
        const double *Wc = W + (c + 1) * 5;
        double *o = out + (size_t)c * 5;
        for (int k = 0; k < 5; ++k) o[k] = 0.0;
        if (!ok[c + 1]) continue;
        const double U = Wc[1], V = Wc[2], Wv = Wc[3];
        double sxx = 0.0, scc = 0.0, sq = 0.0;
        for (int64_t k = s->off[c]; k < s->off[c + 1]; ++k) {
            const double cx = s->u[k] - U, cy = s->v[k] - V, cz = s->w[k] - Wv;
            const double c2 = cx * cx + cy * cy + cz * cz;
            sxx += cx * cx;
            scc += c2;
            sq += cx * c2;
        }
        const double pip = fac * (sxx - scc / 3.0);
        const double qp = fac * 0.5 * sq;
        double piw = 0.0, qw = 0.0;
        if (ok[c] && ok[c + 2]) {
            const double mu = viscosity(s, Wc[4]);
            const double tau = mu / (Wc[0] * cs->R * Wc[4]);
            const double P = absorb_fraction(cs->classify_law, cs->dt, tau);
            const double mue = orc_eps(cs->eps_law, cs->dt / tau) * mu;
            const double dU = (W[(c + 2) * 5 + 1] - W[c * 5 + 1]) / (2.0 * s->dx);
            const double dT = (W[(c + 2) * 5 + 4] - W[c * 5 + 4]) / (2.0 * s->dx);
            piw = -P * (4.0 / 3.0) * mue * dU;
            qw = -P * (15.0 / 4.0) * cs->R * mue * dT;
        }
        o[0] = pip + piw;
        o[1] = qp + qw;
        o[2] = pip;
        o[3] = qp;
        o[4] = s->psi_w[c * 5] / Wc[0];
    }
    free(W);
    free(ok);
    return 0;
}

void orc_get_average(const orc_state *s, double *avg_sum, int64_t *count)
{
    if (avg_sum) memcpy(avg_sum, s->avg, (size_t)s->cs.ncells * 5 * sizeof(double));
    if (count) *count = s->avg_count;
}

void orc_reset_average(orc_state *s)
{
    memset(s->avg, 0, (size_t)s->cs.ncells * 5 * sizeof(double));
    s->avg_count = 0;
}

/* Apply the boundaries to a streamed particle.  Reservoir: leaving the
 * domain deletes it.  Specular wall: mirror position and normal velocity
 * until inside.  Returns 0 when deleted (or stuck after 1000 reflections,
 * or with a position that is not a finite number). */
static int apply_bc(const orc_case *c, double *x, double *u)
{
    for (int it = 0; it < 1000; ++it) {
        if (!isfinite(*x)) return 0;
        if (*x < c->x_lo) {
            if (c->bc_lo == 0) return 0;
            *x = 2.0 * c->x_lo - *x;
            *u = -*u;
        } else if (*x > c->x_hi) {
            if (c->bc_hi == 0) return 0;
            *x = 2.0 * c->x_hi - *x;
            *u = -*u;
        } else {
            return 1;
        }
    }
    return 0;
}

static int64_t cell_of(const orc_state *s, double x)
{
    double f = floor((x - s->cs.x_lo) / s->dx);
    int64_t c = (int64_t)f;
    if (f < 0.0) c = 0;
    if (c > s->cs.ncells - 1) c = s->cs.ncells - 1;
    return c;
}

typedef struct { double x, u, v, w; int64_t cell; } ipart;

/* Double the intermediate array; on failure it is left as it was. */
static int grow(ipart **ib, int64_t *icap)
{
    ipart *q = realloc(*ib, (size_t)(*icap * 2) * sizeof(ipart));
    if (!q) return -1;
    *ib = q;
    *icap *= 2;
    return 0;
}

/* One DUWP step (Sec. 3.4, Steps 2-3) over the stages in mask. */
int orc_step_masked(orc_state *s, int32_t mask)
{
    const orc_case *cs = &s->cs;
    const int C = cs->ncells;
    const double R = cs->R, dt = cs->dt, dx = s->dx;
    const double fac = cs->m_particle / dx;
    int err = 0;

    /* ---- O1: total state per cell, Psi_t = Psi_w + Psi_p (Step 1). ---- */
    double *Wt = malloc((size_t)C * 5 * sizeof(double));
    double *Pc = malloc((size_t)C * sizeof(double));
    int *ok = malloc((size_t)C * sizeof(int));
    double *psi_w0 = malloc((size_t)C * sizeof(double));   /* start-of-step rho_w */
    double *tauc = calloc((size_t)C, sizeof(double));       /* tau = mu/p of the total state */
    /* absorb_stream: moments of absorbed particles that reached another cell,
     * by the cell reached (sources in ascending order), and whether any did */
    double *wab = calloc((size_t)C * 5, sizeof(double));
    int *wabin = calloc((size_t)C, sizeof(int));
    /* intermediate array and the wave-update and sort buffers (below) */
    ipart *ib = NULL;
    int64_t *ioff = NULL, *cnt = NULL;
    double *F = NULL, *D = NULL;
    if (!Wt || !Pc || !ok || !psi_w0 || !tauc || !wab || !wabin) { err = -1; goto done; }
    for (int c = 0; c < C; ++c) {
        double t[5];
        for (int k = 0; k < 5; ++k) t[k] = s->psi_w[c * 5 + k] + s->psi_p[c * 5 + k];
        ok[c] = primitive(t, R, Wt + c * 5);
        psi_w0[c] = s->psi_w[c * 5 + 0];
        if (ok[c]) {
            double T = Wt[c * 5 + 4];
            double tau = viscosity(s, T) / (Wt[c * 5 + 0] * R * T);   /* tau = mu/p */
            Pc[c] = absorb_fraction(cs->classify_law, dt, tau);
            tauc[c] = tau;
        } else {
            Pc[c] = 0.0;
        }
        s->d_abs[c] = s->d_new[c] = s->d_cand[c] = s->d_coll[c] = 0;
    }
    s->d_inj[0] = s->d_inj[1] = 0;
    s->d_out = 0;

    /* Intermediate array: per cell [survivors in canonical order][new by slot],
     * then injected entrants.  Sized generously and grown as needed. */
    int64_t icap = s->n + 1024, ni = 0;
    ib = malloc((size_t)icap * sizeof(ipart));
    ioff = malloc(((size_t)C + 1) * sizeof(int64_t));
    if (!ib || !ioff) { err = -1; goto done; }

    for (int c = 0; c < C; ++c) {
        ioff[c] = ni;
        double P = Pc[c];
        /* ---- O2/O3: classify and absorb (Step 2, Eq. p).  A particle whose
         * sampled free-transport time tau/(1-u) is shorter than dt, i.e.
         * u < P, is absorbed: its moments join the wave part and it is
         * removed.  Absorbed particles do not stream; with absorb_stream they
         * first stream for that free time (-tau ln(1-u) under the exponential
         * law) and join the wave part of the cell they reach, or leave the
         * domain through a reservoir. ---- */
        double sa[5] = { 0, 0, 0, 0, 0 };
        int32_t nabs = 0;
        for (int64_t k = s->off[c]; k < s->off[c + 1]; ++k) {
            int absorbed = 0;
            if ((mask & ORC_CLASSIFY) && P > 0.0) {
                /* one Philox block serves four consecutive particles */
                uint32_t r[4];
                draw(s, (uint32_t)(k >> 2), 0, T_CLS, 0, r);
                absorbed = u01(r[k & 3]) < P;
            }
            if (absorbed) {
                double u = s->u[k], v = s->v[k], w = s->w[k];
                int64_t cland = c;
                if (cs->absorb_stream) {
                    uint32_t r[4];
                    draw(s, (uint32_t)(k >> 2), 0, T_CLS, 0, r);
                    double uc = u01(r[k & 3]);
                    double tf = cs->classify_law == 1 ? -tauc[c] * log(1.0 - uc) : tauc[c] / (1.0 - uc);
                    double x = s->x[k] + u * tf;
                    cland = apply_bc(cs, &x, &u) ? cell_of(s, x) : -1;
                }
                ++nabs;
                if (cland < 0) {
                    s->d_out++;
                } else if (cland == c) {
                    sa[0] += 1.0; sa[1] += u; sa[2] += v; sa[3] += w;
                    sa[4] += 0.5 * (u * u + v * v + w * w);
                } else {
                    double *a = wab + cland * 5;
                    a[0] += 1.0; a[1] += u; a[2] += v; a[3] += w;
                    a[4] += 0.5 * (u * u + v * v + w * w);
                    wabin[cland] = 1;
                }
            } else {
                if (ni >= icap && grow(&ib, &icap)) { err = -1; goto done; }
                ipart p = { s->x[k], s->u[k], s->v[k], s->w[k], c };
                ib[ni++] = p;
            }
        }
        s->d_abs[c] = nabs;
        if (nabs)
            for (int k = 0; k < 5; ++k) s->psi_w[c * 5 + k] += fac * sa[k];

        /* ---- O4: resample 1-P of the start-of-step wave mass as particles
         * from the Maxwellian of the total state (Eq. maxsample), stochastic
         * rounding of the count, at most the whole wave mass; the exact
         * sampled moments leave the wave part so Psi_t is unchanged. ---- */
        if ((mask & ORC_RESAMPLE) && ok[c]) {
            double Mw = dx * psi_w0[c];
            uint32_t r[4];
            draw(s, (uint32_t)c, 0, T_RCNT, 0, r);
            double nf = floor((1.0 - P) * Mw / cs->m_particle + u01(r[0]));
            double cap = floor((Mw > 0.0 ? Mw : 0.0) / cs->m_particle);
            if (nf > cap) nf = cap;
            if (nf < 0.0) nf = 0.0;
            if (nf > 2.0e9) { err = -1; nf = 0.0; }
            int64_t nnew = (int64_t)nf;
            const double *Wc = Wt + c * 5;
            double ss[5] = { 0, 0, 0, 0, 0 };
            for (int64_t q = 0; q < nnew; ++q) {
                uint32_t a[4], b[4];
                draw(s, (uint32_t)c, (uint32_t)q, T_RVEL, 0, a);
                draw(s, (uint32_t)c, (uint32_t)q, T_RVEL, 1, b);
                double uu[6] = { u01(a[1]), u01(a[2]), u01(a[3]), u01(b[0]), u01(b[1]), u01(b[2]) };
                double xi[3];
                maxwell_sample(Wc[1], Wc[2], Wc[3], Wc[4], R, uu, xi);
                ipart p = { cs->x_lo + ((double)c + u01(a[0])) * dx, xi[0], xi[1], xi[2], c };
                if (ni >= icap && grow(&ib, &icap)) { err = -1; goto done; }
                ib[ni++] = p;
                ss[0] += 1.0; ss[1] += xi[0]; ss[2] += xi[1]; ss[3] += xi[2];
                ss[4] += 0.5 * (xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
            }
            s->d_new[c] = (int32_t)nnew;
            if (nnew)
                for (int k = 0; k < 5; ++k) s->psi_w[c * 5 + k] -= fac * ss[k];
        }

        /* ---- O5: DSMC no-time-counter collisions among the cell's particles
         * (Appendix A) over the single-collision duration (1-P) dt, with the
         * number density of the total state.  Candidates are processed in
         * order; each one sees the velocities left by the earlier ones. ---- */
        int64_t Nc = ni - ioff[c];
        if ((mask & ORC_COLLIDE) && ok[c] && Nc >= 2) {
            double dtc = cs->dsmc_full_dt ? dt : (1.0 - P) * dt;
            double cm = s->cr_max[c];
            double seen = 0.0;
            double Mr = 0.5 * (double)(Nc - 1) * s->coll_k * Wt[c * 5 + 0]
                        * pow(s->c_ref / cm, 2.0 * s->ups) * cm * dtc;
            uint32_t r[4];
            draw(s, (uint32_t)c, 0, T_NCNT, 0, r);
            double Mf = floor(Mr + u01(r[0]));
            if (Mf > 2.0e9) { err = -1; Mf = 0.0; }
            int64_t M = (int64_t)Mf;
            int32_t ncoll = 0;
            ipart *seg = ib + ioff[c];
            for (int64_t q = 0; q < M; ++q) {
                uint32_t a[4], b[4];
                draw(s, (uint32_t)c, (uint32_t)q, T_PAIR, 0, a);
                draw(s, (uint32_t)c, (uint32_t)q, T_PAIR, 1, b);
                uint64_t r0 = ((uint64_t)a[0] << 32) | a[1];
                uint64_t r1 = ((uint64_t)a[2] << 32) | a[3];
                uint64_t i = mulhi64(r0, (uint64_t)Nc);
                uint64_t j = mulhi64(r1, (uint64_t)(Nc - 1));
                if (j >= i) j += 1;
                ipart *pi = seg + i, *pj = seg + j;
                double d0 = pi->u - pj->u, d1 = pi->v - pj->v, d2 = pi->w - pj->w;
                double cr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                if (cr > seen) seen = cr;
                /* VHS acceptance sigma c_r / (sigma c_r)_max = (c_r/c_max)^(1-2 upsilon) */
                double pa = pow(cr / cm, 1.0 - 2.0 * s->ups);
                if (u01(b[0]) < pa) {
                    double xi_i[3] = { pi->u, pi->v, pi->w }, xi_j[3] = { pj->u, pj->v, pj->w };
                    double oi[3], oj[3];
                    orc_scatter_pair(xi_i, xi_j, u01(b[1]), u01(b[2]), oi, oj);
                    pi->u = oi[0]; pi->v = oi[1]; pi->w = oi[2];
                    pj->u = oj[0]; pj->v = oj[1]; pj->w = oj[2];
                    ++ncoll;
                }
            }
            s->d_cand[c] = (int32_t)M;
            s->d_coll[c] = ncoll;
            if (seen > cm) s->cr_max[c] = seen;
        }
    }
    ioff[C] = ni;
    /* absorbed moments that reached other cells join their wave parts */
    for (int c = 0; c < C; ++c)
        if (wabin[c])
            for (int k = 0; k < 5; ++k) s->psi_w[c * 5 + k] += fac * wab[c * 5 + k];

    /* ---- O6: free transport x <- x + xi dt (Step 3), boundaries, and
     * reservoir injection from ghost slabs beyond each reservoir side. ---- */
    int64_t kept = 0;
    for (int64_t k = 0; k < ni; ++k) {
        ipart p = ib[k];
        if (mask & ORC_STREAM) {
            p.x = p.x + p.u * dt;
            if (!apply_bc(cs, &p.x, &p.u)) { s->d_out++; continue; }
        }
        p.cell = cell_of(s, p.x);
        ib[kept++] = p;
    }
    ni = kept;
    if (mask & ORC_STREAM) {
        for (int side = 0; side < 2; ++side) {
            if ((side == 0 ? cs->bc_lo : cs->bc_hi) != 0) continue;
            double rho = side == 0 ? cs->rho_L : cs->rho_R;
            double U = side == 0 ? cs->u_L : cs->u_R;
            double T = side == 0 ? cs->T_L : cs->T_R;
            double tau = viscosity(s, T) / (rho * R * T);
            double Ps = absorb_fraction(cs->classify_law, dt, tau);
            double Lg = dt * (fabs(U) + 8.0 * sqrt(R * T));
            uint32_t r[4];
            draw(s, (uint32_t)side, 0, T_ICNT, 0, r);
            double nf = floor((1.0 - Ps) * rho * Lg / cs->m_particle + u01(r[0]));
            if (nf > 2.0e9) { err = -1; nf = 0.0; }
            int64_t ng = (int64_t)nf;
            for (int64_t q = 0; q < ng; ++q) {
                uint32_t a[4], b[4];
                draw(s, (uint32_t)side, (uint32_t)q, T_IVEL, 0, a);
                draw(s, (uint32_t)side, (uint32_t)q, T_IVEL, 1, b);
                double uu[6] = { u01(a[1]), u01(a[2]), u01(a[3]), u01(b[0]), u01(b[1]), u01(b[2]) };
                double xi[3];
                maxwell_sample(U, 0.0, 0.0, T, R, uu, xi);
                ipart p;
                p.x = side == 0 ? cs->x_lo - u01(a[0]) * Lg : cs->x_hi + u01(a[0]) * Lg;
                p.u = xi[0]; p.v = xi[1]; p.w = xi[2];
                p.x = p.x + p.u * dt;
                if (!apply_bc(cs, &p.x, &p.u)) continue;
                p.cell = cell_of(s, p.x);
                if (ni >= icap && grow(&ib, &icap)) { err = -1; goto done; }
                ib[ni++] = p;
                s->d_inj[side]++;
            }
        }
    }

    /* ---- O8: wave-part update with the NS flux of the start-of-step total
     * state (Eq. r1, wave term).  Ghost states: the reservoir state, or the
     * mirror image of the boundary cell at a wall. ---- */
    if (mask & ORC_WAVE) {
        F = calloc(((size_t)C + 1) * 5, sizeof(double));
        D = calloc((size_t)C * 5, sizeof(double));
        if (!F || !D) { err = -1; goto done; }
        double G0[5], G1[5];
        ghost_state(cs, 0, Wt, G0);
        ghost_state(cs, 1, Wt + (C - 1) * 5, G1);
        const int okg0 = cs->bc_lo == 0 || ok[0], okg1 = cs->bc_hi == 0 || ok[C - 1];
        /* second order (flux_order 2): minmod slopes of the primitive state of each
         * cell from its two neighbours (the ghost states beyond the ends); a vacuum
         * cell or neighbour gives no slope */
        if (cs->flux_order == 2) {
            for (int c = 0; c < C; ++c) {
                const double *Wm = c == 0 ? G0 : Wt + (c - 1) * 5;
                const double *Wp = c == C - 1 ? G1 : Wt + (c + 1) * 5;
                const int okm = c == 0 ? okg0 : ok[c - 1], okp = c == C - 1 ? okg1 : ok[c + 1];
                if (!(ok[c] && okm && okp)) continue;
                for (int k = 0; k < 5; ++k)
                    D[c * 5 + k] = minmod(Wt[c * 5 + k] - Wm[k], Wp[k] - Wt[c * 5 + k]);
            }
        }
        for (int f = 0; f <= C; ++f) {
            double Wl[5], Wr[5], ql[5], qr[5];
            memcpy(Wl, f == 0 ? G0 : Wt + (f - 1) * 5, sizeof Wl);
            memcpy(Wr, f == C ? G1 : Wt + f * 5, sizeof Wr);
            /* inviscid face states: the cells' reconstructions; a reservoir ghost
             * has none, and at a wall the ghost's face state is the mirror image
             * of the boundary cell's, so that no mass or energy crosses the wall */
            for (int k = 0; k < 5; ++k) {
                ql[k] = f == 0 ? Wl[k] : Wl[k] + 0.5 * D[(f - 1) * 5 + k];
                qr[k] = f == C ? Wr[k] : Wr[k] - 0.5 * D[f * 5 + k];
            }
            if (f == 0 && cs->bc_lo != 0) { memcpy(ql, qr, sizeof ql); ql[1] = -qr[1]; }
            if (f == C && cs->bc_hi != 0) { memcpy(qr, ql, sizeof qr); qr[1] = -ql[1]; }
            /* an interface touching a vacuum cell carries no wave flux */
            int okl = (f == 0) ? okg0 : ok[f - 1];
            int okr = (f == C) ? okg1 : ok[f];
            if (okl && okr) orc_wave_flux2(s, Wl, Wr, ql, qr, F + f * 5);
        }
        double r = dt / dx;
        for (int c = 0; c < C; ++c)
            for (int k = 0; k < 5; ++k)
                s->psi_w[c * 5 + k] -= r * (F[(c + 1) * 5 + k] - F[c * 5 + k]);
    }

    /* ---- O7: stable counting sort of the intermediate array by cell; the
     * result is the next canonical array. ---- */
    if (reserve(s, ni)) { err = -1; goto done; }
    cnt = calloc((size_t)C + 1, sizeof(int64_t));
    if (!cnt) { err = -1; goto done; }
    for (int64_t k = 0; k < ni; ++k) cnt[ib[k].cell + 1]++;
    for (int c = 0; c < C; ++c) cnt[c + 1] += cnt[c];
    memcpy(s->off, cnt, ((size_t)C + 1) * sizeof(int64_t));
    for (int64_t k = 0; k < ni; ++k) {
        int64_t d = cnt[ib[k].cell]++;
        s->x[d] = ib[k].x; s->u[d] = ib[k].u; s->v[d] = ib[k].v; s->w[d] = ib[k].w;
    }
    s->n = ni;

    /* ---- O9: moments of the new state and the running average of Psi_t. ---- */
    particle_moments(s);
    accumulate_average(s);
    s->step += 1;
done:
    free(cnt); free(F); free(D); free(ib); free(ioff);
    free(Wt); free(Pc); free(ok); free(psi_w0); free(tauc); free(wab); free(wabin);
    return err;
}

int orc_step(orc_state *s, int32_t nsteps)
{
    for (int32_t i = 0; i < nsteps; ++i)
        if (orc_step_masked(s, ORC_ALL)) return -1;
    return 0;
}
