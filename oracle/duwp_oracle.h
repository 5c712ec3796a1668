/*
 * DUWP CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, FP64 implementation of one time step of the direct unified
 * wave-particle (DUWP) method for 1D monatomic gas with 3D velocities
 * (Cao, Liu, Yang, Zhong, "A direct unified wave-particle method for
 * simulating non-equilibrium flows", arXiv 2305.12071).  It exists so that the
 * GPU path can be checked against it; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header or
 * constant table with the GPU library.
 *
 * Every random draw is a Philox4x32-10 block (Salmon et al., SC'11) keyed by
 * (seed, case) with counter (step, a, b, tag<<16 | draw), so a state plus a
 * step number fully determines the next state.
 */
#ifndef DUWP_ORACLE_H
#define DUWP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Case description (inputs only; every derived constant is computed inside). */
typedef struct {
    int32_t kind;          /* 0 shock, 1 Sod, 2 box: informational only */
    int32_t ncells;
    double x_lo, x_hi, x_split;
    double rho_L, u_L, T_L, rho_R, u_R, T_R;
    double R, omega, T_ref;
    double m_mol, d_ref;        /* dimensional gas ...                          */
    double lambda_ref, rho_ref; /* ... or nondimensional (used when lambda_ref>0) */
    double m_particle, dt;
    int32_t bc_lo, bc_hi;       /* 0 reservoir, 1 specular wall */
    int32_t classify_law;       /* 0 P = max(0,1-tau/dt) (Eq. p); 1 P = 1-exp(-dt/tau) */
    int32_t eps_law;            /* 0 eps_1, 1 eps_12, 2 eps_0, 3 eps of Eq. vp */
    int32_t dsmc_full_dt;       /* 1: collide over dt instead of (1-P) dt */
    int32_t flux_order;         /* 2: MUSCL-minmod inviscid face states; else first order */
    int32_t absorb_stream;      /* 1: an absorbed particle streams for its free time first */
} orc_case;

typedef struct orc_state orc_state;

/* Stage mask for orc_step: moments (O1) and the sort/commit (O7) always run. */
enum {
    ORC_CLASSIFY = 1 << 0,   /* O2 + O3 */
    ORC_RESAMPLE = 1 << 1,   /* O4 */
    ORC_COLLIDE  = 1 << 2,   /* O5 */
    ORC_STREAM   = 1 << 3,   /* O6 (free flight, boundaries, injection) */
    ORC_WAVE     = 1 << 4,   /* O8 */
    ORC_ALL      = 0x1f
};

orc_state *orc_create(const orc_case *cs, uint64_t seed, int32_t case_id);
void orc_destroy(orc_state *s);

int64_t orc_num_particles(const orc_state *s);
int32_t orc_num_cells(const orc_state *s);
uint32_t orc_get_step(const orc_state *s);

/* Copy the state out / in.  Arrays: x,u,v,w [n]; off [ncells+1]; psi_w [ncells*5];
 * cr_max [ncells].  set_state recomputes the particle moments. Returns 0 on success. */
int orc_get_state(const orc_state *s, double *x, double *u, double *v, double *w,
                  int64_t *off, double *psi_w, double *cr_max);
int orc_set_state(orc_state *s, int64_t n, const double *x, const double *u,
                  const double *v, const double *w, const int64_t *off,
                  const double *psi_w, const double *cr_max, uint32_t step);

/* Run nsteps full steps (stage mask ORC_ALL) or one masked step. Returns 0, or -1 on error. */
int orc_step(orc_state *s, int32_t nsteps);
int orc_step_masked(orc_state *s, int32_t mask);

/* Per-cell integers of the last step: absorbed, resampled, NTC candidates, accepted collisions. */
void orc_get_diag(const orc_state *s, int32_t *n_abs, int32_t *n_new, int32_t *n_cand,
                  int32_t *n_coll, int64_t *n_inj /*[2]*/, int64_t *n_out);

/* Cell macroscopic state of the current canonical state: [ncells*5] (rho,U,V,W,T),
 * total Psi_t [ncells*5], wave Psi_w is in get_state. */
void orc_get_cells(const orc_state *s, double *prim, double *psi_t, double *psi_p);

/* Time average of Psi_t accumulated after each step since the last reset. */
void orc_get_average(const orc_state *s, double *avg_sum, int64_t *count);
/* Normal stress and heat flux per cell: out[C*5] = (Pi, Q, Pi_p, Q_p, rho_w/rho_t). */
int orc_stress_heat(const orc_state *s, double *out);
void orc_reset_average(orc_state *s);

/* ---- Elementary operations, exposed for the closed-form checks ---- */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_eps(int32_t law, double x);
/* Half-range Maxwellian flux per unit density, sign=+1 (xi>0) or -1. W=(rho,U,V,W,T). */
void orc_kfvs_half(const double W[5], double R, int32_t sign, double H[5]);
/* Wave flux at one interface from left/right primitive states. */
void orc_wave_flux(const orc_state *s, const double Wl[5], const double Wr[5], double F[5]);
void orc_wave_flux2(const orc_state *s, const double Wl[5], const double Wr[5], const double ql[5],
                    const double qr[5], double F[5]);
/* Post-collision velocities of an equal-mass pair for given uniforms (u3: cos theta, u4: phi). */
void orc_scatter_pair(const double xi_i[3], const double xi_j[3], double u3, double u4,
                      double out_i[3], double out_j[3]);
/* Derived constants: [dx, beta, mu_ref, upsilon, c_ref, coll_k]. */
void orc_constants(const orc_state *s, double out[6]);

#ifdef __cplusplus
}
#endif
#endif
