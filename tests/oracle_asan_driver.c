/*
 * Drives the CPU oracle through every entry point for a list of cases, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure; compiled and run by tests/test_oracle_sanitized.py).
 *
 * Input (stdin): a step count, then one case per line as the fields of
 * orc_case in declaration order.  For each case: create, step, read the cells,
 * average, stress and heat flux, diagnostics, save the state and load it into
 * a second oracle, step both, destroy both.  Exit status 0 when every call
 * succeeded.
 */
#include <stdio.h>
#include <stdlib.h>

#include "duwp_oracle.h"

static int read_case(orc_case *c)
{
    int n = scanf("%d %d %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %d %d %d %d %d %d %d",
                  &c->kind, &c->ncells, &c->x_lo, &c->x_hi, &c->x_split, &c->rho_L, &c->u_L, &c->T_L,
                  &c->rho_R, &c->u_R, &c->T_R, &c->R, &c->omega, &c->T_ref, &c->m_mol, &c->d_ref,
                  &c->lambda_ref, &c->rho_ref, &c->m_particle, &c->dt, &c->bc_lo, &c->bc_hi,
                  &c->classify_law, &c->eps_law, &c->dsmc_full_dt, &c->flux_order, &c->absorb_stream);
    return n == 27;
}

int main(void)
{
    int steps = 0, ncase = 0;
    if (scanf("%d", &steps) != 1) return 2;
    orc_case c;
    while (read_case(&c)) {
        orc_state *a = orc_create(&c, 7, ncase);
        if (!a) { fprintf(stderr, "case %d: create failed\n", ncase); return 3; }
        if (orc_step(a, steps)) { fprintf(stderr, "case %d: step failed\n", ncase); return 4; }
        const int C = orc_num_cells(a);
        const int64_t n = orc_num_particles(a);
        double *cells = malloc(sizeof(double) * 5 * (size_t)C * 4);
        int32_t *di = malloc(sizeof(int32_t) * 4 * (size_t)C);
        double *x = malloc(sizeof(double) * 4 * (size_t)(n + 1));
        int64_t *off = malloc(sizeof(int64_t) * (size_t)(C + 1));
        double *cr = malloc(sizeof(double) * (size_t)C);
        if (!cells || !di || !x || !off || !cr) return 5;
        int64_t cnt = 0, inj[2], nout = 0;
        orc_get_cells(a, cells, cells + 5 * C, cells + 10 * C);
        orc_get_average(a, cells, &cnt);
        if (orc_stress_heat(a, cells + 15 * C)) return 6;
        orc_get_diag(a, di, di + C, di + 2 * C, di + 3 * C, inj, &nout);
        orc_get_state(a, x, x + n, x + 2 * n, x + 3 * n, off, cells, cr);
        orc_state *b = orc_create(&c, 7, ncase);
        if (!b) return 7;
        if (orc_set_state(b, n, x, x + n, x + 2 * n, x + 3 * n, off, cells, cr, orc_get_step(a))) return 8;
        if (orc_step(a, 2) || orc_step(b, 2)) return 9;
        if (orc_num_particles(a) != orc_num_particles(b)) { fprintf(stderr, "case %d: resume differs\n", ncase); return 10; }
        orc_reset_average(b);
        orc_destroy(a);
        orc_destroy(b);
        free(cells); free(di); free(x); free(off); free(cr);
        printf("case %d: %d cells, %lld particles, %d+2 steps\n", ncase, C, (long long)n, steps);
        ++ncase;
    }
    return ncase > 0 ? 0 : 11;
}
