/*
 * sanitize_main.c -- driver that runs the CPU oracle (lbmref.c) under the address and
 * undefined-behaviour sanitizers.  TEST INFRASTRUCTURE ONLY, like the oracle itself.
 *
 * Usage: lbmref_sanitize <case file>.  The case file is text:
 *   nx ny nz wall_z0 init_mode film_height steps n_caps body_force_x wall_drho tau0 tau1
 *   coupling node_mass
 *   per capsule: n_nodes n_tri ks C kb kv wet_drho anchor_k, then n_nodes lines "x y z"
 *   and n_tri lines "a b c".
 * It builds the simulation, steps it, and prints the summary, the capsule observables and
 * the meniscus (count and sum of the finite heights), one value per line as "key value",
 * so a test can compare them with the regular build of the same oracle.  It also calls
 * every pure helper of lbmref.h once on the first capsule's mesh.  Exit status 0 on
 * success; the sanitizers abort on the first finding.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbmref.h"

static int read_case(FILE *fp, lbmref_params *p, int *steps, int *ncaps) {
    int wall, mode, coupling;
    double film, gx, drho, t0, t1, mass;
    if (fscanf(fp, "%d %d %d %d %d %lf %d %d %lf %lf %lf %lf %d %lf", &p->nx, &p->ny, &p->nz,
               &wall, &mode, &film, steps, ncaps, &gx, &drho, &t0, &t1, &coupling, &mass) != 14)
        return -1;
    p->coupling = coupling;
    p->node_mass = mass;
    p->wall_z0 = wall;
    p->init_mode = mode;
    p->film_height = film;
    p->body_force[0] = gx;
    p->wall_drho = drho;
    p->tau[0] = t0;
    p->tau[1] = t1;
    return 0;
}

int main(int argc, char **argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s <case file>\n", argv[0]);
        return 2;
    }
    FILE *fp = fopen(argv[1], "r");
    if (!fp) return 2;
    lbmref_params p;
    memset(&p, 0, sizeof p);
    p.G = 3.6; p.rho0 = 1.0; p.sc_norm = 1.0; p.n_threads = 2;
    p.init_rho[0] = 1.0; p.init_rho[1] = 1.0;
    p.rho_maj = 0.7; p.rho_min = 0.04; p.rho_iface = 0.3;
    p.hertz_xi = 1.5; p.hertz_delta0 = 1.5; p.plane_dz = 2.0;
    int steps = 0, ncaps = 0;
    if (read_case(fp, &p, &steps, &ncaps) != 0) return 2;
    lbmref_handle *h = lbmref_create(&p);
    if (!h) {
        fprintf(stderr, "create: %s\n", lbmref_error());
        return 3;
    }
    double *x0 = NULL;
    int32_t *t0 = NULL, nn0 = 0, nt0 = 0;
    lbmref_capsule_params cp0;
    memset(&cp0, 0, sizeof cp0);
    for (int k = 0; k < ncaps; ++k) {
        int nn, nt;
        lbmref_capsule_params cp;
        if (fscanf(fp, "%d %d %lf %lf %lf %lf %lf %lf", &nn, &nt, &cp.ks, &cp.C, &cp.kb, &cp.kv,
                   &cp.wet_drho, &cp.anchor_k) != 8)
            return 2;
        double *x = (double *)malloc(sizeof(double) * 3 * nn);
        int32_t *t = (int32_t *)malloc(sizeof(int32_t) * 3 * nt);
        for (int i = 0; i < 3 * nn; ++i)
            if (fscanf(fp, "%lf", &x[i]) != 1) return 2;
        for (int i = 0; i < 3 * nt; ++i)
            if (fscanf(fp, "%d", &t[i]) != 1) return 2;
        if (lbmref_add_capsule(h, &cp, nn, x, nt, t) < 0) {
            fprintf(stderr, "add_capsule: %s\n", lbmref_error());
            return 3;
        }
        if (k == 0) {
            x0 = x; t0 = t; nn0 = nn; nt0 = nt; cp0 = cp;
        } else {
            free(x);
            free(t);
        }
    }
    fclose(fp);
    int st = lbmref_step(h, steps);
    lbmref_summary s;
    lbmref_get_summary(h, &s);
    printf("status %d\nmass0 %.17g\nmass1 %.17g\n", st, s.mass[0], s.mass[1]);
    for (int d = 0; d < 3; ++d) printf("momentum%d %.17g\npending%d %.17g\n", d, s.momentum[d], d, s.pending[d]);
    printf("step %lld\nlost %lld\nunstable %d\nlinks %lld\n", (long long)s.step,
           (long long)s.lost_reaction, s.unstable, (long long)s.links);
    for (int d = 0; d < 3; ++d) printf("node_momentum%d %.17g\n", d, s.node_momentum[d]);
    for (int k = 0; k < ncaps; ++k) {
        lbmref_capsule_obs o;
        lbmref_capsule_observe(h, k, &o);
        for (int d = 0; d < 3; ++d)
            printf("cap%d_centroid%d %.17g\ncap%d_f_anchor%d %.17g\ncap%d_f_capillary%d %.17g\n"
                   "cap%d_f_hertz%d %.17g\ncap%d_f_fluid%d %.17g\n", k, d, o.centroid[d], k, d,
                   o.f_anchor[d], k, d, o.f_capillary[d], k, d, o.f_hertz[d], k, d, o.f_fluid[d]);
        printf("cap%d_volume %.17g\n", k, o.volume);
    }
    double *men = (double *)malloc(sizeof(double) * (size_t)p.nx * p.ny);
    lbmref_meniscus(h, men);
    double msum = 0.0;
    long mcount = 0;
    for (long i = 0; i < (long)p.nx * p.ny; ++i)
        if (!isnan(men[i])) { msum += men[i]; ++mcount; }
    printf("meniscus_count %ld\nmeniscus_sum %.17g\n", mcount, msum);
    free(men);
    double *rho = (double *)malloc(sizeof(double) * 2 * (size_t)p.nx * p.ny * p.nz);
    double *vel = (double *)malloc(sizeof(double) * 3 * (size_t)p.nx * p.ny * p.nz);
    uint8_t *lab = (uint8_t *)malloc((size_t)p.nx * p.ny * p.nz);
    lbmref_rho(h, rho);
    lbmref_velocity(h, vel);
    lbmref_labels(h, lab);
    long nlab = 0;
    for (long i = 0; i < (long)p.nx * p.ny * p.nz; ++i) nlab += lab[i] != 0 && lab[i] != 255;
    printf("labelled %ld\n", nlab);
    free(rho); free(vel); free(lab);
    if (x0) {
        /* every pure helper once */
        int32_t e[57], opp[19];
        double w[19], u[3] = {0.01, -0.02, 0.005}, fe[19], psi[27], sc[3];
        lbmref_lattice(e, w, opp);
        lbmref_feq(0.7, u, fe);
        for (int i = 0; i < 27; ++i) psi[i] = 0.1 * i;
        lbmref_sc_sum(psi, 1.0, sc);
        double *minv = (double *)malloc(sizeof(double) * 4 * nt0);
        double *a0 = (double *)malloc(sizeof(double) * nt0);
        double *f = (double *)calloc(3 * (size_t)nn0, sizeof(double));
        lbmref_reference_geometry(nn0, x0, nt0, t0, minv, a0);
        double es = lbmref_skalak(nn0, x0, nt0, t0, minv, a0, cp0.ks, cp0.C, f);
        double eb = lbmref_bending(nn0, x0, nt0, t0, NULL, 0.1, f);
        double p0[3] = {x0[0] - 0.3, x0[1] - 0.2, x0[2] - 0.4}, p1[3] = {x0[0] + 0.5, x0[1] + 0.4, x0[2] + 0.3};
        double md = lbmref_miss_distance(p0, p1, x0 + 3 * t0[0], x0 + 3 * t0[1], x0 + 3 * t0[2]);
        double v = lbmref_volume(nn0, x0, nt0, t0);
        lbmref_volume_force(nn0, x0, nt0, t0, 0.3, 0.9 * v, f);
        uint8_t inside[8 * 8 * 8];
        lbmref_column_labels(nn0, x0, nt0, t0, 0, 0, 0, 8, 8, 8, inside);
        printf("helper_feq0 %.17g\nhelper_phi4 %.17g\nhelper_hertz %.17g\nhelper_skalak %.17g\n"
               "helper_bending %.17g\nhelper_volume %.17g\nhelper_miss %.17g\n", fe[0],
               lbmref_phi4(0.3), lbmref_hertz(0.5, 1.5, 1.5), es, eb, v, md);
        free(minv); free(a0); free(f);
        free(x0); free(t0);
    }
    lbmref_destroy(h);
    return 0;
}
