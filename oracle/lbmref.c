/*
 * lbmref.c -- CPU oracle: two-component Shan-Chen D3Q19 lattice Boltzmann fluid with
 * triangulated Skalak capsules coupled by an immersed boundary, or by half-way
 * bounce-back on the membrane with momentum exchange (the coupling of Section 3.1).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU baseline of
 * the benchmark.  It is deliberately plain and slow: one loop per step of the method,
 * no blocking, no fusion, no reordering beyond what each definition states.
 *
 * One time step n (state: post-collision populations f*, node positions X^n, the
 * pending membrane reaction R):
 *   1. side labels of every site from the capsule meshes at X^n
 *   2. capsule volume and centroid (double), then membrane node forces at X^n:
 *      Skalak strain (Section 3.1, eq. strain) by virtual work, volume penalty
 *      (eq. vol_cons), Hertz particle-substrate / particle-particle repulsion
 *      (Section 3.2, eq. interactions), centroid anchor, plus the pending reaction
 *   3. immersed-boundary spreading of node forces with Peskin's 4-point kernel
 *   4. pull streaming with half-way bounce-back at the wall, densities, psi
 *   5. Shan-Chen force (eq. shanchen) with the interior/exterior decoupling of
 *      Section 3.1: across a label change psi is taken from the site's own density
 *      plus a wetting offset; the cross-membrane part is returned to the membrane
 *   6. BGK collision (eq. method:boltzmann) towards eq. lbm:equilibrium at the
 *      Shan-Chen shifted velocity
 *   7. interpolation of the physical velocity to the nodes, node advection, and
 *      gathering of the reaction onto the nodes (applied in the next step)
 *
 * With the bounce-back coupling of Section 3.1 (coupling = 1) steps 3 and 7 become:
 *   3'. every lattice link between a site inside capsule k and a site outside it finds
 *      the membrane triangle it crosses; half-way bounce-back on that moving triangle
 *      (Ladd's moving-wall term with the mean velocity of its three nodes) is applied
 *      to the post-collision populations, and the exchanged momentum goes a third to
 *      each of the triangle's nodes (the homogeneous element-to-node weighting)
 *   7'. the Shan-Chen force across each link is returned to its triangle the same way;
 *      the nodes (mass node_mass, 25 rho0 in Section 3.2) take the membrane forces, the
 *      exchanged momentum spread over this and the next step (against staggered
 *      momenta) and the reaction: v += F / m, x += v
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared lbmref.c -lm
 *        (-DLBMREF_REAL=float for the FP32 diagnostic build).
 */
#include "lbmref.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef LBMREF_REAL
#define LBMREF_REAL double
#endif
typedef LBMREF_REAL real;

/* ----------------------------------------------------------------------------------- */
/* D3Q19 velocity set and weights (Section 3.1): rest weight 1/3, six axis links 1/18,  */
/* twelve diagonal links 1/36; speed of sound c_s^2 = 1/3.                              */
/* ----------------------------------------------------------------------------------- */
static const int EV[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double OMEGA[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPPQ[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

#define LABEL_SOLID 255

static char g_err[512];
const char *lbmref_error(void) { return g_err; }
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }

typedef struct {
    lbmref_capsule_params p;
    int nn, nt;
    real *x;        /* [nn][3] current node positions, unwrapped            */
    real *R;        /* [nn][3] pending reaction, applied in the next step    */
    real *F;        /* [nn][3] total node force of the last evaluation       */
    real *Fh;       /* [nn][3] Hertz part of the last evaluation             */
    int32_t *tri;   /* [nt][3]                                               */
    double *minv;   /* [nt][4] reference inverse, row-major 2x2              */
    double *a0;     /* [nt]    reference area                                */
    int ne;         /* edges shared by two triangles (bending, kb != 0)      */
    int32_t *edge;  /* [ne][4] x1, x2, x3, x4: triangles (x1,x2,x3), (x2,x1,x4) */
    double *th0;    /* [ne] reference dihedral angle                         */
    double v0, c0[3];
    double vol, cen[3];        /* at X^n, computed at the start of the step */
    double f_anchor[3];        /* sum of anchor node forces of the last step */
    /* bounce-back coupling */
    real *V;        /* [nn][3] node velocities                               */
    real *Pex;      /* [nn][3] momentum exchanged with the fluid this step   */
    real *Pprev;    /* [nn][3] momentum exchanged in the previous step       */
    real *Rsc;      /* [nn][3] Shan-Chen reaction of this step's links       */
    double f_fluid[3];         /* fluid force on the membrane of the last step */
} cap_t;

/* a bounce-back link: site a inside capsule k, direction q, b = a + e_q outside it;
 * tri: the membrane triangle it crosses (-1: none found) */
typedef struct {
    long a, b;
    int q, k, tri;
} link_t;

struct lbmref_handle {
    lbmref_params p;
    int nx, ny, nz;
    long N;
    real *f, *fn;      /* [2][19][N] post-collision populations, current and next */
    real *rho, *psi;   /* [2][N] post-streaming density and pseudopotential       */
    uint8_t *label;    /* [N] 0 exterior, k+1 inside capsule k, 255 solid         */
    real *fibm;        /* [4][N] spread force (x,y,z) and kernel coverage c(x)    */
    real *uphys;       /* [3][N] physical velocity of the last collision          */
    real *react;       /* [3][N] reaction of cross-membrane Shan-Chen links       */
    int ncap;
    cap_t *cap;
    int64_t step, lost;
    int unstable;
    link_t *links;     /* bounce-back links of the current step */
    long nlinks, links_cap;
    int64_t lost_links;
};

static inline int wrapi(int a, int n) { a %= n; return a < 0 ? a + n : a; }
static inline long sidx(const lbmref_handle *h, int i, int j, int k) {
    return ((long)k * h->ny + j) * h->nx + i;
}
static inline int is_solid(const lbmref_handle *h, int k) { return h->p.wall_z0 && k == 0; }

/* ----------------------------------------------------------------------------------- */
/* Pure helpers                                                                         */
/* ----------------------------------------------------------------------------------- */

void lbmref_lattice(int32_t e[57], double omega[19], int32_t opp[19]) {
    for (int q = 0; q < 19; ++q) {
        for (int d = 0; d < 3; ++d) e[3 * q + d] = EV[q][d];
        omega[q] = OMEGA[q];
        opp[q] = OPPQ[q];
    }
}

/* Second-order equilibrium, eq. lbm:equilibrium with c_s^2 = 1/3. */
static void feq19(real rho, const real u[3], real out[19]) {
    const real cs2 = (real)(1.0 / 3.0);
    real uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int q = 0; q < 19; ++q) {
        real eu = EV[q][0] * u[0] + EV[q][1] * u[1] + EV[q][2] * u[2];
        out[q] = (real)OMEGA[q] * rho *
                 (1 + eu / cs2 - uu / (2 * cs2) + eu * eu / (2 * cs2 * cs2));
    }
}

void lbmref_feq(double rho, const double u[3], double out[19]) {
    real ur[3] = {(real)u[0], (real)u[1], (real)u[2]}, o[19];
    feq19((real)rho, ur, o);
    for (int q = 0; q < 19; ++q) out[q] = o[q];
}

/* Peskin's 4-point immersed-boundary kernel (one dimension). */
double lbmref_phi4(double r) {
    double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
}
static inline real phi4r(real r) { return (real)lbmref_phi4((double)r); }

/* Shan-Chen stencil sum  sum_i w_i psi(x+e_i) e_i  over a 3x3x3 neighbourhood
 * psi27[(dz+1)*9 + (dy+1)*3 + (dx+1)], with w_i = sc_norm * omega_i. */
void lbmref_sc_sum(const double psi27[27], double sc_norm, double out[3]) {
    out[0] = out[1] = out[2] = 0.0;
    for (int q = 1; q < 19; ++q) {
        double ps = psi27[(EV[q][2] + 1) * 9 + (EV[q][1] + 1) * 3 + (EV[q][0] + 1)];
        for (int d = 0; d < 3; ++d) out[d] += sc_norm * OMEGA[q] * ps * EV[q][d];
    }
}

/* Hertz repulsion magnitude F = xi (delta0 - d)^{3/2} for d < delta0 (Section 3.2). */
double lbmref_hertz(double d, double xi, double delta0) {
    return d < delta0 ? xi * pow(delta0 - d, 1.5) : 0.0;
}

/* Reference geometry of each triangle: the vertices in an orthonormal in-plane frame,
 * P1=(0,0), P2=(a,0), P3=(b,c); minv = inverse of the 2x2 matrix [P2-P1, P3-P1]. */
void lbmref_reference_geometry(int32_t nn, const double *x, int32_t nt, const int32_t *tri,
                               double *minv, double *a0) {
    (void)nn;
    for (int t = 0; t < nt; ++t) {
        const double *p1 = x + 3 * tri[3 * t], *p2 = x + 3 * tri[3 * t + 1],
                     *p3 = x + 3 * tri[3 * t + 2];
        double u[3], v[3];
        for (int d = 0; d < 3; ++d) { u[d] = p2[d] - p1[d]; v[d] = p3[d] - p1[d]; }
        double a = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double e1[3] = {u[0] / a, u[1] / a, u[2] / a};
        double b = v[0] * e1[0] + v[1] * e1[1] + v[2] * e1[2];
        double w[3] = {v[0] - b * e1[0], v[1] - b * e1[1], v[2] - b * e1[2]};
        double c = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        /* [[a, b], [0, c]]^{-1} = [[1/a, -b/(a c)], [0, 1/c]] */
        minv[4 * t + 0] = 1.0 / a;
        minv[4 * t + 1] = -b / (a * c);
        minv[4 * t + 2] = 0.0;
        minv[4 * t + 3] = 1.0 / c;
        a0[t] = 0.5 * a * c;
    }
}

/* Skalak energy of one triangle and its nodal forces (Section 3.1, eq. strain), by the
 * principle of virtual work: F_a = -dE/dx_a with E = A0 * W(I1, I2),
 * W = ks/4 (I1^2 + 2 I1 - 2 I2 + C I2^2), D = [x2-x1, x3-x1] Minv, B = D^T D,
 * I1 = tr B - 2, I2 = det B - 1. */
static double skalak_tri(const real *x1, const real *x2, const real *x3, const double *m,
                         double a0, double ks, double C, real *f1, real *f2, real *f3) {
    real u[3], v[3], d0[3], d1[3];
    for (int d = 0; d < 3; ++d) {
        u[d] = x2[d] - x1[d];
        v[d] = x3[d] - x1[d];
    }
    for (int d = 0; d < 3; ++d) {
        d0[d] = u[d] * (real)m[0] + v[d] * (real)m[2];
        d1[d] = u[d] * (real)m[1] + v[d] * (real)m[3];
    }
    real b00 = d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2];
    real b01 = d0[0] * d1[0] + d0[1] * d1[1] + d0[2] * d1[2];
    real b11 = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
    real I1 = b00 + b11 - 2;
    real detB = b00 * b11 - b01 * b01;
    real I2 = detB - 1;
    real W = (real)(ks / 4) * (I1 * I1 + 2 * I1 - 2 * I2 + (real)C * I2 * I2);
    real W1 = (real)(ks / 2) * (I1 + 1);       /* dW/dI1 */
    real W2 = (real)(ks / 2) * ((real)C * I2 - 1); /* dW/dI2 */
    /* dW/dD = 2 W1 D + 2 W2 det(B) D B^{-1} = 2 W1 D + 2 W2 D adj(B) */
    real P0[3], P1[3];
    for (int d = 0; d < 3; ++d) {
        P0[d] = 2 * W1 * d0[d] + 2 * W2 * (d0[d] * b11 - d1[d] * b01);
        P1[d] = 2 * W1 * d1[d] + 2 * W2 * (-d0[d] * b01 + d1[d] * b00);
    }
    /* dE/du = A0 (P Minv^T)_col0, dE/dv = A0 (P Minv^T)_col1 */
    for (int d = 0; d < 3; ++d) {
        real gu = (real)a0 * (P0[d] * (real)m[0] + P1[d] * (real)m[1]);
        real gv = (real)a0 * (P0[d] * (real)m[2] + P1[d] * (real)m[3]);
        f1[d] += gu + gv;
        f2[d] -= gu;
        f3[d] -= gv;
    }
    return a0 * (double)W;
}

/* Bending (Section 3.1, eq. method:curvature), in the edge form of the Helfrich energy
 * on the triangulation: E_b = sqrt(3) kb sum_e (theta_e - theta0_e)^2, with theta_e the
 * angle between the outward normals of the two triangles that share edge e, signed about
 * the edge, and theta0_e its value on the stress-free reference mesh.  On an equilateral
 * triangulation of a sphere of radius R with edge length a, theta_e = a / (sqrt(3) R); the
 * 3 N_t / 2 edges then give sqrt(3) sum_e theta_e^2 = 8 pi, the Helfrich energy
 * (kb / 2) oint (2H)^2 dA of the sphere, which fixes the prefactor.  The Gaussian-curvature
 * term is a constant on a closed surface (Gauss-Bonnet) and exerts no force.  The force is
 * -dE/dx (virtual work), with the gradient of the dihedral angle in the closed form of
 * Blondel and Karplus (J. Comput. Chem. 17, 1132 (1996)). */

typedef struct { int32_t lo, hi, from, third; } dedge_t;   /* directed edge from -> other */

static int dedge_cmp(const void *a, const void *b) {
    const dedge_t *p = (const dedge_t *)a, *q = (const dedge_t *)b;
    if (p->lo != q->lo) return p->lo < q->lo ? -1 : 1;
    if (p->hi != q->hi) return p->hi < q->hi ? -1 : 1;
    return p->from < q->from ? -1 : (p->from > q->from);
}

/* Edges shared by two consistently oriented triangles: x1 -> x2 in (x1, x2, x3) and the
 * reverse in (x2, x1, x4).  Edges of one triangle only (an open boundary) are skipped.
 * Returns the number of shared edges, or -1 if an edge is used the same way twice or by
 * more than two triangles. */
static int mesh_edges(int nt, const int32_t *tri, int32_t **out) {
    dedge_t *d = (dedge_t *)malloc(sizeof(dedge_t) * 3 * (size_t)nt);
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            int32_t u = tri[3 * t + k], v = tri[3 * t + (k + 1) % 3], w = tri[3 * t + (k + 2) % 3];
            dedge_t e = {u < v ? u : v, u < v ? v : u, u, w};
            d[3 * t + k] = e;
        }
    qsort(d, 3 * (size_t)nt, sizeof(dedge_t), dedge_cmp);
    int32_t *edge = (int32_t *)malloc(sizeof(int32_t) * 4 * 3 * (size_t)nt);
    int ne = 0, bad = 0;
    for (int i = 0; i < 3 * nt;) {
        int j = i;
        while (j < 3 * nt && d[j].lo == d[i].lo && d[j].hi == d[i].hi) ++j;
        if (j - i == 2 && d[i].from != d[i + 1].from) {
            /* d[i] runs lo -> hi: x1 = lo, x2 = hi, x3 its third node; x4 the other's */
            edge[4 * ne] = d[i].lo;
            edge[4 * ne + 1] = d[i].hi;
            edge[4 * ne + 2] = d[i].third;
            edge[4 * ne + 3] = d[i + 1].third;
            ++ne;
        } else if (j - i > 1) {
            bad = 1;
        }
        i = j;
    }
    free(d);
    if (bad) { free(edge); *out = NULL; return -1; }
    *out = edge;
    return ne;
}

static void sub3(const real *a, const real *b, real *o) {
    for (int d = 0; d < 3; ++d) o[d] = a[d] - b[d];
}
static void cross3(const real *a, const real *b, real *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static real dot3(const real *a, const real *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Dihedral angle of the edge x1 - x2 between the outward normals of (x1, x2, x3) and
 * (x2, x1, x4), and (if g) its gradient with respect to x1 .. x4. */
static double dihedral(const real *x1, const real *x2, const real *x3, const real *x4,
                       real g[4][3]) {
    real F[3], G[3], H[3], A[3], B[3], BA[3];
    sub3(x3, x1, F);
    sub3(x1, x2, G);
    sub3(x4, x2, H);
    cross3(F, G, A);   /* outward normal of (x1, x2, x3) */
    cross3(H, G, B);   /* minus the outward normal of (x2, x1, x4) */
    cross3(B, A, BA);
    const real gl = sqrt(dot3(G, G)), a2 = dot3(A, A), b2 = dot3(B, B);
    /* normals n1 = A, n2 = -B, edge direction -G / |G| */
    const double th = atan2(-(double)dot3(BA, G) / gl, -(double)dot3(A, B));
    if (g) {
        const real fg = dot3(F, G) / (a2 * gl), hg = dot3(H, G) / (b2 * gl);
        for (int d = 0; d < 3; ++d) {
            g[2][d] = -gl / a2 * A[d];
            g[3][d] = gl / b2 * B[d];
            g[0][d] = gl / a2 * A[d] + fg * A[d] - hg * B[d];
            g[1][d] = -(g[0][d] + g[2][d] + g[3][d]);
        }
    }
    return th;
}

/* bending energy of one edge, and its forces added to f1 .. f4 */
static double bending_edge(const real *x1, const real *x2, const real *x3, const real *x4,
                           double th0, double kb, real *f1, real *f2, real *f3, real *f4) {
    real g[4][3];
    const double th = dihedral(x1, x2, x3, x4, g);
    const double k = sqrt(3.0) * kb, dth = th - th0;
    real *f[4] = {f1, f2, f3, f4};
    for (int v = 0; v < 4; ++v)
        for (int d = 0; d < 3; ++d) f[v][d] -= (real)(2.0 * k * dth) * g[v][d];
    return k * dth * dth;
}

double lbmref_bending(int32_t nn, const double *x, int32_t nt, const int32_t *tri,
                      const double *ref, double kb, double *force) {
    int32_t *edge = NULL;
    const int ne = mesh_edges(nt, tri, &edge);
    if (ne < 0) return NAN;
    real *xr = (real *)malloc(sizeof(real) * 3 * nn), *rr = (real *)malloc(sizeof(real) * 3 * nn);
    real *fr = (real *)calloc(3 * nn, sizeof(real));
    for (int i = 0; i < 3 * nn; ++i) {
        xr[i] = (real)x[i];
        rr[i] = ref ? (real)ref[i] : 0;
    }
    double E = 0.0;
    for (int e = 0; e < ne; ++e) {
        const int32_t *q = edge + 4 * e;
        const double th0 = ref ? dihedral(rr + 3 * q[0], rr + 3 * q[1], rr + 3 * q[2],
                                          rr + 3 * q[3], NULL) : 0.0;
        E += bending_edge(xr + 3 * q[0], xr + 3 * q[1], xr + 3 * q[2], xr + 3 * q[3], th0, kb,
                          fr + 3 * q[0], fr + 3 * q[1], fr + 3 * q[2], fr + 3 * q[3]);
    }
    if (force)
        for (int i = 0; i < 3 * nn; ++i) force[i] = fr[i];
    free(edge);
    free(xr);
    free(rr);
    free(fr);
    return E;
}

double lbmref_skalak(int32_t nn, const double *x, int32_t nt, const int32_t *tri,
                     const double *minv, const double *a0, double ks, double C, double *force) {
    real *xr = (real *)malloc(sizeof(real) * 3 * nn), *fr = (real *)calloc(3 * nn, sizeof(real));
    for (int i = 0; i < 3 * nn; ++i) xr[i] = (real)x[i];
    double E = 0.0;
    for (int t = 0; t < nt; ++t) {
        int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
        E += skalak_tri(xr + 3 * a, xr + 3 * b, xr + 3 * c, minv + 4 * t, a0[t], ks, C,
                        fr + 3 * a, fr + 3 * b, fr + 3 * c);
    }
    if (force)
        for (int i = 0; i < 3 * nn; ++i) force[i] = fr[i];
    free(xr);
    free(fr);
    return E;
}

/* Enclosed volume of a closed, outward-oriented mesh: V = sum_T x1.(x2 x x3)/6, with the
 * origin moved to the node mean (the sum is origin-independent for a closed surface). */
static double volume_of(int nn, const real *x, int nt, const int32_t *tri, const double *cen) {
    double V = 0.0;
    (void)nn;
    for (int t = 0; t < nt; ++t) {
        double p[3][3];
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) p[k][d] = (double)x[3 * tri[3 * t + k] + d] - cen[d];
        double cx = p[1][1] * p[2][2] - p[1][2] * p[2][1];
        double cy = p[1][2] * p[2][0] - p[1][0] * p[2][2];
        double cz = p[1][0] * p[2][1] - p[1][1] * p[2][0];
        V += (p[0][0] * cx + p[0][1] * cy + p[0][2] * cz) / 6.0;
    }
    return V;
}

static void centroid_of(int nn, const real *x, double *cen) {
    double s[3] = {0, 0, 0};
    for (int i = 0; i < nn; ++i)
        for (int d = 0; d < 3; ++d) s[d] += (double)x[3 * i + d];
    for (int d = 0; d < 3; ++d) cen[d] = s[d] / nn;
}

double lbmref_volume(int32_t nn, const double *x, int32_t nt, const int32_t *tri) {
    real *xr = (real *)malloc(sizeof(real) * 3 * nn);
    for (int i = 0; i < 3 * nn; ++i) xr[i] = (real)x[i];
    double cen[3];
    centroid_of(nn, xr, cen);
    double V = volume_of(nn, xr, nt, tri, cen);
    free(xr);
    return V;
}

/* Volume penalty E = kv (V - V0)^2 / (2 V0) (eq. vol_cons); F_a = -kv (V-V0)/V0 dV/dx_a,
 * dV/dx_a = (x_b x x_c)/6 for each triangle (a, b, c) in cyclic order, with the origin
 * at the node mean. */
static void volume_force_add(int nn, const real *x, int nt, const int32_t *tri, double kv,
                             double V, double V0, const double *cen, real *F) {
    (void)nn;
    double coef = -kv * (V - V0) / V0;
    for (int t = 0; t < nt; ++t) {
        for (int k = 0; k < 3; ++k) {
            int a = tri[3 * t + k], b = tri[3 * t + (k + 1) % 3], c = tri[3 * t + (k + 2) % 3];
            double pb[3], pc[3];
            for (int d = 0; d < 3; ++d) {
                pb[d] = (double)x[3 * b + d] - cen[d];
                pc[d] = (double)x[3 * c + d] - cen[d];
            }
            F[3 * a + 0] += (real)(coef * (pb[1] * pc[2] - pb[2] * pc[1]) / 6.0);
            F[3 * a + 1] += (real)(coef * (pb[2] * pc[0] - pb[0] * pc[2]) / 6.0);
            F[3 * a + 2] += (real)(coef * (pb[0] * pc[1] - pb[1] * pc[0]) / 6.0);
        }
    }
}

void lbmref_volume_force(int32_t nn, const double *x, int32_t nt, const int32_t *tri,
                         double kv, double v0, double *force) {
    if (nn <= 0) return;
    real *xr = (real *)malloc(sizeof(real) * 3 * nn), *fr = (real *)calloc(3 * nn, sizeof(real));
    for (int i = 0; i < 3 * nn; ++i) xr[i] = (real)x[i];
    double cen[3];
    centroid_of(nn, xr, cen);
    double V = volume_of(nn, xr, nt, tri, cen);
    volume_force_add(nn, xr, nt, tri, kv, V, v0, cen, fr);
    for (int i = 0; i < 3 * nn; ++i) force[i] = fr[i];
    free(xr);
    free(fr);
}

/* ----------------------------------------------------------------------------------- */
/* Side labels: a vertical line through lattice column (i, j) crosses the membrane where */
/* the column point lies inside a triangle's xy projection (top-left rule on shared      */
/* edges, zero-area projections skipped); the crossing height is the barycentric         */
/* interpolation of the vertex heights.  A site at height m is inside when an odd number */
/* of crossings lies at or below m.  Decisions use the node positions rounded to FP32,   */
/* evaluated in double.                                                                 */
/* ----------------------------------------------------------------------------------- */
static inline double edgef(double ux, double uy, double vx, double vy, double px, double py) {
    return (vx - ux) * (py - uy) - (vy - uy) * (px - ux);
}
static inline int top_left(double ux, double uy, double vx, double vy) {
    return (vy < uy) || (vy == uy && vx < ux);
}
static inline int edge_in(double w, double ux, double uy, double vx, double vy) {
    return w > 0.0 || (w == 0.0 && top_left(ux, uy, vx, vy));
}

/* Crossing height of the column (px, py) with triangle (a, b, c); returns 0 if none. */
static int column_crossing(const float *a, const float *b, const float *c, double px,
                           double py, double *zc) {
    double ax = a[0], ay = a[1], bx = b[0], by = b[1], cx = c[0], cy = c[1];
    double az = a[2], bz = b[2], cz = c[2];
    double area = edgef(ax, ay, bx, by, cx, cy);
    if (area == 0.0) return 0;
    if (area < 0.0) { /* make the projection counter-clockwise */
        double t;
        t = bx; bx = cx; cx = t;
        t = by; by = cy; cy = t;
        t = bz; bz = cz; cz = t;
    }
    double wa = edgef(bx, by, cx, cy, px, py);
    double wb = edgef(cx, cy, ax, ay, px, py);
    double wc = edgef(ax, ay, bx, by, px, py);
    if (!edge_in(wa, bx, by, cx, cy) || !edge_in(wb, cx, cy, ax, ay) ||
        !edge_in(wc, ax, ay, bx, by))
        return 0;
    *zc = (wa * az + wb * bz + wc * cz) / (wa + wb + wc);
    return 1;
}

/* Inside flags for the box [x0, x0+dx) x [y0, y0+dy) x [z0, z0+dz) (unwrapped). */
static void label_box(int nt, const int32_t *tri, const float *xf, int x0, int y0, int z0,
                      int dx, int dy, int dz, uint8_t *inside) {
    memset(inside, 0, (size_t)dx * dy * dz);
#pragma omp parallel for schedule(dynamic)
    for (int jj = 0; jj < dy; ++jj) {
        double *zs = (double *)malloc(sizeof(double) * 64);
        int cap = 64;
        for (int ii = 0; ii < dx; ++ii) {
            int nz = 0;
            double px = x0 + ii, py = y0 + jj;
            for (int t = 0; t < nt; ++t) {
                double zc;
                if (column_crossing(xf + 3 * tri[3 * t], xf + 3 * tri[3 * t + 1],
                                    xf + 3 * tri[3 * t + 2], px, py, &zc)) {
                    if (nz == cap) { cap *= 2; zs = (double *)realloc(zs, sizeof(double) * cap); }
                    zs[nz++] = zc;
                }
            }
            for (int kk = 0; kk < dz; ++kk) {
                int below = 0;
                for (int s = 0; s < nz; ++s) below += (zs[s] <= (double)(z0 + kk));
                inside[((size_t)kk * dy + jj) * dx + ii] = (uint8_t)(below & 1);
            }
        }
        free(zs);
    }
}

int lbmref_column_labels(int32_t nn, const double *xyz, int32_t nt, const int32_t *tri,
                         int32_t x0, int32_t y0, int32_t z0, int32_t dx, int32_t dy, int32_t dz,
                         uint8_t *inside) {
    float *xf = (float *)malloc(sizeof(float) * 3 * nn);
    for (int i = 0; i < 3 * nn; ++i) xf[i] = (float)xyz[i];
    label_box(nt, tri, xf, x0, y0, z0, dx, dy, dz, inside);
    free(xf);
    return 0;
}

static void compute_labels(lbmref_handle *h) {
    for (long s = 0; s < h->N; ++s) h->label[s] = 0;
    if (h->p.wall_z0)
        for (long s = 0; s < (long)h->nx * h->ny; ++s) h->label[s] = LABEL_SOLID;
    for (int k = 0; k < h->ncap; ++k) {
        cap_t *c = &h->cap[k];
        float *xf = (float *)malloc(sizeof(float) * 3 * c->nn);
        float lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
        for (int i = 0; i < c->nn; ++i)
            for (int d = 0; d < 3; ++d) {
                xf[3 * i + d] = (float)c->x[3 * i + d];
                if (xf[3 * i + d] < lo[d]) lo[d] = xf[3 * i + d];
                if (xf[3 * i + d] > hi[d]) hi[d] = xf[3 * i + d];
            }
        int b0[3], bn[3];
        for (int d = 0; d < 3; ++d) {
            b0[d] = (int)ceil((double)lo[d]);
            bn[d] = (int)floor((double)hi[d]) - b0[d] + 1;
            if (bn[d] < 0) bn[d] = 0;
        }
        uint8_t *in = (uint8_t *)malloc((size_t)bn[0] * bn[1] * bn[2] + 1);
        label_box(c->nt, c->tri, xf, b0[0], b0[1], b0[2], bn[0], bn[1], bn[2], in);
        for (int kk = 0; kk < bn[2]; ++kk)
            for (int jj = 0; jj < bn[1]; ++jj)
                for (int ii = 0; ii < bn[0]; ++ii) {
                    if (!in[((size_t)kk * bn[1] + jj) * bn[0] + ii]) continue;
                    int zi = wrapi(b0[2] + kk, h->nz);
                    if (is_solid(h, zi)) continue;
                    h->label[sidx(h, wrapi(b0[0] + ii, h->nx), wrapi(b0[1] + jj, h->ny), zi)] =
                        (uint8_t)(k + 1);
                }
        free(in);
        free(xf);
    }
}

/* Labels used by the last step (at create / add_capsule: at the initial positions). */
int lbmref_labels(lbmref_handle *h, uint8_t *out) {
    memcpy(out, h->label, (size_t)h->N);
    return 0;
}

/* ----------------------------------------------------------------------------------- */
/* Creation and capsules                                                                */
/* ----------------------------------------------------------------------------------- */

lbmref_handle *lbmref_create(const lbmref_params *p) {
    if (!p || p->nx < 3 || p->ny < 3 || p->nz < 3) { set_err("invalid lattice size"); return NULL; }
    if (!(p->tau[0] > 0.5) || !(p->tau[1] > 0.5)) { set_err("tau must exceed 1/2"); return NULL; }
    if (!(p->rho0 > 0)) { set_err("rho0 must be positive"); return NULL; }
    if (p->init_mode < 0 || p->init_mode > 2) { set_err("invalid init_mode"); return NULL; }
    if (p->init_mode == 2 && !p->init_rho_array) { set_err("init_rho_array missing"); return NULL; }
    if (p->coupling < 0 || p->coupling > 1) { set_err("invalid coupling"); return NULL; }
    if (p->coupling == 1 && !(p->node_mass > 0)) { set_err("node_mass must be positive"); return NULL; }
    lbmref_handle *h = (lbmref_handle *)calloc(1, sizeof *h);
    h->p = *p;
    h->p.init_rho_array = NULL;
    h->nx = p->nx; h->ny = p->ny; h->nz = p->nz;
    h->N = (long)p->nx * p->ny * p->nz;
#ifdef _OPENMP
    if (p->n_threads > 0) omp_set_num_threads(p->n_threads);
#endif
    long N = h->N;
    h->f = (real *)calloc((size_t)38 * N, sizeof(real));
    h->fn = (real *)calloc((size_t)38 * N, sizeof(real));
    h->rho = (real *)calloc((size_t)2 * N, sizeof(real));
    h->psi = (real *)calloc((size_t)2 * N, sizeof(real));
    h->label = (uint8_t *)calloc((size_t)N, 1);
    h->fibm = (real *)calloc((size_t)4 * N, sizeof(real));
    h->uphys = (real *)calloc((size_t)3 * N, sizeof(real));
    h->react = (real *)calloc((size_t)3 * N, sizeof(real));
    if (!h->f || !h->fn || !h->rho || !h->psi || !h->label || !h->fibm || !h->uphys || !h->react) {
        set_err("out of memory");
        lbmref_destroy(h);
        return NULL;
    }
    /* initial densities (Section 3.2 for the film), then f* = f^eq(rho, 0) */
    int kw = p->wall_z0 ? 1 : 0;
    int H = (int)lround(p->film_height);
    for (int k = 0; k < h->nz; ++k)
        for (int j = 0; j < h->ny; ++j)
            for (int i = 0; i < h->nx; ++i) {
                long s = sidx(h, i, j, k);
                if (is_solid(h, k)) continue;
                double r[2];
                if (p->init_mode == 0) {
                    r[0] = p->init_rho[0]; r[1] = p->init_rho[1];
                } else if (p->init_mode == 1) {
                    int layer = k - kw;
                    if (layer < H) { r[0] = p->rho_maj; r[1] = p->rho_min; }
                    else if (layer == H) { r[0] = p->rho_iface; r[1] = p->rho_iface; }
                    else { r[0] = p->rho_min; r[1] = p->rho_maj; }
                } else {
                    r[0] = p->init_rho_array[s];
                    r[1] = p->init_rho_array[N + s];
                }
                real u0[3] = {0, 0, 0}, fe[19];
                for (int c = 0; c < 2; ++c) {
                    feq19((real)r[c], u0, fe);
                    for (int q = 0; q < 19; ++q) h->f[((long)c * 19 + q) * N + s] = fe[q];
                }
            }
    compute_labels(h);
    return h;
}

int lbmref_add_capsule(lbmref_handle *h, const lbmref_capsule_params *cp, int32_t nn,
                       const double *xyz, int32_t nt, const int32_t *tri) {
    if (!h || !cp || nn < 4 || nt < 4 || !xyz || !tri) { set_err("invalid capsule"); return -1; }
    if (h->step > 0) { set_err("capsules must be added before the first step"); return -5; }
    if (!(cp->kb >= 0.0)) { set_err("bending modulus must be >= 0"); return -1; }
    if (h->ncap >= 254) { set_err("too many capsules"); return -1; }
    for (int t = 0; t < 3 * nt; ++t)
        if (tri[t] < 0 || tri[t] >= nn) { set_err("triangle index out of range"); return -1; }
    h->cap = (cap_t *)realloc(h->cap, sizeof(cap_t) * (h->ncap + 1));
    cap_t *c = &h->cap[h->ncap];
    memset(c, 0, sizeof *c);
    c->p = *cp;
    c->nn = nn; c->nt = nt;
    c->x = (real *)malloc(sizeof(real) * 3 * nn);
    c->R = (real *)calloc(3 * nn, sizeof(real));
    c->F = (real *)calloc(3 * nn, sizeof(real));
    c->Fh = (real *)calloc(3 * nn, sizeof(real));
    c->V = (real *)calloc(3 * nn, sizeof(real));
    c->Pex = (real *)calloc(3 * nn, sizeof(real));
    c->Pprev = (real *)calloc(3 * nn, sizeof(real));
    c->Rsc = (real *)calloc(3 * nn, sizeof(real));
    c->tri = (int32_t *)malloc(sizeof(int32_t) * 3 * nt);
    c->minv = (double *)malloc(sizeof(double) * 4 * nt);
    c->a0 = (double *)malloc(sizeof(double) * nt);
    for (int i = 0; i < 3 * nn; ++i) c->x[i] = (real)xyz[i];
    memcpy(c->tri, tri, sizeof(int32_t) * 3 * nt);
    /* reference geometry from the stress-free initial mesh, in double */
    lbmref_reference_geometry(nn, xyz, nt, tri, c->minv, c->a0);
    double cen[3] = {0, 0, 0};
    for (int i = 0; i < nn; ++i)
        for (int d = 0; d < 3; ++d) cen[d] += xyz[3 * i + d];
    for (int d = 0; d < 3; ++d) c->c0[d] = cen[d] / nn;
    c->v0 = lbmref_volume(nn, xyz, nt, tri);
    if (cp->kb != 0.0) {
        /* every edge shared by two triangles; reference angles from the initial mesh */
        c->ne = mesh_edges(nt, tri, &c->edge);
        if (2 * c->ne != 3 * nt) {
            set_err("bending needs a closed, consistently oriented mesh");
            free(c->edge); free(c->x); free(c->R); free(c->F); free(c->Fh); free(c->tri);
            free(c->minv); free(c->a0);
            return -1;
        }
        c->th0 = (double *)malloc(sizeof(double) * c->ne);
        real *xr = (real *)malloc(sizeof(real) * 3 * nn);
        for (int i = 0; i < 3 * nn; ++i) xr[i] = (real)xyz[i];
        for (int e = 0; e < c->ne; ++e) {
            const int32_t *q = c->edge + 4 * e;
            c->th0[e] = dihedral(xr + 3 * q[0], xr + 3 * q[1], xr + 3 * q[2], xr + 3 * q[3], NULL);
        }
        free(xr);
    }
    h->ncap++;
    compute_labels(h);
    return h->ncap - 1;
}

/* ----------------------------------------------------------------------------------- */
/* Membrane forces at X^n                                                               */
/* ----------------------------------------------------------------------------------- */

static double min_image(double d, int n, int periodic) {
    return periodic ? d - n * floor(d / n + 0.5) : d;
}

static void bbox_of(const cap_t *c, double lo[3], double hi[3]) {
    for (int d = 0; d < 3; ++d) { lo[d] = 1e300; hi[d] = -1e300; }
    for (int i = 0; i < c->nn; ++i)
        for (int d = 0; d < 3; ++d) {
            double v = (double)c->x[3 * i + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
}

static int boxes_apart(const lbmref_handle *h, const cap_t *a, const cap_t *b, double d0) {
    double la[3], ha[3], lb[3], hb[3];
    bbox_of(a, la, ha);
    bbox_of(b, lb, hb);
    int nd[3] = {h->nx, h->ny, h->nz}, per[3] = {1, 1, !h->p.wall_z0};
    for (int d = 0; d < 3; ++d) {
        double ca = 0.5 * (la[d] + ha[d]), cb = 0.5 * (lb[d] + hb[d]);
        double gap = fabs(min_image(ca - cb, nd[d], per[d])) - 0.5 * (ha[d] - la[d]) -
                     0.5 * (hb[d] - lb[d]);
        if (gap >= d0) return 1;
    }
    return 0;
}

static void membrane_forces(lbmref_handle *h) {
    const double xi = h->p.hertz_xi, d0 = h->p.hertz_delta0;
    for (int k = 0; k < h->ncap; ++k) {
        cap_t *c = &h->cap[k];
        centroid_of(c->nn, c->x, c->cen);
        c->vol = volume_of(c->nn, c->x, c->nt, c->tri, c->cen);
    }
    for (int k = 0; k < h->ncap; ++k) {
        cap_t *c = &h->cap[k];
        memset(c->F, 0, sizeof(real) * 3 * c->nn);
        memset(c->Fh, 0, sizeof(real) * 3 * c->nn);
        /* Skalak strain, eq. strain */
        for (int t = 0; t < c->nt; ++t) {
            int a = c->tri[3 * t], b = c->tri[3 * t + 1], cc = c->tri[3 * t + 2];
            skalak_tri(c->x + 3 * a, c->x + 3 * b, c->x + 3 * cc, c->minv + 4 * t, c->a0[t],
                       c->p.ks, c->p.C, c->F + 3 * a, c->F + 3 * b, c->F + 3 * cc);
        }
        /* bending, eq. method:curvature (edge form) */
        if (c->p.kb != 0.0)
            for (int e = 0; e < c->ne; ++e) {
                const int32_t *q = c->edge + 4 * e;
                bending_edge(c->x + 3 * q[0], c->x + 3 * q[1], c->x + 3 * q[2], c->x + 3 * q[3],
                             c->th0[e], c->p.kb, c->F + 3 * q[0], c->F + 3 * q[1],
                             c->F + 3 * q[2], c->F + 3 * q[3]);
            }
        /* volume penalty, eq. vol_cons */
        if (c->p.kv != 0.0)
            volume_force_add(c->nn, c->x, c->nt, c->tri, c->p.kv, c->vol, c->v0, c->cen, c->F);
        /* Hertz particle-substrate repulsion against the plane z = 0.5 + plane_dz */
        if (h->p.wall_z0 && xi > 0) {
            double zp = 0.5 + h->p.plane_dz;
            for (int i = 0; i < c->nn; ++i) {
                double f = lbmref_hertz((double)c->x[3 * i + 2] - zp, xi, d0);
                c->Fh[3 * i + 2] += (real)f;
            }
        }
        /* Hertz particle-particle repulsion between nodes of different capsules */
        if (xi > 0) {
            for (int o = 0; o < h->ncap; ++o) {
                if (o == k) continue;
                cap_t *e = &h->cap[o];
                /* exact pruning: skip capsule pairs whose bounding boxes are at least
                 * delta0 apart along some axis (no node pair can then be in range) */
                if (boxes_apart(h, c, e, d0)) continue;
                for (int i = 0; i < c->nn; ++i)
                    for (int m = 0; m < e->nn; ++m) {
                        double r[3], dd = 0;
                        int per[3] = {1, 1, !h->p.wall_z0};
                        int nd[3] = {h->nx, h->ny, h->nz};
                        for (int d = 0; d < 3; ++d) {
                            r[d] = min_image((double)c->x[3 * i + d] - (double)e->x[3 * m + d],
                                             nd[d], per[d]);
                            dd += r[d] * r[d];
                        }
                        dd = sqrt(dd);
                        if (dd < d0 && dd > 0) {
                            double f = lbmref_hertz(dd, xi, d0);
                            for (int d = 0; d < 3; ++d) c->Fh[3 * i + d] += (real)(f * r[d] / dd);
                        }
                    }
            }
        }
        for (int i = 0; i < 3 * c->nn; ++i) c->F[i] += c->Fh[i];
        /* anchor spring on the centroid, distributed equally over the nodes */
        for (int d = 0; d < 3; ++d) c->f_anchor[d] = 0.0;
        if (c->p.anchor_k != 0.0) {
            for (int d = 0; d < 3; ++d) {
                double fa = -(c->p.anchor_k / c->nn) * (c->cen[d] - c->c0[d]);
                for (int i = 0; i < c->nn; ++i) c->F[3 * i + d] += (real)fa;
                c->f_anchor[d] = fa * c->nn;
            }
        }
        /* pending reaction of the previous step */
        for (int i = 0; i < 3 * c->nn; ++i) c->F[i] += c->R[i];
    }
}

/* ----------------------------------------------------------------------------------- */
/* Immersed boundary: spreading, interpolation, reaction gathering                      */
/* ----------------------------------------------------------------------------------- */

static void spread(lbmref_handle *h) {
    long N = h->N;
    memset(h->fibm, 0, sizeof(real) * 4 * N);
    for (int k = 0; k < h->ncap; ++k) {
        cap_t *c = &h->cap[k];
        for (int n = 0; n < c->nn; ++n) {
            const real *X = c->x + 3 * n;
            int b[3];
            for (int d = 0; d < 3; ++d) b[d] = (int)floor((double)X[d]) - 1;
            for (int oz = 0; oz < 4; ++oz)
                for (int oy = 0; oy < 4; ++oy)
                    for (int ox = 0; ox < 4; ++ox) {
                        int zi = wrapi(b[2] + oz, h->nz);
                        if (is_solid(h, zi)) continue;
                        real w = phi4r(X[0] - (real)(b[0] + ox)) * phi4r(X[1] - (real)(b[1] + oy)) *
                                 phi4r(X[2] - (real)(b[2] + oz));
                        long s = sidx(h, wrapi(b[0] + ox, h->nx), wrapi(b[1] + oy, h->ny), zi);
                        for (int d = 0; d < 3; ++d) h->fibm[d * N + s] += w * c->F[3 * n + d];
                        h->fibm[3 * N + s] += w;
                    }
        }
    }
}

static void update_nodes(lbmref_handle *h) {
    long N = h->N;
    for (int k = 0; k < h->ncap; ++k) {
        cap_t *c = &h->cap[k];
        for (int n = 0; n < c->nn; ++n) {
            real *X = c->x + 3 * n;
            int b[3];
            for (int d = 0; d < 3; ++d) b[d] = (int)floor((double)X[d]) - 1;
            real U[3] = {0, 0, 0}, R[3] = {0, 0, 0};
            for (int oz = 0; oz < 4; ++oz)
                for (int oy = 0; oy < 4; ++oy)
                    for (int ox = 0; ox < 4; ++ox) {
                        int zi = wrapi(b[2] + oz, h->nz);
                        if (is_solid(h, zi)) continue;
                        real w = phi4r(X[0] - (real)(b[0] + ox)) * phi4r(X[1] - (real)(b[1] + oy)) *
                                 phi4r(X[2] - (real)(b[2] + oz));
                        long s = sidx(h, wrapi(b[0] + ox, h->nx), wrapi(b[1] + oy, h->ny), zi);
                        for (int d = 0; d < 3; ++d) U[d] += w * h->uphys[d * N + s];
                        real cov = h->fibm[3 * N + s];
                        if (cov > 0)
                            for (int d = 0; d < 3; ++d) R[d] += w * h->react[d * N + s] / cov;
                    }
            for (int d = 0; d < 3; ++d) {
                X[d] += U[d];
                c->R[3 * n + d] = R[d];
            }
        }
    }
}

/* ----------------------------------------------------------------------------------- */
/* Fluid                                                                                */
/* ----------------------------------------------------------------------------------- */

/* Pull streaming: f_i(x) = f*_i(x - e_i); if x - e_i is solid, half-way bounce-back
 * returns the population that left x towards the wall: f_i(x) = f*_{opp(i)}(x). */
static void pull(const lbmref_handle *h, int i, int j, int k, real out[2][19]) {
    long N = h->N, s = sidx(h, i, j, k);
    for (int q = 0; q < 19; ++q) {
        int si = wrapi(i - EV[q][0], h->nx), sj = wrapi(j - EV[q][1], h->ny),
            sk = wrapi(k - EV[q][2], h->nz);
        for (int c = 0; c < 2; ++c) {
            if (is_solid(h, sk))
                out[c][q] = h->f[((long)c * 19 + OPPQ[q]) * N + s];
            else
                out[c][q] = h->f[((long)c * 19 + q) * N + sidx(h, si, sj, sk)];
        }
    }
}

static inline real psi_of(const lbmref_handle *h, real rho) {
    return 1 - (real)exp(-(double)rho / h->p.rho0);
}

/* wetting offset of the boundary between a site labelled `a` and a neighbour `b` */
static double boundary_drho(const lbmref_handle *h, int a, int b) {
    if (b == LABEL_SOLID) return h->p.wall_drho;
    int k = (b != 0) ? b - 1 : a - 1;
    return h->cap[k].p.wet_drho;
}

static void fluid_step(lbmref_handle *h) {
    long N = h->N;
    const double G = h->p.G;
    int bad = 0;
    long lost = 0;
    /* pass 1: densities and pseudopotentials after streaming */
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int k = 0; k < h->nz; ++k) {
        if (is_solid(h, k)) continue;
        for (int j = 0; j < h->ny; ++j)
            for (int i = 0; i < h->nx; ++i) {
                real fl[2][19];
                pull(h, i, j, k, fl);
                long s = sidx(h, i, j, k);
                for (int c = 0; c < 2; ++c) {
                    real r = 0;
                    for (int q = 0; q < 19; ++q) r += fl[c][q];
                    h->rho[c * N + s] = r;
                    h->psi[c * N + s] = psi_of(h, r);
                    if (!(r >= 0) || !isfinite((double)r)) bad = 1;
                }
            }
    }
    /* pass 2: forces and collision */
#pragma omp parallel for schedule(static) reduction(+ : lost)
    for (int k = 0; k < h->nz; ++k) {
        if (is_solid(h, k)) continue;
        for (int j = 0; j < h->ny; ++j)
            for (int i = 0; i < h->nx; ++i) {
                long s = sidx(h, i, j, k);
                real fl[2][19];
                pull(h, i, j, k, fl);
                real rho[2], jm[2][3];
                for (int c = 0; c < 2; ++c) {
                    rho[c] = 0;
                    jm[c][0] = jm[c][1] = jm[c][2] = 0;
                    for (int q = 0; q < 19; ++q) {
                        rho[c] += fl[c][q];
                        for (int d = 0; d < 3; ++d) jm[c][d] += fl[c][q] * EV[q][d];
                    }
                }
                /* Shan-Chen force, eq. shanchen, with the decoupling across labels */
                int lab = h->label[s];
                real F[2][3], rx[3] = {0, 0, 0};
                for (int c = 0; c < 2; ++c) {
                    int cp = 1 - c;
                    real sum[3] = {0, 0, 0}, cross[3] = {0, 0, 0};
                    for (int q = 1; q < 19; ++q) {
                        int ni = wrapi(i + EV[q][0], h->nx), nj = wrapi(j + EV[q][1], h->ny),
                            nk = wrapi(k + EV[q][2], h->nz);
                        long ns = sidx(h, ni, nj, nk);
                        int nl = h->label[ns];
                        real ps;
                        int is_cross = 0;
                        if (nl == lab) {
                            ps = h->psi[cp * N + ns];
                        } else {
                            /* density of the partner component at x itself plus the
                             * wetting offset (sign +1 for component 0, -1 for 1) */
                            double dr = boundary_drho(h, lab, nl);
                            real rv = rho[cp] + (real)((cp == 0 ? 1.0 : -1.0) * dr);
                            if (rv < 0) rv = 0;
                            ps = psi_of(h, rv);
                            is_cross = (nl != LABEL_SOLID);
                        }
                        real wq = (real)(h->p.sc_norm * OMEGA[q]);
                        for (int d = 0; d < 3; ++d) {
                            sum[d] += wq * ps * EV[q][d];
                            if (is_cross) cross[d] += wq * ps * EV[q][d];
                        }
                    }
                    real pc = h->psi[c * N + s];
                    for (int d = 0; d < 3; ++d) {
                        F[c][d] = (real)(-G) * pc * sum[d];
                        rx[d] += (real)G * pc * cross[d];
                    }
                }
                real rt = rho[0] + rho[1];
                real fb[3] = {h->fibm[s], h->fibm[N + s], h->fibm[2 * N + s]};
                for (int c = 0; c < 2; ++c)
                    for (int d = 0; d < 3; ++d) {
                        if (rt > 0) F[c][d] += rho[c] / rt * fb[d];
                        F[c][d] += rho[c] * (real)h->p.body_force[d];
                    }
                /* Shan-Chen common velocity and per-component equilibrium velocity */
                real num[3] = {0, 0, 0}, den = 0;
                for (int c = 0; c < 2; ++c) {
                    real it = (real)(1.0 / h->p.tau[c]);
                    for (int d = 0; d < 3; ++d) num[d] += jm[c][d] * it;
                    den += rho[c] * it;
                }
                real up[3];
                for (int d = 0; d < 3; ++d) up[d] = den > 0 ? num[d] / den : 0;
                for (int c = 0; c < 2; ++c) {
                    real ue[3], fe[19];
                    real tau = (real)h->p.tau[c];
                    for (int d = 0; d < 3; ++d) ue[d] = rho[c] > 0 ? up[d] + tau * F[c][d] / rho[c] : up[d];
                    feq19(rho[c], ue, fe);
                    for (int q = 0; q < 19; ++q)
                        h->fn[((long)c * 19 + q) * N + s] = fl[c][q] - (fl[c][q] - fe[q]) / tau;
                }
                for (int d = 0; d < 3; ++d) {
                    h->uphys[d * N + s] =
                        rt > 0 ? (jm[0][d] + jm[1][d] + (F[0][d] + F[1][d]) / 2) / rt : 0;
                    h->react[d * N + s] = rx[d];
                }
                if (h->p.coupling == 0 && (rx[0] != 0 || rx[1] != 0 || rx[2] != 0) &&
                    !(h->fibm[3 * N + s] > 0))
                    lost++;
            }
    }
    real *t = h->f; h->f = h->fn; h->fn = t;
    h->lost += lost;
    if (bad) h->unstable = 1;
}

/* ----------------------------------------------------------------------------------- */
/* Half-way bounce-back on the membrane with Ladd's momentum exchange (Section 3.1)     */
/* ----------------------------------------------------------------------------------- */

/* six times the signed volume of the tetrahedron (a, b, c, d) */
static double orient3(const double *a, const double *b, const double *c, const double *d) {
    double ab[3], ac[3], ad[3];
    for (int k = 0; k < 3; ++k) {
        ab[k] = b[k] - a[k];
        ac[k] = c[k] - a[k];
        ad[k] = d[k] - a[k];
    }
    return ab[0] * (ac[1] * ad[2] - ac[2] * ad[1]) + ab[1] * (ac[2] * ad[0] - ac[0] * ad[2]) +
           ab[2] * (ac[0] * ad[1] - ac[1] * ad[0]);
}

double lbmref_miss_distance(const double p0[3], const double p1[3], const double a[3],
                            const double b[3], const double c[3]) {
    /* the line crosses the triangle's plane at parameter t (signed distances of the ends) */
    double s0 = orient3(a, b, c, p0), s1 = orient3(a, b, c, p1);
    double den = s0 - s1;
    if (den == 0.0) return INFINITY;
    double t = s0 / den;
    /* barycentric coordinates of that crossing: the line's orientation against each edge */
    double wa = orient3(p0, p1, b, c), wb = orient3(p0, p1, c, a), wc = orient3(p0, p1, a, b);
    double sum = wa + wb + wc;
    if (sum == 0.0) return INFINITY;
    double u = wa / sum, v = wb / sum, w = wc / sum;
    double d = 0.0;
    if (-u > d) d = -u;
    if (-v > d) d = -v;
    if (-w > d) d = -w;
    if (-t > d) d = -t;
    if (t - 1.0 > d) d = t - 1.0;
    return d;
}

/* nearest periodic image of lattice coordinate i to the unwrapped position x */
static int image_of(int i, double x, int n, int periodic) {
    return periodic ? i + n * (int)floor((x - i) / n + 0.5) : i;
}

/* The triangle of capsule c crossed by the segment p0 -> p1 (capsule frame): among the
 * triangles whose bounding box (FP32-rounded nodes) meets the segment's closed bounding
 * box, the one of least miss distance, the lowest index on ties; -1 if none qualifies. */
static int link_triangle(const cap_t *c, const double p0[3], const double p1[3]) {
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = p0[d] < p1[d] ? p0[d] : p1[d];
        hi[d] = p0[d] < p1[d] ? p1[d] : p0[d];
    }
    int best = -1;
    double bd = INFINITY;
    for (int t = 0; t < c->nt; ++t) {
        double v[3][3];
        int ok = 1;
        for (int m = 0; m < 3; ++m)
            for (int d = 0; d < 3; ++d) v[m][d] = (double)(float)c->x[3 * c->tri[3 * t + m] + d];
        for (int d = 0; d < 3 && ok; ++d) {
            double tl = v[0][d], th = v[0][d];
            for (int m = 1; m < 3; ++m) {
                if (v[m][d] < tl) tl = v[m][d];
                if (v[m][d] > th) th = v[m][d];
            }
            if (tl > hi[d] || th < lo[d]) ok = 0;
        }
        if (!ok) continue;
        double md = lbmref_miss_distance(p0, p1, v[0], v[1], v[2]);
        if (md < bd) { bd = md; best = t; }
    }
    return best;
}

/* Find this step's links: every site a inside capsule k (label k+1) and direction q whose
 * neighbour b = a + e_q is fluid of another side (exterior, or a capsule of higher
 * index: the lower index owns a link between two capsules). */
static void find_links(lbmref_handle *h) {
    h->nlinks = 0;
    for (int k = 0; k < h->ncap; ++k) {
        cap_t *c = &h->cap[k];
        double cen[3];
        centroid_of(c->nn, c->x, cen);
        for (int kk = 0; kk < h->nz; ++kk)
            for (int jj = 0; jj < h->ny; ++jj)
                for (int ii = 0; ii < h->nx; ++ii) {
                    long a = sidx(h, ii, jj, kk);
                    if (h->label[a] != k + 1) continue;
                    for (int q = 1; q < 19; ++q) {
                        int bi = wrapi(ii + EV[q][0], h->nx), bj = wrapi(jj + EV[q][1], h->ny),
                            bk = wrapi(kk + EV[q][2], h->nz);
                        long b = sidx(h, bi, bj, bk);
                        int lb = h->label[b];
                        if (lb == k + 1 || lb == LABEL_SOLID || (lb != 0 && lb < k + 1)) continue;
                        double p0[3] = {image_of(ii, cen[0], h->nx, 1),
                                        image_of(jj, cen[1], h->ny, 1),
                                        image_of(kk, cen[2], h->nz, !h->p.wall_z0)};
                        double p1[3] = {p0[0] + EV[q][0], p0[1] + EV[q][1], p0[2] + EV[q][2]};
                        if (h->nlinks == h->links_cap) {
                            h->links_cap = h->links_cap ? 2 * h->links_cap : 4096;
                            h->links = (link_t *)realloc(h->links, sizeof(link_t) * h->links_cap);
                        }
                        link_t *L = &h->links[h->nlinks++];
                        L->a = a; L->b = b; L->q = q; L->k = k;
                        L->tri = link_triangle(c, p0, p1);
                    }
                }
    }
}

/* Bounce-back of every link on the post-collision populations, before streaming: the
 * population of a towards b is replaced by b's population towards a reflected by the
 * membrane, and vice versa, each with the moving-wall term delta = 2 w_q rho u_b.e_q / c_s^2
 * (rho: the mean density of the component over the link's two sites, u_b: the mean velocity
 * of the crossed triangle's nodes), so that plain pull streaming delivers
 * f_q(b) = f*_qbar(b) + delta and f_qbar(a) = f*_q(a) - delta.  The momentum given to the
 * membrane, (2 f*_q(a) - 2 f*_qbar(b) - 2 delta) e_q summed over the components, goes to the
 * crossed triangle, a third to each of its nodes. */
static void bounce_back(lbmref_handle *h) {
    long N = h->N;
    for (int k = 0; k < h->ncap; ++k) memset(h->cap[k].Pex, 0, sizeof(real) * 3 * h->cap[k].nn);
    /* densities of the populations before any link is changed */
    real *rho = (real *)malloc(sizeof(real) * 2 * N);
    for (int c = 0; c < 2; ++c)
        for (long s = 0; s < N; ++s) {
            real r = 0;
            for (int q = 0; q < 19; ++q) r += h->f[((long)c * 19 + q) * N + s];
            rho[c * N + s] = r;
        }
    for (long l = 0; l < h->nlinks; ++l) {
        const link_t *L = &h->links[l];
        cap_t *cp = &h->cap[L->k];
        int q = L->q, qb = OPPQ[q];
        real ub[3] = {0, 0, 0};
        if (L->tri >= 0)
            for (int m = 0; m < 3; ++m)
                for (int d = 0; d < 3; ++d) ub[d] += cp->V[3 * cp->tri[3 * L->tri + m] + d] / 3;
        real eu = ub[0] * EV[q][0] + ub[1] * EV[q][1] + ub[2] * EV[q][2];
        real dp = 0;
        for (int c = 0; c < 2; ++c) {
            real *fa = &h->f[((long)c * 19 + q) * N + L->a];
            real *fb = &h->f[((long)c * 19 + qb) * N + L->b];
            real rb = (rho[c * N + L->a] + rho[c * N + L->b]) / 2;
            real delta = 2 * (real)OMEGA[q] * rb * eu * 3;
            real va = *fa, vb = *fb;
            *fa = vb + delta;
            *fb = va - delta;
            dp += 2 * va - 2 * vb - 2 * delta;
        }
        if (L->tri < 0) { h->lost_links++; continue; }
        for (int m = 0; m < 3; ++m)
            for (int d = 0; d < 3; ++d)
                cp->Pex[3 * cp->tri[3 * L->tri + m] + d] += dp * EV[q][d] / 3;
    }
    free(rho);
}

/* Shan-Chen reaction of every link after the fluid step: the cross-membrane parts of the
 * force on a (from b) and on b (from a), with the same substitution as the fluid step,
 * returned to the crossed triangle, a third to each of its nodes. */
static void link_reaction(lbmref_handle *h) {
    long N = h->N;
    const double G = h->p.G;
    for (int k = 0; k < h->ncap; ++k) memset(h->cap[k].Rsc, 0, sizeof(real) * 3 * h->cap[k].nn);
    for (long l = 0; l < h->nlinks; ++l) {
        const link_t *L = &h->links[l];
        if (L->tri < 0) continue;
        cap_t *cp = &h->cap[L->k];
        int q = L->q, la = h->label[L->a], lb = h->label[L->b];
        real wq = (real)(h->p.sc_norm * OMEGA[q]);
        double dra = boundary_drho(h, la, lb), drb = boundary_drho(h, lb, la);
        real r = 0;
        for (int c = 0; c < 2; ++c) {
            int cq = 1 - c;
            real sg = (real)(cq == 0 ? 1.0 : -1.0);
            real ra = h->rho[cq * N + L->a] + sg * (real)dra;
            real rbv = h->rho[cq * N + L->b] + sg * (real)drb;
            if (ra < 0) ra = 0;
            if (rbv < 0) rbv = 0;
            r += (real)G * wq * (h->psi[c * N + L->a] * psi_of(h, ra) -
                                 h->psi[c * N + L->b] * psi_of(h, rbv));
        }
        for (int m = 0; m < 3; ++m)
            for (int d = 0; d < 3; ++d) cp->Rsc[3 * cp->tri[3 * L->tri + m] + d] += r * EV[q][d] / 3;
    }
}

/* Newtonian nodes of mass m (Section 3.2): the exchanged momentum spread over this and the
 * next step, v += (F_membrane + (P_ex(n) + P_ex(n-1)) / 2 + R_sc) / m, x += v. */
static void update_nodes_bb(lbmref_handle *h) {
    real im = (real)(1.0 / h->p.node_mass);
    for (int k = 0; k < h->ncap; ++k) {
        cap_t *c = &h->cap[k];
        for (int d = 0; d < 3; ++d) c->f_fluid[d] = 0.0;
        for (int n = 0; n < c->nn; ++n)
            for (int d = 0; d < 3; ++d) {
                int i = 3 * n + d;
                real ff = (c->Pex[i] + c->Pprev[i]) / 2 + c->Rsc[i];
                c->f_fluid[d] += ff;
                c->V[i] += (c->F[i] + ff) * im;
                c->x[i] += c->V[i];
                c->Pprev[i] = c->Pex[i];
            }
    }
}

int lbmref_step(lbmref_handle *h, int64_t n) {
    if (!h || n < 0) { set_err("invalid step call"); return -1; }
    for (int64_t s = 0; s < n; ++s) {
        compute_labels(h);
        membrane_forces(h);
        if (h->p.coupling == 1) {
            find_links(h);
            bounce_back(h);
            fluid_step(h);
            link_reaction(h);
            update_nodes_bb(h);
        } else {
            spread(h);
            fluid_step(h);
            update_nodes(h);
        }
        h->step++;
    }
    return h->unstable ? -4 : 0;
}

/* ----------------------------------------------------------------------------------- */
/* Observables                                                                          */
/* ----------------------------------------------------------------------------------- */

int lbmref_rho(const lbmref_handle *h, double *out) {
    long N = h->N;
    for (int c = 0; c < 2; ++c)
        for (long s = 0; s < N; ++s) {
            int k = (int)(s / ((long)h->nx * h->ny));
            if (is_solid(h, k)) { out[c * N + s] = 0.0; continue; }
            real r = 0;
            for (int q = 0; q < 19; ++q) r += h->f[((long)c * 19 + q) * N + s];
            out[c * N + s] = r;
        }
    return 0;
}

int lbmref_velocity(const lbmref_handle *h, double *out) {
    for (long s = 0; s < 3 * h->N; ++s) out[s] = h->uphys[s];
    return 0;
}

/* Meniscus height of each column: the first crossing of phi = (rho1-rho2)/(rho1+rho2)
 * from >= 0 to < 0 going up, linearly interpolated; NaN where there is none or where
 * either site of the crossing lies inside a capsule. */
int lbmref_meniscus(const lbmref_handle *h, double *out) {
    long N = h->N;
    int k0 = h->p.wall_z0 ? 1 : 0;
    for (int j = 0; j < h->ny; ++j)
        for (int i = 0; i < h->nx; ++i) {
            double res = NAN;
            for (int k = k0; k + 1 < h->nz; ++k) {
                double ph[2];
                for (int kk = 0; kk < 2; ++kk) {
                    long s = sidx(h, i, j, k + kk);
                    real r0 = 0, r1 = 0;
                    for (int q = 0; q < 19; ++q) {
                        r0 += h->f[(long)q * N + s];
                        r1 += h->f[((long)19 + q) * N + s];
                    }
                    ph[kk] = ((double)r0 - (double)r1) / ((double)r0 + (double)r1);
                }
                if (ph[0] >= 0.0 && ph[1] < 0.0) {
                    if (h->label[sidx(h, i, j, k)] == 0 && h->label[sidx(h, i, j, k + 1)] == 0)
                        res = k + ph[0] / (ph[0] - ph[1]);
                    break;
                }
            }
            out[(long)j * h->nx + i] = res;
        }
    return 0;
}

int lbmref_capsule_nodes(const lbmref_handle *h, int32_t k, double *xyz) {
    if (!h || k < 0 || k >= h->ncap) { set_err("invalid capsule index"); return -1; }
    const cap_t *c = &h->cap[k];
    for (int i = 0; i < 3 * c->nn; ++i) xyz[i] = c->x[i];
    return 0;
}

int lbmref_capsule_observe(lbmref_handle *h, int32_t k, lbmref_capsule_obs *o) {
    if (!h || k < 0 || k >= h->ncap || !o) { set_err("invalid capsule index"); return -1; }
    cap_t *c = &h->cap[k];
    double cen[3];
    centroid_of(c->nn, c->x, cen);
    for (int d = 0; d < 3; ++d) {
        o->centroid[d] = cen[d];
        o->f_anchor[d] = -c->f_anchor[d];
        double sr = 0, sh = 0;
        for (int i = 0; i < c->nn; ++i) {
            sr += h->p.coupling == 1 ? c->Rsc[3 * i + d] : c->R[3 * i + d];
            sh += c->Fh[3 * i + d];
        }
        o->f_capillary[d] = sr;
        o->f_hertz[d] = sh;
        o->f_fluid[d] = h->p.coupling == 1 ? c->f_fluid[d] : sr;
    }
    o->volume = volume_of(c->nn, c->x, c->nt, c->tri, cen);
    return 0;
}

typedef struct { double s, c; } ksum;
static void kadd(ksum *a, double v) {
    double y = v - a->c, t = a->s + y;
    a->c = (t - a->s) - y;
    a->s = t;
}

int lbmref_get_summary(lbmref_handle *h, lbmref_summary *o) {
    long N = h->N;
    memset(o, 0, sizeof *o);
    /* compensated (Kahan) sums over all populations */
    for (int c = 0; c < 2; ++c) {
        ksum m = {0, 0}, mom[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (long s = 0; s < N; ++s) {
            int k = (int)(s / ((long)h->nx * h->ny));
            if (is_solid(h, k)) continue;
            for (int q = 0; q < 19; ++q) {
                double v = h->f[((long)c * 19 + q) * N + s];
                kadd(&m, v);
                for (int d = 0; d < 3; ++d)
                    if (EV[q][d]) kadd(&mom[d], v * EV[q][d]);
            }
        }
        o->mass[c] = m.s;
        for (int d = 0; d < 3; ++d) o->momentum[d] += mom[d].s;
    }
    for (int k = 0; k < h->ncap; ++k)
        for (int i = 0; i < h->cap[k].nn; ++i)
            for (int d = 0; d < 3; ++d) {
                const cap_t *c = &h->cap[k];
                /* bounce-back: half of the last exchange is still to be applied */
                o->pending[d] += h->p.coupling == 1 ? c->Pprev[3 * i + d] / 2 : c->R[3 * i + d];
                o->node_momentum[d] += h->p.coupling == 1 ? h->p.node_mass * c->V[3 * i + d] : 0.0;
            }
    o->lost_links = h->lost_links;
    o->links = h->nlinks;
    o->step = h->step;
    o->lost_reaction = h->lost;
    o->n_capsules = h->ncap;
    o->unstable = h->unstable;
    return 0;
}

void lbmref_destroy(lbmref_handle *h) {
    if (!h) return;
    for (int k = 0; k < h->ncap; ++k) {
        cap_t *c = &h->cap[k];
        free(c->x); free(c->R); free(c->F); free(c->Fh); free(c->tri); free(c->minv); free(c->a0);
        free(c->edge); free(c->th0);
        free(c->V); free(c->Pex); free(c->Pprev); free(c->Rsc);
    }
    free(h->cap);
    free(h->f); free(h->fn); free(h->rho); free(h->psi); free(h->label);
    free(h->fibm); free(h->uphys); free(h->react);
    free(h->links);
    free(h);
}
