/*
 * lbmref.h -- CPU oracle for the two-component Shan-Chen D3Q19 lattice Boltzmann fluid
 * coupled to triangulated Skalak capsule membranes by an immersed boundary or by
 * half-way bounce-back with momentum exchange (Section 3.1).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the HIP library.
 *
 * Every routine is a plain, slow loop over sites, nodes or triangles in double
 * precision (compile with -DLBMREF_REAL=float for an FP32 diagnostic build).
 * All entry points take and return double data regardless of the internal type.
 */
#ifndef LBMREF_H
#define LBMREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbmref_handle lbmref_handle;

typedef struct {
    int32_t nx, ny, nz;        /* lattice size; periodic in x, y, z                          */
    int32_t wall_z0;           /* 1: layer z=0 is a resting solid wall (half-way bounce-back) */
    double tau[2];             /* BGK relaxation time per component (Section 3.1)            */
    double G;                  /* inter-component coupling G^{12}=G^{21}; G^{cc}=0            */
    double rho0;               /* reference density in psi = 1 - exp(-rho/rho0)              */
    double sc_norm;            /* Shan-Chen stencil weights w_i = sc_norm * omega_i           */
    double body_force[3];      /* acceleration g; force density rho^c g                     */
    double wall_drho;          /* wetting offset of the wall (0: neutral)                    */
    int32_t init_mode;         /* 0 uniform, 1 film, 2 caller array                          */
    int32_t n_threads;         /* OpenMP threads (0: runtime default)                        */
    double init_rho[2];        /* mode 0 densities                                           */
    double film_height;        /* mode 1: number of film layers above the wall               */
    double rho_maj, rho_min, rho_iface;    /* mode 1 densities (Section 3.2)                 */
    const double *init_rho_array;          /* mode 2: [2][nz][ny][nx], copied              */
    double hertz_xi, hertz_delta0;         /* Hertz repulsion strength and range           */
    double plane_dz;           /* repulsive plane at z = 0.5 + plane_dz (wall only)          */
    int32_t coupling;          /* 0: immersed boundary; 1: half-way bounce-back on the
                                  membrane with momentum exchange (Section 3.1)              */
    double node_mass;          /* bounce-back coupling: mass of every membrane node          */
} lbmref_params;

typedef struct {
    double ks;        /* Skalak shear modulus kappa_S                     */
    double C;         /* Skalak area constant C                           */
    double kb;        /* bending modulus kappa_B (eq. method:curvature), >= 0 */
    double kv;        /* volume penalty kappa_V                           */
    double wet_drho;  /* wetting offset of the membrane (0: neutral)      */
    double anchor_k;  /* centroid anchor spring (0: free)                 */
} lbmref_capsule_params;

typedef struct {
    double centroid[3];
    double volume;
    double f_anchor[3];     /* force of the fluid on the anchored capsule (= -sum of anchor forces) */
    double f_capillary[3];  /* sum of the pending membrane reaction R_n          */
    double f_hertz[3];      /* sum of Hertz forces on the capsule nodes          */
    double f_fluid[3];      /* force of the fluid on the membrane in the last step (bounce-
                               back: smoothed momentum exchange plus the Shan-Chen reaction;
                               immersed boundary: the Shan-Chen reaction)              */
} lbmref_capsule_obs;

typedef struct {
    double mass[2];         /* sum over fluid sites of rho^c                      */
    double momentum[3];     /* fluid momentum sum_x sum_c sum_i f*_i e_i          */
    double pending[3];      /* sum over all nodes of the pending reaction R_n     */
    int64_t step;
    int64_t lost_reaction;  /* sites with cross-membrane links and zero coverage  */
    int32_t n_capsules;
    int32_t unstable;       /* 1 if a non-finite or negative density was seen     */
    double node_momentum[3];/* bounce-back coupling: sum of node mass x velocity  */
    int64_t lost_links;     /* bounce-back links that found no triangle           */
    int64_t links;          /* bounce-back links of the last step                 */
} lbmref_summary;

const char *lbmref_error(void);
lbmref_handle *lbmref_create(const lbmref_params *p);
int lbmref_add_capsule(lbmref_handle *h, const lbmref_capsule_params *cp, int32_t n_nodes,
                       const double *xyz, int32_t n_tri, const int32_t *tri);
int lbmref_step(lbmref_handle *h, int64_t n);
int lbmref_rho(const lbmref_handle *h, double *out);           /* [2][nz][ny][nx]        */
int lbmref_velocity(const lbmref_handle *h, double *out);      /* [3][nz][ny][nx]        */
int lbmref_meniscus(const lbmref_handle *h, double *out);      /* [ny][nx], NaN: none    */
int lbmref_labels(lbmref_handle *h, uint8_t *out);             /* [nz][ny][nx] at X^n    */
int lbmref_capsule_nodes(const lbmref_handle *h, int32_t k, double *xyz);
int lbmref_capsule_observe(lbmref_handle *h, int32_t k, lbmref_capsule_obs *out);
int lbmref_get_summary(lbmref_handle *h, lbmref_summary *out);
void lbmref_destroy(lbmref_handle *h);

/* Pure helpers exposed for the pin tests. */
void lbmref_lattice(int32_t e[19 * 3], double omega[19], int32_t opp[19]);
void lbmref_feq(double rho, const double u[3], double out[19]);
double lbmref_phi4(double r);
void lbmref_sc_sum(const double psi27[27], double sc_norm, double out[3]);
void lbmref_reference_geometry(int32_t n_nodes, const double *xyz, int32_t n_tri,
                               const int32_t *tri, double *minv, double *a0);
double lbmref_skalak(int32_t n_nodes, const double *xyz, int32_t n_tri, const int32_t *tri,
                     const double *minv, const double *a0, double ks, double C, double *force);
/* Bending energy sqrt(3) kb sum_e (theta_e - theta0_e)^2 over the edges shared by two
 * triangles, theta0 from ref (node positions of the reference mesh) or 0 if ref is NULL;
 * force [n_nodes][3] = -dE/dx if not NULL.  NaN for a non-manifold mesh. */
double lbmref_bending(int32_t n_nodes, const double *xyz, int32_t n_tri, const int32_t *tri,
                      const double *ref, double kb, double *force);
double lbmref_volume(int32_t n_nodes, const double *xyz, int32_t n_tri, const int32_t *tri);
void lbmref_volume_force(int32_t n_nodes, const double *xyz, int32_t n_tri, const int32_t *tri,
                         double kv, double v0, double *force);
double lbmref_hertz(double d, double xi, double delta0);
/* Miss distance of the segment p0 -> p1 from triangle (a, b, c): 0 when the closed
 * segment meets the closed triangle, else max(-u, -v, -w, -t, t - 1) with (u, v, w) the
 * barycentric coordinates of the segment's line in the triangle's plane and t the segment
 * parameter there; +inf when the line is parallel to the plane.  Evaluated in double. */
double lbmref_miss_distance(const double p0[3], const double p1[3], const double a[3],
                            const double b[3], const double c[3]);
int lbmref_column_labels(int32_t n_nodes, const double *xyz, int32_t n_tri, const int32_t *tri,
                         int32_t x0, int32_t y0, int32_t z0, int32_t dx, int32_t dy, int32_t dz,
                         uint8_t *inside);

#ifdef __cplusplus
}
#endif
#endif
