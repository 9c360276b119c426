/*
 * lbm.h -- C ABI of the MI355X library for the coupled lattice Boltzmann / capsule
 * time step of Wouters, Aouane, Sega and Harting, "Capillary interactions between soft
 * capsules protruding through thin fluid films" (arXiv:2007.15405).
 *
 * One time step (all on the GPU, on the handle's stream):
 *   - side labels of every lattice site from the capsule meshes (interior/exterior
 *     decoupling of the Shan-Chen force, Section 3.1);
 *   - membrane node forces: Skalak strain energy by virtual work (eq. strain), bending
 *     (eq. method:curvature, edge form), volume penalty (eq. vol_cons), Hertz particle-substrate / particle-particle repulsion
 *     (Section 3.2, eq. interactions), a centroid anchor, and the pending reaction of
 *     the cross-membrane Shan-Chen links;
 *   - immersed-boundary spreading of the node forces (Peskin 4-point kernel);
 *   - the fused fluid step: pull streaming with half-way bounce-back at the wall,
 *     densities, pseudopotential psi = 1 - exp(-rho/rho0) (Section 3.1), Shan-Chen
 *     force (eq. shanchen) with the label substitution, BGK collision (eq.
 *     method:boltzmann) towards the second-order equilibrium (eq. lbm:equilibrium) at
 *     the Shan-Chen shifted velocity;
 *   - interpolation of the physical velocity to the nodes, node advection and
 *     gathering of the reaction onto the nodes.
 *
 * With coupling = 1 (lbm_params) the membrane is coupled as in Section 3.1 instead: every
 * lattice link between a site inside a capsule and one outside is bounced back half-way on
 * the membrane triangle it crosses (Ladd's moving-wall term with the mean velocity of the
 * triangle's three nodes), before streaming; the exchanged momentum and the Shan-Chen force
 * across the link go a third to each node of that triangle (homogeneous weighting); the
 * exchanged momentum acts half in this step and half in the next (against staggered
 * momenta); and the nodes, of mass node_mass, follow v += F / m, x += v.  Nothing is
 * spread or interpolated.  Batches take immersed-boundary handles only.
 *
 * Conventions
 *   Lattice units (dx = dt = 1).  Site (i, j, k) sits at position (i, j, k); arrays over
 *   sites are [nz][ny][nx] with x fastest.  The lattice is periodic in x, y and z; with
 *   wall_z0 the layer k = 0 is a resting solid wall, so the fluid occupies k = 1..nz-1
 *   between half-way bounce-back planes at z = 0.5 and z = nz - 0.5.
 *   Component 0 is the film liquid, component 1 the covering fluid.
 *
 * Slabs (independent runs in one lattice)
 *   With slab_nz < nz the lattice holds nz / slab_nz independent boxes of
 *   nx x ny x slab_nz sites stacked along z; slab s occupies k = s * slab_nz ..
 *   (s + 1) * slab_nz - 1 and its own solid layer is k = s * slab_nz.  The wall layer of
 *   the slab above bounds slab s exactly as the periodic wrap bounds a single walled box,
 *   so every slab evolves as the box nx x ny x slab_nz with wall_z0 would on its own.
 *   A capsule belongs to the slab holding its initial centroid; its repulsive plane is
 *   at s * slab_nz + 0.5 + plane_dz, it meets the capsules of its own slab only, and its
 *   site window must stay between the wall layers s * slab_nz and (s + 1) * slab_nz.
 *
 * Ownership and threading
 *   The library owns all device memory of a handle.  Caller buffers passed to the
 *   entry points are host memory owned by the caller, unless the name says "device".
 *   A handle is used by one host thread at a time.  lbm_step only enqueues work on
 *   the handle's stream and returns; the observation calls synchronise the stream.
 *
 * Errors
 *   Every entry point returns an lbm_status; on failure lbm_last_error(h) holds a
 *   message (lbm_last_error(NULL) holds the message of a failed lbm_init).  No C++
 *   exception crosses this interface.  LBM_E_UNSTABLE reports a non-finite or
 *   negative density, a capsule that outgrew its immersed-boundary window or whose
 *   window left its slab; the state is then undefined but the handle can still be
 *   destroyed.
 */
#ifndef LBM_H
#define LBM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_handle lbm_handle;

/* Limits: capsules per simulation, nodes per capsule mesh. */
#define LBM_MAX_CAPSULES 125
#define LBM_MAX_CAPSULE_NODES 8192

typedef enum {
    LBM_OK = 0,
    LBM_E_INVAL = -1,     /* invalid argument or parameter                     */
    LBM_E_NOMEM = -2,     /* device or host allocation failed                  */
    LBM_E_DEVICE = -3,    /* a HIP runtime call failed                         */
    LBM_E_UNSTABLE = -4,  /* non-finite / negative density or capsule overflow */
    LBM_E_STATE = -5      /* call not allowed in the current state             */
} lbm_status;

/* Population storage in HBM.  The collision arithmetic is FP32 in every mode.
 * Modes 1 and 2 store g_i = f_i - w_i * rho_shift[c] (w_i the lattice weights), rounded to
 * nearest even, and decode f_i = g_i + w_i * rho_shift[c].  Mode 3 stores, in FP16, the
 * relative deviation d_i = f_i / (w_i * rho^c(x)) - 1 from the rest equilibrium at the
 * site's own post-collision density rho^c(x), which is stored in FP32 beside the
 * populations, and decodes f_i = w_i * rho^c(x) * (1 + d_i) (w_i here FP32 weights that
 * sum to exactly 1; the rest population absorbs the rounding of the others, so a site's
 * stored mass is its density to one FP16 rounding of a second-order term).  Both phases of a
 * two-component film keep FP16's relative precision (152 + 16 bytes per site update); it
 * needs tau = 1 in both components and the immersed-boundary coupling, and runs the
 * software-pipelined fluid kernels (lbm_set_launch tiles 1..5 and 0 take tile 10). */
typedef enum {
    LBM_STORE_F32 = 0,
    LBM_STORE_F16_SHIFT = 1,
    LBM_STORE_BF16_SHIFT = 2,
    LBM_STORE_F16_LOCAL = 3
} lbm_storage;

typedef struct {
    int32_t nx, ny, nz;        /* lattice size, each >= 3; 10 * nx * ny * nz * (4 bytes for
                                  FP32 storage, 2 for 16-bit) below 2^32                    */
    int32_t wall_z0;           /* 1: solid wall layer at k = 0                               */
    double tau[2];             /* BGK relaxation time per component, > 1/2 (Section 3.1)    */
    double G;                  /* Shan-Chen coupling G^{12} = G^{21}; G^{cc} = 0 (eq. shanchen) */
    double rho0;               /* reference density in psi = 1 - exp(-rho / rho0)          */
    double sc_norm;            /* stencil weights sc_norm * omega_i (1: eq. shanchen as printed) */
    double body_force[3];      /* acceleration g: force density rho^c g                    */
    double wall_drho;          /* wetting offset of the wall in the substitution (0 neutral) */
    int32_t init_mode;         /* 0 uniform init_rho, 1 film (Section 3.2), 2 init_rho_array */
    int32_t storage;           /* lbm_storage                                              */
    double init_rho[2];        /* mode 0 densities                                         */
    double film_height;        /* mode 1: number of film layers above the wall             */
    double rho_maj, rho_min, rho_iface; /* mode 1 densities (0.7, 0.04, 0.3 in the paper) */
    const double *init_rho_array; /* mode 2: host [2][nz][ny][nx], copied during lbm_init */
    double hertz_xi, hertz_delta0; /* Hertz strength and cut-off (1.5, 1.5 in the paper)    */
    double plane_dz;           /* repulsive plane at z = 0.5 + plane_dz (wall only)        */
    double rho_shift[2];       /* 16-bit storage shift per component (paper: rho0)        */
    void *stream;              /* hipStream_t to enqueue on (see stream_given)             */
    int32_t device;            /* HIP device ordinal                                       */
    int32_t stream_given;      /* 1: use `stream` as given, NULL meaning the null stream;
                                  0: NULL makes a private stream of the library             */
    int32_t slab_nz;           /* 0 or nz: one box.  Otherwise the height of each stacked
                                  slab (>= 3, dividing nz; needs wall_z0), see above        */
    const double *slab_film_height; /* mode 1 with slabs: host [nz / slab_nz] film layers per
                                  slab, or NULL for film_height in every slab; read during
                                  lbm_init                                                  */
    int32_t coupling;          /* fluid-membrane coupling: 0 immersed boundary (Peskin
                                  4-point spreading and interpolation, nodes advected with
                                  the fluid); 1 half-way bounce-back on the membrane with
                                  Ladd's momentum exchange (Section 3.1), see below         */
    double node_mass;          /* coupling 1: mass of every membrane node (25 rho0 in
                                  Section 3.2), > 0                                         */
} lbm_params;

typedef struct {
    double ks;        /* Skalak shear modulus kappa_S (eq. strain)                       */
    double C;         /* Skalak area constant C > -1/2; kappa_A = kappa_S (1 + 2C)        */
    double kb;        /* bending modulus kappa_B >= 0 (eq. method:curvature), in the edge
                         form sqrt(3) kb sum_e (theta_e - theta0_e)^2 over the mesh edges,
                         theta the dihedral angle, theta0 that of the reference mesh;
                         kb != 0 needs a closed, consistently oriented mesh            */
    double kv;        /* volume penalty kappa_V (eq. vol_cons)                           */
    double wet_drho;  /* wetting offset of the membrane (0 neutral)                      */
    double anchor_k;  /* centroid anchor spring; 0 leaves the capsule free               */
} lbm_capsule_params;

typedef struct {
    double centroid[3];     /* node mean at the current positions                         */
    double volume;          /* enclosed volume at the current positions                   */
    double f_anchor[3];     /* force of the fluid on an anchored capsule (last step)      */
    double f_capillary[3];  /* sum of the cross-membrane Shan-Chen reaction (immersed
                               boundary: pending for the next step; bounce-back: of the
                               last step)                                                 */
    double f_hertz[3];      /* sum of Hertz forces of the last step                       */
    double f_fluid[3];      /* force of the fluid on the membrane in the last step: with
                               bounce-back the exchanged momentum applied (smoothed) plus
                               the Shan-Chen reaction; with the immersed boundary equal to
                               f_capillary                                                */
} lbm_capsule_obs;

typedef struct {
    double mass[2];         /* sum over fluid sites of rho^c (double accumulation)        */
    double momentum[3];     /* fluid momentum sum_x sum_c sum_i f*_i e_i                  */
    double pending[3];      /* sum over all nodes of the pending reaction (bounce-back:
                               half of the last step's exchanged momentum, still to act)  */
    int64_t step;           /* completed time steps                                       */
    int64_t lost_reaction;  /* site-steps whose reaction found no kernel coverage         */
    int32_t n_capsules;
    int32_t unstable;       /* 1: non-finite / negative density or capsule overflow seen  */
    double node_momentum[3];/* bounce-back coupling: sum over nodes of mass x velocity     */
    int64_t links;          /* bounce-back coupling: membrane links of the last step      */
    int64_t lost_links;     /* bounce-back links that found no triangle (all steps)       */
} lbm_summary;

typedef struct {
    float *rho;                 /* host [2][nz][ny][nx] densities rho^c, or NULL          */
    float *meniscus;            /* host [n_slabs][ny][nx] meniscus height above the slab's
                                   own wall layer (NaN: none), or NULL                    */
    lbm_capsule_obs *capsules;  /* host [n_capsules], or NULL                            */
    double *slab_mass;          /* host [n_slabs][2] mass per slab and component, or NULL */
    lbm_summary summary;        /* always filled                                          */
} lbm_obs;

/* Per-kernel timing, collected when profiling is on (lbm_set_profiling). */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
} lbm_kernel_stat;

/* Create a simulation: validates the parameters, allocates the device state and sets
 * f*_i = f^eq_i(rho^c, 0) (eq. lbm:equilibrium at rest) from the initial densities.
 * init_rho_array is read during the call only.  On failure *out is NULL. */
lbm_status lbm_init(const lbm_params *params, lbm_handle **out);

/* Add a capsule: a closed triangle mesh, outward counter-clockwise,
 * 4 <= n_nodes <= LBM_MAX_CAPSULE_NODES, at most LBM_MAX_CAPSULES per simulation,
 * xyz host [n_nodes][3] (unwrapped lattice coordinates), tri host [n_tri][3].  The mesh
 * at this moment is the stress-free reference (Section 3.1).  Its site window (bounding
 * box widened by the kernel support: floor(max) - floor(min) + 4 sites per axis) must be at
 * most 64 sites and the lattice size per axis, and at most 2048 columns in x * y, and
 * with slabs lie between the wall layers of the capsule's slab; LBM_E_INVAL otherwise (a capsule that outgrows it later is reported by lbm_sync as
 * LBM_E_UNSTABLE).  Copied during the call.
 * Only before the first lbm_step (LBM_E_STATE afterwards).  *id_out gets the index. */
lbm_status lbm_add_capsule(lbm_handle *h, const lbm_capsule_params *cp, int32_t n_nodes,
                           const double *xyz, int32_t n_tri, const int32_t *tri,
                           int32_t *id_out);

/* Add a spherical capsule of the given centre (unwrapped lattice coordinates) and radius:
 * the library builds the mesh in FP64, a geodesic sphere of n_tri = 20 * 4^L triangles
 * (L = 0 .. 6; 1280 and 5120 for the configurations of Section 3.2's particle sizes): the
 * icosahedron with every edge split at its midpoint L times and each new vertex projected
 * onto the sphere, outward counter-clockwise, and adds it as lbm_add_capsule does (same
 * limits and errors; LBM_E_INVAL for another n_tri or a non-finite centre or radius). */
lbm_status lbm_add_sphere_capsule(lbm_handle *h, const lbm_capsule_params *cp,
                                  const double center[3], double radius, int32_t n_tri,
                                  int32_t *id_out);

/* Enqueue n >= 0 time steps on the handle's stream; returns without waiting.  One step is
 * the time step of Section 3.1 as listed at the top of this file: labels, membrane forces,
 * coupling, and the lattice Boltzmann update of eq. method:boltzmann. */
lbm_status lbm_step(lbm_handle *h, int64_t n);

/* Wait for all enqueued work; reports LBM_E_UNSTABLE if an instability was flagged. */
lbm_status lbm_sync(lbm_handle *h);

/* Observables of the current state (synchronises); fills the non-NULL caller buffers:
 * the density fields, the meniscus height of every column (the first upward crossing of
 * (rho1 - rho2) / (rho1 + rho2) through 0, interpolated linearly, NaN where there is none or
 * it lies inside a capsule: the meniscus profiles of Section 4.1), each capsule's centroid,
 * volume and forces (the anchor force is the force sampled on a fixed particle in Section
 * 4.1), masses and momentum. */
lbm_status lbm_observables(lbm_handle *h, lbm_obs *out);

/* Densities rho^c written to a caller-owned DEVICE buffer [2][nz][ny][nx] float, on the
 * handle's stream (no synchronisation).  Solid sites get 0. */
lbm_status lbm_rho_device(lbm_handle *h, float *rho_device);

/* Current node positions of capsule k: host [n_nodes][3] (synchronises). */
lbm_status lbm_capsule_nodes(lbm_handle *h, int32_t k, double *xyz);

/* Site labels used by the last step: host [nz][ny][nx]; 0 exterior, k+1 inside
 * capsule k, 255 wall layer (synchronises). */
lbm_status lbm_labels(lbm_handle *h, uint8_t *out);

/* Checkpoint: populations, node positions, pending reaction and step counter, in a
 * binary file; lbm_load restores them into a handle made with the same parameters and
 * capsules.  Resuming gives the same result as an uninterrupted run, bit for bit. */
lbm_status lbm_save(lbm_handle *h, const char *path);
lbm_status lbm_load(lbm_handle *h, const char *path);

/* Event timing of later steps on the handle's stream: on = 1 brackets every kernel,
 * on = 2 only the fluid kernel (two events per step, for timing a run with the least
 * disturbance), 0 stops.  LBM_E_INVAL for other values.  lbm_kernel_stats copies up to
 * max entries and returns their number in *n (synchronises). */
lbm_status lbm_set_profiling(lbm_handle *h, int32_t on);
lbm_status lbm_kernel_stats(lbm_handle *h, lbm_kernel_stat *out, int32_t max, int32_t *n);

/* Launch shape of the fluid step.  tile 1..5 selects the fused single-read kernel with
 * column tiles of 32x8, 64x4, 32x16, 64x8 or 16x16 sites; 6..10 its software-pipelined
 * form (tau = 1 in both components; otherwise the fused kernel of the same tile) with
 * 32x8, 64x4, 16x16, 32x16 or 64x8; 11 and 12 whole-row tiles 256x2 and 128x4 (nx = 256
 * resp. 128, otherwise 64x8); 13 whole rows of any width 16 <= nx <= 128, 512 / nx rows
 * per tile (otherwise 64x8); tile 0 the two-kernel variant (densities, then forces and
 * collision).  zchunk is the number of z planes one workgroup marches through (0: chosen
 * from the lattice size).  Every variant performs the same arithmetic per site in the
 * same order, so results are identical.  LBM_E_INVAL for other values. */
lbm_status lbm_set_launch(lbm_handle *h, int32_t tile, int32_t zchunk);

/* Shortens the first z-chunk of the fluid launch by `planes` planes; the last chunk takes
 * them, so the number of workgroups is unchanged.  Each workgroup marches its chunk, and the
 * launch lasts as long as its slowest one: where the capsule windows lie in the lower chunk
 * (a film on a wall), its workgroups carry the extra window work, and a shorter lower chunk
 * balances them.  0 <= planes < the launch's z-chunk, and 0 when the launch has one chunk
 * (LBM_E_INVAL otherwise).  Results are identical for every offset.  lbm_set_launch resets
 * it to 0; lbm_autotune chooses it. */
lbm_status lbm_set_zoffset(lbm_handle *h, int32_t planes);
/* The current offset of the first z-chunk (0 for a NULL handle). */
int32_t lbm_zoffset(const lbm_handle *h);

/* Launch-shape autotuner of the fluid step: times reps (1..1000) launches of the fluid
 * kernel, after two untimed ones, with HIP events on the handle's stream for every launch
 * shape that applies to the lattice (tiles 1..13 as in lbm_set_launch, of which 1..5 with
 * tau != 1; z-chunks 0, 8, 12, 16, 24, 32, 48 capped at nz, 0 resolved to its value) and
 * selects the fastest as by lbm_set_launch; then times that shape with its first z-chunk
 * shortened by 1 .. 4 planes (lbm_set_zoffset) and keeps the fastest offset, 0 included.
 * The simulation is not advanced: the timed
 * launches read the current populations and write only the buffer and the window
 * outputs that the next step rewrites, and the status words are restored.  They run on
 * the labels and spread forces of the last step, so call it after at least one step for a
 * timing that includes the capsule sites.  Synchronises.  *tile, *zchunk and *fluid_ms
 * (mean kernel time of the choice, ms) may be NULL.  LBM_E_INVAL for reps out of range. */
lbm_status lbm_autotune(lbm_handle *h, int32_t reps, int32_t *tile, int32_t *zchunk,
                        double *fluid_ms);

/* Algorithmic HBM bytes per fluid-site update of the fused fluid kernel for the
 * handle's storage: 2 components x 19 populations x (load + store), plus for storage 3 the
 * FP32 density of both components (load + store). */
double lbm_bytes_per_site(const lbm_handle *h);
int64_t lbm_fluid_sites(const lbm_handle *h);

const char *lbm_last_error(const lbm_handle *h);
void lbm_destroy(lbm_handle *h);

/* ---- Batches -------------------------------------------------------------------------
 * A batch advances several simulations together: per step, the capsule kernels of each
 * handle, then ONE launch of the software-pipelined fluid kernel over the lattices of all
 * handles (different sizes allowed; each handle may itself hold stacked slabs), then the
 * node updates.  Each handle ends in exactly the state lbm_step would give it: the
 * per-site arithmetic is the same.  The handles must share device, stream and storage
 * mode and have tau = 1 in both components; they stay owned by the caller, who destroys
 * the batch before them.  Observation calls (lbm_sync, lbm_observables, ...) go to the
 * handles.  lbm_batch_create fails with LBM_E_INVAL (message in lbm_batch_last_error(NULL))
 * for handles that do not qualify. */
typedef struct lbm_batch lbm_batch;
lbm_status lbm_batch_create(lbm_handle *const *handles, int32_t n, lbm_batch **out);

/* Tile of the batched fluid launch: 6..10 or 13 as in lbm_set_launch (default 10, 64x8;
 * 13 needs 16 <= nx <= 128 in every handle, LBM_E_INVAL otherwise); zchunk 0 picks 48
 * planes, halved while a part's launch has fewer than 1024 workgroups. */
lbm_status lbm_batch_set_launch(lbm_batch *b, int32_t tile, int32_t zchunk);

/* The autotuner of lbm_autotune for the batched fluid launch: tiles 6..10 and (when every
 * handle has 16 <= nx <= 128) 13, z-chunks 0, 8, 12, 16, 24, 32, 48; each candidate is timed
 * as the fluid launches of all parts back to back on the handles' stream.  Selects the
 * fastest as by lbm_batch_set_launch; the handles are not advanced and their status words
 * are restored.  Synchronises. */
lbm_status lbm_batch_autotune(lbm_batch *b, int32_t reps, int32_t *tile, int32_t *zchunk,
                              double *fluid_ms);

/* Split the handles into `parts` sets of about equal fluid sites (1..4, default 1), each
 * advanced by its own chain of launches on a stream of the batch's own (default priority),
 * so that the latency-bound capsule kernels of one set overlap the fluid kernel of
 * another; lbm_batch_step makes the handles' stream wait for all of them before it
 * returns.  With more than one part the kernel timings of lbm_batch_kernel_stats overlap.
 * LBM_E_INVAL for other values. */
lbm_status lbm_batch_set_parts(lbm_batch *b, int32_t parts);

/* Enqueue n >= 0 steps of every handle; the handles' stream holds them all when the call
 * returns, which is without waiting. */
lbm_status lbm_batch_step(lbm_batch *b, int64_t n);

/* Block schedule of the batched fluid launch.  queue = 0 (the default): one workgroup per
 * tile, numbered so that each XCD runs a contiguous run of tiles.  queue = 1: a resident
 * grid of one 512-thread workgroup (two of 256) per compute unit takes the tiles from a
 * work queue on the device, each XCD its own run first, then those of the others.  The
 * per-tile arithmetic is the same, so results are the same bits.  LBM_E_INVAL for other
 * values. */
lbm_status lbm_batch_set_schedule(lbm_batch *b, int32_t queue);

/* Step replay from a HIP graph: with on = 1, lbm_batch_step runs pairs of steps by
 * launching a graph that holds two whole steps of every part (their kernels and the
 * cross-stream dependencies, recorded once per buffer parity on a stream of the batch's own,
 * at the first step that needs it) on the handles' stream; an odd last step, and every step
 * while event timing is on, is enqueued as usual.  The graphs are dropped and recorded again
 * when the batch's tables change (launch shape, parts, a member stepped alone).  Results are
 * the same bits as without.  on = 0 (the default) enqueues every step.  LBM_E_INVAL for other
 * values. */
lbm_status lbm_batch_set_graph(lbm_batch *b, int32_t on);

/* Event timing of the batch's kernels, as lbm_set_profiling / lbm_kernel_stats. */
lbm_status lbm_batch_set_profiling(lbm_batch *b, int32_t on);
lbm_status lbm_batch_kernel_stats(lbm_batch *b, lbm_kernel_stat *out, int32_t max, int32_t *n);

const char *lbm_batch_last_error(const lbm_batch *b);
void lbm_batch_destroy(lbm_batch *b);

/* ---- Learned surrogate ----------------------------------------------------------------
 * A multilayer perceptron 4 -> 64 -> 64 -> 64 -> 2 with tanh hidden layers that maps a
 * capsule pair's (separation / radius, log10 shear modulus, film height / diameter,
 * contact angle) to (lateral capillary force, meniscus deformation), trained by Adam on
 * data of the batched solver (mean squared error (1 / 2 sum w) sum_i w_i |y_i - t_i|^2).
 * Every matrix product runs on the matrix cores with bfloat16 operands (rounded to
 * nearest even) and float32 sums; parameters, Adam moments and activations are float32.
 * Parameter vector (host float [LBM_SURROGATE_PARAMS]): W1 [4][64], b1 [64], W2 [64][64],
 * b2, W3 [64][64], b3, W4 [64][2], b4 [2], each W [inputs][outputs] row-major, y = x W + b.
 * Inputs and targets are passed normalised by the caller (e.g. zero mean, unit variance
 * per column).  Host buffers are copied during the calls; every call synchronises its
 * private stream (default priority).  Errors: LBM_E_INVAL for bad sizes or non-finite
 * data (message in lbm_surrogate_last_error), LBM_E_STATE for training without data. */
#define LBM_SURROGATE_PARAMS 8770
typedef struct lbm_surrogate lbm_surrogate;

/* Device state for up to max_samples samples (1 .. 2^20), parameters from theta0. */
lbm_status lbm_surrogate_create(int32_t max_samples, const float *theta0, lbm_surrogate **out);

/* Training data: x [n][4], t [n][2], w [n] sample weights >= 0 (NULL: all 1). */
lbm_status lbm_surrogate_set_data(lbm_surrogate *s, int32_t n, const float *x, const float *t,
                                  const float *w);

/* Loss and its gradient [LBM_SURROGATE_PARAMS] at the current parameters over the data. */
lbm_status lbm_surrogate_gradient(lbm_surrogate *s, float *loss, float *grad);

/* steps Adam updates (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the full data. */
lbm_status lbm_surrogate_train(lbm_surrogate *s, int32_t steps, float lr);

/* Network outputs y [n][2] for inputs x [n][4], n <= max_samples. */
lbm_status lbm_surrogate_predict(lbm_surrogate *s, int32_t n, const float *x, float *y);

/* Current parameters into theta [LBM_SURROGATE_PARAMS]. */
lbm_status lbm_surrogate_params(lbm_surrogate *s, float *theta);

/* Cluster evolution driven by the network: the many-capsule clustering of the section on
 * clustering of soft particles in a thin film, reduced to the capsules' centres in the
 * film plane with pair forces from the network.  n capsules of radius `radius` in a periodic
 * square of side `box`, overdamped, p_i += mobility * sum_j f(r_ij) e_ij each step (e_ij the
 * unit vector from capsule j to i, minimum image).  f is the network's lateral force for
 * r_contact <= r / radius <= r_cut (inputs r / radius and the three fixed features below,
 * normalised with in_mean / in_scale, output de-normalised with out_mean / out_scale);
 * closer pairs are outside the network's domain and repel with k_contact (r_contact -
 * r / radius); farther pairs exert no force.  Each step is one kernel that evaluates the
 * network for all n (n - 1) ordered pairs on the matrix cores (same bfloat16 operands and
 * float32 sums as lbm_surrogate_predict) and moves every capsule; the per-capsule sum
 * runs in a fixed order.  Uses the network's current parameters and only the first
 * output (the force); n is not limited by max_samples.  Allocates, per call, two device
 * buffers of n positions and the network in operand layout (33 KB), freed before it
 * returns; positions are float32, wrapped into [0, box). */
typedef struct {
    float box, radius;
    float log10_ks, film, angle;          /* raw values of the other three inputs        */
    float in_mean[4], in_scale[4], out_mean[2], out_scale[2];
    float r_contact, r_cut, k_contact, mobility;
} lbm_cluster_params;

/* xy host [n][2] in/out (caller-owned, copied to the device and back): positions, advanced
 * by `steps` steps.  Errors: LBM_E_INVAL for n < 2, steps < 0, a non-positive box, radius or
 * input scale, r_cut <= r_contact, 2 r_cut radius >= box (the minimum image would miss
 * partners), a negative k_contact or a non-finite mobility;
 * LBM_E_DEVICE if an allocation or launch fails (positions then unchanged). */
lbm_status lbm_surrogate_cluster(lbm_surrogate *s, int32_t n, float *xy, int32_t steps,
                                 const lbm_cluster_params *cp);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lbm_surrogate_cluster without any
 * allocation.  xy_device is a caller-owned DEVICE buffer [n][2] float of positions, in/out
 * (advanced in place by `steps` steps, wrapped into [0, box)).  Everything else it needs
 * (the second position buffer of the step's ping-pong and the network in operand layout,
 * about 161 kB) lives in a file-scope device array of the library, one per GPU, held until
 * the process ends and shared by every call on that GPU: calls that overlap on one GPU
 * race, and each call rewrites what it reads of it.  The arithmetic is that of
 * lbm_surrogate_cluster (same kernels), so the results are identical.  Runs on the
 * surrogate's stream and synchronises it.  Errors: as lbm_surrogate_cluster, and
 * LBM_E_INVAL for n > LBM_CLUSTER_NOALLOC_MAX or a NULL buffer; LBM_E_DEVICE if a launch or
 * the look-up of the array's device address fails (positions then undefined). */
#define LBM_CLUSTER_NOALLOC_MAX 16384
lbm_status lbm_surrogate_cluster_noalloc(lbm_surrogate *s, int32_t n, float *xy_device,
                                         int32_t steps, const lbm_cluster_params *cp);

const char *lbm_surrogate_last_error(const lbm_surrogate *s);
void lbm_surrogate_destroy(lbm_surrogate *s);

#ifdef __cplusplus
}
#endif
#endif
