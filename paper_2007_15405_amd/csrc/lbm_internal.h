// lbm_internal.h -- device-side definitions shared by the HIP sources of liblbm.
//
// D3Q19 lattice (Section 3.1): rest weight 1/3, axis links 1/18, diagonal links 1/36,
// c_s^2 = 1/3.  The population order here is a storage layout: grouped by the z
// component of e_i (in-plane first, then +z and -z), opposite pairs adjacent.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmx {

constexpr int Q = 19;
//                     0  1  2  3  4  5  6  7  8  9 10 11 12 13 14 15 16 17 18
constexpr int CX[Q] = {0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

__host__ __device__ constexpr float wq(int q) {
    return q == 0 ? 1.0f / 3.0f
                  : ((CX[q] * CX[q] + CY[q] * CY[q] + CZ[q] * CZ[q]) == 1 ? 1.0f / 18.0f
                                                                          : 1.0f / 36.0f);
}
// Weights of the shift of storage 3 (f_i stored as f_i - ws_i rho_site): FP32 numbers
// within 4e-8 of w_i whose exact sum is 1.  The FP32 values of 1/3, 1/18 and 1/36 sum to
// 1 + 1.5e-8, which the decode would add to every site's mass in every step.
__host__ __device__ constexpr float wshift(int q) {
    return q == 0 ? 0x1.555558p-2f
                  : ((CX[q] * CX[q] + CY[q] * CY[q] + CZ[q] * CZ[q]) == 1 ? 0x1.c71c7p-5f
                                                                          : 0x1.c71c7p-6f);
}
__host__ __device__ constexpr bool is_axis(int q) {
    return (CX[q] * CX[q] + CY[q] * CY[q] + CZ[q] * CZ[q]) == 1;
}

// Per-site flag byte: bits 0..6 side label (0 exterior, k+1 inside capsule k), bit 7
// set where the site lies inside some capsule's immersed-boundary window, i.e. where
// the spread force is read and the velocity / reaction are written.
constexpr uint8_t LABEL_MASK = 0x7f;
constexpr uint8_t AUX_BIT = 0x80;
constexpr int LABEL_WALL = 127;   // label value used for wall neighbours inside kernels
constexpr int MAX_CAPS = 125;        // LBM_MAX_CAPSULES
constexpr int MAX_CAP_NODES = 8192;  // LBM_MAX_CAPSULE_NODES
constexpr int GMAX = 64;          // maximum edge of a capsule window (sites)
constexpr int GMAX3 = GMAX * GMAX * GMAX;
constexpr int ROWS_MAX = GMAX * GMAX;
constexpr int FILL_COLS = 2048;   // window columns (x * y) the spreading kernel holds in LDS

// status words (device): [0] unstable flag, [1] lost reaction count, [2] window overflow,
// [3] window wider than the spreading plane buffer, [4] unused, [5] a capsule window left
// the slab of its capsule
constexpr int ST_UNSTABLE = 0, ST_LOST = 1, ST_OVERFLOW = 2, ST_WIDE = 3, ST_SLAB = 5,
              ST_BBLOST = 6, ST_BBOVER = 7, ST_WORDS = 8;
// [6] bounce-back links that found no triangle (count), [7] a bounce-back bin or link
// list overflowed, or a triangle spans more than BB_SPAN cells per axis

// Slabs: with a wall, the lattice is a stack of boxes of lz planes, each starting with a
// solid layer (lz = nz: one box).  Position of plane z inside its slab.
__host__ __device__ inline int slab_pos(int z, int lz) { return z % lz; }

// ------------------------------------------------------------------------------------
// Population storage codec.  S = 0: FP32 as is.  S = 1: FP16 of f - w_i rho_s.
// S = 2: BF16 (round to nearest even) of f - w_i rho_s.  Arithmetic is FP32.
// ------------------------------------------------------------------------------------
template <int S> struct Codec;

template <> struct Codec<0> {
    using T = float;
    __device__ static inline float dec(T v, float) { return v; }
    __device__ static inline T enc(float f, float) { return f; }
};

template <> struct Codec<1> {
    using T = _Float16;
    __device__ static inline float val(T v) { return (float)v; }   // the stored value
    __device__ static inline float dec(T v, float s) { return val(v) + s; }
    __device__ static inline T enc(float f, float s) { return (_Float16)(f - s); }
};

// S = 3: FP16 of the relative deviation d_i = f_i / (ws_i rho_site) - 1 of f from the rest
// equilibrium at the site's own density rho_site (stored in FP32 beside the populations).
// The callers pass s = ws_i rho_site; a site of zero density stores 0.  Relative values keep
// the deviations of both phases of a two-component film in FP16's normal range (a minority
// phase of density 0.04 has |f_i - w_i rho| below FP16's smallest normal number at every
// velocity below about 0.02, where an absolute encoding keeps few significant bits).
template <> struct Codec<3> {
    using T = _Float16;
    __device__ static inline float val(T v) { return (float)v; }
    __device__ static inline float dec(T v, float s) { return fmaf(s, val(v), s); }
    __device__ static inline T enc(float f, float s) {
        return s != 0.f ? (_Float16)((f - s) / s) : (_Float16)0.f;
    }
};

template <> struct Codec<2> {
    using T = uint16_t;
    __device__ static inline float val(T v) { return __uint_as_float((uint32_t)v << 16); }
    __device__ static inline float dec(T v, float s) { return val(v) + s; }
    __device__ static inline T enc(float f, float s) {
        uint32_t u = __float_as_uint(f - s);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (T)((u >> 16) | 0x40u);  // quiet NaN
        u += 0x7fffu + ((u >> 16) & 1u);
        return (T)(u >> 16);
    }
};

// ------------------------------------------------------------------------------------
// Kernel arguments
// ------------------------------------------------------------------------------------
struct FluidArgs {
    const void *fin;        // populations of the last step, [2][19][N] of Codec<S>::T
    void *fout;             // populations written by this step
    const float *rin;       // storage 3: [2][N] density of every site of the last step
    float *rout;            // storage 3: [2][N] density written by this step
    const uint8_t *flag;    // [N] label | AUX_BIT
    const float4 *ibm;      // [N] spread force (x, y, z) and kernel coverage (w), aux sites
    float4 *uo;             // [N] physical velocity, aux sites
    float4 *ro;             // [N] cross-membrane reaction, aux sites
    float *psi;             // [2][N] pseudopotential (two-pass kernel)
    int *status;            // status words
    const float *cap_drho;  // [MAX_CAPS] wetting offset per capsule
    int nx, ny, nz, wall;
    int N;                  // nx * ny * nz
    int lz;                 // slab height (nz: one box)
    float tau[2], inv_tau[2];
    float G;                // coupling
    float ws_axis, ws_diag; // stencil weights sc_norm * omega_i
    float inv_rho0;
    float g[3];             // body acceleration
    float wall_drho;
    float shift[2];         // storage shift rho_s per component (16-bit modes)
    int keepf;              // 0: tau = 1 for both components, so f* = f^eq (moments suffice)
    int bb;                 // bounce-back coupling: window sites store (rho0, rho1, psi0,
                            // psi1) in ro instead of the reaction
    int zero_drho;          // 1: the wall and every capsule have a zero wetting offset
    int zoff;               // planes the first z-chunk of the launch is shortened by (the
                            // last takes them; 0 <= zoff < the chunk)
};

// planes [z0, z1) of z-chunk bz of a launch with chunks of zc planes, the first shortened by
// zoff planes and the last taking them, so that the chunk count stays ceil(nz / zc)
__host__ __device__ inline void zchunk_range(int bz, int zc, int zoff, int nz, int &z0, int &z1) {
    const int tz = (nz + zc - 1) / zc;
    z0 = bz == 0 ? 0 : bz * zc - zoff;
    z1 = bz == tz - 1 ? nz : (bz + 1) * zc - zoff;
}

// Device description of one capsule.
struct CapDev {
    int node0, nn;          // first node, node count
    int tri0, nt;           // first triangle, triangle count
    float ks, C, kv, anchor_k;
    float kb;               // bending modulus (edge form of the Helfrich energy)
    float plane_z;          // repulsive plane of the capsule's slab
    int zbase;              // wall layer of the capsule's slab
    double v0;              // reference volume
    double c0[3];           // reference centroid
};

// Per-step capsule state written by the reduction kernel.
struct CapState {
    double cen[3];          // node mean at X^n
    double vol;             // enclosed volume at X^n (capsules with kv != 0; else 0)
    float bmin[3], bmax[3]; // node bounding box (FP32 positions)
    int lo[3], dim[3];      // window: sites lo .. lo + dim - 1 (unwrapped)
    int plo[3], pdim[3];    // the previous step's window, whose flags the window kernel clears
};

struct MembraneArgs {
    const CapDev *caps;
    CapState *cst;
    int ncap;
    double4 *X;             // [Ntot] node positions (unwrapped, FP64 state), w unused
    const int *node_cap;    // [Ntot] capsule index of each node
    float4 *F;              // [Ntot] total node force, in row order (index slot[n])
    float4 *Fh;             // [Ntot] Hertz part
    float4 *R;              // [Ntot] pending reaction
    const int4 *tri;        // [Ttot] global node indices a, b, c and capsule index
    const float4 *minv;     // [Ttot] reference inverse (row-major 2x2)
    const float *a0;        // [Ttot] reference area
    const int *ntri_off;    // [Ntot+1] node -> incident triangle CSR offsets
    const int *ntri;        // incident entries: 3 * triangle + corner
    const int4 *edge;       // [Etot] bending edges x1, x2, x3, x4 (global node indices):
                            // triangles (x1, x2, x3) and (x2, x1, x4)
    const float *eth0;      // [Etot] reference dihedral angle
    const int *nedge_off;   // [Ntot+1] node -> bending edge CSR offsets
    const int *nedge;       // entries: 4 * edge + role (0..3 for x1..x4)
    unsigned long long *marks;  // [ncap][ROWS_MAX] crossings per window column, bit = plane
    int *rowstart;          // [ncap][ROWS_MAX + 1] node rows of each window
    double4 *xrow;          // [Ntot] node positions grouped by row (any order in a row)
    int *slot;              // [Ntot] place of node n in the row order (global index)
    float4 *wbuf;           // [ncap][GMAX3] own spread force and coverage per window site
    uint8_t *wpar;          // [ncap][GMAX3] own crossing parity per window site
    uint8_t *flag;
    float4 *ibm;
    const float4 *uo, *ro;
    int *status;
    int nx, ny, nz, wall;
    int lz;                 // slab height (nz: one box)
    float hertz_xi, hertz_d0;
    int bb;                 // bounce-back coupling: no spreading (labels only), and the
                            // reaction in R is an observable, not a pending force
};

// ------------------------------------------------------------------------------------
// Bounce-back coupling (bounce.hip)
// ------------------------------------------------------------------------------------
constexpr int BB_SPAN = 3;                       // cells per axis a triangle may cover
constexpr int BB_PER_TRI = BB_SPAN * BB_SPAN * BB_SPAN;

// a link from site a inside capsule k to site b = a + e_q outside it, the triangle it
// crosses (-1: none found) and the densities of both sites before the bounce-back
struct BBLink {
    int a, b, q, tri;
    float rho[4];           // component 0 and 1 at a, then at b
};

struct BBArgs {
    const CapDev *caps;
    const CapState *cst;
    int ncap, ntot, ttot;
    const int4 *tri;        // [Ttot] global node indices a, b, c and capsule index
    double4 *X;             // [Ntot] node positions
    double4 *V;             // [Ntot] node velocities
    const float4 *F;        // [Ntot] membrane forces in row order
    const int *slot;        // [Ntot] place of each node in the row order
    const uint8_t *flag;
    void *f;                // populations of this step's input (changed in place)
    const float4 *dens;     // [N] densities and psi of both components, written by the
                            // fluid step on window sites (rho0, rho1, psi0, psi1)
    float4 *tpos;           // [Ttot][3] FP32-rounded triangle vertices of this step
    int *tcell;             // [Ttot] window cells each triangle's box covers, packed
                            // (first cell x, y, z: 6 bits each; extent - 1: 2 bits each),
                            // -1 for a triangle the bins cannot hold
    int N, nx, ny, nz, wall, lz;
    float shift[2];
    int *bstart;            // [ncap][GMAX3 + 1] first entry of each cell
    int *blist;             // [BB_PER_TRI * Ttot] triangle indices by cell
    BBLink *links;          // [ncap][link_cap]
    int link_cap;
    int *nlinks;            // [2][ncap] links of this step, then those of the last step
    long long *pex;         // [Ttot][3] momentum exchanged this step through each triangle's
                            // links, 2^-40 units (cleared at the next step's start)
    long long *rsc;         // [Ttot][3] Shan-Chen reaction of this step, likewise
    const int *ntri_off;    // [Ntot+1] node -> incident triangle CSR offsets
    const int *ntri;        // incident entries: 3 * triangle + corner
    float4 *pprev;          // [Ntot] momentum exchanged in the previous step
    float4 *ffl;            // [Ntot] force of the fluid on each node in the last step
    float4 *R;              // [Ntot] Shan-Chen reaction on each node in the last step
    int *status;
    float G, ws_axis, ws_diag, inv_rho0;
    const float *cap_drho;
    double inv_mass;        // 1 / node mass
};
void launch_bb_before(const BBArgs &b, int storage, hipStream_t st);
void launch_bb_after(const BBArgs &b, int storage, hipStream_t st);

// Launchers (host functions, defined in the .hip files).
// rsite: storage 3, [2][N] site densities (written by launch_init_eq, read by the others);
// nullptr otherwise
template <int S> void launch_init_eq(const double *rho_dev, void *f, int nx, int ny, int nz,
                                     int wall, int lz, float s0, float s1, float *rsite,
                                     hipStream_t st);
template <int S> void launch_fluid(const FluidArgs &a, hipStream_t st);
template <int S> void launch_fluid_tiled(const FluidArgs &a, int tile, int zc, hipStream_t st);
// One launch of the pipelined fluid kernel over several lattices (device tables: the
// arguments of each lattice, and per lattice {first logical block, tiles in x, tiles in
// y, z planes per chunk}); tile 6..10 and 13 as launch_fluid_tiled (13: every lattice
// 16 <= nx <= 128, tiles of rows_tile_height(nx) whole rows).
int rows_tile_height(int nx);
// queue: nullptr for the static block order; else 9 zeroed device ints of a work queue,
// and the launch is a resident grid of ncu (compute units) blocks of 512 threads
template <int S> void launch_fluid_multi(const FluidArgs *tab, const int4 *desc, int ngroups,
                                         int nblocks, int tile, int *queue, int ncu,
                                         hipStream_t st);
template <int S> void launch_rho(const void *f, float *rho, int nx, int ny, int nz, int wall,
                                 int lz, float s0, float s1, const float *rsite, hipStream_t st);
// partial sums [nz / lz][nblocks][5] (mass of both components, momentum) per slab
template <int S> void launch_moments(const void *f, double *partial, int nblocks, int nx, int ny,
                                     int nz, int wall, int lz, float s0, float s1,
                                     const float *rsite, hipStream_t st);
// meniscus heights [nz / lz][ny][nx], measured from each slab's wall layer
void launch_meniscus(const float *rho, const uint8_t *flag, float *out, int nx, int ny, int nz,
                     int wall, int lz, hipStream_t st);

// Capsule kernels of several simulations in one launch each (see membrane.hip): per
// group (simulation with capsules) its first capsule, membrane block and node-update
// block in the launches, node and triangle counts, force-block count and node-update
// block count.
struct MGroup {
    int cap0, mem0, upd0, ntot, ttot, nbf, nbu;
};
struct MGroupTotals {
    int ncap, mem_blocks, upd_blocks;
};
int membrane_blocks(int ntot, int ttot, int *nb_forces);
int node_update_blocks(int ntot);
void launch_capsule_reduce_multi(const MembraneArgs *tab, const MGroup *grp, int ng,
                                 const MGroupTotals &t, hipStream_t st);
void launch_membrane_multi(const MembraneArgs *tab, const MGroup *grp, int ng,
                           const MGroupTotals &t, hipStream_t st);
void launch_window_fill_multi(const MembraneArgs *tab, const MGroup *grp, int ng,
                              const MGroupTotals &t, hipStream_t st);
void launch_node_update_multi(const MembraneArgs *tab, const MGroup *grp, int ng,
                              const MGroupTotals &t, hipStream_t st);

void launch_capsule_reduce(const MembraneArgs &m, hipStream_t st);
void launch_membrane(const MembraneArgs &m, int ntot, int ttot, hipStream_t st);
void launch_window_fill(const MembraneArgs &m, hipStream_t st);
void launch_node_update(const MembraneArgs &m, int ntot, hipStream_t st);

}  // namespace lbmx
