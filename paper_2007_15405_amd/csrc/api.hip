// api.hip -- the C ABI of liblbm (include/lbm.h): handle, parameter validation, device
// state, the per-step launch chain, observables, checkpoints and kernel timing.
#include "lbm.h"
#include "lbm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

using namespace lbmx;

namespace {

thread_local std::string g_init_error;

struct HostCap {
    lbm_capsule_params p;
    int zbase;                 // wall layer of the capsule's slab
    std::vector<double> x0;    // [nn][3]
    std::vector<int32_t> tri;  // [nt][3]
    std::vector<int32_t> edge; // bending (kb != 0): [ne][4] x1, x2, x3, x4 (local nodes)
    std::vector<double> th0;   // [ne] reference dihedral angles
};

struct Timer {
    const char *name;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    int64_t launches = 0;
    double ms = 0.0;
};

// Event timing of kernels on one stream: mode 0 off, 1 every kernel, 2 the fluid kernel
struct Prof {
    int mode = 0;
    std::vector<Timer> timers;
    std::vector<hipEvent_t> pool;
};

constexpr int MOM_BLOCKS = 512;

}  // namespace

struct lbm_handle {
    lbm_params p{};
    std::string err;
    hipStream_t st = nullptr;
    bool own_stream = false;
    int nx = 0, ny = 0, nz = 0, wall = 0, N = 0, storage = 0;
    int lz = 0, nslab = 1;      // slab height and count (one box: lz = nz)
    int mom_blocks = 0;         // moment-reduction blocks per slab
    size_t esize = 4;
    void *f[2] = {nullptr, nullptr};
    float *rsite[2] = {nullptr, nullptr};   // storage 3: [2][N] site densities per buffer
    int cur = 0;
    uint8_t *flag = nullptr;
    float4 *ibm = nullptr, *uo = nullptr, *ro = nullptr;
    float *psi = nullptr, *cap_drho = nullptr, *rho_tmp = nullptr, *men_tmp = nullptr;
    int *status = nullptr;
    double *partial = nullptr;
    std::vector<HostCap> caps;
    bool finalized = false;
    int64_t step = 0;
    int ntot = 0, ttot = 0;
    CapDev *d_caps = nullptr;
    CapState *d_cst = nullptr;
    double4 *d_X = nullptr;
    int *d_node_cap = nullptr;
    float4 *d_F = nullptr, *d_Fh = nullptr, *d_R = nullptr;
    int4 *d_tri = nullptr;
    float4 *d_minv = nullptr;
    float *d_a0 = nullptr;
    int *d_off = nullptr, *d_list = nullptr, *d_rowstart = nullptr, *d_slot = nullptr;
    double4 *d_xrow = nullptr;
    unsigned long long *d_marks = nullptr;
    float4 *d_wbuf = nullptr;
    uint8_t *d_wpar = nullptr;
    int4 *d_edge = nullptr;
    float *d_eth0 = nullptr;
    int *d_eoff = nullptr, *d_elist = nullptr;
    std::vector<CapDev> h_caps;
    int tile = 1, zchunk = 0;
    int zoff = 0;                  // planes the first z-chunk is shortened by
    Prof prof;
    // bounce-back coupling (coupling = 1)
    double4 *d_V = nullptr;
    long long *d_pex = nullptr, *d_rsc = nullptr;
    float4 *d_pprev = nullptr, *d_ffl = nullptr;
    int *d_bstart = nullptr, *d_blist = nullptr, *d_nlinks = nullptr;
    BBLink *d_links = nullptr;
    float4 *d_tpos = nullptr;
    int *d_tcell = nullptr;
    int link_cap = 0;
};

#define HIPCHK(h, expr)                                                               \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            (h)->err = std::string(#expr) + ": " + hipGetErrorString(e_);             \
            return LBM_E_DEVICE;                                                      \
        }                                                                             \
    } while (0)

// Bending edges of a closed, consistently oriented mesh: every edge x1 -> x2 of a
// triangle (x1, x2, x3) whose reverse x2 -> x1 belongs to a triangle (x2, x1, x4), once.
// False if some edge has no reverse or occurs twice in the same direction.
static bool bending_edges(int nt, const int32_t *tri, std::vector<int32_t> &e4) {
    struct Dir { int32_t a, b, w; };
    std::vector<Dir> d;
    d.reserve(3 * (size_t)nt);
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k)
            d.push_back({tri[3 * t + k], tri[3 * t + (k + 1) % 3], tri[3 * t + (k + 2) % 3]});
    auto less = [](const Dir &x, const Dir &y) { return x.a != y.a ? x.a < y.a : x.b < y.b; };
    std::sort(d.begin(), d.end(), less);
    for (size_t i = 1; i < d.size(); ++i)
        if (d[i].a == d[i - 1].a && d[i].b == d[i - 1].b) return false;
    e4.clear();
    for (const Dir &x : d) {
        const Dir key{x.b, x.a, 0};
        auto it = std::lower_bound(d.begin(), d.end(), key, less);
        if (it == d.end() || it->a != x.b || it->b != x.a) return false;
        if (x.a < x.b) e4.insert(e4.end(), {x.a, x.b, x.w, it->w});
    }
    return 2 * e4.size() / 4 == 3 * (size_t)nt;
}

// signed angle between the outward normals of (p1, p2, p3) and (p2, p1, p4) about the
// edge p1 -> p2 (FP64, for the reference mesh)
static double dihedral_of(const double *p1, const double *p2, const double *p3, const double *p4) {
    double e[3], u[3], v[3], n1[3], n2[3];
    for (int d = 0; d < 3; ++d) {
        e[d] = p2[d] - p1[d];
        u[d] = p3[d] - p1[d];
        v[d] = p4[d] - p2[d];
    }
    // n1 = e x u; n2 = (p1 - p2) x (p4 - p2) = v x e
    n1[0] = e[1] * u[2] - e[2] * u[1]; n1[1] = e[2] * u[0] - e[0] * u[2]; n1[2] = e[0] * u[1] - e[1] * u[0];
    n2[0] = v[1] * e[2] - v[2] * e[1]; n2[1] = v[2] * e[0] - v[0] * e[2]; n2[2] = v[0] * e[1] - v[1] * e[0];
    const double el = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    const double c[3] = {n1[1] * n2[2] - n1[2] * n2[1], n1[2] * n2[0] - n1[0] * n2[2],
                         n1[0] * n2[1] - n1[1] * n2[0]};
    return std::atan2((c[0] * e[0] + c[1] * e[1] + c[2] * e[2]) / el,
                      n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2]);
}

static lbm_status fail(lbm_handle *h, lbm_status s, const std::string &m) {
    h->err = m;
    return s;
}

template <typename T> static hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, sizeof(T) * (count ? count : 1));
}

static void free_prof(Prof &pf) {
    for (hipEvent_t e : pf.pool) (void)hipEventDestroy(e);
    for (auto &t : pf.timers)
        for (auto &pr : t.pending) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    pf.pool.clear();
    pf.timers.clear();
}

static void free_all(lbm_handle *h) {
    void *ptrs[] = {h->f[0], h->f[1], h->rsite[0], h->rsite[1], h->flag, h->ibm, h->uo, h->ro, h->psi, h->cap_drho,
                    h->rho_tmp, h->men_tmp, h->status, h->partial, h->d_caps, h->d_cst, h->d_X,
                    h->d_node_cap, h->d_F, h->d_Fh, h->d_R, h->d_tri, h->d_minv, h->d_a0,
                    h->d_off, h->d_list, h->d_marks, h->d_rowstart, h->d_slot, h->d_wbuf,
                    h->d_wpar, h->d_xrow, h->d_edge, h->d_eth0, h->d_eoff,
                    h->d_elist, h->d_V, h->d_pex, h->d_rsc, h->d_pprev, h->d_ffl,
                    h->d_bstart, h->d_blist, h->d_nlinks, h->d_links, h->d_tpos, h->d_tcell};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    free_prof(h->prof);
    if (h->own_stream && h->st) (void)hipStreamDestroy(h->st);
}

// ------------------------------------------------------------------------------------
// Timing
// ------------------------------------------------------------------------------------
static hipEvent_t take_event(Prof &pf) {
    if (!pf.pool.empty()) {
        hipEvent_t e = pf.pool.back();
        pf.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static Timer &timer(Prof &pf, const char *name) {
    for (auto &t : pf.timers)
        if (t.name == name) return t;
    pf.timers.push_back(Timer{name, {}, 0, 0.0});
    return pf.timers.back();
}

template <typename F>
static void timed(Prof &pf, hipStream_t st, const char *name, F &&launch) {
    if (!pf.mode || (pf.mode == 2 && std::strcmp(name, "fluid") != 0)) {
        launch();
        return;
    }
    hipEvent_t a = take_event(pf), b = take_event(pf);
    if (a) (void)hipEventRecord(a, st);
    launch();
    if (b) (void)hipEventRecord(b, st);
    if (a && b) timer(pf, name).pending.push_back({a, b});
}

static void collect_timers(Prof &pf) {
    for (auto &t : pf.timers) {
        for (auto &pr : t.pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
                t.ms += ms;
                t.launches++;
            }
            pf.pool.push_back(pr.first);
            pf.pool.push_back(pr.second);
        }
        t.pending.clear();
    }
}

// copies up to max timer entries (and resets them); the caller has synchronised
static int export_timers(Prof &pf, lbm_kernel_stat *out, int max) {
    collect_timers(pf);
    int k = 0;
    for (auto &t : pf.timers) {
        if (k >= max) break;
        std::memset(&out[k], 0, sizeof(lbm_kernel_stat));
        std::snprintf(out[k].name, sizeof out[k].name, "%s", t.name);
        out[k].launches = t.launches;
        out[k].total_ms = t.ms;
        ++k;
    }
    for (auto &t : pf.timers) { t.launches = 0; t.ms = 0.0; }
    return k;
}

// ------------------------------------------------------------------------------------
// Initial densities (Section 3.2 film, uniform, or caller array)
// ------------------------------------------------------------------------------------
static void initial_density(const lbm_params &p, int lz, std::vector<double> &rho) {
    const long N = (long)p.nx * p.ny * p.nz;
    rho.assign(2 * N, 0.0);
    const int kw = p.wall_z0 ? 1 : 0;
    for (int k = 0; k < p.nz; ++k)
        for (int j = 0; j < p.ny; ++j)
            for (int i = 0; i < p.nx; ++i) {
                const long s = ((long)k * p.ny + j) * p.nx + i;
                const int kr = slab_pos(k, lz);   // plane inside its slab
                if (p.wall_z0 && kr == 0) continue;
                double a, b;
                if (p.init_mode == 0) {
                    a = p.init_rho[0];
                    b = p.init_rho[1];
                } else if (p.init_mode == 1) {
                    const double hf = p.slab_film_height ? p.slab_film_height[k / lz] : p.film_height;
                    const long H = std::lround(hf);
                    const long layer = kr - kw;
                    if (layer < H) { a = p.rho_maj; b = p.rho_min; }
                    else if (layer == H) { a = p.rho_iface; b = p.rho_iface; }
                    else { a = p.rho_min; b = p.rho_maj; }
                } else {
                    a = p.init_rho_array[s];
                    b = p.init_rho_array[N + s];
                }
                rho[s] = a;
                rho[N + s] = b;
            }
}

static float shift_of(const lbm_handle *h, int c) {
    // storage 3 shifts by each site's own density, not by a constant
    return (h->storage == LBM_STORE_F32 || h->storage == LBM_STORE_F16_LOCAL)
               ? 0.0f : (float)h->p.rho_shift[c];
}

// ------------------------------------------------------------------------------------
// lbm_init
// ------------------------------------------------------------------------------------
extern "C" lbm_status lbm_init(const lbm_params *p, lbm_handle **out) {
    if (!out) return LBM_E_INVAL;
    *out = nullptr;
    auto bad = [&](const char *m) {
        g_init_error = m;
        return LBM_E_INVAL;
    };
    if (!p) return bad("params is NULL");
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return bad("nx, ny, nz must be >= 3");
    // the kernels address 10 populations of one component with 32-bit byte offsets
    const double pop_bytes = 10.0 * p->nx * p->ny * p->nz * (p->storage == LBM_STORE_F32 ? 4 : 2);
    if (pop_bytes >= 4294967296.0)
        return bad("lattice too large: 10 populations of one component must fit in 4 GiB "
                   "(107 million sites with FP32 storage, 214 million with 16-bit)");
    if (!(p->tau[0] > 0.5) || !(p->tau[1] > 0.5)) return bad("tau must exceed 1/2");
    if (!(p->rho0 > 0.0)) return bad("rho0 must be positive");
    if (!(p->sc_norm >= 0.0) || !std::isfinite(p->G)) return bad("invalid Shan-Chen coupling");
    if (p->init_mode < 0 || p->init_mode > 2) return bad("init_mode must be 0, 1 or 2");
    if (p->init_mode == 2 && !p->init_rho_array) return bad("init_rho_array is NULL");
    if (p->init_mode == 1 && !(p->film_height >= 0.0)) return bad("film_height must be >= 0");
    const int lz = p->slab_nz == 0 ? p->nz : p->slab_nz;
    if (lz < 3 || lz > p->nz || p->nz % lz != 0)
        return bad("slab_nz must be 0 or a divisor of nz of at least 3");
    if (lz < p->nz && p->wall_z0 != 1) return bad("stacked slabs need wall_z0 = 1");
    if (p->init_mode == 1 && p->slab_film_height)
        for (int sl = 0; sl < p->nz / lz; ++sl)
            if (!(p->slab_film_height[sl] >= 0.0)) return bad("slab_film_height must be >= 0");
    if (p->storage < 0 || p->storage > 3) return bad("storage must be 0, 1, 2 or 3");
    if (p->storage == LBM_STORE_F16_LOCAL && !(p->tau[0] == 1.0 && p->tau[1] == 1.0))
        return bad("storage 3 (FP16 shifted by the site density) needs tau = 1 in both components");
    if (p->storage == LBM_STORE_F16_LOCAL && p->coupling != 0)
        return bad("storage 3 is not available with the bounce-back coupling");
    if (!(p->hertz_xi >= 0.0) || !(p->hertz_delta0 >= 0.0)) return bad("invalid Hertz parameters");
    if (p->wall_z0 != 0 && p->wall_z0 != 1) return bad("wall_z0 must be 0 or 1");
    if (p->coupling != 0 && p->coupling != 1) return bad("coupling must be 0 or 1");
    if (p->coupling == 1 && !(p->node_mass > 0.0 && std::isfinite(p->node_mass)))
        return bad("node_mass must be positive with the bounce-back coupling");

    lbm_handle *h = new (std::nothrow) lbm_handle();
    if (!h) return LBM_E_NOMEM;
    h->p = *p;
    h->p.init_rho_array = nullptr;
    h->p.slab_film_height = nullptr;
    h->nx = p->nx; h->ny = p->ny; h->nz = p->nz; h->wall = p->wall_z0;
    h->lz = lz;
    h->nslab = p->nz / lz;
    h->mom_blocks = std::max(8, MOM_BLOCKS / h->nslab);
    h->N = p->nx * p->ny * p->nz;
    h->storage = p->storage;
    h->esize = p->storage == LBM_STORE_F32 ? 4 : 2;
    auto die = [&](lbm_status s, const std::string &m) {
        g_init_error = m;
        free_all(h);
        delete h;
        return s;
    };
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return die(LBM_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    if (p->stream || p->stream_given) {
        h->st = (hipStream_t)p->stream;
    } else {
        e = hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking);
        if (e != hipSuccess) return die(LBM_E_DEVICE, "hipStreamCreate failed");
        h->own_stream = true;
    }
    const size_t N = (size_t)h->N;
    const size_t fbytes = 2 * (size_t)Q * N * h->esize;
    if (h->storage == LBM_STORE_F16_LOCAL &&
        (dalloc(&h->rsite[0], 2 * N) != hipSuccess || dalloc(&h->rsite[1], 2 * N) != hipSuccess ||
         hipMemsetAsync(h->rsite[1], 0, 2 * N * sizeof(float), h->st) != hipSuccess))
        return die(LBM_E_NOMEM, "device allocation failed");
    if (hipMalloc(&h->f[0], fbytes) != hipSuccess || hipMalloc(&h->f[1], fbytes) != hipSuccess ||
        dalloc(&h->flag, N) != hipSuccess || dalloc(&h->ibm, N) != hipSuccess ||
        dalloc(&h->uo, N) != hipSuccess || dalloc(&h->ro, N) != hipSuccess ||
        dalloc(&h->psi, 2 * N) != hipSuccess || dalloc(&h->cap_drho, (size_t)MAX_CAPS) != hipSuccess ||
        dalloc(&h->rho_tmp, 2 * N) != hipSuccess ||
        dalloc(&h->men_tmp, (size_t)h->nx * h->ny * h->nslab) != hipSuccess ||
        dalloc(&h->status, (size_t)ST_WORDS) != hipSuccess ||
        dalloc(&h->partial, (size_t)h->nslab * h->mom_blocks * 5) != hipSuccess)
        return die(LBM_E_NOMEM, "device allocation failed");
    if (hipMemsetAsync(h->f[0], 0, fbytes, h->st) != hipSuccess ||
        hipMemsetAsync(h->f[1], 0, fbytes, h->st) != hipSuccess ||
        hipMemsetAsync(h->flag, 0, N, h->st) != hipSuccess ||
        hipMemsetAsync(h->ibm, 0, N * sizeof(float4), h->st) != hipSuccess ||
        hipMemsetAsync(h->uo, 0, N * sizeof(float4), h->st) != hipSuccess ||
        hipMemsetAsync(h->ro, 0, N * sizeof(float4), h->st) != hipSuccess ||
        hipMemsetAsync(h->psi, 0, 2 * N * sizeof(float), h->st) != hipSuccess ||
        hipMemsetAsync(h->cap_drho, 0, MAX_CAPS * sizeof(float), h->st) != hipSuccess ||
        hipMemsetAsync(h->status, 0, ST_WORDS * sizeof(int), h->st) != hipSuccess)
        return die(LBM_E_DEVICE, "device memset failed");

    std::vector<double> rho;
    initial_density(*p, lz, rho);
    for (double v : rho)
        if (!std::isfinite(v) || v < 0.0) return die(LBM_E_INVAL, "initial densities must be finite and >= 0");
    double *d_rho = nullptr;
    if (dalloc(&d_rho, 2 * N) != hipSuccess) return die(LBM_E_NOMEM, "device allocation failed");
    e = hipMemcpyAsync(d_rho, rho.data(), 2 * N * sizeof(double), hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess) {
        const float s0 = shift_of(h, 0), s1 = shift_of(h, 1);
        switch (h->storage) {
            case 0: launch_init_eq<0>(d_rho, h->f[0], h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, nullptr, h->st); break;
            case 1: launch_init_eq<1>(d_rho, h->f[0], h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, nullptr, h->st); break;
            case 2: launch_init_eq<2>(d_rho, h->f[0], h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, nullptr, h->st); break;
            default: launch_init_eq<3>(d_rho, h->f[0], h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, h->rsite[0], h->st); break;
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    (void)hipFree(d_rho);
    if (e != hipSuccess) return die(LBM_E_DEVICE, std::string("initialisation: ") + hipGetErrorString(e));
    *out = h;
    return LBM_OK;
}

// ------------------------------------------------------------------------------------
// Capsules
// ------------------------------------------------------------------------------------
extern "C" lbm_status lbm_add_capsule(lbm_handle *h, const lbm_capsule_params *cp,
                                      int32_t n_nodes, const double *xyz, int32_t n_tri,
                                      const int32_t *tri, int32_t *id_out) {
    if (!h) return LBM_E_INVAL;
    if (h->finalized) return fail(h, LBM_E_STATE, "capsules must be added before the first step");
    static_assert(MAX_CAPS == LBM_MAX_CAPSULES && MAX_CAP_NODES == LBM_MAX_CAPSULE_NODES,
                  "limits in lbm.h and the kernels agree");
    if (!cp || !xyz || !tri || n_nodes < 4 || n_tri < 4 || n_nodes > MAX_CAP_NODES)
        return fail(h, LBM_E_INVAL, "invalid capsule mesh");
    if ((int)h->caps.size() >= MAX_CAPS) return fail(h, LBM_E_INVAL, "too many capsules");
    if (!(cp->ks >= 0.0) || !(cp->C > -0.5) || !(cp->kv >= 0.0) || !(cp->anchor_k >= 0.0) ||
        !(cp->kb >= 0.0) || !std::isfinite(cp->kb) || !std::isfinite(cp->wet_drho))
        return fail(h, LBM_E_INVAL, "invalid capsule parameters");
    for (int i = 0; i < 3 * n_tri; ++i)
        if (tri[i] < 0 || tri[i] >= n_nodes) return fail(h, LBM_E_INVAL, "triangle index out of range");
    for (int i = 0; i < 3 * n_nodes; ++i)
        if (!std::isfinite(xyz[i])) return fail(h, LBM_E_INVAL, "non-finite node position");
    {
        // the site window the kernels derive from the FP32-rounded bounding box must fit
        // the window limits and the lattice (the device reports a capsule that later
        // outgrows them)
        const int nd[3] = {h->nx, h->ny, h->nz};
        int dim[3];
        for (int d = 0; d < 3; ++d) {
            float lo = 3e38f, hi = -3e38f;
            for (int i = 0; i < n_nodes; ++i) {
                const float v = (float)xyz[3 * i + d];
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
            dim[d] = (int)std::floor(hi) - (int)std::floor(lo) + 4;
            if (dim[d] > GMAX || dim[d] > nd[d])
                return fail(h, LBM_E_INVAL, "capsule too large for its site window (at most 64 "
                                            "sites and the lattice size per axis)");
        }
        if (dim[0] * dim[1] > FILL_COLS)
            return fail(h, LBM_E_INVAL, "capsule window wider than 2048 lattice columns (x * y)");
    }
    // slab of the capsule: the one holding its node mean
    double cz = 0.0;
    for (int i = 0; i < n_nodes; ++i) cz += xyz[3 * i + 2];
    cz /= n_nodes;
    int zbase = 0;
    if (h->nslab > 1) {
        const int sl = (int)std::floor(cz / h->lz);
        if (sl < 0 || sl >= h->nslab) return fail(h, LBM_E_INVAL, "capsule centroid outside the lattice");
        zbase = sl * h->lz;
        float lo = 3e38f, hi = -3e38f;
        for (int i = 0; i < n_nodes; ++i) {
            lo = std::min(lo, (float)xyz[3 * i + 2]);
            hi = std::max(hi, (float)xyz[3 * i + 2]);
        }
        const int wlo = (int)std::floor(lo) - 1, whi = (int)std::floor(hi) + 2;
        if (wlo < zbase || whi > zbase + h->lz)
            return fail(h, LBM_E_INVAL, "capsule window crosses a wall layer of its slab");
    }
    HostCap c;
    c.p = *cp;
    c.zbase = zbase;
    if (cp->kb != 0.0) {
        if (!bending_edges(n_tri, tri, c.edge))
            return fail(h, LBM_E_INVAL, "bending needs a closed, consistently oriented mesh");
        c.th0.resize(c.edge.size() / 4);
        for (size_t e = 0; e < c.th0.size(); ++e) {
            const int32_t *q = &c.edge[4 * e];
            c.th0[e] = dihedral_of(xyz + 3 * q[0], xyz + 3 * q[1], xyz + 3 * q[2], xyz + 3 * q[3]);
        }
    }
    c.x0.assign(xyz, xyz + 3 * (size_t)n_nodes);
    c.tri.assign(tri, tri + 3 * (size_t)n_tri);
    h->caps.push_back(std::move(c));
    if (id_out) *id_out = (int32_t)h->caps.size() - 1;
    return LBM_OK;
}

// Geodesic sphere: the icosahedron (vertices (0, +-1, +-t) and their cyclic permutations,
// t the golden ratio, on the unit sphere) with every edge split at its midpoint `level`
// times, each new vertex projected back onto the unit sphere; faces outward and
// counter-clockwise.  Level L: 10 * 4^L + 2 nodes, 20 * 4^L triangles.  FP64.
static void icosphere(int level, std::vector<double> &v, std::vector<int32_t> &f) {
    const double t = (1.0 + std::sqrt(5.0)) / 2.0;
    const double iv[12][3] = {{-1, t, 0}, {1, t, 0}, {-1, -t, 0}, {1, -t, 0},
                              {0, -1, t}, {0, 1, t}, {0, -1, -t}, {0, 1, -t},
                              {t, 0, -1}, {t, 0, 1}, {-t, 0, -1}, {-t, 0, 1}};
    const int ifc[20][3] = {{0, 11, 5}, {0, 5, 1}, {0, 1, 7}, {0, 7, 10}, {0, 10, 11},
                            {1, 5, 9}, {5, 11, 4}, {11, 10, 2}, {10, 7, 6}, {7, 1, 8},
                            {3, 9, 4}, {3, 4, 2}, {3, 2, 6}, {3, 6, 8}, {3, 8, 9},
                            {4, 9, 5}, {2, 4, 11}, {6, 2, 10}, {8, 6, 7}, {9, 8, 1}};
    v.clear();
    f.clear();
    auto push_unit = [&](double x, double y, double z) {
        const double n = std::sqrt(x * x + y * y + z * z);
        v.push_back(x / n);
        v.push_back(y / n);
        v.push_back(z / n);
    };
    for (const auto &p : iv) push_unit(p[0], p[1], p[2]);
    for (const auto &q : ifc) f.insert(f.end(), {q[0], q[1], q[2]});
    for (int l = 0; l < level; ++l) {
        std::unordered_map<long long, int> cache;   // edge -> midpoint index
        cache.reserve(f.size());
        auto mid = [&](int a, int b) {
            const long long key = a < b ? (long long)a << 32 | b : (long long)b << 32 | a;
            const auto it = cache.find(key);
            if (it != cache.end()) return it->second;
            push_unit((v[3 * a] + v[3 * b]) * 0.5, (v[3 * a + 1] + v[3 * b + 1]) * 0.5,
                      (v[3 * a + 2] + v[3 * b + 2]) * 0.5);
            const int idx = (int)(v.size() / 3) - 1;
            cache.emplace(key, idx);
            return idx;
        };
        std::vector<int32_t> nf;
        nf.reserve(4 * f.size());
        for (size_t i = 0; i < f.size(); i += 3) {
            const int a = f[i], b = f[i + 1], c = f[i + 2];
            const int ab = mid(a, b), bc = mid(b, c), ca = mid(c, a);
            nf.insert(nf.end(), {a, ab, ca, b, bc, ab, c, ca, bc, ab, bc, ca});
        }
        f.swap(nf);
    }
    // outward orientation: normal . (p0 + p1 + p2) > 0
    for (size_t i = 0; i < f.size(); i += 3) {
        const double *p0 = &v[3 * f[i]], *p1 = &v[3 * f[i + 1]], *p2 = &v[3 * f[i + 2]];
        const double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        const double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
        const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        const double s = n[0] * (p0[0] + p1[0] + p2[0]) + n[1] * (p0[1] + p1[1] + p2[1]) +
                         n[2] * (p0[2] + p1[2] + p2[2]);
        if (s < 0) std::swap(f[i + 1], f[i + 2]);
    }
}

extern "C" lbm_status lbm_add_sphere_capsule(lbm_handle *h, const lbm_capsule_params *cp,
                                             const double center[3], double radius, int32_t n_tri,
                                             int32_t *id_out) {
    if (!h) return LBM_E_INVAL;
    if (!center || !(radius > 0.0) || !std::isfinite(radius) || !std::isfinite(center[0]) ||
        !std::isfinite(center[1]) || !std::isfinite(center[2]))
        return fail(h, LBM_E_INVAL, "invalid sphere centre or radius");
    int level = -1;
    for (int l = 0, nt = 20; l <= 6; ++l, nt *= 4)
        if (nt == n_tri) level = l;
    if (level < 0) return fail(h, LBM_E_INVAL, "n_tri must be 20 * 4^L, L = 0 .. 6");
    std::vector<double> v;
    std::vector<int32_t> f;
    icosphere(level, v, f);
    for (size_t i = 0; i < v.size(); i += 3)
        for (int d = 0; d < 3; ++d) v[i + d] = v[i + d] * radius + center[d];
    return lbm_add_capsule(h, cp, (int32_t)(v.size() / 3), v.data(), (int32_t)(f.size() / 3),
                           f.data(), id_out);
}

// Reference geometry of a triangle (FP64): the vertices in an orthonormal in-plane
// frame, P1 = (0, 0), P2 = (a, 0), P3 = (b, c); returns the inverse of [P2-P1, P3-P1]
// (row-major) and the area.
static void tri_reference(const double *p1, const double *p2, const double *p3, double minv[4],
                          double *area) {
    double u[3], v[3];
    for (int d = 0; d < 3; ++d) { u[d] = p2[d] - p1[d]; v[d] = p3[d] - p1[d]; }
    const double a = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double b = (v[0] * u[0] + v[1] * u[1] + v[2] * u[2]) / a;
    double w2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double wd = v[d] - b * u[d] / a;
        w2 += wd * wd;
    }
    const double c = std::sqrt(w2);
    minv[0] = 1.0 / a;
    minv[1] = -b / (a * c);
    minv[2] = 0.0;
    minv[3] = 1.0 / c;
    *area = 0.5 * a * c;
}

static lbm_status finalize(lbm_handle *h) {
    const int ncap = (int)h->caps.size();
    h->finalized = true;
    if (ncap == 0) return LBM_OK;
    std::vector<double4> X;
    std::vector<int> node_cap, off, list;
    std::vector<int4> tri;
    std::vector<float4> minv;
    std::vector<float> a0;
    std::vector<float> drho(MAX_CAPS, 0.0f);
    h->h_caps.clear();
    for (int k = 0; k < ncap; ++k) {
        const HostCap &c = h->caps[k];
        const int nn = (int)c.x0.size() / 3, nt = (int)c.tri.size() / 3;
        CapDev cd{};
        cd.node0 = (int)X.size();
        cd.nn = nn;
        cd.tri0 = (int)tri.size();
        cd.nt = nt;
        cd.ks = (float)c.p.ks;
        cd.C = (float)c.p.C;
        cd.kv = (float)c.p.kv;
        cd.anchor_k = (float)c.p.anchor_k;
        cd.kb = (float)c.p.kb;
        cd.zbase = c.zbase;
        cd.plane_z = (float)(c.zbase + 0.5 + h->p.plane_dz);
        double cen[3] = {0, 0, 0};
        for (int i = 0; i < nn; ++i) {
            X.push_back(make_double4(c.x0[3 * i], c.x0[3 * i + 1], c.x0[3 * i + 2], 0.0));
            node_cap.push_back(k);
            for (int d = 0; d < 3; ++d) cen[d] += c.x0[3 * i + d];
        }
        for (int d = 0; d < 3; ++d) cd.c0[d] = cen[d] / nn;
        double vol = 0.0;
        for (int t = 0; t < nt; ++t) {
            const double *p1 = &c.x0[3 * c.tri[3 * t]], *p2 = &c.x0[3 * c.tri[3 * t + 1]],
                         *p3 = &c.x0[3 * c.tri[3 * t + 2]];
            double m[4], area;
            tri_reference(p1, p2, p3, m, &area);
            if (!(area > 0.0) || !std::isfinite(m[0] + m[1] + m[3]))
                return fail(h, LBM_E_INVAL, "degenerate reference triangle");
            tri.push_back(make_int4(cd.node0 + c.tri[3 * t], cd.node0 + c.tri[3 * t + 1],
                                    cd.node0 + c.tri[3 * t + 2], k));
            minv.push_back(make_float4((float)m[0], (float)m[1], (float)m[2], (float)m[3]));
            a0.push_back((float)area);
            double a[3], b[3], e[3];
            for (int d = 0; d < 3; ++d) {
                a[d] = p1[d] - cd.c0[d];
                b[d] = p2[d] - cd.c0[d];
                e[d] = p3[d] - cd.c0[d];
            }
            vol += (a[0] * (b[1] * e[2] - b[2] * e[1]) + a[1] * (b[2] * e[0] - b[0] * e[2]) +
                    a[2] * (b[0] * e[1] - b[1] * e[0])) / 6.0;
        }
        if (!(vol > 0.0)) return fail(h, LBM_E_INVAL, "capsule mesh must be closed and outward oriented");
        cd.v0 = vol;
        drho[k] = (float)c.p.wet_drho;
        h->h_caps.push_back(cd);
    }
    h->ntot = (int)X.size();
    h->ttot = (int)tri.size();
    // node -> incident triangle CSR (entries 3 * triangle + corner, triangle order)
    off.assign(h->ntot + 1, 0);
    for (const int4 &t : tri) { off[t.x + 1]++; off[t.y + 1]++; off[t.z + 1]++; }
    for (int i = 0; i < h->ntot; ++i) off[i + 1] += off[i];
    list.assign(off[h->ntot], 0);
    std::vector<int> cur(off.begin(), off.end() - 1);
    for (int t = 0; t < h->ttot; ++t) {
        list[cur[tri[t].x]++] = 3 * t;
        list[cur[tri[t].y]++] = 3 * t + 1;
        list[cur[tri[t].z]++] = 3 * t + 2;
    }
    // bending edges (global node indices) and the node -> (edge, role) CSR
    std::vector<int4> edges;
    std::vector<float> eth0;
    for (int k = 0; k < ncap; ++k) {
        const HostCap &c = h->caps[k];
        const int n0 = h->h_caps[k].node0;
        for (size_t e = 0; e < c.th0.size(); ++e) {
            const int32_t *q = &c.edge[4 * e];
            edges.push_back(make_int4(n0 + q[0], n0 + q[1], n0 + q[2], n0 + q[3]));
            eth0.push_back((float)c.th0[e]);
        }
    }
    std::vector<int> eoff(h->ntot + 1, 0), elist(4 * edges.size());
    for (const int4 &q : edges) { eoff[q.x + 1]++; eoff[q.y + 1]++; eoff[q.z + 1]++; eoff[q.w + 1]++; }
    for (int i = 0; i < h->ntot; ++i) eoff[i + 1] += eoff[i];
    {
        std::vector<int> ecur(eoff.begin(), eoff.end() - 1);
        for (size_t e = 0; e < edges.size(); ++e) {
            const int v[4] = {edges[e].x, edges[e].y, edges[e].z, edges[e].w};
            for (int r = 0; r < 4; ++r) elist[ecur[v[r]]++] = 4 * (int)e + r;
        }
    }
    const size_t nt = h->ntot, tt = h->ttot;
    if (dalloc(&h->d_edge, edges.size()) != hipSuccess || dalloc(&h->d_eth0, eth0.size()) != hipSuccess ||
        dalloc(&h->d_eoff, nt + 1) != hipSuccess || dalloc(&h->d_elist, elist.size()) != hipSuccess)
        return fail(h, LBM_E_NOMEM, "device allocation failed (bending)");
    if (!edges.empty()) {
        HIPCHK(h, hipMemcpyAsync(h->d_edge, edges.data(), edges.size() * sizeof(int4), hipMemcpyHostToDevice, h->st));
        HIPCHK(h, hipMemcpyAsync(h->d_eth0, eth0.data(), eth0.size() * sizeof(float), hipMemcpyHostToDevice, h->st));
        HIPCHK(h, hipMemcpyAsync(h->d_elist, elist.data(), elist.size() * sizeof(int), hipMemcpyHostToDevice, h->st));
    }
    HIPCHK(h, hipMemcpyAsync(h->d_eoff, eoff.data(), (nt + 1) * sizeof(int), hipMemcpyHostToDevice, h->st));
    if (dalloc(&h->d_caps, ncap) != hipSuccess || dalloc(&h->d_cst, ncap) != hipSuccess ||
        dalloc(&h->d_X, nt) != hipSuccess || dalloc(&h->d_node_cap, nt) != hipSuccess ||
        dalloc(&h->d_F, nt) != hipSuccess || dalloc(&h->d_Fh, nt) != hipSuccess ||
        dalloc(&h->d_R, nt) != hipSuccess || dalloc(&h->d_tri, tt) != hipSuccess ||
        dalloc(&h->d_minv, tt) != hipSuccess || dalloc(&h->d_a0, tt) != hipSuccess ||
        dalloc(&h->d_off, nt + 1) != hipSuccess || dalloc(&h->d_list, list.size()) != hipSuccess ||
        dalloc(&h->d_marks, (size_t)ncap * ROWS_MAX) != hipSuccess ||
        dalloc(&h->d_rowstart, (size_t)ncap * (ROWS_MAX + 1)) != hipSuccess ||
        dalloc(&h->d_slot, nt) != hipSuccess || dalloc(&h->d_xrow, nt) != hipSuccess ||
        dalloc(&h->d_wbuf, (size_t)ncap * GMAX3) != hipSuccess ||
        dalloc(&h->d_wpar, (size_t)ncap * GMAX3) != hipSuccess)
        return fail(h, LBM_E_NOMEM, "device allocation failed (capsules)");
    HIPCHK(h, hipMemcpyAsync(h->d_caps, h->h_caps.data(), ncap * sizeof(CapDev), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipMemsetAsync(h->d_cst, 0, ncap * sizeof(CapState), h->st));
    HIPCHK(h, hipMemcpyAsync(h->d_X, X.data(), nt * sizeof(double4), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipMemcpyAsync(h->d_node_cap, node_cap.data(), nt * sizeof(int), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipMemsetAsync(h->d_F, 0, nt * sizeof(float4), h->st));
    HIPCHK(h, hipMemsetAsync(h->d_Fh, 0, nt * sizeof(float4), h->st));
    HIPCHK(h, hipMemsetAsync(h->d_R, 0, nt * sizeof(float4), h->st));
    HIPCHK(h, hipMemcpyAsync(h->d_tri, tri.data(), tt * sizeof(int4), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipMemcpyAsync(h->d_minv, minv.data(), tt * sizeof(float4), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipMemcpyAsync(h->d_a0, a0.data(), tt * sizeof(float), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipMemcpyAsync(h->d_off, off.data(), (nt + 1) * sizeof(int), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipMemcpyAsync(h->d_list, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipMemsetAsync(h->d_marks, 0, (size_t)ncap * ROWS_MAX * sizeof(unsigned long long), h->st));
    HIPCHK(h, hipMemsetAsync(h->d_rowstart, 0, (size_t)ncap * (ROWS_MAX + 1) * sizeof(int), h->st));
    HIPCHK(h, hipMemsetAsync(h->d_slot, 0, nt * sizeof(int), h->st));
    HIPCHK(h, hipMemsetAsync(h->d_xrow, 0, nt * sizeof(double4), h->st));
    HIPCHK(h, hipMemcpyAsync(h->cap_drho, drho.data(), MAX_CAPS * sizeof(float), hipMemcpyHostToDevice, h->st));
    if (h->p.coupling == 1) {
        // links per capsule: a closed surface of area A cuts about 5.74 A lattice links; a
        // triangle of the meshes here has an area of about 0.1 .. 0.3, so 24 links per
        // triangle leave a wide margin (overflow is reported as LBM_E_UNSTABLE)
        int mt = 1;
        for (const CapDev &c : h->h_caps) mt = std::max(mt, c.nt);
        h->link_cap = std::max(4096, 24 * mt);
        if (dalloc(&h->d_V, nt) != hipSuccess || dalloc(&h->d_pex, 3 * tt) != hipSuccess ||
            dalloc(&h->d_rsc, 3 * tt) != hipSuccess || dalloc(&h->d_pprev, nt) != hipSuccess ||
            dalloc(&h->d_ffl, nt) != hipSuccess ||
            dalloc(&h->d_bstart, (size_t)ncap * (GMAX3 + 1)) != hipSuccess ||
            dalloc(&h->d_blist, (size_t)BB_PER_TRI * tt) != hipSuccess ||
            dalloc(&h->d_nlinks, 2 * (size_t)ncap) != hipSuccess ||
            dalloc(&h->d_links, (size_t)ncap * h->link_cap) != hipSuccess ||
            dalloc(&h->d_tpos, 3 * tt) != hipSuccess || dalloc(&h->d_tcell, tt) != hipSuccess)
            return fail(h, LBM_E_NOMEM, "device allocation failed (bounce-back)");
        HIPCHK(h, hipMemsetAsync(h->d_V, 0, nt * sizeof(double4), h->st));
        HIPCHK(h, hipMemsetAsync(h->d_pex, 0, 3 * tt * sizeof(long long), h->st));
        HIPCHK(h, hipMemsetAsync(h->d_rsc, 0, 3 * tt * sizeof(long long), h->st));
        HIPCHK(h, hipMemsetAsync(h->d_pprev, 0, nt * sizeof(float4), h->st));
        HIPCHK(h, hipMemsetAsync(h->d_ffl, 0, nt * sizeof(float4), h->st));
        HIPCHK(h, hipMemsetAsync(h->d_bstart, 0, (size_t)ncap * (GMAX3 + 1) * sizeof(int), h->st));
        HIPCHK(h, hipMemsetAsync(h->d_blist, 0, (size_t)BB_PER_TRI * tt * sizeof(int), h->st));
        HIPCHK(h, hipMemsetAsync(h->d_nlinks, 0, 2 * (size_t)ncap * sizeof(int), h->st));
    }
    HIPCHK(h, hipStreamSynchronize(h->st));
    return LBM_OK;
}

// arguments of the bounce-back kernels for the step reading population buffer cur
static BBArgs bb_args(lbm_handle *h, int cur) {
    BBArgs b{};
    b.caps = h->d_caps; b.cst = h->d_cst;
    b.ncap = (int)h->caps.size(); b.ntot = h->ntot; b.ttot = h->ttot;
    b.tri = h->d_tri; b.X = h->d_X; b.V = h->d_V; b.F = h->d_F; b.slot = h->d_slot;
    b.flag = h->flag;
    b.f = h->f[cur];
    b.dens = h->ro;
    b.tpos = h->d_tpos;
    b.tcell = h->d_tcell;
    b.N = h->N; b.nx = h->nx; b.ny = h->ny; b.nz = h->nz; b.wall = h->wall; b.lz = h->lz;
    b.shift[0] = shift_of(h, 0);
    b.shift[1] = shift_of(h, 1);
    b.bstart = h->d_bstart; b.blist = h->d_blist;
    b.links = h->d_links; b.link_cap = h->link_cap; b.nlinks = h->d_nlinks;
    b.pex = h->d_pex; b.rsc = h->d_rsc; b.ntri_off = h->d_off; b.ntri = h->d_list; b.pprev = h->d_pprev; b.ffl = h->d_ffl; b.R = h->d_R;
    b.status = h->status;
    b.G = (float)h->p.G;
    b.ws_axis = (float)(h->p.sc_norm / 18.0);
    b.ws_diag = (float)(h->p.sc_norm / 36.0);
    b.inv_rho0 = (float)(1.0 / h->p.rho0);
    b.cap_drho = h->cap_drho;
    b.inv_mass = 1.0 / h->p.node_mass;
    return b;
}

// ------------------------------------------------------------------------------------
// Stepping
// ------------------------------------------------------------------------------------
static MembraneArgs membrane_args(lbm_handle *h) {
    MembraneArgs m{};
    m.caps = h->d_caps; m.cst = h->d_cst; m.ncap = (int)h->caps.size();
    m.X = h->d_X; m.node_cap = h->d_node_cap; m.F = h->d_F; m.Fh = h->d_Fh; m.R = h->d_R;
    m.tri = h->d_tri; m.minv = h->d_minv; m.a0 = h->d_a0;
    m.ntri_off = h->d_off; m.ntri = h->d_list;
    m.edge = h->d_edge; m.eth0 = h->d_eth0; m.nedge_off = h->d_eoff; m.nedge = h->d_elist;
    m.marks = h->d_marks; m.rowstart = h->d_rowstart; m.xrow = h->d_xrow; m.slot = h->d_slot;

    m.wbuf = h->d_wbuf; m.wpar = h->d_wpar;
    m.flag = h->flag; m.ibm = h->ibm; m.uo = h->uo; m.ro = h->ro; m.status = h->status;
    m.nx = h->nx; m.ny = h->ny; m.nz = h->nz; m.wall = h->wall; m.lz = h->lz;
    m.hertz_xi = (float)h->p.hertz_xi;
    m.hertz_d0 = (float)h->p.hertz_delta0;
    m.bb = h->p.coupling == 1;
    return m;
}

// arguments of the fluid kernel reading population buffer cur
static FluidArgs fluid_args(lbm_handle *h, int cur) {
    FluidArgs a{};
    a.fin = h->f[cur];
    a.fout = h->f[1 - cur];
    a.rin = h->rsite[cur];
    a.rout = h->rsite[1 - cur];
    a.flag = h->flag; a.ibm = h->ibm; a.uo = h->uo; a.ro = h->ro; a.psi = h->psi;
    a.status = h->status; a.cap_drho = h->cap_drho;
    a.nx = h->nx; a.ny = h->ny; a.nz = h->nz; a.wall = h->wall; a.N = h->N; a.lz = h->lz;
    for (int c = 0; c < 2; ++c) {
        a.tau[c] = (float)h->p.tau[c];
        a.inv_tau[c] = (float)(1.0 / h->p.tau[c]);
        a.shift[c] = shift_of(h, c);
    }
    a.G = (float)h->p.G;
    a.ws_axis = (float)(h->p.sc_norm / 18.0);
    a.ws_diag = (float)(h->p.sc_norm / 36.0);
    a.inv_rho0 = (float)(1.0 / h->p.rho0);
    for (int d = 0; d < 3; ++d) a.g[d] = (float)h->p.body_force[d];
    a.wall_drho = (float)h->p.wall_drho;
    a.keepf = !(h->p.tau[0] == 1.0 && h->p.tau[1] == 1.0);
    a.bb = !h->caps.empty() && h->p.coupling == 1;
    a.zero_drho = h->p.wall_drho == 0.0;
    for (const HostCap &c : h->caps) a.zero_drho = a.zero_drho && c.p.wet_drho == 0.0;
    return a;
}

static const int TILE_X[13] = {0, 32, 64, 32, 64, 16, 32, 64, 16, 32, 64, 256, 128},
                 TILE_Y[13] = {0, 8, 4, 16, 8, 16, 8, 4, 16, 16, 8, 2, 4};
constexpr int TILE_ROWS = 13;   // whole rows of the lattice's width (16 <= nx <= 128)

static bool rows_fit(int nx) { return nx >= 16 && nx <= 128; }

// tiles per plane of a launch shape: (tiles in x, tiles in y); the whole-row shapes fall
// back to 64 x 8 where the width does not fit, as the launcher does
static void tiles_of(int tile, int nx, int ny, int *tx, int *ty) {
    if (tile == TILE_ROWS && rows_fit(nx)) {
        const int h = rows_tile_height(nx);
        *tx = 1;
        *ty = (ny + h - 1) / h;
        return;
    }
    if ((tile == 11 && nx != 256) || (tile == 12 && nx != 128) || tile == TILE_ROWS) tile = 10;
    *tx = (nx + TILE_X[tile] - 1) / TILE_X[tile];
    *ty = (ny + TILE_Y[tile] - 1) / TILE_Y[tile];
}

// z planes per workgroup: enough workgroups to fill the chip (about 1024), at least 4
// planes so the two extra halo planes stay a small share
static int zchunk_for(const lbm_handle *h, int tile, int zchunk) {
    if (zchunk > 0) return zchunk;
    if (tile <= 0) return h->nz;
    int tx, ty;
    tiles_of(tile, h->nx, h->ny, &tx, &ty);
    const int tiles = tx * ty;
    const int chunks = (1024 + tiles - 1) / tiles;
    const int zc = (h->nz + chunks - 1) / chunks;
    return zc < 4 ? 4 : zc;
}

static int zchunk_of(const lbm_handle *h) { return zchunk_for(h, h->tile, h->zchunk); }

extern "C" lbm_status lbm_set_launch(lbm_handle *h, int32_t tile, int32_t zchunk) {
    if (!h) return LBM_E_INVAL;
    if (tile < 0 || tile > TILE_ROWS || zchunk < 0) return fail(h, LBM_E_INVAL, "invalid launch shape");
    h->tile = tile;
    h->zchunk = zchunk;
    h->zoff = 0;
    return LBM_OK;
}

extern "C" lbm_status lbm_set_zoffset(lbm_handle *h, int32_t planes) {
    if (!h) return LBM_E_INVAL;
    const int zc = zchunk_of(h);
    if (planes < 0 || (planes > 0 && (zc >= h->nz || planes >= zc)))
        return fail(h, LBM_E_INVAL, "z offset must be 0 .. z-chunk - 1, and 0 for one chunk");
    h->zoff = planes;
    return LBM_OK;
}

extern "C" int32_t lbm_zoffset(const lbm_handle *h) { return h ? h->zoff : 0; }

// one launch of the fluid kernel of the given shape for the handle's storage, the first
// z-chunk shortened by zoff planes (an offset not below the chunk, which lbm_set_zoffset
// never stores, launches equal chunks)
static void enqueue_fluid(const lbm_handle *h, const FluidArgs &a0, int tile, int zc, int zoff,
                          hipStream_t st) {
    FluidArgs a = a0;
    a.zoff = zoff < zc ? zoff : 0;
    switch (h->storage) {
        case 0: launch_fluid_tiled<0>(a, tile, zc, st); break;
        case 1: launch_fluid_tiled<1>(a, tile, zc, st); break;
        case 2: launch_fluid_tiled<2>(a, tile, zc, st); break;
        default: launch_fluid_tiled<3>(a, tile, zc, st); break;
    }
}

// labels, membrane forces and spreading: the kernels of a step before the fluid kernel
static void capsule_kernels_before(lbm_handle *h, const MembraneArgs &m, Prof &pf) {
    timed(pf, h->st, "capsule_reduce", [&] { launch_capsule_reduce(m, h->st); });
    timed(pf, h->st, "membrane", [&] { launch_membrane(m, h->ntot, h->ttot, h->st); });
    timed(pf, h->st, "window_fill", [&] { launch_window_fill(m, h->st); });
}

extern "C" lbm_status lbm_step(lbm_handle *h, int64_t n) {
    if (!h) return LBM_E_INVAL;
    if (n < 0) return fail(h, LBM_E_INVAL, "negative step count");
    if (!h->finalized) {
        lbm_status s = finalize(h);
        if (s != LBM_OK) return s;
    }
    const bool caps = !h->caps.empty();
    const bool bb = caps && h->p.coupling == 1;
    MembraneArgs m = caps ? membrane_args(h) : MembraneArgs{};
    for (int64_t i = 0; i < n; ++i) {
        if (caps) capsule_kernels_before(h, m, h->prof);
        if (bb) {
            const BBArgs b = bb_args(h, h->cur);
            timed(h->prof, h->st, "bounce_back", [&] { launch_bb_before(b, h->storage, h->st); });
        }
        const FluidArgs a = fluid_args(h, h->cur);
        const int zc = zchunk_of(h);
        timed(h->prof, h->st, "fluid", [&] { enqueue_fluid(h, a, h->tile, zc, h->zoff, h->st); });
        if (bb) {
            const BBArgs b = bb_args(h, h->cur);
            timed(h->prof, h->st, "bb_nodes", [&] { launch_bb_after(b, h->storage, h->st); });
        } else if (caps) {
            timed(h->prof, h->st, "node_update", [&] { launch_node_update(m, h->ntot, h->st); });
        }
        h->cur = 1 - h->cur;
        h->step++;
    }
    HIPCHK(h, hipGetLastError());
    return LBM_OK;
}

// ------------------------------------------------------------------------------------
// Launch-shape autotuner
// ------------------------------------------------------------------------------------
// z-chunk depths the tuners try (0: the default from the lattice size)
static const int TUNE_ZC[] = {0, 8, 12, 16, 24, 32, 48};

// tiles the tuner tries on a lattice of width nx: every fused shape that applies.  With
// tau != 1 the pipelined and whole-row numbers run the fused kernel of 1..5 or 64 x 8, so
// only 1..5 are distinct there.
static bool tile_applies(int tile, int nx, bool keepf, int storage) {
    if (tile < 1 || tile > TILE_ROWS || (keepf && tile >= 6)) return false;
    if (storage == LBM_STORE_F16_LOCAL && tile < 6) return false;   // runs the pipelined tiles
    if (tile == 11) return nx == 256;
    if (tile == 12) return nx == 128;
    if (tile == TILE_ROWS) return rows_fit(nx);
    return true;
}

// mean duration of `reps` calls of `launch` on stream st (events e0, e1), after two untimed
template <typename F>
static hipError_t time_launches(hipStream_t st, int reps, hipEvent_t e0, hipEvent_t e1,
                                F &&launch, double *ms) {
    launch();
    launch();
    hipError_t e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess) e = hipGetLastError();
    *ms = (double)t / reps;
    return e;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t make() {
        hipError_t e = hipEventCreate(&a);
        return e == hipSuccess ? hipEventCreate(&b) : e;
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

extern "C" lbm_status lbm_autotune(lbm_handle *h, int32_t reps, int32_t *tile, int32_t *zchunk,
                                   double *fluid_ms) {
    if (!h) return LBM_E_INVAL;
    if (reps < 1 || reps > 1000) return fail(h, LBM_E_INVAL, "reps must be 1..1000");
    if (!h->finalized) {
        lbm_status s = finalize(h);
        if (s != LBM_OK) return s;
    }
    HIPCHK(h, hipSetDevice(h->p.device));
    int saved[ST_WORDS];
    HIPCHK(h, hipMemcpyAsync(saved, h->status, sizeof saved, hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    EventPair ev;
    HIPCHK(h, ev.make());
    const FluidArgs a = fluid_args(h, h->cur);
    double best = INFINITY;
    int bt = h->tile, bz = h->zchunk;
    for (int t = 1; t <= TILE_ROWS; ++t) {
        if (!tile_applies(t, h->nx, a.keepf, h->storage)) continue;
        int seen[sizeof TUNE_ZC / sizeof TUNE_ZC[0]], ns = 0;
        for (int z : TUNE_ZC) {
            const int zc = std::min(zchunk_for(h, t, z), h->nz);
            if (std::find(seen, seen + ns, zc) != seen + ns) continue;
            seen[ns++] = zc;
            double ms = 0.0;
            HIPCHK(h, time_launches(h->st, reps, ev.a, ev.b,
                                    [&] { enqueue_fluid(h, a, t, zc, 0, h->st); }, &ms));
            if (ms < best) {
                best = ms;
                bt = t;
                bz = zc;
            }
        }
    }
    // the chosen shape with its first z-chunk shortened by 1 .. 4 planes: a launch whose
    // lower chunk holds the capsule sites balances its blocks that way
    int bo = 0;
    for (int d = 1; d <= 4 && bz < h->nz && d < bz; ++d) {
        double ms = 0.0;
        HIPCHK(h, time_launches(h->st, reps, ev.a, ev.b,
                                [&] { enqueue_fluid(h, a, bt, bz, d, h->st); }, &ms));
        if (ms < best) {
            best = ms;
            bo = d;
        }
    }
    // the timed launches wrote only the buffer the next step overwrites and the window
    // outputs it recomputes; the status words (lost-reaction count) are put back
    HIPCHK(h, hipMemcpyAsync(h->status, saved, sizeof saved, hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    h->tile = bt;
    h->zchunk = bz;
    h->zoff = bo;
    if (tile) *tile = bt;
    if (zchunk) *zchunk = bz;
    if (fluid_ms) *fluid_ms = best;
    return LBM_OK;
}

// ------------------------------------------------------------------------------------
// Batches: several handles advanced together, with one launch of each kernel over all
// their lattices and capsules per step
// ------------------------------------------------------------------------------------
// A part: handles advanced by one chain of launches on one stream.  With several parts the
// latency-bound capsule kernels of one part overlap the bandwidth-bound fluid kernel of
// another.
struct BatchPart {
    std::vector<int> idx;          // handles of the part (indices into lbm_batch::hs)
    hipStream_t st = nullptr;      // the batch's stream (one part) or a stream of its own
    bool own_stream = false;
    hipEvent_t done = nullptr;     // recorded on st after the part's last enqueued step
    FluidArgs *d_tab = nullptr;    // [2][handles]: arguments for parity 0 and 1 of the buffers
    int4 *d_desc = nullptr;        // [handles + 1] first logical block, tiles x, tiles y, zchunk
    MembraneArgs *d_mtab = nullptr;  // [groups] capsule-kernel arguments of the handles
    MGroup *d_mgrp = nullptr;        // with capsules, and their places in the launches
    MGroupTotals mtot{};
    int nmg = 0;                   // handles with capsules
    int nblocks = 0;
    int *d_queue = nullptr;        // work queue of the persistent fluid launch (9 ints)
};

struct lbm_batch {
    std::vector<lbm_handle *> hs;
    std::string err;
    hipStream_t st = nullptr;      // the handles' stream
    int storage = 0, device = 0;
    int tile = 10, zchunk = 0, nparts = 1;
    std::vector<BatchPart> parts;
    hipEvent_t start = nullptr;    // on st: work enqueued before a batch step
    std::vector<int64_t> step0;    // step count of each handle when the tables were written
    int64_t since = 0;             // batch steps since then
    bool dirty = true;
    Prof prof;
    bool queue = false;            // fluid launch: resident grid with a work queue
    int ncu = 0;                   // compute units of the device
    bool use_graph = false;        // replay pairs of steps from a captured graph
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // two steps from buffer parity 0 / 1
    hipStream_t gst = nullptr;     // stream the graphs are captured on (the handles' stream
                                   // may be the null stream, which cannot be captured)
};

extern "C" void lbm_batch_destroy(lbm_batch *b);

static lbm_status bfail(lbm_batch *b, lbm_status s, const std::string &m) {
    b->err = m;
    return s;
}

static void free_graphs(lbm_batch *b) {
    for (hipGraphExec_t &g : b->gexec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

static void free_parts(lbm_batch *b) {
    free_graphs(b);   // they hold the parts' tables and streams
    for (BatchPart &pt : b->parts) {
        if (pt.st && pt.own_stream) {
            (void)hipStreamSynchronize(pt.st);
            (void)hipStreamDestroy(pt.st);
        }
        if (pt.done) (void)hipEventDestroy(pt.done);
        void *ptrs[] = {pt.d_tab, pt.d_desc, pt.d_mtab, pt.d_mgrp, pt.d_queue};
        for (void *q : ptrs)
            if (q) (void)hipFree(q);
    }
    b->parts.clear();
}

// z planes per workgroup of a part's fluid launch: 48, halved while the launch has fewer
// than 1024 workgroups (four per compute unit), at least 8
static int batch_zchunk(const lbm_batch *b, const BatchPart &pt, int zc) {
    if (b->zchunk > 0) return b->zchunk;
    long total = 0;
    for (int g : pt.idx) {
        const lbm_handle *h = b->hs[g];
        int tx, ty;
        tiles_of(b->tile, h->nx, h->ny, &tx, &ty);
        total += (long)tx * ty * ((h->nz + zc - 1) / zc);
    }
    return (total >= 1024 || zc <= 8) ? zc : batch_zchunk(b, pt, std::max(8, zc / 2));
}

// split the handles into parts of about equal fluid sites, write every part's tables
static lbm_status batch_tables(lbm_batch *b) {
    const int n = (int)b->hs.size();
    if (hipStreamSynchronize(b->st) != hipSuccess) return bfail(b, LBM_E_DEVICE, "stream synchronisation failed");
    free_parts(b);
    const int np = std::min(b->nparts, n);
    b->parts.resize(np);
    {
        std::vector<int> order(n);
        for (int g = 0; g < n; ++g) order[g] = g;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            return lbm_fluid_sites(b->hs[x]) > lbm_fluid_sites(b->hs[y]);
        });
        std::vector<int64_t> load(np, 0);
        for (int g : order) {
            const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            b->parts[k].idx.push_back(g);
            load[k] += lbm_fluid_sites(b->hs[g]);
        }
        for (BatchPart &pt : b->parts) std::sort(pt.idx.begin(), pt.idx.end());
    }
    for (int g = 0; g < n; ++g) b->step0[g] = b->hs[g]->step;
    b->since = 0;
    for (int k = 0; k < np; ++k) {
        BatchPart &pt = b->parts[k];
        const int m = (int)pt.idx.size();
        const int zc = batch_zchunk(b, pt, 48);
        std::vector<FluidArgs> tab(2 * (size_t)m);
        std::vector<int4> desc(m + 1);
        std::vector<MembraneArgs> mtab;
        std::vector<MGroup> mgrp;
        MGroupTotals t{};
        int start = 0;
        for (int j = 0; j < m; ++j) {
            lbm_handle *h = b->hs[pt.idx[j]];
            if (!h->caps.empty()) {
                MGroup mg{};
                mg.cap0 = t.ncap;
                mg.mem0 = t.mem_blocks;
                mg.upd0 = t.upd_blocks;
                mg.ntot = h->ntot;
                mg.ttot = h->ttot;
                mg.nbu = node_update_blocks(h->ntot);
                t.ncap += (int)h->caps.size();
                t.mem_blocks += membrane_blocks(h->ntot, h->ttot, &mg.nbf);
                t.upd_blocks += mg.nbu;
                mtab.push_back(membrane_args(h));
                mgrp.push_back(mg);
            }
            tab[j] = fluid_args(h, h->cur);
            tab[m + j] = fluid_args(h, 1 - h->cur);
            int tx, ty;
            tiles_of(b->tile, h->nx, h->ny, &tx, &ty);
            desc[j] = make_int4(start, tx, ty, zc);
            start += tx * ty * ((h->nz + zc - 1) / zc);
        }
        desc[m] = make_int4(start, 0, 0, 0);
        pt.nblocks = start;
        pt.nmg = (int)mgrp.size();
        pt.mtot = t;
        bool ok = dalloc(&pt.d_tab, tab.size()) == hipSuccess &&
                  dalloc(&pt.d_desc, desc.size()) == hipSuccess &&
                  dalloc(&pt.d_mtab, mtab.size()) == hipSuccess &&
                  dalloc(&pt.d_mgrp, mgrp.size()) == hipSuccess &&
                  dalloc(&pt.d_queue, 9) == hipSuccess &&
                  hipEventCreateWithFlags(&pt.done, hipEventDisableTiming) == hipSuccess;
        if (ok && np > 1) {
            ok = hipStreamCreateWithFlags(&pt.st, hipStreamNonBlocking) == hipSuccess;
            pt.own_stream = ok;
        } else {
            pt.st = b->st;
        }
        if (!ok) return bfail(b, LBM_E_NOMEM, "device allocation failed (batch)");
        const int zero[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (hipMemcpy(pt.d_queue, zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(pt.d_tab, tab.data(), tab.size() * sizeof(FluidArgs), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(pt.d_desc, desc.data(), desc.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess ||
            (pt.nmg && (hipMemcpy(pt.d_mtab, mtab.data(), mtab.size() * sizeof(MembraneArgs), hipMemcpyHostToDevice) != hipSuccess ||
                        hipMemcpy(pt.d_mgrp, mgrp.data(), mgrp.size() * sizeof(MGroup), hipMemcpyHostToDevice) != hipSuccess)))
            return bfail(b, LBM_E_DEVICE, "batch table upload failed");
    }
    b->dirty = false;
    return LBM_OK;
}

extern "C" lbm_status lbm_batch_create(lbm_handle *const *handles, int32_t n, lbm_batch **out) {
    if (!out) return LBM_E_INVAL;
    *out = nullptr;
    auto bad = [&](const char *m) {
        g_init_error = m;
        return LBM_E_INVAL;
    };
    if (!handles || n < 1) return bad("a batch needs at least one handle");
    for (int g = 0; g < n; ++g) {
        const lbm_handle *h = handles[g];
        if (!h) return bad("NULL handle in batch");
        for (int j = 0; j < g; ++j)
            if (handles[j] == h) return bad("a handle appears twice in the batch");
        if (h->st != handles[0]->st || h->storage != handles[0]->storage ||
            h->p.device != handles[0]->p.device)
            return bad("batched handles must share device, stream and storage mode");
        if (!(h->p.tau[0] == 1.0 && h->p.tau[1] == 1.0))
            return bad("batched handles need tau = 1 in both components");
        if (h->p.coupling != 0)
            return bad("batched handles use the immersed-boundary coupling");
    }
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_E_NOMEM;
    b->hs.assign(handles, handles + n);
    b->st = handles[0]->st;
    b->storage = handles[0]->storage;
    b->device = handles[0]->p.device;
    b->step0.assign(n, 0);
    if (hipSetDevice(b->device) != hipSuccess ||
        hipEventCreateWithFlags(&b->start, hipEventDisableTiming) != hipSuccess ||
        hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->device) !=
            hipSuccess) {
        lbm_batch_destroy(b);
        g_init_error = "device call failed (batch)";
        return LBM_E_DEVICE;
    }
    *out = b;
    return LBM_OK;
}

extern "C" lbm_status lbm_batch_set_launch(lbm_batch *b, int32_t tile, int32_t zchunk) {
    if (!b) return LBM_E_INVAL;
    if (!((tile >= 6 && tile <= 10) || tile == TILE_ROWS) || zchunk < 0)
        return bfail(b, LBM_E_INVAL, "batch tile must be 6..10 or 13");
    if (tile == TILE_ROWS)
        for (const lbm_handle *h : b->hs)
            if (!rows_fit(h->nx))
                return bfail(b, LBM_E_INVAL, "tile 13 needs 16 <= nx <= 128 in every handle");
    b->tile = tile;
    b->zchunk = zchunk;
    b->dirty = true;
    return LBM_OK;
}

extern "C" lbm_status lbm_batch_set_parts(lbm_batch *b, int32_t parts) {
    if (!b) return LBM_E_INVAL;
    if (parts < 1 || parts > 4) return bfail(b, LBM_E_INVAL, "parts must be 1..4");
    b->nparts = parts;
    b->dirty = true;
    return LBM_OK;
}

extern "C" lbm_status lbm_batch_set_schedule(lbm_batch *b, int32_t queue) {
    if (!b) return LBM_E_INVAL;
    if (queue != 0 && queue != 1) return bfail(b, LBM_E_INVAL, "schedule must be 0 or 1");
    b->queue = queue != 0;
    free_graphs(b);   // the recorded fluid launches follow the schedule
    return LBM_OK;
}

extern "C" lbm_status lbm_batch_set_graph(lbm_batch *b, int32_t on) {
    if (!b) return LBM_E_INVAL;
    if (on != 0 && on != 1) return bfail(b, LBM_E_INVAL, "graph must be 0 or 1");
    b->use_graph = on != 0;
    return LBM_OK;
}

// one step of a part on its stream: labels / forces / spreading, fluid, node update
static void part_step(lbm_batch *b, BatchPart &pt) {
    const hipStream_t st = pt.st;
    const MGroupTotals &mt = pt.mtot;
    if (pt.nmg) {
        timed(b->prof, st, "capsule_reduce", [&] {
            launch_capsule_reduce_multi(pt.d_mtab, pt.d_mgrp, pt.nmg, mt, st);
        });
        timed(b->prof, st, "membrane", [&] { launch_membrane_multi(pt.d_mtab, pt.d_mgrp, pt.nmg, mt, st); });
        timed(b->prof, st, "window_fill", [&] {
            launch_window_fill_multi(pt.d_mtab, pt.d_mgrp, pt.nmg, mt, st);
        });
    }
    const int m = (int)pt.idx.size();
    const FluidArgs *tab = pt.d_tab + (size_t)(b->since & 1) * m;
    int *q = b->queue ? pt.d_queue : nullptr;
    timed(b->prof, st, "fluid", [&] {
        switch (b->storage) {
            case 0: launch_fluid_multi<0>(tab, pt.d_desc, m, pt.nblocks, b->tile, q, b->ncu, st); break;
            case 1: launch_fluid_multi<1>(tab, pt.d_desc, m, pt.nblocks, b->tile, q, b->ncu, st); break;
            case 2: launch_fluid_multi<2>(tab, pt.d_desc, m, pt.nblocks, b->tile, q, b->ncu, st); break;
            default: launch_fluid_multi<3>(tab, pt.d_desc, m, pt.nblocks, b->tile, q, b->ncu, st); break;
        }
    });
    if (pt.nmg)
        timed(b->prof, st, "node_update", [&] {
            launch_node_update_multi(pt.d_mtab, pt.d_mgrp, pt.nmg, mt, st);
        });
}

// enqueue n steps of every part (on the parts' streams, forked from and joined back to the
// stream ost) and advance the handles' buffer parity and step counts
static hipError_t enqueue_batch_steps(lbm_batch *b, int64_t n, hipStream_t ost) {
    hipError_t e = hipSuccess;
    bool forked = false;
    for (const BatchPart &pt : b->parts) forked = forked || pt.st != ost;
    if (forked) {   // the parts' streams start after the work already on ost
        e = hipEventRecord(b->start, ost);
        for (BatchPart &pt : b->parts)
            if (e == hipSuccess && pt.st != ost) e = hipStreamWaitEvent(pt.st, b->start, 0);
    }
    for (int64_t i = 0; i < n && e == hipSuccess; ++i) {
        for (BatchPart &pt : b->parts) part_step(b, pt);
        for (lbm_handle *h : b->hs) {
            h->cur = 1 - h->cur;
            h->step++;
        }
        b->since++;
    }
    if (forked)     // and ost continues after all of them
        for (BatchPart &pt : b->parts) {
            if (e == hipSuccess && pt.st != ost) e = hipEventRecord(pt.done, pt.st);
            if (e == hipSuccess && pt.st != ost) e = hipStreamWaitEvent(ost, pt.done, 0);
        }
    return e;
}

// capture two steps starting from buffer parity par (the current one) into gexec[par]; the
// capture only records, so the bookkeeping that enqueue_batch_steps advanced is put back
static hipError_t capture_batch_graph(lbm_batch *b, int par) {
    const int64_t since = b->since;
    std::vector<int> cur;
    std::vector<int64_t> step;
    for (const lbm_handle *h : b->hs) {
        cur.push_back(h->cur);
        step.push_back(h->step);
    }
    hipError_t e = b->gst ? hipSuccess : hipStreamCreateWithFlags(&b->gst, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    // a part that runs on the handles' stream is recorded on the capture stream instead
    std::vector<bool> moved;
    for (BatchPart &pt : b->parts) {
        moved.push_back(pt.st == b->st);
        if (pt.st == b->st) pt.st = b->gst;
    }
    e = hipStreamBeginCapture(b->gst, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t eq = enqueue_batch_steps(b, 2, b->gst);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->gst, &g);
        if (e == hipSuccess) e = eq;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec[par], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
    }
    for (size_t i = 0; i < b->parts.size(); ++i)
        if (moved[i]) b->parts[i].st = b->st;
    b->since = since;
    for (size_t i = 0; i < b->hs.size(); ++i) {
        b->hs[i]->cur = cur[i];
        b->hs[i]->step = step[i];
    }
    return e;
}

extern "C" lbm_status lbm_batch_step(lbm_batch *b, int64_t n) {
    if (!b) return LBM_E_INVAL;
    if (n < 0) return bfail(b, LBM_E_INVAL, "negative step count");
    const int ng = (int)b->hs.size();
    for (lbm_handle *h : b->hs)
        if (!h->finalized) {
            lbm_status s = finalize(h);
            if (s != LBM_OK) return bfail(b, s, h->err);
        }
    // the tables hold both buffer parities and the step stamps; a handle stepped on its
    // own since they were written needs new ones
    for (int g = 0; g < ng && !b->dirty; ++g)
        if (b->hs[g]->step != b->step0[g] + b->since) b->dirty = true;
    if (b->dirty) {
        lbm_status s = batch_tables(b);
        if (s != LBM_OK) return s;
    }
    hipError_t e = hipSuccess;
    int64_t left = n;
    if (b->use_graph && b->prof.mode == 0) {
        // pairs of steps replayed from the graph of the current buffer parity
        for (; left >= 2 && e == hipSuccess; left -= 2) {
            const int par = (int)(b->since & 1);
            if (!b->gexec[par]) e = capture_batch_graph(b, par);
            if (e == hipSuccess) e = hipGraphLaunch(b->gexec[par], b->st);
            if (e != hipSuccess) break;
            for (lbm_handle *h : b->hs) h->step += 2;   // two steps: parity unchanged
            b->since += 2;
        }
    }
    if (e == hipSuccess && left > 0) e = enqueue_batch_steps(b, left, b->st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("batch step: ") + hipGetErrorString(e));
    return LBM_OK;
}

extern "C" lbm_status lbm_batch_autotune(lbm_batch *b, int32_t reps, int32_t *tile,
                                         int32_t *zchunk, double *fluid_ms) {
    if (!b) return LBM_E_INVAL;
    if (reps < 1 || reps > 1000) return bfail(b, LBM_E_INVAL, "reps must be 1..1000");
    const int ng = (int)b->hs.size();
    for (lbm_handle *h : b->hs)
        if (!h->finalized) {
            lbm_status s = finalize(h);
            if (s != LBM_OK) return bfail(b, s, h->err);
        }
    auto dev = [&](hipError_t e) { return e == hipSuccess; };
    std::vector<int> saved((size_t)ng * ST_WORDS);
    if (!dev(hipStreamSynchronize(b->st))) return bfail(b, LBM_E_DEVICE, "stream synchronisation failed");
    for (BatchPart &pt : b->parts)
        if (!dev(hipStreamSynchronize(pt.st))) return bfail(b, LBM_E_DEVICE, "stream synchronisation failed");
    for (int g = 0; g < ng; ++g)
        if (!dev(hipMemcpy(&saved[(size_t)g * ST_WORDS], b->hs[g]->status, ST_WORDS * sizeof(int),
                           hipMemcpyDeviceToHost)))
            return bfail(b, LBM_E_DEVICE, "status copy failed");
    EventPair ev;
    if (!dev(ev.make())) return bfail(b, LBM_E_DEVICE, "event creation failed");
    bool rows = true;
    for (const lbm_handle *h : b->hs) rows = rows && rows_fit(h->nx);
    const int tiles[] = {6, 7, 8, 9, 10, TILE_ROWS};
    double best = INFINITY;
    int bt = b->tile, bz = b->zchunk;
    for (int t : tiles) {
        if (t == TILE_ROWS && !rows) continue;
        for (int z : TUNE_ZC) {
            b->tile = t;
            b->zchunk = z;
            lbm_status s = batch_tables(b);   // per-part z-chunk and block tables of this shape
            if (s != LBM_OK) return s;
            double ms = 0.0;
            hipError_t e = time_launches(b->st, reps, ev.a, ev.b, [&] {
                for (BatchPart &pt : b->parts) {
                    const int m = (int)pt.idx.size();
                    int *q = b->queue ? pt.d_queue : nullptr;
                    switch (b->storage) {
                        case 0: launch_fluid_multi<0>(pt.d_tab, pt.d_desc, m, pt.nblocks, t, q, b->ncu, b->st); break;
                        case 1: launch_fluid_multi<1>(pt.d_tab, pt.d_desc, m, pt.nblocks, t, q, b->ncu, b->st); break;
                        case 2: launch_fluid_multi<2>(pt.d_tab, pt.d_desc, m, pt.nblocks, t, q, b->ncu, b->st); break;
                        default: launch_fluid_multi<3>(pt.d_tab, pt.d_desc, m, pt.nblocks, t, q, b->ncu, b->st); break;
                    }
                }
            }, &ms);
            if (e != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("batch autotune: ") + hipGetErrorString(e));
            if (ms < best) {
                best = ms;
                bt = t;
                bz = z;
            }
        }
    }
    for (int g = 0; g < ng; ++g)
        if (!dev(hipMemcpy(b->hs[g]->status, &saved[(size_t)g * ST_WORDS], ST_WORDS * sizeof(int),
                           hipMemcpyHostToDevice)))
            return bfail(b, LBM_E_DEVICE, "status copy failed");
    b->tile = bt;
    b->zchunk = bz;
    b->dirty = true;
    if (tile) *tile = bt;
    if (zchunk) *zchunk = bz;
    if (fluid_ms) *fluid_ms = best;
    return LBM_OK;
}

extern "C" lbm_status lbm_batch_set_profiling(lbm_batch *b, int32_t on) {
    if (!b) return LBM_E_INVAL;
    if (on < 0 || on > 2) return bfail(b, LBM_E_INVAL, "profiling mode must be 0, 1 or 2");
    b->prof.mode = on;
    return LBM_OK;
}

extern "C" lbm_status lbm_batch_kernel_stats(lbm_batch *b, lbm_kernel_stat *out, int32_t max,
                                             int32_t *n) {
    if (!b || !n || (max > 0 && !out)) return LBM_E_INVAL;
    bool ok = hipStreamSynchronize(b->st) == hipSuccess;
    for (BatchPart &pt : b->parts) ok = ok && hipStreamSynchronize(pt.st) == hipSuccess;
    if (!ok) return bfail(b, LBM_E_DEVICE, "stream synchronisation failed");
    *n = export_timers(b->prof, out, max);
    return LBM_OK;
}

extern "C" const char *lbm_batch_last_error(const lbm_batch *b) {
    return b ? b->err.c_str() : g_init_error.c_str();
}

extern "C" void lbm_batch_destroy(lbm_batch *b) {
    if (!b) return;
    if (b->st) (void)hipStreamSynchronize(b->st);
    free_parts(b);
    if (b->gst) {
        (void)hipStreamSynchronize(b->gst);
        (void)hipStreamDestroy(b->gst);
    }
    if (b->start) (void)hipEventDestroy(b->start);
    free_prof(b->prof);
    delete b;
}

static lbm_status check_status(lbm_handle *h, int st[ST_WORDS]) {
    HIPCHK(h, hipMemcpyAsync(st, h->status, ST_WORDS * sizeof(int), hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return LBM_OK;
}

static bool unstable_flagged(const int *st) {
    return st[ST_UNSTABLE] || st[ST_OVERFLOW] || st[ST_WIDE] || st[ST_SLAB] ||
           st[ST_BBOVER];
}

static const char *unstable_message(const int *st) {
    if (st[ST_BBOVER]) return "bounce-back link list or triangle bins overflowed (deformed capsule)";
    if (st[ST_SLAB]) return "capsule window crossed a wall layer of its slab";
    if (st[ST_WIDE]) return "capsule window wider than 2048 lattice columns (x * y)";
    if (st[ST_OVERFLOW]) return "capsule outgrew its window";
    return "non-finite or negative density";
}

extern "C" lbm_status lbm_sync(lbm_handle *h) {
    if (!h) return LBM_E_INVAL;
    int st[ST_WORDS];
    lbm_status s = check_status(h, st);
    if (s != LBM_OK) return s;
    if (unstable_flagged(st)) return fail(h, LBM_E_UNSTABLE, unstable_message(st));
    return LBM_OK;
}

// ------------------------------------------------------------------------------------
// Observables
// ------------------------------------------------------------------------------------
static void launch_rho_any(lbm_handle *h, float *dst) {
    const float s0 = shift_of(h, 0), s1 = shift_of(h, 1);
    switch (h->storage) {
        case 0: launch_rho<0>(h->f[h->cur], dst, h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, nullptr, h->st); break;
        case 1: launch_rho<1>(h->f[h->cur], dst, h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, nullptr, h->st); break;
        case 2: launch_rho<2>(h->f[h->cur], dst, h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, nullptr, h->st); break;
        default: launch_rho<3>(h->f[h->cur], dst, h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, h->rsite[h->cur], h->st); break;
    }
}

extern "C" lbm_status lbm_observables(lbm_handle *h, lbm_obs *out) {
    if (!h || !out) return LBM_E_INVAL;
    const float s0 = shift_of(h, 0), s1 = shift_of(h, 1);
    switch (h->storage) {
        case 0: launch_moments<0>(h->f[h->cur], h->partial, h->mom_blocks, h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, nullptr, h->st); break;
        case 1: launch_moments<1>(h->f[h->cur], h->partial, h->mom_blocks, h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, nullptr, h->st); break;
        case 2: launch_moments<2>(h->f[h->cur], h->partial, h->mom_blocks, h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, nullptr, h->st); break;
        default: launch_moments<3>(h->f[h->cur], h->partial, h->mom_blocks, h->nx, h->ny, h->nz, h->wall, h->lz, s0, s1, h->rsite[h->cur], h->st); break;
    }
    HIPCHK(h, hipGetLastError());
    std::vector<double> part((size_t)h->nslab * h->mom_blocks * 5);
    HIPCHK(h, hipMemcpyAsync(part.data(), h->partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, h->st));
    if (out->rho || out->meniscus) {
        launch_rho_any(h, h->rho_tmp);
        HIPCHK(h, hipGetLastError());
        if (out->rho)
            HIPCHK(h, hipMemcpyAsync(out->rho, h->rho_tmp, 2 * (size_t)h->N * sizeof(float), hipMemcpyDeviceToHost, h->st));
        if (out->meniscus) {
            launch_meniscus(h->rho_tmp, h->flag, h->men_tmp, h->nx, h->ny, h->nz, h->wall, h->lz, h->st);
            HIPCHK(h, hipGetLastError());
            HIPCHK(h, hipMemcpyAsync(out->meniscus, h->men_tmp, (size_t)h->nx * h->ny * h->nslab * sizeof(float), hipMemcpyDeviceToHost, h->st));
        }
    }
    int st[ST_WORDS];
    lbm_status s = check_status(h, st);
    if (s != LBM_OK) return s;
    lbm_summary &sm = out->summary;
    std::memset(&sm, 0, sizeof sm);
    for (int sl = 0; sl < h->nslab; ++sl) {
        double ms[2] = {0.0, 0.0};
        for (int b = sl * h->mom_blocks; b < (sl + 1) * h->mom_blocks; ++b) {
            ms[0] += part[5 * b];
            ms[1] += part[5 * b + 1];
            for (int d = 0; d < 3; ++d) sm.momentum[d] += part[5 * b + 2 + d];
        }
        sm.mass[0] += ms[0];
        sm.mass[1] += ms[1];
        if (out->slab_mass) {
            out->slab_mass[2 * sl] = ms[0];
            out->slab_mass[2 * sl + 1] = ms[1];
        }
    }
    sm.step = h->step;
    sm.lost_reaction = st[ST_LOST];
    sm.lost_links = st[ST_BBLOST];
    sm.n_capsules = (int)h->caps.size();
    sm.unstable = unstable_flagged(st) ? 1 : 0;
    if (h->finalized && !h->caps.empty()) {
        const bool bb = h->p.coupling == 1;
        std::vector<double4> X(h->ntot), V(bb ? h->ntot : 0);
        std::vector<float4> Fh(h->ntot), R(h->ntot), Pp(bb ? h->ntot : 0), Ff(bb ? h->ntot : 0);
        std::vector<CapState> cs(h->caps.size());
        std::vector<int> nl(bb ? h->caps.size() : 0);
        HIPCHK(h, hipMemcpy(X.data(), h->d_X, X.size() * sizeof(double4), hipMemcpyDeviceToHost));
        HIPCHK(h, hipMemcpy(Fh.data(), h->d_Fh, Fh.size() * sizeof(float4), hipMemcpyDeviceToHost));
        HIPCHK(h, hipMemcpy(R.data(), h->d_R, R.size() * sizeof(float4), hipMemcpyDeviceToHost));
        HIPCHK(h, hipMemcpy(cs.data(), h->d_cst, cs.size() * sizeof(CapState), hipMemcpyDeviceToHost));
        if (bb) {
            HIPCHK(h, hipMemcpy(V.data(), h->d_V, V.size() * sizeof(double4), hipMemcpyDeviceToHost));
            HIPCHK(h, hipMemcpy(Pp.data(), h->d_pprev, Pp.size() * sizeof(float4), hipMemcpyDeviceToHost));
            HIPCHK(h, hipMemcpy(Ff.data(), h->d_ffl, Ff.size() * sizeof(float4), hipMemcpyDeviceToHost));
            HIPCHK(h, hipMemcpy(nl.data(), h->d_nlinks + h->caps.size(), nl.size() * sizeof(int),
                                hipMemcpyDeviceToHost));
            for (int v : nl) sm.links += v;
        }
        for (size_t k = 0; k < h->caps.size(); ++k) {
            const CapDev &cd = h->h_caps[k];
            double cen[3] = {0, 0, 0}, fr[3] = {0, 0, 0}, fh[3] = {0, 0, 0}, ff[3] = {0, 0, 0};
            for (int i = 0; i < cd.nn; ++i) {
                const double4 x = X[cd.node0 + i];
                cen[0] += x.x; cen[1] += x.y; cen[2] += x.z;
                fr[0] += R[cd.node0 + i].x; fr[1] += R[cd.node0 + i].y; fr[2] += R[cd.node0 + i].z;
                fh[0] += Fh[cd.node0 + i].x; fh[1] += Fh[cd.node0 + i].y; fh[2] += Fh[cd.node0 + i].z;
                if (bb) {
                    const float4 p = Pp[cd.node0 + i], f = Ff[cd.node0 + i];
                    const double4 v = V[cd.node0 + i];
                    // half of the last exchange is still to be applied
                    sm.pending[0] += 0.5 * p.x; sm.pending[1] += 0.5 * p.y; sm.pending[2] += 0.5 * p.z;
                    sm.node_momentum[0] += h->p.node_mass * v.x;
                    sm.node_momentum[1] += h->p.node_mass * v.y;
                    sm.node_momentum[2] += h->p.node_mass * v.z;
                    ff[0] += f.x; ff[1] += f.y; ff[2] += f.z;
                }
            }
            for (int d = 0; d < 3; ++d) {
                cen[d] /= cd.nn;
                if (!bb) {
                    sm.pending[d] += fr[d];
                    ff[d] = fr[d];
                }
            }
            if (out->capsules) {
                lbm_capsule_obs &o = out->capsules[k];
                const HostCap &hc = h->caps[k];
                double vol = 0.0;
                for (int t = 0; t < cd.nt; ++t) {
                    const double4 A = X[cd.node0 + hc.tri[3 * t]], B = X[cd.node0 + hc.tri[3 * t + 1]],
                                  C = X[cd.node0 + hc.tri[3 * t + 2]];
                    const double a[3] = {A.x - cen[0], A.y - cen[1], A.z - cen[2]};
                    const double b[3] = {B.x - cen[0], B.y - cen[1], B.z - cen[2]};
                    const double c[3] = {C.x - cen[0], C.y - cen[1], C.z - cen[2]};
                    vol += (a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
                            a[2] * (b[0] * c[1] - b[1] * c[0])) / 6.0;
                }
                o.volume = vol;
                for (int d = 0; d < 3; ++d) {
                    o.centroid[d] = cen[d];
                    o.f_capillary[d] = fr[d];
                    o.f_hertz[d] = fh[d];
                    o.f_fluid[d] = ff[d];
                    // the anchor of the last step acted at its centroid cs.cen
                    o.f_anchor[d] = (h->step > 0 && hc.p.anchor_k != 0.0)
                                        ? hc.p.anchor_k * (cs[k].cen[d] - cd.c0[d]) : 0.0;
                }
            }
        }
    } else if (out->capsules) {
        for (size_t k = 0; k < h->caps.size(); ++k) std::memset(&out->capsules[k], 0, sizeof(lbm_capsule_obs));
    }
    if (sm.unstable) return fail(h, LBM_E_UNSTABLE, unstable_message(st));
    return LBM_OK;
}

extern "C" lbm_status lbm_rho_device(lbm_handle *h, float *rho_device) {
    if (!h || !rho_device) return LBM_E_INVAL;
    launch_rho_any(h, rho_device);
    HIPCHK(h, hipGetLastError());
    return LBM_OK;
}

extern "C" lbm_status lbm_capsule_nodes(lbm_handle *h, int32_t k, double *xyz) {
    if (!h || !xyz || k < 0 || k >= (int)h->caps.size()) return LBM_E_INVAL;
    const HostCap &c = h->caps[k];
    const int nn = (int)c.x0.size() / 3;
    if (!h->finalized) {
        std::memcpy(xyz, c.x0.data(), 3 * nn * sizeof(double));
        return LBM_OK;
    }
    std::vector<double4> X(nn);
    HIPCHK(h, hipStreamSynchronize(h->st));
    HIPCHK(h, hipMemcpy(X.data(), h->d_X + h->h_caps[k].node0, nn * sizeof(double4), hipMemcpyDeviceToHost));
    for (int i = 0; i < nn; ++i) {
        xyz[3 * i] = X[i].x;
        xyz[3 * i + 1] = X[i].y;
        xyz[3 * i + 2] = X[i].z;
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_labels(lbm_handle *h, uint8_t *out) {
    if (!h || !out) return LBM_E_INVAL;
    HIPCHK(h, hipStreamSynchronize(h->st));
    HIPCHK(h, hipMemcpy(out, h->flag, (size_t)h->N, hipMemcpyDeviceToHost));
    const int plane = h->nx * h->ny;
    for (int s = 0; s < h->N; ++s) out[s] &= LABEL_MASK;
    if (h->wall)
        for (int sl = 0; sl < h->nslab; ++sl)
            std::memset(out + (size_t)sl * h->lz * plane, 255, (size_t)plane);
    return LBM_OK;
}

// ------------------------------------------------------------------------------------
// Checkpoints
// ------------------------------------------------------------------------------------
namespace {
// version 3: slab height in the header; version 4: previous window in the capsule state
constexpr int32_t CKPT_VERSION = 4;
struct CkptHeader {
    char magic[8];
    int32_t version, nx, ny, nz, storage, ncap, ntot, lz;
    int64_t step;
};
}  // namespace

extern "C" lbm_status lbm_save(lbm_handle *h, const char *path) {
    if (!h || !path) return LBM_E_INVAL;
    if (!h->finalized) {
        lbm_status s = finalize(h);
        if (s != LBM_OK) return s;
    }
    HIPCHK(h, hipStreamSynchronize(h->st));
    const size_t fbytes = 2 * (size_t)Q * h->N * h->esize;
    std::vector<char> f(fbytes);
    HIPCHK(h, hipMemcpy(f.data(), h->f[h->cur], fbytes, hipMemcpyDeviceToHost));
    std::vector<double4> X(h->ntot);
    std::vector<float4> R(h->ntot);
    std::vector<CapState> cs(h->caps.size());
    if (h->ntot) {
        HIPCHK(h, hipMemcpy(X.data(), h->d_X, X.size() * sizeof(double4), hipMemcpyDeviceToHost));
        HIPCHK(h, hipMemcpy(R.data(), h->d_R, R.size() * sizeof(float4), hipMemcpyDeviceToHost));
        HIPCHK(h, hipMemcpy(cs.data(), h->d_cst, cs.size() * sizeof(CapState), hipMemcpyDeviceToHost));
    }
    FILE *fp = std::fopen(path, "wb");
    if (!fp) return fail(h, LBM_E_INVAL, std::string("cannot open ") + path);
    CkptHeader hd{};
    std::memcpy(hd.magic, "LBMXCKP", 8);
    hd.version = CKPT_VERSION; hd.nx = h->nx; hd.ny = h->ny; hd.nz = h->nz; hd.storage = h->storage;
    hd.ncap = (int)h->caps.size(); hd.ntot = h->ntot; hd.lz = h->lz; hd.step = h->step;
    bool ok = std::fwrite(&hd, sizeof hd, 1, fp) == 1 && std::fwrite(f.data(), 1, fbytes, fp) == fbytes;
    if (h->storage == LBM_STORE_F16_LOCAL) {   // the site densities the populations are shifted by
        std::vector<float> r(2 * (size_t)h->N);
        ok = ok && hipMemcpy(r.data(), h->rsite[h->cur], r.size() * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess &&
             std::fwrite(r.data(), sizeof(float), r.size(), fp) == r.size();
    }
    if (h->ntot)
        ok = ok && std::fwrite(X.data(), sizeof(double4), X.size(), fp) == X.size() &&
             std::fwrite(R.data(), sizeof(float4), R.size(), fp) == R.size() &&
             std::fwrite(cs.data(), sizeof(CapState), cs.size(), fp) == cs.size();
    if (h->ntot && h->p.coupling == 1) {
        // bounce-back: node velocities and the exchanged momentum still to act
        std::vector<double4> V(h->ntot);
        std::vector<float4> Pp(h->ntot);
        ok = ok && hipMemcpy(V.data(), h->d_V, V.size() * sizeof(double4), hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(Pp.data(), h->d_pprev, Pp.size() * sizeof(float4), hipMemcpyDeviceToHost) == hipSuccess &&
             std::fwrite(V.data(), sizeof(double4), V.size(), fp) == V.size() &&
             std::fwrite(Pp.data(), sizeof(float4), Pp.size(), fp) == Pp.size();
    }
    ok = (std::fclose(fp) == 0) && ok;
    return ok ? LBM_OK : fail(h, LBM_E_INVAL, "checkpoint write failed");
}

extern "C" lbm_status lbm_load(lbm_handle *h, const char *path) {
    if (!h || !path) return LBM_E_INVAL;
    if (!h->finalized) {
        lbm_status s = finalize(h);
        if (s != LBM_OK) return s;
    }
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return fail(h, LBM_E_INVAL, std::string("cannot open ") + path);
    CkptHeader hd{};
    const size_t fbytes = 2 * (size_t)Q * h->N * h->esize;
    std::vector<char> f(fbytes);
    std::vector<double4> X(h->ntot);
    std::vector<float4> R(h->ntot);
    std::vector<CapState> cs(h->caps.size());
    bool ok = std::fread(&hd, sizeof hd, 1, fp) == 1 && std::memcmp(hd.magic, "LBMXCKP", 8) == 0 &&
              hd.version == CKPT_VERSION && hd.nx == h->nx && hd.ny == h->ny && hd.nz == h->nz &&
              hd.storage == h->storage && hd.ncap == (int)h->caps.size() && hd.ntot == h->ntot &&
              hd.lz == h->lz &&
              std::fread(f.data(), 1, fbytes, fp) == fbytes;
    std::vector<float> rs(h->storage == LBM_STORE_F16_LOCAL ? 2 * (size_t)h->N : 0);
    if (ok && !rs.empty()) ok = std::fread(rs.data(), sizeof(float), rs.size(), fp) == rs.size();
    if (ok && h->ntot)
        ok = std::fread(X.data(), sizeof(double4), X.size(), fp) == X.size() &&
             std::fread(R.data(), sizeof(float4), R.size(), fp) == R.size() &&
             std::fread(cs.data(), sizeof(CapState), cs.size(), fp) == cs.size();
    const bool bb = h->ntot && h->p.coupling == 1;
    std::vector<double4> V(bb ? h->ntot : 0);
    std::vector<float4> Pp(bb ? h->ntot : 0);
    if (ok && bb)
        ok = std::fread(V.data(), sizeof(double4), V.size(), fp) == V.size() &&
             std::fread(Pp.data(), sizeof(float4), Pp.size(), fp) == Pp.size();
    if (ok) ok = std::fgetc(fp) == EOF;   // nothing left over: the same coupling wrote it
    std::fclose(fp);
    if (!ok) return fail(h, LBM_E_INVAL, "checkpoint does not match this simulation");
    HIPCHK(h, hipStreamSynchronize(h->st));
    HIPCHK(h, hipMemcpy(h->f[h->cur], f.data(), fbytes, hipMemcpyHostToDevice));
    if (!rs.empty()) HIPCHK(h, hipMemcpy(h->rsite[h->cur], rs.data(), rs.size() * sizeof(float), hipMemcpyHostToDevice));
    // every site flag is rebuilt by the next step; windows recorded in cs are cleared
    HIPCHK(h, hipMemset(h->flag, 0, (size_t)h->N));
    if (h->ntot) {
        HIPCHK(h, hipMemcpy(h->d_X, X.data(), X.size() * sizeof(double4), hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(h->d_R, R.data(), R.size() * sizeof(float4), hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(h->d_cst, cs.data(), cs.size() * sizeof(CapState), hipMemcpyHostToDevice));
    }
    if (bb) {
        HIPCHK(h, hipMemcpy(h->d_V, V.data(), V.size() * sizeof(double4), hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(h->d_pprev, Pp.data(), Pp.size() * sizeof(float4), hipMemcpyHostToDevice));
        HIPCHK(h, hipMemset(h->d_pex, 0, 3 * (size_t)h->ttot * sizeof(long long)));
        HIPCHK(h, hipMemset(h->d_rsc, 0, 3 * (size_t)h->ttot * sizeof(long long)));
        HIPCHK(h, hipMemset(h->d_nlinks, 0, 2 * h->caps.size() * sizeof(int)));
    }
    if (h->ntot)   // crossing masks of windows this handle used before the load
        HIPCHK(h, hipMemset(h->d_marks, 0, h->caps.size() * ROWS_MAX * sizeof(unsigned long long)));
    HIPCHK(h, hipMemset(h->status, 0, ST_WORDS * sizeof(int)));
    h->step = hd.step;
    return LBM_OK;
}

// ------------------------------------------------------------------------------------
// Profiling and misc
// ------------------------------------------------------------------------------------
extern "C" lbm_status lbm_set_profiling(lbm_handle *h, int32_t on) {
    if (!h) return LBM_E_INVAL;
    if (on < 0 || on > 2) return fail(h, LBM_E_INVAL, "profiling mode must be 0, 1 or 2");
    h->prof.mode = on;
    return LBM_OK;
}

extern "C" lbm_status lbm_kernel_stats(lbm_handle *h, lbm_kernel_stat *out, int32_t max,
                                       int32_t *n) {
    if (!h || !n || (max > 0 && !out)) return LBM_E_INVAL;
    HIPCHK(h, hipStreamSynchronize(h->st));
    *n = export_timers(h->prof, out, max);
    return LBM_OK;
}

extern "C" double lbm_bytes_per_site(const lbm_handle *h) {
    // storage 3 also reads and writes the FP32 density of both components per site
    return h ? 2.0 * Q * 2.0 * (double)h->esize +
                   (h->storage == LBM_STORE_F16_LOCAL ? 2.0 * 2.0 * 4.0 : 0.0)
             : 0.0;
}

extern "C" int64_t lbm_fluid_sites(const lbm_handle *h) {
    return h ? (int64_t)h->nx * h->ny * (h->nz - h->wall * h->nslab) : 0;
}

extern "C" const char *lbm_last_error(const lbm_handle *h) {
    return h ? h->err.c_str() : g_init_error.c_str();
}

extern "C" void lbm_destroy(lbm_handle *h) {
    if (!h) return;
    if (h->st) (void)hipStreamSynchronize(h->st);
    free_all(h);
    delete h;
}
