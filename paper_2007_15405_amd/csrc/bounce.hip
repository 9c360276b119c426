// bounce.hip -- the fluid-membrane coupling of Section 3.1: half-way bounce-back on the
// moving triangulated membrane with Ladd's momentum exchange, the homogeneous weighting of
// the three nodes of the crossed element, the exchanged momentum spread over two
// consecutive steps, and Newtonian membrane nodes of mass m (25 rho0 in Section 3.2).
//
// Per step, after the capsule reduction (window), the membrane forces and the side labels:
//   k_bb_tri / k_bb_bins: the triangles of each capsule binned into the unit cells of its
//     window (their cell ranges per triangle, then a counting sort in LDS, one workgroup
//     per capsule);
//   k_bb_find: every link from a site inside capsule k to a fluid site of another side
//     (exterior, or a capsule of higher index) is appended to the capsule's link list;
//   k_bb_resolve: 8 lanes per link find its triangle (among the triangles whose bounding
//     box meets the link's, the least miss distance, lowest index on ties) and the
//     densities of both sites before any population is changed;
//   k_bb_swap: the bounce-back on the post-collision populations in place, so that plain
//     pull streaming delivers f_q(b) = f*_qbar(b) + delta and f_qbar(a) = f*_q(a) - delta,
//     delta = 2 w_q rho u_b . e_q / c_s^2 (rho the link-mean density of the component, u_b
//     the mean velocity of the triangle's nodes); the exchanged momentum
//     (2 f*_q(a) - 2 f*_qbar(b) - 2 delta) e_q goes a third to each node of the triangle;
//   (the fluid step)
//   k_bb_reaction: the Shan-Chen force across each link, from the densities and psi the
//     fluid step used (stored on window sites) with the same substitution, returned to
//     the triangle the same way;
//   k_bb_nodes: v += (F_membrane + (P_ex(n) + P_ex(n-1)) / 2 + R_sc) / m, x += v.
// Node sums are 64-bit fixed point (2^-40), so they do not depend on the order of the
// atomic adds.  Decisions (labels, triangle choice) use the FP32-rounded node positions
// evaluated in double without contraction of multiply-adds.
#include "lbm_internal.h"

namespace lbmx {

namespace {

__device__ __forceinline__ int wrapb(int a, int n) {
    a %= n;
    return a < 0 ? a + n : a;
}

__device__ __forceinline__ long long fix40(float v) {
    return (long long)__builtin_rint((double)v * 1099511627776.0);   // 2^40
}
__device__ __forceinline__ float unfix40(long long v) {
    return (float)((double)v * (1.0 / 1099511627776.0));
}

// six times the signed volume of the tetrahedron (a, b, c, d)
__device__ double orient3(const double *a, const double *b, const double *c, const double *d) {
#pragma clang fp contract(off)
    double ab[3], ac[3], ad[3];
    for (int k = 0; k < 3; ++k) {
        ab[k] = b[k] - a[k];
        ac[k] = c[k] - a[k];
        ad[k] = d[k] - a[k];
    }
    return ab[0] * (ac[1] * ad[2] - ac[2] * ad[1]) + ab[1] * (ac[2] * ad[0] - ac[0] * ad[2]) +
           ab[2] * (ac[0] * ad[1] - ac[1] * ad[0]);
}

// miss distance of the segment p0 -> p1 from triangle (a, b, c): 0 when they meet, else
// max(-u, -v, -w, -t, t - 1), u, v, w the barycentric coordinates of the segment's line in
// the triangle's plane and t the segment parameter there; +inf for a parallel line
__device__ double miss_distance(const double *p0, const double *p1, const double *a,
                                const double *b, const double *c) {
#pragma clang fp contract(off)
    const double s0 = orient3(a, b, c, p0), s1 = orient3(a, b, c, p1);
    const double den = s0 - s1;
    if (den == 0.0) return __builtin_inf();
    const double t = s0 / den;
    const double wa = orient3(p0, p1, b, c), wb = orient3(p0, p1, c, a), wc = orient3(p0, p1, a, b);
    const double sum = wa + wb + wc;
    if (sum == 0.0) return __builtin_inf();
    const double u = wa / sum, v = wb / sum, w = wc / sum;
    double d = 0.0;
    if (-u > d) d = -u;
    if (-v > d) d = -v;
    if (-w > d) d = -w;
    if (-t > d) d = -t;
    if (t - 1.0 > d) d = t - 1.0;
    return d;
}

__device__ __forceinline__ void tri_vertices(const BBArgs &b, int t, double (&v)[3][3]) {
    const int4 tr = b.tri[t];
    const double4 P[3] = {b.X[tr.x], b.X[tr.y], b.X[tr.z]};
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        v[m][0] = (double)(float)P[m].x;
        v[m][1] = (double)(float)P[m].y;
        v[m][2] = (double)(float)P[m].z;
    }
}

template <int S>
__device__ __forceinline__ float popl(const void *f, int c, int q, int N, int s, float sh) {
    using T = typename Codec<S>::T;
    return Codec<S>::dec(((const T *)f)[(size_t)(c * Q + q) * N + s], wq(q) * sh);
}
template <int S>
__device__ __forceinline__ void pops(void *f, int c, int q, int N, int s, float v, float sh) {
    using T = typename Codec<S>::T;
    ((T *)f)[(size_t)(c * Q + q) * N + s] = Codec<S>::enc(v, wq(q) * sh);
}

}  // namespace

// ------------------------------------------------------------------------------------
// Triangle bins
// ------------------------------------------------------------------------------------
// the window cells (first and last per axis) that the box of a triangle with vertices v
// covers; false for a triangle wider than BB_SPAN cells or outside the window
__device__ __forceinline__ bool tri_cells(const BBArgs &b, const double (&v)[3][3], int k, int (&c0)[3],
                                          int (&c1)[3]) {
    const CapState cs = b.cst[k];
    for (int d = 0; d < 3; ++d) {
        const double lo = fmin(v[0][d], fmin(v[1][d], v[2][d]));
        const double hi = fmax(v[0][d], fmax(v[1][d], v[2][d]));
        if (!(hi - lo <= (double)(BB_SPAN - 1))) return false;
        c0[d] = max((int)floor(lo) - cs.lo[d], 0);
        c1[d] = min((int)floor(hi) - cs.lo[d], cs.dim[d] - 1);
        if (c0[d] > c1[d]) return false;
    }
    return true;
}

// one thread per triangle: its FP32-rounded vertices, compact for the link search, and the
// window cells its box covers, packed into one word for the sort
static_assert(GMAX <= 64 && BB_SPAN <= 4, "cell ranges are packed into 6 + 2 bits per axis");
__global__ void __launch_bounds__(256) k_bb_tri(BBArgs b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.ttot) return;
    double v[3][3];
    tri_vertices(b, t, v);
#pragma unroll
    for (int m = 0; m < 3; ++m)
        b.tpos[3 * (size_t)t + m] = make_float4((float)v[m][0], (float)v[m][1], (float)v[m][2], 0.f);
    int c0[3], c1[3];
    int packed = -1;
    if (tri_cells(b, v, b.tri[t].w, c0, c1))
        packed = c0[0] | c0[1] << 6 | c0[2] << 12 | (c1[0] - c0[0]) << 18 | (c1[1] - c0[1]) << 20 |
                 (c1[2] - c0[2]) << 22;
    else
        atomicOr(&b.status[ST_BBOVER], 1);
    b.tcell[t] = packed;
    // this step's momentum exchange and reaction through the triangle start from zero
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        b.pex[3 * (size_t)t + d] = 0;
        b.rsc[3 * (size_t)t + d] = 0;
    }
}

// one workgroup per capsule: a counting sort of the capsule's triangles into the unit
// cells of its window.  The cell counters are in LDS; a window of more than BB_LDS_CELLS
// cells is sorted in passes over cell ranges, each pass counting, scanning and filling its
// range.  The entries of one cell come in no fixed order: the link search takes the least
// (distance, index) over them, which does not depend on it.
constexpr int BB_BIN_BLK = 1024;
constexpr int BB_LDS_CELLS = 16384;   // 64 KB of counters
constexpr int BB_BIN_TB = 8;          // triangles per thread whose ranges are loaded together

// the cells of triangle range word w that fall in [p0, p0 + n), in window order, relative to p0
template <typename Fn>
__device__ __forceinline__ void for_cells(int w, int dx, int dy, int p0, int n, Fn &&fn) {
    const int x0 = w & 63, y0 = (w >> 6) & 63, z0 = (w >> 12) & 63;
    const int ex = (w >> 18) & 3, ey = (w >> 20) & 3, ez = (w >> 22) & 3;
    for (int z = z0; z <= z0 + ez; ++z)
        for (int y = y0; y <= y0 + ey; ++y)
            for (int x = x0; x <= x0 + ex; ++x) {
                const int cell = (z * dy + y) * dx + x - p0;
                if (cell >= 0 && cell < n) fn(cell);
            }
}

__global__ void __launch_bounds__(BB_BIN_BLK) k_bb_bins(BBArgs b) {
    const int k = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const CapState cs = b.cst[k];
    const CapDev cd = b.caps[k];
    const int dx = cs.dim[0], dy = cs.dim[1], ncell = dx * dy * cs.dim[2];
    const int lmax = BB_PER_TRI * cd.nt;
    int *st = b.bstart + (size_t)k * (GMAX3 + 1);
    int *list = b.blist + (size_t)BB_PER_TRI * cd.tri0;
    const int *tc = b.tcell + cd.tri0;
    __shared__ int s_cnt[BB_LDS_CELLS];
    __shared__ int s_wsum[BB_BIN_BLK / 64];
    int base = 0;   // entries of the cells before this pass
    for (int p0 = 0; p0 < ncell; p0 += BB_LDS_CELLS) {   // uniform over the block
        const int n = min(BB_LDS_CELLS, ncell - p0);
        for (int i = tid; i < n; i += BB_BIN_BLK) s_cnt[i] = 0;
        __syncthreads();
        for (int t0 = 0; t0 < cd.nt; t0 += BB_BIN_TB * BB_BIN_BLK) {
            int w[BB_BIN_TB];
#pragma unroll
            for (int u = 0; u < BB_BIN_TB; ++u) {
                const int t = t0 + tid + u * BB_BIN_BLK;
                w[u] = t < cd.nt ? tc[t] : -1;
            }
#pragma unroll
            for (int u = 0; u < BB_BIN_TB; ++u)
                if (w[u] >= 0) for_cells(w[u], dx, dy, p0, n, [&](int c) { atomicAdd(&s_cnt[c], 1); });
        }
        __syncthreads();
        // exclusive scan of the pass's counts: each thread sums a contiguous run, the run
        // sums are scanned over the lanes and then over the waves
        const int per = (n + BB_BIN_BLK - 1) / BB_BIN_BLK;
        const int q0 = min(tid * per, n), q1 = min(q0 + per, n);
        int local = 0;
        for (int i = q0; i < q1; ++i) local += s_cnt[i];
        int incl = local;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        if (lane == 63) s_wsum[wid] = incl;
        __syncthreads();
        int run = base + incl - local, total = 0;
        for (int w = 0; w < BB_BIN_BLK / 64; ++w) {
            if (w < wid) run += s_wsum[w];
            total += s_wsum[w];
        }
        for (int i = q0; i < q1; ++i) {
            const int c = s_cnt[i];
            s_cnt[i] = run;
            run += c;
        }
        __syncthreads();
        for (int i = tid; i < n; i += BB_BIN_BLK) st[p0 + i] = s_cnt[i];
        __syncthreads();   // the starts are read before the fill moves the cursors
        for (int t0 = 0; t0 < cd.nt; t0 += BB_BIN_TB * BB_BIN_BLK) {
            int w[BB_BIN_TB];
#pragma unroll
            for (int u = 0; u < BB_BIN_TB; ++u) {
                const int t = t0 + tid + u * BB_BIN_BLK;
                w[u] = t < cd.nt ? tc[t] : -1;
            }
#pragma unroll
            for (int u = 0; u < BB_BIN_TB; ++u) {
                const int t = cd.tri0 + t0 + tid + u * BB_BIN_BLK;
                if (w[u] >= 0)
                    for_cells(w[u], dx, dy, p0, n, [&](int c) {
                        const int pos = atomicAdd(&s_cnt[c], 1);
                        if (pos < lmax) list[pos] = t;
                    });
            }
        }
        base += total;
        __syncthreads();   // the next pass clears the counters and rewrites the wave sums
    }
    if (tid == 0) {
        st[ncell] = base;
        if (base > lmax) atomicOr(&b.status[ST_BBOVER], 1);
    }
}

// ------------------------------------------------------------------------------------
// Links and bounce-back
// ------------------------------------------------------------------------------------
// plane lz of capsule k's window: the links of its inside sites, appended as (a, b, q).
// Each block reserves the places of all its links with one atomic add (the lanes' counts
// scanned over the wave, the waves' totals over the block): the capsules' counters share a
// cache line, and one add per site or per wave queued thousands of atomics on it.  The
// order of the list does not enter any result.
constexpr int BB_FIND_BLK = 1024;   // one pass over a window plane of up to 1024 columns

__global__ void __launch_bounds__(BB_FIND_BLK) k_bb_find(BBArgs b) {
    const int k = blockIdx.y, lz = blockIdx.x, lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const CapState cs = b.cst[k];
    if (lz >= cs.dim[2]) return;
    const int dx = cs.dim[0], dy = cs.dim[1], ncol = dx * dy;
    __shared__ int s_w[BB_FIND_BLK / 64];
    __shared__ int s_base;
    const int uz = cs.lo[2] + lz, z = wrapb(uz, b.nz);
    if (b.wall && slab_pos(z, b.lz) == 0) return;
    // the planes below and above, and whether they are wall planes (uniform over the block)
    const int zm = z == 0 ? b.nz - 1 : z - 1, zp = z == b.nz - 1 ? 0 : z + 1;
    const bool wm = b.wall && slab_pos(zm, b.lz) == 0, wp = b.wall && slab_pos(zp, b.lz) == 0;
    for (int c0 = 0; c0 < ncol; c0 += blockDim.x) {   // uniform over the block
        const int col = c0 + threadIdx.x;
        int sa = 0, x = 0, y = 0, xm = 0, xp = 0, ym = 0, yp = 0;
        unsigned mask = 0u;
        if (col < ncol) {
            const int ly = col / dx, lx = col - ly * dx;
            x = wrapb(cs.lo[0] + lx, b.nx);
            y = wrapb(cs.lo[1] + ly, b.ny);
            sa = (z * b.ny + y) * b.nx + x;
            // neighbour coordinates wrap by one step at most
            xm = x == 0 ? b.nx - 1 : x - 1;
            xp = x == b.nx - 1 ? 0 : x + 1;
            ym = y == 0 ? b.ny - 1 : y - 1;
            yp = y == b.ny - 1 ? 0 : y + 1;
            if ((b.flag[sa] & LABEL_MASK) == k + 1) {
                // every neighbour is a lattice site: its flag is loaded unconditionally, all 18
                // loads issued before the first is tested
                uint8_t fb[Q - 1];
#pragma unroll
                for (int q = 1; q < Q; ++q) {
                    const int xb = CX[q] < 0 ? xm : (CX[q] > 0 ? xp : x);
                    const int yb = CY[q] < 0 ? ym : (CY[q] > 0 ? yp : y);
                    const int zb = CZ[q] < 0 ? zm : (CZ[q] > 0 ? zp : z);
                    fb[q - 1] = b.flag[(zb * b.ny + yb) * b.nx + xb];
                }
#pragma unroll
                for (int q = 1; q < Q; ++q) {
                    if (CZ[q] < 0 ? wm : (CZ[q] > 0 ? wp : false)) continue;
                    const int lb = fb[q - 1] & LABEL_MASK;
                    if (lb == k + 1 || (lb != 0 && lb < k + 1)) continue;
                    mask |= 1u << q;
                }
            }
        }
        const int cnt = __popc(mask);
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        // the waves' totals scanned in LDS, one atomic add per block for all of them (the
        // shuffle runs on every lane: it reads lane 63)
        const int wtot = __shfl(incl, 63, 64);
        if (lane == 0) s_w[wid] = wtot;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w = 0; w < BB_FIND_BLK / 64; ++w) {
                const int v = s_w[w];
                s_w[w] = tot;
                tot += v;
            }
            s_base = tot ? atomicAdd(&b.nlinks[k], tot) : 0;
        }
        __syncthreads();
        int i = s_base + s_w[wid] + incl - cnt;
        __syncthreads();   // s_w and s_base are rewritten by the next pass
        if (!mask) continue;
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            if (!(mask & (1u << q))) continue;
            if (i >= b.link_cap) {
                atomicOr(&b.status[ST_BBOVER], 1);
                break;
            }
            const int xb = CX[q] < 0 ? xm : (CX[q] > 0 ? xp : x);
            const int yb = CY[q] < 0 ? ym : (CY[q] > 0 ? yp : y);
            const int zb = CZ[q] < 0 ? zm : (CZ[q] > 0 ? zp : z);
            BBLink L;
            L.a = sa;
            L.b = (zb * b.ny + yb) * b.nx + xb;
            L.q = q;
            L.tri = -1;
            L.rho[0] = L.rho[1] = L.rho[2] = L.rho[3] = 0.f;
            b.links[(size_t)k * b.link_cap + i] = L;
            ++i;
        }
    }
}

// BB_RL lanes per link: the crossed triangle (least miss distance among the candidates of
// the cells the link's bounding box touches, lowest index on ties; the lanes split the
// candidates and reduce), and both sites' densities before any population changes
constexpr int BB_RL = 8;
static_assert(BB_RL == 4 || BB_RL == 8 || BB_RL == 16, "lanes per link divide 16");
constexpr int BB_RH = 16 / BB_RL;                   // partial density sums per lane
constexpr int BB_RC = BB_RL >= 8 ? 1 : 8 / BB_RL;   // cells per lane

template <int S>
__global__ void __launch_bounds__(256, 3) k_bb_resolve(BBArgs b) {
    const int k = blockIdx.y, sl = threadIdx.x % BB_RL;
    const int nl = min(b.nlinks[k], b.link_cap);
    const CapState cs = b.cst[k];
    const CapDev cd = b.caps[k];
    const int dx = cs.dim[0], dy = cs.dim[1];
    const int *st = b.bstart + (size_t)k * (GMAX3 + 1);
    const int *list = b.blist + (size_t)BB_PER_TRI * cd.tri0;
    const int lmax = BB_PER_TRI * cd.nt;
    // groups of BB_RL lanes take links in a grid-stride loop (uniform inside a group)
    const int g0 = blockIdx.x * (blockDim.x / BB_RL) + threadIdx.x / BB_RL;
    const int gstride = gridDim.x * (blockDim.x / BB_RL);
    for (int i = g0; i < nl; i += gstride) {
        BBLink &L = b.links[(size_t)k * b.link_cap + i];
        const int sa = L.a, sbi = L.b, q = L.q;
        // densities of both sites (issued first, so that their loads are in flight during
        // the candidate search), summed in the order of a 16-wide butterfly whatever the
        // group's width: partial sum j < 16 holds the populations j and j + 16, lane sl
        // holds the partial sums sl + h BB_RL and combines them as that butterfly's first
        // levels do
        float pr[BB_RH][4];
#pragma unroll
        for (int h = 0; h < BB_RH; ++h) {
            pr[h][0] = pr[h][1] = pr[h][2] = pr[h][3] = 0.f;
            for (int qq = sl + h * BB_RL; qq < Q; qq += 16) {
                pr[h][0] += popl<S>(b.f, 0, qq, b.N, sa, b.shift[0]);
                pr[h][1] += popl<S>(b.f, 1, qq, b.N, sa, b.shift[1]);
                pr[h][2] += popl<S>(b.f, 0, qq, b.N, sbi, b.shift[0]);
                pr[h][3] += popl<S>(b.f, 1, qq, b.N, sbi, b.shift[1]);
            }
        }
        // unwrapped coordinates of a in the window's frame, from its lattice index
        const int ax = sa % b.nx, ay = (sa / b.nx) % b.ny, az = sa / (b.nx * b.ny);
        const int ux = cs.lo[0] + wrapb(ax - cs.lo[0], b.nx);
        const int uy = cs.lo[1] + wrapb(ay - cs.lo[1], b.ny);
        const int uz = cs.lo[2] + wrapb(az - cs.lo[2], b.nz);
        const double p0[3] = {(double)ux, (double)uy, (double)uz};
        const double p1[3] = {(double)(ux + CX[q]), (double)(uy + CY[q]), (double)(uz + CZ[q])};
        double lo[3], hi[3];
        int c0[3], nc3[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(p0[d], p1[d]);
            hi[d] = fmax(p0[d], p1[d]);
            c0[d] = max((int)lo[d] - cs.lo[d], 0);
            // one or two cells per axis (a link moves at most one site per axis)
            nc3[d] = max(min((int)hi[d] - cs.lo[d], cs.dim[d] - 1) - c0[d] + 1, 0);
        }
        // the (at most 2 x 2 x 2) cells, x fastest: cell j's start and end are read by lane
        // j mod BB_RL, and the group shares them
        int my_beg[BB_RC], my_cnt[BB_RC];
#pragma unroll
        for (int h = 0; h < BB_RC; ++h) {
            const int j = sl + h * BB_RL;
            my_beg[h] = my_cnt[h] = 0;
            if (j < 8 && j < nc3[0] * nc3[1] * nc3[2]) {
                const int ix = nc3[0] == 2 ? (j & 1) : 0, r1 = nc3[0] == 2 ? j >> 1 : j;
                const int iy = nc3[1] == 2 ? (r1 & 1) : 0, iz = nc3[1] == 2 ? r1 >> 1 : r1;
                const int cell = ((c0[2] + iz) * dy + c0[1] + iy) * dx + c0[0] + ix;
                my_beg[h] = st[cell];
                my_cnt[h] = max(min(st[cell + 1], lmax) - my_beg[h], 0);
            }
        }
        // the first levels of the density butterfly, inside the lane (the cell starts' wait
        // covers the loads): level o pairs partial sum j with j + o
#pragma unroll
        for (int o = 8; o >= BB_RL; o >>= 1)
#pragma unroll
            for (int h = 0; h < o / BB_RL; ++h)
#pragma unroll
                for (int c = 0; c < 4; ++c) pr[h][c] += pr[h + o / BB_RL][c];
        float ra0 = pr[0][0], ra1 = pr[0][1], rb0 = pr[0][2], rb1 = pr[0][3];
        int beg[8], cnt[8], tot = 0;
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            beg[n] = __shfl(my_beg[n / BB_RL < BB_RC ? n / BB_RL : 0], n % BB_RL, BB_RL);
            cnt[n] = __shfl(my_cnt[n / BB_RL < BB_RC ? n / BB_RL : 0], n % BB_RL, BB_RL);
            tot += cnt[n];
        }
        double bd = __builtin_inf();
        int best = 0x7fffffff;
        // the candidates split over the lanes, BB_RB per lane at a time: the list entries
        // are loaded together, then the vertices together
        constexpr int BB_RB = 4;
        for (int e0 = 0; e0 < tot; e0 += BB_RB * BB_RL) {   // uniform inside a group
            int tt[BB_RB];
#pragma unroll
            for (int u = 0; u < BB_RB; ++u) {
                int r = e0 + sl + u * BB_RL, at = -1;
                if (r < tot) {
#pragma unroll
                    for (int n = 0; n < 8; ++n) {
                        if (at < 0) {
                            if (r < cnt[n]) at = beg[n] + r;
                            else r -= cnt[n];
                        }
                    }
                }
                tt[u] = at >= 0 ? list[at] : -1;
            }
            float4 A[BB_RB], B[BB_RB], C[BB_RB];
#pragma unroll
            for (int u = 0; u < BB_RB; ++u) {
                if ((unsigned)tt[u] >= (unsigned)b.ttot) tt[u] = -1;   // out of range: never expected
                const size_t o = 3 * (size_t)(tt[u] < 0 ? 0 : tt[u]);
                if (tt[u] >= 0) {
                    A[u] = b.tpos[o];
                    B[u] = b.tpos[o + 1];
                    C[u] = b.tpos[o + 2];
                }
            }
#pragma unroll
            for (int u = 0; u < BB_RB; ++u) {
                const int t = tt[u];
                if (t < 0) continue;
                const double v[3][3] = {{A[u].x, A[u].y, A[u].z}, {B[u].x, B[u].y, B[u].z},
                                        {C[u].x, C[u].y, C[u].z}};
                bool ok = true;
                for (int d = 0; d < 3 && ok; ++d) {
                    const double tl = fmin(v[0][d], fmin(v[1][d], v[2][d]));
                    const double th = fmax(v[0][d], fmax(v[1][d], v[2][d]));
                    ok = !(tl > hi[d] || th < lo[d]);
                }
                if (!ok) continue;
                const double md = miss_distance(p0, p1, v[0], v[1], v[2]);
                if (md < bd || (md == bd && t < best)) {
                    bd = md;
                    best = t;
                }
            }
        }
        // fixed butterfly over the group: the lexicographic minimum of (distance, index)
        // and the density sums
#pragma unroll
        for (int o = BB_RL / 2; o > 0; o >>= 1) {
            const double od = __shfl_xor(bd, o, BB_RL);
            const int ot = __shfl_xor(best, o, BB_RL);
            if (od < bd || (od == bd && ot < best)) {
                bd = od;
                best = ot;
            }
            ra0 += __shfl_xor(ra0, o, BB_RL);
            ra1 += __shfl_xor(ra1, o, BB_RL);
            rb0 += __shfl_xor(rb0, o, BB_RL);
            rb1 += __shfl_xor(rb1, o, BB_RL);
        }
        if (sl == 0) {
            const bool found = best != 0x7fffffff;
            L.tri = found ? best : -1;
            L.rho[0] = ra0;
            L.rho[1] = ra1;
            L.rho[2] = rb0;
            L.rho[3] = rb1;
            if (!found) atomicAdd(&b.status[ST_BBLOST], 1);
        }
    }
}

template <int S>
__device__ __forceinline__ void bb_swap_one(const BBArgs &b, int k, int i) {
    const BBLink L = b.links[(size_t)k * b.link_cap + i];
    const int q = L.q, qb = OPP[q];
    float ub[3] = {0.f, 0.f, 0.f};
    int4 tr = make_int4(0, 0, 0, 0);
    if (L.tri >= 0) {
        tr = b.tri[L.tri];
        const double4 A = b.V[tr.x], B = b.V[tr.y], C = b.V[tr.z];
        ub[0] = (float)((A.x + B.x + C.x) / 3.0);
        ub[1] = (float)((A.y + B.y + C.y) / 3.0);
        ub[2] = (float)((A.z + B.z + C.z) / 3.0);
    }
    const float eu = ub[0] * CX[q] + ub[1] * CY[q] + ub[2] * CZ[q];
    float dp = 0.f;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const float rb = 0.5f * (L.rho[c] + L.rho[2 + c]);
        const float delta = 6.0f * wq(q) * rb * eu;
        const float va = popl<S>(b.f, c, q, b.N, L.a, b.shift[c]);
        const float vb = popl<S>(b.f, c, qb, b.N, L.b, b.shift[c]);
        pops<S>(b.f, c, q, b.N, L.a, vb + delta, b.shift[c]);
        pops<S>(b.f, c, qb, b.N, L.b, va - delta, b.shift[c]);
        dp += 2.0f * va - 2.0f * vb - 2.0f * delta;
    }
    if (L.tri < 0) return;
    // a third to each node of the triangle: summed per triangle here, per node in k_bb_nodes
    const float third = dp / 3.0f;
    const long long p[3] = {fix40(third * CX[q]), fix40(third * CY[q]), fix40(third * CZ[q])};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (p[d]) atomicAdd((unsigned long long *)&b.pex[3 * (size_t)L.tri + d], (unsigned long long)p[d]);
}

template <int S>
__global__ void __launch_bounds__(256) k_bb_swap(BBArgs b) {
    const int k = blockIdx.y, nl = min(b.nlinks[k], b.link_cap);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += gridDim.x * blockDim.x)
        bb_swap_one<S>(b, k, i);
}

// psi = 1 - exp(-rho / rho0) as the fluid kernel evaluates it
__device__ __forceinline__ float bb_psi(float rho, float inv_rho0) {
    return 1.0f - __expf(-rho * inv_rho0);
}

__device__ __forceinline__ void bb_reaction_one(const BBArgs &b, int k, int i) {
    const BBLink L = b.links[(size_t)k * b.link_cap + i];
    if (L.tri < 0) return;
    const int q = L.q;
    const int la = b.flag[L.a] & LABEL_MASK, lb = b.flag[L.b] & LABEL_MASK;
    // wetting offsets of the boundary seen from each side (the other side's capsule if it
    // is one, else this side's)
    const float dra = b.cap_drho[(lb != 0 ? lb : la) - 1];
    const float drb = b.cap_drho[(la != 0 ? la : lb) - 1];
    // densities and psi of both sites as the fluid step used them (written there on the
    // window sites)
    const float4 A = b.dens[L.a], B = b.dens[L.b];
    const float ra[2] = {A.x, A.y}, pa[2] = {A.z, A.w};
    const float rbv[2] = {B.x, B.y}, pb[2] = {B.z, B.w};
    const float w = is_axis(q) ? b.ws_axis : b.ws_diag;
    float r = 0.f;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int cq = 1 - c;
        const float sg = cq == 0 ? 1.f : -1.f;
        // with a zero offset the substituted psi is the site's own psi of the partner
        const float qa = dra == 0.f ? pa[cq] : bb_psi(fmaxf(ra[cq] + sg * dra, 0.f), b.inv_rho0);
        const float qb = drb == 0.f ? pb[cq] : bb_psi(fmaxf(rbv[cq] + sg * drb, 0.f), b.inv_rho0);
        r += b.G * w * (pa[c] * qa - pb[c] * qb);
    }
    const float third = r / 3.0f;
    const long long p[3] = {fix40(third * CX[q]), fix40(third * CY[q]), fix40(third * CZ[q])};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (p[d]) atomicAdd((unsigned long long *)&b.rsc[3 * (size_t)L.tri + d], (unsigned long long)p[d]);
}

__global__ void __launch_bounds__(256) k_bb_reaction(BBArgs b) {
    const int k = blockIdx.y, nl = min(b.nlinks[k], b.link_cap);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += gridDim.x * blockDim.x)
        bb_reaction_one(b, k, i);
}

// Newtonian nodes: v += (F_membrane + (P_ex(n) + P_ex(n-1)) / 2 + R_sc) / m, x += v; the
// link counts are cleared for the next step
__global__ void __launch_bounds__(256) k_bb_nodes(BBArgs b) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n == 0)   // this step's link counts are kept (observables) and the counters cleared
        for (int k = 0; k < b.ncap; ++k) {
            b.nlinks[b.ncap + k] = b.nlinks[k];
            b.nlinks[k] = 0;
        }
    if (n >= b.ntot) return;
    const float4 Fm = b.F[b.slot[n]];
    const float4 Pp = b.pprev[n];
    // the sums of every incident triangle, each already the third of its links' momentum
    // that goes to each of its nodes (integers: the order of the additions does not matter)
    long long ps[3] = {0, 0, 0}, qs[3] = {0, 0, 0};
    for (int e = b.ntri_off[n]; e < b.ntri_off[n + 1]; ++e) {
        const size_t t = (size_t)(b.ntri[e] / 3);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ps[d] += b.pex[3 * t + d];
            qs[d] += b.rsc[3 * t + d];
        }
    }
    float pe[3], rs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        pe[d] = unfix40(ps[d]);
        rs[d] = unfix40(qs[d]);
    }
    const float ff[3] = {0.5f * (pe[0] + Pp.x) + rs[0], 0.5f * (pe[1] + Pp.y) + rs[1],
                         0.5f * (pe[2] + Pp.z) + rs[2]};
    double4 V = b.V[n], X = b.X[n];
    V.x += ((double)Fm.x + (double)ff[0]) * b.inv_mass;
    V.y += ((double)Fm.y + (double)ff[1]) * b.inv_mass;
    V.z += ((double)Fm.z + (double)ff[2]) * b.inv_mass;
    X.x += V.x;
    X.y += V.y;
    X.z += V.z;
    b.V[n] = V;
    b.X[n] = X;
    b.pprev[n] = make_float4(pe[0], pe[1], pe[2], 0.f);
    b.ffl[n] = make_float4(ff[0], ff[1], ff[2], 0.f);
    b.R[n] = make_float4(rs[0], rs[1], rs[2], 0.f);
}

// ------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------
// link-kernel grid per capsule: enough blocks for the links of an R = 10 capsule in one
// pass, a grid-stride loop beyond
static int link_blocks(const BBArgs &b, int per_block) {
    const int nb = (b.link_cap + per_block - 1) / per_block;
    return nb < 64 ? nb : 64;
}

void launch_bb_before(const BBArgs &b, int storage, hipStream_t st) {
    hipLaunchKernelGGL(k_bb_tri, dim3((b.ttot + 255) / 256), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_bb_bins, dim3(b.ncap), dim3(BB_BIN_BLK), 0, st, b);
    hipLaunchKernelGGL(k_bb_find, dim3(GMAX, b.ncap), dim3(BB_FIND_BLK), 0, st, b);
    const dim3 rg(4 * link_blocks(b, 256 / BB_RL), b.ncap), sg(link_blocks(b, 256), b.ncap);
    switch (storage) {
        case 0:
            hipLaunchKernelGGL(k_bb_resolve<0>, rg, dim3(256), 0, st, b);
            hipLaunchKernelGGL(k_bb_swap<0>, sg, dim3(256), 0, st, b);
            break;
        case 1:
            hipLaunchKernelGGL(k_bb_resolve<1>, rg, dim3(256), 0, st, b);
            hipLaunchKernelGGL(k_bb_swap<1>, sg, dim3(256), 0, st, b);
            break;
        default:
            hipLaunchKernelGGL(k_bb_resolve<2>, rg, dim3(256), 0, st, b);
            hipLaunchKernelGGL(k_bb_swap<2>, sg, dim3(256), 0, st, b);
            break;
    }
}

void launch_bb_after(const BBArgs &b, int storage, hipStream_t st) {
    (void)storage;
    hipLaunchKernelGGL(k_bb_reaction, dim3(link_blocks(b, 256), b.ncap), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_bb_nodes, dim3((b.ntot + 255) / 256), dim3(256), 0, st, b);
}

}  // namespace lbmx
