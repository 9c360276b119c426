// membrane.hip -- capsule membrane and immersed-boundary kernels of liblbm (gfx950).
//
// Each capsule owns a window of lattice sites: its node bounding box widened so that
// it holds the 4x4x4 kernel support of every node and every site next to a label
// change.  Labels and the spread force are computed per window site by gathering (no
// floating-point atomics), so results do not depend on scheduling.
#include "lbm_internal.h"

namespace lbmx {


// Peskin's 4-point kernel in one dimension.
__device__ __forceinline__ float phi4(float r) {
    const float a = fabsf(r);
    if (a <= 1.0f) return (3.0f - 2.0f * a + sqrtf(1.0f + 4.0f * a - 4.0f * a * a)) * 0.125f;
    if (a <= 2.0f) return (5.0f - 2.0f * a - sqrtf(-7.0f + 12.0f * a - 4.0f * a * a)) * 0.125f;
    return 0.0f;
}

__device__ __forceinline__ int wrapm(int a, int n) {
    a %= n;
    return a < 0 ? a + n : a;
}

// nearest periodic image of a separation d along an axis of n sites (inv = 1 / n)
__device__ __forceinline__ double min_image(double d, int n, double inv, bool periodic) {
    return periodic ? d - n * floor(d * inv + 0.5) : d;
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_down(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_down(v, o, 64));
    return v;
}

// Sums over aligned groups of 8 or 16 lanes with DPP moves inside a 16-lane row: pairs
// (quad_perm 1,0,3,2), quads (quad_perm 2,3,0,1), half-row mirror, row mirror.  Every
// lane of the group ends with the same, bitwise identical total.
template <int CTRL> __device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float group_sum8(float v) {
    v += dpp_mov<0xb1>(v);
    v += dpp_mov<0x4e>(v);
    v += dpp_mov<0x141>(v);
    return v;
}
__device__ __forceinline__ float group_sum16(float v) {
    v = group_sum8(v);
    v += dpp_mov<0x140>(v);
    return v;
}

// Fixed-point accumulation (2^-40 units) for sums whose terms arrive in no fixed order.
// fix_mul(w, s) is w s rounded to the nearest integer, ties to even, for |w s| < 2^51: one
// FP64 fused multiply-add adds 1.5 * 2^52, which leaves that integer in the low bits of the
// significand.  (The hardware has no FP-to-int64 conversion.)  Values are clamped to
// |v| < 2^11 before they are scaled by 2^40.
constexpr double FIX_ONE = 1099511627776.0;   // 2^40
__device__ __forceinline__ long long fix_mul(double w, double s) {
    return __double_as_longlong(fma(w, s, 6755399441055744.0)) - 0x4338000000000000ll;
}
__device__ __forceinline__ long long to_fix_d(double v) {
    return fix_mul(fmin(fmax(v, -2047.0), 2047.0), FIX_ONE);
}
__device__ __forceinline__ float from_fix(long long v) {
    return (float)((double)v * (1.0 / 1099511627776.0));
}

// Wave sum of a double in a fixed order: DPP sums inside each 16-lane row, then the four
// row totals in row order.  Lane 0 holds the result.
template <int CTRL> __device__ __forceinline__ double dpp_mov_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_sum_d(double v) {
    v += dpp_mov_d<0xb1>(v);
    v += dpp_mov_d<0x4e>(v);
    v += dpp_mov_d<0x141>(v);
    v += dpp_mov_d<0x140>(v);
    const double r1 = __shfl(v, 16, 64), r2 = __shfl(v, 32, 64), r3 = __shfl(v, 48, 64);
    return ((v + r1) + r2) + r3;
}

// a + o wrapped into [0, n) for |o| small; positions rarely leave [-n, 2n)
__device__ __forceinline__ int wrap_near(int a, int n) {
    if (a >= n) a -= n;
    else if (a < 0) a += n;
    return (a >= 0 && a < n) ? a : wrapm(a, n);
}

// ------------------------------------------------------------------------------------
// Capsule reduction, one block per capsule: first clear the crossing masks of capsule k's
// previous window (and keep that window for the window kernel, which clears its flags),
// then reduce the nodes (sum of X - X_ref, FP32 bounding box)
// and, for capsules with a volume penalty, the triangles (signed tetrahedron volumes with
// apex X_ref, the first node; the volume of a closed mesh does not depend on the apex),
// each thread a strided share, then the waves in a fixed order, so the result does not
// depend on scheduling.  From the totals: centroid, volume, bounding box and site window;
// then the nodes are binned by the (y, z) lattice row of floor(X) inside the window:
// positions in row order (any order inside a row), and each node's place in that order.
// (A capsule has at most LBM_MAX_CAPSULE_NODES nodes, 16 per thread.  Earlier forms
// spread the sums over several blocks per capsule, with a second launch or a last-block
// counter to combine them; one block is one launch and no partial records.)
// ------------------------------------------------------------------------------------
constexpr int RED_BLK = 512, RED_W = RED_BLK / 64;

__device__ __forceinline__ void capsule_reduce_body(const MembraneArgs &m, int k) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const CapDev cd = m.caps[k];
    // the previous window: its crossing masks are cleared here (the membrane kernel marks
    // the new ones); its flags are cleared by the window kernel, spread over its planes
    const CapState old = m.cst[k];
    for (int i = tid; i < old.dim[0] * old.dim[1]; i += RED_BLK)
        m.marks[(size_t)k * ROWS_MAX + i] = 0ull;
    const double4 Xr = m.X[cd.node0];
    double s[3] = {0.0, 0.0, 0.0}, vol = 0.0;
    float mn[3] = {3e38f, 3e38f, 3e38f}, mx[3] = {-3e38f, -3e38f, -3e38f};
    // every node is loaded once, into registers (thread tid holds nodes tid + i RED_BLK),
    // with all of a thread's (clamped) loads in flight at once; the sums, the row count and
    // the scatter below all read these registers
    constexpr int PER = MAX_CAP_NODES / RED_BLK;
    double4 Xn[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i)
        Xn[i] = i * RED_BLK < cd.nn ? m.X[cd.node0 + min(tid + i * RED_BLK, cd.nn - 1)]   // uniform
                                    : make_double4(0.0, 0.0, 0.0, 0.0);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        if (tid + i * RED_BLK >= cd.nn) continue;
        const double p[3] = {Xn[i].x, Xn[i].y, Xn[i].z}, r[3] = {Xr.x, Xr.y, Xr.z};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            s[d] += p[d] - r[d];
            mn[d] = fminf(mn[d], (float)p[d]);
            mx[d] = fmaxf(mx[d], (float)p[d]);
        }
    }
    // the enclosed volume is needed on the device only for the volume penalty
    for (int t = tid; cd.kv != 0.0f && t < cd.nt; t += RED_BLK) {
        const int4 tr = m.tri[cd.tri0 + t];
        const double4 A = m.X[tr.x], B = m.X[tr.y], C = m.X[tr.z];
        const double a[3] = {A.x - Xr.x, A.y - Xr.y, A.z - Xr.z};
        const double b[3] = {B.x - Xr.x, B.y - Xr.y, B.z - Xr.z};
        const double e[3] = {C.x - Xr.x, C.y - Xr.y, C.z - Xr.z};
        vol += (a[0] * (b[1] * e[2] - b[2] * e[1]) + a[1] * (b[2] * e[0] - b[0] * e[2]) +
                a[2] * (b[0] * e[1] - b[1] * e[0])) / 6.0;
    }
    __shared__ double sd[RED_W][4];
    __shared__ float smn[RED_W][3], smx[RED_W][3];
    __shared__ int s_lo[3], s_dim[3];
    __shared__ int cnt[ROWS_MAX];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double v = wave_sum_d(s[d]);
        const float a = wave_min(mn[d]), b = wave_max(mx[d]);
        if (lane == 0) { sd[wid][d] = v; smn[wid][d] = a; smx[wid][d] = b; }
    }
    vol = wave_sum_d(vol);
    if (lane == 0) sd[wid][3] = vol;
    __syncthreads();
    if (tid == 0) {
        double tot[4];
        float bmin[3], bmax[3];
        for (int d = 0; d < 4; ++d) {
            double v = sd[0][d];
            for (int w = 1; w < RED_W; ++w) v += sd[w][d];
            tot[d] = v;
        }
        for (int d = 0; d < 3; ++d) {
            float a = smn[0][d], b = smx[0][d];
            for (int w = 1; w < RED_W; ++w) { a = fminf(a, smn[w][d]); b = fmaxf(b, smx[w][d]); }
            bmin[d] = a;
            bmax[d] = b;
        }
        CapState cs;
        for (int d = 0; d < 3; ++d) {
            cs.plo[d] = old.lo[d];
            cs.pdim[d] = old.dim[d];
        }
        const double r[3] = {Xr.x, Xr.y, Xr.z};
        const int nd[3] = {m.nx, m.ny, m.nz};
        cs.vol = tot[3];
        for (int d = 0; d < 3; ++d) {
            const float a = bmin[d], b = bmax[d];
            cs.cen[d] = r[d] + tot[d] / cd.nn;
            cs.bmin[d] = a;
            cs.bmax[d] = b;
            int fa = 0, dim = min(GMAX, nd[d]);
            if (!(b - a <= (float)GMAX) || !(fabsf(a) < 1e8f) || !(fabsf(b) < 1e8f)) {
                atomicOr(&m.status[ST_OVERFLOW], 1);   // non-finite or exploded capsule
            } else {
                fa = (int)floorf(a);
                dim = (int)floorf(b) - fa + 4;
                if (dim > GMAX || dim > nd[d]) {
                    atomicOr(&m.status[ST_OVERFLOW], 1);
                    dim = min(dim, min(GMAX, nd[d]));
                }
            }
            cs.lo[d] = fa - 1;
            cs.dim[d] = dim;
            s_lo[d] = fa - 1;
            s_dim[d] = dim;
        }
        // stacked slabs: the window must stay between the wall layers of its slab, or it
        // would reach the fluid of the neighbouring slab
        if (m.lz < m.nz && (cs.lo[2] < cd.zbase || cs.lo[2] + cs.dim[2] - 1 > cd.zbase + m.lz))
            atomicOr(&m.status[ST_SLAB], 1);
        m.cst[k] = cs;
    }
    __syncthreads();
    // ---- node rows: counting sort by (z, y) row; order inside a row is arbitrary ----
    const int lo1 = s_lo[1], lo2 = s_lo[2], dim1 = s_dim[1], dim2 = s_dim[2];
    const int rows = dim1 * dim2;
    for (int r = tid; r < rows; r += RED_BLK) cnt[r] = 0;
    __syncthreads();
    auto row_of = [&](double y, double z) {
        const int ry = min(max((int)floor(y) - lo1, 0), dim1 - 1);
        const int rz = min(max((int)floor(z) - lo2, 0), dim2 - 1);
        return rz * dim1 + ry;
    };
#pragma unroll
    for (int i = 0; i < PER; ++i)
        if (tid + i * RED_BLK < cd.nn) atomicAdd(&cnt[row_of(Xn[i].y, Xn[i].z)], 1);
    __syncthreads();
    // exclusive scan: each thread owns a contiguous run of rows
    __shared__ int wsum[RED_W];
    const int per = (rows + RED_BLK - 1) / RED_BLK;
    const int q0 = min(tid * per, rows), q1 = min(q0 + per, rows);
    int local = 0;
    for (int r = q0; r < q1; ++r) local += cnt[r];
    int incl = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int run = incl - local;
    for (int w = 0; w < wid; ++w) run += wsum[w];
    __syncthreads();
    int *rs = m.rowstart + (size_t)k * (ROWS_MAX + 1);
    for (int r = q0; r < q1; ++r) {
        const int cr = cnt[r];
        rs[r] = run;
        cnt[r] = run;   // becomes the scatter cursor, and ends as the end of row r
        run += cr;
    }
    if (tid == 0) rs[rows] = cd.nn;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int n = tid + i * RED_BLK;
        if (n < cd.nn) {
            const int e = cd.node0 + atomicAdd(&cnt[row_of(Xn[i].y, Xn[i].z)], 1);
            m.xrow[e] = Xn[i];
            m.slot[cd.node0 + n] = e;
        }
    }
}

__global__ void __launch_bounds__(RED_BLK) k_capsule_reduce(MembraneArgs m) {
    capsule_reduce_body(m, blockIdx.x);
}

void launch_capsule_reduce(const MembraneArgs &m, hipStream_t st) {
    hipLaunchKernelGGL(k_capsule_reduce, dim3(m.ncap), dim3(RED_BLK), 0, st, m);
}

// ------------------------------------------------------------------------------------
// Membrane node forces at X^n (node-centric gather over the incident triangles):
// Skalak strain (eq. strain) by virtual work, volume penalty (eq. vol_cons), Hertz
// particle-substrate and particle-particle repulsion (eq. interactions), centroid
// anchor, plus the pending reaction.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void skalak_corner(const float3 u, const float3 v, const float4 mi,
                                              float a0, float ks, float C, int corner,
                                              float (&f)[3]) {
    // D = [u v] M^{-1}; B = D^T D; I1 = tr B - 2; I2 = det B - 1
    const float d0[3] = {u.x * mi.x + v.x * mi.z, u.y * mi.x + v.y * mi.z, u.z * mi.x + v.z * mi.z};
    const float d1[3] = {u.x * mi.y + v.x * mi.w, u.y * mi.y + v.y * mi.w, u.z * mi.y + v.z * mi.w};
    const float b00 = d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2];
    const float b01 = d0[0] * d1[0] + d0[1] * d1[1] + d0[2] * d1[2];
    const float b11 = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
    const float I1 = b00 + b11 - 2.0f;
    const float I2 = b00 * b11 - b01 * b01 - 1.0f;
    const float W1 = 0.5f * ks * (I1 + 1.0f);      // dW/dI1
    const float W2 = 0.5f * ks * (C * I2 - 1.0f);  // dW/dI2
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // dW/dD = 2 W1 D + 2 W2 D adj(B); dE/d[u v] = A0 (dW/dD) M^{-T}
        const float P0 = 2.0f * W1 * d0[d] + 2.0f * W2 * (d0[d] * b11 - d1[d] * b01);
        const float P1 = 2.0f * W1 * d1[d] + 2.0f * W2 * (d1[d] * b00 - d0[d] * b01);
        const float gu = a0 * (P0 * mi.x + P1 * mi.y);
        const float gv = a0 * (P0 * mi.z + P1 * mi.w);
        f[d] += corner == 0 ? gu + gv : (corner == 1 ? -gu : -gv);
    }
}

// Crossing masks: for every lattice column inside a triangle's xy projection (top-left
// rule on shared edges; zero-area projections skipped), the crossing height z_c is the
// barycentric interpolation of the vertex heights; sites m >= ceil(z_c) lie above it.
// Bit ceil(z_c) - lo_z of the column's mask is toggled; the parity of the bits at or
// below a plane is the inside parity there.  Decisions use FP32-rounded positions
// evaluated in double.
__device__ __forceinline__ double edgef(double ux, double uy, double vx, double vy, double px,
                                        double py) {
    return (vx - ux) * (py - uy) - (vy - uy) * (px - ux);
}
__device__ __forceinline__ bool edge_in(double w, double ux, double uy, double vx, double vy) {
    return w > 0.0 || (w == 0.0 && ((vy < uy) || (vy == uy && vx < ux)));
}

__device__ void label_marks(const MembraneArgs &m, int t) {
    const int4 tr = m.tri[t];
    const int k = tr.w;
    const CapState cs = m.cst[k];
    const double4 A = m.X[tr.x], B = m.X[tr.y], C = m.X[tr.z];
    double ax = (float)A.x, ay = (float)A.y, az = (float)A.z;
    double bx = (float)B.x, by = (float)B.y, bz = (float)B.z;
    double cx = (float)C.x, cy = (float)C.y, cz = (float)C.z;
    const double area = edgef(ax, ay, bx, by, cx, cy);
    if (area == 0.0) return;
    if (area < 0.0) {
        double tmp;
        tmp = bx; bx = cx; cx = tmp;
        tmp = by; by = cy; cy = tmp;
        tmp = bz; bz = cz; cz = tmp;
    }
    const double xlo = fmin(ax, fmin(bx, cx)), xhi = fmax(ax, fmax(bx, cx));
    const double ylo = fmin(ay, fmin(by, cy)), yhi = fmax(ay, fmax(by, cy));
    // a triangle wider than any window (or with non-finite vertices) marks nothing; the
    // window overflow is reported by the reduction kernel
    if (!(xhi - xlo <= (double)GMAX) || !(yhi - ylo <= (double)GMAX) || !(fabs(az) < 1e9) ||
        !(fabs(bz) < 1e9) || !(fabs(cz) < 1e9) || !(fabs(xlo) < 1e9) || !(fabs(ylo) < 1e9))
        return;
    const int x0 = (int)ceil(xlo), x1 = (int)floor(xhi);
    const int y0 = (int)ceil(ylo), y1 = (int)floor(yhi);
    unsigned long long *mk = m.marks + (size_t)k * ROWS_MAX;
    for (int py = y0; py <= y1; ++py)
        for (int px = x0; px <= x1; ++px) {
            const double wa = edgef(bx, by, cx, cy, px, py);
            const double wb = edgef(cx, cy, ax, ay, px, py);
            const double wc = edgef(ax, ay, bx, by, px, py);
            if (!edge_in(wa, bx, by, cx, cy) || !edge_in(wb, cx, cy, ax, ay) ||
                !edge_in(wc, ax, ay, bx, by))
                continue;
            const double zc = (wa * az + wb * bz + wc * cz) / (wa + wb + wc);
            const int lx = px - cs.lo[0], ly = py - cs.lo[1], lz = (int)ceil(zc) - cs.lo[2];
            if (lx < 0 || ly < 0 || lz < 0 || lx >= cs.dim[0] || ly >= cs.dim[1] || lz >= cs.dim[2])
                continue;
            atomicXor(&mk[ly * cs.dim[0] + lx], 1ull << lz);
        }
}

// One launch, two kinds of block: the first blocks toggle the crossing masks, one thread
// per triangle; the remaining blocks compute node forces, MEM_L lanes per node (incident
// triangles and the candidates of each partner capsule split over the lanes, summed by a
// fixed butterfly).  The short mask blocks come first, so the long force blocks are not
// the ones left waiting for room when the launch exceeds the resident blocks.
constexpr int MEM_BLK = 256, MEM_L = 8, MEM_NPB = MEM_BLK / MEM_L;
static_assert(MEM_BLK >= 128, "two waves list the Hertz partners");

__device__ __forceinline__ void membrane_body(const MembraneArgs &m, int blk, int ntot, int ttot) {
    const int nb_marks = (ttot + MEM_BLK - 1) / MEM_BLK;
    if (blk < nb_marks) {
        const int t = blk * MEM_BLK + threadIdx.x;
        if (t < ttot) label_marks(m, t);
        return;
    }
    blk -= nb_marks;
    __shared__ CapState s_cst[MAX_CAPS];
    __shared__ int s_zb[MAX_CAPS];
    __shared__ int s_near[2][MAX_CAPS], s_nnear[2];
    for (int j = threadIdx.x; j < m.ncap; j += MEM_BLK) {
        s_cst[j] = m.cst[j];
        s_zb[j] = m.caps[j].zbase;
    }
    // the capsules of this block's first and last node (node ranges are contiguous)
    const int nb0 = blk * MEM_NPB, nb1 = min(nb0 + MEM_NPB, ntot) - 1;
    const int kb[2] = {m.node_cap[nb0], m.node_cap[nb1]};
    __syncthreads();
    if (m.hertz_xi > 0.f) {
        // Hertz partner capsules: those of the same slab whose node bounding box comes
        // within delta0 of the bounding box of the block's capsule (periodic images; every
        // pair closer than delta0 passes, so the per-node search below loses nothing)
        const bool per[3] = {true, true, !m.wall};
        const int nd[3] = {m.nx, m.ny, m.nz};
        const float d0 = m.hertz_d0, slack = 1e-3f;
        // wave w (0, 1) lists the partners of capsule kb[w] in ascending order: a lane per
        // candidate, compacted by ballot
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        if (w < 2) {
            int c = 0;
            for (int j0 = 0; j0 < m.ncap; j0 += 64) {   // uniform over the wave
                const int j = j0 + lane;
                bool near = j < m.ncap && j != kb[w] && s_zb[j] == s_zb[kb[w]];
                if (near) {
                    const CapState &A = s_cst[kb[w]], &B = s_cst[j];
                    for (int d = 0; d < 3 && near; ++d) {
                        const float ha = 0.5f * (A.bmax[d] - A.bmin[d]),
                                    hb = 0.5f * (B.bmax[d] - B.bmin[d]);
                        float dc = 0.5f * (A.bmin[d] + A.bmax[d]) - 0.5f * (B.bmin[d] + B.bmax[d]);
                        if (per[d]) {
                            if (2.f * (ha + hb + d0 + 1.f) >= (float)nd[d]) continue;   // box-sized: keep
                            dc -= nd[d] * floorf(dc / nd[d] + 0.5f);
                        }
                        near = fabsf(dc) - ha - hb <= d0 + slack;
                    }
                }
                const unsigned long long b = __ballot(near);
                if (near) s_near[w][c + __popcll(b & ((1ull << lane) - 1ull))] = j;
                c += __popcll(b);
            }
            if (lane == 0) s_nnear[w] = c;
        }
        __syncthreads();
    }
    const int n = blk * MEM_NPB + (threadIdx.x / MEM_L), sl = threadIdx.x % MEM_L;
    if (n >= ntot) return;   // whole groups of MEM_L lanes
    const int k = m.node_cap[n];
    const CapDev cd = m.caps[k];
    const double4 X = m.X[n];
    float f[3] = {0.f, 0.f, 0.f}, fh[3] = {0.f, 0.f, 0.f};
    const double vcoef = cd.kv != 0.0f ? -(double)cd.kv * (s_cst[k].vol - cd.v0) / cd.v0 : 0.0;
    const int e1 = m.ntri_off[n + 1];
    for (int e = m.ntri_off[n] + sl; e < e1; e += MEM_L) {
        const int ent = m.ntri[e];
        const int t = ent / 3, corner = ent - 3 * t;
        const int4 tr = m.tri[t];
        const double4 A = m.X[tr.x], B = m.X[tr.y], C = m.X[tr.z];
        const float3 u = make_float3((float)(B.x - A.x), (float)(B.y - A.y), (float)(B.z - A.z));
        const float3 v = make_float3((float)(C.x - A.x), (float)(C.y - A.y), (float)(C.z - A.z));
        skalak_corner(u, v, m.minv[t], m.a0[t], cd.ks, cd.C, corner, f);
        if (vcoef != 0.0) {
            // dV/dx_a of this triangle with the origin at x_a: (x_b - x_a) x (x_c - x_a) / 6,
            // (a, b, c) the cyclic order starting at this node
            const double4 P = corner == 0 ? B : (corner == 1 ? C : A);
            const double4 Qn = corner == 0 ? C : (corner == 1 ? A : B);
            const double pb[3] = {P.x - X.x, P.y - X.y, P.z - X.z};
            const double pc[3] = {Qn.x - X.x, Qn.y - X.y, Qn.z - X.z};
            f[0] += (float)(vcoef * (pb[1] * pc[2] - pb[2] * pc[1]) / 6.0);
            f[1] += (float)(vcoef * (pb[2] * pc[0] - pb[0] * pc[2]) / 6.0);
            f[2] += (float)(vcoef * (pb[0] * pc[1] - pb[1] * pc[0]) / 6.0);
        }
    }
    if (cd.kb != 0.0f) {
        // bending (eq. method:curvature, edge form): E = sqrt(3) kb sum_e (theta_e - theta0_e)^2
        // with theta_e the signed angle between the outward normals of the triangles
        // (x1, x2, x3) and (x2, x1, x4); this node's share of -dE/dx for each edge it is
        // part of, with the closed-form dihedral gradient (Blondel and Karplus, 1996)
        const float kk = -3.4641016f * cd.kb;   // -2 sqrt(3) kb
        const int b1 = m.nedge_off[n + 1];
        for (int e = m.nedge_off[n] + sl; e < b1; e += MEM_L) {
            const int ent = m.nedge[e];
            const int ed = ent >> 2, role = ent & 3;
            const int4 q = m.edge[ed];
            const double4 P1 = m.X[q.x], P2 = m.X[q.y], P3 = m.X[q.z], P4 = m.X[q.w];
            const float3 F = make_float3((float)(P3.x - P1.x), (float)(P3.y - P1.y), (float)(P3.z - P1.z));
            const float3 G = make_float3((float)(P1.x - P2.x), (float)(P1.y - P2.y), (float)(P1.z - P2.z));
            const float3 H = make_float3((float)(P4.x - P2.x), (float)(P4.y - P2.y), (float)(P4.z - P2.z));
            const float3 A = make_float3(F.y * G.z - F.z * G.y, F.z * G.x - F.x * G.z, F.x * G.y - F.y * G.x);
            const float3 B = make_float3(H.y * G.z - H.z * G.y, H.z * G.x - H.x * G.z, H.x * G.y - H.y * G.x);
            const float gg = G.x * G.x + G.y * G.y + G.z * G.z, gl = sqrtf(gg);
            const float a2 = A.x * A.x + A.y * A.y + A.z * A.z, b2 = B.x * B.x + B.y * B.y + B.z * B.z;
            const float ab = A.x * B.x + A.y * B.y + A.z * B.z;
            // (B x A) . G
            const float bag = (B.y * A.z - B.z * A.y) * G.x + (B.z * A.x - B.x * A.z) * G.y +
                              (B.x * A.y - B.y * A.x) * G.z;
            const float th = atan2f(-bag / gl, -ab);
            const float coef = kk * (th - m.eth0[ed]);
            const float ca = gl / a2, cb = gl / b2;
            const float fg = (F.x * G.x + F.y * G.y + F.z * G.z) / (a2 * gl);
            const float hg = (H.x * G.x + H.y * G.y + H.z * G.z) / (b2 * gl);
            // d theta / d x_role = wa A + wb B
            float wa, wb;
            if (role == 0) { wa = ca + fg; wb = -hg; }
            else if (role == 1) { wa = -fg; wb = hg - cb; }
            else if (role == 2) { wa = -ca; wb = 0.f; }
            else { wa = 0.f; wb = cb; }
            f[0] += coef * (wa * A.x + wb * B.x);
            f[1] += coef * (wa * A.y + wb * B.y);
            f[2] += coef * (wa * A.z + wb * B.z);
        }
    }
    const float xi = m.hertz_xi, d0 = m.hertz_d0;
    if (sl == 0 && m.wall && xi > 0.f) {
        const float d = (float)(X.z - (double)cd.plane_z);
        if (d < d0) fh[2] += xi * (d0 - d) * sqrtf(d0 - d);
    }
    if (xi > 0.f) {
        // particle-particle pairs: only nodes of another capsule whose bounding box lies
        // within delta0 of this node, and there only the (y, z) rows within delta0, can be
        // partners.  The candidates of a row range are split over the lanes; rows list
        // their nodes in no fixed order, so the pair forces are summed in fixed point.
        const bool per[3] = {true, true, !m.wall};
        const int nd[3] = {m.nx, m.ny, m.nz};
        const double inv[3] = {1.0 / m.nx, 1.0 / m.ny, 1.0 / m.nz};
        const double p[3] = {X.x, X.y, X.z};
        const double slack = 1e-3;   // FP32 rounding of the bounding box
        long long acc[3] = {0, 0, 0};
        // the partner lists cover the block's first and last capsule; a block of small
        // meshes holding more capsules scans them all
        const bool listed = kb[1] - kb[0] <= 1;
        const int w = k == kb[0] ? 0 : 1, nj = listed ? s_nnear[w] : m.ncap;
        for (int jj = 0; jj < nj; ++jj) {
            const int j = listed ? s_near[w][jj] : jj;
            if (j == k || (!listed && s_zb[j] != cd.zbase)) continue;
            const CapState &cj = s_cst[j];
            double pl[3];   // this node in the periodic image closest to window j
            bool far = false, small = true;
            for (int d = 0; d < 3; ++d) {
                const double c = cj.lo[d] + 0.5 * cj.dim[d];
                pl[d] = c + min_image(p[d] - c, nd[d], inv[d], per[d]);
                // the row search sees one periodic image of each partner; it is exact while
                // the window plus the cut-off is smaller than half the box, else scan all rows
                const bool fits = 2.0 * (cj.dim[d] + 2.0 * d0 + 2.0) <= nd[d];
                if (fits && (pl[d] < cj.bmin[d] - d0 - slack || pl[d] > cj.bmax[d] + d0 + slack))
                    far = true;
                if (per[d] && !fits) small = false;
            }
            if (far) continue;
            const int ry0 = small ? max((int)floor(pl[1] - d0) - cj.lo[1], 0) : 0;
            const int ry1 = small ? min((int)floor(pl[1] + d0) - cj.lo[1], cj.dim[1] - 1) : cj.dim[1] - 1;
            const int rz0 = small ? max((int)floor(pl[2] - d0) - cj.lo[2], 0) : 0;
            const int rz1 = small ? min((int)floor(pl[2] + d0) - cj.lo[2], cj.dim[2] - 1) : cj.dim[2] - 1;
            if (ry0 > ry1) continue;
            const int *rs = m.rowstart + (size_t)j * (ROWS_MAX + 1);
            const double4 *xr = m.xrow + m.caps[j].node0;
            for (int rz = rz0; rz <= rz1; ++rz) {
                // rows ry0 .. ry1 of plane rz are contiguous in the row order
                const int a = rs[rz * cj.dim[1] + ry0], b = rs[rz * cj.dim[1] + ry1 + 1];
                for (int e = a + sl; e < b; e += MEM_L) {
                    const double4 Y = xr[e];
                    const double r[3] = {min_image(p[0] - Y.x, nd[0], inv[0], per[0]),
                                         min_image(p[1] - Y.y, nd[1], inv[1], per[1]),
                                         min_image(p[2] - Y.z, nd[2], inv[2], per[2])};
                    const double dd = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                    if (dd < d0 && dd > 0.0) {
                        const double g = d0 - dd;
                        const double mag = xi * g * sqrt(g);
                        for (int d = 0; d < 3; ++d) acc[d] += to_fix_d(mag * r[d] / dd);
                    }
                }
            }
        }
        for (int d = 0; d < 3; ++d) fh[d] += from_fix(acc[d]);
    }
    if (sl == 0 && cd.anchor_k != 0.0f) {
        const CapState &cs = s_cst[k];
        const double ka = (double)cd.anchor_k / cd.nn;
        for (int d = 0; d < 3; ++d) f[d] += (float)(-ka * (cs.cen[d] - cd.c0[d]));
    }
    static_assert(MEM_L == 8, "group sums are over 8 lanes");
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        f[d] = group_sum8(f[d]);
        fh[d] = group_sum8(fh[d]);
    }
    if (sl == 0) {
        // the pending reaction of the immersed boundary (with bounce-back R holds the last
        // step's reaction for the observables; the nodes take it in their own update)
        const float4 R = m.bb ? make_float4(0.f, 0.f, 0.f, 0.f) : m.R[n];
        m.F[m.slot[n]] = make_float4(f[0] + fh[0] + R.x, f[1] + fh[1] + R.y, f[2] + fh[2] + R.z, 0.f);
        m.Fh[n] = make_float4(fh[0], fh[1], fh[2], 0.f);
    }
}

__global__ void __launch_bounds__(MEM_BLK) k_membrane(MembraneArgs m, int ntot, int ttot) {
    membrane_body(m, blockIdx.x, ntot, ttot);
}

void launch_membrane(const MembraneArgs &m, int ntot, int ttot, hipStream_t st) {
    const int nbf = (ntot + MEM_NPB - 1) / MEM_NPB, nbm = (ttot + MEM_BLK - 1) / MEM_BLK;
    hipLaunchKernelGGL(k_membrane, dim3(nbf + nbm), dim3(MEM_BLK), 0, st, m, ntot, ttot);
}

// ------------------------------------------------------------------------------------
// Window fill, in two kernels.
//
// k_window_own: one block per (capsule k, plane of its window); the same block first clears
// the flags of plane lz of capsule k's previous window.  Every node whose kernel
// support reaches the plane (node planes lz - 2 .. lz + 1, a contiguous run of the row
// order) adds its 4 x 4 sites of the plane, F_n phi(x - X_n) and phi(x - X_n), into an
// LDS plane buffer.  The sums are 64-bit fixed point (2^-40 units), so the atomic adds
// are exact and the result does not depend on their order.  Neighbours in the row order
// have overlapping supports, so threads take the nodes in a strided permutation of that
// order, which keeps the lanes of one atomic instruction on different columns.  The
// crossing parity of a site is the parity of the set bits of its column mask at or below
// its plane.  Results go to capsule k's window buffers.
//
// k_window_combine: per window site, the sum over every window holding the site, in
// capsule order, of those buffers; the side label is the highest capsule whose parity is
// odd.  Wall sites receive nothing.  Sites in several windows are written with the same
// values by each of them.
// ------------------------------------------------------------------------------------
constexpr int OWN_BLK = 256;

// Columns the spreading kernel's LDS buffer holds (4 x 8 bytes each, dynamic shared memory):
// 2048 (64 KB, two blocks per CU) for launches of at most OWN_FEW capsules, whose few active
// blocks then spread over the CUs; 1024 (32 KB, four blocks per CU) for more capsules, where
// the launch has many times more blocks than the CUs.  Wider windows take passes.
constexpr int OWN_FEW = 24;
static int own_cap(int ncap) { return ncap <= OWN_FEW ? 2048 : 1024; }

__device__ __forceinline__ int gcd_int(int a, int b) {
    while (b) { const int t = a % b; a = b; b = t; }
    return a;
}

// plane lz of capsule k's window
__device__ __forceinline__ void window_own_body(const MembraneArgs &m, int k, int lz, int cap) {
    const int tid = threadIdx.x;
    const CapState ck = m.cst[k];
    if (lz < ck.pdim[2]) {
        // plane lz of the previous step's window: clear its flags (the combine kernel then
        // writes those of the new windows)
        const int pdx = ck.pdim[0], ncol = pdx * ck.pdim[1];
        const int zrow = wrap_near(ck.plo[2] + lz, m.nz) * m.ny;
        for (int i = tid; i < ncol; i += OWN_BLK) {
            const int ly = i / pdx, lx = i - ly * pdx;
            m.flag[(zrow + wrap_near(ck.plo[1] + ly, m.ny)) * m.nx + wrap_near(ck.plo[0] + lx, m.nx)] = 0;
        }
    }
    if (lz >= ck.dim[2]) return;
    const int dx = ck.dim[0], dy = ck.dim[1], ncol = dx * dy;
    // the LDS buffer holds cap columns; a wider window is spread in passes over column ranges
    extern __shared__ unsigned long long s_acc[];   // [4][cap]
    if (ncol > FILL_COLS) {   // uniform over the block
        if (tid == 0) atomicOr(&m.status[ST_WIDE], 1);
        return;
    }
    unsigned long long *acc = s_acc;
    const int stride = cap;
    // nodes with floor(Z) - lo_z in [lz - 2, lz + 1] reach this plane
    const int r0 = max(lz - 2, 0), r1 = min(lz + 1, ck.dim[2] - 1);
    const int *rs = m.rowstart + (size_t)k * (ROWS_MAX + 1);
    const int e0 = rs[r0 * dy], nnode = rs[(r1 + 1) * dy] - e0;
    const int node0 = m.caps[k].node0 + e0;
    // stride p coprime with nnode: i -> i * p mod nnode is a permutation
    int p = nnode / 64 + 1;
    while (nnode > 1 && gcd_int(p, nnode) != 1) ++p;
    const double zs = (double)(ck.lo[2] + lz);
    float4 *wb = m.wbuf + (size_t)k * GMAX3 + (size_t)lz * ncol;
    uint8_t *wp = m.wpar + (size_t)k * GMAX3 + (size_t)lz * ncol;
    const unsigned long long *mk = m.marks + (size_t)k * ROWS_MAX;
    const unsigned long long below = (2ull << lz) - 1ull;   // planes 0 .. lz (lz <= 63)
    for (int c0 = 0; c0 < ncol; c0 += cap) {   // uniform over the block
        const int c1 = min(c0 + cap, ncol);
        for (int i = tid; i < c1 - c0; i += OWN_BLK)
            for (int d = 0; d < 4; ++d) acc[d * stride + i] = 0ull;
        __syncthreads();
        // with bounce-back nothing is spread: the window carries the labels only
        for (int i0 = 0; i0 < (m.bb ? 0 : nnode); i0 += 2 * OWN_BLK) {
            // two nodes per thread, both loaded before either is spread
            double4 X[2];
            float4 F[2];
            bool ok[2];
    #pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int i = i0 + tid + u * OWN_BLK;
                ok[u] = i < nnode;
                const int e = ok[u] ? (int)(((long long)i * p) % nnode) : 0;
                X[u] = m.xrow[node0 + e];
                F[u] = m.F[node0 + e];
            }
    #pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (!ok[u]) continue;
                const double fx = floor(X[u].x), fy = floor(X[u].y);
                const float wz = phi4((float)(X[u].z - zs));
                const float rx = (float)(X[u].x - fx), ry = (float)(X[u].y - fy);
                const int bx = (int)fx - 1 - ck.lo[0], by = (int)fy - 1 - ck.lo[1];
                // the force in fixed-point units, once per node (clamped so that its product with
                // a kernel weight, at most 1, stays below 2^51 units)
                const double fs[3] = {(double)fminf(fmaxf(F[u].x, -2047.f), 2047.f) * FIX_ONE,
                                      (double)fminf(fmaxf(F[u].y, -2047.f), 2047.f) * FIX_ONE,
                                      (double)fminf(fmaxf(F[u].z, -2047.f), 2047.f) * FIX_ONE};
                float wx[4];
    #pragma unroll
                for (int o = 0; o < 4; ++o) wx[o] = phi4(rx + (float)(1 - o));
    #pragma unroll
                for (int oy = 0; oy < 4; ++oy) {
                    const int ly = by + oy;
                    if (ly < 0 || ly >= dy) continue;
                    const float wyz = phi4(ry + (float)(1 - oy)) * wz;
    #pragma unroll
                    for (int ox = 0; ox < 4; ++ox) {
                        const int lx = bx + ox;
                        if (lx < 0 || lx >= dx) continue;
                        const double wgt = (double)(wx[ox] * wyz);
                        const int col = ly * dx + lx - c0;
                        if (col < 0 || col >= c1 - c0) continue;
                        atomicAdd(&acc[col], (unsigned long long)fix_mul(wgt, fs[0]));
                        atomicAdd(&acc[stride + col], (unsigned long long)fix_mul(wgt, fs[1]));
                        atomicAdd(&acc[2 * stride + col], (unsigned long long)fix_mul(wgt, fs[2]));
                        atomicAdd(&acc[3 * stride + col], (unsigned long long)fix_mul(wgt, FIX_ONE));
                    }
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < c1 - c0; i += OWN_BLK) {
            const int col = c0 + i;
            wb[col] = make_float4(from_fix((long long)acc[i]), from_fix((long long)acc[stride + i]),
                                  from_fix((long long)acc[2 * stride + i]),
                                  from_fix((long long)acc[3 * stride + i]));
            wp[col] = (uint8_t)(__popcll(mk[col] & below) & 1);
        }
        __syncthreads();   // the next pass clears the buffer
    }
}

__device__ __forceinline__ void window_combine_body(const MembraneArgs &m, int k, int lz) {
    const int tid = threadIdx.x;
    const CapState ck = m.cst[k];
    if (lz >= ck.dim[2]) return;
    const int dx = ck.dim[0], dy = ck.dim[1];
    __shared__ int s_win[MAX_CAPS + 1];
    __shared__ int s_box[MAX_CAPS][6];   // lo[3], dim[3] of each meeting window
    __shared__ unsigned long long s_meet[2];
    __shared__ int s_n;
    // windows meeting this plane of window k, in capsule order (k included): one thread
    // per capsule tests its window, ballots give each meeting window its place
    static_assert(MAX_CAPS <= 128, "window list uses two ballots");
    {
        const int j = tid;
        bool meet = false;
        int box[6] = {0, 0, 0, 0, 0, 0};
        if (j < m.ncap) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                box[d] = m.cst[j].lo[d];
                box[3 + d] = m.cst[j].dim[d];
            }
            const int ox = wrap_near(box[0] - ck.lo[0], m.nx);
            const int oy = wrap_near(box[1] - ck.lo[1], m.ny);
            const int oz = wrap_near(box[2] - (ck.lo[2] + lz), m.nz);
            meet = (ox < dx || ox + box[3] > m.nx) && (oy < dy || oy + box[4] > m.ny) &&
                   (oz < 1 || oz + box[5] > m.nz);
        }
        const unsigned long long b = __ballot(meet);
        if (tid < 128 && (tid & 63) == 0) s_meet[tid >> 6] = b;
        __syncthreads();
        if (meet) {
            const int lanebit = tid & 63;
            int pos = __popcll(b & ((1ull << lanebit) - 1ull));
            if (tid >= 64) pos += __popcll(s_meet[0]);
#pragma unroll
            for (int d = 0; d < 6; ++d) s_box[pos][d] = box[d];
            s_win[pos] = j;
        }
        if (tid == 0) s_n = __popcll(s_meet[0]) + __popcll(s_meet[1]);
    }
    __syncthreads();
    const int nwin = s_n;
    const int uz = ck.lo[2] + lz, z = wrap_near(uz, m.nz);
    if (m.wall && slab_pos(z, m.lz) == 0) return;   // wall sites receive nothing (uniform)
    for (int col = tid; col < dx * dy; col += blockDim.x) {
        const int ly = col / dx, lx = col - ly * dx;
        const int ux = ck.lo[0] + lx, uy = ck.lo[1] + ly;
        int lab = 0;
        float f[3] = {0.f, 0.f, 0.f}, c = 0.f;
        for (int i = 0; i < nwin; ++i) {
            const int j = s_win[i];
            const int *bj = s_box[i];
            const int l0 = wrap_near(ux - bj[0], m.nx), l1 = wrap_near(uy - bj[1], m.ny),
                      l2 = wrap_near(uz - bj[2], m.nz);
            if (l0 >= bj[3] || l1 >= bj[4] || l2 >= bj[5]) continue;
            const int li = (l2 * bj[4] + l1) * bj[3] + l0;
            const float4 v = m.wbuf[(size_t)j * GMAX3 + li];
            f[0] += v.x;
            f[1] += v.y;
            f[2] += v.z;
            c += v.w;
            if (m.wpar[(size_t)j * GMAX3 + li]) lab = j + 1;
        }
        const int s = (z * m.ny + wrap_near(uy, m.ny)) * m.nx + wrap_near(ux, m.nx);
        m.flag[s] = (uint8_t)(lab | AUX_BIT);
        // bounce-back: no spread force; coverage 1 keeps the fluid step's reaction output
        // (unused then) from counting as lost
        m.ibm[s] = make_float4(f[0], f[1], f[2], m.bb ? 1.0f : c);
    }
}

__global__ void __launch_bounds__(OWN_BLK) k_window_own(MembraneArgs m, int cap) {
    window_own_body(m, blockIdx.y, blockIdx.x, cap);
}

__global__ void __launch_bounds__(256) k_window_combine(MembraneArgs m) {
    window_combine_body(m, blockIdx.y, blockIdx.x);
}

void launch_window_fill(const MembraneArgs &m, hipStream_t st) {
    const int cap = own_cap(m.ncap);
    hipLaunchKernelGGL(k_window_own, dim3(GMAX, m.ncap), dim3(OWN_BLK), 4 * cap * sizeof(unsigned long long),
                       st, m, cap);
    hipLaunchKernelGGL(k_window_combine, dim3(GMAX, m.ncap), dim3(256), 0, st, m);
}

// ------------------------------------------------------------------------------------
// Node update: U_n = sum_x u(x) phi(x - X_n) (wall sites contribute nothing),
// R_n = sum_x r(x) phi(x - X_n) / c(x) over covered sites (the fluid step stores r / c),
// X_n += U_n.  UPD_L = 16 lanes per node, one (x, y) column of 4 sites each, x fastest
// across the lanes, so one load instruction reads 4 contiguous sites of each of 16 rows;
// the 16 column sums are combined by a fixed butterfly.
// ------------------------------------------------------------------------------------
constexpr int UPD_BLK = 256, UPD_L = 16, UPD_NPB = UPD_BLK / UPD_L, UPD_GRID = 1 << 20;

__device__ __forceinline__ void node_update_one(const MembraneArgs &m, int n, int sl) {
    double4 X = m.X[n];
    const int ox = sl & 3, oy = sl >> 2;
    const int bx = (int)floor(X.x) - 1, by = (int)floor(X.y) - 1, bz = (int)floor(X.z) - 1;
    float U[3] = {0.f, 0.f, 0.f}, Rr[3] = {0.f, 0.f, 0.f};
    const float wxy = phi4((float)(X.x - (double)(bx + ox))) *
                      phi4((float)(X.y - (double)(by + oy)));
    const int col = wrap_near(by + oy, m.ny) * m.nx + wrap_near(bx + ox, m.nx);
    // planes bz .. bz + 3, with their slab positions stepped alongside (nz is a multiple
    // of lz, so both wrap together); wall sites contribute nothing.  Every plane's site is
    // a lattice site, so the eight loads are issued before any is used.
    int z = wrap_near(bz, m.nz), zr = m.wall ? slab_pos(z, m.lz) : 1;
    float4 u[4], r[4];
    bool fluid[4];
#pragma unroll
    for (int oz = 0; oz < 4; ++oz) {
        const int s = z * m.ny * m.nx + col;
        u[oz] = m.uo[s];
        r[oz] = m.ro[s];   // reaction / coverage, 0 where uncovered
        fluid[oz] = !(m.wall && zr == 0);
        if (++z == m.nz) z = 0;
        if (++zr == m.lz) zr = 0;
    }
#pragma unroll
    for (int oz = 0; oz < 4; ++oz) {
        if (!fluid[oz]) continue;
        const float w = wxy * phi4((float)(X.z - (double)(bz + oz)));
        U[0] += w * u[oz].x; U[1] += w * u[oz].y; U[2] += w * u[oz].z;
        Rr[0] += w * r[oz].x; Rr[1] += w * r[oz].y; Rr[2] += w * r[oz].z;
    }
    static_assert(UPD_L == 16, "group sums are over 16 lanes");
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        U[d] = group_sum16(U[d]);
        Rr[d] = group_sum16(Rr[d]);
    }
    if (sl == 0) {
        X.x += U[0];
        X.y += U[1];
        X.z += U[2];
        m.X[n] = X;
        m.R[n] = make_float4(Rr[0], Rr[1], Rr[2], 0.f);
    }
}

// block blk of nblk, grid-stride over the nodes
__device__ __forceinline__ void node_update_body(const MembraneArgs &m, int blk, int nblk,
                                                 int ntot) {
    const int sl = threadIdx.x % UPD_L;
    for (int n = blk * UPD_NPB + threadIdx.x / UPD_L; n < ntot; n += nblk * UPD_NPB)
        node_update_one(m, n, sl);
}

__global__ void __launch_bounds__(UPD_BLK) k_node_update(MembraneArgs m, int ntot) {
    node_update_body(m, blockIdx.x, gridDim.x, ntot);
}

int node_update_blocks(int ntot) {
    const int nb = (ntot + UPD_NPB - 1) / UPD_NPB;
    return nb < UPD_GRID ? nb : UPD_GRID;
}

int membrane_blocks(int ntot, int ttot, int *nb_forces) {
    *nb_forces = (ntot + MEM_NPB - 1) / MEM_NPB;
    return *nb_forces + (ttot + MEM_BLK - 1) / MEM_BLK;
}

void launch_node_update(const MembraneArgs &m, int ntot, hipStream_t st) {
    hipLaunchKernelGGL(k_node_update, dim3(node_update_blocks(ntot)), dim3(UPD_BLK), 0, st, m,
                       ntot);
}

// ------------------------------------------------------------------------------------
// The capsule kernels of several simulations in one launch each.  Group g (a simulation
// with capsules) owns capsules grp[g].cap0 .., membrane blocks grp[g].mem0 .. and node
// update blocks grp[g].upd0 .. of the launch; its arguments are tab[g].  The tables are
// read-only for the kernels' lifetime and read through the constant address space.
// ------------------------------------------------------------------------------------
typedef __attribute__((address_space(4))) const int ConstIntM;

__device__ __forceinline__ void load_margs(const MembraneArgs *tab, int g, MembraneArgs &m) {
    static_assert(sizeof(MembraneArgs) % 4 == 0 && sizeof(MGroup) == 28, "word copies");
    ConstIntM *src = (ConstIntM *)(tab + g);
    int *dst = reinterpret_cast<int *>(&m);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(MembraneArgs) / 4); ++i) dst[i] = src[i];
}

// field f of group g (MGroup as 7 ints)
__device__ __forceinline__ int grp_field(const MGroup *grp, int g, int f) {
    return ((ConstIntM *)grp)[7 * g + f];
}

// the last group whose field f (a start index, increasing with g) is <= v
__device__ __forceinline__ int find_group(const MGroup *grp, int ng, int f, int v) {
    int g = 0;
    while (g + 1 < ng && v >= grp_field(grp, g + 1, f)) ++g;
    return g;
}

enum { MG_CAP0 = 0, MG_MEM0 = 1, MG_UPD0 = 2, MG_NTOT = 3, MG_TTOT = 4, MG_NBF = 5, MG_NBU = 6 };

__global__ void __launch_bounds__(RED_BLK) k_capsule_reduce_multi(const MembraneArgs *tab,
                                                                  const MGroup *grp, int ng) {
    const int K = blockIdx.x, g = find_group(grp, ng, MG_CAP0, K);
    MembraneArgs m;
    load_margs(tab, g, m);
    capsule_reduce_body(m, K - grp_field(grp, g, MG_CAP0));
}

__global__ void __launch_bounds__(MEM_BLK) k_membrane_multi(const MembraneArgs *tab,
                                                            const MGroup *grp, int ng) {
    const int B = blockIdx.x, g = find_group(grp, ng, MG_MEM0, B);
    MembraneArgs m;
    load_margs(tab, g, m);
    membrane_body(m, B - grp_field(grp, g, MG_MEM0), grp_field(grp, g, MG_NTOT),
                  grp_field(grp, g, MG_TTOT));
}

__global__ void __launch_bounds__(OWN_BLK) k_window_own_multi(const MembraneArgs *tab,
                                                              const MGroup *grp, int ng, int cap) {
    const int K = blockIdx.y, g = find_group(grp, ng, MG_CAP0, K);
    MembraneArgs m;
    load_margs(tab, g, m);
    window_own_body(m, K - grp_field(grp, g, MG_CAP0), blockIdx.x, cap);
}

__global__ void __launch_bounds__(256) k_window_combine_multi(const MembraneArgs *tab,
                                                              const MGroup *grp, int ng) {
    const int K = blockIdx.y, g = find_group(grp, ng, MG_CAP0, K);
    MembraneArgs m;
    load_margs(tab, g, m);
    window_combine_body(m, K - grp_field(grp, g, MG_CAP0), blockIdx.x);
}

__global__ void __launch_bounds__(UPD_BLK) k_node_update_multi(const MembraneArgs *tab,
                                                               const MGroup *grp, int ng) {
    const int B = blockIdx.x, g = find_group(grp, ng, MG_UPD0, B);
    MembraneArgs m;
    load_margs(tab, g, m);
    node_update_body(m, B - grp_field(grp, g, MG_UPD0), grp_field(grp, g, MG_NBU),
                     grp_field(grp, g, MG_NTOT));
}

void launch_capsule_reduce_multi(const MembraneArgs *tab, const MGroup *grp, int ng,
                                 const MGroupTotals &t, hipStream_t st) {
    hipLaunchKernelGGL(k_capsule_reduce_multi, dim3(t.ncap), dim3(RED_BLK), 0, st, tab, grp, ng);
}

void launch_membrane_multi(const MembraneArgs *tab, const MGroup *grp, int ng,
                           const MGroupTotals &t, hipStream_t st) {
    hipLaunchKernelGGL(k_membrane_multi, dim3(t.mem_blocks), dim3(MEM_BLK), 0, st, tab, grp, ng);
}

void launch_window_fill_multi(const MembraneArgs *tab, const MGroup *grp, int ng,
                              const MGroupTotals &t, hipStream_t st) {
    const int cap = own_cap(t.ncap);
    hipLaunchKernelGGL(k_window_own_multi, dim3(GMAX, t.ncap), dim3(OWN_BLK),
                       4 * cap * sizeof(unsigned long long), st, tab, grp, ng, cap);
    hipLaunchKernelGGL(k_window_combine_multi, dim3(GMAX, t.ncap), dim3(256), 0, st, tab, grp, ng);
}

void launch_node_update_multi(const MembraneArgs *tab, const MGroup *grp, int ng,
                              const MGroupTotals &t, hipStream_t st) {
    hipLaunchKernelGGL(k_node_update_multi, dim3(t.upd_blocks), dim3(UPD_BLK), 0, st, tab, grp,
                       ng);
}

}  // namespace lbmx
