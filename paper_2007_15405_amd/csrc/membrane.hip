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

__device__ __forceinline__ double min_image(double d, int n, bool periodic) {
    return periodic ? d - n * floor(d / n + 0.5) : d;
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

// ------------------------------------------------------------------------------------
// Per capsule (one block of PREP_BLK threads): node mean, enclosed volume (FP64),
// bounding box and the site window; then the node rows of the window: nodes grouped by
// the (y, z) lattice row of floor(X), ordered by node id inside a row.  Fixed reduction
// order throughout.
// ------------------------------------------------------------------------------------
constexpr int PREP_BLK = 1024, PREP_W = PREP_BLK / 64;

__global__ void __launch_bounds__(PREP_BLK) k_capsule_prep(MembraneArgs m) {
    const int k = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const CapDev cd = m.caps[k];
    __shared__ double sd[PREP_W][4];
    __shared__ float smin[PREP_W][3], smax[PREP_W][3];
    __shared__ double cen[3];
    __shared__ int s_lo[3], s_dim[3];
    __shared__ int cnt[ROWS_MAX];
    __shared__ int wsum[PREP_W];
    double sacc[3] = {0, 0, 0};
    float mn[3] = {3e38f, 3e38f, 3e38f}, mx[3] = {-3e38f, -3e38f, -3e38f};
    for (int n = tid; n < cd.nn; n += PREP_BLK) {
        const double4 X = m.X[cd.node0 + n];
        const double p[3] = {X.x, X.y, X.z};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            sacc[d] += p[d];
            const float pf = (float)p[d];
            mn[d] = fminf(mn[d], pf);
            mx[d] = fmaxf(mx[d], pf);
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double v = wave_sum(sacc[d]);
        const float a = wave_min(mn[d]), b = wave_max(mx[d]);
        if (lane == 0) { sd[wid][d] = v; smin[wid][d] = a; smax[wid][d] = b; }
    }
    __syncthreads();
    if (tid < 3) {
        double v = 0;
        for (int w = 0; w < PREP_W; ++w) v += sd[w][tid];
        cen[tid] = v / cd.nn;
    }
    __syncthreads();
    double vol = 0;
    for (int t = tid; t < cd.nt; t += PREP_BLK) {
        const int4 tr = m.tri[cd.tri0 + t];
        const double4 A = m.X[tr.x], B = m.X[tr.y], C = m.X[tr.z];
        const double a[3] = {A.x - cen[0], A.y - cen[1], A.z - cen[2]};
        const double b[3] = {B.x - cen[0], B.y - cen[1], B.z - cen[2]};
        const double c[3] = {C.x - cen[0], C.y - cen[1], C.z - cen[2]};
        vol += (a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
                a[2] * (b[0] * c[1] - b[1] * c[0])) / 6.0;
    }
    vol = wave_sum(vol);
    if (lane == 0) sd[wid][3] = vol;
    __syncthreads();
    if (tid == 0) {
        CapState &cs = m.cst[k];
        double v = 0;
        for (int w = 0; w < PREP_W; ++w) v += sd[w][3];
        cs.vol = v;
        const int nd[3] = {m.nx, m.ny, m.nz};
        for (int d = 0; d < 3; ++d) {
            float a = smin[0][d], b = smax[0][d];
            for (int w = 1; w < PREP_W; ++w) { a = fminf(a, smin[w][d]); b = fmaxf(b, smax[w][d]); }
            cs.cen[d] = cen[d];
            cs.bmin[d] = a;
            cs.bmax[d] = b;
            cs.plo[d] = cs.lo[d];
            cs.pdim[d] = cs.dim[d];
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
    }
    __syncthreads();
    // ---- node rows ----
    const int lo1 = s_lo[1], lo2 = s_lo[2], dim1 = s_dim[1], dim2 = s_dim[2];
    const int rows = dim1 * dim2;
    for (int r = tid; r < rows; r += PREP_BLK) cnt[r] = 0;
    __syncthreads();
    for (int n = tid; n < cd.nn; n += PREP_BLK) {
        const double4 X = m.X[cd.node0 + n];
        const int ry = min(max((int)floor(X.y) - lo1, 0), dim1 - 1);
        const int rz = min(max((int)floor(X.z) - lo2, 0), dim2 - 1);
        atomicAdd(&cnt[rz * dim1 + ry], 1);
    }
    __syncthreads();
    // exclusive scan: each thread owns a contiguous chunk of rows
    const int per = (rows + PREP_BLK - 1) / PREP_BLK;
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
    int base = 0;
    for (int w = 0; w < wid; ++w) base += wsum[w];
    int run = base + incl - local;
    __syncthreads();
    int *rs = m.rowstart + (size_t)k * (ROWS_MAX + 1);
    for (int r = q0; r < q1; ++r) {
        const int c = cnt[r];
        rs[r] = run;
        cnt[r] = run;   // becomes the scatter cursor
        run += c;
    }
    if (tid == 0) rs[rows] = cd.nn;
    __syncthreads();
    int *ids = m.rowids + cd.node0;
    for (int n = tid; n < cd.nn; n += PREP_BLK) {
        const double4 X = m.X[cd.node0 + n];
        const int ry = min(max((int)floor(X.y) - lo1, 0), dim1 - 1);
        const int rz = min(max((int)floor(X.z) - lo2, 0), dim2 - 1);
        ids[atomicAdd(&cnt[rz * dim1 + ry], 1)] = cd.node0 + n;
    }
    __syncthreads();
    // order each row by node id (rows hold a handful of nodes)
    for (int r = tid; r < rows; r += PREP_BLK) {
        const int a = rs[r], b = rs[r + 1];
        for (int i = a + 1; i < b; ++i) {
            const int v = ids[i];
            int j = i - 1;
            while (j >= a && ids[j] > v) { ids[j + 1] = ids[j]; --j; }
            ids[j + 1] = v;
        }
    }
}

void launch_capsule_prep(const MembraneArgs &m, hipStream_t st) {
    hipLaunchKernelGGL(k_capsule_prep, dim3(m.ncap), dim3(PREP_BLK), 0, st, m);
}

// ------------------------------------------------------------------------------------
// Clear the flags of the previous windows; zero the crossing marks of the new windows.
// ------------------------------------------------------------------------------------
__global__ void k_window_clear(MembraneArgs m) {
    const int k = blockIdx.y;
    const CapState cs = m.cst[k];
    const int stride = gridDim.x * blockDim.x, i0 = blockIdx.x * blockDim.x + threadIdx.x;
    const int pv = cs.pdim[0] * cs.pdim[1] * cs.pdim[2];
    for (int i = i0; i < pv; i += stride) {
        const int lx = i % cs.pdim[0], t = i / cs.pdim[0], ly = t % cs.pdim[1], lz = t / cs.pdim[1];
        const int x = wrapm(cs.plo[0] + lx, m.nx), y = wrapm(cs.plo[1] + ly, m.ny),
                  z = wrapm(cs.plo[2] + lz, m.nz);
        m.flag[(z * m.ny + y) * m.nx + x] = 0;
    }
    const int nv = cs.dim[0] * cs.dim[1] * cs.dim[2];
    int *mk = m.marks + (size_t)k * GMAX3;
    for (int i = i0; i < nv; i += stride) mk[i] = 0;
}

void launch_window_clear(const MembraneArgs &m, hipStream_t st) {
    hipLaunchKernelGGL(k_window_clear, dim3(64, m.ncap), dim3(256), 0, st, m);
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

constexpr int MEM_BLK = 128;

__global__ void __launch_bounds__(MEM_BLK) k_membrane_forces(MembraneArgs m, int ntot) {
    __shared__ CapState s_cst[MAX_CAPS];
    for (int j = threadIdx.x; j < m.ncap; j += MEM_BLK) s_cst[j] = m.cst[j];
    __syncthreads();
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= ntot) return;
    const int k = m.node_cap[n];
    const CapDev cd = m.caps[k];
    const double4 X = m.X[n];
    float f[3] = {0.f, 0.f, 0.f}, fh[3] = {0.f, 0.f, 0.f};
    const double vcoef = cd.kv != 0.0f ? -(double)cd.kv * (s_cst[k].vol - cd.v0) / cd.v0 : 0.0;
    for (int e = m.ntri_off[n]; e < m.ntri_off[n + 1]; ++e) {
        const int t = m.ntri[e] / 3, corner = m.ntri[e] - 3 * (m.ntri[e] / 3);
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
    const float xi = m.hertz_xi, d0 = m.hertz_d0;
    if (m.wall && xi > 0.f) {
        const float d = (float)(X.z - (double)m.plane_z);
        if (d < d0) fh[2] += xi * (d0 - d) * sqrtf(d0 - d);
    }
    if (xi > 0.f) {
        // particle-particle pairs: only the node rows of another capsule's window whose
        // (y, z) lattice row lies within delta0 of this node can hold a partner
        const bool per[3] = {true, true, !m.wall};
        const int nd[3] = {m.nx, m.ny, m.nz};
        const double p[3] = {X.x, X.y, X.z};
        for (int j = 0; j < m.ncap; ++j) {
            if (j == k) continue;
            const CapState &cj = s_cst[j];
            double pl[3];   // this node in the periodic image closest to window j
            bool far = false;
            for (int d = 0; d < 3; ++d) {
                const double c = cj.lo[d] + 0.5 * cj.dim[d];
                pl[d] = c + min_image(p[d] - c, nd[d], per[d]);
                if (2.0 * (cj.dim[d] + 2.0 * d0 + 2.0) <= nd[d] &&
                    (pl[d] < cj.lo[d] - d0 || pl[d] > cj.lo[d] + cj.dim[d] + d0))
                    far = true;
            }
            if (far) continue;
            // the row search sees one periodic image of each partner; it is exact while the
            // window plus the cut-off is smaller than half the box, else scan all rows
            bool small = true;
            for (int d = 0; d < 3; ++d)
                if (per[d] && 2.0 * (cj.dim[d] + 2.0 * d0 + 2.0) > nd[d]) small = false;
            const int ry0 = small ? max((int)floor(pl[1] - d0) - cj.lo[1], 0) : 0;
            const int ry1 = small ? min((int)floor(pl[1] + d0) - cj.lo[1], cj.dim[1] - 1) : cj.dim[1] - 1;
            const int rz0 = small ? max((int)floor(pl[2] - d0) - cj.lo[2], 0) : 0;
            const int rz1 = small ? min((int)floor(pl[2] + d0) - cj.lo[2], cj.dim[2] - 1) : cj.dim[2] - 1;
            const int *rs = m.rowstart + (size_t)j * (ROWS_MAX + 1);
            const int node0 = m.caps[j].node0;
            for (int rz = rz0; rz <= rz1; ++rz)
                for (int ry = ry0; ry <= ry1; ++ry) {
                    const int row = rz * cj.dim[1] + ry;
                    for (int e = rs[row]; e < rs[row + 1]; ++e) {
                        const double4 Y = m.X[m.rowids[node0 + e]];
                        const double r[3] = {min_image(p[0] - Y.x, nd[0], per[0]),
                                             min_image(p[1] - Y.y, nd[1], per[1]),
                                             min_image(p[2] - Y.z, nd[2], per[2])};
                        const double dd = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                        if (dd < d0 && dd > 0.0) {
                            const float g = (float)(d0 - dd);
                            const float mag = xi * g * sqrtf(g);
                            for (int d = 0; d < 3; ++d) fh[d] += (float)(mag * r[d] / dd);
                        }
                    }
                }
        }
    }
    if (cd.anchor_k != 0.0f) {
        const CapState &cs = s_cst[k];
        const double ka = (double)cd.anchor_k / cd.nn;
        for (int d = 0; d < 3; ++d) f[d] += (float)(-ka * (cs.cen[d] - cd.c0[d]));
    }
    const float4 R = m.R[n];
    m.F[n] = make_float4(f[0] + fh[0] + R.x, f[1] + fh[1] + R.y, f[2] + fh[2] + R.z, 0.f);
    m.Fh[n] = make_float4(fh[0], fh[1], fh[2], 0.f);
}

void launch_membrane_forces(const MembraneArgs &m, int ntot, hipStream_t st) {
    hipLaunchKernelGGL(k_membrane_forces, dim3((ntot + MEM_BLK - 1) / MEM_BLK), dim3(MEM_BLK), 0, st,
                       m, ntot);
}

// ------------------------------------------------------------------------------------
// Crossing marks: for every lattice column inside a triangle's xy projection (top-left
// rule on shared edges; zero-area projections skipped), the crossing height z_c is the
// barycentric interpolation of the vertex heights; sites m >= ceil(z_c) lie above it.
// The mark at (column, ceil(z_c)) is toggled; a prefix XOR up the column gives the
// inside parity.  Decisions use FP32-rounded positions evaluated in double.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double edgef(double ux, double uy, double vx, double vy, double px,
                                        double py) {
    return (vx - ux) * (py - uy) - (vy - uy) * (px - ux);
}
__device__ __forceinline__ bool edge_in(double w, double ux, double uy, double vx, double vy) {
    return w > 0.0 || (w == 0.0 && ((vy < uy) || (vy == uy && vx < ux)));
}

__global__ void __launch_bounds__(256) k_label_marks(MembraneArgs m, int ttot) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ttot) return;
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
    int *mk = m.marks + (size_t)k * GMAX3;
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
            atomicXor(&mk[(lz * cs.dim[1] + ly) * cs.dim[0] + lx], 1);
        }
}

void launch_label_marks(const MembraneArgs &m, int ttot, hipStream_t st) {
    hipLaunchKernelGGL(k_label_marks, dim3((ttot + 255) / 256), dim3(256), 0, st, m, ttot);
}

// ------------------------------------------------------------------------------------
// Window fill, in two kernels.
//
// k_window_own: one block per (capsule k, plane of its window).  Every node whose kernel
// support reaches the plane (a contiguous run of the row-sorted ids) adds its 4 x 4 sites
// of the plane, F_n phi(x - X_n) and phi(x - X_n), into an LDS plane buffer.  The sums
// are 64-bit fixed point (2^-40 units), so the atomic adds are exact and the result does
// not depend on their order.  Then one thread per column carries the crossing parity up
// the column.  Results go to capsule k's window buffers.
//
// k_window_combine: per window site, the sum over every window holding the site, in
// capsule order, of those buffers; the side label is the highest capsule whose parity is
// odd.  Wall sites receive nothing.  Sites in several windows are written with the same
// values by each of them.
// ------------------------------------------------------------------------------------
constexpr int FILL_COLS = 2048;     // LDS plane capacity: windows up to 2048 columns (x * y)
constexpr float FIX_SCALE = 1099511627776.0f;   // 2^40

__device__ __forceinline__ long long to_fix(float v) { return __float2ll_rn(v * FIX_SCALE); }
__device__ __forceinline__ float from_fix(long long v) {
    return (float)((double)v * (1.0 / 1099511627776.0));
}

__global__ void __launch_bounds__(256) k_window_own(MembraneArgs m) {
    const int k = blockIdx.y, lz = blockIdx.x, tid = threadIdx.x;
    const CapState ck = m.cst[k];
    if (lz >= ck.dim[2]) return;
    const int dx = ck.dim[0], dy = ck.dim[1], ncol = dx * dy;
    __shared__ unsigned long long s_acc[4][FILL_COLS];
    if (ncol > FILL_COLS) {   // uniform over the block
        if (tid == 0) atomicOr(&m.status[ST_WIDE], 1);
        return;
    }
    float4 *wb = m.wbuf + (size_t)k * GMAX3 + (size_t)lz * ncol;
    uint8_t *wp = m.wpar + (size_t)k * GMAX3 + (size_t)lz * ncol;
    unsigned long long *acc = &s_acc[0][0];
    constexpr int stride = FILL_COLS;
    for (int i = tid; i < ncol; i += blockDim.x)
        for (int d = 0; d < 4; ++d) acc[d * stride + i] = 0ull;
    __syncthreads();
    // nodes with floor(Z) - lo_z in [lz - 2, lz + 1] reach this plane
    const int r0 = max(lz - 2, 0), r1 = min(lz + 1, ck.dim[2] - 1);
    const int *rs = m.rowstart + (size_t)k * (ROWS_MAX + 1);
    const int e0 = rs[r0 * dy], e1 = rs[(r1 + 1) * dy];
    const int node0 = m.caps[k].node0;
    const double zs = (double)(ck.lo[2] + lz);
    for (int w = tid; w < (e1 - e0) * 4; w += blockDim.x) {
        const int e = e0 + (w >> 2), oy = w & 3;
        const int n = m.rowids[node0 + e];
        const double4 X = m.X[n];
        const float4 F = m.F[n];
        const double fx = floor(X.x), fy = floor(X.y);
        const float wz = phi4((float)(X.z - zs));
        const int bx = (int)fx - 1 - ck.lo[0], by = (int)fy - 1 - ck.lo[1];
        const int ly = by + oy;
        const float wy = phi4((float)(X.y - fy) + (float)(1 - oy));
        if (ly < 0 || ly >= dy) continue;
        for (int ox = 0; ox < 4; ++ox) {
            const int lx = bx + ox;
            if (lx < 0 || lx >= dx) continue;
            const float wgt = phi4((float)(X.x - fx) + (float)(1 - ox)) * wy * wz;
            const int col = ly * dx + lx;
            atomicAdd(&acc[col], (unsigned long long)to_fix(wgt * F.x));
            atomicAdd(&acc[stride + col], (unsigned long long)to_fix(wgt * F.y));
            atomicAdd(&acc[2 * stride + col], (unsigned long long)to_fix(wgt * F.z));
            atomicAdd(&acc[3 * stride + col], (unsigned long long)to_fix(wgt));
        }
    }
    __syncthreads();
    const int *mk = m.marks + (size_t)k * GMAX3;
    for (int col = tid; col < ncol; col += blockDim.x) {
        int par = 0;
        for (int q = 0; q <= lz; ++q) par ^= mk[q * ncol + col];
        wb[col] = make_float4(from_fix((long long)acc[col]), from_fix((long long)acc[stride + col]),
                              from_fix((long long)acc[2 * stride + col]),
                              from_fix((long long)acc[3 * stride + col]));
        wp[col] = (uint8_t)(par & 1);
    }
}

__global__ void __launch_bounds__(256) k_window_combine(MembraneArgs m) {
    const int k = blockIdx.y, lz = blockIdx.x, tid = threadIdx.x;
    const CapState ck = m.cst[k];
    if (lz >= ck.dim[2]) return;
    const int dx = ck.dim[0], dy = ck.dim[1];
    __shared__ int s_win[MAX_CAPS + 1];
    __shared__ CapState s_cs[MAX_CAPS];
    __shared__ int s_n;
    // windows meeting this plane of window k, in capsule order (k included)
    if (tid == 0) {
        const int nd[3] = {m.nx, m.ny, m.nz};
        const int blo[3] = {ck.lo[0], ck.lo[1], ck.lo[2] + lz};
        const int bdim[3] = {dx, dy, 1};
        int n = 0;
        for (int j = 0; j < m.ncap; ++j) {
            const CapState cj = m.cst[j];
            bool meet = true;
            for (int d = 0; d < 3; ++d) {
                const int off = wrapm(cj.lo[d] - blo[d], nd[d]);
                meet = meet && (off < bdim[d] || off + cj.dim[d] > nd[d]);
            }
            if (meet) { s_cs[n] = cj; s_win[n++] = j; }
        }
        s_n = n;
    }
    __syncthreads();
    const int nwin = s_n;
    const int nd[3] = {m.nx, m.ny, m.nz};
    for (int col = tid; col < dx * dy; col += blockDim.x) {
        const int lx = col % dx, ly = col / dx;
        const int u[3] = {ck.lo[0] + lx, ck.lo[1] + ly, ck.lo[2] + lz};
        const int z = wrapm(u[2], m.nz);
        if (m.wall && z == 0) continue;
        int lab = 0;
        float f[3] = {0.f, 0.f, 0.f}, c = 0.f;
        for (int i = 0; i < nwin; ++i) {
            const int j = s_win[i];
            const CapState &cj = s_cs[i];
            int l[3];
            bool in = true;
            for (int d = 0; d < 3; ++d) {
                l[d] = wrapm(u[d] - cj.lo[d], nd[d]);
                in = in && l[d] < cj.dim[d];
            }
            if (!in) continue;
            const int li = (l[2] * cj.dim[1] + l[1]) * cj.dim[0] + l[0];
            const float4 v = m.wbuf[(size_t)j * GMAX3 + li];
            f[0] += v.x;
            f[1] += v.y;
            f[2] += v.z;
            c += v.w;
            if (m.wpar[(size_t)j * GMAX3 + li]) lab = j + 1;
        }
        const int x = wrapm(u[0], m.nx), y = wrapm(u[1], m.ny);
        const int s = (z * m.ny + y) * m.nx + x;
        m.flag[s] = (uint8_t)(lab | AUX_BIT);
        m.ibm[s] = make_float4(f[0], f[1], f[2], c);
    }
}

void launch_window_fill(const MembraneArgs &m, hipStream_t st) {
    hipLaunchKernelGGL(k_window_own, dim3(GMAX, m.ncap), dim3(256), 0, st, m);
    hipLaunchKernelGGL(k_window_combine, dim3(GMAX, m.ncap), dim3(256), 0, st, m);
}

// ------------------------------------------------------------------------------------
// Node update: U_n = sum_x u(x) phi(x - X_n) (wall sites contribute nothing),
// R_n = sum_x r(x) phi(x - X_n) / c(x) over covered sites (the fluid step stores r / c),
// X_n += U_n.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_node_update(MembraneArgs m, int ntot) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= ntot) return;
    double4 X = m.X[n];
    const int b[3] = {(int)floor(X.x) - 1, (int)floor(X.y) - 1, (int)floor(X.z) - 1};
    float U[3] = {0.f, 0.f, 0.f}, Rr[3] = {0.f, 0.f, 0.f};
    float wx[4], wy[4], wz[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        wx[o] = phi4((float)(X.x - (double)(b[0] + o)));
        wy[o] = phi4((float)(X.y - (double)(b[1] + o)));
        wz[o] = phi4((float)(X.z - (double)(b[2] + o)));
    }
    for (int oz = 0; oz < 4; ++oz) {
        const int z = wrapm(b[2] + oz, m.nz);
        if (m.wall && z == 0) continue;
        for (int oy = 0; oy < 4; ++oy) {
            const int y = wrapm(b[1] + oy, m.ny);
            for (int ox = 0; ox < 4; ++ox) {
                const int x = wrapm(b[0] + ox, m.nx);
                const int s = (z * m.ny + y) * m.nx + x;
                const float w = wx[ox] * wy[oy] * wz[oz];
                const float4 u = m.uo[s];
                const float4 r = m.ro[s];   // reaction / coverage, 0 where uncovered
                U[0] += w * u.x; U[1] += w * u.y; U[2] += w * u.z;
                Rr[0] += w * r.x; Rr[1] += w * r.y; Rr[2] += w * r.z;
            }
        }
    }
    X.x += U[0];
    X.y += U[1];
    X.z += U[2];
    m.X[n] = X;
    m.R[n] = make_float4(Rr[0], Rr[1], Rr[2], 0.f);
}

void launch_node_update(const MembraneArgs &m, int ntot, hipStream_t st) {
    hipLaunchKernelGGL(k_node_update, dim3((ntot + 255) / 256), dim3(256), 0, st, m, ntot);
}

}  // namespace lbmx
