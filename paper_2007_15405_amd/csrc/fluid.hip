// fluid.hip -- lattice Boltzmann kernels of liblbm (gfx950).
//
// Populations are stored structure-of-arrays, population-major: f[c][i][z][y][x], so a
// wavefront touching 64 consecutive x reads 64 consecutive values of one population.
// Streaming is "pull": the step at site x gathers f*_i(x - e_i) from the previous state;
// where x - e_i is the wall layer, half-way bounce-back returns f*_{opp(i)}(x).
//
// The populations of a component are read through two buffer resources (populations
// 0..9 and 10..18; base in scalar registers) with the population's start inside its part
// as the scalar offset and a 32-bit byte offset per lane: no 64-bit address arithmetic
// on the vector ALU, and few scalar registers (four resources per population array
// instead of one per population, which the compiler would otherwise keep live across
// the z march).  Out-of-range offsets read 0 and drop stores instead of faulting.  The
// byte size of 10 populations of one component must fit 32 bits.
#include <algorithm>

#include "lbm_internal.h"

namespace lbmx {

__device__ __forceinline__ int wrap1(int a, int n) {
    a += (a < 0) ? n : 0;
    a -= (a >= n) ? n : 0;
    return a;
}

__device__ __forceinline__ int wrapn(int a, int n) {
    a %= n;
    return a < 0 ? a + n : a;
}

// psi = 1 - exp(-rho / rho0) (Section 3.1), hardware exp2-based exponential
__device__ __forceinline__ float psi_of(float rho, float inv_rho0) {
    return 1.0f - __expf(-rho * inv_rho0);
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ------------------------------------------------------------------------------------
// Population access
// ------------------------------------------------------------------------------------
// weight of population q in the shift of storage S (wshift: mass-exact FP32 weights)
template <int S> __device__ __forceinline__ constexpr float wsh(int q) {
    return S == 3 ? wshift(q) : wq(q);
}

template <int S> struct Pop {
    using T = typename Codec<S>::T;
    static constexpr int QH = 10;   // populations in the first part of a component
    // resource of the part holding population qg (component qg / Q): [QH or Q - QH][N] of T
    __device__ static inline __amdgpu_buffer_rsrc_t res(const void *f, int qg, int N) {
        const int hi = qg % Q >= QH;
        return __builtin_amdgcn_make_buffer_rsrc(
            (void *)((const T *)f + (size_t)((qg / Q) * Q + hi * QH) * N), (short)0,
            (int)((uint32_t)(hi ? Q - QH : QH) * (uint32_t)N * sizeof(T)), 0x00020000);
    }
    // byte offset of population qg inside its part
    __device__ static inline uint32_t qoff(int qg, int N) {
        const int q = qg % Q;
        return (uint32_t)(q >= QH ? q - QH : q) * (uint32_t)N * (uint32_t)sizeof(T);
    }
    __device__ static inline float load(const void *f, int qg, int N, uint32_t site, float sh) {
        const __amdgpu_buffer_rsrc_t r = res(f, qg, N);
        if constexpr (sizeof(T) == 4) {
            return Codec<S>::dec(__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                               r, site * 4u, qoff(qg, N), 0)),
                                 sh);
        } else {
            const uint16_t v = __builtin_amdgcn_raw_buffer_load_b16(r, site * 2u, qoff(qg, N), 0);
            return Codec<S>::dec(__builtin_bit_cast(T, v), sh);
        }
    }
    // the stored value itself, not shifted back (the pipelined kernels add the shifts of a
    // site's populations once; storage 3 decodes with its source site's density later)
    __device__ static inline float load_raw(const void *f, int qg, int N, uint32_t site) {
        static_assert(sizeof(T) == 2, "16-bit storage");
        const uint16_t v = __builtin_amdgcn_raw_buffer_load_b16(res(f, qg, N), site * 2u,
                                                                 qoff(qg, N), 0);
        return Codec<S>::val(__builtin_bit_cast(T, v));
    }
    // the stored bits, zero-extended (FP16: pairs of them feed the packed dot products)
    __device__ static inline uint32_t load_bits(const void *f, int qg, int N, uint32_t site) {
        static_assert(sizeof(T) == 2, "16-bit storage");
        return __builtin_amdgcn_raw_buffer_load_b16(res(f, qg, N), site * 2u, qoff(qg, N), 0);
    }
    // stores are non-temporal: the new state is not read again in this step, and keeping
    // it out of L2 leaves room for the source rows that neighbouring tiles pull again
    static constexpr int STORE_NT = 2;
    __device__ static inline void store(void *f, int qg, int N, uint32_t site, float v, float sh) {
        store_enc(f, qg, N, site, Codec<S>::enc(v, sh));
    }
    // store an encoded value
    __device__ static inline void store_enc(void *f, int qg, int N, uint32_t site, T e) {
        const __amdgpu_buffer_rsrc_t r = res(f, qg, N);
        if constexpr (sizeof(T) == 4)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, e), r, site * 4u,
                                                  qoff(qg, N), STORE_NT);
        else
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, e), r, site * 2u,
                                                  qoff(qg, N), STORE_NT);
    }
};

// Pull the 19 post-streaming populations of both components at site (x, y, z):
// f_i(x) = f*_i(x - e_i), or f*_{opp(i)}(x) where x - e_i is the wall (half-way bounce-back).
// wall_lo: the site below is the wall; wall_hi: the site above is the wall.
template <int S, bool SUM_ONLY>
__device__ __forceinline__ void pull(const void *f, int N, int x, int y, int z, int nx, int ny,
                                     int nz, bool wall_lo, bool wall_hi, float sh0, float sh1,
                                     float (&fl)[2][Q], float &r0, float &r1) {
    const int xm = wrap1(x - 1, nx), xp = wrap1(x + 1, nx);
    const int ym = wrap1(y - 1, ny), yp = wrap1(y + 1, ny);
    const int zm = wrap1(z - 1, nz), zp = wrap1(z + 1, nz);
    const int self = (z * ny + y) * nx + x;
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int xs = CX[q] == 0 ? x : (CX[q] > 0 ? xm : xp);
        const int ys = CY[q] == 0 ? y : (CY[q] > 0 ? ym : yp);
        const int zs = CZ[q] == 0 ? z : (CZ[q] > 0 ? zm : zp);
        const bool bb = (CZ[q] > 0 && wall_lo) || (CZ[q] < 0 && wall_hi);
        const uint32_t src = bb ? self : (uint32_t)((zs * ny + ys) * nx + xs);
        const int qq = bb ? OPP[q] : q;
        const float v0 = Pop<S>::load(f, qq, N, src, wsh<S>(q) * sh0);
        const float v1 = Pop<S>::load(f, Q + qq, N, src, wsh<S>(q) * sh1);
        if (!SUM_ONLY) {
            fl[0][q] = v0;
            fl[1][q] = v1;
        }
        a0 += v0;
        a1 += v1;
    }
    r0 = a0;
    r1 = a1;
}

// Issue the 38 pulls of site (x, y, z) into registers without consuming them, so the
// loads stay in flight while other work runs.  16-bit storages pull the stored values:
// with a constant shift the shifts of a site's populations add rho_s sum_i w_i to its
// density and nothing to its momentum (sum_i w_i e_i = 0), which the caller adds once;
// storage 3 decodes each value with its source site's density.  Links that cross the wall first read the
// (unused) wall site; a wave-uniform fix-up then replaces them by the bounced
// population f*_{opp(i)}(x), keeping the load stream free of per-link branches.
template <int S>
__device__ __forceinline__ void pull_issue(const void *f, int N, int x, int y, int z, int nx,
                                           int ny, int nz, bool wall_lo, bool wall_hi, float sh0,
                                           float sh1, float (&fl)[2][Q]) {
    const int xm = wrap1(x - 1, nx), xp = wrap1(x + 1, nx);
    const int ym = wrap1(y - 1, ny), yp = wrap1(y + 1, ny);
    const int zm = wrap1(z - 1, nz), zp = wrap1(z + 1, nz);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int xs = CX[q] == 0 ? x : (CX[q] > 0 ? xm : xp);
        const int ys = CY[q] == 0 ? y : (CY[q] > 0 ? ym : yp);
        const int zs = CZ[q] == 0 ? z : (CZ[q] > 0 ? zm : zp);
        const uint32_t src = (uint32_t)((zs * ny + ys) * nx + xs);
        if constexpr (S == 1 || S == 2) {   // stored bits, summed later by packed dot products
            fl[0][q] = __uint_as_float(Pop<S>::load_bits(f, q, N, src));
            fl[1][q] = __uint_as_float(Pop<S>::load_bits(f, Q + q, N, src));
        } else if constexpr (S != 0) {   // stored values; the shifts are applied later
            fl[0][q] = Pop<S>::load_raw(f, q, N, src);
            fl[1][q] = Pop<S>::load_raw(f, Q + q, N, src);
        } else {
            fl[0][q] = Pop<S>::load(f, q, N, src, wsh<S>(q) * sh0);
            fl[1][q] = Pop<S>::load(f, Q + q, N, src, wsh<S>(q) * sh1);
        }
    }
    if (wall_lo || wall_hi) {
        const uint32_t self = (uint32_t)((z * ny + y) * nx + x);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if ((CZ[q] > 0 && wall_lo) || (CZ[q] < 0 && wall_hi)) {
                if constexpr (S == 1 || S == 2) {
                    fl[0][q] = __uint_as_float(Pop<S>::load_bits(f, OPP[q], N, self));
                    fl[1][q] = __uint_as_float(Pop<S>::load_bits(f, Q + OPP[q], N, self));
                } else if constexpr (S != 0) {
                    fl[0][q] = Pop<S>::load_raw(f, OPP[q], N, self);
                    fl[1][q] = Pop<S>::load_raw(f, Q + OPP[q], N, self);
                } else {
                    fl[0][q] = Pop<S>::load(f, OPP[q], N, self, wsh<S>(q) * sh0);
                    fl[1][q] = Pop<S>::load(f, Q + OPP[q], N, self, wsh<S>(q) * sh1);
                }
            }
        }
    }
}

// Momentum sum_i f_i e_i; pairs (q, q+1) are opposite links for odd q.
__device__ __forceinline__ void moments(const float (&f)[Q], float &jx, float &jy, float &jz) {
    jx = ((f[1] - f[2]) + (f[5] - f[6])) + ((f[7] - f[8]) + (f[11] - f[12])) + (f[13] - f[14]);
    jy = ((f[3] - f[4]) + (f[5] - f[6])) + ((f[8] - f[7]) + (f[15] - f[16])) + (f[17] - f[18]);
    jz = ((f[9] - f[10]) + (f[11] - f[12])) + ((f[14] - f[13]) + (f[15] - f[16])) + (f[18] - f[17]);
}

// 16-bit storages (FP16, BF16): density and momentum of one component from the stored bits
// of its 19 populations (zero-extended in each float's bits).  Opposite links (q, q + 1)
// share one register as a 16-bit pair, and each sum takes a packed dot product with FP32
// accumulation: (1, 1) for the density, (1, -1) or (-1, 1) for a momentum component, the
// same differences of opposite links as moments().  Products of stored values with +-1 are
// exact; only the accumulation rounds.
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf162v __attribute__((ext_vector_type(2)));
template <int S> struct PairDot;
template <> struct PairDot<1> {
    using V = half2v;
    __device__ static inline V vec(float a, float b) { return V{(_Float16)a, (_Float16)b}; }
    __device__ static inline float dot(V p, V c, float acc) {
        return __builtin_amdgcn_fdot2(p, c, acc, false);
    }
    __device__ static inline float rest(uint32_t bits) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)bits);
    }
};
template <> struct PairDot<2> {
    using V = bf162v;
    __device__ static inline V vec(float a, float b) { return V{(__bf16)a, (__bf16)b}; }
    __device__ static inline float dot(V p, V c, float acc) {
        return __builtin_amdgcn_fdot2_f32_bf16(p, c, acc, false);
    }
    __device__ static inline float rest(uint32_t bits) { return __uint_as_float(bits << 16); }
};
template <int S> __device__ __forceinline__ typename PairDot<S>::V pair_of(const float (&f)[Q], int q) {
    return __builtin_bit_cast(typename PairDot<S>::V,
                              __float_as_uint(f[q]) | (__float_as_uint(f[q + 1]) << 16));
}
template <int S> __device__ __forceinline__ float pair_density(const float (&f)[Q]) {
    using D = PairDot<S>;
    const typename D::V one = D::vec(1.0f, 1.0f);
    float r = D::rest(__float_as_uint(f[0]));
#pragma unroll
    for (int q = 1; q < Q; q += 2) r = D::dot(pair_of<S>(f, q), one, r);
    return r;
}
template <int S>
__device__ __forceinline__ void pair_moments(const float (&f)[Q], float &r, float &jx, float &jy,
                                             float &jz) {
    using D = PairDot<S>;
    using V = typename D::V;
    const V pl = D::vec(1.0f, -1.0f), mi = D::vec(-1.0f, 1.0f);
    r = pair_density<S>(f);
    const V p1 = pair_of<S>(f, 1), p3 = pair_of<S>(f, 3), p5 = pair_of<S>(f, 5);
    const V p7 = pair_of<S>(f, 7), p9 = pair_of<S>(f, 9), p11 = pair_of<S>(f, 11);
    const V p13 = pair_of<S>(f, 13), p15 = pair_of<S>(f, 15), p17 = pair_of<S>(f, 17);
    jx = D::dot(p1, pl, 0.f);
    jx = D::dot(p5, pl, jx);
    jx = D::dot(p7, pl, jx);
    jx = D::dot(p11, pl, jx);
    jx = D::dot(p13, pl, jx);
    jy = D::dot(p3, pl, 0.f);
    jy = D::dot(p5, pl, jy);
    jy = D::dot(p7, mi, jy);
    jy = D::dot(p15, pl, jy);
    jy = D::dot(p17, pl, jy);
    jz = D::dot(p9, pl, 0.f);
    jz = D::dot(p11, pl, jz);
    jz = D::dot(p13, mi, jz);
    jz = D::dot(p15, pl, jz);
    jz = D::dot(p17, mi, jz);
}

// Stencil sum sum_i w_i psi_i e_i of eq. shanchen from the 18 neighbour values
// pn[q - 1] (q = 1..18), evaluated as differences of opposite links.
__device__ __forceinline__ void stencil(const float (&pn)[Q - 1], float wa, float wd, float &sx,
                                        float &sy, float &sz) {
    const float d1 = pn[0] - pn[1], d3 = pn[2] - pn[3], d5 = pn[4] - pn[5], d7 = pn[6] - pn[7];
    const float d9 = pn[8] - pn[9], d11 = pn[10] - pn[11], d13 = pn[12] - pn[13];
    const float d15 = pn[14] - pn[15], d17 = pn[16] - pn[17];
    sx = wa * d1 + wd * ((d5 + d7) + (d11 + d13));
    sy = wa * d3 + wd * ((d5 - d7) + (d15 + d17));
    sz = wa * d9 + wd * ((d11 - d13) + (d15 - d17));
}

// Density and momentum of both components (the same summation order everywhere).
__device__ __forceinline__ void site_moments(const float (&fl)[2][Q], float (&m)[8]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        float r = 0.f;
#pragma unroll
        for (int q = 0; q < Q; ++q) r += fl[c][q];
        m[4 * c] = r;
        moments(fl[c], m[4 * c + 1], m[4 * c + 2], m[4 * c + 3]);
    }
}

// Forces, BGK collision (eq. method:boltzmann) towards eq. lbm:equilibrium at the
// Shan-Chen shifted velocity, store; writes the physical velocity and the reaction
// on window sites.  m: rho, j of both components; S0/S1: stencil sums over the partner
// component of 0 and 1.  KEEPF: relax the pulled populations fl towards f^eq with
// 1/tau; otherwise tau = 1 for both components and f* = f^eq needs only the moments.
template <int S, bool KEEPF>
__device__ __forceinline__ void collide_store(const FluidArgs &a, const float (&fl)[2][Q],
                                              const float (&m)[8], uint32_t s, uint8_t fg,
                                              float psi0, float psi1, const float (&S0)[3],
                                              const float (&S1)[3], const float (&rx)[3]) {
    const float rho[2] = {m[0], m[4]};
    const float jx[2] = {m[1], m[5]}, jy[2] = {m[2], m[6]}, jz[2] = {m[3], m[7]};
    if (!(rho[0] >= 0.f) || !(rho[1] >= 0.f) || !(rho[0] + rho[1] < 3.0e38f))
        atomicOr(&a.status[ST_UNSTABLE], 1);
    const float rt = rho[0] + rho[1];
    const float irt = rt > 0.f ? rcp(rt) : 0.f;
    const bool aux = (fg & AUX_BIT) != 0;
    float fb[4] = {0.f, 0.f, 0.f, 0.f};
    if (aux) {
        const float4 v = a.ibm[s];
        fb[0] = v.x; fb[1] = v.y; fb[2] = v.z; fb[3] = v.w;
    }
    const float m0 = rho[0] * irt, m1 = rho[1] * irt;
    float F0[3], F1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        F0[d] = -a.G * psi0 * S0[d] + m0 * fb[d] + rho[0] * a.g[d];
        F1[d] = -a.G * psi1 * S1[d] + m1 * fb[d] + rho[1] * a.g[d];
    }
    // Shan-Chen common velocity u' = sum_c j^c/tau^c / sum_c rho^c/tau^c
    const float den = rho[0] * a.inv_tau[0] + rho[1] * a.inv_tau[1];
    const float id = den > 0.f ? rcp(den) : 0.f;
    const float up0 = (jx[0] * a.inv_tau[0] + jx[1] * a.inv_tau[1]) * id;
    const float up1 = (jy[0] * a.inv_tau[0] + jy[1] * a.inv_tau[1]) * id;
    const float up2 = (jz[0] * a.inv_tau[0] + jz[1] * a.inv_tau[1]) * id;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const float *Fc = c == 0 ? F0 : F1;
        const float k = rho[c] > 0.f ? a.tau[c] * rcp(rho[c]) : 0.f;
        const float u0 = up0 + k * Fc[0], u1 = up1 + k * Fc[1], u2 = up2 + k * Fc[2];
        const float uu = 1.5f * (u0 * u0 + u1 * u1 + u2 * u2);
        const float om = a.inv_tau[c];
        const float sh = a.shift[c];
        // f^eq of opposite links: symmetric part A, antisymmetric part B; the rest
        // population takes rho - sum so the rounded weights add no mass
        float feq[Q], sum = 0.f;
#pragma unroll
        for (int q = 1; q < Q; q += 2) {
            const float w = wq(q) * rho[c];
            const float eu = CX[q] * u0 + CY[q] * u1 + CZ[q] * u2;
            const float A = w * (1.0f + 4.5f * eu * eu - uu);
            const float B = 3.0f * w * eu;
            feq[q] = A + B;
            feq[q + 1] = A - B;
            sum += feq[q] + feq[q + 1];
        }
        feq[0] = rho[c] - sum;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float fs = KEEPF ? fl[c][q] + om * (feq[q] - fl[c][q]) : feq[q];
            Pop<S>::store(a.fout, c * Q + q, a.N, s, fs, wsh<S>(q) * sh);
        }
    }
    if (aux) {
        // window sites: physical velocity with the kernel coverage c(x) in .w, and the
        // reaction already divided by c(x) (0 where c = 0)
        a.uo[s] = make_float4((jx[0] + jx[1] + 0.5f * (F0[0] + F1[0])) * irt,
                              (jy[0] + jy[1] + 0.5f * (F0[1] + F1[1])) * irt,
                              (jz[0] + jz[1] + 0.5f * (F0[2] + F1[2])) * irt, fb[3]);
        const float ic = fb[3] > 0.f ? 1.0f / fb[3] : 0.f;
        a.ro[s] = a.bb ? make_float4(rho[0], rho[1], psi0, psi1)
                       : make_float4(rx[0] * ic, rx[1] * ic, rx[2] * ic, 0.f);
    }
    if ((rx[0] != 0.f || rx[1] != 0.f || rx[2] != 0.f) && !(aux && fb[3] > 0.f))
        atomicAdd(&a.status[ST_LOST], 1);
}

// Neighbour psi across labels (eq. shanchen with the decoupling of Section 3.1): the
// neighbour's own psi on the same side; across the wall or a membrane the partner's
// density at x itself plus the wetting offset (+ for component 0, - for component 1).
// With zero offsets that value is psi at x itself (psi0, psi1), so no exponential is
// evaluated; the result is the same to the bit.
// Returns the stencil sums and the reaction G sum_c psi^c (cross-membrane part).  Where
// every membrane-crossing link of a site substitutes the site's own psi (always without
// wetting offsets), the reaction G sum over those links of w_i e_i (psi0 psi1 + psi1 psi0)
// is 2 G psi0 psi1 times the stencil of the crossing links' indicator; that form is taken
// whenever it holds, so a site gets the same bits whether or not other capsules of the run
// carry offsets.
__device__ __forceinline__ void sc_general(const FluidArgs &a, const float *cap_drho,
                                           const float (&p0n)[Q - 1], const float (&p1n)[Q - 1],
                                           const int (&nlab)[Q - 1], int lab, float rho0,
                                           float rho1, float psi0, float psi1, float (&S0)[3],
                                           float (&S1)[3], float (&rx)[3]) {
    float e0[Q - 1], e1[Q - 1];
    bool anycross = false, own = true;
    if (a.zero_drho) {
        // zero offsets everywhere: the substituted value is the site's own psi
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            const bool cr = nlab[q - 1] != lab;
            e0[q - 1] = cr ? psi0 : p0n[q - 1];
            e1[q - 1] = cr ? psi1 : p1n[q - 1];
            anycross = anycross || (cr && nlab[q - 1] != LABEL_WALL);
        }
    } else {
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            e0[q - 1] = p0n[q - 1];
            e1[q - 1] = p1n[q - 1];
            if (nlab[q - 1] != lab) {
                const int nl = nlab[q - 1];
                const float dr = nl == LABEL_WALL ? a.wall_drho : cap_drho[(nl != 0 ? nl : lab) - 1];
                e0[q - 1] = psi_of(fmaxf(rho0 + dr, 0.f), a.inv_rho0);
                e1[q - 1] = psi_of(fmaxf(rho1 - dr, 0.f), a.inv_rho0);
                anycross = anycross || nl != LABEL_WALL;
                own = own && (nl == LABEL_WALL || dr == 0.f);
            }
        }
    }
    stencil(e1, a.ws_axis, a.ws_diag, S0[0], S0[1], S0[2]);
    stencil(e0, a.ws_axis, a.ws_diag, S1[0], S1[1], S1[2]);
    rx[0] = rx[1] = rx[2] = 0.f;
    if (anycross && own) {
        float c[Q - 1];
#pragma unroll
        for (int q = 1; q < Q; ++q)
            c[q - 1] = nlab[q - 1] != lab && nlab[q - 1] != LABEL_WALL ? 1.f : 0.f;
        float K[3];
        stencil(c, a.ws_axis, a.ws_diag, K[0], K[1], K[2]);
        const float g2 = 2.0f * a.G * psi0 * psi1;
#pragma unroll
        for (int d = 0; d < 3; ++d) rx[d] = g2 * K[d];
    } else if (anycross) {
        float c1[Q - 1], c0[Q - 1];
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            const bool cr = nlab[q - 1] != lab && nlab[q - 1] != LABEL_WALL;
            c1[q - 1] = cr ? e1[q - 1] : 0.f;
            c0[q - 1] = cr ? e0[q - 1] : 0.f;
        }
        float C0[3], C1[3];
        stencil(c1, a.ws_axis, a.ws_diag, C0[0], C0[1], C0[2]);
        stencil(c0, a.ws_axis, a.ws_diag, C1[0], C1[1], C1[2]);
#pragma unroll
        for (int d = 0; d < 3; ++d) rx[d] = a.G * (psi0 * C0[d] + psi1 * C1[d]);
    }
}

// ------------------------------------------------------------------------------------
// f* = f^eq(rho, 0) = w_i rho at every fluid site (eq. lbm:equilibrium at rest).
// ------------------------------------------------------------------------------------
template <int S>
__global__ void k_init_eq(const double *__restrict__ rho, void *f, int nx, int ny, int nz,
                          int wall, int lz, float sh0, float sh1, float *rsite) {
    const int N = nx * ny * nz;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const int z = s / (nx * ny);
    const bool solid = wall && slab_pos(z, lz) == 0;
    if constexpr (S == 3) {   // shift by the site's own density: w_i rho stores as 0
        sh0 = solid ? 0.0f : (float)rho[s];
        sh1 = solid ? 0.0f : (float)rho[N + s];
        rsite[s] = sh0;
        rsite[N + s] = sh1;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double w = (double)wq(q);
        Pop<S>::store(f, q, N, s, solid ? 0.0f : (float)(w * rho[s]), wsh<S>(q) * sh0);
        Pop<S>::store(f, Q + q, N, s, solid ? 0.0f : (float)(w * rho[N + s]), wsh<S>(q) * sh1);
    }
}

template <int S>
void launch_init_eq(const double *rho_dev, void *f, int nx, int ny, int nz, int wall, int lz,
                    float s0, float s1, float *rsite, hipStream_t st) {
    const int N = nx * ny * nz;
    hipLaunchKernelGGL(k_init_eq<S>, dim3((N + 255) / 256), dim3(256), 0, st, rho_dev, f, nx, ny,
                       nz, wall, lz, s0, s1, rsite);
}

// ------------------------------------------------------------------------------------
// Two-kernel variant: pass 1 writes psi of every site, pass 2 gathers the neighbour psi
// from memory.  Same per-site arithmetic as the fused kernel.
// ------------------------------------------------------------------------------------
template <int S>
__global__ void __launch_bounds__(256) k_density(FluidArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.N) return;
    const int x = s % a.nx, t = s / a.nx, y = t % a.ny, z = t / a.ny;
    const int zr = slab_pos(z, a.lz);
    if (a.wall && zr == 0) return;
    float fl[2][Q], r0, r1;
    pull<S, true>(a.fin, a.N, x, y, z, a.nx, a.ny, a.nz, a.wall && zr == 1,
                  a.wall && zr == a.lz - 1, a.shift[0], a.shift[1], fl, r0, r1);
    a.psi[s] = psi_of(r0, a.inv_rho0);
    a.psi[a.N + s] = psi_of(r1, a.inv_rho0);
}

template <int S, bool KEEPF>
__global__ void __launch_bounds__(256) k_collide(FluidArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.N) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz, N = a.N;
    const int x = s % nx, t = s / nx, y = t % ny, z = t / ny;
    const int zr = slab_pos(z, a.lz);
    if (a.wall && zr == 0) return;
    float fl[2][Q], r0, r1, m[8];
    pull<S, false>(a.fin, N, x, y, z, nx, ny, nz, a.wall && zr == 1, a.wall && zr == a.lz - 1,
                   a.shift[0], a.shift[1], fl, r0, r1);
    site_moments(fl, m);
    const uint8_t fg = a.flag[s];
    const int lab = fg & LABEL_MASK;
    float p0n[Q - 1], p1n[Q - 1];
    int nlab[Q - 1];
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        const int xn = wrap1(x + CX[q], nx), yn = wrap1(y + CY[q], ny), zn = wrap1(z + CZ[q], nz);
        const int sn = (zn * ny + yn) * nx + xn;
        const bool solid_n = a.wall && slab_pos(zn, a.lz) == 0;
        nlab[q - 1] = solid_n ? LABEL_WALL : (a.flag[sn] & LABEL_MASK);
        p0n[q - 1] = solid_n ? 0.f : a.psi[sn];
        p1n[q - 1] = solid_n ? 0.f : a.psi[N + sn];
    }
    float S0[3], S1[3], rx[3];
    sc_general(a, a.cap_drho, p0n, p1n, nlab, lab, m[0], m[4], a.psi[s], a.psi[N + s], S0, S1, rx);
    collide_store<S, KEEPF>(a, fl, m, (uint32_t)s, fg, a.psi[s], a.psi[N + s], S0, S1, rx);
}

template <int S>
void launch_fluid(const FluidArgs &a, hipStream_t st) {
    const dim3 grid((a.N + 255) / 256), blk(256);
    hipLaunchKernelGGL(k_density<S>, grid, blk, 0, st, a);
    if (a.keepf)
        hipLaunchKernelGGL((k_collide<S, true>), grid, blk, 0, st, a);
    else
        hipLaunchKernelGGL((k_collide<S, false>), grid, blk, 0, st, a);
}

// ------------------------------------------------------------------------------------
// Fused single-read fluid step.  A workgroup owns a TX x TY tile of lattice columns and
// marches up a chunk of z planes.  At plane p every thread pulls the 38 populations of
// its site once (kept in registers), computes psi^c and publishes psi and the site flag
// into a three-plane LDS ring that also holds a one-site halo ring around the tile (halo
// sites only sum their pulled populations).  After a barrier the previous plane p-1 is
// collided from registers and the LDS ring, and stored.  A tile-plane whose three LDS
// planes carry no label, window or wall takes the plain path (no label tests).  Each LDS
// position holds the periodically wrapped site, so ragged tiles and boxes smaller than
// a tile need no special case.  Blocks are renumbered so that consecutive tiles run on
// one XCD and share its L2 for the halo re-reads.
// ------------------------------------------------------------------------------------
constexpr uint8_t WALL_FLAG = (uint8_t)LABEL_WALL;

template <int S, int TX, int TY, bool KEEPF>
__global__ void __launch_bounds__(TX * TY) k_fused(FluidArgs a, int zc, int tiles_x, int tiles_y,
                                                   int nblocks) {
    constexpr int KQ = KEEPF ? Q : 1;   // populations held between pull and collision
    constexpr int NT = TX * TY, LX = TX + 2, LY = TY + 2, NL = LX * LY, NH = NL - NT;
    static_assert(NH <= NT, "halo ring larger than the tile");
    __shared__ float s_psi[3][2][NL];
    __shared__ uint8_t s_flag[3][NL];

    // XCD-aware renumbering: hardware block b runs on XCD b % 8; give each XCD a
    // contiguous run of logical tiles
    const int per = (int)gridDim.x / 8;
    const int L = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (L >= nblocks) return;
    const int bx = L % tiles_x, t2 = L / tiles_x, by = t2 % tiles_y, bz = t2 / tiles_y;
    const int nx = a.nx, ny = a.ny, nz = a.nz, N = a.N;
    const int x0 = bx * TX, y0 = by * TY;
    int z0, z1;
    zchunk_range(bz, zc, a.zoff, nz, z0, z1);
    const float sh0 = a.shift[0], sh1 = a.shift[1];

    const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
    const int li = (ly + 1) * LX + (lx + 1);
    const int ix = wrapn(x0 + lx, nx), iy = wrapn(y0 + ly, ny);
    const bool valid = (x0 + lx < nx) && (y0 + ly < ny);
    // halo ring position of this thread (if any): rows -1 and TY, then columns -1 and TX
    int hi = -1, hx = 0, hy = 0;
    if (tid < NH) {
        int h = tid;
        if (h < LX) { hx = h - 1; hy = -1; }
        else if (h < 2 * LX) { hx = h - LX - 1; hy = TY; }
        else { h -= 2 * LX; hy = h >> 1; hx = (h & 1) ? TX : -1; }
        hi = (hy + 1) * LX + (hx + 1);
        hx = wrapn(x0 + hx, nx);
        hy = wrapn(y0 + hy, ny);
    }

    // per site state carried from the pull of plane p to its collision: the moments and,
    // with KEEPF, the populations
    float fa[2][KQ], fb[2][KQ], ma[8], mb[8];
#pragma unroll
    for (int q = 0; q < KQ; ++q) { fa[0][q] = fa[1][q] = fb[0][q] = fb[1][q] = 0.f; }
#pragma unroll
    for (int i = 0; i < 8; ++i) { ma[i] = mb[i] = 0.f; }
    int busy1 = 1, busy2 = 1;   // LDS planes p-1, p-2 carry labels, windows or walls

    // one plane: pull plane p into (nxt, mn), collide plane p - 1 from (cur, mc)
    auto plane = [&](int p, float (&cur)[2][KQ], float (&mc)[8], float (&nxt)[2][KQ],
                     float (&mn)[8]) {
        const int slot = (p - z0 + 1) % 3;
        const int pz = wrapn(p, nz), pr = slab_pos(pz, a.lz);
        const bool solid = a.wall && pr == 0;
        const bool wlo = a.wall && pr == 1, whi = a.wall && pr == a.lz - 1;
        uint8_t fg_me;
        {
            float fl[2][Q], r0 = 0.f, r1 = 0.f;
            if (!solid) {
                pull<S, false>(a.fin, N, ix, iy, pz, nx, ny, nz, wlo, whi, sh0, sh1, fl, r0, r1);
                site_moments(fl, mn);
                if (KEEPF) {
#pragma unroll
                    for (int q = 0; q < KQ; ++q) { nxt[0][q] = fl[0][q]; nxt[1][q] = fl[1][q]; }
                }
            }
            s_psi[slot][0][li] = psi_of(r0, a.inv_rho0);
            s_psi[slot][1][li] = psi_of(r1, a.inv_rho0);
            fg_me = solid ? WALL_FLAG : a.flag[(pz * ny + iy) * nx + ix];
            s_flag[slot][li] = fg_me;
        }
        uint8_t fg_h = 0;
        if (hi >= 0) {
            float r0 = 0.f, r1 = 0.f, dummy[2][Q];
            if (!solid)
                pull<S, true>(a.fin, N, hx, hy, pz, nx, ny, nz, wlo, whi, sh0, sh1, dummy, r0, r1);
            s_psi[slot][0][hi] = psi_of(r0, a.inv_rho0);
            s_psi[slot][1][hi] = psi_of(r1, a.inv_rho0);
            fg_h = solid ? WALL_FLAG : a.flag[(pz * ny + hy) * nx + hx];
            s_flag[slot][hi] = fg_h;
        }
        const int busy0 = __syncthreads_or((fg_me | fg_h) != 0);
        const int pc = p - 1;
        const int cz = wrapn(pc, nz);
        if (pc >= z0 && valid && !(a.wall && slab_pos(cz, a.lz) == 0)) {
            const int sc = (p - z0) % 3, sd = (p - z0 + 2) % 3;   // planes p - 1 and p - 2
            const uint32_t s = (uint32_t)((cz * ny + iy) * nx + ix);
            const float psi0 = s_psi[sc][0][li], psi1 = s_psi[sc][1][li];
            float p0n[Q - 1], p1n[Q - 1];
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                const int ns = CZ[q] == 0 ? sc : (CZ[q] > 0 ? slot : sd);
                const int nl = li + CX[q] + CY[q] * LX;
                p0n[q - 1] = s_psi[ns][0][nl];
                p1n[q - 1] = s_psi[ns][1][nl];
            }
            float S0[3], S1[3], rx[3] = {0.f, 0.f, 0.f};
            uint8_t fg = 0;
            if (!(busy0 | busy1 | busy2)) {
                stencil(p1n, a.ws_axis, a.ws_diag, S0[0], S0[1], S0[2]);
                stencil(p0n, a.ws_axis, a.ws_diag, S1[0], S1[1], S1[2]);
            } else {
                fg = s_flag[sc][li];
                int nlab[Q - 1];
#pragma unroll
                for (int q = 1; q < Q; ++q) {
                    const int ns = CZ[q] == 0 ? sc : (CZ[q] > 0 ? slot : sd);
                    nlab[q - 1] = s_flag[ns][li + CX[q] + CY[q] * LX] & LABEL_MASK;
                }
                sc_general(a, a.cap_drho, p0n, p1n, nlab, fg & LABEL_MASK, mc[0], mc[4], psi0, psi1,
                           S0, S1, rx);
            }
            float fl[2][Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                fl[0][q] = KEEPF ? cur[0][q % KQ] : 0.f;
                fl[1][q] = KEEPF ? cur[1][q % KQ] : 0.f;
            }
            collide_store<S, KEEPF>(a, fl, mc, s, fg, psi0, psi1, S0, S1, rx);
        }
        busy2 = busy1;
        busy1 = busy0;
        __syncthreads();
    };

    int p = z0 - 1;
    for (; p + 1 <= z1; p += 2) {
        plane(p, fb, mb, fa, ma);
        plane(p + 1, fa, ma, fb, mb);
    }
    if (p <= z1) plane(p, fb, mb, fa, ma);
}

// ------------------------------------------------------------------------------------
// Software-pipelined fused step for tau = 1 (f* = f^eq needs only the moments).  Each
// wave issues the pulls of plane p+2 (its tile site and, for the first NH threads, a
// halo site), collides plane p from the LDS ring while those loads are in flight, then
// folds them into moments and psi of plane p+2.  A four-plane LDS ring (p-1 .. p+2)
// needs one barrier per plane; whether a plane holds any label, window or wall is
// reduced per wave with a ballot and published next to the ring.
//
// WX: the tile spans whole rows (TX == nx).  The x wrap then stays inside the tile: the
// halo is the two neighbouring rows only (one site per thread), and the ring columns -1
// and TX are copies of columns TX - 1 and 0.  Whole rows also make every store of a
// plane a run of TX * 4 contiguous bytes per population, which the memory system
// serves better than shorter runs.
// ------------------------------------------------------------------------------------
// Forces and the equilibrium velocity of both components at one site (tau = 1), and the
// outputs of window sites.  m: rho, j of both components; S0/S1: stencil sums over the
// partner component of 0 and 1; ue[c]: u^eq of component c.
__device__ __forceinline__ void eq_velocity(const FluidArgs &a, const float (&m)[8], uint32_t s,
                                            uint8_t fg, const float4 &ibv, float psi0,
                                            float psi1, const float (&S0)[3],
                                            const float (&S1)[3], const float (&rx)[3],
                                            float (&ue)[2][3]) {
    const float rho[2] = {m[0], m[4]};
    const float jx[2] = {m[1], m[5]}, jy[2] = {m[2], m[6]}, jz[2] = {m[3], m[7]};
    if (!(rho[0] >= 0.f) || !(rho[1] >= 0.f) || !(rho[0] + rho[1] < 3.0e38f))
        atomicOr(&a.status[ST_UNSTABLE], 1);
    const float rt = rho[0] + rho[1];
    const float irt = rt > 0.f ? rcp(rt) : 0.f;
    const bool aux = (fg & AUX_BIT) != 0;
    float fb[4] = {0.f, 0.f, 0.f, 0.f};
    if (aux) {
        fb[0] = ibv.x; fb[1] = ibv.y; fb[2] = ibv.z; fb[3] = ibv.w;
    }
    const float m0 = rho[0] * irt, m1 = rho[1] * irt;
    float F0[3], F1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        F0[d] = -a.G * psi0 * S0[d] + m0 * fb[d] + rho[0] * a.g[d];
        F1[d] = -a.G * psi1 * S1[d] + m1 * fb[d] + rho[1] * a.g[d];
    }
    const float den = rho[0] * a.inv_tau[0] + rho[1] * a.inv_tau[1];
    const float id = den > 0.f ? rcp(den) : 0.f;
    const float up0 = (jx[0] * a.inv_tau[0] + jx[1] * a.inv_tau[1]) * id;
    const float up1 = (jy[0] * a.inv_tau[0] + jy[1] * a.inv_tau[1]) * id;
    const float up2 = (jz[0] * a.inv_tau[0] + jz[1] * a.inv_tau[1]) * id;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const float *Fc = c == 0 ? F0 : F1;
        const float k = rho[c] > 0.f ? a.tau[c] * rcp(rho[c]) : 0.f;
        ue[c][0] = up0 + k * Fc[0];
        ue[c][1] = up1 + k * Fc[1];
        ue[c][2] = up2 + k * Fc[2];
    }
    if (aux) {
        // window sites: physical velocity with the kernel coverage c(x) in .w, and the
        // reaction already divided by c(x) (0 where c = 0)
        a.uo[s] = make_float4((jx[0] + jx[1] + 0.5f * (F0[0] + F1[0])) * irt,
                              (jy[0] + jy[1] + 0.5f * (F0[1] + F1[1])) * irt,
                              (jz[0] + jz[1] + 0.5f * (F0[2] + F1[2])) * irt, fb[3]);
        const float ic = fb[3] > 0.f ? 1.0f / fb[3] : 0.f;
        a.ro[s] = a.bb ? make_float4(rho[0], rho[1], psi0, psi1)
                       : make_float4(rx[0] * ic, rx[1] * ic, rx[2] * ic, 0.f);
    }
    if ((rx[0] != 0.f || rx[1] != 0.f || rx[2] != 0.f) && !(aux && fb[3] > 0.f))
        atomicAdd(&a.status[ST_LOST], 1);
}

// The stored values (Codec<S>::T) of f^eq (eq. lbm:equilibrium) of one component at a site
// of density rho and equilibrium velocity u.  Opposite links q, q + 1 (q odd) are
// evaluated as a symmetric part A and an antisymmetric part B (eq_link, q ascending); the
// rest population (eq_rest) takes rho minus the others so the rounded weights add no mass.
// acc carries the running sums between them.
struct EqAcc {
    float a = 0.f, b = 0.f;
};

template <int S>
__device__ __forceinline__ void eq_link(int q, float rho, float u0, float u1, float u2, float uu,
                                        float sh, EqAcc &acc, typename Codec<S>::T &eq,
                                        typename Codec<S>::T &eo) {
    using T = typename Codec<S>::T;
    const float eu = CX[q] * u0 + CY[q] * u1 + CZ[q] * u2;
    if constexpr (S == 3) {
        // relative deviation from the rest equilibrium at this site's new density (stored
        // beside the populations): d_i = f_i^eq / (ws_i rho) - 1
        //     = (w_i / ws_i - 1) + (w_i / ws_i)(3 e.u + 4.5 (e.u)^2 - 1.5 u.u),
        // computed without forming f_i; acc sums the rounded values of axis (a) and diagonal
        // (b) links
        const float r = wq(q) / wshift(q);
        const float A = 4.5f * eu * eu - uu, B = 3.0f * eu;
        eq = (T)((r - 1.0f) + r * (A + B));
        eo = (T)((r - 1.0f) + r * (A - B));
        if (is_axis(q)) acc.a += (float)eq + (float)eo;
        else acc.b += (float)eq + (float)eo;
    } else {
        const float w = wq(q) * rho;
        const float A = w * (1.0f + 4.5f * eu * eu - uu);
        const float B = 3.0f * w * eu;
        const float fq = A + B, fo = A - B;
        acc.a += fq + fo;
        eq = Codec<S>::enc(fq, wsh<S>(q) * sh);
        eo = Codec<S>::enc(fo, wsh<S>(q) * sh);
    }
}

template <int S>
__device__ __forceinline__ typename Codec<S>::T eq_rest(float rho, float sh, const EqAcc &acc) {
    if constexpr (S == 3) {
        // the rest deviation that makes sum_i ws_i rho (1 + d_i) = rho with the others as
        // rounded, so a site's stored mass carries one FP16 rounding of that second-order
        // value (mass conservation)
        constexpr float ka = wshift(1) / wshift(0), kd = wshift(5) / wshift(0);
        return (typename Codec<S>::T)(-(ka * acc.a + kd * acc.b));
    } else {
        return Codec<S>::enc(rho - acc.a, wsh<S>(0) * sh);
    }
}

__device__ __forceinline__ float eq_uu(const float (&u)[3]) {
    return 1.5f * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

template <int S>
__device__ __forceinline__ void eq_encode(const FluidArgs &a, int c, float rho,
                                          const float (&u)[3],
                                          typename Codec<S>::T (&e)[Q]) {
    const float uu = eq_uu(u);
    const float sh = S == 3 ? 0.f : a.shift[c];
    EqAcc acc;
#pragma unroll
    for (int q = 1; q < Q; q += 2) eq_link<S>(q, rho, u[0], u[1], u[2], uu, sh, acc, e[q], e[q + 1]);
    e[0] = eq_rest<S>(rho, sh, acc);
}

// Forces, BGK collision with tau = 1 (f* = f^eq) and store of one site.
template <int S>
__device__ __forceinline__ void collide_store_eq(const FluidArgs &a, const float (&m)[8],
                                                 uint32_t s, uint8_t fg, const float4 &ibv,
                                                 float psi0, float psi1, const float (&S0)[3],
                                                 const float (&S1)[3], const float (&rx)[3]) {
    float ue[2][3];
    eq_velocity(a, m, s, fg, ibv, psi0, psi1, S0, S1, rx, ue);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        typename Codec<S>::T e[Q];
        eq_encode<S>(a, c, m[4 * c], ue[c], e);
#pragma unroll
        for (int q = 0; q < Q; ++q) Pop<S>::store_enc(a.fout, c * Q + q, a.N, s, e[q]);
        if constexpr (S == 3) a.rout[c * a.N + s] = m[4 * c];
    }
}

// One workgroup's tile: logical block L of a lattice tiled tiles_x x tiles_y x (z chunks
// of zc planes).  RT: whole rows chosen at run time, tx = nx (16 .. 128) by
// ty = NT / nx rows; the LDS ring is sized for TX x TY, which holds every such tile, and
// the NT - tx * ty threads left over idle (they pull nothing and park their ring entry
// in the unused end of the ring).
template <int S, int TX, int TY, bool WX, bool RT = false>
__device__ __forceinline__ void pipe_tile(const FluidArgs &a, int L, int zc, int tiles_x,
                                          int tiles_y) {
    constexpr int NT = TX * TY, NLC = (TX + 2) * (TY + 2);
    constexpr int NW = NT / 64;
    static_assert((WX ? 2 * TX : NLC - NT) <= NT && NT % 64 == 0, "tile shape");
    static_assert(!RT || (WX && TX == 128 && TY == 4), "run-time tiles are whole rows");
    const int tx = RT ? a.nx : TX, ty = RT ? NT / a.nx : TY;
    const int LX = tx + 2, NL = LX * (ty + 2);
    const int NH = WX ? 2 * tx : NL - NT;
    __shared__ float s_psi[4][2][NLC];
    __shared__ uint8_t s_flag[4][NLC];
    __shared__ int s_busy[4][NW];
    __shared__ float s_drho[MAX_CAPS];
    // storage 3: the last step's site densities over the tile and a 2-site ring (the sources
    // of the tile's and the halo's pulls), planes p - 1 .. p + 3 of the march in a 4-plane
    // ring (slot of plane z: (z - z0 + 2) & 3); whole-row tiles wrap in x instead
    constexpr bool LOC = S == 3;
    constexpr int NR_MAX = WX ? TX * (TY + 4) : (TX + 4) * (TY + 4);
    constexpr int RPT = (NR_MAX + NT - 1) / NT;
    __shared__ float s_rho[LOC ? 4 : 1][2][LOC ? NR_MAX : 1];

    const int bx = L % tiles_x, t2 = L / tiles_x, by = t2 % tiles_y, bz = t2 / tiles_y;
    const int nx = a.nx, ny = a.ny, nz = a.nz, N = a.N;
    const int x0 = bx * tx, y0 = by * ty;
    int z0, z1;
    zchunk_range(bz, zc, a.zoff, nz, z0, z1);
    const float sh0 = a.shift[0], sh1 = a.shift[1];
    // storages 1 and 2: the pulls are the stored values f_i - w_i rho_s; a site's density
    // takes the sum of its populations' shifts, as encoded (FP32 products w_i rho_s)
    constexpr bool CONST_SHIFT = S == 1 || S == 2;
    float ssum0 = 0.f, ssum1 = 0.f;
    if constexpr (CONST_SHIFT) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            ssum0 += wsh<S>(q) * sh0;
            ssum1 += wsh<S>(q) * sh1;
        }
    }

    const int tid = threadIdx.x, lx = tid % tx, ly = tid / tx;
    const int wave = tid >> 6, lane = tid & 63;
    const bool act = !RT || tid < tx * ty;   // RT: threads beyond the tile idle
    const int li = act ? (ly + 1) * LX + (lx + 1) : NL + (tid - tx * ty);
    const int ix = wrapn(x0 + lx, nx), iy = wrapn(y0 + ly, ny);
    const bool valid = act && (x0 + lx < nx) && (y0 + ly < ny);
    int hi = -1, hx = 0, hy = 0, hxl = 0, hyl = 0;
    if (tid < NH) {
        int h = tid;
        if (WX) { hx = h % tx; hy = h < tx ? -1 : ty; }
        else if (h < LX) { hx = h - 1; hy = -1; }
        else if (h < 2 * LX) { hx = h - LX - 1; hy = ty; }
        else { h -= 2 * LX; hy = h >> 1; hx = (h & 1) ? tx : -1; }
        hi = (hy + 1) * LX + (hx + 1);
        hxl = hx;   // tile coordinates of the halo site
        hyl = hy;
        hx = wrapn(x0 + hx, nx);
        hy = wrapn(y0 + hy, ny);
    }
    const int RW = WX ? tx : tx + 4, NR = RW * (ty + 4);
    float rreg[2][RPT];
    // storage 3: load the region of plane z into registers, then into its ring slot
    auto rho_issue = [&](int z) {
        if constexpr (LOC) {
            const int pz = wrapn(z, nz);
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const int i = tid + k * NT;
                rreg[0][k] = rreg[1][k] = 0.f;
                if (i < NR) {
                    const int rx = i % RW, ry = i / RW;
                    const int gx = WX ? rx : wrapn(x0 - 2 + rx, nx), gy = wrapn(y0 - 2 + ry, ny);
                    const int sg = (pz * ny + gy) * nx + gx;
                    rreg[0][k] = a.rin[sg];
                    rreg[1][k] = a.rin[N + sg];
                }
            }
        }
    };
    auto rho_store = [&](int z) {
        if constexpr (LOC) {
            const int slot = (z - z0 + 2) & 3;
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const int i = tid + k * NT;
                if (i < NR) {
                    s_rho[slot][0][i] = rreg[0][k];
                    s_rho[slot][1][i] = rreg[1][k];
                }
            }
        }
    };
    // storage 3: the pulls of the site at tile coordinates (sx, sy) in plane p were loaded
    // as stored; decode each with ws_q rho of its source (the site itself where it bounced
    // back at the wall)
    auto decode = [&](float (&f)[2][Q], int sx, int sy, int p, bool wlo, bool whi) {
        if constexpr (LOC) {
            const int s0 = (p - z0 + 2) & 3, sm = (p - z0 + 1) & 3, sp = (p - z0 + 3) & 3;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const bool bb = (CZ[q] > 0 && wlo) || (CZ[q] < 0 && whi);
                const int slot = (bb || CZ[q] == 0) ? s0 : (CZ[q] > 0 ? sm : sp);
                const int ox = bb ? sx : sx - CX[q], oy = bb ? sy : sy - CY[q];
                const int idx = WX ? wrap1(ox, tx) + (oy + 2) * RW : (ox + 2) + (oy + 2) * RW;
                f[0][q] = Codec<S>::dec((typename Codec<S>::T)f[0][q],
                                        wshift(q) * s_rho[slot][0][idx]);
                f[1][q] = Codec<S>::dec((typename Codec<S>::T)f[1][q],
                                        wshift(q) * s_rho[slot][1][idx]);
            }
        }
    };
    // WX: ring positions that also hold this thread's value (the wrapped columns)
    const int li_w = !WX || !act ? -1 : (lx == tx - 1 ? li - tx : (lx == 0 ? li + tx : -1));
    const int hi_w = !WX || hi < 0 ? -1
                                   : ((hi % LX) == tx ? hi - tx : ((hi % LX) == 1 ? hi + tx : -1));

    for (int i = tid; i < MAX_CAPS; i += NT) s_drho[i] = a.cap_drho[i];
    // slab position of a plane (uniform), stepped along with the planes instead of divided
    const int lz = a.lz;

    // publish psi, flags and the busy bit of plane p (slab position pr) from the pulled
    // populations
    auto publish = [&](int p, int pr, bool solid, float (&fl)[2][Q], float (&hf)[2][Q],
                       uint8_t fl_me, uint8_t fl_h, float (&m)[8], uint8_t &fg_out) {
        const int slot = (p - z0 + 4) & 3;
        if constexpr (LOC) {
            if (!solid) {
                const bool wlo = a.wall && pr == 1, whi = a.wall && pr == lz - 1;
                if (act) decode(fl, lx, ly, p, wlo, whi);
                if (hi >= 0) decode(hf, hxl, hyl, p, wlo, whi);
            }
        }
        float r0 = 0.f, r1 = 0.f, h0 = 0.f, h1 = 0.f;
        if (!solid && act) {
            if constexpr (S == 1 || S == 2) {
                pair_moments<S>(fl[0], m[0], m[1], m[2], m[3]);
                pair_moments<S>(fl[1], m[4], m[5], m[6], m[7]);
                r0 = m[0];
                r1 = m[4];
                if (hi >= 0) {
                    h0 = pair_density<S>(hf[0]);
                    h1 = pair_density<S>(hf[1]);
                }
            } else {
#pragma unroll
                for (int q = 0; q < Q; ++q) { r0 += fl[0][q]; r1 += fl[1][q]; }
                site_moments(fl, m);
                if (hi >= 0) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) { h0 += hf[0][q]; h1 += hf[1][q]; }
                }
            }
            if constexpr (CONST_SHIFT) {   // the populations' shifts, once per site
                r0 += ssum0;
                r1 += ssum1;
                h0 += ssum0;
                h1 += ssum1;
                m[0] = r0;
                m[4] = r1;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) m[i] = 0.f;
        }
        const uint8_t fg_me = !act ? 0 : (solid ? WALL_FLAG : fl_me);
        fg_out = fg_me;
        const float ps0 = psi_of(r0, a.inv_rho0), ps1 = psi_of(r1, a.inv_rho0);
        s_psi[slot][0][li] = ps0;
        s_psi[slot][1][li] = ps1;
        s_flag[slot][li] = fg_me;
        if constexpr (WX) {
            if (li_w >= 0) {
                s_psi[slot][0][li_w] = ps0;
                s_psi[slot][1][li_w] = ps1;
                s_flag[slot][li_w] = fg_me;
            }
        }
        uint8_t fg_h = 0;
        if (hi >= 0) {
            fg_h = solid ? WALL_FLAG : fl_h;
            const float hp0 = psi_of(h0, a.inv_rho0), hp1 = psi_of(h1, a.inv_rho0);
            s_psi[slot][0][hi] = hp0;
            s_psi[slot][1][hi] = hp1;
            s_flag[slot][hi] = fg_h;
            if constexpr (WX) {
                if (hi_w >= 0) {
                    s_psi[slot][0][hi_w] = hp0;
                    s_psi[slot][1][hi_w] = hp1;
                    s_flag[slot][hi_w] = fg_h;
                }
            }
        }
        const bool any = __builtin_amdgcn_ballot_w64((fg_me | fg_h) != 0) != 0;
        if (lane == 0) s_busy[slot][wave] = any ? 1 : 0;
    };

    auto fwd = [&](int r, int k) { r += k; return r >= lz ? r - lz : r; };
    // issue the pulls and flag reads of plane p at slab position pr (tile site, and the
    // halo site of the first NH threads)
    auto issue = [&](int p, int pr, float (&fl)[2][Q], float (&hf)[2][Q], uint8_t &g_me,
                     uint8_t &g_h) {
        const int pz = wrapn(p, nz);
        const bool wlo = a.wall && pr == 1, whi = a.wall && pr == lz - 1;
        g_me = g_h = 0;
        if (!(a.wall && pr == 0)) {
            if (act) {
                g_me = a.flag[(pz * ny + iy) * nx + ix];
                pull_issue<S>(a.fin, N, ix, iy, pz, nx, ny, nz, wlo, whi, sh0, sh1, fl);
            }
            if (hi >= 0) {
                g_h = a.flag[(pz * ny + hy) * nx + hx];
                pull_issue<S>(a.fin, N, hx, hy, pz, nx, ny, nz, wlo, whi, sh0, sh1, hf);
            }
        }
    };
    auto load_plane = [&](int p, int pr, float (&m)[8], uint8_t &fg_out) {
        float fl[2][Q], hf[2][Q];
        uint8_t g_me, g_h;
        issue(p, pr, fl, hf, g_me, g_h);
        publish(p, pr, a.wall && pr == 0, fl, hf, g_me, g_h, m, fg_out);
    };

    float m0[8], m1[8], m2[8];   // moments of planes p, p+1, p+2
    uint8_t fgx, fg0, fg1;       // this thread's flag in planes z0 - 1, z0 and p + 1
    // the spread force of a window site in a plane, or zeros elsewhere
    auto ibm_load = [&](int p, uint8_t fg) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (fg & AUX_BIT) v = a.ibm[(wrapn(p, nz) * ny + iy) * nx + ix];
        return v;
    };
    int rz = slab_pos(z0, lz);   // slab position of plane p
    if constexpr (LOC) {         // the sources of planes z0 - 1 .. z0 + 1
        for (int z = z0 - 2; z <= z0; ++z) {
            rho_issue(z);
            rho_store(z);
        }
        __syncthreads();
    }
    load_plane(z0 - 1, fwd(rz, lz - 1), m2, fgx);
    if constexpr (LOC) {
        rho_issue(z0 + 1);
        rho_store(z0 + 1);
        __syncthreads();
    }
    load_plane(z0, rz, m0, fg0);
    if constexpr (LOC) {
        rho_issue(z0 + 2);
        rho_store(z0 + 2);
        __syncthreads();
    }
    load_plane(z0 + 1, fwd(rz, 1), m1, fg1);
    if constexpr (LOC) {
        rho_issue(z0 + 3);
        rho_store(z0 + 3);
    }
    float4 ib0 = ibm_load(z0, fg0);   // the spread force of this thread's site in plane p
    __syncthreads();
    for (int p = z0; p < z1; ++p, rz = fwd(rz, 1)) {
        // the spread force of plane p + 1 is loaded before the pulls of plane p + 2: the
        // wait for those pulls (publication of p + 2) then covers it, and a window site
        // costs no wait of its own
        const float4 ibn = p + 1 < z1 ? ibm_load(p + 1, fg1) : make_float4(0.f, 0.f, 0.f, 0.f);
        // issue the pulls of plane p+2 first; they complete while plane p is collided
        const bool more = p + 2 <= z1;
        float fl[2][Q], hf[2][Q];
        uint8_t g_me = 0, g_h = 0;
        const int rn = fwd(rz, 2);
        const bool nsolid = a.wall && rn == 0;
        if (more) issue(p + 2, rn, fl, hf, g_me, g_h);
        // storage 3: the densities of plane p + 4 (sources of plane p + 3), stored after the
        // publication of plane p + 2 into the slot of plane p, which nothing reads any more
        if (LOC && more) rho_issue(p + 4);
        // ---- collide plane p ----
        const int cz = wrapn(p, nz);
        if (valid && !(a.wall && rz == 0)) {
            const int sc = (p - z0 + 4) & 3, su = (p - z0 + 5) & 3, sd = (p - z0 + 3) & 3;
            // the tile-plane takes the general path if any label, window or wall flag lies
            // in its ring planes p - 1 .. p + 1 (all waves meet at the same barrier anyway)
            int busy = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) busy |= s_busy[sc][w] | s_busy[su][w] | s_busy[sd][w];
            const uint32_t s = (uint32_t)((cz * ny + iy) * nx + ix);
            const float psi0 = s_psi[sc][0][li], psi1 = s_psi[sc][1][li];
            float p0n[Q - 1], p1n[Q - 1];
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                const int ns = CZ[q] == 0 ? sc : (CZ[q] > 0 ? su : sd);
                const int nl = li + CX[q] + CY[q] * LX;
                p0n[q - 1] = s_psi[ns][0][nl];
                p1n[q - 1] = s_psi[ns][1][nl];
            }
            float S0[3], S1[3], rx[3] = {0.f, 0.f, 0.f};
            uint8_t fg = 0;
            if (!busy) {
                stencil(p1n, a.ws_axis, a.ws_diag, S0[0], S0[1], S0[2]);
                stencil(p0n, a.ws_axis, a.ws_diag, S1[0], S1[1], S1[2]);
            } else {
                fg = s_flag[sc][li];
                int nlab[Q - 1];
#pragma unroll
                for (int q = 1; q < Q; ++q) {
                    const int ns = CZ[q] == 0 ? sc : (CZ[q] > 0 ? su : sd);
                    nlab[q - 1] = s_flag[ns][li + CX[q] + CY[q] * LX] & LABEL_MASK;
                }
                sc_general(a, s_drho, p0n, p1n, nlab, fg & LABEL_MASK, m0[0], m0[4], psi0, psi1, S0,
                           S1, rx);
            }
            collide_store_eq<S>(a, m0, s, fg, ib0, psi0, psi1, S0, S1, rx);
        }
        // ---- fold plane p+2 into the ring ----
        if (more) {
            float mn[8];
            uint8_t fgn;
            publish(p + 2, rn, nsolid, fl, hf, g_me, g_h, mn, fgn);
            if (LOC) rho_store(p + 4);
#pragma unroll
            for (int i = 0; i < 8; ++i) { m0[i] = m1[i]; m1[i] = mn[i]; }
            fg1 = fgn;
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) m0[i] = m1[i];
        }
        ib0 = ibn;
        __syncthreads();
    }
    (void)m2;
    (void)fgx;
}

// XCD-aware renumbering: hardware block b runs on XCD b % 8; each XCD gets a contiguous
// run of logical tiles, which share its L2 for the halo re-reads
__device__ __forceinline__ int logical_block() {
    const int per = (int)gridDim.x / 8;
    return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}

template <int S, int TX, int TY, bool WX, bool RT = false>
__global__ void __launch_bounds__(TX * TY) k_fused_pipe(FluidArgs a, int zc, int tiles_x,
                                                        int tiles_y, int nblocks) {
    const int L = logical_block();
    if (L >= nblocks) return;
    pipe_tile<S, TX, TY, WX, RT>(a, L, zc, tiles_x, tiles_y);
}

// Several lattices in one launch: group g owns the logical blocks desc[g].x ..
// desc[g + 1].x - 1, tiled desc[g].y x desc[g].z columns with z chunks of desc[g].w planes.
// The tables are read-only for the kernel's lifetime, so they are read through the
// constant address space (scalar loads).
typedef __attribute__((address_space(4))) const int ConstInt;

// logical block L of a multi-lattice launch: find its lattice, run its tile
template <int S, int TX, int TY, bool RT>
__device__ __forceinline__ void pipe_multi_tile(const FluidArgs *tab, const int4 *desc,
                                                int ngroups, int L) {
    static_assert(sizeof(FluidArgs) % 4 == 0, "word copy");
    ConstInt *cd = (ConstInt *)desc;   // int4 rows
    int g = 0;
    while (g + 1 < ngroups && L >= cd[4 * (g + 1)]) ++g;
    FluidArgs a;
    ConstInt *src = (ConstInt *)(tab + g);
    int *dst = reinterpret_cast<int *>(&a);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(FluidArgs) / 4); ++i) dst[i] = src[i];
    pipe_tile<S, TX, TY, RT, RT>(a, L - cd[4 * g], cd[4 * g + 3], cd[4 * g + 1], cd[4 * g + 2]);
}

template <int S, int TX, int TY, bool RT = false>
__global__ void __launch_bounds__(TX * TY) k_fused_pipe_multi(const FluidArgs *tab,
                                                              const int4 *desc, int ngroups,
                                                              int nblocks) {
    const int L = logical_block();
    if (L >= nblocks) return;
    pipe_multi_tile<S, TX, TY, RT>(tab, desc, ngroups, L);
}

// Work-queue form: a resident grid whose blocks take logical tiles from a queue until none
// is left.  queue[x] counts the tickets of XCD x (hardware block b runs on XCD b % 8), which
// owns the run of tiles [x * per, (x + 1) * per) as in the static order; a block whose XCD's
// run is used up takes tickets of the next XCDs.  queue[8] counts the blocks that are done;
// the last one clears the queue, which must be zero when the kernel starts.
template <int S, int TX, int TY, bool RT = false>
__global__ void __launch_bounds__(TX * TY) k_fused_pipe_multi_q(const FluidArgs *tab,
                                                                const int4 *desc, int ngroups,
                                                                int nblocks, int *queue) {
    __shared__ int s_L;
    const int per = (nblocks + 7) / 8;
    int x = (int)(blockIdx.x % 8), tried = 0;   // used by thread 0 only
    for (;;) {
        if (threadIdx.x == 0) {
            int L = -1;
            while (tried < 8) {
                const int t = atomicAdd(&queue[x], 1);
                if (t < per && x * per + t < nblocks) {
                    L = x * per + t;
                    break;
                }
                x = (x + 1) % 8;
                ++tried;
            }
            s_L = L;
        }
        __syncthreads();
        const int L = s_L;
        __syncthreads();   // s_L is written again only after every thread has read it
        if (L < 0) break;
        pipe_multi_tile<S, TX, TY, RT>(tab, desc, ngroups, L);
    }
    if (threadIdx.x == 0 && atomicAdd(&queue[8], 1) == (int)gridDim.x - 1)
        for (int i = 0; i <= 8; ++i) atomicExch(&queue[i], 0);
}

template <int S>
void launch_fluid_multi(const FluidArgs *tab, const int4 *desc, int ngroups, int nblocks,
                        int tile, int *queue, int ncu, hipStream_t st) {
    if (queue) {   // one resident block of 512 threads (two of 256) per compute unit
        const int nt = (tile >= 6 && tile <= 8) ? 256 : 512;
        const dim3 grid(std::max(8, std::min(ncu * (512 / nt), nblocks)));
        switch (tile) {
            case 6: hipLaunchKernelGGL((k_fused_pipe_multi_q<S, 32, 8>), grid, dim3(256), 0, st, tab, desc, ngroups, nblocks, queue); break;
            case 7: hipLaunchKernelGGL((k_fused_pipe_multi_q<S, 64, 4>), grid, dim3(256), 0, st, tab, desc, ngroups, nblocks, queue); break;
            case 8: hipLaunchKernelGGL((k_fused_pipe_multi_q<S, 16, 16>), grid, dim3(256), 0, st, tab, desc, ngroups, nblocks, queue); break;
            case 9: hipLaunchKernelGGL((k_fused_pipe_multi_q<S, 32, 16>), grid, dim3(512), 0, st, tab, desc, ngroups, nblocks, queue); break;
            case 13: hipLaunchKernelGGL((k_fused_pipe_multi_q<S, 128, 4, true>), grid, dim3(512), 0, st, tab, desc, ngroups, nblocks, queue); break;
            default: hipLaunchKernelGGL((k_fused_pipe_multi_q<S, 64, 8>), grid, dim3(512), 0, st, tab, desc, ngroups, nblocks, queue); break;
        }
        return;
    }
    const dim3 grid((nblocks + 7) / 8 * 8);
    switch (tile) {
        case 6: hipLaunchKernelGGL((k_fused_pipe_multi<S, 32, 8>), grid, dim3(256), 0, st, tab, desc, ngroups, nblocks); break;
        case 7: hipLaunchKernelGGL((k_fused_pipe_multi<S, 64, 4>), grid, dim3(256), 0, st, tab, desc, ngroups, nblocks); break;
        case 8: hipLaunchKernelGGL((k_fused_pipe_multi<S, 16, 16>), grid, dim3(256), 0, st, tab, desc, ngroups, nblocks); break;
        case 9: hipLaunchKernelGGL((k_fused_pipe_multi<S, 32, 16>), grid, dim3(512), 0, st, tab, desc, ngroups, nblocks); break;
        case 13: hipLaunchKernelGGL((k_fused_pipe_multi<S, 128, 4, true>), grid, dim3(512), 0, st, tab, desc, ngroups, nblocks); break;
        default: hipLaunchKernelGGL((k_fused_pipe_multi<S, 64, 8>), grid, dim3(512), 0, st, tab, desc, ngroups, nblocks); break;
    }
}

// whole rows of run-time width nx (16 .. 128), 512 / nx rows per tile
int rows_tile_height(int nx) { return 512 / nx; }

template <int S>
static void launch_pipe_rows(const FluidArgs &a, int zc, hipStream_t st) {
    const int ty = rows_tile_height(a.nx);
    const int tyn = (a.ny + ty - 1) / ty, tz = (a.nz + zc - 1) / zc;
    const int nb = tyn * tz;
    const int grid = (nb + 7) / 8 * 8;
    hipLaunchKernelGGL((k_fused_pipe<S, 128, 4, true, true>), dim3(grid), dim3(512), 0, st, a, zc,
                       1, tyn, nb);
}

template <int S, int TX, int TY, bool WX = false>
static void launch_pipe_t(const FluidArgs &a, int zc, hipStream_t st) {
    const int tx = (a.nx + TX - 1) / TX, ty = (a.ny + TY - 1) / TY, tz = (a.nz + zc - 1) / zc;
    const int nb = tx * ty * tz;
    const int grid = (nb + 7) / 8 * 8;
    hipLaunchKernelGGL((k_fused_pipe<S, TX, TY, WX>), dim3(grid), dim3(TX * TY), 0, st, a, zc, tx,
                       ty, nb);
}

template <int S, int TX, int TY>
static void launch_fused_t(const FluidArgs &a, int zc, hipStream_t st) {
    const int tx = (a.nx + TX - 1) / TX, ty = (a.ny + TY - 1) / TY, tz = (a.nz + zc - 1) / zc;
    const int nb = tx * ty * tz;
    const int grid = (nb + 7) / 8 * 8;
    if (a.keepf)
        hipLaunchKernelGGL((k_fused<S, TX, TY, true>), dim3(grid), dim3(TX * TY), 0, st, a, zc, tx,
                           ty, nb);
    else
        hipLaunchKernelGGL((k_fused<S, TX, TY, false>), dim3(grid), dim3(TX * TY), 0, st, a, zc,
                           tx, ty, nb);
}

// tile: 0 two-kernel variant; 1: 32x8; 2: 64x4; 3: 32x16; 4: 64x8; 5: 16x16; 6-10: the
// pipelined kernel with 32x8, 64x4, 16x16, 32x16, 64x8; 11: whole rows 256x2; 12: whole
// rows 128x4; 13: whole rows of width nx (16 .. 128) by 512 / nx
template <int S>
void launch_fluid_tiled(const FluidArgs &a, int tile, int zc, hipStream_t st) {
    if constexpr (S == 3) {
        // storage 3 runs the pipelined kernels only (tau = 1): tiles 1..5 and the two-kernel
        // variant take the pipelined 64 x 8 tile
        switch (tile) {
            case 6: launch_pipe_t<S, 32, 8>(a, zc, st); break;
            case 7: launch_pipe_t<S, 64, 4>(a, zc, st); break;
            case 8: launch_pipe_t<S, 16, 16>(a, zc, st); break;
            case 9: launch_pipe_t<S, 32, 16>(a, zc, st); break;
            case 11:
                if (a.nx == 256) launch_pipe_t<S, 256, 2, true>(a, zc, st);
                else launch_pipe_t<S, 64, 8>(a, zc, st);
                break;
            case 12:
                if (a.nx == 128) launch_pipe_t<S, 128, 4, true>(a, zc, st);
                else launch_pipe_t<S, 64, 8>(a, zc, st);
                break;
            case 13:
                if (a.nx >= 16 && a.nx <= 128) launch_pipe_rows<S>(a, zc, st);
                else launch_pipe_t<S, 64, 8>(a, zc, st);
                break;
            default: launch_pipe_t<S, 64, 8>(a, zc, st); break;
        }
        return;
    } else {
    switch (tile) {
        case 1: launch_fused_t<S, 32, 8>(a, zc, st); break;
        case 2: launch_fused_t<S, 64, 4>(a, zc, st); break;
        case 3: launch_fused_t<S, 32, 16>(a, zc, st); break;
        case 4: launch_fused_t<S, 64, 8>(a, zc, st); break;
        case 5: launch_fused_t<S, 16, 16>(a, zc, st); break;
        case 6: if (a.keepf) launch_fused_t<S, 32, 8>(a, zc, st); else launch_pipe_t<S, 32, 8>(a, zc, st); break;
        case 7: if (a.keepf) launch_fused_t<S, 64, 4>(a, zc, st); else launch_pipe_t<S, 64, 4>(a, zc, st); break;
        case 8: if (a.keepf) launch_fused_t<S, 16, 16>(a, zc, st); else launch_pipe_t<S, 16, 16>(a, zc, st); break;
        case 9: if (a.keepf) launch_fused_t<S, 32, 16>(a, zc, st); else launch_pipe_t<S, 32, 16>(a, zc, st); break;
        case 10: if (a.keepf) launch_fused_t<S, 64, 8>(a, zc, st); else launch_pipe_t<S, 64, 8>(a, zc, st); break;
        // whole-row tiles: need nx equal to the tile width, else the 64 x 8 tile is used
        case 11:
            if (a.keepf) launch_fused_t<S, 64, 8>(a, zc, st);
            else if (a.nx == 256) launch_pipe_t<S, 256, 2, true>(a, zc, st);
            else launch_pipe_t<S, 64, 8>(a, zc, st);
            break;
        case 12:
            if (a.keepf) launch_fused_t<S, 64, 8>(a, zc, st);
            else if (a.nx == 128) launch_pipe_t<S, 128, 4, true>(a, zc, st);
            else launch_pipe_t<S, 64, 8>(a, zc, st);
            break;
        // whole rows of any width 16 .. 128 (512 / nx rows per tile), else 64 x 8
        case 13:
            if (a.keepf) launch_fused_t<S, 64, 8>(a, zc, st);
            else if (a.nx >= 16 && a.nx <= 128) launch_pipe_rows<S>(a, zc, st);
            else launch_pipe_t<S, 64, 8>(a, zc, st);
            break;
        default: launch_fluid<S>(a, st); break;
    }
    }
}

// ------------------------------------------------------------------------------------
// Observables
// ------------------------------------------------------------------------------------
template <int S>
__global__ void k_rho(const void *f, float *__restrict__ rho, int nx, int ny, int nz, int wall,
                      int lz, float sh0, float sh1, const float *__restrict__ rsite) {
    const int N = nx * ny * nz;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const int z = s / (nx * ny);
    float r0 = 0.f, r1 = 0.f;
    if (!(wall && slab_pos(z, lz) == 0)) {
        if constexpr (S == 3) {
            sh0 = rsite[s];
            sh1 = rsite[N + s];
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            r0 += Pop<S>::load(f, q, N, s, wsh<S>(q) * sh0);
            r1 += Pop<S>::load(f, Q + q, N, s, wsh<S>(q) * sh1);
        }
    }
    rho[s] = r0;
    rho[N + s] = r1;
}

template <int S>
void launch_rho(const void *f, float *rho, int nx, int ny, int nz, int wall, int lz, float s0,
                float s1, const float *rsite, hipStream_t st) {
    const int N = nx * ny * nz;
    hipLaunchKernelGGL(k_rho<S>, dim3((N + 255) / 256), dim3(256), 0, st, f, rho, nx, ny, nz, wall,
                       lz, s0, s1, rsite);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// mass^c and fluid momentum, double accumulation; one partial row of 5 per block.
// Block (b, sl) sums sites of slab sl only.
template <int S>
__global__ void __launch_bounds__(256) k_moments(const void *f, double *__restrict__ partial,
                                                 int nx, int ny, int nz, int wall, int lz,
                                                 float sh0, float sh1,
                                                 const float *__restrict__ rsite) {
    const int N = nx * ny * nz, plane = nx * ny;
    const int s_end = (blockIdx.y + 1) * lz * plane;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int s = blockIdx.y * lz * plane + blockIdx.x * blockDim.x + threadIdx.x; s < s_end;
         s += gridDim.x * blockDim.x) {
        const int z = s / plane;
        if (wall && slab_pos(z, lz) == 0) continue;
        if constexpr (S == 3) {
            sh0 = rsite[s];
            sh1 = rsite[N + s];
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double v0 = Pop<S>::load(f, q, N, s, wsh<S>(q) * sh0);
            const double v1 = Pop<S>::load(f, Q + q, N, s, wsh<S>(q) * sh1);
            acc[0] += v0;
            acc[1] += v1;
            if (CX[q]) acc[2] += CX[q] * (v0 + v1);
            if (CY[q]) acc[3] += CY[q] * (v0 + v1);
            if (CZ[q]) acc[4] += CZ[q] * (v0 + v1);
        }
    }
    __shared__ double red[4][5];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const double v = wave_sum(acc[i]);
        if (lane == 0) red[wid][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double v = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w][threadIdx.x];
        partial[(blockIdx.y * gridDim.x + blockIdx.x) * 5 + threadIdx.x] = v;
    }
}

template <int S>
void launch_moments(const void *f, double *partial, int nblocks, int nx, int ny, int nz, int wall,
                    int lz, float s0, float s1, const float *rsite, hipStream_t st) {
    hipLaunchKernelGGL(k_moments<S>, dim3(nblocks, nz / lz), dim3(256), 0, st, f, partial, nx, ny,
                       nz, wall, lz, s0, s1, rsite);
}

// Meniscus height per column of each slab: the first upward crossing of
// phi = (rho0 - rho1) / (rho0 + rho1) from >= 0 to < 0 above the slab's wall layer,
// linearly interpolated; NaN if none or if either site of the crossing lies inside a
// capsule.
__global__ void k_meniscus(const float *__restrict__ rho, const uint8_t *__restrict__ flag,
                           float *__restrict__ out, int nx, int ny, int nz, int wall, int lz) {
    const int plane = nx * ny, N = plane * nz;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= plane * (nz / lz)) return;
    const int col = idx % plane, base = (idx / plane) * lz * plane;
    float res = __builtin_nanf("");
    for (int k = wall ? 1 : 0; k + 1 < lz; ++k) {
        const int s0 = base + k * plane + col, s1 = s0 + plane;
        const double a0 = rho[s0], b0 = rho[N + s0], a1 = rho[s1], b1 = rho[N + s1];
        const double p0 = (a0 - b0) / (a0 + b0), p1 = (a1 - b1) / (a1 + b1);
        if (p0 >= 0.0 && p1 < 0.0) {
            if ((flag[s0] & LABEL_MASK) == 0 && (flag[s1] & LABEL_MASK) == 0)
                res = (float)(k + p0 / (p0 - p1));
            break;
        }
    }
    out[idx] = res;
}

void launch_meniscus(const float *rho, const uint8_t *flag, float *out, int nx, int ny, int nz,
                     int wall, int lz, hipStream_t st) {
    const int cols = nx * ny * (nz / lz);
    hipLaunchKernelGGL(k_meniscus, dim3((cols + 255) / 256), dim3(256), 0, st, rho, flag, out,
                       nx, ny, nz, wall, lz);
}

#define LBMX_INST(S)                                                                        \
    template void launch_init_eq<S>(const double *, void *, int, int, int, int, int, float,  \
                                    float, float *, hipStream_t);                           \
    template void launch_fluid_tiled<S>(const FluidArgs &, int, int, hipStream_t);          \
    template void launch_fluid_multi<S>(const FluidArgs *, const int4 *, int, int, int, int *, \
                                        int, hipStream_t);                                    \
    template void launch_rho<S>(const void *, float *, int, int, int, int, int, float, float, \
                                const float *, hipStream_t);                                \
    template void launch_moments<S>(const void *, double *, int, int, int, int, int, int,    \
                                    float, float, const float *, hipStream_t);
LBMX_INST(0)
LBMX_INST(1)
LBMX_INST(2)
LBMX_INST(3)
template void launch_fluid<0>(const FluidArgs &, hipStream_t);
template void launch_fluid<1>(const FluidArgs &, hipStream_t);
template void launch_fluid<2>(const FluidArgs &, hipStream_t);

}  // namespace lbmx
