// surrogate.hip -- the learned form: a multilayer perceptron 4 -> 64 -> 64 -> 64 -> 2
// (tanh hidden layers, 8770 parameters) that maps a capsule pair's separation,
// softness, film height and contact angle to its lateral capillary force and meniscus
// deformation, trained by Adam on data of the batched solver.
//
// Every matrix product runs on the matrix cores: v_mfma_f32_16x16x16_bf16, operands
// rounded to bfloat16 (nearest, ties to even) when loaded, sums in float32.  One
// wavefront computes one 16 x 16 tile of the product; operand and result layouts are
// given by strides, so the same kernel serves x W, d W^T and a^T d.  Parameters, Adam
// moments, activations and gradients are float32 in HBM (the whole state is ~0.2 MB plus
// 1 kB per sample).
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

namespace {

constexpr int NIN = 4, NH = 64, NOUT = 2, NLAYER = 4;
constexpr int LIN[NLAYER] = {NIN, NH, NH, NH}, LOUT[NLAYER] = {NH, NH, NH, NOUT};
// offsets of W_l ([in][out], row-major) and b_l in the parameter vector
constexpr int woff(int l) { return l == 0 ? 0 : woff(l - 1) + LIN[l - 1] * LOUT[l - 1] + LOUT[l - 1]; }
constexpr int boff(int l) { return woff(l) + LIN[l] * LOUT[l]; }
constexpr int NPAR = boff(NLAYER - 1) + NOUT;
static_assert(NPAR == LBM_SURROGATE_PARAMS, "parameter count");

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest, ties to even (finite values)
    return (short)(u >> 16);
}

enum Epi { EPI_STORE = 0, EPI_BIAS_TANH = 1, EPI_BIAS = 2, EPI_TANH_GRAD = 3 };

// C[M][N] (row stride ldc) = A (M x K, element (i, k) at A[i * sar + k * sac]) times
// B (K x N, element (k, j) at B[k * sbr + j * sbc]), then the epilogue:
//   EPI_STORE      C = AB
//   EPI_BIAS_TANH  C = tanh(AB + bias[j])
//   EPI_BIAS       C = AB + bias[j]
//   EPI_TANH_GRAD  C = AB * (1 - P[i][j]^2), P the layer's tanh output (row stride ldc)
// One wave per 16 x 16 tile of C, four waves per block; elements outside M, N, K are 0.
// Split K (kz > 0, EPI_STORE only): block row y sums k in [y kz, (y + 1) kz) and writes
// its partial product to C + y M ldc; k_sum_slices adds the slices in order.
// MFMA 16x16x16 lane layout: A row = lane % 16, B column = lane % 16, both with k =
// 4 (lane / 16) .. +3; result row = 4 (lane / 16) + i, column = lane % 16.
__global__ void __launch_bounds__(256) k_gemm_bf16(const float *__restrict__ A, int sar, int sac,
                                                   const float *__restrict__ B, int sbr, int sbc,
                                                   float *__restrict__ C, int ldc, int M, int N,
                                                   int K, int epi, const float *__restrict__ bias,
                                                   const float *__restrict__ P, int kz) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tiles_n = (N + 15) / 16;
    const int tile = blockIdx.x * 4 + wave;
    if (tile >= ((M + 15) / 16) * tiles_n) return;   // whole waves
    const int i0 = (tile / tiles_n) * 16, j0 = (tile % tiles_n) * 16;
    const int r = i0 + (lane & 15), c = j0 + (lane & 15), kq = 4 * (lane >> 4);
    const int kb = kz ? (int)blockIdx.y * kz : 0, ke = kz ? min(K, kb + kz) : K;
    if (kz) C += (size_t)blockIdx.y * M * ldc;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += 16) {
        v4s a, b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + kq + j;
            const float av = (r < M && k < ke) ? A[(size_t)r * sar + (size_t)k * sac] : 0.f;
            const float bv = (c < N && k < ke) ? B[(size_t)k * sbr + (size_t)c * sbc] : 0.f;
            a[j] = to_bf16(av);
            b[j] = to_bf16(bv);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    const int col = j0 + (lane & 15);
    if (col >= N) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = i0 + kq + i;
        if (row >= M) continue;
        float v = acc[i];
        if (epi == EPI_BIAS_TANH) v = tanhf(v + bias[col]);
        else if (epi == EPI_BIAS) v += bias[col];
        else if (epi == EPI_TANH_GRAD) {
            const float p = P[(size_t)row * ldc + col];
            v *= 1.0f - p * p;
        }
        C[(size_t)row * ldc + col] = v;
    }
}

// C[i][j] = sum over the slices y = 0 .. ns - 1, in order, of S[y][i][j] (split-K sums)
__global__ void k_sum_slices(const float *__restrict__ S, int ns, int M, int N,
                             float *__restrict__ C, int ldc) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M * N) return;
    const int i = e / N, j = e - i * N;
    float a = 0.f;
    for (int y = 0; y < ns; ++y) a += S[(size_t)y * M * N + e];
    C[(size_t)i * ldc + j] = a;
}

// dY = w (Y - T) / sum(w); per-block partial sums of w (Y - T)^2 for the loss
__global__ void k_loss_grad(const float *__restrict__ Y, const float *__restrict__ T,
                            const float *__restrict__ W, float inv_n, int n,
                            float *__restrict__ dY, float *__restrict__ part) {
    __shared__ float s[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.f;
    if (i < n) {
        for (int o = 0; o < NOUT; ++o) {
            const float r = Y[i * NOUT + o] - T[i * NOUT + o];
            dY[i * NOUT + o] = W[i] * r * inv_n;
            acc += W[i] * r * r;
        }
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// db[j] = sum over the n rows of D[i][j]: one block per column, each thread a strided
// share of the rows, then a fixed tree (the order does not depend on scheduling)
__global__ void __launch_bounds__(256) k_colsum(const float *__restrict__ D, int n, int m,
                                                float *__restrict__ db) {
    __shared__ float s[256];
    const int j = blockIdx.x;
    float a = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) a += D[(size_t)i * m + j];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[j] = s[0];
}

// ------------------------------------------------------------------------------------
// Training in two launches per Adam step.
//
// k_train_chunk: the samples are taken in chunks of TC_ROWS = 32 rows, chunk c by
// workgroup c mod TC_BLOCKS (8 waves).  Per chunk: forward through the four layers, the
// loss gradient and back-propagation, each product on the matrix cores with the operands
// rounded to bfloat16 as they are read (as k_gemm_bf16 does).  A chunk's 32 x 64 product
// is 8 tiles, one per wave (row tile tr); a 64 x 64 weight gradient is 16 tiles, two per
// wave (ti, tj).  The weight gradients stay in accumulator registers across a
// workgroup's chunks: each of their 40 tiles (dW3 16, dW2 16, dW4 4, dW1 4) has one owning
// wave; the bias gradients are float32 column sums of dL/dz (not rounded, as k_colsum),
// one column per lane of an owning wave.  The weights (row stride 65 for the 64-wide
// layers, so that reading W^T does not hit one LDS bank 16 times), the chunk's inputs,
// targets, weights, activations and dL/dz are in LDS.  Rows of a chunk past the last
// sample carry zero inputs and zero loss gradient.  Each workgroup writes its gradient,
// in the parameter layout, to row blockIdx.x of G.
//
// k_train_update: per parameter, the rows of G summed in workgroup order, then Adam
// (Kingma & Ba: bias-corrected moments, step counted from 1).
// Every sum runs in a fixed order, so the result does not depend on scheduling.
// ------------------------------------------------------------------------------------
constexpr int TC_THREADS = 512, TC_ROWS = 32, TC_LD = NH + 1, TC_BLOCKS = 128;
static_assert(TC_ROWS == 32, "one 16 x 16 tile of a chunk product per wave");
constexpr int TW1 = woff(0), TW2 = woff(1), TW3 = woff(2), TW4 = woff(3);
constexpr int TB1 = boff(0), TB2 = boff(1), TB3 = boff(2), TB4 = boff(3);

struct TrainArgs {
    const float *th, *x, *t, *w;
    float *G;                          // [gridDim.x][NPAR] gradients of the workgroups
    int n;
    float inv_wsum;
};

__global__ void __launch_bounds__(TC_THREADS) k_train_chunk(TrainArgs a) {
    // parameters: W1 [4][64], W2, W3 [64][65], W4 [64][2], biases
    __shared__ float sW1[NIN * NH], sW2[NH * TC_LD], sW3[NH * TC_LD], sW4[NH * NOUT];
    __shared__ float sb1[NH], sb2[NH], sb3[NH], sb4[NOUT];
    // the chunk's activations (the three tanh layers), dL/dz of two layers, its data
    __shared__ float sA[3][TC_ROWS * TC_LD], sD[2][TC_ROWS * TC_LD];
    __shared__ float sDy[TC_ROWS * NOUT], sX[TC_ROWS * NIN], sT[TC_ROWS * NOUT], sWt[TC_ROWS];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lc = lane & 15, kq = 4 * (lane >> 4);
    for (int p = tid; p < NPAR; p += TC_THREADS) {
        const float v = a.th[p];
        if (p < TB1) sW1[p] = v;
        else if (p < TW2) sb1[p - TB1] = v;
        else if (p < TB2) { const int q = p - TW2; sW2[(q / NH) * TC_LD + q % NH] = v; }
        else if (p < TW3) sb2[p - TB2] = v;
        else if (p < TB3) { const int q = p - TW3; sW3[(q / NH) * TC_LD + q % NH] = v; }
        else if (p < TW4) sb3[p - TB3] = v;
        else if (p < TB4) sW4[p - TW4] = v;
        else sb4[p - TB4] = v;
    }

    // one 16 x 16 tile of a product: acc += A B over k < KN (A(i, k), B(k, j) given as
    // functions returning 0 outside the operands); row i0 + lc of A and column j0 + lc of
    // B per lane, k = k0 + kq + 0..3
    auto tile = [&](v4f acc, int i0, int j0, auto kn, auto fa, auto fb) {
        constexpr int KN = decltype(kn)::value;
#pragma unroll
        for (int k0 = 0; k0 < KN; k0 += 16) {
            v4s av, bv;
#pragma unroll
            for (int j = 0; j < 4; ++j) {   // hardware conversion, nearest even
                const int k = k0 + kq + j;
                av[j] = __builtin_bit_cast(short, (__bf16)fa(i0 + lc, k));
                bv[j] = __builtin_bit_cast(short, (__bf16)fb(k, j0 + lc));
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
        }
        return acc;
    };
    using K16 = std::integral_constant<int, 16>;
    using KR = std::integral_constant<int, TC_ROWS>;
    using K64 = std::integral_constant<int, 64>;
    const v4f zero = {0.f, 0.f, 0.f, 0.f};
    // this wave's tile of a chunk product (rows tr, columns tj) and its two tiles of a
    // 64 x 64 weight gradient: tiles wave and wave + 8
    const int tr = 16 * (wave >> 2), tj = 16 * (wave & 3);
    const int ti[2] = {16 * (wave >> 2), 16 * ((wave + 8) >> 2)};

    v4f gW3[2] = {zero, zero}, gW2[2] = {zero, zero};   // owned weight-gradient tiles
    v4f gW4 = zero, gW1 = zero;   // waves 0..3: dW4 row tile; waves 4..7: dW1 column tile
    float gB = 0.f;               // waves 4..7: a column of db4, db3, db2, db1
    // column `lane` of the chunk's rows of D (row stride ld), summed in row order
    auto colsum = [&](const float *D, int ld) {
        float acc = 0.f;
#pragma unroll 8
        for (int r = 0; r < TC_ROWS; ++r) acc += D[r * ld + lane];
        gB += acc;
    };
    for (int r0 = blockIdx.x * TC_ROWS; r0 < a.n; r0 += gridDim.x * TC_ROWS) {   // uniform
        const int nr = min(TC_ROWS, a.n - r0);
        __syncthreads();   // the previous chunk is done with the data and activations
        for (int e = tid; e < TC_ROWS * NIN; e += TC_THREADS)
            sX[e] = e < nr * NIN ? a.x[r0 * NIN + e] : 0.f;
        for (int e = tid; e < TC_ROWS * NOUT; e += TC_THREADS)
            sT[e] = e < nr * NOUT ? a.t[r0 * NOUT + e] : 0.f;
        for (int e = tid; e < TC_ROWS; e += TC_THREADS) sWt[e] = e < nr ? a.w[r0 + e] : 0.f;
        __syncthreads();
        // ---- forward: a1 = tanh(x W1 + b1), a2, a3, then the output layer ----
        {
            const v4f c = tile(zero, tr, tj, K16{}, [&](int i, int k) { return k < NIN ? sX[i * NIN + k] : 0.f; },
                               [&](int k, int j) { return k < NIN ? sW1[k * NH + j] : 0.f; });
#pragma unroll
            for (int e = 0; e < 4; ++e)
                sA[0][(tr + kq + e) * TC_LD + tj + lc] = tanhf(c[e] + sb1[tj + lc]);
        }
        __syncthreads();
#pragma unroll
        for (int l = 1; l < 3; ++l) {
            const float *Ap = sA[l - 1], *W = l == 1 ? sW2 : sW3, *b = l == 1 ? sb2 : sb3;
            const v4f c = tile(zero, tr, tj, K64{}, [&](int i, int k) { return Ap[i * TC_LD + k]; },
                               [&](int k, int j) { return W[k * TC_LD + j]; });
#pragma unroll
            for (int e = 0; e < 4; ++e)
                sA[l][(tr + kq + e) * TC_LD + tj + lc] = tanhf(c[e] + b[tj + lc]);
            __syncthreads();
        }
        if (wave < TC_ROWS / 16) {   // y = a3 W4 + b4, then dL/dy = w (y - t) / sum w (0 past n)
            v4f c = tile(zero, 16 * wave, 0, K64{}, [&](int i, int k) { return sA[2][i * TC_LD + k]; },
                         [&](int k, int j) { return j < NOUT ? sW4[k * NOUT + j] : 0.f; });
            if (lc < NOUT) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int i = 16 * wave + kq + e;
                    const float y = c[e] + sb4[lc];
                    sDy[i * NOUT + lc] = i < nr ? sWt[i] * (y - sT[i * NOUT + lc]) * a.inv_wsum : 0.f;
                }
            }
        }
        __syncthreads();
        // ---- back-propagation ----
        // d3 = (dy W4^T) (1 - a3^2); dW4 += a3^T dy (waves 0..3); db4 (wave 4)
        {
            const v4f c = tile(zero, tr, tj, K16{}, [&](int i, int k) { return k < NOUT ? sDy[i * NOUT + k] : 0.f; },
                               [&](int k, int j) { return k < NOUT ? sW4[j * NOUT + k] : 0.f; });
            if (wave < 4)
                gW4 = tile(gW4, 16 * wave, 0, KR{}, [&](int i, int k) { return sA[2][k * TC_LD + i]; },
                           [&](int k, int j) { return j < NOUT ? sDy[k * NOUT + j] : 0.f; });
            else if (wave == 4 && lane < NOUT)
                colsum(sDy, NOUT);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = (tr + kq + e) * TC_LD + tj + lc;
                const float p = sA[2][o];
                sD[0][o] = c[e] * (1.0f - p * p);
            }
        }
        __syncthreads();
        // d2 = (d3 W3^T) (1 - a2^2); dW3 += a2^T d3; db3 (wave 5)
        // d1 = (d2 W2^T) (1 - a1^2); dW2 += a1^T d2; db2 (wave 6)
#pragma unroll
        for (int l = 2; l >= 1; --l) {
            const float *Dn = sD[(2 - l) & 1], *Ap = sA[l - 1], *W = l == 2 ? sW3 : sW2;
            float *Dp = sD[(3 - l) & 1];
            v4f (&gW)[2] = l == 2 ? gW3 : gW2;
            const v4f c = tile(zero, tr, tj, K64{}, [&](int i, int k) { return Dn[i * TC_LD + k]; },
                               [&](int k, int j) { return W[j * TC_LD + k]; });
#pragma unroll
            for (int u = 0; u < 2; ++u)
                gW[u] = tile(gW[u], ti[u], tj, KR{}, [&](int i, int k) { return Ap[k * TC_LD + i]; },
                             [&](int k, int j) { return Dn[k * TC_LD + j]; });
            if (wave == (l == 2 ? 5 : 6)) colsum(Dn, TC_LD);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = (tr + kq + e) * TC_LD + tj + lc;
                const float p = Ap[o];
                Dp[o] = c[e] * (1.0f - p * p);
            }
            __syncthreads();
        }
        // dW1 += x^T d1 (waves 4..7); db1 (wave 7)
        if (wave >= 4) {
            const float *D1 = sD[0];
            gW1 = tile(gW1, 0, 16 * (wave - 4), KR{}, [&](int i, int k) { return i < NIN ? sX[k * NIN + i] : 0.f; },
                       [&](int k, int j) { return D1[k * TC_LD + j]; });
            if (wave == 7) colsum(D1, TC_LD);
        }
    }
    // ---- the workgroup's gradient, in the parameter layout, into its row of G ----
    float *G = a.G + (size_t)blockIdx.x * NPAR;
    auto put = [&](const v4f &g, int base, int i0, int j0, int rows, int cols, int ld) {
        if (j0 + lc >= cols) return;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = i0 + kq + e;
            if (i < rows) G[base + i * ld + j0 + lc] = g[e];
        }
    };
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        put(gW3[u], TW3, ti[u], tj, NH, NH, NH);
        put(gW2[u], TW2, ti[u], tj, NH, NH, NH);
    }
    if (wave < 4) {
        put(gW4, TW4, 16 * wave, 0, NH, NOUT, NOUT);
    } else {
        put(gW1, TW1, 0, 16 * (wave - 4), NIN, NH, NH);
        const int bo[4] = {TB4, TB3, TB2, TB1};
        if (wave > 4 || lane < NOUT) G[bo[wave - 4] + lane] = gB;
    }
}

// per parameter: the workgroups' gradients summed in order, then Adam (bias-corrected
// moments, step counted from 1)
__global__ void k_train_update(float *__restrict__ th, float *__restrict__ m, float *__restrict__ v,
                               const float *__restrict__ G, int nb, float lr, float b1, float b2,
                               float c1, float c2, float eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAR) return;
    float gi = 0.f;
    // rows in groups of 16 with every load of a group in flight, summed in row order
    for (int b0 = 0; b0 < nb; b0 += 16) {
        float r[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) r[k] = b0 + k < nb ? G[(size_t)(b0 + k) * NPAR + i] : 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (b0 + k < nb) gi += r[k];
    }
    const float mi = b1 * m[i] + (1.f - b1) * gi, vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------------------------
// Cluster evolution driven by the network: overdamped capsules in a periodic square,
// p_i += mobility * sum_j f(r_ij) e_ij, f the network's lateral force for separations
// in [r_contact, r_cut] radii, a contact repulsion closer, 0 farther.
//
// One fused kernel per step, one block per capsule i, four waves.  Each wave takes 16
// partners j at a time through the whole network on the matrix cores in transposed
// form, Z^T = W^T H^T: the partners are the 16 columns, so a layer's result tile (16
// neurons as rows, four per lane) is already, lane for lane, the next layer's B operand
// for the same 16 neurons as k, and the activations never leave registers.  The weights
// are A operands held in registers for the whole block (80 VGPRs), loaded ready-made
// from a buffer that k_pack_cluster_net writes once per call; the biases, loaded the same
// way as accumulator tiles, initialise the accumulators.  tanh comes from the hardware exponential
// and reciprocal.  The separations (minimum image through the float32 reciprocal of the
// box) and the network's inputs (scaled by float32 reciprocals of the input scales) are
// computed without contraction into fused multiply-adds, so that each is the correctly
// rounded float32 result of the operations as written (the inputs are then rounded to
// bfloat16, a decision taken in float32).  The partner forces are summed per lane in
// partner order, then over the 16 lanes of each of the four waves in a fixed order: no
// atomics, the result does not depend on scheduling.
// ------------------------------------------------------------------------------------
struct ClusterArgs {
    float xm[4], inv_xs[4], ym, ys;     // normalisation of the inputs / the force output
    float feat[3];                      // log10 ks, film / 2R, contact angle (raw)
    float box, inv_box, inv_radius, r_contact, r_cut, k_contact, mobility;
    int n;
};

constexpr int CL_THREADS = 256, CL_WAVES = CL_THREADS / 64;
// parameter offsets as constants (the recursive woff / boff are not folded for device code)
constexpr int CW1 = woff(0), CW2 = woff(1), CW3 = woff(2), CW4 = woff(3);
constexpr int CB1 = boff(0), CB2 = boff(1), CB3 = boff(2), CB4 = boff(3);
static_assert(CB2 == CB1 + NH + NH * NH && CB3 == CB2 + NH + NH * NH && CB4 == CW4 + NH * NOUT,
              "parameter layout");

// four float32 values to bfloat16 with the hardware conversion (nearest, ties to even)
__device__ __forceinline__ v4s bf16x4(v4f v) {
    v4s o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = __builtin_bit_cast(short, (__bf16)v[k]);
    return o;
}

// tanh x = 1 - 2 / (exp(2x) + 1) with the hardware base-2 exponential and reciprocal:
// absolute error below 1e-6, and +-1 without overflow for large |x| (exp -> inf or 0)
__device__ __forceinline__ float tanh_hw(float x) {
    const float e = __builtin_amdgcn_exp2f(x * 2.88539008f);   // 2 / ln 2
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// The network in the lane layout of the matrix-core operands, written once per call so
// that each block of the step loads it with a few coalesced loads: 40 A-operand fragments
// (bfloat16 x 4 per lane: W1 by output tile, W2 and W3 by output tile and k block, W4 by
// k block) and 13 accumulator tiles of biases (float x 4 per lane: b1, b2, b3 by output
// tile, then b4), each stored as [fragment][lane].  A[row][k] = W[k][row], so lane
// (col = lane % 16, kq = 4 (lane / 16)) holds W[16 kb + kq + j][16 ot + col], j = 0..3,
// and bias rows 16 ot + kq + e, e = 0..3.
constexpr int CL_FRAGS = 40, CL_BTILES = 13;

__global__ void __launch_bounds__(64) k_pack_cluster_net(const float *__restrict__ th,
                                                         uint2 *__restrict__ frag,
                                                         float4 *__restrict__ btile) {
    const int lane = threadIdx.x, col = lane & 15, kq = 4 * (lane >> 4);
    auto put = [&](int f, v4s v) { frag[f * 64 + lane] = __builtin_bit_cast(uint2, v); };
    for (int ot = 0; ot < 4; ++ot) {
        v4s w;
        for (int j = 0; j < 4; ++j) w[j] = kq == 0 ? to_bf16(th[CW1 + j * NH + 16 * ot + col]) : (short)0;
        put(ot, w);
        for (int kb = 0; kb < 4; ++kb) {
            v4s a, b;
            for (int j = 0; j < 4; ++j) {
                const int k = 16 * kb + kq + j;
                a[j] = to_bf16(th[CW2 + k * NH + 16 * ot + col]);
                b[j] = to_bf16(th[CW3 + k * NH + 16 * ot + col]);
            }
            put(4 + 4 * ot + kb, a);
            put(20 + 4 * ot + kb, b);
        }
    }
    for (int kb = 0; kb < 4; ++kb) {
        v4s w;
        for (int j = 0; j < 4; ++j)
            w[j] = col < NOUT ? to_bf16(th[CW4 + (16 * kb + kq + j) * NOUT + col]) : (short)0;
        put(36 + kb, w);
    }
    const int boffs[3] = {CB1, CB2, CB3};
    for (int l = 0; l < 3; ++l)
        for (int ot = 0; ot < 4; ++ot)
            btile[(4 * l + ot) * 64 + lane] =
                make_float4(th[boffs[l] + 16 * ot + kq], th[boffs[l] + 16 * ot + kq + 1],
                            th[boffs[l] + 16 * ot + kq + 2], th[boffs[l] + 16 * ot + kq + 3]);
    float b4[4];
    for (int e = 0; e < 4; ++e) b4[e] = kq + e < NOUT ? th[CB4 + kq + e] : 0.f;
    btile[12 * 64 + lane] = make_float4(b4[0], b4[1], b4[2], b4[3]);
}

__global__ void __launch_bounds__(CL_THREADS, 3) k_cluster_step(const float2 *__restrict__ p,
                                                             float2 *__restrict__ q,
                                                             const uint2 *__restrict__ frag,
                                                             const float4 *__restrict__ btile,
                                                             ClusterArgs c) {
#pragma clang fp contract(off)
    __shared__ float sf[CL_WAVES][2][16];
    const int i = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, kq = 4 * (lane >> 4);
    auto ld = [&](int f) { return __builtin_bit_cast(v4s, frag[f * 64 + lane]); };
    auto lb = [&](int t) {
        const float4 b = btile[t * 64 + lane];
        v4f v = {b.x, b.y, b.z, b.w};
        return v;
    };
    // A operands (weights) and accumulator tiles (biases), see k_pack_cluster_net
    v4s w1[4], w2[4][4], w3[4][4], w4[4];
    v4f bias[3][4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        w1[ot] = ld(ot);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            w2[ot][kb] = ld(4 + 4 * ot + kb);
            w3[ot][kb] = ld(20 + 4 * ot + kb);
        }
#pragma unroll
        for (int l = 0; l < 3; ++l) bias[l][ot] = lb(4 * l + ot);
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) w4[kb] = ld(36 + kb);
    const v4f b4 = lb(12);

    const float2 pi = p[i];
    float fx = 0.f, fy = 0.f;
    for (int j0 = 16 * wave; j0 < c.n; j0 += 16 * CL_WAVES) {   // wave-uniform trip count
        const int j = j0 + col;
        const float2 pj = j < c.n ? p[j] : pi;
        float dx = pi.x - pj.x, dy = pi.y - pj.y;
        dx -= c.box * rintf(dx * c.inv_box);
        dy -= c.box * rintf(dy * c.inv_box);
        const float r = sqrtf(dx * dx + dy * dy), rr = r * c.inv_radius;
        v4s h0 = {0, 0, 0, 0};
        if (kq == 0) {
            h0[0] = to_bf16((rr - c.xm[0]) * c.inv_xs[0]);
#pragma unroll
            for (int k = 1; k < 4; ++k) h0[k] = to_bf16((c.feat[k - 1] - c.xm[k]) * c.inv_xs[k]);
        }
        // each accumulator starts from the bias of its neuron (row), so the matrix core
        // adds it in its float32 sum
        v4s h1[4], h2[4], h3[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            v4f z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1[ot], h0, bias[0][ot], 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) z[e] = tanh_hw(z[e]);
            h1[ot] = bf16x4(z);
        }
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            v4f z = bias[1][ot];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w2[ot][kb], h1[kb], z, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) z[e] = tanh_hw(z[e]);
            h2[ot] = bf16x4(z);
        }
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            v4f z = bias[2][ot];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w3[ot][kb], h2[kb], z, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) z[e] = tanh_hw(z[e]);
            h3[ot] = bf16x4(z);
        }
        v4f y = b4;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w4[kb], h3[kb], y, 0, 0, 0);
        // lanes 0..15 hold output row 0 (the force) of partner j in y[0]
        if (kq == 0 && j < c.n && j != i && r > 0.f && rr <= c.r_cut) {
            const float f = rr < c.r_contact ? c.k_contact * (c.r_contact - rr)
                                             : y[0] * c.ys + c.ym;
            const float fr = f / r;
            fx += fr * dx;
            fy += fr * dy;
        }
    }
    if (kq == 0) {
        sf[wave][0][col] = fx;
        sf[wave][1][col] = fy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float sx = 0.f, sy = 0.f;
        for (int w = 0; w < CL_WAVES; ++w)
            for (int l = 0; l < 16; ++l) {
                sx += sf[w][0][l];
                sy += sf[w][1][l];
            }
        float x = pi.x + c.mobility * sx, y = pi.y + c.mobility * sy;
        x -= c.box * floorf(x / c.box);
        y -= c.box * floorf(y / c.box);
        q[i] = make_float2(x, y);
    }
}

}  // namespace

struct lbm_surrogate {
    std::string err;
    hipStream_t st = nullptr;
    int dev = 0;                         // device of the stream and the buffers
    int cap = 0, n = 0;
    int64_t t = 0;                       // Adam steps taken
    float *th = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    float *x = nullptr, *y = nullptr, *tg = nullptr, *w = nullptr, *dy = nullptr, *part = nullptr;
    float *slices = nullptr;             // split-K partial products [KS_MAX][64][64]
    float *gtrain = nullptr;             // the training workgroups' gradients [TC_BLOCKS][NPAR]
    float *act[NLAYER] = {nullptr, nullptr, nullptr, nullptr};   // input, tanh of 3 layers
    float *d[NLAYER] = {nullptr, nullptr, nullptr, nullptr};     // back-propagated dL/dz
    double wsum = 0.0;
};

namespace {

thread_local std::string g_err;

lbm_status sfail(lbm_surrogate *s, lbm_status c, const std::string &m) {
    s->err = m;
    return c;
}

// split K into at most KS_MAX slices of at least 64 (products with a long K, i.e. the
// weight gradients summed over the samples, would otherwise run on a handful of waves)
constexpr int KS_MAX = 32;

void gemm(hipStream_t st, const float *A, int sar, int sac, const float *B, int sbr, int sbc,
          float *C, int ldc, int M, int N, int K, int epi, const float *bias, const float *P,
          float *slices = nullptr) {
    const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
    if (slices && epi == EPI_STORE && K > 128 && M <= NH && N <= NH) {
        int ns = (K + 63) / 64;
        ns = ns < KS_MAX ? ns : KS_MAX;
        const int kz = ((K + ns - 1) / ns + 15) / 16 * 16;
        ns = (K + kz - 1) / kz;
        hipLaunchKernelGGL(k_gemm_bf16, dim3((tiles + 3) / 4, ns), dim3(256), 0, st, A, sar, sac, B,
                           sbr, sbc, slices, N, M, N, K, EPI_STORE, nullptr, nullptr, kz);
        hipLaunchKernelGGL(k_sum_slices, dim3((M * N + 255) / 256), dim3(256), 0, st, slices, ns, M,
                           N, C, ldc);
        return;
    }
    hipLaunchKernelGGL(k_gemm_bf16, dim3((tiles + 3) / 4), dim3(256), 0, st, A, sar, sac, B, sbr,
                       sbc, C, ldc, M, N, K, epi, bias, P, 0);
}

// forward pass over n rows of X (activations kept for back-propagation), output into Y
void forward(lbm_surrogate *s, const float *X, float *Y, int n) {
    const float *h = X;
    for (int l = 0; l < NLAYER; ++l) {
        const int ki = LIN[l], no = LOUT[l];
        const float *W = s->th + woff(l), *b = s->th + boff(l);
        float *out = l < NLAYER - 1 ? s->act[l + 1] : Y;
        gemm(s->st, h, ki, 1, W, no, 1, out, no, n, no, ki, l < NLAYER - 1 ? EPI_BIAS_TANH : EPI_BIAS,
             b, nullptr);
        h = out;
    }
}

// gradient of the loss at the current parameters over the stored data, into s->g
void backward(lbm_surrogate *s) {
    const int n = s->n;
    forward(s, s->act[0], s->y, n);
    hipLaunchKernelGGL(k_loss_grad, dim3((n + 255) / 256), dim3(256), 0, s->st, s->y, s->tg, s->w,
                       (float)(1.0 / s->wsum), n, s->dy, s->part);
    const float *dl = s->dy;   // dL/dz of layer l
    for (int l = NLAYER - 1; l >= 0; --l) {
        const int ki = LIN[l], no = LOUT[l];
        // dW_l = act_l^T dl   (ki x no, summed over the n rows)
        gemm(s->st, s->act[l], 1, ki, dl, no, 1, s->g + woff(l), no, ki, no, n, EPI_STORE,
             nullptr, nullptr, s->slices);
        hipLaunchKernelGGL(k_colsum, dim3(no), dim3(256), 0, s->st, dl, n, no, s->g + boff(l));
        if (l > 0) {   // dL/dz_{l-1} = (dl W_l^T) * (1 - act_l^2)
            gemm(s->st, dl, no, 1, s->th + woff(l), 1, no, s->d[l - 1], ki, n, ki, no,
                 EPI_TANH_GRAD, nullptr, s->act[l]);
            dl = s->d[l - 1];
        }
    }
}

}  // namespace

extern "C" lbm_status lbm_surrogate_create(int32_t max_samples, const float *theta0,
                                           lbm_surrogate **out) {
    if (!out) return LBM_E_INVAL;
    *out = nullptr;
    if (max_samples < 1 || max_samples > (1 << 20) || !theta0) {
        g_err = "max_samples must be 1 .. 2^20 and theta0 given";
        return LBM_E_INVAL;
    }
    lbm_surrogate *s = new (std::nothrow) lbm_surrogate();
    if (!s) return LBM_E_NOMEM;
    s->cap = max_samples;
    const size_t c = (size_t)max_samples;
    bool ok = hipGetDevice(&s->dev) == hipSuccess &&
              hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) == hipSuccess;
    float **bufs[] = {&s->th, &s->m, &s->v, &s->g};
    for (float **b : bufs) ok = ok && hipMalloc(b, NPAR * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc(&s->y, c * NOUT * sizeof(float)) == hipSuccess &&
         hipMalloc(&s->tg, c * NOUT * sizeof(float)) == hipSuccess &&
         hipMalloc(&s->dy, c * NOUT * sizeof(float)) == hipSuccess &&
         hipMalloc(&s->w, c * sizeof(float)) == hipSuccess &&
         hipMalloc(&s->part, ((c + 255) / 256) * sizeof(float)) == hipSuccess &&
         hipMalloc(&s->slices, (size_t)KS_MAX * NH * NH * sizeof(float)) == hipSuccess &&
         hipMalloc(&s->gtrain, (size_t)TC_BLOCKS * NPAR * sizeof(float)) == hipSuccess;
    for (int l = 0; l < NLAYER && ok; ++l)
        ok = hipMalloc(&s->act[l], c * LIN[l] * sizeof(float)) == hipSuccess &&
             hipMalloc(&s->d[l], c * LOUT[l] * sizeof(float)) == hipSuccess;
    s->x = s->act[0];
    ok = ok && hipMemcpy(s->th, theta0, NPAR * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(s->m, 0, NPAR * sizeof(float)) == hipSuccess &&
         hipMemset(s->v, 0, NPAR * sizeof(float)) == hipSuccess;
    if (!ok) {
        lbm_surrogate_destroy(s);
        g_err = "device allocation failed (surrogate)";
        return LBM_E_NOMEM;
    }
    *out = s;
    return LBM_OK;
}

extern "C" lbm_status lbm_surrogate_set_data(lbm_surrogate *s, int32_t n, const float *x,
                                             const float *t, const float *w) {
    if (!s) return LBM_E_INVAL;
    if (n < 1 || n > s->cap || !x || !t) return sfail(s, LBM_E_INVAL, "need 1 .. max_samples samples");
    std::vector<float> wv(n, 1.0f);
    if (w) wv.assign(w, w + n);
    double ws = 0.0;
    for (float v : wv) {
        if (!(v >= 0.0f) || !std::isfinite(v)) return sfail(s, LBM_E_INVAL, "weights must be finite and >= 0");
        ws += v;
    }
    if (!(ws > 0.0)) return sfail(s, LBM_E_INVAL, "weights sum to zero");
    for (int i = 0; i < n * NIN; ++i)
        if (!std::isfinite(x[i])) return sfail(s, LBM_E_INVAL, "non-finite input");
    for (int i = 0; i < n * NOUT; ++i)
        if (!std::isfinite(t[i])) return sfail(s, LBM_E_INVAL, "non-finite target");
    if (hipStreamSynchronize(s->st) != hipSuccess ||
        hipMemcpy(s->x, x, (size_t)n * NIN * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->tg, t, (size_t)n * NOUT * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->w, wv.data(), (size_t)n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return sfail(s, LBM_E_DEVICE, "data upload failed");
    s->n = n;
    s->wsum = ws;
    return LBM_OK;
}

extern "C" lbm_status lbm_surrogate_gradient(lbm_surrogate *s, float *loss, float *grad) {
    if (!s || !grad) return LBM_E_INVAL;
    if (s->n == 0) return sfail(s, LBM_E_STATE, "no training data");
    backward(s);
    std::vector<float> part((s->n + 255) / 256);
    if (hipMemcpyAsync(grad, s->g, NPAR * sizeof(float), hipMemcpyDeviceToHost, s->st) != hipSuccess ||
        hipMemcpyAsync(part.data(), s->part, part.size() * sizeof(float), hipMemcpyDeviceToHost, s->st) != hipSuccess ||
        hipStreamSynchronize(s->st) != hipSuccess)
        return sfail(s, LBM_E_DEVICE, "gradient read-back failed");
    if (loss) {
        double a = 0.0;
        for (float p : part) a += p;
        *loss = (float)(0.5 * a / s->wsum);
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_surrogate_train(lbm_surrogate *s, int32_t steps, float lr) {
    if (!s) return LBM_E_INVAL;
    if (s->n == 0) return sfail(s, LBM_E_STATE, "no training data");
    if (steps < 0 || !(lr > 0.0f)) return sfail(s, LBM_E_INVAL, "steps >= 0 and lr > 0");
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    // one launch computes the gradient (chunks of TC_ROWS samples over up to TC_BLOCKS workgroups),
    // a second sums the workgroups' gradients and takes the Adam step
    const int chunks = (s->n + TC_ROWS - 1) / TC_ROWS;
    const int nb = chunks < TC_BLOCKS ? chunks : TC_BLOCKS;
    TrainArgs ta{s->th, s->x, s->tg, s->w, s->gtrain, s->n, (float)(1.0 / s->wsum)};
    for (int i = 0; i < steps; ++i) {
        hipLaunchKernelGGL(k_train_chunk, dim3(nb), dim3(TC_THREADS), 0, s->st, ta);
        ++s->t;
        const float c1 = (float)(1.0 - std::pow(0.9, (double)s->t));
        const float c2 = (float)(1.0 - std::pow(0.999, (double)s->t));
        hipLaunchKernelGGL(k_train_update, dim3((NPAR + 255) / 256), dim3(256), 0, s->st, s->th,
                           s->m, s->v, s->gtrain, nb, lr, b1, b2, c1, c2, eps);
    }
    if (hipStreamSynchronize(s->st) != hipSuccess || hipGetLastError() != hipSuccess)
        return sfail(s, LBM_E_DEVICE, "training launch failed");
    return LBM_OK;
}

extern "C" lbm_status lbm_surrogate_predict(lbm_surrogate *s, int32_t n, const float *x, float *y) {
    if (!s) return LBM_E_INVAL;
    if (n < 1 || n > s->cap || !x || !y) return sfail(s, LBM_E_INVAL, "need 1 .. max_samples inputs");
    // the activations of the stored data are overwritten; the data itself is kept
    float *xin = nullptr, *yout = nullptr;
    bool ok = hipMalloc(&xin, (size_t)n * NIN * sizeof(float)) == hipSuccess &&
              hipMalloc(&yout, (size_t)n * NOUT * sizeof(float)) == hipSuccess &&
              hipStreamSynchronize(s->st) == hipSuccess &&
              hipMemcpy(xin, x, (size_t)n * NIN * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
    if (ok) {
        forward(s, xin, yout, n);
        ok = hipMemcpyAsync(y, yout, (size_t)n * NOUT * sizeof(float), hipMemcpyDeviceToHost, s->st) == hipSuccess &&
             hipStreamSynchronize(s->st) == hipSuccess;
    }
    if (xin) (void)hipFree(xin);
    if (yout) (void)hipFree(yout);
    return ok ? LBM_OK : sfail(s, LBM_E_DEVICE, "prediction failed");
}

extern "C" lbm_status lbm_surrogate_cluster(lbm_surrogate *s, int32_t n, float *xy, int32_t steps,
                                            const lbm_cluster_params *cp) {
    if (!s) return LBM_E_INVAL;
    if (!xy || !cp || n < 2 || steps < 0)
        return sfail(s, LBM_E_INVAL, "need n >= 2 capsules, positions and parameters");
    if (!(cp->box > 0.f) || !(cp->radius > 0.f) || !(cp->r_cut > cp->r_contact) ||
        !(cp->r_contact >= 0.f) || !(cp->k_contact >= 0.f) || !std::isfinite(cp->mobility))
        return sfail(s, LBM_E_INVAL, "invalid cluster parameters");
    for (int k = 0; k < 4; ++k)
        if (!(cp->in_scale[k] > 0.f)) return sfail(s, LBM_E_INVAL, "input scales must be > 0");
    // the minimum image finds every partner within the cutoff only if the cutoff is below
    // half the box
    if (!(2.0 * cp->r_cut * cp->radius < cp->box))
        return sfail(s, LBM_E_INVAL, "box must exceed twice the cutoff distance r_cut * radius");
    ClusterArgs c{};
    for (int k = 0; k < 4; ++k) { c.xm[k] = cp->in_mean[k]; c.inv_xs[k] = 1.0f / cp->in_scale[k]; }
    c.ym = cp->out_mean[0];
    c.ys = cp->out_scale[0];
    c.feat[0] = cp->log10_ks; c.feat[1] = cp->film; c.feat[2] = cp->angle;
    c.box = cp->box; c.inv_box = 1.0f / cp->box; c.inv_radius = 1.0f / cp->radius;
    c.r_contact = cp->r_contact; c.r_cut = cp->r_cut; c.k_contact = cp->k_contact;
    c.mobility = cp->mobility; c.n = n;
    float2 *p[2] = {nullptr, nullptr};
    uint2 *frag = nullptr;
    float4 *btile = nullptr;
    bool ok = hipMalloc(&p[0], n * sizeof(float2)) == hipSuccess &&
              hipMalloc(&p[1], n * sizeof(float2)) == hipSuccess &&
              hipMalloc(&frag, CL_FRAGS * 64 * sizeof(uint2)) == hipSuccess &&
              hipMalloc(&btile, CL_BTILES * 64 * sizeof(float4)) == hipSuccess &&
              hipStreamSynchronize(s->st) == hipSuccess &&
              hipMemcpy(p[0], xy, n * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess;
    if (ok && steps > 0)
        hipLaunchKernelGGL(k_pack_cluster_net, dim3(1), dim3(64), 0, s->st, s->th, frag, btile);
    int cur = 0;
    for (int t = 0; t < steps && ok; ++t) {
        hipLaunchKernelGGL(k_cluster_step, dim3(n), dim3(CL_THREADS), 0, s->st, p[cur], p[1 - cur],
                           frag, btile, c);
        cur = 1 - cur;
    }
    ok = ok && hipGetLastError() == hipSuccess &&
         hipMemcpyAsync(xy, p[cur], n * sizeof(float2), hipMemcpyDeviceToHost, s->st) == hipSuccess &&
         hipStreamSynchronize(s->st) == hipSuccess;
    for (float2 *b : p)
        if (b) (void)hipFree(b);
    if (frag) (void)hipFree(frag);
    if (btile) (void)hipFree(btile);
    return ok ? LBM_OK : sfail(s, LBM_E_DEVICE, "cluster evolution failed");
}

// ------------------------------------------------------------------------------------
// Cluster evolution without allocation
// ------------------------------------------------------------------------------------
// File-scope scratch of the allocation-free entry point, one copy per device: the second
// position buffer of the step's ping-pong (LBM_CLUSTER_NOALLOC_MAX float2) and the network
// in operand layout (bfloat16 fragments and bias tiles), each part 256-byte aligned.
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t SCR_POS = 0;
constexpr size_t SCR_FRAG = align256(SCR_POS + (size_t)LBM_CLUSTER_NOALLOC_MAX * sizeof(float2));
constexpr size_t SCR_BTILE = align256(SCR_FRAG + (size_t)CL_FRAGS * 64 * sizeof(uint2));
constexpr size_t SCR_BYTES = align256(SCR_BTILE + (size_t)CL_BTILES * 64 * sizeof(float4));

static __device__ __align__(256) unsigned char scratch[SCR_BYTES];

// device address of `scratch` on each device, taken once per device with that device
// current (the host-side name of the array is not a device address)
constexpr int SCR_MAX_DEVICES = 64;
static std::mutex g_scr_mutex;
static void *g_scr_ptr[SCR_MAX_DEVICES] = {};

static hipError_t scratch_of(int dev, unsigned char **out) {
    if (dev < 0 || dev >= SCR_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scr_mutex);
    if (!g_scr_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scr_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char *>(g_scr_ptr[dev]);
    return hipSuccess;
}

extern "C" lbm_status lbm_surrogate_cluster_noalloc(lbm_surrogate *s, int32_t n, float *xy_device,
                                                    int32_t steps, const lbm_cluster_params *cp) {
    if (!s) return LBM_E_INVAL;
    if (!xy_device || !cp || n < 2 || steps < 0)
        return sfail(s, LBM_E_INVAL, "need n >= 2 capsules, device positions and parameters");
    if (n > LBM_CLUSTER_NOALLOC_MAX)
        return sfail(s, LBM_E_INVAL, "n exceeds LBM_CLUSTER_NOALLOC_MAX (the scratch holds "
                                     "that many positions)");
    if (!(cp->box > 0.f) || !(cp->radius > 0.f) || !(cp->r_cut > cp->r_contact) ||
        !(cp->r_contact >= 0.f) || !(cp->k_contact >= 0.f) || !std::isfinite(cp->mobility))
        return sfail(s, LBM_E_INVAL, "invalid cluster parameters");
    for (int k = 0; k < 4; ++k)
        if (!(cp->in_scale[k] > 0.f)) return sfail(s, LBM_E_INVAL, "input scales must be > 0");
    if (!(2.0 * cp->r_cut * cp->radius < cp->box))
        return sfail(s, LBM_E_INVAL, "box must exceed twice the cutoff distance r_cut * radius");
    // the scratch address is taken, and the kernels run, with the surrogate's device current;
    // the caller's current device is restored on return
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(s->dev) != hipSuccess)
        return sfail(s, LBM_E_DEVICE, "hipSetDevice failed");
    struct Restore {
        int d;
        ~Restore() { (void)hipSetDevice(d); }
    } restore{prev};
    unsigned char *scr = nullptr;
    if (scratch_of(s->dev, &scr) != hipSuccess)
        return sfail(s, LBM_E_DEVICE, "hipGetSymbolAddress of the scratch array failed");
    ClusterArgs c{};
    for (int k = 0; k < 4; ++k) { c.xm[k] = cp->in_mean[k]; c.inv_xs[k] = 1.0f / cp->in_scale[k]; }
    c.ym = cp->out_mean[0];
    c.ys = cp->out_scale[0];
    c.feat[0] = cp->log10_ks; c.feat[1] = cp->film; c.feat[2] = cp->angle;
    c.box = cp->box; c.inv_box = 1.0f / cp->box; c.inv_radius = 1.0f / cp->radius;
    c.r_contact = cp->r_contact; c.r_cut = cp->r_cut; c.k_contact = cp->k_contact;
    c.mobility = cp->mobility; c.n = n;
    float2 *p[2] = {reinterpret_cast<float2 *>(xy_device), reinterpret_cast<float2 *>(scr + SCR_POS)};
    uint2 *frag = reinterpret_cast<uint2 *>(scr + SCR_FRAG);
    float4 *btile = reinterpret_cast<float4 *>(scr + SCR_BTILE);
    // the positions and the network fragments in the scratch are written before they are
    // read in every call, so nothing of an earlier call's contents is used
    if (steps > 0)
        hipLaunchKernelGGL(k_pack_cluster_net, dim3(1), dim3(64), 0, s->st, s->th, frag, btile);
    int cur = 0;
    for (int t = 0; t < steps; ++t) {
        hipLaunchKernelGGL(k_cluster_step, dim3(n), dim3(CL_THREADS), 0, s->st, p[cur], p[1 - cur],
                           frag, btile, c);
        cur = 1 - cur;
    }
    bool ok = hipGetLastError() == hipSuccess;
    if (ok && cur == 1)         // an odd step count leaves the result in the scratch
        ok = hipMemcpyAsync(p[0], p[1], n * sizeof(float2), hipMemcpyDeviceToDevice, s->st) == hipSuccess;
    ok = ok && hipStreamSynchronize(s->st) == hipSuccess;
    return ok ? LBM_OK : sfail(s, LBM_E_DEVICE, "cluster evolution failed");
}

extern "C" lbm_status lbm_surrogate_params(lbm_surrogate *s, float *theta) {
    if (!s || !theta) return LBM_E_INVAL;
    if (hipStreamSynchronize(s->st) != hipSuccess ||
        hipMemcpy(theta, s->th, NPAR * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return sfail(s, LBM_E_DEVICE, "parameter read-back failed");
    return LBM_OK;
}

extern "C" const char *lbm_surrogate_last_error(const lbm_surrogate *s) {
    return s ? s->err.c_str() : g_err.c_str();
}

extern "C" void lbm_surrogate_destroy(lbm_surrogate *s) {
    if (!s) return;
    if (s->st) (void)hipStreamSynchronize(s->st);
    float *bufs[] = {s->th, s->m, s->v, s->g, s->y, s->tg, s->dy, s->w, s->part, s->slices,
                     s->gtrain};
    for (float *b : bufs)
        if (b) (void)hipFree(b);
    for (int l = 0; l < NLAYER; ++l) {
        if (s->act[l]) (void)hipFree(s->act[l]);
        if (s->d[l]) (void)hipFree(s->d[l]);
    }
    if (s->st) (void)hipStreamDestroy(s->st);
    delete s;
}
