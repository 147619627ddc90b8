// Surrogate multilayer perceptron for candidate screening (BF16 MFMA, FP32
// accumulation, FP32 Adam).
//
// Not part of the paper: it learns the map from control-node velocities to
// the (standardised) log-misfit that the finite-difference fitness produces
// during the search, so that candidate particles can be ranked before the
// expensive evaluation.
//
// Network: x_hat = (x - lo)/(hi - lo); h_l = GELU(W_l h_{l-1} + b_l) for three
// hidden layers of width H (exact erf GELU); y = w4 . h_3 + b4.
// Parameters live in one FP32 buffer (master copy, layout below); the weight
// matrices also have a BF16 copy that the MFMA GEMMs read. Activations that
// feed a GEMM are BF16; every GEMM accumulates in FP32.
//
// FP32 parameter layout (P = H*D + H + 2*(H*H + H) + H + 1 floats):
//   W1 [H][D] | b1 [H] | W2 [H][H] | b2 [H] | W3 [H][H] | b3 [H] | w4 [H] | b4 [1]
// BF16 copy: W1 [H][D] | W2 [H][H] | W3 [H][H].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "common.h"

namespace {

struct MlpOff {
    size_t W1, b1, W2, b2, W3, b3, w4, b4, P;   // offsets into the FP32 buffer
    size_t bW1, bW2, bW3, PB;                   // offsets into the BF16 copy
};

MlpOff mlp_offsets(int D, int H) {
    MlpOff o;
    size_t k = 0;
    o.W1 = k; k += (size_t)H * D;
    o.b1 = k; k += H;
    o.W2 = k; k += (size_t)H * H;
    o.b2 = k; k += H;
    o.W3 = k; k += (size_t)H * H;
    o.b3 = k; k += H;
    o.w4 = k; k += H;
    o.b4 = k; k += 1;
    o.P = k;
    k = 0;
    o.bW1 = k; k += (size_t)H * D;
    o.bW2 = k; k += (size_t)H * H;
    o.bW3 = k; k += (size_t)H * H;
    o.PB = k;
    return o;
}

// Workspace of one forward/backward pass over n rows.
struct MlpWs {
    size_t Xb, Z1, Z2, Z3, H1, H2, H3, y, dy, dZ1, dZ2, dZ3, dZ1b, dZ2b, dZ3b, grads, loss, total;
};

MlpWs mlp_ws(int D, int H, int n) {
    MlpWs w;
    const MlpOff o = mlp_offsets(D, H);
    size_t k = 0;
    auto take = [&](size_t bytes) { size_t r = k; k = empso::align_up(k + bytes, 256); return r; };
    const size_t nh = (size_t)n * H;
    w.Xb = take(sizeof(uint16_t) * (size_t)n * D);
    w.Z1 = take(4 * nh); w.Z2 = take(4 * nh); w.Z3 = take(4 * nh);
    w.H1 = take(2 * nh); w.H2 = take(2 * nh); w.H3 = take(2 * nh);
    w.y = take(4 * (size_t)n); w.dy = take(4 * (size_t)n);
    w.dZ1 = take(4 * nh); w.dZ2 = take(4 * nh); w.dZ3 = take(4 * nh);
    w.dZ1b = take(2 * nh); w.dZ2b = take(2 * nh); w.dZ3b = take(2 * nh);
    w.grads = take(4 * o.P);
    w.loss = take(8);
    w.total = k;
    return w;
}

// FP32 -> BF16 with round-to-nearest-even (finite inputs), BF16 -> FP32.
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

enum Epi { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_GELU_GRAD = 2 };

struct Gemm {
    const uint16_t *A, *B;      // BF16 operands: A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]
    int M, N, K;
    int sam, sak, sbk, sbn;
    int epi;
    const float *bias;          // EPI_BIAS_GELU: [N]
    const float *Zin;           // EPI_GELU_GRAD: pre-activation [M][N] (row stride N)
    float *outf;                // FP32 output [M][N] (Z for EPI_BIAS_GELU, dZ for EPI_GELU_GRAD, C for EPI_STORE)
    uint16_t *outb;             // BF16 output [M][N] (GELU(z) or dz), may be NULL
};

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

// C = A * B with one 64-lane wavefront per 16x16 output tile and
// v_mfma_f32_16x16x32_bf16 (K = 32 per instruction): the small batches of the
// surrogate give few output tiles, so small tiles keep more wavefronts busy.
// Operand lanes: lane i supplies A row (i mod 16), B column (i mod 16), and
// the same 8 K indices 8*(i div 16) .. +7 of the 32-wide K slice for both
// operands (the product does not depend on how the instruction orders K
// internally, only on A and B using the same assignment). Result: lane i
// holds column (i mod 16), rows 4*(i div 16) + j for j = 0..3.
// Out-of-range rows, columns and K elements are read as zero.
__global__ __launch_bounds__(256) void k_gemm(const Gemm g) {
    const int lane = threadIdx.x & 63;
    const int tilesN = (g.N + 15) / 16;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tilesM = (g.M + 15) / 16;
    if (tile >= tilesM * tilesN) return;
    const int m0 = (tile / tilesN) * 16, n0 = (tile % tilesN) * 16;
    const int r = lane & 15, kh = (lane >> 4) * 8;
    const int am = m0 + r, bn = n0 + r;
    f4v acc = {};
    for (int k0 = 0; k0 < g.K; k0 += 32) {
        s8v a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + kh + e;
            a[e] = (am < g.M && k < g.K) ? (short)g.A[(size_t)am * g.sam + (size_t)k * g.sak] : (short)0;
            b[e] = (bn < g.N && k < g.K) ? (short)g.B[(size_t)k * g.sbk + (size_t)bn * g.sbn] : (short)0;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), acc,
                                                      0, 0, 0);
    }
    const int col = n0 + r;
    if (col >= g.N) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = m0 + 4 * (lane >> 4) + j;
        if (row >= g.M) continue;
        const size_t o = (size_t)row * g.N + col;
        const float v = acc[j];
        if (g.epi == EPI_STORE) {
            g.outf[o] = v;
        } else if (g.epi == EPI_BIAS_GELU) {
            const float z = v + g.bias[col];
            if (g.outf) g.outf[o] = z;
            g.outb[o] = f2bf(gelu(z));
        } else {
            const float dz = v * gelu_grad(g.Zin[o]);
            g.outf[o] = dz;
            g.outb[o] = f2bf(dz);
        }
    }
}

// The same product for K <= 32 KS (KS <= 8, the surrogate's widths): every
// lane requests all its K slices before the first MFMA, so a wavefront waits
// for one round of loads instead of one per slice; where both operands are
// contiguous along K and 16-byte aligned (VEC) each slice of an operand is
// one 16-byte load instead of eight 2-byte ones (the forward products of the
// hidden layers). The MFMAs run in the same order on the same operands as in
// k_gemm, so the results are bit for bit those of k_gemm.
template <int KS, bool VEC>
__global__ __launch_bounds__(256) void k_gemm_pre(const Gemm g) {
    const int lane = threadIdx.x & 63;
    const int tilesN = (g.N + 15) / 16;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tilesM = (g.M + 15) / 16;
    if (tile >= tilesM * tilesN) return;
    const int m0 = (tile / tilesN) * 16, n0 = (tile % tilesN) * 16;
    const int r = lane & 15, kh = (lane >> 4) * 8;
    const int am = m0 + r, bn = n0 + r;
    s8v a[KS], b[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int kb = 32 * s + kh;
        if (VEC) {
            const s8v z = {};
            a[s] = am < g.M ? *reinterpret_cast<const s8v *>(g.A + (size_t)am * g.sam + kb) : z;
            b[s] = bn < g.N ? *reinterpret_cast<const s8v *>(g.B + (size_t)bn * g.sbn + kb) : z;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = kb + e;
                a[s][e] = (am < g.M && k < g.K) ? (short)g.A[(size_t)am * g.sam + (size_t)k * g.sak] : (short)0;
                b[s][e] = (bn < g.N && k < g.K) ? (short)g.B[(size_t)k * g.sbk + (size_t)bn * g.sbn] : (short)0;
            }
        }
    }
    f4v acc = {};
#pragma unroll
    for (int s = 0; s < KS; ++s)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a[s]), __builtin_bit_cast(bf8, b[s]), acc,
                                                      0, 0, 0);
    const int col = n0 + r;
    if (col >= g.N) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = m0 + 4 * (lane >> 4) + j;
        if (row >= g.M) continue;
        const size_t o = (size_t)row * g.N + col;
        const float v = acc[j];
        if (g.epi == EPI_STORE) {
            g.outf[o] = v;
        } else if (g.epi == EPI_BIAS_GELU) {
            const float z = v + g.bias[col];
            if (g.outf) g.outf[o] = z;
            g.outb[o] = f2bf(gelu(z));
        } else {
            const float dz = v * gelu_grad(g.Zin[o]);
            g.outf[o] = dz;
            g.outb[o] = f2bf(dz);
        }
    }
}

// x_hat = (x - lo)/(hi - lo) in BF16; rows optionally gathered through idx.
__global__ void k_mlp_input(const float *__restrict__ X, const int *__restrict__ idx, const float *__restrict__ lo,
                            const float *__restrict__ hi, int n, int D, uint16_t *__restrict__ Xb) {
    const int64_t total = (int64_t)n * D;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(k / D), d = (int)(k - (int64_t)m * D);
        const int row = idx ? idx[m] : m;
        const float x = X[(size_t)row * D + d];
        Xb[k] = f2bf((x - lo[d]) / (hi[d] - lo[d]));
    }
}

// y[m] = w4 . h3[m] + b4 (FP32 accumulation in a fixed order).
// Sum over the 64 lanes of a wavefront (butterfly: every lane gets the same bits).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// y[m] = w4 . h3[m] + b4, one wavefront per row.
__global__ __launch_bounds__(256) void k_head_fwd(const uint16_t *__restrict__ H3, const float *__restrict__ w4,
                                                  const float *__restrict__ b4, int n, int H, float *__restrict__ y) {
    const int m = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (m >= n) return;
    float s = 0.0f;
    for (int h = lane; h < H; h += 64) s = fmaf(w4[h], bf2f(H3[(size_t)m * H + h]), s);
    s = wave_sum(s);
    if (lane == 0) y[m] = s + b4[0];
}

// Targets from the evaluated fitness: t = (log(max(f, tiny)) - mu)/sigma.
// dy = 2 (y - t)/n, and the loss mean((y - t)^2) summed in a fixed order.
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ y, const float *__restrict__ fit,
                                              const int *__restrict__ idx, float mu, float sigma, int n,
                                              float *__restrict__ dy, float *__restrict__ loss) {
    double s = 0.0;
    for (int m = threadIdx.x; m < n; m += blockDim.x) {
        const float f = fit[idx ? idx[m] : m];
        const float t = (logf(fmaxf(f, 1e-30f)) - mu) / sigma;
        const float r = y[m] - t;
        dy[m] = 2.0f * r / (float)n;
        s += (double)r * (double)r;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(red[0] / n);
}

// Head backward: dw4[h] = sum_m dy[m] h3[m][h], db4 = sum_m dy[m],
// dz3[m][h] = dy[m] w4[h] GELU'(z3[m][h]).
// dZ3[m][h] = dy[m] w4[h] GELU'(Z3[m][h]) (FP32 and BF16 copies).
__global__ __launch_bounds__(256) void k_head_dz(const float *__restrict__ dy, const float *__restrict__ Z3,
                                                 const float *__restrict__ w4, int n, int H, float *__restrict__ dZ3,
                                                 uint16_t *__restrict__ dZ3b) {
    const int64_t total = (int64_t)n * H;
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total; o += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(o / H), h = (int)(o - (int64_t)m * H);
        const float dz = dy[m] * w4[h] * gelu_grad(Z3[o]);
        dZ3[o] = dz;
        dZ3b[o] = f2bf(dz);
    }
}

__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(uint16_t v) { return bf2f(v); }

// out[h] = sum over rows m of (wt ? wt[m] : 1) * A[m][h] in a fixed order:
// the 16 wavefronts of a block take rows w, w + 16, ... for 64 columns (one
// per lane) and their partial sums are added in wavefront order.
template <typename TA>
__global__ __launch_bounds__(1024) void k_colsum(const TA *__restrict__ A, const float *__restrict__ wt, int n, int H,
                                                 float *__restrict__ out) {
    __shared__ float part[16][64];
    const int lane = threadIdx.x & 63, w = (int)(threadIdx.x >> 6);
    const int h = blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (h < H) {
        for (int m = w; m < n; m += 16) {
            const float a = to_f(A[(size_t)m * H + h]);
            s = wt ? fmaf(wt[m], a, s) : s + a;
        }
    }
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && h < H) {
        float t = 0.0f;
#pragma unroll
        for (int k = 0; k < 16; ++k) t += part[k][lane];
        out[h] = t;
    }
}
// Adam on the FP32 parameters; the updated weights of the three matrices are
// also written to their BF16 copy (element k of matrix i at wb + bdst[i] +
// (k - src[i])), which saves the separate conversion launches.
struct BfMap {
    int64_t src[3], len[3], dst[3];
};
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, int64_t P, float lr, float b1, float b2, float eps, float c1, float c2,
                       uint16_t *__restrict__ wb, const BfMap map) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
        const float gk = g[k];
        const float a = b1 * m1[k] + (1.0f - b1) * gk;
        const float b = b2 * m2[k] + (1.0f - b2) * gk * gk;
        m1[k] = a;
        m2[k] = b;
        const float pk = p[k] - lr * (a / c1) / (sqrtf(b / c2) + eps);
        p[k] = pk;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (k >= map.src[i] && k < map.src[i] + map.len[i]) wb[map.dst[i] + (k - map.src[i])] = f2bf(pk);
    }
}

__global__ void k_to_bf16(const float *__restrict__ src, uint16_t *__restrict__ dst, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = f2bf(src[k]);
}

void launch_gemm(const Gemm &g, hipStream_t st) {
    const int tiles = ((g.M + 15) / 16) * ((g.N + 15) / 16);
    const int blocks = (tiles + 3) / 4;
    const int ks = (g.K + 31) / 32;
    // contiguous along K, whole slices, 16-byte aligned rows
    const bool vec = g.sak == 1 && g.sbk == 1 && g.K % 32 == 0 && g.sam % 8 == 0 && g.sbn % 8 == 0 &&
                     reinterpret_cast<uintptr_t>(g.A) % 16 == 0 && reinterpret_cast<uintptr_t>(g.B) % 16 == 0;
    // strided operands with more than two slices: requesting all of their
    // 2-byte loads at once measured slower (about 22 us against 12 us for
    // the backward products of a 256-row batch) than the slice loop
    if (ks > 8 || (!vec && ks > 2)) {
        k_gemm<<<blocks, 256, 0, st>>>(g);
        return;
    }
#define EMPSO_GEMM_CASE(KS)                                                   \
    if (ks == KS) {                                                           \
        if (vec)                                                              \
            k_gemm_pre<KS, true><<<blocks, 256, 0, st>>>(g);                  \
        else                                                                  \
            k_gemm_pre<KS, false><<<blocks, 256, 0, st>>>(g);                 \
        return;                                                               \
    }
    EMPSO_GEMM_CASE(1) EMPSO_GEMM_CASE(2) EMPSO_GEMM_CASE(3) EMPSO_GEMM_CASE(4)
    EMPSO_GEMM_CASE(5) EMPSO_GEMM_CASE(6) EMPSO_GEMM_CASE(7) EMPSO_GEMM_CASE(8)
#undef EMPSO_GEMM_CASE
}

Gemm fwd_gemm(const uint16_t *A, int lda, const uint16_t *W, int M, int N, int K, const float *bias, float *Z,
              uint16_t *Hb) {
    // Z[m][j] = sum_k A[m][k] W[j][k] + bias[j]  (A row stride lda, W [N][K])
    Gemm g = {};
    g.A = A; g.B = W; g.M = M; g.N = N; g.K = K;
    g.sam = lda; g.sak = 1; g.sbk = 1; g.sbn = K;
    g.epi = EPI_BIAS_GELU; g.bias = bias; g.outf = Z; g.outb = Hb;
    return g;
}

bool check_shape(int D, int H, int n) { return D >= 1 && D <= 4096 && H >= 1 && H <= 4096 && n >= 1 && n <= (1 << 22); }

// Forward pass into the workspace (inputs, three hidden layers, head).
void forward(int D, int H, const float *params, const uint16_t *wb, const float *lo, const float *hi, const float *X,
             const int *idx, int n, unsigned char *ws, hipStream_t st) {
    const MlpOff o = mlp_offsets(D, H);
    const MlpWs w = mlp_ws(D, H, n);
    uint16_t *Xb = (uint16_t *)(ws + w.Xb);
    const int blocks = (int)std::min<int64_t>(1024, ((int64_t)n * D + 255) / 256);
    k_mlp_input<<<blocks, 256, 0, st>>>(X, idx, lo, hi, n, D, Xb);
    launch_gemm(fwd_gemm(Xb, D, wb + o.bW1, n, H, D, params + o.b1, (float *)(ws + w.Z1), (uint16_t *)(ws + w.H1)), st);
    launch_gemm(fwd_gemm((uint16_t *)(ws + w.H1), H, wb + o.bW2, n, H, H, params + o.b2, (float *)(ws + w.Z2),
                         (uint16_t *)(ws + w.H2)), st);
    launch_gemm(fwd_gemm((uint16_t *)(ws + w.H2), H, wb + o.bW3, n, H, H, params + o.b3, (float *)(ws + w.Z3),
                         (uint16_t *)(ws + w.H3)), st);
    k_head_fwd<<<(n + 3) / 4, 256, 0, st>>>((uint16_t *)(ws + w.H3), params + o.w4, params + o.b4, n, H,
                                            (float *)(ws + w.y));
}

// Backward pass (after forward) into the gradient buffer of the workspace.
void backward(int D, int H, const float *params, const uint16_t *wb, const float *fit, const int *idx, float mu,
              float sigma, int n, unsigned char *ws, hipStream_t st) {
    const MlpOff o = mlp_offsets(D, H);
    const MlpWs w = mlp_ws(D, H, n);
    float *gr = (float *)(ws + w.grads);
    k_loss<<<1, 256, 0, st>>>((float *)(ws + w.y), fit, idx, mu, sigma, n, (float *)(ws + w.dy), (float *)(ws + w.loss));
    const int eblocks = (int)std::min<int64_t>(1024, ((int64_t)n * H + 255) / 256);
    k_head_dz<<<eblocks, 256, 0, st>>>((float *)(ws + w.dy), (float *)(ws + w.Z3), params + o.w4, n, H,
                                       (float *)(ws + w.dZ3), (uint16_t *)(ws + w.dZ3b));
    k_colsum<uint16_t><<<(H + 63) / 64, 1024, 0, st>>>((uint16_t *)(ws + w.H3), (float *)(ws + w.dy), n, H, gr + o.w4);
    k_colsum<float><<<1, 1024, 0, st>>>((float *)(ws + w.dy), nullptr, n, 1, gr + o.b4);
    const uint16_t *Hin[3] = {(uint16_t *)(ws + w.Xb), (uint16_t *)(ws + w.H1), (uint16_t *)(ws + w.H2)};
    const int Kin[3] = {D, H, H};
    const size_t gW[3] = {o.W1, o.W2, o.W3}, gB[3] = {o.b1, o.b2, o.b3}, bW[3] = {o.bW1, o.bW2, o.bW3};
    float *dZf[3] = {(float *)(ws + w.dZ1), (float *)(ws + w.dZ2), (float *)(ws + w.dZ3)};
    uint16_t *dZb[3] = {(uint16_t *)(ws + w.dZ1b), (uint16_t *)(ws + w.dZ2b), (uint16_t *)(ws + w.dZ3b)};
    const float *Zf[3] = {(float *)(ws + w.Z1), (float *)(ws + w.Z2), (float *)(ws + w.Z3)};
    for (int l = 2; l >= 0; --l) {
        // dW_l[j][k] = sum_m dZ_l[m][j] Hin_l[m][k]
        Gemm g = {};
        g.A = dZb[l]; g.B = Hin[l]; g.M = H; g.N = Kin[l]; g.K = n;
        g.sam = 1; g.sak = H; g.sbk = Kin[l]; g.sbn = 1;
        g.epi = EPI_STORE; g.outf = gr + gW[l];
        launch_gemm(g, st);
        k_colsum<float><<<(H + 63) / 64, 1024, 0, st>>>(dZf[l], nullptr, n, H, gr + gB[l]);
        if (l > 0) {
            // dZ_{l-1}[m][k] = (sum_j dZ_l[m][j] W_l[j][k]) GELU'(Z_{l-1}[m][k])
            Gemm b = {};
            b.A = dZb[l]; b.B = wb + bW[l]; b.M = n; b.N = H; b.K = H;
            b.sam = H; b.sak = 1; b.sbk = H; b.sbn = 1;
            b.epi = EPI_GELU_GRAD; b.Zin = Zf[l - 1]; b.outf = dZf[l - 1]; b.outb = dZb[l - 1];
            launch_gemm(b, st);
        }
    }
}

}  // namespace

extern "C" size_t empso_mlp_param_count(int32_t D, int32_t H) {
    if (D < 1 || H < 1) return 0;
    return mlp_offsets(D, H).P;
}

extern "C" size_t empso_mlp_bf16_count(int32_t D, int32_t H) {
    if (D < 1 || H < 1) return 0;
    return mlp_offsets(D, H).PB;
}

extern "C" size_t empso_mlp_workspace_bytes(int32_t D, int32_t H, int32_t n) {
    if (!check_shape(D, H, n)) return 0;
    return mlp_ws(D, H, n).total;
}

extern "C" int empso_mlp_sync_bf16(int32_t D, int32_t H, const float *params_d, uint16_t *wbf16_d,
                                   empso_stream stream) {
    empso::clear_error();
    if (!params_d || !wbf16_d) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (!check_shape(D, H, 1)) EMPSO_FAIL(EMPSO_EINVAL, "bad shape");
    const MlpOff o = mlp_offsets(D, H);
    hipStream_t st = (hipStream_t)stream;
    k_to_bf16<<<256, 256, 0, st>>>(params_d + o.W1, wbf16_d + o.bW1, (int64_t)H * D);
    k_to_bf16<<<256, 256, 0, st>>>(params_d + o.W2, wbf16_d + o.bW2, (int64_t)H * H);
    k_to_bf16<<<256, 256, 0, st>>>(params_d + o.W3, wbf16_d + o.bW3, (int64_t)H * H);
    EMPSO_HIP(hipGetLastError());
    return EMPSO_OK;
}

extern "C" int empso_mlp_predict(int32_t D, int32_t H, const float *params_d, const uint16_t *wbf16_d,
                                 const float *lo_d, const float *hi_d, const float *X_d, int32_t n, float *y_d,
                                 void *ws, size_t ws_bytes, empso_stream stream) {
    empso::clear_error();
    if (!params_d || !wbf16_d || !lo_d || !hi_d || !X_d || !y_d || !ws) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (!check_shape(D, H, n)) EMPSO_FAIL(EMPSO_EINVAL, "bad shape (D, H, n) = (%d, %d, %d)", D, H, n);
    if (ws_bytes < mlp_ws(D, H, n).total) EMPSO_FAIL(EMPSO_EWORKSPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    unsigned char *w = (unsigned char *)ws;
    forward(D, H, params_d, wbf16_d, lo_d, hi_d, X_d, nullptr, n, w, st);
    EMPSO_HIP(hipMemcpyAsync(y_d, w + mlp_ws(D, H, n).y, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    EMPSO_HIP(hipGetLastError());
    return EMPSO_OK;
}

extern "C" int empso_mlp_grad(int32_t D, int32_t H, const float *params_d, const uint16_t *wbf16_d, const float *lo_d,
                              const float *hi_d, const float *X_d, const float *fit_d, const int32_t *idx_d, int32_t n,
                              float mu, float sigma, float *grads_d, float *loss_d, void *ws, size_t ws_bytes,
                              empso_stream stream) {
    empso::clear_error();
    if (!params_d || !wbf16_d || !lo_d || !hi_d || !X_d || !fit_d || !ws) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (!check_shape(D, H, n)) EMPSO_FAIL(EMPSO_EINVAL, "bad shape (D, H, n) = (%d, %d, %d)", D, H, n);
    if (!(sigma > 0) || !std::isfinite(mu)) EMPSO_FAIL(EMPSO_EINVAL, "need sigma > 0 and finite mu");
    const MlpWs w = mlp_ws(D, H, n);
    if (ws_bytes < w.total) EMPSO_FAIL(EMPSO_EWORKSPACE, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    unsigned char *wsb = (unsigned char *)ws;
    forward(D, H, params_d, wbf16_d, lo_d, hi_d, X_d, idx_d, n, wsb, st);
    backward(D, H, params_d, wbf16_d, fit_d, idx_d, mu, sigma, n, wsb, st);
    const MlpOff o = mlp_offsets(D, H);
    if (grads_d)
        EMPSO_HIP(hipMemcpyAsync(grads_d, wsb + w.grads, sizeof(float) * o.P, hipMemcpyDeviceToDevice, st));
    if (loss_d) EMPSO_HIP(hipMemcpyAsync(loss_d, wsb + w.loss, sizeof(float), hipMemcpyDeviceToDevice, st));
    EMPSO_HIP(hipGetLastError());
    return EMPSO_OK;
}

extern "C" int empso_mlp_train_step(int32_t D, int32_t H, float *params_d, uint16_t *wbf16_d, float *adam_m_d,
                                    float *adam_v_d, int32_t step, float lr, const float *lo_d, const float *hi_d,
                                    const float *X_d, const float *fit_d, const int32_t *idx_d, int32_t n, float mu,
                                    float sigma, float *loss_d, void *ws, size_t ws_bytes, empso_stream stream) {
    empso::clear_error();
    if (!adam_m_d || !adam_v_d) EMPSO_FAIL(EMPSO_EINVAL, "NULL argument");
    if (step < 1 || !(lr > 0)) EMPSO_FAIL(EMPSO_EINVAL, "need step >= 1 and lr > 0");
    int rc = empso_mlp_grad(D, H, params_d, wbf16_d, lo_d, hi_d, X_d, fit_d, idx_d, n, mu, sigma, nullptr, loss_d, ws,
                            ws_bytes, stream);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const MlpOff o = mlp_offsets(D, H);
    const MlpWs w = mlp_ws(D, H, n);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = (float)(1.0 - std::pow(0.9, step)), c2 = (float)(1.0 - std::pow(0.999, step));
    BfMap map;
    const int64_t src[3] = {(int64_t)o.W1, (int64_t)o.W2, (int64_t)o.W3};
    const int64_t len[3] = {(int64_t)H * D, (int64_t)H * H, (int64_t)H * H};
    const int64_t dst[3] = {(int64_t)o.bW1, (int64_t)o.bW2, (int64_t)o.bW3};
    for (int i = 0; i < 3; ++i) {
        map.src[i] = src[i];
        map.len[i] = len[i];
        map.dst[i] = dst[i];
    }
    k_adam<<<256, 256, 0, st>>>(params_d, (const float *)((unsigned char *)ws + w.grads), adam_m_d, adam_v_d,
                                (int64_t)o.P, lr, b1, b2, eps, c1, c2, wbf16_d, map);
    EMPSO_HIP(hipGetLastError());
    return EMPSO_OK;
}
