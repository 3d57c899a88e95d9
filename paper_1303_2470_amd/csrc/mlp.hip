// Surrogate network for D(t)/D_b: 6 -> 256 -> 256 -> 256 -> 1, SiLU, trained
// and evaluated on the GPU with BF16 MFMA (32x32x16, FP32 accumulation),
// FP32 master weights and Adam.
//
// All layer widths are padded to multiples of 32 (input 6 -> 32, output
// 1 -> 32) with zero weights, so one MFMA GEMM serves every layer:
//   forward   Z_l = A_{l-1} W_l^T + b_l,  A_l = silu(Z_l)      (M = batch, N = out, K = in)
//   backward  dA_{l-1} = dZ_l W_l,  dZ_{l-1} = dA_{l-1} * silu'(Z_{l-1})   (N = in, K = out)
//             dW_l = dZ_l^T A_{l-1}                            (M = out, N = in, K = batch)
// Large GEMMs (M, N multiples of 128, K of 32) run k_gemm_lds: a block of 4
// waves owns a 128 x 128 output tile, stages 32-wide K slices of both operands
// through LDS (transposing operands stored K-major on the way) and each wave
// accumulates a 64 x 64 sub-tile as 2 x 2 MFMA tiles, so every operand read
// from LDS feeds two MFMAs. The small ones (the padded 32-wide input and
// output layers) run k_gemm: a wave computes one 32x32 output tile with
// operands read straight from global memory.
#include <cmath>
#include <vector>

#include "lbmp_internal.hpp"

namespace lbmp {
namespace mlp {

using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));
using f32x16 = float __attribute__((ext_vector_type(16)));

constexpr int NLAYER = 4;
constexpr int WIDTH = 256;
constexpr int PAD_IN = 32;   // 6 features padded
constexpr int PAD_OUT = 32;  // 1 output padded
constexpr int NFEAT = 6;

__host__ __device__ constexpr int lin(int l) { return l == 0 ? PAD_IN : WIDTH; }
__host__ __device__ constexpr int lout(int l) { return l == NLAYER - 1 ? PAD_OUT : WIDTH; }
__host__ __device__ constexpr int tin(int l) { return l == 0 ? NFEAT : WIDTH; }   // true fan-in
__host__ __device__ constexpr int tout(int l) { return l == NLAYER - 1 ? 1 : WIDTH; }

enum Epi { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_DACT = 2, EPI_GRAD = 3 };

// The logistic function through the hardware reciprocal (v_rcp_f32, 1 ulp):
// an IEEE division would cost ten instructions per value, and the epilogues
// are rounded to bf16 anyway.
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}

// Epilogue of one 32x32 MFMA tile at (m0, n0) of C (see k_gemm).
template <int epi>
__device__ __forceinline__ void epilogue(const f32x16& acc, int m0, int n0, int lane, int N,
                                         const float* __restrict__ bias, const float* __restrict__ aux,
                                         float* __restrict__ out0, __bf16* __restrict__ out1) {
    // accumulator layout: element v of lane l is C[row][col] with col = l % 32,
    // row = 8*(v/4) + 4*(l/32) + v%4
    const int col = n0 + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = m0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const size_t o = (size_t)row * N + col;
        float c = acc[v];
        if (epi == EPI_HIDDEN) {
            c += bias[col];
            out0[o] = c;
            out1[o] = (__bf16)silu(c);
        } else if (epi == EPI_OUT) {
            out0[o] = c + bias[col];
        } else if (epi == EPI_DACT) {
            out1[o] = (__bf16)(c * silu_grad(aux[o]));
        } else {
            out0[o] = c;
        }
    }
}

// C[M][N] = sum_k A(m, k) B(k, n), bf16 operands, fp32 accumulation.
// A(m, k) = A[m*lda + k] if a_km else A[k*lda + m]; B(k, n) = B[n*ldb + k] if
// b_nk else B[k*ldb + n]. M, N multiples of 32; K a multiple of 16.
// Epilogues (ldc = N):
//  EPI_HIDDEN: Z = C + bias[n] (fp32 out0), act = silu(Z) (bf16 out1)
//  EPI_OUT:    Y = C + bias[n] (fp32 out0)
//  EPI_DACT:   dZ = C * silu'(Zprev[m][n]) (bf16 out1), Zprev = aux
//  EPI_GRAD:   G = C (fp32 out0)
template <bool a_km, bool b_nk, int epi>
__global__ void __launch_bounds__(256) k_gemm(const __bf16* __restrict__ A, int lda,
                                              const __bf16* __restrict__ B, int ldb, int M, int N, int K,
                                              const float* __restrict__ bias, const float* __restrict__ aux,
                                              float* __restrict__ out0, __bf16* __restrict__ out1) {
    const int wave = (blockIdx.x * (blockDim.x / 64)) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    const int tiles_n = N / 32;
    if (wave >= (M / 32) * tiles_n) return;
    const int m0 = (wave / tiles_n) * 32, n0 = (wave % tiles_n) * 32;
    const int r = lane & 31, kh = (lane >> 5) * 8;
    f32x16 acc = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x8 a, b;
        if (a_km) {
            a = *reinterpret_cast<const bf16x8*>(A + (size_t)(m0 + r) * lda + k0 + kh);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = A[(size_t)(k0 + kh + i) * lda + m0 + r];
        }
        if (b_nk) {
            b = *reinterpret_cast<const bf16x8*>(B + (size_t)(n0 + r) * ldb + k0 + kh);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) b[i] = B[(size_t)(k0 + kh + i) * ldb + n0 + r];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    epilogue<epi>(acc, m0, n0, lane, N, bias, aux, out0, out1);
}

constexpr int TBM = 128, TBN = 128, TBK = 32, TPITCH = TBK + 8;  // LDS rows padded against bank conflicts

// Same operation and epilogues as k_gemm, for M, N multiples of 128 and K of
// 32; one block (256 threads) per 128 x 128 output tile.
template <bool a_km, bool b_nk, int epi>
__global__ void __launch_bounds__(256) k_gemm_lds(const __bf16* __restrict__ A, int lda,
                                                  const __bf16* __restrict__ B, int ldb, int M, int N, int K,
                                                  const float* __restrict__ bias, const float* __restrict__ aux,
                                                  float* __restrict__ out0, __bf16* __restrict__ out1) {
    __shared__ __align__(16) __bf16 As[TBM * TPITCH];  // [m][k]
    __shared__ __align__(16) __bf16 Bs[TBN * TPITCH];  // [n][k]
    const int tiles_n = N / TBN;
    const int m0 = (blockIdx.x / tiles_n) * TBM, n0 = (blockIdx.x % tiles_n) * TBN;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int r = lane & 31, kh = (lane >> 5) * 8;
    f32x16 acc[2][2] = {};
    // one 8-element chunk of a K-contiguous operand (rows x 32) or of a
    // K-major one (32 x cols) per thread and i
    auto stage = [&](const __bf16* X, int ldx, int x0, int k0, bool x_k_contiguous, __bf16* S) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int c = t + 256 * i;
            if (x_k_contiguous) {
                const int row = c >> 2, kc = (c & 3) * 8;
                const bf16x8 v = *reinterpret_cast<const bf16x8*>(X + (size_t)(x0 + row) * ldx + k0 + kc);
                *reinterpret_cast<bf16x8*>(S + row * TPITCH + kc) = v;
            } else {
                const int kk = c >> 4, xc = (c & 15) * 8;
                const bf16x8 v = *reinterpret_cast<const bf16x8*>(X + (size_t)(k0 + kk) * ldx + x0 + xc);
#pragma unroll
                for (int j = 0; j < 8; ++j) S[(xc + j) * TPITCH + kk] = v[j];
            }
        }
    };
    for (int k0 = 0; k0 < K; k0 += TBK) {
        stage(A, lda, m0, k0, a_km, As);
        stage(B, ldb, n0, k0, b_nk, Bs);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TBK; kk += 16) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *reinterpret_cast<const bf16x8*>(As + (wm + 32 * i + r) * TPITCH + kk + kh);
                b[i] = *reinterpret_cast<const bf16x8*>(Bs + (wn + 32 * i + r) * TPITCH + kk + kh);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            epilogue<epi>(acc[i][j], m0 + wm + 32 * i, n0 + wn + 32 * j, lane, N, bias, aux, out0, out1);
}

// Fused inference: one block (8 waves) per FS samples runs all four layers
// with the activations in LDS (one buffer: a layer's products read it, and
// after a barrier its epilogue overwrites it) and the weights read as MFMA
// operands straight from global memory, where all blocks share them in L2;
// each weight fragment a wave loads serves the block's 128 samples. The
// arithmetic is that of the layer GEMMs (bf16 operands, fp32 accumulation in
// increasing K, bias and SiLU in fp32, activations rounded to bf16), so
// predictions equal the unfused path's.
constexpr int FS = 128;              // samples per block
constexpr int FWAVES = 8;            // waves per block
constexpr int APITCH = WIDTH + 8;    // bf16 per activation row (padded against bank conflicts)

__global__ void __launch_bounds__(64 * FWAVES) __attribute__((amdgpu_waves_per_eu(4)))
k_mlp_forward(const float* __restrict__ x, int64_t n, const float* __restrict__ norm,
              const __bf16* __restrict__ W0, const float* __restrict__ b0, const __bf16* __restrict__ W1,
              const float* __restrict__ b1, const __bf16* __restrict__ W2, const float* __restrict__ b2,
              const __bf16* __restrict__ W3, const float* __restrict__ b3, float* __restrict__ y) {
    __shared__ __align__(16) __bf16 act[FS * APITCH];
    const int64_t s0 = (int64_t)blockIdx.x * FS;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int r = lane & 31, kh = (lane >> 5) * 8;
    // normalised features, zero padded to PAD_IN columns
    for (int i = t; i < FS * PAD_IN; i += 64 * FWAVES) {
        const int row = i / PAD_IN, c = i % PAD_IN;
        const int64_t si = s0 + row;
        float v = 0.0f;
        if (c < NFEAT && si < n) v = (x[si * NFEAT + c] - norm[c]) / norm[6 + c];
        act[row * APITCH + c] = (__bf16)v;
    }
    __syncthreads();
    // hidden layer: wave w computes output features 32 w .. 32 w + 31 of all
    // FS samples as the transposed product (weights as the MFMA's first
    // operand), so each lane holds runs of 4 consecutive features of one
    // sample and writes them to LDS as one 8-byte store
    constexpr int ST = FS / 32;  // sample tiles
    auto hidden = [&](const __bf16* __restrict__ W, const float* __restrict__ bias, int K) {
        const int n0 = 32 * wave;
        f32x16 acc[ST] = {};
#pragma unroll 2
        for (int k0 = 0; k0 < K; k0 += 16) {
            const bf16x8 w = *reinterpret_cast<const bf16x8*>(W + (size_t)(n0 + r) * K + k0 + kh);
            bf16x8 a[ST];
#pragma unroll
            for (int j = 0; j < ST; ++j) a[j] = *reinterpret_cast<const bf16x8*>(act + (32 * j + r) * APITCH + k0 + kh);
#pragma unroll
            for (int j = 0; j < ST; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, a[j], acc[j], 0, 0, 0);
        }
        __syncthreads();  // every wave has read the layer's input
        using bf16x4 = __bf16 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int nf = n0 + 8 * g + 4 * (lane >> 5);  // features nf .. nf + 3
            const float4 bc = *reinterpret_cast<const float4*>(bias + nf);
#pragma unroll
            for (int j = 0; j < ST; ++j) {
                bf16x4 o;
                o[0] = (__bf16)silu(acc[j][4 * g + 0] + bc.x);
                o[1] = (__bf16)silu(acc[j][4 * g + 1] + bc.y);
                o[2] = (__bf16)silu(acc[j][4 * g + 2] + bc.z);
                o[3] = (__bf16)silu(acc[j][4 * g + 3] + bc.w);
                *reinterpret_cast<bf16x4*>(act + (32 * j + r) * APITCH + nf) = o;
            }
        }
    };
    hidden(W0, b0, PAD_IN);
    __syncthreads();
    hidden(W1, b1, WIDTH);
    __syncthreads();
    hidden(W2, b2, WIDTH);
    __syncthreads();
    // output layer (PAD_OUT features, feature 0 is the network's output), also
    // transposed: waves 0 .. ST - 1 take samples 32 w .. 32 w + 31; feature 0
    // of sample 32 w + r sits in element 0 of lane r
    if (wave < ST) {
        f32x16 acc = {};
#pragma unroll 4
        for (int k0 = 0; k0 < WIDTH; k0 += 16) {
            const bf16x8 w = *reinterpret_cast<const bf16x8*>(W3 + (size_t)r * WIDTH + k0 + kh);
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(act + (32 * wave + r) * APITCH + k0 + kh);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, a, acc, 0, 0, 0);
        }
        const int64_t si = s0 + 32 * wave + r;
        if (lane < 32 && si < n) y[si] = norm[12] + norm[13] * (acc[0] + b3[0]);
    }
}

// Input features (fp32 [B][6]) -> bf16 [B][32], zero padded.
__global__ void k_pack_input(const float* __restrict__ x, int B, __bf16* __restrict__ xb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * PAD_IN) return;
    const int b = i / PAD_IN, c = i % PAD_IN;
    xb[i] = c < NFEAT ? (__bf16)x[b * NFEAT + c] : (__bf16)0.0f;
}

// Output gradient of the loss mean((y - t)^2): dY = 2 (y - t) / B in column 0;
// also per-row squared errors for the loss.
__global__ void k_loss_grad(const float* __restrict__ Y, const float* __restrict__ t, int B,
                            __bf16* __restrict__ dY, float* __restrict__ sq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * PAD_OUT) return;
    const int b = i / PAD_OUT, c = i % PAD_OUT;
    if (c == 0) {
        const float r = Y[b * PAD_OUT] - t[b];
        dY[i] = (__bf16)(2.0f * r / (float)B);
        sq[b] = r * r;
    } else {
        dY[i] = (__bf16)0.0f;
    }
}

// db[n] = sum_b dZ[b][n] in a fixed order: a block of 1024 threads takes 32
// columns; thread (g, c) sums rows g, g + 32, ... of its column, then the 32
// partials of a column are added in order of g.
__global__ void __launch_bounds__(1024) k_bias_grad(const __bf16* __restrict__ dZ, int B, int N,
                                                   float* __restrict__ db) {
    __shared__ float part[32][33];
    const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int n = blockIdx.x * 32 + c;
    float s = 0.0f;
    if (n < N)
        for (int b = g; b < B; b += 32) s += (float)dZ[(size_t)b * N + n];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && n < N) {
        float a = 0.0f;
        for (int i = 0; i < 32; ++i) a += part[i][c];
        db[n] = a;
    }
}

// Parameter gradients split over the batch (the reduction dimension K = B):
// wave w takes the 32x32 tile w % tiles of dW = dZ^T A over the rows
// [split kc, (split + 1) kc), split = w / tiles, and writes its partial to
// P[split]; block (column group, split) sums the same rows of dZ for the bias
// gradient into Pb[split]. k_sum_splits adds the partials in split order
// (deterministic). Spreading K over the waves keeps the whole GPU busy where
// the 256 x 256 weight gradient has only 64 output tiles.
constexpr int GSPLIT_MAX = 32;

__global__ void __launch_bounds__(256) k_grad_w_split(const __bf16* __restrict__ dZ, int O,
                                                      const __bf16* __restrict__ Ap, int I, int kc, int splits,
                                                      float* __restrict__ P) {
    const int wave = (blockIdx.x * (blockDim.x / 64)) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    const int tiles_n = I / 32, tiles = (O / 32) * tiles_n;
    const int split = wave / tiles, t = wave % tiles;
    if (split >= splits) return;
    const int m0 = (t / tiles_n) * 32, n0 = (t % tiles_n) * 32;
    const int r = lane & 31, kh = (lane >> 5) * 8;
    f32x16 acc = {};
    for (int k0 = split * kc; k0 < (split + 1) * kc; k0 += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = dZ[(size_t)(k0 + kh + i) * O + m0 + r];
#pragma unroll
        for (int i = 0; i < 8; ++i) b[i] = Ap[(size_t)(k0 + kh + i) * I + n0 + r];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    epilogue<EPI_GRAD>(acc, m0, n0, lane, I, nullptr, nullptr, P + (size_t)split * O * I, nullptr);
}

__global__ void __launch_bounds__(256) k_grad_b_split(const __bf16* __restrict__ dZ, int O, int kc,
                                                      float* __restrict__ Pb) {
    __shared__ float part[8][33];
    const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int n = blockIdx.x * 32 + c, split = blockIdx.y;
    float s = 0.0f;
    for (int b = split * kc + g; b < (split + 1) * kc; b += 8) s += (float)dZ[(size_t)b * O + n];
    part[g][c] = s;
    __syncthreads();
    if (g == 0) {
        float a = 0.0f;
        for (int i = 0; i < 8; ++i) a += part[i][c];
        Pb[(size_t)split * O + n] = a;
    }
}

__global__ void k_sum_splits(const float* __restrict__ P, int n, int splits, float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float a = 0.0f;
    for (int sp = 0; sp < splits; ++sp) a += P[(size_t)sp * n + i];
    out[i] = a;
}

// Adam on the fp32 master copy (only the unpadded parameters move), then
// bf16 copies W [out][in] and W^T [in][out].
// hyper = {lr, c1, c2}: the step's learning rate and bias corrections, read
// from device memory so that a captured training step can be replayed.
__global__ void k_adam(float* __restrict__ W, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int rows, int cols, int trows, int tcols,
                       const float* __restrict__ hyper, float b1, float b2, float eps,
                       __bf16* __restrict__ Wb, __bf16* __restrict__ WTb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    const float lr = hyper[0], c1 = hyper[1], c2 = hyper[2];
    const int r = i / cols, c = i % cols;
    float w = W[i];
    if (r < trows && c < tcols) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        W[i] = w;
    }
    if (Wb) Wb[i] = (__bf16)w;
    if (WTb) WTb[(size_t)c * rows + r] = (__bf16)w;
}

__global__ void k_set_hyper(float* __restrict__ hyper, float lr, float c1, float c2) {
    hyper[0] = lr;
    hyper[1] = c1;
    hyper[2] = c2;
}

__global__ void k_copy_out(const float* __restrict__ Y, int B, float* __restrict__ y) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) y[b] = Y[(size_t)b * PAD_OUT];
}

}  // namespace mlp
}  // namespace lbmp

// ------------------------------------------------------------------ host side
namespace lbmp {
namespace mlp {

constexpr uint32_t SG_MAGIC = 0x4c425347u;  // "LBSG"

struct Layer {
    float *W, *b, *mW, *vW, *mb, *vb, *gW, *gb;  // fp32 master, Adam moments, gradients
    __bf16 *Wb, *WTb;                            // bf16 W [out][in] and W^T [in][out]
};

}  // namespace mlp
}  // namespace lbmp

struct lbmp_sg {
    uint32_t magic;
    int bmax;
    int64_t step;
    hipStream_t stream;
    lbmp::mlp::Layer L[lbmp::mlp::NLAYER];
    float* norm;         // [6] mean, [6] std, y_mean, y_std
    __bf16* xb;          // [bmax][32]
    float* Z[lbmp::mlp::NLAYER];      // pre-activations [bmax][out]
    __bf16* Ab[lbmp::mlp::NLAYER];    // activations (bf16) [bmax][out]
    __bf16* dZb[lbmp::mlp::NLAYER];   // gradients w.r.t. pre-activations [bmax][out]
    float* xg;           // gathered batch inputs [bmax][6]
    float* yg;           // gathered targets [bmax]
    float* sq;           // per-row squared errors [bmax]
    float* loss;         // [1]
    float* hyper;        // [4] learning rate and Adam bias corrections of the current step
    float* gsplit;       // [GSPLIT_MAX][WIDTH][WIDTH] weight-gradient partials over batch splits
    float* bsplit;       // [GSPLIT_MAX][WIDTH] bias-gradient partials
    // forward + backward + Adam of one batch size captured as a graph and
    // replayed (off with LBMP_SG_GRAPH=0, or on the null stream)
    bool use_graph;
    int graph_B;
    hipGraph_t graph;
    hipGraphExec_t gexec;
};

namespace lbmp {
namespace mlp {

template <typename T>
static void carve_n(Carver& c, T*& p, size_t n) { p = c.take<T>(n); }

static void carve_sg(lbmp_sg* h, Carver& c) {
    for (int l = 0; l < NLAYER; ++l) {
        const size_t nw = (size_t)lout(l) * lin(l), nb = lout(l);
        Layer& L = h->L[l];
        carve_n(c, L.W, nw); carve_n(c, L.mW, nw); carve_n(c, L.vW, nw); carve_n(c, L.gW, nw);
        carve_n(c, L.b, nb); carve_n(c, L.mb, nb); carve_n(c, L.vb, nb); carve_n(c, L.gb, nb);
        carve_n(c, L.Wb, nw); carve_n(c, L.WTb, nw);
    }
    carve_n(c, h->norm, 16);
    const size_t B = (size_t)h->bmax;
    carve_n(c, h->xb, B * PAD_IN);
    for (int l = 0; l < NLAYER; ++l) {
        carve_n(c, h->Z[l], B * lout(l));
        carve_n(c, h->Ab[l], B * lout(l));
        carve_n(c, h->dZb[l], B * lout(l));
    }
    carve_n(c, h->xg, B * NFEAT);
    carve_n(c, h->yg, B);
    carve_n(c, h->sq, B);
    carve_n(c, h->loss, 4);
    carve_n(c, h->hyper, 4);
    carve_n(c, h->gsplit, (size_t)GSPLIT_MAX * WIDTH * WIDTH);
    carve_n(c, h->bsplit, (size_t)GSPLIT_MAX * WIDTH);
}

// Inputs normalised and gathered: x[idx[b]] -> (x - mean)/std, t = (y - y_mean)/y_std.
__global__ void k_gather(const float* __restrict__ x, const float* __restrict__ y,
                         const int32_t* __restrict__ idx, int B, const float* __restrict__ norm,
                         float* __restrict__ xg, float* __restrict__ yg) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int64_t s = idx ? idx[b] : b;
    for (int c = 0; c < NFEAT; ++c) xg[b * NFEAT + c] = (x[s * NFEAT + c] - norm[c]) / norm[6 + c];
    if (y) yg[b] = (y[s] - norm[12]) / norm[13];
}

// y = y_mean + y_std * network output
__global__ void k_denorm(const float* __restrict__ Y, int B, const float* __restrict__ norm,
                         float* __restrict__ y) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) y[b] = norm[12] + norm[13] * Y[(size_t)b * PAD_OUT];
}

__global__ void k_sum(const float* __restrict__ v, int n, float* __restrict__ out) {
    __shared__ float s[256];
    float a = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) a += v[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0] / (float)n;
}

static unsigned gemm_blocks(int M, int N) { return (unsigned)(((M / 32) * (N / 32) + 3) / 4); }

// The LDS-tiled kernel where the shape allows it and gives at least 128
// blocks (large batches), the per-wave one otherwise (at batch 1024 the
// per-wave kernel's 64 blocks beat the tiled kernel's 16).
template <bool a_km, bool b_nk, int epi>
static void gemm(const __bf16* A, int lda, const __bf16* B, int ldb, int M, int N, int K, const float* bias,
                 const float* aux, float* out0, __bf16* out1, hipStream_t s) {
    if (M % TBM == 0 && N % TBN == 0 && K % TBK == 0 && (M / TBM) * (N / TBN) >= 128)
        k_gemm_lds<a_km, b_nk, epi><<<(unsigned)((M / TBM) * (N / TBN)), 256, 0, s>>>(A, lda, B, ldb, M, N, K, bias,
                                                                                     aux, out0, out1);
    else
        k_gemm<a_km, b_nk, epi><<<gemm_blocks(M, N), 256, 0, s>>>(A, lda, B, ldb, M, N, K, bias, aux, out0, out1);
}

// Forward pass over a batch of B (multiple of 32) packed inputs in h->xb.
static void forward(lbmp_sg* h, int B, hipStream_t s) {
    const __bf16* A = h->xb;
    for (int l = 0; l < NLAYER; ++l) {
        const int N = lout(l), K = lin(l);
        if (l < NLAYER - 1)
            gemm<true, true, EPI_HIDDEN>(A, K, h->L[l].Wb, K, B, N, K, h->L[l].b, nullptr, h->Z[l], h->Ab[l], s);
        else
            gemm<true, true, EPI_OUT>(A, K, h->L[l].Wb, K, B, N, K, h->L[l].b, nullptr, h->Z[l], nullptr, s);
        A = h->Ab[l];
    }
}

// Backward pass: parameter gradients into L[l].gW, L[l].gb.
static void backward(lbmp_sg* h, int B, hipStream_t s) {
    k_loss_grad<<<(B * PAD_OUT + 255) / 256, 256, 0, s>>>(h->Z[NLAYER - 1], h->yg, B, h->dZb[NLAYER - 1], h->sq);
    for (int l = NLAYER - 1; l >= 0; --l) {
        const int O = lout(l), I = lin(l);
        const __bf16* Aprev = l == 0 ? h->xb : h->Ab[l - 1];
        // dW[o][i] = sum_b dZ[b][o] A[b][i], db[o] = sum_b dZ[b][o]: over
        // batch splits of 256 rows (B a multiple of 32: fewer, longer splits
        // when B / 256 is small), partials added in split order
        int splits = 1;
        while (splits * 2 <= GSPLIT_MAX && B % (splits * 2 * 16) == 0 && B / (splits * 2) >= 256) splits *= 2;
        const int kc = B / splits;
        const int waves = (O / 32) * (I / 32) * splits;
        k_grad_w_split<<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(h->dZb[l], O, Aprev, I, kc, splits, h->gsplit);
        k_sum_splits<<<(unsigned)((O * I + 255) / 256), 256, 0, s>>>(h->gsplit, O * I, splits, h->L[l].gW);
        k_grad_b_split<<<dim3((unsigned)(O / 32), (unsigned)splits), 256, 0, s>>>(h->dZb[l], O, kc, h->bsplit);
        k_sum_splits<<<(unsigned)((O + 255) / 256), 256, 0, s>>>(h->bsplit, O, splits, h->L[l].gb);
        if (l > 0) {
            // dA[b][i] = sum_o dZ[b][o] W[o][i]; W^T stored [i][o]
            gemm<true, true, EPI_DACT>(h->dZb[l], O, h->L[l].WTb, O, B, I, O, nullptr, h->Z[l - 1], nullptr,
                                       h->dZb[l - 1], s);
        }
    }
}

constexpr float ADAM_B1 = 0.9f, ADAM_B2 = 0.999f, ADAM_EPS = 1e-8f;

// The Adam update of every layer with the hyper-parameters in h->hyper.
static void adam(lbmp_sg* h, hipStream_t s) {
    for (int l = 0; l < NLAYER; ++l) {
        Layer& L = h->L[l];
        const int O = lout(l), I = lin(l);
        k_adam<<<(O * I + 255) / 256, 256, 0, s>>>(L.W, L.mW, L.vW, L.gW, O, I, tout(l), tin(l), h->hyper,
                                                  ADAM_B1, ADAM_B2, ADAM_EPS, L.Wb, L.WTb);
        k_adam<<<(O + 255) / 256, 256, 0, s>>>(L.b, L.mb, L.vb, L.gb, O, 1, tout(l), 1, h->hyper, ADAM_B1,
                                              ADAM_B2, ADAM_EPS, nullptr, nullptr);
    }
}

// Step counter and the learning rate and bias corrections of this step.
static void set_hyper(lbmp_sg* h, float lr, hipStream_t s) {
    h->step += 1;
    const float c1 = 1.0f - powf(ADAM_B1, (float)h->step), c2 = 1.0f - powf(ADAM_B2, (float)h->step);
    k_set_hyper<<<1, 1, 0, s>>>(h->hyper, lr, c1, c2);
}

static lbmp_status check(const lbmp_sg* h) {
    if (!h || h->magic != SG_MAGIC) return fail(LBMP_ESTATE, "invalid surrogate handle");
    return LBMP_OK;
}

// splitmix64: the published 64-bit mixing generator (Steele, Lea, Flood 2014)
static uint64_t splitmix(uint64_t& x) {
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace mlp
}  // namespace lbmp

using namespace lbmp;
using namespace lbmp::mlp;

extern "C" lbmp_status sg_param_count(int64_t* n) {
    if (!n) return fail(LBMP_EINVAL, "n is NULL");
    int64_t c = 0;
    for (int l = 0; l < NLAYER; ++l) c += (int64_t)tout(l) * tin(l) + tout(l);
    *n = c;
    return LBMP_OK;
}

extern "C" lbmp_status sg_workspace_bytes(int batch_max, size_t* bytes) {
    if (batch_max < 32 || batch_max % 32 != 0) return fail(LBMP_EINVAL, "batch_max must be a positive multiple of 32");
    if (!bytes) return fail(LBMP_EINVAL, "bytes is NULL");
    lbmp_sg tmp{};
    tmp.bmax = batch_max;
    Carver c(nullptr, ~size_t(0));
    carve_sg(&tmp, c);
    *bytes = c.off;
    return LBMP_OK;
}

extern "C" lbmp_status sg_set_params(lbmp_sg* h, const float* p);

extern "C" lbmp_status sg_create(int batch_max, uint64_t seed, void* dev_ws, size_t ws_bytes, void* hip_stream,
                                 lbmp_sg** out) {
    if (!out) return fail(LBMP_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    lbmp_status st = sg_workspace_bytes(batch_max, &need);
    if (st != LBMP_OK) return st;
    if (!dev_ws || ws_bytes < need) return fail(LBMP_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, need);
    auto* h = new lbmp_sg();
    h->magic = SG_MAGIC;
    h->bmax = batch_max;
    h->step = 0;
    h->stream = static_cast<hipStream_t>(hip_stream);
    {
        const char* e = getenv("LBMP_SG_GRAPH");
        h->use_graph = h->stream != nullptr && !(e && e[0] == '0');
    }
    h->graph_B = 0;
    h->graph = nullptr;
    h->gexec = nullptr;
    Carver c(dev_ws, ws_bytes);
    carve_sg(h, c);
    hipStream_t s = h->stream;
    // zero everything once (padding rows/columns stay zero for good)
    if (hipMemsetAsync(dev_ws, 0, c.off, s) != hipSuccess) {
        delete h;
        return fail(LBMP_EDEVICE, "memset failed");
    }
    // default initialisation: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from splitmix64(seed)
    int64_t np = 0;
    sg_param_count(&np);
    std::vector<float> p((size_t)np);
    uint64_t x = seed;
    size_t k = 0;
    for (int l = 0; l < NLAYER; ++l) {
        const double bound = 1.0 / std::sqrt((double)tin(l));
        const int n = tout(l) * tin(l) + tout(l);
        for (int i = 0; i < n; ++i) {
            const double u = (double)(splitmix(x) >> 11) * (1.0 / 9007199254740992.0);
            p[k++] = (float)((2.0 * u - 1.0) * bound);
        }
    }
    const float norm[16] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 0, 1, 0, 0};
    if (hipMemcpyAsync(h->norm, norm, sizeof norm, hipMemcpyHostToDevice, s) != hipSuccess) {
        delete h;
        return fail(LBMP_EDEVICE, "copy failed");
    }
    st = sg_set_params(h, p.data());
    if (st != LBMP_OK) {
        delete h;
        return st;
    }
    *out = h;
    return LBMP_OK;
}

// Parameters packed as the FP64 reference orders them: W_1 [256][6], b_1,
// W_2 [256][256], b_2, W_3, b_3, W_4 [1][256], b_4 (fp32).
extern "C" lbmp_status sg_set_params(lbmp_sg* h, const float* p) {
    lbmp_status st = check(h);
    if (st != LBMP_OK) return st;
    if (!p) return fail(LBMP_EINVAL, "params is NULL");
    hipStream_t s = h->stream;
    size_t k = 0;
    for (int l = 0; l < NLAYER; ++l) {
        const int O = lout(l), I = lin(l), to = tout(l), ti = tin(l);
        std::vector<float> W((size_t)O * I, 0.0f), b(O, 0.0f);
        for (int o = 0; o < to; ++o)
            for (int i = 0; i < ti; ++i) W[(size_t)o * I + i] = p[k++];
        for (int o = 0; o < to; ++o) b[o] = p[k++];
        LBMP_HIP(hipMemcpyAsync(h->L[l].W, W.data(), W.size() * 4, hipMemcpyHostToDevice, s));
        LBMP_HIP(hipMemcpyAsync(h->L[l].b, b.data(), b.size() * 4, hipMemcpyHostToDevice, s));
        LBMP_HIP(hipMemsetAsync(h->L[l].mW, 0, W.size() * 4, s));
        LBMP_HIP(hipMemsetAsync(h->L[l].vW, 0, W.size() * 4, s));
        LBMP_HIP(hipMemsetAsync(h->L[l].mb, 0, b.size() * 4, s));
        LBMP_HIP(hipMemsetAsync(h->L[l].vb, 0, b.size() * 4, s));
        // bf16 copies through the Adam kernel with lr = 0 and no moving entries
        k_adam<<<(O * I + 255) / 256, 256, 0, s>>>(h->L[l].W, h->L[l].mW, h->L[l].vW, h->L[l].gW, O, I, 0, 0,
                                                  h->hyper, 0.f, 0.f, 1.f, h->L[l].Wb, h->L[l].WTb);
        LBMP_HIP(hipStreamSynchronize(s));
    }
    h->step = 0;
    return LBMP_OK;
}

extern "C" lbmp_status sg_get_params(lbmp_sg* h, float* p) {
    lbmp_status st = check(h);
    if (st != LBMP_OK) return st;
    if (!p) return fail(LBMP_EINVAL, "params is NULL");
    size_t k = 0;
    for (int l = 0; l < NLAYER; ++l) {
        const int O = lout(l), I = lin(l), to = tout(l), ti = tin(l);
        std::vector<float> W((size_t)O * I), b(O);
        LBMP_HIP(hipMemcpyAsync(W.data(), h->L[l].W, W.size() * 4, hipMemcpyDeviceToHost, h->stream));
        LBMP_HIP(hipMemcpyAsync(b.data(), h->L[l].b, b.size() * 4, hipMemcpyDeviceToHost, h->stream));
        LBMP_HIP(hipStreamSynchronize(h->stream));
        for (int o = 0; o < to; ++o)
            for (int i = 0; i < ti; ++i) p[k++] = W[(size_t)o * I + i];
        for (int o = 0; o < to; ++o) p[k++] = b[o];
    }
    return LBMP_OK;
}

extern "C" lbmp_status sg_set_normalization(lbmp_sg* h, const float* x_mean, const float* x_std, float y_mean,
                                            float y_std) {
    lbmp_status st = check(h);
    if (st != LBMP_OK) return st;
    if (!x_mean || !x_std) return fail(LBMP_EINVAL, "normalisation arrays are NULL");
    float v[16] = {0};
    for (int c = 0; c < NFEAT; ++c) {
        if (!(x_std[c] > 0.0f)) return fail(LBMP_EINVAL, "x_std[%d] must be > 0", c);
        v[c] = x_mean[c];
        v[6 + c] = x_std[c];
    }
    if (!(y_std > 0.0f)) return fail(LBMP_EINVAL, "y_std must be > 0");
    v[12] = y_mean;
    v[13] = y_std;
    LBMP_HIP(hipMemcpyAsync(h->norm, v, sizeof v, hipMemcpyHostToDevice, h->stream));
    LBMP_HIP(hipStreamSynchronize(h->stream));
    return LBMP_OK;
}

static lbmp_status sg_batch_in(lbmp_sg* h, const float* x, const float* y, const int32_t* idx, int B) {
    hipStream_t s = h->stream;
    k_gather<<<(B + 255) / 256, 256, 0, s>>>(x, y, idx, B, h->norm, h->xg, h->yg);
    k_pack_input<<<(B * PAD_IN + 255) / 256, 256, 0, s>>>(h->xg, B, h->xb);
    LBMP_HIP(hipGetLastError());
    return LBMP_OK;
}

extern "C" lbmp_status sg_train_step(lbmp_sg* h, const float* x_dev, const float* y_dev, const int32_t* idx_dev,
                                     int B, float lr, float* loss_host) {
    lbmp_status st = check(h);
    if (st != LBMP_OK) return st;
    if (B < 32 || B > h->bmax || B % 32 != 0) return fail(LBMP_EINVAL, "batch must be a multiple of 32 <= batch_max");
    if (!x_dev || !y_dev) return fail(LBMP_EINVAL, "data pointers are NULL");
    hipStream_t s = h->stream;
    st = sg_batch_in(h, x_dev, y_dev, idx_dev, B);
    if (st != LBMP_OK) return st;
    set_hyper(h, lr, s);
    if (h->use_graph) {
        // the step's kernels do not depend on the batch rows or the learning
        // rate (both in device memory): one graph per batch size
        if (!h->gexec || h->graph_B != B) {
            if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
            if (h->graph) (void)hipGraphDestroy(h->graph);
            h->gexec = nullptr;
            h->graph = nullptr;
            LBMP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            forward(h, B, s);
            backward(h, B, s);
            adam(h, s);
            LBMP_HIP(hipStreamEndCapture(s, &h->graph));
            LBMP_HIP(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
            h->graph_B = B;
        }
        LBMP_HIP(hipGraphLaunch(h->gexec, s));
    } else {
        forward(h, B, s);
        backward(h, B, s);
        adam(h, s);
    }
    LBMP_HIP(hipGetLastError());
    if (loss_host) {
        k_sum<<<1, 256, 0, s>>>(h->sq, B, h->loss);
        LBMP_HIP(hipMemcpyAsync(loss_host, h->loss, 4, hipMemcpyDeviceToHost, s));
        LBMP_HIP(hipStreamSynchronize(s));
    }
    return LBMP_OK;
}

extern "C" lbmp_status sg_gradients(lbmp_sg* h, const float* x_dev, const float* y_dev, int B, float* grads_host,
                                    float* loss_host) {
    lbmp_status st = check(h);
    if (st != LBMP_OK) return st;
    if (B < 32 || B > h->bmax || B % 32 != 0) return fail(LBMP_EINVAL, "batch must be a multiple of 32 <= batch_max");
    hipStream_t s = h->stream;
    st = sg_batch_in(h, x_dev, y_dev, nullptr, B);
    if (st != LBMP_OK) return st;
    forward(h, B, s);
    backward(h, B, s);
    k_sum<<<1, 256, 0, s>>>(h->sq, B, h->loss);
    LBMP_HIP(hipGetLastError());
    size_t k = 0;
    for (int l = 0; l < NLAYER; ++l) {
        const int O = lout(l), I = lin(l), to = tout(l), ti = tin(l);
        std::vector<float> W((size_t)O * I), b(O);
        LBMP_HIP(hipMemcpyAsync(W.data(), h->L[l].gW, W.size() * 4, hipMemcpyDeviceToHost, s));
        LBMP_HIP(hipMemcpyAsync(b.data(), h->L[l].gb, b.size() * 4, hipMemcpyDeviceToHost, s));
        LBMP_HIP(hipStreamSynchronize(s));
        if (grads_host) {
            for (int o = 0; o < to; ++o)
                for (int i = 0; i < ti; ++i) grads_host[k++] = W[(size_t)o * I + i];
            for (int o = 0; o < to; ++o) grads_host[k++] = b[o];
        }
    }
    if (loss_host) {
        LBMP_HIP(hipMemcpyAsync(loss_host, h->loss, 4, hipMemcpyDeviceToHost, s));
        LBMP_HIP(hipStreamSynchronize(s));
    }
    return LBMP_OK;
}

extern "C" lbmp_status sg_predict(lbmp_sg* h, const float* x_dev, int64_t n, float* y_dev) {
    lbmp_status st = check(h);
    if (st != LBMP_OK) return st;
    if (n < 0 || (n > 0 && (!x_dev || !y_dev))) return fail(LBMP_EINVAL, "bad arguments");
    hipStream_t s = h->stream;
    if (n > 0) {
        const Layer* L = h->L;
        k_mlp_forward<<<(unsigned)((n + FS - 1) / FS), 64 * FWAVES, 0, s>>>(x_dev, n, h->norm, L[0].Wb, L[0].b, L[1].Wb,
                                                                    L[1].b, L[2].Wb, L[2].b, L[3].Wb, L[3].b,
                                                                    y_dev);
    }
    LBMP_HIP(hipGetLastError());
    return LBMP_OK;
}

extern "C" lbmp_status sg_sync(lbmp_sg* h) {
    lbmp_status st = check(h);
    if (st != LBMP_OK) return st;
    LBMP_HIP(hipStreamSynchronize(h->stream));
    return LBMP_OK;
}

extern "C" void sg_free(lbmp_sg* h) {
    if (!h || h->magic != SG_MAGIC) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->magic = 0;
    delete h;
}
