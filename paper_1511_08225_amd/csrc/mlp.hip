// mlp.hip -- the warm-start network on gfx950: 4 -> 256 -> 256 -> 256 -> 1792,
// ReLU after the hidden layers.  Weights, biases, inputs and stored
// activations are BF16 (round to nearest even from FP32); products
// accumulate in FP32 on the matrix cores (v_mfma_f32_16x16x32_bf16, operand
// blocks staged in LDS), four wavefronts per 32x32 output block.  Training: backward on the same BF16
// operands (output and hidden gradients rounded to BF16 before each
// product), FP32 weight gradients, Adam on an FP32 master copy.
//
// Parameter vector (element offsets, identical in the BF16 and FP32 copies):
// W1 [256][4], b1 [256], W2 [256][256], b2, W3 [256][256], b3,
// W4 [1792][256], b4 [1792].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "slpic.h"

namespace slpic_mlp {

constexpr int kIn = SLPIC_MLP_IN, kHid = SLPIC_MLP_HIDDEN, kOut = SLPIC_MLP_OUT;
constexpr int64_t oW1 = 0, ob1 = oW1 + kHid * kIn;
constexpr int64_t oW2 = ob1 + kHid, ob2 = oW2 + kHid * kHid;
constexpr int64_t oW3 = ob2 + kHid, ob3 = oW3 + kHid * kHid;
constexpr int64_t oW4 = ob3 + kHid, ob4 = oW4 + (int64_t)kOut * kHid;
static_assert(ob4 + kOut == SLPIC_MLP_PARAMS, "parameter layout");

using bf16 = uint16_t;
typedef float v4f32 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite values)
__device__ __forceinline__ bf16 to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16)(u >> 16);
}
__device__ __forceinline__ float from_bf16(bf16 h) { return __uint_as_float((uint32_t)h << 16); }

enum Epi { kHidden = 0, kOutput = 1, kMasked = 2, kGrad = 3 };

// C[m][n] = sum_k A(m, k) B(k, n) with A(m, k) = A[m sam + k sak] and
// B(k, n) = B[k sbk + n sbn] (BF16), M, N, K multiples of 16.  A workgroup of
// four wavefronts computes a 32 x 32 block of C, wavefront w the 16 x 16 tile
// at rows 16 (w / 2), columns 16 (w % 2), on gfx950's v_mfma_f32_16x16x32_bf16
// (lane l holds A row l % 16 and B column l % 16 at k = 8 (l / 16) + 0..7;
// the accumulator holds rows 4 (l / 16) + 0..3 of column l % 16).  Each step
// of 64 k stages the A block [32 m][64 k] and the B block [32 n][64 k] in LDS,
// k contiguous in both, filled by one 16-byte global load per thread along
// whichever index is contiguous in memory (k, or m / n, then written to LDS
// element by element); rows past M or N and k past K are zero.  Epilogues:
//   kHidden: out_bf16[m][n] = bf16(max(acc + bias[n], 0))     (ldo)
//   kOutput: out_f32[m][n]  = acc + bias[n]
//   kMasked: out_bf16[m][n] = bf16(acc * (h[m][n] > 0))        (h: ldo)
//   kGrad:   out_f32[m][n]  = acc
constexpr int kBlk = 32;            // block tile side (m and n)
constexpr int kKs = 64;             // k per staged step
constexpr int kLdsRow = kKs + 8;    // padded LDS row (bf16): 144 B, rows start 16 B apart mod 128
typedef __bf16 v8bf16 __attribute__((ext_vector_type(8)));

// One operand block [32 rows][64 k] into LDS rows (k contiguous): rows r of
// the operand are X[(r0 + r) srow + (k0 + k) sk]; 256 threads, 8 elements each.
__device__ __forceinline__ void stage_block(const bf16* __restrict__ X, int64_t srow, int64_t sk, int r0,
                                            int rows, int k0, int K, bf16 (*L)[kLdsRow]) {
    const int t = threadIdx.x;
    if (sk == 1) {  // 8 consecutive k of one row
        const int r = t >> 3, k = (t & 7) * 8;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (r0 + r < rows && k0 + k < K) v = *(const uint4*)(X + (int64_t)(r0 + r) * srow + (k0 + k));
        *(uint4*)&L[r][k] = v;
    } else if (srow == 1) {  // 8 consecutive rows at one k
        const int k = t >> 2, r = (t & 3) * 8;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (r0 + r < rows && k0 + k < K) v = *(const uint4*)(X + (int64_t)(r0 + r) + (int64_t)(k0 + k) * sk);
        const bf16* e = (const bf16*)&v;
#pragma unroll
        for (int j = 0; j < 8; ++j) L[r + j][k] = e[j];
    } else {  // neither index contiguous: element by element
        for (int q = t; q < kBlk * kKs; q += blockDim.x) {
            const int r = q / kKs, k = q % kKs;
            L[r][k] = (r0 + r < rows && k0 + k < K) ? X[(int64_t)(r0 + r) * srow + (int64_t)(k0 + k) * sk] : (bf16)0;
        }
    }
}

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(const bf16* __restrict__ A, int64_t sam, int64_t sak,
                                              const bf16* __restrict__ B, int64_t sbk, int64_t sbn, int M, int N,
                                              int K, const bf16* __restrict__ bias, const bf16* __restrict__ h,
                                              void* __restrict__ out, int64_t ldo) {
    __shared__ __align__(16) bf16 As[kBlk][kLdsRow];
    __shared__ __align__(16) bf16 Bs[kBlk][kLdsRow];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int bn_count = (N + kBlk - 1) / kBlk;
    const int bm = (int)(blockIdx.x / bn_count) * kBlk, bn = (int)(blockIdx.x % bn_count) * kBlk;
    const int i = lane & 15, kq = lane >> 4;
    const int ar = 16 * (w >> 1) + i, bc = 16 * (w & 1) + i;  // this lane's A row and B column in the block
    v4f32 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += kKs) {
        stage_block(A, sam, sak, bm, M, k0, K, As);  // A(m, k): rows m
        stage_block(B, sbn, sbk, bn, N, k0, K, Bs);  // B(k, n): rows n
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKs; kk += 32) {
            const v8bf16 a = *(const v8bf16*)&As[ar][kk + 8 * kq];
            const v8bf16 b = *(const v8bf16*)&Bs[bc][kk + 8 * kq];
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const int col = bn + 16 * (w & 1) + i;
    if (col >= N) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = bm + 16 * (w >> 1) + 4 * kq + r;
        if (row >= M) continue;
        const int64_t o = (int64_t)row * ldo + col;
        if (EPI == kHidden) {
            ((bf16*)out)[o] = to_bf16(fmaxf(acc[r] + from_bf16(bias[col]), 0.f));
        } else if (EPI == kOutput) {
            ((float*)out)[o] = acc[r] + from_bf16(bias[col]);
        } else if (EPI == kMasked) {
            ((bf16*)out)[o] = to_bf16(from_bf16(h[o]) > 0.f ? acc[r] : 0.f);
        } else {
            ((float*)out)[o] = acc[r];
        }
    }
}

template <int EPI>
void gemm(const bf16* A, int64_t sam, int64_t sak, const bf16* B, int64_t sbk, int64_t sbn, int M, int N, int K,
          const bf16* bias, const bf16* h, void* out, int64_t ldo, hipStream_t s) {
    const int64_t blocks = (int64_t)((M + kBlk - 1) / kBlk) * ((N + kBlk - 1) / kBlk);
    hipLaunchKernelGGL(k_gemm<EPI>, dim3((unsigned)blocks), dim3(256), 0, s, A, sam, sak, B, sbk, sbn, M, N, K, bias,
                       h, out, ldo);
}

// First layer (K = 4): x -> bf16(x), h1 = bf16(max(x W1^T + b1, 0)).
__global__ void k_layer1(const bf16* __restrict__ P, const float* __restrict__ x, int batch, bf16* __restrict__ xr,
                         bf16* __restrict__ h1) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)batch * kHid) return;
    const int b = (int)(t / kHid), j = (int)(t % kHid);
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kIn; ++k) {
        const bf16 xb = to_bf16(x[b * kIn + k]);
        if (j == 0) xr[b * kIn + k] = xb;
        acc = fmaf(from_bf16(xb), from_bf16(P[oW1 + j * kIn + k]), acc);
    }
    h1[t] = to_bf16(fmaxf(acc + from_bf16(P[ob1 + j]), 0.f));
}

// dW1[j][k] = sum_b dh1[b][j] x[b][k] (K = 4, no matrix-core tile).
__global__ void k_grad_w1(const bf16* __restrict__ dh1, const bf16* __restrict__ xr, int batch,
                          float* __restrict__ g) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kHid * kIn) return;
    const int j = t / kIn, k = t % kIn;
    float acc = 0.f;
    for (int b = 0; b < batch; ++b) acc = fmaf(from_bf16(dh1[(int64_t)b * kHid + j]), from_bf16(xr[b * kIn + k]), acc);
    g[oW1 + t] = acc;
}
// Bias gradients: column sums db[n] = sum_b D[b][n].
__global__ void k_colsum(const bf16* __restrict__ D, int rows, int cols, float* __restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= cols) return;
    float acc = 0.f;
    for (int b = 0; b < rows; ++b) acc += from_bf16(D[(int64_t)b * cols + n]);
    out[n] = acc;
}
__global__ void k_round(const float* __restrict__ in, bf16* __restrict__ out, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = to_bf16(in[t]);
}

// Adam: m, v moving averages of g and g^2; p -= lr (m / c1) / (sqrt(v / c2) + eps)
// with the bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void k_adam(float* __restrict__ p, bf16* __restrict__ pb, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float b1, float b2, float c1, float c2, float lr,
                       float eps) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    const float pt = p[t] - lr * (mt / c1) / (sqrtf(vt / c2) + eps);
    p[t] = pt;
    pb[t] = to_bf16(pt);
}

// Mean squared error over n outputs: dy = 2 (y - t) / n, and the loss
// sum (y - t)^2 / n added to *loss (per-block partial sums, one atomic each).
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t, float* __restrict__ dy, int64_t n,
                      float* __restrict__ loss) {
    __shared__ float part[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float e2 = 0.f;
    if (i < n) {
        const float d = y[i] - t[i];
        dy[i] = 2.f * d / (float)n;
        e2 = d * d;
    }
    for (int o = 32; o >= 1; o >>= 1) e2 += __shfl_xor(e2, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = e2;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, (part[0] + part[1] + part[2] + part[3]) / (float)n);
}

}  // namespace slpic_mlp

using namespace slpic_mlp;

static int last_error() { return hipGetLastError() == hipSuccess ? SLPIC_OK : SLPIC_EHIP; }

// The forward pass on caller buffers: BF16 inputs and the three hidden
// activations go to act ([batch][4 + 3 * 256] BF16), the output to y.
static int forward_impl(const bf16* P, const float* x, float* y, int32_t batch, bf16* act, hipStream_t s) {
    bf16* xr = act;
    bf16* h1 = xr + (int64_t)batch * kIn;
    bf16* h2 = h1 + (int64_t)batch * kHid;
    bf16* h3 = h2 + (int64_t)batch * kHid;
    const int64_t n1 = (int64_t)batch * kHid;
    hipLaunchKernelGGL(k_layer1, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, P, x, batch, xr, h1);
    // h_{l+1}[b][n] = relu(sum_k h_l[b][k] W[n][k] + b[n])
    gemm<kHidden>(h1, kHid, 1, P + oW2, 1, kHid, batch, kHid, kHid, P + ob2, nullptr, h2, kHid, s);
    gemm<kHidden>(h2, kHid, 1, P + oW3, 1, kHid, batch, kHid, kHid, P + ob3, nullptr, h3, kHid, s);
    gemm<kOutput>(h3, kHid, 1, P + oW4, 1, kHid, batch, kOut, kHid, P + ob4, nullptr, y, kOut, s);
    return last_error();
}

// Activation scratch of the allocation-free forward pass: a fixed array in
// device memory, one copy per GPU (loaded with the code object), never
// allocated at run time.  Host code only ever uses the address
// hipGetSymbolAddress returns for the current device: the array's name is a
// host-side stand-in.  Calls that overlap on one GPU share it and race.
constexpr int kNoAllocMaxBatch = SLPIC_MLP_NOALLOC_MAX_BATCH;
constexpr int64_t kNoAllocScratch = (int64_t)kNoAllocMaxBatch * (kIn + 3 * kHid);
static __device__ __align__(256) bf16 scratch[kNoAllocScratch];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices];  // device address of scratch, per device ordinal

// The current device's scratch address, looked up on the first call on that
// device (with it current) and kept.
static int noalloc_scratch(bf16** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SLPIC_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SLPIC_EHIP;
        g_scratch_dev[dev] = p;
    }
    *out = (bf16*)g_scratch_dev[dev];
    return SLPIC_OK;
}

extern "C" {

size_t slpic_mlp_act_bytes(int32_t batch) {
    return batch > 0 ? (size_t)batch * (kIn + 3 * kHid) * sizeof(bf16) : 0;
}
size_t slpic_mlp_work_bytes(int32_t batch) {
    return batch > 0 ? (size_t)batch * (kOut + 3 * kHid) * sizeof(bf16) : 0;
}

int slpic_mlp_to_bf16(const float* d_params_fp32, void* d_params_bf16, void* stream) {
    if (!d_params_fp32 || !d_params_bf16) return SLPIC_EINVAL;
    const int64_t n = SLPIC_MLP_PARAMS;
    hipLaunchKernelGGL(k_round, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, d_params_fp32,
                       (bf16*)d_params_bf16, n);
    return last_error();
}

int slpic_mlp_forward(const void* d_params_bf16, const float* d_x, float* d_y, int32_t batch, void* d_act,
                      void* stream) {
    if (!d_params_bf16 || !d_x || !d_y || !d_act || batch <= 0 || batch % 16) return SLPIC_EINVAL;
    return forward_impl((const bf16*)d_params_bf16, d_x, d_y, batch, (bf16*)d_act, (hipStream_t)stream);
}

int slpic_mlp_forward_noalloc(const void* d_params_bf16, const float* d_x, float* d_y, int32_t batch,
                              void* stream) {
    if (!d_params_bf16 || !d_x || !d_y || batch <= 0 || batch % 16) return SLPIC_EINVAL;
    if (batch > kNoAllocMaxBatch) return SLPIC_ELIMIT;
    bf16* act = nullptr;
    const int rc = noalloc_scratch(&act);
    if (rc != SLPIC_OK) return rc;
    return forward_impl((const bf16*)d_params_bf16, d_x, d_y, batch, act, (hipStream_t)stream);
}

int slpic_mlp_backward(const void* d_params_bf16, const void* d_act, const float* d_dy, float* d_grads,
                       int32_t batch, void* d_work, void* stream) {
    if (!d_params_bf16 || !d_act || !d_dy || !d_grads || !d_work || batch <= 0 || batch % 16) return SLPIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const bf16* P = (const bf16*)d_params_bf16;
    const bf16* xr = (const bf16*)d_act;
    const bf16* h1 = xr + (int64_t)batch * kIn;
    const bf16* h2 = h1 + (int64_t)batch * kHid;
    const bf16* h3 = h2 + (int64_t)batch * kHid;
    bf16* dy = (bf16*)d_work;
    bf16* d3 = dy + (int64_t)batch * kOut;
    bf16* d2 = d3 + (int64_t)batch * kHid;
    bf16* d1 = d2 + (int64_t)batch * kHid;
    float* g = d_grads;
    const int64_t ny = (int64_t)batch * kOut;
    hipLaunchKernelGGL(k_round, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, s, d_dy, dy, ny);
    // layer 4: dW4[o][i] = sum_b dy[b][o] h3[b][i]; db4; d3 = (dy W4) * (h3 > 0)
    gemm<kGrad>(dy, 1, kOut, h3, kHid, 1, kOut, kHid, batch, nullptr, nullptr, g + oW4, kHid, s);
    hipLaunchKernelGGL(k_colsum, dim3((kOut + 255) / 256), dim3(256), 0, s, dy, batch, kOut, g + ob4);
    gemm<kMasked>(dy, kOut, 1, P + oW4, kHid, 1, batch, kHid, kOut, nullptr, h3, d3, kHid, s);
    // layer 3
    gemm<kGrad>(d3, 1, kHid, h2, kHid, 1, kHid, kHid, batch, nullptr, nullptr, g + oW3, kHid, s);
    hipLaunchKernelGGL(k_colsum, dim3((kHid + 255) / 256), dim3(256), 0, s, d3, batch, kHid, g + ob3);
    gemm<kMasked>(d3, kHid, 1, P + oW3, kHid, 1, batch, kHid, kHid, nullptr, h2, d2, kHid, s);
    // layer 2
    gemm<kGrad>(d2, 1, kHid, h1, kHid, 1, kHid, kHid, batch, nullptr, nullptr, g + oW2, kHid, s);
    hipLaunchKernelGGL(k_colsum, dim3((kHid + 255) / 256), dim3(256), 0, s, d2, batch, kHid, g + ob2);
    gemm<kMasked>(d2, kHid, 1, P + oW2, kHid, 1, batch, kHid, kHid, nullptr, h1, d1, kHid, s);
    // layer 1
    hipLaunchKernelGGL(k_grad_w1, dim3((kHid * kIn + 255) / 256), dim3(256), 0, s, d1, xr, batch, g);
    hipLaunchKernelGGL(k_colsum, dim3((kHid + 255) / 256), dim3(256), 0, s, d1, batch, kHid, g + ob1);
    return last_error();
}

int slpic_mlp_mse(const float* d_y, const float* d_t, float* d_dy, int64_t n, float* d_loss, void* stream) {
    if (!d_y || !d_t || !d_dy || !d_loss || n <= 0) return SLPIC_EINVAL;
    hipLaunchKernelGGL(k_mse, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, d_y, d_t, d_dy, n,
                       d_loss);
    return last_error();
}

int slpic_mlp_adam(float* d_params_fp32, void* d_params_bf16, float* d_m, float* d_v, const float* d_grads,
                   float lr, float beta1, float beta2, float eps, int32_t step, void* stream) {
    if (!d_params_fp32 || !d_params_bf16 || !d_m || !d_v || !d_grads || step < 1) return SLPIC_EINVAL;
    const int64_t n = SLPIC_MLP_PARAMS;
    const double c1 = 1.0 - std::pow((double)beta1, step), c2 = 1.0 - std::pow((double)beta2, step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, d_params_fp32,
                       (bf16*)d_params_bf16, d_m, d_v, d_grads, n, beta1, beta2, (float)c1, (float)c2, lr, eps);
    return last_error();
}

}  // extern "C"
