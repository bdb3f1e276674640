// Learned configuration selection: matrix features and a small MLP
// (40 -> 64 -> 64 -> 24, ReLU, fp32) with forward, backward and Adam kernels.
//
// The paper picks the strip height and kernel options by brute-force search
// over measured times (Sec. 6.3) and notes how much per-matrix tuning could
// still gain (Sec. 6.8).  Here the measured times of every (height, schedule)
// class train a network that predicts, from cheap features of the CSR
// structure, the log time of each class relative to the fastest; the
// selector takes the class with the lowest prediction.
//
// Features (kSelFeatures = 40), all from row_ptr / col_ind:
//   [0, 20)   fraction of rows by length in half octaves: bin 0 empty; a
//             length with p = floor(log2 len) goes to 1 + 2p, or 2 + 2p when
//             2 len >= 3 * 2^p; bins above 19 fold into 19 (len >= 512)
//   [20, 36)  fraction of entries by |col - row * cols / rows|: bin 0 for 0,
//             bin b >= 1 for distances in [2^(b-1), 2^b), last bin open
//   36..39    log2(rows)/22, log2(nnz+1)/26, log2(mean length+1)/14,
//             log2(max length+1)/14
// Parameters, packed: W1[40][64], b1[64], W2[64][64], b2[64], W3[64][24], b3[24]
// (8344 floats); activations row-major [batch][width].
#include <math.h>

#include "cmrs_device.hpp"
#include "cmrs_ext.hpp"

namespace cmrs {

constexpr int kSelFeatures = 40, kSelHidden = 64, kSelClasses = 24;
constexpr int kRowBins = 20, kDistBins = 16;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kSelFeatures * kSelHidden;
constexpr int kOffW2 = kOffB1 + kSelHidden;
constexpr int kOffB2 = kOffW2 + kSelHidden * kSelHidden;
constexpr int kOffW3 = kOffB2 + kSelHidden;
constexpr int kOffB3 = kOffW3 + kSelHidden * kSelClasses;
constexpr int kSelParams = kOffB3 + kSelClasses;
static_assert(kSelParams == 8344, "parameter count");

// ------------------------------------------------------------------ features

__device__ inline int row_len_bin(int len) {
    if (len <= 0) return 0;
    const int p = 31 - __clz(len);
    const int b = 1 + 2 * p + ((2LL * len >= (3LL << p)) ? 1 : 0);
    return b < kRowBins - 1 ? b : kRowBins - 1;
}

__device__ inline int dist_bin(long long d) {
    if (d <= 0) return 0;
    const int b = 64 - __clzll(static_cast<unsigned long long>(d));  // d in [2^(b-1), 2^b)
    return b < kDistBins - 1 ? b : kDistBins - 1;
}

// ws: int counts [kRowBins + kDistBins], int max length.  Zeroed first.
__global__ __launch_bounds__(256) void feature_count_kernel(int rows, int cols, const int* __restrict__ row_ptr,
                                                            const int* __restrict__ col_ind, int* __restrict__ ws) {
    __shared__ int hist[kRowBins + kDistBins];
    __shared__ int maxlen;
    if (threadIdx.x < kRowBins + kDistBins) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) maxlen = 0;
    __syncthreads();
    const int lane = lane_id();
    const int wave = static_cast<int>(threadIdx.x) / kWave;
    const double scale = rows > 0 ? static_cast<double>(cols) / rows : 0.0;
    // One wave per 64-row group: lane l takes row r0 + l's length; the group's
    // entries are then walked by all 64 lanes, each entry's row found by a
    // binary search over the lanes' row pointers.
    for (long long r0l = (static_cast<long long>(blockIdx.x) * 4 + wave) * kWave; r0l < rows;
         r0l += static_cast<long long>(gridDim.x) * 4 * kWave) {
        const int r0 = static_cast<int>(r0l);
        const int nr = min(kWave, rows - r0);
        const int my = lane < nr ? row_ptr[r0 + lane] : 0x7fffffff;
        const int e0 = __shfl(my, 0);
        const int e1 = row_ptr[r0 + nr];
        const int next = __shfl(my, lane + 1 < kWave ? lane + 1 : kWave - 1);
        if (lane < nr) {
            const int len = (lane + 1 < nr ? next : e1) - my;
            atomicAdd(&hist[row_len_bin(len)], 1);
            atomicMax(&maxlen, len);
        }
        for (int base = e0; base < e1; base += kWave) {
            const int e = base + lane;
            int lo = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const int v = __shfl(my, lo + step < kWave ? lo + step : kWave - 1);
                if (lo + step < nr && v <= e) lo += step;
            }
            if (e < e1) {
                const long long c = col_ind[e];
                const long long center = static_cast<long long>(static_cast<double>(r0 + lo) * scale);
                const long long d = c > center ? c - center : center - c;
                atomicAdd(&hist[kRowBins + dist_bin(d)], 1);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < kRowBins + kDistBins && hist[threadIdx.x]) atomicAdd(&ws[threadIdx.x], hist[threadIdx.x]);
    if (threadIdx.x == 0 && maxlen) atomicMax(&ws[kRowBins + kDistBins], maxlen);
}

__global__ void feature_finish_kernel(int rows, int nnz, const int* __restrict__ ws, float* __restrict__ feat) {
    const int t = static_cast<int>(threadIdx.x);
    if (t < kRowBins) feat[t] = rows > 0 ? static_cast<float>(ws[t]) / rows : 0.0f;
    if (t >= kRowBins && t < kRowBins + kDistBins) feat[t] = nnz > 0 ? static_cast<float>(ws[t]) / nnz : 0.0f;
    if (t == 0) {
        const float mean = rows > 0 ? static_cast<float>(nnz) / rows : 0.0f;
        feat[36] = log2f(static_cast<float>(rows > 0 ? rows : 1)) / 22.0f;
        feat[37] = log2f(static_cast<float>(nnz) + 1.0f) / 26.0f;
        feat[38] = log2f(mean + 1.0f) / 14.0f;
        feat[39] = log2f(static_cast<float>(ws[kRowBins + kDistBins]) + 1.0f) / 14.0f;
    }
}

// ------------------------------------------------------------------ MLP

// Layer out[b][j] = act(sum_i in[b][i] * W[i][j] + bias[j]); one thread per
// (b, j), sums in index order.
__global__ __launch_bounds__(256) void dense_forward_kernel(int batch, int nin, int nout, const float* __restrict__ in,
                                                            const float* __restrict__ W, const float* __restrict__ bias,
                                                            float* __restrict__ out, int relu) {
    const int t = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= batch * nout) return;
    const int b = t / nout, j = t % nout;
    float s = bias[j];
    for (int i = 0; i < nin; ++i) s = fmaf(in[b * nin + i], W[i * nout + j], s);
    out[t] = relu && s < 0.0f ? 0.0f : s;
}

// dL/dY for L = mean over batch and classes of (Y - T)^2.
__global__ __launch_bounds__(256) void mse_grad_kernel(int n, const float* __restrict__ Y, const float* __restrict__ T,
                                                       float* __restrict__ dY, float scale) {
    const int t = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (t < n) dY[t] = scale * (Y[t] - T[t]);
}

// Weight and bias gradients of one layer: dW[i][j] = sum_b in[b][i] dOut[b][j],
// db[j] = sum_b dOut[b][j], one thread per weight, batch summed in order
// (deterministic).
__global__ __launch_bounds__(256) void dense_weight_grad_kernel(int batch, int nin, int nout,
                                                                const float* __restrict__ in,
                                                                const float* __restrict__ dout,
                                                                float* __restrict__ dW, float* __restrict__ db) {
    const int t = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (t < nin * nout) {
        const int i = t / nout, j = t % nout;
        float s = 0.0f;
        for (int b = 0; b < batch; ++b) s = fmaf(in[b * nin + i], dout[b * nout + j], s);
        dW[t] = s;
    } else if (t < nin * nout + nout) {
        const int j = t - nin * nout;
        float s = 0.0f;
        for (int b = 0; b < batch; ++b) s += dout[b * nout + j];
        db[j] = s;
    }
}

// Input gradient through a layer and the ReLU of its input:
// din[b][i] = (act[b][i] > 0) * sum_j dout[b][j] W[i][j].
__global__ __launch_bounds__(256) void dense_input_grad_kernel(int batch, int nin, int nout,
                                                               const float* __restrict__ act,
                                                               const float* __restrict__ W,
                                                               const float* __restrict__ dout,
                                                               float* __restrict__ din) {
    const int t = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= batch * nin) return;
    const int b = t / nin, i = t % nin;
    float s = 0.0f;
    for (int j = 0; j < nout; ++j) s = fmaf(dout[b * nout + j], W[i * nout + j], s);
    din[t] = act[t] > 0.0f ? s : 0.0f;
}

// Adam (Kingma & Ba), bias-corrected, fp32.
__global__ __launch_bounds__(256) void adam_kernel(int n, float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                   float b2, float eps, float c1, float c2) {
    const int t = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.0f - b1) * gt;
    const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

__global__ void feature_zero_kernel(int* __restrict__ ws, int n) {
    if (static_cast<int>(threadIdx.x) < n) ws[threadIdx.x] = 0;
}

namespace {
inline int blocks_for(long long n) { return static_cast<int>((n + 255) / 256); }
}  // namespace

hipError_t launch_features(int rows, int cols, int nnz, const int* row_ptr, const int* col_ind, float* feat,
                           int* ws, hipStream_t stream) {
    hipLaunchKernelGGL(feature_zero_kernel, dim3(1), dim3(64), 0, stream, ws, kRowBins + kDistBins + 1);
    const int groups = (rows + kWave - 1) / kWave;
    int g = (groups + 3) / 4;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(feature_count_kernel, dim3(g), dim3(256), 0, stream, rows, cols, row_ptr, col_ind, ws);
    hipLaunchKernelGGL(feature_finish_kernel, dim3(1), dim3(64), 0, stream, rows, nnz, ws, feat);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(int batch, const float* X, const float* params, float* H1, float* H2, float* Y,
                              hipStream_t stream) {
    hipLaunchKernelGGL(dense_forward_kernel, dim3(blocks_for(1LL * batch * kSelHidden)), dim3(256), 0, stream, batch,
                       kSelFeatures, kSelHidden, X, params + kOffW1, params + kOffB1, H1, 1);
    hipLaunchKernelGGL(dense_forward_kernel, dim3(blocks_for(1LL * batch * kSelHidden)), dim3(256), 0, stream, batch,
                       kSelHidden, kSelHidden, H1, params + kOffW2, params + kOffB2, H2, 1);
    hipLaunchKernelGGL(dense_forward_kernel, dim3(blocks_for(1LL * batch * kSelClasses)), dim3(256), 0, stream, batch,
                       kSelHidden, kSelClasses, H2, params + kOffW3, params + kOffB3, Y, 0);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(int batch, const float* X, const float* params, const float* H1, const float* H2,
                               const float* dY, float* dH2, float* dH1, float* grads, hipStream_t stream) {
    // Output layer.
    hipLaunchKernelGGL(dense_weight_grad_kernel, dim3(blocks_for(kSelHidden * kSelClasses + kSelClasses)), dim3(256),
                       0, stream, batch, kSelHidden, kSelClasses, H2, dY, grads + kOffW3, grads + kOffB3);
    hipLaunchKernelGGL(dense_input_grad_kernel, dim3(blocks_for(1LL * batch * kSelHidden)), dim3(256), 0, stream,
                       batch, kSelHidden, kSelClasses, H2, params + kOffW3, dY, dH2);
    // Hidden layer 2.
    hipLaunchKernelGGL(dense_weight_grad_kernel, dim3(blocks_for(kSelHidden * kSelHidden + kSelHidden)), dim3(256), 0,
                       stream, batch, kSelHidden, kSelHidden, H1, dH2, grads + kOffW2, grads + kOffB2);
    hipLaunchKernelGGL(dense_input_grad_kernel, dim3(blocks_for(1LL * batch * kSelHidden)), dim3(256), 0, stream,
                       batch, kSelHidden, kSelHidden, H1, params + kOffW2, dH2, dH1);
    // Hidden layer 1.
    hipLaunchKernelGGL(dense_weight_grad_kernel, dim3(blocks_for(kSelFeatures * kSelHidden + kSelHidden)), dim3(256),
                       0, stream, batch, kSelFeatures, kSelHidden, X, dH1, grads + kOffW1, grads + kOffB1);
    return hipGetLastError();
}

hipError_t launch_mse_grad(int n, const float* Y, const float* T, float* dY, float scale, hipStream_t stream) {
    hipLaunchKernelGGL(mse_grad_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, n, Y, T, dY, scale);
    return hipGetLastError();
}

hipError_t launch_adam(int n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                       int step, hipStream_t stream) {
    const float c1 = 1.0f - powf(b1, static_cast<float>(step));
    const float c2 = 1.0f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, n, p, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace cmrs
