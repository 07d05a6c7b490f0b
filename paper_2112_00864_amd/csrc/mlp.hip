// Kernels of the surrogate network: a multilayer perceptron with SiLU activations in FP32,
// forward (inference and training), backward and the Adam step. Matrices are row-major;
// a layer computes Z = X W + b with X [B x K], W [K x N], then H = silu(Z).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>

#include "common.hpp"
#include "mlp.hpp"

namespace bcv {
namespace {

constexpr int kTile = 64, kTileK = 16, kThreads = 256;
constexpr int kSplitRows = 256;  // rows of the reduction dimension per split (weight and bias gradients)

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + __expf(-z)); }

// C[M x N] = op(A) op(B) (+ bias, + C if accumulate). op(A)[m][k] = TA ? A[k * lda + m] :
// A[m * lda + k]; op(B)[k][n] = TB ? B[n * ldb + k] : B[k * ldb + n]. If H is given it also
// receives silu(C). One 256-thread block per 64 x 64 tile, K in steps of 16 through LDS, the products
// on the matrix cores in FP32 (each wave a 32 x 32 quarter as four 16 x 16 MFMA tiles). The sums run
// in a fixed order: results do not depend on the launch.
// Split K: block z covers k in [z k_chunk, (z + 1) k_chunk) and writes its partial product to
// C + z c_stride (no bias, accumulate or H then; the partial products are summed by
// sum_splits_kernel in z order).
typedef float f4_t __attribute__((ext_vector_type(4)));

template <bool TA, bool TB>
__global__ __launch_bounds__(kThreads) void gemm_kernel(int M, int N, int K, const float *__restrict__ A, int lda,
                                                        const float *__restrict__ B, int ldb,
                                                        const float *__restrict__ bias, int accumulate,
                                                        float *__restrict__ C, int ldc, float *__restrict__ H,
                                                        int k_chunk, int64_t c_stride)
{
    __shared__ float As[kTileK][kTile + 1];
    __shared__ float Bs[kTileK][kTile + 1];
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wm = 32 * (wave >> 1), wn = 32 * (wave & 1);  // the wave's 32 x 32 quarter of the tile
    const int k_begin = (int)blockIdx.z * k_chunk, k_end = min(K, k_begin + k_chunk);
    C += (int64_t)blockIdx.z * c_stride;
    // v_mfma_f32_16x16x4f32 (FP32 operands, FP32 accumulation): A[i][k] in lane i + 16 k,
    // B[k][n] in lane n + 16 k, D[i][n] in lane n + 16 (i / 4), element i % 4. Four 16 x 16 tiles
    // per wave.
    f4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = k_begin; k0 < k_end; k0 += kTileK) {
        for (int e = threadIdx.x; e < kTileK * kTile; e += kThreads) {
            const int kk = e / kTile, mm = e % kTile;
            const int m = m0 + mm, k = k0 + kk;
            As[kk][mm] = (m < M && k < k_end) ? (TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k]) : 0.0f;
            const int n = n0 + mm;
            Bs[kk][mm] = (n < N && k < k_end) ? (TB ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n]) : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kTileK; kk += 4) {
            const int kr = kk + lane / 16;
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kr][wm + 16 * i + lane % 16];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[kr][wn + 16 * j + lane % 16];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (lane / 16) + r, n = n0 + wn + 16 * j + lane % 16;
                if (m >= M || n >= N) continue;
                float z = acc[i][j][r];
                if (bias) z += bias[n];
                float *c = C + (int64_t)m * ldc + n;
                if (accumulate) z += *c;
                *c = z;
                if (H) H[(int64_t)m * ldc + n] = z * sigmoid(z);
            }
}

// out[i] = sum over z < splits of part[z * n + i], in z order (+ out[i] if accumulate).
__global__ void sum_splits_kernel(int64_t n, int splits, const float *__restrict__ part, int accumulate,
                                  float *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float s = accumulate ? out[i] : 0.0f;
        for (int z = 0; z < splits; ++z) s += part[(int64_t)z * n + i];
        out[i] = s;
    }
}

// dZ = dH * silu'(Z), silu'(z) = s (1 + z (1 - s)), s = sigmoid(z).
__global__ void silu_backward_kernel(int64_t n, const float *__restrict__ Z, const float *__restrict__ dH,
                                     float *__restrict__ dZ)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float z = Z[i], s = sigmoid(z);
        dZ[i] = dH[i] * s * (1.0f + z * (1.0f - s));
    }
}

// Partial column sums: part[z][n] = sum of dZ[m][n] over rows m in [z rows, (z + 1) rows), in
// order; block (x, z) covers columns 128 x .. 128 x + 127 of row chunk z.
__global__ void column_sum_kernel(int M, int N, int rows, const float *__restrict__ dZ, float *__restrict__ part)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int m0 = (int)blockIdx.y * rows, m1 = min(M, m0 + rows);
    float s = 0.0f;
    for (int m = m0; m < m1; ++m) s += dZ[(int64_t)m * N + n];
    part[(int64_t)blockIdx.y * N + n] = s;
}

// Loss of a batch of B rows Y = (value, log-error) against targets r (mean over the batch):
//   L = mean (y0 - r)^2 + w_err * mean (y1 - log(|y0 - r| + eps))^2,
// the second term with y0 held fixed (the error head learns the size of the value head's miss).
// dY receives dL/dY; loss_terms[i] the two squared terms of row i.
__global__ void loss_kernel(int B, const float *__restrict__ Y, const float *__restrict__ r, float w_err, float eps,
                            float *__restrict__ dY, float *__restrict__ loss_terms)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const float d = Y[2 * i] - r[i];
    const float e = Y[2 * i + 1] - logf(fabsf(d) + eps);
    dY[2 * i] = 2.0f * d / B;
    dY[2 * i + 1] = 2.0f * w_err * e / B;
    loss_terms[2 * i] = d * d;
    loss_terms[2 * i + 1] = e * e;
}

// Adam (Kingma & Ba 2015) with bias correction folded into the step size.
__global__ void adam_kernel(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr_t, float b1, float b2, float eps)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr_t * mi / (sqrtf(vi) + eps);
    }
}

// Gather rows: out[i][:] = in[idx[i]][:] (minibatches), width d.
__global__ void gather_rows_kernel(int B, int d, const int32_t *__restrict__ idx, const float *__restrict__ in,
                                   float *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * d) return;
    const int i = (int)(e / d), c = (int)(e % d);
    out[e] = in[(int64_t)idx[i] * d + c];
}

unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 4096); }

}  // namespace

void gemm(bool ta, bool tb, int M, int N, int K, const float *A, int lda, const float *B, int ldb, const float *bias,
          bool accumulate, float *C, int ldc, float *H, hipStream_t st)
{
    if (M <= 0 || N <= 0) return;
    const dim3 grid((N + kTile - 1) / kTile, (M + kTile - 1) / kTile);
    const int kc = std::max(K, 1);
    if (!ta && !tb)
        gemm_kernel<false, false><<<grid, kThreads, 0, st>>>(M, N, K, A, lda, B, ldb, bias, accumulate, C, ldc, H, kc, 0);
    else if (!ta && tb)
        gemm_kernel<false, true><<<grid, kThreads, 0, st>>>(M, N, K, A, lda, B, ldb, bias, accumulate, C, ldc, H, kc, 0);
    else if (ta && !tb)
        gemm_kernel<true, false><<<grid, kThreads, 0, st>>>(M, N, K, A, lda, B, ldb, bias, accumulate, C, ldc, H, kc, 0);
    else
        gemm_kernel<true, true><<<grid, kThreads, 0, st>>>(M, N, K, A, lda, B, ldb, bias, accumulate, C, ldc, H, kc, 0);
    BCV_HIP(hipGetLastError());
}

int64_t split_workspace(int M, int N, int K) { return (int64_t)((K + kSplitRows - 1) / kSplitRows) * M * N; }

void gemm_tn_split(int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, float *ws,
                   hipStream_t st)
{
    if (M <= 0 || N <= 0) return;
    const int splits = std::max(1, (K + kSplitRows - 1) / kSplitRows);
    const dim3 grid((N + kTile - 1) / kTile, (M + kTile - 1) / kTile, splits);
    gemm_kernel<true, false><<<grid, kThreads, 0, st>>>(M, N, K, A, lda, B, ldb, nullptr, 0, ws, N, nullptr,
                                                         kSplitRows, (int64_t)M * N);
    BCV_HIP(hipGetLastError());
    const int64_t n = (int64_t)M * N;
    sum_splits_kernel<<<grid_for(n), 256, 0, st>>>(n, splits, ws, 0, C);
    BCV_HIP(hipGetLastError());
}

void silu_backward(int64_t n, const float *Z, const float *dH, float *dZ, hipStream_t st)
{
    if (n == 0) return;
    silu_backward_kernel<<<grid_for(n), 256, 0, st>>>(n, Z, dH, dZ);
    BCV_HIP(hipGetLastError());
}

void column_sum(int M, int N, const float *dZ, float *db, float *ws, hipStream_t st)
{
    if (N <= 0) return;
    const int splits = std::max(1, (M + kSplitRows - 1) / kSplitRows);
    column_sum_kernel<<<dim3((N + 127) / 128, splits), 128, 0, st>>>(M, N, kSplitRows, dZ, ws);
    BCV_HIP(hipGetLastError());
    sum_splits_kernel<<<grid_for(N), 256, 0, st>>>(N, splits, ws, 0, db);
    BCV_HIP(hipGetLastError());
}

void loss_grad(int B, const float *Y, const float *r, float w_err, float eps, float *dY, float *terms, hipStream_t st)
{
    loss_kernel<<<(B + 255) / 256, 256, 0, st>>>(B, Y, r, w_err, eps, dY, terms);
    BCV_HIP(hipGetLastError());
}

void adam_step(int64_t n, float *p, const float *g, float *m, float *v, float lr_t, float b1, float b2, float eps,
               hipStream_t st)
{
    adam_kernel<<<grid_for(n), 256, 0, st>>>(n, p, g, m, v, lr_t, b1, b2, eps);
    BCV_HIP(hipGetLastError());
}

// ---- fixed inference workspace (bcv_mlp_forward_noalloc) ---------------------------------------
// Three activation buffers of kNoAllocFloats floats each, in one statically allocated device array
// that every GPU the library runs on holds until the process ends. Its device address is looked up
// once per device, with that device current, and only that address is used from the host: the
// array's name is a host-side stand-in, not a device address.
static __device__ __align__(256) float scratch[3 * kNoAllocFloats];

float *noalloc_workspace(int device)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static float *ptr[kMaxDevices] = {};
    BCV_REQUIRE(device >= 0 && device < kMaxDevices, BCV_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(mu);
    if (ptr[device] == nullptr) {
        int prev = 0;
        BCV_HIP(hipGetDevice(&prev));
        BCV_HIP(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        BCV_HIP(hipSetDevice(prev));
        if (e != hipSuccess) fail(BCV_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        BCV_REQUIRE(p != nullptr, BCV_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        ptr[device] = static_cast<float *>(p);
    }
    return ptr[device];
}

void gather_rows(int B, int d, const int32_t *idx, const float *in, float *out, hipStream_t st)
{
    const int64_t n = (int64_t)B * d;
    if (n == 0) return;
    gather_rows_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(B, d, idx, in, out);
    BCV_HIP(hipGetLastError());
}

}  // namespace bcv
