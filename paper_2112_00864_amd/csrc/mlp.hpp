// Launchers of the surrogate network's kernels (mlp.hip). Device pointers, stream-ordered, FP32.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bcv {

// C[M x N] = op(A) op(B) (+ bias[N]) (+ C if accumulate); if H != nullptr also H = silu(C).
// op(A) is A [M x K] (row stride lda), or A^T with A stored [K x M] when ta; likewise op(B).
void gemm(bool ta, bool tb, int M, int N, int K, const float *A, int lda, const float *B, int ldb, const float *bias,
          bool accumulate, float *C, int ldc, float *H, hipStream_t st);

// C[M x N] = A^T B with A stored [K x M] and B [K x N] (weight gradients: K is the batch), split
// over K in fixed chunks whose partial products go to ws (split_workspace(M, N, K) floats) and are
// summed in chunk order.
int64_t split_workspace(int M, int N, int K);
void gemm_tn_split(int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, float *ws,
                   hipStream_t st);

// dZ = dH * silu'(Z), elementwise over n values.
void silu_backward(int64_t n, const float *Z, const float *dH, float *dZ, hipStream_t st);

// db[n] = sum over the M rows of dZ [M x N], in fixed row chunks (partial sums in ws,
// split_workspace(1, N, M) floats) summed in chunk order.
void column_sum(int M, int N, const float *dZ, float *db, float *ws, hipStream_t st);

// Loss of B rows Y = (value, log-error) against targets r (see mlp.hip): dY = dL/dY, terms = the
// two squared terms per row.
void loss_grad(int B, const float *Y, const float *r, float w_err, float eps, float *dY, float *terms, hipStream_t st);

// One Adam step over n parameters; lr_t includes the bias correction.
void adam_step(int64_t n, float *p, const float *g, float *m, float *v, float lr_t, float b1, float b2, float eps,
               hipStream_t st);

// Device address, on `device`, of the library's fixed inference workspace: 3 * kNoAllocFloats
// floats (three activation buffers of rows x width <= kNoAllocFloats), looked up on the first call
// per device (sets and restores the current device; no allocation).
constexpr int64_t kNoAllocFloats = int64_t(1) << 20;
float *noalloc_workspace(int device);

// out[i] = in[idx[i]] for B rows of width d.
void gather_rows(int B, int d, const int32_t *idx, const float *in, float *out, hipStream_t st);

}  // namespace bcv
