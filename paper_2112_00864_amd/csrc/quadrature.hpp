// High-order box-pair quadrature (quadrature.hip): the training data and the error reference of the
// touching-pair surrogate.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bcv {

constexpr int kQMaxGauss = 16;

// out[p] = int_A int_B 1/|x - y| dy dx for n pairs of axis-aligned boxes; geom holds 12 doubles per
// pair: A lower corner (3), A upper corner (3), B lower corner (3), B upper corner (3). n_gauss
// points per direction (1..16) on every cell of the graded decomposition. A pair whose
// decomposition overflows the kernel's lists gets NaN. Device pointers, stream-ordered.
void box_pair_integrals_device(int64_t n, const double *geom_dev, int n_gauss, double *out_dev, hipStream_t st);

// The same with host arrays, on `device` (synchronous).
void box_pair_integrals(int device, int64_t n, const double *geom_host, int n_gauss, double *out_host);

}  // namespace bcv
