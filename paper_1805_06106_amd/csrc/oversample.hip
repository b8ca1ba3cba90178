// Strengths of an oversampled source quadrature on gfx950 (Section 3: the stage-2
// quadrature discretization evaluates the layer potential with a finer rule on the same
// elements as the density's unisolvent node set).  The density arrives as node values; each
// quadrature node's value is the element's interpolant at that node, times its weight:
//   q_i = w_i * sum_k A[f][k] * mu[e * n_node + k],   (e, f) = divmod(input index of i, n_quad)
// One thread per source in tree order.  Neighbouring threads mostly share an element, so the
// node values and the matrix rows (at most 2^20 entries) are served from L1/L2; the kernel is
// bound by the strength write and the index reads (24 B per source plus the node values).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace gq {

namespace {

__global__ __launch_bounds__(256) void k_strength_interp(int64_t n,
                                                         const int64_t* __restrict__ order,
                                                         const double* __restrict__ w,
                                                         int n_node, int n_quad,
                                                         const double* __restrict__ A,
                                                         const double* __restrict__ mu,
                                                         double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t src = order[i];
  const int64_t e = src / n_quad;
  const int f = (int)(src - e * n_quad);
  const double* a = A + (int64_t)f * n_node;
  const double* m = mu + e * n_node;
  double acc = 0.0;
  for (int k = 0; k < n_node; ++k) acc = fma(a[k], m[k], acc);
  q[i] = w[i] * acc;
}

}  // namespace

void launch_strength_interp(hipStream_t s, int64_t n, const int64_t* order, const double* w,
                            int n_node, int n_quad, const double* interp, const double* density,
                            double* q) {
  if (n <= 0) return;
  const int64_t blocks = (n + 255) / 256;
  k_strength_interp<<<(unsigned)blocks, 256, 0, s>>>(n, order, w, n_node, n_quad, interp, density,
                                                     q);
}

}  // namespace gq
