// qmc_guard.hpp -- FP64 re-decision of near-tie moves in the mixed-precision chain.
//
// The mixed path forms |Psi'/Psi|^2 = R^2 exp(2 dJ) from an FP32 ratio.  When
// the uniform u falls within a relative band around that value the decision
// could differ from the one FP64 arithmetic makes, so it is taken again from
// an FP64 ratio: the inverse column x = A^-1 e_k is refined from the FP32
// column by three steps of x <- x + B (e_k - A x), with the FP64 Slater matrix A
// assembled from the FP64 orbital values the gather kept, and R = v . x.
#pragma once

#include "qmc_device.hpp"

namespace qmc {

// All threads of the block call this (uniform control flow).  Bm: the current
// FP32 inverse of the spin block (row stride ldb); scur: LDS buffer flags of
// the block's electrons; v64: the proposal's FP64 value row; sx, sr: LDS
// scratch of n doubles each; red: LDS scratch of kWaves doubles.
template <typename T>
__device__ __forceinline__ double refined_ratio(const SysParams& P, const Walkers<T>& Wk, const T* Bm, int ldb, int n,
                                size_t item0, const uint8_t* scur, const double* v64, int k, double* sx,
                                double* sr, double* red, int tid) {
  const int lane = tid & 63, wave = wave_of(tid);
  for (int l = tid; l < n; l += kBlock) sx[l] = (double)Bm[(size_t)l * ldb + k];
  __syncthreads();
  // Each wave takes four rows at a time, its lanes striding along the rows (coalesced reads of
  // the FP64 Slater matrix and of B), and adds each row's partial sums across the wave.
  for (int it = 0; it < 3; ++it) {
    for (int j0 = 4 * wave; j0 < n; j0 += 4 * kWaves) {   // r = e_k - A x
      double a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = 0.0;
        const int j = j0 + u;
        if (j < n) {
          const double* arow = Wk.val64 + ((size_t)scur[j] * P.W * P.N + item0 + j) * P.S;
          for (int l = lane; l < n; l += 64) a[u] += arow[l] * sx[l];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = wave_sum_dpp(a[u]);
      if (lane == 0)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (j0 + u < n) sr[j0 + u] = (j0 + u == k ? 1.0 : 0.0) - a[u];
    }
    __syncthreads();
    for (int l0 = 4 * wave; l0 < n; l0 += 4 * kWaves) {   // x += B r
      double a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = 0.0;
        const int l = l0 + u;
        if (l < n)
          for (int j = lane; j < n; j += 64) a[u] += (double)Bm[(size_t)l * ldb + j] * sr[j];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = wave_sum_dpp(a[u]);
      if (lane == 0)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (l0 + u < n) sx[l0 + u] += a[u];
    }
    __syncthreads();
  }
  double part = 0.0;
  for (int l = tid; l < n; l += kBlock) part += v64[l] * sx[l];
  part = wave_sum_dpp(part);
  if (lane == 0) red[wave] = part;
  __syncthreads();
  double R = 0.0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) R += red[q];
  __syncthreads();
  return R;
}

}  // namespace qmc
